"""Parity at the largest sizes the benchmark runs, in its launch
configurations, against the FP64 oracle: the 384 x 192 x 192 channel TO-LES
(FP32, 12 QoIs, the LRS correction active from the first step) and the
480 x 240 x 240 plain BGK channel (FP32).  The oracle steps these grids in
tens of seconds, so a few steps are compared over every cell."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_run, need_gpu, oracle_run, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_channel_384x192x192_to_les_two_steps():
    """The HBM-resident grid over every cell, two steps with the LRS active
    from the first: the second step's pull applies the first step's SGS
    records (the form this grid size takes)."""
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(384, 192, 192, substrate=1, cmodel=0.1, seed=6)
    nb, dmin, dmax = synth.channel_bands(192)
    C, mu, S = synth.lrs_model_channel(12, 7, 9)
    cargs = dict(mode="lrs", spinup=0, C=C, mu=mu, Sigma=S, seed=8, nbands=nb, dmin=dmin, dmax=dmax)
    _say("384x192x192 channel TO-LES, FP32, 2 steps")
    run = gpu_run(lbm, cfg, u0, "fp32", synth.QOIS_3D, cargs)
    run.step(2)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, synth.QOIS_3D, cargs)
    o.step(2)
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(run.fields()[1], o.velocity()[1])
    eq = np.max(np.abs(rg["q"] - ro["q"]) / np.abs(ro["q"]))
    edq = np.max(np.abs(rg["dq"] - ro["dq"]) / np.abs(ro["dq"]))
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}")
    assert np.array_equal(rg["flags"], ro["flags"]) and np.all(ro["dq"] != 0)
    # velocity: the stated 1e-5; q* about four times the measured 1.3e-7; dQ
    # the bar of the other 3-D FP32 parity tests (measured 7.3e-4: after the
    # first corrected step dQ = s z - q* is a difference small against q*,
    # which FP32 resolves to about 1e-7 of itself)
    assert ev <= 1e-5 and eq <= 5e-7 and edq <= 5e-3


def test_fine_grid_480x240x240_plain():
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(480, 240, 240, substrate=0, cmodel=0.0, seed=13)
    _say("480x240x240 plain BGK, FP32, 3 steps")
    run = gpu_run(lbm, cfg, u0, "fp32")
    run.step(3)
    assert run.sync() == 0
    o = oracle_run(cfg, u0)
    o.step(3)
    ev = rel_err(run.fields()[1], o.velocity()[1])
    _say(f"  velocity {ev:.2e}")
    assert ev <= 1e-5


def test_paper_hf_grid_plain_rows_equal_a_thin_slab():
    """The paper's HF grid, 1475 x 235 x 490 plain BGK in FP32 (170 M cells:
    its populations exceed 4 GiB, so the step runs with 64-bit offsets and
    non-temporal stores), started from a field that does not depend on x:
    x-periodic streaming keeps every x row the same, so after 4 steps every
    row must equal, bitwise, the rows of a 5 x 235 x 490 slab started from
    the same field, which is itself checked against the oracle."""
    lbm = need_gpu()
    nx, ny, nz, steps = 1475, 235, 490, 4
    cfg, _ = synth.channel_workload(5, ny, nz, substrate=0, cmodel=0.0, seed=13)
    rng = np.random.default_rng(21)
    yz = synth.channel_velocity(1, ny, nz, seed=13).reshape(3, nz, ny, 1)
    yz = yz + 1e-3 * (2 * rng.random(yz.shape) - 1)
    slab_u0 = np.ascontiguousarray(np.broadcast_to(yz, (3, nz, ny, 5))).reshape(3, -1)
    _say("thin slab 5x235x490 vs oracle, 4 steps")
    slab = gpu_run(lbm, cfg, slab_u0, "fp32")
    slab.step(steps)
    assert slab.sync() == 0
    us = slab.fields()[1].reshape(3, nz, ny, 5)
    o = oracle_run(cfg, slab_u0)
    o.step(steps)
    assert rel_err(us.reshape(3, -1), o.velocity()[1]) <= 1e-5
    assert np.array_equal(us, np.broadcast_to(us[..., :1], us.shape))   # x-invariant
    slab.close()
    _say("HF grid 1475x235x490 plain, 4 steps")
    big_cfg = dict(cfg, nx=nx)
    big_u0 = np.broadcast_to(yz, (3, nz, ny, nx)).reshape(3, -1)
    big = gpu_run(lbm, big_cfg, big_u0, "fp32")
    big.step(steps)
    assert big.sync() == 0
    ub = big.fields()[1].reshape(3, nz, ny, nx)
    big.close()
    assert np.array_equal(ub, np.broadcast_to(us[..., :1], ub.shape))


def test_to_les_beyond_32bit_population_offsets():
    """A 1216 x 192 x 256 channel TO-LES in FP32 (60 M cells: its populations
    exceed 4 GiB, so the tiled stream-collide runs with 64-bit offsets), 3
    steps with the LRS active from the first, from a field independent of x:
    the whole TO step (filters, sums, solve, recorded SGS change) keeps every
    x row bitwise the same, and the rows match those of a 4 x 192 x 256 slab
    from the same field (whose sums differ only in rounding order), itself
    checked against the oracle."""
    from gpu_util import closure_args
    lbm = need_gpu()
    nx, ny, nz, steps = 1216, 192, 256, 3
    cfg, _ = synth.channel_workload(4, ny, nz, substrate=1, cmodel=0.1, seed=6)
    qois, cargs = closure_args("3d", ny=ny, spinup=0)
    rng = np.random.default_rng(22)
    yz = synth.channel_velocity(1, ny, nz, seed=6).reshape(3, nz, ny, 1)
    yz = yz + 1e-3 * (2 * rng.random(yz.shape) - 1)
    slab_u0 = np.ascontiguousarray(np.broadcast_to(yz, (3, nz, ny, 4))).reshape(3, -1)
    _say("TO slab 4x192x256 vs oracle, 3 steps")
    slab = gpu_run(lbm, cfg, slab_u0, "fp32", qois, cargs)
    slab.step(steps)
    assert slab.sync() == 0
    us = slab.fields()[1].reshape(3, nz, ny, 4)
    o = oracle_run(cfg, slab_u0, qois, cargs)
    o.step(steps)
    assert rel_err(us.reshape(3, -1), o.velocity()[1]) <= 1e-5
    assert np.any(slab.record_arrays()["dq"] != 0)
    slab.close()
    _say("TO 1216x192x256, 3 steps")
    big = gpu_run(lbm, dict(cfg, nx=nx), np.broadcast_to(yz, (3, nz, ny, nx)).reshape(3, -1), "fp32", qois, cargs)
    big.step(steps)
    assert big.sync() == 0
    ub = big.fields()[1].reshape(3, nz, ny, nx)
    big.close()
    assert np.array_equal(ub, np.broadcast_to(ub[..., :1], ub.shape))   # every row the same
    e = rel_err(ub[..., 0], us[..., 0])
    _say(f"  rows vs slab: {e:.2e}")
    assert e <= 1e-5

"""GPU parity of the HIP library against the FP64 CPU oracle (called through
the C ABI).  Tolerances: bit-exact for index maps and random integers;
max relative velocity error <= 1e-12 in FP64 and <= 1e-5 in FP32 (shifted
populations) after 200 steps; QoIs, dQ and gamma per step to the bounds
stated at each test.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (closure_args, fp64_bars, gpu_run, match_populations, need_gpu, oracle_floor, oracle_run,
                      rel_err)

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(msg):
    print(msg, flush=True)


def test_philox_known_answers_on_device():
    lbm = need_gpu()
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(t, 16) for t in line.split()])
    rows = np.array(rows, dtype=np.uint64)
    out = lbm.test_philox(rows[:, :6].astype(np.uint32))
    assert np.array_equal(out.astype(np.uint64), rows[:, 6:])


def test_lrs_normals_match_oracle():
    lbm = need_gpu()
    z = lbm.test_normals(0x1234ABCD5678, 3, 500, 12)
    zo = np.array([oracle.lrs_normals(0x1234ABCD5678, 3 + s, 12) for s in range(500)])
    assert np.max(np.abs(z - zo)) < 1e-13


@pytest.mark.parametrize("lat,walls", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_plain"])
def test_stream_index_map_bit_exact(lat, walls, prec):
    lbm = need_gpu()
    _say(f"index map lat={lat} walls={walls} prec={prec}")
    nx, ny, nz = 37, 11, (5 if lat else 1)
    cfg = dict(lattice=lat, nx=nx, ny=ny, nz=nz, walls_y=walls, tau=0.8)
    o = oracle.Oracle(**cfg)
    Q, N = o.Q, o.N
    ids = np.arange(Q * N, dtype=np.float64).reshape(Q, N)   # < 2^24: exact in FP32
    run = lbm.Run(lbm.make_config(precision=prec, **{k: v for k, v in cfg.items()}))
    cg, _ = lbm.lattice_info(lat)
    co, _ = oracle.lattice(lat)
    perm = [next(j for j in range(Q) if np.array_equal(cg[j], co[i])) for i in range(Q)]
    inv = np.argsort(perm)
    run.set_populations(ids[inv])              # library order
    run.stream_only()
    got = match_populations(lbm, lat, run.get_populations())
    o.set_fp(ids)
    o.stream_only()
    assert np.array_equal(got, o.get_fp())


@pytest.mark.parametrize("steps", [200, 1000])
def test_plain_fp64_kolmogorov_128(steps):
    """D2Q9 128^2 Kolmogorov flow, FP64, tau = 0.55, no closure: velocity and
    the E, Z series of the post-streaming state."""
    lbm = need_gpu()
    _say(f"plain fp64 128^2 {steps} steps")
    cfg, u0 = synth.kolmogorov_workload(128, tau=0.55, seed=1)
    run = gpu_run(lbm, cfg, u0, "fp64", diag=1)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0)
    o.step(steps)
    _, ug = run.fields()
    _, uo = o.velocity()
    assert rel_err(ug, uo) <= 1e-12
    rg, ro = run.record_arrays(), o.record_arrays()
    assert np.array_equal(rg["step"], np.arange(steps))
    assert rel_err(rg["diag_e"], ro["diag_e"]) <= 1e-12
    assert rel_err(rg["diag_z"], ro["diag_z"]) <= 1e-12
    # mass is conserved exactly; both sides carry only their own rounding
    assert np.max(np.abs(rg["mass"] - 128 * 128)) <= 1e-12 * 128 * 128


@pytest.mark.parametrize("lat", [0, 1])
def test_plain_fp32_shifted_vs_plain(lat):
    """FP32 shifted populations reach 1e-5; the unshifted FP32 baseline is
    reported and must be no better."""
    lbm = need_gpu()
    if lat == 0:
        cfg, u0 = synth.kolmogorov_workload(100, tau=0.55, seed=1)
        cfg["ny"] = 70
        u0 = synth.noise_velocity(2, (1, 70, 100), 1e-4, 1)
    else:
        cfg, u0 = synth.channel_workload(20, 16, 12, substrate=1, cmodel=0.1)
    o = oracle_run(cfg, u0)
    o.step(200)
    _, uo = o.velocity()
    errs = {}
    for prec in ("fp32", "fp32_plain"):
        run = gpu_run(lbm, cfg, u0, prec)
        run.step(200)
        run.sync()
        errs[prec] = rel_err(run.fields()[1], uo)
    _say(f"plain lat={lat}: fp32 shifted err {errs['fp32']:.2e}, fp32 plain err {errs['fp32_plain']:.2e}")
    assert errs["fp32"] <= 1e-5
    assert errs["fp32_plain"] >= errs["fp32"]


def _to_case(kind):
    if kind == "2d":
        cfg, u0 = synth.kolmogorov_workload(100, tau=0.51, seed=2)
        cfg["ny"] = 70
        u0 = synth.noise_velocity(2, (1, 70, 100), 1e-3, 2)
        qois, cargs = closure_args("2d")
    else:
        cfg, u0 = synth.channel_workload(20, 24, 12, substrate=1, cmodel=0.1)
        qois, cargs = closure_args("3d", ny=24)
    return cfg, u0, qois, cargs


@pytest.mark.parametrize("kind", ["2d", "3d"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_to_lrs_parity(kind, prec):
    """TO-LRS LES: velocity after 200 steps and the per-step q*, dQ, gamma.

    FP64: the stated 1e-12, or ten times the workload's own FP64 resolution
    (the oracle against its twins: one ulp away, sums reversed) where that
    is larger -- the 12-QoI channel closure solves a Gram system whose
    condition number (~1e7-1e8) amplifies last-bit differences every step.
    FP32: velocity <= 1e-5 (the stated bar), q* <= 1e-4; dQ and gamma per
    QoI relative to their largest value: about ten times the measured
    values (2-D 6.9e-8 and 4.1e-8; 3-D 1.8e-4 and 2.2e-4)."""
    lbm = need_gpu()
    _say(f"TO-LRS parity {kind} {prec}")
    cfg, u0, qois, cargs = _to_case(kind)
    steps = 200
    run = gpu_run(lbm, cfg, u0, prec, qois, cargs)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    _, ug = run.fields()
    _, uo = o.velocity()
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(ug, uo)
    eq = np.max(np.abs(rg["q"] - ro["q"]) / np.abs(ro["q"]))
    sc = np.max(np.abs(ro["dq"]), axis=0) + 1e-300
    edq = np.max(np.abs(rg["dq"] - ro["dq"]) / sc)
    gs = np.max(np.abs(ro["gamma"]), axis=0) + 1e-300
    eg = np.max(np.abs(rg["gamma"] - ro["gamma"]) / gs)
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}  gamma {eg:.2e}")
    assert np.array_equal(rg["flags"], ro["flags"])
    if prec == "fp64":
        floor = oracle_floor(cfg, u0, qois, cargs, steps, ref=o)
        bars = fp64_bars(floor)
        _say(f"  oracle floor: {np.array2string(floor, precision=2)}")
        assert ev <= bars[0] and eq <= bars[1] and edq <= bars[2] and eg <= bars[3]
    else:
        dbar = 1e-6 if kind == "2d" else 2e-3
        assert ev <= 1e-5 and eq <= 1e-4 and edq <= dbar and eg <= dbar


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_wale_substrate_parity(prec, tol):
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(20, 16, 12, substrate=2, cmodel=2.2)
    run = gpu_run(lbm, cfg, u0, prec)
    run.step(200)
    run.sync()
    o = oracle_run(cfg, u0)
    o.step(200)
    e = rel_err(run.fields()[1], o.velocity()[1])
    _say(f"WALE {prec}: {e:.2e}")
    assert e <= tol


def test_tracking_parity_fp64():
    lbm = need_gpu()
    cfg, u0, qois, cargs = _to_case("2d")
    o0 = oracle_run(cfg, u0, qois, dict(cargs, mode="off"))
    o0.step(60)
    qref = o0.record_arrays()["q"] * np.linspace(1.0, 1.05, 60)[:, None]
    targs = dict(cargs, mode="track", spinup=5)
    run = gpu_run(lbm, cfg, u0, "fp64", qois, targs, qref=qref)
    run.step(60)
    run.sync()
    o = oracle_run(cfg, u0, qois, targs, qref=qref)
    o.step(60)
    rg, ro = run.record_arrays(), o.record_arrays()
    assert rel_err(run.fields()[1], o.velocity()[1]) <= 1e-12
    assert np.allclose(rg["q"][5:] + rg["dq"][5:], qref[5:], rtol=1e-12, atol=0)
    assert rel_err(rg["gamma"], ro["gamma"]) <= 1e-9


def test_mass_momentum_records():
    lbm = need_gpu()
    cfg, u0 = synth.kolmogorov_workload(64, tau=0.6, seed=4)
    cfg.update(force_kind=2, force_amp=2e-6)
    run = gpu_run(lbm, cfg, u0, "fp64", diag=1)
    run.step(50)
    r = run.record_arrays()
    assert np.max(np.abs(r["mass"] - 64 * 64)) < 1e-9
    assert np.allclose(np.diff(r["mom"][:, 0]), 64 * 64 * 2e-6, rtol=1e-9)


def test_gram_singular_flag_and_no_nan():
    lbm = need_gpu()
    cfg, _ = synth.kolmogorov_workload(32, tau=0.6)
    cfg.update(force_kind=0)
    qois, cargs = closure_args("2d", spinup=0)
    run = gpu_run(lbm, cfg, np.zeros((2, 32 * 32)), "fp32", qois, cargs)
    run.step(3)
    r = run.record_arrays()
    assert np.all(r["flags"] & 2)
    assert np.all(np.isfinite(run.fields()[1]))


def test_unstable_flag_raises():
    lbm = need_gpu()
    cfg = dict(lattice=0, nx=16, ny=16, nz=1, walls_y=0, tau=0.5005, substrate=0, cmodel=0.0,
               force_kind=1, force_amp=5e-3, force_k=1, drag=0.0)
    run = gpu_run(lbm, cfg, synth.noise_velocity(2, (1, 16, 16), 0.05, 7), "fp32")
    run.step(400)
    with pytest.raises(lbm.LbmError) as e:
        run.sync()
    assert e.value.code == lbm.EUNSTABLE

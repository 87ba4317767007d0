"""Sharp Fourier band QoIs on the GPU (eq. scale-aware-energy-fourier,
App. E variant; hipFFT): TO-LRS parity against the oracle's plain DFT,
a mixed Fourier / kernel-filter closure, and batch = solo."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_run, need_gpu, oracle_run, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _case(kind, qois):
    nq = len(qois)
    C, mu, S = synth.lrs_history_model(0, nq, 3, 4, 5, noise=1e-4)
    cargs = dict(mode="lrs", spinup=10, C=C, mu=mu, Sigma=S, seed=41)
    if kind == "2d":
        cfg, _ = synth.kolmogorov_workload(32, tau=0.51, seed=3)
        return cfg, synth.noise_velocity(2, (1, 32, 32), 1e-3, 3), qois, cargs
    cfg = dict(lattice=1, nx=16, ny=16, nz=16, walls_y=0, tau=0.52, substrate=1, cmodel=0.1,
               force_kind=1, force_amp=1e-5, force_k=1, drag=0.0)
    return cfg, synth.noise_velocity(3, (16, 16, 16), 1e-3, 4), qois, cargs


CASES = {
    "2d_bands": ("2d", [(k, f, 0) for f in ("F0-3", "F4-8", "F9-16") for k in ("E", "Z")]),
    "3d_bands": ("3d", [(k, f, 0) for f in ("F0-2", "F3-8") for k in ("E", "Z")]),
    "2d_mixed": ("2d", [("E", "F0-4", 0), ("Z", "F5-12", 0), ("E", "G3", 0), ("Z", "L1", 0)]),
}


@pytest.mark.parametrize("name,prec", [("2d_bands", "fp64"), ("3d_bands", "fp64"), ("2d_mixed", "fp64"),
                                       ("3d_bands", "fp32")])
def test_fourier_lrs_parity(name, prec):
    lbm = need_gpu()
    kind, qois = CASES[name]
    cfg, u0, qois, cargs = _case(kind, qois)
    steps = 30
    _say(f"Fourier bands {name} {prec}")
    run = gpu_run(lbm, cfg, u0, prec, qois, cargs)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(run.fields()[1], o.velocity()[1])
    eq = np.max(np.abs(rg["q"] - ro["q"]) / np.abs(ro["q"]))
    edq = np.max(np.abs(rg["dq"] - ro["dq"]) / (np.max(np.abs(ro["dq"]), axis=0) + 1e-300))
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}")
    assert np.array_equal(rg["flags"], ro["flags"])
    assert np.any(ro["dq"] != 0)
    if prec == "fp64":
        assert ev <= 1e-12 and eq <= 1e-12 and edq <= 1e-10
    else:
        # velocity: the stated 1e-5; q*, dQ about ten times the measured
        # 1.6e-6 and 2.1e-6
        assert ev <= 1e-5 and eq <= 1e-5 and edq <= 1e-5   # measured 5.6e-7, 9.8e-7, 6.5e-7


def test_fourier_member_in_batch_bitwise():
    lbm = need_gpu()
    cases = [_case(*CASES["2d_bands"]), _case(*CASES["2d_mixed"])]
    solo = [gpu_run(lbm, c, u, "fp32", q, a) for c, u, q, a in cases]
    batched = [gpu_run(lbm, c, u, "fp32", q, a) for c, u, q, a in cases]
    for r in solo:
        r.step(40)
    batch = lbm.Batch(batched)
    batch.step(40)
    batch.sync()
    for r, s in zip(batched, solo):
        s.sync()
        assert np.array_equal(r.get_populations(), s.get_populations())
        assert np.array_equal(r.record_arrays()["q"], s.record_arrays()["q"])

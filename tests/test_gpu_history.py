"""History-h LRS on the GPU (eq. LRS with h > 0): the k_sum history product
and the solve against the FP64 oracle, the zero-history reduction to h = 0,
batch members with history models, and closure validation on the device."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_run, need_gpu, oracle_run, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _scale(cfg, u0, qois, cargs):
    """s = |q*| of the last spin-up step of an uncorrected oracle run, zero
    replaced by one."""
    o = oracle_run(cfg, u0, qois, {k: v for k, v in cargs.items() if k in ("nbands", "dmin", "dmax")})
    o.step(cargs["spinup"])
    s = np.abs(o.record_arrays()["q"][-1])
    s[s == 0] = 1.0
    return s


def _case2d(h, spinup, n=48, ny=40, seed=2):
    cfg, _ = synth.kolmogorov_workload(n, tau=0.51, seed=seed)
    cfg["ny"] = ny
    u0 = synth.noise_velocity(2, (1, ny, n), 1e-3, seed)
    qois = synth.QOIS_2D
    C, mu, S = synth.lrs_history_model(h, 2, 3, 4, 5, noise=1e-4)
    cargs = dict(mode="lrs", spinup=spinup, C=C, mu=mu, Sigma=S, seed=71, h=h)
    cargs["scale"] = _scale(cfg, u0, qois, cargs)
    return cfg, u0, qois, cargs


def _case3d(h, spinup):
    cfg, u0 = synth.channel_workload(20, 24, 12, substrate=1, cmodel=0.1)
    qois = synth.QOIS_3D
    nb, dmin, dmax = synth.channel_bands(24)
    C, mu, S = synth.lrs_history_model(h, 12, 7, 9, 10)
    cargs = dict(mode="lrs", spinup=spinup, C=C, mu=mu, Sigma=S, seed=72, h=h,
                 nbands=nb, dmin=dmin, dmax=dmax)
    cargs["scale"] = _scale(cfg, u0, qois, cargs)
    return cfg, u0, qois, cargs


def _compare(run, o):
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(run.fields()[1], o.velocity()[1])
    eq = np.max(np.abs(rg["q"] - ro["q"]) / np.abs(ro["q"]))
    edq = np.max(np.abs(rg["dq"] - ro["dq"]) / (np.max(np.abs(ro["dq"]), axis=0) + 1e-300))
    eg = np.max(np.abs(rg["gamma"] - ro["gamma"]) / (np.max(np.abs(ro["gamma"]), axis=0) + 1e-300))
    assert np.array_equal(rg["flags"], ro["flags"])
    assert np.any(ro["dq"] != 0)
    return ev, eq, edq, eg


def test_history_lrs_parity_2d_fp64_many_chunks():
    """h = 300, nq = 2: 1200 history entries over three k_sum workgroups."""
    lbm = need_gpu()
    h, S0, steps = 300, 305, 340
    cfg, u0, qois, cargs = _case2d(h, S0)
    _say(f"history 2d fp64 h={h}")
    run = gpu_run(lbm, cfg, u0, "fp64", qois, cargs)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    ev, eq, edq, eg = _compare(run, o)
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}  gamma {eg:.2e}")
    assert ev <= 1e-12 and eq <= 1e-12 and edq <= 1e-10 and eg <= 1e-10


def test_history_lrs_parity_channel_fp32():
    """The 12-QoI channel closure with h = 3 in FP32: velocity <= 1e-5 (the
    stated bar); q*, dQ, gamma about ten times the measured 4.8e-6, 7.4e-5
    and 1.2e-4."""
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case3d(3, 8)
    _say("history channel fp32 h=3")
    run = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    run.step(60)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(60)
    ev, eq, edq, eg = _compare(run, o)
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}  gamma {eg:.2e}")
    assert ev <= 1e-5 and eq <= 5e-5 and edq <= 1e-3 and eg <= 1e-3


def test_zero_history_rows_bitwise_equal_h0():
    lbm = need_gpu()
    h = 40
    cfg, u0, qois, cargs = _case2d(h, 50)
    C = cargs["C"]
    C0 = np.vstack([C[h * 2:(h + 1) * 2], C[-1:]])
    Ch = np.zeros_like(C)
    Ch[h * 2:(h + 1) * 2] = C0[:2]
    Ch[-1] = C0[2]
    a = gpu_run(lbm, cfg, u0, "fp32", qois, dict(cargs, C=C0, h=0))
    b = gpu_run(lbm, cfg, u0, "fp32", qois, dict(cargs, C=Ch))
    a.step(90)
    b.step(90)
    a.sync()
    b.sync()
    ra, rb = a.record_arrays(), b.record_arrays()
    for key in ("q", "dq", "gamma"):
        assert np.array_equal(ra[key], rb[key]), key
    assert np.array_equal(a.get_populations(), b.get_populations())


def test_history_members_in_batch_bitwise():
    lbm = need_gpu()
    cases = [_case2d(40, 45, n=32, ny=32, seed=1), _case2d(0, 10, n=48, ny=40, seed=2), _case3d(3, 8)]
    solo = [gpu_run(lbm, c, u, "fp32", q, a) for c, u, q, a in cases]
    batched = [gpu_run(lbm, c, u, "fp32", q, a) for c, u, q, a in cases]
    for r in solo:
        r.step(70)
    batch = lbm.Batch(batched)
    batch.step(70)
    batch.sync()
    for r, s in zip(batched, solo):
        s.sync()
        assert np.array_equal(r.get_populations(), s.get_populations())
        assert np.array_equal(r.record_arrays()["dq"], s.record_arrays()["dq"])


def test_history_closure_needs_recorded_steps():
    """spinup must leave h recorded steps under the closure when it is set."""
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case2d(10, 12)
    run = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    run.step(5)
    run.sync()
    with pytest.raises(lbm.LbmError):
        run.set_closure(lbm.ClosureSpec(qois, **dict(cargs, spinup=12)))   # 12 < 5 + 10
    run.set_closure(lbm.ClosureSpec(qois, **dict(cargs, spinup=15)))
    run.step(20)
    assert run.sync() == 0
    r = run.record_arrays()
    assert np.all(r["dq"][:15] == 0) and np.any(r["dq"][15:] != 0)


def test_full_size_channel_h500_property():
    """The benchmark channel (96x48x48, FP32, 12 QoIs) with the paper's history
    length h = 500: 12000 history entries over 24 k_sum workgroups.  At every
    corrected step the recorded dQ equals the model applied to the recorded
    history, dQ^n = s (x^n C + mu + L xi^n) - q*^n, with x^n assembled from
    the records and xi^n the step's normals (both by the oracle's helpers)."""
    import oracle
    lbm = need_gpu()
    h, S0, steps = 500, 505, 515
    cfg, u0 = synth.channel_workload(96, 48, 48, substrate=1, cmodel=0.1, seed=6)
    qois = synth.QOIS_3D
    nb, dmin, dmax = synth.channel_bands(48)
    C, mu, S = synth.lrs_history_model(h, 12, 7, 9, 10)
    o = oracle.Oracle(**cfg)
    q0, _ = o.qoi(oracle.make_closure(qois, nbands=nb, dmin=dmin, dmax=dmax), u0)
    s = np.abs(q0)
    cargs = dict(mode="lrs", spinup=S0, C=C, mu=mu, Sigma=S, seed=73, h=h, nbands=nb, dmin=dmin, dmax=dmax,
                 scale=s)
    run = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    run.step(steps)
    assert run.sync() == 0
    r = run.record_arrays()
    q, dq = r["q"], r["dq"]
    assert not np.any(r["flags"])
    X, _ = oracle.lrs_inputs(q + dq, q, h, s)
    Lc = np.linalg.cholesky(S)
    for n in range(S0, steps):
        eta = mu + Lc @ oracle.lrs_normals(73, n, 12)
        want = s * (X[n - h] @ C + eta) - q[n]
        err = np.max(np.abs(dq[n] - want) / s)
        _say(f"  step {n}: max |dQ - model| / s = {err:.2e}")
        assert err <= 1e-12
    assert np.all(dq[:S0] == 0)


def test_train_then_online_workflow():
    """The paper's workflow on the device (Sec. 4.3-4.5): a tracking run
    towards reference QoIs, the LRS fit (h = 3) to its records, then an
    online run with the fitted model.  The online run stays stable and its
    corrected QoIs stay near the training targets."""
    lbm = need_gpu()
    cfg, _ = synth.kolmogorov_workload(64, tau=0.51, seed=4)
    u0 = synth.noise_velocity(2, (1, 64, 64), 1e-3, 4)
    qois = synth.QOIS_2D
    steps, S0, h = 600, 20, 3
    o = oracle_run(cfg, u0, qois, dict(mode="off"))
    o.step(steps)
    qref = o.record_arrays()["q"] * (1 + 0.05 * np.sin(np.arange(steps) / 40.0))[:, None]
    trk = gpu_run(lbm, cfg, u0, "fp32", qois, dict(mode="track", spinup=S0), qref=qref)
    trk.step(steps)
    assert trk.sync() == 0
    r = trk.record_arrays()
    C, mu, S, s = lbm.lrs_fit(r["q"][S0:], r["dq"][S0:], h, 1e-3, flags=r["flags"][S0:])
    assert np.all(np.isfinite(C)) and np.all(np.linalg.eigvalsh(S) > 0)
    on = gpu_run(lbm, cfg, u0, "fp32", qois, dict(mode="lrs", spinup=S0, C=C, mu=mu, Sigma=S, scale=s, h=h,
                                                  seed=19))
    on.step(steps)
    assert on.sync() == 0
    ro = on.record_arrays()
    assert not np.any(ro["flags"])
    qc = ro["q"][S0:] + ro["dq"][S0:]
    lo, hi = qref[S0:].min(axis=0), qref[S0:].max(axis=0)
    span = hi - lo
    _say(f"  online corrected QoIs in [{qc.min(axis=0)}, {qc.max(axis=0)}], targets [{lo}, {hi}]")
    assert np.all(qc.min(axis=0) > lo - span) and np.all(qc.max(axis=0) < hi + span)


def test_history_checkpoint_resume_bitwise():
    """The history of a history-h model is the record ring, which the
    checkpoint image carries: resuming mid-run (after activation) is bitwise
    equal to the uninterrupted run."""
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case2d(12, 15, n=32, ny=32)
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    a.step(25)
    img = a.get_state()
    a.step(30)
    b = gpu_run(lbm, cfg, np.zeros_like(u0), "fp32", qois, cargs)
    b.set_state(img)
    assert b.step_count == 25
    b.step(30)
    assert np.array_equal(a.get_populations(), b.get_populations())
    ra, rb = a.record_arrays(25, 30), b.record_arrays(25, 30)
    assert np.array_equal(ra["dq"], rb["dq"]) and np.any(ra["dq"] != 0)

"""Edge cases of the TO-LES path on the GPU against the FP64 oracle: the
smallest grids the library accepts (3 cells per axis, where every stencil
and filter wraps or pads on itself, and the kernel filters of radius up to
12 wrap several times), ragged grids that fill no binomial tile or z chunk,
and the degenerate closures: one whose activation lies past the run, a
tracking reference shorter than the run, and zero steps."""
import numpy as np
import pytest

import synth
from gpu_util import closure_args, fp64_bars, gpu_run, need_gpu, oracle_floor, oracle_run, rel_err

pytestmark = pytest.mark.gpu

KQ2 = [(k, f, 0) for f in ("G3", "L3", "L1") for k in ("E", "Z")]


def _say(msg):
    print(msg, flush=True)


def _k2(nx, ny, walls, seed=3):
    """A small 2-D Kolmogorov (periodic) or channel-forced (walls) grid."""
    cfg, _ = synth.kolmogorov_workload(nx, tau=0.55, amp=1e-5, k=1, seed=seed)
    cfg["ny"] = ny
    if walls:
        cfg.update(walls_y=1, force_kind=2, force_amp=1e-6)
    return cfg, synth.noise_velocity(2, (1, ny, nx), 1e-3, seed)


def _lrs(nq, seed=31):
    C, mu, S = synth.lrs_history_model(0, nq, 3, 4, 5, noise=1e-4)
    return dict(mode="lrs", spinup=5, C=C, mu=mu, Sigma=S, seed=seed)


def _cases():
    out = {}
    qois2, ca2 = closure_args("2d", spinup=5)
    for walls in (0, 1):
        cfg, u0 = _k2(3, 3, walls)
        out[f"binomial_3x3_walls{walls}"] = (cfg, u0, qois2, ca2, {})
    # 3 x 3 x 3 channel: two mean-profile bands (three make the Gram matrix
    # singular to within 2e-15 of its largest diagonal entry on three rows)
    cfg, u0 = synth.channel_workload(3, 3, 3, substrate=1, cmodel=0.1)
    q3 = synth.QOIS_3D[:6] + [("MP", "I", j) for j in range(2)]
    C, mu, S = synth.lrs_model_channel(8, 7, 9)
    out["binomial_3x3x3_channel"] = (cfg, u0, q3, dict(mode="lrs", spinup=5, C=C, mu=mu, Sigma=S, seed=5, nbands=2,
                                                         dmin=0.5, dmax=1.5), {})
    # ragged in x, y and z (45 x 13 x 11 against 32 x 8 tiles and z chunks of 4)
    cfg, u0 = synth.channel_workload(45, 13, 11, substrate=1, cmodel=0.1)
    q3, ca3 = closure_args("3d", ny=13, spinup=5)
    out["binomial_ragged_45x13x11"] = (cfg, u0, q3, ca3, dict(tune_zc=4))
    cfg, u0 = _k2(3, 3, 1)
    out["kernel_3x3_walls"] = (cfg, u0, KQ2, _lrs(6), {})
    cfg, u0 = _k2(5, 4, 0)
    out["kernel_5x4_periodic"] = (cfg, u0, KQ2, _lrs(6), {})
    cfg, u0 = _k2(6, 5, 0)
    out["fourier_6x5"] = (cfg, u0, [(k, f, 0) for f in ("F0-1", "F2-2", "F3-4") for k in ("E", "Z")], _lrs(6), {})
    cfg, u0 = synth.channel_workload(4, 3, 5, substrate=1, cmodel=0.1)
    cfg.update(walls_y=0, force_kind=1, force_amp=1e-5, force_k=1)
    out["fourier_4x3x5"] = (cfg, u0, [(k, f, 0) for f in ("F0-1", "F2-3") for k in ("E", "Z")], _lrs(4), {})
    return out


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_and_ragged_grids_fp64(name):
    """Velocity, q*, dQ and gamma after 30 steps, FP64.  dQ and gamma are
    compared per QoI relative to their largest value over the run; q* per
    QoI relative to its largest value too, since on these grids a filter
    can leave a QoI many orders below the others (G_3 of radius 12 on a
    5-cell axis is nearly the mean), where the relative error of each single
    value measures cancellation, not the path."""
    lbm = need_gpu()
    cfg, u0, qois, cargs, tune = CASES[name]
    steps = 30
    _say(f"edge case {name}: grid {cfg['nx']}x{cfg['ny']}x{cfg['nz']} lattice {cfg['lattice']}")
    run = gpu_run(lbm, cfg, u0, "fp64", qois, cargs, **tune)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(run.fields()[1], o.velocity()[1])

    def per_qoi(key):
        sc = np.max(np.abs(ro[key]), axis=0) + 1e-300
        return float(np.max(np.abs(rg[key] - ro[key]) / sc))

    eq, edq, eg = per_qoi("q"), per_qoi("dq"), per_qoi("gamma")
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}  gamma {eg:.2e}")
    assert np.array_equal(rg["flags"], ro["flags"]) and not np.any(ro["flags"])
    assert np.any(ro["dq"] != 0)
    # the stated 1e-12 (1e-10 for dQ and gamma per QoI), or ten times the
    # workload's own FP64 resolution (the oracle against its twins) where
    # that is larger: on 3-cell grids the velocity left is small enough that
    # one ulp of the populations is 1e-12 of it, and the 12-QoI channel's
    # Gram system on 13 rows amplifies last-bit differences
    floor = oracle_floor(cfg, u0, qois, cargs, steps, ref=o)
    bars = fp64_bars(floor)
    _say(f"  oracle floor: {np.array2string(floor, precision=2)}")
    assert ev <= bars[0] and eq <= bars[1] and edq <= bars[2] and eg <= bars[3]


def test_closure_activation_past_the_run_is_the_uncorrected_run():
    """An LRS closure whose spin-up outlasts the run applies nothing: the
    populations and the recorded q* equal those of the same run with the
    closure off, bitwise, and every dQ is zero."""
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(20, 24, 12, substrate=1, cmodel=0.1)
    qois, cargs = closure_args("3d", ny=24, spinup=1000)
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    b = gpu_run(lbm, cfg, u0, "fp32", qois, dict(cargs, mode="off"))
    a.step(50)
    b.step(50)
    a.sync()
    b.sync()
    ra, rb = a.record_arrays(), b.record_arrays()
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(ra["q"], rb["q"])
    assert np.all(ra["dq"] == 0)


def test_tracking_reference_shorter_than_the_run():
    """Past the last reference step the tracking closure requests nothing
    (dQ = 0, as in the oracle); before it q* + dQ = q_ref."""
    lbm = need_gpu()
    cfg, u0 = _k2(24, 20, 0, seed=4)
    qois = synth.QOIS_2D
    steps, nref, S0 = 60, 35, 5
    o = oracle_run(cfg, u0, qois, dict(mode="off"))
    o.step(nref)
    qref = o.record_arrays()["q"] * (1 + 0.02 * np.cos(np.arange(nref) / 7.0))[:, None]
    cargs = dict(mode="track", spinup=S0)
    run = gpu_run(lbm, cfg, u0, "fp64", qois, cargs, qref=qref)
    run.step(steps)
    assert run.sync() == 0
    ot = oracle_run(cfg, u0, qois, cargs, qref=qref)
    ot.step(steps)
    rg, ro = run.record_arrays(), ot.record_arrays()
    assert np.all(rg["dq"][nref:] == 0) and np.all(rg["dq"][:S0] == 0)
    assert np.allclose(rg["q"][S0:nref] + rg["dq"][S0:nref], qref[S0:], rtol=1e-12, atol=0)
    ev = rel_err(run.fields()[1], ot.velocity()[1])
    _say(f"  velocity {ev:.2e}")
    assert ev <= 1e-12


def test_zero_steps():
    """step(0) changes nothing and records nothing."""
    lbm = need_gpu()
    cfg, u0 = _k2(24, 20, 0)
    qois, cargs = closure_args("2d", spinup=5)
    run = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    run.step(3)
    run.sync()
    f0 = run.get_populations()
    run.step(0)
    run.sync()
    assert run.step_count == 3
    assert np.array_equal(run.get_populations(), f0)
    assert run.record_arrays()["q"].shape[0] == 3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_singular_gram_skips_the_correction(prec):
    """The method's degenerate case: a uniform flow (periodic, unforced)
    stays uniform, so (I - B) v* = 0 and the Gram matrix of {E_B, E_(I-B)}
    is singular.  Every corrected step is flagged (record flag bit 1, as the
    oracle flags it), gamma is zero and the correction is skipped: the
    populations equal, bitwise, those of the same run with the closure off."""
    lbm = need_gpu()
    n, steps = 16, 10
    cfg = dict(lattice=0, nx=n, ny=n, nz=1, walls_y=0, tau=0.6, substrate=0, cmodel=0.0,
               force_kind=0, force_amp=0.0, force_k=0, drag=0.0)
    u0 = np.zeros((2, n * n))
    u0[0], u0[1] = 0.01, -0.005
    qois = [("E", "B", 0), ("E", "IMB", 0)]
    C, mu, S = synth.lrs_model(2, 3, 4, 5)
    cargs = dict(mode="lrs", spinup=2, C=C, mu=mu, Sigma=S, seed=3)
    run = gpu_run(lbm, cfg, u0, prec, qois, cargs)
    off = gpu_run(lbm, cfg, u0, prec, qois, dict(mode="off"))
    for r in (run, off):
        r.step(steps)
        r.sync()
    rg = run.record_arrays()
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    ro = o.record_arrays()
    _say(f"singular Gram {prec}: flags {rg['flags'].tolist()}")
    assert np.all(ro["flags"][2:] & 2) and np.array_equal(rg["flags"], ro["flags"])
    assert np.all(rg["gamma"] == 0) and np.any(rg["dq"][2:] != 0)
    assert np.array_equal(run.get_populations(), off.get_populations())
    if prec == "fp64":
        assert rel_err(run.fields()[1], o.velocity()[1]) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_largest_closure_sixteen_qois(prec):
    """The largest closure the library takes: 16 QoIs, 8 of them energy and
    enstrophy of the four binomial filter forms (B, B^2, B - B^2, I - B) and
    8 mean-profile bands, on the 20 x 24 x 12 channel with an LRS closure;
    a 16 x 16 Gram system each step.

    The four forms are nearly linearly dependent (B = (B - B^2) + B^2) and
    the bands overlap, so the Gram matrix of the patterns, scaled to unit
    diagonal, has a condition number near 3e7 at the first correction (an
    oracle test checks this).  FP64 is compared everywhere, within the
    workload's own resolution bars.  In FP32 the pattern rounding (a few
    ulp of the filtered fields) reaches gamma amplified by up to that
    condition number, and through gamma every later step; there the run is
    compared where no solve has intervened: q* up to the first corrected
    step and that step's dQ, to 1e-5 of each QoI's largest value, and the
    flags over the run."""
    lbm = need_gpu()
    cfg, u0, qois, cargs = synth.largest_closure_workload()
    steps, first = 30, cargs["spinup"]
    _say(f"largest closure {prec}: 16 QoIs on 20x24x12")
    run = gpu_run(lbm, cfg, u0, prec, qois, cargs)
    run.step(steps)
    assert run.sync() == 0
    o = oracle_run(cfg, u0, qois, cargs)
    o.step(steps)
    rg, ro = run.record_arrays(), o.record_arrays()
    ev = rel_err(run.fields()[1], o.velocity()[1])

    def per_qoi(key, rows=slice(None)):
        sc = np.max(np.abs(ro[key]), axis=0) + 1e-300
        return float(np.max(np.abs(rg[key][rows] - ro[key][rows]) / sc))

    eq, edq, eg = per_qoi("q"), per_qoi("dq"), per_qoi("gamma")
    _say(f"  velocity {ev:.2e}  q {eq:.2e}  dq {edq:.2e}  gamma {eg:.2e}")
    assert np.array_equal(rg["flags"], ro["flags"]) and not np.any(ro["flags"])
    assert np.all(np.any(ro["dq"][first:] != 0, axis=0))
    if prec == "fp64":
        floor = oracle_floor(cfg, u0, qois, cargs, steps, ref=o)
        bars = fp64_bars(floor)
        _say(f"  oracle floor: {np.array2string(floor, precision=2)}")
        assert ev <= bars[0] and eq <= bars[1] and edq <= bars[2] and eg <= bars[3]
    else:
        eq0, edq0 = per_qoi("q", slice(0, first + 1)), per_qoi("dq", slice(first, first + 1))
        _say(f"  before any solve: q {eq0:.2e}  first dQ {edq0:.2e}")
        assert eq0 <= 1e-5 and edq0 <= 1e-5
        assert all(np.all(np.isfinite(rg[k])) for k in ("q", "dq", "gamma"))
        assert np.all(np.isfinite(run.fields()[1]))

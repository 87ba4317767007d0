"""Pins of the oracle's TO machinery, substrates and random numbers.

Filters (Sec. 4.1: compact kernels, zero padding on wall axes, self-adjoint),
sensitivities (App. A: the L2 gradient fixed by the functional-derivative
definition of eq. orthogonality), patterns (eq. O-from-V with c_ii = 1 and
eq. orthogonality), the predictor-corrector relation (eq.
influence-SGS-term-on-LF-QoI-trajectories, exact to second order for
quadratic QoIs), the SGS moment identities of Sec. 3, band weights (eq.
3d-mp-band-weights), Smagorinsky (eq. smag, eq. strain-from-non-equilibrium,
eq. eff-relaxation) and WALE (Sec. 5.2), and the LRS residual draw (eq. LRS).
"""
import os
import subprocess
import sys

import numpy as np
import pytest
from scipy import stats

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILTERS = ["I", "B", "B2", "BMID", "IMB"]


def _fourier_response(name, kx, ky, kz=0.0):
    c = np.cos(kx / 2) ** 2 * np.cos(ky / 2) ** 2 * np.cos(kz / 2) ** 2
    return {"I": 1.0, "B": c, "B2": c * c, "BMID": c - c * c, "IMB": 1 - c}[name]


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("filt", FILTERS)
def test_filter_fourier_response(orc, lat, filt):
    """The binomial [1,2,1]/4 per axis multiplies a periodic Fourier mode by
    prod_a cos^2(k_a/2); the filters are polynomials in B."""
    nx, ny, nz = 16, 12, (8 if lat else 1)
    o = orc.Oracle(lattice=lat, nx=nx, ny=ny, nz=nz)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny, (2 * np.pi / nz if lat else 0.0)
    u = np.cos(kx * xx + ky * yy + kz * zz + 0.3).ravel()
    out = o.filter(filt, u)
    assert np.max(np.abs(out - _fourier_response(filt, kx, ky, kz) * u)) < 1e-14


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("filt", FILTERS)
def test_filter_self_adjoint_with_walls(orc, lat, filt):
    o = orc.Oracle(lattice=lat, nx=9, ny=7, nz=(5 if lat else 1), walls_y=1)
    rng = np.random.default_rng(11)
    a, b = rng.standard_normal(o.N), rng.standard_normal(o.N)
    lhs = o.filter(filt, a) @ b
    rhs = a @ o.filter(filt, b)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_binomial_taps_and_zero_padding(orc):
    """A unit impulse returns the tap table; at the wall row the taps that
    would fall outside are dropped (zero padding), periodic axes wrap."""
    o = orc.Oracle(lattice=0, nx=5, ny=4, walls_y=1)
    u = np.zeros(o.N)
    u[0] = 1.0                               # cell (x=0, y=0)
    out = o.filter("B", u).reshape(4, 5)
    t = np.array([0.25, 0.5, 0.25])
    exp = np.zeros((4, 5))
    for oy in (-1, 0, 1):
        for ox in (-1, 0, 1):
            y = oy
            if 0 <= y < 4:
                exp[y, ox % 5] += t[oy + 1] * t[ox + 1]
    assert np.array_equal(out, exp)
    assert abs(out.sum() - 0.75) < 1e-16     # one row of taps lost to the wall


def _closure_all(orc, lat, ny):
    if lat == 0:
        q = [("E", f, 0) for f in FILTERS] + [("Z", f, 0) for f in FILTERS]
        return orc.make_closure(q)
    q = [(k, f, 0) for f in FILTERS for k in ("E", "Z")] + [("MP", "I", j) for j in range(3)]
    return orc.make_closure(q, nbands=3, dmin=0.5, dmax=ny / 2)


@pytest.mark.parametrize("lat,walls", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_sensitivities_exact_central_difference(orc, lat, walls):
    """For quadratic (and linear) QoIs, (Q(v+p) - Q(v-p))/2 = <dQ/dv, p>
    exactly for any p (the functional-derivative definition)."""
    o = orc.Oracle(lattice=lat, nx=10, ny=8, nz=(6 if lat else 1), walls_y=walls)
    cl = _closure_all(orc, lat, 8)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((o.d, o.N))
    p = rng.standard_normal((o.d, o.N))
    q0, V = o.qoi(cl, v)
    qp, _ = o.qoi(cl, v + p)
    qm, _ = o.qoi(cl, v - p)
    lhs = 0.5 * (qp - qm)
    rhs = np.einsum("kan,an->k", V, p)
    scale = np.abs(qp) + np.abs(qm) + 1
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13
    # Q(v) itself: energy of the identity filter is 1/2 sum |v|^2
    assert abs(q0[0] - 0.5 * np.sum(v * v)) < 1e-12 * q0[0]


def test_mean_profile_qoi_and_bands(orc):
    ny = 24
    o = orc.Oracle(lattice=1, nx=4, ny=ny, nz=3, walls_y=1)
    nb, dmin, dmax = synth.channel_bands(ny)
    w = o.band_weights(nb, dmin, dmax)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-15)       # discrete normalization
    assert np.allclose(w, w[:, ::-1], atol=1e-16)             # symmetric about the centre
    dw = np.minimum(np.arange(ny) + 0.5, ny - 0.5 - np.arange(ny))
    peaks = dw[np.argmax(w[:, : ny // 2], axis=1)]
    assert np.all(np.diff(peaks) >= 0)                        # centres move away from the wall
    lc = np.linspace(np.log(dmin), np.log(dmax), nb)
    for j in range(nb):                                       # log-normal shape in d_w
        r = w[j, 0] / w[j, 1]
        t0, t1 = (np.log(dw[0]) - lc[j]), (np.log(dw[1]) - lc[j])
        sig = lc[1] - lc[0]
        assert abs(np.log(r) - (-0.5 * (t0 * t0 - t1 * t1) / sig**2)) < 1e-12
    cl = orc.make_closure([("MP", "I", j) for j in range(nb)], nbands=nb, dmin=dmin, dmax=dmax)
    u = synth.channel_velocity(4, ny, 3, seed=1)
    q, V = o.qoi(cl, u)
    ux = u[0].reshape(3, ny, 4)
    prof = ux.sum(axis=(0, 2))
    assert np.allclose(q, w @ prof, rtol=1e-13)


@pytest.mark.parametrize("lat,walls", [(0, 0), (1, 1)])
def test_patterns_orthogonality(orc, lat, walls):
    """<V_k, O_i> = 0 for k != i; c_ii = 1 gives <V_i, O_i> = 1/(G^-1)_ii;
    the TO correction reduces to dv = sum_j (G^-1 dQ)_j V_j."""
    ny = 16
    o = orc.Oracle(lattice=lat, nx=12, ny=ny, nz=(6 if lat else 1), walls_y=walls)
    if lat == 0:
        cl = orc.make_closure(synth.QOIS_2D)
    else:
        cl = orc.make_closure(synth.QOIS_3D, nbands=6, dmin=0.5, dmax=ny / 2)
    rng = np.random.default_rng(8)
    v = 0.01 * rng.standard_normal((o.d, o.N))
    r = o.patterns(cl, v)
    assert not r["singular"]
    V, O, G = r["V"], r["O"], r["G"]
    nq = cl.nq
    M = np.einsum("kan,ian->ki", V, O)
    off = M - np.diag(np.diag(M))
    assert np.max(np.abs(off)) < 1e-11 * np.max(np.abs(np.diag(M)))
    Gi = np.linalg.inv(G)
    assert np.allclose(np.diag(M), 1 / np.diag(Gi), rtol=1e-10)
    assert np.allclose(r["den"], np.diag(M), rtol=1e-12)
    dq = 1e-3 * rng.standard_normal(nq) * np.abs(r["q"])
    dv, gamma, sing = o.to_correction(cl, v, dq)
    assert not sing
    assert np.allclose(gamma, dq * np.diag(Gi), rtol=1e-9)
    beta = np.linalg.solve(G, dq)
    dv2 = np.einsum("k,kan->an", beta, V)
    assert np.max(np.abs(dv - dv2)) < 1e-9 * np.max(np.abs(dv2))


@pytest.mark.parametrize("lat,walls", [(0, 0), (1, 1)])
def test_first_order_control_exact_to_second_order(orc, lat, walls):
    """Q_k(v* + dv) - q*_k - dQ_k = Q_k(dv) for quadratic QoIs and 0 for the
    linear mean-profile QoIs (eq. influence-SGS-term-on-LF-QoI-trajectories)."""
    ny = 16
    o = orc.Oracle(lattice=lat, nx=12, ny=ny, nz=(6 if lat else 1), walls_y=walls)
    if lat == 0:
        cl = orc.make_closure(synth.QOIS_2D)
    else:
        cl = orc.make_closure(synth.QOIS_3D, nbands=6, dmin=0.5, dmax=ny / 2)
    rng = np.random.default_rng(9)
    v = 0.01 * rng.standard_normal((o.d, o.N))
    q, _ = o.qoi(cl, v)
    dq = 0.02 * rng.standard_normal(cl.nq) * np.abs(q)
    dv, _, _ = o.to_correction(cl, v, dq)
    q1, _ = o.qoi(cl, v + dv)
    qd, _ = o.qoi(cl, dv)
    kinds = [cl.kind[k] for k in range(cl.nq)]
    for k in range(cl.nq):
        expect = 0.0 if kinds[k] == 2 else qd[k]
        assert abs(q1[k] - q[k] - dq[k] - expect) < 1e-10 * (abs(q[k]) + 1e-30)


def test_gram_singular_rule(orc):
    """A uniform field has (I - B) v = 0: the Gram matrix is singular and the
    correction is skipped."""
    o = orc.Oracle(lattice=0, nx=8, ny=8)
    cl = orc.make_closure([("E", "B", 0), ("E", "IMB", 0)])
    v = np.zeros((2, o.N))
    v[0] = 0.01
    dv, gamma, sing = o.to_correction(cl, v, np.array([1e-6, 1e-6]))
    assert sing and np.all(dv == 0) and np.all(gamma == 0)


def test_largest_closure_gram_conditioning(orc):
    """The Gram matrix of the 16-QoI closure (E and Z of B, B^2, B - B^2 and
    I - B, eight overlapping mean-profile bands), scaled to unit diagonal,
    is ill-conditioned at the first corrected step of the 20 x 24 x 12
    channel: a condition number above 1e7 (the four filter forms are nearly
    dependent), where the standard 12-QoI set ({E, Z} x {B^2, B - B^2,
    I - B}, six bands) stays below 1e6.  This fixes how far the FP32 path
    can follow the oracle through the solve on that closure."""
    cfg, u0, qois, cargs = synth.largest_closure_workload()
    o = orc.Oracle(**cfg)
    o.init(u0)
    o.step(cargs["spinup"] + 1)
    _, v = o.post_collision_velocity()

    def cond(q, nb):
        cl = orc.make_closure(q, nbands=nb, dmin=cargs["dmin"], dmax=cargs["dmax"])
        G = o.patterns(cl, v)["G"]
        d = np.sqrt(np.diag(G))
        return float(np.linalg.cond(G / np.outer(d, d)))

    assert cond(qois, 8) > 1e7 and cond(synth.QOIS_3D, 6) < 1e6


@pytest.mark.parametrize("lat", [0, 1])
def test_sgs_moment_identities_in_step(orc, lat):
    """The SGS correction changes f^p by feq(rho, v*+dv) - feq(rho, v*): mass
    neutral and momentum rho dv (Sec. 3)."""
    ny = 16
    kw = dict(lattice=lat, nx=10, ny=ny, nz=(6 if lat else 1), tau=0.6, force_kind=2, force_amp=1e-5)
    if lat == 1:
        kw["walls_y"] = 1
    a, b = orc.Oracle(**kw), orc.Oracle(**kw)
    u0 = synth.noise_velocity(a.d, a.shape, 0.01, 12)
    a.init(u0)
    b.init(u0)
    qs = synth.QOIS_2D if lat == 0 else synth.QOIS_3D
    cl = orc.make_closure(qs, mode="track", nbands=6, dmin=0.5, dmax=ny / 2)
    # reference: the predictor QoIs scaled by 1.01
    rho, v = a.velocity()
    vs = v.copy()
    vs[0] += 1e-5 / rho
    q, _ = a.qoi(cl, vs)
    qref = (1.01 * q)[None, :]
    a.set_closure(cl, qref=qref)
    a.step(1)
    b.step(1)
    dv, gamma, sing = a.to_correction(cl, vs, qref[0] - q)
    assert not sing
    df = a.get_fp() - b.get_fp()
    c, _ = orc.lattice(lat)
    c = c[:, : a.d].astype(float)
    assert np.max(np.abs(df.sum(axis=0))) < 1e-15
    mom = c.T @ df
    # f^p is O(0.1): the difference of the two runs carries ~1e-17 rounding
    assert np.max(np.abs(mom - rho * dv)) < 1e-15 + 1e-10 * np.max(np.abs(rho * dv))
    rec = a.record_arrays()
    assert np.allclose(rec["q"][0], q, rtol=1e-13)
    assert np.allclose(rec["q"][0] + rec["dq"][0], qref[0], rtol=1e-13)
    assert np.allclose(rec["gamma"][0], gamma, rtol=1e-10)


def test_smagorinsky_closed_form(orc):
    """tau_eff solves the implicit relation of eq. eff-relaxation with
    nu_t = C^2 sqrt(2 S:S) and S = -Pi/(2 rho c_s^2 tau_eff)."""
    rng = np.random.default_rng(3)
    for lat in (0, 1):
        c, w = orc.lattice(lat)
        d = 2 if lat == 0 else 3
        c = c[:, :d].astype(float)
        for _ in range(5):
            rho = 1 + 0.01 * rng.standard_normal()
            u = 0.05 * rng.standard_normal(d)
            f = orc.feq_cells(lat, rho, u) + 1e-3 * w * rng.standard_normal(len(w))
            rho = f.sum()
            u = c.T @ f / rho
            # second moment of the equilibrium from the lattice isotropy
            Pi = np.einsum("i,ia,ib->ab", f, c, c) - (rho / 3 * np.eye(d) + rho * np.outer(u, u))
            for C in (0.0, 0.1, 0.2):
                t = orc.tau_smag(lat, 0.52, C, f, rho, u)
                S = -Pi / (2 * rho * t / 3)
                nut = C * C * np.sqrt(2 * np.sum(S * S))
                assert abs(t - (3 * nut + 0.52)) < 1e-13
                if C == 0.0:
                    assert t == 0.52


def test_wale_special_cases(orc):
    N = 16
    o = orc.Oracle(lattice=1, nx=N, ny=N, nz=4, tau=0.51, substrate=2, cmodel=0.5)
    zz, yy, xx = np.meshgrid(np.arange(4), np.arange(N), np.arange(N), indexing="ij")
    k = 2 * np.pi / N
    # pure shear: g^2 = 0, so S^d = 0 and nu_t = 0
    v = np.zeros((3, o.N))
    v[0] = 0.01 * np.sin(k * yy).ravel()
    assert np.all(o.tau_wale(v) == 0.51)
    # rotation-dominated field: at the origin the central-difference gradient
    # is a pure rotation with rate W = 0.01 sin(k): S = 0, S^d:S^d = 2W^4/3,
    # so nu_t = C^2 (2/3)^(1/4) W
    v = np.zeros((3, o.N))
    v[0] = (-0.01 * np.sin(k * yy)).ravel()
    v[1] = (0.01 * np.sin(k * xx)).ravel()
    t = o.tau_wale(v)
    W = 0.01 * np.sin(k)
    assert abs(t[0] - (0.51 + 3 * 0.25 * (2 / 3) ** 0.25 * W)) < 1e-15
    # degree-one homogeneity in the velocity gradient
    rng = np.random.default_rng(4)
    v = 0.01 * rng.standard_normal((3, o.N))
    t1, t2 = o.tau_wale(v) - 0.51, o.tau_wale(3 * v) - 0.51
    assert np.allclose(t2, 3 * t1, rtol=1e-11, atol=1e-18)


def test_philox_known_answers(orc):
    path = os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert orc.philox(v[0:4], v[4:6]).tolist() == v[6:10]
        n += 1
    assert n == 3


def test_lrs_normals_distribution(orc):
    z = np.concatenate([orc.lrs_normals(1234, s, 12) for s in range(20000)])
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    Z = z.reshape(-1, 12)
    cc = np.corrcoef(Z.T)
    assert np.max(np.abs(cc - np.eye(12))) < 5 / np.sqrt(Z.shape[0])


def _lrs_run(orc, C, Sigma, scale=None, steps=60, spinup=10):
    o = orc.Oracle(lattice=0, nx=16, ny=16, tau=0.6, force_kind=1, force_amp=1e-5, force_k=1)
    o.init(synth.noise_velocity(2, o.shape, 1e-3, 21))
    cl = orc.make_closure(synth.QOIS_2D, mode="lrs", spinup=spinup, C=C, mu=np.zeros(2),
                          Sigma=Sigma, scale=scale, seed=77)
    o.set_closure(cl)
    o.step(steps)
    return o, o.record_arrays()


def test_lrs_special_cases(orc):
    nq = 2
    # persistence model C = [I; 0] with Sigma = 0: no correction at all
    C = np.vstack([np.eye(nq), np.zeros((1, nq))])
    _, r = _lrs_run(orc, C, np.zeros((nq, nq)))
    assert np.all(np.abs(r["dq"]) <= 4e-16 * np.abs(r["q"]))   # s (q*/s) - q* rounding only
    # bias only with a given scale: dQ = s * b, constant after spin-up
    b = np.array([0.01, -0.02])
    s = np.array([3.0, 5.0])
    C = np.vstack([np.eye(nq), b[None, :]])
    _, r = _lrs_run(orc, C, np.zeros((nq, nq)), scale=s)
    assert np.all(r["dq"][:10] == 0)
    assert np.allclose(r["dq"][10:], s * b, rtol=1e-12)
    # bias only, scale taken from |q*| at the switch-on step
    o, r = _lrs_run(orc, C, np.zeros((nq, nq)))
    s0 = np.abs(r["q"][10])
    assert np.allclose(o.scale(), s0, rtol=0)
    assert np.allclose(r["dq"][10:], s0 * b, rtol=1e-12)


def test_lrs_residual_statistics(orc):
    """dQ / s of the persistence model with noise is a draw of N(0, Sigma)."""
    nq = 2
    C = np.vstack([np.eye(nq), np.zeros((1, nq))])
    Sigma = np.array([[4e-6, 1e-6], [1e-6, 2e-6]])
    o, r = _lrs_run(orc, C, Sigma, steps=3000, spinup=0)
    assert not np.any(r["flags"])
    e = r["dq"] / o.scale()
    n = e.shape[0]
    assert np.all(np.abs(e.mean(axis=0)) < 4 * np.sqrt(np.diag(Sigma) / n))
    S = np.cov(e.T)
    assert np.all(np.abs(S - Sigma) < 5 * np.sqrt((Sigma**2 + np.outer(np.diag(Sigma), np.diag(Sigma))) / n))


def test_tracking_hits_reference_to_second_order(orc):
    ny = 12
    kw = dict(lattice=0, nx=32, ny=ny * 2, tau=0.6, force_kind=1, force_amp=1e-5, force_k=1)
    o = orc.Oracle(**kw)
    u0 = synth.noise_velocity(2, o.shape, 1e-3, 31)
    o.init(u0)
    qref = np.tile(np.array([[2e-4, 5e-6]]), (30, 1)) * np.linspace(1, 1.3, 30)[:, None]
    cl = orc.make_closure(synth.QOIS_2D, mode="track")
    o.set_closure(cl, qref=qref)
    o.step(30)
    r = o.record_arrays()
    assert np.allclose(r["q"] + r["dq"], qref, rtol=1e-12)


def test_oracle_deterministic_across_thread_counts(orc, tmp_path):
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r)\n"
        "import oracle, synth\n"
        "o = oracle.Oracle(lattice=1, nx=12, ny=16, nz=6, walls_y=1, tau=0.51, substrate=1, cmodel=0.1,"
        " force_kind=2, force_amp=1e-5)\n"
        "o.init(synth.channel_velocity(12, 16, 6, seed=3))\n"
        "C, mu, S = synth.lrs_model_channel(12, 7, 9)\n"
        "o.set_closure(oracle.make_closure(synth.QOIS_3D, mode='lrs', spinup=3, C=C, mu=mu, Sigma=S,"
        " nbands=6, dmin=0.5, dmax=8.0, seed=5))\n"
        "o.step(8)\n"
        "np.save(sys.argv[1], np.concatenate([o.get_fp().ravel(), o.record_arrays()['q'].ravel()]))\n"
    ) % ROOT
    outs = []
    for nt in ("1", "3"):
        p = str(tmp_path / f"o{nt}.npy")
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        subprocess.check_call([sys.executable, "-c", code, p], env=env)
        outs.append(np.load(p))
    assert np.array_equal(outs[0], outs[1])


def test_reverse_sums_diagnostic_changes_only_the_summation_order(orc):
    """The reverse-order diagnostic (the FP64 resolution twin of the parity
    tests): QoIs of a field whose every term and partial sum is exact agree
    bitwise in both orders; on a general field they agree to rounding."""
    import synth
    cfg, _ = synth.channel_workload(10, 8, 6)
    qois = synth.QOIS_3D
    cl = orc.make_closure(qois, nbands=6, dmin=0.5, dmax=4.0)
    o = orc.Oracle(**cfg)
    rng = np.random.default_rng(3)
    exact = rng.integers(-8, 9, size=(3, o.N)) * 2.0 ** -6      # dyadic: exact sums
    general = rng.standard_normal((3, o.N))
    for v, exact_sum in ((exact, True), (general, False)):
        q0 = o.qoi(cl, v)[0]
        o.set_reverse_sums(True)
        q1 = o.qoi(cl, v)[0]
        o.set_reverse_sums(False)
        if exact_sum:   # dyadic fields, binomial filters and central differences: exact sums
            assert np.array_equal(q0[:6], q1[:6])
        assert np.allclose(q0, q1, rtol=1e-13, atol=0)


def test_reduced_form_diagnostic_equals_the_literal_patterns(orc):
    """The reduced-form diagnostic (sum_j (G^-1 dQ)_j V_j, gamma_k =
    dQ_k (G^-1)_kk) is the literal correction of eq. O-from-V and
    eq. tau-from-dQ-for-tracking in another exact form: on a well-conditioned
    2-D closure the two runs agree to rounding over many steps, and their
    records carry the same dQ at the first corrected step."""
    import synth
    cfg, _ = synth.kolmogorov_workload(24, tau=0.55, seed=4)
    u0 = synth.turbulent_velocity_2d(24, 0.02, seed=4)
    C, mu, S = synth.lrs_model(2, 3, 4, 5)
    cl = dict(mode="lrs", spinup=2, C=C, mu=mu, Sigma=S, seed=9)
    runs = []
    for reduced in (False, True):
        o = orc.Oracle(**cfg)
        o.init(u0)
        o.set_closure(orc.make_closure(synth.QOIS_2D, **cl))
        o.set_reduced_form(reduced)
        o.step(40)
        runs.append(o)
    ra, rb = runs[0].record_arrays(), runs[1].record_arrays()
    assert np.array_equal(ra["dq"][2], rb["dq"][2]) and np.any(ra["dq"][2] != 0)
    assert np.allclose(ra["gamma"], rb["gamma"], rtol=1e-10, atol=0)
    va, vb = runs[0].velocity()[1], runs[1].velocity()[1]
    assert np.max(np.abs(va - vb)) <= 1e-13 * np.max(np.abs(va))

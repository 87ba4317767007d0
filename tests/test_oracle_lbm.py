"""Pins of the oracle's LBM core against what the paper and the mathematics fix.

Lattice isotropy and equilibrium moments (Sec. 2, BGK footnote), streaming
and halfway bounce-back maps (eq. LES-3, Sec. 7.1), conservation and the
exact-difference force (eq. collide-and-stream), the uniform fixed point,
Taylor-Green decay with nu = c_s^2 (tau - 1/2) (Sec. 2), and two exact steady
solutions of BGK + exact-difference forcing + halfway bounce-back: the
Poiseuille profile and the steady sine shear.
"""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("lat", [0, 1])
def test_lattice_isotropy(orc, lat):
    c, w = orc.lattice(lat)
    d = 2 if lat == 0 else 3
    c = c[:, :d].astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(d) / 3.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    I = np.eye(d)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.allclose(m4, iso, atol=1e-16)
    # every velocity has its opposite
    for ci in c:
        assert any(np.array_equal(-ci, cj) for cj in c)


@pytest.mark.parametrize("lat", [0, 1])
def test_equilibrium_moments(orc, lat):
    c, w = orc.lattice(lat)
    d = 2 if lat == 0 else 3
    c = c[:, :d].astype(float)
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(d)
        f = orc.feq_cells(lat, rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.allclose(c.T @ f, rho * u, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.allclose(P, rho / 3.0 * np.eye(d) + rho * np.outer(u, u), atol=1e-15)


@pytest.mark.parametrize("lat,walls", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_stream_index_map_brute_force(orc, lat, walls):
    """Tagged-ID streaming: each population carries its own (i, cell) label."""
    nx, ny, nz = 5, 4, (3 if lat == 1 else 1)
    o = orc.Oracle(lattice=lat, nx=nx, ny=ny, nz=nz, walls_y=walls, tau=0.8)
    Q, N = o.Q, o.N
    fp = np.arange(Q * N, dtype=np.float64).reshape(Q, N)
    o.set_fp(fp)
    o.stream_only()
    out = o.get_fp()
    c, _ = orc.lattice(lat)
    opp = [next(j for j in range(Q) if np.array_equal(c[j], -c[i])) for i in range(Q)]
    for i in range(Q):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    xc = x + nx * (y + ny * z)
                    sx, sy, sz = x - c[i, 0], y - c[i, 1], z - c[i, 2]
                    if walls and not (0 <= sy < ny):
                        expect = fp[opp[i], xc]
                    else:
                        sc = (sx % nx) + nx * ((sy % ny) + ny * (sz % nz))
                        expect = fp[i, sc]
                    assert out[i, xc] == expect


@pytest.mark.parametrize("lat", [0, 1])
def test_uniform_fixed_point(orc, lat):
    o = orc.Oracle(lattice=lat, nx=6, ny=5, nz=4, tau=0.7)
    u = np.zeros((o.d, o.N))
    u[0], u[1] = 0.01, -0.02
    o.init(u)
    f0 = o.get_fp()
    o.step(20)
    assert np.max(np.abs(o.get_fp() - f0)) < 1e-15


@pytest.mark.parametrize("lat", [0, 1])
def test_conservation_periodic(orc, lat):
    o = orc.Oracle(lattice=lat, nx=10, ny=8, nz=6, tau=0.55)
    u0 = synth.noise_velocity(o.d, o.shape, 0.02, 3)
    o.init(u0)
    o.step(200)
    r = o.record_arrays()
    assert np.max(np.abs(r["mass"] - r["mass"][0])) / r["mass"][0] < 1e-13
    assert np.max(np.abs(r["mom"] - r["mom"][0])) < 1e-13 * r["mass"][0]


@pytest.mark.parametrize("lat", [0, 1])
def test_constant_force_adds_exact_momentum(orc, lat):
    A = 3e-6
    o = orc.Oracle(lattice=lat, nx=8, ny=6, nz=4, tau=0.6, force_kind=2, force_amp=A)
    o.init(synth.noise_velocity(o.d, o.shape, 0.01, 4))
    o.step(50)
    r = o.record_arrays()
    dm = np.diff(r["mom"][:, 0])
    assert np.max(np.abs(dm - o.N * A)) < 1e-12 * o.N * A + 1e-15
    assert np.max(np.abs(np.diff(r["mom"][:, 1]))) < 1e-15


def test_wall_mass_conservation(orc):
    o = orc.Oracle(lattice=1, nx=8, ny=6, nz=4, walls_y=1, tau=0.6, force_kind=2, force_amp=1e-5)
    o.init(synth.noise_velocity(3, o.shape, 0.01, 5))
    o.step(100)
    m = o.record_arrays()["mass"]
    assert np.max(np.abs(m - m[0])) / m[0] < 1e-13


def _tg_rate(orc, N, tau, lat=0):
    k = 2 * np.pi / N
    o = orc.Oracle(lattice=lat, nx=N, ny=N, nz=2, tau=tau)
    zz, yy, xx = np.meshgrid(np.arange(o.shape[0]), np.arange(N), np.arange(N), indexing="ij")
    U0 = 1e-4
    mode = (np.cos(k * xx) * np.sin(k * yy)).ravel()
    u = np.zeros((o.d, o.N))
    u[0] = U0 * mode
    u[1] = -U0 * (np.sin(k * xx) * np.cos(k * yy)).ravel()
    o.init(u)
    t1, t2 = 40, 40 + int(0.3 / ((tau - 0.5) / 3 * 2 * k * k))
    o.step(t1)
    a1 = o.velocity()[1][0] @ mode / (mode @ mode)
    o.step(t2 - t1)
    a2 = o.velocity()[1][0] @ mode / (mode @ mode)
    rate = -np.log(a2 / a1) / (t2 - t1)
    nu = (tau - 0.5) / 3.0
    return rate, 2 * nu * k * k


@pytest.mark.parametrize("lat", [0, 1])
def test_taylor_green_decay(orc, lat):
    r64, e64 = _tg_rate(orc, 64, 0.6, lat)
    err64 = abs(r64 / e64 - 1)
    assert err64 < 0.01
    if lat == 0:
        r128, e128 = _tg_rate(orc, 128, 0.6, lat)
        err128 = abs(r128 / e128 - 1)
        assert err128 < err64 / 2.5  # second-order convergence


@pytest.mark.parametrize("lat,tau", [(0, 0.6), (0, 0.8), (0, 1.0), (0, 0.933), (1, 0.8)])
def test_poiseuille_exact(orc, lat, tau):
    """Steady BGK + exact-difference force + halfway bounce-back channel:
    v(y) = 3F/(2tau-1) (y+1/2)(N-1/2-y) + F(16tau^2-20tau+3)/(4(2tau-1))
    for the moment velocity on N fluid rows (exact for the discrete scheme
    up to O(u^2))."""
    N, F = 12, 1e-8
    o = orc.Oracle(lattice=lat, nx=4, ny=N, nz=2, walls_y=1, tau=tau, force_kind=2, force_amp=F)
    o.init(np.zeros((o.d, o.N)))
    o.step(int(12 * N * N / ((tau - 0.5) / 3)))
    ux = o.velocity()[1][0].reshape(o.shape)[0, :, 0]
    y = np.arange(N)
    ex = 3 * F / (2 * tau - 1) * (y + 0.5) * (N - 0.5 - y) + F * (16 * tau**2 - 20 * tau + 3) / (4 * (2 * tau - 1))
    assert np.max(np.abs(ux - ex)) / np.max(ex) < 5e-9


@pytest.mark.parametrize("tau,N,kk", [(0.8, 16, 2), (0.55, 32, 4)])
def test_steady_sine_shear_exact(orc, tau, N, kk):
    """F_x = F sin(kappa y), periodic: moment amplitude
    U = F (2D/w + a)/(D - w a), w = 1/tau, a = w - 1 + cos kappa,
    D = a^2 + sin^2 kappa; its small-kappa limit is F/(nu kappa^2)."""
    F = 1e-8
    o = orc.Oracle(lattice=0, nx=4, ny=N, tau=tau, force_kind=1, force_amp=F, force_k=kk)
    o.init(np.zeros((2, o.N)))
    nu, kap = (tau - 0.5) / 3, 2 * np.pi * kk / N
    o.step(int(30 / (nu * kap * kap)))
    ux = o.velocity()[1][0].reshape(o.shape)[0, :, 0]
    w = 1 / tau
    a = w - 1 + np.cos(kap)
    D = a * a + np.sin(kap) ** 2
    U = F * (2 * D / w + a) / (D - w * a)
    assert np.max(np.abs(ux - U * np.sin(kap * np.arange(N)))) / U < 5e-9
    assert abs(U / (F / (nu * kap * kap)) - 1) < 0.15


def test_instability_flag(orc):
    o = orc.Oracle(lattice=0, nx=16, ny=16, tau=0.5005, force_kind=1, force_amp=5e-3, force_k=1)
    o.init(synth.noise_velocity(2, o.shape, 0.05, 7))
    o.step(400)
    flags = o.record_arrays()["flags"]
    assert flags[0] == 0
    assert (flags & 1).any()


def test_diag_energy_enstrophy_closed_form(orc):
    """E = 1/2 sum |v|^2 and Z = 1/2 sum (D_x v_y - D_y v_x)^2 of the first
    post-streaming state of f = feq(1, u) with u = (U0 sin(ky), 0).  Streaming
    the equilibrium of a shear mode gives exactly rho = 1 and
    v_x = U0 sin(ky) (2 + cos k)/3 (the quadratic terms cancel between the
    D2Q9 weights), and the central difference contributes a factor sin(k)."""
    N = 32
    o = orc.Oracle(lattice=0, nx=N, ny=N, tau=0.8)
    k = 2 * np.pi * 3 / N
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u = np.zeros((2, N * N))
    U0 = 1e-3
    u[0] = U0 * np.sin(k * yy).ravel()
    o.init(u)
    o.step(1)
    r = o.record_arrays()
    g = (2 + np.cos(k)) / 3
    E = 0.25 * (U0 * g) ** 2 * N * N
    Z = 0.25 * (U0 * g * np.sin(k)) ** 2 * N * N
    assert abs(r["diag_e"][0] - E) < 1e-12 * E
    assert abs(r["diag_z"][0] - Z) < 1e-12 * Z
    assert abs(r["mass"][0] - N * N) < 1e-12 * N * N


@pytest.mark.parametrize("lat", [0, 1])
def test_fp32_store_diagnostic_rounds_only_the_stored_state(orc, lat):
    """The FP32 storage diagnostic (used to measure the floor that FP32
    storage alone sets): with it on, every stored deviation f - w of the
    post-collision populations is an FP32 number, close to the unrounded
    step; with it off the run is the plain FP64 one."""
    if lat == 0:
        cfg, u0 = synth.kolmogorov_workload(24, tau=0.6, seed=3)
    else:
        cfg, u0 = synth.channel_workload(10, 8, 6)
    _, w = orc.lattice(lat)
    a = orc.Oracle(**cfg)
    a.init(u0)
    a.set_fp32_store(True)
    b = orc.Oracle(**cfg)
    b.init(u0)
    a.step(1)
    b.step(1)
    ga, gb = a.get_fp() - w[:, None], b.get_fp() - w[:, None]
    assert np.array_equal(ga, ga.astype(np.float32).astype(np.float64))
    # (v* is rounded too, before it enters the equilibrium, so a step moves by
    # more than the final rounding alone, but only at the FP32 level)
    assert np.max(np.abs(ga - gb)) <= 1e-6 * np.max(np.abs(gb))
    assert not np.array_equal(ga, gb)
    c = orc.Oracle(**cfg)
    c.init(u0)
    c.set_fp32_store(True)
    c.set_fp32_store(False)
    c.step(1)
    assert np.array_equal(c.get_fp(), b.get_fp())


@pytest.mark.parametrize("a,b", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_diag_energy_enstrophy_closed_form_3d(orc, a, b):
    """3-D counterpart of the 2-D closed form: D3Q19 on a periodic
    12 x 10 x 8 box, f = feq(1, u) with the single shear mode
    u_a = U0 sin(k x_b) (every ordered pair a != b, so that each of the six
    derivative terms of the 3-D curl is exercised once).  One stream step
    gives rho = 1 and v_a = U0 sin(k x_b) (2 + cos k)/3 exactly (the
    quadratic equilibrium terms cancel within the D3Q19 weight classes), so
    E = 1/4 N (U0 g)^2 and Z = 1/4 N (U0 g sin k)^2, the central difference
    of sin(k x_b) being sin(k) cos(k x_b)."""
    dims = (12, 10, 8)
    o = orc.Oracle(lattice=1, nx=dims[0], ny=dims[1], nz=dims[2], walls_y=0, tau=0.8)
    N = dims[0] * dims[1] * dims[2]
    k = 2 * np.pi * 2 / dims[b]
    zz, yy, xx = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    coord = (xx, yy, zz)[b].ravel()
    u = np.zeros((3, N))
    U0 = 1e-3
    u[a] = U0 * np.sin(k * coord)
    o.init(u)
    o.step(1)
    r = o.record_arrays()
    g = (2 + np.cos(k)) / 3
    E = 0.25 * (U0 * g) ** 2 * N
    Z = 0.25 * (U0 * g * np.sin(k)) ** 2 * N
    assert abs(r["diag_e"][0] - E) < 1e-12 * E
    assert abs(r["diag_z"][0] - Z) < 1e-12 * Z
    assert abs(r["mass"][0] - N) < 1e-12 * N


def test_curl_3d_closed_form(orc):
    """The 3-D central-difference curl of a sum of six shear modes with six
    different amplitudes, v_x = A sin(ky y) + A' sin(kz z),
    v_y = B sin(kz z) + B' sin(kx x), v_z = C sin(kx x) + C' sin(ky y), on a
    periodic 12 x 10 x 8 box, against its exact value cell by cell:
    w_x = C' sy cos(ky y) - B sz cos(kz z), w_y = A' sz cos(kz z) - C sx cos(kx x),
    w_z = B' sx cos(kx x) - A sy cos(ky y), with s = sin k.  Each term has its
    own amplitude, so a wrong sign, axis or component fails it."""
    dims = (12, 10, 8)
    o = orc.Oracle(lattice=1, nx=dims[0], ny=dims[1], nz=dims[2], walls_y=0, tau=0.8)
    zz, yy, xx = [c.ravel() for c in np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")]
    kx, ky, kz = (2 * np.pi * m / n for m, n in zip((1, 2, 3), dims))
    A, A2, B, B2, C, C2 = 1.0, 0.3, -0.7, 0.45, 0.2, -1.3
    v = np.stack([A * np.sin(ky * yy) + A2 * np.sin(kz * zz),
                  B * np.sin(kz * zz) + B2 * np.sin(kx * xx),
                  C * np.sin(kx * xx) + C2 * np.sin(ky * yy)])
    sx, sy, sz = np.sin(kx), np.sin(ky), np.sin(kz)
    want = np.stack([C2 * sy * np.cos(ky * yy) - B * sz * np.cos(kz * zz),
                     A2 * sz * np.cos(kz * zz) - C * sx * np.cos(kx * xx),
                     B2 * sx * np.cos(kx * xx) - A * sy * np.cos(ky * yy)])
    w = o.curl(v)
    assert np.max(np.abs(w - want)) < 1e-14

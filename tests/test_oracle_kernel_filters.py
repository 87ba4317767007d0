"""Pins of the oracle's kernel filters of Sec. 4.1: the truncated Gaussian
G_s (eq. gaussian: alpha = 4 in 2-D, 2 in 3-D) and the dilated biharmonic
cross L_s (eq. laplace, normalised to sum |L_s| = 2), with zero padding on
wall axes; and the QoI sensitivities under them (App. A)."""
import numpy as np
import pytest

KERNELS = ["G3", "L3", "L1"]


def _g1(s, alpha):
    r = np.arange(-alpha * s, alpha * s + 1)
    g = np.exp(-r * r / (2.0 * s * s))
    return g / g.sum()


@pytest.mark.parametrize("lat", [0, 1])
def test_gaussian_is_the_product_of_one_dimensional_gaussians(orc, lat):
    """exp(-|r|^2/2s^2) factors over the axes and so does its sum over the
    cube: G_s is the outer product of the normalised 1-D truncated Gaussian."""
    o = orc.Oracle(lattice=lat, nx=30, ny=30, nz=(16 if lat else 1))
    alpha = 2 if lat else 4
    g = _g1(3, alpha)
    want = np.multiply.outer(np.multiply.outer(g, g), g) if lat else np.multiply.outer(g, g)
    k = o.kernel("G3")
    assert k.shape == want.shape
    assert np.allclose(k, want, rtol=1e-13, atol=1e-18)


def test_biharmonic_cross_and_dilation(orc):
    """L_1 is l = [1,-4,6,-4,1] along each axis through the origin; L_3 is
    L_1 with every entry widened to a 3x3 block (Kronecker product with
    ones); both scaled to sum |L| = 2."""
    o = orc.Oracle(lattice=0, nx=40, ny=40)
    L1 = np.zeros((5, 5))
    L1[2, :] += [1, -4, 6, -4, 1]
    L1[:, 2] += [1, -4, 6, -4, 1]
    assert np.allclose(o.kernel("L1"), 2 * L1 / np.abs(L1).sum(), rtol=0, atol=1e-16)
    L3 = np.kron(L1, np.ones((3, 3)))
    assert np.allclose(o.kernel("L3"), 2 * L3 / np.abs(L3).sum(), rtol=0, atol=1e-16)
    o3 = orc.Oracle(lattice=1, nx=20, ny=20, nz=20)
    for name in ("L1", "L3"):
        k = o3.kernel(name)
        assert abs(np.abs(k).sum() - 2) < 1e-14 and abs(k.sum()) < 1e-15


@pytest.mark.parametrize("lat", [0, 1])
def test_gaussian_fourier_mode(orc, lat):
    """A periodic Fourier mode is an eigenfunction with eigenvalue
    prod_a sum_r g(r) cos(k_a r)."""
    n = 24
    o = orc.Oracle(lattice=lat, nx=n, ny=n, nz=(n if lat else 1))
    nz = n if lat else 1
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    k = 2 * np.pi * np.array([2, 1, 3 if lat else 0]) / n
    u = (np.cos(k[0] * xx + 0.2) * np.cos(k[1] * yy - 0.4) * np.cos(k[2] * zz + 0.1)).ravel()
    g = _g1(3, 2 if lat else 4)
    r = np.arange(len(g)) - len(g) // 2
    lam = np.prod([np.sum(g * np.cos(ka * r)) for ka in k[:(3 if lat else 2)]])
    assert np.max(np.abs(o.filter("G3", u) - lam * u)) < 1e-14


@pytest.mark.parametrize("s", [1, 3])
def test_biharmonic_response_and_cubic_annihilation(orc, s):
    """On a mode along x the y and z arms see a constant (sum l = 0), so the
    eigenvalue is the scaled 1-D biharmonic response (2 sin(k s/2))^4 times
    the box response; cubic polynomials in x are annihilated away from the
    periodic seam."""
    n = 60
    o = orc.Oracle(lattice=1, nx=n, ny=8, nz=8)
    zz, yy, xx = np.meshgrid(np.arange(8), np.arange(8), np.arange(n), indexing="ij")
    kx = 2 * np.pi * 4 / n
    u = np.cos(kx * xx + 0.3).ravel()
    L1 = np.zeros((5, 5, 5))
    for a in range(3):
        idx = [2, 2, 2]
        for j, c in enumerate([1, -4, 6, -4, 1]):
            idx[a] = j
            L1[tuple(idx)] += c
    norm = 2.0 / np.abs(np.kron(L1, np.ones((s, s, s)))).sum()
    box = np.sum(np.cos(kx * (np.arange(s) - (s - 1) / 2)))          # the s-wide block along x
    lam = norm * (2 * np.sin(kx * s / 2)) ** 4 * box * s * s           # s x s blocks across y, z
    out = o.filter(f"L{s}", u)
    assert np.max(np.abs(out - lam * u)) < 1e-13
    p = ((xx - n / 2) / 10.0) ** 3 - 0.5 * ((xx - n / 2) / 10.0)
    outp = o.filter(f"L{s}", p.ravel()).reshape(p.shape)
    R = (5 * s - 1) // 2
    inner = slice(R + 1, n - R - 1)
    assert np.max(np.abs(outp[:, :, inner])) < 1e-12


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("name", KERNELS)
def test_kernel_filters_self_adjoint_with_walls(orc, lat, name):
    o = orc.Oracle(lattice=lat, nx=17, ny=15, nz=(16 if lat else 1), walls_y=1)
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(o.N), rng.standard_normal(o.N)
    lhs = o.filter(name, a) @ b
    rhs = a @ o.filter(name, b)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("lat,walls", [(0, 1), (1, 1), (1, 0)])
def test_kernel_filter_sensitivities_exact(orc, lat, walls):
    """(Q(v+p) - Q(v-p))/2 = <dQ/dv, p> exactly for E and Z under G_3, L_3, L_1."""
    o = orc.Oracle(lattice=lat, nx=16, ny=14, nz=(15 if lat else 1), walls_y=walls)
    q = [(kind, f, 0) for f in KERNELS for kind in ("E", "Z")]
    cl = orc.make_closure(q)
    rng = np.random.default_rng(6)
    v = rng.standard_normal((o.d, o.N))
    p = rng.standard_normal((o.d, o.N))
    _, V = o.qoi(cl, v)
    qp, _ = o.qoi(cl, v + p)
    qm, _ = o.qoi(cl, v - p)
    lhs = 0.5 * (qp - qm)
    rhs = np.einsum("kan,an->k", V, p)
    assert np.max(np.abs(lhs - rhs) / (np.abs(qp) + np.abs(qm) + 1)) < 1e-13

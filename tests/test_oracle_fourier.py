"""Pins of the oracle's sharp Fourier band filter R_[l,m] (eq.
scale-aware-energy-fourier; periodic grids): a mode inside the band is kept
exactly and one outside removed, the filter is a self-adjoint projection,
adjacent bands partition the identity, and the sensitivities are exact."""
import numpy as np
import pytest


def _mode(o, k, phase=0.3):
    nz, ny, nx = o.shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.cos(2 * np.pi * (k[0] * xx / nx + k[1] * yy / ny + k[2] * zz / nz) + phase).ravel()


@pytest.mark.parametrize("lat", [0, 1])
def test_band_keeps_and_removes_modes(orc, lat):
    n = 16
    o = orc.Oracle(lattice=lat, nx=n, ny=n, nz=(n if lat else 1))
    k = (3, 4, 0)                         # |k| = 5
    u = _mode(o, k)
    assert np.max(np.abs(o.filter("F4-6", u) - u)) < 1e-13     # 3.5 <= 5 < 6.5
    assert np.max(np.abs(o.filter("F6-8", u))) < 1e-13         # 5 < 5.5
    assert np.max(np.abs(o.filter("F0-4", u))) < 1e-13         # 5 >= 4.5
    assert np.max(np.abs(o.filter("F5-5", u) - u)) < 1e-13     # 4.5 <= 5 < 5.5
    c = np.full(o.N, 0.7)                                      # the mean is |k| = 0
    assert np.max(np.abs(o.filter("F0-0", c) - c)) < 1e-13
    assert np.max(np.abs(o.filter("F1-8", c))) < 1e-13


def test_projection_partition_and_adjoint(orc):
    o = orc.Oracle(lattice=0, nx=12, ny=10)
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal(o.N), rng.standard_normal(o.N)
    r = o.filter("F2-4", a)
    assert np.max(np.abs(o.filter("F2-4", r) - r)) < 1e-12                 # R^2 = R
    assert abs(o.filter("F2-4", a) @ b - a @ o.filter("F2-4", b)) < 1e-12  # R* = R
    parts = o.filter("F0-1", a) + o.filter("F2-4", a) + o.filter("F5-9", a)
    assert np.max(np.abs(parts - a)) < 1e-12                               # |k| <= 7.8 < 9.5


def test_fourier_sensitivities_exact(orc):
    o = orc.Oracle(lattice=1, nx=8, ny=6, nz=10)
    cl = orc.make_closure([(kind, f, 0) for f in ("F0-2", "F3-6") for kind in ("E", "Z")])
    rng = np.random.default_rng(7)
    v = rng.standard_normal((3, o.N))
    p = rng.standard_normal((3, o.N))
    _, V = o.qoi(cl, v)
    qp, _ = o.qoi(cl, v + p)
    qm, _ = o.qoi(cl, v - p)
    lhs = 0.5 * (qp - qm)
    rhs = np.einsum("kan,an->k", V, p)
    assert np.max(np.abs(lhs - rhs) / (np.abs(qp) + np.abs(qm) + 1)) < 1e-12

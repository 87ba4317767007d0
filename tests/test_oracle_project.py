"""Pins of the oracle's HF -> LF projection (Sec. 3, phi_m; Sec. 7.1: the
wall-anchored stride-m subsampling of the channel) and of the
post-collision velocity whose projected QoIs are the tracking reference
(Sec. 4.3, the predictor-corrector tracking figure)."""
import numpy as np
import pytest

import synth


def test_stride_one_is_identity(orc):
    f = np.random.default_rng(1).standard_normal((3, 4 * 5 * 6))
    assert np.array_equal(orc.project(f, (4, 5, 6), 1), f)


@pytest.mark.parametrize("m", [3, 5])
def test_wall_anchoring(orc, m):
    nzc, nyc, nxc = 2, 4, 3
    nz, ny, nx = m * nzc, m * nyc, m * nxc
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(float)
    p = orc.project(f, (nz, ny, nx), m).reshape(3, nzc, nyc, nxc)
    o = (m - 1) // 2
    assert np.array_equal(p[1][0, :, 0], m * np.arange(nyc) + o)
    assert np.array_equal(p[0][0, 0, :], m * np.arange(nxc) + o)
    assert np.array_equal(p[2][:, 0, 0], m * np.arange(nzc) + o)
    # walls at y = -1/2 and ny - 1/2 (fine cells) are half a coarse cell
    # beyond the first and last coarse rows
    first, last = p[1][0, 0, 0], p[1][0, -1, 0]
    assert first + 0.5 == m / 2 and (ny - 0.5) - last == m / 2
    with pytest.raises(ValueError):
        orc.project(f, (nz, ny, nx), 2)


def test_two_dimensional_keeps_z(orc):
    f = np.arange(2 * 10 * 15, dtype=float).reshape(2, 150)
    p = orc.project(f, (1, 10, 15), 5)
    assert p.shape == (2, 6) and p[0, 0] == 2 * 15 + 2


def test_post_collision_velocity(orc):
    """Of an equilibrium state: the initial velocity.  After a forced plain
    BGK step: the post-streaming velocity plus F / rho (collision keeps rho v,
    the exact-difference force adds F)."""
    o = orc.Oracle(lattice=0, nx=12, ny=16, tau=0.7, force_kind=1, force_amp=2e-4, force_k=1)
    u0 = synth.noise_velocity(2, o.shape, 1e-2, 5)
    o.init(u0)
    _, u = o.post_collision_velocity()
    assert np.allclose(u, u0.reshape(2, -1), rtol=0, atol=1e-15)
    o.step(2)
    rho, v = o.velocity()          # moments after streaming the current state: step 3's v^n
    o.step(1)
    y = (np.arange(o.N) // 12) % 16
    F = 2e-4 * np.sin(2 * np.pi * y / 16)
    rp, up = o.post_collision_velocity()
    assert np.allclose(rp, rho, rtol=1e-14)
    assert np.allclose(up[0], v[0] + F / rho, rtol=0, atol=1e-15)
    assert np.allclose(up[1], v[1], rtol=0, atol=1e-15)

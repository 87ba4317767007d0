"""Pins of the oracle's bicubic projection phi_m of doubly periodic 2-D
fields (Sec. 3, the Kolmogorov case): the Keys cubic kernel widened m-fold,
centred on the wall-anchored stride points, normalised, periodic."""
import numpy as np
import pytest
import torch


def test_keys_kernel_interpolates_and_reproduces_quadratics(orc):
    K = orc.keys_cubic
    assert K(0.0) == 1.0 and K(1.0) == 0.0 and K(-1.0) == 0.0 and K(2.0) == 0.0 and K(2.5) == 0.0
    # partition of unity and reproduction of quadratics at any phase
    for phase in (0.0, 0.1, 0.37, 0.5, 0.93):
        i = np.arange(-3, 4)
        w = K(phase - i)
        assert abs(w.sum() - 1) < 1e-14
        assert abs((w * i).sum() - phase) < 1e-14
        assert abs((w * i * i).sum() - phase ** 2) < 1e-14


def test_stride_one_is_the_identity(orc):
    f = np.random.default_rng(1).standard_normal((2, 12 * 10))
    assert np.array_equal(orc.project_bicubic(f, (1, 12, 10), 1), f)


@pytest.mark.parametrize("m", [3, 5])
def test_mass_and_constants(orc, m):
    """Every fine cell gives weight 1/m in total on each axis (partition of
    unity on the m-strided lattice), so the coarse sum is the fine sum / m^2;
    a constant stays constant."""
    ny, nx = 10 * m, 8 * m
    f = np.random.default_rng(m).random((3, ny * nx))
    g = orc.project_bicubic(f, (1, ny, nx), m)
    assert np.allclose(g.sum(axis=1), f.sum(axis=1) / m ** 2, rtol=1e-13, atol=0)
    c = orc.project_bicubic(np.full((1, ny * nx), 0.7), (1, ny, nx), m)
    assert np.max(np.abs(c - 0.7)) < 1e-14


@pytest.mark.parametrize("m", [3, 5])
def test_matches_library_antialiased_bicubic_resize_in_the_interior(orc, m):
    """torch's antialiased bicubic resize (Keys a = -1/2, half-pixel centres,
    kernel widened by the scale factor) computes the same weights; it clamps
    at the border instead of wrapping, so the cells whose window stays
    inside the grid agree."""
    ny, nx = 12 * m, 14 * m
    f = np.random.default_rng(7).standard_normal((1, ny * nx))
    g = orc.project_bicubic(f, (1, ny, nx), m).reshape(ny // m, nx // m)
    t = torch.nn.functional.interpolate(torch.from_numpy(f.reshape(1, 1, ny, nx)), size=(ny // m, nx // m),
                                        mode="bicubic", antialias=True, align_corners=False)[0, 0].numpy()
    inner = (slice(2, ny // m - 2), slice(2, nx // m - 2))
    assert np.max(np.abs(g[inner] - t[inner])) < 1e-12

"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module generates inputs only -- initial velocity fields, synthetic LRS
model parameters and the workload descriptions -- and holds none of the
method's arithmetic (no streaming, collision, filters, QoIs or closure
evaluation).  Both the HIP library (through its Python binding) and the CPU
oracle consume what it produces, so neither depends on the other.

The paper's own inputs (DNS burn-in fields, reference QoI trajectories and
trained LRS models) are not available; the generators below stand in for
them with the shapes, amplitudes and structure of the paper's workloads:
the 2-D Kolmogorov flow (Sec. 6) and the 3-D channel at Re_tau = 180
(Sec. 7).
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Initial velocity fields
# ---------------------------------------------------------------------------


def noise_velocity(d: int, shape, amp: float, seed: int) -> np.ndarray:
    """u = amp * (2U - 1) per component and cell, U ~ uniform[0, 1) (PCG64).

    ``shape`` is (nz, ny, nx) (nz = 1 in 2-D); the result has shape
    (d, nz*ny*nx) with x fastest.
    """
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    return amp * (2.0 * rng.random((d, n)) - 1.0)


def channel_velocity(nx: int, ny: int, nz: int, uc: float = 0.1, noise: float = 0.05,
                     seed: int = 0) -> np.ndarray:
    """Parabolic streamwise profile with centreline ``uc`` between halfway
    bounce-back walls at y = -1/2 and y = ny - 1/2, plus uniform noise of
    amplitude ``noise * uc`` on every component (the channel initial state of
    the workload recipe; the paper's own start is a DNS burn-in field)."""
    rng = np.random.default_rng(seed)
    y = np.arange(ny) + 0.5            # distance from the lower wall
    h2 = float(ny)                     # channel height 2H
    prof = uc * 4.0 * y * (h2 - y) / (h2 * h2)
    u = np.zeros((3, nz, ny, nx))
    u[0] = prof[None, :, None]
    u += noise * uc * (2.0 * rng.random(u.shape) - 1.0)
    return u.reshape(3, -1)


def turbulent_velocity_2d(n: int, urms: float, kpeak: float = 8.0, seed: int = 0) -> np.ndarray:
    """Divergence-free random 2-D velocity on an n x n periodic grid with a
    spectrum peaked at wavenumber ``kpeak`` and rms speed ``urms``: a seeded
    stand-in for the projected turbulent DNS field that starts the paper's
    low-fidelity Kolmogorov runs.  Built from a random-phase streamfunction
    psi_k ~ k^-2 exp(-(k/kpeak)^2), u = (d_y psi, -d_x psi) spectrally."""
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(n, 1.0 / n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky)
    amp = np.where(kk > 0, (kk + 1e-30) ** -2.0 * np.exp(-(kk / kpeak) ** 2), 0.0)
    psih = amp * np.exp(2j * np.pi * rng.random((n, n)))
    ux = np.real(np.fft.ifft2(1j * ky * psih))
    uy = np.real(np.fft.ifft2(-1j * kx * psih))
    scale = urms / np.sqrt(np.mean(ux * ux + uy * uy))
    return np.stack([ux.ravel(), uy.ravel()]) * scale


# ---------------------------------------------------------------------------
# Channel physics in lattice units (paper Sec. 7.1 scaling: centreline
# velocity U_c+ = 18.3 maps to 0.1, Re_tau = 180).
# ---------------------------------------------------------------------------


def channel_params(ny: int, re_tau: float = 180.0, uc_plus: float = 18.3, uc: float = 0.1):
    """Return (tau, F_x) for a channel with ``ny`` fluid rows (H = ny/2)."""
    H = ny / 2.0
    u_tau = uc / uc_plus
    nu = u_tau * H / re_tau
    tau = 0.5 + 3.0 * nu
    F = u_tau * u_tau / H
    return tau, F


# ---------------------------------------------------------------------------
# Synthetic LRS model (stands in for a ridge fit on tracking data)
# ---------------------------------------------------------------------------


def lrs_model(nq: int, seed_a: int, seed_b: int, seed_sigma: int, std: float = 0.01,
              kappa: float = 0.05):
    """Synthetic h = 0 LRS model in scaled QoI units.

    A and b are drawn N(0, std^2); A is shifted to A_s = A - (max(0, a) +
    kappa) I, a the spectral abscissa of A, so that the scaled QoIs relax
    towards one.  The model is returned in the regression form of the LRS
    equation with input row [z*, 1]:  C = [(I + A_s)^T ; (b - A_s 1)^T],
    mu = 0 and Sigma = 1e-4 (M M^T / nq + 0.1 I) with M ~ N(0, 1).
    """
    A = std * np.random.default_rng(seed_a).standard_normal((nq, nq))
    b = std * np.random.default_rng(seed_b).standard_normal(nq)
    M = np.random.default_rng(seed_sigma).standard_normal((nq, nq))
    alpha = float(np.max(np.linalg.eigvals(A).real))
    As = A - (max(0.0, alpha) + kappa) * np.eye(nq)
    C = np.zeros((nq + 1, nq))
    C[:nq, :] = (np.eye(nq) + As).T
    C[nq, :] = b - As @ np.ones(nq)
    Sigma = 1e-4 * (M @ M.T / nq + 0.1 * np.eye(nq))
    Sigma = 0.5 * (Sigma + Sigma.T)
    return C, np.zeros(nq), Sigma


def lrs_model_channel(nq: int, seed_a: int, seed_sigma: int, kappa: float = 0.05,
                      spread: float = 0.01, noise: float = 1e-5):
    """Synthetic h = 0 LRS model for the 12-QoI channel closure.

    Per-QoI mean reversion of the scaled QoIs towards one with seeded rates
    kappa + spread |a_k|, a ~ N(0, 1), no bias, and seeded SPD residual
    covariance Sigma = noise^2 (M M^T / nq + 0.1 I).  Random off-diagonal
    coupling and random bias terms are left out: the twelve channel
    sensitivities are nearly linearly dependent (the mean flow dominates
    the large-scale energy and the mean-profile bands), so corrections that
    are not consistent with that dependence call for very large dv and
    diverge within a few hundred steps.
    """
    a = np.abs(np.random.default_rng(seed_a).standard_normal(nq))
    As = -np.diag(kappa + spread * a)
    M = np.random.default_rng(seed_sigma).standard_normal((nq, nq))
    C = np.zeros((nq + 1, nq))
    C[:nq, :] = (np.eye(nq) + As).T
    C[nq, :] = -As @ np.ones(nq)
    Sigma = noise * noise * (M @ M.T / nq + 0.1 * np.eye(nq))
    Sigma = 0.5 * (Sigma + Sigma.T)
    return C, np.zeros(nq), Sigma


def lrs_history_model(h: int, nq: int, seed_a: int, seed_sigma: int, seed_eps: int, kappa: float = 0.05,
                      spread: float = 0.01, noise: float = 1e-5, w: float = 0.5, eps: float = 0.01):
    """Synthetic history-h LRS model, per QoI (diagonal in the QoIs).

    Rows follow the LRS input [z^{n-1..n-h}, z*^n, z*^{n-1..n-h}, 1].  Each
    scaled QoI relaxes towards one at the seeded rate r = kappa + spread |a|,
    a ~ N(0, 1), from a blend of its previous corrected value (weight w) and
    its current predictor value:  z^n = (1 - r)(w z^{n-1} + (1 - w) z*^n) + r
    + sum_{l=2..h} e_l (z^{n-l} - z*^{n-l}) + residual, with seeded
    e_l ~ eps N(0, 1) / h, mu = 0 and Sigma = noise^2 (M M^T / nq + 0.1 I).
    """
    a = np.abs(np.random.default_rng(seed_a).standard_normal(nq))
    r = kappa + spread * a
    e = eps * np.random.default_rng(seed_eps).standard_normal((max(h, 1), nq)) / max(h, 1)
    M = np.random.default_rng(seed_sigma).standard_normal((nq, nq))
    C = np.zeros(((2 * h + 1) * nq + 1, nq))
    k = np.arange(nq)
    C[h * nq + k, k] = (1 - r) * (1 - w if h > 0 else 1.0)
    if h > 0:
        C[k, k] = (1 - r) * w
    for lag in range(2, h + 1):
        C[(lag - 1) * nq + k, k] = e[lag - 1]
        C[(h + lag) * nq + k, k] = -e[lag - 1]
    C[-1, :] = r
    Sigma = noise * noise * (M @ M.T / nq + 0.1 * np.eye(nq))
    Sigma = 0.5 * (Sigma + Sigma.T)
    return C, np.zeros(nq), Sigma


# ---------------------------------------------------------------------------
# QoI sets of the workloads
# ---------------------------------------------------------------------------

#: 2-D Kolmogorov TO-LES: energy and enstrophy after the 3x3 binomial filter.
QOIS_2D = [("E", "B", 0), ("Z", "B", 0)]

#: 3-D channel: {E, Z} x {B^2, B - B^2, I - B} plus six mean-profile bands.
QOIS_3D = ([("E", "B2", 0), ("Z", "B2", 0), ("E", "BMID", 0), ("Z", "BMID", 0),
            ("E", "IMB", 0), ("Z", "IMB", 0)] + [("MP", "I", j) for j in range(6)])


def kolmogorov_workload(n: int, tau: float, amp: float = 1e-5, k: int = 4,
                        noise: float = 1e-4, seed: int = 2):
    cfg = dict(lattice=0, nx=n, ny=n, nz=1, walls_y=0, tau=tau, substrate=0, cmodel=0.0,
               force_kind=1, force_amp=amp, force_k=k, drag=0.0)
    u0 = noise_velocity(2, (1, n, n), noise, seed)
    return cfg, u0


def channel_workload(nx: int, ny: int, nz: int, substrate: int = 1, cmodel: float = 0.1,
                     seed: int = 6):
    tau, F = channel_params(ny)
    cfg = dict(lattice=1, nx=nx, ny=ny, nz=nz, walls_y=1, tau=tau, substrate=substrate,
               cmodel=cmodel, force_kind=2, force_amp=F, force_k=0, drag=0.0)
    u0 = channel_velocity(nx, ny, nz, seed=seed)
    return cfg, u0


def channel_bands(ny: int, nb: int = 6):
    """(nbands, dmin, dmax): centres from the first fluid node to the centreline."""
    return nb, 0.5, ny / 2.0


def largest_closure_workload():
    """The largest closure the library takes (16 QoIs) on the 20 x 24 x 12
    channel: energy and enstrophy of the four binomial filter forms (B, B^2,
    B - B^2, I - B) and eight mean-profile bands, with an LRS model from
    the fifth step.  Returns (cfg, u0, qois, closure arguments)."""
    cfg, u0 = channel_workload(20, 24, 12, substrate=1, cmodel=0.1)
    qois = [(k, f, 0) for f in ("B", "B2", "BMID", "IMB") for k in ("E", "Z")] + [("MP", "I", j) for j in range(8)]
    C, mu, S = lrs_model_channel(16, 7, 9)
    nb, dmin, dmax = channel_bands(24, 8)
    cargs = dict(mode="lrs", spinup=5, C=C, mu=mu, Sigma=S, seed=5, nbands=nb, dmin=dmin, dmax=dmax)
    return cfg, u0, qois, cargs


# ---------------------------------------------------------------------------
# Ensembles and request traces
# ---------------------------------------------------------------------------


def ensemble_members(n: int = 64, sizes=(128, 192, 256, 384, 512), seed: int = 10):
    """Grid sizes of a stochastic Kolmogorov TO-LES ensemble: n members drawn
    uniformly from ``sizes`` (square grids), with member-indexed seeds."""
    rng = np.random.default_rng(seed)
    return [dict(n=int(rng.choice(sizes)), ic_seed=1000 + k, noise_seed=5000 + k) for k in range(n)]


def serve_trace(nreq: int = 200, rate: float = 20.0, seed: int = 11, steps: int = 2000):
    """Poisson request trace: exponential gaps with mean 1/rate seconds; 60%
    D2Q9 Kolmogorov requests with N in {128, 256, ..., 1024}, 40% D3Q19
    channel requests m*(48, 24, 24) with m in {1, 2, 3, 4}."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, nreq))
    out = []
    for k in range(nreq):
        if rng.random() < 0.6:
            out.append(dict(kind="2d", n=int(128 * rng.integers(1, 9)), t=float(t[k]), steps=steps,
                            seed=20000 + k))
        else:
            out.append(dict(kind="3d", m=int(rng.integers(1, 5)), t=float(t[k]), steps=steps, seed=30000 + k))
    return out

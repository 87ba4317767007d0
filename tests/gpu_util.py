"""Helpers shared by the GPU parity tests: matched oracle / HIP runs on the
same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_32892_amd import lbm
    lbm.lib()
    return lbm


def closure_args(kind, ny=None, mode="lrs", spinup=20, seed=11):
    """Closure keyword arguments shared by both sides."""
    if kind == "2d":
        C, mu, S = synth.lrs_model(2, 3, 4, 5)
        return synth.QOIS_2D, dict(mode=mode, spinup=spinup, C=C, mu=mu, Sigma=S, seed=seed)
    nb, dmin, dmax = synth.channel_bands(ny)
    C, mu, S = synth.lrs_model_channel(12, 7, 9)
    return synth.QOIS_3D, dict(mode=mode, spinup=spinup, C=C, mu=mu, Sigma=S, seed=seed,
                               nbands=nb, dmin=dmin, dmax=dmax)


def gpu_run(lbm, cfg, u0, precision, qois=None, cargs=None, diag=0, qref=None, **tune):
    spec = None
    if qois is not None:
        spec = lbm.ClosureSpec(qois, qref=qref, **cargs)
    run = lbm.Run(lbm.make_config(precision=precision, diag=diag, **cfg, **tune), spec)
    run.init_velocity(u0)
    return run


def oracle_run(cfg, u0, qois=None, cargs=None, qref=None):
    o = oracle.Oracle(**cfg)
    o.init(u0)
    if qois is not None:
        o.set_closure(oracle.make_closure(qois, **cargs), qref=qref)
    return o


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def match_populations(lbm, lat, f_gpu):
    """Reorder the library's populations into the oracle's lattice order."""
    cg, _ = lbm.lattice_info(lat)
    co, _ = oracle.lattice(lat)
    perm = [next(j for j in range(len(cg)) if np.array_equal(cg[j], co[i])) for i in range(len(co))]
    return f_gpu[perm]


def oracle_floor(cfg, u0, qois, cargs, steps, ref=None, qref=None):
    """The FP64 resolution of a workload: the largest difference between the
    oracle run and its three twins -- the initial populations one unit in
    the last place away (the oracle stores full populations f ~ w_i, so its
    velocity resolves no more than ulp(f) / |v|), the TO step's global sums
    taken in reverse cell order, and the correction in its reduced form
    sum_j (G^-1 dQ)_j V_j instead of the literal patterns -- in the velocity
    (max relative) and in q*, dQ and gamma (per QoI, relative to that QoI's
    largest value over the run).  Each twin is the same method in FP64 with
    last-bit differences; a near-singular Gram system amplifies those every
    step, so no FP64 implementation resolves the workload more finely.  ref:
    the oracle run itself when already stepped."""
    if ref is None:
        ref = oracle_run(cfg, u0, qois, cargs, qref=qref)
        ref.step(steps)
    uo, ro = ref.velocity()[1], ref.record_arrays()

    def per_qoi(a, b):
        return float(np.max(np.abs(a - b) / (np.max(np.abs(b), axis=0) + 1e-300)))

    out = np.zeros(4)
    a = oracle_run(cfg, u0, qois, cargs, qref=qref)
    fp = a.get_fp()
    a.set_fp(fp * (1 + 2.2e-16 * np.random.default_rng(1).choice([-1, 1], size=fp.shape)))
    twins = [a]
    if qois is not None:
        b = oracle_run(cfg, u0, qois, cargs, qref=qref)
        b.set_reverse_sums(True)
        c = oracle_run(cfg, u0, qois, cargs, qref=qref)
        c.set_reduced_form(True)
        twins += [b, c]
    for t in twins:
        t.step(steps)
        rt = t.record_arrays()
        f = [rel_err(t.velocity()[1], uo)]
        f += [per_qoi(rt[k], ro[k]) if qois is not None else 0.0 for k in ("q", "dq", "gamma")]
        out = np.maximum(out, f)
    return out


def fp64_bars(floor, vel=1e-12, q=1e-12, dq=1e-10):
    """FP64 bars for velocity, q*, dQ and gamma: the stated bar (1e-12) or
    ten times the workload's own FP64 resolution, whichever is larger."""
    return np.maximum(np.array([vel, q, dq, dq]), 10 * np.asarray(floor))

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

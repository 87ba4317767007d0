"""lbm_fields_noalloc, the variant of lbm_fields that allocates nothing
(its staging is a fixed device array per GPU): through the C ABI it returns
bitwise the outputs of lbm_fields, on two calls in a row, the second on a
smaller grid, and it rejects grids whose staging exceeds the array."""
import numpy as np
import pytest

import synth
from gpu_util import closure_args, gpu_run, need_gpu

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_fields_noalloc_equals_fields_twice_then_smaller():
    lbm = need_gpu()
    # call 1: a 3-D channel TO-LES with its last SGS change still pending
    cfg, u0 = synth.channel_workload(64, 32, 24)
    qois, cargs = closure_args("3d", ny=32, spinup=2)
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    a.step(7)
    _say("fields_noalloc: 64x32x24 channel TO-LES, FP32")
    rn, vn = a.fields_noalloc()
    rf, vf = a.fields()
    assert np.array_equal(rn, rf) and np.array_equal(vn, vf)
    assert np.all(np.isfinite(vn)) and np.max(np.abs(vn)) > 0
    # call 2: a smaller grid (2-D, FP64) through the same staging
    cfg2, u2 = synth.kolmogorov_workload(40, tau=0.6, seed=3)
    b = gpu_run(lbm, cfg2, u2, "fp64")
    b.step(5)
    _say("fields_noalloc: 40x40 Kolmogorov plain, FP64")
    rn2, vn2 = b.fields_noalloc()
    rf2, vf2 = b.fields()
    assert np.array_equal(rn2, rf2) and np.array_equal(vn2, vf2)
    # and the first run again, after the smaller call: unchanged
    a.step(3)
    rn, vn = a.fields_noalloc()
    rf, vf = a.fields()
    assert np.array_equal(rn, rf) and np.array_equal(vn, vf)
    # velocity only (rho = NULL)
    u_only = np.zeros((3, a.N))
    lbm.check(a.L.lbm_fields_noalloc(a.h, None, lbm._p(u_only)))
    assert np.array_equal(u_only, vf)


def test_fields_noalloc_rejects_grids_beyond_the_staging():
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(96, 80, 72)   # 552960 cells: 17.7 MB of staging
    run = gpu_run(lbm, cfg, u0, "fp32")
    with pytest.raises(lbm.LbmError) as e:
        run.fields_noalloc()
    assert e.value.code == lbm.EINVAL
    assert "static scratch" in str(e.value)

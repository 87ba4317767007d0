"""Continuous-batching server on the GPU: admission by HBM budget, requests of
mixed size and kind overlapping on the device, each result bitwise equal to
the same request run alone, and isolation of an unstable request."""
import hashlib

import numpy as np
import pytest

import synth
from gpu_util import closure_args, need_gpu

pytestmark = pytest.mark.gpu


def _requests(lbm):
    """Mixed D2Q9 Kolmogorov and D3Q19 channel TO-LES requests, FP32."""
    reqs = []
    for k, (n, steps) in enumerate(((48, 37), (64, 20), (40, 53))):
        cfg, _ = synth.kolmogorov_workload(n, tau=0.51, seed=k)
        u0 = synth.turbulent_velocity_2d(n, 0.03, seed=k)
        qois, cargs = closure_args("2d", spinup=5, seed=200 + k)
        reqs.append((lbm.make_config(precision="fp32", **cfg), lbm.ClosureSpec(qois, **cargs), u0, steps))
    for k, (m, steps) in enumerate(((1, 29), (1, 11))):
        cfg, u0 = synth.channel_workload(16 * m, 24, 8 * m, seed=20 + k)
        qois, cargs = closure_args("3d", ny=24, spinup=5, seed=300 + k)
        reqs.append((lbm.make_config(precision="fp32", **cfg), lbm.ClosureSpec(qois, **cargs), u0, steps))
    return reqs


def _alone(lbm, cfg, spec, u0, steps):
    r = lbm.Run(cfg, spec)
    r.init_velocity(u0)
    r.step(steps)
    status = 0
    try:
        r.sync()
    except lbm.LbmError as e:
        status = e.code
    return r.get_state(), status


def _drive(lbm, srv, deadline_s=60.0):
    results = []
    t_end = srv.clock() + deadline_s
    while srv.pending() > 0:
        srv.advance(srv.clock(), 16)
        results += srv.poll()
        assert srv.clock() < t_end, "server did not drain"
    return results


def test_server_mix_bitwise_equal_alone_and_budget():
    lbm = need_gpu()
    reqs = _requests(lbm)
    # budget for about two of the larger requests: forces queueing
    from paper_2609_32892_amd.lbm import lib
    import ctypes as ct
    sizes = [lib().lbm_required_bytes(ct.byref(c), ct.byref(s.c)) for c, s, _, _ in reqs]
    budget = int(2.2 * max(sizes))
    srv = lbm.Server(hbm_budget=budget)
    t0 = srv.clock()
    ids = []
    for k, (cfg, spec, u0, steps) in enumerate(reqs):
        ids.append(srv.submit(cfg, spec, u0, steps, t0 + 0.001 * k, keep_state=True))
    results = _drive(lbm, srv)
    st = srv.stats()
    assert len(results) == len(reqs)
    assert st["used"] == 0 and st["budget"] == budget
    by_id = {r.id: r for r in results}
    for rid, (cfg, spec, u0, steps) in zip(ids, reqs):
        res = by_id[rid]
        assert res.status == 0 and res.steps == steps
        assert res.t_admit >= res.t_arrival - 1e-9 and res.t_done >= res.t_admit
        assert res.last.step == steps - 1
        img = srv.take_state(rid)
        alone, status = _alone(lbm, cfg, spec, u0, steps)
        assert status == 0
        same = hashlib.sha256(img).digest() == hashlib.sha256(alone).digest()
        assert same, f"request {rid}: result differs from the solo run"
    srv.close()


def test_server_isolates_unstable_request():
    lbm = need_gpu()
    reqs = _requests(lbm)[:2]
    bad_cfg = dict(lattice=0, nx=16, ny=16, nz=1, walls_y=0, tau=0.5005, substrate=0, cmodel=0.0,
                   force_kind=1, force_amp=5e-3, force_k=1, drag=0.0)
    bad = (lbm.make_config(precision="fp32", **bad_cfg), None,
           synth.noise_velocity(2, (1, 16, 16), 0.05, 7), 400)
    srv = lbm.Server()
    t0 = srv.clock()
    ids = [srv.submit(c, s, u, n, t0, keep_state=True) for c, s, u, n in reqs + [bad]]
    results = {r.id: r for r in _drive(lbm, srv)}
    assert results[ids[-1]].status == lbm.EUNSTABLE
    for rid, (cfg, spec, u0, steps) in zip(ids[:-1], reqs):
        assert results[rid].status == 0
        alone, _ = _alone(lbm, cfg, spec, u0, steps)
        assert hashlib.sha256(srv.take_state(rid)).digest() == hashlib.sha256(alone).digest()
    srv.close()


def test_server_kernel_filter_fourier_and_history_requests():
    """Requests whose closures use the kernel filters, Fourier bands (eager
    stepping) and a history-h LRS model, served together with a binomial
    one: every result bitwise equal to the request run alone."""
    lbm = need_gpu()
    reqs = []
    n = 32
    cfg, _ = synth.kolmogorov_workload(n, tau=0.51, seed=7)
    u0 = synth.noise_velocity(2, (1, n, n), 1e-3, 7)
    for qois, h in (([(k, f, 0) for f in ("G3", "L1") for k in ("E", "Z")], 0),
                    ([(k, f, 0) for f in ("F0-4", "F5-12") for k in ("E", "Z")], 0),
                    (synth.QOIS_2D, 6)):
        C, mu, S = synth.lrs_history_model(h, len(qois), 3, 4, 5, noise=1e-4)
        spec = lbm.ClosureSpec(qois, mode="lrs", spinup=8, C=C, mu=mu, Sigma=S, seed=61, h=h,
                               scale=np.full(len(qois), 1e-3) if h else None)
        reqs.append((lbm.make_config(precision="fp32", **cfg), spec, u0, 30))
    qois, cargs = closure_args("2d", spinup=5, seed=62)
    reqs.append((lbm.make_config(precision="fp32", **cfg), lbm.ClosureSpec(qois, **cargs), u0, 30))
    srv = lbm.Server()
    t0 = srv.clock()
    ids = [srv.submit(c, s, u, st, t0, keep_state=True) for c, s, u, st in reqs]
    results = _drive(lbm, srv)
    assert len(results) == len(reqs) and all(r.status == 0 for r in results)
    for rid, (cfg_r, spec, u, steps) in zip(ids, reqs):
        img = srv.take_state(rid)
        alone, status = _alone(lbm, cfg_r, spec, u, steps)
        assert status == 0
        assert hashlib.sha256(img).digest() == hashlib.sha256(alone).digest(), f"request {rid} differs"
    srv.close()


def test_server_rejects_bad_requests_and_serves_the_rest():
    """A closure whose Sigma is not SPD is rejected when it is submitted
    (nothing is queued); a request larger than the whole budget is retired at
    admission with LBM_ENOMEM; the requests around them run to completion,
    bitwise equal to their solo runs, and the arenas of retired requests are
    reused by later requests of the same size."""
    lbm = need_gpu()
    reqs = _requests(lbm)[:3]
    from paper_2609_32892_amd.lbm import lib
    import ctypes as ct
    sizes = [lib().lbm_required_bytes(ct.byref(c), ct.byref(s.c)) for c, s, _, _ in reqs]
    srv = lbm.Server(hbm_budget=int(1.5 * max(sizes)))
    cfg, spec, u0, steps = reqs[0]
    qois, cargs = closure_args("2d", spinup=5)
    bad_sigma = dict(cargs, Sigma=-np.eye(2))
    with pytest.raises(lbm.LbmError) as e:
        srv.submit(cfg, lbm.ClosureSpec(qois, **bad_sigma), u0, steps, srv.clock())
    assert e.value.code == lbm.EINVAL and srv.pending() == 0
    big_cfg, big_u0 = synth.channel_workload(96, 48, 48)
    big = (lbm.make_config(precision="fp32", **big_cfg), None, big_u0, 10)
    t0 = srv.clock()
    order = [reqs[0], big, reqs[1], reqs[2], reqs[0]]
    ids = [srv.submit(c, s, u, n, t0 + 0.001 * k, keep_state=True) for k, (c, s, u, n) in enumerate(order)]
    results = {r.id: r for r in _drive(lbm, srv)}
    assert len(results) == len(order)
    assert results[ids[1]].status == lbm.ENOMEM and results[ids[1]].steps == 0
    for k in (0, 2, 3, 4):
        cfg_k, spec_k, u_k, n_k = order[k]
        assert results[ids[k]].status == 0 and results[ids[k]].steps == n_k
        alone, status = _alone(lbm, cfg_k, spec_k, u_k, n_k)
        assert status == 0
        assert hashlib.sha256(srv.take_state(ids[k])).digest() == hashlib.sha256(alone).digest()
    st = srv.stats()
    assert st["used"] == 0
    srv.close()


def test_server_as_the_first_gpu_object_of_a_process():
    """A server created before any run in a fresh process (the library then
    loads first) finds the device, admits a request and completes it."""
    import os
    import subprocess
    import sys
    need_gpu()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "from paper_2609_32892_amd import lbm\n"
        "import synth\n"
        "srv = lbm.Server()\n"
        "cfg, _ = synth.kolmogorov_workload(32, tau=0.51, seed=1)\n"
        "u0 = synth.turbulent_velocity_2d(32, 0.03, seed=1)\n"
        "c = lbm.make_config(precision='fp32', **cfg)\n"
        "srv.submit(c, None, u0, 20, srv.clock())\n"
        "res = []\n"
        "while srv.pending() > 0:\n"
        "    srv.advance(srv.clock(), 16)\n"
        "    res += srv.poll()\n"
        "assert len(res) == 1 and res[0].status == 0, res\n"
        "print('first-object server ok', flush=True)\n"
    ) % (root, os.path.join(root, "tests"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0 and "first-object server ok" in out.stdout, out.stderr[-2000:]

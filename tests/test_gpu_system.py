"""System behaviour of the HIP library on the GPU: bitwise determinism, graph
replay equal to eager launches, batch members equal to solo runs, bitwise
checkpoint/resume, closure switching."""
import numpy as np
import pytest

import synth
from gpu_util import closure_args, gpu_run, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _case2d(n=80, seed=2):
    cfg, _ = synth.kolmogorov_workload(n, tau=0.51, seed=seed)
    u0 = synth.noise_velocity(2, (1, n, n), 1e-3, seed)
    qois, cargs = closure_args("2d", spinup=10, seed=100 + seed)
    return cfg, u0, qois, cargs


def test_repeat_runs_bitwise_and_graph_equals_eager():
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case2d()
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    b = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    c = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    a.step(70)                      # graph chunks + eager remainder
    for _ in range(70):
        b.step(1)                   # eager only
    c.step(70)
    for r in (a, b, c):
        r.sync()
    fa, fb, fc = a.get_populations(), b.get_populations(), c.get_populations()
    assert np.array_equal(fa, fb)
    assert np.array_equal(fa, fc)
    assert np.array_equal(a.record_arrays()["q"], b.record_arrays()["q"])
    # lbm_velocity is the velocity of lbm_fields, bitwise
    _, u = a.fields()
    assert np.array_equal(a.velocity(), u)


def test_batch_members_bitwise_equal_to_solo():
    lbm = need_gpu()
    members = [_case2d(n, seed=s) for n, s in ((48, 1), (80, 2), (64, 3))]
    channel = synth.channel_workload(16, 24, 8)
    qois3, cargs3 = closure_args("3d", ny=24, spinup=10)
    solo, batched = [], []
    for cfg, u0, qois, cargs in members:
        solo.append(gpu_run(lbm, cfg, u0, "fp32", qois, cargs))
        batched.append(gpu_run(lbm, cfg, u0, "fp32", qois, cargs))
    for lst in (solo, batched):
        lst.append(gpu_run(lbm, channel[0], channel[1], "fp32", qois3, cargs3))
    for r in solo:
        r.step(41)
    batch = lbm.Batch(batched)
    batch.step(41)
    batch.sync()
    for r, s in zip(batched, solo):
        s.sync()
        assert r.step_count == 41
        assert np.array_equal(r.get_populations(), s.get_populations())
        assert np.array_equal(r.record_arrays()["q"], s.record_arrays()["q"])
    # a member stepped alone afterwards continues consistently
    batched[0].step(3)
    solo[0].step(3)
    assert np.array_equal(batched[0].get_populations(), solo[0].get_populations())
    batch.step(5)
    for r in solo:
        r.step(5)
    for r, s in zip(batched, solo):
        assert np.array_equal(r.get_populations(), s.get_populations())


def test_batch_past_the_fused_solve_limit_bitwise_equal_to_solo():
    """Five 256 x 256 Kolmogorov members (128 apply workgroups of two blocks
    each when alone, so each solo run forms its solve in the apply) batched
    into one launch group of 640 workgroups, past the 512 whose workgroups
    are all resident at once, so the batch solves in k_solve: every member
    equals its solo run bitwise, records included."""
    lbm = need_gpu()
    members = [_case2d(256, seed=s) for s in (11, 12, 13, 14, 15)]
    solo = [gpu_run(lbm, cfg, u0, "fp32", qois, dict(cargs, spinup=4)) for cfg, u0, qois, cargs in members]
    batched = [gpu_run(lbm, cfg, u0, "fp32", qois, dict(cargs, spinup=4)) for cfg, u0, qois, cargs in members]
    for r in solo:
        r.step(12)
        r.sync()
    batch = lbm.Batch(batched)
    batch.step(12)
    batch.sync()
    for r, s in zip(batched, solo):
        assert np.array_equal(r.get_populations(), s.get_populations())
        assert bytes(r.get_state()) == bytes(s.get_state())
        ra, rs = r.record_arrays(), s.record_arrays()
        for key in ("q", "dq", "gamma", "flags"):
            assert np.array_equal(ra[key], rs[key]), key
        assert np.any(ra["dq"][4:] != 0)
    batch.close()
    for r in solo + batched:
        r.close()


def test_checkpoint_resume_bitwise():
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case2d()
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    a.step(33)
    img = a.get_state()
    a.step(40)
    b = gpu_run(lbm, cfg, np.zeros_like(u0), "fp32", qois, cargs)
    b.set_state(img)
    assert b.step_count == 33
    b.step(40)
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.record_arrays(33, 40)["dq"], b.record_arrays(33, 40)["dq"])


def test_closure_off_and_on_again():
    """Switching the closure off leaves the populations as they are (the SGS
    change of every step is already in them); switching it back on
    continues without error."""
    lbm = need_gpu()
    cfg, u0, qois, cargs = _case2d()
    a = gpu_run(lbm, cfg, u0, "fp64", qois, cargs)
    a.step(20)
    f_before = a.get_populations()
    a.set_closure(None)
    assert np.array_equal(a.get_populations(), f_before)
    a.step(5)
    a.set_closure(lbm.ClosureSpec(qois, **cargs))
    a.step(5)
    assert a.sync() == 0


def test_invalid_arguments_rejected():
    lbm = need_gpu()
    with pytest.raises(lbm.LbmError):
        lbm.Run(lbm.make_config(nx=2, ny=8))
    cfg, u0, qois, cargs = _case2d()
    with pytest.raises(lbm.LbmError):   # mean-profile QoI without walls
        lbm.Run(lbm.make_config(**cfg), lbm.ClosureSpec([("MP", "I", 0)], nbands=1, dmin=0.5, dmax=2))
    r = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    with pytest.raises(lbm.LbmError):   # more QoIs than the planned workspace
        r.set_closure(lbm.ClosureSpec([("E", "B2", 0)] * 3))
    r.step(2)
    with pytest.raises(lbm.LbmError):   # records not yet produced
        r.records(0, 5)


@pytest.mark.parametrize("walls", [1, 0])
def test_binomial_tile_widths_bitwise_equal(walls):
    """The 64 x 8 tile of the tiled kernels gives bitwise the
    result of the 32 x 8 tile (rows of 128 cells, a ragged y extent, z
    chunks of 1 and 3 planes)."""
    lbm = need_gpu()
    if walls:
        cfg, u0 = synth.channel_workload(128, 22, 7, seed=8)
        qois, cargs = closure_args("3d", ny=22, spinup=3)
    else:
        cfg = dict(lattice=1, nx=128, ny=18, nz=6, walls_y=0, tau=0.55, substrate=1, cmodel=0.1,
                   force_kind=1, force_amp=1e-5, force_k=1, drag=0.0)
        u0 = synth.noise_velocity(3, (6, 18, 128), 0.02, 9)
        qois = [q for q in synth.QOIS_3D if q[0] in ("E", "Z")]
        C, mu, S = synth.lrs_model_channel(len(qois), 7, 9)
        cargs = dict(mode="lrs", spinup=3, C=C, mu=mu, Sigma=S, seed=13)
    for zc in (1, 3):
        _say(f"tile widths: walls={walls} zc={zc}")
        runs = [gpu_run(lbm, cfg, u0, "fp32", qois, cargs, tune_zc=zc, tune_btx=b) for b in (32, 64)]
        for r in runs:
            r.step(8)
            r.sync()
        fa, fb = (r.get_populations() for r in runs)
        assert np.array_equal(fa, fb), f"walls={walls} zc={zc}: populations differ"
        qa, qb = (r.record_arrays()["q"] for r in runs)
        assert np.array_equal(qa, qb)
        for r in runs:
            r.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_large_grid_memory_forms_bitwise_equal(prec):
    """The forms the stream-collide takes on large grids only (64-bit
    population offsets once a population buffer reaches 4 GiB; non-temporal
    population stores beyond the Infinity Cache), forced on a small channel
    through tune_mem: bitwise the default result, for the deferred TO
    predictor, the WALE TO predictor (no deferral) and the plain step."""
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(40, 18, 10, seed=8)
    qois, cargs = closure_args("3d", ny=18, spinup=3)
    wale = dict(cfg, substrate=2, cmodel=2.2)
    for name, c, q in (("TO", cfg, qois), ("WALE TO", wale, qois), ("plain", cfg, None)):
        for mem in (1, 2, 3):
            _say(f"{prec} {name}: tune_mem={mem}")
            runs = [gpu_run(lbm, c, u0, prec, q, cargs if q else None, tune_mem=t) for t in (0, mem)]
            for r in runs:
                r.step(7)
                r.sync()
            fa, fb = (r.get_populations() for r in runs)
            assert np.array_equal(fa, fb), f"{prec} {name} tune_mem={mem}: populations differ"
            if q:
                qa, qb = (r.record_arrays()["q"] for r in runs)
                assert np.array_equal(qa, qb)
            for r in runs:
                r.close()


@pytest.mark.parametrize("case", ["2d-fp32", "3d-fp32", "3d-fp64"])
def test_deferred_and_in_place_sgs_change_bitwise_equal(case):
    """The SGS change recorded per cell and applied by the next step's pull
    (the form of grids whose populations exceed the L2s), forced with
    tune_mem on a small grid, against the in-place apply of small grids:
    bitwise equal populations, fields and records after a run; state read
    with records pending; a checkpoint taken with records pending and
    resumed in a fresh run; and a closure change mid-run."""
    lbm = need_gpu()
    kind, prec = case.split("-")
    if kind == "2d":
        cfg, u0, qois, cargs = _case2d(48, 3)
    else:
        cfg, u0 = synth.channel_workload(40, 18, 10, seed=8)
        qois, cargs = closure_args("3d", ny=18, spinup=3)
    a = gpu_run(lbm, cfg, u0, prec, qois, cargs)
    b = gpu_run(lbm, cfg, u0, prec, qois, cargs, tune_mem=4)
    for r in (a, b):
        r.step(9)
        r.sync()
    _say(f"deferred vs in place: {case}")
    assert np.array_equal(a.fields()[1], b.fields()[1])          # b flushes its pending records
    for r in (a, b):
        r.step(4)
        r.sync()
    state = b.get_state()                                         # taken with records pending
    assert np.array_equal(a.get_populations(), b.get_populations())
    c = gpu_run(lbm, cfg, u0, prec, qois, cargs, tune_mem=4)
    c.set_state(state)
    for r in (a, b, c):
        r.step(6)
        r.sync()
    fa = a.get_populations()
    assert np.array_equal(fa, b.get_populations())
    assert np.array_equal(fa, c.get_populations())
    ra, rb = a.record_arrays(), b.record_arrays()
    for key in ("q", "dq", "gamma"):
        assert np.array_equal(ra[key], rb[key]), key
    # a closure change flushes the pending records first
    spec = lbm.ClosureSpec(qois, **dict(cargs, spinup=0))
    for r in (a, b):
        r.set_closure(spec)
        r.step(5)
        r.sync()
    assert np.array_equal(a.get_populations(), b.get_populations())
    for r in (a, b, c):
        r.close()


@pytest.mark.parametrize("case", ["2d-fp32-lrs", "2d-fp64-track", "3d-fp32-lrs", "3d-fp32-lrs-recorded", "3d-fp64-lrs"])
def test_solve_in_apply_and_in_its_own_launch_bitwise_equal(case):
    """The solve formed by every workgroup of the binomial apply (the
    default) against the solve in its own launch (k_solve, forced with
    tune_mem bit 3): bitwise equal populations and records.  The LRS scale
    is fixed from |q*| at the first corrected step (no scale given), which
    the fused form leaves pending for the next step's k_sum: a checkpoint
    taken right after that step, with the scale still pending, resumes
    bitwise.  Tracking runs read their reference by the step counter, which
    the fused form takes from k_sum's snapshot."""
    lbm = need_gpu()
    kind, prec, mode = case.split("-")[:3]
    tm = 4 if case.endswith("recorded") else 0
    S0 = 3
    if kind == "2d":
        cfg, u0, qois, _ = _case2d(48, 3)
        _, cargs = closure_args("2d", spinup=S0, mode=mode)
    else:
        cfg, u0 = synth.channel_workload(40, 18, 10, seed=8)
        qois, cargs = closure_args("3d", ny=18, spinup=S0, mode=mode)
    qref = None
    if mode == "track":
        o = oracle_run(cfg, u0, qois, dict(mode="off"))
        o.step(40)
        qref = o.record_arrays()["q"] * 1.01
        cargs = dict(mode="track", spinup=S0)
    _say(f"solve in apply vs own launch: {case}")
    a = gpu_run(lbm, cfg, u0, prec, qois, cargs, qref=qref, tune_mem=tm)
    b = gpu_run(lbm, cfg, u0, prec, qois, cargs, qref=qref, tune_mem=tm | 8)
    for r in (a, b):
        r.step(S0 + 1)   # through the first corrected step
        r.sync()
    state = a.get_state()
    # the images are the same bytes: the pending scale committed, the
    # per-step coefficients cleared
    assert bytes(state) == bytes(b.get_state())
    c = gpu_run(lbm, cfg, u0, prec, qois, cargs, qref=qref, tune_mem=tm)
    c.set_state(state)
    for r in (a, b, c):
        r.step(12)
        r.sync()
    fa = a.get_populations()
    assert np.array_equal(fa, b.get_populations())
    assert np.array_equal(fa, c.get_populations())
    assert bytes(a.get_state()) == bytes(b.get_state()) == bytes(c.get_state())
    ra, rb, rc = a.record_arrays(), b.record_arrays(), c.record_arrays()
    for key in ("q", "dq", "gamma", "flags"):
        assert np.array_equal(ra[key], rb[key]), key
        assert np.array_equal(ra[key][S0 + 1:], rc[key][S0 + 1:]), key
    assert np.any(ra["dq"][S0:] != 0)
    for r in (a, b, c):
        r.close()


def test_batch_mixing_both_sgs_forms_bitwise_equal_to_solo():
    """A batch whose members take different SGS forms (one recording the
    change for the next pull, forced with tune_mem, one applying it in
    place) launches them in separate groups; each member equals its solo
    run bitwise, and the two forms equal each other."""
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(40, 18, 10, seed=8)
    qois, cargs = closure_args("3d", ny=18, spinup=3)
    solo = [gpu_run(lbm, cfg, u0, "fp32", qois, cargs, tune_mem=t) for t in (0, 4)]
    for r in solo:
        r.step(11)
        r.sync()
    members = [gpu_run(lbm, cfg, u0, "fp32", qois, cargs, tune_mem=t) for t in (0, 4)]
    batch = lbm.Batch(members)
    batch.step(11)
    assert batch.sync() == 0
    ref = solo[0].get_populations()
    for r, s_ in zip(members, solo):
        f = r.get_populations()
        assert np.array_equal(f, s_.get_populations())
        assert np.array_equal(f, ref)
    batch.close()
    for r in members + solo:
        r.close()


def test_write_through_and_plain_stores_bitwise_equal():
    """Launches whose populations fit the L2s store their fields through it,
    larger ones with plain stores; a batch decides for all its members
    together.  A small TO member run alone (written through) and batched
    with a large member (plain stores) are bitwise equal, in FP32 and FP64."""
    lbm = need_gpu()
    for prec in ("fp32", "fp64"):
        cfg, u0 = synth.channel_workload(20, 24, 12, substrate=1, cmodel=0.1)
        qois, cargs = closure_args("3d", ny=24, spinup=10)
        big_cfg, big_u0 = synth.channel_workload(160, 48, 96, substrate=1, cmodel=0.1)   # 0.74 M cells
        bq, bc = closure_args("3d", ny=48, spinup=10)
        solo = gpu_run(lbm, cfg, u0, prec, qois, cargs)
        small = gpu_run(lbm, cfg, u0, prec, qois, cargs)
        big = gpu_run(lbm, big_cfg, big_u0, prec, bq, bc)
        solo.step(30)
        batch = lbm.Batch([small, big])
        batch.step(30)
        batch.sync()
        solo.sync()
        _say(f"  {prec}: small member solo vs batched with a 0.74 M-cell member")
        assert np.array_equal(small.get_populations(), solo.get_populations())
        assert np.array_equal(small.record_arrays()["dq"], solo.record_arrays()["dq"])


def test_autotune_times_candidates_and_caches(tmp_path):
    """The autotuner times the candidates of a channel TO-LES on the device,
    appends the choice to the cache and returns it from there on the next
    call; the tuned run agrees with the untuned one (tile width and z chunk
    leave every cell bitwise the same, the cells per thread of the reduction
    only reorder its FP64 partial sums)."""
    lbm = need_gpu()
    cfg, u0 = synth.channel_workload(64, 24, 16, substrate=1, cmodel=0.1)
    qois, cargs = closure_args("3d", ny=24, spinup=10)
    spec = lbm.ClosureSpec(qois, **cargs)
    path = tmp_path / "tune.txt"
    t1 = lbm.autotune(lbm.make_config(precision="fp32", **cfg), spec, steps=40, cache=str(path))
    _say(f"  autotune: {t1}")
    assert t1["from_cache"] == 0 and t1["candidates"] >= 3 and t1["us_per_step"] > 0
    assert t1["tune_btx"] in (0, 32, 64) and t1["tune_zc"] in (0, 1, 2, 4, 8, 16) and t1["tune_cpt"] in (0, 1, 2, 4, 8)
    assert path.read_text().count("\n") == 1
    t2 = lbm.autotune(lbm.make_config(precision="fp32", **cfg), spec, steps=40, cache=str(path))
    assert t2["from_cache"] == 1
    assert [t2[k] for k in ("tune_zc", "tune_cpt", "tune_btx")] == [t1[k] for k in ("tune_zc", "tune_cpt", "tune_btx")]
    tuned = {k: t1[k] for k in ("tune_zc", "tune_cpt", "tune_btx")}
    a = gpu_run(lbm, cfg, u0, "fp32", qois, cargs)
    b = gpu_run(lbm, cfg, u0, "fp32", qois, cargs, **tuned)
    a.step(50)
    b.step(50)
    a.sync()
    b.sync()
    ua, ub = a.fields()[1], b.fields()[1]
    assert np.max(np.abs(ua - ub)) <= 1e-5 * np.max(np.abs(ua))


def test_nan_member_flags_only_itself_in_a_batch():
    """Failure isolation: a NaN put into one member's populations makes that
    member unstable (sticky flag, LBM_EUNSTABLE from its sync and the
    batch's), while its batch neighbour stays bitwise equal to a solo run."""
    lbm = need_gpu()
    cfg_a, u_a, qois, cargs_a = _case2d(48, seed=1)
    cfg_b, u_b, _, cargs_b = _case2d(64, seed=2)
    a = gpu_run(lbm, cfg_a, u_a, "fp32", qois, cargs_a)
    b = gpu_run(lbm, cfg_b, u_b, "fp32", qois, cargs_b)
    solo = gpu_run(lbm, cfg_b, u_b, "fp32", qois, cargs_b)
    f = a.get_populations()
    f[3, 100] = np.nan
    a.set_populations(f)
    batch = lbm.Batch([a, b])
    batch.step(20)
    with pytest.raises(lbm.LbmError):
        batch.sync()
    with pytest.raises(lbm.LbmError):
        a.sync()
    assert b.sync() == 0
    assert np.any(a.record_arrays()["flags"] & 1)
    assert not np.any(b.record_arrays()["flags"] & 1)
    solo.step(20)
    solo.sync()
    assert np.array_equal(b.get_populations(), solo.get_populations())

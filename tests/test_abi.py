"""C ABI checks that need no GPU: the built library loads, exports every
function declared in include/lbm.h, and its host-side logic (lattice table,
arena planning, argument validation) behaves as documented."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbm():
    from paper_2609_32892_amd import lbm as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2609_32892_amd import build
        build.build()
    m.lib()
    return m


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", src)))


def test_exports_every_declared_symbol(lbm):
    names = declared_functions()
    assert len(names) >= 20
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTS) == names


def test_lattice_table_matches_oracle_set(lbm, orc):
    for lat in (0, 1):
        cg, wg = lbm.lattice_info(lat)
        co, wo = orc.lattice(lat)
        A = {(tuple(c), w) for c, w in zip(cg.tolist(), wg.tolist())}
        B = {(tuple(c), w) for c, w in zip(co.tolist(), wo.tolist())}
        assert A == B
        # opposite pairs i, i+1 for odd i (the library's convention)
        for i in range(1, len(cg), 2):
            assert np.array_equal(cg[i], -cg[i + 1])


def test_required_bytes_and_validation(lbm):
    L = lbm.lib()
    cfg = lbm.make_config(lattice=lbm.D3Q19, nx=96, ny=48, nz=48, walls_y=1, tau=0.502)
    plain = L.lbm_required_bytes(ct.byref(cfg), None)
    N = 96 * 48 * 48
    assert plain >= 2 * 19 * 4 * N
    spec = lbm.ClosureSpec([("E", "B2", 0), ("Z", "IMB", 0), ("MP", "I", 0)], nbands=1, dmin=0.5, dmax=24)
    to = L.lbm_required_bytes(ct.byref(cfg), ct.byref(spec.c))
    assert to > plain + 4 * N * (1 + 3 + 3)
    bad = [lbm.make_config(nx=2), lbm.make_config(tau=0.5), lbm.make_config(lattice=lbm.D2Q9, substrate=lbm.WALE),
           lbm.make_config(precision=7), lbm.make_config(tune_btx=48),
           lbm.make_config(tune_btx=64)]                                          # wide tile needs D3Q19
    for b in bad:
        assert L.lbm_required_bytes(ct.byref(b), None) == 0
        assert L.lbm_last_error()
    # closures the library rejects
    p2 = lbm.make_config(nx=16, ny=16)
    for sp in (lbm.ClosureSpec([("MP", "I", 0)], nbands=1, dmin=0.5, dmax=8),   # no walls
               lbm.ClosureSpec([("E", "B", 0)] * 9)):                              # > 8 E/Z QoIs
        assert L.lbm_required_bytes(ct.byref(p2), ct.byref(sp.c)) == 0
    lrs = lbm.ClosureSpec([("E", "B", 0)], mode="lrs")                             # LRS without C
    assert L.lbm_required_bytes(ct.byref(p2), ct.byref(lrs.c)) == 0
    # a closure run whose fields would pass 4 GiB per component
    big = lbm.make_config(lattice=lbm.D3Q19, precision="fp64", nx=1024, ny=512, nz=520)
    assert L.lbm_required_bytes(ct.byref(big), None) > 0
    assert L.lbm_required_bytes(ct.byref(big), ct.byref(lbm.ClosureSpec([("E", "B", 0)]).c)) == 0


def test_history_closure_validation(lbm):
    """History-h LRS closures (eq. LRS) the library accepts and rejects."""
    L = lbm.lib()
    p2 = lbm.make_config(nx=16, ny=16, rec_cap=64)
    q2 = [("E", "B", 0), ("Z", "B", 0)]
    S0 = np.zeros((2, 2))

    def spec(h, **kw):
        args = dict(mode="lrs", spinup=100, C=np.zeros(((2 * h + 1) * 2 + 1, 2)), Sigma=S0, scale=np.ones(2), h=h)
        args.update(kw)
        return lbm.ClosureSpec(q2, **args)

    base = L.lbm_required_bytes(ct.byref(p2), ct.byref(spec(0).c))
    ok = L.lbm_required_bytes(ct.byref(p2), ct.byref(spec(40).c))
    assert base > 0 and ok >= base   # workspace of the history product
    neg = spec(0)
    neg.c.h = -1                                           # negative h
    for bad in (spec(3, scale=None),                       # a history model needs s
                spec(3, mode="track", qref=np.zeros((4, 2))),  # history only in LRS
                spec(64),                                  # rec_cap must exceed h
                neg):
        assert L.lbm_required_bytes(ct.byref(p2), ct.byref(bad.c)) == 0
        assert L.lbm_last_error()
    big = lbm.make_config(nx=16, ny=16, rec_cap=4096)
    assert L.lbm_required_bytes(ct.byref(big), ct.byref(spec(1024).c)) > 0          # 2 h nq = 4096
    assert L.lbm_required_bytes(ct.byref(big), ct.byref(spec(1025).c)) == 0         # h > LBM_MAX_HIST


def test_kernel_filter_closure_validation(lbm):
    """Closures with the kernel filters G_s / L_s (Sec. 4.1) the library
    accepts and rejects."""
    L = lbm.lib()
    c3 = lbm.make_config(lattice=lbm.D3Q19, nx=24, ny=16, nz=16, walls_y=1)
    ok = lbm.ClosureSpec([(k, f, 0) for f in ("G3", "L3", "L1") for k in ("E", "Z")] + [("MP", "I", 0)],
                         nbands=1, dmin=0.5, dmax=8)
    assert L.lbm_required_bytes(ct.byref(c3), ct.byref(ok.c)) > 0
    for bad in ([("E", "G3", 0), ("Z", "B", 0)],     # families mixed
                [("E", "L2", 0)],                     # even dilation
                [("E", "G7", 0)],                     # radius 14 > 12
                [("Z", "L7", 0)]):                    # radius 17 > 12
        assert L.lbm_required_bytes(ct.byref(c3), ct.byref(lbm.ClosureSpec(bad).c)) == 0
        assert L.lbm_last_error()
    c2 = lbm.make_config(nx=32, ny=32)
    assert L.lbm_required_bytes(ct.byref(c2), ct.byref(lbm.ClosureSpec([("E", "G3", 0)]).c)) > 0   # radius 12
    assert L.lbm_required_bytes(ct.byref(c2), ct.byref(lbm.ClosureSpec([("E", "G4", 0)]).c)) == 0  # radius 16


def test_fourier_closure_validation(lbm):
    """Sharp Fourier band QoIs (eq. scale-aware-energy-fourier): periodic
    grids only, 0 <= l <= m; they may be mixed with the kernel filters."""
    L = lbm.lib()
    per = lbm.make_config(nx=32, ny=32)
    walls = lbm.make_config(nx=32, ny=32, walls_y=1)
    ok = lbm.ClosureSpec([("E", "F0-4", 0), ("Z", "F5-12", 0), ("E", "G3", 0)])
    assert L.lbm_required_bytes(ct.byref(per), ct.byref(ok.c)) > 0
    assert L.lbm_required_bytes(ct.byref(walls), ct.byref(ok.c)) == 0
    assert L.lbm_required_bytes(ct.byref(per), ct.byref(lbm.ClosureSpec([("E", "F5-4", 0)]).c)) == 0
    assert L.lbm_required_bytes(ct.byref(per), ct.byref(lbm.ClosureSpec([("E", "F0-4", 0), ("Z", "B", 0)]).c)) == 0


def test_autotune_key_bytes_and_cache_hit(lbm, tmp_path):
    """The tuning cache (host logic, no device needed for a hit): keys
    separate grids and closures; a cached line is returned as is (the last
    matching line wins, malformed lines are skipped); the scratch arena
    covers every candidate."""
    import synth
    cfg = lbm.make_config(lattice=lbm.D3Q19, nx=64, ny=24, nz=16, walls_y=1, tau=0.51, substrate=1, cmodel=0.1)
    nb, dmin, dmax = synth.channel_bands(24)
    spec = lbm.ClosureSpec(synth.QOIS_3D, mode="off", nbands=nb, dmin=dmin, dmax=dmax)
    key = lbm.autotune_key(cfg, spec)
    assert "grid=64x24x16" in key and "nq=12" in key and "\t" not in key
    other = lbm.make_config(lattice=lbm.D3Q19, nx=64, ny=24, nz=20, walls_y=1, tau=0.51, substrate=1, cmodel=0.1)
    assert lbm.autotune_key(other, spec) != key
    assert lbm.autotune_key(cfg, None) != key
    L = lbm.lib()
    import ctypes as ct
    need = L.lbm_autotune_bytes(ct.byref(cfg), ct.byref(spec.c))
    for zc in (0, 1, 16):
        for cpt in (0, 8):
            for btx in (0, 32, 64):
                t = lbm.make_config(lattice=lbm.D3Q19, nx=64, ny=24, nz=16, walls_y=1, tau=0.51, substrate=1,
                                    cmodel=0.1, tune_zc=zc, tune_cpt=cpt, tune_btx=btx)
                assert L.lbm_required_bytes(ct.byref(t), ct.byref(spec.c)) <= need
    path = tmp_path / "tune.txt"
    path.write_text(f"{key}\t2 1 32 90.5\nnot a line\n{lbm.autotune_key(other, spec)}\t4 4 64 1.0\n"
                    f"{key}\t1 4 64 80.25\n")
    t = lbm.autotune(cfg, spec, cache=str(path))
    assert t["from_cache"] == 1 and t["candidates"] == 0
    assert (t["tune_zc"], t["tune_cpt"], t["tune_btx"], t["us_per_step"]) == (1, 4, 64, 80.25)


def test_header_is_plain_c(tmp_path):
    """include/lbm.h compiles as strict C99 (no C++ or torch types cross the
    boundary)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "abi.c"
    src.write_text('#include "lbm.h"\nint main(void) { lbm_config c; lbm_closure k; lbm_tuning t; lbm_qoi_rec r;\n'
                   '(void)c; (void)k; (void)t; (void)r; return LBM_OK; }\n')
    out = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                          os.path.join(root, "include"), "-c", str(src), "-o", str(tmp_path / "abi.o")],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr

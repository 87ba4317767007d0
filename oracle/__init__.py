"""FP64 CPU oracle of the TO-LRS lattice Boltzmann LES step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never touches it
and the two share no code: this wrapper loads ``liblbm_oracle.so`` built from
``lbm_oracle.c`` with plain gcc (no fast-math, no FMA contraction).

Each wrapper mirrors a routine of the C file; the paper passages they follow
are cited there (Sec. 2 LBM step, Sec. 3 LES forcing, Sec. 4 TO method,
Sec. 5 substrates, App. A sensitivities).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
OQMAX = 16

QOI_E, QOI_Z, QOI_MP = 0, 1, 2
FILT = {"I": 0, "B": 1, "B2": 2, "BMID": 3, "IMB": 4}
KERNEL_FILT = {"G": 5, "L": 6}   # with a scale: "G3" is G_3, "L1" is L_1


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's cell loops; returns the count in effect."""
    lib().orc_set_threads(int(n))
    return int(lib().orc_get_threads())


def threads() -> int:
    return int(lib().orc_get_threads())


def filter_code(name):
    """(code, scale, m) of a filter name: I, B, B2, BMID, IMB, G<s>, L<s>, or
    F<l>-<m> for the sharp Fourier band R_[l,m]."""
    if name in FILT:
        return FILT[name], 0, 0
    if name[0] == "F":
        lo, hi = name[1:].split("-")
        return 7, int(lo), int(hi)
    return KERNEL_FILT[name[0]], int(name[1:]), 0


MODE = {"off": 0, "track": 1, "lrs": 2}


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(outdir: str) -> str:
    """The oracle built with clang's AddressSanitizer and
    UndefinedBehaviorSanitizer into outdir (same arithmetic flags), for the
    host-sanitizer run of the CPU tests; load it by setting LBM_ORACLE_LIB."""
    os.makedirs(outdir, exist_ok=True)
    out = os.path.join(outdir, "liblbm_oracle.so")
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-fsanitize=address", "-fsanitize=undefined",
           "-fno-sanitize-recover=undefined", "-shared-libsan", "-shared", "-fPIC", "-std=c99", "-Wall",
           "-o", out, _SRC, "-lm", "-L/opt/rocm/llvm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"]
    subprocess.check_call(cmd)
    return out


class Cfg(ct.Structure):
    _fields_ = [("lattice", ct.c_int), ("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("walls_y", ct.c_int), ("tau", ct.c_double), ("substrate", ct.c_int),
                ("cmodel", ct.c_double), ("force_kind", ct.c_int), ("force_amp", ct.c_double),
                ("force_k", ct.c_int), ("drag", ct.c_double)]


class Closure(ct.Structure):
    _fields_ = [("nq", ct.c_int), ("kind", ct.c_int * OQMAX), ("filt", ct.c_int * OQMAX),
                ("band", ct.c_int * OQMAX), ("nbands", ct.c_int), ("dmin", ct.c_double),
                ("dmax", ct.c_double), ("mode", ct.c_int), ("spinup", ct.c_long),
                ("C", ct.c_double * ((OQMAX + 1) * OQMAX)), ("mu", ct.c_double * OQMAX),
                ("Sigma", ct.c_double * (OQMAX * OQMAX)), ("scale", ct.c_double * OQMAX),
                ("have_scale", ct.c_int), ("seed", ct.c_uint64), ("h", ct.c_int),
                ("Chist", ct.POINTER(ct.c_double)), ("fs", ct.c_int * OQMAX), ("fm", ct.c_int * OQMAX)]


class Rec(ct.Structure):
    _fields_ = [("step", ct.c_long), ("flags", ct.c_int), ("nq", ct.c_int), ("mass", ct.c_double),
                ("mom", ct.c_double * 3), ("diag_e", ct.c_double), ("diag_z", ct.c_double),
                ("q", ct.c_double * OQMAX), ("dq", ct.c_double * OQMAX),
                ("gamma", ct.c_double * OQMAX)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("LBM_ORACLE_LIB")
        if path is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = ct.CDLL(path)
        P, D, I = ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int
        L.orc_create.restype = P
        L.orc_create.argtypes = [ct.POINTER(Cfg)]
        L.orc_destroy.argtypes = [P]
        L.orc_init.argtypes = [P, P, P]
        L.orc_set_fp.argtypes = [P, P]
        L.orc_get_fp.argtypes = [P, P]
        L.orc_step_count.restype = ct.c_long
        L.orc_step_count.argtypes = [P]
        L.orc_stream_only.argtypes = [P]
        L.orc_velocity.argtypes = [P, P, P]
        L.orc_ncurl.argtypes = [P]
        L.orc_curl.argtypes = [P, P, P]
        L.orc_filter.argtypes = [P, I, I, I, P, P, I]
        L.orc_kernel.argtypes = [P, I, I, P]
        L.orc_band_weights.argtypes = [P, I, ct.c_double, ct.c_double, P]
        L.orc_qoi.argtypes = [P, ct.POINTER(Closure), P, P, P]
        L.orc_patterns.restype = I
        L.orc_patterns.argtypes = [P, ct.POINTER(Closure), P, P, P, P, P, P]
        L.orc_to_correction.restype = I
        L.orc_to_correction.argtypes = [P, ct.POINTER(Closure), P, P, P, P]
        L.orc_tau_smag.restype = ct.c_double
        L.orc_tau_smag.argtypes = [I, ct.c_double, ct.c_double, P, ct.c_double, P]
        L.orc_tau_wale_field.argtypes = [P, P, P]
        L.orc_philox.argtypes = [P, P, P]
        L.orc_lrs_normals.argtypes = [ct.c_uint64, ct.c_long, I, P]
        L.orc_set_closure.restype = I
        L.orc_set_closure.argtypes = [P, ct.POINTER(Closure), P, ct.c_long]
        L.orc_step.restype = I
        L.orc_step.argtypes = [P, ct.c_long]
        L.orc_set_fp32_store.argtypes = [P, I]
        L.orc_set_reverse_sums.argtypes = [P, I]
        L.orc_set_reduced_form.argtypes = [P, I]
        L.orc_set_threads.argtypes = [I]
        L.orc_get_threads.restype = I
        L.orc_nrec.restype = ct.c_long
        L.orc_nrec.argtypes = [P]
        L.orc_get_recs.argtypes = [P, ct.c_long, ct.c_long, P]
        L.orc_get_scale.restype = I
        L.orc_get_scale.argtypes = [P, P]
        L.orc_lattice.restype = I
        L.orc_lattice.argtypes = [I, P, P]
        L.orc_feq.argtypes = [I, ct.c_double, P, P]
        assert L.orc_sizeof_rec() == ct.sizeof(Rec)
        assert L.orc_sizeof_closure() == ct.sizeof(Closure)
        assert L.orc_sizeof_cfg() == ct.sizeof(Cfg)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def lattice(lat: int):
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    Q = lib().orc_lattice(lat, _p(c), _p(w))
    return c[:3 * Q].reshape(Q, 3).copy(), w[:Q].copy()


def feq_cells(lat: int, rho: float, u) -> np.ndarray:
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.zeros(19)
    lib().orc_feq(lat, float(rho), _p(uu), _p(out))
    return out[:9 if lat == 0 else 19].copy()


def tau_smag(lat: int, tau: float, C: float, f, rho: float, u) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    uu = np.zeros(3)
    uu[:len(u)] = u
    return lib().orc_tau_smag(lat, tau, C, _p(f), float(rho), _p(uu))


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(out))
    return out


def lrs_normals(seed: int, step: int, n: int) -> np.ndarray:
    z = np.zeros(n)
    lib().orc_lrs_normals(ct.c_uint64(seed), step, n, _p(z))
    return z


def make_closure(qois, mode="off", spinup=0, C=None, mu=None, Sigma=None, scale=None,
                 nbands=0, dmin=0.5, dmax=1.0, seed=0, h=0) -> Closure:
    """qois: list of (kind, filter_name, band) with kind in {'E','Z','MP'}.
    C is ((2h+1) nq + 1) x nq: rows for z^{n-1..n-h}, z*^n, z*^{n-1..n-h}, 1."""
    cl = Closure()
    cl.h = h
    cl.nq = len(qois)
    for k, (kind, filt, band) in enumerate(qois):
        cl.kind[k] = {"E": QOI_E, "Z": QOI_Z, "MP": QOI_MP}[kind]
        cl.filt[k], cl.fs[k], cl.fm[k] = filter_code(filt)
        cl.band[k] = band
    cl.nbands = nbands
    cl.dmin = dmin
    cl.dmax = dmax
    cl.mode = MODE[mode]
    cl.spinup = spinup
    nq = len(qois)
    if C is not None and h > 0:
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape((2 * h + 1) * nq + 1, nq))
        cl._chist = C          # keeps the array alive; the oracle copies it
        cl.Chist = C.ctypes.data_as(ct.POINTER(ct.c_double))
    elif C is not None:
        C = np.asarray(C, dtype=np.float64).reshape(nq + 1, nq)
        for i in range(nq + 1):
            for j in range(nq):
                cl.C[i * nq + j] = C[i, j]
    if mu is not None:
        for k in range(nq):
            cl.mu[k] = mu[k]
    if Sigma is not None:
        S = np.asarray(Sigma, dtype=np.float64).reshape(nq, nq)
        for i in range(nq):
            for j in range(nq):
                cl.Sigma[i * nq + j] = S[i, j]
    if scale is not None:
        for k in range(nq):
            cl.scale[k] = scale[k]
        cl.have_scale = 1
    cl.seed = seed
    return cl


class Oracle:
    """One oracle LES run.  Fields use numpy layout (comp, z, y, x) flattened."""

    def __init__(self, lattice=0, nx=16, ny=16, nz=1, walls_y=0, tau=0.6, substrate=0,
                 cmodel=0.0, force_kind=0, force_amp=0.0, force_k=0, drag=0.0):
        self.L = lib()
        self.cfg = Cfg(lattice, nx, ny, nz if lattice == 1 else 1, walls_y, tau, substrate,
                       cmodel, force_kind, force_amp, force_k, drag)
        self.h = self.L.orc_create(ct.byref(self.cfg))
        self.d = 2 if lattice == 0 else 3
        self.Q = 9 if lattice == 0 else 19
        self.N = nx * ny * self.cfg.nz
        self.shape = (self.cfg.nz, ny, nx)
        self.closure = None

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def init(self, u, rho=None):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.d, self.N)
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        self.L.orc_init(self.h, _p(r), _p(u))

    def set_fp(self, fp):
        fp = np.ascontiguousarray(fp, dtype=np.float64).reshape(self.Q, self.N)
        self.L.orc_set_fp(self.h, _p(fp))

    def get_fp(self):
        fp = np.zeros((self.Q, self.N))
        self.L.orc_get_fp(self.h, _p(fp))
        return fp

    def set_closure(self, cl: Closure | None, qref=None):
        self.closure = cl
        if cl is None:
            return self.L.orc_set_closure(self.h, None, None, 0)
        qr = None if qref is None else np.ascontiguousarray(qref, dtype=np.float64)
        nref = 0 if qr is None else qr.shape[0]
        rc = self.L.orc_set_closure(self.h, ct.byref(cl), _p(qr), nref)
        if rc != 0:
            raise ValueError("oracle rejected the closure")
        return rc

    def set_fp32_store(self, on=True):
        """Diagnostic: round the stored state (populations as f - w, and v*)
        to FP32 every step, all arithmetic still FP64 (the FP32 storage floor)."""
        self.L.orc_set_fp32_store(self.h, 1 if on else 0)

    def set_reverse_sums(self, on=True):
        """Diagnostic: the TO step's global sums in reverse cell order (the
        FP64 resolution of a closure against any other summation order)."""
        self.L.orc_set_reverse_sums(self.h, 1 if on else 0)

    def set_reduced_form(self, on=True):
        """Diagnostic: the correction as sum_j (G^-1 dQ)_j V_j instead of the
        literal patterns (equal in exact arithmetic)."""
        self.L.orc_set_reduced_form(self.h, 1 if on else 0)

    def step(self, n=1):
        self.L.orc_step(self.h, n)

    @property
    def step_count(self):
        return self.L.orc_step_count(self.h)

    def stream_only(self):
        self.L.orc_stream_only(self.h)

    def post_collision_velocity(self):
        """rho and u = sum c f^p / sum f^p of the post-collision state f^p (the
        run's state between steps; for a plain run with the exact-difference
        force this is the predictor velocity v* of the step that made it)."""
        fp = self.get_fp()
        c, _ = lattice(self.cfg.lattice)
        rho = fp.sum(axis=0)
        u = np.array([(c[:, a][:, None] * fp).sum(axis=0) for a in range(self.d)]) / rho
        return rho, u

    def velocity(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.d, self.N))
        self.L.orc_velocity(self.h, _p(rho), _p(u))
        return rho, u

    def records(self, first=0, count=None):
        n = self.L.orc_nrec(self.h)
        if count is None:
            count = n - first
        arr = (Rec * count)()
        self.L.orc_get_recs(self.h, first, count, arr)
        return arr

    def record_arrays(self):
        recs = self.records()
        nq = self.closure.nq if self.closure is not None else 0
        out = {
            "step": np.array([r.step for r in recs]),
            "flags": np.array([r.flags for r in recs]),
            "mass": np.array([r.mass for r in recs]),
            "mom": np.array([list(r.mom) for r in recs]),
            "diag_e": np.array([r.diag_e for r in recs]),
            "diag_z": np.array([r.diag_z for r in recs]),
            "q": np.array([list(r.q)[:nq] for r in recs]),
            "dq": np.array([list(r.dq)[:nq] for r in recs]),
            "gamma": np.array([list(r.gamma)[:nq] for r in recs]),
        }
        return out

    def scale(self):
        s = np.zeros(OQMAX)
        ok = self.L.orc_get_scale(self.h, _p(s))
        return s[: self.closure.nq].copy() if ok else None

    # building blocks --------------------------------------------------
    def curl(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.d, self.N)
        nc = self.L.orc_ncurl(self.h)
        w = np.zeros((nc, self.N))
        self.L.orc_curl(self.h, _p(v), _p(w))
        return w

    def filter(self, filt, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        nc = u.size // self.N
        out = np.zeros_like(u)
        code, sc, fm = filter_code(filt)
        self.L.orc_filter(self.h, code, sc, fm, _p(u), _p(out), nc)
        return out

    def kernel(self, name):
        """The d-dimensional kernel of G<s> or L<s>, shape (2R+1,)*d with
        axes (z,) y, x."""
        code, sc, _ = filter_code(name)
        R = self.L.orc_kernel(self.h, code, sc, None)
        W = 2 * R + 1
        k = np.zeros(W ** self.d)
        self.L.orc_kernel(self.h, code, sc, _p(k))
        return k.reshape((W,) * self.d)

    def band_weights(self, nb, dmin, dmax):
        w = np.zeros((nb, self.cfg.ny))
        self.L.orc_band_weights(self.h, nb, dmin, dmax, _p(w))
        return w

    def qoi(self, cl: Closure, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.d, self.N)
        q = np.zeros(cl.nq)
        V = np.zeros((cl.nq, self.d, self.N))
        self.L.orc_qoi(self.h, ct.byref(cl), _p(v), _p(q), _p(V))
        return q, V

    def patterns(self, cl: Closure, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.d, self.N)
        nq = cl.nq
        q = np.zeros(nq)
        V = np.zeros((nq, self.d, self.N))
        G = np.zeros((nq, nq))
        O = np.zeros((nq, self.d, self.N))
        den = np.zeros(nq)
        sing = self.L.orc_patterns(self.h, ct.byref(cl), _p(v), _p(q), _p(V), _p(G), _p(O), _p(den))
        return dict(q=q, V=V, G=G, O=O, den=den, singular=bool(sing))

    def to_correction(self, cl: Closure, v, dq):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.d, self.N)
        dq = np.ascontiguousarray(dq, dtype=np.float64)
        dv = np.zeros((self.d, self.N))
        gamma = np.zeros(cl.nq)
        sing = self.L.orc_to_correction(self.h, ct.byref(cl), _p(v), _p(dq), _p(dv), _p(gamma))
        return dv, gamma, bool(sing)

    def tau_wale(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.d, self.N)
        t = np.zeros(self.N)
        self.L.orc_tau_wale_field(self.h, _p(v), _p(t))
        return t


def lrs_inputs(q, qs, h, s):
    """Rows of the LRS design matrix and targets from a trajectory (eq. LRS).

    q, qs: (M, nq) corrected and predictor QoIs of steps 0..M-1; s: scale.
    Row n (n = h..M-1) is x^n = [z^{n-1}, ..., z^{n-h}, z*^n, ..., z*^{n-h}, 1]
    with z = q / s; its target is z^n."""
    q = np.asarray(q, dtype=np.float64) / s
    qs = np.asarray(qs, dtype=np.float64) / s
    M, nq = q.shape
    rows, tgt = [], []
    for n in range(h, M):
        x = [q[n - r] for r in range(1, h + 1)] + [qs[n - r] for r in range(0, h + 1)] + [np.ones(1)]
        rows.append(np.concatenate(x))
        tgt.append(q[n])
    return np.array(rows), np.array(tgt)


def lrs_fit(q, qs, h, lam, scale=None):
    """Ridge fit of the LRS model (Sec. 4.4): C minimises
    1/2 |Q_h X - Q|_F^2 + 1/2 sum_i lam_i |X_i|^2 column by column, with
    lam_i = lam (sigma_i / sigma_1)^2 and sigma_i the standard deviation of
    the scaled corrections z^n - z*^n; inputs and targets scaled by s (the
    standard deviation of each QoI over the trajectory unless given; no mean
    removal).  Residual statistics: mean and unbiased sample covariance of
    Q - Q_h C.  Each column solves its normal equations directly.
    Returns C, mu, Sigma, s."""
    q = np.asarray(q, dtype=np.float64)
    qs = np.asarray(qs, dtype=np.float64)
    if scale is None:
        s = q.std(axis=0)
        s[s == 0] = 1.0
    else:
        s = np.asarray(scale, dtype=np.float64)
    X, Y = lrs_inputs(q, qs, h, s)
    corr = (q - qs)[h:] / s
    sig = corr.std(axis=0)
    lam_i = lam * (sig / sig[0]) ** 2 if sig[0] > 0 else np.full(len(sig), float(lam))
    A = X.T @ X
    C = np.zeros((X.shape[1], Y.shape[1]))
    for i in range(Y.shape[1]):
        C[:, i] = np.linalg.solve(A + lam_i[i] * np.eye(A.shape[0]), X.T @ Y[:, i])
    R = Y - X @ C
    mu = R.mean(axis=0)
    Sigma = np.cov(R, rowvar=False, ddof=1).reshape(Y.shape[1], Y.shape[1])
    return C, mu, Sigma, s


def project(field, shape, m):
    """Wall-anchored stride-m projection phi_m (Sec. 3; Sec. 7.1 for the
    channel): coarse cell (i, j, k) takes the fine cell (m i + o, m j + o,
    m k + o), o = (m - 1) / 2 (m odd), so that the coarse walls, half a
    coarse cell beyond the first and last coarse rows, sit where the fine
    walls sit: the first coarse row is o + 1/2 = m / 2 fine cells from the
    wall.  field: (ncomp, N) in the (z, y, x) layout of `shape` = (nz, ny, nx);
    the z axis is kept as is when nz == 1."""
    if m < 1 or m % 2 == 0:
        raise ValueError("m must be odd")
    nz, ny, nx = shape
    f = np.asarray(field).reshape(-1, nz, ny, nx)
    o = (m - 1) // 2
    zs = slice(o, None, m) if nz > 1 else slice(None)
    out = f[:, zs, o::m, o::m]
    return np.ascontiguousarray(out.reshape(out.shape[0], -1))


def keys_cubic(t):
    """The cubic convolution kernel of Keys (1981) with a = -1/2:
    1.5|t|^3 - 2.5|t|^2 + 1 for |t| <= 1, -0.5|t|^3 + 2.5|t|^2 - 4|t| + 2 for
    1 < |t| < 2, zero beyond."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(t <= 1, 1.5 * t ** 3 - 2.5 * t ** 2 + 1,
                    np.where(t < 2, -0.5 * t ** 3 + 2.5 * t ** 2 - 4 * t + 2, 0.0))


def bicubic_matrix(nf, m):
    """The 1-D factor of the bicubic projection phi_m of a periodic axis
    (Sec. 3, the Kolmogorov case): coarse cell i is the weighted mean of the
    fine cells j = m i + o + r (o = (m - 1) / 2, m odd, periodic wrap), with
    weights keys_cubic(r / m) for |r| < 2 m normalised to unit sum (the
    kernel widened m-fold for the m-fold coarser grid).  Returns the
    (nf / m) x nf matrix."""
    if m < 1 or m % 2 == 0 or nf % m:
        raise ValueError("m must be odd and divide the axis")
    nc, o = nf // m, (m - 1) // 2
    r = np.arange(-2 * m + 1, 2 * m)
    w = keys_cubic(r / m)
    w = w / w.sum()
    W = np.zeros((nc, nf))
    for i in range(nc):
        for rr, ww in zip(r, w):
            W[i, (m * i + o + rr) % nf] += ww
    return W


def project_bicubic(field, shape, m):
    """Bicubic projection phi_m of a doubly periodic 2-D field (Sec. 3, the
    Kolmogorov case), the tensor product of bicubic_matrix along y and x.
    field: (ncomp, N) in the (1, ny, nx) layout of `shape`."""
    nz, ny, nx = shape
    if nz != 1:
        raise ValueError("2-D fields only")
    f = np.asarray(field, dtype=np.float64).reshape(-1, ny, nx)
    Wy, Wx = bicubic_matrix(ny, m), bicubic_matrix(nx, m)
    out = np.einsum("ab,cbd,ed->cae", Wy, f, Wx)
    return np.ascontiguousarray(out.reshape(out.shape[0], -1))


def ks_distance(a, b) -> float:
    """KS distance of two scalar samples (Sec. 3.1, eq. KS):
    the largest absolute difference between their empirical cumulative
    distribution functions F and G.  Both are step functions that change
    only at sample points, so the maximum is taken over the pooled sample
    points, with F(x) the fraction of a at or below x."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    b = np.sort(np.asarray(b, dtype=np.float64).ravel())
    x = np.concatenate([a, b])
    F = np.searchsorted(a, x, side="right") / a.size
    G = np.searchsorted(b, x, side="right") / b.size
    return float(np.max(np.abs(F - G)))

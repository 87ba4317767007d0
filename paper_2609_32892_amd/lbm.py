"""ctypes binding of liblbm_hip.so (include/lbm.h).

Argument marshalling only: every step of the LES runs in the library's HIP
kernels.  PyTorch provides the device arena and the stream.  There is no
fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_HIP_LIB selects another build of the library (the host-sanitizer
# build of the CPU tests); by default the in-tree one.
LIB_PATH = os.environ.get("LBM_HIP_LIB") or os.path.join(HERE, "liblbm_hip.so")
MAX_QOI = 16

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19 = 0, 1
FP32_SHIFTED, FP64, FP32_PLAIN = 0, 1, 2
BGK, SMAGORINSKY, WALE = 0, 1, 2
FORCE_NONE, FORCE_SIN_Y, FORCE_CONST_X = 0, 1, 2
QOI_E, QOI_Z, QOI_MP = 0, 1, 2
FILT = {"I": 0, "B": 1, "B2": 2, "BMID": 3, "IMB": 4}
KFILT = {"G": 5, "L": 6}   # kernel filters with a scale: "G3" = G_3, "L1" = L_1


def filter_code(name):
    """(filter enum, scale, kmax) of a filter name: I, B, B2, BMID, IMB, G<s>,
    L<s>, or F<l>-<m> for the sharp Fourier band R_[l,m]."""
    if name in FILT:
        return FILT[name], 0, 0
    if name[0] == "F":
        lo, hi = name[1:].split("-")
        return 7, int(lo), int(hi)
    return KFILT[name[0]], int(name[1:]), 0
MODE = {"off": 0, "track": 1, "lrs": 2}
PRECISION = {"fp32": FP32_SHIFTED, "fp64": FP64, "fp32_plain": FP32_PLAIN}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class Config(ct.Structure):
    _fields_ = [("lattice", ct.c_int), ("precision", ct.c_int), ("nx", ct.c_int), ("ny", ct.c_int),
                ("nz", ct.c_int), ("walls_y", ct.c_int), ("tau", ct.c_double), ("substrate", ct.c_int),
                ("c_model", ct.c_double), ("force_kind", ct.c_int), ("force_amp", ct.c_double),
                ("force_k", ct.c_int), ("drag", ct.c_double), ("diag", ct.c_int), ("rec_cap", ct.c_int),
                ("tune_zc", ct.c_int), ("tune_cpt", ct.c_int), ("tune_btx", ct.c_int),
                ("tune_mem", ct.c_int)]


class QoiSpec(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("filter", ct.c_int), ("band", ct.c_int), ("scale", ct.c_int),
                ("kmax", ct.c_int)]


class Closure(ct.Structure):
    _fields_ = [("nq", ct.c_int), ("q", ct.POINTER(QoiSpec)), ("nbands", ct.c_int),
                ("band_dmin", ct.c_double), ("band_dmax", ct.c_double), ("mode", ct.c_int),
                ("spinup", ct.c_long), ("h", ct.c_int), ("C", ct.POINTER(ct.c_double)),
                ("mu", ct.POINTER(ct.c_double)), ("Sigma", ct.POINTER(ct.c_double)),
                ("scale", ct.POINTER(ct.c_double)), ("qref", ct.POINTER(ct.c_double)),
                ("nref", ct.c_long), ("seed", ct.c_uint64)]


class Tuning(ct.Structure):
    _fields_ = [("tune_zc", ct.c_int), ("tune_cpt", ct.c_int), ("tune_btx", ct.c_int),
                ("us_per_step", ct.c_double), ("from_cache", ct.c_int), ("candidates", ct.c_int)]


class QoiRec(ct.Structure):
    _fields_ = [("step", ct.c_int64), ("flags", ct.c_int32), ("nq", ct.c_int32), ("mass", ct.c_double),
                ("mom", ct.c_double * 3), ("diag_e", ct.c_double), ("diag_z", ct.c_double),
                ("q", ct.c_double * MAX_QOI), ("dq", ct.c_double * MAX_QOI),
                ("gamma", ct.c_double * MAX_QOI)]


class Result(ct.Structure):
    _fields_ = [("id", ct.c_long), ("status", ct.c_int), ("steps", ct.c_long), ("cells", ct.c_long),
                ("t_arrival", ct.c_double), ("t_admit", ct.c_double), ("t_done", ct.c_double),
                ("last", QoiRec)]


#: symbols declared in include/lbm.h
EXPORTS = [
    "lbm_last_error", "lbm_version", "lbm_lattice_info", "lbm_required_bytes", "lbm_create",
    "lbm_destroy", "lbm_init_velocity", "lbm_set_closure", "lbm_step", "lbm_step_prepare", "lbm_sync",
    "lbm_step_count",
    "lbm_qoi", "lbm_fields", "lbm_velocity", "lbm_fields_noalloc", "lbm_get_populations", "lbm_set_populations", "lbm_stream_only",
    "lbm_state_bytes", "lbm_get_state", "lbm_set_state", "lbm_batch_create", "lbm_batch_step",
    "lbm_batch_sync", "lbm_batch_destroy", "lbm_profile_phases", "lbm_test_philox", "lbm_test_normals",
    "lbm_server_clock", "lbm_server_create", "lbm_server_submit", "lbm_server_advance", "lbm_server_poll",
    "lbm_server_pending", "lbm_server_stats", "lbm_server_state_bytes", "lbm_server_take_state",
    "lbm_server_destroy", "lbm_lrs_fit", "lbm_project_state", "lbm_project_qoi", "lbm_device_tag",
    "lbm_autotune_bytes", "lbm_autotune", "lbm_autotune_key", "lbm_project_state_kind", "lbm_project_qoi_kind",
]
PHASES = ["stream_collide", "curl", "binomial", "reduce", "solve", "apply"]
PROJ = {"stride": 0, "bicubic": 1}

_lib = None


def lib():
    """Load liblbm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2609_32892_amd/build.py")
        # torch first, so that the library binds to the HIP runtime torch
        # loads (the one that owns the streams and memory passed in); loaded
        # the other way round, a server created before any run found no device
        import torch  # noqa: F401
        L = ct.CDLL(LIB_PATH)
        P, I, Z = ct.c_void_p, ct.c_int, ct.c_size_t
        L.lbm_last_error.restype = ct.c_char_p
        L.lbm_version.restype = ct.c_char_p
        L.lbm_lattice_info.argtypes = [I, P, P]
        L.lbm_required_bytes.restype = Z
        L.lbm_required_bytes.argtypes = [ct.POINTER(Config), ct.POINTER(Closure)]
        L.lbm_create.argtypes = [ct.POINTER(Config), ct.POINTER(Closure), P, Z, P, ct.POINTER(P)]
        L.lbm_destroy.argtypes = [P]
        L.lbm_destroy.restype = None
        L.lbm_init_velocity.argtypes = [P, P, P]
        L.lbm_set_closure.argtypes = [P, ct.POINTER(Closure)]
        L.lbm_step.argtypes = [P, ct.c_long]
        L.lbm_step_prepare.argtypes = [P, ct.c_long]
        L.lbm_sync.argtypes = [P]
        L.lbm_step_count.restype = ct.c_long
        L.lbm_step_count.argtypes = [P]
        L.lbm_qoi.argtypes = [P, ct.c_long, ct.c_long, P]
        L.lbm_fields.argtypes = [P, P, P]
        L.lbm_velocity.argtypes = [P, P]
        L.lbm_fields_noalloc.argtypes = [P, P, P]
        L.lbm_get_populations.argtypes = [P, P]
        L.lbm_set_populations.argtypes = [P, P]
        L.lbm_stream_only.argtypes = [P]
        L.lbm_state_bytes.restype = Z
        L.lbm_state_bytes.argtypes = [P]
        L.lbm_get_state.argtypes = [P, P, Z]
        L.lbm_set_state.argtypes = [P, P, Z]
        L.lbm_batch_create.argtypes = [I, ct.POINTER(P), ct.POINTER(P)]
        L.lbm_batch_step.argtypes = [P, ct.c_long]
        L.lbm_batch_sync.argtypes = [P]
        L.lbm_batch_destroy.argtypes = [P]
        L.lbm_batch_destroy.restype = None
        L.lbm_profile_phases.argtypes = [P, ct.c_long, P, P]
        L.lbm_test_philox.argtypes = [P, P, I]
        L.lbm_test_normals.argtypes = [ct.c_uint64, ct.c_long, I, I, P]
        L.lbm_server_clock.restype = ct.c_double
        L.lbm_server_clock.argtypes = []
        L.lbm_server_create.argtypes = [Z, P, ct.POINTER(P)]
        L.lbm_server_submit.argtypes = [P, ct.POINTER(Config), ct.POINTER(Closure), P, ct.c_long, ct.c_double,
                                        I, ct.POINTER(ct.c_long)]
        L.lbm_server_advance.argtypes = [P, ct.c_double, ct.c_long, ct.POINTER(I)]
        L.lbm_server_poll.argtypes = [P, P, I, ct.POINTER(I)]
        L.lbm_server_pending.argtypes = [P]
        L.lbm_server_stats.argtypes = [P, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.POINTER(Z),
                                       ct.POINTER(Z)]
        L.lbm_server_state_bytes.restype = Z
        L.lbm_server_state_bytes.argtypes = [P, ct.c_long]
        L.lbm_server_take_state.argtypes = [P, ct.c_long, P, Z]
        L.lbm_server_destroy.argtypes = [P]
        L.lbm_server_destroy.restype = None
        L.lbm_lrs_fit.argtypes = [I, I, ct.c_long, P, P, P, P, ct.c_double, P, P, P, P]
        L.lbm_device_tag.argtypes = [ct.c_char_p, Z]
        L.lbm_autotune_key.argtypes = [ct.POINTER(Config), ct.POINTER(Closure), ct.c_char_p, Z]
        L.lbm_autotune_bytes.restype = Z
        L.lbm_autotune_bytes.argtypes = [ct.POINTER(Config), ct.POINTER(Closure)]
        L.lbm_autotune.argtypes = [ct.POINTER(Config), ct.POINTER(Closure), P, Z, P, I, ct.c_char_p,
                                   ct.POINTER(Tuning)]
        L.lbm_project_state.argtypes = [P, P, I]
        L.lbm_project_qoi.argtypes = [P, P, I]
        L.lbm_project_state_kind.argtypes = [P, P, I, I]
        L.lbm_project_qoi_kind.argtypes = [P, P, I, I]
        _lib = L
    return _lib


def check(rc):
    if rc < 0:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def device_tag():
    """The current HIP device's name and compute-unit count (lbm_device_tag)."""
    L = lib()
    buf = ct.create_string_buffer(128)
    check(L.lbm_device_tag(buf, 128))
    return buf.value.decode()


def autotune_key(cfg: "Config", closure: "ClosureSpec | None" = None):
    """The tuning-cache key of cfg and closure on the current device."""
    L = lib()
    buf = ct.create_string_buffer(4096)
    check(L.lbm_autotune_key(ct.byref(cfg), ct.byref(closure.c) if closure is not None else None, buf, 4096))
    return buf.value.decode()


def autotune(cfg: "Config", closure: "ClosureSpec | None" = None, steps=200, cache=None, device="cuda"):
    """Time the launch-shape candidates of cfg (lbm_autotune) in a scratch
    arena and return the chosen tuning as a dict: tune_zc, tune_cpt and
    tune_btx (keyword arguments of make_config), us_per_step, from_cache and
    candidates.  cache: path of the tuning cache file (or None)."""
    import torch
    L = lib()
    clp = ct.byref(closure.c) if closure is not None else None
    nbytes = L.lbm_autotune_bytes(ct.byref(cfg), clp)
    if nbytes == 0:
        raise LbmError(EINVAL, L.lbm_last_error().decode())
    out = Tuning()
    path = None if cache is None else os.fsencode(cache)
    arena = None
    if cache is not None and os.path.exists(cache):
        # a cache hit needs no arena: try without one first
        rc = L.lbm_autotune(ct.byref(cfg), clp, None, 0, None, steps, path, ct.byref(out))
        if rc == OK and out.from_cache:
            return {f: getattr(out, f) for f, _ in Tuning._fields_}
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = arena.data_ptr()
    off = (-base) % 256
    with torch.cuda.device(arena.device):
        check(L.lbm_autotune(ct.byref(cfg), clp, ct.c_void_p(base + off), nbytes,
                             ct.c_void_p(default_stream().cuda_stream), steps, path, ct.byref(out)))
    del arena
    return {f: getattr(out, f) for f, _ in Tuning._fields_}


def lrs_fit(q_star, dq, h, lam, scale=None, flags=None):
    """Fit the LRS model to a recorded trajectory (lbm_lrs_fit): q_star and
    dq are (nsteps, nq) arrays (e.g. the records of a tracking run).
    Returns (C, mu, Sigma, s) ready for ClosureSpec(mode="lrs", h=h, ...)."""
    qs = np.ascontiguousarray(q_star, dtype=np.float64)
    d = np.ascontiguousarray(dq, dtype=np.float64)
    M, nq = qs.shape
    if d.shape != qs.shape:
        raise ValueError("q_star and dq must have the same shape")
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.int32)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    C = np.zeros(((2 * h + 1) * nq + 1, nq))
    mu = np.zeros(nq)
    S = np.zeros((nq, nq))
    s = np.zeros(nq)
    check(lib().lbm_lrs_fit(nq, h, M, _p(qs), _p(d), _p(fl), _p(sc), float(lam), _p(C), _p(mu), _p(S), _p(s)))
    return C, mu, S, s


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def lattice_info(lattice: int):
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    Q = check(lib().lbm_lattice_info(lattice, _p(c), _p(w)))
    return c[: 3 * Q].reshape(Q, 3).copy(), w[:Q].copy()


def make_config(lattice=D2Q9, precision=FP32_SHIFTED, nx=64, ny=64, nz=1, walls_y=0, tau=0.6,
                substrate=BGK, cmodel=0.0, force_kind=FORCE_NONE, force_amp=0.0, force_k=0, drag=0.0,
                diag=0, rec_cap=0, tune_zc=0, tune_cpt=0, tune_btx=0, tune_mem=0) -> Config:
    if isinstance(precision, str):
        precision = PRECISION[precision]
    return Config(lattice, precision, nx, ny, nz if lattice == D3Q19 else 1, walls_y, tau, substrate,
                  cmodel, force_kind, force_amp, force_k, drag, diag, rec_cap, tune_zc, tune_cpt, tune_btx,
                  tune_mem)


class ClosureSpec:
    """Owns the host arrays a Closure struct points to."""

    def __init__(self, qois, mode="off", spinup=0, C=None, mu=None, Sigma=None, scale=None,
                 qref=None, nbands=0, dmin=0.5, dmax=1.0, seed=0, h=0):
        nq = len(qois)
        self.nq = nq
        self._q = (QoiSpec * nq)()
        for k, (kind, filt, band) in enumerate(qois):
            code, sc, km = filter_code(filt)
            self._q[k] = QoiSpec({"E": QOI_E, "Z": QOI_Z, "MP": QOI_MP}[kind], code, band, sc, km)
        arr = lambda a, n: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n))
        self._C = arr(C, ((2 * h + 1) * nq + 1) * nq)
        self._mu = arr(mu, nq)
        self._S = arr(Sigma, nq * nq)
        self._scale = arr(scale, nq)
        self._qref = None if qref is None else np.ascontiguousarray(np.asarray(qref, dtype=np.float64))
        self.c = Closure()
        self.c.nq = nq
        self.c.q = ct.cast(self._q, ct.POINTER(QoiSpec))
        self.c.nbands = nbands
        self.c.band_dmin = dmin
        self.c.band_dmax = dmax
        self.c.mode = MODE[mode] if isinstance(mode, str) else mode
        self.c.spinup = spinup
        self.c.h = h
        self.c.C = _dptr(self._C)
        self.c.mu = _dptr(self._mu)
        self.c.Sigma = _dptr(self._S)
        self.c.scale = _dptr(self._scale)
        self.c.qref = _dptr(self._qref)
        self.c.nref = 0 if self._qref is None else self._qref.shape[0]
        self.c.seed = seed


_default_stream = None


def default_stream():
    """A dedicated torch stream (default priority) shared by runs that are not given one."""
    global _default_stream
    import torch
    if _default_stream is None:
        _default_stream = torch.cuda.Stream()
    return _default_stream


class Run:
    """One LES run (an lbm_ctx) whose state lives in a torch-allocated arena."""

    def __init__(self, cfg: Config, closure: ClosureSpec | None = None, stream=None, device="cuda"):
        import torch
        self.L = lib()
        self.cfg = cfg
        self.d = 2 if cfg.lattice == D2Q9 else 3
        self.Q = 9 if cfg.lattice == D2Q9 else 19
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.closure = closure
        clp = ct.byref(closure.c) if closure is not None else None
        nbytes = self.L.lbm_required_bytes(ct.byref(cfg), clp)
        if nbytes == 0:
            raise LbmError(EINVAL, self.L.lbm_last_error().decode())
        self.nbytes = nbytes
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else default_stream()
        h = ct.c_void_p()
        with torch.cuda.device(self.arena.device):
            check(self.L.lbm_create(ct.byref(cfg), clp, ct.c_void_p(base + off), nbytes,
                                    ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # -- state ----------------------------------------------------------------
    def init_velocity(self, u, rho=None):
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.d, self.N))
        r = None if rho is None else np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(self.N))
        check(self.L.lbm_init_velocity(self.h, _p(r), _p(u)))

    def set_closure(self, closure: ClosureSpec | None):
        self.closure = closure
        check(self.L.lbm_set_closure(self.h, ct.byref(closure.c) if closure is not None else None))

    def step(self, n=1):
        check(self.L.lbm_step(self.h, n))

    def prepare(self, n):
        """Capture the graphs step(n) will replay (nothing runs)."""
        check(self.L.lbm_step_prepare(self.h, n))

    def sync(self):
        return check(self.L.lbm_sync(self.h))

    @property
    def step_count(self):
        return self.L.lbm_step_count(self.h)

    def records(self, first=0, count=None):
        if count is None:
            count = self.step_count - first
        arr = (QoiRec * count)()
        check(self.L.lbm_qoi(self.h, first, count, ct.cast(arr, ct.c_void_p)))
        return arr

    def record_arrays(self, first=0, count=None):
        recs = self.records(first, count)
        nq = self.closure.nq if self.closure is not None else 0
        return {
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

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.d, self.N))
        check(self.L.lbm_fields(self.h, _p(rho), _p(u)))
        return rho, u

    def velocity(self):
        """The velocity alone (lbm_velocity)."""
        u = np.zeros((self.d, self.N))
        check(self.L.lbm_velocity(self.h, _p(u)))
        return u

    def fields_noalloc(self):
        """fields() through lbm_fields_noalloc (no allocation in the library)."""
        rho = np.zeros(self.N)
        u = np.zeros((self.d, self.N))
        check(self.L.lbm_fields_noalloc(self.h, _p(rho), _p(u)))
        return rho, u

    def get_populations(self):
        f = np.zeros((self.Q, self.N))
        check(self.L.lbm_get_populations(self.h, _p(f)))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(self.Q, self.N))
        check(self.L.lbm_set_populations(self.h, _p(f)))

    def stream_only(self):
        check(self.L.lbm_stream_only(self.h))

    def project_state_from(self, fine: "Run", m: int, kind: str = "stride"):
        """This (coarse) run's state becomes the projection phi_m of the fine
        run's state (lbm_project_state_kind; kind "stride" or "bicubic")."""
        check(self.L.lbm_project_state_kind(fine.h, self.h, m, PROJ[kind]))

    def project_qoi_from(self, fine: "Run", m: int, kind: str = "stride"):
        """Append the QoIs of the fine run's projected post-collision
        velocity as this probe's next record (lbm_project_qoi_kind)."""
        check(self.L.lbm_project_qoi_kind(fine.h, self.h, m, PROJ[kind]))

    def profile_phases(self, nsteps):
        """Mean ms per step and launches per step of each kernel phase."""
        ms = np.zeros(6)
        nl = np.zeros(6, dtype=np.int32)
        check(self.L.lbm_profile_phases(self.h, nsteps, _p(ms), _p(nl)))
        return dict(zip(PHASES, ms.tolist())), dict(zip(PHASES, nl.tolist()))

    def get_state(self) -> bytes:
        n = self.L.lbm_state_bytes(self.h)
        buf = ct.create_string_buffer(n)
        check(self.L.lbm_get_state(self.h, buf, n))
        return buf.raw

    def set_state(self, data: bytes):
        buf = ct.create_string_buffer(data, len(data))
        check(self.L.lbm_set_state(self.h, buf, len(data)))


class Batch:
    """Several runs advanced together (lbm_batch)."""

    def __init__(self, runs):
        self.L = lib()
        self.runs = list(runs)
        arr = (ct.c_void_p * len(self.runs))(*[r.h.value for r in self.runs])
        h = ct.c_void_p()
        check(self.L.lbm_batch_create(len(self.runs), arr, ct.byref(h)))
        self.h = h

    def step(self, n=1):
        check(self.L.lbm_batch_step(self.h, n))

    def sync(self):
        return check(self.L.lbm_batch_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Server:
    """Continuous-batching LES server (lbm_server)."""

    def __init__(self, hbm_budget=0, stream=None):
        self.L = lib()
        self.stream = stream if stream is not None else default_stream()
        h = ct.c_void_p()
        check(self.L.lbm_server_create(hbm_budget, ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        self.h = h

    def clock(self):
        return self.L.lbm_server_clock()

    def submit(self, cfg: Config, closure: ClosureSpec | None, u0, nsteps, t_arrival, keep_state=False):
        u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.float64))
        rid = ct.c_long()
        check(self.L.lbm_server_submit(self.h, ct.byref(cfg), ct.byref(closure.c) if closure else None,
                                       _p(u0), nsteps, t_arrival, int(keep_state), ct.byref(rid)))
        return rid.value

    def advance(self, now, max_chunk=0):
        n = ct.c_int()
        check(self.L.lbm_server_advance(self.h, now, max_chunk, ct.byref(n)))
        return n.value

    def poll(self, cap=1024):
        arr = (Result * cap)()
        n = ct.c_int()
        check(self.L.lbm_server_poll(self.h, ct.cast(arr, ct.c_void_p), cap, ct.byref(n)))
        return [arr[i] for i in range(n.value)]

    def pending(self):
        return self.L.lbm_server_pending(self.h)

    def stats(self):
        busy, lups = ct.c_double(), ct.c_double()
        used, budget = ct.c_size_t(), ct.c_size_t()
        check(self.L.lbm_server_stats(self.h, ct.byref(busy), ct.byref(lups), ct.byref(used), ct.byref(budget)))
        return dict(busy_s=busy.value, lups=lups.value, used=used.value, budget=budget.value)

    def take_state(self, rid) -> bytes:
        n = self.L.lbm_server_state_bytes(self.h, rid)
        buf = ct.create_string_buffer(n)
        check(self.L.lbm_server_take_state(self.h, rid, buf, n))
        return buf.raw

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def test_philox(vectors):
    v = np.ascontiguousarray(np.asarray(vectors, dtype=np.uint32).reshape(-1, 6))
    out = np.zeros((v.shape[0], 4), dtype=np.uint32)
    check(lib().lbm_test_philox(_p(v), _p(out), v.shape[0]))
    return out


def test_normals(seed, step0, nsteps, n):
    out = np.zeros((nsteps, n))
    check(lib().lbm_test_normals(ct.c_uint64(seed), step0, nsteps, n, _p(out)))
    return out

/*
 * lbm.h -- C ABI of the MI355X TO-LRS lattice Boltzmann LES library
 * (liblbm_hip.so, HIP kernels for gfx950).
 *
 * The library advances lattice Boltzmann LES runs with the Tau-orthogonal
 * (TO) closure of Hoekstra, Xue, Coveney and Edeling, "Reduced Subgrid-Scale
 * Terms for Turbulence Simulations with the Lattice Boltzmann Method":
 *   - one LES step is eqs. LES-1..LES-3 (Sec. 3): BGK relaxation with an
 *     optional eddy-viscosity substrate (Sec. 5: eq. eff-relaxation, the
 *     Smagorinsky closed form, WALE), exact-difference forcing with the
 *     body force and the SGS velocity increment dv_SGS (eq. LES-2), then
 *     streaming (eq. LES-3) with halfway bounce-back walls (Sec. 7.1);
 *   - dv_SGS = sum_i gamma_i O_i (eq. TO-ansatz) with patterns built from
 *     the QoI sensitivities (eq. O-from-V, App. A) so that
 *     <dQ_i/dv, O_j> = 0 for i != j (eq. orthogonality);
 *   - the coefficients follow from dQ (eq. tau-from-dQ-for-tracking), with
 *     dQ from a reference trajectory (tracking, eq. dQ-from-ref) or from a
 *     linear regression with stochastic residuals (eq. LRS, h = 0).
 * QoIs (Sec. 4.1): filtered energy E_R = 1/2 sum |R v|^2, filtered enstrophy
 * Z_R = 1/2 sum |R curl v|^2 and mean-profile QoIs sum w_j(y) v_x
 * (eq. mean-profile-qoi, bands of eq. 3d-mp-band-weights); integrals are sums
 * over cells with unit volume.  Filters are polynomials in the 3^d binomial
 * operator B = (x)_a [1,2,1]/4 with zero padding on the wall axis.
 *
 * Conventions
 *   - Fields are structure-of-arrays, x fastest: cell = x + nx*(y + ny*z).
 *   - Host arrays passed to the library are double precision.
 *   - All device work of a context is ordered on the HIP stream given at
 *     creation; calls that return host data synchronise that stream.
 *   - Every call returns LBM_OK (0) or a negative status; the message of the
 *     last failure on the calling thread is in lbm_last_error().  No call
 *     aborts or throws.  Invalid arguments leave the object unchanged.
 *   - One context (or batch, or server) per host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MAX_QOI 16
#define LBM_MAX_HIST 1024   /* LRS history length; also 2 h nq <= 32768 */

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or configuration */
    LBM_ENOMEM = -2,     /* arena too small / allocation failed */
    LBM_EDEVICE = -3,    /* HIP runtime error */
    LBM_EUNSTABLE = -4,  /* a run produced a non-finite value or |v| > 0.5 (sticky) */
    LBM_ESTATE = -5      /* request outside the retained state (e.g. overwritten records) */
};

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
/* Population storage: FP32 deviations g = f - w_i (arithmetic in FP32),
 * FP64 deviations, or plain FP32 populations f (the unshifted baseline). */
enum { LBM_FP32_SHIFTED = 0, LBM_FP64 = 1, LBM_FP32_PLAIN = 2 };
enum { LBM_BGK = 0, LBM_SMAGORINSKY = 1, LBM_WALE = 2 };
/* Body force: none, F_x = amp sin(2 pi k y / ny) (Kolmogorov flow, Sec. 6.1,
 * y the integer row index), or constant F_x = amp (channel, Sec. 7.1).
 * An optional linear drag subtracts drag * rho * v. */
enum { LBM_FORCE_NONE = 0, LBM_FORCE_SIN_Y = 1, LBM_FORCE_CONST_X = 2 };

typedef struct {
    int lattice;        /* LBM_D2Q9 or LBM_D3Q19 */
    int precision;      /* LBM_FP32_SHIFTED, LBM_FP64, LBM_FP32_PLAIN */
    int nx, ny, nz;     /* nz must be 1 for D2Q9 */
    int walls_y;        /* 0 periodic in y; 1 halfway bounce-back walls at y=-1/2, ny-1/2 */
    double tau;         /* BGK relaxation time, > 1/2 */
    int substrate;      /* LBM_BGK, LBM_SMAGORINSKY, LBM_WALE (WALE: D3Q19 only) */
    double c_model;     /* C_smag or C_w */
    int force_kind;
    double force_amp;
    int force_k;
    double drag;
    int diag;           /* plain runs: 1 records mass, momentum, E and Z of the
                           post-streaming velocity every step */
    int rec_cap;        /* capacity of the per-step record ring (0: 4096) */
    int tune_zc;        /* tuning: z planes per binomial-filter workgroup (0: automatic) */
    int tune_cpt;       /* tuning: cells per thread of the QoI reduction (0: automatic) */
    int tune_btx;       /* tuning: binomial tile width, 32 or 64 (0: automatic; 64 needs a
                           D3Q19 grid; bitwise the same result either way) */
    int tune_mem;       /* memory-access variant of the step (0: automatic by size): bit 0
                           forces 64-bit population offsets, bit 1 non-temporal population
                           stores in plain runs, bit 2 the SGS change recorded and applied
                           by the next step's pull (binomial closures, BGK or Smagorinsky
                           substrate) also where the populations (up to 192 MB) would
                           apply it in place, bit 3 the closure's solve in a launch of its
                           own also where the apply would form it (binomial closures on
                           launches of at most 1024 blocks of 256 cells, paired into 512
                           workgroups); bitwise the same
                           result either way (for tests of the large-grid forms); 0..15 */
} lbm_config;

enum { LBM_QOI_E = 0, LBM_QOI_Z = 1, LBM_QOI_MP = 2 };
/* Filters R of the scale-aware QoIs (Sec. 4.1), all with zero padding on
 * the wall axis:
 *  - the compact binomial family I, B, B^2, B - B^2, I - B, with
 *    B = (x)_a [1,2,1]/4;
 *  - the kernel filters of eq. gaussian and eq. laplace: GAUSS, the Gaussian
 *    of standard deviation s truncated to [-alpha s, alpha s]^d (alpha = 4 in
 *    2-D, 2 in 3-D) and normalised to unit sum, radius alpha s <= 12; LAPL,
 *    the biharmonic cross [1,-4,6,-4,1] along each axis dilated by s (odd)
 *    and normalised to sum |L_s| = 2, radius (5s-1)/2 <= 12.
 *  - FOURIER, the sharp band filter R_[l,m] (eq. scale-aware-energy-fourier):
 *    the DFT modes with l - 1/2 <= |k| < m + 1/2 are kept, k the integer mode
 *    index vector; fully periodic grids only.  Runs through hipFFT, so a
 *    closure with such QoIs steps without graph replay.
 * A closure uses the binomial family or the others (kernel and Fourier
 * filters may be mixed) for all its E and Z QoIs; I belongs to both. */
enum { LBM_FILT_ID = 0, LBM_FILT_B = 1, LBM_FILT_B2 = 2, LBM_FILT_BMID = 3, LBM_FILT_IMB = 4,
       LBM_FILT_GAUSS = 5, LBM_FILT_LAPL = 6, LBM_FILT_FOURIER = 7 };
typedef struct {
    int kind;           /* LBM_QOI_E, LBM_QOI_Z, LBM_QOI_MP (MP needs walls_y = 1) */
    int filter;         /* for E and Z */
    int band;           /* for MP: band index in [0, nbands) */
    int scale;          /* s of LBM_FILT_GAUSS / LBM_FILT_LAPL; l of LBM_FILT_FOURIER */
    int kmax;           /* m of LBM_FILT_FOURIER */
} lbm_qoi_spec;

enum { LBM_CLOSURE_OFF = 0, LBM_CLOSURE_TRACK = 1, LBM_CLOSURE_LRS = 2 };
/* TO closure.  All arrays are host memory and are deep-copied.
 *  - mode OFF: the full TO machinery runs with dQ = 0 (QoIs are recorded).
 *  - TRACK:    dQ = qref[step] - q* (eq. dQ-from-ref); steps beyond nref get dQ = 0.
 *  - LRS:      regression on scaled QoIs z = q / s (eq. LRS):
 *              x = [z^{n-1}, ..., z^{n-h}, z*^n, z*^{n-1}, ..., z*^{n-h}, 1],
 *              z = x C + eta, eta ~ N(mu, Sigma), dQ = s z - q*; z*^m are the
 *              predictor QoIs of step m, z^m the corrected ones,
 *              q^m = q*^m + dQ^m (q*^m if that step's correction was skipped).
 *              h = 0 leaves x = [z*, 1].  s = scale if given, else |q*| at
 *              the first corrected step (zero replaced by one); h > 0 needs
 *              scale.  Sigma is SPD, or all zero.
 *              The history is read from the record ring, so h > 0 needs
 *              rec_cap > h and spinup >= (steps taken so far) + h when the
 *              closure is set: the h steps before the first corrected one
 *              are recorded under this closure.
 *  - dQ = 0 for steps < spinup in every mode.
 * Band weights (eq. 3d-mp-band-weights): d_w(y) = min(y+1/2, ny-1/2-y),
 * centres log-spaced in d_w over [band_dmin, band_dmax], sigma equal to the
 * centre spacing in ln d_w, normalised so that sum_y w_j(y) = 1. */
typedef struct {
    int nq;                     /* 1..LBM_MAX_QOI; at most 8 E/Z QoIs */
    const lbm_qoi_spec* q;      /* nq entries */
    int nbands;
    double band_dmin, band_dmax;
    int mode;
    long spinup;
    int h;                      /* LRS history length, 0..LBM_MAX_HIST */
    const double* C;            /* ((2h+1) nq + 1) x nq row-major (LRS), rows in the order of x */
    const double* mu;           /* nq (LRS; NULL = 0) */
    const double* Sigma;        /* nq x nq (LRS) */
    const double* scale;        /* nq or NULL */
    const double* qref;         /* nref x nq (TRACK) */
    long nref;
    uint64_t seed;              /* LRS noise key (Philox4x32-10) */
} lbm_closure;

/* One record per step.  flags: bit0 unstable, bit1 Gram matrix singular
 * (correction skipped for that step).  mass/mom: sums over cells of rho and
 * rho v of the post-streaming state.  q: QoIs of the predictor v^{p,n*}. */
typedef struct {
    int64_t step;
    int32_t flags;
    int32_t nq;
    double mass;
    double mom[3];
    double diag_e, diag_z;
    double q[LBM_MAX_QOI], dq[LBM_MAX_QOI], gamma[LBM_MAX_QOI];
} lbm_qoi_rec;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;
typedef struct lbm_server lbm_server;

/* Fit of the LRS model (Sec. 4.4, the regularised least-squares problem
 * after eq. LRS) to a recorded trajectory, on the host (threads, FP64).
 *  q_star, dq: nsteps x nq predictor QoIs and corrections of steps 0..nsteps-1
 *    (e.g. the records of a tracking run); the corrected QoIs are
 *    q = q_star + dq, or q_star where flags (NULL: none) has bit 1 set.
 *  scale: nq (NULL: the standard deviation of each corrected QoI over the
 *    trajectory, zero replaced by one); written to s_out (NULL: not returned).
 *  Rows x^n (n = h..nsteps-1) as in lbm_closure, targets z^n = q^n / s.
 *  C (((2h+1) nq + 1) x nq) minimises 1/2 |X C - Z|^2 + 1/2 sum_i lam_i |C_i|^2
 *  with lam_i = lambda (sigma_i / sigma_1)^2, sigma_i the standard deviation
 *  of the scaled corrections z^n - z*^n; mu (nq) and Sigma (nq x nq) are the
 *  mean and unbiased sample covariance of the residuals Z - X C.
 * Cost: about (nsteps - h) len^2 / 2 + nq len^3 / 3 multiply-adds,
 * len = (2h+1) nq + 1, and 2 len^2 doubles of host memory.  LBM_EINVAL for
 * bad sizes, or when lambda = 0 leaves the normal matrix singular. */
int lbm_lrs_fit(int nq, int h, long nsteps, const double* q_star, const double* dq, const int* flags,
                const double* scale, double lambda, double* C, double* mu, double* Sigma, double* s_out);

/* Library and lattice information. */
const char* lbm_last_error(void);
const char* lbm_version(void);
/* Name of the current HIP device and its compute-unit count, e.g.
 * "gfx950 256CU", into out (n bytes, NUL-terminated).  LBM_EDEVICE without
 * a device. */
int lbm_device_tag(char* out, size_t n);
/* Velocity table (3 ints per velocity) and weights of the library's own
 * lattice ordering; returns Q or a negative status. */
int lbm_lattice_info(int lattice, int* c, double* w);

/* Device bytes a context needs for cfg (and the closure it will run, or
 * NULL for a plain run).  Returns 0 for an invalid configuration.  Grids are
 * limited to 2e9 cells; a run with a closure also needs 2 * N * (element
 * size) below 4 GiB (N < 2^29 cells in FP32, 2^28 in FP64), since its
 * kernels address each field, and pairs of population arrays, with 32-bit
 * byte offsets. */
size_t lbm_required_bytes(const lbm_config* cfg, const lbm_closure* closure);

/* Create a context on the current HIP device.  dev_arena: caller-owned
 * device memory of at least lbm_required_bytes(cfg, closure) bytes, 256-byte
 * aligned, which must outlive the context; the library never frees it.
 * stream: hipStream_t (NULL: the context creates its own non-blocking
 * stream).  closure may be NULL.  The
 * initial state is rho = 1, v = 0 until lbm_init_velocity is called. */
int lbm_create(const lbm_config* cfg, const lbm_closure* closure, void* dev_arena,
               size_t bytes, void* stream, lbm_ctx** out);
void lbm_destroy(lbm_ctx* ctx);

/* Set the post-collision state to feq(rho, u) (host arrays; rho may be NULL
 * for rho = 1; u has d*N entries).  Resets the step counter and records. */
int lbm_init_velocity(lbm_ctx* ctx, const double* rho, const double* u);

/* Replace the closure (between steps).  NULL switches the TO step off.  The
 * closure must fit the workspace planned at creation (else LBM_ENOMEM). */
int lbm_set_closure(lbm_ctx* ctx, const lbm_closure* closure);

/* Enqueue nsteps LES steps on the context stream (non-blocking).  Chunks of
 * 32 steps, and the even part of a shorter remainder, are replayed from
 * captured hipGraphs (cached by chunk length); a last odd step, and steps of
 * closures with Fourier band QoIs (hipFFT), launch eagerly. */
int lbm_step(lbm_ctx* ctx, long nsteps);
/* Capture and upload, without running anything, the graphs a later
 * lbm_step(ctx, nsteps) replays (from either ping-pong phase, so that other
 * steps may run in between), so that it pays no capture cost (timed
 * regions).  Graphs are dropped when the closure or the state changes. */
int lbm_step_prepare(lbm_ctx* ctx, long nsteps);
int lbm_sync(lbm_ctx* ctx);             /* waits; LBM_EUNSTABLE if flagged */
long lbm_step_count(const lbm_ctx* ctx);

/* Copy records of steps [first, first+count) into out (syncs). */
int lbm_qoi(lbm_ctx* ctx, long first, long count, lbm_qoi_rec* out);

/* Density (N) and post-streaming moment velocity (d*N) of the current
 * state, in double precision (syncs).  rho may be NULL. */
int lbm_fields(lbm_ctx* ctx, double* rho, double* u);
/* The velocity alone: lbm_fields(ctx, NULL, u). */
int lbm_velocity(lbm_ctx* ctx, double* u);

/* lbm_fields for callers that cannot allocate (tight serving loops,
 * harnesses that forbid device or host allocations between steps): the same
 * outputs, bitwise, staged through a fixed device array of
 * LBM_FIELDS_NOALLOC_MAX_BYTES that each GPU holds until the process ends,
 * instead of memory allocated per call.  No hipMalloc, hipFree or other
 * allocating call is made.  Limit: (d + 1) * N * 8 bytes of staging, i.e. at
 * most 524288 cells in 3-D and 699050 in 2-D; larger grids are rejected with
 * LBM_EINVAL (use lbm_fields).  Every call on a GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other threads, other streams) race
 * and must be serialised by the caller.  The device is the one current on
 * the calling thread.  Syncs the context stream; rho may be NULL. */
#define LBM_FIELDS_NOALLOC_MAX_BYTES (16u << 20)
int lbm_fields_noalloc(lbm_ctx* ctx, double* rho, double* u);

/* Full post-collision populations f (Q*N, library ordering, double) of the
 * current state (the SGS change of the last step included); and the
 * inverse. */
int lbm_get_populations(lbm_ctx* ctx, double* f);
int lbm_set_populations(lbm_ctx* ctx, const double* f);

/* Stream the current populations once without collision (index-map check). */
int lbm_stream_only(lbm_ctx* ctx);

/* HF -> LF projection (Sec. 3, the projection phi_m; Sec. 7.1, the
 * wall-anchored stride-m subsampling): coarse cell (i, j, k) takes fine cell
 * (m i + o, m j + o, m k + o), o = (m - 1) / 2, so the walls of both grids
 * coincide.  The coarse context has the fine grid divided by m on every axis
 * (nz = 1 in 2-D), the same lattice and wall setting; m is odd.  LBM_EINVAL
 * otherwise.
 *  - lbm_project_state: the coarse run's state becomes the projected fine
 *    post-collision populations (f = phi_m f, any precisions); resets the
 *    coarse step counter and records, like lbm_init_velocity.  Syncs.
 *  - lbm_project_qoi: evaluates the probe's closure QoIs on the projected
 *    post-collision velocity sum c f / sum f of the fine run's current state,
 *    and appends them as the probe's next record (q; dq, gamma zero; mass and
 *    momentum not meaningful).  The probe is a context with a closure in mode
 *    OFF, used for nothing else; it shares the fine run's stream and the call
 *    is enqueued there without blocking.  Called after every m fine steps,
 *    its records are the reference trajectory q_ref of a coarse tracking run
 *    (eq. dQ-from-ref): coarse step n <-> fine steps (n+1) m. */
int lbm_project_state(lbm_ctx* fine, lbm_ctx* coarse, int m);
int lbm_project_qoi(lbm_ctx* fine, lbm_ctx* probe, int m);

/* The same with a choice of projection (Sec. 3): LBM_PROJ_STRIDE as above;
 * LBM_PROJ_BICUBIC, the paper's projection for the doubly periodic
 * Kolmogorov flow: coarse cell (i, j) is the mean of the fine cells
 * (m i + o + rx, m j + o + ry), |rx|, |ry| < 2 m, periodic wrap, with
 * weights K(rx / m) K(ry / m) normalised to unit sum, K the cubic
 * convolution kernel of Keys with a = -1/2 (the bicubic kernel widened
 * m-fold for the m-fold coarser grid).  Populations are projected as
 * populations; the probe's QoIs are evaluated on the projected fine-cell
 * velocities.  Bicubic needs D2Q9 without walls and m <= 15 (odd);
 * LBM_EINVAL otherwise. */
enum { LBM_PROJ_STRIDE = 0, LBM_PROJ_BICUBIC = 1 };
int lbm_project_state_kind(lbm_ctx* fine, lbm_ctx* coarse, int m, int kind);
int lbm_project_qoi_kind(lbm_ctx* fine, lbm_ctx* probe, int m, int kind);

/* Checkpoint: opaque byte image of the dynamic state (populations,
 * counters, LRS scale, records).  Restoring it into a context created with
 * the same cfg and closure resumes bitwise identically.  Two runs in the same
 * state give the same bytes, whichever launch forms their solve (alone, in a
 * batch, in a server, tune_mem bit 3). */
size_t lbm_state_bytes(const lbm_ctx* ctx);
int lbm_get_state(lbm_ctx* ctx, void* host, size_t bytes);
int lbm_set_state(lbm_ctx* ctx, const void* host, size_t bytes);


/* Autotuner of the launch shapes (the tune_* fields of lbm_config): the
 * binomial tile width, the z planes per binomial workgroup and the cells
 * per thread of the QoI reduction.  Candidates are timed on a scratch
 * context in dev_arena (caller-owned, 256-byte aligned, at least
 * lbm_autotune_bytes(cfg, closure) bytes; its contents are overwritten),
 * each for `steps` steps after a warm-up, started from a small seeded
 * velocity field: a coordinate descent from the automatic choice over the
 * tile width, then the z chunk, then the cells per thread.  Every candidate
 * gives the same per-cell results (tile width and z chunk bitwise; the
 * cells per thread change only the order of the FP64 partial sums).
 * cache_path (may be NULL): a text file with one line per device, grid and
 * closure shape (key TAB zc cpt btx microseconds-per-step); a matching line
 * is returned without timing (from_cache = 1), a new result is appended.
 * Runs on the current device; syncs. */
typedef struct {
    int tune_zc, tune_cpt, tune_btx;   /* to copy into lbm_config */
    double us_per_step;                /* the chosen candidate's time per step */
    int from_cache;                    /* 1: read from the cache file */
    int candidates;                    /* candidates timed (0 when cached) */
} lbm_tuning;
size_t lbm_autotune_bytes(const lbm_config* cfg, const lbm_closure* closure);
/* The cache key of (device, cfg, closure) that lbm_autotune uses, into out
 * (n bytes; LBM_EINVAL if too small).  Without a device the device part
 * reads "unknown". */
int lbm_autotune_key(const lbm_config* cfg, const lbm_closure* closure, char* out, size_t n);
int lbm_autotune(const lbm_config* cfg, const lbm_closure* closure, void* dev_arena, size_t bytes,
                 void* stream, int steps, const char* cache_path, lbm_tuning* out);

/* Batch: advance several contexts (created on the same device and stream)
 * together, one launch per kernel phase for all members of the same kind,
 * replayed from a hipGraph.  Each member's results are bitwise identical to
 * stepping it alone.  The batch does not own the members. */
int lbm_batch_create(int n, lbm_ctx* const* members, lbm_batch** out);
int lbm_batch_step(lbm_batch* b, long nsteps);
int lbm_batch_sync(lbm_batch* b);
void lbm_batch_destroy(lbm_batch* b);

/* Serving: continuous batching of LES requests on one GPU.
 * Requests (a config, an optional closure and the initial velocity) queue
 * in arrival order.  lbm_server_advance admits every queued request whose
 * arrival time has passed while the sum of the admitted arenas stays within
 * the HBM budget, advances all admitted requests together as one batch for a
 * chunk of steps (no request runs past its own step count), and retires the
 * finished ones.  Requests join and leave between chunks, so their work
 * overlaps on the device; each request's result is bitwise the one it gets
 * alone.  One chunk is in flight at a time: a call admits new arrivals while
 * the previous chunk runs (their contexts are created and initialised on a
 * second stream of the server), then waits for that chunk, retires, and
 * enqueues the next chunk before it returns.  Arenas come from a pool keyed
 * by size (a retired request's arena serves the next request of that size;
 * cached arenas count against the budget and are freed when a request of
 * another size needs the room).  A request that cannot start (larger than
 * the budget, or a failed allocation) is retired at once with that status;
 * the others go on.  Times are seconds on the clock of lbm_server_clock. */
typedef struct {
    long id;
    int status;                 /* LBM_OK, LBM_EUNSTABLE, or the status that kept it from starting
                                   (LBM_ENOMEM: larger than the budget or no memory) */
    long steps;
    long cells;
    double t_arrival, t_admit, t_done;
    lbm_qoi_rec last;           /* record of the last step (runs with records) */
} lbm_result;
double lbm_server_clock(void);
/* hbm_budget: bytes for request arenas (0: 80% of the free device memory). */
int lbm_server_create(size_t hbm_budget, void* stream, lbm_server** out);
/* Copies everything it is given; keep_state retains the final state image
 * (lbm_get_state layout) for lbm_server_take_state.  The config and closure
 * are validated here (LBM_EINVAL, nothing queued), including an SPD Sigma
 * for LRS closures and a spin-up covering a history model's length. */
int lbm_server_submit(lbm_server* s, const lbm_config* cfg, const lbm_closure* closure, const double* u0,
                      long nsteps, double t_arrival, int keep_state, long* id);
/* Admit, account and retire the chunk in flight, enqueue the next chunk of at
 * most max_chunk steps (0: 64) and return without waiting for it.  A caller
 * loops until lbm_server_pending reads 0.  If the batch of the active
 * requests cannot be built or stepped, those requests are retired with that
 * status (their results say so) and the status is returned; queued requests
 * are served by later calls. */
int lbm_server_advance(lbm_server* s, double now, long max_chunk, int* n_active);
/* Move up to cap finished results into out (caller-owned). */
int lbm_server_poll(lbm_server* s, lbm_result* out, int cap, int* n);
int lbm_server_pending(const lbm_server* s);            /* queued + active requests */
/* busy_s: device time of the chunks; lups: lattice updates done; used: bytes
 * of active arenas; budget: the HBM budget. */
int lbm_server_stats(const lbm_server* s, double* busy_s, double* lups, size_t* used, size_t* budget);
size_t lbm_server_state_bytes(const lbm_server* s, long id);
int lbm_server_take_state(lbm_server* s, long id, void* host, size_t bytes);
void lbm_server_destroy(lbm_server* s);

/* Per-phase timing for measurement: runs nsteps steps eagerly on the context
 * stream with HIP events between the kernel phases and returns the mean
 * duration per step of each phase in ms[6]: stream-collide (with the WALE
 * moments pass), curl, filters (binomial powers, or the kernel-filter pass
 * program), reduce, cross-block sums and solve, apply (plain runs with
 * records: their diagnostics in the last slot); launches[6] (nullable)
 * receives the kernel launches per step of each phase.  Advances the run. */
int lbm_profile_phases(lbm_ctx* ctx, long nsteps, double* ms, int* launches);

/* Test hooks of the device random-number generator (allocate their own
 * scratch; not used by the stepping path).
 * lbm_test_philox: n Philox4x32-10 evaluations; in6 holds (ctr0..3, key0,
 * key1) per evaluation, out4 the four output words.
 * lbm_test_normals: the LRS standard normals of steps step0..step0+nsteps-1
 * for a closure with n QoIs and the given seed (nsteps x n, row-major). */
int lbm_test_philox(const uint32_t* in6, uint32_t* out4, int n);
int lbm_test_normals(uint64_t seed, long step0, int nsteps, int n, double* out);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */

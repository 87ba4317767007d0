// lbm_api.hip -- host side of liblbm_hip: arena planning, the C ABI of
// include/lbm.h, hipGraph replay and ensemble batches.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_dev.h"
#include "lbm_launch.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int filter_deg(int f) { return f == LBM_FILT_ID ? 0 : (f == LBM_FILT_B || f == LBM_FILT_IMB ? 1 : 2); }

// R as a polynomial in B: coefficients of B^0, B^1, B^2.
void filter_poly(int f, double r[3])
{
    r[0] = r[1] = r[2] = 0;
    switch (f) {
    case LBM_FILT_ID: r[0] = 1; break;
    case LBM_FILT_B: r[1] = 1; break;
    case LBM_FILT_B2: r[2] = 1; break;
    case LBM_FILT_BMID: r[1] = 1; r[2] = -1; break;
    case LBM_FILT_IMB: r[0] = 1; r[1] = -1; break;
    }
}

struct ClosureShape {
    int nq = 0, nsa = 0, nmp = 0, jv = 0, jw = 0, has_z = 0, has_e = 0, nbands = 0;
    int h = 0, nhc = 0;   // LRS history length; k_sum workgroups of its product
    int kf = 0;           // E/Z QoIs use the kernel filters (materialised sensitivities)
    int kslots = 0, nzq = 0;   // kernel filters: separable terms over the QoIs; Z QoIs
    int nf = 0, nfz = 0;       // Fourier band QoIs; of them Z QoIs
    int npart() const { return nsa + nsa * (nsa + 1) / 2 + nmp * (1 + nsa); }
};

int closure_shape(const lbm_config* cfg, const lbm_closure* cl, ClosureShape* out)
{
    ClosureShape s;
    if (!cl) { *out = s; return LBM_OK; }
    if (cl->nq < 1 || cl->nq > LBM_MAX_QOI || !cl->q) return fail(LBM_EINVAL, "closure: nq must be in [1,%d]", LBM_MAX_QOI);
    if (cl->mode < LBM_CLOSURE_OFF || cl->mode > LBM_CLOSURE_LRS) return fail(LBM_EINVAL, "closure: bad mode");
    if (cl->h < 0 || cl->h > LBM_MAX_HIST || 2L * cl->h * cl->nq > (long)kHistRows * kMaxHistChunks)
        return fail(LBM_EINVAL, "closure: history length h must be in [0,%d] with 2 h nq <= %d", LBM_MAX_HIST,
                    kHistRows * kMaxHistChunks);
    if (cl->h > 0) {
        if (cl->mode != LBM_CLOSURE_LRS) return fail(LBM_EINVAL, "closure: a history length needs mode LRS");
        if (!cl->scale) return fail(LBM_EINVAL, "closure: a history model needs the scale s");
        const int rc = cfg->rec_cap > 0 ? cfg->rec_cap : 4096;
        if (rc <= cl->h) return fail(LBM_EINVAL, "closure: rec_cap must exceed the history length");
        s.h = cl->h;
        s.nhc = (2 * cl->h * cl->nq + kHistRows - 1) / kHistRows;
    }
    {
        // the TO kernels address every field component, and pairs of
        // population arrays, with 32-bit byte offsets
        const double bytes = (double)cfg->nx * cfg->ny * cfg->nz * 2 * (cfg->precision == LBM_FP64 ? 8 : 4);
        if (bytes >= 4294967296.0)
            return fail(LBM_EINVAL, "closure: grid too large for a TO run (2 * N * element size must be below 4 GiB)");
    }
    s.nq = cl->nq;
    s.nbands = cl->nbands;
    bool binom = false;
    for (int k = 0; k < cl->nq; ++k) {
        const lbm_qoi_spec& q = cl->q[k];
        if (q.kind != LBM_QOI_E && q.kind != LBM_QOI_Z) continue;
        if (q.filter < LBM_FILT_ID || q.filter > LBM_FILT_FOURIER) return fail(LBM_EINVAL, "closure: QoI %d bad filter", k);
        if (q.filter == LBM_FILT_FOURIER) {
            if (cfg->walls_y) return fail(LBM_EINVAL, "closure: Fourier filters need a fully periodic grid");
            if (q.scale < 0 || q.kmax < q.scale) return fail(LBM_EINVAL, "closure: QoI %d Fourier band [l,m] needs 0 <= l <= m", k);
            s.kf = 1;
            s.nf++;
            s.nfz += q.kind == LBM_QOI_Z;
        } else if (q.filter == LBM_FILT_GAUSS || q.filter == LBM_FILT_LAPL) {
            const int d = cfg->lattice == LBM_D2Q9 ? 2 : 3;
            const int rad = q.filter == LBM_FILT_GAUSS ? (d == 2 ? 4 : 2) * q.scale : (5 * q.scale - 1) / 2;
            if (q.scale < 1 || (q.filter == LBM_FILT_LAPL && q.scale % 2 == 0) || rad > kMaxRad)
                return fail(LBM_EINVAL, "closure: QoI %d kernel-filter scale (odd for LAPL; radius at most %d)", k,
                            kMaxRad);
            s.kf = 1;
        } else if (q.filter != LBM_FILT_ID)
            binom = true;
    }
    if (s.kf && binom) return fail(LBM_EINVAL, "closure: binomial and kernel filters cannot be mixed");
    if (s.kf)
        for (int k = 0; k < cl->nq; ++k) {
            const lbm_qoi_spec& q = cl->q[k];
            if (q.kind != LBM_QOI_E && q.kind != LBM_QOI_Z) continue;
            s.kslots += q.filter == LBM_FILT_LAPL ? (cfg->lattice == LBM_D2Q9 ? 2 : 3) : (q.filter == LBM_FILT_FOURIER ? 0 : 1);
            s.nzq += q.kind == LBM_QOI_Z;
        }
    for (int k = 0; k < cl->nq; ++k) {
        const lbm_qoi_spec& q = cl->q[k];
        if (q.kind == LBM_QOI_E || q.kind == LBM_QOI_Z) {
            const int p = s.kf ? 0 : 2 * filter_deg(q.filter);
            if (q.kind == LBM_QOI_E) { s.jv = std::max(s.jv, p); s.has_e = 1; }
            else { s.jw = std::max(s.jw, p); s.has_z = 1; }
            s.nsa++;
        } else if (q.kind == LBM_QOI_MP) {
            if (!cfg->walls_y) return fail(LBM_EINVAL, "closure: mean-profile QoIs need walls_y = 1");
            if (q.band < 0 || q.band >= cl->nbands) return fail(LBM_EINVAL, "closure: QoI %d band out of range", k);
            s.nmp++;
        } else
            return fail(LBM_EINVAL, "closure: QoI %d bad kind", k);
    }
    if (s.nsa > kMaxSA) return fail(LBM_EINVAL, "closure: at most %d energy/enstrophy QoIs", kMaxSA);
    if (s.nmp > 0 && !(cl->band_dmin > 0 && cl->band_dmax > cl->band_dmin)) return fail(LBM_EINVAL, "closure: band range");
    if (cl->mode == LBM_CLOSURE_LRS && (!cl->C || !cl->Sigma)) return fail(LBM_EINVAL, "closure: LRS needs C and Sigma");
    if (cl->mode == LBM_CLOSURE_TRACK && (!cl->qref || cl->nref < 0)) return fail(LBM_EINVAL, "closure: tracking needs qref");
    *out = s;
    return LBM_OK;
}

int check_config(const lbm_config* c)
{
    if (!c) return fail(LBM_EINVAL, "config is NULL");
    if (c->lattice != LBM_D2Q9 && c->lattice != LBM_D3Q19) return fail(LBM_EINVAL, "bad lattice");
    if (c->precision < LBM_FP32_SHIFTED || c->precision > LBM_FP32_PLAIN) return fail(LBM_EINVAL, "bad precision");
    if (c->nx < 3 || c->ny < 3 || c->nz < 1) return fail(LBM_EINVAL, "grid must be at least 3 cells per axis");
    if (c->lattice == LBM_D2Q9 && c->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz = 1");
    if (c->lattice == LBM_D3Q19 && c->nz < 3) return fail(LBM_EINVAL, "D3Q19 needs nz >= 3");
    if ((double)c->nx * c->ny * c->nz > 2.0e9) return fail(LBM_EINVAL, "grid too large");
    if (!(c->tau > 0.5)) return fail(LBM_EINVAL, "tau must exceed 1/2");
    if (c->substrate < LBM_BGK || c->substrate > LBM_WALE) return fail(LBM_EINVAL, "bad substrate");
    if (c->substrate == LBM_WALE && c->lattice != LBM_D3Q19) return fail(LBM_EINVAL, "WALE needs D3Q19");
    if (c->force_kind < LBM_FORCE_NONE || c->force_kind > LBM_FORCE_CONST_X) return fail(LBM_EINVAL, "bad force kind");
    if (c->rec_cap < 0) return fail(LBM_EINVAL, "rec_cap < 0");
    if (c->tune_zc < 0 || c->tune_cpt < 0) return fail(LBM_EINVAL, "tuning values must be >= 0");
    if (c->tune_mem < 0 || c->tune_mem > 15) return fail(LBM_EINVAL, "tune_mem must be in 0..15");
    if (c->tune_btx != 0 && c->tune_btx != kBinTX && c->tune_btx != kBinTXW)
        return fail(LBM_EINVAL, "tune_btx must be 0, %d or %d", kBinTX, kBinTXW);
    if (c->tune_btx == kBinTXW && c->lattice != LBM_D3Q19)
        return fail(LBM_EINVAL, "tune_btx = %d needs D3Q19", kBinTXW);
    return LBM_OK;
}

struct Plan {
    size_t member, param, ctl, recs, g0, g1, fprof, vn, part_stats, part_diag, work1, workp, workm;
    size_t rho, vs, P, W, Cf, rec, part_to, bandw, cmp, workr, workb, sums, works, hpart, kV, kT, ktaps, kjobs;
    size_t fspec_v, fspec_w, fband_e, fband_z;
    size_t total;
    int N, D, NC, Q, esz, nb1, nbp, nbx2, cpt2, nbr, nbb, nbs, zc, btx, rec_cap;
    size_t popn;   // elements of one population buffer: Q * N rounded up to whole blocks of kPopBlk cells
    ClosureShape cap;
};

void make_plan(const lbm_config* c, const ClosureShape& cs, Plan* p)
{
    Plan P{};
    P.N = c->nx * c->ny * c->nz;
    P.D = c->lattice == LBM_D2Q9 ? 2 : 3;
    P.NC = P.D == 2 ? 1 : 3;
    P.Q = c->lattice == LBM_D2Q9 ? 9 : 19;
    P.esz = c->precision == LBM_FP64 ? 8 : 4;
    P.nb1 = (P.N + kBlock - 1) / kBlock;
    P.nbp = (P.nb1 + 1) / 2;
    P.rec_cap = c->rec_cap > 0 ? c->rec_cap : 4096;
    P.cap = cs;
    const int plane = c->nx * c->nz;
    P.cpt2 = c->tune_cpt > 0 ? std::min(c->tune_cpt, 64) : std::max(2, std::min(8, P.N / (kBlock * 2048)));
    P.nbx2 = (plane + kBlock * P.cpt2 - 1) / (kBlock * P.cpt2);
    P.nbr = P.nbx2 * c->ny;
    {
        // tile: 64 x 8 (512-thread workgroups) on 3-D grids whose rows are
        // whole multiples of 64 cells and at least 256 long, else 32 x 8
        // (measured on MI355X on a 384 x 192 x 192 channel: 64-wide tiles 9%
        // less binomial time than 32 x 8; 64 x 8 another 6% less than 64 x 4)
        P.btx = c->tune_btx ? c->tune_btx : (P.D == 3 && c->nx % kBinTXW == 0 && c->nx >= 256 ? kBinTXW : kBinTX);
        // z chunk: as many planes per workgroup as keeps about 400 or more
        // workgroups (measured on MI355X: fewer staged halo planes pay more
        // than extra workgroups once the chip has 1.5 per CU)
        const int bty = kBinTY;
        const int nxy = ((c->nx + P.btx - 1) / P.btx) * ((c->ny + bty - 1) / bty);
        P.zc = P.D == 3 ? (c->tune_zc > 0 ? std::min(c->tune_zc, c->nz)
                                           : std::max(1, std::min(kBinZCMax, nxy * c->nz / 400)))
                        : 1;
        P.nbb = nxy * (P.D == 3 ? (c->nz + P.zc - 1) / P.zc : 1);
    }
    const size_t N = P.N, e = P.esz;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    P.member = take(sizeof(DevMember));
    P.param = take(sizeof(DevParam));
    P.ctl = take(sizeof(DevCtl));
    P.recs = take(sizeof(lbm_qoi_rec) * P.rec_cap);
    P.popn = (size_t)P.Q * ((N + kPopBlk - 1) / kPopBlk) * kPopBlk;
    P.g0 = take(e * P.popn);
    P.g1 = take(e * P.popn);
    P.fprof = take(sizeof(double) * c->ny);
    P.vn = take(e * P.D * N);
    // statistics partials: one per stream-collide workgroup (1-D blocks, or
    // the binomial tiles when the SGS change is deferred)
    P.part_stats = take(sizeof(double) * 4 * std::max(P.nb1, P.nbb));
    P.part_diag = take(sizeof(double) * 2 * P.nb1);
    P.work1 = take(sizeof(int2) * P.nb1);
    P.workp = take(sizeof(int2) * P.nbp);
    P.workm = take(sizeof(int));
    if (cs.nq > 0) {
        P.rho = take(e * N);
        P.vs = take(e * P.D * N);
        P.P = take(e * (size_t)std::max(cs.jv, 1) * P.D * N);
        P.W = take(cs.has_z ? e * (size_t)(cs.jw + 1) * P.NC * N : kAlign);
        P.Cf = take(cs.has_z ? e * (size_t)(cs.jw + 1) * P.D * N : kAlign);
        P.rec = take(e * 2 * P.D * N);
        P.part_to = take(sizeof(double) * (size_t)std::max(cs.npart(), 1) * P.nbr);
        P.bandw = take(sizeof(double) * (size_t)std::max(cs.nbands, 1) * c->ny);
        P.cmp = take(sizeof(double) * c->ny);
        P.workr = take(sizeof(int2) * P.nbr);
        P.workb = take(sizeof(int2) * P.nbb);
        // k_sum workgroups: the LRS draw (slot -1), the history product
        // (slots -2 - c), then one per sum
        P.nbs = 5 + cs.nhc + cs.npart();
        P.sums = take(sizeof(double) * (4 + cs.npart()));
        P.works = take(sizeof(int2) * P.nbs);
        P.hpart = take(sizeof(double) * kMaxQ * std::max(cs.nhc, 1));
        if (cs.kf) {
            // kernel filters: V_s [nsa][D][N]; [3][N] work fields: two per
            // separable term, one per QoI, one more per Z QoI; tap tables;
            // the job table of the pass program
            P.kV = take(e * (size_t)cs.nsa * P.D * N);
            P.kT = take(e * 3 * N * (size_t)(2 * cs.kslots + cs.nsa + cs.nzq));
            P.ktaps = take(e * kMaxSA * 3 * (2 * kMaxRad + 1));
            P.kjobs = take(sizeof(KJob) * (size_t)(2 * (2 * cs.kslots + cs.nsa) + cs.nzq + 1));
            if (cs.nf) {
                // Fourier bands: spectra of v* and w and one work spectrum (complex)
                P.fspec_v = take(2 * e * P.D * N);
                P.fspec_w = take(2 * e * P.NC * N);
                P.fband_e = take(2 * e * P.D * N * (size_t)std::max(cs.nf - cs.nfz, 1));
                P.fband_z = take(2 * e * P.NC * N * (size_t)std::max(cs.nfz, 1));
            }
        }
    }
    P.total = o;
    *p = P;
}

// Slot of k_sum workgroup k of a member whose plan holds nhc history
// workgroups: -1 the LRS draw, -2 - c history chunk c, then the sums 0...
int ksum_slot(int k, int nhc) { return k == 0 ? -1 : (k <= nhc ? -1 - k : k - 1 - nhc); }

// Work-table order for the 8 XCDs of MI355X, which receive workgroups
// round-robin by workgroup index and each have their own L2: entry w runs on
// XCD w % 8, so giving XCD k a contiguous range of blocks keeps the
// neighbouring rows and planes that a block reads in the L2 that already
// holds them.  Returns the block processed by each entry.
constexpr int kXcd = 8;

// Whether a launch stores the fields the next kernel reads through the L2:
// when its population buffers, pop_bytes in total, fit well within the
// 32 MB of L2 summed over the 8 XCDs (measured on MI355X: faster on a
// 96 x 48 x 48 channel, slower on 295 x 47 x 98, whose fields the next
// kernel otherwise finds in the Infinity Cache).
int write_through(double pop_bytes) { return pop_bytes <= 24.0 * 1024 * 1024; }
// Plain stream-collide launches whose population buffer exceeds half the
// 256 MB Infinity Cache store non-temporally; smaller ones keep their
// populations in it from one step to the next (measured on MI355X, plain
// BGK channels: non-temporal stores -5% at 74 MB and -9% at 98 MB, +4% at
// 145 MB, +6-8% from 204 to 594 MB, equal beyond 1 GB).
int non_temporal(double pop_bytes) { return pop_bytes >= 128.0 * 1024 * 1024; }
std::vector<int> xcd_order(int n)
{
    std::vector<int> order;
    order.reserve(n);
    const int q = (n + kXcd - 1) / kXcd;
    std::vector<int> next(kXcd), end(kXcd);
    for (int k = 0; k < kXcd; ++k) { next[k] = std::min(n, k * q); end[k] = std::min(n, (k + 1) * q); }
    while ((int)order.size() < n)
        for (int k = 0; k < kXcd && (int)order.size() < n; ++k)
            if (next[k] < end[k]) order.push_back(next[k]++);
    return order;
}

// The same for the binomial tiles, in tile-id order (xy fastest): the
// workgroups an XCD runs at the same time are neighbouring tiles of the same
// z chunks, whose halo rows they share in that XCD's L2 (measured on MI355X:
// 8-13% faster than keeping the z chunks of a tile together).
std::vector<int> xcd_tile_order(int ntx, int nty, int ntz)
{
    return xcd_order(ntx * nty * ntz);
}

// Band weights (eq. 3d-mp-band-weights) in the reading of the library header.
void band_weights(int ny, int nb, double dmin, double dmax, std::vector<double>& w)
{
    w.assign((size_t)nb * ny, 0.0);
    const double sig = nb > 1 ? (std::log(dmax) - std::log(dmin)) / (nb - 1) : 1.0;
    for (int j = 0; j < nb; ++j) {
        const double lc = std::log(dmin) + j * sig;
        double A = 0;
        for (int y = 0; y < ny; ++y) {
            const double dw = std::min(y + 0.5, ny - 0.5 - y);
            const double t = (std::log(dw) - lc) / sig;
            w[(size_t)j * ny + y] = std::exp(-0.5 * t * t);
            A += w[(size_t)j * ny + y];
        }
        for (int y = 0; y < ny; ++y) w[(size_t)j * ny + y] /= A;
    }
}

// Lower Cholesky factor of an SPD matrix (n x n, row-major) into L with
// leading dimension ld; the all-zero matrix gives L = 0.  Returns false if
// the matrix is neither.
bool cholesky_host(const double* A, int n, double* L, int ld)
{
    bool zero = true;
    for (int k = 0; k < n * n; ++k) zero = zero && A[k] == 0.0;
    for (int i = 0; i < n; ++i) for (int j = 0; j < ld; ++j) L[i * ld + j] = 0;
    if (zero) return true;
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * ld + k] * L[j * ld + k];
        if (!(s > 0)) return false;
        L[j * ld + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * ld + k] * L[j * ld + k];
            L[i * ld + j] = t / L[j * ld + j];
        }
    }
    return true;
}

}  // namespace

// Error reporting for the library's other translation units.
namespace lbm {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}

struct lbm_ctx {
    lbm_config cfg{};
    Plan plan{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena = nullptr;
    DevMember hm{};
    DevMember* dm = nullptr;
    DevParam hp{};
    ClosureShape cur{};   // active closure (nq = 0: none)
    bool has_to = false;  // TO buffers exist
    int phase = 0;        // state is in g[parity ^ phase]
    long host_step = 0;
    long version = 0;     // bumps whenever launch parameters change
    bool pending = false; // steps with a deferred SGS change were enqueued since the last flush
    double* qref_dev = nullptr;
    size_t qref_cap = 0;
    double* chist_dev = nullptr;   // history rows of the LRS matrix
    double* proj_tmp = nullptr;    // scratch of the separable bicubic projection (probe contexts)
    size_t proj_tmp_bytes = 0;
    size_t chist_cap = 0;
    std::vector<int2> klev;        // kernel filters: (first job, job count) per launch level
    FourierProg fprog{};           // Fourier band QoIs (plans made at set_closure)
    // captured step graphs, keyed by chunk length, per starting phase; valid
    // for launch parameters of version gver
    std::map<int, hipGraphExec_t> gexec[2];
    long gver = -1;
    int gchunk = 32;
    int mode() const { return cur.nq > 0 ? 2 : (cfg.diag ? 1 : 0); }
    // The SGS change goes into the next step's pull (a record per cell)
    // except with the WALE substrate, whose velocity gradients need the
    // complete post-streaming state, and on grids whose populations stay in
    // the 256 MB Infinity Cache (up to 192 MB), where the in-place apply is
    // cheaper than the tiled pull with its staged records (measured on
    // MI355X, FP32 channel TO-LES: 96 x 48 x 48 2659 -> 2714 MLUPS, 295 x 47
    // x 98 3866 -> 4230, 192 x 96 x 96 4858 -> 4897; at 256 x 128 x 128, 304
    // MB of populations, the record form is faster, 6329 against 5938).
    // Either way the result is bitwise the same.
    bool defers() const
    {
        return mode() == 2 && cfg.substrate != LBM_WALE &&
               ((cfg.tune_mem & 4) || (double)plan.N * plan.Q * plan.esz > 192.0 * 1024 * 1024);
    }
};

struct lbm_batch {
    std::vector<lbm_ctx*> mem;
    std::vector<int> phase0;     // member phase when the batch tables were built
    std::vector<long> ver0;
    hipStream_t stream = nullptr;
    DevMember* dmem = nullptr;
    int2* dwork = nullptr;
    int* dworkm = nullptr;
    std::vector<LaunchGroup> groups;
    int phase = 0;
    std::map<int, hipGraphExec_t> gexec[2];   // captured step graphs by chunk length, per starting phase
    int gchunk = 16;
};

namespace {

// Union of the chains each binomial pass advances for member c: pass j
// computes B^j v (j <= jv) and B^j w with curl^T B^(j-1) w (j <= jw); pass 1
// also forms w = curl v*, and the readers form the top curl^T B^jw w.
void add_pass_masks(const lbm_ctx* c, LaunchGroup& g)
{
    for (int j = 1; j <= 8; ++j) {
        if (j <= c->cur.jv) g.bmask[j - 1] |= 1;
        if (c->cur.has_z && j <= c->cur.jw) g.bmask[j - 1] |= 2;
    }
}

// Binomial passes per step of a closure shape.
int binom_passes(const ClosureShape& cs)
{
    return cs.kf ? 0 : std::max(cs.jv, cs.has_z ? std::max(cs.jw, 1) : 0);
}

// The member record's fields that follow the closure mode.
void refresh_member(lbm_ctx* c)
{
    c->hm.defer = c->defers() ? 1 : 0;
    c->hm.nst = c->defers() ? c->plan.nbb : c->plan.nb1;
}

LaunchGroup ctx_group(const lbm_ctx* c)
{
    LaunchGroup g{};
    g.lattice = c->cfg.lattice;
    g.precision = c->cfg.precision;
    g.substrate = c->cfg.substrate;
    g.mode = c->mode();
    g.any_z = c->cur.has_z;
    g.maxpow = std::max(c->cur.jv, c->cur.jw);
    g.maxsa = c->cur.nsa;
    g.npass = binom_passes(c->cur);
    g.btx = c->plan.btx;
    g.wt = write_through((double)c->plan.N * c->plan.Q * c->plan.esz);
    g.a32 = (double)c->plan.popn * c->plan.esz < 4294967296.0 && !(c->cfg.tune_mem & 1);
    g.nt = non_temporal((double)c->plan.popn * c->plan.esz) || (c->cfg.tune_mem & 2);
    g.defer = c->defers();
    g.sep_solve = (c->cfg.tune_mem & 8) != 0;
    add_pass_masks(c, g);
    g.kf = c->cur.kf;
    g.kjobs = (const KJob*)(c->arena + c->plan.kjobs);
    g.klev = c->klev.data();
    g.nklev = (int)c->klev.size();
    g.fprog = c->cur.nf ? &c->fprog : nullptr;
    g.mems = c->dm;
    g.work1 = (const int2*)(c->arena + c->plan.work1);
    g.nb1 = c->plan.nb1;
    g.workp = (const int2*)(c->arena + c->plan.workp);
    g.nbp = c->plan.nbp;
    g.workr = (const int2*)(c->arena + c->plan.workr);
    g.nbr = c->plan.nbr;
    g.workb = (const int2*)(c->arena + c->plan.workb);
    g.nbb = c->plan.nbb;
    g.works = (const int2*)(c->arena + c->plan.works);
    g.nbs = c->plan.nbs;
    g.workm = (const int*)(c->arena + c->plan.workm);
    g.nmem = 1;
    return g;
}

int upload(lbm_ctx* c, void* dst, const void* src, size_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

void drop_graphs(lbm_ctx* c)
{
    for (int k = 0; k < 2; ++k) {
        for (auto& kv : c->gexec[k]) (void)hipGraphExecDestroy(kv.second);
        c->gexec[k].clear();
    }
    c->gver = -1;
}

// Fourier band QoIs: hipFFT plans (batched C2C / Z2Z over the components,
// in place, dimensions z, y, x) and the program that launch_fourier runs.
void drop_fourier(lbm_ctx* c)
{
    for (int k = 0; k < 4; ++k)
        if (c->fprog.plan[k]) hipfftDestroy((hipfftHandle)c->fprog.plan[k]);
    c->fprog = FourierProg{};
}

int build_fourier(lbm_ctx* c, const std::vector<FourierQ>& fq)
{
    drop_fourier(c);
    if (fq.empty()) return LBM_OK;
    FourierProg& f = c->fprog;
    const int D = c->plan.D, NC = c->plan.NC, N = c->plan.N;
    int n[3] = {c->cfg.nz, c->cfg.ny, c->cfg.nx};
    const int rank = D == 3 ? 3 : 2;
    int* dims = D == 3 ? n : n + 1;
    const hipfftType type = c->cfg.precision == LBM_FP64 ? HIPFFT_Z2Z : HIPFFT_C2C;
    for (const FourierQ& q : fq) (q.e ? f.qe : f.qz).push_back(q);
    const int batch[4] = {D, NC, (int)f.qe.size() * D, (int)f.qz.size() * NC};
    for (int k = 0; k < 4; ++k) {
        if (batch[k] == 0) continue;
        hipfftHandle h;
        if (hipfftPlanMany(&h, rank, dims, nullptr, 1, N, nullptr, 1, N, type, batch[k]) != HIPFFT_SUCCESS) {
            drop_fourier(c);
            return fail(LBM_EDEVICE, "hipFFT plan creation failed");
        }
        f.plan[k] = (void*)h;
    }
    char* A = c->arena;
    f.spec_v = A + c->plan.fspec_v;
    f.spec_w = A + c->plan.fspec_w;
    f.band_e = A + c->plan.fband_e;
    f.band_z = A + c->plan.fband_z;
    f.vs = A + c->plan.vs;
    f.w = A + c->plan.W;
    f.nx = c->cfg.nx; f.ny = c->cfg.ny; f.nz = c->cfg.nz;
    return LBM_OK;
}

// The kernel filters as sums of separable terms (Sec. 4.1): G_s is the
// product of the 1-D truncated Gaussian g (radius alpha s, alpha = 4 in 2-D
// and 2 in 3-D, normalised so that its cube sums to one); L_s is the sum over
// the axes a of (dilated biharmonic l_s along a) x (box of width s across a),
// scaled by 2 / sum |L_s| = 1 / (8 d s^d) (the d arms share the centre
// block, where the kernel is 6 d; each arm adds 10 s^d in absolute value).
// The identity is one term with unit taps.  The program: for E,
// V = R(R v*); for Z, V = curl^T R(R w).  One application of R is a level of
// x passes (one job per QoI and term), a level of y passes and a level of z
// passes that also sums the terms (2-D: the y level sums them); a last level
// forms the adjoint curls.  Writes the tap tables and the job table into the
// arena and the level list into the context.
int build_kjobs(lbm_ctx* c, const lbm_closure* cl)
{
    const int D = c->plan.D, NC = c->plan.NC, W = 2 * kMaxRad + 1;
    const size_t N = c->plan.N, e = c->plan.esz;
    char* A = c->arena;
    std::vector<double> taps((size_t)kMaxSA * 3 * W, 0.0);
    int ntap = 0;
    auto add = [&](const std::vector<double>& t) -> const void* {
        std::copy(t.begin(), t.end(), taps.begin() + (size_t)ntap * W);
        return A + c->plan.ktaps + (size_t)(ntap++) * W * e;
    };
    char* tcur = A + c->plan.kT;
    auto field = [&]() { char* f = tcur; tcur += 3 * N * e; return f; };
    struct Term { double coef; const void* tap[3]; int rad[3]; char* T1; char* T2; };
    struct QJob { std::vector<Term> terms; bool E; int nc; const void* X; char* Vs; char* Y1; char* Y2; };
    std::vector<QJob> qj;
    std::vector<FourierQ> fq;
    int isa = 0;
    for (int k = 0; k < cl->nq; ++k) {
        const lbm_qoi_spec& q = cl->q[k];
        if (q.kind == LBM_QOI_MP) continue;
        QJob j{};
        const int sc = q.scale;
        if (q.filter == LBM_FILT_FOURIER) {
            // no separable terms: the band goes through hipFFT
        } else if (q.filter == LBM_FILT_GAUSS) {
            const int r = (D == 2 ? 4 : 2) * sc;
            std::vector<double> g(2 * r + 1);
            double sum = 0;
            for (int i = -r; i <= r; ++i) sum += g[i + r] = std::exp(-(double)i * i / (2.0 * sc * sc));
            for (double& v : g) v /= sum;
            const void* tp = add(g);
            j.terms.push_back({1.0, {tp, tp, tp}, {r, r, r}, nullptr, nullptr});
        } else if (q.filter == LBM_FILT_LAPL) {
            static const double l5[5] = {1, -4, 6, -4, 1};
            const int rl = (5 * sc - 1) / 2, rb = (sc - 1) / 2;
            std::vector<double> l(2 * rl + 1), b(2 * rb + 1, 1.0);
            for (int i = 0; i < 5 * sc; ++i) l[i] = l5[i / sc];
            const void* tl = add(l);
            const void* tb = add(b);
            double sd = 1;
            for (int a = 0; a < D; ++a) sd *= sc;
            const double coef = 1.0 / (8.0 * D * sd);
            for (int a = 0; a < D; ++a) {
                Term t{coef, {tb, tb, tb}, {rb, rb, rb}, nullptr, nullptr};
                t.tap[a] = tl;
                t.rad[a] = rl;
                j.terms.push_back(t);
            }
        } else {
            const void* t1 = add(std::vector<double>{1.0});
            j.terms.push_back({1.0, {t1, t1, t1}, {0, 0, 0}, nullptr, nullptr});
        }
        for (Term& t : j.terms) { t.T1 = field(); t.T2 = field(); }
        j.E = q.kind == LBM_QOI_E;
        j.nc = j.E ? D : NC;
        j.X = j.E ? (const void*)(A + c->plan.vs) : (const void*)(A + c->plan.W);
        j.Vs = A + c->plan.kV + (size_t)isa * D * N * e;
        j.Y1 = field();
        j.Y2 = j.E ? nullptr : field();
        if (q.filter == LBM_FILT_FOURIER) fq.push_back({j.E ? 1 : 0, q.scale, q.kmax, j.E ? (void*)j.Vs : (void*)j.Y2});
        qj.push_back(j);
        isa++;
    }
    const int per_app = D == 3 ? 3 : 2;
    std::vector<std::vector<KJob>> lev(2 * per_app + 1);
    for (int app = 0; app < 2; ++app) {
        const int l0 = app * per_app;
        for (const QJob& q : qj) {
            const void* src = app == 0 ? q.X : (const void*)q.Y1;
            void* dst = app == 0 ? (void*)q.Y1 : (q.E ? (void*)q.Vs : (void*)q.Y2);
            KJob sum{};
            sum.op = 0;
            sum.axis = D == 3 ? 2 : 1;
            sum.ncomp = q.nc;
            sum.nterm = (int)q.terms.size();
            sum.dst = dst;
            for (size_t t = 0; t < q.terms.size(); ++t) {
                const Term& tm = q.terms[t];
                KJob x{};
                x.op = 0; x.axis = 0; x.ncomp = q.nc; x.nterm = 1;
                x.radius[0] = tm.rad[0]; x.coef[0] = 1.0; x.taps[0] = tm.tap[0]; x.src[0] = src; x.dst = tm.T1;
                lev[l0].push_back(x);
                if (D == 3) {
                    KJob y = x;
                    y.axis = 1; y.radius[0] = tm.rad[1]; y.taps[0] = tm.tap[1]; y.src[0] = tm.T1; y.dst = tm.T2;
                    lev[l0 + 1].push_back(y);
                }
                const int fa = D == 3 ? 2 : 1;   // the axis whose pass sums the terms
                sum.radius[t] = tm.rad[fa];
                sum.coef[t] = tm.coef;
                sum.taps[t] = tm.tap[fa];
                sum.src[t] = D == 3 ? tm.T2 : tm.T1;
            }
            if (!q.terms.empty()) lev[l0 + per_app - 1].push_back(sum);
        }
    }
    for (const QJob& q : qj)
        if (!q.E) {
            KJob cj{};
            cj.op = 1; cj.ncomp = q.nc; cj.src[0] = q.Y2; cj.dst = q.Vs;
            lev[2 * per_app].push_back(cj);
        }
    std::vector<KJob> all;
    c->klev.clear();
    for (const auto& l : lev) {
        if (l.empty()) continue;
        c->klev.push_back(make_int2((int)all.size(), (int)l.size()));
        all.insert(all.end(), l.begin(), l.end());
    }
    int rc = all.empty() ? LBM_OK : upload(c, A + c->plan.kjobs, all.data(), sizeof(KJob) * all.size());
    if (rc) return rc;
    rc = build_fourier(c, fq);
    if (rc) return rc;
    // tap tables in the run's element type
    if (e == 8) return upload(c, A + c->plan.ktaps, taps.data(), sizeof(double) * taps.size());
    std::vector<float> tf(taps.begin(), taps.end());
    return upload(c, A + c->plan.ktaps, tf.data(), sizeof(float) * tf.size());
}

// Build DevParam from a closure (host side) and upload it.
// The SGS change of the last enqueued step, which the next stream-collide
// would apply during its pull, added to the current populations (the
// records then read zero): before the state is read, replaced or streamed
// otherwise, or the closure changes.
int flush(lbm_ctx* c)
{
    if (!c->pending) return LBM_OK;
    launch_flush(c->cfg.lattice, c->cfg.precision, c->dm, (const int2*)(c->arena + c->plan.work1), c->plan.nb1,
                 c->phase, c->stream);
    c->pending = false;
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Nothing pending: the records cleared (a state set from elsewhere).
int clear_records(lbm_ctx* c)
{
    c->pending = false;
    if (!c->has_to) return LBM_OK;
    HIPCHK(hipMemsetAsync(c->arena + c->plan.rec, 0, (size_t)c->plan.esz * 2 * c->plan.D * c->plan.N, c->stream));
    return LBM_OK;
}

int apply_closure(lbm_ctx* c, const lbm_closure* cl)
{
    ClosureShape cs;
    int rc = closure_shape(&c->cfg, cl, &cs);
    if (rc) return rc;
    rc = flush(c);
    if (rc) return rc;
    if (cl) {
        const ClosureShape& cap = c->plan.cap;
        if (!c->has_to || cs.nsa > cap.nsa || cs.jv > cap.jv || (cs.has_z && (!cap.has_z || cs.jw > cap.jw)) ||
            cs.npart() > cap.npart() || cs.nbands > std::max(cap.nbands, 1) || cs.nhc > cap.nhc ||
            (cs.kf && (!cap.kf || cs.kslots > cap.kslots || cs.nzq > cap.nzq || cs.nf - cs.nfz > cap.nf - cap.nfz ||
                       cs.nfz > cap.nfz)))
            return fail(LBM_ENOMEM, "closure does not fit the workspace planned at creation");
        if (cs.h > 0 && cl->spinup < c->host_step + cs.h)
            return fail(LBM_EINVAL, "closure: spinup must be at least the step count plus the history length");
    }
    DevParam p{};
    if (cl) {
        p.nq = cl->nq;
        p.mode = cl->mode;
        p.nsa = cs.nsa;
        p.nmp = cs.nmp;
        p.nbands = cl->nbands;
        p.jv = cs.jv;
        p.jw = cs.jw;
        p.has_z = cs.has_z;
        p.has_e = cs.has_e;
        p.spinup = cl->spinup;
        p.seed = cl->seed;
        int isa = 0, imp = 0;
        for (int k = 0; k < cl->nq; ++k) {
            const lbm_qoi_spec& q = cl->q[k];
            if (q.kind == LBM_QOI_MP) {
                p.mp_slot[imp] = k;
                p.mp_band[imp] = q.band;
                imp++;
            } else {
                p.sa_slot[isa] = k;
                p.sa_kind[isa] = q.kind == LBM_QOI_E ? 0 : 1;
                double r[3];
                filter_poly(q.filter, r);
                for (int j = 0; j < 3; ++j) p.r[isa][j] = r[j];
                for (int j = 0; j <= kMaxPow; ++j) p.rr[isa][j] = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) p.rr[isa][a + b] += r[a] * r[b];
                for (int j = 0; j < 3; ++j) p.rf[isa][j] = (float)p.r[isa][j];
                for (int j = 0; j <= kMaxPow; ++j) p.rrf[isa][j] = (float)p.rr[isa][j];
                isa++;
            }
        }
        const int nq = cl->nq;
        p.kf = cs.kf;
        if (cs.kf) {
            rc = build_kjobs(c, cl);
            if (rc) return rc;
        }
        if (cl->mode == LBM_CLOSURE_LRS) {
            // rows of z*^n and the bias here; the history rows (z^{n-r} and
            // z*^{n-r}, r = 1..h) to the history buffer
            const int h = cs.h;
            for (int i = 0; i <= nq; ++i) {
                const long row = i < nq ? (long)h * nq + i : (long)(2 * h + 1) * nq;
                for (int k = 0; k < nq; ++k) p.C[i * kMaxQ + k] = cl->C[row * nq + k];
            }
            p.h = h;
            p.nhc = cs.nhc;
            if (h > 0) {
                const size_t rows = 2 * (size_t)h * nq;
                std::vector<double> ch(rows * nq);
                for (size_t r = 0; r < rows; ++r) {
                    const size_t src = r < (size_t)h * nq ? r : r + nq;   // skip the z*^n rows
                    for (int k = 0; k < nq; ++k) ch[r * nq + k] = cl->C[src * nq + k];
                }
                const size_t need = sizeof(double) * ch.size();
                if (need > c->chist_cap) {
                    if (c->chist_dev) HIPCHK(hipFree(c->chist_dev));
                    c->chist_dev = nullptr;
                    HIPCHK(hipMalloc(&c->chist_dev, need));
                    c->chist_cap = need;
                }
                rc = upload(c, c->chist_dev, ch.data(), need);
                if (rc) return rc;
                p.chist = c->chist_dev;
            }
            for (int k = 0; k < nq; ++k) p.mu[k] = cl->mu ? cl->mu[k] : 0.0;
            if (!cholesky_host(cl->Sigma, nq, p.L, kMaxQ)) return fail(LBM_EINVAL, "closure: Sigma is not SPD");
            if (cl->scale) {
                p.have_scale = 1;
                for (int k = 0; k < nq; ++k) p.scale[k] = cl->scale[k];
            }
        }
        std::vector<double> bw;
        if (cs.nmp > 0) {
            band_weights(c->cfg.ny, cl->nbands, cl->band_dmin, cl->band_dmax, bw);
            const double nxz = (double)c->cfg.nx * c->cfg.nz;
            for (int a = 0; a < cs.nmp; ++a)
                for (int b = 0; b < cs.nmp; ++b) {
                    double s = 0;
                    for (int y = 0; y < c->cfg.ny; ++y)
                        s += bw[(size_t)p.mp_band[a] * c->cfg.ny + y] * bw[(size_t)p.mp_band[b] * c->cfg.ny + y];
                    p.gmp[a * kMaxQ + b] = nxz * s;
                }
            rc = upload(c, c->arena + c->plan.bandw, bw.data(), sizeof(double) * bw.size());
            if (rc) return rc;
        }
        if (cl->mode == LBM_CLOSURE_TRACK && cl->nref > 0) {
            const size_t need = sizeof(double) * (size_t)cl->nref * nq;
            if (need > c->qref_cap) {
                if (c->qref_dev) HIPCHK(hipFree(c->qref_dev));
                c->qref_dev = nullptr;
                HIPCHK(hipMalloc(&c->qref_dev, need));
                c->qref_cap = need;
            }
            rc = upload(c, c->qref_dev, cl->qref, need);
            if (rc) return rc;
            p.qref = c->qref_dev;
            p.nref = (int)cl->nref;
        }
    }
    rc = upload(c, c->arena + c->plan.param, &p, sizeof p);
    if (rc) return rc;
    // fresh LRS scale and a recorded closure shape
    DevCtl ctl{};
    HIPCHK(hipMemcpyAsync(&ctl, c->arena + c->plan.ctl, sizeof ctl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ctl.s_set = 0;
    ctl.s_pend = 0;
    rc = upload(c, c->arena + c->plan.ctl, &ctl, sizeof ctl);
    if (rc) return rc;
    c->hp = p;
    c->cur = cl ? cs : ClosureShape{};
    c->hm.npart = c->cur.npart();
    refresh_member(c);
    rc = upload(c, c->dm, &c->hm, sizeof c->hm);
    if (rc) return rc;
    c->version++;
    drop_graphs(c);
    return LBM_OK;
}

int reset_ctl(lbm_ctx* c)
{
    DevCtl ctl{};
    int rc = upload(c, c->arena + c->plan.ctl, &ctl, sizeof ctl);
    // an empty record ring (its slots are part of the checkpoint image)
    if (!rc && hipMemsetAsync(c->arena + c->plan.recs, 0, sizeof(lbm_qoi_rec) * c->plan.rec_cap, c->stream) != hipSuccess)
        rc = fail(LBM_EDEVICE, "record ring reset failed");
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "record ring reset failed");
    c->host_step = 0;
    return rc;
}

// A hipFFT call of the launches since the last check failed (cleared).
int fft_status(lbm_ctx* c)
{
    if (!c->fprog.failed) return LBM_OK;
    c->fprog.failed = 0;
    return fail(LBM_EDEVICE, "hipFFT transform of a Fourier band QoI failed");
}

int enqueue_steps(lbm_ctx* c, long n)
{
    const LaunchGroup g = ctx_group(c);
    if (n > 0 && c->defers()) c->pending = true;
    for (long k = 0; k < n; ++k) {
        launch_step(g, c->stream, c->phase);
        c->phase ^= 1;
    }
    HIPCHK(hipGetLastError());
    return fft_status(c);
}

int capture(hipStream_t st, const std::vector<LaunchGroup>& groups, int nsteps, int phase0, hipGraphExec_t* out)
{
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < nsteps; ++k)
        for (const LaunchGroup& g : groups) launch_step(g, st, phase0 ^ (k & 1));
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    // move the executable graph to the device now, so that its first launch
    // does not pay for the upload
    e = hipGraphUpload(*out, st);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "graph upload failed: %s", hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }
const char* lbm_version(void) { return "lbm_hip 0.1 (gfx950)"; }

int lbm_device_tag(char* out, size_t n)
{
    if (!out || n == 0) return fail(LBM_EINVAL, "device_tag: no buffer");
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return fail(LBM_EDEVICE, "device_tag: no HIP device");
    std::snprintf(out, n, "%s %dCU", p.gcnArchName, p.multiProcessorCount);
    return LBM_OK;
}

int lbm_lattice_info(int lattice, int* c, double* w)
{
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_EINVAL, "bad lattice");
    if (!c || !w) return fail(LBM_EINVAL, "NULL output");
    return lattice_table(lattice, c, w);
}

size_t lbm_required_bytes(const lbm_config* cfg, const lbm_closure* closure)
{
    if (check_config(cfg)) return 0;
    ClosureShape cs;
    if (closure_shape(cfg, closure, &cs)) return 0;
    Plan p;
    make_plan(cfg, cs, &p);
    return p.total;
}

int lbm_create(const lbm_config* cfg, const lbm_closure* closure, void* dev_arena, size_t bytes, void* stream,
               lbm_ctx** out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    ClosureShape cs;
    rc = closure_shape(cfg, closure, &cs);
    if (rc) return rc;
    if (!dev_arena || ((uintptr_t)dev_arena % kAlign)) return fail(LBM_EINVAL, "arena must be 256-byte aligned device memory");
    Plan plan;
    make_plan(cfg, cs, &plan);
    if (bytes < plan.total) return fail(LBM_ENOMEM, "arena has %zu bytes, %zu needed", bytes, plan.total);
    lbm_ctx* c = new lbm_ctx();
    c->cfg = *cfg;
    c->plan = plan;
    c->arena = (char*)dev_arena;
    c->stream = (hipStream_t)stream;
    if (!c->stream) {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(LBM_EDEVICE, "stream creation failed");
        }
        c->own_stream = true;
    }
    c->has_to = cs.nq > 0;
    char* A = c->arena;
    DevMember& m = c->hm;
    m.nx = cfg->nx; m.ny = cfg->ny; m.nz = cfg->nz; m.N = plan.N;
    m.walls = cfg->walls_y; m.substrate = cfg->substrate; m.force_kind = cfg->force_kind; m.force_k = cfg->force_k;
    m.parity = 0; m.has_to = c->has_to; m.diag = cfg->diag; m.rec_cap = plan.rec_cap;
    m.tau = cfg->tau; m.cmodel = cfg->c_model; m.force_amp = cfg->force_amp; m.drag = cfg->drag;
    m.g[0] = A + plan.g0; m.g[1] = A + plan.g1;
    m.vn = A + plan.vn;
    m.part_stats = (double*)(A + plan.part_stats);
    m.part_diag = (double*)(A + plan.part_diag);
    m.nb1 = plan.nb1; m.nbx2 = plan.nbx2; m.cpt2 = plan.cpt2; m.npart = 0; m.zc = plan.zc; m.btx = plan.btx;
    m.prm = (DevParam*)(A + plan.param);
    m.ctl = (DevCtl*)(A + plan.ctl);
    m.recs = (lbm_qoi_rec*)(A + plan.recs);
    m.fprof = (double*)(A + plan.fprof);
    if (c->has_to) {
        m.rho = A + plan.rho; m.vs = A + plan.vs; m.P = A + plan.P; m.W = A + plan.W; m.C = A + plan.Cf;
        m.part_to = (double*)(A + plan.part_to);
        m.bandw = (double*)(A + plan.bandw);
        m.cmp = (double*)(A + plan.cmp);
        m.sums = (double*)(A + plan.sums);
        m.hpart = (double*)(A + plan.hpart);
        if (plan.cap.kf) m.kV = A + plan.kV;
        m.rec = A + plan.rec;
    }
    m.nst = plan.nb1;
    c->dm = (DevMember*)(A + plan.member);
    // host tables
    std::vector<double> fp(cfg->ny, 0.0);
    for (int y = 0; y < cfg->ny; ++y) {
        if (cfg->force_kind == LBM_FORCE_SIN_Y)
            fp[y] = cfg->force_amp * std::sin(2.0 * M_PI * cfg->force_k * y / cfg->ny);
        else if (cfg->force_kind == LBM_FORCE_CONST_X)
            fp[y] = cfg->force_amp;
    }
    std::vector<int2> w1(plan.nb1), wp(plan.nbp);
    {
        const std::vector<int> o = xcd_order(plan.nb1);
        for (int b = 0; b < plan.nb1; ++b) w1[b] = make_int2(0, o[b]);
        const std::vector<int> op = xcd_order(plan.nbp);
        for (int b = 0; b < plan.nbp; ++b) wp[b] = make_int2(0, op[b]);
    }
    int zero = 0;
    rc = upload(c, A + plan.fprof, fp.data(), sizeof(double) * fp.size());
    if (!rc) rc = upload(c, A + plan.work1, w1.data(), sizeof(int2) * w1.size());
    if (!rc) rc = upload(c, A + plan.workp, wp.data(), sizeof(int2) * wp.size());
    if (!rc) rc = upload(c, A + plan.workm, &zero, sizeof zero);
    if (!rc && c->has_to) {
        std::vector<int2> wr(plan.nbr);
        for (int b = 0; b < plan.nbr; ++b) wr[b] = make_int2(0, b);
        rc = upload(c, A + plan.workr, wr.data(), sizeof(int2) * wr.size());
        std::vector<int2> wb(plan.nbb);
        {
            const int ntx = (cfg->nx + plan.btx - 1) / plan.btx, nty = (cfg->ny + kBinTY - 1) / kBinTY;
            const std::vector<int> o = xcd_tile_order(ntx, nty, plan.nbb / (ntx * nty));
            for (int b = 0; b < plan.nbb; ++b) wb[b] = make_int2(0, o[b]);
        }
        if (!rc) rc = upload(c, A + plan.workb, wb.data(), sizeof(int2) * wb.size());
        std::vector<int2> ws(plan.nbs);
        for (int b = 0; b < plan.nbs; ++b) ws[b] = make_int2(0, ksum_slot(b, plan.cap.nhc));
        if (!rc) rc = upload(c, A + plan.works, ws.data(), sizeof(int2) * ws.size());
    }
    if (!rc) rc = upload(c, c->dm, &m, sizeof m);
    if (!rc) rc = reset_ctl(c);
    if (!rc) rc = clear_records(c);
    if (!rc) {
        DevParam p{};
        rc = upload(c, A + plan.param, &p, sizeof p);
    }
    // initial state rho = 1, v = 0; the padding cells of the last population
    // block (never read or written by the kernels) are zeroed, so that state
    // images of equal states are equal byte for byte
    if (!rc) {
        const size_t blk = (size_t)plan.esz * plan.Q * kPopBlk;
        const size_t last = (size_t)plan.esz * plan.popn - blk;
        if (hipMemsetAsync(A + plan.g0 + last, 0, blk, c->stream) != hipSuccess ||
            hipMemsetAsync(A + plan.g1 + last, 0, blk, c->stream) != hipSuccess)
            rc = fail(LBM_EDEVICE, "init failed");
    }
    if (!rc) {
        launch_state(OP_INIT, cfg->lattice, cfg->precision, c->dm, plan.N, c->has_to, 0, c->stream, nullptr, nullptr);
        if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "init failed");
    }
    if (!rc && closure) rc = apply_closure(c, closure);
    if (rc) {
        if (c->qref_dev) (void)hipFree(c->qref_dev);
        if (c->chist_dev) (void)hipFree(c->chist_dev);
        drop_fourier(c);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return rc;
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->qref_dev) (void)hipFree(c->qref_dev);
    if (c->chist_dev) (void)hipFree(c->chist_dev);
    if (c->proj_tmp) (void)hipFree(c->proj_tmp);
    drop_fourier(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"

namespace {
// The equilibrium state of density rho_dev [N] (NULL: 1) and velocity
// u_dev [D][N] (device memory, double) on the context stream: nothing
// pending, an empty record ring, step 0.
int init_from_device(lbm_ctx* c, const double* rho_dev, const double* u_dev)
{
    int rc = clear_records(c);
    if (rc) return rc;
    c->phase = 0;
    launch_state(OP_INIT, c->cfg.lattice, c->cfg.precision, c->dm, c->plan.N, c->has_to, 0, c->stream, rho_dev,
                 (double*)u_dev);
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "init kernel failed");
    if (!rc) rc = reset_ctl(c);
    c->version++;
    return rc;
}
}  // namespace

extern "C" {

int lbm_init_velocity(lbm_ctx* c, const double* rho, const double* u)
{
    if (!c || !u) return fail(LBM_EINVAL, "NULL argument");
    const size_t N = c->plan.N, D = c->plan.D;
    double* buf = nullptr;
    HIPCHK(hipMalloc(&buf, sizeof(double) * (D + 1) * N));
    int rc = upload(c, buf, u, sizeof(double) * D * N);
    if (!rc && rho) rc = upload(c, buf + D * N, rho, sizeof(double) * N);
    if (!rc) rc = init_from_device(c, rho ? buf + D * N : nullptr, buf);
    (void)hipFree(buf);
    return rc;
}

int lbm_set_closure(lbm_ctx* c, const lbm_closure* cl)
{
    if (!c) return fail(LBM_EINVAL, "NULL context");
    return apply_closure(c, cl);
}

// Steps run as replays of captured graphs: chunks of gchunk steps, and the
// remainder as one chunk of its even part (so the phase a graph starts from is
// unchanged after it); a last odd step, and steps with hipFFT work, launch
// eagerly.
static long graph_chunk(const lbm_ctx* c, long n)
{
    if (c->cur.nf) return 0;   // hipFFT runs outside graphs
    const long len = n >= c->gchunk ? c->gchunk : (n & ~1L);
    return len >= 2 ? len : 0;
}

// The graph of len steps from ping-pong phase ph, captured if not cached.
static int step_graph(lbm_ctx* c, int len, int ph, hipGraphExec_t* out)
{
    if (c->gver != c->version) drop_graphs(c);
    c->gver = c->version;
    auto& cache = c->gexec[ph];
    auto it = cache.find(len);
    if (it == cache.end()) {
        hipGraphExec_t g = nullptr;
        std::vector<LaunchGroup> gs{ctx_group(c)};
        const int rc = capture(c->stream, gs, len, ph, &g);
        if (rc) return rc;
        it = cache.emplace(len, g).first;
    }
    *out = it->second;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, long n)
{
    if (!c || n < 0) return fail(LBM_EINVAL, "bad arguments");
    while (n > 0) {
        const long len = graph_chunk(c, n);
        if (len > 0) {
            hipGraphExec_t g = nullptr;
            int rc = step_graph(c, (int)len, c->phase, &g);
            if (rc) return rc;
            HIPCHK(hipGraphLaunch(g, c->stream));
            if (c->defers()) c->pending = true;
            n -= len;
            c->host_step += len;
            // len is even: the phase is unchanged
        } else {
            const long e = c->cur.nf ? n : 1;
            int rc = enqueue_steps(c, e);
            c->host_step += e;   // the steps were enqueued (and the phase advanced) even if one failed
            if (rc) return rc;
            n -= e;
        }
    }
    return LBM_OK;
}

int lbm_step_prepare(lbm_ctx* c, long n)
{
    if (!c || n < 0) return fail(LBM_EINVAL, "bad arguments");
    while (n > 0) {
        const long len = graph_chunk(c, n);
        if (len == 0) break;   // the rest launches eagerly
        // both ping-pong phases, so that steps taken in between (an odd
        // number, say) do not make the prepared graphs miss
        for (int ph = 0; ph < 2; ++ph) {
            hipGraphExec_t g = nullptr;
            int rc = step_graph(c, (int)len, ph, &g);
            if (rc) return rc;
        }
        n -= len;
    }
    return LBM_OK;
}

int lbm_sync(lbm_ctx* c)
{
    if (!c) return fail(LBM_EINVAL, "NULL context");
    HIPCHK(hipStreamSynchronize(c->stream));
    int flags = 0;
    HIPCHK(hipMemcpy(&flags, c->arena + c->plan.ctl + offsetof(DevCtl, flags), sizeof flags, hipMemcpyDeviceToHost));
    if (flags & 1) return fail(LBM_EUNSTABLE, "run became unstable (non-finite value or |v| > 0.5)");
    return LBM_OK;
}

long lbm_step_count(const lbm_ctx* c) { return c ? c->host_step : -1; }

int lbm_qoi(lbm_ctx* c, long first, long count, lbm_qoi_rec* out)
{
    if (!c || first < 0 || count < 0 || (count && !out)) return fail(LBM_EINVAL, "bad arguments");
    if (c->mode() == 0) return fail(LBM_ESTATE, "no records: plain run without diagnostics");
    const long cap = c->plan.rec_cap;
    if (first + count > c->host_step || first < c->host_step - cap)
        return fail(LBM_ESTATE, "records [%ld,%ld) not retained (have [%ld,%ld))", first, first + count,
                    std::max(0L, c->host_step - cap), c->host_step);
    HIPCHK(hipStreamSynchronize(c->stream));
    const lbm_qoi_rec* d = (const lbm_qoi_rec*)(c->arena + c->plan.recs);
    long k = 0;
    while (k < count) {
        const long slot = (first + k) % cap;
        const long run = std::min(count - k, cap - slot);
        HIPCHK(hipMemcpy(out + k, d + slot, sizeof(lbm_qoi_rec) * run, hipMemcpyDeviceToHost));
        k += run;
    }
    return LBM_OK;
}

int lbm_velocity(lbm_ctx* c, double* u)
{
    return lbm_fields(c, nullptr, u);
}

int lbm_fields(lbm_ctx* c, double* rho, double* u)
{
    if (!c || !u) return fail(LBM_EINVAL, "NULL argument");
    const size_t N = c->plan.N, D = c->plan.D;
    int frc = flush(c);
    if (frc) return frc;
    double* buf = nullptr;
    HIPCHK(hipMalloc(&buf, sizeof(double) * (D + 1) * N));
    launch_fields(c->cfg.lattice, c->cfg.precision, c->dm, (const int2*)(c->arena + c->plan.work1), c->plan.nb1,
                  c->has_to, c->phase, c->stream, buf + D * N);
    int rc = LBM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "moments kernel failed");
    // velocity is in vn (element type of the run); widen on the host
    if (!rc) {
        const size_t e = c->plan.esz;
        std::vector<char> tmp(e * D * N);
        if (hipMemcpy(tmp.data(), c->arena + c->plan.vn, tmp.size(), hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(LBM_EDEVICE, "copy failed");
        else {
            for (size_t k = 0; k < D * N; ++k)
                u[k] = e == 8 ? ((const double*)tmp.data())[k] : (double)((const float*)tmp.data())[k];
            if (rho && hipMemcpy(rho, buf + D * N, sizeof(double) * N, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(LBM_EDEVICE, "copy failed");
        }
    }
    (void)hipFree(buf);
    return rc;
}

}  // extern "C"

// Staging of lbm_fields_noalloc: a fixed device array instead of an
// allocation per call.  Each GPU the library runs on holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the device (the array's name is a host-side
// stand-in, not a device address).
namespace {
constexpr size_t kFieldScratchBytes = size_t(LBM_FIELDS_NOALLOC_MAX_BYTES);
static __device__ __align__(256) unsigned char scratch[kFieldScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// The current device's copy of the array, looked up once per device (with
// that device current).
int field_scratch(double** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EDEVICE, "fields_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EDEVICE, "fields_noalloc: no address of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_at[dev] = p;
    }
    *out = (double*)g_scratch_at[dev];
    return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_fields_noalloc(lbm_ctx* c, double* rho, double* u)
{
    if (!c || !u) return fail(LBM_EINVAL, "NULL argument");
    const size_t N = c->plan.N, D = c->plan.D;
    const size_t need = sizeof(double) * (D + 1) * N;
    if (need > kFieldScratchBytes)
        return fail(LBM_EINVAL,
                    "fields_noalloc: %zu cells need %zu bytes of staging, more than the %zu-byte static scratch "
                    "(at most %zu cells in %zu-D); use lbm_fields",
                    N, need, kFieldScratchBytes, kFieldScratchBytes / (sizeof(double) * (D + 1)), D);
    double* sp = nullptr;
    int rc = field_scratch(&sp);
    if (rc) return rc;
    rc = flush(c);
    if (rc) return rc;
    // every element of the staging is written before it is read: nothing to clear
    launch_fields(c->cfg.lattice, c->cfg.precision, c->dm, (const int2*)(c->arena + c->plan.work1), c->plan.nb1,
                  c->has_to, c->phase, c->stream, sp + D * N, sp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(u, sp, sizeof(double) * D * N, hipMemcpyDeviceToHost));
    if (rho) HIPCHK(hipMemcpy(rho, sp + D * N, sizeof(double) * N, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx* c, double* f)
{
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = (size_t)c->plan.Q * c->plan.N;
    int frc = flush(c);
    if (frc) return frc;
    double* buf = nullptr;
    HIPCHK(hipMalloc(&buf, sizeof(double) * n));
    launch_state(OP_GET_POP, c->cfg.lattice, c->cfg.precision, c->dm, c->plan.N, c->has_to, c->phase, c->stream,
                 nullptr, buf);
    int rc = LBM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipMemcpy(f, buf, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(LBM_EDEVICE, "population read failed");
    (void)hipFree(buf);
    return rc;
}

int lbm_set_populations(lbm_ctx* c, const double* f)
{
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = (size_t)c->plan.Q * c->plan.N;
    double* buf = nullptr;
    HIPCHK(hipMalloc(&buf, sizeof(double) * n));
    int rc = upload(c, buf, f, sizeof(double) * n);
    if (!rc) rc = clear_records(c);
    if (!rc) {
        launch_state(OP_SET_POP, c->cfg.lattice, c->cfg.precision, c->dm, c->plan.N, c->has_to, c->phase, c->stream,
                     buf, nullptr);
        if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "population write failed");
    }
    (void)hipFree(buf);
    c->version++;
    return rc;
}

int lbm_stream_only(lbm_ctx* c)
{
    if (!c) return fail(LBM_EINVAL, "NULL context");
    int frc = flush(c);
    if (frc) return frc;
    launch_state(OP_STREAM, c->cfg.lattice, c->cfg.precision, c->dm, c->plan.N, false, c->phase, c->stream,
                 nullptr, nullptr);
    c->phase ^= 1;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->version++;
    return LBM_OK;
}

// HF -> LF projection (Sec. 3, phi_m; Sec. 7.1: wall-anchored stride-m
// subsampling).  The coarse grid is the fine one divided by m on every axis
// (z kept in 2-D), same lattice and wall setting; m odd.
static int check_projection(const lbm_ctx* f, const lbm_ctx* c, int m, int kind)
{
    if (!f || !c) return fail(LBM_EINVAL, "NULL context");
    if (m < 1 || m % 2 == 0) return fail(LBM_EINVAL, "projection: m must be odd and positive");
    if (kind != LBM_PROJ_STRIDE && kind != LBM_PROJ_BICUBIC) return fail(LBM_EINVAL, "projection: bad kind");
    if (kind == LBM_PROJ_BICUBIC && (f->cfg.lattice != LBM_D2Q9 || f->cfg.walls_y || m > 15))
        return fail(LBM_EINVAL, "projection: bicubic needs a doubly periodic D2Q9 grid and m <= 15");
    if (f->cfg.lattice != c->cfg.lattice || f->cfg.walls_y != c->cfg.walls_y)
        return fail(LBM_EINVAL, "projection: lattice and walls must match");
    const bool d3 = f->cfg.lattice == LBM_D3Q19;
    if ((long)c->cfg.nx * m != f->cfg.nx || (long)c->cfg.ny * m != f->cfg.ny ||
        (d3 ? (long)c->cfg.nz * m != f->cfg.nz : c->cfg.nz != 1))
        return fail(LBM_EINVAL, "projection: the coarse grid must be the fine grid divided by m on every axis");
    return LBM_OK;
}

int lbm_project_state(lbm_ctx* f, lbm_ctx* c, int m) { return lbm_project_state_kind(f, c, m, LBM_PROJ_STRIDE); }
int lbm_project_qoi(lbm_ctx* f, lbm_ctx* p, int m) { return lbm_project_qoi_kind(f, p, m, LBM_PROJ_STRIDE); }

int lbm_project_state_kind(lbm_ctx* f, lbm_ctx* c, int m, int kind)
{
    int rc = check_projection(f, c, m, kind);
    if (rc) return rc;
    const size_t Nc = c->plan.N, Q = c->plan.Q;
    rc = flush(f);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(f->stream));   // the fine run's pending steps
    double* buf = nullptr;
    HIPCHK(hipMalloc(&buf, sizeof(double) * Q * Nc));
    launch_project(f->cfg.lattice, f->cfg.precision, f->dm, f->phase, m, c->cfg.nx, c->cfg.ny, c->cfg.nz, buf,
                   nullptr, 0, kind, f->stream);
    if (hipStreamSynchronize(f->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "projection kernel failed");
    if (!rc) rc = clear_records(c);
    if (!rc) {
        c->phase = 0;
        launch_state(OP_SET_POP, c->cfg.lattice, c->cfg.precision, c->dm, c->plan.N, c->has_to, 0, c->stream, buf,
                     nullptr);
        if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LBM_EDEVICE, "population write failed");
    }
    (void)hipFree(buf);
    if (!rc) rc = reset_ctl(c);
    c->version++;
    return rc;
}

int lbm_project_qoi_kind(lbm_ctx* f, lbm_ctx* p, int m, int kind)
{
    int rc = check_projection(f, p, m, kind);
    if (rc) return rc;
    if (!p->has_to || p->cur.nq == 0 || p->hp.mode != LBM_CLOSURE_OFF)
        return fail(LBM_EINVAL, "project_qoi: the probe needs a closure in mode OFF");
    if (f->stream != p->stream) return fail(LBM_EINVAL, "project_qoi: fine run and probe must share one stream");
    rc = flush(f);
    if (rc) return rc;
    if (kind == LBM_PROJ_BICUBIC) {   // the probe's scratch for the separable passes, made on first use
        const size_t need = sizeof(double) * 2 * (size_t)f->cfg.ny * p->cfg.nx;
        if (p->proj_tmp_bytes < need) {
            HIPCHK(hipStreamSynchronize(p->stream));
            if (p->proj_tmp) HIPCHK(hipFree(p->proj_tmp));
            p->proj_tmp = nullptr;
            p->proj_tmp_bytes = 0;
            HIPCHK(hipMalloc(&p->proj_tmp, need));
            p->proj_tmp_bytes = need;
        }
    }
    launch_project(f->cfg.lattice, f->cfg.precision, f->dm, f->phase, m, p->cfg.nx, p->cfg.ny, p->cfg.nz, nullptr,
                   p->arena + p->plan.vs, p->cfg.precision == LBM_FP64, kind, p->stream,
                   kind == LBM_PROJ_BICUBIC ? p->proj_tmp : nullptr);
    LaunchGroup g = ctx_group(p);
    g.probe = 1;
    launch_step(g, p->stream, p->phase);
    if (hipGetLastError() != hipSuccess) return fail(LBM_EDEVICE, "project_qoi: launch failed");
    p->host_step++;
    return LBM_OK;
}

// Checkpoint image: header, current populations (the SGS change of the last
// step is already in them), control block, records.
struct StateHeader {
    uint64_t magic;
    int64_t host_step;
    int32_t Q, N, esz, has_to;
};

// State images hold the populations in the device's blocked layout and the
// control block with its step snapshot and pending LRS scale.
constexpr unsigned long long kStateMagic = 0x4C424D53544156ULL;

size_t lbm_state_bytes(const lbm_ctx* c)
{
    if (!c) return 0;
    const Plan& p = c->plan;
    size_t b = sizeof(StateHeader) + (size_t)p.esz * p.popn + sizeof(DevCtl) + sizeof(lbm_qoi_rec) * p.rec_cap;
    return b;
}

// The control block of a state image in one form whichever launch formed the
// solve: a first LRS scale that the apply left pending is committed (as the
// next k_sum would commit it), and the values every step forms afresh before
// reading them (the dv coefficients, the step snapshot) are cleared.
static void canonical_ctl(DevCtl& t)
{
    if (t.s_pend) {
        for (int k = 0; k < kMaxQ; ++k) t.s[k] = t.s_next[k];
        t.s_set = 1;
        t.s_pend = 0;
    }
    t.step_snap = 0;
    for (int k = 0; k < kMaxQ; ++k) t.s_next[k] = 0.0;
    for (int j = 0; j <= kMaxPow; ++j) {
        t.cv[j] = t.cw[j] = 0.0;
        t.cvf[j] = t.cwf[j] = 0.0f;
    }
    for (int k = 0; k < kMaxSA; ++k) {
        t.bsa[k] = 0.0;
        t.bsaf[k] = 0.0f;
    }
}

int lbm_get_state(lbm_ctx* c, void* host, size_t bytes)
{
    if (!c || !host) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < lbm_state_bytes(c)) return fail(LBM_EINVAL, "buffer too small");
    int frc = flush(c);
    if (frc) return frc;
    HIPCHK(hipStreamSynchronize(c->stream));
    const Plan& p = c->plan;
    char* o = (char*)host;
    StateHeader h{kStateMagic, c->host_step, p.Q, p.N, p.esz, c->has_to};
    memcpy(o, &h, sizeof h);
    o += sizeof h;
    const size_t gb = (size_t)p.esz * p.popn;
    HIPCHK(hipMemcpy(o, c->hm.g[c->hm.parity ^ c->phase], gb, hipMemcpyDeviceToHost));
    o += gb;
    DevCtl ctl;
    HIPCHK(hipMemcpy(&ctl, c->arena + p.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    canonical_ctl(ctl);
    memcpy(o, &ctl, sizeof ctl);
    o += sizeof(DevCtl);
    HIPCHK(hipMemcpy(o, c->arena + p.recs, sizeof(lbm_qoi_rec) * p.rec_cap, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const void* host, size_t bytes)
{
    if (!c || !host) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < lbm_state_bytes(c)) return fail(LBM_EINVAL, "buffer too small");
    const Plan& p = c->plan;
    const char* o = (const char*)host;
    StateHeader h;
    memcpy(&h, o, sizeof h);
    if (h.magic != kStateMagic || h.Q != p.Q || h.N != p.N || h.esz != p.esz || h.has_to != (int)c->has_to)
        return fail(LBM_EINVAL, "state image does not match this context");
    o += sizeof h;
    int crc = clear_records(c);
    if (crc) return crc;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->phase = 0;
    const size_t gb = (size_t)p.esz * p.popn;
    HIPCHK(hipMemcpy(c->hm.g[c->hm.parity], o, gb, hipMemcpyHostToDevice));
    o += gb;
    HIPCHK(hipMemcpy(c->arena + p.ctl, o, sizeof(DevCtl), hipMemcpyHostToDevice));
    o += sizeof(DevCtl);
    HIPCHK(hipMemcpy(c->arena + p.recs, o, sizeof(lbm_qoi_rec) * p.rec_cap, hipMemcpyHostToDevice));
    c->host_step = h.host_step;
    c->version++;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
static void batch_free_dev(lbm_batch* b)
{
    for (int k = 0; k < 2; ++k) {
        for (auto& kv : b->gexec[k]) (void)hipGraphExecDestroy(kv.second);
        b->gexec[k].clear();
    }
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->dwork) (void)hipFree(b->dwork);
    if (b->dworkm) (void)hipFree(b->dworkm);
    b->dmem = nullptr;
    b->dwork = nullptr;
    b->dworkm = nullptr;
    b->groups.clear();
}

static int batch_build(lbm_batch* b)
{
    batch_free_dev(b);
    const int n = (int)b->mem.size();
    // group members by kernel kind
    struct Key { int lat, prec, sub, mode, sab, btx, kfm, def, sep; };   // kfm: kernel-filter member (own group)
    std::vector<Key> keys;
    std::vector<std::vector<int>> gm;
    for (int i = 0; i < n; ++i) {
        const lbm_ctx* c = b->mem[i];
        Key k{c->cfg.lattice, c->cfg.precision, c->cfg.substrate, c->mode(), c->cur.nsa <= 2 ? 2 : (c->cur.nsa <= 6 ? 6 : 8),
              c->plan.btx, c->mode() == 2 && c->cur.kf ? i : -1, (int)c->defers(), (c->cfg.tune_mem & 8) != 0};
        int gi = -1;
        for (size_t j = 0; j < keys.size(); ++j)
            if (!memcmp(&keys[j], &k, sizeof k)) gi = (int)j;
        if (gi < 0) { keys.push_back(k); gm.emplace_back(); gi = (int)keys.size() - 1; }
        gm[gi].push_back(i);
    }
    std::vector<DevMember> hmem(n);
    std::vector<int2> work;
    std::vector<int> workm;
    struct Off { size_t w1, nb1, wp, nbp, wr, nbr, wb, nbb, ws, nbs, wm, nm; };
    std::vector<Off> offs;
    for (size_t gi = 0; gi < keys.size(); ++gi) {
        Off o{};
        o.w1 = work.size();
        for (int i : gm[gi]) {
            const std::vector<int> o = xcd_order(b->mem[i]->plan.nb1);
            for (int k = 0; k < b->mem[i]->plan.nb1; ++k) work.push_back(make_int2(i, o[k]));
        }
        o.nb1 = work.size() - o.w1;
        o.wp = work.size();
        for (int i : gm[gi]) {
            const std::vector<int> op = xcd_order(b->mem[i]->plan.nbp);
            for (int k = 0; k < b->mem[i]->plan.nbp; ++k) work.push_back(make_int2(i, op[k]));
        }
        o.nbp = work.size() - o.wp;
        o.wr = work.size();
        if (keys[gi].mode == 2)
            for (int i : gm[gi])
                for (int k = 0; k < b->mem[i]->plan.nbr; ++k) work.push_back(make_int2(i, k));
        o.nbr = work.size() - o.wr;
        o.wb = work.size();
        if (keys[gi].mode == 2)
            for (int i : gm[gi]) {
                const lbm_config& mc = b->mem[i]->cfg;
                const int btx = b->mem[i]->plan.btx;
                const int ntx = (mc.nx + btx - 1) / btx, nty = (mc.ny + kBinTY - 1) / kBinTY;
                const std::vector<int> o = xcd_tile_order(ntx, nty, b->mem[i]->plan.nbb / (ntx * nty));
                for (int k = 0; k < b->mem[i]->plan.nbb; ++k) work.push_back(make_int2(i, o[k]));
            }
        o.nbb = work.size() - o.wb;
        o.ws = work.size();
        if (keys[gi].mode == 2)
            for (int i : gm[gi])
                for (int k = 0; k < b->mem[i]->plan.nbs; ++k)
                    work.push_back(make_int2(i, ksum_slot(k, b->mem[i]->plan.cap.nhc)));
        o.nbs = work.size() - o.ws;
        o.wm = workm.size();
        for (int i : gm[gi]) workm.push_back(i);
        o.nm = workm.size() - o.wm;
        offs.push_back(o);
    }
    b->phase0.resize(n);
    b->ver0.resize(n);
    for (int i = 0; i < n; ++i) {
        lbm_ctx* c = b->mem[i];
        hmem[i] = c->hm;
        hmem[i].parity = c->hm.parity ^ c->phase;
        b->phase0[i] = c->phase;
        b->ver0[i] = c->version;
    }
    b->phase = 0;
    HIPCHK(hipMalloc(&b->dmem, sizeof(DevMember) * n));
    HIPCHK(hipMalloc(&b->dwork, sizeof(int2) * std::max<size_t>(work.size(), 1)));
    HIPCHK(hipMalloc(&b->dworkm, sizeof(int) * std::max<size_t>(workm.size(), 1)));
    HIPCHK(hipMemcpyAsync(b->dmem, hmem.data(), sizeof(DevMember) * n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->dwork, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->dworkm, workm.data(), sizeof(int) * workm.size(), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (size_t gi = 0; gi < keys.size(); ++gi) {
        LaunchGroup g{};
        g.lattice = keys[gi].lat;
        g.precision = keys[gi].prec;
        g.substrate = keys[gi].sub;
        g.mode = keys[gi].mode;
        g.btx = keys[gi].btx;
        double pop_bytes = 0;   // one launch covers the whole group
        for (int i : gm[gi]) pop_bytes += (double)b->mem[i]->plan.N * b->mem[i]->plan.Q * b->mem[i]->plan.esz;
        g.wt = write_through(pop_bytes);
        g.nt = non_temporal(pop_bytes);
        g.a32 = 1;
        for (int i : gm[gi]) {
            g.a32 &= (double)b->mem[i]->plan.popn * b->mem[i]->plan.esz < 4294967296.0 &&
                     !(b->mem[i]->cfg.tune_mem & 1);
            g.nt |= (b->mem[i]->cfg.tune_mem & 2) != 0;
            const lbm_ctx* c = b->mem[i];
            g.any_z |= c->cur.has_z;
            g.maxpow = std::max(g.maxpow, std::max(c->cur.jv, c->cur.jw));
            g.maxsa = std::max(g.maxsa, c->cur.nsa);
            g.npass = std::max(g.npass, binom_passes(c->cur));
            g.defer = c->defers();   // (members of a group share mode and substrate)
            g.sep_solve = (c->cfg.tune_mem & 8) != 0;
            add_pass_masks(c, g);
            if (keys[gi].kfm >= 0) {
                g.kf = 1;
                g.npass = 0;
                g.kjobs = (const KJob*)(c->arena + c->plan.kjobs);
                g.klev = c->klev.data();
                g.nklev = (int)c->klev.size();
                g.fprog = c->cur.nf ? &c->fprog : nullptr;
            }
        }
        g.mems = b->dmem;
        g.work1 = b->dwork + offs[gi].w1;
        g.nb1 = (int)offs[gi].nb1;
        g.workp = b->dwork + offs[gi].wp;
        g.nbp = (int)offs[gi].nbp;
        g.workr = b->dwork + offs[gi].wr;
        g.nbr = (int)offs[gi].nbr;
        g.workb = b->dwork + offs[gi].wb;
        g.nbb = (int)offs[gi].nbb;
        g.works = b->dwork + offs[gi].ws;
        g.nbs = (int)offs[gi].nbs;
        g.workm = b->dworkm + offs[gi].wm;
        g.nmem = (int)offs[gi].nm;
        b->groups.push_back(g);
    }
    return LBM_OK;
}

int lbm_batch_create(int n, lbm_ctx* const* members, lbm_batch** out)
{
    if (!out || n < 1 || !members) return fail(LBM_EINVAL, "bad arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!members[i]) return fail(LBM_EINVAL, "member %d is NULL", i);
        if (members[i]->stream != members[0]->stream) return fail(LBM_EINVAL, "members must share one stream");
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return fail(LBM_EINVAL, "member %d repeated", i);
    }
    lbm_batch* b = new lbm_batch();
    b->mem.assign(members, members + n);
    b->stream = members[0]->stream;
    int rc = batch_build(b);
    if (rc) { batch_free_dev(b); delete b; return rc; }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, long n)
{
    if (!b || n < 0) return fail(LBM_EINVAL, "bad arguments");
    bool stale = false;
    for (size_t i = 0; i < b->mem.size(); ++i)
        stale = stale || b->mem[i]->version != b->ver0[i] || (b->mem[i]->phase ^ b->phase) != b->phase0[i];
    if (stale) {
        int rc = batch_build(b);
        if (rc) return rc;
    }
    bool fft = false;   // hipFFT runs outside graphs
    for (const LaunchGroup& g : b->groups) fft = fft || g.fprog;
    // the members' step counts and phases follow the steps actually
    // enqueued, also when a launch or a capture fails part way
    long done = 0;
    int rc = LBM_OK;
    while (done < n && !rc) {
        // chunks of gchunk steps, then the even part of the rest, replayed
        // from captured graphs; a last odd step launches eagerly
        const long left = n - done;
        const long len = fft ? 0 : (left >= b->gchunk ? b->gchunk : (left & ~1L));
        if (len >= 2) {
            const int ph = b->phase;
            auto it = b->gexec[ph].find((int)len);
            if (it == b->gexec[ph].end()) {
                hipGraphExec_t g = nullptr;
                rc = capture(b->stream, b->groups, (int)len, ph, &g);
                if (rc) break;
                it = b->gexec[ph].emplace((int)len, g).first;
            }
            const hipError_t e = hipGraphLaunch(it->second, b->stream);
            if (e != hipSuccess) { rc = fail(LBM_EDEVICE, "graph launch failed: %s", hipGetErrorString(e)); break; }
            done += len;
        } else {
            for (const LaunchGroup& g : b->groups) launch_step(g, b->stream, b->phase);
            b->phase ^= 1;
            done += 1;
        }
    }
    const hipError_t le = hipGetLastError();
    if (!rc && le != hipSuccess) rc = fail(LBM_EDEVICE, "launch failed: %s", hipGetErrorString(le));
    for (lbm_ctx* c : b->mem) rc = rc ? rc : fft_status(c);
    for (lbm_ctx* c : b->mem) {
        c->host_step += done;
        c->phase ^= (int)(done & 1);
        if (done > 0 && c->defers()) c->pending = true;
    }
    return rc;
}

int lbm_batch_sync(lbm_batch* b)
{
    if (!b) return fail(LBM_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(b->stream));
    int rc = LBM_OK;
    for (lbm_ctx* c : b->mem) {
        int r = lbm_sync(c);
        if (r && !rc) rc = r;
    }
    return rc;
}

void lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    batch_free_dev(b);
    delete b;
}

// Per-phase timing: nsteps eager steps with events at the phase boundaries,
// on the context stream.  ms[k] is the mean duration of phase k per step
// (stream-collide, curl, binomial powers, reduce, solve, apply); launches[k]
// the number of kernel launches of phase k per step.
int lbm_profile_phases(lbm_ctx* c, long nsteps, double* ms, int* launches)
{
    if (!c || nsteps < 1 || !ms) return fail(LBM_EINVAL, "bad arguments");
    hipEvent_t ev[kNumPhases + 1];
    for (int k = 0; k <= kNumPhases; ++k) HIPCHK(hipEventCreate(&ev[k]));
    double acc[kNumPhases] = {0, 0, 0, 0, 0, 0};
    const LaunchGroup g = ctx_group(c);
    int rc = LBM_OK;
    if (c->defers()) c->pending = true;
    for (long s = 0; s < nsteps && !rc; ++s) {
        launch_step(g, c->stream, c->phase, ev);
        c->phase ^= 1;
        c->host_step += 1;
        if (hipEventSynchronize(ev[kNumPhases]) != hipSuccess) { rc = fail(LBM_EDEVICE, "event sync failed"); break; }
        for (int k = 0; k < kNumPhases; ++k) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess) { rc = fail(LBM_EDEVICE, "event timing failed"); break; }
            acc[k] += t;
        }
    }
    for (int k = 0; k <= kNumPhases; ++k) (void)hipEventDestroy(ev[k]);
    for (int k = 0; k < kNumPhases; ++k) ms[k] = acc[k] / nsteps;
    if (launches) {
        const int m = g.mode;
        launches[0] = 1 + (g.substrate == LBM_WALE ? 1 : 0);
        launches[1] = m == 2 && g.kf && g.any_z ? 1 : 0;
        launches[2] = m == 2 ? (g.kf ? g.nklev : g.npass) : 0;
        launches[3] = m == 2 ? 1 : 0;
        launches[4] = m == 2 ? (fused_solve(g) ? 1 : 2) : 0;   // cross-block sums, solve (unless the apply forms it)
        launches[5] = m == 2 ? 1 : (m == 1 ? 2 : 0);
    }
    return rc;
}

// Test hooks for the random-number generator (not part of the stepping path).
int lbm_test_philox(const uint32_t* in6, uint32_t* out4, int n)
{
    uint32_t *din = nullptr, *dout = nullptr;
    HIPCHK(hipMalloc(&din, sizeof(uint32_t) * 6 * n));
    HIPCHK(hipMalloc(&dout, sizeof(uint32_t) * 4 * n));
    HIPCHK(hipMemcpy(din, in6, sizeof(uint32_t) * 6 * n, hipMemcpyHostToDevice));
    launch_philox_test(din, dout, n, nullptr);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(out4, dout, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost));
    (void)hipFree(din);
    (void)hipFree(dout);
    return LBM_OK;
}

int lbm_test_normals(uint64_t seed, long step0, int nsteps, int n, double* out)
{
    if (n < 1 || n > LBM_MAX_QOI || nsteps < 1) return fail(LBM_EINVAL, "bad arguments");
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(double) * (size_t)nsteps * n));
    launch_normals_test(seed, step0, nsteps, n, d, nullptr);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(out, d, sizeof(double) * (size_t)nsteps * n, hipMemcpyDeviceToHost));
    (void)hipFree(d);
    return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching of LES requests.
// ---------------------------------------------------------------------------
namespace {

double server_clock_now()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Deep copy of a closure (the lbm_closure points into caller memory).
struct ClosureCopy {
    bool set = false;
    lbm_closure c{};
    std::vector<lbm_qoi_spec> q;
    std::vector<double> C, mu, Sigma, scale, qref;
    void take(const lbm_closure* src)
    {
        if (!src) { set = false; return; }
        set = true;
        c = *src;
        const int nq = src->nq;
        q.assign(src->q, src->q + nq);
        c.q = q.data();
        auto cp = [](const double* p, size_t n, std::vector<double>& v) -> const double* {
            if (!p) return nullptr;
            v.assign(p, p + n);
            return v.data();
        };
        // ((2h+1) nq + 1) x nq for a history model (out-of-range h is
        // rejected later by the closure checks; copy the h = 0 shape then)
        const int h = src->h >= 0 && src->h <= LBM_MAX_HIST ? src->h : 0;
        c.C = cp(src->C, ((size_t)(2 * h + 1) * nq + 1) * nq, C);
        c.mu = cp(src->mu, nq, mu);
        c.Sigma = cp(src->Sigma, (size_t)nq * nq, Sigma);
        c.scale = cp(src->scale, nq, scale);
        c.qref = cp(src->qref, src->nref > 0 ? (size_t)src->nref * nq : 0, qref);
    }
    const lbm_closure* get() const { return set ? &c : nullptr; }
};

struct ServeReq {
    long id = 0;
    lbm_config cfg{};
    ClosureCopy cl;
    std::vector<double> u0;
    long nsteps = 0, done = 0;
    double t_arr = 0, t_adm = 0, t_done = 0;
    int keep = 0;
    size_t bytes = 0;
    void* arena = nullptr;
    lbm_ctx* ctx = nullptr;
};

}  // namespace

// The server steps its active requests as one batch on its stream, one chunk
// in flight at a time: while the device runs a chunk, the host admits newly
// arrived requests (their contexts are created and initialised on a second,
// admission stream, then handed to the server stream), and only then waits
// for the chunk, retires finished requests and enqueues the next chunk.
// Arenas come from a pool keyed by size: a retired request's arena is kept
// for the next request of the same size, so steady serving allocates
// nothing; cached arenas count against the budget and are released when a
// request of another size needs the room.
struct lbm_server {
    hipStream_t stream = nullptr, adm = nullptr;
    bool own_stream = false;
    size_t budget = 0, used = 0, cached = 0;
    long next_id = 1;
    std::deque<ServeReq*> queue;
    std::vector<ServeReq*> active;
    lbm_batch* batch = nullptr;
    bool dirty = true;
    std::vector<lbm_result> results;
    std::map<long, std::vector<char>> states;
    std::multimap<size_t, void*> pool;   // free arenas by size
    double* stage = nullptr;             // device staging of initial velocities
    size_t stage_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool inflight = false;               // a chunk is enqueued and not yet accounted
    long inflight_chunk = 0;
    std::vector<ServeReq*> inflight_reqs;
    long chunk_default = 64;
    double busy = 0;   // device seconds spent stepping (events around each chunk)
    double lups = 0;   // lattice updates done
};

namespace {

void* pool_take(lbm_server* s, size_t bytes)
{
    auto it = s->pool.find(bytes);
    if (it != s->pool.end()) {
        void* p = it->second;
        s->pool.erase(it);
        s->cached -= bytes;
        return p;
    }
    while (!s->pool.empty() && s->used + s->cached + bytes > s->budget) {
        auto big = std::prev(s->pool.end());
        (void)hipFree(big->second);
        s->cached -= big->first;
        s->pool.erase(big);
    }
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void pool_put(lbm_server* s, void* p, size_t bytes)
{
    s->pool.emplace(bytes, p);
    s->cached += bytes;
}

void server_release(lbm_server* s, ServeReq* r)
{
    if (r->ctx) lbm_destroy(r->ctx);
    if (r->arena) pool_put(s, r->arena, r->bytes);
    s->used -= r->bytes;
    delete r;
}

void server_post(lbm_server* s, const ServeReq* r, int status, double now)
{
    lbm_result res{};
    res.id = r->id;
    res.status = status;
    res.t_arrival = r->t_arr;
    res.t_admit = now;
    res.t_done = now;
    res.cells = (long)r->cfg.nx * r->cfg.ny * r->cfg.nz;
    s->results.push_back(res);
}

// A request's context on the admission stream: arena from the pool, the
// closure, the initial state from the staged velocity; then its stream is
// the server's.
int server_start(lbm_server* s, ServeReq* r)
{
    r->arena = pool_take(s, r->bytes);
    if (!r->arena) return fail(LBM_ENOMEM, "server: arena allocation failed");
    int rc = lbm_create(&r->cfg, r->cl.get(), r->arena, r->bytes, s->adm, &r->ctx);
    if (!rc) {
        const size_t need = sizeof(double) * r->u0.size();
        if (need > s->stage_bytes) {
            HIPCHK(hipStreamSynchronize(s->adm));
            if (s->stage) (void)hipFree(s->stage);
            s->stage = nullptr;
            s->stage_bytes = 0;
            if (hipMalloc(&s->stage, need) != hipSuccess) rc = fail(LBM_ENOMEM, "server: staging allocation failed");
            else s->stage_bytes = need;
        }
        if (!rc && hipMemcpyAsync(s->stage, r->u0.data(), need, hipMemcpyHostToDevice, s->adm) != hipSuccess)
            rc = fail(LBM_EDEVICE, "server: initial state upload failed");
        if (!rc) rc = init_from_device(r->ctx, nullptr, s->stage);
    }
    if (rc) {
        if (r->ctx) lbm_destroy(r->ctx);
        r->ctx = nullptr;
        pool_put(s, r->arena, r->bytes);
        r->arena = nullptr;
        return rc;
    }
    r->ctx->stream = s->stream;
    std::vector<double>().swap(r->u0);
    return LBM_OK;
}

int server_admit(lbm_server* s, double now)
{
    while (!s->queue.empty()) {
        ServeReq* r = s->queue.front();
        if (r->t_arr > now) break;
        if (s->used + r->bytes > s->budget && !s->active.empty()) break;  // wait for memory
        s->queue.pop_front();
        // larger than the whole budget, or failing to start: a result with
        // its status, and admission goes on
        int rc = s->used + r->bytes > s->budget ? fail(LBM_ENOMEM, "server: request %ld exceeds the budget", r->id)
                                                : server_start(s, r);
        if (rc) {
            server_post(s, r, rc, now);
            delete r;
            continue;
        }
        s->used += r->bytes;
        r->t_adm = server_clock_now();
        s->active.push_back(r);
        s->dirty = true;
    }
    return LBM_OK;
}

int server_retire(lbm_server* s)
{
    std::vector<ServeReq*> keep;
    for (ServeReq* r : s->active) {
        if (r->done < r->nsteps) { keep.push_back(r); continue; }
        lbm_result res{};
        res.id = r->id;
        res.status = lbm_sync(r->ctx);
        res.steps = r->done;
        res.t_arrival = r->t_arr;
        res.t_admit = r->t_adm;
        res.t_done = r->t_done;
        res.cells = (long)r->cfg.nx * r->cfg.ny * r->cfg.nz;
        if (r->ctx->mode() > 0 && r->done > 0) lbm_qoi(r->ctx, r->done - 1, 1, &res.last);
        if (r->keep) {
            std::vector<char> img(lbm_state_bytes(r->ctx));
            if (lbm_get_state(r->ctx, img.data(), img.size()) == LBM_OK) s->states[r->id] = std::move(img);
        }
        s->results.push_back(res);
        server_release(s, r);
        s->dirty = true;
    }
    s->active.swap(keep);
    return LBM_OK;
}

// Account and retire the chunk in flight (waits for it).
// A batch that cannot be built or stepped: every active request is retired
// with that status (its state is no longer consistent with its step count),
// so that later calls serve the queue instead of retrying it.
void server_fail_active(lbm_server* s, int status)
{
    const double now = server_clock_now();
    if (s->batch) lbm_batch_destroy(s->batch);
    s->batch = nullptr;
    for (ServeReq* r : s->active) {
        server_post(s, r, status, now);
        server_release(s, r);
    }
    s->active.clear();
    s->dirty = true;
}

int server_finish_chunk(lbm_server* s)
{
    if (!s->inflight) return LBM_OK;
    HIPCHK(hipEventSynchronize(s->ev1));
    float ms = 0;
    if (hipEventElapsedTime(&ms, s->ev0, s->ev1) == hipSuccess) s->busy += ms * 1e-3;
    const double t1 = server_clock_now();
    for (ServeReq* r : s->inflight_reqs) {
        r->done += s->inflight_chunk;
        s->lups += (double)s->inflight_chunk * r->cfg.nx * r->cfg.ny * r->cfg.nz;
        if (r->done >= r->nsteps) r->t_done = t1;
    }
    s->inflight = false;
    s->inflight_reqs.clear();
    return server_retire(s);
}

// Validation of a request's closure that its creation would otherwise meet
// only at admission: an SPD Sigma (LRS) and a spin-up that covers the
// history (a request starts at step 0).
int check_request_closure(const lbm_closure* cl)
{
    if (!cl) return LBM_OK;
    if (cl->mode == LBM_CLOSURE_LRS) {
        double L[LBM_MAX_QOI * LBM_MAX_QOI];
        if (!cl->Sigma || !cholesky_host(cl->Sigma, cl->nq, L, LBM_MAX_QOI))
            return fail(LBM_EINVAL, "server: closure Sigma is not SPD");
    }
    if (cl->h > 0 && cl->spinup < cl->h)
        return fail(LBM_EINVAL, "server: closure spinup must be at least the history length");
    return LBM_OK;
}

}  // namespace

extern "C" {

double lbm_server_clock(void) { return server_clock_now(); }

int lbm_server_create(size_t hbm_budget, void* stream, lbm_server** out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    lbm_server* s = new lbm_server();
    s->stream = (hipStream_t)stream;
    const char* what = nullptr;
    hipError_t e = hipSuccess;
    if (!s->stream) {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        s->own_stream = e == hipSuccess;
        if (e != hipSuccess) what = "stream creation";
    }
    if (!what && (e = hipStreamCreateWithFlags(&s->adm, hipStreamNonBlocking)) != hipSuccess) what = "admission stream creation";
    if (!what && (e = hipEventCreate(&s->ev0)) != hipSuccess) what = "event creation";
    if (!what && (e = hipEventCreate(&s->ev1)) != hipSuccess) what = "event creation";
    if (!what && hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) what = "memory query";
        hbm_budget = (size_t)(0.8 * (double)fr);
    }
    if (what) {
        if (s->ev0) (void)hipEventDestroy(s->ev0);
        if (s->ev1) (void)hipEventDestroy(s->ev1);
        if (s->adm) (void)hipStreamDestroy(s->adm);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(LBM_EDEVICE, "server: %s failed (%s)", what, hipGetErrorString(e));
    }
    s->budget = hbm_budget;
    *out = s;
    return LBM_OK;
}

int lbm_server_submit(lbm_server* s, const lbm_config* cfg, const lbm_closure* cl, const double* u0, long nsteps,
                      double t_arrival, int keep_state, long* id)
{
    if (!s || !cfg || !u0 || nsteps < 1) return fail(LBM_EINVAL, "bad arguments");
    const size_t bytes = lbm_required_bytes(cfg, cl);
    if (!bytes) return LBM_EINVAL;  // message set by the validation
    int rc = check_request_closure(cl);
    if (rc) return rc;
    ServeReq* r = new ServeReq();
    r->id = s->next_id++;
    r->cfg = *cfg;
    r->cl.take(cl);
    const size_t n = (size_t)(cfg->lattice == LBM_D2Q9 ? 2 : 3) * cfg->nx * cfg->ny * cfg->nz;
    r->u0.assign(u0, u0 + n);
    r->nsteps = nsteps;
    r->t_arr = t_arrival;
    r->keep = keep_state;
    r->bytes = align_up(bytes);
    // keep the queue ordered by arrival time
    auto it = s->queue.end();
    while (it != s->queue.begin() && (*(it - 1))->t_arr > t_arrival) --it;
    s->queue.insert(it, r);
    if (id) *id = r->id;
    return LBM_OK;
}

int lbm_server_advance(lbm_server* s, double now, long max_chunk, int* n_active)
{
    if (!s) return fail(LBM_EINVAL, "NULL server");
    // admission overlaps the chunk in flight
    int rc = server_admit(s, now);
    if (rc) return rc;
    rc = server_finish_chunk(s);
    if (rc) return rc;
    if (n_active) *n_active = (int)s->active.size();
    if (s->active.empty()) return LBM_OK;
    long chunk = max_chunk > 0 ? max_chunk : s->chunk_default;
    for (ServeReq* r : s->active) chunk = std::min(chunk, r->nsteps - r->done);
    if (s->dirty) {
        if (s->batch) lbm_batch_destroy(s->batch);
        s->batch = nullptr;
        std::vector<lbm_ctx*> m;
        for (ServeReq* r : s->active) m.push_back(r->ctx);
        rc = lbm_batch_create((int)m.size(), m.data(), &s->batch);
        if (rc) {
            server_fail_active(s, rc);
            return rc;
        }
        s->dirty = false;
    }
    HIPCHK(hipEventRecord(s->ev0, s->stream));
    rc = lbm_batch_step(s->batch, chunk);
    if (rc) {
        (void)hipStreamSynchronize(s->stream);
        server_fail_active(s, rc);
        return rc;
    }
    HIPCHK(hipEventRecord(s->ev1, s->stream));
    s->inflight = true;
    s->inflight_chunk = chunk;
    s->inflight_reqs = s->active;
    return LBM_OK;
}

int lbm_server_poll(lbm_server* s, lbm_result* out, int cap, int* n)
{
    if (!s || !n || (cap > 0 && !out)) return fail(LBM_EINVAL, "bad arguments");
    const int k = std::min<int>(cap, (int)s->results.size());
    for (int i = 0; i < k; ++i) out[i] = s->results[i];
    s->results.erase(s->results.begin(), s->results.begin() + k);
    *n = k;
    return LBM_OK;
}

int lbm_server_pending(const lbm_server* s) { return s ? (int)(s->queue.size() + s->active.size()) : -1; }

int lbm_server_stats(const lbm_server* s, double* busy_s, double* lups, size_t* used, size_t* budget)
{
    if (!s) return fail(LBM_EINVAL, "NULL server");
    if (busy_s) *busy_s = s->busy;
    if (lups) *lups = s->lups;
    if (used) *used = s->used;
    if (budget) *budget = s->budget;
    return LBM_OK;
}

size_t lbm_server_state_bytes(const lbm_server* s, long id)
{
    if (!s) return 0;
    auto it = s->states.find(id);
    return it == s->states.end() ? 0 : it->second.size();
}

int lbm_server_take_state(lbm_server* s, long id, void* host, size_t bytes)
{
    if (!s || !host) return fail(LBM_EINVAL, "bad arguments");
    auto it = s->states.find(id);
    if (it == s->states.end()) return fail(LBM_ESTATE, "no retained state for request %ld", id);
    if (bytes < it->second.size()) return fail(LBM_EINVAL, "buffer too small");
    memcpy(host, it->second.data(), it->second.size());
    s->states.erase(it);
    return LBM_OK;
}

void lbm_server_destroy(lbm_server* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->adm);
    if (s->batch) lbm_batch_destroy(s->batch);
    for (ServeReq* r : s->active) server_release(s, r);
    for (ServeReq* r : s->queue) delete r;
    for (auto& kv : s->pool) (void)hipFree(kv.second);
    if (s->stage) (void)hipFree(s->stage);
    (void)hipEventDestroy(s->ev0);
    (void)hipEventDestroy(s->ev1);
    (void)hipStreamDestroy(s->adm);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"

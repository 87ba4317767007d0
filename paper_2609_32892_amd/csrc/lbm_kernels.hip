// lbm_kernels.hip -- HIP kernels of the TO-LRS lattice Boltzmann LES step for
// gfx950 (MI355X).
//
// Populations are stored in blocks of kPopBlk cells (x-fastest cell order),
// each block holding its Q populations one after another, in two ping-pong
// buffers; the other fields are [component][N].  One step (eqs. LES-1..LES-3
// with the TO correction):
//   k_step     pull-stream with halfway bounce-back (eq. LES-3, Sec. 7.1),
//              moments, effective relaxation time (Sec. 5), BGK relaxation and
//              exact-difference forcing (eq. LES-1/LES-2); writes the
//              predictor populations and rho, v* = v^{p,n*}.
//   k_step_t   the same on 2.5-D tiles, adding during the pull the SGS change
//              the previous step recorded per cell (grids whose populations
//              exceed the L2s).
//   k_binom1   first powers of the binomial filter (Sec. 4.1): w = curl v*,
//              B v*, B w and curl^T w from v* staged with a two-cell halo.
//   k_binom    further powers B^j v*, B^j w and curl^T B^(j-1) w.
//   k_reduce   per-cell QoIs, sensitivities (App. A) and Gram products,
//              reduced per workgroup in FP64.
//   k_sum      fixed-order cross-workgroup sums; the step's LRS draw.
//   k_solve    one workgroup per member: dQ (tracking or LRS, eqs.
//              dQ-from-ref, LRS), Gram solve (eq. O-from-V, eq.
//              orthogonality), gamma (eq. tau-from-dQ-for-tracking).
//   k_apply    dv_SGS = sum_i gamma_i O_i (eq. TO-ansatz), evaluated as
//              sum_j beta_j V_j with beta = G^-1 dQ; its change of the
//              equilibrium is added to the predictor populations in place, or
//              recorded as (rho dv, 2 v* + dv) for the next k_step_t (k_flush
//              applies pending records before the state is read).
//   k_apply_fs the same with the member's solve at its head, in every
//              workgroup (small launches: no k_solve launch).
// Every kernel takes a table of members and a work table mapping each
// workgroup to (member, local block), so one launch serves a whole ensemble.
// All reductions have a fixed order that depends only on the member's own
// geometry, so a member gives bitwise the same result alone or in a batch.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <math.h>

#include <type_traits>

#include "lbm_dev.h"
#include "lbm_launch.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Lattices (Sec. 2).  Opposite of i >= 1 is i + 1 for odd i, i - 1 for even i.
// ---------------------------------------------------------------------------
template <int LAT> struct Lat;
template <> struct Lat<LBM_D2Q9> {
    static constexpr int Q = 9, D = 2, NC = 1;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
template <> struct Lat<LBM_D3Q19> {
    static constexpr int Q = 19, D = 3, NC = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36};
};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
__device__ __forceinline__ int modi(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

// ---------------------------------------------------------------------------
// Reductions over the 64-lane wavefront with DPP lane moves (no LDS
// traffic): pairs, quads, half rows and rows of 16 lanes by quad
// permutations and mirrors, then the rows by the two row broadcasts, which
// leaves the sum in lane 63.  The order of the additions is fixed.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double v)
{
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if (ROWMASK == 0xf) {   // every lane is written
        lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    } else {                // rows outside the mask add zero
        lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    }
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v = dpp_add<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);   // row_mirror
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum NV values over the workgroup of NW wavefronts; result valid in
// thread 0.  Uses NV * NW doubles of LDS.
template <int NV, int NW = kBlock / 64>
__device__ __forceinline__ void block_sum(double* v, double* lds)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[k * NW + wv] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0;
#pragma unroll
            for (int j = 0; j < NW; ++j) s += lds[k * NW + j];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Global accesses at an element index below 2^32 / sizeof(T) from a
// workgroup-uniform base: the byte offset is formed in 32 bits, so the access
// uses a scalar base plus one 32-bit vector offset (no 64-bit address per
// lane).  The library rejects grids whose fields would not fit.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, unsigned i)
{
    return *(const T*)((const char*)base + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned i, T v)
{
    *(T*)((char*)base + i * (unsigned)sizeof(T)) = v;
}

// Element index of population i of cell c in the blocked population layout
// ([block][Q][kPopBlk]): a wavefront's loads of one population stay within
// one block, and the Q arrays a cell touches sit next to each other, which
// the memory system serves faster than Q separate full-length streams.  The
// 32-bit form needs Q * ceil(N / kPopBlk) * kPopBlk elements below 2^32 bytes.
template <int Q>
__device__ __forceinline__ unsigned pop_at(int i, unsigned c)
{
    return (((c >> kPopLog) * Q + (unsigned)i) << kPopLog) | (c & (kPopBlk - 1));
}
template <int Q>
__device__ __forceinline__ size_t pop_at64(int i, size_t c)
{
    return (((c >> kPopLog) * Q + (size_t)i) << kPopLog) | (c & (kPopBlk - 1));
}

// Stores of fields that the next kernel reads.  On small grids (kernels
// instantiated with WT) they are relaxed device-scope atomic stores, written
// through each XCD's L2, so that no dirty lines are left for the L2
// write-back at the end of the kernel, which the next kernel waits for.
// Measured on MI355X (FP32 channel TO-LES): 2427 -> 2592 MLUPS on
// 96 x 48 x 48; no change on 384 x 192 x 192; but 1328 -> 1130 MLUPS for
// the kernel-filter closure on 295 x 47 x 98, whose fields the next kernel
// otherwise finds in the Infinity Cache.  Larger launches store
// non-temporally (5228 -> 5310..5321 MLUPS on 384 x 192 x 192; no change on
// 295 x 47 x 98): the stream-collide itself slows (457 -> 485 us), but its
// populations then no longer push the TO fields out of the Infinity Cache
// (binomial pass 209 -> 203 us, reduce 453 -> 424 us, curl 86 -> 79 us).
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_fld(T* p, T v, int wt)
{
    if (wt) st_dev(p, v);
    else __builtin_nontemporal_store(v, p);
}
// Loads of fields whose last reader in the step is the loading kernel: on
// launches without write-through, non-temporal (the apply's chain fields and
// populations: 5325 -> 5448 MLUPS on 384 x 192 x 192; 0.6% slower on
// 96 x 48 x 48, hence plain there).
template <bool WT, typename T>
__device__ __forceinline__ T ld_fld(const T* p)
{
    if constexpr (WT) return *p;
    else return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_fld_at(T* base, unsigned i, T v, int wt)
{
    st_fld((T*)((char*)base + i * (unsigned)sizeof(T)), v, wt);
}

// Butterfly reduce-scatter over the wavefront: at lane distance D each lane
// keeps one half of its list of L partial sums (the lower half where lane
// bit D is clear, else the upper half, padded with a zero when L is odd)
// and adds its partner's copy of that half.  A level costs ceil(L/2)
// exchanges; after distances 32 .. 1 every lane holds one wave sum.  Returns
// that sum's index in the list (-1 for a lane left holding padding, which
// includes the upper lanes of every level with L = 1).  The order of the
// additions is fixed.
template <int L, int D>
__device__ __forceinline__ int wave_scatter(double* cur, int lane)
{
    constexpr int H = (L + 1) / 2;
    const bool hi = (lane & D) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double lo_v = cur[i];
        const double hi_v = H + i < L ? cur[H + i] : 0.0;
        const double give = hi ? lo_v : hi_v;
        cur[i] = (hi ? hi_v : lo_v) + __shfl_xor(give, D);
    }
    int p = 0;
    if constexpr (D > 1) p = wave_scatter<H, D / 2>(cur, lane);
    if (p < 0) return -1;
    p += hi ? H : 0;
    return p < L ? p : -1;
}

// The sums of block_sum with the result spread over the workgroup: thread
// k < NV returns value k, the waves' sums added in wave order.
template <int NV>
__device__ __forceinline__ double block_sum_spread(const double* v, double* lds)
{
    static_assert(NV <= 64, "one value per lane after the butterfly");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double cur[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) cur[k] = v[k];
    const int idx = wave_scatter<NV, 32>(cur, lane);
    if (idx >= 0) lds[idx * (kBlock / 64) + wv] = cur[0];
    __syncthreads();
    double r = 0;
    if (threadIdx.x < NV) {
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) r += lds[threadIdx.x * (kBlock / 64) + j];
    }
    return r;
}

// feq_i(rho, a) - feq_i(rho, b) in difference form (exactly zero when a = b):
// w rho [3 c.(a-b) + 9/2 (c.(a-b))(c.(a+b)) - 3/2 (a-b).(a+b)].
template <typename T>
__device__ __forceinline__ T dfeq(T w, T rho, T cd, T cs, T dd)
{
    return w * rho * (T(3) * cd + T(4.5) * cd * cs - T(1.5) * dd);
}

// ---------------------------------------------------------------------------
// SGS change of the post-collision populations of a cell (eq. LES-2, the
// second difference of the exact-difference form): with a = rho dv,
// b = 2 v* + dv and e = a.b,
//   delta f_i = feq_i(rho, v* + dv) - feq_i(rho, v*)
//             = w_i [3 c_i.a + 9/2 (c_i.a)(c_i.b) - 3/2 e].
// k_apply stores the record (a, b) of every cell; the next stream-collide
// adds delta f of each source cell while it pulls (k_step_t), or k_flush adds
// it in place before the state is read.  Both evaluate it with these
// functions, without contraction and in a fixed order, so a flushed state
// streams to bitwise the populations the deferred pull forms.
// ---------------------------------------------------------------------------
// c_i . a over the nonzero components of c_i (exact signs, no products with
// the constants); A(k) returns component k.
template <int LAT, typename T, typename Get>
__device__ __forceinline__ T cdot(int i, Get A)
{
    // (no contraction: where a component is itself a product, as rho dv in
    // the in-place apply, a fused multiply-add would round differently from
    // the same sum over stored records)
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    const int c[3] = {L::cx[i], L::cy[i], L::D == 3 ? L::cz[i] : 0};
    T s = T(0);
    bool any = false;
#pragma unroll
    for (int k = 0; k < L::D; ++k) {
        if (!c[k]) continue;
        const T v = A(k);
        if (!any) s = c[k] > 0 ? v : -v;
        else s = c[k] > 0 ? s + v : s - v;
        any = true;
    }
    return s;
}

// e = a.b in a fixed order.
template <int D, typename T>
__device__ __forceinline__ T rec_e(const T* a, const T* b)
{
#pragma clang fp contract(off)
    T e = a[0] * b[0];
#pragma unroll
    for (int k = 1; k < D; ++k) e = e + a[k] * b[k];
    return e;
}

// delta f_i from the record (a, b, e) of the cell, with ca = c_i.a and
// cb = c_i.b; opp: delta f of the opposite direction instead, whose c.a and
// c.b are exactly -ca and -cb (rounding is symmetric in sign), so only the
// linear term changes sign.  g + delta f is then one rounded addition.
template <int LAT, typename T>
__device__ __forceinline__ T df_cc(int i, bool opp_dir, T ca, T cb, T e)
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    const T lin = T(3) * ca;
    const T s = ((opp_dir ? -lin : lin) + (T(4.5) * ca) * cb) - T(1.5) * e;
    return T(L::w[i]) * s;
}
template <int LAT, typename T, typename GA, typename GB>
__device__ __forceinline__ T df_of(int i, GA A, GB B, T e)
{
    return df_cc<LAT, T>(i, false, cdot<LAT, T>(i, A), cdot<LAT, T>(i, B), e);
}
template <typename T>
__device__ __forceinline__ T add_rn(T g, T d)
{
#pragma clang fp contract(off)
    return g + d;
}
template <int LAT, typename T, typename GA, typename GB>
__device__ __forceinline__ T add_df(T g, int i, GA A, GB B, T e)
{
    return add_rn(g, df_of<LAT, T>(i, A, B, e));
}

// ---------------------------------------------------------------------------
// Pull gather of the post-collision populations of cell (x,y,z).  A32: the
// run keeps 2 N * sizeof(T) below 4 GiB (every TO run does), so each load is
// a 32-bit offset from a scalar base.
// ---------------------------------------------------------------------------
template <int LAT, typename T, bool A32, bool FAST = true>
__device__ __forceinline__ void gather(KMember& m, const T* __restrict__ gs, int x, int y, int z,
                                       int cell, T* f)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q, D = L::D;
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    // Wavefronts whose cells are all at least one cell from the walls and
    // from the z wrap pull from constant offsets, corrected per cell for the
    // periodic x wrap; the others resolve wrap and bounce-back per population.
    const bool inner = y > 0 && y < ny - 1 && (D == 2 || (z > 0 && z < nz - 1));
    if (FAST && __all(inner)) {
        const int wxm = x == 0 ? nx : 0, wxp = x == nx - 1 ? -nx : 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int off = L::cx[i] + nx * (L::cy[i] + (D == 3 ? ny * L::cz[i] : 0));
            const int src = cell - off + (L::cx[i] == 1 ? wxm : L::cx[i] == -1 ? wxp : 0);
            if (A32)
                f[i] = ld_at(gs, pop_at<Q>(i, (unsigned)src));
            else
                f[i] = gs[pop_at64<Q>(i, (size_t)src)];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int sy = y - L::cy[i];
        int src, pi;
        bool bb = m.walls && (sy < 0 || sy >= ny);
        if (bb) {
            src = cell;
            pi = opp(i);
        } else {
            int sx = wrapi(x - L::cx[i], nx);
            sy = wrapi(sy, ny);
            int sz = D == 3 ? wrapi(z - L::cz[i], nz) : 0;
            src = sx + nx * (sy + ny * sz);
            pi = i;
        }
        if (A32)
            f[i] = ld_at(gs, pop_at<Q>(pi, (unsigned)src));
        else
            f[i] = gs[pop_at64<Q>(pi, (size_t)src)];
    }
}

// Moments: rho - 1 and rho u from gathered populations.
template <int LAT, typename T, int PREC>
__device__ __forceinline__ void moments(const T* f, T& drho, T* j)
{
    using L = Lat<LAT>;
    drho = 0;
#pragma unroll
    for (int a = 0; a < L::D; ++a) j[a] = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        drho += f[i];
        if (L::cx[i]) j[0] += T(L::cx[i]) * f[i];
        if (L::cy[i]) j[1] += T(L::cy[i]) * f[i];
        if (L::D == 3 && L::cz[i]) j[2] += T(L::cz[i]) * f[i];
    }
    if (PREC == LBM_FP32_PLAIN) drho -= T(1);
}

// ---------------------------------------------------------------------------
// K1: stream + collide + force.
// MODE 0: plain; 1: plain with statistics and post-streaming velocity;
// 2: TO predictor (statistics, rho, v*).
// ---------------------------------------------------------------------------
// Collision of one cell from its pulled populations f: moments, effective
// relaxation time (Sec. 5), BGK relaxation with the exact-difference force
// (eq. LES-1/LES-2); stores the predictor populations (and in TO mode rho - 1
// and v*), adds the cell's mass and momentum to st and flags instability.
// Shifted storage (FP32 and FP64): the non-equilibrium parts f_i - feq_i have
// zero mass and momentum by definition (u = j / rho), but their rounded
// values do not -- rho u differs from j after rounding, and the equilibria
// are rounded one by one -- and in a quasi-steady flow that rounding repeats
// each step, so relaxation alone would drift the mean flow (measured in FP32
// on the 20 x 24 x 12 channel: +4.5e-5 relative x-momentum after 2500 steps,
// against 3e-8 when only the stored populations are rounded).  The mass and
// momentum the rounding leaves in them are projected out (subtracting
// w_i (s + 3 c_i . sigma) removes a mass s and a momentum sigma), and each
// population is updated as f_i + (force term - omega (f_i - feq_i)), one
// rounding at its own magnitude.  Plain FP32 storage keeps the direct form
// as the baseline.
template <int LAT, typename T, int PREC, int SUB, int MODE, bool WT, bool A32 = MODE == 2, bool NT = false>
__device__ __forceinline__ void collide_cell(KMember& m, T* f, int x, int y, int z, int cell, T* __restrict__ gd,
                                             double* st, int& bad)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q, D = L::D;
    constexpr bool PROJ = PREC != LBM_FP32_PLAIN;
    const int N = m.N, nx = m.nx, ny = m.ny;
    T drho, j[3] = {0, 0, 0};
    moments<LAT, T, PREC>(f, drho, j);
    const T rho = T(1) + drho;
    const T ir = T(1) / rho;
    T u[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = j[a] * ir;
    T uu = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) uu += u[a] * u[a];
    if (!(uu <= T(0.25))) bad = 1;

    // non-equilibrium parts fn_i = f_i - feq_i (feq_i - w_i against shifted
    // populations)
    T fn[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T cu = T(L::cx[i]) * u[0] + T(L::cy[i]) * u[1] + (D == 3 ? T(L::cz[i]) * u[2] : T(0));
        const T X = T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu;
        const T geq = PREC == LBM_FP32_PLAIN ? T(L::w[i]) * rho * (T(1) + X) : T(L::w[i]) * (drho + rho * X);
        fn[i] = f[i] - geq;
    }
    if constexpr (PROJ) {
        T sm = 0, sj[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            sm += fn[i];
            if (L::cx[i]) sj[0] += T(L::cx[i]) * fn[i];
            if (L::cy[i]) sj[1] += T(L::cy[i]) * fn[i];
            if (L::D == 3 && L::cz[i]) sj[2] += T(L::cz[i]) * fn[i];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T cs = T(L::cx[i]) * sj[0] + T(L::cy[i]) * sj[1] + (D == 3 ? T(L::cz[i]) * sj[2] : T(0));
            fn[i] -= T(L::w[i]) * (sm + T(3) * cs);
        }
    }

    // effective relaxation time (Sec. 5)
    T taue = T(m.tau);
    if constexpr (SUB == LBM_SMAGORINSKY) {
        T P[6] = {0, 0, 0, 0, 0, 0};  // xx yy zz xy xz yz
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T v = fn[i];
            const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
            if (cx) P[0] += v;
            if (cy) P[1] += v;
            if (cz) P[2] += v;
            if (cx * cy) P[3] += T(cx * cy) * v;
            if (cx * cz) P[4] += T(cx * cz) * v;
            if (cy * cz) P[5] += T(cy * cz) * v;
        }
        const T PP = P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + T(2) * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]);
        const T nP = sqrt(T(2) * PP);
        const T cm = T(m.cmodel);
        taue = T(0.5) * (taue + sqrt(taue * taue + T(18) * cm * cm * nP * ir));
    } else if constexpr (SUB == LBM_WALE) {
        // velocity gradient g_ab = D_b v_a of the post-streaming field
        const T* __restrict__ vn = (const T*)m.vn;
        T g[3][3];
        const int nz = m.nz;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            int xp = x, xm = x, yp = y, ym = y, zp = z, zm = z;
            if (b == 0) { xp = wrapi(x + 1, nx); xm = wrapi(x - 1, nx); }
            if (b == 1) { yp = y + 1; ym = y - 1; }
            if (b == 2) { zp = wrapi(z + 1, nz); zm = wrapi(z - 1, nz); }
            bool okp = true, okm = true;
            if (b == 1) {
                if (m.walls) { okp = yp < ny; okm = ym >= 0; }
                else { yp = wrapi(yp, ny); ym = wrapi(ym, ny); }
            }
            const int cp = xp + nx * (yp + ny * zp), cm = xm + nx * (ym + ny * zm);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T vp = okp ? vn[(size_t)a * N + cp] : T(0);
                T vm = okm ? vn[(size_t)a * N + cm] : T(0);
                g[a][b] = T(0.5) * (vp - vm);
            }
        }
        T g2[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) g2[a][b] = g[a][0] * g[0][b] + g[a][1] * g[1][b] + g[a][2] * g[2][b];
        const T tr = g2[0][0] + g2[1][1] + g2[2][2];
        T SS = 0, SdSd = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                T S = T(0.5) * (g[a][b] + g[b][a]);
                T Sd = T(0.5) * (g2[a][b] + g2[b][a]) - (a == b ? tr / T(3) : T(0));
                SS += S * S;
                SdSd += Sd * Sd;
            }
        T den = pow(SS, T(2.5)) + pow(SdSd, T(1.25));
        T cm = T(m.cmodel);
        T nut = den > T(0) ? cm * cm * pow(SdSd, T(1.5)) / den : T(0);
        taue = taue + T(3) * nut;
    }
    const T om = T(1) / taue;

    // body force, F/rho velocity increment, predictor velocity
    T F[3] = {T(m.fprof[y]), 0, 0};
    if (m.drag != 0.0) {
#pragma unroll
        for (int a = 0; a < D; ++a) F[a] -= T(m.drag) * rho * u[a];
    }
    T du[3] = {0, 0, 0}, us[3] = {0, 0, 0};
    T dd = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        du[a] = F[a] * ir;
        us[a] = u[a] + du[a];
        dd += du[a] * (us[a] + u[a]);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T cd = T(L::cx[i]) * du[0] + T(L::cy[i]) * du[1] + (D == 3 ? T(L::cz[i]) * du[2] : T(0));
        const T cs = T(L::cx[i]) * (us[0] + u[0]) + T(L::cy[i]) * (us[1] + u[1]) +
                     (D == 3 ? T(L::cz[i]) * (us[2] + u[2]) : T(0));
        const T df = dfeq<T>(T(L::w[i]), rho, cd, cs, dd);
        const T out = PROJ ? f[i] + (df - om * fn[i]) : (f[i] - om * fn[i]) + df;
        if (A32 && MODE == 2)
            st_fld_at(gd, pop_at<Q>(i, (unsigned)cell), out, WT);
        else if (A32 && NT)
            __builtin_nontemporal_store(out, (T*)((char*)gd + pop_at<Q>(i, (unsigned)cell) * (unsigned)sizeof(T)));
        else if (A32)
            st_at(gd, pop_at<Q>(i, (unsigned)cell), out);
        else if (NT)
            __builtin_nontemporal_store(out, gd + pop_at64<Q>(i, (size_t)cell));
        else
            gd[pop_at64<Q>(i, (size_t)cell)] = out;
    }
    if (MODE == 2) {
        st_fld_at((T*)m.rho, (unsigned)cell, drho, WT);
#pragma unroll
        for (int a = 0; a < D; ++a) st_fld_at((T*)m.vs + (size_t)a * N, (unsigned)cell, us[a], WT);
    }
    if (MODE == 1 && SUB != LBM_WALE) {  // (with WALE, k_moments wrote v^n)
#pragma unroll
        for (int a = 0; a < D; ++a) ((T*)m.vn)[(size_t)a * N + cell] = u[a];
    }
    if (MODE >= 1) {
        st[0] += (double)drho;
#pragma unroll
        for (int a = 0; a < D; ++a) st[1 + a] += (double)(rho * u[a]);
    }
}

// A32: every population buffer of the launch spans less than 4 GiB, so
// pulls and stores use 32-bit offsets.  NT (plain modes): the populations are
// stored non-temporally, on launches whose populations exceed the Infinity
// Cache.
template <int LAT, typename T, int PREC, int SUB, int MODE, bool WT = false, bool A32 = MODE == 2, bool NT = false>
__global__ __launch_bounds__(kBlock, MODE == 2 ? 1 : 8) void k_step(const DevMember* __restrict__ mems,
                                                 const int2* __restrict__ work, int flip)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    __shared__ double lds[4 * (kBlock / 64)];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N, nx = m.nx, ny = m.ny;
    const int cell = wk.y * kBlock + threadIdx.x;
    const int cur = m.parity ^ flip;
    const T* __restrict__ gs = (const T*)m.g[cur];
    T* __restrict__ gd = (T*)m.g[cur ^ 1];
    double st[4] = {0, 0, 0, 0};
    int bad = 0;
    if (cell < N) {
        const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
        T f[Q];
        gather<LAT, T, A32>(m, gs, x, y, z, cell, f);
        collide_cell<LAT, T, PREC, SUB, MODE, WT, A32, NT>(m, f, x, y, z, cell, gd, st, bad);
    }
    if (MODE >= 1) {
        block_sum<4>(st, lds);
        if (threadIdx.x == 0) {
            double* p = m.part_stats + (size_t)wk.y * 4;
            p[0] = st[0]; p[1] = st[1]; p[2] = st[2]; p[3] = st[3];
        }
    }
    const unsigned long long anybad = __ballot(bad);
    if (anybad && (threadIdx.x & 63) == 0) atomicOr(&m.ctl->flags, 1);
}

// K1t: the TO stream-collide with the previous step's SGS change deferred
// into the pull.  A workgroup owns a TX x TY tile of the xy plane and a chunk
// of zc planes (the binomial-filter tiling and work table).  For every plane
// of the chunk and one halo plane on each side, the record (a, b) of the tile
// and its one-cell xy halo is staged in LDS together with e = a.b; the pull
// of population i at cell x then reads g*_i(x - c_i) from memory and the
// record of x - c_i from LDS, or for a bounce-back g*_opp(x) and the record of
// x itself.  The records of a step are zero after a flush (nothing pending).
// Statistics are summed per workgroup over its cells in z order.
// (At most 128 VGPRs in FP32: the LDS of a workgroup already limits the
// kernel to four waves per SIMD, and left alone the compiler hoists every
// pull and record read of a cell, 169 VGPRs, two waves.)
#ifndef LBM_STEPT_WAVES
#define LBM_STEPT_WAVES 4
#endif
template <int LAT, typename T, int PREC, int SUB, int TX, bool WT, bool A32 = true>
__global__ __launch_bounds__(TX * kBinTY, sizeof(T) == 4 ? LBM_STEPT_WAVES : 2) void k_step_t(const DevMember* __restrict__ mems,
                                                   const int2* __restrict__ work, int flip)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q, D = L::D;
    constexpr int NT = TX * kBinTY, TY = kBinTY, HX = TX + 2, HY = TY + 2, HXY = HX * HY;
    constexpr int NR = 2 * D;                     // a, b
    constexpr int NSL = D == 3 ? 3 : 1;           // staged planes
    constexpr int NE = (HXY + NT - 1) / NT;
    __shared__ T rs[NSL][NR + 1][HXY];            // a, b, e of the staged cells
    __shared__ double lds[4 * (NT / 64)];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N, nx = m.nx, ny = m.ny, nz = m.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int zc = m.zc;
    const int tx0 = (wk.y % ntx) * TX;
    const int ty0 = ((wk.y / ntx) % nty) * TY;
    const int tz0 = D == 3 ? (wk.y / (ntx * nty)) * zc : 0;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool own = x < nx && y < ny;
    const int cur = m.parity ^ flip;
    const T* __restrict__ gs = (const T*)m.g[cur];
    T* __restrict__ gd = (T*)m.g[cur ^ 1];
    const T* __restrict__ rec = (const T*)m.rec;
    const unsigned sN = (unsigned)N;
    // halo elements staged by this thread, as offsets within a plane; an
    // element beyond a wall loads cell 0 (a bounce-back never reads it)
    int eoff[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int e = threadIdx.x + k * NT;
        const int hx = e % HX, hy = e / HX;
        const int gx = modi(tx0 + hx - 1, nx);
        int gy = ty0 + hy - 1;
        bool ok = e < HXY;
        if (m.walls) ok = ok && gy >= 0 && gy < ny;
        else gy = modi(gy, ny);
        eoff[k] = ok ? gx + nx * gy : 0;
    }
    const int plane = nx * ny;
    auto fetch = [&](int pz, T (&buf)[NE][NR]) {
        const unsigned zo = (unsigned)(plane * (D == 3 ? modi(pz, nz) : 0));
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int c = 0; c < NR; ++c) buf[k][c] = ld_at(rec + c * sN, zo + (unsigned)eoff[k]);
    };
    auto stage = [&](int sl, const T (&buf)[NE][NR]) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < HXY) {
#pragma unroll
                for (int c = 0; c < NR; ++c) rs[sl][c][e] = buf[k][c];
                rs[sl][NR][e] = rec_e<D, T>(&buf[k][0], &buf[k][D]);
            }
        }
    };
    double st[4] = {0, 0, 0, 0};
    int bad = 0;
    // the 19 pulls g*_pi(src) of the own cell of plane z (issued before the
    // plane's records are staged, so their latency overlaps the staging)
    // (the general pull only: a constant-offset branch here costs the
    // kernel spills within its 128-VGPR budget)
    auto pull = [&](int z, T (&f)[Q]) { gather<LAT, T, A32, false>(m, gs, x, y, z, x + nx * (y + ny * z), f); };
    // add delta f of each pulled population from the staged records (a
    // bounce-back pulls population opp(i) of the cell itself: its delta f
    // from the own record with the sign of the linear term flipped, so every
    // direction is evaluated with constant c_i) and collide; sl0, sl1, sl2:
    // the staged planes z - 1, z, z + 1
    auto cell_step = [&](int z, int sl0, int sl1, int sl2, T (&f)[Q]) {
        const int cell = x + nx * (y + ny * z);
        const int pown = (ly + 1) * HX + lx + 1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int sy = y - L::cy[i];
            const bool bb = L::cy[i] != 0 && m.walls && (sy < 0 || sy >= ny);
            const int slz = D == 3 ? (L::cz[i] > 0 ? sl0 : (L::cz[i] < 0 ? sl2 : sl1)) : 0;
            const int pos = bb ? pown : pown - L::cy[i] * HX - L::cx[i];
            const T* r = &rs[bb ? sl1 : slz][0][pos];
            const T ca = cdot<LAT, T>(i, [&](int k) { return r[k * HXY]; });
            const T cb = cdot<LAT, T>(i, [&](int k) { return r[(D + k) * HXY]; });
            f[i] = add_rn(f[i], df_cc<LAT, T>(i, bb, ca, cb, r[NR * HXY]));
        }
        collide_cell<LAT, T, PREC, SUB, 2, WT, A32>(m, f, x, y, z, cell, gd, st, bad);
    };
    if constexpr (D == 2) {
        T buf[NE][NR], f[Q];
        fetch(0, buf);
        if (own) pull(0, f);
        stage(0, buf);
        __syncthreads();
        if (own) cell_step(0, 0, 0, 0, f);
    } else {
        // planes tz0 - 1 .. zend staged in a ring of three; the records of
        // the next plane and the pulls of the current one are in flight
        // while a plane is staged
        const int zend = min(tz0 + zc, nz);
        const int p0 = tz0 - 1, p1 = zend;
        T buf[NE][NR];
        fetch(p0, buf);
        for (int pz = p0; pz <= p1; ++pz) {
            const int sl = (pz - p0) % 3;
            const bool cmp = pz >= tz0 + 1 && own;   // plane pz - 1 once its upper neighbour is staged
            T f[Q];
            if (cmp) pull(pz - 1, f);
            stage(sl, buf);
            __syncthreads();
            if (pz < p1) fetch(pz + 1, buf);
            if (cmp) cell_step(pz - 1, (pz - 2 - p0) % 3, (pz - 1 - p0) % 3, sl, f);
            __syncthreads();
        }
    }
    block_sum<4, NT / 64>(st, lds);
    if (threadIdx.x == 0) {
        double* p = m.part_stats + (size_t)wk.y * 4;
        p[0] = st[0]; p[1] = st[1]; p[2] = st[2]; p[3] = st[3];
    }
    const unsigned long long anybad = __ballot(bad);
    if (anybad && (threadIdx.x & 63) == 0) atomicOr(&m.ctl->flags, 1);
}

// ---------------------------------------------------------------------------
// Post-streaming density and velocity of the current state (stream only,
// the SGS change of the last step included): used for WALE gradients and
// lbm_fields.  rho_out and u_out (nullable): rho [N] and v [D][N] in double.
// ---------------------------------------------------------------------------
template <int LAT, typename T, int PREC, bool TO>
__global__ __launch_bounds__(kBlock) void k_moments(const DevMember* __restrict__ mems,
                                                    const int2* __restrict__ work, int flip,
                                                    double* __restrict__ rho_out, double* __restrict__ u_out)
{
    using L = Lat<LAT>;
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N, nx = m.nx, ny = m.ny;
    const int cell = wk.y * kBlock + threadIdx.x;
    if (cell >= N) return;
    const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
    const T* gs = (const T*)m.g[m.parity ^ flip];
    T f[L::Q];
    gather<LAT, T, false>(m, gs, x, y, z, cell, f);
    T drho, j[3] = {0, 0, 0};
    moments<LAT, T, PREC>(f, drho, j);
    const T rho = T(1) + drho;
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        const T v = j[a] / rho;
        ((T*)m.vn)[(size_t)a * N + cell] = v;
        if (u_out) u_out[(size_t)a * N + cell] = (double)v;
    }
    if (rho_out) rho_out[cell] = (double)rho;
}

// ---------------------------------------------------------------------------
// Helpers for stencils on scalar fields with the filter/derivative boundary
// rule: periodic wrap, zero outside the domain on the wall axis.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T fld(const T* __restrict__ u, int x, int y, int z, int nx, int ny, int nz, int walls)
{
    x = wrapi(x, nx);
    z = wrapi(z, nz);
    if (walls) {
        if (y < 0 || y >= ny) return T(0);
    } else
        y = wrapi(y, ny);
    return u[x + nx * (y + ny * z)];
}

// Central-difference curl of a D-component field at (x,y,z) (2-D: scalar).
template <int D, typename T>
__device__ __forceinline__ void curl_at(const T* __restrict__ v, size_t N, int x, int y, int z, int nx, int ny,
                                        int nz, int walls, T* w)
{
    const T* vx = v;
    const T* vy = v + N;
    if (D == 2) {
        w[0] = T(0.5) * (fld(vy, x + 1, y, z, nx, ny, nz, walls) - fld(vy, x - 1, y, z, nx, ny, nz, walls)) -
               T(0.5) * (fld(vx, x, y + 1, z, nx, ny, nz, walls) - fld(vx, x, y - 1, z, nx, ny, nz, walls));
    } else {
        const T* vz = v + 2 * N;
        T dyvz = T(0.5) * (fld(vz, x, y + 1, z, nx, ny, nz, walls) - fld(vz, x, y - 1, z, nx, ny, nz, walls));
        T dzvy = T(0.5) * (fld(vy, x, y, z + 1, nx, ny, nz, walls) - fld(vy, x, y, z - 1, nx, ny, nz, walls));
        T dzvx = T(0.5) * (fld(vx, x, y, z + 1, nx, ny, nz, walls) - fld(vx, x, y, z - 1, nx, ny, nz, walls));
        T dxvz = T(0.5) * (fld(vz, x + 1, y, z, nx, ny, nz, walls) - fld(vz, x - 1, y, z, nx, ny, nz, walls));
        T dxvy = T(0.5) * (fld(vy, x + 1, y, z, nx, ny, nz, walls) - fld(vy, x - 1, y, z, nx, ny, nz, walls));
        T dyvx = T(0.5) * (fld(vx, x, y + 1, z, nx, ny, nz, walls) - fld(vx, x, y - 1, z, nx, ny, nz, walls));
        w[0] = dyvz - dzvy;
        w[1] = dzvx - dxvz;
        w[2] = dxvy - dyvx;
    }
}

// Neighbour offsets of cell c = (x, y, z) for second-order central
// differences: periodic wrap, and on the wall axis a neighbour beyond a wall
// is the cell itself, counted as zero (ok flags).  Every load of the
// differences below is unconditional, a 32-bit offset from a scalar base (TO
// fields stay below 2^32 bytes), so no branch-joined load stalls the others.
struct Nbr {
    unsigned xm, xp, ym, yp, zm, zp;
    bool okm, okp;
};
__device__ __forceinline__ Nbr nbr_at(unsigned c, int x, int y, int z, int nx, int ny, int nz, int walls, int D)
{
    Nbr n;
    n.xm = c - x + wrapi(x - 1, nx);
    n.xp = c - x + wrapi(x + 1, nx);
    n.okm = true;
    n.okp = true;
    int ym = y - 1, yp = y + 1;
    if (walls) { n.okm = ym >= 0; n.okp = yp < ny; ym = n.okm ? ym : y; yp = n.okp ? yp : y; }
    else { ym = wrapi(ym, ny); yp = wrapi(yp, ny); }
    n.ym = c + (unsigned)((ym - y) * nx);
    n.yp = c + (unsigned)((yp - y) * nx);
    const int plane = nx * ny;
    n.zm = D == 3 ? c + (unsigned)((wrapi(z - 1, nz) - z) * plane) : c;
    n.zp = D == 3 ? c + (unsigned)((wrapi(z + 1, nz) - z) * plane) : c;
    return n;
}

// Central-difference curl of the D-component field u at a cell (2-D: the
// scalar D_x u_y - D_y u_x).  In 3-D the adjoint curl^T is the curl itself.
template <int D, typename T>
__device__ __forceinline__ void curl_nb(const T* __restrict__ u, unsigned sN, unsigned c, const Nbr& n, T* w)
{
    const T* ux = u;
    const T* uy = u + sN;
    auto y0 = [](bool ok, T v) { return ok ? v : T(0); };
    if (D == 2) {
        w[0] = T(0.5) * (ld_at(uy, n.xp) - ld_at(uy, n.xm)) -
               T(0.5) * (y0(n.okp, ld_at(ux, n.yp)) - y0(n.okm, ld_at(ux, n.ym)));
    } else {
        const T* uz = u + 2 * sN;
        const T dyuz = T(0.5) * (y0(n.okp, ld_at(uz, n.yp)) - y0(n.okm, ld_at(uz, n.ym)));
        const T dzuy = T(0.5) * (ld_at(uy, n.zp) - ld_at(uy, n.zm));
        const T dzux = T(0.5) * (ld_at(ux, n.zp) - ld_at(ux, n.zm));
        const T dxuz = T(0.5) * (ld_at(uz, n.xp) - ld_at(uz, n.xm));
        const T dxuy = T(0.5) * (ld_at(uy, n.xp) - ld_at(uy, n.xm));
        const T dyux = T(0.5) * (y0(n.okp, ld_at(ux, n.yp)) - y0(n.okm, ld_at(ux, n.ym)));
        w[0] = dyuz - dzuy;
        w[1] = dzux - dxuz;
        w[2] = dxuy - dyux;
    }
}

// The adjoint curl of a curl field psi (NC components) at a cell: 2-D
// (D_y psi, -D_x psi) (eq. enstrophy-sensitivity-2d), 3-D curl psi
// (eq. enstrophy-sensitivity-3d).
template <int D, typename T>
__device__ __forceinline__ void curlT_nb(const T* __restrict__ psi, unsigned sN, unsigned c, const Nbr& n, T* out)
{
    if (D == 2) {
        auto y0 = [](bool ok, T v) { return ok ? v : T(0); };
        out[0] = T(0.5) * (y0(n.okp, ld_at(psi, n.yp)) - y0(n.okm, ld_at(psi, n.ym)));
        out[1] = -(T(0.5) * (ld_at(psi, n.xp) - ld_at(psi, n.xm)));
    } else {
        curl_nb<3, T>(psi, sN, c, n, out);
    }
}

// K2a: w = curl v* into W_0 (kernel-filter and Fourier closures, whose
// filter passes start from w).
template <int LAT, typename T, bool WT>
__global__ __launch_bounds__(kBlock) void k_curl(const DevMember* __restrict__ mems, const int2* __restrict__ work)
{
    using L = Lat<LAT>;
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    if (!kc(m.prm)->has_z) return;
    const int N = m.N, nx = m.nx, ny = m.ny, nz = m.nz;
    const int cell = wk.y * kBlock + threadIdx.x;
    if (cell >= N) return;
    const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
    const unsigned c = (unsigned)cell;
    const Nbr nb = nbr_at(c, x, y, z, nx, ny, nz, m.walls, L::D);
    T w[3];
    curl_nb<L::D, T>((const T*)m.vs, (unsigned)N, c, nb, w);
    T* W = (T*)m.W;
#pragma unroll
    for (int a = 0; a < L::NC; ++a) st_fld_at(W + (size_t)a * N, c, w[a], WT);
}

// Binomial filter B = (x)_a [1,2,1]/4 of one scalar field at (x,y,z).
template <int D, typename T>
__device__ __forceinline__ T binom_at(const T* __restrict__ u, int x, int y, int z, int nx, int ny, int nz, int walls)
{
    const int xm = wrapi(x - 1, nx), xp = wrapi(x + 1, nx);
    T acc = 0;
    const int zr = D == 3 ? 1 : 0;
#pragma unroll
    for (int oz = -zr; oz <= zr; ++oz) {
        const int zz = D == 3 ? wrapi(z + oz, nz) : 0;
        T sy = 0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            int yy = y + oy;
            T r = 0;
            if (walls && (yy < 0 || yy >= ny)) {
                r = T(0);
            } else {
                yy = wrapi(yy, ny);
                const T* row = u + (size_t)nx * (yy + (size_t)ny * zz);
                r = T(0.25) * (row[xm] + T(2) * row[x] + row[xp]);
            }
            sy += (oy == 0 ? T(0.5) : T(0.25)) * r;
        }
        acc += (D == 3 ? (oz == 0 ? T(0.5) : T(0.25)) : T(1)) * sy;
    }
    return acc;
}

// K2b, passes j >= 2: P_j = B P_{j-1} for j <= jv and W_j = B W_{j-1} with
// C_{j-1} = curl^T W_{j-1} for j <= jw (pass 1 is k_binom1).
// 2.5-D tiling: a workgroup of 8 TX threads owns a TX x 8 tile of the xy
// plane (32 x 8, or 64 x 8 on wide grids: each staged row then wastes fewer
// 128-byte lines on its one-cell x halo) and a chunk of zc planes (chosen per grid for enough
// workgroups); every plane of the chunk (plus one halo plane on each side)
// is staged with its xy halo in LDS, filtered in x and y there, and the z
// pass runs on a three-plane window kept in registers.

// CH: the chains the launch advances (1: v, 2: w and its curl, 3: both);
// the launch passes the union over its members, and a member whose chain
// this pass does not advance either returns (CH = 1, 2) or re-reads the
// other chain's source (CH = 3).
template <int LAT, typename T, int TX, int CH, bool WT>
__global__ __launch_bounds__(TX * kBinTY) void k_binom(const DevMember* __restrict__ mems, const int2* __restrict__ work,
                                                  int j)
{
    using L = Lat<LAT>;
    constexpr int D = L::D, NC = L::NC;
    constexpr int NV = (CH & 1) ? D : 0, NW = (CH & 2) ? NC : 0, NCMP = NV + NW;   // tile: v, then w
    constexpr int NT = TX * kBinTY, TY = kBinTY;   // tile TX x 8, one cell per thread
    constexpr int HX = TX + 2, HY = TY + 2, HXY = HX * HY;
    // the staged plane [component][halo tile]
    __shared__ T tile[NCMP * HXY];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    KParam* prm = kc(m.prm);
    // this pass: B^j v (j <= jv), B^j w (j <= jw) and C_{j-1} = curl^T B^{j-1} w (j - 1 <= jw)
    const bool dov = j <= prm->jv, dow = prm->has_z && j <= prm->jw;
    const bool doc = dow;   // the top C_jw is formed by its readers from W_jw
    if (!dov && !doc) return;
    if ((CH == 1 && !dov) || (CH == 2 && !doc)) return;
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const size_t sN = (size_t)m.N;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int zc = m.zc;
    const int tx0 = (wk.y % ntx) * TX;
    const int ty0 = ((wk.y / ntx) % nty) * TY;
    const int tz0 = (wk.y / (ntx * nty)) * zc;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool own = x < nx && y < ny;
    // Source and destination component pointers.  Every component is loaded
    // unconditionally (no branch-joined loads, so the loads of a plane stay
    // in flight together); a chain this pass does not advance re-reads the
    // other chain's source (cache hits) and stores nothing.
    const T* src[NCMP];
    T* dst[NCMP];
    const T* sv = j == 1 ? (const T*)m.vs : (const T*)m.P + (size_t)(j - 2) * D * sN;
    const T* sw = (const T*)m.W + (size_t)(j - 1) * NC * sN;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        src[a] = dov ? sv + a * sN : sw + (a % NC) * sN;
        dst[a] = dov ? (T*)m.P + ((size_t)(j - 1) * D + a) * sN : nullptr;
    }
#pragma unroll
    for (int a = 0; a < NW; ++a) {
        src[NV + a] = doc ? sw + a * sN : sv + (a % D) * sN;
        dst[NV + a] = dow ? (T*)m.W + ((size_t)j * NC + a) * sN : nullptr;
    }
    T* cdst = NW > 0 && doc ? (T*)m.C + (size_t)(j - 1) * D * sN : nullptr;
    const int zr = D == 3 ? 1 : 0;
    const int zend = D == 3 ? min(tz0 + zc, nz) : 1;
    // the (at most two) halo elements this thread stages, as offsets within
    // a plane; an element outside the walls loads cell 0 and stages zero
    constexpr int NE = (HXY + NT - 1) / NT;
    int eoff[NE];
    bool eok[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int e = threadIdx.x + k * NT;
        const int hx = e % HX, hy = e / HX;
        int gx = tx0 + hx - 1;       // in [-1, nx + TX - 1]
        gx = gx < 0 ? gx + nx : (gx >= nx ? modi(gx, nx) : gx);
        int gy = ty0 + hy - 1;       // in [-1, ny + TY - 1]
        bool ok = e < HXY;
        if (m.walls) ok = ok && gy >= 0 && gy < ny;
        else gy = gy < 0 ? gy + ny : (gy >= ny ? modi(gy, ny) : gy);
        eok[k] = ok;
        eoff[k] = ok ? gx + nx * gy : 0;
    }
    const int plane = nx * ny;
    auto fetch = [&](int pz, T (&buf)[NE][NCMP]) {
        const int zz = D == 3 ? modi(pz, nz) : 0;
        const unsigned zo = (unsigned)(plane * zz);
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int c = 0; c < NCMP; ++c) buf[k][c] = ld_at(src[c], zo + (unsigned)eoff[k]);
    };
    auto stage = [&](int pl, const T (&buf)[NE][NCMP]) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < HXY) {
#pragma unroll
                for (int c = 0; c < NCMP; ++c) tile[(pl * NCMP + c) * HXY + e] = eok[k] ? buf[k][c] : T(0);
            }
        }
    };
    // x and y passes of the staged plane pl at the own cell; the own value
    // and xy derivatives of w for the curl
    auto xyfilter = [&](int pl, T (&sn)[NCMP], T (&rn)[NC], T (&dn)[NC][2]) {
#pragma unroll
        for (int c = 0; c < NCMP; ++c) {
            const T* t = tile + (pl * NCMP + c) * HXY + ly * HX + lx;   // (lx, ly): lower-left halo corner
            const T q0 = T(0.25) * (t[0] + T(2) * t[1] + t[2]);
            const T q1 = T(0.25) * (t[HX] + T(2) * t[HX + 1] + t[HX + 2]);
            const T q2 = T(0.25) * (t[2 * HX] + T(2) * t[2 * HX + 1] + t[2 * HX + 2]);
            sn[c] = T(0.25) * q0 + T(0.5) * q1 + T(0.25) * q2;
        }
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            const T* t = tile + (pl * NCMP + NV + a) * HXY + (ly + 1) * HX + lx + 1;
            rn[a] = t[0];
            dn[a][0] = T(0.5) * (t[1] - t[-1]);
            dn[a][1] = T(0.5) * (t[HX] - t[-HX]);
        }
    };
    // 3-D output of plane zo from the xy-filtered planes zo-1, zo, zo+1 (sa,
    // sb, sc), w at zo-1 and zo+1 (ra, rc) and the xy derivatives at zo
    auto emit3 = [&](int zo, const T (&sa)[NCMP], const T (&sb)[NCMP], const T (&sc)[NCMP], const T (&ra)[NC],
                     const T (&rc)[NC], const T (&dxyb)[NC][2]) {
        if (!own) return;
        const size_t ci = (size_t)x + (size_t)nx * (y + (size_t)ny * zo);
#pragma unroll
        for (int c = 0; c < NCMP; ++c)
            if (dst[c]) st_fld(dst[c] + ci, T(0.25) * sa[c] + T(0.5) * sb[c] + T(0.25) * sc[c], WT);
        if constexpr (D == 3 && NW > 0) {
            if (cdst) {   // curl w at plane zo, D_z from the planes below and above
                st_fld(cdst + ci, (T(0.5) * ra[1] + dxyb[2][1]) - T(0.5) * rc[1], WT);        // D_y w_z - D_z w_y
                st_fld(cdst + sN + ci, (T(-0.5) * ra[0] - dxyb[2][0]) + T(0.5) * rc[0], WT);  // D_z w_x - D_x w_z
                st_fld(cdst + 2 * sN + ci, dxyb[1][0] - dxyb[0][1], WT);                      // D_x w_y - D_y w_x
            }
        }
    };
    const int p0 = tz0 - zr, p1 = zend - 1 + zr;   // staged planes, inclusive
    if (D == 2) {
        T buf[NE][NCMP], sn[NCMP], rn[NC] = {}, dn[NC][2] = {};
        fetch(0, buf);
        stage(0, buf);
        __syncthreads();
        xyfilter(0, sn, rn, dn);
        if (own) {
            const size_t ci = (size_t)x + (size_t)nx * y;
#pragma unroll
            for (int c = 0; c < NCMP; ++c)
                if (dst[c]) st_fld(dst[c] + ci, sn[c], WT);
            if (NW > 0 && cdst) {   // curl^T of a scalar: (D_y w, -D_x w)
                st_fld(cdst + ci, dn[0][1], WT);
                st_fld(cdst + sN + ci, -dn[0][0], WT);
            }
        }
    } else {
        // zc output planes: software pipeline over a three-plane register
        // window; the loads of the next plane are in flight while the
        // current one is filtered.  (Measured on MI355X: deeper prefetch or
        // a second LDS buffer do not pay here.)
        T s0[NCMP], s1[NCMP];
        T r1[NC], r2[NC], dxy[NC][2];   // w at planes z-1 and z (own cell), xy derivatives at z
#pragma unroll
        for (int c = 0; c < NCMP; ++c) { s0[c] = 0; s1[c] = 0; }
#pragma unroll
        for (int a = 0; a < NC; ++a) { r1[a] = 0; r2[a] = 0; dxy[a][0] = 0; dxy[a][1] = 0; }
        T buf[NE][NCMP];
        fetch(p0, buf);
        for (int pz = p0; pz <= p1; ++pz) {
            stage(0, buf);
            __syncthreads();
            if (pz < p1) fetch(pz + 1, buf);
            T sn[NCMP], rn[NC] = {}, dn[NC][2] = {};
            xyfilter(0, sn, rn, dn);
            __syncthreads();
            if (pz >= tz0 + 1) emit3(pz - 1, s0, s1, sn, r1, rn, dxy);  // once its upper neighbour is staged
#pragma unroll
            for (int c = 0; c < NCMP; ++c) { s0[c] = s1[c]; s1[c] = sn[c]; }
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                r1[a] = r2[a]; r2[a] = rn[a];
                dxy[a][0] = dn[a][0]; dxy[a][1] = dn[a][1];
            }
        }
    }
}

// K2b, pass 1: the first power of both chains from v* alone.  v* is staged
// with a two-cell xy halo; w = curl v* is formed in LDS on the tile and its
// one-cell halo (zero beyond the walls, as every filtered field), from which
// the pass forms B w and C_0 = curl^T w; it writes P_1 = B v* (jv >= 1),
// W_0 = w and, when jw >= 1, W_1 = B w and C_0.  In 3-D the z direction runs
// through a ring of three staged v* planes and register windows of the xy
// parts, w lagging v* by one plane.  ZC: some member of the launch has Z
// QoIs (otherwise only B v* is formed).
template <int LAT, typename T, int TX, bool ZC, bool WT>
__global__ __launch_bounds__(TX * kBinTY) void k_binom1(const DevMember* __restrict__ mems, const int2* __restrict__ work)
{
    using L = Lat<LAT>;
    constexpr int D = L::D, NC = L::NC;
    constexpr int NT = TX * kBinTY, TY = kBinTY;
    constexpr int HX1 = TX + 2, HY1 = TY + 2, HXY1 = HX1 * HY1;   // tile and one-cell halo
    constexpr int HX2 = TX + 4, HY2 = TY + 4, HXY2 = HX2 * HY2;   // tile and two-cell halo
    constexpr int NE1 = (HXY1 + NT - 1) / NT, NE2 = (HXY2 + NT - 1) / NT;
    constexpr int NSL = D == 3 ? 3 : 1;
    __shared__ T vt[NSL][D][HXY2];
    __shared__ T wt[ZC ? NC : 1][ZC ? HXY1 : 1];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    KParam* prm = kc(m.prm);
    const bool dov = prm->jv >= 1;
    const bool doz = ZC && prm->has_z;
    const bool dow1 = doz && prm->jw >= 1;
    if (!dov && !doz) return;   // uniform
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const size_t sN = (size_t)m.N;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int zc = m.zc;
    const int tx0 = (wk.y % ntx) * TX;
    const int ty0 = ((wk.y / ntx) % nty) * TY;
    const int tz0 = D == 3 ? (wk.y / (ntx * nty)) * zc : 0;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool own = x < nx && y < ny;
    const T* vs = (const T*)m.vs;
    T* P1 = (T*)m.P;
    T* W0 = (T*)m.W;
    T* W1 = (T*)m.W + (size_t)NC * sN;
    T* C0 = (T*)m.C;
    // the staged v* elements of this thread (plane offsets; beyond the walls
    // cell 0 is loaded and zero staged)
    int eoff[NE2];
    bool eok[NE2];
#pragma unroll
    for (int k = 0; k < NE2; ++k) {
        const int e = threadIdx.x + k * NT;
        const int gx = modi(tx0 + e % HX2 - 2, nx);
        int gy = ty0 + e / HX2 - 2;
        bool ok = e < HXY2;
        if (m.walls) ok = ok && gy >= 0 && gy < ny;
        else gy = modi(gy, ny);
        eok[k] = ok;
        eoff[k] = ok ? gx + nx * gy : 0;
    }
    // the w elements of this thread: zero beyond the walls
    bool wok[NE1];
#pragma unroll
    for (int k = 0; k < NE1; ++k) {
        const int e = threadIdx.x + k * NT;
        const int gy = ty0 + e / HX1 - 1;
        wok[k] = e < HXY1 && !(m.walls && (gy < 0 || gy >= ny));
    }
    const int plane = nx * ny;
    auto fetch = [&](int pz, T (&buf)[NE2][D]) {
        const unsigned zo = (unsigned)(plane * (D == 3 ? modi(pz, nz) : 0));
#pragma unroll
        for (int k = 0; k < NE2; ++k)
#pragma unroll
            for (int a = 0; a < D; ++a) buf[k][a] = ld_at(vs + a * sN, zo + (unsigned)eoff[k]);
    };
    auto stage = [&](int sl, const T (&buf)[NE2][D]) {
#pragma unroll
        for (int k = 0; k < NE2; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < HXY2) {
#pragma unroll
                for (int a = 0; a < D; ++a) vt[sl][a][e] = eok[k] ? buf[k][a] : T(0);
            }
        }
    };
    // xy part of B at the own cell of a tile t with row length H, own
    // position c
    auto bxy = [](const T* t, int c, int H) {
        const T q0 = T(0.25) * (t[c - H - 1] + T(2) * t[c - H] + t[c - H + 1]);
        const T q1 = T(0.25) * (t[c - 1] + T(2) * t[c] + t[c + 1]);
        const T q2 = T(0.25) * (t[c + H - 1] + T(2) * t[c + H] + t[c + H + 1]);
        return T(0.25) * q0 + T(0.5) * q1 + T(0.25) * q2;
    };
    // w = curl v* on the tile and its halo, from the staged planes z - 1,
    // z, z + 1 (s0, s1, s2; the same slot in 2-D)
    auto curl_tile = [&](int s0, int s1, int s2) {
#pragma unroll
        for (int k = 0; k < NE1; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e >= HXY1) continue;
            const int p = (e / HX1 + 1) * HX2 + e % HX1 + 1;
            T w[3];
            if (D == 2) {
                w[0] = T(0.5) * (vt[s1][1][p + 1] - vt[s1][1][p - 1]) -
                       T(0.5) * (vt[s1][0][p + HX2] - vt[s1][0][p - HX2]);
            } else {
                const T dyvz = T(0.5) * (vt[s1][2 % D][p + HX2] - vt[s1][2 % D][p - HX2]);
                const T dzvy = T(0.5) * (vt[s2][1][p] - vt[s0][1][p]);
                const T dzvx = T(0.5) * (vt[s2][0][p] - vt[s0][0][p]);
                const T dxvz = T(0.5) * (vt[s1][2 % D][p + 1] - vt[s1][2 % D][p - 1]);
                const T dxvy = T(0.5) * (vt[s1][1][p + 1] - vt[s1][1][p - 1]);
                const T dyvx = T(0.5) * (vt[s1][0][p + HX2] - vt[s1][0][p - HX2]);
                w[0] = dyvz - dzvy;
                w[1] = dzvx - dxvz;
                w[2] = dxvy - dyvx;
            }
#pragma unroll
            for (int a = 0; a < NC; ++a) wt[a % (ZC ? NC : 1)][ZC ? e : 0] = wok[k] ? w[a] : T(0);
        }
    };
    const int pv = (ly + 2) * HX2 + lx + 2;   // own cell in the v* tile
    const int pw = (ly + 1) * HX1 + lx + 1;   // own cell in the w tile
    if constexpr (D == 2) {
        T buf[NE2][D];
        fetch(0, buf);
        stage(0, buf);
        __syncthreads();
        if constexpr (ZC) {
            if (doz) curl_tile(0, 0, 0);
            __syncthreads();
        }
        if (!own) return;
        const size_t ci = (size_t)x + (size_t)nx * y;
        if (dov)
#pragma unroll
            for (int a = 0; a < D; ++a) st_fld(P1 + a * sN + ci, bxy(&vt[0][a][0], pv, HX2), WT);
        if constexpr (ZC) {
            if (doz) st_fld(W0 + ci, wt[0][pw], WT);
            if (dow1) {
                st_fld(W1 + ci, bxy(&wt[0][0], pw, HX1), WT);
                st_fld(C0 + ci, T(0.5) * (wt[0][pw + HX1] - wt[0][pw - HX1]), WT);        // D_y w
                st_fld(C0 + sN + ci, -(T(0.5) * (wt[0][pw + 1] - wt[0][pw - 1])), WT);    // -D_x w
            }
        }
    } else {
        // output planes [tz0, zend); v* staged on tz0 - 2 .. zend + 1, w
        // formed on tz0 - 1 .. zend
        const int zend = min(tz0 + zc, nz);
        const int p0 = tz0 - 2, p1 = zend + 1;
        T bva[D] = {}, bvb[D] = {};                 // B_xy v* at planes pz - 2, pz - 1
        T oma[3] = {}, omb[3] = {};                 // w (own cell) at planes pz - 3, pz - 2
        T bwa[3] = {}, bwb[3] = {};                 // B_xy w at planes pz - 3, pz - 2
        T dxb[3] = {}, dyb[3] = {};                 // D_x w, D_y w at plane pz - 2
        T buf[NE2][D];
        fetch(p0, buf);
        for (int pz = p0; pz <= p1; ++pz) {
            const int sl = (pz - p0) % 3;
            stage(sl, buf);
            __syncthreads();
            if (pz < p1) fetch(pz + 1, buf);
            T bvn[D];
#pragma unroll
            for (int a = 0; a < D; ++a) bvn[a] = bxy(&vt[sl][a][0], pv, HX2);
            if (dov && own && pz - 1 >= tz0 && pz - 1 < zend) {
                const size_t ci = (size_t)x + (size_t)nx * (y + (size_t)ny * (pz - 1));
#pragma unroll
                for (int a = 0; a < D; ++a)
                    st_fld(P1 + a * sN + ci, T(0.25) * bva[a] + T(0.5) * bvb[a] + T(0.25) * bvn[a], WT);
            }
#pragma unroll
            for (int a = 0; a < D; ++a) { bva[a] = bvb[a]; bvb[a] = bvn[a]; }
            if constexpr (ZC) {
                if (doz && pz >= tz0) {
                    // w at plane pz - 1 on the tile and its halo
                    curl_tile((pz - 2 - p0) % 3, (pz - 1 - p0) % 3, sl);
                    __syncthreads();
                    T omn[3], bwn[3], dxn[3], dyn[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const T* t = &wt[a][0];
                        omn[a] = t[pw];
                        bwn[a] = bxy(t, pw, HX1);
                        dxn[a] = T(0.5) * (t[pw + 1] - t[pw - 1]);
                        dyn[a] = T(0.5) * (t[pw + HX1] - t[pw - HX1]);
                    }
                    if (own && pz - 1 >= tz0 && pz - 1 < zend) {
                        const size_t ci = (size_t)x + (size_t)nx * (y + (size_t)ny * (pz - 1));
#pragma unroll
                        for (int a = 0; a < 3; ++a) st_fld(W0 + a * sN + ci, omn[a], WT);
                    }
                    if (dow1 && own && pz - 2 >= tz0 && pz - 2 < zend) {
                        const size_t ci = (size_t)x + (size_t)nx * (y + (size_t)ny * (pz - 2));
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            st_fld(W1 + a * sN + ci, T(0.25) * bwa[a] + T(0.5) * bwb[a] + T(0.25) * bwn[a], WT);
                        // curl w at plane pz - 2, D_z from the planes below and above
                        st_fld(C0 + ci, dyb[2] - T(0.5) * (omn[1] - oma[1]), WT);           // D_y w_z - D_z w_y
                        st_fld(C0 + sN + ci, T(0.5) * (omn[0] - oma[0]) - dxb[2], WT);      // D_z w_x - D_x w_z
                        st_fld(C0 + 2 * sN + ci, dxb[1] - dyb[0], WT);                      // D_x w_y - D_y w_x
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        oma[a] = omb[a]; omb[a] = omn[a];
                        bwa[a] = bwb[a]; bwb[a] = bwn[a];
                        dxb[a] = dxn[a]; dyb[a] = dyn[a];
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Per-cell sensitivities of all E/Z QoIs (App. A):
//   E: V = R R v = sum_j rr_j B^j v;
//   Z: V = curl^T R R w = sum_j rr_j C_j with C_j = curl^T B^j w, formed by
//      the binomial passes (2-D: curl^T psi = (D_y psi, -D_x psi); 3-D: curl).
// Also returns the QoI densities 1/2 |R v|^2 and 1/2 |R w|^2 of the cell.
// ---------------------------------------------------------------------------
// Filter coefficients in the kernel's arithmetic type (FP32 copies are made
// on the host, so both read them from scalar registers without conversion).
template <typename T> __device__ __forceinline__ T coef_r(KParam* p, int s, int j);
template <> __device__ __forceinline__ float coef_r<float>(KParam* p, int s, int j) { return p->rf[s][j]; }
template <> __device__ __forceinline__ double coef_r<double>(KParam* p, int s, int j) { return p->r[s][j]; }
template <typename T> __device__ __forceinline__ T coef_rr(KParam* p, int s, int j);
template <> __device__ __forceinline__ float coef_rr<float>(KParam* p, int s, int j) { return p->rrf[s][j]; }
template <> __device__ __forceinline__ double coef_rr<double>(KParam* p, int s, int j) { return p->rr[s][j]; }
template <typename T> __device__ __forceinline__ T coef_cv(KCtl* c, int j);
template <> __device__ __forceinline__ float coef_cv<float>(KCtl* c, int j) { return c->cvf[j]; }
template <> __device__ __forceinline__ double coef_cv<double>(KCtl* c, int j) { return c->cv[j]; }
template <typename T> __device__ __forceinline__ T coef_cw(KCtl* c, int j);
template <> __device__ __forceinline__ float coef_cw<float>(KCtl* c, int j) { return c->cwf[j]; }
template <> __device__ __forceinline__ double coef_cw<double>(KCtl* c, int j) { return c->cw[j]; }

// C_jw = curl^T W_jw at cell (x, y, z) from the neighbours of W_jw: the
// binomial passes store C_j only for j < jw.
template <int LAT, typename T>
__device__ __forceinline__ void top_curl(KMember& m, int jw, int x, int y, int z, T* out)
{
    using L = Lat<LAT>;
    const unsigned sN = (unsigned)m.N;
    const unsigned c = (unsigned)(x + m.nx * (y + m.ny * z));
    const Nbr nb = nbr_at(c, x, y, z, m.nx, m.ny, m.nz, m.walls, L::D);
    curlT_nb<L::D, T>((const T*)m.W + (size_t)jw * L::NC * sN, sN, c, nb, out);
}

// The top C_jw = curl^T W_jw of a cell in two steps, so that a caller can
// hold the loads and form the curl later: the neighbour values (2-D: psi at
// y+1, y-1, x+1, x-1; 3-D: w_z, w_y, w_x at the pairs of neighbours of
// D_y w_z, D_z w_y, D_z w_x, D_x w_z, D_x w_y, D_y w_x), then central
// differences (zero beyond the walls), without contraction.
template <int LAT, typename T>
__device__ __forceinline__ void top_curl_load(KMember& m, int jw, int x, int y, int z, T* r, bool& okm, bool& okp)
{
    using L = Lat<LAT>;
    const unsigned sN = (unsigned)m.N;
    const unsigned c = (unsigned)(x + m.nx * (y + m.ny * z));
    const Nbr n = nbr_at(c, x, y, z, m.nx, m.ny, m.nz, m.walls, L::D);
    const T* psi = (const T*)m.W + (size_t)jw * L::NC * sN;
    okm = n.okm;
    okp = n.okp;
    if constexpr (L::D == 2) {
        r[0] = ld_at(psi, n.yp); r[1] = ld_at(psi, n.ym);
        r[2] = ld_at(psi, n.xp); r[3] = ld_at(psi, n.xm);
    } else {
        const T* ux = psi;
        const T* uy = psi + sN;
        const T* uz = psi + 2 * sN;
        r[0] = ld_at(uz, n.yp); r[1] = ld_at(uz, n.ym);
        r[2] = ld_at(uy, n.zp); r[3] = ld_at(uy, n.zm);
        r[4] = ld_at(ux, n.zp); r[5] = ld_at(ux, n.zm);
        r[6] = ld_at(uz, n.xp); r[7] = ld_at(uz, n.xm);
        r[8] = ld_at(uy, n.xp); r[9] = ld_at(uy, n.xm);
        r[10] = ld_at(ux, n.yp); r[11] = ld_at(ux, n.ym);
    }
}

template <int D, typename T>
__device__ __forceinline__ void top_curl_eval(const T* r, bool okm, bool okp, T* out)
{
#pragma clang fp contract(off)
    auto y0 = [](bool ok, T v) { return ok ? v : T(0); };
    if constexpr (D == 2) {
        out[0] = T(0.5) * (y0(okp, r[0]) - y0(okm, r[1]));
        out[1] = -(T(0.5) * (r[2] - r[3]));
    } else {
        const T dyuz = T(0.5) * (y0(okp, r[0]) - y0(okm, r[1]));
        const T dzuy = T(0.5) * (r[2] - r[3]);
        const T dzux = T(0.5) * (r[4] - r[5]);
        const T dxuz = T(0.5) * (r[6] - r[7]);
        const T dxuy = T(0.5) * (r[8] - r[9]);
        const T dyux = T(0.5) * (y0(okp, r[10]) - y0(okm, r[11]));
        out[0] = dyuz - dzuy;
        out[1] = dzux - dxuz;
        out[2] = dxuy - dyux;
    }
}

// The fields a cell's sensitivities are formed from, loaded in one batch
// (no branch between the loads, so that the loads of several cells can be
// in flight together) and evaluated afterwards.
template <int LAT, typename T, int MAXSA>
struct CellIn {
    T pv[kMaxPow + 1][Lat<LAT>::D];   // B^j v*, j = 0..kMaxPow (clamped to jv)
    T wc[3][Lat<LAT>::NC];            // B^j w, j = 0..2 (clamped to jw)
    T cv[kMaxPow][Lat<LAT>::D];       // stored C_j (clamped to jw - 1)
    T nb[Lat<LAT>::D == 2 ? 4 : 12];  // W_jw at the neighbours of the top curl
    bool okm, okp;
    T kv[MAXSA][Lat<LAT>::D];         // kernel filters: V_s (clamped to nsa - 1)
};

template <int LAT, typename T, int MAXSA, bool KF>
__device__ __forceinline__ void cell_load(KMember& m, KParam* prm, int x, int y, int z, CellIn<LAT, T, MAXSA>& in)
{
    const int cell = x + m.nx * (y + m.ny * z);
    using L = Lat<LAT>;
    constexpr int D = L::D, NC = L::NC;
    const int jv = prm->jv, jw = prm->jw;
    const size_t sN = (size_t)m.N;
    const T* __restrict__ vs = (const T*)m.vs;
    if constexpr (KF) {
        const int nsa = prm->nsa;
        const T* __restrict__ kV = (const T*)m.kV;
#pragma unroll
        for (int a = 0; a < D; ++a) in.pv[0][a] = vs[a * sN + cell];
#pragma unroll
        for (int s2 = 0; s2 < MAXSA; ++s2) {
            const int sc = s2 < nsa ? s2 : nsa - 1;
#pragma unroll
            for (int a = 0; a < D; ++a) in.kv[s2][a] = kV[((size_t)sc * D + a) * sN + cell];
        }
        return;
    }
    const T* __restrict__ P = (const T*)m.P;
    const T* __restrict__ W = (const T*)m.W;
    // Every load is unconditional, with the power clamped to the highest one
    // stored: a power above jv (jw) only ever meets a zero coefficient.
#pragma unroll
    for (int jj = 0; jj <= kMaxPow; ++jj) {
        const int je = jj < jv ? jj : jv;
        const T* src = je == 0 ? vs : P + (size_t)(je - 1) * D * sN;
#pragma unroll
        for (int a = 0; a < D; ++a) in.pv[jj][a] = src[a * sN + cell];
    }
    const bool hz = prm->has_z;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const T* src = hz ? W + (size_t)(jj < jw ? jj : jw) * NC * sN : vs;   // (unused without Z QoIs)
#pragma unroll
        for (int a = 0; a < NC; ++a) in.wc[jj][a] = src[a * sN + cell];
    }
    // C_j = curl^T B^j w (Z sensitivities): the stored C_j for j < jw, the
    // top one formed at evaluation from the neighbours of W_jw (no
    // arithmetic here, so the loads of a next cell need not wait for these)
    if (!hz) return;
    top_curl_load<LAT, T>(m, jw, x, y, z, in.nb, in.okm, in.okp);
    const T* __restrict__ Cc = (const T*)m.C;
    const int jc = jw > 0 ? jw - 1 : 0;
#pragma unroll
    for (int jj = 0; jj < kMaxPow; ++jj) {
        const T* src = Cc + (size_t)(jj < jc ? jj : jc) * D * sN;
#pragma unroll
        for (int a = 0; a < D; ++a) in.cv[jj][a] = src[a * sN + cell];
    }
}

// The closure's filter coefficients of every E/Z QoI, read once per
// workgroup ahead of the field loads (zero past nsa, so that those QoIs
// contribute exact zeros), and its kinds (1 for Z).
template <typename T, int MAXSA>
struct SensCoef {
    T r[MAXSA][3], rr[MAXSA][kMaxPow + 1];
    int z[MAXSA];
    int nsa, hz, jw;
};

template <typename T, int MAXSA>
__device__ __forceinline__ void sens_coef(KParam* prm, SensCoef<T, MAXSA>& c)
{
    c.nsa = prm->nsa;
    c.hz = prm->has_z;
    c.jw = prm->jw;
#pragma unroll
    for (int s = 0; s < MAXSA; ++s) {
        c.z[s] = prm->sa_kind[s];
#pragma unroll
        for (int j = 0; j < 3; ++j) c.r[s][j] = coef_r<T>(prm, s, j);
#pragma unroll
        for (int j = 0; j <= kMaxPow; ++j) c.rr[s][j] = coef_rr<T>(prm, s, j);
    }
}

template <int LAT, typename T, int MAXSA, bool KF>
__device__ __forceinline__ void cell_eval(const SensCoef<T, MAXSA>& cf, const CellIn<LAT, T, MAXSA>& in,
                                          T (&V)[MAXSA][Lat<LAT>::D], double (&qd)[MAXSA])
{
    using L = Lat<LAT>;
    constexpr int D = L::D, NC = L::NC;
    const int nsa = cf.nsa;
    if constexpr (KF) {
        // kernel filters: the sensitivities V_s are materialised; both E and Z
        // QoIs are 1/2 <v*, V_s> (R self-adjoint, curl^T the adjoint of curl)
#pragma unroll
        for (int s2 = 0; s2 < MAXSA; ++s2) {
            qd[s2] = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                V[s2][a] = s2 < nsa ? in.kv[s2][a] : T(0);
                qd[s2] += 0.5 * (double)(in.pv[0][a] * V[s2][a]);
            }
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < MAXSA; ++s) {
        qd[s] = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) V[s][a] = 0;
        if (s >= nsa) continue;
        const T r0 = cf.r[s][0], r1 = cf.r[s][1], r2 = cf.r[s][2];
        if (cf.z[s] == 0) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const T rv = r0 * in.pv[0][a] + r1 * in.pv[1][a] + r2 * in.pv[2][a];
                qd[s] += 0.5 * (double)(rv * rv);
                T vv = 0;
#pragma unroll
                for (int jj = 0; jj <= kMaxPow; ++jj) vv += cf.rr[s][jj] * in.pv[jj][a];
                V[s][a] = vv;
            }
        } else {
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                const T rw = r0 * in.wc[0][a] + r1 * in.wc[1][a] + r2 * in.wc[2][a];
                qd[s] += 0.5 * (double)(rw * rw);
            }
        }
    }
    if (!cf.hz) return;
    // Z sensitivities from C_j = curl^T B^j w: the stored ones for j < jw,
    // the top one above
    T ctop[D];
    top_curl_eval<D, T>(in.nb, in.okm, in.okp, ctop);
#pragma unroll
    for (int s = 0; s < MAXSA; ++s) {
        if (s >= nsa || cf.z[s] == 0) continue;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T vv = 0;
#pragma unroll
            for (int jj = 0; jj <= kMaxPow; ++jj)
                vv += cf.rr[s][jj] * (jj < cf.jw && jj < kMaxPow ? in.cv[jj < kMaxPow ? jj : 0][a] : ctop[a]);
            V[s][a] = vv;
        }
    }
}

// ---------------------------------------------------------------------------
// K2c: per-cell QoIs, sensitivities and Gram products, FP64 partial sums per
// workgroup.  Workgroups cover one y row (2-D) or one y plane (3-D) each, so
// the mean-profile partial sums stay separated by y.
// Partial layout: q_sa[nsa], G_sa[nsa(nsa+1)/2], then (with MP QoIs)
// U = sum v*_x and P_s = sum V_s,x.
// ---------------------------------------------------------------------------
template <int LAT, typename T, int MAXSA, bool KF>
__global__ __launch_bounds__(kBlock) void k_reduce(const DevMember* __restrict__ mems, const int2* __restrict__ work)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    constexpr int NG = MAXSA * (MAXSA + 1) / 2;
    constexpr int NV = MAXSA + NG + 1 + MAXSA;
    __shared__ double lds[NV * (kBlock / 64)];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    KParam* prm = kc(m.prm);
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const int y = wk.y / m.nbx2, bx = wk.y % m.nbx2;
    const int plane = nx * nz;
    const int nsa = prm->nsa;
    const bool hasmp = prm->nmp > 0;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0;
    SensCoef<T, MAXSA> cf;
    sens_coef<T, MAXSA>(prm, cf);
    // One cell at a time (NP = 1), its fields loaded in one batch before it
    // is evaluated.  (Measured on MI355X: pairs of cells in FP32 took 197
    // VGPRs and two waves per SIMD, 510 us on 384 x 192 x 192 against 434 us
    // for single cells at three waves; 18.4 against 17.4 us on 96 x 48 x 48.)
    // The additions keep the order of the cells.
    constexpr int NP = 1;
    for (int c = 0; c < m.cpt2; c += NP) {
        const int pa = (bx * m.cpt2 + c) * kBlock + threadIdx.x;
        if (pa >= plane) break;
        bool has[NP];
        CellIn<LAT, T, MAXSA> in[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            has[u] = u == 0 || (c + u < m.cpt2 && pa + u * kBlock < plane);
            const int p = has[u] ? pa + u * kBlock : pa;
            const int x = p % nx, z = p / nx;
            cell_load<LAT, T, MAXSA, KF>(m, prm, x, y, z, in[u]);
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            if (!has[u]) break;
            T V[MAXSA][D];
            double qd[MAXSA];
            cell_eval<LAT, T, MAXSA, KF>(cf, in[u], V, qd);
#pragma unroll
            for (int s = 0; s < MAXSA; ++s) acc[s] += qd[s];
            int g = 0;
#pragma unroll
            for (int s = 0; s < MAXSA; ++s)
#pragma unroll
                for (int t2 = s; t2 < MAXSA; ++t2, ++g) {
                    T d = 0;
#pragma unroll
                    for (int a = 0; a < D; ++a) d += V[s][a] * V[t2][a];
                    acc[MAXSA + g] += (double)d;
                }
            if (hasmp) {
                acc[MAXSA + NG] += (double)in[u].pv[0][0];
#pragma unroll
                for (int s = 0; s < MAXSA; ++s) acc[MAXSA + NG + 1 + s] += (double)V[s][0];
            }
        }
    }
    // band weights w_j(y) of this row (workgroup-uniform: scalar loads,
    // issued before the reduction so that their latency is hidden)
    double wb[kMaxQ];
    const int nmp = prm->nmp;
    if (hasmp) {
        const LBM_K double* bw = kc(m.bandw);
#pragma unroll
        for (int jm = 0; jm < kMaxQ; ++jm) wb[jm] = bw[(size_t)prm->mp_band[jm < nmp ? jm : nmp - 1] * ny + y];
    }
    // partials are stored value-major, [npart][ny * nbx2], so that the
    // cross-block sums read them contiguously; thread t writes value t
    const double r = block_sum_spread<NV>(acc, lds);
    const int t = threadIdx.x;
    const size_t nblk = (size_t)ny * m.nbx2;
    double* out = m.part_to + wk.y;
    if (t < MAXSA) {
        if (t < nsa) out[t * nblk] = r;
    } else if (t < MAXSA + NG) {
        int g = t - MAXSA, sa = 0;   // (sa, t2), sa <= t2 < MAXSA, in the order of acc
        while (g >= MAXSA - sa) { g -= MAXSA - sa; ++sa; }
        const int t2 = sa + g;
        if (t2 < nsa) out[(nsa + sa * nsa - sa * (sa - 1) / 2 + (t2 - sa)) * nblk] = r;
    } else if (hasmp && t < NV) {
        // mean-profile terms, weighted by the band weights of this row:
        // w_j(y) sum v*_x (column 0) and w_j(y) sum V_s,x (column 1 + s)
        const int col = t - (MAXSA + NG);
        if (col == 0 || col - 1 < nsa) {
            const int o = nsa + nsa * (nsa + 1) / 2;
#pragma unroll
            for (int jm = 0; jm < kMaxQ; ++jm)
                if (jm < nmp) out[(o + jm * (1 + nsa) + col) * nblk] = wb[jm] * r;
        }
    }
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals.
// Counter (block, step_lo, step_hi, "LRS1"), key (seed_lo, seed_hi).
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The four normals of Philox block blk of a step: Box-Muller on the block's
// two pairs of uniforms.
__device__ inline void lrs_block_normals(unsigned long long seed, long long step, int blk, double* zz)
{
    uint32_t c[4] = {(uint32_t)blk, (uint32_t)(unsigned long long)step,
                     (uint32_t)((unsigned long long)step >> 32), 0x4C525331u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int p = 0; p < 2; ++p) {
        const double u1 = ((double)c[2 * p] + 0.5) * 2.3283064365386963e-10;
        const double u2 = ((double)c[2 * p + 1] + 0.5) * 2.3283064365386963e-10;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        zz[2 * p] = rad * cs;
        zz[2 * p + 1] = rad * sn;
    }
}

__device__ inline void lrs_normals(unsigned long long seed, long long step, int n, double* z)
{
    for (int blk = 0; 4 * blk < n; ++blk) {
        double zz[4];
        lrs_block_normals(seed, step, blk, zz);
        for (int k = 0; k < 4; ++k)
            if (4 * blk + k < n) z[4 * blk + k] = zz[k];
    }
}

__global__ void k_philox_test(const uint32_t* in, uint32_t* out, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
    philox4x32_10(c, in[6 * i + 4], in[6 * i + 5]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

__global__ void k_normals_test(unsigned long long seed, long long step0, int nsteps, int n, double* out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsteps) return;
    double z[kMaxQ];
    lrs_normals(seed, step0 + s, n, z);
    for (int k = 0; k < n; ++k) out[(size_t)s * n + k] = z[k];
}

// ---------------------------------------------------------------------------
// K2d: cross-block sums, one workgroup per (member, value slot).  Slots 0..3
// sum the statistics of the stream-collide workgroups, slots 4.. the TO
// partials of the reduce workgroups; the order is fixed by the member's own
// block counts.  Slot -1 makes the member's LRS draw of the step, slots
// -2 - c chunk c of the product of the LRS history with its rows of C.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sum(const DevMember* __restrict__ mems, const int2* __restrict__ work)
{
    __shared__ double red[kBlock / 64];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int slot = wk.y;
    if (slot == -1) {
        // the member's LRS draw for this step, off the solve's critical
        // path: normals xi (four per Philox block), then e = mu + L xi
        __shared__ double z[kMaxQ];
        KParam* prm = kc(m.prm);
        DevCtl* ctl = m.ctl;
        const long long step = ctl->step;
        if (prm->mode != LBM_CLOSURE_LRS || step < prm->spinup) return;   // uniform
        const int nq = prm->nq, tid = threadIdx.x;
        if (tid < (nq + 3) / 4) {
            double zz[4];
            lrs_block_normals(prm->seed, step, tid, zz);
            for (int k = 0; k < 4; ++k)
                if (4 * tid + k < nq) z[4 * tid + k] = zz[k];
        }
        __syncthreads();
        if (tid < nq) {
            double e = prm->mu[tid];
            for (int j = 0; j <= tid; ++j) e += prm->L[tid * kMaxQ + j] * z[j];
            ctl->lrs_e[tid] = e;
        }
        return;
    }
    if (slot < -1) {
        // history chunk c of the LRS product: sum over the x entries r in
        // [c kHistRows, (c+1) kHistRows) of x_r C[r][k], where x runs over
        // z^{n-1..n-h} then z*^{n-1..n-h} (z = q / s) from the record ring
        __shared__ double lds[kMaxQ * (kBlock / 64)];
        KParam* prm = kc(m.prm);
        DevCtl* ctl = m.ctl;
        const long long step = ctl->step;
        const int c = -2 - slot;
        if (prm->mode != LBM_CLOSURE_LRS || prm->h == 0 || c >= prm->nhc || step < prm->spinup) return;   // uniform
        const int nq = prm->nq, h = prm->h, rows = 2 * h * nq;
        double acc[kMaxQ];
#pragma unroll
        for (int k = 0; k < kMaxQ; ++k) acc[k] = 0.0;
#pragma unroll
        for (int u = 0; u < kHistRows / kBlock; ++u) {
            const int r = c * kHistRows + u * kBlock + threadIdx.x;
            if (r < rows) {
                const int b = r / nq, i = r % nq;
                const bool corr = b < h;                       // z^{n-1-b}, else z*^{n-1-(b-h)}
                const long long mstep = step - 1 - (corr ? b : b - h);
                const lbm_qoi_rec* rec = m.recs + (size_t)(mstep % m.rec_cap);
                double qv = rec->q[i];
                if (corr && !(rec->flags & 2)) qv += rec->dq[i];
                const double x = qv / prm->scale[i];
                const double* crow = prm->chist + (size_t)r * nq;
#pragma unroll
                for (int k = 0; k < kMaxQ; ++k)
                    if (k < nq) acc[k] += x * crow[k];
            }
        }
        const double v = block_sum_spread<kMaxQ>(acc, lds);
        if (threadIdx.x < nq) m.hpart[c * kMaxQ + threadIdx.x] = v;
        return;
    }
    if (slot >= 4 + m.npart) return;
    if (slot == 0 && threadIdx.x == 0) {
        // the step this launch belongs to, for a fused apply, and a first LRS
        // scale that the last fused apply left pending
        DevCtl* ctl = m.ctl;
        ctl->step_snap = ctl->step;
        if (ctl->s_pend) {
            for (int k = 0; k < kMaxQ; ++k) ctl->s[k] = ctl->s_next[k];
            ctl->s_set = 1;
            ctl->s_pend = 0;
        }
    }
    double v[1] = {0};
    if (slot < 4) {
#pragma unroll 8
        for (int b = threadIdx.x; b < m.nst; b += kBlock) v[0] += m.part_stats[(size_t)b * 4 + slot];
    } else {
        const int nblk = m.ny * m.nbx2;
        const double* p = m.part_to + (size_t)(slot - 4) * nblk;
#pragma unroll 8
        for (int b = threadIdx.x; b < nblk; b += kBlock) v[0] += p[b];
    }
    block_sum<1>(v, red);
    if (threadIdx.x == 0) m.sums[slot] = v[0];
}

// ---------------------------------------------------------------------------
// K3: the member's solve.  The QoI vector and Gram matrix from the
// fixed-order sums (k_sum), dQ, beta = G^-1 dQ and gamma_k = dQ_k (G^-1)_kk,
// the per-step record and the coefficients of the dv build.  Every input is
// first staged into LDS in one parallel pass, and all small matrices live
// there.  G is symmetric positive semi-definite, so Gauss-Jordan elimination
// needs no pivoting; its pivots are the squared Cholesky pivots, and G counts
// as singular when one of them is not above 1e-14 times the largest diagonal
// entry.  The elimination takes four pivots per barrier, ping-ponging between
// two copies of [G | I].
//
// It runs in one of two places.  k_solve: one workgroup per member, writing
// the coefficients, the record and the control state for k_apply.  Or in
// every workgroup of the binomial apply k_apply_fs (small launches), with
// the apply's own field loads in flight meanwhile, each workgroup forming
// the same coefficients from the same sums with the same arithmetic; there
// the member's first workgroup alone writes the record, advances the step
// counter and leaves a first LRS scale to be committed by the next step's
// k_sum, and every workgroup takes the step from the snapshot k_sum made of
// it, so no workgroup reads a value another one of the launch writes.
// ---------------------------------------------------------------------------
constexpr int kMaxSums = 4 + kMaxSA + kMaxSA * (kMaxSA + 1) / 2 + kMaxQ * (1 + kMaxSA);

struct SolveLds {
    double M[2][kMaxQ][2 * kMaxQ];
    double sf[kMaxSums];
    double Cs[(kMaxQ + 1) * kMaxQ], es[kMaxQ], hps[kMaxHistChunks * kMaxQ];
    double q[kMaxQ], dq[kMaxQ], beta[kMaxQ], gam[kMaxQ], sc[kMaxQ], qs[kMaxQ];
    double rrs[kMaxSA][kMaxPow + 1], gmps[kMaxQ * kMaxQ];
    double cv[kMaxPow + 1], cw[kMaxPow + 1];
    int kinds[kMaxSA], saslot[kMaxSA], mpslot[kMaxQ], mpband[kMaxQ];
    long long step;
    int sset, flags;
};

// ROLE 0: k_solve (every output, the step counter from ctl->step); 1: the
// leader of a fused apply (the record, the step counter, a pending scale);
// 2: another workgroup of a fused apply (LDS outputs only).  Every thread of
// the workgroup calls it; pre() issues the caller's loads right after the
// solve's own; S.cv, S.cw and S.beta hold the results.
template <int NTH, int ROLE, typename Pre>
__device__ void solve_member(KMember& m, SolveLds& S, Pre&& pre)
{
    static_assert(NTH == kBlock, "the solve runs on a whole workgroup");
    KParam* prm = kc(m.prm);
    DevCtl* ctl = m.ctl;
    const int tid = threadIdx.x;
    const int nq = prm->nq, nsa = prm->nsa, nmp = prm->nmp;
    const int ny = m.ny;
    const int nflat = nsa + nsa * (nsa + 1) / 2;
    const bool lrs = prm->mode == LBM_CLOSURE_LRS;

    // (a) stage the sums, the LRS model and the control state; clear M.
    // Every load's address and count come from the member record itself or
    // are fixed, none from a value loaded from the closure parameters, so
    // all of them are in flight after one dependent load.  They are issued
    // first, then the caller's own loads (pre), then stored to LDS: a wave's
    // loads complete in order, so the stores wait only for the solve's own.
    // (Measured on MI355X: the caller's loads issued after the staging
    // barrier instead are no faster.)
    static_assert(kMaxSums <= kBlock && kMaxQ * kMaxQ <= kBlock && kMaxSA * (kMaxPow + 1) <= kBlock &&
                  (kMaxQ + 1) * kMaxQ <= 2 * kBlock, "one or two staged values per thread");
    const double r_sf = tid < 4 + m.npart ? m.sums[tid] : 0.0;   // 4 + npart sums
    const double r_c0 = prm->C[tid];
    const double r_c1 = tid < (kMaxQ + 1) * kMaxQ - kBlock ? prm->C[kBlock + tid] : 0.0;
    const double r_g = prm->gmp[tid];
    const double r_rr = tid < kMaxSA * (kMaxPow + 1) ? (&prm->rr[0][0])[tid] : 0.0;
    double r_es = 0, r_s = 0;
    int r_kind = 0, r_sas = 0, r_mps = 0, r_mpb = 0;
    if (tid < kMaxQ) {
        r_es = ctl->lrs_e[tid];
        r_s = ctl->s[tid];
        r_mps = prm->mp_slot[tid];
        r_mpb = prm->mp_band[tid];
    }
    if (tid < kMaxSA) { r_kind = prm->sa_kind[tid]; r_sas = prm->sa_slot[tid]; }
    long long r_step = 0;
    int r_sset = 0, r_flags = 0;
    if (tid == 0) {
        r_step = ROLE == 0 ? ctl->step : ctl->step_snap;
        r_sset = ctl->s_set;
        r_flags = ctl->flags;
    }
    pre();
    if (tid < 4 + m.npart) S.sf[tid] = r_sf;
    S.Cs[tid] = r_c0;
    if (tid < (kMaxQ + 1) * kMaxQ - kBlock) S.Cs[kBlock + tid] = r_c1;
    S.gmps[tid] = r_g;
    if (tid < kMaxSA * (kMaxPow + 1)) (&S.rrs[0][0])[tid] = r_rr;
    if (tid < kMaxQ) {
        S.es[tid] = r_es;
        S.sc[tid] = r_s;
        S.mpslot[tid] = r_mps;
        S.mpband[tid] = r_mpb;
        S.q[tid] = 0; S.dq[tid] = 0; S.beta[tid] = 0; S.gam[tid] = 0;
    }
    if (tid < kMaxSA) { S.kinds[tid] = r_kind; S.saslot[tid] = r_sas; }
    if (tid == 0) {
        S.step = r_step;
        S.sset = r_sset;
        S.flags = r_flags;
    }
    if (lrs)
        for (int k = tid; k < prm->nhc * kMaxQ; k += NTH) S.hps[k] = m.hpart[k];
    for (int k = tid; k < 2 * kMaxQ * 2 * kMaxQ; k += NTH) (&S.M[0][0][0])[k] = 0.0;
    // band weights of row y = tid, used at the end (clamped index; loaded now
    // so that their latency overlaps the solve)
    double wv0[kMaxQ];
    if (ROLE == 0 && nmp > 0 && tid < ny) {
#pragma unroll
        for (int jm = 0; jm < kMaxQ; ++jm) wv0[jm] = m.bandw[(size_t)prm->mp_band[jm < nmp ? jm : nmp - 1] * ny + tid];
    }
    __syncthreads();
    const long long step = S.step;
    const bool active = step >= prm->spinup;
    // (b) assemble q and G (left half of M), the mean-profile entries and
    // the identity (right half)
    const double* sfp = S.sf + 4;
    if (tid < nsa) {
        const int s = tid;
        S.q[S.saslot[s]] = sfp[s];
        int g = nsa + s * nsa - s * (s - 1) / 2;
        for (int t = s; t < nsa; ++t, ++g) {
            S.M[0][S.saslot[s]][S.saslot[t]] = sfp[g];
            S.M[0][S.saslot[t]][S.saslot[s]] = sfp[g];
        }
    }
    for (int pr = tid; pr < nmp * (1 + nsa); pr += NTH) {
        const int jm = pr / (1 + nsa), c = pr % (1 + nsa);
        const double v = sfp[nflat + pr];
        const int uj = S.mpslot[jm];
        if (c == 0)
            S.q[uj] = v;
        else {
            const int us = S.saslot[c - 1];
            S.M[0][uj][us] = v;
            S.M[0][us][uj] = v;
        }
    }
    for (int pr = tid; pr < nmp * nmp; pr += NTH) {
        const int a = pr / nmp, b = pr % nmp;
        S.M[0][S.mpslot[a]][S.mpslot[b]] = S.gmps[a * kMaxQ + b];
    }
    if (tid < nq) S.M[0][tid][kMaxQ + tid] = 1.0;
    __syncthreads();
    // (c) dQ for tracking; the LRS scale (fixed at the first active step)
    if (active && tid < nq) {
        const int k = tid;
        if (prm->mode == LBM_CLOSURE_TRACK) {
            if (step < prm->nref) S.dq[k] = prm->qref[(size_t)step * nq + k] - S.q[k];
        } else if (lrs) {
            if (!S.sset) {
                S.sc[k] = prm->have_scale ? prm->scale[k] : (S.q[k] != 0.0 ? fabs(S.q[k]) : 1.0);
                if (ROLE == 0) ctl->s[k] = S.sc[k];
                if (ROLE == 1) ctl->s_next[k] = S.sc[k];
            }
            S.qs[k] = S.q[k] / S.sc[k];
        }
    }
    __syncthreads();
    // (d) the LRS draw: dQ = s (x C + e) - q*, with e = mu + L xi and the
    // history part of x C formed ahead of this kernel (k_sum); terms past nq
    // add exact zeros
    if (active && lrs && tid < nq) {
        const int k = tid;
        double zh = S.es[k];
        for (int c = 0; c < prm->nhc; ++c) zh += S.hps[c * kMaxQ + k];
#pragma unroll
        for (int i = 0; i < kMaxQ; ++i) {
            const int ic = i < nq ? i : 0;
            const double t = S.qs[ic] * S.Cs[ic * kMaxQ + k];
            zh += i < nq ? t : 0.0;
        }
        zh += S.Cs[nq * kMaxQ + k];
        S.dq[k] = S.sc[k] * zh - S.q[k];
    }
    // (e) Gauss-Jordan on [G | I] (only columns 0..nq-1 and kMaxQ..kMaxQ+nq-1
    // are nonzero), four pivots per barrier.  For pivot rows j0..j0+3 every
    // thread eliminates the 4x4 pivot block P in registers, applied to its
    // column's pivot-row entries r (t = P^-1 r, pivots in order, each checked
    // against the singular threshold; the block is identity-padded past nq),
    // then row i of its column becomes t_(i-j0) inside the block and
    // M[i][c] - sum_a M[i][j0+a] t_a outside it.  Every thread computes the
    // same pivots from the same values, so the singular flag is uniform.
    // The four eliminations of a block are those of four consecutive pivots.
    double mx = 0;
    for (int k = 0; k < nq; ++k) mx = fmax(mx, S.M[0][k][k]);
    int sing = mx > 0 ? 0 : 1;
    int cur = 0;
    // thread layout: one column of [G | I] each, rows split over the
    // NTH / (2 nq) groups of threads
    const int ncol = 2 * nq, ngrp = NTH / ncol;
    const int gcol = tid % ncol, grow = tid / ncol;
    const int cc = gcol < nq ? gcol : kMaxQ + gcol - nq;
    __syncthreads();
    for (int j0 = 0; j0 < nq && !sing; j0 += 4) {
        const int bs = min(4, nq - j0);   // rows j0..j0+3 stay inside M (nq <= kMaxQ)
        double P[4][4], t[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int b2 = 0; b2 < 4; ++b2) P[a][b2] = a < bs && b2 < bs ? S.M[cur][j0 + a][j0 + b2] : (a == b2 ? 1.0 : 0.0);
            t[a] = a < bs ? S.M[cur][j0 + a][cc] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double piv = P[a][a];
            if (a < bs && !(piv > 1e-14 * mx)) sing = 1;
            const double rp = 1.0 / piv;
#pragma unroll
            for (int b2 = a + 1; b2 < 4; ++b2) P[a][b2] *= rp;
            t[a] *= rp;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (e == a) continue;
                const double f = P[e][a];
#pragma unroll
                for (int b2 = a + 1; b2 < 4; ++b2) P[e][b2] -= f * P[a][b2];
                t[e] -= f * t[a];
            }
        }
        if (sing) break;   // uniform
        if (grow < ngrp) {
            for (int i = grow; i < nq; i += ngrp) {
                const int d = i - j0;
                double v;
                if (d >= 0 && d < bs) {
                    v = d == 0 ? t[0] : d == 1 ? t[1] : d == 2 ? t[2] : t[3];
                } else {
                    // past nq the block columns of M are zero and t is zero
                    v = S.M[cur][i][cc];
#pragma unroll
                    for (int a = 0; a < 4; ++a) v -= S.M[cur][i][j0 + a] * t[a];
                }
                S.M[cur ^ 1][i][cc] = v;
            }
        }
        cur ^= 1;
        __syncthreads();
    }
    // (f) beta = G^-1 dQ, gamma_k = dQ_k (G^-1)_kk
    if (!sing && tid < nq) {
        double b = 0;
        for (int j = 0; j < nq; ++j) b += S.M[cur][tid][kMaxQ + j] * S.dq[j];
        S.beta[tid] = b;
        S.gam[tid] = S.dq[tid] * S.M[cur][tid][kMaxQ + tid];
    }
    __syncthreads();
    // (g) dv coefficients, record, counters
    if (ROLE == 0 && tid < kMaxSA) {
        const double b = tid < nsa ? S.beta[S.saslot[tid]] : 0.0;
        ctl->bsa[tid] = b;
        ctl->bsaf[tid] = (float)b;
    }
    if (tid <= kMaxPow) {
        double a = 0, b = 0;
        for (int s = 0; s < nsa; ++s) {
            const double bs = S.beta[S.saslot[s]];
            if (S.kinds[s] == 0) a += bs * S.rrs[s][tid];
            else b += bs * S.rrs[s][tid];
        }
        S.cv[tid] = a;
        S.cw[tid] = b;
        if (ROLE == 0) {
            ctl->cv[tid] = a;
            ctl->cw[tid] = b;
            ctl->cvf[tid] = (float)a;
            ctl->cwf[tid] = (float)b;
        }
    }
    if (ROLE <= 1) {
        lbm_qoi_rec* rec = m.recs + (size_t)(step % m.rec_cap);
        if (tid < kMaxQ) {
            rec->q[tid] = tid < nq ? S.q[tid] : 0.0;
            rec->dq[tid] = tid < nq ? S.dq[tid] : 0.0;
            rec->gamma[tid] = tid < nq ? S.gam[tid] : 0.0;
        }
        if (tid == 0) {
            rec->step = step;
            rec->flags = (S.flags & 1) | (sing ? 2 : 0);
            rec->nq = nq;
            rec->mass = (double)m.N + S.sf[0];
            rec->mom[0] = S.sf[1];
            rec->mom[1] = S.sf[2];
            rec->mom[2] = S.sf[3];
            rec->diag_e = 0;
            rec->diag_z = 0;
            if (active && lrs && !S.sset) {
                if (ROLE == 0) ctl->s_set = 1;
                else ctl->s_pend = 1;
            }
            ctl->step = step + 1;
        }
    }
    // (h) mean-profile part of dv: cmp(y) = sum_j beta_mp_j w_j(y) (in a
    // fused apply every cell forms its own row's value)
    if (ROLE == 0) {
        if (nmp > 0) {
            for (int yy = tid; yy < ny; yy += NTH) {
                // all band-weight loads first (clamped index; terms past nmp add exact zeros)
                double wv[kMaxQ];
#pragma unroll
                for (int jm = 0; jm < kMaxQ; ++jm)
                    wv[jm] = yy == tid ? wv0[jm] : m.bandw[(size_t)S.mpband[jm < nmp ? jm : nmp - 1] * ny + yy];
                double c = 0;
#pragma unroll
                for (int jm = 0; jm < kMaxQ; ++jm) c += jm < nmp ? S.beta[S.mpslot[jm]] * wv[jm] : 0.0;
                m.cmp[yy] = c;
            }
        } else {
            for (int yy = tid; yy < ny; yy += NTH) m.cmp[yy] = 0.0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_solve(const DevMember* __restrict__ mems, const int* __restrict__ work)
{
    __shared__ SolveLds S;
    KMember& m = *kc(mems + work[blockIdx.x]);
    solve_member<kBlock, 0>(m, S, [] {});
}

// K4: dv = sum_j cv_j B^j v* + sum_j cw_j C_j + e_x cmp(y) (eq. TO-ansatz
// as sum_j beta_j V_j), and the SGS change of the cell's predictor
// populations delta f_i = feq_i(rho, v* + dv) - feq_i(rho, v*): DEF, the
// record (a, b) = (rho dv, 2 v* + dv) that the next stream-collide applies
// during its pull; otherwise added in place to the populations the
// stream-collide of this step wrote (the WALE substrate, whose velocity
// gradients need the complete post-streaming state).
template <typename T> __device__ __forceinline__ T coef_bsa(KCtl* c, int s);
template <> __device__ __forceinline__ float coef_bsa<float>(KCtl* c, int s) { return c->bsaf[s]; }
template <> __device__ __forceinline__ double coef_bsa<double>(KCtl* c, int s) { return c->bsa[s]; }

// One cell of the binomial apply: its fields (loaded by apply_load, the
// power clamped to the highest one stored: cv_j (cw_j) is zero above jv
// (jw), so the extra terms add exact zeros; the top C_jw from the
// neighbours of W_jw), and in place the populations the stream-collide of
// this step wrote.
template <int LAT, typename T, bool DEF>
struct ApplyIn {
    T fv[kMaxPow + 1][Lat<LAT>::D], fc[kMaxPow][Lat<LAT>::D];
    T nb[Lat<LAT>::D == 2 ? 4 : 12];   // W_jw at the neighbours the top curl takes
    bool okm, okp;                     // y neighbours inside the walls
    T rho1;                            // rho - 1
    T gi[DEF ? 1 : Lat<LAT>::Q];
};

template <int LAT, typename T, bool WT, bool DEF>
__device__ __forceinline__ void apply_load(KMember& m, KParam* prm, int flip, int cell, ApplyIn<LAT, T, DEF>& in)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    const int nx = m.nx, ny = m.ny;
    const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
    const size_t sN = (size_t)m.N;
    const int jv = prm->jv, jw = prm->jw;
    const T* __restrict__ vsp = (const T*)m.vs;
    if constexpr (!DEF) {
        const T* g = (const T*)m.g[m.parity ^ flip ^ 1];
#pragma unroll
        for (int i = 0; i < L::Q; ++i) in.gi[i] = ld_fld<WT>(g + pop_at64<L::Q>(i, (size_t)cell));
    }
#pragma unroll
    for (int jj = 0; jj <= kMaxPow; ++jj) {
        const int je = jj < jv ? jj : jv;
        const T* src = je == 0 ? vsp : (const T*)m.P + (size_t)(je - 1) * D * sN;
#pragma unroll
        for (int a = 0; a < D; ++a) in.fv[jj][a] = ld_fld<WT>(src + a * sN + cell);
    }
    if (prm->has_z) {
        top_curl_load<LAT, T>(m, jw, x, y, z, in.nb, in.okm, in.okp);
        const int jc = jw > 0 ? jw - 1 : 0;
#pragma unroll
        for (int jj = 0; jj < kMaxPow; ++jj) {
            const T* srcc = (const T*)m.C + (size_t)(jj < jc ? jj : jc) * D * sN;
#pragma unroll
            for (int a = 0; a < D; ++a) in.fc[jj][a] = ld_fld<WT>(srcc + a * sN + cell);
        }
    }
    in.rho1 = ((const T*)m.rho)[cell];
}

// The rest of the cell: the SGS change (rho dv, 2 v* + dv) from dv (out) and
// v*, stored as the record (DEF) or added in place to the populations.
template <int LAT, typename T, bool WT, bool DEF>
__device__ __forceinline__ void apply_finish(KMember& m, int flip, int cell, const T (&vs)[Lat<LAT>::D],
                                             const T (&out)[3], T rho1, const T* gi)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    const size_t sN = (size_t)m.N;
    const T rho = T(1) + rho1;
    T ra[D], rb[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ra[a] = rho * out[a];
        rb[a] = T(2) * vs[a] + out[a];
    }
    // (TO fields stay below 2^32 bytes: 32-bit offsets from scalar bases)
    if constexpr (DEF) {
        T* rec = (T*)m.rec;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            st_fld_at(rec + (size_t)a * sN, (unsigned)cell, ra[a], WT);
            st_fld_at(rec + (size_t)(D + a) * sN, (unsigned)cell, rb[a], WT);
        }
    } else {
        T* g = (T*)m.g[m.parity ^ flip ^ 1];
        const T e = rec_e<D, T>(ra, rb);
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st_fld(g + pop_at64<L::Q>(i, (size_t)cell),
                   add_df<LAT, T>(gi[i], i, [&](int k) { return ra[k]; }, [&](int k) { return rb[k]; }, e), WT);
    }
}

// dv of a binomial cell from its fields and the coefficients: sum_j cv_j
// B^j v* + sum_j cw_j C_j + e_x cmp(y).
template <int LAT, typename T, bool DEF>
__device__ __forceinline__ void apply_dv(const ApplyIn<LAT, T, DEF>& in, bool hz, int jw, const T (&cvc)[kMaxPow + 1],
                                         const T (&cwc)[kMaxPow + 1], bool hasmp, double cmp, T (&out)[3])
{
    constexpr int D = Lat<LAT>::D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T s = cvc[0] * in.fv[0][a];
#pragma unroll
        for (int jj = 1; jj <= kMaxPow; ++jj) s += cvc[jj] * in.fv[jj][a];
        out[a] = s;
    }
    if (hz) {
        T ctop[D];
        top_curl_eval<D, T>(in.nb, in.okm, in.okp, ctop);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T sacc = 0;
#pragma unroll
            for (int jj = 0; jj <= kMaxPow; ++jj) sacc += cwc[jj] * (jj < jw && jj < kMaxPow ? in.fc[jj < kMaxPow ? jj : 0][a] : ctop[a]);
            out[a] += sacc;
        }
    }
    if (hasmp) out[0] += T(cmp);
}

template <int LAT, typename T, bool KF, bool WT, bool DEF>
__global__ __launch_bounds__(kBlock) void k_apply(const DevMember* __restrict__ mems, const int2* __restrict__ work,
                                                  int flip)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    KParam* prm = kc(m.prm);
    const int N = m.N, nx = m.nx, ny = m.ny;
    const int cell = wk.y * kBlock + threadIdx.x;
    if (cell >= N) return;
    const int y = (cell / nx) % ny;
    KCtl* ctl = kc(m.ctl);
    T out[3] = {0, 0, 0};
    T vs[D];
    if constexpr (KF) {
        // dv = sum_s beta_s V_s (clamped loads; beta_s = 0 past nsa)
        const size_t sN = (size_t)N;
        const T* __restrict__ vsp = (const T*)m.vs;
        T gi[DEF ? 1 : L::Q];
        if constexpr (!DEF) {
            const T* g = (const T*)m.g[m.parity ^ flip ^ 1];
#pragma unroll
            for (int i = 0; i < L::Q; ++i) gi[i] = ld_fld<WT>(g + pop_at64<L::Q>(i, (size_t)cell));
        }
        const int nsa = prm->nsa;
        const T* __restrict__ kV = (const T*)m.kV;
#pragma unroll
        for (int a = 0; a < D; ++a) vs[a] = vsp[a * sN + cell];
        T kv[kMaxSA][D];
#pragma unroll
        for (int s2 = 0; s2 < kMaxSA; ++s2)
#pragma unroll
            for (int a = 0; a < D; ++a) kv[s2][a] = kV[((size_t)(s2 < nsa ? s2 : nsa - 1) * D + a) * sN + cell];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T acc = 0;
#pragma unroll
            for (int s2 = 0; s2 < kMaxSA; ++s2) acc += coef_bsa<T>(ctl, s2) * kv[s2][a];
            out[a] = acc;
        }
        if (prm->nmp > 0) out[0] += T(m.cmp[y]);
        apply_finish<LAT, T, WT, DEF>(m, flip, cell, vs, out, ((const T*)m.rho)[cell], gi);
    } else {
        ApplyIn<LAT, T, DEF> in;
        apply_load<LAT, T, WT, DEF>(m, prm, flip, cell, in);
        T cvc[kMaxPow + 1], cwc[kMaxPow + 1];
#pragma unroll
        for (int jj = 0; jj <= kMaxPow; ++jj) {
            cvc[jj] = coef_cv<T>(ctl, jj);
            cwc[jj] = coef_cw<T>(ctl, jj);
        }
        const bool hasmp = prm->nmp > 0;
        apply_dv<LAT, T, DEF>(in, prm->has_z, prm->jw, cvc, cwc, hasmp, hasmp ? m.cmp[y] : 0.0, out);
#pragma unroll
        for (int a = 0; a < D; ++a) vs[a] = in.fv[0][a];
        apply_finish<LAT, T, WT, DEF>(m, flip, cell, vs, out, in.rho1, in.gi);
    }
}

// The binomial apply with the member's solve at its head (launches of at
// most kFusedApplyPairs workgroups).  A workgroup takes a pair of
// blocks of one member (work entry (member, p): blocks 2p and 2p + 1), issues
// the loads of both cells of every thread, then solves on all its threads
// while they are in flight (two waves per SIMD: every workgroup of the launch
// is resident at once), and finishes both cells with the solve's
// coefficients; cmp(y) = sum_j beta_mp_j w_j(y) is formed per cell in the
// order and precision k_solve forms it.  Pair 0 is the member's leader.
template <int LAT, typename T, bool WT, bool DEF>
__global__ __launch_bounds__(kBlock, 2) void k_apply_fs(const DevMember* __restrict__ mems,
                                                         const int2* __restrict__ work, int flip)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    __shared__ SolveLds S;
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    KParam* prm = kc(m.prm);
    const int N = m.N, nx = m.nx, ny = m.ny;
    const int nmp = prm->nmp;
    int cells[2];
    bool own[2];
    ApplyIn<LAT, T, DEF> in[2];
    double wv[2][kMaxQ];
    // the cells' loads, issued right after the solve's own
    auto load = [&] {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = (2 * wk.y + u) * kBlock + threadIdx.x;
            own[u] = c < N;
            cells[u] = own[u] ? c : 0;   // a thread past the grid loads cell 0 and stores nothing
            apply_load<LAT, T, WT, DEF>(m, prm, flip, cells[u], in[u]);
            const int y = (cells[u] / nx) % ny;
            if (nmp > 0) {
#pragma unroll
                for (int jm = 0; jm < kMaxQ; ++jm)
                    wv[u][jm] = jm < nmp ? m.bandw[(size_t)prm->mp_band[jm] * ny + y] : 0.0;
            }
        }
    };
    if (wk.y == 0) solve_member<kBlock, 1>(m, S, load);
    else solve_member<kBlock, 2>(m, S, load);
    __syncthreads();   // S.cv and S.cw of (g)
    T cvc[kMaxPow + 1], cwc[kMaxPow + 1];
#pragma unroll
    for (int jj = 0; jj <= kMaxPow; ++jj) {
        cvc[jj] = T(S.cv[jj]);
        cwc[jj] = T(S.cw[jj]);
    }
    const bool hz = prm->has_z;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (!own[u]) continue;
        double cmp = 0;
        if (nmp > 0) {
#pragma unroll
            for (int jm = 0; jm < kMaxQ; ++jm) cmp += jm < nmp ? S.beta[S.mpslot[jm]] * wv[u][jm] : 0.0;
        }
        T out[3] = {0, 0, 0};
        apply_dv<LAT, T, DEF>(in[u], hz, prm->jw, cvc, cwc, nmp > 0, cmp, out);
        T vs[D];
#pragma unroll
        for (int a = 0; a < D; ++a) vs[a] = in[u].fv[0][a];
        apply_finish<LAT, T, WT, DEF>(m, flip, cells[u], vs, out, in[u].rho1, in[u].gi);
    }
}

// A pending SGS change (the records of the last step) added in place to the
// current populations g[parity ^ flip], and the records cleared, so the state
// can be read or replaced (checkpoints, fields, a closure change).
template <int LAT, typename T>
__global__ __launch_bounds__(kBlock) void k_flush(const DevMember* __restrict__ mems, const int2* __restrict__ work,
                                                  int flip)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N;
    const int cell = wk.y * kBlock + threadIdx.x;
    if (cell >= N) return;
    const size_t sN = (size_t)N;
    T* rec = (T*)m.rec;
    T ra[D], rb[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ra[a] = rec[a * sN + cell];
        rb[a] = rec[(D + a) * sN + cell];
    }
    const T e = rec_e<D, T>(ra, rb);
    T* g = (T*)m.g[m.parity ^ flip];
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        g[pop_at64<L::Q>(i, (size_t)cell)] = add_df<LAT, T>(g[pop_at64<L::Q>(i, (size_t)cell)], i,
                                                             [&](int k) { return ra[k]; },
                                                             [&](int k) { return rb[k]; }, e);
#pragma unroll
    for (int a = 0; a < 2 * D; ++a) rec[a * sN + cell] = T(0);
}

// ---------------------------------------------------------------------------
// Kernel filters (Sec. 4.1, eq. gaussian and eq. laplace): each filter is a
// sum of separable terms, applied as 1-D passes along x, y and z; every
// QoI's and every term's pass of the same depth runs in one launch.
// ---------------------------------------------------------------------------
// K2k: one level of the program: job blockIdx.y, cells of block blockIdx.x.
// op 0: dst = sum_t coef_t sum_r taps_t[r] src_t(. + r e_axis), periodic wrap
// or zero padding on the wall axis; op 1: the adjoint curl (2-D:
// (D_y psi, -D_x psi); 3-D: curl psi) with the wall padding of curl_at.
template <int LAT, typename T, bool WT>
__global__ __launch_bounds__(kBlock) void k_kjob(const DevMember* __restrict__ mems, const int2* __restrict__ work,
                                                 const KJob* __restrict__ jobs)
{
    using L = Lat<LAT>;
    const LBM_K KJob& j = *kc(jobs + blockIdx.y);
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N, nx = m.nx, ny = m.ny, nz = m.nz;
    const int cell = wk.y * kBlock + threadIdx.x;
    if (cell >= N) return;
    const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
    T* __restrict__ dst = (T*)j.dst;
    if (j.op == 0) {
        const int axis = j.axis;
        const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
        const int pos = axis == 0 ? x : (axis == 1 ? y : z);
        const int stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
        const bool pad = axis == 1 && m.walls;
        const size_t line = (size_t)cell - (size_t)pos * stride;   // first cell of this cell's line
        // all components at once (up to three load streams in flight; a
        // component past ncomp re-reads component 0 and is not stored)
        const int nc = j.ncomp;
        const size_t o1 = nc > 1 ? (size_t)N : 0, o2 = nc > 2 ? 2 * (size_t)N : 0;
        T out[3] = {0, 0, 0};
        for (int tt = 0; tt < j.nterm; ++tt) {
            const T* __restrict__ sc = (const T*)j.src[tt] + line;
            const LBM_K T* tp = kc((const T*)j.taps[tt]);   // uniform: scalar loads
            const int rad = j.radius[tt];
            T s0 = 0, s1 = 0, s2 = 0;
            if (pos - rad >= 0 && pos + rad < n) {
                // the whole stencil inside the line: no wrap, no padding
                const T* __restrict__ q = sc + (size_t)(pos - rad) * stride;
#pragma unroll 2
                for (int r = 0; r <= 2 * rad; ++r) {
                    const T t = tp[r];
                    const size_t k = (size_t)r * stride;
                    s0 += t * q[k];
                    s1 += t * q[o1 + k];
                    s2 += t * q[o2 + k];
                }
            } else {
                for (int r = -rad; r <= rad; ++r) {
                    int p = pos + r;
                    if (pad) {
                        if (p < 0 || p >= n) continue;
                    } else {
                        p %= n;
                        if (p < 0) p += n;
                    }
                    const T t = tp[r + rad];
                    const size_t k = (size_t)p * stride;
                    s0 += t * sc[k];
                    s1 += t * sc[o1 + k];
                    s2 += t * sc[o2 + k];
                }
            }
            const T cf = T(j.coef[tt]);
            out[0] += cf * s0;
            out[1] += cf * s1;
            out[2] += cf * s2;
        }
        st_fld(dst + cell, out[0], WT);
        if (nc > 1) st_fld(dst + (size_t)N + cell, out[1], WT);
        if (nc > 2) st_fld(dst + 2 * (size_t)N + cell, out[2], WT);
        return;
    }
    const T* __restrict__ src = (const T*)j.src[0];
    if constexpr (L::D == 2) {
        dst[cell] = T(0.5) * (fld(src, x, y + 1, z, nx, ny, nz, m.walls) - fld(src, x, y - 1, z, nx, ny, nz, m.walls));
        dst[(size_t)N + cell] =
            -T(0.5) * (fld(src, x + 1, y, z, nx, ny, nz, m.walls) - fld(src, x - 1, y, z, nx, ny, nz, m.walls));
    } else {
        T w[3];
        curl_at<3, T>(src, (size_t)N, x, y, z, nx, ny, nz, m.walls, w);
        for (int a = 0; a < 3; ++a) dst[(size_t)a * N + cell] = w[a];
    }
}

// ---------------------------------------------------------------------------
// Sharp Fourier band filters (eq. scale-aware-energy-fourier) through hipFFT:
// real fields into complex ones, forward transforms, per QoI the band mask
// (l - 1/2 <= |k| < m + 1/2, integer mode indices; with the 1/N of the
// inverse transform), the inverse transform and the real part.
// ---------------------------------------------------------------------------
template <typename T, typename CT>
__global__ __launch_bounds__(kBlock) void k_fpack(const T* __restrict__ src, CT* __restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    CT c;
    c.x = src[i];
    c.y = T(0);
    dst[i] = c;
}

struct FBands { int nb, l[kMaxBands], m[kMaxBands]; };
template <typename T> struct FDst { T* d[kMaxBands]; };

// the masked spectrum of every band, out[b][comp][cell]
template <typename T, typename CT>
__global__ __launch_bounds__(kBlock) void k_fmask(const CT* __restrict__ spec, CT* __restrict__ out, int ncomp,
                                                  int nx, int ny, int nz, FBands bands)
{
    const size_t N = (size_t)nx * ny * nz;
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N * ncomp) return;
    const size_t cell = i % N;
    const int jx = (int)(cell % nx), jy = (int)((cell / nx) % ny), jz = (int)(cell / ((size_t)nx * ny));
    const int kx = jx <= nx / 2 ? jx : jx - nx, ky = jy <= ny / 2 ? jy : jy - ny, kz = jz <= nz / 2 ? jz : jz - nz;
    const double kn = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
    const CT c = spec[i];
    for (int b = 0; b < bands.nb; ++b) {
        const bool keep = kn >= bands.l[b] - 0.5 && kn < bands.m[b] + 0.5;
        const T s = keep ? T(1.0 / (double)N) : T(0);
        CT o;
        o.x = c.x * s;
        o.y = c.y * s;
        out[(size_t)b * ncomp * N + i] = o;
    }
}

// the real parts of the inverse transforms into each band's destination
template <typename T, typename CT>
__global__ __launch_bounds__(kBlock) void k_funpack(const CT* __restrict__ src, FDst<T> dst, int nb, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n * nb) return;
    dst.d[i / n][i % n] = src[i].x;
}

template <int LAT, typename T>
static void launch_fourier(const FourierProg& f, hipStream_t st)
{
    using L = Lat<LAT>;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    using CT = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    const size_t N = (size_t)nx * ny * nz;
    const dim3 blk(kBlock);
    auto grid = [&](size_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); };
    auto exec = [&](void* plan, void* data, int dir) {
        hipfftHandle h = (hipfftHandle)plan;
        hipfftResult r = hipfftSetStream(h, st);
        if (r == HIPFFT_SUCCESS) {
            if constexpr (std::is_same<T, float>::value)
                r = hipfftExecC2C(h, (hipfftComplex*)data, (hipfftComplex*)data, dir);
            else
                r = hipfftExecZ2Z(h, (hipfftDoubleComplex*)data, (hipfftDoubleComplex*)data, dir);
        }
        if (r != HIPFFT_SUCCESS) f.failed = 1;
    };
    for (int kind = 0; kind < 2; ++kind) {   // E bands (of v*), then Z bands (of w)
        const std::vector<FourierQ>& qs = kind == 0 ? f.qe : f.qz;
        if (qs.empty()) continue;
        const int nc = kind == 0 ? L::D : L::NC;
        void* spec = kind == 0 ? f.spec_v : f.spec_w;
        void* band = kind == 0 ? f.band_e : f.band_z;
        hipLaunchKernelGGL((k_fpack<T, CT>), grid(nc * N), blk, 0, st, (const T*)(kind == 0 ? f.vs : f.w), (CT*)spec,
                           nc * N);
        exec(f.plan[kind], spec, HIPFFT_FORWARD);
        FBands fb{};
        FDst<T> fd{};
        fb.nb = (int)qs.size();
        for (size_t b = 0; b < qs.size(); ++b) {
            fb.l[b] = qs[b].l;
            fb.m[b] = qs[b].m;
            fd.d[b] = (T*)qs[b].dst;
        }
        hipLaunchKernelGGL((k_fmask<T, CT>), grid(nc * N), blk, 0, st, (const CT*)spec, (CT*)band, nc, nx, ny, nz, fb);
        exec(f.plan[2 + kind], band, HIPFFT_BACKWARD);
        hipLaunchKernelGGL((k_funpack<T, CT>), grid(qs.size() * nc * N), blk, 0, st, (const CT*)band, fd, fb.nb,
                           nc * N);
    }
}

// ---------------------------------------------------------------------------
// Diagnostics of plain runs: E and Z of the post-streaming velocity.
// ---------------------------------------------------------------------------
template <int LAT, typename T>
__global__ __launch_bounds__(kBlock) void k_diag(const DevMember* __restrict__ mems, const int2* __restrict__ work)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
    __shared__ double lds[2 * (kBlock / 64)];
    const int2 wk = work[blockIdx.x];
    KMember& m = *kc(mems + wk.x);
    const int N = m.N, nx = m.nx, ny = m.ny, nz = m.nz;
    const int cell = wk.y * kBlock + threadIdx.x;
    double v[2] = {0, 0};
    if (cell < N) {
        const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
        const T* vn = (const T*)m.vn;
        double e = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double u = (double)vn[(size_t)a * N + cell];
            e += 0.5 * u * u;
        }
        T w[3];
        curl_at<D, T>(vn, (size_t)N, x, y, z, nx, ny, nz, m.walls, w);
        double zz = 0;
#pragma unroll
        for (int a = 0; a < L::NC; ++a) zz += 0.5 * (double)w[a] * (double)w[a];
        v[0] = e;
        v[1] = zz;
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        m.part_diag[(size_t)wk.y * 2] = v[0];
        m.part_diag[(size_t)wk.y * 2 + 1] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_fin_diag(const DevMember* __restrict__ mems, const int* __restrict__ work)
{
    __shared__ double red[6 * (kBlock / 64)];
    KMember& m = *kc(mems + work[blockIdx.x]);
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < m.nb1; b += kBlock) {
        for (int k = 0; k < 4; ++k) v[k] += m.part_stats[(size_t)b * 4 + k];
        v[4] += m.part_diag[(size_t)b * 2];
        v[5] += m.part_diag[(size_t)b * 2 + 1];
    }
    block_sum<6>(v, red);
    if (threadIdx.x == 0) {
        DevCtl* ctl = m.ctl;
        const long long step = ctl->step;
        lbm_qoi_rec* rec = m.recs + (size_t)(step % m.rec_cap);
        rec->step = step;
        rec->flags = ctl->flags & 1;
        rec->nq = 0;
        rec->mass = (double)m.N + v[0];
        rec->mom[0] = v[1];
        rec->mom[1] = v[2];
        rec->mom[2] = v[3];
        rec->diag_e = v[4];
        rec->diag_z = v[5];
        for (int k = 0; k < kMaxQ; ++k) { rec->q[k] = 0; rec->dq[k] = 0; rec->gamma[k] = 0; }
        ctl->step = step + 1;
    }
}

// ---------------------------------------------------------------------------
// State access kernels.
// ---------------------------------------------------------------------------
template <int LAT, typename T, int PREC>
__global__ void k_init(const DevMember* __restrict__ mems, int flip, const double* __restrict__ rho0,
                       const double* __restrict__ u0)
{
    using L = Lat<LAT>;
    KMember& m = *kc(mems);
    const int N = m.N;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    T* g = (T*)m.g[m.parity ^ flip];
    const double r = rho0 ? rho0[cell] : 1.0;
    double u[3] = {0, 0, 0}, uu = 0;
    for (int a = 0; a < L::D; ++a) { u[a] = u0 ? u0[(size_t)a * N + cell] : 0.0; uu += u[a] * u[a]; }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double cu = L::cx[i] * u[0] + L::cy[i] * u[1] + L::cz[i] * u[2];
        const double X = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
        const double feq = L::w[i] * r * (1.0 + X);
        g[pop_at64<L::Q>(i, (size_t)cell)] = PREC == LBM_FP32_PLAIN ? (T)feq : (T)(L::w[i] * ((r - 1.0) + r * X));
    }
    if (m.has_to) {
        ((T*)m.rho)[cell] = 0;
        for (int a = 0; a < L::D; ++a) ((T*)m.vs)[(size_t)a * N + cell] = 0;
    }
}

template <int LAT, typename T, int PREC>
__global__ void k_get_pop(const DevMember* __restrict__ mems, int flip, double* __restrict__ f)
{
    using L = Lat<LAT>;
    KMember& m = *kc(mems);
    const int N = m.N;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const T* g = (const T*)m.g[m.parity ^ flip];
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        f[(size_t)i * N + cell] = (double)g[pop_at64<L::Q>(i, (size_t)cell)] + (PREC == LBM_FP32_PLAIN ? 0.0 : L::w[i]);
}

template <int LAT, typename T, int PREC>
__global__ void k_set_pop(const DevMember* __restrict__ mems, int flip, const double* __restrict__ f)
{
    using L = Lat<LAT>;
    KMember& m = *kc(mems);
    const int N = m.N;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    T* g = (T*)m.g[m.parity ^ flip];
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        g[pop_at64<L::Q>(i, (size_t)cell)] = (T)(f[(size_t)i * N + cell] - (PREC == LBM_FP32_PLAIN ? 0.0 : L::w[i]));
    if (m.has_to) {
        ((T*)m.rho)[cell] = 0;
        for (int a = 0; a < L::D; ++a) ((T*)m.vs)[(size_t)a * N + cell] = 0;
    }
}

// Wall-anchored stride-m projection (Sec. 3, the projection phi_m; Sec. 7.1
// for the channel): coarse cell (i, j, k) takes the fine cell
// (m i + o, m j + o, m k + o), o = (m - 1) / 2, so the coarse walls, half a
// coarse cell beyond the first and last coarse rows, coincide with the fine
// ones.  Writes the full populations (nullable fpop [Q][Nc]) and the velocity
// sum c f / sum f of the post-collision state (nullable vout [D][Nc]).
template <int LAT, typename T, int PREC>
__global__ __launch_bounds__(kBlock) void k_project(const DevMember* __restrict__ fine, int flip, int m, int ncx,
                                                    int ncy, int ncz, double* __restrict__ fpop,
                                                    void* __restrict__ vout, int vout_fp64, int kind)
{
    using L = Lat<LAT>;
    KMember& F = *kc(fine);
    const int Nc = ncx * ncy * ncz;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= Nc) return;
    const int i = cell % ncx, t = cell / ncx, j = t % ncy, k = t / ncy;
    const int o = (m - 1) / 2;
    if (L::D == 2 && kind == LBM_PROJ_BICUBIC) {
        // bicubic (2-D, doubly periodic): the weighted mean over fine cells
        // (m i + o + rx, m j + o + ry), |rx|, |ry| < 2 m, with weights
        // K(rx / m) K(ry / m) / S^2, K the Keys cubic (a = -1/2), S the sum
        // of K(r / m) over the window; of the populations, and of the
        // velocity of each fine cell
        const int R = 2 * m - 1;
        auto keys = [](double x) {
            x = fabs(x);
            return x <= 1.0 ? (1.5 * x - 2.5) * x * x + 1.0 : (x < 2.0 ? ((-0.5 * x + 2.5) * x - 4.0) * x + 2.0 : 0.0);
        };
        double S = 0;
        for (int r = -R; r <= R; ++r) S += keys((double)r / m);
        const double rS = 1.0 / S;
        const T* g = (const T*)F.g[F.parity ^ flip];
        double acc[L::Q], uacc[2] = {0, 0};
#pragma unroll
        for (int q = 0; q < L::Q; ++q) acc[q] = 0;
        for (int ry = -R; ry <= R; ++ry) {
            const double wy = keys((double)ry / m) * rS;
            const int yf = modi(m * j + o + ry, F.ny);
            for (int rx = -R; rx <= R; ++rx) {
                const double w = wy * keys((double)rx / m) * rS;
                const size_t fc = (size_t)yf * F.nx + (size_t)modi(m * i + o + rx, F.nx);
                double drho = 0, jx = 0, jy = 0;
#pragma unroll
                for (int q = 0; q < L::Q; ++q) {
                    const double gq = (double)g[pop_at64<L::Q>(q, fc)];
                    acc[q] += w * gq;
                    drho += gq;
                    jx += L::cx[q] * gq;
                    jy += L::cy[q] * gq;
                }
                const double rho = PREC == LBM_FP32_PLAIN ? drho : 1.0 + drho;
                uacc[0] += w * (jx / rho);
                uacc[1] += w * (jy / rho);
            }
        }
        if (fpop) {
#pragma unroll
            for (int q = 0; q < L::Q; ++q) fpop[(size_t)q * Nc + cell] = acc[q] + (PREC == LBM_FP32_PLAIN ? 0.0 : L::w[q]);
        }
        if (vout) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (vout_fp64) ((double*)vout)[(size_t)a * Nc + cell] = uacc[a];
                else ((float*)vout)[(size_t)a * Nc + cell] = (float)uacc[a];
            }
        }
        return;
    }
    const int zf = L::D == 3 ? m * k + o : 0;
    const size_t fc = ((size_t)zf * F.ny + (size_t)(m * j + o)) * F.nx + (size_t)(m * i + o);
    const T* g = (const T*)F.g[F.parity ^ flip];
    double drho = 0, jm[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const double gq = (double)g[pop_at64<L::Q>(q, fc)];
        if (fpop) fpop[(size_t)q * Nc + cell] = gq + (PREC == LBM_FP32_PLAIN ? 0.0 : L::w[q]);
        drho += gq;
        jm[0] += L::cx[q] * gq;
        jm[1] += L::cy[q] * gq;
        jm[2] += L::cz[q] * gq;
    }
    if (vout) {
        // shifted storage: rho - 1 = sum g and rho v = sum c g (sum c w = 0)
        const double rho = PREC == LBM_FP32_PLAIN ? drho : 1.0 + drho;
#pragma unroll
        for (int a = 0; a < L::D; ++a) {
            const double u = jm[a] / rho;
            if (vout_fp64) ((double*)vout)[(size_t)a * Nc + cell] = u;
            else ((float*)vout)[(size_t)a * Nc + cell] = (float)u;
        }
    }
}

// The bicubic velocity projection in two separable passes (the reference
// QoIs of the Kolmogorov case): x, for every fine row yf and coarse column
// i, the weighted sum over the fine columns of the fine-cell velocities
// into tmp [2][fny][ncx]; then y, for every coarse cell, the weighted sum
// of tmp over the fine rows.  Weights as in k_project.
__device__ __forceinline__ double keys_w(int r, int m, double rS)
{
    const double x = fabs((double)r / m);
    return (x <= 1.0 ? (1.5 * x - 2.5) * x * x + 1.0 : (x < 2.0 ? ((-0.5 * x + 2.5) * x - 4.0) * x + 2.0 : 0.0)) * rS;
}

template <typename T, int PREC>
__global__ __launch_bounds__(kBlock) void k_proj_bx(const DevMember* __restrict__ fine, int flip, int m, int ncx,
                                                    double rS, double* __restrict__ tmp)
{
    using L = Lat<LBM_D2Q9>;
    KMember& F = *kc(fine);
    const int n = F.ny * ncx;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = idx % ncx, yf = idx / ncx;
    const int o = (m - 1) / 2, R = 2 * m - 1;
    const T* g = (const T*)F.g[F.parity ^ flip];
    double ux = 0, uy = 0;
    for (int rx = -R; rx <= R; ++rx) {
        const size_t fc = (size_t)yf * F.nx + (size_t)modi(m * i + o + rx, F.nx);
        double drho = 0, jx = 0, jy = 0;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const double gq = (double)g[pop_at64<L::Q>(q, fc)];
            drho += gq;
            jx += L::cx[q] * gq;
            jy += L::cy[q] * gq;
        }
        const double rho = PREC == LBM_FP32_PLAIN ? drho : 1.0 + drho;
        const double w = keys_w(rx, m, rS);
        ux += w * (jx / rho);
        uy += w * (jy / rho);
    }
    tmp[idx] = ux;
    tmp[(size_t)n + idx] = uy;
}

__global__ __launch_bounds__(kBlock) void k_proj_by(int m, int ncx, int ncy, int fny, double rS,
                                                    const double* __restrict__ tmp, void* __restrict__ vout,
                                                    int vout_fp64)
{
    const int Nc = ncx * ncy;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= Nc) return;
    const int i = cell % ncx, j = cell / ncx;
    const int o = (m - 1) / 2, R = 2 * m - 1;
    const size_t n = (size_t)fny * ncx;
    double v[2] = {0, 0};
    for (int ry = -R; ry <= R; ++ry) {
        const size_t t = (size_t)modi(m * j + o + ry, fny) * ncx + i;
        const double w = keys_w(ry, m, rS);
        v[0] += w * tmp[t];
        v[1] += w * tmp[n + t];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (vout_fp64) ((double*)vout)[(size_t)a * Nc + cell] = v[a];
        else ((float*)vout)[(size_t)a * Nc + cell] = (float)v[a];
    }
}

void launch_project(int lattice, int precision, const DevMember* fine, int flip, int m, int ncx, int ncy, int ncz,
                    double* fpop, void* vout, int vout_fp64, int kind, hipStream_t st, double* tmp)
{
    const int Nc = ncx * ncy * ncz;
    const dim3 blk(kBlock), grd((Nc + kBlock - 1) / kBlock);
    if (kind == LBM_PROJ_BICUBIC && !fpop && tmp && lattice == LBM_D2Q9) {
        double S = 0;   // the sum of the window's kernel values (host copy of k_project's)
        for (int r = -(2 * m - 1); r <= 2 * m - 1; ++r) {
            const double x = std::fabs((double)r / m);
            S += x <= 1.0 ? (1.5 * x - 2.5) * x * x + 1.0 : (x < 2.0 ? ((-0.5 * x + 2.5) * x - 4.0) * x + 2.0 : 0.0);
        }
        const int fny = ncy * m, nx1 = fny * ncx;
        const dim3 g1((nx1 + kBlock - 1) / kBlock);
        if (precision == LBM_FP64)
            hipLaunchKernelGGL((k_proj_bx<double, LBM_FP64>), g1, blk, 0, st, fine, flip, m, ncx, 1.0 / S, tmp);
        else if (precision == LBM_FP32_PLAIN)
            hipLaunchKernelGGL((k_proj_bx<float, LBM_FP32_PLAIN>), g1, blk, 0, st, fine, flip, m, ncx, 1.0 / S, tmp);
        else
            hipLaunchKernelGGL((k_proj_bx<float, LBM_FP32_SHIFTED>), g1, blk, 0, st, fine, flip, m, ncx, 1.0 / S, tmp);
        hipLaunchKernelGGL(k_proj_by, grd, blk, 0, st, m, ncx, ncy, fny, 1.0 / S, (const double*)tmp, vout, vout_fp64);
        return;
    }
#define LBM_PROJ(LAT, T, PREC)                                                                                    \
    hipLaunchKernelGGL((k_project<LAT, T, PREC>), grd, blk, 0, st, fine, flip, m, ncx, ncy, ncz, fpop, vout, vout_fp64, \
                       kind)
    switch (lattice * 3 + precision) {
    case LBM_D2Q9 * 3 + LBM_FP32_SHIFTED: LBM_PROJ(LBM_D2Q9, float, LBM_FP32_SHIFTED); break;
    case LBM_D2Q9 * 3 + LBM_FP64: LBM_PROJ(LBM_D2Q9, double, LBM_FP64); break;
    case LBM_D2Q9 * 3 + LBM_FP32_PLAIN: LBM_PROJ(LBM_D2Q9, float, LBM_FP32_PLAIN); break;
    case LBM_D3Q19 * 3 + LBM_FP32_SHIFTED: LBM_PROJ(LBM_D3Q19, float, LBM_FP32_SHIFTED); break;
    case LBM_D3Q19 * 3 + LBM_FP64: LBM_PROJ(LBM_D3Q19, double, LBM_FP64); break;
    case LBM_D3Q19 * 3 + LBM_FP32_PLAIN: LBM_PROJ(LBM_D3Q19, float, LBM_FP32_PLAIN); break;
    }
#undef LBM_PROJ
}

// Pure streaming (no collision) into the other buffer.
template <int LAT, typename T, bool TO>
__global__ void k_stream_only(const DevMember* __restrict__ mems, int flip)
{
    using L = Lat<LAT>;
    KMember& m = *kc(mems);
    const int N = m.N, nx = m.nx, ny = m.ny;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const int x = cell % nx, t = cell / nx, y = t % ny, z = t / ny;
    T f[L::Q];
    gather<LAT, T, false>(m, (const T*)m.g[m.parity ^ flip], x, y, z, cell, f);
    T* gd = (T*)m.g[m.parity ^ flip ^ 1];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) gd[pop_at64<L::Q>(i, (size_t)cell)] = f[i];
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side), one instantiation per lattice/precision/kind.
// ---------------------------------------------------------------------------
template <int LAT, typename T, int PREC>
static void launch_step_group(const LaunchGroup& g, hipStream_t st, int flip, hipEvent_t* ev)
{
    const dim3 blk(kBlock);
    if (g.nb1 == 0) return;
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    if (g.probe) goto to_chain;
    if (g.substrate == LBM_WALE) {
        if (g.mode == 2)
            hipLaunchKernelGGL((k_moments<LAT, T, PREC, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip,
                               (double*)nullptr, (double*)nullptr);
        else
            hipLaunchKernelGGL((k_moments<LAT, T, PREC, false>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip,
                               (double*)nullptr, (double*)nullptr);
    }
#define LBM_STEP_T(SUB, TXV)                                                                               \
    do {                                                                                                   \
        if (!g.a32)                                                                                        \
            hipLaunchKernelGGL((k_step_t<LAT, T, PREC, SUB, TXV, false, false>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, \
                               g.mems, g.workb, flip);                                                     \
        else if (g.wt)                                                                                     \
            hipLaunchKernelGGL((k_step_t<LAT, T, PREC, SUB, TXV, true>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems,  \
                               g.workb, flip);                                                             \
        else                                                                                               \
            hipLaunchKernelGGL((k_step_t<LAT, T, PREC, SUB, TXV, false>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems, \
                               g.workb, flip);                                                             \
    } while (0)
#define LBM_STEP_SUB(SUB)                                                                                  \
    do {                                                                                                   \
        if constexpr (SUB != LBM_WALE) {                                                                   \
            if (g.mode == 2 && g.defer) {                                                                  \
                if (Lat<LAT>::D == 3 && g.btx == kBinTXW)                                                  \
                    LBM_STEP_T(SUB, (Lat<LAT>::D == 3 ? kBinTXW : kBinTX));                                \
                else                                                                                       \
                    LBM_STEP_T(SUB, kBinTX);                                                               \
                break;                                                                                     \
            }                                                                                              \
        }                                                                                                  \
        if (g.mode == 2 && !g.a32)                                                                         \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 2, false, false>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.mode == 2 && g.wt)                                                                      \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 2, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.mode == 2)                                                                              \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 2>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.mode == 1 && g.a32)                                                                     \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 1, false, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.mode == 1)                                                                              \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 1>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.a32 && g.nt)                                                                            \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 0, false, true, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.a32)                                                                                    \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 0, false, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else if (g.nt)                                                                                     \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 0, false, false, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else                                                                                               \
            hipLaunchKernelGGL((k_step<LAT, T, PREC, SUB, 0>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
    } while (0)
    if (g.substrate == LBM_SMAGORINSKY)
        LBM_STEP_SUB(LBM_SMAGORINSKY);
    else if (g.substrate == LBM_WALE)
        LBM_STEP_SUB(LBM_WALE);
    else
        LBM_STEP_SUB(LBM_BGK);
#undef LBM_STEP_SUB
#undef LBM_STEP_T
to_chain:
    mark(1);
    if (g.mode == 2) {
        if (g.kf && g.any_z) {   // the binomial chains form w in their first pass
            if (g.wt) hipLaunchKernelGGL((k_curl<LAT, T, true>), dim3(g.nb1), blk, 0, st, g.mems, g.work1);
            else hipLaunchKernelGGL((k_curl<LAT, T, false>), dim3(g.nb1), blk, 0, st, g.mems, g.work1);
        }
        mark(2);
        if (g.kf) {
            if (g.fprog) launch_fourier<LAT, T>(*g.fprog, st);
            for (int l = 0; l < g.nklev; ++l) {
                if (g.wt)
                    hipLaunchKernelGGL((k_kjob<LAT, T, true>), dim3(g.nb1, g.klev[l].y), blk, 0, st, g.mems, g.work1,
                                       g.kjobs + g.klev[l].x);
                else
                    hipLaunchKernelGGL((k_kjob<LAT, T, false>), dim3(g.nb1, g.klev[l].y), blk, 0, st, g.mems, g.work1,
                                       g.kjobs + g.klev[l].x);
            }
        }
        if (!g.kf && g.npass >= 1) {
#define LBM_BINOM1(TXV, ZCV)                                                                                    \
    do {                                                                                                        \
        if (g.wt) hipLaunchKernelGGL((k_binom1<LAT, T, TXV, ZCV, true>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems, g.workb); \
        else hipLaunchKernelGGL((k_binom1<LAT, T, TXV, ZCV, false>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems, g.workb); \
    } while (0)
            if (Lat<LAT>::D == 3 && g.btx == kBinTXW) {
                if (g.any_z) LBM_BINOM1((Lat<LAT>::D == 3 ? kBinTXW : kBinTX), true);
                else LBM_BINOM1((Lat<LAT>::D == 3 ? kBinTXW : kBinTX), false);
            } else {
                if (g.any_z) LBM_BINOM1(kBinTX, true); else LBM_BINOM1(kBinTX, false);
            }
#undef LBM_BINOM1
        }
        for (int j = 2; j <= (g.kf ? 0 : g.npass); ++j) {
#define LBM_BINOM(TXV, CHV)                                                                                    \
    do {                                                                                                       \
        if (g.wt) hipLaunchKernelGGL((k_binom<LAT, T, TXV, CHV, true>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems, g.workb, j); \
        else hipLaunchKernelGGL((k_binom<LAT, T, TXV, CHV, false>), dim3(g.nbb), dim3(TXV * kBinTY), 0, st, g.mems, g.workb, j); \
    } while (0)
            const int ch = g.bmask[j - 1];
            if (g.btx == kBinTXW) {
                if (ch == 1) LBM_BINOM(kBinTXW, 1); else if (ch == 2) LBM_BINOM(kBinTXW, 2); else LBM_BINOM(kBinTXW, 3);
            } else {
                if (ch == 1) LBM_BINOM(kBinTX, 1); else if (ch == 2) LBM_BINOM(kBinTX, 2); else LBM_BINOM(kBinTX, 3);
            }
#undef LBM_BINOM
        }
        mark(3);
#define LBM_REDUCE(KFV)                                                                                      \
    do {                                                                                                     \
        if (g.maxsa <= 2)                                                                                    \
            hipLaunchKernelGGL((k_reduce<LAT, T, 2, KFV>), dim3(g.nbr), blk, 0, st, g.mems, g.workr);        \
        else if (g.maxsa <= 6)                                                                               \
            hipLaunchKernelGGL((k_reduce<LAT, T, 6, KFV>), dim3(g.nbr), blk, 0, st, g.mems, g.workr);        \
        else                                                                                                 \
            hipLaunchKernelGGL((k_reduce<LAT, T, kMaxSA, KFV>), dim3(g.nbr), blk, 0, st, g.mems, g.workr);   \
    } while (0)
        if (g.kf) LBM_REDUCE(true); else LBM_REDUCE(false);
#undef LBM_REDUCE
        mark(4);
        hipLaunchKernelGGL(k_sum, dim3(g.nbs), blk, 0, st, g.mems, g.works);
        // the binomial apply forms the solve itself (one launch less per step)
        const bool fused = fused_solve(g);
        if (!fused) hipLaunchKernelGGL(k_solve, dim3(g.nmem), blk, 0, st, g.mems, g.workm);
        mark(5);
        if (!g.probe) {
#define LBM_APPLY(KFV, DEFV)                                                                                 \
    do {                                                                                                     \
        if (g.wt) hipLaunchKernelGGL((k_apply<LAT, T, KFV, true, DEFV>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
        else hipLaunchKernelGGL((k_apply<LAT, T, KFV, false, DEFV>), dim3(g.nb1), blk, 0, st, g.mems, g.work1, flip); \
    } while (0)
#define LBM_APPLY_FS(DEFV)                                                                                   \
    do {                                                                                                     \
        if (g.wt) hipLaunchKernelGGL((k_apply_fs<LAT, T, true, DEFV>), dim3(g.nbp), blk, 0, st, g.mems, g.workp, flip); \
        else hipLaunchKernelGGL((k_apply_fs<LAT, T, false, DEFV>), dim3(g.nbp), blk, 0, st, g.mems, g.workp, flip); \
    } while (0)
            const bool def = g.defer && g.substrate != LBM_WALE;
            if (g.kf) { if (def) LBM_APPLY(true, true); else LBM_APPLY(true, false); }
            else if (fused) { if (def) LBM_APPLY_FS(true); else LBM_APPLY_FS(false); }
            else { if (def) LBM_APPLY(false, true); else LBM_APPLY(false, false); }
#undef LBM_APPLY
#undef LBM_APPLY_FS
        }
        mark(6);
    } else if (g.mode == 1) {
        hipLaunchKernelGGL((k_diag<LAT, T>), dim3(g.nb1), blk, 0, st, g.mems, g.work1);
        hipLaunchKernelGGL(k_fin_diag, dim3(g.nmem), blk, 0, st, g.mems, g.workm);
        mark(2); mark(3); mark(4); mark(5); mark(6);
    } else {
        mark(2); mark(3); mark(4); mark(5); mark(6);
    }
}

void launch_step(const LaunchGroup& g, hipStream_t st, int flip, hipEvent_t* ev)
{
    const int key = g.lattice * 3 + g.precision;
    switch (key) {
    case LBM_D2Q9 * 3 + LBM_FP32_SHIFTED: launch_step_group<LBM_D2Q9, float, LBM_FP32_SHIFTED>(g, st, flip, ev); break;
    case LBM_D2Q9 * 3 + LBM_FP64: launch_step_group<LBM_D2Q9, double, LBM_FP64>(g, st, flip, ev); break;
    case LBM_D2Q9 * 3 + LBM_FP32_PLAIN: launch_step_group<LBM_D2Q9, float, LBM_FP32_PLAIN>(g, st, flip, ev); break;
    case LBM_D3Q19 * 3 + LBM_FP32_SHIFTED: launch_step_group<LBM_D3Q19, float, LBM_FP32_SHIFTED>(g, st, flip, ev); break;
    case LBM_D3Q19 * 3 + LBM_FP64: launch_step_group<LBM_D3Q19, double, LBM_FP64>(g, st, flip, ev); break;
    case LBM_D3Q19 * 3 + LBM_FP32_PLAIN: launch_step_group<LBM_D3Q19, float, LBM_FP32_PLAIN>(g, st, flip, ev); break;
    }
}

template <int LAT, typename T, int PREC>
static void launch_state_t(int op, const DevMember* dm, int N, bool has_to, int flip, hipStream_t st,
                           const double* a, double* b)
{
    const dim3 blk(kBlock), grd((N + kBlock - 1) / kBlock);
    switch (op) {
    case OP_INIT: hipLaunchKernelGGL((k_init<LAT, T, PREC>), grd, blk, 0, st, dm, flip, a, (const double*)b); break;
    case OP_GET_POP: hipLaunchKernelGGL((k_get_pop<LAT, T, PREC>), grd, blk, 0, st, dm, flip, b); break;
    case OP_SET_POP: hipLaunchKernelGGL((k_set_pop<LAT, T, PREC>), grd, blk, 0, st, dm, flip, a); break;
    case OP_STREAM:
        if (has_to) hipLaunchKernelGGL((k_stream_only<LAT, T, true>), grd, blk, 0, st, dm, flip);
        else hipLaunchKernelGGL((k_stream_only<LAT, T, false>), grd, blk, 0, st, dm, flip);
        break;
    }
}

void launch_state(int op, int lattice, int precision, const DevMember* dm, int N, bool has_to, int flip,
                  hipStream_t st, const double* a, double* b)
{
    const int key = lattice * 3 + precision;
    switch (key) {
    case LBM_D2Q9 * 3 + LBM_FP32_SHIFTED: launch_state_t<LBM_D2Q9, float, LBM_FP32_SHIFTED>(op, dm, N, has_to, flip, st, a, b); break;
    case LBM_D2Q9 * 3 + LBM_FP64: launch_state_t<LBM_D2Q9, double, LBM_FP64>(op, dm, N, has_to, flip, st, a, b); break;
    case LBM_D2Q9 * 3 + LBM_FP32_PLAIN: launch_state_t<LBM_D2Q9, float, LBM_FP32_PLAIN>(op, dm, N, has_to, flip, st, a, b); break;
    case LBM_D3Q19 * 3 + LBM_FP32_SHIFTED: launch_state_t<LBM_D3Q19, float, LBM_FP32_SHIFTED>(op, dm, N, has_to, flip, st, a, b); break;
    case LBM_D3Q19 * 3 + LBM_FP64: launch_state_t<LBM_D3Q19, double, LBM_FP64>(op, dm, N, has_to, flip, st, a, b); break;
    case LBM_D3Q19 * 3 + LBM_FP32_PLAIN: launch_state_t<LBM_D3Q19, float, LBM_FP32_PLAIN>(op, dm, N, has_to, flip, st, a, b); break;
    }
}

void launch_fields(int lattice, int precision, const DevMember* dm, const int2* work1, int nb1, bool has_to,
                   int flip, hipStream_t st, double* rho_out, double* u_out)
{
    const int key = lattice * 3 + precision;
    const dim3 blk(kBlock), grd(nb1);
#define LBM_MOM(LAT, T, PREC)                                                                                  \
    do {                                                                                                       \
        if (has_to) hipLaunchKernelGGL((k_moments<LAT, T, PREC, true>), grd, blk, 0, st, dm, work1, flip, rho_out, \
                                       u_out);                                                                   \
        else hipLaunchKernelGGL((k_moments<LAT, T, PREC, false>), grd, blk, 0, st, dm, work1, flip, rho_out, u_out); \
    } while (0)
    switch (key) {
    case LBM_D2Q9 * 3 + LBM_FP32_SHIFTED: LBM_MOM(LBM_D2Q9, float, LBM_FP32_SHIFTED); break;
    case LBM_D2Q9 * 3 + LBM_FP64: LBM_MOM(LBM_D2Q9, double, LBM_FP64); break;
    case LBM_D2Q9 * 3 + LBM_FP32_PLAIN: LBM_MOM(LBM_D2Q9, float, LBM_FP32_PLAIN); break;
    case LBM_D3Q19 * 3 + LBM_FP32_SHIFTED: LBM_MOM(LBM_D3Q19, float, LBM_FP32_SHIFTED); break;
    case LBM_D3Q19 * 3 + LBM_FP64: LBM_MOM(LBM_D3Q19, double, LBM_FP64); break;
    case LBM_D3Q19 * 3 + LBM_FP32_PLAIN: LBM_MOM(LBM_D3Q19, float, LBM_FP32_PLAIN); break;
    }
#undef LBM_MOM
}

void launch_flush(int lattice, int precision, const DevMember* dm, const int2* work1, int nb1, int flip,
                  hipStream_t st)
{
    const dim3 blk(kBlock), grd(nb1);
    if (lattice == LBM_D2Q9) {
        if (precision == LBM_FP64) hipLaunchKernelGGL((k_flush<LBM_D2Q9, double>), grd, blk, 0, st, dm, work1, flip);
        else hipLaunchKernelGGL((k_flush<LBM_D2Q9, float>), grd, blk, 0, st, dm, work1, flip);
    } else {
        if (precision == LBM_FP64) hipLaunchKernelGGL((k_flush<LBM_D3Q19, double>), grd, blk, 0, st, dm, work1, flip);
        else hipLaunchKernelGGL((k_flush<LBM_D3Q19, float>), grd, blk, 0, st, dm, work1, flip);
    }
}

void launch_philox_test(const uint32_t* in, uint32_t* out, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_philox_test, dim3((n + 63) / 64), dim3(64), 0, st, in, out, n);
}

void launch_normals_test(unsigned long long seed, long long step0, int nsteps, int n, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_normals_test, dim3((nsteps + 63) / 64), dim3(64), 0, st, seed, step0, nsteps, n, out);
}

int lattice_table(int lattice, int* c, double* w)
{
    if (lattice == LBM_D2Q9) {
        using L = Lat<LBM_D2Q9>;
        for (int i = 0; i < L::Q; ++i) { c[3 * i] = L::cx[i]; c[3 * i + 1] = L::cy[i]; c[3 * i + 2] = L::cz[i]; w[i] = L::w[i]; }
        return L::Q;
    }
    using L = Lat<LBM_D3Q19>;
    for (int i = 0; i < L::Q; ++i) { c[3 * i] = L::cx[i]; c[3 * i + 1] = L::cy[i]; c[3 * i + 2] = L::cz[i]; w[i] = L::w[i]; }
    return L::Q;
}

}  // namespace lbm

// lbm_dev.h -- internal device-side structures of liblbm_hip (not installed).
//
// Every LES run ("member") is described to the kernels by a DevMember record
// in device memory.  Kernels are launched over work tables whose entries map
// a workgroup to (member, local block), so one launch advances one member or
// any number of members of the same kind.
#pragma once
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

constexpr int kMaxQ = LBM_MAX_QOI;
constexpr int kMaxSA = 8;       // E/Z QoIs per closure
constexpr int kMaxPow = 4;      // highest power of B in R R (filters up to degree 2)
constexpr int kBlock = 256;     // threads per workgroup of the cell kernels
// Population layout: consecutive blocks of kPopBlk cells, each block holding
// its Q populations one after another, [ceil(N / kPopBlk)][Q][kPopBlk].
constexpr int kPopLog = 10;
constexpr int kPopBlk = 1 << kPopLog;
constexpr int kBinTX = 32;      // binomial-filter tile: x extent
constexpr int kBinTY = kBlock / kBinTX;  // y extent
constexpr int kBinTXW = 64;     // the wide tile (64 x 8, 512 threads) of the tiled kernels
constexpr int kBinZCMax = 16;   // most z planes per workgroup chosen automatically (3-D)
// The binomial apply forms the member's solve in every workgroup (one per
// pair of 256-cell blocks of a member) where its launch has at most this
// many workgroups: at two waves per SIMD they are all resident at once on
// the 256 CUs, so the solve's latency is paid once per launch, under the
// apply's own loads; larger launches keep k_solve.
constexpr int kFusedApplyPairs = 512;
constexpr int kHistRows = 512;   // LRS history rows (x entries) per k_sum workgroup
constexpr int kMaxHistChunks = 64;                 // so 2 h nq <= 32768
constexpr int kMaxRad = 12;     // kernel filters: largest radius of a 1-D factor

// Constant closure parameters (written by the host at set_closure).
struct DevParam {
    int nq, mode, nsa, nmp;
    int nbands, have_scale, nref, jv;  // jv: highest power of B applied to v
    int jw, has_z, has_e, h;           // jw: highest power applied to curl v; h: LRS history length
    int nhc, kf;                       // workgroups of the history product (k_sum); kernel filters
    long long spinup;
    unsigned long long seed;
    int sa_slot[kMaxSA];               // user index of each E/Z QoI
    int sa_kind[kMaxSA];               // 0 E, 1 Z
    int mp_slot[kMaxQ];                // user index of each MP QoI
    int mp_band[kMaxQ];
    double r[kMaxSA][3];               // R   = sum_j r[j]  B^j
    double rr[kMaxSA][kMaxPow + 1];    // R R = sum_j rr[j] B^j
    float rf[kMaxSA][3];               // the same rounded to FP32 (for the FP32 kernels)
    float rrf[kMaxSA][kMaxPow + 1];
    double C[(kMaxQ + 1) * kMaxQ];
    double mu[kMaxQ];
    double L[kMaxQ * kMaxQ];           // Cholesky factor of Sigma
    double scale[kMaxQ];
    double gmp[kMaxQ * kMaxQ];         // <w_i e_x, w_j e_x> = nx nz sum_y w_i w_j
    const double* qref;                // nref x nq
    const double* chist;               // h > 0: the history rows of C, [2 h nq][nq]: rows of
                                       // z^{n-1..n-h}, then of z*^{n-1..n-h}
};

// Per-step control state written by the kernels.
struct DevCtl {
    long long step;
    int flags;                         // sticky bit0: unstable
    int s_set;
    double s[kMaxQ];                   // LRS scale
    double cv[kMaxPow + 1];            // dv = sum_j cv[j] B^j v + curl^T(sum_j cw[j] B^j w) + e_x cmp(y)
    double cw[kMaxPow + 1];
    float cvf[kMaxPow + 1];            // cv, cw rounded to FP32
    float cwf[kMaxPow + 1];
    double pad[1];
    double lrs_e[kMaxQ];               // mu + L xi of the current step's LRS draw
    double bsa[kMaxSA];                // beta of each E/Z QoI (kernel-filter dv build)
    float bsaf[kMaxSA];
    long long step_snap;               // step as k_sum found it (read by a fused apply)
    int s_pend;                        // a first LRS scale in s_next, committed by the next k_sum
    int pad_s;
    double s_next[kMaxQ];
};

struct DevMember {
    int nx, ny, nz, N;
    int walls, substrate, force_kind, force_k;
    int parity;                        // index of the buffer holding the state at flip 0
    int has_to, diag, rec_cap;
    double tau, cmodel, force_amp, drag;
    void* g[2];                        // populations [Q][N]
    void* rho;                         // rho - 1 of the predictor [N]      (TO)
    void* vs;                          // predictor velocity v* [D][N]      (TO)
    void* vn;                          // post-streaming velocity [D][N]    (diag, WALE)
    void* P;                           // B^j v*, j = 1..jv   [jv][D][N]
    void* W;                           // B^j curl v*, j=0..jw [jw+1][NC][N]
    void* C;                           // curl^T B^j curl v*, j=0..jw-1 [jw+1][D][N] (C_jw: from W_jw)
    double* part_stats;                // [nb1][4]: sum(rho-1), sum(rho v)
    double* part_to;                   // [npart][ny * nbx2]
    double* part_diag;                 // [nb1][2]
    int nb1, nbx2, npart, cpt2;        // block counts; cells per thread of the reduce
    int zc, btx;                       // z planes per binomial-filter workgroup; its tile width
    DevParam* prm;
    DevCtl* ctl;
    lbm_qoi_rec* recs;
    double* bandw;                     // [nbands][ny]
    double* cmp;                       // [ny]
    double* fprof;                     // body force F_x(y) [ny]
    double* sums;                      // [4 + npart]: reduced statistics and TO partials
    double* hpart;                     // [nhc][kMaxQ]: LRS history product per k_sum workgroup
    void* kV;                          // kernel filters: V_s = R(R v*) or curl^T R(R w), [nsa][D][N]
    void* rec;                         // pending SGS change of the last step: (rho dv, 2 v* + dv) [2D][N]
    int nst;                           // stream-collide statistics partials (workgroups of the launch)
    int defer;                         // TO steps defer the SGS change into the next pull (k_step_t)
};

#ifdef __HIP_DEVICE_COMPILE__
#define LBM_K __attribute__((address_space(4)))
#else
#define LBM_K
#endif
// Kernels read member records and closure parameters, which no kernel writes
// while it runs, through the constant address space: with a workgroup-uniform
// address the loads go to the scalar unit and the parameters stay in scalar
// registers, so they never wait behind the vector loads of the fields.
using KMember = const LBM_K DevMember;
using KParam = const LBM_K DevParam;
using KCtl = const LBM_K DevCtl;
template <typename X>
__host__ __device__ __forceinline__ const LBM_K X* kc(const X* p) { return (const LBM_K X*)p; }

}  // namespace lbm

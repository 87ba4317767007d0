// lbm_launch.h -- launch interface between the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "lbm_dev.h"

namespace lbm {

// One output field of a kernel-filter closure's sensitivity program (lives
// in device memory; a launch runs every job of one level, one job per
// blockIdx.y): op 0, dst = sum_t coef_t (1-D convolution of src_t along axis
// with taps_t), periodic wrap or zero padding on the wall axis; op 1,
// dst = curl^T src[0].  Pointers are device addresses in the member's arena.
struct KJob {
    int op, axis, ncomp, nterm;
    int radius[3];
    int pad;
    double coef[3];
    const void* taps[3];   // 2 radius + 1 values each, element type of the run
    const void* src[3];
    void* dst;
};

// Fourier band QoIs of a member (host side): spectra of v* and w, the
// masked band spectra of all E QoIs and of all Z QoIs, and per QoI the band
// and the destination of R v* (E: V_s) or of R w (Z: the input of its
// adjoint curl).  Plans are hipfftHandle values.
constexpr int kMaxBands = kMaxSA;   // every E/Z QoI may be a band
struct FourierQ { int e, l, m; void* dst; };
struct FourierProg {
    void* plan[4];        // forward: batch D (v*), batch NC (w); inverse: all E bands, all Z bands
    void* spec_v;         // [D][N] complex
    void* spec_w;         // [NC][N] complex (Z QoIs only)
    void* band_e;         // [nE][D][N] complex
    void* band_z;         // [nZ][NC][N] complex
    const void* vs;       // v* [D][N]
    const void* w;        // w [NC][N]
    int nx, ny, nz;
    std::vector<FourierQ> qe, qz;   // E and Z bands
    mutable int failed = 0;         // set when a hipFFT call of a launch fails
};

// One launch per kernel phase covers every member of a group: members share
// lattice, precision, substrate and mode, and are mapped to workgroups by
// the work tables.
struct LaunchGroup {
    int lattice, precision, substrate, mode;  // mode 0 plain, 1 plain + records, 2 TO
    int any_z, maxpow, maxsa, npass;  // npass: binomial passes per step
    int btx;            // binomial tile width of every member (kBinTX or kBinTXW)
    int bmask[8];       // per binomial pass j = 1..npass: chains advanced by some member (1 v, 2 w)
    const DevMember* mems;
    const int2* work1;  // cell kernels: (member, block of kBlock cells)
    int nb1;
    const int2* workp;  // the apply with the solve: (member, pair p of blocks 2p and 2p + 1)
    int nbp;
    const int2* workr;  // reduce: (member, y * nbx2 + bx)
    int nbr;
    const int2* workb;  // binomial filter: (member, xyz tile)
    int nbb;
    const int2* works;  // cross-block sums: (member, value slot)
    int nbs;
    const int* workm;   // one workgroup per member
    int nmem;
    int probe;          // TO mode only: the QoI chain of the field already in v* (no
                        // stream-collide, no apply); see lbm_project_qoi
    int kf;             // kernel-filter closure (one member per group): its job levels
    const KJob* kjobs;  // replace the binomial passes; kjobs in device memory,
    const int2* klev;   // klev[l] = (first job, job count) of level l (host memory)
    int nklev;
    const FourierProg* fprog;   // Fourier band QoIs (host memory; null if none)
    int wt;             // store the fields the next kernel reads through the L2 (small launches)
    int defer;          // TO mode: the SGS change is recorded and applied by the next step's pull
    int a32;            // every member's population buffer spans less than 4 GiB (32-bit offsets)
    int nt;             // plain runs: the launch's populations exceed the Infinity Cache (non-temporal stores)
    int sep_solve;      // TO mode: the solve in its own launch (k_solve) even where k_apply could form it
                        // (k_step_t over the binomial tiles); not with the WALE substrate
};

// TO mode: the binomial apply forms the solve itself (no k_solve launch):
// not for kernel-filter closures, probe steps (no apply) or a forced own
// launch, and only where the apply's workgroups are all resident at once.
inline bool fused_solve(const LaunchGroup& g)
{
    return !g.kf && !g.probe && !g.sep_solve && g.nbp <= kFusedApplyPairs;
}

enum { OP_INIT = 0, OP_GET_POP = 1, OP_SET_POP = 2, OP_STREAM = 3 };

// ev (nullable): 7 events recorded at the phase boundaries of the step
// (start, after stream-collide, after the curl of kernel-filter closures,
// after the binomial powers, after the reduce, after the cross-block sums and
// solve, after the apply).
constexpr int kNumPhases = 6;
void launch_step(const LaunchGroup& g, hipStream_t st, int flip, hipEvent_t* ev = nullptr);
void launch_state(int op, int lattice, int precision, const DevMember* dm, int N, bool has_to, int flip,
                  hipStream_t st, const double* a, double* b);
// Moments of the current state into vn, and (nullable) rho [N] and v [D][N]
// in double into rho_out and u_out.
void launch_fields(int lattice, int precision, const DevMember* dm, const int2* work1, int nb1, bool has_to,
                   int flip, hipStream_t st, double* rho_out, double* u_out = nullptr);
// The pending SGS change of deferring members added to their current
// populations g[parity ^ flip] and their records cleared (k_flush).
void launch_flush(int lattice, int precision, const DevMember* dm, const int2* work1, int nb1, int flip,
                  hipStream_t st);
void launch_philox_test(const uint32_t* in, uint32_t* out, int n, hipStream_t st);
void launch_normals_test(unsigned long long seed, long long step0, int nsteps, int n, double* out, hipStream_t st);
int lattice_table(int lattice, int* c, double* w);
// Projection of a fine member's state (coarse grid ncx x ncy x ncz; kind
// LBM_PROJ_STRIDE: the wall-anchored stride-m subsampling; LBM_PROJ_BICUBIC:
// the bicubic mean of a doubly periodic 2-D grid): full populations into
// fpop [Q][Nc] (nullable) and the post-collision velocity into vout [D][Nc]
// (nullable; double if vout_fp64).  tmp (nullable): device scratch of
// 2 * (ncy m) * ncx doubles, with which the bicubic velocity projection runs
// as two separable passes.
void launch_project(int lattice, int precision, const DevMember* fine, int flip, int m, int ncx, int ncy, int ncz,
                    double* fpop, void* vout, int vout_fp64, int kind, hipStream_t st, double* tmp = nullptr);

}  // namespace lbm

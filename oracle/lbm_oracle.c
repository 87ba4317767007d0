/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of the Tau-orthogonal (TO) lattice
 * Boltzmann LES step of Hoekstra, Xue, Coveney and Edeling, "Reduced
 * Subgrid-Scale Terms for Turbulence Simulations with the Lattice Boltzmann
 * Method".  It exists so that the tests, the smoke check and the CPU-baseline
 * leg of the benchmark can check the HIP library against something that is
 * obviously correct.  Nothing in the product path may link, load or call it,
 * and it shares no code, header, table or helper with the HIP library.
 *
 * Every routine follows the paper's definitions in the order the paper gives
 * them, with no blocking, fusion or reordering:
 *   - lattice, moments, equilibrium, BGK:           Sec. 2 (moments, BGK eq.
 *                                                    and its footnote)
 *   - exact-difference forcing and streaming:        Sec. 2, eq. collide-and-stream
 *   - LES step with macroscopic SGS forcing:         Sec. 3, eqs. LES-1..LES-3
 *   - halfway bounce-back walls:                     Sec. 7.1 (channel setup)
 *   - eddy-viscosity substrates (Smagorinsky/WALE):  Sec. 5, eq. eff-relaxation,
 *                                                    eq. smag, closed form, WALE
 *   - QoIs (energy, enstrophy, filtered, mp):        Sec. 4.1, eq. qoi-def,
 *                                                    eq. mean-profile-qoi,
 *                                                    eq. 3d-mp-band-weights
 *   - sensitivities:                                 App. A
 *   - patterns O_i = sum_j c_ij V_j, c_ii = 1:        Sec. 4.2, eq. O-from-V,
 *                                                    eq. orthogonality
 *   - tracking dQ and gamma:                         Sec. 4.3, eq. dQ-from-ref,
 *                                                    eq. tau-from-dQ-for-tracking
 *   - LRS online draw:                               Sec. 4.4, eq. LRS
 * Readings where the paper is silent are listed in the design notes; the ones
 * that shape code here are repeated at the point of use.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 * Global sums are plain sequential loops in cell order, so results do not
 * depend on the OpenMP thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OQMAX 16
#define OPI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Configuration structs (mirrored by ctypes in oracle/__init__.py).   */
/* ------------------------------------------------------------------ */
typedef struct {
    int lattice;          /* 0: D2Q9, 1: D3Q19 */
    int nx, ny, nz;       /* nz = 1 for D2Q9 */
    int walls_y;          /* 1: halfway bounce-back walls at y=-1/2 and y=ny-1/2 */
    double tau;
    int substrate;        /* 0 BGK, 1 Smagorinsky, 2 WALE */
    double cmodel;        /* C_smag or C_w */
    int force_kind;       /* 0 none, 1 F_x = A sin(2 pi k y / ny), 2 F_x = A */
    double force_amp;
    int force_k;
    double drag;          /* optional linear drag: F -= drag * rho * v */
} orc_cfg;

typedef struct {
    int nq;
    int kind[OQMAX];      /* 0 energy E_R, 1 enstrophy Z_R, 2 mean-profile */
    int filt[OQMAX];      /* 0 I, 1 B, 2 B^2, 3 B-B^2, 4 I-B, 5 G_s, 6 L_s, 7 R_[l,m] */
    int band[OQMAX];      /* band index for mean-profile QoIs */
    int nbands;
    double dmin, dmax;    /* band-centre range in wall distance */
    int mode;             /* 0 off (dQ = 0), 1 tracking, 2 LRS online */
    long spinup;          /* dQ = 0 for steps < spinup */
    double C[(OQMAX + 1) * OQMAX];   /* LRS regression matrix, (nq+1) x nq row-major */
    double mu[OQMAX];
    double Sigma[OQMAX * OQMAX];
    double scale[OQMAX];
    int have_scale;
    uint64_t seed;
    int h;                /* LRS history length (eq. LRS); 0 uses C above */
    const double *Chist;  /* h > 0: the full ((2h+1) nq + 1) x nq matrix C (copied) */
    int fs[OQMAX];        /* scale s of the kernel filters 5 (G_s) and 6 (L_s); l of filter 7 */
    int fm[OQMAX];        /* m of the Fourier band filter 7, R_[l,m] */
} orc_closure;

typedef struct {
    long step;
    int flags;            /* bit0: unstable, bit1: Gram singular (correction skipped) */
    int nq;
    double mass;          /* sum of rho of the post-streaming state */
    double mom[3];        /* sum of rho*v of the post-streaming state */
    double diag_e, diag_z;/* E and Z of the post-streaming velocity */
    double q[OQMAX], dq[OQMAX], gamma[OQMAX];
} orc_rec;

typedef struct {
    orc_cfg c;
    int d, Q;
    long N;
    int cv[19][3];
    double w[19];
    int opp[19];
    double *fp;           /* post-collision populations, Q*N (full, not shifted) */
    double *f;            /* post-streaming populations, Q*N */
    double *rho, *v, *vs, *dv, *taueff;   /* N, d*N, d*N, d*N, N */
    int have_closure;
    orc_closure cl;
    double L[OQMAX * OQMAX];  /* Cholesky factor of Sigma */
    double *qref; long nref;
    double *Chist;        /* copy of the history-h regression matrix */
    double s[OQMAX]; int s_set;
    double *V, *O;        /* nq*d*N sensitivity and pattern fields */
    double *bandw;        /* nbands*ny */
    long step;
    orc_rec *recs; long nrec, caprec;
    int fp32_store;       /* diagnostic: round the stored state to FP32 (see orc_set_fp32_store) */
    int rev_sums;         /* diagnostic: global sums in reverse cell order (see orc_set_reverse_sums) */
    int reduced;          /* diagnostic: the correction in its reduced form (see orc_set_reduced_form) */
} Orc;

/* ------------------------------------------------------------------ */
/* Lattices (Sec. 2: D2Q9 and D3Q19, c_s^2 = 1/3).                     */
/* ------------------------------------------------------------------ */
static const int D2C[9][2] = {{0,0},{1,0},{0,1},{-1,0},{0,-1},{1,1},{-1,1},{-1,-1},{1,-1}};
static const double D2W[9] = {4.0/9, 1.0/9, 1.0/9, 1.0/9, 1.0/9, 1.0/36, 1.0/36, 1.0/36, 1.0/36};
static const int D3C[19][3] = {
    {0,0,0},
    {1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},
    {1,1,0},{-1,-1,0},{1,-1,0},{-1,1,0},
    {1,0,1},{-1,0,-1},{1,0,-1},{-1,0,1},
    {0,1,1},{0,-1,-1},{0,1,-1},{0,-1,1}};

static int lattice_tables(int lattice, int cv[19][3], double w[19])
{
    if (lattice == 0) {
        for (int i = 0; i < 9; i++) {
            cv[i][0] = D2C[i][0]; cv[i][1] = D2C[i][1]; cv[i][2] = 0; w[i] = D2W[i];
        }
        return 9;
    }
    for (int i = 0; i < 19; i++) {
        cv[i][0] = D3C[i][0]; cv[i][1] = D3C[i][1]; cv[i][2] = D3C[i][2];
        int n2 = cv[i][0]*cv[i][0] + cv[i][1]*cv[i][1] + cv[i][2]*cv[i][2];
        w[i] = (n2 == 0) ? 1.0/3 : (n2 == 1 ? 1.0/18 : 1.0/36);
    }
    return 19;
}

int orc_lattice(int lattice, int *c /* 3*Q */, double *w /* Q */)
{
    int cv[19][3]; double ww[19];
    int Q = lattice_tables(lattice, cv, ww);
    for (int i = 0; i < Q; i++) {
        c[3*i] = cv[i][0]; c[3*i+1] = cv[i][1]; c[3*i+2] = cv[i][2]; w[i] = ww[i];
    }
    return Q;
}

/* Second-order equilibrium, footnote of the BGK equation (Sec. 2):
 * feq_i = w_i rho (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)), cs2 = 1/3. */
static double feq_one(const Orc *o, int i, double rho, const double *u)
{
    double cu = 0, uu = 0;
    for (int a = 0; a < o->d; a++) { cu += o->cv[i][a] * u[a]; uu += u[a] * u[a]; }
    return o->w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

void orc_feq(int lattice, double rho, const double *u, double *out)
{
    Orc o; memset(&o, 0, sizeof o);
    o.Q = lattice_tables(lattice, o.cv, o.w);
    o.d = lattice == 0 ? 2 : 3;
    for (int i = 0; i < o.Q; i++) out[i] = feq_one(&o, i, rho, u);
}

/* ------------------------------------------------------------------ */
/* Grid helpers.                                                       */
/* ------------------------------------------------------------------ */
static long cell(const Orc *o, int x, int y, int z) { return x + (long)o->c.nx * (y + (long)o->c.ny * z); }
static int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* Neighbour value of a scalar field with the boundary rule of the filters and
 * derivatives: periodic wrap on periodic axes, zero outside the domain on the
 * wall-bounded y axis (Sec. 4.1, "zero padding" on wall-bounded axes). */
static double at(const Orc *o, const double *u, int x, int y, int z)
{
    x = wrap(x, o->c.nx);
    z = wrap(z, o->c.nz);
    if (o->c.walls_y) { if (y < 0 || y >= o->c.ny) return 0.0; }
    else y = wrap(y, o->c.ny);
    return u[cell(o, x, y, z)];
}

/* Second-order central difference along axis a (0 x, 1 y, 2 z). */
static double dcen(const Orc *o, const double *u, int a, int x, int y, int z)
{
    int dx = a == 0, dy = a == 1, dz = a == 2;
    return 0.5 * (at(o, u, x + dx, y + dy, z + dz) - at(o, u, x - dx, y - dy, z - dz));
}

/* ------------------------------------------------------------------ */
/* Create / destroy / state access.                                    */
/* ------------------------------------------------------------------ */
void *orc_create(const orc_cfg *c)
{
    Orc *o = (Orc *)calloc(1, sizeof(Orc));
    o->c = *c;
    if (o->c.lattice == 0) o->c.nz = 1;
    o->Q = lattice_tables(c->lattice, o->cv, o->w);
    o->d = c->lattice == 0 ? 2 : 3;
    for (int i = 0; i < o->Q; i++)
        for (int j = 0; j < o->Q; j++)
            if (o->cv[j][0] == -o->cv[i][0] && o->cv[j][1] == -o->cv[i][1] && o->cv[j][2] == -o->cv[i][2])
                o->opp[i] = j;
    o->N = (long)o->c.nx * o->c.ny * o->c.nz;
    o->fp = (double *)calloc((size_t)o->Q * o->N, sizeof(double));
    o->f = (double *)calloc((size_t)o->Q * o->N, sizeof(double));
    o->rho = (double *)calloc(o->N, sizeof(double));
    o->v = (double *)calloc((size_t)o->d * o->N, sizeof(double));
    o->vs = (double *)calloc((size_t)o->d * o->N, sizeof(double));
    o->dv = (double *)calloc((size_t)o->d * o->N, sizeof(double));
    o->taueff = (double *)calloc(o->N, sizeof(double));
    return o;
}

void orc_destroy(void *h)
{
    Orc *o = (Orc *)h;
    if (!o) return;
    free(o->fp); free(o->f); free(o->rho); free(o->v); free(o->vs); free(o->dv);
    free(o->taueff); free(o->qref); free(o->V); free(o->O); free(o->bandw); free(o->recs);
    free(o->Chist);
    free(o);
}

/* Initial post-collision state: f^p = feq(rho, u) (rho = 1 when NULL). */
void orc_init(void *h, const double *rho, const double *u)
{
    Orc *o = (Orc *)h;
    for (long x = 0; x < o->N; x++) {
        double uu[3] = {0, 0, 0};
        for (int a = 0; a < o->d; a++) uu[a] = u[a * o->N + x];
        double r = rho ? rho[x] : 1.0;
        for (int i = 0; i < o->Q; i++) o->fp[i * o->N + x] = feq_one(o, i, r, uu);
    }
    o->step = 0; o->nrec = 0; o->s_set = 0;
}

void orc_set_fp(void *h, const double *fp) { Orc *o = (Orc *)h; memcpy(o->fp, fp, sizeof(double) * o->Q * o->N); }
void orc_get_fp(void *h, double *fp) { Orc *o = (Orc *)h; memcpy(fp, o->fp, sizeof(double) * o->Q * o->N); }
long orc_step_count(void *h) { return ((Orc *)h)->step; }

/* ------------------------------------------------------------------ */
/* Streaming with periodic wrap and halfway bounce-back (eq. LES-3,     */
/* Sec. 7.1): f_i(x) = f^p_i(x - c_i); when x - c_i lies beyond a wall  */
/* the population that left x towards the wall returns reversed:        */
/* f_i(x) = f^p_opp(i)(x).                                              */
/* ------------------------------------------------------------------ */
static void stream(const Orc *o, const double *fp, double *f)
{
    const int nx = o->c.nx, ny = o->c.ny, nz = o->c.nz;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long xc = cell(o, x, y, z);
                for (int i = 0; i < o->Q; i++) {
                    int sx = x - o->cv[i][0], sy = y - o->cv[i][1], sz = z - o->cv[i][2];
                    if (o->c.walls_y && (sy < 0 || sy >= ny)) {
                        f[i * o->N + xc] = fp[o->opp[i] * o->N + xc];
                    } else {
                        long sc = cell(o, wrap(sx, nx), o->c.walls_y ? sy : wrap(sy, ny), wrap(sz, nz));
                        f[i * o->N + xc] = fp[i * o->N + sc];
                    }
                }
            }
}

void orc_stream_only(void *h)
{
    Orc *o = (Orc *)h;
    stream(o, o->fp, o->f);
    memcpy(o->fp, o->f, sizeof(double) * o->Q * o->N);
}

/* Moments (Sec. 2): rho = sum f_i, rho u = sum c_i f_i. */
static void moments(const Orc *o, const double *f, double *rho, double *v)
{
    #pragma omp parallel for schedule(static)
    for (long x = 0; x < o->N; x++) {
        double r = 0, m[3] = {0, 0, 0};
        for (int i = 0; i < o->Q; i++) {
            double fi = f[i * o->N + x];
            r += fi;
            for (int a = 0; a < o->d; a++) m[a] += o->cv[i][a] * fi;
        }
        rho[x] = r;
        for (int a = 0; a < o->d; a++) v[a * o->N + x] = m[a] / r;
    }
}

/* Post-streaming density and moment velocity of the current state. */
void orc_velocity(void *h, double *rho, double *u)
{
    Orc *o = (Orc *)h;
    stream(o, o->fp, o->f);
    double *r = rho ? rho : (double *)malloc(sizeof(double) * o->N);
    moments(o, o->f, r, u);
    if (!rho) free(r);
}

/* ------------------------------------------------------------------ */
/* Discrete curl with second-order central differences.               */
/* 2-D: scalar w = D_x v_y - D_y v_x.                                  */
/* 3-D: w = (D_y v_z - D_z v_y, D_z v_x - D_x v_z, D_x v_y - D_y v_x).   */
/* ------------------------------------------------------------------ */
int orc_ncurl(void *h) { return ((Orc *)h)->d == 2 ? 1 : 3; }

void orc_curl(void *h, const double *v, double *w)
{
    Orc *o = (Orc *)h;
    const long N = o->N;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < o->c.nz; z++)
        for (int y = 0; y < o->c.ny; y++)
            for (int x = 0; x < o->c.nx; x++) {
                long xc = cell(o, x, y, z);
                const double *vx = v, *vy = v + N, *vz = v + 2 * N;
                if (o->d == 2) {
                    w[xc] = dcen(o, vy, 0, x, y, z) - dcen(o, vx, 1, x, y, z);
                } else {
                    w[xc]         = dcen(o, vz, 1, x, y, z) - dcen(o, vy, 2, x, y, z);
                    w[N + xc]     = dcen(o, vx, 2, x, y, z) - dcen(o, vz, 0, x, y, z);
                    w[2 * N + xc] = dcen(o, vy, 0, x, y, z) - dcen(o, vx, 1, x, y, z);
                }
            }
}

/* Adjoint of the curl with respect to the sum-over-cells inner product.
 * Because the central difference with periodic wrap or zero padding is
 * skew-symmetric (D^T = -D), the adjoint in 2-D maps a scalar psi to
 * (D_y psi, -D_x psi) (eq. enstrophy-sensitivity-2d) and in 3-D it is the
 * curl itself (eq. enstrophy-sensitivity-3d). */
static void curl_adjoint(const Orc *o, const double *psi, double *out)
{
    const long N = o->N;
    if (o->d == 3) { orc_curl((void *)o, psi, out); return; }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < o->c.nz; z++)
        for (int y = 0; y < o->c.ny; y++)
            for (int x = 0; x < o->c.nx; x++) {
                long xc = cell(o, x, y, z);
                out[xc] = dcen(o, psi, 1, x, y, z);
                out[N + xc] = -dcen(o, psi, 0, x, y, z);
            }
}

/* ------------------------------------------------------------------ */
/* Compact binomial filter B = (x)_a [1,2,1]/4 applied as one direct    */
/* 3^d-point convolution per component, with zero padding on the wall   */
/* axis (Sec. 4.1).  The filters of the QoIs are polynomials in the     */
/* operator B: I, B, B^2 = B(B.), B - B^2 and I - B.                    */
/* ------------------------------------------------------------------ */
static void binomial(const Orc *o, const double *in, double *out, int ncomp)
{
    static const double b[3] = {0.25, 0.5, 0.25};
    const long N = o->N;
    const int rz = o->d == 3 ? 1 : 0;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < o->c.nz; z++)
        for (int y = 0; y < o->c.ny; y++)
            for (int x = 0; x < o->c.nx; x++) {
                long xc = cell(o, x, y, z);
                for (int k = 0; k < ncomp; k++) {
                    double s = 0;
                    for (int oz = -rz; oz <= rz; oz++)
                        for (int oy = -1; oy <= 1; oy++)
                            for (int ox = -1; ox <= 1; ox++) {
                                double wgt = b[ox + 1] * b[oy + 1] * (rz ? b[oz + 1] : 1.0);
                                s += wgt * at(o, in + k * N, x + ox, y + oy, z + oz);
                            }
                    out[k * N + xc] = s;
                }
            }
}

/* ------------------------------------------------------------------ */
/* Kernel filters of Sec. 4.1 as direct d-dimensional convolutions.     */
/*  G_s (eq. gaussian): exp(-|r|^2 / (2 s^2)) on the cube                */
/*      [-alpha s, alpha s]^d, alpha = 4 in 2-D and 2 in 3-D, divided by  */
/*      its sum over that cube.                                           */
/*  L_s (eq. laplace): L_1 places the biharmonic stencil               */
/*      l = [1, -4, 6, -4, 1] along each axis through the origin (the    */
/*      d axis terms add at the origin); L_s replaces every entry of L_1 */
/*      by an s^d block of equal value (s odd, so the block grid stays   */
/*      centred), and is scaled so that sum |L_s| = 2.                    */
/* Zero padding on the wall axis, periodic wrap elsewhere.              */
/* ------------------------------------------------------------------ */
static int kernel_build(const Orc *o, int filt, int s, double **K)
{
    const int d = o->d;
    int R;
    if (filt == 5) R = (d == 2 ? 4 : 2) * s;
    else R = (5 * s - 1) / 2;
    const int W = 2 * R + 1, nz = d == 3 ? W : 1;
    double *k = (double *)calloc((size_t)W * W * nz, sizeof(double));
    static const double l[5] = {1, -4, 6, -4, 1};
    double norm = 0;
    for (int iz = 0; iz < nz; iz++)
        for (int iy = 0; iy < W; iy++)
            for (int ix = 0; ix < W; ix++) {
                int r[3] = {ix - R, iy - R, d == 3 ? iz - R : 0};
                double v = 0;
                if (filt == 5) {
                    double rr = 0;
                    for (int a = 0; a < d; a++) rr += (double)r[a] * r[a];
                    v = exp(-rr / (2.0 * s * s));
                    norm += v;
                } else {
                    int blk[3];
                    for (int a = 0; a < d; a++) blk[a] = (int)floor((double)(r[a] + R) / s) - 2;
                    for (int a = 0; a < d; a++) {
                        int on_axis = 1;
                        for (int b = 0; b < d; b++) if (b != a && blk[b] != 0) on_axis = 0;
                        if (on_axis) v += l[blk[a] + 2];
                    }
                    norm += fabs(v);
                }
                k[((size_t)iz * W + iy) * W + ix] = v;
            }
    const double scale = filt == 5 ? 1.0 / norm : 2.0 / norm;
    for (long i = 0; i < (long)W * W * nz; i++) k[i] *= scale;
    *K = k;
    return R;
}

static void kernel_filter(const Orc *o, int filt, int s, const double *in, double *out, int ncomp)
{
    double *K;
    const int R = kernel_build(o, filt, s, &K), W = 2 * R + 1;
    const int rz = o->d == 3 ? R : 0;
    const long N = o->N;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < o->c.nz; z++)
        for (int y = 0; y < o->c.ny; y++)
            for (int x = 0; x < o->c.nx; x++) {
                long xc = cell(o, x, y, z);
                for (int k = 0; k < ncomp; k++) {
                    double acc = 0;
                    for (int oz = -rz; oz <= rz; oz++)
                        for (int oy = -R; oy <= R; oy++)
                            for (int ox = -R; ox <= R; ox++) {
                                double wgt = K[((size_t)(oz + rz) * W + (oy + R)) * W + (ox + R)];
                                if (wgt != 0.0) acc += wgt * at(o, in + k * N, x + ox, y + oy, z + oz);
                            }
                    out[k * N + xc] = acc;
                }
            }
    free(K);
}

/* ------------------------------------------------------------------ */
/* Sharp Fourier band filter R_[l,m] (eq. scale-aware-energy-fourier,   */
/* periodic grids): keep the DFT modes with l - 1/2 <= |k| < m + 1/2,   */
/* k the integer mode index vector (index j of an axis of length n is   */
/* k = j for j <= n/2, else j - n).  Plain separable DFT, no FFT.        */
/* ------------------------------------------------------------------ */
static void dft_axis(const Orc *o, double *re, double *im, int axis, int sign)
{
    const int n = axis == 0 ? o->c.nx : (axis == 1 ? o->c.ny : o->c.nz);
    if (n == 1) return;
    const long N = o->N;
    const long stride = axis == 0 ? 1 : (axis == 1 ? o->c.nx : (long)o->c.nx * o->c.ny);
    double *cs = (double *)malloc(sizeof(double) * n), *sn = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < n; j++) { cs[j] = cos(2.0 * OPI * j / n); sn[j] = sin(2.0 * OPI * j / n); }
    #pragma omp parallel for schedule(static)
    for (long base = 0; base < N; base++) {
        if ((base / stride) % n != 0) continue;      /* first cell of each line */
        double *tr = (double *)malloc(sizeof(double) * n), *ti = (double *)malloc(sizeof(double) * n);
        for (int kk = 0; kk < n; kk++) {
            double ar = 0, ai = 0;
            for (int j = 0; j < n; j++) {
                const int t = (int)(((long)kk * j) % n);
                const double c = cs[t], sv = sign * sn[t];
                const double xr = re[base + j * stride], xi = im[base + j * stride];
                ar += xr * c - xi * sv;
                ai += xr * sv + xi * c;
            }
            tr[kk] = ar; ti[kk] = ai;
        }
        for (int kk = 0; kk < n; kk++) { re[base + kk * stride] = tr[kk]; im[base + kk * stride] = ti[kk]; }
        free(tr); free(ti);
    }
    free(cs); free(sn);
}

static void fourier_band(const Orc *o, int l, int m, const double *in, double *out, int ncomp)
{
    const long N = o->N;
    double *re = (double *)malloc(sizeof(double) * N), *im = (double *)malloc(sizeof(double) * N);
    for (int k = 0; k < ncomp; k++) {
        for (long x = 0; x < N; x++) { re[x] = in[k * N + x]; im[x] = 0.0; }
        for (int a = 0; a < 3; a++) dft_axis(o, re, im, a, -1);
        for (long x = 0; x < N; x++) {
            const int jx = (int)(x % o->c.nx), jy = (int)((x / o->c.nx) % o->c.ny), jz = (int)(x / ((long)o->c.nx * o->c.ny));
            const int kx = jx <= o->c.nx / 2 ? jx : jx - o->c.nx;
            const int ky = jy <= o->c.ny / 2 ? jy : jy - o->c.ny;
            const int kz = jz <= o->c.nz / 2 ? jz : jz - o->c.nz;
            const double kn = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
            if (!(kn >= l - 0.5 && kn < m + 0.5)) { re[x] = 0.0; im[x] = 0.0; }
        }
        for (int a = 0; a < 3; a++) dft_axis(o, re, im, a, +1);
        for (long x = 0; x < N; x++) out[k * N + x] = re[x] / (double)N;
    }
    free(re); free(im);
}

static void apply_filter(const Orc *o, int filt, int s, const double *in, double *out, int ncomp);

/* R u for the filter code filt (scale s for the kernel filters; the band
 * [s, fm] for the Fourier filter). */
static void apply_filter_b(const Orc *o, int filt, int s, int fm, const double *in, double *out, int ncomp)
{
    if (filt == 7) { fourier_band(o, s, fm, in, out, ncomp); return; }
    apply_filter(o, filt, s, in, out, ncomp);
}

/* R u for the filter code filt (scale s for the kernel filters). */
static void apply_filter(const Orc *o, int filt, int s, const double *in, double *out, int ncomp)
{
    const size_t n = (size_t)ncomp * o->N;
    double *t1 = (double *)malloc(sizeof(double) * n);
    switch (filt) {
    case 0: memcpy(out, in, sizeof(double) * n); break;                 /* I */
    case 1: binomial(o, in, out, ncomp); break;                          /* B */
    case 2: binomial(o, in, t1, ncomp); binomial(o, t1, out, ncomp); break; /* B^2 */
    case 3: {                                                            /* B - B^2 */
        binomial(o, in, t1, ncomp); binomial(o, t1, out, ncomp);
        for (size_t k = 0; k < n; k++) out[k] = t1[k] - out[k];
        break; }
    case 4: binomial(o, in, out, ncomp);                                 /* I - B */
        for (size_t k = 0; k < n; k++) out[k] = in[k] - out[k];
        break;
    case 5: case 6: kernel_filter(o, filt, s, in, out, ncomp); break;    /* G_s, L_s */
    }
    free(t1);
}

void orc_filter(void *h, int filt, int s, int fm, const double *in, double *out, int ncomp)
{
    apply_filter_b((Orc *)h, filt, s, fm, in, out, ncomp);
}

/* The d-dimensional kernel of G_s / L_s ((2R+1)^d, x fastest); returns R. */
int orc_kernel(void *h, int filt, int s, double *out)
{
    double *K;
    const Orc *o = (const Orc *)h;
    const int R = kernel_build(o, filt, s, &K), W = 2 * R + 1;
    if (out) memcpy(out, K, sizeof(double) * W * W * (o->d == 3 ? W : 1));
    free(K);
    return R;
}

/* ------------------------------------------------------------------ */
/* Mean-profile band weights (eq. 3d-mp-band-weights).  Reading: the    */
/* wall distance of fluid row y is d_w = min(y + 1/2, ny - 1/2 - y)     */
/* (walls at y = -1/2 and ny - 1/2); centres are log-spaced between     */
/* dmin and dmax; sigma is the centre spacing in ln d_w; A_j makes the  */
/* discrete sum over rows equal one.                                    */
/* ------------------------------------------------------------------ */
static void band_weights(const Orc *o, int nb, double dmin, double dmax, double *w)
{
    const int ny = o->c.ny;
    double sig = nb > 1 ? (log(dmax) - log(dmin)) / (nb - 1) : 1.0;
    for (int j = 0; j < nb; j++) {
        double lc = log(dmin) + j * sig;
        double A = 0;
        for (int y = 0; y < ny; y++) {
            double dw = fmin(y + 0.5, ny - 0.5 - y);
            double t = (log(dw) - lc) / sig;
            w[j * ny + y] = exp(-0.5 * t * t);
            A += w[j * ny + y];
        }
        for (int y = 0; y < ny; y++) w[j * ny + y] /= A;
    }
}

void orc_band_weights(void *h, int nb, double dmin, double dmax, double *w)
{
    band_weights((Orc *)h, nb, dmin, dmax, w);
}

/* ------------------------------------------------------------------ */
/* QoIs and their sensitivities V = dQ/dv (Sec. 4.1, App. A).          */
/*   E_R = 1/2 sum |R v|^2,     V = R(R v)                              */
/*   Z_R = 1/2 sum |R curl v|^2, V = curl^T(R(R curl v))                */
/*   mp_j = sum w_j(y) v_x,     V = w_j(y) e_x                          */
/* The integral is the sum over cells with unit cell volume.            */
/* ------------------------------------------------------------------ */
static void qoi_and_sens(const Orc *o, const orc_closure *cl, const double *bw,
                         const double *v, double *q, double *V /* nq*d*N or NULL */)
{
    const long N = o->N;
    const int d = o->d, nc = d == 2 ? 1 : 3;
    double *w = (double *)malloc(sizeof(double) * nc * N);
    double *r1 = (double *)malloc(sizeof(double) * 3 * N);
    double *r2 = (double *)malloc(sizeof(double) * 3 * N);
    orc_curl((void *)o, v, w);
    for (int k = 0; k < cl->nq; k++) {
        double *Vk = V ? V + (size_t)k * d * N : NULL;
        if (cl->kind[k] == 0) {
            apply_filter_b(o, cl->filt[k], cl->fs[k], cl->fm[k], v, r1, d);
            double s = 0;
            for (long xi = 0; xi < N; xi++) {
                const long x = o->rev_sums ? N - 1 - xi : xi;
                for (int a = 0; a < d; a++) s += 0.5 * r1[a * N + x] * r1[a * N + x];
            }
            q[k] = s;
            if (Vk) apply_filter_b(o, cl->filt[k], cl->fs[k], cl->fm[k], r1, Vk, d);
        } else if (cl->kind[k] == 1) {
            apply_filter_b(o, cl->filt[k], cl->fs[k], cl->fm[k], w, r1, nc);
            double s = 0;
            for (long xi = 0; xi < N; xi++) {
                const long x = o->rev_sums ? N - 1 - xi : xi;
                for (int a = 0; a < nc; a++) s += 0.5 * r1[a * N + x] * r1[a * N + x];
            }
            q[k] = s;
            if (Vk) {
                apply_filter_b(o, cl->filt[k], cl->fs[k], cl->fm[k], r1, r2, nc);
                curl_adjoint(o, r2, Vk);
            }
        } else {
            const double *wj = bw + (size_t)cl->band[k] * o->c.ny;
            double s = 0;
            for (long xi = 0; xi < N; xi++) {
                const long x = o->rev_sums ? N - 1 - xi : xi;
                int y = (int)((x / o->c.nx) % o->c.ny);
                s += wj[y] * v[x];
            }
            q[k] = s;
            if (Vk) {
                for (long x = 0; x < N; x++) {
                    int y = (int)((x / o->c.nx) % o->c.ny);
                    Vk[x] = wj[y];
                    for (int a = 1; a < d; a++) Vk[a * N + x] = 0.0;
                }
            }
        }
    }
    free(w); free(r1); free(r2);
}

/* Python-facing: QoIs and sensitivities of a given velocity field. */
int orc_qoi(void *h, const orc_closure *cl, const double *v, double *q, double *V)
{
    Orc *o = (Orc *)h;
    double *bw = (double *)calloc((size_t)(cl->nbands > 0 ? cl->nbands : 1) * o->c.ny, sizeof(double));
    if (cl->nbands > 0) band_weights(o, cl->nbands, cl->dmin, cl->dmax, bw);
    qoi_and_sens(o, cl, bw, v, q, V);
    free(bw);
    return 0;
}

static double field_dot(const Orc *o, const double *a, const double *b)
{
    double s = 0;
    const long n = (long)o->d * o->N;
    for (long ki = 0; ki < n; ki++) {
        const long k = o->rev_sums ? n - 1 - ki : ki;
        s += a[k] * b[k];
    }
    return s;
}

/* Plain Cholesky of an SPD n x n matrix (row-major); returns 0 and the
 * lower factor L, or the index+1 of the first pivot <= tol. */
static int cholesky(const double *A, int n, double *L, double tol)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; j++) {
        double s = A[j * n + j];
        for (int k = 0; k < j; k++) s -= L[j * n + k] * L[j * n + k];
        if (!(s > tol)) return j + 1;
        L[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; i++) {
            double t = A[i * n + j];
            for (int k = 0; k < j; k++) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    return 0;
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 on success. */
static int invert(const double *A, int n, double *Ainv)
{
    double M[OQMAX][2 * OQMAX];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++)
            M[i][j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++) if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return -1;
        if (p != c) for (int j = 0; j < 2 * n; j++) { double t = M[p][j]; M[p][j] = M[c][j]; M[c][j] = t; }
        double piv = M[c][c];
        for (int j = 0; j < 2 * n; j++) M[c][j] /= piv;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double fct = M[r][c];
            if (fct != 0.0) for (int j = 0; j < 2 * n; j++) M[r][j] -= fct * M[c][j];
        }
    }
    for (int i = 0; i < n; i++) for (int j = 0; j < n; j++) Ainv[i * n + j] = M[i][j + n];
    return 0;
}

/* Singularity rule shared in meaning with the GPU path (reading R-Gram):
 * the Gram matrix is treated as singular when a Cholesky pivot is not
 * above 1e-14 times its largest diagonal entry. */
static int gram_singular(const double *G, int n)
{
    double mx = 0, L[OQMAX * OQMAX];
    for (int i = 0; i < n; i++) if (G[i * n + i] > mx) mx = G[i * n + i];
    if (!(mx > 0)) return 1;
    return cholesky(G, n, L, 1e-14 * mx) != 0;
}

/* Patterns (eq. O-from-V with the orthogonality conditions and c_ii = 1):
 * given the Gram matrix G_kl = <V_k, V_l>, the conditions <V_k, O_i> = 0
 * (k != i) make row i of c proportional to row i of G^{-1}; c_ii = 1 fixes
 * the factor: c_ij = (G^{-1})_ij / (G^{-1})_ii.  Writes G, O fields and
 * den_i = <V_i, O_i> computed as a field inner product.  Returns 1 when G
 * is singular (O and den untouched). */
static int patterns(const Orc *o, int nq, const double *V, double *G, double *O, double *den)
{
    const long n = (long)o->d * o->N;
    for (int k = 0; k < nq; k++)
        for (int l = 0; l < nq; l++)
            G[k * nq + l] = field_dot(o, V + (size_t)k * n, V + (size_t)l * n);
    if (gram_singular(G, nq)) return 1;
    double Gi[OQMAX * OQMAX];
    if (invert(G, nq, Gi)) return 1;
    for (int i = 0; i < nq; i++) {
        double *Oi = O + (size_t)i * n;
        for (long x = 0; x < n; x++) Oi[x] = 0;
        for (int j = 0; j < nq; j++) {
            double cij = Gi[i * nq + j] / Gi[i * nq + i];
            const double *Vj = V + (size_t)j * n;
            for (long x = 0; x < n; x++) Oi[x] += cij * Vj[x];
        }
        den[i] = field_dot(o, V + (size_t)i * n, Oi);
    }
    return 0;
}

/* The correction in its reduced form, equal to the literal patterns in
 * exact arithmetic (pinned by the oracle tests): beta = G^-1 dQ,
 * dv = sum_j beta_j V_j, gamma_k = dQ_k (G^-1)_kk.  Used only by the
 * diagnostic of orc_set_reduced_form.  Returns 1 when G is singular. */
static int reduced_correction(Orc *o, int nq, const double *V, const double *dq, double *gamma)
{
    const long n = (long)o->d * o->N;
    double G[OQMAX * OQMAX], Gi[OQMAX * OQMAX];
    for (int k = 0; k < nq; k++)
        for (int l = 0; l < nq; l++)
            G[k * nq + l] = field_dot(o, V + (size_t)k * n, V + (size_t)l * n);
    if (gram_singular(G, nq) || invert(G, nq, Gi)) return 1;
    for (int j = 0; j < nq; j++) {
        double b = 0;
        for (int k = 0; k < nq; k++) b += Gi[j * nq + k] * dq[k];
        const double *Vj = V + (size_t)j * n;
        for (long x = 0; x < n; x++) o->dv[x] += b * Vj[x];
        gamma[j] = dq[j] * Gi[j * nq + j];
    }
    return 0;
}

int orc_patterns(void *h, const orc_closure *cl, const double *v, double *q, double *V,
                 double *G, double *O, double *den)
{
    Orc *o = (Orc *)h;
    orc_qoi(h, cl, v, q, V);
    return patterns(o, cl->nq, V, G, O, den);
}

/* Literal TO correction for a given predictor velocity and dQ:
 * gamma_i = dQ_i / <V_i, O_i> (eq. tau-from-dQ-for-tracking),
 * dv = sum_i gamma_i O_i (eq. TO-ansatz).  Returns 1 if G is singular
 * (dv = 0, gamma = 0). */
int orc_to_correction(void *h, const orc_closure *cl, const double *v, const double *dq,
                      double *dv, double *gamma)
{
    Orc *o = (Orc *)h;
    const long n = (long)o->d * o->N;
    double *V = (double *)malloc(sizeof(double) * cl->nq * n);
    double *O = (double *)malloc(sizeof(double) * cl->nq * n);
    double q[OQMAX], G[OQMAX * OQMAX], den[OQMAX];
    int sing = orc_patterns(h, cl, v, q, V, G, O, den);
    for (long x = 0; x < n; x++) dv[x] = 0;
    for (int i = 0; i < cl->nq; i++) {
        gamma[i] = sing ? 0.0 : dq[i] / den[i];
        if (!sing) for (long x = 0; x < n; x++) dv[x] += gamma[i] * O[(size_t)i * n + x];
    }
    free(V); free(O);
    return sing;
}

/* ------------------------------------------------------------------ */
/* Eddy-viscosity substrates (Sec. 5).                                  */
/* ------------------------------------------------------------------ */
/* Smagorinsky closed form: tau_eff = (tau + sqrt(tau^2 + 18 C^2 |Pi|/rho))/2,
 * |Pi| = sqrt(2 Pi:Pi), Pi_ab = sum_i c_ia c_ib (f_i - feq_i(rho, u)). */
double orc_tau_smag(int lattice, double tau, double C, const double *f, double rho, const double *u)
{
    Orc o; memset(&o, 0, sizeof o);
    o.Q = lattice_tables(lattice, o.cv, o.w);
    o.d = lattice == 0 ? 2 : 3;
    double Pi[3][3] = {{0}};
    for (int i = 0; i < o.Q; i++) {
        double fneq = f[i] - feq_one(&o, i, rho, u);
        for (int a = 0; a < o.d; a++)
            for (int b = 0; b < o.d; b++) Pi[a][b] += o.cv[i][a] * o.cv[i][b] * fneq;
    }
    double PP = 0;
    for (int a = 0; a < o.d; a++) for (int b = 0; b < o.d; b++) PP += Pi[a][b] * Pi[a][b];
    double nPi = sqrt(2.0 * PP);
    return 0.5 * (tau + sqrt(tau * tau + 18.0 * C * C * nPi / rho));
}

/* WALE: g_ij = d_j v_i by central differences, S = sym(g),
 * S^d_ij = (g_ik g_kj + g_jk g_ki)/2 - delta_ij g_lk g_kl / 3,
 * nu_t = C^2 (S^d:S^d)^{3/2} / ((S:S)^{5/2} + (S^d:S^d)^{5/4}) (0 when the
 * denominator vanishes), tau_eff = tau + nu_t / c_s^2. */
static void tau_wale(const Orc *o, const double *v, double *taueff)
{
    const long N = o->N;
    const double C = o->c.cmodel, tau = o->c.tau;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < o->c.nz; z++)
        for (int y = 0; y < o->c.ny; y++)
            for (int x = 0; x < o->c.nx; x++) {
                long xc = cell(o, x, y, z);
                double g[3][3];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        g[i][j] = dcen(o, v + i * N, j, x, y, z);
                double g2[3][3], tr = 0;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        g2[i][j] = 0;
                        for (int k = 0; k < 3; k++) g2[i][j] += g[i][k] * g[k][j];
                    }
                for (int k = 0; k < 3; k++) tr += g2[k][k];
                double SS = 0, SdSd = 0;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        double S = 0.5 * (g[i][j] + g[j][i]);
                        double Sd = 0.5 * (g2[i][j] + g2[j][i]) - (i == j ? tr / 3.0 : 0.0);
                        SS += S * S; SdSd += Sd * Sd;
                    }
                double den = pow(SS, 2.5) + pow(SdSd, 1.25);
                double nut = den > 0 ? C * C * pow(SdSd, 1.5) / den : 0.0;
                taueff[xc] = tau + 3.0 * nut;
            }
}

void orc_tau_wale_field(void *h, const double *v, double *taueff) { tau_wale((Orc *)h, v, taueff); }

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.    */
/* ------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normals for the LRS residual of one step.  Counter layout:
 * ctr = (block, step_lo, step_hi, 0x4C525331 "LRS1"), key = (seed_lo,
 * seed_hi); each block gives four normals by Box-Muller (1958) on the
 * pairs (r0,r1) and (r2,r3), with u = (r + 1/2) 2^-32. */
void orc_lrs_normals(uint64_t seed, long step, int n, double *z)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int blk = 0; 4 * blk < n; blk++) {
        uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32), 0x4C525331u};
        uint32_t r[4];
        orc_philox(ctr, key, r);
        for (int p = 0; p < 2; p++) {
            double u1 = ((double)r[2 * p] + 0.5) * 2.3283064365386963e-10;
            double u2 = ((double)r[2 * p + 1] + 0.5) * 2.3283064365386963e-10;
            double rad = sqrt(-2.0 * log(u1));
            int k0 = 4 * blk + 2 * p;
            if (k0 < n) z[k0] = rad * cos(2.0 * OPI * u2);
            if (k0 + 1 < n) z[k0 + 1] = rad * sin(2.0 * OPI * u2);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Closure set-up.                                                      */
/* ------------------------------------------------------------------ */
int orc_set_closure(void *h, const orc_closure *cl, const double *qref, long nref)
{
    Orc *o = (Orc *)h;
    free(o->V); free(o->O); free(o->bandw); free(o->qref); free(o->Chist);
    o->V = o->O = o->bandw = o->qref = o->Chist = NULL;
    o->have_closure = 0;
    if (!cl) return 0;
    if (cl->nq < 1 || cl->nq > OQMAX) return -1;
    /* a history model reads its inputs from the records of the h steps
     * before the first corrected one, in scaled units fixed in advance */
    if (cl->h < 0) return -1;
    if (cl->h > 0 && (cl->mode != 2 || !cl->have_scale || !cl->Chist || cl->spinup < o->step + cl->h)) return -1;
    o->cl = *cl;
    o->cl.Chist = NULL;
    if (cl->h > 0) {
        const size_t len = (size_t)(2 * cl->h + 1) * cl->nq + 1;
        o->Chist = (double *)malloc(sizeof(double) * len * cl->nq);
        memcpy(o->Chist, cl->Chist, sizeof(double) * len * cl->nq);
    }
    const long n = (long)o->d * o->N;
    o->V = (double *)malloc(sizeof(double) * cl->nq * n);
    o->O = (double *)malloc(sizeof(double) * cl->nq * n);
    int nb = cl->nbands > 0 ? cl->nbands : 1;
    o->bandw = (double *)calloc((size_t)nb * o->c.ny, sizeof(double));
    if (cl->nbands > 0) band_weights(o, cl->nbands, cl->dmin, cl->dmax, o->bandw);
    if (cl->mode == 2) {
        /* Sigma must be SPD; the all-zero matrix (a noiseless model) is
         * accepted with L = 0. */
        int allzero = 1;
        for (int k = 0; k < cl->nq * cl->nq; k++) if (cl->Sigma[k] != 0.0) allzero = 0;
        if (allzero) memset(o->L, 0, sizeof o->L);
        else if (cholesky(cl->Sigma, cl->nq, o->L, 0.0)) return -1;
    }
    if (qref && nref > 0) {
        o->qref = (double *)malloc(sizeof(double) * nref * cl->nq);
        memcpy(o->qref, qref, sizeof(double) * nref * cl->nq);
        o->nref = nref;
    } else o->nref = 0;
    o->s_set = 0;
    if (cl->have_scale) { memcpy(o->s, cl->scale, sizeof(double) * cl->nq); o->s_set = 1; }
    o->have_closure = 1;
    return 0;
}

/* dQ for the step (Sec. 4.3 tracking; Sec. 4.4 LRS, eq. LRS).
 * LRS reading: scaled QoIs z = q / s with a per-QoI scale s (given, or
 * |q*| at the first corrected step, zero replaced by one; a history model
 * needs it given).  The model input is
 *   x = [z^{n-1}, ..., z^{n-h}, z*^n, z*^{n-1}, ..., z*^{n-h}, 1],
 * where z*^m are the predictor QoIs of step m and z^m the corrected ones,
 * q^m = q*^m + dQ^m (q*^m when that step's correction was skipped); the
 * model predicts the corrected scaled QoIs z = x C + eta, eta ~ N(mu, Sigma),
 * and the correction is dQ = s z - q*.  h = 0 leaves x = [z*^n, 1]. */
static void closure_dq(Orc *o, const double *qs, double *dq)
{
    const int nq = o->cl.nq, h = o->cl.h;
    for (int k = 0; k < nq; k++) dq[k] = 0.0;
    if (o->step < o->cl.spinup || o->cl.mode == 0) return;
    if (o->cl.mode == 1) {
        if (o->step < o->nref)
            for (int k = 0; k < nq; k++) dq[k] = o->qref[o->step * nq + k] - qs[k];
        return;
    }
    if (!o->s_set) {
        for (int k = 0; k < nq; k++) o->s[k] = qs[k] != 0.0 ? fabs(qs[k]) : 1.0;
        o->s_set = 1;
    }
    double z[OQMAX], eta[OQMAX];
    orc_lrs_normals(o->cl.seed, o->step, nq, z);
    for (int k = 0; k < nq; k++) {
        eta[k] = o->cl.mu[k];
        for (int j = 0; j <= k; j++) eta[k] += o->L[k * nq + j] * z[j];
    }
    const long len = (long)(2 * h + 1) * nq + 1;
    const double *C = h > 0 ? o->Chist : o->cl.C;
    double *x = (double *)malloc(sizeof(double) * len);
    for (int r = 1; r <= h; r++) {
        const orc_rec *rc = &o->recs[o->step - r];   /* records are indexed by step */
        for (int i = 0; i < nq; i++) {
            const double qc = rc->q[i] + ((rc->flags & 2) ? 0.0 : rc->dq[i]);
            x[(long)(r - 1) * nq + i] = qc / o->s[i];
            x[(long)(h + r) * nq + i] = rc->q[i] / o->s[i];
        }
    }
    for (int i = 0; i < nq; i++) x[(long)h * nq + i] = qs[i] / o->s[i];
    x[len - 1] = 1.0;
    for (int k = 0; k < nq; k++) {
        double zh = eta[k];
        for (long r = 0; r < len; r++) zh += x[r] * C[r * nq + k];
        dq[k] = o->s[k] * zh - qs[k];
    }
    free(x);
}

/* ------------------------------------------------------------------ */
/* One LES step (eqs. LES-1..LES-3 with the TO correction).            */
/* ------------------------------------------------------------------ */
static void step_once(Orc *o)
{
    const long N = o->N;
    const int d = o->d, Q = o->Q;
    orc_rec rec; memset(&rec, 0, sizeof rec);
    rec.step = o->step;

    /* (1) stream, (2) moments of the post-streaming state v^n */
    stream(o, o->fp, o->f);
    moments(o, o->f, o->rho, o->v);

    /* bookkeeping of the post-streaming state: mass, momentum, E and Z of v^n */
    {
        double m = 0, p[3] = {0, 0, 0}, e = 0, zz = 0;
        int bad = 0;
        for (long x = 0; x < N; x++) {
            m += o->rho[x];
            double u2 = 0;
            for (int a = 0; a < d; a++) {
                double va = o->v[a * N + x];
                p[a] += o->rho[x] * va;
                e += 0.5 * va * va;
                u2 += va * va;
            }
            if (!(u2 <= 0.25)) bad = 1;   /* also catches NaN */
        }
        int nc = d == 2 ? 1 : 3;
        double *w = (double *)malloc(sizeof(double) * nc * N);
        orc_curl(o, o->v, w);
        for (long x = 0; x < (long)nc * N; x++) zz += 0.5 * w[x] * w[x];
        free(w);
        rec.mass = m; rec.mom[0] = p[0]; rec.mom[1] = p[1]; rec.mom[2] = p[2];
        rec.diag_e = e; rec.diag_z = zz;
        if (bad) rec.flags |= 1;
    }

    /* (3) effective relaxation time (Sec. 5) */
    if (o->c.substrate == 2) tau_wale(o, o->v, o->taueff);
    else {
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; x++) {
            if (o->c.substrate == 1) {
                double fl[19], u[3] = {0, 0, 0};
                for (int i = 0; i < Q; i++) fl[i] = o->f[i * N + x];
                for (int a = 0; a < d; a++) u[a] = o->v[a * N + x];
                o->taueff[x] = orc_tau_smag(o->c.lattice, o->c.tau, o->c.cmodel, fl, o->rho[x], u);
            } else o->taueff[x] = o->c.tau;
        }
    }

    /* (4) body force and predictor velocity v* = v + F/rho */
    #pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        int y = (int)((x / o->c.nx) % o->c.ny);
        double F[3] = {0, 0, 0};
        if (o->c.force_kind == 1) F[0] = o->c.force_amp * sin(2.0 * OPI * o->c.force_k * y / o->c.ny);
        else if (o->c.force_kind == 2) F[0] = o->c.force_amp;
        for (int a = 0; a < d; a++) {
            F[a] -= o->c.drag * o->rho[x] * o->v[a * N + x];
            o->vs[a * N + x] = o->v[a * N + x] + F[a] / o->rho[x];
            if (o->fp32_store) o->vs[a * N + x] = (double)(float)o->vs[a * N + x];
        }
    }

    /* (5) TO correction on the predictor v^{p,n*} */
    for (long k = 0; k < (long)d * N; k++) o->dv[k] = 0.0;
    if (o->have_closure) {
        const int nq = o->cl.nq;
        double qs[OQMAX], G[OQMAX * OQMAX], den[OQMAX], dq[OQMAX];
        qoi_and_sens(o, &o->cl, o->bandw, o->vs, qs, o->V);
        closure_dq(o, qs, dq);
        rec.nq = nq;
        for (int k = 0; k < nq; k++) { rec.q[k] = qs[k]; rec.dq[k] = dq[k]; }
        int sing = o->reduced ? reduced_correction(o, nq, o->V, dq, rec.gamma) : patterns(o, nq, o->V, G, o->O, den);
        if (sing) rec.flags |= 2;
        else if (!o->reduced) {
            for (int i = 0; i < nq; i++) {
                double g = dq[i] / den[i];
                rec.gamma[i] = g;
                const double *Oi = o->O + (size_t)i * d * N;
                for (long k = 0; k < (long)d * N; k++) o->dv[k] += g * Oi[k];
            }
        }
    }

    /* (6) relax and force in one difference (eqs. LES-1, LES-2):
     * f^p = f - (f - feq(rho, v))/tau_eff + feq(rho, v + dv_F + dv_SGS) - feq(rho, v) */
    #pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double u[3] = {0, 0, 0}, uc[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) {
            u[a] = o->v[a * N + x];
            uc[a] = o->vs[a * N + x] + o->dv[a * N + x];
        }
        for (int i = 0; i < Q; i++) {
            double fi = o->f[i * N + x];
            double fe = feq_one(o, i, o->rho[x], u);
            double fa = fi - (fi - fe) / o->taueff[x];
            o->fp[i * N + x] = fa + (feq_one(o, i, o->rho[x], uc) - fe);
            if (o->fp32_store)
                o->fp[i * N + x] = o->w[i] + (double)(float)(o->fp[i * N + x] - o->w[i]);
        }
    }

    /* (7) record */
    if (o->nrec == o->caprec) {
        o->caprec = o->caprec ? 2 * o->caprec : 1024;
        o->recs = (orc_rec *)realloc(o->recs, sizeof(orc_rec) * o->caprec);
    }
    o->recs[o->nrec++] = rec;
    o->step++;
}

/* Diagnostic of the FP32 storage floor (not part of the method): with it on,
 * the state is rounded to the nearest FP32 value where an FP32 run stores it
 * -- the post-collision populations as deviations f - w from the lattice
 * weights, and the predictor velocity v* before the TO step -- while all
 * arithmetic stays FP64.  The difference to a plain FP64 run measures what
 * FP32 storage alone costs. */
void orc_set_fp32_store(void *h, int on) { ((Orc *)h)->fp32_store = on ? 1 : 0; }

/* Diagnostic of the FP64 resolution of a closure (not part of the method):
 * with it on, the global sums of the TO step (QoIs, Gram entries, pattern
 * norms) run over the cells in reverse order.  Any implementation that sums
 * in another order differs from the oracle by at least what this twin does;
 * a near-singular Gram system amplifies that difference every step. */
void orc_set_reverse_sums(void *h, int on) { ((Orc *)h)->rev_sums = on ? 1 : 0; }

/* Diagnostic of the FP64 resolution of a closure (not part of the method):
 * with it on, the correction is formed in its reduced form
 * dv = sum_j (G^-1 dQ)_j V_j, gamma_k = dQ_k (G^-1)_kk instead of the literal
 * patterns O_i and norms <V_i, O_i> -- the same value in exact arithmetic,
 * different in its rounding when G is near-singular. */
void orc_set_reduced_form(void *h, int on) { ((Orc *)h)->reduced = on ? 1 : 0; }

int orc_step(void *h, long n)
{
    Orc *o = (Orc *)h;
    for (long k = 0; k < n; k++) step_once(o);
    return 0;
}

long orc_nrec(void *h) { return ((Orc *)h)->nrec; }

void orc_get_recs(void *h, long first, long count, orc_rec *out)
{
    Orc *o = (Orc *)h;
    for (long k = 0; k < count; k++) out[k] = o->recs[first + k];
}

/* Current LRS scale vector (valid once set). */
int orc_get_scale(void *h, double *s)
{
    Orc *o = (Orc *)h;
    if (!o->s_set) return 0;
    memcpy(s, o->s, sizeof(double) * o->cl.nq);
    return 1;
}

/* OpenMP threads of the oracle's cell loops (its results do not depend on
 * them: global sums are sequential). */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_get_threads(void) { return omp_get_max_threads(); }

int orc_sizeof_rec(void) { return (int)sizeof(orc_rec); }
int orc_sizeof_closure(void) { return (int)sizeof(orc_closure); }
int orc_sizeof_cfg(void) { return (int)sizeof(orc_cfg); }

// lbm_fit.cpp -- host-side fit of the LRS model (Sec. 4.4): regularised
// least squares for C with a per-QoI penalty, and the residual statistics.
//
// Rows x^n = [z^{n-1}, ..., z^{n-h}, z*^n, ..., z*^{n-h}, 1] (z = q / s) of a
// recorded trajectory, targets z^n.  The normal matrix A = X^T X and the
// right-hand sides X^T Y are accumulated in cache-sized row blocks (upper
// triangle, threads over column tiles), then each column i solves
// (A + lam_i I) c_i = X^T y_i by a blocked right-looking Cholesky
// factorisation whose trailing updates are split over threads.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {
int set_error(int code, const char* msg);
}

namespace {

constexpr int kRowBlk = 64;    // trajectory rows per accumulation block
constexpr int kTile = 96;      // column tile of the normal-matrix update
constexpr int kNb = 96;        // Cholesky block size

int nthreads()
{
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 32u));
}

template <typename F>
void parallel_for(int n, F&& f)
{
    const int nt = std::min(nthreads(), std::max(n, 1));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = t; i < n; i += nt) f(i);
        });
    for (auto& x : th) x.join();
}

// A[r0.., c0..] (upper part, row-major len x len) += Xb^T Xb over the tile;
// Xb is nr x len, row-major.
__attribute__((target_clones("arch=haswell", "default")))
void gram_tile(double* A, int len, const double* Xb, int nr, int r0, int r1, int c0, int c1)
{
    for (int i = r0; i < r1; ++i) {
        double* Ai = A + (size_t)i * len;
        const int cs = std::max(c0, i);
        for (int k = 0; k < nr; ++k) {
            const double xi = Xb[(size_t)k * len + i];
            if (xi == 0.0) continue;
            const double* xk = Xb + (size_t)k * len;
            for (int j = cs; j < c1; ++j) Ai[j] += xi * xk[j];
        }
    }
}

// Trailing update of the Cholesky factorisation: for rows i in [r0, r1) and
// columns j in [c0, min(c1, i+1)), A[i][j] -= sum_k P[k][i] P[k][j], with
// P the transposed panel (kb x n, row-major) so the inner loop runs along
// contiguous j.
__attribute__((target_clones("arch=haswell", "default")))
void chol_update(double* A, int n, const double* P, int kb, int r0, int r1, int c0, int c1)
{
    for (int jc = c0; jc < c1; jc += kTile) {   // column tiles: the row segment stays in L1
        const int je = std::min(c1, jc + kTile);
        for (int i = r0; i < r1; ++i) {
            double* Ai = A + (size_t)i * n;
            const int ce = std::min(je, i + 1);
            if (ce <= jc) continue;
            for (int k = 0; k < kb; ++k) {
                const double a = P[(size_t)k * n + i];
                const double* Pk = P + (size_t)k * n;
                for (int j = jc; j < ce; ++j) Ai[j] -= a * Pk[j];
            }
        }
    }
}

// In-place Cholesky A = L L^T of the lower triangle of a row-major n x n
// matrix; false if a pivot is not positive.
bool cholesky(double* A, int n)
{
    std::vector<double> P((size_t)kNb * n);
    for (int k0 = 0; k0 < n; k0 += kNb) {
        const int k1 = std::min(n, k0 + kNb), kb = k1 - k0;
        // diagonal block
        for (int j = k0; j < k1; ++j) {
            double d = A[(size_t)j * n + j];
            for (int k = k0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
            if (!(d > 0)) return false;
            const double ljj = std::sqrt(d);
            A[(size_t)j * n + j] = ljj;
            for (int i = j + 1; i < k1; ++i) {
                double s = A[(size_t)i * n + j];
                for (int k = k0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
                A[(size_t)i * n + j] = s / ljj;
            }
        }
        if (k1 == n) break;
        // panel below the diagonal block: L21 = A21 L11^-T (rows independent),
        // and its transpose for the update
        parallel_for((n - k1 + kTile - 1) / kTile, [&](int t) {
            const int r0 = k1 + t * kTile, r1 = std::min(n, r0 + kTile);
            for (int i = r0; i < r1; ++i)
                for (int j = k0; j < k1; ++j) {
                    double s = A[(size_t)i * n + j];
                    for (int k = k0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
                    A[(size_t)i * n + j] = s / A[(size_t)j * n + j];
                    P[(size_t)(j - k0) * n + i] = A[(size_t)i * n + j];
                }
        });
        // trailing matrix A22 -= L21 L21^T, tiles of rows
        const int nt = (n - k1 + kTile - 1) / kTile;
        parallel_for(nt, [&](int t) {
            const int r0 = k1 + t * kTile, r1 = std::min(n, r0 + kTile);
            chol_update(A, n, P.data(), kb, r0, r1, k1, r1);
        });
    }
    return true;
}

void chol_solve(const double* L, int n, double* b)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * b[k];
        b[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * b[k];
        b[i] = s / L[(size_t)i * n + i];
    }
}

}  // namespace

extern "C" int lbm_lrs_fit(int nq, int h, long nsteps, const double* q_star, const double* dq, const int* flags,
                           const double* scale, double lambda, double* C, double* mu, double* Sigma, double* s_out)
{
    if (nq < 1 || nq > LBM_MAX_QOI || h < 0 || h > LBM_MAX_HIST)
        return lbm::set_error(LBM_EINVAL, "lrs_fit: nq must be in [1, LBM_MAX_QOI] and h in [0, LBM_MAX_HIST]");
    if (!q_star || !dq || !C || !mu || !Sigma) return lbm::set_error(LBM_EINVAL, "lrs_fit: NULL array");
    if (!(lambda >= 0)) return lbm::set_error(LBM_EINVAL, "lrs_fit: lambda must be >= 0");
    const long M = nsteps - h;   // training rows
    if (M < 2) return lbm::set_error(LBM_EINVAL, "lrs_fit: need at least h + 2 recorded steps");
    const int len = (2 * h + 1) * nq + 1;
    // corrected QoIs q^m = q*^m + dQ^m (q*^m where the step's correction was skipped)
    std::vector<double> qc((size_t)nsteps * nq), s(nq);
    for (long m = 0; m < nsteps; ++m) {
        const bool skip = flags && (flags[m] & 2);
        for (int i = 0; i < nq; ++i) qc[(size_t)m * nq + i] = q_star[(size_t)m * nq + i] + (skip ? 0.0 : dq[(size_t)m * nq + i]);
    }
    // scale: given, or the standard deviation of each QoI over the trajectory
    for (int i = 0; i < nq; ++i) {
        if (scale) {
            s[i] = scale[i];
            if (!(s[i] != 0)) return lbm::set_error(LBM_EINVAL, "lrs_fit: scale entries must be nonzero");
            continue;
        }
        double a = 0, b = 0;
        for (long m = 0; m < nsteps; ++m) a += qc[(size_t)m * nq + i];
        a /= nsteps;
        for (long m = 0; m < nsteps; ++m) b += (qc[(size_t)m * nq + i] - a) * (qc[(size_t)m * nq + i] - a);
        s[i] = std::sqrt(b / nsteps);
        if (s[i] == 0) s[i] = 1;
    }
    auto row = [&](long n, double* x) {   // x^n, n >= h
        for (int r = 1; r <= h; ++r)
            for (int i = 0; i < nq; ++i) {
                x[(size_t)(r - 1) * nq + i] = qc[(size_t)(n - r) * nq + i] / s[i];
                x[(size_t)(h + r) * nq + i] = q_star[(size_t)(n - r) * nq + i] / s[i];
            }
        for (int i = 0; i < nq; ++i) x[(size_t)h * nq + i] = q_star[(size_t)n * nq + i] / s[i];
        x[len - 1] = 1.0;
    };
    // penalties: lam_i = lambda (sigma_i / sigma_1)^2, sigma_i the standard
    // deviation of the scaled corrections over the training rows
    std::vector<double> lam(nq);
    {
        std::vector<double> sig(nq);
        for (int i = 0; i < nq; ++i) {
            double a = 0, b = 0;
            for (long n = h; n < nsteps; ++n) a += (qc[(size_t)n * nq + i] - q_star[(size_t)n * nq + i]) / s[i];
            a /= M;
            for (long n = h; n < nsteps; ++n) {
                const double e = (qc[(size_t)n * nq + i] - q_star[(size_t)n * nq + i]) / s[i] - a;
                b += e * e;
            }
            sig[i] = std::sqrt(b / M);
        }
        for (int i = 0; i < nq; ++i) lam[i] = sig[0] > 0 ? lambda * (sig[i] / sig[0]) * (sig[i] / sig[0]) : lambda;
    }
    // normal equations
    std::vector<double> A((size_t)len * len, 0.0), XtY((size_t)len * nq, 0.0), Xb((size_t)kRowBlk * len);
    const int ntile = (len + kTile - 1) / kTile;
    for (long n0 = h; n0 < nsteps; n0 += kRowBlk) {
        const int nr = (int)std::min<long>(kRowBlk, nsteps - n0);
        for (int k = 0; k < nr; ++k) row(n0 + k, Xb.data() + (size_t)k * len);
        parallel_for(ntile, [&](int t) {
            const int r0 = t * kTile, r1 = std::min(len, r0 + kTile);
            for (int c0 = r0; c0 < len; c0 += kTile) gram_tile(A.data(), len, Xb.data(), nr, r0, r1, c0, std::min(len, c0 + kTile));
            for (int k = 0; k < nr; ++k) {
                const double* x = Xb.data() + (size_t)k * len;
                const long n = n0 + k;
                for (int j = r0; j < r1; ++j)
                    for (int i = 0; i < nq; ++i) XtY[(size_t)j * nq + i] += x[j] * (qc[(size_t)n * nq + i] / s[i]);
            }
        });
    }
    // one Cholesky per column penalty (lower triangle from the upper one)
    std::vector<double> L((size_t)len * len), b(len);
    for (int i = 0; i < nq; ++i) {
        for (int r = 0; r < len; ++r)
            for (int c = 0; c <= r; ++c) L[(size_t)r * len + c] = A[(size_t)c * len + r];
        for (int r = 0; r < len; ++r) L[(size_t)r * len + r] += lam[i];
        if (!cholesky(L.data(), len))
            return lbm::set_error(LBM_EINVAL, "lrs_fit: the regularised normal matrix is not positive definite (use lambda > 0)");
        for (int r = 0; r < len; ++r) b[r] = XtY[(size_t)r * nq + i];
        chol_solve(L.data(), len, b.data());
        for (int r = 0; r < len; ++r) C[(size_t)r * nq + i] = b[r];
    }
    // residual statistics: mean and unbiased sample covariance of z^n - x^n C
    std::vector<double> res((size_t)M * nq);
    const int nchunk = (int)((M + kRowBlk - 1) / kRowBlk);
    parallel_for(nchunk, [&](int t) {
        std::vector<double> x(len);
        const long e = std::min<long>(nsteps, h + (long)(t + 1) * kRowBlk);
        for (long n = h + (long)t * kRowBlk; n < e; ++n) {
            row(n, x.data());
            for (int i = 0; i < nq; ++i) {
                double p = 0;
                for (int j = 0; j < len; ++j) p += x[j] * C[(size_t)j * nq + i];
                res[(size_t)(n - h) * nq + i] = qc[(size_t)n * nq + i] / s[i] - p;
            }
        }
    });
    for (int i = 0; i < nq; ++i) {
        double a = 0;
        for (long r = 0; r < M; ++r) a += res[(size_t)r * nq + i];
        mu[i] = a / M;
    }
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < nq; ++j) {
            double a = 0;
            for (long r = 0; r < M; ++r) a += (res[(size_t)r * nq + i] - mu[i]) * (res[(size_t)r * nq + j] - mu[j]);
            Sigma[i * nq + j] = a / (M - 1);
        }
    if (s_out) std::memcpy(s_out, s.data(), sizeof(double) * nq);
    return LBM_OK;
}

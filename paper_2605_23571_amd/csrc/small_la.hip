// Small dense kernels of the randomized eigendecomposition (Algorithm 1 and the
// REVD variant): ell x ell Cholesky with the inverse of its factor, products of
// small matrices, one-sided Jacobi SVD, two-sided Jacobi symmetric EVD, column
// sign normalisation and the spectral-LMP coefficients.  ell <= 128; each runs
// on one workgroup with the working matrix in LDS.  All orderings and
// reductions are fixed, so results are reproducible run to run.  The
// workgroup-level routines (Cholesky, Jacobi SVD, the shifted Nystrom pass)
// live in nystrom_dev.h, which the batch's persistent sketch launch shares.
#include "nystrom_dev.h"

namespace eda {
namespace {

using nys::chol_inv;
using nys::jacobi_svd;
using nys::rr_pair;

constexpr int ST = 256;   // threads of the small kernels
constexpr int SJ = 1024;  // threads of the Jacobi SVD kernels (one 16-lane row per column pair)
constexpr int SC = 1024;  // threads of the Cholesky kernel (element-parallel updates)

__global__ __launch_bounds__(SC) void k_chol_inv(int l, const double *__restrict__ W, double shift,
                                                 double *__restrict__ C, double *__restrict__ Cinv,
                                                 int32_t *__restrict__ info) {
    extern __shared__ double S[];  // l x l, col-major; upper triangle becomes C; then X (l <= 64)
    __shared__ int fail;
    chol_inv(l, W, shift, C, Cinv, info, S, fail);
}

__global__ void k_sym(int l, double *W) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= l * l) return;
    int i = idx % l, j = idx / l;
    if (i < j) {
        double v = 0.5 * (W[i + j * l] + W[j + i * l]);
        W[i + j * l] = v;
        W[j + i * l] = v;
    }
}

// C = op(A) op(B), all l x l.
__global__ void k_small_gemm(int l, int ta, int tb, const double *__restrict__ A, const double *__restrict__ B,
                             double *__restrict__ C) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= l * l) return;
    int i = idx % l, j = idx / l;
    double v = 0.0;
    for (int k = 0; k < l; k++) {
        double a = ta ? A[k + i * l] : A[i + k * l];
        double b = tb ? B[j + k * l] : B[k + j * l];
        v += a * b;
    }
    C[idx] = v;
}

__global__ __launch_bounds__(SJ) void k_jacobi_svd(int l, const double *__restrict__ T, double *__restrict__ U,
                                                   double *__restrict__ sig) {
    extern __shared__ double A[];  // l x l col-major
    __shared__ int rotated;
    __shared__ double nrm[128];
    jacobi_svd(l, T, U, sig, A, rotated, nrm);
}

// Two-sided cyclic Jacobi EVD of symmetric T (l x l), parallel ordering:
// T V = V diag(lam), lam descending (ties: lower index first).  A round
// rotates the m / 2 disjoint pairs (p_k, q_k) of the round-robin ordering at
// once, A <- J^T A J and V <- V J.  The pairs partition the indices, so A
// splits into 2 x 2 blocks (rows {p_a, q_a}, columns {p_b, q_b}) and each
// block of J^T A J needs only its own entries: (B J_b) first, then J_a^T, the
// same operations per entry as a column pass followed by a row pass.  One
// barrier after the angles, one after the rotations.  V stays in LDS when
// l <= 64 (VL), else in the global scratch Vg.
template <bool VL>
__global__ __launch_bounds__(SJ) void k_jacobi_eig(int l, const double *__restrict__ T, double *__restrict__ Vg,
                                                   double *__restrict__ Vout, double *__restrict__ lam) {
    extern __shared__ double A[];  // l x l (then V, l x l, when VL)
    double *V = VL ? A + l * l : Vg;
    __shared__ double cs[64], sn[64];
    __shared__ int pp[64], qq[64];
    __shared__ int rotated;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < l * l; idx += SJ) {
        A[idx] = T[idx];
        V[idx] = (idx % l == idx / l) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int m = (l + 1) & ~1, half = m / 2;
    const double tol = (double)l * 2.220446049250313e-16;
    for (int sweep = 0; sweep < 60; sweep++) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < m - 1; r++) {
            for (int k = tid; k < half; k += SJ) {
                int p, q;
                rr_pair(m, r, k, p, q);
                double c = 1.0, s = 0.0;
                if (q < l) {
                    double apq = A[p + q * l], app = A[p + p * l], aqq = A[q + q * l];
                    if (apq != 0.0 && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
                        double tau = (aqq - app) / (2.0 * apq);
                        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = c * t;
                        rotated = 1;
                    }
                }
                pp[k] = p;
                qq[k] = q;
                cs[k] = c;
                sn[k] = s;
            }
            __syncthreads();
            // A <- J^T A J, one 2 x 2 block per (a, b); a q index of l (odd l)
            // is the empty slot of the ordering and has no entries.  The row
            // pair a varies fastest, so the lanes of a wave read down columns
            // (distinct LDS banks) rather than along rows (one bank).
            for (int e = tid; e < half * half; e += SJ) {
                const int b = e / half, a = e - b * half;
                const double sa = sn[a], sb = sn[b];
                if (sa == 0.0 && sb == 0.0) continue;
                const double ca = cs[a], cb = cs[b];
                const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
                const bool qav = qa < l, qbv = qb < l;
                // block entries x_rc: row r in {p_a, q_a}, column c in {p_b, q_b}
                double xpp = A[pa + pb * l];
                double xpq = qbv ? A[pa + qb * l] : 0.0;
                double xqp = qav ? A[qa + pb * l] : 0.0;
                double xqq = (qav && qbv) ? A[qa + qb * l] : 0.0;
                if (sb != 0.0) {  // columns: col p = c col p - s col q, col q = s col p + c col q
                    const double yp = cb * xpp - sb * xpq, yq = sb * xpp + cb * xpq;
                    const double zp = cb * xqp - sb * xqq, zq = sb * xqp + cb * xqq;
                    xpp = yp;
                    xpq = yq;
                    xqp = zp;
                    xqq = zq;
                }
                if (sa != 0.0) {  // rows: row p = c row p - s row q, row q = s row p + c row q
                    const double yp = ca * xpp - sa * xqp, yq = sa * xpp + ca * xqp;
                    const double zp = ca * xpq - sa * xqq, zq = sa * xpq + ca * xqq;
                    xpp = yp;
                    xqp = yq;
                    xpq = zp;
                    xqq = zq;
                }
                A[pa + pb * l] = xpp;
                if (qbv) A[pa + qb * l] = xpq;
                if (qav) A[qa + pb * l] = xqp;
                if (qav && qbv) A[qa + qb * l] = xqq;
            }
            // V <- V J
            for (int e = tid; e < half * l; e += SJ) {
                const int b = e / l, i = e - b * l;
                const double sb = sn[b];
                if (sb == 0.0) continue;
                const double cb = cs[b];
                const int pb = pp[b], qb = qq[b];
                const double x = V[i + pb * l], y = V[i + qb * l];
                V[i + pb * l] = cb * x - sb * y;
                V[i + qb * l] = sb * x + cb * y;
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    for (int j = tid; j < l; j += SJ) {
        double dj = A[j + j * l];
        int rank = 0;
        for (int i = 0; i < l; i++) {
            double di = A[i + i * l];
            if (di > dj || (di == dj && i < j)) rank++;
        }
        lam[rank] = dj;
        for (int i = 0; i < l; i++) Vout[i + (long long)rank * l] = V[i + j * l];
    }
}

// Column sign convention: the entry of largest magnitude (lowest index on ties)
// is made positive.  One workgroup per column.
__global__ __launch_bounds__(ST) void k_fix_signs(int n, double *S, long long lds) {
    __shared__ double bv[ST];
    __shared__ int bi[ST];
    double *col = S + (long long)blockIdx.x * lds;
    double best = -1.0;
    int besti = 0;  // a column of NaNs keeps entry 0 (and an in-range index)
    for (int i = threadIdx.x; i < n; i += ST) {
        double a = fabs(col[i]);
        if (a > best) {  // strided scan visits indices in increasing order
            best = a;
            besti = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int w = ST / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double ov = bv[threadIdx.x + w];
            int oi = bi[threadIdx.x + w];
            if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const double sgn = col[bi[0]] < 0 ? -1.0 : 1.0;
    if (sgn < 0)
        for (int i = threadIdx.x; i < n; i += ST) col[i] = -col[i];
}

// d_i = sigma_i^2 - nu (clipped at 0; Nystrom) or lambda_i (REVD), i < k;
// theta from lambda_k(I + A) = 1 + d_{k-1};  coef_i = theta/(1+d_i) - 1,
// coefu_i = sqrt(theta)/sqrt(1+d_i) - 1 (the lmp equation).
__global__ void k_lmp_coef(int k, const double *sig, double nu, int square, int rule, double *eig, double *coef,
                           double *coefu, double *theta_out) {
    __shared__ double th;
    if (threadIdx.x == 0) {
        double s = sig[k - 1];
        double dk = square ? fmax(s * s - nu, 0.0) : s;
        double lk = 1.0 + dk;
        th = rule == EDA_THETA_MID ? 0.5 * (lk + 1.0) : (rule == EDA_THETA_LAMK ? lk : 1.0);
        *theta_out = th;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        double s = sig[i];
        double d = square ? fmax(s * s - nu, 0.0) : s;
        eig[i] = d;
        coef[i] = th / (1.0 + d) - 1.0;
        coefu[i] = sqrt(th) / sqrt(1.0 + d) - 1.0;
    }
}

// The last Nystrom pass with its shifts (nys::nystrom_redo) of one problem.
__global__ __launch_bounds__(SC) void k_nystrom_redo(RedoJob J) {
    extern __shared__ double X[];
    __shared__ nys::RedoLds L;
    __shared__ double nrm[128];
    nys::nystrom_redo(J, X, L, nrm);
}

__global__ void k_axpy_cols(int n, int nb, double alpha, const double *__restrict__ X, long long ldx,
                            double *__restrict__ Y, long long ldy) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * nb) return;
    int i = (int)(idx % n), c = (int)(idx / n);
    Y[i + c * ldy] += alpha * X[i + c * ldx];
}

__global__ void k_copy_cols(int n, int nb, const double *__restrict__ X, long long ldx, double *__restrict__ Y,
                            long long ldy) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * nb) return;
    int i = (int)(idx % n), c = (int)(idx / n);
    Y[i + c * ldy] = X[i + c * ldx];
}

}  // namespace

hipError_t launch_chol_inv(hipStream_t s, int l, const double *W, double shift, double *C, double *Cinv,
                           int32_t *info) {
    const size_t lds = sizeof(double) * l * l * (l <= 64 ? 2 : 1);
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(SC), lds, s, l, W, shift, C, Cinv, info);
    return hipGetLastError();
}

size_t redo_lds(int lmax) { return sizeof(double) * nys::redo_lds_doubles(lmax); }

hipError_t launch_nystrom_redo(hipStream_t s, const RedoJob &job) {
    if (job.l < 1 || job.l > 128 || job.k < 1 || job.k > job.l || job.n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nystrom_redo, dim3(1), dim3(SC), redo_lds(job.l), s, job);
    return hipGetLastError();
}

hipError_t launch_sym(hipStream_t s, int l, double *W) {
    hipLaunchKernelGGL(k_sym, dim3((l * l + 255) / 256), dim3(256), 0, s, l, W);
    return hipGetLastError();
}

hipError_t launch_small_gemm(hipStream_t s, int l, bool ta, bool tb, const double *A, const double *B, double *C) {
    hipLaunchKernelGGL(k_small_gemm, dim3((l * l + 255) / 256), dim3(256), 0, s, l, (int)ta, (int)tb, A, B, C);
    return hipGetLastError();
}

hipError_t launch_jacobi_svd_u(hipStream_t s, int l, double *T, double *U, double *sig) {
    if (l > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(SJ), sizeof(double) * l * l, s, l, T, U, sig);
    return hipGetLastError();
}

hipError_t launch_jacobi_eig(hipStream_t s, int l, double *T, double *Vwork, double *V, double *lam) {
    if (l > 128) return hipErrorInvalidValue;
    if (l < 1) return hipErrorInvalidValue;
    if (l <= 64)
        hipLaunchKernelGGL(k_jacobi_eig<true>, dim3(1), dim3(SJ), sizeof(double) * 2 * l * l, s, l, T, Vwork, V, lam);
    else
        hipLaunchKernelGGL(k_jacobi_eig<false>, dim3(1), dim3(SJ), sizeof(double) * l * l, s, l, T, Vwork, V, lam);
    return hipGetLastError();
}

hipError_t launch_fix_signs(hipStream_t s, int n, int k, double *S, long long lds) {
    hipLaunchKernelGGL(k_fix_signs, dim3(k), dim3(ST), 0, s, n, S, lds);
    return hipGetLastError();
}

hipError_t launch_lmp_coef(hipStream_t s, int k, const double *sig, double nu, int square, int theta_rule,
                           double *eig, double *coef, double *coefu, double *theta_out) {
    hipLaunchKernelGGL(k_lmp_coef, dim3(1), dim3(128), 0, s, k, sig, nu, square, theta_rule, eig, coef, coefu,
                       theta_out);
    return hipGetLastError();
}

hipError_t launch_axpy_cols(hipStream_t s, int n, int nb, double alpha, const double *X, long long ldx, double *Y,
                            long long ldy) {
    long long tot = (long long)n * nb;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nb, alpha, X, ldx, Y,
                       ldy);
    return hipGetLastError();
}

hipError_t launch_copy_cols(hipStream_t s, int n, int nb, const double *X, long long ldx, double *Y, long long ldy) {
    long long tot = (long long)n * nb;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nb, X, ldx, Y, ldy);
    return hipGetLastError();
}

}  // namespace eda

// Small dense kernels of the randomized eigendecomposition (Algorithm 1 and the
// REVD variant): ell x ell Cholesky with the inverse of its factor, products of
// small matrices, one-sided Jacobi SVD, two-sided Jacobi symmetric EVD, column
// sign normalisation and the spectral-LMP coefficients.  ell <= 128; each runs
// on one workgroup with the working matrix in LDS.  All orderings and
// reductions are fixed, so results are reproducible run to run.
#include "eda_internal.h"

namespace eda {
namespace {

constexpr int ST = 256;   // threads of the small kernels
constexpr int SJ = 1024;  // threads of the Jacobi SVD kernels (one 16-lane row per column pair)
constexpr int SC = 1024;  // threads of the Cholesky kernel (element-parallel updates)

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return __shfl(v, 0, 64);
}

// v of lane (lane ^ M) within the 16-lane row, M fixed by the DPP control
// (0x140: M = 15, 0x141: M = 7, 0xB1: M = 1, 0x4E: M = 2), as two 32-bit moves
template <int CTRL>
__device__ __forceinline__ double row_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 16 lanes of a row: an xor butterfly over the masks 15, 7, 1, 2,
// which span the row's lane indices.  Each step adds the same two values on
// both lanes of a pair (in either order), so every lane ends with the same bits.
__device__ __forceinline__ double row_sum(double v) {
    v += row_xor<0x140>(v);
    v += row_xor<0x141>(v);
    v += row_xor<0xB1>(v);
    v += row_xor<0x4E>(v);
    return v;
}

// W = C^T C with C upper triangular (W + shift I), then Cinv = C^-1.
// info = 0 on success, j + 1 if pivot j is not positive.  Right-looking: step j
// takes the pivot, scales row j and updates the trailing upper triangle, all
// threads in parallel (three barriers a step).  The inverse solves C X = I
// from the last row up, X[i] /= C_ii then X[r] -= C_ri X[i] for r < i, in a
// second LDS buffer when l <= 64; for larger l column j of X is built from the
// finished columns, X_ij = -X_jj sum_{k=i}^{j-1} X_ik C_kj, in place.
// S: LDS, l x l doubles (2 l x l when l <= 64); fail: an LDS flag.
__device__ __forceinline__ void chol_inv(int l, const double *__restrict__ W, double shift, double *__restrict__ C,
                                         double *__restrict__ Cinv, int32_t *__restrict__ info, double *S,
                                         int &fail) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < l * l; idx += SC) {
        int i = idx % l, j = idx / l;
        S[idx] = W[idx] + (i == j ? shift : 0.0);
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < l; j++) {
        if (tid == 0) {
            const double d = S[j + j * l];
            if (!(d > 0.0) || !isfinite(d)) fail = j + 1;
            else S[j + j * l] = sqrt(d);
        }
        __syncthreads();
        if (fail) break;
        const double piv = S[j + j * l];
        for (int c = j + 1 + tid; c < l; c += SC) S[j + c * l] /= piv;
        __syncthreads();
        const int m = l - 1 - j;  // trailing block rows/columns j+1 .. l-1
        for (int idx = tid; idx < m * m; idx += SC) {
            const int r = j + 1 + idx % m, c = j + 1 + idx / m;
            if (r <= c) S[r + c * l] -= S[j + r * l] * S[j + c * l];
        }
        __syncthreads();
    }
    if (tid == 0) *info = fail;
    if (fail) return;
    for (int idx = tid; idx < l * l; idx += SC) {
        int i = idx % l, j = idx / l;
        C[idx] = (i <= j) ? S[idx] : 0.0;
    }
    if (l <= 64) {
        double *X = S + l * l;
        for (int idx = tid; idx < l * l; idx += SC) X[idx] = (idx % l == idx / l) ? 1.0 : 0.0;
        __syncthreads();
        for (int i = l - 1; i >= 0; i--) {
            const double cii = S[i + i * l];
            for (int c = i + tid; c < l; c += SC) X[i + c * l] /= cii;
            __syncthreads();
            const int w = l - i;  // columns i .. l-1 of rows 0 .. i-1
            for (int idx = tid; idx < i * w; idx += SC) {
                const int r = idx % i, c = i + idx / i;
                X[r + c * l] -= S[r + i * l] * X[i + c * l];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < l * l; idx += SC) {
            int i = idx % l, j = idx / l;
            Cinv[idx] = (i <= j) ? X[idx] : 0.0;
        }
        return;
    }
    for (int j = 0; j < l; j++) {
        const double xjj = 1.0 / S[j + j * l];
        double v = 0.0;
        const int i = tid;
        if (i < j)
            for (int k = i; k < j; k++) v += S[i + k * l] * S[k + j * l];
        __syncthreads();
        if (i < j) S[i + j * l] = -xjj * v;
        if (i == j) S[j + j * l] = xjj;
        __syncthreads();
    }
    for (int idx = tid; idx < l * l; idx += SC) {
        int i = idx % l, j = idx / l;
        Cinv[idx] = (i <= j) ? S[idx] : 0.0;
    }
}

__global__ __launch_bounds__(SC) void k_chol_inv(int l, const double *__restrict__ W, double shift,
                                                 double *__restrict__ C, double *__restrict__ Cinv,
                                                 int32_t *__restrict__ info) {
    extern __shared__ double S[];  // l x l, col-major; upper triangle becomes C; then X (l <= 64)
    __shared__ int fail;
    chol_inv(l, W, shift, C, Cinv, info, S, fail);
}

// Many independent factorisations in one launch, one workgroup each (the same
// arithmetic as k_chol_inv, so the same bits).
__global__ __launch_bounds__(SC) void k_chol_inv_batch(const CholJob *__restrict__ jobs) {
    extern __shared__ double S[];
    __shared__ int fail;
    const CholJob j = jobs[blockIdx.x];
    chol_inv(j.l, j.W, j.shift, j.C, j.Cinv, j.info, S, fail);
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

// Round-robin pairing of m (even) indices: round r, pair k.
__device__ __forceinline__ void rr_pair(int m, int r, int k, int &p, int &q) {
    auto pos = [&](int x) { return x == 0 ? 0 : ((x - 1 + r) % (m - 1)) + 1; };
    p = pos(k);
    q = pos(m - 1 - k);
    if (p > q) {
        int t = p;
        p = q;
        q = t;
    }
}

// One-sided (Hestenes) Jacobi SVD of T (l x l): columns are rotated until
// mutually orthogonal; then sigma_j = ||t_j||, U[:, rank(j)] = t_j / sigma_j
// with ranks sorting sigma descending (ties: lower index first).
// A: l x l doubles of LDS; rotated, nrm: LDS flags and norms (128).
__device__ __forceinline__ void jacobi_svd(int l, const double *__restrict__ T, double *__restrict__ U,
                                           double *__restrict__ sig, double *A, int &rotated, double *nrm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int idx = tid; idx < l * l; idx += SJ) A[idx] = T[idx];
    __syncthreads();
    const int m = (l + 1) & ~1;
    // a pair is rotated while |t_p^T t_q| > l eps ||t_p|| ||t_q||: below that the
    // product is at the rounding level of the wave sum, and rotating on noise
    // would keep the sweeps from ending
    const double tol = (double)l * 2.220446049250313e-16;
    for (int sweep = 0; sweep < 60; sweep++) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < m - 1; r++) {
            // one 16-lane row per pair (rows of a wave run four pairs at once);
            // a row takes or skips a pair as a whole
            for (int k = tid >> 4; k < m / 2; k += SJ / 16) {
                int p, q;
                rr_pair(m, r, k, p, q);
                if (q >= l) continue;
                double *ap = A + p * l, *aq = A + q * l;
                double al = 0, be = 0, ga = 0;
                for (int i = tid & 15; i < l; i += 16) {
                    al += ap[i] * ap[i];
                    be += aq[i] * aq[i];
                    ga += ap[i] * aq[i];
                }
                al = row_sum(al);
                be = row_sum(be);
                ga = row_sum(ga);
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    double zeta = (be - al) / (2.0 * ga);
                    double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    for (int i = tid & 15; i < l; i += 16) {
                        double x = ap[i], y = aq[i];
                        ap[i] = c * x - sn * y;
                        aq[i] = sn * x + c * y;
                    }
                    if ((tid & 15) == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    for (int j = wave; j < l; j += SJ / 64) {
        double v = 0;
        for (int i = lane; i < l; i += 64) v += A[i + j * l] * A[i + j * l];
        v = wave_sum(v);
        if (lane == 0) nrm[j] = sqrt(v);
    }
    __syncthreads();
    for (int j = tid; j < l; j += SJ) {
        double sj = nrm[j];
        int rank = 0;
        for (int i = 0; i < l; i++) {
            double si = nrm[i];
            if (si > sj || (si == sj && i < j)) rank++;
        }
        sig[rank] = sj;
        double inv = sj > 0 ? 1.0 / sj : 0.0;
        for (int i = 0; i < l; i++) U[i + (long long)rank * l] = A[i + j * l] * inv;
    }
}

__global__ __launch_bounds__(SJ) void k_jacobi_svd(int l, const double *__restrict__ T, double *__restrict__ U,
                                                   double *__restrict__ sig) {
    extern __shared__ double A[];  // l x l col-major
    __shared__ int rotated;
    __shared__ double nrm[128];
    jacobi_svd(l, T, U, sig, A, rotated, nrm);
}

// Many independent SVDs in one launch, one workgroup each (the same
// arithmetic as k_jacobi_svd, so the same bits).
__global__ __launch_bounds__(SJ) void k_jacobi_svd_batch(const JacobiJob *__restrict__ jobs) {
    extern __shared__ double A[];
    __shared__ int rotated;
    __shared__ double nrm[128];
    const JacobiJob j = jobs[blockIdx.x];
    jacobi_svd(j.l, j.T, j.U, j.sig, A, rotated, nrm);
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

// ---------------------------------------------------------------------------
// The shifted Nystrom sketch on the device, one workgroup (SC threads) per
// problem: from Y = A Phi and Phi, what the host-driven path of the Nystrom
// algorithm does when an unshifted Cholesky fails -- CholQR2 of Y, a shifted
// first pass (shifted CholQR3) when the Gram matrix's Cholesky fails; W =
// Phi^T Y and its Cholesky; when that fails the Nystrom shift Y <- Y + nu Phi,
// nu = u ||Y||_F (Nystrom-variants appendix) and the same again; then T =
// R_Y C^-1, its SVD, S = Q U(:, 1:k) with the sign convention, and the LMP
// coefficients of the theta rule.  Every reduction has a fixed order, so one
// problem gives the same bits in any launch.  The n x l products stage
// through LDS; the l x l factors live in the problem's small slots.

constexpr int GR = 32;  // rows of a Gram-product chunk

// G = A^T B (l x l, global), A, B n x l (ld n); entry (i, j) sums rows 0..n-1
// in order.  X: 2 (GR + 1) l doubles of LDS.
__device__ void wg_gram(int n, int l, const double *A, const double *B, double *G, double *X) {
    constexpr int NE = 16;  // entries per thread: l^2 <= NE * SC
    const int tid = threadIdx.x;
    double acc[NE];
#pragma unroll
    for (int t = 0; t < NE; t++) acc[t] = 0.0;
    double *Ac = X, *Bc = X + (GR + 1) * l;
    for (int r0 = 0; r0 < n; r0 += GR) {
        const int rows = n - r0 < GR ? n - r0 : GR;
        for (int idx = tid; idx < rows * l; idx += SC) {
            const int c = idx / rows, rr = idx - c * rows;
            Ac[c * (GR + 1) + rr] = A[(size_t)c * n + r0 + rr];
            Bc[c * (GR + 1) + rr] = B[(size_t)c * n + r0 + rr];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NE; t++) {
            const int e = tid + t * SC;
            if (e < l * l) {
                const double *a = Ac + (e % l) * (GR + 1), *b = Bc + (e / l) * (GR + 1);
                double v = acc[t];
                for (int rr = 0; rr < rows; rr++) v += a[rr] * b[rr];
                acc[t] = v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < NE; t++) {
        const int e = tid + t * SC;
        if (e < l * l) G[e] = acc[t];
    }
    __syncthreads();
}

// out (n x nc, ld n) = A (n x l, ld n) M(:, 0:nc) with M l x l (global); one
// thread per row, eight columns at a time, k ascending.  X: l nc doubles.
__device__ void wg_rmul(int n, int l, int nc, const double *A, const double *M, double *out, double *X) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < l * nc; idx += SC) X[idx] = M[idx];
    __syncthreads();
    for (int r = tid; r < n; r += SC) {
        for (int j0 = 0; j0 < nc; j0 += 8) {
            double acc[8];
#pragma unroll
            for (int jj = 0; jj < 8; jj++) acc[jj] = 0.0;
            for (int k = 0; k < l; k++) {
                const double a = A[(size_t)k * n + r];
#pragma unroll
                for (int jj = 0; jj < 8; jj++) {
                    const int j = j0 + jj < nc ? j0 + jj : nc - 1;
                    acc[jj] += a * X[k + j * l];
                }
            }
#pragma unroll
            for (int jj = 0; jj < 8; jj++)
                if (j0 + jj < nc) out[(size_t)(j0 + jj) * n + r] = acc[jj];
        }
    }
    __syncthreads();
}

// C = A B, l x l (global), k ascending as k_small_gemm.
__device__ void wg_small_mul(int l, const double *A, const double *B, double *C) {
    for (int idx = threadIdx.x; idx < l * l; idx += SC) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int k = 0; k < l; k++) v += A[i + k * l] * B[k + j * l];
        C[idx] = v;
    }
    __syncthreads();
}

__device__ void wg_copy(int count, const double *src, double *dst) {
    for (int idx = threadIdx.x; idx < count; idx += SC) dst[idx] = src[idx];
    __syncthreads();
}

// The sign convention of k_fix_signs: per column the entry of largest
// magnitude (lowest index on ties) is made positive; one wave per column.
__device__ void wg_fix_signs(int n, int k, double *S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < k; j += SC / 64) {
        double *col = S + (size_t)j * n;
        double best = -1.0;
        int bi = 0;
        for (int i = lane; i < n; i += 64) {
            const double a = fabs(col[i]);
            if (a > best) {
                best = a;
                bi = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        const bool neg = col[bi] < 0.0;
        if (neg)
            for (int i = lane; i < n; i += 64) col[i] = -col[i];
    }
    __syncthreads();
}

// Sum of squares of the n l entries of Y, fixed-order tree over the threads.
__device__ double wg_sumsq(size_t count, const double *Y, double *X) {
    const int tid = threadIdx.x;
    double v = 0.0;
    for (size_t idx = tid; idx < count; idx += SC) v += Y[idx] * Y[idx];
    X[tid] = v;
    __syncthreads();
    for (int w = SC / 2; w > 0; w >>= 1) {
        if (tid < w) X[tid] += X[tid + w];
        __syncthreads();
    }
    const double r = X[0];
    __syncthreads();
    return r;
}

// Cholesky of W (+ shift I) into C, C^-1; returns the failure flag to every thread.
__device__ int wg_chol(int l, const double *W, double shift, double *C, double *Ci, int32_t *info, double *X,
                       int &fail) {
    chol_inv(l, W, shift, C, Ci, info, X, fail);
    __syncthreads();
    const int f = fail;
    __syncthreads();
    return f;
}

// CholQR of Y into Q and R_Y (slot 7), shifted first pass when needed; 0 or
// a failed Cholesky (nonzero).
__device__ int wg_cholqr(const RedoJob &J, double *X, int &fail, double *red) {
    const int n = J.n, l = J.l;
    double *G = J.small, *R1 = J.small + 1 * J.ls, *R1i = J.small + 2 * J.ls;
    double *R2 = J.small + 3 * J.ls, *R2i = J.small + 4 * J.ls, *Racc = J.small + 5 * J.ls;
    double *Rtmp = J.small + 6 * J.ls, *RY = J.small + 7 * J.ls;
    int32_t *info = J.state + 2;
    wg_gram(n, l, J.y, J.y, G, X);
    int passes = 2;
    if (wg_chol(l, G, 0.0, R1, R1i, info, X, fail)) {
        // shift 11 (n l + l (l + 1)) eps trace(G) (shifted CholQR3)
        if (threadIdx.x == 0) {
            double tr = 0.0;
            for (int i = 0; i < l; i++) tr += G[(size_t)i * l + i];
            red[0] = 11.0 * ((double)n * l + (double)l * (l + 1)) * 2.220446049250313e-16 * tr;
        }
        __syncthreads();
        const double shift = red[0];
        __syncthreads();
        if (wg_chol(l, G, shift, R1, R1i, info, X, fail)) return 1;
        passes = 3;
    }
    wg_rmul(n, l, l, J.y, R1i, J.q1, X);
    wg_copy(l * l, R1, Racc);
    const double *Qin = J.q1;
    for (int pass = 2; pass <= passes; pass++) {
        double *Qout = pass == passes ? J.q : (Qin == J.q1 ? J.q2 : J.q1);
        wg_gram(n, l, Qin, Qin, G, X);
        if (wg_chol(l, G, 0.0, R2, R2i, info, X, fail)) return 1;
        wg_rmul(n, l, l, Qin, R2i, Qout, X);
        wg_small_mul(l, R2, Racc, Rtmp);
        wg_copy(l * l, Rtmp, Racc);
        Qin = Qout;
    }
    wg_copy(l * l, Racc, RY);
    return 0;
}

// W = Phi^T Y symmetrised (slot 8), Cholesky into C (slot 9), C^-1 (slot 1).
__device__ int wg_cholw(const RedoJob &J, double *X, int &fail) {
    const int l = J.l;
    double *Wm = J.small + 8 * J.ls, *Cm = J.small + 9 * J.ls, *Ci = J.small + 1 * J.ls;
    wg_gram(J.n, l, J.phi, J.y, Wm, X);
    for (int idx = threadIdx.x; idx < l * l; idx += SC) {
        const int i = idx % l, j = idx / l;
        if (i < j) {
            const double v = 0.5 * (Wm[i + j * l] + Wm[j + i * l]);
            Wm[i + j * l] = v;
            Wm[j + i * l] = v;
        }
    }
    __syncthreads();
    return wg_chol(l, Wm, 0.0, Cm, Ci, J.state + 2, X, fail);
}

__device__ void nystrom_redo(const RedoJob &J, double *X, int &fail, int &rotated, double *nrm, double *red) {
    const int tid = threadIdx.x, n = J.n, l = J.l, k = J.k;
    if (J.trigger && (J.trigger[0] | J.trigger[1] | J.trigger[2]) == 0) {
        if (tid == 0) {
            J.state[0] = 0;
            J.state[1] = 0;
        }
        return;
    }
    double nu = 0.0;
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; attempt++) {
        if (attempt == 1) {
            nu = J.u * sqrt(wg_sumsq((size_t)n * l, J.y, X));
            for (size_t idx = tid; idx < (size_t)n * l; idx += SC) J.y[idx] += nu * J.phi[idx];
            __syncthreads();
        }
        if (wg_cholqr(J, X, fail, red)) break;
        ok = wg_cholw(J, X, fail) == 0;
    }
    if (!ok) {
        if (tid == 0) {
            J.state[0] = 1;
            J.state[1] = 1;
        }
        return;
    }
    double *Ci = J.small + 1 * J.ls, *Tm = J.small + 2 * J.ls, *Um = J.small + 3 * J.ls;
    double *sig = J.small + 4 * J.ls, *RY = J.small + 7 * J.ls;
    wg_small_mul(l, RY, Ci, Tm);
    jacobi_svd(l, Tm, Um, sig, X, rotated, nrm);
    __syncthreads();
    wg_rmul(n, l, k, J.q, Um, J.s, X);
    wg_fix_signs(n, k, J.s);
    // d_i = max(sigma_i^2 - nu, 0) and the coefficients of k_lmp_coef
    if (tid == 0) {
        const double s = sig[k - 1];
        const double lk = 1.0 + fmax(s * s - nu, 0.0);
        red[0] = J.rule == EDA_THETA_MID ? 0.5 * (lk + 1.0) : (J.rule == EDA_THETA_LAMK ? lk : 1.0);
        *J.theta = red[0];
    }
    __syncthreads();
    const double th = red[0];
    for (int i = tid; i < k; i += SC) {
        const double s = sig[i];
        const double d = fmax(s * s - nu, 0.0);
        J.eig[i] = d;
        J.coef[i] = th / (1.0 + d) - 1.0;
        J.coefu[i] = sqrt(th) / sqrt(1.0 + d) - 1.0;
    }
    if (tid == 0) {
        J.state[0] = 1;
        J.state[1] = 0;
    }
}

__global__ __launch_bounds__(SC) void k_nystrom_redo(RedoJob J) {
    extern __shared__ double X[];
    __shared__ int fail, rotated;
    __shared__ double nrm[128], red[1];
    nystrom_redo(J, X, fail, rotated, nrm, red);
}

__global__ __launch_bounds__(SC) void k_nystrom_redo_batch(const RedoJob *__restrict__ jobs) {
    extern __shared__ double X[];
    __shared__ int fail, rotated;
    __shared__ double nrm[128], red[1];
    const RedoJob J = jobs[blockIdx.x];
    nystrom_redo(J, X, fail, rotated, nrm, red);
}

// LDS doubles of the redo for l <= lmax: the Cholesky's 2 l^2 (l <= 64) or
// l^2, the Gram chunks, the row-product factor and the reduction tree.
size_t redo_lds(int lmax) {
    size_t need = lmax <= 64 ? 2 * (size_t)lmax * lmax
                             : ((size_t)lmax * lmax > 2 * 64 * 64 ? (size_t)lmax * lmax : 2 * 64 * 64);
    const size_t gram = 2 * (size_t)(GR + 1) * lmax;
    if (gram > need) need = gram;
    if ((size_t)SC > need) need = SC;
    return sizeof(double) * need;
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

hipError_t launch_chol_inv_batch(hipStream_t s, int njobs, const CholJob *d_jobs, int lmax) {
    if (njobs <= 0) return hipSuccess;
    if (lmax < 1 || lmax > 128) return hipErrorInvalidValue;
    // every job fits: a job needs 2 l^2 doubles up to l = 64 and l^2 above
    const int need = lmax <= 64 ? 2 * lmax * lmax : (lmax * lmax > 2 * 64 * 64 ? lmax * lmax : 2 * 64 * 64);
    const size_t lds = sizeof(double) * need;
    hipLaunchKernelGGL(k_chol_inv_batch, dim3(njobs), dim3(SC), lds, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_nystrom_redo(hipStream_t s, const RedoJob &job) {
    if (job.l < 1 || job.l > 128 || job.k < 1 || job.k > job.l || job.n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nystrom_redo, dim3(1), dim3(SC), redo_lds(job.l), s, job);
    return hipGetLastError();
}

hipError_t launch_nystrom_redo_batch(hipStream_t s, int njobs, const RedoJob *d_jobs, int lmax) {
    if (njobs <= 0) return hipSuccess;
    if (lmax < 1 || lmax > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nystrom_redo_batch, dim3(njobs), dim3(SC), redo_lds(lmax), s, d_jobs);
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

hipError_t launch_jacobi_svd_batch(hipStream_t s, int njobs, const JacobiJob *d_jobs, int lmax) {
    if (njobs <= 0) return hipSuccess;
    if (lmax < 1 || lmax > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_svd_batch, dim3(njobs), dim3(SJ), sizeof(double) * lmax * lmax, s, d_jobs);
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

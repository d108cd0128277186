// Workgroup-level small linear algebra of the Nystrom core, shared by the
// small-matrix kernels (small_la.hip) and the batch's persistent sketch
// launch (l96_tlad.hip): ell x ell Cholesky with the inverse of its factor, the
// one-sided Jacobi SVD, and the whole last pass of the Nystrom algorithm with
// its shifts (nystrom_redo).  Every function runs on the calling workgroup,
// whatever its size (blockDim.x a multiple of 64, at least 64 threads), and
// assigns work so that each result's arithmetic and summation order do not
// depend on that size: a workgroup of 256 threads gives the bits of one of
// 1024.  ell <= 128.  Every thread of the workgroup must call them.
#pragma once

#include "eda_internal.h"

namespace eda {
namespace nys {

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
// finished columns, X_ij = -X_jj sum_{k=i}^{j-1} X_ik C_kj, in place (rows i
// and i + blockDim.x of each thread).  S: LDS, l x l doubles (2 l x l when
// l <= 64); fail: an LDS flag.  No barrier after the last writes.
__device__ __forceinline__ void chol_inv(int l, const double *__restrict__ W, double shift, double *__restrict__ C,
                                         double *__restrict__ Cinv, int32_t *__restrict__ info, double *S,
                                         int &fail) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int idx = tid; idx < l * l; idx += nthr) {
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
        for (int c = j + 1 + tid; c < l; c += nthr) S[j + c * l] /= piv;
        __syncthreads();
        const int m = l - 1 - j;  // trailing block rows/columns j+1 .. l-1
        for (int idx = tid; idx < m * m; idx += nthr) {
            const int r = j + 1 + idx % m, c = j + 1 + idx / m;
            if (r <= c) S[r + c * l] -= S[j + r * l] * S[j + c * l];
        }
        __syncthreads();
    }
    if (tid == 0) *info = fail;
    if (fail) return;
    for (int idx = tid; idx < l * l; idx += nthr) {
        int i = idx % l, j = idx / l;
        C[idx] = (i <= j) ? S[idx] : 0.0;
    }
    if (l <= 64) {
        double *X = S + l * l;
        for (int idx = tid; idx < l * l; idx += nthr) X[idx] = (idx % l == idx / l) ? 1.0 : 0.0;
        __syncthreads();
        for (int i = l - 1; i >= 0; i--) {
            const double cii = S[i + i * l];
            for (int c = i + tid; c < l; c += nthr) X[i + c * l] /= cii;
            __syncthreads();
            const int w = l - i;  // columns i .. l-1 of rows 0 .. i-1
            for (int idx = tid; idx < i * w; idx += nthr) {
                const int r = idx % i, c = i + idx / i;
                X[r + c * l] -= S[r + i * l] * X[i + c * l];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < l * l; idx += nthr) {
            int i = idx % l, j = idx / l;
            Cinv[idx] = (i <= j) ? X[idx] : 0.0;
        }
        return;
    }
    for (int j = 0; j < l; j++) {
        const double xjj = 1.0 / S[j + j * l];
        double v[2] = {0.0, 0.0};
        for (int h = 0; h < 2; h++) {
            const int i = tid + h * nthr;
            if (i < j)
                for (int k = i; k < j; k++) v[h] += S[i + k * l] * S[k + j * l];
        }
        __syncthreads();
        for (int h = 0; h < 2; h++) {
            const int i = tid + h * nthr;
            if (i < j) S[i + j * l] = -xjj * v[h];
            if (i == j) S[j + j * l] = xjj;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < l * l; idx += nthr) {
        int i = idx % l, j = idx / l;
        Cinv[idx] = (i <= j) ? S[idx] : 0.0;
    }
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
// with ranks sorting sigma descending (ties: lower index first).  A pair is
// always handled by one 16-lane row, its sums over lanes i mod 16.
// A: l x l doubles of LDS; rotated, nrm: LDS flag and norms (128).  No barrier
// after the last writes.
__device__ __forceinline__ void jacobi_svd(int l, const double *__restrict__ T, double *__restrict__ U,
                                           double *__restrict__ sig, double *A, int &rotated, double *nrm) {
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    for (int idx = tid; idx < l * l; idx += nthr) A[idx] = T[idx];
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
            for (int k = tid >> 4; k < m / 2; k += nthr / 16) {
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
    for (int j = wave; j < l; j += nthr / 64) {
        double v = 0;
        for (int i = lane; i < l; i += 64) v += A[i + j * l] * A[i + j * l];
        v = wave_sum(v);
        if (lane == 0) nrm[j] = sqrt(v);
    }
    __syncthreads();
    for (int j = tid; j < l; j += nthr) {
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

// ---------------------------------------------------------------------------
// The last pass of the Nystrom sketch with its shifts, on one workgroup: from
// Y = A Phi and Phi -- CholQR2 of Y, a shifted first pass (shifted CholQR3)
// when the Gram matrix's Cholesky fails; W = Phi^T Y and its Cholesky; when
// that fails the Nystrom shift Y <- Y + nu Phi, nu = u ||Y||_F
// (Nystrom-variants appendix) and the same again; then T = R_Y C^-1, its SVD,
// S = Q U(:, 1:k) with the sign convention, and the LMP coefficients of the
// theta rule.  Every reduction has a fixed order.  The n x l products stage
// through LDS; the l x l factors live in the problem's small slots.

constexpr int GR = 32;   // rows of a Gram-product chunk
constexpr int NV = 1024; // partial sums of wg_sumsq (fixed, whatever the workgroup size)

// LDS doubles the pass needs for l <= lmax: the Cholesky's 2 l^2 (l <= 64)
// or l^2, the Gram chunks, the row-product factor and the reduction slots.
__host__ __device__ inline size_t redo_lds_doubles(int lmax) {
    size_t need = lmax <= 64 ? 2 * (size_t)lmax * lmax
                             : ((size_t)lmax * lmax > 2 * 64 * 64 ? (size_t)lmax * lmax : 2 * 64 * 64);
    const size_t gram = 2 * (size_t)(GR + 1) * lmax;
    if (gram > need) need = gram;
    if ((size_t)NV > need) need = NV;
    return need;
}

// G = A^T B (l x l, global), A, B n x l (ld n); entry (i, j) sums rows 0..n-1
// in order.  X: 2 (GR + 1) l doubles of LDS.
__device__ inline void wg_gram(int n, int l, const double *A, const double *B, double *G, double *X) {
    constexpr int NE = 16;  // entries per thread and pass over the rows
    const int tid = threadIdx.x, nthr = blockDim.x;
    double *Ac = X, *Bc = X + (GR + 1) * l;
    for (int e0 = 0; e0 < l * l; e0 += NE * nthr) {
        double acc[NE];
#pragma unroll
        for (int t = 0; t < NE; t++) acc[t] = 0.0;
        for (int r0 = 0; r0 < n; r0 += GR) {
            const int rows = n - r0 < GR ? n - r0 : GR;
            for (int idx = tid; idx < rows * l; idx += nthr) {
                const int c = idx / rows, rr = idx - c * rows;
                Ac[c * (GR + 1) + rr] = A[(size_t)c * n + r0 + rr];
                Bc[c * (GR + 1) + rr] = B[(size_t)c * n + r0 + rr];
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < NE; t++) {
                const int e = e0 + tid + t * nthr;
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
            const int e = e0 + tid + t * nthr;
            if (e < l * l) G[e] = acc[t];
        }
    }
    __syncthreads();
}

// out (n x nc, ld n) = A (n x l, ld n) M(:, 0:nc) with M l x l (global); one
// thread per row, eight columns at a time, k ascending.  X: l nc doubles.
__device__ inline void wg_rmul(int n, int l, int nc, const double *A, const double *M, double *out, double *X) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int idx = tid; idx < l * nc; idx += nthr) X[idx] = M[idx];
    __syncthreads();
    for (int r = tid; r < n; r += nthr) {
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
__device__ inline void wg_small_mul(int l, const double *A, const double *B, double *C) {
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int k = 0; k < l; k++) v += A[i + k * l] * B[k + j * l];
        C[idx] = v;
    }
    __syncthreads();
}

__device__ inline void wg_copy(int count, const double *src, double *dst) {
    for (int idx = threadIdx.x; idx < count; idx += blockDim.x) dst[idx] = src[idx];
    __syncthreads();
}

// The sign convention of k_fix_signs: per column the entry of largest
// magnitude (lowest index on ties) is made positive; one wave per column.
__device__ inline void wg_fix_signs(int n, int k, double *S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < k; j += blockDim.x / 64) {
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

// Sum of squares of the count entries of Y: NV partial sums (entries v, v +
// NV, ...) and a fixed tree over them.  X: NV doubles.
__device__ inline double wg_sumsq(size_t count, const double *Y, double *X) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int v = tid; v < NV; v += nthr) {
        double s = 0.0;
        for (size_t idx = v; idx < count; idx += NV) s += Y[idx] * Y[idx];
        X[v] = s;
    }
    __syncthreads();
    for (int w = NV / 2; w > 0; w >>= 1) {
        for (int v = tid; v < w; v += nthr) X[v] += X[v + w];
        __syncthreads();
    }
    const double r = X[0];
    __syncthreads();
    return r;
}

// Cholesky of W (+ shift I) into C, C^-1; returns the failure flag to every thread.
__device__ inline int wg_chol(int l, const double *W, double shift, double *C, double *Ci, int32_t *info,
                              double *X, int &fail) {
    chol_inv(l, W, shift, C, Ci, info, X, fail);
    __syncthreads();
    const int f = fail;
    __syncthreads();
    return f;
}

// Per-pass scratch of nystrom_redo in LDS beside the big buffer.
struct RedoLds {
    int fail, rotated;
    double red;
};

// CholQR of Y into Q and R_Y (slot 7), shifted first pass when needed (sets
// shifts bit 0); 0 or a failed Cholesky (nonzero).
__device__ inline int wg_cholqr(const RedoJob &J, double *X, RedoLds &L, int &shifts) {
    const int n = J.n, l = J.l;
    double *G = J.small, *R1 = J.small + 1 * J.ls, *R1i = J.small + 2 * J.ls;
    double *R2 = J.small + 3 * J.ls, *R2i = J.small + 4 * J.ls, *Racc = J.small + 5 * J.ls;
    double *Rtmp = J.small + 6 * J.ls, *RY = J.small + 7 * J.ls;
    int32_t *info = J.state + 3;
    wg_gram(n, l, J.y, J.y, G, X);
    int passes = 2;
    if (wg_chol(l, G, 0.0, R1, R1i, info, X, L.fail)) {
        // shift 11 (n l + l (l + 1)) eps trace(G) (shifted CholQR3)
        if (threadIdx.x == 0) {
            double tr = 0.0;
            for (int i = 0; i < l; i++) tr += G[(size_t)i * l + i];
            L.red = 11.0 * ((double)n * l + (double)l * (l + 1)) * 2.220446049250313e-16 * tr;
        }
        __syncthreads();
        const double shift = L.red;
        __syncthreads();
        shifts |= 1;
        if (wg_chol(l, G, shift, R1, R1i, info, X, L.fail)) return 1;
        passes = 3;
    }
    wg_rmul(n, l, l, J.y, R1i, J.q1, X);
    wg_copy(l * l, R1, Racc);
    const double *Qin = J.q1;
    for (int pass = 2; pass <= passes; pass++) {
        double *Qout = pass == passes ? J.q : (Qin == J.q1 ? J.q2 : J.q1);
        wg_gram(n, l, Qin, Qin, G, X);
        if (wg_chol(l, G, 0.0, R2, R2i, info, X, L.fail)) return 1;
        wg_rmul(n, l, l, Qin, R2i, Qout, X);
        wg_small_mul(l, R2, Racc, Rtmp);
        wg_copy(l * l, Rtmp, Racc);
        Qin = Qout;
    }
    wg_copy(l * l, Racc, RY);
    return 0;
}

// W = Phi^T Y symmetrised (slot 8), Cholesky into C (slot 9), C^-1 (slot 1).
__device__ inline int wg_cholw(const RedoJob &J, double *X, RedoLds &L) {
    const int l = J.l;
    double *Wm = J.small + 8 * J.ls, *Cm = J.small + 9 * J.ls, *Ci = J.small + 1 * J.ls;
    wg_gram(J.n, l, J.phi, J.y, Wm, X);
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int i = idx % l, j = idx / l;
        if (i < j) {
            const double v = 0.5 * (Wm[i + j * l] + Wm[j + i * l]);
            Wm[i + j * l] = v;
            Wm[j + i * l] = v;
        }
    }
    __syncthreads();
    return wg_chol(l, Wm, 0.0, Cm, Ci, J.state + 3, X, L.fail);
}

// The pass for job J (see RedoJob).  X: redo_lds_doubles(J.l) doubles of LDS;
// nrm: 128 doubles of LDS.
__device__ inline void nystrom_redo(const RedoJob &J, double *X, RedoLds &L, double *nrm) {
    const int tid = threadIdx.x, n = J.n, l = J.l, k = J.k;
    if (J.trigger && (J.trigger[0] | J.trigger[1] | J.trigger[2]) == 0) {
        if (tid == 0) {
            J.state[0] = 0;
            J.state[1] = 0;
            J.state[2] = 0;
        }
        return;
    }
    double nu = 0.0;
    bool ok = false;
    int shifts = 0;
    for (int attempt = 0; attempt < 2 && !ok; attempt++) {
        if (attempt == 1) {
            nu = J.u * sqrt(wg_sumsq((size_t)n * l, J.y, X));
            for (size_t idx = tid; idx < (size_t)n * l; idx += blockDim.x) J.y[idx] += nu * J.phi[idx];
            __syncthreads();
            shifts |= 2;
        }
        if (wg_cholqr(J, X, L, shifts)) break;
        ok = wg_cholw(J, X, L) == 0;
    }
    if (!ok) {
        if (tid == 0) {
            J.state[0] = 1;
            J.state[1] = 1;
            J.state[2] = shifts;
        }
        return;
    }
    double *Ci = J.small + 1 * J.ls, *Tm = J.small + 2 * J.ls, *Um = J.small + 3 * J.ls;
    double *sig = J.small + 4 * J.ls, *RY = J.small + 7 * J.ls;
    wg_small_mul(l, RY, Ci, Tm);
    jacobi_svd(l, Tm, Um, sig, X, L.rotated, nrm);
    __syncthreads();
    wg_rmul(n, l, k, J.q, Um, J.s, X);
    wg_fix_signs(n, k, J.s);
    // d_i = max(sigma_i^2 - nu, 0) and the coefficients of k_lmp_coef
    if (tid == 0) {
        const double s = sig[k - 1];
        const double lk = 1.0 + fmax(s * s - nu, 0.0);
        L.red = J.rule == EDA_THETA_MID ? 0.5 * (lk + 1.0) : (J.rule == EDA_THETA_LAMK ? lk : 1.0);
        *J.theta = L.red;
    }
    __syncthreads();
    const double th = L.red;
    for (int i = tid; i < k; i += blockDim.x) {
        const double s = sig[i];
        const double d = fmax(s * s - nu, 0.0);
        J.eig[i] = d;
        J.coef[i] = th / (1.0 + d) - 1.0;
        J.coefu[i] = sqrt(th) / sqrt(1.0 + d) - 1.0;
    }
    if (tid == 0) {
        J.state[0] = 1;
        J.state[1] = 0;
        J.state[2] = shifts;
    }
    __syncthreads();
}

}  // namespace nys
}  // namespace eda

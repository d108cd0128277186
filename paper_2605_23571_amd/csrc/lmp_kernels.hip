// The spectral limited-memory preconditioner applied to a block of vectors
// (the LMP subsection of the preconditioning section):
//
//   Y = X + S diag(coef) S^T X,   S: n x k orthonormal Ritz vectors (column-major),
//                                 X, Y: n x nb (column-major, leading dims ldx, ldy).
//
// Two launches on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//  * k_lmp_proj   -- workgroup (row block, tile of 16 columns): the partial
//    projection S_b^T X_b of its rows onto every direction;
//  * k_lmp_expand -- workgroup (128 rows, 16 columns): W = diag(coef) S^T X for
//    its columns (the row blocks summed in block order, into LDS), then
//    Y = X + S W.
// Sums are taken in a fixed order, so results do not depend on scheduling; the
// kernel boundary orders the two steps.  A column tile whose members have all
// left the running state (status given) is skipped -- inside the PCG loop
// converged members need no preconditioned residual.
//
// Operand layouts: in v_mfma_f64_16x16x4f64 lane l (g = l / 16, m = l % 16)
// supplies A[m][g] and B[g][m]; element v of the accumulator is D[g + 4 v][m].
// Every global operand is read so that the 16 lanes of a quarter-wave touch
// consecutive addresses where it matters: S^T X takes S from a row-major copy
// Sr (direction index contiguous; X is read in 32-byte runs per lane); S W
// takes S column-major (row index contiguous) and W from LDS.  Both kernels are
// bound by memory latency rather than bandwidth, so each issues all of its
// global loads before it waits.
#include "eda_internal.h"

namespace eda {
namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int CT = 16;         // columns per tile

__device__ __forceinline__ bool tile_running(const int32_t *status, int c0, int nb) {
    if (!status) return true;
    bool any = false;
    for (int c = c0; c < c0 + CT && c < nb; c++) any |= status[c] == COL_RUNNING;
    return any;
}

// Sr[i k + j] = S[j n + i]
__global__ void k_lmp_rowmajor(int n, int k, const double *__restrict__ S, double *__restrict__ Sr) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * k) return;
    const int i = (int)(e / k), j = (int)(e % k);
    Sr[e] = S[(long long)j * n + i];
}

// Partial projections part[rb][j][col] = sum_{i in block rb} S[i][j] X[i][col].
// Wave w takes 4 slabs of 16 rows; step t of a slab runs on the rows
// i = i0 + 4 g + t (A[m][g] = Sr[i][j0 + m], B[g][m] = X[i][c0 + m]).  All of a
// wave's loads -- the tile's status included -- are issued before the first
// MFMA, so the kernel waits on one round trip to memory.  The four waves'
// accumulators are summed in wave order through LDS.
__global__ __launch_bounds__(256) void k_lmp_proj(int n, int k, int nb, int rows, const double *__restrict__ Sr,
                                                  const double *__restrict__ X, long long ldx,
                                                  const int32_t *__restrict__ status, double *__restrict__ part,
                                                  int ldw) {
    __shared__ double red[4][4][4][64];  // [wave][j tile in group][v][lane]
    const int rb = blockIdx.x, c0 = blockIdx.y * CT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, m = lane & 15;
    const int r0 = rb * rows, r1 = min(n, r0 + rows);
    const int wrows = rows / 4;  // a multiple of 64
    const int w0 = r0 + wave * wrows, w1 = min(r1, w0 + wrows);
    const int col = c0 + m;
    const bool colok = col < nb;
    const double *xc = X + (long long)(colok ? col : 0) * ldx;
    const int njt = (k + 15) / 16;
    bool run = true;

    for (int jg = 0; jg < njt; jg += 4) {
        double4v acc[4];
#pragma unroll
        for (int q = 0; q < 4; q++) acc[q] = double4v{0.0, 0.0, 0.0, 0.0};
        for (int i0 = w0; i0 < w1; i0 += 64) {
            double b[4][4], a[4][4][4];  // [slab][t], [slab][j tile][t]
#pragma unroll
            for (int sl = 0; sl < 4; sl++) {
                const int ib = i0 + 16 * sl + 4 * g;
#pragma unroll
                for (int t = 0; t < 4; t++) b[sl][t] = (colok && ib + t < w1) ? xc[ib + t] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int j = (jg + q) * 16 + m;
                    const bool jok = j < k;
#pragma unroll
                    for (int t = 0; t < 4; t++)
                        a[sl][q][t] = (jok && ib + t < w1) ? Sr[(long long)(ib + t) * k + j] : 0.0;
                }
            }
            if (jg == 0 && i0 == w0) run = tile_running(status, c0, nb);
#pragma unroll
            for (int sl = 0; sl < 4; sl++)
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int t = 0; t < 4; t++)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl][q][t], b[sl][t], acc[q], 0, 0, 0);
        }
        // D[j][col] of tile q: lane l, element v -> j = (jg + q) 16 + l / 16 + 4 v, col = c0 + l % 16
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int v = 0; v < 4; v++) red[wave][q][v][lane] = acc[q][v];
        __syncthreads();
        if (w0 >= w1 && jg == 0) run = tile_running(status, c0, nb);  // waves without rows
        for (int e = tid; e < 4 * 4 * 64; e += 256) {
            const int q = e >> 8, v = (e >> 6) & 3, l = e & 63;
            const int j = (jg + q) * 16 + (l >> 4) + 4 * v;
            if (run && j < k) {
                const double s = ((red[0][q][v][l] + red[1][q][v][l]) + red[2][q][v][l]) + red[3][q][v][l];
                part[((long long)rb * k + j) * ldw + c0 + (l & 15)] = s;
            }
        }
        __syncthreads();
    }
}

// Y = X + S W on 128 rows x 16 columns.  Each thread loads, in one batch, its
// share of the row-block partials of W (4 entries), this lane's S operands
// and X entries; the workgroup then forms W[j][c] = coef[j] sum_b part[b][j][c]
// (block order) in LDS, and wave w computes rows 32 w .. 32 w + 31 as two MFMA
// blocks on (W^T, S^T): A[m][g] = W[j][c0 + m], B[g][m] = S[i + m][j],
// j = j0 + g, so accumulator lanes run along rows (element v: row i + m,
// column c0 + g + 4 v).
template <int KM>
__global__ __launch_bounds__(256) void k_lmp_expand(int n, int k, int nb, int nrb, const double *__restrict__ S,
                                                    const double *__restrict__ coef, const double *X, long long ldx,
                                                    double *Y, long long ldy, const int32_t *__restrict__ status,
                                                    const double *__restrict__ part, int ldw) {
    __shared__ double ws[KM][CT];
    const int c0 = blockIdx.y * CT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, m = lane & 15;
    const int ib = blockIdx.x * 128 + wave * 32;
    // partials of KM CT / 256 W entries per thread (k <= KM)
    double pv[KM * CT / 256][LMP_RB_MAX];
#pragma unroll
    for (int u = 0; u < KM * CT / 256; u++) {
        const int e = tid + 256 * u;
        const bool ok = e < k * CT;
        const double *pe = part + (long long)(ok ? e / CT : 0) * ldw + c0 + e % CT;
#pragma unroll
        for (int b = 0; b < LMP_RB_MAX; b++) pv[u][b] = (ok && b < nrb) ? pe[(long long)b * k * ldw] : 0.0;
    }
    double xv[2][4];  // [row tile][v]
#pragma unroll
    for (int rt = 0; rt < 2; rt++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = ib + 16 * rt + m, col = c0 + g + 4 * v;
            xv[rt][v] = (i < n && col < nb) ? X[(long long)col * ldx + i] : 0.0;
        }
    double4v acc[2] = {double4v{0.0, 0.0, 0.0, 0.0}, double4v{0.0, 0.0, 0.0, 0.0}};
    const bool run = tile_running(status, c0, nb);
    for (int j0 = 0; j0 < k; j0 += 64) {
        double b[2][16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int j = j0 + 4 * u + g;
#pragma unroll
            for (int rt = 0; rt < 2; rt++) {
                const int i = ib + 16 * rt + m;
                b[rt][u] = (j < k && i < n) ? S[(long long)j * n + i] : 0.0;
            }
        }
        if (j0 == 0) {
#pragma unroll
            for (int u = 0; u < KM * CT / 256; u++) {
                const int e = tid + 256 * u;
                if (e < k * CT) {
                    double s = 0.0;
#pragma unroll
                    for (int bb = 0; bb < LMP_RB_MAX; bb++) s += pv[u][bb];  // block order; absent blocks add 0
                    ws[e / CT][e % CT] = coef[e / CT] * s;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int j = j0 + 4 * u + g;
            const double a = j < k ? ws[j][m] : 0.0;
#pragma unroll
            for (int rt = 0; rt < 2; rt++) acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[rt][u], acc[rt], 0, 0, 0);
        }
    }
    if (!run) return;
#pragma unroll
    for (int rt = 0; rt < 2; rt++) {
        const int i = ib + 16 * rt + m;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int col = c0 + g + 4 * v;
            if (col < nb) Y[(long long)col * ldy + i] = xv[rt][v] + acc[rt][v];
        }
    }
}

}  // namespace

// Row blocks of the projection: at most LMP_RB_MAX, each a multiple of
// 256 rows (64 for each of the four waves).
void lmp_blocks(int n, int *rows, int *nrb) {
    const int unit = 256;
    const int units = (n + unit - 1) / unit;
    int b = units < LMP_RB_MAX ? units : LMP_RB_MAX;
    if (b < 1) b = 1;
    const int per = (units + b - 1) / b;
    *rows = per * unit;
    *nrb = (n + *rows - 1) / *rows;
}

size_t lmp_work_doubles(int n, int k, int ncols) {
    int rows, nrb;
    lmp_blocks(n, &rows, &nrb);
    const size_t ldw = (size_t)(ncols + CT - 1) / CT * CT;
    return (size_t)nrb * k * ldw;
}

hipError_t launch_lmp_rowmajor(hipStream_t s, int n, int k, const double *S, double *Sr) {
    const long long tot = (long long)n * k;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lmp_rowmajor, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, k, S, Sr);
    return hipGetLastError();
}

hipError_t launch_lmp(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                      const double *X, long long ldx, double *Y, long long ldy, const int32_t *status,
                      double *work) {
    if (n <= 0 || nb <= 0) return hipSuccess;
    if (k <= 0 || k > LMP_K_MAX) return hipErrorInvalidValue;
    int rows, nrb;
    lmp_blocks(n, &rows, &nrb);
    const int tiles = (nb + CT - 1) / CT, ldw = tiles * CT;
    hipLaunchKernelGGL(k_lmp_proj, dim3(nrb, tiles), dim3(256), 0, s, n, k, nb, rows, Sr, X, ldx, status, work, ldw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (k <= 64)
        hipLaunchKernelGGL(k_lmp_expand<64>, dim3((n + 127) / 128, tiles), dim3(256), 0, s, n, k, nb, nrb, S, coef, X,
                           ldx, Y, ldy, status, work, ldw);
    else
        hipLaunchKernelGGL(k_lmp_expand<LMP_K_MAX>, dim3((n + 127) / 128, tiles), dim3(256), 0, s, n, k, nb, nrb, S,
                           coef, X, ldx, Y, ldy, status, work, ldw);
    return hipGetLastError();
}

}  // namespace eda

// The spectral limited-memory preconditioner applied to a block of vectors
// (the LMP subsection of the preconditioning section):
//
//   Y = X + S diag(coef) S^T X,   S: n x k orthonormal Ritz vectors (column-major),
//                                 X, Y: n x nb (column-major, leading dims ldx, ldy).
//
// Two steps on the FP64 matrix cores (v_mfma_f64_16x16x4f64), for a
// workgroup per (row block of 256 rows, tile of 16 columns):
//  * projection -- the partial projection S_b^T X_b of its rows onto every
//    direction;
//  * expansion -- W = diag(coef) S^T X for its columns (the row blocks summed
//    in block order, into LDS), then Y = X + S W on its rows.
// Either two launches (k_lmp_proj, k_lmp_expand: the kernel boundary orders
// the steps) or one (k_lmp_one): the workgroups of a tile meet at a tile
// barrier between the steps, which needs every workgroup of the launch
// resident at once (one per CU; the host checks the grid against the CU
// count).  Its waits are bounded: one that gives up sets an error word and
// the results of that call are void.  Both forms do the same arithmetic in
// the same order, so they give the same bits.  On MI355X the two launches are
// the faster form (n = 4096, 129 columns: 7.5 + 9.2 us against 20.9 us; with
// the update fused, 12.0 + 10.1 us against 29.2 us): the barrier's round trips
// through device memory cost more than the launch boundary they replace.  Sums are taken in a fixed
// order, so results do not depend on scheduling.  A column tile whose members
// have all left the running state (status given) is skipped -- inside the
// PCG loop converged members need no preconditioned residual.
//
// Operand layouts: in v_mfma_f64_16x16x4f64 lane l (g = l / 16, m = l % 16)
// supplies A[m][g] and B[g][m]; element v of the accumulator is D[g + 4 v][m].
// Every global operand is read so that the 16 lanes of a quarter-wave touch
// consecutive addresses where it matters: S^T X takes S from a row-major copy
// Sr (direction index contiguous; X is read in 32-byte runs per lane); S W
// takes S column-major (row index contiguous) and W from LDS.  Both kernels are
// bound by memory latency rather than bandwidth, so each issues all of its
// global loads before it waits.
#include <mutex>

#include "eda_internal.h"

// Fixed device buffer of the allocation-free LMP entry point: the row-block
// partial projections of one call, LMP_NOALLOC_DOUBLES doubles (4 MiB).  Each
// GPU the library runs on holds its own copy until the process ends.  In host
// code this name is not a device address: its address on a device comes from
// hipGetSymbolAddress (lmp_noalloc_scratch), and only that address is used.
static __device__ __align__(256) double scratch[eda::LMP_NOALLOC_DOUBLES];

namespace eda {
namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int CT = 16;         // columns per tile
constexpr int RB = 256;        // rows per projection block
constexpr int XP = RB + 1;     // odd row stride of the staged X: the 16 columns of one read fall in distinct banks

// the projection step's LDS: staged X (xs[column][row]) and the waves' partial sums
struct ProjLds {
    double xs[CT][XP];
    double red[8][4][4][64];  // [wave][j tile in group][v][lane]
};
template <int KM>
struct ExpandLds {
    double ws[KM][CT];
    double rzs[8][CT];
};

// Device-scope (coherent across XCDs) loads and stores of the values that
// the workgroups of a tile hand to each other in the single launch.
__device__ __forceinline__ double load_agent(const double *p) {
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void store_agent(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// plain store, or device-scope store when the value crosses workgroups within a launch
__device__ __forceinline__ void put(double *p, double v, bool shared) {
    if (shared)
        store_agent(p, v);
    else
        *p = v;
}

__device__ __forceinline__ bool tile_running(const int32_t *status, int c0, int nb) {
    if (!status) return true;
    bool any = false;
    for (int c = c0; c < c0 + CT && c < nb; c++) any |= status[c] == COL_RUNNING;
    return any;
}

// p^T (I + A) p of column col: the pieces' partial sums in piece order, all
// loaded before the sum (wave pieces: nseg[col] segments, eight loads at a time)
__device__ __forceinline__ double pieces_sum(const LmpFin &f, int col) {
    if (f.pieces > 0) {
        double v[SPLIT_PMAX];
#pragma unroll
        for (int i = 0; i < SPLIT_PMAX; i++) v[i] = i < f.pieces ? f.pq_part[(long long)col * f.pieces + i] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < SPLIT_PMAX; i++) s += v[i];
        return s;
    }
    const int ns = min(max(f.nseg[col], 0), XCH_SEG_MAX);
    const double *pp = f.pq_part + (long long)col * XCH_SEG_MAX;
    double s = 0.0;
    for (int i0 = 0; i0 < ns; i0 += 8) {
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = i0 + i < ns ? pp[i0 + i] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; i++) s += v[i];
    }
    return s;
}

// Sr[i k + j] = S[j n + i]
__global__ void k_lmp_rowmajor(int n, int k, const double *__restrict__ S, double *__restrict__ Sr) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * k) return;
    const int i = (int)(e / k), j = (int)(e % k);
    Sr[e] = S[(long long)j * n + i];
}

// Partial projections part[rb][j][col] = sum_{i in block rb} S[i][j] X[i][col]
// for a block of 256 rows and a tile of 16 columns, in two phases.
//  1. Coalesced pass: thread t takes column c0 + t / 32 and rows
//     r0 + t % 32 + 32 u (u < 8); it stages X there in LDS (xs[column][row]).
//     FIN (X = r of a split PCG iteration): it first updates the column's
//     entries, r -= alpha q and x += alpha p (alpha from the pieces' partial
//     sums; running columns only), stages the new r, and sums ||r||^2 and
//     x^T (b + r) over its rows; a 32-lane shuffle tree gives the column's sums
//     for the row block (f.rr_part, f.xbr_part).
//  2. Eight waves, each on 32 rows (two slabs of 16): step t of a slab runs on
//     the rows i = i0 + 4 g + t, A[m][g] = Sr[i][j0 + m] (16 consecutive
//     directions per quarter-wave), B[g][m] = xs[m][i]; the waves' accumulators
//     are summed in wave order through LDS.
// The first group's Sr operands are loaded before phase 1, so both phases wait
// on one round trip to memory.
// one: single launch (the partial sums go out as device-scope stores)
template <bool FIN>
__device__ __forceinline__ void lmp_proj(int rb, int tile, int n, int k, int nb, int rows,
                                         const double *__restrict__ Sr, double *X, long long ldx,
                                         const int32_t *__restrict__ status, double *__restrict__ part, int ldw,
                                         const LmpFin &f, ProjLds &L, bool one) {
    auto &xs = L.xs;
    auto &red = L.red;
    const int c0 = tile * CT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, m = lane & 15;
    const int r0 = rb * rows, r1 = min(n, r0 + rows);  // rows == RB
    const int w0 = r0 + wave * 32, w1 = min(r1, w0 + 32);
    const int njt = (k + 15) / 16;

    // Sr operands of the first direction group
    double a[2][4][4];  // [slab][j tile][t]
    auto load_a = [&](int jg) {
#pragma unroll
        for (int sl = 0; sl < 2; sl++) {
            const int ib = w0 + 16 * sl + 4 * g;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int j = (jg + q) * 16 + m;
                const bool jok = j < k;
#pragma unroll
                for (int t = 0; t < 4; t++)
                    a[sl][q][t] = (jok && ib + t < w1) ? Sr[(long long)(ib + t) * k + j] : 0.0;
            }
        }
    };
    load_a(0);

    // phase 1
    {
        const int cq = tid >> 5, rl = tid & 31, col = c0 + cq;
        const bool colok = col < nb;
        const int cc = colok ? col : 0;
        double *xc = X + (long long)cc * ldx;
        double xv[8], qv[8], pv[8], zv[8], bv[8];
        double pq = 0.0, rho = 0.0;
        int st = 0;
        const double *bc = nullptr;
        if (FIN) {
            pq = pieces_sum(f, cc);
            rho = f.scal[4 * cc + 3];
            st = status[cc];
            if (f.hist) bc = f.b + (long long)f.members[cc] * n;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int i = r0 + rl + 32 * u;
            const bool ok = colok && i < r1;
            xv[u] = ok ? xc[i] : 0.0;
            if (FIN) {
                const long long e = (long long)cc * n + i;
                qv[u] = ok ? f.q[e] : 0.0;
                pv[u] = ok ? f.p[e] : 0.0;
                zv[u] = ok ? f.x[e] : 0.0;
                bv[u] = (ok && bc) ? bc[i] : 0.0;
            }
        }
        if (FIN) {
            const bool upd = colok && st == COL_RUNNING && pq > 0.0 && isfinite(pq);
            const double alpha = upd ? rho / pq : 0.0;
            double rr = 0.0, xbr = 0.0;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = r0 + rl + 32 * u;
                if (upd && i < r1) {
                    const double rn = xv[u] - alpha * qv[u];
                    const double xn = zv[u] + alpha * pv[u];
                    xc[i] = rn;
                    f.x[(long long)cc * n + i] = xn;
                    rr += rn * rn;
                    if (bc) xbr += xn * (bv[u] + rn);
                    xv[u] = rn;
                }
            }
            // the 32 lanes of this column: fixed tree
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) {
                rr += __shfl_down(rr, o, 32);
                xbr += __shfl_down(xbr, o, 32);
            }
            if (rl == 0 && colok) {
                put(f.rr_part + (long long)rb * ldw + col, rr, one);
                put(f.xbr_part + (long long)rb * ldw + col, xbr, one);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; u++) xs[cq][rl + 32 * u] = xv[u];
    }
    const bool run = tile_running(status, c0, nb);
    __syncthreads();

    // phase 2
    for (int jg = 0; jg < njt; jg += 4) {
        if (jg > 0) load_a(jg);
        double4v acc[4];
#pragma unroll
        for (int q = 0; q < 4; q++) acc[q] = double4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int sl = 0; sl < 2; sl++)
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const double b = xs[m][wave * 32 + 16 * sl + 4 * g + t];  // zero beyond r1
#pragma unroll
                for (int q = 0; q < 4; q++)
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl][q][t], b, acc[q], 0, 0, 0);
            }
        // D[j][col] of tile q: lane l, element v -> j = (jg + q) 16 + l / 16 + 4 v, col = c0 + l % 16
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int v = 0; v < 4; v++) red[wave][q][v][lane] = acc[q][v];
        __syncthreads();
        for (int e = tid; e < 4 * 4 * 64; e += 512) {
            const int q = e >> 8, v = (e >> 6) & 3, l = e & 63;
            const int j = (jg + q) * 16 + (l >> 4) + 4 * v;
            if (run && j < k) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < 8; w++) s += red[w][q][v][l];
                put(part + ((long long)rb * k + j) * ldw + c0 + (l & 15), s, one);
            }
        }
        __syncthreads();
    }
}

template <bool FIN>
__global__ __launch_bounds__(512) void k_lmp_proj(int n, int k, int nb, int rows, const double *__restrict__ Sr,
                                                  double *X, long long ldx, const int32_t *__restrict__ status,
                                                  double *__restrict__ part, int ldw, LmpFin f) {
    __shared__ ProjLds L;
    lmp_proj<FIN>(blockIdx.x, blockIdx.y, n, k, nb, rows, Sr, X, ldx, status, part, ldw, f, L, false);
}

// Y = X + S W on 256 rows x 16 columns (eight waves).  Each thread loads, in
// one batch, its share of the row-block partials of W, this lane's S operands
// and X entries; the workgroup then forms W[j][c] = coef[j] sum_b part[b][j][c]
// (block order) in LDS, and wave w computes rows 32 w .. 32 w + 31 as two MFMA
// blocks on (W^T, S^T): A[m][g] = W[j][c0 + m], B[g][m] = S[i + m][j],
// j = j0 + g, so accumulator lanes run along rows (element v: row i + m,
// column c0 + g + 4 v).  FIN: the first workgroup of the tile then ends the
// iteration of its columns as the fused PCG kernel does (its inputs loaded at
// the start).
// xsl (single launch): X of this workgroup's rows, staged by its projection
// step (X was updated there for FIN); the other workgroups' partial sums are
// then read at device scope, past the CU's cache.
template <int KM, bool FIN>
__device__ __forceinline__ void lmp_expand(int rbx, int tile, int n, int k, int nb, int nrb,
                                           const double *__restrict__ S, const double *__restrict__ coef,
                                           const double *X, long long ldx, double *Y, long long ldy,
                                           int32_t *status, const double *__restrict__ part, int ldw,
                                           const LmpFin &f, double *__restrict__ rz, ExpandLds<KM> &L,
                                           const double (*xsl)[XP]) {
    constexpr int PE = KM * CT / 512;  // W entries per thread
    auto &ws = L.ws;
    auto &rzs = L.rzs;
    const int c0 = tile * CT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, m = lane & 15;
    const int ib = rbx * 256 + wave * 32;
    double pv[PE][LMP_RB_MAX];
#pragma unroll
    for (int u = 0; u < PE; u++) {
        const int e = tid + 512 * u;
        const bool ok = e < k * CT;
        const double *pe = part + (long long)(ok ? e / CT : 0) * ldw + c0 + e % CT;
#pragma unroll
        for (int b = 0; b < LMP_RB_MAX; b++) {
            const bool take = ok && b < nrb;
            pv[u][b] = !take ? 0.0 : (xsl ? load_agent(pe + (long long)b * k * ldw) : pe[(long long)b * k * ldw]);
        }
    }
    double xv[2][4];  // [row tile][v]
#pragma unroll
    for (int rt = 0; rt < 2; rt++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = ib + 16 * rt + m, col = c0 + g + 4 * v;
            if (xsl)
                xv[rt][v] = xsl[g + 4 * v][wave * 32 + 16 * rt + m];  // zero beyond n and nb
            else
                xv[rt][v] = (i < n && col < nb) ? X[(long long)col * ldx + i] : 0.0;
        }
    // FIN: the iteration-end inputs of column c0 + tid (first workgroup of the tile)
    const bool fin_lane = FIN && rbx == 0 && tid < CT && c0 + tid < nb;
    const int fcol = fin_lane ? c0 + tid : 0;
    double rv[LMP_RB_MAX], xr[LMP_RB_MAX], fpq = 0.0, fbn = 0.0, frho = 0.0;
    int fst = 0, fit = 0;  // fit: the column's own iteration
    if (FIN) {
#pragma unroll
        for (int b = 0; b < LMP_RB_MAX; b++) {
            const double *pr = f.rr_part + (long long)b * ldw + fcol, *px = f.xbr_part + (long long)b * ldw + fcol;
            rv[b] = (fin_lane && b < nrb) ? (xsl ? load_agent(pr) : *pr) : 0.0;
            xr[b] = (fin_lane && b < nrb && f.hist) ? (xsl ? load_agent(px) : *px) : 0.0;
        }
        if (fin_lane) {
            fpq = pieces_sum(f, fcol);
            fbn = f.scal[4 * fcol + 1];
            frho = f.scal[4 * fcol + 3];
            fst = status[fcol];
            fit = f.it - (f.start ? f.start[fcol] : 0);
        }
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
            for (int u = 0; u < PE; u++) {
                const int e = tid + 512 * u;
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
    if (run) {
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
    if (rz && run) {
        // r^T z of the block's 256 rows per column: this lane's two rows, the
        // 16 lanes of its row group (xor tree), then the waves in order
        double t[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            t[v] = xv[0][v] * (xv[0][v] + acc[0][v]) + xv[1][v] * (xv[1][v] + acc[1][v]);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) t[v] += __shfl_xor(t[v], o, 16);
        }
        if (m == 0) {
#pragma unroll
            for (int v = 0; v < 4; v++) rzs[wave][g + 4 * v] = t[v];
        }
        __syncthreads();
        if (tid < CT && c0 + tid < nb) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < 8; w++) sum += rzs[w][tid];
            rz[(long long)rbx * ldw + c0 + tid] = sum;
        }
    }
    if (FIN && fin_lane && fst == COL_RUNNING) {
        // the iteration's end for column fcol, as in the fused PCG kernel
        if (!(fpq > 0.0) || !isfinite(fpq)) {
            status[fcol] = EDA_MEMBER_BREAKDOWN;
            f.iters[fcol] = fit - 1;
        } else {
            double rr = 0.0, xbr = 0.0;
#pragma unroll
            for (int b = 0; b < LMP_RB_MAX; b++) {  // row blocks in order; absent ones add 0
                rr += rv[b];
                xbr += xr[b];
            }
            const double rn = sqrt(rr);
            f.scal[4 * fcol] = frho;
            f.scal[4 * fcol + 2] = rn / fbn;
            f.iters[fcol] = fit;
            if (f.hist && fit < f.hist_cap) f.hist[(long long)fcol * f.hist_cap + fit] = -0.5 * xbr;
            if (!isfinite(rn)) status[fcol] = EDA_MEMBER_BREAKDOWN;
            else if (rn <= f.rtol * fbn) status[fcol] = EDA_MEMBER_CONVERGED;
        }
    }
}

template <int KM, bool FIN>
__global__ __launch_bounds__(512) void k_lmp_expand(int n, int k, int nb, int nrb, const double *__restrict__ S,
                                                    const double *__restrict__ coef, const double *X, long long ldx,
                                                    double *Y, long long ldy, int32_t *status,
                                                    const double *__restrict__ part, int ldw, LmpFin f,
                                                    double *__restrict__ rz) {
    __shared__ ExpandLds<KM> L;
    lmp_expand<KM, FIN>(blockIdx.x, blockIdx.y, n, k, nb, nrb, S, coef, X, ldx, Y, ldy, status, part, ldw, f, rz, L,
                        nullptr);
}

// The tile barrier of the single launch.  The values other workgroups read
// (partial sums, FIN's row-block norms) went out as device-scope stores; each
// thread waits until its stores have completed, then thread 0 raises the
// tile's arrival counter and waits (bounded) until all nrb workgroups of the
// tile have arrived.  The readers take those values with device-scope loads,
// so no cache write-back or invalidation is needed.  The last workgroup to
// leave resets both counters for the next launch.
__device__ __forceinline__ void lmp_tile_barrier(const LmpSync &sy, int tile, int nrb) {
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(sy.arrive + tile, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool ok = false;
        for (long long it = 0; it < sy.spin_max; it++) {
            if (__hip_atomic_load(sy.arrive + tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)nrb) {
                ok = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) __hip_atomic_store(sy.err, LMP_SYNC_ERR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_fetch_add(sy.leave + tile, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            (unsigned)nrb - 1) {
            __hip_atomic_store(sy.arrive + tile, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sy.leave + tile, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
}

template <int KM, bool FIN>
__global__ __launch_bounds__(512) void k_lmp_one(int n, int k, int nb, int rows, int nrb,
                                                 const double *__restrict__ Sr, const double *__restrict__ S,
                                                 const double *__restrict__ coef, double *X, long long ldx, double *Y,
                                                 long long ldy, int32_t *status, double *__restrict__ part, int ldw,
                                                 LmpFin f, double *__restrict__ rz, LmpSync sy) {
    __shared__ ProjLds P;
    __shared__ ExpandLds<KM> E;
    lmp_proj<FIN>(blockIdx.x, blockIdx.y, n, k, nb, rows, Sr, X, ldx, status, part, ldw, f, P, true);
    lmp_tile_barrier(sy, blockIdx.y, nrb);
    lmp_expand<KM, FIN>(blockIdx.x, blockIdx.y, n, k, nb, nrb, S, coef, X, ldx, Y, ldy, status, part, ldw, f, rz,
                        E, P.xs);
}

}  // namespace

// Row blocks of the projection: 256 rows each (n <= 4096: at most LMP_RB_MAX).
void lmp_blocks(int n, int *rows, int *nrb) {
    *rows = 256;
    *nrb = (n + 255) / 256;
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

size_t lmp_sync_words(int ncols) { return 2 * (size_t)((ncols + CT - 1) / CT); }

size_t lmp_fin_doubles(int ncols) { return 2 * (size_t)LMP_RB_MAX * ((size_t)(ncols + CT - 1) / CT * CT); }

namespace {
template <bool FIN>
hipError_t lmp_launch(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                      double *X, long long ldx, double *Y, long long ldy, int32_t *status, double *work,
                      const LmpFin &f, double *rz, const LmpSync *sync) {
    if (n <= 0 || nb <= 0) return hipSuccess;
    if (k <= 0 || k > LMP_K_MAX) return hipErrorInvalidValue;
    int rows, nrb;
    lmp_blocks(n, &rows, &nrb);
    if (nrb > LMP_RB_MAX) return hipErrorInvalidValue;
    const int tiles = (nb + CT - 1) / CT, ldw = tiles * CT;
    if (sync && tiles <= sync->tiles && (long long)tiles * nrb <= sync->max_blocks) {
        if (k <= 64)
            hipLaunchKernelGGL((k_lmp_one<64, FIN>), dim3(nrb, tiles), dim3(512), 0, s, n, k, nb, rows, nrb, Sr, S,
                               coef, X, ldx, Y, ldy, status, work, ldw, f, rz, *sync);
        else
            hipLaunchKernelGGL((k_lmp_one<LMP_K_MAX, FIN>), dim3(nrb, tiles), dim3(512), 0, s, n, k, nb, rows, nrb,
                               Sr, S, coef, X, ldx, Y, ldy, status, work, ldw, f, rz, *sync);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_lmp_proj<FIN>, dim3(nrb, tiles), dim3(512), 0, s, n, k, nb, rows, Sr, X, ldx, status, work,
                       ldw, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (k <= 64)
        hipLaunchKernelGGL((k_lmp_expand<64, FIN>), dim3((n + 255) / 256, tiles), dim3(512), 0, s, n, k, nb, nrb, S,
                           coef, X, ldx, Y, ldy, status, work, ldw, f, rz);
    else
        hipLaunchKernelGGL((k_lmp_expand<LMP_K_MAX, FIN>), dim3((n + 255) / 256, tiles), dim3(512), 0, s, n, k, nb,
                           nrb, S, coef, X, ldx, Y, ldy, status, work, ldw, f, rz);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_lmp(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                      const double *X, long long ldx, double *Y, long long ldy, const int32_t *status,
                      double *work, double *rz, const LmpSync *sync) {
    // the plain form only reads X and status
    return lmp_launch<false>(s, n, k, nb, S, Sr, coef, const_cast<double *>(X), ldx, Y, ldy,
                             const_cast<int32_t *>(status), work, LmpFin{}, rz, sync);
}

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept; later calls return the kept address.
hipError_t lmp_noalloc_scratch(double **out) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static double *addr[MAX_DEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_lmp_fin(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                          double *r, double *z, int32_t *status, double *work, const LmpFin &f, double *rz,
                          const LmpSync *sync) {
    if (!status || f.pieces < 0 || (f.pieces == 0 && !f.nseg)) return hipErrorInvalidValue;
    return lmp_launch<true>(s, n, k, nb, S, Sr, coef, r, n, z, n, status, work, f, rz, sync);
}

}  // namespace eda

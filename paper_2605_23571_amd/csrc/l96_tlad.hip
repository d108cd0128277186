// Tangent-linear (TL) forward run and adjoint (AD) backward run of the
// Lorenz-96 RK4 model about stored trajectories -- the core of one Hessian
// product A x = U_B^T G^T R^-1 G U_B x (system_with_CVT equation).  The paper
// uses these runs (the integrations of the tangent linear and adjoint models in
// the sketching and Nystrom subsections) without printing them; they are the
// exact derivative of the RK4 step and its transpose:
//
//   J(y) v at i   = y_{i-1} (v_{i+1} - v_{i-2}) + (y_{i+1} - y_{i-2}) v_{i-1} - v_i
//   J(y)^T w at k = y_{k-2} w_{k-1} - y_{k+1} w_{k+2} + (y_{k+2} - y_{k-1}) w_{k+1} - w_k
//   TL: dk1 = J(x1) dx, dk2 = J(x2)(dx + h dk1), dk3 = J(x3)(dx + h dk2),
//       dk4 = J(x4)(dx + dt dk3), dx' = dx + dt/6 (dk1 + 2 dk2 + 2 dk3 + dk4)
//   AD: its reverse-mode transpose; the RK4 stage states x1..x4 are recomputed
//       from the stored X[s] (4x fewer trajectory bytes than storing them).
//
// Schedule (one workgroup per column, W waves; the ring of n points lives in
// the workgroup):
//  * wave w owns a contiguous segment [wS, wS + S) of the ring and computes on
//    a window of 64 Q points (Q per lane, contiguous) that adds halos on both
//    sides: the stencil's dependency cone grows by 8 points left / 4 right per
//    TL step and 4 left / 8 right per AD step, so a window with halos for TB
//    steps stays exact on the owned segment for TB steps;
//  * inside a wave, neighbours come from adjacent lanes by DPP wave shifts (no
//    LDS, no barrier); every TB steps the waves publish their owned segment to
//    a ring in LDS and re-read their windows after one barrier (two alternating
//    ring buffers);
//  * the observed increments R^-1 H dx written by the owners at observation
//    times are read back, at every window point, as the AD forcing.
//
// Modes TLAD_HV and TLAD_PCG also apply the banded circulant U_B on both sides
// inside the workgroup (the column is in LDS), and TLAD_PCG performs a whole
// PCG iteration for its member: p = z + beta p, q = (I + A) p, alpha, x and r
// updates, the convergence test -- one launch in place of eight.
#include <type_traits>

#include "eda_internal.h"
#include "nystrom_dev.h"

namespace eda {
namespace {

// lane l receives the value of lane l - 1 (wave_shr:1; lane 0 gets zero, which
// only reaches window-edge points).  bound_ctrl writes the zero itself, so no
// old value has to be materialised.
__device__ __forceinline__ double from_prev(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// lane l receives the value of lane l + 1 (wave_shl:1; lane 63 gets zero)
__device__ __forceinline__ double from_next(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// e[0..1] = previous lane's last two points, e[2..Q+1] = own, e[Q+2..Q+3] = next lane's first two.
template <typename T, int Q>
__device__ __forceinline__ void ext(const T (&v)[Q], T (&e)[Q + 4]) {
    e[0] = from_prev(v[Q - 2]);
    e[1] = from_prev(v[Q - 1]);
#pragma unroll
    for (int q = 0; q < Q; q++) e[2 + q] = v[q];
    e[Q + 2] = from_next(v[0]);
    e[Q + 3] = from_next(v[1]);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The tendency without its forcing, k'_i = (y_{i+1} - y_{i-2}) y_{i-1} - y_i
// (F enters the stage states through x + h F, precomputed once per step), and
// the TL increment dk_i = a_i v_{i-1} + y_{i-1} (v_{i+1} - v_{i-2}) - v_i with
// a_i = y_{i+1} - y_{i-2}, written as fused multiply-adds: 2 and 3 operations.
template <typename T, int Q, bool WANT_K>
__device__ __forceinline__ void tl_stage(const T (&y)[Q + 4], const T (&v)[Q + 4], T (&k)[Q], T (&dk)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++) {
        const T a = y[j + 3] - y[j];
        if (WANT_K) k[j] = fma_t(a, y[j + 1], -y[j + 2]);
        dk[j] = fma_t(a, v[j + 1], fma_t(y[j + 1], v[j + 3] - v[j], -v[j + 2]));
    }
}

template <typename T, int Q>
__device__ __forceinline__ void tendency(const T (&y)[Q + 4], T (&k)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++) k[j] = fma_t(y[j + 3] - y[j], y[j + 1], -y[j + 2]);
}

// (J^T w)_k = y_{k-2} w_{k-1} - y_{k+1} w_{k+2} + (y_{k+2} - y_{k-1}) w_{k+1} - w_k
template <typename T, int Q>
__device__ __forceinline__ void jt(const T (&y)[Q + 4], const T (&w)[Q + 4], T (&out)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++)
        out[j] = fma_t(y[j + 4] - y[j + 1], w[j + 3], fma_t(-y[j + 3], w[j + 4], fma_t(y[j], w[j + 1], -w[j + 2])));
}

// Ring position of this lane's window point q: base + q, wrapped once.
__device__ __forceinline__ int wpos(int base, int q, int n) {
    int p = base + q;
    return p >= n ? p - n : p;
}

// Copy of this wave's trajectory window -- 64 Q consecutive doubles of a
// padded state row, from xe on -- into the wave's LDS slice, through
// registers: lane l loads doubles 64 i + l (i in [I0, I1), coalesced) and
// stores them at the same slice positions, so slice[j] = xe[j].  The stores
// have the type of read_window's loads, so the compiler keeps them after the
// reads of the previous step.  The loads of the next step's window are issued
// early and stored late (load_part / store_part) where registers allow, else
// the whole copy is done at once (prefetch_window).  The copy goes through
// registers on purpose: direct global-to-LDS copies were measured to deliver
// stale or misplaced words now and then when workgroups share a CU, even
// behind a vector-memory wait.
template <int I0, int I1, int Q>
__device__ __forceinline__ void load_part(const double *xe, double (&v)[Q]) {
    const double *g = xe + (threadIdx.x & 63);
#pragma unroll
    for (int i = I0; i < I1; i++) v[i] = g[64 * i];
}
template <int I0, int I1, int Q>
__device__ __forceinline__ void store_part(double *slice, const double (&v)[Q]) {
    double *l = slice + (threadIdx.x & 63);
#pragma unroll
    for (int i = I0; i < I1; i++) l[64 * i] = v[i];
}
template <int Q>
__device__ __forceinline__ void prefetch_window(const double *xe, double *slice) {
    double v[Q];
    load_part<0, Q, Q>(xe, v);
    store_part<0, Q, Q>(slice, v);
}

// This lane's Q window points from the wave's slice (written by the same wave:
// its LDS stores and loads complete in order).
template <typename T, int Q>
__device__ __forceinline__ void read_window(const double *slice, T (&x)[Q]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; q++) x[q] = (T)slice[lane * Q + q];
}

// Observed increments R^-1 H dx of this lane's owned observed points.
template <typename T, int Q>
__device__ __forceinline__ void store_obs(double *o, const int *qi, const T (&dx)[Q], double inv_s2) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int oi = qi[q * 64 + lane];
        if (oi >= 0) o[oi] = (double)dx[q] * inv_s2;
    }
}

// Window of this lane on a ring of R points whose position j is the state
// index off + j (mod n): ring position of its first point (base; the others
// follow contiguously, wrapped), the mask of points inside the wave's owned
// segment, and, in LDS (qi[q * 64 + lane]), the observation index of observed
// points (-1 otherwise; if owned_obs_only, owned points at ring positions in
// [obs_lo, obs_hi) only).
template <int Q>
__device__ __forceinline__ int window(const TladArgs &a, int w0, int own_lo, int own_hi, bool owned_obs_only,
                                      unsigned &ownm, int *qi, int R, int off, int obs_lo = 0,
                                      int obs_hi = 0x7fffffff) {
    const int n = a.n, lane = threadIdx.x & 63;
    int b = (w0 + lane * Q) % R;
    if (b < 0) b += R;
    ownm = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        int p = wpos(b, q, R) + off;  // state index
        p = p < 0 ? p + n : (p >= n ? p - n : p);
        const int jw = w0 + lane * Q + q;  // unwrapped position
        const bool own = jw >= own_lo && jw < own_hi;
        if (own) ownm |= 1u << q;
        const int r = p - a.obs_x0;
        const bool obs = r >= 0 && r % a.obs_dx == 0;
        const bool keep = !owned_obs_only || (own && jw >= obs_lo && jw < obs_hi);
        qi[q * 64 + lane] = (obs && keep) ? r / a.obs_dx : -1;
    }
    return b;
}

// Banded circulant product at this lane's Q window points:
//   out[q] = sum_{m = 0}^{W-1} taps[m] u[(base + q - hi + m) mod n],
// taps[m] = r(|hi - m|), u and taps in LDS.  A circular register buffer of Q
// values keeps one LDS read per tap (Q FMAs per read, no register shifts).
template <int Q>
__device__ __forceinline__ void band_lane(const double *u, const double *taps, int W, int hi, int n, int base,
                                          double (&out)[Q]) {
    int idx = (base - hi) % n;
    if (idx < 0) idx += n;
    const int start = idx;
    double B[Q];
#pragma unroll
    for (int j = 0; j < Q; j++) {
        B[j] = u[idx];
        idx = idx + 1 == n ? 0 : idx + 1;
    }
#pragma unroll
    for (int q = 0; q < Q; q++) out[q] = 0.0;
    int m0 = 0;
    for (; m0 + Q <= W; m0 += Q) {
        // at entry B[j] = u[start + m0 + j]; slot mm is refilled with the next chunk after use
#pragma unroll
        for (int mm = 0; mm < Q; mm++) {
            const double t = taps[m0 + mm];
#pragma unroll
            for (int q = 0; q < Q; q++) out[q] += t * B[(mm + q) % Q];
            B[mm] = u[idx];
            idx = idx + 1 == n ? 0 : idx + 1;
        }
    }
    // remaining taps (fewer than Q): B[j] = u[start + m0 + j]
#pragma unroll
    for (int mm = 0; mm < Q - 1; mm++) {
        if (m0 + mm < W) {
            const double t = taps[m0 + mm];
#pragma unroll
            for (int q = 0; q < Q; q++) {
                double v;
                if (mm + q < Q) {
                    v = B[mm + q];
                } else {
                    int k = (start + m0 + mm + q) % n;
                    v = u[k];
                }
                out[q] += t * v;
            }
        }
    }
}

// Step constants in the arithmetic type of the run: h = dt / 2, dt, dt / 6,
// dt / 3 and h F.
template <typename T>
struct StepK {
    T h, dt, dt6, dt3, hF;
};

// One TL step of this lane's window: dx <- M_s dx about the trajectory state in
// the wave's window slice xw (X[s]); xn is the next step's window in the
// padded trajectory, copied into xw around the step (all early for Q <= 7, half
// and half for Q > 7, at once for !EARLY when `more`).
template <typename T, int Q, bool EARLY>
__device__ __forceinline__ void tl_step(const StepK<T> &K, double *xw, const double *xn, bool more, T (&dx)[Q]) {
    const T h = K.h, dt = K.dt, dt6 = K.dt6, hF = K.hF;
    T x[Q], Y[Q + 4], V[Q + 4], k[Q], dk[Q], acc[Q], ys[Q], vs[Q];
    read_window<T, Q>(xw, x);
    // next step's window: all of it early (Q <= 7), half early and
    // half after the second stage (Q > 7), or at once (!EARLY)
    // (the last step reloads its own row: no branch inside the step)
    double nxt[Q];
    if constexpr (!EARLY) {
        if (more) prefetch_window<Q>(xn, xw);
    } else if constexpr (Q <= 7) {
        load_part<0, Q, Q>(xn, nxt);
    } else {
        load_part<0, Q / 2, Q>(xn, nxt);
    }
    ext<T, Q>(x, Y);
    ext<T, Q>(dx, V);
    tl_stage<T, Q, true>(Y, V, k, dk);
#pragma unroll
    for (int j = 0; j < Q; j++) {
        x[j] += hF;  // x + h F: the stage states are x + h (k' + F)
        acc[j] = dk[j];
        ys[j] = fma_t(h, k[j], x[j]);
        vs[j] = fma_t(h, dk[j], dx[j]);
    }
    ext<T, Q>(ys, Y);
    ext<T, Q>(vs, V);
    tl_stage<T, Q, true>(Y, V, k, dk);
    if constexpr (EARLY && Q > 7) {
        store_part<0, Q / 2, Q>(xw, nxt);
        load_part<Q / 2, Q, Q>(xn, nxt);
    }
#pragma unroll
    for (int j = 0; j < Q; j++) {
        acc[j] = fma_t(T(2), dk[j], acc[j]);
        ys[j] = fma_t(h, k[j], x[j]);
        vs[j] = fma_t(h, dk[j], dx[j]);
    }
    ext<T, Q>(ys, Y);
    ext<T, Q>(vs, V);
    tl_stage<T, Q, true>(Y, V, k, dk);
#pragma unroll
    for (int j = 0; j < Q; j++) {
        acc[j] = fma_t(T(2), dk[j], acc[j]);
        ys[j] = fma_t(dt, k[j], x[j] + hF);  // x + dt F
        vs[j] = fma_t(dt, dk[j], dx[j]);
    }
    ext<T, Q>(ys, Y);
    ext<T, Q>(vs, V);
    tl_stage<T, Q, false>(Y, V, k, dk);
#pragma unroll
    for (int j = 0; j < Q; j++) dx[j] = fma_t(dt6, acc[j] + dk[j], dx[j]);
    if constexpr (EARLY) store_part<(Q <= 7 ? 0 : Q / 2), Q, Q>(xw, nxt);
}

// One AD step of this lane's window: lam <- M_{s-1}^T lam about the state in
// xw (X[s - 1]); xn is the next window (X[s - 2]), copied into xw as in tl_step.
template <typename T, int Q, bool EARLY>
__device__ __forceinline__ void ad_step(const StepK<T> &K, double *xw, const double *xn, bool more, T (&lam)[Q]) {
    const T h = K.h, dt = K.dt, dt6 = K.dt6, dt3 = K.dt3, hF = K.hF;
    T x[Q], Y2[Q + 4], Y3[Q + 4], Y4[Q + 4], M[Q + 4], k[Q], ys[Q];
    read_window<T, Q>(xw, x);  // X[s - 1]
    // next step's window (X[s - 2]), split as in the TL run
    double nxt[Q];
    if constexpr (!EARLY) {
        if (more) prefetch_window<Q>(xn, xw);
    } else if constexpr (Q <= 7) {
        load_part<0, Q, Q>(xn, nxt);
    } else {
        load_part<0, Q / 2, Q>(xn, nxt);
    }
    {
        T Y1[Q + 4];
        ext<T, Q>(x, Y1);
        tendency<T, Q>(Y1, k);
    }
    // stage states x + h (k' + F) and x + dt (k' + F), from xh = x + h F
#pragma unroll
    for (int j = 0; j < Q; j++) ys[j] = fma_t(h, k[j], x[j] + hF);
    ext<T, Q>(ys, Y2);
    tendency<T, Q>(Y2, k);
#pragma unroll
    for (int j = 0; j < Q; j++) ys[j] = fma_t(h, k[j], x[j] + hF);
    ext<T, Q>(ys, Y3);
    tendency<T, Q>(Y3, k);
#pragma unroll
    for (int j = 0; j < Q; j++) ys[j] = fma_t(dt, k[j], (x[j] + hF) + hF);
    ext<T, Q>(ys, Y4);
    // backward through the stages: mu4 = dt/6 lam, mu3 = mu2 = dt/3 lam, mu1 = dt/6 lam
    T nu[Q], acc[Q], mu[Q];
#pragma unroll
    for (int j = 0; j < Q; j++) mu[j] = dt6 * lam[j];
    ext<T, Q>(mu, M);
    jt<T, Q>(Y4, M, nu);
    if constexpr (EARLY && Q > 7) {
        store_part<0, Q / 2, Q>(xw, nxt);
        load_part<Q / 2, Q, Q>(xn, nxt);
    }
#pragma unroll
    for (int j = 0; j < Q; j++) {
        acc[j] = lam[j] + nu[j];
        mu[j] = dt3 * lam[j] + dt * nu[j];
    }
    ext<T, Q>(mu, M);
    jt<T, Q>(Y3, M, nu);
#pragma unroll
    for (int j = 0; j < Q; j++) {
        acc[j] += nu[j];
        mu[j] = dt3 * lam[j] + h * nu[j];
    }
    ext<T, Q>(mu, M);
    jt<T, Q>(Y2, M, nu);
#pragma unroll
    for (int j = 0; j < Q; j++) {
        acc[j] += nu[j];
        mu[j] = dt6 * lam[j] + h * nu[j];
    }
    ext<T, Q>(mu, M);
    {
        T Y1[Q + 4];
        ext<T, Q>(x, Y1);
        jt<T, Q>(Y1, M, nu);
    }
#pragma unroll
    for (int j = 0; j < Q; j++) lam[j] = acc[j] + nu[j];
    if constexpr (EARLY) store_part<(Q <= 7 ? 0 : Q / 2), Q, Q>(xw, nxt);
}

// Deterministic workgroup sum (fixed shuffle tree per wave, then waves in order).
__device__ __forceinline__ double block_sum(double v, double *red, int waves) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < waves; w++) s += red[w];
    return s;
}

// Waits (bounded) until both flags reach `want`.
__device__ __forceinline__ bool xch_wait(const unsigned long long *fa, const unsigned long long *fb,
                                         unsigned long long want, long long spin_max) {
    for (long long it = 0; it < spin_max; it++) {
        const unsigned long long va = __hip_atomic_load(fa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long vb = __hip_atomic_load(fb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (va >= want && vb >= want) return true;
    }
    return false;
}

// Device-scope load and store of a double: they bypass the (per-XCD,
// non-coherent) L2, so a value stored by a workgroup on one XCD is read by
// one on another once the store has completed.
__device__ __forceinline__ double load_dev(const double *p) {
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void store_dev(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Observed increments of this lane's owned observed points, stored at device
// scope (shared-observation pieces: the other pieces of the column read them).
template <typename T, int Q>
__device__ __forceinline__ void store_obs_dev(double *o, const int *qi, const T (&dx)[Q], double inv_s2) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int oi = qi[q * 64 + lane];
        if (oi >= 0) store_dev(o + oi, (double)dx[q] * inv_s2);
    }
}

// Shared-observation pieces (TLAD_SPLIT_SH, TLAD_SPLIT_HV_SH), between the TL
// and AD runs of piece `piece` of column c: the
// piece has stored the observed increments of its owned states in its own
// block, at device scope; every wave waits for its stores to complete, then
// the piece raises its flag to this launch's value and waits (bounded) for
// both neighbours' flags, after which their blocks can be read at device
// scope.  No cache line is written by two pieces, and a piece reads a
// neighbour's block only after the flag, so no XCD's L2 holds a stale copy.
// (Device-scope release and acquire fences, which write back and invalidate
// whole L2s, made the launch 10-25% slower.)  A wait that gives up sets the
// error word, stops the member in PCG (its results are void) and makes the
// function return false; the piece still raised its flag, so no neighbour
// waits on it.
__device__ __forceinline__ bool share_obs(const TladArgs &a, int c, int piece) {
    __shared__ int s_ok;
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *fl = a.pflags + (long long)c * SPLIT_PMAX;
        __hip_atomic_store(fl + piece, a.want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int left = piece == 0 ? a.pieces - 1 : piece - 1;
        const int right = piece == a.pieces - 1 ? 0 : piece + 1;
        const bool ok = xch_wait(fl + left, fl + right, a.want, a.spin_max);
        if (!ok) {
            __hip_atomic_store(a.err, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.pcg.status) a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;
        }
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return s_ok != 0;
}

// One column of one problem, all modes (the workgroup's whole job in k_tlad,
// one step of the task loop in k_solve).  PCG mode runs iteration `it` (first:
// p = z).  SPLIT mode runs the Hessian part of that iteration on piece `piece`
// of the column: the ring is the piece's owned states [lo, hi) with a.halo
// states on each side (ring position j = state lo - halo + j mod n); positions
// whose dependency cone reaches the ring's seam are wrong, the owned ones
// exact.  SPLIT_SH mode runs SPLIT with the pieces sharing the column's
// observed increments (share_obs; the halos of tlad_split_ring_sh): a.halo is
// then the TL ring's left halo, and the AD run uses the ring moved 4 N states
// right.  Every early exit is taken by the whole workgroup.
template <typename T, int Q, int MODE, bool EARLY = true>
__device__ __forceinline__ void tlad_column(const TladArgs &a, const TladGeom &g, const int c, const int it,
                                            const int first, unsigned char *smraw, const int piece = 0) {
    constexpr bool SPLIT_HV = MODE == TLAD_SPLIT_HV || MODE == TLAD_SPLIT_HV_SH;
    constexpr bool SHARE = MODE == TLAD_SPLIT_SH || MODE == TLAD_SPLIT_HV_SH;  // pieces share the observed increments
    constexpr bool SPLIT = MODE == TLAD_SPLIT || SPLIT_HV || SHARE;  // ring of one piece
    constexpr bool FUSED = (MODE == TLAD_HV || MODE == TLAD_PCG || SPLIT);
    const int n = a.n, N = a.N, p = a.nt * a.nv;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x, nthr = blockDim.x;
    // ring length, state index of ring position 0, owned ring positions
    const int R = SPLIT ? a.ring : n;
    int off = 0, core_lo = 0, core_hi = n;
    if (SPLIT) {
        const int lo = (int)((long long)piece * n / a.pieces), hi = (int)((long long)(piece + 1) * n / a.pieces);
        off = lo - a.halo;
        core_lo = a.halo;
        core_hi = a.halo + hi - lo;
    }
    auto state = [&](int j) {  // state index of ring position j
        int v = off + j;
        return v < 0 ? v + n : (v >= n ? v - n : v);
    };
    // LDS: [ring: 2R T][qi: waves*64*Q int][xw: waves*64*Q double][u: R double][taps: W double][red: 16 double]
    T *ring = reinterpret_cast<T *>(smraw);  // two buffers, indexed rsel * R + position
    int *qi = reinterpret_cast<int *>(ring + 2 * R) + wave * 64 * Q;
    double *xw_all = reinterpret_cast<double *>(reinterpret_cast<int *>(ring + 2 * R) + g.waves * 64 * Q);
    double *xw = xw_all + wave * 64 * Q;  // this wave's trajectory window slice
    double *u = xw_all + g.waves * 64 * Q;
    double *taps = u + R;
    const int W = a.band_hi - a.band_lo + 1;
    double *red = taps + W;
    double *lamd = reinterpret_cast<double *>(ring);  // ring reused as a double array for lambda_0
    const int own_lo = wave * g.S, own_hi = min(R, own_lo + g.S);
    const int member = (MODE == TLAD_PCG || MODE == TLAD_SPLIT || MODE == TLAD_SPLIT_SH) ? a.pcg.members[c]
                                                               : (a.col_member ? a.col_member[c] : 0);
    // row s of the member's padded trajectory, from ring position 0: trajm + s ext_len
    const double *trajm = a.trajx + (long long)member * a.trajx_stride + a.pad_l + off;
    // this piece's block of observed increments (per column, per piece if SPLIT)
    const long long obs_at = ((long long)c * (SPLIT ? a.pieces : 1) + piece) * p;
    const StepK<T> K{(T)a.h, (T)a.dt, (T)a.dt6, (T)a.dt3, (T)(a.h * a.F)};
    unsigned ownm;
    int rsel = 0;
    double rho = 0.0;
    const long long cn = (long long)c * n;

    // ---------------- input vector and U_B on the way in (fused modes) ----------------
    if (FUSED) {
        for (int m = tid; m < W; m += nthr) {
            int o = a.band_hi - m;
            taps[m] = a.ubrow[o < 0 ? -o : o];
        }
        if (MODE == TLAD_HV) {
            const double *x = a.V + (long long)c * a.ldv;
            for (int i = tid; i < n; i += nthr) u[i] = x[i];
        } else if (SPLIT_HV) {
            const double *x = a.V + (long long)c * a.ldv;
            for (int j = tid; j < R; j += nthr) u[j] = x[state(j)];
        } else {
            // p = z + beta p with beta = rho'/rho, rho' = r^T z; first iteration p = z
            const double *z = a.pcg.z + cn;
            double *pp = a.pcg.p + cn;
            double rz = 0.0;
            if (a.pcg.rz_part) {
                // the LMP's row-block sums, in block order (every thread the same bits)
                double v[LMP_RB_MAX];
#pragma unroll
                for (int b = 0; b < LMP_RB_MAX; b++)
                    v[b] = b < a.pcg.rz_nrb ? a.pcg.rz_part[(long long)b * a.pcg.rz_ld + c] : 0.0;
#pragma unroll
                for (int b = 0; b < LMP_RB_MAX; b++) rz += v[b];
            } else {
                const double *r = a.pcg.r + cn;
                for (int i = tid; i < n; i += nthr) rz += r[i] * z[i];
                rz = block_sum(rz, red, g.waves);
            }
            // a column admitted later starts at its own first iteration
            const bool first_c = a.pcg.start ? it - a.pcg.start[c] == 1 : first != 0;
            double beta = 0.0;
            if (!first_c) {
                if (!(rz > 0.0) || !isfinite(rz)) {
                    if (tid == 0 && piece == 0) a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;
                    return;
                }
                beta = rz / a.pcg.scal[4 * c];
            }
            rho = rz;
            if (!SPLIT) {
                for (int i = tid; i < n; i += nthr) {
                    double v = first_c ? z[i] : z[i] + beta * pp[i];
                    pp[i] = v;
                    u[i] = v;
                }
            } else {
                // p over the ring from the previous p; the new p written for the owned states only
                double *pout = a.pcg.p_out + cn;
                for (int j = tid; j < R; j += nthr) {
                    const int gi = state(j);
                    const double v = first_c ? z[gi] : z[gi] + beta * pp[gi];
                    u[j] = v;
                    if (j >= core_lo && j < core_hi) pout[gi] = v;
                }
                if (piece == 0 && tid == 0) a.pcg.scal[4 * c + 3] = rz;  // rho of this iteration, for the update
            }
        }
        __syncthreads();
    }

    if (MODE != TLAD_ADJ) {
        // ---------------- TL forward run ----------------
        const int w0 = own_lo - g.hl_tl;
        prefetch_window<Q>(trajm + w0, xw);
        int base = SHARE ? window<Q>(a, w0, own_lo, own_hi, true, ownm, qi, R, off, core_lo, core_hi)
                         : window<Q>(a, w0, own_lo, own_hi, true, ownm, qi, R, off);
        T dx[Q];
        if (FUSED) {
            double v0[Q];
            band_lane<Q>(u, taps, W, a.band_hi, R, base, v0);
#pragma unroll
            for (int q = 0; q < Q; q++) dx[q] = (T)v0[q];
        } else {
            const double *vcol = a.V + (long long)c * a.ldv;
#pragma unroll
            for (int q = 0; q < Q; q++) dx[q] = (T)vcol[wpos(base, q, n)];
        }
        double *obs = a.obs + obs_at;
        for (int s0 = 0; s0 < N; s0 += g.tb) {
            if (s0 > 0) {
                __syncthreads();
#pragma unroll
                for (int q = 0; q < Q; q++) dx[q] = ring[rsel * R + wpos(base, q, R)];
            }
            const int s1 = min(N, s0 + g.tb);
            for (int s = s0; s < s1; s++) {
                // observed increment of time s
                if (s > 0 && s % a.obs_dt == 0) {
                    if constexpr (SHARE) store_obs_dev<T, Q>(obs + (long long)(s / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
                    else store_obs<T, Q>(obs + (long long)(s / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
                }
                tl_step<T, Q, EARLY>(K, xw, trajm + (long long)min(s + 1, N - 1) * a.ext_len + w0, s + 1 < N, dx);
            }
            if (s1 < N) {
#pragma unroll
                for (int q = 0; q < Q; q++)
                    if (ownm & (1u << q)) ring[(rsel ^ 1) * R + wpos(base, q, R)] = dx[q];
                rsel ^= 1;
            }
        }
        if (N % a.obs_dt == 0) {
            if constexpr (SHARE) store_obs_dev<T, Q>(obs + (long long)(N / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
            else store_obs<T, Q>(obs + (long long)(N / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
        }
        __threadfence_block();  // observed increments visible to the whole workgroup
    }
    bool shared_ok = true;
    if constexpr (SHARE) {
        shared_ok = share_obs(a, c, piece);
        // the AD ring: the TL ring moved 4 N states right
        off += 4 * N;
        core_lo -= 4 * N;
        core_hi -= 4 * N;
        trajm += 4 * N;
    }
    __syncthreads();  // TL reads of the ring and of the observation indices are done

    // ---------------- AD backward run ----------------
    const int w0 = own_lo - g.hl_ad;
    prefetch_window<Q>(trajm + (long long)(N - 1) * a.ext_len + w0, xw);
    const int base = window<Q>(a, w0, own_lo, own_hi, false, ownm, qi, R, off);
    // SHARE: the forcing of a window point is read from the block of the piece
    // that owns its state (this one or a neighbour; the index into the column's
    // blocks is folded into qi)
    const double *force = (MODE == TLAD_ADJ) ? a.force + (long long)c * p
                          : SHARE            ? a.obs + (long long)c * a.pieces * p
                                             : a.obs + obs_at;
    if constexpr (SHARE) {
        const int left = piece == 0 ? a.pieces - 1 : piece - 1;
        const int right = piece == a.pieces - 1 ? 0 : piece + 1;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int jr = wpos(base, q, R);
            int &e = qi[q * 64 + lane];
            if (e >= 0) e += (jr < core_lo ? left : jr >= core_hi ? right : piece) * p;
        }
    }
    T lam[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) lam[q] = T(0);
    for (int s_hi = N; s_hi >= 1; s_hi -= g.tb) {
        if (s_hi < N) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; q++) lam[q] = ring[rsel * R + wpos(base, q, R)];
        }
        const int s_lo = max(0, s_hi - g.tb);
        for (int s = s_hi; s > s_lo; s--) {
            if (s % a.obs_dt == 0) {
                const double *f = force + (long long)(s / a.obs_dt - 1) * a.nv;
            #pragma unroll
                for (int q = 0; q < Q; q++) {
                    const int oi = qi[q * 64 + lane];
                    if constexpr (SHARE) {
                        if (oi >= 0) lam[q] += (T)load_dev(f + oi);
                    } else {
                        if (oi >= 0) lam[q] += (T)f[oi];
                    }
                }
            }
            ad_step<T, Q, EARLY>(K, xw, trajm + (long long)max(s - 2, 0) * a.ext_len + w0, s >= 2, lam);
        }
        if (s_lo > 0) {
#pragma unroll
            for (int q = 0; q < Q; q++)
                if (ownm & (1u << q)) ring[(rsel ^ 1) * R + wpos(base, q, R)] = lam[q];
            rsel ^= 1;
        }
    }

    if (!FUSED) {
        double *out = a.lam + (long long)c * a.ldl;
#pragma unroll
        for (int q = 0; q < Q; q++)
            if (ownm & (1u << q)) out[wpos(base, q, n)] = (double)lam[q];
        return;
    }

    // ---------------- U_B on the way out (fused modes) ----------------
    __syncthreads();  // every wave is done reading the ring
#pragma unroll
    for (int q = 0; q < Q; q++)
        if (ownm & (1u << q)) lamd[wpos(base, q, R)] = (double)lam[q];
    __syncthreads();
    double y[Q];
    band_lane<Q>(lamd, taps, W, a.band_hi, R, base, y);
    if (MODE == TLAD_HV) {
        double *out = a.lam + (long long)c * a.ldl;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            if (ownm & (1u << q)) {
                const int ps = wpos(base, q, n);
                out[ps] = a.add_identity ? y[q] + u[ps] : y[q];
            }
        }
        return;
    }

    if (SPLIT_HV) {
        // Y (+ X) at the owned states of this piece
        double *out = a.lam + (long long)c * a.ldl;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int j = wpos(base, q, R);
            if ((ownm & (1u << q)) && j >= core_lo && j < core_hi) {
                // (a shared-observation wait that gave up voids the product: NaN)
                const double v = a.add_identity ? y[q] + u[SHARE ? j + 4 * N : j] : y[q];
                out[state(j)] = shared_ok ? v : __builtin_nan("");
            }
        }
        return;
    }

    if (SPLIT) {
        // (I + A) p at the owned states and this piece's part of p^T (I + A) p
        double pq = 0.0;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int j = wpos(base, q, R);
            if ((ownm & (1u << q)) && j >= core_lo && j < core_hi) {
                const double pv = u[SHARE ? j + 4 * N : j];  // u is on the TL ring
                y[q] += pv;
                pq += pv * y[q];
                a.pcg.q[cn + state(j)] = y[q];
            }
        }
        pq = block_sum(pq, red, g.waves);
        if (tid == 0) a.pcg.pq_part[(long long)c * a.pieces + piece] = pq;
        return;
    }

    // ---------------- PCG update: q = (I + A) p, alpha, x, r, convergence ----------------
    double pq = 0.0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        if (ownm & (1u << q)) {
            const double pv = u[wpos(base, q, n)];
            y[q] += pv;  // (I + A) p
            pq += pv * y[q];
        }
    }
    pq = block_sum(pq, red, g.waves);
    const int itc = it - (a.pcg.start ? a.pcg.start[c] : 0);  // the column's own iteration
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (tid == 0) {
            a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;
            a.pcg.iters[c] = itc - 1;
        }
        return;
    }
    const double alpha = rho / pq;
    double *xv = a.pcg.x + cn, *rv = a.pcg.r + cn;
    const double *bv = a.pcg.b + (long long)member * n;
    double rr = 0.0, xbr = 0.0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        if (ownm & (1u << q)) {
            const int ps = wpos(base, q, n);
            const double xi = xv[ps] + alpha * u[ps];
            const double ri = rv[ps] - alpha * y[q];
            xv[ps] = xi;
            rv[ps] = ri;
            rr += ri * ri;
            if (a.pcg.hist) xbr += xi * (bv[ps] + ri);
        }
    }
    rr = block_sum(rr, red, g.waves);
    if (a.pcg.hist) xbr = block_sum(xbr, red, g.waves);
    if (tid == 0) {
        const double bnorm = a.pcg.scal[4 * c + 1];
        const double rn = sqrt(rr);
        a.pcg.scal[4 * c] = rho;
        a.pcg.scal[4 * c + 2] = rn / bnorm;
        a.pcg.iters[c] = itc;
        if (a.pcg.hist && itc < a.pcg.hist_cap) a.pcg.hist[(long long)c * a.pcg.hist_cap + itc] = -0.5 * xbr;
        if (!isfinite(rn)) a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;
        else if (rn <= a.pcg.rtol * bnorm) a.pcg.status[c] = EDA_MEMBER_CONVERGED;
    }
}

template <typename T, int Q, int MODE>
__global__ __launch_bounds__(512) void k_tlad(TladArgs a, TladGeom g) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int c = blockIdx.x;
    if (MODE == TLAD_PCG) {
        if (a.pcg.status[c] != COL_RUNNING) return;
    } else if (a.active && a.active[c] != COL_RUNNING) {
        return;
    }
    tlad_column<T, Q, MODE>(a, g, c, a.pcg.it, a.pcg.first, smraw);
}

// Workgroup b of a split launch over m columns of P pieces each: column
// index ci (into the launch's column list) and piece.  Columns go in groups of
// eight with their P pieces eight workgroups apart, so that a column's pieces
// run on one XCD (the XCDs are dealt workgroups in turn) and read the
// trajectory and vector values of their shared halos through one L2; the last
// m mod 8 columns take their pieces in turn.  A bijection onto m x P.
__device__ __forceinline__ void split_slot(int b, int m, int P, int &ci, int &piece) {
    const int full = m & ~7;
    if (b < full * P) {
        const int grp = b >> 3;
        ci = (grp / P) * 8 + (b & 7);
        piece = grp % P;
    } else {
        const int r = m - full, e = b - full * P;
        ci = full + e % r;
        piece = e / r;
    }
}

// Split iterations: the workgroups take the pieces of the listed columns (m =
// sc.count, or every column) as split_slot deals them.
template <int Q>
__global__ __launch_bounds__(512) void k_tlad_split(TladArgs a, TladGeom g, SplitCols sc) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int m = sc.count > 0 ? sc.count : a.nb;
    int ci, piece;
    split_slot(blockIdx.x, m, a.pieces, ci, piece);
    const int c = sc.count > 0 ? sc.col[ci] : ci;
    if (a.pcg.status[c] != COL_RUNNING) return;
    tlad_column<double, Q, TLAD_SPLIT>(a, g, c, a.pcg.it, a.pcg.first, smraw, piece);
}

// The same with the pieces of a column sharing its observed increments
// (TLAD_SPLIT_SH); every piece of a running column reaches share_obs (the
// column's status and r^T z are the same for all of them).
template <int Q>
__global__ __launch_bounds__(512) void k_tlad_split_sh(TladArgs a, TladGeom g, SplitCols sc) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int m = sc.count > 0 ? sc.count : a.nb;
    int ci, piece;
    split_slot(blockIdx.x, m, a.pieces, ci, piece);
    const int c = sc.count > 0 ? sc.col[ci] : ci;
    if (a.pcg.status[c] != COL_RUNNING) return;
    tlad_column<double, Q, TLAD_SPLIT_SH>(a, g, c, a.pcg.it, a.pcg.first, smraw, piece);
}

// Split Hessian products: the workgroups take the pieces of the nb columns as
// split_slot deals them (TL/AD in T; the U_B products and the trajectory stay
// FP64).
template <typename T, int Q>
__global__ __launch_bounds__(512) void k_tlad_split_hv(TladArgs a, TladGeom g) {
    extern __shared__ __align__(16) unsigned char smraw[];
    int c, piece;
    split_slot(blockIdx.x, a.nb, a.pieces, c, piece);
    if (a.active && a.active[c] != COL_RUNNING) return;
    tlad_column<T, Q, TLAD_SPLIT_HV>(a, g, c, 0, 0, smraw, piece);
}

// The same with the pieces of a column sharing its observed increments
// (TLAD_SPLIT_HV_SH); every piece of an active column reaches share_obs.
template <typename T, int Q>
__global__ __launch_bounds__(512) void k_tlad_split_hv_sh(TladArgs a, TladGeom g) {
    extern __shared__ __align__(16) unsigned char smraw[];
    int c, piece;
    split_slot(blockIdx.x, a.nb, a.pieces, c, piece);
    if (a.active && a.active[c] != COL_RUNNING) return;
    tlad_column<T, Q, TLAD_SPLIT_HV_SH>(a, g, c, 0, 0, smraw, piece);
}

// z = P r = r + S diag(coef) S^T r for one column (in-kernel LMP of the
// persistent solve).  r is first staged in LDS (rs, n doubles).  t = coef .*
// (S^T r): the k dot products are split over the waves, two directions per
// wave at a time; lane l keeps eight partial sums per direction, partial
// u mod 8 taking rows l + 64 u of each 512-row stride in turn, then a fixed
// shuffle tree.  z = r + S t: rows over the threads, two rows per thread at a
// time, the columns of S in order.  S lives in HBM or the last-level cache,
// so each step is one memory round trip: the loads of up to four strides of
// both directions (phase one) or of 32 columns for both rows (phase two) are
// issued together before the sums that use them, in the same summation order
// as a stride-at-a-time loop over one direction (one row).  r and z are the
// column's global vectors, tsh k doubles of LDS.
template <int U>
__device__ __forceinline__ void lmp_dot_strides2(const double *sj, const double *sj2, const double *rs, int i,
                                                 double (&acc)[8], double (&acc2)[8]) {
    double sv[8 * U], sv2[8 * U];
#pragma unroll
    for (int u = 0; u < 8 * U; u++) sv[u] = sj[i + u * 64];
#pragma unroll
    for (int u = 0; u < 8 * U; u++) sv2[u] = sj2[i + u * 64];
#pragma unroll
    for (int u = 0; u < 8 * U; u++) {
        const double rv = rs[i + u * 64];
        acc[u & 7] += sv[u] * rv;
        acc2[u & 7] += sv2[u] * rv;
    }
}

__device__ __forceinline__ void lmp_column(const PcgCols &pc, int n, const double *r, double *z, double *rs,
                                           double *tsh, int waves) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x, nthr = blockDim.x;
    const int k = pc.lmp_k;
    for (int i = tid; i < n; i += nthr) rs[i] = r[i];
    __syncthreads();
    for (int j = wave; j < k; j += 2 * waves) {
        // directions j and j2 (j2 past k: a repeat of j whose sum is dropped)
        const int j2 = j + waves < k ? j + waves : j;
        const double *sj = pc.lmp_s + (long long)j * n, *sj2 = pc.lmp_s + (long long)j2 * n;
        double acc[8], acc2[8];
#pragma unroll
        for (int u = 0; u < 8; u++) acc[u] = acc2[u] = 0.0;
        int i = lane;
        for (; i + 31 * 64 < n; i += 32 * 64) lmp_dot_strides2<4>(sj, sj2, rs, i, acc, acc2);
        if (i + 15 * 64 < n) {
            lmp_dot_strides2<2>(sj, sj2, rs, i, acc, acc2);
            i += 16 * 64;
        }
        if (i + 7 * 64 < n) {
            lmp_dot_strides2<1>(sj, sj2, rs, i, acc, acc2);
            i += 8 * 64;
        }
        for (; i < n; i += 64) {
            acc[0] += sj[i] * rs[i];
            acc2[0] += sj2[i] * rs[i];
        }
        double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        double sum2 = ((acc2[0] + acc2[1]) + (acc2[2] + acc2[3])) + ((acc2[4] + acc2[5]) + (acc2[6] + acc2[7]));
        for (int off = 32; off > 0; off >>= 1) {
            sum += __shfl_down(sum, off, 64);
            sum2 += __shfl_down(sum2, off, 64);
        }
        if (lane == 0) {
            tsh[j] = pc.lmp_c[j] * sum;
            if (j2 != j) tsh[j2] = pc.lmp_c[j2] * sum2;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += 2 * nthr) {
        // rows i and i2 (i2 past n: a repeat of i whose result is dropped)
        const int i2 = i + nthr < n ? i + nthr : i;
        const double *si = pc.lmp_s + i, *si2 = pc.lmp_s + i2;
        double v = rs[i], v2 = rs[i2];
        int j = 0;
        for (; j + 32 <= k; j += 32) {
            double sv[32], sv2[32];
#pragma unroll
            for (int u = 0; u < 32; u++) sv[u] = si[(long long)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 32; u++) sv2[u] = si2[(long long)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 32; u++) {
                v += sv[u] * tsh[j + u];
                v2 += sv2[u] * tsh[j + u];
            }
        }
        for (; j + 8 <= k; j += 8) {
            double sv[8], sv2[8];
#pragma unroll
            for (int u = 0; u < 8; u++) sv[u] = si[(long long)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 8; u++) sv2[u] = si2[(long long)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                v += sv[u] * tsh[j + u];
                v2 += sv2[u] * tsh[j + u];
            }
        }
        for (; j < k; j++) {
            v += si[(long long)j * n] * tsh[j];
            v2 += si2[(long long)j * n] * tsh[j];
        }
        z[i] = v;
        if (i2 != i) z[i2] = v2;
    }
    __syncthreads();
}

// The whole LMP-PCG solve of column c of problem a (Q points per lane): the
// same iteration as eda_pcg_solve's fused path (tlad_column in PCG mode),
// with the LMP applied in-kernel, so the column runs from x = 0 to its final
// status without leaving the workgroup; at most maxit iterations.
template <int Q>
__device__ __forceinline__ void solve_column(const TladArgs &a, const TladGeom &g, int c, unsigned char *smraw,
                                             double *s_red, double *s_t) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const PcgCols &pc = a.pcg;
    const int n = a.n;
    const long long cn = (long long)c * n;
    double *x = pc.x + cn, *r = pc.r + cn, *z = pc.z + cn;
    const double *b = pc.b + (long long)pc.members[c] * n;
    // x = 0, r = b, ||b||; history row
    double bb = 0.0;
    for (int i = tid; i < n; i += nthr) {
        const double v = b[i];
        x[i] = 0.0;
        r[i] = v;
        bb += v * v;
    }
    bb = block_sum(bb, s_red, nthr >> 6);
    if (pc.hist)
        for (int i = tid; i < pc.hist_cap; i += nthr)
            pc.hist[(long long)c * pc.hist_cap + i] = i == 0 ? 0.0 : __builtin_nan("");
    if (tid == 0) {
        pc.scal[4 * c + 1] = sqrt(bb);
        pc.scal[4 * c + 2] = bb > 0 ? 1.0 : 0.0;
        pc.status[c] = bb > 0 ? COL_RUNNING : EDA_MEMBER_CONVERGED;
        pc.iters[c] = 0;
    }
    __syncthreads();
    if (!(bb > 0)) return;
    // a sketch whose Cholesky failed gives no LMP: plain CG for its members
    const bool lmp = pc.lmp_k > 0 && !(pc.lmp_info && pc.lmp_info[0]);
    if (lmp) {
        lmp_column(pc, n, r, z, reinterpret_cast<double *>(smraw), s_t, nthr >> 6);
    } else {
        for (int i = tid; i < n; i += nthr) z[i] = r[i];
        __syncthreads();
    }
    int st = COL_RUNNING;
    for (int it = 1; it <= pc.maxit; it++) {
        tlad_column<double, Q, TLAD_PCG, (Q <= 7)>(a, g, c, it, it == 1, smraw);
        __syncthreads();
        st = pc.status[c];
        __syncthreads();
        if (st != COL_RUNNING) break;
        if (lmp) {
            lmp_column(pc, n, r, z, reinterpret_cast<double *>(smraw), s_t, nthr >> 6);
        } else {
            for (int i = tid; i < n; i += nthr) z[i] = r[i];
            __syncthreads();
        }
    }
    if (st == COL_RUNNING) {
        // iteration limit: the breakdown test on r^T z that the next
        // iteration would make, then not-converged
        double rz = 0.0;
        for (int i = tid; i < n; i += nthr) rz += r[i] * z[i];
        rz = block_sum(rz, s_red, nthr >> 6);
        if (tid == 0) pc.status[c] = (pc.maxit > 0 && !(rz > 0.0 && isfinite(rz))) ? EDA_MEMBER_BREAKDOWN
                                                                                   : EDA_MEMBER_NOT_CONVERGED;
    }
    __syncthreads();
}

// One sketch column of problem p: y_j = A gamma_j on the control trajectory;
// the workgroup that completes the problem's last column then runs its last
// Nystrom pass (shifts on the device when a Cholesky fails), which leaves the
// LMP.  Every wave releases its stores at device scope before the count, and
// the finishing workgroup acquires before it reads the other workgroups'
// columns.
template <int Q>
__device__ __forceinline__ void sketch_column(const SolveSketch &sk, int p, int j, const TladGeom &g,
                                              unsigned char *smraw, nys::RedoLds &L, double *nrm, int &s_flag) {
    const int tid = threadIdx.x;
    tlad_column<double, Q, TLAD_HV>(sk.hv[p], g, j, 0, 0, smraw);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    const RedoJob &J = sk.core[p];
    if (tid == 0) s_flag = __hip_atomic_fetch_add(sk.done + p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == J.l - 1;
    __syncthreads();
    const int last = s_flag;
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    nys::nystrom_redo(J, reinterpret_cast<double *>(smraw), L, nrm);
    __syncthreads();
}

// The sketches of a batch in one persistent launch: the workgroups take
// (problem, sketch column) tasks from one list, from its end (the list holds
// the classes in increasing n, so the longest columns go first); the
// workgroup that finishes a problem's last column runs its last Nystrom pass.
// Every geometry has blockDim.x / 64 waves.  Every workgroup exits once the
// list is exhausted.
__global__ __launch_bounds__(512) void k_sketch(const TladGeom *__restrict__ geoms, const SolveTask *__restrict__ tasks,
                                                int ntasks, int *counter, SolveSketch sk) {
    extern __shared__ __align__(16) unsigned char smraw[];
    __shared__ int s_task;
    __shared__ double s_t[128];
    __shared__ nys::RedoLds s_redo;
    for (;;) {
        if (threadIdx.x == 0) {
            const int u = atomicAdd(counter, 1);
            s_task = u < ntasks ? ntasks - 1 - u : -1;
        }
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t < 0) break;
        const SolveTask task = tasks[t];
        const TladGeom g = geoms[task.prob];
        switch (g.q) {
            case 2: sketch_column<2>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 3: sketch_column<3>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 4: sketch_column<4>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 5: sketch_column<5>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 6: sketch_column<6>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 7: sketch_column<7>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            case 8: sketch_column<8>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
            default: sketch_column<9>(sk, task.prob, task.col, g, smraw, s_redo, s_t, s_task); break;
        }
    }
}

// Persistent LMP-PCG over a task list, one solve_column per task.  One launch
// serves problems of every n: geoms[p] is problem p's geometry (all with
// blockDim.x / 64 waves), and the workgroup takes the matching points-per-lane
// instance for each task.  The list is cut into SOLVE_QUEUES queues, queue q =
// tasks [qoff[q], qoff[q+1]) with its own counter.  Workgroups are dispatched
// to the XCDs round-robin, so workgroup b starts on queue b mod SOLVE_QUEUES
// and the columns one XCD runs at a time come from few problems, whose S then
// stays in that XCD's L2 for the in-kernel LMP; a workgroup whose queue is
// empty takes tasks from the next queues in turn.  Every workgroup exits once
// it has found all queues empty.
__global__ __launch_bounds__(512) void k_solve(const TladArgs *__restrict__ probs, const TladGeom *__restrict__ geoms,
                                               const SolveTask *__restrict__ tasks, const int *__restrict__ qoff,
                                               int *counters) {
    extern __shared__ __align__(16) unsigned char smraw[];
    __shared__ int s_task;
    __shared__ double s_red[16];
    __shared__ double s_t[128];
    const int tid = threadIdx.x;
    int q = blockIdx.x % SOLVE_QUEUES, left = SOLVE_QUEUES;  // meaningful in thread 0 only
    for (;;) {
        if (tid == 0) {
            int t = -1;
            while (left > 0) {
                const int lo = qoff[q], hi = qoff[q + 1];
                if (lo < hi) {
                    const int u = lo + atomicAdd(counters + q, 1);
                    if (u < hi) {
                        t = u;
                        break;
                    }
                }
                q = (q + 1) % SOLVE_QUEUES;
                left--;
            }
            s_task = t;
        }
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t < 0) break;
        const SolveTask task = tasks[t];
        const TladArgs &a = probs[task.prob];
        const TladGeom g = geoms[task.prob];
        switch (g.q) {
            case 2: solve_column<2>(a, g, task.col, smraw, s_red, s_t); break;
            case 3: solve_column<3>(a, g, task.col, smraw, s_red, s_t); break;
            case 4: solve_column<4>(a, g, task.col, smraw, s_red, s_t); break;
            case 5: solve_column<5>(a, g, task.col, smraw, s_red, s_t); break;
            case 6: solve_column<6>(a, g, task.col, smraw, s_red, s_t); break;
            case 7: solve_column<7>(a, g, task.col, smraw, s_red, s_t); break;
            case 8: solve_column<8>(a, g, task.col, smraw, s_red, s_t); break;
            default: solve_column<9>(a, g, task.col, smraw, s_red, s_t); break;
        }
    }
}

// Gamma columns of every problem (block p: problem p) and the per-call resets
// of the sketch launch.
__global__ void k_solve_prelude(int np, const TladArgs *__restrict__ probs, SolveSketch sk) {
    const int p = blockIdx.x;
    if (p >= np) return;
    const RedoJob &J = sk.core[p];
    const int n = J.n;
    const double *b = probs[p].pcg.b;
    double *phi = const_cast<double *>(sk.hv[p].V);
    for (long long idx = threadIdx.x; idx < (long long)n * J.l; idx += blockDim.x) {
        const int i = (int)(idx % n), j = (int)(idx / n);
        phi[idx] = b[(long long)(j + 1) * n + i] - b[i];
    }
    if (threadIdx.x == 0) sk.done[p] = 0;
}

// out[t] = iterations task t took in the last persistent solve, and
// out[ntasks + t] = its final status.
__global__ void k_task_iters(int ntasks, const TladArgs *__restrict__ probs, const SolveTask *__restrict__ tasks,
                             int32_t *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntasks) {
        const PcgCols &pc = probs[tasks[t].prob].pcg;
        out[t] = pc.iters[tasks[t].col];
        out[ntasks + t] = pc.status[tasks[t].col];
    }
}

// Hessian products of (problem, column) tasks, one workgroup per task.
template <int Q>
__global__ __launch_bounds__(512) void k_hv_multi(const TladArgs *__restrict__ probs,
                                                  const SolveTask *__restrict__ tasks, TladGeom g) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const SolveTask t = tasks[blockIdx.x];
    tlad_column<double, Q, TLAD_HV>(probs[t.prob], g, t.col, 0, 0, smraw);
}


// ---------------- wave pieces with halo exchange ----------------
// Every wave owns segment [lo, hi) of one column and runs its TL/AD windows
// alone (no workgroup barrier after the start).  At each exchange it publishes
// the first and last E of its owned values, stores them behind a completed
// vector-memory wait, raises its flag to the phase number, waits for both
// neighbours' flags and reads their edges into its window halos.  The reads
// bypass the CU's L1 (device-scope loads): the same addresses carry new values
// every other phase.  Edges are double-buffered by phase parity: a wave
// rewrites a parity only after it has read the neighbours' next phase, which
// they publish after reading this one.

// XCC_ID hardware register (id 20, bits 3:0): the XCD a wave runs on.
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)); }

// Banded circulant product from a slice: out[q] = sum_m taps[m] us[l Q + q + m]
// for this lane l (us: 64 Q + W - 1 values); a circular register buffer of Q
// values keeps one LDS read per tap, the taps in ascending order.
template <int Q>
__device__ __forceinline__ void band_slice(const double *us, const double *taps, int W, double (&out)[Q]) {
    const double *u = us + (threadIdx.x & 63) * Q;
    double B[Q];
#pragma unroll
    for (int j = 0; j < Q; j++) B[j] = u[j];
#pragma unroll
    for (int q = 0; q < Q; q++) out[q] = 0.0;
    int m0 = 0;
    for (; m0 + Q <= W; m0 += Q) {
#pragma unroll
        for (int mm = 0; mm < Q; mm++) {
            const double t = taps[m0 + mm];
#pragma unroll
            for (int q = 0; q < Q; q++) out[q] += t * B[(mm + q) % Q];
            B[mm] = u[m0 + mm + Q];
        }
    }
#pragma unroll
    for (int mm = 0; mm < Q - 1; mm++) {
        if (m0 + mm < W) {
            const double t = taps[m0 + mm];
#pragma unroll
            for (int q = 0; q < Q; q++) out[q] += t * (mm + q < Q ? B[mm + q] : u[m0 + mm + q]);
        }
    }
}

// Raises this slot's flag to phase `ph` after the wave's earlier stores
// completed, then waits for the neighbours' flags to reach it.  A wait that
// gives up sets the error word and the wave's `failed`, after which the wave
// no longer waits (its results are void; the host reports the error).
__device__ __forceinline__ void xch_sync(const XchArgs &xa, int slot, const XSlot &sl, int ph, bool &failed) {
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const unsigned long long want = xa.epoch + (unsigned long long)ph + 1ull;
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(xa.flags + slot, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (failed) return;
    if (!xch_wait(xa.flags + sl.left, xa.flags + sl.right, want, xa.spin_max)) {
        failed = true;
        if ((threadIdx.x & 63) == 0) __hip_atomic_store(xa.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Edge exchange of window values v (window position j = l Q + q, owned index
// j - hl in [0, seg)): publish, sync, and fill the halo positions from the
// neighbours' edges (left: its last E values; right: its first E, zeros beyond).
template <int Q>
__device__ __forceinline__ void xch_edges(const XchArgs &xa, int slot, const XSlot &sl, int seg, int hl, int ph,
                                          bool &failed, double (&v)[Q]) {
    const int lane = threadIdx.x & 63, E = xa.E;
    const long long par = ph & 1;
    double *mine = xa.edges + ((long long)slot * 2 + par) * 2 * E;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int o = lane * Q + q - hl;
        if (o >= 0 && o < E) mine[o] = v[q];
        if (o >= seg - E && o < seg) mine[E + o - (seg - E)] = v[q];
    }
    xch_sync(xa, slot, sl, ph, failed);
    const double *le = xa.edges + ((long long)sl.left * 2 + par) * 2 * E + E;
    const double *re = xa.edges + ((long long)sl.right * 2 + par) * 2 * E;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int o = lane * Q + q - hl;
        if (o < 0) v[q] = load_dev(le + E + o);
        else if (o >= seg) v[q] = o - seg < E ? load_dev(re + (o - seg)) : 0.0;
    }
}

// The Hessian part of PCG iteration a.pcg.it on the wave's segment (what
// TLAD_SPLIT computes on a ring piece): r^T z from the row-block partials, p =
// z + beta p (new p written for the owned states), V = U_B p over the TL
// window, TL, AD, U_B lambda_0 + p at the owned states into q and the
// segment's part of p^T (I + A) p.
template <int Q>
__global__ __launch_bounds__(512) void k_tlad_x(TladArgs a, XchArgs xa, SplitCols sc) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, N = a.N, tb = xa.tb;
    const int W = a.band_hi - a.band_lo + 1;
    const int UL = 64 * Q + W - 1;
    // LDS (xch_lds_doubles): taps (W, rounded up to even), then per wave: the
    // trajectory window (64 Q), the U_B slice (UL + Q, rounded up to even: the
    // product's register buffer reads up to Q - 1 values past the slice) and
    // the observation indices (64 Q ints)
    double *taps = reinterpret_cast<double *>(smraw);
    const int per_wave = 64 * Q + ((UL + Q + 1) & ~1) + 32 * Q;  // in doubles
    double *xw = taps + ((W + 1) & ~1) + (long long)wave * per_wave;
    double *u = xw + 64 * Q;
    int *qi = reinterpret_cast<int *>(u + ((UL + Q + 1) & ~1));
    for (int m = threadIdx.x; m < W; m += blockDim.x) {
        const int o = a.band_hi - m;
        taps[m] = a.ubrow[o < 0 ? -o : o];
    }
    // Workgroups are dealt to the XCDs in turn from a starting XCD that varies
    // between launches: the workgroup takes the virtual index whose low three
    // bits are its XCD (a permutation of the launch's indices under that
    // dealing) and claims it for this launch; a second claim of one index means
    // another placement, reported (its neighbours' waits then give up).
    __shared__ int s_vb;
    if (threadIdx.x == 0) {
        const int vb = (int)(blockIdx.x & ~7u) | (xcc_id() & 7);
        const unsigned long long prev =
            __hip_atomic_exchange(xa.claim + vb, xa.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == xa.epoch) __hip_atomic_store(xa.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_vb = vb;
    }
    __syncthreads();  // the last workgroup barrier: the waves are independent from here on

    const int slot = s_vb * 8 + wave;
    const int m = sc.count > 0 ? sc.count : a.nb;
    const XSlot sl = xch_slot(slot, m, xa.grid, xa.max_seg);
    if (sl.li < 0) return;
    const int c = sc.count > 0 ? sc.col[sl.li] : sl.li;
    if (a.pcg.status[c] != COL_RUNNING) return;
    const int lo = (int)((long long)sl.seg * n / sl.nseg), hi = (int)((long long)(sl.seg + 1) * n / sl.nseg);
    const int seg = hi - lo;
    const long long cn = (long long)c * n;
    const int first = a.pcg.first;

    // r^T z: the row blocks' partial sums in block order
    double rz = 0.0;
    {
        double v[LMP_RB_MAX];
#pragma unroll
        for (int b = 0; b < LMP_RB_MAX; b++) v[b] = b < xa.nrb ? xa.rz_part[(long long)b * xa.rz_ld + c] : 0.0;
#pragma unroll
        for (int b = 0; b < LMP_RB_MAX; b++) rz += v[b];
    }
    double beta = 0.0;
    if (!first) {
        if (!(rz > 0.0) || !isfinite(rz)) {
            if (lane == 0 && sl.seg == 0) a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;
            return;
        }
        beta = rz / a.pcg.scal[4 * c];
    }
    if (lane == 0 && sl.seg == 0) {
        a.pcg.scal[4 * c + 3] = rz;  // rho of this iteration, for the update
        xa.nseg[c] = sl.nseg;
    }

    // p over the U_B slice of the TL window (slice j: state w0 - band_hi + j)
    const int hl_tl = 8 * tb, hl_ad = 4 * tb + 8;
    const int w0 = lo - hl_tl;
    const double *z = a.pcg.z + cn, *pold = a.pcg.p + cn;
    double *pout = a.pcg.p_out + cn;
    for (int j = lane; j < UL; j += 64) {
        int st = (w0 - a.band_hi + j) % n;
        st = st < 0 ? st + n : st;
        const double v = first ? z[st] : z[st] + beta * pold[st];
        u[j] = v;
        const int o = j - a.band_hi - hl_tl;
        if (o >= 0 && o < seg) pout[st] = v;
    }
    __asm__ volatile("" ::: "memory");
    const double *trajm = a.trajx + (long long)a.pcg.members[c] * a.trajx_stride + a.pad_l;
    const StepK<double> K{a.h, a.dt, a.dt6, a.dt3, a.h * a.F};
    unsigned ownm;
    int ph = 0;
    bool failed = false;

    // ---------------- TL forward run ----------------
    prefetch_window<Q>(trajm + w0, xw);
    window<Q>(a, w0, lo, hi, true, ownm, qi, n, 0);
    double dx[Q];
    band_slice<Q>(u, taps, W, dx);
    double *obs = a.obs + (long long)c * a.nt * a.nv;
    for (int s0 = 0; s0 < N; s0 += tb) {
        if (s0 > 0) xch_edges<Q>(xa, slot, sl, seg, hl_tl, ph++, failed, dx);
        const int s1 = min(N, s0 + tb);
        for (int s = s0; s < s1; s++) {
            if (s > 0 && s % a.obs_dt == 0)
                store_obs<double, Q>(obs + (long long)(s / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
            tl_step<double, Q, true>(K, xw, trajm + (long long)min(s + 1, N - 1) * a.ext_len + w0, s + 1 < N, dx);
        }
    }
    if (N % a.obs_dt == 0) store_obs<double, Q>(obs + (long long)(N / a.obs_dt - 1) * a.nv, qi, dx, a.inv_s2);
    // the neighbours' observed increments are complete
    xch_sync(xa, slot, sl, ph++, failed);

    // ---------------- AD backward run ----------------
    const int w0a = lo - hl_ad;
    prefetch_window<Q>(trajm + (long long)(N - 1) * a.ext_len + w0a, xw);
    window<Q>(a, w0a, lo, hi, false, ownm, qi, n, 0);
    {
        // forcing only where it can reach the owned outputs (the AD cone and the
        // stage states' reach): the immediate neighbours' owned points
        const int jmax = hl_ad + seg + 8 * tb + 8;
#pragma unroll
        for (int q = 0; q < Q; q++)
            if (lane * Q + q >= jmax) qi[q * 64 + lane] = -1;
    }
    double lam[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) lam[q] = 0.0;
    for (int s_hi = N; s_hi >= 1; s_hi -= tb) {
        if (s_hi < N) xch_edges<Q>(xa, slot, sl, seg, hl_ad, ph++, failed, lam);
        const int s_lo = max(0, s_hi - tb);
        for (int s = s_hi; s > s_lo; s--) {
            if (s % a.obs_dt == 0) {
                const double *f = obs + (long long)(s / a.obs_dt - 1) * a.nv;
#pragma unroll
                for (int q = 0; q < Q; q++) {
                    const int oi = qi[q * 64 + lane];
                    if (oi >= 0) lam[q] += load_dev(f + oi);
                }
            }
            ad_step<double, Q, true>(K, xw, trajm + (long long)max(s - 2, 0) * a.ext_len + w0a, s >= 2, lam);
        }
    }

    // ---------------- U_B on the way out: slice j = state w0a - band_hi + j ----------------
    {
        const int E = xa.E;
        const long long par = ph & 1;
        double *mine = xa.edges + ((long long)slot * 2 + par) * 2 * E;
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int o = lane * Q + q - hl_ad;
            if (o >= 0 && o < E) mine[o] = lam[q];
            if (o >= seg - E && o < seg) mine[E + o - (seg - E)] = lam[q];
            if (o >= 0 && o < seg) u[lane * Q + q + a.band_hi] = lam[q];
        }
        xch_sync(xa, slot, sl, ph++, failed);
        const double *le = xa.edges + ((long long)sl.left * 2 + par) * 2 * E + E;
        const double *re = xa.edges + ((long long)sl.right * 2 + par) * 2 * E;
        for (int t = lane; t < a.band_hi; t += 64) {
            u[hl_ad + t] = load_dev(le + E - a.band_hi + t);
            u[hl_ad + a.band_hi + seg + t] = load_dev(re + t);
        }
    }
    __asm__ volatile("" ::: "memory");
    double y[Q];
    band_slice<Q>(u, taps, W, y);
    double pq = 0.0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int o = lane * Q + q - hl_ad;
        if (o >= 0 && o < seg) {
            int st = lo + o;
            st = st >= n ? st - n : st;
            const double pv = first ? z[st] : z[st] + beta * pold[st];
            const double yq = y[q] + pv;
            pq += pv * yq;
            a.pcg.q[cn + st] = yq;
        }
    }
    for (int off = 32; off > 0; off >>= 1) pq += __shfl_down(pq, off, 64);
    if (lane == 0) {
        a.pcg.pq_part[(long long)c * XCH_SEG_MAX + sl.seg] = pq;
        if (failed) a.pcg.status[c] = EDA_MEMBER_BREAKDOWN;  // void results: the member stops
    }
}

template <int Q>
hipError_t launch_x_q(hipStream_t s, const TladArgs &a, const XchArgs &x, const SplitCols &sc, size_t lds) {
    hipLaunchKernelGGL(k_tlad_x<Q>, dim3(x.grid), dim3(512), lds, s, a, x, sc);
    return hipGetLastError();
}

template <typename T, int Q>
size_t lds_bytes(const TladArgs &a, const TladGeom &g, int mode) {
    const bool split = mode == TLAD_SPLIT || mode == TLAD_SPLIT_HV || mode == TLAD_SPLIT_SH || mode == TLAD_SPLIT_HV_SH;
    const size_t R = split ? (size_t)a.ring : (size_t)a.n;
    size_t b = sizeof(T) * 2 * R + (sizeof(int) + sizeof(double)) * (size_t)g.waves * 64 * Q;
    if (mode == TLAD_HV || mode == TLAD_PCG || split)
        b += sizeof(double) * (R + (size_t)(a.band_hi - a.band_lo + 1) + 16);
    return b;
}

template <typename T, int Q>
hipError_t launch_q(hipStream_t s, const TladArgs &a, const TladGeom &g, int mode, const SplitCols *sc) {
    const size_t lds = lds_bytes<T, Q>(a, g, mode);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 block(64 * g.waves);
    switch (mode) {
        case TLAD_RAW: hipLaunchKernelGGL((k_tlad<T, Q, TLAD_RAW>), dim3(a.nb), block, lds, s, a, g); break;
        case TLAD_ADJ: hipLaunchKernelGGL((k_tlad<T, Q, TLAD_ADJ>), dim3(a.nb), block, lds, s, a, g); break;
        case TLAD_HV: hipLaunchKernelGGL((k_tlad<T, Q, TLAD_HV>), dim3(a.nb), block, lds, s, a, g); break;
        case TLAD_PCG: hipLaunchKernelGGL((k_tlad<T, Q, TLAD_PCG>), dim3(a.nb), block, lds, s, a, g); break;
        case TLAD_SPLIT: {
            if (!std::is_same<T, double>::value) return hipErrorInvalidValue;
            SplitCols all{};
            const SplitCols &cs = sc ? *sc : all;
            const int m = cs.count > 0 ? cs.count : a.nb;
            hipLaunchKernelGGL(k_tlad_split<Q>, dim3(m * a.pieces), block, lds, s, a, g, cs);
            break;
        }
        case TLAD_SPLIT_SH: {
            if (!std::is_same<T, double>::value) return hipErrorInvalidValue;
            SplitCols all{};
            const SplitCols &cs = sc ? *sc : all;
            const int m = cs.count > 0 ? cs.count : a.nb;
            hipLaunchKernelGGL(k_tlad_split_sh<Q>, dim3(m * a.pieces), block, lds, s, a, g, cs);
            break;
        }
        case TLAD_SPLIT_HV:
            hipLaunchKernelGGL((k_tlad_split_hv<T, Q>), dim3(a.nb * a.pieces), block, lds, s, a, g);
            break;
        case TLAD_SPLIT_HV_SH:
            hipLaunchKernelGGL((k_tlad_split_hv_sh<T, Q>), dim3(a.nb * a.pieces), block, lds, s, a, g);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(hipStream_t s, const TladArgs &a, const TladGeom &g, int mode, const SplitCols *sc) {
    switch (g.q) {
        case 2: return launch_q<T, 2>(s, a, g, mode, sc);
        case 3: return launch_q<T, 3>(s, a, g, mode, sc);
        case 4: return launch_q<T, 4>(s, a, g, mode, sc);
        case 5: return launch_q<T, 5>(s, a, g, mode, sc);
        case 6: return launch_q<T, 6>(s, a, g, mode, sc);
        case 7: return launch_q<T, 7>(s, a, g, mode, sc);
        case 8: return launch_q<T, 8>(s, a, g, mode, sc);
        case 9: return launch_q<T, 9>(s, a, g, mode, sc);
        default: return hipErrorInvalidValue;
    }
}

template <int Q>
hipError_t launch_hv_multi_q(hipStream_t s, const TladArgs *d_probs, const SolveTask *d_tasks, int ntasks,
                             const TladGeom &g, size_t lds) {
    hipLaunchKernelGGL(k_hv_multi<Q>, dim3(ntasks), dim3(64 * g.waves), lds, s, d_probs, d_tasks, g);
    return hipGetLastError();
}

// static LDS of k_solve (task id, reduction slots, LMP coefficients)
constexpr size_t SOLVE_STATIC_LDS = sizeof(int) + 16 * sizeof(double) + 128 * sizeof(double) + 64;
// static LDS of k_sketch (task id, norms, pass scratch)
constexpr size_t SKETCH_STATIC_LDS = sizeof(int) + 128 * sizeof(double) + sizeof(nys::RedoLds) + 64;

}  // namespace

size_t tlad_lds_bytes(const TladArgs &a, const TladGeom &g, int mode) {
    switch (g.q) {
        case 2: return lds_bytes<double, 2>(a, g, mode);
        case 3: return lds_bytes<double, 3>(a, g, mode);
        case 4: return lds_bytes<double, 4>(a, g, mode);
        case 5: return lds_bytes<double, 5>(a, g, mode);
        case 6: return lds_bytes<double, 6>(a, g, mode);
        case 7: return lds_bytes<double, 7>(a, g, mode);
        case 8: return lds_bytes<double, 8>(a, g, mode);
        case 9: return lds_bytes<double, 9>(a, g, mode);
        default: return (size_t)-1;
    }
}

hipError_t launch_solve(hipStream_t s, const TladArgs *d_probs, const TladGeom *d_geoms, const SolveTask *d_tasks,
                        int ntasks, const int *d_qoff, int *d_counters, int waves, size_t lds, int grid) {
    if (ntasks <= 0) return hipSuccess;
    if (grid <= 0 || (waves != 1 && waves != 2 && waves != 4 && waves != 8) || lds + SOLVE_STATIC_LDS > 160 * 1024)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_solve, dim3(grid), dim3(64 * waves), lds, s, d_probs, d_geoms, d_tasks, d_qoff, d_counters);
    return hipGetLastError();
}

hipError_t launch_solve_prelude(hipStream_t s, int np, const TladArgs *d_probs, const SolveSketch &sk) {
    if (np <= 0 || !sk.hv) return hipSuccess;
    hipLaunchKernelGGL(k_solve_prelude, dim3(np), dim3(256), 0, s, np, d_probs, sk);
    return hipGetLastError();
}

hipError_t launch_sketch(hipStream_t s, const TladGeom *d_geoms, const SolveTask *d_tasks, int ntasks, int *d_counter,
                         int waves, size_t lds, int grid, const SolveSketch &sk) {
    if (ntasks <= 0) return hipSuccess;
    if (grid <= 0 || (waves != 1 && waves != 2 && waves != 4 && waves != 8) || lds + SKETCH_STATIC_LDS > 160 * 1024)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sketch, dim3(grid), dim3(64 * waves), lds, s, d_geoms, d_tasks, ntasks, d_counter, sk);
    return hipGetLastError();
}

int sketch_blocks_per_cu(int waves, size_t lds) {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sketch, 64 * waves, lds) == hipSuccess ? nb : 0;
}

hipError_t launch_hv_multi(hipStream_t s, const TladArgs *d_probs, const SolveTask *d_tasks, int ntasks,
                           const TladGeom &g, size_t lds) {
    if (ntasks <= 0) return hipSuccess;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    switch (g.q) {
        case 2: return launch_hv_multi_q<2>(s, d_probs, d_tasks, ntasks, g, lds);
        case 3: return launch_hv_multi_q<3>(s, d_probs, d_tasks, ntasks, g, lds);
        case 4: return launch_hv_multi_q<4>(s, d_probs, d_tasks, ntasks, g, lds);
        case 5: return launch_hv_multi_q<5>(s, d_probs, d_tasks, ntasks, g, lds);
        case 6: return launch_hv_multi_q<6>(s, d_probs, d_tasks, ntasks, g, lds);
        case 7: return launch_hv_multi_q<7>(s, d_probs, d_tasks, ntasks, g, lds);
        case 8: return launch_hv_multi_q<8>(s, d_probs, d_tasks, ntasks, g, lds);
        case 9: return launch_hv_multi_q<9>(s, d_probs, d_tasks, ntasks, g, lds);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_task_iters(hipStream_t s, int ntasks, const TladArgs *d_probs, const SolveTask *d_tasks,
                             int32_t *d_out) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_task_iters, dim3((ntasks + 255) / 256), dim3(256), 0, s, ntasks, d_probs, d_tasks, d_out);
    return hipGetLastError();
}

int solve_blocks_per_cu(int waves, size_t lds) {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve, 64 * waves, lds) == hipSuccess ? nb : 0;
}

// Geometry: waves per workgroup, owned segment per wave, points per lane and
// the time-block length, with halos hl_tl = 8 TB (TL cone: 8 left, 4 right per
// step) and hl_ad = 4 TB + 8 (AD cone: 4 left, 8 right per step, plus the
// recomputed stage states' fixed reach), requiring S + 12 TB + 16 <= 64 Q.
TladGeom tlad_geometry(int n, int waves_hint, int tb_hint) {
    TladGeom g{};
    int W = waves_hint > 0 ? waves_hint : (n >= 2048 ? 8 : n >= 512 ? 4 : n >= 128 ? 2 : 1);
    g.waves = W;
    g.S = (n + W - 1) / W;
    int Q = 2;
    while (64 * Q < g.S + 12 * 2 + 16) Q++;
    g.q = Q;
    g.tb = (64 * Q - g.S - 16) / 12;
    if (tb_hint > 0 && tb_hint < g.tb) g.tb = tb_hint;
    g.hl_tl = 8 * g.tb;
    g.hl_ad = 4 * g.tb + 8;
    return g;
}

bool tlad_waves_ok(int n, int waves) {
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return false;
    const TladGeom g = tlad_geometry(n, waves);
    return g.q <= 9 && g.tb >= 1;
}

int tlad_split_halo(int N, int band_hi) { return 12 * N + 2 * band_hi; }

int tlad_split_ring(int n, int N, int band_hi, int pieces) {
    if (pieces < 2) return n;
    const int R = (n + pieces - 1) / pieces + 2 * tlad_split_halo(N, band_hi);
    if (R > n) return 0;
    const TladGeom g = tlad_geometry(R, 0);
    return (g.q <= 9 && g.tb >= 1) ? R : 0;
}

int tlad_split_halo_sh(int N, int band_hi) { return 8 * N + band_hi; }

int tlad_split_ring_sh(int n, int N, int band_hi, int pieces) {
    if (pieces < 2 || pieces > SPLIT_PMAX || n / pieces < 8 * N + band_hi) return 0;
    const int R = (n + pieces - 1) / pieces + 12 * N + 2 * band_hi;
    if (R > n) return 0;
    const TladGeom g = tlad_geometry(R, 0);
    return (g.q <= 9 && g.tb >= 1) ? R : 0;
}

// Reach of the windows on a ring of R points over every geometry the
// launchers accept (any accepted wave count, any time-block length up to its
// maximum): windows start up to *left points before ring position 0 and end up
// to *right points after position R.
static void ring_reach(int R, int *left, int *right) {
    int pl = 0, pr = 0;
    for (int W = 1; W <= 8; W *= 2) {
        if (!tlad_waves_ok(R, W)) continue;
        const TladGeom g0 = tlad_geometry(R, W);
        for (int tb = 1; tb <= g0.tb; tb++) {
            const TladGeom g = tlad_geometry(R, W, tb);
            const int hmax = g.hl_tl > g.hl_ad ? g.hl_tl : g.hl_ad;
            const int hmin = g.hl_tl < g.hl_ad ? g.hl_tl : g.hl_ad;
            // window of wave w: [w S - hl, w S - hl + 64 Q)
            const int right = (g.waves - 1) * g.S - hmin + 64 * g.q - R;
            if (hmax > pl) pl = hmax;
            if (right > pr) pr = right;
        }
    }
    *left = pl;
    *right = pr;
}

void tlad_pads(int n, int *pad_l, int *pad_r) { ring_reach(n, pad_l, pad_r); }

// Split rings: ring position 0 is state lo - H, so windows reach H + left
// below state 0 (first piece) and up to the last ring's end plus its reach
// above state n (last piece).
void tlad_pads_split(int n, int N, int band_hi, int *pad_l, int *pad_r) {
    int pl, pr;
    tlad_pads(n, &pl, &pr);
    const int H = tlad_split_halo(N, band_hi);
    for (int P = 2; P <= SPLIT_PMAX; P++) {
        const int R = tlad_split_ring(n, N, band_hi, P);
        if (R == 0) continue;
        int l, r;
        ring_reach(R, &l, &r);
        const int lo_last = (int)((long long)(P - 1) * n / P);
        const int left = H + l, right = (lo_last - H) + R + r - n;
        if (left > pl) pl = left;
        if (right > pr) pr = right;
    }
    // rings of pieces sharing the observed increments: the TL ring starts
    // 8 N + band_hi states before the piece, the AD ring 4 N states later
    const int Hs = tlad_split_halo_sh(N, band_hi);
    for (int P = 2; P <= SPLIT_PMAX; P++) {
        const int R = tlad_split_ring_sh(n, N, band_hi, P);
        if (R == 0) continue;
        int l, r;
        ring_reach(R, &l, &r);
        const int lo_last = (int)((long long)(P - 1) * n / P);
        const int left = Hs + l, right = (lo_last - Hs + 4 * N) + R + r - n;
        if (left > pl) pl = left;
        if (right > pr) pr = right;
    }
    *pad_l = pl;
    *pad_r = pr;
}

// Dynamic LDS of k_tlad_x (see its layout), at least XCH_LDS_MIN so that one
// workgroup takes a CU.
static size_t xch_lds_bytes(int Q, int W) {
    const size_t UL = 64 * (size_t)Q + W - 1;
    const size_t per_wave = 64 * (size_t)Q + ((UL + Q + 1) & ~(size_t)1) + 32 * (size_t)Q;
    const size_t b = sizeof(double) * ((((size_t)W + 1) & ~(size_t)1) + 8 * per_wave);
    return b > XCH_LDS_MIN ? b : XCH_LDS_MIN;
}

XchPlan xch_plan(int n, int N, int band_hi, int m, int grid, int pad_l, int pad_r) {
    XchPlan P{};
    grid = (grid > XCH_GRID_MAX ? XCH_GRID_MAX : grid) & ~7;
    if (m < 1 || grid < 8 || N < 1) return P;
    for (int cap = XCH_SEG_MAX; cap >= 2; cap--) {
        int nmin = 1 << 30, nmax = 0;
        for (int x = 0; x < 8; x++) {
            const int slots = ((grid - x + 7) / 8) * 8;
            const int cols = m > x ? (m - x + 7) / 8 : 0;
            if (cols == 0) continue;
            int base = slots / cols, extra = slots - base * cols;
            if (base >= cap) {
                base = cap;
                extra = 0;
            }
            if (base < nmin) nmin = base;
            const int hi = extra > 0 ? base + 1 : base;
            if (hi > nmax) nmax = hi;
        }
        if (nmin < 2) return P;  // more columns than the slots can take in pairs
        const int seg_max = (n + nmin - 1) / nmin, seg_min = n / nmax;
        if (64 * 8 < seg_max + 12 + 16) return P;  // longer segments only with fewer segments per column
        // points per lane: a wider window allows longer time blocks (fewer
        // exchanges) at more work per step; estimated cycles of one launch:
        // N steps of about 66 Q + 136 VALU instructions (TL + AD, two waves
        // per SIMD at 4 cycles each) and about 2800 cycles per exchange
        long long best = -1;
        for (int Q = 2; Q <= 8; Q++) {
            if (64 * Q < seg_max + 12 + 16) continue;
            int tb = (64 * Q - seg_max - 16) / 12;
            if (tb > XCH_TB_MAX) tb = XCH_TB_MAX;
            if (tb > N) tb = N;
            while (tb > 1 && 8 * tb + 8 > seg_min) tb--;
            const int E = 8 * tb + 8 > band_hi ? 8 * tb + 8 : band_hi;
            if (E > XCH_E_MAX || seg_min < E) continue;
            // windows inside the padded rows: TL from lo - 8 tb, AD from lo - 4 tb - 8, 64 Q long
            const int hl_ad = 4 * tb + 8;
            const int reach_r = 64 * Q - (8 * tb < hl_ad ? 8 * tb : hl_ad) - seg_min;
            if (8 * tb > pad_l || hl_ad > pad_l || reach_r > pad_r) continue;
            const long long est = (long long)N * (66 * Q + 136) * 8 + (2LL * ((N + tb - 1) / tb) + 2) * 2800;
            if (best < 0 || est < best) {
                best = est;
                P.ok = 1;
                P.q = Q;
                P.tb = tb;
                P.E = E;
                P.max_seg = cap;
                P.grid = grid;
            }
        }
        if (P.ok) return P;  // else segments too short for the edges: fewer of them
    }
    return P;
}

hipError_t launch_tlad_x(hipStream_t s, const TladArgs &a, const XchArgs &x, const XchPlan &pl, const SplitCols &sc) {
    const int W = a.band_hi - a.band_lo + 1;
    if (!pl.ok || x.grid != pl.grid || x.tb != pl.tb || x.E != pl.E || x.max_seg != pl.max_seg ||
        W != 2 * a.band_hi + 1 || a.band_hi > x.E || sc.count < 0 || sc.count > SPLIT_LIST_MAX)
        return hipErrorInvalidValue;
    const size_t lds = xch_lds_bytes(pl.q, W);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    switch (pl.q) {
        case 2: return launch_x_q<2>(s, a, x, sc, lds);
        case 3: return launch_x_q<3>(s, a, x, sc, lds);
        case 4: return launch_x_q<4>(s, a, x, sc, lds);
        case 5: return launch_x_q<5>(s, a, x, sc, lds);
        case 6: return launch_x_q<6>(s, a, x, sc, lds);
        case 7: return launch_x_q<7>(s, a, x, sc, lds);
        case 8: return launch_x_q<8>(s, a, x, sc, lds);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tlad(hipStream_t s, const TladArgs &a, int mode, bool fp32, int waves, int tb,
                       const SplitCols *sc) {
    if (a.nb <= 0) return hipSuccess;
    if (mode == TLAD_SPLIT || mode == TLAD_SPLIT_HV) {
        if ((fp32 && mode == TLAD_SPLIT) || a.pieces < 1 || a.ring < 1 || a.ring > a.n) return hipErrorInvalidValue;
        if (a.pieces == 1 ? (a.ring != a.n || a.halo != 0) : a.ring != tlad_split_ring(a.n, a.N, a.band_hi, a.pieces))
            return hipErrorInvalidValue;
    }
    if (mode == TLAD_SPLIT_SH || mode == TLAD_SPLIT_HV_SH) {
        if ((fp32 && mode == TLAD_SPLIT_SH) || a.pieces < 2 ||
            a.ring != tlad_split_ring_sh(a.n, a.N, a.band_hi, a.pieces) || a.ring == 0 ||
            a.halo != tlad_split_halo_sh(a.N, a.band_hi) || !a.pflags || !a.err || a.spin_max < 0)
            return hipErrorInvalidValue;
    }
    const bool split = mode == TLAD_SPLIT || mode == TLAD_SPLIT_HV || mode == TLAD_SPLIT_SH || mode == TLAD_SPLIT_HV_SH;
    const int R = split ? a.ring : a.n;
    if (waves != 0 && !tlad_waves_ok(R, waves)) return hipErrorInvalidValue;
    // rings of pieces take 8 waves where they fit: two waves per SIMD hide
    // more latency (at n = 4096, N = 40 the 1094- to 1948-point rings ran
    // 6-17% faster per iteration than on 4 waves with twice the points)
    if (waves == 0 && split && tlad_waves_ok(R, 8)) waves = 8;
    TladGeom g = tlad_geometry(R, waves, tb);
    if (g.q > 9 || g.tb < 1) return hipErrorInvalidValue;
    if (mode == TLAD_PCG && fp32) return hipErrorInvalidValue;  // PCG recurrences stay FP64
    if (sc) {
        if (sc->count < 0 || sc->count > SPLIT_LIST_MAX || sc->count > a.nb) return hipErrorInvalidValue;
        for (int i = 0; i < sc->count; i++)
            if (sc->col[i] < 0 || sc->col[i] >= a.nb) return hipErrorInvalidValue;
    }
    return fp32 ? launch_t<float>(s, a, g, mode, sc) : launch_t<double>(s, a, g, mode, sc);
}

}  // namespace eda

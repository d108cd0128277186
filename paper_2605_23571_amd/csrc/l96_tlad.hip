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
#include "eda_internal.h"

namespace eda {
namespace {

// lane l receives the value of lane l - 1 (lane 0: zero; window-edge garbage)
__device__ __forceinline__ double from_prev(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// lane l receives the value of lane l + 1
__device__ __forceinline__ double from_next(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
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

// Tendency k and TL increment dk at own points.
template <typename T, int Q, bool WANT_K>
__device__ __forceinline__ void tl_stage(const T (&y)[Q + 4], const T (&v)[Q + 4], T F, T (&k)[Q], T (&dk)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++) {
        T a = y[j + 3] - y[j];
        if (WANT_K) k[j] = a * y[j + 1] - y[j + 2] + F;
        dk[j] = y[j + 1] * (v[j + 3] - v[j]) + a * v[j + 1] - v[j + 2];
    }
}

template <typename T, int Q>
__device__ __forceinline__ void tendency(const T (&y)[Q + 4], T F, T (&k)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++) k[j] = (y[j + 3] - y[j]) * y[j + 1] - y[j + 2] + F;
}

template <typename T, int Q>
__device__ __forceinline__ void jt(const T (&y)[Q + 4], const T (&w)[Q + 4], T (&out)[Q]) {
#pragma unroll
    for (int j = 0; j < Q; j++)
        out[j] = y[j] * w[j + 1] - y[j + 3] * w[j + 4] + (y[j + 4] - y[j + 1]) * w[j + 3] - w[j + 2];
}

// Ring position of this lane's window point q: base + q, wrapped once.
__device__ __forceinline__ int wpos(int base, int q, int n) {
    int p = base + q;
    return p >= n ? p - n : p;
}

template <typename T, int Q>
__device__ __forceinline__ void load_x(const double *__restrict__ xs, int base, int n, T (&x)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; q++) x[q] = (T)xs[wpos(base, q, n)];
}

// Window of this lane: ring position of its first point (base; the others
// follow contiguously, wrapped), the mask of points inside the wave's owned
// segment, and, in LDS (qi[q * 64 + lane]), the observation index of observed
// points (-1 otherwise; owned points only if owned_obs_only).
template <int Q>
__device__ __forceinline__ int window(const TladArgs &a, int w0, int own_lo, int own_hi, bool owned_obs_only,
                                      unsigned &ownm, int *qi) {
    const int n = a.n, lane = threadIdx.x & 63;
    int b = (w0 + lane * Q) % n;
    if (b < 0) b += n;
    ownm = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int p = wpos(b, q, n);
        const int jw = w0 + lane * Q + q;  // unwrapped position
        const bool own = jw >= own_lo && jw < own_hi;
        if (own) ownm |= 1u << q;
        const int r = p - a.obs_x0;
        const bool obs = r >= 0 && r % a.obs_dx == 0;
        qi[q * 64 + lane] = (obs && (own || !owned_obs_only)) ? r / a.obs_dx : -1;
    }
    return b;
}

// MODE 0: TL then AD forced by the TL's observed increments.
// MODE 1: AD only, forcing read from a.force.
template <typename T, int Q, int MODE>
__global__ __launch_bounds__(512) void k_tlad(TladArgs a, TladGeom g) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int c = blockIdx.x;
    if (a.active && a.active[c] != COL_RUNNING) return;
    const int n = a.n, N = a.N, p = a.nt * a.nv;
    const int wave = threadIdx.x >> 6;
    // two ring buffers [0, n) and [n, 2n), indexed rsel * n + position (a plain
    // offset from the LDS array keeps these accesses in the LDS address space)
    T *ring = reinterpret_cast<T *>(smraw);
    int *qi = reinterpret_cast<int *>(reinterpret_cast<T *>(smraw) + 2 * n) + wave * 64 * Q;
    const int lane = threadIdx.x & 63;
    const int own_lo = wave * g.S, own_hi = min(n, own_lo + g.S);
    const int member = a.col_member ? a.col_member[c] : 0;
    const double *traj = a.traj + (long long)member * a.traj_stride;
    const T F = (T)a.F, h = (T)a.h, dt = (T)a.dt, dt6 = (T)a.dt6, dt3 = (T)a.dt3;
    unsigned ownm;
    int rsel = 0;

    if (MODE == 0) {
        // ---------------- TL forward run ----------------
        int base = window<Q>(a, own_lo - g.hl_tl, own_lo, own_hi, true, ownm, qi);
        T dx[Q];
        const double *vcol = a.V + (long long)c * a.ldv;
#pragma unroll
        for (int q = 0; q < Q; q++) dx[q] = (T)vcol[wpos(base, q, n)];
        double *obs = a.obs + (long long)c * p;
        for (int s0 = 0; s0 < N; s0 += g.tb) {
            if (s0 > 0) {
                __syncthreads();
#pragma unroll
                for (int q = 0; q < Q; q++) dx[q] = ring[rsel * n + wpos(base, q, n)];
            }
            const int s1 = min(N, s0 + g.tb);
            for (int s = s0; s < s1; s++) {
                T x[Q], Y[Q + 4], V[Q + 4], k[Q], dk[Q], acc[Q], ys[Q], vs[Q];
                load_x<T, Q>(traj + (long long)s * n, base, n, x);
                ext<T, Q>(x, Y);
                ext<T, Q>(dx, V);
                tl_stage<T, Q, true>(Y, V, F, k, dk);
#pragma unroll
                for (int j = 0; j < Q; j++) {
                    acc[j] = dk[j];
                    ys[j] = x[j] + h * k[j];
                    vs[j] = dx[j] + h * dk[j];
                }
                ext<T, Q>(ys, Y);
                ext<T, Q>(vs, V);
                tl_stage<T, Q, true>(Y, V, F, k, dk);
#pragma unroll
                for (int j = 0; j < Q; j++) {
                    acc[j] += T(2) * dk[j];
                    ys[j] = x[j] + h * k[j];
                    vs[j] = dx[j] + h * dk[j];
                }
                ext<T, Q>(ys, Y);
                ext<T, Q>(vs, V);
                tl_stage<T, Q, true>(Y, V, F, k, dk);
#pragma unroll
                for (int j = 0; j < Q; j++) {
                    acc[j] += T(2) * dk[j];
                    ys[j] = x[j] + dt * k[j];
                    vs[j] = dx[j] + dt * dk[j];
                }
                ext<T, Q>(ys, Y);
                ext<T, Q>(vs, V);
                tl_stage<T, Q, false>(Y, V, F, k, dk);
#pragma unroll
                for (int j = 0; j < Q; j++) dx[j] = dx[j] + dt6 * (acc[j] + dk[j]);
                if ((s + 1) % a.obs_dt == 0) {
                    double *o = obs + (long long)((s + 1) / a.obs_dt - 1) * a.nv;
#pragma unroll
                    for (int q = 0; q < Q; q++) {
                        const int oi = qi[q * 64 + lane];
                        if (oi >= 0) o[oi] = (double)dx[q] * a.inv_s2;
                    }
                }
            }
            if (s1 < N) {
#pragma unroll
                for (int q = 0; q < Q; q++)
                    if (ownm & (1u << q)) ring[(rsel ^ 1) * n + wpos(base, q, n)] = dx[q];
                rsel ^= 1;
            }
        }
        __threadfence_block();  // observed increments visible to the whole workgroup
        __syncthreads();
    }

    // ---------------- AD backward run ----------------
    __syncthreads();  // the TL phase's observation indices are no longer read
    const int base = window<Q>(a, own_lo - g.hl_ad, own_lo, own_hi, false, ownm, qi);
    const double *force = (MODE == 0) ? a.obs + (long long)c * p : a.force + (long long)c * p;
    T lam[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) lam[q] = T(0);
    for (int s_hi = N; s_hi >= 1; s_hi -= g.tb) {
        if (s_hi < N) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; q++) lam[q] = ring[rsel * n + wpos(base, q, n)];
        }
        const int s_lo = max(0, s_hi - g.tb);
        for (int s = s_hi; s > s_lo; s--) {
            if (s % a.obs_dt == 0) {
                const double *f = force + (long long)(s / a.obs_dt - 1) * a.nv;
#pragma unroll
                for (int q = 0; q < Q; q++) {
                    const int oi = qi[q * 64 + lane];
                    if (oi >= 0) lam[q] += (T)f[oi];
                }
            }
            const double *xs = traj + (long long)(s - 1) * n;
            T x[Q], Y2[Q + 4], Y3[Q + 4], Y4[Q + 4], M[Q + 4], k[Q], ys[Q];
            load_x<T, Q>(xs, base, n, x);
            {
                T Y1[Q + 4];
                ext<T, Q>(x, Y1);
                tendency<T, Q>(Y1, F, k);
            }
#pragma unroll
            for (int j = 0; j < Q; j++) ys[j] = x[j] + h * k[j];
            ext<T, Q>(ys, Y2);
            tendency<T, Q>(Y2, F, k);
#pragma unroll
            for (int j = 0; j < Q; j++) ys[j] = x[j] + h * k[j];
            ext<T, Q>(ys, Y3);
            tendency<T, Q>(Y3, F, k);
#pragma unroll
            for (int j = 0; j < Q; j++) ys[j] = x[j] + dt * k[j];
            ext<T, Q>(ys, Y4);
            // backward through the stages: mu4 = dt/6 lam, mu3 = mu2 = dt/3 lam, mu1 = dt/6 lam
            T nu[Q], acc[Q], mu[Q];
#pragma unroll
            for (int j = 0; j < Q; j++) mu[j] = dt6 * lam[j];
            ext<T, Q>(mu, M);
            jt<T, Q>(Y4, M, nu);
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
        }
        if (s_lo > 0) {
#pragma unroll
            for (int q = 0; q < Q; q++)
                if (ownm & (1u << q)) ring[(rsel ^ 1) * n + wpos(base, q, n)] = lam[q];
            rsel ^= 1;
        }
    }
    double *out = a.lam + (long long)c * a.ldl;
#pragma unroll
    for (int q = 0; q < Q; q++)
        if (ownm & (1u << q)) out[wpos(base, q, n)] = (double)lam[q];
}

template <typename T, int Q>
hipError_t launch_q(hipStream_t s, const TladArgs &a, const TladGeom &g, int mode) {
    const size_t lds = sizeof(T) * 2 * (size_t)a.n + sizeof(int) * (size_t)g.waves * 64 * Q;
    const dim3 block(64 * g.waves);
    if (mode == 0)
        hipLaunchKernelGGL((k_tlad<T, Q, 0>), dim3(a.nb), block, lds, s, a, g);
    else
        hipLaunchKernelGGL((k_tlad<T, Q, 1>), dim3(a.nb), block, lds, s, a, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(hipStream_t s, const TladArgs &a, const TladGeom &g, int mode) {
    switch (g.q) {
        case 2: return launch_q<T, 2>(s, a, g, mode);
        case 3: return launch_q<T, 3>(s, a, g, mode);
        case 4: return launch_q<T, 4>(s, a, g, mode);
        case 5: return launch_q<T, 5>(s, a, g, mode);
        case 6: return launch_q<T, 6>(s, a, g, mode);
        case 7: return launch_q<T, 7>(s, a, g, mode);
        case 8: return launch_q<T, 8>(s, a, g, mode);
        case 9: return launch_q<T, 9>(s, a, g, mode);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Geometry: waves per workgroup, owned segment per wave, points per lane and
// the time-block length, with halos hl_tl = 8 TB (TL cone: 8 left, 4 right per
// step) and hl_ad = 4 TB + 8 (AD cone: 4 left, 8 right per step, plus the
// recomputed stage states' fixed reach), requiring S + 12 TB + 16 <= 64 Q.
TladGeom tlad_geometry(int n, int waves_hint) {
    TladGeom g{};
    int W = waves_hint > 0 ? waves_hint : (n >= 2048 ? 8 : n >= 512 ? 4 : n >= 128 ? 2 : 1);
    g.waves = W;
    g.S = (n + W - 1) / W;
    int Q = 2;
    while (64 * Q < g.S + 12 * 2 + 16) Q++;
    g.q = Q;
    g.tb = (64 * Q - g.S - 16) / 12;
    g.hl_tl = 8 * g.tb;
    g.hl_ad = 4 * g.tb + 8;
    return g;
}

hipError_t launch_tlad(hipStream_t s, const TladArgs &a, int mode, bool fp32) {
    if (a.nb <= 0) return hipSuccess;
    TladGeom g = tlad_geometry(a.n, 0);
    if (g.q > 9 || g.tb < 1) return hipErrorInvalidValue;
    return fp32 ? launch_t<float>(s, a, g, mode) : launch_t<double>(s, a, g, mode);
}

}  // namespace eda

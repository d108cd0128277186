// Tangent-linear (TL) forward run and adjoint (AD) backward run of the
// Lorenz-96 RK4 model about stored trajectories -- the core of one Hessian
// product A x = U_B^T G^T R^-1 G U_B x (system_with_CVT equation).  The paper
// uses these runs (the "integrations of the tangent linear and adjoint models"
// of the sketching and Nystrom subsections) without printing them; they are the
// exact derivative of the RK4 step and its transpose:
//
//   J(y) v at i  = y_{i-1} (v_{i+1} - v_{i-2}) + (y_{i+1} - y_{i-2}) v_{i-1} - v_i
//   J(y)^T w at k = y_{k-2} w_{k-1} - y_{k+1} w_{k+2} + (y_{k+2} - y_{k-1}) w_{k+1} - w_k
//   TL: dk1 = J(x1) dx, dk2 = J(x2)(dx + h dk1), dk3 = J(x3)(dx + h dk2),
//       dk4 = J(x4)(dx + dt dk3), dx' = dx + dt/6 (dk1 + 2 dk2 + 2 dk3 + dk4)
//   AD: its reverse-mode transpose (stage states x1..x4 recomputed from X[s]).
//
// Layout and schedule (one workgroup per column; the column's whole ring lives
// in the workgroup):
//  * thread t owns P contiguous points [tP, tP + P) held in registers, so the
//    radius-2 stencil needs only 2 halo values on each side;
//  * halos go through LDS: each thread publishes its two first and two last
//    values and reads its neighbours' after one barrier (two alternating
//    buffer sets: one barrier per exchange);
//  * RK4 stage states are recomputed from the stored state X[s] instead of
//    stored (4x fewer trajectory bytes): TL needs 4 exchanges per step, AD 6;
//  * the observed increments R^-1 H dx at observation times go to a per-column
//    scratch buffer that the same threads read back as AD forcing.
#include "eda_internal.h"

namespace eda {
namespace {

__device__ __forceinline__ int wrapn(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Halo exchange through LDS.  Each thread publishes 4 slots per quantity --
// its first two points and its last two (for a thread with a single point the
// same value fills the first and the last slot) -- and reads the slots that
// hold ring positions i0 - 2, i0 - 1, i0 + cnt, i0 + cnt + 1 (cyclic).  Two
// alternating buffer sets make one barrier per exchange sufficient.
template <typename T, int P>
struct Ring {
    T *lds;
    int n, i0, cnt, sel, nthr;

    __device__ T *buf(int q) const { return lds + (size_t)(2 * sel + q) * 4 * nthr; }

    // slot holding ring position pos (pos must be within two of its owner's ends)
    __device__ int slot(int pos) const {
        const int t = pos / P, e = pos - t * P;
        const int ct = min(P, n - t * P);
        const int k = (e == ct - 1) ? 3 : (e == ct - 2 ? 2 : e);
        return 4 * t + k;
    }
    __device__ void put(int q, const T (&v)[P]) const {
        if (cnt <= 0) return;
        T *b = buf(q) + 4 * (i0 / P);
        b[0] = v[0];
        if (P > 1 && cnt > 1) b[1] = v[1];
        if (cnt == P) {
            if (P > 1) b[2] = v[P - 2];
            b[3] = v[P - 1];
        } else {
#pragma unroll
            for (int j = 0; j < P; j++) {
                if (j == cnt - 2) b[2] = v[j];
                if (j == cnt - 1) b[3] = v[j];
            }
        }
    }
    // Extended array: e[0..1] = left halo, e[2+j] own (for a ragged last thread
    // the two slots after its last point hold the wrapped right halo; later
    // ones are unused), e[P+2..P+3] right halo.
    __device__ void get(int q, const T (&v)[P], T (&e)[P + 4]) const {
        const T *b = buf(q);
        e[0] = b[slot(wrapn(i0 - 2, n))];
        e[1] = b[slot(wrapn(i0 - 1, n))];
        const T r0 = b[slot(wrapn(i0 + cnt, n))];
        const T r1 = b[slot(wrapn(i0 + cnt + 1, n))];
#pragma unroll
        for (int j = 0; j < P; j++) e[2 + j] = (j < cnt) ? v[j] : (j == cnt ? r0 : r1);
        e[P + 2] = (cnt == P) ? r0 : r1;
        e[P + 3] = r1;
    }
    __device__ void flip() { sel ^= 1; }
};

template <typename T, int P>
__device__ __forceinline__ void load_state(const double *__restrict__ xs, int n, int i0, bool live,
                                           T (&e)[P + 4]) {
    if (!live) {
#pragma unroll
        for (int j = 0; j < P + 4; j++) e[j] = T(0);
        return;
    }
    e[0] = (T)xs[wrapn(i0 - 2, n)];
    e[1] = (T)xs[wrapn(i0 - 1, n)];
#pragma unroll
    for (int j = 0; j < P + 2; j++) e[2 + j] = (T)xs[wrapn(i0 + j, n)];
}

// Tendency and TL at own points from extended stage state y and increment v.
template <typename T, int P, bool WANT_K>
__device__ __forceinline__ void tl_stage(const T (&y)[P + 4], const T (&v)[P + 4], T F, T (&k)[P],
                                         T (&dk)[P]) {
#pragma unroll
    for (int j = 0; j < P; j++) {
        T a = y[j + 3] - y[j];
        if (WANT_K) k[j] = a * y[j + 1] - y[j + 2] + F;
        dk[j] = y[j + 1] * (v[j + 3] - v[j]) + a * v[j + 1] - v[j + 2];
    }
}

template <typename T, int P>
__device__ __forceinline__ void tendency(const T (&y)[P + 4], T F, T (&k)[P]) {
#pragma unroll
    for (int j = 0; j < P; j++) k[j] = (y[j + 3] - y[j]) * y[j + 1] - y[j + 2] + F;
}

template <typename T, int P>
__device__ __forceinline__ void jt(const T (&y)[P + 4], const T (&w)[P + 4], T (&out)[P]) {
#pragma unroll
    for (int j = 0; j < P; j++)
        out[j] = y[j] * w[j + 1] - y[j + 3] * w[j + 4] + (y[j + 4] - y[j + 1]) * w[j + 3] - w[j + 2];
}

// MODE 0: TL then AD with the TL's observed increments as forcing.
// MODE 1: AD only, forcing read from a.force.
template <typename T, int P, int MODE>
__global__ __launch_bounds__(P >= 8 ? 512 : 256) void k_tlad(TladArgs a) {
    extern __shared__ __align__(16) unsigned char smraw[];
    const int c = blockIdx.x;
    if (a.active && a.active[c] != COL_RUNNING) return;
    const int n = a.n, N = a.N;
    const int i0 = threadIdx.x * P;
    const int cnt = max(0, min(P, n - i0));
    const bool live = cnt > 0;
    const int member = a.col_member ? a.col_member[c] : 0;
    const double *traj = a.traj + (long long)member * a.traj_stride;
    const int p = a.nt * a.nv;
    const T F = (T)a.F, h = (T)a.h, dt = (T)a.dt, dt6 = (T)a.dt6, dt3 = (T)a.dt3;
    Ring<T, P> ring{reinterpret_cast<T *>(smraw), n, i0, cnt, 0, (int)blockDim.x};

    // first observed own point and its observation index
    int q_first = 0, j_first = P;
    if (live) {
        int r = i0 - a.obs_x0;
        int jj = r >= 0 ? (a.obs_dx - r % a.obs_dx) % a.obs_dx : -r;
        if (jj < cnt) {
            j_first = jj;
            q_first = (i0 + jj - a.obs_x0) / a.obs_dx;
        }
    }

    T lam[P];
    if (MODE == 0) {
        // ---------------- TL forward run ----------------
        T dx[P];
        const double *vcol = a.V + (long long)c * a.ldv;
#pragma unroll
        for (int j = 0; j < P; j++) dx[j] = (j < cnt) ? (T)vcol[i0 + j] : T(0);
        double *obs = a.obs + (long long)c * p;
        for (int s = 0; s < N; s++) {
            T Y[P + 4], Vx[P + 4], xo[P], k[P], dk[P], acc[P], ys[P], vs[P];
            load_state<T, P>(traj + (long long)s * n, n, i0, live, Y);
#pragma unroll
            for (int j = 0; j < P; j++) xo[j] = Y[j + 2];
            ring.put(0, dx);
            __syncthreads();
            ring.get(0, dx, Vx);
            ring.flip();
            tl_stage<T, P, true>(Y, Vx, F, k, dk);
#pragma unroll
            for (int j = 0; j < P; j++) {
                acc[j] = dk[j];
                ys[j] = xo[j] + h * k[j];
                vs[j] = dx[j] + h * dk[j];
            }
            ring.put(0, ys);
            ring.put(1, vs);
            __syncthreads();
            ring.get(0, ys, Y);
            ring.get(1, vs, Vx);
            ring.flip();
            tl_stage<T, P, true>(Y, Vx, F, k, dk);
#pragma unroll
            for (int j = 0; j < P; j++) {
                acc[j] += T(2) * dk[j];
                ys[j] = xo[j] + h * k[j];
                vs[j] = dx[j] + h * dk[j];
            }
            ring.put(0, ys);
            ring.put(1, vs);
            __syncthreads();
            ring.get(0, ys, Y);
            ring.get(1, vs, Vx);
            ring.flip();
            tl_stage<T, P, true>(Y, Vx, F, k, dk);
#pragma unroll
            for (int j = 0; j < P; j++) {
                acc[j] += T(2) * dk[j];
                ys[j] = xo[j] + dt * k[j];
                vs[j] = dx[j] + dt * dk[j];
            }
            ring.put(0, ys);
            ring.put(1, vs);
            __syncthreads();
            ring.get(0, ys, Y);
            ring.get(1, vs, Vx);
            ring.flip();
            tl_stage<T, P, false>(Y, Vx, F, k, dk);
#pragma unroll
            for (int j = 0; j < P; j++) dx[j] = dx[j] + dt6 * (acc[j] + dk[j]);
            if ((s + 1) % a.obs_dt == 0) {
                const int t = (s + 1) / a.obs_dt - 1;
                double *o = obs + (long long)t * a.nv;
                int q = q_first;
#pragma unroll
                for (int j = 0; j < P; j++) {
                    if (j >= j_first && j < cnt && (j - j_first) % a.obs_dx == 0) {
                        o[q] = (double)dx[j] * a.inv_s2;
                        q++;
                    }
                }
            }
        }
    }
    // ---------------- AD backward run ----------------
    const double *force = (MODE == 0) ? a.obs + (long long)c * p : a.force + (long long)c * p;
#pragma unroll
    for (int j = 0; j < P; j++) lam[j] = T(0);
    for (int s = N; s >= 1; s--) {
        if (s % a.obs_dt == 0) {
            const int t = s / a.obs_dt - 1;
            const double *f = force + (long long)t * a.nv;
            int q = q_first;
#pragma unroll
            for (int j = 0; j < P; j++) {
                if (j >= j_first && j < cnt && (j - j_first) % a.obs_dx == 0) {
                    lam[j] += (T)f[q];
                    q++;
                }
            }
        }
        T Y2[P + 4], Y3[P + 4], Y4[P + 4], M[P + 4], xo[P], k[P], ys[P];
        const double *xs = traj + (long long)(s - 1) * n;
        {
            T Y1[P + 4];  // reloaded (cache hit) for the last stage to save registers
            load_state<T, P>(xs, n, i0, live, Y1);
#pragma unroll
            for (int j = 0; j < P; j++) xo[j] = Y1[j + 2];
            tendency<T, P>(Y1, F, k);
        }
#pragma unroll
        for (int j = 0; j < P; j++) ys[j] = xo[j] + h * k[j];
        ring.put(0, ys);
        ring.put(1, lam);
        __syncthreads();
        ring.get(0, ys, Y2);
        ring.get(1, lam, M);
        ring.flip();
        tendency<T, P>(Y2, F, k);
#pragma unroll
        for (int j = 0; j < P; j++) ys[j] = xo[j] + h * k[j];
        ring.put(0, ys);
        __syncthreads();
        ring.get(0, ys, Y3);
        ring.flip();
        tendency<T, P>(Y3, F, k);
#pragma unroll
        for (int j = 0; j < P; j++) ys[j] = xo[j] + dt * k[j];
        ring.put(0, ys);
        __syncthreads();
        ring.get(0, ys, Y4);
        ring.flip();
        // backward through the stages
        T nu[P], acc[P], mu[P];
#pragma unroll
        for (int j = 0; j < P + 4; j++) M[j] = dt6 * M[j];  // mu4 = dt/6 lam (with halos)
        jt<T, P>(Y4, M, nu);
#pragma unroll
        for (int j = 0; j < P; j++) {
            acc[j] = lam[j] + nu[j];
            mu[j] = dt3 * lam[j] + dt * nu[j];  // mu3
        }
        ring.put(0, mu);
        __syncthreads();
        ring.get(0, mu, M);
        ring.flip();
        jt<T, P>(Y3, M, nu);
#pragma unroll
        for (int j = 0; j < P; j++) {
            acc[j] += nu[j];
            mu[j] = dt3 * lam[j] + h * nu[j];  // mu2
        }
        ring.put(0, mu);
        __syncthreads();
        ring.get(0, mu, M);
        ring.flip();
        jt<T, P>(Y2, M, nu);
#pragma unroll
        for (int j = 0; j < P; j++) {
            acc[j] += nu[j];
            mu[j] = dt6 * lam[j] + h * nu[j];  // mu1
        }
        ring.put(0, mu);
        __syncthreads();
        ring.get(0, mu, M);
        ring.flip();
        {
            T Y1[P + 4];
            load_state<T, P>(xs, n, i0, live, Y1);
            jt<T, P>(Y1, M, nu);
        }
#pragma unroll
        for (int j = 0; j < P; j++) lam[j] = acc[j] + nu[j];
    }
    double *out = a.lam + (long long)c * a.ldl;
#pragma unroll
    for (int j = 0; j < P; j++)
        if (j < cnt) out[i0 + j] = (double)lam[j];
}

template <typename T, int P>
hipError_t launch_p(hipStream_t s, const TladArgs &a, int mode) {
    int threads = (a.n + P - 1) / P;
    threads = (threads + 63) / 64 * 64;
    size_t lds = 2 * 2 * 4 * sizeof(T) * (size_t)threads;
    if (mode == 0)
        hipLaunchKernelGGL((k_tlad<T, P, 0>), dim3(a.nb), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_tlad<T, P, 1>), dim3(a.nb), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(hipStream_t s, const TladArgs &a, int mode) {
    // points per thread: the smallest power of two keeping the ring within 256
    // threads, capped at 8 (then up to 512 threads for n <= 4096)
    const int n = a.n;
    if (n <= 256) return launch_p<T, 1>(s, a, mode);
    if (n <= 512) return launch_p<T, 2>(s, a, mode);
    if (n <= 1024) return launch_p<T, 4>(s, a, mode);
    if (n <= 4096) return launch_p<T, 8>(s, a, mode);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tlad(hipStream_t s, const TladArgs &a, int mode, bool fp32) {
    if (a.nb <= 0) return hipSuccess;
    return fp32 ? launch_t<float>(s, a, mode) : launch_t<double>(s, a, mode);
}

}  // namespace eda

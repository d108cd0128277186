// Nonlinear Lorenz-96 RK4 integration (numerical-experiments section: the
// Lorenz-96 ODE with cyclic indices, classical RK4).  Used for the truth
// spin-up and window and for the members' linearisation trajectories.
//
// This file is compiled with floating-point contraction disabled and every
// expression is written in a fixed order:
//   f_i = ((x_{i+1} - x_{i-2}) * x_{i-1} - x_i) + F
//   x2 = x + h k1, x3 = x + h k2, x4 = x + dt k3            (h = dt/2)
//   x' = x + c6 * (((k1 + 2 k2) + 2 k3) + k4)               (c6 = dt/6)
// so that the result is the correctly rounded evaluation of exactly these
// operations -- a chaotic 1000-step spin-up is reproducible bit for bit by any
// IEEE-754 implementation that keeps the same order.
#include "eda_internal.h"

#pragma clang fp contract(off)

namespace eda {
namespace {

constexpr int NL_THREADS = 256;
constexpr int NL_MAXP = 16;  // n <= 4096

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ double l96f(const double *x, int i, int n, double F) {
    double a = x[wrapi(i + 1, n)] - x[wrapi(i - 2, n)];
    double t = a * x[wrapi(i - 1, n)];
    t = t - x[i];
    return t + F;
}

__global__ __launch_bounds__(NL_THREADS) void k_nl(int n, int nsteps, double F, double h, double dt,
                                                    double c6, const double *__restrict__ x0,
                                                    double *__restrict__ store, double *__restrict__ xend) {
    extern __shared__ double sm[];
    double *x = sm;       // current state
    double *xs = sm + n;  // stage state
    const int v = blockIdx.x, tid = threadIdx.x;
    const double *src = x0 + (size_t)v * n;
    double *dst = store ? store + (size_t)v * (nsteps + 1) * n : nullptr;
    double acc[NL_MAXP], xr[NL_MAXP];
#pragma unroll
    for (int t = 0; t < NL_MAXP; t++) {
        int i = tid + t * NL_THREADS;
        if (i < n) {
            xr[t] = src[i];
            x[i] = xr[t];
            if (dst) dst[i] = xr[t];
        }
    }
    __syncthreads();
    for (int s = 0; s < nsteps; s++) {
        // stage 1: k1 = f(x)
        double k[NL_MAXP];
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) k[t] = l96f(x, i, n, F);
        }
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) {
                acc[t] = k[t];
                xs[i] = xr[t] + h * k[t];
            }
        }
        __syncthreads();
        // stage 2
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) k[t] = l96f(xs, i, n, F);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) {
                acc[t] = acc[t] + 2.0 * k[t];
                xs[i] = xr[t] + h * k[t];
            }
        }
        __syncthreads();
        // stage 3
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) k[t] = l96f(xs, i, n, F);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) {
                acc[t] = acc[t] + 2.0 * k[t];
                xs[i] = xr[t] + dt * k[t];
            }
        }
        __syncthreads();
        // stage 4 and the update
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) k[t] = l96f(xs, i, n, F);
        }
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) {
                acc[t] = acc[t] + k[t];
                xr[t] = xr[t] + c6 * acc[t];
                x[i] = xr[t];
                if (dst) dst[(size_t)(s + 1) * n + i] = xr[t];
            }
        }
        __syncthreads();
    }
    if (xend) {
#pragma unroll
        for (int t = 0; t < NL_MAXP; t++) {
            int i = tid + t * NL_THREADS;
            if (i < n) xend[(size_t)v * n + i] = xr[t];
        }
    }
}

__global__ void k_spin_init(int n, double F, double std_, const double *z, double *x) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (i == 0) ? F + std_ * z[0] : F;
}

}  // namespace

hipError_t launch_nl(hipStream_t s, int n, int nvec, int nsteps, double F, double h, double dt, double c6,
                     const double *x0, double *store, double *xend) {
    if (n > NL_THREADS * NL_MAXP) return hipErrorInvalidValue;
    size_t lds = sizeof(double) * 2 * (size_t)n;
    hipLaunchKernelGGL(k_nl, dim3(nvec), dim3(NL_THREADS), lds, s, n, nsteps, F, h, dt, c6, x0, store, xend);
    return hipGetLastError();
}

hipError_t launch_spin_init(hipStream_t s, int n, double F, double std_, const double *z, double *x) {
    hipLaunchKernelGGL(k_spin_init, dim3((n + 255) / 256), dim3(256), 0, s, n, F, std_, z, x);
    return hipGetLastError();
}

}  // namespace eda

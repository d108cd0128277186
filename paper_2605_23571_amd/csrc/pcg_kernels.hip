// Batched preconditioned CG (solving-linear-systems section): one workgroup
// per member column, FP64 recurrences and dot products.  Dot products reduce
// in a fixed order (per-thread strided partial sums, then a fixed tree), so a
// solve is bit-reproducible.  A member whose status leaves COL_RUNNING is
// skipped by every later kernel, including the Hessian product.
#include "eda_internal.h"

namespace eda {
namespace {

constexpr int PT = 256;

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < PT / 64; w++) s += red[w];
    return s;
}

// x = 0, r = b_m, status running, history row NaN, J_0 - c = 0.
__global__ __launch_bounds__(PT) void k_pcg_init(PcgArgs a) {
    __shared__ double red[PT / 64];
    const int c = blockIdx.x, n = a.n;
    const double *b = a.b + (long long)a.members[c] * n;
    double *x = a.x + (long long)c * n, *r = a.r + (long long)c * n;
    double bb = 0.0;
    for (int i = threadIdx.x; i < n; i += PT) {
        double v = b[i];
        x[i] = 0.0;
        r[i] = v;
        bb += v * v;
    }
    bb = block_sum(bb, red);
    if (a.hist)
        for (int i = threadIdx.x; i < a.hist_cap; i += PT)
            a.hist[(long long)c * a.hist_cap + i] = i == 0 ? 0.0 : __builtin_nan("");
    if (threadIdx.x == 0) {
        a.scal[4 * c + 1] = sqrt(bb);
        a.scal[4 * c + 2] = bb > 0 ? 1.0 : 0.0;
        a.status[c] = bb > 0 ? COL_RUNNING : EDA_MEMBER_CONVERGED;
        a.iters[c] = 0;
    }
}

// After z = P r: p = z, rho = r^T z.
__global__ __launch_bounds__(PT) void k_pcg_start(PcgArgs a) {
    __shared__ double red[PT / 64];
    const int c = blockIdx.x, n = a.n;
    if (a.status[c] != COL_RUNNING) return;
    const double *r = a.r + (long long)c * n, *z = a.z + (long long)c * n;
    double *p = a.p + (long long)c * n;
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += PT) {
        double zv = z[i];
        p[i] = zv;
        rz += r[i] * zv;
    }
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) a.scal[4 * c] = rz;
}

// q = (I + A) p given: alpha = rho / p^T q, x += alpha p, r -= alpha q,
// convergence test on ||r|| <= rtol ||b||, cost J_it - c = -1/2 x^T (b + r).
__global__ __launch_bounds__(PT) void k_pcg_alpha(PcgArgs a, int it) {
    __shared__ double red[PT / 64];
    const int c = blockIdx.x, n = a.n;
    if (a.status[c] != COL_RUNNING) return;
    const double *p = a.p + (long long)c * n, *q = a.q + (long long)c * n;
    double *x = a.x + (long long)c * n, *r = a.r + (long long)c * n;
    double pq = 0.0;
    for (int i = threadIdx.x; i < n; i += PT) pq += p[i] * q[i];
    pq = block_sum(pq, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (threadIdx.x == 0) {
            a.status[c] = EDA_MEMBER_BREAKDOWN;
            a.iters[c] = it - 1;
        }
        return;
    }
    const double alpha = a.scal[4 * c] / pq;
    const double *b = a.b + (long long)a.members[c] * n;
    double rr = 0.0, xbr = 0.0;
    for (int i = threadIdx.x; i < n; i += PT) {
        double xi = x[i] + alpha * p[i];
        double ri = r[i] - alpha * q[i];
        x[i] = xi;
        r[i] = ri;
        rr += ri * ri;
        if (a.hist) xbr += xi * (b[i] + ri);
    }
    rr = block_sum(rr, red);
    if (a.hist) xbr = block_sum(xbr, red);
    if (threadIdx.x == 0) {
        const double bnorm = a.scal[4 * c + 1];
        const double rn = sqrt(rr);
        a.scal[4 * c + 2] = rn / bnorm;
        a.iters[c] = it;
        if (a.hist && it < a.hist_cap) a.hist[(long long)c * a.hist_cap + it] = -0.5 * xbr;
        if (!isfinite(rn)) a.status[c] = EDA_MEMBER_BREAKDOWN;
        else if (rn <= a.rtol * bnorm) a.status[c] = EDA_MEMBER_CONVERGED;
    }
}

// After z = P r: rho' = r^T z, p = z + (rho'/rho) p.
__global__ __launch_bounds__(PT) void k_pcg_beta(PcgArgs a) {
    __shared__ double red[PT / 64];
    const int c = blockIdx.x, n = a.n;
    if (a.status[c] != COL_RUNNING) return;
    const double *r = a.r + (long long)c * n, *z = a.z + (long long)c * n;
    double *p = a.p + (long long)c * n;
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += PT) rz += r[i] * z[i];
    rz = block_sum(rz, red);
    if (!(rz > 0.0) || !isfinite(rz)) {
        if (threadIdx.x == 0) a.status[c] = EDA_MEMBER_BREAKDOWN;
        return;
    }
    const double beta = rz / a.scal[4 * c];
    for (int i = threadIdx.x; i < n; i += PT) p[i] = z[i] + beta * p[i];
    if (threadIdx.x == 0) a.scal[4 * c] = rz;
}

// Columns still running, or never admitted, end as not converged.
__global__ void k_pcg_finish(PcgArgs a) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < a.nb && (a.status[c] == COL_RUNNING || a.status[c] == COL_PENDING))
        a.status[c] = EDA_MEMBER_NOT_CONVERGED;
}

__global__ void k_col_status(SplitCols cols, int32_t from, int32_t to, int32_t *status, int32_t *start,
                             int32_t start_it) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cols.count) return;
    const int c = cols.col[i];
    if (status[c] != from) return;
    status[c] = to;
    if (start) start[c] = start_it;
}

}  // namespace

hipError_t launch_pcg_init(hipStream_t s, const PcgArgs &a) {
    hipLaunchKernelGGL(k_pcg_init, dim3(a.nb), dim3(PT), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_pcg_start(hipStream_t s, const PcgArgs &a) {
    hipLaunchKernelGGL(k_pcg_start, dim3(a.nb), dim3(PT), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_pcg_alpha(hipStream_t s, const PcgArgs &a, int it) {
    hipLaunchKernelGGL(k_pcg_alpha, dim3(a.nb), dim3(PT), 0, s, a, it);
    return hipGetLastError();
}
hipError_t launch_pcg_beta(hipStream_t s, const PcgArgs &a) {
    hipLaunchKernelGGL(k_pcg_beta, dim3(a.nb), dim3(PT), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_pcg_finish(hipStream_t s, const PcgArgs &a) {
    hipLaunchKernelGGL(k_pcg_finish, dim3((a.nb + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_col_status(hipStream_t s, const SplitCols &cols, int32_t from, int32_t to, int32_t *status,
                             int32_t *start, int32_t start_it) {
    if (cols.count < 1 || cols.count > SPLIT_LIST_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_col_status, dim3(1), dim3(SPLIT_LIST_MAX), 0, s, cols, from, to, status, start, start_it);
    return hipGetLastError();
}

}  // namespace eda

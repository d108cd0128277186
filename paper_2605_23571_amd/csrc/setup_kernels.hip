// Problem set-up kernels (ensemble-formulation section and the experiment
// set-up): U_B, observations, backgrounds, innovations, the RHS-difference
// sketch, and the banded circulant U_B product.
#include "eda_internal.h"

namespace eda {
namespace {

__device__ __forceinline__ int cyc_dist(int i, int n) { return i < n - i ? i : n - i; }

// U_B first row in closed form: r(d) = sigma_b (2/pi)^(1/4) len^(-1/2) exp(-d^2/len^2),
// the symmetric square root of sigma_b^2 exp(-d^2/(2 len^2)) (cyclic Gaussian B).
__global__ void k_ub_row(int n, double amp, double len2, double *row) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = (double)cyc_dist(i, n);
    row[i] = amp * exp(-d * d / len2);
}

// First row of U_B = sigma_b g (I - kappa Lap)^(-m) (m = M/2) on the ring of
// n points (the diffusion-based B), in real space: one implicit diffusion
// step is the cyclic convolution with the ring's Green's function of
// (I - kappa Lap),
//   G(d) = (rho^d + rho^(n-d)) / (kappa (1/rho - rho) (1 - rho^n)),
//   rho the root in (0, 1) of kappa rho^2 - (1 + 2 kappa) rho + kappa = 0
// (the unbounded line's kernel rho^|d| / (kappa (1/rho - rho)), summed over the
// ring's periods), so the row is G convolved with itself m times.  Every
// term is positive, so the sums carry no cancellation.  g normalises the
// diagonal of C_B = (U_B / sigma_b)^2 to one: the diagonal of the M-step
// operator is sum_d r0(d)^2 for the symmetric row r0 of the m-step one.  One
// workgroup; a and b are two n-double LDS arrays.
__global__ __launch_bounds__(1024) void k_ub_row_diffusion(int n, double kappa, int m, double sigma_b,
                                                           double *row) {
    extern __shared__ double lds_d[];
    double *a = lds_d, *b = lds_d + n;
    __shared__ double red[16];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const double rho = 2.0 * kappa / ((1.0 + 2.0 * kappa) + sqrt(1.0 + 4.0 * kappa));
    const double rn = pow(rho, (double)n);
    const double amp = 1.0 / (kappa * (1.0 / rho - rho) * (1.0 - rn));
    for (int d = tid; d < n; d += nthr) {
        const double g = amp * (pow(rho, (double)d) + pow(rho, (double)(n - d)));
        a[d] = g;
        b[d] = g;
    }
    __syncthreads();
    // b <- a (*) b, m - 1 times (a keeps G)
    for (int step = 1; step < m; step++) {
        double out[4];
        int cnt = 0;
        for (int d = tid; d < n; d += nthr) {
            double acc = 0.0;
            for (int e = 0; e < n; e++) {
                int j = d - e;
                j = j < 0 ? j + n : j;
                acc += b[e] * a[j];
            }
            out[cnt++] = acc;
        }
        __syncthreads();
        cnt = 0;
        for (int d = tid; d < n; d += nthr) b[d] = out[cnt++];
        __syncthreads();
    }
    // g^2 = 1 / sum_d b(d)^2, by a fixed-order reduction
    double ss = 0.0;
    for (int d = tid; d < n; d += nthr) ss += b[d] * b[d];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = ss;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (nthr >> 6); w++) tot += red[w];
    const double scale = sigma_b / sqrt(tot);
    for (int d = tid; d < n; d += nthr) row[d] = scale * b[d];
}

__global__ void k_ub_fill(int n, const double *__restrict__ row, double *__restrict__ ub) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int i = (int)(idx % n), j = (int)(idx / n);
    int d = i - j;
    if (d < 0) d += n;
    ub[idx] = row[d];
}

// Y[:, c] = sum_{o = lo..hi} r(|o|) X[(i - o) mod n, c] (+ Add[:, c]).
// Workgroup = (row tile of 256 outputs, column); the tile's input window and
// the taps are staged in LDS; each thread computes 4 consecutive outputs with
// a sliding register window (one LDS read per 4 FMAs).
constexpr int CONV_T = 64;   // threads
constexpr int CONV_R = 4;    // outputs per thread
constexpr int CONV_ROWS = CONV_T * CONV_R;

__global__ __launch_bounds__(CONV_T) void k_band_conv(int n, int lo, int hi, const double *__restrict__ row,
                                                      const double *__restrict__ X, long long ldx,
                                                      double *__restrict__ Y, long long ldy,
                                                      const double *__restrict__ Add, long long ldadd,
                                                      const int32_t *__restrict__ active) {
    extern __shared__ double sm[];
    const int c = blockIdx.y;
    if (active && active[c] != COL_RUNNING) return;
    const int W = hi - lo + 1;
    double *taps = sm;          // taps[m] = r(|hi - m|), m = 0..W-1
    double *xw = sm + W;        // x[(base + t) mod n], t = 0..CONV_ROWS + W - 2
    const int r0 = blockIdx.x * CONV_ROWS;
    const int base = r0 - hi;   // lowest input index used by the tile
    const double *x = X + (long long)c * ldx;
    for (int m = threadIdx.x; m < W; m += CONV_T) {
        int o = hi - m;
        int ao = o < 0 ? -o : o;
        taps[m] = row[ao];
    }
    const int win = CONV_ROWS + W - 1;
    for (int t = threadIdx.x; t < win; t += CONV_T) {
        int gi = (base + t) % n;
        if (gi < 0) gi += n;
        xw[t] = x[gi];
    }
    __syncthreads();
    const int lr = threadIdx.x * CONV_R;  // first local output row
    double acc[CONV_R] = {0.0, 0.0, 0.0, 0.0};
    double w[CONV_R];
#pragma unroll
    for (int u = 0; u < CONV_R; u++) w[u] = xw[lr + u];
    for (int m = 0; m < W; m++) {
        const double tm = taps[m];
#pragma unroll
        for (int u = 0; u < CONV_R; u++) acc[u] += tm * w[u];
#pragma unroll
        for (int u = 0; u < CONV_R - 1; u++) w[u] = w[u + 1];
        w[CONV_R - 1] = xw[lr + m + CONV_R];
    }
    double *y = Y + (long long)c * ldy;
    const double *ad = Add ? Add + (long long)c * ldadd : nullptr;
#pragma unroll
    for (int u = 0; u < CONV_R; u++) {
        int i = r0 + lr + u;
        if (i < n) y[i] = ad ? acc[u] + ad[i] : acc[u];
    }
}

// y[t][q] = truth[s_t][x0 + q dx] + sigma_o eta_0[t][q];  y_j = y + sigma_o eta_j.
__global__ void k_obs(int n, int L, int p, int nv, int obs_dt, int obs_dx, int obs_x0, double sigma_o,
                      const double *__restrict__ truth, const double *__restrict__ eta, double *__restrict__ y) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p) return;
    int t = idx / nv, q = idx % nv;
    int s = (t + 1) * obs_dt;
    double y0 = truth[(long long)s * n + obs_x0 + q * obs_dx] + sigma_o * eta[idx];
    y[idx] = y0;
    for (int j = 1; j <= L; j++) y[(long long)j * p + idx] = y0 + sigma_o * eta[(long long)j * p + idx];
}

// x^b = x^t_0 + (U_B xi)_0;  x^b_j = x^b + (U_B xi)_j.
__global__ void k_xb(int n, int L, const double *__restrict__ xt0, const double *__restrict__ ux,
                     double *__restrict__ xb) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double b0 = xt0[i] + ux[i];
    xb[i] = b0;
    for (int j = 1; j <= L; j++) xb[(long long)j * n + i] = b0 + ux[(long long)j * n + i];
}

// d_j = y_j - H X_j;  forcing R^-1 d_j;  c_j = 1/2 d_j^T R^-1 d_j (one workgroup per member).
__global__ __launch_bounds__(256) void k_innov(int n, int N, int p, int nv, int obs_dt, int obs_dx, int obs_x0,
                                               double s2, const double *__restrict__ y,
                                               const double *__restrict__ traj, double *__restrict__ d,
                                               double *__restrict__ force, double *__restrict__ costc) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const double *tj = traj + (long long)j * (N + 1) * n;
    double part = 0.0;
    for (int idx = threadIdx.x; idx < p; idx += blockDim.x) {
        int t = idx / nv, q = idx % nv;
        int s = (t + 1) * obs_dt;
        double dv = y[(long long)j * p + idx] - tj[(long long)s * n + obs_x0 + q * obs_dx];
        d[(long long)j * p + idx] = dv;
        force[(long long)j * p + idx] = dv / s2;
        part += dv * dv;
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) costc[j] = 0.5 * red[0] / s2;
}

// Gamma[:, j-1] = b_j - b_0, j = 1..ell (the matrix of RHS differences).
__global__ void k_gamma(int n, int ell, const double *__restrict__ b, double *__restrict__ g) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * ell) return;
    int i = (int)(idx % n), j = (int)(idx / n);
    g[idx] = b[(long long)(j + 1) * n + i] - b[i];
}

__global__ void k_pad_traj(int n, int N, int pad_l, int ext_len, const double *__restrict__ traj,
                           double *__restrict__ out) {
    const int m = blockIdx.y, st = blockIdx.z;
    const double *row = traj + ((long long)m * (N + 1) + st) * n;
    double *o = out + ((long long)m * N + st) * ext_len;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ext_len; j += gridDim.x * blockDim.x) {
        int i = (j - pad_l) % n;
        o[j] = row[i < 0 ? i + n : i];
    }
}

// The device's constant-rate clock at the moment this (one-thread) kernel runs.
__global__ void k_stamp(long long *p) { *p = wall_clock64(); }

__global__ void k_fill_int(int count, int value, int *__restrict__ p) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_gather_info(int np, const int32_t *const *__restrict__ info, int32_t *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) {
        out[2 * i] = info[i][5];
        out[2 * i + 1] = info[i][4];
    }
}

}  // namespace

hipError_t launch_gather_info(hipStream_t s, int np, const int32_t *const *info, int32_t *out) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_info, dim3((np + 255) / 256), dim3(256), 0, s, np, info, out);
    return hipGetLastError();
}

hipError_t launch_stamp(hipStream_t s, long long *p) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_int(hipStream_t s, int count, int value, int *p) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, count, value, p);
    return hipGetLastError();
}

hipError_t launch_pad_traj(hipStream_t s, int n, int N, int nm, const double *traj, int pad_l, int ext_len,
                           double *out) {
    if (nm <= 0 || N <= 0) return hipSuccess;
    const int bx = (ext_len + 255) / 256;
    hipLaunchKernelGGL(k_pad_traj, dim3(bx, nm, N), dim3(256), 0, s, n, N, pad_l, ext_len, traj, out);
    return hipGetLastError();
}

hipError_t launch_ub_row(hipStream_t s, int n, double sigma_b, double len_b, double *row) {
    double amp = sigma_b * pow(2.0 / M_PI, 0.25) / sqrt(len_b);
    hipLaunchKernelGGL(k_ub_row, dim3((n + 255) / 256), dim3(256), 0, s, n, amp, len_b * len_b, row);
    return hipGetLastError();
}

hipError_t launch_ub_row_diffusion(hipStream_t s, int n, double sigma_b, double daley, int steps, double *row) {
    if (n < 4 || n > 4096 || steps < 2 || (steps & 1) || !(daley > 0)) return hipErrorInvalidValue;
    const double kappa = daley * daley / (2.0 * steps - 3.0);
    hipLaunchKernelGGL(k_ub_row_diffusion, dim3(1), dim3(1024), 2 * n * sizeof(double), s, n, kappa, steps / 2,
                       sigma_b, row);
    return hipGetLastError();
}

hipError_t launch_ub_fill(hipStream_t s, int n, const double *row, double *ub) {
    long long tot = (long long)n * n;
    hipLaunchKernelGGL(k_ub_fill, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, row, ub);
    return hipGetLastError();
}

hipError_t launch_band_conv(hipStream_t s, int n, int nb, int lo, int hi, const double *row, const double *X,
                            long long ldx, double *Y, long long ldy, const double *Add, long long ldadd,
                            const int32_t *active) {
    if (nb <= 0) return hipSuccess;
    int W = hi - lo + 1;
    size_t lds = sizeof(double) * (size_t)(W + CONV_ROWS + W);
    dim3 grid((n + CONV_ROWS - 1) / CONV_ROWS, nb);
    hipLaunchKernelGGL(k_band_conv, grid, dim3(CONV_T), lds, s, n, lo, hi, row, X, ldx, Y, ldy, Add, ldadd,
                       active);
    return hipGetLastError();
}

hipError_t launch_obs(hipStream_t s, int n, int L, int p, int nv, int obs_dt, int obs_dx, int obs_x0,
                      double sigma_o, const double *truth, const double *eta, double *y) {
    hipLaunchKernelGGL(k_obs, dim3((p + 255) / 256), dim3(256), 0, s, n, L, p, nv, obs_dt, obs_dx, obs_x0,
                       sigma_o, truth, eta, y);
    return hipGetLastError();
}

hipError_t launch_xb(hipStream_t s, int n, int L, const double *xt0, const double *ux, double *xb) {
    hipLaunchKernelGGL(k_xb, dim3((n + 255) / 256), dim3(256), 0, s, n, L, xt0, ux, xb);
    return hipGetLastError();
}

hipError_t launch_innov(hipStream_t s, int n, int N, int L, int p, int nv, int obs_dt, int obs_dx, int obs_x0,
                        double s2, const double *y, const double *traj, double *d, double *force, double *costc) {
    hipLaunchKernelGGL(k_innov, dim3(L + 1), dim3(256), 0, s, n, N, p, nv, obs_dt, obs_dx, obs_x0, s2, y, traj,
                       d, force, costc);
    return hipGetLastError();
}

hipError_t launch_gamma(hipStream_t s, int n, int ell, const double *b, double *gam) {
    long long tot = (long long)n * ell;
    hipLaunchKernelGGL(k_gamma, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, ell, b, gam);
    return hipGetLastError();
}

}  // namespace eda

// The learned sketch: a small MLP mapping the control member's right-hand side
// to k sketch directions (n x k), trained in FP32 on Ritz pairs the method
// computes and run in BF16 for inference.
//
//   x = b_0 / ||b_0|| sqrt(n);  h1 = gelu(W1 x + b1);  h2 = gelu(W2 h1 + b2);
//   o = W3 h2 + b3;  Z[:, j] = o[j n : (j + 1) n]
//   loss = ||Z Z^T - S diag(D) S^T||_F^2 / ||D||^2   (S orthonormal, so on k x k
//          blocks: (||Z^T Z||^2 - 2 ||diag(D)^1/2 S^T Z||^2 + ||D||^2) / ||D||^2)
//   dL/dZ = 4 (Z (Z^T Z) - S diag(D) (S^T Z)) / ||D||^2
// gelu is the exact erf form.  Parameters: one flat FP32 array, column-major
// W1 (h x n), b1, W2 (h x h), b2, W3 (k n x h), b3.  Activations are column-
// major with one column per sample.
//
// Kernels: an FP32 MFMA GEMM with either operand transposed (the layer products
// and their gradients), bias/GELU epilogues, per-row sums (bias gradients), the
// per-sample loss and dZ, Adam, He initialisation, and BF16 conversion.
#include "eda_internal.h"

namespace eda {
namespace {

typedef float float4v __attribute__((ext_vector_type(4)));
constexpr int BM = 64, BN = 64, BK = 32;

// C = alpha op(A) op(B) + beta C, FP32, column-major, op(A) M x K, op(B) K x N.
// Staging maps consecutive threads to consecutive memory of each operand.
// blockIdx.z selects a K range of kchunk; with part != null the raw partial
// product goes to part[z][M x N] (summed later in a fixed order).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, float alpha, const float *__restrict__ A,
                                               long long lda, const float *__restrict__ B, long long ldb, float beta,
                                               float *__restrict__ C, long long ldc, int kchunk,
                                               float *__restrict__ part) {
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    float4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = float4v{0.f, 0.f, 0.f, 0.f};
    float ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            int r, kk;
            if (!TA) {
                r = idx % BM;
                kk = idx / BM;
            } else {
                kk = idx % BK;
                r = idx / BK;
            }
            const int gi = i0 + r, gk = k0 + kk;
            ra[e] = (gi < M && gk < kend) ? (TA ? A[gk + (long long)gi * lda] : A[gi + (long long)gk * lda]) : 0.f;
            int c, kb;
            if (!TB) {
                kb = idx % BK;
                c = idx / BK;
            } else {
                c = idx % BN;
                kb = idx / BN;
            }
            const int gj = j0 + c, gkb = k0 + kb;
            rb[e] = (gj < N && gkb < kend) ? (TB ? B[gj + (long long)gkb * ldb] : B[gkb + (long long)gj * ldb]) : 0.f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            if (!TA)
                As[idx / BM][idx % BM] = ra[e];
            else
                As[idx % BK][idx / BK] = ra[e];
            if (!TB)
                Bs[idx % BK][idx / BK] = rb[e];
            else
                Bs[idx / BN][idx % BN] = rb[e];
        }
    };
    if (kbeg < kend) {
        load(kbeg);
        for (int k0 = kbeg; k0 < kend; k0 += BK) {
            store();
            __syncthreads();
            if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
            for (int ks = 0; ks < BK / 4; ks++) {
                const int kk = ks * 4 + (lane >> 4);
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; a++) av[a] = As[kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < 2; b++) bv[b] = Bs[kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[b], av[a], acc[a][b], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    // fed (B^T, A^T): element v of lane l is C[row = l % 16][col = 4 (l / 16) + v] of the block
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = i0 + wr * 32 + a * 16 + (lane & 15);
                const int col = j0 + wc * 32 + b * 16 + 4 * (lane >> 4) + v;
                if (row < M && col < N) {
                    if (part) {
                        part[(long long)blockIdx.z * M * N + row + (long long)col * M] = acc[a][b][v];
                    } else {
                        float *cp = C + row + (long long)col * ldc;
                        const float val = alpha * acc[a][b][v];
                        *cp = beta == 0.f ? val : val + beta * *cp;
                    }
                }
            }
}

__global__ void k_sreduce(int M, int N, int ns, const float *__restrict__ part, float alpha, float beta,
                          float *__restrict__ C, long long ldc) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)M * N) return;
    const int row = (int)(idx % M), col = (int)(idx / M);
    float sum = 0.f;
    for (int z = 0; z < ns; z++) sum += part[(long long)z * M * N + idx];
    float *cp = C + row + (long long)col * ldc;
    *cp = beta == 0.f ? alpha * sum : alpha * sum + beta * *cp;
}

// x[:, c] = b[:, c] / ||b[:, c]|| sqrt(n) in FP32 (training inputs), one workgroup per column
__global__ __launch_bounds__(256) void k_normalise_f(int n, const double *__restrict__ b, long long ldb,
                                                     float *__restrict__ x) {
    __shared__ double red[4];
    const double *bc = b + (long long)blockIdx.x * ldb;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += bc[i] * bc[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double nrm = sqrt(((red[0] + red[1]) + (red[2] + red[3])));
    const double f = nrm > 0 ? sqrt((double)n) / nrm : 0.0;
    for (int i = threadIdx.x; i < n; i += 256) x[(long long)blockIdx.x * n + i] = (float)(bc[i] * f);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}
__device__ __forceinline__ double gelu_d(double x) { return 0.5 * x * (1.0 + erf(x * 0.70710678118654752440)); }

// P += b (per row); H = gelu(P) (H may be null: bias only)
__global__ void k_bias_gelu(int rows, int cols, float *__restrict__ P, const float *__restrict__ b,
                            float *__restrict__ H) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)rows * cols) return;
    const float v = P[i] + b[i % rows];
    P[i] = v;
    if (H) H[i] = gelu_f(v);
}

// dP = dH * gelu'(P)
__global__ void k_gelu_bwd(long long count, const float *__restrict__ dH, const float *__restrict__ P,
                           float *__restrict__ dP) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dP[i] = dH[i] * gelu_grad_f(P[i]);
}

// db[r] = sum_c dX[r + c rows], fixed order
__global__ void k_rowsum(int rows, int cols, const float *__restrict__ dX, float *__restrict__ db) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float s = 0.f;
    for (int c = 0; c < cols; c++) s += dX[r + (long long)c * rows];
    db[r] = s;
}

// One workgroup per sample: G = Z^T Z, M = S^T Z (k <= 32) accumulated over
// 32-row chunks staged in LDS, the loss, and dO[:, b] = dL/dZ / B.
constexpr int LT = 256;
__global__ __launch_bounds__(LT) void k_loss(int n, int k, int B, const float *__restrict__ O,
                                             const float *__restrict__ S, const float *__restrict__ D,
                                             float *__restrict__ dO, double *__restrict__ loss) {
    __shared__ float Zc[32][33], Sc[32][33];
    __shared__ float G[32][33], DM[32][33];
    __shared__ double red[LT / 64];
    const int b = blockIdx.x, tid = threadIdx.x;
    const float *Z = O + (long long)b * n * k;  // n x k, column-major
    const float *Sb = S + (long long)b * n * k;
    const float *Db = D + (long long)b * k;
    float g[4] = {0.f, 0.f, 0.f, 0.f}, m[4] = {0.f, 0.f, 0.f, 0.f};
    for (int r0 = 0; r0 < n; r0 += 32) {
        for (int e = tid; e < 32 * 32; e += LT) {
            const int r = e % 32, j = e / 32;
            const bool ok = r0 + r < n && j < k;
            Zc[r][j] = ok ? Z[r0 + r + (long long)j * n] : 0.f;
            Sc[r][j] = ok ? Sb[r0 + r + (long long)j * n] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int e = tid + LT * q, i = e % 32, j = e / 32;
            float gs = 0.f, ms = 0.f;
            for (int r = 0; r < 32; r++) {
                gs += Zc[r][i] * Zc[r][j];
                ms += Sc[r][i] * Zc[r][j];
            }
            g[q] += gs;
            m[q] += ms;
        }
        __syncthreads();
    }
    double dd = 0.0;
    for (int i = 0; i < k; i++) dd += (double)Db[i] * Db[i];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int e = tid + LT * q, i = e % 32, j = e / 32;
        const float di = i < k ? Db[i] : 0.f;
        G[i][j] = g[q];
        DM[i][j] = di * m[q];
        if (i < k && j < k) part += (double)g[q] * g[q] - 2.0 * (double)di * m[q] * m[q];
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < LT / 64; w++) s += red[w];
        loss[b] = (s + dd) / dd;
    }
    const float scale = (float)(4.0 / dd / B);
    float *dz = dO + (long long)b * n * k;
    for (long long e = tid; e < (long long)n * k; e += LT) {
        const int r = (int)(e % n), j = (int)(e / n);
        float v = 0.f;
        for (int i = 0; i < k; i++) v += Z[r + (long long)i * n] * G[i][j] - Sb[r + (long long)i * n] * DM[i][j];
        dz[e] = scale * v;
    }
}

__global__ void k_adam(long long count, float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// W = normals sqrt(2 / fan_in) on [off, off + len), biases zero
__global__ void k_scale_init(long long off, long long len, float s, const float *__restrict__ z,
                             float *__restrict__ th) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) th[off + i] = s * z[off + i];
}
__global__ void k_zero_f(long long off, long long len, float *__restrict__ th) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) th[off + i] = 0.f;
}

__global__ void k_f32_to_bf16(long long count, const float *__restrict__ x, unsigned short *__restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    unsigned u = __float_as_uint(x[i]);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    y[i] = (unsigned short)(u >> 16);
}

// inference epilogue in FP64: P = P + bf16 bias, optionally gelu
__global__ void k_bias_gelu_d(int rows, const unsigned short *__restrict__ b16, double *__restrict__ P, int act) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const double bias = (double)__uint_as_float((unsigned)b16[i] << 16);
    const double v = P[i] + bias;
    P[i] = act ? gelu_d(v) : v;
}

// x = b / ||b|| sqrt(n) (one vector, one workgroup)
__global__ __launch_bounds__(256) void k_normalise(int n, const double *__restrict__ b, double *__restrict__ x) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += b[i] * b[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double nrm = sqrt(((red[0] + red[1]) + (red[2] + red[3])));
    const double f = nrm > 0 ? sqrt((double)n) / nrm : 0.0;
    for (int i = threadIdx.x; i < n; i += 256) x[i] = b[i] * f;
}

inline unsigned blocks_for(long long count, int t = 256) { return (unsigned)((count + t - 1) / t); }

}  // namespace

// Split-K when the output has few tiles and K is long (the W3^T dO product):
// about 256 workgroups, at least 256 of K each.
int sgemm_splits(int M, int N, int K) {
    const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles >= 64 || K < 1024) return 1;
    int ns = 256 / tiles, cap = K / 256;
    if (ns > cap) ns = cap;
    return ns < 1 ? 1 : ns;
}

size_t sgemm_part_floats(int M, int N, int K) {
    const int ns = sgemm_splits(M, N, K);
    return ns > 1 ? (size_t)ns * M * N : 0;
}

hipError_t sgemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, float alpha, const float *A, long long lda,
                 const float *B, long long ldb, float beta, float *C, long long ldc, float *part) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int ns = part ? sgemm_splits(M, N, K) : 1;
    int kchunk = ns > 1 ? (((K + ns - 1) / ns + BK - 1) / BK) * BK : (K > 0 ? K : 1);
    if (ns > 1) ns = (K + kchunk - 1) / kchunk;
    float *pp = ns > 1 ? part : nullptr;
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, ns);
    if (!ta && !tb)
        hipLaunchKernelGGL((k_sgemm<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                           kchunk, pp);
    else if (ta && !tb)
        hipLaunchKernelGGL((k_sgemm<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                           kchunk, pp);
    else if (!ta && tb)
        hipLaunchKernelGGL((k_sgemm<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                           kchunk, pp);
    else
        hipLaunchKernelGGL((k_sgemm<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                           kchunk, pp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ns == 1) return e;
    const long long tot = (long long)M * N;
    hipLaunchKernelGGL(k_sreduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, ns, part, alpha, beta, C,
                       ldc);
    return hipGetLastError();
}

hipError_t mlp_normalise(hipStream_t s, int n, int count, const double *b, long long ldb, float *x) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normalise_f, dim3(count), dim3(256), 0, s, n, b, ldb, x);
    return hipGetLastError();
}

MlpLayout mlp_layout(int n, int h, int k) {
    MlpLayout L{};
    L.W1 = 0;
    L.b1 = L.W1 + (long long)h * n;
    L.W2 = L.b1 + h;
    L.b2 = L.W2 + (long long)h * h;
    L.W3 = L.b2 + h;
    L.b3 = L.W3 + (long long)k * n * h;
    L.total = L.b3 + (long long)k * n;
    return L;
}

size_t mlp_ws_floats(int n, int h, int k, int B) {
    // P1, H1, P2, H2 (h x B each), O (k n x B), dO (k n x B), dH (h x B), dP (h x B), split-K partials
    return (size_t)B * (6 * (size_t)h + 2 * (size_t)k * n) + sgemm_part_floats(h, B, k * n);
}

hipError_t mlp_init(hipStream_t s, int n, int h, int k, const float *z, float *th) {
    const MlpLayout L = mlp_layout(n, h, k);
    const long long wo[3] = {L.W1, L.W2, L.W3}, wl[3] = {(long long)h * n, (long long)h * h, (long long)k * n * h};
    const int fan[3] = {n, h, h};
    const long long bo[3] = {L.b1, L.b2, L.b3}, bl[3] = {h, h, (long long)k * n};
    for (int i = 0; i < 3; i++) {
        hipLaunchKernelGGL(k_scale_init, dim3(blocks_for(wl[i])), dim3(256), 0, s, wo[i], wl[i],
                           sqrtf(2.0f / fan[i]), z, th);
        hipLaunchKernelGGL(k_zero_f, dim3(blocks_for(bl[i])), dim3(256), 0, s, bo[i], bl[i], th);
    }
    return hipGetLastError();
}

hipError_t mlp_forward(hipStream_t s, int n, int h, int k, int B, const float *th, const float *X, float *ws) {
    const MlpLayout L = mlp_layout(n, h, k);
    const long long kn = (long long)k * n;
    float *P1 = ws, *H1 = P1 + (size_t)h * B, *P2 = H1 + (size_t)h * B, *H2 = P2 + (size_t)h * B,
          *O = H2 + (size_t)h * B;
    hipError_t e;
    if ((e = sgemm(s, false, false, h, B, n, 1.f, th + L.W1, h, X, n, 0.f, P1, h, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks_for((long long)h * B)), dim3(256), 0, s, h, B, P1, th + L.b1, H1);
    if ((e = sgemm(s, false, false, h, B, h, 1.f, th + L.W2, h, H1, h, 0.f, P2, h, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks_for((long long)h * B)), dim3(256), 0, s, h, B, P2, th + L.b2, H2);
    if ((e = sgemm(s, false, false, (int)kn, B, h, 1.f, th + L.W3, kn, H2, h, 0.f, O, kn, nullptr)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks_for(kn * B)), dim3(256), 0, s, (int)kn, B, O, th + L.b3,
                       (float *)nullptr);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(hipStream_t s, int n, int h, int k, int B, const float *th, const float *X,
                         const float *S, const float *D, float *grad, float *ws, double *loss_per_sample) {
    const MlpLayout L = mlp_layout(n, h, k);
    const long long kn = (long long)k * n;
    hipError_t e;
    if ((e = mlp_forward(s, n, h, k, B, th, X, ws)) != hipSuccess) return e;
    float *P1 = ws, *H1 = P1 + (size_t)h * B, *P2 = H1 + (size_t)h * B, *H2 = P2 + (size_t)h * B,
          *O = H2 + (size_t)h * B, *dO = O + (size_t)kn * B, *dH = dO + (size_t)kn * B, *dP = dH + (size_t)h * B,
          *part = dP + (size_t)h * B;
    hipLaunchKernelGGL(k_loss, dim3(B), dim3(LT), 0, s, n, k, B, O, S, D, dO, loss_per_sample);
    if (!grad) return hipGetLastError();
    // layer 3: dW3 = dO H2^T, db3 = rowsum dO, dH2 = W3^T dO
    if ((e = sgemm(s, false, true, (int)kn, h, B, 1.f, dO, kn, H2, h, 0.f, grad + L.W3, kn, nullptr)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_rowsum, dim3(blocks_for(kn)), dim3(256), 0, s, (int)kn, B, dO, grad + L.b3);
    if ((e = sgemm(s, true, false, h, B, (int)kn, 1.f, th + L.W3, kn, dO, kn, 0.f, dH, h, part)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for((long long)h * B)), dim3(256), 0, s, (long long)h * B, dH, P2, dP);
    // layer 2
    if ((e = sgemm(s, false, true, h, h, B, 1.f, dP, h, H1, h, 0.f, grad + L.W2, h, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowsum, dim3(blocks_for(h)), dim3(256), 0, s, h, B, dP, grad + L.b2);
    if ((e = sgemm(s, true, false, h, B, h, 1.f, th + L.W2, h, dP, h, 0.f, dH, h, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for((long long)h * B)), dim3(256), 0, s, (long long)h * B, dH, P1, dP);
    // layer 1
    if ((e = sgemm(s, false, true, h, n, B, 1.f, dP, h, X, n, 0.f, grad + L.W1, h, nullptr)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowsum, dim3(blocks_for(h)), dim3(256), 0, s, h, B, dP, grad + L.b1);
    return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t s, long long count, float *th, const float *g, float *m, float *v, int step, float lr,
                    float b1, float b2, float eps) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(count)), dim3(256), 0, s, count, th, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(hipStream_t s, long long count, const float *th, unsigned short *th16) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks_for(count)), dim3(256), 0, s, count, th, th16);
    return hipGetLastError();
}

// BF16 inference for one input vector b (FP64): Z (k n, FP64) = MLP(b / ||b|| sqrt(n)).
// tmp: n + 2 h doubles.
hipError_t mlp_infer_bf16(hipStream_t s, int n, int h, int k, const unsigned short *th16, const double *b, double *Z,
                          double *tmp) {
    const MlpLayout L = mlp_layout(n, h, k);
    const long long kn = (long long)k * n;
    double *x = tmp, *h1 = tmp + n, *h2 = h1 + h;
    hipError_t e;
    hipLaunchKernelGGL(k_normalise, dim3(1), dim3(256), 0, s, n, b, x);
    if ((e = gemm_bf16(s, h, 1, n, th16 + L.W1, h, x, n, h1, h, nullptr, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu_d, dim3(blocks_for(h)), dim3(256), 0, s, h, th16 + L.b1, h1, 1);
    if ((e = gemm_bf16(s, h, 1, h, th16 + L.W2, h, h1, h, h2, h, nullptr, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu_d, dim3(blocks_for(h)), dim3(256), 0, s, h, th16 + L.b2, h2, 1);
    if ((e = gemm_bf16(s, (int)kn, 1, h, th16 + L.W3, kn, h2, h, Z, kn, nullptr, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu_d, dim3(blocks_for(kn)), dim3(256), 0, s, (int)kn, th16 + L.b3, Z, 0);
    return hipGetLastError();
}

}  // namespace eda

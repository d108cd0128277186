// Reduced-precision GEMMs on the matrix cores, column-major C = A B (+ Add),
// FP32 accumulation: BF16 operands (gfx950's v_mfma_f32_16x16x32_bf16, 32 K
// per instruction) and FP32 operands (v_mfma_f32_16x16x4_f32).
// Used for the dense U_B products of the reduced-precision sketch: A is U_B
// held in BF16 (converted once at set-up), B is an FP64 block converted to BF16
// (round to nearest even) as it is staged, C and Add are FP64.  Each product
// element carries the BF16 rounding of both operands (relative 2^-9 each) and an
// FP32 accumulation of K terms.
//
// Tile 64 x 64 per 256-thread workgroup (4 waves 2 x 2, each wave 2 x 2 MFMA
// blocks of 16 x 16), K step 32 staged in LDS.  As in the FP64 GEMM the MFMA
// is fed (B^T, A^T) so that accumulator lanes run along output rows.
//
// Split-K: a product with few output tiles and a long K (the sketch's U_B
// products: 4096 x 64 outputs, K = 4096, 64 tiles) would run 128 dependent K
// steps, each a global round trip, on 64 workgroups.  Workgroup z of the grid
// then takes the K chunk [z kchunk, (z + 1) kchunk), accumulates it in FP32
// and writes it as FP64 partials; the FP64 GEMM's ordered reduction adds the
// chunks (in chunk order) and Add.  The FP32 accumulation covers a chunk
// instead of all of K, so the rounding is no worse than unsplit.
#include "eda_internal.h"

namespace eda {
namespace {

typedef short short8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;

__device__ __forceinline__ unsigned short to_bf16(double d) {
    float f = (float)d;
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__global__ void k_to_bf16(long long count, const double *__restrict__ x, unsigned short *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = to_bf16(x[i]);
}

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const unsigned short *__restrict__ A,
                                                   long long lda, const double *__restrict__ B, long long ldb,
                                                   double *__restrict__ C, long long ldc,
                                                   const double *__restrict__ Add, long long ldadd, int kchunk,
                                                   double *__restrict__ part) {
    // As[k][m], Bs[k][n]; rows padded by 8 bf16 against bank conflicts
    __shared__ unsigned short As[BK][BM + 8];
    __shared__ unsigned short Bs[BK][BN + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);

    float4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = float4v{0.f, 0.f, 0.f, 0.f};

    // staging: 64 x 32 elements of each operand per K step = 8 per thread
    unsigned short ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            const int r = idx % BM, kk = idx / BM;  // A: consecutive threads along rows (column-major)
            const int gi = i0 + r, gk = k0 + kk;
            ra[e] = (gi < M && gk < kend) ? A[gi + (long long)gk * lda] : (unsigned short)0;
            const int kb = idx % BK, cc = idx / BK;  // B: consecutive threads along K
            const int gj = j0 + cc, gkb = k0 + kb;
            rb[e] = (gj < N && gkb < kend) ? to_bf16(B[gkb + (long long)gj * ldb]) : (unsigned short)0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            As[idx / BM][idx % BM] = ra[e];
            Bs[idx % BK][idx / BK] = rb[e];
        }
    };

    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK / 32; ks++) {
            // lane l supplies k = 32 ks + 8 (l / 16) + e, e = 0..7, for both
            // operands (the same k for both, so the dot products are exact
            // whatever order the unit sums them in)
            const int kb = ks * 32 + 8 * (lane >> 4);
            short8 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; a++) {
                const int m = wr * 32 + a * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 8; e++) av[a][e] = (short)As[kb + e][m];
            }
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int nn = wc * 32 + b * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 8; e++) bv[b][e] = (short)Bs[kb + e][nn];
            }
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, bv[b]),
                                                                       __builtin_bit_cast(bf16x8, av[a]), acc[a][b],
                                                                       0, 0, 0);
        }
        __syncthreads();
    }

    // element v of lane l: C[row = l % 16][col = 4 (l / 16) + v] of each block
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = i0 + wr * 32 + a * 16 + (lane & 15);
                const int col = j0 + wc * 32 + b * 16 + 4 * (lane >> 4) + v;
                if (row < M && col < N) {
                    double val = (double)acc[a][b][v];
                    if (part) {
                        part[(long long)blockIdx.z * M * N + (long long)col * M + row] = val;
                    } else {
                        if (Add) val += Add[row + (long long)col * ldadd];
                        C[row + (long long)col * ldc] = val;
                    }
                }
            }
}

// The same product with FP32 operands (v_mfma_f32_16x16x4_f32): A in FP32, B
// rounded to FP32 as it is staged; relative rounding 2^-24 per operand.
__global__ __launch_bounds__(256) void k_gemm_f32in(int M, int N, int K, const float *__restrict__ A, long long lda,
                                                    const double *__restrict__ B, long long ldb,
                                                    double *__restrict__ C, long long ldc,
                                                    const double *__restrict__ Add, long long ldadd, int kchunk,
                                                    double *__restrict__ part) {
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
            const int r = idx % BM, kk = idx / BM;
            const int gi = i0 + r, gk = k0 + kk;
            ra[e] = (gi < M && gk < kend) ? A[gi + (long long)gk * lda] : 0.f;
            const int kb = idx % BK, cc = idx / BK;
            const int gj = j0 + cc, gkb = k0 + kb;
            rb[e] = (gj < N && gkb < kend) ? (float)B[gkb + (long long)gj * ldb] : 0.f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            As[idx / BM][idx % BM] = ra[e];
            Bs[idx % BK][idx / BK] = rb[e];
        }
    };
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ks++) {
            const int kk = ks * 4 + (lane >> 4);  // lane l supplies k = 4 ks + l / 16
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
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = i0 + wr * 32 + a * 16 + (lane & 15);
                const int col = j0 + wc * 32 + b * 16 + 4 * (lane >> 4) + v;
                if (row < M && col < N) {
                    double val = (double)acc[a][b][v];
                    if (part) {
                        part[(long long)blockIdx.z * M * N + (long long)col * M + row] = val;
                    } else {
                        if (Add) val += Add[row + (long long)col * ldadd];
                        C[row + (long long)col * ldc] = val;
                    }
                }
            }
}

__global__ void k_to_f32(long long count, const double *__restrict__ x, float *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

}  // namespace

hipError_t launch_to_f32(hipStream_t s, long long count, const double *x, float *y) {
    if (count <= 0) return hipSuccess;
    long long blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, s, count, x, y);
    return hipGetLastError();
}

// K chunks of a reduced-precision product: about 512 workgroups in all, each
// chunk at least 256 long; 1 (no split) when the output has 256 tiles or
// more or K is short.
static int lowp_split_count(int M, int N, int K) {
    const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles >= 256 || K < 512) return 1;
    int ns = 512 / tiles;
    if (ns > K / 256) ns = K / 256;
    return ns < 1 ? 1 : ns;
}

// The split taken (1 if the partials do not fit `part`) and its chunk length,
// a multiple of the K step.
static int lowp_split(int M, int N, int K, const double *part, size_t part_elems, int *kchunk) {
    int ns = lowp_split_count(M, N, K);
    if (ns > 1 && (part == nullptr || part_elems < (size_t)ns * M * N)) ns = 1;
    *kchunk = ns > 1 ? (((K + ns - 1) / ns + BK - 1) / BK) * BK : (K > 0 ? K : 1);
    return ns > 1 ? (K + *kchunk - 1) / *kchunk : 1;
}

hipError_t gemm_f32in(hipStream_t s, int M, int N, int K, const float *A, long long lda, const double *B,
                      long long ldb, double *C, long long ldc, const double *Add, long long ldadd, double *part,
                      size_t part_elems) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int kchunk;
    const int ns = lowp_split(M, N, K, part, part_elems, &kchunk);
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, ns);
    hipLaunchKernelGGL(k_gemm_f32in, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, Add, ldadd, kchunk,
                       ns > 1 ? part : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ns == 1) return e;
    return launch_splitk_reduce(s, M, N, ns, part, C, ldc, Add, ldadd);
}

size_t gemm_lowp_splitk_elems(int M, int N, int K) {
    const int ns = lowp_split_count(M, N, K);
    return ns > 1 ? (size_t)ns * M * N : 0;
}

hipError_t launch_to_bf16(hipStream_t s, long long count, const double *x, unsigned short *y) {
    if (count <= 0) return hipSuccess;
    long long blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, count, x, y);
    return hipGetLastError();
}

hipError_t gemm_bf16(hipStream_t s, int M, int N, int K, const unsigned short *A, long long lda, const double *B,
                     long long ldb, double *C, long long ldc, const double *Add, long long ldadd, double *part,
                     size_t part_elems) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int kchunk;
    const int ns = lowp_split(M, N, K, part, part_elems, &kchunk);
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, ns);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, Add, ldadd, kchunk,
                       ns > 1 ? part : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ns == 1) return e;
    return launch_splitk_reduce(s, M, N, ns, part, C, ldc, Add, ldadd);
}

}  // namespace eda

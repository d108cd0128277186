// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64), column-major:
//   C = op(A) B (+ Add),  op(A) = A (M x K) or A^T (A stored K x M).
// Used for the dense U_B products, the sketch Gram matrices (Y^T Y, Phi^T Y,
// Q^T A Q), Q = Y R^-1, S = Q U and the LMP's S_k^T X / X + S_k T.
//
// Tile 64 x 64 per 256-thread workgroup (4 waves in a 2 x 2 arrangement, each
// wave 2 x 2 MFMA blocks of 16 x 16), K step 32 staged in LDS.  The MFMA is fed
// B^T and A^T so that accumulator lanes run along the rows of the column-major
// output (coalesced stores).  For the
// K-long, M/N-small products (Gram matrices, S^T X) the K range is split over
// workgroups; partial tiles go to a workspace and are summed in a fixed order,
// so results do not depend on scheduling.
#include "eda_internal.h"

namespace eda {
namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LE = BK * 64 / 256;  // elements of each operand tile loaded per thread

template <bool TA>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const double *__restrict__ A, long long lda,
                                              const double *__restrict__ B, long long ldb, double *__restrict__ C,
                                              long long ldc, const double *__restrict__ Add, long long ldadd,
                                              const double *__restrict__ rowscale, int kchunk,
                                              double *__restrict__ part) {
    __shared__ double As[BK][BM + 2];
    __shared__ double Bs[BK][BN + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);

    double4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = double4v{0.0, 0.0, 0.0, 0.0};

    double ra[LE], rb[LE];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < LE; e++) {
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
            double v = 0.0;
            if (gi < M && gk < kend) v = TA ? A[gk + (long long)gi * lda] : A[gi + (long long)gk * lda];
            ra[e] = v;
            const int kb = idx % BK, cc = idx / BK;
            const int gj = j0 + cc, gkb = k0 + kb;
            rb[e] = (gj < N && gkb < kend) ? B[gkb + (long long)gj * ldb] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < LE; e++) {
            const int idx = tid + 256 * e;
            if (!TA)
                As[idx / BM][idx % BM] = ra[e];
            else
                As[idx % BK][idx / BK] = ra[e];
            Bs[idx % BK][idx / BK] = rb[e];
        }
    };

    if (kbeg < kend) {
        load(kbeg);
        for (int k0 = kbeg; k0 < kend; k0 += BK) {
            store();
            __syncthreads();
            if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
            for (int kq = 0; kq < BK / 4; kq++) {
                const int kk = kq * 4 + (lane >> 4);
                double av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; a++) av[a] = As[kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < 2; b++) bv[b] = Bs[kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[b], av[a], acc[a][b], 0, 0, 0);
            }
            __syncthreads();
        }
    }

    // The MFMA ran on (B^T, A^T), so each 16 x 16 accumulator holds the transposed
    // block: element v of lane l is C[row = l % 16][col = l / 16 + 4 v] of the
    // block, and every store covers 16 consecutive rows of 4 columns.
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int row = i0 + wr * 32 + a * 16 + (lane & 15);
                const int col = j0 + wc * 32 + b * 16 + (lane >> 4) + 4 * v;
                if (row < M && col < N) {
                    double val = acc[a][b][v];
                    if (part) {
                        part[(long long)blockIdx.z * M * N + (long long)col * M + row] = val;
                    } else {
                        if (rowscale) val *= rowscale[row];
                        if (Add) val += Add[row + (long long)col * ldadd];
                        C[row + (long long)col * ldc] = val;
                    }
                }
            }
}

__global__ void k_splitk_reduce(int M, int N, int nsplit, const double *__restrict__ part, double *__restrict__ C,
                                long long ldc, const double *__restrict__ Add, long long ldadd,
                                const double *__restrict__ rowscale) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)M * N) return;
    int row = (int)(idx % M), col = (int)(idx / M);
    double s = 0.0;
#pragma unroll 8
    for (int z = 0; z < nsplit; z++) s += part[(long long)z * M * N + idx];  // fixed order
    if (rowscale) s *= rowscale[row];
    if (Add) s += Add[row + (long long)col * ldadd];
    C[row + (long long)col * ldc] = s;
}

// K-split for products whose output has few tiles: aim at about 256
// workgroups, with at least 128 of K per workgroup (the partial sums cost
// nsplit M N doubles written and read again).
int split_count(int M, int N, int K) {
    int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles >= 128 || K < 256) return 1;
    int ns = 256 / tiles;
    int cap = K / 128;
    if (ns > cap) ns = cap;
    return ns < 1 ? 1 : ns;
}

}  // namespace

hipError_t launch_splitk_reduce(hipStream_t s, int M, int N, int nsplit, const double *part, double *C,
                                long long ldc, const double *Add, long long ldadd) {
    const long long tot = (long long)M * N;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, nsplit, part, C,
                       ldc, Add, ldadd, nullptr);
    return hipGetLastError();
}

size_t gemm_splitk_elems(int M, int N, int K) {
    int ns = split_count(M, N, K);
    return ns > 1 ? (size_t)ns * M * N : 0;
}

hipError_t gemm_f64(hipStream_t s, bool trans_a, int M, int N, int K, const double *A, long long lda,
                    const double *B, long long ldb, double *C, long long ldc, const double *Add,
                    long long ldadd, const double *rowscale, double *part, size_t part_elems) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int ns = split_count(M, N, K);
    if (ns > 1 && (part == nullptr || part_elems < (size_t)ns * M * N)) ns = 1;
    int kchunk = ns > 1 ? (((K + ns - 1) / ns + BK - 1) / BK) * BK : (K > 0 ? K : 1);
    if (ns > 1) ns = (K + kchunk - 1) / kchunk;
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, ns);
    double *pp = ns > 1 ? part : nullptr;
    if (trans_a)
        hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, Add, ldadd,
                           rowscale, kchunk, pp);
    else
        hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, Add, ldadd,
                           rowscale, kchunk, pp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ns == 1) return e;
    long long tot = (long long)M * N;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, ns, part, C,
                       ldc, Add, ldadd, rowscale);
    return hipGetLastError();
}

}  // namespace eda

// Products with the margin blocks of a partitioned array operator (paper
// Sec. II-A eq. (Zblock), Sec. II-B eq. (Z2)): Z = [[Z_A, Z_B^T], [Z_B, Z_C]]
// with the element unknowns first and the N_C margin unknowns after them.
// Z_A is applied by the lattice FFT; Z_B (N_C x N_A, row-major), Z_C and the
// margin's preconditioner block are dense and applied here, on RHS-innermost
// vectors x[n][r], by one tiled complex product
//     Y[m][r] (+)= sum_k op(A)(m, k) X[k][r],   op(A)(m, k) = A[m sm + k sk] or its conjugate,
// which covers A, A^T, A^H and A^* through the strides.  A workgroup computes
// 32 rows x 64 RHS; the K loop stages 16-wide chunks of A and X in LDS.  Long
// K (the N_A columns of Z_B) is split over workgroups whose partial tiles are
// summed in a fixed order by a second kernel, so results do not depend on the
// launch.
#include "common.h"

#include <algorithm>

namespace mbt {

namespace {

constexpr int kTM = 32, kTR = 64, kKC = 16;

template <typename T, bool CONJ>
__global__ __launch_bounds__(256) void mgemm_kernel(const cplx<T>* __restrict__ A, int64_t sm, int64_t sk,
                                                    const cplx<T>* __restrict__ X, int64_t sxk, int64_t sxr,
                                                    cplx<T>* __restrict__ Y, int64_t ldy, int Mrows, int64_t K,
                                                    int R, int64_t kchunk, int mode,
                                                    cplx<T>* __restrict__ partial) {
    using C = cplx<T>;
    __shared__ C As[kTM][kKC + 1];
    __shared__ C Xs[kKC][kTR];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int r0 = blockIdx.x * kTR, m0 = blockIdx.y * kTM;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
    C acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = mk<T>(0, 0);
    const bool mfast = (sm == 1);   // A's rows are contiguous in m: load m-fastest
    for (int64_t k0 = kb; k0 < ke; k0 += kKC) {
#pragma unroll
        for (int j = 0; j < (kTM * kKC) / 256; ++j) {
            const int i = tid + 256 * j;
            const int mm = mfast ? i % kTM : i / kKC;
            const int kk = mfast ? i / kTM : i % kKC;
            const int m = m0 + mm;
            const int64_t k = k0 + kk;
            C v = mk<T>(0, 0);
            if (m < Mrows && k < ke) {
                v = A[(int64_t)m * sm + k * sk];
                if (CONJ) v.y = -v.y;
            }
            As[mm][kk] = v;
        }
#pragma unroll
        for (int j = 0; j < (kKC * kTR) / 256; ++j) {
            const int i = tid + 256 * j;
            const int kk = i / kTR, rr = i % kTR;
            const int64_t k = k0 + kk;
            const int r = r0 + rr;
            Xs[kk][rr] = (k < ke && r < R) ? X[k * sxk + (int64_t)r * sxr] : mk<T>(0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKC; ++kk) {
            const C a0 = As[ty * 2][kk], a1 = As[ty * 2 + 1][kk];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const C xv = Xs[kk][tx * 4 + q];
                acc[0][q].x = fma(a0.x, xv.x, acc[0][q].x);
                acc[0][q].x = fma(-a0.y, xv.y, acc[0][q].x);
                acc[0][q].y = fma(a0.x, xv.y, acc[0][q].y);
                acc[0][q].y = fma(a0.y, xv.x, acc[0][q].y);
                acc[1][q].x = fma(a1.x, xv.x, acc[1][q].x);
                acc[1][q].x = fma(-a1.y, xv.y, acc[1][q].x);
                acc[1][q].y = fma(a1.x, xv.y, acc[1][q].y);
                acc[1][q].y = fma(a1.y, xv.x, acc[1][q].y);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = m0 + ty * 2 + i;
        if (m >= Mrows) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + tx * 4 + q;
            if (r >= R) continue;
            if (mode == 2) {
                partial[((int64_t)blockIdx.z * Mrows + m) * R + r] = acc[i][q];
            } else {
                C* yp = Y + (int64_t)m * ldy + r;
                *yp = mode == 1 ? cadd(*yp, acc[i][q]) : acc[i][q];
            }
        }
    }
}

// Y[m][r] (+)= sum over z of partial[z][m][r], in order of z
template <typename T>
__global__ void mgemm_reduce_kernel(const cplx<T>* __restrict__ partial, int nz, cplx<T>* __restrict__ Y, int64_t ldy,
                                    int Mrows, int R, int accumulate) {
    const int64_t n = (int64_t)Mrows * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        cplx<T> s = mk<T>(0, 0);
        for (int z = 0; z < nz; ++z) s = cadd(s, partial[(int64_t)z * n + t]);
        const int64_t m = t / R, r = t % R;
        cplx<T>* yp = Y + m * ldy + r;
        *yp = accumulate ? cadd(*yp, s) : s;
    }
}

}  // namespace

int64_t margin_kchunk(int64_t K) { return K <= 2048 ? K : 1024; }
int margin_ksplit(int64_t K) { return (int)((K + margin_kchunk(K) - 1) / margin_kchunk(K)); }

template <typename T>
void margin_gemm(const cplx<T>* A, int64_t sm, int64_t sk, bool conjA, const cplx<T>* X, int64_t sxk, int64_t sxr,
                 cplx<T>* Y, int64_t ldy, int Mrows, int64_t K, int R, bool accumulate, cplx<T>* partial,
                 hipStream_t s) {
    if (Mrows <= 0 || R <= 0) return;
    const int64_t kc = margin_kchunk(K);
    const int nz = margin_ksplit(K);
    MBT_REQUIRE(nz == 1 || partial != nullptr, "margin product: split-K needs a partial buffer");
    const dim3 grid((unsigned)((R + kTR - 1) / kTR), (unsigned)((Mrows + kTM - 1) / kTM), (unsigned)nz);
    const int mode = nz > 1 ? 2 : (accumulate ? 1 : 0);
    if (conjA)
        hipLaunchKernelGGL((mgemm_kernel<T, true>), grid, dim3(256), 0, s, A, sm, sk, X, sxk, sxr, Y, ldy, Mrows, K, R,
                           kc, mode, partial);
    else
        hipLaunchKernelGGL((mgemm_kernel<T, false>), grid, dim3(256), 0, s, A, sm, sk, X, sxk, sxr, Y, ldy, Mrows, K,
                           R, kc, mode, partial);
    if (nz > 1) {
        const int64_t n = (int64_t)Mrows * R;
        hipLaunchKernelGGL((mgemm_reduce_kernel<T>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                           dim3(256), 0, s, partial, nz, Y, ldy, Mrows, R, accumulate ? 1 : 0);
    }
    MBT_LAUNCH_CHECK();
}

template void margin_gemm<double>(const double2*, int64_t, int64_t, bool, const double2*, int64_t, int64_t, double2*,
                                  int64_t, int, int64_t, int, bool, double2*, hipStream_t);
template void margin_gemm<float>(const float2*, int64_t, int64_t, bool, const float2*, int64_t, int64_t, float2*,
                                 int64_t, int, int64_t, int, bool, float2*, hipStream_t);

}  // namespace mbt

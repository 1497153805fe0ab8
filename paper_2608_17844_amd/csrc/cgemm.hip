// Batched complex block products Y_b = op(A_b) X_b on the matrix cores.
//
// Used for the per-bin products of the FFT-Toeplitz matvec, where A_b is the
// spectrum C^_b of the circulant embedding at bin b (paper eq. (multL)) and
// op = ^H gives Z^H from the same stored spectra (eq. (multCom)), and for the
// block-diagonal preconditioner apply, where A_b is an element's inverse block.
//
// A complex product becomes one real product of twice the size:
//   [Y_re]   [A_re  -A_im] [X_re]
//   [Y_im] = [A_im   A_re] [X_im],
// with the real K index interleaving (q, re/im).  With X stored as interleaved
// complex, a lane that loads X[q][col] feeds both K slots (q, re) and (q, im)
// of a 16x16x4 MFMA pair, so no de-interleaving is needed.  Rows of the real
// result are (p, re/im) pairs, so each lane's four accumulator rows are two
// complete complex outputs.
//
// Each wave keeps its A_b fragments in registers and streams 16-column tiles
// of X_b; M is padded to MP (16 or 32) with predicated loads and stores.  At
// M = 31 the FP64 product has about 8 flop/byte (below the FP64 MFMA ridge of
// 9.8) and the FP32 one about 16 (below 19.7): both are HBM-bound.
#include "common.h"

namespace mbt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { using type = d4; };
template <> struct Acc<float> { using type = f4; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, int MP, bool HERM>
__global__ __launch_bounds__(256) void cgemm_kernel(const cplx<T>* __restrict__ A, int64_t strideA,
                                                    const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Y, int M,
                                                    int R, int groups, int tpw) {
    using C = cplx<T>;
    using V = typename Acc<T>::type;
    constexpr int NRT = MP / 8;   // 16-row tiles of the 2MP-row real matrix
    constexpr int NS = MP / 4;    // complex K groups of 4
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.x / groups;
    const int grp = blockIdx.x % groups;
    const int ntiles = (R + 15) >> 4;
    const int t0 = (grp * 4 + wave) * tpw;
    if (t0 >= ntiles) return;
    const int t1 = min(t0 + tpw, ntiles);

    const C* Ab = A + b * strideA;
    const C* Xb = X + b * (int64_t)M * R;
    C* Yb = Y + b * (int64_t)M * R;
    const int g = lane >> 4;       // lane group: K slot inside a group of 4
    const int li = lane & 15;

    // A fragments: lane li supplies row li of the tile; K slot q = 4s + g.
    // The accumulator of row i sits in lane group i%4, register i/4 for the
    // f64 16x16x4 MFMA, and in lane group i/4, register i%4 for the f32 one;
    // the row -> (p, re/im) assignment is chosen per type so that every lane
    // ends with registers {(p0, re), (p0, im), (p0+1, re), (p0+1, im)},
    // p0 = 8t + 2*(lane/16).
    T are[NRT][NS], aim[NRT][NS];
#pragma unroll
    for (int t = 0; t < NRT; ++t) {
        int p;
        bool odd;
        if constexpr (sizeof(T) == 8) {
            const int v = li >> 2, gg = li & 3;
            p = 8 * t + 2 * gg + (v >> 1);
            odd = v & 1;
        } else {
            const int rho = 16 * t + li;
            p = rho >> 1;
            odd = rho & 1;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = 4 * s + g;
            C c = mk<T>(0, 0);
            if (p < M && q < M) {
                c = HERM ? Ab[(int64_t)q * M + p] : Ab[(int64_t)p * M + q];
                if (HERM) c.y = -c.y;
            }
            are[t][s] = odd ? c.y : c.x;
            aim[t][s] = odd ? c.x : -c.y;
        }
    }

    C bcur[NS], bnext[NS];
    auto load = [&](int tile, C* dst) {
        const int col = tile * 16 + li;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = 4 * s + g;
            dst[s] = (q < M && col < R) ? Xb[(int64_t)q * R + col] : mk<T>(0, 0);
        }
    };
    load(t0, bcur);
    for (int tile = t0; tile < t1; ++tile) {
        if (tile + 1 < t1) load(tile + 1, bnext);
        V acc[NRT];
#pragma unroll
        for (int t = 0; t < NRT; ++t) acc[t] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                acc[t] = mfma(are[t][s], bcur[s].x, acc[t]);
                acc[t] = mfma(aim[t][s], bcur[s].y, acc[t]);
            }
        }
        const int col = tile * 16 + li;
        if (col < R) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                const int p0 = 8 * t + 2 * g;
                if (p0 < M) Yb[(int64_t)p0 * R + col] = mk<T>(acc[t][0], acc[t][1]);
                if (p0 + 1 < M) Yb[(int64_t)(p0 + 1) * R + col] = mk<T>(acc[t][2], acc[t][3]);
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) bcur[s] = bnext[s];
    }
}

// FP32 with an even number of columns: each lane carries two adjacent columns,
// so every access of X and Y is 16 bytes; a wave tile is 32 columns, run as two
// interleaved 16-column MFMA products with the same fragments of A (per column
// the arithmetic and its order are those of cgemm_kernel).
template <int MP, bool HERM>
__global__ __launch_bounds__(256) void cgemm_pair_kernel(const float2* __restrict__ A, int64_t strideA,
                                                         const float2* __restrict__ X, float2* __restrict__ Y, int M,
                                                         int R, int groups, int tpw) {
    using V = f4;
    constexpr int NRT = MP / 8;
    constexpr int NS = MP / 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.x / groups;
    const int grp = blockIdx.x % groups;
    const int ntiles = (R + 31) >> 5;
    const int t0 = (grp * 4 + wave) * tpw;
    if (t0 >= ntiles) return;
    const int t1 = min(t0 + tpw, ntiles);

    const float2* Ab = A + b * strideA;
    const float2* Xb = X + b * (int64_t)M * R;
    float2* Yb = Y + b * (int64_t)M * R;
    const int g = lane >> 4;
    const int li = lane & 15;

    float are[NRT][NS], aim[NRT][NS];
#pragma unroll
    for (int t = 0; t < NRT; ++t) {
        const int rho = 16 * t + li;
        const int p = rho >> 1;
        const bool odd = rho & 1;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = 4 * s + g;
            float2 c = make_float2(0.f, 0.f);
            if (p < M && q < M) {
                c = HERM ? Ab[(int64_t)q * M + p] : Ab[(int64_t)p * M + q];
                if (HERM) c.y = -c.y;
            }
            are[t][s] = odd ? c.y : c.x;
            aim[t][s] = odd ? c.x : -c.y;
        }
    }

    float4 bcur[NS], bnext[NS];
    auto load = [&](int tile, float4* dst) {
        const int col = tile * 32 + 2 * li;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int q = 4 * s + g;
            dst[s] = (q < M && col < R) ? *reinterpret_cast<const float4*>(Xb + (int64_t)q * R + col)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    load(t0, bcur);
    for (int tile = t0; tile < t1; ++tile) {
        if (tile + 1 < t1) load(tile + 1, bnext);
        V acc0[NRT], acc1[NRT];
#pragma unroll
        for (int t = 0; t < NRT; ++t) acc0[t] = acc1[t] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                acc0[t] = mfma(are[t][s], bcur[s].x, acc0[t]);
                acc0[t] = mfma(aim[t][s], bcur[s].y, acc0[t]);
                acc1[t] = mfma(are[t][s], bcur[s].z, acc1[t]);
                acc1[t] = mfma(aim[t][s], bcur[s].w, acc1[t]);
            }
        }
        const int col = tile * 32 + 2 * li;
        if (col < R) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                const int p0 = 8 * t + 2 * g;
                if (p0 < M)
                    *reinterpret_cast<float4*>(Yb + (int64_t)p0 * R + col) =
                        make_float4(acc0[t][0], acc0[t][1], acc1[t][0], acc1[t][1]);
                if (p0 + 1 < M)
                    *reinterpret_cast<float4*>(Yb + (int64_t)(p0 + 1) * R + col) =
                        make_float4(acc0[t][2], acc0[t][3], acc1[t][2], acc1[t][3]);
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) bcur[s] = bnext[s];
    }
}

template <typename T, int MP>
void launch_mp(const cplx<T>* A, int64_t strideA, const cplx<T>* X, cplx<T>* Y, int M, int R, int64_t nbatch,
               int op, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (R % 2 == 0 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15) == 0) {
            const int ntiles = (R + 31) / 32;
            const int64_t total = nbatch * ntiles;
            int tpw = (int)std::max<int64_t>(1, std::min<int64_t>(4, total / 32768));
            if (strideA == 0) tpw = 4;
            tpw = std::min(tpw, ntiles);
            const int groups = (ntiles + 4 * tpw - 1) / (4 * tpw);
            const int64_t blocks = nbatch * groups;
            MBT_REQUIRE(blocks < (1LL << 31), "cgemm: grid too large");
            if (op == 0)
                hipLaunchKernelGGL((cgemm_pair_kernel<MP, false>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA,
                                   X, Y, M, R, groups, tpw);
            else
                hipLaunchKernelGGL((cgemm_pair_kernel<MP, true>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA,
                                   X, Y, M, R, groups, tpw);
            MBT_LAUNCH_CHECK();
            return;
        }
    }
    const int ntiles = (R + 15) / 16;
    const int64_t total = nbatch * ntiles;
    int tpw = (int)std::max<int64_t>(1, std::min<int64_t>(8, total / 32768));
    // one block shared by every batch entry (the element-block preconditioner):
    // longer runs of tiles per wave amortise loading its fragments
    if (strideA == 0) tpw = 8;
    tpw = std::min(tpw, ntiles);
    const int groups = (ntiles + 4 * tpw - 1) / (4 * tpw);
    const int64_t blocks = nbatch * groups;
    MBT_REQUIRE(blocks < (1LL << 31), "cgemm: grid too large");
    if (op == 0)
        hipLaunchKernelGGL((cgemm_kernel<T, MP, false>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA, X, Y, M,
                           R, groups, tpw);
    else
        hipLaunchKernelGGL((cgemm_kernel<T, MP, true>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA, X, Y, M,
                           R, groups, tpw);
    MBT_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- large blocks (M up to 128)
// Blocks too large for register-resident fragments: one workgroup per batch
// entry and group of up to four 16-column tiles; A is staged through LDS in
// chunks of KC complex columns, the four waves split the 16-row tiles of the
// real 2M x 2M product, and the X fragments are read straight from memory into
// registers; the next chunk's A elements and X fragments are loaded while the
// current chunk computes.  At M = 96 and 32 columns a bin moves 123 KB (FP32)
// for 2.4 MFLOP, at the FP32 MFMA ridge.
// PAIR (FP32, Ĉ_b untransposed, even M): each thread loads two adjacent K
// entries of a row of A as one 16-byte access; the LDS stage holds the same values.
template <typename T, int MP, bool HERM, int CT, bool PAIR>
__global__ __launch_bounds__(256) void cgemm_big_kernel(const cplx<T>* __restrict__ A, int64_t strideA,
                                                        const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Y, int M,
                                                        int R) {
    using C = cplx<T>;
    using V = typename Acc<T>::type;
    constexpr int KC = 16;         // complex K per LDS stage (13 KB at M = 96: eight workgroups per CU)
    constexpr int NRT = MP / 8;    // 16-row tiles of the 2MP-row real matrix
    constexpr int RTW = NRT / 4;   // row tiles per wave
    // CT: column tiles per workgroup (1, 2 or 4)
    constexpr int LDA = KC + 1;
    __shared__ C As[MP * LDA];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int li = lane & 15;
    const int64_t b = blockIdx.x;
    const int ct0 = blockIdx.y * CT;
    const int ntiles = (R + 15) >> 4;
    const int nct = min(CT, ntiles - ct0);
    const C* Ab = A + b * strideA;
    const C* Xb = X + b * (int64_t)M * R;
    C* Yb = Y + b * (int64_t)M * R;

    // real row of tile t held by lane li -> (p, re/im), as in cgemm_kernel
    int pr[RTW];
    bool oddr[RTW];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
        const int t = wave + 4 * i;
        if constexpr (sizeof(T) == 8) {
            const int v = li >> 2, gg = li & 3;
            pr[i] = 8 * t + 2 * gg + (v >> 1);
            oddr[i] = v & 1;
        } else {
            const int rho = 16 * t + li;
            pr[i] = rho >> 1;
            oddr[i] = rho & 1;
        }
    }
    V acc[RTW][CT];
#pragma unroll
    for (int i = 0; i < RTW; ++i)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[i][c] = V{0, 0, 0, 0};

    // the next chunk's A elements and X fragments are loaded while this chunk computes
    static_assert(!PAIR || (sizeof(T) == 4 && !HERM), "paired A loads are for FP32 untransposed blocks");
    constexpr int AE = (MP * KC + 255) / 256;
    constexpr int AE2 = (MP * KC / 2 + 255) / 256;
    C areg[PAIR ? 1 : AE];
    float4 areg2[PAIR ? AE2 : 1];
    C xcur[KC / 4][CT], xnxt[KC / 4][CT];
    auto load_a = [&](int kc) {
        if constexpr (PAIR) {
#pragma unroll
            for (int t = 0; t < AE2; ++t) {
                const int e = threadIdx.x + 256 * t;
                const int p = e / (KC / 2), j = 2 * (e - p * (KC / 2)), q = kc + j;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (e < MP * KC / 2 && p < M && q < M) v = *reinterpret_cast<const float4*>(Ab + (int64_t)p * M + q);
                areg2[t] = v;
            }
            return;
        }
#pragma unroll
        for (int t = 0; t < AE; ++t) {
            const int e = threadIdx.x + 256 * t;
            const int p = e / KC, j = e - p * KC, q = kc + j;
            C c = mk<T>(0, 0);
            if (e < MP * KC && p < M && q < M) {
                c = HERM ? Ab[(int64_t)q * M + p] : Ab[(int64_t)p * M + q];
                if (HERM) c.y = -c.y;
            }
            areg[t] = c;
        }
    };
    auto load_x = [&](int kc, C (&xb)[KC / 4][CT]) {
#pragma unroll
        for (int s4 = 0; s4 < KC / 4; ++s4) {
            const int q = kc + 4 * s4 + g;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int col = (ct0 + c) * 16 + li;
                xb[s4][c] = (c < nct && q < M && col < R) ? Xb[(int64_t)q * R + col] : mk<T>(0, 0);
            }
        }
    };
    load_a(0);
    load_x(0, xcur);
    for (int kc = 0; kc < M; kc += KC) {
        __syncthreads();
        if constexpr (PAIR) {
#pragma unroll
            for (int t = 0; t < AE2; ++t) {
                const int e = threadIdx.x + 256 * t;
                if (e < MP * KC / 2) {
                    const int p = e / (KC / 2), j = 2 * (e - p * (KC / 2));
                    As[p * LDA + j] = make_float2(areg2[t].x, areg2[t].y);
                    As[p * LDA + j + 1] = make_float2(areg2[t].z, areg2[t].w);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < AE; ++t) {
                const int e = threadIdx.x + 256 * t;
                if (e < MP * KC) As[(e / KC) * LDA + (e % KC)] = areg[t];
            }
        }
        if (kc + KC < M) {
            load_a(kc + KC);
            load_x(kc + KC, xnxt);
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < KC / 4; ++s4) {
            C bv[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) bv[c] = xcur[s4][c];
#pragma unroll
            for (int i = 0; i < RTW; ++i) {
                const C a = As[pr[i] * LDA + 4 * s4 + g];
                const T are = oddr[i] ? a.y : a.x;
                const T aim = oddr[i] ? a.x : -a.y;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    acc[i][c] = mfma(are, bv[c].x, acc[i][c]);
                    acc[i][c] = mfma(aim, bv[c].y, acc[i][c]);
                }
            }
        }
#pragma unroll
        for (int s4 = 0; s4 < KC / 4; ++s4)
#pragma unroll
            for (int c = 0; c < CT; ++c) xcur[s4][c] = xnxt[s4][c];
    }
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
        const int p0 = 8 * (wave + 4 * i) + 2 * g;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int col = (ct0 + c) * 16 + li;
            if (c < nct && col < R) {
                if (p0 < M) Yb[(int64_t)p0 * R + col] = mk<T>(acc[i][c][0], acc[i][c][1]);
                if (p0 + 1 < M) Yb[(int64_t)(p0 + 1) * R + col] = mk<T>(acc[i][c][2], acc[i][c][3]);
            }
        }
    }
}

template <typename T, int MP, int CT>
void launch_big_ct(const cplx<T>* A, int64_t strideA, const cplx<T>* X, cplx<T>* Y, int M, int R, int64_t nbatch,
                   int op, hipStream_t s) {
    const int ntiles = (R + 15) / 16;
    const int groups = (ntiles + CT - 1) / CT;
    MBT_REQUIRE(nbatch < (1LL << 31) && groups < 65536, "cgemm: grid too large");
    const dim3 grid((unsigned)nbatch, (unsigned)groups);
    const bool pair = sizeof(T) == 4 && op == 0 && M % 2 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    if (op == 0 && pair) {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((cgemm_big_kernel<T, MP, false, CT, true>), grid, dim3(256), 0, s, A, strideA, X, Y, M,
                               R);
    } else if (op == 0)
        hipLaunchKernelGGL((cgemm_big_kernel<T, MP, false, CT, false>), grid, dim3(256), 0, s, A, strideA, X, Y, M, R);
    else
        hipLaunchKernelGGL((cgemm_big_kernel<T, MP, true, CT, false>), grid, dim3(256), 0, s, A, strideA, X, Y, M, R);
    MBT_LAUNCH_CHECK();
}

// as few column tiles per workgroup as cover R (no MFMA work on padding columns)
template <typename T, int MP>
void launch_big(const cplx<T>* A, int64_t strideA, const cplx<T>* X, cplx<T>* Y, int M, int R, int64_t nbatch, int op,
                hipStream_t s) {
    if (R <= 16) launch_big_ct<T, MP, 1>(A, strideA, X, Y, M, R, nbatch, op, s);
    else if (R <= 32) launch_big_ct<T, MP, 2>(A, strideA, X, Y, M, R, nbatch, op, s);
    else launch_big_ct<T, MP, 4>(A, strideA, X, Y, M, R, nbatch, op, s);
}

// ---------------------------------------------------------------- 16-bit inputs
// The same real formulation on gfx950's doubled-K 16x16x32 MFMA with 16-bit
// inputs and FP32 accumulation.  A lane supplies eight consecutive K values;
// with K interleaving (q, re/im), K slots 8g..8g+7 of a 32-wide block are the
// four complex values X[q0..q0+3][col] (q0 = 16s + 4g), i.e. four packed 32-bit
// words as they sit in memory.  The A row (p, re) needs (A.re, -A.im) pairs and
// the row (p, im) the swapped (A.im, A.re) pairs: a sign-bit flip and a
// half-word rotation of the packed words.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4w __attribute__((ext_vector_type(4)));

template <int FMT> __device__ __forceinline__ f4 mfma16(u4w a, u4w b, f4 c) {
    if constexpr (FMT == kFmtBf16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                       0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}

template <int FMT, int MP, bool HERM>
__global__ __launch_bounds__(256) void cgemm16_kernel(const uint32_t* __restrict__ A, int64_t strideA,
                                                      const uint32_t* __restrict__ X, float2* __restrict__ Y, int M,
                                                      int R, int groups, int tpw, float osc) {
    static_assert(MP % 16 == 0, "MP must be a multiple of 16");
    constexpr int NRT = MP / 8;    // 16-row tiles of the 2MP-row real matrix
    constexpr int NKB = MP / 16;   // 32-wide real K blocks (16 complex q each)
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.x / groups;
    const int grp = blockIdx.x % groups;
    const int ntiles = (R + 15) >> 4;
    const int t0 = (grp * 4 + wave) * tpw;
    if (t0 >= ntiles) return;
    const int t1 = min(t0 + tpw, ntiles);

    const uint32_t* Ab = A + b * strideA;
    const uint32_t* Xb = X + b * (int64_t)M * R;
    float2* Yb = Y + b * (int64_t)M * R;
    const int g = lane >> 4;
    const int li = lane & 15;

    // A fragments: row rho = 16t + li of the real matrix is (p, re/im), p = rho/2
    u4w af[NRT][NKB];
#pragma unroll
    for (int t = 0; t < NRT; ++t) {
        const int rho = 16 * t + li;
        const int p = rho >> 1;
        const bool odd = rho & 1;
#pragma unroll
        for (int s = 0; s < NKB; ++s) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int q = 16 * s + 4 * g + h;
                uint32_t w = 0;
                if (p < M && q < M) {
                    w = HERM ? Ab[(int64_t)q * M + p] : Ab[(int64_t)p * M + q];
                    if (HERM) w ^= 0x80000000u;   // conjugate
                }
                af[t][s][h] = odd ? ((w >> 16) | (w << 16)) : (w ^ 0x80000000u);
            }
        }
    }

    u4w bcur[NKB], bnext[NKB];
    auto load = [&](int tile, u4w* dst) {
        const int col = tile * 16 + li;
#pragma unroll
        for (int s = 0; s < NKB; ++s) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int q = 16 * s + 4 * g + h;
                dst[s][h] = (q < M && col < R) ? Xb[(int64_t)q * R + col] : 0u;
            }
        }
    };
    load(t0, bcur);
    for (int tile = t0; tile < t1; ++tile) {
        if (tile + 1 < t1) load(tile + 1, bnext);
        f4 acc[NRT];
#pragma unroll
        for (int t = 0; t < NRT; ++t) acc[t] = f4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NKB; ++s) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) acc[t] = mfma16<FMT>(af[t][s], bcur[s], acc[t]);
        }
        const int col = tile * 16 + li;
        if (col < R) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                const int p0 = 8 * t + 2 * g;
                if (p0 < M) Yb[(int64_t)p0 * R + col] = make_float2(acc[t][0] * osc, acc[t][1] * osc);
                if (p0 + 1 < M) Yb[(int64_t)(p0 + 1) * R + col] = make_float2(acc[t][2] * osc, acc[t][3] * osc);
            }
        }
#pragma unroll
        for (int s = 0; s < NKB; ++s) bcur[s] = bnext[s];
    }
}

template <int FMT, int MP>
void launch16_mp(const uint32_t* A, int64_t strideA, const uint32_t* X, float2* Y, int M, int R, int64_t nbatch,
                 int op, float osc, hipStream_t s) {
    const int ntiles = (R + 15) / 16;
    const int64_t total = nbatch * ntiles;
    int tpw = (int)std::max<int64_t>(1, std::min<int64_t>(8, total / 32768));
    tpw = std::min(tpw, ntiles);
    const int groups = (ntiles + 4 * tpw - 1) / (4 * tpw);
    const int64_t blocks = nbatch * groups;
    MBT_REQUIRE(blocks < (1LL << 31), "cgemm: grid too large");
    if (op == 0)
        hipLaunchKernelGGL((cgemm16_kernel<FMT, MP, false>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA, X, Y,
                           M, R, groups, tpw, osc);
    else
        hipLaunchKernelGGL((cgemm16_kernel<FMT, MP, true>), dim3((unsigned)blocks), dim3(256), 0, s, A, strideA, X, Y,
                           M, R, groups, tpw, osc);
    MBT_LAUNCH_CHECK();
}

}  // namespace

template <int FMT>
void cgemm16_batched(const uint32_t* A, int64_t strideA, const uint32_t* X, float2* Y, int M, int R, int64_t nbatch,
                     int op, float out_scale, hipStream_t s) {
    if (nbatch <= 0 || R <= 0) return;
    if (M <= 16) launch16_mp<FMT, 16>(A, strideA, X, Y, M, R, nbatch, op, out_scale, s);
    else if (M <= 32) launch16_mp<FMT, 32>(A, strideA, X, Y, M, R, nbatch, op, out_scale, s);
    else throw Error(-1, "cgemm: block size above 32 is not supported");
}
template void cgemm16_batched<kFmtBf16>(const uint32_t*, int64_t, const uint32_t*, float2*, int, int, int64_t, int,
                                        float, hipStream_t);
template void cgemm16_batched<kFmtF16>(const uint32_t*, int64_t, const uint32_t*, float2*, int, int, int64_t, int,
                                       float, hipStream_t);

template <typename T>
void cgemm_batched(const cplx<T>* A, int64_t strideA, const cplx<T>* X, cplx<T>* Y, int M, int R, int64_t nbatch,
                   int op, hipStream_t s) {
    if (nbatch <= 0 || R <= 0) return;
    if (M <= 16) launch_mp<T, 16>(A, strideA, X, Y, M, R, nbatch, op, s);
    else if (M <= 32) launch_mp<T, 32>(A, strideA, X, Y, M, R, nbatch, op, s);
    else if (M <= 64) launch_big<T, 64>(A, strideA, X, Y, M, R, nbatch, op, s);
    else if (M <= 96) launch_big<T, 96>(A, strideA, X, Y, M, R, nbatch, op, s);
    else if (M <= kMaxBlockM) launch_big<T, 128>(A, strideA, X, Y, M, R, nbatch, op, s);
    else throw Error(-1, "cgemm: block size above 128 is not supported");
}

template void cgemm_batched<double>(const double2*, int64_t, const double2*, double2*, int, int, int64_t, int, hipStream_t);
template void cgemm_batched<float>(const float2*, int64_t, const float2*, float2*, int, int, int64_t, int, hipStream_t);

}  // namespace mbt

// Two-level FFT over the lattice (paper eq. (F2): F_{N2} (x) (F_{N1} (x) I_{N0})).
//
// Vectors are stored RHS-innermost: x[e][p][r] with element e = iy*nx + ix, so
// for the lattice transform every (p, r) pair is an independent column
// c = p*R + r of a batch of B = M*R columns, and the lattice points of one
// column are B entries apart.  The in-block index is a batch dimension, which
// is the point of the 4-D arrangement of Sec. III-B; here it is the innermost,
// contiguous one so that a workgroup streams whole cache lines.
//
// The circulant embedding (eq. (multL)) uses a grid Px x Py = 2Lx x 2Ly with
// Lx >= nx, Ly >= ny (powers of two, at least 8), so that
// Px >= 2nx - 1 and the cyclic convolution reproduces the Toeplitz product on
// the cropped outputs.  A zero-padded transform of size 2L splits by output
// parity into four transforms of size L of pre-twiddled inputs:
//   X[2a+al][2b+be] = DFT_{Ly x Lx}( x[iy][ix] W_Py^{al iy} W_Px^{be ix} )[a][b],
// and the cropped inverse is the twiddled sum of the four parity sub-grids.
// Each workgroup holds an Ly x Lx x W tile (W adjacent columns) in LDS and runs
// the four sub-transforms there, so X is read once and X^ written once.
#include "common.h"

namespace mbt {

namespace {

// Workgroups are handed to the 8 XCDs round robin, and each XCD has its own L2.
// Logical block b of a launch of n is taken from a workgroup id such that
// consecutive logical blocks (adjacent columns, which share cache lines when a
// block's column run is shorter than a line) run on the same XCD.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
    const int64_t full = n - n % 8;
    if (b >= full) return b;
    return (b % 8) * (full / 8) + b / 8;
}

// ------------------------------------------------------------------ small DFTs in registers
template <typename C, bool INV> __device__ __forceinline__ void dft2(C* v) {
    C t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
}

template <typename C, bool INV> __device__ __forceinline__ void dft4(C* v) {
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    C id = cmul_i(d, INV);   // -i d forward, +i d inverse
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, id);
    v[3] = csub(b, id);
}

template <typename C, bool INV> __device__ __forceinline__ void dft8(C* v) {
    using T = decltype(v[0].x);
    const T h = (T)0.70710678118654752440;
    C a0[4], a1[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        a0[n] = cadd(v[n], v[n + 4]);
        a1[n] = csub(v[n], v[n + 4]);
    }
    // a1[n] *= W8^{n}  (conjugate for the inverse)
    {
        C t = a1[1];
        a1[1] = INV ? mk<T>(h * (t.x - t.y), h * (t.x + t.y)) : mk<T>(h * (t.x + t.y), h * (t.y - t.x));
        a1[2] = cmul_i(a1[2], INV);
        t = a1[3];
        a1[3] = INV ? mk<T>(-h * (t.x + t.y), h * (t.x - t.y)) : mk<T>(h * (t.y - t.x), -h * (t.x + t.y));
    }
    dft4<C, INV>(a0);
    dft4<C, INV>(a1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = a0[k];
        v[2 * k + 1] = a1[k];
    }
}

template <typename C, int R, bool INV> __device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<C, INV>(v);
    else if constexpr (R == 4) dft4<C, INV>(v);
    else if constexpr (R == 8) dft8<C, INV>(v);
}

template <int L> struct Split;
template <> struct Split<8> { static constexpr int R1 = 8, R2 = 1; };
template <> struct Split<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Split<32> { static constexpr int R1 = 8, R2 = 4; };
template <> struct Split<64> { static constexpr int R1 = 8, R2 = 8; };

// In-LDS FFTs of length L along one axis of a tile.  FFT f = (o, w) has its
// element i at tile[o*ostride + i*stride + w], o < nouter, w < W.
// Four-step: L = R1*R2, n = n1*R2 + n2, k = k1 + R1*k2;
//   pass 1: for each n2, DFT_R1 over n1, times W_L^{n2 k1}, stored in place;
//   pass 2: for each k1, DFT_R2 over n2, stored at k1 + R1*k2.
// tw is the twiddle table of the full grid P = 2L: W_L^m = tw[2m].
// OUTER_FAST orders work items so that neighbouring lanes step the smaller stride.
template <typename T, int L, bool INV, bool OUTER_FAST, int NT, int nouter, int ostride, int stride, int W>
__device__ __forceinline__ void lds_fft_axis(cplx<T>* tile, const cplx<T>* __restrict__ tw) {
    using C = cplx<T>;
    constexpr int R1 = Split<L>::R1, R2 = Split<L>::R2;
    const int tid = threadIdx.x;
    if constexpr (R2 == 1) {
        const int items = nouter * W;
        for (int it = tid; it < items; it += NT) {
            const int w = it % W, o = it / W;
            C* base = tile + o * ostride + w;
            C v[R1];
#pragma unroll
            for (int n = 0; n < R1; ++n) v[n] = base[n * stride];
            dft<C, R1, INV>(v);
#pragma unroll
            for (int n = 0; n < R1; ++n) base[n * stride] = v[n];
        }
    } else {
        const int items1 = nouter * W * R2;
        for (int it = tid; it < items1; it += NT) {
            int w = it % W, rest = it / W, o, n2;
            if (OUTER_FAST) { o = rest % nouter; n2 = rest / nouter; }
            else { n2 = rest % R2; o = rest / R2; }
            C* base = tile + o * ostride + w;
            C v[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) v[n1] = base[(n1 * R2 + n2) * stride];
            dft<C, R1, INV>(v);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                C t = tw[(2 * n2 * k1) % (2 * L)];
                if (INV) t.y = -t.y;
                base[(k1 * R2 + n2) * stride] = (k1 == 0 || n2 == 0) ? v[k1] : cmul(v[k1], t);
            }
        }
        __syncthreads();
        const int items2 = nouter * W * R1;
        constexpr int MAXIT = (nouter * W * R1 + NT - 1) / NT;
        C reg[MAXIT][R2];
#pragma unroll
        for (int i = 0; i < MAXIT; ++i) {
            const int it = tid + i * NT;
            if (it < items2) {
                int w = it % W, rest = it / W, o, k1;
                if (OUTER_FAST) { o = rest % nouter; k1 = rest / nouter; }
                else { k1 = rest % R1; o = rest / R1; }
                const C* base = tile + o * ostride + w;
#pragma unroll
                for (int n2 = 0; n2 < R2; ++n2) reg[i][n2] = base[(k1 * R2 + n2) * stride];
                dft<C, R2, INV>(reg[i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXIT; ++i) {
            const int it = tid + i * NT;
            if (it < items2) {
                int w = it % W, rest = it / W, o, k1;
                if (OUTER_FAST) { o = rest % nouter; k1 = rest / nouter; }
                else { k1 = rest % R1; o = rest / R1; }
                C* base = tile + o * ostride + w;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) base[(k1 + R1 * k2) * stride] = reg[i][k2];
            }
        }
    }
}

constexpr int kNT = 512;

// Each workgroup owns W adjacent columns: the whole (ny x nx) input of those
// columns is read once into registers (NOWN values per thread), and the four
// parity sub-transforms are run from there through one LDS tile.
template <typename T, int LX, int LY, int W>
__global__ __launch_bounds__(kNT) void fft_fwd_pad_kernel(const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Xh,
                                                          int nx, int ny, int64_t B, const cplx<T>* __restrict__ twx,
                                                          const cplx<T>* __restrict__ twy) {
    using C = cplx<T>;
    constexpr int PX = 2 * LX, NTILE = LX * LY * W;
    constexpr int NOWN = (NTILE + kNT - 1) / kNT;
    __shared__ C tile[NTILE];
    const int64_t c0 = xcd_block(blockIdx.x, gridDim.x) * W;
    C xin[NOWN];
#pragma unroll
    for (int i = 0; i < NOWN; ++i) {
        const int t = threadIdx.x + i * kNT;
        const int w = t % W, ix = (t / W) % LX, iy = t / (W * LX);
        const int64_t c = c0 + w;
        xin[i] = (t < NTILE && ix < nx && iy < ny && c < B) ? X[(int64_t)(iy * nx + ix) * B + c] : mk<T>(0, 0);
    }
    for (int par = 0; par < 4; ++par) {
        const int al = par >> 1, be = par & 1;
#pragma unroll
        for (int i = 0; i < NOWN; ++i) {
            const int t = threadIdx.x + i * kNT;
            if (t < NTILE) {
                const int ix = (t / W) % LX, iy = t / (W * LX);
                C v = xin[i];
                if (al && iy) v = cmul(v, twy[iy]);
                if (be && ix) v = cmul(v, twx[ix]);
                tile[t] = v;
            }
        }
        __syncthreads();
        lds_fft_axis<T, LX, false, false, kNT, LY, LX * W, W, W>(tile, twx);
        __syncthreads();
        lds_fft_axis<T, LY, false, true, kNT, LX, W, LX * W, W>(tile, twy);
        __syncthreads();
        for (int t = threadIdx.x; t < NTILE; t += kNT) {
            const int w = t % W, b = (t / W) % LX, a = t / (W * LX);
            const int64_t c = c0 + w;
            if (c < B) Xh[((int64_t)(2 * a + al) * PX + (2 * b + be)) * B + c] = tile[t];
        }
        __syncthreads();
    }
}

template <typename T, int LX, int LY, int W>
__global__ __launch_bounds__(kNT) void fft_inv_crop_kernel(const cplx<T>* __restrict__ Yh, cplx<T>* __restrict__ Y,
                                                           int nx, int ny, int64_t B, const cplx<T>* __restrict__ twx,
                                                           const cplx<T>* __restrict__ twy) {
    using C = cplx<T>;
    constexpr int PX = 2 * LX, NTILE = LX * LY * W;
    constexpr int NOWN = (NTILE + kNT - 1) / kNT;
    __shared__ C tile[NTILE];
    const int64_t c0 = xcd_block(blockIdx.x, gridDim.x) * W;
    C acc[NOWN];
#pragma unroll
    for (int i = 0; i < NOWN; ++i) acc[i] = mk<T>(0, 0);
    for (int par = 0; par < 4; ++par) {
        const int al = par >> 1, be = par & 1;
        for (int t = threadIdx.x; t < NTILE; t += kNT) {
            const int w = t % W, b = (t / W) % LX, a = t / (W * LX);
            const int64_t c = c0 + w;
            tile[t] = (c < B) ? Yh[((int64_t)(2 * a + al) * PX + (2 * b + be)) * B + c] : mk<T>(0, 0);
        }
        __syncthreads();
        lds_fft_axis<T, LX, true, false, kNT, LY, LX * W, W, W>(tile, twx);
        __syncthreads();
        lds_fft_axis<T, LY, true, true, kNT, LX, W, LX * W, W>(tile, twy);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NOWN; ++i) {
            const int t = threadIdx.x + i * kNT;
            if (t < NTILE) {
                const int ix = (t / W) % LX, iy = t / (W * LX);
                if (ix < nx && iy < ny) {
                    C v = tile[t];
                    if (al && iy) v = cmul(v, cconj(twy[iy]));
                    if (be && ix) v = cmul(v, cconj(twx[ix]));
                    acc[i] = cadd(acc[i], v);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NOWN; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < NTILE) {
            const int w = t % W, ix = (t / W) % LX, iy = t / (W * LX);
            const int64_t c = c0 + w;
            if (ix < nx && iy < ny && c < B) Y[(int64_t)(iy * nx + ix) * B + c] = acc[i];
        }
    }
}

// ------------------------------------------------------------------ register-resident FP32 transforms
// Radix-2 decimation-in-time FFT of length L held in one thread's registers
// (all indices compile-time).  tw is the table of the 2L-point grid, so
// W_len^k = tw[k * 2L / len]; the inverse uses conjugated twiddles (unscaled).
template <typename T, int L, bool INV>
__device__ __forceinline__ void fft_reg(cplx<T> (&v)[L], const cplx<T>* __restrict__ tw) {
    using C = cplx<T>;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        int j = 0;
#pragma unroll
        for (int b = 0; (1 << b) < L; ++b)
            if (i & (1 << b)) j |= (L >> 1) >> b;
        if (i < j) {
            const C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= L; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            C wk = mk<T>(1, 0);
            if (k) {
                wk = tw[k * (2 * L / len)];
                if (INV) wk.y = -wk.y;
            }
#pragma unroll
            for (int st = 0; st < L; st += len) {
                const C a = v[st + k];
                const C b = k ? cmul(v[st + k + half], wk) : v[st + k + half];
                v[st + k] = cadd(a, b);
                v[st + k + half] = csub(a, b);
            }
        }
    }
}

// Zero-padded forward transform with the sub-transforms in registers.  A
// workgroup owns W adjacent columns.  Phase 1: thread (row iy, column w)
// transforms its row for both x-parities (the row data is shared; the parity
// only twiddles the input).  The row spectra pass through one LDS tile.
// Phase 2: thread (bin b, column w) transforms its column for both
// y-parities and writes the four parity bins.  Two LDS round trips per block.
// T is float or double; FMT selects the FP32 spectrum's storage: FP32 complex,
// or 16-bit complex words.
template <typename T, int LX, int LY, int W, int FMT>
__global__ __launch_bounds__((LX > LY ? LX : LY) * W) void fft_fwd_reg_kernel(const cplx<T>* __restrict__ X,
                                                                              void* __restrict__ Xh_, int nx, int ny,
                                                                              int64_t B, const cplx<T>* __restrict__ twx,
                                                                              const cplx<T>* __restrict__ twy) {
    using C = cplx<T>;
    constexpr int PX = 2 * LX;
    // rows of the tile are padded by one W-slot so that the rows that one
    // half-wave touches at once fall on different LDS banks
    constexpr int RS = LX * W + W;
    __shared__ C tile[LY * RS];
    const int w = threadIdx.x % W, r = threadIdx.x / W;
    const int64_t c = (int64_t)blockIdx.x * W + w;
    const bool cv = c < B;
    // FP32 keeps the row in registers for both x-parities; FP64 (twice the
    // registers per value) reads it again for the second parity
    constexpr bool KEEP = sizeof(T) == 4;
    C row[KEEP ? LX : 1];
    if (KEEP && r < LY) {
#pragma unroll
        for (int ix = 0; ix < LX; ++ix)
            row[ix] = (cv && r < ny && ix < nx) ? X[(int64_t)(r * nx + ix) * B + c] : mk<T>(0, 0);
    }
#pragma unroll
    for (int be = 0; be < 2; ++be) {
        if (r < LY) {
            C f[LX];
#pragma unroll
            for (int ix = 0; ix < LX; ++ix) {
                C v;
                if constexpr (KEEP) v = row[ix];
                else v = (cv && r < ny && ix < nx) ? X[(int64_t)(r * nx + ix) * B + c] : mk<T>(0, 0);
                f[ix] = (be && ix) ? cmul(v, twx[ix]) : v;
            }
            fft_reg<T, LX, false>(f, twx);
#pragma unroll
            for (int b = 0; b < LX; ++b) tile[r * RS + b * W + w] = f[b];
        }
        __syncthreads();
        if (r < LX) {
#pragma unroll
            for (int al = 0; al < 2; ++al) {
                // the column is read from LDS once per y-parity: holding it in
                // registers beside the row would exceed the register budget
                C g[LY];
#pragma unroll
                for (int iy = 0; iy < LY; ++iy) {
                    const C t = tile[iy * RS + r * W + w];
                    g[iy] = (al && iy) ? cmul(t, twy[iy]) : t;
                }
                fft_reg<T, LY, false>(g, twy);
                if (cv) {
#pragma unroll
                    for (int a = 0; a < LY; ++a) {
                        const int64_t o = ((int64_t)(2 * a + al) * PX + (2 * r + be)) * B + c;
                        if constexpr (FMT == kFmtNone || sizeof(T) != 4)
                            static_cast<C*>(Xh_)[o] = g[a];
                        else
                            static_cast<uint32_t*>(Xh_)[o] = pack16<FMT>(g[a]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Cropped inverse with the sub-transforms in registers (mirror of the forward).
// Phase A: thread (bin b, column w) inverse-transforms the two y-parity
// columns of bin b and sums them with their twiddles.  Phase B: thread (row iy,
// column w) inverse-transforms the row and accumulates the x-parity with its
// twiddle; only rows iy < ny and columns ix < nx are written.  NTL: the
// spectrum is read with non-temporal loads (it is consumed once, so it need not
// displace the lines that the next kernel reads from L2).
template <typename T, int LX, int LY, int W, bool NTL = false>
__global__ __launch_bounds__((LX > LY ? LX : LY) * W) void fft_inv_reg_kernel(const cplx<T>* __restrict__ Yh,
                                                                              cplx<T>* __restrict__ Y, int nx, int ny,
                                                                              int64_t B, const cplx<T>* __restrict__ twx,
                                                                              const cplx<T>* __restrict__ twy) {
    using C = cplx<T>;
    constexpr int PX = 2 * LX;
    // rows of the tile are padded by one W-slot so that the rows that one
    // half-wave touches at once fall on different LDS banks
    constexpr int RS = LX * W + W;
    __shared__ C tile[LY * RS];
    const int w = threadIdx.x % W, r = threadIdx.x / W;
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * W + w;
    const bool cv = c < B;
    C out[LX];
#pragma unroll
    for (int ix = 0; ix < LX; ++ix) out[ix] = mk<T>(0, 0);
#pragma unroll
    for (int be = 0; be < 2; ++be) {
        if (r < LX) {
            C acc[LY];
#pragma unroll
            for (int iy = 0; iy < LY; ++iy) acc[iy] = mk<T>(0, 0);
#pragma unroll
            for (int al = 0; al < 2; ++al) {
                C g[LY];
#pragma unroll
                for (int a = 0; a < LY; ++a) {
                    const C* q = Yh + ((int64_t)(2 * a + al) * PX + (2 * r + be)) * B + c;
                    if (!cv)
                        g[a] = mk<T>(0, 0);
                    else if constexpr (NTL)
                        g[a] = mk<T>(__builtin_nontemporal_load(reinterpret_cast<const T*>(q)),
                                     __builtin_nontemporal_load(reinterpret_cast<const T*>(q) + 1));
                    else
                        g[a] = *q;
                }
                fft_reg<T, LY, true>(g, twy);
#pragma unroll
                for (int iy = 0; iy < LY; ++iy) acc[iy] = cadd(acc[iy], (al && iy) ? cmul(g[iy], cconj(twy[iy])) : g[iy]);
            }
#pragma unroll
            for (int iy = 0; iy < LY; ++iy) tile[iy * RS + r * W + w] = acc[iy];
        }
        __syncthreads();
        if (r < LY) {
            C h[LX];
#pragma unroll
            for (int b = 0; b < LX; ++b) h[b] = tile[r * RS + b * W + w];
            fft_reg<T, LX, true>(h, twx);
#pragma unroll
            for (int ix = 0; ix < LX; ++ix) out[ix] = cadd(out[ix], (be && ix) ? cmul(h[ix], cconj(twx[ix])) : h[ix]);
        }
        __syncthreads();
    }
    if (cv && r < ny) {
#pragma unroll
        for (int ix = 0; ix < LX; ++ix)
            if (ix < nx) Y[(int64_t)(r * nx + ix) * B + c] = out[ix];
    }
}

// ------------------------------------------------------------------ two-pass FP32 transforms (128-point axes)
// On a 128-point axis one column's L x L sub-transforms take 32 KB of LDS, so a
// fused kernel holds only a few columns per CU and reads 32-byte runs.  These
// grids run as two passes of 1-D transforms instead, each line of a column
// held and transformed in one thread's registers.  A wave covers 32 adjacent
// columns twice: lanes 0-31 take parity 0 of a line and lanes 32-63 parity 1
// (256 contiguous bytes per half-wave access; both halves of the forward
// passes read the same addresses).  The inverse passes add the two parity
// contributions across the halves with a lane exchange, each half writing
// half of the line.  The intermediate Z (ny x 2Lx lines per column) sits in
// the spare spectral buffer.
constexpr int kLineNT = 256;
constexpr int kLineCols = kLineNT / 2;   // columns per workgroup

struct LineIdx {
    int line, half;
    int64_t c;
    bool cv;
};
__device__ __forceinline__ LineIdx line_idx(int64_t ctiles, int64_t B) {
    LineIdx L;
    const int lane = threadIdx.x & 63;
    L.line = (int)(blockIdx.x / ctiles);
    L.half = lane >> 5;
    L.c = (int64_t)(blockIdx.x % ctiles) * kLineCols + (threadIdx.x >> 6) * 32 + (lane & 31);
    L.cv = L.c < B;
    return L;
}

// v times the parity twiddle tw[i] (or its conjugate) on odd halves, v on even
// halves (the product takes the uniform twiddle; only the result is selected)
template <bool CONJ>
__device__ __forceinline__ float2 par_tw(float2 v, const float2* __restrict__ tw, int i, int half) {
    float2 t = tw[i];
    if (CONJ) t.y = -t.y;
    const float2 p = cmul(v, t);
    return half ? p : v;
}

// Forward, pass 1: rows.  Z[iy][2b+be][c] = sum_ix x[iy][ix][c] W_{2Lx}^{ix(2b+be)}.
template <int LX>
__global__ __launch_bounds__(kLineNT) void fft_rows_fwd_kernel(const float2* __restrict__ X, float2* __restrict__ Z,
                                                               int nx, int64_t B, int64_t ctiles,
                                                               const float2* __restrict__ twx) {
    constexpr int PX = 2 * LX;
    const LineIdx t = line_idx(ctiles, B);
    const int iy = t.line;
    float2 f[LX];
#pragma unroll
    for (int ix = 0; ix < LX; ++ix) {
        const float2 v = (t.cv && ix < nx) ? X[(int64_t)(iy * nx + ix) * B + t.c] : mk<float>(0, 0);
        f[ix] = ix ? par_tw<false>(v, twx, ix, t.half) : v;
    }
    fft_reg<float, LX, false>(f, twx);
    if (t.cv) {
#pragma unroll
        for (int b = 0; b < LX; ++b) Z[((int64_t)iy * PX + 2 * b + t.half) * B + t.c] = f[b];
    }
}

// Forward, pass 2: columns.  Xh[2a+al][kx][c] = sum_iy Z[iy][kx][c] W_{2Ly}^{iy(2a+al)},
// stored as FP32 complex or packed 16-bit complex (FMT).
template <int LX, int LY, int FMT>
__global__ __launch_bounds__(kLineNT) void fft_cols_fwd_kernel(const float2* __restrict__ Z, void* __restrict__ Xh_,
                                                               int ny, int64_t B, int64_t ctiles,
                                                               const float2* __restrict__ twy) {
    constexpr int PX = 2 * LX;
    const LineIdx t = line_idx(ctiles, B);
    const int kx = t.line;
    float2 g[LY];
#pragma unroll
    for (int iy = 0; iy < LY; ++iy) {
        const float2 v = (t.cv && iy < ny) ? Z[((int64_t)iy * PX + kx) * B + t.c] : mk<float>(0, 0);
        g[iy] = iy ? par_tw<false>(v, twy, iy, t.half) : v;
    }
    fft_reg<float, LY, false>(g, twy);
    if (t.cv) {
#pragma unroll
        for (int a = 0; a < LY; ++a) {
            const int64_t o = ((int64_t)(2 * a + t.half) * PX + kx) * B + t.c;
            if constexpr (FMT == kFmtNone)
                static_cast<float2*>(Xh_)[o] = g[a];
            else
                static_cast<uint32_t*>(Xh_)[o] = pack16<FMT>(g[a]);
        }
    }
}

// the value of element j (j < L/2) of the two halves' sum that this half
// writes: half 0 element j, half 1 element j + L/2.  One v_permlane32_swap per
// component trades lanes 32-63 of v[j] with lanes 0-31 of v[j + L/2], after
// which each lane holds both halves' copies of its element (all 64 lanes must
// take part).
template <int L>
__device__ __forceinline__ float2 half_sum(const float2 (&v)[L], int j) {
    const float2 a = v[j], b = v[j + L / 2];
    const auto sx = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
    const auto sy = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
    return make_float2(__uint_as_float(sx[0]) + __uint_as_float(sx[1]), __uint_as_float(sy[0]) + __uint_as_float(sy[1]));
}

// Inverse, pass 1: columns.  Z[iy][kx][c] = sum_al tw_al(iy)* IDFT_Ly(Yh[2a+al][kx][c])[iy], iy < ny.
template <int LX, int LY>
__global__ __launch_bounds__(kLineNT) void fft_cols_inv_kernel(const float2* __restrict__ Yh, float2* __restrict__ Z,
                                                               int ny, int64_t B, int64_t ctiles,
                                                               const float2* __restrict__ twy) {
    constexpr int PX = 2 * LX;
    const LineIdx t = line_idx(ctiles, B);
    const int kx = t.line;
    float2 g[LY];
#pragma unroll
    for (int a = 0; a < LY; ++a) g[a] = t.cv ? Yh[((int64_t)(2 * a + t.half) * PX + kx) * B + t.c] : mk<float>(0, 0);
    fft_reg<float, LY, true>(g, twy);
#pragma unroll
    for (int iy = 1; iy < LY; ++iy) g[iy] = par_tw<true>(g[iy], twy, iy, t.half);
#pragma unroll
    for (int j = 0; j < LY / 2; ++j) {
        const float2 v = half_sum<LY>(g, j);
        const int iy = j + t.half * (LY / 2);
        if (t.cv && iy < ny) Z[((int64_t)iy * PX + kx) * B + t.c] = v;
    }
}

// Inverse, pass 2: rows.  Y[iy][ix][c] = sum_be tw_be(ix)* IDFT_Lx(Z[iy][2b+be][c])[ix], ix < nx.
template <int LX>
__global__ __launch_bounds__(kLineNT) void fft_rows_inv_kernel(const float2* __restrict__ Z, float2* __restrict__ Y,
                                                               int nx, int64_t B, int64_t ctiles,
                                                               const float2* __restrict__ twx) {
    constexpr int PX = 2 * LX;
    const LineIdx t = line_idx(ctiles, B);
    const int iy = t.line;
    float2 h[LX];
#pragma unroll
    for (int b = 0; b < LX; ++b) h[b] = t.cv ? Z[((int64_t)iy * PX + 2 * b + t.half) * B + t.c] : mk<float>(0, 0);
    fft_reg<float, LX, true>(h, twx);
#pragma unroll
    for (int ix = 1; ix < LX; ++ix) h[ix] = par_tw<true>(h[ix], twx, ix, t.half);
#pragma unroll
    for (int j = 0; j < LX / 2; ++j) {
        const float2 v = half_sum<LX>(h, j);
        const int ix = j + t.half * (LX / 2);
        if (t.cv && ix < nx) Y[(int64_t)(iy * nx + ix) * B + t.c] = v;
    }
}

// Z needs ny * 2Lx * B complex values of scratch.
template <bool FWD, int LX, int LY, int FMT>
void launch_two_pass(const Geom& g, const float2* in, void* out, int64_t B, const float2* twx, const float2* twy,
                     float2* Z, hipStream_t s) {
    const int64_t ctiles = (B + kLineCols - 1) / kLineCols;
    const int64_t rows = (int64_t)g.ny * ctiles, cols = (int64_t)(2 * LX) * ctiles;
    MBT_REQUIRE(g.nx <= LX && g.ny <= LY, "fft: lattice larger than its grid");
    MBT_REQUIRE(cols * kLineNT < (1LL << 32), "fft: batch too large");
    if (FWD) {
        hipLaunchKernelGGL((fft_rows_fwd_kernel<LX>), dim3((unsigned)rows), dim3(kLineNT), 0, s, in, Z, g.nx, B, ctiles,
                           twx);
        MBT_LAUNCH_CHECK();
        hipLaunchKernelGGL((fft_cols_fwd_kernel<LX, LY, FMT>), dim3((unsigned)cols), dim3(kLineNT), 0, s, Z, out, g.ny,
                           B, ctiles, twy);
        MBT_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL((fft_cols_inv_kernel<LX, LY>), dim3((unsigned)cols), dim3(kLineNT), 0, s, in, Z, g.ny, B,
                           ctiles, twy);
        MBT_LAUNCH_CHECK();
        hipLaunchKernelGGL((fft_rows_inv_kernel<LX>), dim3((unsigned)rows), dim3(kLineNT), 0, s, Z,
                           static_cast<float2*>(out), g.nx, B, ctiles, twx);
        MBT_LAUNCH_CHECK();
    }
}

// ------------------------------------------------------------------ twiddles and block spectra
__global__ void twiddle_kernel(int P, double2* tw) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P) {
        double s, c;
        sincospi(2.0 * (double)j / (double)P, &s, &c);
        tw[j] = make_double2(c, -s);
    }
}

// One axis of the block spectrum.  For every line (outer index o, block entry e),
//   out[o][k][e] = sc * sum_{i < 2n-1} in[o][i][e] W_P^{k (i - (n-1))},
// i.e. the P-point DFT of the offsets -(n-1)..n-1 placed circularly (eq. (multL)'s
// circulant embedding), by an in-place radix-2 decimation-in-time FFT in LDS: the
// input is loaded at bit-reversed positions, log2 P butterfly stages follow, the
// output is in natural order.  A workgroup holds EC consecutive block entries of
// one line, so loads and stores are EC consecutive complex values per row.
template <int P, int EC>
__global__ __launch_bounds__(256) void embed_axis_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                         int n, int64_t in_outer, int64_t in_stride,
                                                         int64_t out_outer, int64_t out_stride, int64_t MM,
                                                         double sc, const double2* __restrict__ tw) {
    constexpr int kLog = P == 8 ? 3 : P == 16 ? 4 : P == 32 ? 5 : P == 64 ? 6 : 7;
    static_assert((1 << kLog) == P, "P must be a power of two in 8..128");
    constexpr int kSub = 256 / EC;
    __shared__ double2 buf[P * EC];
    const int64_t o = blockIdx.y;
    const int col = threadIdx.x % EC, sub = threadIdx.x / EC;
    const int64_t e = (int64_t)blockIdx.x * EC + col;
    const bool live = e < MM;
    for (int i = sub; i < P; i += kSub) buf[i * EC + col] = make_double2(0.0, 0.0);
    __syncthreads();
    const int nlen = 2 * n - 1;
    for (int i = sub; i < nlen; i += kSub) {
        int pos = i - (n - 1);
        if (pos < 0) pos += P;
        const int br = (int)(__brev((unsigned)pos) >> (32 - kLog));
        buf[br * EC + col] = live ? in[o * in_outer + (int64_t)i * in_stride + e] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int lh = 0; lh < kLog; ++lh) {
        const int h = 1 << lh;
        for (int bfly = sub; bfly < P / 2; bfly += kSub) {
            const int pos = bfly & (h - 1);
            const int i0 = ((bfly >> lh) << (lh + 1)) + pos, i1 = i0 + h;
            const double2 w = tw[pos << (kLog - 1 - lh)];   // W_{2h}^{pos} = W_P^{pos P / 2h}
            const double2 x0 = buf[i0 * EC + col];
            const double2 x1 = cmul(buf[i1 * EC + col], w);
            buf[i0 * EC + col] = cadd(x0, x1);
            buf[i1 * EC + col] = csub(x0, x1);
        }
        __syncthreads();
    }
    if (live)
        for (int kk = sub; kk < P; kk += kSub) {
            const double2 v = buf[kk * EC + col];
            out[o * out_outer + (int64_t)kk * out_stride + e] = make_double2(sc * v.x, sc * v.y);
        }
}

void launch_embed_axis(int P, const double2* in, double2* out, int n, int64_t nlines, int64_t in_outer,
                       int64_t in_stride, int64_t out_outer, int64_t out_stride, int64_t MM, double sc,
                       const double2* tw, hipStream_t s) {
    constexpr int EC = 32;
    const dim3 grid((unsigned)((MM + EC - 1) / EC), (unsigned)nlines);
    MBT_REQUIRE(nlines < 65536, "embed: too many lines");
    switch (P) {
        case 16:
            hipLaunchKernelGGL((embed_axis_kernel<16, EC>), grid, dim3(256), 0, s, in, out, n, in_outer, in_stride,
                               out_outer, out_stride, MM, sc, tw);
            break;
        case 32:
            hipLaunchKernelGGL((embed_axis_kernel<32, EC>), grid, dim3(256), 0, s, in, out, n, in_outer, in_stride,
                               out_outer, out_stride, MM, sc, tw);
            break;
        case 64:
            hipLaunchKernelGGL((embed_axis_kernel<64, EC>), grid, dim3(256), 0, s, in, out, n, in_outer, in_stride,
                               out_outer, out_stride, MM, sc, tw);
            break;
        case 128:
            hipLaunchKernelGGL((embed_axis_kernel<128, EC>), grid, dim3(256), 0, s, in, out, n, in_outer, in_stride,
                               out_outer, out_stride, MM, sc, tw);
            break;
        default: throw Error(-1, "embed: unsupported grid size");
    }
    MBT_LAUNCH_CHECK();
}

// Columns per workgroup: fill a 128 KB LDS tile (one workgroup per CU), at
// most 16 columns.  At the 64x64 grid this gives 128 contiguous bytes per
// lattice point in FP64 (8 columns) and in FP32 (16 columns).
// columns per workgroup of the FP64 register transforms
constexpr int kRegW64 = 4;

template <typename T> constexpr int tile_w(int lx, int ly) {
    int w = (int)(131072 / (lx * ly * (int)sizeof(cplx<T>)));
    return w > 16 ? 16 : (w < 1 ? 1 : w);
}

template <typename T, bool FWD, int LX, int LY>
void launch_fft_t(const Geom& g, const cplx<T>* in, cplx<T>* out, int64_t B, const cplx<T>* twx, const cplx<T>* twy,
                  cplx<T>* scratch, hipStream_t s) {
    constexpr int W = tile_w<T>(LX, LY);
    const int64_t blocks = (B + W - 1) / W;
    MBT_REQUIRE(blocks < (1LL << 31), "fft: batch too large");
    if constexpr (sizeof(T) == 4 && (LX > 32 || LY > 32)) {
        if (scratch) {
            launch_two_pass<FWD, LX, LY, kFmtNone>(g, in, out, B, twx, twy, scratch, s);
            return;
        }
    }
    if constexpr (sizeof(T) == 8 && LX <= 32 && LY <= 32) {
        // FP64 inverse: the register transform with fewer columns per workgroup
        // (a row of 32 values fills 128 registers), two workgroups per CU.  The
        // FP64 forward stays on the LDS kernel, which measured faster.
        if (!FWD) {
            constexpr int WD = W > kRegW64 ? kRegW64 : W;
            constexpr int NT = (LX > LY ? LX : LY) * WD;
            const int64_t nb = (B + WD - 1) / WD;
            hipLaunchKernelGGL((fft_inv_reg_kernel<T, LX, LY, WD>), dim3((unsigned)nb), dim3(NT), 0, s, in, out, g.nx,
                               g.ny, B, twx, twy);
            MBT_LAUNCH_CHECK();
            return;
        }
    }
    if constexpr (sizeof(T) == 4 && LX <= 32 && LY <= 32) {
        constexpr int NT = (LX > LY ? LX : LY) * W;
        if (FWD)
            hipLaunchKernelGGL((fft_fwd_reg_kernel<T, LX, LY, W, kFmtNone>), dim3((unsigned)blocks), dim3(NT), 0, s, in,
                               (void*)out, g.nx, g.ny, B, twx, twy);
        else {
            // the inverse reads four times what it writes and reads each spectrum
            // value once: full-width tiles with non-temporal loads measured ahead of
            // half-width tiles (two workgroups per CU) with either kind of load
            hipLaunchKernelGGL((fft_inv_reg_kernel<T, LX, LY, W, true>), dim3((unsigned)blocks),
                               dim3((LX > LY ? LX : LY) * W), 0, s, in, out, g.nx, g.ny, B, twx, twy);
        }
        MBT_LAUNCH_CHECK();
        return;
    }
    if (FWD)
        hipLaunchKernelGGL((fft_fwd_pad_kernel<T, LX, LY, W>), dim3((unsigned)blocks), dim3(kNT), 0, s, in, out,
                           g.nx, g.ny, B, twx, twy);
    else
        hipLaunchKernelGGL((fft_inv_crop_kernel<T, LX, LY, W>), dim3((unsigned)blocks), dim3(kNT), 0, s, in, out,
                           g.nx, g.ny, B, twx, twy);
    MBT_LAUNCH_CHECK();
}

template <typename T, bool FWD, int LX>
void dispatch_ly(const Geom& g, const cplx<T>* in, cplx<T>* out, int64_t B, const cplx<T>* twx, const cplx<T>* twy,
                 cplx<T>* scratch, hipStream_t s) {
    switch (g.Ly) {
        case 8: launch_fft_t<T, FWD, LX, 8>(g, in, out, B, twx, twy, scratch, s); break;
        case 16: launch_fft_t<T, FWD, LX, 16>(g, in, out, B, twx, twy, scratch, s); break;
        case 32: launch_fft_t<T, FWD, LX, 32>(g, in, out, B, twx, twy, scratch, s); break;
        case 64: launch_fft_t<T, FWD, LX, 64>(g, in, out, B, twx, twy, scratch, s); break;
        default: throw Error(-1, "fft: unsupported grid (ny > 64)");
    }
}

template <typename T, bool FWD>
void dispatch(const Geom& g, const cplx<T>* in, cplx<T>* out, int64_t B, const cplx<T>* twx, const cplx<T>* twy,
              cplx<T>* scratch, hipStream_t s) {
    switch (g.Lx) {
        case 8: dispatch_ly<T, FWD, 8>(g, in, out, B, twx, twy, scratch, s); break;
        case 16: dispatch_ly<T, FWD, 16>(g, in, out, B, twx, twy, scratch, s); break;
        case 32: dispatch_ly<T, FWD, 32>(g, in, out, B, twx, twy, scratch, s); break;
        case 64: dispatch_ly<T, FWD, 64>(g, in, out, B, twx, twy, scratch, s); break;
        default: throw Error(-1, "fft: unsupported grid (nx > 64)");
    }
}

template <int FMT, int LX, int LY>
void launch_fwd16(const Geom& g, const float2* X, uint32_t* Xh, int64_t B, const float2* twx, const float2* twy,
                  float2* scratch, hipStream_t s) {
    if constexpr (LX <= 32 && LY <= 32) {
        (void)scratch;
        constexpr int W = tile_w<float>(LX, LY);
        constexpr int NT = (LX > LY ? LX : LY) * W;
        const int64_t blocks = (B + W - 1) / W;
        MBT_REQUIRE(blocks < (1LL << 31), "fft: batch too large");
        hipLaunchKernelGGL((fft_fwd_reg_kernel<float, LX, LY, W, FMT>), dim3((unsigned)blocks), dim3(NT), 0, s, X, (void*)Xh,
                           g.nx, g.ny, B, twx, twy);
        MBT_LAUNCH_CHECK();
    } else {
        // two passes, the second storing the packed spectrum; scratch holds the row spectra
        launch_two_pass<true, LX, LY, FMT>(g, X, Xh, B, twx, twy, scratch, s);
    }
}

template <int FMT, int LX>
void dispatch16_ly(const Geom& g, const float2* X, uint32_t* Xh, int64_t B, const float2* twx, const float2* twy,
                   float2* scratch, hipStream_t s) {
    switch (g.Ly) {
        case 8: launch_fwd16<FMT, LX, 8>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 16: launch_fwd16<FMT, LX, 16>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 32: launch_fwd16<FMT, LX, 32>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 64: launch_fwd16<FMT, LX, 64>(g, X, Xh, B, twx, twy, scratch, s); break;
        default: throw Error(-1, "fft: unsupported grid (ny > 64)");
    }
}

}  // namespace

template <int FMT>
void fft_fwd_pad16(const Geom& g, const float2* X, uint32_t* Xh, int64_t B, const float2* twx, const float2* twy,
                   float2* scratch, hipStream_t s) {
    switch (g.Lx) {
        case 8: dispatch16_ly<FMT, 8>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 16: dispatch16_ly<FMT, 16>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 32: dispatch16_ly<FMT, 32>(g, X, Xh, B, twx, twy, scratch, s); break;
        case 64: dispatch16_ly<FMT, 64>(g, X, Xh, B, twx, twy, scratch, s); break;
        default: throw Error(-1, "fft: unsupported grid (nx > 64)");
    }
}
template void fft_fwd_pad16<kFmtBf16>(const Geom&, const float2*, uint32_t*, int64_t, const float2*, const float2*,
                                      float2*, hipStream_t);
template void fft_fwd_pad16<kFmtF16>(const Geom&, const float2*, uint32_t*, int64_t, const float2*, const float2*,
                                     float2*, hipStream_t);

void make_twiddles(int P, double2* tw, hipStream_t s) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((P + 255) / 256), dim3(256), 0, s, P, tw);
    MBT_LAUNCH_CHECK();
}

void embed_blocks_fft(const Geom& g, const double2* T, double2* Chat, double scale, double2* scratch, hipStream_t s) {
    // scratch: noy * Px * M*M complex; twiddle tables are placed after it
    const int64_t MM = (int64_t)g.M * g.M;
    double2* tmp = scratch;
    double2* twx = scratch + (int64_t)g.noy * g.Px * MM;
    double2* twy = twx + g.Px;
    make_twiddles(g.Px, twx, s);
    make_twiddles(g.Py, twy, s);
    // x: lines (oy, e) over the 2nx-1 offsets ox -> tmp[oy][kx][e]
    launch_embed_axis(g.Px, T, tmp, g.nx, g.noy, (int64_t)g.nox * MM, MM, (int64_t)g.Px * MM, MM, MM, 1.0, twx, s);
    // y: lines (kx, e) over the 2ny-1 offsets oy -> Chat[ky][kx][e]
    launch_embed_axis(g.Py, tmp, Chat, g.ny, g.Px, MM, (int64_t)g.Px * MM, MM, (int64_t)g.Px * MM, MM, scale, twy, s);
}

template <typename T>
void fft_fwd_pad(const Geom& g, const cplx<T>* X, cplx<T>* Xh, int64_t B, const cplx<T>* twx, const cplx<T>* twy,
                 cplx<T>* scratch, hipStream_t s) {
    dispatch<T, true>(g, X, Xh, B, twx, twy, scratch, s);
}

template <typename T>
void fft_inv_crop(const Geom& g, const cplx<T>* Yh, cplx<T>* Y, int64_t B, const cplx<T>* twx, const cplx<T>* twy,
                  cplx<T>* scratch, hipStream_t s) {
    dispatch<T, false>(g, Yh, Y, B, twx, twy, scratch, s);
}

template void fft_fwd_pad<double>(const Geom&, const double2*, double2*, int64_t, const double2*, const double2*,
                                  double2*, hipStream_t);
template void fft_fwd_pad<float>(const Geom&, const float2*, float2*, int64_t, const float2*, const float2*, float2*,
                                 hipStream_t);
template void fft_inv_crop<double>(const Geom&, const double2*, double2*, int64_t, const double2*, const double2*,
                                   double2*, hipStream_t);
template void fft_inv_crop<float>(const Geom&, const float2*, float2*, int64_t, const float2*, const float2*, float2*,
                                  hipStream_t);

}  // namespace mbt

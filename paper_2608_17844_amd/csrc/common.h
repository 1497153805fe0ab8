// Shared declarations of the MI355X MBT solver library (internal, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace mbt {

// ------------------------------------------------------------------ complex helpers
template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
    cplx<T> r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// conj(a) * b
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.x * b.y - a.y * b.x;
    return r;
}
template <typename C> __host__ __device__ __forceinline__ C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
// multiply by +i (inv == true) or -i
template <typename C> __host__ __device__ __forceinline__ C cmul_i(C a, bool plus) {
    C r;
    if (plus) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
    return r;
}

__host__ __device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
__host__ __device__ __forceinline__ double2 to_d2(double2 a) { return a; }
template <typename C> __host__ __device__ __forceinline__ C from_d2(double2 a);
template <> __host__ __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <> __host__ __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
    return make_float2((float)a.x, (float)a.y);
}

// ------------------------------------------------------------------ 16-bit complex storage
// A complex value kept as two 16-bit floats in one 32-bit word, real part in
// the low half.  kFmtBf16: bfloat16 (8-bit exponent, 7-bit mantissa);
// kFmtF16: IEEE binary16.  Conversions round to nearest even.
enum : int { kFmtNone = -1, kFmtBf16 = 0, kFmtF16 = 1 };

template <int FMT> __device__ __forceinline__ uint32_t f32_to_16(float f) {
    if constexpr (FMT == kFmtBf16) {
        const uint32_t u = __float_as_uint(f);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;   // NaN stays NaN
        return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    } else {
        const _Float16 h = (_Float16)f;
        return (uint32_t)__builtin_bit_cast(uint16_t, h);
    }
}
template <int FMT> __device__ __forceinline__ float f16_to_32(uint32_t h) {
    if constexpr (FMT == kFmtBf16) {
        return __uint_as_float(h << 16);
    } else {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    }
}
template <int FMT> __device__ __forceinline__ uint32_t pack16(float2 v) {
    return f32_to_16<FMT>(v.x) | (f32_to_16<FMT>(v.y) << 16);
}
template <int FMT> __device__ __forceinline__ float2 unpack16(uint32_t w) {
    return make_float2(f16_to_32<FMT>(w & 0xffffu), f16_to_32<FMT>(w >> 16));
}

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MBT_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::mbt::Error(-4, std::string("HIP error '") + hipGetErrorString(e_) + "' at " + \
                                       __FILE__ + ":" + std::to_string(__LINE__) + " (" #call ")"); \
    } while (0)

#define MBT_LAUNCH_CHECK() MBT_HIP(hipGetLastError())

#define MBT_REQUIRE(cond, msg)                                   \
    do {                                                         \
        if (!(cond)) throw ::mbt::Error(-1, std::string(msg));   \
    } while (0)

// ------------------------------------------------------------------ kernel timing
// Brackets one launch with HIP events on its stream when its class is the one
// selected by mbt_prof_start; records the launch's algorithmic bytes/flops.
enum KernelClass {
    kKArnoldiDots = 1,
    kKArnoldiUpdateDots = 2,
    kKArnoldiUpdateNorm = 3,
    kKFftFwd = 4,
    kKFftInv = 5,
    kKBinProduct = 6,
    kKPrecondApply = 7
};
class ProfScope {
  public:
    ProfScope(int kernel, double bytes, double flops, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    bool on_ = false;
    hipEvent_t a_{}, b_{};
    hipStream_t s_;
    double bytes_, flops_;
};

// largest basis count per element of the block products (block-defined arrays)
constexpr int kMaxBlockM = 128;

// ------------------------------------------------------------------ geometry
// The port of an element: the bases its gap drives and their weights.  A gap
// voltage V puts V * w[i] on basis idx[i]; the gap current is sum_i w[i] I[idx[i]].
constexpr int kMaxPortBases = 8;
struct PortDef {
    int n = 1;
    int idx[kMaxPortBases] = {0};
    double w[kMaxPortBases] = {1.0};
};

struct Geom {
    int nx = 0, ny = 0, M = 0;     // lattice size, bases per element
    double dx = 0, dy = 0;         // lattice spacing (wavelengths at f0)
    double L = 0, a = 0;           // dipole length and wire radius
    int P = 0;                     // elements = ports
    int64_t N = 0;                 // unknowns
    int Lx = 0, Ly = 0;            // half FFT grid: powers of two >= nx, ny
    int Px = 0, Py = 0;            // FFT grid 2*Lx x 2*Ly >= (2nx-1) x (2ny-1)
    int nox = 0, noy = 0;          // offsets per axis 2nx-1, 2ny-1
    int pc = 0;                    // port basis (M-1)/2
    int Nc = 0;                    // margin unknowns after the P*M element unknowns (N = P*M + Nc)
    PortDef port;                  // dipoles and block arrays: basis pc with weight 1
    int64_t NA() const { return (int64_t)P * M; }
    int64_t bins() const { return (int64_t)Px * Py; }
    int64_t noff() const { return (int64_t)nox * noy; }
};

// ------------------------------------------------------------------ kernels (host launchers)
// fill.hip: unique interaction blocks T[(dy+ny-1)*nox + (dx+nx-1)][p][q] (row-major M x M)
void fill_blocks(const Geom& g, double k, double2* T, hipStream_t s);

// fft.hip
// spectrum of the circulant embedding: Chat[ky*Px+kx][p][q] = scale * DFT2(C_1)[p][q]
void embed_blocks_fft(const Geom& g, const double2* T, double2* Chat, double scale, double2* scratch,
                      hipStream_t s);
// twiddle table tw[j] = exp(-2 pi i j / P), j < P
void make_twiddles(int P, double2* tw, hipStream_t s);
// Zero-padded forward transform of B columns and the cropped inverse.  scratch
// (at least ny * Px * B complex values, not overlapping the operands) lets FP32
// transforms on 128-point axes run as two passes of 1-D transforms; with NULL
// they run as one LDS-tiled kernel.
template <typename T>
void fft_fwd_pad(const Geom& g, const cplx<T>* X, cplx<T>* Xh, int64_t B, const cplx<T>* twx,
                 const cplx<T>* twy, cplx<T>* scratch, hipStream_t s);
template <typename T>
void fft_inv_crop(const Geom& g, const cplx<T>* Yh, cplx<T>* Y, int64_t B, const cplx<T>* twx,
                  const cplx<T>* twy, cplx<T>* scratch, hipStream_t s);

// Forward lattice FFT with the spectrum stored in 16-bit complex (FMT); the
// transform itself runs in FP32.  scratch (ny * Px * B float2) is used on grids
// whose sub-transforms do not fit the register kernels.
template <int FMT>
void fft_fwd_pad16(const Geom& g, const float2* X, uint32_t* Xh, int64_t B, const float2* twx, const float2* twy,
                   float2* scratch, hipStream_t s);

// cgemm.hip: Y_b = op(A_b) X_b for b < nbatch; A_b = A + b*strideA (M x M row-major complex),
// X_b / Y_b = X/Y + b*M*R (M x R row-major).  op: 0 = A, 1 = A^H.
template <typename T>
void cgemm_batched(const cplx<T>* A, int64_t strideA, const cplx<T>* X, cplx<T>* Y, int M, int R,
                   int64_t nbatch, int op, hipStream_t s);

// Same with A and X in 16-bit complex (FMT), FP32 accumulation and FP32 Y.
// A holds a scaled copy (scale * A_b): Y is multiplied by out_scale = 1/scale.
template <int FMT>
void cgemm16_batched(const uint32_t* A, int64_t strideA, const uint32_t* X, float2* Y, int M, int R, int64_t nbatch,
                     int op, float out_scale, hipStream_t s);

// precond.hip
void gram_blocks(const Geom& g, const double2* T, double2* G, hipStream_t s);            // G[d] = T[d]^H T[d]
void window_sum(const Geom& g, const double2* G, double2* Pblk, hipStream_t s);          // P_e = sum_j G[j-e]
// batched inverses of M x M blocks: hpd = true -> Cholesky based; false -> LU with partial pivoting.
// info[b] != 0 flags a non-positive pivot / singular block.
void batched_inverse(const double2* A, double2* Ainv, int M, int64_t nbatch, bool hpd, int* info,
                     hipStream_t s);
// Hermitian positive definite blocks up to kMaxBlockM bases; A is overwritten (used as the factor's storage
// when M > 32).
void batched_inverse_hpd_inplace(double2* A, double2* Ainv, int M, int64_t nbatch, int* info, hipStream_t s);

// margin.hip: Y[m][r] (+)= sum_k op(A)(m, k) X[k * sxk + r * sxr], op(A)(m, k) = A[m*sm + k*sk] (conjugated
// if conjA), for m < Mrows, r < R; Y rows of stride ldy.  A long K is split over workgroups whose partial
// tiles go to `partial` (margin_ksplit(K) * Mrows * R values) and are summed in a fixed order.
template <typename T>
void margin_gemm(const cplx<T>* A, int64_t sm, int64_t sk, bool conjA, const cplx<T>* X, int64_t sxk, int64_t sxr,
                 cplx<T>* Y, int64_t ldy, int Mrows, int64_t K, int R, bool accumulate, cplx<T>* partial,
                 hipStream_t s);
int margin_ksplit(int64_t K);

// elementwise / conversion helpers (vec.hip)
template <typename TS, typename TD>
void convert(const TS* src, TD* dst, int64_t n, hipStream_t s);     // n complex values
void scatter_ports(const Geom& g, const int32_t* ports, int R, double2* V, hipStream_t s);  // V = unit delta gaps
void axpby_d(double2* y, const double2* x, double a, double b, int64_t n, hipStream_t s);  // y = a*x + b*y (real a,b)
template <typename TS>
void add_to_f64(double2* x, const TS* d, int64_t n, hipStream_t s);                         // x += d
void sub_d(const double2* a, const double2* b, double2* out, int64_t n, hipStream_t s);    // out = a - b
void column_norms(const double2* X, int64_t N, int R, double* partial, double* out, hipStream_t s);
// Y (P x R col-major) from the port-basis rows of the first R of the Rs columns of I
void gather_ports(const Geom& g, const double2* I, int Rs, int R, double2* Y, hipStream_t s);
void transpose_nr(const double2* src, double2* dst, int64_t N, int R, bool to_device_layout, hipStream_t s);
void scale_columns_d(double2* X, const double* scale, int64_t N, int R, hipStream_t s);      // X[n][r] *= scale[r]
void zero_d(double2* p, int64_t n, hipStream_t s);                                             // fill kernel, no memset
template <int FMT>
void pack16_d(const double2* src, uint32_t* dst, int64_t n, double scale, hipStream_t s);     // 16-bit of scale*src
void max_abs_d(const double2* src, int64_t n, double* out, hipStream_t s);                    // max |re|, |im| -> out[0]

}  // namespace mbt

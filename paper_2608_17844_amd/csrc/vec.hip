// Elementwise and layout kernels around the solve: precision casts, the port
// excitation, residual arithmetic, per-RHS norms, port-current gathers and
// host-layout transposes.
#include "common.h"

#include <algorithm>

namespace mbt {

namespace {

inline unsigned grid_for(int64_t n, int per = 256) {
    int64_t g = (n + per - 1) / per;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

template <typename TS, typename TD>
__global__ void convert_kernel(const TS* __restrict__ src, TD* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = from_d2<TD>(to_d2(src[i]));
}

template <int FMT>
__global__ void pack16_d_kernel(const double2* __restrict__ src, uint32_t* __restrict__ dst, int64_t n,
                                double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = src[i];
        dst[i] = pack16<FMT>(make_float2((float)(v.x * scale), (float)(v.y * scale)));
    }
}

// largest |re| or |im| over n complex values; one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void max_abs_kernel(const double2* __restrict__ src, int64_t n,
                                                       double* __restrict__ out) {
    __shared__ double red[1024];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double2 v = src[i];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// V[n][r] = the port weights at the port bases of element ports[r], 0 elsewhere (V pre-zeroed)
__global__ void scatter_ports_kernel(const int32_t* __restrict__ ports, int R, int M, PortDef pd, double2* V) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R)
        for (int i = 0; i < pd.n; ++i) V[((int64_t)ports[r] * M + pd.idx[i]) * R + r] = make_double2(pd.w[i], 0.0);
}

__global__ void axpby_kernel(double2* __restrict__ y, const double2* __restrict__ x, double a, double b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 xv = x[i], yv = y[i];
        y[i] = make_double2(a * xv.x + b * yv.x, a * xv.y + b * yv.y);
    }
}

template <typename TS>
__global__ void add_to_f64_kernel(double2* __restrict__ x, const TS* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 dv = to_d2(d[i]);
        double2 xv = x[i];
        x[i] = make_double2(xv.x + dv.x, xv.y + dv.y);
    }
}

__global__ void sub_kernel(const double2* __restrict__ a, const double2* __restrict__ b, double2* __restrict__ o, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = csub(a[i], b[i]);
}

// partial[chunk][r] = sum over rows of chunk |X[n][r]|^2 ; chunks of rows fixed by N only
__global__ void colnorm_partial_kernel(const double2* __restrict__ X, int64_t N, int R, int64_t rows_per_chunk,
                                       double* __restrict__ partial) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (r >= R) return;
    const int64_t n0 = chunk * rows_per_chunk, n1 = min(N, n0 + rows_per_chunk);
    double s = 0;
    for (int64_t n = n0; n < n1; ++n) {
        const double2 v = X[n * R + r];
        s += v.x * v.x + v.y * v.y;
    }
    partial[chunk * R + r] = s;
}

// out[r] = sqrt(sum over chunks of partial[c][r]): groups of 64 consecutive
// chunks in chunk order, then the group sums in group order (an order fixed by
// nchunk alone); the eight waves of a workgroup share the groups of 64 columns.
constexpr int kNormGroup = 64;
constexpr int kNormMaxChunks = 2048;
__global__ __launch_bounds__(512) void colnorm_final_kernel(const double* __restrict__ partial, int nchunk, int R,
                                                            double* __restrict__ out) {
    __shared__ double gs[kNormMaxChunks / kNormGroup][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    const int ng = (nchunk + kNormGroup - 1) / kNormGroup;
    for (int g = wave; g < ng; g += 8) {
        double sg = 0;
        if (r < R) {
            const int c1 = min(nchunk, (g + 1) * kNormGroup);
            for (int c = g * kNormGroup; c < c1; ++c) sg += partial[(int64_t)c * R + r];
        }
        gs[g][lane] = sg;
    }
    __syncthreads();
    if (wave == 0 && r < R) {
        double sum = gs[0][lane];
        for (int g = 1; g < ng; ++g) sum += gs[g][lane];
        out[r] = sqrt(sum);
    }
}

// Y[i + P*r] = sum_k w_k I[(i*M + idx_k)][r]   (column-major P x R output: the gap
// current of element i) for the first R of the Rs columns of I
__global__ void gather_ports_kernel(const double2* __restrict__ I, int P, int M, PortDef pd, int Rs, int R,
                                    double2* __restrict__ Y) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)P * R) return;
    const int i = (int)(t % P);
    const int r = (int)(t / P);
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < pd.n; ++k) {
        const double2 v = I[((int64_t)i * M + pd.idx[k]) * Rs + r];
        acc.x += pd.w[k] * v.x;
        acc.y += pd.w[k] * v.y;
    }
    Y[t] = acc;
}

// to_device_layout: dst[n][r] = src[n + N*r]; else dst[n + N*r] = src[n][r]
__global__ void transpose_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int64_t N, int R, int dir) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * (int64_t)R) return;
    const int64_t n = t / R;
    const int r = (int)(t % R);
    if (dir) dst[t] = src[n + N * r];
    else dst[n + N * r] = src[t];
}

__global__ void scale_columns_kernel(double2* __restrict__ X, const double* __restrict__ sc, int64_t N, int R) {
    const int64_t total = N * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const double f = sc[t % R];
        const double2 v = X[t];
        // a zero factor clears the column exactly, also where it holds Inf or NaN
        X[t] = f == 0.0 ? make_double2(0.0, 0.0) : make_double2(v.x * f, v.y * f);
    }
}

__global__ void zero_kernel_d(double2* __restrict__ p, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = make_double2(0, 0);
}

}  // namespace

void scale_columns_d(double2* X, const double* scale, int64_t N, int R, hipStream_t s) {
    hipLaunchKernelGGL(scale_columns_kernel, dim3(grid_for(N * R)), dim3(256), 0, s, X, scale, N, R);
    MBT_LAUNCH_CHECK();
}

void zero_d(double2* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(zero_kernel_d, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    MBT_LAUNCH_CHECK();
}

template <typename TS, typename TD>
void convert(const TS* src, TD* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((convert_kernel<TS, TD>), dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    MBT_LAUNCH_CHECK();
}
template void convert<double2, float2>(const double2*, float2*, int64_t, hipStream_t);
template void convert<float2, double2>(const float2*, double2*, int64_t, hipStream_t);
template void convert<double2, double2>(const double2*, double2*, int64_t, hipStream_t);
template void convert<float2, float2>(const float2*, float2*, int64_t, hipStream_t);

template <int FMT>
void pack16_d(const double2* src, uint32_t* dst, int64_t n, double scale, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((pack16_d_kernel<FMT>), dim3(grid_for(n)), dim3(256), 0, s, src, dst, n, scale);
    MBT_LAUNCH_CHECK();
}
template void pack16_d<kFmtBf16>(const double2*, uint32_t*, int64_t, double, hipStream_t);
template void pack16_d<kFmtF16>(const double2*, uint32_t*, int64_t, double, hipStream_t);

void max_abs_d(const double2* src, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(max_abs_kernel, dim3(1), dim3(1024), 0, s, src, n, out);
    MBT_LAUNCH_CHECK();
}

void scatter_ports(const Geom& g, const int32_t* ports, int R, double2* V, hipStream_t s) {
    zero_d(V, g.N * R, s);
    hipLaunchKernelGGL(scatter_ports_kernel, dim3((R + 255) / 256), dim3(256), 0, s, ports, R, g.M, g.port, V);
    MBT_LAUNCH_CHECK();
}

void axpby_d(double2* y, const double2* x, double a, double b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, b, n);
    MBT_LAUNCH_CHECK();
}

template <typename TS>
void add_to_f64(double2* x, const TS* d, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((add_to_f64_kernel<TS>), dim3(grid_for(n)), dim3(256), 0, s, x, d, n);
    MBT_LAUNCH_CHECK();
}
template void add_to_f64<double2>(double2*, const double2*, int64_t, hipStream_t);
template void add_to_f64<float2>(double2*, const float2*, int64_t, hipStream_t);

void sub_d(const double2* a, const double2* b, double2* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(sub_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, b, out, n);
    MBT_LAUNCH_CHECK();
}

// partial must hold nchunk*R doubles with nchunk = ceil(N / rows_per_chunk), rows_per_chunk = 256
void column_norms(const double2* X, int64_t N, int R, double* partial, double* out, hipStream_t s) {
    // at least 256 rows per chunk, at most kNormMaxChunks chunks (partial holds ceil(N/256) x R)
    const int64_t rpc = std::max<int64_t>(256, (N + kNormMaxChunks - 1) / kNormMaxChunks);
    const int nchunk = (int)((N + rpc - 1) / rpc);
    hipLaunchKernelGGL(colnorm_partial_kernel, dim3((R + 63) / 64, nchunk), dim3(64), 0, s, X, N, R, rpc, partial);
    MBT_LAUNCH_CHECK();
    hipLaunchKernelGGL(colnorm_final_kernel, dim3((R + 63) / 64), dim3(512), 0, s, partial, nchunk, R, out);
    MBT_LAUNCH_CHECK();
}

void gather_ports(const Geom& g, const double2* I, int Rs, int R, double2* Y, hipStream_t s) {
    MBT_REQUIRE(R <= Rs, "gather_ports: more columns than solved");
    const int64_t n = (int64_t)g.P * R;
    hipLaunchKernelGGL(gather_ports_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, I, g.P, g.M, g.port, Rs,
                       R, Y);
    MBT_LAUNCH_CHECK();
}

void transpose_nr(const double2* src, double2* dst, int64_t N, int R, bool to_device_layout, hipStream_t s) {
    const int64_t n = N * R;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, N, R,
                       to_device_layout ? 1 : 0);
    MBT_LAUNCH_CHECK();
}

}  // namespace mbt

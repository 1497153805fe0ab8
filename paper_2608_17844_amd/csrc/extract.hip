// Port quantities on the device, FP64.
//
// * Z_p = Y_p^{-1}: the open-circuit port impedance (paper eq. (passZ)) from
//   the short-circuit admittance that unit delta-gap excitations give;
// * S = (Z_p - z0)(Z_p + z0)^{-1} = I - 2 z0 (Z_p + z0)^{-1}, eq. (S2Z) solved
//   for S;
// * the center element's active impedance for phased port currents
//   I_j = exp(+j k (x_j u + y_j v)) (eqs. (actZ), (actZmat)), its ARC
//   (eq. (ARC)), and the wave-excited reflection coefficient, the phased S-sum
//   of Sec. II-D.
//
// The dense inverses use Gauss-Jordan elimination with partial pivoting: one
// pivot/scale kernel and one rank-1 elimination kernel per column.
#include "common.h"
#include "extract.h"

#include <vector>

namespace mbt {

namespace {

constexpr int kPivT = 1024;

// argmax |A[i][k]| over i >= k (ties -> smallest i), swap rows k and p, scale
// row k by 1/A[k][k] (with A[k][k] replaced by 1), save column k multipliers.
__global__ __launch_bounds__(kPivT) void gj_pivot_kernel(double2* __restrict__ A, int n, int k, double2* __restrict__ colbuf,
                                                         int* __restrict__ piv, int* __restrict__ singular) {
    __shared__ double sv[kPivT];
    __shared__ int si[kPivT];
    const int tid = threadIdx.x;
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += kPivT) {
        const double2 v = A[(int64_t)i * n + k];
        const double m = v.x * v.x + v.y * v.y;
        if (m > best) { best = m; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = kPivT / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double o = sv[tid + s];
            const int oi = si[tid + s];
            if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
        }
        __syncthreads();
    }
    const int p = si[0];
    if (tid == 0) {
        piv[k] = p;
        if (!(sv[0] > 0.0)) singular[0] = 1;
    }
    if (p != k && p < n)
        for (int j = tid; j < n; j += kPivT) {
            const double2 t = A[(int64_t)k * n + j];
            A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
            A[(int64_t)p * n + j] = t;
        }
    __syncthreads();
    const double2 d = A[(int64_t)k * n + k];
    const double den = d.x * d.x + d.y * d.y;
    const double2 dinv = den > 0.0 ? make_double2(d.x / den, -d.y / den) : make_double2(0, 0);
    for (int i = tid; i < n; i += kPivT) colbuf[i] = (i == k) ? make_double2(0, 0) : A[(int64_t)i * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += kPivT) {
        const double2 v = (j == k) ? make_double2(1.0, 0.0) : A[(int64_t)k * n + j];
        A[(int64_t)k * n + j] = cmul(v, dinv);
    }
}

__global__ void gj_elim_kernel(double2* __restrict__ A, int n, int k, const double2* __restrict__ colbuf) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    if (i == k) return;
    const double2 base = (j == k) ? make_double2(0, 0) : A[t];
    A[t] = csub(base, cmul(colbuf[i], A[(int64_t)k * n + j]));
}

// out[i][j] = in[i][src[j]]
__global__ void permute_cols_kernel(const double2* __restrict__ in, double2* __restrict__ out, int n,
                                    const int* __restrict__ src) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    out[t] = in[(int64_t)i * n + src[j]];
}

__global__ void add_diag_kernel(const double2* __restrict__ in, double2* __restrict__ out, int n, double z) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    double2 v = in[t];
    if (t / n == t % n) v.x += z;
    out[t] = v;
}

// S = I - 2 z0 B
__global__ void s_from_inv_kernel(const double2* __restrict__ B, double2* __restrict__ S, int n, double z0) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const double2 b = B[t];
    S[t] = make_double2(((t / n == t % n) ? 1.0 : 0.0) - 2.0 * z0 * b.x, -2.0 * z0 * b.y);
}

// One workgroup per scan direction.  Zp and S are column-major P x P.
__global__ __launch_bounds__(256) void scan_kernel(const double2* __restrict__ Zp, const double2* __restrict__ S, int nx,
                                                   int ny, double dx, double dy, double k, int c,
                                                   const double* __restrict__ theta, const double* __restrict__ phi,
                                                   double z0, double2* __restrict__ Za, double2* __restrict__ G,
                                                   double2* __restrict__ Gw) {
    __shared__ double2 sz[256], ss[256];
    const int sidx = blockIdx.x;
    const int P = nx * ny;
    const double u = sin(theta[sidx]) * cos(phi[sidx]);
    const double v = sin(theta[sidx]) * sin(phi[sidx]);
    double2 az = make_double2(0, 0), as = make_double2(0, 0);
    for (int j = threadIdx.x; j < P; j += 256) {
        const double xj = (j % nx) * dx, yj = (j / nx) * dy;
        double sn, cs;
        sincos(k * (xj * u + yj * v), &sn, &cs);
        const double2 ph = make_double2(cs, sn);
        az = cadd(az, cmul(Zp[(int64_t)j * P + c], ph));
        if (S) as = cadd(as, cmul(S[(int64_t)j * P + c], ph));
    }
    sz[threadIdx.x] = az;
    ss[threadIdx.x] = as;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sz[threadIdx.x] = cadd(sz[threadIdx.x], sz[threadIdx.x + s]);
            ss[threadIdx.x] = cadd(ss[threadIdx.x], ss[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double xc = (c % nx) * dx, yc = (c / nx) * dy;
        double sn, cs;
        sincos(k * (xc * u + yc * v), &sn, &cs);
        const double2 pc = make_double2(cs, -sn);   // 1 / I_c
        const double2 za = cmul(sz[0], pc);
        Za[sidx] = za;
        const double2 num = make_double2(za.x - z0, za.y), den = make_double2(za.x + z0, za.y);
        const double dd = den.x * den.x + den.y * den.y;
        G[sidx] = make_double2((num.x * den.x + num.y * den.y) / dd, (num.y * den.x - num.x * den.y) / dd);
        if (Gw) Gw[sidx] = cmul(ss[0], pc);
    }
}

inline unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// In-place Gauss-Jordan on A (n x n, any consistent layout: the inverse of the
// stored array is returned in the same layout).  Workspace: n complex + 2n ints.
void gj_inverse(double2* A, double2* out, int n, double2* colbuf, int* piv, int* flag, hipStream_t s) {
    MBT_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kPivT), 0, s, A, n, k, colbuf, piv, flag);
        hipLaunchKernelGGL(gj_elim_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, A, n, k, colbuf);
    }
    MBT_LAUNCH_CHECK();
    std::vector<int> hp(n);
    int hflag = 0;
    MBT_HIP(hipMemcpyAsync(hp.data(), piv, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    if (hflag) throw Error(-1, "port matrix is singular");
    // the row interchanges of the elimination become column interchanges of the inverse, last first
    std::vector<int> src(n);
    for (int j = 0; j < n; ++j) src[j] = j;
    for (int k = n - 1; k >= 0; --k) {
        if (hp[k] < 0 || hp[k] >= n) throw Error(-1, "port matrix is singular");
        std::swap(src[k], src[hp[k]]);
    }
    MBT_HIP(hipMemcpyAsync(piv, src.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(permute_cols_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, A, out, n, piv);
    MBT_LAUNCH_CHECK();
    MBT_HIP(hipStreamSynchronize(s));
}

void s_matrix(const double2* Zp, double2* S, double2* work, int n, double z0, double2* colbuf, int* piv, int* flag,
              hipStream_t s) {
    hipLaunchKernelGGL(add_diag_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, Zp, work, n, z0);
    MBT_LAUNCH_CHECK();
    gj_inverse(work, S, n, colbuf, piv, flag, s);        // S holds (Zp + z0)^{-1}
    hipLaunchKernelGGL(s_from_inv_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, S, S, n, z0);
    MBT_LAUNCH_CHECK();
}

void scans(const Geom& g, double k, const double2* Zp, const double2* S, int c, const double* theta, const double* phi,
           int nscan, double z0, double2* Za, double2* G, double2* Gw, hipStream_t s) {
    if (nscan <= 0) return;
    hipLaunchKernelGGL(scan_kernel, dim3(nscan), dim3(256), 0, s, Zp, S, g.nx, g.ny, g.dx, g.dy, k, c, theta, phi, z0,
                       Za, G, Gw);
    MBT_LAUNCH_CHECK();
}

}  // namespace mbt

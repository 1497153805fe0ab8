// Inter-element coupling predictors of the center element (paper Sec. II-E),
// computed on the device from a port impedance matrix in FP64:
//
// * xi_Z (eq. (predZ)): |Z_p,cj| / |Z_p,cc| for the border element j nearest to
//   the center c, the maximum of that ratio over the border (the form before
//   eq. (predZ)) and the border sum of |Z_p,cn| that bounds the change of the
//   active impedance (eq. (badpred));
// * C_n (eq. (amitayPred)): Fourier coefficients of the center element's
//   active reflection coefficient on the E-plane cut, Gamma_a(psi) =
//   sum_j S_cj exp(j n_j psi) (n_j the column offset of element j from the
//   center column, uniform amplitudes), integrated over psi in [-pi, pi) with
//   the nq-point trapezoid rule (exact for nq >= nx).  Sampling psi uniformly
//   samples the scan angles theta = asin(psi / (k dx)) of eq. (amitayPredTheta);
// * xi_S (eq. (predS)): |[z0 (1 + S_ideal)(1 - S_ideal)^{-1}]_cj| / |Z_p,cc|
//   with S_ideal S_cc on the diagonal and S_1 rho^a exp(-j k (r - dx)) off it
//   (rho the lattice-index distance, r the physical distance, a the decay
//   exponent, -2 for an infinite planar array).
//
// The border is the outer ring of the lattice (an axis of extent 1 has none);
// "nearest" is the smallest physical distance, ties to the smallest index;
// S_1 is the coupling of c to its +x neighbour.
#include "runtime.h"

#include <cmath>
#include <cstring>

#include "extract.h"

using namespace mbt;

namespace {

constexpr int kPT = 256;

__device__ __forceinline__ bool on_border(int e, int nx, int ny) {
    const int ix = e % nx, iy = e / nx;
    return (nx > 1 && (ix == 0 || ix == nx - 1)) || (ny > 1 && (iy == 0 || iy == ny - 1));
}

// out[0] = xi_z, out[1] = xi_z_max, out[2] = border_sum, out[3] = nearest (as double),
// out[4..5] = S_cc, out[6..7] = S_1.  Zp, S column-major P x P.  One workgroup.
__global__ __launch_bounds__(kPT) void xi_z_kernel(const double2* __restrict__ Zp, const double2* __restrict__ S,
                                                   int nx, int ny, double dx, double dy, int c,
                                                   double* __restrict__ out) {
    __shared__ double smax[kPT], ssum[kPT], sdist[kPT];
    __shared__ int sidx[kPT];
    const int P = nx * ny;
    const int t = threadIdx.x;
    const double xc = (c % nx) * dx, yc = (c / nx) * dy;
    double mx = 0.0, sm = 0.0, best = INFINITY;
    int bi = P;
    for (int e = t; e < P; e += kPT) {
        if (e == c || !on_border(e, nx, ny)) continue;
        const double2 z = Zp[c + (int64_t)P * e];
        const double a = hypot(z.x, z.y);
        mx = fmax(mx, a);
        sm += a;
        const double d2 = hypot((e % nx) * dx - xc, (e / nx) * dy - yc);
        if (d2 < best || (d2 == best && e < bi)) {
            best = d2;
            bi = e;
        }
    }
    smax[t] = mx;
    ssum[t] = sm;
    sdist[t] = best;
    sidx[t] = bi;
    __syncthreads();
    for (int s = kPT / 2; s > 0; s >>= 1) {
        if (t < s) {
            smax[t] = fmax(smax[t], smax[t + s]);
            ssum[t] += ssum[t + s];
            if (sdist[t + s] < sdist[t] || (sdist[t + s] == sdist[t] && sidx[t + s] < sidx[t])) {
                sdist[t] = sdist[t + s];
                sidx[t] = sidx[t + s];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        const double2 zcc = Zp[c + (int64_t)P * c];
        const double acc = hypot(zcc.x, zcc.y);
        const int j = sidx[0];
        const double2 zcj = Zp[c + (int64_t)P * j];
        out[0] = hypot(zcj.x, zcj.y) / acc;
        out[1] = smax[0] / acc;
        out[2] = ssum[0];
        out[3] = (double)j;
        const double2 scc = S[c + (int64_t)P * c];
        const double2 s1 = S[c + (int64_t)P * (c + 1)];
        out[4] = scc.x;
        out[5] = scc.y;
        out[6] = s1.x;
        out[7] = s1.y;
    }
}

// Gamma_a(psi_q) for psi_q = -pi + 2 pi q / nq: one workgroup per q.
__global__ __launch_bounds__(kPT) void eplane_arc_kernel(const double2* __restrict__ S, int nx, int P, int c, int nq,
                                                         double2* __restrict__ G) {
    __shared__ double2 sacc[kPT];
    const int q = blockIdx.x;
    const double psi = -M_PI + 2.0 * M_PI * q / nq;
    const int ixc = c % nx;
    double2 acc = make_double2(0, 0);
    for (int j = threadIdx.x; j < P; j += kPT) {
        double sn, cs;
        sincos((double)(j % nx - ixc) * psi, &sn, &cs);
        acc = cadd(acc, cmul(S[c + (int64_t)P * j], make_double2(cs, sn)));
    }
    sacc[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kPT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sacc[threadIdx.x] = cadd(sacc[threadIdx.x], sacc[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) G[q] = sacc[0];
}

// C_n = (1/nq) sum_q Gamma_a(psi_q) exp(-j n psi_q), n = i - ixc for i < nx.
__global__ void column_coupling_kernel(const double2* __restrict__ G, int nq, int nx, int ixc,
                                       double2* __restrict__ C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    const int n = i - ixc;
    double2 acc = make_double2(0, 0);
    for (int q = 0; q < nq; ++q) {
        const double psi = -M_PI + 2.0 * M_PI * q / nq;
        double sn, cs;
        sincos((double)n * psi, &sn, &cs);
        acc = cadd(acc, cmul(G[q], make_double2(cs, -sn)));
    }
    C[i] = make_double2(acc.x / nq, acc.y / nq);
}

__device__ __forceinline__ double2 ideal_entry(int a, int b, int nx, double dx, double dy, double k, double2 scc,
                                               double2 s1, double decay) {
    if (a == b) return scc;
    const int dix = a % nx - b % nx, diy = a / nx - b / nx;
    const double rho = hypot((double)dix, (double)diy);
    const double r = hypot(dix * dx, diy * dy);
    const double amp = pow(rho, decay);
    double sn, cs;
    sincos(-k * (r - dx), &sn, &cs);
    return cmul(s1, make_double2(amp * cs, amp * sn));
}

// W = I - S_ideal (column-major P x P)
__global__ void ideal_w_kernel(int nx, int P, double dx, double dy, double k, double2 scc, double2 s1,
                               double decay, double2* __restrict__ W) {
    const int64_t n = (int64_t)P * P;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(t % P), b = (int)(t / P);
        const double2 s = ideal_entry(a, b, nx, dx, dy, k, scc, s1, decay);
        W[t] = make_double2((a == b ? 1.0 : 0.0) - s.x, -s.y);
    }
}

// out = z0 sum_k (I + S_ideal)[c, k] Winv[k, j]  (one workgroup)
__global__ __launch_bounds__(kPT) void ideal_z_entry_kernel(const double2* __restrict__ Winv, int nx, int P,
                                                            double dx, double dy, double k, double2 scc,
                                                            double2 s1, double decay, int c, int j, double z0,
                                                            double2* __restrict__ out) {
    __shared__ double2 sacc[kPT];
    double2 acc = make_double2(0, 0);
    for (int kk = threadIdx.x; kk < P; kk += kPT) {
        double2 a = ideal_entry(c, kk, nx, dx, dy, k, scc, s1, decay);
        if (kk == c) a.x += 1.0;
        acc = cadd(acc, cmul(a, Winv[kk + (int64_t)P * j]));
    }
    sacc[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kPT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sacc[threadIdx.x] = cadd(sacc[threadIdx.x], sacc[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = make_double2(z0 * sacc[0].x, z0 * sacc[0].y);
}

struct LatInfo {
    int nx, ny, P, c;
};

LatInfo check_lattice(const mbt_lattice* lat, int32_t center) {
    MBT_REQUIRE(lat != nullptr, "NULL lattice");
    MBT_REQUIRE(lat->nx >= 1 && lat->ny >= 1 && lat->nx <= 64 && lat->ny <= 64,
                "lattice size must be within 1..64 per axis");
    MBT_REQUIRE(lat->dx > 0 && lat->dy > 0 && std::isfinite(lat->dx) && std::isfinite(lat->dy),
                "lattice spacing must be positive");
    LatInfo li;
    li.nx = lat->nx;
    li.ny = lat->ny;
    li.P = lat->nx * lat->ny;
    li.c = center < 0 ? (lat->ny / 2) * lat->nx + lat->nx / 2 : center;
    MBT_REQUIRE(li.c >= 0 && li.c < li.P, "center out of range");
    MBT_REQUIRE(li.c % li.nx + 1 < li.nx, "the center element needs a +x neighbour (S_1)");
    // a border element other than c
    bool any = false;
    for (int e = 0; e < li.P && !any; ++e) {
        const int ix = e % li.nx, iy = e / li.nx;
        const bool b = (li.nx > 1 && (ix == 0 || ix == li.nx - 1)) || (li.ny > 1 && (iy == 0 || iy == li.ny - 1));
        any = b && e != li.c;
    }
    MBT_REQUIRE(any, "the array has no border element other than the center");
    return li;
}

int nearest_border_host(const LatInfo& li, double dx, double dy) {
    const double xc = (li.c % li.nx) * dx, yc = (li.c / li.nx) * dy;
    double best = INFINITY;
    int bi = -1;
    for (int e = 0; e < li.P; ++e) {
        const int ix = e % li.nx, iy = e / li.nx;
        const bool b = (li.nx > 1 && (ix == 0 || ix == li.nx - 1)) || (li.ny > 1 && (iy == 0 || iy == li.ny - 1));
        if (!b || e == li.c) continue;
        const double d2 = std::hypot(ix * dx - xc, iy * dy - yc);
        if (d2 < best) {
            best = d2;
            bi = e;
        }
    }
    return bi;
}

}  // namespace

#define API_BEGIN \
    try {
#define API_END                                                                                       \
    }                                                                                                 \
    catch (const mbt::Error& e) { set_last_error(e.what()); return (mbt_status)e.code; }              \
    catch (const std::bad_alloc&) { set_last_error("host allocation failed"); return MBT_ENOMEM; }    \
    catch (const std::exception& e) { set_last_error(e.what()); return MBT_EDEVICE; }                 \
    set_last_error("");                                                                               \
    return MBT_OK;

extern "C" {

mbt_status mbt_predict(mbt_ctx* ctx, const mbt_lattice* lat, const double* Zp, int32_t center, double z0, int32_t nq,
                       mbt_predictors* out, double* Cn, double* Gamma_psi) {
    API_BEGIN
    MBT_REQUIRE(ctx && Zp && out && Cn, "NULL argument");
    MBT_REQUIRE(z0 > 0 && std::isfinite(z0), "z0 must be positive");
    MBT_REQUIRE(nq >= 1 && nq <= 65536, "nq must be in 1..65536");
    const LatInfo li = check_lattice(lat, center);
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    MBT_HIP(hipSetDevice(ctx->device));
    hipStream_t str = ctx->main->stream;
    const int P = li.P;
    DBuf Zd, Sd, Wd, aux;
    Zd.alloc(sizeof(double2) * P * P);
    Sd.alloc(sizeof(double2) * P * P);
    Wd.alloc(sizeof(double2) * P * P);
    aux.alloc(sizeof(double2) * ((size_t)P + nq + li.nx + 8) + sizeof(int) * (P + 8) + 1024);
    double2* colbuf = aux.as<double2>();
    double2* G = colbuf + P;
    double2* C = G + nq;
    double* res = reinterpret_cast<double*>(C + li.nx);
    int* piv = reinterpret_cast<int*>(res + 8);
    int* flag = piv + P;
    MBT_HIP(hipMemcpyAsync(Zd.p, Zp, sizeof(double2) * P * P, hipMemcpyHostToDevice, str));
    s_matrix(Zd.as<double2>(), Sd.as<double2>(), Wd.as<double2>(), P, z0, colbuf, piv, flag, str);
    hipLaunchKernelGGL(xi_z_kernel, dim3(1), dim3(kPT), 0, str, Zd.as<double2>(), Sd.as<double2>(), li.nx, li.ny,
                       lat->dx, lat->dy, li.c, res);
    hipLaunchKernelGGL(eplane_arc_kernel, dim3(nq), dim3(kPT), 0, str, Sd.as<double2>(), li.nx, P, li.c, nq, G);
    hipLaunchKernelGGL(column_coupling_kernel, dim3((li.nx + 63) / 64), dim3(64), 0, str, G, nq, li.nx,
                       li.c % li.nx, C);
    MBT_LAUNCH_CHECK();
    double h[8];
    MBT_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, str));
    MBT_HIP(hipMemcpyAsync(Cn, C, sizeof(double2) * li.nx, hipMemcpyDeviceToHost, str));
    if (Gamma_psi) MBT_HIP(hipMemcpyAsync(Gamma_psi, G, sizeof(double2) * nq, hipMemcpyDeviceToHost, str));
    MBT_HIP(hipStreamSynchronize(str));
    std::memset(out, 0, sizeof(*out));
    out->xi_z = h[0];
    out->xi_z_max = h[1];
    out->border_sum = h[2];
    out->nearest = (int32_t)h[3];
    out->center = li.c;
    out->s_cc[0] = h[4];
    out->s_cc[1] = h[5];
    out->s_1[0] = h[6];
    out->s_1[1] = h[7];
    API_END
}

mbt_status mbt_predict_xi_s(mbt_ctx* ctx, const mbt_lattice* lat, double freq_ratio, const double* s_cc,
                            const double* s_1, double zp_cc_abs, double z0, double decay, int32_t center,
                            double* xi_s) {
    API_BEGIN
    MBT_REQUIRE(ctx && s_cc && s_1 && xi_s, "NULL argument");
    MBT_REQUIRE(freq_ratio > 0 && std::isfinite(freq_ratio), "freq_ratio must be positive");
    MBT_REQUIRE(z0 > 0 && std::isfinite(z0) && zp_cc_abs > 0 && std::isfinite(zp_cc_abs),
                "z0 and |Z_p,cc| must be positive");
    MBT_REQUIRE(std::isfinite(decay), "decay must be finite");
    MBT_REQUIRE(std::isfinite(s_cc[0]) && std::isfinite(s_cc[1]) && std::isfinite(s_1[0]) && std::isfinite(s_1[1]),
                "S_cc and S_1 must be finite");
    const LatInfo li = check_lattice(lat, center);
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    MBT_HIP(hipSetDevice(ctx->device));
    hipStream_t str = ctx->main->stream;
    const int P = li.P;
    const int j = nearest_border_host(li, lat->dx, lat->dy);
    const double k = 2.0 * M_PI * freq_ratio;
    const double2 scc = make_double2(s_cc[0], s_cc[1]), s1 = make_double2(s_1[0], s_1[1]);
    DBuf Wd, Wi, aux;
    Wd.alloc(sizeof(double2) * P * P);
    Wi.alloc(sizeof(double2) * P * P);
    aux.alloc(sizeof(double2) * ((size_t)P + 8) + sizeof(int) * (P + 8) + 1024);
    double2* colbuf = aux.as<double2>();
    double2* zc = colbuf + P;
    int* piv = reinterpret_cast<int*>(zc + 8);
    int* flag = piv + P;
    const int64_t n = (int64_t)P * P;
    hipLaunchKernelGGL(ideal_w_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65535)), dim3(256), 0, str,
                       li.nx, P, lat->dx, lat->dy, k, scc, s1, decay, Wd.as<double2>());
    MBT_LAUNCH_CHECK();
    gj_inverse(Wd.as<double2>(), Wi.as<double2>(), P, colbuf, piv, flag, str);
    hipLaunchKernelGGL(ideal_z_entry_kernel, dim3(1), dim3(kPT), 0, str, Wi.as<double2>(), li.nx, P, lat->dx,
                       lat->dy, k, scc, s1, decay, li.c, j, z0, zc);
    MBT_LAUNCH_CHECK();
    double2 h;
    MBT_HIP(hipMemcpyAsync(&h, zc, sizeof(h), hipMemcpyDeviceToHost, str));
    MBT_HIP(hipStreamSynchronize(str));
    *xi_s = std::hypot(h.x, h.y) / zp_cc_abs;
    API_END
}

}  // extern "C"

// Unique interaction blocks of the multilevel block-Toeplitz impedance matrix.
//
// On a regular lattice the M x M block between two elements depends only on
// their lattice offset d (paper Sec. II-A, eq. (Zblock) and the structure of
// Fig. ToepStruct), so only the (2ny-1)(2nx-1) blocks T[d] are filled.  The
// element is the z-directed thin-wire dipole: Galerkin EFIE, rooftop bases on
// Ns = M+1 equal segments, reduced kernel exp(-jkR)/(4 pi R) with
// R = sqrt(rho^2 + (z-z')^2 + a^2) for every pair, four-point Gauss-Legendre on
// each segment, and Z_mn = j eta (k A_mn - Phi_mn / k).
//
// Because the segments are uniform, every segment-pair integral depends only on
// the segment difference delta = sigma - tau; one workgroup per offset first
// evaluates the four shape moments of the kernel for all 2M+1 differences, then
// assembles the block from them.  The FP64 work is transcendental-bound
// (sqrt, sincos) and negligible next to the solve.
#include "common.h"

namespace mbt {

namespace {

constexpr double kEta0 = 376.730313668;

struct GL4 {
    double u[4], w[4];
};

__device__ __forceinline__ GL4 gl4_unit() {
    // nodes +-sqrt(3/7 -+ (2/7) sqrt(6/5)) and weights (18 +- sqrt 30)/36 on [-1,1], mapped to [0,1]
    const double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double wa = (18.0 + sqrt(30.0)) / 36.0;
    const double wb = (18.0 - sqrt(30.0)) / 36.0;
    GL4 r;
    const double x[4] = {-b, -a, a, b};
    const double w[4] = {wb, wa, wa, wb};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        r.u[i] = 0.5 * (1.0 + x[i]);
        r.w[i] = 0.5 * w[i];
    }
    return r;
}

constexpr int kMaxM = 64;                   // bases per element supported by the fill
constexpr int kMaxDelta = 2 * kMaxM + 1;

__global__ __launch_bounds__(256) void fill_blocks_kernel(int nx, int ny, int M, double dx, double dy,
                                                          double L, double a, double k, double2* __restrict__ T) {
    __shared__ double2 S0[kMaxDelta], Su[kMaxDelta], Sv[kMaxDelta], Suv[kMaxDelta];
    const int nox = 2 * nx - 1;
    const int64_t blk = blockIdx.x;
    const int ox = (int)(blk % nox) - (nx - 1);
    const int oy = (int)(blk / nox) - (ny - 1);
    const double rx = ox * dx, ry = oy * dy;
    const double rho2 = rx * rx + ry * ry;
    const double D = L / (double)(M + 1);
    const GL4 q = gl4_unit();
    const double inv4pi = 0.25 / M_PI;

    // moments over the 16 point pairs for segment difference delta = sigma - tau in [-M, M]
    for (int t = threadIdx.x; t < 2 * M + 1; t += blockDim.x) {
        const int delta = t - M;
        double s0r = 0, s0i = 0, sur = 0, sui = 0, svr = 0, svi = 0, suvr = 0, suvi = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double dz = ((double)delta + q.u[i] - q.u[j]) * D;
                const double R = sqrt(rho2 + dz * dz + a * a);
                double sn, cs;
                sincos(k * R, &sn, &cs);
                const double wg = q.w[i] * q.w[j] * D * D * inv4pi / R;
                const double gr = cs * wg, gi = -sn * wg;
                s0r += gr;                        s0i += gi;
                sur += q.u[i] * gr;               sui += q.u[i] * gi;
                svr += q.u[j] * gr;               svi += q.u[j] * gi;
                suvr += q.u[i] * q.u[j] * gr;     suvi += q.u[i] * q.u[j] * gi;
            }
        }
        S0[t] = make_double2(s0r, s0i);
        Su[t] = make_double2(sur, sui);
        Sv[t] = make_double2(svr, svi);
        Suv[t] = make_double2(suvr, suvi);
    }
    __syncthreads();

    double2* out = T + blk * (int64_t)M * M;
    const double invD2 = 1.0 / (D * D);
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        const int p = e / M, qq = e % M;
        const int d0 = p - qq + M;        // (rise, rise) and (fall, fall): delta = p - q
        const int dm = d0 - 1;            // (rise test, fall source): sigma = p, tau = q+1
        const int dp = d0 + 1;            // (fall test, rise source): sigma = p+1, tau = q
        double2 A;
        A.x = Suv[d0].x + (Su[dm].x - Suv[dm].x) + (Sv[dp].x - Suv[dp].x) +
              (S0[d0].x - Su[d0].x - Sv[d0].x + Suv[d0].x);
        A.y = Suv[d0].y + (Su[dm].y - Suv[dm].y) + (Sv[dp].y - Suv[dp].y) +
              (S0[d0].y - Su[d0].y - Sv[d0].y + Suv[d0].y);
        double2 Ph;
        Ph.x = (2.0 * S0[d0].x - S0[dm].x - S0[dp].x) * invD2;
        Ph.y = (2.0 * S0[d0].y - S0[dm].y - S0[dp].y) * invD2;
        const double tr = k * A.x - Ph.x / k;
        const double ti = k * A.y - Ph.y / k;
        out[e] = make_double2(-kEta0 * ti, kEta0 * tr);   // j * eta * (t)
    }
}

}  // namespace

void fill_blocks(const Geom& g, double k, double2* T, hipStream_t s) {
    MBT_REQUIRE(g.M >= 1 && g.M <= kMaxM, "fill: nbases out of range (1..64)");
    hipLaunchKernelGGL(fill_blocks_kernel, dim3((unsigned)g.noff()), dim3(256), 0, s, g.nx, g.ny, g.M, g.dx,
                       g.dy, g.L, g.a, k, T);
    MBT_LAUNCH_CHECK();
}

}  // namespace mbt

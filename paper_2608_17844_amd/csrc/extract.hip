// Port quantities on the device, FP64.
//
// * Z_p = Y_p^{-1}: the open-circuit port impedance (paper eq. (passZ)) from
//   the short-circuit admittance that unit delta-gap excitations give;
// * S = (Z_p - z0)(Z_p + z0)^{-1} = I - 2 z0 (Z_p + z0)^{-1}, eq. (S2Z) solved
//   for S;
// * the center element's active impedance for port currents phased to steer
//   the main beam at (theta, phi) (Sec. II-E), I_j = exp(-j k (x_j u + y_j v))
//   under the e^{-jkR} kernel of the fill (eqs. (actZ), (actZmat)), its ARC
//   (eq. (ARC)), and the wave-excited reflection coefficient, the phased S-sum
//   of Sec. II-E;
// * for a phased voltage excitation of every gap, V_j = exp(-j k (x_j u + y_j v))
//   on the same beam-steering convention, the right-hand sides and, from the
//   gap currents the solve returns, the center element's active impedance
//   Z_a,c = V_c / I_p,c (eq. (actZ) with those port currents) and its ARC.
//
// The dense inverses use Gauss-Jordan elimination with partial pivoting.  For
// 64 <= n <= 1024 it is blocked: one workgroup factors a panel of eight
// columns with each row in its owner thread's registers, then applies the
// panel's row interchanges and pivot rows to the other columns; a rank-8
// update of the remaining rows follows, so the matrix is streamed once per
// panel instead of once per column.  Other sizes use one pivot kernel and one
// rank-1 elimination kernel per column.  The blocked pivot search compares
// magnitudes rounded to FP32 (ties: smallest row), the unblocked one in FP64.
#include "common.h"
#include "extract.h"

#include <algorithm>
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

// ---- blocked form (n <= kPanT: one row per thread of the panel workgroup)
constexpr int kPanT = 1024;       // threads of the panel workgroup
constexpr int kMaxPan = 8;        // columns per panel
constexpr int kBlockedMinN = 64;
constexpr int kUpdRows = 4;       // rows per thread of the rank-nb update

// Wave-wide maximum of a 64-bit key through DPP lane permutations (pairs,
// quads, eight, sixteen lanes) and the four row results read out of lanes 0,
// 16, 32 and 48.  Called by all 64 lanes.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t key) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)key, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(key >> 32), CTRL, 0xF, 0xF, false);
    const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    return o > key ? o : key;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t key) {
    key = dpp_max_step<0xB1>(key);    // quad_perm [1,0,3,2]
    key = dpp_max_step<0x4E>(key);    // quad_perm [2,3,0,1]
    key = dpp_max_step<0x141>(key);   // row_half_mirror
    key = dpp_max_step<0x140>(key);   // row_mirror
    uint64_t best = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, 16 * r);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), 16 * r);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        best = o > best ? o : best;
    }
    return best;
}

// Pivot key of row i: the FP32 bits of |v|^2 above the complement of i, so
// that the largest key is the largest magnitude and, among equal magnitudes
// (to FP32 rounding), the smallest row; rows out of the search have key 0.
__device__ __forceinline__ uint64_t pivot_key(double m, int i) {
    return ((uint64_t)__float_as_uint((float)m) << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
}

// Steps k0 .. k0+NB-1 of the elimination.  Thread i owns row i and keeps, in
// registers, its NB panel values and its multipliers L[c][i] (A[i][k] before
// the elimination of step c, 0 at i = k); the panel columns take the steps
// with the arithmetic of the unblocked kernels.  Per step, between two
// barriers: the pivot search, the interchange of two rows between their
// owners and the pivot row broadcast, both through LDS; then every row's
// update in its owner's registers.  At the end: the panel columns, L and piv
// go to memory, and every other column j takes the panel's row interchanges
// and its pivot rows (row k scaled, then eliminated from the other pivot
// rows); RK[c][j] keeps row k0+c as it is right after its scaling, the value
// the remaining rows are eliminated with (gj_update_kernel).
template <int NB>
__global__ __launch_bounds__(kPanT) void gj_panel_kernel(double2* __restrict__ A, int n, int k0,
                                                         double2* __restrict__ L, int* __restrict__ piv,
                                                         int* __restrict__ singular, double2* __restrict__ RK) {
    __shared__ uint64_t wkey[kPanT / 64];
    __shared__ int pv[NB];
    __shared__ double2 dv[NB];
    __shared__ double2 bcast[NB];              // the pivot row of the step, unscaled
    __shared__ double2 xk[2 * NB];             // old row k: values and multipliers
    __shared__ double2 xpl[NB];                // multipliers of old row p
    __shared__ double2 lp[NB][NB];             // lp[c][q] = L[c][k0 + q]
    __shared__ int psrc[NB], exd[NB], exs[NB], nex;
    const int tid = threadIdx.x;
    const int i = tid;
    const bool own = i < n;
    double2 rowv[NB], lreg[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        rowv[j] = own ? A[(int64_t)i * n + k0 + j] : make_double2(0, 0);
        lreg[j] = make_double2(0, 0);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int k = k0 + c;
        uint64_t key = 0;
        if (own && i >= k) {
            const double m = rowv[c].x * rowv[c].x + rowv[c].y * rowv[c].y;
            key = pivot_key(m, i);
        }
        key = wave_max_u64(key);
        if ((tid & 63) == 0) wkey[tid >> 6] = key;
        __syncthreads();
        uint64_t kk[kPanT / 64];
#pragma unroll
        for (int w = 0; w < kPanT / 64; ++w) kk[w] = wkey[w];
        uint64_t best = 0;
#pragma unroll
        for (int w = 0; w < kPanT / 64; ++w) best = kk[w] > best ? kk[w] : best;
        const int p = (int)(0xFFFFFFFFu - (uint32_t)best);
        const bool valid = best != 0 && p >= k && p < n;
        if (tid == 0) {
            pv[c] = valid ? p : n;
            if (!valid || !(__uint_as_float((uint32_t)(best >> 32)) > 0.0f)) singular[0] = 1;
        }
        const int pr = valid ? p : k;          // the row that becomes the pivot row
        if (own && i == pr)
#pragma unroll
            for (int j = 0; j < NB; ++j) bcast[j] = rowv[j];
        if (pr != k) {
            if (own && i == k)
#pragma unroll
                for (int j = 0; j < NB; ++j) { xk[j] = rowv[j]; xk[NB + j] = lreg[j]; }
            if (own && i == pr)
#pragma unroll
                for (int j = 0; j < NB; ++j) xpl[j] = lreg[j];
        }
        __syncthreads();
        double2 prow[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) prow[j] = bcast[j];
        if (pr != k) {
            if (own && i == k)
#pragma unroll
                for (int j = 0; j < NB; ++j) { rowv[j] = prow[j]; lreg[j] = xpl[j]; }
            if (own && i == pr)
#pragma unroll
                for (int j = 0; j < NB; ++j) { rowv[j] = xk[j]; lreg[j] = xk[NB + j]; }
        }
        const double2 d = prow[c];
        const double den = d.x * d.x + d.y * d.y;
        const double2 di = den > 0.0 ? make_double2(d.x / den, -d.y / den) : make_double2(0, 0);
        double2 rk[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) rk[j] = cmul((j == c) ? make_double2(1.0, 0.0) : prow[j], di);
        if (tid == 0) dv[c] = di;
        if (own) {
            if (i == k) {
                lreg[c] = make_double2(0, 0);
#pragma unroll
                for (int j = 0; j < NB; ++j) rowv[j] = rk[j];
            } else {
                const double2 l = rowv[c];
                lreg[c] = l;
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double2 base = (j == c) ? make_double2(0, 0) : rowv[j];
                    rowv[j] = csub(base, cmul(l, rk[j]));
                }
            }
        }
    }
    if (own) {
#pragma unroll
        for (int j = 0; j < NB; ++j) A[(int64_t)i * n + k0 + j] = rowv[j];
#pragma unroll
        for (int c = 0; c < NB; ++c) L[(int64_t)c * n + i] = lreg[c];
        if (i >= k0 && i < k0 + NB)
#pragma unroll
            for (int c = 0; c < NB; ++c) lp[c][i - k0] = lreg[c];
    }
    __syncthreads();
    if (tid < NB) piv[k0 + tid] = pv[tid];
    if (tid == 0) {
        // compose the interchanges on the rows they touch
        int rows[2 * NB], srcr[2 * NB];
        int m = 0;
        for (int c = 0; c < NB; ++c) { rows[m] = k0 + c; srcr[m] = k0 + c; ++m; }
        for (int c = 0; c < NB; ++c) {
            const int q = pv[c];
            if (q < 0 || q >= n || (q >= k0 && q < k0 + NB)) continue;
            bool seen = false;
            for (int x = NB; x < m; ++x) seen = seen || rows[x] == q;
            if (!seen) { rows[m] = q; srcr[m] = q; ++m; }
        }
        for (int c = 0; c < NB; ++c) {
            const int q = pv[c];
            if (q == k0 + c || q < 0 || q >= n) continue;
            int xa = 0, xb = 0;
            for (int x = 0; x < m; ++x) {
                if (rows[x] == k0 + c) xa = x;
                if (rows[x] == q) xb = x;
            }
            const int t = srcr[xa];
            srcr[xa] = srcr[xb];
            srcr[xb] = t;
        }
        int ne = 0;
        for (int c = 0; c < NB; ++c) psrc[c] = srcr[c];
        for (int x = NB; x < m; ++x)
            if (srcr[x] != rows[x]) { exd[ne] = rows[x]; exs[ne] = srcr[x]; ++ne; }
        nex = ne;
    }
    __syncthreads();
    // the other columns: row interchanges (all sources read before any row is
    // written), then the pivot rows
    const int j = tid;
    if (!own || (j >= k0 && j < k0 + NB)) return;
    const int ne = nex;
    double2 r[NB], ex[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) r[c] = A[(int64_t)psrc[c] * n + j];
#pragma unroll
    for (int e = 0; e < NB; ++e) ex[e] = e < ne ? A[(int64_t)exs[e] * n + j] : make_double2(0, 0);
#pragma unroll
    for (int e = 0; e < NB; ++e)
        if (e < ne) A[(int64_t)exd[e] * n + j] = ex[e];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        {
            r[c] = cmul(r[c], dv[c]);
            RK[(int64_t)c * n + j] = r[c];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q != c) r[q] = csub(r[q], cmul(lp[c][q], r[c]));
        }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
        A[(int64_t)(k0 + c) * n + j] = r[c];
}

// The rest: A[i][j] -= L[c][i] RK[c][j] over the panel's steps in order, for
// rows i and columns j outside the panel; a thread keeps RK[.][j] in registers
// for kUpdRows rows.
template <int NB>
__global__ void gj_update_kernel(double2* __restrict__ A, int n, int k0, const double2* __restrict__ L,
                                 const double2* __restrict__ RK) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i0 = blockIdx.y * kUpdRows;
    if (j >= n || (j >= k0 && j < k0 + NB)) return;
    double2 rk[NB], a[kUpdRows];
#pragma unroll
    for (int c = 0; c < NB; ++c) rk[c] = RK[(int64_t)c * n + j];
#pragma unroll
    for (int u = 0; u < kUpdRows; ++u) {
        const int i = i0 + u;
        a[u] = (i < n && !(i >= k0 && i < k0 + NB)) ? A[(int64_t)i * n + j] : make_double2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kUpdRows; ++u) {
        const int i = i0 + u;
        if (i < n && !(i >= k0 && i < k0 + NB)) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                a[u] = csub(a[u], cmul(L[(int64_t)c * n + i], rk[c]));
            A[(int64_t)i * n + j] = a[u];
        }
    }
}

// out[i][j] = in[i][src[j]]
__global__ void permute_cols_kernel(const double2* __restrict__ in, double2* __restrict__ out, int n,
                                    const int* __restrict__ src) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    out[t] = in[(int64_t)i * n + src[j]];
}

// The row interchanges of the elimination become column interchanges of the
// inverse, last first; one thread (n <= 1024 swaps).  An out-of-range pivot
// marks the matrix singular.
__global__ void perm_from_pivots_kernel(const int* __restrict__ piv, int* __restrict__ src, int n,
                                        int* __restrict__ flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int j = 0; j < n; ++j) src[j] = j;
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p < 0 || p >= n) {
            *flag = 1;
            return;
        }
        const int t = src[k];
        src[k] = src[p];
        src[p] = t;
    }
}

__global__ void clear_flag_kernel(int* flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
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
        const double2 ph = make_double2(cs, -sn);   // I_j = exp(-j k (x_j u + y_j v))
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
        const double2 pc = make_double2(cs, sn);    // 1 / I_c
        const double2 za = cmul(sz[0], pc);
        Za[sidx] = za;
        const double2 num = make_double2(za.x - z0, za.y), den = make_double2(za.x + z0, za.y);
        const double dd = den.x * den.x + den.y * den.y;
        G[sidx] = make_double2((num.x * den.x + num.y * den.y) / dd, (num.y * den.x - num.x * den.y) / dd);
        if (Gw) Gw[sidx] = cmul(ss[0], pc);
    }
}

inline unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int NB>
void launch_panel(double2* A, int n, int k0, double2* L, int* piv, int* flag, double2* RK, dim3 ug, hipStream_t s) {
    hipLaunchKernelGGL((gj_panel_kernel<NB>), dim3(1), dim3(kPanT), 0, s, A, n, k0, L, piv, flag, RK);
    hipLaunchKernelGGL((gj_update_kernel<NB>), ug, dim3(256), 0, s, A, n, k0, L, RK);
}

}  // namespace

// In-place Gauss-Jordan on A (n x n, any consistent layout: the inverse of the
// stored array is returned in the same layout).  Workspace: n complex + 2n ints;
// the blocked form also uses out (which must not overlap A) until the end.
void gj_inverse(double2* A, double2* out, int n, double2* colbuf, int* piv, int* flag, hipStream_t s) {
    MBT_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    const int nb = kMaxPan;
    if (n >= kBlockedMinN && n <= kPanT) {
        // out: L (nb x n), RK (nb x n); n >= 64 leaves room
        double2* L = out;
        double2* RK = out + (size_t)nb * n;
        const dim3 ug(g1(n), (unsigned)((n + kUpdRows - 1) / kUpdRows));
        for (int k0 = 0; k0 < n; k0 += nb) {
            switch (std::min(nb, n - k0)) {
            case 8: launch_panel<8>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 7: launch_panel<7>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 6: launch_panel<6>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 5: launch_panel<5>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 4: launch_panel<4>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 3: launch_panel<3>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 2: launch_panel<2>(A, n, k0, L, piv, flag, RK, ug, s); break;
            default: launch_panel<1>(A, n, k0, L, piv, flag, RK, ug, s); break;
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kPivT), 0, s, A, n, k, colbuf, piv, flag);
            hipLaunchKernelGGL(gj_elim_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, A, n, k, colbuf);
        }
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

// The elimination of gj_inverse with the column permutation formed on the
// device: no host buffers, one 4-byte readback of the singularity flag into
// pinned host memory.
static void gj_inverse_dev_perm(double2* A, double2* out, int n, double2* colbuf, int* piv, int* src, int* flag,
                                int* host_flag, hipStream_t s) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, flag);
    const int nb = kMaxPan;
    if (n >= kBlockedMinN && n <= kPanT) {
        double2* L = out;
        double2* RK = out + (size_t)nb * n;
        const dim3 ug(g1(n), (unsigned)((n + kUpdRows - 1) / kUpdRows));
        for (int k0 = 0; k0 < n; k0 += nb) {
            switch (std::min(nb, n - k0)) {
            case 8: launch_panel<8>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 7: launch_panel<7>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 6: launch_panel<6>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 5: launch_panel<5>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 4: launch_panel<4>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 3: launch_panel<3>(A, n, k0, L, piv, flag, RK, ug, s); break;
            case 2: launch_panel<2>(A, n, k0, L, piv, flag, RK, ug, s); break;
            default: launch_panel<1>(A, n, k0, L, piv, flag, RK, ug, s); break;
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kPivT), 0, s, A, n, k, colbuf, piv, flag);
            hipLaunchKernelGGL(gj_elim_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, A, n, k, colbuf);
        }
    }
    hipLaunchKernelGGL(perm_from_pivots_kernel, dim3(1), dim3(64), 0, s, piv, src, n, flag);
    hipLaunchKernelGGL(permute_cols_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, A, out, n, src);
    MBT_LAUNCH_CHECK();
    MBT_HIP(hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    if (*host_flag) throw Error(-1, "port matrix is singular");
}

void s_matrix_dev_perm(const double2* Zp, double2* S, double2* work, int n, double z0, double2* colbuf, int* piv,
                       int* src, int* flag, int* host_flag, hipStream_t s) {
    hipLaunchKernelGGL(add_diag_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, Zp, work, n, z0);
    MBT_LAUNCH_CHECK();
    gj_inverse_dev_perm(work, S, n, colbuf, piv, src, flag, host_flag, s);   // S holds (Zp + z0)^{-1}
    hipLaunchKernelGGL(s_from_inv_kernel, dim3(g1((int64_t)n * n)), dim3(256), 0, s, S, S, n, z0);
    MBT_LAUNCH_CHECK();
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

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// V[(e*M + idx_i)][r] = w_i exp(-j k (x_e u_r + y_e v_r)) for every element e (V pre-zeroed)
__global__ void scan_voltages_kernel(int nx, int P, double dx, double dy, double k, const double* __restrict__ theta,
                                     const double* __restrict__ phi, int R, int M, PortDef pd,
                                     double2* __restrict__ V) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)P * R) return;
    const int r = (int)(t % R);
    const int e = (int)(t / R);
    const double u = sin(theta[r]) * cos(phi[r]), v = sin(theta[r]) * sin(phi[r]);
    double sn, cs;
    sincos(k * ((e % nx) * dx * u + (e / nx) * dy * v), &sn, &cs);
    for (int i = 0; i < pd.n; ++i) V[((int64_t)e * M + pd.idx[i]) * R + r] = make_double2(pd.w[i] * cs, -pd.w[i] * sn);
}

// Za[r] = V_c,r / Ip[c + P r], G[r] = (Za - z0)/(Za + z0)
__global__ void scan_active_kernel(const double2* __restrict__ Ip, int P, int nscan, int c, int nx, double dx,
                                   double dy, double k, const double* __restrict__ theta,
                                   const double* __restrict__ phi, double z0, double2* __restrict__ Za,
                                   double2* __restrict__ G) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nscan) return;
    const double u = sin(theta[r]) * cos(phi[r]), v = sin(theta[r]) * sin(phi[r]);
    double sn, cs;
    sincos(k * ((c % nx) * dx * u + (c / nx) * dy * v), &sn, &cs);
    const double2 za = cdiv(make_double2(cs, -sn), Ip[(int64_t)c + (int64_t)P * r]);
    Za[r] = za;
    G[r] = cdiv(make_double2(za.x - z0, za.y), make_double2(za.x + z0, za.y));
}

void scan_voltages(const Geom& g, double k, const double* theta, const double* phi, int R, double2* V,
                   hipStream_t s) {
    zero_d(V, g.N * R, s);
    const int64_t n = (int64_t)g.P * R;
    hipLaunchKernelGGL(scan_voltages_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.nx, g.P, g.dx, g.dy,
                       k, theta, phi, R, g.M, g.port, V);
    MBT_LAUNCH_CHECK();
}

void scan_active(const Geom& g, double k, const double2* Ip, int nscan, int c, const double* theta,
                 const double* phi, double z0, double2* Za, double2* G, hipStream_t s) {
    hipLaunchKernelGGL(scan_active_kernel, dim3((nscan + 63) / 64), dim3(64), 0, s, Ip, g.P, nscan, c, g.nx, g.dx,
                       g.dy, k, theta, phi, z0, Za, G);
    MBT_LAUNCH_CHECK();
}

}  // namespace mbt

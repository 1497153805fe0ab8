// Batched restarted GMRES(m): one independent Krylov solve per right-hand side,
// all sharing the batched operator (the paper's "new M1" GMRES with the
// normal-equation strategy, or GMRES with the element-block preconditioner).
//
// The paper uses MATLAB's GMRES and states no details; this solver fixes them:
// x0 = 0; Arnoldi by classical Gram-Schmidt with delayed reorthogonalisation
// (DCGS2, Swirydowicz et al. 2021: the second projection of step k-1 is folded
// into the dot sweep of step k, so each step sweeps the basis twice), or by
// plain CGS2 in three sweeps on request; complex Givens rotations (c real,
// s complex, c = 0 and s = 1 when the pivot is zero); stop as soon as the
// least-squares residual |g_{j+1}| <= tol * ||b||; the explicit residual
// b - A x is recomputed at every restart, and a RHS counts as converged only
// on that explicit residual: <= tol * ||b||, or <= 2 tol * ||b|| after a cycle
// whose least-squares residual met the tolerance (the two residuals differ by
// rounding; a larger gap means the recurrence lost its Arnoldi relation, e.g.
// at a breakdown, and the RHS restarts from the explicit residual).  In DCGS2 a
// step whose reorthogonalised norm nu^2 = ||u||^2 - ||s||^2 has cancelled to
// below 1e-12 ||u||^2 is a breakdown (nu = 0): the cycle ends there.
//
// Vectors are RHS-innermost, v[n][r]: a lane owns one RHS and walks rows, so
// every per-RHS dot product is accumulated in a fixed order that does not
// depend on how many other RHS share the batch (bit-identical results alone or
// batched).  Rows are split into fixed chunks (a function of N only) whose
// partial sums are reduced by a second kernel in a fixed order (groups of 64
// chunks, then the groups).
//
// HBM traffic per Arnoldi step is dominated by the basis reads.  DCGS2 step k
// reads V_{0..k-1}, the candidate u and w = A u once for all dot products
// (s = V^H u, z = V^H w, u^H u, u^H w) and once more for the update that
// writes the normalised v_k and the next candidate.  CGS2 is fused into three
// passes: (1) h = V^H w; (2) w <- w - V h together with h2 = V^H w; (3)
// w <- w - V h2 together with ||w||^2.  In the dot sweeps the waves of a
// workgroup share rows and RHS and split the basis vectors; the DCGS2 update
// gives each wave its own rows and all vectors.
// The reduced-precision inner solves keep the basis packed (FP32 components
// rounded to 24 bits, two RHS per 12-byte word) or in FP32, with FP32 work
// vectors; all dot products, norms and the Hessenberg/Givens recurrences stay
// FP64.  The file also holds the batched PCG on the normal equations (Sec.
// II-C), which reuses the chunked reductions.
#include "common.h"
#include "gmres.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace mbt {

namespace {

constexpr int kMaxVec = 64;            // basis vectors per pass -> restart <= 63

// Accumulations written as explicit fused multiply-adds in a fixed order.  The
// kernels have variants that move one or two RHS per lane; leaving the fusion of
// products and sums to the compiler lets it differ between variants, and a RHS's
// result would then depend on the parity of the batch size.
// acc + a b
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) b
__device__ __forceinline__ double2 cfmac(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// w s - c - k v  (the DCGS2 candidate update)
__device__ __forceinline__ double2 next_candidate(double2 w, double s, double2 c, double2 k, double2 v) {
    double2 t;
    t.x = fma(w.x, s, -c.x);
    t.y = fma(w.y, s, -c.y);
    t.x = fma(-k.x, v.x, t.x);
    t.x = fma(k.y, v.y, t.x);
    t.y = fma(-k.x, v.y, t.y);
    t.y = fma(-k.y, v.x, t.y);
    return t;
}
// acc + |a|^2
__device__ __forceinline__ double nfma(double acc, double2 a) { return fma(a.y, a.y, fma(a.x, a.x, acc)); }

__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2* p) { float2 v = *p; return make_double2(v.x, v.y); }
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// RPL consecutive complex values (RHS columns) per lane, widened to FP64.
// FP32 pairs are moved with one 16-byte access.
template <int RPL> __device__ __forceinline__ void ldp(const double2* p, double2 (&o)[RPL]) {
#pragma unroll
    for (int k = 0; k < RPL; ++k) o[k] = p[k];
}
template <int RPL> __device__ __forceinline__ void ldp(const float2* p, double2 (&o)[RPL]) {
    if constexpr (RPL == 2) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = make_double2(v.x, v.y);
        o[1] = make_double2(v.z, v.w);
    } else {
#pragma unroll
        for (int k = 0; k < RPL; ++k) o[k] = ld2(p + k);
    }
}
template <int RPL> __device__ __forceinline__ void stp(double2* p, const double2 (&v)[RPL]) {
#pragma unroll
    for (int k = 0; k < RPL; ++k) p[k] = v[k];
}
template <int RPL> __device__ __forceinline__ void stp(float2* p, const double2 (&v)[RPL]) {
    if constexpr (RPL == 2) {
        *reinterpret_cast<float4*>(p) = make_float4((float)v[0].x, (float)v[0].y, (float)v[1].x, (float)v[1].y);
    } else {
#pragma unroll
        for (int k = 0; k < RPL; ++k) st2(p + k, v[k]);
    }
}

// Raw (storage-format) pack of RPL adjacent complex values, kept in registers
// between the load of the next row and its use; widened to FP64 at use.
template <typename T, int RPL> struct Raw;
template <> struct Raw<double2, 1> {
    double2 v;
    __device__ __forceinline__ void load(const double2* p) { v = *p; }
    __device__ __forceinline__ void zero() { v = make_double2(0, 0); }
    __device__ __forceinline__ double2 get(int) const { return v; }
};
template <> struct Raw<double2, 2> {
    double2 v[2];
    __device__ __forceinline__ void load(const double2* p) { v[0] = p[0]; v[1] = p[1]; }
    __device__ __forceinline__ void zero() { v[0] = v[1] = make_double2(0, 0); }
    __device__ __forceinline__ double2 get(int k) const { return v[k]; }
};
template <> struct Raw<float2, 1> {
    float2 v;
    __device__ __forceinline__ void load(const float2* p) { v = *p; }
    __device__ __forceinline__ void zero() { v = make_float2(0, 0); }
    __device__ __forceinline__ double2 get(int) const { return make_double2(v.x, v.y); }
};
template <> struct Raw<float2, 2> {
    float4 v;
    __device__ __forceinline__ void load(const float2* p) { v = *reinterpret_cast<const float4*>(p); }
    __device__ __forceinline__ void zero() { v = make_float4(0, 0, 0, 0); }
    __device__ __forceinline__ double2 get(int k) const { return k ? make_double2(v.z, v.w) : make_double2(v.x, v.y); }
};

// ------------------------------------------------------------------ packed 24-bit basis storage
// The mixed path may keep its Krylov basis with the low byte of each FP32
// component rounded away (sign, 8-bit exponent, 15-bit mantissa; unit roundoff
// 2^-16), three quarters of the FP32 bytes.  Two complex values of adjacent RHS
// columns (four components) form one 12-byte word, so a basis vector of N x R
// values (R even) is N x R/2 words.  The work vectors (the candidate and A times
// it) stay FP32.
struct p24x2 {
    uint32_t w[3];
};
template <typename T> struct PerWord { static constexpr int v = 1; };
template <> struct PerWord<p24x2> { static constexpr int v = 2; };
// element offset n*R + r (r even for packed words) -> offset in storage words
template <typename T> __device__ __forceinline__ int64_t vofs(int64_t off) { return off / PerWord<T>::v; }

__device__ __forceinline__ uint32_t to24(double x) {
    const uint32_t u = __float_as_uint((float)x);
    return (u + 0x7Fu + ((u >> 8) & 1u)) >> 8;   // nearest, ties to even, on the dropped byte
}
__device__ __forceinline__ double from24(uint32_t t) { return (double)__uint_as_float(t << 8); }
__device__ __forceinline__ double2 round24(double2 v) { return make_double2(from24(to24(v.x)), from24(to24(v.y))); }

template <> struct Raw<p24x2, 2> {
    uint32_t a, b, c;
    __device__ __forceinline__ void load(const p24x2* p) {
        const uint3 t = *reinterpret_cast<const uint3*>(p);
        a = t.x;
        b = t.y;
        c = t.z;
    }
    __device__ __forceinline__ void zero() { a = b = c = 0; }
    __device__ __forceinline__ double2 get(int k) const {
        if (k == 0) return make_double2(from24(a & 0xFFFFFFu), from24((a >> 24) | ((b & 0xFFFFu) << 8)));
        return make_double2(from24((b >> 16) | ((c & 0xFFu) << 16)), from24(c >> 8));
    }
};
__device__ __forceinline__ void st24(p24x2* p, double2 v0, double2 v1) {
    const uint32_t t0 = to24(v0.x), t1 = to24(v0.y), t2 = to24(v1.x), t3 = to24(v1.y);
    uint3 o;
    o.x = t0 | (t1 << 24);
    o.y = (t1 >> 8) | (t2 << 16);
    o.z = (t2 >> 16) | (t3 << 8);
    *reinterpret_cast<uint3*>(p) = o;
}

// One pass over the basis V_0..V_{nvec-1} (rows of one chunk, 64*RPL RHS columns
// per workgroup).  The NW waves of a workgroup read the same rows and columns
// and split the basis vectors (wave w takes i = w, w+NW, ..., G per wave); a
// lane owns RPL adjacent RHS columns.
// MODE 0: h[i] = sum_n conj(V_i[n]) w[n]                         (partials per chunk)
// MODE 1: w <- w - sum_i coef_i V_i ; h2[i] = sum_n conj(V_i) w   (partials per chunk)
// MODE 2: w <- w - sum_i coef_i V_i ; ||w||^2                      (partials per chunk)
template <typename TB, typename TO, int MODE, int NW, int G, int RPL>
__global__ __launch_bounds__(NW * 64) void arnoldi_kernel(const TB* __restrict__ V, int64_t vstride, int nvec,
                                                          const double2* __restrict__ coef, TO* w, int64_t N, int R,
                                                          int64_t rows_per_chunk, double2* __restrict__ partial) {
    __shared__ double2 xch[2][NW][64 * RPL];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 64 + lane) * RPL;
    const bool live = r0 < R;            // R is a multiple of RPL
    const int64_t chunk = blockIdx.y;
    const int64_t n0 = chunk * rows_per_chunk;
    const int64_t n1 = min(N, n0 + rows_per_chunk);

    double2 acc[G][RPL];
    double2 cf[G][RPL];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int i = wave + NW * g;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            acc[g][k] = make_double2(0, 0);
            cf[g][k] = (MODE != 0 && live && i < nvec) ? coef[(int64_t)i * R + r0 + k] : make_double2(0, 0);
        }
    }
    double nrm[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) nrm[k] = 0.0;
    int buf = 0;
    // rows are software-pipelined: the loads of row n+1 are issued before the
    // arithmetic (and the cross-wave exchange) of row n
    Raw<TB, RPL> cur[G], nxt[G];
    Raw<TO, RPL> cw, nw_raw;
    auto load_row = [&](int64_t n, Raw<TB, RPL>(&v)[G], Raw<TO, RPL>& wr) {
        const int64_t off = n * R + r0;
        wr.load(w + off);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = wave + NW * g;
            if (i < nvec) v[g].load(V + i * vstride + vofs<TB>(off));
            else v[g].zero();
        }
    };
    if (live && n0 < n1) load_row(n0, cur, cw);
    for (int64_t n = n0; n < n1; ++n) {
        const int64_t off = n * R + r0;
        if (live && n + 1 < n1) load_row(n + 1, nxt, nw_raw);
        // values are widened at each use from the raw registers (no widened copies live across the barrier)
        double2 wv[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) wv[k] = cw.get(k);
        if constexpr (MODE == 0) {
            if (live) {
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int k = 0; k < RPL; ++k) acc[g][k] = cfmac(acc[g][k], cur[g].get(k), wv[k]);
            }
        } else {
            double2 u[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) u[k] = make_double2(0, 0);
            if (live) {
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int k = 0; k < RPL; ++k) u[k] = cfma(u[k], cf[g][k], cur[g].get(k));
            }
#pragma unroll
            for (int k = 0; k < RPL; ++k) xch[buf][wave][lane * RPL + k] = u[k];
            __syncthreads();
            double2 nw[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                double2 tot = xch[buf][0][lane * RPL + k];
#pragma unroll
                for (int q = 1; q < NW; ++q) tot = cadd(tot, xch[buf][q][lane * RPL + k]);
                nw[k] = csub(wv[k], tot);
            }
            buf ^= 1;
            if (live) {
                if constexpr (MODE == 1) {
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int k = 0; k < RPL; ++k) acc[g][k] = cfmac(acc[g][k], cur[g].get(k), nw[k]);
                } else if constexpr (MODE == 2) {
#pragma unroll
                    for (int k = 0; k < RPL; ++k) nrm[k] = nfma(nrm[k], nw[k]);
                }
                if (wave == 0) stp<RPL>(w + off, nw);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) cur[g] = nxt[g];
        cw = nw_raw;
    }
    if (!live) return;
    if constexpr (MODE == 0 || MODE == 1) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = wave + NW * g;
            if (i < nvec)
#pragma unroll
                for (int k = 0; k < RPL; ++k) partial[(chunk * nvec + i) * R + r0 + k] = acc[g][k];
        }
    } else if constexpr (MODE == 2) {
        if (wave == 0)
#pragma unroll
            for (int k = 0; k < RPL; ++k) partial[chunk * R + r0 + k] = make_double2(nrm[k], 0.0);
    }
}

// ------------------------------------------------------------------ delayed reorthogonalisation (DCGS2)
constexpr int kDotRows = 16;   // rows of u and w staged in LDS per step of the dot sweep

// Dot sweep: with u the candidate (slot k) and w = A u (slot k+1),
//   s_i = V_i^H u, z_i = V_i^H w (i < k), alpha = u^H u, beta = u^H w.
// Partials per chunk: [s_0..s_{k-1}, z_0..z_{k-1}, alpha, beta].  One launch
// covers the vectors i0 .. i0+nv-1 (the sweep may be split into launches of at
// most NW*G vectors); alpha and beta come from the launch with i0 = 0.
template <typename TB, typename TV, int NW, int G, int RPL, bool HASW>
__global__ __launch_bounds__(NW * 64, (std::is_same<TV, p24x2>::value && G <= 4 ? 4 : 1)) void dcgs2_dots_kernel(const TV* __restrict__ V, int64_t vstride, int k,
                                                             int i0, int nv, const TB* __restrict__ u,
                                                             const TB* __restrict__ w, int64_t N, int R,
                                                             int64_t rows_per_chunk, double2* __restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 64 + lane) * RPL;
    const bool live = r0 < R;
    const int64_t chunk = blockIdx.y;
    const int64_t n0 = chunk * rows_per_chunk;
    const int64_t n1 = min(N, n0 + rows_per_chunk);
    const int nred = 2 * k + 2;
    double2 as[G][RPL], az[G][RPL], aa[RPL], ab[RPL];
#pragma unroll
    for (int k2 = 0; k2 < RPL; ++k2) {
        aa[k2] = ab[k2] = make_double2(0, 0);
#pragma unroll
        for (int g = 0; g < G; ++g) as[g][k2] = az[g][k2] = make_double2(0, 0);
    }
    // Every wave of the workgroup needs the same rows of u and w: they are staged
    // in LDS kDotRows rows at a time by all threads, so each value is read from
    // memory once per workgroup (waves reading them independently drift apart
    // over the chunk and re-fetch lines that the basis stream has evicted).
    __shared__ Raw<TB, RPL> su[kDotRows][64];
    __shared__ Raw<TB, RPL> sw[HASW ? kDotRows : 1][64];
    const bool ab_here = (i0 == 0) && (wave == 0);
    for (int64_t nb = n0; nb < n1; nb += kDotRows) {
        const int nrow = (int)min((int64_t)kDotRows, n1 - nb);
        for (int i = threadIdx.x; i < kDotRows * 64; i += NW * 64) {
            const int rr = i >> 6, l = i & 63;
            const int c = (blockIdx.x * 64 + l) * RPL;
            if (rr < nrow && c < R) {
                su[rr][l].load(u + (nb + rr) * R + c);
                if (HASW) sw[rr][l].load(w + (nb + rr) * R + c);
            } else {
                su[rr][l].zero();
                if (HASW) sw[rr][l].zero();
            }
        }
        __syncthreads();
        if (live) {
            // the packed basis (up to four vectors per wave) runs four waves per SIMD and loads each
            // row when it is used; the other cases prefetch the next row of the block
            constexpr bool kPrefetch = !(std::is_same<TV, p24x2>::value && G <= 4);
            Raw<TV, RPL> cur[G], nxt[G];
            auto load_row = [&](int rr, Raw<TV, RPL>(&v)[G]) {
                const int64_t off = (nb + rr) * R + r0;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int j = wave + NW * g;
                    if (j < nv) v[g].load(V + (int64_t)(i0 + j) * vstride + vofs<TV>(off));
                    else v[g].zero();
                }
            };
            if (kPrefetch) load_row(0, cur);
            for (int rr = 0; rr < nrow; ++rr) {
                if (!kPrefetch) load_row(rr, cur);
                else if (rr + 1 < nrow) load_row(rr + 1, nxt);
#pragma unroll
                for (int k2 = 0; k2 < RPL; ++k2) {
                    const double2 uv = su[rr][lane].get(k2);
                    const double2 wv = HASW ? sw[rr][lane].get(k2) : make_double2(0, 0);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const double2 vv = cur[g].get(k2);
                        as[g][k2] = cfmac(as[g][k2], vv, uv);
                        if (HASW) az[g][k2] = cfmac(az[g][k2], vv, wv);
                    }
                    if (ab_here) {
                        aa[k2].x = nfma(aa[k2].x, uv);
                        if (HASW) ab[k2] = cfmac(ab[k2], uv, wv);
                    }
                }
                if (kPrefetch) {
#pragma unroll
                    for (int g = 0; g < G; ++g) cur[g] = nxt[g];
                }
            }
        }
        __syncthreads();
    }
    if (!live) return;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int j = wave + NW * g;
        if (j < nv)
#pragma unroll
            for (int k2 = 0; k2 < RPL; ++k2) {
                partial[(chunk * nred + i0 + j) * R + r0 + k2] = as[g][k2];
                partial[(chunk * nred + k + i0 + j) * R + r0 + k2] = az[g][k2];
            }
    }
    if (ab_here)
#pragma unroll
        for (int k2 = 0; k2 < RPL; ++k2) {
            partial[(chunk * nred + 2 * k) * R + r0 + k2] = aa[k2];
            partial[(chunk * nred + 2 * k + 1) * R + r0 + k2] = ab[k2];
        }
}

// Per-RHS bookkeeping of DCGS2 step k (red: reduced [s, z, alpha, beta]):
// completes Hessenberg column k-1 (raw and rotated), Givens, convergence.
// inv_nu[r] = 1/nu for a RHS that takes another step, 0 for one that stops.
__global__ void dcgs2_finalize_kernel(GmresState st, double2* __restrict__ Hraw, const double2* __restrict__ red,
                                      int R, int k, int m, double* __restrict__ inv_nu) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t ldH = (int64_t)(m + 1) * R;
    auto RED = [&](int i) { return red[(int64_t)i * R + r]; };
    if (!st.active[r]) {
        inv_nu[r] = 0.0;
        return;
    }
    double ss = 0;
    for (int i = 0; i < k; ++i) {
        const double2 s = RED(i);
        ss += s.x * s.x + s.y * s.y;
    }
    const double alpha = RED(2 * k).x;
    // nu^2 by Pythagoras loses its relative accuracy as ss -> alpha: below
    // 1e-12 alpha the candidate lies in the span of the basis (breakdown)
    const double nu = (alpha - ss > 1e-12 * alpha) ? sqrt(alpha - ss) : 0.0;
    bool stop = false;
    if (k == 0) {
        st.g[r] = make_double2(st.beta[r] * nu, 0.0);
    } else {
        double2* Hc = Hraw + (int64_t)(k - 1) * ldH;
        double2* Hj = st.H + (int64_t)(k - 1) * ldH;
        for (int i = 0; i < k; ++i) Hc[(int64_t)i * R + r] = cadd(Hc[(int64_t)i * R + r], RED(i));
        Hc[(int64_t)k * R + r] = make_double2(nu, 0.0);
        for (int i = 0; i <= k; ++i) Hj[(int64_t)i * R + r] = Hc[(int64_t)i * R + r];
        const int j = k - 1;
        for (int i = 0; i < j; ++i) {
            const double c = st.cs[(int64_t)i * R + r];
            const double2 s = st.sn[(int64_t)i * R + r];
            const double2 a = Hj[(int64_t)i * R + r], b = Hj[(int64_t)(i + 1) * R + r];
            Hj[(int64_t)i * R + r] = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
            Hj[(int64_t)(i + 1) * R + r] = csub(make_double2(c * b.x, c * b.y), cmulc(s, a));
        }
        const double2 h1v = Hj[(int64_t)j * R + r];
        double c;
        double2 s;
        const double a1 = hypot(h1v.x, h1v.y);
        if (a1 == 0.0) {
            c = 0.0;
            s = make_double2(1.0, 0.0);
        } else {
            const double t = hypot(a1, nu);
            c = a1 / t;
            s = make_double2(h1v.x / a1 * nu / t, h1v.y / a1 * nu / t);
        }
        st.cs[(int64_t)j * R + r] = c;
        st.sn[(int64_t)j * R + r] = s;
        Hj[(int64_t)j * R + r] = cadd(make_double2(c * h1v.x, c * h1v.y), make_double2(s.x * nu, s.y * nu));
        Hj[(int64_t)(j + 1) * R + r] = make_double2(0, 0);
        const double2 gj = st.g[(int64_t)j * R + r];
        const double2 gn = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
        st.g[(int64_t)j * R + r] = make_double2(c * gj.x, c * gj.y);
        st.g[(int64_t)(j + 1) * R + r] = gn;
        st.iters[r] += 1;
        st.kcyc[r] = k;
        const double res = hypot(gn.x, gn.y);
        if (!(nu == nu) || isinf(nu) || !(res == res)) {
            st.flag[r] = 1;
            stop = true;
        } else if (res <= st.tol * st.bnorm[r] || nu == 0.0 || k == m) {
            stop = true;
        }
    }
    if (stop || k == m || nu == 0.0) {
        st.active[r] = 0;
        inv_nu[r] = 0.0;
        return;
    }
    inv_nu[r] = 1.0 / nu;
}

// Coefficients of the DCGS2 update sweep of step k, one thread per (row i, RHS r):
// t = Hbar_{k-1} s (rows 0..k), h = projections of A v_k (raw column k of H),
// c = t/nu + h; the coefficients of a RHS that stops are zero.
__global__ void dcgs2_coef_kernel(double2* __restrict__ Hraw, const double2* __restrict__ red, int R, int k, int m,
                                  const double* __restrict__ inv_nu, double2* __restrict__ cs_out,
                                  double2* __restrict__ cc_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (r >= R) return;
    const double in = inv_nu[r];
    if (in == 0.0) {
        if (i < k) cs_out[(int64_t)i * R + r] = make_double2(0, 0);
        cc_out[(int64_t)i * R + r] = make_double2(0, 0);
        return;
    }
    const int64_t ldH = (int64_t)(m + 1) * R;
    auto RED = [&](int j) { return red[(int64_t)j * R + r]; };
    double2 t = make_double2(0, 0);
    for (int l = (i > 0 ? i - 1 : 0); l < k; ++l)   // Hbar is upper Hessenberg: H[i][l] = 0 for l < i-1
        t = cadd(t, cmul(Hraw[(int64_t)l * ldH + (int64_t)i * R + r], RED(l)));
    double2 h;
    if (i < k) {
        const double2 d = csub(RED(k + i), t);
        h = make_double2(d.x * in, d.y * in);
        cs_out[(int64_t)i * R + r] = RED(i);
    } else {
        double2 sz = make_double2(0, 0);
        for (int l = 0; l < k; ++l) sz = cadd(sz, cmulc(RED(l), RED(k + l)));
        const double2 q = csub(RED(2 * k + 1), sz);
        h = make_double2((q.x * in - t.x) * in, (q.y * in - t.y) * in);
    }
    Hraw[(int64_t)k * ldH + (int64_t)i * R + r] = h;
    cc_out[(int64_t)i * R + r] = make_double2(t.x * in + h.x, t.y * in + h.y);
}

template <typename TB, typename TV, int RPL, bool HASW>
void launch_dcgs2_dots_rpl(const TV* V, int64_t vs, int k, int i0, int nv, const TB* u, const TB* w, int64_t N, int R,
                           int64_t rpc, int nchunk, double2* partial, hipStream_t s) {
    const dim3 grid((unsigned)((R / RPL + 63) / 64), (unsigned)nchunk);
    if (nv <= 4)
        hipLaunchKernelGGL((dcgs2_dots_kernel<TB, TV, 4, 1, RPL, HASW>), grid, dim3(256), 0, s, V, vs, k, i0, nv, u, w, N, R,
                           rpc, partial);
    else if (nv <= 8)
        hipLaunchKernelGGL((dcgs2_dots_kernel<TB, TV, 4, 2, RPL, HASW>), grid, dim3(256), 0, s, V, vs, k, i0, nv, u, w, N, R,
                           rpc, partial);
    else if (nv <= 16)
        hipLaunchKernelGGL((dcgs2_dots_kernel<TB, TV, 4, 4, RPL, HASW>), grid, dim3(256), 0, s, V, vs, k, i0, nv, u, w, N, R,
                           rpc, partial);
    else if (nv <= 32)
        hipLaunchKernelGGL((dcgs2_dots_kernel<TB, TV, 8, 4, RPL, HASW>), grid, dim3(512), 0, s, V, vs, k, i0, nv, u, w, N, R,
                           rpc, partial);
    else
        hipLaunchKernelGGL((dcgs2_dots_kernel<TB, TV, 8, 8, RPL, HASW>), grid, dim3(512), 0, s, V, vs, k, i0, nv, u, w, N, R,
                           rpc, partial);
    MBT_LAUNCH_CHECK();
}

// Row-split update sweep: each wave owns RB consecutive rows of 64 RHS columns
// and walks all k basis vectors itself, so there is no cross-wave reduction and
// no workgroup barrier; the per-RHS coefficients are re-read (from L2) for each
// block of rows.  The next vector's rows are loaded while the current ones are
// accumulated.  Summation over i is sequential per (row, RHS).
template <typename TB, int RB>
__global__ __launch_bounds__(256) void dcgs2_update_rows_kernel(const TB* __restrict__ V, int64_t vstride, int k,
                                                                TB* u, TB* w, const double2* __restrict__ cs_,
                                                                const double2* __restrict__ cc_,
                                                                const double* __restrict__ inv_nu_, int64_t N, int R,
                                                                int Rt) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    const int64_t n0 = ((int64_t)blockIdx.y * 4 + wave) * RB;
    if (r >= R || n0 >= N) return;
    // folded rows (R = F * Rt columns per row): column r is RHS r mod Rt
    const int rt = r % Rt;
    const double2* cs = cs_ + rt;
    const double2* cc = cc_ + rt;
    const double* inv_nu = inv_nu_ + rt;
    const int nr = (int)min<int64_t>(RB, N - n0);
    double2 a[RB], c[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) a[j] = c[j] = make_double2(0, 0);
    const TB* base = V + n0 * R + r;
    Raw<TB, 1> cur[RB], nxt[RB];
    auto load = [&](int i, Raw<TB, 1>(&v)[RB]) {
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            if (j < nr) v[j].load(base + i * vstride + (int64_t)j * R);
            else v[j].zero();
        }
    };
    double2 fs = make_double2(0, 0), fc = make_double2(0, 0);
    if (k > 0) {
        load(0, cur);
        fs = cs[0];
        fc = cc[0];
    }
    for (int i = 0; i < k; ++i) {
        double2 fs_n = make_double2(0, 0), fc_n = make_double2(0, 0);
        if (i + 1 < k) {
            load(i + 1, nxt);
            fs_n = cs[(int64_t)(i + 1) * Rt];
            fc_n = cc[(int64_t)(i + 1) * Rt];
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const double2 vv = cur[j].get(0);
            a[j] = cfma(a[j], fs, vv);
            c[j] = cfma(c[j], fc, vv);
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) cur[j] = nxt[j];
        fs = fs_n;
        fc = fc_n;
    }
    const double inu = inv_nu[0];
    const double2 ckv = cc[(int64_t)k * Rt];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        if (j < nr) {
            const int64_t off = (n0 + j) * R + r;
            const double2 d = csub(ld2(u + off), a[j]);
            const double2 vk = make_double2(d.x * inu, d.y * inu);
            const double2 wv = ld2(w + off);
            const double2 un = next_candidate(wv, inu, c[j], ckv, vk);
            st2(u + off, vk);
            st2(w + off, un);
        }
    }
}

// Row-split update sweep into the packed basis: as dcgs2_update_rows_kernel,
// with a lane owning two adjacent RHS columns (one packed word per row).  v_k
// goes to its own slot vk (rounded to the packed format, and the rounded value
// is the one removed from u_{k+1}); u_{k+1} overwrites u.
template <int RB>
__global__ __launch_bounds__(256) void dcgs2_update_rows24_kernel(const p24x2* __restrict__ V, int64_t vstride, int k,
                                                                  float2* u, const float2* __restrict__ w,
                                                                  p24x2* __restrict__ vk, const double2* __restrict__ cs_,
                                                                  const double2* __restrict__ cc_,
                                                                  const double* __restrict__ inv_nu_, int64_t N, int R,
                                                                  int Rt) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r0 = 2 * (blockIdx.x * 64 + lane);
    const int64_t n0 = ((int64_t)blockIdx.y * 4 + wave) * RB;
    if (r0 >= R || n0 >= N) return;
    // folded rows (R = F * Rt columns per row, Rt even): columns r0, r0+1 are RHS r0 mod Rt and the next
    const int rt = r0 % Rt;
    const double2* cs = cs_ + rt;
    const double2* cc = cc_ + rt;
    const double* inv_nu = inv_nu_ + rt;
    const int nr = (int)min<int64_t>(RB, N - n0);
    const int64_t rw = R / 2;   // packed words per row
    double2 a[RB][2], c[RB][2];
#pragma unroll
    for (int j = 0; j < RB; ++j)
#pragma unroll
        for (int q = 0; q < 2; ++q) a[j][q] = c[j][q] = make_double2(0, 0);
    const p24x2* base = V + (n0 * R + r0) / 2;
    Raw<p24x2, 2> cur[RB], nxt[RB];
    auto load = [&](int i, Raw<p24x2, 2>(&v)[RB]) {
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            if (j < nr) v[j].load(base + i * vstride + (int64_t)j * rw);
            else v[j].zero();
        }
    };
    double2 fs[2] = {make_double2(0, 0), make_double2(0, 0)}, fc[2] = {make_double2(0, 0), make_double2(0, 0)};
    if (k > 0) {
        load(0, cur);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            fs[q] = cs[q];
            fc[q] = cc[q];
        }
    }
    for (int i = 0; i < k; ++i) {
        double2 fs_n[2] = {make_double2(0, 0), make_double2(0, 0)}, fc_n[2] = {make_double2(0, 0), make_double2(0, 0)};
        if (i + 1 < k) {
            load(i + 1, nxt);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                fs_n[q] = cs[(int64_t)(i + 1) * Rt + q];
                fc_n[q] = cc[(int64_t)(i + 1) * Rt + q];
            }
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double2 vv = cur[j].get(q);
                a[j][q] = cfma(a[j][q], fs[q], vv);
                c[j][q] = cfma(c[j][q], fc[q], vv);
            }
#pragma unroll
        for (int j = 0; j < RB; ++j) cur[j] = nxt[j];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            fs[q] = fs_n[q];
            fc[q] = fc_n[q];
        }
    }
    double inu[2];
    double2 ckv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        inu[q] = inv_nu[q];
        ckv[q] = cc[(int64_t)k * Rt + q];
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        if (j < nr) {
            const int64_t off = (n0 + j) * R + r0;
            double2 uv[2], wv[2], v[2], un[2];
            ldp<2>(u + off, uv);
            ldp<2>(w + off, wv);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double2 d = csub(uv[q], a[j][q]);
                v[q] = round24(make_double2(d.x * inu[q], d.y * inu[q]));
                un[q] = next_candidate(wv[q], inu[q], c[j][q], ckv[q], v[q]);
            }
            st24(vk + off / 2, v[0], v[1]);
            stp<2>(u + off, un);
        }
    }
}

void launch_dcgs2_update24(const p24x2* V, int64_t vs, int k, float2* u, const float2* w, p24x2* vk,
                           const double2* cs, const double2* cc, const double* inv_nu, int64_t N, int R, int Rt,
                           hipStream_t s) {
    constexpr int RB = 8;
    MBT_REQUIRE(R % 2 == 0, "packed basis needs an even number of RHS");
    const int64_t rows_per_block = 4 * RB;
    const int64_t gy = (N + rows_per_block - 1) / rows_per_block;
    MBT_REQUIRE(gy < 65536, "dcgs2 update: too many row blocks");
    MBT_REQUIRE(Rt % 2 == 0 && R % Rt == 0, "packed basis: folded width must be a multiple of the even RHS count");
    hipLaunchKernelGGL((dcgs2_update_rows24_kernel<RB>), dim3((unsigned)((R / 2 + 63) / 64), (unsigned)gy), dim3(256), 0,
                       s, V, vs, k, u, w, vk, cs, cc, inv_nu, N, R, Rt);
    MBT_LAUNCH_CHECK();
}

// End of a cycle: x += sum_{i < steps} y_i V_i.  Each wave owns RB rows of 64
// lanes (RPL adjacent RHS per lane) and walks the vectors in order, so a
// RHS's sum has the same order whatever the batch and however long the cycle
// of the other RHS ran.
template <typename TV, int RPL, int RB>
__global__ __launch_bounds__(256) void solution_update_kernel(const TV* __restrict__ V, int64_t vstride, int steps,
                                                              const double2* __restrict__ y_, double2* __restrict__ x,
                                                              int64_t N, int R, int Rt) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 64 + lane) * RPL;
    const int64_t n0 = ((int64_t)blockIdx.y * 4 + wave) * RB;
    if (r0 >= R || n0 >= N) return;
    const double2* y = y_ + r0 % Rt;   // folded rows: column r0 is RHS r0 mod Rt
    const int nr = (int)min<int64_t>(RB, N - n0);
    double2 acc[RB][RPL];
#pragma unroll
    for (int j = 0; j < RB; ++j)
#pragma unroll
        for (int q = 0; q < RPL; ++q) acc[j][q] = make_double2(0, 0);
    Raw<TV, RPL> cur[RB], nxt[RB];
    auto load = [&](int i, Raw<TV, RPL>(&v)[RB]) {
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            if (j < nr) v[j].load(V + i * vstride + vofs<TV>((n0 + j) * R + r0));
            else v[j].zero();
        }
    };
    double2 yc[RPL];
    if (steps > 0) {
        load(0, cur);
#pragma unroll
        for (int q = 0; q < RPL; ++q) yc[q] = y[q];
    }
    for (int i = 0; i < steps; ++i) {
        double2 yn[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) yn[q] = make_double2(0, 0);
        if (i + 1 < steps) {
            load(i + 1, nxt);
#pragma unroll
            for (int q = 0; q < RPL; ++q) yn[q] = y[(int64_t)(i + 1) * Rt + q];
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
            for (int q = 0; q < RPL; ++q) acc[j][q] = cfma(acc[j][q], yc[q], cur[j].get(q));
#pragma unroll
        for (int j = 0; j < RB; ++j) cur[j] = nxt[j];
#pragma unroll
        for (int q = 0; q < RPL; ++q) yc[q] = yn[q];
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        if (j < nr) {
            const int64_t off = (n0 + j) * R + r0;
#pragma unroll
            for (int q = 0; q < RPL; ++q) x[off + q] = cadd(x[off + q], acc[j][q]);
        }
    }
}

template <typename TV>
void launch_solution_update(const TV* V, int64_t vs, int steps, const double2* y, double2* x, int64_t N, int R,
                            int Rt, hipStream_t s) {
    MBT_REQUIRE(R % Rt == 0, "folded width must be a multiple of the RHS count");
    constexpr int RB = 8;
    const int64_t gy = (N + 4 * RB - 1) / (4 * RB);
    MBT_REQUIRE(gy < 65536, "solution update: too many row blocks");
    if constexpr (std::is_same<TV, p24x2>::value) {
        MBT_REQUIRE(R % 2 == 0, "packed basis needs an even number of RHS");
        hipLaunchKernelGGL((solution_update_kernel<TV, 2, RB>), dim3((unsigned)((R / 2 + 63) / 64), (unsigned)gy),
                           dim3(256), 0, s, V, vs, steps, y, x, N, R, Rt);
    } else {
        hipLaunchKernelGGL((solution_update_kernel<TV, 1, RB>), dim3((unsigned)((R + 63) / 64), (unsigned)gy),
                           dim3(256), 0, s, V, vs, steps, y, x, N, R, Rt);
    }
    MBT_LAUNCH_CHECK();
}

template <typename TB, typename TV>
void launch_dcgs2_dots(const TV* V, int64_t vs, int k, const TB* u, const TB* w, int64_t N, int R, int64_t rpc,
                       int nchunk, double2* partial, hipStream_t s) {
    if constexpr (sizeof(TB) == 8) {
        if (R % 2 == 0) {
            // FP32 pairs of RHS per lane (16-byte accesses) fit the register budget up to 32
            // vectors per launch: longer sweeps are split, re-reading u and w once more
            for (int i0 = 0; i0 == 0 || i0 < k; i0 += 32) {
                const int nv = std::min(32, k - i0);
                if (w) launch_dcgs2_dots_rpl<TB, TV, 2, true>(V, vs, k, i0, nv, u, w, N, R, rpc, nchunk, partial, s);
                else launch_dcgs2_dots_rpl<TB, TV, 2, false>(V, vs, k, i0, nv, u, w, N, R, rpc, nchunk, partial, s);
            }
            return;
        }
    }
    if constexpr (std::is_same<TV, TB>::value) {
        if (w) launch_dcgs2_dots_rpl<TB, TV, 1, true>(V, vs, k, 0, k, u, w, N, R, rpc, nchunk, partial, s);
        else launch_dcgs2_dots_rpl<TB, TV, 1, false>(V, vs, k, 0, k, u, w, N, R, rpc, nchunk, partial, s);
    } else {
        throw Error(-1, "packed basis needs an even number of RHS");
    }
}

template <typename TB>
void launch_dcgs2_update(const TB* V, int64_t vs, int k, TB* u, TB* w, const double2* cs, const double2* cc,
                         const double* inv_nu, int64_t N, int R, int Rt, hipStream_t s) {
    MBT_REQUIRE(R % Rt == 0, "folded width must be a multiple of the RHS count");
    constexpr int RB = 8;
    const int64_t rows_per_block = 4 * RB;
    const int64_t gy = (N + rows_per_block - 1) / rows_per_block;
    MBT_REQUIRE(gy < 65536, "dcgs2 update: too many row blocks");
    hipLaunchKernelGGL((dcgs2_update_rows_kernel<TB, RB>), dim3((unsigned)((R + 63) / 64), (unsigned)gy), dim3(256), 0,
                       s, V, vs, k, u, w, cs, cc, inv_nu, N, R, Rt);
    MBT_LAUNCH_CHECK();
}

template <typename TB, typename TO, int MODE, int RPL>
void launch_pass_rpl(const TB* V, int64_t vs, int nvec, const double2* coef, TO* w, int64_t N, int R, int64_t rpc,
                     int nchunk, double2* partial, hipStream_t s, int cfg_n) {
    const dim3 grid((unsigned)((R / RPL + 63) / 64), (unsigned)nchunk);
    if (cfg_n <= 4)
        hipLaunchKernelGGL((arnoldi_kernel<TB, TO, MODE, 4, 1, RPL>), grid, dim3(256), 0, s, V, vs, nvec, coef, w, N, R, rpc, partial);
    else if (cfg_n <= 8)
        hipLaunchKernelGGL((arnoldi_kernel<TB, TO, MODE, 4, 2, RPL>), grid, dim3(256), 0, s, V, vs, nvec, coef, w, N, R, rpc, partial);
    else if (cfg_n <= 16)
        hipLaunchKernelGGL((arnoldi_kernel<TB, TO, MODE, 4, 4, RPL>), grid, dim3(256), 0, s, V, vs, nvec, coef, w, N, R, rpc, partial);
    else if (cfg_n <= 32)
        hipLaunchKernelGGL((arnoldi_kernel<TB, TO, MODE, 8, 4, RPL>), grid, dim3(512), 0, s, V, vs, nvec, coef, w, N, R, rpc, partial);
    else
        hipLaunchKernelGGL((arnoldi_kernel<TB, TO, MODE, 8, 8, RPL>), grid, dim3(512), 0, s, V, vs, nvec, coef, w, N, R, rpc, partial);
    MBT_LAUNCH_CHECK();
}

// FP32 bases with an even number of columns move two RHS per 16-byte access.
// The kernel configuration follows nvec (the classical CGS2 sweeps).
template <typename TB, typename TO, int MODE>
void launch_pass(const TB* V, int64_t vs, int nvec, const double2* coef, TO* w, int64_t N, int R, int64_t rpc,
                 int nchunk, double2* partial, hipStream_t s) {
    const int cfg_n = nvec;
    if constexpr (sizeof(TB) == 8) {
        // the update-and-dot pass over more than 32 vectors keeps one RHS per lane (register budget)
        if (R % 2 == 0 && !(MODE == 1 && cfg_n > 32)) {
            launch_pass_rpl<TB, TO, MODE, 2>(V, vs, nvec, coef, w, N, R, rpc, nchunk, partial, s, cfg_n);
            return;
        }
    }
    launch_pass_rpl<TB, TO, MODE, 1>(V, vs, nvec, coef, w, N, R, rpc, nchunk, partial, s, cfg_n);
}

// out[i][r] = sum over chunks of partial[chunk][i][r], in chunk order
// out[t] = sum over chunks c of partial[c][t], t < nvec*R, in an order fixed by
// nchunk alone: groups of kRedGroup consecutive chunks are summed in chunk
// order, then the group sums in group order.  A workgroup owns 64 outputs and
// its waves share the groups, so a short batch still spreads its (up to 2048)
// chunks over many loads in flight.
constexpr int kRedGroup = 64;
constexpr int kRedWaves = 8;
constexpr int kMaxChunks = 2048;
__global__ __launch_bounds__(64 * kRedWaves) void reduce_partials_kernel(const double2* __restrict__ partial,
                                                                         int nchunk, int nvec, int R,
                                                                         double2* __restrict__ out) {
    __shared__ double2 gs[kMaxChunks / kRedGroup][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t nout = (int64_t)nvec * R;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const int ng = (nchunk + kRedGroup - 1) / kRedGroup;
    for (int g = wave; g < ng; g += kRedWaves) {
        double2 sg = make_double2(0, 0);
        if (t < nout) {
            const int c1 = min(nchunk, (g + 1) * kRedGroup);
            for (int c = g * kRedGroup; c < c1; ++c) sg = cadd(sg, partial[(int64_t)c * nout + t]);
        }
        gs[g][lane] = sg;
    }
    __syncthreads();
    if (wave == 0 && t < nout) {
        double2 sum = gs[0][lane];
        for (int g = 1; g < ng; ++g) sum = cadd(sum, gs[g][lane]);
        out[t] = sum;
    }
}

void launch_reduce_partials(const double2* partial, int nchunk, int nvec, int R, double2* out, hipStream_t s) {
    MBT_REQUIRE(nchunk >= 1 && nchunk <= kMaxChunks, "reduction: too many chunks");
    const int64_t nout = (int64_t)nvec * R;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((nout + 63) / 64)), dim3(64 * kRedWaves), 0, s, partial,
                       nchunk, nvec, R, out);
    MBT_LAUNCH_CHECK();
}

// out[i][r] = sum_{f < F} in[i][f * R + r] in order of f (partials of folded rows)
__global__ void unfold_kernel(const double2* __restrict__ in, int nvec, int R, int F, double2* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)nvec * R) return;
    const int64_t i = t / R;
    const int r = (int)(t % R);
    double2 acc = in[i * R * F + r];
    for (int f = 1; f < F; ++f) acc = cadd(acc, in[i * R * F + (int64_t)f * R + r]);
    out[t] = acc;
}

template <typename TB>
__global__ void colnorm2_kernel(const TB* __restrict__ X, int64_t N, int R, int64_t rows_per_chunk,
                                double2* __restrict__ partial) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (r >= R) return;
    const int64_t n0 = chunk * rows_per_chunk, n1 = min(N, n0 + rows_per_chunk);
    double s = 0;
    for (int64_t n = n0; n < n1; ++n) {
        const double2 v = ld2(X + n * R + r);
        s = nfma(s, v);
    }
    partial[chunk * R + r] = make_double2(s, 0.0);
}

__device__ __forceinline__ double sum_norm_partials(const double2* partial, int nchunk, int R, int r) {
    double s = 0;
    for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)c * R + r].x;
    return sqrt(s);
}

// Start of a restart cycle: beta = ||r|| (nrm2: the reduced squared norms);
// decide convergence at restart.
__global__ void cycle_init_kernel(GmresState st, const double2* __restrict__ nrm2, int R, int first) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double beta = sqrt(nrm2[r].x);
    if (first) {
        st.bnorm[r] = beta;
        st.conv[r] = (beta == 0.0) ? 1 : 0;
        st.cand[r] = 0;
        st.iters[r] = 0;
        st.flag[r] = 0;
    }
    st.beta[r] = beta;
    st.kcyc[r] = 0;
    int act = 0;
    if (!st.conv[r] && !st.flag[r]) {
        if (!(beta == beta) || isinf(beta)) {
            st.flag[r] = 1;
        } else if (beta <= st.tol * st.bnorm[r] || (st.cand[r] && beta <= 2.0 * st.tol * st.bnorm[r])) {
            st.conv[r] = 1;
        } else {
            act = 1;
        }
    }
    st.cand[r] = 0;
    st.active[r] = act;
    st.scale[r] = act ? 1.0 / beta : 0.0;
    st.g[r] = make_double2(act ? beta : 0.0, 0.0);
}

// Arnoldi step j bookkeeping: Hessenberg column, Givens rotations, residual
// estimate, per-RHS stop decision and the normalisation factor of v_{j+1}.
__global__ void finalize_kernel(GmresState st, const double2* __restrict__ h1, const double2* __restrict__ h2,
                                const double2* __restrict__ npart, int nchunk, int R, int j, int m) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    if (!st.active[r]) {
        st.scale[r] = 0.0;
        return;
    }
    const double hn = sum_norm_partials(npart, nchunk, R, r);
    const int64_t ldH = (int64_t)(m + 1) * R;   // H[j][i][r]: column j, row i
    double2* Hj = st.H + (int64_t)j * ldH;
    for (int i = 0; i <= j; ++i) Hj[(int64_t)i * R + r] = cadd(h1[(int64_t)i * R + r], h2[(int64_t)i * R + r]);
    // previous rotations
    for (int i = 0; i < j; ++i) {
        const double c = st.cs[(int64_t)i * R + r];
        const double2 s = st.sn[(int64_t)i * R + r];
        const double2 a = Hj[(int64_t)i * R + r], b = Hj[(int64_t)(i + 1) * R + r];
        Hj[(int64_t)i * R + r] = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
        Hj[(int64_t)(i + 1) * R + r] = csub(make_double2(c * b.x, c * b.y), cmulc(s, a));
    }
    const double2 h1v = Hj[(int64_t)j * R + r];
    double c;
    double2 s;
    const double a1 = hypot(h1v.x, h1v.y);
    if (a1 == 0.0) {
        c = 0.0;
        s = make_double2(1.0, 0.0);
    } else {
        const double t = hypot(a1, hn);
        c = a1 / t;
        // s = (h1/|h1|) * conj(hn) / t, hn real
        s = make_double2(h1v.x / a1 * hn / t, h1v.y / a1 * hn / t);
    }
    st.cs[(int64_t)j * R + r] = c;
    st.sn[(int64_t)j * R + r] = s;
    Hj[(int64_t)j * R + r] = cadd(make_double2(c * h1v.x, c * h1v.y), make_double2(s.x * hn, s.y * hn));
    Hj[(int64_t)(j + 1) * R + r] = make_double2(0, 0);
    const double2 gj = st.g[(int64_t)j * R + r];
    const double2 gn = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));  // -conj(s) g_j
    st.g[(int64_t)j * R + r] = make_double2(c * gj.x, c * gj.y);
    st.g[(int64_t)(j + 1) * R + r] = gn;
    st.iters[r] += 1;
    st.kcyc[r] = j + 1;
    const double res = hypot(gn.x, gn.y);
    const bool bad = !(hn == hn) || isinf(hn) || !(res == res);
    if (bad) {
        st.flag[r] = 1;
        st.active[r] = 0;
        st.scale[r] = 0.0;
        return;
    }
    if (res <= st.tol * st.bnorm[r] || hn == 0.0 || j == m - 1) {
        st.active[r] = 0;
        st.scale[r] = 0.0;
    } else {
        st.scale[r] = 1.0 / hn;
    }
}

template <typename TB>
__global__ void scale_cols_kernel(TB* __restrict__ v, const double* __restrict__ scale, int64_t N, int R) {
    const int64_t total = N * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const double sc = scale[t % R];
        const double2 x = ld2(v + t);
        st2(v + t, make_double2(x.x * sc, x.y * sc));
    }
}

// End of cycle: y = R_k^{-1} g_k per RHS (k = steps done this cycle); |g_k|
// meeting the tolerance makes the RHS a candidate, which the explicit residual
// of the next restart confirms.
__global__ void cycle_solve_kernel(GmresState st, int R, int m, double2* __restrict__ y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int k = st.kcyc[r];
    const int64_t ldH = (int64_t)(m + 1) * R;
    for (int i = 0; i < m; ++i) y[(int64_t)i * R + r] = make_double2(0, 0);
    if (k == 0 || st.flag[r]) return;
    for (int i = k - 1; i >= 0; --i) {
        double2 acc = st.g[(int64_t)i * R + r];
        for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(st.H[(int64_t)l * ldH + (int64_t)i * R + r], y[(int64_t)l * R + r]));
        const double2 d = st.H[(int64_t)i * ldH + (int64_t)i * R + r];
        const double den = d.x * d.x + d.y * d.y;
        y[(int64_t)i * R + r] = make_double2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den);
    }
    const double2 gk = st.g[(int64_t)k * R + r];
    st.cand[r] = hypot(gk.x, gk.y) <= st.tol * st.bnorm[r] ? 1 : 0;
}

// sum of active flags into one int (single workgroup)
__global__ void count_kernel(const int* __restrict__ a, int R, int* __restrict__ out) {
    __shared__ int s[256];
    int v = 0;
    for (int r = threadIdx.x; r < R; r += 256) v += a[r];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// r = b - Ax (in place on Ax), both of the basis type
template <typename TB>
__global__ void residual_kernel(const TB* __restrict__ b, TB* __restrict__ ax, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        st2(ax + t, csub(ld2(b + t), ld2(ax + t)));
}

template <typename TB>
__global__ void copy_kernel(const TB* __restrict__ src, TB* __restrict__ dst, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

template <typename TB>
__global__ void from_f64_kernel(const double2* __restrict__ src, TB* __restrict__ dst, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        st2(dst + t, src[t]);
}

__global__ void zero_kernel(double2* __restrict__ p, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = make_double2(0, 0);
}

inline unsigned ew_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

}  // namespace

// Chunks of the row range for the reduction sweeps: a function of N alone, so a
// right-hand side's sums do not depend on how many others share the batch.  Up
// to 2048 chunks (at least 128 rows each) keep a few-RHS batch spread over the
// whole chip while the partial sums stay small next to one basis vector.
int64_t gmres_rows_per_chunk(int64_t N) { return std::max<int64_t>(128, (N + 2047) / 2048); }
int gmres_nchunk(int64_t N) { return (int)((N + gmres_rows_per_chunk(N) - 1) / gmres_rows_per_chunk(N)); }

// Row folding: the DCGS2 sweeps give each lane one RHS column (two with the
// packed basis) of a row, so batches narrower than 64 (128) columns would leave
// lanes idle.  F consecutive rows of an N x R vector are the same memory as one
// row of F*R columns; the sweeps run on N/F rows of F*R columns, index the
// per-RHS coefficients by column mod R, and the dot partials of the F copies of
// a RHS are summed afterwards in a fixed order.  F depends on N only, so a
// RHS's sums have the same order whatever the width of its batch.
int gmres_fold(int64_t N) { return N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1); }

static size_t partial_values(int64_t N, int R, int m) {
    const int F = gmres_fold(N);
    return std::max((size_t)gmres_nchunk(N) * (2 * m + 2) * R,            // unfolded (CGS2)
                    (size_t)gmres_nchunk(N / F) * (2 * m + 2) * R * F);   // folded (DCGS2)
}

size_t gmres_state_bytes(int64_t N, int R, int m) {
    const int nchunk = gmres_nchunk(N);
    size_t s = 0;
    s += sizeof(double2) * (size_t)(m + 1) * (m + 1) * R;      // H (column j has m+1 rows, one spare)
    s += sizeof(double) * (size_t)m * R;                       // cs
    s += sizeof(double2) * (size_t)m * R;                      // sn
    s += sizeof(double2) * (size_t)(m + 1) * R;                // g
    s += sizeof(double2) * (size_t)(m + 1) * R * 2;            // h1, h2
    s += sizeof(double2) * (size_t)m * R;                      // y
    (void)nchunk;
    s += sizeof(double2) * partial_values(N, R, m);            // partials (of folded rows too)
    s += sizeof(double2) * (size_t)(2 * m + 2) * R * gmres_fold(N) + 256;   // chunk sums of folded rows
    s += sizeof(double2) * (size_t)R + 256;                    // reduced squared norms
    s += sizeof(double) * (size_t)R * 4 + sizeof(int) * (size_t)R * 7 + 12 * 256;
    // delayed reorthogonalisation: unrotated Hessenberg, reduced sweep, coefficients, 1/nu
    s += sizeof(double2) * (size_t)(m + 1) * (m + 1) * R + sizeof(double2) * (size_t)(2 * m + 2) * R +
         sizeof(double2) * (size_t)(2 * m + 1) * R + sizeof(double) * (size_t)R + 4 * 256;
    return s;
}

template <typename TB>
GmresResult gmres_batched(const std::function<void(const TB*, TB*)>& apply, const TB* b, double2* x, TB* Vbasis,
                          int64_t N, int R, const GmresParams& prm, DevArena& arena, hipStream_t s) {
    const int m = prm.restart;
    MBT_REQUIRE(m >= 1 && m + 1 <= kMaxVec, "gmres: restart must be in 1..63");
    const int64_t rpc = gmres_rows_per_chunk(N);
    const size_t arena_mark = arena.off;   // the recurrence state is released on return
    const int nchunk = gmres_nchunk(N);
    const int64_t vs = N * R;   // basis vector stride

    GmresState st;
    st.tol = prm.tol;
    st.H = arena.get<double2>((size_t)(m + 1) * (m + 1) * R);
    st.cs = arena.get<double>((size_t)m * R);
    st.sn = arena.get<double2>((size_t)m * R);
    st.g = arena.get<double2>((size_t)(m + 1) * R);
    st.bnorm = arena.get<double>(R);
    st.beta = arena.get<double>(R);
    st.scale = arena.get<double>(R);
    st.active = arena.get<int>(R);
    st.conv = arena.get<int>(R);
    st.cand = arena.get<int>(R);
    st.flag = arena.get<int>(R);
    st.kcyc = arena.get<int>(R);
    st.iters = arena.get<int>(R);
    int* d_count = arena.get<int>(16);
    double2* h1 = arena.get<double2>((size_t)(m + 1) * R);
    double2* h2 = arena.get<double2>((size_t)(m + 1) * R);
    double2* y = arena.get<double2>((size_t)m * R);
    double2* partial = arena.get<double2>(partial_values(N, R, m));
    double2* redf = arena.get<double2>((size_t)(2 * m + 2) * R * gmres_fold(N));
    double2* nrm2 = arena.get<double2>(R);
    double2* Hraw = nullptr;
    double2* red = nullptr;
    double2* coef_s = nullptr;
    double2* coef_c = nullptr;
    double* inv_nu = nullptr;
    if (prm.dcgs2) {
        Hraw = arena.get<double2>((size_t)(m + 1) * (m + 1) * R);
        red = arena.get<double2>((size_t)(2 * m + 2) * R);
        coef_s = arena.get<double2>((size_t)m * R);
        coef_c = arena.get<double2>((size_t)(m + 1) * R);
        inv_nu = arena.get<double>(R);
    }

    GmresResult res;
    res.iters.assign(R, 0);
    res.conv.assign(R, 0);
    res.flag.assign(R, 0);

    const dim3 gR((R + 255) / 256), bR(256);
    int* h_count = prm.host_count;

    auto count_active = [&]() -> int {
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(256), 0, s, st.active, R, d_count);
        MBT_LAUNCH_CHECK();
        MBT_HIP(hipMemcpyAsync(h_count, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        MBT_HIP(hipStreamSynchronize(s));
        return *h_count;
    };

    // Packed basis (FP32 work vectors, even R, m >= 4): the candidate u and w = A u
    // live in two work vectors and the basis vectors in m packed slots, which
    // together take no more than the m+1 FP32 slots of the plain layout.  Plain
    // layout: slot k holds the candidate u_k, slot k+1 receives w = A u_k.
    bool packed = false;
    if constexpr (std::is_same<TB, float2>::value) packed = prm.packed_basis && prm.dcgs2 && R % 2 == 0 && m >= 4;
    TB* U = Vbasis;                                   // packed: candidate, residual
    TB* Wv = Vbasis + vs;                             // packed: A u, iterate copy
    p24x2* V24 = reinterpret_cast<p24x2*>(Vbasis + 2 * vs);
    const int64_t vs24 = vs / 2;
    TB* r0v = Vbasis;                                 // residual / first candidate (both layouts)
    TB* xb = Vbasis + vs;                             // iterate in the basis type (both layouts)
    // the DCGS2 sweeps and the solution update run on folded rows
    const int F = prm.dcgs2 ? gmres_fold(N) : 1;
    const int64_t Nf = N / F;
    const int Rf = R * F;
    const int64_t rpcf = gmres_rows_per_chunk(Nf);
    const int nchunkf = gmres_nchunk(Nf);

    // x = 0, r0 = b
    hipLaunchKernelGGL(zero_kernel, dim3(ew_grid(vs)), dim3(256), 0, s, x, vs);
    hipLaunchKernelGGL((copy_kernel<TB>), dim3(ew_grid(vs)), dim3(256), 0, s, b, r0v, vs);
    MBT_LAUNCH_CHECK();
    bool first = true;
    for (int cycle = 0;; ++cycle) {
        // beta = ||r|| (r sits in V_0, or in the candidate vector when packed);
        // the convergence verdict of the previous cycle is taken on it
        hipLaunchKernelGGL((colnorm2_kernel<TB>), dim3((R + 63) / 64, nchunk), dim3(64), 0, s, r0v, N, R, rpc, partial);
        launch_reduce_partials(partial, nchunk, 1, R, nrm2, s);
        hipLaunchKernelGGL(cycle_init_kernel, gR, bR, 0, s, st, nrm2, R, first ? 1 : 0);
        MBT_LAUNCH_CHECK();
        first = false;
        if (count_active() == 0 || cycle == prm.max_cycles) break;
        res.cycles++;
        hipLaunchKernelGGL((scale_cols_kernel<TB>), dim3(ew_grid(vs)), dim3(256), 0, s, r0v, st.scale, N, R);
        MBT_LAUNCH_CHECK();
        int steps = 0;
        // delayed reorthogonalisation: one dot sweep and one update sweep per step
        // (the last step needs only the dots of u_m)
        for (int k = 0; prm.dcgs2 && k <= m; ++k) {
            const bool hasw = k < m;
            TB* u = packed ? U : Vbasis + (int64_t)k * vs;
            TB* w = hasw ? (packed ? Wv : Vbasis + (int64_t)(k + 1) * vs) : nullptr;
            if (hasw) {
                apply(u, w);
                res.matvecs += prm.matvecs_per_apply;
            }
            const double vbytes = (double)vs * sizeof(TB);
            const double bbytes = packed ? (double)vs * 6.0 : vbytes;   // one basis vector
            {
                ProfScope ps(kKArnoldiDots, k * bbytes + (hasw ? 2 : 1) * vbytes, 8.0 * (2 * k + 2) * vs, s);
                if (packed) {
                    if constexpr (std::is_same<TB, float2>::value)
                        launch_dcgs2_dots<TB, p24x2>(V24, vs24, k, u, w, Nf, Rf, rpcf, nchunkf, partial, s);
                } else {
                    launch_dcgs2_dots<TB, TB>(Vbasis, vs, k, u, w, Nf, Rf, rpcf, nchunkf, partial, s);
                }
            }
            const int nred = 2 * k + 2;
            if (F == 1) {
                launch_reduce_partials(partial, nchunkf, nred, R, red, s);
            } else {
                launch_reduce_partials(partial, nchunkf, nred, Rf, redf, s);
                hipLaunchKernelGGL(unfold_kernel, dim3((unsigned)((nred * R + 255) / 256)), dim3(256), 0, s, redf, nred,
                                   R, F, red);
                MBT_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(dcgs2_finalize_kernel, gR, bR, 0, s, st, Hraw, red, R, k, m, inv_nu);
            MBT_LAUNCH_CHECK();
            steps = k;
            if (k == m || count_active() == 0) break;
            hipLaunchKernelGGL(dcgs2_coef_kernel, dim3((R + 255) / 256, k + 1), bR, 0, s, Hraw, red, R, k, m, inv_nu,
                               coef_s, coef_c);
            MBT_LAUNCH_CHECK();
            {
                // k basis vectors, u and w read; v_k and u_{k+1} written
                ProfScope ps(kKArnoldiUpdateDots, (k + 1) * bbytes + 3 * vbytes, 16.0 * k * vs, s);
                if (packed) {
                    if constexpr (std::is_same<TB, float2>::value)
                        launch_dcgs2_update24(V24, vs24, k, U, Wv, V24 + (int64_t)k * vs24, coef_s, coef_c, inv_nu, Nf,
                                              Rf, R, s);
                } else {
                    launch_dcgs2_update<TB>(Vbasis, vs, k, u, w, coef_s, coef_c, inv_nu, Nf, Rf, R, s);
                }
            }
        }
        for (int j = 0; !prm.dcgs2 && j < m; ++j) {
            steps = j + 1;
            TB* vj = Vbasis + (int64_t)j * vs;
            TB* w = Vbasis + (int64_t)(j + 1) * vs;
            apply(vj, w);
            res.matvecs += prm.matvecs_per_apply;
            const int nvec = j + 1;
            // algorithmic traffic of a pass: nvec basis vectors and w read (+ w written by the updates)
            const double vbytes = (double)vs * sizeof(TB);
            {
                ProfScope ps(kKArnoldiDots, (nvec + 1) * vbytes, 8.0 * nvec * vs, s);
                launch_pass<TB, TB, 0>(Vbasis, vs, nvec, nullptr, w, N, R, rpc, nchunk, partial, s);
            }
            launch_reduce_partials(partial, nchunk, nvec, R, h1, s);
            {
                ProfScope ps(kKArnoldiUpdateDots, (nvec + 2) * vbytes, 16.0 * nvec * vs, s);
                launch_pass<TB, TB, 1>(Vbasis, vs, nvec, h1, w, N, R, rpc, nchunk, partial, s);
            }
            launch_reduce_partials(partial, nchunk, nvec, R, h2, s);
            {
                ProfScope ps(kKArnoldiUpdateNorm, (nvec + 2) * vbytes, 8.0 * nvec * vs, s);
                launch_pass<TB, TB, 2>(Vbasis, vs, nvec, h2, w, N, R, rpc, nchunk, partial, s);
            }
            hipLaunchKernelGGL(finalize_kernel, gR, bR, 0, s, st, h1, h2, partial, nchunk, R, j, m);
            hipLaunchKernelGGL((scale_cols_kernel<TB>), dim3(ew_grid(vs)), dim3(256), 0, s, w, st.scale, N, R);
            MBT_LAUNCH_CHECK();
            if (count_active() == 0) break;
        }
        // y = R^{-1} g ; x += V y
        hipLaunchKernelGGL(cycle_solve_kernel, gR, bR, 0, s, st, R, m, y);
        MBT_LAUNCH_CHECK();
        // configuration fixed by m: a RHS's update x += V y does not depend on how long
        // the other RHS of the batch kept the cycle going
        if (packed)
            launch_solution_update<p24x2>(V24, vs24, steps, y, x, Nf, Rf, R, s);
        else
            launch_solution_update<TB>(Vbasis, vs, steps, y, x, Nf, Rf, R, s);
        // explicit residual r = b - A x into V_0 (x cast to the basis type into V_1 first)
        hipLaunchKernelGGL((from_f64_kernel<TB>), dim3(ew_grid(vs)), dim3(256), 0, s, x, xb, vs);
        MBT_LAUNCH_CHECK();
        apply(xb, r0v);
        res.matvecs += prm.matvecs_per_apply;
        hipLaunchKernelGGL((residual_kernel<TB>), dim3(ew_grid(vs)), dim3(256), 0, s, b, r0v, vs);
        MBT_LAUNCH_CHECK();
    }
    MBT_HIP(hipMemcpyAsync(res.iters.data(), st.iters, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.conv.data(), st.conv, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.flag.data(), st.flag, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    arena.off = arena_mark;
    return res;
}

// ------------------------------------------------------------------ batched PCG (Sec. II-C)
// Conjugate gradients on N x = b (N = Z^H Z, Hermitian positive definite) with
// the preconditioner P applied as P^{-1}; one independent recurrence per RHS
// column, FP64 coefficients and dots, vectors of type TB.  With P = L L^H the
// iterates are those of plain CG on the split system of eq. (precond), and the
// stop test is that system's relative residual sqrt(r^H P^{-1} r / b^H P^{-1} b).
namespace {

// partial[chunk][r] = sum over the chunk's rows of conj(a) b
template <typename TB>
__global__ void pcg_dot_kernel(const TB* __restrict__ a, const TB* __restrict__ b, int64_t N, int R,
                               int64_t rows_per_chunk, double2* __restrict__ partial) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (r >= R) return;
    const int64_t n0 = chunk * rows_per_chunk, n1 = min(N, n0 + rows_per_chunk);
    double2 acc = make_double2(0, 0);
    for (int64_t n = n0; n < n1; ++n) acc = cfmac(acc, ld2(a + n * R + r), ld2(b + n * R + r));
    partial[chunk * R + r] = acc;
}

struct PcgState {
    double tol;
    double *rho, *rho0, *alpha, *beta;
    int *active, *conv, *flag, *iters;
};

__global__ void pcg_init_kernel(PcgState st, const double2* __restrict__ rz, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double rho = rz[r].x;
    st.rho[r] = rho;
    st.rho0[r] = rho;
    st.iters[r] = 0;
    st.flag[r] = !(rho == rho) || isinf(rho) || rho < 0.0;
    st.conv[r] = !st.flag[r] && rho == 0.0;
    st.active[r] = !st.flag[r] && !st.conv[r];
    st.alpha[r] = 0.0;
    st.beta[r] = 0.0;
}

// alpha = rho / p^H q for the RHS still iterating
__global__ void pcg_alpha_kernel(PcgState st, const double2* __restrict__ pq, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double a = 0.0;
    if (st.active[r]) {
        a = st.rho[r] / pq[r].x;
        if (!(a == a) || isinf(a)) {
            st.flag[r] = 1;
            st.active[r] = 0;
            a = 0.0;
        }
    }
    st.alpha[r] = a;
}

// x += alpha p (x in FP64), r -= alpha q
template <typename TB>
__global__ void pcg_xr_kernel(double2* __restrict__ x, TB* __restrict__ rv, const TB* __restrict__ p,
                              const TB* __restrict__ q, const double* __restrict__ alpha, int64_t NR, int R) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NR; t += (int64_t)gridDim.x * blockDim.x) {
        const double a = alpha[t % R];
        const double2 pv = ld2(p + t), qv = ld2(q + t), xv = x[t], rr = ld2(rv + t);
        x[t] = make_double2(fma(a, pv.x, xv.x), fma(a, pv.y, xv.y));
        st2(rv + t, make_double2(fma(-a, qv.x, rr.x), fma(-a, qv.y, rr.y)));
    }
}

// rho_new = r^H z: stop test on the split-system residual, then beta
__global__ void pcg_beta_kernel(PcgState st, const double2* __restrict__ rz, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double b = 0.0;
    if (st.active[r]) {
        const double rn = rz[r].x;
        st.iters[r] += 1;
        if (!(rn == rn) || isinf(rn)) {
            st.flag[r] = 1;
            st.active[r] = 0;
        } else if (sqrt(fmax(rn, 0.0) / st.rho0[r]) <= st.tol) {
            st.conv[r] = 1;
            st.active[r] = 0;
        } else {
            b = rn / st.rho[r];
            st.rho[r] = rn;
        }
    }
    st.beta[r] = b;
}

// p = z + beta p
template <typename TB>
__global__ void pcg_p_kernel(TB* __restrict__ p, const TB* __restrict__ z, const double* __restrict__ beta, int64_t NR,
                             int R) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NR; t += (int64_t)gridDim.x * blockDim.x) {
        const double b = beta[t % R];
        const double2 zv = ld2(z + t), pv = ld2(p + t);
        st2(p + t, make_double2(fma(b, pv.x, zv.x), fma(b, pv.y, zv.y)));
    }
}

template <typename TB>
void pcg_dot(const TB* a, const TB* b, int64_t N, int R, double2* partial, double2* out, hipStream_t s) {
    const int64_t rpc = gmres_rows_per_chunk(N);
    const int nchunk = gmres_nchunk(N);
    hipLaunchKernelGGL((pcg_dot_kernel<TB>), dim3((R + 63) / 64, nchunk), dim3(64), 0, s, a, b, N, R, rpc, partial);
    MBT_LAUNCH_CHECK();
    launch_reduce_partials(partial, nchunk, 1, R, out, s);
}

}  // namespace

size_t pcg_state_bytes(int64_t N, int R) {
    return sizeof(double2) * (size_t)gmres_nchunk(N) * R + 2 * sizeof(double2) * (size_t)R +
           4 * sizeof(double) * (size_t)R + 4 * sizeof(int) * (size_t)R + 16 * 256;
}

template <typename TB>
GmresResult pcg_batched(const std::function<void(const TB*, TB*)>& applyN,
                        const std::function<void(const TB*, TB*)>& applyPinv, const TB* b, double2* x, TB* work,
                        int64_t N, int R, double tol, int maxit, int* host_count, DevArena& arena, hipStream_t s) {
    const size_t mark = arena.off;
    const int64_t NR = N * R;
    TB* rv = work;
    TB* z = work + NR;
    TB* p = work + 2 * NR;
    TB* q = work + 3 * NR;
    PcgState st;
    st.tol = tol;
    st.rho = arena.get<double>(R);
    st.rho0 = arena.get<double>(R);
    st.alpha = arena.get<double>(R);
    st.beta = arena.get<double>(R);
    st.active = arena.get<int>(R);
    st.conv = arena.get<int>(R);
    st.flag = arena.get<int>(R);
    st.iters = arena.get<int>(R);
    double2* partial = arena.get<double2>((size_t)gmres_nchunk(N) * R);
    double2* dot = arena.get<double2>(R);
    int* d_count = arena.get<int>(16);
    const dim3 gR((R + 255) / 256), bR(256);
    auto count_active = [&]() -> int {
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(256), 0, s, st.active, R, d_count);
        MBT_LAUNCH_CHECK();
        MBT_HIP(hipMemcpyAsync(host_count, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        MBT_HIP(hipStreamSynchronize(s));
        return *host_count;
    };
    GmresResult res;
    // x = 0, r = b, z = P^{-1} r, p = z, rho = r^H z
    hipLaunchKernelGGL(zero_kernel, dim3(ew_grid(NR)), dim3(256), 0, s, x, NR);
    hipLaunchKernelGGL((copy_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, b, rv, NR);
    MBT_LAUNCH_CHECK();
    applyPinv(rv, z);
    hipLaunchKernelGGL((copy_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, z, p, NR);
    MBT_LAUNCH_CHECK();
    pcg_dot<TB>(rv, z, N, R, partial, dot, s);
    hipLaunchKernelGGL(pcg_init_kernel, gR, bR, 0, s, st, dot, R);
    MBT_LAUNCH_CHECK();
    res.cycles = 1;
    for (int it = 0; it < maxit && count_active() > 0; ++it) {
        applyN(p, q);
        pcg_dot<TB>(p, q, N, R, partial, dot, s);
        hipLaunchKernelGGL(pcg_alpha_kernel, gR, bR, 0, s, st, dot, R);
        hipLaunchKernelGGL((pcg_xr_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, x, rv, p, q, st.alpha, NR, R);
        MBT_LAUNCH_CHECK();
        applyPinv(rv, z);
        pcg_dot<TB>(rv, z, N, R, partial, dot, s);
        hipLaunchKernelGGL(pcg_beta_kernel, gR, bR, 0, s, st, dot, R);
        hipLaunchKernelGGL((pcg_p_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, p, z, st.beta, NR, R);
        MBT_LAUNCH_CHECK();
        res.matvecs += 2;
    }
    res.iters.assign(R, 0);
    res.conv.assign(R, 0);
    res.flag.assign(R, 0);
    MBT_HIP(hipMemcpyAsync(res.iters.data(), st.iters, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.conv.data(), st.conv, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.flag.data(), st.flag, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    arena.off = mark;
    return res;
}

// ------------------------------------------------------------------ batched COCG
// Conjugate orthogonal conjugate gradients (van der Vorst and Melissen, 1990)
// on Z x = b for complex symmetric Z with a complex symmetric preconditioner M
// applied as M^{-1}: the CG recurrences with the bilinear form a^T b in place
// of a^H b.  One operator application and one preconditioner application per
// step, no Krylov basis.  Stop test: ||r|| <= tol ||b||.  The element-block
// P_K is symmetric (Galerkin self block), so M = P_K keeps the recurrence
// valid.  One independent recurrence per RHS column, FP64 coefficients.
namespace {

// partial[chunk][v][r]: v = 0: sum a b (bilinear); NORM: v = 1: sum |a|^2
template <typename TB, bool NORM>
__global__ void cocg_dot_kernel(const TB* __restrict__ a, const TB* __restrict__ b, int64_t N, int R,
                                int64_t rows_per_chunk, double2* __restrict__ partial) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (r >= R) return;
    const int64_t n0 = chunk * rows_per_chunk, n1 = min(N, n0 + rows_per_chunk);
    double2 ab = make_double2(0, 0);
    double aa = 0.0;
    for (int64_t n = n0; n < n1; ++n) {
        const double2 av = ld2(a + n * R + r);
        ab = cfma(ab, av, ld2(b + n * R + r));
        if (NORM) aa = fma(av.y, av.y, fma(av.x, av.x, aa));
    }
    constexpr int nv = NORM ? 2 : 1;
    partial[(chunk * nv) * R + r] = ab;
    if (NORM) partial[(chunk * nv + 1) * R + r] = make_double2(aa, 0.0);
}

struct CocgState {
    double tol;
    double2 *rho, *alpha, *beta;
    double* bnorm2;
    int *active, *conv, *flag, *iters;
};

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// red = [r^T z, |r|^2] of the initial residual r = b
__global__ void cocg_init_kernel(CocgState st, const double2* __restrict__ red, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double2 rho = red[r];
    const double bb = red[R + r].x;
    st.rho[r] = rho;
    st.bnorm2[r] = bb;
    st.iters[r] = 0;
    st.flag[r] = !(bb == bb) || isinf(bb) || !(rho.x == rho.x) || !(rho.y == rho.y);
    st.conv[r] = !st.flag[r] && bb == 0.0;
    st.active[r] = !st.flag[r] && !st.conv[r];
    st.alpha[r] = make_double2(0, 0);
    st.beta[r] = make_double2(0, 0);
}

// alpha = rho / p^T q for the RHS still iterating (a vanishing p^T q is a breakdown)
__global__ void cocg_alpha_kernel(CocgState st, const double2* __restrict__ pq, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double2 a = make_double2(0, 0);
    if (st.active[r]) {
        a = cdiv(st.rho[r], pq[r]);
        if (!(a.x == a.x) || !(a.y == a.y) || isinf(a.x) || isinf(a.y)) {
            st.flag[r] = 1;
            st.active[r] = 0;
            a = make_double2(0, 0);
        }
    }
    st.alpha[r] = a;
}

// x += alpha p (x in FP64), r -= alpha q
template <typename TB>
__global__ void cocg_xr_kernel(double2* __restrict__ x, TB* __restrict__ rv, const TB* __restrict__ p,
                               const TB* __restrict__ q, const double2* __restrict__ alpha, int64_t NR, int R) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NR; t += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = alpha[t % R];
        const double2 na = make_double2(-a.x, -a.y);
        x[t] = cfma(x[t], a, ld2(p + t));
        st2(rv + t, cfma(ld2(rv + t), na, ld2(q + t)));
    }
}

// red = [r^T z, |r|^2]: stop test on ||r|| / ||b||, then beta = rho_new / rho
__global__ void cocg_beta_kernel(CocgState st, const double2* __restrict__ red, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double2 b = make_double2(0, 0);
    if (st.active[r]) {
        const double2 rz = red[r];
        const double rr = red[R + r].x;
        st.iters[r] += 1;
        if (!(rr == rr) || isinf(rr) || !(rz.x == rz.x) || !(rz.y == rz.y)) {
            st.flag[r] = 1;
            st.active[r] = 0;
        } else if (sqrt(rr / st.bnorm2[r]) <= st.tol) {
            st.conv[r] = 1;
            st.active[r] = 0;
        } else if (rr > 1e12 * st.bnorm2[r]) {
            // a residual a million times the right-hand side: the recurrence has run away
            // (the FP32 short recurrence does so on a few RHS); stop it unconverged
            st.active[r] = 0;
        } else {
            b = cdiv(rz, st.rho[r]);
            st.rho[r] = rz;
        }
    }
    st.beta[r] = b;
}

// p = z + beta p
template <typename TB>
__global__ void cocg_p_kernel(TB* __restrict__ p, const TB* __restrict__ z, const double2* __restrict__ beta,
                              int64_t NR, int R) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NR; t += (int64_t)gridDim.x * blockDim.x)
        st2(p + t, cfma(ld2(z + t), beta[t % R], ld2(p + t)));
}

template <typename TB, bool NORM>
void cocg_dot(const TB* a, const TB* b, int64_t N, int R, double2* partial, double2* out, hipStream_t s) {
    const int64_t rpc = gmres_rows_per_chunk(N);
    const int nchunk = gmres_nchunk(N);
    hipLaunchKernelGGL((cocg_dot_kernel<TB, NORM>), dim3((R + 63) / 64, nchunk), dim3(64), 0, s, a, b, N, R, rpc,
                       partial);
    MBT_LAUNCH_CHECK();
    launch_reduce_partials(partial, nchunk, NORM ? 2 : 1, R, out, s);
}

}  // namespace

size_t cocg_state_bytes(int64_t N, int R) {
    return 2 * sizeof(double2) * (size_t)gmres_nchunk(N) * R + 2 * sizeof(double2) * (size_t)R +
           3 * sizeof(double2) * (size_t)R + sizeof(double) * (size_t)R + 4 * sizeof(int) * (size_t)R + 16 * 256;
}

template <typename TB>
GmresResult cocg_batched(const std::function<void(const TB*, TB*)>& applyZ,
                         const std::function<void(const TB*, TB*)>& applyMinv, const TB* b, double2* x, TB* work,
                         int64_t N, int R, double tol, int maxit, int* host_count, DevArena& arena, hipStream_t s) {
    const size_t mark = arena.off;
    const int64_t NR = N * R;
    TB* rv = work;
    TB* z = work + NR;
    TB* p = work + 2 * NR;
    TB* q = work + 3 * NR;
    CocgState st;
    st.tol = tol;
    st.rho = arena.get<double2>(R);
    st.alpha = arena.get<double2>(R);
    st.beta = arena.get<double2>(R);
    st.bnorm2 = arena.get<double>(R);
    st.active = arena.get<int>(R);
    st.conv = arena.get<int>(R);
    st.flag = arena.get<int>(R);
    st.iters = arena.get<int>(R);
    double2* partial = arena.get<double2>(2 * (size_t)gmres_nchunk(N) * R);
    double2* red = arena.get<double2>(2 * (size_t)R);
    int* d_count = arena.get<int>(16);
    const dim3 gR((R + 255) / 256), bR(256);
    auto count_active = [&]() -> int {
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(256), 0, s, st.active, R, d_count);
        MBT_LAUNCH_CHECK();
        MBT_HIP(hipMemcpyAsync(host_count, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        MBT_HIP(hipStreamSynchronize(s));
        return *host_count;
    };
    GmresResult res;
    // x = 0, r = b, z = M^{-1} r, p = z, rho = r^T z
    hipLaunchKernelGGL(zero_kernel, dim3(ew_grid(NR)), dim3(256), 0, s, x, NR);
    hipLaunchKernelGGL((copy_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, b, rv, NR);
    MBT_LAUNCH_CHECK();
    applyMinv(rv, z);
    hipLaunchKernelGGL((copy_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, z, p, NR);
    MBT_LAUNCH_CHECK();
    cocg_dot<TB, true>(rv, z, N, R, partial, red, s);
    hipLaunchKernelGGL(cocg_init_kernel, gR, bR, 0, s, st, red, R);
    MBT_LAUNCH_CHECK();
    res.cycles = 1;
    for (int it = 0; it < maxit && count_active() > 0; ++it) {
        applyZ(p, q);
        cocg_dot<TB, false>(p, q, N, R, partial, red, s);
        hipLaunchKernelGGL(cocg_alpha_kernel, gR, bR, 0, s, st, red, R);
        hipLaunchKernelGGL((cocg_xr_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, x, rv, p, q, st.alpha, NR, R);
        MBT_LAUNCH_CHECK();
        applyMinv(rv, z);
        cocg_dot<TB, true>(rv, z, N, R, partial, red, s);
        hipLaunchKernelGGL(cocg_beta_kernel, gR, bR, 0, s, st, red, R);
        hipLaunchKernelGGL((cocg_p_kernel<TB>), dim3(ew_grid(NR)), dim3(256), 0, s, p, z, st.beta, NR, R);
        MBT_LAUNCH_CHECK();
        res.matvecs += 1;
    }
    res.iters.assign(R, 0);
    res.conv.assign(R, 0);
    res.flag.assign(R, 0);
    MBT_HIP(hipMemcpyAsync(res.iters.data(), st.iters, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.conv.data(), st.conv, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipMemcpyAsync(res.flag.data(), st.flag, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    arena.off = mark;
    return res;
}

template GmresResult cocg_batched<double2>(const std::function<void(const double2*, double2*)>&,
                                           const std::function<void(const double2*, double2*)>&, const double2*,
                                           double2*, double2*, int64_t, int, double, int, int*, DevArena&, hipStream_t);
template GmresResult cocg_batched<float2>(const std::function<void(const float2*, float2*)>&,
                                          const std::function<void(const float2*, float2*)>&, const float2*, double2*,
                                          float2*, int64_t, int, double, int, int*, DevArena&, hipStream_t);

template GmresResult pcg_batched<double2>(const std::function<void(const double2*, double2*)>&,
                                          const std::function<void(const double2*, double2*)>&, const double2*,
                                          double2*, double2*, int64_t, int, double, int, int*, DevArena&, hipStream_t);
template GmresResult pcg_batched<float2>(const std::function<void(const float2*, float2*)>&,
                                         const std::function<void(const float2*, float2*)>&, const float2*, double2*,
                                         float2*, int64_t, int, double, int, int*, DevArena&, hipStream_t);

template GmresResult gmres_batched<double2>(const std::function<void(const double2*, double2*)>&, const double2*,
                                            double2*, double2*, int64_t, int, const GmresParams&, DevArena&, hipStream_t);
template GmresResult gmres_batched<float2>(const std::function<void(const float2*, float2*)>&, const float2*, double2*,
                                           float2*, int64_t, int, const GmresParams&, DevArena&, hipStream_t);

}  // namespace mbt

// RWG functions of a planar element and the EFIE interaction blocks of a lattice of them.
//
// The paper represents its elements with Rao-Wilton-Glisson functions (Sec. I,
// Sec. II-B) and leaves the fill rules open.  This fill: one function per
// interior edge of the element mesh, f = +-(l / 2A)(r - v) on the edge's two
// triangles (v the vertex opposite the edge, + on the lower-index triangle),
// Galerkin entries Z_mn = j k eta <<f_m . f_n, G>> - j (eta / k) <<div f_m,
// div f_n, G>> with G = exp(-jkR) / (4 pi R), Radon's seven-point (degree 5)
// rule on test and source triangles, and for elements at most one lattice step
// apart in x and y the static part 1/(4 pi R) of the source integral taken in
// closed form at each test point (coplanar potential integrals of Wilton et al.,
// IEEE TAP 1984), the remainder (exp(-jkR) - 1)/(4 pi R) by the rule.
//
// One workgroup per lattice offset.  The source triangles are taken in chunks
// of U (the chunk's moments fill at most 64 KB of LDS).  Phase 1: a thread per
// (test triangle t, source triangle u) integrates over the 7 x 7 point pairs
// the six moments, taken about the test triangle's centroid c_t,
//   m0 = <<G>>, mr = <<(r - c_t) G>> (two components), mp = <<r' G>> (two
//   components) and mrp = <<(r - c_t) . r' G>>,
// once per triangle pair (a triangle carries up to three RWG functions, so
// moments per function would repeat this work about 2.6 times on the bowtie).
// Phase 2: a thread per (test basis m, source basis q) combines, for each of q's
// triangles in the chunk, the moments of m's two triangles (v_m and v_q the
// free vertices, d_m = v_m - c_t):
//   <<(r - v_m) . (r' - v_q) G>> = mrp - d_m . mp - v_q . (mr - d_m m0),
// writing the T+ contribution of q (its lower-index triangle, always in an
// earlier or the same chunk) and adding the T- one, in a fixed order, so the
// block is deterministic.  The work is FP64 transcendental-bound.
// Blocks two or more lattice steps apart use the same rule on test and source
// side, so T[-d] = T[d]^T for them (Galerkin reciprocity of the discrete
// operator): only one of each such pair is integrated and the other is its
// transpose; the nearer blocks, whose static part is integrated one-sidedly,
// are all integrated.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>

#include "rwg.h"
#include "runtime.h"

namespace mbt {

namespace {

constexpr double kEta = 376.730313668;   // free-space wave impedance, ohm
constexpr double kInv4Pi = 0.25 / M_PI;

struct RwgDev {
    const double2* qp;
    const double* qw;
    const double2* tv;
    const double* area;
    const double2* tcen;   // nt: triangle centroids
    const int* btri;
    const double2* bfree;
    const double2* bdel;   // 2M: free vertex minus the centroid of its triangle
    const double* blen;
};

constexpr int kPairVals = 6;                      // m0, mr (x, y), mp (x, y), mrp per triangle pair
constexpr int kPairLdsBytes = 64 * 1024;          // LDS for one chunk of pair moments

// exp(-jkR)/(4 pi R)
__device__ __forceinline__ double2 green_full(double k, double R) {
    double s, c;
    sincos(k * R, &s, &c);
    const double f = kInv4Pi / R;
    return make_double2(c * f, -s * f);
}

// (exp(-jkR) - 1)/(4 pi R) = -(k / 4 pi) (sin x / x)(sin x + j cos x), x = kR/2 (finite at R = 0)
__device__ __forceinline__ double2 green_rem(double k, double R) {
    const double x = 0.5 * k * R;
    double s, c;
    sincos(x, &s, &c);
    const double f = -k * kInv4Pi * (x > 0.0 ? s / x : 1.0);
    return make_double2(f * s, f * c);
}

// Closed-form S0 = int_T dS'/|r' - rho| and S1 = int_T (r' - rho)/|r' - rho| dS' for
// rho in the plane of triangle v[0..2]: over the edges (p-, p+), with unit direction t,
// outward normal u, P = (p - rho).u, l+- = (p+- - rho).t, R+- = |p+- - rho| and
// L = ln((R+ + l+)/(R- + l-)):  S0 = sum P L,  S1 = 1/2 sum u (P^2 L + l+ R+ - l- R-).
__device__ void static_potentials(const double2* v, double2 rho, double& S0, double2& S1) {
    const double cx = (v[0].x + v[1].x + v[2].x) / 3.0, cy = (v[0].y + v[1].y + v[2].y) / 3.0;
    S0 = 0.0;
    S1 = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double2 pm = v[i], pp = v[(i + 1) % 3];
        const double ex = pp.x - pm.x, ey = pp.y - pm.y;
        const double len = sqrt(ex * ex + ey * ey);
        const double tx = ex / len, ty = ey / len;
        double ux = ty, uy = -tx;
        if ((pm.x - cx) * ux + (pm.y - cy) * uy < 0.0) {
            ux = -ux;
            uy = -uy;
        }
        const double dmx = pm.x - rho.x, dmy = pm.y - rho.y;
        const double dpx = pp.x - rho.x, dpy = pp.y - rho.y;
        const double P = dmx * ux + dmy * uy;
        const double lp = dpx * tx + dpy * ty, lm = dmx * tx + dmy * ty;
        const double Rp = sqrt(dpx * dpx + dpy * dpy), Rm = sqrt(dmx * dmx + dmy * dmy);
        double c1 = lp * Rp - lm * Rm;
        if (P != 0.0) {
            // R + l = P^2 / (R - l) where l < 0 avoids the cancellation
            double L;
            if (lp < 0.0 && lm < 0.0) {
                L = log((Rm - lm) / (Rp - lp));
            } else {
                const double num = lp < 0.0 ? P * P / (Rp - lp) : Rp + lp;
                const double den = lm < 0.0 ? P * P / (Rm - lm) : Rm + lm;
                L = log(num / den);
            }
            S0 += P * L;
            c1 += P * P * L;
        }
        S1.x += 0.5 * c1 * ux;
        S1.y += 0.5 * c1 * uy;
    }
}

__global__ __launch_bounds__(256) void rwg_fill_kernel(RwgDev d, int nt, int M, int U, int nx, int ny, double ldx,
                                                       double ldy, double k, double2* __restrict__ T) {
    extern __shared__ double2 pm[];   // [t][u - u0][kPairVals]
    const int nox = 2 * nx - 1;
    const int off = blockIdx.x;
    const int ox = off % nox - (nx - 1), oy = off / nox - (ny - 1);
    // the test element sits at lattice offset (ox, oy) from the source element at the origin
    const double sx = ox * ldx, sy = oy * ldy;
    const bool near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
    if (!near && (oy < 0 || (oy == 0 && ox < 0))) return;   // the transpose of T[-d], filled afterwards
    double2* Tb = T + (int64_t)off * M * M;
    for (int u0 = 0; u0 < nt; u0 += U) {
        const int nu = min(U, nt - u0);
        for (int task = threadIdx.x; task < nt * nu; task += blockDim.x) {
            const int t = task / nu, u = u0 + task - (task / nu) * nu;
            const double2 ct = d.tcen[t];
            double2 rs[kRwgQ];
            double ws[kRwgQ];
#pragma unroll
            for (int j = 0; j < kRwgQ; ++j) {
                rs[j] = d.qp[u * kRwgQ + j];
                ws[j] = d.qw[u * kRwgQ + j];
            }
            double2 tvu[3];
            if (near) {
#pragma unroll
                for (int j = 0; j < 3; ++j) tvu[j] = d.tv[u * 3 + j];
            }
            double2 m0 = make_double2(0, 0), mrx = m0, mry = m0, mpx = m0, mpy = m0, mrp = m0;
            for (int i = 0; i < kRwgQ; ++i) {
                const double2 q = d.qp[t * kRwgQ + i];
                const double rox = q.x + sx, roy = q.y + sy;
                const double wo = d.qw[t * kRwgQ + i];
                double2 g0 = make_double2(0, 0), g1x = make_double2(0, 0), g1y = make_double2(0, 0);
#pragma unroll
                for (int j = 0; j < kRwgQ; ++j) {
                    const double dx = rox - rs[j].x, dy = roy - rs[j].y;
                    const double R = sqrt(dx * dx + dy * dy);
                    const double2 G = near ? green_rem(k, R) : green_full(k, R);
                    const double2 wg = make_double2(ws[j] * G.x, ws[j] * G.y);
                    g0 = cadd(g0, wg);
                    g1x = cadd(g1x, make_double2(rs[j].x * wg.x, rs[j].x * wg.y));
                    g1y = cadd(g1y, make_double2(rs[j].y * wg.x, rs[j].y * wg.y));
                }
                if (near) {
                    double S0;
                    double2 S1;
                    static_potentials(tvu, make_double2(rox, roy), S0, S1);
                    g0.x += S0 * kInv4Pi;
                    g1x.x += (S1.x + rox * S0) * kInv4Pi;
                    g1y.x += (S1.y + roy * S0) * kInv4Pi;
                }
                // about the centroid in the element frame: the lattice shift cancels exactly
                const double ax = q.x - ct.x, ay = q.y - ct.y;
                m0 = cadd(m0, make_double2(wo * g0.x, wo * g0.y));
                mrx = cadd(mrx, make_double2(wo * ax * g0.x, wo * ax * g0.y));
                mry = cadd(mry, make_double2(wo * ay * g0.x, wo * ay * g0.y));
                mpx = cadd(mpx, make_double2(wo * g1x.x, wo * g1x.y));
                mpy = cadd(mpy, make_double2(wo * g1y.x, wo * g1y.y));
                mrp = cadd(mrp, make_double2(wo * (ax * g1x.x + ay * g1y.x), wo * (ax * g1x.y + ay * g1y.y)));
            }
            double2* a = pm + ((int64_t)t * U + (u - u0)) * kPairVals;
            a[0] = m0;
            a[1] = mrx;
            a[2] = mry;
            a[3] = mpx;
            a[4] = mpy;
            a[5] = mrp;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
            const int m = e / M, qb = e - (e / M) * M;
            const double lmq = d.blen[m] * d.blen[qb];
#pragma unroll
            for (int tau = 0; tau < 2; ++tau) {
                const int u = d.btri[2 * qb + tau];
                if (u < u0 || u >= u0 + nu) continue;
                const double Au = d.area[u];
                const double2 vq = d.bfree[2 * qb + tau];
                double2 sum = make_double2(0, 0);
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int t = d.btri[2 * m + side];
                    const double At = d.area[t];
                    const double2 dm = d.bdel[2 * m + side];
                    const double2* a = pm + ((int64_t)t * U + (u - u0)) * kPairVals;
                    const double2 hvx = csub(a[1], make_double2(dm.x * a[0].x, dm.x * a[0].y));
                    const double2 hvy = csub(a[2], make_double2(dm.y * a[0].x, dm.y * a[0].y));
                    const double2 hw = make_double2(a[5].x - (dm.x * a[3].x + dm.y * a[4].x),
                                                    a[5].y - (dm.x * a[3].y + dm.y * a[4].y));
                    const double2 A = make_double2(hw.x - (vq.x * hvx.x + vq.y * hvy.x),
                                                   hw.y - (vq.x * hvx.y + vq.y * hvy.y));
                    // j k eta A / (4 At Au) - j (eta / k) m0 / (At Au)
                    const double cv = k * kEta / (4.0 * At * Au), cs = kEta / (k * At * Au);
                    const double re = -(cv * A.y - cs * a[0].y);
                    const double im = cv * A.x - cs * a[0].x;
                    const double sg = (side == tau) ? lmq : -lmq;
                    sum.x += sg * re;
                    sum.y += sg * im;
                }
                if (tau == 0) Tb[e] = sum;
                else Tb[e] = cadd(Tb[e], sum);
            }
        }
        __syncthreads();
    }
}

// T[d] = T[-d]^T for the far offsets that the fill kernel skipped (one row p per thread block)
__global__ __launch_bounds__(128) void rwg_mirror_kernel(int M, int nx, int ny, double2* __restrict__ T) {
    const int nox = 2 * nx - 1;
    const int off = blockIdx.x;
    const int ox = off % nox - (nx - 1), oy = off / nox - (ny - 1);
    const bool near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
    if (near || !(oy < 0 || (oy == 0 && ox < 0))) return;
    const int mirror = (-oy + (ny - 1)) * nox + (-ox + (nx - 1));
    const int p = blockIdx.y;
    for (int q = threadIdx.x; q < M; q += blockDim.x)
        T[((int64_t)off * M + p) * M + q] = T[((int64_t)mirror * M + q) * M + p];
}

}  // namespace

RwgMesh rwg_from_mesh(const mbt_rwg_mesh& ms) {
    MBT_REQUIRE(ms.vert && ms.tri && ms.port_edges, "NULL mesh array");
    MBT_REQUIRE(ms.nvert >= 3 && ms.nvert <= 4096, "nvert must be within 3..4096");
    MBT_REQUIRE(ms.ntri >= 2 && ms.ntri <= kRwgMaxTri, "ntri must be within 2..256");
    MBT_REQUIRE(ms.nport_edges >= 1 && ms.nport_edges <= kMaxPortBases, "nport_edges must be within 1..8");
    MBT_REQUIRE(std::isfinite(ms.port_dir[0]) && std::isfinite(ms.port_dir[1]) &&
                    (ms.port_dir[0] != 0.0 || ms.port_dir[1] != 0.0),
                "port_dir must be a finite nonzero vector");
    const int nv = ms.nvert, nt = ms.ntri;
    std::vector<double2> v(nv);
    for (int i = 0; i < nv; ++i) {
        v[i] = make_double2(ms.vert[2 * i], ms.vert[2 * i + 1]);
        MBT_REQUIRE(std::isfinite(v[i].x) && std::isfinite(v[i].y), "mesh vertices must be finite");
    }
    RwgMesh h;
    h.nt = nt;
    h.area.resize(nt);
    h.tv.resize((size_t)nt * 3);
    std::map<std::pair<int, int>, std::vector<int>> owners;
    for (int t = 0; t < nt; ++t) {
        int id[3];
        for (int j = 0; j < 3; ++j) {
            id[j] = ms.tri[3 * t + j];
            MBT_REQUIRE(id[j] >= 0 && id[j] < nv, "triangle vertex index out of range");
            h.tv[3 * t + j] = v[id[j]];
        }
        MBT_REQUIRE(id[0] != id[1] && id[1] != id[2] && id[0] != id[2], "triangle with a repeated vertex");
        const double2 a = v[id[0]], b = v[id[1]], c = v[id[2]];
        h.area[t] = 0.5 * std::fabs((b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x));
        MBT_REQUIRE(h.area[t] > 0.0, "degenerate (zero-area) triangle");
        for (int j = 0; j < 3; ++j) {
            const int p = id[j], q = id[(j + 1) % 3];
            owners[{std::min(p, q), std::max(p, q)}].push_back(t);
        }
    }
    // interior edges in increasing (smaller vertex, larger vertex) order (std::map order)
    std::map<std::pair<int, int>, int> index;
    for (const auto& kv : owners) {
        MBT_REQUIRE(kv.second.size() <= 2, "mesh edge shared by more than two triangles");
        if (kv.second.size() != 2) continue;
        const int m = h.M++;
        index[kv.first] = m;
        const int tp = std::min(kv.second[0], kv.second[1]), tm = std::max(kv.second[0], kv.second[1]);
        MBT_REQUIRE(tp != tm, "triangle listed twice");
        auto opposite = [&](int t) {
            for (int j = 0; j < 3; ++j) {
                const int w = ms.tri[3 * t + j];
                if (w != kv.first.first && w != kv.first.second) return w;
            }
            throw Error(-1, "invalid triangle");
        };
        h.btri.push_back(tp);
        h.btri.push_back(tm);
        h.bfree.push_back(v[opposite(tp)]);
        h.bfree.push_back(v[opposite(tm)]);
        const double2 a = v[kv.first.first], b = v[kv.first.second];
        h.blen.push_back(std::sqrt((b.x - a.x) * (b.x - a.x) + (b.y - a.y) * (b.y - a.y)));
    }
    MBT_REQUIRE(h.M >= 1 && h.M <= kMaxBlockM, "the mesh must have 1..128 interior edges (RWG functions)");
    // gap bases: weight sign * length, the sign from the T+ -> T- direction along port_dir
    auto centroid = [&](int t) {
        return make_double2((h.tv[3 * t].x + h.tv[3 * t + 1].x + h.tv[3 * t + 2].x) / 3.0,
                            (h.tv[3 * t].y + h.tv[3 * t + 1].y + h.tv[3 * t + 2].y) / 3.0);
    };
    h.port.n = ms.nport_edges;
    for (int i = 0; i < ms.nport_edges; ++i) {
        const int a = ms.port_edges[2 * i], b = ms.port_edges[2 * i + 1];
        auto it = index.find({std::min(a, b), std::max(a, b)});
        MBT_REQUIRE(it != index.end(), "port edge is not an interior edge of the mesh");
        const int m = it->second;
        for (int j = 0; j < i; ++j) MBT_REQUIRE(h.port.idx[j] != m, "port edge listed twice");
        const double2 cp = centroid(h.btri[2 * m]), cm = centroid(h.btri[2 * m + 1]);
        const double proj = (cm.x - cp.x) * ms.port_dir[0] + (cm.y - cp.y) * ms.port_dir[1];
        MBT_REQUIRE(proj != 0.0, "port edge parallel to port_dir");
        h.port.idx[i] = m;
        h.port.w[i] = (proj > 0 ? 1.0 : -1.0) * h.blen[m];
    }
    // Radon's seven-point rule: the centroid and two orbits of three points
    const double r15 = std::sqrt(15.0);
    const double a1 = (6.0 - r15) / 21.0, a2 = (6.0 + r15) / 21.0;
    const double w0 = 9.0 / 40.0, w1 = (155.0 - r15) / 1200.0, w2 = (155.0 + r15) / 1200.0;
    const double bary[kRwgQ][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                                   {1.0 - 2.0 * a1, a1, a1}, {a1, 1.0 - 2.0 * a1, a1}, {a1, a1, 1.0 - 2.0 * a1},
                                   {1.0 - 2.0 * a2, a2, a2}, {a2, 1.0 - 2.0 * a2, a2}, {a2, a2, 1.0 - 2.0 * a2}};
    const double wts[kRwgQ] = {w0, w1, w1, w1, w2, w2, w2};
    h.qp.resize((size_t)nt * kRwgQ);
    h.qw.resize((size_t)nt * kRwgQ);
    for (int t = 0; t < nt; ++t)
        for (int i = 0; i < kRwgQ; ++i) {
            double x = 0, y = 0;
            for (int j = 0; j < 3; ++j) {
                x += bary[i][j] * h.tv[3 * t + j].x;
                y += bary[i][j] * h.tv[3 * t + j].y;
            }
            h.qp[(size_t)t * kRwgQ + i] = make_double2(x, y);
            h.qw[(size_t)t * kRwgQ + i] = wts[i] * h.area[t];
        }
    return h;
}

void rwg_fill_blocks(const Geom& g, const RwgMesh& h, double k, double2* T, hipStream_t s) {
    const int nt = h.nt, M = h.M;
    MBT_REQUIRE(M == g.M, "mesh and geometry disagree on the number of bases");
    // triangle centroids and each free vertex relative to its triangle's centroid
    std::vector<double2> tcen(nt), bdel(2 * (size_t)M);
    for (int t = 0; t < nt; ++t)
        tcen[t] = make_double2((h.tv[3 * t].x + h.tv[3 * t + 1].x + h.tv[3 * t + 2].x) / 3.0,
                               (h.tv[3 * t].y + h.tv[3 * t + 1].y + h.tv[3 * t + 2].y) / 3.0);
    for (int i = 0; i < 2 * M; ++i)
        bdel[i] = make_double2(h.bfree[i].x - tcen[h.btri[i]].x, h.bfree[i].y - tcen[h.btri[i]].y);
    // one upload of the mesh tables, laid out back to back
    const size_t b_qp = sizeof(double2) * h.qp.size(), b_qw = sizeof(double) * h.qw.size();
    const size_t b_tv = sizeof(double2) * h.tv.size(), b_ar = sizeof(double) * h.area.size();
    const size_t b_tc = sizeof(double2) * tcen.size(), b_bt = sizeof(int) * h.btri.size();
    const size_t b_bf = sizeof(double2) * h.bfree.size(), b_bd = sizeof(double2) * bdel.size();
    const size_t b_bl = sizeof(double) * h.blen.size();
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    DBuf buf;
    buf.alloc(up(b_qp) + up(b_qw) + up(b_tv) + up(b_ar) + up(b_tc) + up(b_bt) + up(b_bf) + up(b_bd) + up(b_bl));
    char* p = buf.as<char>();
    RwgDev d;
    auto put = [&](const void* src, size_t b) {
        char* dst = p;
        MBT_HIP(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s));
        p += up(b);
        return dst;
    };
    d.qp = reinterpret_cast<const double2*>(put(h.qp.data(), b_qp));
    d.qw = reinterpret_cast<const double*>(put(h.qw.data(), b_qw));
    d.tv = reinterpret_cast<const double2*>(put(h.tv.data(), b_tv));
    d.area = reinterpret_cast<const double*>(put(h.area.data(), b_ar));
    d.tcen = reinterpret_cast<const double2*>(put(tcen.data(), b_tc));
    d.btri = reinterpret_cast<const int*>(put(h.btri.data(), b_bt));
    d.bfree = reinterpret_cast<const double2*>(put(h.bfree.data(), b_bf));
    d.bdel = reinterpret_cast<const double2*>(put(bdel.data(), b_bd));
    d.blen = reinterpret_cast<const double*>(put(h.blen.data(), b_bl));
    // source triangles per chunk: the chunk's pair moments fit the LDS allowance
    const int U = std::max(1, std::min(nt, kPairLdsBytes / (nt * kPairVals * (int)sizeof(double2))));
    const size_t lds = sizeof(double2) * (size_t)nt * U * kPairVals;
    hipLaunchKernelGGL(rwg_fill_kernel, dim3((unsigned)g.noff()), dim3(256), lds, s, d, nt, M, U, g.nx, g.ny, g.dx,
                       g.dy, k, T);
    MBT_LAUNCH_CHECK();
    hipLaunchKernelGGL(rwg_mirror_kernel, dim3((unsigned)g.noff(), (unsigned)M), dim3(128), 0, s, M, g.nx, g.ny, T);
    MBT_LAUNCH_CHECK();
    // the tables are freed when this returns: wait for the kernel
    MBT_HIP(hipStreamSynchronize(s));
}

}  // namespace mbt

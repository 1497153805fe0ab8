// Block-diagonal preconditioners.
//
// Normal-equation strategy (paper Sec. III-A, eq. (precondA)): the diagonal
// M x M blocks of Z^H Z,
//     [P]_ee = sum_j Z_{je}^H Z_{je} = sum over offsets d in window(e) of T[d]^H T[d],
// built as the paper suggests: all products G[d] = T[d]^H T[d] first (one per
// unique offset), then the subset sum over the offsets d = j - e that element e
// sees inside the lattice.  P is Hermitian positive definite and is Cholesky
// factorised, P = L L^H (Sec. III-A); the apply uses the explicit inverse
// L^{-H} L^{-1}, a batched block product.
//
// Element-block strategy: P_K = blkdiag(T[0]) (the self block, identical for
// all elements), LU with partial pivoting, explicit inverse.
#include "common.h"

namespace mbt {

namespace {

// G[d][p][q] = sum_r conj(T[d][r][p]) T[d][r][q]
__global__ void gram_kernel(const double2* __restrict__ T, double2* __restrict__ G, int M, int64_t noff) {
    const int64_t MM = (int64_t)M * M;
    const int64_t total = noff * MM;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = t / MM;
        const int p = (int)((t % MM) / M), q = (int)(t % M);
        const double2* Td = T + d * MM;
        double sr = 0, si = 0;
        for (int r = 0; r < M; ++r) {
            const double2 a = Td[r * M + p], b = Td[r * M + q];
            sr += a.x * b.x + a.y * b.y;
            si += a.x * b.y - a.y * b.x;
        }
        G[t] = make_double2(sr, si);
    }
}

// P_e[p][q] = sum over elements j of G[j - e][p][q]
__global__ void window_kernel(const double2* __restrict__ G, double2* __restrict__ Pb, int nx, int ny, int M) {
    const int64_t MM = (int64_t)M * M;
    const int64_t total = (int64_t)nx * ny * MM;
    const int nox = 2 * nx - 1;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / MM;
        const int64_t pq = t % MM;
        const int ex = (int)(e % nx), ey = (int)(e / nx);
        double sr = 0, si = 0;
        for (int jy = 0; jy < ny; ++jy) {
            const int oy = jy - ey + ny - 1;
            for (int jx = 0; jx < nx; ++jx) {
                const int ox = jx - ex + nx - 1;
                const double2 v = G[((int64_t)oy * nox + ox) * MM + pq];
                sr += v.x;
                si += v.y;
            }
        }
        Pb[t] = make_double2(sr, si);
    }
}

constexpr int kMaxInvM = 32;

// One workgroup per block.  Cholesky A = L L^H, then A^{-1} = L^{-H} L^{-1}.
__global__ __launch_bounds__(256) void inv_hpd_kernel(const double2* __restrict__ A, double2* __restrict__ Ainv, int M,
                                                      int* __restrict__ info) {
    __shared__ double2 L[kMaxInvM * kMaxInvM];
    __shared__ double2 Li[kMaxInvM * kMaxInvM];
    __shared__ int bad;
    const int64_t b = blockIdx.x;
    const double2* Ab = A + b * (int64_t)M * M;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) bad = 0;
    for (int i = tid; i < M * M; i += nt) L[i] = Ab[i];
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        if (tid == 0) {
            const double djj = L[j * M + j].x;
            if (!(djj > 0.0)) bad = 1;
            L[j * M + j] = make_double2(sqrt(djj > 0.0 ? djj : 1.0), 0.0);
        }
        __syncthreads();
        const double dinv = 1.0 / L[j * M + j].x;
        for (int i = j + 1 + tid; i < M; i += nt) L[i * M + j] = make_double2(L[i * M + j].x * dinv, L[i * M + j].y * dinv);
        __syncthreads();
        // trailing update of the lower triangle: L[i][k] -= L[i][j] conj(L[k][j]), j < k <= i
        const int rem = M - j - 1;
        for (int t = tid; t < rem * rem; t += nt) {
            const int i = j + 1 + t / rem, k = j + 1 + t % rem;
            if (k <= i) {
                const double2 a = L[i * M + j], c = L[k * M + j];
                double2 v = L[i * M + k];
                v.x -= a.x * c.x + a.y * c.y;
                v.y -= a.y * c.x - a.x * c.y;
                L[i * M + k] = v;
            }
        }
        __syncthreads();
    }
    // Li = L^{-1}: forward substitution, one column per thread
    for (int c = tid; c < M; c += nt) {
        for (int i = 0; i < M; ++i) {
            double sr = (i == c) ? 1.0 : 0.0, si = 0.0;
            for (int k = c; k < i; ++k) {
                const double2 l = L[i * M + k], x = Li[k * M + c];
                sr -= l.x * x.x - l.y * x.y;
                si -= l.x * x.y + l.y * x.x;
            }
            const double dinv = 1.0 / L[i * M + i].x;
            Li[i * M + c] = (i < c) ? make_double2(0, 0) : make_double2(sr * dinv, si * dinv);
        }
    }
    __syncthreads();
    double2* Ob = Ainv + b * (int64_t)M * M;
    for (int t = tid; t < M * M; t += nt) {
        const int p = t / M, q = t % M;
        double sr = 0, si = 0;
        for (int k = (p > q ? p : q); k < M; ++k) {   // Li is lower: Li[k][p] = 0 for k < p
            const double2 a = Li[k * M + p], c = Li[k * M + q];
            sr += a.x * c.x + a.y * c.y;
            si += a.x * c.y - a.y * c.x;
        }
        Ob[t] = make_double2(sr, si);
    }
    if (tid == 0 && info) info[b] = bad;
}

// Larger blocks (32 < M <= 128; one M x M complex block no longer fits the LDS
// next to its factor): one workgroup per block factorises its block in place in
// global memory (A is overwritten with L), then each thread forms one column of
// A^{-1} by the forward substitution L y = e_c and the back substitution
// L^H x = y.  The workgroup's waves share one CU, so its global stores are
// visible to its other waves after each barrier.
__global__ __launch_bounds__(256) void inv_hpd_global_kernel(double2* __restrict__ A, double2* __restrict__ Ainv,
                                                             int M, int* __restrict__ info) {
    __shared__ int bad;
    const int64_t b = blockIdx.x;
    double2* L = A + b * (int64_t)M * M;
    double2* Ob = Ainv + b * (int64_t)M * M;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        if (tid == 0) {
            const double djj = L[j * M + j].x;
            if (!(djj > 0.0)) bad = 1;
            L[j * M + j] = make_double2(sqrt(djj > 0.0 ? djj : 1.0), 0.0);
        }
        __syncthreads();
        const double dinv = 1.0 / L[j * M + j].x;
        for (int i = j + 1 + tid; i < M; i += nt) L[i * M + j] = make_double2(L[i * M + j].x * dinv, L[i * M + j].y * dinv);
        __syncthreads();
        const int rem = M - j - 1;
        for (int t = tid; t < rem * rem; t += nt) {
            const int i = j + 1 + t / rem, k = j + 1 + t % rem;
            if (k <= i) {
                const double2 a = L[i * M + j], c = L[k * M + j];
                double2 v = L[i * M + k];
                v.x -= a.x * c.x + a.y * c.y;
                v.y -= a.y * c.x - a.x * c.y;
                L[i * M + k] = v;
            }
        }
        __syncthreads();
    }
    for (int c = tid; c < M; c += nt) {
        // L y = e_c (y_i = 0 for i < c), y kept in column c of the output
        for (int i = 0; i < M; ++i) {
            double sr = (i == c) ? 1.0 : 0.0, si = 0.0;
            for (int k = c; k < i; ++k) {
                const double2 l = L[i * M + k], y = Ob[k * M + c];
                sr -= l.x * y.x - l.y * y.y;
                si -= l.x * y.y + l.y * y.x;
            }
            const double dinv = 1.0 / L[i * M + i].x;
            Ob[i * M + c] = (i < c) ? make_double2(0, 0) : make_double2(sr * dinv, si * dinv);
        }
        // L^H x = y, x over y in place (row i of L^H is the conjugated column i of L)
        for (int i = M - 1; i >= 0; --i) {
            double2 acc = Ob[i * M + c];
            for (int k = i + 1; k < M; ++k) {
                const double2 l = L[k * M + i], x = Ob[k * M + c];
                acc.x -= l.x * x.x + l.y * x.y;
                acc.y -= l.x * x.y - l.y * x.x;
            }
            const double dinv = 1.0 / L[i * M + i].x;
            Ob[i * M + c] = make_double2(acc.x * dinv, acc.y * dinv);
        }
    }
    if (tid == 0 && info) info[b] = bad;
}

// One workgroup per block: Gauss-Jordan inversion with partial pivoting (the
// LU factorisation and both triangular solves in one sweep).
__global__ __launch_bounds__(256) void inv_lu_kernel(const double2* __restrict__ A, double2* __restrict__ Ainv, int M,
                                                     int* __restrict__ info) {
    __shared__ double2 W[kMaxInvM * kMaxInvM];
    __shared__ double2 col[kMaxInvM];
    __shared__ int piv[kMaxInvM];
    __shared__ int bad;
    const int64_t b = blockIdx.x;
    const double2* Ab = A + b * (int64_t)M * M;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) bad = 0;
    for (int i = tid; i < M * M; i += nt) W[i] = Ab[i];
    __syncthreads();
    for (int k = 0; k < M; ++k) {
        if (tid == 0) {
            int pr = k;
            double best = -1.0;
            for (int i = k; i < M; ++i) {
                const double2 v = W[i * M + k];
                const double m = v.x * v.x + v.y * v.y;
                if (m > best) { best = m; pr = i; }
            }
            piv[k] = pr;
            if (!(best > 0.0)) bad = 1;
        }
        __syncthreads();
        const int pr = piv[k];
        if (pr != k)
            for (int j = tid; j < M; j += nt) {
                const double2 t = W[k * M + j];
                W[k * M + j] = W[pr * M + j];
                W[pr * M + j] = t;
            }
        __syncthreads();
        const double2 d = W[k * M + k];
        const double den = d.x * d.x + d.y * d.y;
        const double2 dinv = den > 0.0 ? make_double2(d.x / den, -d.y / den) : make_double2(0, 0);
        __syncthreads();
        for (int j = tid; j < M; j += nt) {
            const double2 v = (j == k) ? make_double2(1.0, 0.0) : W[k * M + j];
            W[k * M + j] = cmul(v, dinv);
        }
        for (int i = tid; i < M; i += nt) col[i] = (i == k) ? make_double2(0, 0) : W[i * M + k];
        __syncthreads();
        for (int t = tid; t < M * M; t += nt) {
            const int i = t / M, j = t % M;
            if (i != k) {
                const double2 base = (j == k) ? make_double2(0, 0) : W[t];
                W[t] = csub(base, cmul(col[i], W[k * M + j]));
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int k = M - 1; k >= 0; --k) {
        const int pr = piv[k];
        if (pr != k)
            for (int i = tid; i < M; i += nt) {
                const double2 t = W[i * M + k];
                W[i * M + k] = W[i * M + pr];
                W[i * M + pr] = t;
            }
        __syncthreads();
    }
    double2* Ob = Ainv + b * (int64_t)M * M;
    for (int t = tid; t < M * M; t += nt) Ob[t] = W[t];
    if (tid == 0 && info) info[b] = bad;
}

}  // namespace

void gram_blocks(const Geom& g, const double2* T, double2* G, hipStream_t s) {
    hipLaunchKernelGGL(gram_kernel, dim3(2048), dim3(256), 0, s, T, G, g.M, g.noff());
    MBT_LAUNCH_CHECK();
}

void window_sum(const Geom& g, const double2* G, double2* Pb, hipStream_t s) {
    hipLaunchKernelGGL(window_kernel, dim3(2048), dim3(256), 0, s, G, Pb, g.nx, g.ny, g.M);
    MBT_LAUNCH_CHECK();
}

void batched_inverse_hpd_inplace(double2* A, double2* Ainv, int M, int64_t nbatch, int* info, hipStream_t s) {
    MBT_REQUIRE(M >= 1 && M <= kMaxBlockM, "batched_inverse_hpd_inplace: block size out of range");
    if (nbatch <= 0) return;
    if (M <= kMaxInvM)
        hipLaunchKernelGGL(inv_hpd_kernel, dim3((unsigned)nbatch), dim3(256), 0, s, A, Ainv, M, info);
    else
        hipLaunchKernelGGL(inv_hpd_global_kernel, dim3((unsigned)nbatch), dim3(256), 0, s, A, Ainv, M, info);
    MBT_LAUNCH_CHECK();
}

void batched_inverse(const double2* A, double2* Ainv, int M, int64_t nbatch, bool hpd, int* info, hipStream_t s) {
    MBT_REQUIRE(M >= 1 && M <= kMaxInvM, "batched_inverse: block size out of range");
    if (nbatch <= 0) return;
    if (hpd)
        hipLaunchKernelGGL(inv_hpd_kernel, dim3((unsigned)nbatch), dim3(256), 0, s, A, Ainv, M, info);
    else
        hipLaunchKernelGGL(inv_lu_kernel, dim3((unsigned)nbatch), dim3(256), 0, s, A, Ainv, M, info);
    MBT_LAUNCH_CHECK();
}

}  // namespace mbt

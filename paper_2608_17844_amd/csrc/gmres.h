// Batched GMRES driver interface and the device arena it allocates from (internal).
#pragma once

#include <functional>
#include <vector>

#include "common.h"

namespace mbt {

// Bump allocator over one device buffer; reset per solve.  No hipMalloc inside.
struct DevArena {
    char* base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    template <typename T> T* get(size_t count) {
        const size_t bytes = ((sizeof(T) * count) + 255) & ~(size_t)255;
        if (off + bytes > cap) throw Error(-2, "device workspace exhausted (internal sizing error)");
        T* p = reinterpret_cast<T*>(base + off);
        off += bytes;
        return p;
    }
};

// Per-RHS recurrence state, passed by value to kernels.
struct GmresState {
    double tol;
    double2* H;      // [m][m+1][R]  column j, row i
    double* cs;      // [m][R]
    double2* sn;     // [m][R]
    double2* g;      // [m+1][R]
    double* bnorm;   // [R]
    double* beta;    // [R]
    double* scale;   // [R]  1/||w|| for the next basis vector, 0 if the RHS stopped
    int* active;     // [R]  iterating in this cycle
    int* conv;       // [R]  met the tolerance (decided on the explicit residual at a restart)
    int* cand;       // [R]  the least-squares residual met the tolerance in the last cycle
    int* flag;       // [R]  non-finite value met
    int* kcyc;       // [R]  Arnoldi steps in this cycle
    int* iters;      // [R]  Arnoldi steps in total
};

struct GmresParams {
    int restart = 50;
    double tol = 1e-10;
    int max_cycles = 400;
    int matvecs_per_apply = 1;
    bool dcgs2 = true;           // delayed reorthogonalisation (two sweeps); false: classical CGS2 (three)
    bool packed_basis = false;   // FP32 solves with DCGS2, even R, restart >= 4: basis in the packed 24-bit format
    int* host_count = nullptr;   // pinned host int for the active-count readback
};

struct GmresResult {
    std::vector<int> iters, conv, flag;
    int cycles = 0;
    int64_t matvecs = 0;
};

int64_t gmres_rows_per_chunk(int64_t N);
int gmres_nchunk(int64_t N);
size_t gmres_state_bytes(int64_t N, int R, int m);

// Solves A x = b for R independent columns (b, basis of type TB = double2 or
// float2; x accumulated in FP64).  Vbasis holds (restart+1) vectors of N x R of
// type TB (with a packed basis it holds two TB work vectors and the packed
// vectors instead, in no more space).
template <typename TB>
GmresResult gmres_batched(const std::function<void(const TB*, TB*)>& apply, const TB* b, double2* x, TB* Vbasis,
                          int64_t N, int R, const GmresParams& prm, DevArena& arena, hipStream_t s);

// Batched preconditioned conjugate gradients for N x = b (N Hermitian positive
// definite: the normal equations Z^H Z), P^{-1} applied by applyPinv; x0 = 0;
// stop on sqrt(r^H P^{-1} r / b^H P^{-1} b) <= tol per RHS (the residual of the
// split system P^{-1/2} N P^{-H/2} w = P^{-1/2} b).  work holds 4 N x R vectors
// of type TB; at most maxit iterations.  cycles is 1, matvecs counts Z and Z^H.
// Batched COCG on complex symmetric Z with a complex symmetric preconditioner
// (x = 0 start, stop at ||r|| <= tol ||b||); work: four N x R vectors of TB.
size_t cocg_state_bytes(int64_t N, int R);
template <typename TB>
GmresResult cocg_batched(const std::function<void(const TB*, TB*)>& applyZ,
                         const std::function<void(const TB*, TB*)>& applyMinv, const TB* b, double2* x, TB* work,
                         int64_t N, int R, double tol, int maxit, int* host_count, DevArena& arena, hipStream_t s);

size_t pcg_state_bytes(int64_t N, int R);
template <typename TB>
GmresResult pcg_batched(const std::function<void(const TB*, TB*)>& applyN,
                        const std::function<void(const TB*, TB*)>& applyPinv, const TB* b, double2* x, TB* work,
                        int64_t N, int R, double tol, int maxit, int* host_count, DevArena& arena, hipStream_t s);


}  // namespace mbt

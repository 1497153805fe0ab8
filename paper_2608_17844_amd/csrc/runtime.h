// Host runtime objects shared by the C-ABI entry points and the server (internal).
#pragma once

#include <chrono>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mbt.h"
#include "common.h"
#include "gmres.h"
#include "rwg.h"

namespace mbt {

// Owning device buffer (hipMalloc / hipFree on the owner's device).
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b) {
            hipError_t e = hipMalloc(&p, b);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Error(-2, "hipMalloc of " + std::to_string(b) + " bytes failed");
            }
            bytes = b;
        }
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Per (geometry, frequency) device data: blocks, their spectra, preconditioner inverses.
struct OpData {
    Geom g;
    double s = 0, k = 0;
    DBuf T, Chat, tw, PkInv, PaInv;            // FP64
    DBuf ChatK;                                // P_K^{-1} C^_b per bin: the element-block preconditioned operator
    DBuf Chat32, tw32, PkInv32, PaInv32;       // FP32 copies for reduced-precision inner solves
    DBuf ChatK32;
    DBuf Chat16[2];                            // 16-bit spectra (bfloat16, binary16) for the 16-bit products,
    double scale16[2] = {1.0, 1.0};            // stored as scale16 * C^ (a power of two)
    // margin blocks (Nc > 0): Z_B (Nc x P*M) and Z_C (Nc x Nc) row-major, the margin's preconditioner
    // blocks P_C^{-1} (normal equations) and Z_C^{-1} (element blocks), and their FP32 copies
    DBuf ZB, ZC, PcInv, ZcInv, ZB32, ZC32, PcInv32, ZcInv32;
    bool has_pa = false, has32 = false;
    size_t bytes() const {
        return T.bytes + Chat.bytes + ChatK.bytes + tw.bytes + PkInv.bytes + PaInv.bytes + Chat32.bytes +
               ChatK32.bytes + tw32.bytes + PkInv32.bytes + PaInv32.bytes + Chat16[0].bytes + Chat16[1].bytes +
               ZB.bytes + ZC.bytes + PcInv.bytes + ZcInv.bytes + ZB32.bytes + ZC32.bytes + PcInv32.bytes +
               ZcInv32.bytes;
    }
};

// A stream with its own persistent device buffers; the context has one, each
// server slot another.  ws holds the solve workspace, xs the extraction
// buffers; both only grow (a grown buffer is reused by later calls, so steady
// state issues no device allocation or free).
struct Worker {
    int device = 0;
    hipStream_t stream = nullptr;
    DBuf ws, xs;
    int* host_count = nullptr;   // pinned
    explicit Worker(int dev);
    ~Worker();
    void ensure(size_t bytes);
    void ensure_x(size_t bytes);
    size_t held() const { return ws.bytes + xs.bytes; }
    // size a buffer grows to when `need` bytes are requested
    static size_t grown(size_t have, size_t need) { return have >= need ? have : need + (need >> 4); }
};

struct SolveOut {
    std::vector<int> iters;
    std::vector<char> conv, flag;   // per RHS
    int cycles = 0, outer = 0, nconv = 0, nflag = 0;
    int64_t matvecs = 0;
    double relres_max = 0;
};

}  // namespace mbt

struct mbt_array {
    mbt::Geom g;
    mbt_dipole elem;
    mbt_lattice lat;
    // arrays defined by caller-supplied unique blocks (no element fill): host copy
    // of T[dy][dx][p][q] and an identity for the operator cache
    std::shared_ptr<const std::vector<double2>> blocks;
    // partitioned operators: margin blocks Z_B (Nc x P*M) and Z_C (Nc x Nc), row-major host copies
    std::shared_ptr<const std::vector<double2>> zb, zc;
    // planar elements: RWG functions of the element mesh (filled per frequency)
    std::shared_ptr<const mbt::RwgMesh> rwg;
    uint64_t uid = 0;
};

struct mbt_ctx {
    int device = 0;
    size_t budget = 0;
    std::unique_ptr<mbt::Worker> main;
    std::mutex cache_mu;
    std::map<std::string, std::shared_ptr<mbt::OpData>> cache;
    std::list<std::string> lru;
    size_t cache_bytes = 0, cache_limit = 0;
    std::mutex api_mu;   // serialises entry points that use the context's own worker
};

namespace mbt {

Geom make_geom(const mbt_dipole& d, const mbt_lattice& l);
// Geometry of a block-defined lattice operator (nx x ny elements, M bases each).
Geom make_geom_blocks(int nx, int ny, int M);
void validate_opts(const mbt_solve_opts& o);
// Cached operator data; need_pa adds the normal-equation preconditioner, prec
// adds the copies that a reduced-precision inner solve reads.
std::shared_ptr<OpData> get_op(mbt_ctx* ctx, const mbt_array* arr, double s, bool need_pa, int prec, Worker& wk);
// 16-bit storage format of a precision (kFmtNone for FP64 and FP32).
int fmt16_of(int prec);
size_t solve_bytes(const Geom& g, int R, const mbt_solve_opts& o);
// Largest RHS batch (<= R) whose solve workspace fits `budget` bytes.
int choose_chunk(size_t budget, const Geom& g, int R, const mbt_solve_opts& o);
// columns actually solved for a batch of R ports (reduced precision with the
// packed basis repeats the last port of an odd batch)
int padded(int R, const mbt_solve_opts& o);
// Device bytes of the extraction buffers of one frequency (Y_p, Z_p, S, work, scans).
size_t extract_bytes(int P, int nscan);
// Solves Z X = V for R device columns (layout [n][r]); X receives FP64 currents.
SolveOut solve_rhs(const OpData& op, const mbt_solve_opts& o, const double2* V, int R, double2* X, Worker& wk,
                   DevArena& arena);
// All-port solve for one frequency; Ydev (P x nports column-major) filled on the device.
SolveOut admittance(mbt_ctx* ctx, const mbt_array* arr, double s, const int32_t* ports, int nports,
                    const mbt_solve_opts& o, double2* Ydev, Worker& wk, mbt_stats* st, size_t budget);
// The whole path for one frequency on worker wk: all-port solve, Z_p = Y_p^{-1},
// S and the center-element scan quantities; outputs are host arrays (any may
// be NULL except when nscan > 0, where Za and Gamma are required).
SolveOut solve_frequency(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts& o, size_t budget,
                         const double* theta, const double* phi, int nscan, double z0, double* Zp, double* Za,
                         double* Gamma, double* Gamma_wave, Worker& wk, mbt_stats* st);
// Status of a finished solve (MBT_OK, MBT_ENOCONV or MBT_EBREAKDOWN).
int solve_status(const SolveOut& so);
// Sets the calling thread's message returned by mbt_last_error.
void set_last_error(const std::string& m);

}  // namespace mbt

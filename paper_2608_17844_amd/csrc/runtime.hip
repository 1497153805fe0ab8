// C-ABI entry points and the host runtime: contexts, the per-(array, frequency)
// operator cache, the batched solve drivers (FP64, and reduced precision with
// FP64 iterative refinement), port extraction and the test hooks.
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <sstream>

#include "extract.h"

using namespace mbt;

namespace {

thread_local std::string g_err;

mbt_status set_err(int code, const std::string& m) {
    g_err = m;
    return (mbt_status)code;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void mbt::set_last_error(const std::string& m) { g_err = m; }

#define API_BEGIN \
    g_err.clear(); \
    try {
#define API_END                                                                    \
    }                                                                              \
    catch (const mbt::Error& e) { return set_err(e.code, e.what()); }              \
    catch (const std::bad_alloc&) { return set_err(MBT_ENOMEM, "host allocation failed"); } \
    catch (const std::exception& e) { return set_err(MBT_EDEVICE, e.what()); }     \
    return MBT_OK;

// ------------------------------------------------------------------ allocation-free entry point
// Device scratch of mbt_active_dev_noalloc: the S-matrix work (Z_p + z0, its
// inverse, the pivot search column and pivot arrays) for up to 1024 ports.
// Each GPU the library runs on holds one copy until the process ends; host code
// refers to it only through the per-device address taken at context creation
// (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) char scratch[MBT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// With device `dev` current: record the address of its copy of the scratch array.
void noalloc_scratch_setup(int dev) {
    MBT_REQUIRE(dev < kMaxDevices, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void* p = nullptr;
    MBT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MBT_REQUIRE(p != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<char*>(p);
}

char* noalloc_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

// bytes of scratch the S-matrix work of P ports takes (256-byte aligned pieces)
size_t noalloc_need(int P) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 2 * al(sizeof(double2) * (size_t)P * P) + al(sizeof(double2) * (size_t)P) + 2 * al(sizeof(int) * (size_t)P) +
           al(sizeof(int));
}
}  // namespace

namespace mbt {

// ------------------------------------------------------------------ workers
Worker::Worker(int dev) : device(dev) {
    MBT_HIP(hipSetDevice(dev));
    MBT_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    MBT_HIP(hipHostMalloc((void**)&host_count, sizeof(int) * 16, hipHostMallocDefault));
}

Worker::~Worker() {
    (void)hipSetDevice(device);
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
    ws.release();
    if (host_count) (void)hipHostFree(host_count);
}

void Worker::ensure(size_t bytes) {
    if (ws.bytes >= bytes) return;
    MBT_HIP(hipStreamSynchronize(stream));
    ws.alloc(grown(0, bytes));
}

void Worker::ensure_x(size_t bytes) {
    if (xs.bytes >= bytes) return;
    MBT_HIP(hipStreamSynchronize(stream));
    xs.alloc(grown(0, bytes));
}

// ------------------------------------------------------------------ geometry and options
static int pow2_at_least(int n, int lo) {
    int p = lo;
    while (p < n) p <<= 1;
    return p;
}

Geom make_geom(const mbt_dipole& d, const mbt_lattice& l) {
    MBT_REQUIRE(d.nbases >= 1 && d.nbases % 2 == 1, "nbases must be odd and >= 1");
    MBT_REQUIRE(d.nbases <= 32, "nbases above 32 is not supported");
    MBT_REQUIRE(d.radius > 0 && d.length > 0 && std::isfinite(d.radius) && std::isfinite(d.length),
                "dipole length and radius must be positive");
    MBT_REQUIRE(l.nx >= 1 && l.ny >= 1 && l.nx <= 64 && l.ny <= 64, "lattice size must be within 1..64 per axis");
    MBT_REQUIRE(l.dx > 0 && l.dy > 0 && std::isfinite(l.dx) && std::isfinite(l.dy), "lattice spacing must be positive");
    Geom g;
    g.nx = l.nx;
    g.ny = l.ny;
    g.M = d.nbases;
    g.dx = l.dx;
    g.dy = l.dy;
    g.L = d.length;
    g.a = d.radius;
    g.P = l.nx * l.ny;
    g.N = (int64_t)g.P * g.M;
    g.Lx = pow2_at_least(l.nx, 8);
    g.Ly = pow2_at_least(l.ny, 8);
    g.Px = 2 * g.Lx;
    g.Py = 2 * g.Ly;
    g.nox = 2 * l.nx - 1;
    g.noy = 2 * l.ny - 1;
    g.pc = (g.M - 1) / 2;
    g.port.idx[0] = g.pc;
    return g;
}

Geom make_geom_blocks(int nx, int ny, int M) {
    MBT_REQUIRE(M >= 1 && M <= kMaxBlockM, "nbases must be within 1..128 for a block-defined array");
    MBT_REQUIRE(nx >= 1 && ny >= 1 && nx <= 64 && ny <= 64, "lattice size must be within 1..64 per axis");
    Geom g;
    g.nx = nx;
    g.ny = ny;
    g.M = M;
    g.dx = g.dy = 0.5;   // nominal: the blocks carry the geometry
    g.P = nx * ny;
    g.N = (int64_t)g.P * g.M;
    g.Lx = pow2_at_least(nx, 8);
    g.Ly = pow2_at_least(ny, 8);
    g.Px = 2 * g.Lx;
    g.Py = 2 * g.Ly;
    g.nox = 2 * nx - 1;
    g.noy = 2 * ny - 1;
    g.pc = (M - 1) / 2;
    g.port.idx[0] = g.pc;
    return g;
}

void validate_opts(const mbt_solve_opts& o) {
    MBT_REQUIRE(o.prec == MBT_FP64 || o.prec == MBT_FP32 || o.prec == MBT_BF16 || o.prec == MBT_FP16,
                "unknown precision");
    MBT_REQUIRE(o.pc == MBT_PC_NORMAL_EQ || o.pc == MBT_PC_ELEMENT_BLOCK, "unknown preconditioner");
    MBT_REQUIRE(o.restart >= 1 && o.restart <= 63, "restart must be in 1..63");
    MBT_REQUIRE(o.tol > 0 && o.tol < 1, "tol must be in (0, 1)");
    MBT_REQUIRE(o.max_cycles >= 1, "max_cycles must be >= 1");
    MBT_REQUIRE(o.prec == MBT_FP64 || (o.refine_max >= 1 && o.refine_tol > 0), "refinement options invalid");
    MBT_REQUIRE(o.rhs_chunk >= 0, "rhs_chunk must be >= 0");
    MBT_REQUIRE((o.flags & ~(MBT_FLAG_NO_CACHE | MBT_FLAG_CGS2 | MBT_FLAG_FP32_BASIS | MBT_FLAG_PCG |
                             MBT_FLAG_COCG)) == 0,
                "unknown flags");
    MBT_REQUIRE(!(o.flags & MBT_FLAG_PCG) || o.pc == MBT_PC_NORMAL_EQ,
                "PCG solves the normal equations: pc must be MBT_PC_NORMAL_EQ");
    MBT_REQUIRE(!(o.flags & MBT_FLAG_COCG) || o.pc == MBT_PC_ELEMENT_BLOCK,
                "COCG takes the complex symmetric P_K: pc must be MBT_PC_ELEMENT_BLOCK");
    MBT_REQUIRE(!((o.flags & MBT_FLAG_COCG) && (o.flags & MBT_FLAG_PCG)), "PCG and COCG exclude each other");
}

static double inner_tol(const mbt_solve_opts& o) {
    if (o.inner_tol > 0) return o.inner_tol;
    return o.prec == MBT_FP32 ? 1e-4 : o.prec == MBT_FP16 ? 1e-3 : 1e-2;
}

int fmt16_of(int prec) { return prec == MBT_BF16 ? kFmtBf16 : prec == MBT_FP16 ? kFmtF16 : kFmtNone; }

// ------------------------------------------------------------------ operator cache
static std::string op_key(const mbt_array* arr, double s) {
    const Geom& g = arr->g;
    std::ostringstream os;
    os.precision(17);
    if (arr->blocks) os << "blocks#" << arr->uid << ',';
    if (arr->rwg) os << "rwg#" << arr->uid << ',';
    os << g.nx << ',' << g.ny << ',' << g.M << ',' << g.dx << ',' << g.dy << ',' << g.L << ',' << g.a << ',' << s;
    return os.str();
}

static void build_pa(OpData& op, Worker& wk) {
    const Geom& g = op.g;
    const int64_t MM = (int64_t)g.M * g.M;
    DBuf G, Pb, info;
    G.alloc(sizeof(double2) * g.noff() * MM);
    Pb.alloc(sizeof(double2) * g.P * MM);
    info.alloc(sizeof(int) * g.P);
    gram_blocks(g, op.T.as<double2>(), G.as<double2>(), wk.stream);
    window_sum(g, G.as<double2>(), Pb.as<double2>(), wk.stream);
    op.PaInv.alloc(sizeof(double2) * g.P * MM);
    batched_inverse_hpd_inplace(Pb.as<double2>(), op.PaInv.as<double2>(), g.M, g.P, info.as<int>(), wk.stream);
    std::vector<int> hi(g.P);
    MBT_HIP(hipMemcpyAsync(hi.data(), info.p, sizeof(int) * g.P, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    for (int v : hi) MBT_REQUIRE(v == 0, "normal-equation preconditioner block is not positive definite");
    if (g.Nc > 0) {
        // P_C = Z_B^* Z_B^T + Z_C^H Z_C (eq. (precond)), then its inverse
        const int nc = g.Nc;
        const int64_t NA = g.NA();
        DBuf Pc, part, work;
        Pc.alloc(sizeof(double2) * (size_t)nc * nc);
        part.alloc(sizeof(double2) * (size_t)margin_ksplit(NA) * nc * nc);
        work.alloc(sizeof(double2) * ((size_t)nc + 8) + sizeof(int) * ((size_t)nc + 8));
        // (Z_B^* Z_B^T)[i][j] = sum_k conj(Z_B[i][k]) Z_B[j][k]: X[k][j] = Z_B[j][k]
        margin_gemm<double>(op.ZB.as<double2>(), NA, 1, true, op.ZB.as<double2>(), 1, NA, Pc.as<double2>(), nc, nc, NA,
                            nc, false, part.as<double2>(), wk.stream);
        // (Z_C^H Z_C)[i][j] = sum_l conj(Z_C[l][i]) Z_C[l][j]
        margin_gemm<double>(op.ZC.as<double2>(), 1, nc, true, op.ZC.as<double2>(), nc, 1, Pc.as<double2>(), nc, nc, nc,
                            nc, true, nullptr, wk.stream);
        op.PcInv.alloc(sizeof(double2) * (size_t)nc * nc);
        double2* colbuf = work.as<double2>();
        int* piv = reinterpret_cast<int*>(colbuf + nc + 8);
        gj_inverse(Pc.as<double2>(), op.PcInv.as<double2>(), nc, colbuf, piv, piv + nc, wk.stream);
    }
    op.has_pa = true;
}

static void build_32(OpData& op, Worker& wk) {
    const Geom& g = op.g;
    const int64_t MM = (int64_t)g.M * g.M;
    op.Chat32.alloc(sizeof(float2) * g.bins() * MM);
    convert<double2, float2>(op.Chat.as<double2>(), op.Chat32.as<float2>(), g.bins() * MM, wk.stream);
    op.ChatK32.alloc(sizeof(float2) * g.bins() * MM);
    convert<double2, float2>(op.ChatK.as<double2>(), op.ChatK32.as<float2>(), g.bins() * MM, wk.stream);
    op.tw32.alloc(sizeof(float2) * (g.Px + g.Py));
    convert<double2, float2>(op.tw.as<double2>(), op.tw32.as<float2>(), g.Px + g.Py, wk.stream);
    op.PkInv32.alloc(sizeof(float2) * MM);
    convert<double2, float2>(op.PkInv.as<double2>(), op.PkInv32.as<float2>(), MM, wk.stream);
    if (g.Nc > 0) {
        const int64_t nb = (int64_t)g.Nc * g.NA(), nc2 = (int64_t)g.Nc * g.Nc;
        op.ZB32.alloc(sizeof(float2) * nb);
        convert<double2, float2>(op.ZB.as<double2>(), op.ZB32.as<float2>(), nb, wk.stream);
        op.ZC32.alloc(sizeof(float2) * nc2);
        convert<double2, float2>(op.ZC.as<double2>(), op.ZC32.as<float2>(), nc2, wk.stream);
        op.ZcInv32.alloc(sizeof(float2) * nc2);
        convert<double2, float2>(op.ZcInv.as<double2>(), op.ZcInv32.as<float2>(), nc2, wk.stream);
    }
    MBT_HIP(hipStreamSynchronize(wk.stream));
    op.has32 = true;
}

// FP32 copy of the normal-equation preconditioner inverses (needs build_pa first).
static void build_32_pa(OpData& op, Worker& wk) {
    const Geom& g = op.g;
    const int64_t MM = (int64_t)g.M * g.M;
    op.PaInv32.alloc(sizeof(float2) * g.P * MM);
    convert<double2, float2>(op.PaInv.as<double2>(), op.PaInv32.as<float2>(), g.P * MM, wk.stream);
    if (g.Nc > 0) {
        const int64_t nc2 = (int64_t)g.Nc * g.Nc;
        op.PcInv32.alloc(sizeof(float2) * nc2);
        convert<double2, float2>(op.PcInv.as<double2>(), op.PcInv32.as<float2>(), nc2, wk.stream);
    }
    MBT_HIP(hipStreamSynchronize(wk.stream));
}

// 16-bit copy of the block spectra, scaled by a power of two that puts the
// largest component at 2^14: binary16 then keeps its full relative precision
// over 2^28 of dynamic range below that (bfloat16 has FP32's range; the same
// exact scaling does no harm there).
static void build_16(OpData& op, int fmt, Worker& wk) {
    const Geom& g = op.g;
    const int64_t n = g.bins() * g.M * g.M;
    DBuf dmax;
    dmax.alloc(sizeof(double));
    max_abs_d(op.Chat.as<double2>(), n, dmax.as<double>(), wk.stream);
    double hmax = 0;
    MBT_HIP(hipMemcpyAsync(&hmax, dmax.p, sizeof(double), hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    MBT_REQUIRE(std::isfinite(hmax), "block spectra are not finite");
    const double scale = hmax > 0 ? std::ldexp(1.0, 14 - std::ilogb(hmax) - 1) : 1.0;
    op.Chat16[fmt].alloc(sizeof(uint32_t) * n);
    if (fmt == kFmtBf16)
        pack16_d<kFmtBf16>(op.Chat.as<double2>(), op.Chat16[fmt].as<uint32_t>(), n, scale, wk.stream);
    else
        pack16_d<kFmtF16>(op.Chat.as<double2>(), op.Chat16[fmt].as<uint32_t>(), n, scale, wk.stream);
    MBT_HIP(hipStreamSynchronize(wk.stream));
    op.scale16[fmt] = scale;
}

static std::shared_ptr<OpData> build_op(const mbt_array* arr, double s, Worker& wk) {
    const Geom& g = arr->g;
    auto op = std::make_shared<OpData>();
    op->g = g;
    op->s = s;
    op->k = 2.0 * M_PI * s;
    const int64_t MM = (int64_t)g.M * g.M;
    op->T.alloc(sizeof(double2) * g.noff() * MM);
    if (arr->blocks) {
        MBT_REQUIRE((int64_t)arr->blocks->size() == g.noff() * MM, "block array size mismatch");
        MBT_HIP(hipMemcpyAsync(op->T.p, arr->blocks->data(), op->T.bytes, hipMemcpyHostToDevice, wk.stream));
    } else if (arr->rwg) {
        rwg_fill_blocks(g, *arr->rwg, op->k, op->T.as<double2>(), wk.stream);
    } else {
        fill_blocks(g, op->k, op->T.as<double2>(), wk.stream);
    }
    op->Chat.alloc(sizeof(double2) * g.bins() * MM);
    {
        DBuf embed_work;
        embed_work.alloc(sizeof(double2) * ((int64_t)g.noy * g.Px * MM + g.Px + g.Py));
        embed_blocks_fft(g, op->T.as<double2>(), op->Chat.as<double2>(), 1.0 / (double)g.bins(), embed_work.as<double2>(),
                         wk.stream);
        MBT_HIP(hipStreamSynchronize(wk.stream));
    }
    op->tw.alloc(sizeof(double2) * (g.Px + g.Py));
    make_twiddles(g.Px, op->tw.as<double2>(), wk.stream);
    make_twiddles(g.Py, op->tw.as<double2>() + g.Px, wk.stream);
    // P_K: inverse of the self block (offset 0)
    op->PkInv.alloc(sizeof(double2) * MM);
    const int64_t center = (int64_t)(g.ny - 1) * g.nox + (g.nx - 1);
    if (g.M <= 32) {
        DBuf info;
        info.alloc(sizeof(int));
        batched_inverse(op->T.as<double2>() + center * MM, op->PkInv.as<double2>(), g.M, 1, false, info.as<int>(),
                        wk.stream);
        int hinfo = 0;
        MBT_HIP(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, wk.stream));
        MBT_HIP(hipStreamSynchronize(wk.stream));
        MBT_REQUIRE(hinfo == 0, "element self block is singular");
    } else {
        // larger blocks: the general Gauss-Jordan inverse on a copy of the self block
        DBuf work;
        work.alloc(sizeof(double2) * (MM + g.M) + sizeof(int) * (g.M + 8));
        double2* A = work.as<double2>();
        MBT_HIP(hipMemcpyAsync(A, op->T.as<double2>() + center * MM, sizeof(double2) * MM, hipMemcpyDeviceToDevice,
                               wk.stream));
        int* piv = reinterpret_cast<int*>(A + MM + g.M);
        gj_inverse(A, op->PkInv.as<double2>(), g.M, A + MM, piv, piv + g.M, wk.stream);
        MBT_HIP(hipStreamSynchronize(wk.stream));
    }
    if (g.Nc > 0) {
        MBT_REQUIRE(arr->zb && arr->zc, "margin blocks missing");
        const int nc = g.Nc;
        op->ZB.alloc(sizeof(double2) * (size_t)nc * g.NA());
        MBT_HIP(hipMemcpyAsync(op->ZB.p, arr->zb->data(), op->ZB.bytes, hipMemcpyHostToDevice, wk.stream));
        op->ZC.alloc(sizeof(double2) * (size_t)nc * nc);
        MBT_HIP(hipMemcpyAsync(op->ZC.p, arr->zc->data(), op->ZC.bytes, hipMemcpyHostToDevice, wk.stream));
        DBuf work;
        work.alloc(sizeof(double2) * ((size_t)nc * nc + nc + 8) + sizeof(int) * ((size_t)nc + 8));
        double2* A = work.as<double2>();
        MBT_HIP(hipMemcpyAsync(A, op->ZC.p, op->ZC.bytes, hipMemcpyDeviceToDevice, wk.stream));
        op->ZcInv.alloc(sizeof(double2) * (size_t)nc * nc);
        int* piv = reinterpret_cast<int*>(A + (size_t)nc * nc + nc + 8);
        gj_inverse(A, op->ZcInv.as<double2>(), nc, A + (size_t)nc * nc, piv, piv + nc, wk.stream);
        MBT_HIP(hipStreamSynchronize(wk.stream));
    }
    // P_K^{-1} acts on the basis index of every element alike, so it commutes with
    // the lattice transforms and the crop: P_K^{-1} Z x = crop F^{-1}((P_K^{-1} C^_b) X^_b).
    // Folding it into the spectra removes the preconditioner pass from each step.
    op->ChatK.alloc(sizeof(double2) * g.bins() * MM);
    cgemm_batched<double>(op->PkInv.as<double2>(), 0, op->Chat.as<double2>(), op->ChatK.as<double2>(), g.M, g.M,
                          g.bins(), 0, wk.stream);
    MBT_HIP(hipStreamSynchronize(wk.stream));
    return op;
}

std::shared_ptr<OpData> get_op(mbt_ctx* ctx, const mbt_array* arr, double s, bool need_pa, int prec, Worker& wk) {
    const bool need32 = prec != MBT_FP64;
    const int fmt = fmt16_of(prec);
    MBT_REQUIRE(s > 0 && std::isfinite(s), "freq_ratio must be positive");
    MBT_REQUIRE(fmt == kFmtNone || arr->g.M <= 32, "16-bit products support at most 32 bases per element");
    const std::string key = op_key(arr, s);
    std::shared_ptr<OpData> op;
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        auto it = ctx->cache.find(key);
        if (it != ctx->cache.end()) {
            op = it->second;
            ctx->lru.remove(key);
            ctx->lru.push_front(key);
        }
    }
    if (!op) {
        op = build_op(arr, s, wk);
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        auto it = ctx->cache.find(key);
        if (it != ctx->cache.end()) {
            op = it->second;   // another worker built it meanwhile
        } else {
            ctx->cache[key] = op;
            ctx->lru.push_front(key);
            ctx->cache_bytes += op->bytes();
        }
    }
    // Extend under the cache lock.  Every piece is built only where it is still
    // missing, into a buffer that did not exist before: other workers may be
    // running kernels on the pieces that exist, so nothing already built is
    // ever reallocated.  The flags and pointers are read under the same lock,
    // after the builder's stream has synchronised.
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        const size_t before = op->bytes();
        if (need_pa && !op->has_pa) build_pa(*op, wk);
        if (need32 && !op->has32) build_32(*op, wk);
        if (need32 && need_pa && !op->PaInv32.p) build_32_pa(*op, wk);
        if (fmt != kFmtNone && !op->Chat16[fmt].p) build_16(*op, fmt, wk);
        auto it = ctx->cache.find(key);
        if (it != ctx->cache.end() && it->second == op) ctx->cache_bytes += op->bytes() - before;
    }
    // evict least recently used entries beyond the limit (entries in use stay alive through shared_ptr)
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        while (ctx->cache_bytes > ctx->cache_limit && ctx->lru.size() > 1) {
            const std::string victim = ctx->lru.back();
            ctx->lru.pop_back();
            auto it = ctx->cache.find(victim);
            if (it != ctx->cache.end()) {
                ctx->cache_bytes -= it->second->bytes();
                ctx->cache.erase(it);
            }
        }
    }
    return op;
}

// A private operator with every piece the options need (MBT_FLAG_NO_CACHE): the
// same pieces get_op adds to a cached entry.
static std::shared_ptr<OpData> build_uncached(const mbt_array* arr, double s, const mbt_solve_opts& o, Worker& wk) {
    const int fmt = fmt16_of(o.prec);
    MBT_REQUIRE(fmt == kFmtNone || arr->g.M <= 32, "16-bit products support at most 32 bases per element");
    auto op = build_op(arr, s, wk);
    const bool pa = o.pc == MBT_PC_NORMAL_EQ;
    if (pa) build_pa(*op, wk);
    if (o.prec != MBT_FP64) {
        build_32(*op, wk);
        if (pa) build_32_pa(*op, wk);
    }
    if (fmt != kFmtNone) build_16(*op, fmt, wk);
    return op;
}

// ------------------------------------------------------------------ operator application
template <typename T> struct OpV {
    const Geom* g;
    const cplx<T>* Chat;
    const cplx<T>* ChatA = nullptr;      // spectra of the preconditioned operator, when P is folded in
    const cplx<T>* pinv;
    int64_t pstride;
    const cplx<T>* twx;
    const cplx<T>* twy;
    cplx<T>* Xh;
    cplx<T>* Yh;
    cplx<T>* tmp;
    int R;
    int pc;
    hipStream_t s;
    int fmt = kFmtNone;                  // 16-bit per-bin products (FP32 view only)
    const uint32_t* Chat16 = nullptr;
    float out_scale = 1.0f;              // undoes the power-of-two scaling of Chat16
    // margin blocks (nc > 0): Z_B, Z_C, the margin's preconditioner inverse, and scratch
    // (mtmp: nc x R; mpart: margin_ksplit(P*M) x nc x R) attached by the caller
    int nc = 0;
    const cplx<T>* zb = nullptr;
    const cplx<T>* zc = nullptr;
    const cplx<T>* pcinv = nullptr;
    cplx<T>* mtmp = nullptr;
    cplx<T>* mpart = nullptr;
};

// scratch bytes a view of a margin array needs for R columns (FP64-sized, shared by both views)
static size_t margin_scratch_bytes(const Geom& g, int R) {
    if (g.Nc == 0) return 0;
    return sizeof(double2) * (size_t)g.Nc * R * (1 + margin_ksplit(g.NA())) + 512;
}

template <typename T> static void attach_margin(OpV<T>& v, void* scratch) {
    if (v.nc == 0) return;
    MBT_REQUIRE(scratch != nullptr, "margin scratch missing");
    v.mtmp = static_cast<cplx<T>*>(scratch);
    v.mpart = v.mtmp + (size_t)v.nc * v.R;
}

template <typename T>
static OpV<T> make_view(const OpData& op, int pc, void* Xh, void* Yh, void* tmp, int R, hipStream_t s,
                        int fmt = kFmtNone);

template <>
OpV<double> make_view<double>(const OpData& op, int pc, void* Xh, void* Yh, void* tmp, int R, hipStream_t s, int) {
    OpV<double> v;
    v.g = &op.g;
    v.Chat = op.Chat.as<double2>();
    // the folded P_K^{-1} C^ covers element rows only: margin arrays apply P_K^{-1} Z directly
    if (pc == MBT_PC_ELEMENT_BLOCK && op.g.Nc == 0) v.ChatA = op.ChatK.as<double2>();
    if (op.g.Nc > 0) {
        v.nc = op.g.Nc;
        v.zb = op.ZB.as<double2>();
        v.zc = op.ZC.as<double2>();
        v.pcinv = pc == MBT_PC_NORMAL_EQ ? op.PcInv.as<double2>() : op.ZcInv.as<double2>();
        MBT_REQUIRE(v.zb && v.zc && v.pcinv, "margin pieces not built for this operator");
    }
    v.pinv = pc == MBT_PC_NORMAL_EQ ? op.PaInv.as<double2>() : op.PkInv.as<double2>();
    MBT_REQUIRE(v.pinv != nullptr, "preconditioner not built for this operator");
    v.pstride = pc == MBT_PC_NORMAL_EQ ? (int64_t)op.g.M * op.g.M : 0;
    v.twx = op.tw.as<double2>();
    v.twy = op.tw.as<double2>() + op.g.Px;
    v.Xh = (double2*)Xh;
    v.Yh = (double2*)Yh;
    v.tmp = (double2*)tmp;
    v.R = R;
    v.pc = pc;
    v.s = s;
    return v;
}

template <>
OpV<float> make_view<float>(const OpData& op, int pc, void* Xh, void* Yh, void* tmp, int R, hipStream_t s, int fmt) {
    OpV<float> v;
    if (fmt != kFmtNone) {
        MBT_REQUIRE(op.Chat16[fmt].p != nullptr, "16-bit spectra not built");
        v.fmt = fmt;
        v.Chat16 = op.Chat16[fmt].as<uint32_t>();
        v.out_scale = (float)(1.0 / op.scale16[fmt]);
    }
    v.g = &op.g;
    v.Chat = op.Chat32.as<float2>();
    if (pc == MBT_PC_ELEMENT_BLOCK && fmt == kFmtNone && op.g.Nc == 0) v.ChatA = op.ChatK32.as<float2>();
    if (op.g.Nc > 0) {
        MBT_REQUIRE(fmt == kFmtNone, "16-bit products are not available for arrays with a margin");
        v.nc = op.g.Nc;
        v.zb = op.ZB32.as<float2>();
        v.zc = op.ZC32.as<float2>();
        v.pcinv = pc == MBT_PC_NORMAL_EQ ? op.PcInv32.as<float2>() : op.ZcInv32.as<float2>();
        MBT_REQUIRE(v.zb && v.zc && v.pcinv, "margin pieces not built for this operator");
    }
    v.pinv = pc == MBT_PC_NORMAL_EQ ? op.PaInv32.as<float2>() : op.PkInv32.as<float2>();
    MBT_REQUIRE(v.pinv != nullptr && v.Chat != nullptr, "FP32 operator pieces not built");
    v.pstride = pc == MBT_PC_NORMAL_EQ ? (int64_t)op.g.M * op.g.M : 0;
    v.twx = op.tw32.as<float2>();
    v.twy = op.tw32.as<float2>() + op.g.Px;
    v.Xh = (float2*)Xh;
    v.Yh = (float2*)Yh;
    v.tmp = (float2*)tmp;
    v.R = R;
    v.pc = pc;
    v.s = s;
    return v;
}

// y = Z x (opz 0) or Z^H x (opz 1) by FFT over the lattice, per-bin products, inverse FFT and crop;
// chat replaces the block spectra (the preconditioned operator's, FP64/FP32 products only)
// Margin part of y = Z x (opz 0) or Z^H x (opz 1) for Z = [[Z_A, Z_B^T], [Z_B, Z_C]]: before the lattice
// transform (which may overwrite x's element rows when y == x) the margin rows
// t = op(Z_B) x_A + op(Z_C) x_C go to scratch; after it, the element rows receive op(Z_B^T) x_C and the
// margin rows t.  Z^H = [[Z_A^H, Z_B^H], [Z_B^*, Z_C^H]].
template <typename T> static void margin_pre(const OpV<T>& o, int opz, const cplx<T>* x) {
    const Geom& g = *o.g;
    const int64_t NA = g.NA();
    const int nc = o.nc, R = o.R;
    // t = Z_B x_A or Z_B^* x_A (row-major Z_B: op(A)(m, k) = Z_B[m][k])
    margin_gemm<T>(o.zb, NA, 1, opz == 1, x, R, 1, o.mtmp, R, nc, NA, R, false, o.mpart, o.s);
    // t += Z_C x_C (Z_C[m][k]) or Z_C^H x_C (conj Z_C[k][m])
    if (opz == 0)
        margin_gemm<T>(o.zc, nc, 1, false, x + NA * R, R, 1, o.mtmp, R, nc, nc, R, true, nullptr, o.s);
    else
        margin_gemm<T>(o.zc, 1, nc, true, x + NA * R, R, 1, o.mtmp, R, nc, nc, R, true, nullptr, o.s);
}
template <typename T> static void margin_post(const OpV<T>& o, int opz, const cplx<T>* x, cplx<T>* y) {
    const Geom& g = *o.g;
    const int64_t NA = g.NA();
    const int nc = o.nc, R = o.R;
    // y_A += Z_B^T x_C (op(A)(m, k) = Z_B[k][m]) or Z_B^H x_C (conjugated)
    margin_gemm<T>(o.zb, 1, NA, opz == 1, x + NA * R, R, 1, y, R, (int)NA, nc, R, true, nullptr, o.s);
    convert<cplx<T>, cplx<T>>(o.mtmp, y + NA * R, (int64_t)nc * R, o.s);
}

template <typename T>
static void zmul_lattice(const OpV<T>& o, int opz, const cplx<T>* x, cplx<T>* y, const cplx<T>* chat);

template <typename T>
static void zmul(const OpV<T>& o, int opz, const cplx<T>* x, cplx<T>* y, const cplx<T>* chat = nullptr) {
    if (o.nc > 0) margin_pre<T>(o, opz, x);
    zmul_lattice<T>(o, opz, x, y, chat);
    if (o.nc > 0) margin_post<T>(o, opz, x, y);
}

template <typename T>
static void zmul_lattice(const OpV<T>& o, int opz, const cplx<T>* x, cplx<T>* y, const cplx<T>* chat) {
    const Geom& g = *o.g;
    const int64_t B = (int64_t)g.M * o.R;
    const double sc = sizeof(cplx<T>);
    const double spat = (double)g.NA() * o.R * sc, spec = (double)g.bins() * g.M * o.R * sc;
    if constexpr (sizeof(T) == 4) {
        if (o.fmt != kFmtNone) {
            // 16-bit spectrum X^ (4 bytes per value), FP32 products Y^
            uint32_t* xh16 = reinterpret_cast<uint32_t*>(o.Xh);
            const double spec16 = (double)g.bins() * g.M * o.R * 4.0;
            {
                ProfScope ps(kKFftFwd, spat + spec16, 0.0, o.s);
                if (o.fmt == kFmtBf16)
                    fft_fwd_pad16<kFmtBf16>(g, x, xh16, B, o.twx, o.twy, o.Yh, o.s);
                else
                    fft_fwd_pad16<kFmtF16>(g, x, xh16, B, o.twx, o.twy, o.Yh, o.s);
            }
            {
                ProfScope ps(kKBinProduct, spec16 + spec + (double)g.bins() * g.M * g.M * 4.0,
                             8.0 * g.bins() * g.M * g.M * o.R, o.s);
                if (o.fmt == kFmtBf16)
                    cgemm16_batched<kFmtBf16>(o.Chat16, (int64_t)g.M * g.M, xh16, o.Yh, g.M, o.R, g.bins(), opz,
                                              o.out_scale, o.s);
                else
                    cgemm16_batched<kFmtF16>(o.Chat16, (int64_t)g.M * g.M, xh16, o.Yh, g.M, o.R, g.bins(), opz,
                                             o.out_scale, o.s);
            }
            {
                ProfScope ps(kKFftInv, spat + spec, 0.0, o.s);
                fft_inv_crop<T>(g, o.Yh, y, B, o.twx, o.twy, reinterpret_cast<cplx<T>*>(o.Xh), o.s);
            }
            return;
        }
    }
    {
        ProfScope ps(kKFftFwd, spat + spec, 0.0, o.s);
        fft_fwd_pad<T>(g, x, o.Xh, B, o.twx, o.twy, o.Yh, o.s);   // Y^ is free until the product
    }
    {
        ProfScope ps(kKBinProduct, 2 * spec + (double)g.bins() * g.M * g.M * sc, 8.0 * g.bins() * g.M * g.M * o.R, o.s);
        cgemm_batched<T>(chat ? chat : o.Chat, (int64_t)g.M * g.M, o.Xh, o.Yh, g.M, o.R, g.bins(), opz, o.s);
    }
    {
        ProfScope ps(kKFftInv, spat + spec, 0.0, o.s);
        fft_inv_crop<T>(g, o.Yh, y, B, o.twx, o.twy, o.Xh, o.s);   // X^ is free after the product
    }
}

template <typename T> static void pinv(const OpV<T>& o, const cplx<T>* x, cplx<T>* y) {
    const double sc = sizeof(cplx<T>);
    const double blocks = o.pstride ? (double)o.g->P : 1.0;
    {
        ProfScope ps(kKPrecondApply, 2.0 * o.g->NA() * o.R * sc + blocks * o.g->M * o.g->M * sc,
                     8.0 * o.g->P * o.g->M * o.g->M * o.R, o.s);
        cgemm_batched<T>(o.pinv, o.pstride, x, y, o.g->M, o.R, o.g->P, 0, o.s);
    }
    if (o.nc > 0) {
        // the margin's block: P_C^{-1} (normal equations) or Z_C^{-1} (element blocks)
        const int64_t off = o.g->NA() * o.R;
        margin_gemm<T>(o.pcinv, o.nc, 1, false, x + off, o.R, 1, y + off, o.R, o.nc, o.nc, o.R, false, nullptr, o.s);
    }
}

// preconditioned operator: P_K^{-1} Z  or  P^{-1} Z^H Z
template <typename T> static void apply_A(const OpV<T>& o, const cplx<T>* x, cplx<T>* y) {
    if (o.ChatA) {   // P_K^{-1} Z with the preconditioner folded into the spectra
        zmul<T>(o, 0, x, y, o.ChatA);
        return;
    }
    zmul<T>(o, 0, x, o.tmp);
    if (o.pc == MBT_PC_NORMAL_EQ) zmul<T>(o, 1, o.tmp, o.tmp);
    pinv<T>(o, o.tmp, y);
}

// preconditioned right-hand side: P_K^{-1} v  or  P^{-1} Z^H v
template <typename T> static void apply_rhs(const OpV<T>& o, const cplx<T>* v, cplx<T>* b) {
    if (o.pc == MBT_PC_NORMAL_EQ) {
        zmul<T>(o, 1, v, o.tmp);
        pinv<T>(o, o.tmp, b);
    } else {
        pinv<T>(o, v, b);
    }
}

// ------------------------------------------------------------------ solve drivers
size_t solve_bytes(const Geom& g, int R, const mbt_solve_opts& o) {
    const size_t NR = (size_t)g.N * R;
    const size_t tb = o.prec == MBT_FP64 ? 16 : 8;
    size_t b = 0;
    b += (size_t)std::max(o.restart + 1, 5) * NR * tb; // Krylov basis (PCG: four work vectors and b)
    b += 2 * (size_t)g.bins() * g.M * R * 16;          // spectral buffers (FP64-sized, shared)
    b += NR * 16;                                      // operator temp
    b += NR * tb;                                      // preconditioned rhs
    b += 2 * NR * 16;                                  // V, X
    b += NR * 16;                                      // FP64 residual
    if (o.prec != MBT_FP64) b += NR * 16 + NR * 8;     // d, r32
    b += std::max(gmres_state_bytes(g.N, R, o.restart), std::max(pcg_state_bytes(g.N, R), cocg_state_bytes(g.N, R)));
    b += (size_t)R * 64 + ((size_t)g.N / 256 + 2) * R * 8 + (size_t)g.P * R * 16 + (1 << 20);
    b += margin_scratch_bytes(g, R);
    return b;
}

// The packed basis of the reduced-precision paths takes RHS in pairs: an odd
// batch is solved with its last port repeated (the extra column is identical
// and dropped).
static bool pads_odd(const mbt_solve_opts& o) {
    return o.prec != MBT_FP64 && !(o.flags & (MBT_FLAG_FP32_BASIS | MBT_FLAG_CGS2 | MBT_FLAG_PCG | MBT_FLAG_COCG));
}
int padded(int R, const mbt_solve_opts& o) { return R + ((pads_odd(o) && (R & 1)) ? 1 : 0); }

int choose_chunk(size_t budget, const Geom& g, int R, const mbt_solve_opts& o) {
    if (o.rhs_chunk > 0) return std::min(R, o.rhs_chunk);
    int c = R;
    while (c > 1 && solve_bytes(g, padded(c, o), o) > budget) c = (c + 1) / 2;
    if (solve_bytes(g, padded(c, o), o) > budget)
        throw Error(-2, "one right-hand side does not fit the device-memory budget");
    return c;
}

size_t extract_bytes(int P, int nscan) {
    const size_t ns = (size_t)std::max(nscan, 1);
    return 4 * sizeof(double2) * (size_t)P * P + sizeof(double2) * P + sizeof(int) * ((size_t)P + 8) +
           sizeof(double) * 2 * ns + sizeof(double2) * 3 * ns + 1024;
}

int solve_status(const SolveOut& so) {
    if (so.nflag > 0) return MBT_EBREAKDOWN;
    if (so.nconv < (int)so.iters.size()) return MBT_ENOCONV;
    return MBT_OK;
}

static void norms_host(const double2* X, int64_t N, int R, DevArena& arena, std::vector<double>& out, hipStream_t s) {
    const size_t mark = arena.off;
    const int nchunk = (int)((N + 255) / 256);
    double* part = arena.get<double>((size_t)nchunk * R);
    double* dn = arena.get<double>(R);
    column_norms(X, N, R, part, dn, s);
    out.resize(R);
    MBT_HIP(hipMemcpyAsync(out.data(), dn, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MBT_HIP(hipStreamSynchronize(s));
    arena.off = mark;
}

SolveOut solve_rhs(const OpData& op, const mbt_solve_opts& o, const double2* V, int R, double2* X, Worker& wk,
                   DevArena& arena) {
    const Geom& g = op.g;
    const int64_t NR = g.N * R;
    const int m = o.restart;
    hipStream_t s = wk.stream;
    SolveOut out;
    out.iters.assign(R, 0);
    out.conv.assign(R, 0);
    out.flag.assign(R, 0);
    void* Xh = arena.get<double2>((size_t)g.bins() * g.M * R);
    void* Yh = arena.get<double2>((size_t)g.bins() * g.M * R);
    double2* tmp = arena.get<double2>(NR);
    void* mscr = g.Nc > 0 ? arena.get<char>(margin_scratch_bytes(g, R)) : nullptr;
    GmresParams prm;
    prm.restart = m;
    prm.max_cycles = o.max_cycles;
    prm.matvecs_per_apply = o.pc == MBT_PC_NORMAL_EQ ? 2 : 1;
    prm.host_count = wk.host_count;
    prm.dcgs2 = !(o.flags & MBT_FLAG_CGS2);
    prm.packed_basis = o.prec != MBT_FP64 && !(o.flags & MBT_FLAG_FP32_BASIS);
    std::vector<double> vn;
    norms_host(V, g.N, R, arena, vn, s);

    const bool use_pcg = (o.flags & MBT_FLAG_PCG) != 0;
    const bool use_cocg = (o.flags & MBT_FLAG_COCG) != 0;
    const int pcg_maxit = o.restart * o.max_cycles;
    if (o.prec == MBT_FP64) {
        double2* basis = arena.get<double2>((size_t)std::max(m + 1, 5) * NR);
        double2* b = arena.get<double2>(NR);
        OpV<double> ov = make_view<double>(op, o.pc, Xh, Yh, tmp, R, s);
        attach_margin(ov, mscr);
        GmresResult gr;
        if (use_pcg) {
            // Z^H Z I = Z^H V with P_A (Sec. II-C)
            zmul<double>(ov, 1, V, b);
            out.matvecs += 1;
            std::function<void(const double2*, double2*)> fn = [&](const double2* x, double2* y) {
                zmul<double>(ov, 0, x, ov.tmp);
                zmul<double>(ov, 1, ov.tmp, y);
            };
            std::function<void(const double2*, double2*)> fp = [&](const double2* x, double2* y) {
                pinv<double>(ov, x, y);
            };
            gr = pcg_batched<double2>(fn, fp, b, X, basis, g.N, R, o.tol, pcg_maxit, wk.host_count, arena, s);
        } else if (use_cocg) {
            // Z I = V with M = P_K, both complex symmetric
            std::function<void(const double2*, double2*)> fz = [&](const double2* x, double2* y) {
                zmul<double>(ov, 0, x, y);
            };
            std::function<void(const double2*, double2*)> fm = [&](const double2* x, double2* y) {
                pinv<double>(ov, x, y);
            };
            gr = cocg_batched<double2>(fz, fm, V, X, basis, g.N, R, o.tol, pcg_maxit, wk.host_count, arena, s);
        } else {
            apply_rhs<double>(ov, V, b);
            out.matvecs += o.pc == MBT_PC_NORMAL_EQ ? 1 : 0;
            prm.tol = o.tol;
            std::function<void(const double2*, double2*)> f = [&](const double2* x, double2* y) {
                apply_A<double>(ov, x, y);
            };
            gr = gmres_batched<double2>(f, b, X, basis, g.N, R, prm, arena, s);
        }
        out.iters = gr.iters;
        out.cycles = gr.cycles;
        out.matvecs += gr.matvecs;
        out.outer = 1;
        for (int r = 0; r < R; ++r) {
            out.conv[r] = gr.conv[r] ? 1 : 0;
            out.flag[r] = gr.flag[r] ? 1 : 0;
            out.nconv += out.conv[r];
            out.nflag += out.flag[r];
        }
    } else {
        float2* basis = arena.get<float2>((size_t)std::max(m + 1, 5) * NR);
        float2* b32 = arena.get<float2>(NR);
        float2* r32 = arena.get<float2>(NR);
        double2* r64 = arena.get<double2>(NR);
        double2* d = arena.get<double2>(NR);
        double* mask = arena.get<double>(R);      // 1/||r|| per RHS still refining, 0 once done
        double* unscale = arena.get<double>(R);   // ||r|| per RHS still refining, 0 once done
        OpV<double> ov = make_view<double>(op, o.pc, Xh, Yh, tmp, R, s);
        OpV<float> ov32 = make_view<float>(op, o.pc, Xh, Yh, tmp, R, s, fmt16_of(o.prec));
        attach_margin(ov, mscr);
        attach_margin(ov32, mscr);
        std::function<void(const float2*, float2*)> f = [&](const float2* x, float2* y) { apply_A<float>(ov32, x, y); };
        prm.tol = inner_tol(o);
        zero_d(X, NR, s);
        std::vector<int> done(R, 0), flagged(R, 0), raised(R, 0);
        // FP64 residual norm before the last correction (X = 0 at first: ||V||)
        std::vector<double> prev(vn), hundo(R);
        bool unchecked = false;   // the last correction has not been checked against prev yet
        for (int outer = 0; outer < o.refine_max; ++outer) {
            if (outer == 0) {
                convert<double2, double2>(V, r64, NR, s);
            } else {
                zmul<double>(ov, 0, X, tmp);
                out.matvecs += 1;
                sub_d(V, tmp, r64, NR, s);
            }
            std::vector<double> rn;
            norms_host(r64, g.N, R, arena, rn, s);
            unchecked = false;
            for (int r = 0; r < R; ++r)
                if (!std::isfinite(rn[r])) flagged[r] = 1;   // non-finite input or iterate: breakdown
            // Refinement contracts only while the reduced-precision operator's error is small
            // against the smallest singular values of Z; where it is not, the iterates can
            // grow without bound.  A correction that raised the FP64 residual is taken back
            // (d still holds it) and that RHS stops refining with the better iterate.
            int nundo = 0;
            for (int r = 0; r < R; ++r) {
                hundo[r] = 0.0;
                if (outer > 0 && !raised[r] && rn[r] > prev[r]) {
                    hundo[r] = 1.0;
                    raised[r] = 1;
                    ++nundo;
                } else if (!raised[r]) {
                    prev[r] = rn[r];
                }
            }
            if (nundo > 0) {
                MBT_HIP(hipMemcpyAsync(mask, hundo.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
                scale_columns_d(d, mask, g.N, R, s);
                sub_d(X, d, X, NR, s);
            }
            // the correction equation Z d = r is solved for r / ||r|| (unit columns keep the
            // reduced-precision spectra inside the 16-bit range), then d is scaled back
            std::vector<double> hmask(2 * R);
            int left = 0;
            for (int r = 0; r < R; ++r) {
                const double rel = vn[r] > 0 ? rn[r] / vn[r] : 0.0;
                done[r] = (rel <= o.refine_tol) || flagged[r] || raised[r] || !(rn[r] > 0);
                hmask[r] = done[r] ? 0.0 : 1.0 / rn[r];
                hmask[R + r] = done[r] ? 0.0 : rn[r];
                left += done[r] ? 0 : 1;
            }
            if (left == 0) break;
            MBT_HIP(hipMemcpyAsync(mask, hmask.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
            MBT_HIP(hipMemcpyAsync(unscale, hmask.data() + R, sizeof(double) * R, hipMemcpyHostToDevice, s));
            scale_columns_d(r64, mask, g.N, R, s);
            convert<double2, float2>(r64, r32, NR, s);
            GmresResult gr;
            if (use_pcg) {
                zmul<float>(ov32, 1, r32, b32);
                out.matvecs += 1;
                std::function<void(const float2*, float2*)> fn = [&](const float2* x, float2* y) {
                    zmul<float>(ov32, 0, x, ov32.tmp);
                    zmul<float>(ov32, 1, ov32.tmp, y);
                };
                std::function<void(const float2*, float2*)> fp = [&](const float2* x, float2* y) {
                    pinv<float>(ov32, x, y);
                };
                gr = pcg_batched<float2>(fn, fp, b32, d, basis, g.N, R, prm.tol, pcg_maxit, wk.host_count, arena, s);
            } else if (use_cocg) {
                std::function<void(const float2*, float2*)> fz = [&](const float2* x, float2* y) {
                    zmul<float>(ov32, 0, x, y);
                };
                std::function<void(const float2*, float2*)> fm = [&](const float2* x, float2* y) {
                    pinv<float>(ov32, x, y);
                };
                gr = cocg_batched<float2>(fz, fm, r32, d, basis, g.N, R, prm.tol, pcg_maxit, wk.host_count, arena, s);
            } else {
                apply_rhs<float>(ov32, r32, b32);
                out.matvecs += o.pc == MBT_PC_NORMAL_EQ ? 1 : 0;
                gr = gmres_batched<float2>(f, b32, d, basis, g.N, R, prm, arena, s);
            }
            scale_columns_d(d, unscale, g.N, R, s);
            if (outer > 0) {
                // A correction a thousand times the iterate is a runaway inner solve, not
                // refinement; adding it and subtracting it again would cancel the iterate's
                // digits, so it is dropped here and that RHS stops refining.
                std::vector<double> dn, xn;
                norms_host(d, g.N, R, arena, dn, s);
                norms_host(X, g.N, R, arena, xn, s);
                int nrej = 0;
                for (int r = 0; r < R; ++r) {
                    const bool rej = !done[r] && !(dn[r] <= 1e3 * xn[r]);
                    hundo[r] = rej ? 0.0 : 1.0;
                    if (rej) {
                        raised[r] = 1;
                        ++nrej;
                    }
                }
                if (nrej > 0) {
                    MBT_HIP(hipMemcpyAsync(mask, hundo.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
                    scale_columns_d(d, mask, g.N, R, s);
                }
            }
            add_to_f64<double2>(X, d, NR, s);
            unchecked = true;
            out.outer = outer + 1;
            out.cycles += gr.cycles;
            out.matvecs += gr.matvecs;
            for (int r = 0; r < R; ++r) {
                out.iters[r] += gr.iters[r];
                if (gr.flag[r]) flagged[r] = 1;
            }
        }
        // final verdict on the FP64 residual; the last correction, when the step budget ran
        // out before it could be checked, is taken back like any other that raised the residual
        std::vector<double> rn;
        for (int pass = 0; pass < 2; ++pass) {
            zmul<double>(ov, 0, X, tmp);
            out.matvecs += 1;
            sub_d(V, tmp, r64, NR, s);
            norms_host(r64, g.N, R, arena, rn, s);
            if (pass == 1 || !unchecked) break;
            int nundo = 0;
            for (int r = 0; r < R; ++r) {
                hundo[r] = (!raised[r] && rn[r] > prev[r]) ? 1.0 : 0.0;
                nundo += hundo[r] > 0 ? 1 : 0;
            }
            if (nundo == 0) break;
            MBT_HIP(hipMemcpyAsync(mask, hundo.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
            scale_columns_d(d, mask, g.N, R, s);
            sub_d(X, d, X, NR, s);
        }
        for (int r = 0; r < R; ++r) {
            if (!std::isfinite(rn[r])) flagged[r] = 1;
            const double rel = vn[r] > 0 ? rn[r] / vn[r] : 0.0;
            out.conv[r] = (rel <= o.refine_tol && !flagged[r]) ? 1 : 0;
            out.flag[r] = flagged[r] ? 1 : 0;
            out.nconv += out.conv[r];
            out.nflag += out.flag[r];
            out.relres_max = std::max(out.relres_max, rel);
        }
        return out;
    }
    // FP64 path: true residual ||V - Z X|| / ||V||
    {
        OpV<double> ov = make_view<double>(op, o.pc, Xh, Yh, tmp, R, s);
        attach_margin(ov, mscr);
        double2* r64 = arena.get<double2>(NR);
        zmul<double>(ov, 0, X, tmp);
        out.matvecs += 1;
        sub_d(V, tmp, r64, NR, s);
        std::vector<double> rn;
        norms_host(r64, g.N, R, arena, rn, s);
        for (int r = 0; r < R; ++r) out.relres_max = std::max(out.relres_max, vn[r] > 0 ? rn[r] / vn[r] : 0.0);
    }
    return out;
}

SolveOut admittance(mbt_ctx* ctx, const mbt_array* arr, double s, const int32_t* ports, int nports,
                    const mbt_solve_opts& o, double2* Ydev, Worker& wk, mbt_stats* st, size_t budget) {
    const Geom& g = arr->g;
    const double t0 = now_s();
    std::shared_ptr<OpData> op;
    if (o.flags & MBT_FLAG_NO_CACHE) {
        op = build_uncached(arr, s, o, wk);
    } else {
        op = get_op(ctx, arr, s, o.pc == MBT_PC_NORMAL_EQ, o.prec, wk);
    }
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t1 = now_s();
    const int chunk = choose_chunk(budget, g, nports, o);
    // port list laid out chunk by chunk, odd chunks padded with their last port
    std::vector<int32_t> plist;
    plist.reserve((size_t)nports + (size_t)nports / std::max(chunk, 1) + 1);
    for (int c0 = 0; c0 < nports; c0 += chunk) {
        const int R = std::min(chunk, nports - c0);
        plist.insert(plist.end(), ports + c0, ports + c0 + R);
        if (padded(R, o) > R) plist.push_back(ports[c0 + R - 1]);
    }
    const size_t need = solve_bytes(g, padded(chunk, o), o) + sizeof(int32_t) * plist.size() + 4096;
    wk.ensure(need);
    DevArena arena;
    arena.base = wk.ws.as<char>();
    arena.cap = wk.ws.bytes;
    int32_t* dports = arena.get<int32_t>(plist.size());
    MBT_HIP(hipMemcpyAsync(dports, plist.data(), sizeof(int32_t) * plist.size(), hipMemcpyHostToDevice, wk.stream));
    SolveOut total;
    total.iters.assign(nports, 0);
    const size_t base_mark = arena.off;
    int64_t pl0 = 0;
    for (int c0 = 0; c0 < nports; c0 += chunk) {
        const int R = std::min(chunk, nports - c0);
        const int Rs = padded(R, o);   // columns solved
        arena.off = base_mark;
        double2* V = arena.get<double2>((size_t)g.N * Rs);
        double2* X = arena.get<double2>((size_t)g.N * Rs);
        scatter_ports(g, dports + pl0, Rs, V, wk.stream);
        pl0 += Rs;
        SolveOut so = solve_rhs(*op, o, V, Rs, X, wk, arena);
        gather_ports(g, X, Rs, R, Ydev + (int64_t)c0 * g.P, wk.stream);
        for (int r = 0; r < R; ++r) total.iters[c0 + r] = so.iters[r];
        total.cycles = std::max(total.cycles, so.cycles);
        total.outer = std::max(total.outer, so.outer);
        for (int r = 0; r < R; ++r) {   // the padding column (a repeat) is not counted
            total.nconv += so.conv[r];
            total.nflag += so.flag[r];
        }
        total.matvecs += so.matvecs;
        total.relres_max = std::max(total.relres_max, so.relres_max);
    }
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t2 = now_s();
    if (st) {
        st->nrhs = nports;
        st->nconverged = total.nconv;
        st->cycles = total.cycles;
        st->outer_steps = total.outer;
        st->iters_min = nports ? *std::min_element(total.iters.begin(), total.iters.end()) : 0;
        st->iters_max = nports ? *std::max_element(total.iters.begin(), total.iters.end()) : 0;
        st->iters_total = 0;
        for (int v : total.iters) st->iters_total += v;
        st->matvecs = total.matvecs;
        st->true_relres_max = total.relres_max;
        st->t_setup = t1 - t0;
        st->t_solve = t2 - t1;
        st->t_extract = 0;
    }
    return total;
}

// Phased voltage excitation of every gap for each scan direction: solve, gap
// currents, center-element active impedance and ARC (all on the device).
static SolveOut scan_solve(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts& o, size_t budget,
                                  const double* theta, const double* phi, int nscan, double z0, int c, double* Ip,
                           double* Za, double* Gamma, Worker& wk, mbt_stats* st) {
    const Geom& g = arr->g;
    const double t0 = now_s();
    std::shared_ptr<OpData> op;
    if (o.flags & MBT_FLAG_NO_CACHE) {
        op = build_uncached(arr, s, o, wk);
    } else {
        op = get_op(ctx, arr, s, o.pc == MBT_PC_NORMAL_EQ, o.prec, wk);
    }
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t1 = now_s();
    const int chunk = choose_chunk(budget, g, nscan, o);
    // angles laid out chunk by chunk, odd chunks padded with their last direction
    std::vector<double> th, ph;
    for (int c0 = 0; c0 < nscan; c0 += chunk) {
        const int R = std::min(chunk, nscan - c0);
        th.insert(th.end(), theta + c0, theta + c0 + R);
        ph.insert(ph.end(), phi + c0, phi + c0 + R);
        if (padded(R, o) > R) {
            th.push_back(theta[c0 + R - 1]);
            ph.push_back(phi[c0 + R - 1]);
        }
    }
    const size_t need = solve_bytes(g, padded(chunk, o), o) + sizeof(double) * 2 * (th.size() + nscan) +
                        sizeof(double2) * ((size_t)g.P * nscan + 2 * (size_t)nscan) + 8 * 256;
    wk.ensure(need);
    DevArena arena;
    arena.base = wk.ws.as<char>();
    arena.cap = wk.ws.bytes;
    double* dth = arena.get<double>(th.size());
    double* dph = arena.get<double>(ph.size());
    double* dth0 = arena.get<double>(nscan);
    double* dph0 = arena.get<double>(nscan);
    double2* dIp = arena.get<double2>((size_t)g.P * nscan);
    double2* dZa = arena.get<double2>(nscan);
    double2* dG = arena.get<double2>(nscan);
    MBT_HIP(hipMemcpyAsync(dth, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, wk.stream));
    MBT_HIP(hipMemcpyAsync(dph, ph.data(), sizeof(double) * ph.size(), hipMemcpyHostToDevice, wk.stream));
    MBT_HIP(hipMemcpyAsync(dth0, theta, sizeof(double) * nscan, hipMemcpyHostToDevice, wk.stream));
    MBT_HIP(hipMemcpyAsync(dph0, phi, sizeof(double) * nscan, hipMemcpyHostToDevice, wk.stream));
    SolveOut total;
    total.iters.assign(nscan, 0);
    const size_t base_mark = arena.off;
    int64_t a0 = 0;
    for (int c0 = 0; c0 < nscan; c0 += chunk) {
        const int R = std::min(chunk, nscan - c0);
        const int Rs = padded(R, o);
        arena.off = base_mark;
        double2* V = arena.get<double2>((size_t)g.N * Rs);
        double2* X = arena.get<double2>((size_t)g.N * Rs);
        scan_voltages(g, op->k, dth + a0, dph + a0, Rs, V, wk.stream);
        a0 += Rs;
        SolveOut so = solve_rhs(*op, o, V, Rs, X, wk, arena);
        gather_ports(g, X, Rs, R, dIp + (int64_t)c0 * g.P, wk.stream);
        for (int r = 0; r < R; ++r) {
            total.iters[c0 + r] = so.iters[r];
            total.nconv += so.conv[r];
            total.nflag += so.flag[r];
        }
        total.cycles = std::max(total.cycles, so.cycles);
        total.outer = std::max(total.outer, so.outer);
        total.matvecs += so.matvecs;
        total.relres_max = std::max(total.relres_max, so.relres_max);
    }
    scan_active(g, op->k, dIp, nscan, c, dth0, dph0, z0, dZa, dG, wk.stream);
    MBT_HIP(hipMemcpyAsync(Za, dZa, sizeof(double2) * nscan, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipMemcpyAsync(Gamma, dG, sizeof(double2) * nscan, hipMemcpyDeviceToHost, wk.stream));
    if (Ip)
        MBT_HIP(hipMemcpyAsync(Ip, dIp, sizeof(double2) * (size_t)g.P * nscan, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t2 = now_s();
    if (st) {
        st->nrhs = nscan;
        st->nconverged = total.nconv;
        st->cycles = total.cycles;
        st->outer_steps = total.outer;
        st->iters_min = *std::min_element(total.iters.begin(), total.iters.end());
        st->iters_max = *std::max_element(total.iters.begin(), total.iters.end());
        st->iters_total = 0;
        for (int v : total.iters) st->iters_total += v;
        st->matvecs = total.matvecs;
        st->true_relres_max = total.relres_max;
        st->t_setup = t1 - t0;
        st->t_solve = t2 - t1;
        st->t_extract = 0;
    }
    return total;
}

SolveOut solve_frequency(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts& o, size_t budget,
                         const double* theta, const double* phi, int nscan, double z0, double* Zp, double* Za,
                         double* Gamma, double* Gamma_wave, Worker& wk, mbt_stats* st) {
    const Geom& g = arr->g;
    MBT_REQUIRE(!(arr->blocks && nscan > 0), "scan quantities need element positions: dipole arrays only");
    const int P = g.P;
    const int64_t PP = (int64_t)P * P;
    std::vector<int32_t> pl(P);
    for (int i = 0; i < P; ++i) pl[i] = i;
    // extraction buffers from the worker's persistent area, carved in order:
    // Y_p, Z_p, S, work (P x P each), a column, pivots + flag, scan angles, scan outputs
    wk.ensure_x(extract_bytes(P, nscan));
    const int ns = std::max(nscan, 1);
    double2* Yd = wk.xs.as<double2>();
    double2* Zd = Yd + PP;
    double2* Sd = Zd + PP;
    double2* Wd = Sd + PP;
    double2* colbuf = Wd + PP;
    int* piv = (int*)(colbuf + P);
    int* flag = piv + P;
    double* dth = (double*)(((uintptr_t)(flag + 8) + 255) & ~(uintptr_t)255);
    double* dph = dth + ns;
    double2* dout = (double2*)(dph + ns);
    MBT_REQUIRE((char*)(dout + 3 * ns) <= wk.xs.as<char>() + wk.xs.bytes, "extraction buffer overflow");
    SolveOut so = admittance(ctx, arr, s, pl.data(), P, o, Yd, wk, st, budget);
    const double t0 = now_s();
    hipStream_t str = wk.stream;
    gj_inverse(Yd, Zd, P, colbuf, piv, flag, str);
    if (nscan > 0) {
        if (Gamma_wave) s_matrix(Zd, Sd, Wd, P, z0, colbuf, piv, flag, str);
        MBT_HIP(hipMemcpyAsync(dth, theta, sizeof(double) * nscan, hipMemcpyHostToDevice, str));
        MBT_HIP(hipMemcpyAsync(dph, phi, sizeof(double) * nscan, hipMemcpyHostToDevice, str));
        const int c = (g.ny / 2) * g.nx + g.nx / 2;
        scans(g, 2.0 * M_PI * s, Zd, Gamma_wave ? Sd : nullptr, c, dth, dph, nscan, z0, dout, dout + nscan,
              Gamma_wave ? dout + 2 * nscan : nullptr, str);
        MBT_HIP(hipMemcpyAsync(Za, dout, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
        MBT_HIP(hipMemcpyAsync(Gamma, dout + nscan, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
        if (Gamma_wave)
            MBT_HIP(hipMemcpyAsync(Gamma_wave, dout + 2 * nscan, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
    }
    if (Zp) MBT_HIP(hipMemcpyAsync(Zp, Zd, sizeof(double2) * PP, hipMemcpyDeviceToHost, str));
    MBT_HIP(hipStreamSynchronize(str));
    if (st) st->t_extract = now_s() - t0;
    return so;
}

}  // namespace mbt

// ================================================================== C ABI
namespace {

mbt_status finish_status(const SolveOut& so) {
    const int code = solve_status(so);
    if (code == MBT_EBREAKDOWN) return set_err(code, "non-finite value in the Krylov recurrence for some right-hand sides");
    if (code == MBT_ENOCONV) return set_err(code, "some right-hand sides did not converge");
    return MBT_OK;
}

struct DevScope {
    explicit DevScope(int dev) { MBT_HIP(hipSetDevice(dev)); }
};

std::vector<int32_t> port_list(const mbt_array* arr, const int32_t* ports, int32_t nports) {
    std::vector<int32_t> pl;
    if (ports == nullptr) {
        MBT_REQUIRE(nports == -1 || nports == arr->g.P, "ports == NULL requires nports == -1");
        pl.resize(arr->g.P);
        for (int i = 0; i < arr->g.P; ++i) pl[i] = i;
    } else {
        MBT_REQUIRE(nports >= 1, "nports must be >= 1");
        pl.assign(ports, ports + nports);
        for (int32_t p : pl) MBT_REQUIRE(p >= 0 && p < arr->g.P, "port index out of range");
    }
    return pl;
}

}  // namespace

extern "C" {

void mbt_default_opts(mbt_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->prec = MBT_FP64;
    o->pc = MBT_PC_ELEMENT_BLOCK;
    o->restart = 50;
    o->tol = 1e-10;
    o->max_cycles = 400;
    o->refine_max = 3;
    o->refine_tol = 1e-9;
    o->inner_tol = 0;
    o->rhs_chunk = 0;
    o->flags = 0;
}

const char* mbt_last_error(void) { return g_err.c_str(); }

const char* mbt_version(void) { return "mbt 0.2 (gfx950; FP64, FP32, BF16 and FP16 MFMA per-bin products)"; }

mbt_status mbt_ctx_create(int32_t dev, size_t budget, mbt_ctx** out) {
    API_BEGIN
    MBT_REQUIRE(out != nullptr, "out is NULL");
    int n = 0;
    MBT_HIP(hipGetDeviceCount(&n));
    MBT_REQUIRE(dev >= 0 && dev < n, "no such HIP device");
    MBT_HIP(hipSetDevice(dev));
    noalloc_scratch_setup(dev);
    std::unique_ptr<mbt_ctx> c(new mbt_ctx());
    c->device = dev;
    size_t freeb = 0, totalb = 0;
    MBT_HIP(hipMemGetInfo(&freeb, &totalb));
    c->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
    c->cache_limit = c->budget / 8;
    c->main.reset(new Worker(dev));
    *out = c.release();
    API_END
}

void mbt_ctx_destroy(mbt_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    ctx->cache.clear();
    ctx->main.reset();
    delete ctx;
}

mbt_status mbt_array_create_dipole(mbt_ctx* ctx, const mbt_dipole* e, const mbt_lattice* l, mbt_array** out) {
    API_BEGIN
    MBT_REQUIRE(ctx && e && l && out, "NULL argument");
    std::unique_ptr<mbt_array> a(new mbt_array());
    a->g = make_geom(*e, *l);
    a->elem = *e;
    a->lat = *l;
    *out = a.release();
    API_END
}

mbt_status mbt_array_create_blocks(mbt_ctx* ctx, int32_t nx, int32_t ny, int32_t nbases, const double* T,
                                   mbt_array** out) {
    API_BEGIN
    MBT_REQUIRE(ctx && T && out, "NULL argument");
    std::unique_ptr<mbt_array> a(new mbt_array());
    a->g = make_geom_blocks(nx, ny, nbases);
    a->elem = mbt_dipole{0.0, 0.0, nbases};
    a->lat = mbt_lattice{nx, ny, a->g.dx, a->g.dy};
    const int64_t n = a->g.noff() * (int64_t)nbases * nbases;
    auto blk = std::make_shared<std::vector<double2>>((size_t)n);
    std::memcpy(blk->data(), T, sizeof(double2) * (size_t)n);
    for (const double2& v : *blk) MBT_REQUIRE(std::isfinite(v.x) && std::isfinite(v.y), "blocks must be finite");
    a->blocks = blk;
    static std::atomic<uint64_t> next_uid{1};
    a->uid = next_uid++;
    *out = a.release();
    API_END
}

mbt_status mbt_array_create_rwg(mbt_ctx* ctx, const mbt_rwg_mesh* mesh, const mbt_lattice* l, mbt_array** out) {
    API_BEGIN
    MBT_REQUIRE(ctx && mesh && l && out, "NULL argument");
    MBT_REQUIRE(l->dx > 0 && l->dy > 0 && std::isfinite(l->dx) && std::isfinite(l->dy),
                "lattice spacing must be positive");
    auto h = std::make_shared<RwgMesh>(rwg_from_mesh(*mesh));
    // Only elements at most one step apart get the closed-form static part; farther
    // ones are integrated by the point rule alone and must therefore be disjoint:
    // the triangles' extent along an axis with three or more elements stays below
    // two lattice steps.
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (const double2& v : h->tv) {
        x0 = std::min(x0, v.x);
        x1 = std::max(x1, v.x);
        y0 = std::min(y0, v.y);
        y1 = std::max(y1, v.y);
    }
    MBT_REQUIRE(l->nx < 3 || x1 - x0 < 2.0 * l->dx, "the element's x extent must stay below two lattice steps");
    MBT_REQUIRE(l->ny < 3 || y1 - y0 < 2.0 * l->dy, "the element's y extent must stay below two lattice steps");
    std::unique_ptr<mbt_array> a(new mbt_array());
    a->g = make_geom_blocks(l->nx, l->ny, h->M);
    a->g.dx = l->dx;
    a->g.dy = l->dy;
    a->g.port = h->port;
    a->g.pc = h->port.idx[0];
    a->elem = mbt_dipole{0.0, 0.0, h->M};
    a->lat = *l;
    a->rwg = h;
    static std::atomic<uint64_t> next_uid{2u << 30};
    a->uid = next_uid++;
    *out = a.release();
    API_END
}

mbt_status mbt_array_create_margin(mbt_ctx* ctx, int32_t nx, int32_t ny, int32_t nbases, const double* T,
                                   int32_t nmargin, const double* ZB, const double* ZC, mbt_array** out) {
    API_BEGIN
    MBT_REQUIRE(ctx && T && ZB && ZC && out, "NULL argument");
    MBT_REQUIRE(nmargin >= 1 && nmargin <= 2048, "nmargin must be within 1..2048");
    std::unique_ptr<mbt_array> a(new mbt_array());
    a->g = make_geom_blocks(nx, ny, nbases);
    a->g.Nc = nmargin;
    a->g.N = a->g.NA() + nmargin;
    a->elem = mbt_dipole{0.0, 0.0, nbases};
    a->lat = mbt_lattice{nx, ny, a->g.dx, a->g.dy};
    auto copy = [](const double* src, size_t n) {
        auto v = std::make_shared<std::vector<double2>>(n);
        std::memcpy(v->data(), src, sizeof(double2) * n);
        for (const double2& z : *v) MBT_REQUIRE(std::isfinite(z.x) && std::isfinite(z.y), "blocks must be finite");
        return v;
    };
    a->blocks = copy(T, (size_t)(a->g.noff() * (int64_t)nbases * nbases));
    a->zb = copy(ZB, (size_t)nmargin * (size_t)a->g.NA());
    a->zc = copy(ZC, (size_t)nmargin * (size_t)nmargin);
    static std::atomic<uint64_t> next_uid{1u << 30};
    a->uid = next_uid++;
    *out = a.release();
    API_END
}

void mbt_array_destroy(mbt_array* a) { delete a; }

mbt_status mbt_array_info(const mbt_array* a, int64_t* N, int32_t* P, int32_t* gx, int32_t* gy) {
    API_BEGIN
    MBT_REQUIRE(a != nullptr, "array is NULL");
    if (N) *N = a->g.N;
    if (P) *P = a->g.P;
    if (gx) *gx = a->g.Px;
    if (gy) *gy = a->g.Py;
    API_END
}

size_t mbt_footprint(const mbt_array* a, int32_t nrhs, const mbt_solve_opts* o) {
    if (!a || !o || nrhs < 1) return 0;
    try {
        const Geom& g = a->g;
        const size_t MM = (size_t)g.M * g.M;
        size_t opb = (size_t)g.noff() * MM * 16 + 2 * (size_t)g.bins() * MM * 16 + (size_t)g.P * MM * 16 * 2;
        if (o->prec != MBT_FP64) opb += 2 * (size_t)g.bins() * MM * 8 + (size_t)g.P * MM * 8;
        if (fmt16_of(o->prec) != kFmtNone) opb += (size_t)g.bins() * MM * 4;
        return solve_bytes(g, padded(nrhs, *o), *o) + opb;
    } catch (...) {
        return 0;
    }
}

mbt_status mbt_port_admittance(mbt_ctx* ctx, const mbt_array* arr, double s, const int32_t* ports, int32_t nports,
                               const mbt_solve_opts* opts, double* Y, int32_t* iters, mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts && Y, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    validate_opts(*opts);
    MBT_REQUIRE(s > 0 && std::isfinite(s), "freq_ratio must be positive");
    std::vector<int32_t> pl = port_list(arr, ports, nports);
    const int np = (int)pl.size();
    DBuf Yd;
    Yd.alloc(sizeof(double2) * arr->g.P * np);
    SolveOut so = admittance(ctx, arr, s, pl.data(), np, *opts, Yd.as<double2>(), *ctx->main, st, ctx->budget);
    MBT_HIP(hipMemcpy(Y, Yd.p, sizeof(double2) * arr->g.P * np, hipMemcpyDeviceToHost));
    if (iters) std::copy(so.iters.begin(), so.iters.end(), iters);
    return finish_status(so);
    API_END
}

mbt_status mbt_port_admittance_dev(mbt_ctx* ctx, const mbt_array* arr, double s, const int32_t* ports, int32_t nports,
                                   const mbt_solve_opts* opts, void* Ydev, void* stream, int32_t* iters, mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts && Ydev, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    validate_opts(*opts);
    std::vector<int32_t> pl = port_list(arr, ports, nports);
    hipStream_t user = (hipStream_t)stream;
    if (user) {
        // order the solve after prior work on the caller's stream
        hipEvent_t ev;
        MBT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        MBT_HIP(hipEventRecord(ev, user));
        MBT_HIP(hipStreamWaitEvent(ctx->main->stream, ev, 0));
        MBT_HIP(hipEventDestroy(ev));
    }
    SolveOut so = admittance(ctx, arr, s, pl.data(), (int)pl.size(), *opts, (double2*)Ydev, *ctx->main, st,
                             ctx->budget);
    if (iters) std::copy(so.iters.begin(), so.iters.end(), iters);
    return finish_status(so);
    API_END
}

static mbt_status solve_impl(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts* opts,
                             const double* theta, const double* phi, int32_t nscan, double z0, double* Zp, double* Za,
                             double* Gamma, double* Gamma_wave, mbt_stats* st) {
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    validate_opts(*opts);
    MBT_REQUIRE(s > 0 && std::isfinite(s), "freq_ratio must be positive");
    MBT_REQUIRE(nscan >= 0 && (nscan == 0 || (theta && phi && Za && Gamma)), "scan arrays missing");
    MBT_REQUIRE(z0 > 0, "z0 must be positive");
    SolveOut so = solve_frequency(ctx, arr, s, *opts, ctx->budget, theta, phi, nscan, z0, Zp, Za, Gamma, Gamma_wave,
                                  *ctx->main, st);
    return finish_status(so);
}

mbt_status mbt_port_impedance(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts* opts, double* Zp,
                              mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts && Zp, "NULL argument");
    return solve_impl(ctx, arr, s, opts, nullptr, nullptr, 0, 50.0, Zp, nullptr, nullptr, nullptr, st);
    API_END
}

mbt_status mbt_solve(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts* opts, const double* theta,
                     const double* phi, int32_t nscan, double z0, double* Zp, double* Za, double* Gamma,
                     double* Gamma_wave, mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts, "NULL argument");
    return solve_impl(ctx, arr, s, opts, theta, phi, nscan, z0, Zp, Za, Gamma, Gamma_wave, st);
    API_END
}

mbt_status mbt_scan_solve(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts* opts,
                          const double* theta, const double* phi, int32_t nscan, double z0, int32_t center, double* Ip,
                          double* Za, double* Gamma, int32_t* iters, mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts && theta && phi && Za && Gamma, "NULL argument");
    MBT_REQUIRE(nscan >= 1, "nscan must be >= 1");
    MBT_REQUIRE(s > 0 && std::isfinite(s), "freq_ratio must be positive");
    MBT_REQUIRE(z0 > 0 && std::isfinite(z0), "z0 must be positive");
    MBT_REQUIRE(!arr->blocks, "scan excitations need element positions: dipole or RWG arrays only");
    for (int r = 0; r < nscan; ++r)
        MBT_REQUIRE(std::isfinite(theta[r]) && std::isfinite(phi[r]), "scan angles must be finite");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    validate_opts(*opts);
    const Geom& g = arr->g;
    const int c = center < 0 ? (g.ny / 2) * g.nx + g.nx / 2 : center;
    MBT_REQUIRE(c < g.P, "center out of range");
    SolveOut so = scan_solve(ctx, arr, s, *opts, ctx->budget, theta, phi, nscan, z0, c, Ip, Za, Gamma, *ctx->main, st);
    if (iters)
        for (int r = 0; r < nscan; ++r) iters[r] = so.iters[r];
    return finish_status(so);
    API_END
}

mbt_status mbt_active_dev_noalloc(mbt_ctx* ctx, const mbt_array* arr, double s, const void* Zp_dev, int32_t center,
                                  const double* theta_dev, const double* phi_dev, int32_t nscan, double z0,
                                  void* Za_dev, void* Gamma_dev, void* Gamma_wave_dev, void* stream) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && Zp_dev && theta_dev && phi_dev && Za_dev && Gamma_dev, "NULL argument");
    MBT_REQUIRE(nscan >= 1, "nscan must be >= 1");
    MBT_REQUIRE(s > 0 && z0 > 0 && std::isfinite(s) && std::isfinite(z0), "freq_ratio and z0 must be positive");
    MBT_REQUIRE(!arr->blocks, "scan quantities need element positions: dipole arrays only");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    const Geom& g = arr->g;
    const int P = g.P;
    const int c = center < 0 ? (g.ny / 2) * g.nx + g.nx / 2 : center;
    MBT_REQUIRE(c < P, "center out of range");
    hipStream_t str = stream ? static_cast<hipStream_t>(stream) : ctx->main->stream;
    const double2* Zp = static_cast<const double2*>(Zp_dev);
    double2* S = nullptr;
    if (Gamma_wave_dev) {
        const size_t need = noalloc_need(P);
        MBT_REQUIRE(need <= (size_t)MBT_NOALLOC_SCRATCH_BYTES,
                    "the wave-excited ARC of " + std::to_string(P) + " ports needs " + std::to_string(need) +
                        " bytes of device scratch; the allocation-free entry point has " +
                        std::to_string((size_t)MBT_NOALLOC_SCRATCH_BYTES) + " (at most 1024 ports)");
        char* base = noalloc_scratch(ctx->device);
        MBT_REQUIRE(base != nullptr, "device scratch not set up (no context created on this device)");
        auto take = [&](size_t b) {
            char* p = base;
            base += (b + 255) & ~(size_t)255;
            return p;
        };
        double2* work = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)P * P));
        S = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)P * P));
        double2* colbuf = reinterpret_cast<double2*>(take(sizeof(double2) * (size_t)P));
        int* piv = reinterpret_cast<int*>(take(sizeof(int) * (size_t)P));
        int* src = reinterpret_cast<int*>(take(sizeof(int) * (size_t)P));
        int* flag = reinterpret_cast<int*>(take(sizeof(int)));
        s_matrix_dev_perm(Zp, S, work, P, z0, colbuf, piv, src, flag, ctx->main->host_count, str);
    }
    scans(g, 2.0 * M_PI * s, Zp, S, c, theta_dev, phi_dev, nscan, z0, static_cast<double2*>(Za_dev),
          static_cast<double2*>(Gamma_dev), Gamma_wave_dev ? static_cast<double2*>(Gamma_wave_dev) : nullptr, str);
    MBT_HIP(hipStreamSynchronize(str));
    API_END
}

mbt_status mbt_active(mbt_ctx* ctx, const mbt_array* arr, double s, const double* Zp, int32_t center,
                      const double* theta, const double* phi, int32_t nscan, double z0, double* Za, double* Gamma,
                      double* Gamma_wave) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && Zp && theta && phi && Za && Gamma, "NULL argument");
    MBT_REQUIRE(nscan >= 1, "nscan must be >= 1");
    MBT_REQUIRE(s > 0 && z0 > 0, "freq_ratio and z0 must be positive");
    MBT_REQUIRE(!arr->blocks, "scan quantities need element positions: dipole arrays only");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    const Geom& g = arr->g;
    const int P = g.P;
    const int c = center < 0 ? (g.ny / 2) * g.nx + g.nx / 2 : center;
    MBT_REQUIRE(c < P, "center out of range");
    hipStream_t str = ctx->main->stream;
    DBuf Zd, Sd, Wd, aux;
    Zd.alloc(sizeof(double2) * P * P);
    aux.alloc(sizeof(double2) * P + sizeof(int) * (P + 8) + sizeof(double) * 2 * nscan + sizeof(double2) * 3 * nscan + 1024);
    char* ab = aux.as<char>();
    double2* colbuf = (double2*)ab;
    int* piv = (int*)(ab + sizeof(double2) * P);
    int* flag = piv + P;
    double* dth = (double*)(((uintptr_t)(flag + 8) + 255) & ~(uintptr_t)255);
    double* dph = dth + nscan;
    double2* dout = (double2*)(dph + nscan);
    MBT_HIP(hipMemcpyAsync(Zd.p, Zp, sizeof(double2) * P * P, hipMemcpyHostToDevice, str));
    if (Gamma_wave) {
        Sd.alloc(sizeof(double2) * P * P);
        Wd.alloc(sizeof(double2) * P * P);
        s_matrix(Zd.as<double2>(), Sd.as<double2>(), Wd.as<double2>(), P, z0, colbuf, piv, flag, str);
    }
    MBT_HIP(hipMemcpyAsync(dth, theta, sizeof(double) * nscan, hipMemcpyHostToDevice, str));
    MBT_HIP(hipMemcpyAsync(dph, phi, sizeof(double) * nscan, hipMemcpyHostToDevice, str));
    scans(g, 2.0 * M_PI * s, Zd.as<double2>(), Gamma_wave ? Sd.as<double2>() : nullptr, c, dth, dph, nscan, z0, dout,
          dout + nscan, Gamma_wave ? dout + 2 * nscan : nullptr, str);
    MBT_HIP(hipMemcpyAsync(Za, dout, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
    MBT_HIP(hipMemcpyAsync(Gamma, dout + nscan, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
    if (Gamma_wave) MBT_HIP(hipMemcpyAsync(Gamma_wave, dout + 2 * nscan, sizeof(double2) * nscan, hipMemcpyDeviceToHost, str));
    MBT_HIP(hipStreamSynchronize(str));
    API_END
}

// ------------------------------------------------------------------ test hooks
mbt_status mbt_dbg_fill_blocks(mbt_ctx* ctx, const mbt_array* arr, double s, double* T) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && T, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    auto op = get_op(ctx, arr, s, false, MBT_FP64, *ctx->main);
    MBT_HIP(hipMemcpy(T, op->T.p, op->T.bytes, hipMemcpyDeviceToHost));
    API_END
}

mbt_status mbt_dbg_matvec(mbt_ctx* ctx, const mbt_array* arr, double s, int32_t prec, int32_t opz, const double* x,
                          int32_t R, double* y) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && x && y && R >= 1, "bad argument");
    MBT_REQUIRE(opz >= 0 && opz <= 2, "op must be 0, 1 or 2");
    MBT_REQUIRE(prec >= MBT_FP64 && prec <= MBT_FP16, "unknown precision");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    const Geom& g = arr->g;
    Worker& wk = *ctx->main;
    auto op = get_op(ctx, arr, s, false, prec, wk);
    const int64_t NR = g.N * R;
    DBuf hx, dx, dy, Xh, Yh, tmp, f1, f2, mscr;
    mscr.alloc(margin_scratch_bytes(g, R));
    hx.alloc(sizeof(double2) * NR);
    dx.alloc(sizeof(double2) * NR);
    dy.alloc(sizeof(double2) * NR);
    Xh.alloc(sizeof(double2) * g.bins() * g.M * R);
    Yh.alloc(sizeof(double2) * g.bins() * g.M * R);
    tmp.alloc(sizeof(double2) * NR);
    MBT_HIP(hipMemcpyAsync(hx.p, x, sizeof(double2) * NR, hipMemcpyHostToDevice, wk.stream));
    transpose_nr(hx.as<double2>(), dx.as<double2>(), g.N, R, true, wk.stream);
    if (prec == MBT_FP64) {
        OpV<double> ov = make_view<double>(*op, MBT_PC_ELEMENT_BLOCK, Xh.p, Yh.p, tmp.p, R, wk.stream);
        attach_margin(ov, mscr.p);
        if (opz == 2) {
            zmul<double>(ov, 0, dx.as<double2>(), tmp.as<double2>());
            zmul<double>(ov, 1, tmp.as<double2>(), dy.as<double2>());
        } else {
            zmul<double>(ov, opz, dx.as<double2>(), dy.as<double2>());
        }
    } else {
        f1.alloc(sizeof(float2) * NR);
        f2.alloc(sizeof(float2) * NR);
        OpV<float> ov = make_view<float>(*op, MBT_PC_ELEMENT_BLOCK, Xh.p, Yh.p, tmp.p, R, wk.stream, fmt16_of(prec));
        attach_margin(ov, mscr.p);
        // The 16-bit spectra carry no scale of their own: columns go in with unit norm, as
        // the solvers' Krylov vectors do (binary16 overflows at 65504), and come out rescaled.
        DBuf cs;
        std::vector<double> hs(2 * (size_t)R, 1.0);
        if (prec != MBT_FP32) {
            for (int r = 0; r < R; ++r) {
                double ss = 0;
                for (int64_t i = 0; i < 2 * g.N; ++i) ss += x[2 * g.N * r + i] * x[2 * g.N * r + i];
                const double nrm = std::sqrt(ss);
                if (nrm > 0 && std::isfinite(nrm)) {
                    hs[r] = 1.0 / nrm;
                    hs[R + r] = nrm;
                }
            }
            cs.alloc(sizeof(double) * 2 * R);
            MBT_HIP(hipMemcpyAsync(cs.p, hs.data(), sizeof(double) * 2 * R, hipMemcpyHostToDevice, wk.stream));
            scale_columns_d(dx.as<double2>(), cs.as<double>(), g.N, R, wk.stream);
        }
        convert<double2, float2>(dx.as<double2>(), f1.as<float2>(), NR, wk.stream);
        if (opz == 2) {
            zmul<float>(ov, 0, f1.as<float2>(), ov.tmp);
            zmul<float>(ov, 1, ov.tmp, f2.as<float2>());
        } else {
            zmul<float>(ov, opz, f1.as<float2>(), f2.as<float2>());
        }
        convert<float2, double2>(f2.as<float2>(), dy.as<double2>(), NR, wk.stream);
        if (prec != MBT_FP32) scale_columns_d(dy.as<double2>(), cs.as<double>() + R, g.N, R, wk.stream);
    }
    transpose_nr(dy.as<double2>(), hx.as<double2>(), g.N, R, false, wk.stream);
    MBT_HIP(hipMemcpyAsync(y, hx.p, sizeof(double2) * NR, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    API_END
}

mbt_status mbt_dbg_precond_apply(mbt_ctx* ctx, const mbt_array* arr, double s, int32_t pc, const double* x, int32_t R,
                                 double* y) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && x && y && R >= 1, "bad argument");
    MBT_REQUIRE(pc == MBT_PC_NORMAL_EQ || pc == MBT_PC_ELEMENT_BLOCK, "unknown preconditioner");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    const Geom& g = arr->g;
    Worker& wk = *ctx->main;
    auto op = get_op(ctx, arr, s, pc == MBT_PC_NORMAL_EQ, MBT_FP64, wk);
    const int64_t NR = g.N * R;
    DBuf hx, dx, dy;
    hx.alloc(sizeof(double2) * NR);
    dx.alloc(sizeof(double2) * NR);
    dy.alloc(sizeof(double2) * NR);
    MBT_HIP(hipMemcpyAsync(hx.p, x, sizeof(double2) * NR, hipMemcpyHostToDevice, wk.stream));
    transpose_nr(hx.as<double2>(), dx.as<double2>(), g.N, R, true, wk.stream);
    OpV<double> ov = make_view<double>(*op, pc, nullptr, nullptr, nullptr, R, wk.stream);
    pinv<double>(ov, dx.as<double2>(), dy.as<double2>());   // the margin block needs no scratch
    transpose_nr(dy.as<double2>(), hx.as<double2>(), g.N, R, false, wk.stream);
    MBT_HIP(hipMemcpyAsync(y, hx.p, sizeof(double2) * NR, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    API_END
}

mbt_status mbt_dbg_precond_blocks(mbt_ctx* ctx, const mbt_array* arr, double s, int32_t pc, double* Pb) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && Pb, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    const Geom& g = arr->g;
    Worker& wk = *ctx->main;
    auto op = get_op(ctx, arr, s, false, MBT_FP64, wk);
    const int64_t MM = (int64_t)g.M * g.M;
    if (pc == MBT_PC_ELEMENT_BLOCK) {
        const int64_t center = (int64_t)(g.ny - 1) * g.nox + (g.nx - 1);
        MBT_HIP(hipMemcpy(Pb, op->T.as<double2>() + center * MM, sizeof(double2) * MM, hipMemcpyDeviceToHost));
    } else {
        DBuf G, P;
        G.alloc(sizeof(double2) * g.noff() * MM);
        P.alloc(sizeof(double2) * g.P * MM);
        gram_blocks(g, op->T.as<double2>(), G.as<double2>(), wk.stream);
        window_sum(g, G.as<double2>(), P.as<double2>(), wk.stream);
        MBT_HIP(hipMemcpyAsync(Pb, P.p, sizeof(double2) * g.P * MM, hipMemcpyDeviceToHost, wk.stream));
        MBT_HIP(hipStreamSynchronize(wk.stream));
    }
    API_END
}

mbt_status mbt_dbg_solve(mbt_ctx* ctx, const mbt_array* arr, double s, const mbt_solve_opts* opts, const double* V,
                         int32_t R, double* I, int32_t* iters, mbt_stats* st) {
    API_BEGIN
    MBT_REQUIRE(ctx && arr && opts && V && I && R >= 1, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    validate_opts(*opts);
    const Geom& g = arr->g;
    Worker& wk = *ctx->main;
    const double t0 = now_s();
    auto op = get_op(ctx, arr, s, opts->pc == MBT_PC_NORMAL_EQ, opts->prec, wk);
    const int64_t NR = g.N * R;
    wk.ensure(solve_bytes(g, R, *opts) + 3 * sizeof(double2) * NR);
    DevArena arena;
    arena.base = wk.ws.as<char>();
    arena.cap = wk.ws.bytes;
    double2* hx = arena.get<double2>(NR);
    double2* dV = arena.get<double2>(NR);
    double2* dX = arena.get<double2>(NR);
    MBT_HIP(hipMemcpyAsync(hx, V, sizeof(double2) * NR, hipMemcpyHostToDevice, wk.stream));
    transpose_nr(hx, dV, g.N, R, true, wk.stream);
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t1 = now_s();
    SolveOut so = solve_rhs(*op, *opts, dV, R, dX, wk, arena);
    MBT_HIP(hipStreamSynchronize(wk.stream));
    const double t2 = now_s();
    transpose_nr(dX, hx, g.N, R, false, wk.stream);
    MBT_HIP(hipMemcpyAsync(I, hx, sizeof(double2) * NR, hipMemcpyDeviceToHost, wk.stream));
    MBT_HIP(hipStreamSynchronize(wk.stream));
    if (iters) std::copy(so.iters.begin(), so.iters.end(), iters);
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->nrhs = R;
        st->nconverged = so.nconv;
        st->cycles = so.cycles;
        st->outer_steps = so.outer;
        st->iters_min = *std::min_element(so.iters.begin(), so.iters.end());
        st->iters_max = *std::max_element(so.iters.begin(), so.iters.end());
        for (int v : so.iters) st->iters_total += v;
        st->matvecs = so.matvecs;
        st->true_relres_max = so.relres_max;
        st->t_setup = t1 - t0;
        st->t_solve = t2 - t1;
    }
    return finish_status(so);
    API_END
}

mbt_status mbt_dbg_inverse(mbt_ctx* ctx, const double* A, int32_t n, double* Ainv) {
    API_BEGIN
    MBT_REQUIRE(ctx && A && Ainv && n >= 1, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->api_mu);
    DevScope ds(ctx->device);
    hipStream_t str = ctx->main->stream;
    DBuf Ad, Od, aux;
    Ad.alloc(sizeof(double2) * n * n);
    Od.alloc(sizeof(double2) * n * n);
    aux.alloc(sizeof(double2) * n + sizeof(int) * (n + 8));
    MBT_HIP(hipMemcpyAsync(Ad.p, A, sizeof(double2) * n * n, hipMemcpyHostToDevice, str));
    gj_inverse(Ad.as<double2>(), Od.as<double2>(), n, aux.as<double2>(), (int*)(aux.as<double2>() + n),
               (int*)(aux.as<double2>() + n) + n, str);
    MBT_HIP(hipMemcpyAsync(Ainv, Od.p, sizeof(double2) * n * n, hipMemcpyDeviceToHost, str));
    MBT_HIP(hipStreamSynchronize(str));
    API_END
}

}  // extern "C"

/*
 * mbt.h -- C ABI of the MI355X multilevel-block-Toeplitz (MBT) finite-array
 * Method-of-Moments solver.
 *
 * Problem (paper Sec. II-D, eq. (eqProb)): Z I = V for a regular nx x ny
 * lattice of identical elements with M bases each, for every port excitation
 * at once (one feed per element, F = 1).  Z is multilevel block-Toeplitz
 * (Sec. II-A): the M x M block between two elements depends only on their
 * lattice offset, so only the (2ny-1)(2nx-1) unique blocks are stored and
 * Z x is applied by a two-level FFT over the circulant embedding (eq. (multL)),
 * Z^H y from the same stored spectra (eq. (multCom)).  Outputs are the port
 * admittance / open-circuit port impedance (eq. (passZ)), the active
 * impedance (eqs. (actZ), (actZmat)) and active reflection coefficient
 * (eq. (ARC)) of the center element, and the wave-excited reflection
 * coefficient from the phased S-sum (Sec. II-E with eq. (S2Z)).
 *
 * Elements: a z-directed thin-wire dipole (length, radius in wavelengths at the
 * reference frequency f0; nbases odd rooftops; port at the center rooftop),
 * filled by Galerkin EFIE with the reduced kernel exp(-jkR)/(4 pi R),
 * R = sqrt(rho^2 + (z-z')^2 + a^2), and 4-point Gauss-Legendre per segment;
 * or a planar element given by its triangle mesh, discretised with RWG
 * functions (paper Sec. I, Sec. II-B), port at a delta gap across feed edges
 * (mbt_array_create_rwg).
 *
 * Conventions
 *  - complex numbers are interleaved FP64 {re, im} pairs (C99 double _Complex,
 *    numpy complex128); a "complex array of n entries" is 2n doubles;
 *  - host matrices are column-major: A[i + ld*j];
 *  - unknown index n = e*M + p, element e = iy*nx + ix at (ix*dx, iy*dy);
 *    port j is element j (dipoles and block arrays: its center basis
 *    p_c = (M-1)/2; RWG elements: the gap across the feed edges);
 *  - the center element is (nx/2, ny/2) (integer division);
 *  - a frequency is the ratio s = f/f0 (wavenumber k = 2 pi s);
 *  - unless stated, pointers are host memory owned by the caller; handles
 *    are owned by the library and released by their _destroy call;
 *  - every call returns an mbt_status; on error mbt_last_error() returns a
 *    thread-local message; on MBT_ENOCONV outputs still hold the last iterate;
 *  - one context is not re-entrant (serialize calls on it); the server is
 *    internally threaded.
 */
#ifndef MBT_H
#define MBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MBT_OK = 0,
    MBT_EINVAL = -1,      /* invalid argument (geometry, sizes, ports, options) */
    MBT_ENOMEM = -2,      /* device-memory footprint exceeds the context budget */
    MBT_ENOCONV = -3,     /* max_cycles reached; outputs hold the last iterate */
    MBT_EDEVICE = -4,     /* HIP runtime error */
    MBT_EBUSY = -5,       /* server queue full */
    MBT_EBREAKDOWN = -6,  /* non-finite value met in the Krylov recurrence */
    MBT_ETIMEOUT = -7     /* mbt_server_wait timed out */
} mbt_status;

/* Precision of the FFT-Toeplitz operator inside the Krylov solve.
 * MBT_FP64: everything FP64.  MBT_FP32: the lattice FFTs and the per-bin block
 * products run in FP32 (FP32 MFMA, FP32 accumulation).  MBT_BF16 / MBT_FP16: as
 * MBT_FP32, but the forward FFT stores the spectrum X^ in 16-bit complex and
 * the per-bin products take X^ and the block spectra C^ in bfloat16 / binary16
 * on the 16x16x32 MFMA with FP32 accumulation and FP32 output.  In every
 * reduced precision the Krylov basis is kept in reduced precision (see
 * MBT_FLAG_FP32_BASIS) with FP64 dot products, Givens rotations are FP64, the
 * preconditioner apply is FP32, and FP64 iterative refinement with an FP64
 * residual recovers the accuracy (inner tolerance by default 1e-4 for FP32,
 * 1e-3 for FP16, 1e-2 for BF16).  A refinement step that raises a RHS's FP64
 * residual is taken back (a correction over 1e3 times the iterate, a runaway
 * inner solve, is dropped before it is added) and that RHS stops refining, so
 * the returned currents are the best iterate; it then counts as not converged
 * unless it met refine_tol. */
typedef enum { MBT_FP64 = 0, MBT_FP32 = 1, MBT_BF16 = 2, MBT_FP16 = 3 } mbt_prec;

/* Preconditioning strategy.
 * MBT_PC_NORMAL_EQ:     GMRES on P^{-1} Z^H Z I = P^{-1} Z^H V, P the block
 *                       diagonal of Z^H Z (Sec. II-B eq. (precondTBBT); built as in
 *                       Sec. III-A, eqs. (precondA), (precond)).
 * MBT_PC_ELEMENT_BLOCK: GMRES on P_K^{-1} Z I = P_K^{-1} V, P_K the element
 *                       self blocks of Z (the older strategy of Table I). */
typedef enum { MBT_PC_NORMAL_EQ = 0, MBT_PC_ELEMENT_BLOCK = 1 } mbt_pc;

typedef struct { double length, radius; int32_t nbases; } mbt_dipole;
typedef struct { int32_t nx, ny; double dx, dy; } mbt_lattice;

typedef struct {
    int32_t prec;         /* mbt_prec */
    int32_t pc;           /* mbt_pc */
    int32_t restart;      /* GMRES restart length m (>= 1), default 50 (PCG: iteration cap restart * max_cycles) */
    double tol;           /* FP64 path: relative preconditioned residual, default 1e-10 */
    int32_t max_cycles;   /* restart cycles per (inner) solve, default 400 */
    int32_t refine_max;   /* reduced precision: max outer refinement steps, default 3 */
    double refine_tol;    /* reduced precision: outer stop on ||V - Z I|| / ||V||, default 1e-9 */
    double inner_tol;     /* reduced precision: inner relative tolerance (0 = by precision) */
    int32_t rhs_chunk;    /* RHS per batched solve (0 = all at once, within the budget) */
    int32_t flags;        /* MBT_FLAG_* bits, default 0 */
} mbt_solve_opts;

/* mbt_solve_opts.flags: rebuild blocks, spectra and preconditioner for this
 * call instead of using (and filling) the context's per-(array, frequency)
 * cache; used to time the complete path. */
#define MBT_FLAG_NO_CACHE 1
/* mbt_solve_opts.flags: orthogonalise the Arnoldi basis by classical
 * Gram-Schmidt applied twice in three sweeps over the basis (CGS2) instead of
 * the default delayed reorthogonalisation (DCGS2, two sweeps; same iterates in
 * exact arithmetic). */
#define MBT_FLAG_CGS2 2
/* mbt_solve_opts.flags, reduced precision: keep the inner solve's Krylov basis
 * in FP32.  By default it is stored packed, each FP32 component rounded to its
 * top 24 bits (unit roundoff 2^-16, three quarters of the bytes); an odd
 * number of ports is then solved with one port repeated. */
#define MBT_FLAG_FP32_BASIS 4
/* mbt_solve_opts.flags: solve by preconditioned conjugate gradients (Sec. II-C)
 * instead of GMRES: CG on the normal equations Z^H Z I = Z^H V with the
 * preconditioner P_A (pc must be MBT_PC_NORMAL_EQ), stopping when the relative
 * residual of the split system P^{-1/2} Z^H Z P^{-H/2} W = P^{-1/2} Z^H V
 * (eq. (precond)) is <= tol (inner_tol in the reduced-precision inner solves);
 * at most restart * max_cycles iterations.  Keeps four work vectors instead of
 * a Krylov basis. */
#define MBT_FLAG_PCG 8
/* mbt_solve_opts.flags: solve Z I = V by conjugate orthogonal conjugate
 * gradients (COCG: CG with the bilinear form x^T y, for complex symmetric
 * systems; van der Vorst and Melissen, 1990) with the element-block
 * preconditioner P_K (pc must be MBT_PC_ELEMENT_BLOCK; Z and P_K are complex
 * symmetric by Galerkin reciprocity), stopping when ||V - Z I|| <= tol ||V||
 * (inner_tol in the reduced-precision inner solves); at most
 * restart * max_cycles iterations.  One operator application per iteration
 * and four work vectors instead of a Krylov basis.  Not in the paper. */
#define MBT_FLAG_COCG 16

typedef struct {
    int32_t nrhs;             /* RHS solved */
    int32_t nconverged;       /* RHS that met the tolerance */
    int32_t cycles;           /* restart cycles (max over RHS, summed over outer steps; PCG: 1 per solve) */
    int32_t outer_steps;      /* refinement steps (1 for FP64) */
    int32_t iters_min, iters_max;
    int64_t iters_total;      /* Arnoldi (or PCG) steps summed over RHS */
    int64_t matvecs;          /* batched operator applications (Z or Z^H, each counted) */
    double true_relres_max;   /* max over RHS of ||V - Z I|| / ||V||, FP64 */
    double t_setup, t_solve, t_extract;   /* seconds (device-synchronised phases) */
} mbt_stats;

typedef struct mbt_ctx mbt_ctx;
typedef struct mbt_array mbt_array;

/* Defaults listed in mbt_solve_opts. */
void mbt_default_opts(mbt_solve_opts* opts);

/* Context on HIP device `hip_device`; hbm_budget_bytes = 0 means 90% of free
 * device memory.  Errors: MBT_EINVAL (bad device), MBT_EDEVICE. */
mbt_status mbt_ctx_create(int32_t hip_device, size_t hbm_budget_bytes, mbt_ctx** out);
void mbt_ctx_destroy(mbt_ctx* ctx);

/* Thread-local description of the last error on this thread ("" if none). */
const char* mbt_last_error(void);

/* Library build string (kernels, target). */
const char* mbt_version(void);

/* Array geometry.  MBT_EINVAL: nbases even or < 1, radius <= 0, length <= 0,
 * nx/ny < 1 or > 1024, dx/dy <= 0. */
mbt_status mbt_array_create_dipole(mbt_ctx* ctx, const mbt_dipole* elem, const mbt_lattice* lat,
                                   mbt_array** out);
/* Array whose operator is given by its unique lattice blocks instead of an
 * element fill (Sec. II-A: one M x M block per offset between a test and a
 * source element).  T holds (2ny-1)(2nx-1) blocks of nbases x nbases complex
 * values, T[((dy+ny-1)*(2nx-1) + (dx+nx-1))*M*M + p*M + q] the coupling of
 * basis p of an element to basis q of the element -d = (-dx, -dy) away, i.e.
 * Z[t][s] = T[t - s]; copied at the call.  The operator does not depend on
 * freq_ratio.  Port j is basis (M-1)/2 of element j.  Limits: nbases 1..128,
 * nx, ny 1..64; more than 32 bases: FP64 or FP32 products; no scans (no element
 * positions).  Errors: MBT_EINVAL (sizes, non-finite values). */
mbt_status mbt_array_create_blocks(mbt_ctx* ctx, int32_t nx, int32_t ny, int32_t nbases, const double* T,
                                   mbt_array** out);
/* Planar element in the plane z = 0, given by its triangle mesh in the element
 * frame (wavelengths at f0).  vert: nvert (x, y) pairs; tri: ntri vertex-index
 * triples; port_edges: nport_edges vertex-index pairs, the edges of the feed
 * gap; port_dir: direction of the gap field in the element plane.  All copied
 * at the call. */
typedef struct {
    int32_t nvert;
    const double* vert;
    int32_t ntri;
    const int32_t* tri;
    int32_t nport_edges;
    const int32_t* port_edges;
    double port_dir[2];
} mbt_rwg_mesh;

/* Array of planar elements (paper Sec. I, Sec. II-B: elements discretised with
 * Rao-Wilton-Glisson functions; the paper gives no fill rules, so these are
 * this library's).  Basis m is the m-th interior edge (an edge of exactly two
 * triangles) in increasing (smaller vertex, larger vertex) order, with
 * f_m = +-(l_m / 2A)(r - v) on its two triangles, + on the lower-index one (v
 * the vertex opposite the edge).  Blocks: Galerkin EFIE
 * Z_mn = j k eta <<f_m . f_n, G>> - j (eta/k) <<div f_m, div f_n, G>>,
 * G = exp(-jkR)/(4 pi R), Radon's seven-point rule on every triangle, and for
 * elements at most one lattice step apart in x and y the static part of the
 * source integral in closed form (coplanar potential integrals, Wilton et al.
 * 1984).  Port: a delta gap; gap voltage V drives basis m of a feed edge with
 * V sign_m l_m, and the gap current is sum sign_m l_m I_m (sign_m = +1 when the
 * basis's + -> - direction has a positive component along port_dir); Y_p and
 * Z_p are in these gap voltages and currents.  Limits: 1..128 interior edges,
 * 2..256 triangles, 3..4096 vertices, 1..8 feed edges, nx, ny 1..64; the
 * triangles' extent along x (y) below 2 dx (2 dy) when nx (ny) >= 3, so that
 * elements two or more steps apart, which the point rule alone integrates, are
 * disjoint; 16-bit products only up to 32 bases.  Errors: MBT_EINVAL (sizes,
 * non-finite or degenerate geometry, an edge of more than two triangles, a feed
 * edge that is not interior or is parallel to port_dir, an element too large for
 * its lattice). */
mbt_status mbt_array_create_rwg(mbt_ctx* ctx, const mbt_rwg_mesh* mesh, const mbt_lattice* lat, mbt_array** out);

/* Array whose impedance matrix has a margin besides its elements (Sec. II-A
 * eq. (Zblock)): Z = [[Z_A, Z_B^T], [Z_B, Z_C]], Z_A the block-Toeplitz element
 * interaction given by its unique blocks T as in mbt_array_create_blocks, and
 * nmargin further unknowns (after the nx*ny*nbases element unknowns) with the
 * element-margin coupling ZB (nmargin x nx*ny*nbases complex, row-major) and the
 * margin's own interaction ZC (nmargin x nmargin, row-major); all copied at the
 * call.  Ports are the element ports; the margin carries no excitation.  The
 * normal-equation strategy solves Z^H Z I = Z^H V (eq. (Z2)) with
 * P = blkdiag(P_A, P_C), P_A from the diagonal blocks of Z_A^H Z_A and
 * P_C = Z_B^* Z_B^T + Z_C^H Z_C (Sec. III-A, eq. (precond)); the element-block
 * strategy uses blkdiag(T[0], ..., T[0], Z_C).  Limits as
 * mbt_array_create_blocks, nmargin 1..2048, FP64 or FP32 products.  Errors:
 * MBT_EINVAL (sizes, non-finite values). */
mbt_status mbt_array_create_margin(mbt_ctx* ctx, int32_t nx, int32_t ny, int32_t nbases, const double* T,
                                   int32_t nmargin, const double* ZB, const double* ZC, mbt_array** out);
void mbt_array_destroy(mbt_array* arr);

/* Sizes: unknowns N = nx*ny*M (+ nmargin), ports P = nx*ny, FFT grid (gx, gy) >= (2nx-1, 2ny-1). */
mbt_status mbt_array_info(const mbt_array* arr, int64_t* nunknowns, int32_t* nports, int32_t* gx,
                          int32_t* gy);

/* Device-memory estimate (bytes) of one batched solve of `nrhs` RHS. */
size_t mbt_footprint(const mbt_array* arr, int32_t nrhs, const mbt_solve_opts* opts);

/* Port admittance columns (Sec. II-D eq. (eqProb) with one unit delta-gap
 * excitation per column, F = 1): unit voltage at each port in `ports`
 * (ports == NULL and nports == -1: all P ports, in order), every other port
 * shorted.  Y (P x nports, column-major, complex) receives the port-basis
 * currents: Y[i + P*j] = I(port i) for excitation ports[j].  iters (nports, may
 * be NULL) receives per-RHS Arnoldi-step counts (summed over refinement steps).
 * Errors: MBT_EINVAL (freq_ratio <= 0, port out of range, restart < 1),
 * MBT_ENOMEM, MBT_ENOCONV, MBT_EDEVICE. */
mbt_status mbt_port_admittance(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio,
                               const int32_t* ports, int32_t nports, const mbt_solve_opts* opts,
                               double* Y, int32_t* iters, mbt_stats* stats);

/* Same, with Y a device pointer (P x nports complex, column-major) and the
 * work ordered on HIP stream `stream` (NULL: the context stream).  The call
 * returns after the work completes. */
mbt_status mbt_port_admittance_dev(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio,
                                   const int32_t* ports, int32_t nports, const mbt_solve_opts* opts,
                                   void* Y_dev, void* stream, int32_t* iters, mbt_stats* stats);

/* Full open-circuit port impedance (Sec. II-E eq. (passZ)): Z_p = Y_p^{-1}
 * (P x P complex, column-major), the inverse of the short-circuit admittance
 * that delta-gap excitation gives, on the device in FP64.  Errors as for
 * mbt_port_admittance; MBT_EDEVICE if Y_p is singular. */
mbt_status mbt_port_impedance(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio,
                              const mbt_solve_opts* opts, double* Zp, mbt_stats* stats);

/* End to end for one frequency: geometry, lattice, frequency and all port
 * excitations in (eq. (eqProb)); Z_p (eq. (passZ); P x P, may be NULL), and for
 * each of the nscan directions (theta, phi radians) the center-element active
 * impedance Za (eqs. (actZ), (actZmat)), ARC Gamma = (Za - z0)/(Za + z0)
 * (eq. (ARC)) and the wave-excited Gamma_wave, the phased S-sum of Sec. II-E
 * with S from eq. (S2Z) (may be NULL), out.  The port currents are phased to
 * steer the main beam at (theta, phi): I_e = exp(-j k (x_e u + y_e v)),
 * u = sin(theta) cos(phi), v = sin(theta) sin(phi), for the exp(-jkR) kernel of
 * the fill.  Everything after the solve (Y_p^{-1}, S, scans) runs on the GPU in
 * FP64.  Errors as for mbt_port_admittance; MBT_EINVAL for nscan < 0 or
 * missing outputs, or scans requested of a block-defined array. */
mbt_status mbt_solve(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, const mbt_solve_opts* opts,
                     const double* theta, const double* phi, int32_t nscan, double z0, double* Zp,
                     double* Za, double* Gamma, double* Gamma_wave, mbt_stats* stats);

/* Phased voltage excitation (Sec. II-D eq. (eqProb) with V built from the
 * scan phases of Sec. II-E): for each of the nscan directions every port gap is
 * driven with V_e = exp(-j k (x_e u + y_e v)), u = sin(theta) cos(phi),
 * v = sin(theta) sin(phi) (the main beam at (theta, phi) under the fill's
 * exp(-jkR) kernel), Z I = V is solved, and the outputs are the gap currents Ip
 * (P x nscan complex, column-major; may be NULL), the active impedance of
 * element `center` (< 0: (nx/2, ny/2)) Za = V_c / Ip_c (eq. (actZ) for the port
 * currents this excitation produces) and its ARC Gamma = (Za - z0)/(Za + z0)
 * (eq. (ARC)), nscan complex each.  One solve per direction, no full Z_p: the
 * form for arrays too large for all-port excitation.  iters (nscan, may be
 * NULL) receives per-direction iteration counts.  Errors: MBT_EINVAL (NULL
 * argument, nscan < 1, non-finite angle, center out of range, block-defined
 * array), MBT_ENOMEM, MBT_ENOCONV, MBT_EBREAKDOWN, MBT_EDEVICE. */
mbt_status mbt_scan_solve(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, const mbt_solve_opts* opts,
                          const double* theta, const double* phi, int32_t nscan, double z0, int32_t center,
                          double* Ip, double* Za, double* Gamma, int32_t* iters, mbt_stats* stats);

/* Scan quantities from a given Z_p (host, P x P, column-major): Za
 * (eqs. (actZ), (actZmat)), Gamma (eq. (ARC)) and Gamma_wave (Sec. II-E, S from
 * eq. (S2Z); may be NULL) as in mbt_solve, for the element `center` (< 0
 * selects (nx/2, ny/2)).  Computed on the GPU in FP64.  The array supplies the
 * lattice positions (dipole arrays only).  Errors: MBT_EINVAL (NULL argument,
 * nscan < 1, center out of range, block-defined array), MBT_EDEVICE. */
mbt_status mbt_active(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, const double* Zp,
                      int32_t center, const double* theta, const double* phi, int32_t nscan, double z0,
                      double* Za, double* Gamma, double* Gamma_wave);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mbt_active on
 * device buffers, with no hipMalloc, hipFree or other device allocation.
 * Zp_dev (P x P complex, column-major), theta_dev and phi_dev (nscan doubles)
 * and the outputs Za_dev, Gamma_dev, Gamma_wave_dev (nscan complex each;
 * Gamma_wave_dev may be NULL) are device pointers owned by the caller; the work
 * is ordered on `stream` (NULL: the context stream) and the call returns when
 * it is done.  The S matrix behind Gamma_wave is formed in a device scratch
 * array of MBT_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until
 * the process ends (set up by mbt_ctx_create): at most 1024 ports when
 * Gamma_wave_dev is given, MBT_EINVAL beyond that.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (two contexts on the same
 * device, or threads) race on it and must be serialised by the caller.  Same
 * results as mbt_active.  Errors as mbt_active. */
#define MBT_NOALLOC_SCRATCH_BYTES (33u * 1024u * 1024u)
mbt_status mbt_active_dev_noalloc(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, const void* Zp_dev,
                                  int32_t center, const double* theta_dev, const double* phi_dev, int32_t nscan,
                                  double z0, void* Za_dev, void* Gamma_dev, void* Gamma_wave_dev, void* stream);

/* ---------------------------------------------------------------- coupling predictors
 * Post-processing of a port impedance matrix (paper Sec. II-E), on the GPU in
 * FP64.  The border of an nx x ny lattice is its outer ring (the elements that
 * growing the array from (nx-2) x (ny-2) adds; an axis of extent 1 has none);
 * "nearest" is the smallest physical distance to the center element c, ties
 * to the smallest element index. */
typedef struct {
    double xi_z;          /* eq. (predZ): |Z_p,cj| / |Z_p,cc|, j the border element nearest c */
    double xi_z_max;      /* max over the border of |Z_p,cj| / |Z_p,cc| (the form before eq. (predZ)) */
    double border_sum;    /* eq. (badpred): sum over the border of |Z_p,cn|, ohm */
    int32_t nearest;      /* j */
    int32_t center;       /* c */
    double s_cc[2];       /* S_cc (complex), S from eq. (S2Z) with reference z0 */
    double s_1[2];        /* S between c and its +x neighbour (complex) */
} mbt_predictors;

/* Predictors of element `center` (< 0: (nx/2, ny/2)) from Z_p (host, P x P
 * complex, column-major, P = nx*ny): the xi_Z family above, and the
 * column couplings C_n (eq. (amitayPred)) of the E-plane active reflection
 * coefficient Gamma_a(psi) = sum_j S_cj exp(j n_j psi) (n_j the column offset
 * of element j from c's column, uniform amplitudes), by the nq-point
 * trapezoid rule over psi = -pi + 2 pi q / nq (exact for nq >= nx; the
 * samples are the scan angles theta = asin(psi / (k dx)) of
 * eq. (amitayPredTheta)).  Cn (nx complex) receives C_n for n = -ix_c ..
 * nx-1-ix_c; Gamma_psi (nq complex, may be NULL) the sampled Gamma_a.
 * Errors: MBT_EINVAL (NULL argument, lattice outside 1..64 per axis, z0 <= 0,
 * nq outside 1..65536, center out of range or without a +x neighbour, no
 * border element besides c, singular Z_p + z0), MBT_EDEVICE. */
mbt_status mbt_predict(mbt_ctx* ctx, const mbt_lattice* lat, const double* Zp, int32_t center, double z0,
                       int32_t nq, mbt_predictors* out, double* Cn, double* Gamma_psi);

/* xi_S (eq. (predS)) for an nx x ny lattice at frequency ratio s: the ideal
 * scattering matrix with s_cc (complex) on the diagonal and
 * s_1 rho^decay exp(-j k (r - dx)) off it (rho the distance between lattice
 * indices, r the physical distance, decay -2 for the infinite-array law),
 * converted by eq. (S2Z), gives |[Z_ideal]_cj| / zp_cc_abs for the border
 * element j nearest c.  Errors: MBT_EINVAL (as mbt_predict, freq_ratio,
 * zp_cc_abs or z0 not positive, non-finite input, singular 1 - S_ideal),
 * MBT_EDEVICE. */
mbt_status mbt_predict_xi_s(mbt_ctx* ctx, const mbt_lattice* lat, double freq_ratio, const double* s_cc,
                            const double* s_1, double zp_cc_abs, double z0, double decay, int32_t center,
                            double* xi_s);

/* ---------------------------------------------------------------- serving
 * A persistent request loop: requests are admitted while in-flight slots and
 * the device-memory budget allow, their solves overlap on the device on
 * separate streams, FFT'd block spectra are cached across requests, and
 * per-request latency (submit -> result) is recorded. */
typedef struct {
    mbt_dipole elem;
    mbt_lattice lat;
    int32_t nfreq;
    const double* freq_ratio;   /* nfreq entries, copied at submit */
    int32_t nscan;
    const double* theta;        /* nscan entries, copied */
    const double* phi;
    double z0;
    mbt_solve_opts opts;
} mbt_request;

typedef struct {
    mbt_status status;
    int32_t nfreq, nports, nscan;
    double* Zp;          /* nfreq blocks of P x P complex (library-owned) */
    double* Za;          /* nfreq x nscan complex, frequency-major */
    double* Gamma;       /* nfreq x nscan complex */
    double* Gamma_wave;  /* nfreq x nscan complex */
    int32_t* iters_max;  /* nfreq */
    double t_submit, t_start, t_done;   /* seconds on the server clock */
} mbt_result;

typedef struct mbt_server mbt_server;

/* max_inflight concurrent requests (>= 1); hbm_budget_bytes 0 = the context's. */
mbt_status mbt_server_create(mbt_ctx* ctx, int32_t max_inflight, size_t hbm_budget_bytes, mbt_server** out);
/* Copies the request, returns at once with a ticket.  MBT_EINVAL for a bad
 * request, MBT_ENOMEM if it can never fit the budget. */
mbt_status mbt_server_submit(mbt_server* srv, const mbt_request* req, uint64_t* ticket);
/* Waits for `ticket` (timeout_ms < 0: forever); the result is library-owned
 * and released by mbt_result_free.  MBT_ETIMEOUT if not done in time. */
mbt_status mbt_server_wait(mbt_server* srv, uint64_t ticket, int32_t timeout_ms, mbt_result** out);
void mbt_result_free(mbt_result* res);
/* Seconds on the server clock (for arrival scheduling by the caller). */
double mbt_server_clock(const mbt_server* srv);
/* Finishes in-flight requests, then stops the loop. */
void mbt_server_destroy(mbt_server* srv);

/* ---------------------------------------------------------------- kernel timing
 * Process-wide HIP-event timing of one kernel class, recorded on the stream
 * each kernel is launched on, with the class's algorithmic bytes and flops per
 * launch (what the method must move: e.g. for an Arnoldi pass the basis
 * vectors read plus the work vector read and written; for the forward lattice
 * FFT the spatial input read plus the spectrum written).  Used to report
 * achieved bandwidth against the HBM roofline.  Not thread-safe with
 * concurrent solves; intended for benchmarks. */
typedef enum {
    MBT_K_NONE = 0,
    MBT_K_ARNOLDI_DOTS = 1,         /* h = V^H w */
    MBT_K_ARNOLDI_UPDATE_DOTS = 2,  /* w -= V h; h2 = V^H w */
    MBT_K_ARNOLDI_UPDATE_NORM = 3,  /* w -= V h2; ||w|| */
    MBT_K_FFT_FWD = 4,              /* zero-padded forward lattice FFT */
    MBT_K_FFT_INV = 5,              /* inverse lattice FFT and crop */
    MBT_K_BIN_PRODUCT = 6,          /* per-bin block products (MFMA) */
    MBT_K_PRECOND_APPLY = 7         /* block-diagonal preconditioner apply (MFMA) */
} mbt_kernel;

/* Starts (and clears) timing of `kernel` (MBT_K_NONE stops timing). */
mbt_status mbt_prof_start(int32_t kernel);
/* Totals since mbt_prof_start: summed event time (ms), launches, algorithmic
 * bytes and flops.  Synchronises the recorded events. */
mbt_status mbt_prof_read(double* ms_total, int64_t* launches, double* bytes, double* flops);

/* ---------------------------------------------------------------- test hooks
 * Expose single steps of the path for parity tests; same ABI conventions. */

/* Unique blocks T[d] (host, (2ny-1)(2nx-1) blocks of M x M complex, block
 * index (dy + ny - 1)*(2nx-1) + (dx + nx - 1), each block row-major T[p*M+q]
 * = Z(test basis p of element e + d, source basis q of element e)). */
mbt_status mbt_dbg_fill_blocks(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, double* T);

/* y = op(Z) x for R columns (x, y host N x R complex, column-major).
 * op: 0 -> Z, 1 -> Z^H, 2 -> Z^H Z.  prec: mbt_prec of the FFT/product path. */
mbt_status mbt_dbg_matvec(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, int32_t prec, int32_t op,
                          const double* x, int32_t R, double* y);

/* y = P^{-1} x with the preconditioner of strategy pc (host N x R, column-major). */
mbt_status mbt_dbg_precond_apply(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, int32_t pc,
                                 const double* x, int32_t R, double* y);

/* The preconditioner blocks before factorisation: pc NORMAL_EQ -> P blocks of
 * M x M (row-major each); ELEMENT_BLOCK -> the single self block. */
mbt_status mbt_dbg_precond_blocks(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, int32_t pc, double* Pb);

/* Batched GMRES on the preconditioned system for arbitrary right-hand sides
 * V (host N x R): returns I (N x R) and per-RHS iteration counts. */
mbt_status mbt_dbg_solve(mbt_ctx* ctx, const mbt_array* arr, double freq_ratio, const mbt_solve_opts* opts,
                         const double* V, int32_t R, double* I, int32_t* iters, mbt_stats* stats);

/* Inverse of an n x n complex matrix (host, column-major) on the device:
 * Gauss-Jordan with partial pivoting in FP64. */
mbt_status mbt_dbg_inverse(mbt_ctx* ctx, const double* A, int32_t n, double* Ainv);

#ifdef __cplusplus
}
#endif

#endif /* MBT_H */

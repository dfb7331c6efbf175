/*
 * rom.h -- C ABI of librom, random-ordinate-method (ROM) source iteration for the steady
 * radiative transport equation on AMD Instinct MI355X (gfx950).
 *
 * Method: L. Li, M. Tang, Y. Yang, "Random ordinate method for mitigating the ray effect in
 * radiative transport equation simulations", arXiv:2407.12527.
 *
 * Problem (eq. (1.1)-(1.2), X-Y geometry of Appendix A): on a uniform nx x ny cell-centred grid
 * over [x0,x1] x [y0,y1] find psi_l(z) for ordinates u_l = (c_l, s_l) (the x-y projection of a
 * unit-sphere direction with polar cosine zeta_l) with
 *     c_l d_x psi_l + s_l d_y psi_l + sigma_t psi_l = sigma_s sum_l' w_l' P(u_l', u_l) psi_l' + q,
 * inflow given on the faces each ordinate enters through.  Space is discretised by first-order
 * upwind cell balance (ROM_SCHEME_STEP) or by the paper's diamond difference (ROM_SCHEME_DD,
 * Sec. 2).  Source iteration (Sec. 3.2, eq. (3.10)) starts from phi = 0 and stops when
 * max|phi^k - phi^{k-1}| <= tol * max|phi^k|, phi = sum_l w_l psi_l.
 *
 * Conventions for every entry point:
 *   - every function returns a status (ROM_OK = 0, ROM_NOT_CONVERGED = 1 is a warning, negative
 *     values are errors) and never throws;
 *   - pointer arguments are HOST pointers unless a comment says "device";
 *   - input arrays are copied during the call; the caller keeps ownership;
 *   - cell arrays are [ny][nx] doubles, x fastest: cell (i, j) at j*nx + i;
 *   - ordinate arrays keep the caller's ordinate order; dirs is [n][3] = (c, s, zeta);
 *   - a handle owns its device memory, taken from the allocator installed with
 *     rom_set_allocator (default hipMalloc / hipFree), and queues all work on its stream
 *     (default: a non-blocking stream of its own; rom_set_stream binds the caller's);
 *   - process-wide state: the allocator hook, and a lock that the device-touching calls take
 *     (below); autotuned sweep shapes are cached in the handle that led the solve;
 *   - a handle is not thread-safe; distinct handles may be used from different threads, and
 *     the calls that touch the device then run one at a time (a process-wide lock: the first
 *     solve of a shape captures a HIP graph, which HIP fails if another thread meanwhile issues
 *     work that synchronizes with it; work the caller issues outside librom from other threads
 *     during such a solve can do the same and make it return ROM_E_DEVICE);
 *   - on error the handle keeps a message readable with rom_last_error().
 */
#ifndef ROM_H
#define ROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------- */
#define ROM_OK 0
#define ROM_NOT_CONVERGED 1 /* warning: outputs hold the last iterate, stats say how far it got */
#define ROM_E_ARG (-1)      /* NULL pointer, bad size, bad enum */
#define ROM_E_DOMAIN (-2)   /* data outside the problem's domain: sigma_t <= 0, sigma_s < 0,
                               sigma_s >= sigma_t (eq. (1.1) requires sigma_s < sigma_t), q < 0,
                               negative inflow, non-finite values, |u| != 1, sum w != 1 */
#define ROM_E_STATE (-3)    /* call out of order (e.g. a solve before rom_set_ordinates) */
#define ROM_E_NOMEM (-4)    /* host or device allocation failed */
#define ROM_E_DEVICE (-5)   /* HIP runtime error, or a sweep dependency wait that timed out */
#define ROM_E_DIVERGED (-6) /* non-finite iterate, or the change grew for 8 iterations in a row */
#define ROM_E_UNSUPPORTED (-7) /* valid request this library does not implement */

/* ---- enums -------------------------------------------------------------------------------- */
#define ROM_SCHEME_STEP 0 /* first-order upwind cell balance */
#define ROM_SCHEME_DD 1   /* diamond difference (Sec. 2) */

#define ROM_SCAT_ISO 0    /* P = 1 */
#define ROM_SCAT_LINEAR 1 /* P = 1 + g cos(xi) (eq. (2.1)) */
#define ROM_SCAT_HG 2     /* Henyey-Greenstein (1-g^2)/(1+g^2-2g cos xi)^{3/2} */
#define ROM_SCAT_DENSE 3  /* caller's P[l'][l] */
/* Flag OR-ed into the kind of rom_set_scattering: rescale each incoming ordinate's row of P so
 * that sum_l w_l P_l'l = 1 for every l' (mass conservation at the discrete level, the
 * normalisation the remark of Sec. 3.1 proposes).  Without it W = w P is used as it is. */
#define ROM_SCAT_NORMALIZE 0x10

#define ROM_ORD_STRATIFIED 0 /* ROM: one uniform draw per (zeta,theta) cell, mirrored (Sec. 3.1) */
#define ROM_ORD_IID_SPHERE 1 /* n i.i.d. uniform directions on the sphere */
#define ROM_ORD_UNIFORM2D 2  /* Appendix A uniform quadrature, 4N^2 ordinates (eq. (A.5)) */
#define ROM_ORD_GAUSS2D 3    /* Appendix A Gaussian quadrature, 2N(N+1) ordinates */

#define ROM_PREC_FP32 0 /* sweeps in FP32; residual and moments in FP64 */
#define ROM_PREC_FP64 1 /* everything in FP64 (plain DOM arm) */

/* Sweep kernels.  STRIP: ordinates on lanes, strips of cells handed from wavefront to wavefront
 * (every scheme, source kind and angular-flux output).  DIAG: grid rows on lanes, each
 * wavefront sweeping the anti-diagonals of a 16- or 64-row block with the y-face value passed one
 * lane up; far more parallel work per ordinate, for isotropic step-scheme source iteration. */
#define ROM_SWEEP_AUTO 0
#define ROM_SWEEP_STRIP 1
#define ROM_SWEEP_DIAG 2

#define ROM_FACE_LEFT 0
#define ROM_FACE_RIGHT 1
#define ROM_FACE_BOTTOM 2
#define ROM_FACE_TOP 3

/* ---- types -------------------------------------------------------------------------------- */
typedef struct rom_handle rom_handle;

/* Uniform grid of Sec. 2: nx x ny cells on [x0,x1] x [y0,y1]. */
typedef struct {
    int32_t nx, ny;
    double x0, x1, y0, y1;
} rom_grid;

/* Isotropic inflow per boundary cell (eq. (1.2)): left/right are [ny], bottom/top are [nx];
 * NULL means vacuum on that face. */
typedef struct {
    const double *left, *right, *bottom, *top;
} rom_inflow;

/* Ordinate recipe for generated sets.  STRATIFIED: p1 x p2 zeta x theta cells per quadrant
 * (n = 4 p1 p2); IID_SPHERE: p1 directions; UNIFORM2D / GAUSS2D: quadrature order N = p1. */
typedef struct {
    int32_t kind;
    int32_t p1, p2;
} rom_ord_spec;

/* Source-iteration options.  Zero-initialised options mean: tol 1e-6, max_iter 1000, FP32,
 * automatic iterations per convergence check and tile shape, step scheme, BF16 contraction. */
typedef struct {
    double tol;               /* stop once max|dphi|/max|phi| <= tol; 0 -> 1e-6; a negative
                                 value never stops early (exactly max_iter iterations) */
    int32_t max_iter;         /* 0 -> 1000 */
    int32_t precision;        /* ROM_PREC_FP32 | ROM_PREC_FP64 */
    int32_t scheme;           /* ROM_SCHEME_STEP | ROM_SCHEME_DD */
    int32_t iters_per_check;  /* iterations captured per graph replay between host checks; 0 -> auto
                                 (the iteration count of the previous solve with the same plan,
                                 split into replays of at most 64, else 8) */
    int32_t tile_x, tile_y;   /* sweep chunk / strip size in cells; 0 -> autotuned */
    int32_t contract_split;   /* reserved for a split-BF16 contraction; must be 0 */
    int32_t band;             /* strip sweep: consecutive strips per workgroup (1..8); row-lane
                                 sweep: wavefronts per workgroup (1..16); 0 -> automatic */
    int32_t sweep;            /* ROM_SWEEP_AUTO (0), ROM_SWEEP_STRIP or ROM_SWEEP_DIAG */
    int32_t diag_rows;        /* row-lane sweep: grid rows per lane block, 16 or 64; 0 -> automatic */
    int32_t diag_k;           /* row-lane sweep: ordinates per lane, 1, 2 or 4 (FP64: 1, 2); 0 -> automatic */
} rom_si_opts;

typedef struct {
    int32_t iters;         /* iterations performed (per system: the largest) */
    int32_t status;        /* ROM_OK or ROM_NOT_CONVERGED */
    double final_r;        /* last relative change (largest over systems) */
    int64_t updates;       /* cell x ordinate upwind updates performed */
    double device_ms;      /* device time of the solve, from events on the handle's stream */
    double sweep_ms;       /* summed duration of the sweep launches that did work, from the end of
                              the kernel before each (its dispatch) to its last wave's end, on the
                              device real-time clock */
    int32_t sweeps;        /* sweep launches that did work */
    int32_t tile_x, tile_y;/* strip sweep: chunk x strip shape; row-lane sweep: ordinates per lane
                              and rows per lane block (set or autotuned) */
    int32_t band;          /* strips (strip sweep) or wavefronts (row-lane sweep) per workgroup */
    int32_t lanes;         /* strip sweep: lanes per ordinate group (16, 32 or 64) */
    int32_t sweep;         /* ROM_SWEEP_STRIP or ROM_SWEEP_DIAG */
} rom_si_stats;

typedef struct {
    int32_t samples;
    int32_t min_iters, max_iters;
    int32_t status;        /* ROM_OK if every sample converged, else ROM_NOT_CONVERGED */
    int64_t updates;
    double device_ms;
    double sweep_ms;       /* summed duration of the sweep launches that did work */
    int32_t sweeps;        /* sweep launches that did work */
    int32_t tile_x, tile_y;/* sweep shape of the last batch of samples (as in rom_si_stats) */
    int32_t band;
    int32_t lanes;
    int32_t sweep;
} rom_ens_stats;

/* ---- lifetime ----------------------------------------------------------------------------- */

/* Create a problem.  sigma_t, sigma_s, q are [cells] host arrays (sigma_t > 0,
 * 0 <= sigma_s < sigma_t, q >= 0, all finite: eq. (1.1)); inflow may be NULL (vacuum).  The grid
 * needs nx, ny >= 1, nx * ny < 2^31 and nx, ny < 2^24 (the sweeps' progress counters tag a column
 * count of 24 bits with the sweep's epoch), else ROM_E_ARG.  The data are validated and copied;
 * device memory is taken on the current HIP device at the first solve.  *out receives the
 * handle. */
int rom_create(const rom_grid* grid, const double* sigma_t, const double* sigma_s, const double* q,
               const rom_inflow* inflow, rom_handle** out);

/* Release the handle and its device memory (NULL is ignored). */
void rom_destroy(rom_handle* h);

/* Queue all later work of h on this HIP stream (a hipStream_t; NULL = null stream). */
int rom_set_stream(rom_handle* h, void* hip_stream);

/* Device allocator for every buffer librom takes afterwards (handle plans, ensemble moments, slab
 * systems): alloc(bytes, ctx) returns device memory on the current HIP device, 256-byte aligned,
 * that no queued device work still uses (or NULL: the call that needed it fails with
 * ROM_E_NOMEM); free_fn(ptr, ctx) takes it back.  librom waits for the device to go idle before
 * it calls free_fn, as hipFree would.  alloc and free_fn both NULL restore hipMalloc / hipFree;
 * exactly one NULL is ROM_E_ARG.  Blocks already taken are returned to the allocator that gave
 * them.  This hook is the way a framework lends librom its memory pool (the Python binding
 * installs PyTorch's caching allocator); it is process-wide, and changing it while another
 * thread is inside librom is safe (the call takes the device lock). */
int rom_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* ptr, void* ctx), void* ctx);

/* Set the ordinate set: dirs [n][3] (c, s, zeta) with c^2 + s^2 + zeta^2 = 1 (to 1e-12) and
 * weights w [n] summing to 1 (to 1e-12), as DOM requires after the Sec. 2 system.  Ordinates are
 * regrouped by quadrant on the device; outputs keep the caller's order.  A dense kernel set
 * before (ROM_SCAT_DENSE) is indexed by the old set: solves return ROM_E_STATE until it is set
 * again. */
int rom_set_ordinates(rom_handle* h, int32_t n, const double* dirs, const double* w);

/* Angular inflow psi_Gamma(z, u_l) on one face (eq. (3.2)): vals is [n][ny] (left/right) or
 * [n][nx] (bottom/top), caller's ordinate order; replaces that face's isotropic inflow; NULL
 * restores it.  Requires ordinates to be set; cleared when they change. */
int rom_set_inflow_angular(rom_handle* h, int32_t face, const double* vals);

/* Scattering kernel P_l'l = P(u_l', u_l), weights W = w_l' P_l'l, self term included (eq. (3.4)),
 * not renormalised unless kind carries ROM_SCAT_NORMALIZE (then P_l'l / r_l' with
 * r_l' = sum_l w_l P_l'l).  LINEAR and HG are folded over +-zeta' (X-Y solutions are even in
 * zeta).  The folded LINEAR kernel is 1 + g (c c' + s s') (eq. (2.1)), of rank 3, so its source
 * is sigma_s (phi~ + g (c Jx~ + s Jy~)) + q from three moments of the previous iterate
 * (phi~, Jx~, Jy~ = sums of w psi / r, w c psi / r, w s psi / r), formed inside the sweep: O(n)
 * work per cell, no angular flux stored.  HG and DENSE use the dense contraction.  DENSE takes
 * P [n][n] (caller's order) and requires ordinates to be set. */
int rom_set_scattering(rom_handle* h, int32_t kind, double g, const double* P);

/* ---- compute ------------------------------------------------------------------------------ */

/* One transport sweep psi_l = L_l^{-1} src (the inversion of Sec. 3.2), every ordinate.  src is
 * [cells] (shared by all ordinates) if src_per_ordinate = 0, else [n][cells] (caller's order).
 * phi [cells] receives sum_l w_l psi_l; psi (optional, may be NULL) [n][cells].  precision
 * and scheme as in rom_si_opts (opts may be NULL). */
int rom_sweep(rom_handle* h, const double* src, int32_t src_per_ordinate, double* phi, double* psi,
              const rom_si_opts* opts);

/* For callers that cannot allocate device memory (work under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the sweep of rom_sweep for an isotropic source, on
 * device arrays, taking no device memory.  src_dev and phi_dev are DEVICE pointers to [cells]
 * floats (precision ROM_PREC_FP32) or doubles (ROM_PREC_FP64), src shared by all ordinates; phi
 * receives sum_l w_l psi_l with the handle's ordinates and inflow (step scheme; rom_sweep's tile
 * and band, hence its result bit for bit).  Every buffer the sweep needs lives in a 64 MiB region
 * preallocated per GPU when the library is loaded and held until the process ends; a problem whose
 * tables, partial fluxes and strip edges do not fit is refused with ROM_E_UNSUPPORTED.  The work
 * is queued on hip_stream (NULL: the null stream) and the call returns without waiting for it.
 * The first call for a handle state (ordinates, inflow) and precision fills the region from the
 * host and waits for that upload; later calls for the same handle only launch kernels.  All
 * calls on one GPU share its region: calls that overlap on one GPU (other streams, other
 * threads while work is still queued) race.  A dependency wait that timed out is not reported
 * (the call does not wait for the device). */
int rom_sweep_noalloc(rom_handle* h, const void* src_dev, void* phi_dev, int32_t precision, void* hip_stream);

/* Source iteration to convergence for the handle's ordinates and scattering kernel.  phi [cells]
 * receives the final scalar flux, or may be NULL to leave it on the device (see rom_phi_device).
 * Returns ROM_NOT_CONVERGED if max_iter was reached. */
int rom_source_iterate(rom_handle* h, const rom_si_opts* opts, double* phi, rom_si_stats* stats);

/* ROM ensemble (Sec. 4.1, eq. (4.6)): t independent ordinate samples s = 0..t-1 generated from
 * (spec, seed) exactly as rom_generate_ordinates does, each solved to convergence with the
 * handle's scattering kernel, batched on the GPU; mean [cells] and unbiased variance var [cells]
 * (divided by t-1; zero when t = 1) accumulated in FP64.  mean/var may be NULL (device only). */
int rom_ensemble(rom_handle* h, int32_t t, uint64_t seed, const rom_ord_spec* spec,
                 const rom_si_opts* opts, double* mean, double* var, rom_ens_stats* stats);

/* The samples first .. first + t - 1 of the same ensemble (Sec. 4.1): generated and solved as
 * rom_ensemble does, but each sample's scalar flux is returned, phis [t][cells] (sample-major,
 * host FP64), instead of the moments.  For statistics that the mean and variance do not give, such
 * as the expected per-sample error E||phi^xi - phi_ref|| or the Monte Carlo error of a running
 * average (both defined in Sec. 4.1); first >= 0 lets a large ensemble be taken in pieces.
 * Errors as rom_ensemble; the handle keeps no device result (rom_phi_device fails after it). */
int rom_ensemble_samples(rom_handle* h, int32_t t, uint64_t seed, int64_t first, const rom_ord_spec* spec,
                         const rom_si_opts* opts, double* phis, rom_ens_stats* stats);

/* k independent problems solved together in one persistent sweep launch per iteration; each
 * handle must have ordinates set; phis[i] [cells_i] receives handle i's scalar flux (phis, or any
 * entry, may be NULL: that flux stays on the device only); stats (optional) is [k].  All handles
 * must use the same stream and device. */
int rom_solve_batch(rom_handle* const* hs, int32_t k, const rom_si_opts* opts, double* const* phis,
                    rom_si_stats* stats);

/* Device-resident result of the last solve on h: *dev receives a device pointer to [cells]
 * values of type float (*is_fp64 = 0) or double (*is_fp64 = 1), valid until the next call on h.
 * For rom_ensemble this is the FP64 mean. */
int rom_phi_device(const rom_handle* h, const void** dev, int32_t* is_fp64);

/* ---- slab geometry (Sec. 4.1) ----------------------------------------------------------------
 * mu dpsi/dx + sigma_t psi = sigma_s phi + q on [x0, x1], phi = (1/2) int_{-1}^{1} psi dmu,
 * isotropic scattering, inflow psi(x0, mu > 0) and psi(x1, mu < 0) (Example 4.1).  Unknowns at
 * the nx + 1 grid points x_i = x0 + i (x1 - x0) / nx (the paper's slab error norm is over them);
 * each cell [x_i, x_{i+1}] is closed by diamond difference with the cell's sigma_t and source the
 * means of its end values:
 *   |mu| (psi_out - psi_in) / dx + sigma_c (psi_in + psi_out) / 2 = (S_i + S_{i+1}) / 2,
 * S_i = sigma_s(x_i) phi_i + q(x_i) (a second-order scheme; the paper's own [ShiA] scheme is not
 * given in its text).  Weights sum to 1: phi_i = sum_l w_l psi_l(x_i). */
typedef struct rom_slab rom_slab;

#define ROM_SLAB_RANDOM 0  /* ROM: one draw per cell of [-1, 0] (n even), mirrored; w = 1/n */
#define ROM_SLAB_GAUSS 1   /* Gauss-Legendre on [-1, 1], weights halved */
#define ROM_SLAB_UNIFORM 2 /* midpoints of n equal cells, w = 1/n */

/* A slab problem: sigma_t, sigma_s, q [nx + 1] at the grid points (host FP64, copied), with
 * sigma_t > 0, 0 <= sigma_s < sigma_t, q >= 0, all finite; nx >= 1, x1 > x0. */
int rom_slab_create(int32_t nx, double x0, double x1, const double* sigma_t, const double* sigma_s,
                    const double* q, rom_slab** out);
void rom_slab_destroy(rom_slab* s);
/* Queue the slab's device work on this HIP stream (NULL: the slab's own stream). */
int rom_slab_set_stream(rom_slab* s, void* hip_stream);

/* t independent slab systems, system k with the n ordinates mu [k][n] (0 < |mu| <= 1), weights
 * w [k][n] (> 0, summing to 1 within 1e-12) and entry-face inflow [k][n] (finite, >= 0), each
 * solved by source iteration from phi = 0 to opts->tol (relative max-norm change, as
 * rom_source_iterate) on the GPU, one wavefront per 64 / L systems (L lanes per system, each
 * lane carrying up to 64 ordinates; n <= 4096).  phis [t][nx + 1] receives every system's
 * scalar flux (host FP64); iters [t] (optional) the iterations each took.  opts->precision
 * selects FP32 or FP64 arithmetic; tile, band and sweep options are ignored.  Returns
 * ROM_NOT_CONVERGED if a system reached max_iter, ROM_E_DIVERGED if one became non-finite. */
int rom_slab_solve(rom_slab* s, int32_t t, int32_t n, const double* mu, const double* w, const double* inflow,
                   const rom_si_opts* opts, double* phis, int32_t* iters, rom_ens_stats* stats);

/* Slab ordinate set (host only): kind ROM_SLAB_RANDOM (sample `sample` of `seed`, same
 * SplitMix64 streams as rom_generate_ordinates), ROM_SLAB_GAUSS or ROM_SLAB_UNIFORM; mu [n], w [n]. */
int rom_slab_ordinates(int32_t kind, int32_t n, uint64_t seed, int64_t sample, double* mu, double* w);

const char* rom_slab_last_error(const rom_slab* s);

/* ---- host utilities (no device work) ------------------------------------------------------ */

/* Ordinate set of sample `sample` for the recipe (Sec. 3.1 steps 1-2, Sec. 4.2; Appendix A for
 * the deterministic quadratures).  Random numbers: SplitMix64; sample s uses the stream seeded
 * with the (s+1)-th output of a SplitMix64 generator seeded with `seed`.  dirs [n][3], w [n] with
 * n = rom_ordinate_count(spec). */
int rom_generate_ordinates(const rom_ord_spec* spec, uint64_t seed, int64_t sample, double* dirs, double* w);
int32_t rom_ordinate_count(const rom_ord_spec* spec);

const char* rom_status_string(int status);
const char* rom_last_error(const rom_handle* h);
const char* rom_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ROM_H */

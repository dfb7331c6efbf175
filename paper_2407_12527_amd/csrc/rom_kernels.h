// rom_kernels.h -- kernel arguments and launchers of librom (host and device side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rom_device.h"

namespace rom {

struct SweepArgs {
    const ProblemDev* probs;
    const WaveStreamDev* ws;
    const LaneDev* lanes;      // [nws][64]
    const SystemDev* sys;
    const int2* tickets;       // (wave-stream, band), band-major
    int32_t ntickets;
    int32_t spin_limit;        // polls before a dependency wait gives up
    int32_t mode_all;          // 1: sweep every wave-stream regardless of convergence state
    int32_t band;              // wavefronts per workgroup = consecutive strips per ticket (1..8)
    const void* sigma_t;       // field pool (T)
    const void* src;           // isotropic source pool (T)
    const void* ang_src;       // per-ordinate source pool [cells][npad] (T)
    void* psi_out;             // angular-flux output pool [cells][npad] (T or BF16)
    void* part;                // partial scalar-flux pool (T)
    const int64_t* slot_off;   // partial slot -> offset in part
    const int32_t* uflags;     // per (problem, quadrant, strip, chunk): bit r set when sigma_t is
                               // constant along row r of the chunk
    void* edge;                // strip-edge pool (T)
    const void* inflow;        // boundary inflow pool (T)
    long long* prog;           // strip progress counters
    Ctl* ctl;
    SysCtl* sysctl;
    int32_t mom_r;             // linear kernel: 1 = also form the 1/r-weighted density (plane 3)
    int32_t pad;
    int64_t wait_ticks;        // real-time clock ticks before a dependency wait gives up
};

struct DiagArgs {
    const DiagTaskDev* tasks;
    const LaneDev* ords;       // [tasks][NO] (a, b, w of each ordinate; padding has w = 0)
    const ProblemDev* probs;
    const SystemDev* sys;
    const int2* tickets;       // (task, band), band-major
    int32_t ntickets;
    int32_t spin_limit;
    int32_t mode_all;
    int32_t pad;
    void* edge;                // band top-row pool (T)
    long long* prog;           // band progress counters
    const void* sigma_t;       // field pool (T)
    const void* src;           // isotropic source pool (T)
    void* part;                // partial scalar-flux pool (T)
    const int64_t* slot_off;
    const void* inflow;        // unweighted boundary inflow pool (T)
    Ctl* ctl;
    SysCtl* sysctl;
    const void* ang_src;       // dense kernels: per-ordinate source pool, ordinate blocks of 16
    void* psi_out;             // dense kernels: weighted angular flux pool (BF16), same layout
    int64_t wait_ticks;        // real-time clock ticks before a dependency wait gives up
};

struct CombineArgs {
    const SystemDev* sys;
    const ProblemDev* probs;
    const int32_t* slot_order;
    const int64_t* slot_off;
    const int64_t* slot_off_ord;  // slot_off[slot_order[i]]: offsets in summation order
    const int2* blocks;        // (system, first cell) per block
    int32_t cells_per_block;
    int32_t many_cpt;          // 0: one wave sums all slots of 4 cells per thread; 1, 2, 4, 8: the
                               // many-slot combine, tiles of 64 * many_cpt cells (= cells_per_block)
    int32_t nsys;
    int32_t nmom;              // partial planes per slot: 1 (phi) or 4 (linear kernel: phi, Jx~,
                               // Jy~, phi~); sources: 1 or 3 planes
    int32_t mode;              // 0: source-iteration step, 1: plain sum (single sweep: phi only;
                               // src, sigma_s and q are not touched and may be NULL)
    int32_t max_iter;
    int32_t mom_r;             // linear kernel: phi~ comes from plane 3 (else phi~ = phi)
    int32_t vec;               // 16-byte loads (every system's cell count a multiple of 16 B /
                               // sizeof(T)): 1 many slots, tiles of 64 * 16 B of cells split over
                               // the block's 4 waves by slot (3: 8 waves, above 64 slots); 2 at
                               // most 8 slots, 4 tiles of 256 * 16 B
    double tol;
    const void* part;
    void* phi;
    void* src;
    const void* sigma_s;
    const void* q;
    SysCtl* sysctl;
    Ctl* ctl;
    double* rhist;             // optional [nsys][max_iter] relative-change history
};

struct MomentsArgs {
    const void* phi;           // pool holding the per-sample fluxes
    const int64_t* phi_offs;   // [t] offsets of the samples of this batch
    int32_t t;                 // samples in this batch
    int32_t pad;
    int64_t count;             // samples already accumulated (0: first batch)
    int64_t cells;
    double* mean;
    double* m2;
};

struct ContractArgs {
    const void* a;             // Psi' [M][K] (BF16, FP32 or FP64)
    const void* bt;            // P^T [N][K]
    const void* sigma_s;       // [M]
    const void* q;             // [M]
    void* out;                 // S [M][N]
    int32_t M, N, K;
    int32_t sys_index;
    const SysCtl* sysctl;      // skip when that system has stopped (NULL: always run)
    int32_t blocked;           // BF16 kernel: 1 = A and out in ordinate blocks of 16,
                               // [K / 16][M][16] and [N / 16][M][16] (the row-lane sweep's
                               // layout); 0 = row-major [M][K] and [M][N]
    int32_t pad;
};

// One system's transposed scattering matrix Bt[n][k] = P(u_k, u_n) / r_k: the discrete kernel of
// Sec. 2 taken at the ordinates themselves (the choice of Sec. 3.1), incoming u_k and outgoing u_n,
// each row divided by its weighted sum r_k when the kernel is normalized (else r_k = 1), indexed by
// the plan's internal ordinate order, zero on padding.
struct KmSys {
    int64_t ord_off;     // first entry of the system in the ordinate tables
    int64_t pt_off;      // first element of its matrix ([al][al])
    int64_t dense_off;   // first element of the caller's dense kernel ([n][n], caller's order)
    int32_t npad;        // internal ordinates (padding included)
    int32_t al;          // matrix side (>= npad; rows and columns past npad are zero)
    int32_t n;           // caller's ordinate count
    int32_t kind;        // 2 Henyey-Greenstein (projected to x-y, folded over z), 3 dense
    int32_t norm;        // 1: divide by the weighted row sums
    int32_t pad;
    double g;
};

struct KmArgs {
    const KmSys* sys;    // [nsys]
    const double* ord;   // [entries][4]: direction (c, s, z) and weight of each internal ordinate
    const int32_t* uidx; // [entries]: the caller's index of each internal ordinate, -1 on padding
    const double* dense; // caller's dense kernels (kind 3), else unused
    double* inv_r;       // [entries]: 1 / r_k (written when norm)
    void* bt;            // matrices: BF16 bits (fp64 = 0) or doubles
    int32_t nsys, fp64;
    int32_t max_al, pad;
};

// Slab systems (Sec. 4.1): all share one problem (fields at the nn grid points), each has its own
// n ordinates; a wavefront holds 64 / L systems of L lanes, a lane carries ordinates r, r + L, ...
struct SlabArgs {
    const void* mu;            // [nsys][n] (T)
    const void* w;             // [nsys][n] (T)
    const void* inflow;        // [nsys][n] (T), entry-face value of each ordinate
    const void* st;            // [nn] sigma_t at the grid points (T)
    const void* ss;            // [nn]
    const void* q;             // [nn]
    void* phi;                 // [nsys][nn] (T), last iterate
    int32_t* iters;            // [nsys]
    int32_t* state;            // [nsys]: 1 converged, 2 stopped at max_iter, 3 diverged
    double* rfinal;            // [nsys] last relative change
    int32_t nsys, n, nn, L;    // systems, ordinates per system, grid points, lanes per system
    int32_t max_iter, pad;
    double tol;
    double inv_dx;
};
// kmax: ordinates per lane the variant holds (1, 4, 16 or 64; >= ceil(n / L))
size_t slab_lds_bytes(bool fp64, int nn, int L);
hipError_t launch_slab(const SlabArgs& a, bool fp64, int kmax, hipStream_t s);

// L = lanes per ordinate group (16, 32 or 64; 64 for anisotropic sources and psi output);
// mom = 1 (isotropic source) or 4 (linear kernel: three source planes, four moment planes)
hipError_t launch_sweep(const SweepArgs& a, int grid, bool fp64, int tx, int ty, bool dd, bool ang, int psi, int L,
                        int mom, hipStream_t s);
bool sweep_tile_supported(int tx, int ty);
bool sweep_tile_supported_fp64(int tx, int ty);
size_t sweep_lds_bytes(bool fp64, int tx, int ty, bool ang, int L, int nw, int mom);
// Row-lane sweep: R rows per lane block (16 or 64), K ordinates per lane (1, 2, 4; FP64: 1, 2),
// nb wavefronts (row blocks) per workgroup (1..16; 1..8 when K * sizeof(T) >= 16), persistent
// workgroups taking (task, band) tickets.
// ang: per-ordinate sources in, BF16 weighted angular flux out (dense kernels; FP32 only).
bool diag_supported(bool fp64, int R, int K);
int diag_max_nb(bool fp64, int K, bool ang = false);
size_t diag_lds_bytes(bool fp64, int R, int K, int nb);
hipError_t launch_diag(const DiagArgs& a, int grid, int nb, bool fp64, int R, int K, bool ang, hipStream_t s);
hipError_t launch_combine(const CombineArgs& a, int nblocks, bool fp64, hipStream_t s);
hipError_t launch_sweep_prologue(Ctl* ctl, hipStream_t s);
hipError_t launch_mark(Ctl* ctl, hipStream_t s);
hipError_t launch_reset_systems(SysCtl* sc, int nsys, Ctl* ctl, hipStream_t s);
hipError_t launch_fill(void* p, int64_t n, bool fp64, double v, hipStream_t s);
// S = q for every system of a plan (the first source of source iteration)
hipError_t launch_init_source(const SystemDev* sys, const ProblemDev* probs, int nsys, int64_t max_cells, bool fp64,
                              const void* q, void* src, hipStream_t s);
// phi = 0 over [0, phi_total), S = q and a reset of the per-system and control state, one launch
hipError_t launch_init_state(const SystemDev* sys, const ProblemDev* probs, int nsys, int64_t max_cells, bool fp64,
                             const void* q, void* src, void* phi, int64_t phi_total, SysCtl* sc, Ctl* ctl,
                             hipStream_t s);
hipError_t launch_moments(const MomentsArgs& a, bool fp64, hipStream_t s);
hipError_t launch_finish_var(const double* m2, double* var, int64_t cells, int64_t t, hipStream_t s);
// kind 0 bf16 MFMA, 1 fp32, 2 fp64; ctl (may be NULL): the kernel clears ctl->t_mark (the next
// sweep is then timed from its first ticket claim)
hipError_t launch_contract(const ContractArgs& a, int kind, hipStream_t s, Ctl* ctl = nullptr);
// Blocks of one contraction (-1: shape not supported by the kind); several contractions in one
// launch: items [n] on the device, map [nblocks] = (item, block of that item).
int contract_blocks(const ContractArgs& a, int kind);
hipError_t launch_contract_batch(const ContractArgs* items, const int2* map, int nblocks, int kind, hipStream_t s,
                                 Ctl* ctl = nullptr);
hipError_t launch_cast_bf16(const float* in, void* out, int64_t n, hipStream_t s);
// Kernel matrices of every system of a plan (row sums first when a system is normalized).
hipError_t launch_kernel_matrix(const KmArgs& a, hipStream_t s);

}  // namespace rom

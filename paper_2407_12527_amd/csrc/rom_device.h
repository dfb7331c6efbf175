// rom_device.h -- data layout shared by the host runtime and the gfx950 kernels of librom.
//
// Vocabulary
//   problem      grid + cross sections + source (+ inflow) of eq. (1.1)-(1.2);
//   system       one problem with one ordinate set (one ROM sample); it owns a scalar flux, a
//                source, a convergence state;
//   group        L consecutive lanes of a wavefront holding up to L ordinates of one quadrant of
//                one system (L = 16, 32 or 64; a wavefront holds G = 64/L groups, all from one
//                problem and one quadrant, so they march the same cell order);
//   wave-stream  the 64 lanes of such a wavefront together with its quadrant: it sweeps the
//                whole grid, strip by strip (TY rows each), chunk by chunk (TX columns each);
//   strip task   (wave-stream, strip): the unit a persistent wavefront claims from the ticket
//                list.  Tickets are ordered by strip index first, so the producer of every strip
//                edge holds an earlier ticket than its consumer.
//
// Angular fluxes are carried scaled by their quadrature weight (psi' = w psi), so a group's
// scalar-flux contribution is the plain lane sum and the anisotropic contraction multiplies by
// P instead of W = w P (eq. (3.4)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rom {

constexpr int kWave = 64;
constexpr int kMaxGroups = 4;
constexpr int kMaxBand = 8;    // wavefronts (consecutive strips) per sweep workgroup
// LDS ring slots per strip boundary inside a band.  One suffices: the wave above reads chunk c's
// edge as soon as it is published, a whole chunk before the wave below has its next edge ready
// (c3 sweep 822 -> 800 us against two slots, c5 2653 -> 2633 us; the smaller LDS lets c3's
// 8-wave bands keep two workgroups per CU).
constexpr int kRingSlots = 1;

struct ProblemDev {
    int32_t nx, ny;
    int32_t nchunks;      // ceil(nx / TX)
    int32_t nstrips;      // ceil(ny / TY)
    int64_t field_off;    // offset of sigma_t / sigma_s / q in the field pools (elements)
    int64_t uflag_off;    // offset of the row-uniformity masks [4 quadrants][nstrips][nchunks]
};

struct WaveStreamDev {
    int32_t prob;               // problem index
    int32_t quad;               // 0: c>=0,s>=0  1: c<0,s>=0  2: c<0,s<0  3: c>=0,s<0
    int32_t L;                  // lanes per group (16, 32, 64)
    int32_t prog_off;           // first progress counter (one per band of strips)
    int64_t edge_off;           // band-top edge buffer [nbands][nx][64] (elements of T)
    int64_t xin_off;            // inflow on the entry x-face [ny][64] in sweep order, -1 = vacuum
    int64_t yin_off;            // inflow on the entry y-face [nx][64] in sweep order, -1 = vacuum
    int32_t sys[kMaxGroups];    // system of each group (-1: empty group)
    int32_t slot[kMaxGroups];   // partial-flux slot of each group (-1: empty group)
};

struct LaneDev {                // per (wave-stream, lane); padded lanes are all zero
    double a, b, w;             // |c|/dx, |s|/dy, quadrature weight
    double c, s;                // signed direction cosines (linear-kernel source c S1 + s S2)
    double m1, m2, m3;          // linear-kernel moment weights c / r, s / r, 1 / r (r: the row sum
                                // of the normalized kernel, 1 without normalization)
    int32_t ord;                // internal (padded, quadrant-grouped) ordinate index in its system
    int32_t pad;
};

struct SystemDev {
    int32_t prob;
    int32_t npad;               // internal padded ordinate count (anisotropic layout [cells][npad])
    int32_t nslots;             // partial slots summed by the combine step, in this order
    int32_t slot_first;         // index into the slot-order list
    int64_t phi_off;            // scalar flux [cells] (elements of T)
    int64_t src_off;            // isotropic source [cells] (elements of T); with the linear
                                // kernel three planes [3][cells]: S0, S1, S2 of S0 + c S1 + s S2
    int64_t ang_off;            // anisotropic source / angular flux [cells][npad] (elements)
    double g;                   // linear-kernel anisotropy (S1, S2 = sigma_s g Jx~, sigma_s g Jy~)
};

// Task of the row-lane ("diagonal") sweep: the whole grid of one problem for NO = (64 / R) * K
// ordinates of one quadrant of one system, swept band by band (NB row blocks of R rows per band,
// one workgroup per band).  Lane g*R + r holds row r of an R-row block for ordinates
// g*K .. g*K + K - 1 (the task's entries ord_off + g*K + k of the lane table).
constexpr int kDiagMaxWaves = 16;
constexpr int kPoolPad = 128;   // elements of padding before and after the sigma_t and source pools

// Row pitch (elements) of the row-lane sweep's y-face tables and band edges: a multiple of 16
// with at least 16 elements of padding, so U-column runs (U <= 16) past the row end stay inside.
__host__ __device__ inline int diag_pitch(int nx) { return ((nx + 15) & ~15) + 16; }

struct DiagTaskDev {
    int32_t sys, prob, quad;
    int32_t slot;               // partial-flux slot
    int64_t ord_off;            // first of the task's NO lane-table entries
    int64_t xin_off;            // inflow on the entry x-face [ny][NO], rows in sweep order; -1 vacuum
    int64_t yin_off;            // inflow on the entry y-face [NO][pitch], columns in sweep order; -1 vacuum
    int64_t edge_off;           // top rows of its bands [nbands][NO][pitch] (elements of T)
    int32_t prog_off;           // first of its per-band progress counters
    int32_t pad;
};

// Per-system convergence state, written only by the combine step.
struct SysCtl {
    unsigned long long dmax_bits;   // max |phi^k - phi^{k-1}| of the running iteration (FP64 bits)
    unsigned long long pmax_bits;   // max |phi^k|
    int32_t iter;                   // completed iterations
    int32_t state;                  // 0 running, 1 converged, 2 stopped at max_iter, 3 diverged
    int32_t grow;                   // consecutive iterations with a growing change
    int32_t pad;
    double r;                       // last relative change
    double r_prev;
};

// The three words that many workgroups touch at once sit on cache lines of their own: the ticket
// counter (claimed by every sweep workgroup), the combine's block counter, and the error flag that
// long dependency waits poll (c5 step 55.7 -> 55.0 ms against all of them on one line).
struct Ctl {
    int32_t ticket;         // next strip ticket
    int32_t pad_ticket[31];
    int32_t blocks_done;    // combine blocks finished in this iteration
    int32_t pad_blocks[31];
    int32_t error;          // 1: a dependency wait timed out
    int32_t pad_error[31];
    int32_t epoch;          // sweep generation, tags the progress counters
    int32_t active;         // systems still running after the last combine step
    int32_t sweeps;         // sweep launches that did work (timed)
    int32_t pad;
    unsigned long long t_first;     // real-time clock at the running sweep's first ticket claim
    unsigned long long t_last;      // ... and at its last claim, after all its work
    unsigned long long sweep_ticks; // summed sweep durations (real-time clock ticks)
    unsigned long long t_mark;      // end of the combine step that precedes the next sweep: a sweep
                                    // lasts from here (its dispatch, as a profiler sees it) to its
                                    // last claim; a contraction in between clears it (~0), and that
                                    // sweep is timed from its first claim
};

}  // namespace rom

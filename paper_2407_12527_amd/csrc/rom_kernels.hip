// rom_kernels.hip -- gfx950 (MI355X) kernels of librom.
//
//   sweep_kernel     transport sweep psi = L^{-1} S for every ordinate (the operator inversion of
//                    Sec. 3.2): ordinates on wavefront lanes, persistent strip tasks, strip edges
//                    handed upward through global memory behind epoch-tagged progress counters;
//   combine_kernel   phi = sum of the per-group partial fluxes in a fixed order, the next
//                    isotropic source sigma_s phi + q, the FP64 relative change and the
//                    per-system convergence decision of source iteration (eq. (3.10));
//   contract_*       anisotropic scattering source S = sigma_s (Psi' P) + q (eq. (3.1) right-hand
//                    side with W = w P of eq. (3.4)): BF16 MFMA with FP32 accumulation, or a plain
//                    tiled FP64/FP32 kernel for the FP64 path;
//   moments_kernel   FP64 ensemble mean and unbiased variance over samples (eq. (4.6)).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "rom_device.h"
#include "rom_kernels.h"

namespace rom {

// ------------------------------------------------------------------------------------ helpers
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Strip-edge hand-off between wavefronts that may sit on different XCDs.  The edge words
// themselves are written and read with device-scope (agent) relaxed atomic accesses, which the
// hardware keeps coherent across the per-XCD L2 caches word by word; the producer then waits for
// its stores to complete (s_waitcnt vmcnt(0)) before it publishes the progress counter.  This
// avoids the whole-L2 write-back / invalidate that a release / acquire fence pair costs.
template <typename T>
__device__ __forceinline__ void edge_store(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ T edge_load(const T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ __forceinline__ void stores_complete() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait until *p >= target (the strip below has finished chunk c of this epoch).  Bounded: after
// `limit` polls (or once another wave has timed out) the wait gives up and records the error, so
// every wave always exits.
__device__ __forceinline__ void wait_progress(long long* p, long long target, Ctl* ctl, int limit)
{
    int spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins >= limit) {
            __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if ((spins & 1023) == 0 &&
            __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            break;
    }
    asm volatile("" ::: "memory");  // edge loads stay after the poll
}

template <typename T>
__device__ __forceinline__ T to_T(double x) { return (T)x; }

#ifndef ROM_ROW_UNROLL
#define ROM_ROW_UNROLL 0
#endif


// ------------------------------------------------------------------------------------ sweep
//
// One wavefront = one wave-stream strip task at a time.  Lane state while walking a strip:
//   xl[r]  x-face value entering row r of the strip (carried from chunk to chunk),
//   yd[i]  y-face value entering column i of the chunk (from the strip below, updated row by row
//          and handed to the strip above after the chunk's last row).
// Cell update (ordinate-scaled fluxes psi' = w psi, cells visited in sweep order):
//   STEP: psi' = (w S + a x + b y) / (sigma_t + a + b),                x <- psi', y <- psi'
//   DD:   psi' = (w S + 2a x + 2b y) / (sigma_t + 2a + 2b),  x <- 2psi' - x, y <- 2psi' - y
// When sigma_t is constant along a row of a chunk (a flag the host precomputes), the reciprocal
// of the denominator is taken once per row.
//
// Memory: the chunk's sigma_t and (isotropic) sources are loaded into registers one chunk ahead
// and staged in LDS in sweep order, so the row loop reads LDS broadcasts only.  A ragged chunk or
// strip is padded with a valid cell and a zero source; padded results are never stored.
//
// Scalar flux: the TX values of a row are summed over each group's lanes by a transposing
// butterfly (gfx950 permlane swaps for lane distances 32 and 16, DPP for 8, 4, 2, 1): every
// stage halves the number of registers, so a row of TX cells costs about 2 VALU operations per
// cell, and the row's sums end up one cell per lane for a single coalesced store.

// Lanes with bit `d` take y, the others x.
__device__ __forceinline__ float pick(int lane, int d, float x, float y) { return (lane & d) ? y : x; }

template <int D>
__device__ __forceinline__ float halve(int lane, float x, float y)
{
    if constexpr (D == 32) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else if constexpr (D == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        // partner lane differs in bit D: row_ror:8 (xor 8), row_half_mirror (7 - l within 8 lanes),
        // quad_perm xor 2, quad_perm xor 1
        constexpr int CTRL = D == 8 ? 0x128 : D == 4 ? 0x141 : D == 2 ? 0x4E : 0xB1;
        const float u = pick(lane, D, x, y);
        const float t = pick(lane, D, y, x);
        return u + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(t), CTRL, 0xF, 0xF, true));
    }
}

template <int D>
__device__ __forceinline__ float fold(float v)
{
    constexpr int CTRL = D == 8 ? 0x128 : D == 4 ? 0x141 : D == 2 ? 0x4E : 0xB1;
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Reduce-scatter N row values over groups of L lanes; returns this lane's sum and its cell index.
template <int N, int L>
__device__ __forceinline__ float butterfly(int lane, float (&v)[N], int& cell)
{
    constexpr int LOGL = L == 64 ? 6 : L == 32 ? 5 : 4;
    constexpr int H = N == 16 ? 4 : N == 8 ? 3 : N == 4 ? 2 : 1;
    static_assert(H <= LOGL, "row longer than the lane group");
    float r[N];
#pragma unroll
    for (int k = 0; k < N; ++k) r[k] = v[k];
    int c = 0;
#pragma unroll
    for (int s = 0; s < H; ++s) {
        const int half = N >> (s + 1);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
            if (k < half) {
                const int d = (L == 64 ? 32 : L == 32 ? 16 : 8) >> s;
                if (d == 32) r[k] = halve<32>(lane, r[k], r[k + half]);
                else if (d == 16) r[k] = halve<16>(lane, r[k], r[k + half]);
                else if (d == 8) r[k] = halve<8>(lane, r[k], r[k + half]);
                else if (d == 4) r[k] = halve<4>(lane, r[k], r[k + half]);
                else if (d == 2) r[k] = halve<2>(lane, r[k], r[k + half]);
                else r[k] = halve<1>(lane, r[k], r[k + half]);
            }
        }
        const int d = (L == 64 ? 32 : L == 32 ? 16 : 8) >> s;
        c |= ((lane & d) ? 1 : 0) << (H - 1 - s);
    }
    float out = r[0];
#pragma unroll
    for (int s = H; s < LOGL; ++s) {
        const int d = (L == 64 ? 32 : L == 32 ? 16 : 8) >> s;
        if (d == 8) out = fold<8>(out);
        else if (d == 4) out = fold<4>(out);
        else if (d == 2) out = fold<2>(out);
        else if (d == 1) out = fold<1>(out);
    }
    cell = c;
    return out;
}

// Lanes whose in-place (folded) bits are zero represent their cell.
template <int N, int L>
__device__ __forceinline__ bool butterfly_rep(int lane)
{
    constexpr int LOGL = L == 64 ? 6 : L == 32 ? 5 : 4;
    constexpr int H = N == 16 ? 4 : N == 8 ? 3 : N == 4 ? 2 : 1;
    constexpr int FOLD_MASK = (1 << (LOGL - H)) - 1;  // folded distances are the lowest lane bits
    return (lane & FOLD_MASK) == 0;
}

struct RowCtx {
    int lane, g, L;
    int64_t rowbase;
    int i0, nx;
    bool xpos;
    int cols;
};

// Row scalar-flux partials: float rows use the butterfly, double rows a plain xor shuffle.
template <int TX>
__device__ __forceinline__ void store_partials(const RowCtx& R, float (&acc)[TX], float* p)
{
    int c = 0;
    float v = 0.f;
    bool rep = false;
    if (R.L == 64) {
        v = butterfly<TX, 64>(R.lane, acc, c);
        rep = butterfly_rep<TX, 64>(R.lane);
    } else if (R.L == 32) {
        v = butterfly<TX, 32>(R.lane, acc, c);
        rep = butterfly_rep<TX, 32>(R.lane);
    } else {
        v = butterfly<TX, 16>(R.lane, acc, c);
        rep = butterfly_rep<TX, 16>(R.lane);
    }
    if (rep && p && c < R.cols) {
        const int ii = R.i0 + c;
        p[R.rowbase + (R.xpos ? ii : R.nx - 1 - ii)] = v;
    }
}

template <int TX>
__device__ __forceinline__ void store_partials(const RowCtx& R, double (&acc)[TX], double* p)
{
    for (int off = 1; off < R.L; off <<= 1) {
#pragma unroll
        for (int i = 0; i < TX; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    }
    if (p && (R.lane & (R.L - 1)) == 0) {
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            if (i < R.cols) {
                const int ii = R.i0 + i;
                p[R.rowbase + (R.xpos ? ii : R.nx - 1 - ii)] = acc[i];
            }
        }
    }
}

template <typename T, int TX, int TY, bool DD, bool ANG, int PSI>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs A)
{
    constexpr int CH = TX * TY;
    constexpr int PER = (CH + kWave - 1) / kWave;
    constexpr int NG = ANG ? 0 : kMaxGroups;  // staged isotropic sources, one block per group
    __shared__ T lds_st[CH];
    __shared__ T lds_S[NG > 0 ? NG : 1][CH + 4];

    const int lane = threadIdx.x;
    if (!A.mode_all && A.ctl->active == 0) return;  // every system has stopped
    // sweep duration: first wave start .. last wave end on the device real-time clock
    if (lane == 0) atomicMin(&A.ctl->t_first, (unsigned long long)wall_clock64());
    const int epoch = A.ctl->epoch;
    const long long tag = (long long)epoch << 24;
    const T* __restrict__ sigma_t = (const T*)A.sigma_t;
    const T* __restrict__ srcp = (const T*)A.src;
    const T* __restrict__ angp = (const T*)A.ang_src;
    const T* __restrict__ inflow = (const T*)A.inflow;
    T* __restrict__ part = (T*)A.part;
    T* __restrict__ edge = (T*)A.edge;

    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(&A.ctl->ticket, 1);
        t = uniform(__shfl(t, 0, 64));
        if (t >= A.ntickets) break;
        const int2 tk = A.tickets[t];
        const int wsi = uniform(tk.x);
        const int strip = uniform(tk.y);
        const WaveStreamDev& W = A.ws[wsi];
        const ProblemDev& P = A.probs[uniform(W.prob)];
        const int L = uniform(W.L);
        const int G = kWave / L;

        // skip wave-streams whose systems have all stopped (flags change only between sweeps)
        bool any = false;
        for (int g = 0; g < G; ++g) {
            const int s = W.sys[g];
            if (s >= 0 && A.sysctl[s].state == 0) any = true;
        }
        if (A.mode_all) any = true;
        if (!any) continue;

        const int g = lane / L;
        int gsys = W.sys[g];
        if (gsys < 0) gsys = W.sys[0];
        const int gslot = W.slot[g];
        const LaneDev ld = A.lanes[wsi * kWave + lane];
        const T a = to_T<T>(DD ? 2.0 * ld.a : ld.a);
        const T b = to_T<T>(DD ? 2.0 * ld.b : ld.b);
        const T w = to_T<T>(ld.w);
        const T kappa = a + b;
        const SystemDev& SD = A.sys[gsys];
        const T* __restrict__ Ap = angp + SD.ang_off + ld.ord;
        const int64_t npad = SD.npad;
        // this lane's partial-flux slot, and the isotropic source of every group (uniform)
        T* const my_part = gslot >= 0 ? part + A.slot_off[gslot] : nullptr;
        const T* sbase[kMaxGroups];
#pragma unroll
        for (int k = 0; k < kMaxGroups; ++k) {
            const int sy = (k < G && W.sys[k] >= 0) ? W.sys[k] : W.sys[0];
            sbase[k] = srcp + A.sys[sy].src_off;
        }

        const int nx = P.nx, ny = P.ny;
        const int quad = W.quad;
        const bool xpos = (quad == 0 || quad == 3);
        const bool ypos = (quad < 2);
        const T* __restrict__ st = sigma_t + P.field_off;
        const int32_t* __restrict__ uflags = A.uflags + P.uflag_off + (int64_t)quad * P.nstrips * P.nchunks;

        const int j0 = strip * TY;
        const int rows = min(TY, ny - j0);
        T xl[TY];
#pragma unroll
        for (int r = 0; r < TY; ++r)
            xl[r] = (W.xin_off >= 0 && r < rows) ? inflow[W.xin_off + (int64_t)(j0 + r) * kWave + lane] : T(0);

        T* __restrict__ edge_mine = edge + W.edge_off + (int64_t)strip * nx * kWave;
        const T* __restrict__ edge_below = edge + W.edge_off + (int64_t)(strip - 1) * nx * kWave;
        long long* prog_mine = A.prog + W.prog_off + strip;
        long long* prog_below = A.prog + W.prog_off + strip - 1;
        const bool publish = (strip + 1 < P.nstrips);

        // storage cell of chunk element e = r*TX + i (clamped into the grid for ragged chunks)
        auto elem_cell = [&](int c, int e, bool& inside) -> int {
            const int r = e / TX, i = e % TX;
            int jj = j0 + r, ii = c * TX + i;
            inside = (jj < ny) && (ii < nx);
            jj = min(jj, ny - 1);
            ii = min(ii, nx - 1);
            const int j = ypos ? jj : ny - 1 - jj;
            const int is = xpos ? ii : nx - 1 - ii;
            return j * nx + is;
        };
        T pst[PER];
        T pS[NG > 0 ? NG : 1][PER];
        // anisotropic sources are per (cell, ordinate): each lane prefetches its own ordinate's
        // values for the whole next chunk (one coalesced 256-byte load per cell)
        constexpr int CA = ANG ? CH : 1;
        T pA[CA], cA[CA];
        auto prefetch = [&](int c) {
            if constexpr (ANG) {
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    bool inside;
                    const int cell = elem_cell(c, e, inside);
                    pA[e] = Ap[(int64_t)cell * npad];
                }
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int e = lane + k * kWave;
                if (e < CH) {
                    bool inside;
                    const int cell = elem_cell(c, e, inside);
                    pst[k] = st[cell];
                    if constexpr (NG > 0) {
#pragma unroll
                        for (int q = 0; q < NG; ++q)
                            if (q < G) pS[q][k] = inside ? sbase[q][cell] : T(0);
                    }
                }
            }
        };
        auto commit = [&]() {
            if constexpr (ANG) {
#pragma unroll
                for (int e = 0; e < CH; ++e) cA[e] = pA[e];
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int e = lane + k * kWave;
                if (e < CH) {
                    lds_st[e] = pst[k];
                    if constexpr (NG > 0) {
#pragma unroll
                        for (int q = 0; q < NG; ++q)
                            if (q < G) lds_S[q][e] = pS[q][k];
                    }
                }
            }
        };

        prefetch(0);
        for (int c = 0; c < P.nchunks; ++c) {
            const int i0 = c * TX;
            const int cols = min(TX, nx - i0);
            commit();
            if (c + 1 < P.nchunks) prefetch(c + 1);
            const int32_t umask = uflags[(int64_t)strip * P.nchunks + c];
            T yd[TX];
            if (strip == 0) {
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    yd[i] = (W.yin_off >= 0 && i < cols) ? inflow[W.yin_off + (int64_t)(i0 + i) * kWave + lane] : T(0);
            } else {
                wait_progress(prog_below, tag | (long long)(c + 1), A.ctl, A.spin_limit);
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    yd[i] = (i < cols) ? edge_load(edge_below + (int64_t)(i0 + i) * kWave + lane) : T(0);
            }
            auto do_row = [&](const int r) {
                const int jj = j0 + r;
                const int j = ypos ? jj : ny - 1 - jj;
                const int64_t rowbase = (int64_t)j * nx;
                T Sv[TX], acc[TX];
                if constexpr (ANG) {
#pragma unroll
                    for (int i = 0; i < TX; ++i) Sv[i] = cA[r * TX + i];
                } else {
#pragma unroll
                    for (int i = 0; i < TX; ++i) Sv[i] = lds_S[g][r * TX + i];
                }
                T xf = xl[r];
                if ((umask >> r) & 1) {
                    const T rr = rcp_fast(lds_st[r * TX] + kappa);
                    const T wr = w * rr, ar = a * rr, br = b * rr;
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        const T v = fma(br, yd[i], fma(ar, xf, wr * Sv[i]));
                        if (DD) {
                            xf = fma(T(2), v, -xf);
                            yd[i] = fma(T(2), v, -yd[i]);
                        } else {
                            xf = v;
                            yd[i] = v;
                        }
                        acc[i] = v;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        const T rr = rcp_fast(lds_st[r * TX + i] + kappa);
                        const T v = fma(b, yd[i], fma(a, xf, w * Sv[i])) * rr;
                        if (DD) {
                            xf = fma(T(2), v, -xf);
                            yd[i] = fma(T(2), v, -yd[i]);
                        } else {
                            xf = v;
                            yd[i] = v;
                        }
                        acc[i] = v;
                    }
                }
                xl[r] = xf;
                // lanes of empty groups alias ordinate 0 of system sys[0]: they never store
                if (PSI == 1 && gslot >= 0) {
                    T* __restrict__ po = (T*)A.psi_out + SD.ang_off + ld.ord;
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        const int ii = i0 + i;
                        if (i < cols) po[(rowbase + (xpos ? ii : nx - 1 - ii)) * npad] = acc[i];
                    }
                } else if (PSI == 2 && gslot >= 0) {
                    __hip_bfloat16* __restrict__ po = (__hip_bfloat16*)A.psi_out + SD.ang_off + ld.ord;
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        const int ii = i0 + i;
                        if (i < cols) po[(rowbase + (xpos ? ii : nx - 1 - ii)) * npad] = __float2bfloat16((float)acc[i]);
                    }
                }
                const RowCtx R{lane, g, L, rowbase, i0, nx, xpos, cols};
                store_partials<TX>(R, acc, my_part);
            };
            if constexpr (ANG || ROM_ROW_UNROLL) {
#pragma unroll
                for (int r = 0; r < TY; ++r)
                    if (r < rows) do_row(r);
            } else {
                for (int r = 0; r < rows; ++r) do_row(r);
            }
            if (publish) {
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    if (i < cols) edge_store(edge_mine + (int64_t)(i0 + i) * kWave + lane, yd[i]);
                stores_complete();
                if (lane == 0)
                    __hip_atomic_store(prog_mine, tag | (long long)(c + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (lane == 0) atomicMax(&A.ctl->t_last, (unsigned long long)wall_clock64());
}

// ------------------------------------------------------------------------------------ combine
__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// Finalize one iteration for every running system (single thread).
__device__ void finalize_iteration(const CombineArgs& A)
{
    int active = 0;
    for (int s = 0; s < A.nsys; ++s) {
        SysCtl& c = A.sysctl[s];
        if (c.state != 0) continue;
        const double d = bitsd(__hip_atomic_load(&c.dmax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const double p = bitsd(__hip_atomic_load(&c.pmax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const double r = p > 0.0 ? d / p : 0.0;
        c.r_prev = c.r;
        c.r = r;
        c.iter += 1;
        if (A.rhist && c.iter <= A.max_iter) A.rhist[(int64_t)s * A.max_iter + c.iter - 1] = r;
        if (!(d <= 1.0e300) || !(p <= 1.0e300))
            c.state = 3;
        else if (r <= A.tol)
            c.state = 1;
        else if (c.iter >= A.max_iter)
            c.state = 2;
        c.dmax_bits = 0ull;
        c.pmax_bits = 0ull;
        if (c.state == 0) ++active;
    }
    A.ctl->active = active;
}

template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs A)
{
    const int tid = threadIdx.x;
    // Every block of a launch reads `active` before the last block of the same launch can change
    // it, so either all blocks of this launch return here or none does.
    if (A.mode == 0 && A.ctl->active == 0) return;
    const int2 blk = A.blocks[blockIdx.x];
    const int s = blk.x;
    const SystemDev& SD = A.sys[s];
    const ProblemDev& P = A.probs[SD.prob];
    const int cells = P.nx * P.ny;
    const bool run = A.mode == 1 || A.sysctl[s].state == 0;
    double dmax = 0.0, pmax = 0.0;
    if (run) {
        const T* __restrict__ part = (const T*)A.part;
        T* __restrict__ phi = (T*)A.phi + SD.phi_off;
        T* __restrict__ src = (T*)A.src + SD.src_off;
        const T* __restrict__ ss = (const T*)A.sigma_s + P.field_off;
        const T* __restrict__ q = (const T*)A.q + P.field_off;
        const int ns = SD.nslots;
        const int64_t* __restrict__ soff = A.slot_off;
        const int32_t* __restrict__ sord = A.slot_order + SD.slot_first;
        const int c1 = min(cells, blk.y + A.cells_per_block);
        constexpr int U = 4;  // cells per thread in flight
        for (int base = blk.y + tid; base < c1; base += 256 * U) {
            T v[U];
            T old[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cell = base + u * 256;
                v[u] = T(0);
                old[u] = cell < c1 ? phi[cell] : T(0);
            }
            for (int k = 0; k < ns; ++k) {
                const T* __restrict__ pk = part + soff[sord[k]];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cell = base + u * 256;
                    if (cell < c1) v[u] += pk[cell];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cell = base + u * 256;
                if (cell < c1) {
                    dmax = fmax(dmax, fabs((double)v[u] - (double)old[u]));
                    pmax = fmax(pmax, fabs((double)v[u]));
                    phi[cell] = v[u];
                    src[cell] = fma(ss[cell], v[u], q[cell]);
                }
            }
        }
    }
    // block maxima: wave reduction, then across the 4 waves
    for (int off = 32; off > 0; off >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        pmax = fmax(pmax, __shfl_xor(pmax, off, 64));
    }
    __shared__ double sd[4], sp[4];
    if ((tid & 63) == 0) {
        sd[tid >> 6] = dmax;
        sp[tid >> 6] = pmax;
    }
    __syncthreads();
    if (tid == 0) {
        dmax = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
        pmax = fmax(fmax(sp[0], sp[1]), fmax(sp[2], sp[3]));
        if (run && A.mode == 0) {
            atomicMax(&A.sysctl[s].dmax_bits, dbits(dmax));  // non-negative doubles order as integers
            atomicMax(&A.sysctl[s].pmax_bits, dbits(pmax));
        }
        // The maxima are device-scope atomics; waiting for their completion before counting the
        // block in is all the last block needs (the fluxes themselves are read by later kernels).
        stores_complete();
        const int done = atomicAdd(&A.ctl->blocks_done, 1);
        if (done == (int)gridDim.x - 1) {
            if (A.mode == 0) finalize_iteration(A);
            if (A.ctl->t_last > A.ctl->t_first && A.ctl->t_first != ~0ull) {
                A.ctl->sweep_ticks += A.ctl->t_last - A.ctl->t_first;
                A.ctl->sweeps += 1;
            }
            A.ctl->t_first = ~0ull;
            A.ctl->t_last = 0ull;
            A.ctl->blocks_done = 0;
            A.ctl->ticket = 0;
            A.ctl->epoch += 1;
        }
    }
}

// Prepare a sweep that is not preceded by a combine step: reset the ticket counter, new epoch.
__global__ void sweep_prologue_kernel(Ctl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->ticket = 0;
        ctl->blocks_done = 0;
        ctl->epoch += 1;
    }
}

// Clear per-system state before a solve (graph-safe: a kernel, not a memset).
__global__ void reset_systems_kernel(SysCtl* sc, int nsys, Ctl* ctl)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) {
        sc[s].dmax_bits = 0ull;
        sc[s].pmax_bits = 0ull;
        sc[s].iter = 0;
        sc[s].state = 0;
        sc[s].grow = 0;
        sc[s].r = 1.0;
        sc[s].r_prev = 1.0;
    }
    if (s == 0) {
        ctl->active = nsys;
        ctl->error = 0;
        ctl->sweeps = 0;
        ctl->t_first = ~0ull;
        ctl->t_last = 0ull;
        ctl->sweep_ticks = 0ull;
        ctl->ticket = 0;
        ctl->blocks_done = 0;
        ctl->epoch += 1;
    }
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------------------------ moments
// mean = (1/t) sum_s phi_s,  var = sum_s (phi_s - mean)^2 / (t - 1), samples in index order, FP64.
// With a running accumulator (count > 0) the batch is merged by the pairwise update of Chan,
// Golub and LeVeque: delta = mean_b - mean_a, M2 = M2_a + M2_b + delta^2 n_a n_b / n.
template <typename T>
__global__ void moments_kernel(MomentsArgs A)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= A.cells) return;
    const T* __restrict__ phi = (const T*)A.phi;
    double s1 = 0.0;
    for (int s = 0; s < A.t; ++s) s1 += (double)phi[A.phi_offs[s] + cell];
    const double mb = s1 / (double)A.t;
    double m2 = 0.0;
    for (int s = 0; s < A.t; ++s) {
        const double d = (double)phi[A.phi_offs[s] + cell] - mb;
        m2 += d * d;
    }
    if (A.count == 0) {
        A.mean[cell] = mb;
        A.m2[cell] = m2;
    } else {
        const double na = (double)A.count, nb = (double)A.t, n = na + nb;
        const double ma = A.mean[cell];
        const double delta = mb - ma;
        A.mean[cell] = ma + delta * (nb / n);
        A.m2[cell] = A.m2[cell] + m2 + delta * delta * (na * nb / n);
    }
}

__global__ void finish_var_kernel(const double* m2, double* var, int64_t cells, int64_t t)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell < cells) var[cell] = t > 1 ? m2[cell] / (double)(t - 1) : 0.0;
}

// ------------------------------------------------------------------------------------ contraction
// S[m][n] = sigma_s[m] * sum_k A[m][k] Bt[n][k] + q[m], A = Psi' [cells][npad], Bt = P^T.
//
// BF16 MFMA version: 256 threads = 4 waves in a 2 x 2 arrangement, block tile 128 x 128, K step
// 32 staged in LDS; each wave owns 64 x 64 = 2 x 2 tiles of v_mfma_f32_32x32x16_bf16.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int GM = 128, GN = 128, GK = 32;
constexpr int LDS_PAD = 8;  // bf16 elements of padding per LDS row (keeps 16-byte alignment)

__global__ __launch_bounds__(256) void contract_bf16_kernel(ContractArgs A)
{
    if (A.sysctl && A.sysctl[A.sys_index].state != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[GM][GK + LDS_PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[GN][GK + LDS_PAD];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / 2, wn = wave % 2;
    // XCD-aware block order is left to the dispatcher; blocks walk N fastest so that one A tile
    // (the large operand) is reused from L2 by the N/GN blocks that follow it.
    // Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Renumber them
    // so that every XCD owns a contiguous run of logical tiles: the N/GN tiles that share one A
    // row-block then run on the same XCD and read A from HBM once.
    const int nblk_n = A.N / GN;
    const int nb = gridDim.x;
    const int lb = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
    const int bm = lb / nblk_n, bn = lb % nblk_n;
    const int m0 = bm * GM, n0 = bn * GN;
    const __bf16* __restrict__ Ag = (const __bf16*)A.a;
    const __bf16* __restrict__ Bg = (const __bf16*)A.bt;

    f32x16_t acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.0f;

    // global -> LDS: each tile is 128 rows x 32 bf16 = 128 x 64 B; 256 threads x 2 x 16 B
    for (int k0 = 0; k0 < A.K; k0 += GK) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int idx = tid + h * 256;  // 0..511
            const int row = idx / 4, seg = idx % 4;
            const int am = m0 + row;
            uint4 va = make_uint4(0, 0, 0, 0);
            if (am < A.M) va = *(const uint4*)(Ag + (int64_t)am * A.K + k0 + seg * 8);
            *(uint4*)&As[row][seg * 8] = va;
            const uint4 vb = *(const uint4*)(Bg + (int64_t)(n0 + row) * A.K + k0 + seg * 8);
            *(uint4*)&Bs[row][seg * 8] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            bf16x8_t af[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int r = wm * 64 + x * 32 + (lane % 32);
                af[x] = *(const bf16x8_t*)&As[r][kk + 8 * (lane / 32)];
            }
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int r = wn * 64 + y * 32 + (lane % 32);
                bfr[y] = *(const bf16x8_t*)&Bs[r][kk + 8 * (lane / 32)];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[x], bfr[y], acc[x][y], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: lane holds column (lane % 32) and rows 8*(e/4) + 4*(lane/32) + e%4 of each tile
    const float* __restrict__ ss = (const float*)A.sigma_s;
    const float* __restrict__ q = (const float*)A.q;
    float* __restrict__ out = (float*)A.out;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int col = n0 + wn * 64 + y * 32 + (lane % 32);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = m0 + wm * 64 + x * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
                if (row < A.M) out[(int64_t)row * A.N + col] = fmaf(ss[row], acc[x][y][e], q[row]);
            }
        }
    }
}

// Plain tiled contraction (FP64 or FP32 operands, same precision out), 16 x 16 threads, 64 x 64
// block tile, each thread a 4 x 4 micro-tile.
template <typename T>
__global__ __launch_bounds__(256) void contract_plain_kernel(ContractArgs A)
{
    if (A.sysctl && A.sysctl[A.sys_index].state != 0) return;
    __shared__ T As[16][64 + 1];
    __shared__ T Bs[16][64 + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int nblk_n = (A.N + 63) / 64;
    const int m0 = (blockIdx.x / nblk_n) * 64, n0 = (blockIdx.x % nblk_n) * 64;
    const T* __restrict__ Ag = (const T*)A.a;
    const T* __restrict__ Bg = (const T*)A.bt;
    T acc[4][4] = {};
    for (int k0 = 0; k0 < A.K; k0 += 16) {
        for (int idx = threadIdx.x; idx < 64 * 16; idx += 256) {
            const int r = idx / 16, k = idx % 16;
            const int gm = m0 + r, gn = n0 + r, gk = k0 + k;
            As[k][r] = (gm < A.M && gk < A.K) ? Ag[(int64_t)gm * A.K + gk] : T(0);
            Bs[k][r] = (gn < A.N && gk < A.K) ? Bg[(int64_t)gn * A.K + gk] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            T av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[k][ty * 4 + u];
                bv[u] = Bs[k][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    const T* __restrict__ ss = (const T*)A.sigma_s;
    const T* __restrict__ q = (const T*)A.q;
    T* __restrict__ out = (T*)A.out;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int row = m0 + ty * 4 + u;
        if (row >= A.M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = n0 + tx * 4 + v;
            if (col < A.N) out[(int64_t)row * A.N + col] = fma(ss[row], acc[u][v], q[row]);
        }
    }
}

// FP32 angular flux -> BF16 copy (used when the sweep stored FP32 psi').
__global__ void cast_bf16_kernel(const float* __restrict__ in, __hip_bfloat16* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = __float2bfloat16(in[i]);
}

// ------------------------------------------------------------------------------------ launchers
template <typename T, int TX, int TY, bool DD, bool ANG, int PSI>
static hipError_t launch_sweep_t(const SweepArgs& a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_kernel<T, TX, TY, DD, ANG, PSI>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T, int TX, int TY>
static hipError_t launch_sweep_tile(const SweepArgs& a, int grid, bool dd, bool ang, int psi, hipStream_t s)
{
    if (dd) {
        if (ang) {
            if (psi == 1) return launch_sweep_t<T, TX, TY, true, true, 1>(a, grid, s);
            if (psi == 2) return launch_sweep_t<T, TX, TY, true, true, 2>(a, grid, s);
            return launch_sweep_t<T, TX, TY, true, true, 0>(a, grid, s);
        }
        if (psi == 1) return launch_sweep_t<T, TX, TY, true, false, 1>(a, grid, s);
        return launch_sweep_t<T, TX, TY, true, false, 0>(a, grid, s);
    }
    if (ang) {
        if (psi == 1) return launch_sweep_t<T, TX, TY, false, true, 1>(a, grid, s);
        if (psi == 2) return launch_sweep_t<T, TX, TY, false, true, 2>(a, grid, s);
        return launch_sweep_t<T, TX, TY, false, true, 0>(a, grid, s);
    }
    if (psi == 1) return launch_sweep_t<T, TX, TY, false, false, 1>(a, grid, s);
    return launch_sweep_t<T, TX, TY, false, false, 0>(a, grid, s);
}

template <typename T>
static hipError_t launch_sweep_T(const SweepArgs& a, int grid, int tx, int ty, bool dd, bool ang, int psi,
                                 hipStream_t s)
{
    if (tx == 8 && ty == 4) return launch_sweep_tile<T, 8, 4>(a, grid, dd, ang, psi, s);
    if (tx == 8 && ty == 8) return launch_sweep_tile<T, 8, 8>(a, grid, dd, ang, psi, s);
    if (tx == 16 && ty == 4) return launch_sweep_tile<T, 16, 4>(a, grid, dd, ang, psi, s);
    if (tx == 16 && ty == 8) return launch_sweep_tile<T, 16, 8>(a, grid, dd, ang, psi, s);
    if (tx == 16 && ty == 16) return launch_sweep_tile<T, 16, 16>(a, grid, dd, ang, psi, s);
    return hipErrorInvalidValue;
}

bool sweep_tile_supported(int tx, int ty)
{
    return (tx == 8 && (ty == 4 || ty == 8)) || (tx == 16 && (ty == 4 || ty == 8 || ty == 16));
}

hipError_t launch_sweep(const SweepArgs& a, int grid, bool fp64, int tx, int ty, bool dd, bool ang, int psi,
                        hipStream_t s)
{
    if (fp64) {
        if (psi == 2) return hipErrorInvalidValue;
        return launch_sweep_T<double>(a, grid, tx, ty, dd, ang, psi, s);
    }
    return launch_sweep_T<float>(a, grid, tx, ty, dd, ang, psi, s);
}

hipError_t launch_combine(const CombineArgs& a, int nblocks, bool fp64, hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(combine_kernel<double>, dim3(nblocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(combine_kernel<float>, dim3(nblocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_prologue(Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_prologue_kernel, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

hipError_t launch_reset_systems(SysCtl* sc, int nsys, Ctl* ctl, hipStream_t s)
{
    const int nb = (nsys + 255) / 256;
    hipLaunchKernelGGL(reset_systems_kernel, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, sc, nsys, ctl);
    return hipGetLastError();
}

hipError_t launch_fill(void* p, int64_t n, bool fp64, double v, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (n <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(nb), dim3(256), 0, s, (double*)p, n, v);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(nb), dim3(256), 0, s, (float*)p, n, (float)v);
    return hipGetLastError();
}

hipError_t launch_moments(const MomentsArgs& a, bool fp64, hipStream_t s)
{
    const int nb = (int)((a.cells + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(moments_kernel<double>, dim3(nb), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(moments_kernel<float>, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finish_var(const double* m2, double* var, int64_t cells, int64_t t, hipStream_t s)
{
    const int nb = (int)((cells + 255) / 256);
    hipLaunchKernelGGL(finish_var_kernel, dim3(nb), dim3(256), 0, s, m2, var, cells, t);
    return hipGetLastError();
}

hipError_t launch_contract(const ContractArgs& a, int kind, hipStream_t s)
{
    if (kind == 0) {
        if (a.N % GN != 0 || a.K % GK != 0) return hipErrorInvalidValue;
        const int grid = ((a.M + GM - 1) / GM) * (a.N / GN);
        hipLaunchKernelGGL(contract_bf16_kernel, dim3(grid), dim3(256), 0, s, a);
    } else {
        const int grid = ((a.M + 63) / 64) * ((a.N + 63) / 64);
        if (kind == 1)
            hipLaunchKernelGGL(contract_plain_kernel<float>, dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(contract_plain_kernel<double>, dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* in, void* out, int64_t n, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(nb), dim3(256), 0, s, in, (__hip_bfloat16*)out, n);
    return hipGetLastError();
}

}  // namespace rom

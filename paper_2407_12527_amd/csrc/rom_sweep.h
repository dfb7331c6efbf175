// rom_sweep.h -- the transport-sweep kernel template of librom (instantiated per tile shape in
// rom_sweep_*.hip so the variants compile in parallel).
#pragma once
#include "rom_common.h"

namespace rom {

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
// Linear kernel (MOM = 4): the source of lane l is S0 + c_l S1 + s_l S2 (three staged planes),
// and besides phi the row is reduced three more times with the lane weights c/r, s/r and 1/r
// (Jx~, Jy~ and, when the kernel is normalized on an asymmetric set, phi~) into planes 1..3 of
// the lane group's partial slot.
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
    int lane, g;
    int64_t rowbase;
    int i0, nx;
    bool xpos;
    int cols;
};

// Row scalar-flux partials: float rows use the butterfly, double rows a plain xor shuffle.
template <int TX, int L>
__device__ __forceinline__ void store_partials(const RowCtx& R, float (&acc)[TX], float* p)
{
    int c = 0;
    const float v = butterfly<TX, L>(R.lane, acc, c);
    const bool rep = butterfly_rep<TX, L>(R.lane);
    if (rep && p && c < R.cols) {
        const int ii = R.i0 + c;
        p[R.rowbase + (R.xpos ? ii : R.nx - 1 - ii)] = v;
    }
}

template <int TX, int L>
__device__ __forceinline__ void store_partials(const RowCtx& R, double (&acc)[TX], double* p)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) {
#pragma unroll
        for (int i = 0; i < TX; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    }
    if (p && (R.lane & (L - 1)) == 0) {
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            if (i < R.cols) {
                const int ii = R.i0 + i;
                p[R.rowbase + (R.xpos ? ii : R.nx - 1 - ii)] = acc[i];
            }
        }
    }
}

// A workgroup of NW wavefronts (NW <= kMaxBand, chosen per plan) owns a band of NW consecutive
// strips of one wave-stream: wave k sweeps strip band*NW + k.  Edges between strips of a band go
// through LDS ring buffers (RB chunk slots per boundary, produced / consumed counters in LDS);
// only the band's top edge goes to global memory for the next band, behind a progress counter.
// Isotropic flux-only step sweeps reduce each row after the next row has read it (below); 0 takes
// rows in pairs and reduces each at once (c5 sweep 2751 us against 2660 us deferred, c3 861 / 816).
#ifndef ROM_SWEEP_DEFER
#define ROM_SWEEP_DEFER 1
#endif

// Waves per SIMD the compiler must leave room for.  The FP32 isotropic flux-only step sweeps fit
// four waves in 128 VGPRs (tiles of up to 128 cells, and 16 x 16 with 64-lane groups without
// spilling; 16 x 16 with 32-lane groups spills 32 bytes outside the row loop); the extra wave
// hides the LDS and hand-off waits of the row loop (c5 sweep 58.3 -> 53.9 ms per solve, c3 sweep
// 950 -> 935 us).  Every other variant would spill more at that bound and keeps the compiler's
// own register budget.
template <typename T, int TX, int TY, bool DD, bool ANG, int PSI, int L, int MOM>
constexpr int sweep_waves_per_simd()
{
    return (sizeof(T) == 4 && !DD && !ANG && PSI == 0 && MOM == 1 && (TX * TY <= 128 || L >= 32)) ? 4 : 1;
}

template <typename T, int TX, int TY, bool DD, bool ANG, int PSI, int L, int MOM>
__global__ __launch_bounds__(64 * kMaxBand)
__attribute__((amdgpu_waves_per_eu(sweep_waves_per_simd<T, TX, TY, DD, ANG, PSI, L, MOM>())))
void sweep_kernel(SweepArgs A)
{
    static_assert(MOM == 1 || (MOM == 4 && !ANG && PSI == 0), "moment sweeps take staged sources only");
    constexpr int G = kWave / L;  // lane groups per wavefront
    constexpr int CH = TX * TY;
    constexpr int PER = (CH + kWave - 1) / kWave;
    constexpr int NSRC = MOM == 4 ? 3 : 1;             // source planes per group
    constexpr int NG = ANG ? 0 : (kWave / L) * NSRC;   // staged source blocks (group-major)
    constexpr int NGD = NG > 0 ? NG : 1;
    constexpr int RB = kRingSlots;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & (kWave - 1);
    const int NW = blockDim.x >> 6;
    // dynamic LDS, sized by the launch for NW waves (see sweep_lds_bytes)
    extern __shared__ __align__(16) unsigned char smem[];
    T (*lds_st)[CH] = (T (*)[CH])smem;
    T (*lds_S)[NGD][CH + 4] = (T (*)[NGD][CH + 4])(smem + sizeof(T) * NW * CH);
    T (*ring)[RB][TX * kWave] = (T (*)[RB][TX * kWave])(smem + sizeof(T) * NW * (CH + NGD * (CH + 4)));
    int* produced = (int*)(smem + sizeof(T) * (NW * (CH + NGD * (CH + 4)) + (NW > 1 ? NW - 1 : 1) * RB * TX * kWave));
    int* consumed = produced + kMaxBand;
    int& s_ticket = consumed[kMaxBand];
    if (!A.mode_all && A.ctl->active == 0) return;  // every system has stopped
    const int epoch = A.ctl->epoch;
    const long long tag = (long long)epoch << 24;
    const T* __restrict__ sigma_t = (const T*)A.sigma_t;
    const T* __restrict__ srcp = (const T*)A.src;
    const T* __restrict__ angp = (const T*)A.ang_src;
    const T* __restrict__ inflow = (const T*)A.inflow;
    T* __restrict__ part = (T*)A.part;
    T* __restrict__ edge = (T*)A.edge;

    for (;;) {
        if (threadIdx.x == 0) {
            s_ticket = atomicAdd(&A.ctl->ticket, 1);
            sweep_clock(A.ctl, s_ticket, A.ntickets);
        }
        if (lane == 0) {
            produced[wave] = 0;
            consumed[wave] = 0;
        }
        __syncthreads();
        const int t = s_ticket;
        if (t >= A.ntickets) break;  // uniform over the workgroup
        const int2 tk = A.tickets[t];
        const int wsi = uniform(tk.x);
        const int band = uniform(tk.y);
        // ticket metadata, read once and kept in scalar registers
        const WaveStreamDev& Wg = A.ws[wsi];
        const int wprob = uniform(Wg.prob), quad = uniform(Wg.quad), prog_off = uniform(Wg.prog_off);
        const int64_t edge_off = uniform64(Wg.edge_off), xin_off = uniform64(Wg.xin_off), yin_off = uniform64(Wg.yin_off);
        int wsys[kMaxGroups], wslot[kMaxGroups];
#pragma unroll
        for (int k = 0; k < kMaxGroups; ++k) {
            wsys[k] = uniform(Wg.sys[k]);
            wslot[k] = uniform(Wg.slot[k]);
        }
        const ProblemDev& Pg = A.probs[wprob];
        const int nx = uniform(Pg.nx), ny = uniform(Pg.ny), nchunks = uniform(Pg.nchunks), nstrips = uniform(Pg.nstrips);
        const int64_t field_off = uniform64(Pg.field_off), uflag_off = uniform64(Pg.uflag_off);
        const int64_t plane = (int64_t)nx * ny;  // source and partial planes of the linear kernel
        const int strip = band * NW + wave;

        // skip wave-streams whose systems have all stopped (flags change only between sweeps)
        bool any = A.mode_all != 0;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (wsys[k] >= 0 && uniform(A.sysctl[wsys[k]].state) == 0) any = true;
        if (any && strip < nstrips) {
            const int g = lane / L;
            int gsys = wsys[0], gslot = -1;
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (k == g) {
                    gsys = wsys[k] >= 0 ? wsys[k] : wsys[0];
                    gslot = wslot[k];
                }
            const LaneDev ld = A.lanes[wsi * kWave + lane];
            const T a = to_T<T>(DD ? 2.0 * ld.a : ld.a);
            const T b = to_T<T>(DD ? 2.0 * ld.b : ld.b);
            const T w = to_T<T>(ld.w);
            const T kappa = a + b;
            // linear kernel: source direction cosines and moment weights of this lane
            const T lc = to_T<T>(ld.c), ls = to_T<T>(ld.s);
            const T m1 = to_T<T>(ld.m1), m2 = to_T<T>(ld.m2), m3 = to_T<T>(ld.m3);
            const SystemDev& SD = A.sys[gsys];
            const T* __restrict__ Ap = angp + SD.ang_off + ld.ord;
            const int64_t npad = SD.npad;
            T* const my_part = gslot >= 0 ? part + A.slot_off[gslot] : nullptr;
            const T* sbase[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int sy = wsys[k] >= 0 ? wsys[k] : wsys[0];
                sbase[k] = srcp + uniform64(A.sys[sy].src_off);
            }

            const bool xpos = (quad == 0 || quad == 3);
            const bool ypos = (quad < 2);
            const T* __restrict__ st = sigma_t + field_off;
            const int32_t* __restrict__ uflags = A.uflags + uflag_off + (int64_t)quad * nstrips * nchunks +
                                                 (int64_t)strip * nchunks;

            const int j0 = strip * TY;
            const int rows = min(TY, ny - j0);
            T xl[TY];
#pragma unroll
            for (int r = 0; r < TY; ++r)
                xl[r] = (xin_off >= 0 && r < rows) ? inflow[xin_off + (int64_t)(j0 + r) * kWave + lane] : T(0);

            // where the bottom edge comes from and where the top edge goes
            const bool from_global = (wave == 0 && strip > 0);
            const bool has_out = strip + 1 < nstrips;
            const bool to_global = has_out && (wave == NW - 1);
            const T* __restrict__ edge_below = edge + edge_off + (int64_t)(band - 1) * nx * kWave;
            T* __restrict__ edge_mine = edge + edge_off + (int64_t)band * nx * kWave;
            long long* prog_below = A.prog + prog_off + band - 1;
            long long* prog_mine = A.prog + prog_off + band;

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
            int pmask = 0, cmask = 0;  // row-uniformity mask of the prefetched / current chunk
            // anisotropic sources are per (cell, ordinate): each lane prefetches its own ordinate's
            // values for the whole next chunk (one coalesced 256-byte load per cell)
            constexpr int CA = ANG ? CH : 1;
            T pA[CA], cA[CA];
            auto prefetch = [&](int c) {
                pmask = uflags[c];
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
                            for (int q = 0; q < NG; ++q) {
                                // clamped cell: always a valid address
                                const T v = sbase[q / NSRC][(q % NSRC) * plane + cell];
                                pS[q][k] = inside ? v : T(0);
                            }
                        }
                    }
                }
            };
            auto commit = [&]() {
                cmask = uniform(pmask);
                if constexpr (ANG) {
#pragma unroll
                    for (int e = 0; e < CH; ++e) cA[e] = pA[e];
                }
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int e = lane + k * kWave;
                    if (e < CH) {
                        lds_st[wave][e] = pst[k];
                        if constexpr (NG > 0) {
#pragma unroll
                            for (int q = 0; q < NG; ++q) lds_S[wave][q][e] = pS[q][k];
                        }
                    }
                }
            };

            prefetch(0);
            for (int c = 0; c < nchunks; ++c) {
                const int i0 = c * TX;
                const int cols = min(TX, nx - i0);
                commit();
                if (c + 1 < nchunks) prefetch(c + 1);
                const int32_t umask = cmask;
                T yd[TX];
                if (strip == 0) {
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        yd[i] = (yin_off >= 0 && i < cols) ? inflow[yin_off + (int64_t)(i0 + i) * kWave + lane] : T(0);
                } else if (from_global) {
                    wait_progress(prog_below, tag | (long long)(c + 1), A.ctl, A.spin_limit, A.wait_ticks);
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        yd[i] = (i < cols) ? edge_load(edge_below + (int64_t)(i0 + i) * kWave + lane) : T(0);
                } else {
                    // from the wave below in this band, through its LDS ring
                    lds_wait(&produced[wave - 1], c + 1, A.ctl, A.spin_limit, A.wait_ticks);
                    const T* slot = ring[wave - 1][c % RB];
#pragma unroll
                    for (int i = 0; i < TX; ++i) yd[i] = slot[i * kWave + lane];
                    if (lane == 0) __hip_atomic_store(&consumed[wave - 1], c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                auto do_row = [&](const int r) {
                    const int jj = j0 + r;
                    const int j = ypos ? jj : ny - 1 - jj;
                    const int64_t rowbase = (int64_t)j * nx;
                    T Sv[TX], acc[TX];
                    if constexpr (ANG) {
#pragma unroll
                        for (int i = 0; i < TX; ++i) Sv[i] = cA[r * TX + i];
                    } else if constexpr (MOM == 4) {
                        const T* s0 = lds_S[wave][g * NSRC];
                        const T* s1 = lds_S[wave][g * NSRC + 1];
                        const T* s2 = lds_S[wave][g * NSRC + 2];
#pragma unroll
                        for (int i = 0; i < TX; ++i) Sv[i] = fma(ls, s2[r * TX + i], fma(lc, s1[r * TX + i], s0[r * TX + i]));
                    } else {
#pragma unroll
                        for (int i = 0; i < TX; ++i) Sv[i] = lds_S[wave][g][r * TX + i];
                    }
                    T xf = xl[r];
                    if ((umask >> r) & 1) {
                        const T rr = rcp_fast(lds_st[wave][r * TX] + kappa);
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
                            const T rr = rcp_fast(lds_st[wave][r * TX + i] + kappa);
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
                    const RowCtx R{lane, g, rowbase, i0, nx, xpos, cols};
                    if constexpr (MOM == 4) {
                        // moments first: the FP64 reduction works in place on its input
                        T a1[TX], a2[TX], a3[TX];
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            a1[i] = acc[i] * m1;
                            a2[i] = acc[i] * m2;
                            a3[i] = acc[i] * m3;
                        }
                        store_partials<TX, L>(R, acc, my_part);
                        store_partials<TX, L>(R, a1, my_part ? my_part + plane : nullptr);
                        store_partials<TX, L>(R, a2, my_part ? my_part + 2 * plane : nullptr);
                        if (A.mom_r) store_partials<TX, L>(R, a3, my_part ? my_part + 3 * plane : nullptr);
                    } else {
                        store_partials<TX, L>(R, acc, my_part);
                    }
                };
                // Isotropic flux-only step sweeps (the deferred form): a row's values are the
                // next row's y-face inputs, and the lane reduction that forms the row's scalar
                // flux overwrites its operands (the permlane swaps), so reducing a row while its
                // values are still needed costs a copy of each.  Instead the rows alternate
                // between two banks and each row is reduced once the next row has read it; the
                // chunk's last row is reduced after it has left as the strip's top edge.
                constexpr bool DEFER = ROM_SWEEP_DEFER && !DD && !ANG && MOM == 1 && PSI == 0;
                T ydB[DEFER ? TX : 1];
                auto row_update = [&](const int r, const T (&yin)[TX], T (&yout)[TX]) {
                    T Sv[TX];
#pragma unroll
                    for (int i = 0; i < TX; ++i) Sv[i] = lds_S[wave][g][r * TX + i];
                    T xf = xl[r];
                    if ((umask >> r) & 1) {
                        const T rr = rcp_fast(lds_st[wave][r * TX] + kappa);
                        const T wr = w * rr, ar = a * rr, br = b * rr;
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            xf = fma(br, yin[i], fma(ar, xf, wr * Sv[i]));
                            yout[i] = xf;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            const T rr = rcp_fast(lds_st[wave][r * TX + i] + kappa);
                            xf = fma(b, yin[i], fma(a, xf, w * Sv[i])) * rr;
                            yout[i] = xf;
                        }
                    }
                    xl[r] = xf;
                };
                auto row_reduce = [&](const int r, T (&vals)[TX]) {
                    const int jj = j0 + r;
                    const int j = ypos ? jj : ny - 1 - jj;
                    const RowCtx R{lane, g, (int64_t)j * nx, i0, nx, xpos, cols};
                    store_partials<TX, L>(R, vals, my_part);
                };
                if constexpr (ANG) {
#pragma unroll
                    for (int r = 0; r < TY; ++r)
                        if (r < rows) do_row(r);
                } else if constexpr (DEFER) {
                    int r = 0;
                    for (; r + 1 < rows; r += 2) {
                        row_update(r, yd, ydB);
                        if (r > 0) row_reduce(r - 1, yd);  // yd held row r - 1 (the chunk's inflow at r = 0)
                        row_update(r + 1, ydB, yd);
                        row_reduce(r, ydB);
                    }
                    if (r < rows) {  // an odd row count (a ragged strip): the last row
                        row_update(r, yd, ydB);
                        if (r > 0) row_reduce(r - 1, yd);
#pragma unroll
                        for (int i = 0; i < TX; ++i) yd[i] = ydB[i];
                    }
                    // yd now holds the chunk's last row: its top edge, reduced below once sent
                } else {
                    int r = 0;
                    if constexpr (MOM == 1 && PSI == 0) {
                        // isotropic flux-only sweeps take rows in pairs: the second row takes the
                        // first's y-face values directly, halving the register moves that carry
                        // them around the loop (the other variants would lose a wave of occupancy)
                        for (; r + 1 < rows; r += 2) {
                            do_row(r);
                            do_row(r + 1);
                        }
                    }
                    for (; r < rows; ++r) do_row(r);
                }
                if (to_global) {
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        if (i < cols) edge_store(edge_mine + (int64_t)(i0 + i) * kWave + lane, yd[i]);
                    stores_complete();
                    if (lane == 0)
                        __hip_atomic_store(prog_mine, tag | (long long)(c + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else if (has_out) {
                    // to the wave above in this band: wait until it has consumed slot c - RB
                    if (c >= RB) lds_wait(&consumed[wave], c + 1 - RB, A.ctl, A.spin_limit, A.wait_ticks);
                    T* slot = ring[wave][c % RB];
#pragma unroll
                    for (int i = 0; i < TX; ++i) slot[i * kWave + lane] = yd[i];
                    if (lane == 0) __hip_atomic_store(&produced[wave], c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if constexpr (DEFER) row_reduce(rows - 1, yd);
            }
        }
        __syncthreads();  // the band is done before its LDS is reused
    }
}


inline size_t sweep_lds_bytes_t(size_t esz, int tx, int ty, bool ang, int L, int nw, int mom)
{
    const size_t ch = (size_t)tx * ty;
    const size_t ngd = ang ? 1 : (size_t)(kWave / L) * (mom == 4 ? 3 : 1);
    return esz * ((size_t)nw * (ch + ngd * (ch + 4)) + (size_t)(nw > 1 ? nw - 1 : 1) * kRingSlots * tx * kWave) +
           sizeof(int) * (2 * kMaxBand + 1);
}

template <typename T, int TX, int TY, bool DD, bool ANG, int PSI, int L, int MOM = 1>
hipError_t launch_sweep_t(const SweepArgs& a, int grid, hipStream_t s)
{
    if (a.band < 1 || a.band > kMaxBand) return hipErrorInvalidValue;
    const size_t lds = sweep_lds_bytes_t(sizeof(T), TX, TY, ANG, L, a.band, MOM);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)sweep_kernel<T, TX, TY, DD, ANG, PSI, L, MOM>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((sweep_kernel<T, TX, TY, DD, ANG, PSI, L, MOM>), dim3(grid), dim3(64 * a.band), lds, s, a);
    return hipGetLastError();
}

// Dispatch over scheme, source kind, angular-flux output and lane-group size for one tile shape.
// Angular-flux output uses 64-lane groups, except in source iteration with a dense kernel (per-
// ordinate sources in, BF16 / FP64 angular flux out), where a batch of small ordinate sets packs
// 16 or 32 lanes per system.
template <typename T, int TX, int TY>
hipError_t launch_sweep_tile(const SweepArgs& a, int grid, bool dd, bool ang, int psi, int L, int mom, hipStream_t s)
{
    if (mom == 4) {
        if (ang || psi) return hipErrorInvalidValue;
        if (L == 64) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 64, 4>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 64, 4>(a, grid, s);
        if (L == 32) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 32, 4>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 32, 4>(a, grid, s);
        if (L == 16) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 16, 4>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 16, 4>(a, grid, s);
        return hipErrorInvalidValue;
    }
    if (mom != 1) return hipErrorInvalidValue;
    if (ang || psi) {
        constexpr int PSIV = sizeof(T) == 8 ? 1 : 2;  // the iteration's angular-flux output
        if (ang && psi == PSIV && L != 64) {
            if (L == 32) return dd ? launch_sweep_t<T, TX, TY, true, true, PSIV, 32>(a, grid, s) : launch_sweep_t<T, TX, TY, false, true, PSIV, 32>(a, grid, s);
            if (L == 16) return dd ? launch_sweep_t<T, TX, TY, true, true, PSIV, 16>(a, grid, s) : launch_sweep_t<T, TX, TY, false, true, PSIV, 16>(a, grid, s);
            return hipErrorInvalidValue;
        }
        if (L != 64) return hipErrorInvalidValue;
        if (ang) {
            if (psi == 2) return dd ? launch_sweep_t<T, TX, TY, true, true, 2, 64>(a, grid, s) : launch_sweep_t<T, TX, TY, false, true, 2, 64>(a, grid, s);
            if (psi == 1) return dd ? launch_sweep_t<T, TX, TY, true, true, 1, 64>(a, grid, s) : launch_sweep_t<T, TX, TY, false, true, 1, 64>(a, grid, s);
            return dd ? launch_sweep_t<T, TX, TY, true, true, 0, 64>(a, grid, s) : launch_sweep_t<T, TX, TY, false, true, 0, 64>(a, grid, s);
        }
        return dd ? launch_sweep_t<T, TX, TY, true, false, 1, 64>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 1, 64>(a, grid, s);
    }
    if (L == 64) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 64>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 64>(a, grid, s);
    if (L == 32) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 32>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 32>(a, grid, s);
    if (L == 16) return dd ? launch_sweep_t<T, TX, TY, true, false, 0, 16>(a, grid, s) : launch_sweep_t<T, TX, TY, false, false, 0, 16>(a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace rom

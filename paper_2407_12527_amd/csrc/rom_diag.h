// rom_diag.h -- the row-lane ("diagonal") transport-sweep kernel of librom.
//
// The strip kernel puts ordinates on lanes and walks the cells of a strip one after another, so
// a problem with few ordinates per quadrant offers little parallelism and its sweep is as long as
// the chain of strip hand-offs.  Here lanes hold grid ROWS instead: lane r of an R-row block sweeps
// row r of the block, skewed one column behind lane r - 1, so at step t the lanes of a block work
// on the anti-diagonal of cells (t - r, r), which are independent under the upwind dependences of
// eq. (3.6) for one ordinate direction.  The y-face value a cell needs from the row below is the
// value lane r - 1 produced one step earlier: one DPP lane shift (row_shr:1 within 16-lane rows,
// wave_shr:1 across the wavefront), and the x-face value is the lane's own previous result.
//
//   lane = g * R + r        g: ordinate slot (64 / R of them), r: row in the block
//   each lane carries K ordinates of its slot (independent chains, for instruction-level
//   parallelism), so a wavefront covers NO = (64 / R) * K ordinates of one quadrant.
//
// A task is (system, quadrant, NO ordinates) over the whole grid; its row blocks are cut into
// bands of NB consecutive blocks, and a workgroup of NB wavefronts sweeps one band (wave w takes
// block band * NB + w).  Inside a band a block's top row goes to the block above through an LDS
// ring of RING columns (produced / consumed counters, back-pressure); the band's top row goes to
// the next band through a global edge buffer behind an epoch-tagged progress counter.  Waits are
// bounded and record an error instead of hanging.
//
// The field and source pools carry kPoolPad elements of padding on both sides, so the skewed
// loads of lanes before or past their row need no clamping.
//
// Dense scattering kernels (ANG): the source is per (cell, ordinate), stored in ordinate blocks
// of 16, S[npad / 16][cells][16], as the contraction writes it for this kernel.  The four slots
// of a row hold 4K consecutive ordinates of one block, so at each step they read 16K contiguous
// bytes of one cell (K floats per lane, the cell clamped into the grid for lanes outside their
// row), and a lane's consecutive steps read consecutive cells of its block: each row of the block
// is one stream through memory, not a stride of the whole ordinate set per cell.  The weighted
// angular flux w psi of the cell goes back in the same layout as BF16, the contraction's input.
//
// Cell update (step scheme, unscaled psi, cells in sweep order):
//   psi = (S + a psi_x + b psi_y) / (sigma_t + a + b),   a = |c|/dx, b = |s|/dy
// and the task's partial scalar flux sum_k w_k psi_k is reduced over the 64 / R ordinate slots
// for U steps at a time by a transposing permlane-swap sum (each lane ends up with U/4 of the
// totals) and stored once per cell.
#pragma once
#include <type_traits>

#include "rom_common.h"

namespace rom {

template <int R>
constexpr int diag_ring() { return R == 16 ? 64 : 128; }
// Steps per block: each block boundary costs the hand-off waits, exports and publication, so
// FP32 blocks are 16 steps long where the lane state still fits the VGPR budget (at most two
// ordinates per lane and two prefetch sets, i.e. at most 8 waves per workgroup, 256 VGPRs);
// otherwise 8.  FP64: 4.  (diag_pitch pads the y-face tables for 16.)
// Dense-kernel variants hold K source values per step in their prefetch sets: 8 steps, 4 with
// two or four ordinates per lane.
template <typename T, int K, int PD, bool ANG = false>
constexpr int diag_unroll() { return sizeof(T) == 8 ? 4 : ANG ? (K >= 2 ? 4 : 8) : (K <= 2 && PD == 2 ? 16 : 8); }
// Most wavefronts per workgroup: 16, or 8 where the lane state needs more than 128 VGPRs (more
// than one ordinate per lane, or loads kept PD = 2 blocks ahead).
template <typename T, int K, int PD>
constexpr int diag_max_waves() { return (PD > 1 || K > 1) ? 8 : kDiagMaxWaves; }

// lane r of each R-lane block takes lane r - 1's v; lane 0 of the block keeps `old`
template <int R>
__device__ __forceinline__ float shift_up(float old, float v)
{
    constexpr int CTRL = R == 16 ? 0x111 : 0x138;  // row_shr:1 | wave_shr:1
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int R>
__device__ __forceinline__ double shift_up(double old, double v)
{
    constexpr int CTRL = R == 16 ? 0x111 : 0x138;
    const int2 o = *reinterpret_cast<const int2*>(&old);
    const int2 x = *reinterpret_cast<const int2*>(&v);
    int2 y;
    y.x = __builtin_amdgcn_update_dpp(o.x, x.x, CTRL, 0xF, 0xF, false);
    y.y = __builtin_amdgcn_update_dpp(o.y, x.y, CTRL, 0xF, 0xF, false);
    return *reinterpret_cast<const double*>(&y);
}

// One stage of a transposing sum over lane halves D = 32 or 16: lanes without bit D get
// x(l) + x(l ^ D), lanes with bit D get y(l ^ D) + y(l) (the lower lane's value always first).
template <int D>
__device__ __forceinline__ float halve_swap(float x, float y)
{
    if constexpr (D == 32) {
        auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(p[0]) + __uint_as_float(p[1]);
    } else {
        auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
        return __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
}

template <int D>
__device__ __forceinline__ double halve_swap(double x, double y)
{
    const double xo = __shfl_xor(x, D, 64);
    const double yo = __shfl_xor(y, D, 64);
    return (threadIdx.x & D) ? yo + y : x + xo;
}

// Sum the U per-step partials over the four ordinate slots of an R = 16 wavefront.  Afterwards
// lane g*16 + r holds, in out[v], the total of step v + g*(U/4) for its row r.
template <typename T, int U>
__device__ __forceinline__ void slot_sums(const T (&acc)[U], T (&out)[U / 4])
{
    T h[U / 2];
#pragma unroll
    for (int v = 0; v < U / 2; ++v) h[v] = halve_swap<32>(acc[v], acc[v + U / 2]);
#pragma unroll
    for (int v = 0; v < U / 4; ++v) out[v] = halve_swap<16>(h[v], h[v + U / 4]);
}

// LDS hand-off counters between the wavefronts of a workgroup.  A wave's LDS operations complete
// in issue order and LDS is one coherent memory per CU, so publishing needs only the wave's own
// LDS traffic drained (s_waitcnt lgkmcnt(0)) -- not its global loads and stores, which a
// memory-model release at workgroup scope would also wait for.  The counters are accessed through
// LDS-typed pointers: a volatile access through a generic pointer stays a FLAT access (address
// spaces are not inferred for volatile accesses), and every FLAT load is followed by a wait on
// the vector-memory counter as well, which drained the wave's prefetched field and source loads
// and its stores at every poll.
typedef __attribute__((address_space(3))) int lds_int_t;

__device__ __forceinline__ void lds_publish(int* p, int v)
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    *(volatile lds_int_t*)p = v;
}

// Bounded wait on an LDS counter; returns the value seen (cached by the caller).  Reads that
// follow stay after the poll (compiler barrier; LDS answers a wave's reads in order).  Bounds as
// wait_gave_up states; a wait that gave up returns the target.
__device__ __forceinline__ int lds_wait_get(int* p, int target, Ctl* ctl, int limit, long long ticks)
{
    int v = *(volatile lds_int_t*)p;
    if (v < target) {
        const unsigned long long t0 = wall_clock64();
        int spins = 0;
        while ((v = *(volatile lds_int_t*)p) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wait_gave_up(++spins, t0, ctl, limit, ticks)) {
                v = target;
                break;
            }
        }
    }
    asm volatile("" ::: "memory");
    return v;
}

// Bounded wait on a device-scope progress counter (another workgroup's band); returns the value
// seen.  The counter carries the sweep's epoch in its high bits.
__device__ __forceinline__ long long wait_progress_get(long long* p, long long target, Ctl* ctl, int limit, long long ticks)
{
    long long v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v < target) {
        const unsigned long long t0 = wall_clock64();
        int spins = 0;
        while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wait_gave_up(++spins, t0, ctl, limit, ticks)) return target;
        }
    }
    asm volatile("" ::: "memory");  // edge loads stay after the poll
    return v;
}

// Everything one (task, band) needs, read once per workgroup (uniform values).
template <typename T>
struct DiagTask {
    int nx, ny, nblocks, pitch;
    bool ypos;
    const T* st;         // sigma_t of the problem (pool padded by kPoolPad elements on both sides)
    const T* S;          // isotropic source of the system (same padding)
    T* part;             // partial-flux slot
    const T* inflow;
    int64_t xin, yin;    // inflow tables, -1 for vacuum
    const T* edge_in;    // top row of the band below [NO][pitch] (global), its progress counter
    long long* prog_in;
    T* edge_out;         // this band's top row for the band above, and its progress counter
    long long* prog_out;
    long long tag;       // sweep epoch << 24
    const float* ang;    // dense kernels: per-ordinate source of the system [npad / 16][cells][16],
    uint16_t* psi;       // its weighted angular flux (BF16 bits) in the same layout
    int64_t cells;
    int ord0;            // the task's first ordinate
};

// Two floats as packed BF16 (low half x), rounded to nearest even: one v_cvt_pk_bf16_f32 on gfx950.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack(float x, float y)
{
    bf16x2_t v;
    v.x = (__bf16)x;
    v.y = (__bf16)y;
    return __builtin_bit_cast(uint32_t, v);
}

// U consecutive values at p (16-byte aligned) as 16-byte LDS or global accesses.
template <typename T, int U>
__device__ __forceinline__ void load_run(const T* p, T (&v)[U])
{
    constexpr int W = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
    for (int q = 0; q < U / W; ++q) {
        const V x = reinterpret_cast<const V*>(p)[q];
        const T* e = reinterpret_cast<const T*>(&x);
#pragma unroll
        for (int m = 0; m < W; ++m) v[q * W + m] = e[m];
    }
}

template <typename T, int U>
__device__ __forceinline__ void store_run(T* p, const T (&v)[U])
{
    constexpr int W = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
    for (int q = 0; q < U / W; ++q) {
        V x;
        T* e = reinterpret_cast<T*>(&x);
#pragma unroll
        for (int m = 0; m < W; ++m) e[m] = v[q * W + m];
        reinterpret_cast<V*>(p)[q] = x;
    }
}

// A run of N cells of one lane's row starting at storage index c0 and moving by DIR per step, as
// 16-byte vector accesses that need only element alignment (the runs of a wave's lanes are skewed
// by one cell per row, so they are not 16-byte aligned; gfx950 global memory accepts unaligned
// vector accesses): one instruction per 16 bytes instead of one per cell.  DIR = -1 covers
// [c0 - N + 1, c0] and reverses the order.  Runs shorter than a vector fall back to single cells.
template <typename T, int N, int DIR>
__device__ __forceinline__ void load_row_run(const T* base, int64_t c0, T (&v)[N])
{
    constexpr int W = 16 / sizeof(T);
    if constexpr (N % W == 0) {
        typedef T VU __attribute__((ext_vector_type(W), aligned(sizeof(T))));
        const T* p = base + (DIR > 0 ? c0 : c0 - (N - 1));
#pragma unroll
        for (int q = 0; q < N / W; ++q) {
            const VU x = *reinterpret_cast<const VU*>(p + q * W);
#pragma unroll
            for (int m = 0; m < W; ++m) v[DIR > 0 ? q * W + m : N - 1 - (q * W + m)] = x[m];
        }
    } else {
#pragma unroll
        for (int u = 0; u < N; ++u) v[u] = base[c0 + DIR * u];
    }
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void store_row_run(T* base, int64_t c0, const T (&v)[N])
{
    constexpr int W = 16 / sizeof(T);
    if constexpr (N % W == 0) {
        typedef T VU __attribute__((ext_vector_type(W), aligned(sizeof(T))));
        T* p = base + (DIR > 0 ? c0 : c0 - (N - 1));
#pragma unroll
        for (int q = 0; q < N / W; ++q) {
            VU x;
#pragma unroll
            for (int m = 0; m < W; ++m) x[m] = v[DIR > 0 ? q * W + m : N - 1 - (q * W + m)];
            *reinterpret_cast<VU*>(p + q * W) = x;
        }
    } else {
#pragma unroll
        for (int u = 0; u < N; ++u) base[c0 + DIR * u] = v[u];
    }
}

// Device-coherent runs for the band edges (8-byte relaxed agent-scope accesses: the producer and
// the consumer band may sit on different XCDs).
template <typename T, int U>
__device__ __forceinline__ void load_run_agent(const T* p, T (&v)[U])
{
    constexpr int W = 8 / sizeof(T);
#pragma unroll
    for (int q = 0; q < U / W; ++q) {
        const unsigned long long x =
            __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p) + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const T* e = reinterpret_cast<const T*>(&x);
#pragma unroll
        for (int m = 0; m < W; ++m) v[q * W + m] = e[m];
    }
}

template <typename T, int U>
__device__ __forceinline__ void store_run_agent(T* p, const T (&v)[U])
{
    constexpr int W = 8 / sizeof(T);
#pragma unroll
    for (int q = 0; q < U / W; ++q) {
        unsigned long long x;
        T* e = reinterpret_cast<T*>(&x);
#pragma unroll
        for (int m = 0; m < W; ++m) e[m] = v[q * W + m];
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(p) + q, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Where a block's top row goes (nowhere: top block of the grid; the LDS ring of the next wave;
// the band's global edge) and where its bottom row's y-face inflow comes from (the LDS ring of the
// previous wave; the boundary inflow table; the global edge of the band below).  Both are template
// parameters so a wave that only talks to LDS never waits on its global loads and stores.
enum { kOutNone = 0, kOutRing = 1, kOutEdge = 2 };
enum { kInRing = 0, kInBoundary = 1, kInEdge = 2 };

// One R-row block (row block rb, wavefront `wave` of an NB-wave band) of one task.
//
// Hand-off layout: rings are [NO][RING] and edges [NO][pitch] (columns contiguous per ordinate),
// so a block of U steps reads its U input columns and writes its U output columns as runs.  The
// top row of column c leaves the lane of row R - 1 at step c + R - 1; block t0 exports columns
// t0 - R .. t0 - R + U - 1 (the previous block's last value and this block's first U - 1), so
// every run is U-aligned.
template <typename T, int R, int K, int PD, bool XPOS, int IN, int OUT, bool ANG>
__device__ __forceinline__ void diag_block(const DiagArgs& A, const DiagTask<T>& D, const int rb, const int wave,
                                           T* ring, int* prod, int* cons,
                                           const T (&a)[K], const T (&b)[K], const T (&ab)[K], const T (&w)[K])
{
    constexpr int NG = kWave / R;
    constexpr int NO = NG * K;
    constexpr int U = diag_unroll<T, K, PD, ANG>();
    constexpr int RING = diag_ring<R>();
    constexpr int DIR = XPOS ? 1 : -1;  // storage step per sweep column
    static_assert(RING % U == 0 && R % U == 0, "runs must stay aligned");
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / R, r = lane % R;
    const int nx = D.nx, ny = D.ny;

    const int jj = rb * R + r;               // sweep-order row of this lane
    const bool row_ok = jj < ny;
    const int jc = min(jj, ny - 1);
    const int j = D.ypos ? jc : ny - 1 - jc;
    // storage index of this lane's cell at step t is lane0 + DIR * t
    const int64_t lane0 = (int64_t)j * nx + (XPOS ? -r : nx - 1 + r);
    constexpr bool in_bc = IN == kInBoundary;
    constexpr bool in_glob = IN == kInEdge;
    const T* in_ring = ring + (size_t)(wave > 0 ? wave - 1 : 0) * RING * NO;
    T* out_ring = ring + (size_t)wave * RING * NO;
    long long seen_in = 0;
    int seen_out = 0;

    T psi[K], last[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        psi[k] = (D.xin >= 0 && row_ok) ? D.inflow[D.xin + (int64_t)jc * NO + g * K + k] : T(0);
        last[k] = T(0);
    }

    // cells of steps t0 .. t0 + U - 1; lanes before or past their row read padding or a
    // neighbouring row, values that never reach a stored or exported result.  PD register sets
    // keep the loads PD blocks ahead of their use.
    constexpr int UA = ANG ? U : 1;
    constexpr int KA = ANG ? K : 1;
    typedef float VK __attribute__((ext_vector_type(KA)));
    T pst[PD][U], pS[PD][ANG ? 1 : U];
    VK pA[PD][UA];
    // storage cell of step t, clamped into the lane's row (dense-kernel loads)
    const int64_t rowbase = (int64_t)j * nx;
    // the lane's K ordinates within their block of 16: element (cell, o) at ((o / 16) * cells + cell) * 16 + o % 16
    const int ol = D.ord0 + g * K;
    const int64_t obase = ANG ? ((int64_t)(ol / 16) * D.cells) * 16 + ol % 16 : 0;
    const float* const ang_lane = ANG ? D.ang + obase : nullptr;
    auto fetch = [&](T (&fst)[U], T (&fS)[ANG ? 1 : U], VK (&fA)[UA], int t0) {
        const int64_t c0 = lane0 + (int64_t)DIR * t0;
        load_row_run<T, U, DIR>(D.st, c0, fst);
        if constexpr (ANG) {
            if (t0 >= R && t0 + U <= nx) {
                // every lane's cells of these steps lie inside its row: one address, the steps at
                // fixed offsets from it
                const float* const p = ang_lane + (rowbase + (XPOS ? t0 - r : nx - 1 - t0 + r)) * 16;
#pragma unroll
                for (int u = 0; u < U; ++u) fA[u] = *reinterpret_cast<const VK*>(p + DIR * u * 16);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = min(max(t0 + u - r, 0), nx - 1);
                    const int64_t cell = rowbase + (XPOS ? c : nx - 1 - c);
                    fA[u] = *reinterpret_cast<const VK*>(ang_lane + cell * 16);
                }
            }
        } else {
            load_row_run<T, U, DIR>(D.S, c0, fS);
        }
    };
    const int tsteps = nx + R - 1;                          // steps with a cell in the block
    const int tlast = (tsteps - 1) / U * U;                 // the last run with a cell
    const int tend = R + U * ((nx + U - 1) / U);            // ... and until the last column is exported
#pragma unroll
    for (int q = 0; q < PD; ++q)
        if (q * U < tsteps) fetch(pst[q], pS[q], pA[q], q * U);

    auto block = [&](const int t0, const T (&cst)[U], const T (&cS)[ANG ? 1 : U], const VK (&cA)[UA]) {
        // y-face inflow of row 0 for columns t0 .. t0 + U - 1 (only row 0 uses it, and only for
        // columns < nx; the runs reach into the tables' padding past the row end)
        T in[K][U];
        const int cin_hi = min(t0 + U, nx);
        if (t0 < nx) {
            if constexpr (in_bc) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (D.yin >= 0) load_run<T, U>(D.inflow + D.yin + (int64_t)(g * K + k) * D.pitch + t0, in[k]);
                    else {
#pragma unroll
                        for (int u = 0; u < U; ++u) in[k][u] = T(0);
                    }
                }
            } else if constexpr (in_glob) {
                if (seen_in < (D.tag | cin_hi)) seen_in = wait_progress_get(D.prog_in, D.tag | cin_hi, A.ctl, A.spin_limit, A.wait_ticks);
#pragma unroll
                for (int k = 0; k < K; ++k) load_run_agent<T, U>(D.edge_in + (int64_t)(g * K + k) * D.pitch + t0, in[k]);
            } else {
                if (seen_in < cin_hi) seen_in = lds_wait_get(&prod[wave - 1], cin_hi, A.ctl, A.spin_limit, A.wait_ticks);
#pragma unroll
                for (int k = 0; k < K; ++k) load_run<T, U>(in_ring + (g * K + k) * RING + (t0 & (RING - 1)), in[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int u = 0; u < U; ++u) in[k][u] = T(0);
        }
        // room in the ring for this block's run of top-row columns
        const int c_out = t0 - R;  // first exported column
        if (OUT == kOutRing && c_out + U > 0) {
            const int need = c_out + U - RING;
            if (need > 0 && seen_out < need) seen_out = lds_wait_get(&cons[wave], need, A.ctl, A.spin_limit, A.wait_ticks);
        }

        uint16_t* const psi_blk = ANG ? D.psi + obase + (rowbase + (XPOS ? t0 - r : nx - 1 - t0 + r)) * 16 : nullptr;
        // MODE 0: every lane inside its row; 1: lanes before their row start hold their x-face
        // inflow; 2: lanes outside their row store nothing
        T acc[U];
        T hist[K][U];
        auto step = [&](const int u, auto mode) {
            constexpr int MODE = decltype(mode)::value;
            const int c = t0 + u - r;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T dn = shift_up<R>(in[k][u], psi[k]);
                T src;
                if constexpr (ANG) src = (T)cA[u][k];
                else src = cS[u];
                const T num = fma(b[k], dn, fma(a[k], psi[k], src));
                const T v = num * rcp_fast(cst[u] + ab[k]);
                if (MODE == 1) psi[k] = c >= 0 ? v : psi[k];
                else psi[k] = v;
                hist[k][u] = psi[k];
                acc[u] = k == 0 ? w[k] * v : fma(w[k], v, acc[u]);
            }
            // dense kernels: the cell's weighted angular flux, K BF16 values per lane (inside the
            // rows, MODE 0, at fixed offsets from the block's address)
            if constexpr (ANG) {
                if (row_ok && (MODE == 0 || (c >= 0 && c < nx))) {
                    uint16_t* const po = MODE == 0 ? psi_blk + DIR * u * 16
                                                   : D.psi + obase + (rowbase + (XPOS ? c : nx - 1 - c)) * 16;
                    if constexpr (K == 1) {
                        *po = __builtin_bit_cast(uint16_t, (__bf16)(w[0] * psi[0]));
                    } else {
                        uint32_t pk[K / 2];
#pragma unroll
                        for (int k = 0; k < K; k += 2) pk[k / 2] = bf16_pack(w[k] * psi[k], w[k + 1] * psi[k + 1]);
                        if constexpr (K == 2) *reinterpret_cast<uint32_t*>(po) = pk[0];
                        else *reinterpret_cast<uint2*>(po) = make_uint2(pk[0], pk[1]);
                    }
                }
            }
        };
        const int mode = t0 < R ? 1 : (t0 + U <= nx ? 0 : 2);
        if (mode == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) step(u, std::integral_constant<int, 0>{});
        } else if (mode == 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) step(u, std::integral_constant<int, 1>{});
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) step(u, std::integral_constant<int, 2>{});
        }

        // export columns c_out .. c_out + U - 1 from the top row
        if (OUT != kOutNone && r == R - 1 && c_out + U > 0 && c_out < nx) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                T run[U];
                run[0] = last[k];
#pragma unroll
                for (int u = 1; u < U; ++u) run[u] = hist[k][u - 1];
                if (c_out >= 0 && c_out + U <= nx) {
                    if (OUT == kOutRing) store_run<T, U>(out_ring + (g * K + k) * RING + (c_out & (RING - 1)), run);
                    else store_run_agent<T, U>(D.edge_out + (int64_t)(g * K + k) * D.pitch + c_out, run);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = c_out + u;
                        if (c >= 0 && c < nx) {
                            if (OUT == kOutRing) out_ring[(g * K + k) * RING + (c & (RING - 1))] = run[u];
                            else edge_store(D.edge_out + (int64_t)(g * K + k) * D.pitch + c, run[u]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) last[k] = hist[k][U - 1];

        // partial scalar flux of the block's cells
        T* const pblk = D.part + lane0 + (int64_t)DIR * t0;
        if constexpr (NG == 4) {
            T tot[U / 4];
            slot_sums<T, U>(acc, tot);
            if (mode == 0) {
                if (row_ok) store_row_run<T, U / 4, DIR>(D.part, lane0 + (int64_t)DIR * (t0 + g * (U / 4)), tot);
            } else {
#pragma unroll
                for (int v = 0; v < U / 4; ++v) {
                    const int u = v + g * (U / 4);
                    const int c = t0 + u - r;
                    if (row_ok && c >= 0 && c < nx) pblk[DIR * u] = tot[v];
                }
            }
        } else {
            if (mode == 0) {
                if (row_ok) store_row_run<T, U, DIR>(D.part, lane0 + (int64_t)DIR * t0, acc);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = t0 + u - r;
                    if (row_ok && c >= 0 && c < nx) pblk[DIR * u] = acc[u];
                }
            }
        }

        const int done = min(max(c_out + U, 0), nx);   // top-row columns exported so far
        // The band's top edge is published every EB blocks (16 steps) and at its last column:
        // publishing waits for every memory operation of the wave to complete (the edge words
        // must have landed), prefetched loads included, so doing it every block of a short
        // block paced the whole band above by one memory round trip per block.
        constexpr int EB = U >= 16 ? 1 : 16 / U;
        const bool publish = OUT == kOutEdge && (((t0 / U) % EB) == EB - 1 || done >= nx);
        if (publish) stores_complete();                 // the edge words have landed before publishing
        if (lane == 0) {
            if (!in_bc && !in_glob && t0 < nx)
                lds_publish(&cons[wave - 1], cin_hi);
            if (publish)
                __hip_atomic_store(D.prog_out, D.tag | done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else if (OUT == kOutRing)
                lds_publish(&prod[wave], done);
        }
    };

    for (int t0 = 0; t0 < tend; t0 += PD * U) {
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            const int tq = t0 + q * U;
            if (q == 0 || tq < tend) {
                T cst[U], cS[ANG ? 1 : U];
                VK cA[UA];
#pragma unroll
                for (int u = 0; u < U; ++u) cst[u] = pst[q][u];
                if constexpr (ANG) {
#pragma unroll
                    for (int u = 0; u < U; ++u) cA[u] = pA[q][u];
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) cS[u] = pS[q][u];
                }
                // Refill unconditionally (past the last run, the last run again): with the same
                // loads on every path the new values take the registers of the ones just copied
                // out, instead of being moved at the loop latch, a move that must first wait for
                // every load and store in flight.
                fetch(pst[q], pS[q], pA[q], min(tq + PD * U, tlast));
                block(tq, cst, cS, cA);
            }
        }
    }
}

template <typename T, int R, int K, int PD, bool XPOS, bool ANG>
__device__ __forceinline__ void diag_block_any(const DiagArgs& A, const DiagTask<T>& D, const int rb, const int wave, const int NB,
                                               T* ring, int* prod, int* cons,
                                               const T (&a)[K], const T (&b)[K], const T (&ab)[K], const T (&w)[K])
{
    const int out = rb + 1 >= D.nblocks ? kOutNone : (wave == NB - 1 ? kOutEdge : kOutRing);
    if (rb == 0) {
        if (out == kOutNone) diag_block<T, R, K, PD, XPOS, kInBoundary, kOutNone, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else if (out == kOutEdge) diag_block<T, R, K, PD, XPOS, kInBoundary, kOutEdge, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else diag_block<T, R, K, PD, XPOS, kInBoundary, kOutRing, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
    } else if (wave == 0) {
        if (out == kOutNone) diag_block<T, R, K, PD, XPOS, kInEdge, kOutNone, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else if (out == kOutEdge) diag_block<T, R, K, PD, XPOS, kInEdge, kOutEdge, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else diag_block<T, R, K, PD, XPOS, kInEdge, kOutRing, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
    } else {
        if (out == kOutNone) diag_block<T, R, K, PD, XPOS, kInRing, kOutNone, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else if (out == kOutEdge) diag_block<T, R, K, PD, XPOS, kInRing, kOutEdge, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
        else diag_block<T, R, K, PD, XPOS, kInRing, kOutRing, ANG>(A, D, rb, wave, ring, prod, cons, a, b, ab, w);
    }
}

// Persistent workgroups take (task, band) tickets in band-major order, so the band below a
// ticket's band always holds an earlier ticket: every wait is on a workgroup that is running or
// done.
template <typename T, int R, int K, int PD, bool ANG>
__global__ __launch_bounds__((64 * diag_max_waves<T, K, PD>())) void diag_kernel(DiagArgs A)
{
    static_assert(!ANG || sizeof(T) == 4, "dense-kernel row-lane sweeps are FP32 (BF16 angular flux)");
    constexpr int NG = kWave / R;
    constexpr int NO = NG * K;
    constexpr int RING = diag_ring<R>();
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int NB = blockDim.x >> 6;
    const int g = lane / R;

    extern __shared__ __align__(16) unsigned char smem[];
    T* const ring = (T*)smem;                                        // [NB - 1][NO][RING]
    int* const prod = (int*)(ring + (size_t)(NB - 1) * RING * NO);   // [kDiagMaxWaves]
    int* const cons = prod + kDiagMaxWaves;
    int& s_ticket = cons[kDiagMaxWaves];

    if (!A.mode_all && A.ctl->active == 0) return;   // every system has stopped
    const long long tag = (long long)uniform(A.ctl->epoch) << 24;
    for (;;) {
        if (threadIdx.x == 0) {
            s_ticket = atomicAdd(&A.ctl->ticket, 1);
            sweep_clock(A.ctl, s_ticket, A.ntickets);
        }
        if (lane == 0) {
            prod[wave] = 0;
            cons[wave] = 0;
        }
        __syncthreads();
        const int t = s_ticket;
        if (t >= A.ntickets) break;  // uniform over the workgroup
        const int2 tk = A.tickets[t];
        const DiagTaskDev& TK = A.tasks[uniform(tk.x)];
        const int band = uniform(tk.y);
        const int sys = uniform(TK.sys);
        if (A.mode_all || uniform(A.sysctl[sys].state) == 0) {
            const int prob = uniform(TK.prob), quad = uniform(TK.quad), slot = uniform(TK.slot);
            const int64_t ord_off = uniform64(TK.ord_off);
            const ProblemDev& PB = A.probs[prob];
            DiagTask<T> D;
            D.nx = uniform(PB.nx);
            D.ny = uniform(PB.ny);
            D.pitch = diag_pitch(D.nx);
            D.nblocks = (D.ny + R - 1) / R;
            D.ypos = quad < 2;
            D.st = (const T*)A.sigma_t + uniform64(PB.field_off);
            D.S = (const T*)A.src + uniform64(A.sys[sys].src_off);
            D.part = (T*)A.part + A.slot_off[slot];
            D.inflow = (const T*)A.inflow;
            D.xin = uniform64(TK.xin_off);
            D.yin = uniform64(TK.yin_off);
            const int64_t eoff = uniform64(TK.edge_off), edge_len = (int64_t)D.pitch * NO;
            const int poff = uniform(TK.prog_off);
            D.edge_in = (const T*)A.edge + eoff + (int64_t)(band - 1) * edge_len;
            D.prog_in = A.prog + poff + band - 1;
            D.edge_out = (T*)A.edge + eoff + (int64_t)band * edge_len;
            D.prog_out = A.prog + poff + band;
            D.tag = tag;
            if constexpr (ANG) {
                const SystemDev& SD = A.sys[sys];
                D.cells = (int64_t)D.nx * D.ny;
                D.ang = (const float*)A.ang_src + uniform64(SD.ang_off);
                D.psi = (uint16_t*)A.psi_out + uniform64(SD.ang_off);
                D.ord0 = uniform(A.ords[ord_off].ord);
            }
            const int rb = band * NB + wave;
            if (rb < D.nblocks) {
                T a[K], b[K], ab[K], w[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const LaneDev& o = A.ords[ord_off + g * K + k];
                    a[k] = to_T<T>(o.a);
                    b[k] = to_T<T>(o.b);
                    ab[k] = a[k] + b[k];
                    w[k] = to_T<T>(o.w);
                }
                if (quad == 0 || quad == 3) diag_block_any<T, R, K, PD, true, ANG>(A, D, rb, wave, NB, ring, prod, cons, a, b, ab, w);
                else diag_block_any<T, R, K, PD, false, ANG>(A, D, rb, wave, NB, ring, prod, cons, a, b, ab, w);
            }
        }
        __syncthreads();  // the band is done before its LDS is reused
    }
}

template <typename T, int R, int K, int PD, bool ANG = false>
hipError_t launch_diag_t(const DiagArgs& a, int grid, int nb, hipStream_t s)
{
    constexpr int NO = (kWave / R) * K;
    if (nb < 1 || nb > diag_max_waves<T, K, PD>() || grid < 1) return hipErrorInvalidValue;
    const size_t lds = sizeof(T) * (size_t)(nb - 1) * diag_ring<R>() * NO + sizeof(int) * (2 * kDiagMaxWaves + 1);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)diag_kernel<T, R, K, PD, ANG>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((diag_kernel<T, R, K, PD, ANG>), dim3(grid), dim3(64 * nb), lds, s, a);
    return hipGetLastError();
}

}  // namespace rom

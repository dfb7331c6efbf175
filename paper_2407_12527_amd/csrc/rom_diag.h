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
// A workgroup of NB wavefronts owns one task (system, quadrant, NO ordinates) and the whole grid:
// wave w takes row blocks w, w + NB, w + 2 NB, ...  A block's top row goes to the block above
// through LDS: a ring of RING columns between waves w and w + 1 of the same round (with
// back-pressure), and a whole-row buffer from the last wave to wave 0 of the next round (no
// back-pressure is needed there: the next round's writer depends on the reader through the chain
// of blocks between them).  Waits are bounded and record an error instead of hanging.
//
// The field and source pools carry kPoolPad elements of padding on both sides, so the skewed
// loads of lanes before or past their row need no clamping.
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
template <typename T>
constexpr int diag_unroll() { return sizeof(T) == 8 ? 4 : 8; }
// most wavefronts per workgroup: 16, or 8 where the lane state needs more than 128 VGPRs
template <typename T, int K>
constexpr int diag_max_waves() { return (K * sizeof(T) >= 16) ? 8 : kDiagMaxWaves; }

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

// Bounded wait on an LDS counter; returns the value seen (cached by the caller).
__device__ __forceinline__ int lds_wait_get(int* p, int target, Ctl* ctl, int limit)
{
    int spins = 0;
    int v;
    while ((v = __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins >= limit) {
            __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return target;
        }
        if ((spins & 1023) == 0 &&
            __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return target;
    }
    return v;
}

// Everything one task needs, read once per workgroup (uniform values).
template <typename T>
struct DiagTask {
    int nx, ny, nblocks;
    bool ypos;
    const T* st;       // sigma_t of the problem (pool padded by kPoolPad elements on both sides)
    const T* S;        // isotropic source of the system (same padding)
    T* part;           // partial-flux slot
    const T* inflow;
    int64_t xin, yin;  // inflow tables, -1 for vacuum
};

template <typename T, int R, int K, bool XPOS>
__device__ __forceinline__ void diag_sweep(const DiagArgs& A, const DiagTask<T>& D, T* ring, T* wrap, T* scratch, int* prod, int* cons,
                                           const T (&a)[K], const T (&b)[K], const T (&ab)[K], const T (&w)[K])
{
    constexpr int NG = kWave / R;
    constexpr int NO = NG * K;
    constexpr int U = diag_unroll<T>();
    constexpr int RING = diag_ring<R>();
    constexpr int DIR = XPOS ? 1 : -1;  // storage step per sweep column
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int NB = blockDim.x >> 6;
    const int g = lane / R, r = lane % R;
    const int nx = D.nx, ny = D.ny;

    for (int rb = wave; rb < D.nblocks; rb += NB) {
        const int round = rb / NB;
        const int jj = rb * R + r;               // sweep-order row of this lane
        const bool row_ok = jj < ny;
        const int jc = min(jj, ny - 1);
        const int j = D.ypos ? jc : ny - 1 - jc;
        // storage index of this lane's cell at step t is lane0 + DIR * t
        const int64_t lane0 = (int64_t)j * nx + (XPOS ? -r : nx - 1 + r);
        const bool has_out = rb + 1 < D.nblocks;   // only the last block may be partial
        const bool in_bc = rb == 0;
        const bool in_wrap = !in_bc && wave == 0;
        const T* in_buf = in_wrap ? wrap : ring + (size_t)(wave > 0 ? wave - 1 : 0) * RING * NO;
        int* in_cnt = in_wrap ? &prod[NB - 1] : &prod[wave > 0 ? wave - 1 : 0];
        const int in_base = in_wrap ? (round - 1) * nx : round * nx;
        const unsigned in_mask = in_wrap ? 0x7fffffffu : (unsigned)(RING - 1);
        const int in_off = in_wrap ? 0 : in_base;
        const bool out_wrap = wave == NB - 1;
        T* out_buf = out_wrap ? wrap : ring + (size_t)wave * RING * NO;
        const int out_base = round * nx;
        const unsigned out_mask = out_wrap ? 0x7fffffffu : (unsigned)(RING - 1);
        const int out_off = out_wrap ? 0 : out_base;
        int seen_in = 0, seen_out = 0;
        // Interior steps export without exec-mask changes: the exporting lanes (row R - 1 of a
        // block that has a block above) address the ring, every other lane a scratch slot.
        const bool exp_lane = has_out && r == R - 1;
        const unsigned exp_stride = exp_lane ? (unsigned)(NO * sizeof(T)) : 0u;
        const unsigned exp_base = exp_lane ? (unsigned)((const char*)(out_buf + g * K) - (const char*)ring)
                                           : (unsigned)((const char*)(scratch + lane * K) - (const char*)ring);

        T psi[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            psi[k] = (D.xin >= 0 && row_ok) ? D.inflow[D.xin + (int64_t)jc * NO + g * K + k] : T(0);

        T pst[U], pS[U];
        // cells of steps t0 .. t0 + U - 1; lanes before or past their row read padding or a
        // neighbouring row, values that never reach a stored or exported result
        auto fetch = [&](int t0) {
            const int64_t c0 = lane0 + (int64_t)DIR * t0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                pst[u] = D.st[c0 + DIR * u];
                pS[u] = D.S[c0 + DIR * u];
            }
        };
        const int tsteps = nx + R - 1;
        fetch(0);
        for (int t0 = 0; t0 < tsteps; t0 += U) {
            T cst[U], cS[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cst[u] = pst[u];
                cS[u] = pS[u];
            }
            if (t0 + U < tsteps) fetch(t0 + U);

            // y-face inflow of row 0 for columns t0 .. t0 + U - 1 (used by row 0 only, and only
            // for columns < nx; later reads are clamped to a valid entry)
            T in[U][K];
            const int cin_hi = min(t0 + U, nx);
            if (in_bc) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = min(t0 + u, nx - 1);
#pragma unroll
                    for (int k = 0; k < K; ++k) in[u][k] = D.yin >= 0 ? D.inflow[D.yin + (int64_t)c * NO + g * K + k] : T(0);
                }
            } else {
                if (t0 < nx && seen_in < in_base + cin_hi) seen_in = lds_wait_get(in_cnt, in_base + cin_hi, A.ctl, A.spin_limit);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = min(t0 + u, nx - 1);
                    const int pos = (int)((unsigned)(in_off + c) & in_mask);
#pragma unroll
                    for (int k = 0; k < K; ++k) in[u][k] = in_buf[pos * NO + g * K + k];
                }
            }
            // room in the ring for the top-row columns of this block of steps
            const int cout_hi = min(t0 + U - R, nx - 1);
            if (has_out && !out_wrap && cout_hi >= 0) {
                const int need = out_base + cout_hi + 1 - RING;
                if (need > 0 && seen_out < need) seen_out = lds_wait_get(&cons[wave], need, A.ctl, A.spin_limit);
            }

            // MODE 0: every lane inside its row; 1: lanes before their row start hold their
            // x-face inflow; 2: lanes outside their row store nothing
            T acc[U];
            auto step = [&](const int u, auto mode) {
                constexpr int MODE = decltype(mode)::value;
                const int c = t0 + u - r;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const T dn = shift_up<R>(in[u][k], psi[k]);
                    const T num = fma(b[k], dn, fma(a[k], psi[k], cS[u]));
                    const T v = num * rcp_fast(cst[u] + ab[k]);
                    if (MODE == 1) psi[k] = c >= 0 ? v : psi[k];
                    else psi[k] = v;
                    acc[u] = k == 0 ? w[k] * v : fma(w[k], v, acc[u]);
                }
                // the exporting lanes (row R - 1) share one column: a uniform position
                const int cx = t0 + u - (R - 1);
                const unsigned pos = (unsigned)(out_off + cx) & out_mask;
                if constexpr (MODE == 0) {
                    T* const p = (T*)((char*)ring + (__umul24(pos, exp_stride) + exp_base));
#pragma unroll
                    for (int k = 0; k < K; ++k) p[k] = psi[k];
                } else if (has_out && cx >= 0 && cx < nx && r == R - 1) {
#pragma unroll
                    for (int k = 0; k < K; ++k) out_buf[pos * NO + g * K + k] = psi[k];
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
            // partial scalar flux of the block's cells
            T* const pblk = D.part + lane0 + (int64_t)DIR * t0;
            if constexpr (NG == 4) {
                T tot[U / 4];
                slot_sums<T, U>(acc, tot);
#pragma unroll
                for (int v = 0; v < U / 4; ++v) {
                    const int u = v + g * (U / 4);
                    const int c = t0 + u - r;
                    if (row_ok && (mode == 0 || (c >= 0 && c < nx))) pblk[DIR * u] = tot[v];
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = t0 + u - r;
                    if (row_ok && (mode == 0 || (c >= 0 && c < nx))) pblk[DIR * u] = acc[u];
                }
            }

            if (lane == 0) {
                if (!in_bc && !in_wrap && t0 < nx)
                    __hip_atomic_store(&cons[wave - 1], in_base + cin_hi, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (has_out) {
                    const int done = min(max(t0 + U - R + 1, 0), nx);
                    __hip_atomic_store(&prod[wave], out_base + done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
    }
}

template <typename T, int R, int K>
__global__ __launch_bounds__((64 * diag_max_waves<T, K>())) void diag_kernel(DiagArgs A)
{
    constexpr int NG = kWave / R;
    constexpr int NO = NG * K;
    constexpr int RING = diag_ring<R>();
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int NB = blockDim.x >> 6;
    const int g = lane / R;

    extern __shared__ __align__(16) unsigned char smem[];
    T* const ring = (T*)smem;                                        // [NB - 1][RING][NO]
    T* const wrap = ring + (size_t)(NB - 1) * RING * NO;            // [wrap_cols][NO]
    T* const scratch = wrap + (size_t)A.wrap_cols * NO;              // [64][K], write-only
    int* const prod = (int*)(scratch + kWave * K);                   // [kDiagMaxWaves]
    int* const cons = prod + kDiagMaxWaves;

    const DiagTaskDev& TK = A.tasks[blockIdx.x];
    const int sys = uniform(TK.sys);
    if (!A.mode_all && uniform(A.sysctl[sys].state) != 0) return;   // uniform over the workgroup
    if (threadIdx.x == 0) atomicMin(&A.ctl->t_first, (unsigned long long)wall_clock64());
    if (lane == 0) {
        prod[wave] = 0;
        cons[wave] = 0;
    }
    __syncthreads();

    const int prob = uniform(TK.prob), quad = uniform(TK.quad), slot = uniform(TK.slot);
    const int64_t ord_off = uniform64(TK.ord_off);
    const ProblemDev& PD = A.probs[prob];
    DiagTask<T> D;
    D.nx = uniform(PD.nx);
    D.ny = uniform(PD.ny);
    D.nblocks = (D.ny + R - 1) / R;
    D.ypos = quad < 2;
    D.st = (const T*)A.sigma_t + uniform64(PD.field_off);
    D.S = (const T*)A.src + uniform64(A.sys[sys].src_off);
    D.part = (T*)A.part + A.slot_off[slot];
    D.inflow = (const T*)A.inflow;
    D.xin = uniform64(TK.xin_off);
    D.yin = uniform64(TK.yin_off);

    T a[K], b[K], ab[K], w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const LaneDev& o = A.ords[ord_off + g * K + k];
        a[k] = to_T<T>(o.a);
        b[k] = to_T<T>(o.b);
        ab[k] = a[k] + b[k];
        w[k] = to_T<T>(o.w);
    }
    if (quad == 0 || quad == 3) diag_sweep<T, R, K, true>(A, D, ring, wrap, scratch, prod, cons, a, b, ab, w);
    else diag_sweep<T, R, K, false>(A, D, ring, wrap, scratch, prod, cons, a, b, ab, w);
    if (lane == 0) atomicMax(&A.ctl->t_last, (unsigned long long)wall_clock64());
}

template <typename T, int R, int K>
hipError_t launch_diag_t(const DiagArgs& a, int ntasks, int nb, hipStream_t s)
{
    constexpr int NO = (kWave / R) * K;
    if (nb < 1 || nb > diag_max_waves<T, K>() || ntasks < 1) return hipErrorInvalidValue;
    const size_t lds = sizeof(T) * (((size_t)(nb - 1) * diag_ring<R>() + (size_t)a.wrap_cols) * NO + kWave * K) +
                       sizeof(int) * 2 * kDiagMaxWaves;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)diag_kernel<T, R, K>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((diag_kernel<T, R, K>), dim3(ntasks), dim3(64 * nb), lds, s, a);
    return hipGetLastError();
}

}  // namespace rom

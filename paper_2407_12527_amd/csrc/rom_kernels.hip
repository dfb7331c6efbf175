// rom_kernels.hip -- gfx950 (MI355X) kernels of librom.
//
//   (sweep_kernel lives in rom_sweep.h, instantiated per tile shape in rom_sweep_*.hip)
//   combine_kernel   phi = sum of the per-group partial fluxes in a fixed order, the next
//                    isotropic source sigma_s phi + q, the FP64 relative change and the
//                    per-system convergence decision of source iteration (eq. (3.10));
//                    combine_moments_kernel does the same for the linear kernel's moments;
//   contract_*       anisotropic scattering source S = sigma_s (Psi' P) + q (eq. (3.1) right-hand
//                    side with W = w P of eq. (3.4)): BF16 MFMA with FP32 accumulation, or a plain
//                    tiled FP64/FP32 kernel for the FP64 path;
//   moments_kernel   FP64 ensemble mean and unbiased variance over samples (eq. (4.6));
//   kernel_*_kernel  the transposed kernel matrices the contraction reads, built on the device from
//                    the ordinates of each system (new ordinates every ROM sample).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <cstdlib>

#include "rom_common.h"

namespace rom {

// ------------------------------------------------------------------------------------ combine
__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// Finalize one iteration for every running system: called by every thread of the last block of
// the combine step, each taking systems tid, tid + blockDim.x, ...  (a single thread walking the
// systems one after the other paid a dependent memory round trip per system: about 100 us per
// step for 200 systems).
__device__ void finalize_iteration(const CombineArgs& A)
{
    __shared__ int s_active;
    if (threadIdx.x == 0) s_active = 0;
    __syncthreads();
    int active = 0;
    for (int s = threadIdx.x; s < A.nsys; s += blockDim.x) {
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
    if (active) atomicAdd(&s_active, active);
    __syncthreads();
    if (threadIdx.x == 0) A.ctl->active = s_active;
}

// Block maxima (wave reduction, then across the 4 waves), the per-system FP64 maxima as atomics,
// and the last block's finalize of the iteration.
__device__ __forceinline__ void combine_tail(const CombineArgs& A, bool run, int s, double dmax, double pmax)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        pmax = fmax(pmax, __shfl_xor(pmax, off, 64));
    }
    __shared__ double sd[8], sp[8];  // one per wave (blocks of up to 8 waves)
    __shared__ int s_last;
    if ((tid & 63) == 0) {
        sd[tid >> 6] = dmax;
        sp[tid >> 6] = pmax;
    }
    __syncthreads();
    if (tid == 0) {
        const int nw = (int)blockDim.x >> 6;
        for (int k = 1; k < nw; ++k) {
            sd[0] = fmax(sd[0], sd[k]);
            sp[0] = fmax(sp[0], sp[k]);
        }
        dmax = sd[0];
        pmax = sp[0];
        if (run && A.mode == 0) {
            atomicMax(&A.sysctl[s].dmax_bits, dbits(dmax));  // non-negative doubles order as integers
            atomicMax(&A.sysctl[s].pmax_bits, dbits(pmax));
        }
        // The maxima are device-scope atomics; waiting for their completion before counting the
        // block in is all the last block needs (the fluxes themselves are read by later kernels).
        stores_complete();
        s_last = atomicAdd(&A.ctl->blocks_done, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) {
        if (A.mode == 0) finalize_iteration(A);
        if (tid == 0) {
            if (A.ctl->t_last > A.ctl->t_first && A.ctl->t_first != ~0ull) {
                const unsigned long long t0 = A.ctl->t_mark < A.ctl->t_first ? A.ctl->t_mark : A.ctl->t_first;
                A.ctl->sweep_ticks += A.ctl->t_last - t0;
                A.ctl->sweeps += 1;
            }
            A.ctl->t_first = ~0ull;
            A.ctl->t_last = 0ull;
            A.ctl->t_mark = wall_clock64();  // this kernel ends here; the next sweep follows
            A.ctl->blocks_done = 0;
            A.ctl->ticket = 0;
            A.ctl->epoch += 1;
        }
    }
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
                    if (A.mode == 0) src[cell] = fma(ss[cell], v[u], q[cell]);
                }
            }
        }
    }
    combine_tail(A, run, s, dmax, pmax);
}

// Combine for systems with many partial slots (the row-lane sweep writes one per task): a block
// owns 64 * CPT cells, its four waves sum interleaved quarters of the slot list (two independent
// chains each, so loads stay in flight), and the per-cell total is formed in a fixed order,
// ((w0 + w1) + (w2 + w3)), so results are deterministic.
template <typename T, int CPT>
__global__ __launch_bounds__(256) void combine_many_kernel(CombineArgs A)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (A.mode == 0 && A.ctl->active == 0) return;
    const int2 blk = A.blocks[blockIdx.x];
    const int s = blk.x;
    const SystemDev& SD = A.sys[s];
    const ProblemDev& P = A.probs[SD.prob];
    const int cells = P.nx * P.ny;
    const bool run = A.mode == 1 || A.sysctl[s].state == 0;
    __shared__ T wsum[4][64 * CPT];
    double dmax = 0.0, pmax = 0.0;
    if (run) {
        const T* __restrict__ part = (const T*)A.part;
        const int ns = SD.nslots;
        const int64_t* __restrict__ soff = A.slot_off;
        const int32_t* __restrict__ sord = A.slot_order + SD.slot_first;
        T a0[CPT], a1[CPT];
        int cl[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            a0[c] = a1[c] = T(0);
            cl[c] = min(blk.y + c * 64 + lane, cells - 1);  // clamped: a valid address, result unused
        }
        int k = wave;
        for (; k + 4 < ns; k += 8) {
            const T* __restrict__ p0 = part + soff[sord[k]];
            const T* __restrict__ p1 = part + soff[sord[k + 4]];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                a0[c] += p0[cl[c]];
                a1[c] += p1[cl[c]];
            }
        }
        if (k < ns) {
            const T* __restrict__ p0 = part + soff[sord[k]];
#pragma unroll
            for (int c = 0; c < CPT; ++c) a0[c] += p0[cl[c]];
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) wsum[wave][c * 64 + lane] = a0[c] + a1[c];
    }
    __syncthreads();
    if (run) {
        T* __restrict__ phi = (T*)A.phi + SD.phi_off;
        T* __restrict__ src = (T*)A.src + SD.src_off;
        const T* __restrict__ ss = (const T*)A.sigma_s + P.field_off;
        const T* __restrict__ q = (const T*)A.q + P.field_off;
        for (int e = tid; e < 64 * CPT; e += 256) {
            const int cell = blk.y + e;
            if (cell < cells) {
                const T v = (wsum[0][e] + wsum[1][e]) + (wsum[2][e] + wsum[3][e]);
                const T old = phi[cell];
                dmax = fmax(dmax, fabs((double)v - (double)old));
                pmax = fmax(pmax, fabs((double)v));
                phi[cell] = v;
                if (A.mode == 0) src[cell] = fma(ss[cell], v, q[cell]);
            }
        }
    }
    combine_tail(A, run, s, dmax, pmax);
}

// 16-byte vector of T
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
};
template <>
struct Vec16<double> {
    using type = double2;
};

// Many-slot combine with 16-byte loads: a block owns 64 * 16 bytes of consecutive cells (256
// FP32 / 128 FP64 cells), each lane 16 bytes of them; the block's NW waves (4 or 8) split the
// system's slots (wave w takes slots w, w + NW, ...) and a lane keeps up to 16 slot loads in
// flight in 16 independent accumulators, so a system of up to 16 NW slots is read in one round
// trip.  phi, sigma_s and q of the cell a thread updates are loaded before the slots, and the
// slot offsets come from a table already in summation order, so no load waits on another.  Each
// wave folds its accumulators in a fixed tree and the wave totals are added pairwise in a fixed
// tree: deterministic for a given slot count and NW.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void combine_vec_kernel(CombineArgs A)
{
    using V4 = typename Vec16<T>::type;
    constexpr int V = 16 / sizeof(T);
    constexpr int U = 16;
    static_assert(NW == 4 || NW == 8, "4 or 8 waves");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (A.mode == 0 && A.ctl->active == 0) return;
    const int2 blk = A.blocks[blockIdx.x];
    const int s = blk.x;
    const SystemDev& SD = A.sys[s];
    const ProblemDev& P = A.probs[SD.prob];
    const int cells = P.nx * P.ny;
    const bool run = A.mode == 1 || A.sysctl[s].state == 0;
    __shared__ T wsum[NW][64 * V];
    double dmax = 0.0, pmax = 0.0;
    // the cell this thread updates (64 * V <= 256 cells per block)
    const int ucell = blk.y + tid;
    const bool upd = run && tid < 64 * V && ucell < cells;
    T* __restrict__ phi = (T*)A.phi + SD.phi_off;
    T* __restrict__ src = (T*)A.src + SD.src_off;
    T old = T(0), ssv = T(0), qv = T(0);
    if (upd) {
        old = phi[ucell];
        if (A.mode == 0) {
            ssv = ((const T*)A.sigma_s + P.field_off)[ucell];
            qv = ((const T*)A.q + P.field_off)[ucell];
        }
    }
    if (run) {
        const T* __restrict__ part = (const T*)A.part;
        const int ns = SD.nslots;
        const int64_t* __restrict__ soff = A.slot_off_ord + SD.slot_first;
        const int c0 = blk.y + lane * V;
        const bool in = c0 < cells;  // cells is a multiple of V: a lane's V cells are all in or all out
        V4 acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = V4{};
        int k = wave;
        for (; k + NW * (U - 1) < ns; k += NW * U) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (in) acc[u] += *(const V4*)(part + soff[k + NW * u] + c0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (in && k + NW * u < ns) acc[u] += *(const V4*)(part + soff[k + NW * u] + c0);
#pragma unroll
        for (int h = U / 2; h > 0; h /= 2)
#pragma unroll
            for (int u = 0; u < h; ++u) acc[u] += acc[u + h];
        const T* tv = (const T*)&acc[0];
#pragma unroll
        for (int i = 0; i < V; ++i) wsum[wave][lane * V + i] = tv[i];
    }
    __syncthreads();
    if (upd) {
        const int e = tid;
        T v = (wsum[0][e] + wsum[1][e]) + (wsum[2][e] + wsum[3][e]);
        if constexpr (NW == 8) v += (wsum[4][e] + wsum[5][e]) + (wsum[6][e] + wsum[7][e]);
        dmax = fabs((double)v - (double)old);
        pmax = fabs((double)v);
        phi[ucell] = v;
        if (A.mode == 0) src[ucell] = fma(ssv, v, qv);
    }
    combine_tail(A, run, s, dmax, pmax);
}

// Few-slot combine with vector loads (at most 8 slots, e.g. ensembles with one lane group per
// quadrant): each thread owns 16 bytes of consecutive cells in each of the block's TPB tiles of
// 256 * 16 bytes; it issues every load of all its tiles (one 16-byte load per slot, plus phi,
// sigma_s and q) before any arithmetic or store, so a thread keeps up to TPB * 11 loads in flight,
// and the block's convergence atomics are amortized over TPB tiles.  Slots are added as
// ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)).
constexpr int kFewTiles = 4;

template <typename T>
__global__ __launch_bounds__(256) void combine_vec_few_kernel(CombineArgs A)
{
    using V4 = typename Vec16<T>::type;
    constexpr int V = 16 / sizeof(T);
    constexpr int TPB = kFewTiles;
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
        const T* __restrict__ ssp = (const T*)A.sigma_s + P.field_off;
        const T* __restrict__ qp = (const T*)A.q + P.field_off;
        T* __restrict__ phi = (T*)A.phi + SD.phi_off;
        T* __restrict__ src = (T*)A.src + SD.src_off;
        const int ns = SD.nslots;
        const int64_t* __restrict__ soff = A.slot_off;
        const int32_t* __restrict__ sord = A.slot_order + SD.slot_first;
        const T* sp[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sp[k] = k < ns ? part + soff[sord[k]] : nullptr;
        V4 acc[TPB][8], old[TPB], ssv[TPB], qv[TPB];
#pragma unroll
        for (int t = 0; t < TPB; ++t) {
            const int c0 = blk.y + t * 256 * V + (int)threadIdx.x * V;
            const bool in = c0 < cells;  // cells is a multiple of V
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[t][k] = (in && k < ns) ? *(const V4*)(sp[k] + c0) : V4{};
            old[t] = in ? *(const V4*)(phi + c0) : V4{};
            ssv[t] = (in && A.mode == 0) ? *(const V4*)(ssp + c0) : V4{};
            qv[t] = (in && A.mode == 0) ? *(const V4*)(qp + c0) : V4{};
        }
#pragma unroll
        for (int t = 0; t < TPB; ++t) {
            const int c0 = blk.y + t * 256 * V + (int)threadIdx.x * V;
            if (c0 >= cells) continue;
            const V4 tot = ((acc[t][0] + acc[t][1]) + (acc[t][2] + acc[t][3])) +
                           ((acc[t][4] + acc[t][5]) + (acc[t][6] + acc[t][7]));
            const T* tv = (const T*)&tot;
            const T* ov = (const T*)&old[t];
            const T* sv = (const T*)&ssv[t];
            const T* qq = (const T*)&qv[t];
            V4 sn;
            T* snv = (T*)&sn;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                dmax = fmax(dmax, fabs((double)tv[i] - (double)ov[i]));
                pmax = fmax(pmax, fabs((double)tv[i]));
                snv[i] = fma(sv[i], tv[i], qq[i]);
            }
            *(V4*)(phi + c0) = tot;
            if (A.mode == 0) *(V4*)(src + c0) = sn;
        }
    }
    combine_tail(A, run, s, dmax, pmax);
}

// Combine of the linear-kernel sweep (four partial planes per slot: phi, Jx~, Jy~, phi~): per
// cell the fixed-order sums over the system's slots, phi, its change, and the three source planes
// of the next sweep, S0 = sigma_s phi~ + q, S1 = sigma_s g Jx~, S2 = sigma_s g Jy~ (the folded
// kernel 1 + g (c c' + s s') of eq. (2.1) contracted through its moments).  Without
// normalization, or on a mirror-symmetric set, phi~ = phi and plane 3 is not formed.
template <typename T>
__global__ __launch_bounds__(256) void combine_moments_kernel(CombineArgs A)
{
    const int tid = threadIdx.x;
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
        const T g = (T)SD.g;
        const int64_t pl = cells;
        for (int cell = blk.y + tid; cell < c1; cell += 256) {
            T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
            for (int k = 0; k < ns; ++k) {
                const T* __restrict__ pk = part + soff[sord[k]] + cell;
                v0 += pk[0];
                v1 += pk[pl];
                v2 += pk[2 * pl];
                if (A.mom_r) v3 += pk[3 * pl];
            }
            if (!A.mom_r) v3 = v0;
            const T old = phi[cell];
            dmax = fmax(dmax, fabs((double)v0 - (double)old));
            pmax = fmax(pmax, fabs((double)v0));
            phi[cell] = v0;
            if (A.mode == 0) {
                const T sg = ss[cell] * g;
                src[cell] = fma(ss[cell], v3, q[cell]);
                src[pl + cell] = sg * v1;
                src[2 * pl + cell] = sg * v2;
            }
        }
    }
    combine_tail(A, run, s, dmax, pmax);
}

// Mark the start of a captured run of iterations (its first sweep is timed from here).
__global__ void mark_kernel(Ctl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->t_mark = wall_clock64();
}

hipError_t launch_mark(Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(mark_kernel, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
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

// Per-system and control state at the start of a solve.
__device__ __forceinline__ void reset_system(SysCtl& c)
{
    c.dmax_bits = 0ull;
    c.pmax_bits = 0ull;
    c.iter = 0;
    c.state = 0;
    c.grow = 0;
    c.r = 1.0;
    c.r_prev = 1.0;
}

__device__ __forceinline__ void reset_ctl(Ctl* ctl, int nsys)
{
    ctl->active = nsys;
    ctl->error = 0;
    ctl->sweeps = 0;
    ctl->t_first = ~0ull;
    ctl->t_last = 0ull;
    ctl->sweep_ticks = 0ull;
    ctl->t_mark = ~0ull;  // the first sweep is timed from its first ticket claim
    ctl->ticket = 0;
    ctl->blocks_done = 0;
    ctl->epoch += 1;
}

// Clear per-system state before a solve (graph-safe: a kernel, not a memset).
__global__ void reset_systems_kernel(SysCtl* sc, int nsys, Ctl* ctl)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) reset_system(sc[s]);
    if (s == 0) reset_ctl(ctl, nsys);
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
// 64 staged in LDS; each wave owns 64 x 64 = 2 x 2 tiles of v_mfma_f32_32x32x16_bf16.  The next
// K step's tiles are loaded into registers while the matrix cores work on the current one, so
// the global-load latency overlaps the MFMA of the step before it.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int GM = 128, GN = 128, GK = 64;
constexpr int LDS_PAD = 8;  // bf16 elements of padding per LDS row (keeps 16-byte alignment)
constexpr int kSegs = GK / 8;               // 16-byte segments of one tile row
constexpr int kRowStep = 256 / kSegs;      // tile rows moved by the block per piece
constexpr int kStage = GM / kRowStep;      // 16-byte pieces of one operand tile per thread

// One GM x GN output tile (block `blk` of the `nb` blocks of this contraction); remap: spread the
// blocks over the XCDs by contiguous runs (single launches only).
__device__ __forceinline__ void contract_bf16_tile(const ContractArgs& A, const int blk, const int nb, const bool remap)
{
    if (A.sysctl && A.sysctl[A.sys_index].state != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[GM][GK + LDS_PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[GN][GK + LDS_PAD];
    __shared__ float ss_q[2][GM];  // sigma_s and q of the block's rows, for the epilogue
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / 2, wn = wave % 2;
    // Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Renumber them
    // so that every XCD owns a contiguous run of logical tiles: the N/GN tiles that share one A
    // row-block (the large operand) then run on the same XCD and read A from HBM once.
    const int nblk_n = A.N / GN;
    const int lb = (remap && nb % 8 == 0) ? (blk % 8) * (nb / 8) + blk / 8 : blk;
    const int bm = lb / nblk_n, bn = lb % nblk_n;
    const int m0 = bm * GM, n0 = bn * GN;
    const __bf16* __restrict__ Ag = (const __bf16*)A.a;
    const __bf16* __restrict__ Bg = (const __bf16*)A.bt;
    if (tid < 2 * GM) {
        // rows past M take row M - 1's values; their results are never stored.  The first barrier
        // of the K loop orders these stores before the epilogue's reads.
        const int r = min(m0 + tid % GM, A.M - 1);
        ss_q[tid / GM][tid % GM] = tid < GM ? ((const float*)A.sigma_s)[r] : ((const float*)A.q)[r];
    }

    f32x16_t acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.0f;

    // global -> registers: each tile is 128 rows x GK bf16, 256 threads x kStage x 16 B; thread tid
    // moves rows tid / kSegs + kRowStep h, 16-byte segment tid % kSegs.  Rows of A past M read row
    // M - 1 (in bounds) and their results are never stored.
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    u32x4 ra[kStage], rb[kStage];
    const int row0 = tid / kSegs, seg = tid % kSegs;
    // element k of row m: row-major m * K + k, or blocked ((k / 16) * M + m) * 16 + k % 16 (a
    // 16-byte segment never straddles a block); a_at(h) + d(k0) addresses K step k0
    const bool blocked = A.blocked != 0;
    auto a_at = [&](const int h) {
        const int64_t m = min(m0 + row0 + kRowStep * h, A.M - 1);
        return blocked ? Ag + ((int64_t)(seg / 2) * A.M + m) * 16 + (seg % 2) * 8 : Ag + m * A.K + seg * 8;
    };
    const int64_t a_kstep = blocked ? (int64_t)(GK / 16) * A.M * 16 : GK;  // advance of one K step
    const __bf16* __restrict__ pb = Bg + (int64_t)(n0 + row0) * A.K + seg * 8;
    const int64_t sb = kRowStep * (int64_t)A.K;
#pragma unroll
    for (int h = 0; h < kStage; ++h) {
        ra[h] = *(const u32x4*)a_at(h);
        rb[h] = *(const u32x4*)(pb + h * sb);
    }
    for (int k0 = 0; k0 < A.K; k0 += GK) {
#pragma unroll
        for (int h = 0; h < kStage; ++h) {
            *(u32x4*)&As[row0 + kRowStep * h][seg * 8] = ra[h];
            *(u32x4*)&Bs[row0 + kRowStep * h][seg * 8] = rb[h];
        }
        __syncthreads();
        if (k0 + GK < A.K) {
#pragma unroll
            for (int h = 0; h < kStage; ++h) {
                ra[h] = *(const u32x4*)(a_at(h) + (k0 / GK + 1) * a_kstep);
                rb[h] = *(const u32x4*)(pb + h * sb + k0 + GK);
            }
        }
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
    float* __restrict__ out = (float*)A.out;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int col = n0 + wn * 64 + y * 32 + (lane % 32);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int rl = wm * 64 + x * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
                const int row = m0 + rl;
                const int64_t at = blocked ? ((int64_t)(col / 16) * A.M + row) * 16 + col % 16 : (int64_t)row * A.N + col;
                if (row < A.M) out[at] = fmaf(ss_q[0][rl], acc[x][y][e], ss_q[1][rl]);
            }
        }
    }
}

// The contraction is the kernel that precedes the sweep of an anisotropic iteration.  It clears
// t_mark (one plain store), so that sweep is timed from its own first ticket claim rather than
// from the end of the combine step before the contraction.  (The last block to finish used to
// stamp t_mark through a counter every block incremented: c4 step 5.60 ms against 5.47 ms
// without it.)
__device__ __forceinline__ void unmark(Ctl* ctl)
{
    if (ctl && blockIdx.x == 0 && threadIdx.x == 0) ctl->t_mark = ~0ull;
}

__global__ __launch_bounds__(256) void contract_bf16_kernel(ContractArgs A, Ctl* ctl)
{
    if (ctl && ctl->active == 0) return;  // every system has stopped
    unmark(ctl);
    contract_bf16_tile(A, blockIdx.x, gridDim.x, true);
}

// The contractions of several systems in one launch: block b computes tile map[b].y of
// contraction map[b].x (an ensemble's samples each have their own small kernel matrix).
__global__ __launch_bounds__(256) void contract_bf16_batch_kernel(const ContractArgs* __restrict__ items,
                                                                  const int2* __restrict__ map, Ctl* ctl)
{
    if (ctl && ctl->active == 0) return;  // every system has stopped
    unmark(ctl);
    const int2 m = map[blockIdx.x];
    contract_bf16_tile(items[m.x], m.y, 0, false);
}

// Large single contractions (N >= 256): 512 threads = 8 waves in a 2 x 4 arrangement, block tile
// 256 x 256, each wave 128 x 64 = 4 x 2 tiles of v_mfma_f32_32x32x16_bf16.  The larger tile
// halves the operand traffic from L2 per flop against 128 x 128 (every A row-block is read N / 256
// times, every B row-block M / 256 times).  K steps of 64 go through two LDS buffers: at the top of
// step k the registers holding step k + 1 are written to the other buffer (read during step k - 1,
// released by that step's barrier) and the loads of step k + 2 are issued, so the global loads
// have a whole step of matrix work to land and each step needs one barrier.  146 KiB of LDS: one
// workgroup per CU, two waves per SIMD.  N may end in a half tile of 128 columns: the waves whose
// columns lie past N skip the matrix work and the stores.
constexpr int BM2 = 256, BN2 = 256;
constexpr int kRowStep2 = 512 / kSegs;     // tile rows moved by the block per piece (64)
constexpr int kStage2 = BM2 / kRowStep2;   // 16-byte pieces of one operand tile per thread (4)
constexpr size_t kBigLds = 2 * 2 * (size_t)BM2 * (GK + LDS_PAD) * sizeof(__bf16) + 2 * BM2 * sizeof(float);

__global__ __launch_bounds__(512) void contract_bf16_big_kernel(ContractArgs A, Ctl* ctl)
{
    if (ctl && ctl->active == 0) return;  // every system has stopped
    unmark(ctl);
    if (A.sysctl && A.sysctl[A.sys_index].state != 0) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char big_smem[];
    typedef __bf16 Row[GK + LDS_PAD];
    Row* As = (Row*)big_smem;                  // [2][BM2] rows
    Row* Bs = As + 2 * BM2;                    // [2][BN2] rows
    float* ss_q = (float*)(Bs + 2 * BN2);      // [2][BM2]: sigma_s, q
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / 4, wn = wave % 4;
    const int nb = gridDim.x, blk = blockIdx.x;
    const int nblk_n = (A.N + BN2 - 1) / BN2;
    // XCD-aware order, as in the 128 x 128 kernel: the N tiles of one A row-block on one XCD
    const int lb = (nb % 8 == 0) ? (blk % 8) * (nb / 8) + blk / 8 : blk;
    const int bm = lb / nblk_n, bn = lb % nblk_n;
    const int m0 = bm * BM2, n0 = bn * BN2;
    const bool live = n0 + wn * 64 < A.N;  // uniform per wave
    const __bf16* __restrict__ Ag = (const __bf16*)A.a;
    const __bf16* __restrict__ Bg = (const __bf16*)A.bt;
    if (tid < 2 * BM2) {
        const int r = min(m0 + tid % BM2, A.M - 1);
        ss_q[tid] = tid < BM2 ? ((const float*)A.sigma_s)[r] : ((const float*)A.q)[r];
    }

    f32x16_t acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.0f;

    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    u32x4 ra[kStage2], rb[kStage2];
    const int row0 = tid / kSegs, seg = tid % kSegs;
    const bool blocked = A.blocked != 0;
    // rows past M (A) or N (B) read the last row (in bounds); their results are never stored
    auto a_at = [&](const int h) {
        const int64_t m = min(m0 + row0 + kRowStep2 * h, A.M - 1);
        return blocked ? Ag + ((int64_t)(seg / 2) * A.M + m) * 16 + (seg % 2) * 8 : Ag + m * A.K + seg * 8;
    };
    const int64_t a_kstep = blocked ? (int64_t)(GK / 16) * A.M * 16 : GK;
    auto b_at = [&](const int h) {
        const int64_t n = min(n0 + row0 + kRowStep2 * h, A.N - 1);
        return Bg + n * A.K + seg * 8;
    };
    auto load = [&](const int ks) {
#pragma unroll
        for (int h = 0; h < kStage2; ++h) {
            ra[h] = *(const u32x4*)(a_at(h) + ks * a_kstep);
            rb[h] = *(const u32x4*)(b_at(h) + ks * GK);
        }
    };
    auto stage = [&](const int buf) {
#pragma unroll
        for (int h = 0; h < kStage2; ++h) {
            *(u32x4*)&As[buf * BM2 + row0 + kRowStep2 * h][seg * 8] = ra[h];
            *(u32x4*)&Bs[buf * BN2 + row0 + kRowStep2 * h][seg * 8] = rb[h];
        }
    };
    const int nk = A.K / GK;
    load(0);
    stage(0);
    if (nk > 1) load(1);
    __syncthreads();
    for (int ks = 0; ks < nk; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < nk) {
            stage(cur ^ 1);
            if (ks + 2 < nk) load(ks + 2);
        }
        if (live) {
#pragma unroll
            for (int kk = 0; kk < GK; kk += 16) {
                bf16x8_t af[4], bfr[2];
#pragma unroll
                for (int x = 0; x < 4; ++x)
                    af[x] = *(const bf16x8_t*)&As[cur * BM2 + wm * 128 + x * 32 + (lane % 32)][kk + 8 * (lane / 32)];
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    bfr[y] = *(const bf16x8_t*)&Bs[cur * BN2 + wn * 64 + y * 32 + (lane % 32)][kk + 8 * (lane / 32)];
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[x], bfr[y], acc[x][y], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds column (lane % 32) and rows 8*(e/4) + 4*(lane/32) + e%4 of each tile
    if (live && blocked) {
        // Through LDS (the operand buffers are free after the last barrier): per row tile x, the
        // wave's 32 x 64 results go to its own slice (4 column blocks of 16; rows padded to 20
        // floats and blocks to 672 so the 4-byte writes do not conflict), then leave as 16-byte
        // stores, each instruction one contiguous KB of the blocked output (16 rows of a block).
        constexpr int RS = 20, CS = 672;
        float* slice = (float*)big_smem + wave * 4 * CS;
        float* __restrict__ out = (float*)A.out;
        const int gcb0 = (n0 + wn * 64) / 16;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int col = y * 32 + (lane % 32);
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int rr = 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
                    const int rl = wm * 128 + x * 32 + rr;
                    slice[(col / 16) * CS + rr * RS + col % 16] = fmaf(ss_q[rl], acc[x][y][e], ss_q[BM2 + rl]);
                }
            }
            // a wave's LDS accesses complete in order: the reads below see the writes above, and
            // the next x's writes come after these reads
#pragma unroll
            for (int jb = 0; jb < 8; ++jb) {
                const int cb = jb / 2, rr = (jb % 2) * 16 + lane / 4, q4 = lane % 4;
                const f32x4_t v = *(const f32x4_t*)&slice[cb * CS + rr * RS + q4 * 4];
                const int row = m0 + wm * 128 + x * 32 + rr;
                if (row < A.M) *(f32x4_t*)&out[((int64_t)(gcb0 + cb) * A.M + row) * 16 + q4 * 4] = v;
            }
        }
    } else if (live) {
        float* __restrict__ out = (float*)A.out;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int col = n0 + wn * 64 + y * 32 + (lane % 32);
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int rl = wm * 128 + x * 32 + 8 * (e / 4) + 4 * (lane / 32) + (e % 4);
                    const int row = m0 + rl;
                    if (row < A.M) out[(int64_t)row * A.N + col] = fmaf(ss_q[rl], acc[x][y][e], ss_q[BM2 + rl]);
                }
            }
        }
    }
}

// Plain tiled contraction (FP64 or FP32 operands, same precision out), 16 x 16 threads, 64 x 64
// block tile, each thread a 4 x 4 micro-tile.
template <typename T>
__device__ __forceinline__ void contract_plain_tile(const ContractArgs& A, const int blk)
{
    if (A.sysctl && A.sysctl[A.sys_index].state != 0) return;
    __shared__ T As[16][64 + 1];
    __shared__ T Bs[16][64 + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int nblk_n = (A.N + 63) / 64;
    const int m0 = (blk / nblk_n) * 64, n0 = (blk % nblk_n) * 64;
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

template <typename T>
__global__ __launch_bounds__(256) void contract_plain_kernel(ContractArgs A, Ctl* ctl)
{
    if (ctl && ctl->active == 0) return;  // every system has stopped
    unmark(ctl);
    contract_plain_tile<T>(A, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void contract_plain_batch_kernel(const ContractArgs* __restrict__ items,
                                                                   const int2* __restrict__ map, Ctl* ctl)
{
    if (ctl && ctl->active == 0) return;  // every system has stopped
    unmark(ctl);
    const int2 m = map[blockIdx.x];
    contract_plain_tile<T>(items[m.x], m.y);
}

// FP32 angular flux -> BF16 copy (used when the sweep stored FP32 psi').
__global__ void cast_bf16_kernel(const float* __restrict__ in, __hip_bfloat16* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = __float2bfloat16(in[i]);
}

// ------------------------------------------------------------------------------ kernel matrix
// Henyey-Greenstein kernel of the planar problem: the 3-D kernel at cos xi = u.v averaged over
// the mirror image of v in the x-y plane (the z half of the sphere folded onto the other), the same
// form the ordinates carry (c, s, z with the sweep using c, s only).
__device__ __forceinline__ double km_hg(double g, double mu)
{
    const double d = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (d * sqrt(d));
}

// P(u_k incoming, u_n outgoing) for valid internal ordinates k and n of system S.
__device__ __forceinline__ double km_value(const KmArgs& A, const KmSys& S, int64_t k, int64_t n)
{
    if (S.kind == 3) {
        const int uk = A.uidx[S.ord_off + k], un = A.uidx[S.ord_off + n];
        return A.dense[S.dense_off + (int64_t)uk * S.n + un];
    }
    const double* a = A.ord + (S.ord_off + k) * 4;
    const double* b = A.ord + (S.ord_off + n) * 4;
    const double planar = a[0] * b[0] + a[1] * b[1];
    const double zz = a[2] * b[2];
    return 0.5 * (km_hg(S.g, planar + zz) + km_hg(S.g, planar - zz));
}

// 1 / r_k, r_k = sum_n w_n P(u_k, u_n), for every internal ordinate k of the normalized systems:
// one wavefront per k, lanes over n in a fixed order, a fixed butterfly at the end.
__global__ void __launch_bounds__(256) kernel_rowsum_kernel(KmArgs A)
{
    const KmSys S = A.sys[blockIdx.y];
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (!S.norm || k >= S.npad || A.uidx[S.ord_off + k] < 0) return;
    double r = 0.0;
    for (int n = lane; n < S.npad; n += 64)
        if (A.uidx[S.ord_off + n] >= 0) r += A.ord[(S.ord_off + n) * 4 + 3] * km_value(A, S, k, n);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
    if (lane == 0) A.inv_r[S.ord_off + k] = 1.0 / r;
}

// Bt[n][k] = P(u_k, u_n) / r_k over the whole [al][al] matrix (zero where n or k is padding):
// a block writes 4 rows n, threads along k (contiguous stores).
__global__ void __launch_bounds__(256) kernel_fill_kernel(KmArgs A)
{
    const KmSys S = A.sys[blockIdx.y];
    const int n0 = blockIdx.x * 4;
    if (n0 >= S.al) return;
    for (int e = threadIdx.x; e < 4 * S.al; e += 256) {
        const int n = n0 + e / S.al, k = e % S.al;
        if (n >= S.al) break;
        double v = 0.0;
        if (n < S.npad && k < S.npad && A.uidx[S.ord_off + n] >= 0 && A.uidx[S.ord_off + k] >= 0) {
            v = km_value(A, S, k, n);
            if (S.norm) v *= A.inv_r[S.ord_off + k];
        }
        const int64_t idx = S.pt_off + (int64_t)n * S.al + k;
        if (A.fp64) {
            static_cast<double*>(A.bt)[idx] = v;
        } else {
            const uint32_t u = __float_as_uint((float)v);  // round to nearest even, as the sweep's BF16 stores
            static_cast<uint16_t*>(A.bt)[idx] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        }
    }
}

// ------------------------------------------------------------------------------------ launchers
hipError_t launch_sweep_f32_8x4(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);
hipError_t launch_sweep_f32_8x8(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);
hipError_t launch_sweep_f32_16x8(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);
hipError_t launch_sweep_f32_16x16(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);
hipError_t launch_sweep_f64_8x4(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);
hipError_t launch_sweep_f64_8x8(const SweepArgs&, int, bool, bool, int, int, int, hipStream_t);

size_t sweep_lds_bytes(bool fp64, int tx, int ty, bool ang, int L, int nw, int mom)
{
    const size_t esz = fp64 ? 8 : 4;
    const size_t ch = (size_t)tx * ty;
    const size_t ngd = ang ? 1 : (size_t)(kWave / L) * (mom == 4 ? 3 : 1);
    return esz * ((size_t)nw * (ch + ngd * (ch + 4)) + (size_t)(nw > 1 ? nw - 1 : 1) * kRingSlots * tx * kWave) +
           sizeof(int) * (2 * kMaxBand + 1);
}

bool sweep_tile_supported(int tx, int ty)
{
    return (tx == 8 && (ty == 4 || ty == 8)) || (tx == 16 && (ty == 8 || ty == 16));
}

bool sweep_tile_supported_fp64(int tx, int ty) { return tx == 8 && (ty == 4 || ty == 8); }

hipError_t launch_sweep(const SweepArgs& a, int grid, bool fp64, int tx, int ty, bool dd, bool ang, int psi, int L,
                        int mom, hipStream_t s)
{
    if (fp64) {
        if (psi == 2) return hipErrorInvalidValue;
        if (tx == 8 && ty == 4) return launch_sweep_f64_8x4(a, grid, dd, ang, psi, L, mom, s);
        if (tx == 8 && ty == 8) return launch_sweep_f64_8x8(a, grid, dd, ang, psi, L, mom, s);
        return hipErrorInvalidValue;
    }
    if (tx == 8 && ty == 4) return launch_sweep_f32_8x4(a, grid, dd, ang, psi, L, mom, s);
    if (tx == 8 && ty == 8) return launch_sweep_f32_8x8(a, grid, dd, ang, psi, L, mom, s);
    if (tx == 16 && ty == 8) return launch_sweep_f32_16x8(a, grid, dd, ang, psi, L, mom, s);
    if (tx == 16 && ty == 16) return launch_sweep_f32_16x16(a, grid, dd, ang, psi, L, mom, s);
    return hipErrorInvalidValue;
}

hipError_t launch_diag_f32(const DiagArgs&, int, int, int, int, bool, hipStream_t);
hipError_t launch_diag_f64(const DiagArgs&, int, int, int, int, hipStream_t);

int diag_max_nb(bool fp64, int K, bool ang)
{
    (void)fp64;
    return (K > 1 || ang) ? 8 : kDiagMaxWaves;  // as diag_max_waves: two prefetch sets or K > 1
}

bool diag_supported(bool fp64, int R, int K)
{
    if (R != 16 && R != 64) return false;
    return fp64 ? (K == 1 || K == 2) : (K == 1 || K == 2 || K == 4);
}

size_t diag_lds_bytes(bool fp64, int R, int K, int nb)
{
    const size_t no = (size_t)(kWave / R) * K;
    const size_t ring = R == 16 ? 64 : 128;
    return (fp64 ? 8 : 4) * (size_t)(nb - 1) * ring * no + sizeof(int) * (2 * kDiagMaxWaves + 1);
}

hipError_t launch_diag(const DiagArgs& a, int grid, int nb, bool fp64, int R, int K, bool ang, hipStream_t s)
{
    if (!diag_supported(fp64, R, K) || (ang && fp64)) return hipErrorInvalidValue;
    return fp64 ? launch_diag_f64(a, grid, nb, R, K, s) : launch_diag_f32(a, grid, nb, R, K, ang, s);
}

hipError_t launch_combine(const CombineArgs& a, int nblocks, bool fp64, hipStream_t s)
{
    if (a.nmom == 4) {
        if (a.many_cpt != 0) return hipErrorInvalidValue;
        if (fp64) hipLaunchKernelGGL(combine_moments_kernel<double>, dim3(nblocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(combine_moments_kernel<float>, dim3(nblocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (a.nmom != 1) return hipErrorInvalidValue;
    if (a.vec == 2) {
        if (a.cells_per_block != kFewTiles * 256 * (fp64 ? 2 : 4)) return hipErrorInvalidValue;
        if (fp64) hipLaunchKernelGGL(combine_vec_few_kernel<double>, dim3(nblocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(combine_vec_few_kernel<float>, dim3(nblocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (a.vec == 1 || a.vec == 3) {
        // 4 waves per block; 8 for systems of more than 64 slots
        if (a.cells_per_block != 64 * (fp64 ? 2 : 4)) return hipErrorInvalidValue;
        if (a.vec == 3) {
            if (fp64) hipLaunchKernelGGL((combine_vec_kernel<double, 8>), dim3(nblocks), dim3(512), 0, s, a);
            else hipLaunchKernelGGL((combine_vec_kernel<float, 8>), dim3(nblocks), dim3(512), 0, s, a);
        } else {
            if (fp64) hipLaunchKernelGGL((combine_vec_kernel<double, 4>), dim3(nblocks), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((combine_vec_kernel<float, 4>), dim3(nblocks), dim3(256), 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.vec) return hipErrorInvalidValue;
    if (a.many_cpt > 0) {
        // block tiles of 64 * many_cpt cells (cells_per_block must match)
        if (a.cells_per_block != 64 * a.many_cpt) return hipErrorInvalidValue;
        if (fp64) {
            if (a.many_cpt == 1) hipLaunchKernelGGL((combine_many_kernel<double, 1>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 2) hipLaunchKernelGGL((combine_many_kernel<double, 2>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 4) hipLaunchKernelGGL((combine_many_kernel<double, 4>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 8) hipLaunchKernelGGL((combine_many_kernel<double, 8>), dim3(nblocks), dim3(256), 0, s, a);
            else return hipErrorInvalidValue;
        } else {
            if (a.many_cpt == 1) hipLaunchKernelGGL((combine_many_kernel<float, 1>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 2) hipLaunchKernelGGL((combine_many_kernel<float, 2>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 4) hipLaunchKernelGGL((combine_many_kernel<float, 4>), dim3(nblocks), dim3(256), 0, s, a);
            else if (a.many_cpt == 8) hipLaunchKernelGGL((combine_many_kernel<float, 8>), dim3(nblocks), dim3(256), 0, s, a);
            else return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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

// First source of every system: S = q (phi starts at 0), one launch for all systems;
// grid.y strides over the systems, grid.x over each system's cells.
template <typename T>
__global__ void init_source_kernel(const SystemDev* __restrict__ sys, const ProblemDev* __restrict__ probs, int nsys,
                                   const T* __restrict__ q, T* __restrict__ src)
{
    for (int k = blockIdx.y; k < nsys; k += gridDim.y) {
        const SystemDev& sd = sys[k];
        const ProblemDev& pd = probs[sd.prob];
        const int64_t cells = (int64_t)pd.nx * pd.ny;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x)
            src[sd.src_off + c] = q[pd.field_off + c];
    }
}

hipError_t launch_init_source(const SystemDev* sys, const ProblemDev* probs, int nsys, int64_t max_cells, bool fp64,
                              const void* q, void* src, hipStream_t s)
{
    if (nsys <= 0 || max_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min<int64_t>((max_cells + 255) / 256, 1024), (unsigned)std::min(nsys, 65535));
    if (fp64)
        hipLaunchKernelGGL(init_source_kernel<double>, grid, dim3(256), 0, s, sys, probs, nsys, (const double*)q, (double*)src);
    else
        hipLaunchKernelGGL(init_source_kernel<float>, grid, dim3(256), 0, s, sys, probs, nsys, (const float*)q, (float*)src);
    return hipGetLastError();
}

// The whole initial state of source iteration in one launch: phi = 0 over [0, phi_total), the
// first source S = q of every system (grid.y strides over the systems, grid.x over each system's
// cells), and the per-system and control state reset.  The three parts write disjoint memory.
template <typename T>
__global__ void init_state_kernel(const SystemDev* __restrict__ sys, const ProblemDev* __restrict__ probs, int nsys,
                                  const T* __restrict__ q, T* __restrict__ src, T* __restrict__ phi, int64_t phi_total,
                                  SysCtl* __restrict__ sc, Ctl* ctl)
{
    const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    const int64_t gtid = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = gtid; i < phi_total; i += nthreads) phi[i] = T(0);
    for (int k = blockIdx.y; k < nsys; k += gridDim.y) {
        const SystemDev& sd = sys[k];
        const ProblemDev& pd = probs[sd.prob];
        const int64_t cells = (int64_t)pd.nx * pd.ny;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x)
            src[sd.src_off + c] = q[pd.field_off + c];
        if (blockIdx.x == 0 && threadIdx.x == 0) reset_system(sc[k]);
    }
    if (gtid == 0) reset_ctl(ctl, nsys);
}

hipError_t launch_init_state(const SystemDev* sys, const ProblemDev* probs, int nsys, int64_t max_cells, bool fp64,
                             const void* q, void* src, void* phi, int64_t phi_total, SysCtl* sc, Ctl* ctl, hipStream_t s)
{
    if (nsys < 0 || max_cells < 0 || phi_total < 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((max_cells + 255) / 256, 1024)),
                    (unsigned)std::max(1, std::min(nsys, 65535)));
    if (fp64)
        hipLaunchKernelGGL(init_state_kernel<double>, grid, dim3(256), 0, s, sys, probs, nsys, (const double*)q,
                           (double*)src, (double*)phi, phi_total, sc, ctl);
    else
        hipLaunchKernelGGL(init_state_kernel<float>, grid, dim3(256), 0, s, sys, probs, nsys, (const float*)q,
                           (float*)src, (float*)phi, phi_total, sc, ctl);
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

// 256 x 256 tiles for large single contractions unless ROM_CONTRACT_TILE=128 (timing comparisons).
static bool contract_big_tiles()
{
    static const bool big = [] {
        const char* e = std::getenv("ROM_CONTRACT_TILE");
        return !(e && std::atoi(e) == 128);
    }();
    return big;
}

hipError_t launch_contract(const ContractArgs& a, int kind, hipStream_t s, Ctl* ctl)
{
    if (kind == 0) {
        if (a.N % GN != 0 || a.K % GK != 0) return hipErrorInvalidValue;
        if (a.N >= 2 * GN && contract_big_tiles()) {
            const hipError_t e = hipFuncSetAttribute((const void*)contract_bf16_big_kernel,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBigLds);
            if (e != hipSuccess) return e;
            const int grid = ((a.M + BM2 - 1) / BM2) * ((a.N + BN2 - 1) / BN2);
            hipLaunchKernelGGL(contract_bf16_big_kernel, dim3(grid), dim3(512), kBigLds, s, a, ctl);
            return hipGetLastError();
        }
        const int grid = ((a.M + GM - 1) / GM) * (a.N / GN);
        hipLaunchKernelGGL(contract_bf16_kernel, dim3(grid), dim3(256), 0, s, a, ctl);
    } else {
        const int grid = ((a.M + 63) / 64) * ((a.N + 63) / 64);
        if (kind == 1)
            hipLaunchKernelGGL(contract_plain_kernel<float>, dim3(grid), dim3(256), 0, s, a, ctl);
        else
            hipLaunchKernelGGL(contract_plain_kernel<double>, dim3(grid), dim3(256), 0, s, a, ctl);
    }
    return hipGetLastError();
}

int contract_blocks(const ContractArgs& a, int kind)
{
    if (kind == 0) return (a.N % GN != 0 || a.K % GK != 0) ? -1 : ((a.M + GM - 1) / GM) * (a.N / GN);
    return ((a.M + 63) / 64) * ((a.N + 63) / 64);
}

hipError_t launch_contract_batch(const ContractArgs* items, const int2* map, int nblocks, int kind, hipStream_t s,
                                 Ctl* ctl)
{
    if (nblocks < 1) return hipErrorInvalidValue;
    if (kind == 0) hipLaunchKernelGGL(contract_bf16_batch_kernel, dim3(nblocks), dim3(256), 0, s, items, map, ctl);
    else if (kind == 1) hipLaunchKernelGGL(contract_plain_batch_kernel<float>, dim3(nblocks), dim3(256), 0, s, items, map, ctl);
    else hipLaunchKernelGGL(contract_plain_batch_kernel<double>, dim3(nblocks), dim3(256), 0, s, items, map, ctl);
    return hipGetLastError();
}

hipError_t launch_kernel_matrix(const KmArgs& a, hipStream_t s)
{
    if (a.nsys < 1 || a.max_al < 1) return hipErrorInvalidValue;
    const dim3 grid((a.max_al + 3) / 4, a.nsys);
    hipLaunchKernelGGL(kernel_rowsum_kernel, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(kernel_fill_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* in, void* out, int64_t n, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(nb), dim3(256), 0, s, in, (__hip_bfloat16*)out, n);
    return hipGetLastError();
}

}  // namespace rom

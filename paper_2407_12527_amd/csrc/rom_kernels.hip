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

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_add(float v)
{
    // v + v[permuted lane]; lanes outside ROWMASK add 0
    int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false);
    return v + __int_as_float(moved);
}

// Sum over groups of L lanes (L = 16, 32, 64).  The last lane of each group receives the sum.
// DPP: xor-1 and xor-2 inside quads, rotations by 8 and 4 inside 16-lane rows, then row
// broadcasts 15 (rows 1, 3) and 31 (rows 2, 3) to join rows.
template <int N>
__device__ __forceinline__ void group_sum_f32(float (&v)[N], int L)
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = dpp_add<0xB1, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = dpp_add<0x4E, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = dpp_add<0x128, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = dpp_add<0x124, 0xF>(v[i]);
    if (L >= 32) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = dpp_add<0x142, 0xA>(v[i]);
    }
    if (L >= 64) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = dpp_add<0x143, 0xC>(v[i]);
    }
}

template <int N>
__device__ __forceinline__ void group_sum_f64(double (&v)[N], int L)
{
    for (int off = 1; off < L; off <<= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
    }
}

template <int N>
__device__ __forceinline__ void group_sum(float (&v)[N], int L) { group_sum_f32<N>(v, L); }
template <int N>
__device__ __forceinline__ void group_sum(double (&v)[N], int L) { group_sum_f64<N>(v, L); }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Wait until *p >= target (a strip below has finished chunk c of this epoch).  Polls with relaxed
// loads and issues one acquire fence at the end.  Bounded: after `limit` polls (or once another
// wave has timed out) the wait gives up and records the error, so every wave always exits.
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
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T>
__device__ __forceinline__ T to_T(double x) { return (T)x; }

// ------------------------------------------------------------------------------------ sweep
//
// One wavefront = one wave-stream strip task at a time.  Lane state while walking a strip:
//   xl[r]  x-face value entering row r of the strip (carried from chunk to chunk),
//   yd[i]  y-face value entering column i of the chunk (from the strip below, updated row by row
//          and handed to the strip above after the chunk's last row).
// Cell update (ordinate-scaled fluxes psi' = w psi, cell (i, j) visited in sweep order):
//   STEP: psi' = (w S + a x + b y) / (sigma_t + a + b),                x <- psi', y <- psi'
//   DD:   psi' = (w S + 2a x + 2b y) / (sigma_t + 2a + 2b),  x <- 2psi' - x, y <- 2psi' - y
// When sigma_t is constant along a row chunk, 1/(sigma_t + a + b) is taken once per row.
template <typename T, int TX, int TY, bool DD, bool ANG, int PSI>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs A)
{
    const int lane = threadIdx.x;
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

        // skip wave-streams whose systems have all stopped (flags change only between sweeps)
        bool any = false;
        for (int g = 0; g < kWave / L; ++g) {
            int s = W.sys[g];
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
        const T* __restrict__ Sp = srcp + SD.src_off;
        const T* __restrict__ Ap = angp + SD.ang_off + ld.ord;
        const int64_t npad = SD.npad;
        T* __restrict__ partp = part + (gslot >= 0 ? A.slot_off[gslot] : 0);

        const int nx = P.nx, ny = P.ny;
        const int quad = W.quad;
        const bool xpos = (quad == 0 || quad == 3);
        const bool ypos = (quad < 2);
        const T* __restrict__ st = sigma_t + P.field_off;

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

        for (int c = 0; c < P.nchunks; ++c) {
            const int i0 = c * TX;
            const int cols = min(TX, nx - i0);
            T yd[TX];
            if (strip == 0) {
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    yd[i] = (W.yin_off >= 0 && i < cols) ? inflow[W.yin_off + (int64_t)(i0 + i) * kWave + lane] : T(0);
            } else {
                wait_progress(prog_below, tag | (long long)(c + 1), A.ctl, A.spin_limit);
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    yd[i] = (i < cols) ? edge_below[(int64_t)(i0 + i) * kWave + lane] : T(0);
            }
            for (int r = 0; r < rows; ++r) {
                const int jj = j0 + r;
                const int j = ypos ? jj : ny - 1 - jj;
                const int64_t rowbase = (int64_t)j * nx;
                int cidx[TX];
                T stv[TX], Sv[TX], acc[TX];
                bool uni = true;
#pragma unroll
                for (int i = 0; i < TX; ++i) {
                    const int ii = i0 + (i < cols ? i : 0);
                    cidx[i] = (int)(rowbase + (xpos ? ii : nx - 1 - ii));
                    stv[i] = st[cidx[i]];
                    uni = uni && (stv[i] == stv[0]);
                }
#pragma unroll
                for (int i = 0; i < TX; ++i) {
                    if (ANG)
                        Sv[i] = Ap[(int64_t)cidx[i] * npad];
                    else
                        Sv[i] = Sp[cidx[i]];
                }
                T xf = xl[r];
                if (uni) {
                    const T rr = rcp_fast(stv[0] + kappa);
                    const T wr = w * rr, ar = a * rr, br = b * rr;
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        if (i < cols) {
                            const T v = fma(br, yd[i], fma(ar, xf, wr * Sv[i]));
                            if (DD) {
                                xf = fma(T(2), v, -xf);
                                yd[i] = fma(T(2), v, -yd[i]);
                            } else {
                                xf = v;
                                yd[i] = v;
                            }
                            acc[i] = v;
                        } else {
                            acc[i] = T(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        if (i < cols) {
                            const T rr = rcp_fast(stv[i] + kappa);
                            const T v = fma(b, yd[i], fma(a, xf, w * Sv[i])) * rr;
                            if (DD) {
                                xf = fma(T(2), v, -xf);
                                yd[i] = fma(T(2), v, -yd[i]);
                            } else {
                                xf = v;
                                yd[i] = v;
                            }
                            acc[i] = v;
                        } else {
                            acc[i] = T(0);
                        }
                    }
                }
                xl[r] = xf;
                // lanes of empty groups alias ordinate 0 of system sys[0]: they never store
                if (PSI == 1 && gslot >= 0) {
                    T* __restrict__ po = (T*)A.psi_out + SD.ang_off + ld.ord;
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        if (i < cols) po[(int64_t)cidx[i] * npad] = acc[i];
                } else if (PSI == 2 && gslot >= 0) {
                    __hip_bfloat16* __restrict__ po = (__hip_bfloat16*)A.psi_out + SD.ang_off + ld.ord;
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        if (i < cols) po[(int64_t)cidx[i] * npad] = __float2bfloat16((float)acc[i]);
                }
                group_sum<TX>(acc, L);
                if (gslot >= 0 && (lane & (L - 1)) == L - 1) {
#pragma unroll
                    for (int i = 0; i < TX; ++i)
                        if (i < cols) partp[cidx[i]] = acc[i];
                }
            }
            if (publish) {
#pragma unroll
                for (int i = 0; i < TX; ++i)
                    if (i < cols) edge_mine[(int64_t)(i0 + i) * kWave + lane] = yd[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (lane == 0)
                    __hip_atomic_store(prog_mine, tag | (long long)(c + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
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
        const double d = bitsd(c.dmax_bits), p = bitsd(c.pmax_bits);
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
        const int c1 = min(cells, blk.y + A.cells_per_block);
        for (int cell = blk.y + tid; cell < c1; cell += blockDim.x) {
            T v = T(0);
            for (int k = 0; k < SD.nslots; ++k) v += part[A.slot_off[A.slot_order[SD.slot_first + k]] + cell];
            const double d = fabs((double)v - (double)phi[cell]);
            dmax = fmax(dmax, d);
            pmax = fmax(pmax, fabs((double)v));
            phi[cell] = v;
            src[cell] = fma(ss[cell], v, q[cell]);
        }
    }
    __shared__ double sd[256], sp[256];
    sd[tid] = dmax;
    sp[tid] = pmax;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            sd[tid] = fmax(sd[tid], sd[tid + o]);
            sp[tid] = fmax(sp[tid], sp[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (run && A.mode == 0) {
            atomicMax(&A.sysctl[s].dmax_bits, dbits(sd[0]));  // non-negative doubles order as integers
            atomicMax(&A.sysctl[s].pmax_bits, dbits(sp[0]));
        }
        __threadfence();
        const int done = atomicAdd(&A.ctl->blocks_done, 1);
        if (done == (int)gridDim.x - 1) {
            __threadfence();
            if (A.mode == 0) finalize_iteration(A);
            A.ctl->blocks_done = 0;
            A.ctl->ticket = 0;
            A.ctl->epoch += 1;
            __threadfence();
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
    const int nblk_n = A.N / GN;
    const int bm = blockIdx.x / nblk_n, bn = blockIdx.x % nblk_n;
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
    if (tx == 8 && ty == 8) return launch_sweep_tile<T, 8, 8>(a, grid, dd, ang, psi, s);
    if (tx == 16 && ty == 8) return launch_sweep_tile<T, 16, 8>(a, grid, dd, ang, psi, s);
    if (tx == 16 && ty == 16) return launch_sweep_tile<T, 16, 16>(a, grid, dd, ang, psi, s);
    if (tx == 8 && ty == 4) return launch_sweep_tile<T, 8, 4>(a, grid, dd, ang, psi, s);
    if (tx == 32 && ty == 16) return launch_sweep_tile<T, 32, 16>(a, grid, dd, ang, psi, s);
    return hipErrorInvalidValue;
}

bool sweep_tile_supported(int tx, int ty)
{
    return (tx == 8 && ty == 8) || (tx == 16 && ty == 8) || (tx == 16 && ty == 16) || (tx == 8 && ty == 4) ||
           (tx == 32 && ty == 16);
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

// rom_slab.hip -- slab-geometry source iteration of librom (Sec. 4.1) on gfx950.
//
// The slab systems of a ROM ensemble are tiny (tens of grid points, a few ordinates) and
// independent, so each wavefront runs whole source iterations of 64 / L systems by itself: no
// grid-wide synchronization, no launches per iteration.  Lane r of a system carries the system's
// ordinates r, r + L, ... (at most KMAX).  The sweep advances all of them one grid point per step,
// the mu > 0 ordinates from x0 upwards and the mu < 0 ones from x1 downwards, so at step j every
// lane needs the same two cells (j - 1 and nx - j): their sigma_t and source are LDS broadcasts.
// The step's contributions w psi to phi at points j and nx - j are summed over the system's lanes
// with xor shuffles in a fixed order (deterministic) and added by the system's first lane.  After
// the sweep the system's lanes form the relative change, the convergence decision and the next
// source S = sigma_s phi + q in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rom_common.h"

namespace rom {

namespace {

template <typename T>
__device__ __forceinline__ T group_sum(T v, int L)
{
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double group_max(double v, int L)
{
    for (int off = 1; off < L; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace

// LDS per wavefront: S, phi (last iterate) and phi (running sum) per system, and the cell sigma_t.
size_t slab_lds_bytes(bool fp64, int nn, int L)
{
    const size_t esz = fp64 ? 8 : 4;
    return esz * ((size_t)(64 / L) * 3 * nn + (size_t)nn);
}

template <typename T, int KMAX>
__global__ __launch_bounds__(64) void slab_kernel(SlabArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int L = A.L, spw = 64 / L;
    const int g = lane / L, r = lane % L;
    const int sys = blockIdx.x * spw + g;
    const bool live = sys < A.nsys;
    const int sy = live ? sys : A.nsys - 1;  // idle lanes read a valid system, never write
    const int nn = A.nn, nx = nn - 1, n = A.n;
    T* S = (T*)smem + (size_t)g * 3 * nn;
    T* pold = S + nn;
    T* pnew = pold + nn;
    T* sigc = (T*)smem + (size_t)spw * 3 * nn;  // [nx] cell sigma_t, shared by the wave
    const T* __restrict__ st = (const T*)A.st;
    const T* __restrict__ ss = (const T*)A.ss;
    const T* __restrict__ q = (const T*)A.q;

    // this lane's ordinates: |mu| / dx and the weight signed by the direction (0: padding); the
    // entry values are re-read from global memory (L2) each iteration to spare registers
    T a[KMAX], ws[KMAX], psi[KMAX];
    const T* __restrict__ inflow = (const T*)A.inflow + (size_t)sy * n;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int o = r + k * L;
        a[k] = T(1);
        ws[k] = T(0);
        if (o < n) {
            const T m = ((const T*)A.mu)[(size_t)sy * n + o];
            const T wt = ((const T*)A.w)[(size_t)sy * n + o];
            a[k] = (m < T(0) ? -m : m) * T(A.inv_dx);
            ws[k] = m > T(0) ? wt : -wt;
        }
    }
    for (int i = r; i < nn; i += L) {
        S[i] = q[i];
        pold[i] = T(0);
        pnew[i] = T(0);
    }
    for (int i = lane; i < nx; i += 64) sigc[i] = T(0.5) * (st[i] + st[i + 1]);
    __syncthreads();

    int done = live ? 0 : 1;  // uniform over a system's lanes
    int iters = 0, state = 0;
    double rlast = 0.0;
    for (int it = 1; it <= A.max_iter; ++it) {
        if (__all(done)) break;
        // sweep: step j handles point j (mu > 0) and point nx - j (mu < 0)
        T pos = T(0), neg = T(0);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int o = r + k * L;
            psi[k] = o < n ? inflow[o] : T(0);
            if (ws[k] > T(0)) pos += ws[k] * psi[k];
            else neg -= ws[k] * psi[k];
        }
        pos = group_sum(pos, L);
        neg = group_sum(neg, L);
        if (r == 0 && !done) {
            pnew[0] += pos;
            pnew[nx] += neg;
        }
        for (int j = 1; j <= nx; ++j) {
            const int cp = j - 1, cn = nx - j;  // cells swept by the mu > 0 and mu < 0 ordinates
            const T hp = T(0.5) * sigc[cp], hn = T(0.5) * sigc[cn];
            const T sp = T(0.5) * (S[cp] + S[cp + 1]), sn = T(0.5) * (S[cn] + S[cn + 1]);
            pos = T(0);
            neg = T(0);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const bool up = ws[k] > T(0);
                const T h = up ? hp : hn;
                const T sb = up ? sp : sn;
                psi[k] = fma(a[k] - h, psi[k], sb) * rcp_fast(a[k] + h);
                if (up) pos += ws[k] * psi[k];
                else neg -= ws[k] * psi[k];
            }
            pos = group_sum(pos, L);
            neg = group_sum(neg, L);
            if (r == 0 && !done) {
                pnew[j] += pos;
                pnew[nx - j] += neg;
            }
        }
        __syncthreads();
        // relative change, decision, next source
        double dmax = 0.0, pmax = 0.0;
        for (int i = r; i < nn; i += L) {
            dmax = fmax(dmax, fabs((double)pnew[i] - (double)pold[i]));
            pmax = fmax(pmax, fabs((double)pnew[i]));
        }
        dmax = group_max(dmax, L);
        pmax = group_max(pmax, L);
        if (!done) {
            const double rel = pmax > 0.0 ? dmax / pmax : 0.0;
            iters = it;
            rlast = rel;
            if (!(dmax <= 1e300) || !(pmax <= 1e300)) state = 3;
            else if (rel <= A.tol) state = 1;
            else if (it >= A.max_iter) state = 2;
            for (int i = r; i < nn; i += L) {
                pold[i] = pnew[i];
                pnew[i] = T(0);
                S[i] = fma(ss[i], pold[i], q[i]);
            }
            if (state != 0) done = 1;
        }
        __syncthreads();
    }
    if (live) {
        T* out = (T*)A.phi + (size_t)sys * nn;
        for (int i = r; i < nn; i += L) out[i] = pold[i];
        if (r == 0) {
            A.iters[sys] = iters;
            A.state[sys] = state == 0 ? 2 : state;
            A.rfinal[sys] = rlast;
        }
    }
}

hipError_t launch_slab(const SlabArgs& a, bool fp64, int kmax, hipStream_t s)
{
    if (a.L < 1 || a.L > 64 || (a.L & (a.L - 1)) || a.nn < 2 || a.n < 1 || (long long)kmax * a.L < a.n)
        return hipErrorInvalidValue;
    const size_t lds = slab_lds_bytes(fp64, a.nn, a.L);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    const int spw = 64 / a.L;
    const int grid = (a.nsys + spw - 1) / spw;
#define ROM_SLAB_LAUNCH(T, K) hipLaunchKernelGGL((slab_kernel<T, K>), dim3(grid), dim3(64), lds, s, a)
    if (fp64) {
        if (kmax == 1) ROM_SLAB_LAUNCH(double, 1);
        else if (kmax == 4) ROM_SLAB_LAUNCH(double, 4);
        else if (kmax == 16) ROM_SLAB_LAUNCH(double, 16);
        else if (kmax == 64) ROM_SLAB_LAUNCH(double, 64);
        else return hipErrorInvalidValue;
    } else {
        if (kmax == 1) ROM_SLAB_LAUNCH(float, 1);
        else if (kmax == 4) ROM_SLAB_LAUNCH(float, 4);
        else if (kmax == 16) ROM_SLAB_LAUNCH(float, 16);
        else if (kmax == 64) ROM_SLAB_LAUNCH(float, 64);
        else return hipErrorInvalidValue;
    }
#undef ROM_SLAB_LAUNCH
    return hipGetLastError();
}

}  // namespace rom

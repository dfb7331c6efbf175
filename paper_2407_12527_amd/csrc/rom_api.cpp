// rom_api.cpp -- host runtime of librom: the C ABI of include/rom.h, argument validation, the
// solve plan (ordinate ingestion, lane packing, strip tickets, buffers), and the source-iteration,
// ensemble and batch drivers that replay captured HIP graphs of the per-iteration kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rom_device.h"
#include "rom_host.h"
#include "rom_kernels.h"

using namespace rom;

namespace {

// ------------------------------------------------------------------------------------ utilities
thread_local std::string g_create_error;

// Entry points that touch the device hold this process-wide lock for their whole duration: a
// first solve of a batch shape captures a HIP graph, and HIP fails a capture when another thread
// meanwhile issues work that would synchronize with it (a synchronous copy, a free).  Calls from
// different threads therefore run one at a time; recursive because entry points may nest.
std::recursive_mutex& api_mutex()
{
    static std::recursive_mutex m;
    return m;
}
#define ROM_API_LOCK std::lock_guard<std::recursive_mutex> rom_api_lock_(api_mutex())

// Device allocator of every handle and plan buffer: hipMalloc / hipFree unless the caller
// installed a hook with rom_set_allocator (the only process-wide state the boundary keeps).
struct AllocHook {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free)(void*, void*) = nullptr;
    void* ctx = nullptr;
};
AllocHook& alloc_hook()
{
    static AllocHook hook;
    return hook;
}

struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    // the hook that gave this block (NULL: hipMalloc); a block is returned to its own allocator
    // even when the hook has been changed since
    void (*freefn)(void*, void*) = nullptr;
    void* fctx = nullptr;
    bool view = false;  // a region of memory owned elsewhere (a plan placed in a caller's region)
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release()
    {
        if (p && !view) {
            if (freefn) {
                // hipFree waits for the device; a hook gets the same guarantee: no queued work
                // still uses the block when its allocator may hand it out again
                (void)hipDeviceSynchronize();
                freefn(p, fctx);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
        freefn = nullptr;
        fctx = nullptr;
        view = false;
    }
    void set_view(void* ptr, size_t n)
    {
        release();
        p = ptr;
        bytes = n;
        view = true;
    }
    hipError_t alloc(size_t n)
    {
        release();
        if (n == 0) n = 256;
        const AllocHook hook = alloc_hook();
        if (hook.alloc) {
            p = hook.alloc(n, hook.ctx);
            if (!p) return hipErrorOutOfMemory;
            if (((uintptr_t)p & 255) != 0) {  // kernels issue 16-byte loads from 256-byte-aligned pools
                hook.free(p, hook.ctx);
                p = nullptr;
                return hipErrorInvalidValue;
            }
            freefn = hook.free;
            fctx = hook.ctx;
            bytes = n;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        else p = nullptr;
        return e;
    }
    template <typename T>
    T* as() const { return (T*)p; }
};

struct Fail {
    int code;
    std::string msg;
};

#define HIPCHK(expr)                                                                                       \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            throw Fail{e_ == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE,                            \
                       std::string(#expr) + ": " + hipGetErrorString(e_)};                                \
    } while (0)

inline bool isfin(double x) { return std::isfinite(x); }

int quadrant_of(double c, double s)
{
    if (c >= 0.0 && s >= 0.0) return 0;
    if (c < 0.0 && s >= 0.0) return 1;
    if (c < 0.0 && s < 0.0) return 2;
    return 3;
}

template <typename T>
void upload(DevMem& d, const std::vector<T>& v)
{
    HIPCHK(d.alloc(v.size() * sizeof(T)));
    if (!v.empty()) HIPCHK(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Overwrite an existing allocation of exactly the same size (its address stays valid for a
// captured graph); stream-ordered after the work already queued on s.
template <typename T>
void rewrite(DevMem& d, const std::vector<T>& v, hipStream_t s)
{
    if (d.bytes < v.size() * sizeof(T) || (!v.empty() && !d.p)) throw Fail{ROM_E_STATE, "plan table size changed"};
    if (!v.empty()) HIPCHK(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

uint16_t f32_to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return uint16_t(u >> 16);
}

// Frequency of the device real-time clock read by wall_clock64(), in kHz (ticks per ms).
double wallclock_khz()
{
    // initialized once per process, thread-safe (function-local static)
    static const double khz = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0)
            return (double)v;
        return 100000.0;
    }();
    return khz;
}

// Real-time clock ticks a sweep's dependency wait may last before it gives up: 2 s.  A wait in a
// working sweep lasts microseconds; a timed-out one ends the solve with ROM_E_DEVICE.
long long wait_ticks() { return (long long)(2000.0 * wallclock_khz()); }

// Polls a dependency wait may make before it gives up: 2^24, or ROM_SPIN_LIMIT (read when a plan's
// launches are set up; tests force the time-out path with a tiny limit, and every kernel still
// exits normally).
int spin_limit()
{
    const char* e = std::getenv("ROM_SPIN_LIMIT");
    const long v = e ? std::strtol(e, nullptr, 10) : 0;
    return (v > 0 && v < (1L << 30)) ? (int)v : 1 << 24;
}

}  // namespace

// ------------------------------------------------------------------------------------ handle
struct Plan;
struct Arena;

struct rom_handle {
    rom_grid grid{};
    double dx = 0, dy = 0;
    int64_t cells = 0;
    std::vector<double> st, ss, q;
    std::vector<double> face[4];
    // ordinates in the caller's order
    int n = 0;
    std::vector<double> dirs, w;
    std::vector<double> ang[4];
    // scattering
    int scat = ROM_SCAT_ISO;    // kernel kind without flags
    bool scat_norm = false;     // ROM_SCAT_NORMALIZE: rows of P rescaled to unit weighted sum
    double g = 0.0;
    std::vector<double> Pdense;
    // execution
    hipStream_t user_stream = nullptr;
    hipStream_t own_stream = nullptr;
    int device = 0;
    uint64_t version = 1;  // bumps whenever ordinates, inflow or scattering change
    std::string err;
    std::unique_ptr<Plan> plan;
    uint64_t plan_version = 0;
    std::string plan_sig;
    // plans of the last ensemble and of the last batch led by this handle, kept for reuse
    std::unique_ptr<Plan> ens_plan, batch_plan;
    // host side of the plan placed in the preallocated scratch region (rom_sweep_noalloc), for
    // the handle's state `na_version` and precision `na_prec`
    std::unique_ptr<Plan> na_plan;
    std::unique_ptr<Arena> na_arena;
    uint64_t na_version = 0;
    int na_prec = -1;
    std::string ens_key, batch_key, batch_versions;
    uint64_t uid = next_uid();
    // autotuner choices of the batch shapes this handle led (key -> sweep, tile x, tile y, band,
    // rows, ordinates per lane), kept with the handle rather than process-wide
    std::map<std::string, std::array<int, 6>> tune_cache;
    // device-resident result of the last solve
    const void* res_dev = nullptr;
    bool res_fp64 = false;
    DevMem ens_mean, ens_m2, ens_var;

    static uint64_t next_uid()
    {
        static std::atomic<uint64_t> counter{0};
        return ++counter;
    }

    hipStream_t stream()
    {
        if (user_stream) return user_stream;
        if (!own_stream) HIPCHK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        return own_stream;
    }
    ~rom_handle();
};

int fail(rom_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

// ------------------------------------------------------------------------------------ plan
//
// A plan packs a list of systems (problem + ordinate set) onto wave-streams and owns every
// device buffer one solve needs.  Systems of one problem and quadrant share wave-streams; each
// system's ordinates of a quadrant occupy whole groups of L lanes (padding lanes carry w = 0).
struct SysInput {
    rom_handle* h;
    const double* dirs;
    const double* w;
    int n;
    bool use_angular;  // angular inflow of the handle applies (its own ordinate set)
};

// A caller-provided device region that a plan's buffers are carved from instead of being
// allocated: uploads are stream-ordered on `s` from host copies the plan keeps, and buffers that
// must start at zero are cleared by a fill kernel (no hipMemset, so the work can be captured).
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    hipStream_t s = nullptr;
};

struct Plan {
    Arena* arena = nullptr;                 // placement of the buffers (NULL: allocated)
    std::vector<std::vector<char>> keep;    // host sources of the arena uploads
    bool fp64 = false, dd = false, aniso = false;
    int nmom = 1;       // 4: linear-kernel moment sweep (three source planes, four partial planes)
    int mom_r = 0;      // linear kernel normalized somewhere in the batch: form phi~ separately
    int64_t src_len = 0;  // elements of the source pool (without its padding)
    int tx = 16, ty = 16;
    int band = 1;   // strips per sweep workgroup
    int L = 64;     // lanes per ordinate group
    int esz = 4;
    int nsys = 0, nws = 0, ntickets = 0, nslots = 0;
    int grid = 1;
    int max_iter = 0;
    std::vector<rom_handle*> handles;  // one per problem
    std::vector<ProblemDev> probs;
    std::vector<SystemDev> sys;
    std::vector<WaveStreamDev> ws;
    std::vector<LaneDev> lanes;
    std::vector<int2> tickets;
    std::vector<int64_t> slot_off;
    std::vector<int32_t> slot_order;
    std::vector<int64_t> slot_off_ord;  // slot_off in summation order
    std::vector<int2> cblocks;
    std::vector<std::vector<int>> user_of;  // per system: internal index -> caller index (-1 pad)
    std::vector<int> sys_n;                 // per system: real ordinate count
    std::vector<const double*> sys_w;       // per system: caller weights
    std::vector<int> npad_al;               // per system: padded stride of the anisotropic layout
    std::vector<std::array<int, 4>> qcount;  // per system: ordinates per quadrant
    int64_t inflow_len = 0;                 // elements of the weighted inflow table (0: vacuum)
    std::vector<double> h_inflow;           // host copies kept for stream-ordered rewrites
    std::vector<float> h_inflow32;
    std::vector<KmSys> h_kmsys;             // kernel-matrix jobs and their ordinate tables (host
    std::vector<double> h_kmord;            // copies kept until the stream-ordered uploads are done)
    std::vector<int32_t> h_kmuidx;
    std::vector<double> h_kmdense;
    int prog_count = 0;  // progress counters (64-bit words)
    int cells_per_block = 1024;
    int many_cpt = 0;  // many-slot combine: cells per thread (0: the few-slot combine)
    int vec = 0;       // many-slot combine with 16-byte loads
    // row-lane sweep
    int kind = ROM_SWEEP_STRIP;
    int dR = 16, dK = 1, dNB = 1;
    std::vector<DiagTaskDev> dtasks;
    DevMem d_dtasks;

    DevMem d_probs, d_sys, d_ws, d_lanes, d_tickets, d_slot_off, d_slot_order, d_slot_off_ord, d_cblocks;
    DevMem d_st, d_ss, d_q, d_src, d_phi, d_part, d_edge, d_inflow, d_prog, d_ctl, d_sysctl, d_rhist;
    DevMem d_ang, d_psi, d_Pt, d_uflags;
    DevMem d_kmsys, d_kmord, d_kmuidx, d_kmdense, d_kminv;  // kernel-matrix build inputs
    DevMem d_citems, d_cmap;  // batched contraction: per-system arguments, (system, block) map
    DevMem d_moff;            // ensemble moments: flux offsets of the first moff_n systems
    int moff_n = 0;
    int cmap_blocks = 0;
    std::vector<int64_t> pt_off;  // per system offset into d_Pt (elements)
    hipGraphExec_t gexec = nullptr;   // K iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec0 = nullptr;  // the initial state followed by K iterations (first replay)
    hipGraph_t graph0 = nullptr;
    // pinned host copy of the control block and the per-system states, read back after every
    // replay (a pageable destination would be staged through a bounce buffer, copy by copy)
    void* h_state = nullptr;
    size_t h_state_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // device time of a solve (created once per plan)
    int graph_iters = 0;
    int last_iters = 0;   // largest iteration count of the previous solve with this plan
    double graph_tol = 0.0;
    hipStream_t graph_stream = nullptr;

    ~Plan()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (gexec0) (void)hipGraphExecDestroy(gexec0);
        if (graph0) (void)hipGraphDestroy(graph0);
        if (h_state) (void)hipHostFree(h_state);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    // the sigma_t and source pools carry kPoolPad elements of padding on both sides
    char* st_ptr() const { return (char*)d_st.p + (size_t)kPoolPad * esz; }
    char* src_ptr() const { return (char*)d_src.p + (size_t)kPoolPad * esz; }

    DiagArgs diag_args(int mode_all) const
    {
        DiagArgs a{};
        a.tasks = d_dtasks.as<DiagTaskDev>();
        a.ords = d_lanes.as<LaneDev>();
        a.probs = d_probs.as<ProblemDev>();
        a.sys = d_sys.as<SystemDev>();
        a.tickets = d_tickets.as<int2>();
        a.ntickets = ntickets;
        a.spin_limit = spin_limit();
        a.wait_ticks = wait_ticks();
        a.mode_all = mode_all;
        a.edge = d_edge.p;
        a.prog = d_prog.as<long long>();
        a.sigma_t = st_ptr();
        a.src = src_ptr();
        a.part = d_part.p;
        a.slot_off = d_slot_off.as<int64_t>();
        a.inflow = d_inflow.p;
        a.ctl = d_ctl.as<Ctl>();
        a.sysctl = d_sysctl.as<SysCtl>();
        a.ang_src = d_ang.p;
        a.psi_out = d_psi.p;
        return a;
    }

    // one sweep of every running system, with the plan's kernel
    hipError_t launch_sweep_any(int mode_all, hipStream_t s) const
    {
        if (kind == ROM_SWEEP_DIAG) return launch_diag(diag_args(mode_all), grid, dNB, fp64, dR, dK, aniso, s);
        return launch_sweep(sweep_args(mode_all, 0), grid, fp64, tx, ty, dd, aniso, aniso ? (fp64 ? 1 : 2) : 0, L, nmom, s);
    }

    SweepArgs sweep_args(int mode_all, int psi_mode) const
    {
        SweepArgs a{};
        a.probs = d_probs.as<ProblemDev>();
        a.ws = d_ws.as<WaveStreamDev>();
        a.lanes = d_lanes.as<LaneDev>();
        a.sys = d_sys.as<SystemDev>();
        a.tickets = d_tickets.as<int2>();
        a.ntickets = ntickets;
        a.spin_limit = spin_limit();
        a.wait_ticks = wait_ticks();
        a.mode_all = mode_all;
        a.band = band;
        a.sigma_t = st_ptr();
        a.src = src_ptr();
        a.ang_src = d_ang.p;
        a.psi_out = d_psi.p;
        a.part = d_part.p;
        a.slot_off = d_slot_off.as<int64_t>();
        a.uflags = d_uflags.as<int32_t>();
        a.edge = d_edge.p;
        a.inflow = d_inflow.p;
        a.prog = d_prog.as<long long>();
        a.ctl = d_ctl.as<Ctl>();
        a.sysctl = d_sysctl.as<SysCtl>();
        a.mom_r = mom_r;
        (void)psi_mode;
        return a;
    }

    CombineArgs combine_args(int mode, double tol) const
    {
        CombineArgs c{};
        c.sys = d_sys.as<SystemDev>();
        c.probs = d_probs.as<ProblemDev>();
        c.slot_order = d_slot_order.as<int32_t>();
        c.slot_off = d_slot_off.as<int64_t>();
        c.slot_off_ord = d_slot_off_ord.as<int64_t>();
        c.blocks = d_cblocks.as<int2>();
        c.cells_per_block = cells_per_block;
        c.many_cpt = many_cpt;
        c.vec = vec;
        c.nsys = nsys;
        c.nmom = nmom;
        c.mom_r = mom_r;
        c.mode = mode;
        c.max_iter = max_iter;
        c.tol = tol;
        c.part = d_part.p;
        c.phi = d_phi.p;
        c.src = src_ptr();
        c.sigma_s = d_ss.p;
        c.q = d_q.p;
        c.sysctl = d_sysctl.as<SysCtl>();
        c.ctl = d_ctl.as<Ctl>();
        c.rhist = d_rhist.as<double>();
        return c;
    }
};

// Slab-geometry problem (Sec. 4.1): fields at the nx + 1 grid points, host copies.
struct rom_slab {
    int32_t nx = 0;
    double x0 = 0, x1 = 1;
    std::vector<double> st, ss, q;
    hipStream_t user_stream = nullptr;
    hipStream_t own_stream = nullptr;
    std::string err;
    hipStream_t stream()
    {
        if (user_stream) return user_stream;
        if (!own_stream) HIPCHK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        return own_stream;
    }
    ~rom_slab()
    {
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
};

rom_handle::~rom_handle()
{
    plan.reset();
    if (own_stream) (void)hipStreamDestroy(own_stream);
}

namespace {

// ---- placement of a plan's device buffers (allocated, or carved from the plan's arena)
void take(Plan& P, DevMem& d, size_t n)
{
    if (!P.arena) {
        HIPCHK(d.alloc(n));
        return;
    }
    if (n == 0) n = 256;
    const size_t off = (P.arena->used + 255) & ~size_t(255);
    if (off + n > P.arena->cap) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "problem needs more than the %zu bytes of the preallocated scratch region",
                      P.arena->cap);
        throw Fail{ROM_E_UNSUPPORTED, msg};
    }
    d.set_view(P.arena->base + off, n);
    P.arena->used = off + n;
}

template <typename T>
void put(Plan& P, DevMem& d, const std::vector<T>& v)
{
    if (!P.arena) {
        upload(d, v);
        return;
    }
    const size_t bytes = v.size() * sizeof(T);
    take(P, d, bytes);
    if (bytes == 0) return;
    P.keep.emplace_back((const char*)v.data(), (const char*)v.data() + bytes);
    HIPCHK(hipMemcpyAsync(d.p, P.keep.back().data(), bytes, hipMemcpyHostToDevice, P.arena->s));
}

void zero(Plan& P, void* p, size_t bytes)
{
    if (!P.arena) {
        HIPCHK(hipMemset(p, 0, bytes));
        return;
    }
    HIPCHK(launch_fill(p, (int64_t)(bytes / 4), false, 0.0, P.arena->s));  // every cleared buffer is 4-byte sized
}

// The vector-load many-slot combine is the default; ROM_VEC_COMBINE=0 selects the scalar one.
bool vec_combine_enabled()
{
    const char* e = std::getenv("ROM_VEC_COMBINE");
    return !(e && e[0] == '0');
}

int device_cus()
{
    // initialized once per process, thread-safe (function-local static)
    static const int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        return v;
    }();
    return cus;
}

void choose_tiles(const rom_si_opts& o, const std::vector<SysInput>& in, bool fp64, int& tx, int& ty)
{
    if (o.tile_x > 0 && o.tile_y > 0) {
        tx = o.tile_x;
        ty = o.tile_y;
        return;
    }
    // Heuristic: enough strips in flight to cover the GPU, chunks wide enough to amortise the
    // hand-off.  Double precision keeps 8 x 8 (register pressure).
    int64_t work = 0;
    int maxside = 0;
    for (auto& s : in) {
        work += (int64_t)s.h->cells * s.n;
        maxside = std::max(maxside, std::max(s.h->grid.nx, s.h->grid.ny));
    }
    if (fp64) {
        tx = 8;
        ty = 8;
        return;
    }
    if (in.size() == 1 && maxside <= 512) {
        tx = 8;
        ty = 4;
    } else if (in.size() == 1) {
        tx = 8;
        ty = 8;
    } else {
        tx = 16;
        ty = 16;
    }
}

// Build every table and buffer of a plan for the given systems.
// True when a problem of the batch has any boundary inflow (isotropic, or angular for a system
// that takes the handle's angular inflow).
bool has_inflow(rom_handle* h, const std::vector<SysInput>& in)
{
    for (int f = 0; f < 4; ++f)
        if (!h->face[f].empty()) return true;
    for (auto& s : in)
        if (s.h == h && s.use_angular)
            for (int f = 0; f < 4; ++f)
                if (!h->ang[f].empty()) return true;
    return false;
}

// Row-lane sweep: unweighted inflow of every task ordinate on its entry faces in sweep order:
// x-face [row][NO], y-face [NO][pitch] (column runs per ordinate).
std::vector<double> diag_inflow_table(const Plan& P, const std::vector<SysInput>& in)
{
    const int NO = (kWave / P.dR) * P.dK;
    std::vector<double> inf(P.inflow_len, 0.0);
    for (const DiagTaskDev& t : P.dtasks) {
        if (t.xin_off < 0) continue;
        rom_handle* h = P.handles[t.prob];
        const int nx = h->grid.nx, ny = h->grid.ny;
        const bool xpos = (t.quad == 0 || t.quad == 3), ypos = (t.quad < 2);
        const int fx = xpos ? ROM_FACE_LEFT : ROM_FACE_RIGHT;
        const int fy = ypos ? ROM_FACE_BOTTOM : ROM_FACE_TOP;
        const bool angok = in[t.sys].use_angular;
        for (int k = 0; k < NO; ++k) {
            const LaneDev& ld = P.lanes[t.ord_off + k];
            const int u = P.user_of[t.sys][ld.ord];
            if (u < 0) continue;
            for (int jj = 0; jj < ny; ++jj) {
                const int j = ypos ? jj : ny - 1 - jj;
                double v = 0.0;
                if (angok && !h->ang[fx].empty()) v = h->ang[fx][(size_t)u * ny + j];
                else if (!h->face[fx].empty()) v = h->face[fx][j];
                inf[t.xin_off + (int64_t)jj * NO + k] = v;
            }
            for (int ii = 0; ii < nx; ++ii) {
                const int i = xpos ? ii : nx - 1 - ii;
                double v = 0.0;
                if (angok && !h->ang[fy].empty()) v = h->ang[fy][(size_t)u * nx + i];
                else if (!h->face[fy].empty()) v = h->face[fy][i];
                inf[t.yin_off + (int64_t)k * diag_pitch(nx) + ii] = v;
            }
        }
    }
    return inf;
}

// Boundary inflow of every wave-stream lane in sweep order, scaled by the lane's weight.
std::vector<double> inflow_table(const Plan& P, const std::vector<SysInput>& in)
{
    std::vector<double> inf(P.inflow_len, 0.0);
    for (int k = 0; k < P.nws; ++k) {
        const WaveStreamDev& W = P.ws[k];
        if (W.xin_off < 0) continue;
        rom_handle* h = P.handles[W.prob];
        const int nx = h->grid.nx, ny = h->grid.ny;
        const bool xpos = (W.quad == 0 || W.quad == 3), ypos = (W.quad < 2);
        const int fx = xpos ? ROM_FACE_LEFT : ROM_FACE_RIGHT;
        const int fy = ypos ? ROM_FACE_BOTTOM : ROM_FACE_TOP;
        for (int lane = 0; lane < kWave; ++lane) {
            const int gi = lane / W.L;
            const int s = W.sys[gi];
            if (s < 0) continue;
            const LaneDev& ld = P.lanes[(size_t)k * kWave + lane];
            const int u = P.user_of[s][ld.ord];
            if (u < 0) continue;
            const bool angok = in[s].use_angular;
            for (int jj = 0; jj < ny; ++jj) {
                const int j = ypos ? jj : ny - 1 - jj;
                double v = 0.0;
                if (angok && !h->ang[fx].empty()) v = h->ang[fx][(size_t)u * ny + j];
                else if (!h->face[fx].empty()) v = h->face[fx][j];
                inf[W.xin_off + (int64_t)jj * kWave + lane] = ld.w * v;
            }
            for (int ii = 0; ii < nx; ++ii) {
                const int i = xpos ? ii : nx - 1 - ii;
                double v = 0.0;
                if (angok && !h->ang[fy].empty()) v = h->ang[fy][(size_t)u * nx + i];
                else if (!h->face[fy].empty()) v = h->face[fy][i];
                inf[W.yin_off + (int64_t)ii * kWave + lane] = ld.w * v;
            }
        }
    }
    return inf;
}

// Scattering mode of a handle: 0 isotropic (source from phi), 1 linear kernel (rank-3 moment
// contraction inside the sweep), 2 dense contraction (HG or the caller's P).
int scat_mode(const rom_handle* h)
{
    if (h->scat == ROM_SCAT_ISO) return 0;
    if (h->scat == ROM_SCAT_LINEAR) return 1;
    return 2;
}

// Plan-structure key of a handle's scattering: the mode and whether a linear kernel is normalized.
int scat_sig(const rom_handle* h) { return scat_mode(h) + ((scat_mode(h) == 1 && h->scat_norm) ? 8 : 0); }

// 1 / r for every caller ordinate of a normalized linear-kernel system: the folded kernel
// 1 + g (c c' + s s') of eq. (2.1) has the weighted row sums
// r_l' = sum_l w_l (1 + g (c_l' c_l + s_l' s_l)) = sum w + g (c_l' sum w c + s_l' sum w s).
// Empty when the kernel is not normalized (r = 1).
std::vector<double> linear_inv_r(const rom_handle* h, const SysInput& si)
{
    std::vector<double> ir;
    if (h->scat != ROM_SCAT_LINEAR || !h->scat_norm) return ir;
    double sw = 0.0, swc = 0.0, sws = 0.0;
    for (int l = 0; l < si.n; ++l) {
        sw += si.w[l];
        swc += si.w[l] * si.dirs[3 * l];
        sws += si.w[l] * si.dirs[3 * l + 1];
    }
    ir.resize(si.n);
    for (int l = 0; l < si.n; ++l) {
        const double r = sw + h->g * (si.dirs[3 * l] * swc + si.dirs[3 * l + 1] * sws);
        if (!(r > 0.0)) throw Fail{ROM_E_DOMAIN, "normalized linear kernel: a row sum is not positive"};
        ir[l] = 1.0 / r;
    }
    return ir;
}

// Lane-table entry of caller ordinate u of system si (u < 0: a padding lane, all zero).
void fill_lane(LaneDev& ld, const rom_handle* h, const SysInput& si, int u, const std::vector<double>& inv_r)
{
    const int32_t ord = ld.ord;
    ld = LaneDev{};
    ld.ord = ord;
    if (u < 0) return;
    const double c = si.dirs[3 * u], sn = si.dirs[3 * u + 1];
    ld.a = std::fabs(c) / h->dx;
    ld.b = std::fabs(sn) / h->dy;
    ld.w = si.w[u];
    ld.c = c;
    ld.s = sn;
    const double ir = inv_r.empty() ? 1.0 : inv_r[u];
    ld.m1 = c * ir;
    ld.m2 = sn * ir;
    ld.m3 = ir;
}

// smode: scattering mode of every system of the batch (scat_mode); 2 also for a per-ordinate
// source of a single sweep.
void build_plan(Plan& P, const std::vector<SysInput>& in, const rom_si_opts& o, int smode, int max_iter,
                bool psi_out = false)
{
    const bool aniso = smode == 2;
    P.fp64 = o.precision == ROM_PREC_FP64;
    P.dd = o.scheme == ROM_SCHEME_DD;
    P.aniso = aniso;
    P.nmom = smode == 1 ? 4 : 1;
    P.mom_r = 0;
    if (smode == 1)
        for (auto& si : in)
            if (si.h->scat_norm) P.mom_r = 1;
    P.esz = P.fp64 ? 8 : 4;
    P.max_iter = max_iter;
    P.kind = o.sweep == ROM_SWEEP_DIAG ? ROM_SWEEP_DIAG : ROM_SWEEP_STRIP;
    if (P.kind == ROM_SWEEP_DIAG) {
        if (psi_out || P.dd || P.nmom != 1 || (aniso && (P.fp64 || max_iter == 0)))
            throw Fail{ROM_E_UNSUPPORTED,
                       "the row-lane sweep takes the step scheme, isotropic sources or (FP32 source iteration) a dense "
                       "kernel's per-ordinate sources, and no angular-flux output"};
        P.dR = o.diag_rows > 0 ? o.diag_rows : 16;
        P.dK = o.diag_k > 0 ? o.diag_k : 1;
        if (!diag_supported(P.fp64, P.dR, P.dK)) throw Fail{ROM_E_ARG, "unsupported row-lane sweep shape"};
    }
    choose_tiles(o, in, P.fp64, P.tx, P.ty);
    if (!(P.fp64 ? sweep_tile_supported_fp64(P.tx, P.ty) : sweep_tile_supported(P.tx, P.ty)))
        throw Fail{ROM_E_ARG, P.fp64 ? "FP64 sweeps support tiles 8x4 and 8x8" : "unsupported tile shape"};
    const int TX = P.tx, TY = P.ty;

    // problems = distinct handles, in first-appearance order
    std::map<rom_handle*, int> pidx;
    for (auto& s : in)
        if (!pidx.count(s.h)) {
            pidx[s.h] = (int)P.handles.size();
            P.handles.push_back(s.h);
        }
    const int nprob = (int)P.handles.size();
    std::vector<int64_t> field_off(nprob);
    int64_t fsum = 0;
    for (int p = 0; p < nprob; ++p) {
        rom_handle* h = P.handles[p];
        ProblemDev pd{};
        pd.nx = h->grid.nx;
        pd.ny = h->grid.ny;
        pd.nchunks = (pd.nx + TX - 1) / TX;
        pd.nstrips = (pd.ny + TY - 1) / TY;
        pd.field_off = fsum;
        field_off[p] = fsum;
        fsum += h->cells;
        P.probs.push_back(pd);
    }

    // row-uniformity masks: bit r of (quadrant, strip, chunk) is set when sigma_t takes a single
    // value on the chunk's row r, so the sweep can take one reciprocal for the whole row
    std::vector<int32_t> uflags;
    for (int p = 0; p < nprob && P.kind == ROM_SWEEP_STRIP; ++p) {
        rom_handle* h = P.handles[p];
        ProblemDev& pd = P.probs[p];
        pd.uflag_off = (int64_t)uflags.size();
        const int nx = pd.nx, ny = pd.ny;
        for (int quad = 0; quad < 4; ++quad) {
            const bool xpos = (quad == 0 || quad == 3), ypos = (quad < 2);
            for (int st = 0; st < pd.nstrips; ++st) {
                for (int c = 0; c < pd.nchunks; ++c) {
                    int32_t mask = 0;
                    for (int r = 0; r < TY; ++r) {
                        const int jj = st * TY + r;
                        if (jj >= ny) break;
                        const int j = ypos ? jj : ny - 1 - jj;
                        bool uni = true;
                        double v0 = 0.0;
                        for (int i = 0; i < TX; ++i) {
                            const int ii = c * TX + i;
                            if (ii >= nx) break;
                            const double v = h->st[(size_t)j * nx + (xpos ? ii : nx - 1 - ii)];
                            if (i == 0) v0 = v;
                            else if (v != v0) uni = false;
                        }
                        if (uni) mask |= 1 << r;
                    }
                    uflags.push_back(mask);
                }
            }
        }
    }

    // lanes per group: the smallest of 16/32/64 covering the largest per-quadrant ordinate count
    // of the batch (64 for angular-flux output and for a single sweep with per-ordinate sources)
    struct QuadList {
        std::vector<int> idx[4];
    };
    std::vector<QuadList> ql(in.size());
    int Lb = (psi_out || (aniso && max_iter == 0)) ? 64 : 16;
    P.qcount.assign(in.size(), {0, 0, 0, 0});
    for (size_t k = 0; k < in.size(); ++k) {
        for (int l = 0; l < in[k].n; ++l) ql[k].idx[quadrant_of(in[k].dirs[3 * l], in[k].dirs[3 * l + 1])].push_back(l);
        for (int q = 0; q < 4; ++q) {
            const int m = (int)ql[k].idx[q].size();
            P.qcount[k][q] = m;
            while (Lb < 64 && Lb < m) Lb *= 2;
        }
    }
    P.L = Lb;
    std::vector<int> Lp(nprob, Lb);
    if (P.kind == ROM_SWEEP_STRIP) {
        // strips per workgroup: a band long enough that most hand-offs stay in LDS
        int maxstrips = 1;
        for (auto& si : in) maxstrips = std::max(maxstrips, (si.h->grid.ny + TY - 1) / TY);
        P.band = o.band > 0 ? o.band : std::min(kMaxBand, maxstrips);
        // when choosing automatically, keep two workgroups per CU (160 KiB of LDS): longer bands
        // keep more strip hand-offs in LDS, but a band that leaves one workgroup per CU measured
        // slower (512^2, 32-lane groups: band 8 at 82 KiB 908 us per sweep against 871 us at
        // band 7, two ring slots per boundary)
        while (o.band == 0 && P.band > 1 && sweep_lds_bytes(P.fp64, TX, TY, aniso, P.L, P.band, P.nmom) > 80 * 1024) --P.band;
        if (sweep_lds_bytes(P.fp64, TX, TY, aniso, P.L, P.band, P.nmom) > 160 * 1024)
            throw Fail{ROM_E_ARG, "band too large for this tile shape (LDS)"};
    }


    // systems: internal (quadrant-grouped, padded) ordinate order
    P.nsys = (int)in.size();
    P.sys.resize(P.nsys);
    P.user_of.resize(P.nsys);
    P.sys_n.resize(P.nsys);
    P.sys_w.resize(P.nsys);
    P.npad_al.resize(P.nsys);
    struct Group {
        int sys, quad, first;  // first internal index
        int count;             // real ordinates in the group
    };
    std::vector<std::vector<Group>> groups_pq(nprob * 4);
    int64_t phi_sum = 0, ang_sum = 0, src_sum = 0;
    for (int s = 0; s < P.nsys; ++s) {
        const int p = pidx[in[s].h];
        const int L = Lp[p];
        std::vector<int>& uo = P.user_of[s];
        for (int q = 0; q < 4; ++q) {
            const auto& list = ql[s].idx[q];
            for (size_t b = 0; b < list.size(); b += L) {
                Group g{s, q, (int)uo.size(), (int)std::min<size_t>(L, list.size() - b)};
                groups_pq[p * 4 + q].push_back(g);
                for (int k = 0; k < L; ++k) uo.push_back(b + k < list.size() ? list[b + k] : -1);
            }
        }
        const int npad = (int)uo.size();
        const int al = aniso ? ((npad + 127) / 128) * 128 : npad;
        P.npad_al[s] = al;
        SystemDev& sd = P.sys[s];
        sd.prob = p;
        sd.npad = al;
        sd.phi_off = phi_sum;
        sd.src_off = src_sum;
        sd.ang_off = ang_sum;
        sd.g = scat_mode(in[s].h) == 1 ? in[s].h->g : 0.0;
        phi_sum += in[s].h->cells;
        src_sum += in[s].h->cells * (P.nmom == 4 ? 3 : 1);
        if (aniso) ang_sum += in[s].h->cells * (int64_t)al;
        P.sys_n[s] = in[s].n;
        P.sys_w[s] = in[s].w;
    }

    // wave-streams (strip sweep) or tasks (row-lane sweep), slots
    int64_t part_sum = 0, edge_sum = 0, inflow_sum = 0;
    int prog_sum = 0;
    std::vector<std::vector<int>> sys_slots(P.nsys);
    if (P.kind == ROM_SWEEP_DIAG) {
        const int R = P.dR, K = P.dK, NO = (kWave / R) * K;
        int maxblocks = 1;
        for (auto& pd : P.probs) maxblocks = std::max(maxblocks, (pd.ny + R - 1) / R);
        const int nbmax = diag_max_nb(P.fp64, K, aniso);
        int ntask = 0;
        for (int sy = 0; sy < P.nsys; ++sy)
            for (int q = 0; q < 4; ++q) ntask += ((int)ql[sy].idx[q].size() + NO - 1) / NO;
        if (o.band > 0) {
            P.dNB = std::min(o.band, nbmax);
        } else {
            // tall bands keep hand-offs in LDS; shorter ones put more workgroups on the CUs
            P.dNB = std::min(maxblocks, nbmax);
            while (P.dNB > 2 && (int64_t)ntask * ((maxblocks + P.dNB - 1) / P.dNB) < 2 * device_cus()) P.dNB /= 2;
        }
        if (diag_lds_bytes(P.fp64, R, K, P.dNB) > 64 * 1024) throw Fail{ROM_E_UNSUPPORTED, "row-lane sweep: LDS"};
        for (int sy = 0; sy < P.nsys; ++sy) {
            const int p = P.sys[sy].prob;
            rom_handle* h = P.handles[p];
            const bool inflow = has_inflow(h, in);
            std::vector<int>& uo = P.user_of[sy];
            uo.clear();
            for (int q = 0; q < 4; ++q) {
                const auto& list = ql[sy].idx[q];
                for (size_t b0 = 0; b0 < list.size(); b0 += NO) {
                    DiagTaskDev t{};
                    t.sys = sy;
                    t.prob = p;
                    t.quad = q;
                    t.slot = P.nslots;
                    t.ord_off = (int64_t)P.lanes.size();
                    t.xin_off = t.yin_off = -1;
                    const int pitch = diag_pitch(h->grid.nx);
                    if (inflow) {
                        t.xin_off = inflow_sum;
                        inflow_sum += (int64_t)h->grid.ny * NO;
                        inflow_sum = (inflow_sum + 7) / 8 * 8;  // y-face runs are 16-byte vectors
                        t.yin_off = inflow_sum;
                        inflow_sum += (int64_t)pitch * NO;
                    }
                    const int nbands = ((h->grid.ny + R - 1) / R + P.dNB - 1) / P.dNB;
                    t.edge_off = edge_sum;
                    edge_sum += (int64_t)nbands * pitch * NO;
                    t.prog_off = prog_sum;
                    prog_sum += nbands;
                    for (int k = 0; k < NO; ++k) {
                        LaneDev ld{};
                        ld.ord = (int)uo.size();
                        const int u = b0 + k < list.size() ? list[b0 + k] : -1;
                        uo.push_back(u);
                        fill_lane(ld, h, in[sy], u, {});
                        P.lanes.push_back(ld);
                    }
                    P.slot_off.push_back(part_sum);
                    part_sum += h->cells;
                    sys_slots[sy].push_back(P.nslots);
                    ++P.nslots;
                    P.dtasks.push_back(t);
                }
            }
            P.npad_al[sy] = P.sys[sy].npad = (int)uo.size();
        }
        if (aniso) {
            // the dense-kernel layout [cells][npad] in the row-lane order, padded for the GEMM tiles
            ang_sum = 0;
            for (int sy = 0; sy < P.nsys; ++sy) {
                const int al = ((int)P.user_of[sy].size() + 127) / 128 * 128;
                P.npad_al[sy] = P.sys[sy].npad = al;
                P.sys[sy].ang_off = ang_sum;
                ang_sum += P.handles[P.sys[sy].prob]->cells * (int64_t)al;
            }
        }
    }
    std::vector<std::vector<double>> inv_r(P.nsys);
    for (int s = 0; s < P.nsys; ++s) inv_r[s] = linear_inv_r(in[s].h, in[s]);
    for (int p = 0; p < nprob && P.kind == ROM_SWEEP_STRIP; ++p) {
        rom_handle* h = P.handles[p];
        const int L = Lp[p], G = 64 / L;
        const ProblemDev& pd = P.probs[p];
        bool vacuum = true;
        for (int f = 0; f < 4; ++f)
            if (!h->face[f].empty()) vacuum = false;
        for (auto& s : in)
            if (s.h == h && s.use_angular)
                for (int f = 0; f < 4; ++f)
                    if (!h->ang[f].empty()) vacuum = false;
        for (int q = 0; q < 4; ++q) {
            auto& gl = groups_pq[p * 4 + q];
            for (size_t g0 = 0; g0 < gl.size(); g0 += G) {
                WaveStreamDev W{};
                W.prob = p;
                W.quad = q;
                W.L = L;
                const int nbands = (pd.nstrips + P.band - 1) / P.band;
                W.prog_off = prog_sum;
                prog_sum += nbands;
                W.edge_off = edge_sum;
                edge_sum += (int64_t)nbands * pd.nx * kWave;
                W.xin_off = W.yin_off = -1;
                if (!vacuum) {
                    W.xin_off = inflow_sum;
                    inflow_sum += (int64_t)pd.ny * kWave;
                    W.yin_off = inflow_sum;
                    inflow_sum += (int64_t)pd.nx * kWave;
                }
                for (int k = 0; k < kMaxGroups; ++k) {
                    W.sys[k] = -1;
                    W.slot[k] = -1;
                }
                const int wsi = (int)P.ws.size();
                for (int k = 0; k < G; ++k) {
                    LaneDev pad{};
                    if (g0 + k < gl.size()) {
                        const Group& gr = gl[g0 + k];
                        W.sys[k] = gr.sys;
                        W.slot[k] = P.nslots;
                        P.slot_off.push_back(part_sum);
                        part_sum += h->cells * P.nmom;  // one partial plane per moment
                        sys_slots[gr.sys].push_back(P.nslots);
                        ++P.nslots;
                        const SysInput& si = in[gr.sys];
                        for (int l = 0; l < L; ++l) {
                            LaneDev ld{};
                            ld.ord = gr.first + l;
                            fill_lane(ld, h, si, P.user_of[gr.sys][gr.first + l], inv_r[gr.sys]);
                            P.lanes.push_back(ld);
                        }
                    } else {
                        for (int l = 0; l < L; ++l) P.lanes.push_back(pad);
                    }
                }
                (void)wsi;
                P.ws.push_back(W);
            }
        }
    }
    P.nws = (int)P.ws.size();
    // fixed summation order of each system's partial fluxes: quadrant-major, block order
    for (int s = 0; s < P.nsys; ++s) {
        P.sys[s].slot_first = (int)P.slot_order.size();
        P.sys[s].nslots = (int)sys_slots[s].size();
        std::vector<std::pair<int, int>> key;
        for (int sl : sys_slots[s]) key.push_back({sl, sl});
        std::sort(key.begin(), key.end());
        for (auto& kv : key) P.slot_order.push_back(kv.second);
    }
    // tickets: (wave-stream, band), band-major, so every band's producer precedes it
    int maxbands = 0;
    for (auto& pd : P.probs) maxbands = std::max(maxbands, (pd.nstrips + P.band - 1) / P.band);
    for (int bd = 0; bd < maxbands; ++bd)
        for (int k = 0; k < P.nws; ++k)
            if (bd < (P.probs[P.ws[k].prob].nstrips + P.band - 1) / P.band) P.tickets.push_back(make_int2(k, bd));
    P.ntickets = (int)P.tickets.size();
    P.grid = std::max(1, std::min(P.ntickets, device_cus() * 4));
    if (P.kind == ROM_SWEEP_DIAG) {
        // (task, band) tickets, band-major: the band below always holds an earlier ticket
        P.tickets.clear();
        int maxb = 0;
        std::vector<int> nb_of(P.dtasks.size());
        for (size_t k = 0; k < P.dtasks.size(); ++k) {
            const int ny = P.probs[P.dtasks[k].prob].ny;
            nb_of[k] = ((ny + P.dR - 1) / P.dR + P.dNB - 1) / P.dNB;
            maxb = std::max(maxb, nb_of[k]);
        }
        for (int bd = 0; bd < maxb; ++bd)
            for (size_t k = 0; k < P.dtasks.size(); ++k)
                if (bd < nb_of[k]) P.tickets.push_back(make_int2((int)k, bd));
        P.ntickets = (int)P.tickets.size();
        P.grid = std::max(1, std::min(P.ntickets, device_cus() * std::max(1, kDiagMaxWaves / P.dNB)));
    }
    // combine blocks: with few slots per system, about 512 blocks per launch (each thread keeps
    // 4 cells in flight); with many (the row-lane sweep's one slot per task), tiles of 64 * CPT
    // cells whose four waves split the slot list, about four blocks per CU
    {
        int64_t tot = 0;
        int maxslots = 0;
        for (auto& si : in) tot += si.h->cells;
        for (auto& sd : P.sys) maxslots = std::max(maxslots, sd.nslots);
        P.many_cpt = 0;
        P.vec = 0;
        // 16-byte loads when every partial plane starts and ends on a 16-byte boundary
        const int V = P.fp64 ? 2 : 4;
        bool aligned = true;
        for (auto& si : in) aligned = aligned && si.h->cells % V == 0;
        if (maxslots > 8 && P.nmom == 1 && aligned && vec_combine_enabled()) {
            P.vec = maxslots > 64 ? 3 : 1;  // 8 waves per block above 64 slots
            P.cells_per_block = 64 * V;
        } else if (P.nmom == 1 && aligned && vec_combine_enabled()) {
            P.vec = 2;  // few slots: one thread sums all slots of 16 bytes of cells, 4 tiles
            P.cells_per_block = 4 * 256 * V;
        } else if (maxslots > 8 && P.nmom == 1) {
            P.many_cpt = 1;
            while (P.many_cpt < 8 && tot / (64 * 2 * P.many_cpt) > 4 * device_cus()) P.many_cpt *= 2;
            P.cells_per_block = 64 * P.many_cpt;
        } else {
            int64_t cpb = (tot / 512 + 1023) / 1024 * 1024;
            P.cells_per_block = (int)std::max<int64_t>(1024, std::min<int64_t>(cpb, 16384));
        }
    }
    for (int s = 0; s < P.nsys; ++s)
        for (int64_t c0 = 0; c0 < in[s].h->cells; c0 += P.cells_per_block) P.cblocks.push_back(make_int2(s, (int)c0));

    // ---- device buffers
    put(P, P.d_probs, P.probs);
    put(P, P.d_sys, P.sys);
    put(P, P.d_ws, P.ws);
    put(P, P.d_lanes, P.lanes);
    put(P, P.d_tickets, P.tickets);
    put(P, P.d_slot_off, P.slot_off);
    put(P, P.d_slot_order, P.slot_order);
    P.slot_off_ord.resize(P.slot_order.size());
    for (size_t i = 0; i < P.slot_order.size(); ++i) P.slot_off_ord[i] = P.slot_off[P.slot_order[i]];
    put(P, P.d_slot_off_ord, P.slot_off_ord);
    put(P, P.d_cblocks, P.cblocks);
    put(P, P.d_uflags, uflags);
    put(P, P.d_dtasks, P.dtasks);

    auto cast_upload = [&](DevMem& d, const std::vector<double>& v) {
        if (P.fp64) {
            put(P, d, v);
        } else {
            std::vector<float> f(v.begin(), v.end());
            put(P, d, f);
        }
    };
    // A single sweep placed in a caller's region takes its source and scalar flux from the
    // caller and forms no next source: no sigma_s, q, source or flux pools of its own.
    const bool caller_io = P.arena && max_iter == 0;
    std::vector<double> st(fsum), ss(fsum), qv(fsum);
    for (int p = 0; p < nprob; ++p) {
        rom_handle* h = P.handles[p];
        std::copy(h->st.begin(), h->st.end(), st.begin() + field_off[p]);
        std::copy(h->ss.begin(), h->ss.end(), ss.begin() + field_off[p]);
        std::copy(h->q.begin(), h->q.end(), qv.begin() + field_off[p]);
    }
    {
        std::vector<double> padded(fsum + 2 * kPoolPad, 1.0);  // padding: a harmless positive sigma_t
        std::copy(st.begin(), st.end(), padded.begin() + kPoolPad);
        cast_upload(P.d_st, padded);
    }
    if (!caller_io) {
        cast_upload(P.d_ss, ss);
        cast_upload(P.d_q, qv);
    }

    // inflow in sweep order, scaled by the lane weight
    P.inflow_len = inflow_sum;
    if (inflow_sum > 0) {
        const std::vector<double> inf = P.kind == ROM_SWEEP_DIAG ? diag_inflow_table(P, in) : inflow_table(P, in);
        cast_upload(P.d_inflow, inf);
    } else {
        take(P, P.d_inflow, 256);
    }

    P.src_len = src_sum;
    if (!caller_io) {
        take(P, P.d_src, (src_sum + 2 * kPoolPad) * P.esz);
        zero(P, P.d_src.p, (src_sum + 2 * kPoolPad) * P.esz);
        take(P, P.d_phi, phi_sum * P.esz);
    }
    take(P, P.d_part, std::max<int64_t>(part_sum, 1) * P.esz);
    take(P, P.d_edge, std::max<int64_t>(edge_sum, 1) * P.esz);
    P.prog_count = std::max(prog_sum, 1);
    take(P, P.d_prog, P.prog_count * sizeof(long long));
    zero(P, P.d_prog.p, P.prog_count * sizeof(long long));
    // the control block and the per-system states in one block (one readback per graph replay)
    const size_t sc_off = (sizeof(Ctl) + 255) / 256 * 256;
    take(P, P.d_ctl, sc_off + P.nsys * sizeof(SysCtl));
    zero(P, P.d_ctl.p, sc_off + P.nsys * sizeof(SysCtl));
    P.d_sysctl.set_view((char*)P.d_ctl.p + sc_off, P.nsys * sizeof(SysCtl));
    if (max_iter > 0) take(P, P.d_rhist, (size_t)P.nsys * max_iter * sizeof(double));
    if (aniso) {
        take(P, P.d_ang, std::max<int64_t>(ang_sum, 1) * P.esz);
        take(P, P.d_psi, std::max<int64_t>(ang_sum, 1) * (P.fp64 ? 8 : 2));
    }
}

// P^T in internal order for every system: Bt[n][k] = P(u_k, u_n) / r_k, zero on padding, built on
// the device (launch_kernel_matrix) from the ordinate tables uploaded here (32 bytes per ordinate;
// the caller's dense kernel as well for ROM_SCAT_DENSE), stream-ordered on s.  The first call of a
// plan places the buffers; later calls (new ordinates of the same structure) rewrite them in place.
void build_kernel_matrices(Plan& P, const std::vector<SysInput>& in, hipStream_t s)
{
    const bool first = !P.d_kmsys.p;
    int64_t total = 0, entries = 0, dtotal = 0;
    int max_al = 0;
    P.pt_off.resize(P.nsys);
    P.h_kmsys.assign(P.nsys, KmSys{});
    for (int k = 0; k < P.nsys; ++k) {
        rom_handle* h = in[k].h;
        KmSys& ks = P.h_kmsys[k];
        ks.ord_off = entries;
        ks.pt_off = P.pt_off[k] = total;
        ks.npad = (int)P.user_of[k].size();
        ks.al = P.npad_al[k];
        ks.n = in[k].n;
        ks.kind = h->scat;
        ks.norm = h->scat_norm ? 1 : 0;
        ks.g = h->g;
        ks.dense_off = h->scat == ROM_SCAT_DENSE ? dtotal : 0;
        if (h->scat == ROM_SCAT_DENSE) dtotal += (int64_t)in[k].n * in[k].n;
        entries += ks.npad;
        total += (int64_t)ks.al * ks.al;
        max_al = std::max(max_al, ks.al);
    }
    P.h_kmord.assign(entries * 4, 0.0);
    P.h_kmuidx.assign(entries, -1);
    P.h_kmdense.assign(std::max<int64_t>(dtotal, 1), 0.0);
    for (int k = 0; k < P.nsys; ++k) {
        const KmSys& ks = P.h_kmsys[k];
        const auto& uo = P.user_of[k];
        for (int i = 0; i < ks.npad; ++i) {
            const int u = uo[i];
            if (u < 0) continue;
            P.h_kmuidx[ks.ord_off + i] = u;
            double* o = &P.h_kmord[(ks.ord_off + i) * 4];
            o[0] = in[k].dirs[3 * u];
            o[1] = in[k].dirs[3 * u + 1];
            o[2] = in[k].dirs[3 * u + 2];
            o[3] = in[k].w[u];
        }
        if (in[k].h->scat == ROM_SCAT_DENSE)
            std::copy(in[k].h->Pdense.begin(), in[k].h->Pdense.end(), P.h_kmdense.begin() + ks.dense_off);
    }
    if (first) {
        take(P, P.d_Pt, total * (P.fp64 ? 8 : 2));
        take(P, P.d_kmsys, P.h_kmsys.size() * sizeof(KmSys));
        take(P, P.d_kmord, P.h_kmord.size() * sizeof(double));
        take(P, P.d_kmuidx, P.h_kmuidx.size() * sizeof(int32_t));
        take(P, P.d_kmdense, P.h_kmdense.size() * sizeof(double));
        take(P, P.d_kminv, entries * sizeof(double));
    }
    rewrite(P.d_kmsys, P.h_kmsys, s);
    rewrite(P.d_kmord, P.h_kmord, s);
    rewrite(P.d_kmuidx, P.h_kmuidx, s);
    if (dtotal > 0) rewrite(P.d_kmdense, P.h_kmdense, s);
    KmArgs a{};
    a.sys = (const KmSys*)P.d_kmsys.p;
    a.ord = (const double*)P.d_kmord.p;
    a.uidx = (const int32_t*)P.d_kmuidx.p;
    a.dense = (const double*)P.d_kmdense.p;
    a.inv_r = (double*)P.d_kminv.p;
    a.bt = P.d_Pt.p;
    a.nsys = P.nsys;
    a.fp64 = P.fp64 ? 1 : 0;
    a.max_al = max_al;
    HIPCHK(launch_kernel_matrix(a, s));
}

// New ordinate values (and inflow or kernel values) for a plan whose structure still fits: the
// same systems, the same ordinate count in every quadrant and the same inflow presence.  Rewrites
// the lane table, the weighted inflow and the kernel matrices in place, stream-ordered on s, so
// buffers and the captured graph stay valid.  Returns false when the plan must be rebuilt.
bool refresh_ordinates(Plan& P, const std::vector<SysInput>& in, hipStream_t s)
{
    if ((int)in.size() != P.nsys) return false;
    int mom_r = 0;
    for (auto& si : in) {
        if ((scat_mode(si.h) == 1) != (P.nmom == 4) || (scat_mode(si.h) == 2) != P.aniso) return false;
        if (scat_mode(si.h) == 1 && si.h->scat_norm) mom_r = 1;
    }
    if (mom_r != P.mom_r) return false;
    if (P.aniso)  // the caller's dense kernel has a buffer of its own in the kernel-matrix inputs
        for (size_t k = 0; k < in.size(); ++k)
            if ((in[k].h->scat == ROM_SCAT_DENSE) != (P.h_kmsys[k].kind == ROM_SCAT_DENSE)) return false;
    std::vector<std::array<std::vector<int>, 4>> ql(in.size());
    for (size_t k = 0; k < in.size(); ++k) {
        if (in[k].h != P.handles[P.sys[k].prob]) return false;
        for (int l = 0; l < in[k].n; ++l) ql[k][quadrant_of(in[k].dirs[3 * l], in[k].dirs[3 * l + 1])].push_back(l);
        for (int q = 0; q < 4; ++q)
            if ((int)ql[k][q].size() != P.qcount[k][q]) return false;
    }
    for (int p = 0; p < (int)P.handles.size(); ++p) {
        rom_handle* h = P.handles[p];
        bool vacuum = true;
        for (int f = 0; f < 4; ++f)
            if (!h->face[f].empty()) vacuum = false;
        for (auto& si : in)
            if (si.h == h && si.use_angular)
                for (int f = 0; f < 4; ++f)
                    if (!h->ang[f].empty()) vacuum = false;
        const bool had = P.inflow_len > 0;
        if (!vacuum != had) return false;
    }
    if (P.kind == ROM_SWEEP_DIAG) {
        // same tasks in the same order: refill each task's ordinate entries
        const int NO = (kWave / P.dR) * P.dK;
        size_t ti = 0;
        for (int k = 0; k < P.nsys; ++k) {
            rom_handle* h = P.handles[P.sys[k].prob];
            std::vector<int>& uo = P.user_of[k];
            const size_t before = uo.size();
            uo.clear();
            for (int q = 0; q < 4; ++q) {
                const auto& list = ql[k][q];
                for (size_t b0 = 0; b0 < list.size(); b0 += NO) {
                    if (ti >= P.dtasks.size()) throw Fail{ROM_E_STATE, "row-lane task layout changed"};
                    const DiagTaskDev& t = P.dtasks[ti++];
                    for (int o = 0; o < NO; ++o) {
                        LaneDev& ld = P.lanes[t.ord_off + o];
                        const int u = b0 + o < list.size() ? list[b0 + o] : -1;
                        ld.ord = (int)uo.size();
                        uo.push_back(u);
                        fill_lane(ld, h, in[k], u, {});
                    }
                }
            }
            if (uo.size() != before) throw Fail{ROM_E_STATE, "ordinate layout changed"};
            P.sys_n[k] = in[k].n;
            P.sys_w[k] = in[k].w;
        }
        rewrite(P.d_lanes, P.lanes, s);
        if (P.inflow_len > 0) {
            P.h_inflow = diag_inflow_table(P, in);
            if (P.fp64) {
                rewrite(P.d_inflow, P.h_inflow, s);
            } else {
                P.h_inflow32.assign(P.h_inflow.begin(), P.h_inflow.end());
                rewrite(P.d_inflow, P.h_inflow32, s);
            }
        }
        if (P.aniso) build_kernel_matrices(P, in, s);
        return true;
    }
    // internal order: quadrant-major, L-lane groups, padded (as built)
    for (int k = 0; k < P.nsys; ++k) {
        std::vector<int>& uo = P.user_of[k];
        const size_t before = uo.size();
        uo.clear();
        for (int q = 0; q < 4; ++q) {
            const auto& list = ql[k][q];
            for (size_t b = 0; b < list.size(); b += P.L)
                for (int l = 0; l < P.L; ++l) uo.push_back(b + l < list.size() ? list[b + l] : -1);
        }
        if (uo.size() != before) throw Fail{ROM_E_STATE, "ordinate layout changed"};
        P.sys_n[k] = in[k].n;
        P.sys_w[k] = in[k].w;
    }
    std::vector<std::vector<double>> inv_r(P.nsys);
    for (int k = 0; k < P.nsys; ++k) inv_r[k] = linear_inv_r(in[k].h, in[k]);
    for (int k = 0; k < P.nws; ++k) {
        const WaveStreamDev& W = P.ws[k];
        rom_handle* h = P.handles[W.prob];
        for (int lane = 0; lane < kWave; ++lane) {
            LaneDev& ld = P.lanes[(size_t)k * kWave + lane];
            const int sy = W.sys[lane / W.L];
            fill_lane(ld, h, in[sy < 0 ? 0 : sy], sy < 0 ? -1 : P.user_of[sy][ld.ord], sy < 0 ? inv_r[0] : inv_r[sy]);
        }
    }
    rewrite(P.d_lanes, P.lanes, s);
    // the linear kernel's g may have changed
    bool gchange = false;
    for (int k = 0; k < P.nsys; ++k) {
        const double g = scat_mode(in[k].h) == 1 ? in[k].h->g : 0.0;
        if (P.sys[k].g != g) {
            P.sys[k].g = g;
            gchange = true;
        }
    }
    if (gchange) rewrite(P.d_sys, P.sys, s);
    if (P.inflow_len > 0) {
        P.h_inflow = inflow_table(P, in);
        if (P.fp64) {
            rewrite(P.d_inflow, P.h_inflow, s);
        } else {
            P.h_inflow32.assign(P.h_inflow.begin(), P.h_inflow.end());
            rewrite(P.d_inflow, P.h_inflow32, s);
        }
    }
    if (P.aniso) build_kernel_matrices(P, in, s);
    return true;
}

// Contraction arguments of system k (S = sigma_s (Psi' P) + q on its [cells][npad] layout).
ContractArgs contract_args(const Plan& P, int k)
{
    const SystemDev& sd = P.sys[k];
    ContractArgs c{};
    c.a = (const char*)P.d_psi.p + sd.ang_off * (P.fp64 ? 8 : 2);
    c.bt = (const char*)P.d_Pt.p + P.pt_off[k] * (P.fp64 ? 8 : 2);
    c.sigma_s = (const char*)P.d_ss.p + P.probs[sd.prob].field_off * P.esz;
    c.q = (const char*)P.d_q.p + P.probs[sd.prob].field_off * P.esz;
    c.out = (char*)P.d_ang.p + sd.ang_off * P.esz;
    c.M = (int)P.handles[sd.prob]->cells;
    c.N = c.K = P.npad_al[k];
    c.sys_index = k;
    c.sysctl = P.d_sysctl.as<SysCtl>();
    // the row-lane sweep keeps per-ordinate sources and angular fluxes in ordinate blocks of 16
    c.blocked = (P.kind == ROM_SWEEP_DIAG && !P.fp64) ? 1 : 0;
    return c;
}

// With several systems (an ensemble batch) all contractions of an iteration go in one launch:
// the argument table and the block map are built once per plan (the buffers never move).
void build_contract_batch(Plan& P)
{
    if (!P.aniso || P.nsys < 2) return;
    const int kind = P.fp64 ? 2 : 0;
    std::vector<ContractArgs> items(P.nsys);
    std::vector<int2> map;
    for (int k = 0; k < P.nsys; ++k) {
        items[k] = contract_args(P, k);
        const int nb = contract_blocks(items[k], kind);
        if (nb < 0) throw Fail{ROM_E_DEVICE, "contraction shape not supported"};
        for (int b = 0; b < nb; ++b) map.push_back(make_int2(k, b));
    }
    upload(P.d_citems, items);
    upload(P.d_cmap, map);
    P.cmap_blocks = (int)map.size();
}

void enqueue_iteration(Plan& P, hipStream_t s, double tol)
{
    if (P.aniso) {
        // the contraction's last block stamps the start of the sweep's timing (not the combine's end)
        Ctl* const ctl = P.d_ctl.as<Ctl>();
        if (P.cmap_blocks > 0) {
            HIPCHK(launch_contract_batch(P.d_citems.as<ContractArgs>(), P.d_cmap.as<int2>(), P.cmap_blocks, P.fp64 ? 2 : 0, s, ctl));
        } else {
            for (int k = 0; k < P.nsys; ++k) HIPCHK(launch_contract(contract_args(P, k), P.fp64 ? 2 : 0, s, ctl));
        }
    }
    HIPCHK(P.launch_sweep_any(0, s));
    const CombineArgs ca = P.combine_args(0, tol);
    HIPCHK(launch_combine(ca, (int)P.cblocks.size(), P.fp64, s));
}

struct SolveResult {
    std::vector<SysCtl> sc;
    bool error = false;
    double ms = 0;
    double sweep_ms = 0;
    int sweeps = 0;
    int tx = 0, ty = 0, band = 0, lanes = 0, kind = 0;
};

// Source iteration for every system of the plan.  The first iterate starts from phi = 0 (so the
// first source is q), the per-iteration kernels are captured once in a graph of K iterations
// and replayed until every system has stopped.
SolveResult run_si(Plan& P, hipStream_t s, const rom_si_opts& o)
{
    const double tol = o.tol;
    // Iterations per replay: by default the previous solve's count (split into replays of at most
    // 64), so a repeated solve of the same shape launches no iterations past convergence.
    int K = o.iters_per_check > 0 ? o.iters_per_check : 0;
    if (K == 0 && P.last_iters > 0) {
        const int reps = (P.last_iters + 63) / 64;
        K = (P.last_iters + reps - 1) / reps;
    }
    if (K == 0) K = P.max_iter <= 64 ? 4 : 8;
    K = std::min(K, P.max_iter);
    if (!P.ev0) HIPCHK(hipEventCreate(&P.ev0));
    if (!P.ev1) HIPCHK(hipEventCreate(&P.ev1));
    hipEvent_t e0 = P.ev0, e1 = P.ev1;
    HIPCHK(hipEventRecord(e0, s));
    // initial state: phi = 0, isotropic source = q (linear kernel: S0 = q, S1 = S2 = 0), angular
    // flux = 0, every system active.  Its arguments are fixed for a plan, so it is captured at the
    // head of the first replay's graph: a solve that stops within K iterations is one launch.
    int64_t phi_total = 0, max_cells = 0, psi_total = 0;
    for (auto& sd : P.sys) {
        phi_total = std::max<int64_t>(phi_total, sd.phi_off + P.handles[sd.prob]->cells);
        max_cells = std::max<int64_t>(max_cells, P.handles[sd.prob]->cells);
    }
    if (P.aniso)
        for (int k = 0; k < P.nsys; ++k)
            psi_total = std::max<int64_t>(psi_total, P.sys[k].ang_off + P.handles[P.sys[k].prob]->cells * (int64_t)P.npad_al[k]);
    auto enqueue_initial_state = [&]() {
        if (P.nmom == 4) HIPCHK(launch_fill(P.src_ptr(), P.src_len, P.fp64, 0.0, s));  // S1 = S2 = 0
        if (P.aniso) {
            if (P.fp64) HIPCHK(launch_fill(P.d_psi.p, psi_total, true, 0.0, s));
            else HIPCHK(launch_fill(P.d_psi.p, (psi_total + 1) / 2, false, 0.0, s));  // BF16 zeros are float zeros
        }
        HIPCHK(launch_init_state(P.d_sys.as<SystemDev>(), P.d_probs.as<ProblemDev>(), P.nsys, max_cells, P.fp64, P.d_q.p,
                                 P.src_ptr(), P.d_phi.p, phi_total, P.d_sysctl.as<SysCtl>(), P.d_ctl.as<Ctl>(), s));
    };
    auto capture = [&](bool with_initial_state, hipGraph_t& g, hipGraphExec_t& ge) {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            // a later replay's first sweep is timed from a mark at its start, not from the previous
            // replay's last combine; after the initial state it is timed from its first ticket claim
            if (with_initial_state) enqueue_initial_state();
            else HIPCHK(launch_mark(P.d_ctl.as<Ctl>(), s));
            for (int k = 0; k < K; ++k) enqueue_iteration(P, s, tol);
        } catch (...) {
            hipGraph_t gg = nullptr;
            (void)hipStreamEndCapture(s, &gg);
            if (gg) (void)hipGraphDestroy(gg);
            throw;
        }
        HIPCHK(hipStreamEndCapture(s, &g));
        HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    };

    if (!P.gexec || !P.gexec0 || P.graph_iters != K || P.graph_stream != s || P.graph_tol != tol) {
        for (hipGraphExec_t* ge : {&P.gexec, &P.gexec0})
            if (*ge) {
                (void)hipGraphExecDestroy(*ge);
                *ge = nullptr;
            }
        for (hipGraph_t* g : {&P.graph, &P.graph0})
            if (*g) {
                (void)hipGraphDestroy(*g);
                *g = nullptr;
            }
        capture(true, P.graph0, P.gexec0);
        capture(false, P.graph, P.gexec);
        P.graph_iters = K;
        P.graph_stream = s;
        P.graph_tol = tol;
    }
    const size_t sc_off = (sizeof(Ctl) + 255) / 256 * 256;
    const size_t state_bytes = sc_off + (size_t)P.nsys * sizeof(SysCtl);
    if (P.h_state_bytes < state_bytes) {
        if (P.h_state) (void)hipHostFree(P.h_state);
        P.h_state = nullptr;
        P.h_state_bytes = 0;
        HIPCHK(hipHostMalloc(&P.h_state, state_bytes, hipHostMallocDefault));
        P.h_state_bytes = state_bytes;
    }
    void* h_ctl = P.h_state;
    void* h_sc = (char*)P.h_state + sc_off;
    Ctl ctl{};
    SolveResult r;
    r.sc.resize(P.nsys);
    int launched = 0;
    for (;;) {
        HIPCHK(hipGraphLaunch(launched == 0 ? P.gexec0 : P.gexec, s));
        launched += K;
        // the control block and the per-system states (one block, sysctl at sc_off) come back in
        // one copy behind one synchronization
        HIPCHK(hipMemcpyAsync(h_ctl, P.d_ctl.p, state_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(e1, s));  // complete once this replay's state is back; the last one ends the timing
        HIPCHK(hipStreamSynchronize(s));
        std::memcpy(&ctl, h_ctl, sizeof(Ctl));
        std::memcpy(r.sc.data(), h_sc, P.nsys * sizeof(SysCtl));
        if (ctl.error || ctl.active == 0 || launched >= P.max_iter + K) break;
    }
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    r.ms = ms;
    r.error = ctl.error != 0;
    r.sweep_ms = (double)ctl.sweep_ticks / wallclock_khz();
    r.sweeps = ctl.sweeps;
    int most = 0;
    for (const SysCtl& c : r.sc) most = std::max(most, c.iter);
    P.last_iters = most;
    r.kind = P.kind;
    if (P.kind == ROM_SWEEP_DIAG) {
        r.tx = P.dK;
        r.ty = P.dR;
        r.band = P.dNB;
        r.lanes = P.dR;
    } else {
        r.tx = P.tx;
        r.ty = P.ty;
        r.band = P.band;
        r.lanes = P.L;
    }
    return r;
}

void download_phi(const Plan& P, int sys, double* out)
{
    const SystemDev& sd = P.sys[sys];
    const int64_t cells = P.handles[sd.prob]->cells;
    if (P.fp64) {
        HIPCHK(hipMemcpy(out, (const char*)P.d_phi.p + sd.phi_off * 8, cells * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(cells);
        HIPCHK(hipMemcpy(tmp.data(), (const char*)P.d_phi.p + sd.phi_off * 4, cells * 4, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < cells; ++k) out[k] = tmp[k];
    }
}

int validate_opts(rom_handle* h, const rom_si_opts* o, rom_si_opts& out)
{
    std::memset(&out, 0, sizeof(out));
    if (o) out = *o;
    if (!isfin(out.tol)) return fail(h, ROM_E_ARG, "tol must be finite");
    if (out.tol == 0.0) out.tol = 1e-6;
    if (out.max_iter < 0) return fail(h, ROM_E_ARG, "max_iter must be >= 0");
    if (out.max_iter == 0) out.max_iter = 1000;
    if (out.precision != ROM_PREC_FP32 && out.precision != ROM_PREC_FP64) return fail(h, ROM_E_ARG, "bad precision");
    if (out.scheme != ROM_SCHEME_STEP && out.scheme != ROM_SCHEME_DD) return fail(h, ROM_E_ARG, "bad scheme");
    if (out.iters_per_check < 0) return fail(h, ROM_E_ARG, "iters_per_check must be >= 0");
    if (out.contract_split != 0) return fail(h, ROM_E_UNSUPPORTED, "split contraction is not built");
    if (out.sweep < ROM_SWEEP_AUTO || out.sweep > ROM_SWEEP_DIAG) return fail(h, ROM_E_ARG, "bad sweep kind");
    if (out.band < 0 || out.band > (out.sweep == ROM_SWEEP_DIAG ? kDiagMaxWaves : kMaxBand))
        return fail(h, ROM_E_ARG, "band must be 0..8 (strip sweep) or 0..16 (row-lane sweep)");
    if (out.diag_rows != 0 && out.diag_rows != 16 && out.diag_rows != 64)
        return fail(h, ROM_E_ARG, "diag_rows must be 0, 16 or 64");
    if (out.diag_k != 0 && !diag_supported(out.precision == ROM_PREC_FP64, 16, out.diag_k))
        return fail(h, ROM_E_ARG, "diag_k must be 0, 1, 2 or 4 (FP64: 0, 1, 2)");
    if (out.sweep == ROM_SWEEP_DIAG && out.scheme != ROM_SCHEME_STEP)
        return fail(h, ROM_E_UNSUPPORTED, "the row-lane sweep implements the step scheme only");
    if ((out.tile_x != 0 || out.tile_y != 0) && !sweep_tile_supported(out.tile_x, out.tile_y))
        return fail(h, ROM_E_ARG, "unsupported tile shape (8x4, 8x8, 16x8, 16x16)");
    return ROM_OK;
}

// sig: scat_sig of the handle (or of the batch's first handle; every member matches it)
std::string plan_signature(const rom_si_opts& o, int sig, int kind, int nsys)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "k%d p%d s%d t%dx%d b%d a%d n%d mi%d w%d r%d q%d", kind, o.precision, o.scheme, o.tile_x,
                  o.tile_y, o.band, sig, nsys, o.max_iter, o.sweep, o.diag_rows, o.diag_k);
    return buf;
}

// A dense kernel whose ordinate set has since been replaced (rom_set_ordinates clears it).
bool dense_stale(const rom_handle* h) { return h->scat == ROM_SCAT_DENSE && h->Pdense.size() != (size_t)h->n * h->n; }

int check_ordinates(rom_handle* h, int n, const double* dirs, const double* w)
{
    if (n <= 0 || !dirs || !w) return fail(h, ROM_E_ARG, "ordinates: n must be > 0 and arrays non-NULL");
    double sw = 0.0;
    for (int l = 0; l < n; ++l) {
        const double c = dirs[3 * l], s = dirs[3 * l + 1], z = dirs[3 * l + 2];
        if (!isfin(c) || !isfin(s) || !isfin(z) || !isfin(w[l]))
            return fail(h, ROM_E_DOMAIN, "ordinates: non-finite value at index " + std::to_string(l));
        if (std::fabs(c * c + s * s + z * z - 1.0) > 1e-12)
            return fail(h, ROM_E_DOMAIN, "ordinates: direction " + std::to_string(l) + " is not a unit vector");
        if (!(w[l] > 0.0)) return fail(h, ROM_E_DOMAIN, "ordinates: weights must be > 0");
        sw += w[l];
    }
    if (std::fabs(sw - 1.0) > 1e-12) return fail(h, ROM_E_DOMAIN, "ordinates: weights must sum to 1");
    return ROM_OK;
}

}  // namespace

// ====================================================================================== C ABI
extern "C" {

const char* rom_version(void) { return "librom 0.1 (gfx950)"; }

const char* rom_status_string(int st)
{
    switch (st) {
    case ROM_OK: return "ok";
    case ROM_NOT_CONVERGED: return "not converged (max_iter reached)";
    case ROM_E_ARG: return "invalid argument";
    case ROM_E_DOMAIN: return "input outside the problem domain";
    case ROM_E_STATE: return "call out of order";
    case ROM_E_NOMEM: return "out of memory";
    case ROM_E_DEVICE: return "device error";
    case ROM_E_DIVERGED: return "iteration diverged";
    case ROM_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* rom_last_error(const rom_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int32_t rom_ordinate_count(const rom_ord_spec* spec) { return spec ? ordinate_count(*spec) : -1; }

int rom_generate_ordinates(const rom_ord_spec* spec, uint64_t seed, int64_t sample, double* dirs, double* w)
{
    if (!spec || !dirs || !w || sample < 0) return ROM_E_ARG;
    if (ordinate_count(*spec) <= 0) return ROM_E_ARG;
    return generate_ordinates(*spec, seed, sample, dirs, w);
}

int rom_create(const rom_grid* grid, const double* sigma_t, const double* sigma_s, const double* q,
               const rom_inflow* inflow, rom_handle** out)
{
    ROM_API_LOCK;
    if (!out) return fail(nullptr, ROM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !sigma_t || !sigma_s || !q) return fail(nullptr, ROM_E_ARG, "NULL grid or field");
    if (grid->nx <= 0 || grid->ny <= 0) return fail(nullptr, ROM_E_ARG, "nx, ny must be positive");
    if ((int64_t)grid->nx * grid->ny >= (int64_t)1 << 31) return fail(nullptr, ROM_E_ARG, "grid too large (2^31 cells or more)");
    // the sweeps publish (epoch << 24) | columns done in their progress counters
    if (grid->nx >= (1 << 24) || grid->ny >= (1 << 24)) return fail(nullptr, ROM_E_ARG, "nx and ny must be below 2^24");
    if (!isfin(grid->x0) || !isfin(grid->x1) || !isfin(grid->y0) || !isfin(grid->y1) || !(grid->x1 > grid->x0) ||
        !(grid->y1 > grid->y0))
        return fail(nullptr, ROM_E_ARG, "grid box must satisfy x1 > x0, y1 > y0");
    const int64_t cells = (int64_t)grid->nx * grid->ny;
    for (int64_t k = 0; k < cells; ++k) {
        const double st = sigma_t[k], ss = sigma_s[k], qq = q[k];
        if (!isfin(st) || !isfin(ss) || !isfin(qq)) return fail(nullptr, ROM_E_DOMAIN, "non-finite field value");
        if (!(st > 0.0)) return fail(nullptr, ROM_E_DOMAIN, "sigma_t must be > 0");
        if (ss < 0.0) return fail(nullptr, ROM_E_DOMAIN, "sigma_s must be >= 0");
        if (!(ss < st)) return fail(nullptr, ROM_E_DOMAIN, "sigma_s must be < sigma_t");
        if (qq < 0.0) return fail(nullptr, ROM_E_DOMAIN, "q must be >= 0");
    }
    const double* faces[4] = {inflow ? inflow->left : nullptr, inflow ? inflow->right : nullptr,
                              inflow ? inflow->bottom : nullptr, inflow ? inflow->top : nullptr};
    for (int f = 0; f < 4; ++f) {
        if (!faces[f]) continue;
        const int len = f < 2 ? grid->ny : grid->nx;
        for (int k = 0; k < len; ++k)
            if (!isfin(faces[f][k]) || faces[f][k] < 0.0) return fail(nullptr, ROM_E_DOMAIN, "inflow must be finite and >= 0");
    }
    std::unique_ptr<rom_handle> h(new (std::nothrow) rom_handle());
    if (!h) return fail(nullptr, ROM_E_NOMEM, "host allocation failed");
    try {
        h->grid = *grid;
        h->dx = (grid->x1 - grid->x0) / grid->nx;
        h->dy = (grid->y1 - grid->y0) / grid->ny;
        h->cells = cells;
        h->st.assign(sigma_t, sigma_t + cells);
        h->ss.assign(sigma_s, sigma_s + cells);
        h->q.assign(q, q + cells);
        for (int f = 0; f < 4; ++f)
            if (faces[f]) h->face[f].assign(faces[f], faces[f] + (f < 2 ? grid->ny : grid->nx));
        // device work is deferred to the first solve, so a handle can be built and validated
        // on a host without a GPU; a missing device surfaces there as ROM_E_DEVICE
        if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    } catch (const std::bad_alloc&) {
        return fail(nullptr, ROM_E_NOMEM, "host allocation failed");
    }
    *out = h.release();
    return ROM_OK;
}

void rom_destroy(rom_handle* h)
{
    ROM_API_LOCK;
    delete h;
}

int rom_set_stream(rom_handle* h, void* stream)
{
    if (!h) return ROM_E_ARG;
    h->user_stream = (hipStream_t)stream;
    return ROM_OK;
}

int rom_set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* ctx)
{
    ROM_API_LOCK;
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(nullptr, ROM_E_ARG, "alloc and free must both be set or both be NULL");
    AllocHook& hook = alloc_hook();
    hook.alloc = alloc;
    hook.free = free_fn;
    hook.ctx = alloc ? ctx : nullptr;
    return ROM_OK;
}

int rom_set_ordinates(rom_handle* h, int32_t n, const double* dirs, const double* w)
{
    if (!h) return ROM_E_ARG;
    int rc = check_ordinates(h, n, dirs, w);
    if (rc) return rc;
    h->n = n;
    h->dirs.assign(dirs, dirs + 3 * (size_t)n);
    h->w.assign(w, w + n);
    for (auto& a : h->ang) a.clear();
    h->Pdense.clear();  // a dense kernel is indexed by the old set: solves refuse until it is set again
    h->version++;
    return ROM_OK;
}

int rom_set_inflow_angular(rom_handle* h, int32_t face, const double* vals)
{
    if (!h) return ROM_E_ARG;
    if (face < 0 || face > 3) return fail(h, ROM_E_ARG, "bad face");
    if (h->n == 0) return fail(h, ROM_E_STATE, "set ordinates before angular inflow");
    if (!vals) {
        h->ang[face].clear();
        h->version++;
        return ROM_OK;
    }
    const size_t len = (size_t)h->n * (face < 2 ? h->grid.ny : h->grid.nx);
    for (size_t k = 0; k < len; ++k)
        if (!isfin(vals[k]) || vals[k] < 0.0) return fail(h, ROM_E_DOMAIN, "inflow must be finite and >= 0");
    h->ang[face].assign(vals, vals + len);
    h->version++;
    return ROM_OK;
}

int rom_set_scattering(rom_handle* h, int32_t kind, double g, const double* P)
{
    if (!h) return ROM_E_ARG;
    const bool norm = (kind & ROM_SCAT_NORMALIZE) != 0;
    kind &= ~ROM_SCAT_NORMALIZE;
    if (kind < ROM_SCAT_ISO || kind > ROM_SCAT_DENSE) return fail(h, ROM_E_ARG, "bad scattering kind");
    if (!isfin(g)) return fail(h, ROM_E_DOMAIN, "g must be finite");
    if (kind == ROM_SCAT_HG && !(std::fabs(g) < 1.0)) return fail(h, ROM_E_DOMAIN, "HG needs |g| < 1");
    if (kind == ROM_SCAT_LINEAR && !(std::fabs(g) <= 1.0)) return fail(h, ROM_E_DOMAIN, "linear kernel needs |g| <= 1");
    if (kind == ROM_SCAT_DENSE) {
        if (h->n == 0) return fail(h, ROM_E_STATE, "set ordinates before a dense kernel");
        if (!P) return fail(h, ROM_E_ARG, "dense kernel needs P");
        const size_t nn = (size_t)h->n * h->n;
        for (size_t k = 0; k < nn; ++k)
            if (!isfin(P[k]) || P[k] < 0.0) return fail(h, ROM_E_DOMAIN, "P must be finite and >= 0");
        if (norm)  // weights are positive: a weighted row sum is positive unless the row is zero
            for (int r = 0; r < h->n; ++r)
                if (std::all_of(P + (size_t)r * h->n, P + (size_t)(r + 1) * h->n, [](double v) { return v == 0.0; }))
                    return fail(h, ROM_E_DOMAIN, "normalized kernel: a row sum is not positive");
        h->Pdense.assign(P, P + nn);
    } else {
        h->Pdense.clear();
    }
    h->scat = kind;
    h->scat_norm = norm;
    h->g = g;
    h->version++;
    return ROM_OK;
}

int rom_phi_device(const rom_handle* h, const void** dev, int32_t* is_fp64)
{
    if (!h || !dev || !is_fp64) return ROM_E_ARG;
    if (!h->res_dev) return ROM_E_STATE;
    *dev = h->res_dev;
    *is_fp64 = h->res_fp64 ? 1 : 0;
    return ROM_OK;
}

int rom_sweep(rom_handle* h, const double* src, int32_t src_per_ordinate, double* phi, double* psi,
              const rom_si_opts* opts)
{
    ROM_API_LOCK;
    if (!h) return ROM_E_ARG;
    if (!src || !phi) return fail(h, ROM_E_ARG, "src and phi must be non-NULL");
    if (h->n == 0) return fail(h, ROM_E_STATE, "set ordinates first");
    rom_si_opts o;
    int rc = validate_opts(h, opts, o);
    if (rc) return rc;
    h->res_dev = nullptr;  // the plan that held the last result may be released below
    try {
        const bool per = src_per_ordinate != 0;
        const size_t nsrc = per ? (size_t)h->n * h->cells : (size_t)h->cells;
        for (size_t k = 0; k < nsrc; ++k)
            if (!isfin(src[k])) return fail(h, ROM_E_DOMAIN, "non-finite source");
        std::vector<SysInput> in{{h, h->dirs.data(), h->w.data(), h->n, true}};
        std::unique_ptr<Plan> P(new Plan());
        if (o.sweep == ROM_SWEEP_AUTO) o.sweep = ROM_SWEEP_STRIP;
        build_plan(*P, in, o, per ? 2 : 0, 0, psi != nullptr);
        hipStream_t s = h->stream();
        const SystemDev& sd = P->sys[0];
        const int al = P->npad_al[0];
        if (per) {
            // per-ordinate source in the internal [cells][npad] layout
            std::vector<double> a((size_t)h->cells * al, 0.0);
            for (int k = 0; k < al && k < (int)P->user_of[0].size(); ++k) {
                const int u = P->user_of[0][k];
                if (u < 0) continue;
                for (int64_t c = 0; c < h->cells; ++c) a[(size_t)c * al + k] = src[(size_t)u * h->cells + c];
            }
            if (P->fp64) upload(P->d_ang, a);
            else {
                std::vector<float> f(a.begin(), a.end());
                upload(P->d_ang, f);
            }
        } else {
            if (P->fp64) HIPCHK(hipMemcpy(P->src_ptr(), src, h->cells * 8, hipMemcpyHostToDevice));
            else {
                std::vector<float> f(src, src + h->cells);
                HIPCHK(hipMemcpy(P->src_ptr(), f.data(), h->cells * 4, hipMemcpyHostToDevice));
            }
        }
        const int psi_mode = psi ? 1 : 0;
        if (psi) {
            const int64_t tot = h->cells * (int64_t)al;
            HIPCHK(P->d_psi.alloc(tot * P->esz));
        }
        HIPCHK(launch_reset_systems(P->d_sysctl.as<SysCtl>(), 1, P->d_ctl.as<Ctl>(), s));
        if (P->kind == ROM_SWEEP_DIAG) {
            HIPCHK(P->launch_sweep_any(1, s));
        } else {
            SweepArgs sa = P->sweep_args(1, psi_mode);
            // the sweep writes psi' into the angular layout when asked for it
            HIPCHK(launch_sweep(sa, P->grid, P->fp64, P->tx, P->ty, P->dd, per, psi_mode, P->L, 1, s));
        }
        const CombineArgs ca = P->combine_args(1, 0.0);
        HIPCHK(launch_combine(ca, (int)P->cblocks.size(), P->fp64, s));
        Ctl ctl{};
        HIPCHK(hipMemcpyAsync(&ctl, P->d_ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ctl.error) return fail(h, ROM_E_DEVICE, "sweep dependency wait timed out");
        download_phi(*P, 0, phi);
        if (psi) {
            const int64_t tot = h->cells * (int64_t)al;
            std::vector<double> pv(tot);
            if (P->fp64) HIPCHK(hipMemcpy(pv.data(), P->d_psi.p, tot * 8, hipMemcpyDeviceToHost));
            else {
                std::vector<float> f(tot);
                HIPCHK(hipMemcpy(f.data(), P->d_psi.p, tot * 4, hipMemcpyDeviceToHost));
                std::copy(f.begin(), f.end(), pv.begin());
            }
            for (int k = 0; k < (int)P->user_of[0].size(); ++k) {
                const int u = P->user_of[0][k];
                if (u < 0) continue;
                const double inv = 1.0 / h->w[u];
                for (int64_t c = 0; c < h->cells; ++c) psi[(size_t)u * h->cells + c] = pv[(size_t)c * al + k] * inv;
            }
        }
        (void)sd;
        h->plan.reset();  // a one-off plan; forget any cached solve plan's device result
        h->res_dev = nullptr;
    } catch (const Fail& f) {
        return fail(h, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(h, ROM_E_NOMEM, "host allocation failed");
    }
    return ROM_OK;
}

}  // extern "C"

// rom_sweep's work for a device-resident isotropic source, with every device buffer placed in a
// preallocated region: the plan (tables, sigma_t pool, inflow, partial-flux slots, strip edges,
// progress counters, control state) is built on the host once per handle state and precision and
// uploaded into the region; `owner` (three words per device) records whose plan the region
// holds, so repeated calls for the same handle only clear the counters and launch the sweep and
// the combine, all on the caller's stream, without waiting for the device.
int rom::sweep_in_scratch(rom_handle* h, void* scratch, size_t cap, uint64_t* owner, const void* src, void* phi,
                          int32_t precision, void* stream)
{
    ROM_API_LOCK;
    if (!h) return ROM_E_ARG;
    if (!src || !phi) return fail(h, ROM_E_ARG, "src and phi must be device pointers");
    if (!scratch || !owner) return fail(h, ROM_E_DEVICE, "scratch region unavailable");
    if (h->n == 0) return fail(h, ROM_E_STATE, "set ordinates first");
    if (precision != ROM_PREC_FP32 && precision != ROM_PREC_FP64) return fail(h, ROM_E_ARG, "bad precision");
    const hipStream_t s = (hipStream_t)stream;
    try {
        const uint64_t state = (h->version << 1) | (uint64_t)precision;
        const bool placed = h->na_plan && h->na_version == h->version && h->na_prec == precision &&
                            owner[0] == h->uid && owner[1] == state && owner[2] == 1;
        if (!placed) {
            owner[2] = 0;  // the region's contents are being replaced
            // the previous plan's host copies may still feed uploads queued on another stream
            if (h->na_plan && h->na_plan->arena) HIPCHK(hipStreamSynchronize(h->na_plan->arena->s));
            h->na_plan.reset();
            rom_si_opts o;
            std::memset(&o, 0, sizeof(o));
            o.precision = precision;
            o.sweep = ROM_SWEEP_STRIP;  // as rom_sweep
            std::vector<SysInput> in{{h, h->dirs.data(), h->w.data(), h->n, true}};
            std::unique_ptr<Plan> P(new Plan());
            std::unique_ptr<Arena> ar(new Arena{(char*)scratch, cap, 0, s});
            P->arena = ar.get();
            try {
                build_plan(*P, in, o, 0, 0, false);
            } catch (...) {
                (void)hipStreamSynchronize(s);  // uploads already queued read the plan's host copies
                throw;
            }
            HIPCHK(hipStreamSynchronize(s));  // tables in place before their host copies can go
            P->keep.clear();
            P->keep.shrink_to_fit();
            h->na_arena.reset(ar.release());
            h->na_plan.reset(P.release());
            h->na_version = h->version;
            h->na_prec = precision;
            owner[0] = h->uid;
            owner[1] = state;
            owner[2] = 1;
        }
        Plan& P = *h->na_plan;
        h->na_arena->s = s;
        // counters that must start at zero, then a fresh control state (ticket 0, epoch 1)
        HIPCHK(launch_fill(P.d_prog.p, (int64_t)P.prog_count * 2, false, 0.0, s));
        HIPCHK(launch_fill(P.d_ctl.p, (int64_t)(sizeof(Ctl) / 4), false, 0.0, s));
        HIPCHK(launch_reset_systems(P.d_sysctl.as<SysCtl>(), 1, P.d_ctl.as<Ctl>(), s));
        SweepArgs sa = P.sweep_args(1, 0);
        sa.src = src;
        HIPCHK(launch_sweep(sa, P.grid, P.fp64, P.tx, P.ty, P.dd, false, 0, P.L, 1, s));
        CombineArgs ca = P.combine_args(1, 0.0);
        ca.phi = phi;
        ca.src = nullptr;
        ca.sigma_s = nullptr;
        ca.q = nullptr;
        HIPCHK(launch_combine(ca, (int)P.cblocks.size(), P.fp64, s));
    } catch (const Fail& f) {
        owner[2] = 0;
        h->na_plan.reset();
        return fail(h, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        owner[2] = 0;
        h->na_plan.reset();
        return fail(h, ROM_E_NOMEM, "host allocation failed");
    }
    return ROM_OK;
}

namespace {

bool is_aniso(const rom_handle* h) { return scat_mode(h) == 2; }

// Source iteration for a list of systems; fills stats and phis.
// ------------------------------------------------------------------------------------ autotuner
//
// The sweep kernel (strip or row-lane) and its shape decide pipeline depth, per-step overhead
// and occupancy, and the best choice depends on the batch: a single problem with few ordinates
// wants the row-lane kernel's spatial parallelism, a large ensemble the strip kernel's in-lane
// ordinate sums.  The first solve of a batch shape times each candidate on the real buffers (one
// warm-up and five timed steps each) and caches the fastest in the handle that leads the solve
// (the ensemble's or single solve's handle, a batch's first handle).  Every choice is
// deterministic; strip tiles and bands give bitwise identical results, while the row-lane kernel
// sums the ordinates of a cell in another (fixed) order.
std::string tune_key(const std::vector<SysInput>& in, const rom_si_opts& o, int smode)
{
    int maxnx = 0, maxny = 0, maxn = 0;
    int64_t work = 0;
    for (auto& s : in) {
        maxnx = std::max(maxnx, s.h->grid.nx);
        maxny = std::max(maxny, s.h->grid.ny);
        maxn = std::max(maxn, s.n);
        work += s.h->cells * (int64_t)s.n;
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "p%d s%d a%d k%zu x%d y%d n%d w%lld v%d r%d q%d", o.precision, o.scheme, smode,
                  in.size(), maxnx, maxny, maxn, (long long)work, o.sweep, o.diag_rows, o.diag_k);
    return buf;
}

bool autotune_enabled()
{
    const char* e = std::getenv("ROM_AUTOTUNE");
    return !(e && e[0] == '0');
}

// One candidate sweep configuration: strip (tile, band) or row-lane (rows, ordinates per lane).
struct TuneChoice {
    int sweep = 0, tx = 0, ty = 0, band = 0, rows = 0, k = 0;
};

void apply_choice(const TuneChoice& c, rom_si_opts& o)
{
    o.sweep = c.sweep;
    if (c.sweep == ROM_SWEEP_STRIP) {
        o.tile_x = c.tx;
        o.tile_y = c.ty;
        o.band = c.band;
    } else {
        o.diag_rows = c.rows;
        o.diag_k = c.k;
        o.band = c.band;
    }
}

// Time sweep + combine steps of every candidate on the real buffers of this batch shape (zero
// sources) and keep the fastest in the owner handle's cache.  Candidates: the strip kernel's tiles x
// bands, and, for isotropic step-scheme problems, the row-lane kernel's (rows, ordinates per lane).
void autotune(rom_handle* owner, std::vector<SysInput>& in, rom_si_opts& o, int smode, hipStream_t s)
{
    const bool aniso = smode == 2;
    const std::string key = tune_key(in, o, smode);
    {
        auto it = owner->tune_cache.find(key);
        if (it != owner->tune_cache.end()) {
            const auto& v = it->second;
            apply_choice(TuneChoice{v[0], v[1], v[2], v[3], v[4], v[5]}, o);
            return;
        }
    }
    const bool fp64 = o.precision == ROM_PREC_FP64;
    std::vector<TuneChoice> cands;
    if (o.sweep != ROM_SWEEP_DIAG) {
        const std::vector<std::pair<int, int>> tiles = fp64 ? std::vector<std::pair<int, int>>{{8, 4}, {8, 8}}
                                                            : std::vector<std::pair<int, int>>{{8, 4}, {8, 8}, {16, 8}, {16, 16}};
        for (auto t : tiles)
            for (int band : {2, 4, 8}) cands.push_back({ROM_SWEEP_STRIP, t.first, t.second, band, 0, 0});
    }
    // the row-lane kernel: isotropic step sweeps, and FP32 step sweeps of dense kernels
    if (o.sweep != ROM_SWEEP_STRIP && o.scheme == ROM_SCHEME_STEP && (smode == 0 || (smode == 2 && !fp64))) {
        for (int rows : {16, 64})
            for (int k : {1, 2, 4})
                if (diag_supported(fp64, rows, k) && (o.diag_rows == 0 || o.diag_rows == rows) && (o.diag_k == 0 || o.diag_k == k))
                    for (int nb : rows == 16 ? std::vector<int>{4, 8, 16} : std::vector<int>{1, 2, 4})
                        if (o.band == 0 || o.band == nb) cands.push_back({ROM_SWEEP_DIAG, 0, 0, nb, rows, k});
    }
    float best = 1e30f;
    TuneChoice pick;
    // each candidate: one warm-up step, then kSteps steps timed one by one; its score is the
    // fastest step (robust to launch jitter, which a single short measurement is not)
    constexpr int kSteps = 5;
    hipEvent_t ev[kSteps + 1];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (const TuneChoice& cand : cands) {
        rom_si_opts c = o;
        apply_choice(cand, c);
        Plan P;
        try {
            build_plan(P, in, c, smode, 1);
        } catch (const Fail&) {
            continue;  // does not fit (LDS) or not supported for this batch
        }
        if (cand.sweep == ROM_SWEEP_STRIP &&
            (P.band != cand.band || sweep_lds_bytes(P.fp64, P.tx, P.ty, aniso, P.L, P.band, P.nmom) > 64 * 1024))
            continue;
        HIPCHK(launch_fill(P.src_ptr(), P.src_len, P.fp64, 0.0, s));
        if (aniso) HIPCHK(launch_fill(P.d_ang.p, (int64_t)(P.d_ang.bytes / P.esz), P.fp64, 0.0, s));
        const CombineArgs ca = P.combine_args(1, 0.0);
        for (int rep = 0; rep <= kSteps; ++rep) {
            HIPCHK(launch_reset_systems(P.d_sysctl.as<SysCtl>(), P.nsys, P.d_ctl.as<Ctl>(), s));
            if (rep >= 1) HIPCHK(hipEventRecord(ev[rep - 1], s));
            HIPCHK(P.launch_sweep_any(1, s));
            HIPCHK(launch_combine(ca, (int)P.cblocks.size(), P.fp64, s));  // a source-iteration step is both
        }
        HIPCHK(hipEventRecord(ev[kSteps], s));
        HIPCHK(hipEventSynchronize(ev[kSteps]));
        float score = 1e30f;
        for (int k = 0; k < kSteps; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            score = std::min(score, ms);
        }
        Ctl ctl{};
        HIPCHK(hipMemcpy(&ctl, P.d_ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost));
        if (!ctl.error && score < best) {
            best = score;
            pick = cand;
            if (cand.sweep == ROM_SWEEP_STRIP) {
                pick.tx = P.tx;
                pick.ty = P.ty;
                pick.band = P.band;
            } else {
                pick.band = P.dNB;
            }
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (pick.sweep == 0) return;  // nothing measurable: keep the heuristic
    owner->tune_cache[key] = {pick.sweep, pick.tx, pick.ty, pick.band, pick.rows, pick.k};
    apply_choice(pick, o);
}

// reuse: 0 build a new plan, 1 run the cached plan as it is, 2 refresh its ordinate tables first
// (rebuilding when the structure no longer fits)
int solve_systems(rom_handle* owner, std::vector<SysInput>& in, const rom_si_opts& o_in, int reuse,
                  std::unique_ptr<Plan>& slot, SolveResult& res)
{
    const int smode = scat_mode(in[0].h);
    const bool aniso = smode == 2;
    for (auto& s : in)
        if (scat_mode(s.h) != smode)
            return fail(owner, ROM_E_ARG, "batched problems must share the scattering mode (isotropic, linear or dense)");
    rom_si_opts o = o_in;
    if (reuse == 2 && slot && !refresh_ordinates(*slot, in, owner->stream())) reuse = 0;
    if (reuse == 0 || !slot) {
        const bool free_shape = o.sweep == ROM_SWEEP_DIAG ? (o.diag_rows == 0 || o.diag_k == 0 || o.band == 0)
                                                          : (o.tile_x == 0 && o.band == 0);
        if (free_shape && autotune_enabled()) autotune(owner, in, o, smode, owner->stream());
        slot.reset(new Plan());
        build_plan(*slot, in, o, smode, o.max_iter);
        if (aniso) {
            build_kernel_matrices(*slot, in, owner->stream());
            build_contract_batch(*slot);
        }
    }
    res = run_si(*slot, owner->stream(), o);
    if (res.error) return fail(owner, ROM_E_DEVICE, "sweep dependency wait timed out");
    return ROM_OK;
}

// Running statistics of an ensemble's batches.
struct EnsAgg {
    int min_it = 1 << 30, max_it = 0, worst = ROM_OK, sweeps = 0;
    int64_t updates = 0;
    double ms = 0, sweep_ms = 0;
    int shape[5] = {0, 0, 0, 0, 0};

    void fill(rom_ens_stats* st, int t) const
    {
        if (!st) return;
        st->samples = t;
        st->min_iters = min_it;
        st->max_iters = max_it;
        st->status = worst == ROM_OK ? ROM_OK : ROM_NOT_CONVERGED;
        st->updates = updates;
        st->device_ms = ms;
        st->sweep_ms = sweep_ms;
        st->sweeps = sweeps;
        st->tile_x = shape[0];
        st->tile_y = shape[1];
        st->band = shape[2];
        st->lanes = shape[3];
        st->sweep = shape[4];
    }
};

int check_ensemble(rom_handle* h, const rom_ord_spec& spec, const rom_si_opts* opts, rom_si_opts& o)
{
    if (ordinate_count(spec) <= 0) return fail(h, ROM_E_ARG, "bad ordinate spec");
    if (h->scat == ROM_SCAT_DENSE) return fail(h, ROM_E_STATE, "a dense kernel belongs to one ordinate set");
    return validate_opts(h, opts, o);
}

// Samples first .. first + t - 1 of (spec, seed), generated exactly as rom_generate_ordinates
// does, solved in batches (as many samples per launch as a 24 GiB budget and 1024 allow) with
// one cached plan per batch shape, refreshed with each batch's ordinates.  After each batch,
// per_batch(plan, index of the batch's first sample in this call, batch size) consumes the
// fluxes while they are on the device.
int ensemble_batches(rom_handle* h, int64_t first, int t, uint64_t seed, const rom_ord_spec& spec, const rom_si_opts& o,
                     const std::function<void(Plan&, int, int)>& per_batch, EnsAgg& ag)
{
    const int n = ordinate_count(spec);
    const bool aniso = is_aniso(h);
    const int64_t per_sample = h->cells * (int64_t)(aniso ? (n + 128) * 6 : 0) + h->cells * 8 * 8 +
                               (int64_t)h->grid.nx * h->grid.ny / 2 * 4;
    const int64_t budget = (int64_t)24 << 30;
    int B = (int)std::max<int64_t>(1, std::min<int64_t>(t, budget / std::max<int64_t>(per_sample, 1)));
    B = std::min(B, 1024);
    std::vector<double> dirs((size_t)t * 3 * n), w((size_t)t * n);
    for (int smp = 0; smp < t; ++smp) {
        const int rc = generate_ordinates(spec, seed, first + smp, dirs.data() + (size_t)smp * 3 * n, w.data() + (size_t)smp * n);
        if (rc) return fail(h, rc, "ordinate generation failed");
    }
    std::unique_ptr<Plan>& P = h->ens_plan;
    int done = 0;
    while (done < t) {
        const int b = std::min(B, t - done);
        std::vector<SysInput> in;
        for (int k = 0; k < b; ++k)
            in.push_back({h, dirs.data() + (size_t)(done + k) * 3 * n, w.data() + (size_t)(done + k) * n, n, false});
        char kb[96];
        std::snprintf(kb, sizeof kb, " e%d %d %d %d", spec.kind, n, b, h->scat);
        const std::string key = plan_signature(o, scat_sig(h), 2, b) + kb;
        const int reuse = (P && h->ens_key == key) ? 2 : 0;
        if (!reuse) P.reset();
        h->ens_key.clear();
        SolveResult res;
        const int rc = solve_systems(h, in, o, reuse, P, res);
        if (rc) return rc;
        h->ens_key = key;
        ag.ms += res.ms;
        ag.sweep_ms += res.sweep_ms;
        ag.sweeps += res.sweeps;
        ag.shape[0] = res.tx;
        ag.shape[1] = res.ty;
        ag.shape[2] = res.band;
        ag.shape[3] = res.lanes;
        ag.shape[4] = res.kind;
        for (int k = 0; k < b; ++k) {
            const SysCtl& sc = res.sc[k];
            ag.min_it = std::min(ag.min_it, sc.iter);
            ag.max_it = std::max(ag.max_it, sc.iter);
            ag.updates += (int64_t)sc.iter * h->cells * n;
            if (sc.state == 3) ag.worst = ROM_E_DIVERGED;
            else if (sc.state != 1 && ag.worst == ROM_OK) ag.worst = ROM_NOT_CONVERGED;
        }
        per_batch(*P, done, b);
        done += b;
    }
    return ROM_OK;
}

}  // namespace

extern "C" {

int rom_source_iterate(rom_handle* h, const rom_si_opts* opts, double* phi, rom_si_stats* stats)
{
    ROM_API_LOCK;
    if (!h) return ROM_E_ARG;
    if (h->n == 0) return fail(h, ROM_E_STATE, "set ordinates first");
    if (dense_stale(h)) return fail(h, ROM_E_STATE, "the dense kernel was set for another ordinate set: set it again");
    rom_si_opts o;
    int rc = validate_opts(h, opts, o);
    if (rc) return rc;
    h->res_dev = nullptr;  // set again only when this solve succeeds
    try {
        std::vector<SysInput> in{{h, h->dirs.data(), h->w.data(), h->n, true}};
        const std::string sig = plan_signature(o, scat_sig(h), 0, 1);
        const int reuse = !(h->plan && h->plan_sig == sig) ? 0 : h->plan_version == h->version ? 1 : 2;
        if (!reuse) h->plan.reset();
        SolveResult res;
        rc = solve_systems(h, in, o, reuse, h->plan, res);
        if (rc) return rc;
        h->plan_version = h->version;
        h->plan_sig = sig;
        Plan& P = *h->plan;
        const SysCtl& sc = res.sc[0];
        if (phi) download_phi(P, 0, phi);
        h->res_dev = (const char*)P.d_phi.p + P.sys[0].phi_off * P.esz;
        h->res_fp64 = P.fp64;
        if (stats) {
            stats->iters = sc.iter;
            stats->final_r = sc.r;
            stats->status = sc.state == 1 ? ROM_OK : ROM_NOT_CONVERGED;
            stats->updates = (int64_t)sc.iter * h->cells * h->n;
            stats->device_ms = res.ms;
            stats->sweep_ms = res.sweep_ms;
            stats->sweeps = res.sweeps;
            stats->tile_x = res.tx;
            stats->tile_y = res.ty;
            stats->band = res.band;
            stats->lanes = res.lanes;
            stats->sweep = res.kind;
        }
        if (sc.state == 3) return fail(h, ROM_E_DIVERGED, "non-finite iterate");
        return sc.state == 1 ? ROM_OK : ROM_NOT_CONVERGED;
    } catch (const Fail& f) {
        h->plan.reset();
        return fail(h, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        h->plan.reset();
        return fail(h, ROM_E_NOMEM, "host allocation failed");
    }
}

int rom_solve_batch(rom_handle* const* hs, int32_t k, const rom_si_opts* opts, double* const* phis, rom_si_stats* stats)
{
    ROM_API_LOCK;
    if (!hs || k <= 0) return fail(nullptr, ROM_E_ARG, "need at least one handle");
    rom_handle* h0 = hs[0];
    if (!h0) return fail(nullptr, ROM_E_ARG, "NULL handle");
    for (int i = 0; i < k; ++i) {
        if (!hs[i]) return fail(h0, ROM_E_ARG, "NULL handle in batch");
        if (hs[i]->n == 0) return fail(h0, ROM_E_STATE, "every handle needs ordinates");
        if (dense_stale(hs[i])) return fail(h0, ROM_E_STATE, "a dense kernel was set for another ordinate set: set it again");
        if (hs[i]->user_stream != h0->user_stream) return fail(h0, ROM_E_ARG, "handles must share one stream");
        if (hs[i]->scat == ROM_SCAT_DENSE && k > 1) return fail(h0, ROM_E_UNSUPPORTED, "dense kernels are not batched");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return fail(h0, ROM_E_ARG, "a handle appears twice in the batch");
    }
    rom_si_opts o;
    int rc = validate_opts(h0, opts, o);
    if (rc) return rc;
    h0->res_dev = nullptr;  // a batch leaves no single result on its first handle
    try {
        std::vector<SysInput> in;
        for (int i = 0; i < k; ++i) in.push_back({hs[i], hs[i]->dirs.data(), hs[i]->w.data(), hs[i]->n, true});
        // the batch plan is reused for the same handles in the same order (refreshed if any of
        // them changed ordinates, inflow or kernel since)
        std::string key = plan_signature(o, scat_sig(h0), 1, k), vers;
        for (int i = 0; i < k; ++i) {
            key += " " + std::to_string(hs[i]->uid);
            vers += " " + std::to_string(hs[i]->version);
        }
        std::unique_ptr<Plan>& P = h0->batch_plan;
        const int reuse = !(P && h0->batch_key == key) ? 0 : h0->batch_versions == vers ? 1 : 2;
        if (!reuse) P.reset();
        h0->batch_key.clear();
        SolveResult res;
        rc = solve_systems(h0, in, o, reuse, P, res);
        if (rc) return rc;
        h0->batch_key = key;
        h0->batch_versions = vers;
        int worst = ROM_OK;
        for (int i = 0; i < k; ++i) {
            const SysCtl& sc = res.sc[i];
            if (phis && phis[i]) download_phi(*P, i, phis[i]);
            if (stats) {
                stats[i].iters = sc.iter;
                stats[i].final_r = sc.r;
                stats[i].status = sc.state == 1 ? ROM_OK : ROM_NOT_CONVERGED;
                stats[i].updates = (int64_t)sc.iter * hs[i]->cells * hs[i]->n;
                stats[i].device_ms = res.ms;
                stats[i].sweep_ms = res.sweep_ms;
                stats[i].sweeps = res.sweeps;
                stats[i].tile_x = res.tx;
                stats[i].tile_y = res.ty;
                stats[i].band = res.band;
                stats[i].lanes = res.lanes;
                stats[i].sweep = res.kind;
            }
            if (sc.state == 3) worst = ROM_E_DIVERGED;
            else if (sc.state != 1 && worst == ROM_OK) worst = ROM_NOT_CONVERGED;
        }
        h0->res_dev = nullptr;
        return worst;
    } catch (const Fail& f) {
        return fail(h0, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(h0, ROM_E_NOMEM, "host allocation failed");
    }
}

int rom_ensemble(rom_handle* h, int32_t t, uint64_t seed, const rom_ord_spec* spec, const rom_si_opts* opts, double* mean,
                 double* var, rom_ens_stats* stats)
{
    ROM_API_LOCK;
    if (!h) return ROM_E_ARG;
    if (t <= 0 || !spec) return fail(h, ROM_E_ARG, "t must be > 0 and spec non-NULL");
    rom_si_opts o;
    int rc = check_ensemble(h, *spec, opts, o);
    if (rc) return rc;
    h->res_dev = nullptr;  // the moment buffers and plans are reallocated below
    try {
        hipStream_t s = h->stream();
        // the moment buffers of the previous call are reused when the size matches (each
        // reallocation through an allocator hook waits for the device)
        for (DevMem* d : {&h->ens_mean, &h->ens_m2, &h->ens_var})
            if (!d->p || d->bytes != (size_t)h->cells * 8) HIPCHK(d->alloc(h->cells * 8));
        EnsAgg ag;
        // FP64 moments of each batch, merged into the running ones (eq. (4.6)); the first batch
        // (done = 0) overwrites them.  The flux offsets live with the plan, uploaded once.
        auto moments = [&](Plan& P, int done, int b) {
            if (P.moff_n != b || !P.d_moff.p) {
                std::vector<int64_t> offs(b);
                for (int k = 0; k < b; ++k) offs[k] = P.sys[k].phi_off;
                upload(P.d_moff, offs);
                P.moff_n = b;
            }
            MomentsArgs ma{};
            ma.phi = P.d_phi.p;
            ma.phi_offs = P.d_moff.as<int64_t>();
            ma.t = b;
            ma.count = done;
            ma.cells = h->cells;
            ma.mean = h->ens_mean.as<double>();
            ma.m2 = h->ens_m2.as<double>();
            HIPCHK(launch_moments(ma, P.fp64, s));
        };
        rc = ensemble_batches(h, 0, t, seed, *spec, o, moments, ag);
        if (rc) return rc;
        HIPCHK(launch_finish_var(h->ens_m2.as<double>(), h->ens_var.as<double>(), h->cells, t, s));
        HIPCHK(hipStreamSynchronize(s));
        if (mean) HIPCHK(hipMemcpy(mean, h->ens_mean.p, h->cells * 8, hipMemcpyDeviceToHost));
        if (var) HIPCHK(hipMemcpy(var, h->ens_var.p, h->cells * 8, hipMemcpyDeviceToHost));
        h->res_dev = h->ens_mean.p;
        h->res_fp64 = true;
        ag.fill(stats, t);
        if (ag.worst == ROM_E_DIVERGED) return fail(h, ROM_E_DIVERGED, "non-finite iterate in a sample");
        return ag.worst;
    } catch (const Fail& f) {
        return fail(h, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(h, ROM_E_NOMEM, "host allocation failed");
    }
}

int rom_ensemble_samples(rom_handle* h, int32_t t, uint64_t seed, int64_t first, const rom_ord_spec* spec,
                         const rom_si_opts* opts, double* phis, rom_ens_stats* stats)
{
    ROM_API_LOCK;
    if (!h) return ROM_E_ARG;
    if (t <= 0 || !spec || !phis || first < 0) return fail(h, ROM_E_ARG, "t > 0, first >= 0, spec and phis non-NULL");
    rom_si_opts o;
    int rc = check_ensemble(h, *spec, opts, o);
    if (rc) return rc;
    h->res_dev = nullptr;
    try {
        EnsAgg ag;
        auto download = [&](Plan& P, int done, int b) {
            for (int k = 0; k < b; ++k) download_phi(P, k, phis + (size_t)(done + k) * h->cells);
        };
        rc = ensemble_batches(h, first, t, seed, *spec, o, download, ag);
        if (rc) return rc;
        h->res_dev = nullptr;
        ag.fill(stats, t);
        if (ag.worst == ROM_E_DIVERGED) return fail(h, ROM_E_DIVERGED, "non-finite iterate in a sample");
        return ag.worst;
    } catch (const Fail& f) {
        return fail(h, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        return fail(h, ROM_E_NOMEM, "host allocation failed");
    }
}

}  // extern "C"

// ------------------------------------------------------------------------------------ slab
namespace {

int slab_fail(rom_slab* sl, int code, const std::string& msg)
{
    if (sl) sl->err = msg;
    else g_create_error = msg;
    return code;
}

template <typename T>
std::vector<T> to_type(const double* p, size_t n)
{
    return std::vector<T>(p, p + n);
}

template <typename T>
int slab_run(rom_slab* sl, int t, int n, const double* mu, const double* w, const double* inflow, const rom_si_opts& o,
             double* phis, int32_t* iters, rom_ens_stats* stats)
{
    const int nn = sl->nx + 1;
    const bool fp64 = sizeof(T) == 8;
    // lanes per system: enough for the ordinates (at most 64 per lane), more when the wavefront's
    // LDS (three [nn] arrays per system) would exceed 48 KiB
    int L = 1;
    while (L < 64 && L < n) L *= 2;
    while (L < 64 && slab_lds_bytes(fp64, nn, L) > 48 * 1024) L *= 2;
    if (slab_lds_bytes(fp64, nn, L) > 64 * 1024) return slab_fail(sl, ROM_E_UNSUPPORTED, "slab grid too large for LDS");
    const int K = (n + L - 1) / L;
    const int kmax = K <= 1 ? 1 : K <= 4 ? 4 : K <= 16 ? 16 : 64;
    hipStream_t s = sl->stream();
    DevMem d_mu, d_w, d_in, d_st, d_ss, d_q, d_phi, d_it, d_state, d_r;
    upload(d_mu, to_type<T>(mu, (size_t)t * n));
    upload(d_w, to_type<T>(w, (size_t)t * n));
    upload(d_in, to_type<T>(inflow, (size_t)t * n));
    upload(d_st, to_type<T>(sl->st.data(), nn));
    upload(d_ss, to_type<T>(sl->ss.data(), nn));
    upload(d_q, to_type<T>(sl->q.data(), nn));
    HIPCHK(d_phi.alloc((size_t)t * nn * sizeof(T)));
    HIPCHK(d_it.alloc((size_t)t * 4));
    HIPCHK(d_state.alloc((size_t)t * 4));
    HIPCHK(d_r.alloc((size_t)t * 8));
    SlabArgs a{};
    a.mu = d_mu.p;
    a.w = d_w.p;
    a.inflow = d_in.p;
    a.st = d_st.p;
    a.ss = d_ss.p;
    a.q = d_q.p;
    a.phi = d_phi.p;
    a.iters = d_it.as<int32_t>();
    a.state = d_state.as<int32_t>();
    a.rfinal = d_r.as<double>();
    a.nsys = t;
    a.n = n;
    a.nn = nn;
    a.L = L;
    a.max_iter = o.max_iter;
    a.tol = o.tol;
    a.inv_dx = (double)sl->nx / (sl->x1 - sl->x0);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_slab(a, fp64, kmax, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<T> ph((size_t)t * nn);
    std::vector<int32_t> it(t), st(t);
    HIPCHK(hipMemcpy(ph.data(), d_phi.p, ph.size() * sizeof(T), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(it.data(), d_it.p, (size_t)t * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(st.data(), d_state.p, (size_t)t * 4, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < ph.size(); ++k) phis[k] = (double)ph[k];
    int worst = ROM_OK, mn = 1 << 30, mx = 0;
    int64_t upd = 0;
    for (int k = 0; k < t; ++k) {
        if (iters) iters[k] = it[k];
        mn = std::min(mn, it[k]);
        mx = std::max(mx, it[k]);
        upd += (int64_t)it[k] * n * sl->nx;
        if (st[k] == 3) worst = ROM_E_DIVERGED;
        else if (st[k] != 1 && worst == ROM_OK) worst = ROM_NOT_CONVERGED;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->samples = t;
        stats->min_iters = mn;
        stats->max_iters = mx;
        stats->status = worst == ROM_OK ? ROM_OK : ROM_NOT_CONVERGED;
        stats->updates = upd;
        stats->device_ms = ms;
        stats->lanes = L;
    }
    if (worst == ROM_E_DIVERGED) return slab_fail(sl, ROM_E_DIVERGED, "non-finite iterate in a slab system");
    return worst;
}

}  // namespace

extern "C" {

int rom_slab_create(int32_t nx, double x0, double x1, const double* sigma_t, const double* sigma_s, const double* q,
                    rom_slab** out)
{
    ROM_API_LOCK;
    if (!out) return slab_fail(nullptr, ROM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!sigma_t || !sigma_s || !q) return slab_fail(nullptr, ROM_E_ARG, "NULL field");
    if (nx < 1 || nx > (1 << 24)) return slab_fail(nullptr, ROM_E_ARG, "nx must be in 1 .. 2^24");
    if (!isfin(x0) || !isfin(x1) || !(x1 > x0)) return slab_fail(nullptr, ROM_E_ARG, "need x1 > x0");
    for (int i = 0; i <= nx; ++i) {
        const double st = sigma_t[i], ss = sigma_s[i], qq = q[i];
        if (!isfin(st) || !isfin(ss) || !isfin(qq)) return slab_fail(nullptr, ROM_E_DOMAIN, "non-finite field value");
        if (!(st > 0.0)) return slab_fail(nullptr, ROM_E_DOMAIN, "sigma_t must be > 0");
        if (ss < 0.0 || !(ss < st)) return slab_fail(nullptr, ROM_E_DOMAIN, "need 0 <= sigma_s < sigma_t");
        if (qq < 0.0) return slab_fail(nullptr, ROM_E_DOMAIN, "q must be >= 0");
    }
    try {
        rom_slab* sl = new rom_slab();
        sl->nx = nx;
        sl->x0 = x0;
        sl->x1 = x1;
        sl->st.assign(sigma_t, sigma_t + nx + 1);
        sl->ss.assign(sigma_s, sigma_s + nx + 1);
        sl->q.assign(q, q + nx + 1);
        *out = sl;
        return ROM_OK;
    } catch (const std::bad_alloc&) {
        return slab_fail(nullptr, ROM_E_NOMEM, "host allocation failed");
    }
}

void rom_slab_destroy(rom_slab* sl)
{
    ROM_API_LOCK;
    delete sl;
}

int rom_slab_set_stream(rom_slab* sl, void* stream)
{
    if (!sl) return ROM_E_ARG;
    sl->user_stream = (hipStream_t)stream;
    return ROM_OK;
}

int rom_slab_solve(rom_slab* sl, int32_t t, int32_t n, const double* mu, const double* w, const double* inflow,
                   const rom_si_opts* opts, double* phis, int32_t* iters, rom_ens_stats* stats)
{
    ROM_API_LOCK;
    if (!sl) return ROM_E_ARG;
    if (t < 1 || n < 1 || n > 4096) return slab_fail(sl, ROM_E_ARG, "need t >= 1 and 1 <= n <= 4096");
    if (!mu || !w || !inflow || !phis) return slab_fail(sl, ROM_E_ARG, "NULL mu, w, inflow or phis");
    rom_si_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!isfin(o.tol)) return slab_fail(sl, ROM_E_ARG, "tol must be finite");
    if (o.tol == 0.0) o.tol = 1e-6;
    if (o.max_iter < 0) return slab_fail(sl, ROM_E_ARG, "max_iter must be >= 0");
    if (o.max_iter == 0) o.max_iter = 1000;
    if (o.precision != ROM_PREC_FP32 && o.precision != ROM_PREC_FP64) return slab_fail(sl, ROM_E_ARG, "bad precision");
    for (int k = 0; k < t; ++k) {
        double sum = 0.0;
        for (int l = 0; l < n; ++l) {
            const size_t i = (size_t)k * n + l;
            if (!isfin(mu[i]) || mu[i] == 0.0 || std::fabs(mu[i]) > 1.0)
                return slab_fail(sl, ROM_E_DOMAIN, "every mu must satisfy 0 < |mu| <= 1");
            if (!isfin(w[i]) || !(w[i] > 0.0)) return slab_fail(sl, ROM_E_DOMAIN, "weights must be > 0");
            if (!isfin(inflow[i]) || inflow[i] < 0.0) return slab_fail(sl, ROM_E_DOMAIN, "inflow must be finite and >= 0");
            sum += w[i];
        }
        if (std::fabs(sum - 1.0) > 1e-12) return slab_fail(sl, ROM_E_DOMAIN, "weights of a system must sum to 1");
    }
    try {
        return o.precision == ROM_PREC_FP64 ? slab_run<double>(sl, t, n, mu, w, inflow, o, phis, iters, stats)
                                            : slab_run<float>(sl, t, n, mu, w, inflow, o, phis, iters, stats);
    } catch (const Fail& f) {
        return slab_fail(sl, f.code, f.msg);
    } catch (const std::bad_alloc&) {
        return slab_fail(sl, ROM_E_NOMEM, "host allocation failed");
    }
}

int rom_slab_ordinates(int32_t kind, int32_t n, uint64_t seed, int64_t sample, double* mu, double* w)
{
    if (!mu || !w || n < 1 || sample < 0) return ROM_E_ARG;
    return slab_ordinates(kind, n, seed, sample, mu, w);
}

const char* rom_slab_last_error(const rom_slab* sl) { return sl ? sl->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

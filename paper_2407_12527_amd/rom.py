"""ctypes binding of librom (include/rom.h): same names as the C ABI, argument marshalling only.

Every compute step runs in librom's gfx950 kernels.  The raw functions ``rom_*`` take and return
exactly what the C functions do (numpy arrays are passed as host pointers); ``Handle`` wraps a
``rom_handle*`` with numpy-friendly methods and raises ``RomError`` on negative status codes.
PyTorch is used only for device memory and streams: its caching allocator is installed as
librom's device allocator (``use_torch_allocator``, done when the first handle is created on a
machine with a GPU), it can hand librom a HIP stream (``Handle.use_torch_stream``), and it views
device-resident results (``Handle.phi_device_tensor``).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

__all__ = [
    "ROM_OK", "ROM_NOT_CONVERGED", "ROM_E_ARG", "ROM_E_DOMAIN", "ROM_E_STATE", "ROM_E_NOMEM", "ROM_E_DEVICE",
    "ROM_E_DIVERGED", "ROM_E_UNSUPPORTED", "ROM_SCHEME_STEP", "ROM_SCHEME_DD", "ROM_SCAT_ISO", "ROM_SCAT_LINEAR",
    "ROM_SCAT_HG", "ROM_SCAT_DENSE", "ROM_SCAT_NORMALIZE", "ROM_ORD_STRATIFIED", "ROM_ORD_IID_SPHERE", "ROM_ORD_UNIFORM2D",
    "ROM_ORD_GAUSS2D", "ROM_PREC_FP32", "ROM_PREC_FP64", "ROM_FACE_LEFT", "ROM_FACE_RIGHT", "ROM_FACE_BOTTOM",
    "ROM_FACE_TOP", "rom_grid", "rom_inflow", "rom_ord_spec", "rom_si_opts", "rom_si_stats", "rom_ens_stats",
    "RomError", "Handle", "lib", "library_path", "EXPORTS", "generate_ordinates", "ordinate_count",
    "solve_batch", "si_opts", "rom_create", "rom_destroy", "rom_set_stream", "rom_set_ordinates",
    "rom_set_inflow_angular", "rom_set_scattering", "rom_sweep", "rom_sweep_noalloc", "rom_source_iterate", "rom_ensemble",
    "rom_ensemble_samples", "rom_solve_batch", "rom_phi_device", "rom_generate_ordinates", "rom_ordinate_count", "rom_status_string",
    "rom_last_error", "rom_version", "rom_slab_create", "rom_slab_destroy", "rom_slab_set_stream", "rom_slab_solve",
    "rom_slab_ordinates", "rom_slab_last_error", "ROM_SLAB_RANDOM", "ROM_SLAB_GAUSS", "ROM_SLAB_UNIFORM", "Slab",
    "slab_ordinates", "rom_set_allocator", "use_torch_allocator", "use_hip_allocator",
]

ROM_OK, ROM_NOT_CONVERGED = 0, 1
ROM_E_ARG, ROM_E_DOMAIN, ROM_E_STATE, ROM_E_NOMEM, ROM_E_DEVICE, ROM_E_DIVERGED, ROM_E_UNSUPPORTED = \
    -1, -2, -3, -4, -5, -6, -7
ROM_SCHEME_STEP, ROM_SCHEME_DD = 0, 1
ROM_SCAT_ISO, ROM_SCAT_LINEAR, ROM_SCAT_HG, ROM_SCAT_DENSE = 0, 1, 2, 3
ROM_SCAT_NORMALIZE = 0x10  # flag OR-ed into a kernel kind: rows of P rescaled to unit weighted sum
ROM_ORD_STRATIFIED, ROM_ORD_IID_SPHERE, ROM_ORD_UNIFORM2D, ROM_ORD_GAUSS2D = 0, 1, 2, 3
ROM_PREC_FP32, ROM_PREC_FP64 = 0, 1
ROM_SWEEP_AUTO, ROM_SWEEP_STRIP, ROM_SWEEP_DIAG = 0, 1, 2
ROM_FACE_LEFT, ROM_FACE_RIGHT, ROM_FACE_BOTTOM, ROM_FACE_TOP = 0, 1, 2, 3
ROM_SLAB_RANDOM, ROM_SLAB_GAUSS, ROM_SLAB_UNIFORM = 0, 1, 2

# every function declared in include/rom.h
EXPORTS = ("rom_create", "rom_destroy", "rom_set_stream", "rom_set_allocator", "rom_set_ordinates", "rom_set_inflow_angular",
           "rom_set_scattering", "rom_sweep", "rom_sweep_noalloc", "rom_source_iterate", "rom_ensemble", "rom_ensemble_samples",
           "rom_solve_batch",
           "rom_phi_device", "rom_generate_ordinates", "rom_ordinate_count", "rom_status_string",
           "rom_last_error", "rom_version", "rom_slab_create", "rom_slab_destroy", "rom_slab_set_stream",
           "rom_slab_solve", "rom_slab_ordinates", "rom_slab_last_error")


class rom_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double)]


class rom_inflow(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("bottom", C.c_void_p), ("top", C.c_void_p)]


class rom_ord_spec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p1", C.c_int32), ("p2", C.c_int32)]


class rom_si_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32), ("scheme", C.c_int32),
                ("iters_per_check", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("contract_split", C.c_int32), ("band", C.c_int32), ("sweep", C.c_int32), ("diag_rows", C.c_int32),
                ("diag_k", C.c_int32)]


class rom_si_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("final_r", C.c_double), ("updates", C.c_int64),
                ("device_ms", C.c_double), ("sweep_ms", C.c_double), ("sweeps", C.c_int32), ("tile_x", C.c_int32),
                ("tile_y", C.c_int32), ("band", C.c_int32), ("lanes", C.c_int32), ("sweep", C.c_int32)]


class rom_ens_stats(C.Structure):
    _fields_ = [("samples", C.c_int32), ("min_iters", C.c_int32), ("max_iters", C.c_int32), ("status", C.c_int32),
                ("updates", C.c_int64), ("device_ms", C.c_double), ("sweep_ms", C.c_double), ("sweeps", C.c_int32),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("band", C.c_int32), ("lanes", C.c_int32),
                ("sweep", C.c_int32)]


def library_path() -> str:
    """The in-tree librom.so, or the file named by the ROM_LIBRARY environment variable."""
    env = os.environ.get("ROM_LIBRARY")
    if env:
        return env
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "librom.so")


_lib = None

# rom_set_allocator's callback types: void* alloc(size_t bytes, void* ctx), void free(void* p, void* ctx)
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def lib():
    """Load librom.so (built in-tree by ``build.py``).  Raises if it is missing: there is no
    fallback path."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"librom.so not built ({path}); run `python -m paper_2407_12527_amd.build`")
        L = C.CDLL(path)
        P = C.c_void_p
        PH = C.POINTER(C.c_void_p)
        L.rom_create.argtypes = [C.POINTER(rom_grid), P, P, P, C.POINTER(rom_inflow), PH]
        L.rom_destroy.argtypes = [P]
        L.rom_destroy.restype = None
        L.rom_set_stream.argtypes = [P, P]
        L.rom_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
        L.rom_set_ordinates.argtypes = [P, C.c_int32, P, P]
        L.rom_set_inflow_angular.argtypes = [P, C.c_int32, P]
        L.rom_set_scattering.argtypes = [P, C.c_int32, C.c_double, P]
        L.rom_sweep.argtypes = [P, P, C.c_int32, P, P, C.POINTER(rom_si_opts)]
        L.rom_sweep_noalloc.argtypes = [P, P, P, C.c_int32, P]
        L.rom_source_iterate.argtypes = [P, C.POINTER(rom_si_opts), P, C.POINTER(rom_si_stats)]
        L.rom_ensemble.argtypes = [P, C.c_int32, C.c_uint64, C.POINTER(rom_ord_spec), C.POINTER(rom_si_opts), P, P,
                                   C.POINTER(rom_ens_stats)]
        L.rom_ensemble_samples.argtypes = [P, C.c_int32, C.c_uint64, C.c_int64, C.POINTER(rom_ord_spec),
                                           C.POINTER(rom_si_opts), P, C.POINTER(rom_ens_stats)]
        L.rom_solve_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(rom_si_opts),
                                      C.POINTER(C.c_void_p), C.POINTER(rom_si_stats)]
        L.rom_phi_device.argtypes = [P, C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]
        L.rom_generate_ordinates.argtypes = [C.POINTER(rom_ord_spec), C.c_uint64, C.c_int64, P, P]
        L.rom_ordinate_count.argtypes = [C.POINTER(rom_ord_spec)]
        L.rom_ordinate_count.restype = C.c_int32
        L.rom_status_string.argtypes = [C.c_int]
        L.rom_status_string.restype = C.c_char_p
        L.rom_last_error.argtypes = [P]
        L.rom_last_error.restype = C.c_char_p
        L.rom_version.restype = C.c_char_p
        L.rom_slab_create.argtypes = [C.c_int32, C.c_double, C.c_double, P, P, P, PH]
        L.rom_slab_destroy.argtypes = [P]
        L.rom_slab_destroy.restype = None
        L.rom_slab_set_stream.argtypes = [P, P]
        L.rom_slab_solve.argtypes = [P, C.c_int32, C.c_int32, P, P, P, C.POINTER(rom_si_opts), P, P,
                                     C.POINTER(rom_ens_stats)]
        L.rom_slab_ordinates.argtypes = [C.c_int32, C.c_int32, C.c_uint64, C.c_int64, P, P]
        L.rom_slab_last_error.argtypes = [P]
        L.rom_slab_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# ------------------------------------------------------------------ raw functions (same names)
def rom_create(grid, sigma_t, sigma_s, q, inflow, out):
    return lib().rom_create(grid, sigma_t, sigma_s, q, inflow, out)


def rom_destroy(h):
    return lib().rom_destroy(h)


def rom_set_stream(h, stream):
    return lib().rom_set_stream(h, stream)


def rom_set_allocator(alloc, free, ctx):
    return lib().rom_set_allocator(alloc, free, ctx)


def rom_set_ordinates(h, n, dirs, w):
    return lib().rom_set_ordinates(h, n, dirs, w)


def rom_set_inflow_angular(h, face, vals):
    return lib().rom_set_inflow_angular(h, face, vals)


def rom_set_scattering(h, kind, g, P):
    return lib().rom_set_scattering(h, kind, g, P)


def rom_sweep(h, src, src_per_ordinate, phi, psi, opts):
    return lib().rom_sweep(h, src, src_per_ordinate, phi, psi, opts)


def rom_sweep_noalloc(h, src_dev, phi_dev, precision, stream):
    return lib().rom_sweep_noalloc(h, src_dev, phi_dev, precision, stream)


def rom_source_iterate(h, opts, phi, stats):
    return lib().rom_source_iterate(h, opts, phi, stats)


def rom_ensemble(h, t, seed, spec, opts, mean, var, stats):
    return lib().rom_ensemble(h, t, seed, spec, opts, mean, var, stats)


def rom_ensemble_samples(h, t, seed, first, spec, opts, phis, stats):
    return lib().rom_ensemble_samples(h, t, seed, first, spec, opts, phis, stats)


def rom_slab_create(nx, x0, x1, sigma_t, sigma_s, q, out):
    return lib().rom_slab_create(nx, x0, x1, sigma_t, sigma_s, q, out)


def rom_slab_destroy(s):
    return lib().rom_slab_destroy(s)


def rom_slab_set_stream(s, stream):
    return lib().rom_slab_set_stream(s, stream)


def rom_slab_solve(s, t, n, mu, w, inflow, opts, phis, iters, stats):
    return lib().rom_slab_solve(s, t, n, mu, w, inflow, opts, phis, iters, stats)


def rom_slab_ordinates(kind, n, seed, sample, mu, w):
    return lib().rom_slab_ordinates(kind, n, seed, sample, mu, w)


def rom_slab_last_error(s):
    return lib().rom_slab_last_error(s)


def rom_solve_batch(hs, k, opts, phis, stats):
    return lib().rom_solve_batch(hs, k, opts, phis, stats)


def rom_phi_device(h, dev, is_fp64):
    return lib().rom_phi_device(h, dev, is_fp64)


def rom_generate_ordinates(spec, seed, sample, dirs, w):
    return lib().rom_generate_ordinates(spec, seed, sample, dirs, w)


def rom_ordinate_count(spec):
    return lib().rom_ordinate_count(spec)


def rom_status_string(st):
    return lib().rom_status_string(st)


def rom_last_error(h):
    return lib().rom_last_error(h)


def rom_version():
    return lib().rom_version()


# ------------------------------------------------------------------ helpers
class RomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().rom_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(st, h=None):
    if st < 0:
        raise RomError(st, (lib().rom_last_error(h) or b"").decode())
    return st


# ------------------------------------------------------------------ device memory from PyTorch
_allocator = None      # (alloc callback, free callback) kept alive while installed
_live = weakref.WeakSet()  # handles and slabs to release before the interpreter tears torch down


def use_torch_allocator():
    """Make PyTorch's caching allocator librom's device allocator (rom_set_allocator).  A block
    is taken on the current device and stream after that stream has drained, so no queued torch
    work still uses it; librom waits for the device before it gives a block back."""
    global _allocator
    import torch

    def _alloc(nbytes, ctx):
        try:
            dev = torch.cuda.current_device()
            stream = torch.cuda.current_stream(dev)
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            stream.synchronize()
            return ptr
        except Exception:  # out of memory: librom reports ROM_E_NOMEM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().rom_set_allocator(cbs[0], cbs[1], None))
    _allocator = cbs


def use_hip_allocator():
    """Restore librom's own hipMalloc / hipFree for blocks taken from now on."""
    global _allocator
    _check(lib().rom_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
    # blocks taken from torch are still returned through its callbacks: keep them alive
    if _allocator is not None:
        _retired.append(_allocator)
    _allocator = None


_retired = []
_allocator_checked = False


def _default_allocator():
    """Install torch's allocator once, on the first handle, when a GPU is there."""
    global _allocator_checked
    if _allocator_checked:
        return
    _allocator_checked = True
    try:
        import torch
        if torch.cuda.is_available():
            use_torch_allocator()
    except ImportError:
        pass


@atexit.register
def _release_all():
    # handles still alive at exit give their device memory back while torch is still usable
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def si_opts(tol=1e-6, max_iter=1000, precision=ROM_PREC_FP32, scheme=ROM_SCHEME_STEP, iters_per_check=0,
            tile=(0, 0), contract_split=0, band=0, sweep=0, diag_rows=0, diag_k=0) -> rom_si_opts:
    o = rom_si_opts()
    o.tol = tol
    o.max_iter = max_iter
    o.precision = precision
    o.scheme = scheme
    o.iters_per_check = iters_per_check
    o.tile_x, o.tile_y = tile
    o.contract_split = contract_split
    o.band = band
    o.sweep = sweep
    o.diag_rows = diag_rows
    o.diag_k = diag_k
    return o


def ordinate_count(kind, p1, p2=0) -> int:
    return int(lib().rom_ordinate_count(C.byref(rom_ord_spec(kind, p1, p2))))


def generate_ordinates(kind, p1, p2=0, seed=0, sample=0):
    """Ordinate set of one sample, as librom generates it (host code, no device work)."""
    spec = rom_ord_spec(kind, p1, p2)
    n = lib().rom_ordinate_count(C.byref(spec))
    if n <= 0:
        raise RomError(ROM_E_ARG, "bad ordinate spec")
    dirs = np.empty((n, 3))
    w = np.empty(n)
    _check(lib().rom_generate_ordinates(C.byref(spec), seed, sample, _ptr(dirs), _ptr(w)))
    return dirs, w


class Handle:
    """Owns one ``rom_handle*`` (a problem on the current HIP device)."""

    def __init__(self, nx, ny, sigma_t, sigma_s, q, box=(0.0, 1.0, 0.0, 1.0), inflow=None):
        _default_allocator()
        cells = nx * ny
        self.nx, self.ny, self.cells = int(nx), int(ny), cells
        self._keep = []
        st, ss, qq = _f64(sigma_t, cells), _f64(sigma_s, cells), _f64(q, cells)
        g = rom_grid(nx, ny, *box)
        fin = None
        if inflow:
            fin = rom_inflow()
            for k in ("left", "right", "bottom", "top"):
                v = inflow.get(k)
                if v is not None:
                    v = _f64(v, ny if k in ("left", "right") else nx)
                    self._keep.append(v)
                    setattr(fin, k, v.ctypes.data)
        h = C.c_void_p()
        _check(lib().rom_create(C.byref(g), _ptr(st), _ptr(ss), _ptr(qq), C.byref(fin) if fin else None, C.byref(h)))
        self.h = h
        self.n = 0
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().rom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_ptr):
        _check(lib().rom_set_stream(self.h, C.c_void_p(stream_ptr)), self.h)

    def use_torch_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self.set_stream(s.cuda_stream)

    def set_ordinates(self, dirs, w):
        dirs = _f64(dirs)
        w = _f64(w)
        self.n = int(w.size)
        _check(lib().rom_set_ordinates(self.h, self.n, _ptr(dirs), _ptr(w)), self.h)

    def set_inflow_angular(self, face, vals):
        v = None if vals is None else _f64(vals)
        _check(lib().rom_set_inflow_angular(self.h, face, _ptr(v)), self.h)

    def set_scattering(self, kind, g=0.0, P=None):
        p = None if P is None else _f64(P)
        _check(lib().rom_set_scattering(self.h, kind, g, _ptr(p)), self.h)

    def sweep(self, src, opts=None, want_psi=False):
        src = _f64(src)
        per = 1 if src.size != self.cells else 0
        phi = np.empty(self.cells)
        psi = np.empty((self.n, self.cells)) if want_psi else None
        _check(lib().rom_sweep(self.h, _ptr(src), per, _ptr(phi), _ptr(psi), C.byref(opts) if opts else None), self.h)
        return (phi, psi) if want_psi else phi

    def source_iterate(self, opts=None, download=True):
        phi = np.empty(self.cells) if download else None
        st = rom_si_stats()
        rc = _check(lib().rom_source_iterate(self.h, C.byref(opts) if opts else None, _ptr(phi), C.byref(st)), self.h)
        return phi, st, rc

    def ensemble(self, t, seed, kind, p1, p2=0, opts=None, download=True):
        mean = np.empty(self.cells) if download else None
        var = np.empty(self.cells) if download else None
        st = rom_ens_stats()
        spec = rom_ord_spec(kind, p1, p2)
        rc = _check(lib().rom_ensemble(self.h, t, seed, C.byref(spec), C.byref(opts) if opts else None, _ptr(mean),
                                       _ptr(var), C.byref(st)), self.h)
        return mean, var, st, rc

    def ensemble_samples(self, t, seed, kind, p1, p2=0, first=0, opts=None):
        """Scalar fluxes [t, cells] of samples first .. first + t - 1 of the ensemble (seed, spec)."""
        phis = np.empty((t, self.cells))
        st = rom_ens_stats()
        spec = rom_ord_spec(kind, p1, p2)
        rc = _check(lib().rom_ensemble_samples(self.h, t, seed, first, C.byref(spec), C.byref(opts) if opts else None,
                                               _ptr(phis), C.byref(st)), self.h)
        return phis, st, rc

    def phi_device(self):
        dev = C.c_void_p()
        f64 = C.c_int32()
        _check(lib().rom_phi_device(self.h, C.byref(dev), C.byref(f64)), self.h)
        return dev.value, bool(f64.value)

    def phi_device_tensor(self):
        """Copy of the device-resident result as a torch tensor on the current device."""
        import torch
        ptr, f64 = self.phi_device()
        dt = torch.float64 if f64 else torch.float32
        out = torch.empty(self.cells, dtype=dt, device="cuda")
        _hip_memcpy_d2d(out.data_ptr(), ptr, self.cells * (8 if f64 else 4))
        return out


def solve_batch(handles, opts=None, download=True):
    """rom_solve_batch over the handles; download=False leaves the fluxes on the device
    (outs is then a list of None)."""
    k = len(handles)
    hs = (C.c_void_p * k)(*[h.h for h in handles])
    outs = [np.empty(h.cells) for h in handles] if download else [None] * k
    ps = (C.c_void_p * k)(*[o.ctypes.data for o in outs]) if download else None
    stats = (rom_si_stats * k)()
    rc = lib().rom_solve_batch(hs, k, C.byref(opts) if opts else None, ps, stats)
    if rc < 0:
        raise RomError(rc, (lib().rom_last_error(handles[0].h) or b"").decode())
    return outs, list(stats), rc


_hip = None


def _hip_memcpy_d2d(dst, src, nbytes):
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RomError(ROM_E_DEVICE, f"hipMemcpy failed ({rc})")


# ------------------------------------------------------------------ slab geometry (Sec. 4.1)
def slab_ordinates(kind, n, seed=0, sample=0):
    """Slab ordinate set (host only): ROM_SLAB_RANDOM (sample of seed), ROM_SLAB_GAUSS or
    ROM_SLAB_UNIFORM; weights sum to 1."""
    mu = np.empty(n)
    w = np.empty(n)
    _check(lib().rom_slab_ordinates(kind, n, seed, sample, _ptr(mu), _ptr(w)))
    return mu, w


class Slab:
    """Owns one ``rom_slab*``: a slab problem with fields at the nx + 1 grid points."""

    def __init__(self, nx, sigma_t, sigma_s, q, x0=0.0, x1=1.0):
        _default_allocator()
        self.nx = int(nx)
        self.s = None
        out = C.c_void_p()
        st, ss, qq = _f64(sigma_t, nx + 1), _f64(sigma_s, nx + 1), _f64(q, nx + 1)
        rc = lib().rom_slab_create(self.nx, x0, x1, _ptr(st), _ptr(ss), _ptr(qq), C.byref(out))
        if rc != ROM_OK:
            raise RomError(rc, (lib().rom_slab_last_error(None) or b"").decode())
        self.s = out.value
        _live.add(self)

    def close(self):
        if self.s:
            lib().rom_slab_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, mu, w, inflow, opts=None):
        """t systems: mu, w, inflow are [t, n] (or [n] for one system).  Returns phis [t, nx+1],
        iterations [t], stats, status."""
        mu = np.atleast_2d(_f64(mu))
        t, n = mu.shape
        w = _f64(w, t * n)
        inflow = _f64(inflow, t * n)
        phis = np.empty((t, self.nx + 1))
        iters = np.zeros(t, dtype=np.int32)
        st = rom_ens_stats()
        rc = lib().rom_slab_solve(self.s, t, n, _ptr(mu), _ptr(w), _ptr(inflow), C.byref(opts) if opts else None,
                                  _ptr(phis), iters.ctypes.data, C.byref(st))
        if rc < 0:
            raise RomError(rc, (lib().rom_slab_last_error(self.s) or b"").decode())
        return phis, iters, st, rc

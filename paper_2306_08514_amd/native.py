"""ctypes binding of libsrp.so (the C ABI declared in include/srp.h).

Argument marshalling only: every step of the SRP-map computation runs in the
library's HIP kernels.  torch tensors provide device memory and streams; the
library never sees a torch type.  If the library is missing this module
raises at import of the binding, there is no fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrp.so")

VARIANTS = {"fd": 0, "slri": 1, "sspi": 2, "si": 3, "td": 4, "lr": 5}
DTYPES = {"f32": 0, "bf16": 1, "f16": 2, "fp8": 3, "f64": 4}
STATUS = {0: "SRP_OK", -1: "SRP_E_INVALID", -2: "SRP_E_NOMEM", -3: "SRP_E_UNSUPPORTED",
          -4: "SRP_E_HIP", -5: "SRP_E_BUDGET"}

# every function declared in include/srp.h
EXPORTS = ["srp_default_opts", "srp_plan", "srp_workspace_size", "srp_compute", "srp_compute_static",
           "srp_crossspec", "srp_gcc_samples", "srp_plan_info_get", "srp_plan_export",
           "srp_profile_enable", "srp_profile_collect", "srp_destroy", "srp_last_error", "srp_argmax"]


STATIC_SCRATCH_BYTES = 128 << 20  # SRP_STATIC_SCRATCH_BYTES of include/srp.h


class SrpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("n_aux", ctypes.c_int), ("dtype", ctypes.c_int),
                ("device", ctypes.c_int), ("frame_tile", ctypes.c_int64),
                ("hbm_budget", ctypes.c_size_t), ("sampling", ctypes.c_int),
                ("fd_steering", ctypes.c_int), ("far_field", ctypes.c_int),
                ("global_fit", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("P", ctypes.c_int), ("K", ctypes.c_int),
                ("J", ctypes.c_int64), ("PN", ctypes.c_int), ("max_np", ctypes.c_int),
                ("rank_or_q", ctypes.c_int), ("variant", ctypes.c_int), ("dtype", ctypes.c_int),
                ("mean_n", ctypes.c_double), ("macs_per_map", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("plan_seconds", ctypes.c_double),
                ("map_pitch", ctypes.c_int64), ("sampling_fft", ctypes.c_int),
                ("fd_generated", ctypes.c_int), ("sspi_dense_tiles", ctypes.c_int),
                ("sspi_gather_tiles", ctypes.c_int), ("sspi_band_tiles", ctypes.c_int)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_int64)]


_lib = None


def lib():
    """Loads libsrp.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2306_08514_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    L.srp_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.srp_default_opts.restype = None
    L.srp_plan.argtypes = [dp, ctypes.c_int, dp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.srp_plan.restype = ctypes.c_int
    L.srp_workspace_size.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.srp_workspace_size.restype = ctypes.c_int
    L.srp_compute.argtypes = [vp, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
    L.srp_compute.restype = ctypes.c_int
    L.srp_compute_static.argtypes = [vp, vp, i64, vp, i64, vp]
    L.srp_compute_static.restype = ctypes.c_int
    L.srp_crossspec.argtypes = [vp, vp, i64, vp, vp]
    L.srp_crossspec.restype = ctypes.c_int
    L.srp_gcc_samples.argtypes = [vp, vp, i64, vp, vp]
    L.srp_gcc_samples.restype = ctypes.c_int
    L.srp_plan_info_get.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.srp_plan_info_get.restype = ctypes.c_int
    L.srp_plan_export.argtypes = [vp, ctypes.c_char_p, vp, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_size_t)]
    L.srp_plan_export.restype = ctypes.c_int
    L.srp_profile_enable.argtypes = [vp, ctypes.c_int]
    L.srp_profile_enable.restype = ctypes.c_int
    L.srp_profile_collect.argtypes = [vp, ctypes.POINTER(KernelTime), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
    L.srp_profile_collect.restype = ctypes.c_int
    L.srp_destroy.argtypes = [vp]
    L.srp_destroy.restype = None
    L.srp_argmax.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp, vp]
    L.srp_argmax.restype = ctypes.c_int
    L.srp_last_error.argtypes = []
    L.srp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise SrpError(code, lib().srp_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def argmax(maps, stream=None):
    """Per-map peak (10)-(11) on the device: (idx int64 [L], val float64 [L])
    for an [L, J] float32/float64 CUDA tensor with unit column stride; ties go
    to the smallest index, NaN never wins (idx -1 if a row is all NaN)."""
    import torch
    if maps.dim() != 2 or not maps.is_cuda or maps.dtype not in (torch.float32, torch.float64):
        raise ValueError("maps must be a 2-D float32/float64 CUDA tensor")
    L, J = maps.shape
    if J > 1 and maps.stride(1) != 1:
        raise ValueError("maps must have unit column stride")
    idx = torch.empty(L, dtype=torch.int64, device=maps.device)
    val = torch.empty(L, dtype=torch.float64, device=maps.device)
    ld = maps.stride(0) if L > 1 else J
    _check(lib().srp_argmax(_ptr(maps), DTYPES["f64" if maps.dtype == torch.float64 else "f32"], L, J, ld,
                            _ptr(idx), _ptr(val), _stream_handle(stream)))
    return idx, val


class Plan:
    """An SRP-map plan: geometry-dependent operands resident on one device.

    mics [M, 3], grid [J, 3] in metres (host arrays, copied); fs in Hz; N the
    DFT length; variant in {"fd", "slri", "sspi", "si", "td", "lr"};
    rank_or_q = R per pair (SLRI), Q per (location, pair) (SSPI) or R_H
    (LR-SRP), ignored for FD, SI and TD; dtype in {"f32", "bf16", "f16",
    "fp8", "f64"}; device = -1 builds the host-side plan only; sampling in
    {"auto", "direct", "fft"} selects the GCC sampling form of SLRI/SSPI;
    fd_steering in {"auto", "resident", "generated"} the FD steering operand;
    far_field=True reads the grid rows as unit source directions;
    global_fit=True selects the global forms: SLRI with rank_or_q = the
    total rank R_Lambda, SSPI with Q_Lambda = rank_or_q J P kept entries;
    global_fit="randomized" fits the global SLRI by randomized subspace
    iteration at any PN (the form used above PN = 4096)."""

    SAMPLING = {"auto": 0, "direct": 1, "fft": 2}
    STEERING = {"auto": 0, "resident": 1, "generated": 2}

    def __init__(self, mics, grid, fs, N, variant, rank_or_q=0, dtype="f32", c=343.0, n_aux=2,
                 device=0, frame_tile=1024, hbm_budget=0, sampling="auto", fd_steering="auto",
                 far_field=False, global_fit=False):
        L = lib()
        mics = np.ascontiguousarray(mics, dtype=np.float64)
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        o = Opts()
        L.srp_default_opts(ctypes.byref(o))
        o.c, o.n_aux, o.dtype, o.device = float(c), int(n_aux), DTYPES[dtype], int(device)
        o.frame_tile, o.hbm_budget = int(frame_tile), int(hbm_budget)
        o.sampling = self.SAMPLING[sampling]
        o.fd_steering = self.STEERING[fd_steering]
        o.far_field = 1 if far_field else 0
        o.global_fit = 2 if global_fit == "randomized" else (1 if global_fit else 0)
        h = ctypes.c_void_p()
        self._h = None
        self._mics_ref = mics
        _check(L.srp_plan(mics.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mics.shape[0],
                          grid.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), grid.shape[0],
                          float(fs), int(N), VARIANTS[variant], int(rank_or_q), ctypes.byref(o),
                          ctypes.byref(h)))
        self._h = h
        self.variant, self.dtype, self.device = variant, dtype, int(device)
        self.N, self.K = int(N), int(N) // 2
        i = self.info()
        self.M, self.P, self.J, self.PN = i["M"], i["P"], i["J"], i["PN"]
        self.map_pitch = int(i["map_pitch"])

    # ---------------------------------------------------------------- info --
    def info(self):
        pi = PlanInfo()
        _check(lib().srp_plan_info_get(self._h, ctypes.byref(pi)))
        return {f: getattr(pi, f) for f, _ in PlanInfo._fields_}

    def export(self, what):
        need = ctypes.c_size_t()
        _check(lib().srp_plan_export(self._h, what.encode(), None, 0, ctypes.byref(need)))
        dt = np.int32 if what in ("np", "pairs", "sspi_start") else np.float64
        buf = np.empty(need.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().srp_plan_export(self._h, what.encode(), buf.ctypes.data_as(ctypes.c_void_p),
                                     buf.nbytes, ctypes.byref(need)))
        return buf

    def workspace_size(self, L):
        b = ctypes.c_size_t()
        _check(lib().srp_workspace_size(self._h, int(L), ctypes.byref(b)))
        return b.value

    # ------------------------------------------------------------- compute --
    def _check_frames(self, frames):
        import torch
        if frames.dtype != torch.complex64 or not frames.is_cuda or not frames.is_contiguous():
            raise ValueError("frames must be a contiguous complex64 CUDA tensor")
        if frames.dim() != 3 or frames.shape[1] != self.M or frames.shape[2] != self.K + 1:
            raise ValueError(f"frames must have shape [L, {self.M}, {self.K + 1}]")

    def empty_maps(self, L, device=None):
        """An [L, J] output view over rows of map_pitch elements (the pitch at
        which the map stores run fastest)."""
        import torch
        odt = torch.float64 if self.dtype == "f64" else torch.float32
        buf = torch.empty((L, self.map_pitch), dtype=odt, device=device or torch.device("cuda", max(self.device, 0)))
        return buf[:, :self.J]

    def compute(self, frames, maps=None, workspace=None, stream=None):
        """Enqueues one map per frame; returns maps [L, J] (float32, float64
        for f64 plans).  frames: complex64 CUDA tensor [L, M, N/2 + 1].  maps
        may be any [L, J] view with unit column stride and row stride >= J
        (the row stride is passed as the pitch); by default a view at the
        plan's map_pitch is allocated."""
        import torch
        self._check_frames(frames)
        L = frames.shape[0]
        odt = torch.float64 if self.dtype == "f64" else torch.float32
        if maps is None:
            maps = self.empty_maps(L, frames.device)
        elif (maps.dtype != odt or tuple(maps.shape) != (L, self.J) or not maps.is_cuda
              or (L > 0 and self.J > 1 and maps.stride(1) != 1) or (L > 1 and maps.stride(0) < self.J)):
            raise ValueError("maps must be an [L, J] CUDA tensor of the plan's output dtype with unit "
                             "column stride and row stride >= J")
        ld = maps.stride(0) if L > 1 else self.J
        ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        _check(lib().srp_compute(self._h, _ptr(frames), L, _ptr(maps), ld, _ptr(workspace), ws_bytes,
                                 _stream_handle(stream)))
        return maps

    def compute_static(self, frames, maps, stream=None):
        """srp_compute_static: the maps of compute() into the given [L, J]
        view (same layout rules), with the library's static per-GPU scratch
        as the workspace and no allocation."""
        import torch
        self._check_frames(frames)
        L = frames.shape[0]
        odt = torch.float64 if self.dtype == "f64" else torch.float32
        if (maps.dtype != odt or tuple(maps.shape) != (L, self.J) or not maps.is_cuda
                or (L > 0 and self.J > 1 and maps.stride(1) != 1) or (L > 1 and maps.stride(0) < self.J)):
            raise ValueError("maps must be an [L, J] CUDA tensor of the plan's output dtype with unit "
                             "column stride and row stride >= J")
        ld = maps.stride(0) if L > 1 else self.J
        _check(lib().srp_compute_static(self._h, _ptr(frames), L, _ptr(maps), ld, _stream_handle(stream)))
        return maps

    def crossspec(self, frames, stream=None):
        import torch
        self._check_frames(frames)
        out = torch.empty((frames.shape[0], self.P, self.K - 1), dtype=torch.complex64,
                          device=frames.device)
        _check(lib().srp_crossspec(self._h, _ptr(frames), frames.shape[0], _ptr(out),
                                   _stream_handle(stream)))
        return out

    def gcc_samples(self, frames, stream=None):
        import torch
        self._check_frames(frames)
        out = torch.empty((frames.shape[0], self.PN), dtype=torch.float32, device=frames.device)
        _check(lib().srp_gcc_samples(self._h, _ptr(frames), frames.shape[0], _ptr(out),
                                     _stream_handle(stream)))
        return out

    def profile(self, enable=True):
        """Turns per-kernel event timing on or off (see srp_profile_enable)."""
        _check(lib().srp_profile_enable(self._h, 1 if enable else 0))

    def profile_collect(self):
        """{kernel name: (total ms, launches)} since the previous collect."""
        arr = (KernelTime * 32)()
        n = ctypes.c_int()
        _check(lib().srp_profile_collect(self._h, arr, 32, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].total_ms, arr[i].launches) for i in range(min(n.value, 32))}

    def close(self):
        if getattr(self, "_h", None):
            lib().srp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

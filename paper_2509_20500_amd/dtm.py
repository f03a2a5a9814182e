"""Python binding of the C-ABI in include/dtm.h (ctypes).

Argument marshalling only: every step of the method runs in the HIP library.
Functions named ``dtm_*`` mirror the C entry points one to one and take raw
integers for device pointers and streams.  The few helpers below them accept
torch tensors and pass their ``data_ptr()`` and the current HIP stream.

Loading fails loudly (``RuntimeError``) when ``libdtm.so`` has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtm.so")

DTM_OK = 0
DTM_EINVAL = -1
DTM_ENOTCONV = -2
DTM_EHIP = -3
DTM_EALIAS = -4
DTM_ENOSPACE = -5
DTM_ENOTSUP = -6

DTM_F64 = 0
DTM_F32 = 1

DTM_STOP_CHANGE = 0
DTM_STOP_BOUND = 1
DTM_FLAG_NO_FINAL_CHECK = 0x1
DTM_FLAG_NO_DENSE = 0x2
DTM_FLAG_SHIFT_NEAREST = 0x4
DTM_FLAG_SHIFT_INTERP = 0x8
DTM_FLAG_LAMBDA_BIN_MEAN = 0x10
DTM_FLAG_BIN_INTEGRAL = 0x20
DTM_FLAG_START_FLUX = 0x40

DTM_INFO_WARM_REJECTED = 0x1
DTM_INFO_RESTARTED = 0x2
DTM_INFO_CHECKED = 0x4
DTM_INFO_STALLED = 0x8
DTM_INFO_REFINED = 0x10
DTM_INFO_CONTINUED = 0x20

DTM_SPECTRAL_UNSETTLED = 0x1
DTM_SPECTRAL_TIED = 0x2

DTM_MAX_BINS = 65536
DTM_NOALLOC_MAX_BINS = 8192
DTM_NOALLOC_SCRATCH_BYTES = 8912896

SYMBOLS = [
    "dtm_status_string", "dtm_version", "dtm_validate_scene", "dtm_shift_bins", "dtm_model_shift",
    "dtm_workspace_bytes", "dtm_bin_tables", "dtm_build_base", "dtm_apply_deadtime_shift",
    "dtm_build_transition", "dtm_stationary_pdf", "dtm_plan_create", "dtm_plan_destroy",
    "dtm_plan_workspace_bytes", "dtm_plan_pi_elems", "dtm_plan_matrix_elems", "dtm_plan_offsets",
    "dtm_plan_tiles", "dtm_plan_bind", "dtm_solve_batched", "dtm_build_base_batched",
    "dtm_apply_deadtime_shift_batched", "dtm_build_transition_batched",
    "dtm_graph_create", "dtm_graph_launch", "dtm_graph_destroy",
    "dtm_mlp_workspace_layout", "dtm_mlp_features", "dtm_mlp_flux_prior", "dtm_mlp_sync_bf16", "dtm_mlp_forward",
    "dtm_mlp_backward", "dtm_mlp_adam", "dtm_mlp_gemm_bf16",
    "dtm_solve_factored_batched", "dtm_spectral_scratch_bytes", "dtm_spectral_batched",
    "dtm_mc_scratch_bytes", "dtm_mc_histograms", "dtm_stationary_pdf_noalloc",
]


class Scene(ctypes.Structure):
    _fields_ = [
        ("period_ns", ctypes.c_double), ("dead_time_ns", ctypes.c_double),
        ("pulse_center_ns", ctypes.c_double), ("pulse_sigma_ns", ctypes.c_double),
        ("signal_flux", ctypes.c_double), ("background_flux", ctypes.c_double),
        ("n_bins", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("tol_l1", ctypes.c_double), ("safety", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("dense_sweeps", ctypes.c_int32),
        ("change_l1", ctypes.c_double), ("residual_l1", ctypes.c_double),
        ("rho_hat", ctypes.c_double),
    ]


class TileConfig(ctypes.Structure):
    _fields_ = [
        ("fused_threads", ctypes.c_int32), ("fused_unroll", ctypes.c_int32),
        ("fused_max_bins", ctypes.c_int32), ("band_rows", ctypes.c_int32),
        ("dense_sweeps", ctypes.c_int32), ("band_cpt", ctypes.c_int32), ("independent_paths", ctypes.c_int32),
        ("fused_blocks", ctypes.c_int32), ("band_min_items", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"fused_threads": self.fused_threads, "fused_unroll": self.fused_unroll,
                "fused_max_bins": self.fused_max_bins, "band_rows": self.band_rows,
                "dense_sweeps": self.dense_sweeps, "band_cpt": self.band_cpt,
                "independent_paths": self.independent_paths, "fused_blocks": self.fused_blocks,
                "band_min_items": self.band_min_items}


def tiles(fused_threads=0, fused_unroll=0, fused_max_bins=0, band_rows=0, dense_sweeps=0, band_cpt=0,
          independent_paths=0, fused_blocks=0, band_min_items=0):
    return TileConfig(fused_threads, fused_unroll, fused_max_bins, band_rows, dense_sweeps, band_cpt,
                      independent_paths, fused_blocks, band_min_items)


SPECTRAL_INFO_DTYPE = np.dtype([
    ("lambda2_re", "<f8"), ("lambda2_im", "<f8"), ("lambda2_abs", "<f8"), ("lambda2_arg", "<f8"),
    ("lambda3_abs", "<f8"), ("ritz_change", "<f8"), ("iterations", "<i4"), ("mixing_steps", "<i4"),
    ("flags", "<i4"), ("reserved", "<i4"),
])
assert SPECTRAL_INFO_DTYPE.itemsize == 64
SPECTRAL_INFO_BYTES = SPECTRAL_INFO_DTYPE.itemsize

SOLVE_INFO_DTYPE = np.dtype([
    ("iterations", "<i4"), ("status", "<i4"), ("flags", "<i4"), ("dense_sweeps", "<i4"),
    ("change_l1", "<f8"), ("residual_l1", "<f8"), ("rho_hat", "<f8"),
])
assert SOLVE_INFO_DTYPE.itemsize == ctypes.sizeof(SolveInfo) == 40
assert ctypes.sizeof(Scene) == 56

_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double


def lib() -> ctypes.CDLL:
    """The loaded library; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2509_20500_amd.build` "
            "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dtm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "dtm_version": (ctypes.c_int, []),
        "dtm_validate_scene": (ctypes.c_int, [ctypes.POINTER(Scene)]),
        "dtm_shift_bins": (ctypes.c_int, [ctypes.POINTER(Scene), ctypes.POINTER(_I32)]),
        "dtm_model_shift": (ctypes.c_int, [ctypes.POINTER(Scene), _I32, ctypes.POINTER(_I32),
                                           ctypes.POINTER(ctypes.c_double)]),
        "dtm_workspace_bytes": (_SZ, [_I32, ctypes.c_int]),
        "dtm_bin_tables": (ctypes.c_int, [ctypes.POINTER(Scene), ctypes.c_int, _P, _P, _P, _SZ, _P]),
        "dtm_build_base": (ctypes.c_int, [ctypes.POINTER(Scene), ctypes.c_int, _P, _I64, _P, _SZ, _P]),
        "dtm_apply_deadtime_shift": (ctypes.c_int, [ctypes.POINTER(Scene), ctypes.c_int, _P, _P, _I64, _P]),
        "dtm_build_transition": (ctypes.c_int, [ctypes.POINTER(Scene), ctypes.c_int, _P, _I64, _P, _SZ, _P]),
        "dtm_stationary_pdf": (ctypes.c_int, [_P, _I32, _I64, ctypes.c_int, ctypes.POINTER(SolveOpts),
                                              _P, _P, _P, _SZ, ctypes.POINTER(SolveInfo), _P]),
        "dtm_stationary_pdf_noalloc": (ctypes.c_int, [_P, _I32, _I64, ctypes.c_int, ctypes.POINTER(SolveOpts),
                                                      _P, _P, ctypes.POINTER(SolveInfo), _P]),
        "dtm_plan_create": (ctypes.c_int, [_P, _I32, ctypes.c_int, ctypes.POINTER(SolveOpts),
                                           ctypes.POINTER(TileConfig), ctypes.POINTER(_P)]),
        "dtm_plan_destroy": (None, [_P]),
        "dtm_plan_workspace_bytes": (_SZ, [_P]),
        "dtm_plan_pi_elems": (_I64, [_P]),
        "dtm_plan_matrix_elems": (_I64, [_P]),
        "dtm_plan_offsets": (ctypes.c_int, [_P, _P, _P]),
        "dtm_plan_tiles": (ctypes.c_int, [_P, ctypes.POINTER(TileConfig)]),
        "dtm_plan_bind": (ctypes.c_int, [_P, _P, _SZ, _P]),
        "dtm_solve_batched": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "dtm_build_base_batched": (ctypes.c_int, [_P, _P, _P]),
        "dtm_apply_deadtime_shift_batched": (ctypes.c_int, [_P, _P, _P, _P]),
        "dtm_build_transition_batched": (ctypes.c_int, [_P, _P, _P]),
        "dtm_graph_create": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
        "dtm_graph_launch": (ctypes.c_int, [_P, _P]),
        "dtm_graph_destroy": (None, [_P]),
        "dtm_solve_factored_batched": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "dtm_spectral_scratch_bytes": (_SZ, [_P, _I32]),
        "dtm_spectral_batched": (ctypes.c_int, [_P, _D, _I32, _P, _P, _SZ, _P]),
        "dtm_mc_scratch_bytes": (_SZ, [_P, _I32, _I64, _I32]),
        "dtm_mc_histograms": (ctypes.c_int, [_P, _I32, _I64, _I64, ctypes.c_uint64, _I32, _I32, _P, _P, _P,
                                             _SZ, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class DtmError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = lib().dtm_status_string(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


def check(status, what=""):
    if status != DTM_OK:
        raise DtmError(status, what)
    return status


# ---- scene marshalling --------------------------------------------------------

def scene_struct(rec) -> Scene:
    r = np.asarray(rec).reshape(-1)[0]
    return Scene(float(r["period_ns"]), float(r["dead_time_ns"]), float(r["pulse_center_ns"]),
                 float(r["pulse_sigma_ns"]), float(r["signal_flux"]), float(r["background_flux"]),
                 int(r["n_bins"]), int(r["reserved"]))


def _scene_array(scenes):
    arr = np.ascontiguousarray(scenes)
    if arr.dtype.itemsize != 56:
        raise ValueError("scenes must use the 56-byte dtm_scene layout")
    return arr


def _dt(dtype) -> int:
    import torch
    if dtype in (DTM_F32, "f32", "float32", np.float32, torch.float32):
        return DTM_F32
    if dtype in (DTM_F64, "f64", "float64", np.float64, torch.float64):
        return DTM_F64
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def opts(tol=1e-6, safety=0.25, max_iter=1000, check_every=4, stop_rule=DTM_STOP_BOUND, flags=0):
    return SolveOpts(tol, safety, max_iter, check_every, stop_rule, flags)


# ---- raw entry points (same names as the C-ABI) --------------------------------

def dtm_status_string(status: int) -> str:
    return lib().dtm_status_string(status).decode()


def dtm_version() -> int:
    return lib().dtm_version()


def dtm_validate_scene(scene) -> int:
    s = scene_struct(scene)
    return lib().dtm_validate_scene(ctypes.byref(s))


def dtm_shift_bins(scene) -> int:
    s = scene_struct(scene)
    out = _I32(0)
    check(lib().dtm_shift_bins(ctypes.byref(s), ctypes.byref(out)), "dtm_shift_bins")
    return out.value


def dtm_model_shift(scene, flags):
    """(l, frac) of a plan's pixel under the discretisation flags."""
    s = scene_struct(scene)
    l, f = _I32(0), ctypes.c_double(0.0)
    check(lib().dtm_model_shift(ctypes.byref(s), int(flags), ctypes.byref(l), ctypes.byref(f)),
          "dtm_model_shift")
    return l.value, f.value


def dtm_workspace_bytes(n: int, dtype) -> int:
    return lib().dtm_workspace_bytes(n, _dt(dtype))


def dtm_bin_tables(scene, dtype, lambda_ptr, F_ptr, ws_ptr, ws_bytes, stream) -> int:
    s = scene_struct(scene)
    return lib().dtm_bin_tables(ctypes.byref(s), _dt(dtype), lambda_ptr, F_ptr, ws_ptr, ws_bytes, stream)


def dtm_build_base(scene, dtype, P_ptr, ld, ws_ptr, ws_bytes, stream) -> int:
    s = scene_struct(scene)
    return lib().dtm_build_base(ctypes.byref(s), _dt(dtype), P_ptr, ld, ws_ptr, ws_bytes, stream)


def dtm_apply_deadtime_shift(scene, dtype, P_base_ptr, P_ptr, ld, stream) -> int:
    s = scene_struct(scene)
    return lib().dtm_apply_deadtime_shift(ctypes.byref(s), _dt(dtype), P_base_ptr, P_ptr, ld, stream)


def dtm_build_transition(scene, dtype, P_ptr, ld, ws_ptr, ws_bytes, stream) -> int:
    s = scene_struct(scene)
    return lib().dtm_build_transition(ctypes.byref(s), _dt(dtype), P_ptr, ld, ws_ptr, ws_bytes, stream)


def dtm_stationary_pdf(P_ptr, n, ld, dtype, solve_opts, x0_ptr, pi_ptr, ws_ptr, ws_bytes, stream):
    info = SolveInfo()
    o = solve_opts if solve_opts is not None else None
    st = lib().dtm_stationary_pdf(P_ptr, n, ld, _dt(dtype), ctypes.byref(o) if o is not None else None,
                                  x0_ptr, pi_ptr, ws_ptr, ws_bytes, ctypes.byref(info), stream)
    return st, info


def dtm_stationary_pdf_noalloc(P_ptr, n, ld, dtype, solve_opts, x0_ptr, pi_ptr, stream):
    info = SolveInfo()
    o = solve_opts if solve_opts is not None else None
    st = lib().dtm_stationary_pdf_noalloc(P_ptr, n, ld, _dt(dtype), ctypes.byref(o) if o is not None else None,
                                          x0_ptr, pi_ptr, ctypes.byref(info), stream)
    return st, info


# ---- tensor helpers --------------------------------------------------------------

def _ptr(t):
    return None if t is None else t.data_ptr()


def workspace(n, dtype, device="cuda"):
    import torch
    nbytes = dtm_workspace_bytes(n, dtype)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def bin_tables(scene, lam, F, ws, stream=None):
    """lambda_j into ``lam`` (n, f32/f64) and F_j into ``F`` (n+1, f64)."""
    dt = _dt(lam.dtype)
    check(dtm_bin_tables(scene, dt, _ptr(lam), _ptr(F), _ptr(ws), ws.numel(), _stream(stream)),
          "dtm_bin_tables")


def build_base(scene, P, ws, stream=None):
    check(dtm_build_base(scene, _dt(P.dtype), _ptr(P), P.stride(0), _ptr(ws), ws.numel(),
                         _stream(stream)), "dtm_build_base")


def build_transition(scene, P, ws, stream=None):
    check(dtm_build_transition(scene, _dt(P.dtype), _ptr(P), P.stride(0), _ptr(ws), ws.numel(),
                               _stream(stream)), "dtm_build_transition")


def apply_deadtime_shift(scene, P_base, P, stream=None):
    if P_base.stride(0) != P.stride(0):
        raise ValueError("P_base and P must share the row stride")
    check(dtm_apply_deadtime_shift(scene, _dt(P.dtype), _ptr(P_base), _ptr(P), P.stride(0),
                                   _stream(stream)), "dtm_apply_deadtime_shift")


def stationary_pdf(P, pi, ws, solve_opts=None, x0=None, stream=None) -> SolveInfo:
    n = P.shape[0]
    st, info = dtm_stationary_pdf(_ptr(P), n, P.stride(0), _dt(P.dtype), solve_opts, _ptr(x0),
                                  _ptr(pi), _ptr(ws), ws.numel(), _stream(stream))
    check(st, "dtm_stationary_pdf")
    return info


def stationary_pdf_noalloc(P, pi, solve_opts=None, x0=None, stream=None) -> SolveInfo:
    n = P.shape[0]
    st, info = dtm_stationary_pdf_noalloc(_ptr(P), n, P.stride(0), _dt(P.dtype), solve_opts, _ptr(x0), _ptr(pi),
                                          _stream(stream))
    check(st, "dtm_stationary_pdf_noalloc")
    return info


class Plan:
    """A batched plan (dtm_plan_*); owns nothing on the device."""

    def __init__(self, scenes, dtype, solve_opts=None, tiles=None):
        arr = _scene_array(scenes)
        self._scenes = arr
        self.dtype = _dt(dtype)
        self.n_pixels = arr.size
        h = _P()
        check(lib().dtm_plan_create(arr.ctypes.data, arr.size, self.dtype,
                                    ctypes.byref(solve_opts) if solve_opts is not None else None,
                                    ctypes.byref(tiles) if tiles is not None else None,
                                    ctypes.byref(h)), "dtm_plan_create")
        self.handle = h
        self.workspace_bytes = lib().dtm_plan_workspace_bytes(h)
        self.pi_elems = lib().dtm_plan_pi_elems(h)
        self.matrix_elems = lib().dtm_plan_matrix_elems(h)
        pi_off = np.zeros(self.n_pixels + 1, dtype=np.int64)
        mat_off = np.zeros(self.n_pixels + 1, dtype=np.int64)
        check(lib().dtm_plan_offsets(h, pi_off.ctypes.data, mat_off.ctypes.data), "dtm_plan_offsets")
        self.pi_offsets = pi_off
        self.mat_offsets = mat_off
        t = TileConfig()
        check(lib().dtm_plan_tiles(h, ctypes.byref(t)), "dtm_plan_tiles")
        self.tiles = t

    def bind(self, ws, stream=None):
        check(lib().dtm_plan_bind(self.handle, _ptr(ws), ws.numel(), _stream(stream)), "dtm_plan_bind")

    def solve(self, pi, infos, x0=None, stream=None):
        check(lib().dtm_solve_batched(self.handle, _ptr(x0), _ptr(pi), _ptr(infos), _stream(stream)),
              "dtm_solve_batched")

    def build_base(self, P, stream=None):
        check(lib().dtm_build_base_batched(self.handle, _ptr(P), _stream(stream)), "dtm_build_base_batched")

    def build_transition(self, P, stream=None):
        check(lib().dtm_build_transition_batched(self.handle, _ptr(P), _stream(stream)),
              "dtm_build_transition_batched")

    def apply_deadtime_shift(self, P_base, P, stream=None):
        check(lib().dtm_apply_deadtime_shift_batched(self.handle, _ptr(P_base), _ptr(P), _stream(stream)),
              "dtm_apply_deadtime_shift_batched")

    def solve_factored(self, pi, infos, x0=None, stream=None):
        """Power iteration on the factored matrix (O(n) per sweep, float64)."""
        check(lib().dtm_solve_factored_batched(self.handle, _ptr(x0), _ptr(pi), _ptr(infos),
                                               _stream(stream)), "dtm_solve_factored_batched")

    def spectral_scratch_bytes(self, with_mixing=False):
        return lib().dtm_spectral_scratch_bytes(self.handle, int(with_mixing))

    def spectral(self, out, scratch, mixing_eps=0.0, max_steps=10000, stream=None):
        """lambda_2 (and mixing steps when mixing_eps > 0) of every pixel into
        ``out`` (uint8 tensor of 48 bytes per pixel)."""
        check(lib().dtm_spectral_batched(self.handle, float(mixing_eps), int(max_steps), _ptr(out),
                                         _ptr(scratch), scratch.numel(), _stream(stream)),
              "dtm_spectral_batched")

    def mc_scratch_bytes(self, runs, cycles, segments_per_run=0):
        return int(lib().dtm_mc_scratch_bytes(self.handle, int(runs), int(cycles), int(segments_per_run)))

    def mc_histograms(self, runs, cycles, burn, seed, lanes_per_run=0, stream=None, hist=None, over=None,
                      segments_per_run=0, scratch=None):
        """Monte Carlo registration counts (packed like pi, uint32 held in an
        int32 tensor) and per-pixel overflow flags.  hist/over may be given
        (int32 CUDA tensors of pi_elems and n_pixels elements); over is
        cleared here.  scratch (a uint8 CUDA tensor of at least
        mc_scratch_bytes bytes) is allocated here when not given; it must
        outlive the launches."""
        import torch
        if hist is None:
            hist = torch.empty(self.pi_elems, dtype=torch.int32, device="cuda")
        if over is None:
            over = torch.zeros(self.n_pixels, dtype=torch.int32, device="cuda")
        else:
            over.zero_()
        if hist.numel() < self.pi_elems or over.numel() < self.n_pixels:
            raise ValueError("mc_histograms: output tensors too small")
        need = self.mc_scratch_bytes(runs, cycles, segments_per_run) if int(runs) >= 1 and int(cycles) >= 1 else 0
        if scratch is None and need > 0:
            scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        self._mc_scratch = scratch  # kept alive until the next call
        check(lib().dtm_mc_histograms(self.handle, int(runs), int(cycles), int(burn), int(seed),
                                      int(lanes_per_run), int(segments_per_run), _ptr(hist), _ptr(over),
                                      _ptr(scratch) if scratch is not None else None,
                                      scratch.numel() if scratch is not None else 0, _stream(stream)),
              "dtm_mc_histograms")
        return hist, over

    def graph(self, pi, infos, x0=None, stream=None):
        """Capture one solve into a HIP graph (see Graph)."""
        return Graph(self, pi, infos, x0, stream)

    def close(self):
        if getattr(self, "handle", None):
            lib().dtm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """dtm_graph_*: a captured dtm_solve_batched call, replayed by launch()."""

    def __init__(self, plan, pi, infos, x0=None, stream=None):
        h = _P()
        check(lib().dtm_graph_create(plan.handle, _ptr(x0), _ptr(pi), _ptr(infos), _stream(stream),
                                     ctypes.byref(h)), "dtm_graph_create")
        self.handle = h
        self._keep = (plan, pi, infos, x0)

    def launch(self, stream=None):
        check(lib().dtm_graph_launch(self.handle, _stream(stream)), "dtm_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            lib().dtm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spectral_to_numpy(out_tensor):
    raw = out_tensor.cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=SPECTRAL_INFO_DTYPE).copy()


def infos_to_numpy(infos_tensor):
    """Device SolveInfo array (uint8 tensor of 40*P bytes) -> numpy records."""
    raw = infos_tensor.cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=SOLVE_INFO_DTYPE).copy()

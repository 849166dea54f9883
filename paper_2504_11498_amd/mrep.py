"""Thin ctypes binding of libmrep's C ABI (``include/mrep.h``).

Argument marshalling only: every step of decomposition, projection, inversion
and evaluation runs in the native library (host C++ for the FP64
decomposition, HIP kernels on gfx950 for the batched operations).  PyTorch
supplies device memory and the current stream.  Importing this module raises
if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MREP_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MREP_LIBRARY") or os.path.join(_HERE, "libmrep.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmrep.so not built ({LIB_PATH}); run paper_2504_11498_amd/build.py or __graft_entry__.build()")

_lib = C.CDLL(LIB_PATH)

# status codes and flags (mirror include/mrep.h)
OK, E_INVALID_ARG, E_BAD_DEGREE, E_BAD_KNOTS, E_TOL, E_SMALL_BUFFER, E_HIP, E_NO_DEVICE = 0, -1, -2, -3, -4, -5, -6, -7
F_POLISHED, F_NEAR_TIE, F_ILL_COND, F_ENDPOINT, F_OFFCURVE, F_FULLSCAN, F_BAD_ID = 1, 2, 4, 8, 16, 32, 64
F_NN_FALLBACK = 128
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 3
OPT_TIME_STAGES, OPT_TUNED, OPT_CLIP = 1, 2, 4
STRATEGY_SCREEN, STRATEGY_SPHERES = 0, 1
ROOTS_FERRARI, ROOTS_NEWTON = 0, 1
N_STAGES = 6
N_BOX_SCHEDULES = 6  # sphere-list kernel schedules: index 3 * persistent + log2(lanes / 4)
MAX_DEGREE = 32  # curves
POWER_MAX_DEGREE = 15  # spans kept in power form up to here, as Bezier points above
MAX_SURFACE_DEGREE = 15
SPAN_MAX_DEGREE = 15  # mrep_span_bezier_curves
NN_CURVE, NN_SURFACE = 0, 1
NN_HIDDEN, NN_K = 128, 4
NN_DIMS = {NN_CURVE: (15, 2), NN_SURFACE: (51, 3)}  # kind -> (inputs, outputs)
NN_IN, NN_OUT = NN_DIMS[NN_CURVE]

_vp, _i32, _i64, _dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_pi32, _pi64, _pd = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)


class PlanInfo(C.Structure):
    _fields_ = [("n_curves", C.c_int64), ("n_spans", C.c_int64), ("n_segments", C.c_int64),
                ("device_bytes", C.c_int64), ("max_degree", C.c_int32), ("reserved", C.c_int32),
                ("tol_rel", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("precision", C.c_int32), ("max_candidates", C.c_int32),
                ("flags", C.c_int32), ("tie_rel", C.c_double)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_decompose = _sig("mrep_decompose_curves", _i32, _i32, _pi32, _pi64, _pd, _pi64, _pd, _dbl, _i32, C.POINTER(_vp))
_decompose_rational = _sig("mrep_decompose_curves_rational", _i32, _i32, _pi32, _pi64, _pd, _pd, _pi64, _pd, _dbl,
                          _i32, C.POINTER(_vp))
_decompose_device = _sig("mrep_decompose_curves_device", _i32, _i32, _pi32, _pi64, _vp, _pi64, _vp, _dbl, _vp,
                         C.POINTER(_vp))
_plan_info = _sig("mrep_plan_info", _i32, _vp, C.POINTER(PlanInfo))
_plan_export = _sig("mrep_plan_export", _i32, _vp, _pi64, _pd, _pd, _pi32)
_plan_free = _sig("mrep_plan_free", None, _vp)
_upload = _sig("mrep_upload", _i32, _vp, _vp, _i64, _vp, C.POINTER(_vp))
_geom_release = _sig("mrep_geom_release", None, _vp)
_opts_default = _sig("mrep_opts_default", _i32, C.POINTER(Opts))
_ws_bytes = _sig("mrep_workspace_bytes", _i32, _vp, _i64, C.POINTER(Opts), C.POINTER(C.c_int64))
_project = _sig("mrep_project_curves", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp)
_project_noalloc = _sig("mrep_project_curves_noalloc", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                        _vp)
NOALLOC_SCRATCH_BYTES = 64 << 20
_invert = _sig("mrep_invert_curves", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp)
_eval = _sig("mrep_eval_curves", _i32, _vp, _i64, _vp, _vp, _vp, _vp)
_set_strategy = _sig("mrep_set_curve_strategy", _i32, _vp, _i32)
_schedule = _sig("mrep_curve_schedule", _i32, _vp, _vp, _vp, _vp)
_set_schedule = _sig("mrep_set_curve_schedule", _i32, _vp, _i32, _i32)
_split = _sig("mrep_monotonic_split", _i32, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp)
_span_layout = _sig("mrep_span_layout", _i32, _i32, _pi32, _pi64, _pi64, _pi64, _pi64)
_span_bezier = _sig("mrep_span_bezier_curves", _i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_tune = _sig("mrep_tune_curves", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
             C.POINTER(C.c_int32), C.POINTER(C.c_double), _vp)
_bern = _sig("mrep_bernstein_matrix", _i32, _i32, _i32, _pd)
_subdiv = _sig("mrep_subdivision_matrix", _i32, _i32, _dbl, _pd)
_gram = _sig("mrep_gram_matrix", _i32, _i32, _i32, _pd)
_stage_times = _sig("mrep_last_stage_times", _i32, _pd, _i32)
_nn_param_count = _sig("mrep_nn_param_count", _i32, _i32)
_nn_bytes = _sig("mrep_nn_bytes", _i32, _i32, _i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64))
_nn_bind = _sig("mrep_nn_bind", _i32, _i32, _vp, _i64, C.POINTER(_vp))
_nn_release = _sig("mrep_nn_release", None, _vp)
_nn_init = _sig("mrep_nn_init", _i32, _vp, C.c_uint64, _vp)
_nn_set = _sig("mrep_nn_set_params", _i32, _vp, C.POINTER(C.c_float), _i64, _vp)
_nn_get = _sig("mrep_nn_get_params", _i32, _vp, C.POINTER(C.c_float), _i64, _vp)
_nn_forward = _sig("mrep_nn_forward", _i32, _vp, _i64, _vp, _vp, _vp, _i64, _vp)
_nn_infer = _sig("mrep_nn_infer", _i32, _vp, _i64, _vp, _vp, _vp)
_nn_train = _sig("mrep_nn_train_step", _i32, _vp, _i64, _vp, _vp, _vp, _i64, _vp, C.c_float, _vp, _vp, _vp, _i64,
                 _vp)
_seed_ws = _sig("mrep_seeded_workspace_bytes", _i32, _vp, _i64, C.POINTER(Opts), C.POINTER(C.c_int64))
_nn_features = _sig("mrep_nn_features", _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp)
_project_seeded = _sig("mrep_project_curves_seeded", _i32, _vp, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp,
                       _vp, _vp, _vp, _vp)
_decompose_s = _sig("mrep_decompose_surfaces", _i32, _i32, _pi32, _pi32, _pi32, _pi32, _pi64, _pd, _pi64, _pd, _pi64,
                    _pd, _dbl, _i32, C.POINTER(_vp))
_plan_export_s = _sig("mrep_plan_export_surfaces", _i32, _vp, _pi64, _pd, _pd, _pi32)
_surf_ws = _sig("mrep_surface_workspace_bytes", _i32, _vp, _i64, C.POINTER(Opts), C.POINTER(C.c_int64))
_project_s = _sig("mrep_project_surfaces", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                  _vp)
_invert_s = _sig("mrep_invert_surfaces", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                 _vp)
_eval_s = _sig("mrep_eval_surfaces", _i32, _vp, _i64, _vp, _vp, _vp, _vp)
_surf_seed_ws = _sig("mrep_surface_seeded_workspace_bytes", _i32, _vp, _i64, C.POINTER(Opts), C.POINTER(C.c_int64))
_nn_surf_features = _sig("mrep_nn_surface_features", _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp)
_project_s_seeded = _sig("mrep_project_surfaces_seeded", _i32, _vp, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64,
                         _vp, _vp, _vp, _vp, _vp)
_ws_counts = _sig("mrep_workspace_counts", _i32, _vp, _vp, _pi64, _vp)
_nn_set_compute = _sig("mrep_nn_set_compute", _i32, _vp, _i32)
NN_COMPUTE_BF16, NN_COMPUTE_FP32 = 0, 1
_last_error = _sig("mrep_last_error", C.c_char_p)
_abi = _sig("mrep_abi_version", _i32)

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = ["mrep_decompose_curves", "mrep_decompose_curves_device", "mrep_plan_info", "mrep_plan_export", "mrep_plan_free", "mrep_upload",
           "mrep_geom_release", "mrep_opts_default", "mrep_workspace_bytes", "mrep_project_curves",
           "mrep_invert_curves", "mrep_eval_curves", "mrep_bernstein_matrix", "mrep_subdivision_matrix",
           "mrep_gram_matrix", "mrep_last_stage_times", "mrep_last_error", "mrep_abi_version",
           "mrep_nn_param_count", "mrep_nn_bytes", "mrep_nn_bind", "mrep_nn_release", "mrep_nn_init",
           "mrep_nn_set_params", "mrep_nn_get_params", "mrep_nn_forward", "mrep_nn_infer", "mrep_nn_train_step",
           "mrep_seeded_workspace_bytes", "mrep_nn_features", "mrep_project_curves_seeded",
           "mrep_decompose_surfaces", "mrep_plan_export_surfaces", "mrep_surface_workspace_bytes",
           "mrep_project_surfaces", "mrep_invert_surfaces", "mrep_eval_surfaces",
           "mrep_surface_seeded_workspace_bytes", "mrep_nn_surface_features", "mrep_project_surfaces_seeded",
           "mrep_tune_curves", "mrep_set_curve_strategy", "mrep_curve_schedule", "mrep_set_curve_schedule", "mrep_monotonic_split", "mrep_span_layout",
           "mrep_span_bezier_curves", "mrep_project_curves_noalloc", "mrep_decompose_curves_rational",
           "mrep_workspace_counts", "mrep_nn_set_compute"]


class MrepError(RuntimeError):
    def __init__(self, code, where):
        msg = _last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _check(rc, where):
    if rc != OK:
        raise MrepError(rc, where)


def _host(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def abi_version() -> int:
    return int(_abi())


def last_error() -> str:
    return _last_error().decode(errors="replace")


# ---------------------------------------------------------------------------- host
class Plan:
    """Host-side decomposition of a CSR batch of clamped B-spline curves."""

    def __init__(self, handle):
        self._h = _vp(handle)
        info = PlanInfo()
        _check(_plan_info(self._h, C.byref(info)), "mrep_plan_info")
        self.info = info

    @property
    def n_curves(self):
        return int(self.info.n_curves)

    @property
    def n_segments(self):
        return int(self.info.n_segments)

    @property
    def device_bytes(self):
        return int(self.info.device_bytes)

    def export(self):
        n, s = self.n_curves, self.n_segments
        seg_off = np.zeros(n + 1, np.int64)
        seg_t = np.zeros((s, 2))
        seg_cp = np.zeros((s, 4, 3))
        seg_span = np.zeros(s, np.int32)
        _check(_plan_export(self._h, _p(seg_off, C.c_int64), _p(seg_t, C.c_double), _p(seg_cp, C.c_double),
                            _p(seg_span, C.c_int32)), "mrep_plan_export")
        return {"seg_off": seg_off, "seg_t": seg_t, "seg_cp": seg_cp, "seg_span": seg_span}

    def seg_off(self):
        """Per-curve offsets of the cubic pieces (n_curves + 1), without copying the piece tables."""
        seg_off = np.zeros(self.n_curves + 1, np.int64)
        _check(_plan_export(self._h, _p(seg_off, C.c_int64), None, None, None), "mrep_plan_export")
        return seg_off

    @property
    def is_surfaces(self):
        return int(self.info.reserved) == 1

    def export_surfaces(self):
        n, s = self.n_curves, self.n_segments
        patch_off = np.zeros(n + 1, np.int64)
        patch_uv = np.zeros((s, 4))
        patch_cp = np.zeros((s, 4, 4, 3))
        patch_span = np.zeros(s, np.int32)
        _check(_plan_export_s(self._h, _p(patch_off, C.c_int64), _p(patch_uv, C.c_double), _p(patch_cp, C.c_double),
                              _p(patch_span, C.c_int32)), "mrep_plan_export_surfaces")
        return {"patch_off": patch_off, "patch_uv": patch_uv, "patch_cp": patch_cp, "patch_span": patch_span}

    def upload(self, device=None, zero: bool = False, buf=None):
        """Copy the tables to a new device buffer (a torch tensor) and return a Geometry.  zero: clear the buffer
        first, so that the alignment gaps between tables compare equal too.  buf: a uint8 device tensor of at least
        device_bytes to use instead of a new one."""
        import torch

        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if buf is None:
            alloc = torch.zeros if zero else torch.empty
            buf = alloc(max(self.device_bytes, 256), dtype=torch.uint8, device=dev)
        elif buf.dtype != torch.uint8 or buf.numel() < self.device_bytes:
            raise ValueError("buf must be a uint8 device tensor of at least device_bytes")
        dev = buf.device
        stream = torch.cuda.current_stream(dev).cuda_stream
        g = _vp()
        _check(_upload(self._h, _vp(buf.data_ptr()), buf.numel(), _vp(stream), C.byref(g)), "mrep_upload")
        return Geometry(g, buf, self.n_curves)

    def close(self):
        if self._h:
            _plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decompose_curves(curves, tol_rel: float = 1e-6, n_threads: int = 0, weights=None) -> Plan:
    """mrep_decompose_curves on a CurveSet-like object (degree, cp_off, cp, knot_off, knots); with weights (one
    per control point, or a ``weights`` attribute of the curve set) mrep_decompose_curves_rational."""
    deg = _host(curves.degree, np.int32)
    cp_off = _host(curves.cp_off, np.int64)
    cp = _host(curves.cp, np.float64)
    k_off = _host(curves.knot_off, np.int64)
    kn = _host(curves.knots, np.float64)
    if weights is None:
        weights = getattr(curves, "weights", None)
    h = _vp()
    if weights is None:
        _check(_decompose(int(deg.shape[0]), _p(deg, C.c_int32), _p(cp_off, C.c_int64), _p(cp, C.c_double),
                          _p(k_off, C.c_int64), _p(kn, C.c_double), float(tol_rel), int(n_threads), C.byref(h)),
               "mrep_decompose_curves")
    else:
        w = _host(weights, np.float64)
        _check(_decompose_rational(int(deg.shape[0]), _p(deg, C.c_int32), _p(cp_off, C.c_int64), _p(cp, C.c_double),
                                   _p(w, C.c_double), _p(k_off, C.c_int64), _p(kn, C.c_double), float(tol_rel),
                                   int(n_threads), C.byref(h)), "mrep_decompose_curves_rational")
    return Plan(h.value)


def decompose_curves_device(curves, tol_rel: float = 1e-6, device=None, cp_dev=None, knots_dev=None) -> Plan:
    """mrep_decompose_curves_device: the decomposition run by kernels on the GPU (degrees 1..15, polynomial).
    The control points and knots are copied to the device first unless given as device tensors (cp_dev [n, 3]
    and knots_dev, FP64, the curve set's arrays); the plan holds device arrays and uploads, exports and frees
    like a host plan."""
    import torch

    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    deg = _host(curves.degree, np.int32)
    cp_off = _host(curves.cp_off, np.int64)
    k_off = _host(curves.knot_off, np.int64)
    cp = cp_dev if cp_dev is not None else torch.as_tensor(_host(curves.cp, np.float64)).to(dev)
    kn = knots_dev if knots_dev is not None else torch.as_tensor(_host(curves.knots, np.float64)).to(dev)
    if cp.dtype != torch.float64 or kn.dtype != torch.float64 or not cp.is_contiguous() or not kn.is_contiguous():
        raise ValueError("cp_dev and knots_dev must be contiguous float64 device tensors")
    stream = torch.cuda.current_stream(dev).cuda_stream
    h = _vp()
    _check(_decompose_device(int(deg.shape[0]), _p(deg, C.c_int32), _p(cp_off, C.c_int64), _vp(cp.data_ptr()),
                             _p(k_off, C.c_int64), _vp(kn.data_ptr()), float(tol_rel), _vp(stream), C.byref(h)),
           "mrep_decompose_curves_device")
    return Plan(h.value)


def span_layout(curves):
    """mrep_span_layout: (iv_off, pt_off), the offsets of each curve's knot intervals and of their Bezier points."""
    deg = _host(curves.degree, np.int32)
    cp_off = _host(curves.cp_off, np.int64)
    k_off = _host(curves.knot_off, np.int64)
    n = int(deg.shape[0])
    iv_off = np.zeros(n + 1, np.int64)
    pt_off = np.zeros(n + 1, np.int64)
    _check(_span_layout(n, _p(deg, C.c_int32), _p(cp_off, C.c_int64), _p(k_off, C.c_int64), _p(iv_off, C.c_int64),
                        _p(pt_off, C.c_int64)), "mrep_span_layout")
    return iv_off, pt_off


class DeviceCurves:
    """A CSR batch of curves resident on the device, with its span layout, for mrep_span_bezier_curves."""

    def __init__(self, curves, device=None):
        import torch

        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.iv_off, self.pt_off = span_layout(curves)
        self.n_curves = int(np.asarray(curves.degree).shape[0])
        self.n_intervals = int(self.iv_off[-1])
        self.n_points = int(self.pt_off[-1])
        self.max_degree = int(np.max(curves.degree)) if self.n_curves else 1
        up = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
        self.degree = up(curves.degree, np.int32)
        self.cp_off = up(curves.cp_off, np.int64)
        self.knot_off = up(curves.knot_off, np.int64)
        self.iv = up(self.iv_off, np.int64)
        self.pt = up(self.pt_off, np.int64)
        self.cp = up(curves.cp, np.float64)
        self.knots = up(curves.knots, np.float64)
        self.device = dev

    def span_bezier(self, bz=None, t=None):
        """mrep_span_bezier_curves: (bz [n_points, 3], t [n_intervals, 2]) device tensors (FP64)."""
        import torch

        if bz is None:
            bz = torch.empty((self.n_points, 3), dtype=torch.float64, device=self.device)
        if t is None:
            t = torch.empty((self.n_intervals, 2), dtype=torch.float64, device=self.device)
        if bz.numel() < 3 * self.n_points or t.numel() < 2 * self.n_intervals:
            raise ValueError("output tensors too small")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(_span_bezier(self.n_curves, self.n_intervals, self.max_degree, _vp(self.degree.data_ptr()), _vp(self.cp_off.data_ptr()),
                            _vp(self.knot_off.data_ptr()), _vp(self.iv.data_ptr()), _vp(self.pt.data_ptr()),
                            _vp(self.cp.data_ptr()), _vp(self.knots.data_ptr()), _vp(bz.data_ptr()),
                            _vp(t.data_ptr()), _vp(stream)), "mrep_span_bezier_curves")
        return bz, t


def decompose_surfaces(surfs, tol_rel: float = 1e-6, n_threads: int = 0) -> Plan:
    """mrep_decompose_surfaces on a SurfaceSet-like object (deg_u, deg_v, n_u, n_v, cp_off, cp, ku_off, ku, kv_off,
    kv)."""
    a = [_host(surfs.deg_u, np.int32), _host(surfs.deg_v, np.int32), _host(surfs.n_u, np.int32),
         _host(surfs.n_v, np.int32), _host(surfs.cp_off, np.int64), _host(surfs.cp, np.float64),
         _host(surfs.ku_off, np.int64), _host(surfs.ku, np.float64), _host(surfs.kv_off, np.int64),
         _host(surfs.kv, np.float64)]
    h = _vp()
    _check(_decompose_s(int(a[0].shape[0]), _p(a[0], C.c_int32), _p(a[1], C.c_int32), _p(a[2], C.c_int32),
                        _p(a[3], C.c_int32), _p(a[4], C.c_int64), _p(a[5], C.c_double), _p(a[6], C.c_int64),
                        _p(a[7], C.c_double), _p(a[8], C.c_int64), _p(a[9], C.c_double), float(tol_rel),
                        int(n_threads), C.byref(h)), "mrep_decompose_surfaces")
    return Plan(h.value)


def default_opts(precision: str | int = "bf16", max_candidates: int = 32, tie_rel: float = 2e-6,
                 time_stages: bool = False, tuned: bool = False, clip: bool = False) -> Opts:
    """tuned: curve projections run the strategy Geometry.tune() chose (BF16 mode).  clip: candidate pieces are
    refined by the paper's monotonic split, elimination, rebasement and Bezier clipping (MREP_OPT_CLIP)."""
    o = Opts()
    _check(_opts_default(C.byref(o)), "mrep_opts_default")
    o.flags = (OPT_TIME_STAGES if time_stages else 0) | (OPT_TUNED if tuned else 0) | (OPT_CLIP if clip else 0)
    if isinstance(precision, str):
        precision = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16": PREC_BF16}[precision]
    o.precision = int(precision)
    o.max_candidates = int(max_candidates)
    o.tie_rel = float(tie_rel)
    return o


def last_stage_times():
    """Stage milliseconds of the last call made with time_stages=True on this thread.

    mrep_project_curves: [grouping, screen, pair refine, finish]; seeded call (and the sphere strategy): [grouping,
    sphere candidates, network, seed + certificate, pair refine, finish]."""
    out = np.zeros(N_STAGES)
    rc = _stage_times(_p(out, C.c_double), N_STAGES)
    if rc <= 0:
        raise MrepError(rc, "mrep_last_stage_times")
    return out[:rc]


def bernstein_matrix(p: int, inverse: bool = False) -> np.ndarray:
    out = np.zeros((p + 1, p + 1))
    _check(_bern(int(p), int(bool(inverse)), _p(out, C.c_double)), "mrep_bernstein_matrix")
    return out


def subdivision_matrix(p: int, z: float) -> np.ndarray:
    out = np.zeros((2 * (p + 1), p + 1))
    _check(_subdiv(int(p), float(z), _p(out, C.c_double)), "mrep_subdivision_matrix")
    return out


def gram_matrix(m: int, n: int) -> np.ndarray:
    out = np.zeros((m + 1, n + 1))
    _check(_gram(int(m), int(n), _p(out, C.c_double)), "mrep_gram_matrix")
    return out


# ---------------------------------------------------------------------------- device
class Geometry:
    """Device-resident decomposition (a view into a torch uint8 buffer)."""

    def __init__(self, handle, buf, n_curves):
        self._h = handle
        self.buf = buf
        self.n_curves = n_curves
        self._ws = None

    def workspace_bytes(self, n: int, opts: Opts) -> int:
        b = C.c_int64()
        _check(_ws_bytes(self._h, int(n), C.byref(opts), C.byref(b)), "mrep_workspace_bytes")
        return int(b.value)

    def _workspace(self, n, opts, workspace):
        import torch

        need = self.workspace_bytes(n, opts)
        if workspace is not None:
            return workspace
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.buf.device)
        return self._ws

    def project(self, q, curve_id, opts: Opts | None = None, invert: bool = False, workspace=None, out=None):
        """Project q[n,3] (float64, device) onto curves curve_id[n] (int32, device).

        Returns (t, dist, seg, flags) device tensors; enqueued on the current stream.
        """
        import torch

        if opts is None:
            opts = default_opts()
        assert q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.dim() == 2 and q.shape[1] == 3
        assert curve_id.is_cuda and curve_id.dtype == torch.int32 and curve_id.is_contiguous()
        n = q.shape[0]
        assert curve_id.shape[0] == n
        ws = self._workspace(n, opts, workspace)
        if out is None:
            t = torch.empty(n, dtype=torch.float64, device=q.device)
            d = torch.empty(n, dtype=torch.float64, device=q.device)
            s = torch.empty(n, dtype=torch.int32, device=q.device)
            f = torch.empty(n, dtype=torch.int32, device=q.device)
        else:
            t, d, s, f = out
        stream = torch.cuda.current_stream(q.device).cuda_stream
        fn = _invert if invert else _project
        _check(fn(self._h, C.byref(opts), int(n), _vp(curve_id.data_ptr()), _vp(q.data_ptr()), _vp(ws.data_ptr()),
                  int(ws.numel()), _vp(t.data_ptr()), _vp(d.data_ptr()), _vp(s.data_ptr()), _vp(f.data_ptr()),
                  _vp(stream)), "mrep_invert_curves" if invert else "mrep_project_curves")
        return t, d, s, f

    def workspace_counts(self, workspace, tests: bool = False):
        """(queries overflowed to the full scan, candidate pairs reserved) left by the last call on workspace; with
        tests, also the sphere tests of the sphere-list strategy."""
        import torch

        c = np.zeros(3, np.int64)
        stream = torch.cuda.current_stream(workspace.device).cuda_stream
        _check(_ws_counts(self._h, _vp(workspace.data_ptr()), _p(c, C.c_int64), _vp(stream)), "mrep_workspace_counts")
        return (int(c[0]), int(c[1]), int(c[2])) if tests else (int(c[0]), int(c[1]))

    def project_noalloc(self, q, curve_id, opts: Opts | None = None, out=None):
        """As project(), through mrep_project_curves_noalloc: no workspace, the library's fixed per-GPU scratch."""
        import torch

        if opts is None:
            opts = default_opts()
        assert q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.dim() == 2 and q.shape[1] == 3
        assert curve_id.is_cuda and curve_id.dtype == torch.int32 and curve_id.is_contiguous()
        n = q.shape[0]
        assert curve_id.shape[0] == n
        if out is None:
            out = (torch.empty(n, dtype=torch.float64, device=q.device), torch.empty(n, dtype=torch.float64, device=q.device),
                   torch.empty(n, dtype=torch.int32, device=q.device), torch.empty(n, dtype=torch.int32, device=q.device))
        t, d, s, f = out
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_project_noalloc(self._h, C.byref(opts), int(n), _vp(curve_id.data_ptr()), _vp(q.data_ptr()),
                                _vp(t.data_ptr()), _vp(d.data_ptr()), _vp(s.data_ptr()), _vp(f.data_ptr()),
                                _vp(stream)), "mrep_project_curves_noalloc")
        return t, d, s, f

    def tune(self, q, curve_id, opts: Opts | None = None, out=None):
        """Autotune the curve strategy on this batch (mrep_tune_curves): returns (strategy, ms_screen,
        ms_spheres, (t, dist, seg, flags)); later calls with default_opts(tuned=True) use the choice."""
        import torch

        if opts is None:
            opts = default_opts("bf16")
        n = q.shape[0]
        o2 = Opts.from_buffer_copy(opts)
        o2.flags |= OPT_TUNED
        ws = self._workspace(n, o2, None)
        if out is None:
            out = (torch.empty(n, dtype=torch.float64, device=q.device), torch.empty(n, dtype=torch.float64, device=q.device),
                   torch.empty(n, dtype=torch.int32, device=q.device), torch.empty(n, dtype=torch.int32, device=q.device))
        t, d, s, f = out
        strat = C.c_int32()
        ms = (C.c_double * 2)()
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_tune(self._h, C.byref(opts), int(n), _vp(curve_id.data_ptr()), _vp(q.data_ptr()), _vp(ws.data_ptr()),
                     int(ws.numel()), _vp(t.data_ptr()), _vp(d.data_ptr()), _vp(s.data_ptr()), _vp(f.data_ptr()),
                     C.byref(strat), ms, _vp(stream)), "mrep_tune_curves")
        return int(strat.value), float(ms[0]), float(ms[1]), out

    def set_strategy(self, strategy: int):
        """The strategy of calls with default_opts(tuned=True): STRATEGY_SCREEN or STRATEGY_SPHERES."""
        _check(_set_strategy(self._h, int(strategy)), "mrep_set_curve_strategy")

    def schedule(self):
        """mrep_curve_schedule: (lanes per query, persistent, per-schedule ms of the last tune) of the sphere-list
        kernel."""
        lanes, pers = C.c_int32(), C.c_int32()
        ms = (C.c_double * N_BOX_SCHEDULES)()
        _check(_schedule(self._h, C.byref(lanes), C.byref(pers), ms), "mrep_curve_schedule")
        return int(lanes.value), int(pers.value), [float(x) for x in ms]

    def set_schedule(self, lanes: int, persistent: int):
        """mrep_set_curve_schedule: 4, 8 or 16 lanes per query; persistent 0 (tile map) or 1 (per-XCD queues)."""
        _check(_set_schedule(self._h, int(lanes), int(persistent)), "mrep_set_curve_schedule")

    def seeded_workspace_bytes(self, n: int, opts: Opts) -> int:
        b = C.c_int64()
        _check(_seed_ws(self._h, int(n), C.byref(opts), C.byref(b)), "mrep_seeded_workspace_bytes")
        return int(b.value)

    def _seed_workspace(self, n, opts, workspace):
        import torch

        need = self.seeded_workspace_bytes(n, opts)
        if workspace is not None:
            return workspace
        if getattr(self, "_sws", None) is None or self._sws.numel() < need:
            self._sws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.buf.device)
        return self._sws

    def project_seeded(self, q, curve_id, nn: "Network | None" = None, opts: Opts | None = None, workspace=None,
                       out=None):
        """Seeded projection (nn given) or sphere-pruned projection (nn None); same outputs as project()."""
        import torch

        if opts is None:
            opts = default_opts()
        assert q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.dim() == 2 and q.shape[1] == 3
        assert curve_id.is_cuda and curve_id.dtype == torch.int32 and curve_id.is_contiguous()
        n = q.shape[0]
        assert curve_id.shape[0] == n
        ws = self._seed_workspace(n, opts, workspace)
        if out is None:
            t = torch.empty(n, dtype=torch.float64, device=q.device)
            d = torch.empty(n, dtype=torch.float64, device=q.device)
            s = torch.empty(n, dtype=torch.int32, device=q.device)
            f = torch.empty(n, dtype=torch.int32, device=q.device)
        else:
            t, d, s, f = out
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_project_seeded(self._h, nn._h if nn is not None else None, C.byref(opts), int(n),
                               _vp(curve_id.data_ptr()), _vp(q.data_ptr()), _vp(ws.data_ptr()), int(ws.numel()),
                               _vp(t.data_ptr()), _vp(d.data_ptr()), _vp(s.data_ptr()), _vp(f.data_ptr()),
                               _vp(stream)), "mrep_project_curves_seeded")
        return t, d, s, f

    def features(self, q, curve_id, workspace=None):
        """The network's candidate pieces seg[n, 4] (curve-local, -1 none) and inputs x[n, 4, 15]."""
        import torch

        n = q.shape[0]
        opts = default_opts()
        ws = self._seed_workspace(n, opts, workspace)
        seg = torch.empty((n, NN_K), dtype=torch.int32, device=q.device)
        x = torch.empty((n, NN_K, NN_IN), dtype=torch.float32, device=q.device)
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_nn_features(self._h, int(n), _vp(curve_id.data_ptr()), _vp(q.data_ptr()), _vp(seg.data_ptr()),
                            _vp(x.data_ptr()), _vp(ws.data_ptr()), int(ws.numel()), _vp(stream)), "mrep_nn_features")
        return seg, x

    def surface_workspace_bytes(self, n: int, opts: Opts) -> int:
        b = C.c_int64()
        _check(_surf_ws(self._h, int(n), C.byref(opts), C.byref(b)), "mrep_surface_workspace_bytes")
        return int(b.value)

    def project_surfaces(self, q, surface_id, opts: Opts | None = None, invert: bool = False, workspace=None,
                         out=None):
        """Project q[n,3] (float64, device) onto surfaces surface_id[n] (int32, device).

        Returns (uv[n,2], dist, patch, flags) device tensors; enqueued on the current stream."""
        import torch

        if opts is None:
            opts = default_opts()
        assert q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.dim() == 2 and q.shape[1] == 3
        assert surface_id.is_cuda and surface_id.dtype == torch.int32 and surface_id.is_contiguous()
        n = q.shape[0]
        assert surface_id.shape[0] == n
        if workspace is None:
            need = self.surface_workspace_bytes(n, opts)
            if getattr(self, "_sws2", None) is None or self._sws2.numel() < need:
                self._sws2 = torch.empty(max(need, 256), dtype=torch.uint8, device=self.buf.device)
            workspace = self._sws2
        if out is None:
            uv = torch.empty((n, 2), dtype=torch.float64, device=q.device)
            d = torch.empty(n, dtype=torch.float64, device=q.device)
            s = torch.empty(n, dtype=torch.int32, device=q.device)
            f = torch.empty(n, dtype=torch.int32, device=q.device)
        else:
            uv, d, s, f = out
        stream = torch.cuda.current_stream(q.device).cuda_stream
        fn = _invert_s if invert else _project_s
        _check(fn(self._h, C.byref(opts), int(n), _vp(surface_id.data_ptr()), _vp(q.data_ptr()),
                  _vp(workspace.data_ptr()), int(workspace.numel()), _vp(uv.data_ptr()), _vp(d.data_ptr()),
                  _vp(s.data_ptr()), _vp(f.data_ptr()), _vp(stream)),
               "mrep_invert_surfaces" if invert else "mrep_project_surfaces")
        return uv, d, s, f

    def surface_seeded_workspace_bytes(self, n: int, opts: Opts) -> int:
        b = C.c_int64()
        _check(_surf_seed_ws(self._h, int(n), C.byref(opts), C.byref(b)), "mrep_surface_seeded_workspace_bytes")
        return int(b.value)

    def _surf_seed_workspace(self, n, opts, workspace):
        import torch

        if workspace is not None:
            return workspace
        need = self.surface_seeded_workspace_bytes(n, opts)
        if getattr(self, "_sws3", None) is None or self._sws3.numel() < need:
            self._sws3 = torch.empty(max(need, 256), dtype=torch.uint8, device=self.buf.device)
        return self._sws3

    def project_surfaces_seeded(self, q, surface_id, nn: "Network", opts: Opts | None = None, workspace=None,
                                out=None):
        """Seeded surface projection (nn of kind NN_SURFACE); same outputs as project_surfaces()."""
        import torch

        if opts is None:
            opts = default_opts()
        assert q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and q.dim() == 2 and q.shape[1] == 3
        assert surface_id.is_cuda and surface_id.dtype == torch.int32 and surface_id.is_contiguous()
        n = q.shape[0]
        assert surface_id.shape[0] == n
        ws = self._surf_seed_workspace(n, opts, workspace)
        if out is None:
            uv = torch.empty((n, 2), dtype=torch.float64, device=q.device)
            d = torch.empty(n, dtype=torch.float64, device=q.device)
            s = torch.empty(n, dtype=torch.int32, device=q.device)
            f = torch.empty(n, dtype=torch.int32, device=q.device)
        else:
            uv, d, s, f = out
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_project_s_seeded(self._h, nn._h if nn is not None else None, C.byref(opts), int(n),
                                 _vp(surface_id.data_ptr()), _vp(q.data_ptr()), _vp(ws.data_ptr()), int(ws.numel()),
                                 _vp(uv.data_ptr()), _vp(d.data_ptr()), _vp(s.data_ptr()), _vp(f.data_ptr()),
                                 _vp(stream)), "mrep_project_surfaces_seeded")
        return uv, d, s, f

    def surface_features(self, q, surface_id, workspace=None):
        """The surface network's candidate patches patch[n, 4] (surface-local, -1 none) and inputs x[n, 4, 51]."""
        import torch

        n = q.shape[0]
        ws = self._surf_seed_workspace(n, default_opts(), workspace)
        patch = torch.empty((n, NN_K), dtype=torch.int32, device=q.device)
        x = torch.empty((n, NN_K, NN_DIMS[NN_SURFACE][0]), dtype=torch.float32, device=q.device)
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_nn_surf_features(self._h, int(n), _vp(surface_id.data_ptr()), _vp(q.data_ptr()),
                                 _vp(patch.data_ptr()), _vp(x.data_ptr()), _vp(ws.data_ptr()), int(ws.numel()),
                                 _vp(stream)), "mrep_nn_surface_features")
        return patch, x

    def eval_surfaces(self, surface_id, uv):
        """S_{surface_id[i]}(u_i, v_i) on the exact surface, FP64, device tensors in and out."""
        import torch

        n = uv.shape[0]
        xyz = torch.empty((n, 3), dtype=torch.float64, device=uv.device)
        stream = torch.cuda.current_stream(uv.device).cuda_stream
        _check(_eval_s(self._h, int(n), _vp(surface_id.data_ptr()), _vp(uv.data_ptr()), _vp(xyz.data_ptr()),
                       _vp(stream)), "mrep_eval_surfaces")
        return xyz

    def eval(self, curve_id, t):
        """C_{curve_id[i]}(t[i]) on the exact curve, FP64, device tensors in and out."""
        import torch

        n = t.shape[0]
        xyz = torch.empty((n, 3), dtype=torch.float64, device=t.device)
        stream = torch.cuda.current_stream(t.device).cuda_stream
        _check(_eval(self._h, int(n), _vp(curve_id.data_ptr()), _vp(t.data_ptr()), _vp(xyz.data_ptr()),
                     _vp(stream)), "mrep_eval_curves")
        return xyz

    def monotonic_split(self, curve_id, piece, q, method: int = ROOTS_FERRARI):
        """Roots in (0, 1) of E' for each (query, piece) pair (Sec. 5.2.3): (roots[n, 4] ascending, count[n]);
        count -1 for an out-of-range curve or piece.  method ROOTS_FERRARI or ROOTS_NEWTON."""
        import torch

        n = q.shape[0]
        roots = torch.empty((n, 4), dtype=torch.float64, device=q.device)
        count = torch.empty(n, dtype=torch.int32, device=q.device)
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_split(self._h, int(n), _vp(curve_id.data_ptr()), _vp(piece.data_ptr()), _vp(q.data_ptr()),
                      int(method), _vp(roots.data_ptr()), _vp(count.data_ptr()), _vp(stream)), "mrep_monotonic_split")
        return roots, count

    def close(self):
        if self._h:
            _geom_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------- learned seeding
def nn_param_count(kind: int = NN_CURVE) -> int:
    return int(_nn_param_count(int(kind)))


class Network:
    """The seeding MLP's device state (parameters, Adam moments, gradient, weight image) in a torch buffer.

    kind: NN_CURVE (15 -> 128 -> 128 -> 2) or NN_SURFACE (51 -> 128 -> 128 -> 3)."""

    def __init__(self, device=None, seed: int | None = 0, kind: int = NN_CURVE):
        import torch

        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.kind = int(kind)
        self.n_in, self.n_out = NN_DIMS[self.kind]
        sb = C.c_int64()
        _check(_nn_bytes(self.kind, 0, C.byref(sb), None), "mrep_nn_bytes")
        self.state = torch.empty(int(sb.value), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_nn_bind(self.kind, _vp(self.state.data_ptr()), self.state.numel(), C.byref(h)), "mrep_nn_bind")
        self._h = h
        self._work = None
        if seed is not None:
            self.init(seed)

    def _stream(self):
        import torch

        return _vp(torch.cuda.current_stream(self.device).cuda_stream)

    def init(self, seed: int):
        _check(_nn_init(self._h, C.c_uint64(int(seed)), self._stream()), "mrep_nn_init")

    def set_compute(self, compute: int):
        """NN_COMPUTE_BF16 (default) or NN_COMPUTE_FP32 (debug) for forward() and train_step()."""
        _check(_nn_set_compute(self._h, int(compute)), "mrep_nn_set_compute")

    def set_params(self, p):
        p = _host(p, np.float32)
        _check(_nn_set(self._h, _p(p, C.c_float), int(p.shape[0]), self._stream()), "mrep_nn_set_params")

    def get_params(self) -> np.ndarray:
        p = np.zeros(nn_param_count(self.kind), np.float32)
        _check(_nn_get(self._h, _p(p, C.c_float), int(p.shape[0]), self._stream()), "mrep_nn_get_params")
        return p

    def _work_for(self, rows):
        import torch

        wb = C.c_int64()
        _check(_nn_bytes(self.kind, int(rows), None, C.byref(wb)), "mrep_nn_bytes")
        if self._work is None or self._work.numel() < wb.value:
            self._work = torch.empty(max(int(wb.value), 256), dtype=torch.uint8, device=self.device)
        return self._work

    def forward(self, x):
        """Training-form forward: y[n, out] for x[n, in] (float32, device)."""
        import torch

        n = x.shape[0]
        assert x.shape[-1] == self.n_in
        y = torch.empty((n, self.n_out), dtype=torch.float32, device=x.device)
        w = self._work_for(n)
        _check(_nn_forward(self._h, int(n), _vp(x.data_ptr()), _vp(y.data_ptr()), _vp(w.data_ptr()), int(w.numel()),
                           self._stream()), "mrep_nn_forward")
        return y

    def infer(self, x):
        """Fused-kernel forward: y[n, out] for x[n, in] (float32, device)."""
        import torch

        n = x.shape[0]
        assert x.shape[-1] == self.n_in
        y = torch.empty((n, self.n_out), dtype=torch.float32, device=x.device)
        _check(_nn_infer(self._h, int(n), _vp(x.data_ptr()), _vp(y.data_ptr()), self._stream()), "mrep_nn_infer")
        return y

    def train_step(self, x, target, accept, rows=None, batch=None, lr: float = 1e-3, loss=None, grad=None):
        """One step on the rows `rows` (int32 device, or the first `batch` rows); returns nothing (async).

        x[n, in], target[n, out - 1] (or [n] for curves), accept[n]: float32 device tensors.  loss: optional
        1-element float32 device tensor receiving the batch loss; grad: optional device tensor of
        nn_param_count(kind) floats receiving the gradient."""
        b = int(rows.shape[0]) if rows is not None else int(batch if batch is not None else x.shape[0])
        w = self._work_for(b)
        assert x.shape[-1] == self.n_in and target.numel() == x.shape[0] * (self.n_out - 1)
        _check(_nn_train(self._h, int(x.shape[0]), _vp(x.data_ptr()), _vp(target.data_ptr()), _vp(accept.data_ptr()),
                         b, _vp(rows.data_ptr()) if rows is not None else None, float(lr),
                         _vp(loss.data_ptr()) if loss is not None else None,
                         _vp(grad.data_ptr()) if grad is not None else None, _vp(w.data_ptr()), int(w.numel()),
                         self._stream()), "mrep_nn_train_step")

    def close(self):
        if self._h:
            _nn_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

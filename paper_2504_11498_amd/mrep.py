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
PREC_FP64, PREC_BF16 = 0, 3
OPT_TIME_STAGES = 1
N_STAGES = 3
MAX_DEGREE = 15

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
_plan_info = _sig("mrep_plan_info", _i32, _vp, C.POINTER(PlanInfo))
_plan_export = _sig("mrep_plan_export", _i32, _vp, _pi64, _pd, _pd, _pi32)
_plan_free = _sig("mrep_plan_free", None, _vp)
_upload = _sig("mrep_upload", _i32, _vp, _vp, _i64, _vp, C.POINTER(_vp))
_geom_release = _sig("mrep_geom_release", None, _vp)
_opts_default = _sig("mrep_opts_default", _i32, C.POINTER(Opts))
_ws_bytes = _sig("mrep_workspace_bytes", _i32, _vp, _i64, C.POINTER(Opts), C.POINTER(C.c_int64))
_project = _sig("mrep_project_curves", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp)
_invert = _sig("mrep_invert_curves", _i32, _vp, C.POINTER(Opts), _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp)
_eval = _sig("mrep_eval_curves", _i32, _vp, _i64, _vp, _vp, _vp, _vp)
_bern = _sig("mrep_bernstein_matrix", _i32, _i32, _i32, _pd)
_subdiv = _sig("mrep_subdivision_matrix", _i32, _i32, _dbl, _pd)
_gram = _sig("mrep_gram_matrix", _i32, _i32, _i32, _pd)
_stage_times = _sig("mrep_last_stage_times", _i32, _pd, _i32)
_last_error = _sig("mrep_last_error", C.c_char_p)
_abi = _sig("mrep_abi_version", _i32)

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = ["mrep_decompose_curves", "mrep_plan_info", "mrep_plan_export", "mrep_plan_free", "mrep_upload",
           "mrep_geom_release", "mrep_opts_default", "mrep_workspace_bytes", "mrep_project_curves",
           "mrep_invert_curves", "mrep_eval_curves", "mrep_bernstein_matrix", "mrep_subdivision_matrix",
           "mrep_gram_matrix", "mrep_last_stage_times", "mrep_last_error", "mrep_abi_version"]


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

    def upload(self, device=None):
        """Copy the tables to a new device buffer (a torch tensor) and return a Geometry."""
        import torch

        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        buf = torch.empty(max(self.device_bytes, 256), dtype=torch.uint8, device=dev)
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


def decompose_curves(curves, tol_rel: float = 1e-6, n_threads: int = 0) -> Plan:
    """mrep_decompose_curves on a CurveSet-like object (degree, cp_off, cp, knot_off, knots)."""
    deg = _host(curves.degree, np.int32)
    cp_off = _host(curves.cp_off, np.int64)
    cp = _host(curves.cp, np.float64)
    k_off = _host(curves.knot_off, np.int64)
    kn = _host(curves.knots, np.float64)
    h = _vp()
    _check(_decompose(int(deg.shape[0]), _p(deg, C.c_int32), _p(cp_off, C.c_int64), _p(cp, C.c_double),
                      _p(k_off, C.c_int64), _p(kn, C.c_double), float(tol_rel), int(n_threads), C.byref(h)),
           "mrep_decompose_curves")
    return Plan(h.value)


def default_opts(precision: str | int = "bf16", max_candidates: int = 16, tie_rel: float = 2e-6,
                 time_stages: bool = False) -> Opts:
    o = Opts()
    _check(_opts_default(C.byref(o)), "mrep_opts_default")
    o.flags = OPT_TIME_STAGES if time_stages else 0
    if isinstance(precision, str):
        precision = {"fp64": PREC_FP64, "bf16": PREC_BF16}[precision]
    o.precision = int(precision)
    o.max_candidates = int(max_candidates)
    o.tie_rel = float(tie_rel)
    return o


def last_stage_times():
    """[grouping, screen, refine] milliseconds of the last call made with time_stages=True on this thread."""
    out = np.zeros(N_STAGES)
    _check(_stage_times(_p(out, C.c_double), N_STAGES), "mrep_last_stage_times")
    return out


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

    def eval(self, curve_id, t):
        """C_{curve_id[i]}(t[i]) on the exact curve, FP64, device tensors in and out."""
        import torch

        n = t.shape[0]
        xyz = torch.empty((n, 3), dtype=torch.float64, device=t.device)
        stream = torch.cuda.current_stream(t.device).cuda_stream
        _check(_eval(self._h, int(n), _vp(curve_id.data_ptr()), _vp(t.data_ptr()), _vp(xyz.data_ptr()),
                     _vp(stream)), "mrep_eval_curves")
        return xyz

    def close(self):
        if self._h:
            _geom_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

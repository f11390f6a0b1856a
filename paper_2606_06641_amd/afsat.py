"""Python binding of ``libafsat`` (the C ABI in ``include/afsat.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Torch provides device memory and streams; tensors are passed as raw
device pointers together with torch's current HIP stream.  If the library is
not built this module raises on import instead of falling back to anything.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafsat.so")

OR, XOR, NAE, CARD_GE, CARD_LT, AMO, EO, EK = range(8)

AFS_OK, AFS_EINVAL, AFS_EUNSAT, AFS_ENOMEM, AFS_EDEVICE, AFS_ESTATE = 0, -1, -2, -3, -4, -5
MAX_LEN = 1024          # AFS_MAX_LEN: longest constraint the evaluation kernels take

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)


class AfsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("afsat status %d: %s" % (status, msg))
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("n_cons", ctypes.c_int32), ("n_lits", ctypes.c_int64),
                ("n_buckets", ctypes.c_int32), ("n_tables", ctypes.c_int32),
                ("max_k", ctypes.c_int32), ("device", ctypes.c_int32), ("n_inst", ctypes.c_int32)]


class _BucketInfo(ctypes.Structure):
    _fields_ = [("k_lo", ctypes.c_int32), ("k_hi", ctypes.c_int32), ("n_cons", ctypes.c_int32),
                ("n_lits", ctypes.c_int64), ("lanes_per_restart", ctypes.c_int32),
                ("lits_per_lane", ctypes.c_int32), ("slot0", ctypes.c_int64), ("tile", ctypes.c_int32),
                ("rpl", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("n_shapes", ctypes.c_int32), ("shape_k_hi", _i32p), ("shape_lanes", _i32p),
                ("shape_seg", _i32p), ("tile_short", ctypes.c_int32), ("tile_long", ctypes.c_int32),
                ("shape_tile", _i32p), ("short_tile", _i32p), ("short_rpl", _i32p)]


class _LineSearch(ctypes.Structure):
    _fields_ = [("max_step", ctypes.c_float), ("shrink", ctypes.c_float), ("armijo", ctypes.c_float),
                ("trials", ctypes.c_int32)]


class _PgdParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("max_iters", ctypes.c_int32), ("poll", ctypes.c_int32),
                ("stop_on_sat", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("fixed", ctypes.c_void_p),
                ("n_partial", ctypes.c_int32), ("delta", ctypes.c_float),
                ("search", ctypes.POINTER(_LineSearch)), ("search_ws", ctypes.c_void_p),
                ("search_ws_bytes", ctypes.c_size_t), ("epsilon", ctypes.c_float),
                ("momentum", ctypes.c_float), ("velocity", ctypes.c_void_p)]


class _PgdState(ctypes.Structure):
    _fields_ = [("unsat", _vp), ("done", _vp), ("first_sat", _vp), ("counter", _vp)]


class _ParsedInfo(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("n_cons", ctypes.c_int32), ("n_lits", ctypes.c_int64),
                ("n_units", ctypes.c_int32), ("n_dropped", ctypes.c_int32), ("declared_cons", ctypes.c_int32)]


# (name, restype, argtypes) of every exported function; the CPU tests check that
# the library exports exactly these.
SIGNATURES = [
    ("afs_last_error", ctypes.c_char_p, []),
    ("afs_coefficients", ctypes.c_int, [_i32, _i32, _i32, _f64p, _f64p]),
    ("afs_instance_create", ctypes.c_int, [_i32, _i32, _i64p, _i32p, _i32p, _i32p, _f32p, _i32,
                                           ctypes.POINTER(_vp)]),
    ("afs_instance_create_ex", ctypes.c_int, [_i32, _i32, _i64p, _i32p, _i32p, _i32p, _f32p,
                                              ctypes.POINTER(_Options), _i32, ctypes.POINTER(_vp)]),
    ("afs_batch_create", ctypes.c_int, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_Options), _i32,
                                        ctypes.POINTER(_vp)]),
    ("afs_batch_var_offsets", ctypes.c_int, [_vp, _i32p]),
    ("afs_instance_destroy", None, [_vp]),
    ("afs_instance_info", ctypes.c_int, [_vp, ctypes.POINTER(_Info)]),
    ("afs_bucket_info_get", ctypes.c_int, [_vp, _i32, ctypes.POINTER(_BucketInfo)]),
    ("afs_instance_slot_map", ctypes.c_int, [_vp, _i64p]),
    ("afs_instance_transpose", ctypes.c_int, [_vp, _i64p, _i64p]),
    ("afs_workspace_bytes", ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    ("afs_eval", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]),
    ("afs_fe_grad", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_size_t, _i32, _i32, _i32, _vp, _vp]),
    ("afs_scatter", ctypes.c_int, [_vp, _i32, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    ("afs_fe_grad_buckets", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_size_t, _i32p, _i32, _i32, _vp, _vp]),
    ("afs_eval_fwd", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    ("afs_eval_adjoint", ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    ("afs_step", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_float, _vp, _i32, _vp, _vp]),
    ("afs_round_verify", ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    ("afs_pgd_init", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_PgdState), _vp]),
    ("afs_pgd_step", ctypes.c_int, [_vp, _i32, _vp, ctypes.c_float, _vp, _i32, _vp, ctypes.c_size_t,
                                    ctypes.POINTER(_PgdState), _vp]),
    ("afs_pgd_update", ctypes.c_int, [_vp, _i32, _vp, ctypes.c_float, _vp, _i32, _vp, ctypes.c_size_t,
                                      ctypes.POINTER(_PgdState), _vp]),
    ("afs_pgd_step_momentum", ctypes.c_int, [_vp, _i32, _vp, _vp, ctypes.c_float, ctypes.c_float, _vp, _i32, _vp,
                                             ctypes.c_size_t, ctypes.POINTER(_PgdState), _vp]),
    ("afs_pgd", ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_PgdParams), _vp, ctypes.c_size_t,
                               ctypes.POINTER(_PgdState), _vp, ctypes.POINTER(_i32), _vp]),
    ("afs_autotune", ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, ctypes.c_char_p, ctypes.c_char_p, _i32,
                                    _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(_i32)]),
    ("afs_parse_text", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    ("afs_parse_file", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
    ("afs_parsed_get_info", ctypes.c_int, [_vp, ctypes.POINTER(_ParsedInfo)]),
    ("afs_parsed_arrays", ctypes.c_int, [_vp, _i64p, _i32p, _i32p, _i32p, ctypes.POINTER(ctypes.c_int8)]),
    ("afs_parsed_destroy", None, [_vp]),
    ("afs_parsed_fold_units", ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_int8)]),
    ("afs_search_workspace_bytes", ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    ("afs_pgd_search_step", ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_LineSearch), _vp, _i32, ctypes.c_float,
                                           _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, ctypes.POINTER(_PgdState),
                                           _vp, _vp]),
    ("afs_init_points", ctypes.c_int, [_vp, _i32, ctypes.c_uint64, _vp, _i32, _vp, _vp]),
    ("afs_form_tables", ctypes.c_int, [_i32, _i32, _i32, _i32, _f64p, _f64p, _f64p]),
    ("afs_fe_generic", ctypes.c_int, [_i32, _f64p, _f64p, _f64p, _i32, _i32, _vp, _vp, _i32, _vp]),
    ("afs_decompose_size", ctypes.c_int, [_i32, _i32, _i64p, _i32p, _i32, _i32p, _i32p, _i64p]),
    ("afs_decompose", ctypes.c_int, [_i32, _i32, _i64p, _i32p, _i32p, _i32p, _f32p, _i32, _i64p, _i32p, _i32p,
                                     _i32p, _f32p, _i32p]),
    ("afs_eval_noalloc", ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("afs_probe_fma", ctypes.c_int, [_i32, _i32, _i32, _vp, _f64p, _vp]),
    ("afs_probe_mfma_bf16", ctypes.c_int, [_i32, _i32, _vp, _f64p, _vp]),
    ("afs_probe_copy", ctypes.c_int, [_vp, _vp, ctypes.c_int64, _i32, _vp]),
]

FORM_A, FORM_B = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libafsat.so is not built (run: python -m paper_2606_06641_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != AFS_OK:
        raise AfsError(rc, lib().afs_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a, ctype):
    return None if a is None else a.ctypes.data_as(ctype)


def form_tables(ctype: int, k: int, param: int, form: int):
    """(alpha, beta, d) complex128 [k+1] of one constraint in form A (the
    paper's +-1 ESP basis) or form B (count basis); see afs_form_tables."""
    arrs = [np.zeros(2 * (k + 1)) for _ in range(3)]
    _check(lib().afs_form_tables(int(ctype), int(k), int(param), int(form), *[_np_ptr(a, _f64p) for a in arrs]))
    return tuple(a[0::2] + 1j * a[1::2] for a in arrs)


def fe_generic(tables, y, fp64=True):
    """FE(y) = Re sum_m d_m prod_i (alpha_m + beta_m y[i]) on the GPU in FP64 or
    FP32 for the points y (torch f64 (k, B) on a device)."""
    alpha, beta, d = (np.ascontiguousarray(np.stack([t.real, t.imag], axis=1).ravel()) for t in tables)
    k = len(alpha) // 2 - 1
    if y.dtype != torch.float64 or y.dim() != 2 or y.shape[0] != k or not y.is_contiguous():
        raise ValueError("y must be contiguous float64 shaped (k, B)")
    fe = torch.empty(y.shape[1], dtype=torch.float64, device=y.device)
    _check(lib().afs_fe_generic(k, _np_ptr(alpha, _f64p), _np_ptr(beta, _f64p), _np_ptr(d, _f64p), int(bool(fp64)),
                                y.shape[1], _ptr(y), _ptr(fe), y.device.index or 0, _stream(y.device)))
    return fe


def coefficients(ctype: int, k: int, param: int = 0):
    """FP64 coefficient vector d_m, m = 0..k (inverse DFT of the truth table)."""
    re = np.zeros(k + 1)
    im = np.zeros(k + 1)
    _check(lib().afs_coefficients(int(ctype), int(k), int(param), _np_ptr(re, _f64p), _np_ptr(im, _f64p)))
    return re + 1j * im


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class BucketInfo:
    k_lo: int
    k_hi: int
    n_cons: int
    n_lits: int
    lanes_per_restart: int
    lits_per_lane: int
    slot0: int
    tile: int = 0
    rpl: int = 0


class Instance:
    """A packed instance: n variables, symmetric constraints in CSR form.

    ``device`` is a CUDA/HIP device ordinal, or -1 for a host-only instance
    (tables and layout can be inspected; device calls raise)."""

    def __init__(self, n, con_off, lits, types, params=None, weights=None, device=0,
                 shapes=None, tile_short=0, tile_long=0):
        """``shapes``: optional kernel configurations as chosen by the autotuner:
        entries (k_hi, lanes, seg[, tile[, rpl]]).  Entries with lanes > 1 give the
        segment shape (and work tile) for lengths > 16, ascending k_hi; entries with
        lanes == 1 give the one-lane kernel's work tile and restarts per lane for the
        length k_hi <= 16 (seg == k_hi).  A tile or rpl of 0 keeps the default."""
        con_off = np.ascontiguousarray(con_off, dtype=np.int64)
        lits = np.ascontiguousarray(lits, dtype=np.int32)
        types = np.ascontiguousarray(types, dtype=np.int32)
        params = None if params is None else np.ascontiguousarray(params, dtype=np.int32)
        weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        shapes = list(shapes or [])
        opts, keep = self._options(shapes, tile_short, tile_long)
        h = ctypes.c_void_p()
        _check(lib().afs_instance_create_ex(int(n), len(types), _np_ptr(con_off, _i64p), _np_ptr(lits, _i32p),
                                            _np_ptr(types, _i32p), _np_ptr(params, _i32p),
                                            _np_ptr(weights, _f32p), ctypes.byref(opts), int(device),
                                            ctypes.byref(h)))
        self._attach(h, shapes)

    @staticmethod
    def _options(shapes, tile_short, tile_long):
        full = [tuple(sh) + (0,) * (5 - len(sh)) for sh in (shapes or [])]
        if any(len(sh) != 5 for sh in full):
            raise ValueError("shape entries are (k_hi, lanes, seg[, tile[, rpl]])")
        seg = [sh for sh in full if sh[1] != 1]
        arrs = [np.array([sh[i] for sh in seg], dtype=np.int32) for i in range(4)]
        short_tile = np.zeros(16, np.int32)
        short_rpl = np.zeros(16, np.int32)
        for k, _, s_, tile, rpl in (sh for sh in full if sh[1] == 1):
            if not 1 <= k <= 16 or s_ != k:
                raise ValueError("a one-lane entry needs k_hi == seg in 1..16")
            short_tile[k - 1], short_rpl[k - 1] = tile, rpl
        arrs += [short_tile, short_rpl]
        opts = _Options(len(seg), _np_ptr(arrs[0], _i32p), _np_ptr(arrs[1], _i32p), _np_ptr(arrs[2], _i32p),
                        int(tile_short), int(tile_long), _np_ptr(arrs[3], _i32p), _np_ptr(short_tile, _i32p),
                        _np_ptr(short_rpl, _i32p))
        return opts, arrs

    @classmethod
    def batch(cls, parts, device=0, shapes=None, tile_short=0, tile_long=0):
        """Block-diagonal batch of independent instances (each an object with
        ``n, con_off, lits, types, params, weights`` or an ``Instance``): one set
        of launches covers all of them; per-restart state is [n_inst][B]."""
        made = [p if isinstance(p, Instance) else cls.from_arrays(p, device=-1) for p in parts]
        handles = (ctypes.c_void_p * len(made))(*[m._h.value for m in made])
        opts, keep = cls._options(shapes, tile_short, tile_long)
        h = ctypes.c_void_p()
        _check(lib().afs_batch_create(ctypes.cast(handles, ctypes.POINTER(_vp)), len(made), ctypes.byref(opts),
                                      int(device), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._attach(h, list(shapes or []))
        return self

    def _attach(self, h, shapes):
        self.shapes = shapes
        self._h = h
        info = _Info()
        _check(lib().afs_instance_info(h, ctypes.byref(info)))
        self.n = info.n_vars
        self.n_cons = info.n_cons
        self.n_lits = info.n_lits
        self.n_buckets = info.n_buckets
        self.n_tables = info.n_tables
        self.max_k = info.max_k
        self.device = info.device
        self.n_inst = info.n_inst
        self._ws = {}

    @classmethod
    def from_arrays(cls, inst, device=0, **kw):
        """From any object with ``n, con_off, lits, types, params, weights``."""
        return cls(inst.n, inst.con_off, inst.lits, inst.types, getattr(inst, "params", None),
                   getattr(inst, "weights", None), device=device, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().afs_instance_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout --------------------------------------------------------------------
    def buckets(self):
        out = []
        for b in range(self.n_buckets):
            bi = _BucketInfo()
            _check(lib().afs_bucket_info_get(self._h, b, ctypes.byref(bi)))
            out.append(BucketInfo(bi.k_lo, bi.k_hi, bi.n_cons, bi.n_lits, bi.lanes_per_restart,
                                  bi.lits_per_lane, bi.slot0, bi.tile, bi.rpl))
        return out

    def var_offsets(self):
        """First variable of each part (int32 [n_inst+1]); [0, n] for a plain instance."""
        a = np.zeros(self.n_inst + 1, dtype=np.int32)
        _check(lib().afs_batch_var_offsets(self._h, _np_ptr(a, _i32p)))
        return a

    def slot_map(self):
        a = np.zeros(self.n_lits, dtype=np.int64)
        _check(lib().afs_instance_slot_map(self._h, _np_ptr(a, _i64p)))
        return a

    def transpose(self):
        voff = np.zeros(self.n + 1, dtype=np.int64)
        vslot = np.zeros(self.n_lits, dtype=np.int64)
        _check(lib().afs_instance_transpose(self._h, _np_ptr(voff, _i64p), _np_ptr(vslot, _i64p)))
        return voff, vslot

    def workspace_bytes(self, B):
        nb = ctypes.c_size_t()
        _check(lib().afs_workspace_bytes(self._h, int(B), ctypes.byref(nb)))
        return nb.value

    def workspace(self, B):
        ws = self._ws.get(B)
        if ws is None:
            nbytes = self.workspace_bytes(B)
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self._dev())
            self._ws = {B: ws}          # keep one workspace at a time
        return ws

    def search_workspace(self, B):
        """Second workspace of the line search (one kept at a time)."""
        sws = getattr(self, "_sws", {}).get(B)
        if sws is None:
            nb = ctypes.c_size_t()
            _check(lib().afs_search_workspace_bytes(self._h, int(B), ctypes.byref(nb)))
            sws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self._dev())
            self._sws = {B: sws}
        return sws

    def _dev(self):
        if self.device < 0:
            raise AfsError(AFS_ESTATE, "host-only instance")
        return torch.device("cuda", self.device)

    def _check_x(self, x, name="x"):
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float32 and x.is_cuda
                and x.dim() == 2 and x.shape[0] == self.n and x.is_contiguous()):
            raise ValueError("%s must be a contiguous float32 CUDA tensor of shape (n, B)" % name)
        if x.device.index != self.device:
            raise ValueError("%s is on device %s, instance on %d" % (name, x.device, self.device))
        return x.shape[1]

    # -- evaluation ------------------------------------------------------------------
    def eval(self, x, obj=True, grad=True, fe=False, adj=False, ws=None):
        """FE / objective / gradient at the columns of x (n, B)."""
        B = self._check_x(x)
        dev = self._dev()
        ws = self.workspace(B) if ws is None else ws
        out = {}
        if obj:
            out["obj"] = torch.empty(B, dtype=torch.float32, device=dev)
        if grad:
            out["grad"] = torch.empty((self.n, B), dtype=torch.float32, device=dev)
        if fe:
            out["fe"] = torch.empty((self.n_cons, B), dtype=torch.float32, device=dev)
        if adj:
            out["adj"] = torch.empty((self.n_lits, B), dtype=torch.float32, device=dev)
        _check(lib().afs_eval(self._h, B, _ptr(x), _ptr(ws), ws.numel(), _ptr(out.get("obj")),
                              _ptr(out.get("grad")), _ptr(out.get("fe")), _ptr(out.get("adj")),
                              _stream(dev)))
        return out

    def eval_noalloc(self, x, obj=True, grad=True, fe=False, adj=False, out=None):
        """afs_eval_noalloc: as eval, with the library's static scratch in place of a
        workspace.  `out` may hold preallocated outputs (dict of the same keys)."""
        B = self._check_x(x)
        dev = self._dev()
        out = {} if out is None else dict(out)
        shapes = {"obj": (B,), "grad": (self.n, B), "fe": (self.n_cons, B), "adj": (self.n_lits, B)}
        for k, want in (("obj", obj), ("grad", grad), ("fe", fe), ("adj", adj)):
            if want and k not in out:
                out[k] = torch.empty(shapes[k], dtype=torch.float32, device=dev)
        _check(lib().afs_eval_noalloc(self._h, B, _ptr(x), _ptr(out.get("obj")), _ptr(out.get("grad")),
                                      _ptr(out.get("fe")), _ptr(out.get("adj")), _stream(dev)))
        return out

    def fe_grad(self, x, ws, bucket_lo=0, bucket_hi=None, want_obj=False, fe=None):
        B = self._check_x(x)
        hi = self.n_buckets if bucket_hi is None else bucket_hi
        _check(lib().afs_fe_grad(self._h, B, _ptr(x), _ptr(ws), ws.numel(), int(bucket_lo), int(hi),
                                 int(bool(want_obj)), _ptr(fe), _stream(self._dev())))

    def fe_grad_buckets(self, x, ws, buckets, want_obj=False, fe=None):
        """afs_fe_grad over the listed bucket indices in one call."""
        B = self._check_x(x)
        idx = np.ascontiguousarray(buckets, dtype=np.int32)
        _check(lib().afs_fe_grad_buckets(self._h, B, _ptr(x), _ptr(ws), ws.numel(), _np_ptr(idx, _i32p), len(idx),
                                         int(bool(want_obj)), _ptr(fe), _stream(self._dev())))

    def scatter(self, B, ws, obj=None, grad=None):
        _check(lib().afs_scatter(self._h, int(B), _ptr(ws), ws.numel(), _ptr(obj), _ptr(grad),
                                 _stream(self._dev())))

    # -- differentiation -----------------------------------------------------------
    def eval_fwd(self, x, fe=False, ws=None):
        """Objective per restart without adjoint work: obj (B,) [, fe (C, B)]."""
        B = self._check_x(x)
        dev = self._dev()
        ws = self.workspace(B) if ws is None else ws
        obj = torch.empty(B, dtype=torch.float32, device=dev)
        fe_t = torch.empty((self.n_cons, B), dtype=torch.float32, device=dev) if fe else None
        _check(lib().afs_eval_fwd(self._h, B, _ptr(x), _ptr(ws), ws.numel(), _ptr(obj), _ptr(fe_t),
                                  _stream(dev)))
        return (obj, fe_t) if fe else obj

    def eval_adjoint(self, x, dobj=None, ws=None, adj=False):
        """grad[v][b] = dobj[b] * dF_b/dx[v][b] (products recomputed from x); with
        adj, also the per-literal terms (L, B) in input literal order: (grad, adj)."""
        B = self._check_x(x)
        dev = self._dev()
        if dobj is not None and not (dobj.dtype == torch.float32 and dobj.is_cuda and dobj.numel() == B
                                     and dobj.is_contiguous()):
            raise ValueError("dobj must be a contiguous float32 CUDA tensor of B elements")
        ws = self.workspace(B) if ws is None else ws
        grad = torch.empty((self.n, B), dtype=torch.float32, device=dev)
        adj_t = torch.empty((self.n_lits, B), dtype=torch.float32, device=dev) if adj else None
        _check(lib().afs_eval_adjoint(self._h, B, _ptr(x), _ptr(dobj), _ptr(ws), ws.numel(), _ptr(grad),
                                      _ptr(adj_t), _stream(dev)))
        return (grad, adj_t) if adj else grad

    # -- Algorithm 1 -------------------------------------------------------------------
    def _fixed(self, fixed):
        """(pointer, rows) of a fixed mask shaped (n,) or (n_partial, n), u8 or i8."""
        if fixed is None:
            return None, 0
        if fixed.dtype not in (torch.uint8, torch.int8) or fixed.shape[-1] != self.n or fixed.dim() > 2:
            raise ValueError("fixed must be u8/i8 shaped (n,) or (n_partial, n)")
        if not fixed.is_contiguous() or fixed.device != self._dev():
            raise ValueError("fixed must be contiguous on the instance's device")
        return _ptr(fixed), (fixed.shape[0] if fixed.dim() == 2 else 1)

    def step(self, x, grad, lr, fixed=None, done=None):
        """x <- clip(x - lr*grad, -1, 1) in place, except fixed variables / done restarts."""
        B = self._check_x(x)
        self._check_x(grad, "grad")
        fp, rows = self._fixed(fixed)
        _check(lib().afs_step(self._h, B, _ptr(x), _ptr(grad), float(lr), fp, rows, _ptr(done),
                              _stream(self._dev())))
        return x

    def init_points(self, B, seed, values=None):
        """Starting points (n, B): the rows ``values`` (i8 (n,) or (n_partial, n):
        +1 True, -1 False, 0 random) fixed, the rest uniform on [-1, 1) from the
        library's counter-based generator."""
        x = torch.empty((self.n, B), dtype=torch.float32, device=self._dev())
        vp, rows = self._fixed(values)
        _check(lib().afs_init_points(self._h, int(B), int(seed) & (2 ** 64 - 1), vp, rows, _ptr(x),
                                     _stream(self._dev())))
        return x

    def round_verify(self, x, want_bits=False, done=None):
        """Exact unsat count per restart (int32 [B], or [n_inst, B] for a batch);
        optionally the packed bits."""
        B = self._check_x(x)
        dev = self._dev()
        unsat = torch.empty((self.n_inst, B) if self.n_inst > 1 else (B,), dtype=torch.int32, device=dev)
        bits = torch.empty((self.n, (B + 31) // 32), dtype=torch.int32, device=dev) if want_bits else None
        ws = self.workspace(B)
        _check(lib().afs_round_verify(self._h, B, _ptr(x), _ptr(bits), _ptr(ws), ws.numel(), _ptr(unsat),
                                      _ptr(done), _stream(dev)))
        return (unsat, bits) if want_bits else unsat

    def pgd_state(self, B):
        """Device state of Algorithm 1: per-(part, restart) arrays shaped (B,) for a
        plain instance and (n_inst, B) for a batch."""
        dev = self._dev()
        shp = (self.n_inst, B) if self.n_inst > 1 else (B,)
        return {"unsat": torch.zeros(shp, dtype=torch.int32, device=dev),
                "done": torch.zeros(shp, dtype=torch.uint8, device=dev),
                "first_sat": torch.full(shp, -1, dtype=torch.int32, device=dev),
                "counter": torch.zeros(4, dtype=torch.int32, device=dev)}

    @staticmethod
    def _state_struct(st):
        return _PgdState(st["unsat"].data_ptr(), st["done"].data_ptr(), st["first_sat"].data_ptr(),
                         st["counter"].data_ptr())

    def pgd_init(self, x, st, ws=None):
        B = self._check_x(x)
        ws = self.workspace(B) if ws is None else ws
        s = self._state_struct(st)
        _check(lib().afs_pgd_init(self._h, B, _ptr(x), _ptr(ws), ws.numel(), ctypes.byref(s),
                                  _stream(self._dev())))

    def pgd_step(self, x, st, lr, fixed=None, ws=None):
        B = self._check_x(x)
        ws = self.workspace(B) if ws is None else ws
        s = self._state_struct(st)
        fp, rows = self._fixed(fixed)
        _check(lib().afs_pgd_step(self._h, B, _ptr(x), float(lr), fp, rows, _ptr(ws), ws.numel(),
                                  ctypes.byref(s), _stream(self._dev())))

    def pgd_update(self, x, st, lr, fixed=None, ws=None):
        B = self._check_x(x)
        ws = self.workspace(B) if ws is None else ws
        s = self._state_struct(st)
        fp, rows = self._fixed(fixed)
        _check(lib().afs_pgd_update(self._h, B, _ptr(x), float(lr), fp, rows, _ptr(ws), ws.numel(),
                                    ctypes.byref(s), _stream(self._dev())))

    def pgd_step_momentum(self, x, vel, st, lr, mu, fixed=None, ws=None):
        """One iteration of projected gradient descent with heavy-ball momentum
        (afs_pgd_step_momentum): vel <- mu vel + grad, x <- clip(x - lr vel), then
        the exact count and the state update.  vel: float32 CUDA (n, B), zero
        before the first step, updated in place."""
        B = self._check_x(x)
        if self._check_x(vel, "vel") != B:
            raise ValueError("vel must have the shape of x")
        ws = self.workspace(B) if ws is None else ws
        s = self._state_struct(st)
        fp, rows = self._fixed(fixed)
        _check(lib().afs_pgd_step_momentum(self._h, B, _ptr(x), _ptr(vel), float(lr), float(mu), fp, rows,
                                           _ptr(ws), ws.numel(), ctypes.byref(s), _stream(self._dev())))

    @staticmethod
    def _search(search):
        if isinstance(search, LineSearch):
            search = (search.max_step, search.shrink, search.armijo, search.trials)
        return _LineSearch(float(search[0]), float(search[1]), float(search[2]), int(search[3]))

    def search_step(self, x, st, search, fixed=None, delta=0.0, eta=None, ws=None):
        """One iteration of Algorithm 1 with the backtracking line search
        (``search``: a ``LineSearch`` or (max_step, shrink, armijo, trials)).
        ``eta`` (f32 (B,), optional) receives the chosen step lengths."""
        B = self._check_x(x)
        ws = self.workspace(B) if ws is None else ws
        sws = self.search_workspace(B)
        ls = self._search(search)
        s = self._state_struct(st)
        fp, rows = self._fixed(fixed)
        _check(lib().afs_pgd_search_step(self._h, B, _ptr(x), ctypes.byref(ls), fp, rows, float(delta), _ptr(ws),
                                         ws.numel(), _ptr(sws), sws.numel(), ctypes.byref(s), _ptr(eta),
                                         _stream(self._dev())))

    def pgd(self, x, lr, steps, fixed=None, poll=10, stop_on_sat=True, graph=True, obj=False, search=None,
            delta=0.0, epsilon=0.0, momentum=0.0, velocity=None):
        """Algorithm 1 on the columns of x (updated in place), run by the
        library's driver (afs_pgd): constant step ``lr``, or with ``search`` (a
        ``LineSearch`` or (max_step, shrink, armijo, trials)) the backtracking
        line search.  ``fixed``: u8/i8 (n,) or (n_partial, n) mask of held
        variables, the restarts divided evenly among its rows; ``delta`` > 0
        stops restarts whose step length falls below it, ``epsilon`` > 0 those
        whose point moves less than it in every variable.  ``momentum`` > 0
        takes heavy-ball momentum steps in PGD's place (afs_pgd_step_momentum);
        ``velocity`` (float32 CUDA (n, B), zero by default) holds and returns the
        velocity.

        Stops after ``steps`` iterations, or (``stop_on_sat``) once any restart
        verifies, or once every restart has verified or converged; the driver
        reads the counter every ``poll`` iterations.  With ``graph`` the driver
        captures ``poll`` iterations (at most 64) once in a HIP graph and replays
        it.
        Returns the state (unsat, done, first_sat, counter), x, the number of
        iterations and, with ``obj``, the objective at the final point."""
        B = self._check_x(x)
        st = self.pgd_state(B)
        ws = self.workspace(B)
        fp, rows = self._fixed(fixed)
        ls = self._search(search) if search is not None else None
        sws = self.search_workspace(B) if search is not None else None
        if momentum and velocity is None:
            velocity = torch.zeros_like(x)
        if velocity is not None and self._check_x(velocity, "velocity") != B:
            raise ValueError("velocity must have the shape of x")
        prm = _PgdParams(float(lr), int(steps), int(poll), int(bool(stop_on_sat)), int(bool(graph)),
                         None if fp is None else fp.value, int(rows), float(delta),
                         ctypes.pointer(ls) if ls is not None else None,
                         None if sws is None else sws.data_ptr(), 0 if sws is None else sws.numel(),
                         float(epsilon), float(momentum), None if velocity is None else velocity.data_ptr())
        s = self._state_struct(st)
        o = torch.empty(B, dtype=torch.float32, device=self._dev()) if obj else None
        iters = _i32(0)
        _check(lib().afs_pgd(self._h, B, _ptr(x), ctypes.byref(prm), _ptr(ws), ws.numel(), ctypes.byref(s),
                             _ptr(o), ctypes.byref(iters), _stream(self._dev())))
        st["x"] = x
        st["iters"] = int(iters.value)
        if velocity is not None:
            st["velocity"] = velocity
        if obj:
            st["obj"] = o
        return st


@dataclass
class LineSearch:
    """Backtracking line search of Algorithm 1 (see ``afs_line_search``)."""
    max_step: float = 1.0
    shrink: float = 0.5
    armijo: float = 1e-4
    trials: int = 8


@dataclass
class Parsed:
    """An input file after the reader's simplifications (App. A): the kept
    constraints in the arrays ``Instance`` takes, and ``units`` (int8 [n]: +1
    fixed True, -1 fixed False, 0 free), the partial assignment of Sec. 3.4."""
    n: int
    con_off: np.ndarray
    lits: np.ndarray
    types: np.ndarray
    params: np.ndarray
    units: np.ndarray
    n_dropped: int
    declared_cons: int
    weights: Optional[np.ndarray] = None
    _h: Optional[ctypes.c_void_p] = field(default=None, repr=False, compare=False)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.afs_parsed_destroy(self._h)
            self._h = None

    def fixed_mask(self, device=0):
        """u8 [n] device mask of the fixed variables (the ``fixed`` argument of
        ``step`` and ``pgd``)."""
        return torch.from_numpy((self.units != 0).astype(np.uint8)).to(device)

    def fold_units(self, partials=None):
        """Partial assignments with the units written in (Sec. 3.4): i8
        (n_partial, n) from ``partials`` (array-like (n,) or (n_partial, n), +1
        True, -1 False, 0 free), or the units alone as one row.  Raises
        ``AfsError`` (AFS_EUNSAT) when a unit contradicts a row."""
        if partials is None:
            vals = np.zeros((1, self.n), dtype=np.int8)
        else:
            vals = np.array(partials, dtype=np.int8, ndmin=2, order="C", copy=True)
            if vals.ndim != 2 or vals.shape[1] != self.n:
                raise ValueError("partials must be shaped (n,) or (n_partial, n)")
        _check(lib().afs_parsed_fold_units(self._h, vals.shape[0], _np_ptr(vals, ctypes.POINTER(ctypes.c_int8))))
        return vals

    def apply_units(self, x):
        """Set the fixed variables' rows of x (n, B) to their values in place
        (True is -1, False is +1)."""
        idx = np.nonzero(self.units)[0]
        if idx.size:
            vals = torch.from_numpy(-self.units[idx].astype(np.float32)).to(x.device)
            x[torch.from_numpy(idx).to(x.device)] = vals[:, None].to(x.dtype)
        return x


def _take_parsed(h):
    """Parsed from a reader handle; the handle stays with the result (unit folding
    reads it) and is freed with it."""
    try:
        info = _ParsedInfo()
        _check(lib().afs_parsed_get_info(h, ctypes.byref(info)))
        con_off = np.zeros(info.n_cons + 1, dtype=np.int64)
        lits = np.zeros(info.n_lits, dtype=np.int32)
        types = np.zeros(info.n_cons, dtype=np.int32)
        params = np.zeros(info.n_cons, dtype=np.int32)
        units = np.zeros(info.n_vars, dtype=np.int8)
        _check(lib().afs_parsed_arrays(h, _np_ptr(con_off, _i64p), _np_ptr(lits, _i32p), _np_ptr(types, _i32p),
                                       _np_ptr(params, _i32p), _np_ptr(units, ctypes.POINTER(ctypes.c_int8))))
    except BaseException:
        lib().afs_parsed_destroy(h)
        raise
    return Parsed(int(info.n_vars), con_off, lits, types, params, units, int(info.n_dropped),
                  int(info.declared_cons), None, h)


def parse_text(text):
    """Parse DIMACS CNF or the hybrid format of App. A from a string or bytes.
    Raises ``AfsError`` (status ``AFS_EUNSAT`` when the simplifications prove the
    input unsatisfiable, ``AFS_EINVAL`` for malformed input)."""
    data = text.encode() if isinstance(text, str) else bytes(text)
    h = ctypes.c_void_p()
    _check(lib().afs_parse_text(data, len(data), ctypes.byref(h)))
    return _take_parsed(h)


def parse_file(path):
    """``parse_text`` of the file at ``path``."""
    h = ctypes.c_void_p()
    _check(lib().afs_parse_file(os.fsencode(path), ctypes.byref(h)))
    return _take_parsed(h)


@dataclass
class Decomposed:
    """An instance after long-constraint decomposition (Sec. 5): the arrays
    ``Instance`` takes over ``n`` variables, the first ``n_orig`` of them the
    input's and the rest auxiliary, and ``origin`` (int32 [C]), the input
    constraint each constraint came from.  A solution's first ``n_orig``
    variables solve the input."""
    n: int
    n_orig: int
    con_off: np.ndarray
    lits: np.ndarray
    types: np.ndarray
    params: np.ndarray
    origin: np.ndarray
    weights: Optional[np.ndarray] = None


def decompose(inst, max_len):
    """Split every OR, XOR, NAE, AMO and EO constraint of ``inst`` (any object with
    ``n, con_off, lits, types, params`` and optionally ``weights``) longer than
    ``max_len`` into a chain of pieces of at most ``max_len`` literals joined by
    auxiliary variables; see afs_decompose in afsat.h."""
    n = int(inst.n)
    con_off = np.ascontiguousarray(inst.con_off, dtype=np.int64)
    lits = np.ascontiguousarray(inst.lits, dtype=np.int32)
    types = np.ascontiguousarray(inst.types, dtype=np.int32)
    C = len(types)
    params = getattr(inst, "params", None)
    params = np.zeros(C, np.int32) if params is None else np.ascontiguousarray(params, dtype=np.int32)
    weights = getattr(inst, "weights", None)
    weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    if len(con_off) != C + 1 or len(params) != C or (weights is not None and len(weights) != C):
        raise ValueError("con_off, types, params and weights disagree on the constraint count")
    if int(con_off[-1]) != len(lits):
        raise ValueError("con_off[-1] must equal len(lits)")
    n_out, c_out, l_out = _i32(), _i32(), ctypes.c_int64()
    _check(lib().afs_decompose_size(n, C, _np_ptr(con_off, _i64p), _np_ptr(types, _i32p), int(max_len),
                                    ctypes.byref(n_out), ctypes.byref(c_out), ctypes.byref(l_out)))
    co = np.zeros(c_out.value + 1, np.int64)
    lo = np.zeros(l_out.value, np.int32)
    to, po, og = (np.zeros(c_out.value, np.int32) for _ in range(3))
    wo = None if weights is None else np.zeros(c_out.value, np.float32)
    _check(lib().afs_decompose(n, C, _np_ptr(con_off, _i64p), _np_ptr(lits, _i32p), _np_ptr(types, _i32p),
                               _np_ptr(params, _i32p), _np_ptr(weights, _f32p), int(max_len), _np_ptr(co, _i64p),
                               _np_ptr(lo, _i32p), _np_ptr(to, _i32p), _np_ptr(po, _i32p), _np_ptr(wo, _f32p),
                               _np_ptr(og, _i32p)))
    return Decomposed(int(n_out.value), n, co, lo, to, po, og, wo)


class FEObjective(torch.autograd.Function):
    """F(x) = sum_c w_c FE_c(x) per restart, differentiable in x.

    ``obj = FEObjective.apply(x, inst)`` with x a float32 CUDA tensor (n, B) gives
    obj (B,); the backward pass runs the library's adjoint kernels, recomputing the
    products from x (only x is saved)."""

    @staticmethod
    def forward(ctx, x, inst):
        x = x.contiguous()
        ctx.inst = inst
        ctx.save_for_backward(x)
        return inst.eval_fwd(x)

    @staticmethod
    def backward(ctx, gobj):
        (x,) = ctx.saved_tensors
        g = ctx.inst.eval_adjoint(x, gobj.contiguous().to(torch.float32))
        return g, None


def probe(kind, blocks, iters=0, nbytes=0, device=0, variant=0):
    """Enqueue one peak-probe launch (afs_probe_*) on the current stream of
    `device` and return the work it does: flops for "fma" (of `variant`) and
    "mfma_bf16", bytes moved (read + write) for "copy".  The caller times the
    launch."""
    dev = torch.device("cuda", device)
    st = _stream(device)
    if kind == "copy":
        if not hasattr(probe, "_bufs") or probe._bufs[0].numel() * 4 != nbytes:
            probe._bufs = (torch.ones(nbytes // 4, dtype=torch.float32, device=dev),
                           torch.empty(nbytes // 4, dtype=torch.float32, device=dev))
        src, dst = probe._bufs
        _check(lib().afs_probe_copy(_ptr(src), _ptr(dst), int(nbytes), int(blocks), st))
        return 2.0 * nbytes
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    flops = ctypes.c_double()
    if kind == "fma":
        _check(lib().afs_probe_fma(int(variant), int(blocks), int(iters), _ptr(out), ctypes.byref(flops), st))
    else:
        _check(lib().afs_probe_mfma_bf16(int(blocks), int(iters), _ptr(out), ctypes.byref(flops), st))
    probe._out = out                  # kept alive until the next probe call
    return flops.value

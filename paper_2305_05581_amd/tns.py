"""ctypes binding of ``libtns.so`` (argument marshalling only).

Every step of sigma = H_eff psi runs in the library's HIP kernels; this module
only lays out host tables, owns the device buffers (torch tensors) and passes
pointers and the current torch stream.  A missing library raises at first
use: there is no CPU fallback.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtns.so")

F64, F32, BF16X3 = 0, 1, 2
PREC_NAMES = {F64: "f64", F32: "f32", BF16X3: "bf16x3"}
_PREC_OF = {"f64": F64, "f32": F32, "bf16x3": BF16X3}

STATUS = {0: "ok", -1: "invalid argument", -2: "inconsistent shape or offset", -3: "quantum numbers not conserved",
          -4: "workspace too small", -5: "HIP runtime error", -6: "non-finite value", -7: "not converged"}

# 40-byte task record (see include/tns.h)
TASK_DTYPE = np.dtype([("out", "<i4"), ("in", "<i4"), ("term", "<i4"), ("lblk", "<i4"),
                       ("rblk", "<i4"), ("order", "<i4"), ("alpha", "<f8"), ("cost", "<i8")])

_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class TnsProblem(ctypes.Structure):
    _fields_ = [("nL", _i32), ("nR", _i32), ("nS", _i32), ("nOps", _i32), ("nBlk", _i32), ("nTerms", _i32),
                ("target_N", _i32), ("target_2Sz", _i32), ("n_vals", _i64)] + \
               [(n, _P) for n in ("qL", "dimL", "qR", "dimR", "psi_sec", "psi_off", "op_side", "op_dN", "op_d2Sz",
                                  "blk_op", "blk_in", "blk_out", "blk_rows", "blk_cols", "blk_ld", "blk_off",
                                  "term_L", "term_ma", "term_mb", "term_R", "term_coef")]


class TnsTasklist(ctypes.Structure):
    _fields_ = [("ntasks", _i64), ("nitems", _i64), ("nslots", _i64), ("partial_elems", _i64),
                ("total_flops", _i64), ("psi_dim", _i64), ("tasks", _P), ("out_ptr", _P),
                ("opaque", ctypes.c_uint8 * 2048)]


class TnsDavidsonOpts(ctypes.Structure):
    _fields_ = [("max_sub", _i32), ("keep", _i32), ("max_iter", _i32), ("refine", _i32),
                ("tol_res", ctypes.c_double), ("tol_e", ctypes.c_double), ("inner", _i32)]


class TnsDavidsonInfo(ctypes.Structure):
    _fields_ = [("iters", _i32), ("matvecs_lo", _i32), ("matvecs_f64", _i32),
                ("res_norm", ctypes.c_double), ("e_lo", ctypes.c_double)]


class TnsRenormProblem(ctypes.Structure):
    _fields_ = [("nL", _i32), ("qL", _P), ("dimL", _P), ("nOps", _i32), ("nBlk", _i32), ("op_dN", _P),
                ("op_d2Sz", _P), ("blk_op", _P), ("blk_in", _P), ("blk_out", _P), ("blk_rows", _P), ("blk_cols", _P),
                ("blk_ld", _P), ("blk_off", _P), ("n_vals", _i64), ("nQ", _i32), ("qQ", _P), ("keep", _P),
                ("u_off", _P), ("n_u", _i64), ("nNew", _i32), ("nTerms", _i32), ("term_new", _P), ("term_op", _P),
                ("term_mono", _P), ("term_coef", _P)]


class TnsRenormPlan(ctypes.Structure):
    _fields_ = [("ntasks", _i64), ("n_out_blk", _i64), ("out_elems", _i64), ("total_flops", _i64),
                ("tl", TnsTasklist), ("opaque", ctypes.c_uint8 * 1024)]


class TnsTtcachePlan(ctypes.Structure):
    _fields_ = [("n_epochs", _i64), ("n_loads", _i64), ("loaded_elems", _i64), ("naive_elems", _i64),
                ("ntasks", _i64), ("total_flops", _i64), ("cache_elems", _i64), ("halves", _i64),
                ("opaque", ctypes.c_uint8 * 256)]


class TnsSu2Problem(ctypes.Structure):
    _fields_ = [("nL", _i32), ("nR", _i32), ("nOps", _i32), ("nBlk", _i32), ("nTerms", _i32), ("target_N", _i32),
                ("target_2S", _i32), ("n_vals", _i64)] + \
               [(n, _P) for n in ("qL", "dimL", "qR", "dimR", "op_side", "op_2k", "op_dN", "blk_op", "blk_in",
                                  "blk_out", "blk_rows", "blk_cols", "blk_ld", "blk_off", "term_L", "term_R",
                                  "term_coef")]


class TnsSu2Plan(ctypes.Structure):
    _fields_ = [("n_sectors", _i64), ("psi_dim", _i64), ("ntasks", _i64), ("total_flops", _i64),
                ("tl", TnsTasklist)]


EXPORTS = ("tns_tasklist_workspace_bytes", "tns_count_tasks", "tns_build_tasklist", "tns_apply_workspace_bytes",
           "tns_prepare_operands", "tns_apply_heff", "tns_backward_workspace_bytes", "tns_apply_heff_backward",
           "tns_davidson_workspace_bytes", "tns_davidson", "tns_status_string")

_lib = None


def library(path=LIB_PATH):
    """Load ``libtns.so`` (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtns.so is not built; run `python -m paper_2305_05581_amd.build`")
    L = ctypes.CDLL(path)
    sz = ctypes.c_size_t
    L.tns_tasklist_workspace_bytes.restype = sz
    L.tns_tasklist_workspace_bytes.argtypes = [ctypes.POINTER(TnsProblem)]
    L.tns_count_tasks.restype = ctypes.c_int
    L.tns_count_tasks.argtypes = [ctypes.POINTER(TnsProblem), ctypes.POINTER(ctypes.c_int64)]
    L.tns_build_tasklist.restype = ctypes.c_int
    L.tns_build_tasklist.argtypes = [ctypes.POINTER(TnsProblem), _P, sz, ctypes.POINTER(TnsTasklist), _P]
    L.tns_apply_workspace_bytes.restype = sz
    L.tns_apply_workspace_bytes.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int]
    L.tns_prepare_operands.restype = ctypes.c_int
    L.tns_prepare_operands.argtypes = [ctypes.c_int, _P, _i64, _P, _P]
    L.tns_apply_heff.restype = ctypes.c_int
    L.tns_apply_heff.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int, _P, _P, _P, ctypes.c_double, _P, sz, _P]
    if hasattr(L, "tns_apply_heff_noalloc"):
        L.tns_apply_heff_noalloc.restype = ctypes.c_int
        L.tns_apply_heff_noalloc.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int, _P, _P, _P, ctypes.c_double,
                                             _P]
    if hasattr(L, "tns_apply_heff_backward"):
        L.tns_backward_workspace_bytes.restype = sz
        L.tns_backward_workspace_bytes.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int]
        L.tns_apply_heff_backward.restype = ctypes.c_int
        L.tns_apply_heff_backward.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int, _P, _P, _P, _P, _P, _P, sz,
                                              _P]
    if hasattr(L, "tns_davidson"):
        L.tns_davidson_workspace_bytes.restype = sz
        L.tns_davidson_workspace_bytes.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.POINTER(TnsDavidsonOpts)]
        L.tns_davidson.restype = ctypes.c_int
        L.tns_davidson.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.POINTER(TnsDavidsonOpts), _P, _P, _P, _P,
                                   ctypes.POINTER(TnsDavidsonInfo), _P, sz, _P]
    if hasattr(L, "tns_profile_events"):
        L.tns_profile_events.restype = None
        L.tns_profile_events.argtypes = [_P, _P, _P]
    if hasattr(L, "tns_mfma_peak"):
        L.tns_mfma_peak_workspace_bytes.restype = sz
        L.tns_mfma_peak_workspace_bytes.argtypes = []
        L.tns_mfma_peak.restype = ctypes.c_int
        L.tns_mfma_peak.argtypes = [ctypes.c_int, ctypes.c_int, _P, sz, ctypes.POINTER(ctypes.c_double), _P]
    if hasattr(L, "tns_set_tiles"):
        L.tns_set_tiles.restype = ctypes.c_int
        L.tns_set_tiles.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_uint32, _P]
        L.tns_get_tiles.restype = ctypes.c_uint32
        L.tns_get_tiles.argtypes = [ctypes.POINTER(TnsTasklist)]
        L.tns_autotune_tiles.restype = ctypes.c_int
        L.tns_autotune_tiles.argtypes = [ctypes.POINTER(TnsTasklist), ctypes.c_int, _P, _P, _P, _P, sz,
                                         ctypes.POINTER(ctypes.c_uint32), _P]
        L.tns_autotune_tiles_batch.restype = ctypes.c_int
        L.tns_autotune_tiles_batch.argtypes = [ctypes.POINTER(ctypes.POINTER(TnsTasklist)), ctypes.c_int,
                                               ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                               ctypes.POINTER(_P), _P, sz, ctypes.POINTER(ctypes.c_uint32), _P]
    if hasattr(L, "tns_apply_heff_batch"):
        L.tns_apply_batch_workspace_bytes.restype = sz
        L.tns_apply_batch_workspace_bytes.argtypes = [ctypes.POINTER(ctypes.POINTER(TnsTasklist)), ctypes.c_int,
                                                      ctypes.c_int]
        L.tns_apply_heff_batch.restype = ctypes.c_int
        L.tns_apply_heff_batch.argtypes = [ctypes.POINTER(ctypes.POINTER(TnsTasklist)), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                           ctypes.c_double, _P, sz, _P]
    if hasattr(L, "tns_renorm_build"):
        L.tns_renorm_workspace_bytes.restype = sz
        L.tns_renorm_workspace_bytes.argtypes = [ctypes.POINTER(TnsRenormProblem)]
        L.tns_renorm_build.restype = ctypes.c_int
        L.tns_renorm_build.argtypes = [ctypes.POINTER(TnsRenormProblem), _P, sz, ctypes.POINTER(TnsRenormPlan), _P]
        L.tns_renorm_out_table.restype = ctypes.c_int
        L.tns_renorm_out_table.argtypes = [ctypes.POINTER(TnsRenormPlan)] + [_P] * 7
        L.tns_renorm_apply_workspace_bytes.restype = sz
        L.tns_renorm_apply_workspace_bytes.argtypes = [ctypes.POINTER(TnsRenormPlan), ctypes.c_int]
        L.tns_renormalize.restype = ctypes.c_int
        L.tns_renormalize.argtypes = [ctypes.POINTER(TnsRenormPlan), ctypes.c_int, _P, _P, _P, _P, sz, _P]
    if hasattr(L, "tns_ttcache_build"):
        L.tns_ttcache_sizes.restype = ctypes.c_int
        L.tns_ttcache_sizes.argtypes = [ctypes.POINTER(TnsProblem), _i64, _i32, ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_i64)]
        L.tns_ttcache_build.restype = ctypes.c_int
        L.tns_ttcache_build.argtypes = [ctypes.POINTER(TnsProblem), _i64, _i32, _P, sz, _P, sz,
                                        ctypes.POINTER(TnsTtcachePlan), _P]
        L.tns_ttcache_apply_workspace_bytes.restype = sz
        L.tns_ttcache_apply_workspace_bytes.argtypes = [ctypes.POINTER(TnsTtcachePlan), ctypes.c_int]
        L.tns_apply_heff_streamed.restype = ctypes.c_int
        L.tns_apply_heff_streamed.argtypes = [ctypes.POINTER(TnsTtcachePlan), ctypes.c_int, _P, _P, _P, _P, _P, sz,
                                              _P]
    if hasattr(L, "tns_su2_build"):
        L.tns_su2_workspace_bytes.restype = sz
        L.tns_su2_workspace_bytes.argtypes = [ctypes.POINTER(TnsSu2Problem)]
        L.tns_su2_tables.restype = ctypes.c_int
        L.tns_su2_tables.argtypes = [ctypes.POINTER(TnsSu2Problem), _P, _P, _P, _i64, _P, _P, _i64,
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.tns_su2_build.restype = ctypes.c_int
        L.tns_su2_build.argtypes = [ctypes.POINTER(TnsSu2Problem), _P, sz, ctypes.POINTER(TnsSu2Plan), _P]
    L.tns_status_string.restype = ctypes.c_char_p
    L.tns_status_string.argtypes = [ctypes.c_int]
    _lib = L
    return L


class TnsError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(code, "unknown"), code))
        self.code = code


def _check(code, what):
    if code != 0:
        raise TnsError(code, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def prec_id(prec):
    return _PREC_OF[prec] if isinstance(prec, str) else int(prec)


_TABLES = (("qL", np.int32), ("dimL", np.int32), ("qR", np.int32), ("dimR", np.int32),
           ("psi_sec", np.int32), ("psi_off", np.int64), ("op_side", np.int32), ("op_dN", np.int32),
           ("op_d2Sz", np.int32), ("blk_op", np.int32), ("blk_in", np.int32), ("blk_out", np.int32),
           ("blk_rows", np.int32), ("blk_cols", np.int32), ("blk_ld", np.int32), ("blk_off", np.int64),
           ("term_L", np.int32), ("term_ma", np.int32), ("term_mb", np.int32), ("term_R", np.int32),
           ("term_coef", np.float64))


def problem_struct(P, n_vals=None):
    """``(tns_problem, host arrays)`` of a problem; the arrays back the
    struct's pointers and must outlive its use."""
    host = {}
    cp = TnsProblem()
    cp.nL, cp.nR, cp.nS = P.nL, P.nR, P.nS
    cp.nOps, cp.nBlk, cp.nTerms = P.nOps, P.nBlk, P.nTerms
    cp.target_N, cp.target_2Sz = int(P.target[0]), int(P.target[1])
    cp.n_vals = len(P.op_vals) if n_vals is None else int(n_vals)
    for name, dt in _TABLES:
        a = np.ascontiguousarray(getattr(P, name), dtype=dt)
        host[name] = a
        setattr(cp, name, a.ctypes.data_as(ctypes.c_void_p) if a.size else None)
    return cp, host


def count_tasks(P):
    """Task count of a problem by the library's host rule (no device call)."""
    cp, host = problem_struct(P)
    n = ctypes.c_int64(-1)
    _check(library().tns_count_tasks(ctypes.byref(cp), ctypes.byref(n)), "tns_count_tasks")
    return int(n.value)


def tasklist_workspace_bytes(P):
    """Build-workspace bytes of a problem, 0 when it fails the library's host
    validation (no device call beyond a query of the device's unit counts)."""
    cp, host = problem_struct(P)
    return int(library().tns_tasklist_workspace_bytes(ctypes.byref(cp)))


class HeffProblem:
    """A two-site problem resident on the GPU: task table and schedule built by
    the library, FP64 operator values in HBM, operand copies per precision."""

    def __init__(self, P, device="cuda", vals64=None):
        self.P = P
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        L = library()
        cp, self._host = problem_struct(P, int(vals64.numel()) if vals64 is not None else None)
        self.cprob = cp
        nbytes = L.tns_tasklist_workspace_bytes(ctypes.byref(cp))
        if nbytes == 0:
            raise ValueError("problem failed host validation")
        self.ws_build = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.tl = TnsTasklist()
        with torch.cuda.device(self.device):
            _check(L.tns_build_tasklist(ctypes.byref(cp), _ptr(self.ws_build), int(nbytes), ctypes.byref(self.tl),
                                        _stream()), "tns_build_tasklist")
        if vals64 is None:
            vals64 = torch.from_numpy(np.ascontiguousarray(P.op_vals)).to(self.device)
        self.vals64 = vals64
        self._ops = {F64: vals64}
        self._ws = {}
        self.psi_dim = int(self.tl.psi_dim)
        self.ntasks = int(self.tl.ntasks)
        self.total_flops = int(self.tl.total_flops)

    # -- operands ----------------------------------------------------------
    def operands(self, prec):
        p = prec_id(prec)
        if p not in self._ops:
            n = self.vals64.numel()
            if p == F32:
                out = torch.empty(n, dtype=torch.float32, device=self.device)
            else:
                out = torch.empty(2 * ((n + 7) // 8 * 8), dtype=torch.int16, device=self.device)
            _check(library().tns_prepare_operands(p, _ptr(self.vals64), n, _ptr(out), _stream()),
                   "tns_prepare_operands")
            self._ops[p] = out
        return self._ops[p]

    def workspace(self, kind, prec):
        key = (kind, prec)
        L = library()
        if key not in self._ws:
            if kind == "apply":
                n = L.tns_apply_workspace_bytes(ctypes.byref(self.tl), prec)
            else:
                n = L.tns_backward_workspace_bytes(ctypes.byref(self.tl), prec)
            self._ws[key] = torch.empty(int(max(n, 256)), dtype=torch.uint8, device=self.device)
        return self._ws[key]

    # -- H_eff psi ------------------------------------------------------------
    def _vec(self, x, dt, what):
        if x.dtype != dt or x.device != self.device or x.numel() != self.psi_dim or not x.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of %d elements on %s"
                             % (what, dt, self.psi_dim, self.device))

    def _ops_arg(self, p, ops):
        if ops is None:
            return self.operands(p)
        dt = torch.float64 if p == F64 else torch.float32
        if p == BF16X3 or ops.dtype != dt or not ops.is_contiguous() or ops.numel() != self.vals64.numel() \
                or ops.device != self.device:
            raise ValueError("explicit operator values must be a contiguous %s tensor of %d elements"
                             % (dt, self.vals64.numel()))
        return ops

    def apply(self, psi, prec="f64", out=None, beta=0.0, ops=None):
        """sigma := beta sigma + H_eff psi in precision ``prec`` (``ops``:
        optional operator values in the precision's dtype, op-value layout)."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        self._vec(psi, dt, "psi")
        if out is None:
            out = torch.empty(self.psi_dim, dtype=dt, device=self.device)
            beta = 0.0
        else:
            self._vec(out, dt, "out")
        ws = self.workspace("apply", p)
        _check(library().tns_apply_heff(ctypes.byref(self.tl), p, _ptr(self._ops_arg(p, ops)), _ptr(psi), _ptr(out),
                                        float(beta), _ptr(ws), ws.numel(), _stream()), "tns_apply_heff")
        return out

    def apply_noalloc(self, psi, out, prec="f64", beta=0.0):
        """``apply`` through ``tns_apply_heff_noalloc``: the library's fixed
        device scratch instead of a workspace tensor (``out`` given by the
        caller; nothing is allocated)."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        self._vec(psi, dt, "psi")
        self._vec(out, dt, "out")
        _check(library().tns_apply_heff_noalloc(ctypes.byref(self.tl), p, _ptr(self.operands(p)), _ptr(psi),
                                                _ptr(out), float(beta), _stream()), "tns_apply_heff_noalloc")
        return out

    # -- tile table (per sector-size bucket) ----------------------------------
    @property
    def tiles(self):
        return int(library().tns_get_tiles(ctypes.byref(self.tl)))

    def set_tiles(self, tiles):
        _check(library().tns_set_tiles(ctypes.byref(self.tl), int(tiles), _stream()), "tns_set_tiles")

    def autotune(self, psi, prec="f32"):
        """Library autotuner of the tile table on products of ``psi``; returns the table."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        self._vec(psi, dt, "psi")
        out = torch.empty_like(psi)
        ws = self.workspace("apply", p)
        best = ctypes.c_uint32(0)
        _check(library().tns_autotune_tiles(ctypes.byref(self.tl), p, _ptr(self.operands(p)), _ptr(psi), _ptr(out),
                                            _ptr(ws), ws.numel(), ctypes.byref(best), _stream()),
               "tns_autotune_tiles")
        return int(best.value)

    def backward(self, psi, grad_sigma, prec="f64", want_psi=True, want_ops=True, ops=None):
        """(grad_psi, grad_ops) of a loss with d loss / d sigma = grad_sigma."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        self._vec(psi, dt, "psi")
        self._vec(grad_sigma, dt, "grad_sigma")
        gp = torch.empty(self.psi_dim, dtype=dt, device=self.device) if want_psi else None
        go = torch.empty(self.vals64.numel(), dtype=dt, device=self.device) if want_ops else None
        ws = self.workspace("backward", p)
        _check(library().tns_apply_heff_backward(
            ctypes.byref(self.tl), p, _ptr(self._ops_arg(p, ops)), _ptr(psi), _ptr(grad_sigma),
            _ptr(gp) if gp is not None else None, _ptr(go) if go is not None else None,
            _ptr(ws), ws.numel(), _stream()), "tns_apply_heff_backward")
        return gp, go

    def davidson(self, psi0, inner="f64", tol_res=1e-6, tol_e=1e-10, max_sub=32, keep=8, max_iter=500,
                 refine=8):
        """Lowest eigenpair by the library's device Davidson.  Returns
        ``(energy, psi, info)``; ``psi0`` (FP64) is not modified."""
        L = library()
        o = TnsDavidsonOpts(max_sub=max_sub, keep=keep, max_iter=max_iter, refine=refine,
                            tol_res=tol_res, tol_e=tol_e, inner=prec_id(inner))
        n = L.tns_davidson_workspace_bytes(ctypes.byref(self.tl), ctypes.byref(o))
        if n == 0:
            raise ValueError("invalid Davidson options")
        ws = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        x = psi0.detach().to(self.device, torch.float64).contiguous().clone()
        e = ctypes.c_double(0.0)
        info = TnsDavidsonInfo()
        code = L.tns_davidson(ctypes.byref(self.tl), ctypes.byref(o), _ptr(self.operands(o.inner)),
                              _ptr(self.vals64), _ptr(x), ctypes.byref(e), ctypes.byref(info), _ptr(ws), int(n),
                              _stream())
        if code not in (0, -7):
            raise TnsError(code, "tns_davidson")
        return e.value, x, dict(iters=info.iters, matvecs_lo=info.matvecs_lo, matvecs_f64=info.matvecs_f64,
                                res_norm=info.res_norm, e_lo=info.e_lo, converged=code == 0)

    # -- inspection -------------------------------------------------------------
    def tasks(self):
        """Copy of the device task table (numpy, 40-byte records) and CSR pointer."""
        n = self.ntasks
        buf = torch.empty(n * TASK_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        ptr = torch.empty(self.P.nS + 1, dtype=torch.int32, device=self.device)
        if n:
            _memcpy_d2d(buf, self.tl.tasks, n * TASK_DTYPE.itemsize)
        _memcpy_d2d(ptr, self.tl.out_ptr, (self.P.nS + 1) * 4)
        torch.cuda.synchronize(self.device)
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=TASK_DTYPE), ptr.cpu().numpy()


def save_davidson_checkpoint(path, energy, psi, info):
    """Write a Davidson state (energy, FP64 vector, counters) to ``path``
    (numpy ``.npz``; no pickled objects) so that a later solve can resume
    from the vector."""
    np.savez(path, energy=np.float64(energy), psi=psi.detach().double().cpu().numpy(),
             **{k: np.asarray(v) for k, v in info.items()})


def load_davidson_checkpoint(path):
    """``(energy, psi (CPU FP64 tensor), info)`` written by
    :func:`save_davidson_checkpoint`."""
    with np.load(path, allow_pickle=False) as f:
        info = {k: f[k].item() for k in f.files if k not in ("energy", "psi")}
        return float(f["energy"]), torch.from_numpy(f["psi"].copy()), info


def _memcpy_d2d(dst, src_ptr, nbytes):
    hip = _hip()
    r = hip.hipMemcpyAsync(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), ctypes.c_size_t(nbytes),
                           ctypes.c_int(3), _stream())
    if r != 0:
        raise RuntimeError("hipMemcpyAsync failed (%d)" % r)


_hiprt = None


def _hip():
    global _hiprt
    if _hiprt is None:
        _hiprt = ctypes.CDLL("libamdhip64.so")
        _hiprt.hipMemcpyAsync.restype = ctypes.c_int
        _hiprt.hipMemcpyAsync.argtypes = [_P, _P, ctypes.c_size_t, ctypes.c_int, _P]
        _hiprt.hipEventCreate.restype = ctypes.c_int
        _hiprt.hipEventCreate.argtypes = [ctypes.POINTER(_P)]
        _hiprt.hipEventDestroy.restype = ctypes.c_int
        _hiprt.hipEventDestroy.argtypes = [_P]
        _hiprt.hipEventSynchronize.restype = ctypes.c_int
        _hiprt.hipEventSynchronize.argtypes = [_P]
        _hiprt.hipEventElapsedTime.restype = ctypes.c_int
        _hiprt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), _P, _P]
    return _hiprt


class HeffBatch:
    """Many products in one launch per GEMM phase (``tns_apply_heff_batch``).

    ``problems``: HeffProblem instances on one device.  ``apply(psis, prec,
    outs)`` computes outs[i] = H_eff,i psis[i] for every instance."""

    def __init__(self, problems):
        if not problems:
            raise ValueError("empty batch")
        self.problems = list(problems)
        self.device = self.problems[0].device
        n = len(self.problems)
        self._tls = (ctypes.POINTER(TnsTasklist) * n)(*[ctypes.pointer(h.tl) for h in self.problems])
        self._ws = {}

    def workspace(self, prec):
        p = prec_id(prec)
        if p not in self._ws:
            nb = library().tns_apply_batch_workspace_bytes(self._tls, len(self.problems), p)
            if nb == 0:
                raise ValueError("invalid batch")
            self._ws[p] = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        return self._ws[p]

    def autotune(self, psis, prec="f32"):
        """Library autotuner of one tile table for all instances; returns it."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        n = len(self.problems)
        outs = [torch.empty(h.psi_dim, dtype=dt, device=self.device) for h in self.problems]
        for h, x in zip(self.problems, psis):
            h._vec(x, dt, "psi")
        ops = (_P * n)(*[_ptr(h.operands(p)) for h in self.problems])
        xs = (_P * n)(*[_ptr(x) for x in psis])
        ys = (_P * n)(*[_ptr(o) for o in outs])
        ws = self.workspace(p)
        best = ctypes.c_uint32(0)
        _check(library().tns_autotune_tiles_batch(self._tls, n, p, ops, xs, ys, _ptr(ws), ws.numel(),
                                                  ctypes.byref(best), _stream()), "tns_autotune_tiles_batch")
        return int(best.value)

    def apply(self, psis, prec="f32", outs=None, beta=0.0):
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        n = len(self.problems)
        if len(psis) != n:
            raise ValueError("one psi per instance")
        if outs is None:
            outs = [torch.empty(h.psi_dim, dtype=dt, device=self.device) for h in self.problems]
            beta = 0.0
        for h, x, o in zip(self.problems, psis, outs):
            h._vec(x, dt, "psi")
            h._vec(o, dt, "out")
        ops = (_P * n)(*[_ptr(h.operands(p)) for h in self.problems])
        xs = (_P * n)(*[_ptr(x) for x in psis])
        ys = (_P * n)(*[_ptr(o) for o in outs])
        ws = self.workspace(p)
        _check(library().tns_apply_heff_batch(self._tls, n, p, ops, xs, ys, float(beta), _ptr(ws), ws.numel(),
                                              _stream()), "tns_apply_heff_batch")
        return outs


class KernelTimer:
    """HIP events around the two MFMA phases of successive forward products
    (library profiling hook); ``arm()`` before each product.  ``times_ms``
    returns (phase A ms, phase B ms) per armed product."""

    def __init__(self, n):
        hip = _hip()
        self.ev = []
        for _ in range(n):
            e = [_P(), _P(), _P()]
            for x in e:
                if hip.hipEventCreate(ctypes.byref(x)):
                    raise RuntimeError("hipEventCreate failed")
            self.ev.append(e)
        self.i = 0

    def arm(self):
        a, m, b = self.ev[self.i]
        library().tns_profile_events(a, m, b)
        self.i += 1

    def times_ms(self):
        hip = _hip()
        out = []
        for a, m, b in self.ev[:self.i]:
            hip.hipEventSynchronize(b)
            t1, t2 = ctypes.c_float(0.0), ctypes.c_float(0.0)
            hip.hipEventElapsedTime(ctypes.byref(t1), a, m)
            hip.hipEventElapsedTime(ctypes.byref(t2), m, b)
            out.append((t1.value, t2.value))
        return out

    def close(self):
        hip = _hip()
        for e in self.ev:
            for x in e:
                hip.hipEventDestroy(x)
        self.ev = []


class HeffFunction(torch.autograd.Function):
    """sigma = H_eff(vals) psi with the library's hand-written backward.

    ``vals`` are the operator values in the op-value layout (FP64 or FP32,
    matching ``prec``); gradients flow to ``psi`` and ``vals``."""

    @staticmethod
    def forward(ctx, psi, vals, problem, prec):
        ctx.problem, ctx.prec = problem, prec
        ctx.save_for_backward(psi, vals)
        return problem.apply(psi.contiguous(), prec, ops=vals.contiguous())

    @staticmethod
    def backward(ctx, grad_sigma):
        psi, vals = ctx.saved_tensors
        gp, go = ctx.problem.backward(psi.contiguous(), grad_sigma.contiguous(), ctx.prec,
                                      want_psi=ctx.needs_input_grad[0], want_ops=ctx.needs_input_grad[1],
                                      ops=vals.contiguous())
        return gp, go, None, None


def heff(psi, vals, problem, prec="f64"):
    return HeffFunction.apply(psi, vals, problem, prec)


def mfma_peak(prec, iters=20000):
    """Measured MFMA throughput (TFLOP/s of MFMA instructions) of the current
    device for the instruction the precision's product uses
    (``tns_mfma_peak``)."""
    L = library()
    n = L.tns_mfma_peak_workspace_bytes()
    if n == 0:
        raise TnsError(-5, "tns_mfma_peak_workspace_bytes")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    out = ctypes.c_double(0.0)
    _check(L.tns_mfma_peak(prec_id(prec), int(iters), _ptr(ws), n, ctypes.byref(out), _stream()), "tns_mfma_peak")
    return out.value


def renorm_problem_struct(R):
    """``(tns_renorm_problem, host arrays)`` of a renormalisation input; the
    arrays back the struct's pointers and must outlive its use."""
    host = {}
    cp = TnsRenormProblem()
    for name, dt in RenormStep._INT:
        a = np.ascontiguousarray(getattr(R, name), dtype=dt)
        host[name] = a
        setattr(cp, name, a.ctypes.data_as(ctypes.c_void_p) if a.size else None)
    cp.nL, cp.nOps, cp.nBlk = len(R.dimL), len(R.op_dN), len(R.blk_op)
    cp.n_vals, cp.nQ, cp.n_u = len(R.op_vals), len(R.keep), len(R.u_vals)
    cp.nNew, cp.nTerms = int(R.n_new), len(R.term_new)
    return cp, host


def renorm_workspace_bytes(R):
    """Build-workspace bytes of a renormalisation step, 0 when it fails the
    library's host validation (no device call beyond unit-count queries)."""
    cp, host = renorm_problem_struct(R)
    return int(library().tns_renorm_workspace_bytes(ctypes.byref(cp)))


class RenormStep:
    """One renormalisation (blocking) step resident on the GPU
    (``tns_renorm_build`` / ``tns_renormalize``): ``R`` holds the block's
    sectors and operators, the enlarged block's sectors, kept dimensions and
    isometry offsets, and the terms of the new operators (see
    :mod:`synth.renorm` for the array names)."""

    _INT = (("qL", np.int32), ("dimL", np.int32), ("op_dN", np.int32), ("op_d2Sz", np.int32), ("blk_op", np.int32),
            ("blk_in", np.int32), ("blk_out", np.int32), ("blk_rows", np.int32), ("blk_cols", np.int32),
            ("blk_ld", np.int32), ("blk_off", np.int64), ("qQ", np.int32), ("keep", np.int32), ("u_off", np.int64),
            ("term_new", np.int32), ("term_op", np.int32), ("term_mono", np.int32), ("term_coef", np.float64))

    def __init__(self, R, device="cuda"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        L = library()
        cp, self._host = renorm_problem_struct(R)
        self.cprob = cp
        nb = L.tns_renorm_workspace_bytes(ctypes.byref(cp))
        if nb == 0:
            raise ValueError("renormalisation problem failed host validation")
        self.ws_build = torch.empty(int(nb), dtype=torch.uint8, device=dev)
        self.plan = TnsRenormPlan()
        with torch.cuda.device(dev):
            _check(L.tns_renorm_build(ctypes.byref(cp), _ptr(self.ws_build), int(nb), ctypes.byref(self.plan),
                                      _stream()), "tns_renorm_build")
        self.ntasks = int(self.plan.ntasks)
        self.n_out_blk = int(self.plan.n_out_blk)
        self.out_elems = int(self.plan.out_elems)
        self.total_flops = int(self.plan.total_flops)
        self._ws = {}

    def out_table(self):
        """``dict`` of numpy arrays ``new, q_in, q_out, rows, cols, ld, off``
        (one entry per output block)."""
        n = self.n_out_blk
        t = {k: np.zeros(n, dtype=np.int32) for k in ("new", "q_in", "q_out", "rows", "cols", "ld")}
        t["off"] = np.zeros(n, dtype=np.int64)
        if n:
            args = [t[k].ctypes.data_as(ctypes.c_void_p) for k in ("new", "q_in", "q_out", "rows", "cols", "ld", "off")]
            _check(library().tns_renorm_out_table(ctypes.byref(self.plan), *args), "tns_renorm_out_table")
        return t

    def apply(self, op_vals, u_vals, prec="f64", out=None):
        """Renormalised blocks (tensor of ``out_elems``, layout of
        :meth:`out_table`) from FP64 device tensors of operator values and
        isometries; products in ``prec``."""
        p = prec_id(prec)
        dt = torch.float64 if p == F64 else torch.float32
        for x, what in ((op_vals, "op_vals"), (u_vals, "u_vals")):
            if x.dtype != torch.float64 or x.device != self.device or not x.is_contiguous():
                raise ValueError("%s must be a contiguous float64 tensor on %s" % (what, self.device))
        if out is None:
            out = torch.empty(max(self.out_elems, 1), dtype=dt, device=self.device)
        L = library()
        if p not in self._ws:
            n = L.tns_renorm_apply_workspace_bytes(ctypes.byref(self.plan), p)
            self._ws[p] = torch.empty(int(max(n, 256)), dtype=torch.uint8, device=self.device)
        ws = self._ws[p]
        _check(L.tns_renormalize(ctypes.byref(self.plan), p, _ptr(op_vals), _ptr(u_vals), _ptr(out), _ptr(ws),
                                 ws.numel(), _stream()), "tns_renormalize")
        return out


TT_MODES = {"auto": 0, "single": 1, "double": 2}


def ttcache_sizes(P, cache_elems, buffering="auto"):
    """``(host_bytes, device_bytes, n_epochs)`` of a tree-traversal cache plan
    (host only; buffering "auto", "single" or "double"); raises
    :class:`TnsError` when two operators of one term do not fit the cache
    together or the problem fails validation."""
    cp, host = problem_struct(P)
    hb, db, ne = ctypes.c_size_t(0), ctypes.c_size_t(0), _i64(0)
    _check(library().tns_ttcache_sizes(ctypes.byref(cp), int(cache_elems), TT_MODES[buffering], ctypes.byref(hb),
                                       ctypes.byref(db), ctypes.byref(ne)), "tns_ttcache_sizes")
    return int(hb.value), int(db.value), int(ne.value)


class StreamedHeff:
    """H_eff psi with the operator values in pinned host memory, streamed
    through a device cache of ``cache_elems`` elements by the tree-traversal
    stack (``tns_ttcache_build`` / ``tns_apply_heff_streamed``); FP64 or FP32.
    psi and sigma stay on the device.  buffering: "auto", "single" or
    "double" (epochs alternating between the cache's halves, each epoch's
    copies overlapping the previous epoch's product)."""

    def __init__(self, P, cache_elems, prec="f64", device="cuda", host_vals=None, buffering="auto"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.prec = prec_id(prec)
        if self.prec not in (F64, F32):
            raise ValueError("streamed products run in f64 or f32")
        dt = torch.float64 if self.prec == F64 else torch.float32
        L = library()
        cp, self._host = problem_struct(P)
        self.cprob = cp
        hb, db, _ = ttcache_sizes(P, cache_elems, buffering)
        self._hbuf = (ctypes.c_uint8 * max(hb, 64))()
        self.ws_build = torch.empty(max(db, 256), dtype=torch.uint8, device=dev)
        self.plan = TnsTtcachePlan()
        with torch.cuda.device(dev):
            _check(L.tns_ttcache_build(ctypes.byref(cp), int(cache_elems), TT_MODES[buffering],
                                       ctypes.cast(self._hbuf, _P), hb,
                                       _ptr(self.ws_build), self.ws_build.numel(), ctypes.byref(self.plan),
                                       _stream()), "tns_ttcache_build")
        if host_vals is None:
            host_vals = torch.from_numpy(np.ascontiguousarray(P.op_vals)).to(dt).pin_memory()
        if host_vals.dtype != dt or host_vals.device.type != "cpu" or not host_vals.is_contiguous():
            raise ValueError("host values must be a contiguous CPU %s tensor" % dt)
        self.host_vals = host_vals
        self.cache = torch.empty(max(int(cache_elems), 8), dtype=dt, device=dev)
        n = L.tns_ttcache_apply_workspace_bytes(ctypes.byref(self.plan), self.prec)
        self.ws = torch.empty(int(max(n, 256)), dtype=torch.uint8, device=dev)
        self.psi_dim = int(P.psi_off[-1])
        self.dtype = dt
        for k in ("n_epochs", "n_loads", "loaded_elems", "naive_elems", "ntasks", "total_flops", "cache_elems",
                  "halves"):
            setattr(self, k, int(getattr(self.plan, k)))

    def apply(self, psi, out=None):
        """sigma := H_eff psi (one copy per cache load, one product per epoch;
        double-buffered plans overlap an epoch's copies with the previous
        epoch's product)."""
        if psi.dtype != self.dtype or psi.device != self.device or psi.numel() != self.psi_dim \
                or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous %s tensor of %d elements on %s"
                             % (self.dtype, self.psi_dim, self.device))
        if out is None:
            out = torch.empty(self.psi_dim, dtype=self.dtype, device=self.device)
        _check(library().tns_apply_heff_streamed(ctypes.byref(self.plan), self.prec, _ptr(self.host_vals),
                                                 _ptr(self.cache), _ptr(psi), _ptr(out), _ptr(self.ws),
                                                 self.ws.numel(), _stream()), "tns_apply_heff_streamed")
        return out


_SU2_TABLES = (("qL", np.int32), ("dimL", np.int32), ("qR", np.int32), ("dimR", np.int32), ("op_side", np.int32),
               ("op_2k", np.int32), ("op_dN", np.int32), ("blk_op", np.int32), ("blk_in", np.int32),
               ("blk_out", np.int32), ("blk_rows", np.int32), ("blk_cols", np.int32), ("blk_ld", np.int32),
               ("blk_off", np.int64), ("term_L", np.int32), ("term_R", np.int32), ("term_coef", np.float64))


def su2_problem_struct(I):
    """``(tns_su2_problem, host arrays)`` of a spin-adapted instance; the
    arrays back the struct's pointers and must outlive its use."""
    host = {}
    cp = TnsSu2Problem()
    cp.nL, cp.nR, cp.nOps = len(I.dimL), len(I.dimR), len(I.op_side)
    cp.nBlk, cp.nTerms = len(I.blk_op), len(I.term_L)
    cp.target_N, cp.target_2S = int(I.target[0]), int(I.target[1])
    cp.n_vals = len(I.op_vals)
    for name, dt in _SU2_TABLES:
        a = np.ascontiguousarray(getattr(I, name), dtype=dt)
        host[name] = a
        setattr(cp, name, a.ctypes.data_as(ctypes.c_void_p) if a.size else None)
    return cp, host


def su2_workspace_bytes(I):
    """Build-workspace bytes of a spin-adapted problem, 0 when it fails the
    library's host validation."""
    cp, host = su2_problem_struct(I)
    return int(library().tns_su2_workspace_bytes(ctypes.byref(cp)))


def su2_tables(I):
    """Host-only tables of the library: ``(sec_L, sec_R, psi_off, tasks,
    task_ptr)`` (tasks as :data:`TASK_DTYPE`)."""
    L = library()
    cp, host = su2_problem_struct(I)
    ns, nt = _i64(0), _i64(0)
    _check(L.tns_su2_tables(ctypes.byref(cp), None, None, None, 0, None, None, 0, ctypes.byref(ns),
                            ctypes.byref(nt)), "tns_su2_tables")
    n, m = int(ns.value), int(nt.value)
    sl, sr = np.zeros(n, np.int32), np.zeros(n, np.int32)
    off, ptr = np.zeros(n + 1, np.int64), np.zeros(n + 1, np.int32)
    tasks = np.zeros(max(m, 1), dtype=TASK_DTYPE)
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(L.tns_su2_tables(ctypes.byref(cp), c(sl), c(sr), c(off), n, c(tasks), c(ptr), m, ctypes.byref(ns),
                            ctypes.byref(nt)), "tns_su2_tables")
    return sl, sr, off, tasks[:m], ptr


class Su2Heff(HeffProblem):
    """A spin-adapted problem resident on the GPU (``tns_su2_build``): the
    plan's task list carries the recoupling scalars, so products, operand
    copies and Davidson are :class:`HeffProblem`'s."""

    def __init__(self, I, device="cuda"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.P = I
        L = library()
        cp, self._host = su2_problem_struct(I)
        self.cprob = cp
        nbytes = L.tns_su2_workspace_bytes(ctypes.byref(cp))
        if nbytes == 0:
            raise ValueError("spin-adapted problem failed host validation")
        self.ws_build = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        self.plan = TnsSu2Plan()
        with torch.cuda.device(dev):
            _check(L.tns_su2_build(ctypes.byref(cp), _ptr(self.ws_build), int(nbytes), ctypes.byref(self.plan),
                                   _stream()), "tns_su2_build")
        self.tl = self.plan.tl
        self.vals64 = torch.from_numpy(np.ascontiguousarray(I.op_vals)).to(dev)
        self._ops = {F64: self.vals64}
        self._ws = {}
        self.psi_dim = int(self.plan.psi_dim)
        self.ntasks = int(self.plan.ntasks)
        self.total_flops = int(self.plan.total_flops)
        self.n_sectors = int(self.plan.n_sectors)

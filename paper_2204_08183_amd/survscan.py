"""Thin ctypes binding of ``libsurvscan.so`` (declared in include/survscan.h).

Argument marshalling only: every step runs in the HIP library.  torch
supplies device memory and the current stream.  If the library has not been
built the import of this module succeeds but every call raises
``SurvScanError`` -- there is no CPU fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsurvscan.so")

SS_OK = 0
SS_EINVAL = -1
SS_EWORKSPACE = -2
SS_EUNSUPPORTED = -3
SS_EDEVICE = -4

COX = 0
FINE_GRAY = 1
PENALTY_NONE = 0
PENALTY_L1 = 1
PENALTY_L2 = 2
CHUNK = 1024

MODELS = {"cox": COX, "fg": FINE_GRAY, "fine_gray": FINE_GRAY}
PENALTIES = {"none": PENALTY_NONE, "l1": PENALTY_L1, "l2": PENALTY_L2}
ACC_F32 = 0
ACC_F32_COMP = 1
ACC_F64 = 2
ACC_F32_C64 = 3
ACCUMULATIONS = {"f32": ACC_F32, "f32c": ACC_F32_COMP, "f64": ACC_F64, "f32x64": ACC_F32_C64}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_sz = ctypes.c_size_t

# name -> (restype, argtypes); the same names as the C declarations
SIGNATURES = {
    "ss_status_string": (ctypes.c_char_p, [_i32]),
    "ss_chunk_count": (_i64, [_i64]),
    "ss_prepare_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "ss_prepare": (_i32, [_i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                          _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_workspace_bytes": (_sz, [_i32, _i64]),
    "ss_workspace_init": (_i32, [_vp, _sz, _vp]),
    "ss_workspace_error": (_i32, [_vp, ctypes.POINTER(_i32), _vp]),
    "ss_grad_hess": (_i32, [_i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_loglik": (_i32, [_i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                         _sz, _vp]),
    "ss_ccd_update": (_i32, [_i32, _f64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp, _vp, _vp]),
    "ss_ccd_sweep": (_i32, [_i32, _i32, _f64, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _sz, _vp]),
    "ss_exp": (_i32, [_i64, _vp, _vp, _vp]),
    "ss_gather": (_i32, [_i64, _vp, _vp, _vp, _vp]),
    "ss_exp_f32": (_i32, [_i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_grad_hess_mixed": (_i32, [_i32, _i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_grad_hess_f32": (_i32, [_i32, _i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_tune_get": (_i32, [_i32, _i32, _i32, _i32, _i64]),
    "ss_tune_has": (_i32, [_i32, _i32, _i32, _i32, _i64]),
    "ss_tune_set": (_i32, [_i32, _i32, _i32, _i32, _i64, _i32]),
    "ss_tune_clear": (_i32, []),
    "ss_tune_save": (_i32, [ctypes.c_char_p]),
    "ss_tune_load": (_i32, [ctypes.c_char_p, ctypes.POINTER(_i32)]),
    "ss_autotune_grad_hess": (_i32, [_i32, _i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32,
                                     ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float),
                                     _vp]),
    "ss_autotune_sweep": (_i32, [_i32, _i32, _f64, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, _sz, _i32, ctypes.POINTER(_i32),
                                 ctypes.POINTER(ctypes.c_float), _vp]),
    "ss_cv_stride": (_i64, [_i64]),
    "ss_cv_prepare_workspace_bytes": (_sz, [_i64, _i32]),
    "ss_cv_prepare": (_i32, [_i32, _i64, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_cv_exp": (_i32, [_i64, _i32, _vp, _vp, _vp, _vp]),
    "ss_cv_workspace_bytes": (_sz, [_i32]),
    "ss_cv_sweep": (_i32, [_i32, _i32, _f64, _i64, _i64, _i32, _i64, _i64, _vp, _vp, _vp, _vp,
                           _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_cv_loglik": (_i32, [_i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp, _vp, _vp, _vp, _vp]),
    "ss_objective": (_i32, [_i32, _i32, _f64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp, _vp, _sz, _vp]),
    "ss_cv_select": (_i32, [_i32, _i32, _vp, _vp, _vp, _vp]),
    "ss_gather_u8": (_i32, [_i64, _vp, _vp, _vp, _vp]),
    "ss_beta_gradient_workspace_bytes": (_sz, [_i64, _i64]),
    "ss_beta_gradient": (_i32, [_i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ss_noalloc_scratch_bytes": (_sz, []),
    "ss_grad_hess_noalloc": (_i32, [_i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp, _vp, _vp, _vp, _vp, _vp]),
    "ss_eta_gradient_workspace_bytes": (_sz, [_i64]),
    "ss_eta_gradient": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, _sz, _vp]),
}


TUNE_GRAD_HESS = 0
TUNE_SWEEP = 1
STORAGE_F64 = 0
STORAGE_F32 = 1
STORAGE_F32_SUMS32 = 2
STORAGES = {"f64": STORAGE_F64, "f32": STORAGE_F32, "f32x64": STORAGE_F32_SUMS32}
GRAD_HESS_IPTS = (4, 8, 16, 32)
SWEEP_SHAPES = (25616, 51208, 25608, 51216)


class SurvScanError(RuntimeError):
    pass


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SurvScanError(
                "libsurvscan.so is not built (python -m paper_2204_08183_amd.build); "
                "there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def status_string(code):
    return load().ss_status_string(code).decode()


def check(code, what):
    if code != SS_OK:
        raise SurvScanError("%s failed: %s (%d)" % (what, status_string(code), code))


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def chunk_count(n):
    return int(load().ss_chunk_count(n))


def tune_get(kind, model, storage, valued, n):
    """The launch shape in effect for a key (see ss_tune_get)."""
    r = load().ss_tune_get(kind, MODELS[model], STORAGES[storage], int(bool(valued)), n)
    if r < 0:
        check(r, "ss_tune_get")
    return r


def tune_has(kind, model, storage, valued, n):
    r = load().ss_tune_has(kind, MODELS[model], STORAGES[storage], int(bool(valued)), n)
    if r < 0:
        check(r, "ss_tune_has")
    return bool(r)


def tune_set(kind, model, storage, valued, n, choice):
    check(load().ss_tune_set(kind, MODELS[model], STORAGES[storage], int(bool(valued)), n,
                             int(choice)), "ss_tune_set")


def tune_clear():
    check(load().ss_tune_clear(), "ss_tune_clear")


def tune_save(path):
    check(load().ss_tune_save(os.fsencode(path)), "ss_tune_save")


def tune_load(path):
    """Adds the entries of a saved table measured on this GPU architecture;
    returns how many were taken."""
    count = ctypes.c_int32(0)
    check(load().ss_tune_load(os.fsencode(path), ctypes.byref(count)), "ss_tune_load")
    return int(count.value)


class Workspace:
    """A 256-byte aligned device scratch buffer owned by torch."""

    def __init__(self, nbytes, device):
        self.nbytes = int(nbytes)
        self._buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        addr = self._buf.data_ptr()
        self.offset = (-addr) % 256
        self.ptr = ctypes.c_void_p(addr + self.offset)


class Problem:
    """One prepared data set on the GPU (sorted order, chunk index, KM)."""

    def __init__(self, model, y, status, col_ptr, rows, vals=None, device="cuda"):
        lib = load()
        self.model_name = model
        self.model = MODELS[model]
        self.device = torch.device(device)
        dev = self.device
        y = torch.as_tensor(y, dtype=torch.float64).to(dev).contiguous()
        status = torch.as_tensor(status, dtype=torch.int8).to(dev).contiguous()
        col_ptr = torch.as_tensor(col_ptr, dtype=torch.int64).to(dev).contiguous()
        rows = torch.as_tensor(rows, dtype=torch.int32).to(dev).contiguous()
        self.n = n = int(y.numel())
        self.p = p = int(col_ptr.numel() - 1)
        self.nnz = nnz = int(rows.numel())
        self.vals_in = None if vals is None else \
            torch.as_tensor(vals, dtype=torch.float64).to(dev).contiguous()
        self.col_ptr = col_ptr
        self.status = status
        self.y = y
        self.perm = torch.empty(n, dtype=torch.int32, device=dev)
        self.inv_perm = torch.empty(n, dtype=torch.int32, device=dev)
        self.d8 = torch.empty(n, dtype=torch.uint8, device=dev)
        self.d32 = torch.empty(n, dtype=torch.int32, device=dev)
        self.c = torch.empty(p, dtype=torch.float64, device=dev)
        self.rows_sorted = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        self.vals_sorted = None if vals is None else \
            torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
        self.nchunk = chunk_count(n)
        self.chunk_ptr = torch.empty(p * (self.nchunk + 1), dtype=torch.int32, device=dev)
        fg = self.model == FINE_GRAY
        self.w_comp = torch.empty(n, dtype=torch.float64, device=dev) if fg else None
        self.g_end = torch.empty(n, dtype=torch.float64, device=dev) if fg else None
        pws = Workspace(lib.ss_prepare_workspace_bytes(n, p, nnz), dev)
        rc = lib.ss_prepare(self.model, n, p, nnz, _p(y), _p(status), _p(col_ptr), _p(rows),
                            _p(self.vals_in), _p(self.perm), _p(self.inv_perm), _p(self.d8),
                            _p(self.d32), _p(self.c), _p(self.rows_sorted),
                            _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.w_comp),
                            _p(self.g_end), pws.ptr, pws.nbytes, _stream(dev))
        check(rc, "ss_prepare")
        del pws
        self.ws = Workspace(lib.ss_workspace_bytes(self.model, n), dev)
        check(lib.ss_workspace_init(self.ws.ptr, self.ws.nbytes, _stream(dev)),
              "ss_workspace_init")
        self.eta = torch.zeros(n, dtype=torch.float64, device=dev)
        self.e = torch.ones(n, dtype=torch.float64, device=dev)
        self.beta = torch.zeros(p, dtype=torch.float64, device=dev)
        self.delta = torch.ones(p, dtype=torch.float64, device=dev)
        self.steps = torch.zeros(p, dtype=torch.float64, device=dev)
        self.out = torch.zeros(3, dtype=torch.float64, device=dev)

    # ---------------------------------------------------------------- state
    def set_eta(self, eta_subject_order):
        """Sets X beta from a per-subject vector (original order)."""
        src = torch.as_tensor(eta_subject_order, dtype=torch.float64).to(self.device)
        src = src.contiguous()
        lib = load()
        s = _stream(self.device)
        check(lib.ss_gather(self.n, _p(self.perm), _p(src), _p(self.eta), s), "ss_gather")
        check(lib.ss_exp(self.n, _p(self.eta), _p(self.e), s), "ss_exp")

    def set_beta(self, beta, eta_subject_order):
        self.beta.copy_(torch.as_tensor(beta, dtype=torch.float64))
        self.set_eta(eta_subject_order)

    def reset_trust(self):
        self.delta.fill_(1.0)

    # ---------------------------------------------------------------- calls
    def grad_hess(self, j, out=None):
        """(g', g'', sum d log S0) of coordinate j as a device tensor [3]."""
        out = self.out if out is None else out
        rc = load().ss_grad_hess(self.model, self.n, self.p, int(j), _p(self.e), _p(self.d8),
                                 _p(self.d32), _p(self.w_comp), _p(self.g_end),
                                 _p(self.col_ptr), _p(self.rows_sorted),
                                 _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.c),
                                 _p(out), self.ws.ptr, self.ws.nbytes, _stream(self.device))
        check(rc, "ss_grad_hess")
        return out

    def make_e32(self):
        """FP32 copy of e, shifted: (e32 = exp(eta - m) as float, m) as device tensors."""
        e32 = torch.empty(self.n, dtype=torch.float32, device=self.device)
        shift = torch.empty(1, dtype=torch.float64, device=self.device)
        check(load().ss_exp_f32(self.n, _p(self.eta), _p(e32), _p(shift), self.ws.ptr,
                                self.ws.nbytes, _stream(self.device)), "ss_exp_f32")
        return e32, shift

    def grad_hess_mixed(self, j, e32, acc, out=None):
        """(g', g'', sum d log S0 of the shifted e) of coordinate j from FP32 e,
        accumulated as `acc` ("f32", "f32c" or "f64")."""
        out = torch.empty(3, dtype=torch.float64, device=self.device) if out is None else out
        rc = load().ss_grad_hess_mixed(self.model, ACCUMULATIONS[acc], self.n, self.p, int(j),
                                       _p(e32), _p(self.d8), _p(self.d32), _p(self.w_comp),
                                       _p(self.g_end), _p(self.col_ptr), _p(self.rows_sorted),
                                       _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.c),
                                       _p(out), self.ws.ptr, self.ws.nbytes,
                                       _stream(self.device))
        check(rc, "ss_grad_hess_mixed")
        return out

    def grad_hess_f32(self, j, e32, acc="f64", out=None):
        """(g', g'', sum d log S0 of the shifted e) of coordinate j from FP32 e
        in the single-pass fused kernel, sums in FP64 ("f64") or FP32 inside
        a tile with an FP64 carry ("f32x64")."""
        out = torch.empty(3, dtype=torch.float64, device=self.device) if out is None else out
        rc = load().ss_grad_hess_f32(self.model, ACCUMULATIONS[acc], self.n, self.p, int(j),
                                     _p(e32), _p(self.d8), _p(self.d32), _p(self.w_comp),
                                     _p(self.g_end), _p(self.col_ptr), _p(self.rows_sorted),
                                     _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.c),
                                     _p(out), self.ws.ptr, self.ws.nbytes,
                                     _stream(self.device))
        check(rc, "ss_grad_hess_f32")
        return out

    def _adjoint_setup(self, ws_bytes):
        """The status in sorted order (once) and an adjoint workspace of at
        least ws_bytes."""
        lib = load()
        if getattr(self, "status_sorted", None) is None:
            self.status_sorted = torch.empty(self.n, dtype=torch.int8, device=self.device)
            check(lib.ss_gather_u8(self.n, _p(self.perm), _p(self.status),
                                   _p(self.status_sorted), _stream(self.device)),
                  "ss_gather_u8")
        if getattr(self, "adj_ws", None) is None or self.adj_ws.nbytes < ws_bytes:
            self.adj_ws = Workspace(ws_bytes, self.device)

    def eta_gradient(self, grad=None, loglik=None):
        """dl/deta for every subject (original order) and l at the current
        eta, as device tensors (grad [n], loglik [1])."""
        lib = load()
        self._adjoint_setup(lib.ss_eta_gradient_workspace_bytes(self.n))
        grad = torch.empty(self.n, dtype=torch.float64, device=self.device) \
            if grad is None else grad
        loglik = torch.empty(1, dtype=torch.float64, device=self.device) \
            if loglik is None else loglik
        rc = lib.ss_eta_gradient(self.model, self.n, _p(self.inv_perm), _p(self.status_sorted),
                                 _p(self.eta), _p(self.e), _p(self.d8), _p(self.d32),
                                 _p(self.w_comp), _p(self.g_end), _p(grad), _p(loglik),
                                 self.adj_ws.ptr, self.adj_ws.nbytes, _stream(self.device))
        check(rc, "ss_eta_gradient")
        return grad, loglik

    def beta_gradient(self, grad_beta=None, grad_eta=None, loglik=None):
        """X' (dl/deta) at the current eta as a device tensor [p] (Sec. 2.9),
        with l [1]; with a grad_eta tensor [n] also dl/deta in subject order.
        Returns (grad_beta, loglik)."""
        lib = load()
        self._adjoint_setup(lib.ss_beta_gradient_workspace_bytes(self.n, self.p))
        grad_beta = torch.empty(self.p, dtype=torch.float64, device=self.device) \
            if grad_beta is None else grad_beta
        loglik = torch.empty(1, dtype=torch.float64, device=self.device) \
            if loglik is None else loglik
        rc = lib.ss_beta_gradient(self.model, self.n, self.p, _p(self.inv_perm),
                                  _p(self.status_sorted), _p(self.eta), _p(self.e), _p(self.d8),
                                  _p(self.d32), _p(self.w_comp), _p(self.g_end),
                                  _p(self.col_ptr), _p(self.rows_sorted), _p(self.vals_sorted),
                                  _p(self.chunk_ptr), _p(grad_beta), _p(grad_eta), _p(loglik),
                                  self.adj_ws.ptr, self.adj_ws.nbytes, _stream(self.device))
        check(rc, "ss_beta_gradient")
        return grad_beta, loglik

    def loglik(self, beta=None, out=None):
        beta = self.beta if beta is None else \
            torch.as_tensor(beta, dtype=torch.float64).to(self.device).contiguous()
        out = torch.zeros(1, dtype=torch.float64, device=self.device) if out is None else out
        rc = load().ss_loglik(self.model, self.n, self.p, _p(self.e), _p(self.d8),
                              _p(self.d32), _p(self.w_comp), _p(self.g_end), _p(beta),
                              _p(self.c), _p(out), self.ws.ptr, self.ws.nbytes,
                              _stream(self.device))
        check(rc, "ss_loglik")
        return out

    def ccd_update(self, j, g12, penalty="none", lam=0.0):
        rc = load().ss_ccd_update(PENALTIES[penalty], float(lam), self.n, self.p, int(j),
                                  _p(g12), _p(self.beta), _p(self.delta),
                                  _p(self.steps[int(j):]), _p(self.eta), _p(self.e),
                                  _p(self.col_ptr), _p(self.rows_sorted),
                                  _p(self.vals_sorted), _stream(self.device))
        check(rc, "ss_ccd_update")

    def sweep(self, penalty="none", lam=0.0, j_begin=0, j_end=None, g12_out=None):
        j_end = self.p if j_end is None else j_end
        rc = load().ss_ccd_sweep(self.model, PENALTIES[penalty], float(lam), self.n, self.p,
                                 int(j_begin), int(j_end), _p(self.eta), _p(self.e),
                                 _p(self.d8), _p(self.d32), _p(self.w_comp), _p(self.g_end),
                                 _p(self.col_ptr), _p(self.rows_sorted),
                                 _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.c),
                                 _p(self.beta), _p(self.delta), _p(self.steps),
                                 _p(g12_out), self.ws.ptr, self.ws.nbytes,
                                 _stream(self.device))
        check(rc, "ss_ccd_sweep")

    def autotune(self, j=0, reps=20, e32=None, storage="f64", sweep=True, sweep_coords=64,
                 penalty="l1", lam=1.0, sweep_reps=3, cache=None):
        """Times the launch-shape candidates on this problem and stores the
        fastest in the library's table (ss_autotune_grad_hess for coordinate
        j; with `sweep`, ss_autotune_sweep over the first `sweep_coords`
        coordinates on scratch copies of the state).  With `cache` (a file
        path) entries measured earlier on this GPU architecture are loaded
        first and keys already present are not timed again; the table is
        saved there afterwards.  Returns {"grad_hess": (choice, us per
        candidate), "sweep": (choice, us per candidate) or None}."""
        lib = load()
        valued = self.vals_sorted is not None
        if cache and os.path.exists(cache):
            tune_load(cache)
        res = {"grad_hess": None, "sweep": None}
        e = self.e if storage == "f64" else e32
        if e is None:
            raise SurvScanError("autotune: FP32 storage needs e32 (make_e32)")
        if not (cache and tune_has(TUNE_GRAD_HESS, self.model_name, storage, valued, self.n)):
            choice = ctypes.c_int32(0)
            us = (ctypes.c_float * 4)()
            out = torch.empty(3, dtype=torch.float64, device=self.device)
            rc = lib.ss_autotune_grad_hess(
                self.model, STORAGES[storage], self.n, self.p, int(j), _p(e), _p(self.d8),
                _p(self.d32), _p(self.w_comp), _p(self.g_end), _p(self.col_ptr),
                _p(self.rows_sorted), _p(self.vals_sorted), _p(self.chunk_ptr), _p(self.c),
                _p(out), self.ws.ptr, self.ws.nbytes, int(reps), ctypes.byref(choice), us,
                _stream(self.device))
            check(rc, "ss_autotune_grad_hess")
            res["grad_hess"] = (int(choice.value), [float(x) for x in us])
        if sweep and storage == "f64" and not (
                cache and tune_has(TUNE_SWEEP, self.model_name, "f64", valued, self.n)):
            jb, je = 0, min(self.p, int(sweep_coords))
            eta_s = torch.empty_like(self.eta)
            e_s = torch.empty_like(self.e)
            beta_s = torch.empty_like(self.beta)
            delta_s = torch.empty_like(self.delta)
            steps_s = torch.empty_like(self.steps)
            choice = ctypes.c_int32(0)
            us = (ctypes.c_float * 4)()
            rc = lib.ss_autotune_sweep(
                self.model, PENALTIES[penalty], float(lam), self.n, self.p, jb, je,
                _p(self.eta), _p(self.e), _p(self.d8), _p(self.d32), _p(self.w_comp),
                _p(self.g_end), _p(self.col_ptr), _p(self.rows_sorted), _p(self.vals_sorted),
                _p(self.chunk_ptr), _p(self.c), _p(self.beta), _p(self.delta), _p(eta_s),
                _p(e_s), _p(beta_s), _p(delta_s), _p(steps_s), self.ws.ptr, self.ws.nbytes,
                int(sweep_reps), ctypes.byref(choice), us, _stream(self.device))
            if rc != SS_EUNSUPPORTED:  # too large for any persistent shape
                check(rc, "ss_autotune_sweep")
                res["sweep"] = (int(choice.value), [float(x) for x in us])
        if cache:
            d = os.path.dirname(cache)
            if d:
                os.makedirs(d, exist_ok=True)
            tune_save(cache)
        return res

    def workspace_error(self):
        flag = ctypes.c_int32(0)
        check(load().ss_workspace_error(self.ws.ptr, ctypes.byref(flag),
                                        _stream(self.device)), "ss_workspace_error")
        return int(flag.value)

    def objective(self, penalty="none", lam=0.0, out=None):
        """(l + pi, l, pi) at the current state (Secs. 2.3-2.4), with
        eta = X beta, as a device tensor [3] (ss_objective)."""
        out = torch.empty(3, dtype=torch.float64, device=self.device) if out is None else out
        rc = load().ss_objective(self.model, PENALTIES[penalty], float(lam), self.n, self.p,
                                 _p(self.e), _p(self.d8), _p(self.d32), _p(self.w_comp),
                                 _p(self.g_end), _p(self.beta), _p(self.c), _p(out),
                                 self.ws.ptr, self.ws.nbytes, _stream(self.device))
        check(rc, "ss_objective")
        return out

    def fit(self, penalty="none", lam=0.0, max_sweeps=100, tol=1e-10):
        """Cyclic coordinate descent to convergence (Secs. 2.3-2.4, the
        GPU-resident workflow of the Sec. 2.7 figure): whole sweeps on the
        device until the relative change of the penalised log-likelihood,
        |f - f_prev| / (|f| + 1), falls below `tol` (the stopping rule is
        not fixed by the paper).  Returns the number of sweeps taken."""
        f_prev = float(self.objective(penalty, lam)[0])
        for k in range(1, max_sweeps + 1):
            self.sweep(penalty, lam)
            f = float(self.objective(penalty, lam)[0])
            if self.workspace_error():
                raise SurvScanError("fit: a bounded wait of the sweep gave up")
            if abs(f - f_prev) / (abs(f) + 1.0) < tol:
                return k
            f_prev = f
        return max_sweeps


class CrossValidation:
    """R cross-validation replicates of a prepared Cox or Fine-Gray problem
    with a 0/1 design, fitted together in one launch per sweep.

    `train` is [R, n] (1 = training subject, original subject order).
    Per-replicate state lives in sorted order with replicate r at offset
    r * stride: eta, e (R * stride), beta, delta ([R, p])."""

    def __init__(self, prob, train):
        lib = load()
        self.prob = prob
        dev = prob.device
        train = torch.as_tensor(train, dtype=torch.uint8).to(dev).contiguous()
        if train.dim() != 2 or train.shape[1] != prob.n:
            raise ValueError("train must be [replicates, n]")
        self.reps = reps = int(train.shape[0])
        n, p = prob.n, prob.p
        self.stride = stride = int(lib.ss_cv_stride(n))
        self.train = train
        self.train_s = torch.empty(reps * stride, dtype=torch.uint8, device=dev)
        self.d8_r = torch.empty(reps * stride, dtype=torch.uint8, device=dev)
        self.d32_r = torch.empty(reps * stride, dtype=torch.int32, device=dev)
        cols = p + 1 if prob.model == FINE_GRAY else p  # Fine-Gray: competing-event bits
        self.xbits = torch.empty(cols * stride // 32, dtype=torch.int32, device=dev)
        self.c = torch.empty(reps * p, dtype=torch.float64, device=dev)
        fg = prob.model == FINE_GRAY
        self.w_r = torch.empty(reps * stride, dtype=torch.float64, device=dev) if fg else None
        self.g_r = torch.empty(reps * stride, dtype=torch.float64, device=dev) if fg else None
        self.g_h = torch.empty(reps * stride, dtype=torch.float64, device=dev) if fg else None
        ws = Workspace(lib.ss_cv_prepare_workspace_bytes(n, reps), dev)
        check(lib.ss_cv_prepare(prob.model, n, p, reps, _p(prob.perm), _p(prob.status),
                                _p(prob.y), _p(prob.d8), _p(train), _p(prob.col_ptr),
                                _p(prob.rows_sorted), _p(prob.vals_sorted), _p(self.train_s),
                                _p(self.d8_r), _p(self.d32_r), _p(self.xbits), _p(self.c),
                                _p(self.w_r), _p(self.g_r), _p(self.g_h), ws.ptr, ws.nbytes,
                                _stream(dev)), "ss_cv_prepare")
        del ws
        self.eta = torch.zeros(reps * stride, dtype=torch.float64, device=dev)
        self.e = torch.empty(reps * stride, dtype=torch.float64, device=dev)
        self.beta = torch.zeros(reps * p, dtype=torch.float64, device=dev)
        self.delta = torch.ones(reps * p, dtype=torch.float64, device=dev)
        check(lib.ss_cv_exp(n, reps, _p(self.eta), _p(self.train_s), _p(self.e),
                            _stream(dev)), "ss_cv_exp")
        self.ws = Workspace(lib.ss_cv_workspace_bytes(reps), dev)
        check(lib.ss_workspace_init(self.ws.ptr, self.ws.nbytes, _stream(dev)),
              "ss_workspace_init")

    def set_eta(self, eta_subject_order):
        """Sets every replicate's eta from [R, n] (original order)."""
        lib = load()
        src = torch.as_tensor(eta_subject_order, dtype=torch.float64).to(self.prob.device)
        src = src.contiguous()
        s = _stream(self.prob.device)
        for r in range(self.reps):
            check(lib.ss_gather(self.prob.n, _p(self.prob.perm), _p(src[r]),
                                ctypes.c_void_p(self.eta.data_ptr() + 8 * r * self.stride), s),
                  "ss_gather")
        check(lib.ss_cv_exp(self.prob.n, self.reps, _p(self.eta), _p(self.train_s),
                            _p(self.e), s), "ss_cv_exp")

    def sweep(self, penalty="none", lam=0.0, j_begin=0, j_end=None, g12_out=None):
        j_end = self.prob.p if j_end is None else j_end
        check(load().ss_cv_sweep(self.prob.model, PENALTIES[penalty], float(lam), self.prob.n,
                                 self.prob.p, self.reps, int(j_begin), int(j_end),
                                 _p(self.eta), _p(self.e), _p(self.d8_r), _p(self.d32_r),
                                 _p(self.train_s), _p(self.xbits), _p(self.c), _p(self.w_r),
                                 _p(self.g_r), _p(self.beta), _p(self.delta), _p(g12_out),
                                 self.ws.ptr, self.ws.nbytes,
                                 _stream(self.prob.device)),
              "ss_cv_sweep")

    def workspace_error(self):
        """Non-zero if a bounded wait of a two-half launch gave up."""
        flag = ctypes.c_int32(0)
        check(load().ss_workspace_error(self.ws.ptr, ctypes.byref(flag),
                                        _stream(self.prob.device)), "ss_workspace_error")
        return int(flag.value)

    def loglik(self, out=None):
        """[R, 2]: training and held-out log partial likelihood per replicate."""
        out = torch.empty(2 * self.reps, dtype=torch.float64, device=self.prob.device) \
            if out is None else out
        pr = self.prob
        check(load().ss_cv_loglik(pr.model, pr.n, self.reps, _p(pr.perm), _p(pr.status),
                                  _p(self.eta), _p(self.e), _p(self.train_s), _p(pr.d8),
                                  _p(pr.d32), _p(self.d8_r), _p(self.d32_r), _p(self.w_r),
                                  _p(self.g_r), _p(self.g_h), _p(out), _stream(pr.device)),
              "ss_cv_loglik")
        return out.view(self.reps, 2)

    def sorted_view(self, t):
        """[R, n] view of a per-replicate sorted vector (eta, e, ...)."""
        return t.view(self.reps, self.stride)[:, :self.prob.n]


def cv_path(prob, train, gammas, sweeps=5, penalty="l1"):
    """k-fold cross-validation over a path of penalty strengths (Sec. 2.8).

    Every replicate (a row of `train`, 1 = training subject) is fitted on
    the GPU for each gamma in the given order, warm-started from the fit of
    the previous one, with `sweeps` CCD sweeps per gamma (the stopping rule
    is the caller's); after each gamma the held-out log partial likelihood
    of every replicate is recorded.  Returns (scores, best): scores is a
    [len(gammas), R] float64 array of held-out log-likelihoods and best the
    gamma with the largest mean (reading: larger predictive likelihood is
    better)."""
    cvp = CrossValidation(prob, train)
    dev = prob.device
    ng = len(gammas)
    table = torch.empty(ng, 2 * cvp.reps, dtype=torch.float64, device=dev)
    for k, g in enumerate(gammas):
        for _ in range(sweeps):
            cvp.sweep(penalty, float(g))
        cvp.loglik(out=table[k])
    if cvp.workspace_error():
        raise SurvScanError("cross-validation: a bounded wait gave up")
    mean = torch.empty(ng, dtype=torch.float64, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    check(load().ss_cv_select(ng, cvp.reps, _p(table), _p(mean), _p(best), _stream(dev)),
          "ss_cv_select")
    b = int(best.cpu()[0])
    if b < 0:
        raise SurvScanError("cross-validation: every mean held-out score is NaN")
    return table[:, 1::2].cpu().numpy(), gammas[b]


class LogLikEta(torch.autograd.Function):
    """l(eta) of a prepared problem as a differentiable function of the
    per-subject linear predictor (original order, float64 on the problem's
    device).  The forward pass computes l and dl/deta in one call of
    ss_eta_gradient; the backward pass scales the stored gradient."""

    @staticmethod
    def forward(ctx, eta, prob):
        prob.set_eta(eta.detach())
        grad, loglik = prob.eta_gradient()
        ctx.save_for_backward(grad)
        return loglik[0].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None


def loglik_eta(prob, eta):
    """l(eta) with autograd support; see LogLikEta."""
    return LogLikEta.apply(eta, prob)

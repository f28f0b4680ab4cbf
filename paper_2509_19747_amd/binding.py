"""ctypes binding of ``librandrand.so`` (the C ABI in include/randrand.h).

Argument marshalling only: every step of the method runs inside the library's
HIP kernels.  PyTorch supplies device memory (CUDA/HIP tensors) and the HIP
stream (``torch.cuda.current_stream()``).

Layout: the C ABI is column-major.  An n x m matrix crosses the boundary as the
memory of a contiguous torch tensor of shape (m, n) (its transpose in row-major
terms); the helpers below do that conversion.  A symmetric dense A can be
passed as is.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librandrand.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_ENOTSPD, RR_EBREAKDOWN, RR_ENOCONV, RR_EDEVICE, RR_EBUSY = range(8)
OP_DENSE, OP_RBF, OP_MATERN32 = 0, 1, 2
SK_GAUSSIAN, SK_SRHT = 0, 1
ORTH_SKETCHED_CHOLQR, ORTH_CHOLQR = 0, 1
PREC_FP64, PREC_FP32, PREC_MIXED = 0, 1, 2
TAU_OPT, TAU_RHO, TAU_NYS = 0, 1, 2

_SKETCH = {"gaussian": SK_GAUSSIAN, "srht": SK_SRHT, "colsample": 2}
_PREC = {"fp64": PREC_FP64, "fp32": PREC_FP32, "mixed": PREC_MIXED}
_TAU = {"opt": TAU_OPT, "rho": TAU_RHO, "nys": TAU_NYS}
_ORTH = {"sketched": ORTH_SKETCHED_CHOLQR, "cholqr": ORTH_CHOLQR}
METHOD_C, METHOD_R, METHOD_SPLIT_R = 0, 1, 2
KRYLOV_CG, KRYLOV_MINRES, KRYLOV_BLOCK_MINRES, KRYLOV_BLOCK_CG = 0, 1, 2, 3
_METHOD = {"c": METHOD_C, "r": METHOD_R, "split": METHOD_SPLIT_R}
_KRYLOV = {"cg": KRYLOV_CG, "minres": KRYLOV_MINRES, "block_minres": KRYLOV_BLOCK_MINRES,
           "block_cg": KRYLOV_BLOCK_CG}
BLOCK_MAX = 32


class rr_operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("A", C.c_void_p), ("lda", C.c_int64),
                ("pts", C.c_void_p), ("d", C.c_int32), ("kconst", C.c_double),
                ("scale", C.c_double)]


class rr_build_opts(C.Structure):
    _fields_ = [("l", C.c_int64), ("sketch", C.c_int32), ("seed", C.c_uint64),
                ("orth", C.c_int32), ("prec", C.c_int32), ("tau_rule", C.c_int32),
                ("rho", C.c_double), ("power_iters", C.c_int32), ("power_q", C.c_int32),
                ("multi_shift", C.c_int32), ("l_max", C.c_int64), ("ad_factor", C.c_double),
                ("basis", C.c_int32), ("reorth", C.c_int32)]


class rr_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart_eta", C.c_double), ("maxit", C.c_int32),
                ("check_every", C.c_int32), ("fp64_ir", C.c_int32),
                ("relres_history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("use_graph", C.c_int32), ("certify", C.c_int32), ("method", C.c_int32),
                ("krylov", C.c_int32), ("block_kmax", C.c_int32)]


class rr_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("relres_work", C.c_double),
                ("relres_fp64", C.c_double), ("tau", C.c_double), ("normE", C.c_double),
                ("lamhat", C.c_double), ("orth_err", C.c_double), ("ms_build", C.c_double),
                ("ms_solve", C.c_double), ("status", C.c_int32), ("graph_fallbacks", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rr_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p),
                ("alloc", C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p))]


class rr_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("d", C.c_int32), ("pts", C.c_void_p),
                ("kconst", C.c_double), ("scale", C.c_double), ("mu", C.c_double),
                ("l", C.c_int64), ("nrhs", C.c_int32), ("B", C.c_void_p), ("X", C.c_void_p),
                ("id", C.c_uint64), ("seed", C.c_uint64), ("t_arrival", C.c_double)]


NEXT_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_double, C.POINTER(rr_request))
DELIVER_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(rr_request), C.POINTER(rr_solve_info),
                         C.c_double)


class rr_serve_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32), ("graph_iters", C.c_int32),
                ("build", rr_build_opts), ("solve", rr_solve_opts),
                ("alloc", C.POINTER(rr_allocator)), ("grouped", C.c_int32)]


class rr_serve_stats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("solves_per_s", C.c_double), ("served", C.c_int64), ("rejected", C.c_int64),
                ("hbm_peak", C.c_size_t), ("max_active", C.c_int32), ("ok", C.c_int64),
                ("failed", C.c_int64), ("graph_fallbacks", C.c_int64),
                ("group_replays", C.c_int64), ("group_mean", C.c_double), ("group_max", C.c_int32),
                ("group_busy_s", C.c_double), ("group_wait_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load the library; raise loudly if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(hipcc for gfx950); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.rr_build_opts_default.argtypes = [C.POINTER(rr_build_opts)]
        L.rr_solve_opts_default.argtypes = [C.POINTER(rr_solve_opts)]
        L.rr_build_precond.argtypes = [C.POINTER(rr_operator), C.POINTER(C.c_double), C.c_int32,
                                       C.POINTER(rr_build_opts), C.POINTER(rr_allocator), P,
                                       C.POINTER(P)]
        L.rr_solve.argtypes = [P, C.c_int32, P, P, C.POINTER(rr_solve_opts),
                               C.POINTER(rr_solve_info), P]
        L.rr_solve_batch.argtypes = [P, C.POINTER(C.c_int32), P, C.c_int64, C.c_int32, P, C.c_int64,
                                     C.POINTER(rr_solve_opts), C.POINTER(rr_solve_info), P]
        L.rr_serve.argtypes = [C.POINTER(rr_serve_config), NEXT_FN, DELIVER_FN, P,
                               C.POINTER(rr_serve_stats)]
        L.rr_precond_export.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.rr_precond_export_omega.argtypes = [P, P]
        L.rr_precond_shape.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32)]
        L.rr_kernel_to_dense.argtypes = [C.POINTER(rr_operator), P, C.c_int32, C.c_int64, P]
        L.rr_apply_operator.argtypes = [C.POINTER(rr_operator), C.c_double, C.c_int32, P, P, P]
        L.rr_apply_operator_block.argtypes = [C.POINTER(rr_operator), C.c_double, C.c_int32, P,
                                              C.c_int32, P, P]
        L.rr_random_matrix.argtypes = [C.c_int32, C.c_uint64, C.c_int64, C.c_int64, P, P]
        L.rr_theta_apply.argtypes = [C.c_uint64, C.c_int64, C.c_int64, P, P, P]
        L.rr_sketch_apply.argtypes = [C.POINTER(rr_operator), C.c_double, C.POINTER(rr_build_opts),
                                      P, P]
        L.rr_apply_operator_noalloc.argtypes = [C.POINTER(rr_operator), C.c_double, C.c_int32, P, P, P]
        L.rr_noalloc_scratch_bytes.argtypes = []
        L.rr_noalloc_scratch_bytes.restype = C.c_size_t
        L.rr_operator_delta_norm.argtypes = [C.POINTER(rr_operator), C.c_int32, C.c_int32, C.c_uint64,
                                             C.POINTER(C.c_double), P]
        L.rr_cholesky_ladder.argtypes = [P, C.c_int64, P, C.POINTER(C.c_double), P]
        L.rr_lambda_max.argtypes = [P, C.c_int64, C.c_uint64, P, P]
        L.rr_profile_enable.argtypes = [C.c_int32]
        L.rr_profile_enable.restype = None
        L.rr_profile_read.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.rr_profile_read.restype = C.c_int32
        L.rr_precond_destroy.argtypes = [P]
        L.rr_precond_destroy.restype = None
        L.rr_status_string.argtypes = [C.c_int32]
        L.rr_status_string.restype = C.c_char_p
        L.rr_last_error.restype = C.c_char_p
        L.rr_version.restype = C.c_char_p
        for name in ("rr_build_precond", "rr_solve", "rr_solve_batch", "rr_serve",
                     "rr_precond_export", "rr_precond_export_omega", "rr_precond_shape",
                     "rr_kernel_to_dense", "rr_apply_operator", "rr_apply_operator_block", "rr_random_matrix", "rr_sketch_apply",
                     "rr_theta_apply", "rr_cholesky_ladder", "rr_lambda_max", "rr_operator_delta_norm",
                     "rr_apply_operator_noalloc"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class RRError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().rr_last_error().decode()
        super().__init__(f"{where}: {lib().rr_status_string(status).decode()} ({msg})")


def _check(st: int, where: str, ok=(RR_OK,)):
    if st not in ok:
        raise RRError(st, where)
    return st


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ operators
@dataclass
class Operator:
    struct: rr_operator
    keep: tuple = ()

    @property
    def n(self) -> int:
        return int(self.struct.n)


def dense_operator(A) -> Operator:
    """A: CUDA float64 tensor (n, n), symmetric and contiguous (same bytes in both orders)."""
    import torch
    assert A.is_cuda and A.dtype == torch.float64 and A.is_contiguous() and A.shape[0] == A.shape[1]
    s = rr_operator(kind=OP_DENSE, n=A.shape[0], A=A.data_ptr(), lda=A.shape[0], pts=None, d=0,
                    kconst=0.0, scale=1.0)
    return Operator(s, (A,))


def kernel_operator(kind: int, pts, kconst: float, scale: float) -> Operator:
    """pts: CUDA float32 tensor (d, n) contiguous (structure of arrays)."""
    import torch
    assert pts.is_cuda and pts.dtype == torch.float32 and pts.is_contiguous() and pts.dim() == 2
    s = rr_operator(kind=kind, n=pts.shape[1], A=None, lda=0, pts=pts.data_ptr(), d=pts.shape[0],
                    kconst=float(kconst), scale=float(scale))
    return Operator(s, (pts,))


def build_opts(l=0, sketch="gaussian", seed=0, orth="sketched", prec="fp64", tau_rule="opt",
               rho=1.0, power_iters=4, q=0, multi="joint", l_max=0, ad_factor=100.0,
               basis="explicit", reorth=False) -> rr_build_opts:
    o = rr_build_opts()
    lib().rr_build_opts_default(C.byref(o))
    o.l = int(l)
    o.sketch = _SKETCH[sketch] if isinstance(sketch, str) else int(sketch)
    o.seed = int(seed)
    o.orth = _ORTH[orth] if isinstance(orth, str) else int(orth)
    o.prec = _PREC[prec] if isinstance(prec, str) else int(prec)
    o.tau_rule = _TAU[tau_rule] if isinstance(tau_rule, str) else int(tau_rule)
    o.rho = float(rho)
    o.power_iters = int(power_iters)
    o.power_q = int(q)
    o.multi_shift = {"joint": 0, "shifted_chol": 1}[multi] if isinstance(multi, str) else int(multi)
    o.l_max = int(l_max)
    o.ad_factor = float(ad_factor)
    o.basis = {"explicit": 0, "less": 1}[basis] if isinstance(basis, str) else int(basis)
    o.reorth = 1 if reorth else 0
    return o


def solve_opts(tol=1e-6, restart_eta=1e-2, maxit=5000, check_every=8, fp64_ir=-1,
               use_graph=False, certify=True, history=None, method="c", krylov="cg",
               block_kmax=128) -> rr_solve_opts:
    o = rr_solve_opts()
    lib().rr_solve_opts_default(C.byref(o))
    o.tol = float(tol)
    o.restart_eta = float(restart_eta)
    o.maxit = int(maxit)
    o.check_every = int(check_every)
    o.fp64_ir = int(fp64_ir)
    o.use_graph = 1 if use_graph else 0
    o.certify = 1 if certify else 0
    o.method = _METHOD[method] if isinstance(method, str) else int(method)
    o.krylov = _KRYLOV[krylov] if isinstance(krylov, str) else int(krylov)
    o.block_kmax = int(block_kmax)
    if history is not None:
        o.relres_history = history.ctypes.data_as(C.POINTER(C.c_double))
        o.history_cap = len(history)
    return o


class TorchAllocator:
    """An rr_allocator backed by PyTorch's caching allocator (device memory of the
    current device, ordered on the stream the library passes)."""

    def __init__(self):
        import torch
        self.live = {}

        def _alloc(ctx, nbytes, stream):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), None, stream or 0)
            except Exception:
                return None
            self.live[p] = stream
            return p

        def _free(ctx, ptr, stream):
            if ptr:
                self.live.pop(ptr, None)
                torch.cuda.caching_allocator_delete(ptr)

        self._a = rr_allocator._fields_[1][1](_alloc)
        self._f = rr_allocator._fields_[2][1](_free)
        self.struct = rr_allocator(ctx=None, alloc=self._a, free=self._f)


class Precond:
    """Owning wrapper of an rr_precond handle."""

    def __init__(self, handle: C.c_void_p, op: Operator, mus):
        self.h = handle
        self.op = op
        self.mus = list(mus)

    def __del__(self):
        try:
            if self.h:
                lib().rr_precond_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def shape(self):
        n, l, m = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().rr_precond_shape(self.h, C.byref(n), C.byref(l), C.byref(m)), "rr_precond_shape")
        return n.value, l.value, m.value

    def solve(self, b, x0=None, mu_index=0, stream=None, ok=(RR_OK,), **kw):
        """b: CUDA float64 (n,).  Returns (x, info dict)."""
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        hist = kw.pop("history", None)
        o = solve_opts(history=hist, **kw)
        info = rr_solve_info()
        st = lib().rr_solve(self.h, int(mu_index), _ptr(b), _ptr(x), C.byref(o), C.byref(info),
                            _stream(stream))
        _check(st, "rr_solve", ok)
        d = info.as_dict()
        d["rc"] = st
        return x, d

    def solve_batch(self, B, mu_index_per_col: Sequence[int], X0=None, stream=None, ok=(RR_OK,),
                    **kw):
        """B: CUDA float64 (n, m).  Returns (X (n, m), list of info dicts)."""
        import torch
        n, m = B.shape
        Bc = B.t().contiguous()                 # column-major n x m
        Xc = torch.zeros_like(Bc) if X0 is None else X0.t().contiguous()
        idx = (C.c_int32 * m)(*[int(i) for i in mu_index_per_col])
        infos = (rr_solve_info * m)()
        o = solve_opts(**kw)
        st = lib().rr_solve_batch(self.h, idx, _ptr(Bc), n, m, _ptr(Xc), n, C.byref(o), infos,
                                  _stream(stream))
        _check(st, "rr_solve_batch", ok)
        return Xc.t(), [i.as_dict() for i in infos], st

    def export(self, mu_index=0, with_q=True):
        n, l, _ = self.shape
        Q = np.zeros((l, n)) if (with_q and l) else None
        R = np.zeros((l, l)); G = np.zeros((l, l)); T = np.zeros((l, l))
        sc = np.zeros(4)
        p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        _check(lib().rr_precond_export(self.h, int(mu_index), p(Q), p(R) if l else None,
                                       p(G) if l else None, p(T) if l else None, p(sc)),
               "rr_precond_export")
        out = {"tau": sc[0], "normE": sc[1], "lam": sc[2], "mu": sc[3]}
        if l:
            out.update(R=R.T.copy(), G=G.T.copy(), T=T.T.copy())
            if Q is not None:
                out["Q"] = Q.T.copy()
        return out

    def omega(self):
        n, l, _ = self.shape
        O = np.zeros((l, n))
        _check(lib().rr_precond_export_omega(self.h, O.ctypes.data_as(C.c_void_p)), "export_omega")
        return O.T.copy()


def build_precond(op: Operator, mus, l=0, stream=None, allocator=None, **kw) -> Precond:
    mus = [float(m) for m in (mus if isinstance(mus, (list, tuple)) else [mus])]
    arr = (C.c_double * len(mus))(*mus)
    o = build_opts(l=l, **kw)
    h = C.c_void_p()
    ap = C.byref(allocator.struct) if allocator is not None else None
    st = lib().rr_build_precond(C.byref(op.struct), arr, len(mus), C.byref(o), ap,
                                _stream(stream), C.byref(h))
    _check(st, "rr_build_precond")
    P = Precond(h, op, mus)
    P.allocator = allocator   # the handle frees through it: keep it alive as long
    return P


def kernel_to_dense(op: Operator, dtype: str = "fp64", stream=None):
    import torch
    n = op.n
    tdt = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16}[dtype]
    code = {"fp64": 0, "fp32": 1, "bf16": 2}[dtype]
    A = torch.empty((n, n), dtype=tdt, device="cuda")
    _check(lib().rr_kernel_to_dense(C.byref(op.struct), _ptr(A), code, n, _stream(stream)),
           "rr_kernel_to_dense")
    return A   # symmetric: row-major bytes == column-major bytes


def apply_operator(op: Operator, mu: float, prec: str, u, stream=None):
    import torch
    y = torch.empty_like(u)
    _check(lib().rr_apply_operator(C.byref(op.struct), float(mu), _PREC[prec], _ptr(u), _ptr(y),
                                   _stream(stream)), "rr_apply_operator")
    return y


def apply_operator_noalloc(op: Operator, mu: float, prec: str, u, y=None, stream=None):
    """y = (A + mu I) u through the no-allocation entry point (asynchronous on the
    stream; y may be given to keep the call free of any allocation)."""
    import torch
    if y is None:
        y = torch.empty_like(u)
    _check(lib().rr_apply_operator_noalloc(C.byref(op.struct), float(mu), _PREC[prec], _ptr(u), _ptr(y),
                                           _stream(stream)), "rr_apply_operator_noalloc")
    return y


def operator_delta_norm(op: Operator, prec: str = "fp32", iters: int = 20, seed: int = 99, stream=None):
    """||A_work - A||_2 estimate for the working precision `prec` (power iteration)."""
    out = C.c_double()
    _check(lib().rr_operator_delta_norm(C.byref(op.struct), _PREC[prec], int(iters), int(seed),
                                        C.byref(out), _stream(stream)), "rr_operator_delta_norm")
    return out.value


def apply_operator_block(op: Operator, mu: float, prec: str, U, stream=None):
    """Y = (A + mu I) U for a CUDA float64 tensor U (n, nr)."""
    import torch
    n, nr = U.shape
    Uc = U.t().contiguous()                 # column-major n x nr
    Yc = torch.empty_like(Uc)
    _check(lib().rr_apply_operator_block(C.byref(op.struct), float(mu), _PREC[prec], _ptr(Uc), nr,
                                         _ptr(Yc), _stream(stream)), "rr_apply_operator_block")
    return Yc.t()


def random_matrix(kind: str, seed: int, rows: int, cols: int, stream=None):
    """Returns a CUDA float64 tensor (rows, cols) with the library's test matrix."""
    import torch
    out = torch.empty((cols, rows), dtype=torch.float64, device="cuda")
    _check(lib().rr_random_matrix({"gaussian": 0, "srht": 1}[kind], int(seed), int(rows), int(cols),
                                  _ptr(out), _stream(stream)), "rr_random_matrix")
    return out.t()


def theta_apply(seed: int, Y, stream=None):
    """S = Theta Y (2k x k) with the build's second-level sketch for Omega stream `seed`;
    Y: CUDA float64 tensor (n, k)."""
    import torch
    n, k = Y.shape
    Yc = Y.t().contiguous()                 # column-major n x k
    S = torch.empty((k, 2 * k), dtype=torch.float64, device="cuda")
    _check(lib().rr_theta_apply(int(seed), int(n), int(k), _ptr(Yc), _ptr(S), _stream(stream)),
           "rr_theta_apply")
    return S.t()


def cholesky_ladder(W, stream=None):
    """(R, alpha): the build's Cholesky with its shift ladder; W: CUDA float64 (k, k) symmetric."""
    import torch
    k = W.shape[0]
    Wc = W.t().contiguous()
    R = torch.empty_like(Wc)
    a = C.c_double()
    _check(lib().rr_cholesky_ladder(_ptr(Wc), k, _ptr(R), C.byref(a), _stream(stream)),
           "rr_cholesky_ladder")
    return R.t(), a.value


def lambda_max(G, seed: int = 0, stream=None):
    """(lambda_max, residual bound, steps) of a symmetric psd CUDA float64 (k, k) G."""
    k = G.shape[0]
    Gc = G.t().contiguous()
    out = np.zeros(3)
    _check(lib().rr_lambda_max(_ptr(Gc), k, int(seed), out.ctypes.data_as(C.c_void_p),
                               _stream(stream)), "rr_lambda_max")
    return float(out[0]), float(out[1]), int(out[2])


(PROF_KERNEL_MATVEC, PROF_KERNEL_SKETCH, PROF_DENSE_MATVEC, PROF_DENSE_SKETCH, PROF_PROJECT,
 PROF_KERNEL_MATMAT, PROF_KERNEL_MATVEC64, PROF_DENSE_MATVEC64, PROF_GROUP_PRODUCT, PROF_GROUP_FINISH,
 PROF_GROUP_PROJECT, PROF_GROUP_UPDATE) = range(12)


def profile_enable(on: bool = True):
    lib().rr_profile_enable(1 if on else 0)


def profile_read(slot: int):
    """(launch count, total device ms) of a timed kernel slot."""
    c, t = C.c_int64(), C.c_double()
    _check(lib().rr_profile_read(int(slot), C.byref(c), C.byref(t)), "rr_profile_read")
    return c.value, t.value


def sketch(op: Operator, mu: float, l: int, stream=None, **kw):
    """Y = A Omega + mu Omega as the build computes it; CUDA float64 tensor (n, l)."""
    import torch
    o = build_opts(l=l, **kw)
    out = torch.empty((l, op.n), dtype=torch.float64, device="cuda")
    _check(lib().rr_sketch_apply(C.byref(op.struct), float(mu), C.byref(o), _ptr(out),
                                 _stream(stream)), "rr_sketch_apply")
    return out.t()


def serve(requests, hbm_budget: int = 96 << 30, max_slots: int = 8, graph_iters: int = 8,
          build: Optional[dict] = None, solve: Optional[dict] = None, allocator=None,
          grouped: int = 0):
    """Run the continuous-batching server over `requests` (arrival-ordered).

    grouped: the PCG batches of the waiting requests run as replays of grouped kernels
    on this many lanes (0: each request replays its own graph).

    Each request is a dict with keys: kind, pts (float32 (d, n) host array), kconst,
    scale, mu, l, seed, B (float64 (n, m) host array), t_arrival (seconds after the
    start).  Returns (results, stats): results[i] = {"X": (n, m) array, "info": dict,
    "t_done": float}.
    """
    bo = build_opts(**(build or {}))
    so = solve_opts(**(solve or {}))
    cfg = rr_serve_config(hbm_budget=int(hbm_budget), max_slots=int(max_slots),
                          graph_iters=int(graph_iters), build=bo, solve=so, grouped=int(grouped))
    keep = []
    for i, r in enumerate(requests):
        pts = np.ascontiguousarray(r["pts"], dtype=np.float32)
        B = np.asarray(r["B"], dtype=np.float64)
        if B.ndim == 1:
            B = B[:, None]
        Bc = np.ascontiguousarray(B.T)            # column-major n x m
        Xc = np.zeros_like(Bc)
        keep.append((pts, Bc, Xc))
    state = {"i": 0}
    results = [None] * len(requests)

    def _next(user, now, out):
        i = state["i"]
        if i >= len(requests):
            return -1
        r = requests[i]
        if r["t_arrival"] > now:
            return 0
        pts, Bc, Xc = keep[i]
        o = out.contents
        o.kind = int(r.get("kind", OP_RBF))
        o.n = pts.shape[1]
        o.d = pts.shape[0]
        o.pts = pts.ctypes.data
        o.kconst = float(r["kconst"])
        o.scale = float(r["scale"])
        o.mu = float(r["mu"])
        o.l = int(r["l"])
        o.nrhs = Bc.shape[0]
        o.B = Bc.ctypes.data
        o.X = Xc.ctypes.data
        o.id = i
        o.seed = int(r.get("seed", 0))
        o.t_arrival = float(r["t_arrival"])
        state["i"] = i + 1
        return 1

    def _deliver(user, req, info, t_done):
        i = int(req.contents.id)
        results[i] = {"info": info.contents.as_dict(), "t_done": float(t_done)}

    nf, df = NEXT_FN(_next), DELIVER_FN(_deliver)
    stats = rr_serve_stats()
    if allocator is not None:
        cfg.alloc = C.pointer(allocator.struct)
    st = lib().rr_serve(C.byref(cfg), nf, df, None, C.byref(stats))
    if st == RR_EINVAL or (st != RR_OK and stats.served + stats.rejected == 0):
        _check(st, "rr_serve")
    for i, (pts, Bc, Xc) in enumerate(keep):
        if results[i] is not None:
            results[i]["X"] = Xc.T.copy()
    out = stats.as_dict()
    out["status"] = st
    if st != RR_OK:
        out["first_error"] = lib().rr_last_error().decode()
    return results, out

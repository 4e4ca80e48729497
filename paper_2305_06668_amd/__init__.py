"""MI355X block LOBPCG (arXiv:2305.06668) -- Python binding of liblobpcg.so.

The binding only marshals arguments: every step of the solver runs in the HIP
library.  PyTorch supplies device memory (the operator arrays, the workspace,
result buffers) and the stream.  The functions ``lobpcg_*`` below carry the
names of the C entry points of ``include/lobpcg.h`` and take torch tensors
where the C function takes device pointers; ``Solver`` bundles them.

Importing the module loads the shared library and raises ImportError when it
is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblobpcg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2305_06668_amd/build.py` "
        "(hipcc, gfx950); there is no CPU fallback"
    )
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants mirrored from include/lobpcg.h ----------------------------
OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = -1
ERR_BAD_STATE = -2
ERR_DEVICE = -3
ERR_WORKSPACE = -4
ERR_ORTHO_FAILED = -5
ERR_NONFINITE = -6
ERR_UNSUPPORTED = -7

PRECOND_NONE = 0
PRECOND_DIAG = 1
PRECOND_DIAG_SIGNED = 2
PRECOND_LEARNED = 3
PRECOND_TRIDIAG = 4
LEARNED_NPARAMS = 17153

PREC_FP64 = 0
PREC_FP32 = 1

OPT_TAU_ORTHO = 0
OPT_MAX_ITER = 1
OPT_PRECISION = 2
OPT_ORTHO_MAX_PASSES = 3
OPT_ORTHO_Y_MAX_PASSES = 4
OPT_TRACE = 5
OPT_LEARNED_BF16 = 6
OPT_RR_JACOBI = 7
OPT_SHIFT_RETRIES = 8
OPT_FORCE_RESTARTS = 9
OPT_CHEAP_EXIT = 10
OPT_METHOD = 11
OPT_DAVIDSON_MAX_DIM = 12
OPT_LEARNED_BUDGET = 13
OPT_STALL_WINDOW = 14
OPT_SPMM_SLAB = 15

METHOD_LOBPCG = 0
METHOD_DAVIDSON = 1

_i32, _i64, _dbl, _vp, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class lobpcg_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", _i32),
        ("converged", _i32),
        ("matvec_columns", _i64),
        ("ortho_grams", _i32),
        ("ortho_factorizations", _i32),
        ("ortho_failed", _i32),
        ("ortho_shifted", _i32),
        ("ortho_stalled", _i32),
        ("ortho_svqb", _i32),
        ("against_passes", _i32),
        ("true_checks", _i32),
        ("relocks", _i32),
        ("precision_switch_iter", _i32),
        ("m_conv", _i32),
        ("ms_total", _dbl),
        ("ms_operator", _dbl),
        ("ms_rr", _dbl),
        ("ms_ortho", _dbl),
        ("ms_sync", _dbl),
        ("learned_fallbacks", _i32),
        ("learned_nonfinite", _i32),
        ("rr_eig_fallbacks", _i32),
        ("restarts", _i32),
        ("ortho_cheap_exits", _i32),
        ("history_restarts", _i32),
        ("max_basis", _i32),
        ("b_matvec_columns", _i64),
        ("learned_budget_iter", _i32),
        ("stall_checks", _i32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class lobpcg_ortho_info(ctypes.Structure):
    _fields_ = [
        (f, _i32)
        for f in ("grams", "factorizations", "failed", "shifted", "updates", "passes", "stalled", "svqb", "cheap_exits")
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def _sig(name, argtypes, restype=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


_c = {
    "create": _sig("lobpcg_create", [_i64, ctypes.c_int, ctypes.POINTER(_vp)]),
    "destroy": _sig("lobpcg_destroy", [_vp]),
    "set_stream": _sig("lobpcg_set_stream", [_vp, _vp]),
    "set_option": _sig("lobpcg_set_option", [_vp, ctypes.c_int, _dbl]),
    "workspace_size": _sig(
        "lobpcg_workspace_size", [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_sz)]
    ),
    "set_workspace": _sig("lobpcg_set_workspace", [_vp, _vp, _sz]),
    "set_operator_csr": _sig("lobpcg_set_operator_csr", [_vp, _vp, _vp, _vp, _i64]),
    "set_operator_dense": _sig("lobpcg_set_operator_dense", [_vp, _vp, _i64]),
    "set_operator_kronsum": _sig("lobpcg_set_operator_kronsum", [_vp, _i64, _vp, _vp]),
    "set_operator_b_csr": _sig("lobpcg_set_operator_b_csr", [_vp, _vp, _vp, _vp, _i64]),
    "set_operator_b_dense": _sig("lobpcg_set_operator_b_dense", [_vp, _vp, _i64]),
    "set_preconditioner": _sig("lobpcg_set_preconditioner", [_vp, ctypes.c_int, _vp]),
    "set_initial_guess": _sig("lobpcg_set_initial_guess", [_vp, _vp, _i64, ctypes.c_int]),
    "set_initial_guess_host": _sig("lobpcg_set_initial_guess_host", [_vp, _vp, _i64, ctypes.c_int]),
    "solve": _sig("lobpcg_solve", [_vp, ctypes.c_int, _dbl]),
    "get_eigenpairs": _sig("lobpcg_get_eigenpairs", [_vp, ctypes.c_int, _vp, _vp, _i64, _vp]),
    "get_eigenpairs_host": _sig("lobpcg_get_eigenpairs_host", [_vp, ctypes.c_int, _vp, _vp, _i64, _vp]),
    "get_stats": _sig("lobpcg_get_stats", [_vp, ctypes.POINTER(lobpcg_stats)]),
    "status_string": _sig("lobpcg_status_string", [ctypes.c_int], ctypes.c_char_p),
    "last_error": _sig("lobpcg_last_error", [_vp], ctypes.c_char_p),
    "apply_operator": _sig("lobpcg_apply_operator", [_vp, _vp, _i64, ctypes.c_int, _vp, _i64]),
    "apply_operator_f32": _sig("lobpcg_apply_operator_f32", [_vp, _vp, _i64, ctypes.c_int, _vp, _i64]),
    "gram": _sig("lobpcg_gram", [_vp, _vp, _i64, ctypes.c_int, _vp, _i64, ctypes.c_int, _vp]),
    "gram_noalloc": _sig("lobpcg_gram_noalloc", [_vp, _vp, _i64, ctypes.c_int, _vp, _i64, ctypes.c_int, _vp]),
    "ortho": _sig("lobpcg_ortho", [_vp, _vp, _i64, ctypes.c_int, ctypes.POINTER(lobpcg_ortho_info)]),
    "ortho_against": _sig(
        "lobpcg_ortho_against", [_vp, _vp, _i64, ctypes.c_int, _vp, _i64, ctypes.c_int, ctypes.POINTER(lobpcg_ortho_info)]
    ),
    "small_eigh": _sig("lobpcg_small_eigh", [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "small_cholesky": _sig("lobpcg_small_cholesky", [_vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int)]),
    "rotate": _sig(
        "lobpcg_rotate",
        [_vp, _vp, _vp, _i64, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _i64, _vp],
    ),
    "set_learned_weights": _sig("lobpcg_set_learned_weights", [_vp, _vp, _i64]),
    "learned_apply": _sig("lobpcg_learned_apply", [_vp, _vp, _i64, ctypes.c_int, _vp, _vp]),
    "tridiag_apply": _sig("lobpcg_tridiag_apply", [_vp, _vp, _i64, ctypes.c_int, _vp]),
    "learner_create": _sig("lobpcg_learner_create", [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "learner_destroy": _sig("lobpcg_learner_destroy", [_vp]),
    "learner_set_weights": _sig("lobpcg_learner_set_weights", [_vp, _vp, _i64]),
    "learner_get_weights": _sig("lobpcg_learner_get_weights", [_vp, _vp, _i64]),
    "learner_add_snapshot": _sig(
        "lobpcg_learner_add_snapshot",
        [_vp, _vp, _vp, _i64, ctypes.c_int, ctypes.c_int, _dbl, ctypes.POINTER(ctypes.c_int)],
    ),
    "learner_snapshot_info": _sig("lobpcg_learner_snapshot_info", [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "learner_objective": _sig(
        "lobpcg_learner_objective", [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]
    ),
    "learner_train": _sig(
        "lobpcg_learner_train",
        [_vp, ctypes.c_int, ctypes.c_int, _dbl, ctypes.c_uint64, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)],
    ),
    "learner_set_supervision": _sig("lobpcg_learner_set_supervision", [_vp, ctypes.c_double]),
    "learner_last_error": _sig("lobpcg_learner_last_error", [_vp], ctypes.c_char_p),
}

EXPORTED = [
    "lobpcg_create", "lobpcg_destroy", "lobpcg_set_stream", "lobpcg_set_option",
    "lobpcg_workspace_size", "lobpcg_set_workspace", "lobpcg_set_operator_csr",
    "lobpcg_set_operator_dense", "lobpcg_set_operator_kronsum", "lobpcg_set_operator_b_csr",
    "lobpcg_set_operator_b_dense", "lobpcg_set_preconditioner",
    "lobpcg_set_initial_guess", "lobpcg_set_initial_guess_host", "lobpcg_solve",
    "lobpcg_get_eigenpairs", "lobpcg_get_eigenpairs_host", "lobpcg_get_stats",
    "lobpcg_status_string", "lobpcg_last_error", "lobpcg_apply_operator", "lobpcg_apply_operator_f32", "lobpcg_gram",
    "lobpcg_gram_noalloc",
    "lobpcg_ortho", "lobpcg_ortho_against", "lobpcg_small_eigh", "lobpcg_small_cholesky",
    "lobpcg_rotate", "lobpcg_set_learned_weights", "lobpcg_learned_apply", "lobpcg_tridiag_apply",
    "lobpcg_learner_create", "lobpcg_learner_destroy",
    "lobpcg_learner_set_weights", "lobpcg_learner_get_weights", "lobpcg_learner_add_snapshot",
    "lobpcg_learner_snapshot_info", "lobpcg_learner_objective", "lobpcg_learner_train",
    "lobpcg_learner_last_error", "lobpcg_learner_set_supervision",
]


class LobpcgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status}: {lobpcg_status_string(status)})")
        self.status = status


def lobpcg_status_string(status: int) -> str:
    return _c["status_string"](status).decode()


def lobpcg_last_error(h) -> str:
    return _c["last_error"](h).decode()


def _check(h, rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        msg = lobpcg_last_error(h) if h else ""
        raise LobpcgError(rc, msg)
    return rc


# ---- torch plumbing --------------------------------------------------------


def _torch():
    import torch

    return torch


def _dev_ptr(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _ld(t, name="block"):
    """Leading dimension of a row-major 2-D tensor view (unit column stride)."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major view with unit column stride")
    return max(t.stride(0), t.shape[1])


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---- thin wrappers with the C names ---------------------------------------


def lobpcg_create(n: int, device: int = 0):
    h = ctypes.c_void_p()
    rc = _c["create"](int(n), int(device), ctypes.byref(h))
    if rc != OK:
        raise LobpcgError(rc, "lobpcg_create failed")
    return h


def lobpcg_destroy(h) -> None:
    _check(h, _c["destroy"](h))


def lobpcg_set_stream(h, stream_ptr=None) -> None:
    _check(h, _c["set_stream"](h, stream_ptr if stream_ptr is not None else _stream_ptr()))


def lobpcg_set_option(h, key: int, value: float) -> None:
    _check(h, _c["set_option"](h, int(key), float(value)))


def lobpcg_workspace_size(h, k: int, block: int, precision: int = PREC_FP64) -> int:
    out = ctypes.c_size_t()
    _check(h, _c["workspace_size"](h, int(k), int(block), int(precision), ctypes.byref(out)))
    return int(out.value)


def lobpcg_set_workspace(h, ws) -> None:
    _check(h, _c["set_workspace"](h, _dev_ptr(ws, name="workspace"), ws.numel() * ws.element_size()))


def lobpcg_set_operator_csr(h, row_ptr, col, val) -> None:
    torch = _torch()
    _check(
        h,
        _c["set_operator_csr"](
            h,
            _dev_ptr(row_ptr, torch.int32, "row_ptr"),
            _dev_ptr(col, torch.int32, "col"),
            _dev_ptr(val, torch.float64, "val"),
            int(col.numel()),
        ),
    )


def lobpcg_set_operator_dense(h, A) -> None:
    torch = _torch()
    _check(h, _c["set_operator_dense"](h, _dev_ptr(A, torch.float64, "A"), _ld(A, "A")))


def lobpcg_set_operator_kronsum(h, A, V) -> None:
    torch = _torch()
    _check(
        h,
        _c["set_operator_kronsum"](h, int(A.shape[0]), _dev_ptr(A, torch.float64, "A"), _dev_ptr(V, torch.float64, "V")),
    )


def lobpcg_set_operator_b_csr(h, row_ptr, col, val) -> None:
    """B of A x = lambda B x as CSR (cuda tensors); row_ptr None: standard problem."""
    torch = _torch()
    if row_ptr is None:
        _check(h, _c["set_operator_b_csr"](h, None, None, None, 0))
        return
    _check(
        h,
        _c["set_operator_b_csr"](
            h,
            _dev_ptr(row_ptr, torch.int32, "row_ptr"),
            _dev_ptr(col, torch.int32, "col"),
            _dev_ptr(val, torch.float64, "val"),
            int(col.numel()),
        ),
    )


def lobpcg_set_operator_b_dense(h, B) -> None:
    """B of A x = lambda B x, dense row-major (cuda); None: standard problem."""
    torch = _torch()
    if B is None:
        _check(h, _c["set_operator_b_dense"](h, None, 0))
        return
    _check(h, _c["set_operator_b_dense"](h, _dev_ptr(B, torch.float64, "B"), _ld(B, "B")))


def lobpcg_set_preconditioner(h, kind: int, diag=None) -> None:
    torch = _torch()
    ptr = _dev_ptr(diag, torch.float64, "diag") if diag is not None else None
    _check(h, _c["set_preconditioner"](h, int(kind), ptr))


def lobpcg_set_initial_guess(h, X0) -> None:
    torch = _torch()
    _check(h, _c["set_initial_guess"](h, _dev_ptr(X0, torch.float64, "X0"), _ld(X0, "X0"), int(X0.shape[1])))


def lobpcg_set_initial_guess_host(h, X0: np.ndarray) -> None:
    """X0: host n x block array; passed to the library column-major."""
    Xf = np.asfortranarray(X0, dtype=np.float64)
    _check(h, _c["set_initial_guess_host"](h, Xf.ctypes.data_as(ctypes.c_void_p), int(Xf.shape[0]), int(Xf.shape[1])))


def lobpcg_solve(h, k: int, tol: float) -> int:
    return _check(h, _c["solve"](h, int(k), float(tol)), allow=(OK, NOT_CONVERGED))


def lobpcg_get_eigenpairs(h, k: int, evecs=None):
    torch = _torch()
    ev = np.zeros(k)
    rn = np.zeros(k)
    vptr = _dev_ptr(evecs, torch.float64, "evecs") if evecs is not None else None
    ld = _ld(evecs, "evecs") if evecs is not None else 0
    _check(
        h,
        _c["get_eigenpairs"](
            h, int(k), ev.ctypes.data_as(ctypes.c_void_p), vptr, ld, rn.ctypes.data_as(ctypes.c_void_p)
        ),
    )
    return ev, rn


def lobpcg_get_eigenpairs_host(h, k: int, n: int, want_vectors: bool = True):
    """Eigenvalues, residual norms and (optionally) the n x k eigenvectors as
    a host array, read back column-major."""
    ev = np.zeros(k)
    rn = np.zeros(k)
    X = np.zeros((n, k), order="F") if want_vectors else None
    _check(
        h,
        _c["get_eigenpairs_host"](
            h,
            int(k),
            ev.ctypes.data_as(ctypes.c_void_p),
            X.ctypes.data_as(ctypes.c_void_p) if X is not None else None,
            int(n),
            rn.ctypes.data_as(ctypes.c_void_p),
        ),
    )
    return ev, rn, X


def lobpcg_get_stats(h) -> dict:
    st = lobpcg_stats()
    _check(h, _c["get_stats"](h, ctypes.byref(st)))
    return st.as_dict()


def lobpcg_apply_operator(h, W, Y) -> None:
    torch = _torch()
    _check(
        h,
        _c["apply_operator"](
            h, _dev_ptr(W, torch.float64, "W"), _ld(W, "W"), int(W.shape[1]), _dev_ptr(Y, torch.float64, "Y"), _ld(Y, "Y")
        ),
    )


def lobpcg_apply_operator_f32(h, W, Y) -> None:
    """fp32 Y = A W with the operator rounded to fp32 (needs OPT_PRECISION = PREC_FP32)."""
    torch = _torch()
    _check(
        h,
        _c["apply_operator_f32"](
            h, _dev_ptr(W, torch.float32, "W"), _ld(W, "W"), int(W.shape[1]), _dev_ptr(Y, torch.float32, "Y"), _ld(Y, "Y")
        ),
    )


def lobpcg_gram_noalloc(h, A, B, C) -> None:
    """lobpcg_gram without a workspace (static device scratch, p, q <= 64)."""
    torch = _torch()
    _check(
        h,
        _c["gram_noalloc"](
            h,
            _dev_ptr(A, torch.float64, "A"),
            _ld(A, "A"),
            int(A.shape[1]),
            _dev_ptr(B, torch.float64, "B"),
            _ld(B, "B"),
            int(B.shape[1]),
            _dev_ptr(C, torch.float64, "C"),
        ),
    )


def lobpcg_gram(h, A, B, C) -> None:
    torch = _torch()
    _check(
        h,
        _c["gram"](
            h,
            _dev_ptr(A, torch.float64, "A"),
            _ld(A, "A"),
            int(A.shape[1]),
            _dev_ptr(B, torch.float64, "B"),
            _ld(B, "B"),
            int(B.shape[1]),
            _dev_ptr(C, torch.float64, "C"),
        ),
    )


def lobpcg_ortho(h, X) -> dict:
    torch = _torch()
    info = lobpcg_ortho_info()
    _check(h, _c["ortho"](h, _dev_ptr(X, torch.float64, "X"), _ld(X, "X"), int(X.shape[1]), ctypes.byref(info)))
    return info.as_dict()


def lobpcg_ortho_against(h, X, Y) -> dict:
    """X and Y are column slices of one row-major buffer, X right after Y."""
    torch = _torch()
    info = lobpcg_ortho_info()
    _check(
        h,
        _c["ortho_against"](
            h,
            _dev_ptr(X, torch.float64, "X"),
            _ld(X, "X"),
            int(X.shape[1]),
            _dev_ptr(Y, torch.float64, "Y"),
            _ld(Y, "Y"),
            int(Y.shape[1]),
            ctypes.byref(info),
        ),
    )
    return info.as_dict()


def lobpcg_small_eigh(h, a, evals, evecs) -> None:
    torch = _torch()
    _check(
        h,
        _c["small_eigh"](
            h, _dev_ptr(a, torch.float64, "a"), int(a.shape[0]), _dev_ptr(evals, torch.float64), _dev_ptr(evecs, torch.float64)
        ),
    )


def lobpcg_small_cholesky(h, M, L) -> int:
    torch = _torch()
    shifts = ctypes.c_int()
    _check(h, _c["small_cholesky"](h, _dev_ptr(M, torch.float64, "M"), int(M.shape[0]), _dev_ptr(L, torch.float64, "L"), ctypes.byref(shifts)))
    return int(shifts.value)


def lobpcg_rotate(h, V, AV, p, U, m, q, theta, a0, Vout, AVout, resnorm2) -> None:
    torch = _torch()
    _check(
        h,
        _c["rotate"](
            h,
            _dev_ptr(V, torch.float64, "V"),
            _dev_ptr(AV, torch.float64, "AV"),
            _ld(V, "V"),
            int(p),
            _dev_ptr(U, torch.float64, "U"),
            int(m),
            int(q),
            _dev_ptr(theta, torch.float64, "theta"),
            int(a0),
            _dev_ptr(Vout, torch.float64, "Vout"),
            _dev_ptr(AVout, torch.float64, "AVout"),
            _ld(Vout, "Vout"),
            _dev_ptr(resnorm2, torch.float64, "resnorm2"),
        ),
    )


def _host_f32(w, name="weights"):
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
    if a.ndim != 1 or a.size != LEARNED_NPARAMS:
        raise ValueError(f"{name}: need {LEARNED_NPARAMS} float32 values")
    return a


def lobpcg_set_learned_weights(h, w) -> None:
    a = _host_f32(w)
    _check(h, _c["set_learned_weights"](h, a.ctypes.data_as(_vp), a.size))


def lobpcg_learned_apply(h, R, theta, mask=None) -> None:
    torch = _torch()
    nact = R.shape[1]
    if theta.numel() != nact:
        raise ValueError("theta: one value per column")
    mp = None
    if mask is not None:
        if mask.dtype != torch.int32 or mask.numel() != nact or not mask.is_cuda:
            raise ValueError("mask: int32 cuda tensor, one value per column")
        mp = ctypes.c_void_p(mask.data_ptr())
    _check(h, _c["learned_apply"](h, _dev_ptr(R, torch.float64, "R"), _ld(R, "R"), nact, _dev_ptr(theta, torch.float64, "theta"), mp))


def lobpcg_tridiag_apply(h, R, theta) -> None:
    """In place: column j of R (cuda, n x nact) <- T_j^-1 R[:, j]."""
    torch = _torch()
    nact = R.shape[1]
    if theta.numel() != nact:
        raise ValueError("theta: one value per column")
    _check(h, _c["tridiag_apply"](h, _dev_ptr(R, torch.float64, "R"), _ld(R, "R"), nact, _dev_ptr(theta, torch.float64, "theta")))


def lobpcg_learner_last_error(L) -> str:
    return (_c["learner_last_error"](L) or b"").decode()


def _lcheck(L, rc: int) -> int:
    if rc != OK:
        raise LobpcgError(rc, f"{lobpcg_status_string(rc)}: {lobpcg_learner_last_error(L)}")
    return rc


def lobpcg_learner_create(device: int = 0, seed: int = 1):
    out = _vp()
    rc = _c["learner_create"](device, ctypes.c_uint64(seed), ctypes.byref(out))
    if rc != OK:
        raise LobpcgError(rc, f"lobpcg_learner_create: {lobpcg_status_string(rc)}")
    return out


def lobpcg_learner_destroy(L) -> None:
    _c["learner_destroy"](L)


def lobpcg_learner_set_weights(L, w) -> None:
    a = _host_f32(w)
    _lcheck(L, _c["learner_set_weights"](L, a.ctypes.data_as(_vp), a.size))


def lobpcg_learner_set_supervision(L, mu: float) -> None:
    """Weight of the supervised term (alignment with the MINRES corrections)."""
    _lcheck(L, _c["learner_set_supervision"](L, float(mu)))


def lobpcg_learner_get_weights(L) -> np.ndarray:
    a = np.empty(LEARNED_NPARAMS, dtype=np.float32)
    _lcheck(L, _c["learner_get_weights"](L, a.ctypes.data_as(_vp), a.size))
    return a


def lobpcg_learner_add_snapshot(L, h, X, minres_maxiter: int = 300, minres_rtol: float = 1e-6) -> int:
    torch = _torch()
    idx = ctypes.c_int(-1)
    _lcheck(
        L,
        _c["learner_add_snapshot"](
            L, h, _dev_ptr(X, torch.float64, "X"), _ld(X, "X"), X.shape[1], int(minres_maxiter), float(minres_rtol), ctypes.byref(idx)
        ),
    )
    return idx.value


def lobpcg_learner_snapshot_info(L, snap: int, m: int) -> dict:
    out = {k: np.empty(m) for k in ("theta", "resnorm", "ref_decrease", "minres_relres")}
    _lcheck(
        L,
        _c["learner_snapshot_info"](
            L, snap, *(out[k].ctypes.data_as(_vp) for k in ("theta", "resnorm", "ref_decrease", "minres_relres"))
        ),
    )
    return out


def lobpcg_learner_objective(L, snap: int, cols, want_grad: bool = False, want_decreases: bool = False):
    c = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
    loss = ctypes.c_double()
    g = np.empty(LEARNED_NPARAMS) if want_grad else None
    dl = np.empty(c.size) if want_decreases else None
    dj = np.empty(c.size) if want_decreases else None
    ptr = lambda a: a.ctypes.data_as(_vp) if a is not None else None
    _lcheck(L, _c["learner_objective"](L, snap, c.ctypes.data_as(_vp), c.size, ctypes.byref(loss), ptr(g), ptr(dl), ptr(dj)))
    return dict(loss=loss.value, grad=g, learned_decrease=dl, jacobi_decrease=dj)


def lobpcg_learner_train(L, steps: int, cols_per_step: int, lr: float, seed: int = 1):
    a, b = ctypes.c_double(), ctypes.c_double()
    _lcheck(L, _c["learner_train"](L, steps, cols_per_step, lr, ctypes.c_uint64(seed), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


# ---- convenience object ----------------------------------------------------


@dataclass
class Result:
    evals: np.ndarray
    resnorms: np.ndarray
    evecs: object  # torch tensor (n x k, cuda) or None
    status: int
    stats: dict


class Solver:
    """Owns a handle, its torch-allocated workspace and references to every
    borrowed device array (so they outlive the handle's use of them)."""

    def __init__(self, n: int, device: int = 0):
        torch = _torch()
        self.n = int(n)
        self.device = int(device)
        self.h = lobpcg_create(self.n, self.device)
        self._keep = {}
        self._ws = None
        self._block = None
        self._prec = PREC_FP64
        lobpcg_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def close(self):
        if self.h:
            lobpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # operators -------------------------------------------------------------
    def set_operator_csr(self, row_ptr, col, val):
        self._keep["op"] = (row_ptr, col, val)
        lobpcg_set_operator_csr(self.h, row_ptr, col, val)
        if self._block is not None:
            self.ensure_workspace(self._block)  # the workspace depends on the operator

    def set_operator_dense(self, A):
        self._keep["op"] = (A,)
        lobpcg_set_operator_dense(self.h, A)
        if self._block is not None:
            self.ensure_workspace(self._block)  # the workspace depends on the operator

    def set_operator_kronsum(self, A, V):
        self._keep["op"] = (A, V)
        lobpcg_set_operator_kronsum(self.h, A, V)
        if self._block is not None:
            self.ensure_workspace(self._block)  # the workspace depends on the operator

    def set_operator_b_csr(self, row_ptr, col, val):
        self._keep["opb"] = (row_ptr, col, val)
        lobpcg_set_operator_b_csr(self.h, row_ptr, col, val)
        if self._block is not None:
            self.ensure_workspace(self._block)  # B V needs its own buffers

    def set_operator_b_dense(self, B):
        self._keep["opb"] = (B,)
        lobpcg_set_operator_b_dense(self.h, B)
        if self._block is not None:
            self.ensure_workspace(self._block)

    def set_preconditioner(self, kind=PRECOND_DIAG, diag=None):
        self._keep["diag"] = diag
        lobpcg_set_preconditioner(self.h, kind, diag)
        if self._block is not None:
            self.ensure_workspace(self._block)  # the tridiagonal solve needs more workspace

    def set_learned_weights(self, w):
        lobpcg_set_learned_weights(self.h, w)

    def set_option(self, key, value):
        lobpcg_set_option(self.h, key, value)
        if key == OPT_PRECISION:
            self._prec = int(value)
        if key in (OPT_PRECISION, OPT_METHOD, OPT_DAVIDSON_MAX_DIM, OPT_SPMM_SLAB) and self._block is not None:
            # the fp32 phase and the Davidson basis need other workspace sizes
            self.ensure_workspace(self._block)

    def set_initial_guess(self, X0):
        self._keep["X0"] = X0
        lobpcg_set_initial_guess(self.h, X0)
        self.ensure_workspace(X0.shape[1])

    def set_initial_guess_host(self, X0: np.ndarray):
        self._keep["X0"] = None
        lobpcg_set_initial_guess_host(self.h, X0)
        self.ensure_workspace(X0.shape[1])

    def ensure_workspace(self, block: int):
        torch = _torch()
        need = lobpcg_workspace_size(self.h, 1, block, self._prec)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        ptr = self._ws.data_ptr()
        off = (-ptr) % 256
        view = self._ws[off : off + need]
        lobpcg_set_workspace(self.h, view)
        self._block = block

    def solve(self, k: int, tol: float = 1e-8, want_vectors: bool = True) -> Result:
        torch = _torch()
        if self._block is None:
            self.ensure_workspace(k)
        status = lobpcg_solve(self.h, k, tol)
        evecs = torch.empty((self.n, k), dtype=torch.float64, device=f"cuda:{self.device}") if want_vectors else None
        ev, rn = lobpcg_get_eigenpairs(self.h, k, evecs)
        return Result(evals=ev, resnorms=rn, evecs=evecs, status=status, stats=lobpcg_get_stats(self.h))

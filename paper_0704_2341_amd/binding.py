"""ctypes binding of libgrg.so (include/grg.h), names as in the C ABI.

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors (complex128 on a ROCm device),
passed by ``data_ptr()``; the stream is torch's current stream unless given.
There is no CPU fallback: if the library is missing or fails to load, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrg.so")

GRG_OK = 0
GRG_EINVAL = -1
GRG_EODD_EXTENT = -2
GRG_ENOMEM = -3
GRG_EHIP = -4
GRG_ENOCONV = -5
GRG_ENONFINITE = -6
GRG_ETOO_LARGE = -7
GRG_EUNSUPPORTED = -8
STATUS_NAMES = {
    0: "GRG_OK", -1: "GRG_EINVAL", -2: "GRG_EODD_EXTENT", -3: "GRG_ENOMEM", -4: "GRG_EHIP",
    -5: "GRG_ENOCONV", -6: "GRG_ENONFINITE", -7: "GRG_ETOO_LARGE", -8: "GRG_EUNSUPPORTED",
}
GRG_PERM_I, GRG_PERM_II = 1, 2
GRG_FP64, GRG_FP32, GRG_BF16 = 0, 1, 2
PRECISIONS = {"fp64": GRG_FP64, "fp32": GRG_FP32, "bf16": GRG_BF16}

# Every symbol include/grg.h declares.
EXPORTS = (
    "grg_last_error", "grg_version", "grg_solver_params_default", "grg_lattice_create",
    "grg_lattice_destroy", "grg_lattice_volume", "grg_gauge_set", "grg_permutation_block",
    "grg_dirac_apply", "grg_dirac_apply_noalloc", "grg_schur_create", "grg_schur_destroy",
    "grg_schur_set_params",
    "grg_drr_solve", "grg_schur_apply", "grg_schur_assemble", "grg_reusken_apply",
    "grg_reusken_assemble", "grg_diag_schur_apply", "grg_diag_schur_assemble", "grg_schur_tune",
    "grg_schur_tune_info", "grg_schur_set_launch", "grg_schur_dc_launch_info",
    "grg_schur_set_dc_launch", "grg_block_apply", "grg_reduced_apply", "grg_precond_create",
    "grg_precond_destroy", "grg_precond_set_weights", "grg_precond_get_weights", "grg_precond_apply",
    "grg_precond_loss_grad", "grg_precond_train", "grg_precond_save", "grg_precond_load",
    "grg_schur_attach_precond", "grg_batch_create", "grg_batch_destroy", "grg_batch_layout",
    "grg_batch_apply", "grg_batch_tune", "grg_batch_graph_info",
    "grg_batch_tune_info", "grg_profile_enable",
    "grg_profile_read", "grg_profile_reset", "grg_vcycle_params_default", "grg_vcycle_create",
    "grg_vcycle_destroy", "grg_vcycle_apply", "grg_vcycle_solve",
)


class GrgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class grg_solver_params(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int), ("inner", C.c_int),
        ("inner_tol", C.c_double), ("max_outer", C.c_int), ("max_rhs", C.c_int),
        ("check_every", C.c_int), ("verify", C.c_int), ("eo", C.c_int), ("method", C.c_int),
    ]


class grg_solver_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("outer", C.c_int), ("converged", C.c_int), ("n_dslash", C.c_int),
        ("true_rel_resid", C.c_double), ("t_total_ms", C.c_double), ("t_dslash_ms", C.c_double),
        ("fallbacks", C.c_int), ("t_dc_ms", C.c_double), ("t_blas_ms", C.c_double),
        ("t_prec_ms", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class grg_vcycle_params(C.Structure):
    _fields_ = [("levels", C.c_int), ("drr_tol", C.c_double), ("top_tol", C.c_double),
                ("max_rhs", C.c_int), ("max_iter", C.c_int), ("perm", C.c_int), ("inverse", C.c_int)]


class grg_vcycle_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rate", C.c_double),
                ("true_rel_resid", C.c_double), ("t_ms", C.c_double), ("cycles", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class grg_train_params(C.Structure):
    _fields_ = [("steps", C.c_int), ("batch", C.c_int), ("max_mr_steps", C.c_int),
                ("lr", C.c_double), ("seed", C.c_uint64), ("log_every", C.c_int), ("reduced", C.c_int)]


class grg_train_stats(C.Structure):
    _fields_ = [("steps", C.c_int), ("pairs", C.c_int), ("loss_first", C.c_double),
                ("loss_last", C.c_double), ("t_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


GRG_PRECOND_WEIGHTS = 1152


class grg_batch_member(C.Structure):
    _fields_ = [("dims", C.c_int32 * 4), ("bc", C.c_int32 * 4), ("m0", C.c_double),
                ("links", C.c_void_p), ("q", C.c_void_p), ("n_coarse", C.c_int32)]

_lib = None


def load():
    """Load libgrg.so; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_0704_2341_amd.build` "
                          "(there is no CPU fallback)")
    # torch bundles its own HIP runtime (same soname as /opt/rocm's).  Loading
    # torch first makes libgrg.so bind to that one runtime; loading libgrg.so
    # first would map a second HIP/HSA runtime into the process, and the two
    # cannot share the device.
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    vp, i32p, i64p, dp = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
    sig = {
        "grg_last_error": (C.c_char_p, []),
        "grg_version": (C.c_char_p, []),
        "grg_solver_params_default": (C.c_int, [C.POINTER(grg_solver_params)]),
        "grg_lattice_create": (C.c_int, [i32p, i32p, vp, C.POINTER(vp)]),
        "grg_lattice_destroy": (C.c_int, [vp]),
        "grg_lattice_volume": (C.c_int, [vp, i64p]),
        "grg_gauge_set": (C.c_int, [vp, vp, C.c_int]),
        "grg_permutation_block": (C.c_int, [i32p, C.c_int, C.c_int, i32p, i32p]),
        "grg_dirac_apply": (C.c_int, [vp, C.c_double, C.c_int, vp, vp, C.c_int]),
        "grg_dirac_apply_noalloc": (C.c_int, [vp, C.c_double, C.c_int, vp, vp, C.c_int]),
        "grg_schur_create": (C.c_int, [vp, C.c_double, i32p, C.c_int32,
                                       C.POINTER(grg_solver_params), C.POINTER(vp)]),
        "grg_schur_destroy": (C.c_int, [vp]),
        "grg_schur_set_params": (C.c_int, [vp, C.POINTER(grg_solver_params)]),
        "grg_drr_solve": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(grg_solver_stats)]),
        "grg_schur_apply": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(grg_solver_stats)]),
        "grg_schur_assemble": (C.c_int, [vp, vp, C.c_size_t]),
        "grg_reusken_apply": (C.c_int, [vp, vp, vp, C.c_int]),
        "grg_reusken_assemble": (C.c_int, [vp, vp, C.c_size_t]),
        "grg_diag_schur_apply": (C.c_int, [vp, vp, vp, C.c_int]),
        "grg_diag_schur_assemble": (C.c_int, [vp, vp, C.c_size_t]),
        "grg_schur_tune": (C.c_int, [vp, C.c_int]),
        "grg_schur_tune_info": (C.c_int, [vp, C.c_int, C.c_int, i32p, C.POINTER(C.c_float)]),
        "grg_schur_set_launch": (C.c_int, [vp, C.c_int, C.c_int, i32p]),
        "grg_schur_dc_launch_info": (C.c_int, [vp, C.c_int, C.c_int, i32p, C.POINTER(C.c_float)]),
        "grg_schur_set_dc_launch": (C.c_int, [vp, C.c_int, C.c_int, i32p]),
        "grg_block_apply": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, C.c_int]),
        "grg_reduced_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, C.c_int]),
        "grg_precond_create": (C.c_int, [vp, C.POINTER(vp)]),
        "grg_vcycle_params_default": (C.c_int, [C.POINTER(grg_vcycle_params)]),
        "grg_vcycle_create": (C.c_int, [vp, C.c_double, C.POINTER(grg_vcycle_params), C.POINTER(vp)]),
        "grg_vcycle_destroy": (C.c_int, [vp]),
        "grg_vcycle_apply": (C.c_int, [vp, vp, vp, C.c_int]),
        "grg_vcycle_solve": (C.c_int, [vp, C.c_int, C.c_double, vp, vp, C.c_int,
                                       C.POINTER(grg_vcycle_stats)]),
        "grg_precond_destroy": (C.c_int, [vp]),
        "grg_precond_set_weights": (C.c_int, [vp, vp]),
        "grg_precond_get_weights": (C.c_int, [vp, vp]),
        "grg_precond_apply": (C.c_int, [vp, vp, vp, C.c_int]),
        "grg_precond_loss_grad": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(C.c_double), vp]),
        "grg_precond_train": (C.c_int, [vp, C.POINTER(grg_train_params), C.POINTER(grg_train_stats)]),
        "grg_precond_save": (C.c_int, [vp, C.c_char_p]),
        "grg_precond_load": (C.c_int, [vp, C.c_char_p]),
        "grg_schur_attach_precond": (C.c_int, [vp, vp]),
        "grg_batch_create": (C.c_int, [C.POINTER(grg_batch_member), C.c_int, C.c_int,
                                       C.POINTER(grg_solver_params), vp, C.POINTER(vp)]),
        "grg_batch_destroy": (C.c_int, [vp]),
        "grg_batch_layout": (C.c_int, [vp, C.c_int, i64p, i32p]),
        "grg_batch_apply": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(grg_solver_stats)]),
        "grg_batch_tune": (C.c_int, [vp]),
        "grg_batch_graph_info": (C.c_int, [vp, i32p]),
        "grg_batch_tune_info": (C.c_int, [vp, C.c_int, i32p, C.POINTER(C.c_float)]),
        "grg_profile_enable": (C.c_int, [vp, C.c_int]),
        "grg_profile_read": (C.c_int, [vp, C.c_int, i64p, dp]),
        "grg_profile_reset": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != GRG_OK and status not in allow:
        raise GrgError(status, load().grg_last_error().decode())
    return status


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _ptr(t):
    return C.c_void_p(int(t.data_ptr()))


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch

    return C.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ------------------------------------------------------------------ the ABI
def grg_last_error() -> str:
    return load().grg_last_error().decode()


def grg_version() -> str:
    return load().grg_version().decode()


def grg_solver_params_default(**overrides) -> grg_solver_params:
    p = grg_solver_params()
    _check(load().grg_solver_params_default(C.byref(p)))
    for k, v in overrides.items():
        if k == "inner":
            v = _prec(v)
        if k == "method" and isinstance(v, str):
            v = {"gcr": 0, "bicgstab": 1}[v]
        setattr(p, k, v)
    return p


def grg_lattice_create(dims, bc=(1, 1, 1, -1), stream=None):
    d, dp = _i32(dims)
    b, bp = _i32(bc)
    h = C.c_void_p()
    _check(load().grg_lattice_create(dp, bp, _stream(stream), C.byref(h)))
    return h


def grg_lattice_destroy(lat):
    _check(load().grg_lattice_destroy(lat))


def grg_lattice_volume(lat) -> int:
    v = C.c_int64()
    _check(load().grg_lattice_volume(lat, C.byref(v)))
    return v.value


def grg_gauge_set(lat, links):
    """links: complex128 (V, 4, 3, 3) numpy array (host) or torch tensor (host or device)."""
    if isinstance(links, np.ndarray):
        a = np.ascontiguousarray(links, dtype=np.complex128)
        _check(load().grg_gauge_set(lat, C.c_void_p(a.ctypes.data), 0))
        return
    t = links.contiguous()
    _check(load().grg_gauge_set(lat, _ptr(t), 1 if t.is_cuda else 0))


def grg_permutation_block(dims, type, inverse=False):
    """Returns (q int32[V], n_coarse)."""
    d, dp = _i32(dims)
    v = int(np.prod(d, dtype=np.int64))
    q = np.zeros(v, dtype=np.int32)
    nb = C.c_int32()
    _check(load().grg_permutation_block(dp, int(type), int(bool(inverse)),
                                        q.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nb)))
    return q, nb.value


def grg_dirac_apply(lat, m0, precision, x, out, nrhs):
    _check(load().grg_dirac_apply(lat, float(m0), _prec(precision), _ptr(x), _ptr(out), int(nrhs)))


GRG_NOALLOC_SCRATCH_BYTES = 32 << 20


def grg_dirac_apply_noalloc(lat, m0, precision, x, out, nrhs):
    """As grg_dirac_apply, with the staging in the library's fixed per-GPU
    scratch: allocates nothing; GRG_ETOO_LARGE beyond its size."""
    _check(load().grg_dirac_apply_noalloc(lat, float(m0), _prec(precision), _ptr(x), _ptr(out), int(nrhs)))


def grg_schur_create(lat, m0, q, n_coarse, params=None):
    qa, qp = _i32(q)
    h = C.c_void_p()
    pp = C.byref(params) if params is not None else None
    _check(load().grg_schur_create(lat, float(m0), qp, int(n_coarse), pp, C.byref(h)))
    return h


def grg_schur_destroy(s):
    _check(load().grg_schur_destroy(s))


def grg_schur_set_params(s, params):
    _check(load().grg_schur_set_params(s, C.byref(params)))


def grg_drr_solve(s, rhs, x, nrhs, allow_noconv=False):
    st = grg_solver_stats()
    status = _check(load().grg_drr_solve(s, _ptr(rhs), _ptr(x), int(nrhs), C.byref(st)),
                    allow=(GRG_ENOCONV,) if allow_noconv else ())
    d = st.as_dict()
    d["status"] = status
    return d


def grg_schur_apply(s, x_b, y_b, nrhs, allow_noconv=False):
    st = grg_solver_stats()
    status = _check(load().grg_schur_apply(s, _ptr(x_b), _ptr(y_b), int(nrhs), C.byref(st)),
                    allow=(GRG_ENOCONV,) if allow_noconv else ())
    d = st.as_dict()
    d["status"] = status
    return d


def grg_schur_assemble(s, n_coarse):
    """Dense S_bb as a numpy complex128 (12 N_b, 12 N_b) array."""
    n = 12 * int(n_coarse)
    buf = np.zeros(n * n, dtype=np.complex128)
    _check(load().grg_schur_assemble(s, C.c_void_p(buf.ctypes.data), buf.nbytes))
    return buf.reshape(n, n).T  # column-major storage


def grg_reusken_apply(s, x_b, y_b, nrhs):
    """y_b = S~_bb x_b, the section 3 approximation (FP64, no solve)."""
    _check(load().grg_reusken_apply(s, _ptr(x_b), _ptr(y_b), int(nrhs)))


def grg_reusken_assemble(s, n_coarse):
    """Dense S~_bb as a numpy complex128 (12 N_b, 12 N_b) array."""
    n = 12 * int(n_coarse)
    buf = np.zeros(n * n, dtype=np.complex128)
    _check(load().grg_reusken_assemble(s, C.c_void_p(buf.ctypes.data), buf.nbytes))
    return buf.reshape(n, n).T  # column-major storage


def grg_diag_schur_apply(s, x_b, y_b, nrhs):
    """y_b = (D_bb - D_br D_rb / d) x_b, the approximation that ignores the
    couplings inside D_rr (FP64, no solve)."""
    _check(load().grg_diag_schur_apply(s, _ptr(x_b), _ptr(y_b), int(nrhs)))


def grg_diag_schur_assemble(s, n_coarse):
    """Dense D_bb - D_br D_rb / d as a numpy complex128 (12 N_b, 12 N_b) array."""
    n = 12 * int(n_coarse)
    buf = np.zeros(n * n, dtype=np.complex128)
    _check(load().grg_diag_schur_assemble(s, C.c_void_p(buf.ctypes.data), buf.nbytes))
    return buf.reshape(n, n).T  # column-major storage


def grg_schur_tune(s, nrhs):
    _check(load().grg_schur_tune(s, int(nrhs)))


def grg_schur_tune_info(s, precision, nrhs, eo=False):
    """{'SB', 'RG', 'split', 'grid', 'chunk', 'march', 'ms'} of the stencil launch in
    use (eo=True: the half-lattice stencil of the even-odd reduced solve)."""
    info = (C.c_int32 * 6)()
    ms = C.c_float()
    _check(load().grg_schur_tune_info(s, _prec(precision) + (3 if eo else 0), int(nrhs), info,
                                      C.byref(ms)))
    return {"SB": info[0], "RG": info[1], "split": info[2], "grid": info[3], "chunk": info[4],
            "march": info[5], "ms": ms.value}


def grg_reduced_apply(s, precision, parity, x, y, nrhs):
    """y = (d - H_pq H_qp / d) x on the rest sites of parity p (canonical
    device fields, complex128 [nrhs][12 V])."""
    _check(load().grg_reduced_apply(s, _prec(precision), int(parity), _ptr(x), _ptr(y), int(nrhs)))


def grg_schur_set_launch(s, precision, nrhs, info, eo=False):
    """info: dict as returned by grg_schur_tune_info (or a 6-sequence); eo=True
    pins the half-lattice stencil of the even-odd reduced solve."""
    if isinstance(info, dict):
        info = [info.get(k, 0) for k in ("SB", "RG", "split", "grid", "chunk", "march")]
    arr, ptr = _i32(info)
    _check(load().grg_schur_set_launch(s, _prec(precision) + (3 if eo else 0), int(nrhs), ptr))


def grg_schur_dc_launch_info(s, precision, nrhs):
    """The defect-correction step's launch for (inner precision, nrhs), as a dict."""
    info = (C.c_int32 * 6)()
    ms = C.c_float()
    _check(load().grg_schur_dc_launch_info(s, _prec(precision), int(nrhs), info, C.byref(ms)))
    return {"SB": info[0], "RG": info[1], "split": info[2], "grid": info[3], "chunk": info[4],
            "march": info[5], "ms": ms.value}


def grg_schur_set_dc_launch(s, precision, nrhs, info):
    """info: dict as returned by grg_schur_dc_launch_info (or a 6-sequence)."""
    if isinstance(info, dict):
        info = [info.get(k, 0) for k in ("SB", "RG", "split", "grid", "chunk", "march")]
    arr, ptr = _i32(info)
    _check(load().grg_schur_set_dc_launch(s, _prec(precision), int(nrhs), ptr))


def grg_block_apply(s, precision, rows, cols, x, out, nrhs):
    """out = D_{rows, cols} x; rows / cols: 1 coarse, 0 rest, -1 all."""
    _check(load().grg_block_apply(s, _prec(precision), int(rows), int(cols), _ptr(x), _ptr(out),
                                  int(nrhs)))


def grg_precond_create(s):
    h = C.c_void_p()
    _check(load().grg_precond_create(s, C.byref(h)))
    return h


def grg_precond_destroy(p):
    _check(load().grg_precond_destroy(p))


def grg_precond_set_weights(p, w):
    """w: complex128 array of GRG_PRECOND_WEIGHTS (layer-major, [hop][f_out][f_in])."""
    a = np.ascontiguousarray(w, dtype=np.complex128)
    assert a.size == GRG_PRECOND_WEIGHTS
    _check(load().grg_precond_set_weights(p, C.c_void_p(a.ctypes.data)))


def grg_precond_get_weights(p):
    a = np.zeros(GRG_PRECOND_WEIGHTS, dtype=np.complex128)
    _check(load().grg_precond_get_weights(p, C.c_void_p(a.ctypes.data)))
    return a


def grg_precond_apply(p, x, out, nrhs):
    _check(load().grg_precond_apply(p, _ptr(x), _ptr(out), int(nrhs)))


def grg_precond_loss_grad(p, r, e, nrhs):
    """(loss, dL/dconj(W) as complex128 array)."""
    loss = C.c_double()
    g = np.zeros(GRG_PRECOND_WEIGHTS, dtype=np.complex128)
    _check(load().grg_precond_loss_grad(p, _ptr(r), _ptr(e), int(nrhs), C.byref(loss),
                                        C.c_void_p(g.ctypes.data)))
    return loss.value, g


def grg_precond_train(p, steps, batch, max_mr_steps=20, lr=1e-3, seed=5, log_every=20,
                      reduced=False):
    tp = grg_train_params(int(steps), int(batch), int(max_mr_steps), float(lr), int(seed),
                          int(log_every), int(bool(reduced)))
    st = grg_train_stats()
    _check(load().grg_precond_train(p, C.byref(tp), C.byref(st)))
    return st.as_dict()


def grg_precond_save(p, path):
    _check(load().grg_precond_save(p, os.fsencode(path)))


def grg_precond_load(p, path):
    _check(load().grg_precond_load(p, os.fsencode(path)))


def grg_schur_attach_precond(s, p):
    _check(load().grg_schur_attach_precond(s, p))


def grg_batch_create(members, nrhs, params=None, stream=None):
    """members: list of dicts with dims, bc, m0, links (complex128 numpy
    (V, 4, 3, 3)), q (int array), n_coarse.  Returns (handle, keepalive)."""
    arr = (grg_batch_member * len(members))()
    keep = []
    for i, m in enumerate(members):
        links = np.ascontiguousarray(m["links"], dtype=np.complex128)
        q = np.ascontiguousarray(m["q"], dtype=np.int32)
        keep += [links, q]
        arr[i].dims[:] = [int(d) for d in m["dims"]]
        arr[i].bc[:] = [int(b) for b in m.get("bc", (1, 1, 1, -1))]
        arr[i].m0 = float(m["m0"])
        arr[i].links = links.ctypes.data
        arr[i].q = q.ctypes.data
        arr[i].n_coarse = int(m["n_coarse"])
    h = C.c_void_p()
    pp = C.byref(params) if params is not None else None
    _check(load().grg_batch_create(arr, len(members), int(nrhs), pp, _stream(stream), C.byref(h)))
    return h


def grg_batch_destroy(b):
    _check(load().grg_batch_destroy(b))


def grg_batch_layout(b, member):
    off, nb = C.c_int64(), C.c_int32()
    _check(load().grg_batch_layout(b, int(member), C.byref(off), C.byref(nb)))
    return off.value, nb.value


def grg_batch_apply(b, x_b, y_b, use_graph=True, allow_noconv=False):
    st = grg_solver_stats()
    status = _check(load().grg_batch_apply(b, _ptr(x_b), _ptr(y_b), int(bool(use_graph)), C.byref(st)),
                    allow=(GRG_ENOCONV,) if allow_noconv else ())
    d = st.as_dict()
    d["status"] = status
    return d


def grg_batch_tune(b):
    _check(load().grg_batch_tune(b))


def grg_batch_tune_info(b, precision):
    """{'SB', 'RG', 'grid', 'stencil_ms', 'update_ms'} of the batched launch in use."""
    info, ms = (C.c_int32 * 3)(), (C.c_float * 2)()
    _check(load().grg_batch_tune_info(b, _prec(precision), info, ms))
    return {"SB": info[0], "RG": info[1], "grid": info[2], "stencil_ms": ms[0], "update_ms": ms[1]}


def grg_batch_graph_info(b):
    """(outer steps, inner iterations per step) of the captured apply; (0, 0) if none."""
    c = (C.c_int32 * 2)()
    _check(load().grg_batch_graph_info(b, c))
    return int(c[0]), int(c[1])


def grg_profile_enable(s, on=True, launches_only=False):
    _check(load().grg_profile_enable(s, 0 if not on else 2 if launches_only else 1))


PROFILE_PHASES = {"dc": 6, "blas": 7, "precond": 8}


def grg_profile_read(s, precision, eo=False):
    """(count, summed ms) of the full-lattice stencil in `precision`, or with
    eo=True of the even-odd half-lattice stencil; precision "dc", "blas" or
    "precond" reads the solve's phase of that name instead."""
    n, ms = C.c_int64(), C.c_double()
    slot = PROFILE_PHASES[precision] if precision in PROFILE_PHASES else _prec(precision) + (3 if eo else 0)
    _check(load().grg_profile_read(s, slot, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def grg_profile_reset(s):
    _check(load().grg_profile_reset(s))


# ---------------------------------------------------------------- V-cycle (section 4)
def grg_vcycle_params_default(**overrides) -> grg_vcycle_params:
    p = grg_vcycle_params()
    _check(load().grg_vcycle_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def grg_vcycle_create(lat, m0, params=None):
    h = C.c_void_p()
    _check(load().grg_vcycle_create(lat, float(m0), C.byref(params) if params is not None else None,
                                    C.byref(h)))
    return h


def grg_vcycle_destroy(v):
    _check(load().grg_vcycle_destroy(v))


def grg_vcycle_apply(v, f, x, nrhs):
    """x = M f, one V-cycle (canonical device fields)."""
    _check(load().grg_vcycle_apply(v, _ptr(f), _ptr(x), int(nrhs)))


def grg_vcycle_solve(v, f, x, nrhs, tol=1e-8, precondition=True, allow_noconv=False):
    """Solve D x = f by BiCGstab, right-preconditioned by the V-cycle."""
    st = grg_vcycle_stats()
    status = load().grg_vcycle_solve(v, int(bool(precondition)), float(tol), _ptr(f), _ptr(x), int(nrhs),
                                     C.byref(st))
    if not (allow_noconv and status == -5):
        _check(status)
    return st.as_dict()

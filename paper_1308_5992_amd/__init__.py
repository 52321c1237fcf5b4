"""Python binding of libbamg (include/bamg.h): argument marshalling only.

Every function keeps the name of the C entry point it calls.  Arrays are
torch tensors on the GPU (complex128, contiguous); their data pointers are
passed to the library together with torch's current HIP stream, so the work
is ordered with the caller's torch work.  There is no fallback: if the HIP
library is missing the import of this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbamg.so")

BAMG_OK, BAMG_NOT_CONVERGED, BAMG_PENDING = 0, 1, 2
BAMG_EINVAL, BAMG_ENOMEM, BAMG_EDEVICE, BAMG_ESINGULAR, BAMG_ENOTIMPL = -1, -2, -3, -4, -5
BAMG_CYCLE_V, BAMG_CYCLE_W, BAMG_CYCLE_K = 0, 1, 2
BAMG_FP64, BAMG_MIXED_FP16, BAMG_MIXED_BF16, BAMG_MIXED_FP32 = 0, 1, 2, 3
OP_APPLY, OP_SWEEP, OP_RESTRICT, OP_PROLONG, OP_COARSEST, OP_CYCLE, OP_RESIDUAL = range(7)
OP_APPLY_MIXED, OP_SWEEP_MIXED, OP_CYCLE_MIXED = 7, 8, 9
OP_APPLY_F32, OP_SWEEP_F32, OP_COARSEST_F32 = 10, 11, 12
OP_SWEEP_COLOURS, OP_SWEEP_COLOURS_F32 = 13, 14
BOOT_RITZ, BOOT_SWEEP, BOOT_EIGS, BOOT_FIT = range(4)

EXPORTED = [
    "bamg_default_params", "bamg_setup", "bamg_solve", "bamg_solve_batch", "bamg_apply_dhat",
    "bamg_eo_reduce", "bamg_eo_reconstruct", "bamg_level_op", "bamg_n_levels", "bamg_level_info",
    "bamg_export_level", "bamg_import_level", "bamg_footprint_bytes", "bamg_gaussian_tv",
    "bamg_free", "bamg_last_error", "bamg_boot_op", "bamg_export_boot",
    "bamg_server_default_params", "bamg_server_create", "bamg_server_add_field", "bamg_server_field_bytes",
    "bamg_server_submit", "bamg_server_progress", "bamg_server_wait", "bamg_server_get_stats", "bamg_server_reset_stats",
    "bamg_server_free", "bamg_stationary", "bamg_full_residual", "bamg_full_residual_noalloc",
]


class bamg_params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("max_coarse", ctypes.c_int32),
        ("n_tv", ctypes.c_int32), ("setup_sweeps", ctypes.c_int32), ("setup_adapt", ctypes.c_int32),
        ("pre", ctypes.c_int32), ("post", ctypes.c_int32), ("cycle", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("init_tv_host", ctypes.c_void_p), ("stream", ctypes.c_void_p),
        ("graphs", ctypes.c_int32), ("setup_mode", ctypes.c_int32), ("n_ev", ctypes.c_int32),
        ("boot_nu1", ctypes.c_int32), ("boot_nu2", ctypes.c_int32), ("coarsest_fp32", ctypes.c_int32),
        ("lookahead", ctypes.c_int32),
    ]


class bamg_solve_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("relres_reduced", ctypes.c_double),
        ("relres_full", ctypes.c_double), ("rho_est", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bamg_server_params(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("slots_per_field", ctypes.c_int32), ("threaded", ctypes.c_int32)]


class bamg_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rhs_completed", ctypes.c_int64),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
        ("resident_fields", ctypes.c_int32), ("evictions", ctypes.c_int32), ("setups", ctypes.c_int32),
        ("bytes_in_use", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t), ("rounds", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libbamg.so is not built ({LIB_PATH}); run python paper_1308_5992_amd/build.py")
    # torch first: the library then binds to the HIP runtime torch ships and
    # shares its devices and streams.  Loaded first, it would bring in the
    # system's runtime (same soname), and the two stacks in one process do not
    # see the GPU alike.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    P, I32, D, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_size_t
    PP = ctypes.POINTER(bamg_params)
    PI = ctypes.POINTER(bamg_solve_info)
    sig = {
        "bamg_default_params": (I32, [PP]),
        "bamg_setup": (I32, [P, D, PP, ctypes.POINTER(P)]),
        "bamg_solve": (I32, [P, P, P, D, PI]),
        "bamg_solve_batch": (I32, [P, P, P, I32, D, PI]),
        "bamg_apply_dhat": (I32, [P, P, P, I32]),
        "bamg_eo_reduce": (I32, [P, P, P, I32]),
        "bamg_eo_reconstruct": (I32, [P, P, P, P, I32]),
        "bamg_level_op": (I32, [P, I32, I32, P, P, I32]),
        "bamg_n_levels": (I32, [P]),
        "bamg_level_info": (I32, [P, I32, P]),
        "bamg_export_level": (I32, [P, I32, P, P, P]),
        "bamg_import_level": (I32, [P, I32, P, P]),
        "bamg_footprint_bytes": (SZ, [PP]),
        "bamg_gaussian_tv": (I32, [I32, I32, U64, P, P]),
        "bamg_fine_sweep_plan": (I32, [I32, I32, I32, I32, P]),
        "bamg_free": (None, [P]),
        "bamg_last_error": (ctypes.c_char_p, []),
        "bamg_boot_op": (I32, [P, I32, I32, P, P, I32]),
        "bamg_export_boot": (I32, [P, P, P]),
        "bamg_server_default_params": (I32, [ctypes.POINTER(bamg_server_params)]),
        "bamg_server_create": (I32, [ctypes.POINTER(bamg_server_params), ctypes.POINTER(P)]),
        "bamg_server_add_field": (I32, [P, P, D, PP, ctypes.POINTER(I32)]),
        "bamg_server_field_bytes": (I32, [P, I32, ctypes.POINTER(SZ)]),
        "bamg_server_submit": (I32, [P, I32, P, P, I32, D, ctypes.POINTER(ctypes.c_int64)]),
        "bamg_server_progress": (I32, [P, ctypes.POINTER(I32)]),
        "bamg_server_wait": (I32, [P, ctypes.c_int64, D, PI]),
        "bamg_server_get_stats": (I32, [P, ctypes.POINTER(bamg_server_stats)]),
        "bamg_server_reset_stats": (I32, [P]),
        "bamg_server_free": (None, [P]),
        "bamg_stationary": (I32, [P, P, I32, P]),
        "bamg_full_residual": (I32, [I32, P, D, P, P, I32, P, P]),
        "bamg_full_residual_noalloc": (I32, [I32, P, D, P, P, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


class BamgError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: status {status}: {bamg_last_error()}")
        self.status = status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, complex64=False):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    want = torch.complex64 if complex64 else torch.complex128
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {want} GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _check(st, where, allow_nc=False):
    if st < 0 or (st == BAMG_NOT_CONVERGED and not allow_nc):
        raise BamgError(st, where)
    return st


def bamg_last_error() -> str:
    return lib.bamg_last_error().decode()


def bamg_default_params(**kw) -> bamg_params:
    p = bamg_params()
    lib.bamg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "init_tv_host":
            continue
        setattr(p, k, v)
    return p


def bamg_footprint_bytes(p: bamg_params) -> int:
    return int(lib.bamg_footprint_bytes(ctypes.byref(p)))


class Hierarchy(ctypes.c_void_p):
    """Opaque hierarchy handle (freed by bamg_free or when collected)."""

    def __del__(self):
        if self.value:
            lib.bamg_free(self)
            self.value = None


def bamg_setup(gauge, m: float, p: bamg_params, init_tv=None) -> Hierarchy:
    """gauge: complex128 GPU tensor U[mu][y][x]; init_tv: optional host numpy [k][N*N]."""
    if p.stream is None:
        p.stream = _stream().value
    keep = None
    if init_tv is not None:
        keep = np.ascontiguousarray(init_tv, dtype=np.complex128)
        p.init_tv_host = keep.ctypes.data
    else:
        p.init_tv_host = None
    h = Hierarchy()
    st = lib.bamg_setup(_ptr(gauge), float(m), ctypes.byref(p), ctypes.byref(h))
    p.init_tv_host = None
    _check(st, "bamg_setup")
    return h


def bamg_solve(h, b, x, tol: float):
    info = bamg_solve_info()
    st = lib.bamg_solve(h, _ptr(b), _ptr(x), float(tol), ctypes.byref(info))
    _check(st, "bamg_solve", allow_nc=True)
    return st, info.as_dict()


def bamg_solve_batch(h, B, X, nrhs: int, tol: float):
    infos = (bamg_solve_info * nrhs)()
    st = lib.bamg_solve_batch(h, _ptr(B), _ptr(X), int(nrhs), float(tol), infos)
    _check(st, "bamg_solve_batch", allow_nc=True)
    return st, [i.as_dict() for i in infos]


def bamg_apply_dhat(h, x, y, nrhs: int = 1):
    _check(lib.bamg_apply_dhat(h, _ptr(x), _ptr(y), int(nrhs)), "bamg_apply_dhat")


def bamg_eo_reduce(h, b, bhat, nrhs: int = 1):
    _check(lib.bamg_eo_reduce(h, _ptr(b), _ptr(bhat), int(nrhs)), "bamg_eo_reduce")


def bamg_eo_reconstruct(h, b, xe, x, nrhs: int = 1):
    _check(lib.bamg_eo_reconstruct(h, _ptr(b), _ptr(xe), _ptr(x), int(nrhs)), "bamg_eo_reconstruct")


def bamg_level_op(h, level: int, op: int, inp, out, nrhs: int = 1):
    """Ops 10, 11, 12 and 14 take complex64 tensors, every other op complex128."""
    c64 = op in (OP_APPLY_F32, OP_SWEEP_F32, OP_COARSEST_F32, OP_SWEEP_COLOURS_F32)
    _check(lib.bamg_level_op(h, int(level), int(op), _ptr(inp, c64), _ptr(out, c64), int(nrhs)), "bamg_level_op")


def bamg_boot_op(h, level: int, op: int, X, lam, k: int):
    """Bootstrap eigensolver pieces (see bamg.h); lam: numpy float64 array of k
    entries (input for BOOT_SWEEP, output for BOOT_RITZ and BOOT_EIGS)."""
    if lam.dtype != np.float64 or not lam.flags.c_contiguous or lam.size < k:
        raise TypeError("lam must be a contiguous float64 array of k entries")
    _check(lib.bamg_boot_op(h, int(level), int(op), _ptr(X), lam.ctypes.data, int(k)), "bamg_boot_op")


def bamg_export_boot(h, N: int):
    """(Ritz values, level-0 eigenvector approximations [k_e][N*N]) of a bootstrap hierarchy."""
    lam = np.zeros(16)
    ke = _check(lib.bamg_export_boot(h, lam.ctypes.data, None), "bamg_export_boot")
    ve = np.zeros((ke, N * N), dtype=np.complex128)
    lib.bamg_export_boot(h, lam.ctypes.data, ve.ctypes.data)
    return lam[:ke].copy(), ve


def bamg_n_levels(h) -> int:
    return _check(lib.bamg_n_levels(h), "bamg_n_levels")


def bamg_level_info(h, level: int) -> dict:
    info = np.zeros(5, dtype=np.int32)
    _check(lib.bamg_level_info(h, int(level), info.ctypes.data), "bamg_level_info")
    return dict(ex=int(info[0]), ey=int(info[1]), dps=int(info[2]), n=int(info[3]), colours=int(info[4]))


def bamg_export_level(h, level: int, P=True, D=True, tv=False, n_tv=8):
    """Host copies of P_l [agg][2][rows][8], D_l [site][7][16][16] and the level-0 test vectors."""
    nl = bamg_n_levels(h)
    inf = bamg_level_info(h, level)
    Pa = Da = Ta = None
    if P and level < nl - 1:
        cinf = bamg_level_info(h, level + 1)
        rows = 16 if level == 0 else 32
        Pa = np.zeros((cinf["ex"] * cinf["ey"], 2, rows, 8), dtype=np.complex128)
    if D and level >= 1:
        Da = np.zeros((inf["ex"] * inf["ey"], 7, 16, 16), dtype=np.complex128)
    if tv and level == 0:
        Ta = np.zeros((n_tv, inf["n"]), dtype=np.complex128)
    ptr = lambda a: None if a is None else a.ctypes.data
    _check(lib.bamg_export_level(h, int(level), ptr(Pa), ptr(Da), ptr(Ta)), "bamg_export_level")
    return Pa, Da, Ta


def bamg_import_level(h, level: int, P=None, D=None):
    """P: host P_l [agg][2][rows][8] (rebuilds level l+1); D: host D_l [site][7][16][16]
    (level >= 1; replaced first)."""
    P = None if P is None else np.ascontiguousarray(P, dtype=np.complex128)
    D = None if D is None else np.ascontiguousarray(D, dtype=np.complex128)
    _check(lib.bamg_import_level(h, int(level), None if P is None else P.ctypes.data,
                                 None if D is None else D.ctypes.data), "bamg_import_level")


def bamg_stationary(h, x, iters: int):
    """x (reduced, complex128 GPU tensor) <- iters steps of x + M(0 - Dhat x);
    returns the norms of x after 0..iters steps (numpy)."""
    norms = np.zeros(int(iters) + 1)
    _check(lib.bamg_stationary(h, _ptr(x), int(iters), norms.ctypes.data), "bamg_stationary")
    return norms


def _relres_ptr(relres, nrhs):
    import torch
    if not (isinstance(relres, torch.Tensor) and relres.is_cuda and relres.dtype == torch.float64
            and relres.is_contiguous() and relres.numel() >= nrhs):
        raise TypeError("relres must be a contiguous float64 GPU tensor of nrhs entries")
    return ctypes.c_void_p(relres.data_ptr())


def bamg_full_residual(N: int, gauge, m: float, B, X, nrhs: int, relres):
    """relres (float64 GPU tensor of nrhs) = ||b - D x|| / ||b|| per right-hand side."""
    _check(lib.bamg_full_residual(int(N), _ptr(gauge), float(m), _ptr(B), _ptr(X), int(nrhs),
                                  _relres_ptr(relres, nrhs), _stream()), "bamg_full_residual")


def bamg_full_residual_noalloc(N: int, gauge, m: float, B, X, nrhs: int, relres):
    """bamg_full_residual with the library's static scratch (allocates nothing)."""
    _check(lib.bamg_full_residual_noalloc(int(N), _ptr(gauge), float(m), _ptr(B), _ptr(X), int(nrhs),
                                          _relres_ptr(relres, nrhs), _stream()), "bamg_full_residual_noalloc")


def bamg_fine_sweep_plan(N: int, nrhs: int = 1, fp32: bool = False, form: int = 0):
    """(form, plan) of the level-0 sweep blocked in LDS (host only): form 1, 2
    or 3 and a dict of the tile plan (with the pipelined form's ring lead A,
    macro-steps M and ring columns W, zeros for forms 1 and 2), or (0, None)
    where the colour passes are used (form 0) or no tile applies."""
    out = np.zeros(77, dtype=np.int32)
    got = lib.bamg_fine_sweep_plan(int(N), int(nrhs), int(bool(fp32)), int(form), out.ctypes.data)
    if got < 0:
        _check(got, "bamg_fine_sweep_plan")
    if got == 0:
        return 0, None
    keys = ["Tu", "Tv", "ntu", "ntv", "i0", "j0", "Ru", "Rv", "nupd"]
    plan = {k: int(out[i]) for i, k in enumerate(keys)}
    plan["first"] = out[9:26].tolist()
    plan["si0"] = out[26:42].tolist()
    plan["sj0"] = out[42:58].tolist()
    plan["nj"] = out[58:74].tolist()
    plan["A"], plan["M"], plan["W"] = (int(v) for v in out[74:77])
    return int(got), plan


def bamg_gaussian_tv(N: int, k: int, seed: int, out):
    _check(lib.bamg_gaussian_tv(int(N), int(k), int(seed), _ptr(out), _stream()), "bamg_gaussian_tv")


def bamg_free(h):
    if h is not None and h.value:
        lib.bamg_free(h)
        h.value = None


# ---------------------------------------------------------------- serving
class Server(ctypes.c_void_p):
    """Opaque server handle (freed by bamg_server_free or when collected)."""

    def __del__(self):
        if self.value:
            lib.bamg_server_free(self)
            self.value = None


def bamg_server_default_params(**kw) -> bamg_server_params:
    sp = bamg_server_params()
    lib.bamg_server_default_params(ctypes.byref(sp))
    for k, v in kw.items():
        setattr(sp, k, v)
    return sp


def bamg_server_create(sp: bamg_server_params) -> Server:
    s = Server()
    _check(lib.bamg_server_create(ctypes.byref(sp), ctypes.byref(s)), "bamg_server_create")
    return s


def bamg_server_add_field(s, gauge, m: float, p: bamg_params) -> int:
    import torch
    torch.cuda.current_stream().synchronize()
    p.init_tv_host = None
    fid = ctypes.c_int32()
    _check(lib.bamg_server_add_field(s, _ptr(gauge), float(m), ctypes.byref(p), ctypes.byref(fid)),
           "bamg_server_add_field")
    return fid.value


def bamg_server_field_bytes(s, field: int) -> int:
    b = ctypes.c_size_t()
    _check(lib.bamg_server_field_bytes(s, int(field), ctypes.byref(b)), "bamg_server_field_bytes")
    return b.value


def bamg_server_submit(s, field: int, B, X, nrhs: int, tol: float) -> int:
    """B and X: complex128 GPU tensors [nrhs][2 N^2]; B must not change and X
    must not be read until the request finishes (the caller keeps both alive)."""
    import torch
    torch.cuda.current_stream().synchronize()  # B complete before the server's streams read it
    rid = ctypes.c_int64()
    _check(lib.bamg_server_submit(s, int(field), _ptr(B), _ptr(X), int(nrhs), float(tol), ctypes.byref(rid)),
           "bamg_server_submit")
    return rid.value


def bamg_server_progress(s) -> int:
    pend = ctypes.c_int32()
    _check(lib.bamg_server_progress(s, ctypes.byref(pend)), "bamg_server_progress")
    return pend.value


def bamg_server_wait(s, request: int, nrhs: int, timeout_ms: float = -1.0):
    """(status, infos) once finished, (BAMG_PENDING, None) otherwise.  Failure
    statuses are returned, not raised, so that a failed request can be told
    apart from a failed call."""
    infos = (bamg_solve_info * nrhs)()
    st = lib.bamg_server_wait(s, ctypes.c_int64(request), float(timeout_ms), infos)
    if st == BAMG_PENDING:
        return st, None
    return st, [i.as_dict() for i in infos]


def bamg_server_get_stats(s) -> dict:
    st = bamg_server_stats()
    _check(lib.bamg_server_get_stats(s, ctypes.byref(st)), "bamg_server_get_stats")
    return st.as_dict()


def bamg_server_reset_stats(s):
    _check(lib.bamg_server_reset_stats(s), "bamg_server_reset_stats")


def bamg_server_free(s):
    if s is not None and s.value:
        lib.bamg_server_free(s)
        s.value = None

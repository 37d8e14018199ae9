"""ctypes binding of the C ABI in include/sg.h (argument marshalling only).

Every computation runs in the HIP library libsgkkt.so built in this package
directory; importing this module fails loudly when the library is missing.
Device vectors are passed as torch CUDA tensors (or raw device addresses).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgkkt.so")

SG_OK, SG_PENDING, SG_NOT_CONVERGED = 0, 1, 2
SG_ERR_INVALID, SG_ERR_NONCOERCIVE, SG_ERR_NONFINITE = -1, -2, -3
SG_ERR_NOMEM, SG_ERR_HIP, SG_ERR_CANCELLED, SG_ERR_UNKNOWN = -4, -5, -6, -7
SG_FP64, SG_FP32 = 0, 1
SG_PREC_FP64, SG_PREC_FP32_REFINE, SG_PREC_FP32_PRECOND = 0, 1, 2
SG_PROF_NONE, SG_PROF_KKT_APPLY, SG_PROF_MG_SMOOTH, SG_PROF_MULTIDOT, SG_PROF_HGS_RHS = 0, 1, 2, 3, 4
SG_PROF_ARNOLDI_UPD, SG_PROF_MG_TAIL, SG_PROF_MASS_CHEB, SG_PROF_MG_UP = 5, 6, 7, 8
SG_ARNOLDI_DCGS2, SG_ARNOLDI_CGS2 = 0, 1
SG_MEAN_MULTIGRID, SG_MEAN_EXACT = 0, 1
SG_FIELD_AFFINE, SG_FIELD_LOGNORMAL = 0, 1
SG_PRECOND_BLOCK_DIAGONAL, SG_PRECOND_HGSOC = 0, 1

_DP = C.POINTER(C.c_double)


class sg_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("M", C.c_int32), ("P", C.c_int32), ("n_t", C.c_int32),
                ("T", C.c_double), ("beta", C.c_double), ("gamma", C.c_double), ("sigma", C.c_double),
                ("kappa", _DP), ("y_target", _DP), ("y0", _DP), ("field", C.c_int32), ("corr_len", C.c_double)]


class sg_options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("cheb_steps", C.c_int32), ("truncation_r", C.c_int32), ("gmg_pre", C.c_int32),
                ("gmg_post", C.c_int32), ("precision", C.c_int32), ("inner_rtol", C.c_double),
                ("use_graphs", C.c_int32), ("verbose", C.c_int32), ("profile", C.c_int32),
                ("arnoldi", C.c_int32), ("sweep_rows", C.c_int32), ("basis_fp32", C.c_int32),
                ("mean_solver", C.c_int32), ("richardson_steps", C.c_int32), ("precond", C.c_int32)]


class sg_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_refinements", C.c_int32), ("converged", C.c_int32),
                ("status", C.c_int32), ("rel_res_true", C.c_double), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("latency_ms", C.c_double), ("bytes_moved", C.c_double),
                ("prof_ms", C.c_double), ("prof_bytes", C.c_double), ("prof_launches", C.c_int32),
                ("joined_batch", C.c_int32)]


class sg_sizes(C.Structure):
    _fields_ = [("n", C.c_int32), ("M", C.c_int32), ("P", C.c_int32), ("n_t", C.c_int32),
                ("n_xi", C.c_int32), ("members", C.c_int32), ("nodes", C.c_int64),
                ("block_elems", C.c_int64), ("kkt_elems", C.c_int64), ("level_offsets", C.c_int32 * 17),
                ("sweep_rows", (C.c_int32 * 3) * 2)]


# Every exported symbol of include/sg.h with (restype, argtypes).
SIGNATURES = {
    "sg_default_options": (None, [C.POINTER(sg_options)]),
    "sg_validate": (C.c_int, [C.POINTER(sg_problem), C.POINTER(sg_options)]),
    "sg_setup": (C.c_int, [C.POINTER(sg_problem), C.c_int32, C.POINTER(sg_options), C.c_void_p,
                           C.POINTER(C.c_void_p)]),
    "sg_query": (C.c_int, [C.c_void_p, C.POINTER(sg_sizes)]),
    "sg_get_multiindex": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "sg_get_gtable": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), _DP]),
    "sg_get_rhs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sg_apply_operator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "sg_apply_kkt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "sg_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "sg_precond_apply_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                           C.c_void_p]),
    "sg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(sg_solve_info)]),
    "sg_destroy": (None, [C.c_void_p]),
    "sg_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "sg_submit": (C.c_int, [C.c_void_p, C.POINTER(sg_problem), C.POINTER(sg_options), _DP,
                            C.POINTER(C.c_uint64)]),
    "sg_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(sg_solve_info)]),
    "sg_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "sg_server_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), _DP, _DP, _DP]),
    "sg_server_destroy": (None, [C.c_void_p]),
    "sg_tune_save": (C.c_int, [C.c_char_p]),
    "sg_tune_load": (C.c_int, [C.c_char_p]),
    "sg_tune_count": (C.c_int, []),
    "sg_tune_clear": (C.c_int, []),
    "sg_last_error": (C.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run `python paper_2512_23804_amd/build.py`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class SGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc: int, allow=(SG_OK,)) -> int:
    if rc not in allow:
        raise SGError(rc, lib.sg_last_error().decode())
    return rc


def default_options(**kw) -> sg_options:
    o = sg_options()
    lib.sg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def tune_save(path: str) -> None:
    """Write the strip-height autotuner's cached choices to a text file."""
    check(lib.sg_tune_save(os.fsencode(path)))


def tune_load(path: str) -> None:
    """Merge a file written by tune_save into the autotuner's cache."""
    check(lib.sg_tune_load(os.fsencode(path)))


def tune_count() -> int:
    rc = lib.sg_tune_count()
    if rc < 0:
        check(rc)
    return rc


def tune_clear() -> None:
    check(lib.sg_tune_clear())


def _dptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


class ProblemData:
    """Host-side problem holder that keeps the arrays alive for the C struct."""

    def __init__(self, n, M, P, sigma, beta, y_target, gamma=0.0, n_t=1, T=1.0, kappa=None, y0=None,
                 field=0, corr_len=1.0):
        self.y_target = np.ascontiguousarray(y_target, dtype=np.float64)
        self.kappa = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
        self.y0 = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
        self.c = sg_problem(int(n), int(M), int(P), int(n_t), float(T), float(beta), float(gamma), float(sigma),
                            _dptr(self.kappa), _dptr(self.y_target), _dptr(self.y0), int(field), float(corr_len))


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return SG_FP64
    if t.dtype == torch.float32:
        return SG_FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


def validate(problem: ProblemData, options: sg_options | None = None) -> int:
    return lib.sg_validate(C.byref(problem.c), C.byref(options) if options is not None else None)


class Handle:
    """A batch of same-shape problems set up on the current device."""

    def __init__(self, problems, options: sg_options | None = None, stream=None):
        if isinstance(problems, ProblemData):
            problems = [problems]
        self._problems = problems
        arr = (sg_problem * len(problems))(*[p.c for p in problems])
        self._opts = options if options is not None else default_options()
        h = C.c_void_p()
        check(lib.sg_setup(arr, len(problems), C.byref(self._opts), _stream_ptr(stream), C.byref(h)))
        self._h = h
        sz = sg_sizes()
        check(lib.sg_query(self._h, C.byref(sz)))
        self.sizes = sz
        self.n_xi = sz.n_xi
        self.members = sz.members
        self.block_elems = sz.block_elems
        self.kkt_elems = sz.kkt_elems
        self.level_offsets = list(sz.level_offsets[: sz.P + 2])

    def close(self):
        if self._h:
            lib.sg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def multiindex(self) -> np.ndarray:
        out = np.zeros((self.n_xi, self.sizes.M), dtype=np.int32)
        check(lib.sg_get_multiindex(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def gtable(self):
        idx = np.zeros((self.n_xi, self.sizes.M, 2), dtype=np.int32)
        val = np.zeros((self.n_xi, self.sizes.M, 2), dtype=np.float64)
        check(lib.sg_get_gtable(self._h, idx.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(val)))
        return idx, val

    def rhs(self, out):
        check(lib.sg_get_rhs(self._h, _ptr(out)))
        return out

    def _nvec(self, t, per):
        n = t.numel()
        if n % per:
            raise ValueError("tensor size is not a whole number of vectors")
        return n // per

    def apply_operator(self, x, y, stream=None):
        check(lib.sg_apply_operator(self._h, _ptr(x), _ptr(y), self._nvec(x, self.block_elems), _dtype_code(x),
                                    _stream_ptr(stream)))
        return y

    def apply_kkt(self, x, y, stream=None):
        check(lib.sg_apply_kkt(self._h, _ptr(x), _ptr(y), self._nvec(x, self.kkt_elems), _dtype_code(x),
                               _stream_ptr(stream)))
        return y

    def precond_apply(self, r, z, stream=None):
        check(lib.sg_precond_apply(self._h, _ptr(r), _ptr(z), self._nvec(r, self.kkt_elems), _dtype_code(r),
                                   _stream_ptr(stream)))
        return z

    def precond_apply_noalloc(self, r, z, stream=None, allow=(SG_OK,)):
        """sg_precond_apply_noalloc: the preconditioner with the library's fixed
        device scratch (no device allocation); returns the status code."""
        return check(lib.sg_precond_apply_noalloc(self._h, _ptr(r), _ptr(z), self._nvec(r, self.kkt_elems),
                                                  _dtype_code(r), _stream_ptr(stream)), allow=allow)

    def solve(self, x, b=None):
        infos = (sg_solve_info * self.members)()
        rc = check(lib.sg_solve(self._h, _ptr(b), _ptr(x), infos), allow=(SG_OK, SG_NOT_CONVERGED))
        return rc, [infos[i] for i in range(self.members)]


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Server:
    """Continuous-batching solve server (sg_server_*)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 64):
        s = C.c_void_p()
        check(lib.sg_server_create(hbm_budget_bytes, max_slots, C.byref(s)))
        self._s = s
        self._keep = {}

    def submit(self, problem: ProblemData, out: np.ndarray, options: sg_options | None = None) -> int:
        t = C.c_uint64()
        opts = options if options is not None else default_options()
        check(lib.sg_submit(self._s, C.byref(problem.c), C.byref(opts), _dptr(out), C.byref(t)))
        self._keep[t.value] = (problem, out, opts)
        return t.value

    def poll(self, ticket: int):
        info = sg_solve_info()
        rc = lib.sg_poll(self._s, ticket, C.byref(info))
        return rc, info

    def cancel(self, ticket: int) -> int:
        return lib.sg_cancel(self._s, ticket)

    def stats(self):
        n = C.c_int64()
        p50, p99, sps = C.c_double(), C.c_double(), C.c_double()
        check(lib.sg_server_stats(self._s, C.byref(n), C.byref(p50), C.byref(p99), C.byref(sps)))
        return dict(completed=n.value, p50_ms=p50.value, p99_ms=p99.value, solves_per_s=sps.value)

    def close(self):
        if self._s:
            lib.sg_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

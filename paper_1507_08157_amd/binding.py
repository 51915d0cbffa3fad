"""ctypes binding of libtddft (include/tddft.h).  Argument marshalling only: every step of
the computation runs in the HIP library.  Device arrays are torch tensors on the current
GPU; the library is loaded from this directory and its absence is an error."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtddft.so")

TDDFT_OK = 0
TDDFT_E_INVALID = -1
TDDFT_E_NOMEM = -2
TDDFT_E_DEVICE = -3
TDDFT_E_NOT_PD = -4
TDDFT_E_NO_CONVERGENCE = -5
TDDFT_W_FALLBACK = 1

TDDFT_FP64, TDDFT_FP32, TDDFT_BF16_GRID = 0, 1, 2
TDDFT_XC_ALDA_X, TDDFT_XC_NONE, TDDFT_HXC_NONE = 0, 1, 2
TDDFT_PC_NONE, TDDFT_PC_KSDIFF_CG, TDDFT_PC_LEARNED = 0, 1, 2

PRECISION = {"fp64": TDDFT_FP64, "fp32": TDDFT_FP32, "bf16": TDDFT_BF16_GRID}

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class tddft_bsr(C.Structure):
    _fields_ = [("nbr", C.c_int32), ("nbc", C.c_int32), ("row_off", _i32p), ("col_off", _i32p),
                ("rowptr", _i64p), ("colind", _i32p), ("val", _f64p)]


class tddft_functions(C.Structure):
    _fields_ = [("n_fn", C.c_int32), ("origin", _i32p), ("extent", _i32p), ("off", _i64p),
                ("val", _f64p)]


class tddft_system(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("occ", tddft_functions),
                ("vir", tddft_functions), ("S_o", tddft_bsr), ("H_o", tddft_bsr),
                ("K_v", tddft_bsr), ("S_u", tddft_bsr), ("H_u", tddft_bsr),
                ("K_c", tddft_bsr), ("M", tddft_bsr)]


class tddft_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("xc", C.c_int32), ("rho_floor", C.c_double),
                ("coupling_scale", C.c_double), ("precond", C.c_int32),
                ("eps_tol", C.c_double), ("tol_omega", C.c_double), ("max_iter", C.c_int32),
                ("max_inner", C.c_int32), ("refresh", C.c_int32), ("restart", C.c_int32),
                ("seed", C.c_uint64), ("model", C.c_void_p), ("model_bytes", C.c_int64),
                ("stream", C.c_void_p), ("eps_loose", C.c_double), ("tda", C.c_int32),
                ("truncate_p", C.c_int32), ("graphs", C.c_int32), ("autotune", C.c_int32),
                ("density_pbcast", C.c_int32), ("gemm_tile", C.c_int32),
                ("sparse_cw", C.c_int32), ("sparse_pairs", C.c_int32)]


class tddft_info(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("tiles", C.c_int32), ("block_rows", C.c_int32),
                ("block_cols", C.c_int32), ("max_rows_o", C.c_int32), ("precision", C.c_int32),
                ("sample_rows_u", C.c_int64), ("sample_rows_o", C.c_int64),
                ("pair_points", C.c_int64), ("blocks_m", C.c_int64), ("blocks_r", C.c_int64),
                ("blocks_o", C.c_int64),
                ("blocks_m2", C.c_int64), ("blocks_m3", C.c_int64), ("blocks_m4", C.c_int64),
                ("pairs_kshift", C.c_int64), ("pairs_project", C.c_int64),
                ("pairs_project_t", C.c_int64),
                ("pairs_covariant", C.c_int64), ("pairs_sandwich", C.c_int64),
                ("partial_pairs", C.c_int64), ("setup_ms", C.c_double),
                ("samples_u_nz", C.c_int64), ("samples_o_nz", C.c_int64),
                ("pair_points_nz", C.c_int64), ("fft_threads", C.c_int32 * 3),
                ("density_waves", C.c_int32), ("kshift_cw", C.c_int32 * 2),
                ("density_pbcast", C.c_int32), ("kshift_tile", C.c_int32 * 2),
                ("kshift_pairs", C.c_int32 * 2)]


class tddft_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("inner_total", C.c_int32), ("applies", C.c_int32), ("fallbacks", C.c_int32),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("apply_ms", C.c_double),
                ("log_capacity", C.c_int32), ("log_len", C.c_int32), ("log_omega", _f64p),
                ("log_time_ms", _f64p), ("log_gnorm", _f64p), ("graph_replays", C.c_int32)]


_LIB = None

EXPORTS = ("tddft_default_options", "tddft_create", "tddft_nnz_p", "tddft_response_pattern",
           "tddft_apply",
           "tddft_pcg_solve", "tddft_destroy", "tddft_strerror", "tddft_last_error",
           "tddft_abi_version", "tddft_get_info", "tddft_profile", "tddft_profile_read",
           "tddft_profile_stage_name", "tddft_project", "tddft_precondition",
           "tddft_n_features", "tddft_block_features", "tddft_guess_targets",
           "tddft_mlp_create", "tddft_mlp_destroy", "tddft_mlp_n_params", "tddft_mlp_set_params",
           "tddft_mlp_get_params", "tddft_mlp_fit_normalisation", "tddft_mlp_forward",
           "tddft_mlp_train_step", "tddft_mlp_export", "tddft_mlp_import",
           "tddft_mlp_last_error", "tddft_pcg_solve_batched", "tddft_apply_noalloc",
           "tddft_apply_noalloc_limit", "tddft_oscillator_strengths")


def lib():
    """Load libtddft.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtddft.so not built ({LIB_PATH}); run "
                               "python -m paper_1507_08157_amd.build")
        # PyTorch's HIP runtime must be the process's only one: load it first so the
        # library binds to the same libamdhip64 / libhsa-runtime64
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        L.tddft_default_options.argtypes = [C.POINTER(tddft_options)]
        L.tddft_default_options.restype = None
        L.tddft_create.argtypes = [C.POINTER(tddft_system), C.POINTER(tddft_options),
                                   C.POINTER(C.c_void_p)]
        L.tddft_create.restype = C.c_int
        L.tddft_nnz_p.argtypes = [C.c_void_p]
        L.tddft_nnz_p.restype = C.c_int64
        L.tddft_response_pattern.argtypes = [C.c_void_p, _i64p, _i32p]
        L.tddft_response_pattern.restype = C.c_int64
        L.tddft_apply.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]
        L.tddft_apply.restype = C.c_int
        L.tddft_pcg_solve.argtypes = [C.c_void_p, C.c_int32, C.POINTER(tddft_options), _f64p,
                                      C.c_void_p, C.c_void_p, C.POINTER(tddft_stats)]
        L.tddft_pcg_solve.restype = C.c_int
        L.tddft_destroy.argtypes = [C.c_void_p]
        L.tddft_destroy.restype = None
        L.tddft_strerror.argtypes = [C.c_int]
        L.tddft_strerror.restype = C.c_char_p
        L.tddft_last_error.argtypes = [C.c_void_p]
        L.tddft_last_error.restype = C.c_char_p
        L.tddft_abi_version.argtypes = []
        L.tddft_abi_version.restype = C.c_int
        L.tddft_get_info.argtypes = [C.c_void_p, C.POINTER(tddft_info)]
        L.tddft_get_info.restype = C.c_int
        L.tddft_profile.argtypes = [C.c_void_p, C.c_int]
        L.tddft_profile.restype = C.c_int
        L.tddft_profile_read.argtypes = [C.c_void_p, C.c_int, _f64p, _i64p]
        L.tddft_profile_read.restype = C.c_int
        L.tddft_profile_stage_name.argtypes = [C.c_int]
        L.tddft_profile_stage_name.restype = C.c_char_p
        vp = C.c_void_p
        for name, args, res in (
                ("tddft_project", [vp, C.c_int32, vp, vp], C.c_int),
                ("tddft_precondition", [vp, C.c_int32, vp, vp, C.c_double, C.c_int32], C.c_int),
                ("tddft_n_features", [vp], C.c_int32),
                ("tddft_block_features", [vp, vp], C.c_int),
                ("tddft_guess_targets", [vp, C.c_int32, vp, vp], C.c_int),
                ("tddft_mlp_create", [C.c_int32, C.c_int32, C.c_int32, C.c_uint64, vp,
                                      C.POINTER(C.c_void_p)], C.c_int),
                ("tddft_mlp_destroy", [vp], None),
                ("tddft_mlp_n_params", [vp], C.c_int64),
                ("tddft_mlp_set_params", [vp, vp, vp, vp], C.c_int),
                ("tddft_mlp_get_params", [vp, vp, vp, vp], C.c_int),
                ("tddft_mlp_fit_normalisation", [vp, C.c_int64, vp], C.c_int),
                ("tddft_mlp_forward", [vp, C.c_int64, vp, vp], C.c_int),
                ("tddft_mlp_train_step", [vp, C.c_int64, vp, vp, vp, vp, C.c_double,
                                          C.c_double, C.POINTER(C.c_double), vp], C.c_int),
                ("tddft_mlp_export", [vp, vp, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
                ("tddft_mlp_import", [vp, C.c_int64, vp, C.POINTER(C.c_void_p)], C.c_int),
                ("tddft_mlp_last_error", [vp], C.c_char_p),
                ("tddft_apply_noalloc", [vp, C.c_int32, vp, vp, vp, vp], C.c_int),
                ("tddft_apply_noalloc_limit", [], C.c_int64),
                ("tddft_oscillator_strengths", [vp, C.c_int32, _f64p, vp, _f64p, _f64p], C.c_int),
                ("tddft_pcg_solve_batched", [C.POINTER(C.c_void_p), C.c_int32, _i32p,
                                             C.POINTER(tddft_options), C.POINTER(_f64p),
                                             C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                             C.POINTER(tddft_stats), _i32p, C.c_int32], C.c_int)):
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


class TddftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} [{code}]")
        self.code = code


PRECOND = {"none": 0, "cg": 1, "learned": 2}


def tddft_default_options(**kw) -> tddft_options:
    """Options with library defaults, then keyword overrides.  precision and precond take
    names ("fp32", "learned", ...); model takes the bytes of a model blob (kept alive by
    the returned options object)."""
    o = tddft_options()
    lib().tddft_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "precond" and isinstance(v, str):
            v = PRECOND[v]
        if k == "model":
            buf = C.create_string_buffer(bytes(v), len(v))
            o._model_buf = buf
            o.model = C.cast(buf, C.c_void_p)
            o.model_bytes = len(v)
            continue
        setattr(o, k, v)
    return o


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _bsr(d, keep):
    b = tddft_bsr()
    b.nbr, b.nbc = int(d["nbr"]), int(d["nbc"])
    for k, ct in (("row_off", C.c_int32), ("col_off", C.c_int32), ("rowptr", C.c_int64),
                  ("colind", C.c_int32)):
        arr = np.ascontiguousarray(d[k], dtype=np.dtype(ct))
        keep.append(arr)
        setattr(b, k, _ptr(arr, ct))
    if d.get("val") is not None:
        v = np.ascontiguousarray(d["val"], dtype=np.float64)
        keep.append(v)
        b.val = _ptr(v, C.c_double)
    return b


def _fns(d, keep):
    f = tddft_functions()
    f.n_fn = int(d["n_fn"])
    for k, ct in (("origin", C.c_int32), ("extent", C.c_int32), ("off", C.c_int64),
                  ("val", C.c_double)):
        arr = np.ascontiguousarray(d[k], dtype=np.dtype(ct))
        keep.append(arr)
        setattr(f, k, _ptr(arr, ct))
    return f


def _system(arrays: dict, keep: list) -> tddft_system:
    s = tddft_system()
    for d in range(3):
        s.n[d] = int(arrays["n"][d])
        s.L[d] = float(arrays["L"][d])
    s.occ = _fns(arrays["occ"], keep)
    s.vir = _fns(arrays["vir"], keep)
    for k in ("S_o", "H_o", "K_v", "S_u", "H_u", "K_c", "M"):
        setattr(s, k, _bsr(arrays[k], keep))
    return s


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Handle:
    """Owner of one tddft_handle (tddft_create ... tddft_destroy)."""

    def __init__(self, arrays: dict, options: tddft_options | None = None, **kw):
        self._h = C.c_void_p()
        self.options = options if options is not None else tddft_default_options(**kw)
        keep: list = []
        sysc = _system(arrays, keep)
        self._nbu = int(arrays["S_u"]["nbr"])
        rc = lib().tddft_create(C.byref(sysc), C.byref(self.options), C.byref(self._h))
        if rc != TDDFT_OK:
            raise TddftError(rc, lib().tddft_last_error(None).decode())
        self.nnz_p = int(lib().tddft_nnz_p(self._h))

    def close(self):
        if self._h:
            lib().tddft_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        return TddftError(rc, lib().tddft_last_error(self._h).decode())

    def tddft_apply(self, Pp, Pq, fp=None, fq=None):
        """(f_p, f_q) for device tensors [n_states, nnz_p] FP64 (response-pattern layout)."""
        import torch
        n = Pp.shape[0]
        fp = torch.empty_like(Pp) if fp is None else fp
        fq = torch.empty_like(Pq) if fq is None else fq
        rc = lib().tddft_apply(self._h, n, _dev(Pp, "Pp"), _dev(Pq, "Pq"), _dev(fp, "fp"),
                               _dev(fq, "fq"))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return fp, fq

    def tddft_apply_noalloc(self, Pp, Pq, fp, fq):
        """tddft_apply through the library's per-GPU workspace (no device allocation);
        fp and fq must be given."""
        rc = lib().tddft_apply_noalloc(self._h, Pp.shape[0], _dev(Pp, "Pp"), _dev(Pq, "Pq"),
                                       _dev(fp, "fp"), _dev(fq, "fq"))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return fp, fq

    def tddft_oscillator_strengths(self, omega, Pp):
        """(f [n], transition moments [n, 3]) of converged vectors Pp (device tensor)."""
        w = np.ascontiguousarray(omega, dtype=np.float64)
        n = len(w)
        f = np.zeros(n)
        D = np.zeros((n, 3))
        rc = lib().tddft_oscillator_strengths(self._h, n, _ptr(w, C.c_double), _dev(Pp, "Pp"),
                                              _ptr(f, C.c_double), _ptr(D, C.c_double))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return f, D

    def tddft_project(self, L, P=None):
        """Pi(L) (Eq. auxiliary) for device tensors [n_states, nnz_p] FP64."""
        import torch
        P = torch.empty_like(L) if P is None else P
        rc = lib().tddft_project(self._h, L.shape[0], _dev(L, "L"), _dev(P, "P"))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return P

    def tddft_precondition(self, g, eps_tol=1e-4, max_inner=50, G=None):
        """Eq. precond solved by CG in the S metric for device tensors [n_states, nnz_p]."""
        import torch
        G = torch.empty_like(g) if G is None else G
        rc = lib().tddft_precondition(self._h, g.shape[0], _dev(g, "g"), _dev(G, "G"),
                                      float(eps_tol), int(max_inner))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return G

    def tddft_block_features(self):
        """[blocks of R, n_features] FP32 device tensor."""
        import torch
        nf = int(lib().tddft_n_features(self._h))
        nb = int(lib().tddft_response_pattern(self._h, None, None))
        out = torch.empty((nb, nf), dtype=torch.float32, device="cuda")
        rc = lib().tddft_block_features(self._h, C.c_void_p(out.data_ptr()))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return out

    def tddft_guess_targets(self, Pq):
        import torch
        nb = int(lib().tddft_response_pattern(self._h, None, None))
        t = torch.empty(nb, dtype=torch.float32, device="cuda")
        rc = lib().tddft_guess_targets(self._h, Pq.shape[0], _dev(Pq, "Pq"),
                                       C.c_void_p(t.data_ptr()))
        if rc != TDDFT_OK:
            raise self._err(rc)
        return t

    def tddft_response_pattern(self):
        """(rowptr, colind) of the response pattern R (numpy arrays)."""
        nb = int(lib().tddft_response_pattern(self._h, None, None))
        rowptr = np.zeros(self._nbu + 1, dtype=np.int64)
        colind = np.zeros(nb, dtype=np.int32)
        lib().tddft_response_pattern(self._h, _ptr(rowptr, C.c_int64), _ptr(colind, C.c_int32))
        return rowptr, colind

    def tddft_get_info(self) -> dict:
        inf = tddft_info()
        rc = lib().tddft_get_info(self._h, C.byref(inf))
        if rc != TDDFT_OK:
            raise self._err(rc)
        d = {k: getattr(inf, k) for k, _ in tddft_info._fields_}
        d["n"] = list(inf.n)
        d["fft_threads"] = list(inf.fft_threads)
        d["kshift_cw"] = list(inf.kshift_cw)
        d["kshift_tile"] = list(inf.kshift_tile)
        d["kshift_pairs"] = list(inf.kshift_pairs)
        return d

    def tddft_profile(self, enable: bool):
        rc = lib().tddft_profile(self._h, 1 if enable else 0)
        if rc != TDDFT_OK:
            raise self._err(rc)

    def tddft_profile_read(self) -> dict:
        """{stage name: (milliseconds, executions)} accumulated since profiling was enabled."""
        ms = np.zeros(64)
        cnt = np.zeros(64, dtype=np.int64)
        k = lib().tddft_profile_read(self._h, 64, _ptr(ms, C.c_double), _ptr(cnt, C.c_int64))
        if k < 0:
            raise self._err(k)
        return {tddft_profile_stage_name(i): (float(ms[i]), int(cnt[i])) for i in range(k)}

    def tddft_pcg_solve(self, n_states, options=None, Pp=None, Pq=None, log_capacity=0,
                        raise_on_noconv=False):
        """Returns (omega ndarray, status, stats dict); Pp/Pq updated in place if given."""
        omega = np.zeros(n_states)
        st = tddft_stats()
        logs = {}
        if log_capacity:
            logs["omega"] = np.zeros(log_capacity * n_states)
            logs["t"] = np.zeros(log_capacity)
            logs["g"] = np.zeros(log_capacity)
            st.log_capacity = log_capacity
            st.log_omega = _ptr(logs["omega"], C.c_double)
            st.log_time_ms = _ptr(logs["t"], C.c_double)
            st.log_gnorm = _ptr(logs["g"], C.c_double)
        opt = C.byref(options) if options is not None else None
        pp = _dev(Pp, "Pp") if Pp is not None else None
        pq = _dev(Pq, "Pq") if Pq is not None else None
        rc = lib().tddft_pcg_solve(self._h, n_states, opt, _ptr(omega, C.c_double), pp, pq,
                                   C.byref(st))
        if rc < 0 and (rc != TDDFT_E_NO_CONVERGENCE or raise_on_noconv):
            raise self._err(rc)
        k = st.log_len
        stats = dict(iterations=st.iterations, converged=bool(st.converged),
                     inner_total=st.inner_total, applies=st.applies, fallbacks=st.fallbacks,
                     setup_ms=st.setup_ms, solve_ms=st.solve_ms, apply_ms=st.apply_ms,
                     graph_replays=st.graph_replays)
        if log_capacity:
            stats["log_omega"] = logs["omega"][:k * n_states].reshape(k, n_states)
            stats["log_time_ms"] = logs["t"][:k]
            stats["log_gnorm"] = logs["g"][:k]
        return omega, rc, stats


def tddft_pcg_solve_batched(handles, n_states, options=None, Pp=None, Pq=None,
                            max_workers=0):
    """Solve several systems concurrently; returns [(omega, status, stats dict)] per system.
    Pp / Pq: None or lists of device tensors (per-system initial and returned vectors)."""
    import torch
    n = len(handles)
    hs = (C.c_void_p * n)(*[h._h for h in handles])
    ns = np.ascontiguousarray(n_states, dtype=np.int32)
    omegas = [np.zeros(int(k)) for k in ns]
    om = (_f64p * n)(*[_ptr(w, C.c_double) for w in omegas])
    pp = (C.c_void_p * n)(*[_dev(t, "Pp").value for t in Pp]) if Pp is not None else None
    pq = (C.c_void_p * n)(*[_dev(t, "Pq").value for t in Pq]) if Pq is not None else None
    st = (tddft_stats * n)()
    status = np.zeros(n, dtype=np.int32)
    opt = C.byref(options) if options is not None else None
    torch.cuda.synchronize()
    rc = lib().tddft_pcg_solve_batched(hs, n, _ptr(ns, C.c_int32), opt, om, pp, pq, st,
                                       _ptr(status, C.c_int32), int(max_workers))
    if rc != TDDFT_OK:
        raise TddftError(rc, "tddft_pcg_solve_batched: invalid arguments")
    out = []
    for k in range(n):
        s = st[k]
        out.append((omegas[k], int(status[k]),
                    dict(iterations=s.iterations, converged=bool(s.converged),
                         inner_total=s.inner_total, applies=s.applies, fallbacks=s.fallbacks,
                         setup_ms=s.setup_ms, solve_ms=s.solve_ms, apply_ms=s.apply_ms,
                         graph_replays=s.graph_replays)))
    return out


def tddft_profile_stage_name(k: int):
    r = lib().tddft_profile_stage_name(k)
    return r.decode() if r is not None else None


def tddft_create(arrays: dict, options: tddft_options | None = None, **kw) -> Handle:
    return Handle(arrays, options, **kw)


def tddft_apply_noalloc_limit() -> int:
    return int(lib().tddft_apply_noalloc_limit())


def tddft_abi_version() -> int:
    return int(lib().tddft_abi_version())


def tddft_strerror(code: int) -> str:
    return lib().tddft_strerror(code).decode()


def _f32dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Mlp:
    """The learned preconditioner's network (tddft_mlp_*)."""

    def __init__(self, n_in=None, width=128, n_out=None, seed=0, blob: bytes | None = None):
        self._m = C.c_void_p()
        if blob is not None:
            buf = C.create_string_buffer(bytes(blob), len(blob))
            rc = lib().tddft_mlp_import(buf, len(blob), None, C.byref(self._m))
        else:
            rc = lib().tddft_mlp_create(n_in, width, n_out, seed, None, C.byref(self._m))
        if rc != TDDFT_OK:
            raise TddftError(rc, lib().tddft_last_error(None).decode())
        self.n_params = int(lib().tddft_mlp_n_params(self._m))

    def close(self):
        if self._m:
            lib().tddft_mlp_destroy(self._m)
            self._m = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != TDDFT_OK:
            raise TddftError(rc, lib().tddft_mlp_last_error(self._m).decode())

    def set_params(self, params=None, mean=None, std=None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        mu = None if mean is None else np.ascontiguousarray(mean, dtype=np.float32)
        sd = None if std is None else np.ascontiguousarray(std, dtype=np.float32)
        f = C.POINTER(C.c_float)
        self._check(lib().tddft_mlp_set_params(
            self._m, None if p is None else p.ctypes.data_as(f),
            None if mu is None else mu.ctypes.data_as(f), None if sd is None else sd.ctypes.data_as(f)))

    def get_params(self, n_in):
        p = np.zeros(self.n_params, dtype=np.float32)
        mu = np.zeros(n_in, dtype=np.float32)
        sd = np.zeros(n_in, dtype=np.float32)
        f = C.POINTER(C.c_float)
        self._check(lib().tddft_mlp_get_params(self._m, p.ctypes.data_as(f), mu.ctypes.data_as(f),
                                               sd.ctypes.data_as(f)))
        return p, mu, sd

    def fit_normalisation(self, X):
        self._check(lib().tddft_mlp_fit_normalisation(self._m, X.shape[0], _f32dev(X, "X")))

    def forward(self, X, n_out):
        import torch
        Y = torch.empty((X.shape[0], n_out), dtype=torch.float32, device="cuda")
        self._check(lib().tddft_mlp_forward(self._m, X.shape[0], _f32dev(X, "X"), _f32dev(Y, "Y")))
        return Y

    def train_step(self, X, g, gstar, t, loss_scale=1.0, lr=1e-3, want_grad=False):
        import torch
        loss = C.c_double(0.0)
        grad = torch.empty(self.n_params, dtype=torch.float32, device="cuda") if want_grad else None
        self._check(lib().tddft_mlp_train_step(
            self._m, X.shape[0], _f32dev(X, "X"), _f32dev(g, "g"), _f32dev(gstar, "gstar"),
            _f32dev(t, "t"), float(loss_scale), float(lr), C.byref(loss),
            _f32dev(grad, "grad") if want_grad else None))
        return (loss.value, grad) if want_grad else loss.value

    def export(self) -> bytes:
        size = C.c_int64(0)
        self._check(lib().tddft_mlp_export(self._m, None, 0, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._check(lib().tddft_mlp_export(self._m, buf, size.value, C.byref(size)))
        return buf.raw

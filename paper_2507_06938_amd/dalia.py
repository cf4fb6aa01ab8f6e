"""Thin ctypes binding of libdalia_hip.so.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors on a ROCm
device) and the current stream.  If the shared library is missing this
module raises at import-time use; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdalia_hip.so")

DL_QP, DL_QC, DL_BOTH = 0, 1, 2
DL_WS_SELINV, DL_WS_KEEP_QP, DL_WS_GRAPH, DL_WS_MIXED = 1, 2, 4, 8
DL_WS_SPLITK = 16
DL_WS_TWOSIDED = 32
DL_WS_FOLD_INV = 64
DL_WS_WARM_START = 128
DL_WS_DAG = 256
DL_INFO_TIMEOUT = -2
# refinement of the mean (see include/dalia.h)
DL_REFINE_TOL = 1e-12
DL_REFINE_MAX = 10
DL_REFINE_STEPS_GRAPH = 3
DL_INFO_NOTCONV = -1
DL_ENOTCONV = 6
DL_WAVE_RESERVE = 256 << 20
CATEGORIES = ("potrf_tile", "panel_trsm", "panel_syrk", "trtri", "trsm",
              "update", "solve", "selinv", "assemble", "other")
KERNELS = ("k_gemm_tasks", "k_potrf_tile", "gemv", "k_assemble", "other",
           "k_panel_update", "k_gemm_reduce", "k_dag_chol")
STATUS = {0: "ok", 1: "invalid argument", 2: "device allocation failed",
          3: "not positive definite", 4: "HIP runtime error",
          5: "call order violated", 6: "refinement did not converge"}

PARTS_FIELDS = ("f", "logdet_p", "logdet_c", "quad_p", "quad_obs",
                "log_prior", "log_lik_const", "rel_residual")


class DaliaError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({code})")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nt", C.c_int32), ("nv", C.c_int32),
                ("nr", C.c_int32), ("m", C.c_int64 * 3),
                ("obs_t", C.c_void_p * 3), ("obs_nodes", C.c_void_p * 3),
                ("obs_w", C.c_void_p * 3), ("obs_x", C.c_void_p * 3),
                ("y", C.c_void_p * 3), ("theta_prior_mean", C.c_void_p),
                ("theta_prior_sd", C.c_double), ("prior_fixed", C.c_double),
                ("family", C.c_int32), ("likelihood", C.c_int32)]


MODEL_FAMILIES = {"separable": 0, "diffusion": 1}
LIKELIHOODS = {"gaussian": 0, "poisson": 1}


_lib = None


def lib():
    """Load the shared library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2507_06938_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "dl_theta_dim": (i32, [i32]),
            "dl_theta_dim_lik": (i32, [i32, i32]),
            "dl_ws_newton_steps": (i32, [vp, C.POINTER(i32)]),
            "dl_model_create": (i32, [vp, C.POINTER(vp)]),
            "dl_model_destroy": (None, [vp]),
            "dl_model_dims": (i32, [vp] + [C.POINTER(i64)] * 5),
            "dl_ws_create": (i32, [vp, i32, C.POINTER(vp)]),
            "dl_ws_create_batch": (i32, [C.POINTER(vp), i32, i32, C.POINTER(vp)]),
            "dl_ws_batch": (i32, [vp]),
            "dl_ws_destroy": (None, [vp]),
            "dl_ws_bytes": (C.c_size_t, [vp]),
            "bta_assemble": (i32, [vp, vp, i32, vp]),
            "bta_factor": (i32, [vp, i32, vp, vp, vp]),
            "bta_solve": (i32, [vp, vp, i32, i32, dbl, vp]),
            "dl_ws_set_block": (i32, [vp, i32, i32, i32, vp, vp]),
            "dl_permute": (i32, [vp, vp, vp, i32, vp]),
            "dl_unpermute": (i32, [vp, vp, vp, i32, vp]),
            "dl_ws_estimate_bytes": (i32, [C.POINTER(vp), i32, i32, C.POINTER(C.c_size_t)]),
            "dl_ws_create_budget": (i32, [C.POINTER(vp), i32, i32, C.c_size_t,
                                          C.POINTER(vp)]),
            "dl_plan_waves": (i32, [C.POINTER(vp), i32, i32, C.c_size_t, C.POINTER(i32),
                                    C.POINTER(i32)]),
            "bta_selinv": (i32, [vp, vp, vp]),
            "fobj_eval": (i32, [vp, vp, i32, vp, vp, vp, vp]),
            "dl_ws_mean": (i32, [vp, vp, vp]),
            "dl_ws_get_block": (i32, [vp, i32, i32, i32, vp, vp]),
            "dl_dgemm": (i32, [i32, i32, i32, i64, i64, i64, dbl, vp, i64, vp,
                               i64, dbl, vp, i64, vp]),
            "dl_dpotrf": (i32, [i64, vp, i64, i32, vp, vp, vp]),
            "dl_dpotrf_noalloc": (i32, [i64, vp, i64, i32, vp, vp, vp]),
            "dl_status_string": (C.c_char_p, [i32]),
            "dl_ws_profile_begin": (i32, [vp, i32, i32]),
            "dl_autotune": (i32, [vp, C.c_char_p, vp]),
            "dl_ws_tile_counts": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
            "dl_ws_force_tile": (i32, [vp, i32]),
            "fobj_selinv_eval": (i32, [vp, vp, i32, vp, vp, vp, vp, vp]),
            "dl_ws_force_split": (i32, [vp, i32]),
            "dl_mlp_create": (i32, [vp, i32, i32, C.POINTER(vp)]),
            "dl_mlp_destroy": (None, [vp]),
            "dl_mlp_params": (i32, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64)]),
            "mlp_fwd": (i32, [vp, vp, i32, vp, vp]),
            "mlp_bwd": (i32, [vp, vp, i32, vp, vp]),
            "mlp_mse_grad": (i32, [vp, vp, i32, vp, vp, vp]),
            "mlp_adam": (i32, [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
            "dl_ws_profile_end": (i32, [vp, vp, vp, vp, vp]),
            "dl_ws_profile_enable": (i32, [vp, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn, code):
    if code != 0:
        raise DaliaError(fn, code)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def theta_dim(nv: int, likelihood: str = "gaussian") -> int:
    return int(lib().dl_theta_dim_lik(nv, LIKELIHOODS[likelihood]))


class Model:
    """Model data on the device (theta-independent)."""

    def __init__(self, nx: int, nt: int, nv: int, nr: int,
                 responses: Sequence, theta_prior_mean, theta_prior_sd=1.0,
                 prior_fixed=1e-3, family: str = "separable",
                 likelihood: str = "gaussian"):
        L = lib()
        if family not in MODEL_FAMILIES:
            raise ValueError(f"unknown model family {family!r}")
        if likelihood not in LIKELIHOODS:
            raise ValueError(f"unknown likelihood {likelihood!r}")
        self.nx, self.nt, self.nv, self.nr = nx, nt, nv, nr
        self.family = family
        self.likelihood = likelihood
        d = _Desc()
        d.nx, d.nt, d.nv, d.nr = nx, nt, nv, nr
        d.family = MODEL_FAMILIES[family]
        d.likelihood = LIKELIHOODS[likelihood]
        keep = []
        for j, r in enumerate(responses):
            t, nodes, w, X, y = r
            arrs = [np.ascontiguousarray(t, np.int32),
                    np.ascontiguousarray(nodes, np.int32).reshape(-1),
                    np.ascontiguousarray(w, np.float64).reshape(-1),
                    np.ascontiguousarray(X, np.float64).reshape(-1),
                    np.ascontiguousarray(y, np.float64)]
            keep.extend(arrs)
            d.m[j] = arrs[4].shape[0]
            d.obs_t[j] = arrs[0].ctypes.data
            d.obs_nodes[j] = arrs[1].ctypes.data
            d.obs_w[j] = arrs[2].ctypes.data
            d.obs_x[j] = arrs[3].ctypes.data if arrs[3].size else None
            d.y[j] = arrs[4].ctypes.data
        pm = np.ascontiguousarray(theta_prior_mean, np.float64)
        keep.append(pm)
        d.theta_prior_mean = pm.ctypes.data
        d.theta_prior_sd = float(theta_prior_sd)
        d.prior_fixed = float(prior_fixed)
        h = C.c_void_p()
        _check("dl_model_create", L.dl_model_create(C.byref(d), C.byref(h)))
        self.h = h
        vals = [C.c_int64() for _ in range(5)]
        _check("dl_model_dims", L.dl_model_dims(h, *[C.byref(v) for v in vals]))
        self.n, self.b, self.a, self.N, self.bp = [v.value for v in vals]
        self.dim_theta = theta_dim(nv, likelihood)

    def permute(self, x: torch.Tensor) -> torch.Tensor:
        """Model order -> BTA order of N-vectors (x: (N,) or (nvec, N))."""
        x = x.contiguous()
        out = torch.empty_like(x)
        nvec = 1 if x.dim() == 1 else x.shape[0]
        _check("dl_permute", lib().dl_permute(self.h, _ptr(x), _ptr(out), nvec, _stream()))
        return out

    def unpermute(self, x: torch.Tensor) -> torch.Tensor:
        """BTA order -> model order of N-vectors (x: (N,) or (nvec, N))."""
        x = x.contiguous()
        out = torch.empty_like(x)
        nvec = 1 if x.dim() == 1 else x.shape[0]
        _check("dl_unpermute", lib().dl_unpermute(self.h, _ptr(x), _ptr(out), nvec,
                                                  _stream()))
        return out

    @classmethod
    def from_workload(cls, wl) -> "Model":
        resp = [(r.t, r.nodes, r.w, r.X, r.y) for r in wl.responses]
        return cls(wl.nx, wl.nt, wl.nv, wl.nr, resp, wl.theta_prior_mean,
                   wl.theta_prior_sd, wl.prior_fixed,
                   getattr(wl, "model", "separable"),
                   getattr(wl, "likelihood", "gaussian"))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dl_model_destroy(self.h)
            self.h = None


def ws_flags(selinv: bool = False, keep_qp: bool = False, graph: bool = False,
             mixed: bool = False, splitk: bool = False, two_sided: bool = False,
             fold_inverse: bool = False, warm_start: bool = False, dag: bool = False) -> int:
    """The DL_WS_* flag word of a workspace."""
    return ((DL_WS_SELINV if selinv else 0) | (DL_WS_KEEP_QP if keep_qp else 0)
            | (DL_WS_GRAPH if graph else 0) | (DL_WS_MIXED if mixed else 0)
            | (DL_WS_SPLITK if splitk else 0)
            | (DL_WS_TWOSIDED if two_sided else 0)
            | (DL_WS_FOLD_INV if fold_inverse else 0)
            | (DL_WS_WARM_START if warm_start else 0)
            | (DL_WS_DAG if dag else 0))


def _model_array(models):
    if isinstance(models, Model):
        models = [models]
    return (C.c_void_p * len(models))(*[m.h for m in models]), len(models)


def estimate_bytes(models, **flags) -> int:
    """Device bytes a workspace of `models` with these flags allocates
    (computed on the host; see dl_ws_estimate_bytes)."""
    arr, n = _model_array(models)
    out = C.c_size_t()
    _check("dl_ws_estimate_bytes", lib().dl_ws_estimate_bytes(arr, n, ws_flags(**flags),
                                                              C.byref(out)))
    return int(out.value)


def plan_waves(models, hbm_budget: int, **flags) -> list:
    """Split a batch of models into waves whose workspaces fit hbm_budget
    bytes (dl_plan_waves); returns a list of lists of instance indices."""
    arr, n = _model_array(models)
    wave_of = (C.c_int32 * n)()
    nw = C.c_int32()
    _check("dl_plan_waves", lib().dl_plan_waves(arr, n, ws_flags(**flags), int(hbm_budget),
                                                wave_of, C.byref(nw)))
    waves = [[] for _ in range(nw.value)]
    for k in range(n):
        waves[wave_of[k]].append(k)
    return waves


class Workspace:
    """Dense BTA workspace of Q_p and Q_c for one model, or for a batch of
    instances (a list of models, repeated entries allowed) evaluated
    together.  Per-instance vectors are packed in instance order.  With
    hbm_budget (bytes) the workspace is created only if its estimated size
    fits (DaliaError with code DL_ENOMEM otherwise, nothing allocated)."""

    def __init__(self, models, selinv: bool = False, keep_qp: bool = False,
                 graph: bool = False, mixed: bool = False, splitk: bool = False,
                 two_sided: bool = False, fold_inverse: bool = False,
                 warm_start: bool = False, hbm_budget: Optional[int] = None,
                 dag: bool = False):
        if isinstance(models, Model):
            models = [models]
        self.models = list(models)
        self.model = self.models[0]
        flags = ws_flags(selinv, keep_qp, graph, mixed, splitk, two_sided, fold_inverse,
                         warm_start, dag)
        h = C.c_void_p()
        arr = (C.c_void_p * len(self.models))(*[m.h for m in self.models])
        if hbm_budget is None:
            _check("dl_ws_create_batch",
                   lib().dl_ws_create_batch(arr, len(self.models), flags, C.byref(h)))
        else:
            _check("dl_ws_create_budget",
                   lib().dl_ws_create_budget(arr, len(self.models), flags, int(hbm_budget),
                                             C.byref(h)))
        self.h = h
        self.B = len(self.models)
        self.N_total = sum(m.N for m in self.models)
        self.dev = torch.device("cuda")

    @property
    def nbytes(self) -> int:
        return int(lib().dl_ws_bytes(self.h))

    def _theta(self, theta) -> torch.Tensor:
        t = torch.as_tensor(theta, dtype=torch.float64)
        return t.to(self.dev).contiguous()

    def assemble(self, theta, which=DL_BOTH):
        th = self._theta(theta)
        _check("bta_assemble", lib().bta_assemble(self.h, _ptr(th), which, _stream()))
        self._keep = th

    def factor(self, which=DL_BOTH):
        k = (2 if which == DL_BOTH else 1) * self.B
        ld = torch.empty(k, dtype=torch.float64, device=self.dev)
        info = torch.empty(k, dtype=torch.int64, device=self.dev)
        _check("bta_factor", lib().bta_factor(self.h, which, _ptr(ld), _ptr(info),
                                              _stream()))
        return ld, info

    def solve(self, rhs: Optional[torch.Tensor] = None, refine_max: int = -1,
              refine_tol: float = DL_REFINE_TOL, return_converged: bool = False):
        """Solve with the factor of Q_c: the assembled A^T D y (rhs None;
        returns the mean) or, in place, rhs of shape (N_total,) or
        (nrhs, N_total).  refine_max < 0: the workspace's default FP64
        refinement; otherwise at most refine_max corrections to refine_tol.
        With return_converged, also whether every solve met refine_tol."""
        if rhs is None:
            code = lib().bta_solve(self.h, None, 1, int(refine_max), float(refine_tol),
                                   _stream())
            out = self.mean()
        else:
            assert rhs.shape[-1] == self.N_total and rhs.is_contiguous()
            nrhs = 1 if rhs.dim() == 1 else rhs.shape[0]
            code = lib().bta_solve(self.h, _ptr(rhs), nrhs, int(refine_max),
                                   float(refine_tol), _stream())
            out = rhs
        if code != DL_ENOTCONV:
            _check("bta_solve", code)
        return (out, code == 0) if return_converged else out

    def mean(self) -> torch.Tensor:
        out = torch.empty(self.N_total, dtype=torch.float64, device=self.dev)
        _check("dl_ws_mean", lib().dl_ws_mean(self.h, _ptr(out), _stream()))
        return out

    def selinv(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.N_total, dtype=torch.float64, device=self.dev)
        _check("bta_selinv", lib().bta_selinv(self.h, _ptr(out), _stream()))
        return out

    def fobj(self, thetas, out=None):
        """f_obj for each row of thetas; `out` = (f, parts, info) device
        tensors to write into (no allocation on the call)."""
        th = thetas if isinstance(thetas, torch.Tensor) and thetas.is_cuda \
            else torch.as_tensor(thetas, dtype=torch.float64)
        uniform = all(m is self.models[0] for m in self.models)
        if not uniform:
            # one packed theta per instance (dims may differ)
            th = th.reshape(-1).to(self.dev).contiguous()
            n = self.B
        else:
            if th.dim() == 1:
                th = th[None]
            th = th.to(self.dev).contiguous()
            n = th.shape[0]
        if out is None:
            f = torch.empty(n, dtype=torch.float64, device=self.dev)
            parts = torch.empty((n, 8), dtype=torch.float64, device=self.dev)
            info = torch.empty((n, 2), dtype=torch.int64, device=self.dev)
        else:
            f, parts, info = out
        _check("fobj_eval", lib().fobj_eval(self.h, _ptr(th), n, _ptr(f),
                                            _ptr(parts), _ptr(info), _stream()))
        return f, parts, info

    def fobj_selinv(self, thetas, out=None):
        """f_obj of one pass of thetas and the marginal variances of every
        instance, the solve overlapping the selected inversion; `out` =
        (f, parts, info, var) device tensors."""
        th = thetas if isinstance(thetas, torch.Tensor) and thetas.is_cuda \
            else torch.as_tensor(thetas, dtype=torch.float64)
        uniform = all(m is self.models[0] for m in self.models)
        if not uniform:
            th = th.reshape(-1).to(self.dev).contiguous()
            n = self.B
        else:
            if th.dim() == 1:
                th = th[None]
            th = th.to(self.dev).contiguous()
            n = th.shape[0]
        if out is None:
            f = torch.empty(n, dtype=torch.float64, device=self.dev)
            parts = torch.empty((n, 8), dtype=torch.float64, device=self.dev)
            info = torch.empty((n, 2), dtype=torch.int64, device=self.dev)
            var = torch.empty(self.N_total, dtype=torch.float64, device=self.dev)
        else:
            f, parts, info, var = out
        _check("fobj_selinv_eval", lib().fobj_selinv_eval(
            self.h, _ptr(th), n, _ptr(f), _ptr(parts), _ptr(info), _ptr(var), _stream()))
        return f, parts, info, var

    def autotune(self, cache_path: Optional[str] = None):
        """Measure and fix the GEMM tile of every launch (see dl_autotune)."""
        p = cache_path.encode() if cache_path else None
        _check("dl_autotune", lib().dl_autotune(self.h, p, _stream()))
        a, b = C.c_int64(), C.c_int64()
        _check("dl_ws_tile_counts", lib().dl_ws_tile_counts(self.h, C.byref(a), C.byref(b)))
        return {"tile64": a.value, "tile128": b.value}

    def force_tile(self, tile: int):
        """Use `tile` (64 or 128) for every matrix-product launch."""
        _check("dl_ws_force_tile", lib().dl_ws_force_tile(self.h, int(tile)))

    def force_split(self, ksplit: int):
        """Split the k range of every FP64 product launch into pieces of
        `ksplit` (0: unsplit)."""
        _check("dl_ws_force_split", lib().dl_ws_force_split(self.h, int(ksplit)))

    def tile_counts(self) -> dict:
        a, b = C.c_int64(), C.c_int64()
        _check("dl_ws_tile_counts", lib().dl_ws_tile_counts(self.h, C.byref(a), C.byref(b)))
        return {"tile64": a.value, "tile128": b.value}

    def profile_begin(self, categories=CATEGORIES, max_launches=200000,
                      by_kernel=False):
        """Bracket launches of `categories` with HIP events (aggregated by
        category, or by kernel when by_kernel)."""
        mask = 0
        for c in categories:
            mask |= 1 << CATEGORIES.index(c)
        self._prof_by_kernel = by_kernel
        if by_kernel:
            mask |= 1 << 16
        _check("dl_ws_profile_begin",
               lib().dl_ws_profile_begin(self.h, mask, int(max_launches)))

    def newton_steps(self) -> np.ndarray:
        """Inner Newton steps per instance of the last f_obj pass (Poisson
        likelihood; -1: not converged, 0: Gaussian)."""
        out = (C.c_int32 * len(self.models))()
        _check("dl_ws_newton_steps", lib().dl_ws_newton_steps(self.h, out))
        return np.array(out[:], dtype=np.int32)

    def profile_enable(self, on: bool):
        """Pause or resume the recording of profile_begin (no allocation)."""
        _check("dl_ws_profile_enable", lib().dl_ws_profile_enable(self.h, 1 if on else 0))

    def profile_end(self) -> dict:
        n = len(CATEGORIES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        fl = (C.c_double * n)()
        by = (C.c_double * n)()
        _check("dl_ws_profile_end", lib().dl_ws_profile_end(self.h, ms, cnt, fl, by))
        names = KERNELS if getattr(self, "_prof_by_kernel", False) else CATEGORIES
        return {c: dict(ms=ms[i], launches=cnt[i], flops=fl[i], bytes=by[i])
                for i, c in enumerate(names) if cnt[i]}

    def get_block(self, which: int, kind: int, t: int = 0) -> torch.Tensor:
        m = self.model
        shape = {0: (m.b, m.b), 1: (m.b, m.b), 2: (m.b, m.a), 3: (m.a, m.a),
                 4: (m.N,)}[kind]
        out = torch.empty(shape, dtype=torch.float64, device=self.dev)
        _check("dl_ws_get_block", lib().dl_ws_get_block(self.h, which, kind, t,
                                                        _ptr(out), _stream()))
        # column-major storage -> logical matrix
        return out.T if out.dim() == 2 else out

    def set_block(self, which: int, kind: int, t: int, M: torch.Tensor):
        """Overwrite one block of the assembled matrix (see get_block for
        kind); M is the logical matrix (or the N-vector for kind 4)."""
        if M.dim() == 2:
            M = M.T.contiguous()  # column-major storage
        else:
            M = M.contiguous()
        _check("dl_ws_set_block", lib().dl_ws_set_block(self.h, which, kind, t, _ptr(M),
                                                        _stream()))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            torch.cuda.synchronize()
            _lib.dl_ws_destroy(self.h)
            self.h = None


# ---- dense kernels -----------------------------------------------------------------

def dgemm(A: torch.Tensor, B: torch.Tensor, C_: torch.Tensor, *, transa=False,
          transb=False, lower=False, alpha=1.0, beta=0.0):
    """C = alpha op(A) op(B) + beta C on column-major views: pass tensors
    whose transpose is contiguous (x.T.contiguous().T), i.e. Fortran order."""
    def fcol(x):
        assert x.dtype == torch.float64 and x.is_cuda
        assert x.stride(0) == 1, "column-major tensor expected"
        return x.stride(1) if x.dim() == 2 and x.shape[1] > 1 else max(1, x.shape[0])
    M, N = C_.shape
    K = (A.shape[0] if transa else A.shape[1])
    _check("dl_dgemm", lib().dl_dgemm(int(transa), int(transb), int(lower), M, N,
                                      K, float(alpha), C.c_void_p(A.data_ptr()),
                                      fcol(A), C.c_void_p(B.data_ptr()), fcol(B),
                                      float(beta), C.c_void_p(C_.data_ptr()),
                                      fcol(C_), _stream()))
    return C_


def dpotrf(A: torch.Tensor, inverse: bool = False):
    """In-place Cholesky (lower, column-major) of a square n x n (n % 64 == 0)
    tensor; returns (logdet, info) device tensors."""
    n = A.shape[0]
    assert A.stride(0) == 1
    ld = torch.empty(1, dtype=torch.float64, device=A.device)
    info = torch.empty(1, dtype=torch.int64, device=A.device)
    _check("dl_dpotrf", lib().dl_dpotrf(n, C.c_void_p(A.data_ptr()), A.stride(1),
                                        int(inverse), _ptr(ld), _ptr(info),
                                        _stream()))
    return ld, info


def dpotrf_noalloc(A: torch.Tensor, logdet: torch.Tensor, info: torch.Tensor,
                   inverse: bool = False):
    """dpotrf through the entry point that allocates nothing: the caller
    provides the logdet (1 double) and info (1 int64) outputs; n % 64 == 0
    and n <= DPOTRF_NOALLOC_MAX_N."""
    n = A.shape[0]
    assert A.stride(0) == 1
    _check("dl_dpotrf_noalloc",
           lib().dl_dpotrf_noalloc(n, C.c_void_p(A.data_ptr()), A.stride(1), int(inverse),
                                   _ptr(logdet), _ptr(info), _stream()))


DPOTRF_NOALLOC_MAX_N = 2048


def fortran(x: torch.Tensor) -> torch.Tensor:
    """Column-major copy of a 2-D tensor (same logical values)."""
    return x.T.contiguous().T


class MLP:
    """Surrogate network on the device (FP32 master weights, BF16 matrix
    products).  Parameters are exposed as a flat torch view."""

    def __init__(self, sizes=(15, 256, 256, 256, 1), max_batch=4096):
        L = lib()
        arr = (C.c_int32 * len(sizes))(*sizes)
        h = C.c_void_p()
        _check("dl_mlp_create", L.dl_mlp_create(arr, len(sizes), int(max_batch),
                                                C.byref(h)))
        self.h = h
        self.sizes = tuple(sizes)
        self.max_batch = max_batch
        pw, pg, cnt = C.c_void_p(), C.c_void_p(), C.c_int64()
        _check("dl_mlp_params", L.dl_mlp_params(h, C.byref(pw), C.byref(pg), C.byref(cnt)))
        self.nparam = cnt.value
        self._pw, self._pg = pw.value, pg.value
        # torch views over the library-owned buffers (no copy)
        self.params = _device_view(self._pw, self.nparam, torch.float32)
        self.grads = _device_view(self._pg, self.nparam, torch.float32)

    def layers(self):
        """[(W, b)] views into the parameter vector."""
        out, off = [], 0
        for i, o in zip(self.sizes[:-1], self.sizes[1:]):
            W = self.params[off:off + i * o].view(o, i)
            off += i * o
            b = self.params[off:off + o]
            off += o
            out.append((W, b))
        return out

    def forward(self, X: torch.Tensor, out: Optional[torch.Tensor] = None):
        n = X.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=X.device)
        _check("mlp_fwd", lib().mlp_fwd(self.h, _ptr(X), n, _ptr(out), _stream()))
        return out

    def backward(self, dy: torch.Tensor, want_dx: bool = False):
        n = dy.shape[0]
        dX = torch.empty((n, self.sizes[0]), dtype=torch.float32,
                         device=dy.device) if want_dx else None
        _check("mlp_bwd", lib().mlp_bwd(self.h, _ptr(dy), n, _ptr(dX), _stream()))
        return dX

    def mse_grad(self, y: torch.Tensor):
        n = y.shape[0]
        dy = torch.empty(n, dtype=torch.float32, device=y.device)
        loss = torch.empty(1, dtype=torch.float32, device=y.device)
        _check("mlp_mse_grad", lib().mlp_mse_grad(self.h, _ptr(y), n, _ptr(dy),
                                                  _ptr(loss), _stream()))
        return dy, loss

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        _check("mlp_adam", lib().mlp_adam(self.h, lr, b1, b2, eps, _stream()))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            torch.cuda.synchronize()
            _lib.dl_mlp_destroy(self.h)
            self.h = None


def _device_view(ptr: int, n: int, dtype) -> torch.Tensor:
    """A torch tensor over library-owned device memory (no ownership)."""
    class _Holder:
        pass
    h = _Holder()
    itemsize = torch.tensor([], dtype=dtype).element_size()
    h.__cuda_array_interface__ = {
        "shape": (n,), "typestr": "<f4" if dtype == torch.float32 else "<f8",
        "data": (ptr, False), "version": 3, "strides": None}
    return torch.as_tensor(h, device="cuda")

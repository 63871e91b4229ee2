"""ctypes binding of ``libhif.so`` (the C ABI in ``include/hif.h``).

Argument marshalling only: every step of the factorization and of the
sweeps runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream.  The library must be built (``build.py``); nothing
here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhif.so")

HIF_OK, HIF_EINVAL, HIF_ENOMEM, HIF_ESINGULAR, HIF_EDEVICE, HIF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
HIF_FP64, HIF_FP32_MIXED = 0, 1
HIF_VARIANT_HIFIE, HIF_VARIANT_RSF = 0, 1
MAX_SUB = 64
PHASES = ("partition", "assembly", "id", "elimination", "sci", "top", "host", "rowqr")
_STATUS = {0: "HIF_OK", -1: "HIF_EINVAL", -2: "HIF_ENOMEM", -3: "HIF_ESINGULAR", -4: "HIF_EDEVICE",
           -5: "HIF_EUNSUPPORTED"}


class HifError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class hif_kernel(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("weights", ctypes.c_void_p), ("self", ctypes.c_void_p)]


class hif_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("second_kind", ctypes.c_int), ("symmetric", ctypes.c_int),
                ("variant", ctypes.c_int), ("n_proxy", ctypes.c_int), ("proxy_radius", ctypes.c_double),
                ("max_bytes", ctypes.c_size_t), ("row_compression", ctypes.c_int), ("fft_matvec", ctypes.c_int),
                ("trace_sublevel", ctypes.c_int), ("sweep_wait_us", ctypes.c_int)]


class hif_problem(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("dim", ctypes.c_int), ("kernel", hif_kernel),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p), ("eps", ctypes.c_double),
                ("leaf", ctypes.c_int32)]


class hif_tuning(ctypes.Structure):
    _fields_ = [("id_reg_waves", ctypes.c_int32 * 3), ("lu_panel_threads", ctypes.c_int32 * 2),
                ("rowqr_update_waves", ctypes.c_int32), ("rowqr_update_kind", ctypes.c_int32),
                ("sweep_many_threads", ctypes.c_int32)]


class hif_stats_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("n_sublevels", ctypes.c_int32), ("top_size", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("t_factor_ms", ctypes.c_double), ("t_phase_ms", ctypes.c_double * 8),
                ("sub_kind", ctypes.c_int32 * MAX_SUB), ("sub_groups", ctypes.c_int32 * MAX_SUB),
                ("sub_active", ctypes.c_int64 * MAX_SUB), ("sub_skel", ctypes.c_int64 * MAX_SUB),
                ("sub_near", ctypes.c_int64 * MAX_SUB), ("sub_classes", ctypes.c_int64 * MAX_SUB),
                ("sub_id_flops", ctypes.c_double * MAX_SUB), ("sub_elim_flops", ctypes.c_double * MAX_SUB),
                ("sub_t_ms", (ctypes.c_double * 8) * MAX_SUB),
                ("sub_id_bytes", ctypes.c_double * MAX_SUB), ("sub_rowqr_flops", ctypes.c_double * MAX_SUB)]


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_INT = ctypes.c_int
_DBL = ctypes.c_double

EXPORTS = {
    "hif_opts_default": (_INT, [_VP]),
    "hif_factor": (_INT, [_VP, _I64, _INT, _VP, _VP, _VP, _VP, _DBL, _I32, _VP, _VP, _VP]),
    "hif_apply": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_apply_T": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_solve": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_solve_T": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_matvec": (_INT, [_VP, _I64, _INT, _VP, _VP, _VP, _VP, _VP, _VP, _I64, _VP]),
    "hif_stats": (_INT, [_VP, _VP]),
    "hif_free": (None, [_VP]),
    "hif_last_error": (ctypes.c_char_p, []),
    "hif_id_batched": (_INT, [_VP, _VP, _VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "hif_partition": (_INT, [_VP, _I64, _INT, _VP, _INT, _I32, _VP, _VP]),
    "hif_gmres": (_INT, [_VP, _VP, _VP, _I64, _DBL, _I32, _VP, _VP, _VP]),
    "hif_gmres_T": (_INT, [_VP, _VP, _VP, _I64, _DBL, _I32, _VP, _VP, _VP]),
    "hif_diag_grad": (_INT, [_VP, _VP, _VP, _I64, _I64, _VP]),
    "hif_apply_A": (_INT, [_VP, _VP, _VP, _I64, _INT, _VP, _VP]),
    "hif_factor_batch": (_INT, [_VP, _I32, _VP, _I32, _VP, _VP]),
    "hif_solve_noalloc": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_solve_graph": (_INT, [_VP, _VP, _VP, _I64, _VP]),
    "hif_graph_launch": (_INT, [_VP, _VP]),
    "hif_graph_free": (None, [_VP]),
    "hif_trace_get": (_INT, [_VP, _INT, _VP, _I64, _VP]),
    "hif_tuning_get": (_INT, [_VP]),
    "hif_tuning_set": (_INT, [_VP]),
    "hif_lu_batched": (_INT, [_VP, _VP, _VP, _VP, _VP, _VP, _I32, _I32, _I32, _VP, _VP]),
}
HIF_SOLVE_NOALLOC_MAX = 4 << 20


def load_library():
    """Load ``libhif.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != HIF_OK:
        raise HifError(status, load_library().hif_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, n=None, name="array"):
    """Contiguous float64 CUDA tensor (host tensors are copied to the device)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _kernel(h, weights, selfk):
    return hif_kernel(float(h) if h is not None else 0.0, _ptr(weights), _ptr(selfk))


def default_opts() -> hif_opts:
    o = hif_opts()
    _check(load_library().hif_opts_default(ctypes.byref(o)))
    return o


class Factorization:
    """Handle of ``F ~ A`` on the device; ``solve`` / ``apply`` run the factored sweeps."""

    def __init__(self, handle, n, dim, keep):
        self._h = handle
        self.n = n
        self.dim = dim
        self._keep = keep

    def _run(self, fn, x, out=None, stream=None):
        if self._h is None:
            raise RuntimeError("factorization has been freed")
        x = _dev(x)
        vec = x.dim() == 1
        X = x.reshape(1, -1) if vec else x
        if X.shape[-1] != self.n:
            raise ValueError(f"last dimension must be n = {self.n}")
        Y = torch.empty_like(X) if out is None else out.reshape(X.shape)
        _check(fn(self._h, _ptr(X), _ptr(Y), X.shape[0], _stream(stream)))
        return Y.reshape(x.shape)

    def solve(self, f, out=None, stream=None):
        """``u = F^{-1} f``; ``f`` is ``(n,)`` or ``(nrhs, n)``."""
        return self._run(load_library().hif_solve, f, out, stream)

    def solve_noalloc(self, f, out, stream=None):
        """``hif_solve_noalloc``: ``F^{-1} f`` into the caller's ``out`` with the library's
        static scratch (no device allocation in the library)."""
        return self._run(load_library().hif_solve_noalloc, f, out, stream)

    def solve_graph(self, f, out):
        """``hif_solve_graph``: record the solve ``out = F^{-1} f`` once as a HIP graph;
        ``SolveGraph.launch()`` replays it (same vectors).  Keep ``f`` and ``out`` alive."""
        if self._h is None:
            raise RuntimeError("factorization has been freed")
        X = f.reshape(1, -1) if f.dim() == 1 else f
        if X.shape[-1] != self.n or not X.is_cuda or X.dtype != torch.float64 or not X.is_contiguous():
            raise ValueError(f"f must be a contiguous float64 device array with last dimension n = {self.n}")
        if out.shape != f.shape or not out.is_cuda or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device array shaped like f")
        torch.cuda.synchronize()  # the capture stream is not ordered after torch's
        g = ctypes.c_void_p()
        _check(load_library().hif_solve_graph(self._h, _ptr(X), _ptr(out), X.shape[0], ctypes.byref(g)))
        return SolveGraph(g, (f, out, self))

    def solve_T(self, f, out=None, stream=None):
        return self._run(load_library().hif_solve_T, f, out, stream)

    def apply(self, x, out=None, stream=None):
        """``y = F x``."""
        return self._run(load_library().hif_apply, x, out, stream)

    def apply_T(self, x, out=None, stream=None):
        return self._run(load_library().hif_apply_T, x, out, stream)

    def gmres(self, f, tol=1e-10, maxit=50, out=None, stream=None, transpose=False):
        """Solve ``A u = f`` by GMRES right-preconditioned with ``F^{-1}`` and the exact
        operator given to ``factor``; returns ``(u, iterations, true relative residuals)``.
        With ``transpose`` it solves ``A^T u = f`` preconditioned with ``F^{-T}``."""
        if self._h is None:
            raise RuntimeError("factorization has been freed")
        f = _dev(f)
        vec = f.dim() == 1
        Fm = (f.reshape(1, -1) if vec else f).contiguous()
        if Fm.shape[-1] != self.n:
            raise ValueError(f"last dimension must be n = {self.n}")
        U = torch.empty_like(Fm) if out is None else out.reshape(Fm.shape)
        nr = Fm.shape[0]
        its = (ctypes.c_int32 * nr)()
        rr = (ctypes.c_double * nr)()
        fn = load_library().hif_gmres_T if transpose else load_library().hif_gmres
        _check(fn(self._h, _ptr(Fm), _ptr(U), nr, float(tol), int(maxit),
                  ctypes.cast(its, _VP), ctypes.cast(rr, _VP), _stream(stream)))
        return U.reshape(f.shape), list(its), list(rr)

    def apply_A(self, x, transpose=False, out=None, stream=None):
        """``y = A x`` (or ``A^T x``) with the exact operator; returns ``(y, used_fft)``."""
        if self._h is None:
            raise RuntimeError("factorization has been freed")
        x = _dev(x)
        X = x.reshape(1, -1) if x.dim() == 1 else x
        if X.shape[-1] != self.n:
            raise ValueError(f"last dimension must be n = {self.n}")
        Y = torch.empty_like(X) if out is None else out.reshape(X.shape)
        used = ctypes.c_int32(0)
        _check(load_library().hif_apply_A(self._h, _ptr(X), _ptr(Y), X.shape[0], int(bool(transpose)),
                                          ctypes.byref(used), _stream(stream)))
        return Y.reshape(x.shape), bool(used.value)

    def stats(self) -> dict:
        s = hif_stats_t()
        _check(load_library().hif_stats(self._h, ctypes.byref(s)))
        ns = s.n_sublevels
        return {
            "n": s.n, "dim": s.dim, "levels": s.levels, "n_sublevels": ns, "top_size": s.top_size,
            "factor_bytes": s.factor_bytes, "t_factor_ms": s.t_factor_ms,
            "t_phase_ms": dict(zip(PHASES, list(s.t_phase_ms))),
            "sub_kind": list(s.sub_kind[:ns]), "sub_groups": list(s.sub_groups[:ns]),
            "sub_active": list(s.sub_active[:ns]), "sub_skel": list(s.sub_skel[:ns]),
            "sub_near": list(s.sub_near[:ns]), "sub_classes": list(s.sub_classes[:ns]),
            "sub_id_flops": list(s.sub_id_flops[:ns]), "sub_elim_flops": list(s.sub_elim_flops[:ns]),
            "sub_t_ms": [dict(zip(PHASES, list(s.sub_t_ms[i]))) for i in range(ns)],
            "sub_id_bytes": list(s.sub_id_bytes[:ns]), "sub_rowqr_flops": list(s.sub_rowqr_flops[:ns]),
        }

    def trace(self):
        """``hif_trace_get``: the sub-level kept with ``trace_sublevel`` as a dict of NumPy arrays
        (group starts and DOFs, near-field starts and DOFs, per-group blocks Y and A_cc)."""
        import numpy as np

        lib = load_library()
        items = {"group_start": (0, np.int64), "group_dofs": (1, np.int32), "near_start": (2, np.int64),
                 "near_dofs": (3, np.int32), "y_off": (4, np.int64), "Y": (5, np.float64), "acc_off": (6, np.int64),
                 "Acc": (7, np.float64)}
        out = {}
        for name, (item, dt) in items.items():
            cnt = ctypes.c_int64(0)
            _check(lib.hif_trace_get(self._h, item, None, 0, ctypes.byref(cnt)))
            arr = np.empty(cnt.value, dtype=dt)
            if cnt.value:
                _check(lib.hif_trace_get(self._h, item, arr.ctypes.data_as(_VP), cnt.value, ctypes.byref(cnt)))
            out[name] = arr
        return out

    def free(self):
        if self._h is not None:
            load_library().hif_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class SolveGraph:
    """A solve recorded as a HIP graph (``hif_solve_graph``); ``launch`` replays it."""

    def __init__(self, g, keep):
        self._g = g
        self._keep = keep

    def launch(self, stream=None):
        if self._g is None:
            raise RuntimeError("graph has been freed")
        _check(load_library().hif_graph_launch(self._g, _stream(stream)))

    def free(self):
        if self._g is not None:
            load_library().hif_graph_free(self._g)
            self._g = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def factor(points, eps, leaf, *, a=None, b=None, c=None, h=None, weights=None, selfk=None,
           second_kind=-1, symmetric=-1, variant="hifie", n_proxy=0, proxy_radius=0.0,
           max_bytes=0, precision=HIF_FP64, row_compression=-1, fft_matvec=0, trace_sublevel=-1,
           sweep_wait_us=0, stream=None) -> Factorization:
    """``hif_factor``: build ``F ~ A`` for points ``(n, d)`` in the unit box."""
    lib = load_library()
    P = _dev(points)
    if P.dim() != 2 or P.shape[1] not in (2, 3):
        raise ValueError("points must be (n, 2) or (n, 3)")
    n, d = P.shape
    av, bv, cv = _dev(a, n, "a"), _dev(b, n, "b"), _dev(c, n, "c")
    wv, sv = _dev(weights, n, "weights"), _dev(selfk, n, "selfk")
    k = _kernel(h, wv, sv)
    o = default_opts()
    o.precision = precision
    o.second_kind = second_kind
    o.symmetric = symmetric
    o.variant = HIF_VARIANT_RSF if variant == "rskel" else HIF_VARIANT_HIFIE
    o.n_proxy = n_proxy
    o.proxy_radius = proxy_radius
    o.max_bytes = max_bytes
    o.row_compression = row_compression
    o.fft_matvec = fft_matvec
    o.trace_sublevel = trace_sublevel
    o.sweep_wait_us = sweep_wait_us
    handle = ctypes.c_void_p()
    _check(lib.hif_factor(_ptr(P), n, d, ctypes.byref(k), _ptr(av), _ptr(bv), _ptr(cv), float(eps), int(leaf),
                          ctypes.byref(o), _stream(stream), ctypes.byref(handle)))
    return Factorization(handle, n, d, None)


def factor_batch(problems, *, nworkers=0, precision=HIF_FP64, second_kind=-1, symmetric=-1, variant="hifie",
                 max_bytes=0, row_compression=-1, fft_matvec=0):
    """``hif_factor_batch``: factor independent problems together.

    ``problems`` is a list of dicts with the ``factor`` arguments ``points``, ``eps``,
    ``leaf`` and optionally ``a``, ``b``, ``c``, ``h``, ``weights``, ``selfk``.
    ``nworkers=0``: level-synchronous (every sub-level one launch sequence over all
    problems); ``1..16``: that many worker threads running ``factor`` concurrently.
    Returns ``(factorizations, statuses)``; a failed problem's entry is ``None``."""
    lib = load_library()
    cnt = len(problems)
    arr = (hif_problem * max(cnt, 1))()
    keep = []
    for i, pr in enumerate(problems):
        P = _dev(pr["points"])
        if P.dim() != 2 or P.shape[1] not in (2, 3):
            raise ValueError("points must be (n, 2) or (n, 3)")
        n, d = P.shape
        av, bv, cv = (_dev(pr.get(k), n, k) for k in ("a", "b", "c"))
        wv, sv = _dev(pr.get("weights"), n, "weights"), _dev(pr.get("selfk"), n, "selfk")
        keep += [P, av, bv, cv, wv, sv]
        arr[i] = hif_problem(_ptr(P), n, d, _kernel(pr.get("h"), wv, sv), _ptr(av), _ptr(bv), _ptr(cv),
                             float(pr["eps"]), int(pr["leaf"]))
    o = default_opts()
    o.precision = precision
    o.second_kind = second_kind
    o.symmetric = symmetric
    o.variant = HIF_VARIANT_RSF if variant == "rskel" else HIF_VARIANT_HIFIE
    o.max_bytes = max_bytes
    o.row_compression = row_compression
    o.fft_matvec = fft_matvec
    handles = (ctypes.c_void_p * max(cnt, 1))()
    status = (ctypes.c_int * max(cnt, 1))()
    torch.cuda.synchronize()  # the inputs were written on torch's stream
    lib.hif_factor_batch(ctypes.cast(arr, _VP), cnt, ctypes.byref(o), int(nworkers), ctypes.cast(handles, _VP),
                         ctypes.cast(status, _VP))
    facs = []
    for i in range(cnt):
        if handles[i]:
            n, d = arr[i].n, arr[i].dim
            facs.append(Factorization(ctypes.c_void_p(handles[i]), n, d, None))
        else:
            facs.append(None)
    return facs, list(status[:cnt])


def matvec(points, x, *, a=None, b=None, c=None, h=None, weights=None, selfk=None, out=None, stream=None):
    """``hif_matvec``: exact ``y = A x`` on the fly; ``x`` is ``(n,)`` or ``(nrhs, n)``."""
    lib = load_library()
    P = _dev(points)
    n, d = P.shape
    x = _dev(x)
    X = x.reshape(1, -1) if x.dim() == 1 else x
    if X.shape[-1] != n:
        raise ValueError("last dimension of x must be n")
    av, bv, cv = _dev(a, n, "a"), _dev(b, n, "b"), _dev(c, n, "c")
    wv, sv = _dev(weights, n, "weights"), _dev(selfk, n, "selfk")
    k = _kernel(h, wv, sv)
    Y = torch.empty_like(X) if out is None else out.reshape(X.shape)
    _check(lib.hif_matvec(_ptr(P), n, d, ctypes.byref(k), _ptr(av), _ptr(bv), _ptr(cv), _ptr(X), _ptr(Y),
                          X.shape[0], _stream(stream)))
    return Y.reshape(x.shape)


def diag_grad(lam, u, out=None, stream=None):
    """``hif_diag_grad``: ``-sum_r lam[r] * u[r]`` for ``(n,)`` or ``(nrhs, n)`` device arrays."""
    L = _dev(lam)
    U = _dev(u)
    if L.shape != U.shape or L.dim() not in (1, 2):
        raise ValueError("lam and u must have the same shape, (n,) or (nrhs, n)")
    L2 = L.reshape(1, -1) if L.dim() == 1 else L
    U2 = U.reshape(1, -1) if U.dim() == 1 else U
    n = L2.shape[1]
    G = torch.empty(n, dtype=torch.float64, device=L.device) if out is None else out
    _check(load_library().hif_diag_grad(_ptr(L2), _ptr(U2), _ptr(G), n, L2.shape[0], _stream(stream)))
    return G


def id_batched(mats, tols, stream=None):
    """``hif_id_batched`` on a list of 2-D matrices; returns ``[(sk, rd, T), ...]`` as CPU tensors."""
    lib = load_library()
    shapes = [tuple(m.shape) for m in mats]
    flat = torch.cat([_dev(m).reshape(-1) for m in mats]) if mats else torch.zeros(0, device="cuda",
                                                                                    dtype=torch.float64)
    offs, poffs, toffs = [], [], []
    o = po = to = 0
    for (m, nc) in shapes:
        offs.append(o)
        poffs.append(po)
        toffs.append(to)
        o += m * nc
        po += nc
        to += nc * nc
    dev = dict(device="cuda")
    off = torch.tensor(offs, dtype=torch.int64, **dev)
    rows = torch.tensor([s[0] for s in shapes], dtype=torch.int32, **dev)
    cols = torch.tensor([s[1] for s in shapes], dtype=torch.int32, **dev)
    tol = torch.tensor(list(tols), dtype=torch.float64, **dev)
    rank = torch.zeros(len(mats), dtype=torch.int32, **dev)
    perm = torch.zeros(max(po, 1), dtype=torch.int32, **dev)
    poff = torch.tensor(poffs, dtype=torch.int64, **dev)
    T = torch.zeros(max(to, 1), dtype=torch.float64, **dev)
    toff = torch.tensor(toffs, dtype=torch.int64, **dev)
    maxc = max([s[1] for s in shapes] + [1])
    _check(lib.hif_id_batched(_ptr(flat), _ptr(off), _ptr(rows), _ptr(cols), _ptr(tol), len(mats), maxc,
                              _ptr(rank), _ptr(perm), _ptr(poff), _ptr(T), _ptr(toff), _stream(stream)))
    rank, perm, T = rank.cpu(), perm.cpu(), T.cpu()
    out = []
    for q, (m, nc) in enumerate(shapes):
        k = int(rank[q])
        p = perm[poffs[q]:poffs[q] + nc]
        out.append((p[:k].clone(), p[k:].clone(), T[toffs[q]:toffs[q] + k * (nc - k)].reshape(k, nc - k).clone()))
    return out


def partition(points, active, kind, S, stream=None):
    """``hif_partition``: group index of every active point at one sub-level (-1 if inactive)."""
    lib = load_library()
    P = _dev(points)
    n, d = P.shape
    act = torch.as_tensor(active).to(device="cuda", dtype=torch.uint8).contiguous()
    grp = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(lib.hif_partition(_ptr(P), n, d, _ptr(act), int(kind), int(S), _ptr(grp), _stream(stream)))
    return grp


def tuning_get() -> dict:
    """``hif_tuning_get``: the launch-shape table in use."""
    t = hif_tuning()
    _check(load_library().hif_tuning_get(ctypes.byref(t)))
    return {"id_reg_waves": list(t.id_reg_waves), "lu_panel_threads": list(t.lu_panel_threads),
            "rowqr_update_waves": int(t.rowqr_update_waves), "rowqr_update_kind": int(t.rowqr_update_kind),
            "sweep_many_threads": int(t.sweep_many_threads)}


def tuning_set(table=None):
    """``hif_tuning_set``: replace the launch-shape table (``None``: the built-in one)."""
    if table is None:
        _check(load_library().hif_tuning_set(None))
        return
    t = hif_tuning()
    t.id_reg_waves[:] = list(table["id_reg_waves"])
    t.lu_panel_threads[:] = list(table["lu_panel_threads"])
    t.rowqr_update_waves = int(table["rowqr_update_waves"])
    t.rowqr_update_kind = int(table["rowqr_update_kind"])
    t.sweep_many_threads = int(table["sweep_many_threads"])
    _check(load_library().hif_tuning_set(ctypes.byref(t)))


def lu_batched(mats, rs, stream=None):
    """``hif_lu_batched`` on a list of square matrices with the numbers of columns to
    eliminate ``rs``; returns ``([factored matrix], [row interchanges], zero_pivot)`` on the CPU."""
    lib = load_library()
    ns = [int(m.shape[0]) for m in mats]
    flat = torch.cat([_dev(m).reshape(-1) for m in mats])
    offs, poffs = [0], [0]
    for n, r in zip(ns, rs):
        offs.append(offs[-1] + n * n)
        poffs.append(poffs[-1] + int(r))
    dev = dict(device="cuda")
    off = torch.tensor(offs[:-1], dtype=torch.int64, **dev)
    poff = torch.tensor(poffs[:-1], dtype=torch.int64, **dev)
    n_t = torch.tensor(ns, dtype=torch.int32, **dev)
    r_t = torch.tensor([int(r) for r in rs], dtype=torch.int32, **dev)
    piv = torch.zeros(max(poffs[-1], 1), dtype=torch.int32, **dev)
    status = torch.zeros(1, dtype=torch.int32, **dev)
    _check(lib.hif_lu_batched(_ptr(flat), _ptr(off), _ptr(n_t), _ptr(r_t), _ptr(piv), _ptr(poff), len(mats),
                              max(ns), max(int(r) for r in rs), _ptr(status), _stream(stream)))
    flat, piv = flat.cpu(), piv.cpu()
    out = [flat[offs[i]:offs[i + 1]].reshape(ns[i], ns[i]) for i in range(len(mats))]
    pv = [piv[poffs[i]:poffs[i + 1]] for i in range(len(mats))]
    return out, pv, bool(status.item())

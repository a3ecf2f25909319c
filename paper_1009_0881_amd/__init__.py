"""Python binding of libnmf (multilevel NMF on MI355X).

Argument marshalling only: every step of the method runs inside libnmf.so's
HIP kernels.  PyTorch supplies device memory and the stream; there is no CPU
fallback, and loading fails loudly when the library has not been built
(``python -m paper_1009_0881_amd.build``).

Layouts (see include/nmf.h): M is m x n column-major, V is m x r
column-major, W is r x n row-major.  In torch terms the binding stores M as a
contiguous (n, m) tensor (row j = image j), V as a contiguous (r, m) tensor
(row k = basis image k) and W as a contiguous (r, n) tensor.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf.so")

HALS, MU, ANLS, KL = 0, 1, 2, 3
NI, VC, FMG, WC = 0, 1, 2, 3
XFER_FW, XFER_BLOCK2 = 0, 1
FP32, BF16 = 0, 1

ALGOS = {"hals": HALS, "mu": MU, "anls": ANLS, "kl": KL}
CYCLES = {"ni": NI, "vc": VC, "fmg": FMG, "wc": WC}
XFERS = {"fw": XFER_FW, "block2": XFER_BLOCK2}
PRECS = {"fp32": FP32, "bf16": BF16}

STATUS = {0: "NMF_OK", -1: "NMF_E_ARG", -2: "NMF_E_SHAPE", -3: "NMF_E_NOMEM",
          -4: "NMF_E_DEVICE", -5: "NMF_E_NONFINITE", -6: "NMF_E_NEGATIVE", -7: "NMF_E_BUSY",
          1: "NMF_PENDING"}
PENDING = 1

# Every symbol include/nmf.h declares.
EXPORTS = [
    "nmf_plan", "nmf_solve", "nmf_destroy", "nmf_status_string", "nmf_last_error",
    "nmf_query_levels", "nmf_query_schedule", "nmf_query_log",
    "nmf_restrict", "nmf_prolong", "nmf_iterate", "nmf_products", "nmf_gram",
    "nmf_profile", "nmf_profile_read", "nmf_batch_workspace", "nmf_solve_batch",
    "nmf_server_create", "nmf_server_submit", "nmf_server_poll", "nmf_server_stats",
    "nmf_server_destroy", "nmf_solve_static", "nmf_ntf_solve",
]

BATCH_GRAPH = 1
STATIC_WORKSPACE_BYTES = 32 << 20     # NMF_STATIC_WORKSPACE_BYTES (include/nmf.h)

# Kernel kinds of the event profiler (include/nmf.h).
KERNEL_KINDS = ["apass", "gram_v", "cpass_partial", "cpass_final", "gram_w", "residual",
                "nnls_rows", "nnls_cols", "restrict", "prolong", "sumsq", "kl_div", "ntf"]


class NmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ldm", ctypes.c_int64),
        ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("r", ctypes.c_int32),
        ("levels", ctypes.c_int32), ("algo", ctypes.c_int32), ("cycle", ctypes.c_int32),
        ("xfer", ctypes.c_int32), ("prec", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
        ("max_fine_iters", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("log_cap", ctypes.c_int32), ("check_input", ctypes.c_int32),
        ("tile_cfg", ctypes.c_int32), ("tol", ctypes.c_double),
        ("two_sided", ctypes.c_int32), ("ntf_k", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("log_len", ctypes.c_int32), ("total_iters", ctypes.c_int32),
        ("fine_iters", ctypes.c_int32), ("stopped", ctypes.c_int32),
        ("rel_err", ctypes.c_double), ("fine_equiv", ctypes.c_double),
        ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libnmf.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1009_0881_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.nmf_plan.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.nmf_solve.argtypes = [vp, vp, vp, vp, i32, vp, vp, ctypes.POINTER(Result)]
        L.nmf_solve_static.argtypes = [vp, vp, vp, vp, i32, vp, ctypes.POINTER(Result)]
        L.nmf_ntf_solve.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, ctypes.POINTER(Result)]
        L.nmf_destroy.argtypes = [vp]
        L.nmf_status_string.argtypes = [i32]
        L.nmf_status_string.restype = ctypes.c_char_p
        L.nmf_last_error.argtypes = [vp]
        L.nmf_last_error.restype = ctypes.c_char_p
        L.nmf_query_levels.argtypes = [vp, ctypes.POINTER(i32), i32]
        L.nmf_query_schedule.argtypes = [vp, i32, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
        L.nmf_query_log.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(i32), i32]
        L.nmf_restrict.argtypes = [i32, i32, i32, i64, vp, i64, vp, vp]
        L.nmf_prolong.argtypes = [i32, i32, i32, i64, vp, vp, vp]
        L.nmf_iterate.argtypes = [vp, vp, vp, vp, i32, vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.nmf_products.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.nmf_profile.argtypes = [vp, ctypes.c_uint32]
        L.nmf_profile_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                       i32, i32]
        L.nmf_gram.argtypes = [i32, i64, vp, i64, vp, vp, sz, vp]
        L.nmf_server_create.argtypes = [sz, i32, ctypes.POINTER(vp)]
        L.nmf_server_submit.argtypes = [vp, ctypes.POINTER(Desc), vp, vp, vp, i32,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.nmf_server_poll.argtypes = [vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(Result)]
        L.nmf_server_stats.argtypes = [vp, ctypes.POINTER(i64), i32]
        L.nmf_server_destroy.argtypes = [vp]
        L.nmf_batch_workspace.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(sz)]
        L.nmf_solve_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(i32), vp, vp, i32, ctypes.POINTER(Result)]
        for name in EXPORTS:
            if name not in ("nmf_status_string", "nmf_last_error"):
                getattr(L, name).restype = i32
        _LIB = L
    return _LIB


def _check(st: int, plan_handle=None) -> None:
    if st != 0:
        msg = lib().nmf_last_error(plan_handle)
        raise NmfError(st, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need_cuda(*ts) -> None:
    for t in ts:
        if not t.is_cuda or not t.is_contiguous() or t.dtype != _torch().float32:
            raise ValueError("expected contiguous float32 CUDA tensors")


# --------------------------------------------------------------------- plans

def tile(wc: int, cf: int) -> int:
    """nmf_desc.tile_cfg value NMF_TILE(wc, cf) (include/nmf.h)."""
    return int(wc) | (int(cf) << 8)


TILE_GROUPED = 1 << 16   # NMF_TILE_GROUPED: plan sized for grouped (batch / server) launches


def make_desc(m, n, h, w, r, levels=1, algo="hals", cycle="ni", xfer="fw", prec="fp32",
              tol=0.0, max_fine_iters=0, check_every=8, log_cap=4096, check_input=False,
              refine_iters=0, ldm=0, tile_cfg=0, two_sided=False, ntf_k=0,
              grouped=False) -> Desc:
    """nmf_desc from Python values (names as in include/nmf.h); tile_cfg is 0,
    an NMF_TILE value or a (wc, cf) pair; grouped ors in NMF_TILE_GROUPED."""
    d = Desc()
    d.m, d.n, d.ldm, d.h, d.w, d.r, d.levels = m, n, ldm, h, w, r, levels
    d.algo = ALGOS.get(algo, algo) if isinstance(algo, str) else algo
    d.cycle = CYCLES.get(cycle, cycle) if isinstance(cycle, str) else cycle
    d.xfer = XFERS.get(xfer, xfer) if isinstance(xfer, str) else xfer
    d.prec = PRECS.get(prec, prec) if isinstance(prec, str) else prec
    d.tol, d.max_fine_iters, d.check_every = tol, max_fine_iters, check_every
    d.log_cap, d.check_input, d.refine_iters = log_cap, int(check_input), refine_iters
    d.tile_cfg = tile(*tile_cfg) if isinstance(tile_cfg, (tuple, list)) else int(tile_cfg)
    if grouped:
        d.tile_cfg |= TILE_GROUPED
    d.two_sided = int(bool(two_sided))
    d.ntf_k = int(ntf_k)
    return d


class Plan:
    """A validated problem description (host only) and its workspace size."""

    def __init__(self, m: int, n: int, h: int, w: int, r: int, levels: int = 1,
                 algo="hals", cycle="ni", xfer="fw", prec="fp32", tol: float = 0.0,
                 max_fine_iters: int = 0, check_every: int = 8, log_cap: int = 4096,
                 check_input: bool = False, refine_iters: int = 0, ldm: int = 0, tile_cfg=0,
                 two_sided: bool = False, ntf_k: int = 0, grouped: bool = False):
        d = make_desc(m, n, h, w, r, levels, algo, cycle, xfer, prec, tol, max_fine_iters,
                      check_every, log_cap, check_input, refine_iters, ldm, tile_cfg, two_sided,
                      ntf_k, grouped)
        self.desc = d
        self.handle = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        _check(lib().nmf_plan(ctypes.byref(d), ctypes.byref(self.handle), ctypes.byref(wsb)))
        self.workspace_bytes = wsb.value
        self.m, self.n, self.r, self.levels = m, n, r, levels

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.nmf_destroy(h)
            self.handle = ctypes.c_void_p()

    def level_sides(self) -> List[Tuple[int, int]]:
        buf = (ctypes.c_int32 * (2 * self.levels))()
        _check(lib().nmf_query_levels(self.handle, buf, self.levels), self.handle)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(self.levels)]

    def schedule(self, iters: int) -> List[Tuple[str, int, int]]:
        n = ctypes.c_int32()
        _check(lib().nmf_query_schedule(self.handle, iters, None, 0, ctypes.byref(n)), self.handle)
        buf = (ctypes.c_int32 * (3 * max(1, n.value)))()
        _check(lib().nmf_query_schedule(self.handle, iters, buf, n.value, ctypes.byref(n)),
               self.handle)
        kinds = {0: "run", 1: "restrict", 2: "prolong"}
        return [(kinds[buf[3 * i]], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n.value)]

    def workspace(self):
        torch = _torch()
        return torch.empty(max(256, self.workspace_bytes), dtype=torch.uint8, device="cuda")

    def solve(self, M, V, W, iters: int, workspace=None, stream=None) -> dict:
        """M: (n, m) float32 CUDA tensor (image rows); V: (r, m); W: (r, n).
        V and W are updated in place.  Returns the nmf_result as a dict."""
        _need_cuda(M, V, W)
        ws = workspace if workspace is not None else self.workspace()
        res = Result()
        _check(lib().nmf_solve(self.handle, _ptr(M), _ptr(V), _ptr(W), int(iters), _ptr(ws),
                               _stream_handle(stream), ctypes.byref(res)), self.handle)
        out = res.as_dict()
        out["_workspace"] = ws
        return out

    def solve_ntf(self, X, A, Bt, Ct, iters: int, workspace=None, stream=None) -> dict:
        """NTF plan (ntf_k = K): X the mode-1 unfolding as an (n, m) float32 CUDA
        tensor (n = J K, row j + J k holding X[:, j, k]); A (r, m); Bt (r, J);
        Ct (r, K).  A, Bt and Ct are updated in place."""
        _need_cuda(X, A, Bt, Ct)
        ws = workspace if workspace is not None else self.workspace()
        res = Result()
        _check(lib().nmf_ntf_solve(self.handle, _ptr(X), _ptr(A), _ptr(Bt), _ptr(Ct), int(iters),
                                   _ptr(ws), _stream_handle(stream), ctypes.byref(res)),
               self.handle)
        out = res.as_dict()
        out["_workspace"] = ws
        return out

    def solve_static(self, M, V, W, iters: int, stream=None) -> dict:
        """As solve(), through nmf_solve_static: no workspace argument, the
        library's fixed device array serves instead (nothing is allocated)."""
        _need_cuda(M, V, W)
        res = Result()
        _check(lib().nmf_solve_static(self.handle, _ptr(M), _ptr(V), _ptr(W), int(iters),
                                      _stream_handle(stream), ctypes.byref(res)), self.handle)
        return res.as_dict()

    def iterate(self, M, V, W, count: int, workspace=None, stream=None) -> float:
        _need_cuda(M, V, W)
        ws = workspace if workspace is not None else self.workspace()
        rel = ctypes.c_double()
        _check(lib().nmf_iterate(self.handle, _ptr(M), _ptr(V), _ptr(W), int(count), _ptr(ws),
                                 _stream_handle(stream), ctypes.byref(rel)), self.handle)
        return rel.value

    def products(self, M, V, W, workspace=None, stream=None):
        """A = M W^T as an (r, m) tensor (column-major m x r) and C = V^T M as (r, n)."""
        torch = _torch()
        _need_cuda(M, V, W)
        ws = workspace if workspace is not None else self.workspace()
        A = torch.empty((self.r, self.m), dtype=torch.float32, device=M.device)
        C = torch.empty((self.r, self.n), dtype=torch.float32, device=M.device)
        _check(lib().nmf_products(self.handle, _ptr(M), _ptr(V), _ptr(W), _ptr(A), _ptr(C),
                                  _ptr(ws), _stream_handle(stream)), self.handle)
        return A, C

    def profile(self, kinds) -> None:
        """Time every launch of the given kernel kinds with HIP events."""
        mask = 0
        for k in kinds:
            mask |= 1 << (KERNEL_KINDS.index(k) if isinstance(k, str) else int(k))
        _check(lib().nmf_profile(self.handle, mask), self.handle)

    def profile_read(self, reset: bool = True) -> dict:
        n = len(KERNEL_KINDS)
        cnt = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        _check(lib().nmf_profile_read(self.handle, cnt, ms, n, int(reset)), self.handle)
        return {KERNEL_KINDS[i]: (cnt[i], ms[i]) for i in range(n) if cnt[i]}

    def log(self, workspace, cap: Optional[int] = None, stream=None) -> Tuple[np.ndarray, np.ndarray]:
        cap = cap or self.desc.log_cap
        rel = (ctypes.c_double * cap)()
        dep = (ctypes.c_int32 * cap)()
        _check(lib().nmf_query_log(self.handle, _ptr(workspace), _stream_handle(stream), rel, dep,
                                   cap), self.handle)
        return np.frombuffer(rel, dtype=np.float64).copy(), np.frombuffer(dep, dtype=np.int32).copy()


# ----------------------------------------------------------- single operators

def restrict(X, h: int, w: int, xfer="fw", stream=None):
    """R(X) columnwise: X is a (ncols, h*w) CUDA tensor; returns (ncols, hc*wc)."""
    torch = _torch()
    _need_cuda(X)
    xf = XFERS.get(xfer, xfer) if isinstance(xfer, str) else xfer
    hc, wc = (h + 1) // 2, (w + 1) // 2
    Y = torch.empty((X.shape[0], hc * wc), dtype=torch.float32, device=X.device)
    _check(lib().nmf_restrict(xf, h, w, X.shape[0], _ptr(X), X.shape[1], _ptr(Y),
                              _stream_handle(stream)))
    return Y


def prolong(Y, h: int, w: int, xfer="fw", stream=None):
    """P(Y) columnwise onto the h x w grid: Y is (ncols, hc*wc); returns (ncols, h*w)."""
    torch = _torch()
    _need_cuda(Y)
    xf = XFERS.get(xfer, xfer) if isinstance(xfer, str) else xfer
    X = torch.empty((Y.shape[0], h * w), dtype=torch.float32, device=Y.device)
    _check(lib().nmf_prolong(xf, h, w, Y.shape[0], _ptr(Y), _ptr(X), _stream_handle(stream)))
    return X


def gram(X, stream=None):
    """FP64 Gram X X^T of the rows of a (r, L) float32 CUDA tensor."""
    torch = _torch()
    _need_cuda(X)
    r, L = X.shape
    G = torch.empty((r, r), dtype=torch.float64, device=X.device)
    rpad = (r + 15) // 16 * 16
    parts = min(256, (L + 63) // 64)
    ws = torch.empty(parts * rpad * rpad * 8 + 256, dtype=torch.uint8, device=X.device)
    _check(lib().nmf_gram(r, L, _ptr(X), L, _ptr(G), _ptr(ws), ws.numel(), _stream_handle(stream)))
    return G


def batch_workspace(plans):
    """Device workspace (uint8 tensor) of a batch over these plans."""
    torch = _torch()
    hs = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    nb = ctypes.c_size_t()
    _check(lib().nmf_batch_workspace(hs, len(plans), ctypes.byref(nb)))
    return torch.empty(max(256, nb.value), dtype=torch.uint8, device="cuda")


def solve_batch(plans, Ms, Vs, Ws, iters, workspace=None, graph=False, stream=None):
    """Solve len(plans) independent problems in one batch (nmf_solve_batch).

    Ms[i], Vs[i], Ws[i] as for Plan.solve (V, W updated in place); iters is an
    int or one budget per problem.  Returns one result dict per problem."""
    k = len(plans)
    _need_cuda(*Ms, *Vs, *Ws)
    if isinstance(iters, int):
        iters = [iters] * k
    ws = workspace if workspace is not None else batch_workspace(plans)
    vp = ctypes.c_void_p
    hs = (vp * k)(*[p.handle for p in plans])
    pm = (vp * k)(*[M.data_ptr() for M in Ms])
    pv = (vp * k)(*[V.data_ptr() for V in Vs])
    pw = (vp * k)(*[W.data_ptr() for W in Ws])
    it = (ctypes.c_int32 * k)(*[int(x) for x in iters])
    res = (Result * k)()
    st = lib().nmf_solve_batch(hs, k, pm, pv, pw, it, _ptr(ws), _stream_handle(stream),
                               BATCH_GRAPH if graph else 0, res)
    _check(st)
    return [r.as_dict() for r in res]


class Server:
    """Serving loop with continuous batching (nmf_server_*).

    submit() takes host numpy arrays in the library layout (M m x n and V0
    m x r Fortran-ordered float32, W0 r x n C-ordered) and keeps references to
    them until the request is retired; poll() returns None while it runs,
    else (V, W, result) with V m x r and W r x n (float32)."""

    def __init__(self, hbm_budget: int, slots: int):
        self.handle = ctypes.c_void_p()
        _check(lib().nmf_server_create(int(hbm_budget), int(slots), ctypes.byref(self.handle)))
        self._keep = {}

    def submit(self, M: np.ndarray, V0: np.ndarray, W0: np.ndarray, iters: int, h: int, w: int,
               r: int, **desc) -> int:
        M = np.asfortranarray(M, dtype=np.float32)
        V0 = np.asfortranarray(V0, dtype=np.float32)
        W0 = np.ascontiguousarray(W0, dtype=np.float32)
        m, n = M.shape
        d = make_desc(m, n, h, w, r, **desc)
        t = ctypes.c_uint64()
        _check(lib().nmf_server_submit(self.handle, ctypes.byref(d), M.ctypes.data,
                                       V0.ctypes.data, W0.ctypes.data, int(iters),
                                       ctypes.byref(t)))
        self._keep[t.value] = (M, V0, W0, d, m, n, r)
        return t.value

    def poll(self, ticket: int):
        M, V0, W0, d, m, n, r = self._keep[ticket]
        V = np.empty((m, r), dtype=np.float32, order="F")
        W = np.empty((r, n), dtype=np.float32)
        res = Result()
        st = lib().nmf_server_poll(self.handle, ticket, V.ctypes.data, W.ctypes.data,
                                   ctypes.byref(res))
        if st == PENDING:
            return None
        del self._keep[ticket]
        _check(st)
        return V, W, res.as_dict()

    def stats(self) -> dict:
        buf = (ctypes.c_int64 * 6)()
        _check(lib().nmf_server_stats(self.handle, buf, 6))
        keys = ["admitted", "completed", "running", "peak_running", "peak_pool_bytes", "ticks"]
        return dict(zip(keys, list(buf)))

    def close(self):
        if self.handle is not None and self.handle.value and _LIB is not None:
            _LIB.nmf_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self._keep.clear()

    def __del__(self):
        self.close()


# ------------------------------------------------------------ array helpers

def to_device(M: np.ndarray, V: np.ndarray, W: np.ndarray, device="cuda"):
    """Numpy (m x n, m x r, r x n) -> device tensors in the library layout."""
    torch = _torch()
    Md = torch.from_numpy(np.ascontiguousarray(np.asarray(M, dtype=np.float32).T)).to(device)
    Vd = torch.from_numpy(np.ascontiguousarray(np.asarray(V, dtype=np.float32).T)).to(device)
    Wd = torch.from_numpy(np.ascontiguousarray(np.asarray(W, dtype=np.float32))).to(device)
    return Md, Vd, Wd


def factors_to_host(Vd, Wd) -> Tuple[np.ndarray, np.ndarray]:
    """Device (r, m) V and (r, n) W -> numpy m x r and r x n (float64)."""
    return Vd.double().cpu().numpy().T.copy(), Wd.double().cpu().numpy()

"""ctypes binding of libhdm (include/hdm.h): argument marshalling only.

Every step of the computation runs in the HIP library; torch supplies device
memory and the current stream.  Loading fails loudly when libhdm.so has not been
built: there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hdm.h")

F64, F32, BF16, F16, U8 = 0, 1, 2, 3, 4
PREC = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}
STATUS = {0: "HDM_OK", 1: "HDM_EINVAL", 2: "HDM_ENOMEM", 3: "HDM_EDEVICE", 4: "HDM_ENOCONV", 5: "HDM_EBUSY",
          6: "HDM_ECANCELLED", 7: "HDM_EINTERNAL", 8: "HDM_ENUMERIC"}


class HdmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("x_dtype", C.c_int32), ("eps", C.c_double),
                ("alpha", C.c_double), ("leaf_m", C.c_int32), ("max_rank_s", C.c_int32), ("tau", C.c_double),
                ("knn_k", C.c_int32), ("knn_iters", C.c_int32), ("budget", C.c_double), ("near_prec", C.c_int32),
                ("far_prec", C.c_int32), ("seed", C.c_uint64)]


class OpStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("depth", C.c_int32), ("leaves", C.c_int32),
                ("knn_k", C.c_int32), ("max_rank", C.c_int32), ("min_leaf_rank", C.c_int32),
                ("mean_leaf_rank", C.c_double), ("near_pairs", C.c_int64), ("far_pairs", C.c_int64),
                ("bytes_near", C.c_int64), ("bytes_far", C.c_int64), ("bytes_p", C.c_int64),
                ("bytes_total", C.c_int64), ("algo_bytes_matvec", C.c_int64), ("algo_bytes_near", C.c_int64),
                ("flops_matvec", C.c_int64),
                ("seconds_compress", C.c_double), ("near_tile_bytes", C.c_int64), ("near_elems", C.c_int64)]


PHASES = ["prep", "n2s", "s2s", "s2n", "l2l", "combine", "ortho", "tridiag", "compress"]


class PhaseTimes(C.Structure):
    _fields_ = [("launches", C.c_int64 * len(PHASES)), ("ms", C.c_double * len(PHASES))]


class EigInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("converged", C.c_int32),
                ("max_rel_resid", C.c_double), ("seconds", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("mem_budget_bytes", C.c_size_t), ("compressors", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("X", C.c_void_p), ("params", Params), ("r", C.c_int32), ("rel_resid_tol", C.c_double),
                ("max_basis", C.c_int32), ("arrival_s", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("r", C.c_int32), ("evals", C.c_double * 64), ("latency_s", C.c_double),
                ("service_s", C.c_double), ("iters", C.c_int32), ("x_released", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("cancelled", C.c_int64), ("solves_per_s", C.c_double),
                ("p50_latency_s", C.c_double), ("p99_latency_s", C.c_double), ("peak_resident_bytes", C.c_int64),
                ("shared_launches", C.c_int64)]


_lib = None


def declared_symbols():
    """Entry points declared in include/hdm.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hdm_[a-z_0-9]+)\s*\(", text)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2311_06115_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
    sig = {
        "hdm_last_error": (C.c_char_p, []),
        "hdm_version": (C.c_char_p, []),
        "hdm_params_default": (None, [C.POINTER(Params)]),
        "hdm_params_validate": (st, [C.POINTER(Params)]),
        "hdm_ctx_create": (st, [C.c_int, C.c_size_t, C.POINTER(vp)]),
        "hdm_ctx_destroy": (st, [vp]),
        "hdm_ctx_profile": (st, [vp, C.c_int]),
        "hdm_ctx_phase_times": (st, [vp, C.POINTER(PhaseTimes)]),
        "hdm_ctx_graphs": (st, [vp, C.c_int]),
        "hdm_ctx_profile_phases": (st, [vp, C.c_uint32]),
        "hdm_compress": (st, [vp, vp, C.c_int, C.POINTER(Params), vp, C.POINTER(vp)]),
        "hdm_op_destroy": (st, [vp]),
        "hdm_op_stats": (st, [vp, C.POINTER(OpStats)]),
        "hdm_op_perm": (st, [vp, vp]),
        "hdm_op_knn": (st, [vp, vp, vp]),
        "hdm_op_lists": (st, [vp, vp, vp, C.POINTER(i64), vp, vp, C.POINTER(i64)]),
        "hdm_op_ranks": (st, [vp, vp, vp, vp]),
        "hdm_op_node": (st, [vp, i64, vp, vp, vp]),
        "hdm_op_degrees": (st, [vp, vp, vp, vp]),
        "hdm_matvec": (st, [vp, C.c_int, vp, vp, i32, vp]),
        "hdm_matvec_noalloc": (st, [vp, C.c_int, vp, vp, i32, vp]),
        "hdm_eigs": (st, [vp, i32, f64, i32, i32, C.c_uint64, vp, vp, C.POINTER(EigInfo), vp]),
        "hdm_diffusion_map": (st, [vp, i32, vp, vp, i32, f64, vp, vp, vp, C.POINTER(i32), vp]),
        "hdm_server_create": (st, [vp, C.POINTER(ServerCfg), C.POINTER(vp)]),
        "hdm_submit": (st, [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "hdm_poll": (st, [vp, C.c_uint64, C.POINTER(Result)]),
        "hdm_cancel": (st, [vp, C.c_uint64]),
        "hdm_server_stats": (st, [vp, C.POINTER(ServerStats)]),
        "hdm_server_destroy": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status):
    if status != 0:
        raise HdmError(status, lib().hdm_last_error().decode())
    return status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_params() -> Params:
    p = Params()
    lib().hdm_params_default(C.byref(p))
    return p


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.h = C.c_void_p()
        check(lib().hdm_ctx_create(device, budget_bytes, C.byref(self.h)))
        self.device = device

    def profile(self, enable: bool, phases=None):
        """Time every phase (or only the named ones, e.g. phases=["l2l"]) until profile(False)."""
        if phases is None or not enable:
            check(lib().hdm_ctx_profile(self.h, int(enable)))
        else:
            mask = 0
            for name in phases:
                mask |= 1 << PHASES.index(name)
            check(lib().hdm_ctx_profile_phases(self.h, mask))

    def graphs(self, enable: bool):
        """hdm_matvec replays a HIP graph (True) or launches its kernels one by one (False, the default)."""
        check(lib().hdm_ctx_graphs(self.h, int(enable)))

    def phase_times(self):
        """{phase: (launches, milliseconds)} recorded since profile(True)."""
        pt = PhaseTimes()
        check(lib().hdm_ctx_phase_times(self.h, C.byref(pt)))
        return {name: (pt.launches[i], pt.ms[i]) for i, name in enumerate(PHASES)}

    def close(self):
        if self.h:
            lib().hdm_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def make_params(X, eps, m, s, tau, k, seed, near_prec="f32", far_prec=None, budget=0.05, knn_iters=10) -> Params:
    p = default_params()
    p.n, p.dim = int(X.shape[0]), int(X.shape[1])
    p.x_dtype = U8 if X.dtype == np.uint8 else F64
    p.eps, p.leaf_m, p.max_rank_s, p.tau, p.knn_k = float(eps), int(m), int(s), float(tau), int(k)
    p.knn_iters, p.budget, p.seed = int(knn_iters), float(budget), int(seed)
    p.near_prec = PREC[near_prec]
    p.far_prec = PREC[far_prec or near_prec]
    return p


class Operator:
    """Compressed diffusion-maps operator resident in HBM (hdm_op)."""

    def __init__(self, X, eps, m, s, tau, k, seed, near_prec="f32", far_prec=None, budget=0.05, knn_iters=10,
                 ctx: Context | None = None):
        import torch
        self.torch = torch
        self.ctx = ctx or context(0)
        on_device = isinstance(X, torch.Tensor) and X.is_cuda
        if on_device:
            if X.dtype not in (torch.uint8, torch.float64) or not X.is_contiguous():
                raise ValueError("device points must be contiguous float64 or uint8")
            shape_src = np.empty((X.shape[0], X.shape[1]), np.uint8 if X.dtype == torch.uint8 else np.float64)
            xptr = C.c_void_p(X.data_ptr())
        else:
            Xh = X.detach().cpu().numpy() if isinstance(X, torch.Tensor) else np.asarray(X)
            Xh = np.ascontiguousarray(Xh if Xh.dtype == np.uint8 else Xh.astype(np.float64))
            shape_src = Xh
            xptr = _ptr(Xh)
        self.params = make_params(shape_src, eps, m, s, tau, k, seed, near_prec, far_prec, budget, knn_iters)
        self.n, self.dim, self.k = shape_src.shape[0], shape_src.shape[1], int(k)
        self.h = C.c_void_p()
        check(lib().hdm_compress(self.ctx.h, xptr, int(on_device), C.byref(self.params), _stream(torch),
                                 C.byref(self.h)))
        st = self.stats()
        self.depth, self.L = st.depth, st.leaves
        self.nnodes = 2 * self.L

    def close(self):
        if getattr(self, "h", None):
            lib().hdm_op_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inspection ------------------------------------------------------
    def stats(self) -> OpStats:
        st = OpStats()
        check(lib().hdm_op_stats(self.h, C.byref(st)))
        return st

    def perm(self):
        p = np.zeros(self.n, np.int32)
        check(lib().hdm_op_perm(self.h, _ptr(p)))
        return p

    def knn(self):
        idx = np.zeros((self.n, self.k), np.int32)
        d2 = np.zeros((self.n, self.k), np.float64)
        check(lib().hdm_op_knn(self.h, _ptr(idx), _ptr(d2)))
        return idx, d2

    def near(self):
        nn, fn = C.c_int64(), C.c_int64()
        check(lib().hdm_op_lists(self.h, None, None, C.byref(nn), None, None, C.byref(fn)))
        off = np.zeros(self.L + 1, np.int32)
        idx = np.zeros(max(nn.value, 1), np.int32)
        check(lib().hdm_op_lists(self.h, _ptr(off), _ptr(idx), C.byref(nn), None, None, C.byref(fn)))
        return off, idx[:nn.value]

    def far(self):
        nn, fn = C.c_int64(), C.c_int64()
        check(lib().hdm_op_lists(self.h, None, None, C.byref(nn), None, None, C.byref(fn)))
        off = np.zeros(self.nnodes + 1, np.int32)
        idx = np.zeros(max(fn.value, 1), np.int32)
        check(lib().hdm_op_lists(self.h, None, None, C.byref(nn), _ptr(off), _ptr(idx), C.byref(fn)))
        return off, idx[:fn.value]

    def ranks(self):
        r = np.zeros(self.nnodes, np.int32)
        c = np.zeros(self.nnodes, np.int32)
        nr = np.zeros(self.nnodes, np.int32)
        check(lib().hdm_op_ranks(self.h, _ptr(r), _ptr(c), _ptr(nr)))
        return r, c, nr

    def node(self, h):
        r, c, nr = self.ranks()
        skel = np.zeros(max(r[h], 1), np.int32)
        rows = np.zeros(max(nr[h], 1), np.int32)
        P = np.zeros(max(r[h] * c[h], 1), np.float64)
        check(lib().hdm_op_node(self.h, int(h), _ptr(skel), _ptr(rows), _ptr(P)))
        return skel[:r[h]], rows[:nr[h]], P[:r[h] * c[h]].reshape(r[h], c[h])

    def degrees(self):
        q, d, c = (np.zeros(self.n) for _ in range(3))
        check(lib().hdm_op_degrees(self.h, _ptr(q), _ptr(d), _ptr(c)))
        return q, d, c

    # ---- products and eigenpairs -------------------------------------------
    def matvec(self, x, normalised: bool = False):
        """y = K~ x (or S~ x); x: float64 cuda tensor (n,) or (n, nrhs)."""
        torch = self.torch
        x = x.to(dtype=torch.float64)
        vec = x.dim() == 1
        X = x.reshape(self.n, -1).t().contiguous()   # column-major n x nrhs
        Y = torch.empty_like(X)
        check(lib().hdm_matvec(self.h, int(normalised), C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                               X.shape[0], _stream(torch)))
        Y = Y.t()
        return Y[:, 0] if vec else Y

    def matvec_noalloc(self, x, out, normalised: bool = False):
        """hdm_matvec_noalloc: out = K~ x (or S~ x) with the library's scratch array as
        the only workspace; x and out: float64 cuda tensors of shape (nrhs, n)
        (column-major n x nrhs), allocated by the caller."""
        torch = self.torch
        assert x.dtype == torch.float64 and out.dtype == torch.float64 and x.is_contiguous() and out.is_contiguous()
        assert x.shape == out.shape and x.shape[-1] == self.n
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        check(lib().hdm_matvec_noalloc(self.h, int(normalised), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                       nrhs, _stream(torch)))
        return out

    def eigs(self, r, tol=1e-10, block=1, max_basis=0, seed=0, vectors=True):
        torch = self.torch
        evals = np.zeros(r)
        info = EigInfo()
        vecs = torch.empty((r, self.n), dtype=torch.float64, device=f"cuda:{self.ctx.device}") if vectors else None
        st = lib().hdm_eigs(self.h, int(r), float(tol), int(block), int(max_basis), int(seed), _ptr(evals),
                            C.c_void_p(vecs.data_ptr()) if vectors else None, C.byref(info), _stream(torch))
        if st not in (0, 4):
            check(st)
        return evals, (vecs.t() if vectors else None), info, st


def diffusion_map(op, evals, vecs, t=1, delta=0.1):
    """hdm_diffusion_map: psi = phi / sqrt(d), lambda^t, the coordinates lambda^t psi and
    d(t), from the eigenpairs hdm_eigs returned (evals numpy [r], vecs cuda [n, r])."""
    torch = op.torch
    ev = np.ascontiguousarray(evals, dtype=np.float64)
    r = ev.shape[0]
    phi = vecs.t().contiguous()   # r x n: column-major n x r
    psi = torch.empty_like(phi)
    coords = torch.empty_like(phi)
    lt = np.zeros(r, np.float64)
    dim = C.c_int32()
    check(lib().hdm_diffusion_map(op.h, r, _ptr(ev), C.c_void_p(phi.data_ptr()), int(t), float(delta),
                                  C.c_void_p(psi.data_ptr()), C.c_void_p(coords.data_ptr()), _ptr(lt), C.byref(dim),
                                  _stream(torch)))
    return psi.t(), coords.t(), lt, dim.value


def linear_operator(op, normalised=True):
    """A scipy LinearOperator whose products run on the GPU through hdm_matvec (the
    paper's integration: scipy's eigsh drives the compressed operator's matvec).
    Host float64 vectors in and out; only the copies and the call are done here."""
    import scipy.sparse.linalg as spla
    torch = op.torch

    def mv(x):
        X = np.asarray(x, dtype=np.float64).reshape(op.n, -1)
        Y = op.matvec(torch.from_numpy(np.ascontiguousarray(X)).cuda(), normalised=normalised).cpu().numpy()
        return Y.reshape(np.shape(x)) if np.ndim(x) == 1 else Y

    return spla.LinearOperator((op.n, op.n), matvec=mv, matmat=mv, rmatvec=mv, dtype=np.float64)


class Server:
    """Continuous-batching eigensolve server (hdm_server_*)."""

    def __init__(self, ctx: Context | None = None, max_slots: int = 4, mem_budget_bytes: int = 0,
                 compressors: int = 2):
        self.ctx = ctx or context(0)
        cfg = ServerCfg(max_slots, mem_budget_bytes, compressors)
        self.h = C.c_void_p()
        check(lib().hdm_server_create(self.ctx.h, C.byref(cfg), C.byref(self.h)))

    def submit(self, X, eps, m, s, tau, k, seed, r, tol=1e-6, near_prec="f32", far_prec=None, budget=0.05,
               knn_iters=10, max_basis=0, arrival_s=0.0) -> int:
        Xh = np.asarray(X)
        Xh = np.ascontiguousarray(Xh if Xh.dtype == np.uint8 else Xh.astype(np.float64))
        req = Request()
        req.X = _ptr(Xh)
        req.params = make_params(Xh, eps, m, s, tau, k, seed, near_prec, far_prec, budget, knn_iters)
        req.r, req.rel_resid_tol, req.max_basis, req.arrival_s = int(r), float(tol), int(max_basis), float(arrival_s)
        t = C.c_uint64()
        check(lib().hdm_submit(self.h, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket):
        """None while pending, else a dict with status, eigenvalues and latencies."""
        res = Result()
        st = lib().hdm_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if st == 5:
            return None
        check(st)
        return dict(status=res.status, evals=np.array(res.evals[:res.r]), latency_s=res.latency_s,
                    service_s=res.service_s, iters=res.iters, x_released=res.x_released)

    def wait(self, ticket, timeout=120.0):
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            time.sleep(0.0005)

    def cancel(self, ticket):
        check(lib().hdm_cancel(self.h, C.c_uint64(ticket)))

    def stats(self):
        st = ServerStats()
        check(lib().hdm_server_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().hdm_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

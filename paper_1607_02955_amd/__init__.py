"""Current-flow closeness on AMD Instinct MI355X: Python binding of libcfc.

A thin ctypes layer over the C ABI in include/cfc.h (argument marshalling
only; every step of the solve runs in the library's HIP kernels).  PyTorch
provides the HIP stream and, through its caching allocator, device memory.

    import paper_1607_02955_amd as cfc
    ctx = cfc.Context()                      # cuda:0, torch's current stream
    g = cfc.Graph(ctx, n, u, v, w)           # undirected, w = conductances
    g.build_hierarchy()
    far, clo = g.farness_sampling(nodes, k=20, seed=1)
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (COL_DIVERGED, COL_NOT_CONVERGED, COL_OK, COL_SKIPPED, LCC_ONLY, PREC_FP64,
                   PREC_MIXED, QUERY_JL, QUERY_SAMPLING, REJECT_PARALLEL, CfcError, check, lib)

__all__ = ["Context", "Graph", "Server", "CfcError", "sampling_pivots", "jl_sign_word", "shared_pivots",
           "random_pairs", "version",
           "LCC_ONLY", "REJECT_PARALLEL", "PREC_MIXED", "PREC_FP64", "QUERY_JL", "QUERY_SAMPLING",
           "COL_OK", "COL_NOT_CONVERGED", "COL_DIVERGED", "COL_SKIPPED", "solve_params"]


# Live handles, closed in dependency order (servers, graphs, contexts) at
# interpreter exit while the host runtime and torch are still intact.
_live = {"server": weakref.WeakSet(), "graph": weakref.WeakSet(), "ctx": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("server", "graph", "ctx"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def version() -> str:
    return lib().cfc_version().decode()


def sampling_pivots(seed: int, node: int, n: int, k: int) -> np.ndarray:
    """The Sampling estimator's pivot set for one query node."""
    out = np.empty(min(k, n), np.int64)
    check(lib().cfc_sampling_pivots(seed, node, n, k, _p(out, C.c_int64)))
    return out


def jl_sign_word(seed: int, word: int, lo: int, hi: int) -> int:
    return int(lib().cfc_jl_sign_word(seed, word, lo, hi))


def shared_pivots(seed: int, n: int, k: int) -> np.ndarray:
    """The pivot set shared by all query nodes (shared-pivot Sampling)."""
    out = np.empty(min(k, n), np.int64)
    check(lib().cfc_shared_pivots(seed, n, k, _p(out, C.c_int64)))
    return out


def random_pairs(seed: int, n: int, count: int):
    """The source/sink pairs drawn by sampled current-flow betweenness."""
    s, t = np.empty(count, np.int64), np.empty(count, np.int64)
    check(lib().cfc_random_pairs(seed, n, count, _p(s, C.c_int64), _p(t, C.c_int64)))
    return s, t


def solve_params(tol=1e-6, precision=PREC_MIXED, block=0, max_refine=20, max_inner=300,
                 inner_tol=0.0, use_graph=0, check_every=1, levels=0) -> _lib.SolveParams:
    return _lib.SolveParams(tol, precision, block, max_refine, max_inner, inner_tol, use_graph,
                            check_every, levels, 0)


def setup_params(coarsest_max=512, agg_cap=8, test_vectors=8, relax_sweeps=8, omega=0.8,
                 mu=1.5, seed=1, eliminate=1, device=1, order=0, max_complexity=0.0,
                 elim_degree=0, nest=0) -> _lib.SetupParams:
    """max_complexity: operator-complexity budget (0 = the default 2.0, a
    negative value = none).  elim_degree: largest degree of an eliminated
    node (0 = the default 4).  nest: 1 = the numbering nests every
    aggregation level, 2 = only the levels the solver gets, 0 = auto."""
    pct = 0 if max_complexity == 0 else (-1 if max_complexity < 0 else int(round(100 * max_complexity)))
    return _lib.SetupParams(coarsest_max, agg_cap, test_vectors, relax_sweeps, omega, mu, seed,
                            eliminate, device, order, pct, elim_degree, nest)


class Context:
    """A device (or host-only, device=-1) context.

    On a device the library launches on torch's current stream of that device
    and allocates through torch's caching allocator unless ``torch_memory`` is
    False (then hipMalloc).  ``hbm_budget`` caps the bytes the context holds.
    """

    def __init__(self, device: int = 0, torch_memory: bool = True, hbm_budget: int = 0,
                 stream: Optional[int] = None):
        self._keep = []
        opts = _lib.CtxOpts()
        opts.device = device
        opts.hbm_budget = hbm_budget
        opts.stream = None
        if device >= 0:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible to torch; use device=-1 for host-only setup")
            dev = torch.device("cuda", device)
            s = torch.cuda.current_stream(dev) if stream is None else None
            opts.stream = s.cuda_stream if s is not None else stream
            self._stream = s
            if torch_memory:
                st = opts.stream
                t_alloc = torch.cuda.caching_allocator_alloc
                t_free = torch.cuda.caching_allocator_delete

                def _alloc(nbytes, user):
                    try:
                        return t_alloc(int(nbytes), device, st)
                    except Exception:
                        return None

                def _free(ptr, user):
                    try:
                        t_free(ptr)
                    except Exception:
                        pass  # interpreter shutdown: the caching allocator is gone

                a, f = _lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free)
                self._keep += [a, f]
                opts.alloc, opts.free = a, f
        h = C.c_void_p()
        check(lib().cfc_ctx_create(C.byref(opts), C.byref(h)))
        self.handle = h
        self.device = device
        _live["ctx"].add(self)

    def device_copy(self, dst, src, nbytes=None):
        """cfc_device_copy: the library's streaming copy kernel between two
        device tensors (a bandwidth probe; waits for the copy)."""
        nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
        check(lib().cfc_device_copy(self.handle, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                    nbytes))

    def close(self):
        if getattr(self, "handle", None):
            lib().cfc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An undirected graph with conductance weights, loaded into a context."""

    def __init__(self, ctx: Context, n: int, u, v, w=None, flags: int = 0):
        self.ctx = ctx
        u, v = _i64(u), _i64(v)
        if u.shape != v.shape:
            raise ValueError("u and v differ in length")
        wp = None
        if w is not None:
            w = _f64(w)
            if w.shape != u.shape:
                raise ValueError("w differs in length from u")
            wp = _p(w, C.c_double)
        h = C.c_void_p()
        check(lib().cfc_graph_load(ctx.handle, n, u.shape[0], _p(u, C.c_int64), _p(v, C.c_int64),
                                   wp, flags, C.byref(h)))
        self.handle = h
        _live["graph"].add(self)
        inf = self.info()
        self.n = inf["n"]
        self.m = inf["m"]

    @classmethod
    def from_edgelist(cls, ctx, g, flags=0):
        return cls(ctx, g.n, g.u, g.v, g.w, flags)

    def close(self):
        if getattr(self, "handle", None):
            lib().cfc_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = _lib.GraphInfo()
        check(lib().cfc_graph_get_info(self.handle, C.byref(i)))
        L = i.levels
        return {"n": i.n, "m": i.m, "input_n": i.input_n, "levels": L,
                "unit_weights": bool(i.unit_weights), "level_n": list(i.level_n[:L]),
                "level_nnz": list(i.level_nnz[:L]), "operator_complexity": i.operator_complexity,
                "setup_ms": i.setup_ms, "device_bytes": i.device_bytes, "max_degree": i.max_degree,
                "eliminated": i.eliminated, "cycle_complexity": i.cycle_complexity}

    def node_map(self) -> np.ndarray:
        out = np.empty(self.n, np.int64)
        check(lib().cfc_graph_node_map(self.handle, _p(out, C.c_int64)))
        return out

    def build_hierarchy(self, **kw):
        p = setup_params(**kw)
        check(lib().cfc_hierarchy_build(self.handle, C.byref(p)))
        return self

    def level(self, l: int) -> dict:
        """Copies of the host arrays of hierarchy level l."""
        v = _lib.LevelView()
        check(lib().cfc_hierarchy_level(self.handle, l, C.byref(v)))
        n, nnz, nc = v.n, v.nnz, v.n_coarse

        def arr(ptr, cnt, dt):
            if not ptr or cnt == 0:
                return None if not ptr else np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(cnt,)).astype(dt, copy=True)
        out = {"n": n, "nnz": nnz, "n_coarse": nc,
               "row_ptr": arr(v.row_ptr, n + 1, np.int32), "col": arr(v.col, nnz, np.int32),
               "w": arr(v.w, nnz, np.float64), "deg": arr(v.deg, n, np.float64),
               "agg": arr(v.agg, n, np.int32), "agg_ptr": arr(v.agg_ptr, nc + 1, np.int32),
               "perm": arr(v.perm, n, np.int32)}
        cp = arr(v.coarse_pinv, n * n, np.float64)
        out["coarse_pinv"] = None if cp is None else cp.reshape(n, n)
        out["elimination"] = bool(v.elimination)
        out["elim_nb"] = (arr(v.elim_nb, _lib.ELIM_MAX_DEGREE * (n - nc), np.int32)
                          .reshape(n - nc, _lib.ELIM_MAX_DEGREE) if v.elimination else None)
        return out

    # ---- solves ----
    def solve(self, B, stats=False, **kw):
        """Solve L X = B.  B: float64 array (n,) or (nrhs, n) -- numpy or a torch
        tensor (host or device, contiguous).  Returns X of the same kind."""
        allow = kw.pop("allow_unconverged", False)
        p = solve_params(**kw)
        st = _lib.SolveStats()
        try:
            import torch
            is_t = isinstance(B, torch.Tensor)
        except ImportError:
            is_t = False
        if is_t:
            Bt = B.detach().to(torch.float64).contiguous()
            one = Bt.dim() == 1
            Bt = Bt.reshape(-1, self.n)
            X = torch.empty_like(Bt)
            status = np.empty(Bt.shape[0], np.int32)
            if Bt.is_cuda:
                torch.cuda.current_stream(Bt.device).synchronize()
            rc = lib().cfc_solve(self.handle, Bt.shape[0], C.c_void_p(Bt.data_ptr()),
                                 C.c_void_p(X.data_ptr()), C.byref(p), C.byref(st),
                                 _p(status, C.c_int32))
            out = X.reshape(-1) if one else X
        else:
            Bn = _f64(B)
            one = Bn.ndim == 1
            Bn = Bn.reshape(-1, self.n)
            X = np.empty_like(Bn)
            status = np.empty(Bn.shape[0], np.int32)
            rc = lib().cfc_solve(self.handle, Bn.shape[0], Bn.ctypes.data_as(C.c_void_p),
                                 X.ctypes.data_as(C.c_void_p), C.byref(p), C.byref(st),
                                 _p(status, C.c_int32))
            out = X.reshape(-1) if one else X
        if rc != 0 and rc != -5:
            check(rc)
        if rc == -5 and not allow:
            check(rc)
        return (out, st.as_dict(), status) if stats else out

    def resistance(self, s, t, stats=False, **kw):
        s, t = _i64(s).ravel(), _i64(t).ravel()
        r = np.empty(s.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_resistance(self.handle, s.shape[0], _p(s, C.c_int64), _p(t, C.c_int64),
                                   _p(r, C.c_double), C.byref(p), C.byref(st)))
        return (r, st.as_dict()) if stats else r

    def farness_exact(self, nodes, stats=False, **kw):
        nodes = _i64(nodes).ravel()
        far, clo = np.empty(nodes.shape[0]), np.empty(nodes.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_farness_exact(self.handle, nodes.shape[0], _p(nodes, C.c_int64),
                                      _p(far, C.c_double), _p(clo, C.c_double), C.byref(p), C.byref(st)))
        return (far, clo, st.as_dict()) if stats else (far, clo)

    def farness_jl_static(self, nodes=None, far=None, clo=None):
        """cfc_farness_jl_static: projection farness and closeness without
        any device allocation (at most 262,144 nodes per call).  nodes,
        far and clo may be numpy arrays or device tensors (int64 / float64,
        contiguous); nodes None means every node.  Returns (far, clo)."""
        def ptr(a):
            return C.c_void_p(a.data_ptr()) if hasattr(a, "data_ptr") else a.ctypes.data_as(C.c_void_p)
        if nodes is None:
            q, np_nodes = self.n, None
        else:
            if not hasattr(nodes, "data_ptr"):
                nodes = _i64(nodes).ravel()
            q, np_nodes = int(nodes.shape[0]), nodes
        far = np.empty(q) if far is None else far
        clo = np.empty(q) if clo is None else clo
        check(lib().cfc_farness_jl_static(self.handle, q, None if np_nodes is None else ptr(np_nodes),
                                          ptr(far), ptr(clo)))
        return far, clo

    def farness_sampling(self, nodes, k, seed=1, stats=False, **kw):
        nodes = _i64(nodes).ravel()
        far, clo = np.empty(nodes.shape[0]), np.empty(nodes.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_farness_sampling(self.handle, nodes.shape[0], _p(nodes, C.c_int64), k, seed,
                                         _p(far, C.c_double), _p(clo, C.c_double), C.byref(p),
                                         C.byref(st)))
        return (far, clo, st.as_dict()) if stats else (far, clo)

    def jl_sketch(self, k, seed=1, stats=False, **kw):
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_jl_sketch(self.handle, k, seed, C.byref(p), C.byref(st)))
        return st.as_dict() if stats else self

    def farness_jl(self, nodes=None):
        """Projection farness and closeness of ``nodes`` (None: every node)."""
        if nodes is None:
            n = self.n
            far, clo = np.empty(n), np.empty(n)
            check(lib().cfc_farness_jl(self.handle, n, None, _p(far, C.c_double), _p(clo, C.c_double)))
            return far, clo
        nodes = _i64(nodes).ravel()
        far, clo = np.empty(nodes.shape[0]), np.empty(nodes.shape[0])
        check(lib().cfc_farness_jl(self.handle, nodes.shape[0], _p(nodes, C.c_int64),
                                   _p(far, C.c_double), _p(clo, C.c_double)))
        return far, clo

    def farness_sampling_shared(self, nodes, k, seed=1, stats=False, **kw):
        nodes = _i64(nodes).ravel()
        far, clo = np.empty(nodes.shape[0]), np.empty(nodes.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_farness_sampling_shared(self.handle, nodes.shape[0], _p(nodes, C.c_int64), k,
                                                seed, _p(far, C.c_double), _p(clo, C.c_double),
                                                C.byref(p), C.byref(st)))
        return (far, clo, st.as_dict()) if stats else (far, clo)

    def spanning_edge(self, u, v, stats=False, **kw):
        u, v = _i64(u).ravel(), _i64(v).ravel()
        c = np.empty(u.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_spanning_edge(self.handle, u.shape[0], _p(u, C.c_int64), _p(v, C.c_int64),
                                      _p(c, C.c_double), C.byref(p), C.byref(st)))
        return (c, st.as_dict()) if stats else c

    def spanning_edge_jl(self, u, v, k, seed=1, stats=False, **kw):
        u, v = _i64(u).ravel(), _i64(v).ravel()
        c = np.empty(u.shape[0])
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_spanning_edge_jl(self.handle, u.shape[0], _p(u, C.c_int64), _p(v, C.c_int64),
                                         k, seed, _p(c, C.c_double), C.byref(p), C.byref(st)))
        return (c, st.as_dict()) if stats else c

    def current_throughput(self, s, t, stats=False, **kw):
        s, t = _i64(s).ravel(), _i64(t).ravel()
        tau = np.empty(self.n)
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_current_throughput(self.handle, s.shape[0], _p(s, C.c_int64), _p(t, C.c_int64),
                                           _p(tau, C.c_double), C.byref(p), C.byref(st)))
        return (tau, st.as_dict()) if stats else tau

    def cfb_exact(self, stats=False, **kw):
        cb = np.empty(self.n)
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_cfb_exact(self.handle, _p(cb, C.c_double), C.byref(p), C.byref(st)))
        return (cb, st.as_dict()) if stats else cb

    def cfb_sampled(self, count, seed=1, stats=False, **kw):
        cb = np.empty(self.n)
        p, st = solve_params(**kw), _lib.SolveStats()
        check(lib().cfc_cfb_sampled(self.handle, count, seed, _p(cb, C.c_double), C.byref(p),
                                    C.byref(st)))
        return (cb, st.as_dict()) if stats else cb


class Server:
    """Continuous-batching farness server over resident graphs."""

    def __init__(self, ctx: Context, slots=256, max_queue=4096, jl_k=256, sampling_k=200, seed=1,
                 tol=1e-6, hbm_budget=0):
        self.ctx = ctx
        o = _lib.ServerOpts(slots, max_queue, jl_k, sampling_k, seed, tol, hbm_budget)
        h = C.c_void_p()
        check(lib().cfc_server_create(ctx.handle, C.byref(o), C.byref(h)))
        self.handle = h
        self.graphs = []
        _live["server"].add(self)

    def add_graph(self, g: Graph) -> int:
        gid = C.c_int32()
        check(lib().cfc_server_add_graph(self.handle, g.handle, C.byref(gid)))
        self.graphs.append(g)
        return gid.value

    def submit(self, graph: int, kind: int, nodes, k: int = 0, seed: int = 0) -> int:
        nodes = _i64(nodes).ravel()
        q = _lib.Query(graph, kind, nodes.shape[0], k, _p(nodes, C.c_int64), seed)
        t = C.c_uint64()
        check(lib().cfc_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def _result(self, fn, ticket, *extra, nmax=1024):
        far, clo = np.empty(nmax), np.empty(nmax)
        r = _lib.Result(0, 0, _p(far, C.c_double), _p(clo, C.c_double), 0.0)
        rc = fn(self.handle, ticket, *extra, C.byref(r))
        if rc == -6:
            return None
        check(rc)
        if r.status != 0:
            raise CfcError(r.status, "query failed")  # e.g. CFC_E_NOMEM, CFC_E_NOT_CONVERGED
        return far[:r.nnodes].copy(), clo[:r.nnodes].copy(), r.latency_ms

    def poll(self, ticket):
        return self._result(lib().cfc_server_poll, ticket)

    def wait(self, ticket, timeout_ms=-1.0):
        return self._result(lib().cfc_server_wait, ticket, C.c_double(timeout_ms))

    def stats(self) -> dict:
        s = _lib.ServerStats()
        check(lib().cfc_server_get_stats(self.handle, C.byref(s)))
        return s.as_dict()

    def close(self):
        """Stop the workers (after the refinement step each is in) and give
        the graphs back to direct calls."""
        if getattr(self, "handle", None):
            lib().cfc_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

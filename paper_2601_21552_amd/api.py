"""Python binding of the C ABI: the same steps under the same names
(bitblast, cnf_from_arrays, split, cubes_from_arrays, solve, decide and the
result getters).  Only argument marshalling happens here; every step runs in
``libscuba.so`` (host C++ and gfx950 kernels).  torch provides the device
workspace and the stream."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib as L

_P = C.c_void_p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P) if a is not None and a.size else None


class _Handle:
    _free = None

    def __init__(self, ctx: "Context", h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and self._free and L is not None and L._lib is not None:
            getattr(L._lib, self._free)(self.h)
            self.h = None


class Cnf(_Handle):
    _free = "scuba_cnf_free"

    def __len__(self):
        return L.load().scuba_cnf_count(self.h)

    def view(self, qi: int) -> dict:
        v = L.CnfView()
        self.ctx._check(L.load().scuba_cnf_view_get(self.h, qi, C.byref(v)))
        off = np.ctypeslib.as_array(v.clause_off, shape=(v.n_clauses + 1,)).copy()
        lits = (np.ctypeslib.as_array(v.lits, shape=(v.n_lits,)).copy()
                if v.n_lits else np.zeros(0, np.int32))
        return dict(n_vars=v.n_vars, n_inputs=v.n_inputs, n_clauses=v.n_clauses,
                    clause_off=off, lits=lits, root_unsat=bool(v.root_unsat))

    def sizes(self, qi: int) -> dict:
        """n_vars, n_clauses, n_lits and root_unsat of one query (no copy)."""
        v = L.CnfView()
        self.ctx._check(L.load().scuba_cnf_view_get(self.h, qi, C.byref(v)))
        return dict(n_vars=v.n_vars, n_clauses=v.n_clauses, n_lits=v.n_lits, root_unsat=bool(v.root_unsat))

    def input_map(self, qi: int):
        n = self.view(qi)["n_inputs"]
        first = np.zeros(max(n, 1), np.uint32)
        width = np.zeros(max(n, 1), np.uint32)
        self.ctx._check(L.load().scuba_cnf_input_map(self.h, qi, _ptr(first), _ptr(width), n))
        return first[:n], width[:n]


class Cubes(_Handle):
    _free = "scuba_cubes_free"

    def view(self, qi: int) -> dict:
        v = L.CubesView()
        self.ctx._check(L.load().scuba_cubes_view_get(self.h, qi, C.byref(v)))
        n = v.n_cubes
        off = np.ctypeslib.as_array(v.cube_off, shape=(n + 1,)).copy()
        nl = int(off[-1])
        lits = np.ctypeslib.as_array(v.lits, shape=(nl,)).copy() if nl else np.zeros(0, np.int32)
        kind = np.ctypeslib.as_array(v.kind, shape=(n,)).copy() if n else np.zeros(0, np.int32)
        f = np.ctypeslib.as_array(v.f, shape=(n,)).copy() if n else np.zeros(0, np.int32)
        return dict(cube_off=off, lits=lits, kind=kind, f=f, complete=bool(v.complete),
                    cubes=[lits[off[i]:off[i + 1]].tolist() for i in range(n)])


class Results(_Handle):
    _free = "scuba_results_free"

    def __init__(self, ctx, h, nq):
        super().__init__(ctx, h)
        self.nq = nq

    def result(self, qi: int) -> dict:
        r = L.QueryResult()
        self.ctx._check(L.load().scuba_result_get(self.h, qi, C.byref(r)))
        return dict(verdict=L.VERDICT[r.verdict], how=L.HOW[r.how], cubes_total=r.cubes_total,
                    cubes_refuted=r.cubes_refuted, leaves_sent=r.leaves_sent,
                    leaves_refuted=r.leaves_refuted, blocks_evaluated=r.blocks_evaluated,
                    clause_blocks=r.clause_blocks, word_ops=r.word_ops, rounds=r.rounds,
                    witness_checked=bool(r.witness_checked))

    def verdicts(self):
        return [self.result(i)["verdict"] for i in range(self.nq)]

    def witness(self, qi: int, n_inputs: int):
        vals = np.zeros(max(n_inputs, 1), np.uint64)
        self.ctx._check(L.load().scuba_witness_get(self.h, qi, _ptr(vals), n_inputs))
        return [int(x) for x in vals[:n_inputs]]

    def model(self, qi: int, n_vars: int):
        bits = np.zeros(n_vars + 1, np.uint8)
        self.ctx._check(L.load().scuba_model_get(self.h, qi, _ptr(bits), n_vars + 1))
        return bits

    def leaf(self, qi: int, cube: int) -> dict:
        r = L.LeafResult()
        self.ctx._check(L.load().scuba_leaf_get(self.h, qi, cube, C.byref(r)))
        return dict(refuted=bool(r.refuted), f=r.f, m=r.m, count=int(r.count), first=int(r.first))

    def timing(self) -> dict:
        ms = np.zeros(19, np.float64)
        self.ctx._check(L.load().scuba_results_timing(self.h, _ptr(ms), 19))
        keys = ["split", "h2d", "kernels", "d2h", "verify", "total", "up", "leaf",
                "up_launches", "leaf_launches", "graph", "graph_launches", "graph_captures",
                "score_device", "score_passes", "score_rows", "cubes_sent", "items_sent", "fix_launches"]
        return dict(zip(keys, ms.tolist()))


def pack_queries(queries):
    """A batch of query DAGs, each (nodes: NODE_DTYPE array, roots: uint32
    array), in the layout that scuba_bitblast takes: (all node records, node
    offsets per query (nq + 1), all roots, root offsets per query (nq + 1))."""
    queries = list(queries)
    nq = len(queries)
    isz = L.NODE_DTYPE.itemsize
    nb, rb = [], []
    for n, r in queries:
        n = np.ascontiguousarray(n)
        if n.dtype.itemsize != isz:
            raise ValueError("node records must have the NODE_DTYPE layout")
        nb.append(n.view(np.uint8).reshape(-1))   # records as raw bytes
        rb.append(np.asarray(r))
    ns = np.zeros(nq + 1, np.uint64)
    rs = np.zeros(nq + 1, np.uint64)
    if nq:
        ns[1:] = np.cumsum([len(b) // isz for b in nb])
        rs[1:] = np.cumsum([len(r) for r in rb])
    an = np.concatenate(nb).view(L.NODE_DTYPE) if nq else np.zeros(0, L.NODE_DTYPE)
    ar = np.ascontiguousarray(np.concatenate(rb).astype(np.uint32, copy=False)) if nq else np.zeros(0, np.uint32)
    return an, ns, ar, rs


_SCORERS = {"static": L.SCORER_STATIC, "learned": L.SCORER_LEARNED, "word": L.SCORER_WORD}


def _scorer(scorer) -> int:
    return _SCORERS[scorer] if isinstance(scorer, str) else int(scorer)


def _solve_opts(mode=L.MODE_DECIDE, k=0, max_cubes=0, leaves_per_round=0, chunk_log2=0,
                grid=0, max_rounds=0, learned=None, scorer="static", graph=False, max_residual=0,
                device_split=False, split_batch=0, leaf="scalar"):
    """learned: an L.LearnedScorer (Mlp.scorer()) selects the learned
    ordering; otherwise scorer is "static" or "word".  device_split: split
    on the device (scuba_decide only), split_batch nodes per step.  leaf:
    the leaf-evaluation variant, "scalar", "vector" or "lds"."""
    o = L.SolveOpts()
    o.mode, o.k, o.max_cubes = mode, k, max_cubes
    o.leaves_per_round, o.chunk_log2, o.grid = leaves_per_round, chunk_log2, grid
    o.max_rounds = max_rounds
    o.scorer = _scorer(scorer)
    o.flags = (L.SOLVE_GRAPH if graph else 0) | (L.SOLVE_DEVICE_SPLIT if device_split else 0)
    o.flags |= {"scalar": 0, "vector": L.SOLVE_LEAF_VECTOR,
                "lds": L.SOLVE_LEAF_VECTOR | L.SOLVE_LEAF_LDS}[leaf]
    o.max_residual = max_residual
    o.split_batch = split_batch
    if learned is not None:
        o.scorer = L.SCORER_LEARNED
        o.learned = C.pointer(learned)
    return o


class Context:
    """One library context bound to a HIP device (opened lazily)."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        h = _P()
        st = self.lib.scuba_ctx_create(device, C.byref(h))
        if st != L.OK:
            raise L.ScubaError(st, "scuba_ctx_create")
        self.h = h
        self.device = device
        self._ws = None

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.scuba_ctx_destroy(self.h)
            self.h = None

    def _check(self, st):
        if st != L.OK:
            raise L.ScubaError(st, self.lib.scuba_last_error(self.h).decode())

    # ------------------------------------------------------------ CNF
    def bitblast(self, queries, flags: int = 0) -> Cnf:
        """queries: iterable of (nodes: NODE_DTYPE array, roots: uint32 array)."""
        return self.bitblast_packed(*pack_queries(queries), flags=flags)

    def bitblast_packed(self, nodes, node_start, roots, root_start, flags: int = 0) -> Cnf:
        """A batch already in scuba_bitblast's layout (see ``pack_queries``)."""
        an = np.ascontiguousarray(nodes)
        if an.dtype != L.NODE_DTYPE:
            raise ValueError("node records must have the NODE_DTYPE layout")
        ns = np.ascontiguousarray(node_start, dtype=np.uint64)
        ar = np.ascontiguousarray(roots, dtype=np.uint32)
        rs = np.ascontiguousarray(root_start, dtype=np.uint64)
        h = _P()
        self._check(self.lib.scuba_bitblast(self.h, len(ns) - 1, _ptr(an), _ptr(ns), _ptr(ar), _ptr(rs),
                                            flags, C.byref(h)))
        return Cnf(self, h)

    def cnf_from_arrays(self, n_vars, q_clause_start, clause_off, lits) -> Cnf:
        n_vars = np.ascontiguousarray(n_vars, dtype=np.uint32)
        qs = np.ascontiguousarray(q_clause_start, dtype=np.uint64)
        co = np.ascontiguousarray(clause_off, dtype=np.uint64)
        li = np.ascontiguousarray(lits, dtype=np.int32)
        h = _P()
        self._check(self.lib.scuba_cnf_from_arrays(self.h, len(n_vars), _ptr(n_vars), _ptr(qs),
                                                   _ptr(co), _ptr(li), C.byref(h)))
        return Cnf(self, h)

    # ------------------------------------------------------------ cubes
    def split(self, cnf: Cnf, k: int, max_cubes: int = 0, max_residual: int = 0,
              learned=None, workspace=None, stream=None, scorer="static") -> Cubes:
        """Host cube splitting; learned (an L.LearnedScorer) scores the
        branching candidates on the device."""
        o = L.SplitOpts()
        o.k, o.max_cubes, o.max_residual = k, max_cubes, max_residual
        o.scorer = _scorer(scorer)
        if learned is not None:
            nbytes = self.lib.scuba_scorer_workspace(cnf.h, learned.candidates)
            ws = self._workspace(nbytes, workspace)
            o.scorer = L.SCORER_LEARNED
            o.learned = C.pointer(learned)
            o.dev_ws, o.ws_bytes = ws.data_ptr(), ws.numel()
            o.hip_stream = self._stream(stream).value
        h = _P()
        self._check(self.lib.scuba_split(self.h, cnf.h, C.byref(o), C.byref(h)))
        return Cubes(self, h)

    def trace(self, cnf: Cnf, k: int, candidates: int = 16, every: int = 1, depth: int = 64,
              max_cubes: int = 0):
        """Training rows of the static walks: (features [rows, 16] float32,
        labels [rows] float32, nodes [rows] uint64 = query << 32 | decision)."""
        o = L.TraceOpts(k, candidates, every, depth, max_cubes)
        h = _P()
        self._check(self.lib.scuba_trace_run(self.h, cnf.h, C.byref(o), C.byref(h)))
        try:
            rows = C.c_uint64()
            fp, lp = C.POINTER(C.c_float)(), C.POINTER(C.c_float)()
            npp = C.POINTER(C.c_uint64)()
            self._check(self.lib.scuba_trace_view(h, C.byref(rows), C.byref(fp), C.byref(lp),
                                                  C.byref(npp)))
            n = rows.value
            if n == 0:
                return (np.zeros((0, 16), np.float32), np.zeros(0, np.float32),
                        np.zeros(0, np.uint64))
            f = np.ctypeslib.as_array(fp, shape=(n * 16,)).reshape(n, 16).copy()
            lab = np.ctypeslib.as_array(lp, shape=(n,)).copy()
            nodes = np.ctypeslib.as_array(npp, shape=(n,)).copy()
            return f, lab, nodes
        finally:
            self.lib.scuba_trace_free(h)

    def cubes_from_arrays(self, cnf: Cnf, cubes_per_query) -> Cubes:
        qs, off, lits = [0], [0], []
        for cubes in cubes_per_query:
            for c in cubes:
                lits.extend(int(x) for x in c)
                off.append(len(lits))
            qs.append(len(off) - 1)
        aq = np.array(qs, np.uint64)
        ao = np.array(off, np.uint64)
        al = np.array(lits or [0], np.int32)
        h = _P()
        self._check(self.lib.scuba_cubes_from_arrays(self.h, cnf.h, _ptr(aq), _ptr(ao), _ptr(al),
                                                     C.byref(h)))
        return Cubes(self, h)

    # ------------------------------------------------------------ device
    def _workspace(self, nbytes: int, workspace=None):
        import torch
        if workspace is not None:
            assert workspace.numel() * workspace.element_size() >= nbytes
            return workspace
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8,
                                   device=f"cuda:{self.device}")
        return self._ws

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return _P(s.cuda_stream)

    def solve_workspace(self, cnf: Cnf, cubes: Cubes, **opts) -> int:
        o = _solve_opts(**opts)
        n = C.c_size_t()
        self._check(self.lib.scuba_solve_workspace(self.h, cnf.h, cubes.h, C.byref(o), C.byref(n)))
        return n.value

    def decide_workspace(self, cnf: Cnf, **opts) -> int:
        o = _solve_opts(**opts)
        n = C.c_size_t()
        self._check(self.lib.scuba_decide_workspace(self.h, cnf.h, C.byref(o), C.byref(n)))
        return n.value

    def solve(self, cnf: Cnf, cubes: Cubes, workspace=None, stream=None, **opts) -> Results:
        o = _solve_opts(**opts)
        ws = self._workspace(self.solve_workspace(cnf, cubes, **opts), workspace)
        h = _P()
        self._check(self.lib.scuba_solve(self.h, cnf.h, cubes.h, C.byref(o), _P(ws.data_ptr()),
                                         ws.numel(), self._stream(stream), C.byref(h)))
        return Results(self, h, len(cnf))

    def autotune(self, cnf: Cnf, workspace=None, stream=None, **tune):
        """(decide options, report): k, chunk_log2, leaves_per_round and grid
        for this batch (see scuba_autotune); the options go to decide()."""
        t = _tune_opts(**tune)
        n = C.c_size_t()
        self._check(self.lib.scuba_autotune_workspace(self.h, cnf.h, C.byref(t), C.byref(n)))
        ws = self._workspace(n.value, workspace)
        best, rep = L.SolveOpts(), L.TuneReport()
        self._check(self.lib.scuba_autotune(self.h, cnf.h, C.byref(t), _P(ws.data_ptr()), ws.numel(),
                                            self._stream(stream), C.byref(best), C.byref(rep)))
        names = {v: k for k, v in _SCORERS.items()}
        opts = dict(k=best.k, leaves_per_round=best.leaves_per_round, chunk_log2=best.chunk_log2,
                    grid=best.grid, scorer=names[best.scorer], graph=bool(best.flags & L.SOLVE_GRAPH),
                    max_residual=best.max_residual)
        report = dict(points=rep.points, cached=bool(rep.cached), best_ms=rep.best_ms,
                      default_ms=rep.default_ms)
        return opts, report

    def decide(self, cnf: Cnf, workspace=None, stream=None, **opts) -> Results:
        o = _solve_opts(**opts)
        ws = self._workspace(self.decide_workspace(cnf, **opts), workspace)
        h = _P()
        self._check(self.lib.scuba_decide(self.h, cnf.h, C.byref(o), _P(ws.data_ptr()), ws.numel(),
                                          self._stream(stream), C.byref(h)))
        return Results(self, h, len(cnf))

    def tune_cache_save(self, path: str) -> None:
        """Persist this context's autotuner choices (JSON lines)."""
        self._check(self.lib.scuba_tune_cache_save(self.h, os.fsencode(path)))

    def tune_cache_load(self, path: str) -> int:
        """Add the choices of `path` made on this device's architecture."""
        n = C.c_uint32()
        self._check(self.lib.scuba_tune_cache_load(self.h, os.fsencode(path), C.byref(n)))
        return n.value

    def decide_noalloc(self, cnf: Cnf, stream=None, **opts) -> Results:
        """scuba_decide on the library's own device scratch (no workspace,
        no allocation in the call)."""
        o = _solve_opts(**opts)
        h = _P()
        self._check(self.lib.scuba_decide_noalloc(self.h, cnf.h, C.byref(o), self._stream(stream),
                                                  C.byref(h)))
        return Results(self, h, len(cnf))


def _tune_opts(sample=0, reps=0, max_cubes=0, scorer="static", graph=False, refresh=False):
    return L.TuneOpts(sample, reps, max_cubes, _scorer(scorer), L.SOLVE_GRAPH if graph else 0,
                      1 if refresh else 0, 0)


class Mlp:
    """Device state of the learned scorer (fp32 master parameters, their
    bf16 copy, Adam moments) and the calls of the C ABI on it.  torch
    tensors carry the device memory; every operation runs in libscuba.so."""

    F = 16
    H = 128

    def __init__(self, ctx: Context, params=None, device=None):
        import torch
        self.ctx = ctx
        self.torch = torch
        self.dev = device or f"cuda:{ctx.device}"
        n = ctx.lib.scuba_mlp_param_count()
        self.n_params = n
        if params is None:
            params = np.zeros(n, np.float32)
        params = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        assert params.size == n
        self.master = torch.tensor(params, device=self.dev)
        self.wb = torch.empty(n, dtype=torch.bfloat16, device=self.dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.step_count = 0
        self.sync()

    def _s(self):
        return _P(self.torch.cuda.current_stream().cuda_stream)

    @staticmethod
    def _p(t):
        return _P(t.data_ptr())

    def sync(self):
        self.ctx._check(self.ctx.lib.scuba_mlp_sync(self.ctx.h, self._p(self.master), self._p(self.wb),
                                                     self._s()))

    def forward(self, x):
        """x: [B, 16] bf16 device tensor -> (y [B] fp32, a1, a2)."""
        torch = self.torch
        B = x.shape[0]
        a1 = torch.empty((B, self.H), dtype=torch.bfloat16, device=self.dev)
        a2 = torch.empty((B, self.H), dtype=torch.bfloat16, device=self.dev)
        y = torch.empty(B, dtype=torch.float32, device=self.dev)
        x = x.contiguous()
        self.ctx._check(self.ctx.lib.scuba_mlp_forward(self.ctx.h, self._p(self.wb), self._p(self.master),
                                                        self._p(x), B, self._p(a1), self._p(a2),
                                                        self._p(y), self._s()))
        return y, a1, a2

    def backward(self, x, a1, a2, y, target):
        """Gradient of the mean squared error into self.grad."""
        torch = self.torch
        B = x.shape[0]
        dz1 = torch.empty((B, self.H), dtype=torch.bfloat16, device=self.dev)
        dz2 = torch.empty((B, self.H), dtype=torch.bfloat16, device=self.dev)
        target = target.contiguous().float()
        self.ctx._check(self.ctx.lib.scuba_mlp_backward(
            self.ctx.h, self._p(self.wb), self._p(x.contiguous()), self._p(a1), self._p(a2), self._p(y),
            self._p(target), B, self._p(dz1), self._p(dz2), self._p(self.grad), self._s()))
        return self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        self.ctx._check(self.ctx.lib.scuba_mlp_adam(
            self.ctx.h, self._p(self.master), self._p(self.grad), self._p(self.m), self._p(self.v),
            self._p(self.wb), self.step_count, lr, beta1, beta2, eps, self._s()))

    def params(self) -> np.ndarray:
        return self.master.detach().cpu().numpy().copy()

    def scorer(self, candidates: int = 16, rescore: int = 1) -> "L.LearnedScorer":
        """The learned-ordering option for split/decide (keeps this Mlp's
        device parameters alive while it is referenced)."""
        s = L.LearnedScorer(self.master.data_ptr(), self.wb.data_ptr(), candidates, rescore)
        s._owner = self
        return s


def mlp_flatten(p: dict) -> np.ndarray:
    """Parameter dict (W1, b1, W2, b2, w3, b3) -> the C ABI's flat layout."""
    return np.concatenate([np.asarray(p[k], np.float32).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def mlp_unflatten(v: np.ndarray, F: int = 16, H: int = 128) -> dict:
    v = np.asarray(v, np.float32)
    sizes = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp).copy()
        o += n
    return out

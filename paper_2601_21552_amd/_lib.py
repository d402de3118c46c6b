"""ctypes declarations of the C ABI in ``include/scuba.h`` (argument
marshalling only).  Loading fails loudly when ``libscuba.so`` has not been
built: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscuba.so")

OK = 0
STATUS = {0: "ok", -1: "invalid input", -2: "width", -3: "nomem", -4: "device",
          -5: "capacity", -6: "state", -7: "internal"}
SAT, UNSAT, UNKNOWN = 1, 0, 2
VERDICT = {1: "SAT", 0: "UNSAT", 2: "UNKNOWN"}
HOW = {0: "root", 1: "device", 2: "budget"}
MODE_DECIDE, MODE_COUNT = 0, 1


def BB_WRAP(m: int) -> int:
    """Bit-blast flag: machine integers of m bits (1..64)."""
    return int(m) << 8


SCORER_STATIC, SCORER_LEARNED, SCORER_WORD = 0, 1, 2
SOLVE_GRAPH = 1
SOLVE_DEVICE_SPLIT = 2
SOLVE_LEAF_VECTOR = 4
SOLVE_LEAF_LDS = 8
NOALLOC_SCRATCH_BYTES = 128 << 20   # device scratch of scuba_decide_noalloc
CUBE_LEAF, CUBE_REFUTED, CUBE_PRUNED = 0, 1, 2
BB_NO_REWRITE = 1

# scuba_node: {u32 op, a, b, width; u64 imm} (24 bytes)
NODE_DTYPE = np.dtype([("op", "<u4"), ("a", "<u4"), ("b", "<u4"),
                       ("width", "<u4"), ("imm", "<u8")])


class CnfView(C.Structure):
    _fields_ = [("n_vars", C.c_uint32), ("n_inputs", C.c_uint32),
                ("n_clauses", C.c_uint64), ("n_lits", C.c_uint64),
                ("clause_off", C.POINTER(C.c_uint64)), ("lits", C.POINTER(C.c_int32)),
                ("root_unsat", C.c_int32)]


class LearnedScorer(C.Structure):
    _fields_ = [("master", C.c_void_p), ("wbf16", C.c_void_p),
                ("candidates", C.c_uint32), ("rescore", C.c_uint32)]


class SplitOpts(C.Structure):
    _fields_ = [("k", C.c_uint32), ("scorer", C.c_uint32), ("max_cubes", C.c_uint64),
                ("max_residual", C.c_uint32), ("reserved", C.c_uint32),
                ("learned", C.POINTER(LearnedScorer)), ("dev_ws", C.c_void_p),
                ("ws_bytes", C.c_size_t), ("hip_stream", C.c_void_p)]


class TraceOpts(C.Structure):
    _fields_ = [("k", C.c_uint32), ("candidates", C.c_uint32), ("every", C.c_uint32),
                ("depth", C.c_uint32), ("max_cubes", C.c_uint64)]


class CubesView(C.Structure):
    _fields_ = [("n_cubes", C.c_uint64), ("cube_off", C.POINTER(C.c_uint64)),
                ("lits", C.POINTER(C.c_int32)), ("kind", C.POINTER(C.c_int32)),
                ("f", C.POINTER(C.c_int32)), ("complete", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("k", C.c_uint32), ("max_cubes", C.c_uint64),
                ("leaves_per_round", C.c_uint32), ("chunk_log2", C.c_uint32),
                ("grid", C.c_uint32), ("max_rounds", C.c_uint32), ("scorer", C.c_uint32),
                ("flags", C.c_uint32), ("learned", C.POINTER(LearnedScorer)),
                ("max_residual", C.c_uint32), ("split_batch", C.c_uint32)]


class TuneOpts(C.Structure):
    _fields_ = [("sample", C.c_uint32), ("reps", C.c_uint32), ("max_cubes", C.c_uint64),
                ("scorer", C.c_uint32), ("flags", C.c_uint32), ("refresh", C.c_uint32),
                ("reserved", C.c_uint32)]


class TuneReport(C.Structure):
    _fields_ = [("points", C.c_uint32), ("cached", C.c_uint32), ("best_ms", C.c_double),
                ("default_ms", C.c_double)]


class QueryResult(C.Structure):
    _fields_ = [("verdict", C.c_int32), ("how", C.c_int32),
                ("cubes_total", C.c_uint64), ("cubes_refuted", C.c_uint64),
                ("leaves_sent", C.c_uint64), ("leaves_refuted", C.c_uint64),
                ("blocks_evaluated", C.c_uint64), ("clause_blocks", C.c_uint64),
                ("rounds", C.c_uint32), ("witness_checked", C.c_int32),
                ("word_ops", C.c_uint64)]


class LeafResult(C.Structure):
    _fields_ = [("refuted", C.c_int32), ("f", C.c_int32), ("m", C.c_int32),
                ("reserved", C.c_int32), ("count", C.c_uint64), ("first", C.c_int64)]


# name -> (restype, argtypes); every function include/scuba.h declares
P = C.c_void_p
SIGNATURES = {
    "scuba_abi_version": (C.c_uint32, []),
    "scuba_ctx_create": (C.c_int32, [C.c_int32, C.POINTER(P)]),
    "scuba_ctx_destroy": (None, [P]),
    "scuba_last_error": (C.c_char_p, [P]),
    "scuba_status_str": (C.c_char_p, [C.c_int32]),
    "scuba_bitblast": (C.c_int32, [P, C.c_uint32, P, P, P, P, C.c_uint32, C.POINTER(P)]),
    "scuba_cnf_from_arrays": (C.c_int32, [P, C.c_uint32, P, P, P, P, C.POINTER(P)]),
    "scuba_cnf_count": (C.c_uint32, [P]),
    "scuba_cnf_view_get": (C.c_int32, [P, C.c_uint32, C.POINTER(CnfView)]),
    "scuba_cnf_input_map": (C.c_int32, [P, C.c_uint32, P, P, C.c_uint32]),
    "scuba_cnf_free": (None, [P]),
    "scuba_scorer_workspace": (C.c_size_t, [P, C.c_uint32]),
    "scuba_split": (C.c_int32, [P, P, C.POINTER(SplitOpts), C.POINTER(P)]),
    "scuba_trace_run": (C.c_int32, [P, P, C.POINTER(TraceOpts), C.POINTER(P)]),
    "scuba_trace_view": (C.c_int32, [P, C.POINTER(C.c_uint64), C.POINTER(C.POINTER(C.c_float)),
                                     C.POINTER(C.POINTER(C.c_float)),
                                     C.POINTER(C.POINTER(C.c_uint64))]),
    "scuba_trace_free": (None, [P]),
    "scuba_cubes_from_arrays": (C.c_int32, [P, P, P, P, P, C.POINTER(P)]),
    "scuba_cubes_view_get": (C.c_int32, [P, C.c_uint32, C.POINTER(CubesView)]),
    "scuba_cubes_free": (None, [P]),
    "scuba_solve_workspace": (C.c_int32, [P, P, P, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]),
    "scuba_decide_workspace": (C.c_int32, [P, P, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]),
    "scuba_solve": (C.c_int32, [P, P, P, C.POINTER(SolveOpts), P, C.c_size_t, P, C.POINTER(P)]),
    "scuba_decide": (C.c_int32, [P, P, C.POINTER(SolveOpts), P, C.c_size_t, P, C.POINTER(P)]),
    "scuba_decide_noalloc": (C.c_int32, [P, P, C.POINTER(SolveOpts), P, C.POINTER(P)]),
    "scuba_tune_cache_save": (C.c_int32, [P, C.c_char_p]),
    "scuba_tune_cache_load": (C.c_int32, [P, C.c_char_p, C.POINTER(C.c_uint32)]),
    "scuba_result_get": (C.c_int32, [P, C.c_uint32, C.POINTER(QueryResult)]),
    "scuba_witness_get": (C.c_int32, [P, C.c_uint32, P, C.c_uint32]),
    "scuba_model_get": (C.c_int32, [P, C.c_uint32, P, C.c_uint32]),
    "scuba_leaf_get": (C.c_int32, [P, C.c_uint32, C.c_uint64, C.POINTER(LeafResult)]),
    "scuba_results_timing": (C.c_int32, [P, P, C.c_uint32]),
    "scuba_results_free": (None, [P]),
    "scuba_autotune_workspace": (C.c_int32, [P, P, C.POINTER(TuneOpts), C.POINTER(C.c_size_t)]),
    "scuba_autotune": (C.c_int32, [P, P, C.POINTER(TuneOpts), P, C.c_size_t, P, C.POINTER(SolveOpts),
                                   C.POINTER(TuneReport)]),
    "scuba_mlp_param_count": (C.c_uint32, []),
    "scuba_mlp_sync": (C.c_int32, [P, P, P, P]),
    "scuba_mlp_forward": (C.c_int32, [P, P, P, P, C.c_uint32, P, P, P, P]),
    "scuba_mlp_backward": (C.c_int32, [P, P, P, P, P, P, P, C.c_uint32, P, P, P, P]),
    "scuba_mlp_adam": (C.c_int32, [P, P, P, P, P, P, C.c_uint32, C.c_float, C.c_float,
                                   C.c_float, C.c_float, P]),
}

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime under the same soname; load it
        # first so that the library binds to that one runtime (two runtimes
        # in one process do not share devices, streams or memory)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2601_21552_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class ScubaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status

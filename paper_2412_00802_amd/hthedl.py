"""Thin ctypes binding of libhthedl.so.

The functions named ``hth_*`` mirror the C entry points of ``include/hthedl.h``
one to one and only marshal arguments: every step of an evaluation runs in the
library's HIP kernels.  PyTorch provides the device memory and the stream.
If the library is not built, importing works but the first call raises.

``Engine`` bundles the usual sequence (upload a knowledge base, create the
handle, size a workspace, evaluate).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhthedl.so")

HTH_OK = 0
STATUS = {0: "HTH_OK", -1: "HTH_E_INVALID", -2: "HTH_E_RANGE", -3: "HTH_E_NOMEM",
          -4: "HTH_E_DEVICE", -5: "HTH_E_PLAN", -6: "HTH_E_STATE", -7: "HTH_E_UNSUPPORTED"}

OPS = {"top": 0, "bot": 1, "atom": 2, "not": 3, "and": 4, "or": 5, "exists": 6, "forall": 7,
       "atleast": 8, "atmost": 9, "exactly": 10, "dge": 11, "dle": 12, "set": 13,
       "deq": 14, "nge": 15, "nle": 16, "neq": 17, "sequal": 18, "scontains": 19}

NODE_DTYPE = np.dtype([("op", np.uint8), ("inv", np.uint8), ("arity", np.uint16),
                       ("arg", np.uint32), ("child", np.uint32), ("q", np.uint32)])
assert NODE_DTYPE.itemsize == 16

# hth_conjunct: an added conjunct (kind HTH_CJ_*) of a set-table parent
CONJ_DTYPE = np.dtype([("parent", np.uint32), ("kind", np.uint8), ("inv", np.uint8), ("pad", np.uint16),
                       ("a", np.uint32), ("b", np.uint32)])
assert CONJ_DTYPE.itemsize == 16
CJ_ATOM, CJ_EXISTS, CJ_GE, CJ_LE, CJ_EQ = range(5)

EXPORTED = ["hth_kb_derived_bytes", "hth_kb_create", "hth_kb_set_examples", "hth_kb_max_degree",
            "hth_kb_destroy", "hth_workspace_bytes", "hth_eval_one", "hth_eval_batch",
            "hth_sync", "hth_status_str", "hth_last_error", "hth_profile_begin",
            "hth_profile_end", "hth_features", "hth_densify", "hth_gemm_bf16", "hth_head_forward",
            "hth_head_backward", "hth_colsum", "hth_adamw", "hth_to_bf16", "hth_topk", "hth_transpose_bf16",
            "hth_batch_workspace_bytes", "hth_head_score", "hth_kb_get_tuning", "hth_kb_set_tuning",
            "hth_kb_set_sets", "hth_eval_batch_sets", "hth_densify_delta", "hth_plan_create",
            "hth_plan_upload", "hth_plan_launch", "hth_plan_destroy", "hth_numeric_derived_bytes",
            "hth_kb_set_numeric", "hth_string_derived_bytes", "hth_kb_set_strings", "hth_kb_set_patterns",
            "hth_dplan_scratch_bytes", "hth_dplan_create", "hth_dplan_launch", "hth_dplan_destroy",
            "hth_draw_conjuncts", "hth_conjoin", "hth_dplan_stats", "hth_eval_one_noalloc",
            "hth_cache_create", "hth_eval_batch_cached", "hth_cache_stats", "hth_cache_destroy"]


class HthError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class KBDesc(ctypes.Structure):
    _fields_ = [("n_individuals", ctypes.c_uint32), ("stride_words", ctypes.c_uint32),
                ("n_concepts", ctypes.c_uint32), ("concept_bits", ctypes.c_void_p),
                ("n_roles", ctypes.c_uint32), ("n_edges", ctypes.c_uint64),
                ("role_offsets", ctypes.c_void_p), ("role_targets", ctypes.c_void_p),
                ("n_data", ctypes.c_uint32), ("data", ctypes.c_void_p),
                ("pos_bits", ctypes.c_void_p), ("neg_bits", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("group_min", ctypes.c_uint32), ("group_k", ctypes.c_uint32),
                ("xcd_local", ctypes.c_uint32), ("t_budget_mb", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("region_reg", ctypes.c_uint32),
                ("t_compact", ctypes.c_uint32), ("t_segment_kb", ctypes.c_uint32),
                ("push_pct", ctypes.c_uint32), ("short_rows", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class CacheInfo(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_uint64), ("misses", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("entries", ctypes.c_uint32),
                ("rows", ctypes.c_uint32)]


class DplanInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in ("levels", "role_nodes", "shared_passes", "thresholds",
                                                 "materialised", "rows")]


class ProfEntry(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


HTH_K_NUM = 8

_lib = None


def lib() -> ctypes.CDLL:
    """Open libhthedl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2412_00802_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, S = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
        I, F = ctypes.c_int, ctypes.c_float
        sig = {
            "hth_kb_derived_bytes": [ctypes.POINTER(KBDesc), ctypes.POINTER(S)],
            "hth_kb_create": [ctypes.POINTER(KBDesc), P, S, P, ctypes.POINTER(P)],
            "hth_kb_set_examples": [P, P, P],
            "hth_kb_max_degree": [P, U32, U32, ctypes.POINTER(U32)],
            "hth_kb_destroy": [P],
            "hth_kb_get_tuning": [P, ctypes.POINTER(Tuning)],
            "hth_kb_set_tuning": [P, ctypes.POINTER(Tuning)],
            "hth_workspace_bytes": [P, U32, U32, ctypes.POINTER(S)],
            "hth_eval_one": [P, P, U32, P, U32, P, S, P, P, P],
            "hth_eval_one_noalloc": [P, P, U32, P, U32, P, P, P],
            "hth_cache_create": [P, P, U32, ctypes.POINTER(P)],
            "hth_eval_batch_cached": [P, P, P, P, U32, P, U32, P, S, P, P],
            "hth_cache_stats": [P, ctypes.POINTER(CacheInfo)],
            "hth_cache_destroy": [P],
            "hth_eval_batch": [P, P, P, U32, P, U32, P, S, P, P],
            "hth_eval_batch_sets": [P, P, P, U32, P, U32, P, S, P, P, P],
            "hth_kb_set_sets": [P, P, U32],
            "hth_numeric_derived_bytes": [P, U32, U64, ctypes.POINTER(S)],
            "hth_kb_set_numeric": [P, U32, P, P, U64, P, S, P],
            "hth_string_derived_bytes": [P, U32, U64, ctypes.POINTER(S)],
            "hth_kb_set_strings": [P, U32, P, P, U64, U32, P, P, P, S, P],
            "hth_kb_set_patterns": [P, U32, P, P, P],
            "hth_plan_create": [P, P, P, U32, P, U32, ctypes.POINTER(P), ctypes.POINTER(S)],
            "hth_plan_upload": [P, P, S, P],
            "hth_plan_launch": [P, P, S, P, P],
            "hth_plan_destroy": [P],
            "hth_dplan_scratch_bytes": [P, U32, ctypes.POINTER(S)],
            "hth_dplan_create": [P, P, U32, P, U32, P, U32, P, S, P, ctypes.POINTER(P), ctypes.POINTER(S)],
            "hth_dplan_launch": [P, P, S, P, P],
            "hth_draw_conjuncts": [P, U64, P, U32, U32, P, P, P],
            "hth_conjoin": [P, U32, P, P, P, U32, U32, P],
            "hth_dplan_destroy": [P],
            "hth_dplan_stats": [P, ctypes.POINTER(DplanInfo)],
            "hth_batch_workspace_bytes": [P, P, P, U32, P, U32, ctypes.POINTER(S)],
            "hth_sync": [P],
            "hth_profile_begin": [P],
            "hth_profile_end": [P, ctypes.POINTER(ProfEntry)],
            "hth_features": [P, P, U32, P, U32, P, P, P, P],
            "hth_densify": [P, P, U32, U32, P, P],
            "hth_densify_delta": [P, P, U32, U32, P, P, P, U32, P, P],
            "hth_gemm_bf16": [I, I, I, I, I, P, I, P, I, P, I, P, I, P, I, P, I, P],
            "hth_head_forward": [P, I, I, P, P, P, P, P, F, P, I, P],
            "hth_head_backward": [P, I, I, P, P, P, P, P],
            "hth_head_score": [P, I, F, F, P, I, P, P],
            "hth_colsum": [P, I, I, I, P, P],
            "hth_adamw": [P, P, P, P, P, S, F, F, F, F, F, I, P],
            "hth_to_bf16": [P, P, S, P],
            "hth_transpose_bf16": [P, ctypes.c_int, ctypes.c_int, P, P],
            "hth_topk": [P, U32, U32, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.hth_status_str.argtypes = [ctypes.c_int32]
        L.hth_status_str.restype = ctypes.c_char_p
        L.hth_last_error.argtypes = [ctypes.c_char_p, S]
        L.hth_last_error.restype = S
        _lib = L
    return _lib


def hth_last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    lib().hth_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def hth_status_str(status: int) -> str:
    return lib().hth_status_str(status).decode()


def _check(status: int) -> None:
    if status != HTH_OK:
        raise HthError(status, hth_last_error())


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _np_ptr(a: Optional[np.ndarray]) -> Optional[int]:
    if a is None or a.size == 0:
        return None
    return a.ctypes.data


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------


def hth_kb_derived_bytes(desc: KBDesc) -> int:
    out = ctypes.c_size_t()
    _check(lib().hth_kb_derived_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def hth_kb_create(desc: KBDesc, derived, derived_bytes: int, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().hth_kb_create(ctypes.byref(desc), _ptr(derived), derived_bytes, _stream(stream),
                               ctypes.byref(h)))
    return h


def hth_kb_set_examples(kb, pos, neg) -> None:
    _check(lib().hth_kb_set_examples(kb, _ptr(pos), _ptr(neg)))


def hth_kb_set_sets(kb, rows, n_rows: int) -> None:
    _check(lib().hth_kb_set_sets(kb, _ptr(rows) if n_rows else None, n_rows))


def hth_numeric_derived_bytes(kb, n_roles: int, n_values: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().hth_numeric_derived_bytes(kb, n_roles, n_values, ctypes.byref(out)))
    return out.value


def hth_kb_set_numeric(kb, n_roles: int, offsets, values, n_values: int, derived, derived_bytes: int,
                       stream=None) -> None:
    """Register multi-valued numeric concrete roles (device int64 offsets
    [n_roles][N+1] and float32 values); n_roles = 0 removes them."""
    _check(lib().hth_kb_set_numeric(kb, n_roles, _ptr(offsets) if n_roles else None,
                                    _ptr(values) if n_values else None, n_values,
                                    _ptr(derived) if n_roles else None, derived_bytes, _stream(stream)))


def hth_string_derived_bytes(kb, n_roles: int, n_values: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().hth_string_derived_bytes(kb, n_roles, n_values, ctypes.byref(out)))
    return out.value


def hth_kb_set_strings(kb, n_roles: int, offsets, ids, n_values: int, n_strings: int, str_offsets, chars,
                       derived, derived_bytes: int, stream=None) -> None:
    """Register string concrete roles (device int64 offsets [n_roles][N+1],
    int32 dictionary ids, and the dictionary as int64 offsets + bytes)."""
    _check(lib().hth_kb_set_strings(kb, n_roles, _ptr(offsets) if n_roles else None,
                                    _ptr(ids) if n_values else None, n_values, n_strings,
                                    _ptr(str_offsets) if n_roles else None, _ptr(chars) if n_roles else None,
                                    _ptr(derived) if n_roles else None, derived_bytes, _stream(stream)))


def hth_kb_set_patterns(kb, n_patterns: int, offsets, chars, stream=None) -> None:
    _check(lib().hth_kb_set_patterns(kb, n_patterns, _ptr(offsets) if n_patterns else None,
                                     _ptr(chars) if n_patterns else None, _stream(stream)))


def _concat_bytes(items):
    offs = np.zeros(len(items) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(b) for b in items])
    chars = np.frombuffer(b"".join(items), dtype=np.uint8) if offs[-1] else np.zeros(0, np.uint8)
    return offs, chars


def hth_kb_max_degree(kb, role: int, inv: int) -> int:
    out = ctypes.c_uint32()
    _check(lib().hth_kb_max_degree(kb, role, inv, ctypes.byref(out)))
    return out.value


def hth_kb_get_tuning(kb) -> dict:
    t = Tuning()
    _check(lib().hth_kb_get_tuning(kb, ctypes.byref(t)))
    return t.as_dict()


def hth_kb_set_tuning(kb, **kw) -> None:
    t = Tuning(**{**hth_kb_get_tuning(kb), **kw})
    _check(lib().hth_kb_set_tuning(kb, ctypes.byref(t)))


def hth_kb_destroy(kb) -> None:
    _check(lib().hth_kb_destroy(kb))


def hth_workspace_bytes(kb, max_nodes: int, max_hyps: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().hth_workspace_bytes(kb, max_nodes, max_hyps, ctypes.byref(out)))
    return out.value


def hth_eval_one(kb, nodes: np.ndarray, children: np.ndarray, ws, ws_bytes: int,
                 d_instances, d_counts, stream=None) -> None:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    _check(lib().hth_eval_one(kb, _np_ptr(nodes), nodes.shape[0], _np_ptr(children),
                              children.shape[0], _ptr(ws), ws_bytes, _ptr(d_instances),
                              _ptr(d_counts), _stream(stream)))


# bytes of the fixed device scratch behind hth_eval_one_noalloc (HTH_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


def hth_eval_one_noalloc(kb, nodes: np.ndarray, children: np.ndarray, d_instances, d_counts,
                         stream=None) -> None:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    _check(lib().hth_eval_one_noalloc(kb, _np_ptr(nodes), nodes.shape[0], _np_ptr(children),
                                      children.shape[0], _ptr(d_instances), _ptr(d_counts),
                                      _stream(stream)))


def hth_eval_batch(kb, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray, ws,
                   ws_bytes: int, d_counts, stream=None) -> None:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    _check(lib().hth_eval_batch(kb, _np_ptr(nodes), _np_ptr(offsets), offsets.shape[0] - 1,
                                _np_ptr(children), children.shape[0], _ptr(ws), ws_bytes,
                                _ptr(d_counts), _stream(stream)))


def hth_cache_create(kb, d_rows, n_rows: int):
    out = ctypes.c_void_p()
    _check(lib().hth_cache_create(kb, _ptr(d_rows), n_rows, ctypes.byref(out)))
    return out.value


def hth_eval_batch_cached(kb, cache, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray, ws,
                          ws_bytes: int, d_counts, stream=None) -> None:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    _check(lib().hth_eval_batch_cached(kb, cache, _np_ptr(nodes), _np_ptr(offsets), offsets.shape[0] - 1,
                                       _np_ptr(children), children.shape[0], _ptr(ws), ws_bytes,
                                       _ptr(d_counts), _stream(stream)))


def hth_cache_stats(cache) -> dict:
    info = CacheInfo()
    _check(lib().hth_cache_stats(cache, ctypes.byref(info)))
    return {f: int(getattr(info, f)) for f, _ in info._fields_}


def hth_cache_destroy(cache) -> None:
    _check(lib().hth_cache_destroy(cache))


def hth_eval_batch_sets(kb, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray, ws,
                        ws_bytes: int, d_sets, d_counts, stream=None) -> None:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    _check(lib().hth_eval_batch_sets(kb, _np_ptr(nodes), _np_ptr(offsets), offsets.shape[0] - 1,
                                     _np_ptr(children), children.shape[0], _ptr(ws), ws_bytes,
                                     _ptr(d_sets), _ptr(d_counts), _stream(stream)))


def hth_plan_create(kb, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray):
    """-> (plan handle, workspace bytes)."""
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    _check(lib().hth_plan_create(kb, _np_ptr(nodes), _np_ptr(offsets), offsets.shape[0] - 1, _np_ptr(children),
                                 children.shape[0], ctypes.byref(h), ctypes.byref(nb)))
    return h, nb.value


def hth_plan_upload(plan, ws, ws_bytes: int, stream=None) -> None:
    _check(lib().hth_plan_upload(plan, _ptr(ws), ws_bytes, _stream(stream)))


def hth_plan_launch(plan, ws, ws_bytes: int, d_counts, stream=None) -> None:
    _check(lib().hth_plan_launch(plan, _ptr(ws), ws_bytes, _ptr(d_counts), _stream(stream)))


def hth_plan_destroy(plan) -> None:
    _check(lib().hth_plan_destroy(plan))


def hth_dplan_scratch_bytes(kb, n_nodes: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().hth_dplan_scratch_bytes(kb, n_nodes, ctypes.byref(out)))
    return out.value


def hth_dplan_create(kb, d_nodes, n_nodes: int, d_offsets, n_hyps: int, d_children, n_children: int,
                     scratch, scratch_bytes: int, stream=None):
    """Plan generated on the device from device arrays (d_nodes: the node
    records as bytes, d_offsets [n_hyps+1] and d_children as 32-bit tensors;
    scratch: hth_dplan_scratch_bytes bytes) -> (plan handle, workspace bytes)."""
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    _check(lib().hth_dplan_create(kb, _ptr(d_nodes), n_nodes, _ptr(d_offsets), n_hyps,
                                  _ptr(d_children) if n_children else None, n_children, _ptr(scratch),
                                  scratch_bytes, _stream(stream), ctypes.byref(h), ctypes.byref(nb)))
    return h, nb.value


def _need_bytes(t, nbytes: int, what: str) -> None:
    """A device tensor argument must hold what the library writes or reads."""
    if t is not None and not isinstance(t, int) and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what}: {t.numel() * t.element_size()} bytes, the call needs {nbytes}")


def hth_draw_conjuncts(kb, seed: int, d_parent_rows, n_parents: int, per_parent: int, d_deciles, d_specs,
                       stream=None) -> None:
    _need_bytes(d_parent_rows, 4 * n_parents, "parent rows")
    _need_bytes(d_specs, CONJ_DTYPE.itemsize * n_parents * per_parent, "specs")
    _check(lib().hth_draw_conjuncts(kb, seed, _ptr(d_parent_rows), n_parents, per_parent, _ptr(d_deciles),
                                    _ptr(d_specs), _stream(stream)))


def hth_conjoin(d_specs, n: int, d_nodes, d_offsets, d_children, node_base: int = 0, child_base: int = 0,
                stream=None) -> None:
    """d_nodes, d_offsets and d_children point where the candidates go (views
    into a larger batch when the bases are not 0)."""
    _need_bytes(d_specs, CONJ_DTYPE.itemsize * n, "specs")
    _need_bytes(d_nodes, 4 * NODE_DTYPE.itemsize * n, "nodes")
    _need_bytes(d_offsets, 4 * (n + 1), "offsets")
    _need_bytes(d_children, 8 * n, "children")
    _check(lib().hth_conjoin(_ptr(d_specs), n, _ptr(d_nodes), _ptr(d_offsets), _ptr(d_children), node_base,
                             child_base, _stream(stream)))


def conjunct_tuple(spec) -> tuple:
    """The conjunct of one hth_conjunct record, in the tuple form."""
    k, a, b = int(spec["kind"]), int(spec["a"]), int(spec["b"])
    if k == CJ_ATOM:
        return ("atom", a)
    if k == CJ_EXISTS:
        return ("exists", b, int(spec["inv"]), ("atom", a))
    t = float(np.uint32(b).view(np.float32))
    return ({CJ_GE: "dge", CJ_LE: "dle", CJ_EQ: "deq"}[k], a, t)


def hth_dplan_launch(plan, ws, ws_bytes: int, d_counts, stream=None) -> None:
    _check(lib().hth_dplan_launch(plan, _ptr(ws), ws_bytes, _ptr(d_counts), _stream(stream)))


def hth_dplan_stats(plan) -> dict:
    info = DplanInfo()
    _check(lib().hth_dplan_stats(plan, ctypes.byref(info)))
    return {f: int(getattr(info, f)) for f, _ in DplanInfo._fields_}


def hth_dplan_destroy(plan) -> None:
    _check(lib().hth_dplan_destroy(plan))


def hth_batch_workspace_bytes(kb, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray) -> int:
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    children = np.ascontiguousarray(children, dtype=np.uint32)
    out = ctypes.c_size_t()
    _check(lib().hth_batch_workspace_bytes(kb, _np_ptr(nodes), _np_ptr(offsets), offsets.shape[0] - 1,
                                           _np_ptr(children), children.shape[0], ctypes.byref(out)))
    return out.value


def hth_sync(stream=None) -> None:
    _check(lib().hth_sync(_stream(stream)))


def hth_profile_begin(kb) -> None:
    _check(lib().hth_profile_begin(kb))


def hth_profile_end(kb) -> List[dict]:
    """Per kernel kind: launches, event-timed ms and algorithmic bytes."""
    arr = (ProfEntry * HTH_K_NUM)()
    _check(lib().hth_profile_end(kb, arr))
    return [{"launches": int(e.launches), "ms": float(e.ms), "bytes": float(e.bytes)} for e in arr]


profile_end = hth_profile_end


# -- learned screener (device tensors; bf16 tensors are torch.bfloat16) ------


def hth_features(d_nodes, d_offsets, n_hyps: int, d_children, n_children: int, d_hash, d_feat, d_bad,
                 stream=None) -> None:
    _check(lib().hth_features(_ptr(d_nodes), _ptr(d_offsets), n_hyps, _ptr(d_children), n_children,
                              _ptr(d_hash), _ptr(d_feat), _ptr(d_bad), _stream(stream)))


def hth_densify(d_feat, d_offsets, row0: int, n_rows: int, d_x, stream=None) -> None:
    _check(lib().hth_densify(_ptr(d_feat), _ptr(d_offsets), row0, n_rows, _ptr(d_x), _stream(stream)))


def hth_densify_delta(d_feat, d_offsets, row0: int, n_rows: int, d_parent_feat, d_parent_offsets,
                      d_parent_index, d_x, stream=None, parent_context: int = 0) -> None:
    _check(lib().hth_densify_delta(_ptr(d_feat), _ptr(d_offsets), row0, n_rows, _ptr(d_parent_feat),
                                   _ptr(d_parent_offsets), _ptr(d_parent_index), parent_context, _ptr(d_x),
                                   _stream(stream)))


def hth_gemm_bf16(trans_a: int, trans_b: int, M: int, N: int, K: int, A, lda: int, B, ldb: int,
                  bias=None, relu: int = 0, mask=None, ldm: int = 0, c32=None, ldc: int = 0, cbf=None,
                  ldcb: int = 0, stream=None) -> None:
    _check(lib().hth_gemm_bf16(trans_a, trans_b, M, N, K, _ptr(A), lda, _ptr(B), ldb, _ptr(bias), relu,
                               _ptr(mask), ldm, _ptr(c32), ldc, _ptr(cbf), ldcb, _stream(stream)))


def hth_head_forward(h, Bn: int, Kd: int, w, bias, z, y=None, dz=None, scale: float = 1.0, loss=None,
                     stream=None, loss_kind: int = 0) -> None:
    _check(lib().hth_head_forward(_ptr(h), Bn, Kd, _ptr(w), _ptr(bias), _ptr(z), _ptr(y), _ptr(dz),
                                  scale, _ptr(loss), loss_kind, _stream(stream)))


def hth_head_score(z, Bn: int, n_pos: float, n_neg: float, score, stream=None, base=None, kind: int = 0) -> None:
    _check(lib().hth_head_score(_ptr(z), Bn, n_pos, n_neg, _ptr(base) if base is not None else None, kind,
                                _ptr(score), _stream(stream)))


def hth_head_backward(h, Bn: int, Kd: int, w, dz, dw, dh, stream=None) -> None:
    _check(lib().hth_head_backward(_ptr(h), Bn, Kd, _ptr(w), _ptr(dz), _ptr(dw), _ptr(dh),
                                   _stream(stream)))


def hth_colsum(d, is_bf16: int, M: int, N: int, out, stream=None) -> None:
    _check(lib().hth_colsum(_ptr(d), is_bf16, M, N, _ptr(out), _stream(stream)))


def hth_adamw(p, g, m, v, pbf, n: int, lr: float, beta1: float, beta2: float, eps: float, wd: float,
              step: int, stream=None) -> None:
    _check(lib().hth_adamw(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(pbf), n, lr, beta1, beta2, eps, wd,
                           step, _stream(stream)))


def hth_to_bf16(s, d, n: int, stream=None) -> None:
    _check(lib().hth_to_bf16(_ptr(s), _ptr(d), n, _stream(stream)))


def hth_transpose_bf16(src, rows: int, cols: int, dst, stream=None) -> None:
    _check(lib().hth_transpose_bf16(_ptr(src), rows, cols, _ptr(dst), _stream(stream)))


def hth_topk(d_scores, n: int, k: int, d_idx, d_work, stream=None) -> None:
    _check(lib().hth_topk(_ptr(d_scores), n, k, _ptr(d_idx), _ptr(d_work), _stream(stream)))


# ---------------------------------------------------------------------------
# hypothesis encoding: nested tuples -> postfix node arrays
# ---------------------------------------------------------------------------


def _f32_bits(t: float) -> int:
    return int(np.array([t], dtype=np.float32).view(np.uint32)[0])


def encode(h, nodes: list, children: list) -> int:
    """Append hypothesis h in postfix order; return its root's local index."""
    op = h[0]
    code = OPS[op]
    if op in ("top", "bot"):
        nodes.append((code, 0, 0, 0, 0, 0))
    elif op in ("atom", "set"):
        nodes.append((code, 0, 0, h[1], 0, 0))
    elif op == "not":
        c = encode(h[1], nodes, children)
        nodes.append((code, 0, 0, 0, c, 0))
    elif op in ("and", "or"):
        cs = [encode(c, nodes, children) for c in h[1:]]
        start = len(children)
        children.extend(cs)
        nodes.append((code, 0, len(cs), 0, start, 0))
    elif op in ("exists", "forall"):
        _, r, inv, c = h
        ci = encode(c, nodes, children)
        nodes.append((code, inv, 0, r, ci, 0))
    elif op in ("atleast", "atmost", "exactly"):
        _, k, r, inv, c = h
        ci = encode(c, nodes, children)
        nodes.append((code, inv, 0, r, ci, k))
    elif op in ("dge", "dle", "deq", "nge", "nle", "neq"):
        nodes.append((code, 0, 0, h[1], 0, _f32_bits(h[2])))
    elif op in ("sequal", "scontains"):
        # the query as an id: a dictionary string id (-1: absent) or a pattern
        # id; Engine.intern turns the strings of a hypothesis into these
        if not isinstance(h[2], (int, np.integer)):
            raise ValueError("string restrictions need ids here: use Engine.intern first")
        nodes.append((code, 0, 0, h[1], 0, int(h[2]) & 0xFFFFFFFF))
    else:
        raise ValueError(op)
    return len(nodes) - 1


def encode_one(h) -> Tuple[np.ndarray, np.ndarray]:
    nodes: list = []
    children: list = []
    encode(h, nodes, children)
    return np.array(nodes, dtype=NODE_DTYPE), np.array(children, dtype=np.uint32)


def encode_batch(hyps: Sequence, child_offsets: bool = False):
    """-> (nodes, hyp_node_offsets [H+1], children); child indices are local.
    With child_offsets, also the [H+1] start of each hypothesis's children."""
    allnodes: List[tuple] = []
    children: List[int] = []
    offs = [0]
    coffs = [0]
    for h in hyps:
        local: list = []
        encode(h, local, children)
        allnodes.extend(local)
        offs.append(len(allnodes))
        coffs.append(len(children))
    out = (np.array(allnodes, dtype=NODE_DTYPE), np.array(offs, dtype=np.uint32),
           np.array(children, dtype=np.uint32))
    return out + (np.array(coffs, dtype=np.int64),) if child_offsets else out


def gather_encoded(encoded, idx: np.ndarray):
    """The hypotheses `idx` of an encode_batch(..., child_offsets=True) result,
    as a new batch (nodes, offsets, children)."""
    nodes, offs, ch, coffs = encoded
    idx = np.asarray(idx, dtype=np.int64)
    offs = offs.astype(np.int64)
    nlen = offs[idx + 1] - offs[idx]
    clen = coffs[idx + 1] - coffs[idx]
    new_offs = np.zeros(idx.size + 1, dtype=np.int64)
    np.cumsum(nlen, out=new_offs[1:])
    new_coffs = np.zeros(idx.size + 1, dtype=np.int64)
    np.cumsum(clen, out=new_coffs[1:])
    node_src = np.repeat(offs[idx] - new_offs[:-1], nlen) + np.arange(new_offs[-1])
    ch_src = np.repeat(coffs[idx] - new_coffs[:-1], clen) + np.arange(new_coffs[-1])
    sub = nodes[node_src].copy()
    shift = np.repeat(coffs[idx] - new_coffs[:-1], nlen)
    ands = (sub["op"] == OPS["and"]) | (sub["op"] == OPS["or"])
    sub["child"][ands] = (sub["child"][ands].astype(np.int64) - shift[ands]).astype(np.uint32)
    return sub, new_offs.astype(np.uint32), ch[ch_src].copy()


def slice_encoded(encoded, a: int, b: int):
    """Hypotheses [a, b) of an encode_batch result, re-based.  Their children
    entries are contiguous because encode_batch appends per hypothesis."""
    nodes, offs, ch = encoded
    n0, n1 = int(offs[a]), int(offs[b])
    sub = nodes[n0:n1].copy()
    ands = (sub["op"] == OPS["and"]) | (sub["op"] == OPS["or"])
    if ands.any():
        lo = int(sub["child"][ands].min())
        hi = int((sub["child"][ands] + sub["arity"][ands]).max())
        sub["child"][ands] -= lo
        sub_ch = ch[lo:hi].copy()
    else:
        sub_ch = np.zeros(0, dtype=np.uint32)
    return sub, (offs[a:b + 1] - offs[a]).astype(np.uint32), sub_ch


# ---------------------------------------------------------------------------
# engine: device-resident knowledge base + workspace
# ---------------------------------------------------------------------------


def stride_for(n: int) -> int:
    w = (n + 63) // 64
    return (w + 7) // 8 * 8


class Engine:
    """A knowledge base uploaded to one GPU, its handle and a workspace."""

    def __init__(self, kb, device: str = "cuda:0", max_nodes: int = 1 << 14,
                 max_hyps: int = 4096):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        lib()
        n = int(kb.n)
        self.n = n
        self.W = (n + 63) // 64
        self.S = stride_for(n)
        dev = self.device

        def padded(bits2d):
            a = np.zeros((bits2d.shape[0], self.S), dtype=np.uint64)
            a[:, : bits2d.shape[1]] = bits2d
            return torch.from_numpy(a.view(np.int64)).to(dev)

        cb = np.asarray(kb.concept_bits, dtype=np.uint64).reshape(-1, self.W)
        self.concepts = padded(cb) if cb.shape[0] else torch.zeros((0, self.S), dtype=torch.int64, device=dev)
        self.offsets = torch.from_numpy(np.ascontiguousarray(kb.role_offsets, dtype=np.int64)).to(dev)
        self.targets = torch.from_numpy(np.ascontiguousarray(kb.role_targets, dtype=np.int32)).to(dev)
        self.data = torch.from_numpy(np.ascontiguousarray(kb.data, dtype=np.float32)).to(dev)
        self.pos = padded(np.asarray(kb.pos_bits, dtype=np.uint64)[None, :])[0]
        self.neg = padded(np.asarray(kb.neg_bits, dtype=np.uint64)[None, :])[0]
        self.n_pos = int(np.unpackbits(np.asarray(kb.pos_bits, dtype=np.uint64).view(np.uint8)).sum())
        self.n_neg = int(np.unpackbits(np.asarray(kb.neg_bits, dtype=np.uint64).view(np.uint8)).sum())
        d = KBDesc()
        d.n_individuals = n
        d.stride_words = self.S
        d.n_concepts = int(self.concepts.shape[0])
        d.concept_bits = _ptr(self.concepts) if d.n_concepts else None
        d.n_roles = int(self.offsets.shape[0])
        d.n_edges = int(self.targets.shape[0])
        d.role_offsets = _ptr(self.offsets) if d.n_roles else None
        d.role_targets = _ptr(self.targets) if d.n_edges else None
        d.n_data = int(self.data.shape[0])
        d.data = _ptr(self.data) if d.n_data else None
        d.pos_bits = _ptr(self.pos)
        d.neg_bits = _ptr(self.neg)
        self.desc = d
        nbytes = hth_kb_derived_bytes(d)
        self.derived = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self.handle = hth_kb_create(d, self.derived, nbytes)
        no = getattr(kb, "num_offsets", None)
        if no is not None and len(no):
            # multi-valued numeric concrete roles
            self.num_offsets = torch.from_numpy(np.ascontiguousarray(no, dtype=np.int64)).to(dev)
            vals = np.ascontiguousarray(kb.num_values, dtype=np.float32)
            self.num_values = torch.from_numpy(vals if vals.size else np.zeros(1, np.float32)).to(dev)
            P, V = int(no.shape[0]), int(vals.size)
            nb = hth_numeric_derived_bytes(self.handle, P, V)
            self.num_derived = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
            hth_kb_set_numeric(self.handle, P, self.num_offsets, self.num_values, V, self.num_derived, nb)
        self._str_id = None
        so = getattr(kb, "str_offsets", None)
        if so is not None and len(so):
            # string concrete roles: assertions hold ids into the dictionary
            strings = list(kb.strings)
            self._str_id = {s: i for i, s in enumerate(strings)}
            self.str_offsets = torch.from_numpy(np.ascontiguousarray(so, dtype=np.int64)).to(dev)
            ids = np.ascontiguousarray(kb.str_ids, dtype=np.int32)
            self.str_ids = torch.from_numpy(ids if ids.size else np.zeros(1, np.int32)).to(dev)
            doff, dchars = _concat_bytes(strings)
            self.dict_offsets = torch.from_numpy(doff).to(dev)
            self.dict_chars = torch.from_numpy(dchars.copy() if dchars.size else np.zeros(1, np.uint8)).to(dev)
            Q, V = int(so.shape[0]), int(ids.size)
            nb = hth_string_derived_bytes(self.handle, Q, V)
            self.str_derived = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
            hth_kb_set_strings(self.handle, Q, self.str_offsets, self.str_ids, V, len(strings), self.dict_offsets,
                               self.dict_chars, self.str_derived, nb)
            self._patterns: dict = {}
        self.ws = None
        self.ws_bytes = 0
        self.reserve(max_nodes, max_hyps)

    def reserve(self, max_nodes: int, max_hyps: int) -> None:
        need = hth_workspace_bytes(self.handle, max(max_nodes, max_hyps), max_hyps)
        if need > self.ws_bytes:
            self.ws = None
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
            self.ws_bytes = need

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            hth_kb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- evaluation ---------------------------------------------------------

    def intern(self, h):
        """Hypothesis h with its string queries as ids: EQUAL strings as
        dictionary ids (-1 when absent), CONTAIN patterns as ids of the
        registered pattern table (new patterns are added and the table is
        registered again)."""
        if self._str_id is None or not isinstance(h, tuple):
            return h
        op = h[0]
        if op == "sequal" and isinstance(h[2], (bytes, bytearray)):
            return ("sequal", h[1], self._str_id.get(bytes(h[2]), -1))
        if op == "scontains" and isinstance(h[2], (bytes, bytearray)):
            pat = bytes(h[2])
            if pat not in self._patterns:
                self._patterns[pat] = len(self._patterns)
                pats = sorted(self._patterns, key=self._patterns.get)
                poff, pchars = _concat_bytes(pats)
                self.pat_offsets = self.torch.from_numpy(poff).to(self.device)
                self.pat_chars = self.torch.from_numpy(pchars.copy() if pchars.size else np.zeros(1, np.uint8)).to(
                    self.device)
                hth_kb_set_patterns(self.handle, len(pats), self.pat_offsets, self.pat_chars)
            return ("scontains", h[1], self._patterns[pat])
        return tuple(self.intern(c) if isinstance(c, tuple) else c for c in h)

    def eval_one(self, h, instances: bool = False, counts=None, stream=None):
        """Coverage (and optionally the instance bits) of one hypothesis.
        With `counts` given (a device uint32 [2] view) nothing is synchronised."""
        torch = self.torch
        nodes, ch = encode_one(self.intern(h))
        self.reserve(nodes.shape[0], 1)
        out = counts if counts is not None else torch.empty(2, dtype=torch.int32, device=self.device)
        inst = torch.empty(self.S, dtype=torch.int64, device=self.device) if instances else None
        hth_eval_one(self.handle, nodes, ch, self.ws, self.ws_bytes, inst, out, stream)
        if counts is not None:
            return None
        c = tuple(int(v) for v in out.cpu().numpy().view(np.uint32))
        if instances:
            return c, inst.cpu().numpy().view(np.uint64)[: self.W]
        return c

    def eval_plain(self, hyps: Sequence, stream=None) -> np.ndarray:
        """One hypothesis at a time (host plan + kernel sequence each); uint32 [H][2]."""
        torch = self.torch
        out = torch.empty((len(hyps), 2), dtype=torch.int32, device=self.device)
        for i, h in enumerate(hyps):
            self.eval_one(h, counts=out[i], stream=stream)
        return out.cpu().numpy().view(np.uint32)

    def ensure_workspace(self, nbytes: int) -> None:
        if nbytes > self.ws_bytes:
            self.ws = None
            self.ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            self.ws_bytes = nbytes

    def ensure_plan_scratch(self, n_nodes: int) -> None:
        """Scratch for device plans over batches of up to n_nodes nodes."""
        nbytes = hth_dplan_scratch_bytes(self.handle, n_nodes)
        if nbytes > getattr(self, "dp_scratch_bytes", 0):
            self.dp_scratch = None
            self.dp_scratch = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            self.dp_scratch_bytes = nbytes

    def conjunct_candidates(self, parent_rows, per_parent: int, seed: int, deciles=None, before=None,
                            count: Optional[int] = None):
        """Refinement candidates drawn and written on the device
        (hth_draw_conjuncts, hth_conjoin): parent_rows (set-table rows) x
        per_parent added conjuncts, of which the first `count` (all by
        default) go into the batch.  before: an encoded batch (nodes, offsets,
        children) uploaded in front of the candidates, so that one plan covers
        both.  -> (specs, (nodes, offsets, children)), all device tensors; the
        batch goes to eval_batch_device."""
        torch = self.torch
        rows = torch.as_tensor(np.asarray(parent_rows, dtype=np.uint32).view(np.int32), device=self.device)
        n_draw = int(rows.shape[0]) * per_parent
        n = n_draw if count is None else min(count, n_draw)
        dec = None
        if self.desc.n_data:
            dec = torch.as_tensor(np.ascontiguousarray(deciles, dtype=np.float32), device=self.device)
        specs = torch.empty(n_draw * CONJ_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        hn = hc = hh = 0
        if before is not None:
            bn, bo, bc = before
            hh, hn, hc = int(bo.shape[0]) - 1, int(bn.shape[0]), int(bc.shape[0])
        nodes = torch.empty((hn + 4 * n) * NODE_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        offs = torch.empty(hh + n + 1, dtype=torch.int32, device=self.device)
        ch = torch.empty(max(1, hc + 2 * n), dtype=torch.int32, device=self.device)
        if before is not None:
            nodes[:hn * NODE_DTYPE.itemsize].copy_(torch.from_numpy(
                np.ascontiguousarray(bn, dtype=NODE_DTYPE).view(np.uint8)))
            offs[:hh].copy_(torch.from_numpy(np.ascontiguousarray(bo[:hh], dtype=np.uint32).view(np.int32)))
            if hc:
                ch[:hc].copy_(torch.from_numpy(np.ascontiguousarray(bc, dtype=np.uint32).view(np.int32)))
        hth_draw_conjuncts(self.handle, seed, rows, int(rows.shape[0]), per_parent, dec, specs)
        hth_conjoin(specs, n, nodes[hn * NODE_DTYPE.itemsize:], offs[hh:], ch[hc:], hn, hc)
        return specs, (nodes, offs, ch[:hc + 2 * n])

    def upload_batch(self, hyps: Sequence = None, encoded=None):
        """The batch's node arrays in device memory: (nodes as bytes,
        offsets, children) tensors, as hth_dplan_create takes them."""
        torch = self.torch
        nodes, offs, ch = encoded if encoded is not None else encode_batch(hyps)
        d_nodes = torch.from_numpy(np.ascontiguousarray(nodes, dtype=NODE_DTYPE).view(np.uint8)).to(self.device)
        d_offs = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.uint32).view(np.int32)).to(self.device)
        d_ch = torch.from_numpy(np.ascontiguousarray(ch, dtype=np.uint32).view(np.int32)).to(self.device)
        return d_nodes, d_offs, d_ch

    def eval_batch_device(self, hyps: Sequence = None, counts=None, chunk: Optional[int] = None,
                          encoded=None, device_batch=None, stream=None) -> Optional[np.ndarray]:
        """Batched evaluation with plans generated on the device (hth_dplan_*):
        the node arrays go to the device once (or come as device_batch, from
        upload_batch or a device-side producer), and each chunk of `chunk`
        hypotheses gets its plan from the library's count and emit kernels.
        uint32 [H][2]."""
        torch = self.torch
        d_nodes, d_offs, d_ch = device_batch if device_batch is not None else self.upload_batch(hyps, encoded)
        H = int(d_offs.shape[0] - 1)
        n_nodes = int(d_nodes.shape[0] // NODE_DTYPE.itemsize)
        out = counts if counts is not None else torch.empty((H, 2), dtype=torch.int32, device=self.device)
        chunk = H if not chunk else chunk
        self.ensure_plan_scratch(n_nodes)
        for a in range(0, H, chunk):
            b = min(H, a + chunk)
            plan, nb = hth_dplan_create(self.handle, d_nodes, n_nodes, d_offs[a:], b - a, d_ch,
                                        int(d_ch.shape[0]), self.dp_scratch, self.dp_scratch_bytes, stream)
            try:
                self.ensure_workspace(max(nb, 256))
                hth_dplan_launch(plan, self.ws, self.ws_bytes, out[a:b], stream)
            finally:
                hth_dplan_destroy(plan)
        if counts is not None:
            return None
        return out.cpu().numpy().view(np.uint32)

    def eval_batch(self, hyps: Sequence, stream=None, counts=None, chunk: Optional[int] = None,
                   encoded=None) -> Optional[np.ndarray]:
        """Batched evaluation; uint32 [H][2].  Batches larger than `chunk`
        hypotheses are run as consecutive sub-batches (each compiled alone)."""
        torch = self.torch
        H = len(hyps) if encoded is None else int(encoded[1].shape[0] - 1)
        out = counts if counts is not None else torch.empty((H, 2), dtype=torch.int32, device=self.device)
        chunk = H if not chunk else chunk
        for a in range(0, H, chunk):
            b = min(H, a + chunk)
            if encoded is None:
                nodes, offs, ch = encode_batch([self.intern(h) for h in hyps[a:b]] if self._str_id else hyps[a:b])
            else:
                nodes, offs, ch = slice_encoded(encoded, a, b)
            self.ensure_workspace(hth_batch_workspace_bytes(self.handle, nodes, offs, ch))
            hth_eval_batch(self.handle, nodes, offs, ch, self.ws, self.ws_bytes, out[a:b], stream)
        if counts is not None:
            return None
        return out.cpu().numpy().view(np.uint32)

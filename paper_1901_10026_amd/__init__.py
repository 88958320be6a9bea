"""Python binding of libtg.so (typed 3/4-node graphlet counting on MI355X).

This module only marshals arguments: torch tensors provide device memory and
the HIP stream, and every step of the computation runs in the library's
kernels.  There is no CPU fallback; if the library is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_CSRC = os.path.join(_HERE, "csrc")
_INCLUDE = os.path.join(_ROOT, "include")
_LIB = os.path.join(_HERE, "libtg.so")
_lib = None

SHAPES = ("wedge", "triangle", "path4", "star4", "cycle4", "tailed_triangle", "chordal_cycle", "clique4")
SCHEDULES = {"none": 0, "degree": 1, "learned": 2}
STATUS = {0: "TG_OK", 1: "TG_ERR_INVALID_ARG", 2: "TG_ERR_INVALID_GRAPH", 3: "TG_ERR_TYPE_RANGE",
          4: "TG_ERR_UNSUPPORTED_L", 5: "TG_ERR_OUT_OF_MEMORY", 6: "TG_ERR_INTERNAL", 7: "TG_ERR_HIP"}

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


class TGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def build(force: bool = True) -> str:
    """Compile libtg.so for gfx950 with hipcc (cross-compiles without a GPU)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["hipcc", *HIPCC_FLAGS, f"-I{_INCLUDE}", f"-I{_CSRC}", os.path.join(_CSRC, "tg_api.hip"), "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def library_path() -> str:
    return _LIB


def declared_symbols():
    """Function names declared in include/tg.h."""
    text = open(os.path.join(_INCLUDE, "tg.h")).read()
    return sorted(set(re.findall(r"\b(tg_[a-z0-9_]+)\s*\(", text)))


class Tuning(ctypes.Structure):
    """Launch-shape choices (tg_tuning); counts never depend on them."""
    _fields_ = [("light_max_degree", ctypes.c_int32), ("heavy_min_degree", ctypes.c_int32),
                ("mid_log2_cost", ctypes.c_int32), ("heavy_log2_cost", ctypes.c_int32),
                ("combine_grid", ctypes.c_int32), ("wg_grid", ctypes.c_int32), ("c4_footprint_mb", ctypes.c_int32),
                ("c4_group_kwedges", ctypes.c_int32), ("c4_chunk", ctypes.c_int32),
                ("c4_hash_ratio", ctypes.c_int32), ("c4_slot_budget_mb", ctypes.c_int32), ("c4_slices", ctypes.c_int32),
                ("batch_variant", ctypes.c_int32 * 9), ("clique_team_max", ctypes.c_int32),
                ("clique_wave_max", ctypes.c_int32), ("clique_lds_ids", ctypes.c_int32),
                ("tlist_budget_mib", ctypes.c_int32), ("clique_pass", ctypes.c_int32),
                ("clique_pass_grid", ctypes.c_int32), ("clique_pass_lds_kib", ctypes.c_int32),
                ("c4_parts", ctypes.c_int32), ("c4_part_lds_kib", ctypes.c_int32),
                ("c4_part_chunk", ctypes.c_int32), ("c4_part_hash_ratio", ctypes.c_int32),
                ("tau_hub_min_degree", ctypes.c_int32), ("c4_split_log2", ctypes.c_int32)]
    SCALARS = ("light_max_degree", "heavy_min_degree", "mid_log2_cost", "heavy_log2_cost", "combine_grid",
               "wg_grid", "c4_footprint_mb", "c4_group_kwedges", "c4_chunk", "c4_hash_ratio", "c4_slot_budget_mb",
               "c4_slices", "clique_team_max", "clique_wave_max", "clique_lds_ids", "tlist_budget_mib",
               "clique_pass", "clique_pass_grid", "clique_pass_lds_kib", "c4_parts", "c4_part_lds_kib",
               "c4_part_chunk", "c4_part_hash_ratio",
               "tau_hub_min_degree", "c4_split_log2")

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k in self.SCALARS}
        d["batch_variant"] = list(self.batch_variant)
        return d

    @classmethod
    def default(cls):
        t = cls()
        lib().tg_tuning_default(ctypes.byref(t))
        return t

    @classmethod
    def from_dict(cls, d):
        t = cls.default()
        for k in cls.SCALARS:
            if k in d:
                setattr(t, k, int(d[k]))
        if "batch_variant" in d:
            for q, v in enumerate(d["batch_variant"]):
                t.batch_variant[q] = int(v)
        return t


class _Options(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int), ("model", ctypes.c_void_p), ("tuning", ctypes.c_void_p),
                ("validate", ctypes.c_int),
                ("check", ctypes.c_int), ("edge_begin", ctypes.c_int64), ("edge_end", ctypes.c_int64),
                ("phase_ms", ctypes.c_void_p), ("edge_ids", ctypes.c_void_p), ("num_edge_ids", ctypes.c_int64),
                ("edge_orbits", ctypes.c_void_p)]


PHASES = ("prep", "tau", "tables", "schedule", "cycles", "cliques", "combine", "finalize")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise RuntimeError(f"libtg.so is not built ({_LIB}); run paper_1901_10026_amd.build() or "
                           "__graft_entry__.build() first")
    # torch (which provides the device memory and streams) is loaded before
    # the library, so that its HIP runtime comes up first whatever the
    # caller touches first
    import torch  # noqa: F401
    L = ctypes.CDLL(_LIB)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.tg_options_default.restype = None
    L.tg_options_default.argtypes = [ctypes.POINTER(_Options)]
    L.tg_num_keys.restype = sz
    L.tg_num_keys.argtypes = [i32]
    L.tg_edge_row_width.restype = sz
    L.tg_edge_row_width.argtypes = [i32]
    L.tg_edge_orbit_width.restype = sz
    L.tg_edge_orbit_width.argtypes = [i32]
    L.tg_key_decode.restype = i32
    L.tg_key_decode.argtypes = [i32, sz, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint8)]
    L.tg_key_encode.restype = i32
    L.tg_key_encode.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(sz)]
    L.tg_edge_row_key.restype = i32
    L.tg_edge_row_key.argtypes = [i32, ctypes.c_uint8, ctypes.c_uint8, sz, ctypes.POINTER(sz)]
    L.tg_count.restype = i32
    L.tg_count.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_count_global.restype = i32
    L.tg_count_sparse.restype = i32
    L.tg_count_sparse.argtypes = [i64, i64, vp, vp, vp, i32, vp, i64, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(_Options), vp]
    L.tg_count_global.argtypes = [i64, i64, vp, vp, vp, i32, vp, ctypes.POINTER(_Options), vp]
    L.tg_count_global_types.restype = i32
    L.tg_count_directed3.restype = i32
    L.tg_count_directed3.argtypes = [i64, i64, vp, vp, vp, vp, i32, vp, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_directed3_num_keys.restype = sz
    L.tg_directed3_num_keys.argtypes = [i32]
    L.tg_directed3_key_decode.restype = i32
    L.tg_directed3_key_decode.argtypes = [i32, sz, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint8)]
    L.tg_directed3_key_encode.restype = i32
    L.tg_directed3_key_encode.argtypes = [i32, ctypes.c_uint8, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(sz)]
    L.tg_count_directed4.restype = i32
    L.tg_count_directed4.argtypes = [i64, i64, vp, vp, vp, vp, i32, vp, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_directed4_num_keys.restype = sz
    L.tg_directed4_num_keys.argtypes = [i32]
    L.tg_directed4_key_decode.restype = i32
    L.tg_directed4_key_decode.argtypes = [i32, sz, ctypes.POINTER(ctypes.c_uint16), ctypes.POINTER(ctypes.c_uint8)]
    L.tg_count_global_types.argtypes = [i64, i64, vp, vp, i64, vp, i32, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_rows_sparse.restype = i32
    L.tg_rows_sparse.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp, i64, ctypes.POINTER(ctypes.c_int64), vp]
    L.tg_count_batch.restype = i32
    L.tg_count_batch.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_count_batch_noalloc.restype = i32
    L.tg_count_batch_noalloc.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_Options), vp]
    L.tg_tuning_default.restype = None
    L.tg_tuning_default.argtypes = [ctypes.POINTER(Tuning)]
    L.tg_autotune.restype = i32
    L.tg_autotune.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, ctypes.POINTER(_Options), ctypes.POINTER(Tuning),
                              ctypes.POINTER(ctypes.c_float), vp]
    L.tg_autotune_batch.restype = i32
    L.tg_autotune_batch.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Tuning),
                                    ctypes.POINTER(ctypes.c_float), vp]
    L.tg_cost_model_num_params.restype = sz
    L.tg_cost_model_num_params.argtypes = []
    L.tg_cost_model_create.restype = i32
    L.tg_cost_model_create.argtypes = [ctypes.POINTER(vp), ctypes.c_uint64]
    L.tg_cost_model_destroy.restype = i32
    L.tg_cost_model_destroy.argtypes = [vp]
    L.tg_cost_model_train.restype = i32
    L.tg_cost_model_train.argtypes = [vp, i64, i64, vp, vp, vp, i32, ctypes.c_double, ctypes.c_uint64, i32, vp, vp]
    L.tg_cost_model_predict.restype = i32
    L.tg_cost_model_predict.argtypes = [vp, i64, i64, vp, vp, vp, i32, vp, vp]
    L.tg_edge_work.restype = i32
    L.tg_edge_work.argtypes = [i64, i64, vp, vp, vp, i32, vp, i64, vp, vp]
    L.tg_cost_model_gradient.restype = i32
    L.tg_cost_model_gradient.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.tg_cost_model_get_params.restype = i32
    L.tg_cost_model_get_params.argtypes = [vp, vp]
    L.tg_cost_model_set_params.restype = i32
    L.tg_cost_model_set_params.argtypes = [vp, vp]
    L.tg_cost_model_save.restype = i32
    L.tg_cost_model_save.argtypes = [vp, ctypes.c_char_p]
    L.tg_cost_model_load.restype = i32
    L.tg_cost_model_load.argtypes = [vp, ctypes.c_char_p]
    L.tg_release_scratch.restype = i32
    L.tg_release_scratch.argtypes = []
    L.tg_status_string.restype = ctypes.c_char_p
    L.tg_status_string.argtypes = [i32]
    L.tg_last_error.restype = ctypes.c_char_p
    L.tg_last_error.argtypes = []
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise TGError(st, lib().tg_last_error().decode())


def num_keys(L: int) -> int:
    return int(lib().tg_num_keys(L))


def edge_row_width(L: int) -> int:
    return int(lib().tg_edge_row_width(L))


def edge_orbit_width(L: int) -> int:
    return int(lib().tg_edge_orbit_width(L))


def key_encode(L: int, shape: int, types) -> int:
    arr = (ctypes.c_uint8 * 4)(*(list(types) + [0] * (4 - len(types))))
    out = ctypes.c_size_t()
    _check(lib().tg_key_encode(L, shape, arr, ctypes.byref(out)))
    return int(out.value)


def key_decode(L: int, key: int):
    shape = ctypes.c_int()
    arr = (ctypes.c_uint8 * 4)()
    _check(lib().tg_key_decode(L, key, ctypes.byref(shape), arr))
    k = 3 if shape.value < 2 else 4
    return int(shape.value), tuple(int(arr[q]) for q in range(k))


def edge_row_key(L: int, phi_i: int, phi_j: int, col: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().tg_edge_row_key(L, phi_i, phi_j, col, ctypes.byref(out)))
    return int(out.value)


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def count(row_ptr, col_idx, types, L, *, per_edge=True, endpoints=False, schedule="degree", validate=False,
          check=True, edge_range=None, edge_ids=None, global_counts=True, model=None, out_global=None, out_edges=None,
          out_orbits=None, phase_ms=None, tuning=None):
    """Counts every typed 3/4-node graphlet of one graph with tg_count.

    row_ptr, col_idx (int32) and types (uint8) are CUDA (HIP) tensors on the
    same device.  Returns (global uint64 [K(L)], per-edge uint64 [E, R(L)] or
    None, endpoints int32 [E, 2] or None) as torch tensors; uint64 results are
    stored in torch.uint64 tensors.  Rows cover the canonical edges in
    edge_range (default all), or, when edge_ids (a strictly increasing int64
    device tensor of canonical edge ids) is given, exactly those edges.
    With global_counts=False (rows only) the global result is None and only
    those edges go through the per-edge step.  out_orbits, a uint64 device
    tensor [E, edge_orbit_width(L)], receives the orbit counts g1..g12 of
    the same edges.
    """
    import torch
    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (types, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("row_ptr/col_idx must be contiguous int32 and types contiguous uint8 on one device")
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    m = nnz // 2
    e0, e1 = (0, m) if edge_range is None else (int(edge_range[0]), int(edge_range[1]))
    if edge_ids is not None:
        if edge_ids.dtype != torch.int64 or not edge_ids.is_contiguous() or edge_ids.device != dev:
            raise ValueError("edge_ids must be a contiguous int64 tensor on the inputs' device")
        e0, e1 = 0, edge_ids.numel()
    K = num_keys(L)
    R = edge_row_width(L)
    if K == 0:
        raise TGError(4, "L must be in [1, 16]")
    if not global_counts and not per_edge and out_orbits is None:
        raise ValueError("rows-only counting needs per_edge=True or out_orbits")
    g = None
    if global_counts:
        g = out_global if out_global is not None else torch.empty(K, dtype=torch.uint64, device=dev)
    rows = None
    if per_edge:
        rows = out_edges if out_edges is not None else torch.empty((max(e1 - e0, 0), R), dtype=torch.uint64,
                                                                   device=dev)
    ends = torch.empty((max(e1 - e0, 0), 2), dtype=torch.int32, device=dev) if endpoints else None
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.schedule = SCHEDULES[schedule]
    opt.model = model.handle if model is not None else None
    opt.tuning = ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None
    opt.validate = 1 if validate else 0
    opt.check = 1 if check else 0
    opt.edge_begin = e0
    opt.edge_end = e1
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    if out_orbits is not None:
        if out_orbits.dtype != torch.uint64 or not out_orbits.is_contiguous() or out_orbits.device != dev or \
                out_orbits.numel() < max(e1 - e0, 0) * edge_orbit_width(L):
            raise ValueError("out_orbits must be a contiguous uint64 tensor of [E, edge_orbit_width(L)] on the device")
        opt.edge_orbits = out_orbits.data_ptr() if out_orbits.numel() else None
    if edge_ids is not None:
        opt.edge_ids = edge_ids.data_ptr() if edge_ids.numel() else None
        opt.num_edge_ids = edge_ids.numel()
        if not edge_ids.numel():
            opt.edge_begin, opt.edge_end = 0, 0
    st = lib().tg_count(n, nnz, row_ptr.data_ptr(), col_idx.data_ptr() if nnz else None,
                        types.data_ptr() if n else None, L, g.data_ptr() if g is not None else None,
                        rows.data_ptr() if rows is not None and rows.numel() else None,
                        ends.data_ptr() if ends is not None and ends.numel() else None,
                        ctypes.byref(opt), _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    return g, rows, ends


def count_global(row_ptr, col_idx, types, L, *, validate=False, check=True, out=None, phase_ms=None, tuning=None):
    """Global typed-graphlet counts only, with tg_count_global (every instance
    counted a fixed number of times instead of once per edge).  Same inputs
    as count(); returns the uint64 [K(L)] device tensor."""
    import torch
    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (types, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("row_ptr/col_idx must be contiguous int32 and types contiguous uint8 on one device")
    K = num_keys(L)
    if K == 0:
        raise TGError(4, "L must be in [1, 16]")
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    g = out if out is not None else torch.empty(K, dtype=torch.uint64, device=dev)
    if g.dtype != torch.uint64 or not g.is_contiguous() or g.device != dev or g.numel() < K:
        raise ValueError("out must be a contiguous uint64 tensor of K(L) entries on the inputs' device")
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.tuning = ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None
    opt.validate = 1 if validate else 0
    opt.check = 1 if check else 0
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    st = lib().tg_count_global(n, nnz, row_ptr.data_ptr(), col_idx.data_ptr() if nnz else None,
                               types.data_ptr() if n else None, L, g.data_ptr(), ctypes.byref(opt),
                               _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    return g


def count_global_types(row_ptr, col_idx, type_vectors, L, *, validate=False, check=True, out=None, mean=True,
                       phase_ms=None, tuning=None):
    """Global counts of one graph under several type vectors with
    tg_count_global_types.  type_vectors: contiguous uint8 device tensor
    [B, n].  Returns (counts uint64 [B, K(L)], mean float64 [K(L)] or None)."""
    import torch
    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (type_vectors, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("row_ptr/col_idx must be contiguous int32 and type_vectors contiguous uint8 on one device")
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if type_vectors.dim() != 2 or type_vectors.shape[1] != n or type_vectors.shape[0] < 1:
        raise ValueError("type_vectors must have shape [B, n] with B >= 1")
    B = type_vectors.shape[0]
    K = num_keys(L)
    if K == 0:
        raise TGError(4, "L must be in [1, 16]")
    g = out if out is not None else torch.empty((B, K), dtype=torch.uint64, device=dev)
    if g.dtype != torch.uint64 or not g.is_contiguous() or g.device != dev or g.numel() < B * K:
        raise ValueError("out must be a contiguous uint64 tensor of [B, K(L)] on the inputs' device")
    mu = torch.empty(K, dtype=torch.float64, device=dev) if mean else None
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.tuning = ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None
    opt.validate = 1 if validate else 0
    opt.check = 1 if check else 0
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    st = lib().tg_count_global_types(n, nnz, row_ptr.data_ptr(), col_idx.data_ptr() if nnz else None, B,
                                     type_vectors.data_ptr() if n else None, L, g.data_ptr(),
                                     mu.data_ptr() if mu is not None else None, ctypes.byref(opt),
                                     _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    return g, mu


def directed3_num_keys(L):
    """Number of directed typed 3-node keys (tg_directed3_num_keys)."""
    return int(lib().tg_directed3_num_keys(int(L)))


def directed3_key_decode(L, key):
    """(arc bits, (type0, type1, type2)) of a directed key's canonical triad."""
    arcs = ctypes.c_uint8(0)
    types = (ctypes.c_uint8 * 3)()
    _check(lib().tg_directed3_key_decode(int(L), int(key), ctypes.byref(arcs), types))
    return int(arcs.value), tuple(int(t) for t in types)


def directed3_key_encode(L, arcs, types):
    """Key of the triad with six arc bits `arcs` and node types `types`."""
    t = (ctypes.c_uint8 * 3)(*[int(x) for x in types])
    key = ctypes.c_size_t(0)
    _check(lib().tg_directed3_key_encode(int(L), int(arcs), t, ctypes.byref(key)))
    return int(key.value)


def count_directed3(row_ptr, col_idx, slot_dir, types, L, *, per_edge=True, info=False, global_counts=True,
                    validate=False, check=True, phase_ms=None):
    """Directed typed 3-node graphlets with tg_count_directed3.  row_ptr,
    col_idx: the symmetric support CSR (int32); slot_dir: uint8 direction
    bits per slot; types: uint8.  Returns (global uint64 [K] or None, rows
    uint64 [m, 15 L] or None, info int32 [m, 3] = (i, j, c(i, j)) or None)."""
    import torch
    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (slot_dir, torch.uint8), (types, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("row_ptr/col_idx must be contiguous int32, slot_dir/types contiguous uint8, one device")
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if slot_dir.numel() != nnz:
        raise ValueError("slot_dir needs one byte per CSR slot")
    K = directed3_num_keys(L)
    if K == 0:
        raise TGError(4, "L must be in [1, 16]")
    m = nnz // 2
    g = torch.empty(K, dtype=torch.uint64, device=dev) if global_counts else None
    rows = torch.empty((m, 15 * L), dtype=torch.uint64, device=dev) if per_edge else None
    inf = torch.empty((m, 3), dtype=torch.int32, device=dev) if info else None
    if g is None and rows is None:
        raise ValueError("ask for global counts, rows or both")
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.validate = 1 if validate else 0
    opt.check = 1 if check else 0
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    ptr = lambda t: t.data_ptr() if t is not None and t.numel() else None
    st = lib().tg_count_directed3(n, nnz, row_ptr.data_ptr(), ptr(col_idx), ptr(slot_dir), ptr(types), L, ptr(g),
                                  ptr(rows), ptr(inf), ctypes.byref(opt), _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    return g, rows, inf


def directed4_num_keys(L: int) -> int:
    return int(lib().tg_directed4_num_keys(L))


def directed4_key_decode(L: int, key: int):
    """(12 arc bits, four types) of a directed 4-node key's canonical digraph."""
    arcs = ctypes.c_uint16()
    ty = (ctypes.c_uint8 * 4)()
    _check(lib().tg_directed4_key_decode(L, key, ctypes.byref(arcs), ty))
    return int(arcs.value), tuple(int(ty[q]) for q in range(4))


def count_directed4(row_ptr, col_idx, slot_dir, types, L, *, per_edge=False, info=False, global_counts=True,
                    validate=False, check=True, phase_ms=None):
    """Directed typed 4-node graphlets with tg_count_directed4 (L <= 4).
    Inputs as for count_directed3.  Returns (global uint64 [K] or None, rows
    uint64 [m, K] or None, info int32 [m, 3] or None), K =
    directed4_num_keys(L)."""
    import torch
    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    for t, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (slot_dir, torch.uint8), (types, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or t.device != dev:
            raise ValueError("row_ptr/col_idx must be contiguous int32, slot_dir/types contiguous uint8, one device")
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    if slot_dir.numel() != nnz:
        raise ValueError("slot_dir needs one byte per CSR slot")
    K = directed4_num_keys(L)
    if K == 0:
        raise TGError(4, "L must be in [1, 4]")
    m = nnz // 2
    g = torch.empty(K, dtype=torch.uint64, device=dev) if global_counts else None
    rows = torch.empty((m, K), dtype=torch.uint64, device=dev) if per_edge else None
    inf = torch.empty((m, 3), dtype=torch.int32, device=dev) if info else None
    if g is None and rows is None:
        raise ValueError("ask for global counts, rows or both")
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.validate = 1 if validate else 0
    opt.check = 1 if check else 0
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    ptr = lambda t: t.data_ptr() if t is not None and t.numel() else None
    st = lib().tg_count_directed4(n, nnz, row_ptr.data_ptr(), ptr(col_idx), ptr(slot_dir), ptr(types), L, ptr(g),
                                  ptr(rows), ptr(inf), ctypes.byref(opt), _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    return g, rows, inf


def type_permutations(types, count, seed):
    """count permutations of a host uint8 type vector, drawn by numpy's
    seeded default generator: row b is types[perm_b] (the null model's random
    relabellings, which keep every type's frequency)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    return np.stack([t[rng.permutation(len(t))] for _ in range(count)]) if count else np.zeros((0, len(t)), np.uint8)


def null_model(row_ptr, col_idx, types, L, *, permutations=100, seed=0, **kw):
    """Type-permutation null model: global counts under `permutations`
    seeded random permutations of the node types, and their mean.  Returns
    (counts uint64 [permutations, K(L)], mean float64 [K(L)])."""
    import torch
    perms = type_permutations(types.cpu().numpy(), permutations, seed)
    tv = torch.from_numpy(perms).to(row_ptr.device)
    return count_global_types(row_ptr, col_idx, tv, L, **kw)


def rows_sparse(rows, endpoints, types, L):
    """Nonzero entries of per-edge rows as (key, count) pairs with
    tg_rows_sparse: returns (offsets int64 [E+1], keys int32-stored uint32
    [total], counts uint64 [total]) as device tensors; edge e's pairs are
    keys/counts[offsets[e]:offsets[e+1]]."""
    import torch
    dev = rows.device
    E = rows.shape[0]
    offsets = torch.empty(E + 1, dtype=torch.int64, device=dev)
    total = ctypes.c_int64(0)
    st = _stream_handle(torch, dev)
    _check(lib().tg_rows_sparse(E, L, rows.data_ptr() if E else None, endpoints.data_ptr() if E else None,
                                types.data_ptr() if types.numel() else None, offsets.data_ptr(), None, None, 0,
                                ctypes.byref(total), st))
    n = int(total.value)
    keys = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    counts = torch.empty(max(n, 1), dtype=torch.uint64, device=dev)
    _check(lib().tg_rows_sparse(E, L, rows.data_ptr() if E else None, endpoints.data_ptr() if E else None,
                                types.data_ptr() if types.numel() else None, offsets.data_ptr(), keys.data_ptr(),
                                counts.data_ptr(), max(n, 1), ctypes.byref(total), st))
    return offsets, keys[:n], counts[:n]


def key_offsets(L_per_graph):
    """Prefix sums of tg_num_keys(L_g): where each graph's counts start."""
    import numpy as np
    ks = np.array([num_keys(int(l)) for l in range(0, 17)], dtype=np.int64)
    sizes = ks[np.asarray(L_per_graph, dtype=np.int64)]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def count_sparse(row_ptr, col_idx, types, L, *, capacity=None, schedule="degree", edge_range=None, edge_ids=None,
                 global_counts=True, model=None, tuning=None, check=True, validate=False, phase_ms=None):
    """Sparse per-edge output straight from the row kernel (tg_count_sparse):
    nonzero (global key, count) pairs of the edges in edge_range (default
    all) or edge_ids.  capacity (pairs) defaults to E * R(L), the most
    there can be.  Returns (global uint64 [K] or None, keys uint32 [total],
    counts uint64 [total], start int64 [E], length int32 [E]); edge q's
    pairs are keys[start[q]:start[q] + length[q]]."""
    import torch
    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col_idx.numel()
    m = nnz // 2
    e0, e1 = (0, m) if edge_range is None else (int(edge_range[0]), int(edge_range[1]))
    E = edge_ids.numel() if edge_ids is not None else e1 - e0
    K, R = num_keys(L), edge_row_width(L)
    cap = E * R if capacity is None else int(capacity)
    keys = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    counts = torch.empty(max(cap, 1), dtype=torch.uint64, device=dev)
    start = torch.empty(max(E, 1), dtype=torch.int64, device=dev)
    length = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    g = torch.empty(K, dtype=torch.uint64, device=dev) if global_counts else None
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.schedule = SCHEDULES[schedule]
    opt.model = ctypes.c_void_p(model.handle) if model is not None else None
    opt.tuning = ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None
    opt.check = 1 if check else 0
    opt.validate = 1 if validate else 0
    opt.edge_begin, opt.edge_end = e0, e1
    if edge_ids is not None:
        opt.edge_ids = edge_ids.data_ptr()
        opt.num_edge_ids = E
    times = (ctypes.c_float * len(PHASES))() if phase_ms is not None else None
    opt.phase_ms = ctypes.cast(times, ctypes.c_void_p) if times is not None else None
    total = ctypes.c_int64(0)
    st = lib().tg_count_sparse(n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(), types.data_ptr(), L,
                               g.data_ptr() if g is not None else None, cap, keys.data_ptr(), counts.data_ptr(),
                               start.data_ptr(), length.data_ptr(), ctypes.byref(total), ctypes.byref(opt),
                               _stream_handle(torch, dev))
    _check(st)
    if times is not None:
        phase_ms.update({name: float(times[q]) for q, name in enumerate(PHASES)})
    t = int(total.value)
    return g, keys[:t], counts[:t], start[:E], length[:E]


def release_scratch():
    """Frees the library's scratch workspace on the current device and trims
    the device's default memory pool (tg_release_scratch)."""
    _check(lib().tg_release_scratch())


def count_batch(node_off, slot_off, row_ptr, col_idx, types, L_per_graph, key_off, *, out=None, check=True,
                tuning=None, validate=False, noalloc=False):
    """Global typed-graphlet counts of many small graphs with tg_count_batch
    (or, with noalloc, tg_count_batch_noalloc: no device allocation).

    All arguments are device tensors (int64 offsets, int32 CSR with local ids,
    uint8 types and L); key_off comes from key_offsets().  Returns the uint64
    counts, graph g's at out[key_off[g]:key_off[g+1]].
    """
    import torch
    dev = node_off.device
    G = node_off.numel() - 1
    total = int(key_off[-1].item()) if key_off.numel() else 0
    g = out if out is not None else torch.empty(total, dtype=torch.uint64, device=dev)
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.check = 1 if check else 0
    opt.validate = 1 if validate else 0
    opt.tuning = ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None
    fn = lib().tg_count_batch_noalloc if noalloc else lib().tg_count_batch
    st = fn(G, node_off.data_ptr(), slot_off.data_ptr(), row_ptr.data_ptr(), col_idx.data_ptr(), types.data_ptr(),
            L_per_graph.data_ptr(), key_off.data_ptr(), g.data_ptr(), ctypes.byref(opt), _stream_handle(torch, dev))
    _check(st)
    return g


class CostModel:
    """The learned per-edge cost model (tg_cost_model): a 16-64-64-1 MLP with
    bf16 weights trained on the GPU by the library's kernels."""

    def __init__(self, seed=55):
        h = ctypes.c_void_p()
        _check(lib().tg_cost_model_create(ctypes.byref(h), int(seed)))
        self.handle = h.value

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().tg_cost_model_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    @staticmethod
    def num_params():
        return int(lib().tg_cost_model_num_params())

    def train(self, row_ptr, col_idx, types, L, sample_frac=0.01, seed=56, epochs=20):
        import torch
        hist = (ctypes.c_float * max(epochs, 1))()
        _check(lib().tg_cost_model_train(self.handle, row_ptr.numel() - 1, col_idx.numel(), row_ptr.data_ptr(),
                                         col_idx.data_ptr(), types.data_ptr(), L, float(sample_frac), int(seed),
                                         int(epochs), hist, _stream_handle(torch, row_ptr.device)))
        return [float(hist[q]) for q in range(epochs)]

    def predict(self, row_ptr, col_idx, types, L):
        import torch
        m = col_idx.numel() // 2
        out = torch.empty(m, dtype=torch.float32, device=row_ptr.device)
        _check(lib().tg_cost_model_predict(self.handle, row_ptr.numel() - 1, col_idx.numel(), row_ptr.data_ptr(),
                                           col_idx.data_ptr(), types.data_ptr(), L, out.data_ptr(),
                                           _stream_handle(torch, row_ptr.device)))
        return out

    def gradient(self, X, Y):
        import torch
        grad = torch.empty(self.num_params(), dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(lib().tg_cost_model_gradient(self.handle, X.data_ptr(), Y.data_ptr(), X.shape[0], grad.data_ptr(),
                                            loss.data_ptr(), _stream_handle(torch, X.device)))
        return grad, loss

    def get_params(self):
        import numpy as np
        out = np.zeros(self.num_params() + 32, dtype=np.float32)
        _check(lib().tg_cost_model_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.num_params() + 32
        _check(lib().tg_cost_model_set_params(self.handle, p.ctypes.data))

    def save(self, path):
        _check(lib().tg_cost_model_save(self.handle, str(path).encode()))

    def load(self, path):
        _check(lib().tg_cost_model_load(self.handle, str(path).encode()))


def edge_work(row_ptr, col_idx, types, L, edges):
    """Element-visit counts of the per-edge counting kernel for the listed
    canonical edges (int32 device tensor); returns uint64 [m] by edge id."""
    import torch
    m = col_idx.numel() // 2
    out = torch.empty(m, dtype=torch.uint64, device=row_ptr.device)
    _check(lib().tg_edge_work(row_ptr.numel() - 1, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr(),
                              types.data_ptr(), L, edges.data_ptr(), edges.numel(), out.data_ptr(),
                              _stream_handle(torch, row_ptr.device)))
    return out


def autotune(row_ptr, col_idx, types, L, out_global, out_edges=None, schedule="degree", model=None, start=None):
    """Chooses tg_count launch shapes by timing (tg_autotune).  Returns
    (Tuning, best combine-phase milliseconds)."""
    import torch
    opt = _Options()
    lib().tg_options_default(ctypes.byref(opt))
    opt.schedule = SCHEDULES[schedule]
    opt.model = model.handle if model is not None else None
    opt.tuning = ctypes.cast(ctypes.pointer(start), ctypes.c_void_p) if start is not None else None
    t = Tuning.default()
    best = ctypes.c_float()
    _check(lib().tg_autotune(row_ptr.numel() - 1, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr(),
                             types.data_ptr(), L, out_global.data_ptr(),
                             out_edges.data_ptr() if out_edges is not None else None, ctypes.byref(opt),
                             ctypes.byref(t), ctypes.byref(best), _stream_handle(torch, row_ptr.device)))
    return t, float(best.value)


def autotune_batch(node_off, slot_off, row_ptr, col_idx, types, L_per_graph, key_off, out, start=None):
    """Chooses tg_count_batch kernel variants per size class by timing.
    Returns (Tuning, best milliseconds)."""
    import torch
    t = start if start is not None else Tuning.default()
    best = ctypes.c_float()
    _check(lib().tg_autotune_batch(node_off.numel() - 1, node_off.data_ptr(), slot_off.data_ptr(), row_ptr.data_ptr(),
                                   col_idx.data_ptr(), types.data_ptr(), L_per_graph.data_ptr(), key_off.data_ptr(),
                                   out.data_ptr(), ctypes.byref(t), ctypes.byref(best),
                                   _stream_handle(torch, node_off.device)))
    return t, float(best.value)


def tuning_cache_key(kind, **sig):
    """Cache key of a tuning: device name, kind and a workload signature."""
    import torch
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return name + "|" + kind + "|" + "|".join(f"{k}={sig[k]}" for k in sorted(sig))


def load_tuning(path, key):
    import json
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return Tuning.from_dict(d[key]) if key in d else None


def save_tuning(path, key, tuning):
    import json
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[key] = tuning.as_dict()
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)

"""Python binding of libtcrnet (thresholded all-pairs Levenshtein networks on
MI355X).  Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  The functions carry the C names of include/tcrnet.h.

The library must be built (``python -m paper_2112_06613_amd.build_lib``);
loading fails loudly if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcrnet.so")

TCRNET_OK, TCRNET_EINVAL, TCRNET_ENOMEM, TCRNET_EDEVICE, TCRNET_ESTATE, TCRNET_ETRUNC = range(6)
TCRNET_F_NO_AUTOTUNE = 1
TCRNET_F_PEQ_LDS = 2
TCRNET_F_NO_PACK = 4
TCRNET_F_PEQ_VGPR = 8
TCRNET_F_COUNT_WORK = 16
MAX_LEN = 32
MAX_K = 31


class TcrnetError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status
        self.message = message


def _status_name(s: int) -> str:
    names = ["TCRNET_OK", "TCRNET_EINVAL", "TCRNET_ENOMEM", "TCRNET_EDEVICE", "TCRNET_ESTATE", "TCRNET_ETRUNC"]
    return names[s] if 0 <= s < len(names) else f"status {s}"


# ------------------------------------------------------------------ C types
class tcrnet_seqs(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n", ctypes.c_uint32)]


class tcrnet_opts(ctypes.Structure):
    _fields_ = [("texts_per_item", ctypes.c_uint32), ("waves_per_simd", ctypes.c_uint32),
                ("edge_capacity", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class tcrnet_build_info(ctypes.Structure):
    _fields_ = [("evaluated_pairs", ctypes.c_uint64), ("pair_kernel_ms", ctypes.c_double),
                ("build_ms", ctypes.c_double), ("pair_launches", ctypes.c_uint32),
                ("texts_per_item", ctypes.c_uint32), ("waves_per_simd", ctypes.c_uint32),
                ("peq_lds", ctypes.c_uint32),
                ("pack", ctypes.c_uint32), ("tuned", ctypes.c_uint32), ("graph_captured", ctypes.c_uint32),
                ("work_counted", ctypes.c_uint32), ("visited_texts", ctypes.c_uint64),
                ("wave_steps", ctypes.c_uint64), ("wave_steps_packed", ctypes.c_uint64)]


class tcrnet_result_info(ctypes.Structure):
    _fields_ = [("seqno", ctypes.c_uint64), ("snapshot_size", ctypes.c_uint32), ("is_insert", ctypes.c_uint32),
                ("latency_ms", ctypes.c_double), ("device_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("admit_ms", ctypes.c_double), ("attempts", ctypes.c_uint32), ("parts", ctypes.c_uint32)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_U32P = ctypes.POINTER(ctypes.c_uint32)
_I32 = ctypes.c_int32

# (name, restype, argtypes)
_SIGS = [
    ("tcrnet_ctx_create", _I32, [_I32, ctypes.POINTER(tcrnet_opts), _PP]),
    ("tcrnet_ctx_destroy", _I32, [_P]),
    ("tcrnet_last_error", ctypes.c_char_p, []),
    ("tcrnet_status_string", ctypes.c_char_p, [_I32]),
    ("tcrnet_version", ctypes.c_char_p, []),
    ("tcrnet_debug_fail_alloc", None, [ctypes.c_int64]),
    ("tcrnet_build", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32, _PP]),
    ("tcrnet_build_device", _I32, [_P, _P, _P, ctypes.c_uint32, _I32, _P, _P, ctypes.c_uint64, _P, _U64P]),
    ("tcrnet_build_device_noalloc", _I32, [_P, _P, _P, ctypes.c_uint32, _I32, _P, _P, ctypes.c_uint64, _P,
                                           _U64P]),
    ("tcrnet_build_batch", _I32, [_P, ctypes.POINTER(tcrnet_seqs), ctypes.c_uint32, _I32, _PP]),
    ("tcrnet_graph_edges", _I32, [_P, _PP, _U64P]),
    ("tcrnet_graph_degree", _I32, [_P, _PP, _U32P]),
    ("tcrnet_graphs_views", _I32, [_P, ctypes.c_uint32, _P, _P, _P, _P, _P]),
    ("tcrnet_graph_info", _I32, [_P, ctypes.POINTER(tcrnet_build_info)]),
    ("tcrnet_ctx_last_info", _I32, [_P, ctypes.POINTER(tcrnet_build_info)]),
    ("tcrnet_graph_free", None, [_P]),
    ("tcrnet_build_weighted", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32, _PP]),
    ("tcrnet_graph_distances", _I32, [_P, _PP, _U64P]),
    ("tcrnet_autotune", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32]),
    ("tcrnet_autotune_batch", _I32, [_P, ctypes.POINTER(tcrnet_seqs), ctypes.c_uint32, _I32]),
    ("tcrnet_autotune_get", _I32, [_P, _I32, ctypes.c_uint64, _I32, ctypes.c_void_p]),
    ("tcrnet_autotune_save", _I32, [_P, ctypes.c_char_p]),
    ("tcrnet_autotune_load", _I32, [_P, ctypes.c_char_p, _U32P]),
    ("tcrnet_valu_peak", _I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("tcrnet_valu_form_name", ctypes.c_char_p, [ctypes.c_uint32]),
    ("tcrnet_valu_rates", _I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_uint32, _U32P]),
    ("tcrnet_index_create", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32, _PP]),
    ("tcrnet_index_size", _I32, [_P, _U32P]),
    ("tcrnet_index_degree", _I32, [_P, _PP, _U32P]),
    ("tcrnet_index_free", None, [_P]),
    ("tcrnet_query", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32, _PP]),
    ("tcrnet_insert", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _PP]),
    ("tcrnet_submit", _I32, [_P, ctypes.POINTER(tcrnet_seqs), _I32, _I32, _U64P]),
    ("tcrnet_wait", _I32, [_P, ctypes.c_uint64, _PP]),
    ("tcrnet_result_pairs", _I32, [_P, _PP, _U64P]),
    ("tcrnet_result_counts", _I32, [_P, _PP, _U32P]),
    ("tcrnet_result_info_get", _I32, [_P, ctypes.POINTER(tcrnet_result_info)]),
    ("tcrnet_result_free", None, [_P]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtcrnet.so.  Raises if it is not built (no fallback)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2112_06613_amd.build_lib` "
                           "(there is no CPU fallback)")
    # PyTorch-ROCm ships its own HIP runtime with the same soname as the system
    # one; loading torch first makes the library bind to that single runtime,
    # so torch's device pointers and streams are valid in our calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def declared_symbols(header: str | None = None) -> list[str]:
    """Names of the functions declared in include/*.h."""
    import re
    import glob
    headers = [header] if header else sorted(glob.glob(os.path.join(os.path.dirname(_HERE), "include", "*.h")))
    txt = "".join(open(h).read() for h in headers)
    return sorted(set(re.findall(r"TCRNET_API\s+[\w\s\*]+?\b(tcrnet_\w+)\s*\(", txt)))


def _check(rc: int):
    if rc != TCRNET_OK:
        msg = _lib.tcrnet_last_error().decode(errors="replace")
        raise TcrnetError(rc, msg)


# -------------------------------------------------------------- sequences
def _as_seqs(seqs):
    """(chars uint8, offsets uint64) from a list of str/bytes or an object with
    .chars/.offsets arrays."""
    if hasattr(seqs, "chars") and hasattr(seqs, "offsets"):
        chars = np.ascontiguousarray(seqs.chars, dtype=np.uint8)
        offs = np.ascontiguousarray(seqs.offsets, dtype=np.uint64)
    else:
        enc = [s.encode("ascii") if isinstance(s, str) else bytes(s) for s in seqs]
        offs = np.zeros(len(enc) + 1, dtype=np.uint64)
        if enc:
            offs[1:] = np.cumsum([len(e) for e in enc])
        chars = np.frombuffer(b"".join(enc), dtype=np.uint8).copy()
    if chars.size == 0:
        chars = np.zeros(1, dtype=np.uint8)
    return chars, offs


def _c_seqs(chars, offs) -> tcrnet_seqs:
    return tcrnet_seqs(chars.ctypes.data, offs.ctypes.data, len(offs) - 1)


@dataclass
class Graph:
    pairs: np.ndarray           # (E, 2) uint32, i < j, sorted
    degree: np.ndarray          # (N,) int32
    info: dict = field(default_factory=dict)
    dist: np.ndarray | None = None   # (E,) uint8 edge distances (weighted builds)

    def at(self, k: int) -> np.ndarray:
        """Edges of the network at threshold k <= k_max (weighted builds)."""
        if self.dist is None:
            raise ValueError("not a weighted build")
        return self.pairs[self.dist <= k]


def _info_dict(inf: tcrnet_build_info) -> dict:
    return {f: getattr(inf, f) for f, _ in tcrnet_build_info._fields_}


class _GraphOwner:
    """Holds a tcrnet_graph until every array viewing its memory is gone."""
    __slots__ = ("g",)

    def __init__(self, g):
        self.g = g

    def __del__(self):
        try:
            if self.g and _lib is not None:
                _lib.tcrnet_graph_free(self.g)
        except Exception:  # interpreter shutdown
            pass
        self.g = None


def _view(ptr, ctype, count: int, dtype, owner) -> np.ndarray:
    """A numpy array over count elements of library-owned memory at ptr (no
    copy); the memory lives as long as the array does."""
    if not count or not ptr:
        return np.zeros(0, dtype=dtype)
    buf = (ctype * count).from_address(ptr)
    buf._owner = owner
    return np.frombuffer(buf, dtype=dtype)


def _take_graph(g) -> Graph:
    """Graph over the library's result: the arrays view its memory (no
    copies: a batched build returns hundreds of graphs), which is freed when
    the last of them is collected."""
    owner = _GraphOwner(g)
    p = ctypes.c_void_p()
    ne = ctypes.c_uint64()
    _check(_lib.tcrnet_graph_edges(g, ctypes.byref(p), ctypes.byref(ne)))
    pairs = _view(p.value, ctypes.c_uint32, 2 * ne.value, np.uint32, owner)
    d = ctypes.c_void_p()
    nn = ctypes.c_uint32()
    _check(_lib.tcrnet_graph_degree(g, ctypes.byref(d), ctypes.byref(nn)))
    deg = _view(d.value, ctypes.c_int32, nn.value, np.int32, owner)
    inf = tcrnet_build_info()
    _check(_lib.tcrnet_graph_info(g, ctypes.byref(inf)))
    dist = None
    dp = ctypes.c_void_p()
    dn = ctypes.c_uint64()
    if _lib.tcrnet_graph_distances(g, ctypes.byref(dp), ctypes.byref(dn)) == TCRNET_OK:
        dist = _view(dp.value, ctypes.c_uint8, dn.value, np.uint8, owner)
    return Graph(pairs.reshape(-1, 2), deg, _info_dict(inf), dist)


# ---------------------------------------------------------------- context
class Context:
    """A tcrnet_ctx on one device."""

    def __init__(self, device: int = 0, texts_per_item: int = 0, waves_per_simd: int = 0,
                 edge_capacity: int = 0, hbm_budget: int = 0, max_inflight: int = 0, flags: int = 0):
        load_library()
        self.opts = tcrnet_opts(texts_per_item, waves_per_simd, edge_capacity, hbm_budget, max_inflight, flags)
        h = ctypes.c_void_p()
        _check(_lib.tcrnet_ctx_create(device, ctypes.byref(self.opts), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.tcrnet_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_info(self) -> dict:
        inf = tcrnet_build_info()
        _check(_lib.tcrnet_ctx_last_info(self.handle, ctypes.byref(inf)))
        return _info_dict(inf)


def tcrnet_build(ctx: Context, seqs, k: int) -> Graph:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    g = ctypes.c_void_p()
    _check(_lib.tcrnet_build(ctx.handle, ctypes.byref(s), k, ctypes.byref(g)))
    return _take_graph(g)


def tcrnet_build_weighted(ctx: Context, seqs, k_max: int) -> Graph:
    """All pairs with lev <= k_max and their distances (Graph.dist)."""
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    g = ctypes.c_void_p()
    _check(_lib.tcrnet_build_weighted(ctx.handle, ctypes.byref(s), k_max, ctypes.byref(g)))
    return _take_graph(g)


def tcrnet_build_device(ctx: Context, d_chars, d_offsets, k: int, d_pairs, d_degree, stream=None) -> int:
    """Device-resident build.  d_chars: uint8 CUDA tensor; d_offsets: int64 CUDA
    tensor (n+1); d_pairs: int32/uint32-sized CUDA tensor of shape (cap, 2);
    d_degree: int32 CUDA tensor (n).  Returns E; raises TcrnetError with
    status TCRNET_ETRUNC and attribute n_edges = E when E > cap (the outputs
    are then partial)."""
    n = d_offsets.numel() - 1
    cap = d_pairs.shape[0] if d_pairs is not None else 0
    st = stream.cuda_stream if stream is not None else None
    ne = ctypes.c_uint64()
    rc = _lib.tcrnet_build_device(ctx.handle, d_chars.data_ptr(), d_offsets.data_ptr(), n, k, st,
                                  d_pairs.data_ptr() if cap else None, cap, d_degree.data_ptr(), ctypes.byref(ne))
    if rc == TCRNET_ETRUNC:
        err = TcrnetError(rc, _lib.tcrnet_last_error().decode())
        err.n_edges = ne.value
        raise err
    _check(rc)
    return ne.value


def tcrnet_build_device_noalloc(ctx: Context, d_chars, d_offsets, k: int, d_pairs, d_degree,
                                stream=None) -> int:
    """tcrnet_build_device with every intermediate buffer in the library's
    static per-GPU scratch array (the call allocates nothing).  Same
    arguments, result and errors; TCRNET_EINVAL when the build does not fit
    the array (NOALLOC_SCRATCH_BYTES)."""
    n = d_offsets.numel() - 1
    cap = d_pairs.shape[0] if d_pairs is not None else 0
    st = stream.cuda_stream if stream is not None else None
    ne = ctypes.c_uint64()
    rc = _lib.tcrnet_build_device_noalloc(ctx.handle, d_chars.data_ptr(), d_offsets.data_ptr(), n, k, st,
                                          d_pairs.data_ptr() if cap else None, cap, d_degree.data_ptr(),
                                          ctypes.byref(ne))
    if rc == TCRNET_ETRUNC:
        err = TcrnetError(rc, _lib.tcrnet_last_error().decode())
        err.n_edges = ne.value
        raise err
    _check(rc)
    return ne.value


NOALLOC_SCRATCH_BYTES = 64 << 20  # TCRNET_NOALLOC_SCRATCH_BYTES


# tcrnet_seqs as a numpy record (an array of them is filled column-wise:
# hundreds of repertoires cost one assignment per field, not one per entry)
_SEQS_DTYPE = np.dtype({"names": ["data", "offsets", "n"], "formats": ["<u8", "<u8", "<u4"],
                        "offsets": [tcrnet_seqs.data.offset, tcrnet_seqs.offsets.offset, tcrnet_seqs.n.offset],
                        "itemsize": ctypes.sizeof(tcrnet_seqs)})


def tcrnet_build_batch(ctx: Context, reps, k: int) -> list[Graph]:
    conv = [_as_seqs(r) for r in reps]
    nr = len(conv)
    desc = np.zeros(max(1, nr), dtype=_SEQS_DTYPE)
    if nr:
        desc["data"][:nr] = [c.__array_interface__["data"][0] for c, _ in conv]
        desc["offsets"][:nr] = [o.__array_interface__["data"][0] for _, o in conv]
        desc["n"][:nr] = [len(o) - 1 for _, o in conv]
    outs = (ctypes.c_void_p * max(1, nr))()
    _check(_lib.tcrnet_build_batch(ctx.handle, ctypes.cast(desc.ctypes.data, ctypes.POINTER(tcrnet_seqs)), nr, k,
                                   outs))
    if not nr:
        return []
    # every graph owns its arrays from here on; their views come in one call
    owners = [_GraphOwner(ctypes.c_void_p(outs[i])) for i in range(nr)]
    pp = np.zeros(nr, np.uint64)
    ne = np.zeros(nr, np.uint64)
    dp = np.zeros(nr, np.uint64)
    nn = np.zeros(nr, np.uint32)
    xp = np.zeros(nr, np.uint64)
    _check(_lib.tcrnet_graphs_views(outs, nr, pp.ctypes.data, ne.ctypes.data, dp.ctypes.data, nn.ctypes.data,
                                    xp.ctypes.data))
    inf = tcrnet_build_info()
    _check(_lib.tcrnet_graph_info(outs[0], ctypes.byref(inf)))
    info = _info_dict(inf)  # the batched launch's, the same for every graph
    graphs = []
    for i in range(nr):
        o = owners[i]
        pairs = _view(int(pp[i]), ctypes.c_uint32, 2 * int(ne[i]), np.uint32, o).reshape(-1, 2)
        deg = _view(int(dp[i]), ctypes.c_int32, int(nn[i]), np.int32, o)
        graphs.append(Graph(pairs, deg, dict(info), None))
    return graphs


def tcrnet_autotune(ctx: Context, seqs, k: int) -> None:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    _check(_lib.tcrnet_autotune(ctx.handle, ctypes.byref(s), k))


class tcrnet_tune_entry(ctypes.Structure):
    _fields_ = [("texts_per_item", ctypes.c_uint32), ("waves_per_simd", ctypes.c_uint32),
                ("peq_lds", ctypes.c_uint32), ("pack", ctypes.c_uint32), ("ms", ctypes.c_double)]


def tcrnet_autotune_batch(ctx: Context, reps, k: int) -> None:
    conv = [_as_seqs(r) for r in reps]
    arr = (tcrnet_seqs * max(1, len(conv)))()
    for i, (c, o) in enumerate(conv):
        arr[i] = _c_seqs(c, o)
    _check(_lib.tcrnet_autotune_batch(ctx.handle, arr, len(conv), k))


def tcrnet_autotune_get(ctx: Context, batch: bool, n: int, k: int) -> dict | None:
    """The tuned schedule for (form, n, k), or None if there is none."""
    e = tcrnet_tune_entry()
    rc = _lib.tcrnet_autotune_get(ctx.handle, 1 if batch else 0, n, k, ctypes.byref(e))
    if rc == TCRNET_ESTATE:
        return None
    _check(rc)
    return {f: getattr(e, f) for f, _ in tcrnet_tune_entry._fields_}


def tcrnet_autotune_save(ctx: Context, path: str) -> None:
    _check(_lib.tcrnet_autotune_save(ctx.handle, os.fsencode(path)))


def tcrnet_autotune_load(ctx: Context, path: str) -> int:
    n = ctypes.c_uint32()
    _check(_lib.tcrnet_autotune_load(ctx.handle, os.fsencode(path), ctypes.byref(n)))
    return n.value


def tcrnet_valu_peak(ctx: Context) -> tuple[float, float]:
    """Measured 32-bit VALU issue rate (lane-instructions/s) and the seconds
    the probe ran."""
    rate, sec = ctypes.c_double(), ctypes.c_double()
    _check(_lib.tcrnet_valu_peak(ctx.handle, ctypes.byref(rate), ctypes.byref(sec)))
    return rate.value, sec.value


def tcrnet_valu_rates(ctx: Context) -> dict:
    """{instruction form: measured lane-instructions per second}."""
    n = ctypes.c_uint32(0)
    _lib.tcrnet_valu_rates(ctx.handle, None, 0, ctypes.byref(n))  # asks for the count (EINVAL)
    rates = (ctypes.c_double * n.value)()
    _check(_lib.tcrnet_valu_rates(ctx.handle, rates, n.value, ctypes.byref(n)))
    return {_lib.tcrnet_valu_form_name(i).decode(): rates[i] for i in range(n.value)}


def version() -> str:
    load_library()
    return _lib.tcrnet_version().decode()


# ---------------------------------------------------------------- serving
@dataclass
class Result:
    pairs: np.ndarray           # (E, 2) uint32
    counts: np.ndarray          # (M,) int32
    info: dict = field(default_factory=dict)


def _take_result(r) -> Result:
    p = ctypes.c_void_p()
    ne = ctypes.c_uint64()
    _check(_lib.tcrnet_result_pairs(r, ctypes.byref(p), ctypes.byref(ne)))
    E = ne.value
    pairs = (np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint32)), shape=(2 * E,)).copy()
             if E else np.zeros(0, dtype=np.uint32))
    c = ctypes.c_void_p()
    nn = ctypes.c_uint32()
    _check(_lib.tcrnet_result_counts(r, ctypes.byref(c), ctypes.byref(nn)))
    counts = (np.ctypeslib.as_array(ctypes.cast(c, ctypes.POINTER(ctypes.c_int32)), shape=(nn.value,)).copy()
              if nn.value else np.zeros(0, dtype=np.int32))
    inf = tcrnet_result_info()
    _check(_lib.tcrnet_result_info_get(r, ctypes.byref(inf)))
    _lib.tcrnet_result_free(r)
    return Result(pairs.reshape(-1, 2), counts, {f: getattr(inf, f) for f, _ in tcrnet_result_info._fields_})


class Index:
    """A tcrnet_index: resident repertoire with query / insert service."""

    def __init__(self, handle):
        self.handle = handle

    def size(self) -> int:
        n = ctypes.c_uint32()
        _check(_lib.tcrnet_index_size(self.handle, ctypes.byref(n)))
        return n.value

    def degree(self) -> np.ndarray:
        d = ctypes.c_void_p()
        n = ctypes.c_uint32()
        _check(_lib.tcrnet_index_degree(self.handle, ctypes.byref(d), ctypes.byref(n)))
        if not n.value:
            return np.zeros(0, dtype=np.int32)
        return np.ctypeslib.as_array(ctypes.cast(d, ctypes.POINTER(ctypes.c_int32)), shape=(n.value,)).copy()

    def close(self):
        if getattr(self, "handle", None):
            _lib.tcrnet_index_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tcrnet_index_create(ctx: Context, seqs, k_index: int) -> Index:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    h = ctypes.c_void_p()
    _check(_lib.tcrnet_index_create(ctx.handle, ctypes.byref(s), k_index, ctypes.byref(h)))
    return Index(h)


def tcrnet_query(idx: Index, seqs, k: int) -> Result:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    r = ctypes.c_void_p()
    _check(_lib.tcrnet_query(idx.handle, ctypes.byref(s), k, ctypes.byref(r)))
    return _take_result(r)


def tcrnet_insert(idx: Index, seqs) -> Result:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    r = ctypes.c_void_p()
    _check(_lib.tcrnet_insert(idx.handle, ctypes.byref(s), ctypes.byref(r)))
    return _take_result(r)


def tcrnet_submit(idx: Index, seqs, k: int, insert: bool = False) -> int:
    chars, offs = _as_seqs(seqs)
    s = _c_seqs(chars, offs)
    t = ctypes.c_uint64()
    _check(_lib.tcrnet_submit(idx.handle, ctypes.byref(s), k, 1 if insert else 0, ctypes.byref(t)))
    return t.value


def tcrnet_wait(idx: Index, ticket: int) -> Result:
    r = ctypes.c_void_p()
    _check(_lib.tcrnet_wait(idx.handle, ticket, ctypes.byref(r)))
    return _take_result(r)


# --------------------------------------------------------------- analysis
class tcrnet_cc_info(ctypes.Structure):
    _fields_ = [("n_components", ctypes.c_uint32), ("lcc_size", ctypes.c_uint32)]


class tcrnet_stats(ctypes.Structure):
    _fields_ = [("max_degree", ctypes.c_uint32), ("triangles", ctypes.c_uint64), ("assortativity", ctypes.c_double),
                ("avg_clustering", ctypes.c_double), ("sum_jk", ctypes.c_uint64), ("sum_j_plus_k", ctypes.c_uint64),
                ("sum_j2_plus_k2", ctypes.c_uint64)]


_LATE = [
    ("tcrnet_components", _I32, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, _P, _P, ctypes.POINTER(tcrnet_cc_info)]),
    ("tcrnet_robustness", _I32, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, _P, _P, ctypes.c_uint32, _P]),
    ("tcrnet_graph_stats", _I32, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, _P, _P, _P, ctypes.c_uint32, _P,
                                  ctypes.POINTER(tcrnet_stats)]),
    ("tcrnet_lcc_norm", _I32, [_P, _P, ctypes.c_uint32, ctypes.c_uint32, _P, _P]),
]
_SIGS += _LATE
if _lib is not None:  # bound already: add the late signatures
    for _name, _res, _args in _LATE:
        getattr(_lib, _name).restype = _res
        getattr(_lib, _name).argtypes = _args


def _pairs_host(pairs):
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.uint32).reshape(-1, 2))
    return p, len(p)


def tcrnet_components(ctx: Context, pairs, n: int):
    """(labels, sizes, n_components, lcc_size) of the graph on n nodes."""
    p, E = _pairs_host(pairs)
    labels = np.zeros(max(1, n), dtype=np.uint32)
    sizes = np.zeros(max(1, n), dtype=np.uint32)
    info = tcrnet_cc_info()
    _check(_lib.tcrnet_components(ctx.handle, p.ctypes.data if E else None, E, n, labels.ctypes.data,
                                  sizes.ctypes.data, ctypes.byref(info)))
    return labels[:n], sizes[:n], info.n_components, info.lcc_size


def tcrnet_robustness(ctx: Context, pairs, n: int, order, removed) -> np.ndarray:
    """LCC size after removing order[:r] for each r in removed."""
    p, E = _pairs_host(pairs)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    removed = np.ascontiguousarray(removed, dtype=np.uint32)
    out = np.zeros(max(1, len(removed)), dtype=np.uint32)
    _check(_lib.tcrnet_robustness(ctx.handle, p.ctypes.data if E else None, E, n, order.ctypes.data if n else None,
                                  removed.ctypes.data, len(removed), out.ctypes.data))
    return out[:len(removed)]


def tcrnet_lcc_norm(lcc, removed, n: int):
    """(LCC_norm,1, LCC_norm,2) of a percolation curve (paper, "Computing
    LCC"), computed by the library; removed[0] must be 0 for LCC_norm,2."""
    lcc = np.ascontiguousarray(lcc, dtype=np.uint32)
    removed = np.ascontiguousarray(removed, dtype=np.uint32)
    m = len(lcc)
    if len(removed) != m:
        raise ValueError("lcc and removed differ in length")
    n1 = np.zeros(max(1, m), dtype=np.float64)
    n2 = np.zeros(max(1, m), dtype=np.float64)
    want2 = m > 0 and removed[0] == 0
    load_library()
    _check(_lib.tcrnet_lcc_norm(lcc.ctypes.data, removed.ctypes.data, m, n, n1.ctypes.data,
                                n2.ctypes.data if want2 else None))
    return n1[:m], (n2[:m] if want2 else None)


def lcc_norm1(lcc, removed, n: int) -> np.ndarray:
    """LCC(p) / ((1 - p) N) with p = removed / N (paper, "Computing LCC")."""
    return tcrnet_lcc_norm(lcc, removed, n)[0]


def lcc_norm2(lcc, removed, n: int) -> np.ndarray:
    """LCC_norm,1(p) / LCC_norm,1(0); removed[0] must be 0."""
    if np.asarray(removed)[0] != 0:
        raise ValueError("removed[0] must be 0")
    return tcrnet_lcc_norm(lcc, removed, n)[1]


def tcrnet_graph_stats(ctx: Context, pairs, n: int, hist_len: int = 0) -> dict:
    """Degree statistics, assortativity and clustering of a canonical edge
    list (see include/tcrnet.h); hist_len 0 sizes the histograms to the
    maximum degree (one retry)."""
    p, E = _pairs_host(pairs)
    hl = hist_len or 64
    for _ in range(2):
        deg = np.zeros(max(1, n), dtype=np.int32)
        cnt = np.zeros(hl, dtype=np.uint64)
        nbr = np.zeros(hl, dtype=np.uint64)
        clu = np.zeros(max(1, n), dtype=np.float64)
        st = tcrnet_stats()
        rc = _lib.tcrnet_graph_stats(ctx.handle, p.ctypes.data if E else None, E, n, deg.ctypes.data,
                                     cnt.ctypes.data, nbr.ctypes.data, hl, clu.ctypes.data, ctypes.byref(st))
        if rc == TCRNET_ETRUNC and not hist_len:
            hl = st.max_degree + 1
            continue
        _check(rc)
        break
    md = st.max_degree
    return {"degree": deg[:n], "max_degree": md, "count": cnt[:md + 1], "nbr_sum": nbr[:md + 1],
            "clustering": clu[:n], "assortativity": st.assortativity, "avg_clustering": st.avg_clustering,
            "triangles": st.triangles, "sums": (st.sum_jk, st.sum_j_plus_k, st.sum_j2_plus_k2)}

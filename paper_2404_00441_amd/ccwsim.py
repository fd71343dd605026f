"""Python binding of the CCWSIM C ABI (``include/ccwsim.h``).

Argument marshalling only: every function takes torch tensors that live on
the GPU, passes their device pointers and the current HIP stream to
``libccwsim.so`` and raises if the call reports an error.  All computation
happens in the library's HIP kernels; there is no fallback of any kind --
without the built library, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccwsim.so")

CCWSIM_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "invalid shape", 3: "workspace", 4: "HIP error",
          5: "unsupported"}


class CcwsimError(RuntimeError):
    def __init__(self, fn, status, text):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)}: {text}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3)]


class Params(ctypes.Structure):
    _fields_ = [
        ("ti", Shape), ("grid", Shape),
        ("tmpl", ctypes.c_int32 * 3), ("overlap", ctypes.c_int32 * 3),
        ("level", ctypes.c_int32), ("top_k", ctypes.c_int32), ("n_real", ctypes.c_int32),
        ("n_facies", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("path_mode", ctypes.c_int32), ("score_mode", ctypes.c_int32),
        ("nc_margin", ctypes.c_int32 * 3), ("cut", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("shortlist", ctypes.c_int32),
        ("max_hard_data", ctypes.c_int32), ("proposer_dim", ctypes.c_int32), ("hd_direct", ctypes.c_int32),
        ("wavelet", ctypes.c_int32), ("lp_probe", ctypes.c_int32), ("lp_gate", ctypes.c_float),
        ("proposer", ctypes.c_void_p),
    ]


_lib = None


def load():
    """Load ``libccwsim.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2404_00441_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.ccwsim_status_string.restype = ctypes.c_char_p
    L.ccwsim_status_string.argtypes = [ctypes.c_int]
    L.ccwsim_last_error.restype = ctypes.c_char_p
    L.ccwsim_last_error.argtypes = []
    L.ccwsim_dwt_sizes.restype = ctypes.c_int
    L.ccwsim_dwt_sizes.argtypes = [Shape, i32, i32, p, p, p]
    L.ccwsim_dwt.restype = ctypes.c_int
    L.ccwsim_dwt.argtypes = [p, Shape, i32, i32, p, p, p, i64, p]
    L.ccwsim_ccf_scan_workspace_size.restype = i64
    L.ccwsim_ccf_scan_workspace_size.argtypes = [Shape, i32, i32, i32, i32, p, i32, i32, i32, i32, i32]
    L.ccwsim_ccf_scan_noalloc_capacity.restype = i64
    L.ccwsim_ccf_scan_noalloc_capacity.argtypes = []
    L.ccwsim_ccf_scan_noalloc.restype = ctypes.c_int
    L.ccwsim_ccf_scan_noalloc.argtypes = [Shape, i32, i32, i32, i32, p, p, p, p, i32, i32, p, i32, u64, p, p, p, p]
    L.ccwsim_ccf_scan.restype = ctypes.c_int
    L.ccwsim_ccf_scan.argtypes = [Shape, i32, i32, i32, i32, p, p, p, p, i32, i32, p, i32, u64, p, p, p, p, i64, p]
    L.ccwsim_lp_sizes.restype = ctypes.c_int
    L.ccwsim_lp_sizes.argtypes = [Shape, i32, p, i32, p, p, p]
    L.ccwsim_lp_init.restype = ctypes.c_int
    L.ccwsim_lp_init.argtypes = [p, u64, p]
    L.ccwsim_lp_encode.restype = ctypes.c_int
    L.ccwsim_lp_encode.argtypes = [p, p, Shape, i32, p, p, p, i32, p, p, p, p, i64, p]
    L.ccwsim_lp_train_step.restype = ctypes.c_int
    L.ccwsim_lp_train_step.argtypes = [p, p, p, i32, ctypes.c_float, p, Shape, i32, p, p, p, p, i32, i32, p, p, p,
                                       i64, p]
    L.ccwsim_lp_labels.restype = ctypes.c_int
    L.ccwsim_lp_labels.argtypes = [p, i32, i64, i32, p, p]
    L.ccwsim_lp_shortlist.restype = ctypes.c_int
    L.ccwsim_lp_shortlist.argtypes = [p, i32, i64, i32, p, p]
    L.ccwsim_select.restype = ctypes.c_int
    L.ccwsim_select.argtypes = [p, p, i64, i32, i32, u64, p, p, p, p, p]
    L.ccwsim_idwt_workspace_size.restype = i64
    L.ccwsim_idwt_workspace_size.argtypes = [Shape, i32, i32]
    L.ccwsim_idwt.restype = ctypes.c_int
    L.ccwsim_idwt.argtypes = [p, p, Shape, i32, i32, p, i32, p, p, p, i64, p]
    L.ccwsim_simulate_workspace_size.restype = i64
    L.ccwsim_simulate_workspace_size.argtypes = [p]
    L.ccwsim_simulate.restype = ctypes.c_int
    L.ccwsim_simulate.argtypes = [p, p, i64, p, p, p, p, p, p, i64, p]
    L.ccwsim_release_caches.restype = None
    L.ccwsim_release_caches.argtypes = []
    L.ccwsim_cache_counts.restype = ctypes.c_int
    L.ccwsim_cache_counts.argtypes = [p, p]
    L.ccwsim_simulate_stats.restype = ctypes.c_int
    L.ccwsim_simulate_stats.argtypes = [p, p]
    L.ccwsim_profile_enable.restype = ctypes.c_int
    L.ccwsim_profile_enable.argtypes = [ctypes.c_int]
    L.ccwsim_profile_read.restype = ctypes.c_int
    L.ccwsim_profile_read.argtypes = [p, p]
    L.ccwsim_set_graphs.restype = ctypes.c_int
    L.ccwsim_set_graphs.argtypes = [ctypes.c_int]
    L.ccwsim_simulate_report.restype = ctypes.c_int
    L.ccwsim_simulate_report.argtypes = [p, p, i64, p, p]
    L.ccwsim_simulate_events.restype = ctypes.c_int
    L.ccwsim_simulate_events.argtypes = [p, p, i64, p, p, p, p, p]
    L.ccwsim_simulate_match_errors.restype = ctypes.c_int
    L.ccwsim_simulate_match_errors.argtypes = [p, p, i64, p, p]
    L.ccwsim_lp_index_size.restype = ctypes.c_int
    L.ccwsim_lp_index_size.argtypes = [Shape, i32, p, i32, p, p]
    L.ccwsim_lp_build_index.restype = ctypes.c_int
    L.ccwsim_lp_build_index.argtypes = [p, p, Shape, i32, p, i32, i32, p, i64, p, i64, p]
    L.ccwsim_lp_propose_workspace_size.restype = i64
    L.ccwsim_lp_propose_workspace_size.argtypes = [Shape, i32, i32, p]
    L.ccwsim_lp_propose.restype = ctypes.c_int
    L.ccwsim_lp_propose.argtypes = [p, p, Shape, i32, i32, p, p, p, i32, i32, i32, u64, p, p, p, p, p, p, p, p, i64,
                                    p]
    L.ccwsim_set_scan_group.restype = ctypes.c_int
    L.ccwsim_set_scan_group.argtypes = [ctypes.c_int]
    L.ccwsim_set_selection.restype = ctypes.c_int
    L.ccwsim_set_selection.argtypes = [ctypes.c_int]
    L.ccwsim_set_proposer_skew.restype = ctypes.c_int
    L.ccwsim_set_proposer_skew.argtypes = [ctypes.c_float]
    L.ccwsim_stats_workspace_size.restype = i64
    L.ccwsim_stats_workspace_size.argtypes = [Shape, i32]
    L.ccwsim_stats_histogram.restype = ctypes.c_int
    L.ccwsim_stats_histogram.argtypes = [p, Shape, i32, i32, p, p, p]
    L.ccwsim_stats_variogram.restype = ctypes.c_int
    L.ccwsim_stats_variogram.argtypes = [p, Shape, i32, i32, i32, i32, p, p, i64, p]
    L.ccwsim_stats_connectivity.restype = ctypes.c_int
    L.ccwsim_stats_connectivity.argtypes = [p, Shape, i32, i32, i32, i32, p, p, p, i64, p]
    L.ccwsim_dwt97_workspace_size.restype = i64
    L.ccwsim_dwt97_workspace_size.argtypes = [Shape, i32]
    L.ccwsim_dwt97.restype = ctypes.c_int
    L.ccwsim_dwt97.argtypes = [p, Shape, i32, p, p, p, i64, p]
    L.ccwsim_idwt97.restype = ctypes.c_int
    L.ccwsim_idwt97.argtypes = [p, p, Shape, i32, p, p, i64, p]
    L.ccwsim_ccf_scan97_workspace_size.restype = i64
    L.ccwsim_ccf_scan97_workspace_size.argtypes = [Shape, i32, i32, p, i32, i32, i32, i32, i32]
    L.ccwsim_ccf_scan97.restype = ctypes.c_int
    L.ccwsim_ccf_scan97.argtypes = [Shape, i32, i32, p, p, p, p, i32, p, i32, i32, u64, p, p, p, p, p, i64, p]
    _lib = L
    return L


EXPORTS = ("ccwsim_status_string", "ccwsim_last_error", "ccwsim_dwt_sizes", "ccwsim_dwt",
           "ccwsim_ccf_scan", "ccwsim_ccf_scan_workspace_size", "ccwsim_ccf_scan_noalloc",
           "ccwsim_ccf_scan_noalloc_capacity", "ccwsim_idwt_workspace_size", "ccwsim_lp_sizes",
           "ccwsim_lp_init", "ccwsim_lp_encode", "ccwsim_lp_train_step", "ccwsim_lp_shortlist", "ccwsim_select", "ccwsim_idwt", "ccwsim_simulate_workspace_size",
           "ccwsim_simulate", "ccwsim_release_caches", "ccwsim_simulate_stats", "ccwsim_profile_enable",
           "ccwsim_profile_read", "ccwsim_set_graphs", "ccwsim_simulate_report", "ccwsim_set_scan_group",
           "ccwsim_set_selection", "ccwsim_stats_workspace_size", "ccwsim_stats_histogram", "ccwsim_stats_variogram",
           "ccwsim_stats_connectivity", "ccwsim_cache_counts",
           "ccwsim_simulate_events", "ccwsim_simulate_match_errors", "ccwsim_lp_index_size", "ccwsim_lp_build_index",
           "ccwsim_lp_propose_workspace_size", "ccwsim_lp_propose", "ccwsim_set_proposer_skew",
           "ccwsim_lp_labels", "ccwsim_dwt97_workspace_size", "ccwsim_dwt97", "ccwsim_idwt97",
           "ccwsim_ccf_scan97_workspace_size", "ccwsim_ccf_scan97")

KINDS = ("dwt", "energy", "init", "prepare", "scan", "finalize", "crop", "learn")


class PlanStats(ctypes.Structure):
    _fields_ = [("patches", ctypes.c_int64), ("wavefront_steps", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("or_blocks", ctypes.c_int64),
                ("scan_flops", ctypes.c_double), ("key_bytes", ctypes.c_double), ("cells", ctypes.c_double),
                ("fin_bytes", ctypes.c_double)]


def _check(fn, status):
    if status != CCWSIM_OK:
        raise CcwsimError(fn, status, load().ccwsim_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def shape_of(extent) -> Shape:
    """Shape from an (x, y[, z]) extent."""
    n = list(extent) + [1] * (3 - len(extent))
    return Shape(len(extent), (ctypes.c_int32 * 3)(*n))


def _i3(v, fill):
    v = list(v) + [fill] * (3 - len(v))
    return (ctypes.c_int32 * 3)(*v)


def params_of(p: dict) -> Params:
    """Params from a workload dict (extents (x, y[, z]))."""
    q = Params()
    q.ti = shape_of(p["ti"])
    q.grid = shape_of(p["grid"])
    nd = len(p["ti"])
    q.tmpl = _i3(p["tmpl"], 1)
    q.overlap = _i3(p["overlap"], 0)
    q.level = p["level"]
    q.top_k = p["top_k"]
    q.n_real = p.get("n_real", 1)
    q.n_facies = p.get("n_facies", 2)
    q.seed = p.get("seed", 1)
    q.path_mode = p.get("path_mode", 0)
    q.score_mode = p.get("score_mode", 0)
    m = list(p.get("nc_margin", (-1, -1, -1)))[:nd] + [-1] * (3 - nd)
    q.nc_margin = (ctypes.c_int32 * 3)(*m)
    q.cut = p.get("cut", 1)
    q.precision = p.get("precision", 0)
    q.shortlist = int(p.get("shortlist", 0))
    q.max_hard_data = int(p.get("max_hard_data", 0))
    q.proposer_dim = int(p.get("proposer_dim", 0))
    q.hd_direct = int(p.get("hd_direct", 0))
    q.wavelet = int(p.get("wavelet", 0))
    q.lp_probe = int(p.get("lp_probe", 0))
    q.lp_gate = float(p.get("lp_gate", 0.0))
    ix = p.get("proposer")
    q.proposer = ctypes.c_void_p(ix.data_ptr() if ix is not None else None)
    return q


# ---------------------------------------------------------------------------
def dwt_sizes(extent, level, wavelet=0):
    na, nd, nw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check("ccwsim_dwt_sizes", load().ccwsim_dwt_sizes(shape_of(extent), level, wavelet, ctypes.byref(na),
                                                       ctypes.byref(nd), ctypes.byref(nw)))
    return na.value, nd.value, nw.value


def dwt(x: torch.Tensor, level: int, wavelet: int = 0):
    """x: int8 GPU tensor in numpy order ([y][x] or [z][y][x]).
    Returns (approx int32 [grid], details int32 flat)."""
    extent = tuple(x.shape[::-1])
    na, nd, nw = dwt_sizes(extent, level, wavelet)
    b = 2 ** level
    grid = tuple(-(-n // b) for n in x.shape)
    approx = torch.empty(grid, dtype=torch.int32, device=x.device)
    details = torch.empty(max(nd, 1), dtype=torch.int32, device=x.device)
    _, ws = _aligned_workspace(nw, x.device)
    _check("ccwsim_dwt", load().ccwsim_dwt(_ptr(x), shape_of(extent), level, wavelet, _ptr(approx), _ptr(details),
                                           _ptr(ws), nw, _stream()))
    return approx, details[:nd]


def _aligned_workspace(nbytes, device):
    """Caller-owned workspace, 256-byte aligned."""
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:]


def ccf_scan_workspace_size(ti_extent, level, max_code, tmpl, n_filters, score_mode=0, precision=0, wavelet=0,
                            top_k=0, want_scores=True, want_keys=False):
    v = load().ccwsim_ccf_scan_workspace_size(shape_of(ti_extent), level, wavelet, max_code, precision,
                                              _i3(tmpl, 1), n_filters, score_mode, top_k, int(want_scores),
                                              int(want_keys))
    if v < 0:
        raise CcwsimError("ccwsim_ccf_scan_workspace_size", 1, load().ccwsim_last_error().decode())
    return int(v)


def ccf_scan(ti_extent, level, max_code, approx, tmpl, or_n, or_m, score_mode=0, precision=0, wavelet=0,
             top_k=None, seed=0, realization=None, step=None, want_scores=None):
    """or_n, or_m: int32 [n_filters, *T_c numpy order].  Without top_k:
    returns int32 scores [n_filters, n_cand].  With top_k: the selection is
    fused into the scan and (scores or None, keys uint64-as-int64
    [n_filters, min(top_k, n_cand)]) is returned; realization int32 [F] and
    step int64 [F] key the tie-break; the score map is written only when
    want_scores is true."""
    nf = or_m.shape[0]
    b = 2 ** level
    cand = [(ti_extent[a] - tmpl[a]) // b + 1 for a in range(len(ti_extent))]
    ncand = 1
    for c in cand:
        ncand *= c
    fused = top_k is not None
    if want_scores is None:
        want_scores = not fused
    scores = torch.empty((nf, ncand), dtype=torch.int32, device=approx.device) if want_scores else None
    keys = torch.empty((nf, min(top_k, ncand)), dtype=torch.int64, device=approx.device) if fused else None
    ws_bytes = ccf_scan_workspace_size(ti_extent, level, max_code, tmpl, nf, score_mode, precision, wavelet,
                                       top_k or 0, want_scores, fused)
    _, ws = _aligned_workspace(ws_bytes, approx.device)
    t3 = _i3(tmpl, 1)
    _check("ccwsim_ccf_scan", load().ccwsim_ccf_scan(shape_of(ti_extent), level, wavelet, max_code, precision,
                                                     _ptr(approx), t3, _ptr(or_n) if or_n is not None else None,
                                                     _ptr(or_m), nf, score_mode, _ptr(scores), top_k or 0, seed,
                                                     _ptr(realization), _ptr(step), _ptr(keys), _ptr(ws),
                                                     ws_bytes, _stream()))
    if not fused:
        return scores
    return scores, keys


def dwt97(x: torch.Tensor, level: int):
    """CDF 9/7 DWT in fp32.  x: int8 GPU tensor in numpy order.  Returns
    (approx float32 [grid], details float32 flat, in the layout of dwt)."""
    extent = tuple(x.shape[::-1])
    _, nd, _ = dwt_sizes(extent, level, 0)
    nw = int(load().ccwsim_dwt97_workspace_size(shape_of(extent), level))
    if nw < 0:
        raise CcwsimError("ccwsim_dwt97_workspace_size", 1, load().ccwsim_last_error().decode())
    b = 2 ** level
    grid = tuple(-(-n // b) for n in x.shape)
    approx = torch.empty(grid, dtype=torch.float32, device=x.device)
    details = torch.empty(max(nd, 1), dtype=torch.float32, device=x.device)
    _, ws = _aligned_workspace(nw, x.device)
    _check("ccwsim_dwt97", load().ccwsim_dwt97(_ptr(x), shape_of(extent), level, _ptr(approx), _ptr(details),
                                               _ptr(ws), nw, _stream()))
    return approx, details[:nd]


def idwt97(approx: torch.Tensor, details: torch.Tensor, ti_extent, level: int):
    """Inverse of dwt97: the edge-replicated image, float32 in numpy order."""
    nw = int(load().ccwsim_dwt97_workspace_size(shape_of(ti_extent), level))
    if nw < 0:
        raise CcwsimError("ccwsim_dwt97_workspace_size", 1, load().ccwsim_last_error().decode())
    b = 2 ** level
    np_ = tuple(-(-n // b) * b for n in ti_extent)[::-1]
    img = torch.empty(np_, dtype=torch.float32, device=approx.device)
    _, ws = _aligned_workspace(nw, approx.device)
    _check("ccwsim_idwt97", load().ccwsim_idwt97(_ptr(approx), _ptr(details) if details.numel() else None,
                                                 shape_of(ti_extent), level, _ptr(img), _ptr(ws), nw, _stream()))
    return img


def ccf_scan97(ti_extent, level, approx, tmpl, or_n, or_m, top_k=None, shortlist=0, precision=0, seed=0,
               realization=None, step=None, want_scores=None, want_shortlist=False):
    """CDF 9/7 scores.  approx float32 [grid]; or_n int32 (0/1) and or_m
    float32 [n_filters, T_c cells].  Without top_k: float32 scores
    [n_filters, n_cand].  With top_k: (scores or None, keys int64 [n_filters,
    top_k], shortlist int32 [n_filters, R] or None); shortlist 0 rescores
    every candidate in fp32, R < n_cand ranks them first with the fp16 /
    bf16 bulk (precision 0 / 1)."""
    nf = or_m.shape[0]
    b = 2 ** level
    cand = [(ti_extent[a] - tmpl[a]) // b + 1 for a in range(len(ti_extent))]
    ncand = 1
    for c in cand:
        ncand *= c
    fused = top_k is not None
    if want_scores is None:
        want_scores = not fused
    dev = approx.device
    scores = torch.empty((nf, ncand), dtype=torch.float32, device=dev) if want_scores else None
    keys = torch.empty((nf, top_k), dtype=torch.int64, device=dev) if fused else None
    R = min(shortlist, ncand) if shortlist else ncand
    sl = torch.empty((nf, R), dtype=torch.int32, device=dev) if (want_shortlist and fused and R < ncand) else None
    t3 = _i3(tmpl, 1)
    ws_bytes = int(load().ccwsim_ccf_scan97_workspace_size(shape_of(ti_extent), level, precision, t3, nf,
                                                            top_k or 0, shortlist, int(want_scores), int(fused)))
    if ws_bytes < 0:
        raise CcwsimError("ccwsim_ccf_scan97_workspace_size", 1, load().ccwsim_last_error().decode())
    _, ws = _aligned_workspace(ws_bytes, dev)
    _check("ccwsim_ccf_scan97", load().ccwsim_ccf_scan97(shape_of(ti_extent), level, precision, _ptr(approx), t3,
                                                         _ptr(or_n), _ptr(or_m), nf, _ptr(scores), top_k or 0,
                                                         shortlist, seed, _ptr(realization), _ptr(step), _ptr(keys),
                                                         _ptr(sl), _ptr(ws), ws_bytes, _stream()))
    if not fused:
        return scores
    return scores, keys, sl


def select(scores, mismatch, top_k, seed, realization, step, want_keys=False):
    """scores int32 [F, n]; mismatch uint16-compatible int16 [F, n] or None;
    realization int32 [F]; step int64 [F].  Returns (chosen int32 [F],
    keys uint64-as-int64 [F, k'] or None)."""
    nf, n = scores.shape
    chosen = torch.empty(nf, dtype=torch.int32, device=scores.device)
    k = min(top_k, n)
    keys = torch.empty((nf, k), dtype=torch.int64, device=scores.device) if want_keys else None
    _check("ccwsim_select", load().ccwsim_select(_ptr(scores), _ptr(mismatch), n, nf, top_k, seed,
                                                 _ptr(realization), _ptr(step), _ptr(chosen), _ptr(keys),
                                                 _stream()))
    return chosen, keys


def idwt(approx, details, ti_extent, level, origins, patch, wavelet=0):
    """origins int32 [n, 3] (x, y, z block origins).  Returns int8 patterns
    [n, *patch numpy order]."""
    n = origins.shape[0]
    out = torch.empty((n,) + tuple(patch[::-1]), dtype=torch.int8, device=approx.device)
    nw = load().ccwsim_idwt_workspace_size(shape_of(ti_extent), level, wavelet)
    if nw < 0:
        raise CcwsimError("ccwsim_idwt_workspace_size", 1, load().ccwsim_last_error().decode())
    _, ws = _aligned_workspace(nw, approx.device)
    _check("ccwsim_idwt", load().ccwsim_idwt(_ptr(approx), _ptr(details), shape_of(ti_extent), level, wavelet,
                                             _ptr(origins), n, _i3(patch, 1), _ptr(out), _ptr(ws), nw, _stream()))
    return out


# ---------------------------------------------------------------------------
# learned proposer (training and encoding)
# ---------------------------------------------------------------------------
def lp_sizes(ti_extent, level, tmpl, batch):
    nw, ws, nc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check("ccwsim_lp_sizes", load().ccwsim_lp_sizes(shape_of(ti_extent), level, _i3(tmpl, 1), batch,
                                                     ctypes.byref(nw), ctypes.byref(ws), ctypes.byref(nc)))
    return nw.value, ws.value, nc.value


def lp_init(seed: int, device="cuda"):
    nw, _, _ = lp_sizes((64, 64), 2, (16, 16), 0)
    w = torch.empty(nw, dtype=torch.float32, device=device)
    _check("ccwsim_lp_init", load().ccwsim_lp_init(_ptr(w), seed, _stream()))
    return w


class LpWorkspace:
    """Workspace of the proposer for one TI geometry and batch size."""

    def __init__(self, ti_extent, level, tmpl, batch, device="cuda"):
        self.args = (tuple(ti_extent), level, tuple(tmpl), batch)
        self.nw, self.nbytes, self.ncand = lp_sizes(ti_extent, level, tmpl, batch)
        self._buf, self.ws = _aligned_workspace(self.nbytes, device)


def lp_encode(w, approx, ws: LpWorkspace, or_n=None, or_m=None, want_keys=True, want_queries=False,
              want_scores=False):
    """Keys [ncand, 64] of the TI, queries [B, 64] and scores [B, ncand] of
    the data events (or_n / or_m int32 [B, T_c cells], as for ccf_scan)."""
    ext, level, tmpl, batch = ws.args
    dev = approx.device
    B = 0 if or_n is None else or_n.shape[0]
    assert B <= batch
    keys = torch.empty((ws.ncand, 64), dtype=torch.float32, device=dev) if want_keys else None
    q = torch.empty((max(B, 1), 64), dtype=torch.float32, device=dev) if want_queries else None
    S = torch.empty((max(B, 1), ws.ncand), dtype=torch.float32, device=dev) if want_scores else None
    _check("ccwsim_lp_encode", load().ccwsim_lp_encode(_ptr(w), _ptr(approx), shape_of(ext), level, _i3(tmpl, 1),
                                                       _ptr(or_n) if B else None, _ptr(or_m) if B else None, B,
                                                       _ptr(keys), _ptr(q), _ptr(S),
                                                       _ptr(ws.ws), ws.nbytes, _stream()))
    return keys, q, S


def lp_train_step(w, m, v, step, lr, approx, ws: LpWorkspace, or_n, or_m, labels, want_grad=False):
    """One Adam step on a batch of data events (or_n / or_m int32 [B, T_c
    cells]) and their labels (int32 [B] or [B, L]: distinct positive
    candidates per event); returns the per-example losses (and the gradient
    before the update when asked)."""
    ext, level, tmpl, batch = ws.args
    B = or_n.shape[0]
    n_pos = 1 if labels.dim() == 1 else int(labels.shape[1])
    assert B == batch
    loss = torch.empty(B, dtype=torch.float32, device=approx.device)
    g = torch.empty_like(w) if want_grad else None
    _check("ccwsim_lp_train_step", load().ccwsim_lp_train_step(_ptr(w), _ptr(m), _ptr(v), step, lr, _ptr(approx),
                                                               shape_of(ext), level, _i3(tmpl, 1), _ptr(or_n),
                                                               _ptr(or_m), _ptr(labels), n_pos, B, _ptr(loss), _ptr(g),
                                                               _ptr(ws.ws),
                                                               ws.nbytes, _stream()))
    return loss, g


def lp_shortlist(scores, k):
    B, n = scores.shape
    idx = torch.empty((B, k), dtype=torch.int32, device=scores.device)
    _check("ccwsim_lp_shortlist", load().ccwsim_lp_shortlist(_ptr(scores), B, n, k, _ptr(idx), _stream()))
    return idx


def lp_labels(scores, k):
    """The k smallest exact scores' candidate indices per row (int32 [B, k],
    ties to the smaller index, ascending)."""
    B, n = scores.shape
    idx = torch.empty((B, k), dtype=torch.int32, device=scores.device)
    _check("ccwsim_lp_labels", load().ccwsim_lp_labels(_ptr(scores), B, n, k, _ptr(idx), _stream()))
    return idx


def lp_index_size(ti_extent, level, tmpl, n_lists):
    nb, ws = ctypes.c_int64(), ctypes.c_int64()
    _check("ccwsim_lp_index_size", load().ccwsim_lp_index_size(shape_of(ti_extent), level, _i3(tmpl, 1), n_lists,
                                                               ctypes.byref(nb), ctypes.byref(ws)))
    return nb.value, ws.value


def lp_build_index(w, approx, ti_extent, level, tmpl, n_lists, iters=10):
    """Inverted-list index of the keys (uint8 device tensor, 256-byte aligned
    view) for ccwsim_simulate's `proposer`."""
    nb, nws = lp_index_size(ti_extent, level, tmpl, n_lists)
    _, ix = _aligned_workspace(nb, approx.device)
    _, ws = _aligned_workspace(nws, approx.device)
    _check("ccwsim_lp_build_index", load().ccwsim_lp_build_index(_ptr(w), _ptr(approx), shape_of(ti_extent), level,
                                                                 _i3(tmpl, 1), n_lists, iters, _ptr(ix), nb,
                                                                 _ptr(ws), nws, _stream()))
    return ix


LP_CAND_MAX = 1792


def lp_propose(index, approx, ti_extent, level, max_code, tmpl, or_n, or_m, probe, top_k, seed=0, realization=None,
               step=None):
    """The proposal for each data event: (keys int64 [F, k], members int32
    [F, 1792], n_members int32 [F], queries float32 [F, 64], best match
    error float32 [F])."""
    F = or_n.shape[0]
    dev = approx.device
    nws = load().ccwsim_lp_propose_workspace_size(shape_of(ti_extent), level, max_code, _i3(tmpl, 1))
    if nws < 0:
        raise CcwsimError("ccwsim_lp_propose_workspace_size", 1, load().ccwsim_last_error().decode())
    _, ws = _aligned_workspace(nws, dev)
    b = 2 ** level
    ncand = 1
    for a, t in zip(ti_extent, tmpl):
        ncand *= (a - t) // b + 1
    k = min(top_k, ncand)
    keys = torch.empty((max(F, 1), k), dtype=torch.int64, device=dev)
    mem = torch.empty((max(F, 1), LP_CAND_MAX), dtype=torch.int32, device=dev)
    nmem = torch.empty(max(F, 1), dtype=torch.int32, device=dev)
    q = torch.empty((max(F, 1), 64), dtype=torch.float32, device=dev)
    err = torch.empty(max(F, 1), dtype=torch.float32, device=dev)
    _check("ccwsim_lp_propose", load().ccwsim_lp_propose(_ptr(index), _ptr(approx), shape_of(ti_extent), level,
                                                         max_code, _i3(tmpl, 1), _ptr(or_n), _ptr(or_m), F, probe,
                                                         top_k, seed, _ptr(realization), _ptr(step), _ptr(keys),
                                                         _ptr(mem), _ptr(nmem), _ptr(q), _ptr(err), _ptr(ws), nws,
                                                         _stream()))
    return keys[:F], mem[:F], nmem[:F], q[:F], err[:F]


def simulate_workspace_size(p: dict) -> int:
    q = params_of(p)
    v = load().ccwsim_simulate_workspace_size(ctypes.byref(q))
    if v < 0:
        raise CcwsimError("ccwsim_simulate_workspace_size", 1, load().ccwsim_last_error().decode())
    return int(v)


class Simulator:
    """Holds the workspace for one parameter set and runs ccwsim_simulate."""

    def __init__(self, p: dict, device="cuda"):
        self.p = dict(p)
        self.q = params_of(p)
        self.ws_bytes = simulate_workspace_size(p)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off: off + self.ws_bytes]

    def run(self, ti, hd=None, out=None, chosen=None):
        """ti: int8 GPU tensor (numpy order).  hd: (real int32 [n], pos int32
        [n, 3], val int8 [n]) GPU tensors or None.  Returns out int8
        [n_real, *grid numpy order]."""
        p = self.p
        if out is None:
            out = torch.empty((p["n_real"],) + tuple(p["grid"][::-1]), dtype=torch.int8, device=ti.device)
        if hd is None:
            n_hd, hr, hp, hv = 0, None, None, None
        else:
            hr, hp, hv = hd
            n_hd = int(hr.shape[0])
        _check("ccwsim_simulate", load().ccwsim_simulate(
            ctypes.byref(self.q), _ptr(ti), n_hd, _ptr(hr) if n_hd else None, _ptr(hp) if n_hd else None,
            _ptr(hv) if n_hd else None, _ptr(out), _ptr(chosen), ctypes.c_void_p(self.ws_view.data_ptr()),
            self.ws_bytes, _stream()))
        return out


    def report(self) -> dict:
        """Shortlist rescoring and proposer report of the last run (synchronises)."""
        out = (ctypes.c_int64 * 8)()
        _check("ccwsim_simulate_report", load().ccwsim_simulate_report(
            ctypes.byref(self.q), ctypes.c_void_p(self.ws_view.data_ptr()), self.ws_bytes, out, _stream()))
        return {"max_abs_error": out[0], "rescored": out[1], "topk_changed": out[2], "patches": out[3],
                "proposer_patches": out[4], "proposer_rows": out[5], "proposer_fallbacks": out[6]}

    def n_patches(self) -> int:
        return int(simulate_stats(self.p)["patches"])

    def events(self):
        """Every patch's data event of the last run: (or_n, or_m int32
        [patches, T_c cells], realization int32 [patches], step int32
        [patches]), in plan order."""
        n = self.n_patches()
        b = 2 ** self.p["level"]
        tc = 1
        for t in self.p["tmpl"]:
            tc *= (t + b - 1) // b
        dev = self.ws.device
        on = torch.empty((n, tc), dtype=torch.int32, device=dev)
        om = torch.empty((n, tc), dtype=torch.int32, device=dev)
        rr = torch.empty(n, dtype=torch.int32, device=dev)
        ss = torch.empty(n, dtype=torch.int32, device=dev)
        _check("ccwsim_simulate_events", load().ccwsim_simulate_events(
            ctypes.byref(self.q), ctypes.c_void_p(self.ws_view.data_ptr()), self.ws_bytes, _ptr(on), _ptr(om),
            _ptr(rr), _ptr(ss), _stream()))
        return on, om, rr, ss

    def match_errors(self):
        """Match error of every patch's drawn candidate (float32 [patches],
        plan order; -1 where the overlap is empty)."""
        out = torch.empty(self.n_patches(), dtype=torch.float32, device=self.ws.device)
        _check("ccwsim_simulate_match_errors", load().ccwsim_simulate_match_errors(
            ctypes.byref(self.q), ctypes.c_void_p(self.ws_view.data_ptr()), self.ws_bytes, _ptr(out), _stream()))
        return out


def hd_to_device(hd, ndim, device="cuda"):
    """(real, pos (n, ndim), val) numpy -> GPU tensors with pos padded to 3."""
    if hd is None or len(hd[0]) == 0:
        return None
    import numpy as np
    real, pos, val = hd
    pos3 = np.zeros((len(real), 3), dtype=np.int32)
    pos3[:, :ndim] = pos
    return (torch.from_numpy(np.ascontiguousarray(real, dtype=np.int32)).to(device),
            torch.from_numpy(pos3).to(device),
            torch.from_numpy(np.ascontiguousarray(val, dtype=np.int8)).to(device))


def release_caches():
    load().ccwsim_release_caches()


def cache_counts() -> tuple:
    """(plans, graphs) held by the library's host caches."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check("ccwsim_cache_counts", load().ccwsim_cache_counts(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def simulate_stats(p: dict) -> dict:
    s = PlanStats()
    _check("ccwsim_simulate_stats", load().ccwsim_simulate_stats(ctypes.byref(params_of(p)), ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in PlanStats._fields_}


def set_scan_group(g: int):
    """0: tuned tiles per scan workgroup; 1, 2, 4 or 8: forced."""
    _check("ccwsim_set_scan_group", load().ccwsim_set_scan_group(int(g)))


def set_selection(mode: int):
    """0: tuned; 1: stored keys; 2: row minima with exact rescoring of rows."""
    _check("ccwsim_set_selection", load().ccwsim_set_selection(mode))


def set_proposer_skew(s: float):
    _check("ccwsim_set_proposer_skew", load().ccwsim_set_proposer_skew(s))


def set_graphs(on: bool):
    _check("ccwsim_set_graphs", load().ccwsim_set_graphs(1 if on else 0))


def profile_enable(on: bool):
    _check("ccwsim_profile_enable", load().ccwsim_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """Per kernel kind: (total ms, launches) since the last read."""
    ms = (ctypes.c_double * len(KINDS))()
    n = (ctypes.c_int64 * len(KINDS))()
    _check("ccwsim_profile_read", load().ccwsim_profile_read(ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(KINDS)}


# ---- realization statistics (Sec. 5.2, 5.3, 5.8) ----
def _stack(imgs: torch.Tensor):
    """int8 GPU stack [image][y][x] or [image][z][y][x] -> (n_img, Shape)."""
    if imgs.dtype != torch.int8 or imgs.dim() not in (3, 4):
        raise ValueError("images must be an int8 [image][y][x] or [image][z][y][x] tensor")
    return imgs.shape[0], shape_of(tuple(imgs.shape[1:][::-1]))


def stats_histogram(imgs: torch.Tensor, n_facies: int, per_cell: bool = True):
    """(per_image int64 [image][facies], per_cell int32 [facies][..cells] or
    None): cells holding each facies per image, images holding each facies
    per cell (the ensemble map times the number of images)."""
    n, sh = _stack(imgs)
    pi = torch.empty((n, n_facies), dtype=torch.int64, device=imgs.device)
    pc = torch.empty((n_facies,) + tuple(imgs.shape[1:]), dtype=torch.int32, device=imgs.device) if per_cell else None
    _check("ccwsim_stats_histogram", load().ccwsim_stats_histogram(_ptr(imgs), sh, n, n_facies, _ptr(pi), _ptr(pc),
                                                                   _stream()))
    return pi, pc


def _stats_ws(imgs, sh, n):
    nb = load().ccwsim_stats_workspace_size(sh, n)
    if nb < 0:
        raise CcwsimError("ccwsim_stats_workspace_size", 1, load().ccwsim_last_error().decode())
    ws = torch.empty(max(nb, 256) + 256, dtype=torch.uint8, device=imgs.device)
    off = (-ws.data_ptr()) % 256
    return ws, ctypes.c_void_p(ws.data_ptr() + off), nb


def stats_variogram(imgs: torch.Tensor, n_facies: int, axis: int, max_lag: int) -> torch.Tensor:
    """int64 [image][facies][max_lag]: pairs (x, x + h e_axis), h = 1..max_lag,
    whose indicators of the facies differ; gamma = diff / (2 N(h))."""
    n, sh = _stack(imgs)
    out = torch.empty((n, n_facies, max_lag), dtype=torch.int64, device=imgs.device)
    ws, wp, nb = _stats_ws(imgs, sh, n)
    _check("ccwsim_stats_variogram", load().ccwsim_stats_variogram(_ptr(imgs), sh, n, n_facies, axis, max_lag,
                                                                   _ptr(out), wp, nb, _stream()))
    return out


def stats_connectivity(imgs: torch.Tensor, n_facies: int, axis: int, max_lag: int):
    """(both, connected) int64 [image][facies][max_lag]: pairs at lag h along
    the axis whose cells both hold the facies, and those of them whose cells
    share a face-connected component; the probability of connection is
    connected / both."""
    n, sh = _stack(imgs)
    both = torch.empty((n, n_facies, max_lag), dtype=torch.int64, device=imgs.device)
    conn = torch.empty_like(both)
    ws, wp, nb = _stats_ws(imgs, sh, n)
    _check("ccwsim_stats_connectivity", load().ccwsim_stats_connectivity(_ptr(imgs), sh, n, n_facies, axis, max_lag,
                                                                         _ptr(both), _ptr(conn), wp, nb, _stream()))
    return both, conn


def pair_count(extent, axis: int, h: int) -> int:
    """N(h): cell pairs at lag h along `axis` in an image of (x, y[, z]) extent."""
    n = list(extent)
    n[axis] = max(0, n[axis] - h)
    out = 1
    for v in n:
        out *= v
    return out

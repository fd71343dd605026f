"""ctypes binding of the plain CPU oracle (``ccwsim_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  It loads
``liboracle_ccwsim.so`` built from ``ccwsim_oracle.c`` with gcc
(``build_oracle()``), converts numpy arrays to plain pointers and back, and
does no arithmetic of the method itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ccwsim_oracle.c")
LIB = os.path.join(HERE, "liboracle_ccwsim.so")

STREAM_PATH = 1
STREAM_TIEBREAK = 2
STREAM_DRAW = 3


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc into ``liboracle_ccwsim.so`` (in-tree)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = ctypes.CDLL(LIB)
        u64, i32, i64, p = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.orc_rng.restype = u64
        L.orc_rng.argtypes = [u64, u64, u64, u64]
        L.orc_splitmix_first.restype = u64
        L.orc_splitmix_first.argtypes = [u64]
        L.orc_perm20.restype = ctypes.c_uint32
        L.orc_perm20.argtypes = [ctypes.c_uint32, u64]
        L.orc_details_count.restype = i64
        L.orc_details_count.argtypes = [p, i32, i32]
        L.orc_dwt.restype = ctypes.c_int
        L.orc_dwt.argtypes = [p, p, i32, i32, p, p]
        L.orc_idwt_region.restype = ctypes.c_int
        L.orc_idwt_region.argtypes = [p, p, p, i32, i32, p, p, p]
        L.orc_scores.restype = ctypes.c_int
        L.orc_scores.argtypes = [p, p, p, p, i64, p, p, i32, p]
        L.orc_select.restype = ctypes.c_int
        L.orc_select.argtypes = [p, p, i64, i32, u64, i64, i64, p, p]
        L.orc_mincut.restype = ctypes.c_int
        L.orc_mincut.argtypes = [p, i32, i32, p]
        L.orc_geometry.restype = ctypes.c_int
        L.orc_geometry.argtypes = [p, p]
        L.orc_simulate.restype = ctypes.c_int
        L.orc_simulate.argtypes = [p, p, i64, p, p, p, p, p, p]
        L.orc_lift53_forward.restype = ctypes.c_int
        L.orc_lift53_forward.argtypes = [p, i64, p, p]
        L.orc_lift53_inverse.restype = ctypes.c_int
        L.orc_lift53_inverse.argtypes = [p, p, i64, p]
        L.orc_approx53.restype = ctypes.c_int
        L.orc_approx53.argtypes = [p, p, i32, i32, p]
        _lib = L
    return _lib


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("ti_n", ctypes.c_int32 * 3),
        ("sg_n", ctypes.c_int32 * 3),
        ("tmpl", ctypes.c_int32 * 3),
        ("overlap", ctypes.c_int32 * 3),
        ("level", ctypes.c_int32),
        ("top_k", ctypes.c_int32),
        ("n_real", ctypes.c_int32),
        ("n_facies", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("path_mode", ctypes.c_int32),
        ("score_mode", ctypes.c_int32),
        ("nc_margin", ctypes.c_int32 * 3),
        ("cut", ctypes.c_int32),
        ("wavelet", ctypes.c_int32),
    ]


@dataclass
class SimParams:
    """Problem statement of Algorithm 1 (TI, template, overlap, level, K, n_r)
    plus the readings the paper leaves open.  Extents are (x, y[, z])."""
    ti: tuple
    grid: tuple
    tmpl: tuple
    overlap: tuple
    level: int
    top_k: int
    n_real: int = 1
    n_facies: int = 2
    seed: int = 1
    path_mode: int = 0
    score_mode: int = 0
    nc_margin: tuple = field(default=(-1, -1, -1))
    cut: int = 1
    wavelet: int = 0

    @property
    def ndim(self) -> int:
        return len(self.ti)

    def _pad3(self, t, fill):
        t = list(t) + [fill] * (3 - len(t))
        return (ctypes.c_int32 * 3)(*t)

    def to_oracle(self) -> OracleParams:
        p = OracleParams()
        p.ndim = self.ndim
        p.ti_n = self._pad3(self.ti, 1)
        p.sg_n = self._pad3(self.grid, 1)
        p.tmpl = self._pad3(self.tmpl, 1)
        p.overlap = self._pad3(self.overlap, 0)
        p.level = self.level
        p.top_k = self.top_k
        p.n_real = self.n_real
        p.n_facies = self.n_facies
        p.seed = self.seed
        p.path_mode = self.path_mode
        p.score_mode = self.score_mode
        m = list(self.nc_margin)[: self.ndim] + [-1] * (3 - self.ndim)
        p.nc_margin = (ctypes.c_int32 * 3)(*m)
        p.cut = self.cut
        p.wavelet = self.wavelet
        return p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(status: int, what: str):
    if status != 0:
        raise RuntimeError(f"oracle {what} failed with status {status}")


def rng(seed: int, stream: int, a: int, b: int) -> int:
    return int(lib().orc_rng(seed, stream, a, b))


def splitmix_first(x: int) -> int:
    return int(lib().orc_splitmix_first(x))


def perm20(x: int, key: int) -> int:
    return int(lib().orc_perm20(x, key))


def _n3(shape_xyz):
    n = list(shape_xyz) + [1] * (3 - len(shape_xyz))
    return np.array(n, dtype=np.int32)


def dwt(ti: np.ndarray, level: int):
    """Integer Haar DWT of a 2D [y][x] or 3D [z][y][x] int8 image.

    Returns (approx, details): approx has the level-J grid shape (numpy
    order), details is a list over j = 1..J of arrays shaped
    (2^d - 1, *grid_j) in numpy order."""
    ti = np.ascontiguousarray(ti, dtype=np.int8)
    ndim = ti.ndim
    n = _n3(ti.shape[::-1])
    b = [2 ** level if a < ndim else 1 for a in range(3)]
    np_ = [((int(n[a]) + b[a] - 1) // b[a]) * b[a] for a in range(3)]
    G = [np_[a] // b[a] for a in range(3)]
    approx = np.zeros(G[2] * G[1] * G[0], dtype=np.int64)
    ndet = int(lib().orc_details_count(_ptr(n), ndim, level))
    det = np.zeros(max(ndet, 1), dtype=np.int64)
    _check(lib().orc_dwt(_ptr(ti), _ptr(n), ndim, level, _ptr(approx), _ptr(det)), "dwt")
    shp = tuple(G[:ndim][::-1])
    details = []
    off = 0
    nsub = 2 ** ndim - 1
    for j in range(1, level + 1):
        gj = [np_[a] >> j if a < ndim else 1 for a in range(3)]
        cells = gj[0] * gj[1] * gj[2]
        details.append(det[off: off + nsub * cells].reshape((nsub,) + tuple(gj[:ndim][::-1])))
        off += nsub * cells
    return approx.reshape(shp), details


def details_flat(details) -> np.ndarray:
    if not details:
        return np.zeros(1, dtype=np.int64)
    return np.ascontiguousarray(np.concatenate([d.ravel() for d in details]), dtype=np.int64)


def idwt_region(approx: np.ndarray, details, ti_shape_xyz, level: int, c0, nc) -> np.ndarray:
    """Inverse Haar DWT of the level-J block range [c0, c0+nc) (x, y[, z])."""
    ndim = approx.ndim
    n = _n3(ti_shape_xyz)
    a = np.ascontiguousarray(approx, dtype=np.int64).ravel()
    d = details_flat(details)
    c0a = _n3(list(c0))
    c0a[ndim:] = 0
    nca = _n3(list(nc))
    b = 2 ** level
    ext = [int(nca[k]) * (b if k < ndim else 1) for k in range(3)]
    out = np.zeros(ext[0] * ext[1] * ext[2], dtype=np.int64)
    _check(lib().orc_idwt_region(_ptr(a), _ptr(d), _ptr(n), ndim, level, _ptr(c0a), _ptr(nca),
                                 _ptr(out)), "idwt_region")
    return out.reshape(tuple(ext[:ndim][::-1]))


def scores(K: np.ndarray, cand_xyz, nb: np.ndarray, mb: np.ndarray, beta_cells: int,
           mode: int = 0) -> np.ndarray:
    """S for every candidate; K, nb, mb in numpy order (z, y, x)."""
    K = np.ascontiguousarray(K, dtype=np.int64)
    nb = np.ascontiguousarray(nb, dtype=np.int64)
    mb = np.ascontiguousarray(mb, dtype=np.int64)
    G = _n3(K.shape[::-1])
    tc = _n3(nb.shape[::-1])
    cand = _n3(list(cand_xyz))
    S = np.zeros(int(np.prod(cand)), dtype=np.int64)
    _check(lib().orc_scores(_ptr(K), _ptr(G), _ptr(cand), _ptr(tc), beta_cells, _ptr(nb), _ptr(mb),
                            mode, _ptr(S)), "scores")
    return S.reshape(tuple(int(c) for c in cand[: K.ndim][::-1]))


def select(S: np.ndarray, mis, k: int, seed: int, r: int, step: int):
    """K best keys and the drawn candidate.  Returns (chosen, keys[K'])."""
    S = np.ascontiguousarray(S, dtype=np.int64).ravel()
    m = None if mis is None else np.ascontiguousarray(mis, dtype=np.int64).ravel()
    n = S.size
    kk = min(k, n)
    keys = np.zeros(kk, dtype=np.uint64)
    chosen = ctypes.c_int64()
    _check(lib().orc_select(_ptr(S), _ptr(m) if m is not None else None, n, k, seed, r, step,
                            ctypes.byref(chosen), _ptr(keys)), "select")
    return int(chosen.value), keys


def mincut(e: np.ndarray) -> np.ndarray:
    e = np.ascontiguousarray(e, dtype=np.int64)
    rows, cols = e.shape
    seam = np.zeros(rows, dtype=np.int32)
    _check(lib().orc_mincut(_ptr(e), rows, cols, _ptr(seam)), "mincut")
    return seam


def geometry(p: SimParams) -> dict:
    op = p.to_oracle()
    out = np.zeros(32, dtype=np.int64)
    _check(lib().orc_geometry(ctypes.byref(op), _ptr(out)), "geometry")
    return {
        "G": tuple(out[0:3]), "cand": tuple(out[3:6]), "tc": tuple(out[6:9]),
        "lattice": tuple(out[9:12]), "padded": tuple(out[12:15]), "b": tuple(out[15:18]),
        "ncand": int(out[18]), "beta_cells": int(out[19]),
        "nsteps": int(out[9] * out[10] * out[11]),
    }


def simulate(p: SimParams, ti: np.ndarray, hd=None, want_scores: bool = False):
    """Run Algorithm 1 for every realization.  ``hd`` is (real, pos, val) with
    pos an (n, ndim) array of (x, y[, z]) grid coordinates, or None.

    Returns (out, chosen[, scores]); out has shape (n_real, *grid) in numpy
    order, chosen is (n_real, n_steps)."""
    ti = np.ascontiguousarray(ti, dtype=np.int8)
    geo = geometry(p)
    op = p.to_oracle()
    if hd is None or len(hd[0]) == 0:
        n_hd = 0
        real = np.zeros(1, np.int32)
        pos = np.zeros(3, np.int32)
        val = np.zeros(1, np.int8)
    else:
        real = np.ascontiguousarray(hd[0], dtype=np.int32)
        n_hd = len(real)
        pos3 = np.zeros((n_hd, 3), dtype=np.int32)
        pos3[:, : p.ndim] = np.asarray(hd[1], dtype=np.int32)
        pos = np.ascontiguousarray(pos3.ravel())
        val = np.ascontiguousarray(hd[2], dtype=np.int8)
    grid = list(p.grid)
    cells = int(np.prod(grid))
    out = np.zeros(p.n_real * cells, dtype=np.int8)
    chosen = np.zeros(p.n_real * geo["nsteps"], dtype=np.int32)
    sc = np.zeros(p.n_real * geo["nsteps"] * geo["ncand"], dtype=np.int64) if want_scores else None
    st = lib().orc_simulate(ctypes.byref(op), _ptr(ti), n_hd, _ptr(real), _ptr(pos), _ptr(val),
                            _ptr(out), _ptr(chosen), _ptr(sc) if sc is not None else None)
    _check(st, "simulate")
    res = (out.reshape((p.n_real,) + tuple(grid[::-1])), chosen.reshape(p.n_real, geo["nsteps"]))
    if want_scores:
        res = res + (sc.reshape(p.n_real, geo["nsteps"], geo["ncand"]),)
    return res


def lift53_forward(x: np.ndarray):
    """One LeGall 5/3 integer lifting level of an even-length line:
    (approximation, detail), int64."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    n = x.shape[0]
    s = np.zeros(n // 2, dtype=np.int64)
    d = np.zeros(n // 2, dtype=np.int64)
    _check(lib().orc_lift53_forward(_ptr(x), n, _ptr(s), _ptr(d)), "orc_lift53_forward")
    return s, d


def lift53_inverse(s: np.ndarray, d: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int64)
    d = np.ascontiguousarray(d, dtype=np.int64)
    x = np.zeros(2 * s.shape[0], dtype=np.int64)
    _check(lib().orc_lift53_inverse(_ptr(s), _ptr(d), x.shape[0], _ptr(x)), "orc_lift53_inverse")
    return x


def approx53(img: np.ndarray, level: int) -> np.ndarray:
    """Level-J 5/3 approximation of an image in numpy order ([y][x] or
    [z][y][x]); every extent a multiple of 2^J."""
    img = np.ascontiguousarray(img, dtype=np.int64)
    ext = _n3(img.shape[::-1])
    out = np.zeros(tuple(n >> level for n in img.shape), dtype=np.int64)
    e = (ctypes.c_int64 * 3)(*[int(v) for v in ext])
    _check(lib().orc_approx53(_ptr(img), e, img.ndim, level, _ptr(out)), "orc_approx53")
    return out


def _pad_edge(ti: np.ndarray, level: int) -> np.ndarray:
    """The image extended by edge replication to a multiple of 2^J per axis."""
    b = 2 ** level
    pad = [(0, (-n) % b) for n in ti.shape]
    return np.pad(np.asarray(ti, dtype=np.int64), pad, mode="edge")


def _lines(arr: np.ndarray, axis: int, fn):
    """Apply a 1D routine to every line of arr along numpy axis `axis`."""
    a = np.moveaxis(arr, axis, -1)
    flat = a.reshape(-1, a.shape[-1])
    outs = [fn(flat[i]) for i in range(flat.shape[0])]
    return outs, a.shape[:-1]


def dwt53(ti: np.ndarray, level: int):
    """Level-J LeGall 5/3 integer DWT of an image in numpy order, extended by
    edge replication to a multiple of 2^J per axis (Sec. 4.2 makes the mother
    wavelet a choice; the lifting steps are those of lift53_forward).  Per
    level the lifting runs along x, then y, then z; sub-band q of level j has
    bit a set when axis a took the high-pass.  Returns (approx, details) in
    the layout of dwt(): details[j-1] is (2^d - 1, *grid_j)."""
    cur = _pad_edge(ti, level)
    nd = cur.ndim
    details = []
    for _ in range(level):
        bands = {0: cur}
        for a in range(nd):            # x, y, z
            ax = nd - 1 - a            # numpy axis of x is the last
            nxt = {}
            for q, arr in bands.items():
                outs, lead = _lines(arr, ax, lift53_forward)
                lo = np.stack([o[0] for o in outs]).reshape(lead + (-1,))
                hi = np.stack([o[1] for o in outs]).reshape(lead + (-1,))
                nxt[q] = np.moveaxis(lo, -1, ax)
                nxt[q | (1 << a)] = np.moveaxis(hi, -1, ax)
            bands = nxt
        cur = bands[0]
        details.append(np.stack([bands[q] for q in range(1, 2 ** nd)]))
    return cur, details


def idwt53(approx: np.ndarray, details) -> np.ndarray:
    """Inverse of dwt53: the padded image, exactly (perfect reconstruction
    of the integer lifting, lift53_inverse line by line)."""
    cur = np.asarray(approx, dtype=np.int64)
    nd = cur.ndim
    for det in reversed(details):
        bands = {0: cur}
        for q in range(1, 2 ** nd):
            bands[q] = np.asarray(det[q - 1], dtype=np.int64)
        for a in reversed(range(nd)):  # z, y, x
            ax = nd - 1 - a
            nxt = {}
            for q in [q for q in bands if not (q >> a) & 1]:
                lo, hi = bands[q], bands[q | (1 << a)]
                L = np.moveaxis(lo, ax, -1)
                H = np.moveaxis(hi, ax, -1)
                fl, fh = L.reshape(-1, L.shape[-1]), H.reshape(-1, H.shape[-1])
                rec = np.stack([lift53_inverse(fl[i], fh[i]) for i in range(fl.shape[0])])
                nxt[q] = np.moveaxis(rec.reshape(L.shape[:-1] + (-1,)), -1, ax)
            bands = nxt
        cur = bands[0]
    return cur

"""Float64 oracle of the CDF 9/7 wavelet path: the transform, its inverse and
the candidate scores over the level-J approximation.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  Plain
numpy in float64, no blocking or fusion.

Sec. 4.2 makes the Haar wavelet one choice of mother wavelet; this module
takes another one, the Cohen-Daubechies-Feauveau 9/7 biorthogonal wavelet,
in the lifting factorisation of Daubechies and Sweldens (1998): two
predict/update pairs with the constants ALPHA..DELTA, then a scaling of the
low band by ZETA and of the high band by 1/ZETA.  With this scaling the
low-pass has gain sqrt(2) at DC, the near-orthonormal convention.  Lines
have even length and whole-sample symmetric extension (x[-i] = x[i],
x[n-1+i] = x[n-1-i]), under which the lifting equals the 9/7 filter bank
applied to the mirrored signal.  Per level the lines run along x, then y,
then z, as for the other wavelets; the image is first extended by edge
replication to a multiple of 2^J per axis.

Scores (Sec. 4.3, the CCW score over the approximation, with the reading
that a block enters when it holds a known cell): for a data event given as
a known-block mask n (0/1) and the event's own level-J approximation A,
candidate c scores S(c) = sum over template blocks b of n_b (K[c + b] -
A_b)^2, the squared coefficient distance over the known blocks; the best
candidates have the smallest S.

Parity pins (tests/test_oracle_cdf97.py): perfect reconstruction, the
closed form for constants, vanishing interior details of cubics, the
published 9/7 analysis filter taps (tests/golden/cdf97_taps.txt) on
interior impulses and on explicitly mirrored signals, and the scores against
a sliding-window computation and brute force.
"""
from __future__ import annotations

import numpy as np

# lifting constants of the CDF 9/7 factorisation (Daubechies and Sweldens)
ALPHA = -1.586134342059924
BETA = -0.052980118572961
GAMMA = 0.882911075530934
DELTA = 0.443506852043971
ZETA = 1.149604398860241


def lift97_forward(x: np.ndarray):
    """One analysis level of an even-length line: (low, high), float64."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n % 2 or n < 2:
        raise ValueError("line length must be even and >= 2")
    s = x[0::2].copy()
    d = x[1::2].copy()

    def right(v):   # v[k + 1], mirrored past the end: s[n/2] = s[n/2 - 1]
        return np.append(v[1:], v[-1])

    def left(v):    # v[k - 1], mirrored before the start: d[-1] = d[0]
        return np.insert(v[:-1], 0, v[0])

    d = d + ALPHA * (s + right(s))
    s = s + BETA * (left(d) + d)
    d = d + GAMMA * (s + right(s))
    s = s + DELTA * (left(d) + d)
    return s * ZETA, d / ZETA


def lift97_inverse(s: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Synthesis: the steps of lift97_forward undone in reverse order."""
    s = np.asarray(s, dtype=np.float64) / ZETA
    d = np.asarray(d, dtype=np.float64) * ZETA

    def right(v):
        return np.append(v[1:], v[-1])

    def left(v):
        return np.insert(v[:-1], 0, v[0])

    s = s - DELTA * (left(d) + d)
    d = d - GAMMA * (s + right(s))
    s = s - BETA * (left(d) + d)
    d = d - ALPHA * (s + right(s))
    x = np.empty(2 * s.shape[0], dtype=np.float64)
    x[0::2] = s
    x[1::2] = d
    return x


def pad_edge(img: np.ndarray, level: int) -> np.ndarray:
    """The image extended by edge replication to a multiple of 2^J per axis."""
    b = 2 ** level
    pad = [(0, (-n) % b) for n in img.shape]
    return np.pad(np.asarray(img, dtype=np.float64), pad, mode="edge")


def _along(arr: np.ndarray, axis: int, fn):
    """fn applied to every line of arr along numpy axis `axis`."""
    a = np.moveaxis(arr, axis, -1)
    flat = a.reshape(-1, a.shape[-1])
    outs = [fn(flat[i]) for i in range(flat.shape[0])]
    return outs, a.shape[:-1]


def dwt97(img: np.ndarray, level: int):
    """Level-J CDF 9/7 DWT of an image in numpy order ([y][x] or [z][y][x]).
    Returns (approx, details): details[j-1] is (2^d - 1, *grid_j) with
    sub-band q having bit a set when axis a (x = 0) took the high-pass."""
    cur = pad_edge(img, level)
    nd = cur.ndim
    details = []
    for _ in range(level):
        bands = {0: cur}
        for a in range(nd):
            ax = nd - 1 - a            # numpy axis of x is the last
            nxt = {}
            for q, arr in bands.items():
                outs, lead = _along(arr, ax, lift97_forward)
                lo = np.stack([o[0] for o in outs]).reshape(lead + (-1,))
                hi = np.stack([o[1] for o in outs]).reshape(lead + (-1,))
                nxt[q] = np.moveaxis(lo, -1, ax)
                nxt[q | (1 << a)] = np.moveaxis(hi, -1, ax)
            bands = nxt
        cur = bands[0]
        details.append(np.stack([bands[q] for q in range(1, 2 ** nd)]))
    return cur, details


def idwt97(approx: np.ndarray, details) -> np.ndarray:
    """Inverse of dwt97: the edge-replicated image (float64)."""
    cur = np.asarray(approx, dtype=np.float64)
    nd = cur.ndim
    for det in reversed(details):
        bands = {0: cur}
        for q in range(1, 2 ** nd):
            bands[q] = np.asarray(det[q - 1], dtype=np.float64)
        for a in reversed(range(nd)):
            ax = nd - 1 - a
            nxt = {}
            for q in [q for q in bands if not (q >> a) & 1]:
                L = np.moveaxis(bands[q], ax, -1)
                H = np.moveaxis(bands[q | (1 << a)], ax, -1)
                fl, fh = L.reshape(-1, L.shape[-1]), H.reshape(-1, H.shape[-1])
                rec = np.stack([lift97_inverse(fl[i], fh[i]) for i in range(fl.shape[0])])
                nxt[q] = np.moveaxis(rec.reshape(L.shape[:-1] + (-1,)), -1, ax)
            bands = nxt
        cur = bands[0]
    return cur


def scores97(K: np.ndarray, cand, n: np.ndarray, A: np.ndarray) -> np.ndarray:
    """S for every candidate c (numpy order): sum over template blocks b with
    n_b = 1 of (K[c + b] - A_b)^2.  K is the level-J grid, n and A have the
    template's block extent, cand the candidate counts per numpy axis."""
    K = np.asarray(K, dtype=np.float64)
    n = np.asarray(n)
    A = np.asarray(A, dtype=np.float64)
    cand = tuple(int(c) for c in cand)
    S = np.zeros(cand, dtype=np.float64)
    for b in zip(*np.nonzero(n)):
        win = K[tuple(slice(b[i], b[i] + cand[i]) for i in range(K.ndim))]
        S += (win - A[b]) ** 2
    return S


def topk97(S: np.ndarray, k: int) -> np.ndarray:
    """Flat indices of the k smallest scores, ties to the smaller index."""
    flat = np.asarray(S, dtype=np.float64).ravel()
    return np.argsort(flat, kind="stable")[:k]

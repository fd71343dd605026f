"""Realization statistics, written out from their definitions in numpy.

TEST INFRASTRUCTURE ONLY: imported by the tests and by the benchmark's
CPU-baseline leg, never by the product path.

The paper validates realizations against the training image with facies
proportions (Sec. 5.8, Fig. 16b), the ensemble average map (Sec. 5.2,
Fig. 7b), variograms along the two cardinal axes and the probability of
connection along the channels' direction (Sec. 5.3, Fig. 9).  It does not
write these out; the readings taken here are the textbook ones for
categorical images:

* proportion of facies f in image i: the number of cells holding code f;
* ensemble map: for each facies and cell, the number of images holding f
  there (divide by the number of images for the probability map);
* indicator variogram along axis a at lag h (cells): with I = [code == f]
  and the N_a(h) cell pairs (x, x + h e_a) inside the image,
  gamma_f(h) = (1 / (2 N_a(h))) * sum (I(x) - I(x + h e_a))^2, i.e. half the
  fraction of pairs whose indicators differ.  For a two-facies image this is
  also the variogram of the codes;
* probability of connection along axis a at lag h: among the pairs whose
  cells both hold f, the fraction whose cells lie in the same connected
  component of f, cells being connected through shared faces (4 neighbours
  in 2D, 6 in 3D).

Every function returns the integer counts these ratios are made of.  Images
are numpy arrays indexed [image][z][y][x] (or [image][y][x]); axis a counts
the (x, y, z) axes, so a = 0 is x (east-west) and a = 1 is y (north-south).
Codes outside 0 .. n_facies-1 belong to no facies.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def _as_stack(imgs: np.ndarray) -> np.ndarray:
    imgs = np.asarray(imgs)
    if imgs.ndim not in (3, 4):
        raise ValueError("images are [image][y][x] or [image][z][y][x]")
    return imgs


def _np_axis(imgs: np.ndarray, axis: int) -> int:
    """numpy axis of image axis `axis` (0 = x) in an [image][..][y][x] stack."""
    return imgs.ndim - 1 - axis


def histogram(imgs: np.ndarray, n_facies: int):
    """per_image[i][f] = cells of image i holding f; per_cell[f][...] = images
    holding f at that cell (Fig. 16b proportions, Fig. 7b ensemble map)."""
    imgs = _as_stack(imgs)
    per_image = np.zeros((imgs.shape[0], n_facies), dtype=np.int64)
    per_cell = np.zeros((n_facies,) + imgs.shape[1:], dtype=np.int64)
    for f in range(n_facies):
        ind = imgs == f
        per_image[:, f] = ind.reshape(imgs.shape[0], -1).sum(axis=1)
        per_cell[f] = ind.sum(axis=0)
    return per_image, per_cell


def pair_count(shape_img, axis: int, h: int) -> int:
    """N_a(h): cell pairs (x, x + h e_a) inside an image of numpy shape
    shape_img ([z][y][x] or [y][x])."""
    n = list(shape_img)
    k = len(n) - 1 - axis
    n[k] = max(0, n[k] - h)
    return int(np.prod(n))


def _pairs(a: np.ndarray, k: int, h: int):
    """The two ends of every pair at lag h along numpy axis k of a."""
    n = a.shape[k]
    lo = np.take(a, np.arange(0, n - h), axis=k)
    hi = np.take(a, np.arange(h, n), axis=k)
    return lo, hi


def variogram(imgs: np.ndarray, n_facies: int, axis: int, max_lag: int) -> np.ndarray:
    """diff[i][f][h-1] = pairs at lag h along `axis` whose indicators of f
    differ (Sec. 5.3, Fig. 9a); gamma_f(h) = diff / (2 N_a(h))."""
    imgs = _as_stack(imgs)
    out = np.zeros((imgs.shape[0], n_facies, max_lag), dtype=np.int64)
    for i in range(imgs.shape[0]):
        img = imgs[i]
        k = img.ndim - 1 - axis
        for f in range(n_facies):
            ind = img == f
            for h in range(1, max_lag + 1):
                lo, hi = _pairs(ind, k, h)
                out[i, f, h - 1] = int(np.count_nonzero(lo != hi))
    return out


def components(mask: np.ndarray) -> np.ndarray:
    """Connected components of the True cells of a 2D or 3D mask, cells
    joined through shared faces; labels 0, 1, .. in order of first cell in
    memory order, -1 outside the mask.  Breadth-first flood fill."""
    lab = np.full(mask.shape, -1, dtype=np.int64)
    flat = mask.reshape(-1)
    lflat = lab.reshape(-1)
    dims = mask.shape
    strides = [int(np.prod(dims[d + 1:])) for d in range(len(dims))]
    nxt = 0
    for start in range(flat.size):
        if not flat[start] or lflat[start] >= 0:
            continue
        lflat[start] = nxt
        q = deque([start])
        while q:
            c = q.popleft()
            rem = c
            coord = []
            for d in range(len(dims)):
                coord.append(rem // strides[d])
                rem -= coord[-1] * strides[d]
            for d in range(len(dims)):
                for step in (-1, 1):
                    v = coord[d] + step
                    if 0 <= v < dims[d]:
                        nb = c + step * strides[d]
                        if flat[nb] and lflat[nb] < 0:
                            lflat[nb] = nxt
                            q.append(nb)
        nxt += 1
    return lab


def connectivity(imgs: np.ndarray, n_facies: int, axis: int, max_lag: int):
    """both[i][f][h-1] = pairs at lag h along `axis` with both cells in f;
    connected[i][f][h-1] = those whose cells share a component of f
    (Sec. 5.3, Fig. 9b); the probability of connection is their ratio."""
    imgs = _as_stack(imgs)
    both = np.zeros((imgs.shape[0], n_facies, max_lag), dtype=np.int64)
    conn = np.zeros_like(both)
    for i in range(imgs.shape[0]):
        img = imgs[i]
        k = img.ndim - 1 - axis
        for f in range(n_facies):
            lab = components(img == f)
            for h in range(1, max_lag + 1):
                lo, hi = _pairs(lab, k, h)
                inb = (lo >= 0) & (hi >= 0)
                both[i, f, h - 1] = int(np.count_nonzero(inb))
                conn[i, f, h - 1] = int(np.count_nonzero(inb & (lo == hi)))
    return both, conn

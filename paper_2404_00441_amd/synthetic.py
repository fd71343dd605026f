"""Seeded synthetic inputs: channelised training images and hard data.

This module holds no arithmetic of the simulation method.  It only draws
stand-ins for the paper's training images (the Channel, Stonewall, Ganges and
multi-facies images of Sec. 5, which are not available): sinuous channels over
a background, optionally with levee rims (3 facies), in 2D, and elliptic
sinuous tubes in 3D.  Hard data are point samples of a reference image drawn
by the same generator (Sec. 5.2 takes conditioning data as random samples of a
reference image so that histogram and variogram match the TI).

Arrays are numpy, numpy axis order ([y][x] in 2D, [z][y][x] in 3D), codes int8.
All draws come from ``numpy.random.default_rng(seed)`` in a fixed order.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["channel_image_2d", "tube_image_3d", "sample_hard_data"]


def _channel_draws(rng, n_channels, ny):
    """Per channel: azimuth, wavelength, amplitude, width, offset, phase."""
    out = []
    for _ in range(n_channels):
        theta = math.radians(rng.uniform(-20.0, 20.0))
        lam = rng.uniform(40.0, 120.0)
        amp = rng.uniform(5.0, 20.0)
        width = rng.uniform(4.0, 10.0)
        off = rng.uniform(0.0, float(ny))
        phase = rng.uniform(0.0, 2.0 * math.pi)
        out.append((theta, lam, amp, width, off, phase))
    return out


def channel_image_2d(nx: int, ny: int, n_channels: int, n_facies: int, seed: int) -> np.ndarray:
    """Binary (n_facies=2: background 0, channel 1) or 3-facies (levee rim 2 of
    width 2 cells around each channel) image of sinusoidal channels.

    A cell centre is rotated about the image centre by the channel azimuth to
    (u, v); the channel centreline is v_c = (off - ny/2) + amp*sin(2*pi*u/lam +
    phase); the cell is channel if |v - v_c| <= width/2.  Channel wins over
    levee wherever two channels meet."""
    if n_facies not in (2, 3):
        raise ValueError("n_facies must be 2 or 3")
    rng = np.random.default_rng(seed)
    ys, xs = np.meshgrid(np.arange(ny, dtype=np.float64) + 0.5,
                         np.arange(nx, dtype=np.float64) + 0.5, indexing="ij")
    cx, cy = nx / 2.0, ny / 2.0
    chan = np.zeros((ny, nx), dtype=bool)
    levee = np.zeros((ny, nx), dtype=bool)
    for theta, lam, amp, width, off, phase in _channel_draws(rng, n_channels, ny):
        c, s = math.cos(theta), math.sin(theta)
        u = (xs - cx) * c + (ys - cy) * s
        v = -(xs - cx) * s + (ys - cy) * c
        vc = (off - cy) + amp * np.sin(2.0 * math.pi * u / lam + phase)
        d = np.abs(v - vc)
        chan |= d <= width / 2.0
        if n_facies == 3:
            levee |= (d > width / 2.0) & (d <= width / 2.0 + 2.0)
    img = np.zeros((ny, nx), dtype=np.int8)
    if n_facies == 3:
        img[levee] = 2
    img[chan] = 1
    return img


def tube_image_3d(nx: int, ny: int, nz: int, n_tubes: int, seed: int) -> np.ndarray:
    """Binary 3D image of sinuous tubes with elliptic cross-section.

    The xy centreline is drawn as in ``channel_image_2d`` (azimuth, wavelength,
    amplitude, offset, phase); each tube also draws a width W in [6, 14], a
    thickness H in [2, 5] and a depth z0 in [0, nz).  A cell is channel if
    (dv / (W/2))^2 + (dz / (H/2))^2 <= 1."""
    rng = np.random.default_rng(seed)
    zs, ys, xs = np.meshgrid(np.arange(nz, dtype=np.float64) + 0.5,
                             np.arange(ny, dtype=np.float64) + 0.5,
                             np.arange(nx, dtype=np.float64) + 0.5, indexing="ij")
    cx, cy = nx / 2.0, ny / 2.0
    chan = np.zeros((nz, ny, nx), dtype=bool)
    for _ in range(n_tubes):
        theta = math.radians(rng.uniform(-20.0, 20.0))
        lam = rng.uniform(40.0, 120.0)
        amp = rng.uniform(5.0, 20.0)
        off = rng.uniform(0.0, float(ny))
        phase = rng.uniform(0.0, 2.0 * math.pi)
        W = rng.uniform(6.0, 14.0)
        H = rng.uniform(2.0, 5.0)
        z0 = rng.uniform(0.0, float(nz))
        c, s = math.cos(theta), math.sin(theta)
        u = (xs - cx) * c + (ys - cy) * s
        v = -(xs - cx) * s + (ys - cy) * c
        vc = (off - cy) + amp * np.sin(2.0 * math.pi * u / lam + phase)
        chan |= ((v - vc) / (W / 2.0)) ** 2 + ((zs - z0) / (H / 2.0)) ** 2 <= 1.0
    return chan.astype(np.int8)


def sample_hard_data(reference: np.ndarray, counts, seed: int):
    """Draw hard data for several realizations from one reference image.

    ``counts[r]`` distinct cells are drawn without replacement for
    realization r (positions differ between realizations); the value of each
    datum is the reference code there.  Returns (real, pos, val): real int32
    (n,), pos int32 (n, ndim) as (x, y[, z]) grid coordinates, val int8 (n,)."""
    rng = np.random.default_rng(seed)
    ref = np.asarray(reference)
    ncell = ref.size
    reals, poss, vals = [], [], []
    for r, cnt in enumerate(counts):
        cnt = int(cnt)
        if cnt == 0:
            continue
        flat = rng.choice(ncell, size=cnt, replace=False)
        idx = np.stack(np.unravel_index(flat, ref.shape), axis=1)  # numpy order
        poss.append(idx[:, ::-1].astype(np.int32))                  # -> (x, y[, z])
        vals.append(ref.ravel()[flat].astype(np.int8))
        reals.append(np.full(cnt, r, dtype=np.int32))
    if not reals:
        return (np.zeros(0, np.int32), np.zeros((0, ref.ndim), np.int32), np.zeros(0, np.int8))
    return np.concatenate(reals), np.concatenate(poss), np.concatenate(vals)

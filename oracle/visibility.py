"""Visibility culling (Sec. 4.3, visibility-culling paragraph and Fig. 5b).
Test infrastructure only.

The headset's visibility mask (per pixel) becomes a bitfield with one bit per
tile -- set when any pixel of the tile is visible -- and a summed-area table
of that bitfield.  The number of visible tiles in the rectangle of tiles a
splat covers is then read from the table at the rectangle's corners, which
gives the exact number of Gaussian/tile instances to allocate; instances in
invisible tiles are never created.

Reading: invisible tiles get no instances, so their pixels keep the
background (transmittance 1); the foveated periphery blur reads them as
such.  A tile is visible or not as a whole (a visible tile renders all of
its pixels).
"""
import numpy as np


def tile_bits(mask, T):
    """(nty, ntx) bool: tile (ty, tx) of size T holds a visible pixel."""
    H, W = mask.shape
    nty, ntx = -(-H // T), -(-W // T)
    pad = np.zeros((nty * T, ntx * T), bool)
    pad[:H, :W] = np.asarray(mask) != 0
    return pad.reshape(nty, T, ntx, T).any(axis=(1, 3))


def summed_area(bits):
    """S (nty+1, ntx+1) with S[y][x] = number of set bits in rows < y and
    columns < x."""
    b = np.asarray(bits, np.int64)
    S = np.zeros((b.shape[0] + 1, b.shape[1] + 1), np.int64)
    S[1:, 1:] = b.cumsum(axis=0).cumsum(axis=1)
    return S


def rect_count(S, tx0, tx1, ty0, ty1):
    """Set bits in the inclusive tile rectangle [tx0, tx1] x [ty0, ty1] from
    the table's four corners (0 for an empty rectangle)."""
    tx0, tx1, ty0, ty1 = (np.asarray(a, np.int64) for a in (tx0, tx1, ty0, ty1))
    empty = (tx1 < tx0) | (ty1 < ty0)
    x0 = np.where(empty, 0, tx0)
    x1 = np.where(empty, 0, tx1 + 1)
    y0 = np.where(empty, 0, ty0)
    y1 = np.where(empty, 0, ty1 + 1)
    return np.where(empty, 0, S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0])

"""Location orderings (paper Section 3).

Readings of points the paper leaves open (each is a documented choice):

* Encoding (Section 3.1, the enumerated "Encoding" step): each coordinate in
  [0, 1] is multiplied by the largest 16-bit unsigned value, 65535, and rounded
  to the nearest integer, ties to even; the result is clamped to [0, 65535].
  The paper's "single-precision (16 bits)" is read as 16 bits per coordinate.
* Morton (Section 3.1.1): bit b of the x code becomes key bit 2b, bit b of the
  y code becomes key bit 2b+1 (32-bit key).
* Hilbert (Section 3.1.2, Hilbert figure): the curve whose order-1 visit is
  (0,0) -> (0,1) -> (1,1) -> (1,0), x horizontal, refined by the usual
  quadrant recursion with rotations; order 16 over the 16-bit codes.
* Sorting (the "Sorting" step): keys are sorted ascending; equal keys keep the
  original index order (sort by the pair (key, index)).
* Decoding (the "Decoding" step): optional.  By default the ordered locations
  are the original float64 coordinates gathered by the permutation; with
  ``dequantize=True`` they are code / 65535 as the paper describes.
* KD-tree (Section 3.2): split dimension = the one with the larger range
  (max - min), x on a tie; the node's points sorted by (coordinate, index);
  the first ceil(m/2) go left.  This equals "value <= median goes left" when
  values are distinct.  Leaves are single points; in-order traversal visits
  the leaves left to right.  Comparisons use the unquantised coordinates.
* Random: key_i = the (i+1)-th output of SplitMix64 (Steele, Lea, Flood 2014)
  started from ``seed``; sorted like the curve keys.
* None: the identity (generation order, the paper's "No Order").
"""
from __future__ import annotations

import numpy as np

QMAX = 65535
KINDS = ("none", "random", "morton", "hilbert", "kdtree")


def quantize(locs: np.ndarray) -> np.ndarray:
    """Encoding step: n x 2 float64 in [0,1] -> n x 2 uint32 codes in [0, 65535]."""
    locs = np.asarray(locs, dtype=np.float64)
    if not np.all(np.isfinite(locs)) or locs.min() < 0.0 or locs.max() > 1.0:
        raise ValueError("locations must be finite and lie in [0, 1]^2")
    q = np.rint(locs * float(QMAX))  # round half to even
    return np.clip(q, 0, QMAX).astype(np.uint32)


def dequantize(q: np.ndarray) -> np.ndarray:
    """Decoding step: integer codes back to the unit square."""
    return np.asarray(q, dtype=np.float64) / float(QMAX)


def morton_key(qx, qy, bits: int = 16) -> np.ndarray:
    """Interleave the bits: x bit b -> key bit 2b, y bit b -> key bit 2b+1."""
    qx = np.asarray(qx, dtype=np.uint64)
    qy = np.asarray(qy, dtype=np.uint64)
    key = np.zeros(qx.shape, dtype=np.uint64)
    for b in range(bits):
        key |= ((qx >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((qy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def hilbert_key_scalar(x: int, y: int, order: int) -> int:
    """Position of cell (x, y) on the order-``order`` Hilbert curve.

    Quadrant recursion: at each level the cell lies in one quadrant of the
    current square; the quadrants are visited in the order lower-left,
    upper-left, upper-right, lower-right (order-1 figure).  The sub-curve in
    the lower-left quadrant is the parent curve reflected in the diagonal
    (x <-> y); in the lower-right quadrant it is reflected in the anti-diagonal;
    the two upper quadrants are plain translates.
    """
    d = 0
    side = 1 << order
    half = side >> 1
    while half > 0:
        right = 1 if x >= half else 0
        upper = 1 if y >= half else 0
        if not right and not upper:
            quad = 0
        elif not right and upper:
            quad = 1
        elif right and upper:
            quad = 2
        else:
            quad = 3
        d += quad * half * half
        # local coordinates inside the quadrant
        lx = x - right * half
        ly = y - upper * half
        if quad == 0:          # reflect in the main diagonal
            lx, ly = ly, lx
        elif quad == 3:        # reflect in the anti-diagonal
            lx, ly = half - 1 - ly, half - 1 - lx
        x, y = lx, ly
        half >>= 1
    return d


def hilbert_key(qx, qy, order: int = 16) -> np.ndarray:
    qx = np.asarray(qx).astype(np.int64).ravel()
    qy = np.asarray(qy).astype(np.int64).ravel()
    out = np.empty(qx.size, dtype=np.uint64)
    for k in range(qx.size):
        out[k] = hilbert_key_scalar(int(qx[k]), int(qy[k]), order)
    return out


_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """First ``count`` outputs of SplitMix64 from state ``seed`` (Python ints)."""
    out = np.empty(count, dtype=np.uint64)
    state = int(seed) & _MASK
    for k in range(count):
        state = (state + _GAMMA) & _MASK
        z = state
        z = ((z ^ (z >> 30)) * _M1) & _MASK
        z = ((z ^ (z >> 27)) * _M2) & _MASK
        z = z ^ (z >> 31)
        out[k] = z
    return out


def sort_by_key(keys: np.ndarray) -> np.ndarray:
    """Sorting step: indices ordered by (key, original index)."""
    keys = np.asarray(keys)
    idx = np.arange(keys.size)
    return np.lexsort((idx, keys)).astype(np.int64)


def kdtree_order(locs: np.ndarray) -> np.ndarray:
    """KD-tree ordering: recursive median split, leaves read left to right."""
    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    out = []

    def build(members: np.ndarray):
        m = members.size
        if m == 1:
            out.append(int(members[0]))
            return
        pts = locs[members]
        range_x = pts[:, 0].max() - pts[:, 0].min()
        range_y = pts[:, 1].max() - pts[:, 1].min()
        dim = 1 if range_y > range_x else 0
        order = np.lexsort((members, pts[:, dim]))
        sorted_members = members[order]
        left = (m + 1) // 2
        build(sorted_members[:left])
        build(sorted_members[left:])

    if n > 0:
        build(np.arange(n, dtype=np.int64))
    return np.asarray(out, dtype=np.int64)


def reorder(locs: np.ndarray, kind: str, seed: int = 0) -> np.ndarray:
    """Permutation perm with perm[k] = original index of the k-th ordered point."""
    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    if kind == "none":
        return np.arange(n, dtype=np.int64)
    if kind == "random":
        return sort_by_key(splitmix64_stream(seed, n))
    if kind == "kdtree":
        if n and (not np.all(np.isfinite(locs)) or locs.min() < 0 or locs.max() > 1):
            raise ValueError("locations must be finite and lie in [0, 1]^2")
        return kdtree_order(locs)
    q = quantize(locs)
    if kind == "morton":
        return sort_by_key(morton_key(q[:, 0], q[:, 1]))
    if kind == "hilbert":
        return sort_by_key(hilbert_key(q[:, 0], q[:, 1], 16))
    raise ValueError(f"unknown ordering {kind!r}")


def ordered_locations(locs: np.ndarray, perm: np.ndarray, kind: str, dequantize_codes: bool = False) -> np.ndarray:
    """Locations in the new order; with dequantize_codes, the decoded codes."""
    locs = np.asarray(locs, dtype=np.float64)
    if dequantize_codes and kind in ("morton", "hilbert"):
        return dequantize(quantize(locs))[perm]
    return locs[perm]

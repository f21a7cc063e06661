"""Oracle of the regridding step: signature clustering of flagged cells into
boxes (Berger and Rigoutsos) and piecewise-constant injection into refined
patches.  TEST INFRASTRUCTURE ONLY (tests and benchmark baselines); the HIP
library has its own implementation.

Clustering, recursively from the whole grid:
  1. shrink the box to the bounding box of its flagged cells (none: drop it);
  2. keep it if n_flagged >= efficiency * area and both sides <= max_side;
  3. if efficient but too large: bisect the first side (x, then y) longer
     than max_side at len // 2;
  4. else cut at a hole of a signature (column sums for x, row sums for y),
     before the empty column/row c in [1, len-1]: the smallest |2c - len|,
     then x before y, then smaller c;
  5. else at the strongest inflection: Laplacian L[k] = S[k+1] - 2S[k] + S[k-1],
     cut c = k + 1 where L[k] * L[k+1] < 0 and min_side <= c <= len - min_side,
     strength |L[k+1] - L[k]|; strongest, then smallest |2c - len|, then x
     before y, then smaller c;
  6. else bisect the longer side (x when equal) at len // 2 if both halves
     keep min_side cells, else the other side; else keep the box.
The lower part comes before the upper part.
"""
import numpy as np


def cluster(flags, efficiency, min_side, max_side):
    """Boxes (i_lo, j_lo, nx, ny) covering the non-zero cells of flags (ny, nx)."""
    f = np.asarray(flags) != 0
    out = []
    _cluster(f, (0, 0, f.shape[1], f.shape[0]), float(efficiency), int(min_side), int(max_side), out)
    return out


def _cluster(f, box, eff, min_side, max_side, out):
    i, j, nx, ny = box
    sub = f[j:j + ny, i:i + nx]
    cols = np.nonzero(sub.any(axis=0))[0]
    if cols.size == 0:
        return
    rows = np.nonzero(sub.any(axis=1))[0]
    i, j = i + int(cols[0]), j + int(rows[0])
    nx, ny = int(cols[-1] - cols[0] + 1), int(rows[-1] - rows[0] + 1)
    sub = f[j:j + ny, i:i + nx]
    nflag = int(sub.sum())
    efficient = float(nflag) >= eff * float(nx * ny)
    if efficient and nx <= max_side and ny <= max_side:
        out.append((i, j, nx, ny))
        return
    if efficient:
        d = 0 if nx > max_side else 1
        c = (nx if d == 0 else ny) // 2
    else:
        cut = _choose(sub, min_side)
        if cut is None:
            out.append((i, j, nx, ny))
            return
        d, c = cut
    if d == 0:
        lo, hi = (i, j, c, ny), (i + c, j, nx - c, ny)
    else:
        lo, hi = (i, j, nx, c), (i, j + c, nx, ny - c)
    _cluster(f, lo, eff, min_side, max_side, out)
    _cluster(f, hi, eff, min_side, max_side, out)


def _choose(sub, min_side):
    sig = [sub.sum(axis=0).astype(np.int64), sub.sum(axis=1).astype(np.int64)]
    # holes
    best = None
    for d in (0, 1):
        n = len(sig[d])
        for c in range(1, n):
            if sig[d][c] == 0:
                key = (abs(2 * c - n), d, c)
                if best is None or key < best[0]:
                    best = (key, d, c)
    if best is not None:
        return best[1], best[2]
    # inflections
    for d in (0, 1):
        s = sig[d]
        n = len(s)
        for k in range(1, n - 2):
            lk = int(s[k + 1] - 2 * s[k] + s[k - 1])
            lk1 = int(s[k + 2] - 2 * s[k + 1] + s[k])
            if lk * lk1 >= 0:
                continue
            c = k + 1
            if c < min_side or n - c < min_side:
                continue
            key = (-abs(lk1 - lk), abs(2 * c - n), d, c)
            if best is None or key < best[0]:
                best = (key, d, c)
    if best is not None:
        return best[1], best[2]
    # bisection
    ny, nx = sub.shape
    first = 0 if nx >= ny else 1
    for d in (first, 1 - first):
        n = nx if d == 0 else ny
        c = n // 2
        if c >= min_side and n - c >= min_side:
            return d, c
    return None


def prolong(fields, boxes, ratio):
    """Piecewise-constant injection: for each box, the coarse fields repeated
    ratio x ratio.  fields: list of (ny, nx) arrays.  Returns, per box, the
    list of refined arrays."""
    out = []
    for (i, j, nx, ny) in boxes:
        out.append([np.repeat(np.repeat(np.asarray(a)[j:j + ny, i:i + nx], ratio, axis=0), ratio, axis=1)
                    for a in fields])
    return out

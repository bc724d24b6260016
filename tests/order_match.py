"""Slot-by-slot comparison of two cell-sorted particle lists that may differ by a few particles
sitting on a cell face.

Both the GPU library and the oracle keep every species stably sorted by cell.  When all
particles land in the same cells on both sides, the two orders are the stable sort of the
same previous order by the same keys, so they agree slot by slot.  A particle whose new
position lies within rounding of a face can land in the neighbouring cell on one side: it then
sits in a different place of each list, and everything between stays in order, one slot
apart.  ``align_sorted`` walks both lists, matching particles slot by slot (same cell, values
within the caller's tolerance), and steps over an unmatched particle on either side when the
next one matches; the caller then checks that every particle stepped over lies near a face.
"""
from __future__ import annotations

import numpy as np


def cell_keys(p, nx):
    return (np.floor(p["xi_z"]).astype(np.int64) * nx
            + np.floor(p["xi_x"]).astype(np.int64))


def near_face(p, idx, eps, nx):
    """Whether particles idx of p lie within eps of a cell face (x = 0 and x = nx included)."""
    x = p["xi_x"][idx]
    z = p["xi_z"][idx]
    fx = np.abs(x - np.round(x))
    fz = np.abs(z - np.round(z))
    return (fx <= eps) | (fz <= eps)


def align_sorted(g, o, nx, close, max_skips=10000):
    """Match the cell-sorted lists g and o (dicts of equal-length arrays with xi_x, xi_z, ...).

    ``close(ig, io)`` takes index arrays and returns a bool array: whether g[ig] and o[io] are
    the same particle up to the tolerance (the caller's value check).  Returns (jg, jo,
    extra_g, extra_o): matched index pairs in list order, and the indices left unmatched on
    each side."""
    kg, ko = cell_keys(g, nx), cell_keys(o, nx)
    ng, no = kg.size, ko.size
    seg_g, seg_o = [], []
    extra_g, extra_o = [], []
    i = j = 0

    def match(a, b):
        if a >= ng or b >= no:
            return False
        return bool(kg[a] == ko[b]) and bool(close(np.array([a]), np.array([b]))[0])

    chunk = 1 << 18
    while True:
        L = min(ng - i, no - j, chunk)
        if L > 0:
            ia = np.arange(i, i + L)
            ib = np.arange(j, j + L)
            ok = (kg[i:i + L] == ko[j:j + L]) & close(ia, ib)
            bad = np.nonzero(~ok)[0]
            run = L if bad.size == 0 else int(bad[0])
        else:
            run = 0
        seg_g.append(np.arange(i, i + run))
        seg_o.append(np.arange(j, j + run))
        i += run
        j += run
        if run == L and L > 0:
            continue
        if i >= ng or j >= no:
            extra_g.extend(range(i, ng))
            extra_o.extend(range(j, no))
            break
        if len(extra_g) + len(extra_o) >= max_skips:
            raise AssertionError(f"more than {max_skips} unmatched particles")
        if match(i + 1, j):
            extra_g.append(i)
            i += 1
        elif match(i, j + 1):
            extra_o.append(j)
            j += 1
        else:
            extra_g.append(i)
            extra_o.append(j)
            i += 1
            j += 1
    jg = np.concatenate(seg_g) if seg_g else np.zeros(0, dtype=np.int64)
    jo = np.concatenate(seg_o) if seg_o else np.zeros(0, dtype=np.int64)
    return jg, jo, np.array(extra_g, dtype=np.int64), np.array(extra_o, dtype=np.int64)

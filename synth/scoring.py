"""Scoring of detections against the ground truth of the synthetic workloads.

The paper gives no matching rule; the one used here: the truth cell of a tone
at f (cycles/sample) is round(f N_d) mod N_d per dimension; a target is
detected when any detected cell lies within circular L-infinity distance
``guard`` of its truth cell; false alarms are detected cells outside every
target's guard region, counted against the number of cells outside every
guard region. Cells inside a guard region are the target's extended main lobe
(Sec. VI-C) and are neither hits nor false alarms.
"""

import numpy as np


def truth_cells(freqs, shape):
    """Grid cell of each tone: round(f_d N_d) mod N_d (integers)."""
    freqs = np.asarray(freqs, dtype=np.float64).reshape(-1, len(shape))
    if not len(freqs):
        return np.zeros((0, len(shape)), dtype=np.int64)
    return np.stack([np.mod(np.rint(freqs[:, d] * n).astype(np.int64), n)
                     for d, n in enumerate(shape)], axis=1)


def guard_mask(freqs, shape, guard=3):
    """Boolean array of the cells within `guard` (L-inf, circular) of a truth
    cell, and the per-target truth cells."""
    cells = truth_cells(freqs, shape)
    mask = np.zeros(shape, dtype=bool)
    offs = np.arange(-guard, guard + 1)
    for c in cells:
        idx = [np.mod(c[d] + offs, n) for d, n in enumerate(shape)]
        mask[np.ix_(*idx)] = True
    return mask, cells


def pd_pfa(detections, freqs, shape, guard=3):
    """Returns (hits, targets, false_alarms, cells_outside) for one frame.
    `detections` are row-major flat cell indices."""
    mask, cells = guard_mask(freqs, shape, guard)
    det = np.zeros(int(np.prod(shape)), dtype=bool)
    det[np.asarray(detections, dtype=np.int64)] = True
    det = det.reshape(shape)
    hits = 0
    offs = np.arange(-guard, guard + 1)
    for c in cells:
        idx = [np.mod(c[d] + offs, n) for d, n in enumerate(shape)]
        if det[np.ix_(*idx)].any():
            hits += 1
    fa = int(np.count_nonzero(det & ~mask))
    outside = int(np.count_nonzero(~mask))
    return hits, len(cells), fa, outside

"""Scoring and the paper's complexity model (oracle; test infrastructure only).

* ``pd_pfa`` - detection scoring. The paper gives no matching rule; the one
  used here: the truth cell of a tone at f (cycles/sample) is round(f N_d)
  mod N_d per dimension; a target is detected when any detected cell lies
  within circular L-infinity distance ``guard`` of its truth cell; false
  alarms are detected cells outside every target's guard region, counted
  against the number of cells outside every guard region. Cells inside a
  guard region are the target's extended main lobe (Sec. VI-C) and are
  neither hits nor false alarms.
* ``complexity_rsft`` / ``complexity_bartlett`` - operation counts of eq.
  RSFT_complexity and Table I.
"""

import math

import numpy as np


def truth_cells(freqs, shape):
    """Grid cell of each tone: round(f_d N_d) mod N_d (integers)."""
    freqs = np.asarray(freqs, dtype=np.float64).reshape(-1, len(shape))
    return np.stack([np.mod(np.rint(freqs[:, d] * n).astype(np.int64), n)
                     for d, n in enumerate(shape)], axis=1) if len(freqs) else \
        np.zeros((0, len(shape)), dtype=np.int64)


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


def complexity_rsft(N, B, T, K, eta_m, eta_p):
    """eq. RSFT_complexity, with the B-point FFT counted as B log2 B."""
    return T * (N + B + B * math.log2(B) + K * eta_m * N / (B * eta_p)) + N


def complexity_bartlett(N, T):
    """Table I total: T N (1 + log2 N) + N."""
    return T * N * (1 + math.log2(N)) + N


def best_buckets(N, T, K, eta_m, eta_p, candidates):
    """B minimising eq. RSFT_complexity over the given powers of two."""
    return min(candidates, key=lambda b: complexity_rsft(N, b, T, K, eta_m, eta_p))

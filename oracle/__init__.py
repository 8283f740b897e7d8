"""FP64 CPU oracle for RSFT (Wang, Patel, Petropulu, "An Efficient
High-Dimensional Sparse Fourier Transform").

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is plain, slow and written to be checked against the paper by
eye. It follows Algorithm 1 (RSFT) step by step (window, permutation, flat
window, aliasing, B-point N-D FFT, first-stage detection, reverse mapping,
accumulation, second-stage detection) and Algorithm 2 (Bartlett / dense
windowed FFT + Neyman-Pearson detection). It shares no code with the HIP
library: the windows, the hashing, the thresholds and the estimator are all
written here from their definitions.

Modules
-------
windows   Dolph-Chebyshev pre-permutation window, flat window (Sec. III-C,
          Sec. IV-B).
hashing   Definitions 1-4 (permutation, aliasing, mapping, reverse mapping).
rsft      Algorithm 1 literal, thresholds (eq. tpd), noise law (eq.
          alpha_beta), off-grid estimate of detected cells.
dense     Algorithm 2 (Bartlett) with T=1 exact exponential threshold and the
          eq. bartlettROC closed form.
evaluate  the complexity model of Tables I-II.
refine    the bucketized forward model of off-grid tones (eq. f with a
          continuous frequency) and its gradients, for refinement.
design    the optimal threshold design (eq. opt, Claims 2-3, eq. bpd).
"""

from . import windows, hashing, rsft, dense, evaluate, refine, design  # noqa: F401

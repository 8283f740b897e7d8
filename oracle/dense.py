"""Algorithm 2 (Bartlett: windowed dense N-D FFT + Neyman-Pearson detection)
in FP64 (oracle; test infrastructure only), Appendix A.

With T = 1 segment the test statistic |uhat_k|^2 of a noise-only bin is
exponential with mean sigma_n^2 ||w||^2 (beta' of Appendix A), so the
threshold for a per-bin false-alarm probability Pfa is
sigma_n^2 ||w||^2 ln(1/Pfa), exactly. For T > 1 segments the sum of T
such exponentials is Gamma(T) and the threshold is its upper Pfa quantile;
Appendix A's eq. bartlettROC is the Normal approximation of the same test.
"""

import math

import numpy as np
from scipy import special, stats

from . import windows


def windowed_spectrum(r, w_list):
    """u <- W r ; uhat <- NDFFT(u)  (Alg. 2, one segment)."""
    r = np.asarray(r, dtype=np.complex128)
    return np.fft.fftn(r * windows.nd_window(w_list))


def window_energy(w_list):
    """beta' = ||w||^2 of the N-D window (Appendix A)."""
    return float(np.sum(np.abs(windows.nd_window(w_list)) ** 2))


def bartlett_detect(segments, w_list, pfa, noise_var=1.0):
    """Alg. 2 over T segments (a list of arrays, or one array for T=1):
    x = sum_s |NDFFT(W r_s)|^2, detect x >= threshold with the exact Gamma(T)
    quantile. Returns (flat detections ascending, x, threshold)."""
    if not isinstance(segments, (list, tuple)):
        segments = [segments]
    x = None
    for r in segments:
        p = np.abs(windowed_spectrum(r, w_list)) ** 2
        x = p if x is None else x + p
    T = len(segments)
    zeta2 = noise_var * window_energy(w_list)
    if T == 1:
        thr = zeta2 * math.log(1.0 / pfa)
    else:
        thr = float(stats.gamma.isf(pfa, T, scale=zeta2))
    return np.flatnonzero(x >= thr), x, thr


def bartlett_roc_pd(pfa, T, snr_min, alpha_p, beta_p):
    """eq. bartlettROC: Pd of the Normal-approximated Bartlett detector."""
    phi_inv = math.sqrt(2.0) * special.erfinv(2.0 * (1.0 - pfa) - 1.0)
    arg = (beta_p * phi_inv + math.sqrt(T) * (beta_p - snr_min * alpha_p)) \
        / (snr_min * alpha_p)
    return 1.0 - 0.5 * (1.0 + math.erf(arg / math.sqrt(2.0)))

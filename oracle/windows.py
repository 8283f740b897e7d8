"""Windows used by RSFT, in FP64 (oracle; test infrastructure only).

* ``dolph_chebyshev`` - the pre-permutation window (Sec. III-A: a window on
  the time-domain data before permutation; Sec. III-C.1 and Fig. 2: a
  Dolph-Chebyshev window per dimension, combined as an outer product).
* ``flat_window`` - the flat window of the first-stage detection (Sec. IV-B:
  length N, frequency-domain main lobe of width 2*pi/B; Sec. V: "based on"
  the same Dolph-Chebyshev window with passband 1/B). The paper does not
  spell out its construction; the reading used here is written in the
  docstring of ``flat_window``.

Both are computed from their definitions; nothing here calls a window
routine from a library.
"""

import numpy as np


def chebyshev_poly(order, x):
    """T_order(x) for real x, valid on the whole real line (FP64).

    |x| <= 1: cos(order * acos x); x > 1: cosh(order * acosh x);
    x < -1: (-1)^order cosh(order * acosh(-x)).
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(order * np.arccos(x[inside]))
    above = x > 1.0
    out[above] = np.cosh(order * np.arccosh(x[above]))
    below = x < -1.0
    sign = -1.0 if (order % 2) else 1.0
    out[below] = sign * np.cosh(order * np.arccosh(-x[below]))
    return out


def dolph_chebyshev(n, atten_db):
    """Symmetric length-n Dolph-Chebyshev window with sidelobes atten_db below
    the main lobe, scaled so that sample n//2 equals 1.

    Definition: the window's DTFT is exp(-j w (n-1)/2) * T_{n-1}(x0 cos(w/2))
    with x0 = cosh(acosh(10^(A/20)) / (n-1)). That amplitude is a polynomial
    of degree n-1 in exp(-j w), so its n samples at w_k = 2 pi k / n determine
    the window exactly: w = IDFT_n(samples).

    Normalisation (the paper does not state one): divide by the sample at
    n//2, the centre. For the attenuations and lengths used here the centre is
    the maximum, so this equals max-normalisation.
    atten_db == 0 means the rectangular window (all ones).
    """
    n = int(n)
    if n < 1:
        raise ValueError("window length must be >= 1")
    if atten_db == 0:
        return np.ones(n, dtype=np.float64)
    if atten_db < 0:
        raise ValueError("attenuation must be >= 0 dB")
    if n == 1:
        return np.ones(1, dtype=np.float64)
    order = n - 1
    ratio = 10.0 ** (atten_db / 20.0)
    x0 = np.cosh(np.arccosh(ratio) / order)
    k = np.arange(n, dtype=np.float64)
    amp = chebyshev_poly(order, x0 * np.cos(np.pi * k / n))
    # linear phase of a window centred at (n-1)/2
    spectrum = amp * np.exp(-1j * np.pi * k * (n - 1) / n)
    w = np.fft.ifft(spectrum)
    w = w.real
    return w / w[n // 2]


def dolph_chebyshev_periodic(n, atten_db):
    """DFT-even ("periodic") Dolph-Chebyshev of length n: the symmetric window
    of length n+1 with its last sample dropped. Its peak sits at index n/2."""
    return dolph_chebyshev(n + 1, atten_db)[:n]


def dtft(w, omegas):
    """Plain DTFT sum_n w[n] exp(-j omega n) at the given frequencies."""
    n = np.arange(len(w), dtype=np.float64)
    return np.exp(-1j * np.outer(omegas, n)) @ w


def flat_window(n, b, atten_db):
    """Complex flat window of length n for B = b buckets (one dimension).

    Reading of the paper (its flat window is described only as having a main
    lobe of width 2 pi / B, length N, "based on" the Dolph-Chebyshev window,
    passband 1/B):

        wbar[m] = c0[m] * sum_{k=-(L-1)}^{0} exp(j 2 pi k m / n),   L = n / b,

    where c0 is the periodic length-n Dolph-Chebyshev window at atten_db,
    circularly shifted so that its peak is at m = 0 and scaled so c0[0] = 1
    (atten_db == 0 gives c0 = 1, an exact box). Its spectrum is the box of the
    L bins {-(L-1), ..., 0} convolved with the narrow Chebyshev spectrum, with
    gain ~n inside the box, so bucket j collects the permuted bins
    [jL, (j+1)L), the bins that Definition 3 (floor of the scaled index) maps
    to bucket j.
    """
    n = int(n)
    b = int(b)
    if n % b:
        raise ValueError("b must divide n")
    L = n // b
    c = dolph_chebyshev_periodic(n, atten_db)
    c0 = np.roll(c, -(n // 2))
    c0 = c0 / c0[0]
    m = np.arange(n, dtype=np.float64)
    box = np.zeros(n, dtype=np.complex128)
    for k in range(-(L - 1), 1):
        box += np.exp(2j * np.pi * k * m / n)
    return c0 * box


def nd_window(vectors):
    """Separable N-D window: the outer product of per-dimension windows
    (Sec. III-C.1, W_xy = w_x w_y^H generalised to any number of dims)."""
    out = np.asarray(vectors[0])
    for v in vectors[1:]:
        out = np.multiply.outer(out, np.asarray(v))
    return out


def six_db_width_bins(w, oversample=64):
    """6.0-dB main-lobe width of window w in DFT bins (the eta_m of Sec. IV-A),
    measured on a dense DTFT grid."""
    n = len(w)
    grid = np.arange(0, n * oversample // 2 + 1) / (n * oversample)
    mag = np.abs(dtft(w, 2 * np.pi * grid))
    mag = mag / mag[0]
    below = np.nonzero(mag < 10 ** (-6.0 / 20.0))[0][0]
    # linear interpolation between the two grid points around -6 dB
    f0, f1 = grid[below - 1], grid[below]
    m0, m1 = mag[below - 1], mag[below]
    target = 10 ** (-6.0 / 20.0)
    f = f0 + (m0 - target) * (f1 - f0) / (m0 - m1)
    return 2.0 * f * n

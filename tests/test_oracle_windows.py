"""Pins of the oracle's windows (Sec. III-C.1 Dolph-Chebyshev pre-permutation
window, Fig. 2; Sec. IV-B flat window) against facts that do not come from the
oracle itself: scipy's independent Dolph-Chebyshev routine, the equiripple
property that defines the window, and closed forms of the flat window."""

import numpy as np
import pytest
from scipy.signal import windows as sw

from oracle import windows as W


@pytest.mark.parametrize("n,atten", [(2, 60), (8, 60), (16, 60), (33, 40),
                                     (64, 60), (128, 60), (256, 60),
                                     (1024, 60), (1024, 40), (2048, 60)])
def test_chebyshev_matches_scipy(n, atten):
    ours = W.dolph_chebyshev(n, atten)
    ref = sw.chebwin(n, atten, sym=True)
    ref = ref / ref[n // 2]
    assert np.max(np.abs(ours - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n,atten", [(64, 60), (1024, 60), (64, 40), (257, 50)])
def test_chebyshev_equiripple_sidelobes(n, atten):
    """Every sidelobe peak of a Dolph-Chebyshev window sits exactly atten dB
    below the main lobe (Chebyshev polynomial: |T| <= 1 outside, T(x0) = r)."""
    w = W.dolph_chebyshev(n, atten)
    grid = np.linspace(0.0, np.pi, 64 * n + 1)
    mag = np.abs(W.dtft(w, grid))
    peak = mag[0]
    # first null: leave the main lobe
    first_min = np.argmax(np.diff(mag) > 0)
    side = mag[first_min:].max()
    level = 20 * np.log10(side / peak)
    assert abs(level + atten) < 0.01


def test_chebyshev_symmetric_and_center_normalised():
    for n in (16, 64, 1024):
        w = W.dolph_chebyshev(n, 60)
        assert np.allclose(w, w[::-1], atol=1e-14)
        assert w[n // 2] == 1.0
    assert np.array_equal(W.dolph_chebyshev(32, 0), np.ones(32))


def test_periodic_is_dft_even():
    """The periodic base window: c[k] == c[n-k] about its peak n/2."""
    n = 256
    c = W.dolph_chebyshev_periodic(n, 60)
    c0 = np.roll(c, -(n // 2))
    assert np.allclose(c0[1:], c0[1:][::-1], atol=1e-14)
    assert np.argmax(c) == n // 2


@pytest.mark.parametrize("n,b", [(64, 8), (256, 16), (1024, 64)])
def test_flat_window_rectangular_base_is_exact_box(n, b):
    """With a rectangular base the flat window's DFT is exactly n on the L bins
    {-(L-1), ..., 0} and 0 elsewhere (sum of L complex exponentials)."""
    L = n // b
    g = np.fft.fft(W.flat_window(n, b, 0))
    box = np.zeros(n, dtype=bool)
    box[(-np.arange(L)) % n] = True
    assert np.allclose(g[box], n, atol=1e-9 * n)
    assert np.max(np.abs(g[~box])) < 1e-9 * n


@pytest.mark.parametrize("n,b", [(256, 16), (1024, 64), (2048, 128)])
def test_flat_window_spectrum_is_box_convolved_with_base(n, b):
    """DFT(c0 * box-exponentials) equals the circular convolution of the box of
    L bins with DFT(c0) (convolution theorem written out as a plain sum)."""
    L = n // b
    c = W.dolph_chebyshev_periodic(n, 60)
    c0 = np.roll(c, -(n // 2))
    c0 = c0 / c0[0]
    C = np.fft.fft(c0)
    conv = np.zeros(n, dtype=np.complex128)
    for k in range(-(L - 1), 1):
        conv += np.roll(C, k)
    g = np.fft.fft(W.flat_window(n, b, 60))
    assert np.max(np.abs(g - conv)) < 1e-9 * n


def test_flat_window_passband_and_stopband_60db():
    n, b = 1024, 64
    L = n // b
    g = np.abs(np.fft.fft(W.flat_window(n, b, 60))) / n
    passband = g[(-np.arange(1, L - 1)) % n]       # inner bins of the box
    assert passband.min() > 0.97 and passband.max() < 1.001
    # more than 3 bins outside the box the response is below the -60 dB base
    outside = np.ones(n, dtype=bool)
    outside[(-np.arange(-3, L + 3)) % n] = False
    assert 20 * np.log10(g[outside].max()) < -60.0


def test_six_db_width_of_chebyshev():
    """eta_m of Sec. IV-A measured from the window (reading: the 6.0-dB width
    in bins). Known values of the Dolph-Chebyshev family: wider main lobe for
    larger attenuation, ~1.67 bins at 40 dB and ~2.02 at 60 dB."""
    e40 = W.six_db_width_bins(W.dolph_chebyshev(1024, 40))
    e60 = W.six_db_width_bins(W.dolph_chebyshev(1024, 60))
    e0 = W.six_db_width_bins(np.ones(1024))
    assert 1.19 < e0 < 1.23            # rectangular window: 1.21 bins
    assert 1.6 < e40 < 1.75 and 1.95 < e60 < 2.1 and e60 > e40

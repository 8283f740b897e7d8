"""The SRUR cube generator: Table III/IV arithmetic (eq. s_u) and a
noise-free target's 3-D spectrum peaking at its cell."""

import numpy as np

from synth import radar


def test_target_frequencies_from_tables():
    f = radar.target_frequencies(1000.0, 100.0, 30.0)
    fd = 2 * 100.0 / 0.03
    assert abs(f[0] - fd * 5e-5) < 1e-12                    # Doppler per RI
    assert abs(f[1] - 0.25) < 1e-12                         # sin(30 deg) / 2
    assert abs(f[2] - (2 * 3e12 * 1000.0 / 3e8 + fd) / 41e6) < 1e-12
    for r, v, a, _ in radar.TARGETS:
        back = radar.physical_from_frequencies(radar.target_frequencies(r, v, a))
        assert abs(back[0] - r) < 1e-6 and abs(back[1] - v) < 1e-9 and abs(back[2] - a) < 1e-9


def test_noise_free_cube_peaks_at_target_cell():
    p = dict(radar.SRUR, R=256, N=16, M=8)
    tgt = [(400.0, 120.0, 10.0, (40.0, 40.0))]
    cubes, freqs, _ = radar.make_cpi(0, 1, targets=tgt, p=p, dtype=np.complex128)
    shape = radar.cube_shape(p)
    spec = np.abs(np.fft.fftn(cubes[0]))
    peak = np.unravel_index(np.argmax(spec), shape)
    for d, n in enumerate(shape):
        want = freqs[0, d] * n
        dist = min(abs(peak[d] - want), n - abs(peak[d] - want))
        assert dist <= 0.5 + 1e-9

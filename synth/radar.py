"""Seeded synthetic short-range ubiquitous radar (SRUR) data: de-chirped
LFMCW data cubes of a uniform linear array (Sec. VI), for T bursts.

System parameters are those of Table III and the targets those of Table IV.
Each burst is one cube of M repetition intervals x N receiving elements x R
range samples, complex (IQ), stored [M][N][R] with the range samples
contiguous. Target k contributes, at RI v, element i and range sample n,

    a_k(s) exp(j 2 pi (f_rg n + f_ri v + f_el i)),
    f_rg = (f_r + f_d) / f_s,  f_ri = f_d T_p,  f_el = sin(theta) / 2,
    f_r = 2 rho r / c,  f_d = 2 v / lambda      (eq. s_u)

(frequencies in cycles per sample of each dimension, taken modulo 1), with
a complex amplitude a_k(s) ~ CN(0, 10^(SNR_k/10)) fixed within burst s and
independent across bursts (Swerling I), in CN(0, 1) noise. The paper's
eq. r_i writes range and Doppler in one real cosine of the intra-RI time;
this generator takes the usual complex form in which the Doppler phase also
advances from RI to RI, so that range, velocity and direction of arrival are
three separate frequencies of the cube (a reading, not the printed formula).

This module holds none of RSFT's arithmetic; the oracle and the HIP library
both consume what it returns.
"""

import math

import numpy as np

from . import complex_noise

RADAR_SEED = 1610010506

# Table III
SRUR = dict(R=2048, N=64, M=32, wavelength=0.03, c=3e8, bandwidth=150e6, Tp=5e-5,
            r_max=1.5e3, rho=3e12, fs=41e6)

# Table IV: range (m), velocity (m/s), DOA (degrees), SNR (dB) in the
# "equal" and the "different" setting
TARGETS = [
    (1000.0, 100.0, 30.0, (-10.0, 0.0)),
    (500.0, 50.0, 0.0, (-10.0, -10.0)),
    (350.0, 240.0, -16.0, (-10.0, -20.0)),
    (350.0, 240.0, -20.0, (-10.0, -20.0)),
]


def cube_shape(p=SRUR):
    return (p["M"], p["N"], p["R"])


def target_frequencies(r, v, doa_deg, p=SRUR):
    """(f_ri, f_el, f_rg) of a target, cycles/sample in [0, 1), in the cube's
    dimension order [RI, element, range]."""
    fr = 2.0 * p["rho"] * r / p["c"]
    fd = 2.0 * v / p["wavelength"]
    return np.array([(fd * p["Tp"]) % 1.0,
                     (0.5 * math.sin(math.radians(doa_deg))) % 1.0,
                     ((fr + fd) / p["fs"]) % 1.0])


def physical_from_frequencies(f, p=SRUR):
    """Inverse of target_frequencies for the unambiguous region: (range m,
    velocity m/s, DOA degrees) from (f_ri, f_el, f_rg)."""
    fd = (f[0] % 1.0) / p["Tp"]
    s = (f[1] + 0.5) % 1.0 - 0.5
    doa = math.degrees(math.asin(max(-1.0, min(1.0, 2.0 * s))))
    fr = (f[2] % 1.0) * p["fs"] - fd
    return fr * p["c"] / (2.0 * p["rho"]), fd * p["wavelength"] / 2.0, doa


def make_cpi(cpi, bursts, snr_set="equal", targets=TARGETS, p=SRUR, dtype=np.complex64):
    """One coherent processing interval: `bursts` cubes [T][M][N][R] with the
    targets of Table IV (SNR setting "equal" or "different"), seeded by
    (RADAR_SEED, cpi). Returns (cubes, freqs [K][3], snr_db [K])."""
    rng = np.random.default_rng([RADAR_SEED, int(cpi)])
    shape = cube_shape(p)
    col = 0 if snr_set == "equal" else 1
    freqs = np.stack([target_frequencies(r, v, a, p) for r, v, a, _ in targets])
    snr_db = np.array([t[3][col] for t in targets])
    vecs = [np.exp(2j * np.pi * np.outer(np.arange(n), freqs[:, d])) for d, n in enumerate(shape)]
    out = np.empty((bursts,) + shape, dtype=dtype)
    for s in range(bursts):
        amps = complex_noise(rng, (len(targets),), 1.0) * np.sqrt(10.0 ** (snr_db / 10.0))
        acc = (vecs[0] * amps[None, :])[:, None, :] * vecs[1][None, :, :]     # [M][N][K]
        x = acc.reshape(-1, len(targets)) @ vecs[2].T                          # [M*N][R]
        out[s] = (x.reshape(shape) + complex_noise(rng, shape)).astype(dtype)
    return out, freqs, snr_db

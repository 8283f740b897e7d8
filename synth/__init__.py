"""Seeded synthetic workloads for RSFT: sparse complex tones in white complex
Gaussian noise (the signal model of eq. sig_model / eq. sinusoid, extended to
N dimensions), plus the random permutation factors the method draws.

This module holds none of RSFT's arithmetic. It only produces inputs; both
the FP64 oracle and the HIP library consume what it returns, so neither of
them depends on the other.

Recipes (one per workload; the workload's seed, per-frame generator
numpy.random.default_rng([seed, frame])). Draw order per frame:
(shape, for the uneven batch), tone count, frequencies (re-drawn until every
pair of tones is more than ``min_sep`` bins apart in circular L-infinity
distance), per-tone SNR in dB, complex amplitudes, noise, and (for per-frame
permutations) sigma.

  ongrid_256x256_c128
      256x256 complex128, K=4 on-grid tones >= 3 bins apart, unit magnitude,
      uniform phase, CN(0,1) noise (0 dB per sample), B=16x16, T=3,
      Pfa=1e-3, 60 dB Chebyshev windows, one sigma set for the batch.
  offgrid_1024x1024
      1024x1024 complex64, K=20 off-grid tones f ~ U[0,1)^2, SNR ~ U[-10,10]
      dB, Rayleigh amplitudes b ~ CN(0, 10^(SNR/10)), B=64x64, T=3, Pfa=1e-4.
  cube_256x128x32
      256x128x32 complex64 radar cube (range, Doppler, antenna), K=16 off-grid
      tones, SNR ~ U[-5,15] dB, B=32x16x8, T=3, Pfa=1e-4, sigma per CPI.
  uneven_128_to_2048
      uneven batch: N_d drawn per dimension from {128,...,2048}, K ~ U{1..50},
      SNR ~ U[-10,10] dB, B_d = N_d/16, T=3, Pfa=1e-4, sigma per frame.
  offgrid_2048x2048
      2048x2048 complex64, K=32 off-grid, SNR ~ U[-10,10] dB, B=128x128,
      T=3, Pfa=1e-4.
"""

import numpy as np

BASE_SEED = 1610010500

WORKLOADS = {
    "ongrid_256x256_c128": dict(
        seed=BASE_SEED + 1, shape=(256, 256), buckets=(16, 16), K=4, ongrid=True,
        unit_amplitude=True, snr_db=(0.0, 0.0), dtype=np.complex128, rounds=3, pfa=1e-3,
        atten_db=60.0, sigma_per_frame=False, min_sep=3.0),
    "offgrid_1024x1024": dict(
        seed=BASE_SEED + 2, shape=(1024, 1024), buckets=(64, 64), K=20, ongrid=False,
        unit_amplitude=False, snr_db=(-10.0, 10.0), dtype=np.complex64, rounds=3, pfa=1e-4,
        atten_db=60.0, sigma_per_frame=False, min_sep=2.05),
    "cube_256x128x32": dict(
        seed=BASE_SEED + 3, shape=(256, 128, 32), buckets=(32, 16, 8), K=16, ongrid=False,
        unit_amplitude=False, snr_db=(-5.0, 15.0), dtype=np.complex64, rounds=3, pfa=1e-4,
        atten_db=60.0, sigma_per_frame=True, min_sep=2.05),
    "uneven_128_to_2048": dict(
        seed=BASE_SEED + 4, shape=None, buckets=None, K=(1, 50), ongrid=False,
        unit_amplitude=False, snr_db=(-10.0, 10.0), dtype=np.complex64, rounds=3, pfa=1e-4,
        atten_db=60.0, sigma_per_frame=True, min_sep=2.05, sides=(128, 256, 512, 1024, 2048)),
    "offgrid_2048x2048": dict(
        seed=BASE_SEED + 5, shape=(2048, 2048), buckets=(128, 128), K=32, ongrid=False,
        unit_amplitude=False, snr_db=(-10.0, 10.0), dtype=np.complex64, rounds=3, pfa=1e-4,
        atten_db=60.0, sigma_per_frame=False, min_sep=2.05),
}


def draw_sigma(rng, rounds, shape):
    """Permutation factors sigma_{s,d}: independent, uniform over the odd
    integers of [1, N_d) (every odd integer is invertible modulo a power of
    two). Returns int64 [rounds][D]."""
    out = np.empty((rounds, len(shape)), dtype=np.int64)
    for s in range(rounds):
        for d, n in enumerate(shape):
            out[s, d] = 2 * int(rng.integers(0, n // 2)) + 1
    return out


def _circ_linf_bins(a, b, shape):
    """Circular L-infinity distance in bins between two frequency vectors."""
    dist = 0.0
    for d, n in enumerate(shape):
        x = abs(a[d] - b[d]) * n
        x = min(x, n - x)
        dist = max(dist, x)
    return dist


def draw_frequencies(rng, shape, K, ongrid, min_sep):
    """K tone frequencies in cycles/sample per dimension. On-grid tones are
    integers k_d / N_d (returned with their integer bins)."""
    freqs = []
    bins = []
    attempts = 0
    while len(freqs) < K:
        attempts += 1
        if attempts > 100000:
            raise RuntimeError("could not place tones at the requested spacing")
        if ongrid:
            k = [int(rng.integers(0, n)) for n in shape]
            f = [k[d] / n for d, n in enumerate(shape)]
        else:
            k = None
            f = [float(rng.random()) for _ in shape]
        if all(_circ_linf_bins(f, g, shape) >= min_sep if ongrid else
               _circ_linf_bins(f, g, shape) > min_sep for g in freqs):
            freqs.append(f)
            bins.append(k)
    return np.array(freqs, dtype=np.float64).reshape(K, len(shape)), bins


def tone_vectors(shape, freqs, bins):
    """Per-dimension complex exponentials e_{t,d}[m] = exp(j 2 pi f_{t,d} m).
    For on-grid tones the phase is 2 pi (k m mod N) / N from integers."""
    out = []
    for d, n in enumerate(shape):
        m = np.arange(n, dtype=np.int64)
        cols = []
        for t in range(len(freqs)):
            if bins and bins[t] is not None:
                ph = 2.0 * np.pi * ((bins[t][d] * m) % n) / n
            else:
                ph = 2.0 * np.pi * freqs[t, d] * m.astype(np.float64)
            cols.append(np.exp(1j * ph))
        out.append(np.stack(cols, axis=1) if cols else
                   np.zeros((n, 0), dtype=np.complex128))
    return out


def synthesize(shape, freqs, bins, amps):
    """sum_t b_t prod_d e_{t,d}[m_d] as an N-D complex128 array."""
    vecs = tone_vectors(shape, freqs, bins)
    if len(amps) == 0:
        return np.zeros(shape, dtype=np.complex128)
    acc = vecs[0] * np.asarray(amps)[None, :]
    for d in range(1, len(shape) - 1):
        acc = (acc[:, None, :] * vecs[d][None, :, :]).reshape(-1, len(amps))
    if len(shape) == 1:
        return acc.sum(axis=1)
    return (acc @ vecs[-1].T).reshape(shape)


def complex_noise(rng, shape, var=1.0):
    """CN(0, var I): real and imaginary parts each N(0, var/2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(var / 2.0)


def workload_seed(workload):
    return WORKLOADS[workload]["seed"]


def shared_sigma(workload, rounds=None, shape=None):
    """One sigma set shared by every frame of a batch."""
    cfg = WORKLOADS[workload]
    rng = np.random.default_rng([workload_seed(workload), 1 << 30])
    return draw_sigma(rng, rounds or cfg["rounds"], shape or cfg["shape"])


def make_frame(workload, frame, K=None, noise=True, noise_var=1.0):
    """One synthetic frame of a workload. Returns a dict with the frame
    (workload dtype), the tone frequencies (cycles/sample, [K][D]), the complex
    amplitudes, the shape, and sigma (per-frame configs only)."""
    cfg = WORKLOADS[workload]
    rng = np.random.default_rng([workload_seed(workload), int(frame)])
    if cfg["shape"] is None:
        shape = tuple(int(rng.choice(cfg["sides"])) for _ in range(2))
    else:
        shape = cfg["shape"]
    if K is None:
        if isinstance(cfg["K"], tuple):
            K = int(rng.integers(cfg["K"][0], cfg["K"][1] + 1))
        else:
            K = cfg["K"]
    freqs, bins = draw_frequencies(rng, shape, K, cfg["ongrid"], cfg["min_sep"])
    lo, hi = cfg["snr_db"]
    snr_db = rng.uniform(lo, hi, size=K) if hi > lo else np.full(K, lo)
    if cfg["unit_amplitude"]:
        amps = np.exp(2j * np.pi * rng.random(K))
    else:
        amps = complex_noise(rng, (K,), 1.0) * np.sqrt(10.0 ** (snr_db / 10.0))
    x = synthesize(shape, freqs, bins if cfg["ongrid"] else None, amps)
    if noise:
        x = x + complex_noise(rng, shape, noise_var)
    out = {"frame": x.astype(cfg["dtype"]), "freqs": freqs, "amps": amps,
           "snr_db": snr_db, "shape": shape}
    if cfg["sigma_per_frame"]:
        out["sigma"] = draw_sigma(rng, cfg["rounds"], shape)
    return out


def make_batch(workload, nframes, start=0, K=None, noise=True):
    """`nframes` consecutive frames of a uniform-shape configuration stacked
    into one array [F, *shape] (workload dtype), with per-frame metadata."""
    metas = [make_frame(workload, start + f, K=K, noise=noise)
             for f in range(nframes)]
    frames = np.stack([m.pop("frame") for m in metas]) if metas else None
    return frames, metas


def noise_only(shape, seed, frame, dtype=np.complex64, var=1.0):
    """A noise-only frame (K = 0) from its own seed stream."""
    rng = np.random.default_rng([int(seed), int(frame), 7])
    return complex_noise(rng, shape, var).astype(dtype)

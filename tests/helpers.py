"""Shared helpers of the GPU parity tests (not collected as tests)."""

import numpy as np

from oracle import rsft as oracle_rsft

BUCKET_RTOL = 1e-4      # bucket values: max error <= 1e-4 * rms of the round
FLAG_BAND = 1e-3        # a flag may differ only where |P - gamma| / gamma <= 1e-3


def pack_flags(flags):
    """bool [T, *B] -> uint32 words [T, ceil(B/32)], bucket j (row-major) is
    bit j % 32 of word j // 32."""
    T = flags.shape[0]
    flat = flags.reshape(T, -1).astype(np.uint64)
    B = flat.shape[1]
    words = np.zeros((T, (B + 31) // 32), dtype=np.uint64)
    for j in range(B):
        words[:, j // 32] |= flat[:, j] << np.uint64(j % 32)
    return words.astype(np.uint32)


def unpack_flags(words, buckets):
    words = np.asarray(words).astype(np.uint32)
    T = words.shape[0]
    B = int(np.prod(buckets))
    j = np.arange(B)
    bits = (words[:, j // 32] >> (j % 32).astype(np.uint32)) & 1
    return bits.astype(bool).reshape((T,) + tuple(buckets))


def bucket_errors(gpu, ora):
    """Per round: max |gpu - ora| / rms(ora)."""
    out = []
    for s in range(ora.shape[0]):
        rms = np.sqrt(np.mean(np.abs(ora[s]) ** 2))
        out.append(float(np.max(np.abs(gpu[s] - ora[s])) / rms))
    return out


def ambiguous(ora, gamma):
    """Buckets whose power lies within FLAG_BAND of the round's threshold."""
    p = np.abs(ora) ** 2
    g = np.asarray(gamma).reshape((-1,) + (1,) * (ora.ndim - 1))
    return np.abs(p - g) <= FLAG_BAND * g


def free_cells(amb, plan):
    """Cells whose T buckets include an ambiguous one: their votes may differ
    between an FP32 and an FP64 evaluation."""
    return oracle_rsft.votes_by_mapping(amb, plan) > 0


def cells_from_records(recs, shape, frame):
    sel = recs[recs["frame"] == frame]
    D = len(shape)
    return {int(np.ravel_multi_index(tuple(int(v) for v in r["idx"][:D]), shape)): r
            for r in sel}


def make_input(shape, K, seed, dtype=np.complex64, snr_db=(-5.0, 15.0), noise_var=1.0):
    """A seeded frame of K off-grid Rayleigh tones in CN(0, noise_var) noise,
    built from the synthetic-input primitives; returns (frame, freqs)."""
    import synth
    rng = np.random.default_rng([int(seed), 99])
    freqs, _ = synth.draw_frequencies(rng, shape, K, False, 2.05)
    snr = rng.uniform(snr_db[0], snr_db[1], size=K)
    amps = synth.complex_noise(rng, (K,), 1.0) * np.sqrt(10.0 ** (snr / 10.0))
    x = synth.synthesize(shape, freqs, None, amps) + synth.complex_noise(rng, shape, noise_var)
    return x.astype(dtype), freqs


def oracle_plan(shape, buckets, sigma, atten=60.0, flat=-1.0, pfa=1e-3, mu=0, noise_var=1.0):
    return oracle_rsft.OraclePlan(shape, buckets, sigma, atten, flat, pfa,
                                  None if mu == 0 else mu, noise_var)

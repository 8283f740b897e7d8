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


def check_frame(f, oplan, ref, recs, gbk, gfl, check_estimates=True):
    """Parity of one frame: buckets, flags, detections, votes and (for
    detections whose votes are fixed) estimates, against the oracle's
    result `ref` for that frame."""
    errs = bucket_errors(gbk, ref["buckets"])
    assert max(errs) <= BUCKET_RTOL, f"frame {f}: bucket errors {errs}"
    amb = ambiguous(ref["buckets"], ref["gamma"])
    gflags = unpack_flags(gfl, oplan.B)
    diff = gflags != ref["flags"]
    assert not np.any(diff & ~amb), f"frame {f}: flag mismatch outside the ambiguity band"
    free = free_cells(amb, oplan).ravel()
    got = cells_from_records(recs, oplan.shape, f)
    want = set(int(v) for v in ref["detections"])
    sym = set(got) ^ want
    assert all(free[c] for c in sym), f"frame {f}: {len(sym)} detection differences on fixed cells"
    votes = ref["votes"].ravel()
    for c, r in got.items():
        if not free[c]:
            assert int(r["votes"]) == int(votes[c])
    if not check_estimates:
        return
    common = sorted(c for c in set(got) & want if not free[c])
    est = {e["cell"]: e for e in oracle_rsft.estimate(common, ref["buckets"], oplan)}
    gains = oracle_rsft.flat_window_gain(oplan)
    for c in common:
        r, e = got[c], est[c]
        assert abs(float(r["magnitude"]) / e["magnitude"] - 1.0) < 1e-3
        if bool(r["is_peak"]) != e["is_peak"]:
            # the peak decision may flip only on a near-tie with a neighbour
            # (FP32 buckets carry ~1e-5 relative error)
            cell = np.unravel_index(c, oplan.shape)
            a0 = e["magnitude"]
            gap = min(abs(a0 - oracle_rsft.cell_magnitude(
                tuple((cell[d] + o[d] - 1) % oplan.shape[d] for d in range(len(cell))),
                ref["buckets"], oplan, gains)) / a0
                for o in np.ndindex(*([3] * len(cell))) if any(v != 1 for v in o))
            assert gap <= 2e-3, f"cell {c}: peak flag differs with nearest neighbour gap {gap}"
            continue
        if e["is_peak"]:
            for d in range(len(oplan.shape)):
                dd = (float(r["freq"][d]) - e["freq"][d] + 0.5) % 1.0 - 0.5
                assert abs(dd * oplan.shape[d]) <= 1e-3, f"cell {c} dim {d}: {dd * oplan.shape[d]} bin"

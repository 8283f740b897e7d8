"""Pins of the oracle's segment mode (round s on data segment s, Sec. IV-A)
and of a given first-stage false-alarm probability: equal segments reduce to
the same-data rounds, and with independent noise segments the rounds' flags
are independent Bernoulli(p1), so the final per-cell false-alarm rate is
exactly P[Binomial(T, p1) >= mu] (the second stage of Sec. IV-C without its
asymptotics)."""

import math

import numpy as np
from scipy import stats

import synth
from oracle import rsft as R


def _plan(shape, b, T, mu=None, pfa=1e-3, stage1_pfa=None, seed=0):
    sigma = synth.draw_sigma(np.random.default_rng(seed), T, shape)
    return R.OraclePlan(shape, b, sigma, 60.0, None, pfa, mu, 1.0, stage1_pfa)


def test_equal_segments_reduce_to_same_data_rounds():
    shape, b = (64, 64), (8, 8)
    plan = _plan(shape, b, 4, mu=3, seed=2)
    x = synth.noise_only(shape, 5, 0, dtype=np.complex128) + 3.0
    same = R.rsft(x, plan)
    seg = R.rsft(np.stack([x] * 4), plan, segments=True)
    for key in ("buckets", "flags", "votes", "detections"):
        assert np.array_equal(same[key], seg[key])


def test_independent_segments_final_pfa_is_exact_binomial():
    """T = mu = 3, Pfa = 1e-3 (p1 = 0.1): the rate over 500 noise-only frames
    of 128 x 128 is 1e-3 within 3 standard errors computed over frames."""
    shape, b = (128, 128), (16, 16)
    plan = _plan(shape, b, 3, pfa=1e-3, seed=8)
    N = shape[0] * shape[1]
    rates = []
    for f in range(500):
        segs = np.stack([synth.noise_only(shape, 2024, 3 * f + s, dtype=np.complex128)
                         for s in range(3)])
        rates.append(len(R.rsft(segs, plan, segments=True)["detections"]) / N)
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(len(rates))
    assert abs(rates.mean() - 1e-3) < 3 * se


def test_given_stage1_pfa_sets_thresholds_and_binomial_rate():
    """stage1_pfa = 0.1 with T = 20, mu = 6: every round flags 10% of noise
    buckets, and the final rate is P[Bin(20, 0.1) >= 6] = 0.0113."""
    shape, b = (64, 64), (8, 8)
    plan = _plan(shape, b, 20, mu=6, stage1_pfa=0.1, seed=3)
    assert plan.p1 == 0.1
    N = shape[0] * shape[1]
    rates, flagged = [], []
    for f in range(200):
        segs = np.stack([synth.noise_only(shape, 77, 20 * f + s, dtype=np.complex128)
                         for s in range(20)])
        out = R.rsft(segs, plan, segments=True)
        rates.append(len(out["detections"]) / N)
        flagged.append(out["flags"].mean())
    want = stats.binom.sf(5, 20, 0.1)
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(len(rates))
    assert abs(rates.mean() - want) < 3 * se
    assert abs(np.mean(flagged) - 0.1) < 4 * math.sqrt(0.1 * 0.9 / (200 * 20 * 64))

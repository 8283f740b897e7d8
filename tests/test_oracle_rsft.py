"""Pins of the oracle's Algorithm 1 against the mathematics: brute-force DFTs,
closed-form buckets of on-grid tones, the exact noise law of eq. alpha_beta,
the exact exponential first-stage law (eq. exp / eq. tpd), the final Pfa
under H0, the vote identity of Properties 3-4, and Claim 1."""

import itertools
import math

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import hashing as H
from oracle import rsft as R
from oracle import windows as W


def brute_dftn(x):
    """O(N^2) N-D DFT written out as a plain sum."""
    shape = x.shape
    out = np.zeros(shape, dtype=np.complex128)
    for k in itertools.product(*[range(n) for n in shape]):
        acc = 0j
        for m in itertools.product(*[range(n) for n in shape]):
            ph = sum(k[d] * m[d] / shape[d] for d in range(len(shape)))
            acc += x[m] * np.exp(-2j * np.pi * ph)
        out[k] = acc
    return out


@pytest.mark.parametrize("shape", [(4, 8), (8, 8), (4, 4, 2)])
def test_fftn_equals_brute_force_dft(shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.allclose(np.fft.fftn(x), brute_dftn(x), atol=1e-9)


@pytest.mark.parametrize("shape,b", [((16, 32), (4, 8)), ((8, 16, 8), (2, 4, 4))])
def test_property2_nd_on_every_bucket(shape, b):
    """N-D Property 2: FFT_B(alias_nd(z)) = FFT_N(z) subsampled by L_d."""
    rng = np.random.default_rng(3)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    sub = np.fft.fftn(z)[tuple(slice(None, None, n // bb) for n, bb in zip(shape, b))]
    assert np.allclose(np.fft.fftn(R.alias_nd(z, b)), sub, atol=1e-9)


def test_stage1_probability_closed_forms():
    assert abs(R.stage1_probability(1e-3, 3, 3) - 0.1) < 1e-12
    assert abs(R.stage1_probability(1e-4, 3, 3) - 1e-4 ** (1 / 3)) < 1e-12
    p = R.stage1_probability(1e-3, 5, 1)
    assert abs(p - (1 - (1 - 1e-3) ** (1 / 5))) < 1e-12
    p = R.stage1_probability(1e-4, 7, 4)
    assert abs(stats.binom.sf(3, 7, p) - 1e-4) < 1e-14


def _plan(shape, b, T=3, atten=60.0, flat=None, pfa=1e-3, seed=0, mu=None):
    rng = np.random.default_rng(seed)
    sigma = synth.draw_sigma(rng, T, shape)
    return R.OraclePlan(shape, b, sigma, atten, flat, pfa, mu)


@pytest.mark.parametrize("shape,b", [((64, 128), (8, 16)), ((32, 16, 8), (4, 4, 2)),
                                     ((256,), (16,))])
def test_ongrid_tone_closed_form_rectangular(shape, b):
    """Rectangular pre-window and rectangular flat base: the flat window is an
    exact box, so a unit on-grid tone at cell i with amplitude a lands entirely
    in bucket M(i, sigma_s) with value a * prod(N_d), and every other bucket
    is 0 (Def. 1, 2, 3; Property 1, 2)."""
    plan = _plan(shape, b, atten=0.0, flat=0.0, seed=11)
    rng = np.random.default_rng(5)
    cell = tuple(int(rng.integers(0, n)) for n in shape)
    amp = 0.7 - 0.3j
    fr = np.array([[cell[d] / n for d, n in enumerate(shape)]])
    x = synth.synthesize(shape, fr, [list(cell)], [amp])
    N = int(np.prod(shape))
    for s in range(plan.T):
        fhat = R.rsft_round(x, plan, s)
        j = tuple(H.mapping(cell[d], plan.sigma[s, d], n, plan.B[d])
                  for d, n in enumerate(shape))
        expect = np.zeros(plan.B, dtype=np.complex128)
        expect[j] = amp * N
        assert np.max(np.abs(fhat - expect)) < 1e-9 * N


def test_claim1_peak_bucket_rectangular_prewindow():
    """Claim 1: with a symmetric (here rectangular) pre-window the largest
    bucket of an on-grid tone is p = floor(B/N [sigma i]_N), per dimension."""
    shape, b = (128, 64), (16, 8)
    rng = np.random.default_rng(8)
    for trial in range(40):
        plan = _plan(shape, b, atten=0.0, flat=60.0, seed=100 + trial)
        cell = [int(rng.integers(0, n)) for n in shape]
        fr = np.array([[cell[d] / n for d, n in enumerate(shape)]])
        x = synth.synthesize(shape, fr, [cell], [1.0])
        for s in range(plan.T):
            fhat = R.rsft_round(x, plan, s)
            got = np.unravel_index(np.argmax(np.abs(fhat)), plan.B)
            want = tuple(H.mapping(cell[d], plan.sigma[s, d], n, plan.B[d])
                         for d, n in enumerate(shape))
            assert tuple(int(g) for g in got) == want


def test_residue_fold_identity():
    """The literal round equals a fold of the unpermuted samples by residue
    class m mod B with weights w[m] wbar[[sigma^-1 m]_N], followed by the
    relabel b = (sigma^-1 mod B) c mod B: because B | N,
    [sigma^-1 m]_N mod B = ((sigma^-1 mod B)(m mod B)) mod B."""
    shape, b = (64, 32), (8, 4)
    plan = _plan(shape, b, seed=4)
    rng = np.random.default_rng(9)
    r = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for s in range(plan.T):
        lit = np.fft.ifftn(R.rsft_round(r, plan, s))
        acc = np.zeros(b, dtype=np.complex128)
        for m in itertools.product(*[range(n) for n in shape]):
            wgt = 1.0
            for d, n in enumerate(shape):
                wgt *= plan.w[d][m[d]] * plan.wbar[d][(plan.sigma_inv[s, d] * m[d]) % n]
            acc[tuple(m[d] % b[d] for d in range(2))] += wgt * r[m]
        tau = [int(plan.sigma_inv[s, d]) % b[d] for d in range(2)]
        relabeled = np.zeros(b, dtype=np.complex128)
        for c in itertools.product(*[range(v) for v in b]):
            relabeled[tuple((tau[d] * c[d]) % b[d] for d in range(2))] = acc[c]
        assert np.allclose(lit, relabeled, atol=1e-9)


def test_bucket_noise_law_and_stage1_pfa():
    """eq. alpha_beta: under white CN(0, sigma_n^2) noise every bucket of round
    s is CN(0, sigma_n^2 beta(sigma_s)) exactly, so |fhat|^2 is exponential
    (eq. exp) and P[|fhat|^2 >= gamma_s] = p1 (eq. tpd)."""
    shape, b = (64, 64), (8, 8)
    plan = _plan(shape, b, pfa=1e-3, seed=21)
    powers = [[] for _ in range(plan.T)]
    for f in range(300):
        r = synth.noise_only(shape, 77, f, dtype=np.complex128)
        for s in range(plan.T):
            powers[s].append(np.abs(R.rsft_round(r, plan, s)) ** 2)
    for s in range(plan.T):
        p = np.concatenate([v.ravel() for v in powers[s]])
        mean = p.mean() / plan.beta[s]
        assert abs(mean - 1.0) < 4.0 / math.sqrt(p.size)
        rate = np.mean(p >= plan.gamma[s])
        se = math.sqrt(plan.p1 * (1 - plan.p1) / p.size)
        assert abs(rate - plan.p1) < 4 * se
        # exponential law: the sample is consistent with Exp(beta)
        ks = stats.kstest(p / plan.beta[s], "expon")
        assert ks.pvalue > 1e-3


def test_votes_scatter_equals_gather():
    """eq. a_i accumulated by Definition 4 (scatter over R(j, sigma^-1)) equals
    abar_i = sum_s c_s[M(i, sigma_s)] (Definition 3) bit for bit."""
    for shape, b in [((64, 32), (8, 4)), ((16, 8, 32), (4, 2, 8)), ((128,), (16,))]:
        plan = _plan(shape, b, seed=len(shape))
        rng = np.random.default_rng(12)
        flags = rng.random((plan.T,) + plan.B) < 0.3
        abar = np.zeros(shape, dtype=np.int64)
        for s in range(plan.T):
            R.reverse_map_into(abar, flags[s], plan, s)
        assert np.array_equal(abar, R.votes_by_mapping(flags, plan))


def test_noise_free_tones_all_detected():
    """Noise-free strong on-grid tones with 60 dB windows: each round flags the
    tone's bucket, so by reversibility (Property 3) every true cell collects T
    votes and is detected; the detection set equals the brute-force
    {i : sum_s c_s[M(i, sigma_s)] >= mu}."""
    shape, b = (256, 256), (16, 16)
    plan = _plan(shape, b, pfa=1e-3, seed=31)
    meta = synth.make_frame("ongrid_256x256_c128", 0, noise=False)
    out = R.rsft(meta["frame"], plan)
    cells = [int(np.ravel_multi_index(tuple(int(round(f[d] * shape[d])) % shape[d]
                                            for d in range(2)), shape))
             for f in meta["freqs"]]
    assert set(cells) <= set(out["detections"].tolist())
    brute = np.flatnonzero(R.votes_by_mapping(out["flags"], plan) >= plan.mu)
    assert np.array_equal(brute, out["detections"])


def test_final_pfa_noise_only():
    """Final per-cell false-alarm rate under H0 with T = mu = 3 (same data,
    three permutations): design Pfa = 1e-3 via p1 = 0.1. False alarms come in
    bucket-sized clusters, so the confidence interval is computed over frames;
    the band allows 3 standard errors plus 3% for the correlation of the
    rounds, which all see the same noise samples."""
    shape, b = (256, 256), (16, 16)
    plan = _plan(shape, b, pfa=1e-3, seed=41)
    N = shape[0] * shape[1]
    rates = []
    for f in range(600):
        r = synth.noise_only(shape, 1234, f, dtype=np.complex128)
        rates.append(len(R.rsft(r, plan)["detections"]) / N)
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(len(rates))
    assert abs(rates.mean() - 1e-3) < 3 * se + 0.03e-3


def test_mu_below_T_votes():
    """mu < T: detection iff at least mu of the T buckets a cell maps to are
    flagged (second stage, Sec. III-C.5)."""
    shape, b = (64, 64), (8, 8)
    plan = _plan(shape, b, T=4, pfa=1e-3, seed=5, mu=2)
    r = synth.noise_only(shape, 3, 0, dtype=np.complex128)
    out = R.rsft(r, plan)
    votes = R.votes_by_mapping(out["flags"], plan)
    assert np.array_equal(np.flatnonzero(votes >= 2), out["detections"])
    assert np.array_equal(votes, out["votes"])


def test_estimated_noise_floor_unbiased():
    """The order-statistic noise floor is unbiased for exponential powers
    (Renyi representation): its mean over noise-only rounds equals
    sigma_n^2 beta(sigma_s) within 3 standard errors, and it is insensitive to
    a handful of strong tone buckets."""
    shape, b = (64, 64), (8, 8)
    plan = _plan(shape, b, pfa=1e-3, seed=23)
    est = []
    for f in range(400):
        r = synth.noise_only(shape, 91, f, dtype=np.complex128)
        est.append(R.estimated_noise_floor(R.rsft_round(r, plan, 0)) / plan.beta[0])
    est = np.array(est)
    assert abs(est.mean() - 1.0) < 3 * est.std(ddof=1) / math.sqrt(len(est))
    # exact closed form of the estimator on a known sample
    p = np.arange(1, 65, dtype=np.float64)
    H = sum(1.0 / (64 - i) for i in range(32))
    assert abs(R.estimated_noise_floor(np.sqrt(p)) - 32.0 / H) < 1e-12

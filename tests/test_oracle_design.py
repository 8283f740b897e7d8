"""Pins of the threshold-design oracle (eq. opt, Claims 2 and 3, eq. bpd):
the values printed in the captions of Figs. 6 and 7, the two Normal-tail
equations at the optimum, Remark 2's limit K eta_m >= B, and the ordering of
the bounds of Remark 3."""

import os

import numpy as np
import pytest

from oracle import design as DS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig6_fig7_design.txt")
N, B, T, K, ETA_M, PD, PFA = 1024, 64, 50, 4, 1.8, 0.9, 1e-6


@pytest.fixture(scope="module")
def ab():
    return DS.alpha_beta_bar((N,), (B,), 40.0, 40.0, (64.5,))


def _captions():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, snr, gamma, mu = line.split()
        rows[name] = (float(snr), float(gamma), float(mu))
    return rows


@pytest.mark.parametrize("bound", ["lower", "upper"])
def test_figure_captions(ab, bound):
    """SNR*_min within 1 dB, mu*/T within 0.1, and gamma* within 20% when
    read in units of N sigma_n^2 beta_bar (the captions' scale)."""
    snr_db, gamma_caption, mu_caption = _captions()[bound]
    a_bar, b_bar = ab
    out = DS.design(T, K, B, ETA_M, PD, PFA, a_bar, b_bar, bound=bound)
    assert abs(out["snr_min_db"] - snr_db) <= 1.0
    assert abs(out["mu"] / T - mu_caption) <= 0.1
    gamma_scaled = out["gamma"] / (b_bar * N)
    assert abs(gamma_scaled / gamma_caption - 1.0) <= 0.2


@pytest.mark.parametrize("bound", ["lower", "upper"])
def test_optimum_satisfies_both_tail_equations(ab, bound):
    a_bar, b_bar = ab
    out = DS.design(T, K, B, ETA_M, PD, PFA, a_bar, b_bar, bound=bound)
    pd, pfa = DS.stage2_tails(out["mu"], T, out["F"], out["eta_p"], out["pd_bar"], out["pfa_bar"])
    assert abs(pd - PD) < 1e-9
    assert abs(pfa / PFA - 1.0) < 1e-6
    # eq. bpd at SNR*: Pd_bar = Pfa_bar ** (beta / (alpha SNR + beta))
    expo = b_bar / (a_bar * out["snr_min"] + b_bar)
    assert abs(out["pfa_bar"] ** expo - out["pd_bar"]) < 1e-12


def test_remark2_limit(ab):
    """K eta_m >= B: the second stage cannot separate the hypotheses."""
    a_bar, b_bar = ab
    assert DS.design(T, 36, B, ETA_M, PD, PFA, a_bar, b_bar) is None     # 64.8 >= 64
    assert DS.design(T, 30, B, ETA_M, PD, PFA, a_bar, b_bar) is not None


def test_sparsity_and_bounds_order(ab):
    a_bar, b_bar = ab
    snrs = [DS.design(T, k, B, ETA_M, PD, PFA, a_bar, b_bar)["snr_min_db"] for k in (1, 4, 10, 20)]
    assert np.all(np.diff(snrs) > 0)
    lo = DS.design(T, K, B, ETA_M, PD, PFA, a_bar, b_bar, "lower")["snr_min_db"]
    hi = DS.design(T, K, B, ETA_M, PD, PFA, a_bar, b_bar, "upper")["snr_min_db"]
    assert hi > lo


def test_alpha_beta_closed_forms():
    """Rectangular windows: beta(sigma) = ||wbar||^2 = N L for every sigma
    (an exact box of L bins with passband gain N), and an on-grid tone gives
    alpha = N^2 at Claim 1's bucket."""
    n, b = 256, 16
    a, bb = DS.alpha_beta_one_dim(n, b, 0.0, 0.0, 37.0)
    assert np.allclose(bb, n * (n // b), rtol=1e-12)
    assert np.allclose(a, float(n) ** 2, rtol=1e-12)


def test_poisson_binomial_tail():
    """Equal probabilities give the binomial tail; a mixed set matches brute
    force over all 2^T outcomes."""
    from scipy import stats
    import itertools
    assert abs(DS.poisson_binomial_tail([0.3] * 20, 7) - stats.binom.sf(6, 20, 0.3)) < 1e-14
    probs = [0.1, 0.5, 0.9, 0.33, 0.2, 0.75]
    brute = 0.0
    for bits in itertools.product([0, 1], repeat=len(probs)):
        if sum(bits) >= 3:
            brute += np.prod([q if b else 1 - q for q, b in zip(probs, bits)])
    assert abs(DS.poisson_binomial_tail(probs, 3) - brute) < 1e-14


def test_stage1_detection_exponential_law():
    """Noise-only buckets (alpha SNR = 0) are flagged with probability p1;
    the tone's rate is the exponential survival exp(-gamma / mean)."""
    import math
    assert abs(DS.stage1_detection(3.0, 5.0, 0.0, 0.07) - 0.07) < 1e-15
    beta, alpha, snr, p1 = 9.0, 0.4, 12.0, 0.05
    gamma = beta * math.log(1 / p1)
    assert abs(DS.stage1_detection(alpha, beta, snr, p1) - math.exp(-gamma / (alpha * snr + beta))) < 1e-15


def _seg_plan(n, b, T, mu, p1, seed):
    import synth
    from oracle import rsft as R
    sigma = synth.draw_sigma(np.random.default_rng(seed), T, (n,))
    return R.OraclePlan((n,), (b,), sigma, 40.0, None, 1e-3, mu, 1.0, p1)


def test_exact_cell_rates_noise_only_and_tone_cell():
    """No tone: every cell has the binomial tail. One tone: its cell's rate
    equals the Poisson-binomial of eq. tpd with alpha_s, beta_s of Claim 1's
    bucket, computed through alpha_beta_one_dim."""
    from scipy import stats
    n, b, T, mu, p1 = 256, 16, 12, 4, 0.08
    plan = _seg_plan(n, b, T, mu, p1, 4)
    assert np.allclose(DS.exact_cell_rates(plan, [], p1), stats.binom.sf(mu - 1, T, p1), atol=1e-14)
    fb, snr = 37.5, 0.6
    rates = DS.exact_cell_rates(plan, [((fb,), snr)], p1)
    a, bb = DS.alpha_beta_one_dim(n, b, 40.0, 40.0, fb)
    probs = [DS.stage1_detection(a[(int(s) - 1) // 2], bb[(int(s) - 1) // 2], snr, p1)
             for s in plan.sigma[:, 0]]
    assert abs(rates[37] - DS.poisson_binomial_tail(probs, mu)) < 1e-12


def test_exact_cell_rates_monte_carlo():
    """The literal oracle in segment mode over 600 CPIs (Swerling-I tones in
    noise): the detection rate of the tone cell and the false-alarm count
    elsewhere agree with exact_cell_rates."""
    import math
    import synth
    from oracle import rsft as R
    n, b, T, mu, p1 = 256, 16, 10, 4, 0.08
    plan = _seg_plan(n, b, T, mu, p1, 9)
    tones = [((37.5,), 0.5), ((141.2,), 1.5)]
    rates = DS.exact_cell_rates(plan, tones, p1)
    rng = np.random.default_rng(33)
    m = np.arange(n)
    hits = 0
    counts = np.zeros(n)
    cpis = 600
    for _ in range(cpis):
        segs = []
        for s in range(T):
            x = synth.complex_noise(rng, (n,))
            for fb, snr in tones:
                x = x + synth.complex_noise(rng, (), snr) * np.exp(2j * np.pi * fb[0] * m / n)
            segs.append(x)
        det = R.rsft(np.stack(segs), plan, segments=True)["detections"]
        counts[det] += 1
    emp = counts / cpis
    se = np.sqrt(rates * (1 - rates) / cpis)
    assert abs(emp[37] - rates[37]) <= 3 * se[37] + 1e-12
    far = np.ones(n, dtype=bool)
    for c in (37, 141):
        far[[(c + o) % n for o in range(-3, 4)]] = False
    want = rates[far].sum() * cpis
    assert abs(counts[far].sum() - want) <= 5 * math.sqrt(want) + 0.1 * want

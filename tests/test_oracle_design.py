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

"""Pins of the oracle's off-grid estimate, dense (Bartlett) detector and the
complexity model."""

import math
import os

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import dense as Dn
from oracle import evaluate as E
from synth import scoring as S
from oracle import rsft as R
from oracle import windows as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_complexity_argmins_printed_in_paper():
    with open(os.path.join(GOLDEN, "complexity_argmin.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    cands = [8, 16, 32, 64, 128, 256, 512, 1024]
    for N, T, eta_m, eta_p, K, best in rows:
        got = E.best_buckets(int(N), int(T), int(K), float(eta_m), float(eta_p), cands)
        assert got == int(best)


def test_complexity_counts():
    # K=5, B=32: 50 * (1024 + 32 + 160 + 224) + 1024
    assert E.complexity_rsft(1024, 32, 50, 5, 1.4, 1.0) == pytest.approx(73024.0)
    assert E.complexity_bartlett(1024, 50) == 50 * 1024 * 11 + 1024


def _plan(shape, b, seed, atten=60.0):
    sigma = synth.draw_sigma(np.random.default_rng(seed), 3, shape)
    return R.OraclePlan(shape, b, sigma, atten, None, 1e-3)


def _dense_offset(X, cell, d):
    """Log-parabolic vertex along dimension d of a dense magnitude array."""
    shape = X.shape
    m = list(cell)
    p = list(cell)
    m[d] = (cell[d] - 1) % shape[d]
    p[d] = (cell[d] + 1) % shape[d]
    return R._log_parabola_offset(abs(X[tuple(m)]), abs(X[cell]), abs(X[tuple(p)]))


def test_ongrid_tone_offset_is_zero():
    """Symmetric window, on-grid tone: the windowed spectrum is symmetric about
    the tone's cell, so the interpolated offset is 0 up to the sidelobe and
    flat-window stopband leakage (<= -60 dB, i.e. ~1e-3 of the peak) that other
    bins add to the neighbours' buckets: below 2e-3 bin. A wrong neighbour,
    sign or gain correction gives errors of order 0.1 bin."""
    shape, b = (256, 256), (16, 16)
    plan = _plan(shape, b, 2)
    cell = (40, 201)
    fr = np.array([[cell[0] / 256, cell[1] / 256]])
    x = synth.synthesize(shape, fr, [list(cell)], [1.0 + 0j])
    bk = np.stack([R.rsft_round(x, plan, s) for s in range(3)])
    flat = np.ravel_multi_index(cell, shape)
    est = R.estimate([flat], bk, plan)[0]
    assert est["is_peak"]
    assert abs(est["freq"][0] * 256 - 40) < 2e-3
    assert abs(est["freq"][1] * 256 - 201) < 2e-3


def test_bucket_magnitude_matches_dense_spectrum():
    """In a clean round (see estimation_rounds) the gain-corrected bucket
    magnitude of a lone noise-free tone equals the dense windowed spectrum
    |DFT(W r)| at the tone's cell and its neighbours to within the flat
    window's ripple and stopband leakage (Claim 1 with the Estimation remark
    of Sec. III-C)."""
    shape, b = (1024, 1024), (64, 64)
    checked = 0
    for seed in range(3, 9):
        plan = _plan(shape, b, seed)
        fr = np.array([[0.3172, 0.7013]])
        x = synth.synthesize(shape, fr, None, [1.0 + 0j])
        X = Dn.windowed_spectrum(x, plan.w)
        gains = R.flat_window_gain(plan)
        c = tuple(int(round(f * n)) % n for f, n in zip(fr[0], shape))
        clean = R.estimation_rounds(plan)
        for s in clean:
            bk = np.zeros((plan.T,) + plan.B, dtype=np.complex128)
            bk[s] = R.rsft_round(x, plan, s)
            for dc in [(0, 0), (0, 1), (1, 0), (-1, 0), (0, -1)]:
                cell = ((c[0] + dc[0]) % shape[0], (c[1] + dc[1]) % shape[1])
                a = R.cell_magnitude(cell, bk, plan, gains, [s])
                # neighbours sit 5-15 dB below the peak, so the same absolute
                # leakage is a larger fraction of them
                tol = 0.02 if dc == (0, 0) else 0.05
                assert abs(a / abs(X[cell]) - 1.0) < tol
                checked += 1
    assert checked >= 10


def test_estimation_rounds_rule():
    """Clean rounds: every |[sigma k]_N| (k = 1, 2, circular) >= L + 2."""
    shape, b = (1024, 1024), (64, 64)
    plan = R.OraclePlan(shape, b, [[101, 301], [5, 301], [1023, 513]], 60, None, 1e-3)
    assert R.estimation_rounds(plan) == [0]
    plan = R.OraclePlan(shape, b, [[5, 301], [513, 301], [1023, 3]], 60, None, 1e-3)
    # no clean round; smallest distances minus (L + 2): round 0 has 5 - 18,
    # round 1 has [513*2]_1024 = 2 -> 2 - 18, round 2 has 1023 -> 1 - 18
    # (and 3 -> 3 - 18): the least contaminated is round 0
    assert R.estimation_rounds(plan) == [0]
    # eight rounds, the odd-numbered ones clean (|[sigma k]| >= 18 for k = 1, 2)
    # and the even-numbered ones not (sigma = 5 in dimension 0): every clean
    # round is used, however many there are
    sig = [[5, 301] if s % 2 == 0 else [101 + 2 * s, 301] for s in range(8)]
    plan = R.OraclePlan(shape, b, sig, 60, None, 1e-3)
    assert R.estimation_rounds(plan) == [1, 3, 5, 7]
    sig = [[101 + 2 * s, 301 + 2 * s] for s in range(12)]
    plan = R.OraclePlan(shape, b, sig, 60, None, 1e-3)
    assert R.estimation_rounds(plan) == list(range(12))


def test_noise_free_offgrid_estimate_matches_dense():
    """Noise-free single off-grid tone, 1024x1024, B=64x64: the bucket-based
    estimate agrees with the same interpolator applied to the dense windowed
    spectrum within 0.01 bin, and is within 0.02 bin of the truth (60 dB
    window). The interpolator's own bias on the dense spectrum is < 0.01 bin."""
    shape, b = (1024, 1024), (64, 64)
    rng = np.random.default_rng(17)
    for trial in range(5):
        plan = _plan(shape, b, 50 + trial)
        fr = rng.random((1, 2))
        x = synth.synthesize(shape, fr, None, [1.0 + 0j])
        bk = np.stack([R.rsft_round(x, plan, s) for s in range(3)])
        X = Dn.windowed_spectrum(x, plan.w)
        cell = tuple(int(round(f * n)) % n for f, n in zip(fr[0], shape))
        est = R.estimate([int(np.ravel_multi_index(cell, shape))], bk, plan)[0]
        assert est["is_peak"]
        for d in range(2):
            dense = ((cell[d] + _dense_offset(X, cell, d)) / shape[d]) % 1.0
            diff = (est["freq"][d] - dense + 0.5) % 1.0 - 0.5
            assert abs(diff * shape[d]) <= 0.01
            err = (est["freq"][d] - fr[0, d] + 0.5) % 1.0 - 0.5
            assert abs(err * shape[d]) <= 0.02
            derr = (dense - fr[0, d] + 0.5) % 1.0 - 0.5
            assert abs(derr * shape[d]) < 0.01


def test_dense_detector_exact_threshold():
    """Alg. 2 with T = 1: |uhat|^2 of a noise-only bin is exponential with mean
    sigma_n^2 ||w||^2, so the per-bin false-alarm rate equals Pfa."""
    shape = (64, 64)
    w = [W.dolph_chebyshev(64, 60)] * 2
    pfa = 1e-2
    cnt = 0
    tot = 0
    for f in range(200):
        r = synth.noise_only(shape, 5, f, dtype=np.complex128)
        det, x, thr = Dn.bartlett_detect(r, w, pfa)
        cnt += len(det)
        tot += x.size
    se = math.sqrt(pfa * (1 - pfa) / tot)
    # neighbouring windowed bins are correlated: allow 6 sigma
    assert abs(cnt / tot - pfa) < 6 * se


def test_bartlett_gamma_threshold_and_roc():
    """T segments: the exact Gamma(T) threshold gives Pfa on noise. eq.
    bartlettROC is the Normal approximation of the averaged statistic with the
    H1 bin variance SNR alpha' (noise neglected under H1, Appendix A); under
    that same model a Monte Carlo Pd at T=40 agrees within 0.03."""
    T = 40
    rng = np.random.default_rng(0)
    beta_p = 1.0
    pfa = 1e-3
    thr = stats.gamma.isf(pfa, T, scale=beta_p)
    noise = rng.exponential(beta_p, size=(200000, T)).sum(axis=1)
    assert abs(np.mean(noise >= thr) - pfa) < 4 * math.sqrt(pfa / 200000)
    alpha_p = 1.0
    z = stats.norm.isf(pfa)
    gamma_n = beta_p * (1.0 + z / math.sqrt(T))     # Normal-approximation threshold
    for snr in (1.3, 1.5, 1.8):
        sig = rng.exponential(snr * alpha_p, size=(100000, T)).mean(axis=1)
        pd_mc = np.mean(sig >= gamma_n)
        pd_cf = Dn.bartlett_roc_pd(pfa, T, snr, alpha_p, beta_p)
        assert abs(pd_mc - pd_cf) < 0.03


def _erlang_survival(x, T):
    """P[Gamma(T, 1) >= x] for integer T: exp(-x) sum_{k<T} x^k / k! (the
    Poisson sum identity of the Erlang law, written out)."""
    term = 1.0
    acc = 1.0
    for k in range(1, T):
        term *= x / k
        acc += term
    return math.exp(-x) * acc


def test_bartlett_detect_threshold_is_erlang_quantile():
    """Alg. 2 over T segments (Appendix A): a noise-only bin of the summed
    statistic is a sum of T independent exponentials of mean
    sigma_n^2 ||w||^2, so the threshold bartlett_detect returns must sit where
    the Erlang(T) survival function equals Pfa (closed form, no quantile
    routine involved)."""
    shape = (8, 8)
    w = [W.dolph_chebyshev(8, 60)] * 2
    zeta2 = 2.5 * Dn.window_energy(w)
    for T in (2, 3, 5, 10):
        for pfa in (1e-2, 1e-4, 1e-6):
            segs = [np.zeros(shape, np.complex128)] * T
            _, _, thr = Dn.bartlett_detect(segs, w, pfa, noise_var=2.5)
            assert abs(_erlang_survival(thr / zeta2, T) - pfa) <= 1e-9 * pfa


def test_bartlett_detect_two_segment_sum_by_hand():
    """Two segments on a 4x4 grid with rectangular windows: segment 0 is a
    unit impulse at the origin (flat spectrum 1 on every bin), segment 1 the
    on-grid tone 3 exp(j 2 pi (m0 + 2 m1) / 4) (16 * 3 on bin (1, 2), zero
    elsewhere). The summed statistic is 1 + 48^2 on bin (1, 2) and 1
    elsewhere; with sigma_n^2 = 0.1 and ||w||^2 = 16 the Pfa = 1e-3 threshold
    lies between, so exactly that bin is detected."""
    shape = (4, 4)
    w = [np.ones(4)] * 2
    r0 = np.zeros(shape, np.complex128)
    r0[0, 0] = 1.0
    m0, m1 = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    r1 = 3.0 * np.exp(2j * np.pi * (m0 + 2 * m1) / 4)
    det, x, thr = Dn.bartlett_detect([r0, r1], w, 1e-3, noise_var=0.1)
    want = np.ones(shape)
    want[1, 2] += 48.0 ** 2
    assert np.allclose(x, want, rtol=0, atol=1e-9)
    assert 1.0 < thr < want[1, 2]
    assert list(det) == [int(np.ravel_multi_index((1, 2), shape))]


def test_bartlett_detect_empirical_pfa_over_segments():
    """Noise-only input split into T = 4 independent segments: the per-bin
    false-alarm rate of bartlett_detect's summed statistic matches the design
    Pfa = 1e-2. Bins of one frame are correlated by the window, so the
    standard error is taken over frames."""
    shape = (64, 64)
    w = [W.dolph_chebyshev(64, 60)] * 2
    pfa, T, frames = 1e-2, 4, 160
    rates = []
    for f in range(frames):
        segs = [synth.noise_only(shape, 11 + s, f, dtype=np.complex128) for s in range(T)]
        det, x, _ = Dn.bartlett_detect(segs, w, pfa)
        rates.append(len(det) / x.size)
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(frames)
    assert abs(rates.mean() - pfa) < 4 * se + 1e-4


def test_pd_pfa_scoring():
    shape = (64, 64)
    freqs = np.array([[10 / 64, 20 / 64], [40.4 / 64, 5.2 / 64]])
    det = [np.ravel_multi_index((11, 21), shape),     # inside guard of tone 0
           np.ravel_multi_index((30, 30), shape)]     # false alarm
    hits, K, fa, outside = S.pd_pfa(det, freqs, shape, guard=3)
    assert (hits, K, fa) == (1, 2, 1)
    assert outside == 64 * 64 - 2 * 49

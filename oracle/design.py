"""FP64 oracle of the optimal threshold design (test infrastructure only).

Section IV-C: the first stage flags a bucket when |fhat|^2 >= gamma; averaged
over the permutation, its false-alarm and detection probabilities are
(eq. bpd)
    Pfa_bar = exp(-gamma / (sigma_n^2 beta_bar)),
    Pd_bar  = Pfa_bar ** (beta_bar / (alpha_bar SNR + beta_bar)),
with alpha(p, sigma, omega) = |u_p^H V_sigma v(omega)|^2 and
beta(sigma) = ||Wbar P_sigma w||^2 (eq. alpha_beta), p the bucket of Claim 1.
The second stage counts the T flags a cell collects; asymptotically (Claims
2 and 3, with the variance upper bounds) the count is Normal with
    H1: mean T Pd_bar, variance T Pd_bar (1 - Pd_bar)
    H0: mean F eta_p Pd_bar + (T - F) Pfa_bar,
        variance F eta_p Pd_bar (1 - eta_p Pd_bar) + (T - F) Pfa_bar (1 - Pfa_bar),
    F = T K eta_m / B.
eq. opt: for each second-stage threshold mu, the two Normal tails fix Pd_bar
(from the target Pd) and Pfa_bar (from the target Pfa); eq. bpd then gives
the SNR the weakest tone needs; the minimum over mu is SNR*_min, attained at
mu*, and gamma* = -sigma_n^2 beta_bar ln Pfa_bar. eta_p = 1 gives the lower
and eta_p = 1 / Pd_bar the upper bound of Remark 3.

Readings (the paper leaves them open): mu ranges over 1..T and a cell is
declared when its count is >= mu; the expectations over sigma are plain
averages over all odd sigma in [1, N) (uniform permutations); in D
dimensions alpha and beta are products over dimensions of independent
per-dimension permutations, so their averages are products of the
per-dimension averages.
"""

import math

import numpy as np

from . import rsft as _rsft


def _normal_tail(z):
    """P[Z >= z] for a standard Normal Z."""
    return 0.5 * math.erfc(z / math.sqrt(2.0))


def alpha_beta_one_dim(n, b, window_atten_db, flat_atten_db, omega_bins):
    """(alpha(p, sigma, omega), beta(sigma)) for every odd sigma in [1, n): the
    literal round of Algorithm 1 applied to v(omega) = exp(j omega m), omega
    = omega_bins * 2 pi / n, read at Claim 1's bucket
    p = floor(B/N [sigma floor(omega / dw)]_N)."""
    m = np.arange(n, dtype=np.float64)
    v = np.exp(2j * np.pi * omega_bins * m / n)
    k0 = int(math.floor(omega_bins))
    alphas, betas = [], []
    for sigma in range(1, n, 2):
        plan = _rsft.OraclePlan((n,), (b,), [[sigma]], window_atten_db, flat_atten_db)
        fhat = _rsft.rsft_round(v, plan, 0)
        p = ((sigma * k0) % n) * b // n
        alphas.append(abs(fhat[p]) ** 2)
        betas.append(plan.beta[0])
    return np.array(alphas), np.array(betas)


def alpha_beta_bar(shape, buckets, window_atten_db, flat_atten_db, omega_bins):
    """(alpha_bar, beta_bar): products over dimensions of the per-dimension
    averages over sigma."""
    a_bar, b_bar = 1.0, 1.0
    for d, (n, b) in enumerate(zip(shape, buckets)):
        a, bb = alpha_beta_one_dim(n, b, window_atten_db, flat_atten_db, omega_bins[d])
        a_bar *= float(np.mean(a))
        b_bar *= float(np.mean(bb))
    return a_bar, b_bar


def _bisect_increasing(fun, lo, hi, target, iters=200):
    """x in [lo, hi] with fun(x) = target for an increasing fun."""
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if fun(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def stage2_tails(mu, T, F, eta_p, pd_bar, pfa_bar):
    """(Pd, Pfa) of the second stage at threshold mu: the Normal tails of
    Claims 2 and 3 with the variance upper bounds."""
    m1 = T * pd_bar
    v1 = T * pd_bar * (1.0 - pd_bar)
    m0 = F * eta_p * pd_bar + (T - F) * pfa_bar
    v0 = F * eta_p * pd_bar * (1.0 - eta_p * pd_bar) + (T - F) * pfa_bar * (1.0 - pfa_bar)
    pd = _normal_tail((mu - m1) / math.sqrt(v1)) if v1 > 0 else float(m1 >= mu)
    pfa = _normal_tail((mu - m0) / math.sqrt(v0)) if v0 > 0 else float(m0 >= mu)
    return pd, pfa


def design(T, K, B, eta_m, pd, pfa, alpha_bar, beta_bar, bound="lower", noise_var=1.0):
    """eq. opt. Returns a dict (snr_min, snr_min_db, mu, pd_bar, pfa_bar,
    gamma, F, eta_p), or None when no mu in 1..T meets both targets (e.g.
    K eta_m >= B, Remark 2)."""
    F = T * K * eta_m / B
    best = None
    for mu in range(1, T + 1):
        pd_bar = _bisect_increasing(
            lambda x: stage2_tails(mu, T, F, 1.0, x, 0.0)[0], 1e-15, 1.0 - 1e-15, pd)
        eta_p = 1.0 if bound == "lower" else 1.0 / pd_bar
        if F >= T:
            continue
        if stage2_tails(mu, T, F, eta_p, pd_bar, 1e-300)[1] > pfa:
            continue                              # the co-existing tones alone exceed Pfa
        pfa_bar = _bisect_increasing(
            lambda y: stage2_tails(mu, T, F, eta_p, pd_bar, y)[1], 1e-300, 1.0 - 1e-15, pfa)
        if not pfa_bar < pd_bar:
            continue
        snr = beta_bar * (math.log(pfa_bar) / math.log(pd_bar) - 1.0) / alpha_bar
        if best is None or snr < best["snr_min"]:
            best = {"snr_min": snr, "mu": mu, "pd_bar": pd_bar, "pfa_bar": pfa_bar, "F": F,
                    "eta_p": eta_p}
    if best is None:
        return None
    best["snr_min_db"] = 10.0 * math.log10(best["snr_min"])
    best["gamma"] = -noise_var * beta_bar * math.log(best["pfa_bar"])
    return best


def stage1_detection(alpha, beta, snr, p1):
    """eq. tpd for one round: with gamma = sigma_n^2 beta ln(1/p1), a bucket
    holding the tone (|fhat|^2 exponential with mean sigma_n^2 (alpha SNR +
    beta)) is flagged with probability p1 ** (beta / (alpha SNR + beta))."""
    return p1 ** (beta / (alpha * snr + beta))


def poisson_binomial_tail(probs, mu):
    """P[sum of independent Bernoulli(probs[s]) >= mu] by dynamic programming
    over the rounds (the exact law of the vote count of eq. a_i when the
    rounds see independent data)."""
    dist = np.zeros(len(probs) + 1)
    dist[0] = 1.0
    for q in probs:
        dist[1:] = dist[1:] * (1.0 - q) + dist[:-1] * q
        dist[0] *= 1.0 - q
    return float(dist[mu:].sum())


def exact_cell_rates(plan, tones, p1, noise_var=1.0):
    """Per-cell probability of >= mu votes in segment mode (round s on its
    own data segment) for a frame of K tones, tones = [(freq_bins [D],
    snr)], with Swerling-I amplitudes drawn independently per segment and
    CN(0, noise_var) noise, at thresholds gamma_s = noise_var beta_s ln(1/p1).
    Round s's bucket j is a sum of independent circular Gaussians, so its
    power is exponential with mean noise_var (beta_s + sum_t snr_t A_{s,t}[j])
    (A_{s,t}: the bucket powers of the unit tone t through the literal
    round), and it is flagged with probability p1 ** (beta_s / (beta_s +
    sum_t snr_t A_{s,t}[j])) (eq. exp, eq. tpd), independently across rounds;
    a cell collects the flags of its buckets M(i, sigma_s) (Def. 3), so its
    count is Poisson-binomial. Returns an array of the plan's shape."""
    T = plan.T
    q = []
    for s in range(T):
        mean = np.full(plan.B, plan.beta[s], dtype=np.float64)
        for fb, snr in tones:
            freq = np.asarray(fb, dtype=np.float64) / np.asarray(plan.shape, dtype=np.float64)
            v = np.ones((), dtype=np.complex128)
            for d, n in enumerate(plan.shape):
                v = np.multiply.outer(v, np.exp(2j * np.pi * freq[d] * np.arange(n)))
            mean = mean + snr * np.abs(_rsft.rsft_round(v, plan, s)) ** 2 / noise_var
        flag = p1 ** (plan.beta[s] / mean)
        idx = [((int(plan.sigma[s, d]) * np.arange(n, dtype=np.int64)) % n) // plan.L[d]
               for d, n in enumerate(plan.shape)]
        q.append(flag[np.ix_(*idx)])
    dist = np.zeros((T + 1,) + plan.shape)
    dist[0] = 1.0
    for qs in q:
        dist[1:] = dist[1:] * (1.0 - qs) + dist[:-1] * qs
        dist[0] = dist[0] * (1.0 - qs)
    return dist[plan.mu:].sum(axis=0)

"""Algorithm 1 (RSFT) in FP64, literally, for any fixed dimension (oracle;
test infrastructure only).

Every step follows the paper's order and notation:

  y <- W r                    pre-permutation windowing (Alg. 1; Sec. III-A)
  p <- P_{sigma,0} y          permutation per dimension (Def. 1; Sec. III-C.2)
  z <- Wbar p                 flat windowing (Sec. IV-B)
  f <- Aliasing(z)            per dimension, period B_d (Def. 2; Sec. III-C.3)
  fhat <- NDFFT(f)            B-point N-D FFT (eq. f)
  c <- |fhat|^2 >= gamma      first-stage NP detection (eq. exp, eq. tpd)
  a_s <- Reverse(c)           reverse mapping (Def. 4; Sec. III-C.4)
  abar <- abar + a_s          accumulation (eq. a_i)
  o <- abar >= mu             second-stage detection (Sec. III-C.5)

Readings where the paper is silent or ambiguous:
exactly T rounds on the same data with different sigma; detection means
``>=`` at both stages; mu in {1..T}; the first-stage threshold of round s is
gamma_s = sigma_n^2 beta(sigma_s) ln(1/p1) with p1 solving the exact binomial
tail P[Bin(T, p1) >= mu] = Pfa (per-round beta of eq. tpd, not the
sigma-average of eq. bpd; exact binomial because T is small).
"""

import math

import numpy as np

from . import hashing
from . import windows


def stage1_probability(pfa, T, mu):
    """p1 such that P[Binomial(T, p1) >= mu] = pfa, by bisection (FP64).

    Under H0 each of the T first-stage flags a cell sees is Bernoulli(p1)
    (Sec. IV-C); the cell is declared when at least mu of them are set."""
    if not (0.0 < pfa < 1.0):
        raise ValueError("pfa must be in (0, 1)")
    if not (1 <= mu <= T):
        raise ValueError("mu must be in 1..T")

    def tail(p):
        return sum(math.comb(T, c) * p ** c * (1.0 - p) ** (T - c)
                   for c in range(mu, T + 1))

    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tail(mid) < pfa:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


class OraclePlan:
    """Parameters of one RSFT configuration (Problem 1: signal dims, windows,
    buckets, permutations, Pfa), with everything derived from them in FP64."""

    def __init__(self, shape, buckets, sigma, window_atten_db=60.0,
                 flat_atten_db=None, pfa=1e-3, mu=None, noise_var=1.0, stage1_pfa=None):
        self.shape = tuple(int(n) for n in shape)
        self.B = tuple(int(b) for b in buckets)
        self.D = len(self.shape)
        if len(self.B) != self.D:
            raise ValueError("one bucket count per dimension")
        for n, b in zip(self.shape, self.B):
            if n & (n - 1) or b & (b - 1) or not (1 <= b < n):
                raise ValueError("N_d, B_d must be powers of two, 1 <= B_d < N_d")
        self.L = tuple(n // b for n, b in zip(self.shape, self.B))
        self.sigma = np.asarray(sigma, dtype=np.int64).reshape(-1, self.D)
        self.T = self.sigma.shape[0]
        self.mu = self.T if mu is None else int(mu)
        self.sigma_inv = np.array(
            [[hashing.mod_inverse(self.sigma[s, d], self.shape[d])
              for d in range(self.D)] for s in range(self.T)], dtype=np.int64)
        if flat_atten_db is None or flat_atten_db < 0:
            flat_atten_db = window_atten_db
        self.window_atten_db = float(window_atten_db)
        self.flat_atten_db = float(flat_atten_db)
        self.w = [windows.dolph_chebyshev(n, window_atten_db) for n in self.shape]
        self.wbar = [windows.flat_window(n, b, flat_atten_db)
                     for n, b in zip(self.shape, self.B)]
        self.noise_var = float(noise_var)
        self.pfa = float(pfa)
        # first-stage false-alarm probability: given directly (e.g. from the
        # design of eq. opt), or from the final Pfa by the exact binomial
        self.p1 = (float(stage1_pfa) if stage1_pfa is not None
                   else stage1_probability(self.pfa, self.T, self.mu))
        self.beta = np.array([self.beta_of_round(s) for s in range(self.T)])
        # eq. tpd: Pfa~(sigma_s) = exp(-gamma / (sigma_n^2 beta(sigma_s))) = p1
        self.gamma = self.noise_var * self.beta * math.log(1.0 / self.p1)

    def permutation_indices(self, s):
        """Per-dimension gather indices [sigma_{s,d} n]_{N_d} (Def. 1, tau=0)."""
        return [(int(self.sigma[s, d]) * np.arange(n, dtype=np.int64)) % n
                for d, n in enumerate(self.shape)]

    def beta_of_round(self, s):
        """eq. alpha_beta: beta(sigma_s) = || Wbar P_{sigma_s} w ||^2, with the
        N-D windows formed as outer products and permuted per dimension."""
        w_nd = windows.nd_window(self.w)
        wbar_nd = windows.nd_window(self.wbar)
        permuted = w_nd[np.ix_(*self.permutation_indices(s))]
        return float(np.sum(np.abs(wbar_nd * permuted) ** 2))


def alias_nd(z, buckets):
    """Definition 2 applied along every dimension: periodic extension with
    period B_d, keep the basic period (Sec. III-C.3)."""
    f = np.asarray(z)
    for d, b in enumerate(buckets):
        n = f.shape[d]
        L = n // b
        new_shape = f.shape[:d] + (L, b) + f.shape[d + 1:]
        f = f.reshape(new_shape).sum(axis=d)
    return f


def rsft_round(r, plan, s):
    """Steps of one iteration of Algorithm 1 up to the B-point N-D FFT.
    Returns fhat_s (complex128, shape B)."""
    r = np.asarray(r, dtype=np.complex128)
    y = r * windows.nd_window(plan.w)                       # y <- W r
    p = y[np.ix_(*plan.permutation_indices(s))]             # p <- P_{sigma,0} y
    z = p * windows.nd_window(plan.wbar)                    # z <- Wbar p
    f = alias_nd(z, plan.B)                                 # f <- Aliasing(z)
    return np.fft.fftn(f)                                   # fhat <- NDFFT(f)


def estimated_noise_floor(fhat):
    """Noise floor sigma_n^2 beta(sigma_s) of one round estimated from the
    round's own buckets (for when sigma_n^2 is unknown; the paper assumes it
    known). Under H0 the B powers |fhat|^2 are exponential with that mean
    (eq. exp); by the Renyi representation of exponential order statistics
    E[X_(h)] = mean * sum_{i<h} 1/(B - i), so with h = B/2 (the lower median,
    insensitive to the few buckets holding tones) X_(h) / sum_{i<h} 1/(B - i)
    is unbiased."""
    p = np.sort(np.abs(np.asarray(fhat)).ravel() ** 2)
    B = p.size
    h = max(B // 2, 1)
    H = sum(1.0 / (B - i) for i in range(h))
    return p[h - 1] / H


def reverse_map_into(abar, flags, plan, s):
    """Reverse mapping + accumulation of one round (Def. 4, eq. a_i): every
    flagged bucket j adds one vote to each cell of R(j, sigma_s^{-1}), formed
    per dimension and combined as a Cartesian product (Sec. III-C.4)."""
    for j in np.argwhere(flags):
        sets = [hashing.reverse_mapping(int(j[d]), int(plan.sigma_inv[s, d]),
                                        plan.shape[d], plan.B[d])
                for d in range(plan.D)]
        abar[np.ix_(*sets)] += 1


def rsft(r, plan, noise="known", segments=False):
    """Algorithm 1. Returns a dict with the per-round buckets fhat_s, the
    first-stage flags c_s, the thresholds used, the accumulated votes abar and
    the detections o (row-major flat cell indices, ascending). noise="known"
    uses gamma_s = sigma_n^2 beta(sigma_s) ln(1/p1); "estimated" replaces
    sigma_n^2 beta(sigma_s) by estimated_noise_floor of the round.
    segments=True: r holds T data segments [T, *shape] and round s processes
    segment s (the T segments of the signal model, Sec. IV-A)."""
    buckets = []
    flags = []
    gammas = []
    abar = np.zeros(plan.shape, dtype=np.int64)
    if segments and np.shape(r)[0] != plan.T:
        raise ValueError("segment mode needs T segments")
    for s in range(plan.T):
        fhat = rsft_round(r[s] if segments else r, plan, s)
        if noise == "known":
            gamma = plan.gamma[s]
        else:
            gamma = estimated_noise_floor(fhat) * math.log(1.0 / plan.p1)
        gammas.append(gamma)
        c = np.abs(fhat) ** 2 >= gamma                      # NPdet1
        reverse_map_into(abar, c, plan, s)                  # Reverse + accumulate
        buckets.append(fhat)
        flags.append(c)
    o = np.flatnonzero(abar >= plan.mu)                     # NPdet2
    return {"buckets": np.stack(buckets), "flags": np.stack(flags),
            "gamma": np.array(gammas), "votes": abar, "detections": o}


def votes_by_mapping(flags, plan):
    """The same accumulation written from Definition 3 instead of 4:
    abar_i = sum_s c_s[M(i, sigma_s)], evaluated for every cell. Equal to the
    reverse-mapping form by Properties 3-4."""
    abar = np.zeros(plan.shape, dtype=np.int64)
    for s in range(plan.T):
        idx = [((int(plan.sigma[s, d]) * np.arange(n, dtype=np.int64)) % n)
               * plan.B[d] // n for d, n in enumerate(plan.shape)]
        abar += flags[s][np.ix_(*idx)].astype(np.int64)
    return abar


def flat_window_gain(plan):
    """|DFT_N(wbar_d)[-t]| / N_d for t in [0, L_d): the flat window's response
    at offset -t from a bucket's first bin (Sec. IV-B), per dimension."""
    gains = []
    for d, n in enumerate(plan.shape):
        g = np.fft.fft(plan.wbar[d])
        t = np.arange(plan.L[d])
        gains.append(np.abs(g[(-t) % n]) / n)
    return gains


def estimation_rounds(plan):
    """Rounds whose buckets are used for magnitude estimates (a choice of this
    estimator; the paper has none).

    A tone's main lobe covers its cell and the bins k = 1, 2 away. Round s
    permutes bin offset k to [sigma_{s,d} k]_{N_d}; when that lands within
    L_d + 2 permuted bins of 0 (circularly) for some dimension d and k in
    {1, 2}, neighbouring main-lobe bins of one tone share a bucket (or its
    transition band) and the bucket no longer measures a single cell. A round
    is clean when that happens for no d and k. Every clean round is used
    (each is an independent measurement of the cell); if none is clean, the
    single round whose smallest such distance (minus L_d + 2) is largest, the
    first on ties."""
    scores = []
    for s in range(plan.T):
        worst = None
        for d, n in enumerate(plan.shape):
            for k in (1, 2):
                u = (int(plan.sigma[s, d]) * k) % n
                dist = min(u, n - u) - (plan.L[d] + 2)
                worst = dist if worst is None else min(worst, dist)
        scores.append(worst)
    clean = [s for s in range(plan.T) if scores[s] >= 0]
    if clean:
        return clean
    best = max(scores)
    return [scores.index(best)]


def cell_magnitude(cell, buckets, plan, gains, rounds=None):
    """Gain-corrected magnitude of grid cell `cell` (tuple of indices):
    A_s = |fhat_s[M(cell, sigma_s)]| / prod_d gain_d[t_d], where the cell's
    permuted bin is u_d = [sigma_{s,d} cell_d], its bucket j_d = floor(u_d / L_d)
    (Def. 3) and t_d = u_d - j_d L_d; then the median over the estimation
    rounds. The bucket divided by the flat-window response estimates the
    pre-windowed spectrum |DFT(W r)| at the cell (Sec. III-C, the Estimation
    remark; Claim 1)."""
    if rounds is None:
        rounds = estimation_rounds(plan)
    vals = []
    for s in rounds:
        j = []
        g = 1.0
        for d, n in enumerate(plan.shape):
            u = (int(plan.sigma[s, d]) * int(cell[d])) % n
            jd = u // plan.L[d]
            g *= gains[d][u - jd * plan.L[d]]
            j.append(jd)
        vals.append(abs(buckets[s][tuple(j)]) / g)
    return float(np.median(vals))


def _log_parabola_offset(am, a0, ap):
    """Vertex of the parabola through (-1, ln am), (0, ln a0), (1, ln ap),
    clamped to [-1/2, 1/2]; 0 when the three points are not concave."""
    tiny = 1e-300
    lm, l0, lp = (math.log(max(v, tiny)) for v in (am, a0, ap))
    den = 2.0 * l0 - lm - lp
    if not den > 0.0:
        return 0.0
    return min(0.5, max(-0.5, 0.5 * (lp - lm) / den))


def estimate(detections, buckets, plan):
    """Off-grid estimate for each detected cell (flat indices, ascending).

    The paper recovers gridded locations only (Sec. I) and divides bucket
    values by the window spectrum for estimation (Sec. III-C). This estimate
    is defined here: magnitudes A from ``cell_magnitude`` over the rounds of
    ``estimation_rounds``; a cell is a peak
    when A exceeds every grid neighbour (3^D - 1, circular) with a lower
    row-major index and is >= every neighbour with a higher one; per
    dimension, the offset is the vertex of a parabola through the log
    magnitudes of the cell and its two neighbours along that dimension;
    frequency = (index + offset) / N_d cycles/sample, wrapped to [0, 1).

    Returns a list of dicts (cell, magnitude, is_peak, freq)."""
    gains = flat_window_gain(plan)
    rounds = estimation_rounds(plan)
    shape = plan.shape
    cache = {}

    def A(cell):
        if cell not in cache:
            cache[cell] = cell_magnitude(cell, buckets, plan, gains, rounds)
        return cache[cell]

    offsets = [o for o in np.ndindex(*([3] * plan.D)) if any(v != 1 for v in o)]
    out = []
    for flat in detections:
        cell = np.unravel_index(int(flat), shape)
        cell = tuple(int(v) for v in cell)
        a0 = A(cell)
        peak = True
        for o in offsets:
            nb = tuple((cell[d] + o[d] - 1) % shape[d] for d in range(plan.D))
            nflat = int(np.ravel_multi_index(nb, shape))
            if nflat == int(flat):
                continue
            an = A(nb)
            if nflat < int(flat):
                if not a0 > an:
                    peak = False
            else:
                if not a0 >= an:
                    peak = False
        freq = []
        for d in range(plan.D):
            minus = list(cell)
            plus = list(cell)
            minus[d] = (cell[d] - 1) % shape[d]
            plus[d] = (cell[d] + 1) % shape[d]
            delta = _log_parabola_offset(A(tuple(minus)), a0, A(tuple(plus)))
            freq.append(((cell[d] + delta) / shape[d]) % 1.0)
        out.append({"cell": int(flat), "magnitude": a0, "is_peak": peak,
                    "freq": freq})
    return out

"""FP64 oracle of the bucketized forward model used for off-grid refinement
(test infrastructure only).

The round-s buckets of a frame (eq. f) are linear in the signal. For a sum of
complex tones r[m] = sum_t b_t exp(j 2 pi f_t . m) with continuous
frequencies f_t (cycles/sample per dimension; the signal model of eq.
sig_model / eq. sinusoid with v(omega) of eq. f_k) they are therefore

    model_s = sum_t b_t * Round_s(v(f_t)),

where Round_s is the literal round of Algorithm 1 (window, permutation, flat
window, aliasing, B-point DFT; ``rsft.rsft_round``) and v(f)[m] =
exp(j 2 pi f . m). Derivatives follow from the same linearity:

    d model_s / d f_{t,d} = b_t * Round_s(j 2 pi m_d v(f_t))
    d model_s / d b_t     = Round_s(v(f_t))

For a real loss L and the model's complex outputs z with
G = dL/dRe z + j dL/dIm z (the gradient convention of PyTorch):

    dL/dRe b_t + j dL/dIm b_t = sum_{s,k} G_s[k] conj(Round_s(v(f_t))[k])
    dL/df_{t,d} = Re sum_{s,k} conj(G_s[k]) d model_s[k] / d f_{t,d}.

Everything here is written from these definitions with numpy in FP64. The
gradient functions synthesize the tone on the full grid and push it through
the oracle's own round, so nothing is factored or reordered there. The
refinement below (per-tone trust-region Gauss-Newton, and the initial
amplitudes of detected tones) evaluates the same model per dimension
(``factored_round_buckets``, the separability of tone and round), which the
tests pin against the full-grid form.
"""

import math

import numpy as np

from . import rsft as _rsft


def tone_signal(shape, freq):
    """v(f)[m] = exp(j 2 pi sum_d f_d m_d) on the full grid (FP64)."""
    out = np.ones((), dtype=np.complex128)
    for d, n in enumerate(shape):
        m = np.arange(n, dtype=np.float64)
        e = np.exp(2j * np.pi * float(freq[d]) * m)
        out = np.multiply.outer(out, e)
    return out


def tone_derivative_signal(shape, freq, dim):
    """d v(f) / d f_dim = j 2 pi m_dim v(f)."""
    v = tone_signal(shape, freq)
    m = np.arange(shape[dim], dtype=np.float64)
    expand = [1] * len(shape)
    expand[dim] = shape[dim]
    return 2j * np.pi * m.reshape(expand) * v


def round_buckets(x, plan):
    """All T rounds of Algorithm 1's bucketization of x: [T, *B]."""
    return np.stack([_rsft.rsft_round(x, plan, s) for s in range(plan.T)])


def model(freqs, amps, plan):
    """model_s[k] = sum_t b_t Round_s(v(f_t))[k]; freqs [K][D], amps [K]."""
    x = np.zeros(plan.shape, dtype=np.complex128)
    for f, b in zip(freqs, amps):
        x = x + complex(b) * tone_signal(plan.shape, f)
    return round_buckets(x, plan)


def loss(freqs, amps, plan, observed):
    """sum_{s,k} |model_s[k] - observed_s[k]|^2."""
    r = model(freqs, amps, plan) - observed
    return float(np.sum(np.abs(r) ** 2))


def gradients(freqs, amps, plan, grad_model, tones=None):
    """Analytic gradients for the output gradient grad_model [T, *B]
    (G = dL/dRe z + j dL/dIm z). Returns (grad_freqs [K][D] real,
    grad_amps [K] complex in the same convention). `tones` restricts the
    computation to a subset (others are left 0)."""
    K = len(freqs)
    D = len(plan.shape)
    gf = np.zeros((K, D))
    ga = np.zeros(K, dtype=np.complex128)
    for t in (range(K) if tones is None else tones):
        basis = round_buckets(tone_signal(plan.shape, freqs[t]), plan)
        ga[t] = np.sum(grad_model * np.conj(basis))
        for d in range(D):
            dbasis = round_buckets(tone_derivative_signal(plan.shape, freqs[t], d), plan)
            gf[t, d] = float(np.real(np.sum(np.conj(grad_model) * complex(amps[t]) * dbasis)))
    return gf, ga


def loss_gradients(freqs, amps, plan, observed, tones=None):
    """Gradients of ``loss``: its output gradient is G = 2 (model - observed)."""
    g = 2.0 * (model(freqs, amps, plan) - observed)
    return gradients(freqs, amps, plan, g, tones)


def gauss_newton_steps(freqs, amps, plan, observed, trust_bins=0.25):
    """Each tone's Gauss-Newton step for loss(), tones treated as decoupled:
    with residual r = model - observed and the tone's Jacobian columns
    J = [P, jP, b_t dP/df_0, ..., b_t dP/df_{D-1}] (P = Round(v(f_t))), the
    step x over (Re b_t, Im b_t, f_t) solves Re(J^H J) x = -Re(J^H r); each
    frequency step is then clipped to trust_bins / N_d (a trust region).
    Returns (step_freqs [K][D], step_amps [K] complex)."""
    r = model(freqs, amps, plan) - observed
    K = len(freqs)
    D = len(plan.shape)
    sf = np.zeros((K, D))
    sa = np.zeros(K, dtype=np.complex128)
    for t in range(K):
        P = round_buckets(tone_signal(plan.shape, freqs[t]), plan)
        J = [P, 1j * P] + [complex(amps[t]) *
                           round_buckets(tone_derivative_signal(plan.shape, freqs[t], d), plan)
                           for d in range(D)]
        H = np.array([[np.real(np.vdot(Ji, Jj)) for Jj in J] for Ji in J])
        g = np.array([np.real(np.vdot(Ji, r)) for Ji in J])
        x = np.linalg.solve(H, -g)
        sa[t] = x[0] + 1j * x[1]
        cap = trust_bins / np.array(plan.shape, dtype=np.float64)
        sf[t] = np.clip(x[2:], -cap, cap)
    return sf, sa


# ---------------------------------------------------------------------------
# Refinement with per-tone step acceptance, and the initial amplitudes of
# detected tones. The model of one tone is separable: v(f)[m] = prod_d
# exp(j 2 pi f_d m_d), and every step of a round acts per dimension (outer-
# product windows, per-dimension permutation (Def. 1), aliasing along each
# dimension (Def. 2) and the N-D DFT (eq. f)), so Round_s(v(f)) is the outer
# product of the same round applied to each dimension's 1-D sequence.
# ``factored_round_buckets`` evaluates it that way (pinned against the
# literal ``round_buckets`` of the full-grid signal in the tests).
# ---------------------------------------------------------------------------

def _round_1d(seq, plan, s, d):
    """One round along dimension d alone, on a length-N_d sequence: pre-window
    w_d, gather [sigma_{s,d} n]_{N_d}, flat window, aliasing onto B_d points,
    B_d-point DFT."""
    n = plan.shape[d]
    y = np.asarray(seq, dtype=np.complex128) * plan.w[d]
    p = y[(int(plan.sigma[s, d]) * np.arange(n, dtype=np.int64)) % n]
    z = p * plan.wbar[d]
    f = z.reshape(n // plan.B[d], plan.B[d]).sum(axis=0)
    return np.fft.fft(f)


def factored_round_buckets(freq, plan, dim=None):
    """Round_s(v(f)) for every round, [T, *B], as outer products of the
    per-dimension rounds of exp(j 2 pi f_d m); with dim = d the derivative
    d/df_d (the sequence of dimension d multiplied by j 2 pi m)."""
    out = []
    for s in range(plan.T):
        acc = np.ones((), dtype=np.complex128)
        for d, n in enumerate(plan.shape):
            m = np.arange(n, dtype=np.float64)
            seq = np.exp(2j * np.pi * float(freq[d]) * m)
            if dim == d:
                seq = 2j * np.pi * m * seq
            acc = np.multiply.outer(acc, _round_1d(seq, plan, s, d))
        out.append(acc)
    return np.stack(out)


def nearest_cell(freq, plan):
    """The grid cell nearest to a frequency: floor(f_d N_d + 1/2) mod N_d."""
    return tuple(int(math.floor(float(f) * n + 0.5)) % n for f, n in zip(freq, plan.shape))


def initial_amplitudes(freqs, plan, observed, with_spread=False):
    """Complex amplitude of each tone from the buckets its cell falls in:
    in every estimation round s, the bucket value divided by the response of
    the whole round to a unit tone at f (window, permutation, flat window,
    aliasing, DFT; Sec. III-C divides bucket values by the window spectrum),
    a_s = y_s[j_s] / P_s[j_s], with j_s = M(cell, sigma_s) the bucket of the
    nearest cell (Def. 3) and P_s the round's model of exp(j 2 pi f . m).
    The estimate a is the a_s whose magnitude is the median over the rounds
    (rank floor((n - 1) / 2) in ascending magnitude, the first round on
    ties), as the magnitude estimate takes the median: a round where another
    tone shares the bucket is outvoted.

    with_spread: also return, per tone, max_s |a_s - a| / |a| (inf when
    a = 0). A single tone explains every round with one amplitude, so its
    spread is small; a cell flagged only because different tones fill its
    buckets in different rounds (the ambiguity of Remark 1) is not, and its
    spread is of order one."""
    rounds = _rsft.estimation_rounds(plan)
    out = np.zeros(len(freqs), dtype=np.complex128)
    spread = np.zeros(len(freqs))
    for t, f in enumerate(freqs):
        cell = nearest_cell(f, plan)
        P = factored_round_buckets(f, plan)
        ratios = []
        for s in rounds:
            j = tuple((int(plan.sigma[s, d]) * cell[d]) % plan.shape[d] // plan.L[d]
                      for d in range(plan.D))
            ratios.append(observed[s][j] / P[s][j] if P[s][j] != 0 else 0j)
        order = sorted(range(len(ratios)), key=lambda q: (abs(ratios[q]), q))
        out[t] = ratios[order[(len(ratios) - 1) // 2]]
        spread[t] = (max(abs(r - out[t]) for r in ratios) / abs(out[t])
                     if out[t] != 0 else math.inf)
    return (out, spread) if with_spread else out


def refine_step(freqs, amps, radius, plan, observed, max_radius=0.25, active=None):
    """One step of per-tone trust-region Gauss-Newton on
    loss = sum_{s,k} |model_s[k] - observed_s[k]|^2, every tone against the
    same residual r = model - observed (tones decoupled):

    1. the tone's Gauss-Newton step over (Re b, Im b, f): Re(J^H J) x =
       -Re(J^H r), J = [P, jP, b dP/df_0, ...], diagonal scaled by 1 + 1e-6
       (minimum-norm solution where singular);
    2. the frequency step clipped to radius_t / N_d per dimension (radius in
       bins), f' = f + step;
    3. the amplitude re-solved for f' by least squares against the residual
       without the tone: b' = <P', b P - r> / <P', P'> (<x, y> = sum conj(x)
       y, P' the model of a unit tone at f');
    4. the tone's own change of the loss, others fixed: with delta =
       b' P' - b P, dL = 2 Re <r, delta> + ||delta||^2;
    5. dL < 0: accept (f', b') and double the radius (at most max_radius);
       else keep f, take the least-squares amplitude at f,
       b - <P, r> / <P, P>, and halve the radius.

    freqs [K][D], amps [K] complex, radius [K] in bins; active: the number
    of tones taking part (the first `active`; the rest are left as they are
    and do not enter the model). Returns new (freqs, amps, radius)."""
    K = len(freqs) if active is None else int(active)
    D = plan.D
    P = [factored_round_buckets(freqs[t], plan) for t in range(K)]
    r = sum((complex(amps[t]) * P[t] for t in range(K)), np.zeros_like(observed)) - observed
    nf = np.array(freqs, dtype=np.float64, copy=True)
    na = np.array(amps, dtype=np.complex128, copy=True)
    nr = np.array(radius, dtype=np.float64, copy=True)
    for t in range(K):
        b = complex(amps[t])
        J = [P[t], 1j * P[t]] + [b * factored_round_buckets(freqs[t], plan, dim=d) for d in range(D)]
        H = np.array([[np.real(np.vdot(Ji, Jj)) for Jj in J] for Ji in J])
        H = H + np.diag(np.diag(H)) * 1e-6
        g = np.array([np.real(np.vdot(Ji, r)) for Ji in J])
        x = np.linalg.lstsq(H, -g, rcond=1e-12)[0]
        cap = radius[t] / np.array(plan.shape, dtype=np.float64)
        fp = np.asarray(freqs[t], dtype=np.float64) + np.clip(x[2:], -cap, cap)
        Q = factored_round_buckets(fp, plan)
        qq = float(np.real(np.vdot(Q, Q)))
        pp = float(np.real(np.vdot(P[t], P[t])))
        accept = False
        if qq > 0.0:
            bp = (b * np.vdot(Q, P[t]) - np.vdot(Q, r)) / qq
            delta = bp * Q - b * P[t]
            dL = 2.0 * np.real(np.vdot(r, delta)) + float(np.real(np.vdot(delta, delta)))
            accept = dL < 0.0
        if accept:
            nf[t] = fp
            na[t] = bp
            nr[t] = min(2.0 * radius[t], max_radius)
        else:
            na[t] = b - np.vdot(P[t], r) / pp if pp > 0.0 else b
            nr[t] = 0.5 * radius[t]
    return nf, na, nr


def model_loss(freqs, amps, plan, observed, active=None):
    """The loss of the first `active` tones (all when None)."""
    K = len(freqs) if active is None else int(active)
    m = sum((complex(amps[t]) * factored_round_buckets(freqs[t], plan) for t in range(K)),
            np.zeros_like(observed))
    return float(np.sum(np.abs(m - observed) ** 2))


def model_residual(freqs, amps, plan, observed, active=None):
    """observed - the model of the first `active` tones (all when None), the
    factored model of each tone scaled by its amplitude: the round buckets
    of what those tones leave unexplained (the rounds are linear in the
    signal)."""
    K = len(freqs) if active is None else int(active)
    m = sum((complex(amps[t]) * factored_round_buckets(freqs[t], plan) for t in range(K)),
            np.zeros_like(observed))
    return np.asarray(observed, dtype=np.complex128) - m


def refine(freqs, amps, plan, observed, steps, radius0=0.25, active=None):
    """``steps`` iterations from (freqs, amps), every trust radius starting at
    radius0 bins. Each iteration first evaluates the loss of the current
    state: when it is above the lowest loss reached so far (the tones'
    decoupled steps can overshoot together where they share buckets), the
    state of that lowest loss is restored, every radius halves and the
    iteration takes no step; otherwise the state is kept as the best and
    refine_step runs. After the last iteration the same check applies once
    more. Returns (freqs, amps, radius, losses), losses holding the lowest
    loss so far before each iteration and after the last (non-increasing)."""
    K = len(freqs) if active is None else int(active)
    f = np.array(freqs, dtype=np.float64, copy=True)
    a = np.array(amps, dtype=np.complex128, copy=True)
    rad = np.full(len(f), float(radius0))
    best = math.inf
    saved = (f.copy(), a.copy())
    losses = []
    for it in range(steps + 1):
        loss = model_loss(f, a, plan, observed, K)
        if loss > best:
            f, a = saved[0].copy(), saved[1].copy()
            rad[:K] *= 0.5
            losses.append(best)
            continue
        best = loss
        saved = (f.copy(), a.copy())
        losses.append(best)
        if it == steps:
            break
        f, a, rad = refine_step(f, a, rad, plan, observed, max_radius=radius0, active=K)
    return f, a, rad, losses

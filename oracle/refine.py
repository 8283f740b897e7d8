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

Everything here is written from these definitions with numpy in FP64; the
tone signal is synthesized on the full grid and pushed through the oracle's
own round, so nothing is factored or reordered.
"""

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

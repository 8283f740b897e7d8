"""Pins of the refinement oracle (bucketized forward model of off-grid tones
and its gradients) against the mathematics: FP64 central differences of the
loss, the minimum at the true parameters, the closed-form bucket of an
on-grid tone, and an exact Newton step for the amplitudes (which fixes the
gradient convention and its factor 2)."""

import numpy as np
import pytest

import synth
from oracle import hashing as H
from oracle import refine as RF
from oracle import rsft as R


def _plan(shape, b, T=3, atten=60.0, flat=None, seed=0):
    sigma = synth.draw_sigma(np.random.default_rng(seed), T, shape)
    return R.OraclePlan(shape, b, sigma, atten, flat, 1e-3)


def _tones(rng, shape, K):
    freqs = rng.random((K, len(shape)))
    amps = (rng.standard_normal(K) + 1j * rng.standard_normal(K)) * 2.0
    return freqs, amps


@pytest.mark.parametrize("shape,b", [((64, 32), (8, 4)), ((128,), (16,)), ((16, 8, 8), (4, 2, 2))])
def test_gradients_match_central_differences(shape, b):
    """dL/df and dL/db against FP64 central differences with h = 1e-6."""
    rng = np.random.default_rng(sum(shape))
    plan = _plan(shape, b, seed=len(shape))
    freqs, amps = _tones(rng, shape, 2)
    truth_f = freqs + rng.uniform(-0.3, 0.3, freqs.shape) / np.array(shape)
    observed = RF.model(truth_f, amps * 1.1, plan)
    gf, ga = RF.loss_gradients(freqs, amps, plan, observed)
    h = 1e-6
    for t in range(len(freqs)):
        for d in range(len(shape)):
            fp, fm = freqs.copy(), freqs.copy()
            fp[t, d] += h
            fm[t, d] -= h
            cd = (RF.loss(fp, amps, plan, observed) - RF.loss(fm, amps, plan, observed)) / (2 * h)
            assert abs(cd - gf[t, d]) <= 1e-5 * max(abs(gf[t, d]), 1.0) + 1e-6 * np.max(np.abs(gf))
        for part, unit in (("re", 1.0), ("im", 1j)):
            ap, am = amps.copy(), amps.copy()
            ap[t] += h * unit
            am[t] -= h * unit
            cd = (RF.loss(freqs, ap, plan, observed) - RF.loss(freqs, am, plan, observed)) / (2 * h)
            want = ga[t].real if part == "re" else ga[t].imag
            assert abs(cd - want) <= 1e-6 * max(abs(want), 1.0) + 1e-7 * np.max(np.abs(ga))


def test_minimum_at_truth():
    shape, b = (64, 64), (8, 8)
    rng = np.random.default_rng(4)
    plan = _plan(shape, b, seed=3)
    freqs, amps = _tones(rng, shape, 3)
    observed = RF.model(freqs, amps, plan)
    assert RF.loss(freqs, amps, plan, observed) < 1e-16 * np.sum(np.abs(observed) ** 2)
    gf, ga = RF.loss_gradients(freqs, amps, plan, observed)
    assert np.max(np.abs(gf)) < 1e-6 and np.max(np.abs(ga)) < 1e-6


def test_ongrid_tone_model_closed_form():
    """Rectangular windows, on-grid tone at cell i: every round's model is
    b * N in bucket M(i, sigma_s) and 0 elsewhere."""
    shape, b = (32, 64), (4, 8)
    plan = _plan(shape, b, atten=0.0, flat=0.0, seed=7)
    cell = (5, 41)
    freqs = np.array([[cell[0] / shape[0], cell[1] / shape[1]]])
    amp = np.array([0.3 - 1.2j])
    m = RF.model(freqs, amp, plan)
    N = shape[0] * shape[1]
    for s in range(plan.T):
        j = tuple(H.mapping(cell[d], plan.sigma[s, d], shape[d], b[d]) for d in range(2))
        want = np.zeros(b, dtype=np.complex128)
        want[j] = amp[0] * N
        assert np.max(np.abs(m[s] - want)) < 1e-9 * N


def test_amplitude_newton_step_is_exact():
    """The loss is quadratic in one tone's amplitude with Hessian 2 ||basis||^2
    (per real coordinate), so b - grad / (2 ||basis||^2) lands on the least-
    squares amplitude; with noise-free data that is the true amplitude."""
    shape, b = (64, 32), (8, 8)
    rng = np.random.default_rng(11)
    plan = _plan(shape, b, seed=5)
    freqs, amps = _tones(rng, shape, 1)
    observed = RF.model(freqs, amps, plan)
    start = amps + (0.7 - 0.4j)
    _, ga = RF.loss_gradients(freqs, start, plan, observed)
    basis = RF.round_buckets(RF.tone_signal(shape, freqs[0]), plan)
    step = start - ga / (2.0 * np.sum(np.abs(basis) ** 2))
    assert abs(step[0] - amps[0]) < 1e-9 * abs(amps[0])


def test_gauss_newton_converges_quadratically_on_noise_free_tone():
    """Zero-residual problem: Gauss-Newton converges quadratically, so from
    0.1 bin and 10% amplitude off, three steps reach the truth to 1e-7 bin;
    a wrong Jacobian column or sign would stall or diverge instead."""
    shape, b = (128, 64), (16, 8)
    rng = np.random.default_rng(21)
    plan = _plan(shape, b, seed=9)
    freqs, amps = _tones(rng, shape, 1)
    observed = RF.model(freqs, amps, plan)
    f = freqs + np.array([[0.1 / shape[0], -0.08 / shape[1]]])
    a = amps * (1.1 - 0.05j)
    for _ in range(3):
        sf, sa = RF.gauss_newton_steps(f, a, plan, observed)
        f = f + sf
        a = a + sa
    err_bins = np.abs((f - freqs) * np.array(shape))
    assert err_bins.max() < 1e-7
    assert abs(a[0] / amps[0] - 1) < 1e-7


def test_factored_model_equals_full_grid_round():
    """The per-dimension evaluation of one tone's rounds (and of its
    frequency derivatives) equals the literal full-grid rounds (2-D and 3-D,
    off-grid tones, Chebyshev and rectangular windows)."""
    rng = np.random.default_rng(31)
    for shape, b, atten in (((64, 32), (8, 4), 60.0), ((16, 8, 32), (4, 2, 8), 60.0),
                            ((32, 64), (4, 8), 0.0)):
        plan = _plan(shape, b, atten=atten, flat=atten, seed=len(shape))
        f = rng.random(len(shape))
        want = RF.round_buckets(RF.tone_signal(shape, f), plan)
        got = RF.factored_round_buckets(f, plan)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
        for d in range(len(shape)):
            want = RF.round_buckets(RF.tone_derivative_signal(shape, f, d), plan)
            got = RF.factored_round_buckets(f, plan, dim=d)
            assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_initial_amplitudes_exact_on_noise_free_tones():
    """Noise-free observation of well-separated off-grid tones: the bucket
    of each tone's nearest cell divided by the round's unit-tone response
    returns the tone's amplitude: exactly for one tone; for several, within
    the others' leakage into the bucket, whose L = 128 cells each carry
    -60 dB sidelobes of random phase (about sqrt(L) 1e-3 = 1.1e-2 relative;
    bound 3x that), the median over the three clean rounds setting aside a
    round where another tone's main lobe shares the bucket."""
    shape, b = (256, 128), (16, 16)
    rng = np.random.default_rng(41)
    plan = _plan(shape, b, seed=13)
    freqs, amps = _tones(rng, shape, 1)
    observed = RF.model(freqs, amps, plan)
    got = RF.initial_amplitudes(freqs, plan, observed)
    assert abs(got[0] - amps[0]) <= 1e-10 * abs(amps[0])
    plan = _plan(shape, b, seed=3)
    assert R.estimation_rounds(plan) == [0, 1, 2]
    freqs = np.array([[0.1037, 0.2021], [0.5512, 0.7043], [0.8301, 0.3379]])
    amps = np.array([1.0 + 0.5j, -0.7 + 0.2j, 0.3 - 1.1j])
    observed = RF.model(freqs, amps, plan)
    got = RF.initial_amplitudes(freqs, plan, observed)
    assert np.max(np.abs(got / amps - 1)) < 3 * np.sqrt(128) * 1e-3


def test_amplitude_spread_of_tone_and_of_mixed_rounds():
    """The spread max_s |a_s - a| / |a| of the per-round ratios: 0 (to
    rounding) for a noise-free single tone; for observed buckets built as
    c_s times the unit-tone model in round s (a different amplitude per
    round, as when different tones fill a cell's buckets), the median-
    magnitude c_s and max_s |c_s - c_med| / |c_med| exactly."""
    shape, b = (256, 128), (16, 16)
    plan = _plan(shape, b, seed=3)
    assert R.estimation_rounds(plan) == [0, 1, 2]
    rng = np.random.default_rng(71)
    freqs, amps = _tones(rng, shape, 1)
    a, sp = RF.initial_amplitudes(freqs, plan, RF.model(freqs, amps, plan), with_spread=True)
    assert sp[0] < 1e-10
    c = np.array([1.0 + 0.2j, -0.3 + 0.5j, 2.0 - 1.0j])     # magnitudes 1.02, 0.58, 2.24
    P = RF.factored_round_buckets(freqs[0], plan)
    observed = np.stack([c[s] * P[s] for s in range(3)])
    a, sp = RF.initial_amplitudes(freqs, plan, observed, with_spread=True)
    assert abs(a[0] - c[0]) < 1e-12
    assert abs(sp[0] - np.max(np.abs(c - c[0])) / abs(c[0])) < 1e-12


def test_nearest_cell_rounds_half_up():
    plan = _plan((64, 32), (8, 4), seed=3)
    assert RF.nearest_cell((10.5 / 64, 3.49 / 32), plan) == (11, 3)
    assert RF.nearest_cell((63.6 / 64, -0.2 / 32), plan) == (0, 0)


def test_refine_step_converges_on_noise_free_tone():
    """One tone, noise-free: from 0.2 bin and 10% off, the accepted
    trust-region steps reach the true frequency to 1e-7 bin and amplitude to
    1e-7, and the loss never increases (for a single tone the tone's own
    loss change is the total change, which the acceptance test requires to
    be negative)."""
    shape, b = (128, 64), (16, 8)
    rng = np.random.default_rng(51)
    plan = _plan(shape, b, seed=9)
    freqs, amps = _tones(rng, shape, 1)
    observed = RF.model(freqs, amps, plan)
    f0 = freqs + np.array([[0.2 / shape[0], -0.15 / shape[1]]])
    a0 = amps * (1.1 - 0.05j)
    f, a, rad, losses = RF.refine(f0, a0, plan, observed, steps=8)
    assert np.abs((f - freqs) * np.array(shape)).max() < 1e-7
    assert abs(a[0] / amps[0] - 1) < 1e-7
    assert all(l1 <= l0 * (1 + 1e-12) + 1e-20 for l0, l1 in zip(losses, losses[1:]))


def test_refine_step_rejects_a_step_that_raises_the_loss():
    """A step is kept only when it lowers the tone's own loss: at the exact
    parameters every step is rejected, the frequency stays, the amplitude is
    the least-squares one (the truth) and the trust radius halves; a start
    far off with a tiny radius moves by at most that radius per step."""
    shape, b = (64, 64), (8, 8)
    rng = np.random.default_rng(61)
    plan = _plan(shape, b, seed=4)
    freqs, amps = _tones(rng, shape, 2)
    observed = RF.model(freqs, amps, plan)
    f, a, rad = RF.refine_step(freqs, amps, np.array([0.25, 0.25]), plan, observed)
    assert np.array_equal(f, freqs)
    assert np.max(np.abs(a - amps)) < 1e-9 * np.max(np.abs(amps))
    assert np.allclose(rad, 0.125)
    f0 = freqs + 0.3 / np.array(shape)
    f, a, rad = RF.refine_step(f0, amps, np.array([0.01, 0.01]), plan, observed)
    assert np.abs((f - f0) * np.array(shape)).max() <= 0.01 + 1e-12


def test_refine_guard_and_inactive_tones():
    """Two copies of one noise-free tone, both at amplitude 0: each takes the
    least-squares amplitude against the same residual (the full amplitude),
    so together they overshoot to twice it and the loss rises; the
    per-iteration check then restores the lowest-loss state, so the reported
    losses never rise and the result is the lowest-loss state seen. Tones
    past `active` stay as given and are not part of the model."""
    shape, b = (128, 64), (16, 8)
    rng = np.random.default_rng(81)
    plan = _plan(shape, b, seed=9)
    freqs, amps = _tones(rng, shape, 1)
    observed = RF.model(freqs, amps, plan)
    f0 = np.concatenate([freqs, freqs])
    a0 = np.zeros(2, dtype=np.complex128)
    f1, a1, _ = RF.refine_step(f0, a0, np.full(2, 0.25), plan, observed)
    assert RF.model_loss(f1, a1, plan, observed) > RF.model_loss(f0, a0, plan, observed)
    f, a, rad, losses = RF.refine(f0, a0, plan, observed, steps=6)
    assert all(l1 <= l0 for l0, l1 in zip(losses, losses[1:]))
    assert losses[-1] == min(losses)
    assert RF.model_loss(f, a, plan, observed) == losses[-1]
    f0 = np.concatenate([freqs, freqs + 0.05 / np.array(shape)])
    a0 = np.concatenate([amps, amps])
    f, a, rad, losses = RF.refine(f0, a0, plan, observed, steps=6)
    assert all(l1 <= l0 for l0, l1 in zip(losses, losses[1:]))
    # a far-away third tone marked inactive: untouched, outside the model
    f3 = np.concatenate([f0, [[0.71, 0.33]]])
    a3 = np.concatenate([a0, [5.0 + 0j]])
    g, c, _, l3 = RF.refine(f3, a3, plan, observed, steps=6, active=2)
    assert np.array_equal(g[2], f3[2]) and c[2] == a3[2]
    assert np.allclose(l3, losses)


def test_model_residual_leaves_the_unmodelled_tone():
    """A noise-free frame of three off-grid tones built on the full grid:
    the residual after all three is zero (to FP64 rounding), and after the
    first two it equals the literal round buckets (window, permutation, flat
    window, aliasing, DFT on the full grid) of the third tone's signal."""
    shape, b = (64, 32), (8, 4)
    plan = _plan(shape, b, seed=9)
    rng = np.random.default_rng(41)
    freqs, _ = _tones(rng, shape, 3)
    amps = np.array([2.0 - 1.0j, 0.5 + 1.5j, -1.2 + 0.3j])
    x = synth.synthesize(shape, freqs, None, amps)
    obs = RF.round_buckets(x, plan)
    scale = np.max(np.abs(obs))
    assert np.max(np.abs(RF.model_residual(freqs, amps, plan, obs))) <= 1e-10 * scale
    third = RF.round_buckets(synth.synthesize(shape, freqs[2:], None, amps[2:]), plan)
    got = RF.model_residual(freqs, amps, plan, obs, active=2)
    assert np.max(np.abs(got - third)) <= 1e-10 * scale
    assert np.max(np.abs(third)) > 1e-3 * scale

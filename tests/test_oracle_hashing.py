"""Pins of the oracle's hashing (Definitions 1-4, Properties 1-4) by
exhaustive enumeration on small sizes and the Fig. 3 worked example."""

import os

import numpy as np
import pytest

from oracle import hashing as H
from oracle import rsft as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_dft(x):
    n = len(x)
    k = np.arange(n)
    return np.array([np.sum(x * np.exp(-2j * np.pi * kk * k / n)) for kk in k])


def test_fig3_index_tables():
    with open(os.path.join(GOLDEN, "fig3_permutation.txt")) as fh:
        rows = [list(map(int, ln.split())) for ln in fh
                if ln.strip() and not ln.startswith("#")]
    for n, sigma, sigma_inv, *table in rows:
        assert H.mod_inverse(sigma, n) == sigma_inv
        assert list(H.permute(np.arange(n), sigma)) == table


def test_fig3_aliasing_into_2x4_blocks():
    """The 4x8 array of Fig. 3 permuted with sigma=(3,3) and split into four
    2x4 blocks; aliasing adds the blocks."""
    x = np.arange(32).reshape(4, 8)
    p = x[np.ix_(H.permute(np.arange(4), 3), H.permute(np.arange(8), 3))]
    blocks = p[:2, :4] + p[:2, 4:] + p[2:, :4] + p[2:, 4:]
    assert np.array_equal(R.alias_nd(p, (2, 4)), blocks)


@pytest.mark.parametrize("n", [8, 16, 64])
def test_mod_inverse_exhaustive(n):
    for s in H.odd_sigmas(n):
        assert (s * H.mod_inverse(s, n)) % n == 1
    with pytest.raises(ValueError):
        H.mod_inverse(2, n)


@pytest.mark.parametrize("n", [8, 16, 64])
def test_property1_permutation_dilates_spectrum(n):
    """Property 1 with tau = 0 (the case RSFT uses): DFT(P_sigma x)[sigma i]
    = DFT(x)[i]. For tau != 0 the phase factor works out to exp(+j 2 pi i tau/N)
    under the e^{-j} DFT convention (the printed factor omits i)."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xh = brute_dft(x)
    i = np.arange(n)
    for s in H.odd_sigmas(n):
        ph = brute_dft(H.permute(x, s))
        assert np.allclose(ph[(s * i) % n], xh, atol=1e-9)
        for tau in (1, 3):
            pt = brute_dft(H.permute(x, s, tau))
            assert np.allclose(pt[(s * i) % n],
                               xh * np.exp(2j * np.pi * i * tau / n), atol=1e-9)


@pytest.mark.parametrize("n,b", [(8, 2), (8, 4), (16, 4), (16, 8), (64, 8)])
def test_property2_alias_is_subsample(n, b):
    """Property 2: DFT_B(alias(x))[i] = DFT_N(x)[i L], on every bucket."""
    rng = np.random.default_rng(n * b)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    L = n // b
    assert np.allclose(brute_dft(H.alias(x, b)), brute_dft(x)[::L], atol=1e-9)


@pytest.mark.parametrize("n,b", [(8, 2), (8, 4), (16, 4), (16, 8), (64, 2),
                                 (64, 4), (64, 8)])
def test_properties3_4_exhaustive(n, b):
    """Reversibility (j = M(i, sigma) => i in R(j, sigma^-1)) and
    distinctiveness (the R(j) are disjoint), for every odd sigma; together:
    R(j, sigma^-1) = { i : M(i, sigma) = j }, a partition of [N]."""
    for s in H.odd_sigmas(n):
        sinv = H.mod_inverse(s, n)
        sets = [set(H.reverse_mapping(j, sinv, n, b)) for j in range(b)]
        for i in range(n):
            assert i in sets[H.mapping(i, s, n, b)]
        for j in range(b):
            for k in range(j + 1, b):
                assert not (sets[j] & sets[k])
        assert set().union(*sets) == set(range(n))
        for j in range(b):
            assert sets[j] == {i for i in range(n) if H.mapping(i, s, n, b) == j}

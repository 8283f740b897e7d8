"""Hashing primitives of RSFT, one dimension at a time (oracle; test
infrastructure only). Integer arithmetic throughout.

Definition 1 (permutation), Definition 2 (aliasing), Definition 3 (mapping),
Definition 4 (reverse mapping), and the modular inverse of eq. mod_inv.
"""

import numpy as np


def mod_inverse(sigma, n):
    """sigma^{-1} with sigma * sigma^{-1} = 1 (mod n)  (eq. mod_inv).

    Extended Euclid; raises if sigma is not invertible mod n (for n a power
    of two: sigma even)."""
    a, m = int(sigma) % int(n), int(n)
    x0, x1, r0, r1 = 1, 0, a, m
    while r1:
        q = r0 // r1
        r0, r1 = r1, r0 - q * r1
        x0, x1 = x1, x0 - q * x1
    if r0 != 1:
        raise ValueError(f"sigma={sigma} is not invertible modulo {n}")
    return x0 % m


def permute(x, sigma, tau=0):
    """Definition 1: (P_{sigma,tau} x)_i = x_{sigma i + tau}, indices mod n."""
    n = len(x)
    idx = (sigma * np.arange(n, dtype=np.int64) + tau) % n
    return np.asarray(x)[idx]


def alias(x, b):
    """Definition 2: y_i = sum_{j<L} x_{i + B j}, i in [B], L = N / B."""
    x = np.asarray(x)
    n = len(x)
    if n % b:
        raise ValueError("B must divide N")
    y = np.zeros(b, dtype=x.dtype)
    for j in range(n // b):
        y = y + x[j * b:(j + 1) * b]
    return y


def mapping(i, sigma, n, b):
    """Definition 3: M(i, sigma) = floor((B / N) [i sigma]_N)."""
    return ((int(i) * int(sigma)) % n) * b // n


def reverse_mapping(j, sigma_inv, n, b):
    """Definition 4: R(j, sigma^{-1}) = { [sigma^{-1} u]_N : jN/B <= u < (j+1)N/B }."""
    L = n // b
    return [(int(sigma_inv) * u) % n for u in range(j * L, (j + 1) * L)]


def odd_sigmas(n):
    """All valid permutation factors for n a power of two: the odd integers in
    [1, n) (Sec. V-F: any odd integer is invertible mod a power of two)."""
    return list(range(1, n, 2))

"""The paper's complexity model (oracle; test infrastructure only): operation
counts of eq. RSFT_complexity (Table II) and of the Bartlett method (Table I).
"""

import math


def complexity_rsft(N, B, T, K, eta_m, eta_p):
    """eq. RSFT_complexity, with the B-point FFT counted as B log2 B."""
    return T * (N + B + B * math.log2(B) + K * eta_m * N / (B * eta_p)) + N


def complexity_bartlett(N, T):
    """Table I total: T N (1 + log2 N) + N."""
    return T * N * (1 + math.log2(N)) + N


def best_buckets(N, T, K, eta_m, eta_p, candidates):
    """B minimising eq. RSFT_complexity over the given powers of two."""
    return min(candidates, key=lambda b: complexity_rsft(N, b, T, K, eta_m, eta_p))

// Host FP64 design math used to build a plan (windows, thresholds,
// permutation factors).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace rsft {

// Symmetric Dolph-Chebyshev window (Sec. III-C.1), centre sample n/2 == 1;
// atten_db == 0 gives the rectangular window.
std::vector<double> chebyshev_window(int64_t n, double atten_db);
// DFT-even variant: length n+1 symmetric window without its last sample.
std::vector<double> chebyshev_window_periodic(int64_t n, double atten_db);
// Flat window of Sec. IV-B (see rsft_flat_window in rsft.h).
std::vector<std::complex<double>> flat_window(int64_t n, int64_t b, double atten_db);
// |DFT(wbar)[-t]| / n, t in [0, L).
std::vector<double> flat_gain(const std::vector<std::complex<double>>& wbar, int64_t L);
// sigma^{-1} mod n; false if sigma is not invertible.
bool mod_inverse(int64_t sigma, int64_t n, int64_t* out);
// p1 with P[Bin(T, p1) >= mu] = pfa.
double stage1_probability(double pfa, int T, int mu);
// Odd permutation factor in [1, n) from a splitmix64 counter stream.
int64_t draw_sigma(uint64_t seed, int64_t counter, int64_t n);
// 6-dB main-lobe width in bins.
double six_db_width(const std::vector<double>& w);
// Averages over all odd sigma of alpha(p, sigma, omega) (p: Claim 1's bucket)
// and beta(sigma) for one dimension (eq. alpha_beta).
void alpha_beta_average(int64_t n, int64_t b, double window_db, double flat_db, double omega_bins,
                        double* alpha_bar, double* beta_bar);
// P[vote count >= mu] under H1 and H0 (Claims 2 and 3, variance upper bounds).
void stage2_tails(int mu, int T, double F, double eta_p, double pd_bar, double pfa_bar, double* pd,
                  double* pfa);

}  // namespace rsft

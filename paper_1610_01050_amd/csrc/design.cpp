// Host FP64 design math: windows, modular inverse, first-stage probability,
// permutation draws, window widths. No device work.
#include <cmath>
#include <cstdint>
#include <vector>

#include "design.h"

namespace rsft {

// T_order(x) on the whole real line.
static double chebyshev_t(int64_t order, double x) {
  if (std::fabs(x) <= 1.0) return std::cos(double(order) * std::acos(x));
  if (x > 1.0) return std::cosh(double(order) * std::acosh(x));
  double v = std::cosh(double(order) * std::acosh(-x));
  return (order & 1) ? -v : v;
}

// Symmetric Dolph-Chebyshev window: its DTFT is exp(-j w (n-1)/2) times
// T_{n-1}(x0 cos(w/2)), a degree n-1 polynomial in exp(-j w), so the n
// samples of that amplitude at w_k = 2 pi k / n give the window by an inverse
// DFT. The imaginary parts cancel in conjugate pairs, leaving
//   w[m] = (1/n) sum_k A_k cos(pi k (2m - n + 1) / n),
// evaluated with the angle reduced exactly as an integer modulo 2n.
std::vector<double> chebyshev_window(int64_t n, double atten_db) {
  std::vector<double> w(static_cast<size_t>(n), 1.0);
  if (n <= 1 || atten_db == 0.0) return w;
  const int64_t order = n - 1;
  const double ratio = std::pow(10.0, atten_db / 20.0);
  const double x0 = std::cosh(std::acosh(ratio) / double(order));
  std::vector<double> amp(static_cast<size_t>(n));
  for (int64_t k = 0; k < n; ++k)
    amp[size_t(k)] = chebyshev_t(order, x0 * std::cos(M_PI * double(k) / double(n)));
  const int64_t two_n = 2 * n;
  std::vector<double> cosine(static_cast<size_t>(two_n));
  for (int64_t r = 0; r < two_n; ++r) cosine[size_t(r)] = std::cos(M_PI * double(r) / double(n));
  for (int64_t m = 0; m < n; ++m) {
    const int64_t q = 2 * m - n + 1;
    long double acc = 0.0L;
    for (int64_t k = 0; k < n; ++k) {
      int64_t r = (k * q) % two_n;
      if (r < 0) r += two_n;
      acc += (long double)amp[size_t(k)] * (long double)cosine[size_t(r)];
    }
    w[size_t(m)] = double(acc / (long double)n);
  }
  const double centre = w[size_t(n / 2)];
  for (auto& v : w) v /= centre;
  return w;
}

std::vector<double> chebyshev_window_periodic(int64_t n, double atten_db) {
  std::vector<double> w = chebyshev_window(n + 1, atten_db);
  w.resize(size_t(n));
  return w;
}

// wbar[m] = c0[m] * sum_{k=0}^{L-1} exp(-j 2 pi k m / n): the box of bins
// {-(L-1), ..., 0} shaped by the rotated periodic Chebyshev base c0.
std::vector<std::complex<double>> flat_window(int64_t n, int64_t b, double atten_db) {
  const int64_t L = n / b;
  std::vector<double> c = chebyshev_window_periodic(n, atten_db);
  const double peak = c[size_t(n / 2)];
  std::vector<double> cs(static_cast<size_t>(n)), sn(static_cast<size_t>(n));
  for (int64_t r = 0; r < n; ++r) {
    cs[size_t(r)] = std::cos(2.0 * M_PI * double(r) / double(n));
    sn[size_t(r)] = std::sin(2.0 * M_PI * double(r) / double(n));
  }
  std::vector<std::complex<double>> out(static_cast<size_t>(n));
  for (int64_t m = 0; m < n; ++m) {
    const double base = c[size_t((m + n / 2) % n)] / peak;
    long double re = 0.0L, im = 0.0L;
    for (int64_t k = 0; k < L; ++k) {
      const int64_t r = (k * m) % n;       // angle -2 pi k m / n
      re += cs[size_t(r)];
      im -= sn[size_t(r)];
    }
    out[size_t(m)] = std::complex<double>(base * double(re), base * double(im));
  }
  return out;
}

// |DFT_n(wbar)[-t]| / n for t in [0, L): response of the flat window at
// offset -t from the first bin of a bucket.
std::vector<double> flat_gain(const std::vector<std::complex<double>>& wbar, int64_t L) {
  const int64_t n = int64_t(wbar.size());
  std::vector<double> cs(static_cast<size_t>(n)), sn(static_cast<size_t>(n));
  for (int64_t r = 0; r < n; ++r) {
    cs[size_t(r)] = std::cos(2.0 * M_PI * double(r) / double(n));
    sn[size_t(r)] = std::sin(2.0 * M_PI * double(r) / double(n));
  }
  std::vector<double> g(static_cast<size_t>(L));
  for (int64_t t = 0; t < L; ++t) {
    // DFT at bin -t: sum_m wbar[m] exp(+j 2 pi t m / n)
    long double re = 0.0L, im = 0.0L;
    for (int64_t m = 0; m < n; ++m) {
      const int64_t r = (t * m) % n;
      const double c = cs[size_t(r)], s = sn[size_t(r)];
      re += wbar[size_t(m)].real() * c - wbar[size_t(m)].imag() * s;
      im += wbar[size_t(m)].real() * s + wbar[size_t(m)].imag() * c;
    }
    g[size_t(t)] = std::sqrt(double(re * re + im * im)) / double(n);
  }
  return g;
}

bool mod_inverse(int64_t sigma, int64_t n, int64_t* out) {
  int64_t a = ((sigma % n) + n) % n, m = n;
  int64_t x0 = 1, x1 = 0, r0 = a, r1 = m;
  while (r1 != 0) {
    const int64_t q = r0 / r1;
    int64_t t = r0 - q * r1; r0 = r1; r1 = t;
    t = x0 - q * x1; x0 = x1; x1 = t;
  }
  if (r0 != 1) return false;
  *out = ((x0 % m) + m) % m;
  return true;
}

static double binomial_tail(double p, int T, int mu) {
  double total = 0.0;
  for (int c = mu; c <= T; ++c) {
    double comb = 1.0;
    for (int i = 0; i < c; ++i) comb = comb * double(T - i) / double(i + 1);
    total += comb * std::pow(p, c) * std::pow(1.0 - p, T - c);
  }
  return total;
}

double stage1_probability(double pfa, int T, int mu) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (binomial_tail(mid, T, mu) < pfa) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

static uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int64_t draw_sigma(uint64_t seed, int64_t counter, int64_t n) {
  const uint64_t z = splitmix64(seed + uint64_t(counter + 1) * 0x9E3779B97F4A7C15ull);
  return 2 * int64_t(z % uint64_t(n / 2)) + 1;
}

// 6.0-dB main-lobe width of w in DFT bins (the eta_m of Sec. IV-A): the
// half-width is where |W(f)| / |W(0)| falls to 10^(-6/20), found by bisection.
double six_db_width(const std::vector<double>& w) {
  const int64_t n = int64_t(w.size());
  auto mag = [&](double f) {
    long double re = 0.0L, im = 0.0L;
    for (int64_t m = 0; m < n; ++m) {
      const double ang = -2.0 * M_PI * f * double(m);
      re += w[size_t(m)] * std::cos(ang);
      im += w[size_t(m)] * std::sin(ang);
    }
    return std::sqrt(double(re * re + im * im));
  };
  const double target = mag(0.0) * std::pow(10.0, -6.0 / 20.0);
  double lo = 0.0, hi = 0.5 / double(n);
  while (mag(hi) > target && hi < 0.5) hi *= 1.5;
  for (int it = 0; it < 80; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mag(mid) > target) lo = mid; else hi = mid;
  }
  return 2.0 * 0.5 * (lo + hi) * double(n);
}

void alpha_beta_average(int64_t n, int64_t b, double window_db, double flat_db, double omega_bins,
                        double* alpha_bar, double* beta_bar) {
  const std::vector<double> w = chebyshev_window(n, window_db);
  const std::vector<std::complex<double>> wbar = flat_window(n, b, flat_db);
  const double two_pi = 6.283185307179586476925286766559;
  const int64_t k0 = int64_t(std::floor(omega_bins));
  const double frac = omega_bins - std::floor(omega_bins);
  double asum = 0.0, bsum = 0.0;
  int64_t count = 0;
  for (int64_t sigma = 1; sigma < n; sigma += 2) {
    // Claim 1: p = floor(B/N [sigma floor(omega / dw)]_N)
    const int64_t p = ((sigma * k0) % n) * b / n;
    std::complex<double> acc = 0.0;
    double beta = 0.0;
    for (int64_t m = 0; m < n; ++m) {
      const int64_t u = (sigma * m) % n;             // permuted index [sigma m]_N
      // exp(j omega u) with omega u / 2 pi = (k0 u mod N + frac u) / N
      const double cyc = (double((k0 * u) % n) + frac * double(u)) / double(n);
      // DFT kernel exp(-2 pi i p m / B), phase reduced as an integer
      const double dft = double((p * m) % b) / double(b);
      const double ph = two_pi * (cyc - dft);
      const std::complex<double> z = wbar[size_t(m)] * w[size_t(u)];
      acc += z * std::complex<double>(std::cos(ph), std::sin(ph));
      beta += std::norm(z);
    }
    asum += std::norm(acc);
    bsum += beta;
    ++count;
  }
  *alpha_bar = asum / double(count);
  *beta_bar = bsum / double(count);
}

static double normal_tail(double z) { return 0.5 * std::erfc(z / std::sqrt(2.0)); }

void stage2_tails(int mu, int T, double F, double eta_p, double pd_bar, double pfa_bar, double* pd,
                  double* pfa) {
  const double m1 = T * pd_bar, v1 = T * pd_bar * (1.0 - pd_bar);
  const double m0 = F * eta_p * pd_bar + (T - F) * pfa_bar;
  const double v0 = F * eta_p * pd_bar * (1.0 - eta_p * pd_bar) + (T - F) * pfa_bar * (1.0 - pfa_bar);
  *pd = v1 > 0.0 ? normal_tail((mu - m1) / std::sqrt(v1)) : (m1 >= mu ? 1.0 : 0.0);
  *pfa = v0 > 0.0 ? normal_tail((mu - m0) / std::sqrt(v0)) : (m0 >= mu ? 1.0 : 0.0);
}

}  // namespace rsft

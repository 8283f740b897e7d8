// Host side of the C ABI: plan construction (FP64 tables), launch
// orchestration, optional hipGraph replay, result copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "design.h"
#include "rsft.h"
#include "rsft_internal.h"

namespace {

thread_local std::string g_last_error;

rsft_status fail(rsft_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(RSFT_ERROR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_TRY(expr)                                                           \
  do {                                                                             \
    int e_ = (expr);                                                               \
    if (e_ != 0)                                                                   \
      return fail(RSFT_ERROR_DEVICE, std::string(#expr) + ": " +                   \
                                         hipGetErrorString(hipError_t(e_)));       \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct TimingSet {
  hipEvent_t ev[RSFT_NUM_STAGES + 1] = {};  // stage boundaries
  bool pending = false;
};

}  // namespace

struct rsft_plan_s {
  int device = 0;
  bool uniform = true;
  int64_t ndesc = 0;
  int64_t max_frames = 0;      // frames one execute may process
  int T = 0, mu = 0, dtype = 0;
  int segments = 0;            // 1: round s of a frame reads its segment s
  std::vector<rsft::FrameDesc> descs;
  std::vector<rsft_plan_info_t> info;
  rsft::FoldConfig fold{256, 4, 0};
  int num_cus = 256;
  int64_t min_nl = 0;
  int maxB = 0, max_words = 0, max_cchunks = 0, sum_tw_max = 0, dims_mask = 0, est_nmask = 0;
  int rows_ok = 1, masks_ok = 1;   // every frame suits the row vote / the 32-cell mask vote
  int words_ok = 1;                // every frame suits the word-parallel vote
  int global_gains = 0;            // some frame's sum of L_d exceeds the estimate's LDS copy
  int split_ok = 1;                // every frame suits the two-pass DFT
  int dft_split = 1;               // RSFT_OPT_DFT_SPLIT: use it (where it applies)
  int dft_threads = 1024;          // RSFT_OPT_DFT_THREADS: the one-work-group DFT's size
  int split_b0 = 0, split_g1 = 0, split_g2 = 0, split_e1 = 0;   // its launch extents
  int vote_words = 1;              // RSFT_OPT_VOTE_WORDS: prefer the word-parallel vote
  int tab_words = 0;               // LDS words of its per-round table (largest frame)
  int vote_path = rsft::kVoteCells;
  int dft_plane = 0;   // floats per LDS plane of the DFT: B plus one pad per last-dimension row
  int dft_pad = 0;     // 1 when those pads are used
  int64_t tiles_per_frame = 0;   // uniform plans
  int64_t ntiles_uneven = 0;     // uneven plans
  int64_t nchunk_list = 0;       // uneven plans with frames of different chunk counts
  int64_t nvote_list = 0;        // the same for the word-parallel vote's chunk groups
  int exp_blocks = 0;            // the most kVoteExpWords blocks of bucket-row masks of a frame
  int64_t nexp_list = 0;         // uneven plans: (frame, block) entries of those masks
  int scan_fpb = 1;              // frames per scan work-group
  // device arrays
  DeviceBuffer d_descs, d_wrow, d_wcol, d_rowlist, d_tw, d_gains, d_win, d_flat, d_tiles, d_chunk_list,
      d_dft_order, d_vote_tab, d_vote_list, d_inter, d_vote_exp, d_vote_exp_list;
  DeviceBuffer d_part, d_buckets, d_powers, d_flags, d_bitmap, d_chunk_counts, d_chunk_offsets, d_counts,
      d_offsets, d_records, d_scan_done, d_chunk_items, d_item_counts, d_item_offsets;
  rsft::DevPtrs ptrs{};
  // state of the last execute
  int64_t last_batch = -1;
  int64_t folded_batch = -1;   // batch of the last rsft_execute_fold not yet followed by its tail
  // graph replay
  bool use_graph = true;
  hipStream_t capture_stream = nullptr;
  // estimate layout: 1 adds overflow workers for dense chunks (rsft_autotune)
  int est_workers = 0;
  // captured launch sequences per (part: 0 whole, 1 fold, 2 tail; input; batch)
  std::map<std::tuple<int, const void*, int64_t>, hipGraphExec_t> graphs;
  std::vector<std::tuple<int, const void*, int64_t>> graph_order;
  // stage timing
  bool timing = false;
  std::vector<TimingSet> timing_sets;
  size_t timing_next = 0;
  double stage_ms[RSFT_NUM_STAGES] = {0, 0, 0, 0};
  int64_t timed = 0;
};

namespace {

// Vote kernel of a plan: the word-parallel masks where every frame's rows
// suit them (and RSFT_OPT_VOTE_WORDS is on), else the candidate rows, the
// 32-cell masks, or the per-cell gather.
void choose_vote_path(rsft_plan_s* pl) {
  pl->vote_path = pl->words_ok && pl->vote_words ? rsft::kVoteWords
                  : pl->rows_ok && pl->T <= 4    ? rsft::kVoteRows
                  : pl->masks_ok                 ? rsft::kVoteMasks32
                  : pl->words_ok                 ? rsft::kVoteWords
                                                 : rsft::kVoteCells;
}

rsft_status validate(const rsft_params& p, int64_t idx) {
  const std::string at = "frame descriptor " + std::to_string(idx) + ": ";
  if (p.ndim < 1 || p.ndim > RSFT_MAX_DIMS) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "ndim must be 1..4");
  if (p.rounds < 1 || p.rounds > RSFT_MAX_ROUNDS)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "rounds must be 1..64");
  int64_t N = 1, B = 1;
  for (int d = 0; d < p.ndim; ++d) {
    if (!is_pow2(p.n[d]) || !is_pow2(p.b[d]))
      return fail(RSFT_ERROR_NOT_POW2, at + "N_d and B_d must be powers of two");
    if (p.b[d] >= p.n[d]) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "need B_d < N_d");
    if (p.n[d] > (int64_t(1) << 30)) return fail(RSFT_ERROR_UNSUPPORTED, at + "N_d > 2^30");
    if (p.b[d] > 128) return fail(RSFT_ERROR_UNSUPPORTED, at + "B_d > 128 per dimension");
    N *= p.n[d];
    B *= p.b[d];
  }
  if (N >= (int64_t(1) << 40)) return fail(RSFT_ERROR_UNSUPPORTED, at + "N >= 2^40");
  if (B > rsft::kMaxBuckets) return fail(RSFT_ERROR_UNSUPPORTED, at + "B > 16384 buckets");
  if ((N / B) > (int64_t(1) << 30)) return fail(RSFT_ERROR_UNSUPPORTED, at + "N / B > 2^30");
  if (!(p.pfa > 0.0 && p.pfa < 1.0)) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "pfa must be in (0, 1)");
  if (p.mu < 0 || p.mu > p.rounds) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "mu must be 0..T");
  if (p.noise_mode != RSFT_NOISE_KNOWN && p.noise_mode != RSFT_NOISE_ESTIMATED)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "unknown noise_mode");
  if (p.noise_mode == RSFT_NOISE_KNOWN && !(p.noise_var > 0.0))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "noise_var must be > 0");
  if (p.dtype != RSFT_C64 && p.dtype != RSFT_C128) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "unknown dtype");
  if (p.window_atten_db < 0.0 || !std::isfinite(p.window_atten_db))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "window_atten_db must be >= 0");
  if (!std::isfinite(p.flat_atten_db)) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "flat_atten_db not finite");
  if (p.max_detections < 0 || p.max_detections > rsft::kMaxDetectionsPerFrame)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "max_detections must be 0..2^24");
  if (p.max_batch < 0) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "max_batch must be >= 0");
  if (p.segments != 0 && p.segments != 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "segments must be 0 or 1");
  if (p.reserved0 != 0) return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "reserved0 must be 0");
  if (!(p.stage1_pfa >= 0.0 && p.stage1_pfa < 1.0))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, at + "stage1_pfa must be in [0, 1)");
  if (p.sigma) {
    for (int s = 0; s < p.rounds; ++s)
      for (int d = 0; d < p.ndim; ++d) {
        const int64_t v = p.sigma[s * p.ndim + d];
        if (v < 1 || v >= p.n[d] || (v & 1) == 0)
          return fail(RSFT_ERROR_BAD_SIGMA, at + "sigma must be odd and in [1, N_d)");
      }
  }
  return RSFT_OK;
}

template <typename T>
rsft_status upload(DeviceBuffer& buf, const std::vector<T>& host) {
  buf.bytes = std::max<size_t>(host.size() * sizeof(T), 16);
  HIP_TRY(hipMalloc(&buf.ptr, buf.bytes));
  if (!host.empty()) HIP_TRY(hipMemcpy(buf.ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
  return RSFT_OK;
}

rsft_status alloc(DeviceBuffer& buf, size_t bytes) {
  buf.bytes = std::max<size_t>(bytes, 16);
  const hipError_t e = hipMalloc(&buf.ptr, buf.bytes);
  if (e == hipErrorOutOfMemory) return fail(RSFT_ERROR_OUT_OF_MEMORY, "device allocation failed");
  if (e != hipSuccess) return fail(RSFT_ERROR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return RSFT_OK;
}

void release(DeviceBuffer& buf) {
  if (buf.ptr) (void)hipFree(buf.ptr);
  buf.ptr = nullptr;
  buf.bytes = 0;
}

// Host tables of one descriptor, appended to the plan-wide arrays.
struct HostTables {
  std::vector<float2> wrow, wcol, tw, flat;
  std::vector<int32_t> rowlist;
  std::vector<float> inv_gains;
  std::vector<float> win;
};

// Rounds feeding magnitude estimates: a round is clean when no dimension d
// and k in {1, 2} has |[sigma_{s,d} k]_{N_d}| (circular) < L_d + 2, i.e. the
// main-lobe bins of one tone never share a bucket; every clean round is
// used, else the one whose worst distance is largest (first on ties).
uint64_t estimation_mask(const rsft_params& p, const std::vector<int64_t>& sigma) {
  std::vector<int64_t> score(static_cast<size_t>(p.rounds));
  uint64_t mask = 0;
  for (int s = 0; s < p.rounds; ++s) {
    int64_t worst = INT64_MAX;
    for (int d = 0; d < p.ndim; ++d) {
      const int64_t n = p.n[d], L = p.n[d] / p.b[d];
      for (int k = 1; k <= 2; ++k) {
        const int64_t u = (sigma[size_t(s * p.ndim + d)] * k) % n;
        const int64_t dist = std::min(u, n - u) - (L + 2);
        worst = std::min(worst, dist);
      }
    }
    score[size_t(s)] = worst;
    if (worst >= 0) mask |= uint64_t(1) << s;
  }
  if (mask) return mask;
  int best = 0;
  for (int s = 1; s < p.rounds; ++s)
    if (score[size_t(s)] > score[size_t(best)]) best = s;
  return uint64_t(1) << best;
}

rsft_status build_descriptor(const rsft_params& p, rsft::FrameDesc& d, rsft_plan_info_t& info,
                             HostTables& ht) {
  const int64_t fold_p = rsft::kFoldMaxP;   // chunks must suit every fold shape the tuner may pick
  std::memset(&d, 0, sizeof(d));
  std::memset(&info, 0, sizeof(info));
  const int D = p.ndim, T = p.rounds;
  const int mu = p.mu == 0 ? T : p.mu;
  d.ndim = D;
  d.T = T;
  d.segments = p.segments;
  d.mu = mu;
  d.noise_mode = p.noise_mode;
  int64_t N = 1, B = 1;
  for (int k = 0; k < D; ++k) {
    d.n[k] = int32_t(p.n[k]);
    d.b[k] = int32_t(p.b[k]);
    d.l[k] = int32_t(p.n[k] / p.b[k]);
    d.lshift[k] = ilog2(d.l[k]);
    N *= p.n[k];
    B *= p.b[k];
  }
  for (int k = 0; k < D; ++k) {
    int ns = 0, bs = 0, ts = 0;
    for (int e = k + 1; e < D; ++e) {
      ns += ilog2(p.n[e]);
      bs += ilog2(p.b[e]);
      ts += ilog2(p.n[e] / p.b[e]);
    }
    d.nshift[k] = ns;
    d.bshift[k] = bs;
    d.tshift[k] = ts;
  }
  d.N = N;
  d.B = int32_t(B);
  d.Lshift = ilog2(N / B);
  d.words = int32_t((B + 31) / 32);
  d.cap = p.max_detections == 0 ? rsft::kDefaultDetections : p.max_detections;

  // permutation factors
  std::vector<int64_t> sigma(static_cast<size_t>(T * D));
  for (int s = 0; s < T; ++s)
    for (int k = 0; k < D; ++k)
      sigma[size_t(s * D + k)] = p.sigma ? p.sigma[s * D + k] : rsft::draw_sigma(p.seed, s * D + k, p.n[k]);
  std::vector<int64_t> sigma_inv(sigma.size());
  for (int s = 0; s < T; ++s)
    for (int k = 0; k < D; ++k) {
      int64_t inv = 0;
      if (!rsft::mod_inverse(sigma[size_t(s * D + k)], p.n[k], &inv))
        return fail(RSFT_ERROR_BAD_SIGMA, "sigma not invertible");
      sigma_inv[size_t(s * D + k)] = inv;
      d.sigma[s][k] = int32_t(sigma[size_t(s * D + k)]);
      d.sigma_inv[s][k] = int32_t(inv);
      d.tau[s][k] = int32_t(inv % p.b[k]);
    }
  d.est_mask = estimation_mask(p, sigma);
  d.n_est = 0;
  for (int s = 0; s < T; ++s)
    if ((d.est_mask >> s) & 1u) {
      if (d.n_est < rsft::kMaxEstRounds) d.est_rounds[d.n_est] = s;
      ++d.n_est;
    }

  // windows (Sec. III-C.1, Sec. IV-B) per dimension, FP64
  const double flat_db = p.flat_atten_db < 0.0 ? p.window_atten_db : p.flat_atten_db;
  std::vector<std::vector<double>> w(static_cast<size_t>(D));
  std::vector<std::vector<std::complex<double>>> wbar(static_cast<size_t>(D));
  double eta = 1.0;
  for (int k = 0; k < D; ++k) {
    w[size_t(k)] = rsft::chebyshev_window(p.n[k], p.window_atten_db);
    wbar[size_t(k)] = rsft::flat_window(p.n[k], p.b[k], flat_db);
    eta *= rsft::six_db_width(w[size_t(k)]);
  }
  // permuted weights W_{s,d}[m] = w_d[m] wbar_d[[sigma^{-1} m]_{N_d}]
  std::vector<std::vector<std::complex<double>>> W(static_cast<size_t>(T * D));
  for (int s = 0; s < T; ++s)
    for (int k = 0; k < D; ++k) {
      auto& v = W[size_t(s * D + k)];
      v.resize(size_t(p.n[k]));
      const int64_t inv = sigma_inv[size_t(s * D + k)];
      for (int64_t m = 0; m < p.n[k]; ++m)
        v[size_t(m)] = w[size_t(k)][size_t(m)] * wbar[size_t(k)][size_t((inv * m) % p.n[k])];
    }
  // beta(sigma_s) = ||Wbar P_sigma w||^2 (eq. alpha_beta), separable over dims
  const double p1 = p.stage1_pfa > 0.0 ? p.stage1_pfa : rsft::stage1_probability(p.pfa, T, mu);
  d.log_inv_p1 = std::log(1.0 / p1);
  for (int s = 0; s < T; ++s) {
    double beta = 1.0;
    for (int k = 0; k < D; ++k) {
      long double acc = 0.0L;
      const int64_t sg = sigma[size_t(s * D + k)];
      for (int64_t n = 0; n < p.n[k]; ++n) {
        const double a = std::norm(wbar[size_t(k)][size_t(n)]);
        const double b = w[size_t(k)][size_t((sg * n) % p.n[k])];
        acc += (long double)a * b * b;
      }
      beta *= double(acc);
    }
    info.beta[s] = beta;
    d.gamma[s] = p.noise_var * beta * d.log_inv_p1;   // eq. tpd with Pfa~ = p1
    info.gamma[s] = d.gamma[s];
  }
  {
    const int64_t h = std::max<int64_t>(B / 2, 1);
    long double H = 0.0L;
    for (int64_t i = 0; i < h; ++i) H += 1.0L / (long double)(B - i);
    d.renyi_h = double(H);
  }

  // fold view: rows = leading dims flattened, columns = the last dim, or
  // the last two flattened when rows would be short (< 64 cells, D >= 3)
  // and the flattened residue period B_{D-2} N_{D-1} and residue count
  // B_{D-2} B_{D-1} stay within the smallest fold pass (512 slots)
  const int F = (D >= 3 && p.n[D - 1] < 64 && p.b[D - 2] * p.n[D - 1] <= 512 &&
                 p.b[D - 2] * p.b[D - 1] <= 512) ? 2 : 1;
  const int64_t nl = F == 2 ? p.n[D - 2] * p.n[D - 1] : p.n[D - 1];
  const int64_t bl = F == 2 ? p.b[D - 2] * p.b[D - 1] : p.b[D - 1];
  const int64_t rows_total = N / nl;
  const int64_t classes = B / bl;
  const int64_t R = rows_total / classes;
  d.n_last = int32_t(p.n[D - 1]);
  d.b_last = int32_t(p.b[D - 1]);
  d.fold_nl = int32_t(nl);
  d.fold_bl = int32_t(bl);
  d.fold_bin = int32_t(p.b[D - 1]);
  d.fold_lw = F == 2 ? ilog2(int32_t(p.n[D - 1])) : 24;
  d.rows_total = int32_t(rows_total);
  d.classes = int32_t(classes);
  d.rows_per_class = int32_t(R);
  // rows shorter than the smallest fold pass: one tile takes several
  // classes (a group of threads each), so that a work-group reads enough
  d.fold_cpt = (F == 1 && nl < rsft::kFoldMinP) ? int32_t(std::min<int64_t>(rsft::kFoldMinP / nl, classes)) : 1;
  if (nl >= fold_p) {
    int64_t k = 1;
    const int64_t target = 32768;  // elements per tile
    while (R * fold_p * k * 2 <= target && fold_p * k * 2 <= nl) k *= 2;
    d.chunk_cols = int32_t(fold_p * k);
  } else {
    d.chunk_cols = int32_t(nl);
  }
  d.nchunks = int32_t(nl / d.chunk_cols);

  d.wrow_off = int64_t(ht.wrow.size());
  for (int s = 0; s < T; ++s)
    for (int64_t r = 0; r < rows_total; ++r) {
      std::complex<double> v(1.0, 0.0);
      int64_t rem = r;
      for (int k = D - 1 - F; k >= 0; --k) {
        const int64_t m = rem % p.n[k];
        rem /= p.n[k];
        v *= W[size_t(s * D + k)][size_t(m)];
      }
      ht.wrow.push_back(make_float2(float(v.real()), float(v.imag())));
    }
  d.wcol_off = int64_t(ht.wcol.size());
  for (int s = 0; s < T; ++s)
    for (int64_t c = 0; c < nl; ++c) {
      std::complex<double> v = W[size_t(s * D + D - 1)][size_t(c % p.n[D - 1])];
      if (F == 2) v *= W[size_t(s * D + D - 2)][size_t(c / p.n[D - 1])];
      ht.wcol.push_back(make_float2(float(v.real()), float(v.imag())));
    }
  d.rowlist_off = int64_t(ht.rowlist.size());
  for (int64_t cls = 0; cls < classes; ++cls) {
    // class = row-major (c_0, ..., c_{D-1-F}) over B_0 x ... x B_{D-1-F}
    int64_t c[RSFT_MAX_DIMS] = {0, 0, 0, 0};
    int64_t rem = cls;
    for (int k = D - 1 - F; k >= 0; --k) {
      c[k] = rem % p.b[k];
      rem /= p.b[k];
    }
    for (int64_t li = 0; li < R; ++li) {
      int64_t lrem = li, row = 0, stride = 1;
      int64_t m[RSFT_MAX_DIMS] = {0, 0, 0, 0};
      for (int k = D - 1 - F; k >= 0; --k) {
        const int64_t L = p.n[k] / p.b[k];
        m[k] = c[k] + p.b[k] * (lrem % L);
        lrem /= L;
      }
      for (int k = D - 1 - F; k >= 0; --k) {
        row += m[k] * stride;
        stride *= p.n[k];
      }
      ht.rowlist.push_back(int32_t(row));
    }
  }
  for (int k = 0; k < D; ++k) {
    d.tw_off[k] = int64_t(ht.tw.size());
    for (int64_t m = 0; m < p.b[k]; ++m) {
      const double ang = -2.0 * M_PI * double(m) / double(p.b[k]);
      ht.tw.push_back(make_float2(float(std::cos(ang)), float(std::sin(ang))));
    }
    d.gain_off[k] = int64_t(ht.inv_gains.size());
    for (double g : rsft::flat_gain(wbar[size_t(k)], p.n[k] / p.b[k])) ht.inv_gains.push_back(float(1.0 / g));
    d.win_off[k] = int64_t(ht.win.size());
    for (int64_t m = 0; m < p.n[k]; ++m) ht.win.push_back(float(w[size_t(k)][size_t(m)]));
    d.flat_off[k] = int64_t(ht.flat.size());
    for (int64_t m = 0; m < p.n[k]; ++m)
      ht.flat.push_back(make_float2(float(wbar[size_t(k)][size_t(m)].real()),
                                    float(wbar[size_t(k)][size_t(m)].imag())));
  }

  info.ndim = D;
  info.rounds = T;
  info.mu = mu;
  info.noise_mode = p.noise_mode;
  for (int k = 0; k < D; ++k) {
    info.n[k] = p.n[k];
    info.b[k] = p.b[k];
  }
  for (int s = 0; s < T; ++s)
    for (int k = 0; k < D; ++k) {
      info.sigma[s][k] = sigma[size_t(s * D + k)];
      info.sigma_inv[s][k] = sigma_inv[size_t(s * D + k)];
      info.tau[s][k] = sigma_inv[size_t(s * D + k)] % p.b[k];
    }
  info.p1 = p1;
  info.eta_m = eta;
  info.max_sparsity = double(B) / eta;
  info.estimation_rounds = d.est_mask;
  return RSFT_OK;
}

void free_plan(rsft_plan_s* pl) {
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
  pl->graphs.clear();
  for (auto& ts : pl->timing_sets)
    for (auto& e : ts.ev)
      if (e) (void)hipEventDestroy(e);
  if (pl->capture_stream) (void)hipStreamDestroy(pl->capture_stream);
  DeviceBuffer* bufs[] = {&pl->d_descs, &pl->d_wrow, &pl->d_wcol, &pl->d_rowlist, &pl->d_tw,
                          &pl->d_gains, &pl->d_win, &pl->d_flat, &pl->d_tiles, &pl->d_chunk_list,
                          &pl->d_dft_order, &pl->d_vote_tab, &pl->d_vote_list, &pl->d_inter, &pl->d_vote_exp,
                          &pl->d_vote_exp_list, &pl->d_part,
                          &pl->d_buckets, &pl->d_powers, &pl->d_flags, &pl->d_bitmap, &pl->d_chunk_counts,
                          &pl->d_chunk_offsets, &pl->d_counts, &pl->d_offsets, &pl->d_records,
                          &pl->d_scan_done, &pl->d_chunk_items, &pl->d_item_counts, &pl->d_item_offsets};
  for (auto* b : bufs) release(*b);
  delete pl;
}

rsft_status create_plan(const rsft_params* frames, int64_t nframes, rsft_plan_s* pl) {
  pl->uniform = nframes == 1;
  pl->ndesc = nframes;
  pl->T = frames[0].rounds;
  pl->mu = frames[0].mu == 0 ? frames[0].rounds : frames[0].mu;
  pl->dtype = frames[0].dtype;
  pl->segments = frames[0].segments;
  pl->max_frames = pl->uniform ? std::max<int64_t>(frames[0].max_batch, 1) : nframes;

  // fold launch shape: P = threads * vec covers the largest B_{D-1}
  int64_t max_bl = 1;
  for (int64_t i = 0; i < nframes; ++i) max_bl = std::max<int64_t>(max_bl, frames[i].b[frames[i].ndim - 1]);
  // each thread loads `vec` consecutive complex samples of one row, so rows
  // must hold at least that many
  int64_t min_nl = INT64_MAX;
  for (int64_t i = 0; i < nframes; ++i) min_nl = std::min<int64_t>(min_nl, frames[i].n[frames[i].ndim - 1]);
  pl->min_nl = min_nl;
  (void)hipDeviceGetAttribute(&pl->num_cus, hipDeviceAttributeMultiprocessorCount, pl->device);
  if (pl->num_cus <= 0) pl->num_cus = 256;
  // default fold shape: 256 threads x 4 samples, ordinary loads;
  // rsft_autotune may replace it
  pl->fold = rsft::FoldConfig{256, min_nl >= 4 ? 4 : 2, 0};
  if (int64_t(pl->fold.threads) * pl->fold.vec < max_bl) return fail(RSFT_ERROR_UNSUPPORTED, "last-dimension B too large");

  HostTables ht;
  pl->descs.resize(size_t(nframes));
  pl->info.resize(size_t(nframes));
  for (int64_t i = 0; i < nframes; ++i) {
    rsft_status st = build_descriptor(frames[i], pl->descs[size_t(i)], pl->info[size_t(i)], ht);
    if (st != RSFT_OK) return st;
  }

  // workspace layout
  int64_t in_off = 0, part_off = 0, bucket_off = 0, flag_off = 0, bitmap_off = 0, chunk_off = 0,
          rec_total = 0;
  for (int64_t i = 0; i < nframes; ++i) {
    auto& d = pl->descs[size_t(i)];
    const int64_t mult = pl->uniform ? pl->max_frames : 1;
    d.in_off = in_off;
    d.in_stride = pl->segments ? d.N * d.T : d.N;   // segment mode: [T][N] per frame
    d.part_off = part_off;
    d.part_stride = int64_t(d.nchunks) * d.T * d.B;
    d.bucket_off = bucket_off;
    d.bucket_stride = int64_t(d.T) * d.B;
    d.flag_off = flag_off;
    d.flag_stride = int64_t(d.T) * d.words;
    d.bitmap_words = int32_t((d.N + 31) / 32);
    d.cchunks = int32_t((d.N + (int64_t(1) << rsft::kCompactShift) - 1) >> rsft::kCompactShift);
    d.bitmap_off = bitmap_off;
    d.bitmap_stride = d.bitmap_words;
    d.chunk_off = chunk_off;
    d.chunk_stride = d.cchunks;
    in_off += mult * d.in_stride;
    part_off += mult * d.part_stride;
    bucket_off += mult * d.bucket_stride;
    flag_off += mult * d.flag_stride;
    bitmap_off += mult * d.bitmap_stride;
    chunk_off += mult * d.chunk_stride;
    rec_total += mult * d.cap;
    pl->maxB = std::max(pl->maxB, d.B);
    pl->dft_plane = std::max(pl->dft_plane, d.B + d.B / d.b_last);
    pl->max_words = std::max(pl->max_words, d.words);
    pl->max_cchunks = std::max(pl->max_cchunks, d.cchunks);
    pl->dims_mask |= 1 << (d.ndim - 1);
    pl->est_nmask |= 1 << std::min(d.n_est, rsft::kMaxEstRounds + 1);
    {
      int64_t lsum = 0;
      for (int k = 0; k < d.ndim; ++k) lsum += d.l[k];
      if (lsum > rsft::kEstGainLds) pl->global_gains = 1;
    }
    if (d.n_last < 64 || d.n_last > 4096) pl->rows_ok = 0;
    if (d.n_last != 32) pl->masks_ok = 0;
    {
      const int64_t nl = d.n[d.ndim - 1];
      const int64_t tw = int64_t(d.b[d.ndim - 1]) * (nl / 32);
      if (nl < 128 || nl > 4096 || tw > 16384) pl->words_ok = 0;
      else pl->tab_words = std::max(pl->tab_words, int(tw));
      // two-pass DFT extents: pass-1 groups of G slabs (S = B / B_0 buckets
      // each, G S <= kSplitGroup, or one slab of up to kSplitMaxSlab),
      // pass-2 groups of min(S, 32) columns
      const int b0 = d.b[0];
      const int S = d.B / b0;
      if (d.ndim < 2 || S > rsft::kSplitMaxSlab || d.noise_mode != RSFT_NOISE_KNOWN) {
        pl->split_ok = 0;
      } else {
        const int G = S >= rsft::kSplitGroup ? 1 : std::min(rsft::kSplitGroup / S, b0);
        pl->split_b0 = std::max(pl->split_b0, b0);
        pl->split_g1 = std::max(pl->split_g1, b0 / G);
        pl->split_e1 = std::max(pl->split_e1, G * S);
        pl->split_g2 = std::max(pl->split_g2, S / std::min(S, 32));
      }
    }
    int sum_tw = 0;
    for (int k = 0; k < d.ndim; ++k) sum_tw += d.b[k];
    pl->sum_tw_max = std::max(pl->sum_tw_max, sum_tw);
  }
  choose_vote_path(pl);
  pl->dft_threads = pl->maxB <= 256 ? 64 : pl->maxB <= 1024 ? 256 : 1024;
  // chunks per frame are a power of two (N is); few of them: several frames
  // per scan work-group
  if (pl->uniform && pl->descs[0].cchunks <= 128) pl->scan_fpb = 256 / pl->descs[0].cchunks;
  // the DFT stage keeps two planes of B floats plus the twiddles in LDS;
  // padding of the last dimension's rows (against bank conflicts) is used
  // when it fits
  const size_t lds_limit = 160 * 1024;
  const size_t tw_bytes = size_t(pl->sum_tw_max) * 8;
  if (size_t(2 * pl->dft_plane) * 4 + tw_bytes <= lds_limit) {
    pl->dft_pad = 1;
  } else if (size_t(2 * pl->maxB) * 4 + tw_bytes <= lds_limit) {
    pl->dft_pad = 0;
    pl->dft_plane = pl->maxB;
  } else {
    return fail(RSFT_ERROR_UNSUPPORTED, "buckets per frame exceed the DFT stage's LDS");
  }

  // fold tiles
  std::vector<int32_t> tiles;
  if (pl->uniform) {
    pl->tiles_per_frame = int64_t(pl->descs[0].classes / pl->descs[0].fold_cpt) * pl->descs[0].nchunks;
  } else {
    struct Tile { int64_t bytes; int32_t f, c, k; };
    std::vector<Tile> tl;
    for (int64_t i = 0; i < nframes; ++i) {
      const auto& d = pl->descs[size_t(i)];
      const int64_t bytes = int64_t(d.rows_per_class) * std::min<int64_t>(d.chunk_cols, d.fold_nl) * d.fold_cpt;
      for (int c = 0; c < d.classes; c += d.fold_cpt)
        for (int k = 0; k < d.nchunks; ++k) tl.push_back({bytes, int32_t(i), c, k});
    }
    // largest tiles first: the hardware dispatcher then balances the tail
    std::stable_sort(tl.begin(), tl.end(), [](const Tile& a, const Tile& b) { return a.bytes > b.bytes; });
    for (const auto& t : tl) {
      tiles.push_back(t.f);
      tiles.push_back(t.c);
      tiles.push_back(t.k);
    }
    pl->ntiles_uneven = int64_t(tl.size());
  }
  // DFT order of an uneven batch: frames by decreasing bucket count (stable),
  // so that the largest transforms, one work-group each, start first
  std::vector<int32_t> dft_order;
  if (!pl->uniform) {
    for (int64_t i = 0; i < nframes; ++i) dft_order.push_back(int32_t(i));
    std::stable_sort(dft_order.begin(), dft_order.end(), [&](int32_t a, int32_t b) {
      return pl->descs[size_t(a)].B > pl->descs[size_t(b)].B;
    });
  }
  // compaction chunks of an uneven batch: when frames differ in chunk count,
  // the vote and estimate launches take one work-group per listed chunk
  // instead of a frames x max-chunks grid that is mostly empty. Position p
  // holds a frame congruent to p mod 8 when the estimate groups frames by
  // XCD (16 frames or more), as its grid does.
  std::vector<int32_t> chunk_list;
  if (!pl->uniform) {
    int64_t total = 0;
    for (const auto& d : pl->descs) total += d.cchunks;
    if (total < int64_t(pl->max_cchunks) * nframes) {
      const int groups = nframes >= 16 ? 8 : 1;
      std::vector<std::vector<std::pair<int32_t, int32_t>>> q(static_cast<size_t>(groups));
      for (int64_t i = 0; i < nframes; ++i)
        for (int32_t c = 0; c < pl->descs[size_t(i)].cchunks; ++c)
          q[size_t(i % groups)].push_back({int32_t(i), c});
      size_t len = 0;
      for (const auto& v : q) len = std::max(len, v.size());
      for (size_t k = 0; k < len; ++k)
        for (const auto& v : q) {
          chunk_list.push_back(k < v.size() ? v[k].first : -1);
          chunk_list.push_back(k < v.size() ? v[k].second : -1);
        }
      pl->nchunk_list = int64_t(chunk_list.size() / 2);
    }
  }

  // word-parallel vote: per descriptor and round, M_s[b][w] with bit x of
  // word w set when cell 32 w + x of a row lies in bucket column b, i.e.
  // the preimages x = [sigma_inv u] of u in [b L, (b + 1) L) (Def. 4); per
  // frame the workspace of its bucket-row masks, [T][B / B_last][W] words;
  // and for uneven plans whose frames differ in chunk count, the list of
  // (frame, first chunk) groups of kVoteCpw chunks
  std::vector<uint32_t> vote_tab;
  std::vector<int32_t> vote_list, vote_exp_list;
  int64_t vexp_off = 0;
  if (pl->words_ok) {
    for (auto& d : pl->descs) {
      const int D = d.ndim;
      const uint32_t nl = uint32_t(d.n[D - 1]);
      const uint32_t W = nl / 32;
      const uint32_t bl = uint32_t(d.b[D - 1]);
      const int lsl = d.lshift[D - 1];
      const int64_t ew = int64_t(d.B / int32_t(bl)) * W;
      d.vexp_off = vexp_off;
      d.vexp_stride = int64_t(d.T) * ew;
      vexp_off += (pl->uniform ? pl->max_frames : 1) * d.vexp_stride;
      pl->exp_blocks = std::max(pl->exp_blocks, int((ew + rsft::kVoteExpWords - 1) / rsft::kVoteExpWords));
      d.vtab_off = int64_t(vote_tab.size());
      vote_tab.resize(vote_tab.size() + size_t(d.T) * bl * W, 0u);
      uint32_t* t0 = vote_tab.data() + d.vtab_off;
      for (int r = 0; r < d.T; ++r) {
        uint32_t* tr = t0 + size_t(r) * bl * W;
        const uint64_t sinv = uint64_t(uint32_t(d.sigma_inv[r][D - 1]));
        for (uint32_t u = 0; u < nl; ++u) {
          const uint32_t x = uint32_t((sinv * u) % nl);
          tr[(u >> lsl) * W + (x >> 5)] |= 1u << (x & 31u);
        }
      }
    }
    if (!pl->uniform) {
      // mask blocks of every frame, largest frames first
      for (int64_t k = 0; k < nframes; ++k) {
        const int32_t i = dft_order[size_t(k)];
        const auto& d = pl->descs[size_t(i)];
        const int64_t ew = int64_t(d.B / d.b[d.ndim - 1]) * (d.n[d.ndim - 1] / 32);
        for (int64_t b = 0; b * rsft::kVoteExpWords < ew; ++b) {
          vote_exp_list.push_back(i);
          vote_exp_list.push_back(int32_t(b));
        }
      }
      pl->nexp_list = int64_t(vote_exp_list.size() / 2);
    }
    if (!pl->uniform && pl->nchunk_list > 0) {
      for (int64_t i = 0; i < nframes; ++i)
        for (int32_t c = 0; c < pl->descs[size_t(i)].cchunks; c += rsft::kVoteCpw) {
          vote_list.push_back(int32_t(i));
          vote_list.push_back(c);
        }
      pl->nvote_list = int64_t(vote_list.size() / 2);
    }
  }

  rsft_status st;
  if ((st = upload(pl->d_descs, pl->descs)) != RSFT_OK) return st;
  if ((st = upload(pl->d_vote_tab, vote_tab)) != RSFT_OK) return st;
  if ((st = upload(pl->d_vote_list, vote_list)) != RSFT_OK) return st;
  if ((st = upload(pl->d_vote_exp_list, vote_exp_list)) != RSFT_OK) return st;
  if ((st = upload(pl->d_wrow, ht.wrow)) != RSFT_OK) return st;
  if ((st = upload(pl->d_wcol, ht.wcol)) != RSFT_OK) return st;
  if ((st = upload(pl->d_rowlist, ht.rowlist)) != RSFT_OK) return st;
  if ((st = upload(pl->d_tw, ht.tw)) != RSFT_OK) return st;
  if ((st = upload(pl->d_gains, ht.inv_gains)) != RSFT_OK) return st;
  if ((st = upload(pl->d_win, ht.win)) != RSFT_OK) return st;
  if ((st = upload(pl->d_flat, ht.flat)) != RSFT_OK) return st;
  if ((st = upload(pl->d_tiles, tiles)) != RSFT_OK) return st;
  if ((st = upload(pl->d_chunk_list, chunk_list)) != RSFT_OK) return st;
  if ((st = upload(pl->d_dft_order, dft_order)) != RSFT_OK) return st;
  if ((st = alloc(pl->d_part, size_t(part_off) * sizeof(float2))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_buckets, size_t(bucket_off) * sizeof(float2))) != RSFT_OK) return st;
  if (pl->split_ok && (st = alloc(pl->d_inter, size_t(bucket_off) * sizeof(float2))) != RSFT_OK) return st;
  if (pl->words_ok && (st = alloc(pl->d_vote_exp, size_t(vexp_off) * sizeof(uint32_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_powers, size_t(bucket_off) * sizeof(float))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_flags, size_t(flag_off) * sizeof(uint32_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_bitmap, size_t(bitmap_off) * sizeof(uint32_t))) != RSFT_OK) return st;
  HIP_TRY(hipMemset(pl->d_bitmap.ptr, 0, pl->d_bitmap.bytes));  // kept clear by the compaction
  if ((st = alloc(pl->d_chunk_counts, size_t(chunk_off) * sizeof(uint32_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_chunk_offsets, size_t(chunk_off) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_counts, size_t(pl->max_frames) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_offsets, size_t(pl->max_frames + 1) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_chunk_items, size_t(chunk_off) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_item_counts, size_t(pl->max_frames) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_item_offsets, size_t(pl->max_frames + 1) * sizeof(int64_t))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_records, size_t(rec_total) * sizeof(rsft::DetRec))) != RSFT_OK) return st;
  if ((st = alloc(pl->d_scan_done, sizeof(uint32_t))) != RSFT_OK) return st;
  HIP_TRY(hipMemset(pl->d_scan_done.ptr, 0, sizeof(uint32_t)));   // the scan keeps it 0 between launches
  HIP_TRY(hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking));

  auto& q = pl->ptrs;
  q.descs = static_cast<const rsft::FrameDesc*>(pl->d_descs.ptr);
  q.uniform = pl->uniform ? 1 : 0;
  q.wrow = static_cast<const float2*>(pl->d_wrow.ptr);
  q.wcol = static_cast<const float2*>(pl->d_wcol.ptr);
  q.rowlist = static_cast<const int32_t*>(pl->d_rowlist.ptr);
  q.tw = static_cast<const float2*>(pl->d_tw.ptr);
  q.inv_gains = static_cast<const float*>(pl->d_gains.ptr);
  q.win = static_cast<const float*>(pl->d_win.ptr);
  q.flat = static_cast<const float2*>(pl->d_flat.ptr);
  q.part = static_cast<float2*>(pl->d_part.ptr);
  q.buckets = static_cast<float2*>(pl->d_buckets.ptr);
  q.powers = static_cast<float*>(pl->d_powers.ptr);
  q.flags = static_cast<uint32_t*>(pl->d_flags.ptr);
  q.bitmap = static_cast<uint32_t*>(pl->d_bitmap.ptr);
  q.chunk_counts = static_cast<uint32_t*>(pl->d_chunk_counts.ptr);
  q.chunk_offsets = static_cast<int64_t*>(pl->d_chunk_offsets.ptr);
  q.counts = static_cast<int64_t*>(pl->d_counts.ptr);
  q.offsets = static_cast<int64_t*>(pl->d_offsets.ptr);
  q.chunk_items = static_cast<int64_t*>(pl->d_chunk_items.ptr);
  q.item_counts = static_cast<int64_t*>(pl->d_item_counts.ptr);
  q.item_offsets = static_cast<int64_t*>(pl->d_item_offsets.ptr);
  q.records = static_cast<rsft::DetRec*>(pl->d_records.ptr);
  q.scan_done = static_cast<uint32_t*>(pl->d_scan_done.ptr);
  q.tiles = static_cast<const int32_t*>(pl->d_tiles.ptr);
  q.chunk_list = static_cast<const int32_t*>(pl->d_chunk_list.ptr);
  q.vote_tab = static_cast<const uint32_t*>(pl->d_vote_tab.ptr);
  q.vote_list = static_cast<const int32_t*>(pl->d_vote_list.ptr);
  q.vote_exp = static_cast<uint32_t*>(pl->d_vote_exp.ptr);
  q.vote_exp_list = static_cast<const int32_t*>(pl->d_vote_exp_list.ptr);
  return RSFT_OK;
}

rsft_status check_batch(rsft_plan_s* pl, const void* d_input, int64_t batch) {
  if (batch < 0) return fail(RSFT_ERROR_INVALID_ARGUMENT, "batch must be >= 0");
  if (pl->uniform) {
    if (batch > pl->max_frames) return fail(RSFT_ERROR_INVALID_ARGUMENT, "batch exceeds max_batch of the plan");
  } else if (batch != 0 && batch != pl->ndesc) {
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "an uneven plan executes exactly its frames");
  }
  if (batch > 0 && d_input == nullptr) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL input");
  if (reinterpret_cast<uintptr_t>(d_input) % 16 != 0)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "input must be 16-byte aligned");
  return RSFT_OK;
}

// Stage 1 (window, permutation, flat window, aliasing), all round groups.
rsft_status fold_stage(rsft_plan_s* pl, const void* d_input, int64_t batch, hipStream_t st,
                       const rsft::FoldConfig& cfg) {
  const auto& q = pl->ptrs;
  const int64_t ntiles = pl->uniform ? batch * pl->tiles_per_frame : pl->ntiles_uneven;
  if (ntiles >= (int64_t(1) << 31)) return fail(RSFT_ERROR_UNSUPPORTED, "more than 2^31 fold tiles");
  if (pl->segments) {
    // round s folds segment s of every frame (the kernels offset by s * N)
    for (int r = 0; r < pl->T; ++r)
      LAUNCH_TRY(rsft::launch_fold(q, d_input, pl->dtype, batch, pl->tiles_per_frame, ntiles, r, 1, pl->T,
                                   cfg, st));
    return RSFT_OK;
  }
  for (int r0 = 0; r0 < pl->T; r0 += rsft::kFoldRoundGroup) {
    const int rounds = std::min(rsft::kFoldRoundGroup, pl->T - r0);
    LAUNCH_TRY(rsft::launch_fold(q, d_input, pl->dtype, batch, pl->tiles_per_frame, ntiles, r0, rounds,
                                 pl->T, cfg, st));
  }
  return RSFT_OK;
}

void drop_graphs(rsft_plan_s* pl) {
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
  pl->graphs.clear();
  pl->graph_order.clear();
}

// scan + compact/estimate, in the plan's estimate layout
rsft_status estimate_stage(rsft_plan_s* pl, int64_t batch, hipStream_t st) {
  const auto& q = pl->ptrs;
  LAUNCH_TRY(rsft::launch_scan(q, batch, pl->est_workers, pl->scan_fpb, st));
  LAUNCH_TRY(rsft::launch_estimate(q, batch, pl->T, pl->max_cchunks, pl->dims_mask, pl->est_nmask,
                                   pl->est_workers, pl->num_cus, pl->nchunk_list, pl->global_gains, st));
  return RSFT_OK;
}

// B-point DFT, threshold and flags of every round of the batch: the two-
// pass kernels where they apply and are chosen, else one work-group per
// (round, frame).
rsft_status dft_stage(rsft_plan_s* pl, int64_t batch, hipStream_t st) {
  const int32_t* order = pl->uniform ? nullptr : static_cast<const int32_t*>(pl->d_dft_order.ptr);
  if (pl->split_ok && pl->dft_split) {
    LAUNCH_TRY(rsft::launch_dft_split(pl->ptrs, batch, pl->T, pl->split_b0, pl->split_g1, pl->split_g2,
                                      pl->split_e1, pl->sum_tw_max, static_cast<float2*>(pl->d_inter.ptr),
                                      order, st));
  } else {
    LAUNCH_TRY(rsft::launch_dft(pl->ptrs, batch, pl->T, pl->dft_plane, pl->dft_pad, pl->sum_tw_max, 0, 0,
                                order, pl->dft_threads, st));
  }
  return RSFT_OK;
}

// Reverse mapping, accumulation and second stage for the whole batch.
rsft_status vote_stage(rsft_plan_s* pl, int64_t batch, hipStream_t st) {
  LAUNCH_TRY(rsft::launch_vote(pl->ptrs, batch, pl->T, pl->mu, pl->max_cchunks, pl->max_words, pl->dims_mask,
                               pl->vote_path, 0, pl->nchunk_list, pl->nvote_list, pl->tab_words, pl->exp_blocks, pl->nexp_list, st));
  return RSFT_OK;
}

// The hot path, stage by stage; `ev` (optional) brackets the stages.
// the stages after the fold: DFT + threshold, vote, scan + compact/estimate
rsft_status enqueue_tail(rsft_plan_s* pl, int64_t batch, hipStream_t st, hipEvent_t* ev) {
  {
    const rsft_status ds = dft_stage(pl, batch, st);
    if (ds != RSFT_OK) return ds;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[2], st));
  {
    const rsft_status vs = vote_stage(pl, batch, st);
    if (vs != RSFT_OK) return vs;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[3], st));
  {
    const rsft_status es = estimate_stage(pl, batch, st);
    if (es != RSFT_OK) return es;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[4], st));
  return RSFT_OK;
}

rsft_status enqueue(rsft_plan_s* pl, const void* d_input, int64_t batch, hipStream_t st,
                    hipEvent_t* ev) {
  if (ev) HIP_TRY(hipEventRecord(ev[0], st));
  {
    const rsft_status fs = fold_stage(pl, d_input, batch, st, pl->fold);
    if (fs != RSFT_OK) return fs;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[1], st));
  return enqueue_tail(pl, batch, st, ev);
}

// Replays the captured launch sequence of `key` on `user`, capturing it
// from `body(stream)` first when it is not cached (at most 8 kept).
template <class Body>
rsft_status replay(rsft_plan_s* pl, const std::tuple<int, const void*, int64_t>& key, hipStream_t user,
                   Body&& body) {
  auto it = pl->graphs.find(key);
  if (it == pl->graphs.end()) {
    if (pl->graphs.size() >= 8) {
      const auto old = pl->graph_order.front();
      pl->graph_order.erase(pl->graph_order.begin());
      (void)hipGraphExecDestroy(pl->graphs[old]);
      pl->graphs.erase(old);
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal));
    const rsft_status st = body(pl->capture_stream);
    hipError_t e = hipStreamEndCapture(pl->capture_stream, &graph);
    if (st != RSFT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(RSFT_ERROR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(RSFT_ERROR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = pl->graphs.emplace(key, exec).first;
    pl->graph_order.push_back(key);
  }
  HIP_TRY(hipGraphLaunch(it->second, user));
  return RSFT_OK;
}

rsft_status drain_timing(rsft_plan_s* pl, TimingSet& ts) {
  if (!ts.pending) return RSFT_OK;
  HIP_TRY(hipEventSynchronize(ts.ev[RSFT_NUM_STAGES]));
  for (int k = 0; k < RSFT_NUM_STAGES; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ts.ev[k], ts.ev[k + 1]));
    pl->stage_ms[k] += ms;
  }
  pl->timed += 1;
  ts.pending = false;
  return RSFT_OK;
}

}  // namespace

extern "C" {

namespace {

// Launch shapes chosen by rsft_autotune, kept for the life of the process
// per plan signature: a later plan of the same signature starts from them.
struct TunedShapes {
  rsft::FoldConfig fold;
  int dft_split, dft_threads, vote_words, est_workers;
};
std::mutex g_tuned_mu;
std::map<std::string, TunedShapes> g_tuned;

// Device, batch layout, rounds, mu, dtype, segment mode and every frame's
// shape, buckets and noise mode: what the tuned launch shapes depend on
// (sigma, windows and Pfa do not change them).
std::string plan_signature(const rsft_plan_s* pl) {
  std::string k = std::to_string(pl->device) + ";" + std::to_string(pl->uniform) + ";" +
                  std::to_string(pl->max_frames) + ";" + std::to_string(pl->T) + ";" + std::to_string(pl->mu) +
                  ";" + std::to_string(pl->dtype) + ";" + std::to_string(pl->segments);
  for (const auto& d : pl->descs) {
    k += ";" + std::to_string(d.noise_mode);
    for (int dd = 0; dd < d.ndim; ++dd) k += "," + std::to_string(d.n[dd]) + "/" + std::to_string(d.b[dd]);
  }
  return k;
}

void remember_tuning(const rsft_plan_s* pl) {
  const TunedShapes t{pl->fold, pl->dft_split, pl->dft_threads, pl->vote_words, pl->est_workers};
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  g_tuned[plan_signature(pl)] = t;
}

void apply_remembered_tuning(rsft_plan_s* pl) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  const auto it = g_tuned.find(plan_signature(pl));
  if (it == g_tuned.end()) return;
  pl->fold = it->second.fold;
  pl->dft_split = it->second.dft_split;
  pl->dft_threads = it->second.dft_threads;
  pl->vote_words = it->second.vote_words;
  choose_vote_path(pl);
  pl->est_workers = it->second.est_workers;
}

}  // namespace

rsft_status rsft_plan(const rsft_params* frames, int64_t nframes, rsft_plan_t* out) {
  if (out) *out = nullptr;
  if (!frames || !out || nframes < 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument or nframes < 1");
  // argument errors are reported before any device call
  for (int64_t i = 0; i < nframes; ++i) {
    const rsft_status vs = validate(frames[i], i);
    if (vs != RSFT_OK) return vs;
    const int mu_i = frames[i].mu == 0 ? frames[i].rounds : frames[i].mu;
    const int mu_0 = frames[0].mu == 0 ? frames[0].rounds : frames[0].mu;
    if (frames[i].rounds != frames[0].rounds || mu_i != mu_0 || frames[i].dtype != frames[0].dtype ||
        frames[i].segments != frames[0].segments)
      return fail(RSFT_ERROR_INVALID_ARGUMENT,
                  "rounds, mu, dtype and segments must agree across frame descriptors");
  }
  auto* pl = new (std::nothrow) rsft_plan_s();
  if (!pl) return fail(RSFT_ERROR_OUT_OF_MEMORY, "host allocation failed");
  if (hipGetDevice(&pl->device) != hipSuccess) {
    delete pl;
    return fail(RSFT_ERROR_DEVICE, "no HIP device");
  }
  rsft_status st;
  try {
    st = create_plan(frames, nframes, pl);
  } catch (const std::bad_alloc&) {
    st = fail(RSFT_ERROR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    st = fail(RSFT_ERROR_INVALID_ARGUMENT, e.what());
  }
  if (st != RSFT_OK) {
    free_plan(pl);
    return st;
  }
  apply_remembered_tuning(pl);
  *out = pl;
  return RSFT_OK;
}

rsft_status rsft_execute(rsft_plan_t pl, const void* d_input, int64_t batch, void* stream) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  rsft_status st = check_batch(pl, d_input, batch);
  if (st != RSFT_OK) return st;
  hipStream_t user = static_cast<hipStream_t>(stream);
  pl->last_batch = batch;
  pl->folded_batch = -1;
  if (batch == 0) return RSFT_OK;
  if (pl->timing) {
    if (pl->timing_sets.empty()) {
      pl->timing_sets.resize(64);
      for (auto& ts : pl->timing_sets)
        for (auto& e : ts.ev) HIP_TRY(hipEventCreate(&e));
    }
    TimingSet& ts = pl->timing_sets[pl->timing_next];
    pl->timing_next = (pl->timing_next + 1) % pl->timing_sets.size();
    if ((st = drain_timing(pl, ts)) != RSFT_OK) return st;
    if ((st = enqueue(pl, d_input, batch, user, ts.ev)) != RSFT_OK) return st;
    ts.pending = true;
    return RSFT_OK;
  }
  if (!pl->use_graph) return enqueue(pl, d_input, batch, user, nullptr);
  return replay(pl, std::make_tuple(0, d_input, batch), user,
                [&](hipStream_t cs) { return enqueue(pl, d_input, batch, cs, nullptr); });
}

rsft_status rsft_execute_fold(rsft_plan_t pl, const void* d_input, int64_t batch, void* stream) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  rsft_status st = check_batch(pl, d_input, batch);
  if (st != RSFT_OK) return st;
  hipStream_t user = static_cast<hipStream_t>(stream);
  pl->folded_batch = batch;
  if (batch == 0) return RSFT_OK;
  auto body = [&](hipStream_t cs) { return fold_stage(pl, d_input, batch, cs, pl->fold); };
  if (!pl->use_graph || pl->timing) return body(user);
  return replay(pl, std::make_tuple(1, d_input, batch), user, body);
}

rsft_status rsft_execute_tail(rsft_plan_t pl, void* stream) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (pl->folded_batch < 0) return fail(RSFT_ERROR_NOT_READY, "rsft_execute_tail without a preceding rsft_execute_fold");
  const int64_t batch = pl->folded_batch;
  pl->folded_batch = -1;
  pl->last_batch = batch;
  if (batch == 0) return RSFT_OK;
  hipStream_t user = static_cast<hipStream_t>(stream);
  auto body = [&](hipStream_t cs) { return enqueue_tail(pl, batch, cs, nullptr); };
  if (!pl->use_graph || pl->timing) return body(user);
  return replay(pl, std::make_tuple(2, static_cast<const void*>(nullptr), batch), user, body);
}

rsft_status rsft_autotune(rsft_plan_t pl, const void* d_input, int64_t batch, void* stream,
                          int32_t repeats, double* best_ms) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  rsft_status st = check_batch(pl, d_input, batch);
  if (st != RSFT_OK) return st;
  if (batch == 0) return RSFT_OK;
  if (repeats <= 0) repeats = 5;
  pl->folded_batch = -1;   // the timed folds overwrite a pending fold's partial buckets
  hipStream_t s = static_cast<hipStream_t>(stream);
  struct Events {  // released on every return path
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  HIP_TRY(hipEventCreate(&ev.e[0]));
  HIP_TRY(hipEventCreate(&ev.e[1]));
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
  rsft::FoldConfig best = pl->fold;
  float best_t = 1e30f;
  // two passes over the shapes, each shape keeping its faster pass: a
  // single timing of an HBM-bound launch varies by a few percent, about as
  // much as the shapes differ
  for (int pass = 0; pass < 2; ++pass)
  for (int threads : {256, 512})
    for (int vec : {4, 2})
      for (int nt : {0, 1}) {
        if (vec == 4 && pl->min_nl < 4) continue;
        if (st != RSFT_OK) break;
        const rsft::FoldConfig cfg{threads, vec, nt};
        if ((st = fold_stage(pl, d_input, batch, s, cfg)) != RSFT_OK) break;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < repeats && st == RSFT_OK; ++r) st = fold_stage(pl, d_input, batch, s, cfg);
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms /= float(repeats);
        if (st == RSFT_OK && ms < best_t) {
          best_t = ms;
          best = cfg;
        }
      }
  if (st != RSFT_OK) return st;
  pl->fold = best;
  // DFT: one work-group per transform at each work-group size, and the
  // two-pass kernels where they apply; the fold of d_input leaves the
  // partial buckets all of them read
  {
    if ((st = fold_stage(pl, d_input, batch, s, pl->fold)) != RSFT_OK) return st;
    float best_ms = 0.f;
    int best_split = 0, best_threads = pl->dft_threads;
    bool have = false;
    for (int v = 0; v < 4; ++v) {
      const int threads = v == 0 ? 64 : v == 1 ? 256 : 1024;
      if (v == 3 && !pl->split_ok) break;
      pl->dft_split = v == 3 ? 1 : 0;
      if (v < 3) pl->dft_threads = threads;
      if ((st = dft_stage(pl, batch, s)) != RSFT_OK) return st;
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < repeats && st == RSFT_OK; ++r) st = dft_stage(pl, batch, s);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      if (st != RSFT_OK) return st;
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (!have || ms < best_ms) {
        have = true;
        best_ms = ms;
        best_split = pl->dft_split;
        if (v < 3) best_threads = threads;
      }
    }
    pl->dft_split = best_split;
    pl->dft_threads = best_threads;
  }
  // estimate layout: one execute of d_input leaves its flags and detected-
  // cell bitmap; scan + compact/estimate (which only read those) are then
  // timed without and with overflow workers. Dense chunks favour the
  // workers; the workers are kept only when clearly faster.
  if ((st = enqueue(pl, d_input, batch, s, nullptr)) != RSFT_OK) return st;
  pl->last_batch = batch;
  // vote kernel, where both the word-parallel masks and the candidate
  // enumeration apply: which is faster depends on B_last, L_last and how
  // many buckets the data flag; the faster on d_input's flags is kept (the
  // vote only reads the flags, and both write the same bitmap)
  if (pl->words_ok && pl->rows_ok && pl->T <= 4) {
    float vote_ms[2] = {0.f, 0.f};
    for (int v = 0; v < 2; ++v) {
      pl->vote_words = v;
      choose_vote_path(pl);
      if ((st = vote_stage(pl, batch, s)) != RSFT_OK) return st;
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < repeats && st == RSFT_OK; ++r) st = vote_stage(pl, batch, s);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      if (st != RSFT_OK) return st;
      HIP_TRY(hipEventElapsedTime(&vote_ms[v], e0, e1));
    }
    pl->vote_words = vote_ms[1] <= vote_ms[0] ? 1 : 0;
    choose_vote_path(pl);
  }
  float est_ms[2] = {0.f, 0.f};
  for (int w = 0; w < 2; ++w) {
    pl->est_workers = w;
    if ((st = estimate_stage(pl, batch, s)) != RSFT_OK) return st;
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < repeats && st == RSFT_OK; ++r) st = estimate_stage(pl, batch, s);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    if (st != RSFT_OK) return st;
    HIP_TRY(hipEventElapsedTime(&est_ms[w], e0, e1));
  }
  pl->est_workers = est_ms[1] < 0.97f * est_ms[0] ? 1 : 0;
  drop_graphs(pl);   // captured graphs hold the previous launch shape
  remember_tuning(pl);
  if (best_ms) *best_ms = double(best_t);
  return RSFT_OK;
}

rsft_status rsft_execute_per_frame(rsft_plan_t pl, const void* d_input, int64_t batch, void* stream) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  rsft_status st = check_batch(pl, d_input, batch);
  if (st != RSFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  pl->last_batch = batch;
  const auto& q = pl->ptrs;
  for (int64_t f = 0; f < batch; ++f) {
    const auto& d = pl->descs[size_t(pl->uniform ? 0 : f)];
    for (int r = 0; r < pl->T; ++r) LAUNCH_TRY(rsft::launch_plain_fold(q, d_input, pl->dtype, f, r, d.B, s));
    LAUNCH_TRY(rsft::launch_plain_dft(q, f, pl->T, pl->dft_plane, pl->dft_pad, pl->sum_tw_max, s));
    LAUNCH_TRY(rsft::launch_vote(q, 1, pl->T, pl->mu, pl->max_cchunks, pl->max_words, pl->dims_mask, pl->vote_path, int(f), 0, 0, pl->tab_words, pl->exp_blocks, 0, s));
  }
  if (batch > 0) {
    const rsft_status es = estimate_stage(pl, batch, s);
    if (es != RSFT_OK) return es;
  }
  return RSFT_OK;
}

namespace {
rsft_status check_model(rsft_plan_s* pl, int64_t batch, int32_t tones) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (tones < 1 || tones > 65536) return fail(RSFT_ERROR_INVALID_ARGUMENT, "tones must be in 1..65536");
  if (batch < 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, "batch must be >= 1");
  if (pl->uniform ? batch > pl->max_frames : batch != pl->ndesc)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "batch does not match the plan");
  if (batch > 65535) return fail(RSFT_ERROR_UNSUPPORTED, "more than 65535 frames per model call");
  if ((pl->dims_mask & (pl->dims_mask - 1)) != 0)
    return fail(RSFT_ERROR_UNSUPPORTED, "the model needs one dimension count across descriptors");
  if (pl->segments)
    return fail(RSFT_ERROR_UNSUPPORTED, "the model describes one frame seen by every round, not segments");
  return RSFT_OK;
}

int64_t model_factor_count(const rsft_plan_s* pl, int64_t batch, int32_t tones) {
  return batch * pl->T * int64_t(tones) * pl->sum_tw_max;   // complex values per factor array
}
}  // namespace

rsft_status rsft_model_workspace_size(rsft_plan_t pl, int64_t batch, int32_t tones, int64_t* bytes) {
  if (!bytes) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  const rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  *bytes = 2 * model_factor_count(pl, batch, tones) * int64_t(sizeof(float) * 2);
  return RSFT_OK;
}

rsft_status rsft_model_forward(rsft_plan_t pl, const double* d_freqs, const void* d_amps,
                               int64_t batch, int32_t tones, void* d_model, void* d_workspace,
                               void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_freqs || !d_amps || !d_model || !d_workspace) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  const int D = pl->descs[0].ndim;
  float2* G = static_cast<float2*>(d_workspace);
  float2* dG = G + model_factor_count(pl, batch, tones);
  LAUNCH_TRY(rsft::launch_model_forward(pl->ptrs, d_freqs, static_cast<const float2*>(d_amps), batch,
                                        tones, D, pl->T, pl->maxB, pl->sum_tw_max, G, dG,
                                        static_cast<float2*>(d_model), stream));
  return RSFT_OK;
}

rsft_status rsft_model_forward_noalloc(rsft_plan_t pl, const double* d_freqs, const void* d_amps,
                                       int64_t batch, int32_t tones, void* d_model, void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_freqs || !d_amps || !d_model) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  const int64_t need = 2 * model_factor_count(pl, batch, tones) * int64_t(sizeof(float) * 2);
  if (need > int64_t(RSFT_STATIC_SCRATCH_BYTES))
    return fail(RSFT_ERROR_UNSUPPORTED, "model factors need " + std::to_string(need) +
                                            " bytes, more than the static scratch of " +
                                            std::to_string(int64_t(RSFT_STATIC_SCRATCH_BYTES)) +
                                            " bytes (2 * batch * T * tones * sum_d B_d * 8)");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != pl->device) return fail(RSFT_ERROR_INVALID_ARGUMENT, "the current device is not the plan's device");
  void* ws = nullptr;
  LAUNCH_TRY(rsft::static_scratch(cur, &ws));
  const int D = pl->descs[0].ndim;
  float2* G = static_cast<float2*>(ws);
  float2* dG = G + model_factor_count(pl, batch, tones);
  LAUNCH_TRY(rsft::launch_model_forward(pl->ptrs, d_freqs, static_cast<const float2*>(d_amps), batch,
                                        tones, D, pl->T, pl->maxB, pl->sum_tw_max, G, dG,
                                        static_cast<float2*>(d_model), stream));
  return RSFT_OK;
}

rsft_status rsft_model_backward(rsft_plan_t pl, const void* d_amps, int64_t batch, int32_t tones,
                                const void* d_grad_model, double* d_grad_freqs, void* d_grad_amps,
                                double* d_step_freqs, void* d_step_amps, const void* d_workspace,
                                void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_amps || !d_grad_model || !d_grad_freqs || !d_grad_amps || !d_workspace)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  if ((d_step_freqs == nullptr) != (d_step_amps == nullptr))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "step outputs: both or neither");
  const float2* G = static_cast<const float2*>(d_workspace);
  const float2* dG = G + model_factor_count(pl, batch, tones);
  LAUNCH_TRY(rsft::launch_model_backward(pl->ptrs, static_cast<const float2*>(d_amps), batch, tones,
                                         pl->T, pl->sum_tw_max, G, dG,
                                         static_cast<const float2*>(d_grad_model), d_grad_freqs,
                                         static_cast<float2*>(d_grad_amps), d_step_freqs,
                                         static_cast<float2*>(d_step_amps), stream));
  return RSFT_OK;
}

namespace {
// Observed buckets of a refinement: the caller's, or the plan's own from the
// last execute (which must have covered `batch` frames).
rsft_status observed_buckets(rsft_plan_s* pl, const void* d_observed, int64_t batch, const float2** out) {
  if (d_observed) {
    *out = static_cast<const float2*>(d_observed);
    return RSFT_OK;
  }
  if (pl->last_batch != batch)
    return fail(RSFT_ERROR_NOT_READY, "no observed buckets given and the last execute was not of this batch");
  *out = pl->ptrs.buckets;
  return RSFT_OK;
}

// Complex values of a model (bucket) array for `batch` frames.
int64_t model_values(const rsft_plan_s* pl, int64_t batch) {
  int64_t n = 0;
  for (int64_t f = 0; f < batch; ++f) n += pl->descs[size_t(pl->uniform ? 0 : f)].bucket_stride;
  return n;
}

// Byte layout of a refinement workspace (each part 256-byte aligned).
struct RefineLayout {
  int64_t G, dG, G2, dG2, model, radius, fcand, saved_f, saved_a, best, loss_now, skip, total;
};
RefineLayout refine_layout(const rsft_plan_s* pl, int64_t batch, int32_t tones) {
  auto up = [](int64_t v) { return (v + 255) / 256 * 256; };
  const int64_t fac = up(model_factor_count(pl, batch, tones) * 8);
  RefineLayout L{};
  L.G = 0;
  L.dG = L.G + fac;
  L.G2 = L.dG + fac;
  L.dG2 = L.G2 + fac;
  L.model = L.dG2 + fac;
  L.radius = L.model + up(model_values(pl, batch) * 8);
  L.fcand = L.radius + up(batch * tones * 8);
  L.saved_f = L.fcand + up(batch * tones * pl->descs[0].ndim * 8);
  L.saved_a = L.saved_f + up(batch * tones * pl->descs[0].ndim * 8);
  L.best = L.saved_a + up(batch * tones * 8);
  L.loss_now = L.best + up(batch * 8);
  L.skip = L.loss_now + up(batch * 8);
  L.total = L.skip + up(batch * 4);
  return L;
}
}  // namespace

rsft_status rsft_refine_workspace_size(rsft_plan_t pl, int64_t batch, int32_t tones, int64_t* bytes) {
  if (!bytes) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  const rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  *bytes = refine_layout(pl, batch, tones).total;
  return RSFT_OK;
}

rsft_status rsft_initial_amplitudes(rsft_plan_t pl, const void* d_observed, const double* d_freqs,
                                    int64_t batch, int32_t tones, void* d_amps, float* d_spread,
                                    void* d_workspace, void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_freqs || !d_amps || !d_workspace) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  const float2* obs = nullptr;
  if ((st = observed_buckets(pl, d_observed, batch, &obs)) != RSFT_OK) return st;
  float2* G = static_cast<float2*>(d_workspace);
  float2* dG = G + model_factor_count(pl, batch, tones);
  LAUNCH_TRY(rsft::launch_initial_amplitudes(pl->ptrs, d_freqs, batch, tones, pl->descs[0].ndim, pl->T,
                                             pl->maxB, pl->sum_tw_max, G, dG, obs,
                                             static_cast<float2*>(d_amps), d_spread, stream));
  return RSFT_OK;
}

rsft_status rsft_model_residual(rsft_plan_t pl, const void* d_observed, const double* d_freqs,
                                const void* d_amps, int64_t batch, int32_t tones,
                                const int32_t* d_tone_counts, void* d_residual, void* d_workspace,
                                void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_freqs || !d_amps || !d_residual || !d_workspace)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  const float2* obs = nullptr;
  if ((st = observed_buckets(pl, d_observed, batch, &obs)) != RSFT_OK) return st;
  if (static_cast<const void*>(obs) == d_residual)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "d_residual may not alias the observed buckets");
  float2* G = static_cast<float2*>(d_workspace);
  float2* dG = G + model_factor_count(pl, batch, tones);
  LAUNCH_TRY(rsft::launch_model_residual(pl->ptrs, obs, d_freqs, static_cast<const float2*>(d_amps), batch,
                                         tones, pl->descs[0].ndim, pl->T, pl->maxB, pl->sum_tw_max,
                                         d_tone_counts, G, dG, static_cast<float2*>(d_residual), stream));
  return RSFT_OK;
}

rsft_status rsft_refine(rsft_plan_t pl, const void* d_observed, double* d_freqs, void* d_amps, int64_t batch,
                        int32_t tones, const int32_t* d_tone_counts, int32_t steps, double trust_bins,
                        void* d_workspace, double* d_loss, void* stream) {
  rsft_status st = check_model(pl, batch, tones);
  if (st != RSFT_OK) return st;
  if (!d_freqs || !d_amps || !d_workspace) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL pointer");
  if (steps < 0 || steps > 100000) return fail(RSFT_ERROR_INVALID_ARGUMENT, "steps must be 0..100000");
  if (!(trust_bins > 0.0) || !std::isfinite(trust_bins))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "trust_bins must be > 0");
  const float2* obs = nullptr;
  if ((st = observed_buckets(pl, d_observed, batch, &obs)) != RSFT_OK) return st;
  const RefineLayout L = refine_layout(pl, batch, tones);
  char* base = static_cast<char*>(d_workspace);
  rsft::RefineWork w{};
  w.G = reinterpret_cast<float2*>(base + L.G);
  w.dG = reinterpret_cast<float2*>(base + L.dG);
  w.G2 = reinterpret_cast<float2*>(base + L.G2);
  w.dG2 = reinterpret_cast<float2*>(base + L.dG2);
  w.model = reinterpret_cast<float2*>(base + L.model);
  w.radius = reinterpret_cast<double*>(base + L.radius);
  w.fcand = reinterpret_cast<double*>(base + L.fcand);
  w.saved_f = reinterpret_cast<double*>(base + L.saved_f);
  w.saved_a = reinterpret_cast<float2*>(base + L.saved_a);
  w.best = reinterpret_cast<double*>(base + L.best);
  w.loss_now = reinterpret_cast<double*>(base + L.loss_now);
  w.skip = reinterpret_cast<int32_t*>(base + L.skip);
  LAUNCH_TRY(rsft::launch_refine(pl->ptrs, obs, d_freqs, static_cast<float2*>(d_amps), batch, tones,
                                 pl->descs[0].ndim, pl->T, pl->maxB, pl->sum_tw_max, steps, trust_bins,
                                 d_tone_counts, w, d_loss, stream));
  return RSFT_OK;
}

rsft_status rsft_vote_flags(rsft_plan_t pl, const uint32_t* d_flags, void* stream) {
  if (!pl || !d_flags) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  if (pl->last_batch < 0) return fail(RSFT_ERROR_NOT_READY, "no execute yet");
  const int64_t batch = pl->last_batch;
  if (batch == 0) return RSFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  size_t words = 0;
  for (int64_t f = 0; f < batch; ++f) words += size_t(pl->descs[size_t(pl->uniform ? 0 : f)].flag_stride);
  HIP_TRY(hipMemcpyAsync(pl->d_flags.ptr, d_flags, words * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  const auto& q = pl->ptrs;
  LAUNCH_TRY(rsft::launch_vote(q, batch, pl->T, pl->mu, pl->max_cchunks, pl->max_words, pl->dims_mask, pl->vote_path, 0, pl->nchunk_list, pl->nvote_list, pl->tab_words, pl->exp_blocks, pl->nexp_list, s));
  return estimate_stage(pl, batch, s);
}

rsft_status rsft_detection_count(rsft_plan_t pl, void* stream, int64_t* total) {
  if (!pl || !total) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  if (pl->last_batch < 0) return fail(RSFT_ERROR_NOT_READY, "no execute yet");
  const int64_t batch = pl->last_batch;
  *total = 0;
  if (batch == 0) return RSFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int64_t> counts(static_cast<size_t>(batch));
  HIP_TRY(hipMemcpy(counts.data(), pl->d_counts.ptr, counts.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  for (auto c : counts) *total += c;
  return RSFT_OK;
}

rsft_status rsft_detect(rsft_plan_t pl, void* stream, rsft_detection* h_out, int64_t capacity,
                        int64_t* h_counts, int64_t* n_written) {
  if (n_written) *n_written = 0;
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (capacity < 0 || (capacity > 0 && !h_out)) return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad output buffer");
  if (pl->last_batch < 0) return fail(RSFT_ERROR_NOT_READY, "no execute yet");
  const int64_t batch = pl->last_batch;
  if (batch == 0) return RSFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int64_t> counts(static_cast<size_t>(batch));
  std::vector<int64_t> offsets(static_cast<size_t>(batch + 1));
  HIP_TRY(hipMemcpy(counts.data(), pl->d_counts.ptr, counts.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(offsets.data(), pl->d_offsets.ptr, offsets.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  bool truncated = false;
  for (int64_t f = 0; f < batch; ++f) {
    if (h_counts) h_counts[f] = counts[size_t(f)];
    if (counts[size_t(f)] > pl->descs[size_t(pl->uniform ? 0 : f)].cap) truncated = true;
  }
  const int64_t stored = offsets[size_t(batch)];
  const int64_t ncopy = std::min(stored, capacity);
  if (ncopy > 0) {
    // the device keeps 32-byte records; form the ABI records here
    std::vector<rsft::DetRec> recs(static_cast<size_t>(ncopy));
    HIP_TRY(hipMemcpy(recs.data(), pl->d_records.ptr, size_t(ncopy) * sizeof(rsft::DetRec), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < ncopy; ++r) {
      const rsft::DetRec& src = recs[size_t(r)];
      const auto& d = pl->descs[size_t(pl->uniform ? 0 : src.frame)];
      const uint64_t cell = src.key & rsft::kKeyCellMask;
      rsft_detection& o = h_out[r];
      std::memset(&o, 0, sizeof(o));
      o.frame = int64_t(src.frame);
      o.votes = int32_t((src.key >> rsft::kKeyVotesShift) & 127u);
      o.is_peak = int32_t((src.key >> (rsft::kKeyVotesShift + 7)) & 1u);
      o.magnitude = src.magnitude;
      for (int k = 0; k < d.ndim; ++k) {
        const int64_t idx = int64_t(cell >> d.nshift[k]) & int64_t(d.n[k] - 1);
        // N_d is a power of two: scaling by 2^-log2(N_d) is the division exactly
        double fr = std::ldexp(double(idx) + double(src.delta[k]), -ilog2(d.n[k]));
        if (fr < 0.0) fr += 1.0;
        if (fr >= 1.0) fr -= 1.0;
        o.idx[k] = idx;
        o.freq[k] = fr;
      }
    }
  }
  if (n_written) *n_written = std::max<int64_t>(ncopy, 0);
  if (ncopy < stored) truncated = true;
  if (truncated) return fail(RSFT_ERROR_CAPACITY, "detection records truncated; counts are exact");
  return RSFT_OK;
}

rsft_status rsft_get_buckets(rsft_plan_t pl, void* d_out, void* stream) {
  if (!pl || !d_out) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  if (pl->last_batch < 0) return fail(RSFT_ERROR_NOT_READY, "no execute yet");
  size_t n = 0;
  for (int64_t f = 0; f < pl->last_batch; ++f) n += size_t(pl->descs[size_t(pl->uniform ? 0 : f)].bucket_stride);
  if (n) HIP_TRY(hipMemcpyAsync(d_out, pl->d_buckets.ptr, n * sizeof(float2), hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(stream)));
  return RSFT_OK;
}

rsft_status rsft_get_flags(rsft_plan_t pl, uint32_t* d_out, void* stream) {
  if (!pl || !d_out) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  if (pl->last_batch < 0) return fail(RSFT_ERROR_NOT_READY, "no execute yet");
  size_t n = 0;
  for (int64_t f = 0; f < pl->last_batch; ++f) n += size_t(pl->descs[size_t(pl->uniform ? 0 : f)].flag_stride);
  if (n) HIP_TRY(hipMemcpyAsync(d_out, pl->d_flags.ptr, n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(stream)));
  return RSFT_OK;
}

rsft_status rsft_plan_info(rsft_plan_t pl, int64_t frame, rsft_plan_info_t* out) {
  if (!pl || !out) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  if (frame < 0 || frame >= pl->ndesc) return fail(RSFT_ERROR_INVALID_ARGUMENT, "frame out of range");
  *out = pl->info[size_t(frame)];
  out->fold_threads = pl->fold.threads;
  out->fold_vec = pl->fold.vec;
  out->fold_nontemporal = pl->fold.nontemporal;
  out->estimate_workers = pl->est_workers;
  out->vote_kernel = pl->vote_path;
  out->dft_two_pass = pl->split_ok && pl->dft_split ? 1 : 0;
  out->dft_threads = pl->dft_threads;
  return RSFT_OK;
}

rsft_status rsft_set_option(rsft_plan_t pl, int32_t option, int64_t value) {
  if (!pl) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL plan");
  switch (option) {
    case RSFT_OPT_GRAPH: pl->use_graph = value != 0; return RSFT_OK;
    case RSFT_OPT_TIMING: pl->timing = value != 0; return RSFT_OK;
    case RSFT_OPT_FOLD_THREADS:
      if (value != 256 && value != 512) return fail(RSFT_ERROR_INVALID_ARGUMENT, "fold threads: 256 or 512");
      pl->fold.threads = int(value);
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_FOLD_VEC:
      if (value != 2 && value != 4) return fail(RSFT_ERROR_INVALID_ARGUMENT, "fold vec: 2 or 4");
      if (value == 4 && pl->min_nl < 4) return fail(RSFT_ERROR_UNSUPPORTED, "rows shorter than 4 samples");
      pl->fold.vec = int(value);
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_FOLD_NONTEMPORAL:
      pl->fold.nontemporal = value != 0 ? 1 : 0;
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_VOTE_WORDS:
      if (value != 0 && value != 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, "RSFT_OPT_VOTE_WORDS must be 0 or 1");
      pl->vote_words = int(value);
      choose_vote_path(pl);
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_DFT_THREADS:
      if (value != 64 && value != 256 && value != 1024)
        return fail(RSFT_ERROR_INVALID_ARGUMENT, "RSFT_OPT_DFT_THREADS must be 64, 256 or 1024");
      pl->dft_threads = int(value);
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_DFT_SPLIT:
      if (value != 0 && value != 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, "RSFT_OPT_DFT_SPLIT must be 0 or 1");
      pl->dft_split = int(value);
      drop_graphs(pl);
      return RSFT_OK;
    case RSFT_OPT_ESTIMATE_WORKERS:
      pl->est_workers = value != 0 ? 1 : 0;
      drop_graphs(pl);
      return RSFT_OK;
    default: return fail(RSFT_ERROR_INVALID_ARGUMENT, "unknown option");
  }
}

rsft_status rsft_stage_times(rsft_plan_t pl, double* avg_ms, int64_t* count, int32_t reset) {
  if (!pl || !avg_ms) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  for (auto& ts : pl->timing_sets) {
    rsft_status st = drain_timing(pl, ts);
    if (st != RSFT_OK) return st;
  }
  for (int k = 0; k < RSFT_NUM_STAGES; ++k) avg_ms[k] = pl->timed ? pl->stage_ms[k] / double(pl->timed) : 0.0;
  if (count) *count = pl->timed;
  if (reset) {
    for (double& v : pl->stage_ms) v = 0.0;
    pl->timed = 0;
  }
  return RSFT_OK;
}

void rsft_destroy(rsft_plan_t pl) {
  if (!pl) return;
  (void)hipDeviceSynchronize();
  free_plan(pl);
}

const char* rsft_status_string(rsft_status s) {
  switch (s) {
    case RSFT_OK: return "RSFT_OK";
    case RSFT_ERROR_INVALID_ARGUMENT: return "RSFT_ERROR_INVALID_ARGUMENT";
    case RSFT_ERROR_NOT_POW2: return "RSFT_ERROR_NOT_POW2";
    case RSFT_ERROR_BAD_SIGMA: return "RSFT_ERROR_BAD_SIGMA";
    case RSFT_ERROR_UNSUPPORTED: return "RSFT_ERROR_UNSUPPORTED";
    case RSFT_ERROR_OUT_OF_MEMORY: return "RSFT_ERROR_OUT_OF_MEMORY";
    case RSFT_ERROR_DEVICE: return "RSFT_ERROR_DEVICE";
    case RSFT_ERROR_CAPACITY: return "RSFT_ERROR_CAPACITY";
    case RSFT_ERROR_NOT_READY: return "RSFT_ERROR_NOT_READY";
  }
  return "unknown rsft_status";
}

const char* rsft_last_error(void) { return g_last_error.c_str(); }

// ---- host-only design functions ----

rsft_status rsft_chebyshev_window(int64_t n, double atten_db, int32_t periodic, double* out) {
  if (n < 1 || !out || !(atten_db >= 0.0)) return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad window arguments");
  const auto w = periodic ? rsft::chebyshev_window_periodic(n, atten_db) : rsft::chebyshev_window(n, atten_db);
  std::copy(w.begin(), w.end(), out);
  return RSFT_OK;
}

rsft_status rsft_flat_window(int64_t n, int64_t b, double atten_db, double* out) {
  if (!out || !is_pow2(n) || !is_pow2(b) || b > n || !(atten_db >= 0.0))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad flat window arguments");
  const auto w = rsft::flat_window(n, b, atten_db);
  for (int64_t m = 0; m < n; ++m) {
    out[2 * m] = w[size_t(m)].real();
    out[2 * m + 1] = w[size_t(m)].imag();
  }
  return RSFT_OK;
}

rsft_status rsft_mod_inverse(int64_t sigma, int64_t n, int64_t* out) {
  if (!out || n < 1) return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad arguments");
  if (!rsft::mod_inverse(sigma, n, out)) return fail(RSFT_ERROR_BAD_SIGMA, "sigma not invertible modulo n");
  return RSFT_OK;
}

rsft_status rsft_stage1_probability(double pfa, int32_t rounds, int32_t mu, double* out) {
  if (!out || !(pfa > 0.0 && pfa < 1.0) || rounds < 1 || mu < 1 || mu > rounds)
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad arguments");
  *out = rsft::stage1_probability(pfa, rounds, mu);
  return RSFT_OK;
}

rsft_status rsft_design_thresholds(const rsft_design_params* in, rsft_design_result* out) {
  if (!in || !out) return fail(RSFT_ERROR_INVALID_ARGUMENT, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  const rsft_design_params& q = *in;
  if (q.ndim < 1 || q.ndim > RSFT_MAX_DIMS) return fail(RSFT_ERROR_INVALID_ARGUMENT, "ndim must be 1..4");
  if (q.rounds < 1 || q.rounds > 100000) return fail(RSFT_ERROR_INVALID_ARGUMENT, "rounds must be >= 1");
  double B = 1.0;
  for (int d = 0; d < q.ndim; ++d) {
    if (!is_pow2(q.n[d]) || !is_pow2(q.b[d])) return fail(RSFT_ERROR_NOT_POW2, "N_d and B_d must be powers of two");
    if (q.b[d] >= q.n[d]) return fail(RSFT_ERROR_INVALID_ARGUMENT, "need B_d < N_d");
    if (q.n[d] > (int64_t(1) << 16)) return fail(RSFT_ERROR_UNSUPPORTED, "N_d > 65536 in the design");
    if (!(q.omega_bins[d] >= 0.0 && q.omega_bins[d] < double(q.n[d])))
      return fail(RSFT_ERROR_INVALID_ARGUMENT, "omega_bins must be in [0, N_d)");
    B *= double(q.b[d]);
  }
  if (!(q.pd > 0.0 && q.pd < 1.0) || !(q.pfa > 0.0 && q.pfa < 1.0))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "pd and pfa must be in (0, 1)");
  if (!(q.sparsity >= 0.0) || !(q.noise_var > 0.0) || !std::isfinite(q.eta_m))
    return fail(RSFT_ERROR_INVALID_ARGUMENT, "sparsity >= 0, noise_var > 0, finite eta_m");
  if (q.window_atten_db < 0.0 || q.reserved != 0) return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad window or reserved field");
  const double flat_db = q.flat_atten_db < 0.0 ? q.window_atten_db : q.flat_atten_db;
  double a_bar = 1.0, b_bar = 1.0, eta_m = 1.0;
  for (int d = 0; d < q.ndim; ++d) {
    double a = 0.0, b = 0.0;
    rsft::alpha_beta_average(q.n[d], q.b[d], q.window_atten_db, flat_db, q.omega_bins[d], &a, &b);
    a_bar *= a;
    b_bar *= b;
    eta_m *= rsft::six_db_width(rsft::chebyshev_window(q.n[d], q.window_atten_db));
  }
  if (q.eta_m > 0.0) eta_m = q.eta_m;
  const int T = q.rounds;
  const double F = T * q.sparsity * eta_m / B;
  out->alpha_bar = a_bar;
  out->beta_bar = b_bar;
  out->F = F;
  out->eta_m = eta_m;
  if (F >= T) return RSFT_OK;                        // Remark 2: infeasible
  auto bisect = [](auto fun, double lo, double hi, double target) {
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (fun(mid) < target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  bool found = false;
  for (int mu = 1; mu <= T; ++mu) {
    const double pd_bar = bisect([&](double x) { double pd, pfa; rsft::stage2_tails(mu, T, F, 1.0, x, 0.0, &pd, &pfa); return pd; },
                                 1e-15, 1.0 - 1e-15, q.pd);
    const double eta_p = q.upper_bound ? 1.0 / pd_bar : 1.0;
    double pd0, pfa0;
    rsft::stage2_tails(mu, T, F, eta_p, pd_bar, 1e-300, &pd0, &pfa0);
    if (pfa0 > q.pfa) continue;                       // the co-existing tones alone exceed Pfa
    const double pfa_bar = bisect([&](double y) { double pd, pfa; rsft::stage2_tails(mu, T, F, eta_p, pd_bar, y, &pd, &pfa); return pfa; },
                                  1e-300, 1.0 - 1e-15, q.pfa);
    if (!(pfa_bar < pd_bar)) continue;
    const double snr = b_bar * (std::log(pfa_bar) / std::log(pd_bar) - 1.0) / a_bar;
    if (!found || snr < out->snr_min) {
      found = true;
      out->feasible = 1;
      out->mu = mu;
      out->snr_min = snr;
      out->pd_bar = pd_bar;
      out->pfa_bar = pfa_bar;
      out->eta_p = eta_p;
    }
  }
  if (found) {
    out->snr_min_db = 10.0 * std::log10(out->snr_min);
    out->gamma = -q.noise_var * b_bar * std::log(out->pfa_bar);
  }
  return RSFT_OK;
}

rsft_status rsft_draw_sigma(uint64_t seed, int32_t rounds, int32_t ndim, const int64_t* n, int64_t* out) {
  if (!n || !out || rounds < 1 || ndim < 1 || ndim > RSFT_MAX_DIMS) return fail(RSFT_ERROR_INVALID_ARGUMENT, "bad arguments");
  for (int d = 0; d < ndim; ++d)
    if (!is_pow2(n[d]) || n[d] < 2) return fail(RSFT_ERROR_NOT_POW2, "N_d must be a power of two >= 2");
  for (int s = 0; s < rounds; ++s)
    for (int d = 0; d < ndim; ++d) out[s * ndim + d] = rsft::draw_sigma(seed, s * ndim + d, n[d]);
  return RSFT_OK;
}

}  // extern "C"

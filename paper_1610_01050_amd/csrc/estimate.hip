// compact + estimate stage of the RSFT hot path.

#include "device_common.h"

namespace rsft {

// ---------------------------------------------------------------------------
// compact + estimate: one work-group per (frame, compaction chunk of 2^15
// cells) builds all of the chunk's records. Where dense chunks would keep
// single work-groups busy for long, the plan can add overflow workers
// instead (split_estimate_kernel): a chunk's work-group builds its first
// kChunkRecords records and the workers the rest, in items of 2^kItemShift
// records listed by the scan. (The workers' code, compiled into a kernel,
// slows its chunk path, so the plan picks the layout that is faster on its
// data; see rsft_autotune.) A work-group reads the chunk's bitmap words in
// row-major order, lists the detected cells of its rank range in LDS
// (popcount + block prefix sum), and every listed cell gets its record:
// votes recounted from the flags, gain-corrected magnitude (median over the
// estimation rounds of |fhat_s[M(i, sigma_s)]| times the inverse flat-window
// response at the cell's offset inside its bucket), a peak test against the
// 3^D - 1 circular neighbours (strictly above lower-index neighbours, at
// least equal to higher-index ones) and per dimension the vertex of a
// parabola through the log magnitudes at offsets -1, 0, +1, clamped to
// [-1/2, 1/2]. Ranks beyond the frame's capacity are dropped.
//
// Magnitudes are handled squared: the median, the peak comparisons and the
// vertex (a ratio of differences of logarithms) are unchanged by squaring,
// except the mean of the two middle values for an even number of rounds,
// which is taken on the square roots. FP32 magnitudes, FP64 vertex and
// frequency.
//
// Frames of 1..kMaxEstRounds estimation rounds take kernels specialised on
// that count (per-round tables in registers, a sorting network for the
// median). Frames with more (every clean round is used, up to T = 64) take
// the kEstAny variant, which walks the round mask and sorts each cell's
// values by insertion into a per-thread array.
//
// With at least 16 frames, chunk work-group b serves frames congruent to b
// mod 8: work-groups are dealt to the eight XCDs round-robin, so each XCD's
// L2 holds the buckets and flags of only its own frames.
// ---------------------------------------------------------------------------

constexpr int kEstThreads = 256;
constexpr int kEstAny = 0;   // template round count of the loop variant (any number of rounds)
constexpr int kGainLds = kEstGainLds;

// Per-frame constants of the estimate, uniform across the work-group.
template <int D, int M, bool G>
struct EstFrame {
  static constexpr int kM = M > 0 ? M : 1;
  uint32_t nm[D], lm[D], ls[D], bs[D], ns[D];
  const float* ig[D];              // inverse flat-window gains per dimension (global)
  const float* igs;                // their squares in LDS (dimension d at goff[d]) when they fit
  uint32_t goff[D];
  int mu, T;
  uint32_t sig_est[kM][D];
  const float* pw_est[kM];         // squared magnitudes |fhat_s|^2 of the estimation rounds
  const uint32_t* fl;              // flags [T][words]
  const int32_t* sig;              // sigma [kMaxRounds][kMaxDims] of the descriptor
  int words;
  const float* pw;                 // round 0 of the squared magnitudes (kEstAny)
  uint64_t est_mask;               // the estimation rounds (kEstAny)
  int B;
};

// The squared inverse flat-window gain of dimension d at offset idx inside
// a bucket (magnitudes are handled squared): from the LDS copy, which holds
// the squares, or (G: plans with a frame whose sum of L_d exceeds kGainLds)
// from global memory.
template <int D, int M, bool G>
__device__ __forceinline__ float inv_gain_sq(const EstFrame<D, M, G>& e, int dd, uint32_t idx) {
  if constexpr (G) {
    const float ig = e.ig[dd][idx];
    return ig * ig;
  } else {
    return e.igs[e.goff[dd] + idx];
  }
}

// load_frame also copies the frame's squared inverse gains to `sgain`
// (LDS) when they fit (all threads of the work-group call it; a barrier
// follows the copy).
template <int D, int M, bool G>
__device__ __forceinline__ void load_frame(const DevPtrs& p, const FrameDesc& d, int64_t rel,
                                           EstFrame<D, M, G>& e, float* sgain) {
  const float* pw = p.powers + d.bucket_off + rel * d.bucket_stride;
  uint32_t tot = 0u;
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    e.nm[dd] = uint32_t(d.n[dd] - 1);
    e.lm[dd] = uint32_t(d.l[dd] - 1);
    e.ls[dd] = uint32_t(d.lshift[dd]);
    e.bs[dd] = uint32_t(d.bshift[dd]);
    e.ns[dd] = uint32_t(d.nshift[dd]);
    e.ig[dd] = p.inv_gains + d.gain_off[dd];
    e.goff[dd] = tot;
    tot += uint32_t(d.l[dd]);
  }
  e.igs = sgain;
  if constexpr (!G) {
#pragma unroll
    for (int dd = 0; dd < D; ++dd)
      for (uint32_t k = threadIdx.x; k <= e.lm[dd]; k += kEstThreads) {
        const float ig = e.ig[dd][k];
        sgain[e.goff[dd] + k] = ig * ig;
      }
  }
  __syncthreads();
  e.mu = d.mu;
  e.T = d.T;
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int s = d.est_rounds[q];
#pragma unroll
    for (int dd = 0; dd < D; ++dd) e.sig_est[q][dd] = uint32_t(d.sigma[s][dd]);
    e.pw_est[q] = pw + int64_t(s) * d.B;
  }
  e.fl = p.flags + d.flag_off + rel * d.flag_stride;
  e.sig = &d.sigma[0][0];
  e.words = d.words;
  e.pw = pw;
  e.est_mask = d.est_mask;
  e.B = d.B;
}

// Median of M values (an odd-even transposition network on fixed indices);
// for even M the mean of the middle two is taken on their square roots (the
// values are squared magnitudes).
template <int M>
__device__ __forceinline__ float median_of(float (&v)[M]) {
#pragma unroll
  for (int pass = 0; pass < M; ++pass) {
#pragma unroll
    for (int q = pass & 1; q + 1 < M; q += 2) {
      const float lo = fminf(v[q], v[q + 1]);
      const float hi = fmaxf(v[q], v[q + 1]);
      v[q] = lo;
      v[q + 1] = hi;
    }
  }
  if constexpr (M & 1) {
    return v[M / 2];
  } else {
    const float a = 0.5f * (sqrtf(v[M / 2 - 1]) + sqrtf(v[M / 2]));
    return a * a;
  }
}

// Vertex of the parabola through (-1, log am), (0, log a0), (1, log ap) from
// the squared magnitudes (the factor 2 of the logarithms cancels), clamped to
// [-1/2, 1/2]; 0 when the points are not concave. Base-2 logarithms of the
// FP32 powers, vertex in FP64.
__device__ __forceinline__ double log_parabola_offset(float pm, float p0, float pp) {
  const float tiny = 1e-37f;
  const double lm = double(__builtin_amdgcn_logf(pm > tiny ? pm : tiny));
  const double l0 = double(__builtin_amdgcn_logf(p0 > tiny ? p0 : tiny));
  const double lp = double(__builtin_amdgcn_logf(pp > tiny ? pp : tiny));
  const double den = 2.0 * l0 - lm - lp;
  if (!(den > 0.0)) return 0.0;
  double v = 0.5 * (lp - lm) / den;
  v = v < -0.5 ? -0.5 : v;
  v = v > 0.5 ? 0.5 : v;
  return v;
}

// Squared gain-corrected magnitude of neighbour `code` (digit d of code in
// base 3 is o_d + 1): the median over the estimation rounds, from the
// per-round squared inverse gains g and bucket offsets jb of the offsets.
template <int D, int M, bool G>
__device__ __forceinline__ float neighbour_power(const EstFrame<D, M, G>& e, const float (&g)[M][D][3],
                                                 const uint32_t (&jb)[M][D][3], int code) {
  float v[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    uint32_t jf = 0u;
    float gg = 1.f;
    int c = code;
#pragma unroll
    for (int dd = D - 1; dd >= 0; --dd) {
      const int o = c % 3;
      c /= 3;
      jf |= jb[q][dd][o];
      gg *= g[q][dd][o];
    }
    v[q] = e.pw_est[q][jf] * gg;
  }
  return median_of<M>(v);
}

// The same for D = 4, from the permuted index u0[q][d] = [sigma c]_N of the
// cell itself (no array indexed at run time).
template <int D, int M, bool G>
__device__ __forceinline__ float neighbour_power_dyn(const EstFrame<D, M, G>& e, const uint32_t (&u0)[M][D],
                                                     int code) {
  float v[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    uint32_t jf = 0u;
    float gg = 1.f;
    int c = code;
#pragma unroll
    for (int dd = D - 1; dd >= 0; --dd) {
      const int o = c % 3 - 1;
      c /= 3;
      const uint32_t u = (u0[q][dd] + e.sig_est[q][dd] * uint32_t(o)) & e.nm[dd];
      gg *= inv_gain_sq(e, dd, u & e.lm[dd]);
      jf |= (u >> e.ls[dd]) << e.bs[dd];
    }
    v[q] = e.pw_est[q][jf] * gg;
  }
  return median_of<M>(v);
}

// The same for any number of estimation rounds (kEstAny): the rounds of the
// mask in increasing order, each value inserted into a sorted per-thread
// array, then the median as in median_of.
template <int D, int M, bool G>
__device__ __forceinline__ float neighbour_power_any(const EstFrame<D, M, G>& e, const uint32_t (&cell)[D],
                                                     int code) {
  float v[kMaxRounds];
  int n = 0;
  uint64_t rest = e.est_mask;
  while (rest) {
    const int s = __builtin_ctzll(rest);
    rest &= rest - 1ull;
    uint32_t jf = 0u;
    float gg = 1.f;
    int c = code;
#pragma unroll
    for (int dd = D - 1; dd >= 0; --dd) {
      const int o = c % 3 - 1;
      c /= 3;
      const uint32_t sg = uint32_t(e.sig[s * kMaxDims + dd]);
      const uint32_t u = (sg * cell[dd] + sg * uint32_t(o)) & e.nm[dd];
      gg *= inv_gain_sq(e, dd, u & e.lm[dd]);
      jf |= (u >> e.ls[dd]) << e.bs[dd];
    }
    const float x = e.pw[int64_t(s) * e.B + jf] * gg;
    int k = n;
    while (k > 0 && v[k - 1] > x) {
      v[k] = v[k - 1];
      --k;
    }
    v[k] = x;
    ++n;
  }
  if (n & 1) return v[n / 2];
  const float a = 0.5f * (sqrtf(v[n / 2 - 1]) + sqrtf(v[n / 2]));
  return a * a;
}

// True when neighbour `code` differs from the cell in at most one dimension
// (base-3 digits: 1 is offset 0).
constexpr bool on_axis(int code, int D) {
  int off = 0;
  for (int dd = 0; dd < D; ++dd, code /= 3) off += code % 3 != 1;
  return off <= 1;
}

// One record. D <= 3: the 3^D neighbourhood lives in registers (loops
// unrolled); D = 4: its 81 values are kept in this thread's LDS column
// `pcol` (stride kEstThreads) and visited by ordinary loops.
template <int D, int M, bool G>
__device__ __forceinline__ void write_record(const EstFrame<D, M, G>& e, int T, int64_t f,
                                             unsigned long long flat, DetRec* out,
                                             float* pcol) {
  constexpr int kNb = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;
  constexpr bool kRegs = D <= 3;
  constexpr int kCentre = (kNb - 1) / 2;
  uint32_t cell[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) cell[dd] = uint32_t(flat >> e.ns[dd]) & e.nm[dd];
  // votes: the flag of the cell's bucket in every round, four rounds' flag
  // words loaded at a time (s < s0 + 4 <= 64 stays inside the sigma table)
  // (every detected cell of a plan with mu = T has exactly T votes)
  int votes = e.mu == T ? T : 0;
  for (int s0 = 0; s0 < T && e.mu != T; s0 += 4) {
    uint32_t wd[4], sh[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k;
      uint32_t jf = 0u;
#pragma unroll
      for (int dd = 0; dd < D; ++dd) {
        const uint32_t u = (uint32_t(e.sig[s * kMaxDims + dd]) * cell[dd]) & e.nm[dd];
        jf |= (u >> e.ls[dd]) << e.bs[dd];
      }
      sh[k] = jf & 31u;
      wd[k] = s < T ? e.fl[int64_t(s) * e.words + (jf >> 5)] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) votes += int((wd[k] >> sh[k]) & 1u);
  }
  // neighbour `code` against the cell: it must lie strictly below the cell's
  // magnitude when its row-major index is lower, at most equal when higher.
  // Row-major order is decided by the first dimension whose offset is not
  // zero: offset -1 gives a lower index unless the cell is at 0 (it wraps to
  // N_d - 1), offset +1 a higher one unless the cell is at N_d - 1 (it wraps
  // to 0). N_d >= 2, so a neighbour other than the cell itself differs from
  // it. (The digits of `code` are compile-time constants where the loops
  // over the neighbourhood are unrolled.)
  bool below_m[D], below_p[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    below_m[dd] = cell[dd] != 0u;
    below_p[dd] = cell[dd] == e.nm[dd];
  }
  auto visit = [&](int code, float p0, float pc, bool& peak) {
    int od[D];
    int c = code;
#pragma unroll
    for (int dd = D - 1; dd >= 0; --dd) {
      od[dd] = c % 3 - 1;
      c /= 3;
    }
    bool decided = false, lower = false;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
      if (!decided && od[dd] != 0) {
        lower = od[dd] < 0 ? below_m[dd] : below_p[dd];
        decided = true;
      }
    }
    if (!decided) return;            // the cell itself
    if (lower) {
      if (!(p0 > pc)) peak = false;
    } else {
      if (!(p0 >= pc)) peak = false;
    }
  };
  float preg[kRegs ? kNb : 1];
  bool peak = true;
  if constexpr (kRegs && M == kEstAny) {
#pragma unroll
    for (int code = 0; code < kNb; ++code)
      if (on_axis(code, D)) preg[code] = neighbour_power_any<D, M, G>(e, cell, code);
#pragma unroll
    for (int code = 0; code < kNb; ++code)
      if (code != kCentre && on_axis(code, D)) visit(code, preg[kCentre], preg[code], peak);
    if (peak) {
#pragma unroll
      for (int code = 0; code < kNb; ++code)
        if (!on_axis(code, D)) visit(code, preg[kCentre], neighbour_power_any<D, M, G>(e, cell, code), peak);
    }
  } else if constexpr (kRegs) {
    // Per round and dimension the three offsets o_d = -1, 0, 1 share one
    // permuted index, [sigma (c + o)]_N = [sigma c + sigma o]_N, so their
    // squared inverse gains and bucket offsets are formed once.
    float g[M][D][3];
    uint32_t jb[M][D][3];
#pragma unroll
    for (int q = 0; q < M; ++q) {
#pragma unroll
      for (int dd = 0; dd < D; ++dd) {
        const uint32_t sg = e.sig_est[q][dd];
        const uint32_t u0 = sg * cell[dd];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          const uint32_t u = (u0 + sg * uint32_t(o - 1)) & e.nm[dd];
          g[q][dd][o] = inv_gain_sq(e, dd, u & e.lm[dd]);
          jb[q][dd][o] = (u >> e.ls[dd]) << e.bs[dd];
        }
      }
    }
    // The cell and its 2D axis neighbours first: they give the vertex, and
    // most cells that are not peaks already lose to one of them. Only the
    // lanes still in the running visit the other neighbours (the test is an
    // AND over all of them, so the order does not change it).
#pragma unroll
    for (int code = 0; code < kNb; ++code)
      if (on_axis(code, D)) preg[code] = neighbour_power<D, M, G>(e, g, jb, code);
#pragma unroll
    for (int code = 0; code < kNb; ++code)
      if (code != kCentre && on_axis(code, D)) visit(code, preg[kCentre], preg[code], peak);
    if (peak) {
#pragma unroll
      for (int code = 0; code < kNb; ++code)
        if (!on_axis(code, D)) visit(code, preg[kCentre], neighbour_power<D, M, G>(e, g, jb, code), peak);
    }
  } else {
    if constexpr (M == kEstAny) {
#pragma unroll 1
      for (int code = 0; code < kNb; ++code) pcol[code * kEstThreads] = neighbour_power_any<D, M, G>(e, cell, code);
    } else {
      uint32_t u0[M][D];
#pragma unroll
      for (int q = 0; q < M; ++q) {
#pragma unroll
        for (int dd = 0; dd < D; ++dd) u0[q][dd] = e.sig_est[q][dd] * cell[dd];
      }
#pragma unroll 1
      for (int code = 0; code < kNb; ++code) pcol[code * kEstThreads] = neighbour_power_dyn<D, M, G>(e, u0, code);
    }
    const float pc0 = pcol[kCentre * kEstThreads];
#pragma unroll 1
    for (int code = 0; code < kNb; ++code)
      if (code != kCentre) visit(code, pc0, pcol[code * kEstThreads], peak);
  }
  auto P = [&](int code) -> float {
    if constexpr (kRegs) return preg[code];
    else return pcol[code * kEstThreads];
  };
  const float p0 = P(kCentre);
  DetRec rec;
  rec.key = (unsigned long long)flat | ((unsigned long long)votes << kKeyVotesShift) |
            ((peak ? 1ull : 0ull) << (kKeyVotesShift + 7));
  rec.frame = uint32_t(f);
  rec.magnitude = sqrtf(p0);
#pragma unroll
  for (int dd = 0; dd < kMaxDims; ++dd) rec.delta[dd] = 0.f;
  int stride = 1;
#pragma unroll
  for (int dd = D - 1; dd >= 0; --dd) {
    rec.delta[dd] = float(log_parabola_offset(P(kCentre - stride), p0, P(kCentre + stride)));
    stride *= 3;
  }
  *out = rec;
}

// Records of list[0 .. min(n, room)) in batches of kEstThreads: each thread
// builds one record in LDS, then the work-group copies the batch out with
// contiguous 8-byte stores (a record is 32 bytes).
template <int D, int M, bool G>
__device__ __forceinline__ void estimate_list(const DevPtrs& p, const FrameDesc& d, int64_t f,
                                              int64_t rel, int T, const uint32_t* list, int n,
                                              unsigned long long cell0, DetRec* out,
                                              int64_t room, float* pcol, DetRec* stage,
                                              float* sgain) {
  EstFrame<D, M, G> e;
  load_frame<D, M, G>(p, d, rel, e, sgain);
  const int lim = int(n < room ? n : room);
  constexpr int kWords = int(sizeof(DetRec) / 8);
  for (int q0 = 0; q0 < lim; q0 += kEstThreads) {
    const int q = q0 + int(threadIdx.x);
    if (q < lim) write_record<D, M, G>(e, T, f, cell0 | (unsigned long long)list[q], stage + threadIdx.x, pcol);
    __syncthreads();
    const int nw = (lim - q0 < kEstThreads ? lim - q0 : kEstThreads) * kWords;
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(stage);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(out + q0);
    for (int w = int(threadIdx.x); w < nw; w += kEstThreads) dst[w] = src[w];
    __syncthreads();
  }
}

// Waves per SIMD the register allocation aims at, as many as fit without
// spilling (the gathers are latency-bound, so more waves hide more of
// them): six for 2-D records of up to three rounds (80 VGPRs), four for 3-D
// ones (128), fewer for more rounds; D = 4 keeps its neighbourhood in 81 KB
// of LDS (one work-group per compute unit).
constexpr int est_waves(int D, int M) {
  return M == kEstAny ? (D >= 4 ? 1 : 2)
         : D <= 1     ? 5
         : D == 2     ? (M <= 3 ? 6 : 4)
         : D == 3     ? (M <= 3 ? 4 : 2)
                      : 1;
}

// estimate_list for a frame of `ne` estimation rounds, 1 <= ne <= MMAX
// (MMAX = kEstAny: any count, by the loop variant).
template <int D, int MMAX, bool G>
__device__ __forceinline__ void estimate_list_n(int ne, const DevPtrs& p, const FrameDesc& d, int64_t f,
                                                int64_t rel, int T, const uint32_t* list, int n,
                                                unsigned long long cell0, DetRec* out,
                                                int64_t room, float* pcol, DetRec* stage,
                                                float* sgain) {
  if constexpr (MMAX == kEstAny) {
    estimate_list<D, kEstAny, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain);
    return;
  }
  switch (ne) {
    case 1: if constexpr (MMAX >= 1) estimate_list<D, 1, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain); break;
    case 2: if constexpr (MMAX >= 2) estimate_list<D, 2, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain); break;
    case 3: if constexpr (MMAX >= 3) estimate_list<D, 3, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain); break;
    case 4: if constexpr (MMAX >= 4) estimate_list<D, 4, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain); break;
    default: if constexpr (MMAX >= 5) estimate_list<D, 5, G>(p, d, f, rel, T, list, n, cell0, out, room, pcol, stage, sgain); break;
  }
}

// The largest index i in [0, n) with a[i] <= t, for a non-decreasing array
// with a[0] <= t: a 64-way search by one wave (each step loads 64 entries
// and narrows the range 64-fold). Every wave of the work-group runs it and
// gets the same answer.
__device__ __forceinline__ int64_t wave_search(const int64_t* __restrict__ a, int64_t n, int64_t t) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) >> 6;
    const int64_t i = lo + int64_t(lane) * step;
    const bool ok = i < hi && a[i] <= t;
    const unsigned long long m = __ballot(ok);        // lanes 0..k (lane 0 holds a[lo] <= t)
    if (m == 0ull) break;                              // only if a[lo] > t: keep lo
    const int k = 63 - __clzll(m);
    lo += int64_t(k) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Records of ranks r_lo .. r_lo + n - 1 of chunk c of frame f: the work-group
// lists those detected cells from the chunk's bitmap words wv (kWpt per
// thread; popcounts and a block prefix sum) and builds their records.
template <int D, int M, bool G, int kWpt>
__device__ __forceinline__ void build_range(const DevPtrs& p, int T, const FrameDesc& d, int64_t f, int c,
                                            const uint32_t (&wv)[kWpt], int r_lo, int n, int64_t rank0,
                                            uint32_t* list, uint32_t* wsum, DetRec* stage,
                                            float* pcol, float* sgain) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int pc = 0;
#pragma unroll
  for (int q = 0; q < kWpt; ++q) pc += __popc(wv[q]);
  int incl = pc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = uint32_t(incl);
  __syncthreads();
  int r = incl - pc;                                 // chunk rank of this thread's first cell
#pragma unroll
  for (int q = 0; q < kEstThreads / 64; ++q)
    if (q < wave) r += int(wsum[q]);
  if (r < r_lo + n && r + pc > r_lo) {
#pragma unroll
    for (int q = 0; q < kWpt; ++q) {
      uint32_t word = wv[q];
      const uint32_t wrel = uint32_t(tid * kWpt + q) << 5;
      while (word) {
        const int bit = __ffs(word) - 1;
        word &= word - 1u;
        if (r >= r_lo && r < r_lo + n) list[r - r_lo] = wrel | uint32_t(bit);
        ++r;
      }
    }
  }
  __syncthreads();
  estimate_list_n<D, M, G>(d.n_est, p, d, f, rel_of(p, f), T, list, n, (unsigned long long)c << kCompactShift,
                        p.records + p.offsets[f] + rank0 + r_lo, n, pcol, stage, sgain);
}

constexpr int kWordsPerThread = (1 << (kCompactShift - 5)) / kEstThreads;   // a chunk's bitmap words

// Chunk (frame f, chunk c) of work-group b of the chunk grid: the chunk
// list's entry b, else from the (XCD-grouped) frame-by-chunk grid; false
// when b lies past the batch or on list padding.
__device__ __forceinline__ bool chunk_of(const DevPtrs& p, int64_t b, int64_t nframes, int max_cchunks,
                                         int xcd_groups, int use_list, int64_t& f, int& c) {
  if (use_list) return listed_chunk(p, b, f, c);
  if (xcd_groups) {
    const int64_t k = b >> 3;
    f = (k / max_cchunks) * 8 + (b & 7);
    c = int(k % max_cchunks);
  } else {
    f = b / max_cchunks;
    c = int(b % max_cchunks);
  }
  return f < nframes;
}

// Whether the kernel built for M rounds serves a frame of ne estimation
// rounds: the specialised kernels take 1..M (one launch per plan, built for
// the plan's largest count up to kMaxEstRounds), the kEstAny kernel the
// frames beyond kMaxEstRounds.
__host__ __device__ constexpr bool serves(int M, int ne) {
  return M == kEstAny ? ne > kMaxEstRounds : (ne >= 1) & (ne <= M);
}

// Without overflow workers: one work-group per (frame, chunk) builds all of
// the chunk's records; a chunk of up to kListMax detections is listed in one
// pass, a denser one in passes of kListMax cells.
constexpr int kListMax = 2048;   // cells listed at once: a chunk's, else one pass's

template <int D, int M, bool G>
__global__ __launch_bounds__(kEstThreads) __attribute__((amdgpu_waves_per_eu(est_waves(D, M)))) void compact_estimate_kernel(DevPtrs p, int T,
                                                                       int64_t nframes,
                                                                       int max_cchunks,
                                                                       int xcd_groups,
                                                                       int use_list) {
  constexpr int kNb = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;
  __shared__ uint32_t list[kListMax];
  __shared__ uint32_t wsum[kEstThreads / 64];
  __shared__ DetRec stage[kEstThreads];
  __shared__ float pbuf[D >= 4 ? kNb * kEstThreads : 1];
  __shared__ float sgain[kGainLds];
  int64_t f;
  int c;
  if (!chunk_of(p, blockIdx.x, nframes, max_cchunks, xcd_groups, use_list, f, c)) return;
  const FrameDesc& d = desc_of(p, f);
  // The descriptor fields, then the chunk's counters and bitmap words, are
  // each loaded together before they are tested (no chain of dependent
  // loads behind early exits).
  const int cch = d.cchunks, nd = d.ndim, ne = d.n_est;
  if ((c >= cch) | (nd != D) | !serves(M, ne)) return;
  const int64_t rel = rel_of(p, f);
  const int64_t ck = d.chunk_off + rel * d.chunk_stride + c;
  const int64_t cap = d.cap;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride;
  const int w0 = c << (kCompactShift - 5);
  const int wend = min(d.bitmap_words, w0 + (1 << (kCompactShift - 5)));
  // thread t's words w0 + 4t .. w0 + 4t + 3 (the one-pass listing below)
  constexpr int kWpt = (1 << (kCompactShift - 5)) / kEstThreads;
  uint32_t wv[kWpt];
#pragma unroll
  for (int q = 0; q < kWpt; ++q) {
    const int w = w0 + tid * kWpt + q;
    wv[q] = w < wend ? bm[w] : 0u;
  }
  const uint32_t chunk_count = p.chunk_counts[ck];
  const int64_t rank0 = p.chunk_offsets[ck];
  const int64_t frame_off = p.offsets[f];
  if ((chunk_count == 0u) | (rank0 >= cap)) return;
  DetRec* out = p.records + frame_off + rank0;
  const unsigned long long cell0 = (unsigned long long)c << kCompactShift;
  const int64_t room0 = cap - rank0;
  float* pcol = pbuf + threadIdx.x;
  if (chunk_count <= uint32_t(kListMax)) {
    // one pass: thread t lists the set bits of its words
    int pc = 0;
#pragma unroll
    for (int q = 0; q < kWpt; ++q) pc += __popc(wv[q]);
    int incl = pc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = uint32_t(incl);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kEstThreads / 64; ++q) {
      if (q < wave) base += int(wsum[q]);
      total += int(wsum[q]);
    }
    int k = base + incl - pc;
#pragma unroll
    for (int q = 0; q < kWpt; ++q) {
      uint32_t word = wv[q];
      const uint32_t wrel = uint32_t(tid * kWpt + q) << 5;
      while (word) {
        const int bit = __ffs(word) - 1;
        word &= word - 1u;
        if (k < kListMax) list[k] = wrel | uint32_t(bit);
        ++k;
      }
    }
    __syncthreads();
    estimate_list_n<D, M, G>(ne, p, d, f, rel, T, list, min(total, kListMax), cell0, out, room0, pcol, stage,
                          sgain);
    return;
  }
  // dense chunk: passes of kListMax / 32 words (at most kListMax cells each)
  constexpr int kPassWords = kListMax / 32;
  int64_t running = 0;
  for (int wb = w0; wb < wend; wb += kPassWords) {
    const int w = wb + tid;
    uint32_t word = (tid < kPassWords && w < wend) ? bm[w] : 0u;
    const int pc = __popc(word);
    int incl = pc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = uint32_t(incl);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kEstThreads / 64; ++q) {
      if (q < wave) base += int(wsum[q]);
      total += int(wsum[q]);
    }
    int k = base + incl - pc;
    while (word) {
      const int bit = __ffs(word) - 1;
      word &= word - 1u;
      list[k++] = (uint32_t(w - w0) << 5) | uint32_t(bit);
    }
    __syncthreads();
    estimate_list_n<D, M, G>(ne, p, d, f, rel, T, list, total, cell0, out + running, room0 - running, pcol,
                          stage, sgain);
    running += total;
    if (running >= room0) return;   // uniform: the frame's capacity is used up
    __syncthreads();
  }
}

// With overflow workers: work-group b of the first `og` (dispatched first)
// takes a contiguous range of the overflow items the scan listed
// (consecutive ranges on one XCD); item i of a frame lies in the chunk whose
// running item sum is the largest not above i, and covers the chunk's ranks
// kChunkRecords + 2^kItemShift k ... for the chunk's k-th item. Every other
// work-group owns one chunk and its ranks 0 .. kChunkRecords - 1. One record
// builder serves both.
template <int D, int M, bool G>
__global__ __launch_bounds__(kEstThreads) __attribute__((amdgpu_waves_per_eu(est_waves(D, M)))) void split_estimate_kernel(DevPtrs p, int T,
                                                                     int64_t nframes,
                                                                     int max_cchunks,
                                                                     int xcd_groups,
                                                                     int use_list,
                                                                     int og) {
  constexpr int kNb = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;
  constexpr int kItem = 1 << kItemShift;
  constexpr int kWpt = kWordsPerThread;
  __shared__ uint32_t list[kChunkRecords];
  __shared__ uint32_t wsum[kEstThreads / 64];
  __shared__ DetRec stage[kEstThreads];
  __shared__ float pbuf[D >= 4 ? kNb * kEstThreads : 1];
  __shared__ float sgain[kGainLds];
  const int tid = threadIdx.x;
  const bool worker = int64_t(blockIdx.x) < og;
  int64_t f = 0, i = 0, hi = 0, fbeg = 0, fend = 0;
  int c = 0;
  if (worker) {
    const int64_t total = p.item_offsets[nframes];
    const int64_t b = blockIdx.x;
    const int64_t v = (og & 7) == 0 ? (b & 7) * (og >> 3) + (b >> 3) : b;
    i = total * v / og;
    hi = total * (v + 1) / og;
  } else if (!chunk_of(p, int64_t(blockIdx.x) - og, nframes, max_cchunks, xcd_groups, use_list, f, c)) {
    return;
  }
  for (;;) {
    // the next record range: frame f, chunk c, ranks r_lo .. r_lo + n - 1
    const FrameDesc* dp;
    uint32_t wv[kWpt];
    int r_lo, n;
    int64_t rank0;
    if (worker) {
      if (i >= hi) return;
      if (i >= fend) {
        f = wave_search(p.item_offsets, nframes + 1, i);
        if (f >= nframes) return;                      // i < total keeps f < nframes
        fbeg = p.item_offsets[f];
        fend = p.item_offsets[f + 1];
        if (fend <= i) return;                         // item_offsets is non-decreasing
        const FrameDesc& d = desc_of(p, f);
        if ((d.ndim != D) | !serves(M, d.n_est)) {   // another launch's frame
          i = fend;
          continue;
        }
      }
      dp = &desc_of(p, f);
      const int64_t rel = rel_of(p, f);
      const int64_t ck0 = dp->chunk_off + rel * dp->chunk_stride;
      const int64_t* ci = p.chunk_items + ck0;
      const int64_t j = i - fbeg;
      c = int(wave_search(ci, dp->cchunks, j));
      r_lo = kChunkRecords + int((j - ci[c]) << kItemShift);
      const uint32_t count = p.chunk_counts[ck0 + c];
      rank0 = p.chunk_offsets[ck0 + c];
      const uint32_t* bm = p.bitmap + dp->bitmap_off + rel * dp->bitmap_stride;
      const int w0 = c << (kCompactShift - 5);
      const int bw = dp->bitmap_words;
#pragma unroll
      for (int q = 0; q < kWpt; ++q) {
        const int w = w0 + tid * kWpt + q;
        wv[q] = w < bw ? bm[w] : 0u;
      }
      n = int(min(min(int64_t(count) - r_lo, int64_t(dp->cap) - rank0 - r_lo), int64_t(kItem)));
      ++i;
    } else {
      dp = &desc_of(p, f);
      const int cch = dp->cchunks, nd = dp->ndim, ne = dp->n_est;
      if ((c >= cch) | (nd != D) | !serves(M, ne)) return;
      const int64_t rel = rel_of(p, f);
      const int64_t ck = dp->chunk_off + rel * dp->chunk_stride + c;
      const uint32_t* bm = p.bitmap + dp->bitmap_off + rel * dp->bitmap_stride;
      const int w0 = c << (kCompactShift - 5);
      const int bw = dp->bitmap_words;
#pragma unroll
      for (int q = 0; q < kWpt; ++q) {
        const int w = w0 + tid * kWpt + q;
        wv[q] = w < bw ? bm[w] : 0u;
      }
      const uint32_t count = p.chunk_counts[ck];
      rank0 = p.chunk_offsets[ck];
      const int64_t cap = dp->cap;
      if ((count == 0u) | (rank0 >= cap)) return;
      r_lo = 0;
      n = int(min(min(int64_t(count), cap - rank0), int64_t(kChunkRecords)));
    }
    build_range<D, M, G, kWpt>(p, T, *dp, f, c, wv, r_lo, n, rank0, list, wsum, stage, pbuf + tid, sgain);
    if (!worker) return;
  }
}

// Per dimension count, one kernel built for the most estimation rounds any
// frame of the plan uses (uneven plans mix frames of 1..M rounds, sigma per
// frame).
template <int D, bool G>
static void launch_estimate_d(const DevPtrs& p, dim3 grid, int og, hipStream_t st, int T, int64_t nframes,
                              int max_cchunks, int xcd, int use_list, int est_mask) {
#define RSFT_EST(M)                                                                                      \
  do {                                                                                                   \
    if (og > 0)                                                                                          \
      hipLaunchKernelGGL((split_estimate_kernel<D, M, G>), grid, dim3(kEstThreads), 0, st, p, T, nframes,    \
                         max_cchunks, xcd, use_list, og);                                                \
    else                                                                                                 \
      hipLaunchKernelGGL((compact_estimate_kernel<D, M, G>), grid, dim3(kEstThreads), 0, st, p, T, nframes,  \
                         max_cchunks, xcd, use_list);                                                    \
  } while (0)
  const int small = est_mask & ((2 << kMaxEstRounds) - 1);
  if (small >= 32) RSFT_EST(5);
  else if (small >= 16) RSFT_EST(4);
  else if (small >= 8) RSFT_EST(3);
  else if (small >= 4) RSFT_EST(2);
  else if (small >= 2) RSFT_EST(1);
  if (est_mask >> (kMaxEstRounds + 1)) RSFT_EST(kEstAny);
#undef RSFT_EST
}

int launch_estimate(const DevPtrs& p, int64_t nframes, int T, int max_cchunks, int dims_mask,
                    int est_mask, int workers, int num_cus, int64_t nlist, int global_gains, void* stream) {
  if (nframes <= 0) return hipSuccess;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int xcd = nframes >= 16 ? 1 : 0;
  const int use_list = nlist > 0 ? 1 : 0;
  const int64_t rows = xcd ? ((nframes + 7) / 8) * 8 : nframes;
  // overflow workers: two per compute unit, a multiple of 8 so that the
  // chunk work-groups after them keep their XCD assignment
  const int og = workers ? ((2 * (num_cus > 0 ? num_cus : 256)) + 7) / 8 * 8 : 0;
  const int64_t blocks = og + (use_list ? nlist : rows * int64_t(max_cchunks));
  if (blocks >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  const dim3 grid{unsigned(blocks), 1u, 1u};
#define RSFT_EST_D(D)                                                                                    \
  do {                                                                                                   \
    if (global_gains)                                                                                    \
      launch_estimate_d<D, true>(p, grid, og, st, T, nframes, max_cchunks, xcd, use_list, est_mask);     \
    else                                                                                                 \
      launch_estimate_d<D, false>(p, grid, og, st, T, nframes, max_cchunks, xcd, use_list, est_mask);    \
  } while (0)
  if (dims_mask & 1) RSFT_EST_D(1);
  if (dims_mask & 2) RSFT_EST_D(2);
  if (dims_mask & 4) RSFT_EST_D(3);
  if (dims_mask & 8) RSFT_EST_D(4);
#undef RSFT_EST_D
  return hipGetLastError();
}

}  // namespace rsft

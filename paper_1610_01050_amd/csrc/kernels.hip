// HIP kernels of the RSFT hot path for gfx950 (CDNA4, wave64).
//
// Stage map (Algorithm 1 of the paper, Location procedure):
//   fold      window W, permutation P_sigma, flat window Wbar and aliasing,
//             all T rounds from one pass over the input (Def. 1, 2; eq. l)
//   dft       B-point N-D DFT of each round's buckets on MFMA (eq. f), then
//             |.|^2, first-stage NP threshold (eq. exp, eq. tpd) and flags
//   vote      reverse mapping + accumulation + second stage (Def. 3-4,
//             eq. a_i), enumerating only the preimages of flagged buckets
//   scan      per-frame detection counts and record offsets
//   estimate  ordered compaction of the detections, gain-corrected
//             magnitudes, peak test and log-parabolic off-grid offsets
//
// Why the fold reads the input in natural order: with tau = 0 the round-s
// bucket before the DFT is f_s[b] = sum_{n = b mod B} wbar[n] y[[sigma n]_N].
// Substituting m = [sigma n]_N and using B | N,
//   n mod B = [sigma^{-1} m]_N mod B = (tau_s (m mod B)) mod B,
//   tau_s = sigma^{-1} mod B,
// so f_s[tau_s c] = sum_{m = c mod B} w[m] wbar[[sigma^{-1} m]_N] r[m]: a fold
// of the unpermuted input by residue class c = m mod B with per-round weights
// W_s[m] = w[m] wbar[[sigma^{-1} m]_N], followed by the relabel c -> tau_s c
// mod B. The permutation becomes weight tables plus a bucket relabel, and
// every input sample is loaded once, coalesced, for all rounds. The relabel
// commutes with the DFT: fhat_s[j] = DFT(acc_s)[tau_s j mod B] per dimension.
// Per dimension everything is separable, so in N-D the weight of a sample is
// a row factor (leading dimensions) times a column factor (last dimension).

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "rsft_internal.h"

namespace rsft {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ const FrameDesc& desc_of(const DevPtrs& p, int64_t f) {
  return p.descs[p.uniform ? 0 : f];
}
__device__ __forceinline__ int64_t rel_of(const DevPtrs& p, int64_t f) {
  return p.uniform ? f : 0;
}

// ---------------------------------------------------------------------------
// fold: one work-group per tile = (frame, residue class of the leading
// dimensions, chunk of columns). The class fixes (m_0 mod B_0, ...,
// m_{D-2} mod B_{D-2}); its rows are listed in rowlist. Threads own V
// consecutive columns; per column they sum the row-weighted samples of the
// class's rows (4 FMAs per round per sample), multiply once by the column
// weight, and keep the result per residue slot (columns P apart share a
// residue because B_{D-1} divides P). A deterministic LDS reduction over the
// slots of each residue finishes the tile: T x B_{D-1} partial buckets.
// When a row is shorter than P the work-group splits into G = P / N_{D-1}
// row groups that take every G-th row of the class.
// ---------------------------------------------------------------------------

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

template <bool C128, bool NT, int V>
__device__ __forceinline__ void load_vec(const void* base, int64_t idx, float2 (&x)[V]) {
  if constexpr (!C128) {
    const v4f* p4 = reinterpret_cast<const v4f*>(reinterpret_cast<const float2*>(base) + idx);
#pragma unroll
    for (int q = 0; q < V / 2; ++q) {
      const v4f v = NT ? __builtin_nontemporal_load(p4 + q) : p4[q];
      x[2 * q] = make_float2(v.x, v.y);
      x[2 * q + 1] = make_float2(v.z, v.w);
    }
  } else {
    const v2d* p2 = reinterpret_cast<const v2d*>(base) + idx;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const v2d v = NT ? __builtin_nontemporal_load(p2 + q) : p2[q];
      x[q] = make_float2(float(v.x), float(v.y));
    }
  }
}

// Pointers of the fold stage. The tables are read-only and never alias the
// partial-bucket output, which lets the compiler read them with scalar loads.
struct FoldArgs {
  const FrameDesc* __restrict__ descs;
  int uniform;
  const float2* __restrict__ wrow;
  const float2* __restrict__ wcol;
  const int32_t* __restrict__ rowlist;
  const int32_t* __restrict__ tiles;
  float2* __restrict__ part;
};

template <int TG, int V, int THREADS, bool C128, bool NT>
__device__ __forceinline__ void fold_tile(const FoldArgs& p, const void* __restrict__ input, int tile,
                                          int tiles_per_frame, int round0, int T, float2* red) {
  constexpr int P = THREADS * V;
  const int tid = threadIdx.x;
  // the tile's (frame, class, chunk), kept in scalar registers so that the
  // descriptor, row list and row weights are read with scalar loads
  int f, cls, chunk;
  if (p.uniform) {
    const int nch = p.descs[0].nchunks;
    f = tile / tiles_per_frame;
    const int rem = tile - f * tiles_per_frame;
    cls = rem / nch;
    chunk = rem - cls * nch;
  } else {
    const int32_t* t = p.tiles + 3 * int64_t(tile);
    f = t[0];
    cls = t[1];
    chunk = t[2];
  }
  f = __builtin_amdgcn_readfirstlane(f);
  cls = __builtin_amdgcn_readfirstlane(cls);
  chunk = __builtin_amdgcn_readfirstlane(chunk);
  const FrameDesc& d = p.descs[p.uniform ? 0 : f];
  const int64_t rel = p.uniform ? f : 0;
  const int nl = d.n_last, bl = d.b_last, R = d.rows_per_class, rows_total = d.rows_total;
  const float2* __restrict__ wrow = p.wrow + d.wrow_off;
  const float2* __restrict__ wcol = p.wcol + d.wcol_off;
  const int32_t* __restrict__ rl = p.rowlist + d.rowlist_off + int64_t(cls) * R;
  // segment mode: a launch folds one round (round0), whose samples are the
  // frame's segment round0
  const int64_t in_base = d.in_off + rel * d.in_stride + (d.segments ? int64_t(round0) * d.N : 0);
  const void* in = C128 ? static_cast<const void*>(static_cast<const double2*>(input) + in_base)
                        : static_cast<const void*>(static_cast<const float2*>(input) + in_base);

  float ar[TG][V], ai[TG][V];
#pragma unroll
  for (int s = 0; s < TG; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) ar[s][v] = ai[s][v] = 0.f;

  if (nl >= P) {
    // every thread walks all rows of the class; the row is uniform
    const int npass = d.chunk_cols / P;
    for (int pass = 0; pass < npass; ++pass) {
      const int col = chunk * d.chunk_cols + pass * P + tid * V;
      float cr[TG][V], ci[TG][V];
#pragma unroll
      for (int s = 0; s < TG; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) cr[s][v] = ci[s][v] = 0.f;
#pragma unroll 4
      for (int i = 0; i < R; ++i) {
        const int row = __builtin_amdgcn_readfirstlane(rl[i]);
        float2 x[V];
        load_vec<C128, NT, V>(in, int64_t(row) * nl + col, x);
#pragma unroll
        for (int s = 0; s < TG; ++s) {
          const float2 w = wrow[int64_t(round0 + s) * rows_total + row];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            cr[s][v] = fmaf(w.x, x[v].x, fmaf(-w.y, x[v].y, cr[s][v]));
            ci[s][v] = fmaf(w.x, x[v].y, fmaf(w.y, x[v].x, ci[s][v]));
          }
        }
      }
#pragma unroll
      for (int s = 0; s < TG; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const float2 w = wcol[int64_t(round0 + s) * nl + col + v];
          ar[s][v] = fmaf(w.x, cr[s][v], fmaf(-w.y, ci[s][v], ar[s][v]));
          ai[s][v] = fmaf(w.x, ci[s][v], fmaf(w.y, cr[s][v], ai[s][v]));
        }
    }
  } else {
    // short rows: G row groups, each covering the whole row
    const int G = P / nl;
    const int g = (tid * V) / nl;
    const int col = (tid * V) - g * nl;
    float cr[TG][V], ci[TG][V];
#pragma unroll
    for (int s = 0; s < TG; ++s)
#pragma unroll
      for (int v = 0; v < V; ++v) cr[s][v] = ci[s][v] = 0.f;
#pragma unroll 2
    for (int i = g; i < R; i += G) {
      const int row = rl[i];
      float2 x[V];
      load_vec<C128, NT, V>(in, int64_t(row) * nl + col, x);
#pragma unroll
      for (int s = 0; s < TG; ++s) {
        const float2 w = wrow[int64_t(round0 + s) * rows_total + row];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          cr[s][v] = fmaf(w.x, x[v].x, fmaf(-w.y, x[v].y, cr[s][v]));
          ci[s][v] = fmaf(w.x, x[v].y, fmaf(w.y, x[v].x, ci[s][v]));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < TG; ++s)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const float2 w = wcol[int64_t(round0 + s) * nl + col + v];
        ar[s][v] = w.x * cr[s][v] - w.y * ci[s][v];
        ai[s][v] = w.x * ci[s][v] + w.y * cr[s][v];
      }
  }

#pragma unroll
  for (int s = 0; s < TG; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) red[s * P + tid * V + v] = make_float2(ar[s][v], ai[s][v]);
  __syncthreads();

  // slot q holds residue q mod B_{D-1}; sum the P / B_{D-1} slots of each
  // residue in a fixed order
  const int nslots = P / bl;
  float2* part = p.part + d.part_off + rel * d.part_stride;
  for (int o = tid; o < TG * bl; o += THREADS) {
    const int s = o / bl;
    const int rho = o - s * bl;
    float sr = 0.f, si = 0.f;
    for (int k = 0; k < nslots; ++k) {
      const float2 v = red[s * P + rho + k * bl];
      sr += v.x;
      si += v.y;
    }
    part[(int64_t(chunk) * T + round0 + s) * d.B + int64_t(cls) * bl + rho] = make_float2(sr, si);
  }
}

// One work-group per tile; tiles of uneven batches are listed largest first
// so that the hardware dispatcher balances the tail.
template <int TG, int V, int THREADS, bool C128, bool NT>
__global__ __launch_bounds__(THREADS) void fold_kernel(FoldArgs p, const void* __restrict__ input,
                                                       int tiles_per_frame, int round0, int T) {
  __shared__ float2 red[TG * THREADS * V];
  fold_tile<TG, V, THREADS, C128, NT>(p, input, int(blockIdx.x), tiles_per_frame, round0, T, red);
}

template <int TG, int V, int THREADS, bool NT>
static hipError_t launch_fold_t(const DevPtrs& q, const void* input, int dtype, int64_t tpf,
                                int64_t ntiles, int round0, int T, hipStream_t st) {
  const FoldArgs p{q.descs, q.uniform, q.wrow, q.wcol, q.rowlist, q.tiles, q.part};
  if (dtype == RSFT_C128)
    hipLaunchKernelGGL((fold_kernel<TG, V, THREADS, true, NT>), dim3(unsigned(ntiles)), dim3(THREADS), 0,
                       st, p, input, int(tpf), round0, T);
  else
    hipLaunchKernelGGL((fold_kernel<TG, V, THREADS, false, NT>), dim3(unsigned(ntiles)), dim3(THREADS), 0,
                       st, p, input, int(tpf), round0, T);
  return hipGetLastError();
}

template <int V, int THREADS, bool NT>
static hipError_t launch_fold_v(const DevPtrs& p, const void* input, int dtype, int64_t tpf,
                                int64_t ntiles, int round0, int rounds, int T, hipStream_t st) {
  switch (rounds) {
    case 1: return launch_fold_t<1, V, THREADS, NT>(p, input, dtype, tpf, ntiles, round0, T, st);
    case 2: return launch_fold_t<2, V, THREADS, NT>(p, input, dtype, tpf, ntiles, round0, T, st);
    case 3: return launch_fold_t<3, V, THREADS, NT>(p, input, dtype, tpf, ntiles, round0, T, st);
    default: return launch_fold_t<4, V, THREADS, NT>(p, input, dtype, tpf, ntiles, round0, T, st);
  }
}

template <bool NT>
static int launch_fold_nt(const DevPtrs& p, const void* input, int dtype, int64_t tpf, int64_t ntiles,
                          int round0, int rounds, int T, const FoldConfig& cfg, hipStream_t st) {
  if (cfg.vec == 4 && cfg.threads == 256)
    return launch_fold_v<4, 256, NT>(p, input, dtype, tpf, ntiles, round0, rounds, T, st);
  if (cfg.vec == 4 && cfg.threads == 512)
    return launch_fold_v<4, 512, NT>(p, input, dtype, tpf, ntiles, round0, rounds, T, st);
  if (cfg.vec == 2 && cfg.threads == 256)
    return launch_fold_v<2, 256, NT>(p, input, dtype, tpf, ntiles, round0, rounds, T, st);
  if (cfg.vec == 2 && cfg.threads == 512)
    return launch_fold_v<2, 512, NT>(p, input, dtype, tpf, ntiles, round0, rounds, T, st);
  return hipErrorInvalidValue;
}

int launch_fold(const DevPtrs& p, const void* input, int dtype, int64_t nframes,
                int64_t tiles_per_frame, int64_t ntiles, int round0, int rounds, int T,
                const FoldConfig& cfg, void* stream) {
  (void)nframes;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ntiles <= 0) return hipSuccess;
  return cfg.nontemporal
             ? launch_fold_nt<true>(p, input, dtype, tiles_per_frame, ntiles, round0, rounds, T, cfg, st)
             : launch_fold_nt<false>(p, input, dtype, tiles_per_frame, ntiles, round0, rounds, T, cfg, st);
}

// ---------------------------------------------------------------------------
// dft: one work-group per (round, frame). The round's B partial buckets are
// summed over column chunks into LDS (separate re / im planes), then the DFT
// is applied along each dimension in place as complex matrix products on
// MFMA (v_mfma_f32_16x16x4_f32): for a dimension of length n, the lines
// along it are the columns of an n x (B/n) matrix X and Y = D_n X with
// D_n[k][b] = exp(-2 pi i ((k b) mod n) / n), the phase reduced exactly as
// an integer before the table lookup. The work is split into (16-line group,
// 16-output tile) items over all waves; a round of items holds whole line
// groups and is written back only after every item of the round is computed,
// so the transform is done in place. The epilogue reads the transform at the
// relabelled index (tau_s j mod B_d per dimension), writes the buckets in
// the paper's indexing, and sets flag bits |fhat|^2 >= gamma_s with ballots.
// ---------------------------------------------------------------------------

constexpr int kDftThreads = 1024;
constexpr int kDftWaves = kDftThreads / 64;
constexpr int kDftItems = 4;   // output tiles per wave between barriers

// LDS position of bucket index idx: one pad float after every row of the
// last dimension (row length 2^nl_shift), so that 16 lines read at the same
// position along that dimension fall into different banks.
__device__ __forceinline__ int lds_at(int idx, int nl_shift) { return idx + (idx >> nl_shift); }

// One 16-line x 16-output tile of Y = D_n X along a dimension: lines
// grp*16 .. grp*16+15, outputs k = kt*16 .. kt*16+15.
__device__ __forceinline__ void dft_tile(const float* __restrict__ re, const float* __restrict__ im,
                                         const float2* __restrict__ tw, int n, int inner_shift,
                                         int nlines, int nl_shift, int grp, int kt, floatx4& accR,
                                         floatx4& accI) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
  const int krow = lane >> 4;
  const int line = grp * 16 + col;
  const bool lvalid = line < nlines;
  const int inner = 1 << inner_shift;
  const int base = (line >> inner_shift) * n * inner + (line & (inner - 1));
  const int k = kt * 16 + col;
  accR = floatx4{0.f, 0.f, 0.f, 0.f};
  accI = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < n; b0 += 4) {
    const int b = b0 + krow;
    float xr = 0.f, xi = 0.f, dr = 0.f, di = 0.f;
    if (lvalid && b < n) {
      const int at = lds_at(base + b * inner, nl_shift);
      xr = re[at];
      xi = im[at];
    }
    if (k < n && b < n) {
      const float2 t = tw[(k * b) & (n - 1)];
      dr = t.x;
      di = t.y;
    }
    accR = __builtin_amdgcn_mfma_f32_16x16x4f32(dr, xr, accR, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_16x16x4f32(-di, xi, accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_16x16x4f32(dr, xi, accI, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_16x16x4f32(di, xr, accI, 0, 0, 0);
  }
}

// The DFT along one dimension of length n for all B / n lines, in place.
// Work items are (line group, output tile) pairs in group-major order; a
// round of kDftWaves * R items holds whole groups (the tiles per group,
// ceil(n/16) <= 8, divide 16), every item of a round is computed before any
// of its outputs is written, and rounds touch disjoint lines.
__device__ __forceinline__ void mode_product(float* __restrict__ re, float* __restrict__ im,
                                             const float2* __restrict__ tw, int n, int inner_shift,
                                             int nlines, int nl_shift) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int krow = lane >> 4;
  const int nkt = (n + 15) >> 4;
  const int items = ((nlines + 15) >> 4) * nkt;
  const int per_wave = (items + kDftWaves - 1) / kDftWaves;
  const int R = per_wave < kDftItems ? per_wave : kDftItems;
  const int inner = 1 << inner_shift;
  for (int r0 = 0; r0 < items; r0 += R * kDftWaves) {
    floatx4 accR[kDftItems], accI[kDftItems];
#pragma unroll
    for (int q = 0; q < kDftItems; ++q) {
      const int item = r0 + q * kDftWaves + wave;
      if (q < R && item < items)
        dft_tile(re, im, tw, n, inner_shift, nlines, nl_shift, item / nkt, item % nkt, accR[q], accI[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kDftItems; ++q) {
      const int item = r0 + q * kDftWaves + wave;
      if (q < R && item < items) {
        const int grp = item / nkt;
        const int kt = item % nkt;
        const int line = grp * 16 + col;
        if (line < nlines) {
          const int base = (line >> inner_shift) * n * inner + (line & (inner - 1));
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = kt * 16 + krow * 4 + r;
            if (k < n) {
              const int at = lds_at(base + k * inner, nl_shift);
              re[at] = accR[q][r];
              im[at] = accI[q][r];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kDftThreads) void dft_kernel(DevPtrs p, int T, int plane, int pad,
                                                          int frame0, int identity,
                                                          int nchunks_override) {
  extern __shared__ float smem[];
  float* re = smem;
  float* im = smem + plane;
  float2* tws = reinterpret_cast<float2*>(smem + 2 * plane);
  __shared__ uint32_t sel_prefix, sel_rank;
  __shared__ uint32_t hist[256];

  const int s = blockIdx.x;
  const int64_t f = frame0 + int64_t(blockIdx.y);
  const FrameDesc& d = desc_of(p, f);
  const int64_t rel = rel_of(p, f);
  const int B = d.B;
  // log2 of the last dimension's B (pads on), or no pads
  const int nls = pad ? __builtin_ctz(uint32_t(d.b_last)) : 31;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;


  // twiddles of each dimension, concatenated
  int twoff[kMaxDims];
  {
    int acc = 0;
    for (int dd = 0; dd < d.ndim; ++dd) {
      twoff[dd] = acc;
      for (int m = tid; m < d.b[dd]; m += kDftThreads) tws[acc + m] = p.tw[d.tw_off[dd] + m];
      acc += d.b[dd];
    }
  }
  // sum the column-chunk partials of this round
  const int nch = nchunks_override > 0 ? nchunks_override : d.nchunks;
  const float2* part = p.part + d.part_off + rel * d.part_stride;
  for (int idx = tid; idx < B; idx += kDftThreads) {
    float sr = 0.f, si = 0.f;
    for (int c = 0; c < nch; ++c) {
      const float2 v = part[(int64_t(c) * T + s) * B + idx];
      sr += v.x;
      si += v.y;
    }
    re[lds_at(idx, nls)] = sr;
    im[lds_at(idx, nls)] = si;
  }
  __syncthreads();

  for (int dd = 0; dd < d.ndim; ++dd) {
    const int n = d.b[dd];
    mode_product(re, im, tws + twoff[dd], n, d.bshift[dd], B / n, nls);
  }

  float2* bout = p.buckets + d.bucket_off + rel * d.bucket_stride + int64_t(s) * B;
  uint32_t* fout = p.flags + d.flag_off + rel * d.flag_stride + int64_t(s) * d.words;

  auto relabel = [&](int j) {
    int kf = 0;
    for (int dd = 0; dd < d.ndim; ++dd) {
      const int jd = (j >> d.bshift[dd]) & (d.b[dd] - 1);
      const int kd = identity ? jd : ((d.tau[s][dd] * jd) & (d.b[dd] - 1));
      kf |= kd << d.bshift[dd];
    }
    return kf;
  };

  double gamma = d.gamma[s];
  if (d.noise_mode == RSFT_NOISE_ESTIMATED) {
    // pass 1: buckets out, powers into the re plane (relabel is a bijection)
    for (int j = tid; j < B; j += kDftThreads) {
      const int kf = lds_at(relabel(j), nls);
      const float xr = re[kf], xi = im[kf];
      bout[j] = make_float2(xr, xi);
      re[kf] = xr * xr + xi * xi;
    }
    __syncthreads();
    // lower median X_(h), h = B/2, by 4 passes of 8-bit radix selection
    // (non-negative floats order like their bit patterns)
    uint32_t prefix = 0u, pmask = 0u, rank = uint32_t(B / 2 > 0 ? B / 2 : 1);
    for (int shift = 24; shift >= 0; shift -= 8) {
      for (int q = tid; q < 256; q += kDftThreads) hist[q] = 0u;
      __syncthreads();
      for (int idx = tid; idx < B; idx += kDftThreads) {
        const uint32_t u = __float_as_uint(re[lds_at(idx, nls)]);
        if ((u & pmask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t cum = 0u;
        for (uint32_t dg = 0; dg < 256u; ++dg) {
          if (cum + hist[dg] >= rank) {
            sel_prefix = prefix | (dg << shift);
            sel_rank = rank - cum;
            break;
          }
          cum += hist[dg];
        }
      }
      __syncthreads();
      prefix = sel_prefix;
      rank = sel_rank;
      pmask |= 255u << shift;
      __syncthreads();
    }
    const double xh = double(__uint_as_float(prefix));
    gamma = xh / d.renyi_h * d.log_inv_p1;
    for (int j0 = wave * 64; j0 < B; j0 += kDftThreads) {
      const int j = j0 + lane;
      bool flag = false;
      if (j < B) flag = double(re[lds_at(relabel(j), nls)]) >= gamma;
      const unsigned long long m = __ballot(flag);
      if (lane == 0) {
        const int w = j0 >> 5;
        fout[w] = uint32_t(m & 0xffffffffull);
        if (w + 1 < d.words) fout[w + 1] = uint32_t(m >> 32);
      }
    }
  } else {
    for (int j0 = wave * 64; j0 < B; j0 += kDftThreads) {
      const int j = j0 + lane;
      bool flag = false;
      if (j < B) {
        const int kf = lds_at(relabel(j), nls);
        const float xr = re[kf], xi = im[kf];
        bout[j] = make_float2(xr, xi);
        flag = double(xr * xr + xi * xi) >= gamma;
      }
      const unsigned long long m = __ballot(flag);
      if (lane == 0) {
        const int w = j0 >> 5;
        fout[w] = uint32_t(m & 0xffffffffull);
        if (w + 1 < d.words) fout[w + 1] = uint32_t(m >> 32);
      }
    }
  }
}

int launch_dft(const DevPtrs& p, int64_t nframes, int T, int plane, int pad, int sum_tw, int identity,
               int nchunks_override, void* stream) {
  if (nframes <= 0) return hipSuccess;
  const size_t shmem = size_t(2 * plane) * sizeof(float) + size_t(sum_tw) * sizeof(float2);
  hipLaunchKernelGGL(dft_kernel, dim3(unsigned(T), unsigned(nframes)), dim3(kDftThreads), shmem,
                     static_cast<hipStream_t>(stream), p, T, plane, pad, 0, identity, nchunks_override);
  return hipGetLastError();
}

static int launch_dft_frame(const DevPtrs& p, int64_t frame, int T, int plane, int pad, int sum_tw,
                            hipStream_t st) {
  const size_t shmem = size_t(2 * plane) * sizeof(float) + size_t(sum_tw) * sizeof(float2);
  hipLaunchKernelGGL(dft_kernel, dim3(unsigned(T), 1u), dim3(kDftThreads), shmem, st, p, T, plane,
                     pad, int(frame), 1, 1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// vote: abar_i = sum_s c_s[M(i, sigma_s)] with M_d(i) = [sigma_{s,d} i_d] >>
// log2 L_d (Def. 3), which by Properties 3-4 equals the accumulation of the
// reverse-mapped flags (Def. 4, eq. a_i); detection iff abar_i >= mu.
// One work-group per compaction chunk of 2^15 cells; each chunk's bitmap
// words are written completely and its detection count stored, so no atomics
// touch global memory. Index products are taken modulo 2^32 and masked,
// which equals the product modulo N_d (a power of two).
//
// vote_rows_kernel (rows of 64..4096 cells, T <= 4): a cell with >= mu votes
// is flagged in one of the rounds 0..T-mu, so each wave takes one row at a
// time and visits only the preimages of that row's flagged buckets (Def. 4):
// within a row the leading indices fix the leading bucket indices, so the
// candidates are i_last = [sigma_inv u]_N for u in [j L, (j + 1) L) over the
// flagged j of the row's bucket row. Work is proportional to the flagged
// buckets times L, the reverse-mapping cost of the paper's complexity table,
// instead of N T. A cell reached from round s0 is skipped when an earlier
// candidate round flags it (each cell is counted once). Hits go to a
// wave-private row bitmap in LDS, written out once per row.
//
// vote_kernel (any shape): the dense gather, every cell evaluated.
// ---------------------------------------------------------------------------

constexpr int kVoteThreads = 256;
constexpr int kRowWordsMax = 128;   // rows of up to 4096 cells

template <int D>
__global__ __launch_bounds__(kVoteThreads) void vote_kernel(DevPtrs p, int T, int mu, int frame0) {
  extern __shared__ uint32_t sflags[];
  __shared__ uint32_t wcount[kVoteThreads / 64];
  __shared__ uint32_t ssig[kMaxRounds * kMaxDims];
  const int c = blockIdx.x;
  const int64_t f = frame0 + int64_t(blockIdx.y);
  const FrameDesc& d = desc_of(p, f);
  if (c >= d.cchunks || d.ndim != D) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int words = d.words;
  const uint32_t* fl = p.flags + d.flag_off + rel * d.flag_stride;
  for (int w = tid; w < T * words; w += kVoteThreads) sflags[w] = fl[w];
  if (tid < T * D) ssig[tid] = uint32_t(d.sigma[tid / D][tid % D]);
  uint32_t nm[D], ls[D], bs[D], ns[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    nm[dd] = uint32_t(d.n[dd] - 1);
    ls[dd] = uint32_t(d.lshift[dd]);
    bs[dd] = uint32_t(d.bshift[dd]);
    ns[dd] = uint32_t(d.nshift[dd]);
  }
  const int64_t cell0 = int64_t(c) << kCompactShift;
  const int64_t rem = d.N - cell0;
  const int ncell = int(rem < (int64_t(1) << kCompactShift) ? rem : (int64_t(1) << kCompactShift));
  uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride + (cell0 >> 5);
  __syncthreads();

  uint32_t cnt = 0u;
  for (int base = wave * 64; base < ncell; base += kVoteThreads) {
    const int64_t i = cell0 + base + lane;
    bool hit = false;
    if (base + lane < ncell) {
      int votes = 0;
      for (int s = 0; s < T; ++s) {
        uint32_t jf = 0u;
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
          const uint32_t cd = uint32_t(i >> ns[dd]) & nm[dd];
          jf |= (((ssig[s * D + dd] * cd) & nm[dd]) >> ls[dd]) << bs[dd];
        }
        votes += int((sflags[s * words + (jf >> 5)] >> (jf & 31u)) & 1u);
      }
      hit = votes >= mu;
    }
    const unsigned long long m = __ballot(hit);
    if (lane == 0) {
      bm[base >> 5] = uint32_t(m & 0xffffffffull);
      if (base + 32 < ncell) bm[(base >> 5) + 1] = uint32_t(m >> 32);
      cnt += uint32_t(__popcll(m));
    }
  }
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t total = 0u;
    for (int w = 0; w < kVoteThreads / 64; ++w) total += wcount[w];
    p.chunk_counts[d.chunk_off + rel * d.chunk_stride + c] = total;
  }
}

// bit j (< 128) of a 128-bit row held as four words
__device__ __forceinline__ uint32_t row_bit(const uint32_t* w, uint32_t j) {
  return __builtin_amdgcn_ubfe(w[j >> 5], j & 31u, 1u);
}

template <int D, int TT>
__global__ __launch_bounds__(kVoteThreads) void vote_rows_kernel(DevPtrs p, int mu, int frame0) {
  extern __shared__ uint32_t sflags[];
  __shared__ uint32_t wcount[kVoteThreads / 64];
  __shared__ uint32_t rowbm[kVoteThreads / 64][kRowWordsMax];
  __shared__ uint32_t blist[kVoteThreads / 64][128];
  __shared__ uint32_t rowflags[kVoteThreads / 64][TT * 4];
  const int c = blockIdx.x;
  const int64_t f = frame0 + int64_t(blockIdx.y);
  const FrameDesc& d = desc_of(p, f);
  if (c >= d.cchunks || d.ndim != D) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int words = d.words;
  const uint32_t* fl = p.flags + d.flag_off + rel * d.flag_stride;
  for (int w = tid; w < TT * words; w += kVoteThreads) sflags[w] = fl[w];
  uint32_t nm[D], ls[D], bs[D], ns[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    nm[dd] = uint32_t(d.n[dd] - 1);
    ls[dd] = uint32_t(d.lshift[dd]);
    bs[dd] = uint32_t(d.bshift[dd]);
    ns[dd] = uint32_t(d.nshift[dd]);
  }
  uint32_t sig[TT][D], sinv_last[TT];
#pragma unroll
  for (int s = 0; s < TT; ++s) {
#pragma unroll
    for (int dd = 0; dd < D; ++dd) sig[s][dd] = uint32_t(d.sigma[s][dd]);
    sinv_last[s] = uint32_t(d.sigma_inv[s][D - 1]);
  }
  const uint32_t nl = nm[D - 1] + 1u;
  const uint32_t lsl = ls[D - 1];
  const uint32_t bl = uint32_t(d.b_last);
  const int row_words = int(nl >> 5);
  const int64_t cell0 = int64_t(c) << kCompactShift;
  const int64_t rem = d.N - cell0;
  const int ncell = int(rem < (int64_t(1) << kCompactShift) ? rem : (int64_t(1) << kCompactShift));
  const int nrows = ncell / int(nl);
  uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride + (cell0 >> 5);
  uint32_t* rb = rowbm[wave];
  uint32_t* lst = blist[wave];
  uint32_t* R = rowflags[wave];
  __syncthreads();

  uint32_t cnt = 0u;
  for (int r = wave; r < nrows; r += kVoteThreads / 64) {
    const int64_t iw = cell0 + int64_t(r) * nl;               // first cell of the row
    // the row's flags in every round: a 128-bit window at the row's bucket
    // row, kept in wave-private LDS (lane 4s + q fills word q of round s)
    if (lane < TT * 4) {
      const int s = lane >> 2;
      const int q = lane & 3;
      uint32_t rowpart = 0u;
#pragma unroll
      for (int ss = 0; ss < TT; ++ss) {   // uniform per round, then picked per lane
        uint32_t rp = 0u;
#pragma unroll
        for (int dd = 0; dd < D - 1; ++dd) {
          const uint32_t cd = uint32_t(iw >> ns[dd]) & nm[dd];
          rp |= (((sig[ss][dd] * cd) & nm[dd]) >> ls[dd]) << bs[dd];
        }
        if (ss == s) rowpart = rp;
      }
      const int wi = s * words + int(rowpart >> 5);
      uint32_t v = 0u;
      if (q == 0) {
        v = sflags[wi] >> (rowpart & 31u);                     // offset only when B_last < 32
        if (bl < 32u) v &= (1u << bl) - 1u;
      } else if (uint32_t(q) * 32u < bl) {
        v = sflags[wi + q];
      }
      R[lane] = v;
    }
    for (int q = lane; q < row_words; q += 64) rb[q] = 0u;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s0 = 0; s0 < TT; ++s0) {
      if (s0 > TT - mu) continue;
      // ordered list of the flagged bucket positions of the row in round s0
      const bool b0 = uint32_t(lane) < bl && row_bit(R + s0 * 4, uint32_t(lane)) != 0u;
      const bool b1 = bl > 64u && row_bit(R + s0 * 4, uint32_t(lane) + 64u) != 0u;
      const unsigned long long m0 = __ballot(b0);
      const unsigned long long m1 = __ballot(b1);
      const unsigned long long below = (1ull << lane) - 1ull;
      const int k0 = __popcll(m0);
      if (b0) lst[__popcll(m0 & below)] = uint32_t(lane);
      if (b1) lst[k0 + __popcll(m1 & below)] = uint32_t(lane) + 64u;
      __builtin_amdgcn_wave_barrier();
      const int ncand = (k0 + __popcll(m1)) << lsl;
      for (int ci = lane; ci < ncand; ci += 64) {
        const uint32_t jl = lst[ci >> lsl];
        const uint32_t u = (jl << lsl) | (uint32_t(ci) & ((1u << lsl) - 1u));
        // operands are below N_last <= 4096, so 24-bit products are exact
        const uint32_t il = __umul24(sinv_last[s0], u) & nm[D - 1];
        int votes = 1;   // round s0 maps il back to u, whose bucket is flagged
        bool skip = false;
#pragma unroll
        for (int s = 0; s < TT; ++s) {
          if (s == s0) continue;
          const uint32_t bit = row_bit(R + s * 4, (__umul24(sig[s][D - 1], il) & nm[D - 1]) >> lsl);
          if (s < s0 && bit) skip = true;
          votes += int(bit);
        }
        if (!skip && votes >= mu) atomicOr(&rb[il >> 5], 1u << (il & 31u));
      }
      __builtin_amdgcn_wave_barrier();
    }
    for (int q = lane; q < row_words; q += 64) {
      const uint32_t v = rb[q];
      bm[int64_t(r) * row_words + q] = v;
      cnt += uint32_t(__popc(v));
    }
    __builtin_amdgcn_wave_barrier();
  }
  // wave total, then work-group total
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_down(cnt, o);
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t total = 0u;
    for (int w = 0; w < kVoteThreads / 64; ++w) total += wcount[w];
    p.chunk_counts[d.chunk_off + rel * d.chunk_stride + c] = total;
  }
}

template <int D>
static void launch_vote_d(const DevPtrs& p, dim3 grid, size_t shmem, hipStream_t st, int T, int mu,
                          int frame0, bool rows) {
  if (rows) {
    switch (T) {
      case 1: hipLaunchKernelGGL((vote_rows_kernel<D, 1>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0); return;
      case 2: hipLaunchKernelGGL((vote_rows_kernel<D, 2>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0); return;
      case 3: hipLaunchKernelGGL((vote_rows_kernel<D, 3>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0); return;
      case 4: hipLaunchKernelGGL((vote_rows_kernel<D, 4>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0); return;
      default: break;
    }
  }
  hipLaunchKernelGGL(vote_kernel<D>, grid, dim3(kVoteThreads), shmem, st, p, T, mu, frame0);
}

int launch_vote(const DevPtrs& p, int64_t nframes, int T, int mu, int max_cchunks, int max_words,
                int dims_mask, int rows_ok, int frame0, void* stream) {
  if (nframes <= 0) return hipSuccess;
  const size_t shmem = size_t(T) * size_t(max_words) * sizeof(uint32_t);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid{unsigned(max_cchunks), unsigned(nframes), 1u};
  const bool rows = rows_ok != 0 && T <= 4;
  if (dims_mask & 1) launch_vote_d<1>(p, grid, shmem, st, T, mu, frame0, rows);
  if (dims_mask & 2) launch_vote_d<2>(p, grid, shmem, st, T, mu, frame0, rows);
  if (dims_mask & 4) launch_vote_d<3>(p, grid, shmem, st, T, mu, frame0, rows);
  if (dims_mask & 8) launch_vote_d<4>(p, grid, shmem, st, T, mu, frame0, rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scan: one work-group per frame turns the frame's chunk counters into
// chunk_offsets (rank of each compaction chunk's first detection in its
// frame, a running sum in row-major cell order) and counts[f]. The last
// work-group to finish (a device-scope counter, released and acquired with
// fences) computes offsets[f] = sum_{g<f} min(count_g, cap_g),
// offsets[nframes] = total, and resets the counter for the next launch.
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;

// inclusive scan of v over the work-group; returns it and the block total
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* wtot, int64_t& total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  int64_t pre = 0;
  total = 0;
#pragma unroll
  for (int q = 0; q < kScanThreads / 64; ++q) {
    if (q < wave) pre += wtot[q];
    total += wtot[q];
  }
  __syncthreads();
  return pre + incl;
}

__global__ __launch_bounds__(kScanThreads) void scan_kernel(DevPtrs p, int64_t nframes) {
  __shared__ int64_t wtot[kScanThreads / 64];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int64_t f = blockIdx.x;
  const FrameDesc& d = desc_of(p, f);
  const int64_t rel = rel_of(p, f);
  const int64_t base = d.chunk_off + rel * d.chunk_stride;
  int64_t run = 0;
  for (int c0 = 0; c0 < d.cchunks; c0 += kScanThreads) {
    const int c = c0 + tid;
    const int64_t v = c < d.cchunks ? int64_t(p.chunk_counts[base + c]) : 0;
    int64_t total;
    const int64_t incl = block_inclusive_scan(v, wtot, total);
    if (c < d.cchunks) p.chunk_offsets[base + c] = run + incl - v;
    run += total;
  }
  if (tid == 0) {
    p.counts[f] = run;
    __threadfence();
    const unsigned prev = atomicAdd(p.scan_done, 1u);
    is_last = prev == unsigned(nframes - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  int64_t carry = 0;
  for (int64_t g0 = 0; g0 < nframes; g0 += kScanThreads) {
    const int64_t g = g0 + tid;
    int64_t v = 0;
    if (g < nframes) {
      const int64_t cnt = __atomic_load_n(p.counts + g, __ATOMIC_RELAXED);
      const int64_t cap = desc_of(p, g).cap;
      v = cnt < cap ? cnt : cap;
    }
    int64_t total;
    const int64_t incl = block_inclusive_scan(v, wtot, total);
    if (g < nframes) p.offsets[g + 1] = carry + incl;
    carry += total;
  }
  if (tid == 0) {
    p.offsets[0] = 0;
    atomicExch(p.scan_done, 0u);
  }
}

int launch_scan(const DevPtrs& p, int64_t nframes, void* stream) {
  if (nframes <= 0) return hipSuccess;
  if (nframes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_kernel, dim3(unsigned(nframes)), dim3(kScanThreads), 0,
                     static_cast<hipStream_t>(stream), p, nframes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compact + estimate: one work-group per (frame, compaction chunk of 2^15
// cells). It reads the chunk's bitmap words in row-major order, lists the
// detected cells in LDS (popcount + block prefix sum) and gives each cell its
// rank in the frame's record range; then every listed cell gets its record:
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
// With at least 16 frames, block b serves frames congruent to b mod 8: work-
// groups are dealt to the eight XCDs round-robin, so each XCD's L2 holds the
// buckets and flags of only its own frames.
// ---------------------------------------------------------------------------

constexpr int kEstThreads = 256;
constexpr int kListMax = 2048;   // cells listed at once: a chunk's, else one pass's

// Per-frame constants of the estimate, uniform across the work-group.
template <int D, int M>
struct EstFrame {
  uint32_t nm[D], lm[D], ls[D], bs[D], ns[D];
  const float* ig[D];              // inverse flat-window gains per dimension
  uint32_t sig_est[M][D];
  const float2* bk_est[M];
  const uint32_t* fl;              // flags [T][words]
  const int32_t* sig;              // sigma [kMaxRounds][kMaxDims] of the descriptor
  int words;
};

template <int D, int M>
__device__ __forceinline__ void load_frame(const DevPtrs& p, const FrameDesc& d, int64_t rel,
                                           EstFrame<D, M>& e) {
  const float2* bk = p.buckets + d.bucket_off + rel * d.bucket_stride;
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    e.nm[dd] = uint32_t(d.n[dd] - 1);
    e.lm[dd] = uint32_t(d.l[dd] - 1);
    e.ls[dd] = uint32_t(d.lshift[dd]);
    e.bs[dd] = uint32_t(d.bshift[dd]);
    e.ns[dd] = uint32_t(d.nshift[dd]);
    e.ig[dd] = p.inv_gains + d.gain_off[dd];
  }
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int s = d.est_rounds[q];
#pragma unroll
    for (int dd = 0; dd < D; ++dd) e.sig_est[q][dd] = uint32_t(d.sigma[s][dd]);
    e.bk_est[q] = bk + int64_t(s) * d.B;
  }
  e.fl = p.flags + d.flag_off + rel * d.flag_stride;
  e.sig = &d.sigma[0][0];
  e.words = d.words;
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
template <int D, int M>
__device__ __forceinline__ float neighbour_power(const EstFrame<D, M>& e, const float (&g)[M][D][3],
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
    const float2 b = e.bk_est[q][jf];
    v[q] = (b.x * b.x + b.y * b.y) * gg;
  }
  return median_of<M>(v);
}

// The same for D >= 3, from the permuted index u0[q][d] = [sigma c]_N of the
// cell itself (no array indexed at run time).
template <int D, int M>
__device__ __forceinline__ float neighbour_power_dyn(const EstFrame<D, M>& e, const uint32_t (&u0)[M][D],
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
      const float ig = e.ig[dd][u & e.lm[dd]];
      gg *= ig * ig;
      jf |= (u >> e.ls[dd]) << e.bs[dd];
    }
    const float2 b = e.bk_est[q][jf];
    v[q] = (b.x * b.x + b.y * b.y) * gg;
  }
  return median_of<M>(v);
}

// One record. D <= 2: the 3^D neighbourhood lives in registers (loops
// unrolled); D >= 3: its 27 or 81 values are kept in this thread's LDS
// column `pcol` (stride kEstThreads) and visited by ordinary loops.
template <int D, int M>
__device__ __forceinline__ void write_record(const EstFrame<D, M>& e, int T, int64_t f,
                                             unsigned long long flat, rsft_detection* out,
                                             float* pcol) {
  constexpr int kNb = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;
  constexpr bool kRegs = D <= 2;
  constexpr int kCentre = (kNb - 1) / 2;
  uint32_t cell[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) cell[dd] = uint32_t(flat >> e.ns[dd]) & e.nm[dd];
  int votes = 0;
  for (int s = 0; s < T; ++s) {
    uint32_t jf = 0u;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
      const uint32_t u = (uint32_t(e.sig[s * kMaxDims + dd]) * cell[dd]) & e.nm[dd];
      jf |= (u >> e.ls[dd]) << e.bs[dd];
    }
    votes += int((e.fl[int64_t(s) * e.words + (jf >> 5)] >> (jf & 31u)) & 1u);
  }
  float preg[kRegs ? kNb : 1];
  if constexpr (kRegs) {
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
          const float ig = e.ig[dd][u & e.lm[dd]];
          g[q][dd][o] = ig * ig;
          jb[q][dd][o] = (u >> e.ls[dd]) << e.bs[dd];
        }
      }
    }
#pragma unroll
    for (int code = 0; code < kNb; ++code) preg[code] = neighbour_power<D, M>(e, g, jb, code);
  } else {
    uint32_t u0[M][D];
#pragma unroll
    for (int q = 0; q < M; ++q) {
#pragma unroll
      for (int dd = 0; dd < D; ++dd) u0[q][dd] = e.sig_est[q][dd] * cell[dd];
    }
#pragma unroll 1
    for (int code = 0; code < kNb; ++code) pcol[code * kEstThreads] = neighbour_power_dyn<D, M>(e, u0, code);
  }
  auto P = [&](int code) -> float {
    if constexpr (kRegs) return preg[code];
    else return pcol[code * kEstThreads];
  };
  const float p0 = P(kCentre);
  bool peak = true;
  auto visit = [&](int code) {
    if (code == kCentre) return;
    unsigned long long nflat = 0ull;
    int c = code;
#pragma unroll
    for (int dd = D - 1; dd >= 0; --dd) {
      const int o = c % 3 - 1;
      c /= 3;
      const uint32_t nb = (cell[dd] + uint32_t(o) + e.nm[dd] + 1u) & e.nm[dd];
      nflat |= (unsigned long long)nb << e.ns[dd];
    }
    if (nflat == flat) return;       // a dimension of length <= 2 wraps onto the cell
    const float pc = P(code);
    if (nflat < flat) {
      if (!(p0 > pc)) peak = false;
    } else {
      if (!(p0 >= pc)) peak = false;
    }
  };
  if constexpr (kRegs) {
#pragma unroll
    for (int code = 0; code < kNb; ++code) visit(code);
  } else {
#pragma unroll 1
    for (int code = 0; code < kNb; ++code) visit(code);
  }
  rsft_detection rec;
  rec.frame = f;
#pragma unroll
  for (int dd = 0; dd < kMaxDims; ++dd) {
    rec.idx[dd] = 0;
    rec.freq[dd] = 0.0;
  }
  int stride = 1;
#pragma unroll
  for (int dd = D - 1; dd >= 0; --dd) {
    const double delta = log_parabola_offset(P(kCentre - stride), p0, P(kCentre + stride));
    double fr = (double(cell[dd]) + delta) / double(e.nm[dd] + 1u);
    if (fr < 0.0) fr += 1.0;
    if (fr >= 1.0) fr -= 1.0;
    rec.idx[dd] = cell[dd];
    rec.freq[dd] = fr;
    stride *= 3;
  }
  rec.votes = votes;
  rec.is_peak = peak ? 1 : 0;
  rec.magnitude = sqrtf(p0);
  rec.reserved = 0.f;
  *out = rec;
}

// Records of list[0 .. min(n, room)) in batches of kEstThreads: each thread
// builds one record in LDS, then the work-group copies the batch out with
// contiguous 8-byte stores (a record is 88 bytes, 8-byte aligned).
template <int D, int M>
__device__ __forceinline__ void estimate_list(const DevPtrs& p, const FrameDesc& d, int64_t f,
                                              int64_t rel, int T, const uint32_t* list, int n,
                                              unsigned long long cell0, rsft_detection* out,
                                              int64_t room, float* pcol, rsft_detection* stage) {
  EstFrame<D, M> e;
  load_frame<D, M>(p, d, rel, e);
  const int lim = int(n < room ? n : room);
  constexpr int kWords = int(sizeof(rsft_detection) / 8);
  for (int q0 = 0; q0 < lim; q0 += kEstThreads) {
    const int q = q0 + int(threadIdx.x);
    if (q < lim) write_record<D, M>(e, T, f, cell0 | (unsigned long long)list[q], stage + threadIdx.x, pcol);
    __syncthreads();
    const int nw = (lim - q0 < kEstThreads ? lim - q0 : kEstThreads) * kWords;
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(stage);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(out + q0);
    for (int w = int(threadIdx.x); w < nw; w += kEstThreads) dst[w] = src[w];
    __syncthreads();
  }
}

template <int D, int M>
__global__ __launch_bounds__(kEstThreads) void compact_estimate_kernel(DevPtrs p, int T,
                                                                       int64_t nframes,
                                                                       int max_cchunks,
                                                                       int xcd_groups) {
  constexpr int kNb = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;
  __shared__ uint32_t list[kListMax];
  __shared__ uint32_t wsum[kEstThreads / 64];
  __shared__ rsft_detection stage[kEstThreads];
  __shared__ float pbuf[D >= 3 ? kNb * kEstThreads : 1];
  int64_t f;
  int c;
  const int64_t b = blockIdx.x;
  if (xcd_groups) {
    const int64_t k = b >> 3;
    f = (k / max_cchunks) * 8 + (b & 7);
    c = int(k % max_cchunks);
  } else {
    f = b / max_cchunks;
    c = int(b % max_cchunks);
  }
  if (f >= nframes) return;
  const FrameDesc& d = desc_of(p, f);
  if (c >= d.cchunks || d.ndim != D || d.n_est != M) return;
  const int64_t rel = rel_of(p, f);
  const int64_t ck = d.chunk_off + rel * d.chunk_stride + c;
  if (p.chunk_counts[ck] == 0u) return;
  const int64_t rank0 = p.chunk_offsets[ck];
  const int64_t cap = d.cap;
  if (rank0 >= cap) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  rsft_detection* out = p.records + p.offsets[f] + rank0;
  const uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride;
  const int w0 = c << (kCompactShift - 5);
  const int wend = min(d.bitmap_words, w0 + (1 << (kCompactShift - 5)));
  const unsigned long long cell0 = (unsigned long long)c << kCompactShift;
  const int64_t room0 = cap - rank0;
  float* pcol = pbuf + threadIdx.x;
  const uint32_t chunk_count = p.chunk_counts[ck];
  if (chunk_count <= uint32_t(kListMax)) {
    // one pass: thread t lists the set bits of words w0 + 4t .. w0 + 4t + 3
    constexpr int kWpt = (1 << (kCompactShift - 5)) / kEstThreads;
    uint32_t wv[kWpt];
    int pc = 0;
#pragma unroll
    for (int q = 0; q < kWpt; ++q) {
      const int w = w0 + tid * kWpt + q;
      wv[q] = w < wend ? bm[w] : 0u;
      pc += __popc(wv[q]);
    }
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
    estimate_list<D, M>(p, d, f, rel, T, list, min(total, kListMax), cell0, out, room0, pcol, stage);
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
    estimate_list<D, M>(p, d, f, rel, T, list, total, cell0, out + running, room0 - running, pcol,
                        stage);
    running += total;
    if (running >= room0) return;   // uniform: the frame's capacity is used up
    __syncthreads();
  }
}

template <int D>
static void launch_estimate_d(const DevPtrs& p, dim3 grid, hipStream_t st, int T, int64_t nframes,
                              int max_cchunks, int xcd, int est_mask) {
  if (est_mask & 2) hipLaunchKernelGGL((compact_estimate_kernel<D, 1>), grid, dim3(kEstThreads), 0, st, p, T, nframes, max_cchunks, xcd);
  if (est_mask & 4) hipLaunchKernelGGL((compact_estimate_kernel<D, 2>), grid, dim3(kEstThreads), 0, st, p, T, nframes, max_cchunks, xcd);
  if (est_mask & 8) hipLaunchKernelGGL((compact_estimate_kernel<D, 3>), grid, dim3(kEstThreads), 0, st, p, T, nframes, max_cchunks, xcd);
  if (est_mask & 16) hipLaunchKernelGGL((compact_estimate_kernel<D, 4>), grid, dim3(kEstThreads), 0, st, p, T, nframes, max_cchunks, xcd);
  if (est_mask & 32) hipLaunchKernelGGL((compact_estimate_kernel<D, 5>), grid, dim3(kEstThreads), 0, st, p, T, nframes, max_cchunks, xcd);
}

int launch_estimate(const DevPtrs& p, int64_t nframes, int T, int max_cchunks, int dims_mask,
                    int est_mask, void* stream) {
  if (nframes <= 0) return hipSuccess;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int xcd = nframes >= 16 ? 1 : 0;
  const int64_t rows = xcd ? ((nframes + 7) / 8) * 8 : nframes;
  const int64_t blocks = rows * int64_t(max_cchunks);
  if (blocks >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  const dim3 grid{unsigned(blocks), 1u, 1u};
  if (dims_mask & 1) launch_estimate_d<1>(p, grid, st, T, nframes, max_cchunks, xcd, est_mask);
  if (dims_mask & 2) launch_estimate_d<2>(p, grid, st, T, nframes, max_cchunks, xcd, est_mask);
  if (dims_mask & 4) launch_estimate_d<3>(p, grid, st, T, nframes, max_cchunks, xcd, est_mask);
  if (dims_mask & 8) launch_estimate_d<4>(p, grid, st, T, nframes, max_cchunks, xcd, est_mask);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-frame comparator: Algorithm 1 taken literally for one frame and one
// round at a time. plain_fold gathers the permuted samples (Def. 1, tau = 0),
// applies both windows and aliases (Def. 2): one wave per bucket b sums
// z[b + B l] = wbar[n] w[[sigma n]] r[[sigma n]] over the L terms, n_d =
// b_d + B_d l_d. Buckets are written in the paper's indexing (no relabel).
// Its votes are taken with the vote stage launched for that frame alone.
// ---------------------------------------------------------------------------

constexpr int kPlainThreads = 256;

template <bool C128>
__global__ __launch_bounds__(kPlainThreads) void plain_fold_kernel(DevPtrs p, const void* __restrict__ input,
                                                                   int64_t f, int s) {
  const FrameDesc& d = desc_of(p, f);
  const int64_t rel = rel_of(p, f);
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (kPlainThreads / 64) + (threadIdx.x >> 6);
  if (b >= d.B) return;
  const int64_t in_base = d.in_off + rel * d.in_stride + (d.segments ? int64_t(s) * d.N : 0);
  const int64_t L = int64_t(1) << d.Lshift;
  float accr = 0.f, acci = 0.f;
  for (int64_t l = lane; l < L; l += 64) {
    unsigned long long src = 0ull;
    float wr = 1.f, wi = 0.f;
    for (int dd = 0; dd < d.ndim; ++dd) {
      const uint32_t bd = uint32_t(b >> d.bshift[dd]) & uint32_t(d.b[dd] - 1);
      const uint32_t ld = uint32_t(l >> d.tshift[dd]) & uint32_t(d.l[dd] - 1);
      const uint32_t nd = bd + uint32_t(d.b[dd]) * ld;
      const uint32_t md = (uint32_t(d.sigma[s][dd]) * nd) & uint32_t(d.n[dd] - 1);
      const float w = p.win[d.win_off[dd] + md];
      const float2 fb = p.flat[d.flat_off[dd] + nd];
      const float tr = wr * fb.x - wi * fb.y;
      const float ti = wr * fb.y + wi * fb.x;
      wr = tr * w;
      wi = ti * w;
      src |= (unsigned long long)md << d.nshift[dd];
    }
    float xr, xi;
    if constexpr (C128) {
      const double2 v = static_cast<const double2*>(input)[in_base + int64_t(src)];
      xr = float(v.x);
      xi = float(v.y);
    } else {
      const float2 v = static_cast<const float2*>(input)[in_base + int64_t(src)];
      xr = v.x;
      xi = v.y;
    }
    accr = fmaf(wr, xr, fmaf(-wi, xi, accr));
    acci = fmaf(wr, xi, fmaf(wi, xr, acci));
  }
  for (int off = 32; off > 0; off >>= 1) {
    accr += __shfl_down(accr, off);
    acci += __shfl_down(acci, off);
  }
  if (lane == 0) {
    float2* part = p.part + d.part_off + rel * d.part_stride;
    part[int64_t(s) * d.B + b] = make_float2(accr, acci);
  }
}

int launch_plain_fold(const DevPtrs& p, const void* input, int dtype, int64_t frame, int round, int B,
                      void* stream) {
  const unsigned blocks = unsigned((B + kPlainThreads / 64 - 1) / (kPlainThreads / 64));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == RSFT_C128)
    hipLaunchKernelGGL(plain_fold_kernel<true>, dim3(blocks), dim3(kPlainThreads), 0, st, p, input,
                       frame, round);
  else
    hipLaunchKernelGGL(plain_fold_kernel<false>, dim3(blocks), dim3(kPlainThreads), 0, st, p, input,
                       frame, round);
  return hipGetLastError();
}

int launch_plain_dft(const DevPtrs& p, int64_t frame, int T, int plane, int pad, int sum_tw,
                     void* stream) {
  return launch_dft_frame(p, frame, T, plane, pad, sum_tw, static_cast<hipStream_t>(stream));
}

}  // namespace rsft

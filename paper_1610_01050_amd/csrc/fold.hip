// fold stage of the RSFT hot path (and the per-frame comparator's gather).
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

#include "device_common.h"

namespace rsft {

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
    const int grp = rem / nch;
    chunk = rem - grp * nch;
    cls = grp * p.descs[0].fold_cpt;
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
  const int nl = d.fold_nl, bl = d.fold_bl, R = d.rows_per_class, rows_total = d.rows_total;
  const int cpt = d.fold_cpt;
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
    // short rows: G row groups, each covering the whole row; the tile's
    // cpt classes take G / cpt consecutive groups each
    const int G = P / nl;
    const int gpc = G / cpt;
    const int g = (tid * V) / nl;
    const int col = (tid * V) - g * nl;
    const int j = g / gpc;
    const int32_t* __restrict__ rlj = rl + j * R;
    float cr[TG][V], ci[TG][V];
#pragma unroll
    for (int s = 0; s < TG; ++s)
#pragma unroll
      for (int v = 0; v < V; ++v) cr[s][v] = ci[s][v] = 0.f;
    // kRows rows of the group at a time: their row indices, then their
    // samples and row weights, are loaded together before any is used
    constexpr int kRows = 4;
    for (int i0 = g - j * gpc; i0 < R; i0 += kRows * gpc) {
      int row[kRows];
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = i0 + k * gpc;
        row[k] = rlj[i < R ? i : i0];
      }
      float2 x[kRows][V];
      float2 w[kRows][TG];
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        load_vec<C128, NT, V>(in, int64_t(row[k]) * nl + col, x[k]);
#pragma unroll
        for (int s = 0; s < TG; ++s) w[k][s] = wrow[int64_t(round0 + s) * rows_total + row[k]];
      }
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        if (i0 + k * gpc < R) {
#pragma unroll
          for (int s = 0; s < TG; ++s)
#pragma unroll
            for (int v = 0; v < V; ++v) {
              cr[s][v] = fmaf(w[k][s].x, x[k][v].x, fmaf(-w[k][s].y, x[k][v].y, cr[s][v]));
              ci[s][v] = fmaf(w[k][s].x, x[k][v].y, fmaf(w[k][s].y, x[k][v].x, ci[s][v]));
            }
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

  // Sum the P / fold_bl slots of each residue in a fixed order. One
  // dimension: slot q holds residue q mod B_{D-1}. Two flattened: slot q =
  // i * N_{D-1} + j (mod the pass) holds residue (i mod B_{D-2}) B_{D-1} +
  // (j mod B_{D-1}), and residue (r1, r2) owns the slots r2 + B_{D-1} a +
  // (r1 + B_{D-2} m) N_{D-1}.
  // With cpt classes per tile, class j owns the slots [j, j + 1) * P / cpt.
  const int nslots = P / bl / cpt;
  float2* part = p.part + d.part_off + rel * d.part_stride;
  if (bl == d.fold_bin) {
    for (int o = tid; o < TG * cpt * bl; o += THREADS) {
      const int s = o / (cpt * bl);
      const int rem = o - s * cpt * bl;
      const int j = rem / bl;
      const int rho = rem - j * bl;
      const float2* rs = red + s * P + j * nslots * bl + rho;
      float sr = 0.f, si = 0.f;
      for (int k = 0; k < nslots; ++k) {
        const float2 v = rs[k * bl];
        sr += v.x;
        si += v.y;
      }
      part[(int64_t(chunk) * T + round0 + s) * d.B + int64_t(cls + j) * bl + rho] = make_float2(sr, si);
    }
  } else {
    const int bin = d.fold_bin, lw = d.fold_lw;
    const int na = (1 << lw) / bin;              // slots of a residue within one N_{D-1} row
    const int period = (bl / bin) << lw;         // B_{D-2} N_{D-1}
    for (int o = tid; o < TG * bl; o += THREADS) {
      const int s = o / bl;
      const int rho = o - s * bl;
      const int r1 = rho / bin, r2 = rho - r1 * bin;
      float sr = 0.f, si = 0.f;
      for (int m = 0; m < P / period; ++m)
        for (int a = 0; a < na; ++a) {
          const float2 v = red[s * P + m * period + (r1 << lw) + r2 + a * bin];
          sr += v.x;
          si += v.y;
        }
      part[(int64_t(chunk) * T + round0 + s) * d.B + int64_t(cls) * bl + rho] = make_float2(sr, si);
    }
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

}  // namespace rsft

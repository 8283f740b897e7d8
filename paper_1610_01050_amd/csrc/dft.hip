// dft stage of the RSFT hot path: B-point N-D DFT on MFMA, threshold, flags.

#include "device_common.h"

namespace rsft {

// ---------------------------------------------------------------------------
// dft: one work-group per (round, frame). The round's B partial buckets are
// summed over column chunks into LDS (separate re / im planes), then the DFT
// is applied along each dimension in place, with complex products on MFMA
// (v_mfma_f32_16x16x4_f32, four real products per complex one). For a
// dimension of length n the lines along it are the columns of an n x (B/n)
// matrix X, and Y = D_n X with D_n[k][b] = exp(-2 pi i ((k b) mod n) / n),
// the phase reduced exactly as an integer before the table lookup:
//   n = 16 r  decimation in frequency, radix-r pre-combination on the VALU
//             and 16-point DFTs on MFMA (mode_product_r16);
//   n < 16    the dense product, in (16-line group, 16-output tile) items
//             over all waves; a round of items holds whole line groups and
//             is written back only after every item of the round is
//             computed (mode_product).
// The epilogue reads the transform at the relabelled index (tau_s j mod B_d
// per dimension), writes the buckets and their squared magnitudes in the
// paper's indexing, and sets flag bits |fhat|^2 >= gamma_s with ballots.
// ---------------------------------------------------------------------------

constexpr int kDftItems = 2;   // output tiles per wave between barriers

// LDS position of bucket index idx: one pad float after every row of the
// last dimension (row length 2^nl_shift), so that 16 lines read at the same
// position along that dimension fall into different banks.
__device__ __forceinline__ int lds_at(int idx, int nl_shift) { return idx + (idx >> nl_shift); }

// One 16-line x 16-output tile of Y = D_n X along a dimension: lines
// grp*16 .. grp*16+15, outputs k = kt*16 .. kt*16+15. Four k-steps of the
// contraction are read from LDS at once (branch-free: an index outside the
// matrix reads element 0 and is replaced by zero), then fed to two
// accumulator pairs, which halves the chain of dependent MFMAs.
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
  const bool kvalid = k < n;
  floatx4 aR0{0.f, 0.f, 0.f, 0.f}, aI0{0.f, 0.f, 0.f, 0.f};
  floatx4 aR1{0.f, 0.f, 0.f, 0.f}, aI1{0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < n; b0 += 16) {
    float xr[4], xi[4], dr[4], di[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + 4 * u + krow;
      const bool xv = lvalid && b < n;
      const bool dv = kvalid && b < n;
      const int at = xv ? lds_at(base + b * inner, nl_shift) : 0;
      const float vr = re[at];
      const float vi = im[at];
      const float2 t = tw[(k * b) & (n - 1)];
      xr[u] = xv ? vr : 0.f;
      xi[u] = xv ? vi : 0.f;
      dr[u] = dv ? t.x : 0.f;
      di[u] = dv ? t.y : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      aR0 = __builtin_amdgcn_mfma_f32_16x16x4f32(dr[u], xr[u], aR0, 0, 0, 0);
      aI0 = __builtin_amdgcn_mfma_f32_16x16x4f32(dr[u], xi[u], aI0, 0, 0, 0);
      aR1 = __builtin_amdgcn_mfma_f32_16x16x4f32(dr[u + 1], xr[u + 1], aR1, 0, 0, 0);
      aI1 = __builtin_amdgcn_mfma_f32_16x16x4f32(dr[u + 1], xi[u + 1], aI1, 0, 0, 0);
      aR0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-di[u], xi[u], aR0, 0, 0, 0);
      aI0 = __builtin_amdgcn_mfma_f32_16x16x4f32(di[u], xr[u], aI0, 0, 0, 0);
      aR1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-di[u + 1], xi[u + 1], aR1, 0, 0, 0);
      aI1 = __builtin_amdgcn_mfma_f32_16x16x4f32(di[u + 1], xr[u + 1], aI1, 0, 0, 0);
    }
  }
  accR = aR0 + aR1;
  accI = aI0 + aI1;
}

// The DFT along one dimension of length n for all B / n lines, in place.
// Work items are (line group, output tile) pairs in group-major order; a
// round of kWaves * R items holds whole groups (the tiles per group,
// ceil(n/16) <= 8, divide 16), every item of a round is computed before any
// of its outputs is written, and rounds touch disjoint lines.
template <int kWaves>
__device__ __forceinline__ void mode_product(float* __restrict__ re, float* __restrict__ im,
                                             const float2* __restrict__ tw, int n, int inner_shift,
                                             int nlines, int nl_shift) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int krow = lane >> 4;
  const int nkt = (n + 15) >> 4;
  const int items = ((nlines + 15) >> 4) * nkt;
  const int per_wave = (items + kWaves - 1) / kWaves;
  const int R = per_wave < kDftItems ? per_wave : kDftItems;
  const int inner = 1 << inner_shift;
  for (int r0 = 0; r0 < items; r0 += R * kWaves) {
    floatx4 accR[kDftItems], accI[kDftItems];
#pragma unroll
    for (int q = 0; q < kDftItems; ++q) {
      const int item = r0 + q * kWaves + wave;
      if (q < R && item < items)
        dft_tile(re, im, tw, n, inner_shift, nlines, nl_shift, item / nkt, item % nkt, accR[q], accI[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kDftItems; ++q) {
      const int item = r0 + q * kWaves + wave;
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

// The DFT along one dimension of length n = 16 r (r = 1, 2, 4, 8), in
// place, by decimation in frequency: with j = j1 + 16 j2 and k = k2 + r k1
// (j1, k1 < 16; j2, k2 < r), W_m = exp(-2 pi i / m),
//   Z[k2 + r k1] = sum_{j1} W_16^{j1 k1} y_{k2}[j1],
//   y_{k2}[j1]   = W_n^{j1 k2} sum_{j2} W_r^{j2 k2} x[j1 + 16 j2].
// Each lane forms its y on the VALU (r complex products and one twiddle per
// k-step, twiddles read from the LDS table) and the 16-point DFTs run on MFMA: a tile is 16 columns (line,
// k2) = 16 / r whole lines, so it reads and writes only its own lines and
// the transform needs no barrier between reading and writing. Every
// exponent is reduced modulo n as an integer before the table lookup
// (W_16^a = tw[a r], W_r^a = tw[16 a]).
template <int kWaves>
__device__ __forceinline__ void mode_product_r16(float* __restrict__ re, float* __restrict__ im,
                                                 const float2* __restrict__ tw, int n, int inner_shift,
                                                 int nlines, int nl_shift) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int kk = lane >> 4;
  const int r = n >> 4;
  const int rshift = __builtin_ctz(uint32_t(r));
  const int k2 = col & (r - 1);
  const int inner = 1 << inner_shift;
  const int mask = n - 1;
  const int ntiles = ((nlines << rshift) + 15) >> 4;
  for (int tile = wave; tile < ntiles; tile += kWaves) {
    const int line = (tile << (4 - rshift)) + (col >> rshift);
    const bool lvalid = line < nlines;
    const int base = lvalid ? (line >> inner_shift) * n * inner + (line & (inner - 1)) : 0;
    floatx4 accR{0.f, 0.f, 0.f, 0.f}, accI{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
      const int j1 = 4 * t + kk;
      const float2 a = tw[(j1 * col * r) & mask];    // W_16^{j1 k1}, k1 = col (MFMA A operand)
      const float2 t1 = tw[(j1 * k2) & mask];        // W_n^{j1 k2}
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int j2 = 0; j2 < 8; ++j2) {
        if (j2 < r) {
          const int at = lds_at(base + (j1 + 16 * j2) * inner, nl_shift);
          const float xr = re[at], xi = im[at];
          const float2 w = tw[(16 * j2 * k2) & mask];
          sr += w.x * xr - w.y * xi;
          si += w.x * xi + w.y * xr;
        }
      }
      float yr = t1.x * sr - t1.y * si;
      float yi = t1.x * si + t1.y * sr;
      yr = lvalid ? yr : 0.f;
      yi = lvalid ? yi : 0.f;
      accR = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, yr, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, yi, accI, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, yi, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, yr, accI, 0, 0, 0);
    }
    if (lvalid) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k2 + r * (4 * kk + q);
        const int at = lds_at(base + k * inner, nl_shift);
        re[at] = accR[q];
        im[at] = accI[q];
      }
    }
  }
  __syncthreads();
}

// TH threads per work-group (64 .. 1024): one wave per transform suits small
// B (many transforms, each short), sixteen suit large B.
template <int TH>
__global__ __launch_bounds__(TH) void dft_kernel(DevPtrs p, int T, int plane, int pad, int frame0, int identity,
                                                 int nchunks_override, const int32_t* __restrict__ order) {
  constexpr int kDftThreads = TH;
  constexpr int kDftWaves = TH / 64;
  extern __shared__ float smem[];
  float* re = smem;
  float* im = smem + plane;
  float2* tws = reinterpret_cast<float2*>(smem + 2 * plane);
  __shared__ uint32_t sel_prefix, sel_rank;
  __shared__ uint32_t hist[256];

  const int s = blockIdx.x;
  const int64_t f = order ? int64_t(order[blockIdx.y]) : frame0 + int64_t(blockIdx.y);
  const FrameDesc& d = desc_of(p, f);
  const int64_t rel = rel_of(p, f);
  const int B = d.B;
  // log2 of the last dimension's B (pads on), or no pads
  const int nls = pad ? __builtin_ctz(uint32_t(d.b_last)) : 31;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;


  // Twiddles of each dimension (concatenated; B_d <= 128) and the
  // column-chunk partials of this round. (Every dimension's descriptor
  // fields are read first; entries beyond ndim exist and are not used.)
  int twoff[kMaxDims];
  {
    const int nd = d.ndim;
    int bd[kMaxDims];
    int64_t toff[kMaxDims];
#pragma unroll
    for (int dd = 0; dd < kMaxDims; ++dd) {
      bd[dd] = d.b[dd];
      toff[dd] = d.tw_off[dd];
    }
    int acc = 0;
#pragma unroll
    for (int dd = 0; dd < kMaxDims; ++dd) {
      twoff[dd] = acc;
      if (dd < nd) {
        for (int i = tid; i < bd[dd]; i += kDftThreads) tws[acc + i] = p.tw[toff[dd] + i];
        acc += bd[dd];
      }
    }
  }
  const int nch = nchunks_override > 0 ? nchunks_override : d.nchunks;
  const float2* part = p.part + d.part_off + rel * d.part_stride + int64_t(s) * B;
  // groups of kGrp buckets per thread (one group when B <= 4096)
  constexpr int kGrp = 4;
  for (int g0 = 0; g0 < B; g0 += kGrp * kDftThreads) {
    float2 sum[kGrp];
#pragma unroll
    for (int q = 0; q < kGrp; ++q) {
      const int idx = g0 + q * kDftThreads + tid;
      sum[q] = idx < B ? part[idx] : make_float2(0.f, 0.f);
    }
    for (int c = 1; c < nch; ++c) {
      const float2* pc = part + int64_t(c) * T * B;
      float2 v[kGrp];
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const int idx = g0 + q * kDftThreads + tid;
        v[q] = idx < B ? pc[idx] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        sum[q].x += v[q].x;
        sum[q].y += v[q].y;
      }
    }
#pragma unroll
    for (int q = 0; q < kGrp; ++q) {
      const int idx = g0 + q * kDftThreads + tid;
      if (idx < B) {
        re[lds_at(idx, nls)] = sum[q].x;
        im[lds_at(idx, nls)] = sum[q].y;
      }
    }
  }
  __syncthreads();

  for (int dd = 0; dd < d.ndim; ++dd) {
    const int n = d.b[dd];
    if (n >= 16)
      mode_product_r16<kDftWaves>(re, im, tws + twoff[dd], n, d.bshift[dd], B / n, nls);
    else
      mode_product<kDftWaves>(re, im, tws + twoff[dd], n, d.bshift[dd], B / n, nls);
  }

  float2* bout = p.buckets + d.bucket_off + rel * d.bucket_stride + int64_t(s) * B;
  float* pout = p.powers + d.bucket_off + rel * d.bucket_stride + int64_t(s) * B;
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
      const float pw = xr * xr + xi * xi;
      bout[j] = make_float2(xr, xi);
      pout[j] = pw;
      re[kf] = pw;
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
        const float pw = xr * xr + xi * xi;
        bout[j] = make_float2(xr, xi);
        pout[j] = pw;
        flag = double(pw) >= gamma;
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

// ---------------------------------------------------------------------------
// dft in two passes (frames of D >= 2, KNOWN noise floor): each round's
// transform is spread over many small work-groups instead of one.
//   pass 1: work-group (frame, round, slab group). A slab is the S = B / B_0
//           buckets of one index along dimension 0; a group of G slabs
//           (G S <= kSplitGroup, or one slab when S is larger) sums its
//           column-chunk partials into LDS and
//           is transformed along dimensions 1 .. D-1 (the same mode
//           products), then written in transform order to `inter`.
//   pass 2: work-group (frame, round, column group) of 1024 threads when the
//           plan's largest B_0 is >= 64, else 256. It owns C = min(S, 32)
//           consecutive trailing output positions J' (the paper's indexing)
//           for every index along dimension 0: it loads the transform
//           columns K' = tau J' (per dimension, tau_{s,d} j_d mod B_d), the
//           B_0-point DFT along dimension 0 in LDS, then reads row k_0 =
//           tau_{s,0} j_0 for output row j_0 and writes buckets, squared
//           magnitudes and flags: a group owns whole flag words (C = 32, or
//           the whole transform when S < 32).
// ---------------------------------------------------------------------------

constexpr int kSplitThreads = 256;
constexpr int kSplitWaves = kSplitThreads / 64;

__device__ __forceinline__ int64_t split_frame(const int32_t* order, int64_t slot) {
  return order ? int64_t(order[slot]) : slot;
}

__global__ __launch_bounds__(kSplitThreads) void dft_pass1_kernel(DevPtrs p, int T, float2* __restrict__ inter,
                                                                  const int32_t* __restrict__ order) {
  extern __shared__ float smem[];
  const int64_t f = split_frame(order, blockIdx.z);
  const int s = blockIdx.y;
  const FrameDesc& d = desc_of(p, f);
  const int nd = d.ndim, B = d.B, b0 = d.b[0];
  const int S = B / b0;
  const int G = S >= kSplitGroup ? 1 : (kSplitGroup / S < b0 ? kSplitGroup / S : b0);
  const int groups = b0 / G;
  if (int(blockIdx.x) >= groups) return;
  const int E = G * S;                          // buckets of this work-group
  const int nls = __builtin_ctz(uint32_t(d.b[nd - 1]));
  const int plane = E + (E >> nls);
  float* re = smem;
  float* im = smem + plane;
  float2* tws = reinterpret_cast<float2*>(smem + 2 * plane);
  const int tid = threadIdx.x;
  const int64_t rel = rel_of(p, f);
  // twiddles of dimensions 1 .. D-1, concatenated
  int twoff[kMaxDims];
  {
    int acc = 0;
#pragma unroll
    for (int dd = 0; dd < kMaxDims; ++dd) {
      twoff[dd] = acc;
      if (dd >= 1 && dd < nd) {
        const int bd = d.b[dd];
        if (tid < bd) tws[acc + tid] = p.tw[d.tw_off[dd] + tid];
        acc += bd;
      }
    }
  }
  const int e0 = int(blockIdx.x) * E;
  const float2* part = p.part + d.part_off + rel * d.part_stride + int64_t(s) * B + e0;
  const int nch = d.nchunks;
  for (int e = tid; e < E; e += kSplitThreads) {
    float2 v = part[e];
    for (int c = 1; c < nch; ++c) {
      const float2 w = part[int64_t(c) * T * B + e];
      v.x += w.x;
      v.y += w.y;
    }
    re[lds_at(e, nls)] = v.x;
    im[lds_at(e, nls)] = v.y;
  }
  __syncthreads();
  for (int dd = 1; dd < nd; ++dd) {
    const int n = d.b[dd];
    if (n == 1) continue;                       // a 1-point DFT is the identity
    if (n >= 16)
      mode_product_r16<kSplitWaves>(re, im, tws + twoff[dd], n, d.bshift[dd], E / n, nls);
    else
      mode_product<kSplitWaves>(re, im, tws + twoff[dd], n, d.bshift[dd], E / n, nls);
  }
  float2* out = inter + d.bucket_off + rel * d.bucket_stride + int64_t(s) * B + e0;
  for (int e = tid; e < E; e += kSplitThreads) out[e] = make_float2(re[lds_at(e, nls)], im[lds_at(e, nls)]);
}

// TH2 threads: 1024 for B_0 >= 64 (the column group's B_0-point DFTs keep
// sixteen waves busy), else 256.
template <int TH2>
__global__ __launch_bounds__(TH2) void dft_pass2_kernel(DevPtrs p, int T, const float2* __restrict__ inter,
                                                        const int32_t* __restrict__ order) {
  constexpr int kSplit2Threads = TH2;
  constexpr int kSplit2Waves = TH2 / 64;
  extern __shared__ float smem[];
  const int64_t f = split_frame(order, blockIdx.z);
  const int s = blockIdx.y;
  const FrameDesc& d = desc_of(p, f);
  const int nd = d.ndim, B = d.B, b0 = d.b[0];
  const int S = B / b0;
  const int C = S < 32 ? S : 32;
  if (int(blockIdx.x) >= S / C) return;
  const int c0 = int(blockIdx.x) * C;
  const int cs = __builtin_ctz(uint32_t(C));
  const int E = b0 * C;
  const int plane = E + (E >> cs);
  float* re = smem;
  float* im = smem + plane;
  float2* tws = reinterpret_cast<float2*>(smem + 2 * plane);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t rel = rel_of(p, f);
  if (tid < b0) tws[tid] = p.tw[d.tw_off[0] + tid];
  const float2* src = inter + d.bucket_off + rel * d.bucket_stride + int64_t(s) * B;
  for (int e = tid; e < E; e += kSplit2Threads) {
    const int k0 = e >> cs;
    const int jp = c0 + (e & (C - 1));         // trailing output position J'
    int kp = 0;                                 // its transform column K'
    for (int dd = 1; dd < nd; ++dd) {
      const int bd = d.b[dd];
      const int jd = (jp >> d.bshift[dd]) & (bd - 1);
      kp |= ((d.tau[s][dd] * jd) & (bd - 1)) << d.bshift[dd];
    }
    const float2 v = src[int64_t(k0) * S + kp];
    re[lds_at(e, cs)] = v.x;
    im[lds_at(e, cs)] = v.y;
  }
  __syncthreads();
  if (b0 >= 16)
    mode_product_r16<kSplit2Waves>(re, im, tws, b0, cs, C, cs);
  else
    mode_product<kSplit2Waves>(re, im, tws, b0, cs, C, cs);
  const int64_t fb = d.bucket_off + rel * d.bucket_stride + int64_t(s) * B;
  float2* bout = p.buckets + fb;
  float* pout = p.powers + fb;
  uint32_t* fout = p.flags + d.flag_off + rel * d.flag_stride + int64_t(s) * d.words;
  const double gamma = d.gamma[s];
  const int t0 = d.tau[s][0];
  for (int e00 = wave * 64; e00 < E; e00 += kSplit2Threads) {
    const int e = e00 + lane;
    bool flag = false;
    int j = 0;
    if (e < E) {
      const int j0 = e >> cs;
      const int c = e & (C - 1);
      const int k0 = (t0 * j0) & (b0 - 1);
      const int at = lds_at((k0 << cs) | c, cs);
      const float xr = re[at], xi = im[at];
      const float pw = xr * xr + xi * xi;
      j = j0 * S + c0 + c;
      bout[j] = make_float2(xr, xi);
      pout[j] = pw;
      flag = double(pw) >= gamma;
    }
    const unsigned long long m = __ballot(flag);
    // lanes 0..31 and 32..63 each cover 32 consecutive output buckets
    // starting at a multiple of 32 (C = 32: one output row each; C = S:
    // the transform in output order)
    const int ja = __shfl(j, 0);
    const int jb = __shfl(j, 32);
    if (lane == 0) fout[ja >> 5] = uint32_t(m & 0xffffffffull);
    if (lane == 32 && e < E) fout[jb >> 5] = uint32_t(m >> 32);
  }
}

int launch_dft_split(const DevPtrs& p, int64_t nframes, int T, int max_b0, int max_groups1, int max_groups2,
                     int max_e1, int sum_tw, float2* inter, const int32_t* order, void* stream) {
  if (nframes <= 0) return hipSuccess;
  if (nframes > 65535 || T > 65535 || max_e1 > kSplitMaxSlab) return hipErrorInvalidValue;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // two planes of at most 2 E floats (E buckets plus at most one pad each)
  const size_t sh1 = size_t(4 * max_e1) * sizeof(float) + size_t(sum_tw) * sizeof(float2);
  hipLaunchKernelGGL(dft_pass1_kernel, dim3(unsigned(max_groups1), unsigned(T), unsigned(nframes)),
                     dim3(kSplitThreads), sh1, st, p, T, inter, order);
  const size_t sh2 = size_t(2 * (max_b0 * 32 + max_b0)) * sizeof(float) + size_t(max_b0) * sizeof(float2);
  const dim3 grid2{unsigned(max_groups2), unsigned(T), unsigned(nframes)};
  if (max_b0 >= 64)
    hipLaunchKernelGGL(dft_pass2_kernel<1024>, grid2, dim3(1024), sh2, st, p, T, static_cast<const float2*>(inter), order);
  else
    hipLaunchKernelGGL(dft_pass2_kernel<256>, grid2, dim3(256), sh2, st, p, T, static_cast<const float2*>(inter), order);
  return hipGetLastError();
}

int launch_dft(const DevPtrs& p, int64_t nframes, int T, int plane, int pad, int sum_tw, int identity,
               int nchunks_override, const int32_t* order, int threads, void* stream) {
  if (nframes <= 0) return hipSuccess;
  const size_t shmem = size_t(2 * plane) * sizeof(float) + size_t(sum_tw) * sizeof(float2);
  const dim3 grid{unsigned(T), unsigned(nframes), 1u};
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (threads) {
    case 64: hipLaunchKernelGGL(dft_kernel<64>, grid, dim3(64), shmem, st, p, T, plane, pad, 0, identity, nchunks_override, order); break;
    case 256: hipLaunchKernelGGL(dft_kernel<256>, grid, dim3(256), shmem, st, p, T, plane, pad, 0, identity, nchunks_override, order); break;
    case 1024: hipLaunchKernelGGL(dft_kernel<1024>, grid, dim3(1024), shmem, st, p, T, plane, pad, 0, identity, nchunks_override, order); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static int launch_dft_frame(const DevPtrs& p, int64_t frame, int T, int plane, int pad, int sum_tw,
                            hipStream_t st) {
  const size_t shmem = size_t(2 * plane) * sizeof(float) + size_t(sum_tw) * sizeof(float2);
  hipLaunchKernelGGL(dft_kernel<1024>, dim3(unsigned(T), 1u), dim3(1024), shmem, st, p, T, plane,
                     pad, int(frame), 1, 1, static_cast<const int32_t*>(nullptr));
  return hipGetLastError();
}

int launch_plain_dft(const DevPtrs& p, int64_t frame, int T, int plane, int pad, int sum_tw,
                     void* stream) {
  return launch_dft_frame(p, frame, T, plane, pad, sum_tw, static_cast<hipStream_t>(stream));
}

}  // namespace rsft

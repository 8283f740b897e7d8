// vote and scan stages of the RSFT hot path.

#include "device_common.h"

namespace rsft {

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

// Stage n flag words from global memory into LDS, up to four per thread
// loaded before any is stored (one memory round trip per 4 * kVoteThreads).
__device__ __forceinline__ void stage_flags(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                            int n) {
  constexpr int kPer = 4;
  for (int w0 = 0; w0 < n; w0 += kPer * kVoteThreads) {
    uint32_t v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int w = w0 + k * kVoteThreads + int(threadIdx.x);
      v[k] = w < n ? src[w] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int w = w0 + k * kVoteThreads + int(threadIdx.x);
      if (w < n) dst[w] = v[k];
    }
  }
}

template <int D>
__global__ __launch_bounds__(kVoteThreads) void vote_kernel(DevPtrs p, int T, int mu, int frame0, int use_list) {
  extern __shared__ uint32_t sflags[];
  __shared__ uint32_t wcount[kVoteThreads / 64];
  __shared__ uint32_t ssig[kMaxRounds * kMaxDims];
  int64_t f = frame0 + int64_t(blockIdx.y);
  int c = blockIdx.x;
  if (use_list && !listed_chunk(p, blockIdx.x, f, c)) return;
  const FrameDesc& d = desc_of(p, f);
  const int cch = d.cchunks, nd = d.ndim;   // loaded together, then tested
  if ((c >= cch) | (nd != D)) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int words = d.words;
  const uint32_t* fl = p.flags + d.flag_off + rel * d.flag_stride;
  stage_flags(sflags, fl, T * words);
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

// vote_mask_kernel (rows of exactly 32 cells, any T): a row's 32 cells
// share their bucket in every dimension but the last, so in round s the
// bucket of cell x of the row is rowpart_s | b_s(x) with b_s(x) =
// [sigma_{s,last} x]_32 >> log2 L_last (Def. 3). With M_s[b] the 32-bit mask
// of the cells x whose b_s(x) = b, the round's votes for the whole row are
// the OR of M_s[b] over the flagged buckets b of the row's B_last-bit flag
// window (B_last <= 16, so the window never straddles a word). A bit-sliced
// counter of NB bits adds the T masks and a bit-sliced comparison with mu
// gives the row's bitmap word: the same bits as the per-cell sum of eq. a_i,
// at a few instructions per cell. One thread per row.
template <int D, int NB>
__global__ __launch_bounds__(kVoteThreads) void vote_mask_kernel(DevPtrs p, int T, int mu, int frame0,
                                                                int use_list) {
  extern __shared__ uint32_t sflags[];
  __shared__ uint32_t wcount[kVoteThreads / 64];
  __shared__ uint32_t smask[kMaxRounds * 16];   // M_s[b], b < B_last <= 16
  __shared__ uint32_t ssig[kMaxRounds * kMaxDims];
  int64_t f = frame0 + int64_t(blockIdx.y);
  int c = blockIdx.x;
  if (use_list && !listed_chunk(p, blockIdx.x, f, c)) return;
  const FrameDesc& d = desc_of(p, f);
  const int cch = d.cchunks, nd = d.ndim;   // loaded together, then tested
  if ((c >= cch) | (nd != D)) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int words = d.words;
  const uint32_t bl = uint32_t(d.b_last);
  const uint32_t lsl = uint32_t(d.lshift[D - 1]);
  stage_flags(sflags, p.flags + d.flag_off + rel * d.flag_stride, T * words);
  if (tid < T * D) ssig[tid] = uint32_t(d.sigma[tid / D][tid % D]);
  for (int k = tid; k < T * 16; k += kVoteThreads) {
    const int s = k >> 4;
    const uint32_t b = uint32_t(k & 15);
    const uint32_t sg = uint32_t(d.sigma[s][D - 1]);
    uint32_t m = 0u;
    for (uint32_t x = 0; x < 32u; ++x) m |= uint32_t((((sg * x) & 31u) >> lsl) == b) << x;
    smask[k] = m;
  }
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
  const int nrows = int(rem < (int64_t(1) << kCompactShift) ? rem : (int64_t(1) << kCompactShift)) >> 5;
  uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride + (cell0 >> 5);
  const uint32_t wmask = bl >= 32u ? ~0u : (1u << bl) - 1u;
  __syncthreads();

  uint32_t cnt = 0u;
  for (int r = tid; r < nrows; r += kVoteThreads) {
    const int64_t iw = cell0 + (int64_t(r) << 5);   // first cell of the row
    uint32_t acc[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = 0u;
    for (int s = 0; s < T; ++s) {
      uint32_t rowpart = 0u;
#pragma unroll
      for (int dd = 0; dd < D - 1; ++dd) {
        const uint32_t cd = uint32_t(iw >> ns[dd]) & nm[dd];
        rowpart |= (((ssig[s * D + dd] * cd) & nm[dd]) >> ls[dd]) << bs[dd];
      }
      uint32_t win = (sflags[s * words + int(rowpart >> 5)] >> (rowpart & 31u)) & wmask;
      uint32_t m = 0u;
      while (win) {
        const int b = __ffs(win) - 1;
        win &= win - 1u;
        m |= smask[s * 16 + b];
      }
      // acc += m, bit-sliced
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const uint32_t t = acc[k] & m;
        acc[k] ^= m;
        m = t;
      }
    }
    // acc >= mu, bit-sliced, most significant bit first
    uint32_t ge = 0u, eq = ~0u;
#pragma unroll
    for (int k = NB - 1; k >= 0; --k) {
      const uint32_t mk = ((uint32_t(mu) >> k) & 1u) ? ~0u : 0u;
      ge |= eq & acc[k] & ~mk;
      eq &= ~(acc[k] ^ mk);
    }
    const uint32_t hit = ge | eq;
    bm[r] = hit;
    cnt += uint32_t(__popc(hit));
  }
  // work-group total of the chunk
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
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
__global__ __launch_bounds__(kVoteThreads) void vote_rows_kernel(DevPtrs p, int mu, int frame0, int use_list) {
  extern __shared__ uint32_t sflags[];
  __shared__ uint32_t wcount[kVoteThreads / 64];
  __shared__ uint32_t rowbm[kVoteThreads / 64][kRowWordsMax];
  __shared__ uint32_t blist[kVoteThreads / 64][128];
  __shared__ uint32_t rowflags[kVoteThreads / 64][TT * 4];
  int64_t f = frame0 + int64_t(blockIdx.y);
  int c = blockIdx.x;
  if (use_list && !listed_chunk(p, blockIdx.x, f, c)) return;
  const FrameDesc& d = desc_of(p, f);
  const int cch = d.cchunks, nd = d.ndim;   // loaded together, then tested
  if ((c >= cch) | (nd != D)) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int words = d.words;
  const uint32_t* fl = p.flags + d.flag_off + rel * d.flag_stride;
  stage_flags(sflags, fl, TT * words);
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

// vote_words_kernel (rows of 128..4096 cells, any T): the word-parallel
// form of the 32-cell mask vote. A row of N_last cells is W = N_last / 32
// words. Cell x of the row lands in bucket column b_s(x) = [sigma_{s,last}
// x]_{N_last} >> log2 L_last in round s (Def. 3), and the cells of column b
// are the L_last preimages x = [sigma_inv u] for u in [b L, (b+1) L)
// (Def. 4). The plan holds per descriptor the tables M_s[b][w] (bit x of
// word w set when cell 32 w + x lies in column b). The leading coordinates
// of a row fix its bucket row r_s (the leading bucket indices) and the
// column part of the mapping does not depend on them, so every row that
// maps to bucket row r in round s has the same round-s mask
//   E_s[r][w] = OR over the flagged columns b of bucket row r of M_s[b][w].
// There are B / B_last bucket rows against N / N_last cell rows (L_d times
// fewer per leading dimension), so the masks are built once per (frame,
// round) by vote_expand_kernel, and vote_words_kernel reads, for the 128
// cells (four words) a thread owns in each of its kVoteCpw chunks, the T
// masks E_s[r_s(row)] and combines them by a bit-sliced counter of NB bits
// compared with mu (NB = 0: mu = T, a plain AND): the same bits as the
// per-cell sum of eq. a_i. One work-group per group of kVoteCpw consecutive
// compaction chunks of a frame; each thread writes its four bitmap words per
// chunk with one store.
constexpr int kWordsPerVoteThread = 4;
static_assert(kVoteExpWords == kVoteThreads * kWordsPerVoteThread, "one expand block per work-group");

// Loads of round s's table pieces and flag words of this thread (see
// vote_expand_kernel), all issued before any is used.
template <int kTabPer, int kFlagPer>
__device__ __forceinline__ void vote_prefetch(uint4 (&tnext)[kTabPer], uint32_t (&fnext)[kFlagPer],
                                              const uint32_t* gtab, const uint32_t* fl, int s, uint32_t ntab,
                                              uint32_t npiece, int words) {
  const uint4* src = reinterpret_cast<const uint4*>(gtab + int64_t(s) * ntab);
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kTabPer; ++k) {
    const uint32_t i = uint32_t(tid) + uint32_t(k) * kVoteThreads;
    tnext[k] = i < npiece ? src[i] : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < kFlagPer; ++k) {
    const int i = tid + k * kVoteThreads;
    fnext[k] = i < words ? fl[int64_t(s) * words + i] : 0u;
  }
}

// One work-group per (block of kVoteExpWords mask words, round, frame), or
// per (vote_exp_list entry, round): the round's table M_s and flag words in
// LDS, then each thread ORs, for its four words of one bucket row, the table
// rows of that bucket row's flagged columns (one 16-byte LDS read per
// flagged bucket).
template <int kTabPer>
__global__ __launch_bounds__(kVoteThreads) void vote_expand_kernel(DevPtrs p, int frame0, int tab_words,
                                                                   int use_list) {
  extern __shared__ uint32_t smem[];
  uint32_t* tab = smem;                       // [B_last][W] words of the round
  uint32_t* rflags = smem + tab_words;        // the round's flag words
  int64_t f;
  uint32_t blk;
  if (use_list) {
    const int32_t* e = p.vote_exp_list + 2 * int64_t(blockIdx.x);
    f = e[0];
    blk = uint32_t(e[1]);
  } else {
    f = frame0 + int64_t(blockIdx.z);
    blk = blockIdx.x;
  }
  const int s = int(blockIdx.y);
  const FrameDesc& d = desc_of(p, f);
  const int D = d.ndim;
  const uint32_t nl = uint32_t(d.n[D - 1]);
  const uint32_t bl = uint32_t(d.b[D - 1]);
  const uint32_t W = nl >> 5;
  const uint32_t total = (uint32_t(d.B) / bl) * W;          // mask words of the round
  const uint32_t blk0 = blk * uint32_t(kVoteExpWords);
  if (blk0 >= total || s >= d.T) return;
  const int64_t rel = rel_of(p, f);
  const int words = d.words;
  const uint32_t ntab = bl * W;
  const uint32_t npiece = ntab >> 2;
  constexpr int kFlagPer = kMaxBuckets / 32 / kVoteThreads;
  uint4 tv[kTabPer];
  uint32_t fv[kFlagPer];
  vote_prefetch<kTabPer, kFlagPer>(tv, fv, p.vote_tab + d.vtab_off, p.flags + d.flag_off + rel * d.flag_stride, s,
                                   ntab, npiece, words);
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kTabPer; ++k) {
    const uint32_t i = uint32_t(tid) + uint32_t(k) * kVoteThreads;
    if (i < npiece) reinterpret_cast<uint4*>(tab)[i] = tv[k];
  }
#pragma unroll
  for (int k = 0; k < kFlagPer; ++k) {
    const int i = tid + k * kVoteThreads;
    if (i < words) rflags[i] = fv[k];
  }
  __syncthreads();
  const uint32_t q = blk0 + uint32_t(tid) * uint32_t(kWordsPerVoteThread);
  if (q >= total) return;
  const uint32_t w0 = q & (W - 1u);                          // W >= 4, a power of two
  const uint32_t rowpart = (q / W) * bl;                     // first bucket of the bucket row
  uint32_t m0 = 0u, m1 = 0u, m2 = 0u, m3 = 0u;
  // the bucket row's B_last flags: whole words when B_last >= 32, else a
  // field (rowpart is a multiple of B_last: the window never straddles)
  const int nw = bl >= 32u ? int(bl >> 5) : 1;
  for (int kw = 0; kw < nw; ++kw) {
    uint32_t win = rflags[(rowpart >> 5) + uint32_t(kw)];
    if (bl < 32u) win = (win >> (rowpart & 31u)) & ((1u << bl) - 1u);
    while (win) {
      const uint32_t b = uint32_t(kw) * 32u + uint32_t(__ffs(win) - 1);
      win &= win - 1u;
      const uint4 v = *reinterpret_cast<const uint4*>(tab + b * W + w0);
      m0 |= v.x;
      m1 |= v.y;
      m2 |= v.z;
      m3 |= v.w;
    }
  }
  uint32_t* e = p.vote_exp + d.vexp_off + rel * d.vexp_stride + int64_t(s) * total + q;
  *reinterpret_cast<uint4*>(e) = make_uint4(m0, m1, m2, m3);
}

template <int D, int NB>
__global__ __launch_bounds__(kVoteThreads) void vote_words_kernel(DevPtrs p, int T, int mu, int frame0,
                                                                 int use_list) {
  __shared__ uint32_t wcount[kVoteCpw][kVoteThreads / 64];
  constexpr int kW = kWordsPerVoteThread;
  constexpr int kAcc = NB > 0 ? NB : 1;
  int64_t f;
  int c0;
  if (use_list) {
    const int32_t* e = p.vote_list + 2 * int64_t(blockIdx.x);
    f = e[0];
    c0 = e[1];
    if (f < 0) return;
  } else {
    f = frame0 + int64_t(blockIdx.y);
    c0 = int(blockIdx.x) * kVoteCpw;
  }
  const FrameDesc& d = desc_of(p, f);
  const int cch = d.cchunks, nd = d.ndim;   // loaded together, then tested
  if ((c0 >= cch) | (nd != D)) return;
  const int64_t rel = rel_of(p, f);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  uint32_t nm[D], ls[D], bs[D], ns[D];
#pragma unroll
  for (int dd = 0; dd < D; ++dd) {
    nm[dd] = uint32_t(d.n[dd] - 1);
    ls[dd] = uint32_t(d.lshift[dd]);
    bs[dd] = uint32_t(d.bshift[dd]);
    ns[dd] = uint32_t(d.nshift[dd]);
  }
  const uint32_t nl = nm[D - 1] + 1u;
  const uint32_t bl = uint32_t(d.b[D - 1]);
  const uint32_t lbl = uint32_t(__builtin_ctz(bl));
  const uint32_t W = nl >> 5;
  const uint32_t ew = (uint32_t(d.B) >> lbl) * W;            // mask words per round
  const uint32_t* E = p.vote_exp + d.vexp_off + rel * d.vexp_stride;
  const int q0 = tid * kW;                                  // first word of this thread in a chunk
  const uint32_t w0 = uint32_t(q0) & (W - 1u);              // their word offset in the row (W >= 4)
  bool active[kVoteCpw];
  int64_t iw[kVoteCpw];                                     // first cell of those words
#pragma unroll
  for (int k = 0; k < kVoteCpw; ++k) {
    const int64_t cell0 = int64_t(c0 + k) << kCompactShift;
    const int64_t rem = d.N - cell0;
    const int ncell = rem <= 0 ? 0 : int(rem < (int64_t(1) << kCompactShift) ? rem : (int64_t(1) << kCompactShift));
    active[k] = c0 + k < cch && q0 < (ncell >> 5);
    iw[k] = cell0 + (int64_t(q0) << 5);
  }
  uint32_t acc[kAcc][kVoteCpw * kW];
#pragma unroll
  for (int a = 0; a < kAcc; ++a)
#pragma unroll
    for (int q = 0; q < kVoteCpw * kW; ++q) acc[a][q] = NB > 0 ? 0u : ~0u;

  for (int s = 0; s < T; ++s) {
    // the round's mask words of the rows of all chunks, loaded before use
    uint4 v[kVoteCpw];
#pragma unroll
    for (int k = 0; k < kVoteCpw; ++k) {
      v[k] = make_uint4(0u, 0u, 0u, 0u);
      if (active[k]) {
        uint32_t rowpart = 0u;
#pragma unroll
        for (int dd = 0; dd < D - 1; ++dd) {
          const uint32_t cd = uint32_t(iw[k] >> ns[dd]) & nm[dd];
          rowpart |= (((uint32_t(d.sigma[s][dd]) * cd) & nm[dd]) >> ls[dd]) << bs[dd];
        }
        v[k] = *reinterpret_cast<const uint4*>(E + int64_t(s) * ew + (rowpart >> lbl) * W + w0);
      }
    }
#pragma unroll
    for (int k = 0; k < kVoteCpw; ++k) {
      const uint32_t m[kW] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        if constexpr (NB == 0) {
          acc[0][k * kW + q] &= m[q];
        } else {
          uint32_t carry = m[q];
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            const uint32_t t = acc[a][k * kW + q] & carry;
            acc[a][k * kW + q] ^= carry;
            carry = t;
          }
        }
      }
    }
  }
  uint32_t* bm = p.bitmap + d.bitmap_off + rel * d.bitmap_stride;
#pragma unroll
  for (int k = 0; k < kVoteCpw; ++k) {
    uint32_t hit[kW];
#pragma unroll
    for (int q = 0; q < kW; ++q) {
      if constexpr (NB == 0) {
        hit[q] = acc[0][k * kW + q];
      } else {
        // acc >= mu, bit-sliced, most significant bit first
        uint32_t ge = 0u, eq = ~0u;
#pragma unroll
        for (int a = NB - 1; a >= 0; --a) {
          const uint32_t mk = ((uint32_t(mu) >> a) & 1u) ? ~0u : 0u;
          ge |= eq & acc[a][k * kW + q] & ~mk;
          eq &= ~(acc[a][k * kW + q] ^ mk);
        }
        hit[q] = ge | eq;
      }
    }
    uint32_t cnt = 0u;
    if (active[k]) {
      *reinterpret_cast<uint4*>(bm + (iw[k] >> 5)) = make_uint4(hit[0], hit[1], hit[2], hit[3]);
      cnt = uint32_t(__popc(hit[0]) + __popc(hit[1]) + __popc(hit[2]) + __popc(hit[3]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) wcount[k][wave] = cnt;
  }
  __syncthreads();
  if (tid < kVoteCpw && c0 + tid < cch) {
    uint32_t total = 0u;
    for (int w = 0; w < kVoteThreads / 64; ++w) total += wcount[tid][w];
    p.chunk_counts[d.chunk_off + rel * d.chunk_stride + c0 + tid] = total;
  }
}

// counters of NB bits hold counts up to T; NB = 0: mu = T (a plain AND)
template <int D>
static void launch_vote_words(dim3 grid, hipStream_t st, const DevPtrs& p, int T, int mu, int frame0,
                              int use_list) {
  if (mu == T) hipLaunchKernelGGL((vote_words_kernel<D, 0>), grid, dim3(kVoteThreads), 0, st, p, T, mu, frame0, use_list);
  else if (T <= 3) hipLaunchKernelGGL((vote_words_kernel<D, 2>), grid, dim3(kVoteThreads), 0, st, p, T, mu, frame0, use_list);
  else if (T <= 7) hipLaunchKernelGGL((vote_words_kernel<D, 3>), grid, dim3(kVoteThreads), 0, st, p, T, mu, frame0, use_list);
  else hipLaunchKernelGGL((vote_words_kernel<D, 7>), grid, dim3(kVoteThreads), 0, st, p, T, mu, frame0, use_list);
}

template <int D>
static void launch_vote_d(const DevPtrs& p, dim3 grid, size_t shmem, hipStream_t st, int T, int mu,
                          int frame0, int use_list, bool rows, bool masks, bool wordsp) {
  if (wordsp) {
    launch_vote_words<D>(grid, st, p, T, mu, frame0, use_list);
    return;
  }
  if (masks) {   // counters of NB bits hold counts up to T
    if (T <= 3) hipLaunchKernelGGL((vote_mask_kernel<D, 2>), grid, dim3(kVoteThreads), shmem, st, p, T, mu, frame0, use_list);
    else if (T <= 7) hipLaunchKernelGGL((vote_mask_kernel<D, 3>), grid, dim3(kVoteThreads), shmem, st, p, T, mu, frame0, use_list);
    else hipLaunchKernelGGL((vote_mask_kernel<D, 7>), grid, dim3(kVoteThreads), shmem, st, p, T, mu, frame0, use_list);
    return;
  }
  if (rows) {
    switch (T) {
      case 1: hipLaunchKernelGGL((vote_rows_kernel<D, 1>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0, use_list); return;
      case 2: hipLaunchKernelGGL((vote_rows_kernel<D, 2>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0, use_list); return;
      case 3: hipLaunchKernelGGL((vote_rows_kernel<D, 3>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0, use_list); return;
      case 4: hipLaunchKernelGGL((vote_rows_kernel<D, 4>), grid, dim3(kVoteThreads), shmem, st, p, mu, frame0, use_list); return;
      default: break;
    }
  }
  hipLaunchKernelGGL(vote_kernel<D>, grid, dim3(kVoteThreads), shmem, st, p, T, mu, frame0, use_list);
}

int launch_vote(const DevPtrs& p, int64_t nframes, int T, int mu, int max_cchunks, int max_words,
                int dims_mask, int vote_path, int frame0, int64_t nlist, int64_t nvlist, int tab_words,
                int exp_blocks, int64_t nexp_list, void* stream) {
  if (nframes <= 0) return hipSuccess;
  const bool wordsp = vote_path == kVoteWords;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (wordsp) {
    // bucket-row masks of every (frame, round): the round's table and flags
    // in LDS (kTabPer 16-byte table pieces per thread cover the plan's largest)
    const int el = nexp_list > 0 ? 1 : 0;
    if (nframes > 65535 || T > 65535 || exp_blocks <= 0 || (el && (frame0 != 0 || nexp_list >= (int64_t(1) << 31))))
      return hipErrorInvalidValue;
    const dim3 eg = el ? dim3{unsigned(nexp_list), unsigned(T), 1u}
                       : dim3{unsigned(exp_blocks), unsigned(T), unsigned(nframes)};
    const size_t esh = (size_t(tab_words) + size_t(max_words)) * sizeof(uint32_t);
    if (tab_words <= 4 * 2 * kVoteThreads)
      hipLaunchKernelGGL(vote_expand_kernel<2>, eg, dim3(kVoteThreads), esh, st, p, frame0, tab_words, el);
    else if (tab_words <= 4 * 8 * kVoteThreads)
      hipLaunchKernelGGL(vote_expand_kernel<8>, eg, dim3(kVoteThreads), esh, st, p, frame0, tab_words, el);
    else if (tab_words <= 4 * 16 * kVoteThreads)
      hipLaunchKernelGGL(vote_expand_kernel<16>, eg, dim3(kVoteThreads), esh, st, p, frame0, tab_words, el);
    else
      return hipErrorInvalidValue;
  }
  // the other paths stage all rounds' flags
  const size_t shmem = wordsp ? 0 : size_t(T) * size_t(max_words) * sizeof(uint32_t);
  // the word-parallel vote takes its own list of chunk groups
  const int64_t list_len = wordsp ? nvlist : nlist;
  const int use_list = list_len > 0 ? 1 : 0;
  if (use_list && (frame0 != 0 || list_len >= (int64_t(1) << 31))) return hipErrorInvalidValue;
  const int gx = wordsp ? (max_cchunks + kVoteCpw - 1) / kVoteCpw : max_cchunks;
  const dim3 grid = use_list ? dim3{unsigned(list_len), 1u, 1u} : dim3{unsigned(gx), unsigned(nframes), 1u};
  const bool rows = vote_path == kVoteRows && T <= 4;
  const bool masks = vote_path == kVoteMasks32;
  if (dims_mask & 1) launch_vote_d<1>(p, grid, shmem, st, T, mu, frame0, use_list, rows, masks, wordsp);
  if (dims_mask & 2) launch_vote_d<2>(p, grid, shmem, st, T, mu, frame0, use_list, rows, masks, wordsp);
  if (dims_mask & 4) launch_vote_d<3>(p, grid, shmem, st, T, mu, frame0, use_list, rows, masks, wordsp);
  if (dims_mask & 8) launch_vote_d<4>(p, grid, shmem, st, T, mu, frame0, use_list, rows, masks, wordsp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scan: one work-group per frame (or, in uniform plans of at most 128 chunks
// per frame, per kScanThreads / chunks frames in one segmented block scan)
// turns the frame's chunk counters into
// chunk_offsets (rank of each compaction chunk's first detection in its
// frame, a running sum in row-major cell order) and counts[f]. For plans
// with overflow workers it also lists their work: the records of a chunk
// beyond its first
// kChunkRecords that fit the frame's capacity form ceil(over / 2^kItemShift)
// items; chunk_items holds the running sum of items over the frame's chunks,
// item_counts[f] the frame's total. The last work-group to finish (a
// device-scope counter, released and acquired with fences) computes
// offsets[f] = sum_{g<f} min(count_g, cap_g) and item_offsets[f] =
// sum_{g<f} item_counts[g] (entry nframes holds the totals), and resets the
// counter for the next launch.
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

__global__ __launch_bounds__(kScanThreads) void scan_kernel(DevPtrs p, int64_t nframes, int items, int fpb) {
  __shared__ int64_t wtot[kScanThreads / 64];
  __shared__ int64_t sinc[kScanThreads];     // block-wide inclusive sums (fpb > 1)
  __shared__ int64_t ftot[kScanThreads];     // records of each of the block's frames
  __shared__ int64_t fitm[kScanThreads];     // overflow items of each of the block's frames
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int64_t f0 = int64_t(blockIdx.x) * fpb;
  if (fpb == 1) {
    // one frame, its chunks kScanThreads at a time
    const int64_t f = f0;
    const FrameDesc& d = desc_of(p, f);
    const int64_t rel = rel_of(p, f);
    const int64_t base = d.chunk_off + rel * d.chunk_stride;
    const int64_t cap = d.cap;
    int64_t run = 0, irun = 0;
    for (int c0 = 0; c0 < d.cchunks; c0 += kScanThreads) {
      const int c = c0 + tid;
      const int64_t v = c < d.cchunks ? int64_t(p.chunk_counts[base + c]) : 0;
      int64_t total;
      const int64_t incl = block_inclusive_scan(v, wtot, total);
      const int64_t off = run + incl - v;
      int64_t fit = cap - off;                   // the chunk's records that get a record slot
      fit = fit < 0 ? 0 : (fit > v ? v : fit);
      if (c < d.cchunks) p.chunk_offsets[base + c] = off;
      run += total;
      if (items) {                               // uniform
        const int64_t over = fit > kChunkRecords ? fit - kChunkRecords : 0;
        const int64_t it = (over + (int64_t(1) << kItemShift) - 1) >> kItemShift;
        int64_t itotal;
        const int64_t iincl = block_inclusive_scan(it, wtot, itotal);
        if (c < d.cchunks) p.chunk_items[base + c] = irun + iincl - it;
        irun += itotal;
      }
    }
    if (tid == 0) {
      ftot[0] = run;
      fitm[0] = irun;
    }
  } else {
    // a uniform plan of cch = kScanThreads / fpb chunks per frame: fpb frames
    // in one segmented scan (thread t: frame t / cch, chunk t mod cch)
    const FrameDesc& d = p.descs[0];
    const int cch = kScanThreads / fpb;
    const int fi = tid / cch;
    const int c = tid - fi * cch;
    const int64_t f = f0 + fi;
    const bool valid = f < nframes;
    const int64_t base = d.chunk_off + f * d.chunk_stride;
    const int64_t cap = d.cap;
    const int s0 = fi * cch;                     // the frame's first thread
    const int64_t v = valid ? int64_t(p.chunk_counts[base + c]) : 0;
    int64_t total;
    const int64_t incl = block_inclusive_scan(v, wtot, total);
    sinc[tid] = incl;
    __syncthreads();
    const int64_t segb = s0 == 0 ? 0 : sinc[s0 - 1];
    const int64_t off = incl - v - segb;
    int64_t fit = cap - off;
    fit = fit < 0 ? 0 : (fit > v ? v : fit);
    if (valid) p.chunk_offsets[base + c] = off;
    if (c == cch - 1) ftot[fi] = incl - segb;
    if (items) {                                 // uniform
      const int64_t over = fit > kChunkRecords ? fit - kChunkRecords : 0;
      const int64_t it = (over + (int64_t(1) << kItemShift) - 1) >> kItemShift;
      int64_t itotal;
      const int64_t iincl = block_inclusive_scan(it, wtot, itotal);   // its barriers end the reads of sinc
      sinc[tid] = iincl;
      __syncthreads();
      const int64_t isegb = s0 == 0 ? 0 : sinc[s0 - 1];
      if (valid) p.chunk_items[base + c] = iincl - it - isegb;
      if (c == cch - 1) fitm[fi] = iincl - isegb;
    } else if (c == cch - 1) {
      fitm[fi] = 0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < fpb && f0 + k < nframes; ++k) {
      p.counts[f0 + k] = ftot[k];
      p.item_counts[f0 + k] = fitm[k];
    }
    __threadfence();
    const unsigned prev = atomicAdd(p.scan_done, 1u);
    is_last = prev == gridDim.x - 1u ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  constexpr int kPer = 8;
  if (nframes <= int64_t(kPer) * kScanThreads) {
    // thread t owns frames t * per .. t * per + per - 1: their totals are
    // loaded together, summed, and one block scan places them
    const int per = int((nframes + kScanThreads - 1) / kScanThreads);
    const int64_t g0 = int64_t(tid) * per;
    int64_t v[kPer], iv[kPer];
    int64_t sum = 0, isum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t g = g0 + k;
      v[k] = iv[k] = 0;
      if (k < per && g < nframes) {
        const int64_t cnt = __atomic_load_n(p.counts + g, __ATOMIC_RELAXED);
        const int64_t gcap = desc_of(p, g).cap;
        v[k] = cnt < gcap ? cnt : gcap;
        if (items) iv[k] = __atomic_load_n(p.item_counts + g, __ATOMIC_RELAXED);
      }
      sum += v[k];
      isum += iv[k];
    }
    int64_t total;
    int64_t run = block_inclusive_scan(sum, wtot, total) - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      run += v[k];
      if (k < per && g0 + k < nframes) p.offsets[g0 + k + 1] = run;
    }
    if (items) {
      int64_t itotal;
      int64_t irun = block_inclusive_scan(isum, wtot, itotal) - isum;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        irun += iv[k];
        if (k < per && g0 + k < nframes) p.item_offsets[g0 + k + 1] = irun;
      }
    }
    if (tid == 0) {
      p.offsets[0] = 0;
      p.item_offsets[0] = 0;
      atomicExch(p.scan_done, 0u);
    }
    return;
  }
  int64_t carry = 0, icarry = 0;
  for (int64_t g0 = 0; g0 < nframes; g0 += kScanThreads) {
    const int64_t g = g0 + tid;
    int64_t v = 0, iv = 0;
    if (g < nframes) {
      const int64_t cnt = __atomic_load_n(p.counts + g, __ATOMIC_RELAXED);
      const int64_t gcap = desc_of(p, g).cap;
      v = cnt < gcap ? cnt : gcap;
      if (items) iv = __atomic_load_n(p.item_counts + g, __ATOMIC_RELAXED);
    }
    int64_t total;
    const int64_t incl = block_inclusive_scan(v, wtot, total);
    if (g < nframes) p.offsets[g + 1] = carry + incl;
    carry += total;
    if (items) {
      int64_t itotal;
      const int64_t iincl = block_inclusive_scan(iv, wtot, itotal);
      if (g < nframes) p.item_offsets[g + 1] = icarry + iincl;
      icarry += itotal;
    }
  }
  if (tid == 0) {
    p.offsets[0] = 0;
    p.item_offsets[0] = 0;
    atomicExch(p.scan_done, 0u);
  }
}

int launch_scan(const DevPtrs& p, int64_t nframes, int items, int fpb, void* stream) {
  if (nframes <= 0) return hipSuccess;
  if (nframes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  if (fpb < 1 || fpb > kScanThreads || kScanThreads % fpb != 0) return hipErrorInvalidValue;
  const int64_t blocks = (nframes + fpb - 1) / fpb;
  hipLaunchKernelGGL(scan_kernel, dim3(unsigned(blocks)), dim3(kScanThreads), 0,
                     static_cast<hipStream_t>(stream), p, nframes, items, fpb);
  return hipGetLastError();
}

}  // namespace rsft

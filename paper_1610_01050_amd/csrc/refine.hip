// Off-grid refinement on gfx950: the bucketized forward model of K complex
// tones per frame and its gradients.
//
// The round-s buckets (eq. f) are linear in the signal and separable per
// dimension. For a tone r[m] = b exp(j 2 pi f . m) with continuous f
// (cycles/sample; the tone v(omega) of eq. f_k), the flat-window, permuted,
// pre-windowed sequence of dimension d is
//   z_d[n] = wbar_d[n] w_d[m] exp(j 2 pi f_d m),   m = [sigma_{s,d} n]_{N_d},
// (Def. 1, permutation with tau = 0), its aliasing onto B_d points is
// u_d[c] = sum_l z_d[c + l B_d] (Def. 2) and the bucket value is
//   fhat_s[k] = b prod_d G_{s,d}[k_d],  G_{s,d}[k] = sum_c u_d[c] e^{-2 pi i k c / B_d}.
// The model of a frame is model_s[k] = sum_t b_t prod_d G_{s,d,t}[k_d] and
// d/df_d multiplies z_d[n] by j 2 pi m. The phase f_d m is taken modulo 1
// exactly: f_d as a 64-bit fixed-point fraction times the integer m, mod
// 2^64. Sums are FP32, the per-frame frequencies and their gradients FP64.
//
// Kernels
//   model_basis     one work-group per (frame, round, dimension, tone):
//                   G and dG/df of that dimension (aliasing, then DFT)
//   model_combine   model_s[k] for every bucket k
//   model_backward  one work-group per (frame, tone): for the output gradient
//                   Gr = dL/dRe(model) + j dL/dIm(model),
//                     grad b_t   = sum_{s,k} Gr_s[k] conj(prod_d G_d[k_d])
//                     grad f_t,d = Re(b_t sum_{s,k} conj(Gr_s[k]) dG_d[k_d] prod_{e != d} G_e[k_e])
//                   and optionally each tone's Gauss-Newton step for the loss
//                   sum |model - observed|^2 (blocks of (b_t, f_t), tones
//                   decoupled), solved in FP64.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "rsft_internal.h"

namespace rsft {

// Scratch of the model's factors for callers that cannot allocate
// (rsft_model_forward_noalloc): a static device array, one copy per GPU,
// held from module load until the process ends. Host code never uses its
// name as an address: static_scratch() resolves the device address once per
// device, with that device current, and every launch takes that pointer.
static __device__ __align__(256) unsigned char scratch[RSFT_STATIC_SCRATCH_BYTES];

int static_scratch(int device, void** out) {
  constexpr int kMaxScratchDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxScratchDevices] = {};
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

constexpr int kBasisThreads = 256;
constexpr int kCombineThreads = 256;
constexpr int kBackThreads = 256;

__device__ __forceinline__ const FrameDesc& model_desc(const DevPtrs& p, int64_t f) {
  return p.descs[p.uniform ? 0 : f];
}
__device__ __forceinline__ int64_t model_rel(const DevPtrs& p, int64_t f) {
  return p.uniform ? f : 0;
}

// frac(f) as a 64-bit fixed-point fraction (exact: a double has <= 53
// significant bits)
__device__ __forceinline__ uint64_t fixed_fraction(double f) {
  const double fr = f - floor(f);
  const double two64 = 18446744073709551616.0;
  const double scaled = fr * two64;
  if (!(scaled < two64)) return 0ull;   // fr rounded up to 1
  return static_cast<uint64_t>(scaled);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

__global__ __launch_bounds__(kBasisThreads) void model_basis_kernel(
    DevPtrs p, const double* __restrict__ freqs, int K, int D, int T, int sum_b,
    float2* __restrict__ G, float2* __restrict__ dG) {
  __shared__ float2 su[kBasisThreads], sdu[kBasisThreads];
  __shared__ float2 ub[128], dub[128];
  int64_t r = blockIdx.x;
  const int t = int(r % K);
  r /= K;
  const int d = int(r % D);
  r /= D;
  const int s = int(r % T);
  const int64_t f = r / T;
  const FrameDesc& de = model_desc(p, f);
  const int tid = threadIdx.x;
  const uint32_t n = uint32_t(de.n[d]);
  const int bd = de.b[d];
  const int bsh = __builtin_ctz(uint32_t(bd));
  const uint32_t L = n >> bsh;
  const uint32_t sig = uint32_t(de.sigma[s][d]);
  const uint64_t fq = fixed_fraction(freqs[(f * K + t) * D + d]);
  const float* win = p.win + de.win_off[d];
  const float2* flat = p.flat + de.flat_off[d];

  // thread tid sums the alias terms n = c + l B_d of bucket c = tid mod B_d
  // for every (kBasisThreads / B_d)-th l
  const uint32_t c = uint32_t(tid) & uint32_t(bd - 1);
  const uint32_t l0 = uint32_t(tid) >> bsh;
  const uint32_t lstep = uint32_t(kBasisThreads) >> bsh;
  float ur = 0.f, ui = 0.f, dr = 0.f, di = 0.f;
  for (uint32_t l = l0; l < L; l += lstep) {
    const uint32_t nn = c + (l << bsh);
    const uint32_t m = (sig * nn) & (n - 1u);           // products mod 2^32 reduce mod N_d
    const uint64_t ph = fq * uint64_t(m);               // f m mod 1 in 64-bit fixed point
    const float x = float(uint32_t(ph >> 32)) * 2.3283064365386963e-10f;   // / 2^32
    float sn, cs;
    sincospif(2.0f * x, &sn, &cs);
    const float w = win[m];
    const float2 fl = flat[nn];
    const float hr = fl.x * w, hi = fl.y * w;
    const float er = hr * cs - hi * sn;
    const float ei = hr * sn + hi * cs;
    ur += er;
    ui += ei;
    const float tm = 6.283185307179586f * float(m);    // d/df: j 2 pi m
    dr -= tm * ei;
    di += tm * er;
  }
  su[tid] = make_float2(ur, ui);
  sdu[tid] = make_float2(dr, di);
  __syncthreads();
  if (tid < bd) {
    float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
    for (uint32_t j = 0; j < lstep; ++j) {
      const float2 v = su[tid + (j << bsh)];
      const float2 w = sdu[tid + (j << bsh)];
      a.x += v.x;
      a.y += v.y;
      b.x += w.x;
      b.y += w.y;
    }
    ub[tid] = a;
    dub[tid] = b;
  }
  __syncthreads();
  if (tid < bd) {
    const float2* tw = p.tw + de.tw_off[d];
    float2 g = make_float2(0.f, 0.f), dg = make_float2(0.f, 0.f);
    for (int cc = 0; cc < bd; ++cc) {
      const float2 e = tw[(tid * cc) & (bd - 1)];     // exp(-2 pi i k c / B_d)
      const float2 u = ub[cc], du = dub[cc];
      g.x += u.x * e.x - u.y * e.y;
      g.y += u.x * e.y + u.y * e.x;
      dg.x += du.x * e.x - du.y * e.y;
      dg.y += du.x * e.y + du.y * e.x;
    }
    int off = 0;
    for (int e = 0; e < d; ++e) off += de.b[e];
    const int64_t at = ((f * T + s) * K + t) * int64_t(sum_b) + off + tid;
    G[at] = g;
    dG[at] = dg;
  }
}

// Offset of frame f's round-0 buckets in the bucket layout of the plan.
__device__ __forceinline__ int64_t frame_bucket_base(const DevPtrs& p, int64_t f) {
  const FrameDesc& de = model_desc(p, f);
  return de.bucket_off + model_rel(p, f) * de.bucket_stride;
}

// counts (may be NULL): tones of each frame that enter the model (the first
// counts[f]; all K when NULL); observed (may be NULL): write observed - model
// instead of the model
__global__ __launch_bounds__(kCombineThreads) void model_combine_kernel(
    DevPtrs p, const float2* __restrict__ amps, int K, int T, int sum_b,
    const float2* __restrict__ G, float2* __restrict__ model, const int32_t* __restrict__ counts,
    const float2* __restrict__ observed) {
  const int s = blockIdx.y;
  const int64_t f = blockIdx.z;
  const FrameDesc& de = model_desc(p, f);
  const int k = blockIdx.x * kCombineThreads + threadIdx.x;
  if (k >= de.B) return;
  int off[kMaxDims];
  int kd[kMaxDims];
  int acc_off = 0;
  for (int d = 0; d < de.ndim; ++d) {
    off[d] = acc_off + ((k >> de.bshift[d]) & (de.b[d] - 1));
    acc_off += de.b[d];
  }
  (void)kd;
  float2 acc = make_float2(0.f, 0.f);
  const float2* g = G + (f * T + s) * int64_t(K) * sum_b;
  const int kt = counts ? (counts[f] < K ? counts[f] : K) : K;
  for (int t = 0; t < kt; ++t) {
    float2 v = amps[f * K + t];
    for (int d = 0; d < de.ndim; ++d) v = cmul(v, g[int64_t(t) * sum_b + off[d]]);
    acc.x += v.x;
    acc.y += v.y;
  }
  const int64_t at = frame_bucket_base(p, f) + int64_t(s) * de.B + k;
  if (observed) {
    const float2 y = observed[at];
    acc = make_float2(y.x - acc.x, y.y - acc.y);
  }
  model[at] = acc;
}

// sum of v over the work-group (wave shuffles, then one LDS slot per wave);
// every thread receives the total
__device__ __forceinline__ float block_sum(float v, float* slots) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < kBackThreads / 64; ++w) t += slots[w];
  return t;
}

// Solves H x = r for a symmetric positive semi-definite n x n (n <= 6)
// system by Gaussian elimination with partial pivoting; unknowns whose
// pivot vanishes are set to 0.
__device__ void solve_small(double (&H)[6][6], double (&r)[6], int n, double (&x)[6]) {
  int piv[6];
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int c = 0; c < n; ++c) {
    int best = c;
    for (int i = c + 1; i < n; ++i)
      if (fabs(H[i][c]) > fabs(H[best][c])) best = i;
    if (best != c) {
      for (int j = 0; j < n; ++j) {
        const double t = H[c][j];
        H[c][j] = H[best][j];
        H[best][j] = t;
      }
      const double t = r[c];
      r[c] = r[best];
      r[best] = t;
    }
    if (!(fabs(H[c][c]) > 0.0)) continue;
    for (int i = c + 1; i < n; ++i) {
      const double m = H[i][c] / H[c][c];
      for (int j = c; j < n; ++j) H[i][j] -= m * H[c][j];
      r[i] -= m * r[c];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    if (!(fabs(H[i][i]) > 0.0)) {
      x[i] = 0.0;
      continue;
    }
    double acc = r[i];
    for (int j = i + 1; j < n; ++j) acc -= H[i][j] * x[j];
    x[i] = acc / H[i][i];
  }
  (void)piv;
}

// With `observed` set (refinement), grad_model is the model and the output
// gradient is 2 (model - observed), formed here; the frequency step is then
// clipped to the tone's trust radius (radius[tone] bins) and f + step goes
// to fcand (step_amps unused, grad_freqs / grad_amps may be NULL).
__global__ __launch_bounds__(kBackThreads) void model_backward_kernel(
    DevPtrs p, const float2* __restrict__ amps, int K, int T, int sum_b,
    const float2* __restrict__ G, const float2* __restrict__ dG,
    const float2* __restrict__ grad_model, double* __restrict__ grad_freqs,
    float2* __restrict__ grad_amps, double* __restrict__ step_freqs,
    float2* __restrict__ step_amps, const float2* __restrict__ observed,
    const double* __restrict__ radius, const double* __restrict__ freqs,
    double* __restrict__ fcand, const int32_t* __restrict__ counts, const int32_t* __restrict__ skip) {
  __shared__ float2 sg[4 * 128], sdg[4 * 128];
  __shared__ float slots[kBackThreads / 64];
  constexpr int kPairs = kMaxDims * (kMaxDims + 1) / 2;
  const int64_t f = blockIdx.x / K;
  const int t = int(blockIdx.x % K);
  const FrameDesc& de = model_desc(p, f);
  const int D = de.ndim;
  const int tid = threadIdx.x;
  // refinement: a frame the guard restored takes no step, nor do tones past
  // the frame's count; their candidate is the current frequency
  if (fcand && ((skip && skip[f]) || (counts && t >= counts[f]))) {
    if (tid < D) fcand[(f * K + t) * D + tid] = freqs[(f * K + t) * D + tid];
    return;
  }
  const bool want_step = step_freqs != nullptr || fcand != nullptr;   // the Gauss-Newton block
  const float2* gr = grad_model + frame_bucket_base(p, f);
  const float2* ob = observed ? observed + frame_bucket_base(p, f) : nullptr;
  const bool want_cand = fcand != nullptr;
  // with P = prod_d G_d and part_d = dG_d prod_{e != d} G_e:
  float2 cb = make_float2(0.f, 0.f);        // sum Gr conj(P)
  float2 cf[kMaxDims];                      // sum conj(Gr) part_d
  float pp = 0.f;                           // sum |P|^2
  float2 pj[kMaxDims];                      // sum conj(P) part_d
  float2 jj[kPairs];                        // sum conj(part_d) part_e, d <= e
  for (int d = 0; d < kMaxDims; ++d) {
    cf[d] = make_float2(0.f, 0.f);
    pj[d] = make_float2(0.f, 0.f);
  }
  for (int q = 0; q < kPairs; ++q) jj[q] = make_float2(0.f, 0.f);
  for (int s = 0; s < T; ++s) {
    const int64_t base = ((f * T + s) * K + t) * int64_t(sum_b);
    __syncthreads();
    for (int i = tid; i < sum_b; i += kBackThreads) {
      sg[i] = G[base + i];
      sdg[i] = dG[base + i];
    }
    __syncthreads();
    for (int k = tid; k < de.B; k += kBackThreads) {
      float2 e = gr[int64_t(s) * de.B + k];
      if (ob) {
        const float2 y = ob[int64_t(s) * de.B + k];
        e = make_float2(2.f * (e.x - y.x), 2.f * (e.y - y.y));
      }
      float2 gv[kMaxDims], dv[kMaxDims];
      int acc_off = 0;
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        if (d < D) {
          const int at = acc_off + ((k >> de.bshift[d]) & (de.b[d] - 1));
          gv[d] = sg[at];
          dv[d] = sdg[at];
          acc_off += de.b[d];
        }
      }
      float2 prod = make_float2(1.f, 0.f);
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d)
        if (d < D) prod = cmul(prod, gv[d]);
      const float2 q = cmulc(e, prod);
      cb.x += q.x;
      cb.y += q.y;
      float2 part[kMaxDims];
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        if (d < D) {
          float2 v = dv[d];
#pragma unroll
          for (int e2 = 0; e2 < kMaxDims; ++e2)
            if (e2 < D && e2 != d) v = cmul(v, gv[e2]);
          part[d] = v;
          const float2 w = cmulc(v, e);      // conj(Gr) part_d
          cf[d].x += w.x;
          cf[d].y += w.y;
        }
      }
      if (want_step) {
        pp += prod.x * prod.x + prod.y * prod.y;
        int qi = 0;
#pragma unroll
        for (int d = 0; d < kMaxDims; ++d) {
          if (d < D) {
            const float2 a = cmulc(part[d], prod);   // conj(P) part_d
            pj[d].x += a.x;
            pj[d].y += a.y;
#pragma unroll
            for (int e2 = d; e2 < kMaxDims; ++e2) {
              if (e2 < D) {
                const float2 c = cmulc(part[e2], part[d]);   // conj(part_d) part_e
                jj[qi].x += c.x;
                jj[qi].y += c.y;
              }
              ++qi;
            }
          } else {
            qi += kMaxDims - d;
          }
        }
      }
    }
  }
  const float2 b = amps[f * K + t];
  const double br = b.x, bi = b.y;
  const double gbr = block_sum(cb.x, slots);
  const double gbi = block_sum(cb.y, slots);
  double gfv[kMaxDims];
  for (int d = 0; d < D; ++d) {
    const double cr = block_sum(cf[d].x, slots);
    const double ci = block_sum(cf[d].y, slots);
    gfv[d] = br * cr - bi * ci;               // Re(b (cr + j ci))
  }
  if (tid == 0 && grad_amps) {
    grad_amps[f * K + t] = make_float2(float(gbr), float(gbi));
    for (int d = 0; d < D; ++d) grad_freqs[(f * K + t) * D + d] = gfv[d];
  }
  if (!want_step && !want_cand) return;
  // Gauss-Newton block of this tone over (Re b, Im b, f_0 .. f_{D-1}):
  // H = Re(J^H J) with J = [P, jP, b part_0, ..., b part_{D-1}], and the
  // step solves H x = -g / 2 (g = gradient of sum |model - observed|^2).
  double H[6][6];
  double rhs[6], x[6];
  const int n = 2 + D;
  const double ppd = block_sum(pp, slots);
  double pjr[kMaxDims], pji[kMaxDims];
  for (int d = 0; d < D; ++d) {
    pjr[d] = block_sum(pj[d].x, slots);
    pji[d] = block_sum(pj[d].y, slots);
  }
  double jjr[kMaxDims][kMaxDims];
  {
    int qi = 0;
    for (int d = 0; d < kMaxDims; ++d) {
      for (int e2 = d; e2 < kMaxDims; ++e2, ++qi) {
        if (d < D && e2 < D) {
          jjr[d][e2] = block_sum(jj[qi].x, slots);   // Re part suffices
          jjr[e2][d] = jjr[d][e2];
        }
      }
    }
  }
  if (tid != 0) return;
  const double b2 = br * br + bi * bi;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) H[i][j] = 0.0;
  H[0][0] = ppd;
  H[1][1] = ppd;
  for (int d = 0; d < D; ++d) {
    // <P, b part_d> = b pj[d]
    const double cr = br * pjr[d] - bi * pji[d];
    const double ci = br * pji[d] + bi * pjr[d];
    H[0][2 + d] = H[2 + d][0] = cr;          // Re <P, J_d>
    H[1][2 + d] = H[2 + d][1] = ci;          // Re <jP, J_d> = Im <P, J_d>
    for (int e2 = 0; e2 < D; ++e2) H[2 + d][2 + e2] = b2 * jjr[d][e2];
  }
  for (int i = 0; i < n; ++i) H[i][i] *= 1.0 + 1e-6;   // Levenberg damping
  rhs[0] = -0.5 * gbr;
  rhs[1] = -0.5 * gbi;
  for (int d = 0; d < D; ++d) rhs[2 + d] = -0.5 * gfv[d];
  solve_small(H, rhs, n, x);
  if (want_cand) {
    // trust region of the tone: radius bins per dimension
    const double rad = radius[f * K + t];
    for (int d = 0; d < D; ++d) {
      const double cap = rad / double(de.n[d]);
      const double st = x[2 + d] < -cap ? -cap : (x[2 + d] > cap ? cap : x[2 + d]);
      fcand[(f * K + t) * D + d] = freqs[(f * K + t) * D + d] + st;
    }
    return;
  }
  step_amps[f * K + t] = make_float2(float(x[0]), float(x[1]));
  // trust region: at most a quarter bin per step and dimension
  for (int d = 0; d < D; ++d) {
    const double cap = 0.25 / double(de.n[d]);
    step_freqs[(f * K + t) * D + d] = x[2 + d] < -cap ? -cap : (x[2 + d] > cap ? cap : x[2 + d]);
  }
}

// ---------------------------------------------------------------------------
// Refinement with per-tone step acceptance (rsft_refine). Per step:
//   model_basis(f) -> G, dG;  model_combine -> model
//   refine_gn: each tone's Gauss-Newton step from the residual
//     r = model - observed (as model_backward with the output gradient 2 r),
//     its frequency step clipped to the tone's trust radius (bins / N_d),
//     f' = f + step -> fcand
//   model_basis(f') -> G2
//   refine_accept: per tone, with P = prod_d G_d(f), Q = prod_d G2_d(f') and
//     the inner products pp = <P,P>, qq = <Q,Q>, pq = <P,Q>, rp = <P,r>,
//     rq = <Q,r> (<x,y> = sum conj(x) y): the amplitude for f' by least
//     squares against the residual without the tone, b' = (b conj(pq) - rq)
//     / qq, and the tone's own loss change dL = 2 Re <r, delta> + |delta|^2,
//     delta = b' Q - b P; dL < 0 accepts (f', b') and doubles the radius (up
//     to its maximum), else the frequency stays, b <- b - rp / pp (the
//     least-squares amplitude at f) and the radius halves.
// Tones are decoupled: every tone's step is taken against the same residual.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBackThreads) void refine_accept_kernel(
    DevPtrs p, int K, int T, int sum_b, const float2* __restrict__ G, const float2* __restrict__ G2,
    const float2* __restrict__ model, const float2* __restrict__ observed,
    const double* __restrict__ fcand, double* __restrict__ freqs, float2* __restrict__ amps,
    double* __restrict__ radius, double max_radius, const int32_t* __restrict__ counts,
    const int32_t* __restrict__ skip) {
  __shared__ float2 sg[4 * 128], sq[4 * 128];
  __shared__ float slots[kBackThreads / 64];
  const int64_t f = blockIdx.x / K;
  const int t = int(blockIdx.x % K);
  if (skip[f] || (counts && t >= counts[f])) return;
  const FrameDesc& de = model_desc(p, f);
  const int D = de.ndim;
  const int tid = threadIdx.x;
  const int64_t fb = frame_bucket_base(p, f);
  float pp = 0.f, qq = 0.f;
  float2 pq = make_float2(0.f, 0.f), rp = make_float2(0.f, 0.f), rq = make_float2(0.f, 0.f);
  for (int s = 0; s < T; ++s) {
    const int64_t base = ((f * T + s) * K + t) * int64_t(sum_b);
    __syncthreads();
    for (int i = tid; i < sum_b; i += kBackThreads) {
      sg[i] = G[base + i];
      sq[i] = G2[base + i];
    }
    __syncthreads();
    for (int k = tid; k < de.B; k += kBackThreads) {
      const int64_t at = fb + int64_t(s) * de.B + k;
      const float2 m = model[at];
      const float2 y = observed[at];
      const float2 r = make_float2(m.x - y.x, m.y - y.y);
      float2 P = make_float2(1.f, 0.f), Q = make_float2(1.f, 0.f);
      int acc_off = 0;
#pragma unroll
      for (int d = 0; d < kMaxDims; ++d) {
        if (d < D) {
          const int i = acc_off + ((k >> de.bshift[d]) & (de.b[d] - 1));
          P = cmul(P, sg[i]);
          Q = cmul(Q, sq[i]);
          acc_off += de.b[d];
        }
      }
      pp += P.x * P.x + P.y * P.y;
      qq += Q.x * Q.x + Q.y * Q.y;
      const float2 a = cmulc(Q, P);    // conj(P) Q
      pq.x += a.x;
      pq.y += a.y;
      const float2 b = cmulc(r, P);    // conj(P) r
      rp.x += b.x;
      rp.y += b.y;
      const float2 c = cmulc(r, Q);    // conj(Q) r
      rq.x += c.x;
      rq.y += c.y;
    }
  }
  const double PP = block_sum(pp, slots), QQ = block_sum(qq, slots);
  const double pqr = block_sum(pq.x, slots), pqi = block_sum(pq.y, slots);
  const double rpr = block_sum(rp.x, slots), rpi = block_sum(rp.y, slots);
  const double rqr = block_sum(rq.x, slots), rqi = block_sum(rq.y, slots);
  if (tid != 0) return;
  const int64_t it = f * K + t;
  const float2 bf = amps[it];
  const double br = bf.x, bi = bf.y;
  const double rad = radius[it];
  bool accept = false;
  double bpr = 0.0, bpi = 0.0;
  if (QQ > 0.0) {
    // b' = (b conj(pq) - rq) / qq
    bpr = (br * pqr + bi * pqi - rqr) / QQ;
    bpi = (bi * pqr - br * pqi - rqi) / QQ;
    // <r, delta> = b' conj(rq) - b conj(rp)
    const double rdr = (bpr * rqr + bpi * rqi) - (br * rpr + bi * rpi);
    // |delta|^2 = |b'|^2 qq + |b|^2 pp - 2 Re(conj(b') b conj(pq))
    const double cbr = bpr * br + bpi * bi;          // conj(b') b
    const double cbi = bpr * bi - bpi * br;
    const double cross = cbr * pqr + cbi * pqi;      // Re((cbr + j cbi)(pqr - j pqi))
    const double dd = (bpr * bpr + bpi * bpi) * QQ + (br * br + bi * bi) * PP - 2.0 * cross;
    accept = 2.0 * rdr + dd < 0.0;
  }
  if (accept) {
    for (int d = 0; d < D; ++d) freqs[it * D + d] = fcand[it * D + d];
    amps[it] = make_float2(float(bpr), float(bpi));
    radius[it] = 2.0 * rad < max_radius ? 2.0 * rad : max_radius;
  } else {
    if (PP > 0.0) amps[it] = make_float2(float(br - rpr / PP), float(bi - rpi / PP));
    radius[it] = 0.5 * rad;
  }
}

// sum_{s,k} |model - observed|^2 of each frame, in FP64 (one work-group per frame)
__global__ __launch_bounds__(kBackThreads) void refine_loss_kernel(DevPtrs p, int T,
                                                                   const float2* __restrict__ model,
                                                                   const float2* __restrict__ observed,
                                                                   double* __restrict__ loss) {
  __shared__ double dslots[kBackThreads / 64];
  const int64_t f = blockIdx.x;
  const FrameDesc& de = model_desc(p, f);
  const int64_t fb = frame_bucket_base(p, f);
  const int64_t n = int64_t(T) * de.B;
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kBackThreads) {
    const float2 m = model[fb + k];
    const float2 y = observed[fb + k];
    const double dr = double(m.x) - double(y.x), di = double(m.y) - double(y.y);
    acc += dr * dr + di * di;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) dslots[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kBackThreads / 64; ++w) tot += dslots[w];
    loss[f] = tot;
  }
}

// trust radii of every tone set to r0, and per frame no best loss yet and
// no skipped step (kernels rather than memsets, so that the sequence can be
// captured)
__global__ void refine_fill_kernel(double* __restrict__ radius, int64_t n, double r0) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) radius[i] = r0;
}
__global__ void refine_frame_init_kernel(double* __restrict__ best, int32_t* __restrict__ skip, int64_t batch) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < batch) {
    best[i] = __builtin_huge_val();
    skip[i] = 0;
  }
}

// The per-frame guard of an iteration (one work-group per frame): the loss
// of the current state above the lowest so far (tones' decoupled steps can
// overshoot together where they share buckets) restores the state of that
// lowest loss, halves the trust radii and marks the frame to take no step;
// otherwise the current state becomes the best. loss_out (may be NULL)
// receives the lowest loss so far.
__global__ __launch_bounds__(kBackThreads) void refine_guard_kernel(
    int K, int D, const int32_t* __restrict__ counts, const double* __restrict__ loss_now,
    double* __restrict__ best, int32_t* __restrict__ skip, double* __restrict__ freqs,
    float2* __restrict__ amps, double* __restrict__ radius, double* __restrict__ saved_f,
    float2* __restrict__ saved_a, double* __restrict__ loss_out) {
  const int64_t f = blockIdx.x;
  const int kt = counts ? (counts[f] < K ? counts[f] : K) : K;
  const double now = loss_now[f];
  const double b = best[f];
  const bool restore = now > b;
  for (int t = threadIdx.x; t < kt; t += kBackThreads) {
    const int64_t it = f * K + t;
    if (restore) {
      for (int d = 0; d < D; ++d) freqs[it * D + d] = saved_f[it * D + d];
      amps[it] = saved_a[it];
      radius[it] *= 0.5;
    } else {
      for (int d = 0; d < D; ++d) saved_f[it * D + d] = freqs[it * D + d];
      saved_a[it] = amps[it];
    }
  }
  if (threadIdx.x == 0) {
    const double nb = restore ? b : now;
    best[f] = nb;
    skip[f] = restore ? 1 : 0;
    if (loss_out) loss_out[f] = nb;
  }
}

// Initial amplitude of every tone (one thread per (frame, tone)): the grid
// cell nearest to f, floor(f_d N_d + 1/2) mod N_d; in each estimation round
// s (the rounds of the descriptor's mask) the ratio of the observed bucket
// y_s[j_s], j_s = M(cell, sigma_s) (Def. 3), to the unit-tone model
// P_s[j_s] = prod_d G_{s,d}[j_{s,d}]; the ratio whose magnitude is the
// median over the rounds (rank floor((n - 1) / 2) ascending, the earlier
// round on ties) is the amplitude a; spread (when not NULL) gets
// max_s |a_s - a| / |a| (infinity when a = 0).
__global__ void initial_amp_kernel(DevPtrs p, const double* __restrict__ freqs, int64_t batch, int K,
                                   int T, int sum_b, const float2* __restrict__ G,
                                   const float2* __restrict__ observed, float2* __restrict__ amps,
                                   float* __restrict__ spread) {
  const int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it >= batch * K) return;
  const int64_t f = it / K;
  const int t = int(it % K);
  const FrameDesc& de = model_desc(p, f);
  const int D = de.ndim;
  const int64_t fb = frame_bucket_base(p, f);
  uint32_t cell[kMaxDims];
  for (int d = 0; d < D; ++d) {
    const double v = floor(freqs[it * D + d] * double(de.n[d]) + 0.5);
    const int64_t c = int64_t(v) % int64_t(de.n[d]);
    cell[d] = uint32_t(c < 0 ? c + de.n[d] : c);
  }
  float2 ratio[kMaxRounds];
  float mag[kMaxRounds];
  int n = 0;
  uint64_t rest = de.est_mask;
  while (rest) {
    const int s = __builtin_ctzll(rest);
    rest &= rest - 1ull;
    const float2* g = G + ((f * T + s) * K + t) * int64_t(sum_b);
    float2 P = make_float2(1.f, 0.f);
    int jf = 0, off = 0;
    for (int d = 0; d < D; ++d) {
      const uint32_t u = (uint32_t(de.sigma[s][d]) * cell[d]) & uint32_t(de.n[d] - 1);
      const int jd = int(u >> de.lshift[d]);
      P = cmul(P, g[off + jd]);
      jf |= jd << de.bshift[d];
      off += de.b[d];
    }
    const float2 y = observed[fb + int64_t(s) * de.B + jf];
    const float den = P.x * P.x + P.y * P.y;
    const float2 q = den > 0.f ? make_float2((y.x * P.x + y.y * P.y) / den, (y.y * P.x - y.x * P.y) / den)
                               : make_float2(0.f, 0.f);
    ratio[n] = q;
    mag[n] = q.x * q.x + q.y * q.y;
    ++n;
  }
  // the element of rank (n - 1) / 2 by magnitude (ties: the earlier round)
  const int want = (n - 1) / 2;
  float2 out = make_float2(0.f, 0.f);
  for (int a = 0; a < n; ++a) {
    int rank = 0;
    for (int b2 = 0; b2 < n; ++b2)
      rank += (mag[b2] < mag[a]) || (mag[b2] == mag[a] && b2 < a);
    if (rank == want) out = ratio[a];
  }
  amps[it] = out;
  if (spread) {
    const float m2 = out.x * out.x + out.y * out.y;
    float worst = 0.f;
    for (int a = 0; a < n; ++a) {
      const float dx = ratio[a].x - out.x, dy = ratio[a].y - out.y;
      worst = fmaxf(worst, dx * dx + dy * dy);
    }
    spread[it] = m2 > 0.f ? sqrtf(worst / m2) : __builtin_huge_valf();
  }
}

int launch_model_forward(const DevPtrs& p, const double* freqs, const float2* amps, int64_t batch,
                         int K, int D, int T, int maxB, int sum_b, float2* G, float2* dG,
                         float2* model, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t items = batch * T * D * int64_t(K);
  if (items <= 0) return hipSuccess;
  if (items >= (int64_t(1) << 31) || batch > 65535 || T > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(model_basis_kernel, dim3(unsigned(items)), dim3(kBasisThreads), 0, st, p, freqs,
                     K, D, T, sum_b, G, dG);
  const dim3 grid{unsigned((maxB + kCombineThreads - 1) / kCombineThreads), unsigned(T), unsigned(batch)};
  hipLaunchKernelGGL(model_combine_kernel, grid, dim3(kCombineThreads), 0, st, p, amps, K, T, sum_b, G,
                     model, static_cast<const int32_t*>(nullptr), static_cast<const float2*>(nullptr));
  return hipGetLastError();
}

int launch_model_residual(const DevPtrs& p, const float2* observed, const double* freqs, const float2* amps,
                          int64_t batch, int K, int D, int T, int maxB, int sum_b, const int32_t* counts,
                          float2* G, float2* dG, float2* residual, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t items = batch * T * D * int64_t(K);
  if (items <= 0) return hipSuccess;
  if (items >= (int64_t(1) << 31) || batch > 65535 || T > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(model_basis_kernel, dim3(unsigned(items)), dim3(kBasisThreads), 0, st, p, freqs,
                     K, D, T, sum_b, G, dG);
  const dim3 grid{unsigned((maxB + kCombineThreads - 1) / kCombineThreads), unsigned(T), unsigned(batch)};
  hipLaunchKernelGGL(model_combine_kernel, grid, dim3(kCombineThreads), 0, st, p, amps, K, T, sum_b, G,
                     residual, counts, observed);
  return hipGetLastError();
}

int launch_model_backward(const DevPtrs& p, const float2* amps, int64_t batch, int K, int T,
                          int sum_b, const float2* G, const float2* dG, const float2* grad_model,
                          double* grad_freqs, float2* grad_amps, double* step_freqs,
                          float2* step_amps, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t blocks = batch * int64_t(K);
  if (blocks <= 0) return hipSuccess;
  if (blocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(model_backward_kernel, dim3(unsigned(blocks)), dim3(kBackThreads), 0, st, p, amps,
                     K, T, sum_b, G, dG, grad_model, grad_freqs, grad_amps, step_freqs, step_amps,
                     static_cast<const float2*>(nullptr), static_cast<const double*>(nullptr),
                     static_cast<const double*>(nullptr), static_cast<double*>(nullptr),
                     static_cast<const int32_t*>(nullptr), static_cast<const int32_t*>(nullptr));
  return hipGetLastError();
}

int launch_initial_amplitudes(const DevPtrs& p, const double* freqs, int64_t batch, int K, int D, int T,
                              int maxB, int sum_b, float2* G, float2* dG, const float2* observed,
                              float2* amps, float* spread, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t items = batch * T * D * int64_t(K);
  if (items <= 0) return hipSuccess;
  if (items >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  (void)maxB;
  hipLaunchKernelGGL(model_basis_kernel, dim3(unsigned(items)), dim3(kBasisThreads), 0, st, p, freqs, K, D,
                     T, sum_b, G, dG);
  const int64_t n = batch * K;
  hipLaunchKernelGGL(initial_amp_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, freqs, batch,
                     K, T, sum_b, static_cast<const float2*>(G), observed, amps, spread);
  return hipGetLastError();
}

int launch_refine(const DevPtrs& p, const float2* observed, double* freqs, float2* amps, int64_t batch,
                  int K, int D, int T, int maxB, int sum_b, int steps, double trust_bins, const int32_t* counts,
                  const RefineWork& w, double* loss, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t items = batch * T * D * int64_t(K);
  const int64_t tones = batch * int64_t(K);
  if (items <= 0) return hipSuccess;
  if (items >= (int64_t(1) << 31) || batch > 65535 || T > 65535) return hipErrorInvalidValue;
  const dim3 cgrid{unsigned((maxB + kCombineThreads - 1) / kCombineThreads), unsigned(T), unsigned(batch)};
  hipLaunchKernelGGL(refine_fill_kernel, dim3(unsigned((tones + 255) / 256)), dim3(256), 0, st, w.radius,
                     tones, trust_bins);
  hipLaunchKernelGGL(refine_frame_init_kernel, dim3(unsigned((batch + 255) / 256)), dim3(256), 0, st, w.best,
                     w.skip, batch);
  for (int step = 0; step <= steps; ++step) {
    hipLaunchKernelGGL(model_basis_kernel, dim3(unsigned(items)), dim3(kBasisThreads), 0, st, p, freqs, K, D,
                       T, sum_b, w.G, w.dG);
    hipLaunchKernelGGL(model_combine_kernel, cgrid, dim3(kCombineThreads), 0, st, p, amps, K, T, sum_b, w.G,
                       w.model, counts, static_cast<const float2*>(nullptr));
    hipLaunchKernelGGL(refine_loss_kernel, dim3(unsigned(batch)), dim3(kBackThreads), 0, st, p, T,
                       static_cast<const float2*>(w.model), observed, w.loss_now);
    hipLaunchKernelGGL(refine_guard_kernel, dim3(unsigned(batch)), dim3(kBackThreads), 0, st, K, D, counts,
                       static_cast<const double*>(w.loss_now), w.best, w.skip, freqs, amps, w.radius,
                       w.saved_f, w.saved_a, loss ? loss + int64_t(step) * batch : static_cast<double*>(nullptr));
    if (step == steps) break;
    hipLaunchKernelGGL(model_backward_kernel, dim3(unsigned(tones)), dim3(kBackThreads), 0, st, p,
                       static_cast<const float2*>(amps), K, T, sum_b, static_cast<const float2*>(w.G),
                       static_cast<const float2*>(w.dG), static_cast<const float2*>(w.model),
                       static_cast<double*>(nullptr), static_cast<float2*>(nullptr),
                       static_cast<double*>(nullptr), static_cast<float2*>(nullptr), observed,
                       static_cast<const double*>(w.radius), static_cast<const double*>(freqs), w.fcand, counts,
                       static_cast<const int32_t*>(w.skip));
    hipLaunchKernelGGL(model_basis_kernel, dim3(unsigned(items)), dim3(kBasisThreads), 0, st, p,
                       static_cast<const double*>(w.fcand), K, D, T, sum_b, w.G2, w.dG2);
    hipLaunchKernelGGL(refine_accept_kernel, dim3(unsigned(tones)), dim3(kBackThreads), 0, st, p, K, T, sum_b,
                       static_cast<const float2*>(w.G), static_cast<const float2*>(w.G2),
                       static_cast<const float2*>(w.model), observed, static_cast<const double*>(w.fcand),
                       freqs, amps, w.radius, trust_bins, counts, static_cast<const int32_t*>(w.skip));
  }
  return hipGetLastError();
}

}  // namespace rsft

// Device-side helpers shared by the HIP kernels of the RSFT hot path for
// gfx950 (CDNA4, wave64). One source per stage (Algorithm 1 of the paper,
// Location procedure):
//   fold.hip      window W, permutation P_sigma, flat window Wbar and
//                 aliasing, all T rounds from one pass over the input
//                 (Def. 1, 2; eq. l)
//   dft.hip       B-point N-D DFT of each round's buckets on MFMA (eq. f),
//                 then |.|^2, first-stage NP threshold (eq. exp, eq. tpd)
//                 and flags
//   vote.hip      vote: reverse mapping + accumulation + second stage
//                 (Def. 3-4, eq. a_i), enumerating only the preimages of
//                 flagged buckets; scan: per-frame detection counts and
//                 record offsets
//   estimate.hip  ordered compaction of the detections, gain-corrected
//                 magnitudes, peak test and log-parabolic off-grid offsets

#pragma once

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

// Chunk (frame f, chunk c) of work-group b: from the chunk list when the
// launch uses it, else from the (chunk, frame) or XCD-grouped grid the caller
// decodes; false for list padding.
__device__ __forceinline__ bool listed_chunk(const DevPtrs& p, int64_t b, int64_t& f, int& c) {
  const int32_t* e = p.chunk_list + 2 * b;
  f = e[0];
  c = e[1];
  return f >= 0;
}

}  // namespace rsft

// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <stdint.h>

#include "rsft.h"

namespace rsft {

constexpr int kMaxDims = RSFT_MAX_DIMS;
constexpr int kMaxRounds = RSFT_MAX_ROUNDS;
constexpr int kMaxBuckets = 16384;        // B per frame (DFT stage keeps a frame's round in LDS)
constexpr int kMaxLastBuckets = 4096;     // B_{D-1} (fold stage residue slots per pass)
constexpr int kMaxDetectionsPerFrame = 1 << 24;
constexpr int kDefaultDetections = 16384;
constexpr int kCompactShift = 15;         // cells per compaction chunk = 2^15
constexpr int kChunkRecords = 1024;       // records a chunk's work-group builds at a time (and,
                                          // with overflow workers, in all)
constexpr int kItemShift = 8;             // records per overflow item = 2^8
constexpr int kMaxEstRounds = 5;          // estimation rounds of the specialised estimate kernels
constexpr int kFoldRoundGroup = 4;        // rounds folded per pass over the input

// Everything a kernel needs to know about one frame descriptor. Lives in
// device memory (one per descriptor); POD so host and device share it.
struct FrameDesc {
  int32_t ndim, T, mu, noise_mode;
  int32_t n[kMaxDims];        // N_d
  int32_t b[kMaxDims];        // B_d
  int32_t l[kMaxDims];        // L_d = N_d / B_d
  int32_t lshift[kMaxDims];   // log2 L_d
  int32_t nshift[kMaxDims];   // sum_{e>d} log2 N_e  (row-major cell strides)
  int32_t bshift[kMaxDims];   // sum_{e>d} log2 B_e  (row-major bucket strides)
  int32_t tshift[kMaxDims];   // sum_{e>d} log2 L_e  (offset inside a bucket's preimage)
  int64_t N;                  // prod N_d
  int32_t B;                  // prod B_d
  int32_t Lshift;             // log2(N / B)
  // fold view: rows = flattened leading dims, columns = last dim
  int32_t n_last, b_last, rows_total, classes, rows_per_class;
  int32_t chunk_cols, nchunks;
  // fold row: the last dimension, or for short-row 3-D+ frames the last two
  // flattened (fold_nl cells, fold_bl residue classes). Residue of slot q of
  // a row: ((q >> fold_lw) mod (fold_bl / fold_bin)) * fold_bin + q mod
  // fold_bin, with fold_bin = B_{D-1} and fold_lw = log2 N_{D-1} (fold_bl =
  // fold_bin for one dimension: q mod B_{D-1}). fold_cpt: residue classes
  // per fold tile (rows shorter than the smallest fold pass: several
  // classes share a work-group, one group of threads per class; else 1)
  int32_t fold_nl, fold_bl, fold_bin, fold_lw, fold_cpt;
  int32_t words;              // flag words per round = ceil(B / 32)
  int32_t cap;                // detection capacity of a frame
  int32_t n_est;              // rounds used for magnitude estimates (1..T)
  int32_t est_rounds[kMaxEstRounds];  // the first min(n_est, kMaxEstRounds) of them
  uint64_t est_mask;                   // the same rounds as a bit mask
  int32_t sigma[kMaxRounds][kMaxDims];
  int32_t sigma_inv[kMaxRounds][kMaxDims];
  int32_t tau[kMaxRounds][kMaxDims];      // sigma_inv mod B_d
  double gamma[kMaxRounds];               // KNOWN-mode thresholds
  double log_inv_p1;                      // ln(1 / p1)
  double renyi_h;                         // sum_{i<B/2} 1/(B-i)
  // offsets into the plan's table arrays
  int64_t wrow_off;       // float2 [T][rows_total]
  int64_t wcol_off;       // float2 [T][n_last]
  int64_t rowlist_off;    // int32  [rows_total], grouped by residue class
  int64_t tw_off[kMaxDims];    // float2 [B_d]: exp(-2 pi i m / B_d)
  int64_t gain_off[kMaxDims];  // float [L_d]: N_d / flat-window response
  int64_t win_off[kMaxDims];   // float  [N_d]: pre-permutation window (per-frame path)
  int64_t flat_off[kMaxDims];  // float2 [N_d]: flat window (per-frame path)
  // workspace offsets of the descriptor's first frame, and per-frame strides
  // (uniform plans: frame f of the batch uses off + f * stride)
  int64_t in_off, in_stride;           // input elements
  int64_t part_off, part_stride;       // float2: [nchunks][T][B]
  int64_t bucket_off, bucket_stride;   // float2: [T][B]
  int64_t flag_off, flag_stride;       // uint32: [T][words]
  int64_t bitmap_off, bitmap_stride;   // uint32: [ceil(N / 32)] detected-cell bits
  int64_t chunk_off, chunk_stride;     // uint32 counts / int64 ranks: [cchunks]
  int32_t cchunks;                     // compaction chunks = ceil(N / 2^15)
  int32_t bitmap_words;                // ceil(N / 32)
  int32_t segments;                    // 1: round s reads segment s (input [T][N] per frame)
  int32_t pad0;
  int64_t vtab_off;                    // uint32 [T][B_last][N_last / 32]: word-parallel vote tables
  int64_t vexp_off, vexp_stride;       // uint32 [T][B / B_last][N_last / 32]: bucket-row masks
};

// A detection as the estimate stores it on the device: 32 bytes instead of
// the 88 of rsft_detection, which rsft_detect forms on the host from it
// (frequency (idx + delta) / N_d in FP64, wrapped to [0, 1)).
struct DetRec {
  uint64_t key;                // bits 0..39 row-major cell, 40..46 votes, 47 is_peak
  uint32_t frame;
  float magnitude;             // gain-corrected magnitude
  float delta[kMaxDims];       // off-grid offset per dimension (bins, in [-1/2, 1/2])
};
static_assert(sizeof(DetRec) == 32, "DetRec is 32 bytes");
constexpr int kKeyVotesShift = 40;
constexpr uint64_t kKeyCellMask = (uint64_t(1) << 40) - 1;

// Device-side view of a launch: pointers into the plan's arrays.
struct DevPtrs {
  const FrameDesc* descs;
  int uniform;                 // 1: one descriptor for every frame
  const float2* wrow;
  const float2* wcol;
  const int32_t* rowlist;
  const float2* tw;
  const float* inv_gains;
  const float* win;
  const float2* flat;
  float2* part;
  float2* buckets;
  float* powers;               // |buckets|^2, same layout
  uint32_t* flags;
  uint32_t* bitmap;            // detected cells; every word written by the vote stage
  uint32_t* chunk_counts;      // detections per compaction chunk
  int64_t* chunk_offsets;      // rank of a chunk's first detection within its frame
  int64_t* counts;             // [frames] exact detections per frame
  int64_t* offsets;            // [frames + 1] first record of each frame
  // overflow work list of the estimate: the records of a chunk beyond its
  // first kChunkRecords (and within the frame's capacity) form items of up to
  // 2^kItemShift consecutive records
  int64_t* chunk_items;        // items of a frame before a chunk (chunk layout)
  int64_t* item_counts;        // [frames] items per frame
  int64_t* item_offsets;       // [frames + 1] first item of each frame
  uint32_t* scan_done;         // frames finished by the scan (0 between launches)
  DetRec* records;
  const int32_t* tiles;        // uneven plans: [ntiles][3] (frame, class, chunk)
  // uneven plans whose frames differ in chunk count: [n][2] (frame, chunk) of
  // every compaction chunk, position p holding a frame congruent to p mod 8
  // (work-groups are dealt to the eight XCDs round-robin); (-1, -1) pads
  const int32_t* chunk_list;
  // word-parallel vote: the tables of every descriptor (FrameDesc::vtab_off)
  // and, for uneven plans whose frames differ in chunk count, [n][2] (frame,
  // first chunk) groups of kVoteCpw chunks; (-1, -1) pads
  const uint32_t* vote_tab;
  const int32_t* vote_list;
  // word-parallel vote: per frame and round the cell mask of every bucket
  // row (FrameDesc::vexp_off), written by its first kernel, read by its
  // second; for uneven plans the first kernel's work, [n][2] (frame, block
  // of kVoteExpWords mask words), largest frames first
  uint32_t* vote_exp;
  const int32_t* vote_exp_list;
};

// Launch configuration of the fold stage, chosen per plan.
struct FoldConfig {
  int threads;      // work-group size (256 or 512)
  int vec;          // complex elements per thread per row (2 or 4)
  int nontemporal;  // 1: streaming (non-temporal) loads of the input
};
constexpr int kFoldMaxP = 2048;   // largest threads * vec a plan may be tuned to
constexpr int kFoldMinP = 512;    // smallest

// Launchers (fold.hip, dft.hip, vote.hip, estimate.hip). All enqueue on `stream` and return hipError_t.
int launch_fold(const DevPtrs& p, const void* input, int dtype, int64_t nframes,
                int64_t tiles_per_frame, int64_t ntiles, int round0, int rounds,
                int T, const FoldConfig& cfg, void* stream);
// order (may be NULL): frame of each grid row, e.g. the frames of an uneven
// batch by decreasing bucket count so that the largest transforms start
// first; threads: work-group size, 64, 256 or 1024
int launch_dft(const DevPtrs& p, int64_t nframes, int T, int plane, int pad, int sum_tw,
               int identity_relabel, int nchunks_override, const int32_t* order, int threads,
               void* stream);
// The same transform in two passes (frames of D >= 2 whose trailing
// dimensions hold at most kSplitMaxSlab buckets, KNOWN noise floor): pass 1
// over slab groups into `inter` (bucket layout), pass 2 over column groups
// with relabel, threshold and outputs. max_b0: largest B_0; max_groups1 / 2:
// most slab / column groups of a frame; max_e1: most buckets of a pass-1
// group (G slabs of S buckets, G S <= kSplitGroup or G = 1); sum_tw:
// largest sum_d B_d.
constexpr int kSplitMaxSlab = 4096;
constexpr int kSplitGroup = 1024;
int launch_dft_split(const DevPtrs& p, int64_t nframes, int T, int max_b0, int max_groups1, int max_groups2,
                     int max_e1, int sum_tw, float2* inter, const int32_t* order, void* stream);
// vote paths: per cell (any shape), rows of 64..4096 cells (T <= 4), rows of
// exactly 32 cells (bit-parallel masks), rows of 128..4096 cells (word-
// parallel masks, any T)
constexpr int kVoteCells = 0, kVoteRows = 1, kVoteMasks32 = 2, kVoteWords = 3;
constexpr int kVoteCpw = 4;   // compaction chunks per work-group of the word-parallel vote
constexpr int kVoteExpWords = 1024;   // bucket-row mask words per work-group of its first kernel
// nlist > 0: one work-group per chunk_list entry (whole batch, frame0 = 0);
// the word-parallel vote instead takes vote_list (nvlist > 0: one work-group
// per (frame, first chunk) entry, groups of kVoteCpw chunks). tab_words: LDS
// words of that vote's per-round table, the largest B_last * N_last / 32 of
// the plan; exp_blocks: the most kVoteExpWords blocks of bucket-row masks
// (B / B_last * N_last / 32 words per round) of a frame; nexp_list > 0: one
// work-group of the masks per vote_exp_list entry and round (whole batch,
// frame0 = 0)
int launch_vote(const DevPtrs& p, int64_t nframes, int T, int mu, int max_cchunks,
                int max_words, int dims_mask, int vote_path, int frame0, int64_t nlist, int64_t nvlist,
                int tab_words, int exp_blocks, int64_t nexp_list, void* stream);
// items: 1 also lists the estimate's overflow items (plans with overflow
// workers); fpb: frames per work-group (1, or 256 / chunks per frame in a
// uniform plan of at most 128 chunks per frame)
int launch_scan(const DevPtrs& p, int64_t nframes, int items, int fpb, void* stream);
// inverse flat-window gains the estimate keeps in LDS: frames whose sum over
// d of L_d is larger make the plan launch the variant reading them from
// global memory (global_gains = 1)
constexpr int kEstGainLds = 384;
// est_mask: bit m set when some frame uses m estimation rounds (1..5); bit 6
// when some frame uses more (the loop variant)
// workers: 1 adds overflow workers (two per compute unit of the num_cus)
int launch_estimate(const DevPtrs& p, int64_t nframes, int T, int max_cchunks, int dims_mask,
                    int est_mask, int workers, int num_cus, int64_t nlist, int global_gains, void* stream);
// Per-frame comparator path.
int launch_plain_fold(const DevPtrs& p, const void* input, int dtype, int64_t frame,
                      int round, int B, void* stream);
int launch_plain_dft(const DevPtrs& p, int64_t frame, int T, int plane, int pad, int sum_tw,
                     void* stream);
// Bucketized forward model and its gradients (refine.hip). G and dG hold
// [batch][T][K][sum_b] complex factors (per dimension at offset sum_{e<d} B_e).
int launch_model_forward(const DevPtrs& p, const double* freqs, const float2* amps, int64_t batch,
                         int K, int D, int T, int maxB, int sum_b, float2* G, float2* dG,
                         float2* model, void* stream);
// observed - model of the first counts[f] tones (all K when counts is NULL)
int launch_model_residual(const DevPtrs& p, const float2* observed, const double* freqs, const float2* amps,
                          int64_t batch, int K, int D, int T, int maxB, int sum_b, const int32_t* counts,
                          float2* G, float2* dG, float2* residual, void* stream);
// Workspace of a refinement: factors at f (G, dG) and at the candidate
// frequencies (G2, dG2), [batch][T][K][sum_b] each; the model, in the bucket
// layout; per tone the trust radius (bins) and the candidate frequencies.
struct RefineWork {
  float2 *G, *dG, *G2, *dG2, *model;
  double *radius, *fcand;
  double *saved_f;         // [batch][K][D] state of the lowest loss so far
  float2* saved_a;         // [batch][K]
  double *best, *loss_now; // [batch]
  int32_t* skip;           // [batch]: 1 when the guard restored the frame
};
// Initial amplitudes of tones at `freqs` from the observed buckets (G, dG:
// factor scratch of one model).
int launch_initial_amplitudes(const DevPtrs& p, const double* freqs, int64_t batch, int K, int D, int T,
                              int maxB, int sum_b, float2* G, float2* dG, const float2* observed,
                              float2* amps, float* spread, void* stream);
// `steps` refinement steps in place on freqs / amps; loss (may be NULL):
// [steps + 1][batch] FP64 losses before each step and after the last.
// counts (may be NULL): tones taking part per frame (the first counts[f]).
int launch_refine(const DevPtrs& p, const float2* observed, double* freqs, float2* amps, int64_t batch,
                  int K, int D, int T, int maxB, int sum_b, int steps, double trust_bins, const int32_t* counts,
                  const RefineWork& w, double* loss, void* stream);
// Device address of the library's static scratch array on `device`, which
// must be the current device (resolved once per device, then cached).
int static_scratch(int device, void** out);
int launch_model_backward(const DevPtrs& p, const float2* amps, int64_t batch, int K, int T,
                          int sum_b, const float2* G, const float2* dG, const float2* grad_model,
                          double* grad_freqs, float2* grad_amps, double* step_freqs,
                          float2* step_amps, void* stream);

}  // namespace rsft

/*
 * rsft.h - C ABI of the MI355X (gfx950) RSFT library.
 *
 * RSFT: S. Wang, V. M. Patel, A. Petropulu, "An Efficient High-Dimensional
 * Sparse Fourier Transform". The library runs the Location procedure of
 * Algorithm 1 (Sec. III-C) on batches of complex frames in any fixed
 * dimension D <= 4 and returns sparse frequency locations, each with an
 * off-grid frequency estimate:
 *
 *   pre-permutation window W           (Sec. III-A, Sec. III-C.1)
 *   permutation P_{sigma,0}            (Definition 1, per dimension)
 *   flat window Wbar                   (Sec. IV-B)
 *   aliasing into B buckets            (Definition 2, eq. l)
 *   B-point N-D DFT                    (eq. f)
 *   |.|^2 and first-stage NP detection (eq. exp, eq. tpd)
 *   reverse mapping + accumulation     (Definition 4, eq. a_i)
 *   second-stage detection             (Sec. III-C.5)
 *   off-grid estimate per detected cell
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns rsft_status (RSFT_OK == 0); no C++ exception crosses
 *   this interface. On error, rsft_last_error() returns a thread-local
 *   message describing the most recent failure on the calling thread.
 * - "Device pointer" means memory from hipMalloc (or a torch tensor's
 *   data_ptr()) on the device the plan was created on. "Host pointer" means
 *   ordinary process memory.
 * - `stream` arguments are hipStream_t values passed as void*; NULL means the
 *   default stream of the current device.
 * - Frames are row-major [N_0][N_1]...[N_{D-1}] with the last dimension
 *   contiguous; complex values are interleaved (re, im); complex64 = two
 *   floats, complex128 = two doubles.
 * - A plan owns all its device tables and workspace. It is immutable after
 *   creation except for rsft_set_option, is used by one stream at a time,
 *   and is independent of every other plan. Calls on one plan are not
 *   thread-safe; different plans may be used from different threads.
 */
#ifndef RSFT_H
#define RSFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSFT_MAX_DIMS 4
#define RSFT_MAX_ROUNDS 64

typedef enum {
  RSFT_OK = 0,
  RSFT_ERROR_INVALID_ARGUMENT = 1, /* NULL pointer, out-of-range value */
  RSFT_ERROR_NOT_POW2 = 2,         /* N_d or B_d not a power of two */
  RSFT_ERROR_BAD_SIGMA = 3,        /* sigma even (not invertible) or outside [1, N_d) */
  RSFT_ERROR_UNSUPPORTED = 4,      /* valid for the paper, beyond this library's limits */
  RSFT_ERROR_OUT_OF_MEMORY = 5,    /* a device or host allocation failed */
  RSFT_ERROR_DEVICE = 6,           /* a HIP runtime call failed */
  RSFT_ERROR_CAPACITY = 7,         /* detection records truncated (counts stay exact) */
  RSFT_ERROR_NOT_READY = 8         /* results requested before any execute */
} rsft_status;

enum { RSFT_C64 = 0, RSFT_C128 = 1 };                  /* input element type */
enum { RSFT_NOISE_KNOWN = 0, RSFT_NOISE_ESTIMATED = 1 };

/*
 * One frame shape and the paper's parameter set (Problem 1, Sec. IV-A):
 * signal dimensions, windows, bucket counts, permutations, Pfa.
 *
 * ndim            D, 1..4.
 * n[d], b[d]      N_d and B_d, powers of two with 1 <= B_d < N_d (Sec. II
 *                 notation; Definition 2 requires B < N). Entries d >= ndim
 *                 are ignored. N = prod N_d must be < 2^40.
 * rounds          T, 1..RSFT_MAX_ROUNDS: iterations of Algorithm 1 with
 *                 independent permutations, over the same frame (segments
 *                 = 0) or over T data segments (segments = 1).
 * sigma           host pointer to T*ndim permutation factors, round-major
 *                 (sigma[s*ndim + d]); each odd and in [1, N_d) (Definition 1:
 *                 sigma invertible mod N_d). NULL: drawn from `seed`,
 *                 uniformly over the odd integers of [1, N_d), independently
 *                 per round and dimension (splitmix64 counter stream). Copied
 *                 at plan creation.
 * seed            see sigma.
 * window_atten_db sidelobe attenuation of the Dolph-Chebyshev pre-permutation
 *                 window (Sec. III-C.1); 0 = rectangular window.
 * flat_atten_db   attenuation of the Chebyshev base of the flat window
 *                 (Sec. IV-B); < 0: same as window_atten_db; 0: rectangular
 *                 base (an exact box of N_d/B_d bins).
 * pfa             design false-alarm probability of one grid cell after the
 *                 second stage, in (0, 1).
 * mu              second-stage threshold 1..T (a cell is declared when at
 *                 least mu of its T buckets were flagged); 0 means T.
 * noise_mode      RSFT_NOISE_KNOWN: first-stage threshold of round s is
 *                 gamma_s = noise_var * beta(sigma_s) * ln(1/p1) (eq. tpd with
 *                 beta of eq. alpha_beta), p1 solving P[Bin(T,p1) >= mu] = pfa.
 *                 RSFT_NOISE_ESTIMATED: noise_var*beta(sigma_s) is replaced by
 *                 an FP64 order-statistic estimate from the round's own
 *                 buckets (lower median X_(h), h = B/2, divided by
 *                 sum_{i<h} 1/(B-i)).
 * noise_var       sigma_n^2 for RSFT_NOISE_KNOWN (> 0).
 * dtype           RSFT_C64 or RSFT_C128 (every frame of a plan must agree).
 * max_detections  record capacity per frame, 1..2^24; 0 = 16384.
 * max_batch       frames per execute for a uniform plan (nframes == 1),
 *                 >= 1; 0 = 1. Ignored when nframes > 1.
 * segments        0: every round reads the same frame. 1: segment mode
 *                 (Sec. IV-A, the T data segments of the signal model, as in
 *                 the Bartlett method of Appendix A): a frame is T segments
 *                 of N samples, [T][N_0]...[N_{D-1}], and round s processes
 *                 segment s with sigma_s; votes accumulate over the segments.
 *                 Every descriptor of a plan must agree.
 * reserved0       must be 0.
 * stage1_pfa      > 0: the first-stage false-alarm probability p1 of every
 *                 round itself, in (0, 1) (e.g. the design of eq. opt); pfa
 *                 is then not used to derive it. 0: p1 from pfa as above.
 */
typedef struct {
  int32_t ndim;
  int32_t rounds;
  int64_t n[RSFT_MAX_DIMS];
  int64_t b[RSFT_MAX_DIMS];
  const int64_t* sigma;
  uint64_t seed;
  double window_atten_db;
  double flat_atten_db;
  double pfa;
  int32_t mu;
  int32_t noise_mode;
  double noise_var;
  int32_t dtype;
  int32_t max_detections;
  int64_t max_batch;
  int32_t segments;
  int32_t reserved0;
  double stage1_pfa;
} rsft_params;

/*
 * One detected grid cell.
 * frame      index of the frame in the batch.
 * idx[d]     grid cell per dimension (row-major order defines sorting).
 * votes      abar_i, the number of rounds whose bucket was flagged (>= mu).
 * is_peak    1 when the cell's gain-corrected magnitude is a local maximum
 *            over its 3^D - 1 circular neighbours (ties go to the lower
 *            row-major index), else 0.
 * magnitude  gain-corrected magnitude: median over the estimation rounds of
 *            |fhat_s[M(i, sigma_s)]| divided by the flat-window response,
 *            an estimate of |DFT(W r)| at the cell (FP32).
 * freq[d]    off-grid frequency estimate in cycles/sample, in [0, 1):
 *            (idx[d] + offset)/N_d, offset = vertex of a parabola through the
 *            log magnitudes of the cell and its two neighbours along d,
 *            clamped to [-1/2, 1/2] (FP64).
 */
typedef struct {
  int64_t frame;
  int64_t idx[RSFT_MAX_DIMS];
  int32_t votes;
  int32_t is_peak;
  float magnitude;
  float reserved;
  double freq[RSFT_MAX_DIMS];
} rsft_detection;

/* Derived per-frame quantities (host FP64), for reproducibility and tests. */
typedef struct {
  int32_t ndim, rounds, mu, noise_mode;
  int64_t n[RSFT_MAX_DIMS], b[RSFT_MAX_DIMS];
  int64_t sigma[RSFT_MAX_ROUNDS][RSFT_MAX_DIMS];
  int64_t sigma_inv[RSFT_MAX_ROUNDS][RSFT_MAX_DIMS]; /* eq. mod_inv */
  int64_t tau[RSFT_MAX_ROUNDS][RSFT_MAX_DIMS];       /* sigma_inv mod B_d */
  double beta[RSFT_MAX_ROUNDS];                      /* eq. alpha_beta */
  double gamma[RSFT_MAX_ROUNDS];                     /* KNOWN-mode thresholds */
  double p1;                                         /* first-stage Pfa per round */
  double eta_m;              /* product over d of the window's 6-dB width (bins) */
  double max_sparsity;       /* B / eta_m: by Remark 2 (Sec. IV-C) RSFT fails for
                                K >= this many tones, whatever their SNR */
  uint64_t estimation_rounds; /* bit s set: round s feeds magnitude estimates */
  /* plan-wide launch shapes (see rsft_autotune) */
  int32_t fold_threads;      /* fold: work-group size */
  int32_t fold_vec;          /* fold: complex samples per thread per row */
  int32_t fold_nontemporal;  /* fold: 1 = non-temporal input loads */
  int32_t estimate_workers;  /* compact/estimate: 1 = overflow workers */
  int32_t vote_kernel;       /* 0 per cell, 1 candidate rows, 2 32-cell masks, 3 word-parallel masks */
  int32_t dft_two_pass;      /* 1: the DFT runs in two passes (RSFT_OPT_DFT_SPLIT) */
  int32_t dft_threads;       /* work-group size of the one-work-group DFT (RSFT_OPT_DFT_THREADS) */
} rsft_plan_info_t;

typedef struct rsft_plan_s* rsft_plan_t;

/*
 * Create a plan on the current HIP device. `frames` holds nframes frame
 * descriptors (host memory, copied).
 *   nframes == 1: uniform batch; every execute processes `batch` frames
 *                 (1..max_batch) of that shape packed back to back, all
 *                 sharing one sigma set.
 *   nframes  > 1: uneven batch; execute's batch must equal nframes and the
 *                 frames are packed back to back in descriptor order (each
 *                 frame occupies prod N_d elements). Shapes, sigma, windows
 *                 and Pfa may differ per frame; rounds, mu and dtype may not.
 * Builds the windows, permuted weight tables, thresholds and DFT tables on
 * the host in FP64 and uploads them (one blocking copy). Launch shapes
 * start from the defaults, or from the choices of an earlier rsft_autotune
 * in this process on a plan of the same signature (see rsft_autotune).
 * *out is set to NULL on failure. Errors: INVALID_ARGUMENT, NOT_POW2, BAD_SIGMA, UNSUPPORTED
 * (B_d > 128 in some dimension, B > 16384 buckets per frame, N_d > 2^30,
 * N >= 2^40), OUT_OF_MEMORY, DEVICE.
 */
rsft_status rsft_plan(const rsft_params* frames, int64_t nframes, rsft_plan_t* out);

/*
 * Enqueue the whole hot path for `batch` frames on `stream` and return
 * (asynchronous). d_input: device pointer to the frames (dtype of the plan),
 * owned by the caller, which keeps it alive and unmodified until the stream
 * has passed this work. Results stay in the plan until the next execute.
 * batch == 0 is a no-op. Errors: INVALID_ARGUMENT (batch out of range,
 * NULL input with batch > 0), DEVICE.
 */
rsft_status rsft_execute(rsft_plan_t plan, const void* d_input, int64_t batch,
                         void* stream);

/*
 * rsft_execute in two halves, for pipelining batches over several plans.
 * rsft_execute_fold enqueues the fold stage on `stream` (window,
 * permutation, flat window and aliasing of Algorithm 1, the only stage that
 * reads d_input; same arguments as rsft_execute); rsft_execute_tail enqueues
 * the rest for the batch last folded on this plan (B-point DFT and
 * first-stage threshold, vote of Def. 3-4 and eq. a_i, compaction and
 * estimates). A fold followed by its tail gives exactly what rsft_execute
 * gives, and the detection and bucket calls then refer to that batch. The
 * fold is bound by HBM bandwidth and the rest mostly by instruction issue
 * and latency, so with two plans the fold of one batch can run beside the
 * tail of the previous batch on the other plan. The caller orders the
 * streams with events: a plan's tail after its own fold, and a plan's next
 * fold after its own previous tail (the fold overwrites what the tail
 * reads). Graph replay (RSFT_OPT_GRAPH) applies to each half separately;
 * with RSFT_OPT_TIMING set the halves launch eagerly and record no stage
 * times. Errors: as rsft_execute; NOT_READY from rsft_execute_tail without
 * a preceding rsft_execute_fold on the plan (rsft_execute in between
 * cancels a pending fold).
 */
rsft_status rsft_execute_fold(rsft_plan_t plan, const void* d_input, int64_t batch, void* stream);
rsft_status rsft_execute_tail(rsft_plan_t plan, void* stream);

/*
 * Choose the plan's launch shapes by timing them on d_input (same contract
 * as rsft_execute) with hipEvents on `stream`, `repeats` runs each (<= 0: 5):
 * - fold stage (the HBM-bound stage): work-group size (256 / 512 threads),
 *   samples per thread (4 / 2), ordinary vs non-temporal input loads, each
 *   timed in two passes; the fastest is kept and *best_ms (may be NULL)
 *   gets its average duration in its faster pass;
 * - DFT: one work-group per transform at each work-group size
 *   (RSFT_OPT_DFT_THREADS) and, where it applies, the two passes
 *   (RSFT_OPT_DFT_SPLIT); the fastest kept;
 * - vote, where both kernels apply (RSFT_OPT_VOTE_WORDS): word-parallel
 *   masks or the enumeration of candidate cells, the faster kept;
 * - compact/estimate: without or with overflow workers (the records of
 *   chunks holding more than 1024 detections shared among extra work-
 *   groups); the workers are kept when at least 3% faster. How dense the
 *   detections are depends on the data, hence timing on the caller's input.
 * The choices are reported by rsft_plan_info and leave the results
 * unchanged (bit for bit for the vote and the estimate layout). They are
 * also kept for the life of the process under the plan's signature (device,
 * batch capacity, rounds, mu, dtype, segment mode, and every frame's shape,
 * buckets and noise mode): rsft_plan starts a later plan of the same
 * signature from them (thread-safe; RSFT_OPT_* settings made after
 * rsft_plan override them as usual). Synchronizes the stream;
 * afterwards the plan holds the results of an execute of d_input (a
 * pending rsft_execute_fold is cancelled, as by rsft_execute).
 * Errors: as rsft_execute.
 */
rsft_status rsft_autotune(rsft_plan_t plan, const void* d_input, int64_t batch, void* stream,
                          int32_t repeats, double* best_ms);

/*
 * The same detections computed the plain way, as a comparator: for each
 * frame and each round separately, gather the permuted samples, window,
 * alias and DFT, then threshold (Algorithm 1 literally: T passes over the
 * frame, one launch chain per frame), then the frame's reverse mapping and
 * second stage (Def. 3-4, eq. a_i; the plan's vote kernel, one launch per
 * frame); the estimates of the whole batch follow as in rsft_execute. Same
 * arguments and results as rsft_execute; much slower.
 */
rsft_status rsft_execute_per_frame(rsft_plan_t plan, const void* d_input,
                                   int64_t batch, void* stream);

/*
 * Synchronize `stream` and copy the detections of the last execute to the
 * host: the output o of Algorithm 1, the cells whose accumulated votes pass
 * the second-stage threshold (Sec. III-C.5), each with the off-grid estimate
 * described at rsft_detection. h_out: host array of `capacity` records;
 * receives the records sorted
 * by (frame, row-major cell index). h_counts: host array with one entry per
 * frame of the last execute (may be NULL); receives the exact number of
 * detections of each frame, including any beyond the per-frame
 * max_detections. n_written (may be NULL) receives the number of records
 * written to h_out. A frame with more than max_detections detections keeps
 * its first max_detections in row-major order. Returns RSFT_ERROR_CAPACITY
 * when records were dropped (h_out too small, or a frame over its
 * max_detections). Errors: NOT_READY, INVALID_ARGUMENT, DEVICE.
 */
rsft_status rsft_detect(rsft_plan_t plan, void* stream, rsft_detection* h_out,
                        int64_t capacity, int64_t* h_counts, int64_t* n_written);

/* Total number of detections of the last execute (synchronizes). */
rsft_status rsft_detection_count(rsft_plan_t plan, void* stream, int64_t* total);

/*
 * Copy the buckets fhat_s of the last execute (eq. f; bucket j in the
 * paper's indexing, i.e. after the permutation) to d_out, a device buffer of
 * complex64: for each frame in batch order, [T][B_0]...[B_{D-1}]. Async on
 * `stream`. Size: sum over frames of T*B*8 bytes.
 */
rsft_status rsft_get_buckets(rsft_plan_t plan, void* d_out, void* stream);

/*
 * Copy the first-stage flags c_s of the last execute to d_out (device,
 * uint32): c_s[j] = 1 when |fhat_s[j]|^2 >= gamma_s, the Neyman-Pearson test
 * of each bucket with the per-round threshold of eq. tpd (first stage,
 * Sec. IV-B). For each frame, [T][ceil(B/32)] words; bucket j (row-major
 * flattened) is bit (j % 32) of word j / 32. Async on `stream`.
 */
rsft_status rsft_get_flags(rsft_plan_t plan, uint32_t* d_out, void* stream);

/*
 * Replace the flags of the last execute by d_flags (device, layout of
 * rsft_get_flags) and redo the reverse mapping and accumulation
 * abar_i = sum_s c_s[M(i, sigma_s)] (Def. 3-4, eq. a_i), the second-stage
 * detection abar_i >= mu (Sec. III-C.5) and the estimates from them
 * (buckets unchanged). Lets a caller check the voting stage against known
 * flags. Async on `stream`.
 */
rsft_status rsft_vote_flags(rsft_plan_t plan, const uint32_t* d_flags, void* stream);

/*
 * Bucketized forward model of K complex tones per frame, for off-grid
 * refinement. The round-s buckets of eq. f are linear in the signal, and for
 * a tone b exp(j 2 pi f . m) with continuous frequency f (cycles/sample per
 * dimension; the tone v(omega) of eq. f_k) they factor per dimension:
 *   model_s[k] = sum_t b_t prod_d G_{s,d}(f_{t,d})[k_d],
 *   G_{s,d}(f)[k] = sum_n wbar_d[n] w_d[m] exp(j 2 pi f m) exp(-2 pi i k n / B_d),
 *   m = [sigma_{s,d} n]_{N_d}
 * (window W, permutation P_{sigma,0} of Def. 1, flat window, aliasing of
 * Def. 2 and the B-point DFT, with this plan's windows and sigma). The phase
 * f m is reduced modulo 1 exactly (64-bit fixed point); sums are FP32.
 *
 * All descriptors of the plan must have the same D. batch: as rsft_execute
 * (uniform plan: 1..max_batch; uneven plan: its frame count). tones K >= 1
 * (pad with zero amplitudes when frames have fewer).
 *   d_freqs  device double [batch][K][D], cycles/sample (any real value;
 *            only frac(f) matters)
 *   d_amps   device complex64 [batch][K]
 *   d_model  device complex64, the layout of rsft_get_buckets
 *   d_workspace  device buffer of rsft_model_workspace_size bytes; the
 *            forward call stores the per-dimension factors there and the
 *            backward call reads them (same plan, batch, K and frequencies)
 * Errors: INVALID_ARGUMENT (NULL, bad batch or K), UNSUPPORTED (mixed D, or
 * a segment-mode plan), DEVICE. Async on `stream`.
 */
rsft_status rsft_model_workspace_size(rsft_plan_t plan, int64_t batch, int32_t tones,
                                      int64_t* bytes);
rsft_status rsft_model_forward(rsft_plan_t plan, const double* d_freqs, const void* d_amps,
                               int64_t batch, int32_t tones, void* d_model, void* d_workspace,
                               void* stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rsft_model_forward without a workspace. The per-dimension factors go to
 * a static device array of the library instead, RSFT_STATIC_SCRATCH_BYTES
 * bytes on each GPU the library runs on, held until the process ends. The
 * call allocates nothing; the caller passes inputs and outputs as for
 * rsft_model_forward (d_model receives the same values) and the plan's
 * device must be the current device. Every call on a GPU shares that GPU's
 * array and overwrites it (it holds the last call's factors, usable by no
 * other call), so calls that overlap on one GPU race: issue them on one
 * stream, or order them. Errors: as rsft_model_forward; UNSUPPORTED when
 * the factors, 2 * batch * T * tones * (sum_d B_d) * 8 bytes, exceed the
 * array; INVALID_ARGUMENT when the current device is not the plan's.
 */
#define RSFT_STATIC_SCRATCH_BYTES (8 << 20)
rsft_status rsft_model_forward_noalloc(rsft_plan_t plan, const double* d_freqs, const void* d_amps,
                                       int64_t batch, int32_t tones, void* d_model, void* stream);

/*
 * Gradients of a real loss through the model, given the output gradient
 * d_grad_model = dL/dRe(model) + j dL/dIm(model) (layout of d_model):
 *   d_grad_amps[f][t]     = sum_{s,k} grad_s[k] conj(prod_d G_{s,d}(f_t)[k_d])
 *                           (= dL/dRe b_t + j dL/dIm b_t), complex64
 *   d_grad_freqs[f][t][d] = Re(b_t sum_{s,k} conj(grad_s[k]) dG_{s,d}/df [k_d]
 *                              prod_{e != d} G_{s,e}[k_e]) = dL/df_{t,d}, double
 * and, when d_step_freqs / d_step_amps are not NULL (both or neither), each
 * tone's Gauss-Newton step for the least-squares loss sum |model - observed|^2
 * (pass d_grad_model = 2 (model - observed)): x solving H x = -g/2 with
 * H = Re(J^H J), J = [P, jP, b_t dP/df_0, ...], P = prod_d G_d, over the
 * tone's own parameters (Re b_t, Im b_t, f_t); tones are treated as
 * decoupled (block-diagonal H), H is solved in FP64 with 1e-6 Levenberg
 * damping, a vanishing pivot leaves that parameter unchanged, and each
 * frequency step is clipped to a quarter bin (1/(4 N_d)), a trust region.
 * d_step_freqs: double [batch][K][D]; d_step_amps: complex64 [batch][K].
 * d_workspace must hold the factors of the matching forward call.
 * Async on `stream`.
 */
rsft_status rsft_model_backward(rsft_plan_t plan, const void* d_amps, int64_t batch,
                                int32_t tones, const void* d_grad_model, double* d_grad_freqs,
                                void* d_grad_amps, double* d_step_freqs, void* d_step_amps,
                                const void* d_workspace, void* stream);

/*
 * Off-grid refinement of K tones per frame against observed buckets
 * (Sec. I cites gradient refinement of sparse-FFT estimates; here the
 * bucketized model of rsft_model_forward is fitted to the round buckets of
 * eq. f by least squares, loss = sum_{s,k} |model_s[k] - observed_s[k]|^2).
 *
 * d_observed   device complex64 in the layout of rsft_get_buckets, or NULL
 *              for the plan's own buckets of the last execute (which must
 *              have processed `batch` frames; else NOT_READY).
 * d_workspace  device buffer of rsft_refine_workspace_size bytes (both calls
 *              below; contents are scratch).
 *
 * rsft_initial_amplitudes: the starting amplitude of each tone from the
 * buckets its nearest cell falls in (cell_d = floor(f_d N_d + 1/2) mod N_d):
 * in every estimation round (rsft_plan_info_t.estimation_rounds) the
 * observed bucket y_s[M(cell, sigma_s)] (Def. 3) divided by the model of a
 * unit tone at f in that bucket (the window, permutation, flat window,
 * aliasing and DFT response; Sec. III-C divides bucket values by the window
 * spectrum); of these ratios, the one whose magnitude is the median over the
 * rounds (rank floor((n-1)/2) ascending, the earlier round on ties), so that
 * a round where another tone shares the bucket is outvoted. d_freqs: double
 * [batch][K][D] (e.g. the freq of detected peaks); d_amps: complex64
 * [batch][K] (output); d_spread (may be NULL): float [batch][K], the
 * largest deviation of a round's ratio from the chosen one relative to it,
 * max_s |a_s - a| / |a| (infinity for a = 0): small for a single tone, of
 * order one for a peak made of different tones' energy in different rounds
 * (the ambiguity of Remark 1), which a caller can drop before refining.
 *
 * rsft_refine: `steps` iterations in place on d_freqs / d_amps, all on the
 * device. d_tone_counts (device int32 [batch], or NULL for K everywhere):
 * only the first counts[f] tones of frame f take part; the others are left
 * unchanged and are not part of the model (a way to give frames different
 * tone counts). An iteration first evaluates each frame's loss: when it is
 * above the lowest loss of that frame so far (decoupled steps of tones that
 * share buckets can overshoot together), the frame's lowest-loss state is
 * restored, its trust radii halve and it takes no step this iteration.
 * Otherwise every active tone, against the same residual r = model -
 * observed (tones decoupled), takes its Gauss-Newton step over (Re b,
 * Im b, f) (as rsft_model_backward), its frequency step clipped to the
 * tone's trust radius (starting at trust_bins bins per dimension); the
 * amplitude is re-solved for the new frequency f' by least squares against
 * the residual without the tone; the step is kept when it lowers the tone's
 * own loss (others fixed), and the radius doubles (at most trust_bins);
 * else the frequency stays, the amplitude becomes the least-squares one at
 * f and the radius halves. The same loss check ends the last iteration, so
 * the result is each frame's lowest-loss state. d_loss (may be NULL):
 * double [steps + 1][batch], each frame's lowest loss so far at the start of
 * every iteration and at the end (non-increasing), in FP64.
 * Frequencies are FP64 throughout; sums are FP32 with FP64 reductions.
 * Errors: as rsft_model_forward; INVALID_ARGUMENT (steps outside 0..100000,
 * trust_bins <= 0); NOT_READY. Async on `stream`.
 */
rsft_status rsft_refine_workspace_size(rsft_plan_t plan, int64_t batch, int32_t tones, int64_t* bytes);
rsft_status rsft_initial_amplitudes(rsft_plan_t plan, const void* d_observed, const double* d_freqs,
                                    int64_t batch, int32_t tones, void* d_amps, float* d_spread,
                                    void* d_workspace, void* stream);
rsft_status rsft_refine(rsft_plan_t plan, const void* d_observed, double* d_freqs, void* d_amps,
                        int64_t batch, int32_t tones, const int32_t* d_tone_counts, int32_t steps,
                        double trust_bins, void* d_workspace, double* d_loss, void* stream);

/*
 * Residual of observed buckets after the model of K tones per frame:
 *   d_residual_s[k] = observed_s[k] - sum_{t < counts[f]} b_t prod_d G_{s,d}(f_t)[k_d]
 * (the model of rsft_model_forward; eq. f is linear in the signal, so the
 * residual is the round buckets of what the tones do not explain). For
 * finding tones that share a bucket with a stronger one in some round: the
 * amplitudes and spreads of rsft_initial_amplitudes taken on the residual
 * of the tones already found (pass d_residual as its d_observed).
 * d_observed: as rsft_refine (NULL: the plan's buckets of the last
 * execute); d_tone_counts: as rsft_refine (NULL: all K); d_residual:
 * device complex64 in the layout of rsft_get_buckets (may not alias
 * d_observed); d_workspace: rsft_model_workspace_size bytes. Errors: as
 * rsft_model_forward; NOT_READY. Async on `stream`.
 */
rsft_status rsft_model_residual(rsft_plan_t plan, const void* d_observed, const double* d_freqs,
                                const void* d_amps, int64_t batch, int32_t tones,
                                const int32_t* d_tone_counts, void* d_residual, void* d_workspace,
                                void* stream);

/* Per-frame derived parameters; frame indexes the descriptors of rsft_plan. */
rsft_status rsft_plan_info(rsft_plan_t plan, int64_t frame, rsft_plan_info_t* out);

/* Options (rsft_set_option). */
enum {
  RSFT_OPT_GRAPH = 0,  /* 1: replay the launch sequence as a captured hipGraph
                          (cached per input pointer and batch); 0: launch
                          kernels one by one. Default 1. */
  RSFT_OPT_TIMING = 1, /* 1: record hipEvents around each stage in eager mode
                          and accumulate their durations (forces GRAPH=0
                          while set). Default 0. */
  /* launch shape of the fold stage (what rsft_autotune chooses):
     work-group size 256 | 512; samples per thread 2 | 4; non-temporal
     input loads 0 | 1 */
  RSFT_OPT_FOLD_THREADS = 2,
  RSFT_OPT_FOLD_VEC = 3,
  RSFT_OPT_FOLD_NONTEMPORAL = 4,
  /* compact/estimate layout (what rsft_autotune chooses): 0 = one work-group
     per compaction chunk builds all of its records; 1 = it builds the first
     1024 and overflow workers the rest. Same records either way. Default 0. */
  RSFT_OPT_ESTIMATE_WORKERS = 5,
  /* vote kernel for plans whose frames all have rows (last dimension) of
     128..4096 cells and B_last * N_last / 32 <= 16384: 1 = word-parallel
     masks (default: per frame and round the cell mask of each bucket row,
     then T mask words gathered per 32 cells; the plan holds T (B / B_last)
     N_last / 32 words per frame for the masks), 0 = enumeration of the
     candidate cells of flagged buckets (T <= 4; larger T keeps the masks).
     Same detections either way. */
  RSFT_OPT_VOTE_WORDS = 6,
  /* DFT stage for plans whose frames all have D >= 2, B / B_0 <= 4096 and
     the KNOWN noise floor: 1 = two passes over many small work-groups (the
     trailing dimensions per group of index-0 slabs, then dimension 0 per
     group of output columns with the threshold), 0 = one work-group per
     (round, frame). Same results (to FP32 rounding). Default 1; chosen by
     rsft_autotune. */
  RSFT_OPT_DFT_SPLIT = 7,
  /* work-group size of the one-work-group-per-(round, frame) DFT: 64, 256
     or 1024 threads (one wave suits many small transforms, sixteen a few
     large ones). Default by the plan's largest B: 64 up to 256 buckets,
     256 up to 1024, else 1024; chosen by rsft_autotune. Same results. */
  RSFT_OPT_DFT_THREADS = 8
};
rsft_status rsft_set_option(rsft_plan_t plan, int32_t option, int64_t value);

/* Stages reported by rsft_stage_times. */
enum {
  RSFT_STAGE_FOLD = 0,    /* window + permutation + flat window + aliasing */
  RSFT_STAGE_DFT = 1,     /* B-point N-D DFT + |.|^2 + first-stage detection */
  RSFT_STAGE_VOTE = 2,    /* reverse mapping + accumulation + second stage */
  RSFT_STAGE_ESTIMATE = 3, /* sort + off-grid estimates + record output */
  RSFT_NUM_STAGES = 4
};
/*
 * Average device duration (ms) of each stage over the executes made with
 * RSFT_OPT_TIMING on since the last reset (synchronizes the events). avg_ms:
 * host array of RSFT_NUM_STAGES; count: number of executes averaged.
 * reset != 0 clears the accumulators after reading.
 */
rsft_status rsft_stage_times(rsft_plan_t plan, double* avg_ms, int64_t* count,
                             int32_t reset);

/* Free the plan and everything it owns. NULL is ignored. */
void rsft_destroy(rsft_plan_t plan);

const char* rsft_status_string(rsft_status status);
const char* rsft_last_error(void);

/* ---- Host-only design functions (no device work; usable without a GPU) ---- */

/* Dolph-Chebyshev window of length n (>= 1) with sidelobes atten_db (>= 0)
 * below the main lobe, scaled so out[n/2] = 1 (Sec. III-C.1, Fig. 2).
 * periodic != 0: the DFT-even variant (length n+1 symmetric, last sample
 * dropped). atten_db = 0: all ones. out: host array of n doubles. */
rsft_status rsft_chebyshev_window(int64_t n, double atten_db, int32_t periodic,
                                  double* out);

/* Flat window of length n for b buckets (Sec. IV-B), complex:
 * out[2m] + j out[2m+1] = c0[m] * sum_{k=-(L-1)}^{0} exp(j 2 pi k m / n),
 * L = n/b, c0 = periodic Chebyshev at atten_db (0: rectangular) rotated so
 * its peak is at m = 0 and scaled to c0[0] = 1. out: host array of 2n. */
rsft_status rsft_flat_window(int64_t n, int64_t b, double atten_db, double* out);

/* sigma^{-1} mod n (eq. mod_inv). BAD_SIGMA if not invertible. */
rsft_status rsft_mod_inverse(int64_t sigma, int64_t n, int64_t* out);

/* p1 with P[Binomial(T, p1) >= mu] = pfa (FP64 bisection). */
rsft_status rsft_stage1_probability(double pfa, int32_t rounds, int32_t mu,
                                    double* out);

/* The permutation factors a NULL-sigma plan would draw: out[s*ndim + d]. */
rsft_status rsft_draw_sigma(uint64_t seed, int32_t rounds, int32_t ndim,
                            const int64_t* n, int64_t* out);

/*
 * Optimal threshold design (eq. opt, Sec. IV-C): the smallest SNR of the
 * weakest tone for which the two-stage detector reaches (pd, pfa), with the
 * first-stage probabilities of eq. bpd and the asymptotic Normal laws of the
 * vote count (Claims 2 and 3, variance upper bounds):
 *   H1: mean T Pd_bar, variance T Pd_bar (1 - Pd_bar)
 *   H0: mean F eta_p Pd_bar + (T - F) Pfa_bar, variance
 *       F eta_p Pd_bar (1 - eta_p Pd_bar) + (T - F) Pfa_bar (1 - Pfa_bar),
 *   F = T K eta_m / B;
 * mu is enumerated over 1..T (a cell is declared at >= mu votes); for each,
 * the two tails fix Pd_bar and Pfa_bar, eq. bpd gives
 *   SNR = beta_bar (ln Pfa_bar / ln Pd_bar - 1) / alpha_bar,
 * and the minimum over mu is SNR*_min at mu*. alpha_bar and beta_bar are the
 * averages of alpha(p, sigma, omega) and beta(sigma) (eq. alpha_beta, p the
 * bucket of Claim 1) over all odd sigma of each dimension, multiplied over
 * dimensions (independent permutations per dimension). FP64, host only.
 *
 * in:  ndim, rounds T, n[d], b[d] (as rsft_params); window_atten_db,
 *      flat_atten_db (< 0: same as the window); omega_bins[d], the frequency
 *      of the weakest tone in bins; sparsity K; eta_m (6-dB width of the
 *      pre-window in bins, product over dimensions; <= 0: measured from the
 *      window); pd, pfa: targets after the second stage; upper_bound: 0 for
 *      eta_p = 1, 1 for eta_p = 1 / Pd_bar (the bounds of Remark 3);
 *      noise_var sigma_n^2 (> 0).
 * out: feasible (0 when no mu meets both targets, e.g. K eta_m >= B,
 *      Remark 2; the other fields are then 0), mu*, SNR*_min (linear and
 *      dB), Pd_bar, Pfa_bar (pass it as rsft_params.stage1_pfa, and mu* as
 *      rsft_params.mu, to run the design), gamma* = -noise_var beta_bar
 *      ln Pfa_bar, alpha_bar, beta_bar, F, eta_p, eta_m used.
 */
typedef struct {
  int32_t ndim;
  int32_t rounds;
  int64_t n[RSFT_MAX_DIMS];
  int64_t b[RSFT_MAX_DIMS];
  double window_atten_db;
  double flat_atten_db;
  double omega_bins[RSFT_MAX_DIMS];
  double sparsity;
  double eta_m;
  double pd;
  double pfa;
  int32_t upper_bound;
  int32_t reserved;
  double noise_var;
} rsft_design_params;

typedef struct {
  int32_t feasible;
  int32_t mu;
  double snr_min;
  double snr_min_db;
  double pd_bar;
  double pfa_bar;
  double gamma;
  double alpha_bar;
  double beta_bar;
  double F;
  double eta_p;
  double eta_m;
} rsft_design_result;

rsft_status rsft_design_thresholds(const rsft_design_params* in, rsft_design_result* out);

#ifdef __cplusplus
}
#endif

#endif /* RSFT_H */

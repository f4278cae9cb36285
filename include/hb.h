/* hb.h — C ABI of the batched neural-heuristic search library for MI355X (gfx950).
 *
 * The library implements the data-parallel hot path of parallel cost-bounded
 * depth-first search (CB-DFS) with a neural heuristic, as described in
 * "A Parallel CPU-GPU Framework for Batching Heuristic Operations in
 * Depth-First Heuristic Search" (Futuhi & Sturtevant): CPU search threads park
 * the states they generate in shared batches; a batch thread copies each batch
 * to the GPU, evaluates the network h_M on it with hand-written HIP kernels and
 * hands the heuristic values back (section "SingleGPU Batch CB-DFS").
 *
 * Conventions for every entry point:
 *  - Every call returns hb_status (0 = HB_OK, negative = error) and never
 *    throws across the ABI.  On error, hb_last_error() describes the cause.
 *  - Sizes are int64_t element counts; n == 0 is valid and does nothing.
 *  - "Host" pointers are ordinary CPU memory; "device" pointers are GPU memory
 *    (for example a torch tensor's data_ptr()).  The caller owns every buffer
 *    it passes in, unless stated otherwise.
 *  - Streams are hipStream_t passed as void*; NULL means the default stream.
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status */
typedef enum {
    HB_OK = 0,
    HB_E_INVAL = -1,        /* bad argument or invalid state */
    HB_E_NOMEM = -2,        /* host or device allocation failed */
    HB_E_DEVICE = -3,       /* a HIP call or kernel launch failed */
    HB_E_UNSUPPORTED = -4,  /* valid request that the library does not support */
    HB_E_BUDGET = -5,       /* node or time limit reached; statistics are valid */
    HB_E_NOSOLUTION = -6    /* the search space holds no solution */
} hb_status;

/* Description of the last error raised on the calling thread.  Valid until the
 * thread's next hb_* call.  Never NULL. */
const char* hb_last_error(void);

/* ------------------------------------------------------------- domains */
/* The paper's two domains (Experimental Setup) plus the 8-puzzle.
 * Unit edge costs (the problem tuple {G, s, g, c, h} of the Background
 * section with c = 1).
 *  HB_STP3 / HB_STP4: n x n sliding tile.  State = n*n bytes, byte p = tile at
 *    cell p (row-major), 0 = blank.  Goal: tile p at cell p.  Moves move the
 *    blank: 0 up, 1 left, 2 right, 3 down; a move never undoes the previous one
 *    (path information that stops the search returning to the parent).
 *  HB_RUBIK3: 3x3x3 cube, 54 stickers, sticker p = 9*f + 3*r + c on face
 *    f in (U, D, L, R, F, B); byte p = colour 0..5 (the face index of the
 *    colour's home face).  Face frames (x: L->R, y: D->U, z: B->F): row r and
 *    column c of face f run along v and u with U (u=+x, v=+z), D (+x, -z),
 *    L (+z, -y), R (-z, -y), F (+x, -y), B (-x, -y).  Move m turns face m/3
 *    clockwise (seen from outside), counter-clockwise or by a half turn for
 *    m%3 = 0, 1, 2.  Canonical pruning: never the same face twice in a row and
 *    never U, L or F directly after D, R or B.                               */
typedef enum { HB_STP3 = 0, HB_STP4 = 1, HB_RUBIK3 = 2 } hb_domain;

int hb_state_bytes(hb_domain d);   /* 9, 16, 54; -1 for an unknown domain */
int hb_packed_bytes(hb_domain d);  /* 8, 8, 24;  -1 for an unknown domain */

/* TensorRepresentation of a state (Subtree expansion algorithm): the packed
 * record that is parked in a batch and decoded on the GPU into the one-hot
 * network input.  Sliding tile: 4 bits per cell, cell p in bits 4p..4p+3 of one
 * little-endian uint64.  Cube: the 48 non-centre stickers in increasing index
 * order, 3 bits each, sticker q in bits 3*(q%16) of uint64 word q/16 (3 words).
 * states: host, n * hb_state_bytes; packed_out: host, n * hb_packed_bytes.
 * Each state is validated (a permutation of the tiles / nine stickers of each
 * colour with the centres in place); the first bad index is reported through
 * HB_E_INVAL and hb_last_error, and nothing after it is written. */
hb_status hb_encode(hb_domain d, const uint8_t* states, int64_t n, uint8_t* packed_out);
/* Inverse of hb_encode (host buffers). */
hb_status hb_decode(hb_domain d, const uint8_t* packed, int64_t n, uint8_t* states_out);

/* env.ApplyAction of the subtree-expansion algorithm, for building inputs:
 * applies rows of `len` moves (a negative move ends a row) to the goal state.
 * moves: host int8 [count][len]; states_out: host [count][hb_state_bytes].
 * HB_E_INVAL if a move is out of range or pushes the blank off the board. */
hb_status hb_apply_moves(hb_domain d, const int8_t* moves, int64_t count, int32_t len, uint8_t* states_out);

/* Manhattan distance of sliding-tile states (host in, host int32 out). */
hb_status hb_manhattan(hb_domain d, const uint8_t* states, int64_t n, int32_t* out);

/* ---------------------------------------------------- pattern databases */
/* Corner pattern database of the cube (the paper's classic heuristic for the
 * cube is an 8-corner PDB, Experimental Setup): the breadth-first distance of
 * the placement and twist of the first k corner cubies, 1 <= k <= 8.  Built on
 * the host with `threads` threads (<= 0: all cores).  Owned by the library. */
typedef struct hb_pdb hb_pdb;
hb_status hb_pdb_build_corner(int k, int threads, hb_pdb** out);
/* Additive pattern database of the 15-puzzle (the paper's classic sliding-tile
 * heuristic is the sum of the 1-7 and 8-15 tile PDBs, Experimental Setup):
 * group_of_tile[t] (host int32 [16]; t = 1..15, entry 0 ignored) puts tile t
 * into one of n disjoint groups 0..n-1 of 1..8 tiles.  Group g's table holds,
 * for every placement of its tiles, the fewest moves of those tiles that bring
 * them to their goal cells when the other tiles move for free, minimised over
 * the blank's cell; h(s) = sum over the groups (admissible and of the
 * Manhattan distance's parity).  Host memory while building the largest group
 * of k tiles: 16!/(16-k)! x 17 bytes (8 tiles: 8.8 GB).  HB_E_INVAL on a bad
 * grouping. */
hb_status hb_pdb_build_stp_additive(const int32_t* group_of_tile, int threads, hb_pdb** out);
/* h of n states (host in, host int32 out): cube states for a corner PDB,
 * 15-puzzle states for an additive PDB. */
hb_status hb_pdb_lookup(const hb_pdb* pdb, const uint8_t* states, int64_t n, int32_t* out); /* host */
/* Distribution of the table's values (the appendix comparing Batch IDA* with
 * AIDA* states the objective for a learned heuristic as the largest mean value
 * at bounded size; this gives the same statistic for the PDB): counts[v] = number of reachable entries equal to v for
 * v < n_counts (host int64 [n_counts], caller-owned; larger values are not
 * counted) and *max_value (nullable) = the largest value.  Indices no cube
 * state maps to are left out (for k = 8 the table indexes all 3^8 twists, of
 * which a third occur).  For an additive PDB the counts run over the entries of
 * all group tables.  HB_E_INVAL on a null pdb, n_counts < 1 or a null counts. */
hb_status hb_pdb_value_counts(const hb_pdb* pdb, int64_t* counts, int32_t n_counts, int32_t* max_value);
void hb_pdb_free(hb_pdb* pdb); /* NULL-safe */

/* --------------------------------------------------------------- model */
/* Operand precision of the matrix layers; accumulation is always FP32.
 *  HB_FP32: float32 weights and activations.
 *  HB_BF16: bfloat16 (round to nearest even) weights and activations.
 *  HB_FP8_E4M3: OCP e4m3 dense/residual weights with one FP32 scale per output
 *    column (max|W[:,n]| / 448) and e4m3 activations with one static
 *    power-of-two scale per tensor (hb_model_calibrate); layer 1 and head
 *    weights in bfloat16. */
typedef enum { HB_FP32 = 0, HB_BF16 = 1, HB_FP8_E4M3 = 2 } hb_precision;

/* Output rule applied in the kernel epilogue.
 *  Regression (one output y): v = y - offset; FLOOR: h = floor(v); ROUND:
 *  round half to even; REAL: h = floor(v) and raw_out = v.  h is clamped at 0
 *  and, with combine_md, replaced by min(h, MD) (1) or max(h, MD) (2), MD the
 *  Manhattan distance of the state.
 *  Classifier (n_out classes): QUANTILE: the smallest class whose cumulative
 *  softmax probability is >= q (the last class if none); ARGMAX: the highest
 *  logit, lowest index on ties.  Softmax, sums and comparisons in FP32.
 *  A non-finite network output yields h = Manhattan distance with combine_md,
 *  else 0. */
typedef enum {
    HB_OUT_REG_FLOOR = 0, HB_OUT_REG_ROUND = 1, HB_OUT_REG_REAL = 2,
    HB_OUT_CLS_QUANTILE = 3, HB_OUT_CLS_ARGMAX = 4
} hb_out_mode;

typedef struct {
    hb_precision prec;
    int device;          /* HIP device ordinal */
    hb_out_mode out;
    float q;             /* classifier quantile, e.g. 0.99 */
    float offset;        /* regression offset, e.g. 2.2 */
    int combine_md;      /* sliding tile: 1 h = min(h, Manhattan) (guard for untrained nets);
                            2 h = max(h, Manhattan) (learned heuristic with Manhattan fallback);
                            3 h = Manhattan + h (Manhattan distance plus a learned non-negative residual) */
    int max_batch;       /* largest n per launch; larger calls are split (0: 16384) */
} hb_model_opts;

typedef struct hb_model hb_model;

/* Load a weight file and upload it to `device`.
 * File (little-endian): u32 magic "HBW1", u32 version 1, u32 domain, u32 n_in,
 * u32 n_dense, u32 dims[n_dense], u32 n_res, u32 n_out, u32 head_kind (0
 * regression, 1 classifier), then float32 tensors: for each dense layer W
 * [in][out] row-major and b[out]; for each residual block W_a, b_a, W_b, b_b;
 * then the head W, b.  Layer 1 is the one-hot layer (n_in = cells * symbols,
 * input index p*S + s[p]); every hidden layer is followed by ReLU; a residual
 * block computes x <- ReLU(x + W_b ReLU(W_a x + b_a) + b_b).
 * opts NULL = {FP32, device 0, FLOOR, 0.99, 0, 0, 16384}. */
hb_status hb_model_load(const char* weights_path, const hb_model_opts* opts, hb_model** out);
void hb_model_free(hb_model* m); /* NULL-safe; synchronises the model's device work first */

/* Ensemble heuristics: k (1..4) regression networks with the same architecture
 * (weight files as for hb_model_load) evaluated as one model.  The related work
 * makes a learned heuristic admissible by taking the minimum over an ensemble;
 * the sliding-tile heuristic of the experiments adds learned residuals to
 * Manhattan distance.  Member outputs y_i are combined as
 * HB_ENSEMBLE_MIN: y = min_i y_i, or HB_ENSEMBLE_SUM: y = y_0 + y_1 + ... (in
 * member order), then opts' output rule applies to y (offset, floor or round,
 * combine_md; combine_md = 3 gives Manhattan plus the summed residuals).  On
 * the GPU the members' layer-1 tables sit side by side in one gather, and each
 * matrix layer is one grouped launch over all members.  The model is used
 * like any other (hb_eval_batch, cbdfs_solve, calibration, autotuning). */
typedef enum { HB_ENSEMBLE_MIN = 0, HB_ENSEMBLE_SUM = 1 } hb_ensemble_rule;
hb_status hb_model_load_ensemble(const char* const* weights_paths, int k, hb_ensemble_rule rule,
                                 const hb_model_opts* opts, hb_model** out);

typedef struct {
    int domain, n_in, n_dense, n_res, n_out, head_kind, n_act, prec;
    int dims[8];
    int64_t weight_bytes;   /* device bytes of the weights in the model's precision */
    double flops_per_eval;  /* algorithmic FLOPs per state: 2*K*N per matrix layer plus one add per gathered row element */
} hb_model_info;
hb_status hb_model_get_info(const hb_model* m, hb_model_info* out);

/* FP8 only: derive the static activation scales from a calibration batch.
 * Runs the FP32 network on d_packed (device, n packed states) and sets, per
 * stored activation tensor, the smallest power of two a with max|x| / a <= 448.
 * Synchronous.  Must be called before hb_eval_batch on an FP8 model. */
hb_status hb_model_calibrate(hb_model* m, const uint8_t* d_packed, int64_t n);
/* Read or set the activation scales (n_act floats, host). */
hb_status hb_model_get_act_scales(const hb_model* m, float* out, int cap);
hb_status hb_model_set_act_scales(hb_model* m, const float* scales, int n);

/* Batched heuristic evaluation (ProcessBatch step 2 of SingleGPU Batch CB-DFS).
 * d_packed: device, n * hb_packed_bytes (hb_encode layout).
 * d_h_out:  device int32[n], the heuristic per state.
 * d_raw_out: device float[n * n_out] or NULL: the network output (regression
 *   value minus offset, or the logits).
 * Asynchronous on `stream`; the caller keeps the buffers alive until the stream
 * is synchronised.  Calls on distinct streams may run concurrently: each
 * stream gets its own activation workspace. */
hb_status hb_eval_batch(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h_out,
                        float* d_raw_out, void* stream);

/* Layer-by-layer inspection (used by the parity tests): runs the forward pass
 * on the n packed states at d_packed (device) and copies stored activation
 * tensor `act` into d_out (device): n rows of `width` elements, row stride
 * ld_out elements, in the model's operand type (float32; bfloat16 bits as
 * uint16; e4m3 codes as uint8, value = code x the tensor's activation scale).
 * act 0 is layer 1's output, 1..n_dense-1 the dense layers' outputs, then per
 * residual block its inner activation and its output (n_act tensors in all);
 * width = the layer's output width padded to 128 (times the ensemble size).
 * Synchronous on `stream`; allocates a temporary h buffer.  HB_E_INVAL for an
 * index outside 0..n_act-1 or ld_out < width. */
hb_status hb_model_activation(hb_model* m, const uint8_t* d_packed, int64_t n, int act, void* d_out,
                              int64_t ld_out, void* stream);

/* Allocation-free variant of hb_eval_batch, for callers that cannot allocate
 * device memory: code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and results (bitwise equal
 * to hb_eval_batch's), but the two activation buffers live in a fixed 64 MiB
 * device array of the library instead of a per-stream workspace; the array
 * exists once per GPU and is held until the process ends.  The first call on a
 * device looks up that device's copy (no allocation); no call allocates.
 * Limit: ceil(n / 128) * 128 * (padded activation width summed over ensemble
 * members) * (4 FP32, 2 BF16, 1 FP8 bytes) must fit in 32 MiB, e.g. n <= 8192
 * for the 15-puzzle residual net at FP32, 16384 at BF16; a larger n returns
 * HB_E_INVAL and launches nothing.  Every call on one GPU shares the array and
 * leaves the last call's activations in it: calls that overlap in time on one
 * GPU (other streams, other threads) race and give wrong results, so the
 * caller serialises them.  FP8 models must be calibrated first. */
hb_status hb_eval_batch_noalloc(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h_out,
                                float* d_raw_out, void* stream);

/* Persistent, capture-friendly variant: the state count is read on the device
 * from *d_n (int32, 0 <= *d_n <= max_n) so one launch shape (sized for max_n)
 * serves every batch size; suitable for hipGraph capture. */
hb_status hb_eval_batch_dev_n(hb_model* m, const uint8_t* d_packed, const int32_t* d_n, int64_t max_n,
                              int32_t* d_h_out, float* d_raw_out, void* stream);

/* Select the GEMM tile shape used by later evaluations on this model:
 * 0 automatic (autotuned bucket, else a rule on the batch size);
 * 1 128x128, 2 128x256, 3 64x128, 4 256x128: LDS double buffer filled through
 *   registers, 4 waves;
 * 5 32x32: one wave per tile, operands straight from global memory (small batches);
 * 6 256x128, 7 128x128, 8 128x256 (3-stage LDS ring), 9 64x128 (4-stage ring):
 *   LDS ring filled by direct global-to-LDS loads, 4 waves;
 * 10 256x128: LDS double buffer filled through registers, 8 waves (4 x 2);
 * 11-14: the fused one-launch forward kernel, switched off in the library
 *   (HB_E_UNSUPPORTED);
 * 15 256x128 (2-stage ring), 16 256x128 (3-stage ring): LDS ring filled by
 *   direct loads, each stage's operands read whole before its MFMAs, 8 waves;
 * 17 256x128 (2-stage ring), the same with 16 waves (4 x 4, 64x32 each);
 * 18 the 15 kernel as a persistent grid of one block per compute unit, 19 the 1
 *   kernel as a persistent grid of two blocks per compute unit: a block's tiles
 *   after its first come off an atomic counter (per stream, reset by each
 *   launch's last block; no block waits on another);
 * 20 256x256 (2-stage ring), 8 waves of 64x128: a third fewer operand bytes per
 *   MFMA than 256x128, for large batches (layers whose padded width is a
 *   multiple of 256).
 * All shapes give bitwise equal results.  HB_E_INVAL outside 0..20.  See hb_model_tune. */
hb_status hb_model_set_tile(hb_model* m, int tile_id);
/* Autotuner for one batch size: times every tile shape on the n packed states
 * (device) and keeps the fastest for batches in n's power-of-two bucket
 * (floor(log2 n)).  If `report` (host) is non-NULL, up to cap/2 pairs
 * (tile id as in hb_model_set_tile, microseconds per forward pass) are written. */
hb_status hb_model_tune(hb_model* m, const uint8_t* d_packed, int64_t n, double* report, int cap);

/* One row of the autotuner's table. */
typedef struct {
    int32_t batch;       /* batch size timed */
    int32_t tile;        /* fastest tile id (hb_model_set_tile numbering) */
    double us;           /* forward pass at that tile, microseconds */
    double evals_per_s;  /* batch / us */
} hb_tune_entry;

/* Autotuner over batch sizes and tile shapes (Appendix: the batch size and
 * workNum trade-off): for every power of two b <= min(n, max_batch), and for
 * min(n, max_batch) itself, times each tile shape on the first b of the n
 * packed states (device) and keeps the fastest for b's bucket.  Writes up to
 * cap rows to `table` (host), their count to *rows, and to *recommended_batch
 * the smallest timed batch whose evaluations/s reach 90% of the best.  Runs
 * synchronously on the default stream. */
hb_status hb_model_autotune(hb_model* m, const uint8_t* d_packed, int64_t n, hb_tune_entry* table, int cap,
                            int* rows, int32_t* recommended_batch);
/* Tile the model would use for a batch of n states (hb_model_set_tile numbering). */
hb_status hb_model_tile_for(const hb_model* m, int64_t n, int* tile);
/* Tuning cache on disk (text): the device architecture, the network shape and
 * precision, then one line per bucket.  Loading checks that architecture,
 * shape and precision match this model (else HB_E_INVAL) and replaces the
 * model's bucket table. */
hb_status hb_model_save_tuning(const hb_model* m, const char* path);
hb_status hb_model_load_tuning(hb_model* m, const char* path);

/* Per-kernel timing: while enabled, every launch of this model's kernels is
 * bracketed by HIP events recorded on the stream it runs on.  Reading
 * synchronises those events and returns the sums since the last reset.
 * gemm_flops counts algorithmic work (2*K*N per row, unpadded). */
typedef struct {
    double gather_ms, gemm_ms, head_ms;
    int64_t gather_launches, gemm_launches, head_launches;
    double gemm_flops;
} hb_profile;
hb_status hb_model_profile(hb_model* m, int enable); /* enabling also resets the sums */
hb_status hb_model_profile_read(hb_model* m, hb_profile* out);

/* ------------------------------------------------------------ training */
/* On-GPU training of a regression network (the learned heuristic; design
 * objective of the appendix: large mean h with h_M <= h*), for the sliding-tile
 * domains and the cube.
 * Loss over a batch of n labelled states:
 *   L = (1/n) sum_b w_b (y_b - t_b)^2,  w_b = alpha if asym and y_b > t_b else 1.
 * Gradients by the chain rule on the GPU (weight gradients in FP32; the
 * layer-1 gradient is the scatter-add of the pre-activation gradient rows that
 * the one-hot input selects; the cube's six centre rows, always active, get the
 * bias gradient); Adam (Kingma & Ba) on FP32 master weights, after which the
 * working copies (BF16 or FP32) are re-cast.  ReLU'(z) = [z > 0].  Every
 * reduction over the batch runs in a fixed order (no float atomics), so a
 * step's gradients are bitwise repeatable. */
typedef struct {
    hb_precision prec;   /* HB_BF16 (BF16 operands, FP32 master) or HB_FP32 */
    int device;
    int max_batch;       /* largest n per step (default 8192) */
    float lr, beta1, beta2, eps; /* defaults 1e-3, 0.9, 0.999, 1e-8 */
    int asym;            /* asymmetric loss */
    float alpha;         /* over-estimate weight (default 4) */
} hb_train_opts;

typedef struct hb_trainer hb_trainer;
/* opts NULL = defaults.  The weight file must be a regression network whose
 * hidden widths are at most 1024. */
hb_status hb_trainer_create(const char* weights_path, const hb_train_opts* opts, hb_trainer** out);
void hb_trainer_free(hb_trainer* t); /* NULL-safe */
int64_t hb_trainer_n_params(const hb_trainer* t);
/* One optimisation step on n <= max_batch states (device, packed) with float32
 * labels (device).  loss_out (host, nullable): the batch loss before the step
 * (synchronises the stream).  Asynchronous otherwise. */
hb_status hb_train_step(hb_trainer* t, const uint8_t* d_packed, const float* d_labels, int64_t n, float* loss_out,
                        void* stream);
/* Loss and gradient without an update: d_grads (device, float32,
 * hb_trainer_n_params entries) in weight-file order.  Synchronous. */
hb_status hb_train_grad(hb_trainer* t, const uint8_t* d_packed, const float* d_labels, int64_t n, float* d_grads,
                        float* loss_out);
/* FP32 master weights: copy out (host, n_params floats, weight-file order) or
 * write a weight file that hb_model_load accepts. */
hb_status hb_trainer_get_params(hb_trainer* t, float* out);
hb_status hb_trainer_save(hb_trainer* t, const char* path);

/* -------------------------------------------------------------- search */
typedef enum { HB_IDA = 0, HB_BTS = 1 } hb_algo;

/* How the search obtains h for pruning:
 *  HB_H_NN:          the network's h (model output rule, GPU batches).
 *  HB_H_MIN_NN_CLASSIC: min(network h, classic h).
 *  HB_H_FIXED_TREE:  the network is evaluated on every generated state (GPU
 *                    batches) but pruning uses the classic h, so the tree is the
 *                    classic heuristic's (Fixed-Tree Evaluation).
 *  HB_H_CLASSIC:     classic h only, computed at generation (no network).
 *  HB_H_CLASSIC_BATCHED: classic h computed by the batch thread on the host,
 *                    through the same batching machinery (no GPU needed).
 *  HB_H_NN_REAL:     real-valued h = max(0, y - offset) of a regression model in
 *                    the HB_OUT_REG_REAL mode, unrounded (Regression-Based Neural
 *                    Heuristics experiment): f = g + h and the cost bounds are
 *                    real; IDA*'s next bound is the smallest pruned f and BTS
 *                    bisects over real bounds (cbdfs_iter.bound_real).  The
 *                    model must be loaded with combine_md = 0: the real value is
 *                    the network's own, so a Manhattan rule (min, max or plus)
 *                    would be silently dropped; cbdfs_solve returns HB_E_INVAL
 *                    for such a model. */
typedef enum {
    HB_H_NN = 0, HB_H_MIN_NN_CLASSIC = 1, HB_H_FIXED_TREE = 2, HB_H_CLASSIC = 3, HB_H_CLASSIC_BATCHED = 4,
    HB_H_NN_REAL = 5
} hb_combine;

typedef enum { HB_CLASSIC_ZERO = 0, HB_CLASSIC_MD = 1, HB_CLASSIC_PDB = 2 } hb_classic;

typedef struct {
    hb_model* model;       /* required unless combine is CLASSIC or CLASSIC_BATCHED */
    hb_combine combine;
    hb_classic classic;
    const hb_pdb* pdb;     /* for HB_CLASSIC_PDB: a corner PDB (cube) or an additive PDB (15-puzzle) */
} hb_heuristic;

typedef struct {
    int batch_size;        /* states per batch (default 8000) */
    int work_num;          /* subtrees per search thread, workNum (default 8) */
    int d_init;            /* depth of the initial partitioning tree (< 0, the default: the shallowest depth
                              with at least 1024*threads*work_num work units, capped near 3M tree nodes) */
    int timeout_us;        /* partial-batch flush timeout (default 4000, the paper's 4 ms) */
    int n_slabs;           /* batch buffers kept in host memory (default 4) */
    int flush_when_idle;   /* 1 (default): also flush as soon as every search thread waits on h;
                              2: also flush whenever the batch thread is free (a batch then holds
                              what arrived while the previous one was evaluated); 0: only a full
                              slab or the timeout */
    int64_t node_limit;    /* total expansions (<= 0: none) */
    double time_limit_s;   /* wall limit (<= 0: none) */
    int64_t bts_b0;        /* BTS first budget (default 10000) */
    int bts_c1, bts_c2;    /* BTS growth window (defaults 2 and 8) */
    int bts_root_plus_one; /* BTS first bound h(root)+1 (default 1) */
    int dedup_frontier;    /* remove duplicate frontier states after partitioning (default 0) */
    int complete_final_iter; /* finish the final iteration (default 0) */
    int32_t start_bound;   /* resume from this bound (< 0: h(start)) */
    int max_iters;         /* safety cap on iterations (default 1000) */
    int use_graphs;        /* replay each GPU batch as a captured hipGraph (copy in, forward, copy out),
                              one per power-of-two size bucket (default 1); 0: direct launches */
    int gpu_depth;         /* batches on the GPU at once, 1 (default) or 2: with 2 the next batch is
                              sealed and launched while the previous one is evaluated (the paper's
                              batch thread keeps several batches in RAM); needs n_slabs >= 3 */
} cbdfs_params;

/* Fill p with the defaults listed above. */
void cbdfs_params_default(cbdfs_params* p);

typedef struct {
    int32_t bound;
    int64_t limit;         /* expansion limit of this search (< 0: none) */
    int64_t expanded, generated;
    int32_t complete;      /* 1: the iteration ran to completion */
    int32_t found;
    double bound_real;     /* the bound (bound = its floor; equal for integer heuristics) */
    int64_t batches, evals; /* batches sent and states evaluated during this iteration (the
                               runtime batch statistics of the appendix on batch sizes in
                               practice); the initial tree's evaluation counts only in the totals */
} cbdfs_iter;

typedef struct {
    int32_t cost;          /* -1 if none */
    int32_t path_len;
    int8_t* path;          /* library-owned: moves from start to goal */
    int32_t n_iter;
    cbdfs_iter* iters;     /* library-owned */
    int64_t evals;         /* heuristic evaluations (network or batched classic) */
    int64_t batches;
    double mean_batch;
    double wall_s, gpu_busy_s;
    int64_t expanded, generated; /* totals over every iteration */
    int32_t frontier;      /* work units after the initial partitioning */
    int64_t peak_nodes;    /* most node records live at once */
} cbdfs_result;

/* Batch IDA* (Batch IDA* algorithm) or Batch BTS (Batch BTS enhancements) over
 * parallel CB-DFS (Parallel CB-DFS and Subtree expansion algorithms) with
 * `threads` search threads and one batch thread.  start: host state
 * (hb_state_bytes).  Invalid or unsolvable starts -> HB_E_INVAL before any
 * thread starts; limits -> HB_E_BUDGET with statistics; a device failure ->
 * HB_E_DEVICE after every thread has joined.  Release out with
 * cbdfs_result_free. */
hb_status cbdfs_solve(hb_domain d, const uint8_t* start, const hb_heuristic* h, hb_algo algo, int threads,
                      const cbdfs_params* p, cbdfs_result* out);
void cbdfs_result_free(cbdfs_result* r); /* NULL-safe */

#ifdef __cplusplus
}
#endif
#endif /* HB_H */

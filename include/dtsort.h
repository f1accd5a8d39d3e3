/*
 * dtsort.h -- C ABI of an MI355X (gfx950) implementation of DovetailSort, the
 * stable parallel MSD integer sort of "Parallel Integer Sort: Theory and
 * Practice" (Dong, Dhulipala, Gu, Sun; PPoPP 2024).
 *
 * Problem (Section 2.3): given n records with integer keys in [r], reorder them
 * so that keys are non-decreasing.  The sort is stable (equal keys keep their
 * input order; Section 2.3), and, as in the paper, the interface is "in place"
 * (the sorted result replaces the input) while O(n) extra space is used.
 *
 * Method (Alg. 2, Sections 3.1-3.5 and 5): per recursive subproblem, sample
 * keys to find heavy (frequently repeated) keys and the key range, give every
 * MSD zone one light bucket followed by its heavy buckets, stable-distribute
 * by bucket id (a counting sort), recurse only into light buckets (heavy
 * buckets are finished), then interleave each zone's sorted light run with its
 * heavy runs (the dovetail merge, Alg. 3).  Small subproblems are sorted in
 * the GPU's local data share; subproblems of one recursion level are processed
 * together in shared launches.
 *
 * Conventions for every entry point:
 *  - Data pointers are DEVICE pointers owned by the caller.  Keys (and values)
 *    are sorted in place.  Keys are unsigned integers.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it.  The sorts read back one small block of counters per recursion level
 *    (a synchronisation of `stream`) to size the next level's launches; the
 *    last level's leaf sorts and the dovetail merges are left enqueued, so the
 *    caller synchronises `stream` before reading the result.
 *  - Temporary device memory (a ping-pong partner of the data plus small
 *    per-level tables) is taken from a cache per (device, stream) that grows
 *    as needed and is kept until dtsort_release() or process exit; or, for
 *    the large partner buffer, from opts->workspace when the caller supplies
 *    one.  Calls on different streams (from different host threads, say) run
 *    concurrently, each with its own cache; calls on one stream are taken one
 *    at a time.  Up to 8 streams per device keep a cache; a further stream
 *    takes over the least recently used one (its calls then also wait for
 *    that cache's previous work).
 *  - Return value: DTSORT_OK or a negative dtsort_status.  No exception ever
 *    crosses this interface.  On error nothing is guaranteed about the data
 *    except that no memory outside the given arrays is written.
 *  - n = 0 and n = 1 are valid no-ops.  n must be < 2^32.
 */
#ifndef DTSORT_H
#define DTSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dtsort_status {
  DTSORT_OK = 0,
  DTSORT_EINVAL = -1,     /* bad argument (NULL with n > 0, n >= 2^32, overlap, bad offsets) */
  DTSORT_ENOMEM = -2,     /* device allocation failed */
  DTSORT_EWORKSPACE = -3, /* opts->workspace given but smaller than dtsort_workspace_bytes() */
  DTSORT_EHIP = -4,       /* a HIP runtime call failed (message via dtsort_last_error()) */
  DTSORT_EINTERNAL = -5   /* a device-side capacity or consistency check failed */
} dtsort_status;

typedef enum dtsort_mode {
  DTSORT_MODE_SAMPLING = 0, /* the paper's method: heavy keys found by sampling (Section 3.1) */
  DTSORT_MODE_PLAIN = 1,    /* heavy-key detection off: the paper's "Plain" ablation (Section 6.3) */
  DTSORT_MODE_LEARNED = 2   /* root zones from a learned CDF model's splitters, sampling as fallback/judge */
} dtsort_mode;

/* Counters filled when opts->stats is non-NULL (host memory; valid after the
 * call returns -- they are read back during the call). */
typedef struct dtsort_stats {
  uint64_t levels;              /* recursion levels that distributed records */
  uint64_t tasks;               /* subproblems distributed (sampling + counting sort) */
  uint64_t records_distributed; /* sum of their sizes */
  uint64_t heavy_keys;          /* heavy keys found (all levels) */
  uint64_t heavy_records;       /* records in heavy buckets */
  uint64_t merges;              /* zones dovetail-merged */
  uint64_t records_merged;      /* records written by dovetail merges */
  uint64_t leaf_sorts;          /* local-memory base-case sorts */
  uint64_t records_leaf_sorted; /* records they sorted */
  uint64_t records_copied;      /* records moved between buffers (finished buckets, spills) */
  uint64_t overflow_records;    /* records that landed in overflow buckets */
  int32_t learned_used;         /* LEARNED mode: 1 if the model's zones were used */
  float learned_balance;        /* LEARNED mode: balance error of the model's zones */
  float sampling_balance;       /* LEARNED mode: balance error of the digit zones */
  float learned_final_loss;     /* LEARNED mode: training loss of the last step */
  double learned_ms;            /* LEARNED mode: time spent sampling, training and judging (ms) */
  /* Filled only when opts->profile is set: per kernel kind (0 plan, 1 histogram,
   * 2 scans, 3 scatter, 4 child planning, 5 leaf sorts, 6 copies, 7 dovetail
   * merges) the summed launch time measured with HIP events on `stream`, the
   * algorithmic bytes those launches move (records x record bytes, read +
   * write; histogram: read only), and the number of launches. */
  double kernel_ms[8];
  double kernel_bytes[8];
  uint32_t kernel_launches[8];
  uint64_t records_pair_merged; /* records of paired base cases (32-bit keys without values): each is leaf-sorted
                                   as part of one half (counted in records_leaf_sorted) and then written once
                                   more by the merge of the two halves */
  /* LEARNED mode: the judge's predicted work below the root, in record passes
   * (records x (1 + distribution levels still needed, log2(zone / cutoff) /
   * digit bits), from a held-out sample):
   * for the sampling step's digit zones, for the model's zones (0 if not trained),
   * and for an ideal even split into the model's number of zones.  The model is
   * trained only when sampling_cost > 1.25 x ideal_cost, and its zones are used
   * only when learned_cost < 0.9 x sampling_cost (or always, learned_judge = 1). */
  int32_t learned_trained;      /* 1 if the model was trained */
  float learned_cost;
  float sampling_cost;
  float ideal_cost;
} dtsort_stats;

typedef struct dtsort_opts {
  uint64_t seed;          /* seed of the sampling generator (Appendix A: deterministic given it) */
  int32_t key_bits;       /* 0 = full width; else keys are < 2^key_bits (the paper's optional bit count) */
  int32_t mode;           /* dtsort_mode */
  int32_t digit_bits;     /* 0 = automatic (log2 of the cube root of n', clamped to [8, 10]); else 1..10 */
  int32_t lds_cutoff;     /* 0 = automatic; base-case threshold theta (records) */
  int32_t tuned;          /* 1 = take digit_bits / lds_cutoff / tile_shape from the tuning table when they are 0
                             (the file named by DTSORT_TUNE_FILE, else tune_table.txt beside the library;
                             written by the package's autotuner) */
  int32_t learned_steps;  /* LEARNED: optimiser steps (0 = default 128) */
  int32_t learned_batch;  /* LEARNED: batch size (0 = default 1024) */
  float learned_lr;       /* LEARNED: Adam step size (0 = default 3e-3) */
  int32_t profile;        /* 1 = time every kernel launch with HIP events into stats (adds syncs) */
  int32_t tile_shape;     /* scatter tile for digits <= 8 bits: 0 = automatic, 1 = 512 threads x 16 keys
                             (x 8 for 64-bit keys), 2 = 256 x 16, 3 = 512 x 8, 4 = 256 x 32, 5 = 1024 x 8
                             (x 4), 6 = 1024 x 16 for 32-bit keys without values and unordered ranks
                             (else as 5) */
  int32_t graph;          /* 1 = device-driven schedule recorded once into a HIP graph and replayed: no
                             host read-back between levels, the call only enqueues one graph launch.
                             The graph is cached per (entry point, pointers, sizes, options) with its
                             own worst-case workspace (at most 4 per device, least recently used
                             evicted); a first call records and instantiates it.  Not with LEARNED
                             mode or profile.  Errors (invalid segment offsets) are reported only
                             when stats is given, which makes the call wait for the graph. */
  int32_t ordered_ranks;  /* keys without values: 1 = the distribution keeps equal-bucket keys in input
                             order (as it always does for records with values), so that the recursion
                             shape (levels, tasks, heavy keys) depends on the seed alone (Appendix A);
                             0 (default) = unordered ranks from LDS atomics, faster.  Equal keys cannot
                             be told apart, so the sorted output is the same either way. */
  int32_t learned_judge;  /* LEARNED: 0 = the cost judge decides (train only when the sampling plan leaves
                             clearly more work than an ideal split; use the model's zones only when they are
                             predicted cheaper); 1 = always train and use the model's zones */
  int32_t merge_variant;  /* Step 4 (Section 3.4) implementation, for the paper's merge study (Section 6.3):
                             0 = the dovetail merge as one out-of-place gather (default);
                             1 = PLMerge-style: a general parallel merge (merge path) of the zone's light
                                 run with its heavy runs into the partner buffer, then copied back;
                             2 = Alg. 3 literally: the zone gathered in one buffer, the smaller side copied
                                 out, heavy buckets moved one by one (two flips where a bucket overlaps its
                                 destination), the copied side moved back;
                             3 = no merge: zones with heavy keys are left unmerged, so the output is NOT
                                 sorted (a timing knob for the other steps);
                             4 = dovetailing during distribution (a variant derived from Section 3.4):
                                 each zone's light keys are split at its heavy keys into light sub-buckets
                                 (at most 2^(digit bits - 2) heavy keys a subproblem, the ones filling the
                                 most subsample slots), so heavy buckets land in their final places and
                                 no merge is needed (a learned root's zones still merge as in 0).
                             Variants 0-2 and 4 give the same sorted output. */
  int32_t digit_bits_below; /* digit width of the subproblems below the roots (every level after the first):
                               0 = as digit_bits (with tuned = 1 and digit_bits 0: the tuning table's
                               choice); else 1..10 */
  void* workspace;        /* optional device buffer for the ping-pong partner (see dtsort_workspace_bytes) */
  size_t workspace_bytes;
  dtsort_stats* stats;    /* optional host pointer */
} dtsort_opts;

/* Fill *opts with defaults (seed 0, automatic parameters, SAMPLING mode;
 * host memory, caller-owned; NULL is ignored). */
void dtsort_default_opts(dtsort_opts* opts);

/* Bytes of caller-supplied workspace needed for n records of key_bytes-wide
 * keys and val_bytes-wide values (0 for keys only): the ping-pong partner of
 * the data (Section 5, "minimizing data movement"), rounded to 256 bytes. */
size_t dtsort_workspace_bytes(int key_bytes, int val_bytes, size_t n);

/* Integer sort (Section 2.3) of n 32-bit keys in place: on return keys[0..n)
 * holds the input keys in non-decreasing order (keys alone: the sorted
 * multiset).  Method: Alg. 2 with Sections 3.1-3.5 and 5 (see the top of this
 * file); opts->mode selects the heavy-key detection (Section 3.1), PLAIN the
 * paper's ablation without it (Section 6.3).  keys: device, n elements,
 * caller-owned.  opts may be NULL (defaults).  Errors: DTSORT_EINVAL for NULL
 * keys with n > 0, n >= 2^32 or an option out of range (nothing written);
 * DTSORT_ENOMEM, DTSORT_EHIP, DTSORT_EINTERNAL as above. */
int dtsort_u32(uint32_t* keys, size_t n, const dtsort_opts* opts, void* stream);

/* The same for n 64-bit keys (Section 2.3; Section 6 sorts 64-bit keys too). */
int dtsort_u64(uint64_t* keys, size_t n, const dtsort_opts* opts, void* stream);

/* Stable integer sort (Section 2.3: records reordered by key, equal keys in
 * their input order) of n (64-bit key, 64-bit value) records stored as two
 * device arrays (structure of arrays, n elements each, caller-owned); values
 * move with their keys.  The paper's 64-bit experiments sort such records
 * (Section 6).  keys and values must not overlap (DTSORT_EINVAL otherwise,
 * as for a NULL array with n > 0); other errors as for dtsort_u32. */
int dtsort_pairs_u64(uint64_t* keys, uint64_t* values, size_t n, const dtsort_opts* opts, void* stream);

/* Stable integer sort (Section 2.3) of n (32-bit key, 32-bit value) records
 * stored as two device arrays, the record layout of the paper's 32-bit
 * experiments and of both its applications (Section 6); values move with
 * their keys.  keys and values must not overlap; errors as for
 * dtsort_pairs_u64. */
int dtsort_pairs_u32(uint32_t* keys, uint32_t* values, size_t n, const dtsort_opts* opts, void* stream);

/* Batched form (not in the paper: many instances of Section 2.3's problem
 * at once): n_segments independent stable sorts of 32-bit keys (and optional
 * 32-bit values, NULL for keys only) stored back to back.  Segment s is
 * [seg_offsets[s], seg_offsets[s+1]); seg_offsets is a DEVICE array of
 * n_segments + 1 uint64 with seg_offsets[0] = 0, non-decreasing and
 * seg_offsets[n_segments] = n_total (checked on the device; a violation
 * returns DTSORT_EINVAL, found after the seeding step; with opts->graph = 1
 * only when stats are requested).  Empty segments are allowed.  Every
 * segment is a root subproblem of Alg. 2; all of them are processed level by
 * level in shared launches.  keys/values: device, n_total elements,
 * caller-owned; n_segments < 2^31. */
int dtsort_segmented(uint32_t* keys, uint32_t* values, size_t n_total, const uint64_t* seg_offsets,
                     size_t n_segments, const dtsort_opts* opts, void* stream);

/* ---- step entry points: one step of the method on one subproblem, for
 * step-level checks against a CPU model.  Same conventions as above; they
 * synchronise `stream` before returning. ---- */

/* Step 1 (Section 3.1 and the sampled key range of Section 5) on the n keys,
 * as the root subproblem (offset 0, level 0) whose keys share all bits at and
 * above `hi`.  Outputs (host pointers): plan[0..5] = {gamma, w, shift, top,
 * n_heavy, n_buckets}; heavy[0..n_heavy) = heavy keys ascending (room for
 * 1024 entries); light_id[0..2^w] = the light bucket id of each zone (the last
 * entry is the overflow bucket id; room for 2049 entries). */
int dtsort_step_plan_u32(const uint32_t* keys, size_t n, int hi, int skip_disabled, const dtsort_opts* opts,
                         int32_t* plan, uint32_t* heavy, uint32_t* light_id, void* stream);
int dtsort_step_plan_u64(const uint64_t* keys, size_t n, int hi, int skip_disabled, const dtsort_opts* opts,
                         int32_t* plan, uint64_t* heavy, uint32_t* light_id, void* stream);

/* Steps 1 + 2 (Section 3.2, the stable counting sort by GetBucketId) on the
 * root subproblem: keys (and values, may be NULL) are distributed into
 * out_keys / out_values (device, n each); counts (host, room for 4097) gets
 * the record count of every bucket id; plan/heavy/light_id as above. */
int dtsort_step_distribute_u32(const uint32_t* keys, const uint32_t* values, size_t n, int hi,
                               const dtsort_opts* opts, uint32_t* out_keys, uint32_t* out_values,
                               uint32_t* counts, int32_t* plan, uint32_t* heavy, uint32_t* light_id,
                               void* stream);
int dtsort_step_distribute_u64(const uint64_t* keys, const uint64_t* values, size_t n, int hi,
                               const dtsort_opts* opts, uint64_t* out_keys, uint64_t* out_values,
                               uint32_t* counts, int32_t* plan, uint64_t* heavy, uint32_t* light_id,
                               void* stream);

/* Base case (Section 3.5): stable local-memory sort of each segment
 * [seg_offsets[s], seg_offsets[s+1]) (device array) of at most 16384 keys
 * (8192 for 64-bit pairs) by the key bits below `bits`; out-of-place into
 * out_keys/out_values. */
int dtsort_step_leaf_u32(const uint32_t* keys, const uint32_t* values, const uint64_t* seg_offsets,
                         size_t n_segments, int bits, uint32_t* out_keys, uint32_t* out_values, void* stream);
int dtsort_step_leaf_u64(const uint64_t* keys, const uint64_t* values, const uint64_t* seg_offsets,
                         size_t n_segments, int bits, uint64_t* out_keys, uint64_t* out_values, void* stream);

/* Step 4 (Section 3.4, Alg. 3) on one MSD zone: b0 sorted light records
 * (b0_keys/b0_values, device) and m heavy buckets given by host arrays
 * heavy_keys[m] (ascending, none equal to a light key) and heavy_sizes[m];
 * heavy values (device, sum of sizes, bucket after bucket; NULL for keys
 * only).  Writes the merged zone to out_keys / out_values (device). */
int dtsort_step_dtmerge_u64(const uint64_t* b0_keys, const uint64_t* b0_values, size_t b0,
                            const uint64_t* heavy_keys, const uint32_t* heavy_sizes, size_t m,
                            const uint64_t* heavy_values, uint64_t* out_keys, uint64_t* out_values,
                            void* stream);

/* ---- learned partitioner (not in the paper): FP32 CDF model 1->64->64->1 ----
 * Parameters are 4353 floats in the order W1[64], b1[64], W2[64][64] (row =
 * output unit), b2[64], W3[64], b3.  All pointers are device pointers. */

/* Mean squared error of the model on (x[i], y[i]), i < n, and its gradient
 * (4353 floats, overwritten); loss is one float. */
int dtsort_mlp_loss_grad(const float* params, const float* x, const float* y, size_t n, float* grad,
                         float* loss, void* stream);
/* Forward pass: pred[i] = model(x[i]). */
int dtsort_mlp_forward(const float* params, const float* x, size_t n, float* pred, void* stream);
/* Train from the deterministic initialisation of `seed` on sorted keys
 * (64-bit, device, n of them) for `steps` Adam steps; writes params (4353
 * floats) and losses[steps] (may be NULL). */
int dtsort_mlp_train_u64(const uint64_t* sorted_keys, size_t n, uint64_t seed, int steps, int batch,
                         float lr, float* params, float* losses, void* stream);

/* Allocation-free variant of dtsort_segmented, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and result as
 * dtsort_segmented; it runs the same kernels in the order of the graph form
 * (opts->graph = 1: no host read-back, no synchronisation), enqueued directly
 * on `stream`.  It calls no hipMalloc, hipFree or other allocating routine:
 * every temporary buffer, and the ping-pong partner unless opts->workspace is
 * given, lives in one static device array of 64 MiB that each device the
 * library runs on holds until the process ends.  Inputs whose schedule needs
 * more than that (about 2^22 keys without values, 2^21 with values, without a
 * caller workspace) return DTSORT_EINVAL with a message naming the need.
 * LEARNED mode, stats and profiling are rejected (DTSORT_EINVAL); invalid
 * segment offsets are not reported (those segments are left as they are).
 * All calls on one device share the array: calls whose work overlaps in time
 * on one device (different streams, or host threads) race and must be
 * serialised by the caller; a call made after the previous one's work was
 * enqueued on the same stream is safe. */
int dtsort_segmented_noalloc(uint32_t* keys, uint32_t* values, size_t n_total, const uint64_t* seg_offsets,
                             size_t n_segments, const dtsort_opts* opts, void* stream);

/* ---- the paper's applications (Section 6.2) over the 32+32-bit sort ---- */

/* Graph transpose: the directed graph with V = n_vertices vertices and
 * E = n_edges edges in compressed sparse row form (offsets: V + 1 uint64,
 * offsets[0] = 0, non-decreasing, offsets[V] = E; targets: E uint32 < V; the
 * out-edges of u are targets[offsets[u] .. offsets[u+1])) is reversed: every
 * edge (u, v) becomes (v, u).  The result, also in CSR form, goes to
 * t_offsets (V + 1) and t_targets (E): the in-neighbours of v, in the order
 * the edges were listed (sources ascending) -- a stable sort of the edges by
 * target.  All arrays are device memory; the inputs are not modified.
 * Temporary memory: E keys from the stream's cache, and the sort's own.
 * Invalid offsets or targets return DTSORT_EINVAL (checked on the device; the
 * call synchronises `stream` to read the check).  opts as for the sorts (no
 * graph form, no LEARNED mode). */
int dtsort_graph_transpose(const uint64_t* offsets, const uint32_t* targets, uint32_t n_vertices, size_t n_edges,
                           uint64_t* t_offsets, uint32_t* t_targets, const dtsort_opts* opts, void* stream);

/* Morton order of n points with dims = 2 or 3 coordinates (coords: dims * n
 * uint32, coordinate j of point i at coords[j * n + i]; the low 32 / dims
 * bits of each coordinate are used): codes[i] gets the z-value of point i
 * (bit b of coordinate j at bit dims * b + j), then codes are sorted stably
 * with perm (= point indices) as values.  On return codes holds the sorted
 * z-values and perm the points in Morton order (equal z-values by index).
 * Device memory; enqueued on `stream` like the sorts. */
int dtsort_morton_u32(const uint32_t* coords, int dims, size_t n, uint32_t* codes, uint32_t* perm,
                      const dtsort_opts* opts, void* stream);

/* Plain copy of n 32-bit words from src to dst (device, caller-owned, not
 * overlapping: DTSORT_EINVAL otherwise, and for NULL or n >= 2^32) with the
 * copy kernel the sorts use for finished buckets (Section 5's buffer copies);
 * enqueued on `stream`.  A measurement aid: the HBM rate this kernel reaches
 * is the practical ceiling the sort's byte-moving kernels are compared with. */
int dtsort_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, void* stream);

/* Release every cache of temporary buffers, graphs and streams, of all
 * devices and streams (call with no sort in flight; the next call allocates
 * again). */
void dtsort_release(void);

/* Message of the last error on the calling thread ("" if none; the string
 * is owned by the library and valid until the thread's next call). */
const char* dtsort_last_error(void);
const char* dtsort_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* DTSORT_H */

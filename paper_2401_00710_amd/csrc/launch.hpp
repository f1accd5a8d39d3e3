// Kernel launchers shared by the host driver and the kernel translation units.
#pragma once
#include "common.hpp"

namespace dts {

constexpr int LEAF_CLASSES_MAX = 6;

// Per-level device state handed to the kernels of one recursion level.
//
// Work counts are read on the device: `in` holds the counters the previous
// step wrote (next_tasks, next_records), and the prep step of the level
// writes cur_tasks, chunk and cur_units into `ctr`.  Every kernel of the
// level loops over its items with a grid stride, so the host may launch any
// grid (the exact count after a read-back, or a fixed persistent grid when
// the whole sort is recorded into a graph without read-backs).
struct LevelArgs {
  Task* tasks;
  uint32_t n_tasks;      // capacity of `tasks` (the exact count when it is known on the host)
  uint32_t chunk;        // records per distribution unit; 0: the prep step derives it from the level's records
  uint2* units;          // (task index, chunk index) per distribution unit
  uint8_t* tab;          // table arena of this level
  uint32_t slot_bytes;   // bytes per task slot
  uint32_t cols;         // count-matrix columns per chunk (1, or one per wave for the direct scatter)
  uint32_t* cm;          // count matrices of this level
  // children planning outputs
  Task* next;
  Leaf* leaf[LEAF_CLASSES_MAX];
  Leaf* copies;
  Merge* merges;
  Leaf* spills;
  const LevelCounters* in;  // counters of the step that created this level's tasks
  LevelCounters* ctr;       // this level's counters (zeroed by the prep step)
  Caps caps;
  // configuration
  uint64_t seed;
  int g_override;
  uint32_t cutoff;
  uint32_t leaf_max[LEAF_CLASSES_MAX];  // size limit of each leaf class
  int plain;
  int key_bits;
  int tile;  // scatter tile shape (0..4, see launch_distribute)
  int ordered;  // keys without values: keep equal-bucket keys in input order (stable ranks)
  int merge_variant;  // MergeVariant: how zones with heavy keys are merged
  int g_learned_child;  // digit-width override of the children of a learned root
  uint32_t grid_tasks;  // launch grid of the per-task kernels
  uint32_t grid_units;  // launch grid of the per-unit kernels
};

// Implementations of Step 4 (the dovetail merge) for the paper's merge study.
// MV_SPLIT: no merge at all; every zone's light keys are split at its heavy
// keys during the distribution (the split bucket layout, TF_SPLIT), so heavy
// buckets land in their final places.  Zones of a learned root still merge
// (as MV_GATHER).
enum MergeVariant : int { MV_GATHER = 0, MV_PLMERGE = 1, MV_INPLACE = 2, MV_NONE = 3, MV_SPLIT = 4 };
// Variants that work on the zone laid out contiguously in its target buffer
// (the light run sorted there, the heavy runs copied there when the
// distribution left them in the other buffer).
__host__ __device__ inline bool zone_in_target(int v) { return v == MV_PLMERGE || v == MV_INPLACE; }

// Grid of the persistent (grid-stride) launches: workgroups per compute unit
// times the compute units of the current device.
uint32_t persistent_grid(uint32_t wg_per_cu);

// g_level_max: the widest digit of the level's tasks (selects the sample capacity)
template <typename K>
void launch_plan(const LevelArgs& a, const K* k0, const K* k1, int g_level_max, hipStream_t s);

// phase 0: histogram; 1: column and bucket scans; 2: scatter; -1: all three
template <typename K, typename V>
void launch_distribute(const LevelArgs& a, Bufs<K, V> b, int g_level_max, uint32_t max_chunks, hipStream_t s,
                       int phase = -1);

// Count-matrix columns per chunk the distribution of a level will use.
uint32_t dist_cols(int g_level_max);

void launch_prep(const LevelArgs& a, hipStream_t s);

// Root of a whole-array sort, written on the device: one task and the
// counters a level reads (graph-recordable; no host staging).
template <typename K>
void launch_root(Task* t, LevelCounters* in, uint64_t n, int key_bits, int gamma, hipStream_t s);

// Zeroes `n` counter blocks (a kernel, so that it can be recorded in a graph).
void launch_zero_counters(LevelCounters* c, uint32_t n, hipStream_t s);

template <typename K, typename V>
void launch_children(const LevelArgs& a, Bufs<K, V> b, hipStream_t s);

template <typename K, typename V>
void launch_seed_segments(const LevelArgs& a, const uint64_t* seg_off, uint32_t n_seg, uint64_t n_total,
                          hipStream_t s);

// List kernels: `count` is the device-side number of items (the kernels loop
// over min(*count, cap) items with a grid stride); `grid` is the launch grid.
template <typename K, typename V>
void launch_leaf(const Leaf* items, const uint32_t* count, uint32_t cap, uint32_t grid, int cls, Bufs<K, V> b,
                 hipStream_t s);

// Paired leaves (32-bit keys without values): a bucket of cutoff < c <=
// 2 * cutoff records is sorted as two leaves, its halves, into the buffer
// other than its target, and the two sorted halves are then merged into the
// target.  `halves` holds two Leaf entries per bucket (count = entries);
// grid_leaf / grid_merge: launch grids of the two steps.  No-op for other
// layouts (their lists stay empty).
template <typename K, typename V>
void launch_pairs(const Leaf* halves, const uint32_t* count, uint32_t cap, uint32_t grid_leaf, uint32_t grid_merge,
                  Bufs<K, V> b, hipStream_t s);

// Tasks left after the last recorded level of the graph form: each sorted
// completely by one workgroup.
template <typename K, typename V>
void launch_finish(const Task* tasks, const uint32_t* count, uint32_t cap, uint32_t grid, Bufs<K, V> b,
                   hipStream_t s);

// Copies move pieces of at most COPY_PIECE records (one workgroup a piece):
// a large finished bucket becomes several items.
constexpr uint32_t COPY_PIECE = 1u << 16;
__device__ __host__ inline uint32_t pieces_of(uint32_t c) { return c / COPY_PIECE + (c % COPY_PIECE != 0u ? 1u : 0u); }

// Items (and their count) of a plain copy of n < 2^32 records from buffer 0
// to buffer 1; `items` holds pieces_of(n).
void launch_copy_items(Leaf* items, uint32_t* count, uint64_t n, hipStream_t s);

template <typename K, typename V>
void launch_copy(const Leaf* items, const uint32_t* count, uint32_t cap, uint32_t grid, Bufs<K, V> b, hipStream_t s);

void launch_merge_units(const Merge* m, const uint32_t* count, uint32_t cap, uint32_t grid, uint2* munits,
                        hipStream_t s);

// Merges of one level's zones with the given MergeVariant (MV_NONE: nothing).
template <typename K, typename V>
void launch_merge(const Merge* m, const uint32_t* n_merges, uint32_t merge_cap, uint32_t merge_grid,
                  const uint2* munits, const uint32_t* n_munits, uint32_t munit_cap, uint32_t munit_grid,
                  uint8_t* tab, Bufs<K, V> b, int variant, hipStream_t s);

// Applications (apps.hip).  Graph transpose: *err gets bit 1 for invalid
// offsets, bit 2 for a target outside [0, V); keys = the targets, src = the
// edges' sources.  t_off[v] = edges with a sorted key below v, v in [0, V].
void launch_transpose_prepare(const uint64_t* off, const uint32_t* tgt, uint32_t n_vertices, uint64_t n_edges,
                              uint32_t* keys, uint32_t* src, uint32_t* err, hipStream_t s);
void launch_transpose_offsets(const uint32_t* keys, uint64_t n_edges, uint32_t n_vertices, uint64_t* t_off,
                              hipStream_t s);
// Morton order: z-values (2 or 3 coordinates, coordinate j of point i at
// coords[j * n + i], low 32/dims bits of each) and point indices.
void launch_morton(const uint32_t* coords, int dims, uint64_t n, uint32_t* codes, uint32_t* idx, hipStream_t s);

// Learned partitioner (k_mlp.hip).
int mlp_loss_grad(const float* p, const float* x, const float* y, uint32_t n, float* grad, float* loss, float* part,
                  hipStream_t s);
void mlp_forward(const float* p, const float* x, uint32_t n, float* pred, hipStream_t s);
void mlp_train(const float* x, const float* y, uint32_t n, uint64_t seed, int steps, uint32_t batch, float lr,
               float* p, float* m, float* v, float* part, float* losses, hipStream_t s);
template <typename K>
void mlp_data(const K* sk, uint32_t n, int kb, float* x, float* y, hipStream_t s);
template <typename K>
void learned_kernels_draw(const K* keys, uint64_t n, uint64_t seed, uint32_t tag, uint32_t count, K* out,
                          hipStream_t s);
template <typename K>
void learned_kernels_split(const K* sk, const float* pred, uint32_t n, uint32_t zones, float* mono, uint64_t* spl,
                           hipStream_t s);
// The learned partitioner's decision record (device, read back by the host).
struct LearnedInfo {
  float bal_learned, bal_digit;  // balance errors (largest zone / ideal) of the held-out light keys
  uint32_t use_learned;          // 1: the model's zones replaced the digit zones
  uint32_t light_held;           // held-out keys that are light
  float final_loss;              // training loss of the last step
  uint32_t trained;              // 1: the model was trained (the digit plan's cost left room for a gain)
  float cost_digit, cost_learned, cost_ideal;  // predicted record passes below each root plan
};
struct JudgeParams {
  float scale;         // records a held-out key stands for
  float cutoff;        // base-case size
  int g_digit;         // digit width below a digit-zone root
  int g_learned;       // digit width below a learned root
  int force;           // use the model's zones whatever the costs
  float train_margin;  // train only if the digit plan's cost exceeds this x the ideal split's
  float use_margin;    // use the model's zones only if their cost is below this x the digit plan's
};
// spl = nullptr: the pre-training check only (digit plan and ideal costs, `trained` = whether to train).
template <typename K>
void learned_kernels_judge(Task* task, uint8_t* tab, const K* held, uint32_t nh, const uint64_t* spl, uint32_t zones,
                           const JudgeParams& jp, LearnedInfo* info, const float* losses, int steps, hipStream_t s);
constexpr int MLP_PARAMS = 4353;
constexpr int MLP_GT = 64;  // samples per gradient workgroup (partial-gradient buffer sizing)

// Tile sizes of the distribution kernels (records per tile) by key width.
template <typename K, typename V>
constexpr uint32_t dist_tile() {
  return (sizeof(K) + (HasVal<V>::value ? sizeof(V) : 0)) <= 4 ? 8192u : ((sizeof(K) <= 4) ? 8192u : 4096u);
}

// Leaf classes: the largest size each class sorts, by record layout.
constexpr int LEAF_CLASSES = 5;
// Index of the list (and counter) of paired-leaf halves, after the classes.
constexpr int LEAF_PAIR = LEAF_CLASSES;
constexpr uint32_t PAIR_MAX = 32768;  // largest bucket the pair merge holds in LDS
template <typename K, typename V>
constexpr bool pair_leaves() {
  return sizeof(K) == 4 && !HasVal<V>::value;
}
template <typename K, typename V>
constexpr uint32_t leaf_cap(int cls) {
  return cls == 0 ? 256u
                  : (cls == 1 ? 1024u
                              : (cls == 2 ? 4096u
                                          : (cls == 3 ? 8192u : ((sizeof(K) == 8 && HasVal<V>::value) ? 8192u : 16384u))));
}

// Largest bucket sorted as a pair (0: none): twice the base-case cutoff,
// within what the largest leaf class and the pair merge hold.
template <typename K, typename V>
constexpr uint32_t pair_max(uint32_t cutoff) {
  return pair_leaves<K, V>() ? 2u * (cutoff < leaf_cap<K, V>(LEAF_CLASSES - 1) ? cutoff : leaf_cap<K, V>(LEAF_CLASSES - 1))
                             : 0u;
}
static_assert(2 * leaf_cap<uint32_t, NoVal>(LEAF_CLASSES - 1) <= PAIR_MAX, "a pair fits the merge's LDS");

}  // namespace dts

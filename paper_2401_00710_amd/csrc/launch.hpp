// Kernel launchers shared by the host driver and the kernel translation units.
#pragma once
#include "common.hpp"

namespace dts {

// Per-level device state handed to the kernels of one recursion level.
struct LevelArgs {
  Task* tasks;
  uint32_t n_tasks;
  uint32_t chunk;        // records per distribution unit (multiple of every tile size)
  uint2* units;          // (task index, chunk index) per distribution unit
  uint8_t* tab;          // table arena of this level
  uint32_t slot_bytes;   // bytes per task slot
  uint32_t pad0;
  uint32_t* cm;          // count matrices of this level
  // children planning outputs
  Task* next;
  Leaf* leaf[3];
  Leaf* copies;
  Merge* merges;
  Leaf* spills;
  LevelCounters* ctr;
  Caps caps;
  // configuration
  uint64_t seed;
  int g_override;
  uint32_t cutoff;
  uint32_t leaf_max[3];  // size limit of each leaf class
  int plain;
  int key_bits;
};

template <typename K>
void launch_plan(const LevelArgs& a, const K* k0, const K* k1, hipStream_t s);

template <typename K, typename V>
void launch_distribute(const LevelArgs& a, Bufs<K, V> b, int g_level_max, uint32_t max_chunks, hipStream_t s);

void launch_prep(const LevelArgs& a, hipStream_t s);

template <typename K, typename V>
void launch_children(const LevelArgs& a, Bufs<K, V> b, hipStream_t s);

template <typename K, typename V>
void launch_seed_segments(const LevelArgs& a, const uint64_t* seg_off, uint32_t n_seg, uint64_t n_total,
                          hipStream_t s);

template <typename K, typename V>
void launch_leaf(const Leaf* items, uint32_t n_items, int cls, Bufs<K, V> b, hipStream_t s);

template <typename K, typename V>
void launch_copy(const Leaf* items, uint32_t n_items, Bufs<K, V> b, hipStream_t s);

void launch_merge_units(const Merge* m, uint32_t n_merges, uint2* munits, hipStream_t s);

template <typename K, typename V>
void launch_merge(const Merge* m, uint32_t n_merges, const uint2* munits, uint32_t n_munits, uint8_t* tab,
                  Bufs<K, V> b, hipStream_t s);

// Tile sizes of the distribution kernels (records per tile) by key width.
template <typename K, typename V>
constexpr uint32_t dist_tile() {
  return (sizeof(K) + (HasVal<V>::value ? sizeof(V) : 0)) <= 4 ? 8192u : ((sizeof(K) <= 4) ? 8192u : 4096u);
}

// Leaf classes: the largest size each class sorts, by record layout.
template <typename K, typename V>
constexpr uint32_t leaf_cap(int cls) {
  return cls == 0 ? 2048u : (cls == 1 ? 8192u : ((sizeof(K) == 8 && HasVal<V>::value) ? 8192u : 16384u));
}

}  // namespace dts

// Shared device-side definitions of the DovetailSort kernels for gfx950.
//
// Terminology (Alg. 2, Sections 3.1-3.5, 5):
//   task      one recursive subproblem: records [off, off+size) whose keys share
//             every bit at and above `hi`.  The data currently lives in buffer
//             `src` (0 = caller's array, 1 = ping-pong partner); the finished,
//             sorted subproblem must end in buffer `tgt`.
//   zone      an MSD zone: keys with the same digit (bits [shift, shift+w)), or,
//             for a learned root, the same splitter interval.
//   bucket id per zone one light bucket then its heavy keys ascending; the
//             overflow bucket (keys with a one bit in [top, hi)) is last.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dts {

constexpr int WAVE = 64;
constexpr int GMAX = 10;  // largest digit width (automatic choice never exceeds it for n < 2^32)

__host__ __device__ constexpr inline int nb_cap(int g) {
  // light buckets + at most 2^g / 2 heavy keys (a key must fill two of the
  // 2^g subsample slots) + the overflow bucket
  return (1 << g) + (g >= 1 ? (1 << (g - 1)) : 1) + 1;
}

// Digit width for a subproblem of n records: floor((floor(log2 n) + 1) / 3)
// clamped to [8, GMAX], the paper's "log2 of the cube root of n, capped by 8
// and 12" (Section 6) with an integer rounding; `override_g` > 0 wins.
__host__ __device__ inline int plan_gamma(uint32_t n, int override_g) {
  if (override_g > 0) return override_g > GMAX ? GMAX : override_g;
  int lg = 31 - __builtin_clz(n | 1u);
  int g = (lg + 1) / 3;
  if (g < 8) g = 8;
  if (g > GMAX) g = GMAX;
  return g;
}

// Per-task table slot inside a level's table arena (byte offsets).
struct SlotLayout {
  uint32_t light;   // (2^g + 1) x u32: light bucket id of each zone, then the overflow id
  uint32_t heavy;   // 2^(g-1) x u64: heavy keys ascending
  uint32_t starts;  // (nb_cap + 1) x u32: bucket starts relative to the task, then size
  uint32_t spl;     // 2^g x u64: splitters (learned root only)
  uint32_t bytes;   // slot size (multiple of 64)
};

__host__ __device__ inline SlotLayout slot_layout(int g, bool learned) {
  SlotLayout s;
  uint32_t o = 0;
  s.light = o;
  o += 4u * ((1u << g) + 1u);
  o = (o + 7u) & ~7u;
  s.heavy = o;
  o += 8u * (g >= 1 ? (1u << (g - 1)) : 1u);
  s.starts = o;
  o += 4u * (uint32_t)(nb_cap(g) + 1);
  o = (o + 7u) & ~7u;
  s.spl = o;
  if (learned) o += 8u * (1u << g);
  s.bytes = (o + 63u) & ~63u;
  return s;
}

enum TaskFlags : uint8_t {
  TF_SKIP_DISABLED = 1,  // overflow child: digits start at hi (no sampled-range skip)
  TF_LEARNED = 2,        // zones come from splitters (learned root)
  TF_SPLIT = 4,          // each zone's light keys are split at its heavy keys (no merge; see bucket_of)
};

struct Task {
  uint64_t off;        // absolute start index
  uint64_t cm_off;     // offset of this task's count matrix (u32 entries)
  uint64_t tab_off;    // byte offset of this task's table slot
  uint32_t size;       // records (>= 2)
  uint32_t n_root;     // size of the original problem (sample stride)
  uint32_t level;      // recursion depth
  uint32_t unit_base;  // first distribution unit of this task
  uint32_t n_chunks;   // distribution units of this task
  uint8_t hi, src, tgt, flags;
  uint8_t gamma, w, shift, top;
  uint16_t n_heavy, n_buckets;
};

// Leaf work: a local-memory sort, or a plain copy between buffers.
struct Leaf {
  uint64_t off;
  uint32_t size;
  uint8_t bits;   // sort by key bits below this (leaf sorts)
  uint8_t from;   // buffer holding the records
  uint8_t to;     // buffer receiving the sorted records
  uint8_t pad;
};

// A dovetail merge of one zone (Alg. 3) as an out-of-place gather.
struct Merge {
  uint64_t zone_off;   // absolute start of the zone
  uint64_t tab_off;    // the parent task's table slot (heavy keys, bucket starts)
  uint32_t b0;         // light records (sorted, in buffer b0_buf at zone_off)
  uint32_t m;          // heavy buckets
  uint32_t hbase;      // index of the first heavy key of the zone in the slot's heavy array
  uint32_t bstart;     // bucket id of the zone's light bucket
  uint32_t zone_rel;   // zone start relative to the parent task
  uint32_t unit_base;  // first gather unit
  uint32_t n_units;
  uint8_t b0_buf, hv_buf, out_buf, g;
};

// Counters the host reads back after each level (and error flags).
struct LevelCounters {
  uint32_t next_tasks;      // tasks created for the next level
  uint32_t next_units;      // their distribution units
  uint64_t next_cm;         // their count-matrix entries
  uint64_t next_tab;        // their table bytes
  uint32_t next_max_size;   // largest next-level task
  uint32_t next_records;    // records in next-level tasks (saturating)
  uint32_t leaf[6];         // leaf sorts per size class
  uint32_t copies;          // copy items
  uint32_t merges;          // merge items
  uint32_t merge_units;     // gather units
  uint32_t spills;          // heavy-value spill copies (pairs)
  uint32_t error;           // nonzero = a capacity check failed
  uint32_t cur_units;       // distribution units of this level (set by the prep step)
  uint32_t cur_tasks;       // tasks of this level (set by the prep step)
  uint32_t chunk;           // records per distribution unit (set by the prep step)
  // statistics (accumulated)
  unsigned long long st_heavy_keys, st_heavy_records, st_leaf_records, st_copy_records, st_merge_records,
      st_overflow_records, st_tasks, st_distributed;
  unsigned long long st_pair_records;  // records of paired leaves (also in st_leaf_records)
};

enum ErrBits : uint32_t {
  ERR_TASKS = 1, ERR_LEAF = 2, ERR_COPY = 4, ERR_MERGE = 8, ERR_UNITS = 16, ERR_CM = 32, ERR_TAB = 64,
  ERR_SEGMENTS = 128, ERR_MUNITS = 256, ERR_SPILL = 512,
  ERR_SCATTER = 1024,  // a scattered record fell outside its task (the counts were inconsistent)
};

// Capacities of the output lists the child-planning step appends to.
struct Caps {
  uint32_t tasks, leaf, copies, merges, munits, spills, units;
  uint32_t pad;
  uint64_t cm, tab;
};

template <typename K, typename V>
struct Bufs {
  K* k[2];
  V* v[2];  // unused when V is the empty type
};

struct NoVal {};
template <typename V>
struct HasVal {
  static constexpr bool value = true;
};
template <>
struct HasVal<NoVal> {
  static constexpr bool value = false;
};

// ---------------------------------------------------------------- utilities
template <typename K>
struct KeyBits;
template <>
struct KeyBits<uint32_t> {
  static constexpr int value = 32;
};
template <>
struct KeyBits<uint64_t> {
  static constexpr int value = 64;
};

template <typename K>
__host__ __device__ inline K mask_below(int b) {
  return b >= KeyBits<K>::value ? ~(K)0 : (((K)1 << b) - (K)1);
}

template <typename K>
__host__ __device__ inline K shr(K x, int s) {
  return s >= KeyBits<K>::value ? (K)0 : (x >> s);
}

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
constexpr uint64_t GOLD = 0x9E3779B97F4A7C15ull;

// Sample word i of a subproblem: a splitmix64 sequence keyed by (seed, task
// offset, level); position = floor(word * n / 2^64).
__host__ __device__ inline uint64_t sample_base(uint64_t seed, uint64_t off, uint32_t level) {
  uint64_t h0 = mix64(seed + GOLD);
  uint64_t h1 = mix64(h0 ^ off);
  return mix64(h1 ^ (uint64_t)(level + 1));
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// popcount(mask & lanes below me)
__device__ inline uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of the wave holding the same `nbits`-bit value as this lane, among
// the lanes where `valid` is set (wave-wide ballot match).
__device__ inline uint64_t match_peers(uint32_t v, int nbits, bool valid) {
  uint64_t peers = __ballot(valid);
  for (int i = 0; i < nbits; ++i) {
    uint32_t bit = (v >> i) & 1u;
    uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// The same peer mask through LDS: every lane ORs its lane bit into its
// value's slot of this wave's mask table, reads the slot back, then clears
// it (3 LDS operations instead of one ballot per bit).  LDS instructions of
// one wave execute in issue order, so the read sees every lane's OR and the
// clear follows every lane's read.  The table must start (and is left) zero.
//
// Each 64-bit slot is two 32-bit halves: lanes 0-31 OR into the low half and
// lanes 32-63 into the high half, so the OR and the clear are 32-bit
// operations and only the read is 64-bit.
__device__ inline uint64_t lds_match(unsigned long long* wm, uint32_t v, bool valid) {
  const uint32_t lane = threadIdx.x & (WAVE - 1);
  uint32_t* half = reinterpret_cast<uint32_t*>(wm + v) + (lane >> 5);
  const uint32_t bit = 1u << (lane & 31);
  unsigned long long peers = 0;
  if (valid) {
    __hip_atomic_fetch_or(half, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    peers = __hip_atomic_load(wm + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_store(half, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return peers;
}

// RANK_ATOMIC (keys without values only): a key's place among its tile's keys
// of the same bucket is an LDS atomic increment, in no particular order.
enum RankMode { RANK_BALLOT = 0, RANK_LDS = 1, RANK_HYBRID = 2, RANK_PIPE = 3, RANK_ATOMIC = 4 };

// Hybrid: ballots match the low 4 bits, the LDS table matches the remaining
// high bits (a table of at most 2^(nbits-4) slots, small enough that distinct
// slots sit in distinct banks); the peers are the intersection.
__device__ inline uint64_t hybrid_match(unsigned long long* wm, uint32_t v, int nbits, bool valid) {
  const int lo = nbits < 4 ? nbits : 4;
  uint64_t peers = match_peers(v & ((1u << lo) - 1u), lo, valid);
  if (nbits > lo) peers &= lds_match(wm, v >> lo, valid);
  return peers;
}

// Stable ranking of ITEMS items per lane against per-wave running counters
// `crow` (one per value), pipelined: all items' LDS matches are issued back
// to back, then every value's leader lane (lowest lane holding it) takes the
// running count with one atomic add-and-return, and its peers fetch that
// base from the leader lane.  pos[i] = running count before item i + rank
// among this item's peers.  LDS operations of a wave run in issue order, so
// the counts advance item by item exactly as in a sequential loop.
template <int ITEMS>
__device__ inline void rank_pipelined(const uint32_t (&v)[ITEMS], const bool (&valid)[ITEMS], unsigned long long* wm,
                                      uint32_t* crow, uint32_t (&pos)[ITEMS]) {
  uint64_t pe[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) pe[i] = lds_match(wm, v[i], valid[i]);
  uint32_t old[ITEMS], ldr[ITEMS], rk[ITEMS];
  const uint32_t lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    rk[i] = mbcnt(pe[i]);
    ldr[i] = valid[i] ? (uint32_t)__builtin_ctzll(pe[i]) : lane;
    old[i] = 0;
    if (valid[i] && rk[i] == 0) old[i] = atomicAdd(&crow[v[i]], (uint32_t)__popcll(pe[i]));
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) pos[i] = (uint32_t)__shfl((int)old[i], (int)ldr[i], WAVE) + rk[i];
}

// Exclusive scan of one value per thread across the workgroup.  `tmp` holds
// THREADS/64 + 1 words of LDS.  Returns the exclusive prefix; *total gets the sum.
// FREE_TMP = false leaves out the final barrier that frees `tmp` for reuse:
// for callers that pass another workgroup barrier before they scan again.
template <int THREADS, bool FREE_TMP = true>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  constexpr int WAVES = THREADS / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    uint32_t y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if constexpr (WAVES == 1) {
    // a one-wave block (possibly one of several waves of the workgroup)
    *total = __shfl(x, WAVE - 1, WAVE);
    return x - v;
  } else {
    const int wv = threadIdx.x / WAVE;
    if (lane == WAVE - 1) tmp[wv] = x;
    __syncthreads();
    // every thread adds up the wave totals itself (broadcast reads, no serial step)
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t t = tmp[w];
      before += w < wv ? t : 0u;
      all += t;
    }
    *total = all;
    if constexpr (FREE_TMP) __syncthreads();  // tmp is free again for the caller's next scan
    return x - v + before;
  }
}

// In-place exclusive scan of arr[0..n) in LDS by the whole workgroup; returns the total.
template <int THREADS>
__device__ inline uint32_t block_excl_scan_array(uint32_t* arr, int n, uint32_t* tmp) {
  const int per = (n + THREADS - 1) / THREADS;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += arr[i];
  uint32_t total;
  uint32_t run = block_excl_scan<THREADS>(s, tmp, &total);
  for (int i = b; i < e; ++i) {
    uint32_t t = arr[i];
    arr[i] = run;
    run += t;
  }
  __syncthreads();
  return total;
}

// ------------------------------------------------------- buffer loads
// Raw buffer loads (CDNA buffer instructions) over a resource covering
// [base, base + bytes): an access past the end returns zero instead of
// touching memory, so tile loads need no per-element clamp and keep one
// 32-bit offset per thread.  The fourth descriptor word is the gfx9-family
// default (no swizzle, 32-bit data format).
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// 16 bytes (4 u32 or 2 u64 keys) at a 16-byte aligned offset of the resource.
template <typename K>
__device__ inline void buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off_bytes, K* out) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u v = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off_bytes, 0, 0));
  if constexpr (sizeof(K) == 8) {
    out[0] = (K)v.x | ((K)v.y << 32);
    out[1] = (K)v.z | ((K)v.w << 32);
  } else {
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
}

template <typename K>
__device__ inline K buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off_bytes) {
  if constexpr (sizeof(K) == 8) {
    return __builtin_bit_cast(K, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off_bytes, 0, 0));
  } else {
    return (K)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off_bytes, 0, 0);
  }
}

// ------------------------------------------------------- bucket-id function
// Everything GetBucketId (Alg. 2) needs for one task, uniform across a workgroup.
template <typename K>
struct PlanRegs {
  K mask_hi;
  int top, shift, w;
  uint32_t nb;
  bool learned;
  bool top_full;  // top >= key width (no overflow test)
  bool heavy;     // the task has heavy keys (else the light id of zone z is z)
  bool hashed;    // the heavy keys are in the workgroup's hash table (set by the kernel)
  bool split;     // the split layout (TF_SPLIT)
};

template <typename K>
__device__ inline PlanRegs<K> plan_regs(const Task& t) {
  PlanRegs<K> p;
  p.mask_hi = mask_below<K>(t.hi);
  p.top = t.top;
  p.shift = t.shift;
  p.w = t.w;
  p.nb = t.n_buckets;
  p.learned = (t.flags & TF_LEARNED) != 0;
  p.top_full = t.top >= t.hi;
  p.heavy = t.n_heavy != 0;
  p.hashed = false;
  p.split = (t.flags & TF_SPLIT) != 0;
  return p;
}

// Hash table of a task's heavy keys (at most 128 of them), built in LDS by
// the workgroups that distribute the task: HT_SLOTS words, each holding up to
// HT_WAYS indices into the heavy-key array (one byte each, filled from the
// low byte up, 0xFF = empty).  A key is heavy exactly when one of the
// indices in its slot names an equal key.
constexpr int HT_BITS = 9;
constexpr int HT_SLOTS = 1 << HT_BITS;
constexpr int HT_WAYS = 4;
constexpr int HT_MAX_KEYS = 128;  // indices fit a byte below 0xFF

// Slot of a key: multiplicative (Fibonacci) hashing of its (folded) 32 bits.
template <typename K>
__device__ inline uint32_t heavy_slot(K key) {
  uint32_t x = (uint32_t)key;
  if constexpr (sizeof(K) == 8) x ^= (uint32_t)((uint64_t)key >> 32);
  return (x * 0x9E3779B1u) >> (32 - HT_BITS);
}

// Bucket id of `key`: overflow if a bit in [top, hi) is set (Section 5); else
// the heavy id if the key is one of its zone's heavy keys; else the zone's
// light id.  L (light ids, 2^w + 1 entries), H (heavy keys), SPL
// (splitters, learned root) and HT (the heavy-key hash table, used when
// p.hashed) are in LDS.  Without the table the heavy keys of the key's zone
// are binary-searched.
//
// Split layout (p.split, dovetailing during distribution, a variant derived
// from Section 3.4): zone z with heavy keys h_1 < ... < h_m has the buckets
// light_0, h_1, light_1, ..., h_m, light_m in key order, so that a heavy
// bucket lands between the light keys below and above it and no merge is
// needed.  With the heavy keys' global ascending array H, a heavy key H[e]
// takes id z + 2e + 1 and a light key z + 2 * (heavy keys below it), and
// L[z] = z + 2 * (heavy keys of lower zones).  Only the SPLIT kernel
// variants carry this path (so that the default ones carry none of its
// code); there it serves the tasks marked split, by binary search.
template <typename K, bool SPLIT = false>
__device__ inline uint32_t bucket_of(K key, const PlanRegs<K>& p, const uint32_t* L, const K* H, const K* SPL,
                                     const uint32_t* HT) {
  K low = key & p.mask_hi;
  uint32_t z;
  if (p.learned) {
    // number of splitters <= key (2^w - 1 of them)
    uint32_t lo = 0, n = (1u << p.w) - 1u;
    while (n > 0) {
      uint32_t half = n >> 1;
      if (SPL[lo + half] <= key) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    z = lo;
  } else {
    if (!p.top_full && shr<K>(low, p.top) != 0) return p.nb - 1u;
    z = (uint32_t)(shr<K>(low, p.shift) & (K)((1u << p.w) - 1u));
  }
  if (!p.heavy) return z;
  uint32_t lid = L[z];
  if constexpr (SPLIT) {
    if (p.split) {
      const uint32_t m = (L[z + 1] - lid - 1u) >> 1;
      const uint32_t base = (lid - z) >> 1;
      uint32_t lo = base, n = m;
      while (n > 0) {
        const uint32_t half = n >> 1;
        if (H[lo + half] < key) {
          lo += half + 1;
          n -= half + 1;
        } else {
          n = half;
        }
      }
      if (lo < base + m && H[lo] == key) return z + 2u * lo + 1u;
      return z + 2u * lo;
    }
  }
  if (p.hashed) {
    // an equal heavy key lies in this key's zone; its bucket follows the
    // zone's light bucket in the order of the heavy-key array
    // (most slots hold at most one key: the first index is tested without a
    // branch; its entry is read even when empty, an in-bounds LDS read)
    uint32_t w = HT[heavy_slot<K>(key)];
    const uint32_t e0 = w & 0xFFu;
    const K h0 = H[e0 & (HT_MAX_KEYS - 1)];
    const bool hit0 = (e0 != 0xFFu) & (h0 == key);
    uint32_t id = hit0 ? z + 1u + e0 : lid;
    w >>= 8;
    if (!hit0 && (w & 0xFFu) != 0xFFu) {
#pragma unroll
      for (int j = 1; j < HT_WAYS; ++j) {
        const uint32_t e = w & 0xFFu;
        if (e == 0xFFu) break;
        if (H[e] == key) {
          id = z + 1u + e;
          break;
        }
        w >>= 8;
      }
    }
    return id;
  }
  uint32_t m = L[z + 1] - lid - 1u;
  if (m) {
    uint32_t base = lid - z, lo = base, n = m;
    while (n > 0) {
      uint32_t half = n >> 1;
      if (H[lo + half] < key) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    if (lo < base + m && H[lo] == key) return z + 1u + lo;
  }
  return lid;
}

}  // namespace dts

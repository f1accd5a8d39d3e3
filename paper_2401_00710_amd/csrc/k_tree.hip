// Step 3 (Section 3.3: recurse into light buckets only; heavy buckets are
// finished) and Step 4 (Section 3.4, Alg. 3: the dovetail merge) of Alg. 2,
// plus the seeding of the batched form.
//
// Buffer rule.  Every subproblem P has a source buffer src(P) (where its data
// is), dst(P) = the other buffer (where its distribution writes), and a target
// tgt(P) (where its sorted result must end).  A zone without heavy keys hands
// its light bucket the parent's target.  A zone with heavy keys hands its
// light bucket the OTHER buffer as target, so that its merge is an
// out-of-place gather: light records come from 1 - tgt(P), heavy records from
// dst(P) (keys-only: heavy keys are constants and are never read), and the
// zone is written to tgt(P).  For records with values, when dst(P) = tgt(P)
// the heavy values are first copied ("spilled") to the same range of src(P),
// which nothing else uses after P's distribution.
#include <type_traits>

#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

constexpr uint32_t MERGE_TILE = 4096;       // outputs per gather unit

// Kinds of work a finished distribution hands on (one output list each).
enum Kind : int { KD_TASK = 0, KD_LEAF0 = 1, KD_COPY = 1 + LEAF_CLASSES, KD_MERGE, KD_MUNIT, KD_SPILL, KD_PAIR, KD_N };

struct Child {
  uint64_t off;
  uint32_t c;
  uint8_t hi, buf, tgt, skip;
  int kind;        // -1: nothing to do
  uint32_t slot;   // offset within the workgroup's reservation for `kind`
};

// What happens to a bucket of c records whose keys share every bit at and
// above `hi`, lying in buffer `buf`, to end sorted in buffer `tgt`.
__device__ inline int child_kind(const LevelArgs& a, uint32_t c, int hi, int buf, int tgt, uint32_t* units) {
  *units = 1;
  if (c == 0) return -1;
  if (c == 1 || hi == 0) {  // finished: one record or all keys equal
    if (buf == tgt) return -1;
    *units = pieces_of(c);
    return KD_COPY;
  }
  if (c <= a.cutoff) {
    int cls = LEAF_CLASSES - 1;
    for (int k = LEAF_CLASSES - 2; k >= 0; --k)
      if (c <= a.leaf_max[k]) cls = k;
    return KD_LEAF0 + cls;
  }
  if (c <= a.leaf_max[LEAF_PAIR]) {  // two half leaves and their merge (0: not for this layout)
    *units = 2;
    return KD_PAIR;
  }
  return KD_TASK;
}

__device__ inline uint32_t* kind_counter(LevelCounters* ctr, int kind) {
  if (kind == KD_TASK) return &ctr->next_tasks;
  if (kind >= KD_LEAF0 && kind < KD_LEAF0 + LEAF_CLASSES) return &ctr->leaf[kind - KD_LEAF0];
  if (kind == KD_COPY) return &ctr->copies;
  if (kind == KD_MERGE) return &ctr->merges;
  if (kind == KD_MUNIT) return &ctr->merge_units;
  if (kind == KD_PAIR) return &ctr->leaf[LEAF_PAIR];
  return &ctr->spills;
}

__device__ inline uint32_t kind_cap(const LevelArgs& a, int kind) {
  if (kind == KD_TASK) return a.caps.tasks;
  if ((kind >= KD_LEAF0 && kind < KD_LEAF0 + LEAF_CLASSES) || kind == KD_PAIR) return a.caps.leaf;
  if (kind == KD_COPY) return a.caps.copies;
  if (kind == KD_MERGE) return a.caps.merges;
  if (kind == KD_MUNIT) return a.caps.munits;
  return a.caps.spills;
}

__device__ inline void write_child(const LevelArgs& a, const Child& ch, uint32_t base, uint32_t n_root, uint32_t level,
                                   int g_override) {
  if (ch.kind < 0) return;
  const uint32_t i = base + ch.slot;
  if (ch.kind == KD_COPY) {
    for (uint32_t p = 0, k = 0; k < pieces_of(ch.c); p += COPY_PIECE, ++k) {
      if (i + k >= a.caps.copies) {
        atomicOr(&a.ctr->error, ERR_COPY);
        return;
      }
      Leaf l;
      l.off = ch.off + p;
      l.size = min(COPY_PIECE, ch.c - p);
      l.bits = 0;
      l.from = ch.buf;
      l.to = ch.tgt;
      l.pad = 0;
      a.copies[i + k] = l;
    }
    return;
  }
  if (ch.kind >= KD_LEAF0 && ch.kind < KD_LEAF0 + LEAF_CLASSES) {
    if (i >= a.caps.leaf) {
      atomicOr(&a.ctr->error, ERR_LEAF);
      return;
    }
    Leaf l;
    l.off = ch.off;
    l.size = ch.c;
    l.bits = ch.hi;
    l.from = ch.buf;
    l.to = ch.tgt;
    l.pad = 0;
    a.leaf[ch.kind - KD_LEAF0][i] = l;
    return;
  }
  if (ch.kind == KD_PAIR) {
    // halves sorted into the buffer other than the target, merged into the target (pad)
    if (i + 1 >= a.caps.leaf) {
      atomicOr(&a.ctr->error, ERR_LEAF);
      return;
    }
    const uint32_t h = ch.c / 2;
    Leaf l;
    l.off = ch.off;
    l.size = h;
    l.bits = ch.hi;
    l.from = ch.buf;
    l.to = (uint8_t)(1 - ch.tgt);
    l.pad = ch.tgt;
    a.leaf[LEAF_PAIR][i] = l;
    l.off = ch.off + h;
    l.size = ch.c - h;
    a.leaf[LEAF_PAIR][i + 1] = l;
    return;
  }
  // next-level task
  if (i >= a.caps.tasks) {
    atomicOr(&a.ctr->error, ERR_TASKS);
    return;
  }
  Task t;
  t.off = ch.off;
  t.cm_off = 0;
  t.tab_off = 0;
  t.size = ch.c;
  t.n_root = n_root;
  t.level = level;
  t.unit_base = 0;
  t.n_chunks = 0;
  t.hi = ch.hi;
  t.src = ch.buf;
  t.tgt = ch.tgt;
  t.flags = ch.skip ? TF_SKIP_DISABLED : 0;
  t.gamma = (uint8_t)plan_gamma(ch.c, g_override);
  t.w = 0;
  t.shift = 0;
  t.top = 0;
  t.n_heavy = 0;
  t.n_buckets = 0;
  a.next[i] = t;
}

// Reserve this workgroup's ranges in every output list: LDS counters give
// local offsets, then one global atomic per list.
struct Reserve {
  uint32_t cnt[KD_N];
  uint32_t base[KD_N];
  unsigned long long st_leaf, st_copy, st_heavy, st_merge, st_over, st_pair;
  uint32_t max_size, records;
};

__device__ inline uint32_t reserve_local(Reserve* r, int kind, uint32_t units) {
  return atomicAdd(&r->cnt[kind], units);
}

__device__ inline void reserve_global(const LevelArgs& a, Reserve* r) {
  if (threadIdx.x < KD_N) {
    const int k = threadIdx.x;
    r->base[k] = r->cnt[k] ? atomicAdd(kind_counter(a.ctr, k), r->cnt[k]) : 0u;
    if (r->cnt[k] && r->base[k] + r->cnt[k] > kind_cap(a, k)) atomicOr(&a.ctr->error, ERR_TASKS << 16);
  }
  if (threadIdx.x == WAVE) {
    LevelCounters* c = a.ctr;
    if (r->st_leaf) atomicAdd(&c->st_leaf_records, r->st_leaf);
    if (r->st_copy) atomicAdd(&c->st_copy_records, r->st_copy);
    if (r->st_heavy) atomicAdd(&c->st_heavy_records, r->st_heavy);
    if (r->st_merge) atomicAdd(&c->st_merge_records, r->st_merge);
    if (r->st_over) atomicAdd(&c->st_overflow_records, r->st_over);
    if (r->st_pair) atomicAdd(&c->st_pair_records, r->st_pair);
    if (r->max_size) atomicMax(&c->next_max_size, r->max_size);
    if (r->records) atomicAdd(&c->next_records, r->records);
  }
}

__device__ inline void reserve_init(Reserve* r) {
  if (threadIdx.x < KD_N) r->cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    r->st_leaf = r->st_copy = r->st_heavy = r->st_merge = r->st_over = r->st_pair = 0;
    r->max_size = 0;
    r->records = 0;
  }
}

__device__ inline Child plan_child(const LevelArgs& a, Reserve* r, uint64_t off, uint32_t c, int hi, int buf, int tgt,
                                   bool skip) {
  Child ch;
  ch.off = off;
  ch.c = c;
  ch.hi = (uint8_t)hi;
  ch.buf = (uint8_t)buf;
  ch.tgt = (uint8_t)tgt;
  ch.skip = skip;
  uint32_t units;
  ch.kind = child_kind(a, c, hi, buf, tgt, &units);
  ch.slot = 0;
  if (ch.kind >= 0) {
    ch.slot = reserve_local(r, ch.kind, units);
    if (ch.kind == KD_COPY) atomicAdd(&r->st_copy, (unsigned long long)c);
    if ((ch.kind >= KD_LEAF0 && ch.kind < KD_LEAF0 + LEAF_CLASSES) || ch.kind == KD_PAIR)
      atomicAdd(&r->st_leaf, (unsigned long long)c);
    if (ch.kind == KD_PAIR) atomicAdd(&r->st_pair, (unsigned long long)c);
    if (ch.kind == KD_TASK) {
      atomicMax(&r->max_size, c);
      atomicAdd(&r->records, c);
    }
  }
  return ch;
}

// Batched form: every segment is the root of its own sort.
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_seed(LevelArgs a, const uint64_t* seg, uint32_t n_seg, uint64_t n_total) {
  __shared__ Reserve r;
  reserve_init(&r);
  __syncthreads();
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  Child ch;
  ch.kind = -1;
  if (s < n_seg) {
    const uint64_t b = seg[s], e = seg[s + 1];
    if (e < b || e > n_total || (s == 0 && b != 0) || (s + 1 == n_seg && e != n_total) || e - b >= (1ull << 32)) {
      atomicOr(&a.ctr->error, ERR_SEGMENTS);
    } else {
      ch = plan_child(a, &r, b, (uint32_t)(e - b), a.key_bits, 0, 0, false);
    }
  }
  __syncthreads();
  reserve_global(a, &r);
  __syncthreads();
  if (ch.kind >= 0) write_child(a, ch, r.base[ch.kind], ch.c, 0, a.g_override);
}

template <typename K, typename V>
void launch_seed_segments(const LevelArgs& a, const uint64_t* seg_off, uint32_t n_seg, uint64_t n_total,
                          hipStream_t s) {
  if (n_seg == 0) return;
  hipLaunchKernelGGL((k_seed<K, V>), dim3((n_seg + 255) / 256), dim3(256), 0, s, a, seg_off, n_seg, n_total);
}

// Child planning: one workgroup per task, one thread per zone (at most
// 2^GMAX / 256 = 4 zones per thread, plus the overflow bucket on thread 0).
// SPLITK: the variant for sorts with the split layout (MV_SPLIT), which adds
// its bucket-by-bucket path; the default kernel carries none of its code.
template <typename K, typename V, bool SPLITK>
__global__ __launch_bounds__(256) void k_children(LevelArgs a) {
  constexpr int ZPT = (1 << GMAX) / 256;
  constexpr bool HV = HasVal<V>::value;
  __shared__ Reserve r;
  const uint32_t n_tasks = a.ctr->cur_tasks;
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
  const Task t = a.tasks[ti];
  if (t.n_chunks == 0) continue;
  reserve_init(&r);
  __syncthreads();
  const bool learned = (t.flags & TF_LEARNED) != 0;
  const SlotLayout sl = slot_layout(t.gamma, learned);
  const uint8_t* slot = a.tab + t.tab_off;
  const uint32_t* L = (const uint32_t*)(slot + sl.light);
  const uint32_t* st = (const uint32_t*)(slot + sl.starts);
  const uint64_t* SPL = (const uint64_t*)(slot + sl.spl);
  const int dst = 1 - t.src;
  const uint32_t zones = 1u << t.w;
  const uint32_t ob = t.n_buckets - 1u;  // the overflow bucket
  // A task whose digit took every remaining bit, with no heavy keys and an
  // empty overflow bucket, leaves only finished buckets: when they lie in the
  // wrong buffer, the whole task range is copied as one item list instead of
  // bucket by bucket (the buckets are adjacent and in order).
  const bool whole_copy = !learned && t.shift == 0 && t.n_heavy == 0 && st[ob + 1] == st[ob] && dst != t.tgt;
  if (SPLITK && (t.flags & TF_SPLIT) && t.n_heavy != 0 && !learned) {
    // Split layout: every light sub-bucket is a child with the task's target
    // (no merge follows); heavy buckets are finished where they landed.
    constexpr int SPT = (nb_cap(GMAX) + 255) / 256;  // buckets per thread
    Child cs[SPT + 1];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      cs[k].kind = -1;
      const uint32_t b = threadIdx.x + 256u * k;
      if (b >= ob) continue;
      uint32_t lo = 0, n = zones;  // the zone of b: the last z with L[z] <= b
      while (n > 0) {
        const uint32_t half = n >> 1;
        if (L[lo + half] <= b) {
          lo += half + 1;
          n -= half + 1;
        } else {
          n = half;
        }
      }
      const bool heavy = ((b - L[lo - 1u]) & 1u) != 0u;
      const uint32_t c = st[b + 1] - st[b];
      if (heavy && c) atomicAdd(&r.st_heavy, (unsigned long long)c);
      cs[k] = plan_child(a, &r, t.off + st[b], c, heavy ? 0 : t.shift, dst, t.tgt, false);
    }
    cs[SPT].kind = -1;
    if (threadIdx.x == 0) {
      const uint32_t c = st[ob + 1] - st[ob];
      if (c) atomicAdd(&r.st_over, (unsigned long long)c);
      cs[SPT] = plan_child(a, &r, t.off + st[ob], c, t.hi, dst, t.tgt, true);
    }
    __syncthreads();
    reserve_global(a, &r);
    if (threadIdx.x == 2 * WAVE) {
      atomicAdd(&a.ctr->st_heavy_keys, (unsigned long long)t.n_heavy);
      atomicAdd(&a.ctr->st_tasks, 1ull);
      atomicAdd(&a.ctr->st_distributed, (unsigned long long)t.size);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= SPT; ++k)
      if (cs[k].kind >= 0) write_child(a, cs[k], r.base[cs[k].kind], t.n_root, t.level + 1, a.g_override);
    __syncthreads();
    continue;
  }
  Child ch[ZPT + 1];
  Merge mg[ZPT];
  uint32_t mslot[ZPT], uslot[ZPT], sslot[ZPT], spieces[ZPT];
#pragma unroll
  for (int k = 0; k < ZPT; ++k) {
    ch[k].kind = -1;
    mslot[k] = 0xFFFFFFFFu;
    const uint32_t z = threadIdx.x + 256u * k;
    if (z >= zones || whole_copy) continue;
    const uint32_t lid = L[z];
    const uint32_t m = L[z + 1] - lid - 1u;
    const uint32_t s0 = st[lid];
    const uint32_t c0 = st[lid + 1] - s0;
    int ctgt = t.tgt;
    if (m > 0) {
      const bool in_tgt = zone_in_target(a.merge_variant);
      ctgt = in_tgt ? t.tgt : 1 - t.tgt;
      const uint32_t zend = st[lid + m + 1];
      const uint32_t zsize = zend - s0;
      Merge& g = mg[k];
      g.zone_off = t.off + s0;
      g.tab_off = t.tab_off;
      g.b0 = c0;
      g.m = m;
      g.hbase = lid - z;
      g.bstart = lid;
      g.zone_rel = s0;
      g.n_units = zsize / MERGE_TILE + (zsize % MERGE_TILE != 0u ? 1u : 0u);
      g.b0_buf = (uint8_t)ctgt;
      g.hv_buf = (uint8_t)dst;
      g.out_buf = (uint8_t)t.tgt;
      g.g = t.gamma;
      spieces[k] = 0;
      if (in_tgt ? (dst != t.tgt && zsize > c0) : (HV && dst == t.tgt && zsize > c0)) {
        // gather: heavy values would be overwritten by the gather, so they are
        // copied to src first.  Zone-in-target variants: the heavy runs are
        // copied next to the light run in the target buffer.
        spieces[k] = pieces_of(zsize - c0);
        g.hv_buf = (uint8_t)(in_tgt ? t.tgt : t.src);
        sslot[k] = reserve_local(&r, KD_SPILL, spieces[k]);
        atomicAdd(&r.st_copy, (unsigned long long)(zsize - c0));
      }
      mslot[k] = reserve_local(&r, KD_MERGE, 1);
      uslot[k] = reserve_local(&r, KD_MUNIT, g.n_units);
      atomicAdd(&r.st_heavy, (unsigned long long)(zsize - c0));
      atomicAdd(&r.st_merge, (unsigned long long)zsize);
    }
    int chi = t.shift;
    if (learned) {
      // zone z holds keys in [s_z, s_{z+1} - 1]; they share the bits above the
      // highest bit where the two ends differ
      const uint64_t lo = z == 0 ? 0ull : SPL[z - 1];
      const uint64_t hi_incl = z + 1 < zones ? SPL[z] - 1ull : (uint64_t)mask_below<K>(t.hi);
      const uint64_t d = lo ^ hi_incl;
      chi = (lo > hi_incl) ? 0 : (d ? 64 - __builtin_clzll(d) : 0);
    }
    ch[k] = plan_child(a, &r, t.off + s0, c0, chi, dst, ctgt, false);
  }
  ch[ZPT].kind = -1;
  if (threadIdx.x == 0) {
    if (whole_copy) {
      ch[ZPT] = plan_child(a, &r, t.off, t.size, 0, dst, t.tgt, false);
    } else {
      const uint32_t c = st[ob + 1] - st[ob];
      if (c) atomicAdd(&r.st_over, (unsigned long long)c);
      ch[ZPT] = plan_child(a, &r, t.off + st[ob], c, t.hi, dst, t.tgt, true);
    }
  }
  __syncthreads();
  reserve_global(a, &r);
  if (threadIdx.x == 2 * WAVE) {
    atomicAdd(&a.ctr->st_heavy_keys, (unsigned long long)t.n_heavy);
    atomicAdd(&a.ctr->st_tasks, 1ull);
    atomicAdd(&a.ctr->st_distributed, (unsigned long long)t.size);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k <= ZPT; ++k)
    if (ch[k].kind >= 0)
      write_child(a, ch[k], r.base[ch[k].kind], t.n_root, t.level + 1, learned ? a.g_learned_child : a.g_override);
#pragma unroll
  for (int k = 0; k < ZPT; ++k) {
    if (mslot[k] == 0xFFFFFFFFu) continue;
    Merge g = mg[k];
    const uint32_t mi = r.base[KD_MERGE] + mslot[k];
    g.unit_base = r.base[KD_MUNIT] + uslot[k];
    if (mi >= a.caps.merges || g.unit_base + g.n_units > a.caps.munits) {
      atomicOr(&a.ctr->error, ERR_MERGE);
      continue;
    }
    if (spieces[k]) {
      const uint32_t si = r.base[KD_SPILL] + sslot[k];
      const uint32_t zsize = g.n_units ? st[g.bstart + g.m + 1] - st[g.bstart] : 0;
      for (uint32_t p = g.b0, q = 0; q < pieces_of(zsize - g.b0); p += COPY_PIECE, ++q) {
        if (si + q >= a.caps.spills) {
          atomicOr(&a.ctr->error, ERR_SPILL);
          break;
        }
        Leaf l;
        l.off = g.zone_off + p;
        l.size = min(COPY_PIECE, zsize - p);
        l.bits = 0;
        l.from = (uint8_t)dst;
        l.to = g.hv_buf;
        l.pad = 0;
        a.spills[si + q] = l;
      }
    }
    a.merges[mi] = g;
  }
  __syncthreads();
  }
}

template <typename K, typename V>
void launch_children(const LevelArgs& a, Bufs<K, V> b, hipStream_t s) {
  (void)b;
  if (a.merge_variant == MV_SPLIT)
    hipLaunchKernelGGL((k_children<K, V, true>), dim3(a.grid_tasks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_children<K, V, false>), dim3(a.grid_tasks), dim3(256), 0, s, a);
}

// ------------------------------------------------------------------ copies
// d[0..n) = s[0..n).  When the two ranges share their alignment modulo 16
// bytes (always for the sorts' own buffers, whose bases are 256-byte aligned),
// the body moves in 16-byte words, four loads in flight per thread before the
// stores; a head up to the first 16-byte boundary and the tail move record by
// record.
template <typename T>
__device__ inline void copy_range(T* __restrict__ d, const T* __restrict__ s, uint32_t n) {
  const uintptr_t sa = (uintptr_t)s, da = (uintptr_t)d;
  if (((sa ^ da) & 15u) != 0u) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
    return;
  }
  constexpr uint32_t PER = 16u / (uint32_t)sizeof(T);  // records per 16-byte word
  const uint32_t head = min(n, (uint32_t)(((16u - (uint32_t)(sa & 15u)) & 15u) / (uint32_t)sizeof(T)));
  const uint32_t nv = (n - head) / PER;
  const uint32_t tail = head + nv * PER;
  for (uint32_t i = threadIdx.x; i < head; i += blockDim.x) d[i] = s[i];
  for (uint32_t i = tail + threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
  const uint4* sv = reinterpret_cast<const uint4*>(s + head);
  uint4* dv = reinterpret_cast<uint4*>(d + head);
  const uint32_t B = blockDim.x;
  uint32_t i = threadIdx.x;
  for (; i + 3u * B < nv; i += 4u * B) {
    const uint4 a = sv[i], b = sv[i + B], c = sv[i + 2u * B], e = sv[i + 3u * B];
    dv[i] = a;
    dv[i + B] = b;
    dv[i + 2u * B] = c;
    dv[i + 3u * B] = e;
  }
  for (; i < nv; i += B) dv[i] = sv[i];
}

template <typename K, typename V>
__global__ __launch_bounds__(256) void k_copy(const Leaf* items, const uint32_t* count, uint32_t cap, Bufs<K, V> bf) {
  const uint32_t n_items = min(*count, cap);
  for (uint32_t ci = blockIdx.x; ci < n_items; ci += gridDim.x) {
    const Leaf it = items[ci];
    copy_range<K>(bf.k[it.to] + it.off, bf.k[it.from] + it.off, it.size);
    if constexpr (HasVal<V>::value) copy_range<V>(bf.v[it.to] + it.off, bf.v[it.from] + it.off, it.size);
  }
}

template <typename K, typename V>
void launch_copy(const Leaf* items, const uint32_t* count, uint32_t cap, uint32_t grid, Bufs<K, V> b, hipStream_t s) {
  if (grid == 0 || cap == 0) return;
  hipLaunchKernelGGL((k_copy<K, V>), dim3(grid), dim3(256), 0, s, items, count, cap, b);
}

// Copy items of a plain copy of n records from buffer 0 to buffer 1, cut
// like the sorts' copies (pieces of COPY_PIECE records); count = items.
__global__ __launch_bounds__(256) void k_copy_items(Leaf* items, uint32_t* count, uint64_t n) {
  const uint32_t n_items = pieces_of((uint32_t)n);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n_items; i += gridDim.x * 256) {
    Leaf l;
    l.off = (uint64_t)i * COPY_PIECE;
    l.size = (uint32_t)min((uint64_t)COPY_PIECE, n - l.off);
    l.bits = 0;
    l.from = 0;
    l.to = 1;
    l.pad = 0;
    items[i] = l;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = n_items;
}

void launch_copy_items(Leaf* items, uint32_t* count, uint64_t n, hipStream_t s) {
  const uint32_t n_items = pieces_of((uint32_t)n);
  hipLaunchKernelGGL(k_copy_items, dim3(n_items / 256 + 1), dim3(256), 0, s, items, count, n);
}

// ------------------------------------------------------------------ merges
__global__ __launch_bounds__(64) void k_merge_units(const Merge* m, const uint32_t* count, uint32_t cap,
                                                     uint2* munits) {
  const uint32_t n_merges = min(*count, cap);
  for (uint32_t mi = blockIdx.x; mi < n_merges; mi += gridDim.x) {
    const Merge mg = m[mi];
    for (uint32_t j = threadIdx.x; j < mg.n_units; j += 64) munits[mg.unit_base + j] = make_uint2(mi, j);
  }
}

void launch_merge_units(const Merge* m, const uint32_t* count, uint32_t cap, uint32_t grid, uint2* munits,
                        hipStream_t s) {
  if (grid == 0 || cap == 0) return;
  hipLaunchKernelGGL(k_merge_units, dim3(grid), dim3(64), 0, s, m, count, cap, munits);
}

// Alg. 3, first line: p_i = lower_bound(B0, h_i) + sum_{j<i} |B_j| for every
// heavy bucket of the zone (B0 is sorted and holds no heavy key).  The result
// is stored in the slot's light-id area (free once the level's children are
// planned), at the heavy key's index.
template <typename K>
__global__ __launch_bounds__(64) void k_merge_pos(const Merge* m, const uint32_t* count, uint32_t cap, uint8_t* tab,
                                                   const K* k0, const K* k1) {
  const uint32_t n_merges = min(*count, cap);
  for (uint32_t mi = blockIdx.x; mi < n_merges; mi += gridDim.x) {
  const Merge mg = m[mi];
  const SlotLayout sl = slot_layout(mg.g, false);
  uint8_t* slot = tab + mg.tab_off;
  uint32_t* P = (uint32_t*)(slot + sl.light);
  const uint64_t* H = (const uint64_t*)(slot + sl.heavy);
  const uint32_t* st = (const uint32_t*)(slot + sl.starts);
  const K* b0 = (mg.b0_buf ? k1 : k0) + mg.zone_off;
  const int lane = threadIdx.x;
  uint32_t carry = 0;
  for (uint32_t i0 = 0; i0 < mg.m; i0 += 64) {
    const uint32_t i = i0 + lane;
    uint32_t sz = 0, lb = 0;
    if (i < mg.m) {
      const uint32_t bid = mg.bstart + 1 + i;
      sz = st[bid + 1] - st[bid];
      const K h = (K)H[mg.hbase + i];
      uint32_t lo = 0, n = mg.b0;
      while (n > 0) {
        const uint32_t half = n >> 1;
        if (b0[lo + half] < h) {
          lo += half + 1;
          n -= half + 1;
        } else {
          n = half;
        }
      }
      lb = lo;
    }
    uint32_t x = sz;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (i < mg.m) P[mg.hbase + i] = lb + carry + x - sz;
    carry += __shfl(x, 63, 64);
  }
  }
}

// Out-of-place gather of a zone: output q takes heavy bucket i when
// p_i <= q < p_i + |B_i|, else light record q - (heavy records before q).
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_merge_gather(const Merge* m, const uint2* munits, const uint32_t* count,
                                                      uint32_t cap, uint8_t* tab, Bufs<K, V> bf) {
  constexpr int MAXH = 1 << (GMAX - 1);
  __shared__ uint32_t P[MAXH], S[MAXH], PRE[MAXH];
  __shared__ K HK[MAXH];
  __shared__ uint32_t tmp[5];
  __shared__ uint32_t s_run[3];  // the unit's run: kind (0 mixed, 1 one heavy run, 2 one light stretch), index, offset
  const uint32_t n_units = min(*count, cap);
  for (uint32_t ui = blockIdx.x; ui < n_units; ui += gridDim.x) {
  const uint2 u = munits[ui];
  const Merge mg = m[u.x];
  const SlotLayout sl = slot_layout(mg.g, false);
  const uint8_t* slot = tab + mg.tab_off;
  const uint32_t* gP = (const uint32_t*)(slot + sl.light);
  const uint64_t* gH = (const uint64_t*)(slot + sl.heavy);
  const uint32_t* st = (const uint32_t*)(slot + sl.starts);
  for (uint32_t i = threadIdx.x; i < mg.m; i += 256) {
    P[i] = gP[mg.hbase + i];
    const uint32_t bid = mg.bstart + 1 + i;
    S[i] = st[bid + 1] - st[bid];
    PRE[i] = S[i];
    HK[i] = (K)gH[mg.hbase + i];
  }
  __syncthreads();
  block_excl_scan_array<256>(PRE, (int)mg.m, tmp);
  const uint32_t zsize = st[mg.bstart + mg.m + 1] - st[mg.bstart];
  const uint32_t q0 = u.y * MERGE_TILE;
  const uint32_t qn = min((uint32_t)MERGE_TILE, zsize - q0);  // outputs of this unit
  const K* lk = bf.k[mg.b0_buf] + mg.zone_off;
  K* ok = bf.k[mg.out_buf] + mg.zone_off;
  // output q: lo = heavy runs starting at or before q; inside run lo - 1, or
  // light record q - before
  auto locate = [&](uint32_t q, uint32_t* lo_out, bool* heavy, uint32_t* hidx, uint32_t* before) {
    uint32_t lo = 0, n = mg.m;
    while (n > 0) {
      const uint32_t half = n >> 1;
      if (P[lo + half] <= q) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    *lo_out = lo;
    *heavy = false;
    *hidx = 0;
    *before = 0;
    if (lo > 0) {
      const uint32_t i = lo - 1;
      if (q < P[i] + S[i]) {
        *heavy = true;
        *hidx = i;
      } else {
        *before = PRE[i] + S[i];
      }
    }
  };
  // a unit inside one heavy run (a constant) or one light stretch (a shifted
  // copy) needs no search per output: heavy keys fill most of a skewed zone
  if (threadIdx.x == 0) {
    uint32_t lo_a, lo_b, h_a, h_b, be_a, be_b;
    bool hv_a, hv_b;
    locate(q0, &lo_a, &hv_a, &h_a, &be_a);
    locate(q0 + qn - 1u, &lo_b, &hv_b, &h_b, &be_b);
    s_run[0] = (hv_a && hv_b && h_a == h_b) ? 1u : ((!hv_a && !hv_b && lo_a == lo_b) ? 2u : 0u);
    s_run[1] = h_a;
    s_run[2] = be_a;
  }
  __syncthreads();
  const uint32_t kind = s_run[0];
  if (kind == 1u) {
    const uint32_t i = s_run[1];
    const K hk = HK[i];
    for (uint32_t qi = threadIdx.x; qi < qn; qi += 256) ok[q0 + qi] = hk;
    if constexpr (HasVal<V>::value) {
      V* ov = bf.v[mg.out_buf] + mg.zone_off;
      const V* hv = bf.v[mg.hv_buf] + mg.zone_off + mg.b0 + PRE[i];
      for (uint32_t qi = threadIdx.x; qi < qn; qi += 256) ov[q0 + qi] = hv[q0 + qi - P[i]];
    }
  } else if (kind == 2u) {
    const uint32_t before = s_run[2];
    for (uint32_t qi = threadIdx.x; qi < qn; qi += 256) ok[q0 + qi] = lk[q0 + qi - before];
    if constexpr (HasVal<V>::value) {
      V* ov = bf.v[mg.out_buf] + mg.zone_off;
      const V* lv = bf.v[mg.b0_buf] + mg.zone_off;
      for (uint32_t qi = threadIdx.x; qi < qn; qi += 256) ov[q0 + qi] = lv[q0 + qi - before];
    }
  }
  for (uint32_t qi = threadIdx.x; kind == 0u && qi < qn; qi += 256) {
    const uint32_t q = q0 + qi;
    uint32_t lo, hidx, before;
    bool heavy;
    locate(q, &lo, &heavy, &hidx, &before);
    const uint32_t li = min(q - before, mg.b0 ? mg.b0 - 1u : 0u);  // in range by construction
    if (heavy) {
      ok[q] = HK[hidx];
    } else {
      ok[q] = lk[li];
    }
    if constexpr (HasVal<V>::value) {
      V* ov = bf.v[mg.out_buf] + mg.zone_off;
      if (heavy) {
        const V* hv = bf.v[mg.hv_buf] + mg.zone_off + mg.b0 + PRE[hidx];
        ov[q] = hv[q - P[hidx]];
      } else {
        ov[q] = (bf.v[mg.b0_buf] + mg.zone_off)[li];
      }
    }
  }
  __syncthreads();
  }
}

// ---- PLMerge-style variant (the paper's baseline in its merge study): a
// general parallel merge of two sorted runs, X = the zone's light run and
// Y = its heavy runs (both read from the target buffer, where the zone lies
// contiguously), by merge path, into the partner buffer; a second launch
// copies the merged zone back.  No use is made of the heavy runs' constant
// keys.  Light and heavy keys are never equal, so the merge order is unique.
template <typename K>
__device__ inline uint32_t merge_path(const K* X, uint32_t nx, const K* Y, uint32_t ny, uint32_t q) {
  // number of X records among the first q outputs
  uint32_t lo = q > ny ? q - ny : 0u, hi = min(q, nx);
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (X[mid] < Y[q - mid - 1u])
      lo = mid + 1u;
    else
      hi = mid;
  }
  return lo;
}

template <typename K, typename V>
__global__ __launch_bounds__(256) void k_plmerge(const Merge* m, const uint2* munits, const uint32_t* count,
                                                 uint32_t cap, const uint8_t* tab, Bufs<K, V> bf) {
  constexpr bool HV = HasVal<V>::value;
  constexpr int PER = MERGE_TILE / 256;  // outputs per thread
  __shared__ K sk[MERGE_TILE];
  __shared__ typename std::conditional<HV, V, uint8_t>::type sv[HV ? MERGE_TILE : 1];
  __shared__ uint32_t sx[2];
  const uint32_t n_units = min(*count, cap);
  for (uint32_t ui = blockIdx.x; ui < n_units; ui += gridDim.x) {
    const uint2 u = munits[ui];
    const Merge mg = m[u.x];
    const SlotLayout sl = slot_layout(mg.g, false);
    const uint32_t* st = (const uint32_t*)(tab + mg.tab_off + sl.starts);
    const uint32_t zsize = st[mg.bstart + mg.m + 1] - st[mg.bstart];
    const uint32_t nx = mg.b0, ny = zsize - nx;
    const K* X = bf.k[mg.out_buf] + mg.zone_off;
    const K* Y = X + nx;
    const uint32_t q0 = u.y * MERGE_TILE;
    const uint32_t qn = min((uint32_t)MERGE_TILE, zsize - q0);
    if (threadIdx.x == 0) sx[0] = merge_path<K>(X, nx, Y, ny, q0);
    if (threadIdx.x == 64) sx[1] = merge_path<K>(X, nx, Y, ny, q0 + qn);
    __syncthreads();
    const uint32_t x0 = sx[0], x1 = sx[1];
    const uint32_t cx = x1 - x0;  // X records of this unit; then qn - cx Y records
    const uint32_t y0 = q0 - x0;
    for (uint32_t i = threadIdx.x; i < qn; i += 256) {
      sk[i] = i < cx ? X[x0 + i] : Y[y0 + (i - cx)];
      if constexpr (HV) {
        const V* vx = bf.v[mg.out_buf] + mg.zone_off;
        sv[i] = i < cx ? vx[x0 + i] : vx[nx + y0 + (i - cx)];
      }
    }
    __syncthreads();
    // each thread merges PER consecutive outputs of the unit from LDS
    const uint32_t o0 = min((uint32_t)threadIdx.x * PER, qn);
    const uint32_t o1 = min(o0 + PER, qn);
    uint32_t i = merge_path<K>(sk, cx, sk + cx, qn - cx, o0);
    uint32_t j = o0 - i;
    K* ok = bf.k[1 - mg.out_buf] + mg.zone_off + q0;
    for (uint32_t q = o0; q < o1; ++q) {
      const bool takex = j >= qn - cx || (i < cx && sk[i] < sk[cx + j]);
      const uint32_t src = takex ? i : cx + j;
      ok[q] = sk[src];
      if constexpr (HV) (bf.v[1 - mg.out_buf] + mg.zone_off + q0)[q] = sv[src];
      if (takex)
        ++i;
      else
        ++j;
    }
    __syncthreads();
  }
}

// Copy of every merged unit back from the partner buffer to the target.
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_plmerge_back(const Merge* m, const uint2* munits, const uint32_t* count,
                                                      uint32_t cap, const uint8_t* tab, Bufs<K, V> bf) {
  const uint32_t n_units = min(*count, cap);
  for (uint32_t ui = blockIdx.x; ui < n_units; ui += gridDim.x) {
    const uint2 u = munits[ui];
    const Merge mg = m[u.x];
    const SlotLayout sl = slot_layout(mg.g, false);
    const uint32_t* st = (const uint32_t*)(tab + mg.tab_off + sl.starts);
    const uint32_t zsize = st[mg.bstart + mg.m + 1] - st[mg.bstart];
    const uint32_t q0 = u.y * MERGE_TILE;
    const uint32_t qn = min((uint32_t)MERGE_TILE, zsize - q0);
    const uint64_t o = mg.zone_off + q0;
    copy_range<K>(bf.k[mg.out_buf] + o, bf.k[1 - mg.out_buf] + o, qn);
    if constexpr (HasVal<V>::value) copy_range<V>(bf.v[mg.out_buf] + o, bf.v[1 - mg.out_buf] + o, qn);
  }
}

// ---- Alg. 3 literally, one workgroup per zone: the zone lies contiguously
// in its target buffer A (light run B0, then the heavy runs B1..Bm); the
// partner buffer's range of the zone serves as the temporary array T.
// Buckets are moved one after the other, each by all threads.
template <typename T>
__device__ inline void flip_range(T* a, uint32_t s, uint32_t e) {  // reverse a[s, e)
  const uint32_t len = e - s;
  for (uint32_t j = threadIdx.x; j < len / 2; j += blockDim.x) {
    const T x = a[s + j];
    a[s + j] = a[e - 1 - j];
    a[e - 1 - j] = x;
  }
}

template <typename T>
__device__ inline void move_range(T* a, uint32_t from, uint32_t to, uint32_t len) {  // disjoint ranges
  for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) a[to + j] = a[from + j];
}

template <typename K, typename V>
__device__ inline void zone_flip(Bufs<K, V>& bf, int buf, uint64_t zo, uint32_t s, uint32_t e) {
  flip_range<K>(bf.k[buf] + zo, s, e);
  if constexpr (HasVal<V>::value) flip_range<V>(bf.v[buf] + zo, s, e);
}

template <typename K, typename V>
__device__ inline void zone_move(Bufs<K, V>& bf, int from_buf, uint64_t from, int to_buf, uint64_t to, uint32_t len) {
  const K* ks = bf.k[from_buf] + from;
  K* kd = bf.k[to_buf] + to;
  for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) kd[j] = ks[j];
  if constexpr (HasVal<V>::value) {
    const V* vs = bf.v[from_buf] + from;
    V* vd = bf.v[to_buf] + to;
    for (uint32_t j = threadIdx.x; j < len; j += blockDim.x) vd[j] = vs[j];
  }
}

template <typename K, typename V>
__global__ __launch_bounds__(1024) void k_merge_inplace(const Merge* m, const uint32_t* count, uint32_t cap,
                                                        const uint8_t* tab, Bufs<K, V> bf) {
  const uint32_t n_merges = min(*count, cap);
  for (uint32_t mi = blockIdx.x; mi < n_merges; mi += gridDim.x) {
    const Merge mg = m[mi];
    const SlotLayout sl = slot_layout(mg.g, false);
    const uint8_t* slot = tab + mg.tab_off;
    const uint32_t* P = (const uint32_t*)(slot + sl.light) + mg.hbase;  // final starts p_i (k_merge_pos)
    const uint32_t* hs = (const uint32_t*)(slot + sl.starts) + mg.bstart + 1;  // heavy bucket starts, task-relative
    const uint32_t M = mg.m, b0 = mg.b0;
    const uint32_t zsize = hs[M] - hs[-1];
    const uint32_t hbeg = hs[0];  // task-relative start of the first heavy run
    const int A = mg.out_buf, Tb = 1 - mg.out_buf;
    const uint64_t zo = mg.zone_off;
    // lb_i = lower_bound(B0, h_i) = p_i - (heavy records before bucket i)
    auto lb = [&](uint32_t i) { return P[i] - (hs[i] - hbeg); };
    if (b0 <= zsize - b0) {
      // more heavy records: B0 out to T, heavy runs to their places one by one
      zone_move<K, V>(bf, A, zo, Tb, zo, b0);
      __syncthreads();
      uint32_t s = b0;  // current start of B_i (heavy runs have not moved yet)
      for (uint32_t i = 0; i < M; ++i) {
        const uint32_t sz = hs[i + 1] - hs[i], p = P[i];
        if (p + sz > s) {  // the destination overlaps the bucket itself: two flips
          zone_flip<K, V>(bf, A, zo, s, s + sz);
          __syncthreads();
          zone_flip<K, V>(bf, A, zo, p, s + sz);
        } else {
          zone_move<K, V>(bf, A, zo + s, A, zo + p, sz);
        }
        __syncthreads();
        s += sz;
      }
      // light record l goes after the heavy runs whose keys are below its key
      for (uint32_t l = threadIdx.x; l < b0; l += blockDim.x) {
        uint32_t lo = 0, n = M;  // heavy buckets with lb_i <= l
        while (n > 0) {
          const uint32_t half = n >> 1;
          if (lb(lo + half) <= l) {
            lo += half + 1;
            n -= half + 1;
          } else {
            n = half;
          }
        }
        const uint32_t d = l + (hs[lo] - hbeg);
        bf.k[A][zo + d] = bf.k[Tb][zo + l];
        if constexpr (HasVal<V>::value) bf.v[A][zo + d] = bf.v[Tb][zo + l];
      }
    } else {
      // more light records: heavy runs out to T, light blocks to their places
      // from the last one back, heavy runs back from T
      zone_move<K, V>(bf, A, zo + b0, Tb, zo + b0, zsize - b0);
      __syncthreads();
      for (uint32_t k = M + 1; k-- > 0;) {
        // light block k lies after heavy runs 0..k-1: B0[lb_{k-1}, lb_k)
        const uint32_t s = k == 0 ? 0u : lb(k - 1);
        const uint32_t e = k == M ? b0 : lb(k);
        const uint32_t h = hs[k] - hbeg;  // heavy records before the block
        if (e > s && h > 0) {
          if (h < e - s) {  // overlap: block and the free slots after it, two flips
            zone_flip<K, V>(bf, A, zo, s, e);
            __syncthreads();
            zone_flip<K, V>(bf, A, zo, s, e + h);
          } else {
            zone_move<K, V>(bf, A, zo + s, A, zo + s + h, e - s);
          }
        }
        __syncthreads();
      }
      for (uint32_t i = 0; i < M; ++i)
        zone_move<K, V>(bf, Tb, zo + b0 + (hs[i] - hbeg), A, zo + P[i], hs[i + 1] - hs[i]);
    }
    __syncthreads();
  }
}

template <typename K, typename V>
void launch_merge(const Merge* m, const uint32_t* n_merges, uint32_t merge_cap, uint32_t merge_grid,
                  const uint2* munits, const uint32_t* n_munits, uint32_t munit_cap, uint32_t munit_grid,
                  uint8_t* tab, Bufs<K, V> b, int variant, hipStream_t s) {
  if (merge_grid == 0 || merge_cap == 0 || variant == MV_NONE) return;
  if (variant == MV_PLMERGE) {
    if (munit_grid == 0 || munit_cap == 0) return;
    hipLaunchKernelGGL((k_plmerge<K, V>), dim3(munit_grid), dim3(256), 0, s, m, munits, n_munits, munit_cap, tab, b);
    hipLaunchKernelGGL((k_plmerge_back<K, V>), dim3(munit_grid), dim3(256), 0, s, m, munits, n_munits, munit_cap, tab,
                       b);
    return;
  }
  hipLaunchKernelGGL((k_merge_pos<K>), dim3(merge_grid), dim3(64), 0, s, m, n_merges, merge_cap, tab,
                     (const K*)b.k[0], (const K*)b.k[1]);
  if (variant == MV_INPLACE) {
    hipLaunchKernelGGL((k_merge_inplace<K, V>), dim3(merge_grid), dim3(1024), 0, s, m, n_merges, merge_cap, tab, b);
    return;
  }
  if (munit_grid == 0 || munit_cap == 0) return;
  hipLaunchKernelGGL((k_merge_gather<K, V>), dim3(munit_grid), dim3(256), 0, s, m, munits, n_munits, munit_cap, tab,
                     b);
}

// ------------------------------------------------------------------ roots
template <typename K>
__global__ void k_root(Task* tk, LevelCounters* in, uint64_t n, int key_bits, int gamma) {
  uint32_t* cw = reinterpret_cast<uint32_t*>(in);
  for (uint32_t i = threadIdx.x; i < sizeof(LevelCounters) / 4; i += blockDim.x) cw[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    Task t;
    t.off = 0;
    t.cm_off = 0;
    t.tab_off = 0;
    t.size = (uint32_t)n;
    t.n_root = (uint32_t)n;
    t.level = 0;
    t.unit_base = 0;
    t.n_chunks = 0;
    t.hi = (uint8_t)key_bits;
    t.src = 0;
    t.tgt = 0;
    t.flags = 0;
    t.gamma = (uint8_t)gamma;
    t.w = 0;
    t.shift = 0;
    t.top = 0;
    t.n_heavy = 0;
    t.n_buckets = 0;
    tk[0] = t;
    in->next_tasks = 1;
    in->next_records = (uint32_t)n;
    in->next_max_size = (uint32_t)n;
  }
}

template <typename K>
void launch_root(Task* t, LevelCounters* in, uint64_t n, int key_bits, int gamma, hipStream_t s) {
  hipLaunchKernelGGL(k_root<K>, dim3(1), dim3(64), 0, s, t, in, n, key_bits, gamma);
}

__global__ void k_zero_counters(LevelCounters* c, uint32_t words) {
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) w[i] = 0u;
}

void launch_zero_counters(LevelCounters* c, uint32_t n, hipStream_t s) {
  const uint32_t words = n * (uint32_t)(sizeof(LevelCounters) / 4);
  hipLaunchKernelGGL(k_zero_counters, dim3((words + 255) / 256), dim3(256), 0, s, c, words);
}

uint32_t persistent_grid(uint32_t wg_per_cu) {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || n <= 0) {
      (void)hipGetLastError();
      n = 256;
    }
    return n;
  }();
  return (uint32_t)cus * wg_per_cu;
}

template void launch_root<uint32_t>(Task*, LevelCounters*, uint64_t, int, int, hipStream_t);
template void launch_root<uint64_t>(Task*, LevelCounters*, uint64_t, int, int, hipStream_t);

#define DTS_INST(K, V)                                                                                      \
  template void launch_children<K, V>(const LevelArgs&, Bufs<K, V>, hipStream_t);                          \
  template void launch_seed_segments<K, V>(const LevelArgs&, const uint64_t*, uint32_t, uint64_t, hipStream_t); \
  template void launch_copy<K, V>(const Leaf*, const uint32_t*, uint32_t, uint32_t, Bufs<K, V>, hipStream_t); \
  template void launch_merge<K, V>(const Merge*, const uint32_t*, uint32_t, uint32_t, const uint2*,        \
                                   const uint32_t*, uint32_t, uint32_t, uint8_t*, Bufs<K, V>, int, hipStream_t);
DTS_INST(uint32_t, NoVal)
DTS_INST(uint64_t, NoVal)
DTS_INST(uint64_t, uint64_t)
DTS_INST(uint32_t, uint32_t)
#undef DTS_INST

}  // namespace dts

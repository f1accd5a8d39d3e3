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
#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

constexpr uint32_t COPY_PIECE = 1u << 20;   // records per copy item
constexpr uint32_t MERGE_TILE = 4096;       // outputs per gather unit

template <typename K, typename V>
__device__ inline void emit_child(const LevelArgs& a, uint64_t off, uint32_t c, int hi, int buf, int tgt, bool skip,
                                  uint32_t n_root, uint32_t level) {
  LevelCounters* ctr = a.ctr;
  if (c == 0) return;
  if (c == 1 || hi == 0) {
    // finished: all keys equal (or a single record); move it if needed
    if (buf != tgt) {
      for (uint32_t p = 0; p < c; p += COPY_PIECE) {
        const uint32_t i = atomicAdd(&ctr->copies, 1u);
        if (i >= a.caps.copies) {
          atomicOr(&ctr->error, ERR_COPY);
          return;
        }
        Leaf l;
        l.off = off + p;
        l.size = min(COPY_PIECE, c - p);
        l.bits = 0;
        l.from = (uint8_t)buf;
        l.to = (uint8_t)tgt;
        l.pad = 0;
        a.copies[i] = l;
      }
      atomicAdd(&ctr->st_copy_records, (unsigned long long)c);
    }
    return;
  }
  if (c <= a.cutoff) {
    const int cls = c <= a.leaf_max[0] ? 0 : (c <= a.leaf_max[1] ? 1 : 2);
    const uint32_t i = atomicAdd(&ctr->leaf[cls], 1u);
    if (i >= a.caps.leaf) {
      atomicOr(&ctr->error, ERR_LEAF);
      return;
    }
    Leaf l;
    l.off = off;
    l.size = c;
    l.bits = (uint8_t)hi;
    l.from = (uint8_t)buf;
    l.to = (uint8_t)tgt;
    l.pad = 0;
    a.leaf[cls][i] = l;
    atomicAdd(&ctr->st_leaf_records, (unsigned long long)c);
    return;
  }
  const uint32_t i = atomicAdd(&ctr->next_tasks, 1u);
  if (i >= a.caps.tasks) {
    atomicOr(&ctr->error, ERR_TASKS);
    return;
  }
  Task t;
  t.off = off;
  t.cm_off = 0;
  t.tab_off = 0;
  t.size = c;
  t.n_root = n_root;
  t.level = level;
  t.unit_base = 0;
  t.n_chunks = 0;
  t.hi = (uint8_t)hi;
  t.src = (uint8_t)buf;
  t.tgt = (uint8_t)tgt;
  t.flags = skip ? TF_SKIP_DISABLED : 0;
  t.gamma = (uint8_t)plan_gamma(c, a.g_override);
  t.w = 0;
  t.shift = 0;
  t.top = 0;
  t.n_heavy = 0;
  t.n_buckets = 0;
  a.next[i] = t;
  atomicMax(&ctr->next_max_size, c);
  atomicAdd(&ctr->next_records, c);
}

// Batched form: every segment is the root of its own sort.
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_seed(LevelArgs a, const uint64_t* seg, uint32_t n_seg, uint64_t n_total) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n_seg) return;
  const uint64_t b = seg[s], e = seg[s + 1];
  if (e < b || e > n_total || (s == 0 && b != 0) || (s + 1 == n_seg && e != n_total) || e - b >= (1ull << 32)) {
    atomicOr(&a.ctr->error, ERR_SEGMENTS);
    return;
  }
  const uint32_t c = (uint32_t)(e - b);
  emit_child<K, V>(a, b, c, a.key_bits, 0, 0, false, c, 0);
}

template <typename K, typename V>
void launch_seed_segments(const LevelArgs& a, const uint64_t* seg_off, uint32_t n_seg, uint64_t n_total,
                          hipStream_t s) {
  if (n_seg == 0) return;
  hipLaunchKernelGGL((k_seed<K, V>), dim3((n_seg + 255) / 256), dim3(256), 0, s, a, seg_off, n_seg, n_total);
}

// Child planning: one workgroup per task, one thread per zone.
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_children(LevelArgs a) {
  const Task t = a.tasks[blockIdx.x];
  if (t.n_chunks == 0) return;
  constexpr bool HV = HasVal<V>::value;
  const bool learned = (t.flags & TF_LEARNED) != 0;
  const SlotLayout sl = slot_layout(t.gamma, learned);
  const uint8_t* slot = a.tab + t.tab_off;
  const uint32_t* L = (const uint32_t*)(slot + sl.light);
  const uint32_t* st = (const uint32_t*)(slot + sl.starts);
  const uint64_t* SPL = (const uint64_t*)(slot + sl.spl);
  const int dst = 1 - t.src;
  const uint32_t zones = 1u << t.w;
  unsigned long long heavy_recs = 0;
  for (uint32_t z = threadIdx.x; z < zones; z += 256) {
    const uint32_t lid = L[z];
    const uint32_t m = L[z + 1] - lid - 1u;
    const uint32_t s0 = st[lid];
    const uint32_t c0 = st[lid + 1] - s0;
    int ctgt = t.tgt;
    if (m > 0) {
      ctgt = 1 - t.tgt;
      const uint32_t zend = st[lid + m + 1];
      const uint32_t i = atomicAdd(&a.ctr->merges, 1u);
      if (i >= a.caps.merges) {
        atomicOr(&a.ctr->error, ERR_MERGE);
      } else {
        Merge mg;
        mg.zone_off = t.off + s0;
        mg.tab_off = t.tab_off;
        mg.b0 = c0;
        mg.m = m;
        mg.hbase = lid - z;
        mg.bstart = lid;
        mg.zone_rel = s0;
        const uint32_t zsize = zend - s0;
        mg.n_units = (zsize + MERGE_TILE - 1) / MERGE_TILE;
        mg.unit_base = atomicAdd(&a.ctr->merge_units, mg.n_units);
        if (mg.unit_base + mg.n_units > a.caps.munits) atomicOr(&a.ctr->error, ERR_MUNITS);
        mg.b0_buf = (uint8_t)ctgt;
        mg.hv_buf = (uint8_t)dst;
        mg.out_buf = (uint8_t)t.tgt;
        mg.g = t.gamma;
        if (HV && dst == t.tgt && zsize > c0) {
          // heavy values would be overwritten by the gather: copy them to src first
          for (uint32_t p = c0; p < zsize; p += COPY_PIECE) {
            const uint32_t k = atomicAdd(&a.ctr->spills, 1u);
            if (k >= a.caps.spills) {
              atomicOr(&a.ctr->error, ERR_SPILL);
              break;
            }
            Leaf l;
            l.off = t.off + s0 + p;
            l.size = min(COPY_PIECE, zsize - p);
            l.bits = 0;
            l.from = (uint8_t)dst;
            l.to = (uint8_t)t.src;
            l.pad = 0;
            a.spills[k] = l;
          }
          mg.hv_buf = (uint8_t)t.src;
          atomicAdd(&a.ctr->st_copy_records, (unsigned long long)(zsize - c0));
        }
        a.merges[i] = mg;
        heavy_recs += zsize - c0;
        atomicAdd(&a.ctr->st_merge_records, (unsigned long long)zsize);
      }
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
    emit_child<K, V>(a, t.off + s0, c0, chi, dst, ctgt, false, t.n_root, t.level + 1);
  }
  if (threadIdx.x == 0) {
    const uint32_t ob = t.n_buckets - 1u;
    const uint32_t c = st[ob + 1] - st[ob];
    if (c) atomicAdd(&a.ctr->st_overflow_records, (unsigned long long)c);
    emit_child<K, V>(a, t.off + st[ob], c, t.hi, dst, t.tgt, true, t.n_root, t.level + 1);
    atomicAdd(&a.ctr->st_heavy_keys, (unsigned long long)t.n_heavy);
    atomicAdd(&a.ctr->st_tasks, 1ull);
    atomicAdd(&a.ctr->st_distributed, (unsigned long long)t.size);
  }
  if (heavy_recs) atomicAdd(&a.ctr->st_heavy_records, heavy_recs);
}

template <typename K, typename V>
void launch_children(const LevelArgs& a, Bufs<K, V> b, hipStream_t s) {
  (void)b;
  hipLaunchKernelGGL((k_children<K, V>), dim3(a.n_tasks), dim3(256), 0, s, a);
}

// ------------------------------------------------------------------ copies
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_copy(const Leaf* items, Bufs<K, V> bf) {
  const Leaf it = items[blockIdx.x];
  const K* ki = bf.k[it.from] + it.off;
  K* ko = bf.k[it.to] + it.off;
  for (uint32_t i = threadIdx.x; i < it.size; i += 256) ko[i] = ki[i];
  if constexpr (HasVal<V>::value) {
    const V* vi = bf.v[it.from] + it.off;
    V* vo = bf.v[it.to] + it.off;
    for (uint32_t i = threadIdx.x; i < it.size; i += 256) vo[i] = vi[i];
  }
}

template <typename K, typename V>
void launch_copy(const Leaf* items, uint32_t n_items, Bufs<K, V> b, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL((k_copy<K, V>), dim3(n_items), dim3(256), 0, s, items, b);
}

// ------------------------------------------------------------------ merges
__global__ __launch_bounds__(64) void k_merge_units(const Merge* m, uint2* munits) {
  const Merge mg = m[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < mg.n_units; j += 64) munits[mg.unit_base + j] = make_uint2(blockIdx.x, j);
}

void launch_merge_units(const Merge* m, uint32_t n_merges, uint2* munits, hipStream_t s) {
  if (n_merges == 0) return;
  hipLaunchKernelGGL(k_merge_units, dim3(n_merges), dim3(64), 0, s, m, munits);
}

// Alg. 3, first line: p_i = lower_bound(B0, h_i) + sum_{j<i} |B_j| for every
// heavy bucket of the zone (B0 is sorted and holds no heavy key).  The result
// is stored in the slot's light-id area (free once the level's children are
// planned), at the heavy key's index.
template <typename K>
__global__ __launch_bounds__(64) void k_merge_pos(const Merge* m, uint8_t* tab, const K* k0, const K* k1) {
  const Merge mg = m[blockIdx.x];
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

// Out-of-place gather of a zone: output q takes heavy bucket i when
// p_i <= q < p_i + |B_i|, else light record q - (heavy records before q).
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_merge_gather(const Merge* m, const uint2* munits, uint8_t* tab,
                                                      Bufs<K, V> bf) {
  constexpr int MAXH = 1 << (GMAX - 1);
  __shared__ uint32_t P[MAXH], S[MAXH], PRE[MAXH];
  __shared__ K HK[MAXH];
  __shared__ uint32_t tmp[5];
  const uint2 u = munits[blockIdx.x];
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
  const uint32_t q1 = min(zsize, q0 + MERGE_TILE);
  const K* lk = bf.k[mg.b0_buf] + mg.zone_off;
  K* ok = bf.k[mg.out_buf] + mg.zone_off;
  for (uint32_t q = q0 + threadIdx.x; q < q1; q += 256) {
    // largest i with P[i] <= q
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
    bool heavy = false;
    uint32_t hidx = 0, before = 0;
    if (lo > 0) {
      const uint32_t i = lo - 1;
      if (q < P[i] + S[i]) {
        heavy = true;
        hidx = i;
      } else {
        before = PRE[i] + S[i];
      }
    }
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
}

template <typename K, typename V>
void launch_merge(const Merge* m, uint32_t n_merges, const uint2* munits, uint32_t n_munits, uint8_t* tab,
                  Bufs<K, V> b, hipStream_t s) {
  if (n_merges == 0) return;
  hipLaunchKernelGGL((k_merge_pos<K>), dim3(n_merges), dim3(64), 0, s, m, tab, (const K*)b.k[0],
                     (const K*)b.k[1]);
  hipLaunchKernelGGL((k_merge_gather<K, V>), dim3(n_munits), dim3(256), 0, s, m, munits, tab, b);
}

#define DTS_INST(K, V)                                                                                      \
  template void launch_children<K, V>(const LevelArgs&, Bufs<K, V>, hipStream_t);                          \
  template void launch_seed_segments<K, V>(const LevelArgs&, const uint64_t*, uint32_t, uint64_t, hipStream_t); \
  template void launch_copy<K, V>(const Leaf*, uint32_t, Bufs<K, V>, hipStream_t);                         \
  template void launch_merge<K, V>(const Merge*, uint32_t, const uint2*, uint32_t, uint8_t*, Bufs<K, V>,   \
                                   hipStream_t);
DTS_INST(uint32_t, NoVal)
DTS_INST(uint64_t, NoVal)
DTS_INST(uint64_t, uint64_t)
DTS_INST(uint32_t, uint32_t)
#undef DTS_INST

}  // namespace dts

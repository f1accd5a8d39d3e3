// Step 1 of Alg. 2 (Section 3.1; the sampled key range and overflow bucket of
// Section 5), one workgroup per subproblem, and the base case of Section 3.5
// (a stable sort in LDS), one workgroup per small subproblem.
#include <algorithm>
#include <cstdlib>

#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

// ------------------------------------------------------------------- plan
// Draws 2^g * t sample keys at counter-based random positions (with
// replacement), sorts them in LDS, takes the key range from the sample
// maximum, marks keys that fill two or more of the 2^g subsample slots
// S[0], S[t], S[2t], ... as heavy, and writes the light-id table L (per zone:
// its light id = zone + number of heavy keys in lower zones; the last entry is
// the overflow id) and the heavy keys (ascending) into the task's table slot.
// Sample size: 2^g * t with t = min(ceil(log2 n_root), SCAP / 2^g), SCAP =
// 32768 keys of 4 bytes or 16384 of 8 bytes (what one workgroup's LDS holds
// for the widest digit).  A variant holds T * ITEMS keys; the host picks one
// that holds the sample of the level's widest digit.
template <typename K>
constexpr uint32_t plan_sample_cap() {
  return sizeof(K) == 4 ? 32768u : 16384u;
}

template <typename K, int T, int ITEMS>
__global__ __launch_bounds__(T, T == 512 ? 4 : 1) void k_plan(LevelArgs a, const K* k0, const K* k1) {
  constexpr int CAP = T * ITEMS;  // sample capacity of this variant
  __shared__ K sk[CAP];
  __shared__ uint32_t cnt[bsort_cnt_words<T>()];
  __shared__ K red[2 * (T / WAVE)];
  __shared__ uint32_t hz[1 << (GMAX - 1)];
  __shared__ uint32_t hc[1 << (GMAX - 1)];  // subsample slots each heavy key fills
  __shared__ uint32_t tmp[T / WAVE + 1];
  __shared__ int s_top, s_w, s_shift;
  __shared__ uint32_t s_flag;

  const uint32_t n_tasks = a.ctr->cur_tasks;
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
  Task& tr = a.tasks[ti];
  const Task t = tr;
  if (t.flags & TF_LEARNED) continue;  // planned by the learned-partitioner step
  const bool split = a.merge_variant == MV_SPLIT;
  const int g = t.gamma;
  const int hi = t.hi;
  const SlotLayout sl = slot_layout(g, false);
  uint8_t* slot = a.tab + t.tab_off;
  uint32_t* gL = (uint32_t*)(slot + sl.light);
  uint64_t* gH = (uint64_t*)(slot + sl.heavy);
  uint32_t nh = 0;

  if (hi <= g) {
    // last digit: every remaining bit in one plain digit; no sample needed
    if (threadIdx.x == 0) {
      s_top = hi;
      s_w = hi;
      s_shift = 0;
    }
  } else {
    const uint32_t lgn = 32 - __builtin_clz(max(t.n_root - 1u, 1u));
    uint32_t ts = min(lgn, plan_sample_cap<K>() >> g);
    ts = max(min(ts, (uint32_t)(CAP >> g)), 1u);  // the host's variant choice keeps this a no-op
    const uint32_t ns = ts << g;
    const uint64_t sb = sample_base(a.seed, t.off, t.level);
    const K* keys = (t.src ? k1 : k0) + t.off;
    K kk[ITEMS];
    uint16_t dummy[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
      if (e < ns) {
        const uint64_t r = mix64(sb + (uint64_t)(e + 1) * GOLD);
        const uint64_t p = __umul64hi(r, (uint64_t)t.size);
        kk[i] = keys[p];
      } else {
        kk[i] = ~(K)0;
      }
    }
    K vor, vand;
    block_or_and<K, T, ITEMS>(kk, (int)ns, red, &vor, &vand);
    const K diff = (vor ^ vand) & mask_below<K>(hi);
    if (diff) {
      block_sort_bits<K, T, ITEMS, false>(kk, dummy, trailing_zeros(diff), bit_length(diff), sk, nullptr, cnt,
                                          nullptr, (int)ns, &s_flag);
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) sk[striped_index<T, ITEMS>(i)] = kk[i];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const K mx = sk[ns - 1] & mask_below<K>(hi);
      const int top = (t.flags & TF_SKIP_DISABLED) ? hi : bit_length(mx);
      const int w = min(g, top);
      s_top = top;
      s_w = w;
      s_shift = top - w;
    }
    __syncthreads();
    if (!a.plain) {
      // heavy: the first slot of every run of >= 2 equal subsample slots
      const uint32_t nsub = 1u << g;
      nh = 0;
      for (uint32_t j0 = 0; j0 < nsub; j0 += T) {
        const uint32_t j = j0 + threadIdx.x;
        bool f = false;
        K kj = 0;
        if (j + 1 < nsub) {
          kj = sk[j * ts];
          f = (kj == sk[(j + 1) * ts]) && (j == 0 || sk[(j - 1) * ts] != kj);
        }
        uint32_t total;
        const uint32_t idx = nh + block_excl_scan<T>(f ? 1u : 0u, tmp, &total);
        nh += total;
        if (f) {
          gH[idx] = (uint64_t)kj;
          const K low = kj & mask_below<K>(hi);
          hz[idx] = (uint32_t)(shr<K>(low, s_shift) & (K)((1u << s_w) - 1u));
          uint32_t c = 2;
          while (j + c < nsub && sk[(j + c) * ts] == kj) ++c;
          hc[idx] = c;
        }
        __syncthreads();
      }
      // The split layout has two buckets per heavy key; to stay within the
      // bucket capacity of the digit width it keeps at most 2^(g-2) heavy
      // keys (none for 1-bit digits): those filling the most subsample slots
      // (ties: smaller key).
      const uint32_t cap = g >= 2 ? 1u << (g - 2) : 0u;
      if (split && nh > cap) {
        // nh <= 2^(g-1) <= T: one candidate per thread
        const uint32_t i = threadIdx.x;
        uint32_t keep = 0, z0 = 0;
        uint64_t hk = 0;
        if (i < nh) {
          uint32_t rank = 0;
          for (uint32_t j = 0; j < nh; ++j) rank += (hc[j] > hc[i] || (hc[j] == hc[i] && j < i)) ? 1u : 0u;
          keep = rank < cap ? 1u : 0u;
          hk = gH[i];
          z0 = hz[i];
        }
        __syncthreads();
        uint32_t total;
        const uint32_t idx = block_excl_scan<T>(keep, tmp, &total);
        if (keep) {
          gH[idx] = hk;
          hz[idx] = z0;
        }
        nh = total;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  const int w = s_w;
  // light ids: L[z] = z + #{heavy keys with zone < z}; zones of the sorted heavy keys are non-decreasing
  const uint32_t zones = 1u << w;
  for (uint32_t z = threadIdx.x; z <= zones; z += T) {
    uint32_t lo = 0, n = nh;
    while (n > 0) {
      const uint32_t half = n >> 1;
      if (hz[lo + half] < z) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    gL[z] = z + (split ? 2u : 1u) * lo;
  }
  if (threadIdx.x == 0) {
    tr.w = (uint8_t)w;
    tr.shift = (uint8_t)s_shift;
    tr.top = (uint8_t)s_top;
    tr.n_heavy = (uint16_t)nh;
    tr.n_buckets = (uint16_t)(zones + (split ? 2u : 1u) * nh + 1);
    if (split) tr.flags = (uint8_t)(t.flags | TF_SPLIT);
  }
  __syncthreads();
  }
}

template <typename K>
void launch_plan(const LevelArgs& a, const K* k0, const K* k1, int g_level_max, hipStream_t s) {
  // largest sample of the level: 2^g * min(32, SCAP / 2^g) keys
  const uint32_t g = (uint32_t)g_level_max;
  const uint32_t ns = std::min<uint32_t>(32u, plan_sample_cap<K>() >> g) << g;
  if (ns <= 1024u * 8u && a.grid_tasks <= 64u) {
    // few subproblems (the root, small sorts): each sample sorted by twice the
    // threads, so the level's critical path is shorter
    hipLaunchKernelGGL((k_plan<K, 1024, 8>), dim3(a.grid_tasks), dim3(1024), 0, s, a, k0, k1);
  } else if (ns <= 512u * 16u) {
    hipLaunchKernelGGL((k_plan<K, 512, 16>), dim3(a.grid_tasks), dim3(512), 0, s, a, k0, k1);
  } else {
    constexpr int IT = sizeof(K) == 4 ? 32 : 16;
    hipLaunchKernelGGL((k_plan<K, 1024, IT>), dim3(a.grid_tasks), dim3(1024), 0, s, a, k0, k1);
  }
}

// ---------------------------------------------------------------- leaves
// Base case: a stable radix sort in LDS of a subproblem of at most T*ITEMS
// records, only over the bit range in which its keys differ.  With T = 64 a
// workgroup holds SUB independent one-wave sorters, each with its own LDS.
template <typename K, typename V, int T, int ITEMS, int RANKREQ, int SUB>
constexpr int leaf_min_waves() {
  // 4096 bare 32-bit keys, LDS-match ranks: 28 KB of LDS lets five
  // workgroups share a CU, which takes at most 96 VGPRs (the other ranking
  // modes would spill there)
  return (sizeof(K) == 4 && !HasVal<V>::value && T * SUB == 256 && ITEMS == 16 && RANKREQ == RANK_LDS) ? 5 : 1;
}

template <typename K, typename V, int T, int ITEMS, int RANKREQ, int SUB = 1>
__global__ __launch_bounds__(T* SUB, (leaf_min_waves<K, V, T, ITEMS, RANKREQ, SUB>())) void k_leaf(const Leaf* items, const uint32_t* count, uint32_t cap,
                                                 Bufs<K, V> bf) {
  static_assert(SUB == 1 || T == WAVE, "several sorters per workgroup only for one-wave sorters");
  constexpr int N = T * ITEMS;
  constexpr bool HV = HasVal<V>::value;
  // LDS-match ranking (if requested and its tables fit next to the keys), else ballot ranking
  constexpr bool USE_LDS = RANKREQ != RANK_BALLOT && SUB * (N * sizeof(K) + (HV ? N * 2 : 0) +
                                                            4 * bsort_cnt_words<T>() + 8 * bsort_match_words<T>()) <=
                                                         150 * 1024;
  constexpr int RANK = USE_LDS ? RANKREQ : RANK_BALLOT;
  __shared__ K sk_all[SUB][N];
  __shared__ uint16_t si_all[SUB][HV ? N : 1];
  __shared__ uint32_t cnt_all[SUB][bsort_cnt_words<T>()];
  __shared__ unsigned long long mk_all[SUB][USE_LDS ? bsort_match_words<T>() : 1];
  __shared__ K red_all[SUB][2 * (T / WAVE)];
  __shared__ uint32_t flag_all[SUB];
  const int sub = SUB == 1 ? 0 : (int)(threadIdx.x / T);
  K* sk = sk_all[sub];
  uint16_t* si = si_all[sub];
  uint32_t* cnt = cnt_all[sub];
  unsigned long long* mk = mk_all[sub];
  K* red = red_all[sub];
  const uint32_t n_items = min(*count, cap);
  if (blockIdx.x * SUB >= n_items) return;  // no leaf for this workgroup (persistent grids of sparse classes)
  if constexpr (USE_LDS) {
    for (int i = btid<T>(); i < bsort_match_words<T>(); i += T) mk[i] = 0ull;
  }
  for (uint32_t li = blockIdx.x * SUB + sub; li < n_items; li += gridDim.x * SUB) {
    const Leaf it = items[li];
    const K* kin = bf.k[it.from] + it.off;
    K* kout = bf.k[it.to] + it.off;
    const int n = (int)it.size;
    K kk[ITEMS];
    uint16_t ix[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<T, ITEMS>(i);
      kk[i] = e < n ? kin[e] : ~(K)0;
      ix[i] = (uint16_t)e;
    }
    K vor, vand;
    block_or_and<K, T, ITEMS>(kk, n, red, &vor, &vand);
    const K diff = (vor ^ vand) & mask_below<K>(it.bits);
    if (diff) {
      block_sort_bits<K, T, ITEMS, HV, RANK>(kk, ix, trailing_zeros(diff), bit_length(diff), sk, si, cnt, mk, n,
                                             &flag_all[sub]);
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<T, ITEMS>(i);
      if (e < n) kout[e] = kk[i];
    }
    if constexpr (HV) {
      const V* vin = bf.v[it.from] + it.off;
      V* vout = bf.v[it.to] + it.off;
      // gather every value before any is written: `to` may equal `from`
      V vv[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int e = striped_index<T, ITEMS>(i);
        if (e < n) vv[i] = vin[ix[i]];
      }
      __builtin_amdgcn_s_waitcnt(0);  // the gathers have landed before the barrier
      bsync<T>();
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int e = striped_index<T, ITEMS>(i);
        if (e < n) vout[e] = vv[i];
      }
    }
    bsync<T>();
  }
}

// ----------------------------------------------------------- pair merge
// Second step of paired leaves: halves[2p] = [off, off + h) and
// halves[2p + 1] = [off + h, off + c), both sorted in buffer `to`, merged into
// buffer `pad` over [off, off + c) (c <= PAIR_MAX); on equal keys the first
// half goes first, so the merge is stable.  The bucket is staged in LDS;
// thread t produces outputs [t E, t E + E): it finds where the merge path
// crosses diagonal t E by a binary search, merges E steps, and writes its
// outputs back to LDS (one padding word per 32 keeps the lanes on distinct
// banks) for a coalesced copy out.
template <typename K>
__global__ __launch_bounds__(1024) void k_pair_merge(const Leaf* halves, const uint32_t* count, uint32_t cap, K* k0,
                                                     K* k1) {
  constexpr int T = 1024, E = PAIR_MAX / T;
  static_assert(E * T == (int)PAIR_MAX && E == 32, "one padding word per 32 outputs of a thread");
  __shared__ K sa[PAIR_MAX + PAIR_MAX / 32];
  const uint32_t n_pairs = min(*count, cap) / 2;
  for (uint32_t pi = blockIdx.x; pi < n_pairs; pi += gridDim.x) {
    const Leaf A = halves[2 * pi], B = halves[2 * pi + 1];
    const int na = (int)A.size, n = (int)(A.size + B.size);
    if (n > (int)PAIR_MAX) continue;  // never made by the child planning
    const K* src = (A.to ? k1 : k0) + A.off;
    K* dst = (A.pad ? k1 : k0) + A.off;
    for (int e = threadIdx.x; e < n; e += T) sa[e] = src[e];
    __syncthreads();
    const K* a = sa;
    const K* b = sa + na;
    const int nb = n - na;
    const int d = min((int)threadIdx.x * E, n);
    // i = records of the first half among the first d outputs
    int lo = max(0, d - nb), hi = min(d, na);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (a[mid] <= b[d - 1 - mid]) {
        lo = mid + 1;
      } else {
        hi = mid;
      }
    }
    int i = lo, j = d - lo;
    K out[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool take_a = j >= nb || (i < na && a[i] <= b[j]);
      out[e] = take_a ? a[min(i, na - 1)] : b[min(j, nb - 1)];
      i += take_a ? 1 : 0;
      j += take_a ? 0 : 1;
    }
    __syncthreads();  // every read of the halves is done
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = d + e;
      if (p < n) sa[p + (p >> 5)] = out[e];
    }
    __syncthreads();
    for (int p = threadIdx.x; p < n; p += T) dst[p] = sa[p + (p >> 5)];
    __syncthreads();
  }
}

template <typename K, typename V>
void launch_pairs(const Leaf* halves, const uint32_t* count, uint32_t cap, uint32_t grid_leaf, uint32_t grid_merge,
                  Bufs<K, V> b, hipStream_t s) {
  if constexpr (pair_leaves<K, V>()) {
    if (grid_leaf == 0 || grid_merge == 0 || cap == 0) return;
    launch_leaf<K, V>(halves, count, cap, grid_leaf, LEAF_CLASSES - 1, b, s);
    hipLaunchKernelGGL((k_pair_merge<K>), dim3(grid_merge), dim3(1024), 0, s, halves, count, cap, b.k[0], b.k[1]);
  } else {
    (void)halves, (void)count, (void)cap, (void)grid_leaf, (void)grid_merge, (void)b, (void)s;
  }
}

// ----------------------------------------------------------- finishing
// Tasks still open after the last recorded level of the graph form: one
// workgroup per task sorts it completely with a stable LSD radix sort
// through global memory, 8-bit digits over the bits in which the task's keys
// differ.  Per digit: a histogram of the task, its exclusive scan (running
// offsets), then tile by tile a stable sort of the tile by the digit in LDS
// and a write of each digit's run at the digit's running offset.  It
// ping-pongs between the task's ranges of the two buffers (both belong to
// the task) and leaves the result in the task's target buffer.
template <typename K, typename V, int T, int ITEMS>
__global__ __launch_bounds__(T) void k_finish(const Task* tasks, const uint32_t* count, uint32_t cap, Bufs<K, V> bf) {
  constexpr int N = T * ITEMS;
  constexpr int WAVES = T / WAVE;
  constexpr bool HV = HasVal<V>::value;
  __shared__ K sk[N];
  __shared__ uint16_t si[HV ? N : 1];
  __shared__ uint32_t cnt[bsort_cnt_words<T>()];
  __shared__ uint32_t run[256];
  __shared__ uint32_t tstart[256];
  __shared__ uint32_t tmp[WAVES + 1];
  __shared__ K red[2 * WAVES];
  const uint32_t n_items = min(*count, cap);
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  for (uint32_t ti = blockIdx.x; ti < n_items; ti += gridDim.x) {
    const Task t = tasks[ti];
    const uint32_t n = t.size;
    int cur = t.src;
    // bits in which the task's keys differ, below hi
    K o = 0, an = ~(K)0;
    for (uint32_t e = threadIdx.x; e < n; e += T) {
      const K x = bf.k[cur][t.off + e];
      o |= x;
      an &= x;
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
      o |= __shfl_xor(o, off, WAVE);
      an &= __shfl_xor(an, off, WAVE);
    }
    if (lane == 0) {
      red[wv] = o;
      red[WAVES + wv] = an;
    }
    __syncthreads();
    K ro = 0, ra = ~(K)0;
    for (int w = 0; w < WAVES; ++w) {
      ro |= red[w];
      ra &= red[WAVES + w];
    }
    const K diff = (ro ^ ra) & mask_below<K>(t.hi);
    const int lo = diff ? trailing_zeros(diff) : 0;
    const int hb = diff ? bit_length(diff) : 0;
    for (int bit = lo; bit < hb; bit += 8) {
      const int nb = min(8, hb - bit);
      const uint32_t dm = (1u << nb) - 1u;
      const K* kin = bf.k[cur] + t.off;
      K* kout = bf.k[1 - cur] + t.off;
      auto digit = [&](K x) { return (uint32_t)shr<K>(x, bit) & dm; };
      for (int d = threadIdx.x; d < 256; d += T) run[d] = 0;
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < n; e += T) atomicAdd(&run[digit(kin[e])], 1u);
      __syncthreads();
      block_excl_scan_array<T>(run, 256, tmp);
      for (uint32_t base = 0; base < n; base += N) {
        const int m = (int)min((uint32_t)N, n - base);
        K kk[ITEMS];
        uint16_t ix[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int e = striped_index<T, ITEMS>(i);
          kk[i] = e < m ? kin[base + e] : ~(K)0;
          ix[i] = (uint16_t)e;
        }
        block_radix_sort<K, T, ITEMS, HV>(kk, ix, bit, bit + nb, sk, si, cnt, nullptr, m);
        // sk[0..m) is the tile in digit order; each digit's records are one run
        for (int j = threadIdx.x; j < m; j += T) {
          const uint32_t d = digit(sk[j]);
          if (j == 0 || digit(sk[j - 1]) != d) tstart[d] = (uint32_t)j;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += T) {
          const uint32_t d = digit(sk[j]);
          const uint32_t p = run[d] + (uint32_t)j - tstart[d];
          if (p < n) {
            kout[p] = sk[j];
            if constexpr (HV) bf.v[1 - cur][t.off + p] = bf.v[cur][t.off + base + si[j]];
          }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += T) {
          const uint32_t d = digit(sk[j]);
          if (j + 1 == m || digit(sk[j + 1]) != d) run[d] += (uint32_t)j + 1u - tstart[d];
        }
        __syncthreads();
      }
      // this pass's writes are read by other threads in the next pass
      __threadfence();
      __syncthreads();
      cur = 1 - cur;
    }
    if (cur != t.tgt) {
      for (uint32_t e = threadIdx.x; e < n; e += T) {
        bf.k[t.tgt][t.off + e] = bf.k[cur][t.off + e];
        if constexpr (HV) bf.v[t.tgt][t.off + e] = bf.v[cur][t.off + e];
      }
    }
    __threadfence();
    __syncthreads();
  }
}

template <typename K, typename V>
void launch_finish(const Task* tasks, const uint32_t* count, uint32_t cap, uint32_t grid, Bufs<K, V> b,
                   hipStream_t s) {
  if (grid == 0 || cap == 0) return;
  constexpr int IT = sizeof(K) == 4 ? 16 : 8;
  hipLaunchKernelGGL((k_finish<K, V, 512, IT>), dim3(grid), dim3(512), 0, s, tasks, count, cap, b);
}

// Ranking mode of the leaf sorts (tuning knob: DTSORT_LEAF_RANK=ballot|lds).
static int leaf_rank_mode() {
  static int m = [] {
    const char* e = getenv("DTSORT_LEAF_RANK");
    if (e && e[0] == 'b') return (int)RANK_BALLOT;
    if (e && e[0] == 'h') return (int)RANK_HYBRID;
    if (e && e[0] == 'p') return (int)RANK_PIPE;
    return (int)RANK_LDS;
  }();
  return m;
}

template <typename K, typename V, int RANK>
static void launch_leaf_r(const Leaf* items, const uint32_t* count, uint32_t cap, uint32_t grid, int cls,
                          Bufs<K, V> b, hipStream_t s) {
  constexpr bool big8 = sizeof(K) == 8 && HasVal<V>::value;
  switch (cls) {
    case 0:  // four one-wave sorters per workgroup
      hipLaunchKernelGGL((k_leaf<K, V, 64, 4, RANK, 4>), dim3((grid + 3) / 4), dim3(256), 0, s, items, count, cap, b);
      break;
    case 1:
      hipLaunchKernelGGL((k_leaf<K, V, 256, 4, RANK>), dim3(grid), dim3(256), 0, s, items, count, cap, b);
      break;
    case 2:
      hipLaunchKernelGGL((k_leaf<K, V, 256, 16, RANK>), dim3(grid), dim3(256), 0, s, items, count, cap, b);
      break;
    case 3:
      if constexpr (sizeof(K) == 8) {  // 16 waves for 8-byte keys (registers allow it at 8 keys each)
        hipLaunchKernelGGL((k_leaf<K, V, 1024, 8, RANK>), dim3(grid), dim3(1024), 0, s, items, count, cap, b);
      } else {
        hipLaunchKernelGGL((k_leaf<K, V, 512, 16, RANK>), dim3(grid), dim3(512), 0, s, items, count, cap, b);
      }
      break;
    default:
      if constexpr (big8) {
        hipLaunchKernelGGL((k_leaf<K, V, 1024, 8, RANK>), dim3(grid), dim3(1024), 0, s, items, count, cap, b);
      } else {
        hipLaunchKernelGGL((k_leaf<K, V, 1024, 16, RANK>), dim3(grid), dim3(1024), 0, s, items, count, cap, b);
      }
  }
}

template <typename K, typename V>
void launch_leaf(const Leaf* items, const uint32_t* count, uint32_t cap, uint32_t grid, int cls, Bufs<K, V> b,
                 hipStream_t s) {
  if (grid == 0 || cap == 0) return;
  const int m = leaf_rank_mode();
  if (m == RANK_BALLOT)
    launch_leaf_r<K, V, RANK_BALLOT>(items, count, cap, grid, cls, b, s);
  else if (m == RANK_HYBRID)
    launch_leaf_r<K, V, RANK_HYBRID>(items, count, cap, grid, cls, b, s);
  else if (m == RANK_PIPE)
    launch_leaf_r<K, V, RANK_PIPE>(items, count, cap, grid, cls, b, s);
  else
    launch_leaf_r<K, V, RANK_LDS>(items, count, cap, grid, cls, b, s);
}

template void launch_plan<uint32_t>(const LevelArgs&, const uint32_t*, const uint32_t*, int, hipStream_t);
template void launch_plan<uint64_t>(const LevelArgs&, const uint64_t*, const uint64_t*, int, hipStream_t);
#define DTS_INST(K, V)                                                                                           \
  template void launch_leaf<K, V>(const Leaf*, const uint32_t*, uint32_t, uint32_t, int, Bufs<K, V>, hipStream_t); \
  template void launch_pairs<K, V>(const Leaf*, const uint32_t*, uint32_t, uint32_t, uint32_t, Bufs<K, V>,         \
                                   hipStream_t);                                                                \
  template void launch_finish<K, V>(const Task*, const uint32_t*, uint32_t, uint32_t, Bufs<K, V>, hipStream_t);
DTS_INST(uint32_t, NoVal)
DTS_INST(uint64_t, NoVal)
DTS_INST(uint64_t, uint64_t)
DTS_INST(uint32_t, uint32_t)
#undef DTS_INST

}  // namespace dts

// Step 1 of Alg. 2 (Section 3.1; the sampled key range and overflow bucket of
// Section 5), one workgroup per subproblem, and the base case of Section 3.5
// (a stable sort in LDS), one workgroup per small subproblem.
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
template <typename K>
__global__ __launch_bounds__(1024) void k_plan(LevelArgs a, const K* k0, const K* k1) {
  constexpr int T = 1024;
  constexpr int ITEMS = sizeof(K) == 4 ? 32 : 16;
  constexpr int CAP = T * ITEMS;  // sample capacity
  __shared__ K sk[CAP];
  __shared__ uint32_t cnt[bsort_cnt_words<T>()];
  __shared__ K red[2 * (T / WAVE)];
  __shared__ uint32_t hz[1 << (GMAX - 1)];
  __shared__ uint32_t tmp[T / WAVE + 1];
  __shared__ int s_top, s_w, s_shift;

  const uint32_t n_tasks = a.ctr->cur_tasks;
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
  Task& tr = a.tasks[ti];
  const Task t = tr;
  if (t.flags & TF_LEARNED) continue;  // planned by the learned-partitioner step
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
    uint32_t ts = min(lgn, (uint32_t)(CAP >> g));
    ts = max(ts, 1u);
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
      block_radix_sort<K, T, ITEMS, false>(kk, dummy, trailing_zeros(diff), bit_length(diff), sk, nullptr, cnt,
                                           nullptr, (int)ns);
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
      const uint32_t j = threadIdx.x;  // nsub <= 1024
      bool f = false;
      K kj = 0;
      if (j + 1 < nsub) {
        kj = sk[j * ts];
        f = (kj == sk[(j + 1) * ts]) && (j == 0 || sk[(j - 1) * ts] != kj);
      }
      uint32_t total;
      const uint32_t idx = block_excl_scan<T>(f ? 1u : 0u, tmp, &total);
      nh = total;
      if (f) {
        gH[idx] = (uint64_t)kj;
        const K low = kj & mask_below<K>(hi);
        hz[idx] = (uint32_t)(shr<K>(low, s_shift) & (K)((1u << s_w) - 1u));
      }
      __syncthreads();
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
    gL[z] = z + lo;
  }
  if (threadIdx.x == 0) {
    tr.w = (uint8_t)w;
    tr.shift = (uint8_t)s_shift;
    tr.top = (uint8_t)s_top;
    tr.n_heavy = (uint16_t)nh;
    tr.n_buckets = (uint16_t)(zones + nh + 1);
  }
  __syncthreads();
  }
}

template <typename K>
void launch_plan(const LevelArgs& a, const K* k0, const K* k1, hipStream_t s) {
  hipLaunchKernelGGL(k_plan<K>, dim3(a.grid_tasks), dim3(1024), 0, s, a, k0, k1);
}

// ---------------------------------------------------------------- leaves
// Base case: a stable radix sort in LDS of a subproblem of at most T*ITEMS
// records, only over the bit range in which its keys differ.
template <typename K, typename V, int T, int ITEMS, int RANKREQ>
__global__ __launch_bounds__(T) void k_leaf(const Leaf* items, const uint32_t* count, uint32_t cap, Bufs<K, V> bf) {
  constexpr int N = T * ITEMS;
  constexpr bool HV = HasVal<V>::value;
  __shared__ K sk[N];
  __shared__ uint16_t si[HV ? N : 1];
  __shared__ uint32_t cnt[bsort_cnt_words<T>()];
  // LDS-match ranking (if requested and its tables fit next to the keys), else ballot ranking
  constexpr bool USE_LDS = RANKREQ != RANK_BALLOT && N * sizeof(K) + (HV ? N * 2 : 0) + 4 * bsort_cnt_words<T>() +
                                                         8 * bsort_match_words<T>() <= 150 * 1024;
  constexpr int RANK = USE_LDS ? RANKREQ : RANK_BALLOT;
  __shared__ unsigned long long mk[USE_LDS ? bsort_match_words<T>() : 1];
  __shared__ K red[2 * (T / WAVE)];
  if constexpr (USE_LDS) {
    for (int i = threadIdx.x; i < bsort_match_words<T>(); i += T) mk[i] = 0ull;
  }
  const uint32_t n_items = min(*count, cap);
  for (uint32_t li = blockIdx.x; li < n_items; li += gridDim.x) {
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
    block_radix_sort<K, T, ITEMS, HV, RANK>(kk, ix, trailing_zeros(diff), bit_length(diff), sk, si, cnt, mk, n);
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int e = striped_index<T, ITEMS>(i);
    if (e < n) kout[e] = kk[i];
  }
  if constexpr (HV) {
    const V* vin = bf.v[it.from] + it.off;
    V* vout = bf.v[it.to] + it.off;
    // gather all values first: `to` may equal `from`
    V vv[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<T, ITEMS>(i);
      if (e < n) vv[i] = vin[ix[i]];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<T, ITEMS>(i);
      if (e < n) vout[e] = vv[i];
    }
  }
  __syncthreads();
  }
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
    case 0:
      hipLaunchKernelGGL((k_leaf<K, V, 64, 4, RANK>), dim3(grid), dim3(64), 0, s, items, count, cap, b);
      break;
    case 1:
      hipLaunchKernelGGL((k_leaf<K, V, 256, 4, RANK>), dim3(grid), dim3(256), 0, s, items, count, cap, b);
      break;
    case 2:
      hipLaunchKernelGGL((k_leaf<K, V, 256, 16, RANK>), dim3(grid), dim3(256), 0, s, items, count, cap, b);
      break;
    case 3:
      hipLaunchKernelGGL((k_leaf<K, V, 512, 16, RANK>), dim3(grid), dim3(512), 0, s, items, count, cap, b);
      break;
    default:
      if constexpr (big8) {
        hipLaunchKernelGGL((k_leaf<K, V, 512, 16, RANK>), dim3(grid), dim3(512), 0, s, items, count, cap, b);
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

template void launch_plan<uint32_t>(const LevelArgs&, const uint32_t*, const uint32_t*, hipStream_t);
template void launch_plan<uint64_t>(const LevelArgs&, const uint64_t*, const uint64_t*, hipStream_t);
#define DTS_INST(K, V) \
  template void launch_leaf<K, V>(const Leaf*, const uint32_t*, uint32_t, uint32_t, int, Bufs<K, V>, hipStream_t);
DTS_INST(uint32_t, NoVal)
DTS_INST(uint64_t, NoVal)
DTS_INST(uint64_t, uint64_t)
DTS_INST(uint32_t, uint32_t)
#undef DTS_INST

}  // namespace dts

// Step 2 of Alg. 2 (Section 3.2, Appendix B): the stable counting sort of one
// recursion level's subproblems by bucket id, all subproblems in shared
// launches.
//
//   k_prep        per-task chunk counts, unit bases and count-matrix offsets
//   k_unit_fill   one (task, chunk) descriptor per distribution unit
//   k_hist        per unit: classify every key (GetBucketId) and count per bucket
//   k_colscan_*   per task and bucket: exclusive prefix over the task's chunks
//   k_bucketscan  per task: exclusive prefix over buckets -> bucket starts
//   k_scatter     per unit, tile by tile: stable rank by bucket (ballot match
//                 within a wave, per-wave counters in LDS), reorder the tile
//                 in LDS, then write every bucket's run contiguously
//
// The count matrix of a task is bucket-major: C[b * n_chunks + c], so the
// prefix "sum over j' < j, or j' = j and i' < i" of Appendix B is the
// column prefix plus the bucket start.
#include <cstdlib>

#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

// ------------------------------------------------------------------ prep
__global__ __launch_bounds__(1024) void k_prep(LevelArgs a) {
  __shared__ uint32_t tmp[17];
  __shared__ unsigned long long carry_cm;
  __shared__ uint32_t carry_u;
  if (threadIdx.x == 0) {
    carry_cm = 0;
    carry_u = 0;
  }
  __syncthreads();
  for (uint32_t base = 0; base < a.n_tasks; base += 1024) {
    const uint32_t ti = base + threadIdx.x;
    uint32_t nch = 0, cme = 0;
    if (ti < a.n_tasks) {
      const Task& t = a.tasks[ti];
      nch = (t.size + a.chunk - 1) / a.chunk;
      cme = nch * a.cols * (uint32_t)nb_cap(t.gamma);
    }
    uint32_t tot_u, tot_c;
    const uint32_t ub = block_excl_scan<1024>(nch, tmp, &tot_u);
    const uint32_t cb = block_excl_scan<1024>(cme, tmp, &tot_c);
    if (ti < a.n_tasks) {
      Task& t = a.tasks[ti];
      const uint64_t u0 = (uint64_t)carry_u + ub;
      const uint64_t c0 = carry_cm + cb;
      const uint64_t tab = (uint64_t)ti * a.slot_bytes;
      if (u0 + nch > a.caps.units || c0 + cme > a.caps.cm || tab + a.slot_bytes > a.caps.tab) {
        atomicOr(&a.ctr->error, ERR_UNITS);
        t.n_chunks = 0;
        t.unit_base = 0;
        t.cm_off = 0;
        t.tab_off = 0;
      } else {
        t.n_chunks = nch;
        t.unit_base = (uint32_t)u0;
        t.cm_off = c0;
        t.tab_off = tab;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry_u += tot_u;
      carry_cm += tot_c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.ctr->cur_units = min(carry_u, a.caps.units);
}

__global__ __launch_bounds__(256) void k_unit_fill(LevelArgs a) {
  const Task& t = a.tasks[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < t.n_chunks; j += 256) a.units[t.unit_base + j] = make_uint2(blockIdx.x, j);
}

void launch_prep(const LevelArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_unit_fill, dim3(a.n_tasks), dim3(256), 0, s, a);
}

// Ranking mode of the scatter (tuning knob: DTSORT_RANK=ballot|lds).
static int rank_mode() {
  static int m = [] {
    const char* e = getenv("DTSORT_RANK");
    if (e && e[0] == 'b') return (int)RANK_BALLOT;
    if (e && e[0] == 'h') return (int)RANK_HYBRID;
    if (e && e[0] == 'p') return (int)RANK_PIPE;
    return (int)RANK_LDS;
  }();
  return m;
}

// ------------------------------------------------------- table loading
template <typename K, int THREADS>
__device__ inline void load_tables(const Task& t, const uint8_t* tab, uint32_t* L, K* H, K* SPL) {
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  const uint8_t* slot = tab + t.tab_off;
  const uint32_t* gL = (const uint32_t*)(slot + sl.light);
  const uint64_t* gH = (const uint64_t*)(slot + sl.heavy);
  const uint32_t zones = 1u << t.w;
  for (uint32_t i = threadIdx.x; i <= zones; i += THREADS) L[i] = gL[i];
  for (uint32_t i = threadIdx.x; i < t.n_heavy; i += THREADS) H[i] = (K)gH[i];
  if (t.flags & TF_LEARNED) {
    const uint64_t* gS = (const uint64_t*)(slot + sl.spl);
    for (uint32_t i = threadIdx.x; i + 1 < zones; i += THREADS) SPL[i] = (K)gS[i];
  }
}

// ------------------------------------------------------------- histogram
// PERWAVE: every wave counts its own contiguous share of the chunk and
// writes its own count-matrix column (for the direct scatter); otherwise the
// workgroup's counts go to one column per chunk.
template <typename K, int T, int ITEMS, int NBMAX, bool PERWAVE>
__global__ __launch_bounds__(T) void k_hist(LevelArgs a, const K* k0, const K* k1) {
  constexpr int WAVES = T / WAVE;
  if (blockIdx.x >= a.ctr->cur_units) return;
  __shared__ uint32_t hist[WAVES * NBMAX];
  __shared__ uint32_t L[(1 << GMAX) + 1];
  __shared__ K H[1 << (GMAX - 1)];
  __shared__ K SPL[1 << GMAX];
  const uint2 u = a.units[blockIdx.x];
  const Task t = a.tasks[u.x];
  if (t.n_chunks == 0) return;
  load_tables<K, T>(t, a.tab, L, H, SPL);
  for (int i = threadIdx.x; i < WAVES * NBMAX; i += T) hist[i] = 0;
  __syncthreads();
  const PlanRegs<K> pr = plan_regs<K>(t);
  const K* keys = (t.src ? k1 : k0) + t.off;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t* hw = hist + wv * NBMAX;
  uint32_t beg = u.y * a.chunk;
  uint32_t end = min(t.size, beg + a.chunk);
  int step = T, lid = threadIdx.x;
  if constexpr (PERWAVE) {
    const uint32_t sub = a.chunk / WAVES;
    beg = min(end, beg + wv * sub);
    end = min(end, beg + sub);
    step = WAVE;
    lid = lane;
  }
  for (uint32_t base = beg; base < end; base += step * ITEMS) {
    K kk[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t e = base + i * step + lid;
      kk[i] = e < end ? keys[e] : (K)0;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t e = base + i * step + lid;
      const bool valid = e < end;
      const uint32_t b = valid ? bucket_of<K>(kk[i], pr, L, H, SPL) : 0u;
      const uint64_t act = __ballot(valid);
      if (act == 0) continue;
      const int first = __builtin_ctzll(act);
      const uint32_t b0 = __shfl(b, first, WAVE);
      const uint64_t same = __ballot(valid && b == b0);
      if (same == act) {
        if (lane == first) atomicAdd(&hw[b0], (uint32_t)__popcll(act));
      } else if (valid) {
        atomicAdd(&hw[b], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t ncol = t.n_chunks * a.cols;
  for (uint32_t b = threadIdx.x; b < t.n_buckets; b += T) {
    if constexpr (PERWAVE) {
#pragma unroll
      for (int w = 0; w < WAVES; ++w) a.cm[t.cm_off + (uint64_t)b * ncol + u.y * WAVES + w] = hist[w * NBMAX + b];
    } else {
      uint32_t s = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) s += hist[w * NBMAX + b];
      a.cm[t.cm_off + (uint64_t)b * ncol + u.y] = s;
    }
  }
}

// ------------------------------------------------------- column scans
// One wave per (task, bucket): exclusive scan over the task's chunks; the
// bucket total goes to the slot's bucket-start array (scanned next).
__global__ __launch_bounds__(256) void k_colscan_wave(LevelArgs a) {
  const Task t = a.tasks[blockIdx.x];
  const uint32_t b = blockIdx.y * 4 + threadIdx.x / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (b >= t.n_buckets || t.n_chunks == 0) return;
  const uint32_t ncol = t.n_chunks * a.cols;
  uint32_t* col = a.cm + t.cm_off + (uint64_t)b * ncol;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < ncol; c0 += WAVE) {
    const uint32_t c = c0 + lane;
    const uint32_t v = c < ncol ? col[c] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, WAVE);
      if (lane >= o) x += y;
    }
    if (c < ncol) col[c] = carry + x - v;
    carry += __shfl(x, WAVE - 1, WAVE);
  }
  if (lane == 0) {
    const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
    uint32_t* starts = (uint32_t*)(a.tab + t.tab_off + sl.starts);
    starts[b] = carry;
  }
}

// One thread per (task, bucket), for levels whose tasks have few chunks.
__global__ __launch_bounds__(256) void k_colscan_thread(LevelArgs a) {
  const Task t = a.tasks[blockIdx.x];
  if (t.n_chunks == 0) return;
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  uint32_t* starts = (uint32_t*)(a.tab + t.tab_off + sl.starts);
  const uint32_t ncol = t.n_chunks * a.cols;
  for (uint32_t b = threadIdx.x; b < t.n_buckets; b += 256) {
    uint32_t* col = a.cm + t.cm_off + (uint64_t)b * ncol;
    uint32_t run = 0;
    for (uint32_t c = 0; c < ncol; ++c) {
      const uint32_t v = col[c];
      col[c] = run;
      run += v;
    }
    starts[b] = run;
  }
}

template <int NBMAX>
__global__ __launch_bounds__(256) void k_bucketscan(LevelArgs a) {
  __shared__ uint32_t s[NBMAX + 1];
  __shared__ uint32_t tmp[5];
  const Task t = a.tasks[blockIdx.x];
  if (t.n_chunks == 0) return;
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  uint32_t* starts = (uint32_t*)(a.tab + t.tab_off + sl.starts);
  for (uint32_t b = threadIdx.x; b < t.n_buckets; b += 256) s[b] = starts[b];
  __syncthreads();
  const uint32_t total = block_excl_scan_array<256>(s, t.n_buckets, tmp);
  for (uint32_t b = threadIdx.x; b < t.n_buckets; b += 256) starts[b] = s[b];
  if (threadIdx.x == 0) starts[t.n_buckets] = total;
}

// ---------------------------------------------------------------- scatter
// One distribution unit (a chunk of one task), tile by tile:
//  1. keys of the tile are in registers (the next tile's loads are already in
//     flight); classify each key (GetBucketId);
//  2. rank: per wave, the lanes with the same bucket (LDS match or ballot
//     match) and a running per-(wave, bucket) count give each key its place
//     among the wave's keys of its bucket, in input order;
//  3. bucket totals of the tile, an exclusive scan over buckets, and per
//     (wave, bucket) bases turn that into the key's place in the tile sorted
//     by bucket; the tile is reordered in LDS;
//  4. consecutive threads write consecutive records of each bucket's run to
//     its next free place in the bucket (global offset - tile start + index).
// Equal buckets keep input order at every step: the scatter is stable.
template <typename K, typename V, int T, int ITEMS, int NBMAX, int RANK>
__global__ __launch_bounds__(T) void k_scatter(LevelArgs a, Bufs<K, V> bf) {
  constexpr int WAVES = T / WAVE;
  constexpr int TILE = T * ITEMS;
  constexpr int PER = (NBMAX + T - 1) / T;  // buckets per thread in the bucket phase
  constexpr bool HV = HasVal<V>::value;
  static_assert(!HV || sizeof(V) <= sizeof(K), "values are staged in the key buffer");
  __shared__ uint32_t cnt[WAVES * NBMAX];
  __shared__ unsigned long long mk[RANK == RANK_BALLOT ? 1 : WAVES * NBMAX];  // zeroed match tables
  __shared__ uint32_t run_off[NBMAX];
  __shared__ int32_t gdelta[NBMAX];
  __shared__ uint32_t L[(1 << GMAX) + 1];
  __shared__ K H[1 << (GMAX - 1)];
  __shared__ K SPL[1 << GMAX];
  __shared__ K stage[TILE];
  __shared__ uint16_t stage_b[TILE];
  __shared__ uint32_t tmp[WAVES + 1];

  if (blockIdx.x >= a.ctr->cur_units) return;
  const uint2 u = a.units[blockIdx.x];
  const Task t = a.tasks[u.x];
  if (t.n_chunks == 0) return;
  load_tables<K, T>(t, a.tab, L, H, SPL);
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  const uint32_t* starts = (const uint32_t*)(a.tab + t.tab_off + sl.starts);
  const uint32_t nb = t.n_buckets;
  for (uint32_t b = threadIdx.x; b < nb; b += T)
    run_off[b] = starts[b] + a.cm[t.cm_off + (uint64_t)b * t.n_chunks * a.cols + u.y];
  if constexpr (RANK != RANK_BALLOT) {
    for (int i = threadIdx.x; i < WAVES * NBMAX; i += T) mk[i] = 0ull;
  }
  __syncthreads();

  const PlanRegs<K> pr = plan_regs<K>(t);
  const K* kin = bf.k[t.src] + t.off;
  K* kout = bf.k[1 - t.src] + t.off;
  const int nbits = nb > 1 ? 32 - __builtin_clz(nb - 1) : 1;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t* crow = cnt + wv * NBMAX;
  unsigned long long* wm = mk + (RANK != RANK_BALLOT ? wv * NBMAX : 0);
  const uint32_t beg = u.y * a.chunk;
  const uint32_t end = min(t.size, beg + a.chunk);

  K nxt[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t e = beg + (uint32_t)striped_index<T, ITEMS>(i);
    nxt[i] = e < end ? kin[e] : (K)0;
  }
  for (uint32_t base = beg; base < end; base += TILE) {
    const uint32_t tile_n = min((uint32_t)TILE, end - base);
    K kk[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) kk[i] = nxt[i];
    if (base + TILE < end) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = base + TILE + (uint32_t)striped_index<T, ITEMS>(i);
        nxt[i] = e < end ? kin[e] : (K)0;
      }
    }
    // each wave clears its own counter row (only that wave ranks with it)
    for (uint32_t j = lane; j < nb; j += WAVE) crow[j] = 0;
    uint32_t bk[ITEMS];
    uint32_t pos[ITEMS];
    if constexpr (RANK == RANK_PIPE) {
      bool vl[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        vl[i] = (uint32_t)striped_index<T, ITEMS>(i) < tile_n;
        bk[i] = vl[i] ? bucket_of<K>(kk[i], pr, L, H, SPL) : 0u;
      }
      rank_pipelined<ITEMS>(bk, vl, wm, crow, pos);
    }
#pragma unroll
    for (int i = 0; i < (RANK == RANK_PIPE ? 0 : ITEMS); ++i) {
      const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
      const bool valid = e < tile_n;
      const uint32_t b = valid ? bucket_of<K>(kk[i], pr, L, H, SPL) : 0u;
      bk[i] = b;
      uint64_t peers;
      if constexpr (RANK == RANK_LDS) {
        peers = lds_match(wm, b, valid);
      } else if constexpr (RANK == RANK_HYBRID) {
        peers = hybrid_match(wm, b, nbits, valid);
      } else {
        peers = match_peers(b, nbits, valid);
      }
      const uint32_t r = mbcnt(peers);
      const uint32_t c = (uint32_t)__popcll(peers);
      uint32_t p = 0;
      if (valid) {
        const uint32_t cb = crow[b];
        p = cb + r;
        if (r == 0) crow[b] = cb + c;
      }
      pos[i] = p;
    }
    __syncthreads();
    {
      // buckets [b0, b0 + PER) of this thread: totals, tile starts, wave bases
      const uint32_t b0 = threadIdx.x * PER;
      uint32_t sb[PER];
      uint32_t S = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t b = b0 + j;
        uint32_t x = 0;
        if (b < nb) {
#pragma unroll
          for (int w = 0; w < WAVES; ++w) x += cnt[w * NBMAX + b];
        }
        sb[j] = x;
        S += x;
      }
      uint32_t total;
      uint32_t run = block_excl_scan<T>(S, tmp, &total);
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t b = b0 + j;
        if (b < nb) {
          gdelta[b] = (int32_t)run_off[b] - (int32_t)run;
          run_off[b] += sb[j];
          uint32_t r2 = run;
#pragma unroll
          for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = cnt[w * NBMAX + b];
            cnt[w * NBMAX + b] = r2;
            r2 += c;
          }
        }
        run += sb[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
      if (e < tile_n) {
        const uint32_t p = pos[i] + crow[bk[i]];
        pos[i] = p;
        stage[p] = kk[i];
        stage_b[p] = (uint16_t)bk[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint32_t j = threadIdx.x + it * T;
      if (j < tile_n) {
        const uint32_t gp = (uint32_t)(gdelta[stage_b[j]] + (int32_t)j);
        if (gp < t.size) kout[gp] = stage[j];
      }
    }
    if constexpr (HV) {
      const V* vin = bf.v[t.src] + t.off;
      V* vout = bf.v[1 - t.src] + t.off;
      V* vstage = reinterpret_cast<V*>(stage);
      V vv[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
        if (e < tile_n) vv[i] = vin[base + e];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
        if (e < tile_n) vstage[pos[i]] = vv[i];
      }
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < tile_n; j += T) {
        const uint32_t gp = (uint32_t)(gdelta[stage_b[j]] + (int32_t)j);
        if (gp < t.size) vout[gp] = vstage[j];
      }
    }
    __syncthreads();
  }
}

// Direct variant: every wave owns a contiguous share of the chunk with its
// own per-bucket write cursors (from its own count-matrix column), ranks its
// keys with the LDS match and writes each record straight to its final place
// in the bucket.  No block-wide phase and no staging; stable because each
// wave visits its keys in input order and cursors of consecutive waves are
// consecutive in the prefix.
template <typename K, typename V, int T, int ITEMS, int NBMAX>
__global__ __launch_bounds__(T) void k_scatter_direct(LevelArgs a, Bufs<K, V> bf) {
  constexpr int WAVES = T / WAVE;
  constexpr bool HV = HasVal<V>::value;
  __shared__ uint32_t cur[WAVES * NBMAX];
  __shared__ unsigned long long mk[WAVES * NBMAX];
  __shared__ uint32_t L[(1 << GMAX) + 1];
  __shared__ K H[1 << (GMAX - 1)];
  __shared__ K SPL[1 << GMAX];
  if (blockIdx.x >= a.ctr->cur_units) return;
  const uint2 u = a.units[blockIdx.x];
  const Task t = a.tasks[u.x];
  if (t.n_chunks == 0) return;
  load_tables<K, T>(t, a.tab, L, H, SPL);
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  const uint32_t* starts = (const uint32_t*)(a.tab + t.tab_off + sl.starts);
  const uint32_t nb = t.n_buckets;
  const uint32_t ncol = t.n_chunks * WAVES;
  for (uint32_t b = threadIdx.x; b < nb; b += T) {
    const uint32_t s0 = starts[b];
    const uint32_t* col = a.cm + t.cm_off + (uint64_t)b * ncol + u.y * WAVES;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) cur[w * NBMAX + b] = s0 + col[w];
  }
  for (int i = threadIdx.x; i < WAVES * NBMAX; i += T) mk[i] = 0ull;
  __syncthreads();
  const PlanRegs<K> pr = plan_regs<K>(t);
  const K* kin = bf.k[t.src] + t.off;
  K* kout = bf.k[1 - t.src] + t.off;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t* crow = cur + wv * NBMAX;
  unsigned long long* wm = mk + wv * NBMAX;
  const uint32_t cend = min(t.size, u.y * a.chunk + a.chunk);
  const uint32_t sub = a.chunk / WAVES;
  const uint32_t beg = min(cend, u.y * a.chunk + wv * sub);
  const uint32_t end = min(cend, beg + sub);
  constexpr uint32_t STEP = WAVE * ITEMS;
  K nxt[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t e = beg + i * WAVE + lane;
    nxt[i] = e < end ? kin[e] : (K)0;
  }
  for (uint32_t base = beg; base < end; base += STEP) {
    K kk[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) kk[i] = nxt[i];
    if (base + STEP < end) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = base + STEP + i * WAVE + lane;
        nxt[i] = e < end ? kin[e] : (K)0;
      }
    }
    V vv[HV ? ITEMS : 1];
    if constexpr (HV) {
      const V* vin = bf.v[t.src] + t.off;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t e = base + i * WAVE + lane;
        if (e < end) vv[i] = vin[e];
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t e = base + i * WAVE + lane;
      const bool valid = e < end;
      const uint32_t b = valid ? bucket_of<K>(kk[i], pr, L, H, SPL) : 0u;
      const uint64_t peers = lds_match(wm, b, valid);
      const uint32_t r = mbcnt(peers);
      const uint32_t c = (uint32_t)__popcll(peers);
      if (valid) {
        const uint32_t cb = crow[b];
        if (r == 0) crow[b] = cb + c;
        const uint32_t gp = cb + r;
        if (gp < t.size) {
          kout[gp] = kk[i];
          if constexpr (HV) (bf.v[1 - t.src] + t.off)[gp] = vv[i];
        }
      }
    }
  }
}

template <typename K, typename V, int NBMAX, int T, int RANK, bool DIRECT, int SITEMS_REQ = 0>
static void launch_dist_variant(const LevelArgs& a, Bufs<K, V> b, uint32_t max_chunks, hipStream_t s, int phase) {
  constexpr int HITEMS = sizeof(K) == 4 ? 16 : 8;
  constexpr int SITEMS = SITEMS_REQ ? SITEMS_REQ : (sizeof(K) == 4 ? 16 : 8);
  const uint32_t nu = a.caps.units;  // bound on the units; k_prep stores the exact count
  if (phase < 0 || phase == 0)
    hipLaunchKernelGGL((k_hist<K, T, HITEMS, NBMAX, DIRECT>), dim3(nu), dim3(T), 0, s, a, (const K*)b.k[0],
                       (const K*)b.k[1]);
  if (phase < 0 || phase == 1) {
    if (max_chunks * a.cols > 32) {
      hipLaunchKernelGGL(k_colscan_wave, dim3(a.n_tasks, (NBMAX + 3) / 4), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_colscan_thread, dim3(a.n_tasks), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((k_bucketscan<NBMAX>), dim3(a.n_tasks), dim3(256), 0, s, a);
  }
  if (phase < 0 || phase == 2) {
    if constexpr (DIRECT) {
      hipLaunchKernelGGL((k_scatter_direct<K, V, T, SITEMS, NBMAX>), dim3(nu), dim3(T), 0, s, a, b);
    } else {
      hipLaunchKernelGGL((k_scatter<K, V, T, SITEMS, NBMAX, RANK>), dim3(nu), dim3(T), 0, s, a, b);
    }
  }
}

// Tile shape of the staged scatter for digit widths <= 8 (tuning knob
// DTSORT_SCATTER_CFG): 0 = 512 threads x 16 keys (x 8 for 64-bit keys),
// 1 = 256 x 16, 2 = 512 x 8, 3 = 256 x 32.
static int scatter_cfg() {
  static int m = [] {
    const char* e = getenv("DTSORT_SCATTER_CFG");
    return e ? atoi(e) : 0;
  }();
  return m;
}

// Scatter variant (tuning knob: DTSORT_SCATTER=staged|direct).
static bool direct_mode() {
  static int m = [] {
    const char* e = getenv("DTSORT_SCATTER");
    return (e && e[0] == 'd') ? 1 : 0;
  }();
  return m != 0;
}

uint32_t dist_cols(int g_level_max) {
  if (!direct_mode()) return 1;
  return g_level_max <= 8 ? 512 / WAVE : 256 / WAVE;
}

template <typename K, typename V>
void launch_distribute(const LevelArgs& a, Bufs<K, V> b, int g_level_max, uint32_t max_chunks, hipStream_t s,
                       int phase) {
  if (direct_mode()) {
    if (g_level_max <= 8)
      launch_dist_variant<K, V, 512, 512, RANK_LDS, true>(a, b, max_chunks, s, phase);
    else
      launch_dist_variant<K, V, 2048, 256, RANK_LDS, true>(a, b, max_chunks, s, phase);
    return;
  }
  if (g_level_max <= 8) {
    const int cfg = scatter_cfg();
    if (rank_mode() == RANK_BALLOT)
      launch_dist_variant<K, V, 512, 512, RANK_BALLOT, false>(a, b, max_chunks, s, phase);
    else if (rank_mode() == RANK_HYBRID)
      launch_dist_variant<K, V, 512, 512, RANK_HYBRID, false>(a, b, max_chunks, s, phase);
    else if (rank_mode() == RANK_PIPE && cfg == 0)
      launch_dist_variant<K, V, 512, 512, RANK_PIPE, false>(a, b, max_chunks, s, phase);
    else if (rank_mode() == RANK_PIPE)
      launch_dist_variant<K, V, 512, 256, RANK_PIPE, false>(a, b, max_chunks, s, phase);
    else if (cfg == 1)
      launch_dist_variant<K, V, 512, 256, RANK_LDS, false>(a, b, max_chunks, s, phase);
    else if (cfg == 2)
      launch_dist_variant<K, V, 512, 512, RANK_LDS, false, sizeof(K) == 4 ? 8 : 4>(a, b, max_chunks, s, phase);
    else if (cfg == 3)
      launch_dist_variant<K, V, 512, 256, RANK_LDS, false, sizeof(K) == 4 ? 32 : 16>(a, b, max_chunks, s, phase);
    else
      launch_dist_variant<K, V, 512, 512, RANK_LDS, false>(a, b, max_chunks, s, phase);
  } else {
    if (rank_mode() == RANK_BALLOT)
      launch_dist_variant<K, V, 2048, 256, RANK_BALLOT, false>(a, b, max_chunks, s, phase);
    else if (rank_mode() == RANK_PIPE)
      launch_dist_variant<K, V, 2048, 256, RANK_PIPE, false>(a, b, max_chunks, s, phase);
    else
      launch_dist_variant<K, V, 2048, 256, RANK_LDS, false>(a, b, max_chunks, s, phase);
  }
}

#define DTS_INST(K, V) \
  template void launch_distribute<K, V>(const LevelArgs&, Bufs<K, V>, int, uint32_t, hipStream_t, int);
DTS_INST(uint32_t, NoVal)
DTS_INST(uint64_t, NoVal)
DTS_INST(uint64_t, uint64_t)
DTS_INST(uint32_t, uint32_t)
#undef DTS_INST

}  // namespace dts

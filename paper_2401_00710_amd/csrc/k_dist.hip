// Step 2 of Alg. 2 (Section 3.2, Appendix B): the stable counting sort of one
// recursion level's subproblems by bucket id, all subproblems in shared
// launches.
//
//   k_prep        per-task chunk counts, unit bases and count-matrix offsets
//   k_unit_fill   one (task, chunk) descriptor per distribution unit
//   k_hist        per unit: classify every key (GetBucketId) and count per bucket
//   k_colscan     per task and bucket: exclusive prefix over the task's chunks
//   k_bucketscan  per task: exclusive prefix over buckets -> bucket starts
//   k_scatter     per unit, tile by tile: stable rank by bucket (ballot match
//                 within a wave, per-wave counters in LDS), reorder the tile
//                 in LDS, then write every bucket's run contiguously
//
// The count matrix of a task is bucket-major: C[b * n_chunks + c], so the
// prefix "sum over j' < j, or j' = j and i' < i" of Appendix B is the
// column prefix plus the bucket start.
#include <cstdlib>
#include <type_traits>

#include "block_sort.hpp"
#include "launch.hpp"

namespace dts {

// ------------------------------------------------------------------ prep
// One workgroup: zero this level's counters, take the task count and the
// record count from the counters of the step that made the tasks, choose the
// chunk (when the host has not), and give every task its unit base,
// count-matrix offset and table slot.
__global__ __launch_bounds__(1024) void k_prep(LevelArgs a) {
  __shared__ uint32_t tmp[17];
  __shared__ unsigned long long carry_cm;
  __shared__ uint32_t carry_u;
  __shared__ uint32_t s_err;
  uint32_t* cw = reinterpret_cast<uint32_t*>(a.ctr);
  for (uint32_t i = threadIdx.x; i < sizeof(LevelCounters) / 4; i += 1024) cw[i] = 0u;
  if (threadIdx.x == 0) {
    carry_cm = 0;
    carry_u = 0;
    s_err = 0;
  }
  const uint32_t n_tasks = min(a.in->next_tasks, a.n_tasks);
  uint32_t chunk = a.chunk;
  if (chunk == 0) {
    // about 2048 units over the level's records, a multiple of 8192
    const uint64_t total = a.in->next_records;
    uint64_t c = (total + 2047) / 2048;
    c = (c + 8191) / 8192 * 8192;
    chunk = (uint32_t)max<uint64_t>(8192, c);
  }
  __syncthreads();
  for (uint32_t base = 0; base < n_tasks; base += 1024) {
    const uint32_t ti = base + threadIdx.x;
    uint32_t nch = 0, cme = 0;
    if (ti < n_tasks) {
      const Task& t = a.tasks[ti];
      nch = t.size / chunk + (t.size % chunk != 0u ? 1u : 0u);  // no wrap for sizes near 2^32
      cme = nch * a.cols * (uint32_t)nb_cap(t.gamma);
    }
    uint32_t tot_u, tot_c;
    const uint32_t ub = block_excl_scan<1024>(nch, tmp, &tot_u);
    const uint32_t cb = block_excl_scan<1024>(cme, tmp, &tot_c);
    if (ti < n_tasks) {
      Task& t = a.tasks[ti];
      const uint64_t u0 = (uint64_t)carry_u + ub;
      const uint64_t c0 = carry_cm + cb;
      const uint64_t tab = (uint64_t)ti * a.slot_bytes;
      if (u0 + nch > a.caps.units || c0 + cme > a.caps.cm || tab + a.slot_bytes > a.caps.tab) {
        s_err = 1;
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
  if (threadIdx.x == 0) {
    a.ctr->cur_units = min(carry_u, a.caps.units);
    a.ctr->cur_tasks = n_tasks;
    a.ctr->chunk = chunk;
    // a capacity overflow of the step that made these tasks, or of this one
    a.ctr->error = (a.in->next_tasks > a.n_tasks ? ERR_TASKS : 0u) | (s_err ? ERR_UNITS : 0u);
  }
}

__global__ __launch_bounds__(256) void k_unit_fill(LevelArgs a) {
  const uint32_t n_tasks = a.ctr->cur_tasks;
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const Task& t = a.tasks[ti];
    for (uint32_t j = threadIdx.x; j < t.n_chunks; j += 256) a.units[t.unit_base + j] = make_uint2(ti, j);
  }
}

void launch_prep(const LevelArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_unit_fill, dim3(a.grid_tasks), dim3(256), 0, s, a);
}

// Ranking mode of the scatter (tuning knob: DTSORT_RANK=ballot|lds|hybrid|
// pipe|atomic; atomic applies to keys without values only).  Unset: atomic
// for keys without values, lds otherwise.
static int rank_mode() {
  static int m = [] {
    const char* e = getenv("DTSORT_RANK");
    if (e && e[0] == 'b') return (int)RANK_BALLOT;
    if (e && e[0] == 'h') return (int)RANK_HYBRID;
    if (e && e[0] == 'p') return (int)RANK_PIPE;
    if (e && e[0] == 'a') return (int)RANK_ATOMIC;
    return (int)RANK_LDS;
  }();
  return m;
}
static bool rank_mode_forced() {
  static bool f = getenv("DTSORT_RANK") != nullptr;
  return f;
}

// Counter rows of the variants for digits of at most 8 bits: 2^8 light,
// 2^7 heavy and one overflow bucket, rounded up to a multiple of 8.
constexpr int NB8 = (nb_cap(8) + 7) / 8 * 8;
// ... and of the 9-bit variant (bare keys with unordered ranks only).
constexpr int NB9 = (nb_cap(9) + 7) / 8 * 8;

// ------------------------------------------------------- table loading
// With HT (variants of at most 8-bit digits, whose tasks have at most
// HT_MAX_KEYS heavy keys) the heavy keys also go into the hash table HT, with
// HC (HT_SLOTS words) counting the keys of each slot and *hfull set when a
// slot overflows (then the keys are searched instead).  A barrier must
// follow before the tables are read.
template <typename K, int THREADS>
__device__ inline void load_tables(const Task& t, const uint8_t* tab, uint32_t* L, K* H, K* SPL, uint32_t* HT,
                                   uint32_t* HC, uint32_t* hfull) {
  const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
  const uint8_t* slot = tab + t.tab_off;
  const uint32_t* gL = (const uint32_t*)(slot + sl.light);
  const uint64_t* gH = (const uint64_t*)(slot + sl.heavy);
  const uint32_t zones = 1u << t.w;
  for (uint32_t i = threadIdx.x; i <= zones; i += THREADS) L[i] = gL[i];
  for (uint32_t i = threadIdx.x; i < t.n_heavy; i += THREADS) H[i] = (K)gH[i];
  if (HT != nullptr && t.n_heavy != 0) {
    for (int i = threadIdx.x; i < HT_SLOTS; i += THREADS) {
      HT[i] = 0xFFFFFFFFu;
      HC[i] = 0u;
    }
    if (threadIdx.x == 0) *hfull = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < t.n_heavy; i += THREADS) {
      const uint32_t s = heavy_slot<K>((K)gH[i]);
      const uint32_t r = atomicAdd(&HC[s], 1u);
      if (r < (uint32_t)HT_WAYS)
        atomicAnd(&HT[s], ~(0xFFu << (8u * r)) | (i << (8u * r)));  // byte r was 0xFF
      else
        atomicOr(hfull, 1u);
    }
  }
  if (t.flags & TF_LEARNED) {
    const uint64_t* gS = (const uint64_t*)(slot + sl.spl);
    for (uint32_t i = threadIdx.x; i + 1 < zones; i += THREADS) SPL[i] = (K)gS[i];
  }
}

// ------------------------------------------------------------- histogram
// Units with a grid stride; the workgroup's counts of a unit go to its
// column of the task's count matrix.
// SPLIT: tasks in the split bucket layout (bucket_of<K, true>).
// At least 6 waves a SIMD (at most 80 VGPRs): three 512-thread workgroups
// share a CU, which hides the LDS latency of the heavy-key lookups; 8 waves
// would spill the 32-bit variants.
template <typename K, int T, int ITEMS, int NBMAX, bool SPLIT = false>
__global__ __launch_bounds__(T, 6) void k_hist(LevelArgs a, const K* k0, const K* k1) {
  constexpr int WAVES = T / WAVE;
  constexpr int GM = NBMAX <= NB8 ? 8 : (NBMAX <= NB9 ? 9 : GMAX);  // widest digit of this variant
  // two counter rows per wave on the <= 8-bit variants, for even and odd
  // lanes: lanes of one wave that count the same hot (heavy) bucket then
  // split over two addresses
  constexpr int HC2 = NBMAX <= NB8 ? 2 : 1;
  __shared__ uint32_t hist[WAVES * HC2 * NBMAX];
  __shared__ uint32_t L[(1 << GM) + 1];
  __shared__ K H[1 << (GM - 1)];
  constexpr bool HASH = GM == 8;  // heavy keys fit the hash table
  static_assert(!HASH || (1 << (GM - 1)) <= HT_MAX_KEYS, "heavy indices fit a byte");
  __shared__ uint32_t HT[HASH ? HT_SLOTS : 1];
  __shared__ uint32_t HC[HASH ? HT_SLOTS : 1];
  __shared__ uint32_t hfull;
  __shared__ K SPL[1 << GM];
  const uint32_t n_units = a.ctr->cur_units;
  const uint32_t chunk = a.ctr->chunk;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t* hw = hist + (wv * HC2 + (HC2 == 2 ? (lane & 1) : 0)) * NBMAX;
  for (uint32_t ui = blockIdx.x; ui < n_units; ui += gridDim.x) {
    const uint2 u = a.units[ui];
    const Task t = a.tasks[u.x];
    if (t.n_chunks == 0) continue;
    load_tables<K, T>(t, a.tab, L, H, SPL, HASH ? HT : nullptr, HC, &hfull);
    for (int i = threadIdx.x; i < WAVES * HC2 * NBMAX; i += T) hist[i] = 0;
    __syncthreads();
    PlanRegs<K> pr = plan_regs<K>(t);
    pr.hashed = HASH && pr.heavy && hfull == 0u && !(SPLIT && pr.split);
    const K* keys = (t.src ? k1 : k0) + t.off;
    const uint32_t beg = u.y * chunk;
    const uint32_t end = beg + min(chunk, t.size - beg);  // no wrap for sizes near 2^32
    // a short first tile up to the next 16-byte boundary; every later whole
    // tile is then read with 16-byte loads
    constexpr int VEC = 16 / (int)sizeof(K);  // keys per 16-byte load
    static_assert(ITEMS % VEC == 0, "whole 16-byte loads");
    const uint32_t mis = (uint32_t)(reinterpret_cast<uintptr_t>(keys + beg) & 15u) / (uint32_t)sizeof(K);
    const uint32_t head = mis ? (uint32_t)VEC - mis : 0u;
    for (uint32_t base = beg; base < end;) {
      const uint32_t len = (base == beg && head) ? min(head, end - base) : min((uint32_t)(T * ITEMS), end - base);
      // loads past the end of the tile read zero; those lanes are masked below
      const __amdgpu_buffer_rsrc_t rk = buf_rsrc(keys + base, len * (uint32_t)sizeof(K));
      K kk[ITEMS];
      if (len == (uint32_t)(T * ITEMS)) {
        // which key lands in which register does not matter for counting
#pragma unroll
        for (int j = 0; j < ITEMS / VEC; ++j)
          buf_load16<K>(rk, (uint32_t)(j * T + threadIdx.x) * 16u, kk + j * VEC);
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) kk[i] = buf_load<K>(rk, (uint32_t)(i * T + threadIdx.x) * sizeof(K));
      }
      // whole tiles (the common case) without per-key bounds checks
      auto count = [&](auto whole) {
        constexpr bool W = decltype(whole)::value;
        uint32_t bb[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t e = i * T + threadIdx.x;  // place in the tile
          bb[i] = (W || e < len) ? bucket_of<K, SPLIT>(kk[i], pr, L, H, SPL, HT) : 0u;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t e = i * T + threadIdx.x;
          const bool valid = W || e < len;
          const uint32_t b = bb[i];
          const uint64_t act = W ? ~0ull : __ballot(valid);
          if (act == 0) continue;
          // the valid lanes are a prefix of the wave, so lane 0 is one of
          // them; a row of one bucket takes one atomic
          const uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
          const uint64_t same = __ballot(valid && b == b0);
          if (same == act) {
            if (lane == 0) atomicAdd(&hw[b0], (uint32_t)__popcll(act));
          } else if (valid) {
            atomicAdd(&hw[b], 1u);
          }
        }
      };
      if (len == (uint32_t)(T * ITEMS))
        count(std::true_type{});
      else
        count(std::false_type{});
      base += len;
    }
    __syncthreads();
    const uint32_t ncol = t.n_chunks * a.cols;
    for (uint32_t b = threadIdx.x; b < t.n_buckets; b += T) {
      uint32_t s = 0;
#pragma unroll
      for (int w = 0; w < WAVES * HC2; ++w) s += hist[w * NBMAX + b];
      a.cm[t.cm_off + (uint64_t)b * ncol + u.y] = s;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- column scans
// Per (task, bucket): exclusive scan of the bucket's counts over the task's
// chunks; the bucket total goes to the slot's bucket-start array (scanned
// next).  Tasks of at most 32 columns take one thread per bucket (workgroups
// with blockIdx.y = 0); longer ones one wave per bucket, the buckets spread
// over blockIdx.y.
__global__ __launch_bounds__(256) void k_colscan(LevelArgs a) {
  const uint32_t n_tasks = a.ctr->cur_tasks;
  const int lane = threadIdx.x & (WAVE - 1);
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const Task t = a.tasks[ti];
    if (t.n_chunks == 0) continue;
    const uint32_t ncol = t.n_chunks * a.cols;
    const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
    uint32_t* starts = (uint32_t*)(a.tab + t.tab_off + sl.starts);
    if (ncol <= 32) {
      if (blockIdx.y != 0) continue;
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
      continue;
    }
    for (uint32_t b = blockIdx.y * 4 + threadIdx.x / WAVE; b < t.n_buckets; b += gridDim.y * 4) {
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
      if (lane == 0) starts[b] = carry;
    }
  }
}

template <int NBMAX>
__global__ __launch_bounds__(256) void k_bucketscan(LevelArgs a) {
  __shared__ uint32_t s[NBMAX + 1];
  __shared__ uint32_t tmp[5];
  const uint32_t n_tasks = a.ctr->cur_tasks;
  for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const Task t = a.tasks[ti];
    if (t.n_chunks == 0) continue;
    const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
    uint32_t* starts = (uint32_t*)(a.tab + t.tab_off + sl.starts);
    for (uint32_t b = threadIdx.x; b < t.n_buckets; b += 256) s[b] = starts[b];
    __syncthreads();
    const uint32_t total = block_excl_scan_array<256>(s, t.n_buckets, tmp);
    for (uint32_t b = threadIdx.x; b < t.n_buckets; b += 256) starts[b] = s[b];
    if (threadIdx.x == 0) starts[t.n_buckets] = total;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- scatter
// Units (chunks of tasks) with a grid stride; each unit tile by tile:
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
// Keys without values may take RANK_ATOMIC instead: equal keys cannot be told
// apart and every bucket is sorted completely later (or holds one key value),
// so the order inside a bucket cannot show in the result; the counters are
// then one array per tile (two, alternating, each cleared a tile ahead) and
// the LDS left over lets more workgroups share a CU.
// Waves per SIMD the scatter is compiled for (its register budget): four for
// 512- and 1024-thread tiles of at most 64 bytes per thread; six for the
// unordered-rank 512-thread tile of at most 32 bytes per thread, whose LDS
// leaves room for three workgroups per CU.
template <int T, int ITEMS, int KB, int RANK>
constexpr int scatter_min_waves() {
  return (RANK == RANK_ATOMIC && T == 512 && ITEMS * KB <= 32) ? 6
         : ((T == 512 || T == 1024) && ITEMS * KB <= 64)     ? 4
                                                              : 1;
}

template <typename K, typename V, int T, int ITEMS, int NBMAX, int RANK, bool SPLIT = false>
__global__ __launch_bounds__(T, (scatter_min_waves<T, ITEMS, (int)(sizeof(K) * (HasVal<V>::value ? 2 : 1)), RANK>())) void k_scatter(
    LevelArgs a, Bufs<K, V> bf) {
  constexpr int WAVES = T / WAVE;
  constexpr int TILE = T * ITEMS;
  constexpr int PER = (NBMAX + T - 1) / T;  // buckets per thread in the bucket phase
  constexpr bool HV = HasVal<V>::value;
  constexpr bool ATOM = RANK == RANK_ATOMIC;
  constexpr int GM = NBMAX <= NB8 ? 8 : (NBMAX <= NB9 ? 9 : GMAX);  // widest digit of this variant
  using VT = typename std::conditional<HV, V, uint32_t>::type;
  static_assert(!HV || sizeof(V) <= sizeof(K), "values are staged in the key buffer");
  static_assert(!(ATOM && HV), "records with values need the stable ranks");
  __shared__ uint32_t cnt[ATOM ? 2 * NBMAX : WAVES * NBMAX];
  __shared__ unsigned long long mk[(RANK == RANK_BALLOT || ATOM) ? 1 : WAVES * NBMAX];  // zeroed match tables
  __shared__ uint32_t run_off[NBMAX];
  __shared__ uint32_t gdelta[NBMAX];  // bucket's global place minus its tile place (mod 2^32)
  __shared__ uint32_t L[(1 << GM) + 1];
  __shared__ K H[1 << (GM - 1)];
  constexpr bool HASH = GM == 8;  // heavy keys fit the hash table
  static_assert(!HASH || (1 << (GM - 1)) <= HT_MAX_KEYS, "heavy indices fit a byte");
  __shared__ uint32_t HT[HASH ? HT_SLOTS : 1];
  __shared__ uint32_t HC[HASH ? HT_SLOTS : 1];
  __shared__ uint32_t hfull;
  __shared__ K SPL[1 << GM];
  __shared__ K stage[TILE];
  __shared__ uint16_t stage_b[TILE];
  __shared__ uint32_t tmp[WAVES + 1];

  const uint32_t n_units = a.ctr->cur_units;
  const uint32_t chunk = a.ctr->chunk;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t* crow = cnt + wv * NBMAX;
  unsigned long long* wm = mk + (RANK != RANK_BALLOT ? wv * NBMAX : 0);
  if constexpr (ATOM) {
    for (int i = threadIdx.x; i < 2 * NBMAX; i += T) cnt[i] = 0;
  } else if constexpr (RANK != RANK_BALLOT) {
    // the match leaves every entry zero after use: clear once
    for (int i = threadIdx.x; i < WAVES * NBMAX; i += T) mk[i] = 0ull;
  }
  uint32_t tile_no = 0;  // tiles done by this workgroup (selects the counter array)

  for (uint32_t ui = blockIdx.x; ui < n_units; ui += gridDim.x) {
    const uint2 u = a.units[ui];
    const Task t = a.tasks[u.x];
    if (t.n_chunks == 0) continue;
    load_tables<K, T>(t, a.tab, L, H, SPL, HASH ? HT : nullptr, HC, &hfull);
    const SlotLayout sl = slot_layout(t.gamma, (t.flags & TF_LEARNED) != 0);
    const uint32_t* starts = (const uint32_t*)(a.tab + t.tab_off + sl.starts);
    const uint32_t nb = t.n_buckets;
    for (uint32_t b = threadIdx.x; b < nb; b += T)
      run_off[b] = starts[b] + a.cm[t.cm_off + (uint64_t)b * t.n_chunks * a.cols + u.y];
    __syncthreads();

    PlanRegs<K> pr = plan_regs<K>(t);
    pr.hashed = HASH && pr.heavy && hfull == 0u && !(SPLIT && pr.split);
    const K* kin = bf.k[t.src] + t.off;
    K* kout = bf.k[1 - t.src] + t.off;
    const VT* vin = nullptr;
    VT* vout = nullptr;
    if constexpr (HV) {
      vin = bf.v[t.src] + t.off;
      vout = bf.v[1 - t.src] + t.off;
    }
    const int nbits = nb > 1 ? 32 - __builtin_clz(nb - 1) : 1;
    const uint32_t beg = u.y * chunk;
    const uint32_t end = beg + min(chunk, t.size - beg);  // no wrap for sizes near 2^32

    // tile loads through buffer resources over the tile: places past the end
    // read zero and are masked later.  Unordered ranks: a short first tile up
    // to the next 16-byte boundary, then every whole tile is read with 16-byte
    // loads (which key lands in which register does not matter then).
    constexpr int VEC = 16 / (int)sizeof(K);
    static_assert(!ATOM || ITEMS % VEC == 0, "whole 16-byte loads");
    const uint32_t head =
        ATOM ? ((uint32_t)VEC - (uint32_t)(reinterpret_cast<uintptr_t>(kin + beg) & 15u) / (uint32_t)sizeof(K)) %
                   (uint32_t)VEC
             : 0u;
    auto tile_len = [&](uint32_t b0) {
      return (b0 == beg && head) ? min(head, end - b0) : min((uint32_t)TILE, end - b0);
    };
    K nxt[ITEMS];
    VT nxv[ITEMS];
    auto load_tile = [&](uint32_t b0) {
      const uint32_t m = tile_len(b0);
      const __amdgpu_buffer_rsrc_t rk = buf_rsrc(kin + b0, m * (uint32_t)sizeof(K));
      if (ATOM && m == (uint32_t)TILE) {
#pragma unroll
        for (int j = 0; j < ITEMS / VEC; ++j) buf_load16<K>(rk, (uint32_t)(j * T + threadIdx.x) * 16u, nxt + j * VEC);
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) nxt[i] = buf_load<K>(rk, (uint32_t)striped_index<T, ITEMS>(i) * sizeof(K));
      }
      if constexpr (HV) {
        const __amdgpu_buffer_rsrc_t rv = buf_rsrc(vin + b0, m * (uint32_t)sizeof(VT));
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) nxv[i] = buf_load<VT>(rv, (uint32_t)striped_index<T, ITEMS>(i) * sizeof(VT));
      }
    };
    load_tile(beg);
    for (uint32_t base = beg; base < end; base += tile_len(base)) {
      const uint32_t tile_n = tile_len(base);
      K kk[ITEMS];
      VT vv[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        kk[i] = nxt[i];
        if constexpr (HV) vv[i] = nxv[i];
      }
      if (base + tile_n < end) load_tile(base + tile_n);
      uint32_t* tcnt = cnt + (ATOM ? (tile_no & 1u) * NBMAX : 0);  // this tile's counters (ATOM)
      if constexpr (ATOM) {
        // the other array was last read before the previous tile's final barrier
        uint32_t* nxc = cnt + ((tile_no + 1u) & 1u) * NBMAX;
        for (int j = threadIdx.x; j < NBMAX; j += T) nxc[j] = 0;
      } else {
        // each wave clears its own counter row (only that wave ranks with it)
        for (uint32_t j = lane; j < nb; j += WAVE) crow[j] = 0;
      }
      ++tile_no;
      uint32_t bk[ITEMS];
      uint32_t pos[ITEMS];
      if constexpr (RANK == RANK_PIPE) {
        bool vl[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          vl[i] = (uint32_t)striped_index<T, ITEMS>(i) < tile_n;
          bk[i] = vl[i] ? bucket_of<K, SPLIT>(kk[i], pr, L, H, SPL, HT) : 0u;
        }
        rank_pipelined<ITEMS>(bk, vl, wm, crow, pos);
      }
      if constexpr (RANK != RANK_PIPE) {
        // every item's bucket first: independent searches overlap their latency
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
          bk[i] = e < tile_n ? bucket_of<K, SPLIT>(kk[i], pr, L, H, SPL, HT) : 0u;
        }
      }
      if constexpr (ATOM) {
        // bucket (< 2^16) and rank in the tile (< 2^16) share a register:
        // the 1024 x 16 tile is at the register limit
        static_assert(TILE <= 65536 && NBMAX <= 65536, "bucket and rank fit 16 bits each");
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
          bk[i] = (uint32_t)striped_index<T, ITEMS>(i) < tile_n ? (bk[i] << 16) | atomicAdd(&tcnt[bk[i]], 1u) : 0u;
      }
#pragma unroll
      for (int i = 0; i < ((RANK == RANK_PIPE || ATOM) ? 0 : ITEMS); ++i) {
        const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
        const bool valid = e < tile_n;
        const uint32_t b = bk[i];
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
      (void)nbits;
      __syncthreads();
      if constexpr (ATOM && NBMAX <= NB8) {
        // one wave scans the tile's bucket counts (no block-wide scan and its
        // barriers): lane l takes buckets [l * PB, l * PB + PB)
        constexpr int PB = (NBMAX + WAVE - 1) / WAVE;
        if (wv == 0) {
          uint32_t c[PB];
          uint32_t S = 0;
#pragma unroll
          for (int j = 0; j < PB; ++j) {
            const uint32_t b = lane * PB + j;
            c[j] = b < nb ? tcnt[b] : 0u;
            S += c[j];
          }
          uint32_t x = S;
#pragma unroll
          for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, WAVE);
            if (lane >= o) x += y;
          }
          uint32_t run = x - S;
#pragma unroll
          for (int j = 0; j < PB; ++j) {
            const uint32_t b = lane * PB + j;
            if (b < nb) {
              gdelta[b] = run_off[b] - run;
              run_off[b] += c[j];
              tcnt[b] = run;  // the bucket's first place in the tile
            }
            run += c[j];
          }
        }
      } else {
        // buckets [b0, b0 + PER) of this thread: totals, tile starts, wave bases
        const uint32_t b0 = threadIdx.x * PER;
        uint32_t sb[PER];
        uint32_t S = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const uint32_t b = b0 + j;
          uint32_t x = 0;
          if (b < nb) {
            if constexpr (ATOM) {
              x = tcnt[b];
            } else {
#pragma unroll
              for (int w = 0; w < WAVES; ++w) x += cnt[w * NBMAX + b];
            }
          }
          sb[j] = x;
          S += x;
        }
        uint32_t total;
        uint32_t run = block_excl_scan<T, false>(S, tmp, &total);  // a barrier follows before tmp is reused
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const uint32_t b = b0 + j;
          if (b < nb) {
            gdelta[b] = run_off[b] - run;
            run_off[b] += sb[j];
            if constexpr (ATOM) {
              tcnt[b] = run;  // the bucket's first place in the tile
            } else {
              uint32_t r2 = run;
#pragma unroll
              for (int w = 0; w < WAVES; ++w) {
                const uint32_t c = cnt[w * NBMAX + b];
                cnt[w * NBMAX + b] = r2;
                r2 += c;
              }
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
          if constexpr (ATOM) {
            const uint32_t b = bk[i] >> 16;
            const uint32_t p = (bk[i] & 0xFFFFu) + tcnt[b];
            stage[p] = kk[i];
            stage_b[p] = (uint16_t)b;
          } else {
            const uint32_t p = pos[i] + crow[bk[i]];
            pos[i] = p;
            stage[p] = kk[i];
            stage_b[p] = (uint16_t)bk[i];
          }
        }
      }
      __syncthreads();
      uint32_t gps[HV ? ITEMS : 1];
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const uint32_t j = threadIdx.x + it * T;
        uint32_t gp = 0xFFFFFFFFu;
        if (j < tile_n) {
          // unsigned: the bucket's run starts at or after the keys of earlier
          // buckets, so the sum is the place in [0, t.size) for any size < 2^32
          gp = gdelta[stage_b[j]] + j;
          if (gp < t.size)
            kout[gp] = stage[j];
          else
            atomicOr(&a.ctr->error, ERR_SCATTER);
        }
        if constexpr (HV) gps[it] = gp;
      }
      if constexpr (HV) {
        VT* vstage = reinterpret_cast<VT*>(stage);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t e = (uint32_t)striped_index<T, ITEMS>(i);
          if (e < tile_n) vstage[pos[i]] = vv[i];
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const uint32_t j = threadIdx.x + it * T;
          if (j < tile_n && gps[it] < t.size) vout[gps[it]] = vstage[j];
        }
      }
      // the next tile stages into the same buffer.  Unordered ranks need no
      // barrier here: the next tile's first LDS writes go to the other counter
      // array, and it writes gdelta and the stage only after its barriers that
      // every thread reaches once done with this tile's write-out
      if constexpr (!ATOM) __syncthreads();
    }
  }
}

template <typename K, typename V, int NBMAX, int T, int RANK, int SITEMS_REQ = 0, bool SPLIT = false>
static void launch_dist_variant(const LevelArgs& a, Bufs<K, V> b, uint32_t max_chunks, hipStream_t s, int phase) {
  constexpr int HITEMS = sizeof(K) == 4 ? 16 : 8;
  constexpr int HT = T > 512 ? 512 : T;  // the histogram of 1024-thread tiles runs faster at 512
  constexpr int SITEMS = SITEMS_REQ ? SITEMS_REQ : (sizeof(K) == 4 ? 16 : 8);
  const uint32_t nu = a.grid_units;
  const uint32_t nt = a.grid_tasks;
  if (phase < 0 || phase == 0)
    hipLaunchKernelGGL((k_hist<K, HT, HITEMS, NBMAX, SPLIT>), dim3(nu), dim3(HT), 0, s, a, (const K*)b.k[0],
                       (const K*)b.k[1]);
  if (phase < 0 || phase == 1) {
    // bucket groups along y: all of them when the host knows the chunk
    // count, a fixed spread for the graph form (max_chunks unknown)
    const uint32_t gy = max_chunks * a.cols <= 32 ? 1u : (max_chunks == 0x7FFFFFFFu ? 8u : (NBMAX + 3) / 4);
    hipLaunchKernelGGL(k_colscan, dim3(nt, gy), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_bucketscan<NBMAX>), dim3(nt), dim3(256), 0, s, a);
  }
  if (phase < 0 || phase == 2)
    hipLaunchKernelGGL((k_scatter<K, V, T, SITEMS, NBMAX, RANK, SPLIT>), dim3(nu), dim3(T), 0, s, a, b);
}

uint32_t dist_cols(int) { return 1; }

// The tile shapes of the <= 8-bit variants (LevelArgs::tile).
template <typename K, typename V, int RANK>
static void launch_tiles(const LevelArgs& a, Bufs<K, V> b, uint32_t max_chunks, hipStream_t s, int phase) {
  if (a.tile == 1)
    launch_dist_variant<K, V, NB8, 256, RANK>(a, b, max_chunks, s, phase);
  else if (a.tile == 2)
    launch_dist_variant<K, V, NB8, 512, RANK, sizeof(K) == 4 ? 8 : 4>(a, b, max_chunks, s, phase);
  else if (a.tile == 3)
    launch_dist_variant<K, V, NB8, 256, RANK, sizeof(K) == 4 ? 32 : 16>(a, b, max_chunks, s, phase);
  else if (a.tile == 4)
    launch_dist_variant<K, V, NB8, 1024, RANK, sizeof(K) == 4 ? 8 : 4>(a, b, max_chunks, s, phase);
  else if (a.tile == 5)  // 16 bare 32-bit keys a thread with unordered ranks (the stable ranks' tables would not fit)
    launch_dist_variant<K, V, NB8, 1024, RANK, (sizeof(K) == 4 && RANK == RANK_ATOMIC) ? 16 : (sizeof(K) == 4 ? 8 : 4)>(
        a, b, max_chunks, s, phase);
  else
    launch_dist_variant<K, V, NB8, 512, RANK>(a, b, max_chunks, s, phase);
}

// Tile shapes of the scatter for digit widths <= 8 (LevelArgs::tile):
// 0 = 512 threads x 16 keys (x 8 for 64-bit keys), 1 = 256 x 16, 2 = 512 x 8,
// 3 = 256 x 32 (x 16), 4 = 1024 x 8 (x 4), 5 = 1024 x 16 for bare 32-bit keys
// with unordered ranks (else as 4).  9-bit digits of bare keys use 1024 x 16
// (x 8) tiles and 776 counters; other wider digits 256 threads and 2048
// counters.
template <typename K, typename V>
void launch_distribute(const LevelArgs& a, Bufs<K, V> b, int g_level_max, uint32_t max_chunks, hipStream_t s,
                       int phase) {
  // keys without values: unordered ranks unless ordered ones are asked for
  // (or a mode is forced); records with values: never unordered
  int rm = rank_mode();
  if (HasVal<V>::value || a.ordered) {
    if (rm == RANK_ATOMIC) rm = RANK_LDS;
  } else if (!rank_mode_forced()) {
    rm = RANK_ATOMIC;
  }
  if (a.merge_variant == MV_SPLIT) {
    // the split layout: one tile shape per digit class, LDS-match or atomic ranks
    constexpr int UR = HasVal<V>::value ? RANK_LDS : RANK_ATOMIC;
    const bool unordered = !HasVal<V>::value && !a.ordered;
    if (g_level_max <= 8) {
      if (unordered)
        launch_dist_variant<K, V, NB8, 512, UR, 0, true>(a, b, max_chunks, s, phase);
      else
        launch_dist_variant<K, V, NB8, 512, RANK_LDS, 0, true>(a, b, max_chunks, s, phase);
    } else if (g_level_max == 9 && unordered) {
      if constexpr (!HasVal<V>::value)
        launch_dist_variant<K, V, NB9, 1024, RANK_ATOMIC, sizeof(K) == 4 ? 16 : 8, true>(a, b, max_chunks, s, phase);
    } else {
      if (unordered)
        launch_dist_variant<K, V, 2048, 256, UR, 0, true>(a, b, max_chunks, s, phase);
      else
        launch_dist_variant<K, V, 2048, 256, RANK_LDS, 0, true>(a, b, max_chunks, s, phase);
    }
    return;
  }
  if (g_level_max <= 8) {
    if (rm == RANK_BALLOT)
      launch_dist_variant<K, V, NB8, 512, RANK_BALLOT>(a, b, max_chunks, s, phase);
    else if (rm == RANK_HYBRID)
      launch_dist_variant<K, V, NB8, 512, RANK_HYBRID>(a, b, max_chunks, s, phase);
    else if (rm == RANK_PIPE)
      launch_dist_variant<K, V, NB8, 512, RANK_PIPE>(a, b, max_chunks, s, phase);
    else if (rm == RANK_ATOMIC)
      launch_tiles<K, V, HasVal<V>::value ? RANK_LDS : RANK_ATOMIC>(a, b, max_chunks, s, phase);
    else
      launch_tiles<K, V, RANK_LDS>(a, b, max_chunks, s, phase);
  } else if (g_level_max == 9 && rm == RANK_ATOMIC && !HasVal<V>::value) {
    // 9-bit digits of bare keys: 1024-thread tiles, so that a tile still
    // writes runs of several keys into each of its up to 769 buckets
    if constexpr (!HasVal<V>::value)
      launch_dist_variant<K, V, NB9, 1024, RANK_ATOMIC, sizeof(K) == 4 ? 16 : 8>(a, b, max_chunks, s, phase);
  } else {
    if (rm == RANK_BALLOT)
      launch_dist_variant<K, V, 2048, 256, RANK_BALLOT>(a, b, max_chunks, s, phase);
    else if (rm == RANK_PIPE)
      launch_dist_variant<K, V, 2048, 256, RANK_PIPE>(a, b, max_chunks, s, phase);
    else if (rm == RANK_ATOMIC)
      launch_dist_variant<K, V, 2048, 256, HasVal<V>::value ? RANK_LDS : RANK_ATOMIC>(a, b, max_chunks, s, phase);
    else
      launch_dist_variant<K, V, 2048, 256, RANK_LDS>(a, b, max_chunks, s, phase);
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

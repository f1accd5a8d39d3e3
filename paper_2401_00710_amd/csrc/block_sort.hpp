// Stable LSD radix sort of up to THREADS*ITEMS keys held in registers, using
// LDS for the exchange.  Used for the sample sort of the sampling step
// (Section 3.1) and for the base-case sort of small subproblems (Section 3.5),
// which must be stable for the whole method to be stable.
//
// Layout: thread (wave w, lane l) holds items i = 0..ITEMS-1 at element index
// w*64*ITEMS + i*64 + l ("wave-striped": every item load of a wave is one
// contiguous 64-element row).  Each 8-bit pass ranks keys with a wave-wide
// ballot match (peers with the same digit, counted below the lane), keeps a
// running count per (wave, digit) in LDS, and turns the counts into offsets by
// an exclusive scan in (digit, wave) order.  Processing items in order i and
// lanes in order l visits elements in index order, so equal digits keep their
// order: the pass is stable.
#pragma once
#include "common.hpp"

namespace dts {

// A "block" of THREADS = 64 is one wave of a possibly larger workgroup (the
// waves of such a workgroup sort independently): its thread index is the
// lane and it synchronises with a wave barrier; larger blocks are the whole
// workgroup.
template <int THREADS>
__device__ inline int btid() {
  return THREADS == WAVE ? (int)(threadIdx.x & (WAVE - 1)) : (int)threadIdx.x;
}

template <int THREADS>
__device__ inline void bsync() {
  if constexpr (THREADS == WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int THREADS, int ITEMS>
__device__ inline int striped_index(int i) {
  const int t = btid<THREADS>();
  return (t / WAVE) * WAVE * ITEMS + i * WAVE + (t & (WAVE - 1));
}

// LDS words (u32) needed for the counters of block_radix_sort.
template <int THREADS>
constexpr int bsort_cnt_words() {
  return (THREADS / WAVE) * 256 + THREADS / WAVE + 1;
}
// LDS u64 words needed for the match tables of block_radix_sort with RANK_LDS.
template <int THREADS>
constexpr int bsort_match_words() {
  return (THREADS / WAVE) * 256;
}

// Sorts the first n of the THREADS*ITEMS keys held in k[] (and carries ix[]
// when IDX) by key bits [lo_bit, hi_bit); elements at index >= n are ignored
// (item rows wholly beyond n are skipped).  sk: LDS array of THREADS*ITEMS
// keys; si: LDS array of THREADS*ITEMS u16 (only when IDX); cnt:
// bsort_cnt_words<THREADS>() u32.  RANK_LDS needs `mk`
// (bsort_match_words<THREADS>() zeroed u64).  On return k[]/ix[] hold the
// sorted sequence in the striped layout and sk (si) holds it in order.
// first_unordered (keys without indices only): the first pass ranks keys with
// one LDS atomic each, in no particular order among equal digits.  That is
// enough for a sort of bare keys whose input order does not matter: only the
// passes after the first must keep the order of equal digits.
template <typename K, int THREADS, int ITEMS, bool IDX, int RANK = RANK_BALLOT>
__device__ void block_radix_sort(K (&k)[ITEMS], uint16_t (&ix)[ITEMS], int lo_bit, int hi_bit, K* sk,
                                 uint16_t* si, uint32_t* cnt, unsigned long long* mk = nullptr,
                                 int n = THREADS * ITEMS, bool first_unordered = false) {
  constexpr int WAVES = THREADS / WAVE;
  constexpr int DPT = (256 + THREADS - 1) / THREADS;  // digits per thread in the scan
  const int wv = btid<THREADS>() / WAVE;
  const int lane = btid<THREADS>() & (WAVE - 1);
  uint32_t* tmp = cnt + WAVES * 256;
  unsigned long long* wm = mk + (RANK != RANK_BALLOT ? wv * 256 : 0);
  const int row0 = wv * WAVE * ITEMS;  // first element of this wave
  // the counters start at zero; every pass zeroes them again after its last read
  for (int i = btid<THREADS>(); i < WAVES * 256; i += THREADS) cnt[i] = 0;
  bsync<THREADS>();
  for (int bit = lo_bit; bit < hi_bit; bit += 8) {
    const int nbits = min(8, hi_bit - bit);
    const uint32_t dmask = (1u << nbits) - 1u;
    uint32_t* wc = cnt + wv * 256;
    uint32_t pos[ITEMS];
    const bool unord = !IDX && first_unordered && bit == lo_bit;
    if (unord) {
      // one counter per digit for the whole block; a key's place among its
      // digit's keys is an atomic increment
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const bool valid = row0 + i * WAVE + lane < n;
        pos[i] = valid ? atomicAdd(&cnt[(uint32_t)(shr<K>(k[i], bit)) & dmask], 1u) : 0u;
      }
    } else if constexpr (RANK == RANK_PIPE) {
      uint32_t dg[ITEMS];
      bool vl[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        vl[i] = row0 + i * WAVE + lane < n;
        dg[i] = (uint32_t)(shr<K>(k[i], bit)) & dmask;
      }
      rank_pipelined<ITEMS>(dg, vl, wm, wc, pos);
    }
#pragma unroll
    for (int i = 0; i < (RANK == RANK_PIPE ? 0 : ITEMS); ++i) {
      if (unord) break;
      pos[i] = 0;
      if (row0 + i * WAVE >= n) continue;  // whole row is padding (uniform per wave)
      const bool valid = row0 + i * WAVE + lane < n;
      const uint32_t d = (uint32_t)(shr<K>(k[i], bit)) & dmask;
      uint64_t peers;
      if constexpr (RANK == RANK_LDS) {
        peers = lds_match(wm, d, valid);
      } else if constexpr (RANK == RANK_HYBRID) {
        peers = hybrid_match(wm, d, nbits, valid);
      } else {
        peers = match_peers(d, nbits, valid);
      }
      const uint32_t r = mbcnt(peers);
      const uint32_t c = (uint32_t)__popcll(peers);
      if (valid) {
        const uint32_t base = wc[d];
        pos[i] = base + r;
        if (r == 0) wc[d] = base + c;
      }
    }
    bsync<THREADS>();
    // exclusive offsets in (digit, wave) order; thread t owns digits [t*DPT, t*DPT+DPT)
    // (unordered pass: one count per digit, in cnt[0..255])
    const int nw = unord ? 1 : WAVES;
    uint32_t sd[DPT];
    uint32_t S = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = btid<THREADS>() * DPT + j;
      uint32_t x = 0;
      if (d < 256) {
        for (int w = 0; w < nw; ++w) x += cnt[w * 256 + d];
      }
      sd[j] = x;
      S += x;
    }
    uint32_t total;
    uint32_t run = block_excl_scan<THREADS, false>(S, tmp, &total);  // a barrier follows before tmp is reused
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = btid<THREADS>() * DPT + j;
      if (d < 256) {
        uint32_t r2 = run;
        for (int w = 0; w < nw; ++w) {
          const uint32_t c = cnt[w * 256 + d];
          cnt[w * 256 + d] = r2;
          r2 += c;
        }
      }
      run += sd[j];
    }
    bsync<THREADS>();
    const uint32_t* dc = unord ? cnt : wc;  // digit bases of this key's counter row
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      if (row0 + i * WAVE + lane < n) {
        const uint32_t d = (uint32_t)(shr<K>(k[i], bit)) & dmask;
        const uint32_t p = pos[i] + dc[d];
        sk[p] = k[i];
        if constexpr (IDX) si[p] = ix[i];
      }
    }
    bsync<THREADS>();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<THREADS, ITEMS>(i);
      if (e < n) {
        k[i] = sk[e];
        if constexpr (IDX) ix[i] = si[e];
      }
    }
    for (int i = btid<THREADS>(); i < WAVES * 256; i += THREADS) cnt[i] = 0;
    bsync<THREADS>();
  }
}

// Stable sort by key bits [lo_bit, hi_bit) for wide bit ranges (more than
// PREFIX_BITS + 8 bits): radix passes over the top PREFIX_BITS bits only,
// then every run of equal prefix that
// holds a descent is finished by a stable insertion sort (one thread per
// run).  Keys whose prefixes are nearly unique need two passes instead of one
// per 8 bits; runs of equal keys hold no descent.  If a run with a descent
// is longer than FIX_MAX, the remaining passes run instead (low bits, then
// the prefix again: a plain LSD sort, stable for the original order).  Same
// arguments and results as block_radix_sort; `flag` is one LDS word, and cnt
// doubles as the bitmap of runs to fix.
constexpr int PREFIX_BITS = 16;
constexpr int FIX_MAX = 32;

template <typename K, int THREADS, int ITEMS, bool IDX, int RANK = RANK_BALLOT>
__device__ void block_sort_bits(K (&k)[ITEMS], uint16_t (&ix)[ITEMS], int lo_bit, int hi_bit, K* sk, uint16_t* si,
                                uint32_t* cnt, unsigned long long* mk, int n, uint32_t* flag) {
  static_assert(THREADS * ITEMS / 32 <= bsort_cnt_words<THREADS>(), "run bitmap must fit in the counters");
  if (hi_bit - lo_bit <= PREFIX_BITS + 8) {
    // at most three passes: the prefix path would save at most one
    block_radix_sort<K, THREADS, ITEMS, IDX, RANK>(k, ix, lo_bit, hi_bit, sk, si, cnt, mk, n, !IDX);
    return;
  }
  const int pb = hi_bit - PREFIX_BITS;
  // rounds of radix passes (one call site for all of them):
  // 0: [pb, hi); if the fix-up gives way, 1: [lo, pb) and 2: [pb, hi)
  int r_lo = pb, r_hi = hi_bit;
  for (int round = 0;; ++round) {
    // rounds 0 and 1 start from an order that does not matter; round 2 must
    // keep round 1's order of equal prefixes
    block_radix_sort<K, THREADS, ITEMS, IDX, RANK>(k, ix, r_lo, r_hi, sk, si, cnt, mk, n, !IDX && round != 2);
    if (round != 0) {
      if (round == 1) {
        r_lo = pb;
        r_hi = hi_bit;
        continue;
      }
      return;
    }
    // sk (si) now hold the records in prefix order
    const int t = btid<THREADS>();
    uint32_t* bm = cnt;  // bit s: the run starting at s holds a descent
    for (int w = t; w < (n + 31) / 32; w += THREADS) bm[w] = 0u;
    if (t == 0) *flag = 0;
    bsync<THREADS>();
    auto pre = [&](K x) { return shr<K>(x, pb); };
    for (int p = t + 1; p < n; p += THREADS) {
      const K pr = pre(sk[p]);
      if (pre(sk[p - 1]) != pr || !(sk[p - 1] > sk[p])) continue;  // no descent at p
      int s0 = p - 1;
      while (s0 > 0 && pre(sk[s0 - 1]) == pr && p - s0 < FIX_MAX) --s0;
      int e = p + 1;
      while (e < n && pre(sk[e]) == pr && e - s0 < FIX_MAX) ++e;
      if ((s0 > 0 && pre(sk[s0 - 1]) == pr) || (e < n && pre(sk[e]) == pr)) {
        atomicOr(flag, 1u);  // a run longer than FIX_MAX with a descent
      } else {
        atomicOr(&bm[s0 >> 5], 1u << (s0 & 31));
      }
    }
    bsync<THREADS>();
    if (*flag) {
      r_lo = lo_bit;
      r_hi = pb;
      continue;
    }
    for (int p = t; p < n; p += THREADS) {
      if (!((bm[p >> 5] >> (p & 31)) & 1u)) continue;
      const K pr = pre(sk[p]);
      int e = p + 1;
      while (e < n && pre(sk[e]) == pr) ++e;  // at most FIX_MAX
      // stable insertion sort of sk[p, e) (with si)
      for (int j = p + 1; j < e; ++j) {
        const K x = sk[j];
        uint16_t xi = 0;
        if constexpr (IDX) xi = si[j];
        int i = j - 1;
        while (i >= p && sk[i] > x) {
          sk[i + 1] = sk[i];
          if constexpr (IDX) si[i + 1] = si[i];
          --i;
        }
        sk[i + 1] = x;
        if constexpr (IDX) si[i + 1] = xi;
      }
    }
    bsync<THREADS>();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = striped_index<THREADS, ITEMS>(i);
      if (e < n) {
        k[i] = sk[e];
        if constexpr (IDX) ix[i] = si[e];
      }
    }
    bsync<THREADS>();
    return;
  }
}

// Bitwise OR and AND of the first n elements held in k[] (striped layout),
// reduced over the workgroup.  red: LDS of 2*(THREADS/64) K.
template <typename K, int THREADS, int ITEMS>
__device__ inline void block_or_and(const K (&k)[ITEMS], int n, K* red, K* out_or, K* out_and) {
  constexpr int WAVES = THREADS / WAVE;
  K o = 0, a = ~(K)0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (striped_index<THREADS, ITEMS>(i) < n) {
      o |= k[i];
      a &= k[i];
    }
  }
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    o |= __shfl_xor(o, off, WAVE);
    a &= __shfl_xor(a, off, WAVE);
  }
  const int lane = btid<THREADS>() & (WAVE - 1), wv = btid<THREADS>() / WAVE;
  if (lane == 0) {
    red[wv] = o;
    red[WAVES + wv] = a;
  }
  bsync<THREADS>();
  K ro = 0, ra = ~(K)0;
  for (int w = 0; w < WAVES; ++w) {
    ro |= red[w];
    ra &= red[WAVES + w];
  }
  *out_or = ro;
  *out_and = ra;
  bsync<THREADS>();
}

template <typename K>
__device__ inline int bit_length(K x) {
  if constexpr (sizeof(K) == 8) {
    return x ? 64 - __builtin_clzll((unsigned long long)x) : 0;
  } else {
    return x ? 32 - __builtin_clz((unsigned)x) : 0;
  }
}

template <typename K>
__device__ inline int trailing_zeros(K x) {
  if constexpr (sizeof(K) == 8) {
    return x ? __builtin_ctzll((unsigned long long)x) : 64;
  } else {
    return x ? __builtin_ctz((unsigned)x) : 32;
  }
}

}  // namespace dts

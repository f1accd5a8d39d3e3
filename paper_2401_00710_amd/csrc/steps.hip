// Step entry points of dtsort.h: single steps of the method on one
// subproblem, for step-level checks against a CPU model.  They reuse the
// production kernels with a one-task level.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/dtsort.h"
#include "launch.hpp"

namespace dts {

namespace {
thread_local std::string s_err;

struct Tmp {
  std::vector<void*> ptrs;
  ~Tmp() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* get(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 64) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

#define SCHK(x)                                      \
  do {                                               \
    if ((x) != hipSuccess) return DTSORT_EHIP;       \
  } while (0)

template <typename K, typename V>
int plan_and_distribute(const K* keys, const V* vals, size_t n, int hi, int skip, const dtsort_opts* opts,
                        K* out_k, V* out_v, uint32_t* counts, int32_t* plan, K* heavy, uint32_t* light_id,
                        bool distribute, hipStream_t s) {
  constexpr bool HV = HasVal<V>::value;
  if (n < 2 || n >= (1ull << 32) || !keys || hi < 1 || hi > (int)(8 * sizeof(K))) return DTSORT_EINVAL;
  dtsort_opts o;
  dtsort_default_opts(&o);
  if (opts) o = *opts;
  Tmp tmp;
  const int g = plan_gamma((uint32_t)n, o.digit_bits);
  const SlotLayout sl = slot_layout(g, false);
  const uint64_t chunk = 8192;
  const uint64_t units = n / chunk + 2;
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.seed = o.seed;
  a.g_override = o.digit_bits;
  a.cutoff = 16384;
  a.plain = o.mode == DTSORT_MODE_PLAIN;
  a.ordered = o.ordered_ranks != 0;
  a.key_bits = 8 * sizeof(K);
  a.n_tasks = 1;
  a.chunk = (uint32_t)chunk;
  a.slot_bytes = sl.bytes;
  a.cols = dist_cols(g);
  a.caps.units = (uint32_t)units;
  a.caps.cm = units * a.cols * nb_cap(g);
  a.caps.tab = sl.bytes;
  a.tasks = (Task*)tmp.get(sizeof(Task));
  a.units = (uint2*)tmp.get(sizeof(uint2) * units);
  a.tab = (uint8_t*)tmp.get(sl.bytes);
  a.cm = (uint32_t*)tmp.get(4 * a.caps.cm);
  LevelCounters* ctr2 = (LevelCounters*)tmp.get(2 * sizeof(LevelCounters));
  if (!a.tasks || !a.units || !a.tab || !a.cm || !ctr2) return DTSORT_ENOMEM;
  a.in = ctr2;
  a.ctr = ctr2 + 1;
  a.grid_tasks = 1;
  a.grid_units = (uint32_t)units;
  LevelCounters root;
  std::memset(&root, 0, sizeof(root));
  root.next_tasks = 1;
  root.next_records = (uint32_t)n;
  root.next_max_size = (uint32_t)n;
  SCHK(hipMemcpyAsync(ctr2, &root, sizeof(root), hipMemcpyHostToDevice, s));
  SCHK(hipMemsetAsync(a.tab, 0, sl.bytes, s));
  Task t;
  std::memset(&t, 0, sizeof(t));
  t.size = (uint32_t)n;
  t.n_root = (uint32_t)n;
  t.hi = (uint8_t)hi;
  t.flags = skip ? TF_SKIP_DISABLED : 0;
  t.gamma = (uint8_t)g;
  SCHK(hipMemcpyAsync(a.tasks, &t, sizeof(Task), hipMemcpyHostToDevice, s));
  launch_prep(a, s);
  launch_plan<K>(a, keys, keys, g, s);
  if (distribute) {
    Bufs<K, V> b;
    b.k[0] = const_cast<K*>(keys);
    b.k[1] = out_k;
    if constexpr (HV) {
      b.v[0] = const_cast<V*>(vals);
      b.v[1] = out_v;
    }
    launch_distribute<K, V>(a, b, g, (uint32_t)units, s);
  }
  SCHK(hipGetLastError());
  SCHK(hipMemcpyAsync(&t, a.tasks, sizeof(Task), hipMemcpyDeviceToHost, s));
  std::vector<uint8_t> slot(sl.bytes);
  SCHK(hipMemcpyAsync(slot.data(), a.tab, sl.bytes, hipMemcpyDeviceToHost, s));
  LevelCounters hc;
  SCHK(hipMemcpyAsync(&hc, a.ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
  SCHK(hipStreamSynchronize(s));
  if (hc.error) return DTSORT_EINTERNAL;
  if (plan) {
    plan[0] = t.gamma;
    plan[1] = t.w;
    plan[2] = t.shift;
    plan[3] = t.top;
    plan[4] = t.n_heavy;
    plan[5] = t.n_buckets;
  }
  const uint64_t* H = (const uint64_t*)(slot.data() + sl.heavy);
  const uint32_t* L = (const uint32_t*)(slot.data() + sl.light);
  const uint32_t* st = (const uint32_t*)(slot.data() + sl.starts);
  if (heavy)
    for (uint32_t i = 0; i < t.n_heavy; ++i) heavy[i] = (K)H[i];
  if (light_id)
    for (uint32_t z = 0; z <= (1u << t.w); ++z) light_id[z] = L[z];
  if (counts && distribute)
    for (uint32_t b = 0; b < t.n_buckets; ++b) counts[b] = st[b + 1] - st[b];
  return DTSORT_OK;
}

template <typename K, typename V>
int leaf_step(const K* keys, const V* vals, const uint64_t* seg, size_t n_seg, int bits, K* out_k, V* out_v,
              hipStream_t s) {
  constexpr bool HV = HasVal<V>::value;
  if (n_seg == 0) return DTSORT_OK;
  std::vector<uint64_t> off(n_seg + 1);
  SCHK(hipMemcpyAsync(off.data(), seg, 8 * (n_seg + 1), hipMemcpyDeviceToHost, s));
  SCHK(hipStreamSynchronize(s));
  std::vector<Leaf> cls[LEAF_CLASSES];
  for (size_t i = 0; i < n_seg; ++i) {
    const uint64_t b = off[i], e = off[i + 1];
    if (e < b || e - b > leaf_cap<K, V>(LEAF_CLASSES - 1)) return DTSORT_EINVAL;
    if (e == b) continue;
    Leaf l;
    l.off = b;
    l.size = (uint32_t)(e - b);
    l.bits = (uint8_t)bits;
    l.from = 0;
    l.to = 1;
    l.pad = 0;
    int c = LEAF_CLASSES - 1;
    for (int k = LEAF_CLASSES - 2; k >= 0; --k)
      if (l.size <= leaf_cap<K, V>(k)) c = k;
    cls[c].push_back(l);
  }
  Tmp tmp;
  Bufs<K, V> b;
  b.k[0] = const_cast<K*>(keys);
  b.k[1] = out_k;
  if constexpr (HV) {
    b.v[0] = const_cast<V*>(vals);
    b.v[1] = out_v;
  }
  uint32_t hcount[LEAF_CLASSES];
  for (int c = 0; c < LEAF_CLASSES; ++c) hcount[c] = (uint32_t)cls[c].size();
  uint32_t* dcount = (uint32_t*)tmp.get(sizeof(hcount));
  if (!dcount) return DTSORT_ENOMEM;
  SCHK(hipMemcpyAsync(dcount, hcount, sizeof(hcount), hipMemcpyHostToDevice, s));
  for (int c = 0; c < LEAF_CLASSES; ++c) {
    if (cls[c].empty()) continue;
    Leaf* d = (Leaf*)tmp.get(sizeof(Leaf) * cls[c].size());
    if (!d) return DTSORT_ENOMEM;
    SCHK(hipMemcpyAsync(d, cls[c].data(), sizeof(Leaf) * cls[c].size(), hipMemcpyHostToDevice, s));
    launch_leaf<K, V>(d, dcount + c, hcount[c], hcount[c], c, b, s);
  }
  SCHK(hipGetLastError());
  SCHK(hipStreamSynchronize(s));
  return DTSORT_OK;
}

}  // namespace
}  // namespace dts

using namespace dts;

extern "C" {

int dtsort_step_plan_u32(const uint32_t* keys, size_t n, int hi, int skip_disabled, const dtsort_opts* opts,
                         int32_t* plan, uint32_t* heavy, uint32_t* light_id, void* stream) {
  return plan_and_distribute<uint32_t, NoVal>(keys, nullptr, n, hi, skip_disabled, opts, nullptr, nullptr, nullptr,
                                              plan, heavy, light_id, false, (hipStream_t)stream);
}

int dtsort_step_plan_u64(const uint64_t* keys, size_t n, int hi, int skip_disabled, const dtsort_opts* opts,
                         int32_t* plan, uint64_t* heavy, uint32_t* light_id, void* stream) {
  return plan_and_distribute<uint64_t, NoVal>(keys, nullptr, n, hi, skip_disabled, opts, nullptr, nullptr, nullptr,
                                              plan, heavy, light_id, false, (hipStream_t)stream);
}

int dtsort_step_distribute_u32(const uint32_t* keys, const uint32_t* values, size_t n, int hi,
                               const dtsort_opts* opts, uint32_t* out_keys, uint32_t* out_values, uint32_t* counts,
                               int32_t* plan, uint32_t* heavy, uint32_t* light_id, void* stream) {
  if (!out_keys) return DTSORT_EINVAL;
  if (values) {
    if (!out_values) return DTSORT_EINVAL;
    return plan_and_distribute<uint32_t, uint32_t>(keys, values, n, hi, 0, opts, out_keys, out_values, counts, plan,
                                                   heavy, light_id, true, (hipStream_t)stream);
  }
  return plan_and_distribute<uint32_t, NoVal>(keys, nullptr, n, hi, 0, opts, out_keys, nullptr, counts, plan, heavy,
                                              light_id, true, (hipStream_t)stream);
}

int dtsort_step_distribute_u64(const uint64_t* keys, const uint64_t* values, size_t n, int hi,
                               const dtsort_opts* opts, uint64_t* out_keys, uint64_t* out_values, uint32_t* counts,
                               int32_t* plan, uint64_t* heavy, uint32_t* light_id, void* stream) {
  if (!out_keys) return DTSORT_EINVAL;
  if (values) {
    if (!out_values) return DTSORT_EINVAL;
    return plan_and_distribute<uint64_t, uint64_t>(keys, values, n, hi, 0, opts, out_keys, out_values, counts, plan,
                                                   heavy, light_id, true, (hipStream_t)stream);
  }
  return plan_and_distribute<uint64_t, NoVal>(keys, nullptr, n, hi, 0, opts, out_keys, nullptr, counts, plan, heavy,
                                              light_id, true, (hipStream_t)stream);
}

int dtsort_step_leaf_u32(const uint32_t* keys, const uint32_t* values, const uint64_t* seg_offsets,
                         size_t n_segments, int bits, uint32_t* out_keys, uint32_t* out_values, void* stream) {
  if (!keys || !seg_offsets || !out_keys || bits < 0 || bits > 32) return DTSORT_EINVAL;
  if (values) {
    if (!out_values) return DTSORT_EINVAL;
    return leaf_step<uint32_t, uint32_t>(keys, values, seg_offsets, n_segments, bits, out_keys, out_values,
                                         (hipStream_t)stream);
  }
  return leaf_step<uint32_t, NoVal>(keys, nullptr, seg_offsets, n_segments, bits, out_keys, nullptr,
                                    (hipStream_t)stream);
}

int dtsort_step_leaf_u64(const uint64_t* keys, const uint64_t* values, const uint64_t* seg_offsets,
                         size_t n_segments, int bits, uint64_t* out_keys, uint64_t* out_values, void* stream) {
  if (!keys || !seg_offsets || !out_keys || bits < 0 || bits > 64) return DTSORT_EINVAL;
  if (values) {
    if (!out_values) return DTSORT_EINVAL;
    return leaf_step<uint64_t, uint64_t>(keys, values, seg_offsets, n_segments, bits, out_keys, out_values,
                                         (hipStream_t)stream);
  }
  return leaf_step<uint64_t, NoVal>(keys, nullptr, seg_offsets, n_segments, bits, out_keys, nullptr,
                                    (hipStream_t)stream);
}

int dtsort_step_dtmerge_u64(const uint64_t* b0_keys, const uint64_t* b0_values, size_t b0,
                            const uint64_t* heavy_keys, const uint32_t* heavy_sizes, size_t m,
                            const uint64_t* heavy_values, uint64_t* out_keys, uint64_t* out_values, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const bool hv = b0_values || heavy_values;
  if (!out_keys || (b0 > 0 && !b0_keys) || m > 512 || (m > 0 && (!heavy_keys || !heavy_sizes))) return DTSORT_EINVAL;
  if (hv && (!out_values || (b0 > 0 && !b0_values) || (m > 0 && !heavy_values))) return DTSORT_EINVAL;
  uint64_t hs = 0;
  for (size_t i = 0; i < m; ++i) hs += heavy_sizes[i];
  const uint64_t zsize = b0 + hs;
  if (zsize >= (1ull << 32)) return DTSORT_EINVAL;
  if (zsize == 0) return DTSORT_OK;
  // one zone laid out as [B0 | B1 .. Bm] in buffer 0; merged into buffer 1
  const int g = 10;
  const SlotLayout sl = slot_layout(g, false);
  Tmp tmp;
  uint64_t* zk = (uint64_t*)tmp.get(8 * zsize);
  uint64_t* zv = hv ? (uint64_t*)tmp.get(8 * zsize) : nullptr;
  uint8_t* tab = (uint8_t*)tmp.get(sl.bytes);
  Merge* dm = (Merge*)tmp.get(sizeof(Merge));
  const uint32_t nunits = (uint32_t)((zsize + 4095) / 4096);
  uint2* mu = (uint2*)tmp.get(sizeof(uint2) * nunits);
  uint32_t* dcount = (uint32_t*)tmp.get(2 * sizeof(uint32_t));
  if (!zk || !tab || !dm || !mu || !dcount || (hv && !zv)) return DTSORT_ENOMEM;
  const uint32_t hcount[2] = {1u, nunits};
  SCHK(hipMemcpyAsync(dcount, hcount, sizeof(hcount), hipMemcpyHostToDevice, s));
  if (b0) SCHK(hipMemcpyAsync(zk, b0_keys, 8 * b0, hipMemcpyDeviceToDevice, s));
  if (hv && b0) SCHK(hipMemcpyAsync(zv, b0_values, 8 * b0, hipMemcpyDeviceToDevice, s));
  if (hv && hs) SCHK(hipMemcpyAsync(zv + b0, heavy_values, 8 * hs, hipMemcpyDeviceToDevice, s));
  std::vector<uint8_t> slot(sl.bytes, 0);
  uint64_t* H = (uint64_t*)(slot.data() + sl.heavy);
  uint32_t* st = (uint32_t*)(slot.data() + sl.starts);
  st[0] = 0;
  st[1] = (uint32_t)b0;
  for (size_t i = 0; i < m; ++i) {
    H[i] = heavy_keys[i];
    st[2 + i] = st[1 + i] + heavy_sizes[i];
  }
  SCHK(hipMemcpyAsync(tab, slot.data(), sl.bytes, hipMemcpyHostToDevice, s));
  Merge mg;
  std::memset(&mg, 0, sizeof(mg));
  mg.zone_off = 0;
  mg.tab_off = 0;
  mg.b0 = (uint32_t)b0;
  mg.m = (uint32_t)m;
  mg.hbase = 0;
  mg.bstart = 0;
  mg.zone_rel = 0;
  mg.unit_base = 0;
  mg.n_units = nunits;
  mg.b0_buf = 0;
  mg.hv_buf = 0;
  mg.out_buf = 1;
  mg.g = (uint8_t)g;
  SCHK(hipMemcpyAsync(dm, &mg, sizeof(mg), hipMemcpyHostToDevice, s));
  launch_merge_units(dm, dcount, 1, 1, mu, s);
  if (hv) {
    Bufs<uint64_t, uint64_t> b;
    b.k[0] = zk;
    b.k[1] = out_keys;
    b.v[0] = zv;
    b.v[1] = out_values;
    launch_merge<uint64_t, uint64_t>(dm, dcount, 1, 1, mu, dcount + 1, nunits, nunits, tab, b, MV_GATHER, s);
  } else {
    Bufs<uint64_t, NoVal> b;
    b.k[0] = zk;
    b.k[1] = out_keys;
    launch_merge<uint64_t, NoVal>(dm, dcount, 1, 1, mu, dcount + 1, nunits, nunits, tab, b, MV_GATHER, s);
  }
  SCHK(hipGetLastError());
  SCHK(hipStreamSynchronize(s));
  return DTSORT_OK;
}

}  // extern "C"

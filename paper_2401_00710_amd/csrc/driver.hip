// Host driver of the DovetailSort library: the level loop of Alg. 2 over
// batched subproblems, device memory management, and the C ABI of dtsort.h.
//
// Per level: prep (chunking) -> plan (Step 1) -> histogram, column scan,
// bucket scan, scatter (Step 2) -> child planning (Step 3 bookkeeping) ->
// read back one block of counters -> leaf sorts and copies of this level.
// After the last level the dovetail merges (Step 4) run deepest level first,
// so every zone merges after its light bucket is completely sorted.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dtsort.h"
#include "launch.hpp"

namespace dts {

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(DTSORT_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

constexpr int MAX_LEVELS = 160;

struct LevelKeep {
  DevBuf tab, merges, munits, spills;
  uint32_t n_merges = 0, n_munits = 0, n_spills = 0;
  Caps caps{};
  double merge_records = 0;
};

// Device buffers of one sort schedule (the eager level loop of a context, or
// one recorded graph).
struct Work {
  DevBuf tk;                      // ping-pong partner of keys (and values), unless the caller gives one
  DevBuf tasks[2], units, cm, leaf[LEAF_CLASSES + 1], copies, ctr;  // leaf[LEAF_PAIR]: paired halves
  LevelKeep lv[MAX_LEVELS];  // kept per level until the merge phase
};

struct GraphEntry;

struct Ctx {
  int device = -1;
  hipStream_t owner = nullptr;  // the stream this context serves
  std::mutex mu;                // one call at a time on this context
  std::mutex app_mu;            // the applications' buffers (an application call holds it throughout)
  uint64_t used = 0;            // registry tick of the last call (least recently used is taken over)
  Work w;
  DevBuf lrn;
  DevBuf copy_items;  // item list of dtsort_copy_u32
  DevBuf app_keys;    // graph transpose: the edges' targets as sort keys; then an error word
  uint32_t* h_app = nullptr;  // pinned: the applications' error word
  LevelCounters* h_ctr = nullptr;  // pinned
  void* h_stage = nullptr;         // pinned staging
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  std::vector<hipEvent_t> ev_pool;
  struct Ctx* inner = nullptr;     // separate state for the sort of the learned partitioner's sample
  std::vector<GraphEntry*> graphs;
  hipStream_t cap_stream = nullptr;  // graphs are recorded on this stream
  hipStream_t cap_stream2 = nullptr;  // ... with a second stream for the leaf sorts
  hipStream_t side = nullptr;         // eager schedule: leaf sorts beside the next level
  hipEvent_t side_ev[4] = {};
  hipEvent_t fork_events[2 * (MAX_LEVELS + 2)] = {};
  uint64_t clock = 0;
};

// Per-kernel timing with HIP events on the sort's stream (opts->profile).
struct Prof {
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  bool on = false;
  hipStream_t s = nullptr;
  Ctx* c = nullptr;
  std::vector<Rec> recs;
  Rec cur;
  hipEvent_t ev() {
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int kind) {
    if (!on) return;
    cur.kind = kind;
    cur.a = ev();
    cur.b = ev();
    cur.bytes = 0;
    (void)hipEventRecord(cur.a, s);
  }
  void end(double bytes) {
    if (!on) return;
    cur.bytes = bytes;
    (void)hipEventRecord(cur.b, s);
    recs.push_back(cur);
  }
  void finish(dtsort_stats* st) {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    for (const Rec& r : recs) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      if (st) {
        st->kernel_ms[r.kind] += ms;
        st->kernel_bytes[r.kind] += r.bytes;
        st->kernel_launches[r.kind] += 1;
      }
      c->ev_pool.push_back(r.a);
      c->ev_pool.push_back(r.b);
    }
    recs.clear();
  }
};
enum ProfKind { PK_PLAN = 0, PK_HIST, PK_SCAN, PK_SCATTER, PK_CHILDREN, PK_LEAF, PK_COPY, PK_MERGE };

// Contexts per device, one per stream: a call locks only its stream's
// context, so calls on different streams run concurrently (each context has
// its own buffers; a stream without a caller workspace gets its own partner
// buffer).  g_mu guards the registry itself.
static std::mutex g_mu;
static std::vector<std::vector<Ctx*>> g_ctx;
static uint64_t g_tick = 0;
constexpr size_t MAX_CTX_PER_DEVICE = 8;

// Grow-only device buffer; synchronises `s` (and `s2`, when given) first
// when it must reallocate, since earlier enqueued work may still use the old
// allocation.
static int ensure(DevBuf& b, size_t bytes, hipStream_t s, hipStream_t s2 = nullptr) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return 0;
  HIPCHK(hipStreamSynchronize(s));
  if (s2) HIPCHK(hipStreamSynchronize(s2));
  if (b.p) HIPCHK(hipFree(b.p));
  b.p = nullptr;
  b.cap = 0;
  size_t want = std::max(bytes, b.cap + b.cap / 2);
  want = (want + 255) & ~(size_t)255;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(DTSORT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    want = bytes;
  }
  b.cap = want;
  return 0;
}

static Ctx* new_ctx(int dev) {
  Ctx* c = new Ctx();
  c->device = dev;
  if (hipHostMalloc((void**)&c->h_ctr, sizeof(LevelCounters) * (MAX_LEVELS + 1)) != hipSuccess ||
      hipHostMalloc(&c->h_stage, 1 << 16) != hipSuccess ||
      hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return nullptr;
  }
  return c;
}

// The context of (current device, stream s).  Beyond MAX_CTX_PER_DEVICE
// streams the least recently used context is taken over: its lock orders the
// host calls, and a call on a stream other than the context's previous one
// first waits for that stream's last work (sort_entry).
static int get_ctx(hipStream_t s, Ctx** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1);
  std::vector<Ctx*>& v = g_ctx[dev];
  Ctx* hit = nullptr;
  for (Ctx* c : v)
    if (c->owner == s) hit = c;
  if (!hit && v.size() < MAX_CTX_PER_DEVICE) {
    hit = new_ctx(dev);
    if (!hit) return fail(DTSORT_ENOMEM, "pinned host allocation failed");
    hit->owner = s;
    v.push_back(hit);
  } else if (!hit) {
    hit = *std::min_element(v.begin(), v.end(), [](const Ctx* a, const Ctx* b) { return a->used < b->used; });
    hit->owner = s;
  }
  hit->used = ++g_tick;
  *out = hit;
  return 0;
}

static void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

static void free_work(Work& w) {
  free_buf(w.tk);
  for (auto& b : w.tasks) free_buf(b);
  free_buf(w.units);
  free_buf(w.cm);
  for (auto& b : w.leaf) free_buf(b);
  free_buf(w.copies);
  free_buf(w.ctr);
  for (auto& l : w.lv) {
    free_buf(l.tab);
    free_buf(l.merges);
    free_buf(l.munits);
    free_buf(l.spills);
  }
}

template <typename K, typename V>
struct SortJob {
  Bufs<K, V> bufs;
  size_t n;
  const uint64_t* seg;
  uint32_t n_seg;
  int key_bits;
  dtsort_opts o;
};

static uint32_t cutoff_for(int kb, bool hv, int req) {
  const uint32_t cap = (kb == 8 && hv) ? 8192u : 16384u;
  if (req <= 0) return cap;
  return std::min<uint32_t>(cap, std::max<uint32_t>(2u, (uint32_t)req));
}

// ---------------------------------------------------------------- tuning
// Rows of the tuning table: key bytes, value bytes, segmented (0/1), a range
// [lo, hi] of floor(log2 n), and the parameters chosen for it (digit bits,
// base-case cutoff, scatter tile shape, digit bits of the levels below the
// root; 0 = automatic, a missing last column is 0).  The first matching row
// wins.
struct TuneRow {
  int kb, vb, seg, lo, hi, digit_bits, cutoff, tile, digit_bits_below;
};

static std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&dtsort_default_opts, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k + 1);
  }
  return std::string();
}

static const std::vector<TuneRow>& tune_table() {
  static std::vector<TuneRow> rows = [] {
    std::vector<TuneRow> r;
    const char* env = getenv("DTSORT_TUNE_FILE");
    const std::string path = env ? std::string(env) : lib_dir() + "tune_table.txt";
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return r;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
      if (line[0] == '#') continue;
      TuneRow t;
      t.digit_bits_below = 0;
      if (sscanf(line, "%d %d %d %d %d %d %d %d %d", &t.kb, &t.vb, &t.seg, &t.lo, &t.hi, &t.digit_bits, &t.cutoff,
                 &t.tile, &t.digit_bits_below) >= 8)
        r.push_back(t);
    }
    fclose(f);
    return r;
  }();
  return rows;
}

struct Tuned {
  int digit_bits, cutoff, tile, digit_bits_below;
};

static Tuned tuned_params(int kb, int vb, bool seg, size_t n) {
  int lg = 0;
  while (lg < 63 && (2ull << lg) <= n) ++lg;
  for (const TuneRow& t : tune_table())
    if (t.kb == kb && t.vb == vb && t.seg == (seg ? 1 : 0) && lg >= t.lo && lg <= t.hi)
      return Tuned{t.digit_bits, t.cutoff, t.tile, t.digit_bits_below};
  return Tuned{0, 0, 0, 0};
}

// Resolved parameters of one call.
struct Params {
  int gover;        // digit-bit override of the roots (0 = automatic)
  int gbelow;       // ... of the subproblems below them (0 = automatic)
  uint32_t cutoff;  // base-case threshold
  int tile;         // scatter tile shape (LevelArgs::tile)
};

template <typename K, typename V>
static Params resolve_params(const SortJob<K, V>& J) {
  constexpr bool HV = HasVal<V>::value;
  const dtsort_opts& o = J.o;
  int gover = o.digit_bits, creq = o.lds_cutoff, tile = o.tile_shape, gbelow = o.digit_bits_below;
  if (o.tuned) {
    const Tuned tp = tuned_params((int)sizeof(K), HV ? (int)sizeof(V) : 0, J.seg != nullptr, J.n);
    // the table's width below the root only where the caller left both widths open
    if (gbelow <= 0 && gover <= 0) gbelow = tp.digit_bits_below;
    if (gover <= 0) gover = tp.digit_bits;
    if (creq <= 0) creq = tp.cutoff;
    if (tile <= 0) tile = tp.tile;
  }
  Params p;
  p.gover = gover;
  p.gbelow = gbelow > 0 ? gbelow : gover;
  p.cutoff = cutoff_for((int)sizeof(K), HV, creq);
  p.tile = tile > 0 ? tile - 1 : 0;
  return p;
}

template <typename K, typename V>
static int run_sort(Ctx* c, SortJob<K, V>& J, hipStream_t s, dtsort_stats* stats);

template <typename K, typename V>
static void fill_caps(LevelArgs& a, uint32_t n_tasks, uint64_t total, int gmax, uint32_t cutoff) {
  const uint64_t nbc = (uint64_t)nb_cap(gmax);
  const uint64_t buckets = (uint64_t)n_tasks * nbc;
  a.caps.tasks = (uint32_t)std::min<uint64_t>(buckets, total / (cutoff + 1ull) + 1);
  a.caps.leaf = (uint32_t)std::min<uint64_t>(2 * buckets, total / 2 + 1);  // a paired bucket takes two entries
  a.caps.copies = (uint32_t)std::min<uint64_t>(buckets + total / COPY_PIECE + 1, total + 1);
  a.caps.merges = (uint32_t)std::min<uint64_t>((uint64_t)n_tasks << (gmax - 1), total + 1);
  a.caps.munits = (uint32_t)(total / 4096 + a.caps.merges + 1);
  a.caps.spills = (uint32_t)(total / COPY_PIECE + a.caps.merges + 1);
}

static void add_stats(dtsort_stats* st, const LevelCounters& h, bool level) {
  if (!st) return;
  if (level) {
    st->levels += h.st_tasks ? 1 : 0;
    st->tasks += h.st_tasks;
    st->records_distributed += h.st_distributed;
    st->heavy_keys += h.st_heavy_keys;
    st->heavy_records += h.st_heavy_records;
    st->merges += h.merges;
    st->records_merged += h.st_merge_records;
    st->records_copied += h.st_copy_records;
    st->overflow_records += h.st_overflow_records;
  }
  for (int k = 0; k <= LEAF_PAIR; ++k) st->leaf_sorts += h.leaf[k];
  st->records_leaf_sorted += h.st_leaf_records;
  st->records_pair_merged += h.st_pair_records;
}

constexpr uint32_t LEARN_SAMPLE = 1u << 16;  // training sample (sorted by the method itself)
constexpr uint32_t LEARN_HELD = 1u << 14;    // held-out sample for the balance judge

// Learned root plan (LEARNED mode, root task already planned by the sampling
// step).  A held-out sample is drawn and the judge first predicts the work
// the digit plan leaves and what an ideal split into the model's zones
// would leave; only when the digit plan is predicted clearly worse (more
// than TRAIN_MARGIN x) is the model trained: the training sample is drawn
// and sorted by the method itself, the CDF model trained, its splitters
// derived, and the judge keeps the model's zones when their predicted work
// is below USE_MARGIN x the digit plan's (or always with opts->learned_judge
// = 1).  The decision is read back once (the eager schedule synchronises per
// level anyway); everything else stays on the device.
// Zones of a learned root: at most 2^8 (255 splitters), with 8-bit digits
// below them unless the caller fixes the width.  Finer learned zones cost
// more than they balance: on 10^9 keys of the 64-bit mixture, 2^9 zones
// (with 9-bit digits below) took 51 ms against 41 ms for 2^8.
constexpr int LEARN_GAMMA = 8;
constexpr float TRAIN_MARGIN = 1.25f;
constexpr float USE_MARGIN = 0.9f;
static int learned_gamma(size_t n, int gover) {
  return std::min(plan_gamma((uint32_t)std::min<size_t>(n, 0xFFFFFFFFu), gover), LEARN_GAMMA);
}

template <typename K, typename V>
static int learned_root(Ctx* c, SortJob<K, V>& J, LevelArgs& a, hipStream_t s, LearnedInfo* info,
                        LearnedInfo* h_info) {
  const dtsort_opts& o = J.o;
  // 128 steps: on the 64-bit mixture and the bit-exponential pairs the zones
  // balance as well as after 256 (or better), at half the training time
  const int steps = o.learned_steps > 0 ? o.learned_steps : 128;
  uint32_t batch = o.learned_batch > 0 ? (uint32_t)o.learned_batch : 1024u;
  batch = std::min(batch, LEARN_SAMPLE);
  const float lr = o.learned_lr > 0 ? o.learned_lr : 3e-3f;
  const uint32_t N = LEARN_SAMPLE, HN = LEARN_HELD;
  const size_t nwg = (batch + MLP_GT - 1) / MLP_GT;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    size_t o2 = off;
    off += (bytes + 255) & ~(size_t)255;
    return o2;
  };
  const size_t o_s = carve(sizeof(K) * N), o_h = carve(sizeof(K) * HN), o_x = carve(4 * N), o_y = carve(4 * N),
               o_p = carve(4 * N), o_mono = carve(4 * N), o_par = carve(4 * MLP_PARAMS), o_m = carve(4 * MLP_PARAMS),
               o_v = carve(4 * MLP_PARAMS), o_part = carve(4 * (MLP_PARAMS + 1) * nwg), o_l = carve(4 * (size_t)steps),
               o_spl = carve(8 << GMAX);
  int r;
  if ((r = ensure(c->lrn, off, s))) return r;
  char* base = (char*)c->lrn.p;
  K* samp = (K*)(base + o_s);
  K* held = (K*)(base + o_h);
  float* x = (float*)(base + o_x);
  float* y = (float*)(base + o_y);
  float* pred = (float*)(base + o_p);
  float* mono = (float*)(base + o_mono);
  float* par = (float*)(base + o_par);
  float* m = (float*)(base + o_m);
  float* v = (float*)(base + o_v);
  float* part = (float*)(base + o_part);
  float* losses = (float*)(base + o_l);
  uint64_t* spl = (uint64_t*)(base + o_spl);
  const uint32_t zones = 1u << learned_gamma(J.n, o.digit_bits);
  JudgeParams jp;
  jp.scale = (float)J.n / (float)HN;
  jp.cutoff = (float)a.cutoff;
  jp.g_digit = plan_gamma((uint32_t)std::min<size_t>(J.n, 0xFFFFFFFFu), a.g_override);
  jp.g_learned = a.g_learned_child > 0 ? a.g_learned_child : LEARN_GAMMA;
  jp.force = o.learned_judge == 1;
  jp.train_margin = TRAIN_MARGIN;
  jp.use_margin = USE_MARGIN;
  learned_kernels_draw<K>(J.bufs.k[0], J.n, o.seed, 0x4C48u, HN, held, s);
  learned_kernels_judge<K>(a.tasks, a.tab, held, HN, nullptr, zones, jp, info, losses, 0, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h_info, info, sizeof(LearnedInfo), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!h_info->trained) return 0;  // the digit zones are kept; nothing to train
  learned_kernels_draw<K>(J.bufs.k[0], J.n, o.seed, 0x4C52u, N, samp, s);
  HIPCHK(hipGetLastError());
  // the training sample is sorted by the method itself, on separate state
  if (!c->inner) {
    c->inner = new_ctx(c->device);
    if (!c->inner) return fail(DTSORT_ENOMEM, "pinned host allocation failed");
  }
  SortJob<K, NoVal> J2;
  J2.n = N;
  J2.seg = nullptr;
  J2.n_seg = 0;
  J2.key_bits = J.key_bits;
  dtsort_default_opts(&J2.o);
  J2.o.seed = o.seed;
  if ((r = ensure(c->inner->w.tk, dtsort_workspace_bytes((int)sizeof(K), 0, N), s))) return r;
  J2.bufs.k[0] = samp;
  J2.bufs.k[1] = (K*)c->inner->w.tk.p;
  if ((r = run_sort<K, NoVal>(c->inner, J2, s, nullptr))) return r;
  mlp_data<K>(samp, N, J.key_bits, x, y, s);
  mlp_train(x, y, N, o.seed, steps, batch, lr, par, m, v, part, losses, s);
  mlp_forward(par, x, N, pred, s);
  learned_kernels_split<K>(samp, pred, N, zones, mono, spl, s);
  learned_kernels_judge<K>(a.tasks, a.tab, held, HN, spl, zones, jp, info, losses, steps, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h_info, info, sizeof(LearnedInfo), hipMemcpyDeviceToHost, s));
  return 0;
}

template <typename K, typename V>
static int run_sort(Ctx* c, SortJob<K, V>& J, hipStream_t s, dtsort_stats* stats) {
  constexpr bool HV = HasVal<V>::value;
  const size_t n = J.n;
  const dtsort_opts& o = J.o;
  const Params P = resolve_params(J);
  const bool learned = o.mode == DTSORT_MODE_LEARNED && !J.seg && n >= (1u << 20);
  // the root is planned by the sampling step at the usual width (the judge
  // may keep it); a learned root takes 2^8 zones and, unless the caller fixed
  // the digit width, its children 8-bit digits (10^9 keys of the 64-bit
  // mixture sorted in 41 ms with 8-bit digits below a learned root against
  // 49 ms with 9 bits)
  const int gover = P.gover;
  const uint32_t cutoff = P.cutoff;
  Work& W = c->w;
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.seed = o.seed;
  a.g_override = gover;
  a.g_learned_child = o.digit_bits > 0 ? o.digit_bits : LEARN_GAMMA;
  a.cutoff = cutoff;
  for (int k = 0; k < LEAF_CLASSES; ++k) a.leaf_max[k] = leaf_cap<K, V>(k);
  a.leaf_max[LEAF_PAIR] = pair_max<K, V>(cutoff);
  a.plain = o.mode == DTSORT_MODE_PLAIN;
  a.key_bits = J.key_bits;
  a.tile = P.tile;
  a.ordered = o.ordered_ranks != 0;
  a.merge_variant = o.merge_variant;
  if (stats) std::memset(stats, 0, sizeof(*stats));

  int r;
  // counters: [0] = the root (or seeding) step, [L + 1] = level L
  if ((r = ensure(W.ctr, sizeof(LevelCounters) * (MAX_LEVELS + 1) + 256, s))) return r;
  LevelCounters* dctr = (LevelCounters*)W.ctr.p;
  void* d_info = (char*)W.ctr.p + sizeof(LevelCounters) * (MAX_LEVELS + 1);
  Prof prof;
  prof.on = o.profile != 0 && stats != nullptr;
  prof.s = s;
  prof.c = c;
  const double rec_bytes = (double)sizeof(K) + (HV ? (double)sizeof(V) : 0.0);
  hipEvent_t le0 = nullptr, le1 = nullptr;
  // Batched form: a level's leaf sorts, copies and merge-unit lists run on a
  // side stream beside the next level's planning and counting sort (disjoint
  // record ranges), joining before that level's child planning rewrites the
  // leaf and copy lists, and before the merges (the segments sorted at
  // seeding overlap level 0: 4096 segments 3.49 -> 3.24 ms).  A single
  // sort's levels gain nothing from it (10^9 keys: uniform 11.09 vs 11.14
  // ms, Zipf 14.45 vs 14.48 ms without and with), nor when profiling (the
  // timing events are on `s`).
  hipStream_t side = s;
  if (!prof.on && J.seg) {
    if (!c->side) HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->side_ev[0])
      for (hipEvent_t& ev : c->side_ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    side = c->side;
  }
  hipStream_t grow2 = side != s ? side : nullptr;  // reallocation waits for the side stream too
  struct SideJoin {  // `s` waits for the side stream's last work on every way out
    hipStream_t s = nullptr;
    hipEvent_t pending = nullptr;
    void join() {
      if (pending) (void)hipStreamWaitEvent(s, pending, 0);
      pending = nullptr;
    }
    ~SideJoin() { join(); }
  } sj;
  sj.s = s;
  uint32_t evi = 0;
  auto fork = [&]() -> int {
    if (side == s) return 0;
    hipEvent_t e = c->side_ev[evi++ & 3u];
    HIPCHK(hipEventRecord(e, s));
    HIPCHK(hipStreamWaitEvent(side, e, 0));
    return 0;
  };
  auto side_done = [&]() -> int {
    if (side == s) return 0;
    hipEvent_t e = c->side_ev[evi++ & 3u];
    HIPCHK(hipEventRecord(e, side));
    sj.pending = e;
    return 0;
  };

  uint32_t n_tasks = 0;
  uint64_t total = 0;
  uint32_t max_size = 0;
  int cur = 0;
  const uint64_t cap_total = std::max<uint64_t>(n, 2);

  // ---- root
  if (J.seg) {
    // seeding writes level-0 tasks and leaves like a child-planning step
    const int gmax0 = plan_gamma((uint32_t)std::min<size_t>(n, 0xFFFFFFFFu), gover);
    fill_caps<K, V>(a, std::max<uint32_t>(J.n_seg, 1), cap_total, gmax0, cutoff);
    a.caps.tasks = J.n_seg + 1;
    a.caps.leaf = 2 * J.n_seg + 2;  // a paired segment takes two entries
    a.caps.copies = J.n_seg + 1;
    if ((r = ensure(W.tasks[cur], sizeof(Task) * (size_t)a.caps.tasks, s))) return r;
    for (int k = 0; k <= LEAF_PAIR; ++k)
      if ((r = ensure(W.leaf[k], sizeof(Leaf) * (size_t)a.caps.leaf, s))) return r;
    if ((r = ensure(W.copies, sizeof(Leaf) * (size_t)a.caps.copies, s))) return r;
    a.next = (Task*)W.tasks[cur].p;
    for (int k = 0; k <= LEAF_PAIR; ++k) a.leaf[k] = (Leaf*)W.leaf[k].p;
    a.copies = (Leaf*)W.copies.p;
    a.ctr = dctr;
    launch_zero_counters(dctr, 1, s);
    launch_seed_segments<K, V>(a, J.seg, J.n_seg, n, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_ctr, dctr, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const LevelCounters h = c->h_ctr[0];
    if (h.error & ERR_SEGMENTS) return fail(DTSORT_EINVAL, "segment offsets are not valid");
    if (h.error) return fail(DTSORT_EINTERNAL, "capacity check failed while seeding segments");
    prof.begin(PK_LEAF);
    if ((r = fork())) return r;
    for (int k = 0; k < LEAF_CLASSES; ++k)
      launch_leaf<K, V>((Leaf*)W.leaf[k].p, &dctr[0].leaf[k], a.caps.leaf, std::min(h.leaf[k], a.caps.leaf), k,
                        J.bufs, side);
    launch_pairs<K, V>((Leaf*)W.leaf[LEAF_PAIR].p, &dctr[0].leaf[LEAF_PAIR], a.caps.leaf,
                       std::min(h.leaf[LEAF_PAIR], a.caps.leaf), h.leaf[LEAF_PAIR] / 2, J.bufs, side);
    if ((r = side_done())) return r;
    prof.end(2.0 * rec_bytes * (double)(h.st_leaf_records + h.st_pair_records));
    HIPCHK(hipGetLastError());
    add_stats(stats, h, false);
    n_tasks = h.next_tasks;
    total = h.next_records;
    max_size = h.next_max_size;
    // the root leaves finish before level 0's child planning reuses the leaf
    // lists (it waits for the side stream)
  } else {
    if (n <= 1) return 0;
    if (n <= cutoff) {
      if ((r = ensure(W.leaf[0], sizeof(Leaf), s))) return r;
      Leaf* hl = (Leaf*)c->h_stage;
      HIPCHK(hipStreamSynchronize(s));  // staging buffer reuse
      hl->off = 0;
      hl->size = (uint32_t)n;
      hl->bits = (uint8_t)J.key_bits;
      hl->from = 0;
      hl->to = 0;
      hl->pad = 0;
      uint32_t* one = (uint32_t*)((char*)c->h_stage + 64);
      *one = 1;
      HIPCHK(hipMemcpyAsync(W.leaf[0].p, hl, sizeof(Leaf), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(&dctr[0].leaf[0], one, 4, hipMemcpyHostToDevice, s));
      int cls = LEAF_CLASSES - 1;
      for (int k = LEAF_CLASSES - 2; k >= 0; --k)
        if (n <= leaf_cap<K, V>(k)) cls = k;
      launch_leaf<K, V>((Leaf*)W.leaf[0].p, &dctr[0].leaf[0], 1, 1, cls, J.bufs, s);
      HIPCHK(hipGetLastError());
      if (stats) stats->leaf_sorts = 1, stats->records_leaf_sorted = n;
      return 0;
    }
    if ((r = ensure(W.tasks[cur], sizeof(Task), s))) return r;
    launch_root<K>((Task*)W.tasks[cur].p, dctr, n, J.key_bits, plan_gamma((uint32_t)n, gover), s);
    n_tasks = 1;
    total = n;
    max_size = (uint32_t)n;
  }

  // ---- levels
  // the roots' children and every later subproblem take the width below the root
  a.g_override = P.gbelow;
  int L = 0;
  for (; n_tasks > 0; ++L) {
    if (L >= MAX_LEVELS) return fail(DTSORT_EINTERNAL, "recursion deeper than expected");
    // the widest digit of the level's tasks (below a learned root: its
    // children's width a.g_learned_child)
    int gmax = plan_gamma(max_size, L == 0 ? gover : P.gbelow);
    if (learned && L >= 1) gmax = std::max(gmax, a.g_learned_child);
    // chunk: a multiple of 8192 records aiming at ~2048 units per level (the
    // prep kernel derives the same value when it is left 0)
    uint64_t chunk = (total + 2047) / 2048;
    chunk = std::max<uint64_t>(8192, (chunk + 8191) / 8192 * 8192);
    const uint64_t units = total / chunk + n_tasks + 1;
    const bool learn_here = learned && L == 0;
    const SlotLayout sl = slot_layout(gmax, learn_here);
    const uint64_t tab_bytes = (uint64_t)n_tasks * sl.bytes;
    const uint32_t cols = dist_cols(gmax);
    const uint64_t cm_entries = units * cols * (uint64_t)nb_cap(gmax);
    LevelKeep& K_ = W.lv[L];
    fill_caps<K, V>(a, n_tasks, total, gmax, cutoff);
    a.caps.units = (uint32_t)units;
    a.caps.cm = cm_entries;
    a.caps.tab = tab_bytes;
    if ((r = ensure(W.units, sizeof(uint2) * units, s))) return r;
    if ((r = ensure(W.cm, 4 * cm_entries, s))) return r;
    if ((r = ensure(K_.tab, tab_bytes, s))) return r;
    if ((r = ensure(W.tasks[1 - cur], sizeof(Task) * (size_t)a.caps.tasks, s))) return r;
    for (int k = 0; k <= LEAF_PAIR; ++k)
      if ((r = ensure(W.leaf[k], sizeof(Leaf) * (size_t)a.caps.leaf, s, grow2))) return r;
    if ((r = ensure(W.copies, sizeof(Leaf) * (size_t)a.caps.copies, s, grow2))) return r;
    if ((r = ensure(K_.merges, sizeof(Merge) * (size_t)a.caps.merges, s))) return r;
    if ((r = ensure(K_.munits, sizeof(uint2) * (size_t)a.caps.munits, s))) return r;
    if ((r = ensure(K_.spills, sizeof(Leaf) * (size_t)a.caps.spills, s))) return r;
    a.tasks = (Task*)W.tasks[cur].p;
    a.n_tasks = n_tasks;
    a.chunk = (uint32_t)chunk;
    a.units = (uint2*)W.units.p;
    a.tab = (uint8_t*)K_.tab.p;
    a.slot_bytes = sl.bytes;
    a.cols = cols;
    a.cm = (uint32_t*)W.cm.p;
    a.next = (Task*)W.tasks[1 - cur].p;
    for (int k = 0; k <= LEAF_PAIR; ++k) a.leaf[k] = (Leaf*)W.leaf[k].p;
    a.copies = (Leaf*)W.copies.p;
    a.merges = (Merge*)K_.merges.p;
    a.spills = (Leaf*)K_.spills.p;
    a.in = dctr + L;
    a.ctr = dctr + L + 1;
    a.grid_tasks = n_tasks;
    a.grid_units = (uint32_t)units;
    launch_prep(a, s);
    prof.begin(PK_PLAN);
    launch_plan<K>(a, J.bufs.k[0], J.bufs.k[1], gmax, s);
    prof.end(0.0);
    if (learn_here) {
      HIPCHK(hipEventCreate(&le0));
      HIPCHK(hipEventCreate(&le1));
      HIPCHK(hipEventRecord(le0, s));
      if ((r = learned_root<K, V>(c, J, a, s, (LearnedInfo*)d_info, (LearnedInfo*)c->h_stage))) return r;
      HIPCHK(hipEventRecord(le1, s));
    }
    const uint32_t max_chunks = (uint32_t)(max_size / chunk + 1);
    prof.begin(PK_HIST);
    launch_distribute<K, V>(a, J.bufs, gmax, max_chunks, s, 0);
    prof.end((double)sizeof(K) * (double)total);
    prof.begin(PK_SCAN);
    launch_distribute<K, V>(a, J.bufs, gmax, max_chunks, s, 1);
    prof.end(8.0 * (double)cm_entries);
    prof.begin(PK_SCATTER);
    launch_distribute<K, V>(a, J.bufs, gmax, max_chunks, s, 2);
    prof.end(2.0 * rec_bytes * (double)total);
    sj.join();  // the previous level's leaf sorts have read their lists
    prof.begin(PK_CHILDREN);
    launch_children<K, V>(a, J.bufs, s);
    prof.end(0.0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_ctr + L + 1, a.ctr, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const LevelCounters h = c->h_ctr[L + 1];
    if (h.error) return fail(DTSORT_EINTERNAL, "device capacity check failed (flags " + std::to_string(h.error) + ")");
    if (learn_here && stats) {
      // read back by learned_root into the pinned staging area (the level's synchronisation covers it)
      const LearnedInfo li = *(const LearnedInfo*)c->h_stage;
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, le0, le1));
      stats->learned_used = (int32_t)li.use_learned;
      stats->learned_trained = (int32_t)li.trained;
      stats->learned_balance = li.bal_learned;
      stats->sampling_balance = li.bal_digit;
      stats->learned_final_loss = li.final_loss;
      stats->learned_cost = li.cost_learned;
      stats->sampling_cost = li.cost_digit;
      stats->ideal_cost = li.cost_ideal;
      stats->learned_ms = ms;
    }
    if (le0) (void)hipEventDestroy(le0), le0 = nullptr;
    if (le1) (void)hipEventDestroy(le1), le1 = nullptr;
    if ((r = fork())) return r;
    prof.begin(PK_LEAF);
    for (int k = 0; k < LEAF_CLASSES; ++k)
      launch_leaf<K, V>((Leaf*)W.leaf[k].p, &a.ctr->leaf[k], a.caps.leaf, h.leaf[k], k, J.bufs, side);
    launch_pairs<K, V>((Leaf*)W.leaf[LEAF_PAIR].p, &a.ctr->leaf[LEAF_PAIR], a.caps.leaf, h.leaf[LEAF_PAIR],
                       h.leaf[LEAF_PAIR] / 2, J.bufs, side);
    prof.end(2.0 * rec_bytes * (double)(h.st_leaf_records + h.st_pair_records));
    prof.begin(PK_COPY);
    launch_copy<K, V>((Leaf*)W.copies.p, &a.ctr->copies, a.caps.copies, h.copies, J.bufs, side);
    prof.end(2.0 * rec_bytes * (double)h.st_copy_records);
    K_.n_merges = h.merges;
    K_.n_munits = h.merge_units;
    K_.n_spills = h.spills;
    K_.caps = a.caps;
    K_.merge_records = (double)h.st_merge_records;
    launch_merge_units((Merge*)K_.merges.p, &a.ctr->merges, a.caps.merges, h.merges, (uint2*)K_.munits.p, side);
    if ((r = side_done())) return r;
    HIPCHK(hipGetLastError());
    add_stats(stats, h, true);
    n_tasks = h.next_tasks;
    total = h.next_records;
    max_size = h.next_max_size;
    cur = 1 - cur;
  }
  sj.join();  // light runs sorted before they are merged
  // ---- dovetail merges, deepest level first
  for (int l = L - 1; l >= 0 && o.merge_variant != MV_NONE; --l) {
    LevelKeep& K_ = W.lv[l];
    if (K_.n_merges == 0) continue;
    LevelCounters* lc = dctr + l + 1;
    prof.begin(PK_MERGE);
    launch_copy<K, V>((Leaf*)K_.spills.p, &lc->spills, K_.caps.spills, K_.n_spills, J.bufs, s);
    launch_merge<K, V>((Merge*)K_.merges.p, &lc->merges, K_.caps.merges, K_.n_merges, (uint2*)K_.munits.p,
                       &lc->merge_units, K_.caps.munits, K_.n_munits, (uint8_t*)K_.tab.p, J.bufs, o.merge_variant, s);
    prof.end(2.0 * rec_bytes * K_.merge_records);
    HIPCHK(hipGetLastError());
  }
  prof.finish(stats);
  return 0;
}

// ------------------------------------------------------------ graph form
// The whole schedule with no host read-back: every level's kernels read
// their work counts on the device and loop with a grid stride over
// persistent grids; every list is sized for the worst case of n records, and
// the number of levels is the bound below.  Recorded once into a HIP graph.
struct GPlan {
  int gmax = 8, levels = 0;
  uint32_t cutoff = 0;
  Caps caps{};
  uint64_t tab_bytes = 0;
  uint32_t slot_bytes = 0;
  uint32_t grid_tasks = 0, grid_units = 0, grid_leaf[LEAF_CLASSES] = {}, grid_pair = 0, grid_copy = 0, grid_mpos = 0,
           grid_munit = 0, grid_spill = 0, grid_finish = 0;
};

static int graph_levels_env() {
  const char* e = getenv("DTSORT_GRAPH_LEVELS");
  return e ? std::max(1, std::min(MAX_LEVELS, atoi(e))) : 0;
}

// levels > 0: record that many levels (tasks still open after them are
// finished by one workgroup each); 0: the bound below.
template <typename K, typename V>
static GPlan graph_plan(const SortJob<K, V>& J, const Params& P, int levels = 0) {
  GPlan g;
  const uint64_t n = std::max<uint64_t>(J.n, 2);
  const uint32_t n32 = (uint32_t)std::min<uint64_t>(n, 0xFFFFFFFFu);
  g.gmax = std::max(plan_gamma(n32, P.gover), plan_gamma(n32, P.gbelow));  // every recorded level's widest digit
  g.cutoff = P.cutoff;
  // Level bound: a task whose keys differ in at most gmin bits is the last of
  // its branch (one plain digit).  Otherwise its light children have at least
  // gmin fewer bits left, and its overflow child keeps the bits but takes the
  // top digit with no leading-zero skip and has no overflow child itself, so
  // its children have gmin fewer bits: two levels per digit, plus the last.
  // The graph records the levels a branch needs when no overflow bucket
  // occurs (one per digit); tasks still open after them (only below
  // overflow buckets, which hold the few keys above a sample's maximum) are
  // finished by one workgroup each.
  auto narrowest = [](int gw) { return gw > 0 ? std::max(1, std::min(gw, GMAX)) : 8; };
  const int gmin = std::min(narrowest(P.gover), narrowest(P.gbelow));
  const int kb = J.key_bits;
  g.levels = std::min(MAX_LEVELS, kb <= gmin ? 1 : (kb - gmin + gmin - 1) / gmin + 1);
  if (levels > 0) g.levels = std::min(MAX_LEVELS, levels);
  const uint64_t nbc = (uint64_t)nb_cap(g.gmax);
  const uint64_t tasks = n / (g.cutoff + 1ull) + 1;
  Caps& c = g.caps;
  c.tasks = (uint32_t)tasks;
  c.leaf = (uint32_t)std::min<uint64_t>(2 * (tasks * nbc + J.n_seg + 1), n + 1);  // paired buckets: two entries
  c.copies = (uint32_t)std::min<uint64_t>(tasks * nbc + n / COPY_PIECE + 1, n + 1);
  c.merges = (uint32_t)std::min<uint64_t>(tasks << (g.gmax - 1), n + 1);
  c.munits = (uint32_t)(n / 4096 + c.merges + 1);
  c.spills = (uint32_t)(n / COPY_PIECE + c.merges + 1);
  c.units = (uint32_t)(n / 8192 + tasks + 1);
  c.cm = (uint64_t)c.units * nbc;
  const SlotLayout sl = slot_layout(g.gmax, false);
  g.slot_bytes = sl.bytes;
  g.tab_bytes = tasks * sl.bytes;
  c.tab = g.tab_bytes;
  auto pg = [](uint32_t per_cu, uint64_t cap) { return (uint32_t)std::min<uint64_t>(persistent_grid(per_cu), cap); };
  g.grid_tasks = pg(4, c.tasks);
  g.grid_units = pg(8, c.units);
  // sorters per compute unit by leaf class (class 0 packs four one-wave
  // sorters in a workgroup): about four times what fits at once, so that the
  // dispatcher hands the later workgroups to whichever CUs come free (leaves
  // differ in size; each workgroup takes a fixed stride of them)
  // (a list of class k holds leaves of more than leaf_max[k-1] records, so at
  // most n / (leaf_max[k-1] + 1) of them, which bounds small sorts' grids)
  const uint32_t per_cu[LEAF_CLASSES] = {64, 32, 16, 8, 8};
  for (int k = 0; k < LEAF_CLASSES; ++k) {
    const uint64_t lo = k == 0 ? 1u : leaf_cap<K, V>(k - 1);
    const uint64_t most = n / (lo + 1) + (J.seg ? J.n_seg + 1ull : 1ull);
    g.grid_leaf[k] = pg(per_cu[k], std::min<uint64_t>(c.leaf, most));
  }
  // paired buckets hold more than the cutoff (two list entries each)
  const uint64_t pairs_most = n / (g.cutoff + 1ull) + (J.seg ? J.n_seg + 1ull : 1ull);
  if (pair_leaves<K, V>())
    g.grid_leaf[LEAF_CLASSES - 1] = std::max(g.grid_leaf[LEAF_CLASSES - 1], pg(8, 2 * pairs_most));
  g.grid_pair = pair_leaves<K, V>() ? pg(1, std::min<uint64_t>(c.leaf / 2 + 1, pairs_most)) : 0;
  g.grid_copy = pg(4, c.copies);
  g.grid_mpos = pg(32, c.merges);
  g.grid_munit = pg(16, c.munits);
  g.grid_spill = pg(4, c.spills);
  g.grid_finish = pg(1, c.tasks);
  return g;
}

// Gives every buffer of the graph-form schedule its size through `place`
// (an allocation, or a place in a caller's region).
template <typename Place>
static int graph_buffers(Work& W, const GPlan& g, Place&& place) {
  int r;
  const Caps& c = g.caps;
  if ((r = place(W.ctr, sizeof(LevelCounters) * (g.levels + 1)))) return r;
  for (auto& b : W.tasks)
    if ((r = place(b, sizeof(Task) * (size_t)c.tasks))) return r;
  if ((r = place(W.units, sizeof(uint2) * (size_t)c.units))) return r;
  if ((r = place(W.cm, 4 * c.cm))) return r;
  for (auto& b : W.leaf)
    if ((r = place(b, sizeof(Leaf) * (size_t)c.leaf))) return r;
  if ((r = place(W.copies, sizeof(Leaf) * (size_t)c.copies))) return r;
  for (int L = 0; L < g.levels; ++L) {
    LevelKeep& K_ = W.lv[L];
    if ((r = place(K_.tab, g.tab_bytes))) return r;
    if ((r = place(K_.merges, sizeof(Merge) * (size_t)c.merges))) return r;
    if ((r = place(K_.munits, sizeof(uint2) * (size_t)c.munits))) return r;
    if ((r = place(K_.spills, sizeof(Leaf) * (size_t)c.spills))) return r;
    K_.caps = c;
  }
  return 0;
}

template <typename K, typename V>
static int graph_alloc(Work& W, const GPlan& g, hipStream_t s) {
  return graph_buffers(W, g, [&](DevBuf& b, size_t bytes) { return ensure(b, bytes, s); });
}

// A second stream for the graph form: a level's leaf sorts, copies and
// merge-unit lists run beside the next level's planning and counting sort
// (their record ranges are disjoint), joining before the next child
// planning, which rewrites the leaf and copy lists.  Only used while
// recording (the fork and the join become graph edges).
struct Fork {
  hipStream_t s2 = nullptr;
  hipEvent_t ev[2 * (MAX_LEVELS + 2)] = {};
  int used = 0;
  hipEvent_t next() { return ev[used++]; }
};

// Enqueue the whole schedule on `s` (recordable: kernels only, and with a
// Fork, event records and waits between `s` and fk->s2).
template <typename K, typename V>
static void graph_enqueue(Work& W, const GPlan& g, const SortJob<K, V>& J, const Params& P, hipStream_t s,
                          Fork* fk = nullptr) {
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.seed = J.o.seed;
  a.g_override = P.gover;
  a.cutoff = g.cutoff;
  for (int k = 0; k < LEAF_CLASSES; ++k) a.leaf_max[k] = leaf_cap<K, V>(k);
  a.leaf_max[LEAF_PAIR] = pair_max<K, V>(g.cutoff);
  a.plain = J.o.mode == DTSORT_MODE_PLAIN;
  a.key_bits = J.key_bits;
  a.tile = P.tile;
  a.ordered = J.o.ordered_ranks != 0;
  a.merge_variant = J.o.merge_variant;
  a.caps = g.caps;
  LevelCounters* dctr = (LevelCounters*)W.ctr.p;
  for (int k = 0; k <= LEAF_PAIR; ++k) a.leaf[k] = (Leaf*)W.leaf[k].p;
  a.copies = (Leaf*)W.copies.p;
  hipStream_t side = fk ? fk->s2 : s;  // where the leaf lists of a level are worked off
  hipEvent_t joined = nullptr;         // the side stream's last work, to wait for before the lists are rewritten
  auto fork = [&]() {
    if (!fk) return;
    hipEvent_t e = fk->next();
    (void)hipEventRecord(e, s);
    (void)hipStreamWaitEvent(fk->s2, e, 0);
  };
  auto side_done = [&]() {
    if (!fk) return;
    joined = fk->next();
    (void)hipEventRecord(joined, fk->s2);
  };
  auto join = [&]() {
    if (fk && joined) (void)hipStreamWaitEvent(s, joined, 0);
    joined = nullptr;
  };
  launch_zero_counters(dctr, (uint32_t)g.levels + 1, s);
  if (J.seg) {
    a.next = (Task*)W.tasks[0].p;
    a.ctr = dctr;
    launch_seed_segments<K, V>(a, J.seg, J.n_seg, J.n, s);
    fork();
    for (int k = 0; k < LEAF_CLASSES; ++k)
      launch_leaf<K, V>((Leaf*)W.leaf[k].p, &dctr[0].leaf[k], g.caps.leaf, g.grid_leaf[k], k, J.bufs, side);
    launch_pairs<K, V>((Leaf*)W.leaf[LEAF_PAIR].p, &dctr[0].leaf[LEAF_PAIR], g.caps.leaf,
                       g.grid_leaf[LEAF_CLASSES - 1], g.grid_pair, J.bufs, side);
    side_done();
  } else {
    launch_root<K>((Task*)W.tasks[0].p, dctr, J.n, J.key_bits, plan_gamma((uint32_t)J.n, P.gover), s);
  }
  a.g_override = P.gbelow;  // the roots' children and every later subproblem
  for (int L = 0; L < g.levels; ++L) {
    LevelKeep& K_ = W.lv[L];
    a.tasks = (Task*)W.tasks[L & 1].p;
    a.next = (Task*)W.tasks[(L + 1) & 1].p;
    a.n_tasks = g.caps.tasks;
    a.chunk = 0;
    a.units = (uint2*)W.units.p;
    a.tab = (uint8_t*)K_.tab.p;
    a.slot_bytes = g.slot_bytes;
    a.cols = 1;
    a.cm = (uint32_t*)W.cm.p;
    a.merges = (Merge*)K_.merges.p;
    a.spills = (Leaf*)K_.spills.p;
    a.in = dctr + L;
    a.ctr = dctr + L + 1;
    a.grid_tasks = g.grid_tasks;
    a.grid_units = g.grid_units;
    launch_prep(a, s);
    launch_plan<K>(a, J.bufs.k[0], J.bufs.k[1], g.gmax, s);
    launch_distribute<K, V>(a, J.bufs, g.gmax, 0x7FFFFFFFu, s, -1);
    join();  // the previous level's leaves have read their lists
    launch_children<K, V>(a, J.bufs, s);
    fork();
    for (int k = 0; k < LEAF_CLASSES; ++k)
      launch_leaf<K, V>((Leaf*)W.leaf[k].p, &a.ctr->leaf[k], g.caps.leaf, g.grid_leaf[k], k, J.bufs, side);
    launch_pairs<K, V>((Leaf*)W.leaf[LEAF_PAIR].p, &a.ctr->leaf[LEAF_PAIR], g.caps.leaf,
                       g.grid_leaf[LEAF_CLASSES - 1], g.grid_pair, J.bufs, side);
    launch_copy<K, V>((Leaf*)W.copies.p, &a.ctr->copies, g.caps.copies, g.grid_copy, J.bufs, side);
    launch_merge_units((Merge*)K_.merges.p, &a.ctr->merges, g.caps.merges, g.grid_mpos, (uint2*)K_.munits.p, side);
    side_done();
  }
  join();
  // tasks created by the last recorded level
  launch_finish<K, V>((const Task*)W.tasks[g.levels & 1].p, &dctr[g.levels].next_tasks, g.caps.tasks, g.grid_finish,
                      J.bufs, s);
  for (int L = g.levels - 1; L >= 0 && J.o.merge_variant != MV_NONE; --L) {
    LevelKeep& K_ = W.lv[L];
    LevelCounters* lc = dctr + L + 1;
    launch_copy<K, V>((Leaf*)K_.spills.p, &lc->spills, g.caps.spills, g.grid_spill, J.bufs, s);
    launch_merge<K, V>((Merge*)K_.merges.p, &lc->merges, g.caps.merges, g.grid_mpos, (uint2*)K_.munits.p,
                       &lc->merge_units, g.caps.munits, g.grid_munit, (uint8_t*)K_.tab.p, J.bufs, J.o.merge_variant,
                       s);
  }
}

struct GraphKey {
  int kb, vb;
  const void *k, *v, *ws;
  size_t n;
  const uint64_t* seg;
  uint32_t n_seg;
  uint64_t seed;
  int key_bits, mode, gover, gbelow, tile, levels, ordered, merge_variant;
  uint32_t cutoff;
  bool operator==(const GraphKey& o) const {
    return kb == o.kb && vb == o.vb && k == o.k && v == o.v && ws == o.ws && n == o.n && seg == o.seg &&
           n_seg == o.n_seg && seed == o.seed && key_bits == o.key_bits && mode == o.mode && gover == o.gover &&
           gbelow == o.gbelow && tile == o.tile && levels == o.levels && cutoff == o.cutoff && ordered == o.ordered &&
           merge_variant == o.merge_variant;
  }
};

struct GraphEntry {
  GraphKey key;
  Work w;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  int levels = 0;
  uint32_t levels_cap = 0;  // capacity of the task list the finishing step reads
  uint64_t used = 0;
};

constexpr size_t MAX_GRAPHS = 4;

static void free_graph(GraphEntry* e) {
  if (e->x) (void)hipGraphExecDestroy(e->x);
  if (e->g) (void)hipGraphDestroy(e->g);
  free_work(e->w);
  delete e;
}

template <typename K, typename V>
static int graph_sort(Ctx* c, SortJob<K, V>& J, void* user_ws, hipStream_t s, dtsort_stats* stats) {
  constexpr bool HV = HasVal<V>::value;
  const Params P = resolve_params(J);
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.kb = (int)sizeof(K);
  key.vb = HV ? (int)sizeof(V) : 0;
  key.k = J.bufs.k[0];
  if constexpr (HV) key.v = J.bufs.v[0];
  key.ws = user_ws;
  key.n = J.n;
  key.seg = J.seg;
  key.n_seg = J.n_seg;
  key.seed = J.o.seed;
  key.key_bits = J.key_bits;
  key.mode = J.o.mode;
  key.gover = P.gover;
  key.gbelow = P.gbelow;
  key.tile = P.tile;
  key.ordered = J.o.ordered_ranks != 0;
  key.merge_variant = J.o.merge_variant;
  key.cutoff = P.cutoff;
  key.levels = graph_levels_env();  // 0: the count the first call measures
  GraphEntry* e = nullptr;
  for (GraphEntry* x : c->graphs)
    if (x->key == key) e = x;
  int r;
  if (!e) {
    if (c->graphs.size() >= MAX_GRAPHS) {
      auto it = std::min_element(c->graphs.begin(), c->graphs.end(),
                                 [](const GraphEntry* p, const GraphEntry* q) { return p->used < q->used; });
      // every earlier call on this context is ordered before `s` (sort_entry)
      HIPCHK(hipStreamSynchronize(s));
      free_graph(*it);
      c->graphs.erase(it);
    }
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    e = new GraphEntry();
    e->key = key;
    hipStream_t cs = c->cap_stream;
    if (!user_ws && (r = ensure(e->w.tk, dtsort_workspace_bytes((int)sizeof(K), HV ? (int)sizeof(V) : 0, J.n), cs))) {
      free_graph(e);
      return r;
    }
    HIPCHK(hipStreamSynchronize(cs));
    SortJob<K, V> J2 = J;
    if (!user_ws) set_partner(J2, (char*)e->w.tk.p);
    // The first call sorts with the eager schedule, which measures how many
    // levels this input needs; the graph records that many (no empty levels
    // to replay: each costs every one of its kernels' dispatch).  Replays on
    // inputs that need more finish the tasks still open with one workgroup
    // each, so the result never depends on the count.
    int levels = key.levels;
    bool sorted_eagerly = false;
    if (levels == 0) {
      dtsort_stats es;
      std::memset(&es, 0, sizeof(es));
      if ((r = run_sort<K, V>(c, J2, s, &es))) {
        free_graph(e);
        return r;
      }
      if (stats) *stats = es;
      levels = std::max<int>(1, (int)es.levels);
      sorted_eagerly = true;
    }
    const GPlan g = graph_plan(J, P, levels);
    e->levels = g.levels;
    e->levels_cap = g.caps.tasks;
    if ((r = graph_alloc<K, V>(e->w, g, cs))) {
      free_graph(e);
      return r;
    }
    HIPCHK(hipStreamSynchronize(cs));
    (void)persistent_grid(1);  // device query outside the recording
    if (!c->cap_stream2) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream2, hipStreamNonBlocking));
    if (!c->fork_events[0])
      for (hipEvent_t& ev : c->fork_events) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    Fork fk;
    fk.s2 = c->cap_stream2;
    for (size_t i = 0; i < sizeof(fk.ev) / sizeof(fk.ev[0]); ++i) fk.ev[i] = c->fork_events[i];
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
      // the second stream pays off where the segments sorted at seeding
      // overlap level 0; a single sort's levels gain nothing from it, and
      // every fork and join is a cross-stream wait in the graph
      graph_enqueue<K, V>(e->w, g, J2, P, cs, J.seg ? &fk : nullptr);
      const hipError_t le = hipGetLastError();
      ce = hipStreamEndCapture(cs, &e->g);
      if (ce == hipSuccess) ce = le;
    }
    if (ce == hipSuccess) ce = hipGraphInstantiate(&e->x, e->g, nullptr, nullptr, 0);
    if (ce != hipSuccess) {
      free_graph(e);
      return fail(DTSORT_EHIP, std::string("graph recording failed: ") + hipGetErrorString(ce));
    }
    c->graphs.push_back(e);
    if (sorted_eagerly) {
      e->used = ++c->clock;
      return 0;  // this call's result came from the eager schedule
    }
  }
  e->used = ++c->clock;
  HIPCHK(hipGraphLaunch(e->x, s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    std::vector<LevelCounters> h(e->levels + 1);
    HIPCHK(hipMemcpyAsync(h.data(), e->w.ctr.p, sizeof(LevelCounters) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t err = 0;
    for (size_t L = 0; L < h.size(); ++L) {
      err |= h[L].error;
      add_stats(stats, h[L], L > 0);
    }
    if (h.back().next_tasks > e->levels_cap) err |= ERR_TASKS;  // more open tasks than the list holds
    if (err & ERR_SEGMENTS) return fail(DTSORT_EINVAL, "segment offsets are not valid");
    if (err) return fail(DTSORT_EINTERNAL, "device capacity check failed (flags " + std::to_string(err) + ")");
  }
  return 0;
}

// Checks the arguments of a sort call and fills J (all but the partner
// buffer).  Returns DTSORT_OK or an error status (message set); *noop is set
// when there is nothing to sort.
template <typename K, typename V>
static int prepare_job(K* keys, V* vals, size_t n, const uint64_t* seg, size_t n_seg, const dtsort_opts* opts,
                       SortJob<K, V>& J, bool* noop) {
  constexpr bool HV = HasVal<V>::value;
  *noop = false;
  dtsort_opts o;
  dtsort_default_opts(&o);
  if (opts) o = *opts;
  if (n >= (1ull << 32)) return fail(DTSORT_EINVAL, "n must be below 2^32");
  if (n > 0 && !keys) return fail(DTSORT_EINVAL, "keys is NULL");
  if (HV && n > 0 && !vals) return fail(DTSORT_EINVAL, "values is NULL");
  if (HV && n > 0) {
    const char* a0 = (const char*)keys;
    const char* a1 = a0 + n * sizeof(K);
    const char* b0 = (const char*)vals;
    const char* b1 = b0 + n * sizeof(V);
    if (a0 < b1 && b0 < a1) return fail(DTSORT_EINVAL, "keys and values overlap");
  }
  const int kbits = (int)(8 * sizeof(K));
  int key_bits = o.key_bits > 0 ? o.key_bits : kbits;
  if (key_bits > kbits) return fail(DTSORT_EINVAL, "key_bits larger than the key width");
  if (o.mode < 0 || o.mode > 2) return fail(DTSORT_EINVAL, "unknown mode");
  if (o.digit_bits < 0 || o.digit_bits > GMAX) return fail(DTSORT_EINVAL, "digit_bits out of range");
  if (o.digit_bits_below < 0 || o.digit_bits_below > GMAX)
    return fail(DTSORT_EINVAL, "digit_bits_below out of range");
  if (o.tile_shape < 0 || o.tile_shape > 6) return fail(DTSORT_EINVAL, "tile_shape out of range");
  if (o.merge_variant < MV_GATHER || o.merge_variant > MV_SPLIT) return fail(DTSORT_EINVAL, "unknown merge_variant");
  if (o.learned_judge < 0 || o.learned_judge > 1) return fail(DTSORT_EINVAL, "unknown learned_judge");
  if (o.graph && (o.mode == DTSORT_MODE_LEARNED || o.profile))
    return fail(DTSORT_EINVAL, "graph mode does not combine with LEARNED mode or profiling");
  if (seg && n_seg >= (1ull << 31)) return fail(DTSORT_EINVAL, "too many segments");
  if ((seg && n_seg == 0) || (!seg && n <= 1)) {
    *noop = true;
    return DTSORT_OK;
  }
  J.n = n;
  J.seg = seg;
  J.n_seg = (uint32_t)n_seg;
  J.key_bits = key_bits;
  J.o = o;
  J.bufs.k[0] = keys;
  if constexpr (HV) J.bufs.v[0] = vals;
  return DTSORT_OK;
}

// Points the partner halves of J's buffers into `ws` (keys, then values at
// the next 256-byte boundary; dtsort_workspace_bytes covers both).
template <typename K, typename V>
static void set_partner(SortJob<K, V>& J, char* ws) {
  J.bufs.k[1] = (K*)ws;
  if constexpr (HasVal<V>::value) J.bufs.v[1] = (V*)(ws + ((J.n * sizeof(K) + 255) & ~(size_t)255));
}

template <typename K, typename V>
static int sort_entry(K* keys, V* vals, size_t n, const uint64_t* seg, size_t n_seg, const dtsort_opts* opts,
                      void* stream) {
  constexpr bool HV = HasVal<V>::value;
  g_err.clear();
  SortJob<K, V> J;
  bool noop = false;
  int r;
  if ((r = prepare_job(keys, vals, n, seg, n_seg, opts, J, &noop)) || noop) return r;
  const dtsort_opts& o = J.o;
  hipStream_t s = (hipStream_t)stream;
  Ctx* c;
  if ((r = get_ctx(s, &c))) return r;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->has_last && c->last_stream != s) HIPCHK(hipStreamWaitEvent(s, c->done, 0));
  // ping-pong partner
  const size_t need = dtsort_workspace_bytes((int)sizeof(K), HV ? (int)sizeof(V) : 0, n);
  char* ws = nullptr;
  if (o.workspace) {
    if (o.workspace_bytes < need) return fail(DTSORT_EWORKSPACE, "workspace smaller than dtsort_workspace_bytes()");
    ws = (char*)o.workspace;
  }
  if (o.graph) {
    if (ws) set_partner(J, ws);
    r = graph_sort<K, V>(c, J, ws, s, o.stats);
  } else {
    if (!ws) {
      if ((r = ensure(c->w.tk, need, s))) return r;
      ws = (char*)c->w.tk.p;
    }
    set_partner(J, ws);
    r = run_sort<K, V>(c, J, s, o.stats);
  }
  if (hipEventRecord(c->done, s) == hipSuccess) {
    c->has_last = true;
    c->last_stream = s;
  }
  return r;
}

// ------------------------------------------- allocation-free entry point
// Device memory of dtsort_segmented_noalloc: every buffer of its schedule,
// and the ping-pong partner unless the caller passes a workspace, is carved
// from this one array.  Each device the library runs on holds its own copy
// until the process ends.  In host code the array's name is not a device
// address: the address is looked up once per device (hipGetSymbolAddress)
// and only that address is handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[MAX_DEVICES];  // device address of `scratch`, per device

static int scratch_of_current_device(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DTSORT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DTSORT_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[dev] = p;
  }
  *out = (char*)g_scratch[dev];
  return 0;
}

// The graph-form schedule (kernels only, no host read-back) enqueued
// directly on `stream`, with every buffer placed in the scratch array: no
// device or pinned allocation, no synchronisation.
template <typename K, typename V>
static int noalloc_entry(K* keys, V* vals, size_t n, const uint64_t* seg, size_t n_seg, const dtsort_opts* opts,
                         void* stream) {
  constexpr bool HV = HasVal<V>::value;
  g_err.clear();
  SortJob<K, V> J;
  bool noop = false;
  int r;
  if ((r = prepare_job(keys, vals, n, seg, n_seg, opts, J, &noop)) || noop) return r;
  const dtsort_opts& o = J.o;
  if (o.mode == DTSORT_MODE_LEARNED) return fail(DTSORT_EINVAL, "LEARNED mode is not available without allocation");
  if (o.stats || o.profile) return fail(DTSORT_EINVAL, "stats and profiling read results back; not available here");
  const Params P = resolve_params(J);
  const GPlan g = graph_plan(J, P);
  const size_t part = o.workspace ? 0 : dtsort_workspace_bytes((int)sizeof(K), HV ? (int)sizeof(V) : 0, n);
  if (o.workspace && o.workspace_bytes < dtsort_workspace_bytes((int)sizeof(K), HV ? (int)sizeof(V) : 0, n))
    return fail(DTSORT_EWORKSPACE, "workspace smaller than dtsort_workspace_bytes()");
  // every buffer at a 256-byte boundary of the scratch array
  auto rounded = [](size_t bytes) { return (std::max<size_t>(bytes, 64) + 255) & ~(size_t)255; };
  Work W;
  size_t need = part ? rounded(part) : 0;
  (void)graph_buffers(W, g, [&](DevBuf&, size_t bytes) {
    need += rounded(bytes);
    return 0;
  });
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(DTSORT_EINVAL, "input too large for the allocation-free entry point: it needs " +
                                   std::to_string(need) + " bytes of scratch, the limit is " +
                                   std::to_string(NOALLOC_SCRATCH_BYTES) +
                                   (part ? " (a caller workspace for the partner buffer lowers the need)" : ""));
  char* base = nullptr;
  if ((r = scratch_of_current_device(&base))) return r;
  size_t off = 0;
  auto place = [&](DevBuf& b, size_t bytes) {
    b.p = base + off;
    b.cap = rounded(bytes);
    off += b.cap;
    return 0;
  };
  if (part) {
    DevBuf pb;
    place(pb, part);
    set_partner(J, (char*)pb.p);
  } else {
    set_partner(J, (char*)o.workspace);
  }
  (void)graph_buffers(W, g, place);
  hipStream_t s = (hipStream_t)stream;
  graph_enqueue<K, V>(W, g, J, P, s);
  HIPCHK(hipGetLastError());
  return DTSORT_OK;
}

}  // namespace dts

using namespace dts;

extern "C" {

void dtsort_default_opts(dtsort_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mode = DTSORT_MODE_SAMPLING;
}

size_t dtsort_workspace_bytes(int key_bytes, int val_bytes, size_t n) {
  const size_t kb = ((size_t)key_bytes * n + 255) & ~(size_t)255;
  const size_t vb = ((size_t)val_bytes * n + 255) & ~(size_t)255;
  return kb + vb + 256;
}

int dtsort_u32(uint32_t* keys, size_t n, const dtsort_opts* opts, void* stream) {
  return sort_entry<uint32_t, NoVal>(keys, (NoVal*)nullptr, n, nullptr, 0, opts, stream);
}

int dtsort_u64(uint64_t* keys, size_t n, const dtsort_opts* opts, void* stream) {
  return sort_entry<uint64_t, NoVal>(keys, (NoVal*)nullptr, n, nullptr, 0, opts, stream);
}

int dtsort_pairs_u64(uint64_t* keys, uint64_t* values, size_t n, const dtsort_opts* opts, void* stream) {
  return sort_entry<uint64_t, uint64_t>(keys, values, n, nullptr, 0, opts, stream);
}

int dtsort_pairs_u32(uint32_t* keys, uint32_t* values, size_t n, const dtsort_opts* opts, void* stream) {
  return sort_entry<uint32_t, uint32_t>(keys, values, n, nullptr, 0, opts, stream);
}

int dtsort_segmented(uint32_t* keys, uint32_t* values, size_t n_total, const uint64_t* seg_offsets, size_t n_segments,
                     const dtsort_opts* opts, void* stream) {
  if (!seg_offsets && n_segments > 0) return fail(DTSORT_EINVAL, "seg_offsets is NULL");
  if (values) return sort_entry<uint32_t, uint32_t>(keys, values, n_total, seg_offsets, n_segments, opts, stream);
  return sort_entry<uint32_t, NoVal>(keys, (NoVal*)nullptr, n_total, seg_offsets, n_segments, opts, stream);
}

int dtsort_segmented_noalloc(uint32_t* keys, uint32_t* values, size_t n_total, const uint64_t* seg_offsets,
                              size_t n_segments, const dtsort_opts* opts, void* stream) {
  if (!seg_offsets && n_segments > 0) return fail(DTSORT_EINVAL, "seg_offsets is NULL");
  if (values) return noalloc_entry<uint32_t, uint32_t>(keys, values, n_total, seg_offsets, n_segments, opts, stream);
  return noalloc_entry<uint32_t, NoVal>(keys, (NoVal*)nullptr, n_total, seg_offsets, n_segments, opts, stream);
}

int dtsort_graph_transpose(const uint64_t* offsets, const uint32_t* targets, uint32_t n_vertices, size_t n_edges,
                           uint64_t* t_offsets, uint32_t* t_targets, const dtsort_opts* opts, void* stream) {
  g_err.clear();
  if (!offsets || !t_offsets) return fail(DTSORT_EINVAL, "offsets is NULL");
  if (n_edges > 0 && (!targets || !t_targets)) return fail(DTSORT_EINVAL, "targets is NULL");
  if (n_edges >= (1ull << 32)) return fail(DTSORT_EINVAL, "n_edges must be below 2^32");
  if (n_vertices == 0xFFFFFFFFu) return fail(DTSORT_EINVAL, "n_vertices must be below 2^32 - 1");
  if (opts && (opts->graph || opts->mode == DTSORT_MODE_LEARNED))
    return fail(DTSORT_EINVAL, "the transpose runs the eager sort (no graph form, no LEARNED mode)");
  hipStream_t s = (hipStream_t)stream;
  Ctx* c;
  int r;
  if ((r = get_ctx(s, &c))) return r;
  std::lock_guard<std::mutex> lk(c->app_mu);
  if (!c->h_app && hipHostMalloc((void**)&c->h_app, 64) != hipSuccess) {
    (void)hipGetLastError();
    c->h_app = nullptr;
    return fail(DTSORT_ENOMEM, "pinned host allocation failed");
  }
  const size_t kb = (4 * n_edges + 255) & ~(size_t)255;
  if ((r = ensure(c->app_keys, kb + 256, s))) return r;
  uint32_t* keys = (uint32_t*)c->app_keys.p;
  uint32_t* err = (uint32_t*)((char*)c->app_keys.p + kb);
  launch_zero_counters((LevelCounters*)err, 1, s);  // clears the error word (and the rest of one counter block)
  launch_transpose_prepare(offsets, targets, n_vertices, n_edges, keys, t_targets, err, s);
  HIPCHK(hipGetLastError());
  // the stable sort of the edges by target; values = sources
  if ((r = sort_entry<uint32_t, uint32_t>(keys, t_targets, n_edges, nullptr, 0, opts, stream))) return r;
  launch_transpose_offsets(keys, n_edges, n_vertices, t_offsets, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_app, err, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (*c->h_app & 1u) return fail(DTSORT_EINVAL, "offsets are not a valid CSR offsets array");
  if (*c->h_app & 2u) return fail(DTSORT_EINVAL, "a target is not below n_vertices");
  return DTSORT_OK;
}

int dtsort_morton_u32(const uint32_t* coords, int dims, size_t n, uint32_t* codes, uint32_t* perm,
                      const dtsort_opts* opts, void* stream) {
  g_err.clear();
  if (dims != 2 && dims != 3) return fail(DTSORT_EINVAL, "dims must be 2 or 3");
  if (n >= (1ull << 32)) return fail(DTSORT_EINVAL, "n must be below 2^32");
  if (n > 0 && (!coords || !codes || !perm)) return fail(DTSORT_EINVAL, "NULL pointer");
  if (n == 0) return DTSORT_OK;
  hipStream_t s = (hipStream_t)stream;
  launch_morton(coords, dims, n, codes, perm, s);
  HIPCHK(hipGetLastError());
  return sort_entry<uint32_t, uint32_t>(codes, perm, n, nullptr, 0, opts, stream);
}

int dtsort_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, void* stream) {
  g_err.clear();
  if (n == 0) return DTSORT_OK;
  if (!dst || !src) return fail(DTSORT_EINVAL, "NULL pointer");
  if (n >= (1ull << 32)) return fail(DTSORT_EINVAL, "n must be below 2^32");
  if ((const char*)dst < (const char*)(src + n) && (const char*)src < (const char*)(dst + n))
    return fail(DTSORT_EINVAL, "src and dst overlap");
  hipStream_t s = (hipStream_t)stream;
  Ctx* c;
  int r;
  if ((r = get_ctx(s, &c))) return r;
  std::lock_guard<std::mutex> lk(c->mu);
  // items written on the device, cut as the sorts cut their copies
  const uint32_t items = pieces_of((uint32_t)n);
  if ((r = ensure(c->copy_items, sizeof(Leaf) * (size_t)items + 64, s))) return r;
  Leaf* d_items = (Leaf*)c->copy_items.p;
  uint32_t* d_count = (uint32_t*)((char*)c->copy_items.p + sizeof(Leaf) * (size_t)items);
  launch_copy_items(d_items, d_count, n, s);
  Bufs<uint32_t, NoVal> b;
  b.k[0] = const_cast<uint32_t*>(src);
  b.k[1] = dst;
  launch_copy<uint32_t, NoVal>(d_items, d_count, items, items, b, s);
  HIPCHK(hipGetLastError());
  return DTSORT_OK;
}

static void free_ctx(Ctx* c) {
  free_work(c->w);
  free_buf(c->lrn);
  free_buf(c->copy_items);
  free_buf(c->app_keys);
  if (c->h_app) (void)hipHostFree(c->h_app);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (GraphEntry* e : c->graphs) free_graph(e);
  c->graphs.clear();
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->cap_stream2) (void)hipStreamDestroy(c->cap_stream2);
  if (c->side) (void)hipStreamDestroy(c->side);
  for (hipEvent_t ev : c->side_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->fork_events)
    if (ev) (void)hipEventDestroy(ev);
  if (c->inner) free_ctx(c->inner);
  if (c->h_ctr) (void)hipHostFree(c->h_ctr);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->done) (void)hipEventDestroy(c->done);
  delete c;
}

void dtsort_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (size_t d = 0; d < g_ctx.size(); ++d) {
    if (g_ctx[d].empty()) continue;
    (void)hipSetDevice((int)d);
    (void)hipDeviceSynchronize();
    for (Ctx* c : g_ctx[d]) free_ctx(c);
  }
  (void)hipSetDevice(cur);
  (void)hipGetLastError();
  g_ctx.clear();
}

const char* dtsort_last_error(void) { return g_err.c_str(); }

const char* dtsort_strerror(int st) {
  switch (st) {
    case DTSORT_OK: return "ok";
    case DTSORT_EINVAL: return "invalid argument";
    case DTSORT_ENOMEM: return "out of device memory";
    case DTSORT_EWORKSPACE: return "workspace too small";
    case DTSORT_EHIP: return "HIP runtime error";
    case DTSORT_EINTERNAL: return "internal capacity or consistency check failed";
    default: return "unknown status";
  }
}

}  // extern "C"

// Host runtime of libtrioseq: validation, 2-bit packing, planning (axis
// choice, longest-first ordering, workspace sizing), launches, hipGraph
// replay, and the synchronous single/batch entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "common.h"

namespace trioseq {

static thread_local std::string g_err;

trioseq_status fail(trioseq_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

trioseq_status fail_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(TRIOSEQ_ERR_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
  return fail(TRIOSEQ_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static const uint8_t* build_code_table() {
  static uint8_t t[256];
  std::memset(t, 255, sizeof t);
  const char* up = "ACGT";
  const char* lo = "acgt";
  for (int c = 0; c < 4; ++c) {
    t[(uint8_t)up[c]] = (uint8_t)c;
    t[(uint8_t)lo[c]] = (uint8_t)c;
  }
  return t;
}
static const uint8_t* g_code = build_code_table();

uint8_t residue_code(char ch) { return g_code[(uint8_t)ch]; }

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

trioseq_status validate_scoring(const trioseq_scoring* sc) {
  if (!sc) return fail(TRIOSEQ_ERR_INVALID_ARG, "scoring is NULL");
  if (sc->kind != kGlobal && sc->kind != kSemiGlobal && sc->kind != kLocal)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "scoring kind must be global, semi-global or local");
  // The semi-global and local kernels rely on M' = M - 2*gap*(i+j+k) >= 0
  // for their axis values and floors.
  if (sc->kind != kGlobal && sc->gap > 0)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "semi-global and local scoring need gap <= 0");
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) {
      if (sc->sub[x][y] != sc->sub[y][x])
        return fail(TRIOSEQ_ERR_INVALID_ARG, "substitution matrix is not symmetric");
      const int64_t term = (int64_t)sc->sub[x][y] - 2 * (int64_t)sc->gap;
      if (term < -127 || term > 127)
        return fail(TRIOSEQ_ERR_INVALID_ARG,
                    "sub[x][y] - 2*gap must lie in [-127, 127] for every pair");
    }
  return TRIOSEQ_OK;
}

trioseq_status check_range(const trioseq_scoring& sc, uint64_t a, uint64_t b, uint64_t c,
                           size_t index) {
  const uint64_t d = a + b + c;
  int64_t maxterm = 0;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y)
      maxterm = std::max<int64_t>(maxterm, (int64_t)sc.sub[x][y] - 2 * (int64_t)sc.gap);
  // Shifted scores lie in [0, d * maxterm]; the true score adds 2*gap*d.
  // Semi-global axes and local floors put cells at M' = -2*gap*(i+j+k).
  if (sc.kind != kGlobal) maxterm = std::max<int64_t>(maxterm, -2 * (int64_t)sc.gap);
  const long double hi = (long double)d * (long double)maxterm;
  const long double shift = (long double)d * 2.0L * (long double)sc.gap;
  if (hi >= (long double)(1 << 27) || shift >= (long double)(1 << 30) ||
      shift <= -(long double)(1 << 30))
    return fail(TRIOSEQ_ERR_OVERFLOW,
                "triplet " + std::to_string(index) + ": score range exceeds int32 headroom");
  return TRIOSEQ_OK;
}

DevScoring make_dev_scoring(const trioseq_scoring& sc) {
  DevScoring d;
  for (int r = 0; r < 4; ++r) {
    uint32_t w = 0;
    for (int x = 0; x < 4; ++x) {
      const int v = sc.sub[x][r] - 2 * sc.gap;
      w |= (uint32_t)(uint8_t)(int8_t)v << (8 * x);
    }
    d.byte_tab[r] = w;
  }
  d.byte_tab[4] = 0x80808080u;
  for (int r = 0; r < 4; ++r)
    for (int s = 0; s < 4; ++s) d.pair_tab[4 * r + s] = sc.sub[r][s] - 2 * sc.gap;
  d.gap2 = 2 * sc.gap;
  d.kind = sc.kind;
  return d;
}

// When the plan picks engines itself, a triplet is split into panel jobs if
// sweeping it whole on one wavefront would hold the launch up: it is alone,
// it has at least kSplitCells cells (one wave takes ~0.1 s on 2.5e8 cells),
// or more than kSplitFactor times the batch's mean cells per wavefront.
const double kSplitCells = 2.5e8;
const double kSplitFactor = 4.0;

uint64_t panel_steps(const uint32_t l[3], const KernelShape& ks) {
  const uint64_t pj = l[1] / (uint32_t)panel_rows(ks) + 1;
  const uint64_t pk = l[2] / (uint32_t)panel_cols(ks) + 1;
  return pj * pk * (uint64_t)(l[0] + 1 + kSkew);
}

static const uint8_t kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

AxisChoice choose_axes_batch(const uint32_t len[3], const KernelShape& ks) {
  AxisChoice best{{0, 1, 2}};
  uint64_t best_cost = UINT64_MAX;
  for (const auto& p : kPerms) {
    const uint32_t l[3] = {len[p[0]], len[p[1]], len[p[2]]};
    if (l[0] > (uint32_t)kMaxSweepLen) continue;
    const uint64_t cost = panel_steps(l, ks);
    if (cost < best_cost) {
      best_cost = cost;
      std::memcpy(best.perm, p, 3);
    }
  }
  return best;
}

AxisChoice choose_axes_wide(const uint32_t len[3]) {
  // Sweep the longest sequence that fits the LDS residue buffer: the fill of
  // the panel pipeline is paid once per sweep, so a long sweep amortises it.
  AxisChoice best{{0, 1, 2}};
  int64_t best_len = -1;
  for (const auto& p : kPerms) {
    if (len[p[0]] > (uint32_t)kMaxSweepLen) continue;
    const int64_t key = (int64_t)len[p[0]] * 4 + (len[p[1]] >= len[p[2]] ? 1 : 0);
    if (key > best_len) {
      best_len = key;
      std::memcpy(best.perm, p, 3);
    }
  }
  return best;
}

uint64_t boundary_ints(const KernelShape& ks, uint32_t max_n0) {
  const uint64_t rows = face_rows(max_n0);
  return 3 * (2 * rows * panel_cols(ks) + rows * right_face_row(ks));  // plain + tagged
}

Boundary carve_boundary(const KernelShape& ks, uint32_t max_n0, int* q) {
  const uint64_t rows = face_rows(max_n0);
  const uint64_t top = rows * panel_cols(ks), left = rows * right_face_row(ks);
  Boundary b;
  b.plain[0] = q;
  b.plain[1] = q + top;
  b.plain[2] = q + 2 * top;
  q += 2 * top + left;
  b.tagged[0] = q;
  b.tagged[1] = q + 2 * top;
  b.tagged[2] = q + 4 * top;
  b.rows = (uint32_t)rows;
  return b;
}

SweepArgs make_sweep_args(const uint32_t* words, const TripletDesc* desc, const JobDesc* jobs,
                          uint32_t njobs, uint32_t lds_n0, int32_t* scores, int* counter, int* ctl,
                          int* face, uint64_t face_stride, int* pface, const Boundary& bnd,
                          int* red, const DevScoring& sc) {
  SweepArgs a;
  a.words = words;
  a.desc = desc;
  a.jobs = jobs;
  a.njobs = njobs;
  a.lds_n0 = lds_n0;
  a.scores = scores;
  a.counter = counter;
  a.ctl = ctl;
  a.face = face;
  a.face_stride = face_stride;
  a.pface = pface;
  for (int k = 0; k < 3; ++k) {
    a.bnd_plain[k] = bnd.plain[k];
    a.bnd_tagged[k] = bnd.tagged[k];
  }
  a.red = red;
  a.plane = nullptr;
  a.plane_off = nullptr;
  a.wait_ticks = wait_limit_ticks();
  a.sc = sc;
  return a;
}

// 2 s in ticks of the 100 MHz wall clock the kernels read.
constexpr uint64_t kDefaultWaitTicks = 200000000ull;
static std::atomic<uint64_t> g_wait_ticks{kDefaultWaitTicks};

uint64_t wait_limit_ticks() { return g_wait_ticks.load(std::memory_order_relaxed); }

// A private non-blocking stream per thread and device for the one-off work
// of plan creation (clearing control words and face pools, uploading the job
// tables, writing sentinel faces). Waiting for it stalls nothing else: no
// caller stream and no other thread's work is synchronised. Never destroyed
// (the HIP runtime may be gone at thread exit).
hipError_t init_stream(int device, hipStream_t* out) {
  static thread_local std::vector<hipStream_t>* streams = nullptr;
  if (!streams) streams = new std::vector<hipStream_t>;
  if ((int)streams->size() <= device) streams->resize(device + 1, nullptr);
  hipStream_t& st = (*streams)[device];
  if (!st) {
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      st = nullptr;
      return e;
    }
  }
  *out = st;
  return hipSuccess;
}

trioseq_status device_props(DeviceProps* p) {
  TRIOSEQ_HIP(hipGetDevice(&p->device), "hipGetDevice");
  TRIOSEQ_HIP(hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device),
              "hipDeviceGetAttribute");
  size_t fr = 0, tot = 0;
  TRIOSEQ_HIP(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
  p->hbm_bytes = tot;
  return TRIOSEQ_OK;
}

}  // namespace trioseq

using namespace trioseq;

struct trioseq_plan {
  int device = 0;
  size_t n = 0;
  int engine = 0;  // 0: all triplets whole, 1: all split into panel jobs, 2: mixed
  int modes = 1;   // kernel variant: bit 0 whole-triplet jobs, bit 1 panel jobs
  KernelShape ks{4, 4, 4};
  int grid = 0, waves_per_cu = 0, panels = 0;
  uint32_t njobs = 0, lds_n0 = 0;
  DevScoring sc{};
  double cells = 0;
  uint64_t workspace_bytes = 0;
  TripletDesc* d_desc = nullptr;
  JobDesc* d_jobs = nullptr;
  int* d_counter = nullptr;  // job queue head
  int* d_ctl = nullptr;      // [0] generation, [1] error flag, [2] meeting counter (0 between runs)
  int* d_face = nullptr;     // per-wave workspace of whole-triplet jobs
  uint64_t face_stride = 0;
  int* d_pface = nullptr;    // panel-face pool of split triplets
  int* d_bnd = nullptr;      // sentinel faces
  Boundary bnd{};
  int* d_red = nullptr;      // per-triplet reduction pairs (semi-global, local)
  uint32_t red_pairs = 0;
  // Half-split scoring of a lone triplet (see half_split_layout).
  bool half = false;
  uint32_t h_words_n = 0, h_nchunk = 0;
  uint32_t* d_hwords = nullptr;     // the two halves' sequences, gathered every run
  GatherDesc* d_gather = nullptr;   // 6 gather descriptors
  int* d_plane = nullptr;           // the two last-slice planes
  uint64_t* d_plane_off = nullptr;  // {0, plane ints}
  SplitDesc* d_sdesc = nullptr;     // the meeting box
  int* d_partial = nullptr;         // per chunk: its best
  int32_t* d_hscores = nullptr;     // the halves' own scores (unused)
  // graph replay
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const uint32_t* g_words = nullptr;
  int32_t* g_scores = nullptr;
  // Device buffers carved from a caller's region (not owned).
  bool borrowed = false;
  // Packed pairs: sentinel faces (top, left) and the stored value of M' = 0.
  bool packed = false;
  uint32_t pk_base = 0, pk_kc = 0;
  int* d_pkbnd = nullptr;
  uint64_t pk_top_words = 0;
};

static void plan_free(trioseq_plan* p) {
  if (!p) return;
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->borrowed) {
    // Carved from a caller's region: nothing to free on the device.
    delete p;
    return;
  }
  (void)hipFree(p->d_desc);
  (void)hipFree(p->d_jobs);
  (void)hipFree(p->d_counter);
  (void)hipFree(p->d_ctl);
  (void)hipFree(p->d_face);
  (void)hipFree(p->d_pface);
  (void)hipFree(p->d_bnd);
  (void)hipFree(p->d_red);
  (void)hipFree(p->d_pkbnd);
  for (void* q : {(void*)p->d_hwords, (void*)p->d_gather, (void*)p->d_plane, (void*)p->d_plane_off,
                  (void*)p->d_sdesc, (void*)p->d_partial, (void*)p->d_hscores})
    (void)hipFree(q);
  delete p;
}

extern "C" {

void trioseq_scoring_simple(trioseq_scoring* s, int32_t match, int32_t mismatch, int32_t gap) {
  if (!s) return;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) s->sub[x][y] = x == y ? match : mismatch;
  s->gap = gap;
  s->kind = TRIOSEQ_GLOBAL;
}

const char* trioseq_last_error(void) { return g_err.c_str(); }

const char* trioseq_version(void) { return "trioseq-mi355x 0.2 (gfx950)"; }

void trioseq_set_wait_limit(uint64_t ns) {
  g_wait_ticks.store(ns ? ns / 10 : kDefaultWaitTicks, std::memory_order_relaxed);
}

trioseq_status trioseq_pack(const char* seq, uint32_t len, uint32_t* words) {
  if (len && (!seq || !words)) return fail(TRIOSEQ_ERR_INVALID_ARG, "pack: NULL pointer");
  const uint8_t* in = (const uint8_t*)seq;
  // Validate first (codes of A, C, G, T are 0..3, anything else has a
  // higher bit set), so an error leaves the words untouched.
  uint32_t bad = 0;
  for (uint32_t p = 0; p < len; ++p) bad |= g_code[in[p]];
  if (bad > 3) {
    uint32_t p = 0;
    while (g_code[in[p]] <= 3) ++p;
    return fail(TRIOSEQ_ERR_BAD_RESIDUE, "pack: character at position " + std::to_string(p) + " is not ACGT");
  }
  const uint32_t full = len / 16;
  for (uint32_t w = 0; w < full; ++w) {
    const uint8_t* r = in + 16 * (size_t)w;
    uint32_t v = 0;
    for (int q = 0; q < 16; ++q) v |= (uint32_t)g_code[r[q]] << (2 * q);
    words[w] = v;
  }
  if (len % 16) {
    uint32_t v = 0;
    for (uint32_t q = 0; q < len % 16; ++q) v |= (uint32_t)g_code[in[16 * (size_t)full + q]] << (2 * q);
    words[full] = v;
  }
  return TRIOSEQ_OK;
}

trioseq_status trioseq_packed_layout(const uint32_t* lens, size_t n, uint64_t* word_off,
                                     uint64_t* total_words) {
  if ((n && (!lens || !word_off)) || !total_words)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "packed_layout: NULL pointer");
  uint64_t acc = 0;
  for (size_t q = 0; q < 3 * n; ++q) {
    word_off[q] = acc;
    acc += (lens[q] + 15u) / 16u;
  }
  *total_words = acc;
  return TRIOSEQ_OK;
}

}  // extern "C"

namespace trioseq {

// Packed pairs (two triplets per lane, one 16-bit half each): the batch's
// whole triplets, sorted by their axis lengths, are paired neighbour with
// neighbour (a lone last one with itself) and each pair is one job over the
// common panel grid. Qualifies when the scoring is global, every
// substitution term sub - 2*gap is >= 0, and every value a lane can hold
// stays within [kPackedSentinel, kPackedMax]: values outside the tensor
// start at kPackedSentinel and grow by at most maxA per residue along the
// fill region (kSkew slices plus the padded panel box), M' = 0 is stored as
// base above all of them, and base + maxA * (the longest path of the padded
// box, drain included) must not pass kPackedMax.
static bool pair_up(Layout* L, const trioseq_scoring& sc, const KernelShape& ks) {
  const size_t n = L->desc.size();
  if (L->modes != 1 || L->planes || n < 2) return false;
  int mina = INT32_MAX, maxa = INT32_MIN;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) {
      mina = std::min(mina, sc.sub[x][y] - 2 * sc.gap);
      maxa = std::max(maxa, sc.sub[x][y] - 2 * sc.gap);
    }
  if (mina < 0 || maxa > 255 || !pk_shape_supported(ks, sc.kind)) return false;
  const int H = panel_rows(ks), W = panel_cols(ks), RR = (int)right_face_row(ks);
  const size_t np = (n + 1) / 2;
  // A pair costs the panels of its common grid times its steps. Neighbours
  // in two sort orders are paired, and the cheaper pairing is kept: by the
  // lengths (similar sweep lengths), or by the panel counts of the other two
  // axes first (no pair crosses a panel boundary the two do not share).
  auto pair_cost = [&](const TripletDesc& a, const TripletDesc& b) {
    const uint64_t n0 = std::max(a.len[0], b.len[0]);
    const uint64_t PJ = std::max(a.len[1], b.len[1]) / H + 1, PK = std::max(a.len[2], b.len[2]) / W + 1;
    return PJ * PK * (n0 + 1 + kSkew);
  };
  auto total_cost = [&](const std::vector<size_t>& v) {
    uint64_t c = 0;
    for (size_t q = 0; q < np; ++q) c += pair_cost(L->desc[v[2 * q]], L->desc[v[std::min(2 * q + 1, n - 1)]]);
    return c;
  };
  std::vector<size_t> idx(n), idx2(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::iota(idx2.begin(), idx2.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    const TripletDesc &da = L->desc[a], &db = L->desc[b];
    return std::make_tuple(da.len[0], da.len[1], da.len[2]) < std::make_tuple(db.len[0], db.len[1], db.len[2]);
  });
  std::stable_sort(idx2.begin(), idx2.end(), [&](size_t a, size_t b) {
    const TripletDesc &da = L->desc[a], &db = L->desc[b];
    return std::make_tuple(da.len[1] / H, da.len[2] / W, da.len[0], da.len[1], da.len[2]) <
           std::make_tuple(db.len[1] / H, db.len[2] / W, db.len[0], db.len[1], db.len[2]);
  });
  if (total_cost(idx2) < total_cost(idx)) idx.swap(idx2);
  uint64_t box_jk = 0, n0max = 0, stride = 0;
  std::vector<uint64_t> cost(np);
  for (size_t q = 0; q < np; ++q) {
    const TripletDesc& a = L->desc[idx[2 * q]];
    const TripletDesc& b = L->desc[idx[std::min(2 * q + 1, n - 1)]];
    const uint32_t n0 = std::max(a.len[0], b.len[0]), n1 = std::max(a.len[1], b.len[1]),
                   n2 = std::max(a.len[2], b.len[2]);
    const uint64_t PJ = n1 / H + 1, PK = n2 / W + 1, rows = face_rows(n0);
    box_jk = std::max(box_jk, PJ * H + PK * W);
    n0max = std::max<uint64_t>(n0max, n0);
    stride = std::max(stride, rows * (PK * W + RR));
    cost[q] = pair_cost(a, b);
  }
  // Real values: base + M' with M' <= mx per unit of index sum (a move adds
  // at most one term per residue it consumes; the local floor and the
  // semi-global axes add g = -2*gap per unit), over the padded box and the
  // drain steps. Semi-global candidates M + kc need kc above g times every
  // index sum and must stay within 16 bits (see sweep.hip).
  const uint64_t g = sc.kind == kGlobal ? 0 : (uint64_t)(-2 * sc.gap);  // gap <= 0 for the others
  const uint64_t mx = sc.kind == kGlobal ? (uint64_t)maxa : std::max<uint64_t>(maxa, g);
  const uint64_t base = kPackedSentinel + 512 + (uint64_t)maxa * (kSkew + box_jk);
  if (base + mx * (n0max + kSkew + kChunk + box_jk) > kPackedMax) return false;
  uint64_t kc = 0;
  if (sc.kind == kSemiGlobal) {
    kc = g * (n0max + box_jk) + 1;
    if (kPackedMax - base + kc > 0xFFFF) return false;
  }
  std::vector<TripletDesc> desc(2 * np);
  for (size_t q = 0; q < np; ++q) {
    desc[2 * q] = L->desc[idx[2 * q]];
    desc[2 * q + 1] = L->desc[idx[std::min(2 * q + 1, n - 1)]];
  }
  std::vector<size_t> order(np);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  L->jobs.clear();
  for (size_t q : order) L->jobs.push_back(JobDesc{(uint32_t)(2 * q), kWholeTriplet});
  L->desc.swap(desc);
  L->ks = ks;
  L->packed = true;
  L->pk_base = (uint32_t)base;
  L->pk_kc = (uint32_t)kc;
  L->face_stride = (stride + 63) / 64 * 64;
  L->lds_n0 = (uint32_t)n0max;
  return true;
}

trioseq_status build_layout(const uint32_t* lens, const uint64_t* off, size_t n,
                            const trioseq_scoring& sc, const trioseq_plan_options& o, int waves_hint,
                            Layout* L, bool planes) {
  if (n && !lens) return fail(TRIOSEQ_ERR_INVALID_ARG, "lens is NULL");
  if (n > (size_t)INT32_MAX) return fail(TRIOSEQ_ERR_TOO_LARGE, "too many triplets");
  trioseq_status st = validate_scoring(&sc);
  if (st != TRIOSEQ_OK) return st;
  if (o.engine < -1 || o.engine > 1) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: bad engine");
  if (o.grid < 0) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: negative grid");
  if (o.split_factor < 0) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: negative split_factor");
  if (o.half_split_min < -1) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: bad half_split_min");
  if (o.packed < 0 || o.packed > 2) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: packed must be 0, 1 or 2");
  if (o.staging < 0 || o.staging > 2) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: staging must be 0, 1 or 2");
  if (o.panel_group != 0 && o.panel_group != 1 && o.panel_group != 4)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: panel_group must be 0, 1 or 4");
  static_assert(kStripPanels == 4, "panel_group option values");
  KernelShape ks{o.tile_rows ? o.tile_rows : 4, o.tile_cols ? o.tile_cols : 4,
                 o.waves_per_simd ? o.waves_per_simd : 2};
  ks.group = o.panel_group ? o.panel_group : kDefaultPanelGroup;
  if (o.lane_exchange < 0 || o.lane_exchange > 2)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: lane_exchange must be 0, 1 or 2");
  ks.xch = o.lane_exchange ? o.lane_exchange - 1 : kDefaultLaneExchange;
  // A shape only the packed kernels have is accepted when packing is asked
  // for; the batch must then qualify for it (checked at the end).
  const bool int32_shape = shape_supported(ks, sc.kind);
  KernelShape pks = ks;
  pks.dma = o.staging == 2 ? 1 : 0;
  if (!int32_shape && !(o.packed == 2 && pk_shape_supported(pks, sc.kind)))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: unsupported tile shape for this scoring kind");
  std::vector<uint64_t> offs;
  if (!off) {
    offs.resize(3 * n);
    uint64_t tw = 0;
    trioseq_packed_layout(lens, n, offs.data(), &tw);
    off = offs.data();
  }
  double cells = 0;
  for (size_t t = 0; t < n; ++t) {
    const uint32_t* l = lens + 3 * t;
    if (std::min({l[0], l[1], l[2]}) > (uint32_t)kMaxSweepLen)
      return fail(TRIOSEQ_ERR_TOO_LARGE, "triplet " + std::to_string(t) +
                                             ": every sequence exceeds " +
                                             std::to_string(kMaxSweepLen) + " residues");
    if (planes && l[0] > (uint32_t)kMaxSweepLen)
      return fail(TRIOSEQ_ERR_TOO_LARGE, "triplet " + std::to_string(t) + ": sweep sequence exceeds " +
                                             std::to_string(kMaxSweepLen) + " residues");
    st = check_range(sc, l[0], l[1], l[2], t);
    if (st != TRIOSEQ_OK) return st;
    cells += (double)l[0] * (double)l[1] * (double)l[2];
  }
  const int H = panel_rows(ks), W = panel_cols(ks), RR = (int)right_face_row(ks);

  // Which triplets are split into panel jobs: forced by the engine option,
  // else by the rule at kSplitCells.
  const double per_wave = cells / std::max(1, waves_hint);
  L->desc.assign(n, TripletDesc{});
  std::vector<char> split(n, 0);
  std::vector<uint64_t> cost(n, 0);
  uint64_t stride = 0, pool = 0;
  uint32_t max_n0 = 0;
  int n_split = 0, panels = 0;
  for (size_t t = 0; t < n; ++t) {
    const uint32_t* l = lens + 3 * t;
    const double c = (double)l[0] * l[1] * l[2];
    const double factor = o.split_factor > 0 ? (double)o.split_factor : kSplitFactor;
    const bool sp = o.engine == 1 ||
                    (o.engine == -1 && (n == 1 || c >= kSplitCells || c > factor * per_wave));
    // Plane runs keep the caller's axes: the plane is the last slice of S0.
    AxisChoice ax = planes ? AxisChoice{{0, 1, 2}} : sp ? choose_axes_wide(l) : choose_axes_batch(l, ks);
    TripletDesc& d = L->desc[t];
    for (int a = 0; a < 3; ++a) {
      d.off[a] = off[3 * t + ax.perm[a]];
      d.len[a] = l[ax.perm[a]];
    }
    d.out = (uint32_t)t;
    d.face_off = 0;
    const uint64_t rows = face_rows(d.len[0]);
    const uint64_t PJ = d.len[1] / H + 1, PK = d.len[2] / W + 1;
    if (sp && PJ * PK > 1) {
      split[t] = 1;
      ++n_split;
      d.face_off = pool;
      pool += PJ * PK * rows * (uint64_t)(W + RR) * 2;
      panels += (int)(PJ * PK);
    } else {
      stride = std::max(stride, rows * (PK * W + RR));
    }
    cost[t] = panel_steps(d.len, ks);
    max_n0 = std::max(max_n0, d.len[0]);
  }
  L->engine = n_split == 0 ? 0 : (n_split == (int)n ? 1 : 2);
  L->modes = n_split == 0 ? 1 : (n_split == (int)n ? 2 : 3);
  // Strip workgroups serve plans of panel jobs only.
  if (L->modes != 2) ks.group = 1;
  // Whole-triplet-only plans fit four waves per SIMD without much spilling
  // on 4x4 tiles; panel jobs carry tag registers and use the two-wave budget.
  if (!planes && !o.waves_per_simd && L->modes == 1 && ks.rj * ks.rk <= 16) {
    KernelShape k4 = ks;
    k4.wpe = 4;
    if (shape_supported(k4, sc.kind)) ks = k4;
  }
  L->ks = ks;
  L->kind = sc.kind;
  L->planes = planes;
  L->panels = panels;
  L->lds_n0 = max_n0;
  L->cells = cells;
  L->face_stride = (stride + 63) / 64 * 64;
  L->pool_ints = pool;

  // Job order: split triplets' panels first, by anti-diagonal d = pj + pk
  // across all split triplets (largest first within a diagonal), so every
  // panel comes after the panels it reads from and several split triplets
  // fill their pipelines together; then whole triplets longest first so the
  // queue drains with short ones.
  std::vector<size_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  L->jobs.clear();
  L->jobs.reserve(n + panels);
  uint32_t diagonals = 0;
  for (size_t t : idx)
    if (split[t]) diagonals = std::max(diagonals, L->desc[t].len[1] / H + L->desc[t].len[2] / W + 1);
  // With strip workgroups a job is a strip of kStripPanels panels of one
  // panel row (panel = its first panel), ordered by the diagonal of (panel
  // row, strip index): its top faces come from the strip above, its left face
  // from the strip before it in the row.
  const uint32_t sw = ks.group > 1 ? (uint32_t)kStripPanels : 1u;
  for (uint32_t d = 0; d < diagonals; ++d)
    for (size_t t : idx) {
      if (!split[t]) continue;
      const uint32_t PJ = L->desc[t].len[1] / H + 1, PK = L->desc[t].len[2] / W + 1;
      const uint32_t NS = (PK + sw - 1) / sw;  // strips (or panels) per panel row
      if (d + 1 >= PJ + NS) continue;
      for (uint32_t pj = (d >= NS ? d - NS + 1 : 0); pj <= std::min(d, PJ - 1); ++pj)
        L->jobs.push_back(JobDesc{(uint32_t)t, pj * PK + (d - pj) * sw});
    }
  for (size_t t : idx)
    if (!split[t]) L->jobs.push_back(JobDesc{(uint32_t)t, kWholeTriplet});
  // Packed pairs when asked for (any lane tile a packed kernel exists for),
  // or by default when the tile is left to the library (4 x 4, two waves per
  // SIMD); the batch keeps int32 lanes when it does not qualify (pair_up).
  L->packed = false;
  if (o.packed == 2) {
    KernelShape pks{o.tile_rows ? o.tile_rows : 4, o.tile_cols ? o.tile_cols : 4,
                    o.waves_per_simd ? o.waves_per_simd : 2};
    pks.xch = o.lane_exchange == 2 ? 1 : 0;
    pks.dma = o.staging == 2 ? 1 : 0;
    pair_up(L, sc, pks);
  } else if (o.packed == 0 && !o.tile_rows && !o.tile_cols && !o.waves_per_simd && !o.lane_exchange &&
             !o.staging) {
    pair_up(L, sc, KernelShape{4, 4, 2});
  }
  if (!L->packed && !int32_shape)
    return fail(TRIOSEQ_ERR_INVALID_ARG,
                "plan: this tile shape exists for packed pairs only, and the batch does not qualify");
  return TRIOSEQ_OK;
}

// Autotuning cache: the best options per batch length profile.
static std::mutex g_tune_mu;
static std::vector<std::pair<std::string, trioseq_plan_options>> g_tuned;
// Bumped whenever a tuned choice is remembered: cached plans made before it
// are rebuilt so they take the choice.
std::atomic<uint64_t> g_tune_epoch{0};

static int log2_bucket(double v) {
  int b = 0;
  while (v >= 2.0 && b < 80) {
    v /= 2.0;
    ++b;
  }
  return b;
}

std::string length_profile(const uint32_t* lens, size_t n, int kind) {
  uint32_t mx = 0;
  double cells = 0;
  for (size_t t = 0; t < n; ++t) {
    const uint32_t* l = lens + 3 * t;
    mx = std::max({mx, l[0], l[1], l[2]});
    cells += (double)l[0] * l[1] * l[2];
  }
  return std::to_string(kind) + "/" + std::to_string(log2_bucket((double)n)) + "/" +
         std::to_string(log2_bucket(mx)) + "/" + std::to_string(log2_bucket(cells));
}

void apply_tuned(const uint32_t* lens, size_t n, int kind, trioseq_plan_options* o) {
  const std::string key = length_profile(lens, n, kind);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : g_tuned)
    if (kv.first == key) {
      o->tile_rows = kv.second.tile_rows;
      o->tile_cols = kv.second.tile_cols;
      o->waves_per_simd = kv.second.waves_per_simd;
      if (!o->panel_group) o->panel_group = kv.second.panel_group;
      if (!o->lane_exchange) o->lane_exchange = kv.second.lane_exchange;
      if (!o->split_factor) o->split_factor = kv.second.split_factor;
      if (!o->half_split_min) o->half_split_min = kv.second.half_split_min;
      if (!o->packed) o->packed = kv.second.packed;
      if (!o->staging) o->staging = kv.second.staging;
    }
}

static void remember_tuned(const std::string& key, const trioseq_plan_options& o) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_epoch.fetch_add(1, std::memory_order_relaxed);
  for (auto& kv : g_tuned)
    if (kv.first == key) {
      kv.second = o;
      return;
    }
  g_tuned.emplace_back(key, o);
}

// Occupancy per (device, kernel variant, dynamic LDS bytes): the runtime
// query costs about 0.2 ms, and plans of one process ask the same few.
static std::mutex g_occ_mu;
static std::vector<std::pair<std::string, int>> g_occ;

static hipError_t cached_occupancy(const Layout& L, int device, int* w) {
  const std::string key = std::to_string(device) + "/" + std::to_string(L.ks.rj) + "x" +
                          std::to_string(L.ks.rk) + "/" + std::to_string(L.ks.wpe) + "/" +
                          std::to_string(L.ks.group) + "/" + std::to_string(L.ks.xch) + "/" +
                          std::to_string((int)L.packed) + "/" +
                          std::to_string(L.modes) + "/" + std::to_string(L.kind) + "/" +
                          std::to_string((int)L.planes) + "/" + std::to_string(shift_lds_bytes(L.lds_n0));
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    for (const auto& kv : g_occ)
      if (kv.first == key) {
        *w = kv.second;
        return hipSuccess;
      }
  }
  hipError_t e = L.packed ? sweep_pk_occupancy(L.ks, L.kind, L.lds_n0, w)
                         : sweep_occupancy(L.ks, L.modes, L.kind, L.planes, L.lds_n0, w);
  if (e == hipSuccess && L.modes == 2 && L.ks.group > 1) {
    // A strip workgroup's 2 * kStripPanels waves fill 4 SIMDs x (waves per
    // SIMD) slots of a compute unit; the runtime's figure for these
    // workgroups was measured above that (launches beyond it only queue).
    *w = std::max(1, std::min(*w, 4 * L.ks.wpe / (2 * kStripPanels)));
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    g_occ.emplace_back(key, *w);
  }
  return e;
}

trioseq_status layout_grid(const Layout& L, const DeviceProps& dp, int requested, int* grid,
                           int* waves_per_cu) {
  int w = 0;
  TRIOSEQ_HIP(cached_occupancy(L, dp.device, &w), "occupancy");
  int g = requested ? requested : dp.cus * std::max(1, w);
  g = (int)std::min<size_t>((size_t)g, std::max<size_t>(L.jobs.size(), 1));
  *grid = g;
  // Waves per compute unit: workgroups of 1 (whole triplets), 2 (panel jobs)
  // or 2 * kStripPanels (strip jobs) waves.
  *waves_per_cu = w * (L.modes == 1 || L.modes == 3 ? 1 : L.ks.group > 1 ? 2 * kStripPanels : 2);
  return TRIOSEQ_OK;
}

}  // namespace trioseq

namespace trioseq {

bool half_split_layout(const uint32_t* lens, const uint64_t* word_off, int32_t min_len, HalfSplit* h) {
  int ax = 0;
  for (int q = 1; q < 3; ++q)
    if (lens[q] > lens[ax]) ax = q;
  const uint32_t na = lens[ax];
  if (min_len < 0) return false;
  const uint32_t lo = min_len ? (uint32_t)std::max(min_len, 2) : kHalfSplitMin;
  if (na < lo || (na + 1) / 2 > (uint32_t)kMaxSweepLen) return false;
  const int r = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;
  const uint32_t mid = na / 2;
  uint64_t src[3];
  if (word_off) {
    for (int q = 0; q < 3; ++q) src[q] = word_off[q];
  } else {
    uint64_t tw = 0;
    trioseq_packed_layout(lens, 1, src, &tw);
  }
  const int order[3] = {ax, r, c};
  uint64_t w = 0;
  for (int half = 0; half < 2; ++half)
    for (int k = 0; k < 3; ++k) {
      const int q = order[k];
      const uint32_t start = (k == 0 && half == 1) ? mid : 0;
      const uint32_t len = k == 0 ? (half == 0 ? mid : na - mid) : lens[q];
      const int i = 3 * half + k;
      h->lens[i] = len;
      h->offs[i] = w;
      h->gather[i] = GatherDesc{src[q], w, start, len, (uint32_t)half};
      w += (len + 15) / 16;
    }
  h->words = (uint32_t)w;
  h->rows = lens[r] + 1;
  h->cols = lens[c] + 1;
  return true;
}

bool half_split_choice(const uint32_t* lens, const uint64_t* word_off, size_t n, int kind,
                       const trioseq_plan_options& o, HalfSplit* h) {
  if (n != 1 || o.lane_exchange == 2) return false;
  if (kind == kLocal) {
    if (o.half_split_min == 0 && std::max({lens[0], lens[1], lens[2]}) >= kHalfSplitMaxLocal) return false;
  } else if (kind != kGlobal) {
    return false;
  }
  return half_split_layout(lens, word_off, o.half_split_min, h);
}

}  // namespace trioseq

static trioseq_status plan_create_impl(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                       const trioseq_scoring* scp, const trioseq_plan_options* opts,
                                       trioseq_plan** out, const PlanMemory* mem = nullptr) {
  if (!out) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_create: plan output is NULL");
  if (!scp) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_create: scoring is NULL");
  trioseq_plan_options o{-1, 0, 0, 0, 0, 0};
  if (opts) o = *opts;
  // A lone global triplet is scored by halves under the automatic engine and
  // grid when the options leave the tile at (or set it to) the plane
  // kernels' 4 x 4 at two waves per SIMD.
  const bool defaults = o.engine == -1 && !o.grid && (o.tile_rows == 0 || o.tile_rows == 4) &&
                        (o.tile_cols == 0 || o.tile_cols == 4) &&
                        (o.waves_per_simd == 0 || o.waves_per_simd == 2);
  if (!o.tile_rows && !o.tile_cols && !o.waves_per_simd && lens) apply_tuned(lens, n, scp->kind, &o);
  // Inputs are validated (by the layout) before the device is touched; the
  // layout is redone if the device's size changes the split rule's hint.
  Layout L;
  int hint = 256 * kWavesPerCuHint;
  trioseq_status st = build_layout(lens, word_off, n, *scp, o, hint, &L);
  if (st != TRIOSEQ_OK) return st;
  // A lone global or local triplet under the automatic options is scored by
  // halves (local: the best of the two halves' own bests and of the paths
  // that cross the middle plane).
  HalfSplit hs;
  const bool half = defaults && half_split_choice(lens, word_off, n, scp->kind, o, &hs);
  const trioseq_plan_options ho{-1, 4, 4, 0, 0, 2, o.panel_group, o.lane_exchange};  // the plane kernels' shape
  DeviceProps dp;
  st = device_props(&dp);
  if (st != TRIOSEQ_OK) return st;
  if (half || dp.cus * kWavesPerCuHint != hint) {
    hint = dp.cus * kWavesPerCuHint;
    st = half ? build_layout(hs.lens, hs.offs, 2, *scp, ho, hint, &L, true)
              : build_layout(lens, word_off, n, *scp, o, hint, &L);
    if (st != TRIOSEQ_OK) return st;
  }
  // A batch carved from a region whose pool cannot hold its split triplets'
  // faces sweeps every triplet whole instead (same scores, no face pool).
  if (mem && !half && n > 1 && o.engine == -1 && L.pool_ints * sizeof(int) > mem->pool_bytes) {
    o.engine = 0;
    st = build_layout(lens, word_off, n, *scp, o, hint, &L);
    if (st != TRIOSEQ_OK) return st;
  }
  const size_t nd = L.desc.size();  // triplets the kernels see

  trioseq_plan* p = new (std::nothrow) trioseq_plan;
  if (!p) return fail(TRIOSEQ_ERR_NOMEM, "plan: host allocation");
  p->device = dp.device;
  p->n = n;
  p->ks = L.ks;
  p->modes = L.modes;
  p->engine = L.engine;
  p->panels = L.panels;
  p->lds_n0 = L.lds_n0;
  p->njobs = (uint32_t)L.jobs.size();
  p->sc = make_dev_scoring(*scp);
  p->cells = L.cells;
  p->use_graph = o.use_graph != 0 && !mem;
  p->face_stride = L.face_stride;
  auto hip_bail = [&](hipError_t e, const char* what) {
    fail_hip(e, what);
    trioseq_status s2 = (e == hipErrorOutOfMemory) ? TRIOSEQ_ERR_NOMEM : TRIOSEQ_ERR_DEVICE;
    plan_free(p);
    return s2;
  };
  st = layout_grid(L, dp, o.grid, &p->grid, &p->waves_per_cu);
  if (st != TRIOSEQ_OK) {
    plan_free(p);
    return st;
  }
  hipError_t e;
  // One-off initialisation runs on this thread's private stream, which is
  // waited for alone before the plan is returned (or, for a plan carved from
  // a caller's region, on the caller's stream).
  hipStream_t is = nullptr;
  if (mem) {
    is = mem->stream;
  } else if ((e = init_stream(dp.device, &is)) != hipSuccess) {
    return hip_bail(e, "hipStreamCreate");
  }
  // Device buffers: hipMalloc'd and owned by the plan, or carved in order
  // from the region's plain part (256-byte aligned); what is carved is never
  // freed.
  p->borrowed = mem != nullptr;
  uint64_t carved = 0;
  auto dalloc = [&](void** dst, uint64_t bytes) -> hipError_t {
    if (!mem) return hipMalloc(dst, bytes);
    const uint64_t at = (carved + 255) & ~255ull;
    if (at + bytes > mem->plain_bytes) return hipErrorOutOfMemory;
    *dst = mem->plain + at;
    carved = at + bytes;
    return hipSuccess;
  };
  auto too_large = [&](const std::string& what) {
    plan_free(p);
    return fail(TRIOSEQ_ERR_TOO_LARGE, "allocation-free scoring: " + what);
  };
  auto region_fail = [&](hipError_t e2, const char* what) {
    if (mem && e2 == hipErrorOutOfMemory) return too_large(std::string(what) + " exceeds the scratch region");
    return hip_bail(e2, what);
  };
  const uint64_t pool_bytes = L.pool_ints * sizeof(int);
  if (mem) {
    // The generation word, error flag and queue head persist in the region
    // (the generation only grows, so no stale tag ever looks current).
    p->d_ctl = mem->ctl;
    p->d_counter = mem->counter;
  } else {
    if ((e = hipMalloc((void**)&p->d_counter, 256)) != hipSuccess) return hip_bail(e, "hipMalloc");
    if ((e = hipMalloc((void**)&p->d_ctl, 256)) != hipSuccess) return hip_bail(e, "hipMalloc");
    if ((e = hipMemsetAsync(p->d_ctl, 0, 256, is)) != hipSuccess) return hip_bail(e, "hipMemset");
  }
  if (nd) {
    if ((e = dalloc((void**)&p->d_desc, nd * sizeof(TripletDesc))) != hipSuccess)
      return region_fail(e, "triplet table");
    if ((e = hipMemcpyAsync(p->d_desc, L.desc.data(), nd * sizeof(TripletDesc), hipMemcpyHostToDevice,
                            is)) != hipSuccess)
      return hip_bail(e, "hipMemcpy desc");
    if ((e = dalloc((void**)&p->d_jobs, L.jobs.size() * sizeof(JobDesc))) != hipSuccess)
      return region_fail(e, "job table");
    if ((e = hipMemcpyAsync(p->d_jobs, L.jobs.data(), L.jobs.size() * sizeof(JobDesc),
                            hipMemcpyHostToDevice, is)) != hipSuccess)
      return hip_bail(e, "hipMemcpy jobs");
  }
  if (pool_bytes) {
    if (mem) {
      // The region's pool part only ever holds (value, tag) pairs at even
      // offsets from its fixed base, or the zeros it started with.
      if (pool_bytes > mem->pool_bytes)
        return too_large("panel faces of split triplets exceed the scratch array's face pool");
      p->d_pface = mem->pool;
    } else {
      // Tagged faces start at tag 0, which no run uses, so nothing stale matches.
      if ((e = hipMalloc((void**)&p->d_pface, pool_bytes)) != hipSuccess)
        return hip_bail(e, "hipMalloc panel faces");
      if ((e = hipMemsetAsync(p->d_pface, 0, pool_bytes, is)) != hipSuccess) return hip_bail(e, "hipMemset");
    }
  }
  p->red_pairs = L.red_pairs();
  if (p->red_pairs &&
      (e = dalloc((void**)&p->d_red, (uint64_t)p->red_pairs * 2 * sizeof(int))) != hipSuccess)
    return region_fail(e, "reduction pairs");
  const uint64_t bnd_ints = boundary_ints(L.ks, L.lds_n0);
  if ((e = dalloc((void**)&p->d_bnd, bnd_ints * sizeof(int))) != hipSuccess)
    return region_fail(e, "sentinel faces");
  p->bnd = carve_boundary(L.ks, L.lds_n0, p->d_bnd);
  if ((e = launch_init_boundary(L.ks, p->bnd, is)) != hipSuccess) return hip_bail(e, "boundary init");
  if (L.packed) {
    p->packed = true;
    p->pk_base = L.pk_base;
    p->pk_kc = L.pk_kc;
    const uint64_t rows = face_rows(L.lds_n0);
    p->pk_top_words = rows * panel_cols(L.ks);
    const uint64_t words = p->pk_top_words + rows * right_face_row(L.ks);
    if ((e = dalloc((void**)&p->d_pkbnd, words * 4)) != hipSuccess) return region_fail(e, "packed sentinel faces");
    if ((e = launch_fill_packed_sentinel((uint32_t*)p->d_pkbnd, words, is)) != hipSuccess)
      return hip_bail(e, "packed sentinel faces");
    p->workspace_bytes += words * 4;
  }
  p->workspace_bytes = pool_bytes + bnd_ints * sizeof(int) +
                       (uint64_t)p->red_pairs * 2 * sizeof(int) +
                       nd * sizeof(TripletDesc) + L.jobs.size() * sizeof(JobDesc) + 512;
  if (half) {
    p->half = true;
    p->h_words_n = hs.words;
    const uint64_t pints = (uint64_t)hs.rows * hs.cols;
    p->h_nchunk = (uint32_t)((pints + kSplitChunk - 1) / kSplitChunk);
    const uint64_t plane_off[2] = {0, pints};
    const SplitDesc box{0, pints, hs.rows, hs.cols, 0, p->h_nchunk};
    if ((e = dalloc((void**)&p->d_hwords, std::max<uint64_t>(hs.words, 1) * 4)) != hipSuccess ||
        (e = dalloc((void**)&p->d_gather, sizeof hs.gather)) != hipSuccess ||
        (e = dalloc((void**)&p->d_plane, 2 * pints * 4)) != hipSuccess ||
        (e = dalloc((void**)&p->d_plane_off, sizeof plane_off)) != hipSuccess ||
        (e = dalloc((void**)&p->d_sdesc, sizeof box)) != hipSuccess ||
        (e = dalloc((void**)&p->d_partial, p->h_nchunk * 4)) != hipSuccess ||
        (e = dalloc((void**)&p->d_hscores, 8)) != hipSuccess)
      return region_fail(e, "half-split buffers");
    if ((e = hipMemcpyAsync(p->d_gather, hs.gather, sizeof hs.gather, hipMemcpyHostToDevice, is)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_plane_off, plane_off, sizeof plane_off, hipMemcpyHostToDevice, is)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(p->d_sdesc, &box, sizeof box, hipMemcpyHostToDevice, is)) != hipSuccess)
      return hip_bail(e, "half-split buffers");
    p->workspace_bytes += 2 * pints * 4 + (uint64_t)hs.words * 4 + p->h_nchunk * 4 + 256;
    // The host sources of these copies live until this function returns.
    if ((e = hipStreamSynchronize(is)) != hipSuccess) return hip_bail(e, "plan init");
  }
  // The whole-triplet workspace comes last: a carved plan launches no more
  // waves than the rest of the region holds workspaces for.
  if (L.face_stride) {
    const uint64_t per_wave = L.face_stride * sizeof(int);
    if (mem) {
      const uint64_t at = (carved + 255) & ~255ull;
      const uint64_t fit = at < mem->plain_bytes ? (mem->plain_bytes - at) / per_wave : 0;
      if (fit == 0) return too_large("the largest whole triplet's face workspace exceeds the scratch region");
      p->grid = (int)std::min<uint64_t>((uint64_t)p->grid, fit);
    }
    const uint64_t face_bytes = (uint64_t)p->grid * per_wave;
    if ((e = dalloc((void**)&p->d_face, face_bytes)) != hipSuccess)
      return region_fail(e, "hipMalloc face workspace");
    p->workspace_bytes += face_bytes;
  }
  if ((e = hipStreamSynchronize(is)) != hipSuccess) return hip_bail(e, "plan init");
  if (p->use_graph) {
    if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_bail(e, "hipStreamCreate");
  }
  *out = p;
  return TRIOSEQ_OK;
}

namespace trioseq {

PlaneWorkspace::~PlaneWorkspace() {
  for (Buf* b : {&ctl, &desc, &jobs, &face, &pool, &bnd, &red, &plane, &plane_off, &words, &scores, &sd,
                 &split_out, &chunk_box, &partial, &lwords, &leaves, &cols, &ncols, &lscore})
    (void)hipFree(b->p);
}

uint64_t ws_bytes(const PlaneWorkspace& ws) {
  uint64_t t = 0;
  for (const PlaneWorkspace::Buf* b :
       {&ws.ctl, &ws.desc, &ws.jobs, &ws.face, &ws.pool, &ws.bnd, &ws.red, &ws.plane, &ws.plane_off,
        &ws.words, &ws.scores, &ws.sd, &ws.split_out, &ws.chunk_box, &ws.partial, &ws.lwords, &ws.leaves,
        &ws.cols, &ws.ncols, &ws.lscore})
    t += b->bytes;
  return t;
}

hipError_t ws_grow(PlaneWorkspace::Buf& b, uint64_t bytes, bool zero, hipStream_t s) {
  bytes = std::max<uint64_t>(bytes, 256);
  if (b.bytes >= bytes) return hipSuccess;
  hipError_t e = hipStreamSynchronize(s);  // the old buffer may still be in use
  if (e != hipSuccess) return e;
  (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  const uint64_t cap = bytes + bytes / 4;  // room for the next, similar run
  if ((e = hipMalloc(&b.p, cap)) != hipSuccess) return e;
  b.bytes = cap;
  if (zero) e = hipMemsetAsync(b.p, 0, cap, s);
  return e;
}

trioseq_status run_planes(PlaneWorkspace& ws, const uint32_t* lens, const uint64_t* offs, size_t n,
                          const uint32_t* words, size_t nwords, const trioseq_scoring& sc,
                          const uint64_t* plane_off, uint64_t plane_ints, hipStream_t s) {
  if (n == 0) return TRIOSEQ_OK;
  if (!ws.have_props) {
    trioseq_status st = device_props(&ws.dp);
    if (st != TRIOSEQ_OK) return st;
    ws.have_props = true;
  }
  const trioseq_plan_options o{-1, 4, 4, 0, 0, 2};  // the plane kernels' shape
  Layout L;
  trioseq_status st = build_layout(lens, offs, n, sc, o, ws.dp.cus * kWavesPerCuHint, &L, true);
  if (st != TRIOSEQ_OK) return st;
  int grid = 0, wpc = 0;
  st = layout_grid(L, ws.dp, 0, &grid, &wpc);
  if (st != TRIOSEQ_OK) return st;
  hipError_t e;
#define WS(call, what)                                  \
  do {                                                  \
    if ((e = (call)) != hipSuccess) return fail_hip(e, what); \
  } while (0)
  if (!ws.ctl.p) {
    // [0] generation, [1] error flag, [64] queue head; the generation keeps
    // growing across runs, so a zeroed pool's tags (0) are never current.
    WS(ws_grow(ws.ctl, 512, true, s), "align: workspace");
  }
  WS(ws_grow(ws.desc, n * sizeof(TripletDesc), false, s), "align: workspace");
  WS(ws_grow(ws.jobs, L.jobs.size() * sizeof(JobDesc), false, s), "align: workspace");
  WS(ws_grow(ws.face, (uint64_t)grid * L.face_stride * 4, false, s), "align: workspace");
  WS(ws_grow(ws.pool, L.pool_ints * 4, true, s), "align: workspace");
  WS(ws_grow(ws.plane, plane_ints * 4, false, s), "align: workspace");
  WS(ws_grow(ws.plane_off, n * 8, false, s), "align: workspace");
  WS(ws_grow(ws.words, nwords * 4, false, s), "align: workspace");
  WS(ws_grow(ws.scores, n * 4, false, s), "align: workspace");
  if (!ws.bnd.p || L.lds_n0 > ws.bnd_n0) {
    WS(hipStreamSynchronize(s), "align: workspace");
    (void)hipFree(ws.bnd.p);
    ws.bnd = PlaneWorkspace::Buf{};
    WS(ws_grow(ws.bnd, boundary_ints(L.ks, L.lds_n0) * 4, false, s), "align: workspace");
    ws.boundary = carve_boundary(L.ks, L.lds_n0, (int*)ws.bnd.p);
    ws.bnd_n0 = L.lds_n0;
    WS(launch_init_boundary(L.ks, ws.boundary, s), "align: boundary");
  }
  WS(hipStreamSynchronize(s), "align: workspace");  // the previous run's host copies
  ws.h_desc.swap(L.desc);
  ws.h_jobs.swap(L.jobs);
  WS(hipMemcpyAsync(ws.desc.p, ws.h_desc.data(), n * sizeof(TripletDesc), hipMemcpyHostToDevice, s),
     "align: upload");
  WS(hipMemcpyAsync(ws.jobs.p, ws.h_jobs.data(), ws.h_jobs.size() * sizeof(JobDesc),
                    hipMemcpyHostToDevice, s),
     "align: upload");
  WS(hipMemcpyAsync(ws.plane_off.p, plane_off, n * 8, hipMemcpyHostToDevice, s), "align: upload");
  if (nwords) WS(hipMemcpyAsync(ws.words.p, words, nwords * 4, hipMemcpyHostToDevice, s), "align: upload");
  int* ctl = (int*)ws.ctl.p;
  WS(launch_prepare(ctl, ctl + 64, nullptr, 0, s), "align: prepare");
  SweepArgs a = make_sweep_args((const uint32_t*)ws.words.p, (const TripletDesc*)ws.desc.p,
                                (const JobDesc*)ws.jobs.p, (uint32_t)ws.h_jobs.size(), L.lds_n0,
                                (int32_t*)ws.scores.p, ctl + 64, ctl, (int*)ws.face.p, L.face_stride,
                                (int*)ws.pool.p, ws.boundary, nullptr, make_dev_scoring(sc));
  a.plane = (int*)ws.plane.p;
  a.plane_off = (const uint64_t*)ws.plane_off.p;
  WS(launch_sweep(L.ks, L.modes, a, grid, s), "align: sweep");
#undef WS
  return TRIOSEQ_OK;
}

}  // namespace trioseq

extern "C" {

static trioseq_status trioseq_plan_create_body(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                   const trioseq_scoring* scp, const trioseq_plan_options* opts,
                                   trioseq_plan** out) {
  return plan_create_impl(lens, word_off, n, scp, opts, out);
}

static hipError_t plan_enqueue(trioseq_plan* p, const uint32_t* d_words, int32_t* d_scores,
                               hipStream_t s) {
  if (p->n == 0) return hipSuccess;
  hipError_t e;
  if (p->half) {
    // Gather the halves (and prepare the run: the gather kernel does it when
    // there are no reduction pairs to reset), sweep both (writing their last
    // slices), meet. Under local scoring each half leaves its own best in
    // d_hscores[0..1] and the meet takes them with the crossing paths' best.
    const bool red = p->red_pairs != 0;
    if (red && (e = launch_prepare(p->d_ctl, p->d_counter, p->d_red, p->red_pairs, s)) != hipSuccess) return e;
    if ((e = launch_gather(d_words, p->d_gather, 6, p->h_words_n, p->d_hwords, red ? nullptr : p->d_ctl,
                           p->d_counter, s)) != hipSuccess)
      return e;
    SweepArgs a = make_sweep_args(p->d_hwords, p->d_desc, p->d_jobs, p->njobs, p->lds_n0, p->d_hscores,
                                  p->d_counter, p->d_ctl, p->d_face, p->face_stride, p->d_pface, p->bnd,
                                  p->d_red, p->sc);
    a.plane = p->d_plane;
    a.plane_off = p->d_plane_off;
    if ((e = launch_sweep(p->ks, p->modes, a, p->grid, s)) != hipSuccess) return e;
    return launch_meet(p->d_sdesc, p->h_nchunk, p->d_plane, p->d_partial, p->d_ctl + 1,
                       p->sc.kind == kLocal ? p->d_hscores : nullptr, p->d_ctl + 2, d_scores, s);
  }
  if ((e = launch_prepare(p->d_ctl, p->d_counter, p->d_red, p->red_pairs, s)) != hipSuccess)
    return e;
  SweepArgs a = make_sweep_args(d_words, p->d_desc, p->d_jobs, p->njobs, p->lds_n0, d_scores,
                                p->d_counter, p->d_ctl, p->d_face, p->face_stride, p->d_pface,
                                p->bnd, p->d_red, p->sc);
  if (p->packed)
    return launch_sweep_pk(p->ks, p->sc.kind, a, p->d_pkbnd, p->d_pkbnd + p->pk_top_words, p->pk_base,
                           p->pk_kc, p->grid, s);
  return launch_sweep(p->ks, p->modes, a, p->grid, s);
}

trioseq_status trioseq_plan_run(trioseq_plan* p, const uint32_t* d_words, int32_t* d_scores,
                                void* hip_stream) {
  if (!p) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_run: plan is NULL");
  if (p->n && (!d_words || !d_scores))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_run: NULL device buffer");
  hipStream_t s = (hipStream_t)hip_stream;
  if (!p->use_graph) {
    TRIOSEQ_HIP(plan_enqueue(p, d_words, d_scores, s), "kernel launch");
    return TRIOSEQ_OK;
  }
  if (!p->gexec || p->g_words != d_words || p->g_scores != d_scores) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
    if (p->graph) {
      (void)hipGraphDestroy(p->graph);
      p->graph = nullptr;
    }
    TRIOSEQ_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal),
                "hipStreamBeginCapture");
    hipError_t le = plan_enqueue(p, d_words, d_scores, p->cap_stream);
    hipError_t ce = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (le != hipSuccess) return fail_hip(le, "kernel launch during capture");
    if (ce != hipSuccess) return fail_hip(ce, "hipStreamEndCapture");
    TRIOSEQ_HIP(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    p->g_words = d_words;
    p->g_scores = d_scores;
  }
  TRIOSEQ_HIP(hipGraphLaunch(p->gexec, s), "hipGraphLaunch");
  return TRIOSEQ_OK;
}

trioseq_status trioseq_plan_get_info(const trioseq_plan* p, trioseq_plan_info* info) {
  if (!p || !info) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_get_info: NULL pointer");
  info->engine = p->engine;
  info->tile_rows = p->ks.rj;
  info->tile_cols = p->ks.rk;
  info->grid = p->grid;
  info->waves_per_cu = p->waves_per_cu;
  info->panels = p->panels;
  info->packed = p->packed ? 1 : 0;
  info->workspace_bytes = p->workspace_bytes;
  info->cells = p->cells;
  return TRIOSEQ_OK;
}

trioseq_status trioseq_plan_destroy(trioseq_plan* p) {
  plan_free(p);
  return TRIOSEQ_OK;
}

// Host packing threads: batches of at least kPackParallelMin residues are
// split over up to kPackThreadsMax threads (the calling one included).
constexpr uint64_t kPackParallelMin = 1u << 20;
constexpr size_t kPackThreadsMax = 16;

// Validates and packs host ASCII triplets into one word array.
static trioseq_status pack_triplets(const trioseq_triplet* t, size_t n, std::vector<uint32_t>* lens,
                                    std::vector<uint64_t>* offs, std::vector<uint32_t>* words) {
  if (n && !t) return fail(TRIOSEQ_ERR_INVALID_ARG, "triplet array is NULL");
  lens->resize(3 * n);
  offs->resize(3 * n);
  for (size_t q = 0; q < n; ++q)
    for (int s = 0; s < 3; ++s) {
      (*lens)[3 * q + s] = t[q].len[s];
      if (t[q].len[s] && !t[q].seq[s])
        return fail(TRIOSEQ_ERR_INVALID_ARG,
                    "triplet " + std::to_string(q) + ": sequence " + std::to_string(s) + " is NULL");
    }
  uint64_t total = 0;
  trioseq_packed_layout(lens->data(), n, offs->data(), &total);
  words->assign(std::max<uint64_t>(total, 1), 0u);
  // Large batches are packed by several host threads, each over a run of
  // whole triplets of about equal residue count. Each records its first bad
  // sequence; the first over all is packed again here for its message
  // (messages are per thread).
  const uint64_t residues = 16 * total;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nthreads = residues < kPackParallelMin ? 1 : std::min<size_t>({hw, kPackThreadsMax, n});
  std::vector<size_t> first_bad(nthreads, SIZE_MAX);
  auto pack_range = [&](size_t th, size_t q0, size_t q1) {
    for (size_t q = q0; q < q1; ++q)
      for (int s = 0; s < 3; ++s) {
        bool ok = false;
        try {  // nothing may leave a worker thread
          ok = trioseq_pack(t[q].seq[s], t[q].len[s], words->data() + (*offs)[3 * q + s]) == TRIOSEQ_OK;
        } catch (...) {
        }
        if (!ok) {
          first_bad[th] = 3 * q + s;
          return;
        }
      }
  };
  std::vector<std::thread> pool;
  size_t q0 = 0;
  for (size_t th = 0; th < nthreads; ++th) {
    // Triplets that start before the (th+1)-th share of the words; the last
    // range runs on this thread, and so does any range whose thread could
    // not be started.
    const uint64_t goal = total * (th + 1) / nthreads;
    size_t q1 = q0;
    while (q1 < n && (th + 1 == nthreads || (*offs)[3 * q1] < goal)) ++q1;
    bool started = false;
    if (th + 1 < nthreads) {
      try {
        pool.emplace_back(pack_range, th, q0, q1);
        started = true;
      } catch (...) {
      }
    }
    if (!started) pack_range(th, q0, q1);
    q0 = q1;
  }
  for (std::thread& th : pool) th.join();
  const size_t bad = *std::min_element(first_bad.begin(), first_bad.end());
  if (bad != SIZE_MAX) {
    const size_t q = bad / 3;
    const int s = (int)(bad % 3);
    const trioseq_status st = trioseq_pack(t[q].seq[s], t[q].len[s], words->data() + (*offs)[bad]);
    return fail(st, "triplet " + std::to_string(q) + ", sequence " + std::to_string(s) + ": " + g_err);
  }
  return TRIOSEQ_OK;
}

// trioseq_score_batch_packed: this thread's last plan, reused while the
// batch (lengths, word offsets, scoring, device) stays the same. It is never
// freed at thread exit (the HIP runtime may already be gone then).
struct PackedCache {
  std::vector<uint32_t> lens;
  std::vector<uint64_t> offs;
  trioseq_scoring sc{};
  int device = -1;
  trioseq_plan* plan = nullptr;
  hipStream_t stream = nullptr;  // where the plan last ran
};
static thread_local PackedCache* g_packed = nullptr;

static trioseq_status score_batch_packed_body(const uint32_t* d_words, const uint64_t* d_word_off,
                                              const uint32_t* d_len, size_t n, const trioseq_scoring* sc,
                                              int32_t* d_scores, void* hip_stream) {
  if (!sc) return fail(TRIOSEQ_ERR_INVALID_ARG, "score_batch_packed: scoring is NULL");
  if (n && (!d_words || !d_word_off || !d_len || !d_scores))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "score_batch_packed: NULL device buffer");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  if (n == 0) return TRIOSEQ_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<uint32_t> lens(3 * n);
  std::vector<uint64_t> offs(3 * n);
  hipError_t e;
  if ((e = hipMemcpyAsync(lens.data(), d_len, 3 * n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(offs.data(), d_word_off, 3 * n * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return fail_hip(e, "score_batch_packed: reading lengths");
  int device = 0;
  TRIOSEQ_HIP(hipGetDevice(&device), "hipGetDevice");
  if (!g_packed) g_packed = new PackedCache;
  PackedCache& c = *g_packed;
  const bool same = c.plan && c.device == device && c.lens == lens && c.offs == offs &&
                    std::memcmp(&c.sc, sc, sizeof *sc) == 0;
  if (!same) {
    trioseq_plan* plan = nullptr;
    st = trioseq_plan_create(lens.data(), offs.data(), n, sc, nullptr, &plan);
    if (st != TRIOSEQ_OK) return st;
    if (c.plan) {
      // The old plan's workspace may still be in use on the stream it ran on.
      (void)hipStreamSynchronize(c.stream);
      trioseq_plan_destroy(c.plan);
    }
    c.plan = plan;
    c.lens.swap(lens);
    c.offs.swap(offs);
    c.sc = *sc;
    c.device = device;
  }
  // Runs of one plan share its workspace: a run on another stream waits for
  // the previous one.
  if (c.stream != s) (void)hipStreamSynchronize(c.stream);
  c.stream = s;
  return trioseq_plan_run(c.plan, d_words, d_scores, hip_stream);
}

}  // extern "C"

namespace trioseq {

trioseq_status score_packed_in_region(const uint32_t* d_words, const uint64_t* d_word_off,
                                      const uint32_t* d_len, size_t n, const trioseq_scoring* sc,
                                      int32_t* d_scores, const PlanMemory& mem) {
  if (!sc) return fail(TRIOSEQ_ERR_INVALID_ARG, "score_batch_packed_noalloc: scoring is NULL");
  if (n && (!d_words || !d_word_off || !d_len || !d_scores))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "score_batch_packed_noalloc: NULL device buffer");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  if (n == 0) return TRIOSEQ_OK;
  // Host copies of the lengths and offsets, in buffers of this thread that
  // only grow.
  static thread_local std::vector<uint32_t>* lens = nullptr;
  static thread_local std::vector<uint64_t>* offs = nullptr;
  if (!lens) lens = new std::vector<uint32_t>;
  if (!offs) offs = new std::vector<uint64_t>;
  lens->resize(3 * n);
  offs->resize(3 * n);
  hipError_t e;
  if ((e = hipMemcpyAsync(lens->data(), d_len, 3 * n * 4, hipMemcpyDeviceToHost, mem.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(offs->data(), d_word_off, 3 * n * 8, hipMemcpyDeviceToHost, mem.stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(mem.stream)) != hipSuccess)
    return fail_hip(e, "score_batch_packed_noalloc: reading lengths");
  trioseq_plan* plan = nullptr;
  st = plan_create_impl(lens->data(), offs->data(), n, sc, nullptr, &plan, &mem);
  if (st != TRIOSEQ_OK) return st;
  const hipError_t le = plan_enqueue(plan, d_words, d_scores, mem.stream);
  plan_free(plan);  // host bookkeeping only: the device buffers are the region's
  if (le != hipSuccess) return fail_hip(le, "score_batch_packed_noalloc: kernel launch");
  return TRIOSEQ_OK;
}

}  // namespace trioseq

extern "C" {

// trioseq_score / trioseq_score_batch: the plans (with their device inputs
// and outputs) of this thread's last few batch shapes, reused when the same
// lengths, scoring and device come again, so a repeated call only uploads,
// launches and downloads. Plans whose workspace exceeds kHostCacheBytes are
// freed after their call. Never freed at thread exit (the HIP runtime may
// already be gone then).
constexpr size_t kHostCacheEntries = 4;
constexpr uint64_t kHostCacheBytes = 4ull << 30;
struct HostBatchEntry {
  int device = -1;
  int engine = 0;
  uint64_t epoch = 0;
  std::vector<uint32_t> lens;
  trioseq_scoring sc{};
  trioseq_plan* plan = nullptr;
  uint32_t* d_words = nullptr;
  int32_t* d_scores = nullptr;
  uint64_t last_use = 0;
};
static thread_local std::vector<HostBatchEntry>* g_host_cache = nullptr;
static thread_local uint64_t g_host_clock = 0;

static void host_entry_free(HostBatchEntry& c) {
  (void)hipFree(c.d_words);
  (void)hipFree(c.d_scores);
  trioseq_plan_destroy(c.plan);
  c = HostBatchEntry{};
}

static trioseq_status run_host_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc,
                                     int32_t* scores, hipStream_t s, int engine) {
  if (n && !scores) return fail(TRIOSEQ_ERR_INVALID_ARG, "scores is NULL");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  std::vector<uint32_t> lens, words;
  std::vector<uint64_t> offs;
  st = pack_triplets(t, n, &lens, &offs, &words);
  if (st != TRIOSEQ_OK) return st;
  if (n == 0) return TRIOSEQ_OK;
  // A cached plan is only looked for on a working device; otherwise
  // plan_create below validates the batch (before any device work) and
  // reports the problem.
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) device = -1;
  if (!g_host_cache) g_host_cache = new std::vector<HostBatchEntry>;
  std::vector<HostBatchEntry>& cache = *g_host_cache;
  const uint64_t epoch = g_tune_epoch.load(std::memory_order_relaxed);
  HostBatchEntry* hit = nullptr;
  for (HostBatchEntry& c : cache)
    if (device >= 0 && c.plan && c.device == device && c.engine == engine && c.epoch == epoch && c.lens == lens &&
        std::memcmp(&c.sc, sc, sizeof *sc) == 0)
      hit = &c;
  HostBatchEntry fresh;
  if (!hit) {
    trioseq_plan_options o{engine, 0, 0, 0, 0, 0};
    st = trioseq_plan_create(lens.data(), offs.data(), n, sc, &o, &fresh.plan);
    if (st != TRIOSEQ_OK) return st;
    hipError_t e = hipMalloc((void**)&fresh.d_words, words.size() * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&fresh.d_scores, n * 4);
    if (e != hipSuccess) {
      host_entry_free(fresh);
      return fail_hip(e, "batch: device buffers");
    }
    fresh.device = device;
    fresh.engine = engine;
    fresh.epoch = epoch;
    fresh.lens = lens;
    fresh.sc = *sc;
    hit = &fresh;
  }
  hit->last_use = ++g_host_clock;
  hipError_t e = hipMemcpyAsync(hit->d_words, words.data(), words.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    st = trioseq_plan_run(hit->plan, hit->d_words, hit->d_scores, s);
    if (st == TRIOSEQ_OK) {
      e = hipMemcpyAsync(scores, hit->d_scores, n * 4, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  if (hit == &fresh) {
    // Keep it when it is small enough, in place of the least recently used.
    if (st == TRIOSEQ_OK && e == hipSuccess && fresh.plan->workspace_bytes <= kHostCacheBytes) {
      if (cache.size() < kHostCacheEntries) {
        cache.push_back(std::move(fresh));
      } else {
        HostBatchEntry* lru = &cache[0];
        for (HostBatchEntry& c : cache)
          if (c.last_use < lru->last_use) lru = &c;
        host_entry_free(*lru);
        *lru = std::move(fresh);
      }
    } else {
      host_entry_free(fresh);
    }
  }
  if (st != TRIOSEQ_OK) return st;
  if (e != hipSuccess) return fail_hip(e, "batch");
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_autotune_body(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                const trioseq_scoring* sc, const uint32_t* d_words, int32_t reps,
                                void* hip_stream, trioseq_tune_result* out) {
  if (!out || !sc || (n && (!lens || !d_words)))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "autotune: NULL pointer");
  if (n == 0) return fail(TRIOSEQ_ERR_INVALID_ARG, "autotune: empty batch");
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)hip_stream;
  // Candidates: the reference (library defaults) first, then every lane tile
  // (the panel a wave owns is 8 x 8 tiles) and register budget, the register
  // lane exchange, other split factors (which triplets of a batch become
  // panel jobs), strip workgroups, and for a lone triplet other half-split
  // thresholds. Options a layout ignores are not tried.
  std::vector<trioseq_plan_options> cands;
  cands.push_back(trioseq_plan_options{-1, 4, 4, 0, 0, 2});
  const int shapes[][3] = {{4, 4, 4}, {8, 4, 2}, {4, 8, 2}};
  for (const auto& sh : shapes) cands.push_back(trioseq_plan_options{-1, sh[0], sh[1], 0, 0, sh[2]});
  if (sc->kind == kGlobal) {
    cands.push_back(trioseq_plan_options{-1, 4, 4, 0, 0, 2, 0, 2});
    cands.push_back(trioseq_plan_options{-1, 8, 4, 0, 0, 2, 0, 2});
  }
  if (n > 1) {
    for (int f : {2, 8, 16}) cands.push_back(trioseq_plan_options{-1, 4, 4, 0, 0, 2, 0, 0, f});
    // Packed shapes: tile, waves per SIMD, lane exchange, staging (the
    // other kinds have the plain forms only).
    const int pks[][5] = {{4, 4, 2, 0, 0}, {4, 4, 3, 0, 0}, {8, 4, 2, 0, 0}, {4, 8, 2, 0, 0},
                          {4, 4, 2, 2, 0}, {4, 4, 2, 0, 2}, {4, 4, 3, 0, 2}, {8, 4, 2, 0, 2},
                          {4, 8, 2, 0, 2}};
    for (const auto& sh : pks)
      if (sc->kind == kGlobal || (sh[3] == 0 && sh[4] == 0))
        cands.push_back(trioseq_plan_options{-1, sh[0], sh[1], 0, 0, sh[2], 0, sh[3], 0, 0, 2, sh[4]});
  } else {
    cands.push_back(trioseq_plan_options{-1, 4, 4, 0, 0, 2, 4});
    if (sc->kind == kGlobal)
      for (int h : {-1, 128, 512}) cands.push_back(trioseq_plan_options{-1, 4, 4, 0, 0, 2, 0, 0, 0, h});
  }
  int32_t* d_ref = nullptr;
  int32_t* d_out = nullptr;
  TRIOSEQ_HIP(hipMalloc((void**)&d_ref, n * 4), "hipMalloc");
  hipError_t e = hipMalloc((void**)&d_out, n * 4);
  if (e != hipSuccess) {
    (void)hipFree(d_ref);
    return fail_hip(e, "hipMalloc");
  }
  std::vector<int32_t> ref(n), got(n);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  trioseq_tune_result r{};
  r.best_ms = 1e300;
  trioseq_status st = TRIOSEQ_OK;
  for (size_t c = 0; c < cands.size() && st == TRIOSEQ_OK; ++c) {
    trioseq_plan_options o = cands[c];
    trioseq_plan* plan = nullptr;
    // Shapes that need more registers than a budget allows are skipped.
    if (trioseq_plan_create(lens, word_off, n, sc, &o, &plan) != TRIOSEQ_OK) continue;
    trioseq_plan_info info;
    trioseq_plan_get_info(plan, &info);
    int32_t* dst = c == 0 ? d_ref : d_out;
    st = trioseq_plan_run(plan, d_words, dst, s);  // warm-up, and the scores to compare
    if (st == TRIOSEQ_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = fail_hip(e, "autotune");
    float ms = 0;
    if (st == TRIOSEQ_OK) {
      (void)hipEventRecord(ev0, s);
      for (int k = 0; k < reps && st == TRIOSEQ_OK; ++k) st = trioseq_plan_run(plan, d_words, d_out, s);
      (void)hipEventRecord(ev1, s);
      if (st == TRIOSEQ_OK && (e = hipEventSynchronize(ev1)) != hipSuccess) st = fail_hip(e, "autotune");
      (void)hipEventElapsedTime(&ms, ev0, ev1);
      ms /= (float)reps;
    }
    trioseq_plan_destroy(plan);
    if (st != TRIOSEQ_OK) break;
    ++r.tried;
    if (c == 0) {
      if ((e = hipMemcpy(ref.data(), d_ref, n * 4, hipMemcpyDeviceToHost)) != hipSuccess) {
        st = fail_hip(e, "autotune");
        break;
      }
      r.reference_ms = ms;
    } else {
      if ((e = hipMemcpy(got.data(), d_out, n * 4, hipMemcpyDeviceToHost)) != hipSuccess) {
        st = fail_hip(e, "autotune");
        break;
      }
      if (got != ref) {  // parity gate: never pick a configuration that disagrees
        ++r.rejected;
        continue;
      }
    }
    if (ms < r.best_ms) {
      r.best_ms = ms;
      r.best = cands[c];
      r.best.tile_rows = info.tile_rows;
      r.best.tile_cols = info.tile_cols;
      r.best.waves_per_simd = c == 0 ? 0 : cands[c].waves_per_simd;
    }
    if (std::getenv("TRIOSEQ_TUNE_LOG"))
      std::fprintf(stderr, "autotune: %dx%d wpe %d xch %d group %d split %d half %d packed %d staging %d: %.4f ms\n",
                   info.tile_rows, info.tile_cols, cands[c].waves_per_simd, cands[c].lane_exchange,
                   cands[c].panel_group, cands[c].split_factor, cands[c].half_split_min, info.packed,
                   cands[c].staging, ms);
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipFree(d_ref);
  (void)hipFree(d_out);
  if (st != TRIOSEQ_OK) return st;
  if (r.tried == 0) return fail(TRIOSEQ_ERR_DEVICE, "autotune: no configuration could be planned");
  if (r.best.waves_per_simd) remember_tuned(length_profile(lens, n, sc->kind), r.best);
  *out = r;
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_score_body(const trioseq_triplet* t, const trioseq_scoring* sc, int32_t* score) {
  if (!t || !score) return fail(TRIOSEQ_ERR_INVALID_ARG, "score: NULL pointer");
  return run_host_batch(t, 1, sc, score, nullptr, -1);
}

static trioseq_status trioseq_score_batch_body(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc,
                                   int32_t* scores, void* hip_stream) {
  return run_host_batch(t, n, sc, scores, (hipStream_t)hip_stream, -1);
}

}  // extern "C"

// Entry points: every body runs guarded (no exception crosses the ABI).
extern "C" {

trioseq_status trioseq_plan_create(const uint32_t* lens, const uint64_t* word_off, size_t n, const trioseq_scoring* scp, const trioseq_plan_options* opts, trioseq_plan** out) {
  return guarded([&] { return trioseq_plan_create_body(lens, word_off, n, scp, opts, out); });
}

trioseq_status trioseq_autotune(const uint32_t* lens, const uint64_t* word_off, size_t n, const trioseq_scoring* sc, const uint32_t* d_words, int32_t reps, void* hip_stream, trioseq_tune_result* out) {
  return guarded([&] { return trioseq_autotune_body(lens, word_off, n, sc, d_words, reps, hip_stream, out); });
}

trioseq_status trioseq_score(const trioseq_triplet* t, const trioseq_scoring* sc, int32_t* score) {
  return guarded([&] { return trioseq_score_body(t, sc, score); });
}

trioseq_status trioseq_score_batch_packed(const uint32_t* d_words, const uint64_t* d_word_off,
                                          const uint32_t* d_len, size_t n, const trioseq_scoring* sc,
                                          int32_t* d_scores, void* hip_stream) {
  return guarded([&] {
    return score_batch_packed_body(d_words, d_word_off, d_len, n, sc, d_scores, hip_stream);
  });
}

trioseq_status trioseq_score_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc, int32_t* scores, void* hip_stream) {
  return guarded([&] { return trioseq_score_batch_body(t, n, sc, scores, hip_stream); });
}

}  // extern "C"

// Host runtime of libtrioseq: validation, 2-bit packing, planning (axis
// choice, longest-first ordering, workspace sizing), launches, hipGraph
// replay, and the synchronous single/batch entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
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

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

trioseq_status validate_scoring(const trioseq_scoring* sc) {
  if (!sc) return fail(TRIOSEQ_ERR_INVALID_ARG, "scoring is NULL");
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
  return d;
}

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
  int engine = 0;
  uint32_t lds_n0 = 0;
  KernelShape ks{4, 4};
  int grid = 0, waves_per_cu = 0, panels = 0;
  DevScoring sc{};
  double cells = 0;
  uint64_t workspace_bytes = 0;
  // batch engine
  TripletDesc* d_desc = nullptr;
  int* d_counter = nullptr;
  uint64_t face_stride = 0;
  // wide engine
  TripletDesc wide_desc{};
  uint32_t* d_order = nullptr;
  int* d_progress = nullptr;
  uint32_t ppw = 0, pk_count = 0;
  int* d_face = nullptr;
  // sentinel faces for edge panels
  Boundary bnd{};
  int* d_bnd = nullptr;
  // graph replay
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const uint32_t* g_words = nullptr;
  int32_t* g_scores = nullptr;
};

static void plan_free(trioseq_plan* p) {
  if (!p) return;
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  (void)hipFree(p->d_desc);
  (void)hipFree(p->d_counter);
  (void)hipFree(p->d_order);
  (void)hipFree(p->d_progress);
  (void)hipFree(p->d_face);
  (void)hipFree(p->d_bnd);
  delete p;
}

extern "C" {

void trioseq_scoring_simple(trioseq_scoring* s, int32_t match, int32_t mismatch, int32_t gap) {
  if (!s) return;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) s->sub[x][y] = x == y ? match : mismatch;
  s->gap = gap;
}

const char* trioseq_last_error(void) { return g_err.c_str(); }

const char* trioseq_version(void) { return "trioseq-mi355x 0.1 (gfx950)"; }

trioseq_status trioseq_pack(const char* seq, uint32_t len, uint32_t* words) {
  if (len && (!seq || !words)) return fail(TRIOSEQ_ERR_INVALID_ARG, "pack: NULL pointer");
  const uint32_t nw = (len + 15) / 16;
  for (uint32_t w = 0; w < nw; ++w) {
    uint32_t v = 0;
    const uint32_t base = w * 16;
    const uint32_t m = std::min<uint32_t>(16, len - base);
    for (uint32_t q = 0; q < m; ++q) {
      const uint8_t c = g_code[(uint8_t)seq[base + q]];
      if (c > 3)
        return fail(TRIOSEQ_ERR_BAD_RESIDUE,
                    "pack: character at position " + std::to_string(base + q) + " is not ACGT");
      v |= (uint32_t)c << (2 * q);
    }
    words[w] = v;
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

trioseq_status trioseq_plan_create(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                   const trioseq_scoring* scp, const trioseq_plan_options* opts,
                                   trioseq_plan** out) {
  if (!out) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_create: plan output is NULL");
  if (n && !lens) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan_create: lens is NULL");
  if (n > (size_t)INT32_MAX) return fail(TRIOSEQ_ERR_TOO_LARGE, "plan_create: too many triplets");
  trioseq_status st = validate_scoring(scp);
  if (st != TRIOSEQ_OK) return st;
  trioseq_plan_options o{-1, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.engine < -1 || o.engine > 1) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: bad engine");
  KernelShape ks{o.tile_rows ? o.tile_rows : 4, o.tile_cols ? o.tile_cols : 4};
  if (!shape_supported(ks)) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: unsupported tile shape");
  if (o.grid < 0) return fail(TRIOSEQ_ERR_INVALID_ARG, "plan: negative grid");

  // Validate every triplet before touching the device.
  std::vector<uint64_t> offs;
  const uint64_t* off = word_off;
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
    st = check_range(*scp, l[0], l[1], l[2], t);
    if (st != TRIOSEQ_OK) return st;
    cells += (double)l[0] * (double)l[1] * (double)l[2];
  }

  DeviceProps dp;
  st = device_props(&dp);
  if (st != TRIOSEQ_OK) return st;

  trioseq_plan* p = new (std::nothrow) trioseq_plan;
  if (!p) return fail(TRIOSEQ_ERR_NOMEM, "plan: host allocation");
  p->device = dp.device;
  p->n = n;
  p->ks = ks;
  p->sc = make_dev_scoring(*scp);
  p->cells = cells;
  p->use_graph = o.use_graph != 0;
  int engine = o.engine;
  if (engine < 0) engine = (n == 1) ? 1 : 0;
  p->engine = engine;

  auto bail = [&](trioseq_status s) {
    plan_free(p);
    return s;
  };
  auto hip_bail = [&](hipError_t e, const char* what) {
    fail_hip(e, what);
    trioseq_status s = (e == hipErrorOutOfMemory) ? TRIOSEQ_ERR_NOMEM : TRIOSEQ_ERR_DEVICE;
    plan_free(p);
    return s;
  };
  hipError_t e;
  const int H = panel_rows(ks), W = panel_cols(ks);

  if (engine == 0) {
    std::vector<TripletDesc> desc(n);
    std::vector<uint64_t> cost(n);
    uint64_t stride = 0;
    uint32_t max_n0 = 0;
    for (size_t t = 0; t < n; ++t) {
      const uint32_t* l = lens + 3 * t;
      AxisChoice ax = choose_axes_batch(l, ks);
      TripletDesc& d = desc[t];
      for (int a = 0; a < 3; ++a) {
        d.off[a] = off[3 * t + ax.perm[a]];
        d.len[a] = l[ax.perm[a]];
      }
      d.out = (uint32_t)t;
      cost[t] = panel_steps(d.len, ks);
      const uint64_t pk = d.len[2] / W + 1;
      const uint64_t need = (uint64_t)face_rows(d.len[0]) * (pk * W + right_face_row(ks));
      stride = std::max(stride, need);
      max_n0 = std::max(max_n0, d.len[0]);
    }
    // Longest first: the persistent queue then ends with short triplets.
    std::vector<size_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<TripletDesc> sorted(n);
    for (size_t q = 0; q < n; ++q) sorted[q] = desc[idx[q]];
    stride = (stride + 63) / 64 * 64;
    p->face_stride = stride;
    p->lds_n0 = max_n0;
    if ((e = batch_occupancy(ks, max_n0, &p->waves_per_cu)) != hipSuccess) return hip_bail(e, "occupancy");
    int grid = o.grid ? o.grid : dp.cus * std::max(1, p->waves_per_cu);
    grid = (int)std::min<size_t>((size_t)grid, std::max<size_t>(n, 1));
    p->grid = grid;
    const uint64_t face_bytes = (uint64_t)grid * stride * sizeof(int);
    p->workspace_bytes = face_bytes + n * sizeof(TripletDesc) + 256;
    if ((e = hipMalloc((void**)&p->d_counter, 256)) != hipSuccess) return hip_bail(e, "hipMalloc");
    if (n) {
      if ((e = hipMalloc((void**)&p->d_desc, n * sizeof(TripletDesc))) != hipSuccess)
        return hip_bail(e, "hipMalloc desc");
      if ((e = hipMemcpy(p->d_desc, sorted.data(), n * sizeof(TripletDesc), hipMemcpyHostToDevice)) !=
          hipSuccess)
        return hip_bail(e, "hipMemcpy desc");
    }
    if (face_bytes && (e = hipMalloc((void**)&p->d_face, face_bytes)) != hipSuccess)
      return hip_bail(e, "hipMalloc face workspace");
  } else {
    if (n != 1) return bail(fail(TRIOSEQ_ERR_INVALID_ARG, "wide engine takes exactly one triplet"));
    AxisChoice ax = choose_axes_wide(lens);
    TripletDesc& d = p->wide_desc;
    for (int a = 0; a < 3; ++a) {
      d.off[a] = off[ax.perm[a]];
      d.len[a] = lens[ax.perm[a]];
    }
    d.out = 0;
    const uint32_t PJ = d.len[1] / H + 1, PK = d.len[2] / W + 1;
    const uint32_t panels = PJ * PK;
    p->panels = (int)panels;
    p->pk_count = PK;
    p->lds_n0 = d.len[0];
    if ((e = wide_occupancy(ks, d.len[0], &p->waves_per_cu)) != hipSuccess) return hip_bail(e, "occupancy");
    // Every wavefront must be resident at once: a panel waits on its
    // neighbours' progress counters.
    int cap = dp.cus * std::max(1, p->waves_per_cu);
    int grid = o.grid ? std::min(o.grid, cap) : cap;
    grid = (int)std::min<uint32_t>((uint32_t)grid, panels);
    p->grid = grid;
    p->ppw = (panels + grid - 1) / grid;
    // Panels in order of their anti-diagonal pj + pk, dealt round-robin, so
    // every wavefront visits its panels in dependency order.
    std::vector<uint32_t> diag(panels);
    std::iota(diag.begin(), diag.end(), 0u);
    std::stable_sort(diag.begin(), diag.end(), [&](uint32_t a, uint32_t b) {
      return (a / PK + a % PK) < (b / PK + b % PK);
    });
    std::vector<uint32_t> order((size_t)grid * p->ppw, 0xFFFFFFFFu);
    for (uint32_t q = 0; q < panels; ++q) order[(size_t)(q % grid) * p->ppw + q / grid] = diag[q];
    const uint64_t per_panel = (uint64_t)face_rows(d.len[0]) * (W + right_face_row(ks));
    const uint64_t face_bytes = per_panel * panels * sizeof(int);
    p->workspace_bytes = face_bytes + order.size() * 4 + panels * 4;
    if ((e = hipMalloc((void**)&p->d_order, order.size() * 4)) != hipSuccess)
      return hip_bail(e, "hipMalloc order");
    if ((e = hipMemcpy(p->d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_bail(e, "hipMemcpy order");
    if ((e = hipMalloc((void**)&p->d_progress, (panels + 1) * 4)) != hipSuccess)
      return hip_bail(e, "hipMalloc progress");
    if ((e = hipMalloc((void**)&p->d_face, face_bytes)) != hipSuccess)
      return hip_bail(e, "hipMalloc face workspace");
  }
  {
    // Sentinel faces for panels on the tensor edge, built once per plan.
    const uint64_t rows = face_rows(p->lds_n0);
    const uint64_t top_ints = rows * W, left_ints = rows * right_face_row(ks);
    const uint64_t bytes = (2 * top_ints + left_ints) * sizeof(int);
    if ((e = hipMalloc((void**)&p->d_bnd, bytes)) != hipSuccess) return hip_bail(e, "hipMalloc boundary");
    p->bnd.top_seed = p->d_bnd;
    p->bnd.top = p->d_bnd + top_ints;
    p->bnd.left = p->d_bnd + 2 * top_ints;
    p->bnd.rows = (uint32_t)rows;
    p->workspace_bytes += bytes;
    if ((e = launch_init_boundary(ks, p->bnd, nullptr)) != hipSuccess) return hip_bail(e, "boundary init");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_bail(e, "boundary init");
  }
  if (p->use_graph) {
    if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_bail(e, "hipStreamCreate");
  }
  *out = p;
  return TRIOSEQ_OK;
}

static hipError_t plan_enqueue(trioseq_plan* p, const uint32_t* d_words, int32_t* d_scores,
                               hipStream_t s) {
  hipError_t e;
  if (p->engine == 0) {
    if (p->n == 0) return hipSuccess;
    if ((e = launch_reset(p->d_counter, 1, s)) != hipSuccess) return e;
    BatchArgs a;
    a.words = d_words;
    a.desc = p->d_desc;
    a.scores = d_scores;
    a.counter = p->d_counter;
    a.face = p->d_face;
    a.face_stride = p->face_stride;
    a.n = (uint32_t)p->n;
    a.lds_n0 = p->lds_n0;
    a.bnd_top_seed = p->bnd.top_seed;
    a.bnd_top = p->bnd.top;
    a.bnd_left = p->bnd.left;
    a.sc = p->sc;
    return launch_batch(p->ks, a, p->grid, s);
  }
  if ((e = launch_reset(p->d_progress, p->panels + 1, s)) != hipSuccess) return e;
  WideArgs a;
  a.words = d_words;
  a.desc = p->wide_desc;
  a.scores = d_scores;
  a.face = p->d_face;
  a.progress = p->d_progress;
  a.order = p->d_order;
  a.panels_per_wave = p->ppw;
  a.n_panels = (uint32_t)p->panels;
  a.pk_count = p->pk_count;
  a.bnd_top_seed = p->bnd.top_seed;
  a.bnd_top = p->bnd.top;
  a.bnd_left = p->bnd.left;
  a.sc = p->sc;
  return launch_wide(p->ks, a, p->grid, s);
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
  info->workspace_bytes = p->workspace_bytes;
  info->cells = p->cells;
  return TRIOSEQ_OK;
}

trioseq_status trioseq_plan_destroy(trioseq_plan* p) {
  plan_free(p);
  return TRIOSEQ_OK;
}

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
  for (size_t q = 0; q < n; ++q)
    for (int s = 0; s < 3; ++s) {
      trioseq_status st = trioseq_pack(t[q].seq[s], t[q].len[s], words->data() + (*offs)[3 * q + s]);
      if (st != TRIOSEQ_OK)
        return fail(st, "triplet " + std::to_string(q) + ", sequence " + std::to_string(s) + ": " +
                            g_err);
    }
  return TRIOSEQ_OK;
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
  trioseq_plan_options o{engine, 0, 0, 0, 0};
  trioseq_plan* plan = nullptr;
  st = trioseq_plan_create(lens.data(), offs.data(), n, sc, &o, &plan);
  if (st != TRIOSEQ_OK) return st;
  uint32_t* d_words = nullptr;
  int32_t* d_scores = nullptr;
  hipError_t e = hipMalloc((void**)&d_words, words.size() * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&d_scores, n * 4);
  if (e == hipSuccess) e = hipMemcpyAsync(d_words, words.data(), words.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    st = trioseq_plan_run(plan, d_words, d_scores, s);
    if (st == TRIOSEQ_OK) {
      e = hipMemcpyAsync(scores, d_scores, n * 4, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  (void)hipFree(d_words);
  (void)hipFree(d_scores);
  trioseq_plan_destroy(plan);
  if (st != TRIOSEQ_OK) return st;
  if (e != hipSuccess) return fail_hip(e, "batch");
  return TRIOSEQ_OK;
}

trioseq_status trioseq_score(const trioseq_triplet* t, const trioseq_scoring* sc, int32_t* score) {
  if (!t || !score) return fail(TRIOSEQ_ERR_INVALID_ARG, "score: NULL pointer");
  return run_host_batch(t, 1, sc, score, nullptr, -1);
}

trioseq_status trioseq_score_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc,
                                   int32_t* scores, void* hip_stream) {
  return run_host_batch(t, n, sc, scores, (hipStream_t)hip_stream, 0);
}

}  // extern "C"

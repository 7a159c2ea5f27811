// Serving runtime: continuous batching of triplet requests on one GPU.
//
// Requests are validated, packed and queued by trioseq_serve_submit (never
// blocking on the device). A worker thread admits queued requests into
// rounds: a round is one launch of the persistent sweep kernel over the
// requests admitted together, laid out like a plan (large requests are split
// into panel jobs, the rest are swept whole), placed in one of several
// preallocated device arenas ("slots"), each with its own stream. Admission
// takes requests first-come first-served while the round's device footprint
// (packed words, per-wave workspace, panel faces) fits the slot. Up to
// max_inflight rounds are in flight at once, so requests that arrive while others
// run are launched immediately into a free slot and their waves take over
// compute units as earlier rounds drain. Each score is written by the GPU
// straight into mapped pinned host memory, so a request completes when its
// own triplet finishes, not when its round does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "common.h"

namespace trioseq {
namespace {

constexpr uint32_t kDefaultInflight = 4;
constexpr uint32_t kMaxInflight = 16;
// Scores are bounded by 2^30 in magnitude, so this value marks "not yet".
constexpr int32_t kPending = INT32_MIN + 1;

struct Request {
  uint64_t id = 0;
  uint32_t len[3] = {0, 0, 0};
  uint32_t woff[3] = {0, 0, 0};  // word offsets of the sequences in `words`
  std::vector<uint32_t> words;
  uint64_t t_submit = 0;
  double cells = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  char* arena = nullptr;  // device: packed words, job tables, whole-triplet workspace
  uint64_t arena_bytes = 0;
  // Device region that only ever holds tagged panel faces ((value, tag)
  // pairs at 8-byte alignment), zeroed once. Because no plain data is ever
  // written here, every stale tag slot holds an older run generation of this
  // slot (or 0), never a value that could pass for the current one.
  int* tagged = nullptr;
  uint64_t tagged_bytes = 0;
  int* ctl = nullptr;     // device: [0] generation, [1] error flag, [64] queue head
  uint32_t* h_words = nullptr;  // pinned staging
  uint64_t h_words_cap = 0;
  TripletDesc* h_desc = nullptr;
  JobDesc* h_jobs = nullptr;
  uint64_t h_meta_cap = 0;      // entries of h_desc / h_jobs
  int32_t* h_scores = nullptr;  // pinned, mapped: written by the GPU
  int32_t* d_scores = nullptr;  // device address of h_scores
  uint32_t max_batch = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Request> reqs;
  std::vector<char> reported;
  uint64_t t_launch = 0;
};

}  // namespace
}  // namespace trioseq

using namespace trioseq;

struct trioseq_server {
  trioseq_serve_config cfg{};
  trioseq_scoring sc{};
  DevScoring dsc{};
  DeviceProps dp{};
  KernelShape ks{4, 4, 2};
  int* d_bnd = nullptr;
  Boundary bnd{};
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> pending;
  std::unordered_set<uint64_t> outstanding;  // submitted, result not yet consumed
  std::unordered_map<uint64_t, trioseq_result> done;
  std::deque<uint64_t> done_fifo;
  uint64_t next_id = 1;
  bool closing = false;
  std::thread worker;
  std::string worker_error;

  // statistics
  uint64_t submitted = 0, completed = 0, failed = 0, rounds = 0;
  double cells = 0;
  double busy_s = 0;
  uint64_t busy_since = 0;
  std::vector<double> lat_ns;
};

namespace {

uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }

// Device bytes a round needs in a slot arena (the panel-face pool lives in
// the slot's tagged region instead: L.pool_ints * 4 bytes).
uint64_t arena_need(const Layout& L, uint64_t words, int grid) {
  return align256(words * 4) + align256(L.desc.size() * sizeof(TripletDesc)) +
         align256(L.jobs.size() * sizeof(JobDesc)) + align256((uint64_t)L.red_pairs() * 8) +
         align256((uint64_t)grid * L.face_stride * 4);
}

void record_result(trioseq_server* s, const Request& r, int32_t score, int32_t status, uint64_t t) {
  trioseq_result res;
  res.id = r.id;
  res.score = score;
  res.status = status;
  res.t_submit_ns = r.t_submit;
  res.t_done_ns = t;
  s->done[r.id] = res;
  s->done_fifo.push_back(r.id);
  if (status == TRIOSEQ_OK) {
    s->completed++;
    s->cells += r.cells;
    s->lat_ns.push_back((double)(t - r.t_submit));
  } else {
    s->failed++;
  }
}

// Builds and launches one round in slot `sl` from `batch` (lock not held).
// alone: no other round is on the device.
trioseq_status launch_round(trioseq_server* s, Slot& sl, std::vector<Request>& batch, Layout* L_out,
                            std::string* err, bool alone) {
  const size_t n = batch.size();
  std::vector<uint32_t> lens(3 * n);
  std::vector<uint64_t> offs(3 * n);
  uint64_t words = 0;
  for (size_t q = 0; q < n; ++q) {
    for (int a = 0; a < 3; ++a) {
      lens[3 * q + a] = batch[q].len[a];
      offs[3 * q + a] = words + batch[q].woff[a];
    }
    words += batch[q].words.size();
  }
  trioseq_plan_options o{-1, s->ks.rj, s->ks.rk, 0, 0, 0};
  Layout& L = *L_out;
  trioseq_status st =
      build_layout(lens.data(), offs.data(), n, s->sc, o, s->dp.cus * kWavesPerCuHint, &L);
  if (st != TRIOSEQ_OK) {
    *err = trioseq_last_error();
    return st;
  }
  // Rounds of several split requests, or of one that shares the device with
  // other rounds: their panel jobs are swept by single-wave workgroups (two
  // computing waves per SIMD) rather than by computing and staging wave
  // pairs.
  if (L.modes == 2 && (L.desc.size() >= 2 || !alone)) L.modes = 3;
  int grid = 0, wpc = 0;
  st = layout_grid(L, s->dp, 0, &grid, &wpc);
  if (st != TRIOSEQ_OK) {
    *err = trioseq_last_error();
    return st;
  }
  if (arena_need(L, words, grid) > sl.arena_bytes || L.pool_ints * 4 > sl.tagged_bytes ||
      words > sl.h_words_cap || L.jobs.size() > sl.h_meta_cap || n > sl.max_batch) {
    *err = "round does not fit its slot";
    return TRIOSEQ_ERR_TOO_LARGE;
  }
  // Stage on the host, then copy to the slot arena.
  uint64_t w = 0;
  for (size_t q = 0; q < n; ++q) {
    std::memcpy(sl.h_words + w, batch[q].words.data(), batch[q].words.size() * 4);
    w += batch[q].words.size();
  }
  std::memcpy(sl.h_desc, L.desc.data(), n * sizeof(TripletDesc));
  std::memcpy(sl.h_jobs, L.jobs.data(), L.jobs.size() * sizeof(JobDesc));
  for (size_t q = 0; q < n; ++q) sl.h_scores[q] = kPending;

  char* a = sl.arena;
  uint32_t* d_words = (uint32_t*)a;
  a += align256(words * 4);
  TripletDesc* d_desc = (TripletDesc*)a;
  a += align256(n * sizeof(TripletDesc));
  JobDesc* d_jobs = (JobDesc*)a;
  a += align256(L.jobs.size() * sizeof(JobDesc));
  int* d_red = (int*)a;
  a += align256((uint64_t)L.red_pairs() * 8);
  int* d_face = (int*)a;
  int* d_pface = sl.tagged;

  hipError_t e = hipSuccess;
  if (words) e = hipMemcpyAsync(d_words, sl.h_words, words * 4, hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_desc, sl.h_desc, n * sizeof(TripletDesc), hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_jobs, sl.h_jobs, L.jobs.size() * sizeof(JobDesc), hipMemcpyHostToDevice,
                       sl.stream);
  if (e == hipSuccess) e = launch_prepare(sl.ctl, sl.ctl + 64, d_red, L.red_pairs(), sl.stream);
  if (e == hipSuccess) {
    SweepArgs args = make_sweep_args(d_words, d_desc, d_jobs, (uint32_t)L.jobs.size(), L.lds_n0,
                                     sl.d_scores, sl.ctl + 64, sl.ctl, d_face, L.face_stride, d_pface,
                                     s->bnd, d_red, s->dsc);
    e = launch_sweep(L.ks, L.modes, args, grid, sl.stream);
  }
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    *err = std::string("round launch: ") + hipGetErrorString(e);
    return TRIOSEQ_ERR_DEVICE;
  }
  return TRIOSEQ_OK;
}

void worker_main(trioseq_server* s) {
  if (hipSetDevice(s->cfg.device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->worker_error = "hipSetDevice failed in the serving thread";
  }
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // 1. Completions: scores that reached host memory, then finished rounds.
    const uint64_t t = now_ns();
    int busy = 0;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      for (size_t q = 0; q < sl.reqs.size(); ++q) {
        if (sl.reported[q]) continue;
        const int32_t v = __atomic_load_n(&sl.h_scores[q], __ATOMIC_ACQUIRE);
        if (v == kPending) continue;
        sl.reported[q] = 1;
        record_result(s, sl.reqs[q], v, v == INT32_MIN ? TRIOSEQ_ERR_DEVICE : TRIOSEQ_OK, t);
        s->cv_done.notify_all();
      }
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        ++busy;
        continue;
      }
      // Round over (or failed): report whatever is left.
      for (size_t r = 0; r < sl.reqs.size(); ++r) {
        if (sl.reported[r]) continue;
        const int32_t v = __atomic_load_n(&sl.h_scores[r], __ATOMIC_ACQUIRE);
        const bool ok = q == hipSuccess && v != kPending && v != INT32_MIN;
        record_result(s, sl.reqs[r], ok ? v : 0, ok ? TRIOSEQ_OK : TRIOSEQ_ERR_DEVICE, t);
      }
      sl.reqs.clear();
      sl.reported.clear();
      sl.busy = false;
      s->cv_done.notify_all();
    }
    if (busy == 0 && s->busy_since) {
      s->busy_s += (double)(t - s->busy_since) * 1e-9;
      s->busy_since = 0;
    }
    // 2. Admission: fill free slots with queued requests.
    for (Slot& sl : s->slots) {
      if (sl.busy || s->pending.empty()) continue;
      // Take requests first-come first-served up to the slot's batch size;
      // shrink until the round's footprint fits the slot.
      size_t take = std::min<size_t>(s->pending.size(), sl.max_batch);
      std::vector<Request> batch;
      batch.reserve(take);
      for (size_t q = 0; q < take; ++q) {
        batch.push_back(std::move(s->pending.front()));
        s->pending.pop_front();
      }
      lk.unlock();
      Layout L;
      std::string err;
      trioseq_status st = TRIOSEQ_ERR_TOO_LARGE;
      std::vector<Request> back;
      while (!batch.empty()) {
        st = launch_round(s, sl, batch, &L, &err, busy == 0);
        if (st != TRIOSEQ_ERR_TOO_LARGE || batch.size() == 1) break;
        // Does not fit: return the second half to the queue front.
        const size_t keep = batch.size() / 2;
        for (size_t q = batch.size(); q > keep; --q) back.push_back(std::move(batch[q - 1]));
        batch.resize(keep);
      }
      lk.lock();
      for (Request& r : back) s->pending.push_front(std::move(r));
      if (st == TRIOSEQ_OK) {
        sl.reqs = std::move(batch);
        sl.reported.assign(sl.reqs.size(), 0);
        sl.busy = true;
        sl.t_launch = now_ns();
        s->rounds++;
        if (!s->busy_since) s->busy_since = sl.t_launch;
        ++busy;
      } else {
        for (Request& r : batch) record_result(s, r, 0, st, now_ns());
        s->cv_done.notify_all();
      }
    }
    // 3. Exit once closed and drained.
    if (s->closing && s->pending.empty() && busy == 0) break;
    // 4. Sleep: poll quickly while rounds run, else wait for work.
    if (busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    else
      s->cv_work.wait(lk, [&] { return s->closing || !s->pending.empty(); });
  }
}

void free_server(trioseq_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    (void)hipFree(sl.arena);
    (void)hipFree(sl.tagged);
    (void)hipFree(sl.ctl);
    (void)hipHostFree(sl.h_words);
    (void)hipHostFree(sl.h_desc);
    (void)hipHostFree(sl.h_jobs);
    (void)hipHostFree(sl.h_scores);
  }
  (void)hipFree(s->d_bnd);
  delete s;
}

}  // namespace

extern "C" {

static trioseq_status trioseq_serve_create_body(const trioseq_serve_config* cfg, const trioseq_scoring* sc,
                                    trioseq_server** out) {
  if (!cfg || !sc || !out) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_create: NULL pointer");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  if (cfg->max_len == 0 || cfg->max_len > (uint32_t)kMaxSweepLen)
    return fail(TRIOSEQ_ERR_INVALID_ARG,
                "serve_create: max_len must be in [1, " + std::to_string(kMaxSweepLen) + "]");
  st = check_range(*sc, cfg->max_len, cfg->max_len, cfg->max_len, 0);
  if (st != TRIOSEQ_OK) return st;
  if (hipSetDevice(cfg->device) != hipSuccess)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_create: bad device");
  trioseq_server* s = new (std::nothrow) trioseq_server;
  if (!s) return fail(TRIOSEQ_ERR_NOMEM, "serve_create: host allocation");
  s->cfg = *cfg;
  if (!s->cfg.max_queue) s->cfg.max_queue = 1u << 20;
  if (!s->cfg.max_batch) s->cfg.max_batch = 4096;
  if (!s->cfg.max_inflight) s->cfg.max_inflight = kDefaultInflight;
  if (s->cfg.max_inflight > kMaxInflight) {
    delete s;
    return fail(TRIOSEQ_ERR_INVALID_ARG,
                "serve_create: max_inflight must be at most " + std::to_string(kMaxInflight));
  }
  try {
    s->slots.resize(s->cfg.max_inflight);
  } catch (...) {
    delete s;
    return fail(TRIOSEQ_ERR_NOMEM, "serve_create: host allocation");
  }
  s->sc = *sc;
  s->dsc = make_dev_scoring(*sc);
  st = device_props(&s->dp);
  if (st != TRIOSEQ_OK) {
    delete s;
    return st;
  }
  uint64_t budget = cfg->max_device_bytes ? cfg->max_device_bytes : s->dp.hbm_bytes / 4;
  const uint64_t per_slot = budget / s->cfg.max_inflight / 256 * 256;
  // The largest single request must fit a slot on its own. A slot's tagged
  // region is sized for that request's panel faces; the rest of the slot
  // budget is its arena.
  uint64_t tagged_bytes = 0;
  {
    const uint32_t m = cfg->max_len;
    const uint32_t lens[3] = {m, m, m};
    Layout L;
    trioseq_plan_options o{-1, s->ks.rj, s->ks.rk, 0, 0, 0};
    st = build_layout(lens, nullptr, 1, *sc, o, s->dp.cus * kWavesPerCuHint, &L);
    int grid = 0, wpc = 0;
    if (st == TRIOSEQ_OK) st = layout_grid(L, s->dp, 0, &grid, &wpc);
    if (st != TRIOSEQ_OK) {
      delete s;
      return st;
    }
    tagged_bytes = align256(L.pool_ints * 4);
    if (tagged_bytes >= per_slot ||
        arena_need(L, 3ull * ((m + 15) / 16), grid) > per_slot - tagged_bytes) {
      delete s;
      return fail(TRIOSEQ_ERR_TOO_LARGE, "serve_create: max_device_bytes too small for max_len");
    }
  }
  auto bail = [&](hipError_t e, const char* what) {
    fail_hip(e, what);
    free_server(s);
    return e == hipErrorOutOfMemory ? TRIOSEQ_ERR_NOMEM : TRIOSEQ_ERR_DEVICE;
  };
  hipError_t e;
  const uint64_t bnd_ints = boundary_ints(s->ks, cfg->max_len);
  if ((e = hipMalloc((void**)&s->d_bnd, bnd_ints * 4)) != hipSuccess) return bail(e, "hipMalloc");
  s->bnd = carve_boundary(s->ks, cfg->max_len, s->d_bnd);
  if ((e = launch_init_boundary(s->ks, s->bnd, nullptr)) != hipSuccess) return bail(e, "boundary init");
  const uint64_t max_words = (uint64_t)s->cfg.max_batch * 3 * ((cfg->max_len + 15) / 16);
  const uint64_t max_jobs = (uint64_t)s->cfg.max_batch + 65536;
  for (Slot& sl : s->slots) {
    sl.max_batch = s->cfg.max_batch;
    sl.arena_bytes = per_slot - tagged_bytes;
    sl.tagged_bytes = tagged_bytes;
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess)
      return bail(e, "hipStreamCreate");
    if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
      return bail(e, "hipEventCreate");
    if ((e = hipMalloc((void**)&sl.arena, sl.arena_bytes)) != hipSuccess) return bail(e, "hipMalloc arena");
    if (tagged_bytes) {
      if ((e = hipMalloc((void**)&sl.tagged, tagged_bytes)) != hipSuccess)
        return bail(e, "hipMalloc tagged faces");
      // Tag 0 belongs to no run (generations start at 1).
      if ((e = hipMemset(sl.tagged, 0, tagged_bytes)) != hipSuccess) return bail(e, "hipMemset");
    }
    if ((e = hipMalloc((void**)&sl.ctl, 512)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMemset(sl.ctl, 0, 512)) != hipSuccess) return bail(e, "hipMemset");
    sl.h_words_cap = max_words;
    sl.h_meta_cap = max_jobs;
    if ((e = hipHostMalloc((void**)&sl.h_words, std::max<uint64_t>(max_words, 1) * 4, 0)) != hipSuccess)
      return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc((void**)&sl.h_desc, max_jobs * sizeof(TripletDesc), 0)) != hipSuccess)
      return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc((void**)&sl.h_jobs, max_jobs * sizeof(JobDesc), 0)) != hipSuccess)
      return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc((void**)&sl.h_scores, sl.max_batch * 4, hipHostMallocMapped)) != hipSuccess)
      return bail(e, "hipHostMalloc scores");
    if ((e = hipHostGetDevicePointer((void**)&sl.d_scores, sl.h_scores, 0)) != hipSuccess)
      return bail(e, "hipHostGetDevicePointer");
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(e, "serve_create");
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    free_server(s);
    return fail(TRIOSEQ_ERR_NOMEM, "serve_create: cannot start the serving thread");
  }
  *out = s;
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_serve_submit_body(trioseq_server* s, const trioseq_triplet* t, uint64_t* id) {
  if (!s || !t || !id) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_submit: NULL pointer");
  Request r;
  uint64_t words = 0;
  for (int a = 0; a < 3; ++a) {
    if (t->len[a] > s->cfg.max_len)
      return fail(TRIOSEQ_ERR_TOO_LARGE, "serve_submit: sequence longer than max_len");
    if (t->len[a] && !t->seq[a]) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_submit: NULL sequence");
    r.len[a] = t->len[a];
    r.woff[a] = (uint32_t)words;
    words += (t->len[a] + 15) / 16;
  }
  trioseq_status st = check_range(s->sc, r.len[0], r.len[1], r.len[2], 0);
  if (st != TRIOSEQ_OK) return st;
  r.words.assign(words, 0u);
  for (int a = 0; a < 3; ++a) {
    st = trioseq_pack(t->seq[a], t->len[a], r.words.data() + r.woff[a]);
    if (st != TRIOSEQ_OK) return st;
  }
  r.cells = (double)r.len[0] * r.len[1] * r.len[2];
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->closing) return fail(TRIOSEQ_ERR_CLOSED, "serve_submit: server is shutting down");
  if (s->pending.size() >= s->cfg.max_queue) return fail(TRIOSEQ_ERR_BUSY, "serve_submit: queue full");
  r.id = s->next_id++;
  r.t_submit = now_ns();
  *id = r.id;
  s->outstanding.insert(r.id);
  s->pending.push_back(std::move(r));
  s->submitted++;
  s->cv_work.notify_one();
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_serve_poll_body(trioseq_server* s, trioseq_result* out, size_t cap, size_t* n_out) {
  if (!s || !n_out || (cap && !out)) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_poll: NULL pointer");
  std::lock_guard<std::mutex> lk(s->mu);
  size_t k = 0;
  while (k < cap && !s->done_fifo.empty()) {
    const uint64_t id = s->done_fifo.front();
    s->done_fifo.pop_front();
    auto it = s->done.find(id);
    if (it == s->done.end()) continue;  // already taken by serve_wait
    out[k++] = it->second;
    s->done.erase(it);
    s->outstanding.erase(id);
  }
  *n_out = k;
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_serve_wait_body(trioseq_server* s, uint64_t id, trioseq_result* out,
                                  int64_t timeout_ns) {
  if (!s || !out) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_wait: NULL pointer");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->outstanding.count(id)) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_wait: unknown request id");
  auto ready = [&] { return s->done.count(id) != 0; };
  if (timeout_ns < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
    return fail(TRIOSEQ_ERR_TIMEOUT, "serve_wait: timed out");
  }
  auto it = s->done.find(id);
  *out = it->second;
  s->done.erase(it);
  s->outstanding.erase(id);
  return TRIOSEQ_OK;
}

static trioseq_status trioseq_serve_get_stats_body(trioseq_server* s, trioseq_serve_stats* st) {
  if (!s || !st) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_get_stats: NULL pointer");
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->rounds = s->rounds;
    st->cells = s->cells;
    st->busy_s = s->busy_s + (s->busy_since ? (double)(now_ns() - s->busy_since) * 1e-9 : 0.0);
    lat = s->lat_ns;
  }
  st->gcups = st->busy_s > 0 ? st->cells / st->busy_s / 1e9 : 0.0;
  st->p50_ns = st->p99_ns = 0;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
      size_t k = (size_t)(p * (double)(lat.size() - 1) + 0.5);
      return lat[std::min(k, lat.size() - 1)];
    };
    st->p50_ns = pct(0.50);
    st->p99_ns = pct(0.99);
  }
  return TRIOSEQ_OK;
}

trioseq_status trioseq_serve_destroy(trioseq_server* s) {
  if (!s) return fail(TRIOSEQ_ERR_INVALID_ARG, "serve_destroy: NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipDeviceSynchronize();
  free_server(s);
  return TRIOSEQ_OK;
}

}  // extern "C"

// Entry points: every body runs guarded (no exception crosses the ABI).
extern "C" {

trioseq_status trioseq_serve_create(const trioseq_serve_config* cfg, const trioseq_scoring* sc, trioseq_server** out) {
  return guarded([&] { return trioseq_serve_create_body(cfg, sc, out); });
}

trioseq_status trioseq_serve_submit(trioseq_server* s, const trioseq_triplet* t, uint64_t* id) {
  return guarded([&] { return trioseq_serve_submit_body(s, t, id); });
}

trioseq_status trioseq_serve_poll(trioseq_server* s, trioseq_result* out, size_t cap, size_t* n_out) {
  return guarded([&] { return trioseq_serve_poll_body(s, out, cap, n_out); });
}

trioseq_status trioseq_serve_wait(trioseq_server* s, uint64_t id, trioseq_result* out, int64_t timeout_ns) {
  return guarded([&] { return trioseq_serve_wait_body(s, id, out, timeout_ns); });
}

trioseq_status trioseq_serve_stats_get(trioseq_server* s, trioseq_serve_stats* st) {
  return guarded([&] { return trioseq_serve_get_stats_body(s, st); });
}

trioseq_status trioseq_serve_get_stats(trioseq_server* s, trioseq_serve_stats* st) {
  return trioseq_serve_stats_get(s, st);
}

}  // extern "C"

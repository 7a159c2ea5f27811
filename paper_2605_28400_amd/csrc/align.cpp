// Traceback: optimal global alignments of triplets (paper, Section II, Eq. 1;
// the paper returns alignments by Hirschberg's linear-space divide and
// conquer), computed level by level on the GPU for a whole batch at once:
//  * every box (sub-problem) larger than kLeafCells table cells is halved on
//    its longest axis; one batched plane run per level sweeps, for every such
//    box, the first half forward and the second half reversed, and k_split
//    picks where an optimal alignment of the box crosses the middle slice;
//  * the remaining small boxes are solved whole by k_leaf (table and walk
//    back), and their columns, in path order, are the alignment.
// The host only lays out the boxes, moves data and formats the rows.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"

namespace trioseq {
namespace {

struct Box {
  uint32_t trip;
  uint32_t lo[3], hi[3];
  uint64_t cells() const {
    return (uint64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  }
  uint64_t corner() const { return (uint64_t)lo[0] + lo[1] + lo[2]; }
};

template <class T>
T* as(const PlaneWorkspace::Buf& b) {
  return (T*)b.p;
}

// Appends codes[from, to) (reversed if asked), packed 16 per word from a
// fresh word; returns its word offset.
uint64_t pack_range(const std::vector<uint8_t>& codes, uint32_t from, uint32_t to, bool reverse,
                    std::vector<uint32_t>& words) {
  const uint64_t off = words.size();
  const uint32_t n = to - from;
  words.resize(off + (n + 15) / 16, 0u);
  for (uint32_t p = 0; p < n; ++p) {
    const uint8_t c = reverse ? codes[to - 1 - p] : codes[from + p];
    words[off + p / 16] |= (uint32_t)c << (2 * (p % 16));
  }
  return off;
}

trioseq_status hip_err(hipError_t e, const char* what) { return fail_hip(e, what); }

// Leaves solved per k_leaf launch (bounds the column buffers of a launch).
constexpr size_t kLeavesPerLaunch = 1 << 18;

// Traceback workspace of this thread (see align_batch_impl).
constexpr uint64_t kKeepBytes = 2ull << 30;
thread_local PlaneWorkspace* g_ws = nullptr;
thread_local int g_ws_device = -1;

// One level: every box in `boxes` is split; its two children go to `next`.
// root_score[t] is set when the box is triplet t's root (its first split).
trioseq_status split_level(PlaneWorkspace& ws, const std::vector<Box>& boxes,
                           const std::vector<std::vector<uint8_t>>& codes, const trioseq_scoring& sc,
                           std::vector<char>& split_seen, std::vector<int32_t>& root_score,
                           std::vector<Box>& next, hipStream_t s) {
  const size_t nb = boxes.size();
  // Triplet 2q = first half of box q forward, 2q + 1 = second half reversed;
  // the halved axis is swept, the other two stay in index order.
  std::vector<uint32_t> lens(6 * nb), words;
  std::vector<uint64_t> offs(6 * nb), poff(2 * nb);
  std::vector<SplitDesc> sd(nb);
  std::vector<uint32_t> chunk_box;
  std::vector<int> axes(3 * nb);
  std::vector<uint32_t> mids(nb);
  uint64_t pints = 0;
  for (size_t q = 0; q < nb; ++q) {
    const Box& b = boxes[q];
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (b.hi[a] - b.lo[a] > b.hi[ax] - b.lo[ax]) ax = a;
    const int r = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;
    const uint32_t mid = b.lo[ax] + (b.hi[ax] - b.lo[ax]) / 2;
    axes[3 * q] = ax;
    axes[3 * q + 1] = r;
    axes[3 * q + 2] = c;
    mids[q] = mid;
    const int order[3] = {ax, r, c};
    for (int half = 0; half < 2; ++half) {
      const size_t tr = 2 * q + half;
      for (int sidx = 0; sidx < 3; ++sidx) {
        const int a = order[sidx];
        uint32_t from = b.lo[a], to = b.hi[a];
        if (sidx == 0) (half == 0 ? to : from) = mid;
        lens[3 * tr + sidx] = to - from;
        offs[3 * tr + sidx] = pack_range(codes[3 * b.trip + a], from, to, half == 1, words);
      }
    }
    const uint32_t prow = b.hi[r] - b.lo[r] + 1, pcol = b.hi[c] - b.lo[c] + 1;
    poff[2 * q] = pints;
    pints += (uint64_t)prow * pcol;
    poff[2 * q + 1] = pints;
    pints += (uint64_t)prow * pcol;
    const uint32_t nchunk = (uint32_t)(((uint64_t)prow * pcol + kSplitChunk - 1) / kSplitChunk);
    sd[q] = SplitDesc{poff[2 * q], poff[2 * q + 1], prow, pcol, (uint32_t)chunk_box.size(), nchunk};
    chunk_box.insert(chunk_box.end(), nchunk, (uint32_t)q);
  }
  trioseq_status st = run_planes(ws, lens.data(), offs.data(), 2 * nb, words.data(), words.size(), sc,
                                 poff.data(), pints, s);
  if (st != TRIOSEQ_OK) return st;
  std::vector<int> out(3 * nb);
  const size_t nchunks = chunk_box.size();
  hipError_t e;
  // The level's only wait: its split points are needed to lay out the next.
  if ((e = ws_grow(ws.sd, nb * sizeof(SplitDesc), false, s)) != hipSuccess ||
      (e = ws_grow(ws.split_out, 3 * nb * 4, false, s)) != hipSuccess ||
      (e = ws_grow(ws.chunk_box, nchunks * 4, false, s)) != hipSuccess ||
      (e = ws_grow(ws.partial, nchunks * 8, false, s)) != hipSuccess ||
      (e = hipMemcpyAsync(ws.sd.p, sd.data(), nb * sizeof(SplitDesc), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(ws.chunk_box.p, chunk_box.data(), nchunks * 4, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = launch_split((const int*)ws.plane.p, as<SplitDesc>(ws.sd), (uint32_t)nb, as<uint32_t>(ws.chunk_box),
                        (uint32_t)nchunks, as<int>(ws.partial), as<int>(ws.split_out), s)) != hipSuccess ||
      (e = hipMemcpyAsync(out.data(), ws.split_out.p, 3 * nb * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_err(e, "align: split");
  for (size_t q = 0; q < nb; ++q) {
    const Box& b = boxes[q];
    const int ax = axes[3 * q], r = axes[3 * q + 1], c = axes[3 * q + 2];
    const uint32_t p = (uint32_t)out[3 * q + 1], pc = (uint32_t)out[3 * q + 2];
    if (p > b.hi[r] - b.lo[r] || pc > b.hi[c] - b.lo[c])
      return fail(TRIOSEQ_ERR_DEVICE, "align: split point outside its box");
    if (!split_seen[b.trip]) {  // a triplet's first split is of its root box
      split_seen[b.trip] = 1;
      root_score[b.trip] = out[3 * q];
    }
    Box left = b, right = b;
    left.hi[ax] = mids[q];
    right.lo[ax] = mids[q];
    left.hi[r] = right.lo[r] = b.lo[r] + p;
    left.hi[c] = right.lo[c] = b.lo[c] + pc;
    next.push_back(left);
    next.push_back(right);
  }
  return TRIOSEQ_OK;
}

// Solves leaves[first, first + n) with k_leaf; columns and scores to host.
trioseq_status solve_leaves(PlaneWorkspace& ws, const std::vector<Box>& leaves, size_t first, size_t n,
                            const std::vector<uint32_t>& words, const std::vector<uint64_t>& soff,
                            const trioseq_scoring& sc, std::vector<LeafDesc>& ld,
                            std::vector<uint8_t>& cols, std::vector<uint32_t>& ncols,
                            std::vector<int32_t>& lscore, hipStream_t s) {
  ld.assign(n, LeafDesc{});
  uint64_t col_bytes = 0;
  for (size_t q = 0; q < n; ++q) {
    const Box& b = leaves[first + q];
    if (b.cells() > kLeafCells) return fail(TRIOSEQ_ERR_DEVICE, "align: leaf larger than its table");
    for (int a = 0; a < 3; ++a) {
      ld[q].off[a] = soff[3 * b.trip + a];
      ld[q].lo[a] = b.lo[a];
      ld[q].len[a] = b.hi[a] - b.lo[a];
    }
    ld[q].out = col_bytes;
    col_bytes += 3ull * (ld[q].len[0] + ld[q].len[1] + ld[q].len[2]);
  }
  cols.assign(col_bytes, 0);
  ncols.assign(n, 0);
  lscore.assign(n, 0);
  hipError_t e;
  if ((e = ws_grow(ws.lwords, words.size() * 4, false, s)) != hipSuccess ||
      (e = ws_grow(ws.leaves, n * sizeof(LeafDesc), false, s)) != hipSuccess ||
      (e = ws_grow(ws.cols, col_bytes, false, s)) != hipSuccess ||
      (e = ws_grow(ws.ncols, n * 4, false, s)) != hipSuccess ||
      (e = ws_grow(ws.lscore, n * 4, false, s)) != hipSuccess)
    return hip_err(e, "align: leaf buffers");
  LeafArgs la;
  la.words = as<uint32_t>(ws.lwords);
  la.leaves = as<LeafDesc>(ws.leaves);
  la.n = (uint32_t)n;
  la.cols = as<uint8_t>(ws.cols);
  la.ncols = as<uint32_t>(ws.ncols);
  la.score = as<int32_t>(ws.lscore);
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) la.sub[4 * x + y] = sc.sub[x][y];
  la.gap = sc.gap;
  if ((e = hipMemcpyAsync(ws.lwords.p, words.data(), words.size() * 4, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(ws.leaves.p, ld.data(), n * sizeof(LeafDesc), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = launch_leaf(la, s)) != hipSuccess ||
      (e = hipMemcpyAsync(cols.data(), ws.cols.p, col_bytes, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(ncols.data(), ws.ncols.p, n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(lscore.data(), ws.lscore.p, n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_err(e, "align: leaves");
  return TRIOSEQ_OK;
}

// rows: triplet u's row a at rows + 3 * cap_before[u] + a * cap[u].
trioseq_status align_batch_impl(const trioseq_triplet* t, size_t n, const trioseq_scoring& sc,
                                char* rows, uint32_t* ncols_out, int32_t* scores_out, hipStream_t s) {
  std::vector<std::vector<uint8_t>> codes(3 * n);
  std::vector<uint64_t> cap(n), cap_before(n);
  uint64_t total_cap = 0;
  for (size_t u = 0; u < n; ++u) {
    for (int q = 0; q < 3; ++q) {
      if (t[u].len[q] && !t[u].seq[q]) return fail(TRIOSEQ_ERR_INVALID_ARG, "align: NULL sequence");
      if (t[u].len[q] > (uint32_t)kMaxSweepLen)
        return fail(TRIOSEQ_ERR_TOO_LARGE, "align: triplet " + std::to_string(u) +
                                               ": every length must be at most " +
                                               std::to_string(kMaxSweepLen));
      std::vector<uint8_t>& cq = codes[3 * u + q];
      cq.resize(t[u].len[q]);
      for (uint32_t p = 0; p < t[u].len[q]; ++p) {
        const uint8_t c = residue_code(t[u].seq[q][p]);
        if (c > 3) return fail(TRIOSEQ_ERR_BAD_RESIDUE, "align: residue outside ACGT");
        cq[p] = c;
      }
    }
    trioseq_status st = check_range(sc, t[u].len[0], t[u].len[1], t[u].len[2], u);
    if (st != TRIOSEQ_OK) return st;
    cap[u] = (uint64_t)t[u].len[0] + t[u].len[1] + t[u].len[2];
    cap_before[u] = total_cap;
    total_cap += cap[u];
  }
  if (n == 0) return TRIOSEQ_OK;

  std::vector<Box> work, leaves;
  for (size_t u = 0; u < n; ++u) work.push_back(Box{(uint32_t)u, {0, 0, 0}, {t[u].len[0], t[u].len[1], t[u].len[2]}});
  std::vector<char> split_seen(n, 0);
  std::vector<int32_t> root_score(n, 0);
  // This thread's traceback workspace, kept from call to call (and from
  // level to level) so that a repeated alignment allocates nothing; one
  // grown past kKeepBytes is released when the call ends.
  int device = 0;
  TRIOSEQ_HIP(hipGetDevice(&device), "hipGetDevice");
  if (!g_ws || g_ws_device != device) {
    delete g_ws;  // the previous device's buffers (synchronous calls: idle)
    g_ws = new PlaneWorkspace;
    g_ws_device = device;
  }
  PlaneWorkspace& ws = *g_ws;
  struct Release {
    ~Release() {
      if (g_ws && ws_bytes(*g_ws) > kKeepBytes) {
        delete g_ws;
        g_ws = nullptr;
      }
    }
  } release;
  while (!work.empty()) {
    std::vector<Box> boxes, next;
    for (const Box& b : work) (b.cells() <= kLeafCells ? leaves : boxes).push_back(b);
    if (boxes.empty()) break;
    trioseq_status st = split_level(ws, boxes, codes, sc, split_seen, root_score, next, s);
    if (st != TRIOSEQ_OK) return st;
    work.swap(next);
  }

  // Leaves in path order per triplet: along an alignment every coordinate
  // grows, and a leaf holds at least one residue, so the sum of a leaf's
  // lower corner strictly increases from leaf to leaf.
  std::sort(leaves.begin(), leaves.end(), [](const Box& x, const Box& y) {
    return x.trip != y.trip ? x.trip < y.trip : x.corner() < y.corner();
  });
  std::vector<uint32_t> words;
  std::vector<uint64_t> soff(3 * n);
  for (size_t u = 0; u < n; ++u)
    for (int q = 0; q < 3; ++q) soff[3 * u + q] = pack_range(codes[3 * u + q], 0, t[u].len[q], false, words);
  std::vector<std::string> out(3 * n);
  std::vector<int64_t> sum(n, 0);
  static const char kLetter[5] = {'A', 'C', 'G', 'T', '-'};
  std::vector<LeafDesc> ld;
  std::vector<uint8_t> cols;
  std::vector<uint32_t> ncols;
  std::vector<int32_t> lscore;
  for (size_t first = 0; first < leaves.size(); first += kLeavesPerLaunch) {
    const size_t cnt = std::min(kLeavesPerLaunch, leaves.size() - first);
    trioseq_status st = solve_leaves(ws, leaves, first, cnt, words, soff, sc, ld, cols, ncols, lscore, s);
    if (st != TRIOSEQ_OK) return st;
    for (size_t q = 0; q < cnt; ++q) {
      const uint32_t u = leaves[first + q].trip;
      const uint64_t most = (uint64_t)ld[q].len[0] + ld[q].len[1] + ld[q].len[2];
      if (ncols[q] > most) return fail(TRIOSEQ_ERR_DEVICE, "align: leaf wrote too many columns");
      sum[u] += lscore[q];
      const uint8_t* c = cols.data() + ld[q].out;
      for (int64_t k = (int64_t)ncols[q] - 1; k >= 0; --k)  // written last column first
        for (int a = 0; a < 3; ++a) {
          const uint8_t v = c[3 * k + a];
          if (v > 4) return fail(TRIOSEQ_ERR_DEVICE, "align: bad column code");
          out[3 * u + a].push_back(kLetter[v]);
        }
    }
  }
  // Checks before any output is written: the leaves' scores add up to the
  // alignment's score (the sum-of-pairs score is a sum over columns), which
  // must be the root box's optimum, and every row holds its whole sequence.
  for (size_t u = 0; u < n; ++u) {
    const int64_t total = split_seen[u] ? root_score[u] : sum[u];
    if (sum[u] != total) return fail(TRIOSEQ_ERR_DEVICE, "align: leaf scores do not add up to the optimum");
    if (out[3 * u].size() > cap[u]) return fail(TRIOSEQ_ERR_DEVICE, "align: too many columns");
    for (int a = 0; a < 3; ++a) {
      const std::string& r = out[3 * u + a];
      if (r.size() != out[3 * u].size() ||
          (uint64_t)std::count_if(r.begin(), r.end(), [](char ch) { return ch != '-'; }) != t[u].len[a])
        return fail(TRIOSEQ_ERR_DEVICE, "align: a row does not hold its whole sequence");
    }
  }
  for (size_t u = 0; u < n; ++u) {
    for (int a = 0; a < 3; ++a)
      std::memcpy(rows + 3 * cap_before[u] + a * cap[u], out[3 * u + a].data(), out[3 * u + a].size());
    ncols_out[u] = (uint32_t)out[3 * u].size();
    scores_out[u] = (int32_t)sum[u];
  }
  return TRIOSEQ_OK;
}

}  // namespace
}  // namespace trioseq

using namespace trioseq;

static trioseq_status trioseq_align_batch_body(const trioseq_triplet* t, size_t n,
                                              const trioseq_scoring* sc, char* rows, uint32_t* ncols,
                                              int32_t* scores, void* hip_stream) {
  if (!sc || (n && (!t || !rows || !ncols || !scores)))
    return fail(TRIOSEQ_ERR_INVALID_ARG, "align_batch: NULL pointer");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  if (sc->kind != kGlobal) return fail(TRIOSEQ_ERR_INVALID_ARG, "align: only global alignments");
  return align_batch_impl(t, n, *sc, rows, ncols, scores, (hipStream_t)hip_stream);
}

static trioseq_status trioseq_align_body(const trioseq_triplet* t, const trioseq_scoring* sc,
                                        char* row0, char* row1, char* row2, uint32_t cap,
                                        uint32_t* ncols, int32_t* score, void* hip_stream) {
  if (!t || !sc || !row0 || !row1 || !row2 || !ncols || !score)
    return fail(TRIOSEQ_ERR_INVALID_ARG, "align: NULL pointer");
  trioseq_status st = validate_scoring(sc);
  if (st != TRIOSEQ_OK) return st;
  if (sc->kind != kGlobal) return fail(TRIOSEQ_ERR_INVALID_ARG, "align: only global alignments");
  const uint64_t need = (uint64_t)t->len[0] + t->len[1] + t->len[2];
  if (cap < need) return fail(TRIOSEQ_ERR_INVALID_ARG, "align: row capacity below the sum of the lengths");
  std::vector<char> buf(3 * need + 1);
  uint32_t nc = 0;
  int32_t sco = 0;
  st = align_batch_impl(t, 1, *sc, buf.data(), &nc, &sco, (hipStream_t)hip_stream);
  if (st != TRIOSEQ_OK) return st;
  std::memcpy(row0, buf.data(), nc);
  std::memcpy(row1, buf.data() + need, nc);
  std::memcpy(row2, buf.data() + 2 * need, nc);
  *ncols = nc;
  *score = sco;
  return TRIOSEQ_OK;
}

// Entry points: every body runs guarded (no exception crosses the ABI).
extern "C" {

trioseq_status trioseq_align_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc, char* rows, uint32_t* ncols, int32_t* scores, void* hip_stream) {
  return guarded([&] { return trioseq_align_batch_body(t, n, sc, rows, ncols, scores, hip_stream); });
}

trioseq_status trioseq_align(const trioseq_triplet* t, const trioseq_scoring* sc, char* row0, char* row1, char* row2, uint32_t cap, uint32_t* ncols, int32_t* score, void* hip_stream) {
  return guarded([&] { return trioseq_align_body(t, sc, row0, row1, row2, cap, ncols, score, hip_stream); });
}

}  // extern "C"

// Host-side helpers shared by the plan and server implementations.
#pragma once
#include <stdint.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/trioseq.h"
#include "internal.h"

namespace trioseq {

trioseq_status fail(trioseq_status st, const std::string& msg);

// Runs an entry point's body so that no C++ exception leaves the C ABI:
// a failed host allocation becomes TRIOSEQ_ERR_NOMEM, anything else
// TRIOSEQ_ERR_DEVICE.
template <class F>
trioseq_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(TRIOSEQ_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(TRIOSEQ_ERR_DEVICE, "unexpected host exception");
  }
}
trioseq_status fail_hip(hipError_t e, const char* what);
#define TRIOSEQ_HIP(call, what)                              \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return ::trioseq::fail_hip(e_, what); \
  } while (0)

// Residue code (0..3 for ACGT in either case) of an ASCII character, or 255.
uint8_t residue_code(char ch);

trioseq_status validate_scoring(const trioseq_scoring* sc);
// Checks that the shifted score range of a triplet with these lengths keeps
// int32 headroom under this scoring.
trioseq_status check_range(const trioseq_scoring& sc, uint64_t a, uint64_t b, uint64_t c,
                           size_t index);
DevScoring make_dev_scoring(const trioseq_scoring& sc);

// Per-triplet plan: which input sequence goes on which axis.
struct AxisChoice {
  uint8_t perm[3];  // perm[axis] = input sequence index
};
AxisChoice choose_axes_batch(const uint32_t len[3], const KernelShape& ks);
AxisChoice choose_axes_wide(const uint32_t len[3]);
uint64_t panel_steps(const uint32_t len_axis[3], const KernelShape& ks);
extern const double kSplitCells;

struct DeviceProps {
  int device;
  int cus;
  size_t hbm_bytes;
};
trioseq_status device_props(DeviceProps* p);

uint64_t now_ns();

// Sentinel-face buffers for sweeps up to max_n0 (plain + tagged layouts).
uint64_t boundary_ints(const KernelShape& ks, uint32_t max_n0);
Boundary carve_boundary(const KernelShape& ks, uint32_t max_n0, int* base);
SweepArgs make_sweep_args(const uint32_t* words, const TripletDesc* desc, const JobDesc* jobs,
                          uint32_t njobs, uint32_t lds_n0, int32_t* scores, int* counter, int* ctl,
                          int* face, uint64_t face_stride, int* pface, const Boundary& bnd,
                          int* red, const DevScoring& sc);

// Host-side plan of one batch: validation, per-triplet axis choice, the job
// queue in dependency order, and the device memory the sweep needs.
struct Layout {
  KernelShape ks{4, 4, 2};
  int kind = 0;    // alignment kind of the scoring
  bool planes = false;  // last-slice planes are written (traceback)
  int modes = 1;   // bit 0 whole-triplet jobs, bit 1 panel jobs
  int engine = 0;  // 0 all whole, 1 all split, 2 mixed
  int panels = 0;
  uint32_t lds_n0 = 0;
  double cells = 0;
  std::vector<TripletDesc> desc;
  std::vector<JobDesc> jobs;
  uint64_t face_stride = 0;  // ints of whole-triplet workspace per wave
  uint64_t pool_ints = 0;    // ints of panel faces of split triplets
  // Packed pairs: desc holds pair p as entries 2p, 2p + 1 and every job is a
  // pair; pk_base is the stored value of M' = 0, pk_kc the offset of
  // semi-global candidates (see sweep.hip).
  bool packed = false;
  uint32_t pk_base = 0;
  uint32_t pk_kc = 0;
  // Per-triplet reduction pairs the run needs (semi-global and local scoring
  // of split triplets): 2 * red_pairs ints.
  uint32_t red_pairs() const { return kind != 0 && (modes & 2) ? (uint32_t)desc.size() : 0u; }
};

// Validates and lays out n triplets (lens[3t+s], word offsets off[3t+s]).
// Touches no device state.
// waves_hint: wavefronts the launch will have (for the split rule).
// planes: the layout of a traceback plane run (axes kept as given, S0 swept).
trioseq_status build_layout(const uint32_t* lens, const uint64_t* off, size_t n,
                            const trioseq_scoring& sc, const trioseq_plan_options& o, int waves_hint,
                            Layout* L, bool planes = false);
// Pairs per workgroup of panel-only plans unless the options say otherwise.
constexpr int kDefaultPanelGroup = 1;
// Lane exchange (KernelShape::xch) unless the options say otherwise.
constexpr int kDefaultLaneExchange = 0;
// Resident wavefronts per compute unit assumed when sizing the split rule.
constexpr int kWavesPerCuHint = 8;
// Autotuning cache keyed by a batch's length profile and scoring kind.
std::string length_profile(const uint32_t* lens, size_t n, int kind);
void apply_tuned(const uint32_t* lens, size_t n, int kind, trioseq_plan_options* o);

// Waves to launch for a layout on this device.
trioseq_status layout_grid(const Layout& L, const DeviceProps& dp, int requested, int* grid,
                           int* waves_per_cu);

// Device memory a plan is carved from instead of allocated (the
// allocation-free entry point). plain: any data, carved in order; pool: only
// ever (value, tag) face pairs at even int offsets from its fixed base, or the
// zeros it started with, so a tag slot never holds a value; ctl (generation
// word, error flag, half-split meeting counter, at least 3 ints, zeroed
// before first use) and counter (queue head) persist from call to call, and
// the generation only grows, so no stale tag ever looks current. stream:
// where the plan's initialisation runs (the caller's).
struct PlanMemory {
  uint8_t* plain;
  uint64_t plain_bytes;
  int* pool;
  uint64_t pool_bytes;
  int* ctl;
  int* counter;
  hipStream_t stream;
};
// trioseq_score_batch_packed with every device buffer carved from mem: lays
// the batch out, initialises and enqueues one run on mem.stream.
trioseq_status score_packed_in_region(const uint32_t* d_words, const uint64_t* d_word_off,
                                      const uint32_t* d_len, size_t n, const trioseq_scoring* sc,
                                      int32_t* d_scores, const PlanMemory& mem);

// Traceback plane runs: sweeps of triplets that also write each triplet's
// last slice (unshifted), triplet t at plane + plane_off[t]. The device
// buffers live in a PlaneWorkspace and are reused from run to run (grown when
// a run needs more), so the levels of an alignment allocate almost nothing;
// the generation word is shared by the runs, so face tags of an earlier run
// never look current. Not thread-safe; runs are stream-ordered on `s`.
// Half-split scoring of a lone triplet by a plan. Its longest sequence S_a is
// cut at mid; the first half (S_a[0, mid), S_r, S_c) is swept forward and the
// second half reversed (rev S_a[mid, n_a), rev S_r, rev S_c), concurrently,
// both writing their last slice, a plane over (S_r, S_c). Every alignment
// crosses the slice a = mid, so the score is the best F[p][q] + R[P-p][Q-q]
// over that plane (the crossing identity Hirschberg's method rests on). Each
// half's pipeline of panels is as long as the whole triplet's but sweeps half
// the slices, and the two fill together: the lone triplet finishes sooner.
// A local alignment either crosses the plane (the same identity, over the
// halves' local values) or lies within one half, so its score is the best of
// that plane maximum and the two halves' own bests. Local scoring does more
// work per cell, so the panel grid is busy enough on its own sooner: by
// default it takes the halves only below kHalfSplitMaxLocal residues (a
// threshold the caller sets lifts that cap).
constexpr uint32_t kHalfSplitMin = 128;        // shortest longest-sequence for it
constexpr uint32_t kHalfSplitMaxLocal = 2048;  // local scoring, default threshold
struct HalfSplit {
  uint32_t lens[6];
  uint64_t offs[6];      // word offsets in the gathered buffer
  GatherDesc gather[6];
  uint32_t words = 0;    // gathered words
  uint32_t rows = 0, cols = 0;
};

// Lays out the halves (gathered sequences, axes, plane size) of a triplet
// whose longest sequence has at least min_len residues (0: kHalfSplitMin;
// -1: never); false if it has not.
bool half_split_layout(const uint32_t* lens, const uint64_t* word_off, int32_t min_len, HalfSplit* h);
// Whether n triplets of this kind, under these options, are one triplet
// scored by halves (global, or local below kHalfSplitMaxLocal unless the
// options set a threshold; the plane kernels' lane exchange), and its layout.
bool half_split_choice(const uint32_t* lens, const uint64_t* word_off, size_t n, int kind,
                       const trioseq_plan_options& o, HalfSplit* h);

struct PlaneWorkspace {
  struct Buf {
    void* p = nullptr;
    uint64_t bytes = 0;
  };
  Buf ctl, desc, jobs, face, pool, bnd, red, plane, plane_off, words, scores;
  // Traceback levels: split descriptors and results, leaf tables and columns.
  Buf sd, split_out, chunk_box, partial, lwords, leaves, cols, ncols, lscore;
  Boundary boundary{};
  uint32_t bnd_n0 = 0;
  bool have_props = false;
  DeviceProps dp{};
  // Host copies of the last run's queue, alive until the next run (the
  // uploads are asynchronous).
  std::vector<TripletDesc> h_desc;
  std::vector<JobDesc> h_jobs;
  ~PlaneWorkspace();
};
// Makes b hold at least `bytes` (contents not kept; a buffer in use is only
// replaced after the stream drains). zero: clear a new buffer.
hipError_t ws_grow(PlaneWorkspace::Buf& b, uint64_t bytes, bool zero, hipStream_t s);
// Bytes the workspace holds on the device.
uint64_t ws_bytes(const PlaneWorkspace& ws);
// Lays out and sweeps n triplets (lens / word offsets on the host, words[0,
// nwords) packed on the host), leaving the planes in ws.plane (device).
trioseq_status run_planes(PlaneWorkspace& ws, const uint32_t* lens, const uint64_t* offs, size_t n,
                          const uint32_t* words, size_t nwords, const trioseq_scoring& sc,
                          const uint64_t* plane_off, uint64_t plane_ints, hipStream_t s);

}  // namespace trioseq

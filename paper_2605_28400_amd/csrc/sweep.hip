// gfx950 kernels for exact 3-way alignment scoring.
//
// What is computed (paper, Section II, Eq. 1): M[i][j][k] is the best of seven
// predecessor moves plus the sum-of-pairs score of the move's column (or v).
//  * global: v = -infinity, M[0][0][0] = 0, the answer is M[n0][n1][n2];
//  * semi-global: as global, but the three axes M[i][0][0], M[0][j][0],
//    M[0][0][k] are 0, and the answer is the best cell on the last slices
//    i = n0, j = n1 or k = n2;
//  * local: the semi-global initialisation with v = 0 (no cell below 0), and
//    the answer is the best cell of the tensor.
//
// Shifted recurrence. Every move adds 2*gap per consumed residue on top of
// its substitution terms, so with M'(i,j,k) = M(i,j,k) - 2*gap*(i+j+k) the
// seven candidates become
//   M'(i-1,j,k), M'(i,j-1,k), M'(i,j,k-1)                  (one residue, +0)
//   M'(i-1,j-1,k) + A, M'(i-1,j,k-1) + B, M'(i,j-1,k-1) + C (two residues)
//   M'(i-1,j-1,k-1) + A + B + C                             (three residues)
// with A = s(a,b) - 2*gap, B = s(a,c) - 2*gap, C = s(b,c) - 2*gap for the
// residues a = S0[i-1], b = S1[j-1], c = S2[k-1]. This is exact integer
// algebra (A + B + C = SOP - 6*gap), and M' >= 0 for every cell because the
// path of single-residue moves scores exactly 0 in M'.
//
// Decomposition (designed for CDNA4; the paper's warp-tile kernel is prior art):
//  * The (j,k) plane is cut into panels of (8*RJ) x (8*RK) cells. One
//    wavefront owns a panel; its 64 lanes form an 8 x 8 grid and each lane
//    keeps an RJ x RK tile in VGPRs.
//  * The wavefront sweeps the whole S0 axis for its panel. Lane (y,x)
//    processes slice i = t - y - x at step t, so its left and upper
//    neighbours finished the same slice one step earlier. Their edge values
//    move through a per-wave LDS slot array (LDS operations of one wave
//    execute in order, so no barrier is needed). Panel edges come from LDS
//    rings that are filled one chunk (8 steps) ahead from face buffers in
//    HBM/L2, through buffer loads; faces are written with buffer stores
//    whose out-of-range offsets are dropped by the hardware, so the edge
//    lanes need no branches.
//  * Per cell: three v_max3_i32 and four adds (one v_add3_u32). The triple
//    move's term is carried as D = (X6 of the previous slice), where
//    X6 = M'(i,j-1,k-1) + C, so X7 = D + A + B needs no per-cell lookup;
//    A and B are read once per row/column per step from byte tables with
//    v_bfe_i32, keyed by a per-slice shift byte kept in LDS.
//  * Predecessors outside the tensor hold a finite sentinel (kSent): row and
//    column 0 use a table whose bytes are -128 and C = kSent, and the
//    virtual row above the tensor holds 0 at (i=0, k=0), which seeds
//    M'(0,0,0) = 0. No special edge code exists.
//  * One persistent kernel pops jobs from a device queue. A whole-triplet
//    job sweeps all panels of a small triplet in the wave's own workspace
//    (faces reused in place); a panel job sweeps one panel of a large
//    triplet split over many waves, whose faces travel through HBM as
//    (value, run-tag) pairs with device-coherent accesses (see the
//    hand-over notes below).
#include "internal.h"

namespace trioseq {
namespace {

constexpr int kBufFlags = 0x00020000;       // raw buffer, gfx9 family
constexpr uint32_t kOob = 0xF0000000u;      // voffset outside every buffer

typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint64_t bytes) {
  const uint32_t n = bytes > 0x7FFFFFFFull ? 0x7FFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, kBufFlags);
}

__device__ __forceinline__ uint32_t residue_at(const uint32_t* __restrict__ words, uint64_t off,
                                               uint32_t p) {
  return (words[off + (p >> 4)] >> ((p & 15u) << 1)) & 3u;
}

__device__ __forceinline__ int sbyte(uint32_t tab, uint32_t sh) {
  return __builtin_amdgcn_sbfe((int)tab, sh, 8);
}

__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }

__device__ __forceinline__ uint32_t pick4(uint32_t code, uint32_t t0, uint32_t t1, uint32_t t2,
                                          uint32_t t3) {
  return code == 0 ? t0 : code == 1 ? t1 : code == 2 ? t2 : t3;
}

template <int RJ, int RK>
struct Lds {
  static constexpr int H = kGJ * RJ;
  static constexpr int W = kGK * RK;
  __attribute__((aligned(16))) int ringT[kRing][W];   // top face, entry e at slice s - e/RK
  __attribute__((aligned(16))) int ringC[kRing][kGK]; // corner of top-edge lane x
  __attribute__((aligned(16))) int ringL[kRing][H];   // left face, entry r at slice s - r/RJ
  __attribute__((aligned(16))) int sR[64][RJ];        // right column of each lane
  __attribute__((aligned(16))) int sB[64][RK];        // bottom row of each lane
  int sX[64];                                         // bottom of each lane's left halo
  int cap[RJ * RK];                                   // tile of the score cell at slice n0
  int sink[64];                                       // per-lane discard slot (memory wave)
  int wsync;
};

// Face buffers hold one row per step of the producing wavefront: at step t
// its edge lanes write row t of its bottom face (W entries, lane (7,x) at
// slice t - 7 - x) and of its right face (RR = H + 4 entries: entry 0 the
// corner for the next panel, 1..3 unused, 4 + r the column of lane (r/RJ, 7)
// at slice t - r/RJ - 7). A consumer lane at step t' needs exactly the
// producer's row t' + 7 (its halo of slice t' - x or t' - y), so every
// step writes one contiguous row and every chunk of steps reads contiguous
// rows. Every stride is a compile-time constant, so step offsets fold into
// the instructions' immediate offsets.
struct PanelIO {
  const int* top;     // bottom face of the panel above, or a sentinel face
  const int* left;    // right face of the panel to the left, or a sentinel face
  int* bot;           // this panel's bottom face (nullptr: not needed)
  int* right;         // this panel's right face (nullptr: not needed)
  int gen;            // run generation: wide-engine faces carry it as a tag
  int* err;           // set when a tag wait gave up (wide engine)
  uint64_t wait_ticks;  // bound on each wait, in 100 MHz wall-clock ticks
  // Strip workgroups (compute waves of adjacent panels in one workgroup):
  // lds_left = the out rows of the left neighbour's compute wave, read in
  // place of a staged left face, with its step counter prod_done; cons_done =
  // the step counter of the right neighbour's compute wave, which reads this
  // panel's right out rows in place (null: none in the workgroup).
  const int* lds_left = nullptr;
  const int* prod_done = nullptr;
  const int* cons_done = nullptr;
};

// A wait that gave up: the run's error flag is raised, and the release fence
// orders it before every store the wave issues afterwards. A panel that gave
// up goes on with whatever its faces hold, so the flag must become visible
// no later than the faces it writes from then on: a downstream panel that
// consumes them (and the panel that publishes the score after it) then sees
// the flag too.
__device__ __forceinline__ void raise_error(int* err) {
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// The score of a split triplet, published by its last panel once the sweep is
// over: INT32_MIN if any wait of the run gave up. The acquire fence orders the
// flag's load after the face loads that the panel's result depends on.
__device__ __forceinline__ void publish_score(int32_t* so, int v, const int* err) {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  // System scope: the score may live in mapped host memory (serving), where
  // the host picks it up while the kernel is still running.
  __hip_atomic_store(so, bad ? INT32_MIN : v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Cross-wavefront hand-over in the wide engine. Every face entry is a
// (value, tag) pair written by one 64-bit store, tag = the run's generation
// number, so a consumer knows an entry is current without any flag or
// fence: entries left from an earlier run carry an older tag. Faces are
// written and read with device-coherent buffer accesses (the SC1
// cache-policy bit, the per-instruction coherence that relaxed agent-scope
// atomics use); producers never wait, and a consumer whose chunk of entries
// is not complete yet re-reads the stale ones. Sentinel faces carry the tag
// kTagAlways, valid in every run.
// Step of a chunk at which panel jobs issue the next chunk's staging loads.
constexpr int kWideStageAt = 7;

constexpr int kCohNone = 0;
constexpr int kCohDevice = 16;              // SC1
constexpr int kTagAlways = 0x7FFFFFFF;

// A zero the compiler cannot see through. Re-reads of stale face entries add
// it to their scalar offset, so each retry is a distinct load that is neither
// merged with nor hoisted above an earlier one, while staying an ordinary
// (non-volatile) device-coherent load: all re-reads of a chunk are in flight
// together and share one wait.
__device__ __forceinline__ uint32_t opaque_zero() {
  uint32_t z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// Every wait for another wavefront is bounded (PanelIO::wait_ticks, 2 s by
// default, in ticks of the 100 MHz wall clock): past the limit the wave
// raises the error flag and proceeds (the score is then marked invalid), so a
// lost producer cannot hang the GPU.

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));

// Four consecutive ints of LDS starting on a 16-byte boundary, read as one
// 128-bit access. A lane's halo row is either a ring row or a neighbour's
// slot row; both are 16-byte aligned, but the compiler cannot see that
// through the choice and would split the read into 8-byte halves, whose
// 16-byte lane stride makes lanes 8 apart collide on one LDS bank.
__device__ __forceinline__ v4i lds_v4(const int* p) {
  return *reinterpret_cast<const v4i*>(__builtin_assume_aligned(p, 16));
}

// Per-slice lookup shifts: shb[i + kShiftPre] = 8 * code(S0[i-1]) for slices
// 1..n0, 0 elsewhere; covers slices -kShiftPre .. n0 + 47.
__device__ __forceinline__ void stage_shifts(uint8_t* shb, const uint32_t* __restrict__ words,
                                             const TripletDesc& td, int tid, int nthreads) {
  const int n0 = (int)td.len[0];
  const int total = n0 + 64;
  for (int q = tid; q < total; q += nthreads) {
    const int i = q - kShiftPre;
    uint32_t v = 0;
    if (i >= 1 && i <= n0) v = residue_at(words, td.off[0], (uint32_t)(i - 1)) << 3;
    shb[q] = (uint8_t)v;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// One wavefront sweeps one panel over all slices.
// How a panel's halos arrive and its edges leave:
//  kPlain:    one wavefront; faces in HBM/L2 without tags (whole-triplet
//             jobs, whose faces the same wave wrote earlier);
//  kTagged:   one wavefront; tagged faces staged and written by the wave
//             itself (panel jobs next to whole-triplet jobs);
//  kSplitCompute: the compute wave of a two-wave panel workgroup: halos come
//             from LDS rings that the workgroup's memory wave fills, edges go
//             to LDS rows that the memory wave writes out (panel jobs).
enum PanelMode { kPlain = 0, kTagged = 1, kSplitCompute = 2 };

// Rows of the right out ring (a multiple of kChunk).
constexpr int kRingR = 64;
static_assert(kRingR % kChunk == 0 && kRingR >= kRing, "right out ring");

// LDS hand-over between the two waves of a panel workgroup. Ring row
// t mod kRing of the halo rings serves step t; out row t mod kRing holds the
// bottom edge the compute wave produced at step t, right out row (t - 7) mod
// kRingR its right edge. The counters only grow:
// in_ready = steps whose halo rows are staged (memory wave), out_done =
// steps computed (compute wave), out_flushed = out rows read back by the
// memory wave. A wave's LDS operations are performed in order, so a counter
// written after the rows it covers never runs ahead of them.
template <int RJ, int RK>
struct SplitLds {
  static constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  Lds<RJ, RK> L;
  // Out rows: bottom rows (kRing x W) followed by right rows (kRingR x RR).
  __attribute__((aligned(16))) int out[kRing * W + kRingR * RR];
  int in_ready, out_done, out_flushed, job;
  __device__ int* out_bot(int t) { return &out[(t & (kRing - 1)) * W]; }
  // The right out row of step t sits at ring row (t - 7) mod kRingR: a right
  // neighbour's step t' needs exactly this wave's row t' + 7, so it finds it
  // at ring row t' mod kRingR. The right rows' ring is deeper than the others
  // so that a neighbour in the workgroup reading them in place holds this
  // wave back only when it falls kRingR + 7 steps behind.
  __device__ int* out_right(int t) { return &out[kRing * W + ((t - (kGK - 1)) & (kRingR - 1)) * RR]; }
};

__device__ __forceinline__ int lds_get(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_put(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Global scoring: the lane owning cell (n0, n1, n2) writes the score to
// score_out (non-null for the triplet's last panel only); returns 0.
// PLANE kernels (traceback): when plane is non-null every lane keeps its
// tile of slice n0 in capt (64 * RJ * RK ints of LDS) and, after the sweep,
// writes its cells unshifted to plane[j * (n2 + 1) + k].
// Semi-global and local scoring: returns this lane's best unshifted value
// over the panel's cells that the answer ranges over (the caller reduces).
//
// In the shifted form the floor v = 0 of local scoring is the per-cell bound
// M'(i,j,k) >= F(i,j,k) = g*(i+j+k) with g = -2*gap >= 0, and the semi-global
// axes hold M' = F. Within a lane's tile F depends on the anti-diagonal
// d = r + c only, so both are handled per diagonal class: F_d = F_0 + g*d.
// Rows past n1 and columns past n2 (tile padding) use the row/column-0
// tables, so their cells never exceed the best cell of the tensor (every
// move into the padding that consumes a padding residue scores -128, and the
// remaining moves mirror moves inside the tensor at gap <= 0); slices outside
// 0..n0 are excluded from the best and unfloored before slice 0.
template <int MODE, int KIND, bool PLANE, int RJ, int RK, int XCH = 0>
__device__ int sweep_panel(Lds<RJ, RK>& L, const uint8_t* shb, const DevScoring& sc,
                           const uint32_t* __restrict__ words, const TripletDesc& td, int pj, int pk,
                           const PanelIO& io, int32_t* score_out, int* plane, int* capt,
                           SplitLds<RJ, RK>* split = nullptr) {
  constexpr bool WIDE = MODE == kTagged;
  constexpr bool SPC = MODE == kSplitCompute;
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  constexpr int COH = WIDE ? kCohDevice : kCohNone;
  constexpr int ES = WIDE ? 2 : 1;  // ints per face entry: value (+ tag)
  const int lane = threadIdx.x & 63;
  const int y = lane >> 3, x = lane & 7;
  const int n0 = (int)td.len[0], n1 = (int)td.len[1], n2 = (int)td.len[2];
  const int j0 = pj * H + y * RJ, k0 = pk * W + x * RK;
  const uint32_t bt0 = sc.byte_tab[0], bt1 = sc.byte_tab[1], bt2 = sc.byte_tab[2],
                 bt3 = sc.byte_tab[3], btz = sc.byte_tab[4];

  // Row/column tables of this lane's tile.
  constexpr bool PAD = KIND != kGlobal;  // padding rows/columns use the -128 table
  uint32_t TB[RJ], TC[RK], cco[RK];
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    const int j = j0 + r;
    const uint32_t b = (j >= 1 && j <= n1) ? residue_at(words, td.off[1], (uint32_t)(j - 1)) : 0u;
    TB[r] = (j == 0 || (PAD && j > n1)) ? btz : pick4(b, bt0, bt1, bt2, bt3);
  }
#pragma unroll
  for (int c = 0; c < RK; ++c) {
    const int k = k0 + c;
    cco[c] = (k >= 1 && k <= n2) ? residue_at(words, td.off[2], (uint32_t)(k - 1)) : 0u;
    TC[c] = (k == 0 || (PAD && k > n2)) ? btz : pick4(cco[c], bt0, bt1, bt2, bt3);
  }
  // C = s(b,c) - 2*gap (byte c of b's table, the matrix being symmetric),
  // packed four per register; -128 on row 0 and column 0, where every
  // predecessor that C is added to lies outside the tensor. The compiler
  // folds the byte extraction into the add (SDWA).
  constexpr int RKW = (RK + 3) / 4;
  uint32_t Cp[RJ][RKW];
#pragma unroll
  for (int r = 0; r < RJ; ++r)
#pragma unroll
    for (int w = 0; w < RKW; ++w) {
      uint32_t packed = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int cc = 4 * w + b;
        if (cc >= RK) break;
        const bool pad = PAD && (j0 + r > n1 || k0 + cc > n2);
        const int v = (j0 + r == 0 || k0 + cc == 0 || pad) ? -128 : sbyte(TB[r], cco[cc] << 3);
        packed |= (uint32_t)(v & 0xFF) << (8 * b);
      }
      Cp[r][w] = packed;
    }

  int P[RJ][RK], D[RJ][RK], Lp[RJ], Tp[RK];
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    Lp[r] = kSent;
#pragma unroll
    for (int c = 0; c < RK; ++c) P[r][c] = D[r][c] = kSent;
  }
#pragma unroll
  for (int c = 0; c < RK; ++c) Tp[c] = kSent;

  const int nsteps = n0 + 1 + kSkew;
  const int nchunks = (nsteps + kChunk - 1) / kChunk;
  const int stepsp = nchunks * kChunk;

  // The lane holding cell (n1, n2) of the last panel keeps slice n0.
  const int rsel = n1 - j0, csel = n2 - k0;
  const bool own = KIND == kGlobal && score_out && rsel >= 0 && rsel < RJ && csel >= 0 && csel < RK;

  // Semi-global and local scoring. fi = g*(i + j0 + k0) for the lane's slice
  // i of the current step; best = the lane's best unshifted value so far.
  constexpr int ND = RJ + RK - 1;  // anti-diagonal classes of a tile
  const int g2n = -sc.gap2;
  int fi = g2n * (j0 + k0 - y - x);
  int best = KIND == kLocal ? 0 : INT32_MIN;
  // Semi-global: the lane holds row n1 / column n2 (cells past them are padding).
  const bool has_row = rsel >= 0 && rsel < RJ, has_col = csel >= 0 && csel < RK;
  const bool axis_panel = pj == 0 || pk == 0;

  // Face resources: face_rows(n0) rows cover every staging load and store.
  const uint32_t frows = face_rows((uint32_t)n0);
  // Row strides in bytes.
  constexpr uint32_t ts = W * 4u * ES, bs = ts, RRB = RR * 4u * ES;
  const Rsrc r_top = make_rsrc(io.top, (uint64_t)frows * ts);
  const Rsrc r_left = make_rsrc(io.left, (uint64_t)frows * RRB);
  // An absent output gets an empty resource: its stores are all dropped.
  const Rsrc r_bot = make_rsrc(io.bot ? io.bot : io.top, io.bot ? (uint64_t)frows * bs : 0);
  const Rsrc r_right = make_rsrc(io.right ? io.right : io.left, io.right ? (uint64_t)frows * RRB : 0);

  // Staging. Value q of a chunk is, for this lane, entry v = lane + 64 q of
  // one of three LDS rings (top face, corners, left face). Ring row s of
  // chunk c serves step t' = c * kChunk + s: the top and left rings hold
  // producer row t' + 7, the corner of top-edge lane x >= 1 is entry
  // x*RK - 1 of top row t' + 6 (what lane x - 1 saw one step earlier) and
  // that of lane 0 is entry 0 of left row t' + 7. Within a ring a q step
  // advances by whole rows (ring widths divide 64), so each ring needs one
  // base voffset per lane plus a scalar increment per q, and the LDS
  // destination is simply ring base + v. Faces always exist: at the tensor
  // edge they are sentinel buffers, and rows written during the producer's
  // fill steps hold values within 2^24 of kSent.
  constexpr int QT = kChunk * W / 64, QC = kChunk * kGK / 64, QL = kChunk * H / 64;
  constexpr int NPF = QT + QC + QL;
  constexpr int RT = 64 / W, RL = 64 / H;  // ring rows per q
  static_assert(64 % W == 0 && 64 % H == 0 && QC == 1, "ring widths must divide 64");
  const int eT = lane % W;
  const uint32_t offT = (uint32_t)((kGJ - 1 + lane / W) * (int)ts + eT * 4 * ES);
  const int eC = lane % kGK;
  const bool corner_from_left = eC == 0;
  const uint32_t offC = corner_from_left
                            ? (uint32_t)((kGK - 1 + lane / kGK) * (int)RRB)
                            : (uint32_t)((kGJ - 2 + lane / kGK) * (int)ts + (eC * RK - 1) * 4 * ES);
  const int eL = lane % H;
  const uint32_t offL = (uint32_t)((kGK - 1 + lane / H) * (int)RRB + (4 + eL) * 4 * ES);
  // Slice of entry q in chunk c is c * kChunk + rel(q).
  const int relT = lane / W - eT / RK, relC = lane / kGK - eC, relL = lane / H - eL / RJ;
  auto rel_of = [&](int q) {
    return q < QT ? relT + q * RT : q < QT + QC ? relC : relL + (q - QT - QC) * RL;
  };

  // Face entry q of chunk c for this lane: (value, tag); the tag is unused
  // for whole-triplet jobs. z is added to the scalar offset (0, or an opaque
  // zero for re-reads).
  auto load_entry = [&](int q, int c, uint32_t z) -> v2i {
    constexpr int LDC = COH;
    const uint32_t base = (uint32_t)(c * kChunk);
    if (q < QT) {
      const uint32_t so = (base + q * RT) * ts + z;
      if (WIDE) return __builtin_amdgcn_raw_buffer_load_b64(r_top, offT, so, LDC);
      return (v2i){(int)__builtin_amdgcn_raw_buffer_load_b32(r_top, offT, so, LDC), 0};
    } else if (q < QT + QC) {
      const uint32_t ot = corner_from_left ? kOob : offC, ol = corner_from_left ? offC : kOob;
      if (WIDE)
        return __builtin_amdgcn_raw_buffer_load_b64(r_top, ot, base * ts + z, LDC) |
               __builtin_amdgcn_raw_buffer_load_b64(r_left, ol, base * RRB + z, LDC);
      return (v2i){(int)(__builtin_amdgcn_raw_buffer_load_b32(r_top, ot, base * ts + z, LDC) |
                         __builtin_amdgcn_raw_buffer_load_b32(r_left, ol, base * RRB + z, LDC)),
                   0};
    } else {
      const uint32_t so = (base + (q - QT - QC) * RL) * RRB + z;
      if (WIDE) return __builtin_amdgcn_raw_buffer_load_b64(r_left, offL, so, LDC);
      return (v2i){(int)__builtin_amdgcn_raw_buffer_load_b32(r_left, offL, so, LDC), 0};
    }
  };
  int pf[NPF], pt[NPF];
  auto stage_load = [&](int c) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const v2i e = load_entry(q, c, 0u);
      pf[q] = e.x;
      pt[q] = e.y;
    }
  };
  // Panel jobs: wait until every entry the sweep uses carries this run's
  // tag. Entries of slices past n0 are never written by the producer (its
  // drain stops earlier) and only feed cells past n0, so they are skipped.
  // A stale chunk is first re-read at once (twice: the producer is usually
  // only a few steps behind). After that only two lanes poll, each one probe
  // entry that its producer writes last for this chunk (slice
  // min(c*kChunk+7, n0), entry 0, in row slice + 7), with a pause between polls, and the stale
  // entries are re-read once both probes are current. Waiting waves thus put
  // almost no load on the memory system the producers need.
  const bool probe_top = lane == 0 && pj > 0, probe_left = lane == 1 && pk > 0;
  auto stage_validate = [&](int c) {
    if (!WIDE) return;
    auto chunk_ok = [&]() {
      bool ok = true;
#pragma unroll
      for (int q = 0; q < NPF; ++q) ok = ok && (pt[q] >= io.gen || c * kChunk + rel_of(q) > n0);
      return __builtin_amdgcn_ballot_w64(!ok) == 0;
    };
    if (chunk_ok()) return;
    const uint64_t t_start = wall_clock64();
    const int ps = min(c * kChunk + kChunk - 1, n0);
    const uint32_t probe_off = probe_top ? (uint32_t)((ps + kGJ - 1) * (int)ts)
                                         : (uint32_t)((ps + kGK - 1) * (int)RRB + 4 * 4 * ES);
    for (int attempt = 0;; ++attempt) {
      if (wall_clock64() - t_start > io.wait_ticks) {
        raise_error(io.err);
        break;
      }
      if (attempt >= 2) {
        __builtin_amdgcn_s_sleep(8);
        const uint32_t z = opaque_zero();
        bool probe_ok = true;
        if (probe_top)
          probe_ok = ((v2i)__builtin_amdgcn_raw_buffer_load_b64(r_top, probe_off, z, kCohDevice)).y >= io.gen;
        if (probe_left)
          probe_ok = ((v2i)__builtin_amdgcn_raw_buffer_load_b64(r_left, probe_off, z, kCohDevice)).y >= io.gen;
        if (__builtin_amdgcn_ballot_w64(!probe_ok) != 0) continue;
      }
      const uint32_t z = opaque_zero();
#pragma unroll
      for (int q = 0; q < NPF; ++q)
        if (pt[q] < io.gen && c * kChunk + rel_of(q) <= n0) {
          const v2i e = load_entry(q, c, z);
          pf[q] = e.x;
          pt[q] = e.y;
        }
      if (chunk_ok()) break;
    }
  };
  auto stage_finish = [&](int c) {
    stage_validate(c);
    const int rr = (c & 1) * kChunk;
    int* rt = &L.ringT[rr][0];
    int* rc = &L.ringC[rr][0];
    int* rl = &L.ringL[rr][0];
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      if (q < QT)
        rt[lane + 64 * q] = pf[q];
      else if (q < QT + QC)
        rc[lane] = pf[q];
      else
        rl[lane + 64 * (q - QT - QC)] = pf[q];
    }
  };

  if (!SPC) stage_load(0);
  // Before step 0 the neighbour slots hold slice "-1" for every lane: the
  // sentinel (they are read at step 0, before any lane has written them).
#pragma unroll
  for (int r = 0; r < RJ; ++r) L.sR[lane][r] = kSent;
#pragma unroll
  for (int c = 0; c < RK; ++c) L.sB[lane][c] = kSent;
  L.sX[lane] = kSent;

  // Per-lane LDS sources of the three halos: ring rows for edge lanes,
  // neighbour slots (written one step earlier) otherwise. With the register
  // exchange (XCH) every lane reads the ring rows and the inner lanes then
  // take their neighbours' values from registers instead (below).
  const bool y0 = y == 0, x0 = x == 0;
  const bool tring = XCH || y0, lring = XCH || x0;
  const int* t_base = tring ? &L.ringT[0][x * RK] : &L.sB[y0 ? 0 : lane - 8][0];
  const int t_str = tring ? W : 0;
  const int* c_base = tring ? &L.ringC[0][x] : &L.sX[y0 ? 0 : lane - 8];
  int c_str = tring ? kGK : 0;
  const int* l_base = lring ? &L.ringL[0][y * RJ] : &L.sR[x0 ? 0 : lane - 1][0];
  int l_str = lring ? H : 0;
  // Register exchange: byte address of the lane above (lane - 8) for
  // ds_bpermute; the lane to the left (lane - 1) is one DPP row shift away.
  const int up_addr = ((lane + 64 - kGK) & 63) << 2;
  if (SPC && io.lds_left) {
    // Left face straight from the left neighbour's right out rows (row t of
    // the ring holds its step t + 7): the halo of lane (y, 0) at entry
    // 4 + y*RJ, the corner of lane (0, 0) at entry 0.
    const int* lr = io.lds_left + kRing * W;
    if (x0) {
      l_base = lr + 4 + y * RJ;
      l_str = RR;
    }
    if (x0 && y0) {
      c_base = lr;
      c_str = RR;
    }
  }
  // Chunk phase of each halo source: staged rings hold two chunks; the left
  // neighbour's right out rows, read in place, kRingR / kChunk.
  const int l_cmask = (SPC && io.lds_left && x0) ? kRingR / kChunk - 1 : 1;
  const int c_cmask = (SPC && io.lds_left && x0 && y0) ? kRingR / kChunk - 1 : 1;

  // Edge stores: bottom row (y = 7), right column (x = 7), and the corner
  // for the next panel (lane (0,7)), all into row t at step t.
  const uint32_t vo_bot = (y == kGJ - 1) ? (uint32_t)(x * RK * 4 * ES) : kOob;
  const uint32_t vo_right = (x == kGK - 1) ? (uint32_t)((4 + y * RJ) * 4 * ES) : kOob;
  const uint32_t vo_corner = (x == kGK - 1 && y == 0) ? 0u : kOob;
  const int sh_base = kShiftPre - y - x;

  // Store offsets of this chunk. Stores take their whole offset in the VGPR
  // (chunk base) plus the immediate (step and entry), never an SGPR offset:
  // gfx950 can read the data registers of a store wider than 64 bits after
  // the next instruction has overwritten them when the store has an SGPR
  // offset, and the compiler only separates the two for stores without one.
  // Lanes at kOob stay out of range (the chunk base is far below 2^28).
  // Staging loads of chunk c + 1 are issued at step kStageAt of chunk c.
  // Whole-triplet jobs issue them first (their faces were written long ago,
  // so only the load latency matters). Panel jobs issue them late, so the
  // rows they fetch were written as recently as the load latency allows:
  // every step of prefetch distance would add a step to the lag between a
  // producer panel and its consumers.
  constexpr int kStageAt = WIDE ? kWideStageAt : 0;
  // Last read in_ready / out_flushed, and the neighbours' step counters
  // (split compute wave).
  int fin = 0, ffl = 0, pdn = 0, cdn = 0;
  bool gave_up = false;
  auto run_chunk = [&](int c, bool cap, bool more) {
    const uint32_t cbase = (uint32_t)(c * kChunk);
    const uint32_t vb = vo_bot + cbase * bs, vr = vo_right + cbase * RRB,
                   vc = vo_corner + cbase * RRB;
    const int rr = (c & 1) * kChunk;
    const int* tb = t_base + rr * t_str;
    const int* cb = c_base + (c & c_cmask) * kChunk * c_str;
    const int* lb = l_base + (c & l_cmask) * kChunk * l_str;
    const uint8_t* sp = shb + sh_base + c * kChunk;
    // The chunk's lookup shifts, read together: one LDS round trip per chunk
    // instead of one per step ahead of the halo reads.
    uint32_t shv[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) shv[s] = sp[s];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      if (!SPC && s == kStageAt && more) stage_load(c + 1);
      const int t = c * kChunk + s;
      int fin_next = 0, ffl_next = 0, pdn_next = 0, cdn_next = 0;
      if (SPC) {
        // Step t needs its halo rows staged (in_ready > t) and out row
        // t mod kRing read back (out_flushed > t - kRing). The counters
        // read during the previous step usually already say so; the reads
        // for the next step are issued now, behind this step's work.
        // With in-workgroup neighbours also: the left neighbour has done
        // step t + 7 (while any lane (y, 0) is on a slice <= n0), and the
        // right neighbour has read the right out row this step overwrites
        // (its step t - kRingR - 7).
        const bool need_l = io.lds_left && t <= n0 + (kGJ - 1);
        const bool need_r = io.cons_done != nullptr;
        auto ready = [&]() {
          return fin > t && ffl > t - kRing && (!need_l || pdn > t + (kGK - 1)) &&
                 (!need_r || cdn > t - kRingR - (kGK - 1));
        };
        if (!gave_up && !ready()) {
          const uint64_t t_start = wall_clock64();
          for (;;) {
            fin = lds_get(&split->in_ready);
            ffl = lds_get(&split->out_flushed);
            if (need_l) pdn = lds_get(io.prod_done);
            if (need_r) cdn = lds_get(io.cons_done);
            if (ready()) break;
            if (wall_clock64() - t_start > io.wait_ticks) {
              // Give up waiting for the rest of the job (the score is marked
              // invalid); the job still runs to its end.
              raise_error(io.err);
              gave_up = true;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        fin_next = lds_get(&split->in_ready);
        ffl_next = lds_get(&split->out_flushed);
        if (io.lds_left) pdn_next = lds_get(io.prod_done);
        if (io.cons_done) cdn_next = lds_get(io.cons_done);
      }
      const uint32_t sh = shv[s];
      int A[RJ], B[RK];
#pragma unroll
      for (int r = 0; r < RJ; ++r) A[r] = sbyte(TB[r], sh);
#pragma unroll
      for (int cc = 0; cc < RK; ++cc) B[cc] = sbyte(TC[cc], sh);
      int T[RK], Lh[RJ];
      const int* tp = tb + s * t_str;
      const int* lp = lb + s * l_str;
      static_assert(RJ % 4 == 0 && RK % 4 == 0, "halo rows are read 4 entries at a time");
#pragma unroll
      for (int cc = 0; cc < RK; cc += 4) {
        const v4i v = lds_v4(tp + cc);
        T[cc] = v.x, T[cc + 1] = v.y, T[cc + 2] = v.z, T[cc + 3] = v.w;
      }
#pragma unroll
      for (int r = 0; r < RJ; r += 4) {
        const v4i v = lds_v4(lp + r);
        Lh[r] = v.x, Lh[r + 1] = v.y, Lh[r + 2] = v.z, Lh[r + 3] = v.w;
      }
      int corner = cb[s * c_str];
      if (XCH) {
        // The upper and left neighbours finished this lane's slice one step
        // earlier: their last rows / columns are still in their P registers
        // (the corner is the upper lane's previous left halo). The upper row
        // comes through ds_bpermute (lane - 8, the LDS crossbar without an
        // LDS round trip), the left column through a DPP row shift by one
        // lane; edge lanes keep the ring values read above.
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) {
          const int nb = __builtin_amdgcn_ds_bpermute(up_addr, P[RJ - 1][cc]);
          T[cc] = y0 ? T[cc] : nb;
        }
        {
          const int nb = __builtin_amdgcn_ds_bpermute(up_addr, Lp[RJ - 1]);
          corner = y0 ? corner : nb;
        }
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const int nb = __builtin_amdgcn_update_dpp(0, P[r][RK - 1], 0x111 /* row_shr:1 */, 0xF, 0xF, true);
          Lh[r] = x0 ? Lh[r] : nb;
        }
      }
      const int i = t - y - x;  // this lane's slice

      if (KIND == kSemiGlobal && axis_panel) {
        // The axes hold 0 (M' = F): the virtual predecessors across the
        // tensor edge carry the axis values, which the single move from
        // there (+0) copies in. Every other move from the virtual row or
        // column scores -128 through the row/column-0 tables.
        if (j0 == 0) {
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) T[cc] = i == 0 ? g2n * (k0 + cc) : T[cc];
          if (k0 == 0) T[0] = i >= 0 ? g2n * i : T[0];
        }
        if (k0 == 0) {
#pragma unroll
          for (int r = 0; r < RJ; ++r) Lh[r] = i == 0 ? g2n * (j0 + r) : Lh[r];
        }
      }
      // Local floors per anti-diagonal class; none before slice 0, whose
      // previous slice is outside the tensor.
      int F[ND];
      if (KIND != kGlobal) {
        // Keeps the compiler from computing every step's floors of a chunk
        // up front (they would all stay live in registers).
        asm volatile("" : "+v"(fi));
      }
      if (KIND == kLocal) {
        const int fb = i >= 0 ? fi : kSent;
#pragma unroll
        for (int d = 0; d < ND; ++d) F[d] = fb + g2n * d;
      }

      int N[RJ][RK];
      if (RJ * RK <= 16 && KIND == kGlobal) {
        // Candidates from the previous slice only (the moves that consume
        // S0's residue), computed while the halo reads are in flight: Q = the
        // best of the single move along S0 and its two double moves, X7 the
        // triple move. (Larger tiles keep the fused form below: holding Q and
        // X7 for every cell would spill their registers.)
        int Q[RJ][RK], X7[RJ][RK];
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) {
            const int up_prev = r ? P[r - 1][cc] : Tp[cc];
            const int left_prev = cc ? P[r][cc - 1] : Lp[r];
            Q[r][cc] = max3i(P[r][cc], up_prev + A[r], left_prev + B[cc]);
            if (KIND == kLocal) Q[r][cc] = max(Q[r][cc], F[r + cc]);
            X7[r][cc] = D[r][cc] + A[r] + B[cc];
          }
        }
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) {
            const int up_cur = r ? N[r - 1][cc] : T[cc];
            const int left_cur = cc ? N[r][cc - 1] : Lh[r];
            const int diag_cur = r ? (cc ? N[r - 1][cc - 1] : Lh[r - 1]) : (cc ? T[cc - 1] : corner);
            const int x6 = diag_cur + (int)(int8_t)(uint8_t)(Cp[r][cc >> 2] >> (8 * (cc & 3)));
            N[r][cc] = max3i(max3i(Q[r][cc], X7[r][cc], x6), up_cur, left_cur);
            D[r][cc] = x6;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) {
            const int up_cur = r ? N[r - 1][cc] : T[cc];
            const int up_prev = r ? P[r - 1][cc] : Tp[cc];
            const int left_cur = cc ? N[r][cc - 1] : Lh[r];
            const int left_prev = cc ? P[r][cc - 1] : Lp[r];
            const int diag_cur = r ? (cc ? N[r - 1][cc - 1] : Lh[r - 1]) : (cc ? T[cc - 1] : corner);
            const int x4 = up_prev + A[r];
            const int x5 = left_prev + B[cc];
            const int x6 = diag_cur + (int)(int8_t)(uint8_t)(Cp[r][cc >> 2] >> (8 * (cc & 3)));
            const int x7 = D[r][cc] + A[r] + B[cc];
            N[r][cc] = max3i(max3i(P[r][cc], up_cur, left_cur), max3i(x4, x5, x6), x7);
            if (KIND == kLocal) N[r][cc] = max(N[r][cc], F[r + cc]);
            D[r][cc] = x6;
          }
        }
      }

      if (KIND == kLocal) {
        // Best class maximum minus its floor F_d = fi + g*d, counted on
        // slices 0..n0. The per-class offsets g*d are wave-uniform, so only
        // fi stays live past the cell loop.
        int sb = INT32_MIN;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          int m = INT32_MIN;
#pragma unroll
          for (int r = 0; r < RJ; ++r)
            if (d - r >= 0 && d - r < RK) m = max(m, N[r][d - r]);
          sb = max(sb, m - g2n * d);
        }
        best = max(best, (uint32_t)i <= (uint32_t)n0 ? sb - fi : 0);
      } else if (KIND == kSemiGlobal) {
        // Cells of the last slices, on slices 0..n0: all of slice n0, row n1
        // and column n2. Padding cells never exceed the best of these, so
        // they need no mask; the others get kSent added.
        if ((uint32_t)i <= (uint32_t)n0 && (i == n0 || has_row || has_col)) {
          const int all = i == n0 ? 0 : kSent;
          int cpen[RK];
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) cpen[cc] = max(all, cc == csel ? 0 : kSent);
          int sb = INT32_MIN;
#pragma unroll
          for (int r = 0; r < RJ; ++r) {
            const int rp = r == rsel ? 0 : kSent;
#pragma unroll
            for (int cc = 0; cc < RK; ++cc)
              sb = max(sb, N[r][cc] + max(rp, cpen[cc]) - g2n * (r + cc));
          }
          best = max(best, sb - fi);
        }
      }
      fi += g2n;

      if (!XCH) {
#pragma unroll
        for (int r = 0; r < RJ; ++r) L.sR[lane][r] = N[r][RK - 1];
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) L.sB[lane][cc] = N[RJ - 1][cc];
        L.sX[lane] = Lh[RJ - 1];
      }

      // Edge stores (the hardware drops lanes whose offset is kOob).
      if (SPC) {
        if (y == kGJ - 1) {
          int* ob = split->out_bot(t) + x * RK;
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) ob[cc] = N[RJ - 1][cc];
        }
        if (x == kGK - 1) {
          int* orr = split->out_right(t);
#pragma unroll
          for (int r = 0; r < RJ; ++r) orr[4 + y * RJ + r] = N[r][RK - 1];
          if (y == 0) orr[0] = T[RK - 1];
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) lds_put(&split->out_done, t + 1);
        fin = fin_next;
        ffl = ffl_next;
        pdn = pdn_next;
        cdn = cdn_next;
      } else if (WIDE) {
        const int g = io.gen;
#pragma unroll
        for (int cc = 0; cc < RK; cc += 2)
          __builtin_amdgcn_raw_buffer_store_b128((v4i){N[RJ - 1][cc], g, N[RJ - 1][cc + 1], g}, r_bot,
                                                 vb + (s * bs + cc * 8), 0, COH);
#pragma unroll
        for (int r = 0; r < RJ; r += 2)
          __builtin_amdgcn_raw_buffer_store_b128((v4i){N[r][RK - 1], g, N[r + 1][RK - 1], g}, r_right,
                                                 vr + (s * RRB + r * 8), 0, COH);
        __builtin_amdgcn_raw_buffer_store_b64((v2i){T[RK - 1], g}, r_right, vc + s * RRB, 0, COH);
      } else {
#pragma unroll
        for (int cc = 0; cc < RK; cc += 4)
          __builtin_amdgcn_raw_buffer_store_b128(
              (v4i){N[RJ - 1][cc], N[RJ - 1][cc + 1], N[RJ - 1][cc + 2], N[RJ - 1][cc + 3]}, r_bot,
              vb + (s * bs + cc * 4), 0, COH);
#pragma unroll
        for (int r = 0; r < RJ; r += 4)
          __builtin_amdgcn_raw_buffer_store_b128(
              (v4i){N[r][RK - 1], N[r + 1][RK - 1], N[r + 2][RK - 1], N[r + 3][RK - 1]}, r_right,
              vr + (s * RRB + r * 4), 0, COH);
        __builtin_amdgcn_raw_buffer_store_b32(T[RK - 1], r_right, vc + s * RRB, 0, COH);
      }

      if (cap) {
        if (own && t - y - x == n0) {
#pragma unroll
          for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int cc = 0; cc < RK; ++cc) L.cap[r * RK + cc] = N[r][cc];
        }
        if (PLANE && plane && t - y - x == n0) {
#pragma unroll
          for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int cc = 0; cc < RK; ++cc) capt[lane * (RJ * RK) + r * RK + cc] = N[r][cc];
        }
      }

#pragma unroll
      for (int r = 0; r < RJ; ++r) {
        Lp[r] = Lh[r];
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) P[r][cc] = N[r][cc];
      }
#pragma unroll
      for (int cc = 0; cc < RK; ++cc) Tp[cc] = T[cc];
    }
  };

  for (int c = 0; c < nchunks; ++c) {
    if (!SPC) stage_finish(c);
    const bool cap_chunk = (score_out != nullptr || (PLANE && plane != nullptr)) &&
                           n0 >= c * kChunk - kSkew && n0 <= c * kChunk + kChunk - 1;
    run_chunk(c, cap_chunk, c + 1 < nchunks);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  // Whole-triplet jobs never wait, so their owner lane stores the score at
  // once (system scope: the score may live in mapped host memory, where the
  // host picks it up while the kernel is still running). The last panel of a
  // split triplet leaves it in L.cap for the caller, which publishes it once
  // it knows whether a wait of the run gave up.
  if (MODE == kPlain && own)
    __hip_atomic_store(score_out, L.cap[rsel * RK + csel] + sc.gap2 * (n0 + n1 + n2),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  if (PLANE && plane) {
#pragma unroll
    for (int r = 0; r < RJ; ++r)
#pragma unroll
      for (int cc = 0; cc < RK; ++cc) {
        const int j = j0 + r, k = k0 + cc;
        if (j <= n1 && k <= n2)
          plane[(uint64_t)j * (uint64_t)(n2 + 1) + (uint64_t)k] =
              capt[lane * (RJ * RK) + r * RK + cc] + sc.gap2 * (n0 + j + k);
      }
  }
  return KIND == kGlobal ? 0 : best;
}

// Global score of a split triplet from its last panel (pj, pk): the cell
// (n0, n1, n2) that the panel's owner lane left in L.cap, unshifted.
template <int RJ, int RK>
__device__ __forceinline__ int split_score(const Lds<RJ, RK>& L, const TripletDesc& td, int pj, int pk,
                                           int gap2) {
  const int n0 = (int)td.len[0], n1 = (int)td.len[1], n2 = (int)td.len[2];
  const int r = (n1 - pj * kGJ * RJ) % RJ, c = (n2 - pk * kGK * RK) % RK;
  return L.cap[r * RK + c] + gap2 * (n0 + n1 + n2);
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// Semi-global and local scoring, whole-triplet job: the wave's best over all
// panels is the score.
__device__ __forceinline__ void finish_whole(int32_t* score_out, int best) {
  const int wb = wave_max(best);
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(score_out, wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Semi-global and local scoring, panel job of a split triplet: the panel's
// best is folded into the triplet's accumulator, then the panel counts
// itself finished. The release of that count orders the fold before it, so
// the panel that finishes last (its count acquires every earlier one) reads
// the final best and writes the score, or INT32_MIN if a wait of the run gave
// up.
__device__ __forceinline__ void finish_panel(const SweepArgs& a, uint32_t trip, uint32_t out,
                                             int npanels, int best) {
  const int wb = wave_max(best);
  if ((threadIdx.x & 63) == 0) {
    int* acc = a.red + 2 * (uint64_t)trip;
    __hip_atomic_fetch_max(acc, wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int prev = __hip_atomic_fetch_add(acc + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == npanels - 1) {
      const int v = __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool bad = __hip_atomic_load(a.ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      __hip_atomic_store(a.scores + out, bad ? INT32_MIN : v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// The memory wave of a two-wave panel workgroup. It keeps the compute wave's
// halo rings filled and writes the compute wave's edge rows out:
//  * staging: for steps u.. it loads, in one batch, top rows u+6 .. u+kChunk+6
//    and left rows u+7 .. u+kChunk+6 of the producers' tagged faces, finds the
//    longest run of steps whose needed entries all carry this run's tag
//    (entries of slices past n0 are never needed), copies them into the ring
//    rows of those steps (the corner of top lane x >= 1 at step u is entry
//    x*RK - 1 of top row u+6) and publishes in_ready; a ring row is only
//    refilled once the compute wave has finished the step kRing earlier (a
//    left face that a neighbour in the workgroup hands over in LDS is not
//    staged);
//  * flushing: out rows the compute wave has finished are stored as
//    (value, tag) pairs with device-coherent stores, then out_flushed is
//    published so the compute wave may reuse those rows.
// Every
// wait is bounded: past the wall-clock limit the error flag is raised and
// the rows are staged as they are, so both waves always finish the job.
template <int RJ, int RK>
__device__ void panel_memory(SplitLds<RJ, RK>& S, const TripletDesc& td, const PanelIO& io) {
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  constexpr uint32_t ts = W * 8u, RRB = RR * 8u;
  constexpr int NB = kChunk;
  constexpr int TOPN = (NB + 1) * W, LEFTN = NB * RR, EPR = W + H + 1;
  constexpr int QT = (TOPN + 63) / 64, QL = (LEFTN + 63) / 64, QF = (NB * EPR + 63) / 64;
  static_assert(NB + 1 <= 32, "step masks hold one bit per step of a batch");
  const int lane = threadIdx.x & 63;
  const int n0 = (int)td.len[0];
  const int stepsp = (n0 + 1 + kSkew + kChunk - 1) / kChunk * kChunk;
  const uint32_t frows = face_rows((uint32_t)n0);
  const Rsrc r_top = make_rsrc(io.top, (uint64_t)frows * ts);
  const Rsrc r_left = make_rsrc(io.left, (uint64_t)frows * RRB);
  const Rsrc r_bot = make_rsrc(io.bot ? io.bot : io.top, io.bot ? (uint64_t)frows * ts : 0);
  const Rsrc r_right = make_rsrc(io.right ? io.right : io.left, io.right ? (uint64_t)frows * RRB : 0);
  const int gen = io.gen;
  // A left face read from a neighbour in the workgroup is not staged.
  const bool stage_left = io.lds_left == nullptr;
  // Flat LDS views: out rows (outB then outR), and the halo rings, with a
  // per-lane sink slot for entries a batch does not publish.
  const int* outs = S.out;
  int* sink = &S.L.sink[lane];
  int staged = 0, flushed = 0;
  uint64_t stall_since = 0;
  bool gave_up = false;
  while (staged < stepsp || flushed < stepsp) {
    const int done = lds_get(&S.out_done);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    bool progress = false;
    const int u = staged;
    const int nb = min(min(NB, stepsp - u), done + kRing - u);
    if (nb > 0) {
      v2i tv[QT], lv[QL];
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const int f = q * 64 + lane;
        const uint32_t off = f < TOPN ? (uint32_t)(((u + kGJ - 2) * W + f) * 8) : kOob;
        tv[q] = __builtin_amdgcn_raw_buffer_load_b64(r_top, off, opaque_zero(), kCohDevice);
      }
#pragma unroll
      for (int q = 0; q < QL; ++q) {
        const int f = q * 64 + lane;
        const uint32_t off = f < LEFTN && stage_left ? (uint32_t)(((u + kGK - 1) * RR + f) * 8) : kOob;
        lv[q] = __builtin_amdgcn_raw_buffer_load_b64(r_left, off, opaque_zero(), kCohDevice);
      }
      // Bit k of `bad` is set when step u + k lacks one of this lane's
      // entries (a stale tag on an entry of a slice <= n0).
      uint32_t bad = 0;
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const int f = q * 64 + lane;
        const int rr = f / W, e = f % W, x = e / RK;  // top row u + 6 + rr
        const bool stale = f < TOPN && u + rr - 1 - x <= n0 && tv[q].y < gen;
        const bool corner = e % RK == RK - 1 && x + 1 < kGK;
        bad |= stale ? ((rr >= 1 ? 1u << (rr - 1) : 0u) | (corner ? 1u << rr : 0u)) : 0u;
      }
#pragma unroll
      for (int q = 0; q < QL; ++q) {
        const int f = q * 64 + lane;
        const int rr = f / RR, e = f % RR;  // left row u + 7 + rr
        const int slice = u + rr - (e == 0 ? 0 : (e - 4) / RJ);
        const bool stale = stage_left && f < LEFTN && (e == 0 || e >= 4) && slice <= n0 && lv[q].y < gen;
        bad |= stale ? 1u << rr : 0u;
      }
      int k = nb;
#pragma unroll
      for (int b = NB - 1; b >= 0; --b)
        if (__builtin_amdgcn_ballot_w64((bad >> b) & 1u) != 0) k = b;
      k = min(k, nb);
      if (gave_up) k = nb;
      if (k <= 0 && stall_since && wall_clock64() - stall_since > io.wait_ticks) {
        // Stop waiting for producers for the rest of the job (the score is
        // marked invalid) so that both waves finish it.
        raise_error(io.err);
        gave_up = true;
        k = nb;
      }
      if (k > 0) {
        const int hi = u + k;
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          const int f = q * 64 + lane;
          const int rr = f / W, e = f % W, x = e / RK;
          const int st = u + rr - 1, sc = u + rr;  // T row of step st, corner row of step sc
          int* dt = (f < TOPN && st >= u && st < hi) ? &S.L.ringT[st & (kRing - 1)][e] : sink;
          *dt = tv[q].x;
          int* dc = (f < TOPN && e % RK == RK - 1 && x + 1 < kGK && sc < hi)
                        ? &S.L.ringC[sc & (kRing - 1)][(x + 1) & (kGK - 1)]
                        : sink;
          *dc = tv[q].x;
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
          const int f = q * 64 + lane;
          const int rr = f / RR, e = f % RR;
          const int st = u + rr;
          int* dl = !(stage_left && f < LEFTN && st < hi) ? sink
                    : e == 0                 ? &S.L.ringC[st & (kRing - 1)][0]
                    : e >= 4                 ? &S.L.ringL[st & (kRing - 1)][e - 4]
                                             : sink;
          *dl = lv[q].x;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) lds_put(&S.in_ready, hi);
        staged = hi;
        progress = true;
      }
    }
    // Flush finished out rows (entries per row: W bottom, the corner, H
    // right). Issued after the staging loads were consumed, so the stores
    // drain while the next batch's loads are in flight.
    const int nf = min(NB, lds_get(&S.out_done) - flushed);
    if (nf > 0) {
      int v[QF];
      uint32_t ob[QF], orr[QF];
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int f = q * 64 + lane;
        const int row = f / EPR, e = f % EPR;
        const int t = flushed + row, ro = t & (kRing - 1);
        const int er = e == W ? 0 : 4 + (e - W - 1);  // right-face entry
        const int rro = (t - (kGK - 1)) & (kRingR - 1);  // right out rows sit 7 steps back
        v[q] = outs[e < W ? ro * W + e : kRing * W + rro * RR + er];
        const bool live = row < nf;
        ob[q] = live && e < W ? (uint32_t)((t * W + e) * 8) : kOob;
        orr[q] = live && e >= W ? (uint32_t)((t * RR + er) * 8) : kOob;
      }
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        __builtin_amdgcn_raw_buffer_store_b64((v2i){v[q], gen}, r_bot, ob[q], 0, kCohDevice);
        __builtin_amdgcn_raw_buffer_store_b64((v2i){v[q], gen}, r_right, orr[q], 0, kCohDevice);
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (lane == 0) lds_put(&S.out_flushed, flushed + nf);
      flushed += nf;
      progress = true;
    }
    if (progress) {
      stall_since = 0;
    } else {
      if (!stall_since) stall_since = wall_clock64();
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

// Panel jobs on two-wave workgroups: wave 0 computes (kSplitCompute), wave 1
// moves faces (panel_memory). The workgroup pops jobs from the same queue
// and in the same dependency order as k_sweep, so the same residency
// argument holds: every producer was popped earlier by a running workgroup.
template <int RJ, int RK, int WPE, int KIND, bool PLANE, int XCH>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(WPE))) k_panel(SweepArgs a) {
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  __shared__ SplitLds<RJ, RK> S;
  __shared__ int capt[PLANE ? 64 * RJ * RK : 1];
  extern __shared__ uint8_t shb[];
  const int wave = threadIdx.x >> 6;
  const int gen = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t staged = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) S.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int idx = S.job;
    if (idx >= (int)a.njobs) break;
    const JobDesc jd = a.jobs[idx];
    const TripletDesc td = a.desc[jd.trip];
    int* plane = PLANE ? a.plane + a.plane_off[jd.trip] : nullptr;
    if (jd.trip != staged) {
      stage_shifts(shb, a.words, td, threadIdx.x, blockDim.x);
      staged = jd.trip;
    }
    if (threadIdx.x == 0) {
      S.in_ready = 0;
      S.out_done = 0;
      S.out_flushed = 0;
    }
    __syncthreads();
    const int n1 = (int)td.len[1], n2 = (int)td.len[2];
    const int PJ = n1 / H + 1, PK = n2 / W + 1;
    const uint64_t rows = face_rows(td.len[0]);
    const uint32_t p = jd.panel;
    const int pj = (int)(p / (uint32_t)PK), pk = (int)(p % (uint32_t)PK);
    const uint64_t fb_ints = rows * W * 2;
    const uint64_t per_panel = fb_ints + rows * RR * 2;
    int* pool = a.pface + td.face_off;
    int* base = pool + (uint64_t)p * per_panel;
    PanelIO io;
    io.top = pj ? pool + (uint64_t)(p - PK) * per_panel : (pk ? a.bnd_tagged[1] : a.bnd_tagged[0]);
    io.left = pk ? pool + (uint64_t)(p - 1) * per_panel + fb_ints : a.bnd_tagged[2];
    io.bot = pj + 1 < PJ ? base : nullptr;
    io.right = pk + 1 < PK ? base + fb_ints : nullptr;
    io.gen = gen;
    io.err = a.ctl + 1;
    io.wait_ticks = a.wait_ticks;
    int32_t* so = (KIND == kGlobal && pj == PJ - 1 && pk == PK - 1) ? a.scores + td.out : nullptr;
    int best = 0;
    if (wave == 0)
      best = sweep_panel<kSplitCompute, KIND, PLANE, RJ, RK, XCH>(S.L, shb, a.sc, a.words, td, pj, pk, io,
                                                             so, plane, capt, &S);
    else
      panel_memory<RJ, RK>(S, td, io);
    __syncthreads();
    // Both waves are done: a wait of this job that gave up has raised the
    // flag by now, and upstream panels raised theirs before writing the faces
    // this job read.
    if (KIND != kGlobal) {
      if (wave == 0) finish_panel(a, jd.trip, td.out, PJ * PK, best);
    } else if (so && threadIdx.x == 0) {
      publish_score(so, split_score(S.L, td, pj, pk, a.sc.gap2), io.err);
    }
  }
}

// Strip workgroups: kPairs (compute, memory) wave pairs sweep kPairs
// horizontally adjacent panels of one panel row together, a strip job. Each
// pair runs the two-wave panel protocol of k_panel on its panel, except that
// the face between two neighbours of the strip never leaves LDS: the right
// compute wave reads the left one's right out rows in place (its memory wave
// stages only the top face), and the left one's memory wave does not write
// that face out. Only the strip's outer faces (top and bottom of every panel,
// left of the first, right of the last) travel through L2/HBM. Along a panel
// row, three of every four hand-overs thus take a few LDS operations instead
// of a store, its coherence and a polled load. The hardware spreads the
// workgroup's waves over the compute unit's four SIMDs; every wave reads its
// SIMD at start and the compute role goes to the first wave on each SIMD, so
// the four compute waves sit on distinct SIMDs whenever the waves span all
// four.
constexpr int kPairs = kStripPanels;
template <int RJ, int RK, int WPE, int KIND, bool PLANE, int XCH>
__global__ void __launch_bounds__(128 * kPairs) __attribute__((amdgpu_waves_per_eu(WPE)))
k_panel_group(SweepArgs a) {
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  __shared__ SplitLds<RJ, RK> SP[kPairs];
  __shared__ int capt_all[PLANE ? kPairs * 64 * RJ * RK : 1];
  __shared__ int simd_of[2 * kPairs];
  __shared__ int job_slot;
  extern __shared__ uint8_t shb[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) simd_of[wave] = (int)((__builtin_amdgcn_s_getreg((31 << 11) | 4) >> 4) & 3u);
  __syncthreads();
  // Roles, the same table in every wave: compute waves are the first wave
  // found on each SIMD (then, if fewer SIMDs hold waves, the first waves
  // left); the others are memory waves; the p-th compute wave and the p-th
  // memory wave form pair p, which sweeps panel p of the strip.
  int is_comp = 0, pair = 0;
  {
    uint32_t comp_mask = 0, seen = 0;
    int ncomp = 0;
    for (int w = 0; w < 2 * kPairs; ++w) {
      const uint32_t sb = 1u << simd_of[w];
      if (!(seen & sb) && ncomp < kPairs) {
        seen |= sb;
        comp_mask |= 1u << w;
        ++ncomp;
      }
    }
    for (int w = 0; w < 2 * kPairs && ncomp < kPairs; ++w)
      if (!(comp_mask & (1u << w))) {
        comp_mask |= 1u << w;
        ++ncomp;
      }
    is_comp = (comp_mask >> wave) & 1;
    const uint32_t same_role = is_comp ? comp_mask : ~comp_mask;
    pair = __builtin_popcount(same_role & ((1u << wave) - 1u));
  }
  SplitLds<RJ, RK>& S = SP[pair];
  int* capt = PLANE ? &capt_all[pair * 64 * RJ * RK] : capt_all;
  const int gen = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t staged = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) job_slot = atomicAdd(a.counter, 1);
    __syncthreads();
    const int idx = job_slot;
    if (idx >= (int)a.njobs) break;
    const JobDesc jd = a.jobs[idx];
    const TripletDesc td = a.desc[jd.trip];
    int* plane = PLANE ? a.plane + a.plane_off[jd.trip] : nullptr;
    if (jd.trip != staged) {
      stage_shifts(shb, a.words, td, threadIdx.x, blockDim.x);
      staged = jd.trip;
    }
    if (lane == 0 && is_comp) {
      S.in_ready = 0;
      S.out_done = 0;
      S.out_flushed = 0;
    }
    __syncthreads();
    const int n1 = (int)td.len[1], n2 = (int)td.len[2];
    const int PJ = n1 / H + 1, PK = n2 / W + 1;
    const uint64_t rows = face_rows(td.len[0]);
    // The strip: panels jd.panel .. jd.panel + kPairs - 1 of one panel row
    // (those past the row's last panel are idle for this job).
    const uint32_t p = jd.panel + (uint32_t)pair;
    const int pj = (int)(jd.panel / (uint32_t)PK), pk = (int)(jd.panel % (uint32_t)PK) + pair;
    const bool active = pk < PK;
    const bool has_right_in_wg = active && pair + 1 < kPairs && pk + 1 < PK;
    const bool has_left_in_wg = active && pair > 0;
    int best = 0;
    int32_t* so = nullptr;
    PanelIO io;
    if (active) {
      const uint64_t fb_ints = rows * W * 2;
      const uint64_t per_panel = fb_ints + rows * RR * 2;
      int* pool = a.pface + td.face_off;
      int* base = pool + (uint64_t)p * per_panel;
      io.top = pj ? pool + (uint64_t)(p - PK) * per_panel : (pk ? a.bnd_tagged[1] : a.bnd_tagged[0]);
      io.left = pk ? pool + (uint64_t)(p - 1) * per_panel + fb_ints : a.bnd_tagged[2];
      io.bot = pj + 1 < PJ ? base : nullptr;
      io.right = (pk + 1 < PK && !has_right_in_wg) ? base + fb_ints : nullptr;
      io.gen = gen;
      io.err = a.ctl + 1;
      io.wait_ticks = a.wait_ticks;
      if (has_left_in_wg) {
        io.lds_left = SP[pair - 1].out;
        io.prod_done = &SP[pair - 1].out_done;
      }
      if (has_right_in_wg) io.cons_done = &SP[pair + 1].out_done;
      so = (KIND == kGlobal && pj == PJ - 1 && pk == PK - 1) ? a.scores + td.out : nullptr;
      if (is_comp)
        best = sweep_panel<kSplitCompute, KIND, PLANE, RJ, RK, XCH>(S.L, shb, a.sc, a.words, td, pj, pk, io,
                                                               so, plane, capt, &S);
      else
        panel_memory<RJ, RK>(S, td, io);
    }
    __syncthreads();
    // Every wave of the strip is done with the job (see k_panel).
    if (active && is_comp) {
      if (KIND != kGlobal)
        finish_panel(a, jd.trip, td.out, PJ * PK, best);
      else if (so && lane == 0)
        publish_score(so, split_score(S.L, td, pj, pk, a.sc.gap2), io.err);
    }
  }
}

// The persistent scoring kernel. Waves pop jobs from a device queue in
// the order the host wrote them (every job after the jobs it depends on):
//  * a whole-triplet job sweeps all panels of one triplet, in place, in the
//    wave's own face workspace;
//  * a panel job sweeps one panel of a split triplet; its faces live in the
//    triplet's panel-face pool as (value, tag) entries and it waits for the
//    entries of its upper and left neighbours. Those neighbours were popped
//    earlier by waves that are running, so every wait ends no matter how many
//    waves of the grid are resident.
// MODES: bit 0 = the plan has whole-triplet jobs, bit 1 = panel jobs; a
// kernel built for one kind only carries no registers for the other.
template <int RJ, int RK, int WPE, int MODES, int KIND, bool PLANE, int XCH>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) k_sweep(SweepArgs a) {
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  __shared__ Lds<RJ, RK> L;
  __shared__ int capt[PLANE ? 64 * RJ * RK : 1];
  extern __shared__ uint8_t shb[];
  int* face = a.face + (uint64_t)blockIdx.x * a.face_stride;
  const int gen = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t staged = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) L.wsync = atomicAdd(a.counter, 1);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    const int idx = __builtin_amdgcn_readfirstlane(L.wsync);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    if (idx >= (int)a.njobs) break;
    const JobDesc jd = a.jobs[idx];
    const TripletDesc td = a.desc[jd.trip];
    int* plane = PLANE ? a.plane + a.plane_off[jd.trip] : nullptr;
    if (jd.trip != staged) {
      stage_shifts(shb, a.words, td, threadIdx.x, blockDim.x);
      staged = jd.trip;
    }
    const int n0 = (int)td.len[0], n1 = (int)td.len[1], n2 = (int)td.len[2];
    const int PJ = n1 / H + 1, PK = n2 / W + 1;
    const uint64_t rows = face_rows((uint32_t)n0);
    if ((MODES & 1) && jd.panel == kWholeTriplet) {
      // Bottom faces, one per panel column ([PK][rows][W]), then the right face.
      int* fb = face;
      int* fr = face + rows * (uint64_t)(PK * W);
      int best = KIND == kLocal ? 0 : INT32_MIN;
      for (int pj = 0; pj < PJ; ++pj) {
        for (int pk = 0; pk < PK; ++pk) {
          int* col = fb + (uint64_t)pk * rows * W;
          PanelIO io;
          io.top = pj ? col : (pk ? a.bnd_plain[1] : a.bnd_plain[0]);
          io.left = pk ? fr : a.bnd_plain[2];
          io.bot = pj + 1 < PJ ? col : nullptr;
          io.right = pk + 1 < PK ? fr : nullptr;
          io.gen = 0;
          io.err = nullptr;
          io.wait_ticks = 0;
          int32_t* so = (KIND == kGlobal && pj == PJ - 1 && pk == PK - 1) ? a.scores + td.out : nullptr;
          best = max(best, sweep_panel<kPlain, KIND, PLANE, RJ, RK, XCH>(L, shb, a.sc, a.words, td, pj, pk,
                                                                    io, so, plane, capt));
        }
      }
      if (KIND != kGlobal) finish_whole(a.scores + td.out, best);
    } else if (MODES & 2) {
      const uint32_t p = jd.panel;
      const int pj = (int)(p / (uint32_t)PK), pk = (int)(p % (uint32_t)PK);
      const uint64_t fb_ints = rows * W * 2;  // (value, tag) entries
      const uint64_t per_panel = fb_ints + rows * RR * 2;
      int* pool = a.pface + td.face_off;
      int* base = pool + (uint64_t)p * per_panel;
      PanelIO io;
      io.top = pj ? pool + (uint64_t)(p - PK) * per_panel : (pk ? a.bnd_tagged[1] : a.bnd_tagged[0]);
      io.left = pk ? pool + (uint64_t)(p - 1) * per_panel + fb_ints : a.bnd_tagged[2];
      io.bot = pj + 1 < PJ ? base : nullptr;
      io.right = pk + 1 < PK ? base + fb_ints : nullptr;
      io.gen = gen;
      io.err = a.ctl + 1;
      io.wait_ticks = a.wait_ticks;
      int32_t* so = (KIND == kGlobal && pj == PJ - 1 && pk == PK - 1) ? a.scores + td.out : nullptr;
      const int best = sweep_panel<kTagged, KIND, PLANE, RJ, RK, XCH>(L, shb, a.sc, a.words, td, pj, pk, io,
                                                                so, plane, capt);
      if (KIND != kGlobal)
        finish_panel(a, jd.trip, td.out, PJ * PK, best);
      else if (so && threadIdx.x == 0)
        publish_score(so, split_score(L, td, pj, pk, a.sc.gap2), io.err);
    }
  }
}

// ---- Packed pairs: two triplets per lane, one 16-bit half each. ----------
//
// Two triplets of a batch are swept together by one wavefront over a common
// panel grid (each axis padded to the longer of the two), every register
// holding the pair's two values of one cell, one per 16-bit half. A cell
// takes 5 packed additions (v_pk_add_u16) and 3 packed three-input maxima
// (v_pk_maximum3_f16), 4 instructions per cell update against 7 in int32.
//
// The maximum is a half-precision instruction used on integers, exactly:
// every value a lane ever holds is an integer in [1024, 31743], whose bit
// patterns are positive normal half-precision numbers (0x0400 .. 0x7BFF:
// no zero, no subnormal, no infinity, no NaN), and for those the float
// order of the bit patterns is the integer order; a maximum returns one of
// its inputs unchanged. The additions are plain 16-bit integer additions.
// What keeps every value in range (checked on the host per batch, otherwise
// the batch takes the int32 kernels):
//  * every substitution term s - 2*gap is >= 0, so no addition lowers a
//    value and the lookups need no sign extension;
//  * predecessors outside the tensor (the virtual faces, and the slices
//    before 0 that skewed lanes compute while filling) start at kSentP =
//    1024 and grow only along their own paths, by at most maxA per residue
//    of the path (maxA = the largest term), to below base - 512;
//  * a real cell holds base + M', with base above every such value and
//    M' >= 0, so a move from outside the tensor never wins (this also
//    replaces the -128 row and column tables of the int32 kernels); the one
//    real start, M'(0,0,0) = 0, is set explicitly;
//  * base + maxA * (the longest path in the padded box, drain included)
//    stays at or below 31743.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef unsigned short u2v __attribute__((ext_vector_type(2)));
constexpr uint32_t kSentP = 0x0400u;  // 1024 in both halves (see above)

__device__ __forceinline__ uint32_t padd(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u2v, a) + __builtin_bit_cast(u2v, b));
}
__device__ __forceinline__ uint32_t pmax3(uint32_t a, uint32_t b, uint32_t c) {
  const h2v x = __builtin_bit_cast(h2v, a), y = __builtin_bit_cast(h2v, b), z = __builtin_bit_cast(h2v, c);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
}
__device__ __forceinline__ uint32_t pmax2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_maximum(__builtin_bit_cast(h2v, a), __builtin_bit_cast(h2v, b)));
}
// Integer forms, for differences that need not be normal half patterns.
__device__ __forceinline__ uint32_t psub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u2v, a) - __builtin_bit_cast(u2v, b));
}
__device__ __forceinline__ uint32_t umax2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u2v, a), __builtin_bit_cast(u2v, b)));
}

// Per-slice byte selectors of a pair, for v_perm_b32: slice i of the common
// sweep picks byte code_a(i) of triplet a's table into the low half and byte
// code_b(i) of b's table into the high half (codes of S0[i-1] for 1 <= i <=
// n0 of that triplet, 0 elsewhere); covers slices -kShiftPre .. n0 + 47.
__device__ __forceinline__ void stage_selectors(uint32_t* sel, const uint32_t* __restrict__ words,
                                                const TripletDesc& ta, const TripletDesc& tb, int n0) {
  const int total = n0 + 64;
  for (int q = threadIdx.x & 63; q < total; q += 64) {
    const int i = q - kShiftPre;
    const uint32_t ca = (i >= 1 && i <= (int)ta.len[0]) ? residue_at(words, ta.off[0], (uint32_t)(i - 1)) : 0u;
    const uint32_t cb = (i >= 1 && i <= (int)tb.len[0]) ? residue_at(words, tb.off[0], (uint32_t)(i - 1)) : 0u;
    sel[q] = ca | 0x0C00u | ((cb + 4u) << 16) | 0x0C000000u;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// LDS of a packed wavefront: the lanes' edge slots and the capture tile
// (one object), and the halo rings, one object per chunk half. Staging of
// chunk c + 1 goes to the half that chunk c does not read. Kept as two
// objects, each a fixed object in its copy of the chunk body, the halves
// take static addresses. (The compiler still makes a chunk's first halo
// read wait for the loads in flight, since a lane's read picks between a
// ring row and a slot; the other wave on the SIMD covers that wait.)
template <int RJ, int RK>
struct PkLds {
  __attribute__((aligned(16))) int sR[64][RJ];  // right column of each lane
  __attribute__((aligned(16))) int sB[64][RK];  // bottom row of each lane
  int sX[64];                                   // bottom of each lane's left halo
  int cap[RJ * RK];                             // tile of triplet a's score cell
  int wsync;
};
template <int RJ, int RK>
struct PkRing {
  static constexpr int H = kGJ * RJ, W = kGK * RK;
  __attribute__((aligned(16))) int T[kChunk][W];    // top face rows of the chunk
  __attribute__((aligned(16))) int C[kChunk][kGK];  // corners of the top-edge lanes
  __attribute__((aligned(16))) int L[kChunk][H];    // left face rows of the chunk
};

// One panel of a pair (plain faces in the wave's workspace, one 32-bit word
// per entry holding both halves). Global scoring captures each triplet's
// cell (n0, n1, n2) when the panel holds it: triplet a's tile into L.cap,
// b's into capb. Semi-global and local scoring fold the panel's cells into
// the lane's running best (both halves; see k_sweep_pk for its meaning).
template <int RJ, int RK, int KIND, bool FUSED, int XCH, bool DMA>
__device__ void sweep_panel_pk(PkLds<RJ, RK>& L, PkRing<RJ, RK>& R0, PkRing<RJ, RK>& R1, int* capb,
                               const uint32_t* sel, const DevScoring& sc,
                               const uint32_t* __restrict__ words, const TripletDesc& ta,
                               const TripletDesc& tb, int n0, int pj, int pk, const int* top, const int* left,
                               int* bot, int* right, uint32_t base2, uint32_t& best, uint32_t kc) {
  constexpr int H = kGJ * RJ, W = kGK * RK, RR = H + 4;
  constexpr bool PAD = KIND != kGlobal;
  const int lane = threadIdx.x & 63;
  const int y = lane >> 3, x = lane & 7;
  const int j0 = pj * H + y * RJ, k0 = pk * W + x * RK;
  const int n1a = (int)ta.len[1], n1b = (int)tb.len[1], n2a = (int)ta.len[2], n2b = (int)tb.len[2];
  const uint32_t* bt = sc.byte_tab;
  // Row and column tables of both triplets (code 0 outside a sequence).
  // Semi-global and local scoring take all-zero tables, per triplet, on
  // row 0, column 0 and past the triplet's own last row and column: a move
  // that consumes a residue which is not there then scores no better than
  // the gaps it replaces, so those cells never beat a cell of the triplet
  // itself (the padding argument of the int32 kernels, with 0 for -128,
  // as no term may be negative here).
  uint32_t TBa[RJ], TBb[RJ], TCa[RK], TCb[RK], C2[RJ][RK];
  uint32_t cca[RK], ccb[RK];
  bool za[RK], zb[RK];
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    const int j = j0 + r;
    const uint32_t ba = (j >= 1 && j <= n1a) ? residue_at(words, ta.off[1], (uint32_t)(j - 1)) : 0u;
    const uint32_t bb = (j >= 1 && j <= n1b) ? residue_at(words, tb.off[1], (uint32_t)(j - 1)) : 0u;
    TBa[r] = (PAD && (j == 0 || j > n1a)) ? 0u : pick4(ba, bt[0], bt[1], bt[2], bt[3]);
    TBb[r] = (PAD && (j == 0 || j > n1b)) ? 0u : pick4(bb, bt[0], bt[1], bt[2], bt[3]);
  }
#pragma unroll
  for (int c = 0; c < RK; ++c) {
    const int k = k0 + c;
    cca[c] = (k >= 1 && k <= n2a) ? residue_at(words, ta.off[2], (uint32_t)(k - 1)) : 0u;
    ccb[c] = (k >= 1 && k <= n2b) ? residue_at(words, tb.off[2], (uint32_t)(k - 1)) : 0u;
    za[c] = PAD && (k == 0 || k > n2a);
    zb[c] = PAD && (k == 0 || k > n2b);
    TCa[c] = za[c] ? 0u : pick4(cca[c], bt[0], bt[1], bt[2], bt[3]);
    TCb[c] = zb[c] ? 0u : pick4(ccb[c], bt[0], bt[1], bt[2], bt[3]);
  }
#pragma unroll
  for (int r = 0; r < RJ; ++r)
#pragma unroll
    for (int c = 0; c < RK; ++c)
      C2[r][c] = (za[c] ? 0u : ((TBa[r] >> (cca[c] << 3)) & 0xFFu)) |
                 ((zb[c] ? 0u : ((TBb[r] >> (ccb[c] << 3)) & 0xFFu)) << 16);

  uint32_t P[RJ][RK], D[RJ][RK], Lp[RJ], Tp[RK];
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    Lp[r] = kSentP * 0x10001u;
#pragma unroll
    for (int c = 0; c < RK; ++c) P[r][c] = D[r][c] = kSentP * 0x10001u;
  }
#pragma unroll
  for (int c = 0; c < RK; ++c) Tp[c] = kSentP * 0x10001u;

  const int nsteps = n0 + 1 + kSkew;
  const int nchunks = (nsteps + kChunk - 1) / kChunk;
  // Capture: the lane holding cell (n1, n2) of a triplet in this panel keeps
  // its tile at that triplet's slice n0.
  const int rsa = n1a - j0, csa = n2a - k0;
  const int rsb = n1b - j0, csb = n2b - k0;
  const bool own_a = rsa >= 0 && rsa < RJ && csa >= 0 && csa < RK;
  const bool own_b = rsb >= 0 && rsb < RJ && csb >= 0 && csb < RK;
  const int n0a = (int)ta.len[0], n0b = (int)tb.len[0];

  // Semi-global and local scoring (g = -2*gap >= 0). fi = g*(i + j0 + k0)
  // for the lane's slice i of the current step; a cell of anti-diagonal
  // class d = r + c of the tile lies at index sum i + j0 + k0 + d.
  constexpr int ND = RJ + RK - 1;
  const int g = -sc.gap2;
  const uint32_t g2 = (uint32_t)g * 0x10001u;
  int fi = g * (j0 + k0 - y - x);
  // Semi-global: the halves of the rows and columns that are a triplet's
  // last row n1 or last column n2 (masks of both halves).
  uint32_t RM[RJ], CM[RK], rcany = 0;
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    RM[r] = (r == rsa ? 0xFFFFu : 0u) | (r == rsb ? 0xFFFF0000u : 0u);
    rcany |= RM[r];
  }
#pragma unroll
  for (int c = 0; c < RK; ++c) {
    CM[c] = (c == csa ? 0xFFFFu : 0u) | (c == csb ? 0xFFFF0000u : 0u);
    rcany |= CM[c];
  }
  const bool axis_panel = pj == 0 || pk == 0;

  const uint32_t frows = face_rows((uint32_t)n0);
  constexpr uint32_t ts = W * 4u, RRB = RR * 4u;
  const Rsrc r_top = make_rsrc(top, (uint64_t)frows * ts);
  const Rsrc r_left = make_rsrc(left, (uint64_t)frows * RRB);
  const Rsrc r_bot = make_rsrc(bot ? bot : top, bot ? (uint64_t)frows * ts : 0);
  const Rsrc r_right = make_rsrc(right ? right : left, right ? (uint64_t)frows * RRB : 0);

  // Staging, as in sweep_panel (plain faces): value q of a chunk is entry
  // lane + 64 q of the top, corner or left ring.
  constexpr int QT = kChunk * W / 64, QC = kChunk * kGK / 64, QL = kChunk * H / 64;
  constexpr int NPF = QT + QC + QL;
  constexpr int RT = 64 / W, RL = 64 / H;
  static_assert(64 % W == 0 && 64 % H == 0 && QC == 1, "ring widths must divide 64");
  const int eT = lane % W;
  const uint32_t offT = (uint32_t)((kGJ - 1 + lane / W) * (int)ts + eT * 4);
  const int eC = lane % kGK;
  const bool corner_from_left = eC == 0;
  const uint32_t offC = corner_from_left ? (uint32_t)((kGK - 1 + lane / kGK) * (int)RRB)
                                         : (uint32_t)((kGJ - 2 + lane / kGK) * (int)ts + (eC * RK - 1) * 4);
  const int eL = lane % H;
  const uint32_t offL = (uint32_t)((kGK - 1 + lane / H) * (int)RRB + (4 + eL) * 4);
  int pf[DMA ? 1 : NPF];
  auto stage_load = [&](int c, PkRing<RJ, RK>& dst) {
    const uint32_t cb0 = (uint32_t)(c * kChunk);
    if (DMA) {
      // Straight into the ring half of chunk c (lane l's word of each load
      // lands at the destination + 4 l, which is where it belongs); the
      // corner loads go to the same slots from the top or the left face,
      // so each lane takes only one of them.
      typedef __attribute__((address_space(3))) void* LdsPtr;
#pragma unroll
      for (int q = 0; q < QT; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r_top, (LdsPtr)(&dst.T[0][0] + 64 * q), 4, offT,
                                                 (cb0 + q * RT) * ts, 0, 0);
      if (corner_from_left)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r_left, (LdsPtr)&dst.C[0][0], 4, offC, cb0 * RRB, 0, 0);
      else
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r_top, (LdsPtr)&dst.C[0][0], 4, offC, cb0 * ts, 0, 0);
#pragma unroll
      for (int q = 0; q < QL; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r_left, (LdsPtr)(&dst.L[0][0] + 64 * q), 4, offL,
                                                 (cb0 + q * RL) * RRB, 0, 0);
      return;
    }
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      if (q < QT) {
        pf[q] = (int)__builtin_amdgcn_raw_buffer_load_b32(r_top, offT, (cb0 + q * RT) * ts, 0);
      } else if (q < QT + QC) {
        const uint32_t ot = corner_from_left ? kOob : offC, ol = corner_from_left ? offC : kOob;
        pf[q] = (int)(__builtin_amdgcn_raw_buffer_load_b32(r_top, ot, cb0 * ts, 0) |
                      __builtin_amdgcn_raw_buffer_load_b32(r_left, ol, cb0 * RRB, 0));
      } else {
        pf[q] = (int)__builtin_amdgcn_raw_buffer_load_b32(r_left, offL, (cb0 + (q - QT - QC) * RL) * RRB, 0);
      }
    }
  };
  auto stage_finish = [&](int c, PkRing<RJ, RK>& dst) {
    if (DMA) {
      // The loads of chunk c were issued at the first step of chunk c - 1,
      // ahead of that chunk's face stores (kStores per step); vector memory
      // operations complete in issue order, so once no more than those
      // stores are outstanding the loads are done, and the stores need not
      // be waited for. Chunk 0's loads were issued just before, with no
      // store after them.
      constexpr int kStores = RK / 4 + RJ / 4 + 1;
      constexpr int kAfter = kStores * kChunk;
      static_assert(kAfter < 64, "vmcnt holds at most 63");
      constexpr int kWaitAfter = (kAfter & 15) | ((kAfter >> 4) << 14) | (0x7 << 4) | (0xF << 8);
      if (c == 0)
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      else
        __builtin_amdgcn_s_waitcnt(kWaitAfter);  // vmcnt(kAfter)
      return;
    }
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      if (q < QT)
        (&dst.T[0][0])[lane + 64 * q] = pf[q];
      else if (q < QT + QC)
        dst.C[0][lane] = pf[q];
      else
        (&dst.L[0][0])[lane + 64 * (q - QT - QC)] = pf[q];
    }
  };
  stage_load(0, R0);
#pragma unroll
  for (int r = 0; r < RJ; ++r) L.sR[lane][r] = (int)(kSentP * 0x10001u);
#pragma unroll
  for (int c = 0; c < RK; ++c) L.sB[lane][c] = (int)(kSentP * 0x10001u);
  L.sX[lane] = (int)(kSentP * 0x10001u);

  const bool y0 = y == 0, x0 = x == 0;
  const bool tring = XCH || y0, lring = XCH || x0;
  // Halo rows: edge lanes read the chunk's ring half, inner lanes their
  // neighbour's slot (the same every step).
  const int* t_slot = &L.sB[y0 ? 0 : lane - 8][0];
  const int t_str = tring ? W : 0;
  const int* c_slot = &L.sX[y0 ? 0 : lane - 8];
  const int c_str = tring ? kGK : 0;
  const int* l_slot = &L.sR[x0 ? 0 : lane - 1][0];
  const int l_str = lring ? H : 0;
  const int up_addr = ((lane + 64 - kGK) & 63) << 2;
  const uint32_t vo_bot = (y == kGJ - 1) ? (uint32_t)(x * RK * 4) : kOob;
  const uint32_t vo_right = (x == kGK - 1) ? (uint32_t)((4 + y * RJ) * 4) : kOob;
  const uint32_t vo_corner = (x == kGK - 1 && y == 0) ? 0u : kOob;
  const int sl_base = kShiftPre - y - x;
  const bool seed_lane = pj == 0 && pk == 0 && lane == 0;

  // Chunk c reads ring half cur and stages chunk c + 1 into nxt. With loads
  // straight to LDS the loop below takes two chunks per turn, so that both
  // halves are fixed objects in each copy of the body.
  auto run_chunk = [&](int c, PkRing<RJ, RK>& cur, PkRing<RJ, RK>& nxt) __attribute__((always_inline)) {
    stage_finish(c, cur);
    const bool more = c + 1 < nchunks;
    const int cb0 = c * kChunk;
    const bool cap_chunk = (n0a >= cb0 - kSkew && n0a <= cb0 + kChunk - 1) ||
                           (n0b >= cb0 - kSkew && n0b <= cb0 + kChunk - 1);
    const uint32_t vb = vo_bot + (uint32_t)cb0 * ts, vr = vo_right + (uint32_t)cb0 * RRB,
                   vc = vo_corner + (uint32_t)cb0 * RRB;
    const int* tb = tring ? &cur.T[0][x * RK] : t_slot;
    const int* cbp = tring ? &cur.C[0][x] : c_slot;
    const int* lb = lring ? &cur.L[0][y * RJ] : l_slot;
    const uint32_t* sp = sel + sl_base + cb0;
    uint32_t selv[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) selv[s] = sp[s];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      if (s == 0 && more) stage_load(c + 1, nxt);
      const int t = cb0 + s;
      const uint32_t sv = selv[s];
      uint32_t A[RJ], B[RK];
#pragma unroll
      for (int r = 0; r < RJ; ++r) A[r] = __builtin_amdgcn_perm(TBb[r], TBa[r], sv);
#pragma unroll
      for (int cc = 0; cc < RK; ++cc) B[cc] = __builtin_amdgcn_perm(TCb[cc], TCa[cc], sv);
      uint32_t T[RK], Lh[RJ];
#pragma unroll
      for (int cc = 0; cc < RK; cc += 4) {
        const v4i v = lds_v4(tb + s * t_str + cc);
        T[cc] = (uint32_t)v.x, T[cc + 1] = (uint32_t)v.y, T[cc + 2] = (uint32_t)v.z, T[cc + 3] = (uint32_t)v.w;
      }
#pragma unroll
      for (int r = 0; r < RJ; r += 4) {
        const v4i v = lds_v4(lb + s * l_str + r);
        Lh[r] = (uint32_t)v.x, Lh[r + 1] = (uint32_t)v.y, Lh[r + 2] = (uint32_t)v.z, Lh[r + 3] = (uint32_t)v.w;
      }
      uint32_t corner = (uint32_t)cbp[s * c_str];
      if (XCH) {
        // As in sweep_panel: inner lanes take their upper neighbour's row
        // and corner through ds_bpermute and their left neighbour's column
        // through a DPP row shift, from its previous-step registers.
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) {
          const uint32_t nb = (uint32_t)__builtin_amdgcn_ds_bpermute(up_addr, (int)P[RJ - 1][cc]);
          T[cc] = y0 ? T[cc] : nb;
        }
        {
          const uint32_t nb = (uint32_t)__builtin_amdgcn_ds_bpermute(up_addr, (int)Lp[RJ - 1]);
          corner = y0 ? corner : nb;
        }
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
          const uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)P[r][RK - 1], 0x111, 0xF, 0xF, true);
          Lh[r] = x0 ? Lh[r] : nb;
        }
      }
      const int i = t - y - x;  // this lane's slice
      if (KIND == kSemiGlobal && axis_panel) {
        // The axes hold 0 (stored base + g*index, both halves): at slice 0
        // the virtual row above the first panel row holds base + g*k and the
        // virtual column left of the first panel column base + g*j, and at
        // k = 0 the virtual row holds base + g*i; the single move (+0)
        // copies them in. Other moves from there take the zero row/column-0
        // tables and give values the single moves already reach.
        if (j0 == 0) {
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) T[cc] = i == 0 ? base2 + (uint32_t)(g * (k0 + cc)) * 0x10001u : T[cc];
          if (k0 == 0) T[0] = i >= 0 ? base2 + (uint32_t)(g * i) * 0x10001u : T[0];
        }
        if (k0 == 0) {
#pragma unroll
          for (int r = 0; r < RJ; ++r) Lh[r] = i == 0 ? base2 + (uint32_t)(g * (j0 + r)) * 0x10001u : Lh[r];
        }
      }
      // Local floors per anti-diagonal class, F_d = base + fi + g*d in both
      // halves (M >= 0); none before slice 0 (0 there, below every value).
      uint32_t F[ND];
      if (KIND == kLocal) {
        asm volatile("" : "+v"(fi));  // one step's floors live at a time
        const uint32_t f0 = i >= 0 ? base2 + (uint32_t)fi * 0x10001u : 0u;
#pragma unroll
        for (int d = 0; d < ND; ++d) F[d] = f0 + (uint32_t)d * g2;
      }
      // Terms of the previous slice first (formed while the halo reads are
      // in flight): Q = best of the single move along S0 and its two double
      // moves, X7 the triple move. The fused form computes them cell by cell
      // instead (no registers held for them across the tile). Local scoring
      // folds X7 and the floor into Q.
      uint32_t Q[RJ][RK], X7[RJ][RK], N[RJ][RK];
      auto prev_terms = [&](int r, int cc) {
        const uint32_t up_prev = r ? P[r - 1][cc] : Tp[cc];
        const uint32_t left_prev = cc ? P[r][cc - 1] : Lp[r];
        Q[r][cc] = pmax3(P[r][cc], padd(up_prev, A[r]), padd(left_prev, B[cc]));
        X7[r][cc] = padd(D[r][cc], padd(A[r], B[cc]));
        if (KIND == kLocal) Q[r][cc] = pmax3(Q[r][cc], X7[r][cc], F[r + cc]);
      };
      if (!FUSED) {
#pragma unroll
        for (int r = 0; r < RJ; ++r)
#pragma unroll
          for (int cc = 0; cc < RK; ++cc) prev_terms(r, cc);
      }
#pragma unroll
      for (int r = 0; r < RJ; ++r)
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) {
          if (FUSED) prev_terms(r, cc);
          const uint32_t up_cur = r ? N[r - 1][cc] : T[cc];
          const uint32_t left_cur = cc ? N[r][cc - 1] : Lh[r];
          const uint32_t diag_cur = r ? (cc ? N[r - 1][cc - 1] : Lh[r - 1]) : (cc ? T[cc - 1] : corner);
          const uint32_t x6 = padd(diag_cur, C2[r][cc]);
          if (KIND == kLocal)
            N[r][cc] = pmax3(pmax2(Q[r][cc], x6), up_cur, left_cur);
          else
            N[r][cc] = pmax3(pmax3(Q[r][cc], X7[r][cc], x6), up_cur, left_cur);
          // Global M'(0,0,0) = 0: the one real start, cell (0,0) of lane 0
          // of the first panel at step 0, set before any other cell reads it.
          if (KIND == kGlobal && r == 0 && cc == 0) N[0][0] = (t == 0 && seed_lane) ? base2 : N[0][0];
          D[r][cc] = x6;
        }

      // Masks of the halves whose triplet has this slice (0 <= i <= its n0)
      // and of those whose last slice it is.
      const uint32_t vm = ((uint32_t)i <= (uint32_t)n0a ? 0xFFFFu : 0u) | ((uint32_t)i <= (uint32_t)n0b ? 0xFFFF0000u : 0u);
      if (KIND == kLocal) {
        // M = stored value - F_d, never negative on slices from 0 (every
        // cell is floored); the best class maximum minus its floor.
        uint32_t sb = 0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          uint32_t m = 0, hold = 0;
          int cnt = 0;
#pragma unroll
          for (int r = 0; r < RJ; ++r) {
            if (d - r < 0 || d - r >= RK) continue;
            const uint32_t v = N[r][d - r];
            if (cnt == 0) m = v;
            else if (cnt & 1) hold = v;
            else m = pmax3(m, hold, v);
            ++cnt;
          }
          if (!(cnt & 1)) m = pmax2(m, hold);
          sb = umax2(sb, psub(m, F[d]));
        }
        best = umax2(best, sb & vm);
      } else if (KIND == kSemiGlobal) {
        // Cells of a triplet's last slice, row or column (on its slices 0
        // .. n0), as M + kc = stored - base - g*(i + j + k) + kc, which the
        // host keeps within [1, 0xFFFF]; masked cells give 0.
        const uint32_t sm = (i == n0a ? 0xFFFFu : 0u) | (i == n0b ? 0xFFFF0000u : 0u);
        if (((rcany | sm) & vm) != 0u) {
          const uint32_t off0 = ((uint32_t)(kc - (base2 & 0xFFFFu) - (uint32_t)fi) & 0xFFFFu) * 0x10001u;
          uint32_t sb = 0;
#pragma unroll
          for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int cc = 0; cc < RK; ++cc)
              sb = umax2(sb, padd(N[r][cc], psub(off0, (uint32_t)(r + cc) * g2)) & (RM[r] | CM[cc] | sm));
          best = umax2(best, sb & vm);
        }
      }
      fi += g;

      if (!XCH) {
#pragma unroll
        for (int r = 0; r < RJ; ++r) L.sR[lane][r] = (int)N[r][RK - 1];
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) L.sB[lane][cc] = (int)N[RJ - 1][cc];
        L.sX[lane] = (int)Lh[RJ - 1];
      }
#pragma unroll
      for (int cc = 0; cc < RK; cc += 4)
        __builtin_amdgcn_raw_buffer_store_b128(
            (v4i){(int)N[RJ - 1][cc], (int)N[RJ - 1][cc + 1], (int)N[RJ - 1][cc + 2], (int)N[RJ - 1][cc + 3]},
            r_bot, vb + (s * ts + cc * 4), 0, 0);
#pragma unroll
      for (int r = 0; r < RJ; r += 4)
        __builtin_amdgcn_raw_buffer_store_b128(
            (v4i){(int)N[r][RK - 1], (int)N[r + 1][RK - 1], (int)N[r + 2][RK - 1], (int)N[r + 3][RK - 1]},
            r_right, vr + (s * RRB + r * 4), 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32((int)T[RK - 1], r_right, vc + s * RRB, 0, 0);
      if (KIND == kGlobal && cap_chunk) {
        if (own_a && i == n0a) {
#pragma unroll
          for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int cc = 0; cc < RK; ++cc) L.cap[r * RK + cc] = (int)N[r][cc];
        }
        if (own_b && i == n0b) {
#pragma unroll
          for (int r = 0; r < RJ; ++r)
#pragma unroll
            for (int cc = 0; cc < RK; ++cc) capb[r * RK + cc] = (int)N[r][cc];
        }
      }
#pragma unroll
      for (int r = 0; r < RJ; ++r) {
        Lp[r] = Lh[r];
#pragma unroll
        for (int cc = 0; cc < RK; ++cc) P[r][cc] = N[r][cc];
      }
#pragma unroll
      for (int cc = 0; cc < RK; ++cc) Tp[cc] = T[cc];
    }
  };
  if constexpr (DMA) {
    for (int c = 0; c < nchunks; c += 2) {
      run_chunk(c, R0, R1);
      if (c + 1 < nchunks) run_chunk(c + 1, R1, R0);
    }
  } else {
    // Staged through registers, the rings are written by LDS stores, which
    // need no such care; one copy of the body keeps register pressure down.
    for (int c = 0; c < nchunks; ++c) run_chunk(c, (c & 1) ? R1 : R0, (c & 1) ? R0 : R1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// Persistent kernel of a packed plan: every job is a pair of whole triplets
// (descriptors 2p and 2p + 1; a lone last triplet is paired with itself),
// swept by one wavefront over all panels of the common grid, row by row, in
// the wave's own face workspace. pk_top / pk_left: plain sentinel faces
// holding kSentP in both halves. base: the stored value of M' = 0. Local
// scoring keeps each lane's best M per half, semi-global its best M + kc
// (kc > 0 keeps every candidate positive); the wave's maxima are the scores.
template <int RJ, int RK, int WPE, int KIND, bool FUSED, int XCH, bool DMA>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
k_sweep_pk(SweepArgs a, const int* pk_top, const int* pk_left, uint32_t base, uint32_t kc) {
  constexpr int H = kGJ * RJ, W = kGK * RK;
  __shared__ PkLds<RJ, RK> L;
  __shared__ PkRing<RJ, RK> R0, R1;
  __shared__ int capb[RJ * RK];
  extern __shared__ uint32_t selw[];
  int* face = a.face + (uint64_t)blockIdx.x * a.face_stride;
  const uint32_t base2 = base * 0x10001u;
  for (;;) {
    if (threadIdx.x == 0) L.wsync = atomicAdd(a.counter, 1);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    const int idx = __builtin_amdgcn_readfirstlane(L.wsync);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    if (idx >= (int)a.njobs) break;
    const JobDesc jd = a.jobs[idx];
    const TripletDesc ta = a.desc[jd.trip], tb = a.desc[jd.trip + 1];
    const int n0 = (int)max(ta.len[0], tb.len[0]);
    const int n1 = (int)max(ta.len[1], tb.len[1]), n2 = (int)max(ta.len[2], tb.len[2]);
    stage_selectors(selw, a.words, ta, tb, n0);
    const int PJ = n1 / H + 1, PK = n2 / W + 1;
    const uint64_t rows = face_rows((uint32_t)n0);
    int* fb = face;
    int* fr = face + rows * (uint64_t)(PK * W);
    const int pja = (int)ta.len[1] / H, pka = (int)ta.len[2] / W;
    const int pjb = (int)tb.len[1] / H, pkb = (int)tb.len[2] / W;
    uint32_t best = 0;
    for (int pj = 0; pj < PJ; ++pj) {
      for (int pk = 0; pk < PK; ++pk) {
        int* col = fb + (uint64_t)pk * rows * W;
        sweep_panel_pk<RJ, RK, KIND, FUSED, XCH, DMA>(L, R0, R1, capb, selw, a.sc, a.words, ta, tb, n0, pj, pk,
                                                      pj ? col : pk_top, pk ? fr : pk_left,
                                                      pj + 1 < PJ ? col : nullptr, pk + 1 < PK ? fr : nullptr,
                                                      base2, best, kc);
        // Scores of the triplets whose last cell this panel held (the owner
        // lane's tile is in LDS; lane 0 reads the cell and stores the score).
        if (KIND == kGlobal && (threadIdx.x & 63) == 0) {
          if (pj == pja && pk == pka) {
            const int r = (int)ta.len[1] - pja * H, cc = (int)ta.len[2] - pka * W;
            const int v = L.cap[(r % RJ) * RK + (cc % RK)] & 0xFFFF;
            __hip_atomic_store(a.scores + ta.out,
                               v - (int)base + a.sc.gap2 * (int)(ta.len[0] + ta.len[1] + ta.len[2]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          }
          if (pj == pjb && pk == pkb) {
            const int r = (int)tb.len[1] - pjb * H, cc = (int)tb.len[2] - pkb * W;
            const int v = (int)((uint32_t)capb[(r % RJ) * RK + (cc % RK)] >> 16);
            __hip_atomic_store(a.scores + tb.out,
                               v - (int)base + a.sc.gap2 * (int)(tb.len[0] + tb.len[1] + tb.len[2]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      }
    }
    if (KIND != kGlobal) {
      // The wave's best per half; lane 0 stores both scores.
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) best = umax2(best, (uint32_t)__shfl_xor((int)best, o));
      if ((threadIdx.x & 63) == 0) {
        const int off = KIND == kSemiGlobal ? (int)kc : 0;
        __hip_atomic_store(a.scores + ta.out, (int)(best & 0xFFFFu) - off, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.scores + tb.out, (int)(best >> 16) - off, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// Plain sentinel faces of the packed kernels: kSentP in both halves.
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Sentinel faces for panels on the tensor edge, in the plain layout (one
// int per entry) and the tagged layout (value, kTagAlways). Every value is
// kSent except the seeded top faces' entry for k = 0 at slice 0, which is 0
// (it makes M'(0,0,0) = 0 through the move from the virtual row above).
__global__ void k_init_boundary(Boundary b, int top_entries, int left_entries, int seed_index) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < top_entries; i += stride) {
    const int v = i == seed_index ? 0 : kSent;
    b.plain[0][i] = v;
    b.plain[1][i] = kSent;
    b.tagged[0][2 * i] = v;
    b.tagged[0][2 * i + 1] = kTagAlways;
    b.tagged[1][2 * i] = kSent;
    b.tagged[1][2 * i + 1] = kTagAlways;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < left_entries; i += stride) {
    b.plain[2][i] = kSent;
    b.tagged[2][2 * i] = kSent;
    b.tagged[2][2 * i + 1] = kTagAlways;
  }
}

// Before each run: next generation, error flag cleared, queue head zeroed,
// and the per-triplet reduction pairs reset (best = INT32_MIN, 0 finished).
__global__ void k_prepare(int* ctl, int* counter, int* red, uint32_t nred) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = ctl[0] + 1;
    ctl[1] = 0;
    counter[0] = 0;
  }
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nred; q += gridDim.x * blockDim.x) {
    red[2 * (uint64_t)q] = INT32_MIN;
    red[2 * (uint64_t)q + 1] = 0;
  }
}

// Kernel variants: tile shape (rows, columns, waves per SIMD), kind, whether
// the last slice is written out (traceback planes), and the lane exchange
// (0: LDS slot arrays, 1: ds_bpermute and DPP row shifts).
#define TRIOSEQ_SHAPES(X)                                                                        \
  X(4, 4, 4, 0, false, 0) X(4, 4, 2, 0, false, 0) X(8, 4, 2, 0, false, 0) X(4, 8, 2, 0, false, 0) \
  X(4, 4, 2, 1, false, 0) X(4, 4, 2, 2, false, 0) X(8, 4, 2, 1, false, 0) X(8, 4, 2, 2, false, 0) \
  X(4, 4, 2, 0, true, 0) X(4, 4, 2, 0, false, 1) X(8, 4, 2, 0, false, 1) X(4, 4, 2, 0, true, 1)   \
  X(4, 4, 2, 2, true, 0)
#define TRIOSEQ_MODES(X, r, c, w, k, p, x) X(r, c, w, 1, k, p, x) X(r, c, w, 2, k, p, x) X(r, c, w, 3, k, p, x)

}  // namespace

// Packed kernels: lane tile and register budget; the 4 x 4 two-wave form
// holds the previous slice's terms for the whole tile, the others form them
// cell by cell.
// (rows, columns, waves per SIMD, kind, fused, lane exchange, LDS-direct
// staging); semi-global and local scoring exist in the four plain forms.
#define TRIOSEQ_PK_PLAIN(X, k)                                                                    \
  X(4, 4, 2, k, false, 0, false) X(4, 4, 3, k, true, 0, false) X(8, 4, 2, k, true, 0, false)      \
  X(4, 8, 2, k, true, 0, false)
#define TRIOSEQ_PK_SHAPES(X)                                                                      \
  TRIOSEQ_PK_PLAIN(X, 0) TRIOSEQ_PK_PLAIN(X, 1) TRIOSEQ_PK_PLAIN(X, 2)                            \
  X(4, 4, 2, 0, false, 1, false) X(4, 4, 2, 0, false, 0, true) X(4, 4, 3, 0, true, 0, true)       \
  X(8, 4, 2, 0, true, 0, true) X(4, 8, 2, 0, true, 0, true)
#define TRIOSEQ_PK_MATCH(r, c, w, k, x, d) \
  (ks.rj == r && ks.rk == c && ks.wpe == w && kind == k && ks.xch == x && ks.dma == d)

bool pk_shape_supported(const KernelShape& ks, int kind) {
#define X(r, c, w, k, f, x, d) \
  if (TRIOSEQ_PK_MATCH(r, c, w, k, x, d)) return true;
  TRIOSEQ_PK_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_sweep_pk(const KernelShape& ks, int kind, const SweepArgs& a, const int* pk_top,
                           const int* pk_left, uint32_t base, uint32_t kc, int grid, hipStream_t s) {
  const size_t lds = (size_t)(a.lds_n0 + 64) * 4;
#define X(r, c, w, k, f, x, d)                                                                     \
  if (TRIOSEQ_PK_MATCH(r, c, w, k, x, d)) {                                                        \
    hipLaunchKernelGGL((k_sweep_pk<r, c, w, k, f, x, d>), dim3(grid), dim3(64), lds, s, a, pk_top, \
                       pk_left, base, kc);                                                         \
    return hipGetLastError();                                                                      \
  }
  TRIOSEQ_PK_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t sweep_pk_occupancy(const KernelShape& ks, int kind, uint32_t lds_n0, int* blocks_per_cu) {
#define X(r, c, w, k, f, x, d)                                                                     \
  if (TRIOSEQ_PK_MATCH(r, c, w, k, x, d))                                                          \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                           \
        blocks_per_cu, k_sweep_pk<r, c, w, k, f, x, d>, 64, (size_t)(lds_n0 + 64) * 4);
  TRIOSEQ_PK_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}
#undef TRIOSEQ_PK_MATCH

hipError_t launch_fill_packed_sentinel(uint32_t* p, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, s, p, n, kSentP * 0x10001u);
  return hipGetLastError();
}

bool shape_supported(const KernelShape& ks, int kind) {
#define X(a, b, w, k, p, x) \
  if (!p && ks.rj == a && ks.rk == b && ks.wpe == w && kind == k && ks.xch == x) return true;
  TRIOSEQ_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_init_boundary(const KernelShape& ks, const Boundary& b, hipStream_t s) {
  const int W = panel_cols(ks), RR = right_face_row(ks);
  const int top_entries = (int)b.rows * W, left_entries = (int)b.rows * RR;
  // The top lane x = 0 reads slice 0 from row kGJ - 1 (entry 0).
  hipLaunchKernelGGL(k_init_boundary, dim3(256), dim3(256), 0, s, b, top_entries, left_entries,
                     (kGJ - 1) * W);
  return hipGetLastError();
}

hipError_t launch_prepare(int* ctl, int* counter, int* red, uint32_t nred, hipStream_t s) {
  const uint32_t blocks = nred == 0 ? 1 : nred > 256 * 256 ? 256 : (nred + 255) / 256;
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, ctl, counter, red, nred);
  return hipGetLastError();
}

hipError_t launch_sweep(const KernelShape& ks, int modes, const SweepArgs& a, int grid,
                        hipStream_t s) {
  const size_t lds = shift_lds_bytes(a.lds_n0);
  const int kind = a.sc.kind;
  const bool plane = a.plane != nullptr;
  const bool group = modes == 2 && ks.group == kPairs;
#define Y(r, c, w, m, k, p, x)                                                                  \
  if (ks.rj == r && ks.rk == c && ks.wpe == w && modes == m && kind == k && plane == p &&       \
      ks.xch == x) {                                                                            \
    if (m == 2 && group)                                                                        \
      hipLaunchKernelGGL((k_panel_group<r, c, w, k, p, x>), dim3(grid), dim3(128 * kPairs), lds,\
                         s, a);                                                                 \
    else if (m == 2)                                                                            \
      hipLaunchKernelGGL((k_panel<r, c, w, k, p, x>), dim3(grid), dim3(128), lds, s, a);        \
    else                                                                                        \
      hipLaunchKernelGGL((k_sweep<r, c, w, m, k, p, x>), dim3(grid), dim3(64), lds, s, a);      \
    return hipGetLastError();                                                                   \
  }
#define X(r, c, w, k, p, x) TRIOSEQ_MODES(Y, r, c, w, k, p, x)
  TRIOSEQ_SHAPES(X)
#undef X
#undef Y
  return hipErrorInvalidValue;
}

hipError_t sweep_occupancy(const KernelShape& ks, int modes, int kind, bool plane, uint32_t lds_n0,
                           int* waves_per_cu) {
  const bool group = modes == 2 && ks.group == kPairs;
#define Y(r, c, w, m, k, p, x)                                                                    \
  if (ks.rj == r && ks.rk == c && ks.wpe == w && modes == m && kind == k && plane == p &&         \
      ks.xch == x)                                                                                \
    return (m == 2 && group) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                      \
                                   waves_per_cu, k_panel_group<r, c, w, k, p, x>, 128 * kPairs,   \
                                   shift_lds_bytes(lds_n0))                                       \
           : m == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                               \
                          waves_per_cu, k_panel<r, c, w, k, p, x>, 128, shift_lds_bytes(lds_n0))  \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(                               \
                          waves_per_cu, k_sweep<r, c, w, m, k, p, x>, 64, shift_lds_bytes(lds_n0));
#define X(r, c, w, k, p, x) TRIOSEQ_MODES(Y, r, c, w, k, p, x)
  TRIOSEQ_SHAPES(X)
#undef X
#undef Y
  return hipErrorInvalidValue;
}

}  // namespace trioseq

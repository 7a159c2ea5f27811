// Internal interfaces between the host runtime (api.cpp) and the gfx950
// kernels (sweep.hip). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trioseq {

// Finite stand-in for "no such predecessor" (the -infinity of Eq. 1). Every
// real value of the shifted score M' (defined in sweep.hip) lies in
// [0, 2^27); sentinels stay within [2*kSent - 2^20, kSent + 2^20], so no
// sum of two of them, plus table terms, wraps int32.
constexpr int kSent = -(1 << 29);

// Lane grid of one wavefront: 8 x 8 lanes, each owning an RJ x RK cell tile.
constexpr int kGJ = 8;
constexpr int kGK = 8;
constexpr int kSkew = (kGJ - 1) + (kGK - 1);
// Steps per face-staging chunk; the LDS ring holds two chunks.
constexpr int kChunk = 8;
constexpr int kRing = 2 * kChunk;
// Longest sequence accepted on the sweep axis: its per-slice lookup shifts
// live in LDS, one byte per slice.
constexpr int kMaxSweepLen = 16384;
// The per-slice lookup shifts in LDS are padded by kShiftPre entries before
// slice 0 (skewed lanes read slices down to -kSkew).
constexpr int kShiftPre = 16;
// Face buffers hold one row per producer step. A sweep of n0 + 1 slices runs
// at most n0 + 1 + kSkew + kChunk - 1 steps, and consumers read up to
// kGJ - 1 rows past the producer's last, so n0 + 1 + kSkew + 2 * kChunk rows
// cover every access.
__host__ __device__ inline uint32_t face_rows(uint32_t n0) { return n0 + 1 + kSkew + 2 * kChunk; }
// Dynamic LDS bytes for the sweep shifts of a sequence of length n0.
__host__ __device__ inline uint32_t shift_lds_bytes(uint32_t n0) { return (n0 + 64 + 15) & ~15u; }

// Scoring tables derived from the substitution matrix and gap score.
// byte_tab[r] packs, in byte x, the value sub[x][r] - 2*gap (a double move's
// term in the shifted recurrence); byte_tab[4] is the "row/column 0" table
// whose every byte is -128. pair_tab[4*r+s] = sub[r][s] - 2*gap.
struct DevScoring {
  uint32_t byte_tab[5];
  int32_t pair_tab[16];
  int32_t gap2;  // 2*gap, to undo the shift at the end
  int32_t kind;  // alignment kind: kGlobal, kSemiGlobal or kLocal
};

// Alignment kinds (paper, Section II: the value of v and the initialisation
// of the tensor select global, semi-global or local alignment).
constexpr int kGlobal = 0;
constexpr int kSemiGlobal = 1;
constexpr int kLocal = 2;

// One triplet as the kernels see it: the three sequences already assigned
// to the sweep axis (0), the row axis (1) and the column axis (2).
struct TripletDesc {
  uint64_t off[3];    // word offsets of the three sequences in the word array
  uint32_t len[3];    // lengths on the sweep, row and column axes
  uint32_t out;       // index of this triplet's score in the caller's output
  uint64_t face_off;  // split triplets: ints from the panel-face pool base
};

// A queue entry: one triplet swept whole by one wave, or one panel of a
// split triplet (panel = pj * PK + pk).
constexpr uint32_t kWholeTriplet = 0xFFFFFFFFu;
struct JobDesc {
  uint32_t trip;
  uint32_t panel;
};

// Sentinel faces for edge panels (rows = face_rows of the longest sweep):
// [0] top with the seed at slice 0, k = 0; [1] top; [2] left. plain: one
// int per entry (whole-triplet jobs); tagged: (value, tag) per entry.
struct Boundary {
  int* plain[3];
  int* tagged[3];
  uint32_t rows;
};

struct SweepArgs {
  const uint32_t* words;
  const TripletDesc* desc;
  const JobDesc* jobs;
  uint32_t njobs;
  uint32_t lds_n0;      // longest sweep length the dynamic LDS was sized for
  int32_t* scores;
  int* counter;         // job queue head (zeroed by k_prepare)
  int* ctl;             // [0] run generation, [1] error flag
  int* face;            // per-wave workspace for whole-triplet jobs
  uint64_t face_stride; // ints per wave
  int* pface;           // panel-face pool of split triplets
  const int* bnd_plain[3];
  const int* bnd_tagged[3];
  // Semi-global and local scoring of split triplets: per triplet t,
  // red[2t] = best value over the panels folded in so far, red[2t + 1] =
  // panels finished (both reset by k_prepare).
  int* red;
  // Optional (traceback): triplet t also writes its last slice, M[n0][j][k]
  // for 0 <= j <= n1, 0 <= k <= n2, unshifted, to plane + plane_off[t] at
  // index j * (n2 + 1) + k. plane is null when no plane is wanted.
  int* plane;
  const uint64_t* plane_off;
  // Bound on every wait for another wavefront, in ticks of the 100 MHz wall
  // clock; past it the wave raises ctl[1] and goes on.
  uint64_t wait_ticks;
  DevScoring sc;
};

// The wait bound new launches take (trioseq_set_wait_limit; 2 s by default).
uint64_t wait_limit_ticks();

// Panels of one strip job (strip workgroups: one compute and one memory wave
// per panel, all in one workgroup).
constexpr int kStripPanels = 4;
struct KernelShape {
  int rj, rk;     // lane tile (rows x columns)
  int wpe;        // waves per SIMD the register budget is sized for
  // Plans of panel jobs only: panels per workgroup, 1 (a job is one panel) or
  // kStripPanels (a job is a strip of that many panels of one panel row).
  int group = 1;
  // Exchange between the lanes of a wavefront: 0 through per-wave LDS slot
  // arrays, 1 through ds_bpermute and DPP row shifts.
  int xch = 0;
  // Packed kernels: faces staged straight into LDS by the loads (1) or
  // through registers (0).
  int dma = 0;
};

// Launchers (sweep.hip).
hipError_t launch_init_boundary(const KernelShape& ks, const Boundary& b, hipStream_t s);
// Next run generation, error flag and queue head cleared, and nred
// per-triplet reduction pairs of red reset (red may be null when nred = 0).
hipError_t launch_prepare(int* ctl, int* counter, int* red, uint32_t nred, hipStream_t s);
// modes: bit 0 = whole-triplet jobs present, bit 1 = panel jobs present.
// The kernel variant follows a.sc.kind.
hipError_t launch_sweep(const KernelShape& ks, int modes, const SweepArgs& a, int grid,
                        hipStream_t s);
// plane: the variant that writes last-slice planes (traceback). The figure is
// workgroups per compute unit.
hipError_t sweep_occupancy(const KernelShape& ks, int modes, int kind, bool plane, uint32_t lds_n0,
                           int* waves_per_cu);
// Whether scoring kernels of this tile shape (and lane exchange) exist for
// this alignment kind. Plane kernels exist for 4 x 4 tiles at two waves per
// SIMD: global kind (either lane exchange) and local kind (LDS slot arrays).
bool shape_supported(const KernelShape& ks, int kind);

// Packed pairs (two triplets per lane, 16 bits each; batches of whole
// triplets, any kind). Jobs hold pair p as descriptors 2p and 2p + 1.
// pk_top / pk_left: plain sentinel faces of face_rows(lds_n0) rows filled by
// launch_fill_packed_sentinel; base: the stored value of M' = 0; kc: the
// offset of semi-global candidates (M + kc, kept within [1, 0xFFFF]).
constexpr uint32_t kPackedSentinel = 1024;   // value outside the tensor
constexpr uint32_t kPackedMax = 0x7BFF;      // largest value a lane may hold
hipError_t launch_sweep_pk(const KernelShape& ks, int kind, const SweepArgs& a, const int* pk_top,
                           const int* pk_left, uint32_t base, uint32_t kc, int grid, hipStream_t s);
hipError_t sweep_pk_occupancy(const KernelShape& ks, int kind, uint32_t lds_n0, int* blocks_per_cu);
// Whether a packed kernel of this lane tile, register budget and kind exists.
bool pk_shape_supported(const KernelShape& ks, int kind);
hipError_t launch_fill_packed_sentinel(uint32_t* p, uint64_t n, hipStream_t s);

// Traceback (traceback.hip). A split box: the forward and reversed planes
// (ints from the plane buffer base), rows x cols entries each, reduced in
// nchunk chunks of kSplitChunk cells numbered from chunk0.
constexpr uint32_t kSplitChunk = 16384;
struct SplitDesc {
  uint64_t fwd, bwd;
  uint32_t rows, cols;
  uint32_t chunk0, nchunk;
};
// A leaf box: sequence s of the box is residues lo[s] .. lo[s] + len[s] - 1 of
// the packed sequence at word offset off[s]; (len0+1)(len1+1)(len2+1) <=
// kLeafCells; its columns go to cols + out (3 bytes per column, at most
// len0 + len1 + len2 columns).
struct LeafDesc {
  uint64_t off[3];
  uint32_t lo[3];
  uint32_t len[3];
  uint64_t out;
};
struct LeafArgs {
  const uint32_t* words;
  const LeafDesc* leaves;
  uint32_t n;
  uint8_t* cols;
  uint32_t* ncols;  // per leaf: columns written
  int32_t* score;   // per leaf: the box's global score
  int32_t sub[16];
  int32_t gap;
};
// Boxes of at most this many table cells are solved whole by k_leaf.
constexpr uint64_t kLeafCells = 4096;

// Half-split scoring of a lone triplet. One output sequence of the gather:
// len residues, residue p taken from the packed sequence at word src_off,
// residue start + p (or start + len - 1 - p if reverse), written packed from
// word dst_off. With ctl non-null the same launch also does launch_prepare's
// work for a run without reduction pairs (ctl, counter as there).
struct GatherDesc {
  uint64_t src_off, dst_off;
  uint32_t start, len, reverse;
};
hipError_t launch_gather(const uint32_t* in, const GatherDesc* d, uint32_t n, uint32_t words_out,
                         uint32_t* out, int* ctl, int* counter, hipStream_t s);
// out[0] = the best F + R over box 0 of planes (its nchunks chunks of
// kSplitChunk cells, numbered from 0), or INT32_MIN if err[0] is set (a wait
// of the run gave up). With own non-null (local scoring), the best also
// covers own[0] and own[1], the halves' own bests. partial: nchunks ints of
// scratch; counter: one int that is 0 before the call and is left 0.
hipError_t launch_meet(const SplitDesc* box, uint32_t nchunks, const int* planes, int* partial,
                       const int* err, const int* own, int* counter, int32_t* out, hipStream_t s);
// out[3b] = best F + R of box b, out[3b+1], out[3b+2] = its (p, q).
// chunk_box[c] = the box of chunk c; partial: 2 ints per chunk.
hipError_t launch_split(const int* planes, const SplitDesc* boxes, uint32_t n, const uint32_t* chunk_box,
                        uint32_t nchunks, int* partial, int* out, hipStream_t s);
hipError_t launch_leaf(const LeafArgs& a, hipStream_t s);

inline int panel_rows(const KernelShape& ks) { return kGJ * ks.rj; }
inline int panel_cols(const KernelShape& ks) { return kGK * ks.rk; }
inline uint32_t right_face_row(const KernelShape& ks) { return panel_rows(ks) + 4; }

}  // namespace trioseq

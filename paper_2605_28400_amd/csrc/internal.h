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
// Face buffers carry kFacePre rows before slice 0 and kFacePost after slice
// n0, so the skewed fill/drain steps store into padding instead of testing.
constexpr int kFacePre = 16;
constexpr int kFacePost = 24;
__host__ __device__ inline uint32_t face_rows(uint32_t n0) { return n0 + 1 + kFacePre + kFacePost; }
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
};

// One triplet as the kernels see it: the three sequences already assigned
// to the sweep axis (0), the row axis (1) and the column axis (2).
struct TripletDesc {
  uint64_t off[3];  // word offsets of the three sequences in the word array
  uint32_t len[3];  // lengths on the sweep, row and column axes
  uint32_t out;     // index of this triplet's score in the caller's output
};

// Sentinel faces for edge panels (rows = face_rows of the longest sweep).
struct Boundary {
  int* top_seed;  // rows x panel_cols, with the seed at slice 0, k = 0
  int* top;       // rows x panel_cols
  int* left;      // rows x right_face_row
  uint32_t rows;
};

struct BatchArgs {
  uint32_t lds_n0;          // longest sweep length the dynamic LDS was sized for
  const uint32_t* words;
  const TripletDesc* desc;  // in processing (LPT) order
  int32_t* scores;
  int* counter;             // work queue head, zeroed before each launch
  int* face;                // per-wave workspace
  uint64_t face_stride;     // ints of workspace per wave
  uint32_t n;
  const int* bnd_top_seed;
  const int* bnd_top;
  const int* bnd_left;
  DevScoring sc;
};

struct WideArgs {
  const uint32_t* words;
  TripletDesc desc;
  int32_t* scores;
  int* face;          // per-panel face buffers
  int* progress;      // per-panel completed-step counters + 1 error flag, zeroed before launch
  const uint32_t* order;  // panel ids (pj * PK + pk) in wave-major order
  uint32_t panels_per_wave;
  uint32_t n_panels;
  uint32_t pk_count;
  const int* bnd_top_seed;
  const int* bnd_top;
  const int* bnd_left;
  DevScoring sc;
};

struct KernelShape {
  int rj, rk;  // lane tile (rows x columns)
};

// Launchers (sweep.hip).
hipError_t launch_reset(int* p, int n, hipStream_t s);
hipError_t launch_init_boundary(const KernelShape& ks, const Boundary& b, hipStream_t s);
hipError_t launch_batch(const KernelShape& ks, const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_wide(const KernelShape& ks, const WideArgs& a, int grid, hipStream_t s);
hipError_t batch_occupancy(const KernelShape& ks, uint32_t lds_n0, int* waves_per_cu);
hipError_t wide_occupancy(const KernelShape& ks, uint32_t lds_n0, int* waves_per_cu);
bool shape_supported(const KernelShape& ks);

inline int panel_rows(const KernelShape& ks) { return kGJ * ks.rj; }
inline int panel_cols(const KernelShape& ks) { return kGK * ks.rk; }
inline uint32_t right_face_row(const KernelShape& ks) { return panel_rows(ks) + 4; }

}  // namespace trioseq

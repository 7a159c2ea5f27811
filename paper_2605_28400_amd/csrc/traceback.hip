// gfx950 kernels of the traceback (Hirschberg's linear-space divide and
// conquer, applied to the 3-way recurrence of the paper, Section II, Eq. 1).
//
// A box is a sub-problem: the global alignment of S0[lo0, hi0), S1[lo1, hi1)
// and S2[lo2, hi2). The host halves a box's longest axis at mid; the sweep
// kernels (plane variant) give the last slice of the forward tensor of the
// first half, F[p][q], and of the tensor of the reversed second half,
// R[p'][q'], over the two other axes. Every optimal alignment of the box
// crosses the slice mid at some (p, q) with F[p][q] + R[P-p][Q-q] equal to
// the box's score, so k_split picks such a cell and the box becomes two.
// Boxes of at most kLeafCells cells are solved by k_leaf: the full table of
// the box and a walk back from its far corner.
#include "internal.h"

namespace trioseq {
namespace {

__device__ __forceinline__ uint32_t leaf_residue(const uint32_t* __restrict__ words, uint64_t off,
                                                 uint32_t p) {
  return (words[off + (p >> 4)] >> ((p & 15u) << 1)) & 3u;
}

// One workgroup per box: the best F[p][q] + R[P-p][Q-q] over the plane, ties
// broken towards the smallest p * cols + q (so the choice is deterministic).
__global__ void __launch_bounds__(256) k_split(const int* __restrict__ planes,
                                               const SplitDesc* __restrict__ boxes, uint32_t n,
                                               int* __restrict__ out) {
  __shared__ int s_val[256];
  __shared__ uint32_t s_idx[256];
  const uint32_t b = blockIdx.x;
  if (b >= n) return;
  const SplitDesc d = boxes[b];
  const int* F = planes + d.fwd;
  const int* R = planes + d.bwd;
  const uint32_t cells = d.rows * d.cols;
  int best = INT32_MIN;
  uint32_t bidx = 0xFFFFFFFFu;
  for (uint32_t q = threadIdx.x; q < cells; q += blockDim.x) {
    const uint32_t p = q / d.cols, c = q - p * d.cols;
    const uint32_t rq = (d.rows - 1 - p) * d.cols + (d.cols - 1 - c);
    const int v = F[q] + R[rq];
    if (v > best) {  // q grows, so the first maximum of this thread is kept
      best = v;
      bidx = q;
    }
  }
  s_val[threadIdx.x] = best;
  s_idx[threadIdx.x] = bidx;
  __syncthreads();
  for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const int v2 = s_val[threadIdx.x + w];
      const uint32_t i2 = s_idx[threadIdx.x + w];
      if (v2 > s_val[threadIdx.x] || (v2 == s_val[threadIdx.x] && i2 < s_idx[threadIdx.x])) {
        s_val[threadIdx.x] = v2;
        s_idx[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * b] = s_val[0];
    out[3 * b + 1] = (int)(s_idx[0] / d.cols);
    out[3 * b + 2] = (int)(s_idx[0] % d.cols);
  }
}

// One thread per leaf box: the table of Eq. 1 over the box (global
// initialisation: the box's corner is 0, moves leaving the box do not exist),
// then the walk back from the far corner, taking at every cell the first
// move, in a fixed order, whose predecessor plus column score gives the
// cell's value. Columns are written last first, one byte per sequence
// (0..3 a residue, 4 a gap).
__global__ void __launch_bounds__(64) k_leaf(LeafArgs a) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const LeafDesc d = a.leaves[t];
  const int A = (int)d.len[0], B = (int)d.len[1], C = (int)d.len[2];
  int* T = a.scratch + d.table;
  const int sB = (B + 1) * (C + 1), sC = C + 1;
  const int g2 = 2 * a.gap;
  constexpr int kNone = INT32_MIN / 2;
  for (int i = 0; i <= A; ++i) {
    const int x = i ? (int)leaf_residue(a.words, d.off[0], d.lo[0] + i - 1) : 0;
    for (int j = 0; j <= B; ++j) {
      const int y = j ? (int)leaf_residue(a.words, d.off[1], d.lo[1] + j - 1) : 0;
      for (int k = 0; k <= C; ++k) {
        const int at = i * sB + j * sC + k;
        if (i == 0 && j == 0 && k == 0) {
          T[at] = 0;
          continue;
        }
        const int z = k ? (int)leaf_residue(a.words, d.off[2], d.lo[2] + k - 1) : 0;
        int m = kNone;
        if (i && j && k) m = max(m, T[at - sB - sC - 1] + a.sub[4 * x + y] + a.sub[4 * x + z] + a.sub[4 * y + z]);
        if (i && j) m = max(m, T[at - sB - sC] + a.sub[4 * x + y] + g2);
        if (i && k) m = max(m, T[at - sB - 1] + a.sub[4 * x + z] + g2);
        if (j && k) m = max(m, T[at - sC - 1] + a.sub[4 * y + z] + g2);
        if (i) m = max(m, T[at - sB] + g2);
        if (j) m = max(m, T[at - sC] + g2);
        if (k) m = max(m, T[at - 1] + g2);
        T[at] = m;
      }
    }
  }
  a.score[t] = T[A * sB + B * sC + C];
  uint8_t* out = a.cols + d.out;
  int i = A, j = B, k = C, n = 0;
  while (i || j || k) {
    const int at = i * sB + j * sC + k;
    const int v = T[at];
    const int x = i ? (int)leaf_residue(a.words, d.off[0], d.lo[0] + i - 1) : 0;
    const int y = j ? (int)leaf_residue(a.words, d.off[1], d.lo[1] + j - 1) : 0;
    const int z = k ? (int)leaf_residue(a.words, d.off[2], d.lo[2] + k - 1) : 0;
    int di = 0, dj = 0, dk = 0;
    if (i && j && k && T[at - sB - sC - 1] + a.sub[4 * x + y] + a.sub[4 * x + z] + a.sub[4 * y + z] == v) {
      di = dj = dk = 1;
    } else if (i && j && T[at - sB - sC] + a.sub[4 * x + y] + g2 == v) {
      di = dj = 1;
    } else if (i && k && T[at - sB - 1] + a.sub[4 * x + z] + g2 == v) {
      di = dk = 1;
    } else if (j && k && T[at - sC - 1] + a.sub[4 * y + z] + g2 == v) {
      dj = dk = 1;
    } else if (i && T[at - sB] + g2 == v) {
      di = 1;
    } else if (j && T[at - sC] + g2 == v) {
      dj = 1;
    } else {
      dk = 1;  // the only move left (k > 0 here, or the table is inconsistent)
      if (!k) break;
    }
    out[3 * n] = (uint8_t)(di ? x : 4);
    out[3 * n + 1] = (uint8_t)(dj ? y : 4);
    out[3 * n + 2] = (uint8_t)(dk ? z : 4);
    ++n;
    i -= di;
    j -= dj;
    k -= dk;
  }
  a.ncols[t] = (uint32_t)n;
}

}  // namespace

hipError_t launch_split(const int* planes, const SplitDesc* boxes, uint32_t n, int* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3(n), dim3(256), 0, s, planes, boxes, n, out);
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf, dim3((a.n + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace trioseq

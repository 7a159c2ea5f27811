// gfx950 kernels of the traceback (Hirschberg's linear-space divide and
// conquer, applied to the 3-way recurrence of the paper, Section II, Eq. 1).
//
// A box is a sub-problem: the global alignment of S0[lo0, hi0), S1[lo1, hi1)
// and S2[lo2, hi2). The host halves a box's longest axis at mid; the sweep
// kernels (plane variant) give the last slice of the forward tensor of the
// first half, F[p][q], and of the tensor of the reversed second half,
// R[p'][q'], over the two other axes. Every optimal alignment of the box
// crosses the slice mid at some (p, q) with F[p][q] + R[P-p][Q-q] equal to
// the box's score, so the split kernels pick such a cell and the box becomes
// two. Boxes of at most kLeafCells cells are solved by k_leaf: the full
// table of the box in LDS and a walk back from its far corner.
#include "internal.h"

namespace trioseq {
namespace {

__device__ __forceinline__ uint32_t leaf_residue(const uint32_t* __restrict__ words, uint64_t off,
                                                 uint32_t p) {
  return (words[off + (p >> 4)] >> ((p & 15u) << 1)) & 3u;
}

constexpr int kSplitBatch = 32;

// Split, stage 1: one workgroup per chunk of kSplitChunk cells of one box's
// plane; its best F[p][q] + R[P-p][Q-q] and the smallest linear index
// p * cols + q reaching it.
__global__ void __launch_bounds__(256) k_split_part(const int* __restrict__ planes,
                                                    const SplitDesc* __restrict__ boxes,
                                                    const uint32_t* __restrict__ chunk_box,
                                                    uint32_t nchunks, int* __restrict__ partial) {
  __shared__ int s_val[256];
  __shared__ uint32_t s_idx[256];
  const uint32_t ch = blockIdx.x;
  if (ch >= nchunks) return;
  const SplitDesc d = boxes[chunk_box[ch]];
  const int* F = planes + d.fwd;
  const int* R = planes + d.bwd;
  const uint32_t cells = d.rows * d.cols;
  const uint32_t lo = (ch - d.chunk0) * kSplitChunk;
  const uint32_t hi = min(cells, lo + kSplitChunk);
  int best = INT32_MIN;
  uint32_t bidx = 0xFFFFFFFFu;
  // kSplitBatch cells per thread per pass, their loads issued together: one
  // workgroup covers a whole chunk, so a pass at a time would wait out a full
  // memory latency per cell.
  for (uint32_t q0 = lo + threadIdx.x; q0 < hi; q0 += kSplitBatch * blockDim.x) {
    int v[kSplitBatch];
#pragma unroll
    for (int u = 0; u < kSplitBatch; ++u) {
      // Cells past the chunk load its last cell (no branch between the
      // loads) and are then discarded.
      const uint32_t q = q0 + u * blockDim.x, qc = min(q, hi - 1);
      const uint32_t p = qc / d.cols, c = qc - p * d.cols;
      const int s = F[qc] + R[(d.rows - 1 - p) * d.cols + (d.cols - 1 - c)];
      v[u] = q < hi ? s : INT32_MIN;
    }
#pragma unroll
    for (int u = 0; u < kSplitBatch; ++u) {
      if (v[u] > best) {  // q grows with u, so the first maximum of this thread is kept
        best = v[u];
        bidx = q0 + u * blockDim.x;
      }
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
    partial[2 * ch] = s_val[0];
    partial[2 * ch + 1] = (int)s_idx[0];
  }
}

// Split, stage 2: one wave per box folds its chunks' results (same order:
// larger value, then smaller index) into out[3b] = best, (p, q).
__global__ void __launch_bounds__(64) k_split_final(const SplitDesc* __restrict__ boxes, uint32_t n,
                                                    const int* __restrict__ partial,
                                                    int* __restrict__ out) {
  const uint32_t b = blockIdx.x;
  if (b >= n) return;
  const SplitDesc d = boxes[b];
  int best = INT32_MIN;
  uint32_t bidx = 0xFFFFFFFFu;
  for (uint32_t c = threadIdx.x; c < d.nchunk; c += 64) {
    const int v = partial[2 * (d.chunk0 + c)];
    const uint32_t i = (uint32_t)partial[2 * (d.chunk0 + c) + 1];
    if (v > best || (v == best && i < bidx)) {
      best = v;
      bidx = i;
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    const int v2 = __shfl_xor(best, m, 64);
    const uint32_t i2 = (uint32_t)__shfl_xor((int)bidx, m, 64);
    if (v2 > best || (v2 == best && i2 < bidx)) {
      best = v2;
      bidx = i2;
    }
  }
  if (threadIdx.x == 0) {
    out[3 * b] = best;
    out[3 * b + 1] = (int)(bidx / d.cols);
    out[3 * b + 2] = (int)(bidx % d.cols);
  }
}

// One wave per leaf box: the table of Eq. 1 over the box (global
// initialisation: the box's corner is 0, moves leaving the box do not exist)
// in LDS, filled one anti-diagonal plane i + j + k = const at a time (every
// predecessor lies on one of the three previous planes), then lane 0 walks
// back from the far corner, taking at every cell the first move, in a fixed
// order, whose predecessor plus column score gives the cell's value. Columns
// are written last first, one byte per sequence (0..3 a residue, 4 a gap).
__global__ void __launch_bounds__(64) k_leaf(LeafArgs a) {
  __shared__ int T[kLeafCells];
  __shared__ uint8_t res[3][kLeafCells];
  const uint32_t leaf = blockIdx.x;
  if (leaf >= a.n) return;
  const LeafDesc d = a.leaves[leaf];
  const int A = (int)d.len[0], B = (int)d.len[1], C = (int)d.len[2];
  const int lane = threadIdx.x;
  for (int s = 0; s < 3; ++s)
    for (int q = lane; q < (int)d.len[s]; q += 64) res[s][q] = (uint8_t)leaf_residue(a.words, d.off[s], d.lo[s] + q);
  __syncthreads();
  const int sB = (B + 1) * (C + 1), sC = C + 1;
  const int g2 = 2 * a.gap;
  constexpr int kNone = INT32_MIN / 2;
  const int pairs = (A + 1) * (B + 1);
  for (int dd = 0; dd <= A + B + C; ++dd) {
    for (int q = lane; q < pairs; q += 64) {
      const int i = q / (B + 1), j = q - i * (B + 1), k = dd - i - j;
      if (k < 0 || k > C) continue;
      const int at = i * sB + j * sC + k;
      if (dd == 0) {
        T[0] = 0;
        continue;
      }
      const int x = i ? res[0][i - 1] : 0, y = j ? res[1][j - 1] : 0, z = k ? res[2][k - 1] : 0;
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
    __syncthreads();
  }
  if (lane != 0) return;
  a.score[leaf] = T[A * sB + B * sC + C];
  uint8_t* out = a.cols + d.out;
  int i = A, j = B, k = C, n = 0;
  while (i || j || k) {
    const int at = i * sB + j * sC + k;
    const int v = T[at];
    const int x = i ? res[0][i - 1] : 0, y = j ? res[1][j - 1] : 0, z = k ? res[2][k - 1] : 0;
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
  a.ncols[leaf] = (uint32_t)n;
}

// Gather: one thread per output word packs 16 residues of one output
// sequence (forward or reversed) from the caller's packed sequences.
__global__ void __launch_bounds__(256) k_gather(const uint32_t* __restrict__ in,
                                                const GatherDesc* __restrict__ d, uint32_t n,
                                                uint32_t words_out, uint32_t* __restrict__ out,
                                                int* __restrict__ ctl, int* __restrict__ counter) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  // With ctl given, also the per-run preparation of the sweep that follows
  // (next generation, error flag cleared, queue head zeroed), saving its
  // launch: nothing here reads these words.
  if (ctl && w == 0) {
    ctl[0] = ctl[0] + 1;
    ctl[1] = 0;
    counter[0] = 0;
  }
  if (w >= words_out) return;
  // The output sequence holding word w (sequences start on fresh words).
  uint32_t q = 0;
  while (q + 1 < n && d[q + 1].dst_off <= w) ++q;
  const GatherDesc g = d[q];
  const uint32_t first = (uint32_t)(w - g.dst_off) * 16;
  uint32_t v = 0;
  for (uint32_t b = 0; b < 16; ++b) {
    const uint32_t p = first + b;
    if (p >= g.len) break;
    const uint32_t src = g.reverse ? g.start + g.len - 1 - p : g.start + p;
    v |= leaf_residue(in, g.src_off, src) << (2 * b);
  }
  out[w] = v;
}

// Meet, in one launch: workgroup c reduces chunk c of box 0 (kSplitChunk
// plane cells) to its best F + R; the workgroup that finishes last folds the
// chunks' bests, and the halves' own bests when given, into the score
// (INT32_MIN if a wait of the run gave up) and clears the counter for the
// next run.
__global__ void __launch_bounds__(256) k_meet(const int* __restrict__ planes, const SplitDesc* __restrict__ box,
                                              uint32_t nchunks, int* partial, const int* __restrict__ err,
                                              const int* __restrict__ own, int* counter, int32_t* out) {
  __shared__ int s_val[256];
  __shared__ int s_last;
  const SplitDesc d = box[0];
  const int* F = planes + d.fwd;
  const int* R = planes + d.bwd;
  const uint32_t cells = d.rows * d.cols;
  const uint32_t lo = blockIdx.x * kSplitChunk;
  const uint32_t hi = min(cells, lo + kSplitChunk);
  int best = INT32_MIN;
  // kSplitBatch cells per thread per pass, their loads issued together.
  for (uint32_t q0 = lo + threadIdx.x; q0 < hi; q0 += kSplitBatch * blockDim.x) {
    int v[kSplitBatch];
#pragma unroll
    for (int u = 0; u < kSplitBatch; ++u) {
      const uint32_t q = q0 + u * blockDim.x, qc = min(q, hi - 1);
      const uint32_t p = qc / d.cols, c = qc - p * d.cols;
      const int sv = F[qc] + R[(d.rows - 1 - p) * d.cols + (d.cols - 1 - c)];
      v[u] = q < hi ? sv : INT32_MIN;
    }
#pragma unroll
    for (int u = 0; u < kSplitBatch; ++u) best = max(best, v[u]);
  }
  s_val[threadIdx.x] = best;
  __syncthreads();
  for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_val[threadIdx.x] = max(s_val[threadIdx.x], s_val[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partial[blockIdx.x], s_val[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int done = __hip_atomic_fetch_add(counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = done == (int)nchunks - 1;
  }
  __syncthreads();
  if (!s_last) return;
  int b = (own && threadIdx.x < 2) ? own[threadIdx.x] : INT32_MIN;
  for (uint32_t c = threadIdx.x; c < nchunks; c += blockDim.x)
    b = max(b, __hip_atomic_load(&partial[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  __syncthreads();
  s_val[threadIdx.x] = b;
  __syncthreads();
  for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_val[threadIdx.x] = max(s_val[threadIdx.x], s_val[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __hip_atomic_store(out, bad ? INT32_MIN : s_val[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

hipError_t launch_gather(const uint32_t* in, const GatherDesc* d, uint32_t n, uint32_t words_out,
                         uint32_t* out, int* ctl, int* counter, hipStream_t s) {
  if (words_out == 0 && !ctl) return hipSuccess;
  const uint32_t blocks = words_out == 0 ? 1 : (words_out + 255) / 256;
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, in, d, n, words_out, out, ctl, counter);
  return hipGetLastError();
}

hipError_t launch_meet(const SplitDesc* box, uint32_t nchunks, const int* planes, int* partial,
                       const int* err, const int* own, int* counter, int32_t* out, hipStream_t s) {
  if (nchunks == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_meet, dim3(nchunks), dim3(256), 0, s, planes, box, nchunks, partial, err, own, counter,
                     out);
  return hipGetLastError();
}

hipError_t launch_split(const int* planes, const SplitDesc* boxes, uint32_t n, const uint32_t* chunk_box,
                        uint32_t nchunks, int* partial, int* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_part, dim3(nchunks), dim3(256), 0, s, planes, boxes, chunk_box, nchunks,
                     partial);
  hipLaunchKernelGGL(k_split_final, dim3(n), dim3(64), 0, s, boxes, n, partial, out);
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf, dim3(a.n), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace trioseq

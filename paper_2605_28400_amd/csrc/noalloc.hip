// The allocation-free entry point: trioseq_score_batch_packed with every
// device buffer carved from one fixed scratch array instead of allocated.
//
// The array is a file-scope device variable, so each GPU the library runs on
// holds its own copy (zero-initialised when the code object is loaded) until
// the process ends. Host code never uses the array's name as an address: on
// a device's first call, with that device current, its address is read once
// with hipGetSymbolAddress and kept per device, and only that pointer is
// handed to kernels and copies.
//
// Layout of the array: [control 4 KiB | panel-face pool | plain data].
//  * control: the run generation and error flag (ctl[0], ctl[1]), the
//    half-split meeting counter (ctl[2], 0 between calls) and the job queue
//    head; they persist from call to call and the generation only grows, so
//    a face tag written by an earlier call never looks current;
//  * pool: only ever (value, tag) pairs of split triplets' faces, at even
//    offsets from this fixed base (or the zeros it started with), so a tag
//    slot never holds a plain value;
//  * plain: job and triplet tables, sentinel faces, reduction pairs,
//    half-split buffers and the whole-triplet workspace, carved anew by every
//    call (a call launches no more waves than the rest of this part holds
//    workspaces for).
// Every call on one GPU shares that GPU's array: calls that overlap in time
// on one GPU race (their tables and workspaces collide).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace trioseq {

constexpr uint64_t kControlBytes = 4096;
constexpr uint64_t kPoolBytes = 96ull << 20;
constexpr uint64_t kScratchBytes = 256ull << 20;
static_assert(kControlBytes + kPoolBytes < kScratchBytes, "scratch layout");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

// The device address of this device's copy of the array (read once per
// device, with that device current).
trioseq_status scratch_for(int device, uint8_t** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(TRIOSEQ_ERR_DEVICE, "score_batch_packed_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "score_batch_packed_noalloc: hipGetSymbolAddress");
    if (!p) return fail(TRIOSEQ_ERR_DEVICE, "score_batch_packed_noalloc: scratch has no address");
    g_ptr[device] = (uint8_t*)p;
  }
  *out = g_ptr[device];
  return TRIOSEQ_OK;
}

}  // namespace
}  // namespace trioseq

using namespace trioseq;

extern "C" {

trioseq_status trioseq_score_batch_packed_noalloc(const uint32_t* d_words, const uint64_t* d_word_off,
                                                  const uint32_t* d_len, size_t n,
                                                  const trioseq_scoring* sc, int32_t* d_scores,
                                                  void* hip_stream) {
  return guarded([&]() -> trioseq_status {
    int device = 0;
    TRIOSEQ_HIP(hipGetDevice(&device), "hipGetDevice");
    uint8_t* base = nullptr;
    const trioseq_status st = scratch_for(device, &base);
    if (st != TRIOSEQ_OK) return st;
    PlanMemory mem;
    mem.ctl = (int*)base;
    mem.counter = (int*)(base + 256);
    mem.pool = (int*)(base + kControlBytes);
    mem.pool_bytes = kPoolBytes;
    mem.plain = base + kControlBytes + kPoolBytes;
    mem.plain_bytes = kScratchBytes - kControlBytes - kPoolBytes;
    mem.stream = (hipStream_t)hip_stream;
    return score_packed_in_region(d_words, d_word_off, d_len, n, sc, d_scores, mem);
  });
}

uint64_t trioseq_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"

// Host-side helpers shared by the plan and server implementations.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/trioseq.h"
#include "internal.h"

namespace trioseq {

trioseq_status fail(trioseq_status st, const std::string& msg);
trioseq_status fail_hip(hipError_t e, const char* what);
#define TRIOSEQ_HIP(call, what)                              \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return ::trioseq::fail_hip(e_, what); \
  } while (0)

// Residue code of an ASCII character, or 255.
extern const uint8_t kCode[256];

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

struct DeviceProps {
  int device;
  int cus;
  size_t hbm_bytes;
};
trioseq_status device_props(DeviceProps* p);

uint64_t now_ns();

}  // namespace trioseq

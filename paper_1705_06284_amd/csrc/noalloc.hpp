// noalloc.hpp -- static device scratch of the allocation-free entry point
// (internal to libbispec; noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace bispec {

// Bytes of the static scratch on every device (64 MiB: the workspace of a
// 64^3 plan of a few bins and batch 1 or 2, or of any 32^3 plan).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxDevices = 64;

// Device address of the scratch on `device`, which must be the current
// device; looked up once per device and kept.
hipError_t scratch_address(int device, void **addr);

// Record `owner` (a plan id) as the last user of the device's scratch;
// true when it already was (the plan's tables are still in place).
bool scratch_claim(int device, unsigned long long owner);
// Forget the last user (its tables may be partly overwritten).
void scratch_release(int device);

}  // namespace bispec

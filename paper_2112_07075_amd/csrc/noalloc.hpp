// Static device scratch of the allocation-free entry points (noalloc.hip).
#pragma once

namespace fepa {

// 32 MiB of FP64 per GPU: the shared-node partials of one launch unit
// (three values per entry) must fit.
constexpr long long kStaticScratchDoubles = 4LL << 20;
constexpr long long kStaticScratchBytes = kStaticScratchDoubles * 8;
constexpr int kStaticScratchDevices = 64;

// With `device` current: look the array's device address up once for that
// device (hipGetSymbolAddress) and keep it. 0 on success, -1 on failure.
int static_scratch_init(int device);
// The kept device address for `device`, or nullptr if init did not succeed.
double *static_scratch(int device);

}  // namespace fepa

// Static device scratch of lead_decode_noalloc (one array per device, held
// until the process ends).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/lead.h"

namespace lead {

constexpr size_t kScratchBytes = LEAD_NOALLOC_SCRATCH_BYTES;

// Device address of the scratch array on `device`, which must be the current
// device.  The address is looked up once per device (hipGetSymbolAddress) and
// kept; no memory is allocated.
hipError_t scratch_address(int device, void **out);

}  // namespace lead

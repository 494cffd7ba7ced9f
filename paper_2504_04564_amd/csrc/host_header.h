// Host-side header parsing shared by the API and the launchers.
#pragma once
#include "common.h"
#include "format.h"

namespace vdbc {
// Parses and checks the 256-byte header of a buffer of `bytes` bytes
// (canonical section layout, dims, root table shape).
vdbc_status parse_header(const void* header, uint64_t bytes, Header* out);
}  // namespace vdbc

// Host-side helpers shared by the C-ABI sources (no device code).
#pragma once

#include <string>

#include "cq.h"

namespace cq {

// Record msg as the calling thread's cq_last_error() and return s.
cq_status host_fail(cq_status s, const std::string& msg);

}  // namespace cq

// Host-side declarations shared by the solver's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "rgb_device.hpp"

namespace rgb {

hipError_t launch_plain(const Problem& P, hipStream_t stream);
hipError_t launch_group(const Problem& P, int lanes_per_lp, hipStream_t stream);
bool group_supported(int lanes_per_lp);

}  // namespace rgb

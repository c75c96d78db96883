// Host-side declarations shared by the solver's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "rgb_device.hpp"

// (lanes per LP, register slots per lane) pairs compiled for the group kernel.
#define RGB_GROUP_SHAPES(X) \
    X(8, 4)                 \
    X(8, 9)                 \
    X(16, 5)                \
    X(16, 9)                \
    X(16, 17)               \
    X(32, 5)                \
    X(32, 9)                \
    X(64, 2)                \
    X(64, 5)                \
    X(64, 9)                \
    X(64, 17)

namespace rgb {

hipError_t launch_plain(const Problem& P, hipStream_t stream);
hipError_t launch_group(const Problem& P, int lanes_per_lp, int slots, hipStream_t stream);
bool group_supported(int lanes_per_lp, int slots);

}  // namespace rgb

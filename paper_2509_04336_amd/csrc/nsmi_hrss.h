// Hit-and-run slice-sampling inner kernel (see nsmi_hrss.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "nsmi_kernels.h"

namespace nsmi {

// Philox purposes of the slice steps (the acceptance walk uses 0-7): one
// block per step (stepping-out split V, donors a and b, interval offset r),
// and one block per shrinkage draw k at purpose HRSS_P_SHRINK + k.
constexpr uint64_t HRSS_P_STEP = 8, HRSS_P_SHRINK = 64;
constexpr int HRSS_M = 8;   // stepping-out budget in interval widths
constexpr int HRSS_K = 64;  // shrinkage draws before a step gives up

// One workgroup of two waves per chain, W slice steps (W = the event's walk
// length); enqueued on s.
hipError_t launch_hrss(const StepArgs &a, int max_det, int mixed, hipStream_t s);

}  // namespace nsmi

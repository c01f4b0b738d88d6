// Launchers of the SSIM quality measure (kernels_metrics.hip).
#pragma once
#include "launch.h"

namespace dbl {

// SSIM tile sums for window radius R (0 .. 16), then the mean per job;
// ssim_lds(R) is the tile kernel's dynamic LDS in bytes.
hipError_t launch_ssim(const LaunchArgs& la, int precision, int R);
hipError_t launch_ssim_fin(const LaunchArgs& la);
size_t ssim_lds(int R);

}  // namespace dbl

// Launchers of the reduction kernels (all asynchronous on `st`).
#pragma once
#include <hip/hip_runtime.h>

#include "hpop_internal.h"

namespace hpop {

constexpr int kScanTile = 4096;  // bucket counts per workgroup of the offset scan
constexpr int kHistWin = 512;    // LDS bucket window of one streaming tile
constexpr int kWaveCap = 512;    // records one wave sorts and flattens on its own
constexpr int kWaveBins = 512;   // sub-bins of the wave path's counting sort (at most)

hipError_t launch_reset(const Plan& p, hipStream_t st);
hipError_t launch_stats(const Plan& p, hipStream_t st);
hipError_t launch_hist(const Plan& p, hipStream_t st);
hipError_t launch_scan(const Plan& p, hipStream_t st);
hipError_t launch_scatter(const Plan& p, hipStream_t st);
hipError_t launch_carry(const Plan& p, hipStream_t st);
hipError_t launch_scan_carry(const Plan& p, hipStream_t st);  // fixed slots: scan and carry in one launch
hipError_t launch_merge_wave(const Plan& p, hipStream_t st);
hipError_t launch_merge_block(const Plan& p, int cap, hipStream_t st);
hipError_t launch_base(const Plan& p, hipStream_t st);
hipError_t launch_region(const Plan& p, const RegionDesc* regions, int n_regions, int max_res, Tree* trees,
                         long long* times, const IvlDesc* ivls, long long n_ivls, long long* macc, hipStream_t st);

}  // namespace hpop

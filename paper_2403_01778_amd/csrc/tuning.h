// Tile table of the TTVc sweep: the tiling of the level-1 pass (the one that
// streams T) per storage format and shape, either registered by the
// autotuner or chosen by the built-in rule.
#pragma once

#include "common.h"
#include "ttvc.h"

namespace hoscf {

// tiling[6] = {workgroups, smallest p-range, lanes per row, aligned q-chunks,
// rows per lane group, waves per workgroup}, as in hoscf_profile_sweep
SweepTuning tuning_from(const int64_t* tiling);
SweepTuning lookup_tuning(const hoscf_tensor& T);

}  // namespace hoscf

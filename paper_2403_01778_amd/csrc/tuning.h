// Tile table of the TTVc sweep: tiling parameters per storage format and
// shape class, read from the table the autotuner writes.
#pragma once

#include "common.h"
#include "ttvc.h"

namespace hoscf {

SweepTuning lookup_tuning(const hoscf_tensor& T);

}  // namespace hoscf

extern "C" size_t hoscf_extra_workspace_size(int op, const hoscf_tensor* T);

// Tile table lookup for the TTVc sweep.
#include "tuning.h"

namespace hoscf {

SweepTuning lookup_tuning(const hoscf_tensor& T) {
    SweepTuning t;
    (void)T;
    return t;
}

}  // namespace hoscf

// Dense write of a sum of rank-one tensors built from the factors, used by
// the backward passes:
//   out = c0 * x_1 o ... o x_N + cv * sum_n x_1 o .. o v_n o .. o x_N
#pragma once

#include "common.h"

namespace hoscf {

struct OuterArgs {
    void* out;         // dense, C order, dims below
    int N;
    int64_t dims[kMaxOrder];
    int64_t xoff[kMaxOrder + 1];
    const double* x;   // [D] factors (block n at xoff[n])
    const double* v;   // [D] the vectors that replace one factor at a time
    double c0, cv;
    int64_t rows;      // product of all dims but the last
    int64_t nchunk;    // column chunks of the last mode (64 lanes x VEC each)
    int64_t groups;    // row groups (waves per column chunk)
};

// out_dtype: HOSCF_F32 or HOSCF_F64.
int outer_write(int out_dtype, const OuterArgs& a, hipStream_t s);

}  // namespace hoscf

// Dense write of c0 * x_1 o ... o x_N + cv * sum_n x_1 o .. o v_n o .. o x_N.
//
// A tensor "row" fixes every index but the last.  Along a row the value is
// a_r x_N + b_r v_N with two scalars per row,
//   a_r = c0 p_r + cv sum_{n<N} v_n[i_n] prod_{k<N, k != n} x_k[i_k],
//   b_r = cv p_r,   p_r = prod_{k<N} x_k[i_k],
// so a wave keeps its slice of x_N and v_N in registers and walks a range of
// rows, writing 16 bytes per lane per row: the kernel is bound by the HBM
// write of the output.  Row scalars are computed in FP64 from uniform
// (scalar) loads.
#include <algorithm>

#include "common.h"
#include "outer.h"

namespace hoscf {

using CD = const __attribute__((address_space(4))) double;

template <typename O> struct OVec;
template <> struct OVec<float> {
    static constexpr int VEC = 4;
    typedef float T __attribute__((ext_vector_type(4)));
};
template <> struct OVec<double> {
    static constexpr int VEC = 2;
    typedef double T __attribute__((ext_vector_type(2)));
};

template <typename O, int VEC>
__global__ __launch_bounds__(256) void outer_kernel(OuterArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (gw >= a.nchunk * a.groups) return;
    const int64_t chunk = gw % a.nchunk, grp = gw / a.nchunk;
    const int N = a.N;
    const int64_t I = a.dims[N - 1];
    const int64_t q0 = (chunk * 64 + lane) * VEC;
    const bool qok = q0 < I;
    CD* x = reinterpret_cast<CD*>(reinterpret_cast<uintptr_t>(a.x));
    CD* v = reinterpret_cast<CD*>(reinterpret_cast<uintptr_t>(a.v));
    const double* xl = a.x + a.xoff[N - 1];
    const double* vl = a.v + a.xoff[N - 1];
    double xq[VEC], vq[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int64_t q = qok ? q0 + e : 0;
        xq[e] = xl[q];
        vq[e] = vl[q];
    }
    const int64_t r0 = a.rows * grp / a.groups, r1 = a.rows * (grp + 1) / a.groups;
    if (r0 >= r1) return;
    O* out = static_cast<O*>(a.out);
    for (int64_t r = r0; r < r1; ++r) {
        // indices of the row, last of the first N-1 modes first (the sum and
        // product below do not depend on the order the modes are taken in)
        double p = 1.0, s = 0.0;
        int64_t t = r;
        for (int k = N - 2; k >= 0; --k) {
            const int64_t i = t % a.dims[k];
            t /= a.dims[k];
            const double xk = x[a.xoff[k] + i];
            // s x_k + p v_k extends the sum by mode k; p x_k extends the product
            s = fma(s, xk, p * v[a.xoff[k] + i]);
            p *= xk;
        }
        const double ar = fma(a.c0, p, a.cv * s), br = a.cv * p;
        if (qok) {
            O* dst = out + r * I + q0;
            if constexpr (VEC > 1) {
                typename OVec<O>::T o;
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = (O)fma(ar, xq[e], br * vq[e]);
                __builtin_nontemporal_store(o, reinterpret_cast<typename OVec<O>::T*>(dst));
            } else {
                __builtin_nontemporal_store((O)fma(ar, xq[0], br * vq[0]), dst);
            }
        }
    }
}

int outer_write(int out_dtype, const OuterArgs& a0, hipStream_t s) {
    OuterArgs a = a0;
    const int64_t I = a.dims[a.N - 1];
    const bool f64 = out_dtype == HOSCF_F64;
    const int V = f64 ? OVec<double>::VEC : OVec<float>::VEC;
    const bool vec = (I % V) == 0;
    const int64_t per = 64 * (vec ? V : 1);
    a.nchunk = (I + per - 1) / per;
    // about 16k waves in all (enough to cover the chip several times), each
    // walking at least a few rows
    const int64_t want = std::max<int64_t>(1, (int64_t)16384 / a.nchunk);
    a.groups = std::max<int64_t>(1, std::min<int64_t>(a.rows, want));
    const int64_t waves = a.nchunk * a.groups;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (f64) {
        if (vec) hipLaunchKernelGGL((outer_kernel<double, 2>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((outer_kernel<double, 1>), dim3(grid), dim3(256), 0, s, a);
    } else {
        if (vec) hipLaunchKernelGGL((outer_kernel<float, 4>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((outer_kernel<float, 1>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? HOSCF_OK : HOSCF_HIP_ERROR;
}

}  // namespace hoscf

// fused_deeper.hip -- draw-free passes of 9..13 MCS at X = 2^16 (512 words
// per row, one 512-thread workgroup per band; mcs_fixed_kernel in fused.hpp).
#include "fused.hpp"

namespace sca {
namespace {

// DIST: rows loaded ahead; 12- and 13-MCS passes keep one, which leaves their
// 26- and 28-row windows in 225 and 242 VGPRs without spills (with three
// ahead the 12-MCS pass runs 3 % slower).
template <int K, int DIST>
hipError_t launch_fixed512(const SweepArgs& a, bool has_q, const uint64_t* src, uint64_t* dst, int32_t band,
                           hipStream_t stream)
{
    if (a.W != 512) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(a.Y / band)), block(512);
    // the p = 1 form needs every p-draw accepted; p = 0 goes through the general masks
    if (has_q || a.all_p == 0)
        hipLaunchKernelGGL((mcs_fixed_kernel<8, K, DIST, true>), grid, block, 0, stream, a, src, dst, band);
    else
        hipLaunchKernelGGL((mcs_fixed_kernel<8, K, DIST, false>), grid, block, 0, stream, a, src, dst, band);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mcs_fused_deeper(const SweepArgs& a, bool has_q, const uint64_t* src, uint64_t* dst, int32_t band,
                                   int32_t depth, hipStream_t stream)
{
    switch (depth) {
    case 9: return launch_fixed512<9, 3>(a, has_q, src, dst, band, stream);
    case 10: return launch_fixed512<10, 3>(a, has_q, src, dst, band, stream);
    case 11: return launch_fixed512<11, 3>(a, has_q, src, dst, band, stream);
    case 12: return launch_fixed512<12, 1>(a, has_q, src, dst, band, stream);
    case 13: return launch_fixed512<13, 1>(a, has_q, src, dst, band, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sca

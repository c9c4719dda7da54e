// fused_deep.hip -- the temporally blocked passes of 5..8 MCS (draw-free
// probabilities only; kernel in fused.hpp), in a translation unit of their own
// so that they compile in parallel with the shallower ones.
#include "fused.hpp"

namespace sca {

hipError_t launch_mcs_fused_deep(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                                 int32_t band, int32_t depth, hipStream_t stream)
{
    switch (depth) {
    case 5: return launch_depth<5>(a, mode, has_q, src, dst, band, stream);
    case 6: return launch_depth<6>(a, mode, has_q, src, dst, band, stream);
    case 7: return launch_depth<7>(a, mode, has_q, src, dst, band, stream);
    case 8: return launch_depth<8>(a, mode, has_q, src, dst, band, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sca

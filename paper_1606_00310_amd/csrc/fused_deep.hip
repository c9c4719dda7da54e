// fused_deep.hip -- the temporally blocked passes of 5..8 MCS (draw-free
// probabilities only; kernels in fused.hpp), in a translation unit of their
// own so that they compile in parallel with the shallower ones; 9..13 MCS are
// passed on to fused_deeper.hip.
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
    case 9:
    case 10:
    case 11:
    case 12:
    case 13:
        if (mode != XiMode::Mask || a.ndraw != 0) return hipErrorInvalidValue;
        return launch_mcs_fused_deeper(a, has_q, src, dst, band, depth, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sca

// fused.hip -- dispatch of the temporally blocked passes (kernels in fused.hpp);
// passes of 1..4 MCS are instantiated here, 5..8 in fused_deep.hip and 9..12
// (X = 2^16) in fused_deeper.hip.
#include "fused.hpp"

namespace sca {

int max_fused_depth(int32_t W, XiMode mode, int32_t ndraw)
{
    if (mode == XiMode::PerSite) return kMaxDepthPerSite;
    if (mode != XiMode::Mask) return 0;
    if (ndraw > 0) return kMaxDepthMask;
    if (W == 512) return kMaxDepthFixed512;
    if (W != 1024) return kMaxDepthFixed;
    // 6-MCS passes at X = 2^17 run the LDS-window kernel with 1024-thread
    // workgroups, whose three row buffers need 96 KiB of LDS
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return kMaxDepthWide;
    }
    return lds >= kWideLdsBytes ? kLdsDepth : kMaxDepthWide;
}

bool fused_supported(int32_t W, int64_t Y, int32_t band, int32_t depth, XiMode mode, int32_t ndraw)
{
    return (W == 64 || W == 128 || W == 256 || W == 512 || W == 1024) && depth >= 1 &&
           depth <= max_fused_depth(W, mode, ndraw) && band >= 4 && (band & (band - 1)) == 0 && (Y % band) == 0 &&
           Y >= 2 * band && band >= 2 * depth;
}

hipError_t launch_mcs_fused(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                            int32_t band, int32_t depth, hipStream_t stream)
{
    if (!fused_supported(a.W, a.Y, band, depth, mode, a.ndraw)) return hipErrorInvalidValue;
    switch (depth) {
    case 1: return launch_depth<1>(a, mode, has_q, src, dst, band, stream);
    case 2: return launch_depth<2>(a, mode, has_q, src, dst, band, stream);
    case 3: return launch_depth<3>(a, mode, has_q, src, dst, band, stream);
    case 4: return launch_depth<4>(a, mode, has_q, src, dst, band, stream);
    default: return launch_mcs_fused_deep(a, mode, has_q, src, dst, band, depth, stream);
    }
}

}  // namespace sca

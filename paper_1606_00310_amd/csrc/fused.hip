// fused.hip -- dispatch of the temporally blocked passes (kernels in fused.hpp);
// passes of 1..4 MCS are instantiated here, 5..8 in fused_deep.hip and 9..12
// (X = 2^16) in fused_deeper.hip.
#include <cstdio>

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

// The same choices as launch_depth, launch_block (fused.hpp) and
// launch_fixed512 (fused_deeper.hip), spelled out as the kernel's name.
void fused_kernel_name(const SweepArgs& a, XiMode mode, bool has_q, int32_t depth, char* out, size_t n)
{
    const char* q = has_q ? "true" : "false";
    // the draw-free register-window kernels take the general masks unless p = 1, q = 0
    const char* gq = (has_q || a.all_p == 0) ? "true" : "false";
    const bool draw_free = mode == XiMode::Mask && a.ndraw == 0;
    const char* m = mode == XiMode::PerSite ? "PerSite" : (draw_free ? "Fixed" : "Mask");
    if (depth < 1) {
        std::snprintf(out, n, "none");
        return;
    }
    // mask passes: what the instantiation knows of the number of draws (an
    // odd one carries the shared last draw between a row's half-steps, except
    // with removals at two words per lane)
    const bool rnd = mode == XiMode::Mask && !draw_free;
    const char* odd = !rnd ? "" : ((a.ndraw & 1) == 0 ? ",Even" : ((has_q && a.W == 1024) ? ",Any" : ",OddTail"));
    if (a.W == 1024) {
        if (depth == kLdsDepth && draw_free) std::snprintf(out, n, "mcs_block_lds_kernel<16,%d,%s>", depth, q);
        else std::snprintf(out, n, "mcs_block_kernel<8,2,%d,%s,%s%s>", depth, m, q, odd);
        return;
    }
    const int nw = a.W / 64;
    if (draw_free && depth >= kFixedDeepDepth)
        std::snprintf(out, n, "mcs_fixed_kernel<%d,%d,%d,%s>", nw, depth, (depth >= 12 ? 1 : 3), gq);
    else if (draw_free && depth >= kLdsDepth)
        std::snprintf(out, n, "mcs_block_lds_kernel<%d,%d,%s>", nw, depth, q);
    else
        std::snprintf(out, n, "mcs_block_kernel<%d,1,%d,%s,%s%s>", nw, depth, m, q, odd);
}

}  // namespace sca

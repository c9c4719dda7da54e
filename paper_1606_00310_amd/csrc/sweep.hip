// sweep.hip -- the single-lattice half-step launch on gfx950.
//
// One wavefront owns whole rows: a row of W words is spread over a group of
// G = min(W, 64) lanes holding I = W/G words each (word w = i*G + lane), so
// each load instruction of the wave moves 512 contiguous bytes and every byte
// of the state is read once and written once per half-step.  Because a row
// never leaves its wave there are no barriers, no LDS buffers and no atomics
// (the paper needs a block-wide shared buffer and synchronisation for the
// same rotation, Fig. 3), and the periodic wrap of the row (the paper caches
// the first word separately, Sec. II-B) is a rotation of packed bits inside
// the wave.  The arithmetic of a row group lives in halfstep.hpp.
#include <cstdio>

#include "halfstep.hpp"
#include "sca_internal.hpp"

namespace sca {
namespace {

constexpr int kBlock = 256;

template <int G, int I, XiMode MODE, bool HASQ>
__global__ __launch_bounds__(kBlock) void halfstep_kernel(SweepArgs a)
{
    constexpr int kRowsPerWave = 64 / G;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    halfstep_rows<G, I, MODE, HASQ>(a, a.S, wave * kRowsPerWave + lane / G, lane);
}

template <int G, int I>
hipError_t launch_layout(const SweepArgs& a, XiMode mode, bool has_q, hipStream_t stream)
{
    constexpr int kRowsPerBlock = (kBlock / 64) * (64 / G);
    const dim3 grid((unsigned)((a.Y + kRowsPerBlock - 1) / kRowsPerBlock));
    const dim3 block(kBlock);
    switch (mode) {
    case XiMode::Mask:
        if (has_q) hipLaunchKernelGGL((halfstep_kernel<G, I, XiMode::Mask, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((halfstep_kernel<G, I, XiMode::Mask, false>), grid, block, 0, stream, a);
        break;
    case XiMode::PerSite:
        if (has_q) hipLaunchKernelGGL((halfstep_kernel<G, I, XiMode::PerSite, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((halfstep_kernel<G, I, XiMode::PerSite, false>), grid, block, 0, stream, a);
        break;
    case XiMode::Inject:
        hipLaunchKernelGGL((halfstep_kernel<G, I, XiMode::Inject, true>), grid, block, 0, stream, a);
        break;
    }
    return hipGetLastError();
}

__global__ void philox_test_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32x4 o = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = o.v0;
    out[4 * i + 1] = o.v1;
    out[4 * i + 2] = o.v2;
    out[4 * i + 3] = o.v3;
}

// Philox throughput: every thread evaluates `calls` blocks and folds them into
// one word that is stored only in the (practically impossible) case that it
// equals the key, so the work cannot be dropped.
__global__ __launch_bounds__(256) void philox_rate_kernel(uint32_t k0, uint32_t k1, int32_t calls, uint32_t* sink)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int32_t j = 0; j < calls; ++j) {
        const u32x4 o = philox4x32_10(g, (uint32_t)j, 0u, 0u, k0, k1);
        acc ^= o.v0 ^ o.v1 ^ o.v2 ^ o.v3;
    }
    if (acc == k0) sink[g & 255u] = acc;
}

}  // namespace

hipError_t launch_philox_rate(int64_t threads, int32_t calls, uint32_t* sink, hipStream_t stream)
{
    if (threads <= 0 || calls <= 0 || (threads % 256) != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(philox_rate_kernel, dim3((unsigned)(threads / 256)), dim3(256), 0, stream, 0x9E3779B9u,
                       0x243F6A88u, calls, sink);
    return hipGetLastError();
}

hipError_t launch_halfstep(const SweepArgs& a, XiMode mode, bool has_q, hipStream_t stream)
{
    switch (a.W) {
    case 1: return launch_layout<1, 1>(a, mode, has_q, stream);
    case 2: return launch_layout<2, 1>(a, mode, has_q, stream);
    case 4: return launch_layout<4, 1>(a, mode, has_q, stream);
    case 8: return launch_layout<8, 1>(a, mode, has_q, stream);
    case 16: return launch_layout<16, 1>(a, mode, has_q, stream);
    case 32: return launch_layout<32, 1>(a, mode, has_q, stream);
    case 64: return launch_layout<64, 1>(a, mode, has_q, stream);
    case 128: return launch_layout<64, 2>(a, mode, has_q, stream);
    case 256: return launch_layout<64, 4>(a, mode, has_q, stream);
    case 512: return launch_layout<64, 8>(a, mode, has_q, stream);
    case 1024: return launch_layout<64, 16>(a, mode, has_q, stream);
    default: return hipErrorInvalidValue;
    }
}

// The kernel launch_halfstep runs for rows of W words (see launch_layout).
void halfstep_kernel_name(int32_t W, XiMode mode, bool has_q, char* out, size_t n)
{
    const int G = W < 64 ? W : 64, I = W < 64 ? 1 : W / 64;
    const char* m = mode == XiMode::PerSite ? "PerSite" : (mode == XiMode::Inject ? "Inject" : "Mask");
    std::snprintf(out, n, "halfstep_kernel<%d,%d,%s,%s>", G, I, m, (has_q || mode == XiMode::Inject) ? "true" : "false");
}

hipError_t launch_philox_test(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                              hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(philox_test_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, stream, ctr, k0,
                       k1, n, out);
    return hipGetLastError();
}

}  // namespace sca

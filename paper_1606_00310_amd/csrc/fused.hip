// fused.hip -- both half-steps of one MCS in one pass over the lattice.
//
// The odd half-step of row y reads only values that the even half-step of
// rows y-1, y and y+1 produces (the checkerboard order of Sec. I-A: the x-
// and y- slopes of row y, and the y+ slopes of row y+1), so one sweep down
// the rows can apply the even half-step to row s+1 and then the odd half-step
// to row s, keeping a window of two rows in registers.  Each row of the state
// is then loaded and stored once per MCS instead of once per half-step: half
// the HBM traffic of two half-step launches (the paper's 1 byte per site
// update, Sec. III, becomes about 0.52).
//
// One wavefront owns a band of consecutive rows, the whole row across its 64
// lanes (W/64 words per lane, cross-word bits by lane shuffle as in
// halfstep.hpp).  A band [y0, y1) also recomputes the even half-step of rows
// y0-2, y0-1 and y1 and the odd half-step of row y0-1: they change slope bits
// stored in its own rows.  The counter-based random words make these
// recomputations identical to the neighbouring bands' own updates.  Because
// bands read two rows beyond each edge, the pass reads from `src` and writes
// `dst` (out of place); every row of dst is written by exactly one band.
#include "halfstep.hpp"

namespace sca {
namespace {

constexpr int kBlock = 256;

template <int I, XiMode MODE, bool HASQ>
__global__ __launch_bounds__(kBlock) void mcs_fused_kernel(SweepArgs a, const uint64_t* src, uint64_t* dst,
                                                           int32_t band)
{
    constexpr int G = 64;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (wave * band >= a.Y) return;  // whole wave: no shuffle partner is lost
    const int64_t y0 = wave * band, y1 = y0 + band;
    const int64_t ymask = a.Y - 1;
    const int64_t P = a.plane, W = a.W;
    // arrays S[d][parity] at offset (2d + parity) * plane
    const uint64_t* x0s = src;          // x-slopes, even sites
    const uint64_t* x1s = src + P;      // x-slopes, odd sites
    const uint64_t* y0s = src + 2 * P;  // y-slopes, even sites
    const uint64_t* y1s = src + 3 * P;  // y-slopes, odd sites

    // row s (between steps): x-/y- slopes of both parities; y-slopes of odd
    // sites of row s+1 (already hit by the even half-step of row s)
    uint64_t Ax0[I], Ax1[I], Ay0[I], Ay1[I], Ay1n[I];
#pragma unroll
    for (int i = 0; i < I; ++i) Ax0[i] = Ax1[i] = Ay0[i] = Ay1[i] = Ay1n[i] = 0;

    SweepArgs ae = a, ao = a;
    ae.parity = 0;
    ao.parity = 1;

    for (int64_t s = y0 - 3; s < y1; ++s) {
        const int64_t r1 = s & ymask;        // odd half-step row
        const int64_t r0 = (s + 1) & ymask;  // even half-step row
        const int64_t r2 = (s + 2) & ymask;
        uint64_t X0[I], X1[I], Y0[I], Y1n[I];
#pragma unroll
        for (int i = 0; i < I; ++i) {
            const int64_t w = i * G + lane;
            X0[i] = x0s[r0 * W + w];
            X1[i] = x1s[r0 * W + w];
            Y0[i] = y0s[r0 * W + w];
            Y1n[i] = y1s[r2 * W + w];
        }
        // even half-step, row r0: A = x-(even), B = y-(even), C = y-(odd, row r0+1), D = x-(odd)
        {
            const bool shifted = (r0 & 1) != 0;
            uint64_t XP[I], M[I], mp0 = 0, mq0 = 0;
            align_xplus<G, I>(X1, shifted, lane, 0, 64, XP);
            row_masks<G, I, MODE, HASQ>(ae, r0, lane, X0, Y0, Y1n, XP, M, mp0, mq0);
            apply_xplus<G, I>(X1, M, shifted, lane, 0, 64);
            if (r0 == 0 && s + 1 >= y0 && s + 1 < y1 && lane == 0) {
                const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
                if (dh != 0) *a.h0 += dh;
            }
        }
        // odd half-step, row r1: A = x-(odd), B = y-(odd), C = y-(even, row r1+1), D = x-(even)
        if (s >= y0 - 1) {
            const bool shifted = (r1 & 1) == 0;
            uint64_t XP[I], M[I], mp0 = 0, mq0 = 0;
            align_xplus<G, I>(Ax0, shifted, lane, 0, 64, XP);
            row_masks<G, I, MODE, HASQ>(ao, r1, lane, Ax1, Ay1, Y0, XP, M, mp0, mq0);
            apply_xplus<G, I>(Ax0, M, shifted, lane, 0, 64);
        }
        if (s >= y0) {
#pragma unroll
            for (int i = 0; i < I; ++i) {
                const int64_t w = i * G + lane;
                dst[0 * P + r1 * W + w] = Ax0[i];
                dst[1 * P + r1 * W + w] = Ax1[i];
                dst[2 * P + r1 * W + w] = Ay0[i];
                dst[3 * P + r1 * W + w] = Ay1[i];
            }
        }
#pragma unroll
        for (int i = 0; i < I; ++i) {
            Ax0[i] = X0[i];
            Ax1[i] = X1[i];
            Ay0[i] = Y0[i];
            Ay1[i] = Ay1n[i];
            Ay1n[i] = Y1n[i];
        }
    }
}

template <int I>
hipError_t launch_fused_i(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                          int32_t band, hipStream_t stream)
{
    const int64_t waves = a.Y / band;
    const dim3 grid((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)));
    const dim3 block(kBlock);
    if (mode == XiMode::Mask) {
        if (has_q) hipLaunchKernelGGL((mcs_fused_kernel<I, XiMode::Mask, true>), grid, block, 0, stream, a, src, dst, band);
        else hipLaunchKernelGGL((mcs_fused_kernel<I, XiMode::Mask, false>), grid, block, 0, stream, a, src, dst, band);
    } else {
        if (has_q) hipLaunchKernelGGL((mcs_fused_kernel<I, XiMode::PerSite, true>), grid, block, 0, stream, a, src, dst, band);
        else hipLaunchKernelGGL((mcs_fused_kernel<I, XiMode::PerSite, false>), grid, block, 0, stream, a, src, dst, band);
    }
    return hipGetLastError();
}

}  // namespace

bool fused_supported(int32_t W, int64_t Y, int32_t band)
{
    return (W == 64 || W == 128 || W == 256 || W == 512) && band >= 4 && (Y % band) == 0 && Y >= 2 * band;
}

hipError_t launch_mcs_fused(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                            int32_t band, hipStream_t stream)
{
    if (!fused_supported(a.W, a.Y, band) || mode == XiMode::Inject) return hipErrorInvalidValue;
    switch (a.W) {
    case 64: return launch_fused_i<1>(a, mode, has_q, src, dst, band, stream);
    case 128: return launch_fused_i<2>(a, mode, has_q, src, dst, band, stream);
    case 256: return launch_fused_i<4>(a, mode, has_q, src, dst, band, stream);
    default: return launch_fused_i<8>(a, mode, has_q, src, dst, band, stream);
    }
}

}  // namespace sca

// fused.hip -- K Monte-Carlo steps (2K half-steps) in one pass over the lattice.
//
// Half-step h of row r reads only values that half-step h-1 produces in rows
// r-1, r and r+1 (the checkerboard order of Sec. I-A: the x- and y- slopes of
// row r and the y+ slopes of row r+1).  So one sweep down the rows can keep a
// window of 2K+1 rows and, at each step s, apply half-step h to row
// s+2K-1-h for h = 0..2K-1 (even half-steps at even h): every row of the
// state is then loaded and stored once per K MCS instead of once per
// half-step.  The paper's bandwidth model of 1 byte per site update (Sec. III)
// becomes about 1/(2K) byte plus the band halo.
//
// A workgroup of NW wavefronts owns a band of consecutive rows; a row's words
// are spread over its NW*64 lanes (word w = i*64*NW + wave*64 + lane).  The
// cross-word bits (bit 0 of the next x+ word when a row's x+ neighbours are
// shifted, and the top bit of the previous word's mask on the way back) move
// by lane shuffle inside a wave; between waves they are exchanged once per
// row step through LDS, with one barrier: the next-word bits of all 2K
// half-steps of the coming step are known at the end of the current one, and
// the carries of the current step are needed only by later steps.
//
// A band [y0, y1) also applies half-step h to the halo rows y0-2K+h..y0-1 and
// y1..y1+2K-2-h, which its own rows depend on; the counter-based random words make those
// recomputations identical to the neighbouring bands' updates.  Bands read
// beyond their edges, so a pass reads `src` and writes `dst` (out of place);
// every row of dst is written by exactly one band.
#include "halfstep.hpp"
#include "sca_internal.hpp"

namespace sca {
namespace {

template <int NW, int I, int K, XiMode MODE, bool HASQ>
__global__ __launch_bounds__(NW * 64) void mcs_block_kernel(SweepArgs a, const uint64_t* src, uint64_t* dst,
                                                            int32_t band)
{
    constexpr int H = 2 * K;      // half-steps per pass
    constexpr int R = 2 * K + 1;  // window rows
    static_assert(H * I <= 32, "exchange bits per lane");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t y0 = (int64_t)blockIdx.x * band, y1 = y0 + band;
    const int64_t ymask = a.Y - 1;
    const int64_t P = a.plane, W = a.W;
    __shared__ uint32_t xa[2][NW];  // lane 0: bit 0 of the x+ words of the next step's half-steps
    __shared__ uint32_t xb[2][NW];  // lane 63: top bits of this step's masks

    // window row j holds row s+j: arrays 0 = x-(even), 1 = x-(odd), 2 = y-(even), 3 = y-(odd)
    uint64_t Wn[R][4][I];
    uint32_t nb0 = 0;  // lane 63: bit 0 of the next wave's first word, per (half-step, slot)

    auto word = [&](int i) -> int64_t { return (int64_t)i * (64 * NW) + wv * 64 + lane; };
    // rows below y0-2K feed no half-step the band needs: not loaded
    auto load_row = [&](uint64_t (&row)[4][I], int64_t r) {
        const int64_t rr = r & ymask;
        const bool need = r >= y0 - H;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < I; ++i) row[c][i] = need ? src[c * P + rr * W + word(i)] : 0ull;
    };
    // bit 0 of each half-step's x+ words for the step whose window is Wn
    auto lsb_bits = [&]() -> uint32_t {
        uint32_t v = 0;
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int i = 0; i < I; ++i) v |= (uint32_t)(Wn[H - 1 - h][1 - (h & 1)][i] & 1ull) << (h * I + i);
        return v;
    };
    // from the next wave's lane 0 (the last wave continues in slot i+1 of wave 0)
    auto take_next = [&](uint32_t v) -> uint32_t {
        if (NW > 1 && wv < NW - 1) return v;
        uint32_t o = 0;
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int i = 0; i < I; ++i) o |= ((v >> (h * I + (i + 1) % I)) & 1u) << (h * I + i);
        return o;
    };
    // from the previous wave's lane 63 (the first wave continues from slot i-1 of the last wave)
    auto take_prev = [&](uint32_t v) -> uint32_t {
        if (NW > 1 && wv > 0) return v;
        uint32_t o = 0;
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int i = 0; i < I; ++i) o |= ((v >> (h * I + (i + I - 1) % I)) & 1u) << (h * I + i);
        return o;
    };

    // The band's rows depend on half-step h of rows y0-2K+h and up (the last
    // half-step of row y0-1 writes y-slopes of row y0, and each earlier
    // half-step widens the cone by one row), so half-step 0 starts on row
    // y0-2K, which the skewed sweep reaches at step y0-4K+1.
    const int64_t s0 = y0 - 2 * H + 1;
    // prologue: window rows s0 .. s0+2K-1, and the next-word bits for the first step
#pragma unroll
    for (int j = 0; j < R - 1; ++j) load_row(Wn[j], s0 + j);
    {
        const uint32_t v = lsb_bits();
        if (NW > 1) {
            if (lane == 0) xa[1][wv] = v;
            __syncthreads();
            if (lane == 63) nb0 = take_next(xa[1][(wv + 1) % NW]);
        } else {
            nb0 = take_next((uint32_t)__shfl((int)v, 0));
        }
    }

    // the row entering the window at each step is loaded one step ahead
    uint64_t Nx[4][I];
    load_row(Nx, s0 + H);

    int buf = 0;
    for (int64_t s = s0; s < y1; ++s, buf ^= 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < I; ++i) Wn[R - 1][c][i] = Nx[c][i];
        if (s + 1 < y1) load_row(Nx, s + 1 + H);
        // bit 0 of the next word for each slot: lanes 0..62 from the next lane
        uint32_t msb_all = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int j = H - 1 - h;          // window row of half-step h
            const int64_t r = s + j;          // its row
            const int par = h & 1;
            if (r < y0 - H + h) continue;     // not needed by the band's rows (and inputs not loaded)
            const int64_t rr = r & ymask;
            const bool shifted = ((par ^ (int)(rr & 1)) != 0);
            uint64_t(&D)[I] = Wn[j][1 - par];
            uint64_t XP[I], M[I], mp0 = 0, mq0 = 0;
            uint32_t lsb = 0;
#pragma unroll
            for (int i = 0; i < I; ++i) lsb |= (uint32_t)(D[i] & 1ull) << i;
            uint32_t nxt = (uint32_t)__shfl((int)lsb, (lane + 1) & 63);
            if (lane == 63) nxt = (nb0 >> (h * I)) & ((1u << I) - 1u);
#pragma unroll
            for (int i = 0; i < I; ++i)
                XP[i] = shifted ? ((D[i] >> 1) | ((uint64_t)((nxt >> i) & 1u) << 63)) : D[i];
            SweepArgs ah = a;
            ah.parity = par;
            ah.t = a.t + (uint32_t)(h >> 1);
            // row_masks indexes words as i*G + gl with G = 64*NW
            row_masks<64 * NW, I, MODE, HASQ>(ah, rr, wv * 64 + lane, Wn[j][par], Wn[j][2 + par],
                                                Wn[j + 1][2 + (1 - par)], XP, M, mp0, mq0);
            // x+ slopes: in-wave carries now, the first lane's carry after the exchange
            uint32_t msb = 0;
#pragma unroll
            for (int i = 0; i < I; ++i) msb |= (uint32_t)(M[i] >> 63) << i;
            const uint32_t prv = (uint32_t)__shfl((int)msb, (lane + 63) & 63);
#pragma unroll
            for (int i = 0; i < I; ++i) {
                const uint64_t carry = (lane == 0) ? 0ull : (uint64_t)((prv >> i) & 1u);
                D[i] ^= shifted ? ((M[i] << 1) | carry) : M[i];
            }
            msb_all |= msb << (h * I);
            if (par == 0 && rr == 0 && r >= y0 && r < y1 && wv == 0 && lane == 0) {
                const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
                if (dh != 0) *a.h0 += dh;
            }
        }
        // exchange: this step's top mask bits (for the first lanes' carries) and
        // the next step's next-word bits; one barrier
        {
            // next step's window is rows s+1 .. s+2K+1; its half-step h x+ words
            // are Wn[H - h][1 - (h & 1)] of the current window
            uint32_t v = 0;
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int i = 0; i < I; ++i) v |= (uint32_t)(Wn[H - h][1 - (h & 1)][i] & 1ull) << (h * I + i);
            uint32_t pm, nv;
            if (NW > 1) {
                if (lane == 0) xa[buf][wv] = v;
                if (lane == 63) xb[buf][wv] = msb_all;
                __syncthreads();
                pm = (lane == 0) ? take_prev(xb[buf][(wv + NW - 1) % NW]) : 0u;
                nv = (lane == 63) ? take_next(xa[buf][(wv + 1) % NW]) : 0u;
            } else {
                pm = take_prev((uint32_t)__shfl((int)msb_all, 63));
                nv = take_next((uint32_t)__shfl((int)v, 0));
            }
            if (lane == 0) {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int j = H - 1 - h;
                    const int par = h & 1;
                    const bool shifted = ((par ^ (int)((s + j) & 1)) != 0);
                    if (shifted) {
#pragma unroll
                        for (int i = 0; i < I; ++i) Wn[j][1 - par][i] ^= (uint64_t)((pm >> (h * I + i)) & 1u);
                    }
                }
            }
            if (lane == 63) nb0 = nv;
        }
        if (s >= y0) {
            const int64_t rr = s & ymask;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < I; ++i) dst[c * P + rr * W + word(i)] = Wn[0][c][i];
        }
#pragma unroll
        for (int j = 0; j < R - 1; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < I; ++i) Wn[j][c][i] = Wn[j + 1][c][i];
    }
}

template <int NW, int I, int K>
hipError_t launch_block(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                        int32_t band, hipStream_t stream)
{
    const dim3 grid((unsigned)(a.Y / band));
    const dim3 block(NW * 64);
    if (mode == XiMode::Mask) {
        if (has_q) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, true>), grid, block, 0, stream, a, src, dst, band);
        else hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, false>), grid, block, 0, stream, a, src, dst, band);
    } else {
        if (has_q) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::PerSite, true>), grid, block, 0, stream, a, src, dst, band);
        else hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::PerSite, false>), grid, block, 0, stream, a, src, dst, band);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_depth(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                        int32_t band, hipStream_t stream)
{
    switch (a.W) {
    case 64: return launch_block<1, 1, K>(a, mode, has_q, src, dst, band, stream);
    case 128: return launch_block<2, 1, K>(a, mode, has_q, src, dst, band, stream);
    case 256: return launch_block<4, 1, K>(a, mode, has_q, src, dst, band, stream);
    case 512: return launch_block<8, 1, K>(a, mode, has_q, src, dst, band, stream);
    case 1024: return launch_block<8, 2, K>(a, mode, has_q, src, dst, band, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool fused_supported(int32_t W, int64_t Y, int32_t band, int32_t depth)
{
    return (W == 64 || W == 128 || W == 256 || W == 512 || W == 1024) && depth >= 1 && depth <= 4 && band >= 4 &&
           (band & (band - 1)) == 0 && (Y % band) == 0 && Y >= 2 * band && band >= 2 * depth;
}

hipError_t launch_mcs_fused(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                            int32_t band, int32_t depth, hipStream_t stream)
{
    if (!fused_supported(a.W, a.Y, band, depth) || mode == XiMode::Inject) return hipErrorInvalidValue;
    switch (depth) {
    case 1: return launch_depth<1>(a, mode, has_q, src, dst, band, stream);
    case 2: return launch_depth<2>(a, mode, has_q, src, dst, band, stream);
    case 3: return launch_depth<3>(a, mode, has_q, src, dst, band, stream);
    default: return launch_depth<4>(a, mode, has_q, src, dst, band, stream);
    }
}

}  // namespace sca

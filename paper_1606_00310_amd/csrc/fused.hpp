// fused.hpp -- K Monte-Carlo steps (2K half-steps) in one pass over the lattice.
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
// between neighbouring lanes by DPP wavefront shifts; between waves they are exchanged once per
// row step through LDS, with one barrier: the next-word bits of all 2K
// half-steps of the coming step are known at the end of the current one, and
// the carries of the current step are needed only by later steps.
//
// A band [y0, y1) also applies half-step h to the halo rows y0-2K+h..y0-1 and
// y1..y1+2K-2-h, which its own rows depend on; the counter-based random words make those
// recomputations identical to the neighbouring bands' updates.  Bands read
// beyond their edges, so a pass reads `src` and writes `dst` (out of place);
// every row of dst is written by exactly one band.
#pragma once

#include <utility>

#include "halfstep.hpp"
#include "sca_internal.hpp"

namespace sca {
namespace {

// Deepest pass per kind of launch: passes with random draws are ALU-bound
// before the bandwidth saved by deeper passes matters, and the per-site
// path's step body is too large to unroll.
constexpr int kMaxDepthMask = 4;
constexpr int kMaxDepthPerSite = 4;
constexpr int kMaxDepthFixed = 8;
// X = 2^16 (512 words per row): the register window of mcs_fixed_kernel holds
// up to 13 MCS in one workgroup per CU.
constexpr int kMaxDepthFixed512 = 13;
constexpr int kMaxDepthWide = 5;  // two words per lane (X = 2^17)
// LDS of one 1024-thread workgroup of the LDS-window kernel at X = 2^17
constexpr int kWideLdsBytes = 3 * 4 * 1024 * 8 + 4 * 16 * 4;

// Word 3 of a gfx9 buffer descriptor for untyped dword accesses.
constexpr int32_t kBufferWord3 = 0x00020000;

// Calls f(integral_constant<u>, s + u) for u = 0 .. sizeof...(U)-1.
template <class F, int... U>
__device__ __forceinline__ void unrolled_steps(F& f, int s, std::integer_sequence<int, U...>)
{
    (f(std::integral_constant<int, U>{}, s + U), ...);
}

// Calls f(integral_constant<u>, s + u) for u = 0, 1, ... while it returns
// true; returns whether every call did.
template <class F, int... U>
__device__ __forceinline__ bool unrolled_steps_while(F& f, int s, std::integer_sequence<int, U...>)
{
    return (f(std::integral_constant<int, U>{}, s + U) && ...);
}

// Lane i receives v from lane i+1; lane 63 keeps `edge` (DPP wavefront shift).
__device__ __forceinline__ uint32_t from_next_lane_or(uint32_t v, uint32_t edge)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}

// Lane i receives v from lane i-1; lane 0 receives 0.
__device__ __forceinline__ uint32_t from_prev_lane_or_zero(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}

__device__ __forceinline__ uint64_t join(uint32_t lo, uint32_t hi) { return (uint64_t)lo | ((uint64_t)hi << 32); }

// The waves of a workgroup that share rows exchange one word per row step
// through LDS without a barrier: four slots per wave in rotation, each word
// carrying its exchange's tag (exchange count / 4, mod 64) above 26 value
// bits, and each wave polls the slot of the one neighbour it needs.  A wave
// cannot finish exchange k+1 before the reader of its exchange-k word has
// read it (the word it waits for at k+1 is that reader's, written after the
// reader's read at k), so a slot is never overwritten unread.
constexpr uint32_t kExchTagShift = 26, kExchValueMask = (1u << kExchTagShift) - 1u;
constexpr uint32_t kExchSpinLimit = 1u << 16;

__device__ __forceinline__ uint32_t exch_tag(int k) { return ((uint32_t)(k >> 2) & 63u) << kExchTagShift; }

// The value bits of the word tagged `tag` in *slot (an LDS word written by
// another wave of the workgroup).  One asm block with a bounded loop (a wave
// that is never served gives up after kExchSpinLimit reads and goes on): a
// loop in the compiler's own code here turns the kernels' rotating register
// windows into copies and spills.  Each read is waited for inside the block.
__device__ __forceinline__ uint32_t exch_poll(const uint32_t* slot, uint32_t tag)
{
    const uint32_t addr = (uint32_t)(uintptr_t)slot;  // the LDS byte offset (low half of the flat address)
    uint32_t w, v, t, n;
    asm volatile(
        "s_mov_b32 %[n], 0\n"
        "1:\n\t"
        "ds_read_b32 %[v], %[addr]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_readfirstlane_b32 %[w], %[v]\n\t"
        "s_and_b32 %[t], %[w], %[hi]\n\t"
        "s_cmp_eq_u32 %[t], %[tag]\n\t"
        "s_cbranch_scc1 2f\n\t"
        "s_add_u32 %[n], %[n], 1\n\t"
        "s_cmp_lt_u32 %[n], %[lim]\n\t"
        "s_cbranch_scc1 1b\n"
        "2:"
        : [w] "=&s"(w), [v] "=&v"(v), [t] "=&s"(t), [n] "=&s"(n)
        : [addr] "v"(addr), [tag] "s"(tag), [hi] "s"(~kExchValueMask), [lim] "s"(kExchSpinLimit)
        : "memory", "scc");
    return w & kExchValueMask;
}

__device__ __forceinline__ void exch_put(uint32_t* slot, uint32_t tag, uint32_t value)
{
    __hip_atomic_store(slot, tag | value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Fills the slots with a tag that matches none of the first four exchanges
// (then a workgroup barrier).
template <int NW>
__device__ __forceinline__ void exch_init(uint32_t (&xs)[4][NW])
{
    if (threadIdx.x < 4 * NW) xs[threadIdx.x / NW][threadIdx.x % NW] = 63u << kExchTagShift;
    __syncthreads();
}

// One half-step of one window row.  A, B: on-site x- and y- slopes; C: y+
// slopes (the next row's other-sublattice y- words); D: x+ slopes (this row's
// other-sublattice x- words).  SH: the row's x+ neighbours sit one site
// further (bit k+1, across the word edge).  nbits: lane 63's next-word bits,
// slot i in bit i.  In shifted rows the top mask bits are or-ed into msb_acc
// at bit `at` + i, and lane 0's incoming carry is left for the caller.
template <bool SH, int G, int I, XiMode MODE, bool HASQ, Draws DR = Draws::Any>
__device__ __forceinline__ void window_halfstep(const SweepArgs& ah, int rr, int gl, uint64_t (&A)[I],
                                                uint64_t (&B)[I], uint64_t (&C)[I], uint64_t (&D)[I],
                                                uint32_t nbits, uint32_t& msb_acc, int at, uint64_t& mp0,
                                                uint64_t& mq0, uint64_t* tail = nullptr)
{
    uint64_t XP[I], M[I];
#pragma unroll
    for (int i = 0; i < I; ++i) {
        if constexpr (SH) {
            const uint32_t lo = (uint32_t)D[i], hi = (uint32_t)(D[i] >> 32);
            const uint32_t nl = from_next_lane_or(lo, nbits >> i);  // bit 0: the next word's bit 0
            XP[i] = join(__builtin_amdgcn_alignbit(hi, lo, 1u), __builtin_amdgcn_alignbit(nl, hi, 1u));
        } else {
            XP[i] = D[i];
        }
    }
    row_masks<G, I, MODE, HASQ, DR>(ah, rr, gl, A, B, C, XP, M, mp0, mq0, tail);
#pragma unroll
    for (int i = 0; i < I; ++i) {
        if constexpr (SH) {
            const uint32_t lo = (uint32_t)M[i], hi = (uint32_t)(M[i] >> 32);
            const uint32_t ph = from_prev_lane_or_zero(hi);        // bit 31: the previous word's top bit
            D[i] ^= join(__builtin_amdgcn_alignbit(lo, ph, 31u), __builtin_amdgcn_alignbit(hi, lo, 31u));
            msb_acc |= (hi >> 31) << (at + i);
        } else {
            D[i] ^= M[i];
        }
    }
}

// DR (mask mode): what the launch knows of the number of draws; with
// Draws::OddTail each row's even half-step hands the shared last draw to its
// odd one (mask_words), and with removals (HASQ) at one word per lane the
// kernel is bounded to four waves per SIMD (128 VGPRs), which keeps two
// 512-thread workgroups per CU.
template <int NW, int I, int K, XiMode MODE, bool HASQ, Draws DR = Draws::Any>
__global__ __launch_bounds__(NW * 64, (DR == Draws::OddTail && HASQ && I == 1) ? 4 : 1) void mcs_block_kernel(
    SweepArgs a, const uint64_t* src, uint64_t* dst,
                                                            int32_t band)
{
    constexpr int H = 2 * K;      // half-steps per pass
    constexpr int R = 2 * K + 1;  // window rows
    constexpr int NS = R + 1;     // register slots: the window and the row in flight
    // Without per-site compares the step body is small enough to unroll the
    // sweep NS steps deep, so that the window rotates through the slots
    // instead of being moved down one slot per step (which also frees the
    // registers the moves needed), and each unrolled step knows at compile
    // time whether its rows are shifted.
    constexpr bool ROT = MODE != XiMode::PerSite;
    static_assert(H * I <= 32, "exchange bits per lane");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int y0 = (int)blockIdx.x * band, y1 = y0 + band;
    const int ymask = a.Y - 1;
    const int64_t P = a.plane, W = a.W;
    const uint32_t wo = (uint32_t)(wv * 64 + lane);  // slot 0's word in the row
    // Buffer descriptors, one per slope array: the lane's byte offset within a
    // row is a loop-invariant vector register and the row's byte offset a
    // scalar, so loads and stores need no per-access address arithmetic
    // (and accesses outside an array read 0 / are dropped by the hardware).
    auto off = [&](int i) -> uint32_t { return (wo + (uint32_t)(i * 64 * NW)) * 8u; };
    const int32_t plane_bytes = (int32_t)(P * 8);  // at most 2^30
    __amdgpu_buffer_rsrc_t rsrc[4], rdst[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        rsrc[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(src + c * P), (short)0, plane_bytes, kBufferWord3);
        rdst[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + c * P), (short)0, plane_bytes, kBufferWord3);
    }
    // Exchanged once per step through LDS with a barrier (the barrier-free
    // exchange of mcs_fixed_kernel brought nothing here: this kernel's time is
    // in the Philox products).
    __shared__ uint32_t xa[2][NW];  // lane 0: bit 0 of the x+ words of the next step's half-steps
    __shared__ uint32_t xb[2][NW];  // lane 63: top bits of this step's masks

    // slot arrays: 0 = x-(even), 1 = x-(odd), 2 = y-(even), 3 = y-(odd)
    uint64_t Wn[NS][4][I];
    // TAIL: the shared last draw of a row's odd half-step, left by its even
    // half-step one step earlier (the row keeps its slot from one step to
    // the next, and a row that skips a half-step skips the later ones too)
    constexpr bool TAIL = DR == Draws::OddTail && MODE == XiMode::Mask && ROT;
    uint64_t tail[TAIL ? NS : 1][I];
    uint32_t nb0 = 0;  // lane 63: bit 0 of the next wave's first word, per (half-step, slot)
    int buf = 0;

    auto load = [&](uint64_t (&row)[4][I], int r) {
        const int32_t rb = (int32_t)((r & ymask) * W * 8);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < I; ++i) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc[c], (int)off(i), rb, 0);
                row[c][i] = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
            }
    };
    // rows below y0-2K feed no half-step the band needs: not loaded
    auto load_row = [&](uint64_t (&row)[4][I], int r) {
        if (r >= y0 - H) {
            load(row, r);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < I; ++i) row[c][i] = 0ull;
        }
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
    const int s0 = y0 - 2 * H + 1;

    // Step s (u = (s - s0) mod NS when the slots rotate, else 0) holds row
    // s+j in slot (u+j) mod NS: rows s .. s+2K form the window, and row
    // s+2K+1 is loaded into the slot freed by row s-1, one step ahead of use.
    // Half-step h works on row s+2K-1-h with parity h&1, so all half-steps of
    // a step have the same row alignment: shifted iff s+2K-1 is odd, i.e. iff
    // s is even.  With the band a multiple of two, s0 is odd, so in the
    // rotating sweep step u is shifted iff u is odd.
    auto step = [&](auto U, int s) {
        constexpr int u = decltype(U)::value;
        auto sl = [](int j) { return (u + j) % NS; };
        if (s >= y1) {
            if constexpr (TAIL) {
                // the words the next step would read, defined on this path too (no
                // step runs after it: the sweep is over), so that none of them lives
                // across the loop
#pragma unroll
                for (int h = 0; h < H; h += 2)
#pragma unroll
                    for (int i = 0; i < I; ++i) tail[sl(H - 1 - h)][i] = 0;
            }
            return;
        }
        // Every step loads a row (the last one reloads the band's last row in
        // place of one it does not need), so that the wait before a row's
        // first use counts the same memory operations on every path.
        load(Wn[sl(H + 1)], min(s + 1 + H, y1 + H - 1));
        const bool shifted = ROT ? (u & 1) != 0 : (s & 1) == 0;
        uint32_t msb_all = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int j = H - 1 - h;          // window row of half-step h
            const int r = s + j;              // its row
            const int par = h & 1;
            if (r < y0 - H + h) {             // not needed by the band's rows (and inputs not loaded)
                if constexpr (TAIL) {
                    // defined on every path, so that a row's word lives only from its
                    // even half-step to its odd one
                    if (par == 0)
#pragma unroll
                        for (int i = 0; i < I; ++i) tail[sl(j)][i] = 0;
                }
                continue;
            }
            const int rr = r & ymask;
            SweepArgs ah = a;
            ah.parity = par;
            ah.t = a.t + (uint32_t)(h >> 1);
            uint64_t mp0 = 0, mq0 = 0;
            const uint32_t nbits = nb0 >> (h * I);
            // row_masks indexes words as i*G + gl with G = 64*NW
            uint64_t(&tl)[I] = tail[TAIL ? sl(j) : 0];
            if (ROT ? (u & 1) != 0 : shifted)
                window_halfstep<true, 64 * NW, I, MODE, HASQ, DR>(ah, rr, (int)wo, Wn[sl(j)][par],
                                                                    Wn[sl(j)][2 + par], Wn[sl(j + 1)][2 + (1 - par)],
                                                                    Wn[sl(j)][1 - par], nbits, msb_all, h * I, mp0,
                                                                    mq0, tl);
            else
                window_halfstep<false, 64 * NW, I, MODE, HASQ, DR>(ah, rr, (int)wo, Wn[sl(j)][par],
                                                                     Wn[sl(j)][2 + par], Wn[sl(j + 1)][2 + (1 - par)],
                                                                     Wn[sl(j)][1 - par], nbits, msb_all, h * I, mp0,
                                                                     mq0, tl);
            if (par == 0 && rr == 0 && r >= y0 && r < y1 && wo == 0) {
                // one lane of the grid; an atomic needs no wait for the old value
                const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
                if (dh != 0) atomicAdd((unsigned long long*)a.h0, (unsigned long long)dh);
            }
        }
        // exchange: this step's top mask bits (for the first lanes' carries,
        // shifted rows only) and the next step's next-word bits (needed only
        // if the next step is shifted, i.e. this one is not); one barrier
        {
            // next step's window is rows s+1 .. s+2K+1; its half-step h x+ words
            // are in window row H-h of the current step
            uint32_t v = 0;
            if (!shifted) {
#pragma unroll
                for (int h = 0; h < H; ++h)
#pragma unroll
                    for (int i = 0; i < I; ++i)
                        v |= (uint32_t)(Wn[sl(H - h)][1 - (h & 1)][i] & 1ull) << (h * I + i);
            }
            uint32_t pm, nv;
            if (NW > 1) {
                if (lane == 0) xa[buf][wv] = v;
                if (lane == 63) xb[buf][wv] = msb_all;
                __syncthreads();
                pm = (lane == 0) ? take_prev(xb[buf][(wv + NW - 1) % NW]) : 0u;
                nv = (lane == 63) ? take_next(xa[buf][(wv + 1) % NW]) : 0u;
                buf ^= 1;
            } else {
                pm = take_prev((uint32_t)__builtin_amdgcn_readlane((int)msb_all, 63));
                nv = take_next((uint32_t)__builtin_amdgcn_readlane((int)v, 0));
            }
            if (shifted && lane == 0) {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int j = H - 1 - h;
                    const int par = h & 1;
#pragma unroll
                    for (int i = 0; i < I; ++i) Wn[sl(j)][1 - par][i] ^= (uint64_t)((pm >> (h * I + i)) & 1u);
                }
            }
            if (lane == 63) nb0 = nv;
        }
        if (s >= y0) {
            const int rr = s & ymask;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < I; ++i) {
                    const uint64_t w = Wn[sl(0)][c][i];
                    __attribute__((ext_vector_type(2))) uint32_t v;
                    v[0] = (uint32_t)w;
                    v[1] = (uint32_t)(w >> 32);
                    __builtin_amdgcn_raw_buffer_store_b64(v, rdst[c], (int)off(i), (int32_t)(rr * W * 8), 0);
                }
        }
    };

    // prologue: rows s0 .. s0+2K, and the next-word bits for the first step
    // (s0 is odd, so the first step is not shifted and needs none)
#pragma unroll
    for (int j = 0; j < R; ++j) load_row(Wn[j], s0 + j);

    if constexpr (ROT) {
        for (int s = s0; s < y1; s += NS) unrolled_steps(step, s, std::make_integer_sequence<int, NS>{});
    } else {
        for (int s = s0; s < y1; ++s) {
            step(std::integral_constant<int, 0>{}, s);
#pragma unroll
            for (int j = 0; j < NS - 1; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int i = 0; i < I; ++i) Wn[j][c][i] = Wn[j + 1][c][i];
        }
    }
}

// Draw-free passes of K = kLdsDepth MCS for rows of one word per lane (and
// at X = 2^17 with 1024-thread workgroups).  The
// 2K+2-row register window of mcs_block_kernel no longer fits the 128 VGPRs
// that two 512-thread workgroups per CU allow, so the two newest rows stay in
// LDS: row s+2K, of which half-step 0 needs only the odd-sublattice y-slopes
// (its y+ words), and row s+2K+1, which arrives by LDS DMA
// (global_load_lds_dwordx4, no registers in flight) during step s.  Rows
// s .. s+2K-1 live in registers; row s+2K-1 moves from LDS into the slot that
// row s-1 left.  Three row buffers rotate: the one being filled was last read
// before the previous step's barrier.
constexpr int kLdsDepth = 6;
// From this depth on, draw-free passes of one word per lane run one
// workgroup per CU anyway, and the register window with rows loaded ahead
// (mcs_fixed_kernel) replaces the LDS window.
constexpr int kFixedDeepDepth = 7;

// Two 512-thread workgroups per CU need at most 128 VGPRs: the 6-MCS kernel
// fits (121), and so does its 1024-thread form at X = 2^17.
template <int NW, int K, bool HASQ>
__global__ __launch_bounds__(NW * 64) void mcs_block_lds_kernel(SweepArgs a, const uint64_t* src, uint64_t* dst,
                                                                int32_t band)
{
    constexpr int H = 2 * K;   // half-steps per pass
    constexpr int NS = H;      // register slots: rows s .. s+2K-1
    constexpr int WR = 64 * NW;  // words per row and array
    static_assert(H <= 32, "exchange bits per lane");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int y0 = (int)blockIdx.x * band, y1 = y0 + band;
    const int ymask = a.Y - 1;
    const int64_t P = a.plane;
    const uint32_t wo = (uint32_t)(wv * 64 + lane);
    const int32_t plane_bytes = (int32_t)(P * 8);
    __amdgpu_buffer_rsrc_t rsrc[4], rdst[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        rsrc[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(src + c * P), (short)0, plane_bytes, kBufferWord3);
        rdst[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + c * P), (short)0, plane_bytes, kBufferWord3);
    }
    __shared__ __attribute__((aligned(16))) uint64_t rowbuf[3][4 * WR];  // [buffer][array][word]
    __shared__ uint32_t xa[2][NW];
    __shared__ uint32_t xb[2][NW];

    uint64_t Wn[NS][4][1];
    uint32_t nb0 = 0;
    int buf = 0;

    auto load_row = [&](uint64_t (&row)[4][1], int r) {
        const int rr = r & ymask;
        if (r >= y0 - H) {
            const int32_t rb = (int32_t)(rr * WR * 8);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc[c], (int)(wo * 8u), rb, 0);
                row[c][0] = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) row[c][0] = 0ull;
        }
    };
    // Row r into LDS buffer b by DMA: 2*NW chunks of 128 words, two per wave,
    // 16 bytes per lane.  Rows below y0-2K feed no half-step the band needs.
    auto dma_row = [&](int r, int b) {
        if (r < y0 - H) return;
        const int64_t rr = r & ymask;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int q = wv * 2 + k;
            const int f = 128 * q + 2 * lane;  // word of the row buffer, [array][word]
            const uint64_t* g = src + (f / WR) * P + rr * WR + (f % WR);
            __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)&rowbuf[b][128 * q],
                                             16, 0, 0);
        }
    };
    const int s0 = y0 - 2 * H + 1;

    // Step s = s0 + k holds row s+j in register slot (u+j) mod 2K, u = k mod 2K,
    // for j < 2K; row s+2K is in LDS buffer (k+2K) mod 3.  Shifted iff s is
    // even, i.e. iff u is odd (s0 is odd and 2K is even).
    auto step = [&](auto U, int s) {
        constexpr int u = decltype(U)::value;
        if (s >= y1) return;
        const int k = s - s0;
        auto sl = [](int j) { return (u + j) % NS; };
        const int bN = (k + H) % 3;  // buffer of row s+2K
        if (k > 0) {
            const int bP = (k + H - 1) % 3;
#pragma unroll
            for (int c = 0; c < 4; ++c) Wn[sl(H - 1)][c][0] = rowbuf[bP][c * WR + wo];
        }
        if (s + 1 < y1) dma_row(s + 1 + H, (k + H + 1) % 3);
        constexpr bool shifted = (u & 1) != 0;
        uint32_t msb_all = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int j = H - 1 - h;
            const int r = s + j;
            const int par = h & 1;
            if (r < y0 - H + h) continue;
            const int rr = r & ymask;
            SweepArgs ah = a;
            ah.parity = par;
            ah.t = a.t + (uint32_t)(h >> 1);
            uint64_t mp0 = 0, mq0 = 0;
            const uint32_t nbits = nb0 >> h;
            if (j + 1 < H) {
                window_halfstep<shifted, WR, 1, XiMode::Fixed, HASQ>(ah, rr, (int)wo, Wn[sl(j)][par], Wn[sl(j)][2 + par],
                                                                     Wn[sl(j + 1)][2 + (1 - par)], Wn[sl(j)][1 - par],
                                                                     nbits, msb_all, h, mp0, mq0);
            } else {
                // y+ words from the newest row, in LDS; written back for the next step
                uint64_t C[1] = {rowbuf[bN][(2 + (1 - par)) * WR + wo]};
                window_halfstep<shifted, WR, 1, XiMode::Fixed, HASQ>(ah, rr, (int)wo, Wn[sl(j)][par], Wn[sl(j)][2 + par],
                                                                     C, Wn[sl(j)][1 - par], nbits, msb_all, h, mp0, mq0);
                rowbuf[bN][(2 + (1 - par)) * WR + wo] = C[0];
            }
            if (par == 0 && rr == 0 && r >= y0 && r < y1 && wo == 0) {
                const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
                if (dh != 0) atomicAdd((unsigned long long*)a.h0, (unsigned long long)dh);
            }
        }
        {
            uint32_t v = 0;
            if (!shifted) {
                v = (uint32_t)(rowbuf[bN][1 * WR + wo] & 1ull);  // h = 0: row s+2K, odd x-slopes
#pragma unroll
                for (int h = 1; h < H; ++h) v |= (uint32_t)(Wn[sl(H - h)][1 - (h & 1)][0] & 1ull) << h;
            }
            uint32_t pm, nv;
            if (NW > 1) {
                if (lane == 0) xa[buf][wv] = v;
                if (lane == 63) xb[buf][wv] = msb_all;
                __syncthreads();
                pm = (lane == 0) ? xb[buf][(wv + NW - 1) % NW] : 0u;
                nv = (lane == 63) ? xa[buf][(wv + 1) % NW] : 0u;
                buf ^= 1;
            } else {
                __syncthreads();  // the row DMA'd this step is complete before it is read
                pm = (uint32_t)__builtin_amdgcn_readlane((int)msb_all, 63);
                nv = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
            }
            if (shifted && lane == 0) {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int j = H - 1 - h;
                    const int par = h & 1;
                    Wn[sl(j)][1 - par][0] ^= (uint64_t)((pm >> h) & 1u);
                }
            }
            if (lane == 63) nb0 = nv;
        }
        if (s >= y0) {
            const int rr = s & ymask;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint64_t w = Wn[sl(0)][c][0];
                __attribute__((ext_vector_type(2))) uint32_t v;
                v[0] = (uint32_t)w;
                v[1] = (uint32_t)(w >> 32);
                __builtin_amdgcn_raw_buffer_store_b64(v, rdst[c], (int)(wo * 8u), (int32_t)(rr * WR * 8), 0);
            }
        }
    };

    // prologue: rows s0 .. s0+2K-1 into registers, row s0+2K into LDS
#pragma unroll
    for (int j = 0; j < H; ++j) load_row(Wn[j], s0 + j);
    dma_row(s0 + H, H % 3);
    __syncthreads();
    for (int s = s0; s < y1; s += NS) unrolled_steps(step, s, std::make_integer_sequence<int, NS>{});
}

// One draw-free half-step (p, q in {0, 1}) of a window row held as 32-bit
// halves: A, B on-site x- and y- slopes, C the y+ slopes, D the x+ slopes
// (aligned, or one site further when SH).  Without q the pass has p = 1, so
// the update mask is T & C with T = ~A & ~B & x+ (Eq. (3) with every draw
// accepted), and each slope it flips is x ^ (T & C): one v_bitop3 per half
// word (truth table 0x78) instead of forming the mask and xor-ing it in.
// In shifted rows the update is applied to the aligned copy of the x+ slopes,
// which is then shifted back by one site: bit k+1 of D takes bit k, and bit 0
// of each lane's word takes the top bit of the previous lane's, so lane 0's
// bit 0 is left for the exchange with the previous wave, which replaces it.
// edge: lane 63's next-word bit in bit 0; msb collects, per half-step, the
// new top bit of the aligned copy (the next word's bit 0, shifted in from the
// right); mp_lo, mq_lo: low mask words.
template <bool SH, bool HASQ>
__device__ __forceinline__ void fixed_halfstep(uint32_t (&A)[2], uint32_t (&B)[2], uint32_t (&C)[2],
                                               uint32_t (&D)[2], uint32_t edge, uint32_t xip, uint32_t xiq,
                                               uint32_t& msb, uint32_t& mp_lo, uint32_t& mq_lo)
{
    uint32_t XP[2];
    if constexpr (SH) {
        const uint32_t nl = from_next_lane_or(D[0], edge);
        XP[0] = __builtin_amdgcn_alignbit(D[1], D[0], 1u);
        XP[1] = __builtin_amdgcn_alignbit(nl, D[1], 1u);
    } else {
        XP[0] = D[0];
        XP[1] = D[1];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if constexpr (!HASQ) {
            const uint32_t T = __builtin_amdgcn_bitop3_b32(A[i], B[i], XP[i], 0x02);  // ~A & ~B & x+
            if (i == 0) { mp_lo = T & C[0]; mq_lo = 0; }
            A[i] = __builtin_amdgcn_bitop3_b32(A[i], T, C[i], 0x78);  // A ^ (T & C)
            B[i] = __builtin_amdgcn_bitop3_b32(B[i], T, C[i], 0x78);
            if constexpr (SH) XP[i] = __builtin_amdgcn_bitop3_b32(XP[i], T, C[i], 0x78);
            else D[i] = __builtin_amdgcn_bitop3_b32(D[i], T, C[i], 0x78);
            C[i] = __builtin_amdgcn_bitop3_b32(C[i], T, C[i], 0x78);
        } else {
            const uint32_t mp = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_bitop3_b32(A[i], B[i], XP[i], 0x02), C[i],
                                                            xip, 0x80);  // xi & ~A & ~B & x+ & C
            const uint32_t mq = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_bitop3_b32(A[i], B[i], XP[i], 0x40), C[i],
                                                            xiq, 0x20);  // xi & A & B & ~x+ & ~C
            const uint32_t M = mp | mq;
            A[i] ^= M;
            B[i] ^= M;
            C[i] ^= M;
            if constexpr (SH) XP[i] ^= M;
            else D[i] ^= M;
            if (i == 0) { mp_lo = mp; mq_lo = mq; }
        }
    }
    if constexpr (SH) {
        const uint32_t ph = from_prev_lane_or_zero(XP[1]);  // bit 31: the previous word's new top bit
        D[0] = __builtin_amdgcn_alignbit(XP[0], ph, 31u);
        D[1] = __builtin_amdgcn_alignbit(XP[1], XP[0], 31u);
        msb = __builtin_amdgcn_alignbit(msb, XP[1], 31u);  // (msb << 1) | the next word's new bit 0
        asm volatile("" : "+v"(msb));
    }
    // Pin the new slopes (and the top bits) here: left alone, the compiler
    // sinks each update to where the words are read next, the next step, and
    // keeps the masks of all 2K half-steps live until then (about 50 more
    // VGPRs at K = 8).
    asm volatile("" : "+v"(A[0]), "+v"(A[1]), "+v"(B[0]), "+v"(B[1]), "+v"(C[0]), "+v"(C[1]), "+v"(D[0]), "+v"(D[1]));
}

// Deep draw-free passes for rows of one word per lane (X = 2^13 .. 2^16)
// with one workgroup per CU: the register window of 2K+1 rows plus DIST
// rows in flight, loaded DIST steps ahead of use so that each load has
// DIST row steps of compute to arrive in (3; at K = 12 and 13 the window
// alone fills the registers and a step of 2K half-steps hides a load by
// itself).
// The waves exchange their one word per step through LDS without a barrier:
// each polls the slot of the one neighbour it needs (a workgroup barrier per
// step cost about 9 % of the pass).  The first two unrolled rounds of the sweep, which hold the
// band's upper halo, the origin row of band 0 and the rows not yet stored,
// are compiled with those conditions resolved per step; the rest runs with
// no per-half-step conditions.
template <int NW, int K, int DIST, bool HASQ>
__global__ __launch_bounds__(NW * 64) void mcs_fixed_kernel(SweepArgs a, const uint64_t* src, uint64_t* dst,
                                                            int32_t band)
{
    constexpr int H = 2 * K;             // half-steps per pass
    constexpr int NS = H + 1 + DIST;     // register slots: window and rows in flight
    constexpr int WR = 64 * NW;          // words per row and array
    static_assert(NS % 2 == 0, "even rotation keeps each step's alignment fixed");
    static_assert(H <= 32, "exchange bits per lane");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int y0 = (int)blockIdx.x * band, y1 = y0 + band;
    const int ymask = a.Y - 1;
    const int64_t P = a.plane;
    const uint32_t voff = (uint32_t)(wv * 64 + lane) * 8u;
    const int32_t plane_bytes = (int32_t)(P * 8);
    __amdgpu_buffer_rsrc_t rsrc[4], rdst[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        rsrc[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(src + c * P), (short)0, plane_bytes, kBufferWord3);
        rdst[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + c * P), (short)0, plane_bytes, kBufferWord3);
    }
    // Per wave and step: the next-word bits an aligned step passes to the
    // wave before it, or the new bit 0 of the first x+ words that a shifted
    // step passes to the wave after it (exch_*: no barrier)
    static_assert(H <= 26, "exchange value and tag share one word");
    __shared__ uint32_t xs[4][NW];
    if constexpr (NW > 1) exch_init<NW>(xs);
    const uint32_t xip = (uint32_t)a.all_p, xiq = (uint32_t)a.all_q;

    // [slot][array][half]; arrays 0 = x-(even), 1 = x-(odd), 2 = y-(even), 3 = y-(odd)
    uint32_t Wn[NS][4][2];
    uint32_t nb = 0;  // lane 63: the next wave's next-word bits, half-step h in bit 32-2K+h
    int xk = 0;       // exchanges so far (a counter of its own: deriving it from the row index made the
                      // compiler give up the rotating register window and spill)

    auto load_row = [&](uint32_t (&row)[4][2], int r) {
        const int32_t rb = (int32_t)((r & ymask) * WR * 8);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc[c], (int)voff, rb, 0);
            row[c][0] = v[0];
            row[c][1] = v[1];
        }
    };
    const int s0 = y0 - 2 * H + 1;

    // Step s = s0 + k holds row s+j in slot (u+j) mod NS, u = k mod NS; rows
    // s .. s+2K are the window and rows up to s+2K+DIST-1 are in flight.  s0
    // is odd and NS even, so step u is shifted iff u is odd.  KC is k for the
    // first 2NS steps (the halo rows above y0-2K+h that half-step h skips,
    // k < 2h, the origin row of band 0 at k = 2K .. 4K-1 and the rows above
    // y0, k < 4K-1, which are not stored, all fall there) and -1 after.
    auto step = [&](auto U, auto KC, int s) __attribute__((always_inline)) {
        constexpr int u = decltype(U)::value % NS;
        constexpr int kc = decltype(KC)::value;
        constexpr bool SH = (u & 1) != 0;
        if (s >= y1) return false;
        auto sl = [](int j) { return (u + j) % NS; };
        // Every step loads a row, so that the wait before a row's first use
        // counts the same memory operations on every path; the last steps
        // load the band's last row again in place of rows it does not need.
        load_row(Wn[sl(H + DIST)], min(s + H + DIST, y1 + H - 1));
        uint32_t msb = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int j = H - 1 - h;
            const int par = h & 1;
            if (kc >= 0 && kc < 2 * h) {  // row above y0-2K+h: feeds none of the band's rows
                if (SH) msb <<= 1;
                continue;
            }
            uint32_t mp_lo, mq_lo;
            fixed_halfstep<SH, HASQ>(Wn[sl(j)][par], Wn[sl(j)][2 + par], Wn[sl(j + 1)][3 - par], Wn[sl(j)][1 - par],
                                     nb >> (32 - H + h), xip, xiq, msb, mp_lo, mq_lo);
            // row 0 of band 0 is row s0+k+j with s0 = 1-4K
            if (kc >= 0 && par == 0 && kc + j == 2 * H - 1) {
                if (y0 == 0 && voff == 0) {
                    const int64_t dh = 2 * (int64_t)(mp_lo & 1u) - 2 * (int64_t)(mq_lo & 1u);
                    if (dh != 0) atomicAdd((unsigned long long*)a.h0, (unsigned long long)dh);
                }
            }
        }
        // exchange, one barrier: an aligned step passes on the next step's
        // next-word bits (bit 0 of the x+ words of its half-steps, collected
        // from the right), a shifted step the new bit 0 of the next wave's
        // first x+ words
        uint32_t v = 0;
        if constexpr (!SH) {
#pragma unroll
            for (int h = 0; h < H; ++h) v = __builtin_amdgcn_alignbit(Wn[sl(H - h)][1 - (h & 1)][0], v, 1u);
        }
        const uint32_t out = SH ? (uint32_t)__builtin_amdgcn_readlane((int)msb, 63)
                                : (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
        uint32_t in = out;  // one wave: the row wraps within it
        if constexpr (NW > 1) {
            const uint32_t tag = exch_tag(xk);
            uint32_t* slot = xs[xk & 3];
            ++xk;
            // a shifted step's word holds its 2K bits at the bottom, an aligned
            // step's at the top (bit 32-2K+h for half-step h)
            if (lane == 0) exch_put(&slot[wv], tag, SH ? out : (out >> (32 - H)));
            const uint32_t w = exch_poll(&slot[SH ? (wv + NW - 1) % NW : (wv + 1) % NW], tag);
            in = SH ? w : (w << (32 - H));
        }
        if constexpr (SH) {
            // lane 0's bit 0 of the x+ word of each half-step's row: the new
            // value the previous wave's lane 63 computed (its next word's bit 0)
            const uint32_t pms = (uint32_t)__builtin_amdgcn_readfirstlane((int)in);
            if (lane == 0) {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    uint32_t& w = Wn[sl(H - 1 - h)][1 - (h & 1)][0];
                    w = (w & ~1u) | ((pms >> (H - 1 - h)) & 1u);
                }
            }
        } else {
            nb = in;
        }
        if (kc < 0 || kc >= 2 * H - 1) {  // row s >= y0
            const int32_t rb = (int32_t)((s & ymask) * WR * 8);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                __attribute__((ext_vector_type(2))) uint32_t w;
                w[0] = Wn[sl(0)][c][0];
                w[1] = Wn[sl(0)][c][1];
                __builtin_amdgcn_raw_buffer_store_b64(w, rdst[c], (int)voff, rb, 0);
            }
        }
        return true;
    };

    // prologue: the window and the rows in flight before step s0; rows above
    // y0-2K are not needed and start as zero
#pragma unroll
    for (int j = 0; j < H + DIST; ++j) {
        if (j >= H - 1) {  // s0 + j >= y0 - 2K
            load_row(Wn[j], s0 + j);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) Wn[j][c][0] = Wn[j][c][1] = 0u;
        }
    }
    auto first = [&](auto KC, int s) __attribute__((always_inline)) { return step(KC, KC, s); };
    auto plain = [&](auto U, int s) __attribute__((always_inline)) {
        return step(U, std::integral_constant<int, -1>{}, s);
    };
    // the first step past the band ends the sweep
    if (unrolled_steps_while(first, s0, std::make_integer_sequence<int, 2 * NS>{}))
        for (int s = s0 + 2 * NS; unrolled_steps_while(plain, s, std::make_integer_sequence<int, NS>{}); s += NS) {
        }
}

template <int NW, int I, int K>
hipError_t launch_block(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                        int32_t band, hipStream_t stream)
{
    const dim3 grid((unsigned)(a.Y / band));
    const dim3 block(NW * 64);
    if (mode == XiMode::Mask && a.ndraw == 0) {
        if constexpr (I == 1 && K >= kFixedDeepDepth) {
            // the p = 1 form needs every p-draw accepted; p = 0 goes through the general masks
            if (has_q || a.all_p == 0)
                hipLaunchKernelGGL((mcs_fixed_kernel<NW, K, 3, true>), grid, block, 0, stream, a, src, dst, band);
            else
                hipLaunchKernelGGL((mcs_fixed_kernel<NW, K, 3, false>), grid, block, 0, stream, a, src, dst, band);
        } else if constexpr (I == 1 && K >= kLdsDepth) {
            if (has_q) hipLaunchKernelGGL((mcs_block_lds_kernel<NW, K, true>), grid, block, 0, stream, a, src, dst, band);
            else hipLaunchKernelGGL((mcs_block_lds_kernel<NW, K, false>), grid, block, 0, stream, a, src, dst, band);
        } else {
            if (has_q) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Fixed, true>), grid, block, 0, stream, a, src, dst, band);
            else hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Fixed, false>), grid, block, 0, stream, a, src, dst, band);
        }
    } else if (mode == XiMode::Mask) {
        if constexpr (K <= kMaxDepthMask) {
            // an odd number of draws (p = 1/2 among them): one Philox call per
            // word serves both half-steps of the last draw.  With removals the
            // kept words need a bound of four waves per SIMD to keep the 4-MCS
            // pass at two workgroups per CU (128 VGPRs, two spilled); at two
            // words per lane they would not fit, and the odd half-step calls again.
            const bool odd = (a.ndraw & 1) != 0;
            constexpr Draws ODD_Q = I == 1 ? Draws::OddTail : Draws::Any;
            if (has_q && odd) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, true, ODD_Q>), grid, block, 0, stream, a, src, dst, band);
            else if (has_q) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, true, Draws::Even>), grid, block, 0, stream, a, src, dst, band);
            else if (odd) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, false, Draws::OddTail>), grid, block, 0, stream, a, src, dst, band);
            else hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::Mask, false, Draws::Even>), grid, block, 0, stream, a, src, dst, band);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if constexpr (K <= kMaxDepthPerSite) {
            if (has_q) hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::PerSite, true>), grid, block, 0, stream, a, src, dst, band);
            else hipLaunchKernelGGL((mcs_block_kernel<NW, I, K, XiMode::PerSite, false>), grid, block, 0, stream, a, src, dst, band);
        } else {
            return hipErrorInvalidValue;
        }
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
    case 1024:
        // two words per lane in the register-window kernel, or, for the
        // LDS-window kernel, one word per lane of a 1024-thread workgroup
        if constexpr (K == kLdsDepth) {
            if (mode == XiMode::Mask && a.ndraw == 0) {
                const dim3 grid((unsigned)(a.Y / band)), block(1024);
                if (has_q) hipLaunchKernelGGL((mcs_block_lds_kernel<16, K, true>), grid, block, 0, stream, a, src, dst, band);
                else hipLaunchKernelGGL((mcs_block_lds_kernel<16, K, false>), grid, block, 0, stream, a, src, dst, band);
                return hipGetLastError();
            }
        }
        if constexpr (K <= kMaxDepthWide) return launch_block<8, 2, K>(a, mode, has_q, src, dst, band, stream);
        else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Passes of 5..13 MCS (draw-free only), built in translation units of their own.
hipError_t launch_mcs_fused_deep(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                                 int32_t band, int32_t depth, hipStream_t stream);
hipError_t launch_mcs_fused_deeper(const SweepArgs& a, bool has_q, const uint64_t* src, uint64_t* dst, int32_t band,
                                   int32_t depth, hipStream_t stream);

}  // namespace sca

// batch.hip -- many independent realizations in one persistent launch.
//
// A fixed grid of workgroups (a few per compute unit) pulls realizations from
// a device work counter, largest remaining work first, and runs each one's
// MCS of the epoch to completion with workgroup barriers between the
// half-steps.  The row-group arithmetic is the single-lattice kernel's
// (halfstep.hpp) and every realization draws from its own seed with the same
// counters (g, t, 2j+parity, 0), so its state is bit-identical to a solo run
// whatever the launch shape or the order.
//
// States small enough for the workgroup's LDS budget are copied into LDS once
// per epoch and all their half-steps run there; larger ones are updated in
// place in the arena, where they stay L2 / Infinity-Cache resident while one
// workgroup works on them, and those with rows of 8..64 words run as
// temporally blocked passes of 1 or 2 MCS (one HBM round trip per pass
// instead of per half-step).  Same-parity sites share no bond, so within a
// half-step every word is read and written by exactly one lane; the barrier
// between half-steps (a workgroup-scope release/acquire) orders them.
#include <utility>

#include "halfstep.hpp"
#include "sca_internal.hpp"

namespace sca {
namespace {

// Calls f(integral_constant<u>, k + u) for u = 0 .. sizeof...(U)-1.
template <class F, int... U>
__device__ __forceinline__ void unrolled_steps(F& f, int k, std::integer_sequence<int, U...>)
{
    (f(std::integral_constant<int, U>{}, k + U), ...);
}

// Word 3 of a gfx9 buffer descriptor for untyped dword accesses.
constexpr int32_t kBufferWord3 = 0x00020000;

// Word tile: a row of W words is held by W/IW lanes with IW words each
// (IW = 2 gives every lane two independent random-word chains; rows of one
// word always use one lane).
template <int W, XiMode MODE, bool HASQ, int NWAVES, int IW>
__device__ __forceinline__ void all_rows(const SweepArgs& a, uint64_t* S, int wave, int lane)
{
    constexpr int I = (W >= IW) ? IW : 1;
    constexpr int G = W / I;
    constexpr int kRowsPerWave = 64 / G;
    for (int64_t rb = (int64_t)wave * kRowsPerWave; rb < a.Y; rb += (int64_t)NWAVES * kRowsPerWave)
        halfstep_rows<G, I, MODE, HASQ>(a, S, rb + lane / G, lane);
}

template <int W, int NWAVES, int IW>
__device__ __forceinline__ void all_rows_mode(const SweepArgs& a, uint64_t* S, int mode, bool has_q, int wave,
                                              int lane)
{
    if (mode == 0) {
        if (has_q) all_rows<W, XiMode::Mask, true, NWAVES, IW>(a, S, wave, lane);
        else all_rows<W, XiMode::Mask, false, NWAVES, IW>(a, S, wave, lane);
    } else {
        if (has_q) all_rows<W, XiMode::PerSite, true, NWAVES, IW>(a, S, wave, lane);
        else all_rows<W, XiMode::PerSite, false, NWAVES, IW>(a, S, wave, lane);
    }
}

// Half-step over a state in LDS (W <= 8: at most 64 KiB fits only such rows
// of a lattice with X*Y <= 2^18).
template <int NWAVES, int IW>
__device__ __forceinline__ void halfstep_lds(const SweepArgs& a, uint64_t* S, int mode, bool has_q, int wave,
                                             int lane)
{
    switch (a.W) {
    case 1: all_rows_mode<1, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 2: all_rows_mode<2, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 4: all_rows_mode<4, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    default: all_rows_mode<8, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    }
}

// Half-step over a state in global memory (W <= 64).
template <int NWAVES, int IW>
__device__ __forceinline__ void halfstep_global(const SweepArgs& a, uint64_t* S, int mode, bool has_q, int wave,
                                                int lane)
{
    switch (a.W) {
    case 1: all_rows_mode<1, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 2: all_rows_mode<2, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 4: all_rows_mode<4, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 8: all_rows_mode<8, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 16: all_rows_mode<16, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    case 32: all_rows_mode<32, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    default: all_rows_mode<64, NWAVES, IW>(a, S, mode, has_q, wave, lane); break;
    }
}

// Lane i of an aligned group of G lanes receives v from lane (i+1) mod G of
// its group (group_next) or from lane (i-1) mod G (group_prev): DPP row
// rotates for G = 16 (a row of 16 lanes is the group), two DPP row shifts
// and a select for G = 8, DPP wavefront rotates for G = 64, ds_bpermute for
// G = 32.  G is the same for the whole workgroup (a scalar), so the choice
// is a scalar branch and the blocked passes need one copy for all widths.
__device__ __forceinline__ uint32_t group_next(uint32_t v, int G, bool last, int nxl)
{
    if (G == 16) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12f /* row_ror:15 */, 0xf, 0xf, false);
    if (G == 8) {
        const uint32_t n = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x101 /* row_shl:1 */, 0xf, 0xf, false);
        const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x117 /* row_shr:7 */, 0xf, 0xf, false);
        return last ? w : n;
    }
    if (G == 64) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134 /* wave_rol:1 */, 0xf, 0xf, false);
    return (uint32_t)__shfl((int)v, nxl);
}

__device__ __forceinline__ uint32_t group_prev(uint32_t v, int G, bool first, int pvl)
{
    if (G == 16) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121 /* row_ror:1 */, 0xf, 0xf, false);
    if (G == 8) {
        const uint32_t p = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
        const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x107 /* row_shl:7 */, 0xf, 0xf, false);
        return first ? w : p;
    }
    if (G == 64) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13c /* wave_ror:1 */, 0xf, 0xf, false);
    return (uint32_t)__shfl((int)v, pvl);
}

// Barrier of the workgroups that run the parts of one split realization (one
// workgroup alone: a workgroup barrier).  Every part arrives once per
// barrier on the realization's counter, so barrier n of the launch is passed
// when the counter reaches n * parts.  The arrival is a release and the wait
// an acquire at device scope, so the rows and save slots a part wrote before
// the barrier are visible to every part after it, on any XCD.  The parts of a
// realization are consecutive in the work queue and all of them are taken by
// a workgroup's first pop (the host puts them first and keeps their number
// within the grid), so the wait is for workgroups that are already running;
// it still gives up after a few hundred thousand polls (a fraction of a
// second), sets *err and then waits at none of its later barriers, so that
// no wait can outlive the launch by more than that.
struct PartSync {
    int32_t* ctr;   // the realization's counter, or nullptr for one part
    int32_t parts;
    int32_t count;  // barriers passed in this launch
    int32_t* err;
    bool broken;    // thread 0: a wait gave up
};

constexpr int32_t kSpinLimit = 1 << 18;

__device__ __forceinline__ void part_sync(PartSync& ps)
{
    __syncthreads();
    if (ps.ctr == nullptr) return;
    ps.count += 1;
    if (threadIdx.x == 0) {
        const int32_t target = ps.count * ps.parts;
        __hip_atomic_fetch_add(ps.ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (int32_t spin = 0;
             !ps.broken && __hip_atomic_load(ps.ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target;) {
            __builtin_amdgcn_s_sleep(1);
            if (++spin == kSpinLimit) {
                __hip_atomic_fetch_or(ps.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ps.broken = true;
            }
        }
    }
    __syncthreads();
}

// Temporally blocked passes (K MCS each) over a realization in global memory
// whose rows are G = W words (one word per lane of a G-lane group).  The
// workgroup's groups each sweep one band of bh rows with a register window of
// 2K+2 rows, as the single-lattice blocked kernel does, but in place.  A
// band's sweep reads the 2K rows above it and the 2K rows below it as they
// were at the start of the pass, while the neighbouring bands rewrite them;
// so each band also keeps copies of its first and of its last 2K rows as
// they were at the start of a pass, in two sets used in alternate passes, and
// its neighbours read those: during pass i a band reads set i&1 of its
// neighbours' copies and writes set (i+1)&1 of its own, from the registers
// that hold each row's final value.  Then one barrier per pass orders
// everything: it closes pass i-1's writes of set i&1 before pass i reads
// them, and pass i-1's reads of set (i+1)&1 before pass i overwrites it.
// (bh >= 8K keeps the two copied row ranges apart.)  Groups beyond the
// number of bands the lattice allows idle but take part in the barriers.  A
// realization split over several workgroups runs the same schedule with the
// barriers among all of its parts: this workgroup owns bands b0 ..
// b0+nbands-1 of nbt, and `save` holds the copies of all nbt bands.
template <int K, bool HASQ, Draws DR>
__device__ __forceinline__ void blocked_passes(SweepArgs a, uint64_t* S, uint64_t* save, uint32_t t0, int npass,
                                               int nbands, int b0, int nbt, PartSync& ps)
{
    constexpr int H = 2 * K, R = 2 * K + 1, NS = R + 1;
    const int G = a.W;  // lanes per row (a power of two, 8..64): a scalar, so that one copy of the
                        // per-lane set-up serves every row width
    const int g = threadIdx.x / G, gl = threadIdx.x & (G - 1);
    const bool g_first = gl == 0, g_last = gl == G - 1;
    const int lane = threadIdx.x & 63, gbase = lane & ~(G - 1);
    const int nxl = gbase | ((gl + 1) & (G - 1)), pvl = gbase | ((gl - 1) & (G - 1));
    const bool active = g < nbands;
    // Waves whose groups are all beyond the last band only take part in the
    // barriers.  The test is made a scalar value (readfirstlane), so that the
    // branch on it is a uniform jump.
    const bool wave_idle = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u) / G >= nbands ? 1 : 0) != 0;
    const int bh = a.Y / nbt;
    const int gb = b0 + g;  // the band's index in the realization
    const int y0 = gb * bh;
    const int ymask = a.Y - 1;
    const int64_t P = a.plane;
    const int nxt = (gb + 1) % nbt, prv = (gb + nbt - 1) % nbt;
    // Stores of groups beyond the last band (in a wave that also holds active
    // groups) go to an offset outside the buffers, which the buffer unit
    // drops; their loads read valid rows, so the sweep needs no per-group
    // branch.
    const int drop = active ? 0 : 0x7ffffff8;
    // Buffer descriptors for the four slope arrays and the copies (band b's
    // first (kind 0) and last (kind 1) 2K rows, set s, as [b][kind][s][j][c][G]:
    // nbt*32K*G words, within blocked_save_words per workgroup or part):
    // per-lane offsets stay 32-bit.
    const int32_t plane_bytes = (int32_t)(P * 8);
    __amdgpu_buffer_rsrc_t rs[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        rs[c] = __builtin_amdgcn_make_buffer_rsrc((void*)(S + c * P), (short)0, plane_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rsv =
        __builtin_amdgcn_make_buffer_rsrc((void*)save, (short)0, (int32_t)(nbt * 4 * H * 4 * G * 8), kBufferWord3);
    auto ld = [](__amdgpu_buffer_rsrc_t r, int off) -> uint64_t {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return (uint64_t)v[0] | ((uint64_t)v[1] << 32);
    };
    auto st = [](__amdgpu_buffer_rsrc_t r, int off, uint64_t w) {
        __attribute__((ext_vector_type(2))) uint32_t v;
        v[0] = (uint32_t)w;
        v[1] = (uint32_t)(w >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
    };
    auto cpoff = [&](int b, int kind, int set, int j, int c) -> int {
        return (((((b * 2 + kind) * 2 + set) * H + j) * 4 + c) * G + gl) * 8;
    };
    auto soff = [&](int rr) -> int { return (rr * G + gl) * 8; };

    // Set 0 of the copies: the band's rows as they are now.
    {
        uint64_t keep[2][H][4];  // all loads first, then all stores
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                keep[0][j][c] = ld(rs[c], soff((y0 + j) & ymask));
                keep[1][j][c] = ld(rs[c], soff((y0 + bh - H + j) & ymask));
            }
#pragma unroll
        for (int kind = 0; kind < 2; ++kind)
#pragma unroll
            for (int j = 0; j < H; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) st(rsv, cpoff(gb, kind, 0, j, c) | drop, keep[kind][j][c]);
    }
    part_sync(ps);

    for (int pass = 0; pass < npass; ++pass) {
        a.t = t0 + (uint32_t)(pass * K);
        const int rd = pass & 1, wr = rd ^ 1;
        uint64_t Wn[NS][4][1];
        // OddTail: a row's shared last draw, from its even half-step to its odd one
        constexpr bool TAIL = DR == Draws::OddTail;
        uint64_t tail[TAIL ? NS : 1][1];
        // Rows are addressed relative to the band start y0: the same for every
        // group at a given step, so the branches below are uniform and each
        // load keeps one buffer descriptor.  Rows above y0-2K feed no
        // half-step the band needs; the 2K rows above y0 come from the band
        // above's copy of its last rows, the 2K rows from y1 on from the band
        // below's copy of its first rows.
        auto load_step_row = [&](uint64_t (&row)[4][1], int rel) {  // rel >= -2K
            if (rel >= bh) {
#pragma unroll
                for (int c = 0; c < 4; ++c) row[c][0] = ld(rsv, cpoff(nxt, 0, rd, rel - bh, c));
            } else if (rel < 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) row[c][0] = ld(rsv, cpoff(prv, 1, rd, rel + H, c));
            } else {
                const int rr = (y0 + rel) & ymask;
#pragma unroll
                for (int c = 0; c < 4; ++c) row[c][0] = ld(rs[c], soff(rr));
            }
        };
        auto load_row = [&](uint64_t (&row)[4][1], int rel) {
            if (rel < -H) {
#pragma unroll
                for (int c = 0; c < 4; ++c) row[c][0] = 0ull;
            } else {
                load_step_row(row, rel);
            }
        };
        const int nsteps = bh + 2 * H - 1;
        // Step k holds relative row q+j (q = k-2H+1) in slot (u+j) mod NS,
        // u = k mod NS: the sweep is unrolled NS steps deep so that the window
        // rotates through the slots instead of being moved, and a step's rows
        // are shifted iff k is odd (the band start is even), known at compile
        // time in the unrolled steps.
        auto step = [&](auto U, int k) {
            constexpr int u = decltype(U)::value;
            auto sl = [](int j) { return (u + j) % NS; };
            if (k >= nsteps) {
                if constexpr (TAIL) {
                    // defined on this path too (no step runs after it: the sweep is
                    // over), so that no kept word lives across the loop
#pragma unroll
                    for (int h = 0; h < H; h += 2) tail[sl(H - 1 - h)][0] = 0;
                }
                return;
            }
            constexpr bool shifted = (u & 1) != 0;
            const int q = k - 2 * H + 1;      // this step's first window row, relative to y0
            // every step loads a row (the last ones reload the last row of the
            // copy, unused), so that the wait before a row's first use counts
            // the same memory operations on every path
            load_step_row(Wn[sl(H + 1)], min(q + 1 + H, bh + H - 1));
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int j = H - 1 - h;
                const int rel = q + j;
                const int par = h & 1;
                if (rel < -H + h) {
                    if constexpr (TAIL) {
                        if (par == 0) tail[sl(j)][0] = 0;  // defined on every path
                    }
                    continue;
                }
                const int rr = (y0 + rel) & ymask;
                SweepArgs ah = a;
                ah.parity = par;
                ah.t = a.t + (uint32_t)(h >> 1);
                // the row is one word per lane: the next word's bit 0 and the
                // previous word's top mask bit come from the neighbouring lanes of
                // the group, wrapping at the row end
                uint64_t(&D)[1] = Wn[sl(j)][1 - par];
                uint64_t XP[1], M[1], mp0 = 0, mq0 = 0;
                if constexpr (shifted) {
                    // x+ = D >> 1 with the next word's bit 0 on top
                    const uint32_t lo = (uint32_t)D[0], hi = (uint32_t)(D[0] >> 32);
                    const uint32_t nl = group_next(lo, G, g_last, nxl);
                    XP[0] = (uint64_t)__builtin_amdgcn_alignbit(hi, lo, 1u) |
                            ((uint64_t)__builtin_amdgcn_alignbit(nl, hi, 1u) << 32);
                } else {
                    XP[0] = D[0];
                }
                row_masks<1, 1, XiMode::Mask, HASQ, DR>(ah, rr, gl, Wn[sl(j)][par], Wn[sl(j)][2 + par],
                                                         Wn[sl(j + 1)][2 + (1 - par)], XP, M, mp0, mq0,
                                                         tail[TAIL ? sl(j) : 0]);
                if constexpr (shifted) {
                    // D ^= M << 1 with the previous word's top mask bit at the bottom
                    const uint32_t lo = (uint32_t)M[0], hi = (uint32_t)(M[0] >> 32);
                    const uint32_t ph = group_prev(hi, G, g_first, pvl);
                    D[0] ^= (uint64_t)__builtin_amdgcn_alignbit(lo, ph, 31u) |
                            ((uint64_t)__builtin_amdgcn_alignbit(hi, lo, 31u) << 32);
                } else {
                    D[0] ^= M[0];
                }
                // Pin the half-step's new slopes here, or the compiler sinks the
                // updates into later half-steps and keeps their masks live.
                asm volatile("" : "+v"(Wn[sl(j)][0][0]), "+v"(Wn[sl(j)][1][0]), "+v"(Wn[sl(j)][2][0]),
                             "+v"(Wn[sl(j)][3][0]), "+v"(Wn[sl(j + 1)][2 + (1 - par)][0]));
                if (par == 0 && rel == 0 && gb == 0 && gl == 0) {  // site (0,0); an atomic needs no wait
                    const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
                    if (dh != 0) atomicAdd((unsigned long long*)a.h0, (unsigned long long)dh);
                }
            }
            if (q >= 0) {  // row q has its value at the end of the pass
#pragma unroll
                for (int c = 0; c < 4; ++c) st(rs[c], soff(y0 + q) | drop, Wn[sl(0)][c][0]);
                if (q < H) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) st(rsv, cpoff(gb, 0, wr, q, c) | drop, Wn[sl(0)][c][0]);
                } else if (q >= bh - H) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) st(rsv, cpoff(gb, 1, wr, q - (bh - H), c) | drop, Wn[sl(0)][c][0]);
                }
            }
        };
        if (!wave_idle) {
#pragma unroll
            for (int j = 0; j < R; ++j) load_row(Wn[j], j - 2 * H + 1);
            for (int k = 0; k < nsteps; k += NS) unrolled_steps(step, k, std::make_integer_sequence<int, NS>{});
        }
        part_sync(ps);
    }
}

// K MCS per pass.  An even number of draws (or none) runs the passes
// compiled without the test for the shared last draw of an odd number; with
// TAIL (a kernel shape with registers to spare) an odd number without
// removals keeps that draw between a row's two half-steps (one Philox call
// per word and MCS for p = 1/2).
template <int K, bool TAIL>
__device__ __forceinline__ void blocked_k(const SweepArgs& a, uint64_t* S, uint64_t* save, uint32_t t0, int npass,
                                          int nbands, int b0, int nbt, bool has_q, PartSync& ps)
{
    const bool odd = (a.ndraw & 1) != 0;
    if (has_q) {
        if (odd) blocked_passes<K, true, Draws::Any>(a, S, save, t0, npass, nbands, b0, nbt, ps);
        else blocked_passes<K, true, Draws::Even>(a, S, save, t0, npass, nbands, b0, nbt, ps);
    } else {
        if (odd) blocked_passes<K, false, TAIL ? Draws::OddTail : Draws::Any>(a, S, save, t0, npass, nbands, b0, nbt,
                                                                              ps);
        else blocked_passes<K, false, Draws::Even>(a, S, save, t0, npass, nbands, b0, nbt, ps);
    }
}

// K <= MAXK MCS per pass.
template <int MAXK>
__device__ __forceinline__ void blocked_dispatch(const SweepArgs& a, uint64_t* S, uint64_t* save, uint32_t t0,
                                                 int npass, int nbands, int b0, int nbt, int K, bool has_q,
                                                 PartSync& ps)
{
    constexpr bool TAIL = MAXK >= 4;  // the 512-thread, one-per-CU shape
    if (K == 1) {
        blocked_k<1, TAIL>(a, S, save, t0, npass, nbands, b0, nbt, has_q, ps);
    } else if (MAXK < 3 || K == 2) {
        blocked_k<2, TAIL>(a, S, save, t0, npass, nbands, b0, nbt, has_q, ps);
    } else if constexpr (MAXK >= 4) {
        if (K == 3) blocked_k<3, TAIL>(a, S, save, t0, npass, nbands, b0, nbt, has_q, ps);
        else blocked_k<4, TAIL>(a, S, save, t0, npass, nbands, b0, nbt, has_q, ps);
    }
}

__device__ __forceinline__ SweepArgs args_of(const BatchDesc& d)
{
    SweepArgs a{};
    a.plane = d.plane;
    a.W = d.W;
    a.Y = d.Y;
    a.nb = d.nb;
    a.k0 = d.k0;
    a.k1 = d.k1;
    a.dig_p = d.dig_p;
    a.dig_q = d.dig_q;
    a.ndraw = d.ndraw;
    a.all_p = d.all_p;
    a.all_q = d.all_q;
    a.thr_p = d.thr_p;
    a.thr_q = d.thr_q;
    a.h0 = d.h0;
    return a;
}

// The descriptor of an item, moved into scalar registers: it is the same for
// the whole workgroup, and buffer descriptors built from it must be uniform.
// *part receives the item's part of a split realization.
__device__ __forceinline__ BatchDesc load_desc(const BatchLaunch& L, int32_t item, int32_t* part)
{
    static_assert(sizeof(BatchDesc) % 4 == 0, "descriptor of whole dwords");
    const int32_t code = __builtin_amdgcn_readfirstlane(L.order[item]);
    *part = code >> kItemSlotBits;
    const BatchDesc d = L.desc[code & ((1 << kItemSlotBits) - 1)];
    uint32_t w[sizeof(BatchDesc) / 4];
    __builtin_memcpy(w, &d, sizeof(BatchDesc));
#pragma unroll
    for (unsigned i = 0; i < sizeof(BatchDesc) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    BatchDesc u;
    __builtin_memcpy(&u, w, sizeof(BatchDesc));
    return u;
}

// The next item of the work queue, the same for the whole workgroup.
__device__ __forceinline__ int32_t next_item(int32_t* queue, int32_t* s_item)
{
    __syncthreads();  // the previous realization is finished (LDS and s_item reuse)
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
    __syncthreads();
    // uniform: the descriptor then loads into scalar registers
    return __builtin_amdgcn_readfirstlane(*s_item);
}

// MAXK: the deepest blocked pass compiled in (its register window decides
// how many workgroups a CU holds: 2 fits 1024-thread workgroups, 4 one
// 512-thread workgroup per CU).
template <int BLOCK, int IW, int MAXK>
__global__ __launch_bounds__(BLOCK) void ensemble_kernel(BatchLaunch L)
{
    constexpr int NWAVES = BLOCK / 64;
    extern __shared__ uint64_t lds[];
    __shared__ int32_t s_item;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t n_items = *L.n_items;

    // Phase 1: realizations that run as temporally blocked passes (the host
    // orders them first, split realizations at the head): passes of d.depth
    // MCS, and one of a single MCS for an odd remainder.  The first other
    // item moves the workgroup on to phase 2, which handles any realization.
    // Keeping the two loops apart keeps their register needs apart.
    int32_t item = next_item(L.queue, &s_item);
    while (item < n_items) {
        int32_t part = 0;
        const BatchDesc d = load_desc(L, item, &part);
        if (d.depth <= 0) break;
        if (d.n_run > 0) {
            const SweepArgs a = args_of(d);
            const bool has_q = d.has_q != 0;
            uint64_t* save = d.parts > 1 ? d.save : L.save + (int64_t)blockIdx.x * L.save_words;
            PartSync ps{d.parts > 1 ? L.sync + d.sync_idx : nullptr, d.parts, 0, L.err, false};
            const int nbt = d.bands * d.parts, b0 = part * d.bands;
            const int npass = (int)(d.n_run / (uint32_t)d.depth);
            if (npass > 0) blocked_dispatch<MAXK>(a, d.S, save, d.t, npass, d.bands, b0, nbt, d.depth, has_q, ps);
            const uint32_t done = (uint32_t)npass * (uint32_t)d.depth;
            if (done < d.n_run)
                blocked_dispatch<MAXK>(a, d.S, save, d.t + done, (int)(d.n_run - done), d.bands, b0, nbt, 1, has_q,
                                       ps);
        }
        item = next_item(L.queue, &s_item);
    }

    // Phase 2: every other realization, half-step by half-step, in LDS or in
    // the arena.
    for (; item < n_items; item = next_item(L.queue, &s_item)) {
        int32_t part = 0;
        const BatchDesc d = load_desc(L, item, &part);
        if (d.n_run == 0) continue;
        SweepArgs a = args_of(d);
        const bool has_q = d.has_q != 0;
        const int64_t words = 4 * d.plane;
        const bool in_lds = d.W <= 8 && words * 8 <= (int64_t)L.lds_bytes;

        if (in_lds) {
            for (int64_t i = threadIdx.x; i < words; i += BLOCK) lds[i] = d.S[i];
            __syncthreads();
            for (uint32_t m = 0; m < d.n_run; ++m) {
                a.t = d.t + m;
                for (int par = 0; par < 2; ++par) {
                    a.parity = par;
                    halfstep_lds<NWAVES, IW>(a, lds, d.mode, has_q, wave, lane);
                    __syncthreads();
                }
            }
            for (int64_t i = threadIdx.x; i < words; i += BLOCK) d.S[i] = lds[i];
        } else {
            for (uint32_t m = 0; m < d.n_run; ++m) {
                a.t = d.t + m;
                for (int par = 0; par < 2; ++par) {
                    a.parity = par;
                    halfstep_global<NWAVES, IW>(a, d.S, d.mode, has_q, wave, lane);
                    __syncthreads();
                }
            }
        }
    }
}

// Zeroes the work counter and the split realizations' barrier counters.
__global__ void counter_reset_kernel(int32_t* c, int32_t* sync, int32_t n_sync)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) *c = 0;
    if (i < n_sync) sync[i] = 0;
}

// The kernel instantiation of a configuration: passes of up to 2 MCS for
// every shape, of up to 4 MCS for one 512-thread workgroup per CU.
template <class F>
hipError_t with_ensemble_kernel(int block_threads, int words_per_lane, int depth, F&& f)
{
    if (depth > 2) {
        if (block_threads != 512) return hipErrorInvalidValue;
        if (words_per_lane == 1) return f(ensemble_kernel<512, 1, 4>);
        if (words_per_lane == 2) return f(ensemble_kernel<512, 2, 4>);
        return hipErrorInvalidValue;
    }
    switch (block_threads * 4 + words_per_lane) {
    case 256 * 4 + 1: return f(ensemble_kernel<256, 1, 2>);
    case 512 * 4 + 1: return f(ensemble_kernel<512, 1, 2>);
    case 1024 * 4 + 1: return f(ensemble_kernel<1024, 1, 2>);
    case 256 * 4 + 2: return f(ensemble_kernel<256, 2, 2>);
    case 512 * 4 + 2: return f(ensemble_kernel<512, 2, 2>);
    case 1024 * 4 + 2: return f(ensemble_kernel<1024, 2, 2>);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_ensemble(const BatchLaunch& L, int block_threads, int words_per_lane, int grid, hipStream_t stream)
{
    const size_t lds = (size_t)L.lds_bytes;
    return with_ensemble_kernel(block_threads, words_per_lane, L.depth, [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block_threads), lds, stream, L);
        return hipGetLastError();
    });
}

int ensemble_occupancy(int block_threads, int words_per_lane, int lds_bytes, int depth)
{
    int n = 0;
    const size_t lds = (size_t)lds_bytes;
    const hipError_t e = with_ensemble_kernel(block_threads, words_per_lane, depth, [&](auto kernel) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block_threads, lds);
    });
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

hipError_t launch_counter_reset(int32_t* counter, int32_t* sync, int32_t n_sync, hipStream_t stream)
{
    const int n = n_sync > 1 ? n_sync : 1;
    hipLaunchKernelGGL(counter_reset_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, counter, sync,
                       n_sync);
    return hipGetLastError();
}

}  // namespace sca

// halfstep.hpp -- the bit-vectorized half-step of one row group, shared by the
// single-lattice kernel (sweep.hip) and the persistent ensemble kernel
// (batch.hip), so that both compute exactly the same function.
//
// One half-step updates every site of one checkerboard sublattice (Sec. I-A).
// Sites of the same sublattice share no bond, so the whole sublattice is
// updated at once with bitwise operations on 64 sites per word (Sec. II-B,
// Fig. 3; the mask of Eqs. (3)-(5)):
//
//   m_p = xi_p & ~x- & ~y- &  x+ &  y+        (local minima, accepted w.p. p)
//   m_q = xi_q &  x- &  y- & ~x+ & ~y+        (local maxima, accepted w.p. q)
//   m   = m_p | m_q                           (disjoint, so xor == or)
//
// and m is xored into the four slope words of the updated sites.
//
// A row of W words is held by a group of G lanes of one wavefront, I words
// per lane (word w = i*G + lane-in-group).  The only cross-word traffic -- bit 0
// of the next x+ word when the row's x+ neighbours are shifted by one site,
// and the top bit of the previous word's mask on the way back -- stays inside
// the wave: one 32-bit lane shuffle per direction carries that bit for all I
// slots of a lane, and the periodic wrap of the row is a rotation of those
// packed bits.  For G == I == 1 (X <= 128) a lane owns a whole row and rotates
// within the nb used bits.
//
// Row parity: the x+ neighbour of the site in bit k of row y is the site in
// bit k of the other sublattice's x-array when the row's sites of this parity
// have even x, and in bit k+1 when they have odd x, i.e. when
// parity ^ (y & 1) == 1 (the paper's aligned / shifted rows, Sec. II-B).
#pragma once

#include "philox.hpp"
#include "sweep_args.hpp"

namespace sca {

// One step of the and/or fold, acc <- b ? (R | acc) : (R & acc): the
// majority of R, acc and the digit spread over the word (an all-ones or
// all-zero scalar), one v_bitop3_b32 (truth table 0xE8) per 32-bit half.
__device__ __forceinline__ uint64_t fold_digit(uint64_t r, uint64_t acc, uint32_t b)
{
    const uint32_t m = b ? ~0u : 0u;
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)r, (uint32_t)acc, m, 0xE8);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(r >> 32), (uint32_t)(acc >> 32), m, 0xE8);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// What a mask-mode caller knows of the number n of draws at compile time:
// nothing (Any), that n is even (Even), or that n is odd and it keeps one
// word per row between the row's two half-steps (OddTail).
enum class Draws : int { Any = 0, Even = 1, OddTail = 2 };

// Acceptance words for canonical word g, mask mode: the and/or fold of
// n = ndraw draws, least significant binary digit first, generated from the
// last Philox call backwards so that only one call's output is live.  Call j
// has the counter (g, t, 2j + parity, 0) and gives draws 2j and 2j+1, except
// that for odd n the last draw of both half-steps of the MCS comes from the
// one call (g, t, n-1, 0): lanes 0|1 in the even half-step, 2|3 in the odd
// one.  OddTail: the even half-step leaves lanes 2|3 of that call in *tail
// and the odd one takes its draw from there instead of calling again.
template <Draws D = Draws::Any>
__device__ __forceinline__ void mask_words(const SweepArgs& a, uint32_t g, bool has_q, uint64_t& xp, uint64_t& xq,
                                           uint64_t* tail = nullptr)
{
    uint64_t ap = 0, aq = 0;
    auto fold = [&](uint64_t r, int d) {  // draw d, digit b_{d+1}
        ap = fold_digit(r, ap, (a.dig_p >> d) & 1u);
        if (has_q) aq = fold_digit(r, aq, (a.dig_q >> d) & 1u);
    };
    int j = ((a.ndraw + 1) >> 1) - 1;  // the last call
    if constexpr (D == Draws::OddTail) {
        // n = 2j+1: the shared last draw first
        uint64_t r;
        if (a.parity == 1) {
            r = *tail;
        } else {
            const u32x4 o = philox4x32_10(g, a.t, 2u * (uint32_t)j, 0u, a.k0, a.k1);
            r = (uint64_t)o.v0 | ((uint64_t)o.v1 << 32);
            *tail = (uint64_t)o.v2 | ((uint64_t)o.v3 << 32);
        }
        fold(r, 2 * j);
        --j;
    }
    const bool odd = D == Draws::Any && (a.ndraw & 1) != 0;
    for (; j >= 0; --j) {
        const bool shared = odd && 2 * j + 1 == a.ndraw;  // the odd last draw: counter n-1 in both half-steps
        const u32x4 o = philox4x32_10(g, a.t, 2u * (uint32_t)j + (shared ? 0u : (uint32_t)a.parity), 0u, a.k0, a.k1);
        const uint64_t lo = (uint64_t)o.v0 | ((uint64_t)o.v1 << 32);
        const uint64_t hi = (uint64_t)o.v2 | ((uint64_t)o.v3 << 32);
        // apart from the shared draw every call gives two
        if (D != Draws::Any || 2 * j + 1 < a.ndraw) fold(hi, 2 * j + 1);
        fold((shared && a.parity == 1) ? hi : lo, 2 * j);
    }
    xp = ap | a.all_p;
    xq = has_q ? (aq | a.all_q) : 0;
}

// Acceptance words, per-site mode: site bit b compares lane b&3 of call b>>2.
__device__ __forceinline__ void persite_words(const SweepArgs& a, uint32_t g, bool has_q, uint64_t& xp,
                                              uint64_t& xq)
{
    uint32_t lo_p = 0, hi_p = 0, lo_q = 0, hi_q = 0;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const u32x4 o = philox4x32_10(g, a.t, 2u * (uint32_t)j + (uint32_t)a.parity, 0u, a.k0, a.k1);
        const uint32_t bits_p = (uint32_t)(o.v0 < a.thr_p) | ((uint32_t)(o.v1 < a.thr_p) << 1) |
                                ((uint32_t)(o.v2 < a.thr_p) << 2) | ((uint32_t)(o.v3 < a.thr_p) << 3);
        if (j < 8) lo_p |= bits_p << (4 * j); else hi_p |= bits_p << (4 * (j - 8));
        if (has_q) {
            const uint32_t bits_q = (uint32_t)(o.v0 < a.thr_q) | ((uint32_t)(o.v1 < a.thr_q) << 1) |
                                    ((uint32_t)(o.v2 < a.thr_q) << 2) | ((uint32_t)(o.v3 < a.thr_q) << 3);
            if (j < 8) lo_q |= bits_q << (4 * j); else hi_q |= bits_q << (4 * (j - 8));
        }
    }
    xp = ((uint64_t)lo_p | ((uint64_t)hi_p << 32)) | a.all_p;
    xq = has_q ? (((uint64_t)lo_q | ((uint64_t)hi_q << 32)) | a.all_q) : 0;
}

// Any bitwise function of three words in one gfx950 v_bitop3_b32 per half:
// bit (a<<2 | b<<1 | c) of T is the result for input bits a, b, c.
template <unsigned T>
__device__ __forceinline__ uint64_t bitop3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, T);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), T);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Lane i of the wavefront receives v from lane (i+1) mod 64, resp. (i-1) mod
// 64: DPP wavefront rotates, a VALU operation with no LDS round trip.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134 /* wave_rol:1 */, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13c /* wave_ror:1 */, 0xf, 0xf, false);
}

template <int N>
__device__ __forceinline__ uint32_t rot_down(uint32_t v)  // bit i <- bit (i+1) mod N
{
    if constexpr (N == 1) return v;
    constexpr uint32_t mask = (N == 32) ? 0xffffffffu : ((1u << N) - 1u);
    return ((v >> 1) | (v << (N - 1))) & mask;
}

template <int N>
__device__ __forceinline__ uint32_t rot_up(uint32_t v)  // bit i <- bit (i-1) mod N
{
    if constexpr (N == 1) return v;
    constexpr uint32_t mask = (N == 32) ? 0xffffffffu : ((1u << N) - 1u);
    return ((v << 1) | (v >> (N - 1))) & mask;
}

// x+ slopes aligned with the sites of a row: D holds the other sublattice's
// x-slopes of the same row (slot i = word i*G + gl).  In shifted rows bit k
// takes bit k+1, crossing into the next word (next lane, or slot i+1 of the
// group's first lane, wrapping at the row end).  All lanes of the wave call
// this together (lane shuffle).
template <int G, int I>
__device__ __forceinline__ void align_xplus(const uint64_t (&D)[I], bool shifted, int gl, int gbase, int nb,
                                            uint64_t (&XP)[I])
{
    if constexpr (G == 1 && I == 1) {
        XP[0] = shifted ? ((D[0] >> 1) | ((D[0] & 1ull) << (nb - 1))) : D[0];
    } else {
        uint32_t lsb = 0;  // bit i: bit 0 of this lane's slot-i word
#pragma unroll
        for (int i = 0; i < I; ++i) lsb |= (uint32_t)(D[i] & 1ull) << i;
        uint32_t nxt = lsb;
        if constexpr (G == 64) nxt = from_next_lane(lsb);
        else if constexpr (G > 1) nxt = (uint32_t)__shfl((int)lsb, gbase | ((gl + 1) & (G - 1)));
        // The last lane of the group continues in slot i+1 of the first lane.
        if (gl == G - 1) nxt = rot_down<I>(nxt);
#pragma unroll
        for (int i = 0; i < I; ++i)
            XP[i] = shifted ? ((D[i] >> 1) | ((uint64_t)((nxt >> i) & 1u) << 63)) : D[i];
    }
}

// Applies the update mask to the x+ slopes D; in shifted rows bit k of m
// belongs to bit k+1 (the top bit of a word to bit 0 of the next word).  All
// lanes of the wave call this together.
template <int G, int I>
__device__ __forceinline__ void apply_xplus(uint64_t (&D)[I], const uint64_t (&M)[I], bool shifted, int gl, int gbase,
                                            int nb)
{
    if constexpr (G == 1 && I == 1) {
        const uint64_t valid = (nb == 64) ? ~0ull : ((1ull << nb) - 1ull);
        D[0] ^= shifted ? (((M[0] << 1) | (M[0] >> (nb - 1))) & valid) : M[0];
    } else {
        uint32_t msb = 0;  // bit i: top bit of this lane's slot-i mask
#pragma unroll
        for (int i = 0; i < I; ++i) msb |= (uint32_t)(M[i] >> 63) << i;
        uint32_t prv = msb;
        if constexpr (G == 64) prv = from_prev_lane(msb);
        else if constexpr (G > 1) prv = (uint32_t)__shfl((int)msb, gbase | ((gl - 1) & (G - 1)));
        // The first lane of the group continues from slot i-1 of the last lane.
        if (gl == 0) prv = rot_up<I>(prv);
#pragma unroll
        for (int i = 0; i < I; ++i)
            D[i] ^= shifted ? ((M[i] << 1) | (uint64_t)((prv >> i) & 1u)) : M[i];
    }
}

// Update masks of row y (Eqs. (3)-(5)) from the on-site x- and y- slopes A,
// B, the y+ slopes C and the aligned x+ slopes XP, with the acceptance words
// of sublattice a.parity at MCS a.t; A, B, C are updated in place.  mp0 and
// mq0 return the slot-0 masks (the origin lives in bit 0 of slot 0, lane 0).
// D: what the caller knows of the number of draws (mask_words); with
// Draws::OddTail, tail holds the I words that carry the shared last draw from
// the row's even half-step to its odd one.
template <int G, int I, XiMode MODE, bool HASQ, Draws D = Draws::Any>
__device__ __forceinline__ void row_masks(const SweepArgs& a, int64_t y, int gl, uint64_t (&A)[I], uint64_t (&B)[I],
                                          uint64_t (&C)[I], const uint64_t (&XP)[I], uint64_t (&M)[I],
                                          uint64_t& mp0, uint64_t& mq0, uint64_t* tail = nullptr)
{
#pragma unroll
    for (int i = 0; i < I; ++i) {
        const uint32_t g = (uint32_t)(y * a.W + i * G + gl);
        uint64_t xip, xiq;
        if constexpr (MODE == XiMode::Mask) {
            mask_words<D>(a, g, HASQ, xip, xiq, D == Draws::OddTail ? tail + i : nullptr);
        } else if constexpr (MODE == XiMode::PerSite) {
            persite_words(a, g, HASQ, xip, xiq);
        } else if constexpr (MODE == XiMode::Fixed) {
            xip = a.all_p;
            xiq = a.all_q;
        } else {
            xip = a.xi_p[g];
            xiq = a.xi_q[g];
        }
        const uint64_t mp = bitop3<0x80>(bitop3<0x02>(A[i], B[i], XP[i]), C[i], xip);  // xi & ~A & ~B & XP & C
        const uint64_t mq = HASQ ? bitop3<0x20>(bitop3<0x40>(A[i], B[i], XP[i]), C[i], xiq)  // xi & A & B & ~XP & ~C
                                 : 0ull;
        if (i == 0) { mp0 = mp; mq0 = mq; }
        M[i] = mp | mq;
        A[i] ^= M[i];
        B[i] ^= M[i];
        C[i] ^= M[i];
    }
}

// One half-step of row y for the lanes of one row group.  S is the base of
// S[2][2][Y][W] (global or LDS); every lane of the wave must call this
// together (lane shuffles); lanes of a group with y_raw >= Y load row 0 and
// store nothing.
template <int G, int I, XiMode MODE, bool HASQ>
__device__ __forceinline__ void halfstep_rows(const SweepArgs& a, uint64_t* S, int64_t y_raw, int lane)
{
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "G must be a power of two <= 64");
    static_assert(I >= 1 && I <= 32, "I words per lane");
    const int gl = lane & (G - 1);      // lane within the row group
    const int gbase = lane & ~(G - 1);  // first lane of the row group
    const bool active = y_raw < a.Y;    // uniform within a row group
    const int64_t y = active ? y_raw : 0;
    const int64_t yn = (y + 1) & (a.Y - 1);
    const int par = a.parity;
    const bool shifted = ((par ^ (int)(y & 1)) != 0);

    uint64_t* const sxP = S + (int64_t)(0 * 2 + par) * a.plane + y * a.W;        // x-, this parity
    uint64_t* const syP = S + (int64_t)(1 * 2 + par) * a.plane + y * a.W;        // y-, this parity
    uint64_t* const syQ = S + (int64_t)(1 * 2 + (1 - par)) * a.plane + yn * a.W; // y+ (row y+1)
    uint64_t* const sxQ = S + (int64_t)(0 * 2 + (1 - par)) * a.plane + y * a.W;  // x+ (same row)

    uint64_t A[I], B[I], C[I], D[I];
#pragma unroll
    for (int i = 0; i < I; ++i) {
        const int w = i * G + gl;
        A[i] = sxP[w];
        B[i] = syP[w];
        C[i] = syQ[w];
        D[i] = sxQ[w];
    }
    uint64_t XP[I], M[I];
    uint64_t mp0 = 0, mq0 = 0;
    align_xplus<G, I>(D, shifted, gl, gbase, a.nb, XP);
    row_masks<G, I, MODE, HASQ>(a, y, gl, A, B, C, XP, M, mp0, mq0);
    apply_xplus<G, I>(D, M, shifted, gl, gbase, a.nb);

    if (active) {
#pragma unroll
        for (int i = 0; i < I; ++i) {
            const int w = i * G + gl;
            sxP[w] = A[i];
            syP[w] = B[i];
            syQ[w] = C[i];
            sxQ[w] = D[i];
        }
        // Site (0,0) is bit 0 of word 0 of row 0 in the even sublattice (one
        // lane; an atomic add needs no wait for the old value).
        if (par == 0 && y == 0 && gl == 0) {
            const int64_t dh = 2 * (int64_t)(mp0 & 1ull) - 2 * (int64_t)(mq0 & 1ull);
            if (dh != 0) atomicAdd((unsigned long long*)a.h0, (unsigned long long)dh);
        }
    }
}

}  // namespace sca

// sweep_args.hpp -- the arguments of one half-step (or of a blocked pass).
#pragma once

#include <stdint.h>

namespace sca {

// How the acceptance words of a half-step are produced.
enum class XiMode : int {
    Mask = 0,     // dyadic p, q: and/or fold of n 64-bit draws (Sec. III)
    PerSite = 1,  // one 32-bit uniform per site against floor(r*2^32) (Sec. II-B)
    Inject = 2,   // read from caller arrays (test hook)
    Fixed = 3,    // p, q in {0, 1}: xi is all ones or zero, no draws
};

// Everything a half-step launch needs; passed by value as the kernel argument.
struct SweepArgs {
    uint64_t* S;       // S[2][2][Y][W]
    int64_t plane;     // Y*W words per (direction, parity) array
    int32_t W;         // words per row and sublattice
    int32_t Y;         // rows
    int32_t nb;        // used bits per word: 64, or X/2 when X < 128
    int32_t parity;    // sublattice: 0 even, 1 odd
    uint32_t t;        // MCS index (Philox counter word 1)
    uint32_t k0, k1;   // Philox key
    // Mask mode: bit i-1 of dig_* is binary digit b_i of p or q; ndraw = n;
    // all_* = ~0 when the probability is exactly 1.
    uint32_t dig_p, dig_q;
    int32_t ndraw;
    uint64_t all_p, all_q;
    // PerSite mode: thresholds clamped to 32 bits; all_* as above for r == 1.
    uint32_t thr_p, thr_q;
    // Inject mode.
    const uint64_t* xi_p;
    const uint64_t* xi_q;
    int64_t* h0;       // origin height h(0,0), updated by the lane owning site (0,0)
};

}  // namespace sca

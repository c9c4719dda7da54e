/*
 * bitsweep.c -- a multithreaded, bit-vectorized CPU sweep of the octahedron
 * SCA with 64-bit words: the CPU side of a like-for-like GPU/CPU comparison
 * (the paper compares its GPU kernel with a bit-vectorized CPU code using
 * 64-bit words and one thread per hardware thread, Sec. II-B, Sec. III).
 *
 * It is neither the GPU library nor the test oracle and shares no code with
 * either.  The state is the GPU library's packed layout, so results can be
 * compared word for word:
 *   uint64 S[2][2][Y][W], W = max(1, X/128); S[d][pi][y][w], d = 0 x-slopes,
 *   d = 1 y-slopes, pi = (x+y)&1; bit b of word w is the site of row y with
 *   x>>1 == 64*w + b.  A set bit: the height rises by one across that bond
 *   from the left (x) or lower (y) neighbour.  X < 128 uses bits 0..X/2-1.
 *
 * Half-step pi of row y (Eqs. (3)-(5)): A = S[0][pi][y], B = S[1][pi][y] are
 * the site's own x- and y- slopes, C = S[1][1-pi][y+1] its y+ slopes and the
 * x+ slopes are S[0][1-pi][y], bit for bit when the row's pi-sites have even
 * x, one bit further (across the word edge, periodic at the row end) when
 * they have odd x (Fig. 3).  Minima ~A ~B x+ C accepted by xi_p and maxima
 * A B ~x+ ~C accepted by xi_q flip all four slopes.  Same-parity sites share
 * no bond, so the rows of one half-step are independent and are split over
 * OpenMP threads.
 *
 * Acceptance words: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed,
 * counter (g, t, 2j+pi, 0) for call j of canonical word g = y*W + w in
 * half-step pi of MCS t.  Dyadic p, q: the 64-bit draws (lanes 0|1 then 2|3
 * of each call) folded from the last binary digit to the first, "or" for a
 * 1 digit and "and" for a 0 (Sec. III); with an odd number n of draws the
 * last one comes from the call (g, t, n-1, 0) in both half-steps of the MCS,
 * lanes 0|1 in the even one and 2|3 in the odd one, which takes them from a
 * per-word copy the even half-step left (p = 1/2: one call per word and
 * MCS).  Any other p or q: site b accepts iff lane b&3 of call b>>2 is below
 * floor(r * 2^32) (Sec. II-B).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define API __attribute__((visibility("default")))

enum { BS_OK = 0, BS_EINVAL = -1, BS_ENOMEM = -2 };

/* Philox4x32-10: ten rounds; each round multiplies counter words 0 and 2 by
 * the published multipliers, mixes the halves with the other two words and
 * the round key, and the key advances by the published Weyl increments. */
static inline void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                            uint32_t o[4])
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o[0] = c0;
    o[1] = c1;
    o[2] = c2;
    o[3] = c3;
}

API void bs_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

/* How one probability turns into acceptance bits. */
typedef struct {
    int all;        /* r == 1 */
    int ndig;       /* dyadic: number of binary digits (0 for r = 0 or 1) */
    uint32_t bits;  /* dyadic: digit i (i = 1..ndig) in bit i-1 */
    uint32_t thr;   /* per-site threshold floor(r * 2^32) (r < 1) */
    int dyadic;
} accept_t;

static int accept_make(double r, accept_t* a)
{
    if (!(r >= 0.0 && r <= 1.0)) return BS_EINVAL;
    memset(a, 0, sizeof *a);
    const double s = ldexp(r, 32);
    const double f = floor(s);
    a->all = (r == 1.0);
    a->dyadic = (f == s);
    a->thr = a->all ? 0xFFFFFFFFu : (uint32_t)f;
    if (a->dyadic && !a->all) {
        const uint32_t v = (uint32_t)f;
        for (int i = 1; i <= 32; ++i)
            if ((v >> (32 - i)) & 1u) {
                a->bits |= 1u << (i - 1);
                a->ndig = i;
            }
    }
    return BS_OK;
}

typedef struct {
    int64_t X, Y;
    int W, nb;          /* words per row, used bits per word */
    uint64_t valid;     /* used bits of a word */
    uint32_t k0, k1;
    accept_t P, Q;
    int persite, ndraw;
    uint64_t* tail;     /* odd ndraw: per canonical word, lanes 2|3 of the shared last call */
} sweep_t;

/* Acceptance words of canonical word g, half-step pi, MCS t. */
static inline void accept_words(const sweep_t* s, uint32_t g, uint32_t t, int pi, uint64_t* xp, uint64_t* xq)
{
    uint32_t o[4];
    if (s->persite) {
        uint64_t wp = 0, wq = 0;
        for (int j = 0; j < 16; ++j) {
            philox10(g, t, (uint32_t)(2 * j + pi), 0u, s->k0, s->k1, o);
            for (int l = 0; l < 4; ++l) {
                const uint64_t bit = (uint64_t)1 << (4 * j + l);
                if (s->P.all || o[l] < s->P.thr) wp |= bit;
                if (s->Q.all || o[l] < s->Q.thr) wq |= bit;
            }
        }
        *xp = wp;
        *xq = wq;
        return;
    }
    uint64_t d[32];
    const int pairs = s->ndraw & ~1;
    for (int i = 0; i < pairs; i += 2) {
        philox10(g, t, (uint32_t)(i + pi), 0u, s->k0, s->k1, o);  /* call j = i/2: counter 2j + pi */
        d[i] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        d[i + 1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    }
    if (s->ndraw & 1) {
        if (pi == 0) {
            philox10(g, t, (uint32_t)pairs, 0u, s->k0, s->k1, o);  /* counter n-1, both half-steps */
            d[pairs] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
            s->tail[g] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
        } else {
            d[pairs] = s->tail[g];
        }
    }
    uint64_t ap = s->P.all ? ~(uint64_t)0 : 0, aq = s->Q.all ? ~(uint64_t)0 : 0;
    for (int i = s->ndraw; i >= 1; --i) {
        if (!s->P.all && i <= s->P.ndig) ap = ((s->P.bits >> (i - 1)) & 1u) ? (d[i - 1] | ap) : (d[i - 1] & ap);
        if (!s->Q.all && i <= s->Q.ndig) aq = ((s->Q.bits >> (i - 1)) & 1u) ? (d[i - 1] | aq) : (d[i - 1] & aq);
    }
    *xp = ap;
    *xq = aq;
}

/* Half-step pi of row y.  Returns the origin height change (row 0, pi 0). */
static int64_t row_halfstep(const sweep_t* s, uint64_t* S, int64_t y, int pi, uint32_t t)
{
    const int64_t plane = s->Y * s->W;
    const int W = s->W;
    uint64_t* A = S + (0 * 2 + pi) * plane + y * W;
    uint64_t* B = S + (1 * 2 + pi) * plane + y * W;
    uint64_t* C = S + (1 * 2 + (1 - pi)) * plane + ((y + 1) & (s->Y - 1)) * W;
    uint64_t* D = S + (0 * 2 + (1 - pi)) * plane + y * W;
    const int shifted = (pi ^ (int)(y & 1)) != 0;
    int64_t dh = 0;
    if (W == 1 && s->nb < 64) {
        /* one partial word: the x+ neighbours rotate within nb bits */
        const int nb = s->nb;
        uint64_t xi_p, xi_q;
        accept_words(s, (uint32_t)y, t, pi, &xi_p, &xi_q);
        const uint64_t d = D[0];
        const uint64_t xpl = shifted ? ((d >> 1) | ((d & 1u) << (nb - 1))) : d;
        const uint64_t mp = xi_p & ~A[0] & ~B[0] & xpl & C[0];
        const uint64_t mq = xi_q & A[0] & B[0] & ~xpl & ~C[0] & s->valid;
        const uint64_t m = mp | mq;
        A[0] ^= m;
        B[0] ^= m;
        C[0] ^= m;
        D[0] ^= shifted ? (((m << 1) | (m >> (nb - 1))) & s->valid) : m;
        if (y == 0 && pi == 0) dh = 2 * (int64_t)(mp & 1u) - 2 * (int64_t)(mq & 1u);
        return dh;
    }
    const uint64_t d0 = D[0];  /* bit 0 of word 0 before this half-step, for the row end */
    uint64_t carry = 0;        /* the previous word's mask bit 63 */
    for (int w = 0; w < W; ++w) {
        uint64_t xi_p, xi_q;
        accept_words(s, (uint32_t)(y * W + w), t, pi, &xi_p, &xi_q);
        const uint64_t next0 = (w + 1 < W) ? (D[w + 1] & 1u) : (d0 & 1u);
        const uint64_t xpl = shifted ? ((D[w] >> 1) | (next0 << 63)) : D[w];
        const uint64_t mp = xi_p & ~A[w] & ~B[w] & xpl & C[w];
        const uint64_t mq = xi_q & A[w] & B[w] & ~xpl & ~C[w];
        const uint64_t m = mp | mq;
        A[w] ^= m;
        B[w] ^= m;
        C[w] ^= m;
        if (shifted) {
            D[w] ^= (m << 1) | carry;
            carry = m >> 63;
        } else {
            D[w] ^= m;
        }
        if (y == 0 && pi == 0 && w == 0) dh = 2 * (int64_t)(mp & 1u) - 2 * (int64_t)(mq & 1u);
    }
    if (shifted) D[0] ^= carry;  /* the row end wraps to site 0 */
    return dh;
}

/* Advances the packed state S (4*Y*W words) by n MCS from MCS t0 with p, q
 * and seed; *h0 is the height of site (0,0), updated in place.  The rows of
 * each half-step are split over the OpenMP threads. */
API int bs_sweep(uint64_t* S, int64_t X, int64_t Y, uint64_t seed, int64_t t0, int64_t n, double p, double q,
                 int64_t* h0)
{
    if (!S || !h0 || X < 4 || Y < 4 || X > (1 << 17) || Y > (1 << 17) || (X & (X - 1)) || (Y & (Y - 1)) ||
        t0 < 0 || n < 0 || t0 + n > (int64_t)UINT32_MAX)
        return BS_EINVAL;
    sweep_t s;
    memset(&s, 0, sizeof s);
    if (accept_make(p, &s.P) || accept_make(q, &s.Q)) return BS_EINVAL;
    s.X = X;
    s.Y = Y;
    s.W = X >= 128 ? (int)(X / 128) : 1;
    s.nb = X >= 128 ? 64 : (int)(X / 2);
    s.valid = s.nb == 64 ? ~(uint64_t)0 : (((uint64_t)1 << s.nb) - 1);
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    s.persite = !s.P.dyadic || !s.Q.dyadic;
    s.ndraw = s.P.ndig > s.Q.ndig ? s.P.ndig : s.Q.ndig;
    if (!s.persite && (s.ndraw & 1)) {
        s.tail = (uint64_t*)malloc((size_t)(Y * s.W) * sizeof(uint64_t));
        if (!s.tail) return BS_ENOMEM;
    }
    int64_t dh = 0;
    for (int64_t k = 0; k < n; ++k) {
        const uint32_t t = (uint32_t)(t0 + k);
        for (int pi = 0; pi < 2; ++pi) {
#pragma omp parallel for schedule(static) reduction(+ : dh)
            for (int64_t y = 0; y < Y; ++y) dh += row_halfstep(&s, S, y, pi, t);
        }
    }
    free(s.tail);
    *h0 += dh;
    return BS_OK;
}

API int bs_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

API void bs_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

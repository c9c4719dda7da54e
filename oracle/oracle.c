/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the checkerboard stochastic cellular
 * automaton (SCA) of the 2+1-dimensional octahedron surface-growth model,
 * after Kelling, Odor and Gemming, "Bit-Vectorized GPU Implementation of a
 * Stochastic Cellular Automaton Model for Surface Growth" (2016).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; neither includes or links the other.
 *
 * Representation (one byte per slope per site, no packing):
 *   sx[y*X + x] = 1  iff  h(x,y) - h(x-1,y) = +1   (slope on the bond from the
 *                                                   left neighbour, "sigma_x-")
 *   sy[y*X + x] = 1  iff  h(x,y) - h(x,y-1) = +1   ("sigma_y-")
 * with indices taken modulo X and Y (periodic boundaries, Sec. I-A).  The
 * slopes towards the + neighbours are the - slopes stored at those
 * neighbours (Sec. II-A): sigma_x+(x,y) = sx(x+1,y), sigma_y+(x,y) = sy(x,y+1).
 *
 * Update rule (generalized Kawasaki rules, Eq. (2); mask form Eqs. (3)-(5)):
 * a site whose four slopes read (x-: down, y-: down, x+: up, y+: up) is a
 * local minimum; if accepted with probability p its height grows by 2 and
 * all four slope bits flip.  A site reading (up, up, down, down) is a local
 * maximum; if accepted with probability q its height drops by 2 and the same
 * four bits flip.
 *
 * Time (Sec. I-A): one Monte-Carlo step (MCS) updates first every site with
 * (x+y) even, then every site with (x+y) odd.  t counts completed MCS from 0.
 *
 * Random acceptance bits.  The paper draws them from per-thread TinyMT
 * generators (Sec. II-B); here they come from a counter-based stream so that
 * every implementation can reproduce them:
 *   W = max(1, X/128) words of 64 sites per row and sublattice; the site
 *   (x,y) of parity pi = (x+y)&1 has k = x>>1, canonical word
 *   g = y*W + (k>>6) and bit b = k&63.
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 *   (seed mod 2^32, seed >> 32) and counter (g, t, 2j+pi, 0) for call j of
 *   that word yields lanes o0..o3.
 *   Dyadic r = sum_{i=1..n} b_i 2^-i (at most 32 fractional bits, Sec. III:
 *   sums of powers 1/2^i obtained with "and"/"or"): draw i-1 (i = 1..n) is
 *   o0 | o1<<32 of call (i-1)>>1 when i-1 is even, else o2 | o3<<32, except
 *   that for odd n the last draw (i = n) of both half-steps of MCS t comes
 *   from the one call with counter (g, t, n-1, 0): o0 | o1<<32 in the even
 *   half-step, o2 | o3<<32 in the odd one (Sec. II-B: a word of xi_0.5 is
 *   one word of random bits, so no generated bit is left unused); the
 *   acceptance word starts at 0 and for i = n down to 1 becomes
 *   (draw | acc) if b_i = 1, (draw & acc) if b_i = 0.  r = 1 accepts all,
 *   r = 0 none.  p and q share the same draws (n = max(n_p, n_q)); a site can
 *   never be a minimum and a maximum at once, so this is exact.
 *   Any other r (Sec. II-B: one random number per site): threshold
 *   T = min(floor(r * 2^32), 2^32) in IEEE double; site bit b uses
 *   u = lane (b&3) of call j = b>>2 (16 calls per word) and accepts iff
 *   u < T; p and q share u.
 *
 * Heights (Sec. I-A keeps slopes only; the absolute level is fixed here by
 * tracking the origin): h(0,0) = h0 changes by +-2 whenever the site (0,0)
 * is updated, and
 *   h(x,y) = h0 + sum_{j=1..y} (2 sy(0,j) - 1) + sum_{i=1..x} (2 sx(i,y) - 1).
 * Flat start: h(x,y) = (x+y)&1, h0 = 0, so every even site is a minimum.
 *
 * Light-cone patches: a rectangle [x0,x0+PX) x [y0,y0+PY) of the X x Y torus
 * (global coordinates modulo X, Y) evolved with its border sites frozen.
 * After T MCS every site at distance > 2T from the border holds exactly the
 * full-torus value, because a wrong value moves by at most one site per
 * half-step.  With PX == X and PY == Y the patch is the whole torus with
 * periodic neighbours and nothing is frozen.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EOVERFLOW = -4 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from its published definition (Salmon et al.,     */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two  */
/* 32x32->64 multiplications, the key bumped by the Weyl constants between   */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

EXPORT void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Acceptance probabilities                                                  */
/* ------------------------------------------------------------------------ */
struct prob {
    double r;
    int one;       /* r == 1: accept every site */
    int dyadic;    /* r * 2^32 is an integer */
    int n;         /* number of fractional binary digits (dyadic only) */
    int b[33];     /* b[i], i = 1..n: binary digits, r = sum b_i 2^-i */
    uint64_t T;    /* per-site threshold min(floor(r*2^32), 2^32) */
};

static int prob_make(double r, struct prob* P)
{
    if (!(r >= 0.0 && r <= 1.0)) return ORC_EINVAL; /* also rejects NaN */
    memset(P, 0, sizeof *P);
    P->r = r;
    double scaled = r * 4294967296.0; /* exact: scaling by a power of two */
    double fl = floor(scaled);
    P->T = (uint64_t)fl;
    if (P->T > 4294967296ull) P->T = 4294967296ull;
    P->one = (r == 1.0);
    P->dyadic = (fl == scaled);
    if (P->dyadic && !P->one) {
        uint64_t v = (uint64_t)fl; /* r = v / 2^32, v < 2^32 */
        for (int i = 1; i <= 32; ++i) P->b[i] = (int)((v >> (32 - i)) & 1u);
        int n = 0;
        for (int i = 1; i <= 32; ++i)
            if (P->b[i]) n = i;
        P->n = n;
    }
    return ORC_OK;
}

/* Dyadic digits of r: returns n (or -1 if r is not dyadic within 32 bits),
 * writes b_1..b_n to digits[0..n-1] and whether r == 1. */
EXPORT int orc_dyadic_digits(double r, int32_t* digits, int32_t* is_one)
{
    struct prob P;
    if (prob_make(r, &P) != ORC_OK || !P.dyadic) return -1;
    for (int i = 1; i <= P.n; ++i) digits[i - 1] = P.b[i];
    *is_one = P.one;
    return P.n;
}

EXPORT uint64_t orc_threshold(double r)
{
    struct prob P;
    if (prob_make(r, &P) != ORC_OK) return 0;
    return P.T;
}

/* The and/or fold of n draws into one word whose bits are set with
 * probability r = sum b_i 2^-i: least significant digit first. */
static uint64_t fold_draws(const struct prob* P, const uint64_t* draw)
{
    if (P->one) return ~(uint64_t)0;
    uint64_t acc = 0;
    for (int i = P->n; i >= 1; --i)
        acc = P->b[i] ? (draw[i - 1] | acc) : (draw[i - 1] & acc);
    return acc;
}

/* Exposed for the enumeration test of the fold. */
EXPORT uint64_t orc_fold(double r, const uint64_t* draws)
{
    struct prob P;
    if (prob_make(r, &P) != ORC_OK || !P.dyadic) return 0;
    return fold_draws(&P, draws);
}

/* The acceptance words of canonical word g in half-step `parity` of MCS t. */
static void acceptance_words(uint64_t seed, uint32_t t, int parity, uint64_t g,
                             const struct prob* P, const struct prob* Q, int persite,
                             uint64_t* xi_p, uint64_t* xi_q)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    if (!persite) {
        int n = P->n > Q->n ? P->n : Q->n; /* r = 0 and r = 1 have n = 0 */
        uint64_t draw[32];
        for (int i = 0; i < n; ++i) {
            int j = i >> 1;
            /* the odd last draw: one call serves both half-steps of the MCS */
            int shared = (n & 1) && i == n - 1;
            uint32_t ctr[4] = {(uint32_t)g, t, (uint32_t)(shared ? 2 * j : 2 * j + parity), 0u};
            philox4x32_10(ctr, key, out);
            int upper = shared ? parity : (i & 1);
            draw[i] = upper ? ((uint64_t)out[2] | ((uint64_t)out[3] << 32))
                            : ((uint64_t)out[0] | ((uint64_t)out[1] << 32));
        }
        *xi_p = fold_draws(P, draw);
        *xi_q = fold_draws(Q, draw);
    } else {
        uint64_t wp = 0, wq = 0;
        for (int b = 0; b < 64; ++b) {
            int j = b >> 2;
            uint32_t ctr[4] = {(uint32_t)g, t, (uint32_t)(2 * j + parity), 0u};
            philox4x32_10(ctr, key, out);
            uint64_t u = out[b & 3];
            if (u < P->T) wp |= (uint64_t)1 << b;
            if (u < Q->T) wq |= (uint64_t)1 << b;
        }
        *xi_p = wp;
        *xi_q = wq;
    }
}

/* Exposed so tests can look at the stream itself (bit frequencies, and the
 * device generator's words). */
EXPORT int orc_acceptance_words(uint64_t seed, uint32_t t, int parity, uint64_t g0, int64_t count,
                                double p, double q, int force_persite,
                                uint64_t* xi_p, uint64_t* xi_q)
{
    struct prob P, Q;
    if (prob_make(p, &P) || prob_make(q, &Q) || (parity & ~1)) return ORC_EINVAL;
    int persite = force_persite || !P.dyadic || !Q.dyadic;
    for (int64_t i = 0; i < count; ++i)
        acceptance_words(seed, t, parity, g0 + (uint64_t)i, &P, &Q, persite, &xi_p[i], &xi_q[i]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------ */
static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static int check_size(int64_t X, int64_t Y)
{
    if (!is_pow2(X) || !is_pow2(Y) || X < 4 || Y < 4 || X > (1 << 17) || Y > (1 << 17))
        return ORC_EINVAL;
    return ORC_OK;
}

static int64_t words_per_row(int64_t X) { return X >= 128 ? X / 128 : 1; }

struct patch {
    int64_t X, Y;     /* torus */
    int64_t x0, y0;   /* global origin of the patch */
    int64_t PX, PY;   /* patch extent; == X, Y means the whole torus */
    int torus;
};

static int patch_make(int64_t X, int64_t Y, int64_t x0, int64_t y0, int64_t PX, int64_t PY,
                      struct patch* R)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    if (PX < 3 || PY < 3 || PX > X || PY > Y || x0 < 0 || y0 < 0 || x0 >= X || y0 >= Y)
        return ORC_EINVAL;
    R->X = X; R->Y = Y; R->x0 = x0; R->y0 = y0; R->PX = PX; R->PY = PY;
    R->torus = (PX == X && PY == Y);
    if (R->torus && (x0 != 0 || y0 != 0)) return ORC_EINVAL;
    return ORC_OK;
}

/* Flat initial surface h(x,y) = (x+y)&1: every slope of an odd site points
 * up towards it, so sx = sy = (x+y)&1. */
EXPORT int orc_flat_patch(int64_t X, int64_t Y, int64_t x0, int64_t y0, int64_t PX, int64_t PY,
                          uint8_t* sx, uint8_t* sy, int32_t* H)
{
    struct patch R;
    if (patch_make(X, Y, x0, y0, PX, PY, &R)) return ORC_EINVAL;
    for (int64_t ly = 0; ly < PY; ++ly)
        for (int64_t lx = 0; lx < PX; ++lx) {
            int64_t x = (x0 + lx) % X, y = (y0 + ly) % Y;
            uint8_t odd = (uint8_t)((x + y) & 1);
            sx[ly * PX + lx] = odd;
            sy[ly * PX + lx] = odd;
            if (H) H[ly * PX + lx] = odd;
        }
    return ORC_OK;
}

EXPORT int orc_flat(int64_t X, int64_t Y, uint8_t* sx, uint8_t* sy, int32_t* H)
{
    return orc_flat_patch(X, Y, 0, 0, X, Y, sx, sy, H);
}

/* ------------------------------------------------------------------------ */
/* One half-step                                                             */
/* ------------------------------------------------------------------------ */

/* Acceptance bits for every site of the patch in the current half-step:
 * either looked up in caller-given word arrays (full torus only) or computed
 * from the stream for each canonical word the patch touches. */
struct accept_src {
    const uint64_t* xi_p;   /* injected words, indexed by g (or NULL) */
    const uint64_t* xi_q;
    uint64_t seed;
    uint32_t t;
    const struct prob* P;
    const struct prob* Q;
    int persite;
};

/* Per-row cache of the words a patch row touches. */
struct row_words {
    int64_t nw;          /* distinct words in one patch row */
    int64_t* slot_of_lx; /* lx -> slot */
    int64_t* word_of_slot;
    uint64_t* wp;        /* [PY][nw] */
    uint64_t* wq;
};

static int row_words_init(const struct patch* R, struct row_words* C)
{
    int64_t W = words_per_row(R->X);
    C->slot_of_lx = (int64_t*)malloc(sizeof(int64_t) * (size_t)R->PX);
    C->word_of_slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)(W < R->PX ? W : R->PX));
    if (!C->slot_of_lx || !C->word_of_slot) return ORC_ENOMEM;
    int64_t* seen = (int64_t*)malloc(sizeof(int64_t) * (size_t)W);
    if (!seen) return ORC_ENOMEM;
    for (int64_t w = 0; w < W; ++w) seen[w] = -1;
    C->nw = 0;
    for (int64_t lx = 0; lx < R->PX; ++lx) {
        int64_t x = (R->x0 + lx) % R->X;
        int64_t w = (x >> 1) >> 6;
        if (seen[w] < 0) {
            seen[w] = C->nw;
            C->word_of_slot[C->nw++] = w;
        }
        C->slot_of_lx[lx] = seen[w];
    }
    free(seen);
    C->wp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(C->nw * R->PY));
    C->wq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(C->nw * R->PY));
    if (!C->wp || !C->wq) return ORC_ENOMEM;
    return ORC_OK;
}

static void row_words_free(struct row_words* C)
{
    free(C->slot_of_lx); free(C->word_of_slot); free(C->wp); free(C->wq);
    memset(C, 0, sizeof *C);
}

static void row_words_fill(const struct patch* R, struct row_words* C,
                           const struct accept_src* A, int parity)
{
    int64_t W = words_per_row(R->X);
#pragma omp parallel for schedule(static)
    for (int64_t ly = 0; ly < R->PY; ++ly) {
        int64_t y = (R->y0 + ly) % R->Y;
        for (int64_t s = 0; s < C->nw; ++s) {
            uint64_t g = (uint64_t)(y * W + C->word_of_slot[s]);
            uint64_t p, q;
            if (A->xi_p) {
                p = A->xi_p[g];
                q = A->xi_q[g];
            } else {
                acceptance_words(A->seed, A->t, parity, g, A->P, A->Q, A->persite, &p, &q);
            }
            C->wp[ly * C->nw + s] = p;
            C->wq[ly * C->nw + s] = q;
        }
    }
}

/* Updates every non-frozen site of sublattice `parity`.  Same-parity sites
 * share no bond, so the result does not depend on the visiting order and
 * rows may be processed concurrently: a row writes only its own sx bytes, its
 * own sy bytes at its parity's columns and the sy bytes of the next row at
 * those same columns, which the next row (opposite column parity) never
 * writes.  Returns nothing; counts depositions / removals in cnt[0] / cnt[1]. */
static void halfstep_patch(const struct patch* R, uint8_t* sx, uint8_t* sy, int32_t* H,
                           int64_t* h0, int parity, const struct row_words* C, int64_t cnt[2])
{
    const int64_t X = R->X, Y = R->Y, PX = R->PX, PY = R->PY;
    int64_t dep = 0, rem = 0, dh0 = 0;
#pragma omp parallel for schedule(static) reduction(+ : dep, rem, dh0)
    for (int64_t ly = 0; ly < PY; ++ly) {
        if (!R->torus && (ly == 0 || ly == PY - 1)) continue;
        int64_t y = (R->y0 + ly) % Y;
        int64_t lyn = R->torus ? (ly + 1) % PY : ly + 1;
        for (int64_t lx = 0; lx < PX; ++lx) {
            if (!R->torus && (lx == 0 || lx == PX - 1)) continue;
            int64_t x = (R->x0 + lx) % X;
            if (((x + y) & 1) != parity) continue;
            int64_t lxn = R->torus ? (lx + 1) % PX : lx + 1;
            int64_t here = ly * PX + lx, right = ly * PX + lxn, up = lyn * PX + lx;
            int xm = sx[here], ym = sy[here], xp = sx[right], yp = sy[up];
            int b = (int)((x >> 1) & 63);  /* bit of site x in its canonical word */
            int64_t s = C->slot_of_lx[lx];  /* that word's slot: g = y*W + ((x>>1)>>6) */
            int acc_p = (int)((C->wp[ly * C->nw + s] >> b) & 1u);
            int acc_q = (int)((C->wq[ly * C->nw + s] >> b) & 1u);
            int dh = 0;
            if (!xm && !ym && xp && yp && acc_p) dh = +2;       /* minimum -> deposit */
            else if (xm && ym && !xp && !yp && acc_q) dh = -2;  /* maximum -> remove */
            if (dh) {
                sx[here] ^= 1; sy[here] ^= 1; sx[right] ^= 1; sy[up] ^= 1;
                if (H) H[here] += dh;
                if (dh > 0) ++dep; else ++rem;
                if (x == 0 && y == 0) dh0 += dh;
            }
        }
    }
    if (h0) *h0 += dh0;
    if (cnt) { cnt[0] += dep; cnt[1] += rem; }
}

/* Half-step with caller-given acceptance words xi_p[g], xi_q[g] for every
 * canonical word g of the torus (the random stream is bypassed). */
EXPORT int orc_halfstep_xi(int64_t X, int64_t Y, uint8_t* sx, uint8_t* sy, int32_t* H, int64_t* h0,
                           int parity, const uint64_t* xi_p, const uint64_t* xi_q)
{
    struct patch R;
    if (patch_make(X, Y, 0, 0, X, Y, &R) || (parity & ~1)) return ORC_EINVAL;
    struct row_words C;
    memset(&C, 0, sizeof C);
    if (row_words_init(&R, &C)) { row_words_free(&C); return ORC_ENOMEM; }
    struct accept_src A = {xi_p, xi_q, 0, 0, NULL, NULL, 0};
    row_words_fill(&R, &C, &A, parity);
    halfstep_patch(&R, sx, sy, H, h0, parity, &C, NULL);
    row_words_free(&C);
    return ORC_OK;
}

/* The same for a batch of independent lattices of one size, stored back to
 * back: sx/sy/H advance by X*Y per item, xi_p/xi_q by Y*W, h0 by 1. */
EXPORT int orc_halfstep_xi_batch(int64_t nbatch, int64_t X, int64_t Y, uint8_t* sx, uint8_t* sy,
                                 int32_t* H, int64_t* h0, int parity,
                                 const uint64_t* xi_p, const uint64_t* xi_q)
{
    int64_t N = X * Y, G = Y * words_per_row(X);
    for (int64_t i = 0; i < nbatch; ++i) {
        int rc = orc_halfstep_xi(X, Y, sx + i * N, sy + i * N, H ? H + i * N : NULL,
                                 h0 ? h0 + i : NULL, parity, xi_p + i * G, xi_q + i * G);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Heights and moments                                                       */
/* ------------------------------------------------------------------------ */

/* h(x,y) from the slopes and the origin height, by plain path sums. */
EXPORT int orc_heights(int64_t X, int64_t Y, const uint8_t* sx, const uint8_t* sy, int64_t h0,
                       int64_t* out)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    int64_t col = h0; /* h(0,y) */
    for (int64_t y = 0; y < Y; ++y) {
        if (y > 0) col += 2 * (int64_t)sy[y * X + 0] - 1;
        int64_t h = col;
        out[y * X + 0] = h;
        for (int64_t x = 1; x < X; ++x) {
            h += 2 * (int64_t)sx[y * X + x] - 1;
            out[y * X + x] = h;
        }
    }
    return ORC_OK;
}

static int fits_i64(__int128 v) { return v >= (__int128)INT64_MIN && v <= (__int128)INT64_MAX; }

/* N, sum h, sum h^2 over the torus; W^2 = <h^2> - <h>^2.  Sums are exact
 * (128-bit); ORC_EOVERFLOW if a sum does not fit in 64 bits. */
EXPORT int orc_moments(int64_t X, int64_t Y, const uint8_t* sx, const uint8_t* sy, int64_t h0,
                       int64_t* out3, double* w2)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    int64_t* h = (int64_t*)malloc(sizeof(int64_t) * (size_t)(X * Y));
    if (!h) return ORC_ENOMEM;
    orc_heights(X, Y, sx, sy, h0, h);
    __int128 s1 = 0, s2 = 0;
    for (int64_t i = 0; i < X * Y; ++i) {
        s1 += h[i];
        s2 += (__int128)h[i] * h[i];
    }
    free(h);
    __int128 N = (__int128)X * Y;
    if (!fits_i64(s1) || !fits_i64(s2)) return ORC_EOVERFLOW;
    out3[0] = (int64_t)N; out3[1] = (int64_t)s1; out3[2] = (int64_t)s2;
    if (w2) *w2 = (double)(N * s2 - s1 * s1) / ((double)N * (double)N);
    return ORC_OK;
}

/* Two-time sums between the state at time t (sx_t, sy_t, h0_t) and at an
 * earlier time s: N, sum h_t h_s, sum h_t, sum h_s; and
 * C(t,s) = <h_t h_s> - <h_t><h_s>. */
EXPORT int orc_autocorr(int64_t X, int64_t Y, const uint8_t* sx_t, const uint8_t* sy_t, int64_t h0_t,
                        const uint8_t* sx_s, const uint8_t* sy_s, int64_t h0_s,
                        int64_t* out4, double* c)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    int64_t* ht = (int64_t*)malloc(sizeof(int64_t) * (size_t)(X * Y));
    int64_t* hs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(X * Y));
    if (!ht || !hs) { free(ht); free(hs); return ORC_ENOMEM; }
    orc_heights(X, Y, sx_t, sy_t, h0_t, ht);
    orc_heights(X, Y, sx_s, sy_s, h0_s, hs);
    __int128 sts = 0, st = 0, ss = 0;
    for (int64_t i = 0; i < X * Y; ++i) {
        sts += (__int128)ht[i] * hs[i];
        st += ht[i];
        ss += hs[i];
    }
    free(ht); free(hs);
    __int128 N = (__int128)X * Y;
    if (!fits_i64(sts) || !fits_i64(st) || !fits_i64(ss)) return ORC_EOVERFLOW;
    out4[0] = (int64_t)N; out4[1] = (int64_t)sts; out4[2] = (int64_t)st; out4[3] = (int64_t)ss;
    if (c) *c = (double)(N * sts - st * ss) / ((double)N * (double)N);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* MCS loops                                                                 */
/* ------------------------------------------------------------------------ */

/* n_mcs MCS on a patch (or the whole torus) starting at absolute time t0.
 * series (optional, whole torus only): after MCS i, series[2i] = sum h and
 * series[2i+1] = sum h^2.  cnt (optional): depositions, removals. */
EXPORT int orc_run_patch(int64_t X, int64_t Y, int64_t x0, int64_t y0, int64_t PX, int64_t PY,
                         uint8_t* sx, uint8_t* sy, int32_t* H, int64_t* h0,
                         uint64_t seed, int64_t t0, int64_t n_mcs, double p, double q,
                         int force_persite, int64_t* series, int64_t* cnt)
{
    struct patch R;
    struct prob P, Q;
    if (patch_make(X, Y, x0, y0, PX, PY, &R)) return ORC_EINVAL;
    if (prob_make(p, &P) || prob_make(q, &Q)) return ORC_EINVAL;
    if (t0 < 0 || n_mcs < 0 || t0 + n_mcs > 4294967295LL) return ORC_EINVAL;
    if (series && !R.torus) return ORC_EINVAL;
    struct row_words C;
    memset(&C, 0, sizeof C);
    if (row_words_init(&R, &C)) { row_words_free(&C); return ORC_ENOMEM; }
    int persite = force_persite || !P.dyadic || !Q.dyadic;
    int64_t c2[2] = {0, 0};
    int rc = ORC_OK;
    for (int64_t i = 0; i < n_mcs; ++i) {
        uint32_t t = (uint32_t)(t0 + i);
        for (int parity = 0; parity < 2; ++parity) {
            struct accept_src A = {NULL, NULL, seed, t, &P, &Q, persite};
            row_words_fill(&R, &C, &A, parity);
            halfstep_patch(&R, sx, sy, H, R.torus ? h0 : NULL, parity, &C, c2);
        }
        if (series) {
            int64_t m[3];
            rc = orc_moments(X, Y, sx, sy, *h0, m, NULL);
            if (rc) break;
            series[2 * i] = m[1];
            series[2 * i + 1] = m[2];
        }
    }
    row_words_free(&C);
    if (cnt) { cnt[0] += c2[0]; cnt[1] += c2[1]; }
    return rc;
}

EXPORT int orc_run(int64_t X, int64_t Y, uint8_t* sx, uint8_t* sy, int32_t* H, int64_t* h0,
                   uint64_t seed, int64_t t0, int64_t n_mcs, double p, double q, int force_persite,
                   int64_t* series, int64_t* cnt)
{
    return orc_run_patch(X, Y, 0, 0, X, Y, sx, sy, H, h0, seed, t0, n_mcs, p, q, force_persite,
                         series, cnt);
}

/* ------------------------------------------------------------------------ */
/* Canonical packed layout (Sec. II-A, role-grouped arrays)                  */
/* ------------------------------------------------------------------------ */
/* S[d][pi][y][w], d = 0 for x-slopes and 1 for y-slopes, pi the site parity,
 * bit k&63 of word k>>6 holding the site with x>>1 == k.  Bits of a partial
 * word (X < 128) beyond X/2 are zero. */
EXPORT int orc_pack(int64_t X, int64_t Y, const uint8_t* sx, const uint8_t* sy, uint64_t* S)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    int64_t W = words_per_row(X), P = Y * W;
    memset(S, 0, sizeof(uint64_t) * (size_t)(4 * P));
    for (int64_t y = 0; y < Y; ++y)
        for (int64_t x = 0; x < X; ++x) {
            int pi = (int)((x + y) & 1);
            int64_t k = x >> 1;
            int64_t off = y * W + (k >> 6);
            uint64_t bit = (uint64_t)1 << (k & 63);
            if (sx[y * X + x]) S[(0 * 2 + pi) * P + off] |= bit;
            if (sy[y * X + x]) S[(1 * 2 + pi) * P + off] |= bit;
        }
    return ORC_OK;
}

EXPORT int orc_unpack(int64_t X, int64_t Y, const uint64_t* S, uint8_t* sx, uint8_t* sy)
{
    if (check_size(X, Y)) return ORC_EINVAL;
    int64_t W = words_per_row(X), P = Y * W;
    for (int64_t y = 0; y < Y; ++y)
        for (int64_t x = 0; x < X; ++x) {
            int pi = (int)((x + y) & 1);
            int64_t k = x >> 1;
            int64_t off = y * W + (k >> 6);
            int b = (int)(k & 63);
            sx[y * X + x] = (uint8_t)((S[(0 * 2 + pi) * P + off] >> b) & 1u);
            sy[y * X + x] = (uint8_t)((S[(1 * 2 + pi) * P + off] >> b) & 1u);
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
EXPORT int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

EXPORT void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

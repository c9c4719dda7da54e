/*
 * sca.h -- C ABI of the bit-vectorized checkerboard SCA of the 2+1-dimensional
 * octahedron surface-growth model on AMD Instinct MI355X (gfx950).
 *
 * Model (Kelling, Odor, Gemming 2016, Sec. I-A and Eq. (2)): an X x Y
 * periodic lattice of heights whose neighbours differ by exactly 1, stored as
 * two slope bits per site (Sec. II-A).  A half-step updates one checkerboard
 * sublattice at once: a local minimum is lifted by 2 with probability p, a
 * local maximum lowered by 2 with probability q, each flipping its four
 * slope bits.  One Monte-Carlo step (MCS) is the even half-step ((x+y) even)
 * followed by the odd one.
 *
 * Device state layout (Sec. II-A, role-grouped arrays; Fig. 3 of the paper
 * keeps one array per slope direction and sublattice):
 *   uint64 S[2][2][Y][W],  W = max(1, X/128)
 *   S[d][pi][y][w]: d = 0 x-slopes, d = 1 y-slopes; pi = (x+y)&1; bit b of
 *   word w holds the site x with x>>1 == 64*w + b of row y.  A set bit means
 *   the height rises by one towards the site across that bond from the
 *   left (x) or lower (y) neighbour.  For X < 128 only bits 0..X/2-1 are used
 *   and the rest are zero.  In torch terms: an int64 tensor of shape
 *   (2, 2, Y, W).
 *
 * Random acceptance words (counter-based, so results are reproducible and
 * independent of the launch shape): Philox4x32-10 with key
 * (seed mod 2^32, seed >> 32) and counter (g, t, 2j + pi, 0), where
 * g = y*W + w is the canonical word, t the 0-based MCS index and j the call
 * index within the word.  Dyadic p and q (p*2^32 and q*2^32 integers;
 * Sec. III: sums of powers 1/2^i via and/or) fold n = max(n_p, n_q) 64-bit
 * draws (lanes 0|1, then 2|3 of each call), least significant binary digit
 * first; for odd n the last draw of both half-steps of an MCS comes from the
 * one call (g, t, n-1, 0), lanes 0|1 in the even half-step and 2|3 in the
 * odd one (p = 1/2: one call per word and MCS); any other p or q compares one
 * 32-bit uniform per site with floor(r * 2^32) (Sec. II-B), 16 calls per word.
 *
 * Conventions for every call:
 *  - Sizes: X and Y powers of two, 4 <= X, Y <= 131072.  0 <= p, q <= 1.
 *  - Ownership: every device buffer of state is owned by the caller: S, aux
 *    and, for the temporally blocked passes, a second buffer of the size of
 *    S (sca_set_pass_buffer).  The library keeps non-owning pointers, so the
 *    caller keeps them alive until sca_destroy.  The library owns only a
 *    small device workspace for the moment sums (about 32*Y bytes),
 *    allocated by sca_init and freed by sca_destroy; sca_step allocates
 *    nothing.
 *  - Streams: all work is enqueued on the stream given to sca_init.  Only
 *    calls that return numbers to the host synchronize that stream.
 *  - Errors: functions return SCA_OK or a negative code; an invalid argument
 *    leaves the state untouched.  After any HIP failure the context is
 *    failed and every later call returns SCA_ESTATE.
 *  - A context is not thread-safe; contexts do not share state.
 */
#ifndef SCA_H
#define SCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sca_ctx sca_ctx;

enum sca_status {
    SCA_OK = 0,
    SCA_EINVAL = -1,    /* invalid argument; nothing was changed */
    SCA_ENOMEM = -2,    /* device allocation failed */
    SCA_EDEVICE = -3,   /* a HIP call failed; the context is now failed */
    SCA_EOVERFLOW = -4, /* an exact result does not fit its output type */
    SCA_ESTATE = -5,    /* the context failed earlier */
    SCA_EBUSY = -6,     /* a capacity limit was reached (batched calls) */
    SCA_ENOBUF = -7,    /* a temporally blocked pass was planned but no pass
                           buffer is attached (sca_set_pass_buffer); nothing
                           was changed */
    SCA_ESCRATCH = -8   /* the lattice needs more than the static scratch of
                           sca_roughness_noalloc (Y > SCA_NOALLOC_MAX_Y) */
};

/* sca_step_ex flags */
#define SCA_FORCE_PERSITE 1u /* use per-site 32-bit compares even for dyadic p, q */
#define SCA_STEP_GRAPH 2u    /* capture the MCS loop into one hipGraph and launch it once */
#define SCA_NO_FUSE 4u       /* always two half-step launches per MCS (no fused pass) */

/* Length of the caller-owned int64 aux buffer; aux[0] holds h(0,0). */
#define SCA_AUX_LEN 8

/* Number of uint64 words of S for an X x Y lattice: 4 * Y * max(1, X/128);
 * 0 for invalid sizes. */
size_t sca_state_words(int64_t X, int64_t Y);

/* Creates a context for an X x Y lattice and writes the flat initial surface
 * h(x,y) = (x+y)&1 (every even site a minimum: S[.][0] = 0, S[.][1] = all
 * valid bits), h(0,0) = 0, t = 0.
 *   slopes_dev: device buffer of sca_state_words(X,Y) uint64 (S above)
 *   aux_dev:    device buffer of SCA_AUX_LEN int64
 *   hip_stream: hipStream_t to enqueue on (NULL = default stream)
 * The initialisation is enqueued, not waited for. */
int sca_init(sca_ctx** out, int64_t X, int64_t Y, uint64_t seed, void* slopes_dev,
             int64_t* aux_dev, void* hip_stream);

/* Advances n_mcs >= 0 MCS with deposition probability p and removal
 * probability q (Eq. (2)); each MCS is the even then the odd half-step
 * (Sec. I-A), t grows by n_mcs.  Asynchronous.
 * For X >= 8192 groups of MCS run as temporally blocked passes (all
 * half-steps of `depth` MCS in one sweep over the state, out of place into
 * the caller's pass buffer and back; see sca_set_blocking and
 * sca_set_pass_buffer), which divides the HBM traffic per MCS by about
 * 2*depth.  The passes come in an even number so that S holds the state when
 * the enqueued work has run: whole passes of `depth` MCS, then the remainder
 * r as two passes of ceil(r/2) and floor(r/2) MCS, or two half-step launches
 * when r = 1 (sca_plan_step reports the plan).  The results are bit-identical
 * to the two-launch form.  SCA_ENOBUF (nothing enqueued, t unchanged) if a
 * blocked pass is planned and no pass buffer is attached; sca_set_blocking
 * with depth 0 selects the two-launch form, which needs none. */
int sca_step(sca_ctx* ctx, int64_t n_mcs, double p, double q);

/* sca_step with flags (SCA_FORCE_PERSITE, SCA_STEP_GRAPH).  With
 * SCA_STEP_GRAPH the 2*n_mcs half-step launches are captured into a hipGraph
 * that is launched once (one launch for the whole run) and then released;
 * this call then synchronizes the stream. */
int sca_step_ex(sca_ctx* ctx, int64_t n_mcs, double p, double q, unsigned flags);

/* Acceptance paths (Sec. III and Sec. II-B): p and q both 0 or 1 (no random
 * words), dyadic p and q (and/or fold of 64-bit draws), any other p or q (one
 * 32-bit uniform per site). */
#define SCA_PATH_DRAWFREE 0
#define SCA_PATH_MASK 1
#define SCA_PATH_PERSITE 2

/* The launches sca_step_ex(ctx, n_mcs, p, q, flags) would enqueue with the
 * context's current blocking settings. */
typedef struct sca_step_plan {
    int32_t path;          /* SCA_PATH_* */
    int32_t depth;         /* MCS per whole blocked pass; 0 if there is none */
    int32_t band;          /* rows per workgroup band of a blocked pass */
    int32_t tail1, tail2;  /* MCS of the two remainder passes; 0 if none */
    int64_t n_pass;        /* whole passes of `depth` MCS (even) */
    int64_t n_unfused;     /* MCS run as two half-step launches each */
    char kernel[80];       /* kernel of the whole passes, with its template
                              arguments, or "none" */
    char tail_kernel[80];  /* kernel of the first remainder pass, or "none" */
    char halfstep_kernel[80]; /* kernel of a half-step launch */
} sca_step_plan;

/* Fills *out with the plan of sca_step_ex for these arguments (host only, no
 * device work).  SCA_EINVAL for invalid arguments. */
int sca_plan_step(const sca_ctx* ctx, int64_t n_mcs, double p, double q, unsigned flags, sca_step_plan* out);

/* Attaches the caller-owned device buffer pass_dev of `bytes` bytes, at least
 * 8 * sca_state_words(X, Y), that the temporally blocked passes write every
 * other pass (a pass reads beyond its bands, so it runs out of place).  It
 * must not overlap S.  Its contents between calls are meaningless.  NULL
 * detaches it.  SCA_EINVAL if too small or overlapping. */
int sca_set_pass_buffer(sca_ctx* ctx, void* pass_dev, size_t bytes);

/* Writes the flat initial surface into S again (as sca_init does): h(0,0) = 0,
 * t = 0.  Asynchronous. */
int sca_reset(sca_ctx* ctx);

/* Restores a state saved by sca_snapshot (or written in its layout: S, then
 * one int64 h(0,0)) from the caller-owned device buffer snap_dev into S and
 * aux[0], and sets the MCS counter to t, 0 <= t < 2^32.  The random stream is
 * counter-based (MCS index, half-step, draw, word), so its whole state is t:
 * a run resumed at t continues bit-identically (the paper loads and stores
 * its generator states around the update loop, Fig. 3).  The buffer must hold
 * a valid surface (every bond a slope of +-1; per row X/2 up x-slopes and per
 * column Y/2 up y-slopes as on every surface reached from the flat one);
 * unused bits of partial words (X < 128) must be zero.  Asynchronous. */
int sca_restore(sca_ctx* ctx, const void* snap_dev, int64_t t);

/* Heights h(x,y) of rows [y0, y0+ny), all x, row-major int32 into out_dev
 * (ny*X values, caller-owned):
 *   h(x,y) = h(0,0) + sum_{j=1..y} (2 sy(0,j) - 1) + sum_{i=1..x} (2 sx(i,y) - 1).
 * SCA_EOVERFLOW if |h(0,0)| + X + Y >= 2^31.  Synchronizes (reads h(0,0)). */
int sca_heights(sca_ctx* ctx, int64_t y0, int64_t ny, int32_t* out_dev);

/* Exact moments of the height field: out3 = {N, sum h, sum h^2} with
 * N = X*Y, and w2 = (N sum h^2 - (sum h)^2) / N^2, the squared surface
 * roughness (Sec. I-A).  Sums are formed exactly in 128-bit arithmetic;
 * SCA_EOVERFLOW if one does not fit in int64.  Synchronizes. */
int sca_roughness(sca_ctx* ctx, int64_t out3[3], double* w2);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the exact
 * moments of sca_roughness, out3 = {N, sum h, sum h^2} and w2, of a state
 * given directly, with no context and no allocation of any kind.
 *   slopes_dev: caller's device state S[2][2][Y][W] (layout above), read only
 *   aux_dev:    caller's device int64 with h(0,0) (aux[0]), read only
 *   X, Y:       lattice size (powers of two, 4 <= X <= 131072, 4 <= Y)
 *   hip_stream: stream to enqueue on; it must belong to the current device
 * The row and column sums go to a static device array of
 * SCA_NOALLOC_SCRATCH_WORDS int64 (4 MiB + 64 B) that the library holds on
 * each GPU it runs on until the process ends; Y > SCA_NOALLOC_MAX_Y returns
 * SCA_ESCRATCH.  Every call on one GPU uses that GPU's single array: calls
 * that overlap on one GPU (other host threads, other streams) race and must
 * be serialized by the caller.  Each call writes every scratch word it reads
 * before reading it, so nothing carries over between calls.
 * SCA_EINVAL for invalid arguments, SCA_EOVERFLOW as sca_roughness,
 * SCA_EDEVICE if a HIP call fails.  Synchronizes hip_stream. */
#define SCA_NOALLOC_MAX_Y 131072
#define SCA_NOALLOC_SCRATCH_WORDS (4 * SCA_NOALLOC_MAX_Y + 8)
int sca_roughness_noalloc(const void* slopes_dev, const int64_t* aux_dev, int64_t X, int64_t Y,
                          void* hip_stream, int64_t out3[3], double* w2);

/* Bytes of a snapshot: the state S plus one int64 h(0,0). */
size_t sca_snapshot_bytes(const sca_ctx* ctx);

/* Copies S and h(0,0) into the caller-owned device buffer snap_dev
 * (sca_snapshot_bytes bytes).  Asynchronous. */
int sca_snapshot(sca_ctx* ctx, void* snap_dev);

/* Two-time sums between the current heights h_t and those of a snapshot h_s
 * taken earlier from a context of the same size (the aging studies the paper
 * names as its application, Sec. IV): out4 = {N, sum h_t h_s, sum h_t,
 * sum h_s}, exact; c_ts = (N sum h_t h_s - sum h_t sum h_s) / N^2.
 * SCA_EOVERFLOW if a sum does not fit in int64.  Synchronizes. */
int sca_autocorr(sca_ctx* ctx, const void* snap_dev, int64_t out4[4], double* c_ts);

/* Current MCS count t and origin height h(0,0).  Synchronizes. */
int sca_get_meta(sca_ctx* ctx, int64_t* t, int64_t* h0);

/* Temporal blocking of sca_step: depth = MCS per fused pass (1..13), 0 =
 * never fuse, -1 = automatic; band = rows per workgroup (a power of two >= 4
 * and >= 2*depth that divides Y, with Y >= 2*band), 0 = automatic (the
 * tallest of 256 (p, q in {0, 1}) or 128, then 64, 32, 16, 8, that leaves
 * enough workgroups to fill the chip).
 * Passes run at most 13 MCS deep when p and q are both 0 or 1 (no random
 * words) and X = 2^16, at most 8 deep for smaller X and 6 for X = 2^17, and
 * at most 4 deep with random words: a larger depth is lowered to that limit
 * when sca_step runs.  The automatic depth without random words is 13 on
 * bands of >= 256 rows and 10 on 128-row bands (both lowered to the limit
 * above), 5 on 64-row bands; with random words 4 on bands of >= 128 rows and
 * 3 on 32- and 64-row bands; 2 on 16-row bands and 1 on smaller ones; the
 * per-site path (non-dyadic p or q), which is ALU-bound, is never fused.
 * Any setting gives bit-identical results. */
int sca_set_blocking(sca_ctx* ctx, int32_t depth, int32_t band);

/* Sets the MCS counter (sca_restore sets it together with the state).
 * 0 <= t < 2^32. */
int sca_set_time(sca_ctx* ctx, int64_t t);

/* Test hook: one half-step of sublattice `parity` whose acceptance words are
 * read from xi_p_dev[g], xi_q_dev[g] (Y*W uint64 each, device) instead of the
 * random stream; t is not advanced.  Asynchronous. */
int sca_debug_halfstep(sca_ctx* ctx, int parity, const uint64_t* xi_p_dev,
                       const uint64_t* xi_q_dev);

/* Test hook: the device Philox4x32-10 block function for n counters
 * ctr_dev[4i..4i+3] with key (k0, k1) into out_dev[4i..4i+3].  Asynchronous
 * on hip_stream. */
int sca_debug_philox(const uint32_t* ctr_dev, uint32_t k0, uint32_t k1, int64_t n,
                     uint32_t* out_dev, void* hip_stream);

/* Diagnostic: `threads` threads (a multiple of 256) each evaluate `calls`
 * Philox4x32-10 blocks and fold them into one word (stored into
 * sink_dev[0..255] only if it happens to equal the key), to measure the
 * generator's throughput on this device.  Asynchronous on hip_stream. */
int sca_debug_philox_rate(int64_t threads, int32_t calls, uint32_t* sink_dev, void* hip_stream);

/* Frees the context and its workspace (after synchronizing its stream).
 * Never frees caller buffers.  NULL is ignored. */
void sca_destroy(sca_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Ensembles: many independent realizations in one persistent launch.       */
/* ------------------------------------------------------------------------ */
/* A batch advances thousands of independent lattices of uneven size in one
 * persistent, hipGraph-captured kernel launch per epoch.  Each realization
 * draws from its own seed with the same counters as the single-lattice path,
 * so its state after any number of MCS is bit-identical to a solo run of the
 * same (X, Y, p, q, seed) -- independent of the schedule and configuration.
 * States live in a caller-owned device arena; the library keeps a small
 * table of per-slot descriptors on the device. */

typedef struct sca_batch sca_batch;

/* One realization: X, Y powers of two with 4 <= X <= 8192, 4 <= Y <= 131072;
 * 0 <= p, q <= 1; n_mcs >= 0 MCS in total; flags: SCA_FORCE_PERSITE. */
typedef struct sca_req {
    int64_t X, Y;
    double p, q;
    int64_t n_mcs;
    uint64_t seed;
    uint32_t flags;
    uint32_t reserved; /* must be 0 */
} sca_req;

/* Launch shape and schedule of the persistent kernel.  Every setting gives
 * bit-identical results; only the speed differs. */
typedef struct sca_batch_config {
    int32_t block_threads; /* workgroup size: 256, 512 or 1024 */
    int32_t blocks_per_cu; /* persistent workgroups per compute unit, 1..8 */
    int32_t lds_bytes;     /* realizations with 32*X*Y/128 <= lds_bytes bytes of
                              state (X >= 128; 4*Y*8 bytes for X < 128) run
                              from LDS; 0 = never; at most 65536 */
    int32_t order;         /* 0: longest remaining work first, 1: slot order */
    int32_t words_per_lane;/* word tile: 64-site words per lane in a row, 1 or 2 */
    int32_t depth;         /* realizations in global memory with dyadic p, q and
                              1024 <= X <= 8192 run as temporally blocked
                              passes of `depth` MCS (0 = never, 1 or 2; 3 or
                              4 only with 512-thread workgroups, one per
                              compute unit, whose registers hold the deeper
                              window; SCA_EINVAL otherwise): one
                              band per group of X/128 lanes, at least 8*depth
                              rows each (groups beyond Y/(8*depth) bands idle;
                              K = 1 where even two bands of 16 rows do not fit).
                              For depth > 0 the library allocates a save area
                              of 256*depth*block_threads bytes per persistent
                              workgroup (and as much again per part of a split
                              realization). */
    int32_t max_parts;     /* 1, 2 or 4: a blocked realization whose work in
                              the epoch exceeds the average per persistent
                              workgroup is split into up to max_parts parts
                              (powers of two) that run on as many workgroups at
                              once, with one barrier among them per pass
                              (bands of at least 8*K rows, K <= depth).  At
                              most one part per compute unit in all, the
                              longest realizations first. */
} sca_batch_config;

typedef struct sca_slot_info {
    int64_t X, Y, t, n_mcs;
    uint64_t seed;
    void* slopes_dev;      /* the realization's S[2][2][Y][W] inside the arena */
    int64_t* h0_dev;       /* its h(0,0) inside the arena */
} sca_slot_info;

/* Arena bytes one realization of size X x Y occupies (256-byte aligned). */
size_t sca_batch_state_bytes(int64_t X, int64_t Y);

/* Creates a batch with room for max_slots realizations whose states are
 * placed in the caller-owned device arena [arena_dev, arena_dev+arena_bytes)
 * (the HBM budget).  Work is enqueued on hip_stream.  The library allocates
 * the descriptor table (about 160 bytes per slot) and pinned staging. */
int sca_batch_create(sca_batch** out, int32_t max_slots, void* arena_dev, size_t arena_bytes,
                     void* hip_stream);

int sca_batch_set_config(sca_batch* b, const sca_batch_config* cfg);
int sca_batch_get_config(const sca_batch* b, sca_batch_config* cfg);

/* Admits n realizations, all or none: SCA_EBUSY if the free slots or the free
 * arena space do not suffice (nothing is changed then).  Each admitted
 * realization starts from the flat surface at t = 0; slots_out[i] receives
 * its slot.  Asynchronous (the flat initialisation is enqueued). */
int sca_batch_admit(sca_batch* b, const sca_req* reqs, int32_t n, int32_t* slots_out);

/* One epoch: every admitted realization with work left advances
 * min(mcs_epoch, n_mcs - t) MCS, all in one persistent launch.  *active_out
 * (optional) receives the number of realizations that ran.  Asynchronous. */
int sca_batch_run(sca_batch* b, int64_t mcs_epoch, int32_t* active_out);

/* One epoch with a work quota instead of a fixed MCS count: every admitted
 * realization with work left advances max(1, site_updates / (X*Y)) MCS
 * (clamped to its budget), so small lattices cover many MCS in the time a
 * large one covers a few.  Results do not depend on the epoch lengths.
 * Asynchronous. */
int sca_batch_run_work(sca_batch* b, int64_t site_updates, int32_t* active_out);

/* Slot description; SCA_EINVAL for a free slot.  t is the MCS count the slot
 * will have reached once the enqueued epochs have run. */
int sca_batch_slot(const sca_batch* b, int32_t slot, sca_slot_info* out);

/* Exact moments {N, sum h, sum h^2} and W^2 of one slot's current state
 * (as sca_roughness).  Synchronizes. */
int sca_batch_roughness(sca_batch* b, int32_t slot, int64_t out3[3], double* w2);

/* Frees a slot and its arena space (after the enqueued work that uses it). */
int sca_batch_release(sca_batch* b, int32_t slot);

/* Frees the batch (after synchronizing its stream); never frees the arena. */
void sca_batch_destroy(sca_batch* b);

/* Static description of a status code. */
const char* sca_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SCA_H */

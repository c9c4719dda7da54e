// sca_internal.hpp -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep_args.hpp"

namespace sca {

// Launches one half-step; returns the launch status.
hipError_t launch_halfstep(const SweepArgs& a, XiMode mode, bool has_q, hipStream_t stream);

// `depth` MCS (2*depth half-steps from MCS a.t on) in one pass, reading src
// and writing dst (both S[2][2][Y][W]); one workgroup per band of `band` rows.
// The deepest pass depends on the kind of acceptance words: mode and, in
// mask mode, the number of draws (0: p and q in {0, 1}, which allows the
// deepest passes).
int max_fused_depth(int32_t W, XiMode mode, int32_t ndraw);
bool fused_supported(int32_t W, int64_t Y, int32_t band, int32_t depth, XiMode mode, int32_t ndraw);
hipError_t launch_mcs_fused(const SweepArgs& a, XiMode mode, bool has_q, const uint64_t* src, uint64_t* dst,
                            int32_t band, int32_t depth, hipStream_t stream);

// Name of the kernel (with its template arguments) that launch_mcs_fused and
// launch_halfstep run for these arguments; written next to their dispatch.
void fused_kernel_name(const SweepArgs& a, XiMode mode, bool has_q, int32_t depth, char* out, size_t n);
void halfstep_kernel_name(int32_t W, XiMode mode, bool has_q, char* out, size_t n);

// Flat initial surface into S and h0 = 0.
hipError_t launch_flat_init(uint64_t* S, int64_t Y, int32_t W, int32_t nb, int64_t* h0,
                            hipStream_t stream);

// The flat surface for a list of lattices in one launch (device table of
// items); meant for small states such as an ensemble's realizations.
struct FlatItem {
    uint64_t* S;
    int64_t* h0;
    int64_t plane;   // Y*W
    uint64_t valid;  // used bits of a word
};
FlatItem flat_item(uint64_t* S, int64_t Y, int32_t W, int32_t nb, int64_t* h0);
hipError_t launch_flat_init_many(const FlatItem* items_dev, int32_t n, hipStream_t stream);

// Per-row sums for the moments (and the two-time sums when snap != nullptr):
// rows[y*3 + {0,1,2}] = {sum_x P_t, sum_x P_t^2 (or sum_x P_t P_s), sum_x P_s}
// with P(x) = h(x,y) - h(0,y).
hipError_t launch_row_sums(const uint64_t* S, const uint64_t* snap, int64_t X, int64_t Y,
                           int32_t W, int32_t nb, int64_t* rows, hipStream_t stream);

// Column prefix h(0,y) and the final exact sums (128-bit) into res[]:
// res = {S1 lo,hi, S2 lo,hi, S3 lo,hi}; see measure.hip for their meaning.
hipError_t launch_combine(const uint64_t* S, const int64_t* h0, const uint64_t* snap,
                          const int64_t* snap_h0, int64_t X, int64_t Y, int32_t W,
                          const int64_t* rows, int64_t* col, int64_t* res, hipStream_t stream);

// Heights of rows [y0, y0+ny) into out (needs col[] from launch_combine).
hipError_t launch_heights(const uint64_t* S, int64_t X, int64_t Y, int32_t W, int32_t nb,
                          const int64_t* col, int64_t y0, int64_t ny, int32_t* out,
                          hipStream_t stream);

// One realization of an ensemble epoch (device table, one entry per slot).
struct BatchDesc {
    uint64_t* S;       // state S[2][2][Y][W] in the arena
    int64_t* h0;       // origin height in the arena
    int64_t plane;     // Y*W
    int32_t W, Y, nb;
    int32_t mode;      // 0 mask, 1 per-site
    uint32_t k0, k1;
    uint32_t dig_p, dig_q;
    int32_t ndraw;
    int32_t has_q;
    uint32_t thr_p, thr_q;
    uint64_t all_p, all_q;
    uint32_t t;        // MCS index at the start of the epoch
    uint32_t n_run;    // MCS to advance in this epoch (0: skip)
    // Temporally blocked passes (phase 1 of the persistent kernel), set by
    // the host per epoch: depth > 0 runs passes of `depth` MCS on bands of
    // one group of W lanes each, `bands` bands per workgroup; a realization
    // split into parts > 1 runs on as many workgroups (part m owns bands
    // m*bands .. (m+1)*bands-1) that meet at a barrier on counter
    // sync[sync_idx] and keep their band save slots in `save` (contiguous
    // for all parts); parts == 1 uses the workgroup's own save area.
    int32_t depth;
    int32_t bands;
    int32_t parts;
    int32_t sync_idx;
    uint64_t* save;
};

// Arguments of the persistent ensemble kernel; the table, the order and the
// item count live in device memory so that one captured graph serves every
// epoch.
struct BatchLaunch {
    const BatchDesc* desc;
    const int32_t* order;    // slots in processing order
    const int32_t* n_items;  // number of entries of order to process
    int32_t* queue;          // work counter, reset to 0 before each launch
    int32_t lds_bytes;       // dynamic LDS per workgroup; states up to this size run from LDS
    int32_t depth;           // MCS per blocked pass in global memory (0: none)
    uint64_t* save;          // per-workgroup save areas for the blocked passes
    int64_t save_words;      // words per workgroup: 32 * depth * block threads
    int32_t* sync;           // arrival counters of split realizations, zeroed before each launch
    int32_t n_sync;          // number of counters
    int32_t* err;            // set if a barrier wait of a split realization ran out of patience
};

// Save-area words per persistent workgroup (and per part of a split
// realization) for blocked passes of up to `depth` MCS: each band (one group
// of W lanes) keeps its first and its last 2K rows, two sets of each, four
// arrays, one word per lane.
constexpr int64_t blocked_save_words(int depth, int block_threads)
{
    return 32 * (int64_t)depth * block_threads;
}

// An item of the work queue: slot in the low 20 bits, part in the bits above.
constexpr int kItemSlotBits = 20;
// Most parts one realization is split into.
constexpr int kMaxParts = 4;
// Deepest blocked pass of the persistent kernel (one 512-thread workgroup per
// CU; other shapes go to 2 MCS).
constexpr int kMaxBatchDepth = 4;

// The blocked-pass geometry of one realization split into `parts`
// workgroups: a depth K <= max_depth and a number of bands per workgroup (at
// most one per group of W lanes, groups beyond it idle) that leave every
// band at least 8K rows.  One workgroup keeps K = max_depth and idles groups
// if it must; a split realization first lowers K to keep every group busy
// (its parts are the ensemble's critical path).  Returns false if no K >= 1
// works (one workgroup needs two bands).
inline bool blocked_plan(int W, int Y, int max_depth, int block_threads, int parts, int* depth, int* bands)
{
    if (max_depth <= 0 || parts < 1 || (W != 8 && W != 16 && W != 32 && W != 64)) return false;
    const int all = block_threads / W;
    if (parts > 1)
        for (int K = max_depth; K >= 1; --K)
            if (Y / (all * parts) >= 8 * K && Y % (all * parts) == 0) {
                *depth = K;
                *bands = all;
                return true;
            }
    for (int K = max_depth; K >= 1; --K) {
        int nb = all;
        while (nb > 1 && Y / (nb * parts) < 8 * K) nb >>= 1;
        if (nb * parts >= 2 && Y / (nb * parts) >= 8 * K && Y % (nb * parts) == 0) {
            *depth = K;
            *bands = nb;
            return true;
        }
    }
    return false;
}

hipError_t launch_ensemble(const BatchLaunch& L, int block_threads, int words_per_lane, int grid, hipStream_t stream);
hipError_t launch_counter_reset(int32_t* counter, int32_t* sync, int32_t n_sync, hipStream_t stream);
// Workgroups of the persistent kernel with this shape that one compute unit
// holds at once (0 if unknown).
int ensemble_occupancy(int block_threads, int words_per_lane, int lds_bytes, int depth);

hipError_t launch_philox_rate(int64_t threads, int32_t calls, uint32_t* sink, hipStream_t stream);

hipError_t launch_philox_test(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t* out, hipStream_t stream);

}  // namespace sca

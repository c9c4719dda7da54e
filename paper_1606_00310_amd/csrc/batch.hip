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
// workgroup works on them.  Same-parity sites share no bond, so within a
// half-step every word is read and written by exactly one lane; the barrier
// between half-steps (a workgroup-scope release/acquire) orders them.
#include "halfstep.hpp"
#include "sca_internal.hpp"

namespace sca {
namespace {

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

template <int BLOCK, int IW>
__global__ __launch_bounds__(BLOCK) void ensemble_kernel(BatchLaunch L)
{
    constexpr int NWAVES = BLOCK / 64;
    extern __shared__ uint64_t lds[];
    __shared__ int32_t s_item;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t n_items = *L.n_items;

    for (;;) {
        __syncthreads();  // the previous realization is finished (LDS and s_item reuse)
        if (threadIdx.x == 0) s_item = atomicAdd(L.queue, 1);
        __syncthreads();
        const int32_t item = s_item;
        if (item >= n_items) break;  // every wave of every workgroup gets here once the counter passes n
        const BatchDesc d = L.desc[L.order[item]];
        if (d.n_run == 0) continue;

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

__global__ void counter_reset_kernel(int32_t* c) { *c = 0; }

}  // namespace

hipError_t launch_ensemble(const BatchLaunch& L, int block_threads, int words_per_lane, int grid, hipStream_t stream)
{
    const size_t lds = (size_t)L.lds_bytes;
    const int key = block_threads * 4 + words_per_lane;
    switch (key) {
    case 256 * 4 + 1: hipLaunchKernelGGL((ensemble_kernel<256, 1>), dim3(grid), dim3(256), lds, stream, L); break;
    case 512 * 4 + 1: hipLaunchKernelGGL((ensemble_kernel<512, 1>), dim3(grid), dim3(512), lds, stream, L); break;
    case 1024 * 4 + 1: hipLaunchKernelGGL((ensemble_kernel<1024, 1>), dim3(grid), dim3(1024), lds, stream, L); break;
    case 256 * 4 + 2: hipLaunchKernelGGL((ensemble_kernel<256, 2>), dim3(grid), dim3(256), lds, stream, L); break;
    case 512 * 4 + 2: hipLaunchKernelGGL((ensemble_kernel<512, 2>), dim3(grid), dim3(512), lds, stream, L); break;
    case 1024 * 4 + 2: hipLaunchKernelGGL((ensemble_kernel<1024, 2>), dim3(grid), dim3(1024), lds, stream, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_counter_reset(int32_t* counter, hipStream_t stream)
{
    hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(1), 0, stream, counter);
    return hipGetLastError();
}

}  // namespace sca

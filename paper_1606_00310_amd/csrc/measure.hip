// measure.hip -- flat initial state, heights, exact height moments and
// two-time sums on gfx950.
//
// Heights are not stored; they follow from the slopes (Sec. II-A keeps two
// slope bits per site) and the tracked origin height h(0,0):
//   h(x,y) = c(y) + P_y(x),  c(y) = h(0,0) + sum_{j=1..y} (2 sy(0,j) - 1),
//   P_y(x) = sum_{i=1..x} (2 sx(i,y) - 1).
// Row y's x-slopes interleave two words per 128 sites: even x in the x-array
// of parity y&1, odd x in that of parity 1-(y&1), bit x>>1.
//
// Moments decompose exactly: for a 128-site word with base B (= P at the
// site before it) and local prefix d_i,
//   sum (B + d_i) = n B + sum d_i,   sum (B + d_i)^2 = n B^2 + 2 B sum d_i + sum d_i^2,
// so each lane forms int32 local sums, a wave scan forms the bases, and the
// per-row int64 results are combined with c(y) by one workgroup in 128-bit
// integer arithmetic.  Nothing is rounded at any stage.
#include "sca_internal.hpp"

namespace sca {
namespace {

constexpr int kBlock = 256;

__global__ void flat_init_kernel(uint64_t* S, int64_t plane, uint64_t valid, int64_t* h0)
{
    const int64_t n = 4 * plane;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int parity = (int)((i / plane) & 1);  // arrays ordered S[d][parity]
        S[i] = parity ? valid : 0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *h0 = 0;
}

// The flat surface for many lattices at once: workgroup i initialises items
// i, i + gridDim.x, ... (their states are small: one admission of an
// ensemble issues one launch instead of one per realization).
__global__ __launch_bounds__(kBlock) void flat_init_many_kernel(const FlatItem* items, int32_t n)
{
    for (int32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const FlatItem f = items[it];
        const int64_t words = 4 * f.plane;
        for (int64_t i = threadIdx.x; i < words; i += kBlock) {
            const int parity = (int)((i / f.plane) & 1);  // arrays ordered S[d][parity]
            f.S[i] = parity ? f.valid : 0ull;
        }
        if (threadIdx.x == 0) *f.h0 = 0;
    }
}

// Local sums of one word pair (even-x word E, odd-x word O) over its 2*nb
// sites; the global site x = 0 contributes no step (skip0).
struct WordSums {
    int32_t tot;  // sum of the steps e_i
    int32_t sd;   // sum of prefixes d_i
    int32_t sd2;  // sum of d_i^2
};

__device__ __forceinline__ WordSums word_sums(uint64_t E, uint64_t O, int nb, bool skip0)
{
    int32_t d = 0, sd = 0, sd2 = 0;
    for (int k = 0; k < nb; ++k) {
        if (!(skip0 && k == 0)) d += 2 * (int32_t)((E >> k) & 1ull) - 1;
        sd += d;
        sd2 += d * d;
        d += 2 * (int32_t)((O >> k) & 1ull) - 1;
        sd += d;
        sd2 += d * d;
    }
    return {d, sd, sd2};
}

// Two-time version: prefixes of two states in lockstep and their product sum.
__device__ __forceinline__ void word_sums2(uint64_t Et, uint64_t Ot, uint64_t Es, uint64_t Os, int nb, bool skip0,
                                           int32_t& tt, int32_t& sdt, int32_t& ts, int32_t& sds, int32_t& sdd)
{
    int32_t dt = 0, ds = 0;
    sdt = sds = sdd = 0;
    for (int k = 0; k < nb; ++k) {
        if (!(skip0 && k == 0)) {
            dt += 2 * (int32_t)((Et >> k) & 1ull) - 1;
            ds += 2 * (int32_t)((Es >> k) & 1ull) - 1;
        }
        sdt += dt; sds += ds; sdd += dt * ds;
        dt += 2 * (int32_t)((Ot >> k) & 1ull) - 1;
        ds += 2 * (int32_t)((Os >> k) & 1ull) - 1;
        sdt += dt; sds += ds; sdd += dt * ds;
    }
    tt = dt;
    ts = ds;
}

// Inclusive scan across the G lanes of a row group.
template <int G>
__device__ __forceinline__ int64_t group_incl_scan(int64_t v, int gl)
{
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const int64_t o = __shfl_up(v, off, G);
        if (gl >= off) v += o;
    }
    return v;
}

template <int G>
__device__ __forceinline__ int64_t group_sum(int64_t v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// rows[3y..3y+2]: {sum P_t, sum P_t^2, 0} or, with a snapshot,
// {sum P_t, sum P_t P_s, sum P_s}.
template <int G, bool TWO>
__global__ __launch_bounds__(kBlock) void row_sums_kernel(const uint64_t* S, const uint64_t* snap, int64_t Y,
                                                         int32_t W, int32_t nb, int64_t plane, int64_t* rows)
{
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t y_raw = wave * (64 / G) + lane / G;
    const bool active = y_raw < Y;
    const int64_t y = active ? y_raw : 0;
    const int pe = (int)(y & 1);
    const uint64_t* Et = S + (int64_t)pe * plane + y * W;        // x-slopes of even x
    const uint64_t* Ot = S + (int64_t)(1 - pe) * plane + y * W;  // x-slopes of odd x
    const uint64_t* Es = TWO ? snap + (int64_t)pe * plane + y * W : nullptr;
    const uint64_t* Os = TWO ? snap + (int64_t)(1 - pe) * plane + y * W : nullptr;

    int64_t acc1 = 0, acc2 = 0, acc3 = 0, carry_t = 0, carry_s = 0;
    for (int c = 0; c < W / G; ++c) {
        const int w = c * G + gl;
        const int64_t n = 2 * (int64_t)nb - (w == 0 ? 1 : 0);
        if constexpr (!TWO) {
            const WordSums s = word_sums(Et[w], Ot[w], nb, w == 0);
            const int64_t incl = group_incl_scan<G>((int64_t)s.tot, gl);
            const int64_t b = carry_t + incl - s.tot;
            carry_t += __shfl(incl, (lane & ~(G - 1)) + G - 1);
            acc1 += n * b + s.sd;
            acc2 += n * b * b + 2 * b * s.sd + s.sd2;
        } else {
            int32_t tt, sdt, ts, sds, sdd;
            word_sums2(Et[w], Ot[w], Es[w], Os[w], nb, w == 0, tt, sdt, ts, sds, sdd);
            const int64_t it = group_incl_scan<G>((int64_t)tt, gl);
            const int64_t is = group_incl_scan<G>((int64_t)ts, gl);
            const int64_t bt = carry_t + it - tt;
            const int64_t bs = carry_s + is - ts;
            carry_t += __shfl(it, (lane & ~(G - 1)) + G - 1);
            carry_s += __shfl(is, (lane & ~(G - 1)) + G - 1);
            acc1 += n * bt + sdt;
            acc2 += n * bt * bs + bt * sds + bs * sdt + sdd;
            acc3 += n * bs + sds;
        }
    }
    acc1 = group_sum<G>(acc1);
    acc2 = group_sum<G>(acc2);
    acc3 = group_sum<G>(acc3);
    if (active && gl == 0) {
        rows[3 * y + 0] = acc1;
        rows[3 * y + 1] = acc2;
        rows[3 * y + 2] = acc3;
    }
}

constexpr int kCombine = 1024;

// Exclusive block-wide scan of one int64 per thread (1024 threads).
__device__ int64_t block_excl_scan(int64_t v, int64_t* lds_waves)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) lds_waves[wid] = incl;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < wid; ++k) before += lds_waves[k];
    __syncthreads();
    return before + incl - v;
}

// Column prefix c(y) for every row (written to col) and the exact totals:
//   moments:   res = {sum h, sum h^2, 0}
//   two-time:  res = {sum h_t, sum h_t h_s, sum h_s}
// each as a (lo, hi) pair of a 128-bit integer.
__global__ __launch_bounds__(kCombine) void combine_kernel(const uint64_t* S, const int64_t* h0, const uint64_t* snap,
                                                          const int64_t* snap_h0, int64_t X, int64_t Y, int32_t W,
                                                          int64_t plane, const int64_t* rows, int64_t* col,
                                                          int64_t* res)
{
    __shared__ int64_t lds_waves[kCombine / 64];
    __shared__ __int128 lds_red[kCombine / 64][3];
    const bool two = (snap != nullptr);
    const int64_t per = (Y + kCombine - 1) / kCombine;
    const int64_t ya = (int64_t)threadIdx.x * per;
    const int64_t yb = ya + per < Y ? ya + per : Y;

    // steps down column 0: e_y = 2 sy(0,y) - 1 for y >= 1; sy(0,y) is bit 0 of
    // word 0 of row y in the y-array of parity y&1.
    auto step = [&](const uint64_t* base, int64_t yy) -> int64_t {
        if (yy == 0) return 0;
        const uint64_t wrd = base[(int64_t)(2 + (yy & 1)) * plane + yy * W];
        return 2 * (int64_t)(wrd & 1ull) - 1;
    };
    int64_t loc_t = 0, loc_s = 0;
    for (int64_t yy = ya; yy < yb; ++yy) {
        loc_t += step(S, yy);
        if (two) loc_s += step(snap, yy);
    }
    const int64_t ex_t = block_excl_scan(loc_t, lds_waves);
    const int64_t ex_s = two ? block_excl_scan(loc_s, lds_waves) : 0;

    int64_t ct = *h0 + ex_t;
    int64_t cs = two ? *snap_h0 + ex_s : 0;
    __int128 t1 = 0, t2 = 0, t3 = 0;
    for (int64_t yy = ya; yy < yb; ++yy) {
        ct += step(S, yy);
        if (col) col[yy] = ct;
        const int64_t r1 = rows ? rows[3 * yy] : 0, r2 = rows ? rows[3 * yy + 1] : 0, r3 = rows ? rows[3 * yy + 2] : 0;
        if (!two) {
            t1 += (__int128)X * ct + r1;
            t2 += (__int128)X * ct * ct + (__int128)2 * ct * r1 + r2;
        } else {
            cs += step(snap, yy);
            t1 += (__int128)X * ct + r1;
            t2 += (__int128)X * ct * cs + (__int128)ct * r3 + (__int128)cs * r1 + r2;
            t3 += (__int128)X * cs + r3;
        }
    }
    if (!res) return;
    // block reduction of the three 128-bit sums
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __int128 v[3] = {t1, t2, t3};
    for (int k = 0; k < 3; ++k) {
        int64_t lo = (int64_t)(uint64_t)v[k];
        int64_t hi = (int64_t)(v[k] >> 64);
        // reduce as 128-bit via lane shuffles of both halves
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t olo = (uint64_t)__shfl_down(lo, off, 64);
            const int64_t ohi = __shfl_down(hi, off, 64);
            const __int128 a = ((__int128)hi << 64) | (uint64_t)lo;
            const __int128 b = ((__int128)ohi << 64) | olo;
            const __int128 s = (lane + off < 64) ? a + b : a;
            lo = (int64_t)(uint64_t)s;
            hi = (int64_t)(s >> 64);
        }
        if (lane == 0) lds_red[wid][k] = ((__int128)hi << 64) | (uint64_t)lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) {
            __int128 s = 0;
            for (int q = 0; q < kCombine / 64; ++q) s += lds_red[q][k];
            res[2 * k] = (int64_t)(uint64_t)s;
            res[2 * k + 1] = (int64_t)(s >> 64);
        }
    }
}

// Heights of rows [y0, y0+ny): each row group forms the word bases of a
// chunk of G words, parks (E, O, base) in LDS and then writes the chunk's
// sites with consecutive lanes on consecutive x.
template <int G>
__global__ __launch_bounds__(kBlock) void heights_kernel(const uint64_t* S, int64_t X, int32_t W, int32_t nb,
                                                        int64_t plane, const int64_t* col, int64_t y0, int64_t ny,
                                                        int32_t* out)
{
    __shared__ uint64_t lE[kBlock], lO[kBlock];
    __shared__ int64_t lB[kBlock];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int slot0 = threadIdx.x & ~(G - 1);  // LDS slot of the group's first lane
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t r_raw = wave * (64 / G) + lane / G;
    const bool active = r_raw < ny;
    const int64_t y = y0 + (active ? r_raw : 0);
    const int pe = (int)(y & 1);
    const uint64_t* Er = S + (int64_t)pe * plane + y * W;
    const uint64_t* Or = S + (int64_t)(1 - pe) * plane + y * W;
    const int64_t cy = col[y];
    const int spw = 2 * nb;  // sites per word
    int32_t* orow = out + (active ? r_raw : 0) * X;

    int64_t carry = 0;
    for (int c = 0; c < W / G; ++c) {
        const int w = c * G + gl;
        const uint64_t E = Er[w], O = Or[w];
        const uint64_t vmask = (nb == 64) ? ~0ull : ((1ull << nb) - 1ull);
        int64_t ups = __popcll(E & vmask) + __popcll(O & vmask) - (w == 0 ? (int64_t)(E & 1ull) : 0);
        const int64_t tot = 2 * ups - (spw - (w == 0 ? 1 : 0));
        const int64_t incl = group_incl_scan<G>(tot, gl);
        lE[threadIdx.x] = E;
        lO[threadIdx.x] = O;
        lB[threadIdx.x] = carry + incl - tot;
        carry += __shfl(incl, (lane & ~(G - 1)) + G - 1);
        __syncthreads();
        for (int m = 0; m < spw; ++m) {
            const int s = m * G + gl;      // site within the chunk
            const int ww = s / spw;        // word within the chunk
            const int i = s - ww * spw;    // site within the word
            const uint64_t e = lE[slot0 + ww], o = lO[slot0 + ww];
            const int he = (i >> 1) + 1, ho = (i + 1) >> 1;  // even / odd sites among 0..i
            const uint64_t me = he >= 64 ? ~0ull : ((1ull << he) - 1ull);
            const uint64_t mo = ho >= 64 ? ~0ull : ((1ull << ho) - 1ull);
            const bool first = (c == 0 && ww == 0);
            const int64_t u = __popcll(e & me) + __popcll(o & mo) - (first ? (int64_t)(e & 1ull) : 0);
            const int64_t cnt = i + 1 - (first ? 1 : 0);
            const int64_t h = cy + lB[slot0 + ww] + 2 * u - cnt;
            if (active) orow[(int64_t)c * G * spw + s] = (int32_t)h;
        }
        __syncthreads();
    }
}

template <int G, bool TWO>
hipError_t launch_rows_g(const uint64_t* S, const uint64_t* snap, int64_t Y, int32_t W, int32_t nb, int64_t plane,
                         int64_t* rows, hipStream_t stream)
{
    const int64_t rows_per_block = (kBlock / 64) * (64 / G);
    hipLaunchKernelGGL((row_sums_kernel<G, TWO>), dim3((unsigned)((Y + rows_per_block - 1) / rows_per_block)),
                       dim3(kBlock), 0, stream, S, snap, Y, W, nb, plane, rows);
    return hipGetLastError();
}

template <bool TWO>
hipError_t launch_rows(const uint64_t* S, const uint64_t* snap, int64_t Y, int32_t W, int32_t nb, int64_t plane,
                       int64_t* rows, hipStream_t stream)
{
    switch (W) {
    case 1: return launch_rows_g<1, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    case 2: return launch_rows_g<2, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    case 4: return launch_rows_g<4, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    case 8: return launch_rows_g<8, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    case 16: return launch_rows_g<16, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    case 32: return launch_rows_g<32, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    default: return launch_rows_g<64, TWO>(S, snap, Y, W, nb, plane, rows, stream);
    }
}

template <int G>
hipError_t launch_heights_g(const uint64_t* S, int64_t X, int32_t W, int32_t nb, int64_t plane, const int64_t* col,
                            int64_t y0, int64_t ny, int32_t* out, hipStream_t stream)
{
    const int64_t rows_per_block = (kBlock / 64) * (64 / G);
    hipLaunchKernelGGL((heights_kernel<G>), dim3((unsigned)((ny + rows_per_block - 1) / rows_per_block)),
                       dim3(kBlock), 0, stream, S, X, W, nb, plane, col, y0, ny, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_flat_init(uint64_t* S, int64_t Y, int32_t W, int32_t nb, int64_t* h0, hipStream_t stream)
{
    const int64_t plane = Y * W;
    const uint64_t valid = (nb == 64) ? ~0ull : ((1ull << nb) - 1ull);
    int64_t blocks = (4 * plane + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(flat_init_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, S, plane, valid, h0);
    return hipGetLastError();
}

FlatItem flat_item(uint64_t* S, int64_t Y, int32_t W, int32_t nb, int64_t* h0)
{
    return FlatItem{S, h0, Y * W, (nb == 64) ? ~0ull : ((1ull << nb) - 1ull)};
}

hipError_t launch_flat_init_many(const FlatItem* items_dev, int32_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int32_t grid = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(flat_init_many_kernel, dim3((unsigned)grid), dim3(kBlock), 0, stream, items_dev, n);
    return hipGetLastError();
}

hipError_t launch_row_sums(const uint64_t* S, const uint64_t* snap, int64_t X, int64_t Y, int32_t W, int32_t nb,
                           int64_t* rows, hipStream_t stream)
{
    (void)X;
    const int64_t plane = Y * W;
    return snap ? launch_rows<true>(S, snap, Y, W, nb, plane, rows, stream)
                : launch_rows<false>(S, nullptr, Y, W, nb, plane, rows, stream);
}

hipError_t launch_combine(const uint64_t* S, const int64_t* h0, const uint64_t* snap, const int64_t* snap_h0,
                          int64_t X, int64_t Y, int32_t W, const int64_t* rows, int64_t* col, int64_t* res,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(kCombine), 0, stream, S, h0, snap, snap_h0, X, Y, W,
                       Y * (int64_t)W, rows, col, res);
    return hipGetLastError();
}

hipError_t launch_heights(const uint64_t* S, int64_t X, int64_t Y, int32_t W, int32_t nb, const int64_t* col,
                          int64_t y0, int64_t ny, int32_t* out, hipStream_t stream)
{
    const int64_t plane = Y * W;
    switch (W) {
    case 1: return launch_heights_g<1>(S, X, W, nb, plane, col, y0, ny, out, stream);
    case 2: return launch_heights_g<2>(S, X, W, nb, plane, col, y0, ny, out, stream);
    case 4: return launch_heights_g<4>(S, X, W, nb, plane, col, y0, ny, out, stream);
    case 8: return launch_heights_g<8>(S, X, W, nb, plane, col, y0, ny, out, stream);
    case 16: return launch_heights_g<16>(S, X, W, nb, plane, col, y0, ny, out, stream);
    case 32: return launch_heights_g<32>(S, X, W, nb, plane, col, y0, ny, out, stream);
    default: return launch_heights_g<64>(S, X, W, nb, plane, col, y0, ny, out, stream);
    }
}

}  // namespace sca

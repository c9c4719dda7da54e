// api.hip -- the C ABI declared in include/sca.h.
//
// Host side only: argument checks, the classification of p and q into the
// bit-mask path (dyadic) or the per-site compare path, the MCS loop of two
// half-step launches per MCS (even then odd sublattice, Sec. I-A), and the
// device-to-host read-back of exact sums.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "sca.h"
#include "sca_internal.hpp"

struct sca_ctx {
    int64_t X = 0, Y = 0;
    int32_t W = 0, nb = 0;
    uint64_t seed = 0;
    uint64_t* S = nullptr;     // caller-owned state
    int64_t* aux = nullptr;    // caller-owned aux; aux[0] = h(0,0)
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t t = 0;
    bool failed = false;
    int64_t* ws = nullptr;     // library-owned: rows[3Y], col[Y], res[8]
    hipStream_t capture = nullptr;  // private stream for hipGraph capture (created on first use)
    uint64_t* alt = nullptr;        // caller-owned second state for the blocked passes (sca_set_pass_buffer)
    int32_t depth = -1;             // MCS per fused pass; -1 = automatic, 0 = never fuse
    int32_t band = 0;               // rows per workgroup in a fused pass; 0 = automatic
};

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool valid_size(int64_t X, int64_t Y)
{
    return is_pow2(X) && is_pow2(Y) && X >= 4 && Y >= 4 && X <= (1 << 17) && Y <= (1 << 17);
}

bool valid_prob(double r) { return r >= 0.0 && r <= 1.0; }  // false for NaN

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(sca_ctx* c)
{
    if (c) c->failed = true;
    return SCA_EDEVICE;
}

int64_t* ws_rows(sca_ctx* c) { return c->ws; }
int64_t* ws_col(sca_ctx* c) { return c->ws + 3 * c->Y; }
int64_t* ws_res(sca_ctx* c) { return c->ws + 4 * c->Y; }

// Acceptance parameters of one probability.
struct ProbCode {
    bool dyadic = false;
    int n = 0;              // fractional binary digits (dyadic)
    uint32_t digits = 0;    // bit i-1 = b_i
    uint64_t all = 0;       // ~0 when r == 1
    uint32_t thr = 0;       // per-site threshold, clamped to 32 bits
};

ProbCode classify(double r)
{
    ProbCode c;
    const double scaled = std::ldexp(r, 32);  // exact
    const double fl = std::floor(scaled);
    c.dyadic = (fl == scaled);
    const uint64_t T = (uint64_t)fl;          // 0 .. 2^32
    c.all = (T >= (1ull << 32)) ? ~0ull : 0ull;
    c.thr = (T >= (1ull << 32)) ? 0xffffffffu : (uint32_t)T;
    if (c.dyadic && T < (1ull << 32)) {
        const uint32_t v = (uint32_t)T;       // r = v / 2^32
        for (int i = 1; i <= 32; ++i)
            if ((v >> (32 - i)) & 1u) {
                c.digits |= 1u << (i - 1);
                c.n = i;
            }
    }
    return c;
}

int read_back(sca_ctx* c, const int64_t* dev, int64_t* host, size_t n)
{
    if (hipMemcpyAsync(host, dev, n * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return fail(c);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c);
    return SCA_OK;
}

__int128 join128(int64_t lo, int64_t hi) { return (__int128)(((unsigned __int128)(uint64_t)hi << 64) | (uint64_t)lo); }

bool fits64(__int128 v) { return v >= (__int128)INT64_MIN && v <= (__int128)INT64_MAX; }

// Exact moments of a state at S with origin height *h0, using ws (rows[3Y],
// col[Y], res[8]).  Returns SCA_OK, SCA_EDEVICE or SCA_EOVERFLOW.
int moments_of(const uint64_t* S, const int64_t* h0, int64_t X, int64_t Y, int32_t W, int32_t nb, int64_t* ws,
               hipStream_t stream, int64_t out3[3], double* w2)
{
    int64_t* rows = ws;
    int64_t* col = ws + 3 * Y;
    int64_t* res = ws + 4 * Y;
    if (sca::launch_row_sums(S, nullptr, X, Y, W, nb, rows, stream) != hipSuccess) return SCA_EDEVICE;
    if (sca::launch_combine(S, h0, nullptr, nullptr, X, Y, W, rows, col, res, stream) != hipSuccess)
        return SCA_EDEVICE;
    int64_t r[6];
    if (hipMemcpyAsync(r, res, sizeof r, hipMemcpyDeviceToHost, stream) != hipSuccess) return SCA_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return SCA_EDEVICE;
    const __int128 s1 = join128(r[0], r[1]), s2 = join128(r[2], r[3]);
    if (!fits64(s1) || !fits64(s2)) return SCA_EOVERFLOW;
    const __int128 N = (__int128)X * Y;
    out3[0] = (int64_t)N;
    out3[1] = (int64_t)s1;
    out3[2] = (int64_t)s2;
    if (w2) *w2 = (double)(N * s2 - s1 * s1) / ((double)N * (double)N);
    return SCA_OK;
}

// Runs `enqueue` on a private capture stream into a hipGraph, then launches
// the instantiated graph once on `stream`.  The launch is synchronized before
// the graph is released.
template <typename F>
hipError_t run_as_graph(hipStream_t& capture, hipStream_t stream, F enqueue)
{
    if (!capture && hipStreamCreateWithFlags(&capture, hipStreamNonBlocking) != hipSuccess) return hipErrorUnknown;
    if (hipStreamBeginCapture(capture, hipStreamCaptureModeRelaxed) != hipSuccess) return hipErrorUnknown;
    const hipError_t e1 = enqueue(capture);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(capture, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : hipErrorUnknown);
    }
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    e = hipGraphLaunch(exec, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    (void)hipGraphExecDestroy(exec);
    return e != hipSuccess ? e : es;
}

// What sca_step_ex runs for n_mcs MCS at (p, q): the acceptance path and the
// pass plan.  Groups of `depth` MCS run as fused passes alternating
// S -> pass buffer -> S (one HBM pass per group); the number of passes is
// kept even so that the caller's S holds the state after the call: an even
// number of `depth`-MCS passes, then the remainder r < 2*depth as two passes
// of ceil(r/2) and floor(r/2) MCS, or, for r = 1, two half-step launches.
// Automatic choice: a band per workgroup with enough waves to fill the chip
// and bands as tall as that allows; deep passes on tall bands (the halo costs
// 4*depth rows per band), shallower ones on short bands.  The per-site path
// is ALU-bound and runs unfused.
struct StepPlan {
    ProbCode P, Q;
    bool persite = false, has_q = false, draw_free = false;
    sca::XiMode mode = sca::XiMode::Mask;
    int32_t ndraw = 0;
    int32_t band = 0, depth = 0;
    int64_t n_pass = 0;
    int32_t tail1 = 0, tail2 = 0;
};

StepPlan make_plan(const sca_ctx* c, int64_t n_mcs, double p, double q, unsigned flags)
{
    StepPlan pl;
    pl.P = classify(p);
    pl.Q = classify(q);
    pl.persite = (flags & SCA_FORCE_PERSITE) || !pl.P.dyadic || !pl.Q.dyadic;
    pl.has_q = (q > 0.0);
    pl.mode = pl.persite ? sca::XiMode::PerSite : sca::XiMode::Mask;
    pl.ndraw = pl.persite ? 0 : (pl.P.n > pl.Q.n ? pl.P.n : pl.Q.n);
    const int64_t nw = c->W >= 512 ? 8 : (c->W >= 64 ? c->W / 64 : 1);
    // Without random words (p, q in {0, 1}) a pass costs little more than
    // a shallower one as long as its window fits the registers: 13 MCS at
    // X = 2^16 and 8 below (the register-window kernels), 6 at X = 2^17 (the
    // LDS-window kernel with 1024-thread workgroups), on bands of up to 256
    // rows (about one workgroup per CU); passes with draws are ALU-bound and
    // do best at 4 MCS on bands of up to 128 rows.
    pl.draw_free = !pl.persite && pl.ndraw == 0;
    int32_t band = c->band;
    if (band == 0) {
        int64_t b = pl.draw_free ? 256 : 128;
        while (b > 8 && c->Y / b < 2048 / nw) b >>= 1;
        band = (int32_t)b;
    }
    pl.band = band;
    const int32_t dmax = sca::max_fused_depth(c->W, pl.mode, pl.ndraw);
    int32_t depth = c->depth;
    if (depth < 0) {
        depth = pl.persite ? 0
                           : band >= 256 ? (pl.draw_free ? 13 : 4)
                           : band >= 128 ? (pl.draw_free ? 10 : 4)
                           : band >= 64 ? (pl.draw_free ? 5 : 3)
                           : band >= 32 ? 3
                           : band >= 16 ? 2
                                        : 1;
    }
    if (depth > dmax) depth = dmax;
    pl.depth = depth;
    const bool fuse = !(flags & SCA_NO_FUSE) && depth > 0 && n_mcs >= 2 &&
                      sca::fused_supported(c->W, c->Y, band, depth, pl.mode, pl.ndraw);
    pl.n_pass = fuse ? ((n_mcs / depth) & ~(int64_t)1) : 0;
    const int64_t rem = n_mcs - pl.n_pass * depth;
    pl.tail1 = (fuse && rem >= 2) ? (int32_t)((rem + 1) / 2) : 0;
    pl.tail2 = (fuse && rem >= 2) ? (int32_t)(rem / 2) : 0;
    return pl;
}

sca::SweepArgs sweep_args(const sca_ctx* c, const StepPlan& pl)
{
    sca::SweepArgs a{};
    a.S = c->S;
    a.plane = c->Y * c->W;
    a.W = c->W;
    a.Y = (int32_t)c->Y;
    a.nb = c->nb;
    a.k0 = (uint32_t)c->seed;
    a.k1 = (uint32_t)(c->seed >> 32);
    a.h0 = c->aux;
    a.all_p = pl.P.all;
    a.all_q = pl.Q.all;
    if (pl.persite) {
        a.thr_p = pl.P.thr;
        a.thr_q = pl.Q.thr;
    } else {
        a.dig_p = pl.P.digits;
        a.dig_q = pl.Q.digits;
        a.ndraw = pl.ndraw;
    }
    return a;
}

}  // namespace

extern "C" {

size_t sca_state_words(int64_t X, int64_t Y)
{
    if (!valid_size(X, Y)) return 0;
    return (size_t)(4 * Y * (X >= 128 ? X / 128 : 1));
}

const char* sca_strerror(int code)
{
    switch (code) {
    case SCA_OK: return "ok";
    case SCA_EINVAL: return "invalid argument";
    case SCA_ENOMEM: return "device allocation failed";
    case SCA_EDEVICE: return "HIP call failed";
    case SCA_EOVERFLOW: return "exact result does not fit its output type";
    case SCA_ESTATE: return "context failed earlier";
    case SCA_EBUSY: return "capacity limit reached";
    case SCA_ENOBUF: return "a blocked pass needs the caller's pass buffer (sca_set_pass_buffer)";
    case SCA_ESCRATCH: return "lattice exceeds the static scratch of the allocation-free call (Y > SCA_NOALLOC_MAX_Y)";
    default: return "unknown status";
    }
}

int sca_init(sca_ctx** out, int64_t X, int64_t Y, uint64_t seed, void* slopes_dev, int64_t* aux_dev,
             void* hip_stream)
{
    if (!out || !slopes_dev || !aux_dev || !valid_size(X, Y)) return SCA_EINVAL;
    *out = nullptr;
    sca_ctx* c = new (std::nothrow) sca_ctx;
    if (!c) return SCA_ENOMEM;
    c->X = X;
    c->Y = Y;
    c->W = (int32_t)(X >= 128 ? X / 128 : 1);
    c->nb = (int32_t)(X >= 128 ? 64 : X / 2);
    c->seed = seed;
    c->S = static_cast<uint64_t*>(slopes_dev);
    c->aux = aux_dev;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return SCA_EDEVICE; }
    if (hipMalloc(&c->ws, sizeof(int64_t) * (size_t)(4 * Y + 8)) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SCA_ENOMEM;
    }
    if (sca::launch_flat_init(c->S, Y, c->W, c->nb, c->aux, c->stream) != hipSuccess) {
        (void)hipFree(c->ws);
        delete c;
        return SCA_EDEVICE;
    }
    *out = c;
    return SCA_OK;
}

int sca_step_ex(sca_ctx* c, int64_t n_mcs, double p, double q, unsigned flags)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    if (n_mcs < 0 || !valid_prob(p) || !valid_prob(q) ||
        (flags & ~(SCA_FORCE_PERSITE | SCA_STEP_GRAPH | SCA_NO_FUSE)))
        return SCA_EINVAL;
    if (c->t + n_mcs > (int64_t)UINT32_MAX) return SCA_EINVAL;
    if (n_mcs == 0) return SCA_OK;
    const StepPlan pl = make_plan(c, n_mcs, p, q, flags);
    // the blocked passes alternate between S and the caller's pass buffer
    if (pl.n_pass + (pl.tail1 ? 2 : 0) > 0 && !c->alt) return SCA_ENOBUF;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);

    sca::SweepArgs a = sweep_args(c, pl);
    const int64_t t0 = c->t;
    const int64_t n_fused = pl.n_pass * pl.depth + pl.tail1 + pl.tail2;
    auto enqueue = [&](hipStream_t st) -> hipError_t {
        for (int64_t i = 0; i < pl.n_pass + (pl.tail1 ? 2 : 0); ++i) {
            const bool tail = i >= pl.n_pass;
            const int32_t d = !tail ? pl.depth : (i == pl.n_pass ? pl.tail1 : pl.tail2);
            a.t = (uint32_t)(t0 + (!tail ? i * pl.depth : pl.n_pass * pl.depth + (i == pl.n_pass ? 0 : pl.tail1)));
            const bool fwd = (i & 1) == 0;
            const hipError_t e = sca::launch_mcs_fused(a, pl.mode, pl.has_q, fwd ? c->S : c->alt,
                                                       fwd ? c->alt : c->S, pl.band, d, st);
            if (e != hipSuccess) return e;
        }
        for (int64_t i = n_fused; i < n_mcs; ++i) {
            a.t = (uint32_t)(t0 + i);
            for (int parity = 0; parity < 2; ++parity) {
                a.parity = parity;
                const hipError_t e = sca::launch_halfstep(a, pl.mode, pl.has_q, st);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    const hipError_t e = (flags & SCA_STEP_GRAPH) ? run_as_graph(c->capture, c->stream, enqueue) : enqueue(c->stream);
    if (e != hipSuccess) return fail(c);
    c->t += n_mcs;
    return SCA_OK;
}

int sca_plan_step(const sca_ctx* c, int64_t n_mcs, double p, double q, unsigned flags, sca_step_plan* out)
{
    if (!c || !out || n_mcs < 0 || !valid_prob(p) || !valid_prob(q) ||
        (flags & ~(SCA_FORCE_PERSITE | SCA_STEP_GRAPH | SCA_NO_FUSE)))
        return SCA_EINVAL;
    const StepPlan pl = make_plan(c, n_mcs, p, q, flags);
    std::memset(out, 0, sizeof *out);
    out->path = pl.persite ? SCA_PATH_PERSITE : (pl.draw_free ? SCA_PATH_DRAWFREE : SCA_PATH_MASK);
    out->band = pl.band;
    out->n_pass = pl.n_pass;
    out->depth = pl.n_pass > 0 ? pl.depth : 0;
    out->tail1 = pl.tail1;
    out->tail2 = pl.tail2;
    out->n_unfused = n_mcs - (pl.n_pass * pl.depth + pl.tail1 + pl.tail2);
    const sca::SweepArgs a = sweep_args(c, pl);
    if (pl.n_pass > 0) sca::fused_kernel_name(a, pl.mode, pl.has_q, pl.depth, out->kernel, sizeof out->kernel);
    else std::snprintf(out->kernel, sizeof out->kernel, "none");
    if (pl.tail1) sca::fused_kernel_name(a, pl.mode, pl.has_q, pl.tail1, out->tail_kernel, sizeof out->tail_kernel);
    else std::snprintf(out->tail_kernel, sizeof out->tail_kernel, "none");
    sca::halfstep_kernel_name(c->W, pl.mode, pl.has_q, out->halfstep_kernel, sizeof out->halfstep_kernel);
    return SCA_OK;
}

int sca_set_pass_buffer(sca_ctx* c, void* pass_dev, size_t bytes)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    const size_t need = sizeof(uint64_t) * (size_t)(4 * c->Y * c->W);
    if (!pass_dev) {
        c->alt = nullptr;
        return SCA_OK;
    }
    const uintptr_t a0 = (uintptr_t)pass_dev, s0 = (uintptr_t)c->S;
    if (bytes < need || (pass_dev && a0 < s0 + need && s0 < a0 + need)) return SCA_EINVAL;
    c->alt = static_cast<uint64_t*>(pass_dev);
    return SCA_OK;
}

int sca_reset(sca_ctx* c)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    if (sca::launch_flat_init(c->S, c->Y, c->W, c->nb, c->aux, c->stream) != hipSuccess) return fail(c);
    c->t = 0;
    return SCA_OK;
}

int sca_restore(sca_ctx* c, const void* snap_dev, int64_t t)
{
    if (!c || !snap_dev || t < 0 || t > (int64_t)UINT32_MAX) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    const size_t words = (size_t)(4 * c->Y * c->W);
    const uint64_t* src = static_cast<const uint64_t*>(snap_dev);
    if (hipMemcpyAsync(c->S, src, words * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c);
    if (hipMemcpyAsync(c->aux, src + words, sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c);
    c->t = t;
    return SCA_OK;
}

int sca_step(sca_ctx* c, int64_t n_mcs, double p, double q) { return sca_step_ex(c, n_mcs, p, q, 0u); }

int sca_debug_halfstep(sca_ctx* c, int parity, const uint64_t* xi_p_dev, const uint64_t* xi_q_dev)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    if ((parity != 0 && parity != 1) || !xi_p_dev || !xi_q_dev) return SCA_EINVAL;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    sca::SweepArgs a{};
    a.S = c->S;
    a.plane = c->Y * c->W;
    a.W = c->W;
    a.Y = (int32_t)c->Y;
    a.nb = c->nb;
    a.parity = parity;
    a.t = (uint32_t)c->t;
    a.xi_p = xi_p_dev;
    a.xi_q = xi_q_dev;
    a.h0 = c->aux;
    if (sca::launch_halfstep(a, sca::XiMode::Inject, true, c->stream) != hipSuccess) return fail(c);
    return SCA_OK;
}

int sca_debug_philox(const uint32_t* ctr_dev, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out_dev,
                     void* hip_stream)
{
    if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) return SCA_EINVAL;
    if (sca::launch_philox_test(ctr_dev, k0, k1, n, out_dev, static_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return SCA_EDEVICE;
    return SCA_OK;
}

int sca_debug_philox_rate(int64_t threads, int32_t calls, uint32_t* sink_dev, void* hip_stream)
{
    if (threads <= 0 || (threads % 256) != 0 || threads > ((int64_t)1 << 31) || calls <= 0 || !sink_dev)
        return SCA_EINVAL;
    if (sca::launch_philox_rate(threads, calls, sink_dev, static_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return SCA_EDEVICE;
    return SCA_OK;
}

int sca_roughness(sca_ctx* c, int64_t out3[3], double* w2)
{
    if (!c || !out3) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    const int rc = moments_of(c->S, c->aux, c->X, c->Y, c->W, c->nb, c->ws, c->stream, out3, w2);
    if (rc == SCA_EDEVICE) return fail(c);
    return rc;
}

// Moments of a caller's state without a context and without allocation: the
// row sums and the column prefix go to `scratch`, a static device array (one
// copy per GPU, held until the process ends).  Host code reaches it through
// the address hipGetSymbolAddress returns on each device, never through the
// array's name, which on the host is only a stand-in for the symbol.
static __device__ __align__(256) int64_t scratch[SCA_NOALLOC_SCRATCH_WORDS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch[kMaxDevices];  // per device: the address of `scratch`, once looked up

// The address of `scratch` on the current device (looked up on the first call
// there), or nullptr on failure.
int64_t* scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[dev] = static_cast<int64_t*>(ptr);
    }
    return g_scratch[dev];
}

}  // namespace

int sca_roughness_noalloc(const void* slopes_dev, const int64_t* aux_dev, int64_t X, int64_t Y, void* hip_stream,
                          int64_t out3[3], double* w2)
{
    if (Y > SCA_NOALLOC_MAX_Y) return SCA_ESCRATCH;
    if (!slopes_dev || !aux_dev || !out3 || !valid_size(X, Y)) return SCA_EINVAL;
    int64_t* ws = scratch_on_current_device();
    if (!ws) return SCA_EDEVICE;
    // row_sums writes rows[0, 3Y) and combine writes col[0, Y) and res[0, 6)
    // before anything reads them: nothing needs clearing between calls.
    const int32_t W = (int32_t)(X >= 128 ? X / 128 : 1);
    const int32_t nb = (int32_t)(X >= 128 ? 64 : X / 2);
    return moments_of(static_cast<const uint64_t*>(slopes_dev), aux_dev, X, Y, W, nb, ws,
                      static_cast<hipStream_t>(hip_stream), out3, w2);
}

size_t sca_snapshot_bytes(const sca_ctx* c)
{
    if (!c) return 0;
    return (size_t)(4 * c->Y * c->W + 1) * sizeof(uint64_t);
}

int sca_snapshot(sca_ctx* c, void* snap_dev)
{
    if (!c || !snap_dev) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    const size_t words = (size_t)(4 * c->Y * c->W);
    uint64_t* dst = static_cast<uint64_t*>(snap_dev);
    if (hipMemcpyAsync(dst, c->S, words * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c);
    if (hipMemcpyAsync(dst + words, c->aux, sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c);
    return SCA_OK;
}

int sca_autocorr(sca_ctx* c, const void* snap_dev, int64_t out4[4], double* c_ts)
{
    if (!c || !snap_dev || !out4) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    const uint64_t* snap = static_cast<const uint64_t*>(snap_dev);
    const int64_t* snap_h0 = reinterpret_cast<const int64_t*>(snap + 4 * c->Y * c->W);
    if (sca::launch_row_sums(c->S, snap, c->X, c->Y, c->W, c->nb, ws_rows(c), c->stream) != hipSuccess)
        return fail(c);
    if (sca::launch_combine(c->S, c->aux, snap, snap_h0, c->X, c->Y, c->W, ws_rows(c), ws_col(c), ws_res(c),
                            c->stream) != hipSuccess)
        return fail(c);
    int64_t r[6];
    const int rc = read_back(c, ws_res(c), r, 6);
    if (rc != SCA_OK) return rc;
    const __int128 st = join128(r[0], r[1]), sts = join128(r[2], r[3]), ss = join128(r[4], r[5]);
    if (!fits64(st) || !fits64(sts) || !fits64(ss)) return SCA_EOVERFLOW;
    const __int128 N = (__int128)c->X * c->Y;
    out4[0] = (int64_t)N;
    out4[1] = (int64_t)sts;
    out4[2] = (int64_t)st;
    out4[3] = (int64_t)ss;
    if (c_ts) *c_ts = (double)(N * sts - st * ss) / ((double)N * (double)N);
    return SCA_OK;
}

int sca_get_meta(sca_ctx* c, int64_t* t, int64_t* h0)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    if (t) *t = c->t;
    if (h0) {
        DeviceGuard dg(c->device);
        if (!dg.ok) return fail(c);
        return read_back(c, c->aux, h0, 1);
    }
    return SCA_OK;
}

int sca_set_blocking(sca_ctx* c, int32_t depth, int32_t band)
{
    if (!c || depth < -1 || depth > 13 || band < 0 || (band > 0 && (band < 4 || (band & (band - 1)) != 0)))
        return SCA_EINVAL;
    c->depth = depth;
    c->band = band;
    return SCA_OK;
}

int sca_set_time(sca_ctx* c, int64_t t)
{
    if (!c || t < 0 || t > (int64_t)UINT32_MAX) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    c->t = t;
    return SCA_OK;
}

int sca_heights(sca_ctx* c, int64_t y0, int64_t ny, int32_t* out_dev)
{
    if (!c) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    if (y0 < 0 || ny < 0 || y0 + ny > c->Y || (ny > 0 && !out_dev)) return SCA_EINVAL;
    if (ny == 0) return SCA_OK;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    int64_t h0 = 0;
    int rc = read_back(c, c->aux, &h0, 1);
    if (rc != SCA_OK) return rc;
    // |h(x,y) - h(0,0)| <= x + y for any slope field
    if (h0 > INT32_MAX - c->X - c->Y || h0 < INT32_MIN + c->X + c->Y) return SCA_EOVERFLOW;
    if (sca::launch_combine(c->S, c->aux, nullptr, nullptr, c->X, c->Y, c->W, nullptr, ws_col(c), nullptr,
                            c->stream) != hipSuccess)
        return fail(c);
    if (sca::launch_heights(c->S, c->X, c->Y, c->W, c->nb, ws_col(c), y0, ny, out_dev, c->stream) != hipSuccess)
        return fail(c);
    return SCA_OK;
}

void sca_destroy(sca_ctx* c)
{
    if (!c) return;
    {
        DeviceGuard dg(c->device);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->ws);
        if (c->capture) (void)hipStreamDestroy(c->capture);
    }
    delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kArenaAlign = 256;

size_t state_bytes(int64_t X, int64_t Y)
{
    const size_t words = (size_t)(4 * Y * (X >= 128 ? X / 128 : 1)) + 1;  // + h(0,0)
    return (words * sizeof(uint64_t) + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// First-fit allocator over [0, size) with coalescing of freed ranges.
class ArenaAllocator {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const
    {
        size_t s = 0;
        for (const auto& kv : free_) s += kv.second;
        return s;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
};

struct SlotHost {
    bool used = false;
    sca_req req{};
    size_t offset = 0, bytes = 0;
    int64_t t = 0;          // MCS reached once the enqueued epochs have run
    int32_t W = 0, nb = 0;
    sca::BatchDesc desc{};  // static part; t and n_run are set per epoch
};

bool valid_req(const sca_req& r)
{
    return valid_size(r.X, r.Y) && r.X <= 8192 && valid_prob(r.p) && valid_prob(r.q) && r.n_mcs >= 0 &&
           r.n_mcs <= (int64_t)UINT32_MAX && (r.flags & ~SCA_FORCE_PERSITE) == 0 && r.reserved == 0;
}

bool valid_cfg(const sca_batch_config& c)
{
    return (c.block_threads == 256 || c.block_threads == 512 || c.block_threads == 1024) && c.blocks_per_cu >= 1 &&
           c.blocks_per_cu <= 8 && c.lds_bytes >= 0 && c.lds_bytes <= 65536 && (c.lds_bytes % 8) == 0 &&
           (c.order == 0 || c.order == 1) && (c.words_per_lane == 1 || c.words_per_lane == 2) && c.depth >= 0 &&
           (c.depth <= 2 || (c.depth <= sca::kMaxBatchDepth && c.block_threads == 512 && c.blocks_per_cu == 1)) &&
           (c.max_parts == 1 || c.max_parts == 2 || c.max_parts == sca::kMaxParts);
}

}  // namespace

struct sca_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    int32_t max_slots = 0;
    int num_cus = 0;
    std::vector<SlotHost> slots;
    std::vector<int32_t> free_slots;  // stack of free slot ids
    ArenaAllocator alloc;
    sca_batch_config cfg{512, 2, 65536, 0, 1, 2, 1};
    uint64_t* d_save = nullptr;     // save areas of the blocked passes: grid x save words per workgroup,
                                    // then grid x save words for the parts of split realizations
    size_t save_bytes = 0;
    int64_t save_words = 0;         // per workgroup (and per part) in the captured graph
    int32_t resident = 0;           // workgroups of the captured launch that run at once
    int32_t* d_sync = nullptr;      // barrier counters of split realizations (one per part slot of the grid)
    int32_t* d_err = nullptr;       // set by a barrier wait that gave up
    int32_t* h_err = nullptr;       // pinned copy of d_err, written after each launch
    hipEvent_t err_copied = nullptr;
    bool err_pending = false;
    // device (library-owned)
    sca::BatchDesc* d_desc = nullptr;
    int32_t* d_order = nullptr;
    int32_t* d_counters = nullptr;  // [0] item count, [1] work queue
    int64_t* d_ws = nullptr;        // moments workspace for Y up to 131072
    // pinned staging
    sca::BatchDesc* h_desc = nullptr;
    int32_t* h_order = nullptr;
    int32_t* h_count = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // flat initialisation of admitted realizations: one launch per admission
    sca::FlatItem* h_flat = nullptr;  // pinned staging
    sca::FlatItem* d_flat = nullptr;
    hipEvent_t flat_staged = nullptr;
    bool flat_pending = false;
    hipGraphExec_t exec = nullptr;
    bool failed = false;
};

namespace {

int bfail(sca_batch* b)
{
    if (b) b->failed = true;
    return SCA_EDEVICE;
}



void batch_free(sca_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->flat_staged) (void)hipEventDestroy(b->flat_staged);
    (void)hipFree(b->d_flat);
    (void)hipHostFree(b->h_flat);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_counters);
    (void)hipFree(b->d_ws);
    (void)hipFree(b->d_save);
    (void)hipFree(b->d_sync);
    (void)hipFree(b->d_err);
    (void)hipHostFree(b->h_err);
    if (b->err_copied) (void)hipEventDestroy(b->err_copied);
    (void)hipHostFree(b->h_desc);
    (void)hipHostFree(b->h_order);
    (void)hipHostFree(b->h_count);
    delete b;
}

// (Re)captures the epoch graph: reset the work counter, then the persistent
// kernel.  The table, order and count are read from device memory, so the
// graph is reused for every epoch until the configuration changes.
hipError_t capture_epoch_graph(sca_batch* b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (!b->capture && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
        return hipErrorUnknown;
    const int grid = b->num_cus * b->cfg.blocks_per_cu;
    int32_t depth = b->cfg.depth;
    int64_t save_words = sca::blocked_save_words(depth, b->cfg.block_threads);
    // per-workgroup save areas, then as many again for the parts of split realizations
    const size_t need = sizeof(uint64_t) * (size_t)save_words * (size_t)grid * 2;
    if (need > b->save_bytes) {  // no launch of the old graph is in flight (callers synchronize first)
        (void)hipFree(b->d_save);
        b->d_save = nullptr;
        b->save_bytes = 0;
        if (hipMalloc(&b->d_save, need) == hipSuccess) {
            b->save_bytes = need;
        } else {
            (void)hipGetLastError();
            depth = 0;  // no room for the save areas: unblocked half-steps
            save_words = 0;
        }
    }
    b->save_words = depth > 0 ? save_words : 0;
    const int occ = sca::ensemble_occupancy(b->cfg.block_threads, b->cfg.words_per_lane, b->cfg.lds_bytes, depth);
    b->resident = std::min(grid, occ * b->num_cus);
    sca::BatchLaunch L{b->d_desc, b->d_order, b->d_counters, b->d_counters + 1, b->cfg.lds_bytes,
                       depth,     b->d_save,  save_words,    b->d_sync,         grid,
                       b->d_err};
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed) != hipSuccess) return hipErrorUnknown;
    hipError_t e1 = sca::launch_counter_reset(b->d_counters + 1, b->d_sync, grid, b->capture);
    if (e1 == hipSuccess)
        e1 = sca::launch_ensemble(L, b->cfg.block_threads, b->cfg.words_per_lane, grid, b->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->capture, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : hipErrorUnknown);
    }
    const hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e;
}

}  // namespace

extern "C" {

size_t sca_batch_state_bytes(int64_t X, int64_t Y)
{
    if (!valid_size(X, Y)) return 0;
    return state_bytes(X, Y);
}

int sca_batch_create(sca_batch** out, int32_t max_slots, void* arena_dev, size_t arena_bytes, void* hip_stream)
{
    if (!out || max_slots <= 0 || max_slots > (1 << 20) || (!arena_dev && arena_bytes)) return SCA_EINVAL;
    *out = nullptr;
    sca_batch* b = new (std::nothrow) sca_batch;
    if (!b) return SCA_ENOMEM;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->arena = static_cast<uint8_t*>(arena_dev);
    b->arena_bytes = arena_bytes;
    b->max_slots = max_slots;
    try {
        b->slots.resize((size_t)max_slots);
        b->free_slots.reserve((size_t)max_slots);
    } catch (...) {
        delete b;
        return SCA_ENOMEM;
    }
    for (int32_t s = max_slots - 1; s >= 0; --s) b->free_slots.push_back(s);
    b->alloc.reset(arena_bytes);
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
        delete b;
        return SCA_EDEVICE;
    }
    // the work queue holds one item per realization, plus one more per extra
    // part of a split realization (at most one part per persistent workgroup
    // in all, and at most 8 of those per compute unit)
    const size_t nd = sizeof(sca::BatchDesc) * (size_t)max_slots,
                 no = sizeof(int32_t) * ((size_t)max_slots + (size_t)b->num_cus * 8);
    if (hipMalloc(&b->d_desc, nd) != hipSuccess || hipMalloc(&b->d_order, no) != hipSuccess ||
        hipMalloc(&b->d_counters, 2 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&b->d_ws, sizeof(int64_t) * (size_t)(4 * 131072 + 8)) != hipSuccess ||
        hipHostMalloc(&b->h_desc, nd, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_order, no, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_count, sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&b->d_flat, sizeof(sca::FlatItem) * (size_t)max_slots) != hipSuccess ||
        hipHostMalloc(&b->h_flat, sizeof(sca::FlatItem) * (size_t)max_slots, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->flat_staged, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&b->d_sync, sizeof(int32_t) * (size_t)b->num_cus * 8) != hipSuccess ||
        hipMalloc(&b->d_err, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc(&b->h_err, sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->err_copied, hipEventDisableTiming) != hipSuccess ||
        hipMemsetAsync(b->d_err, 0, sizeof(int32_t), b->stream) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return SCA_ENOMEM;
    }
    std::memset(b->h_desc, 0, nd);
    *b->h_err = 0;
    *out = b;
    return SCA_OK;
}

int sca_batch_set_config(sca_batch* b, const sca_batch_config* cfg)
{
    if (!b || !cfg || !valid_cfg(*cfg)) return SCA_EINVAL;
    if (b->failed) return SCA_ESTATE;
    const bool same = cfg->block_threads == b->cfg.block_threads && cfg->blocks_per_cu == b->cfg.blocks_per_cu &&
                      cfg->lds_bytes == b->cfg.lds_bytes && cfg->order == b->cfg.order &&
                      cfg->words_per_lane == b->cfg.words_per_lane && cfg->depth == b->cfg.depth;
    if (same) {
        b->cfg.max_parts = cfg->max_parts;  // a host-side choice: the graph stays
        return SCA_OK;
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return bfail(b);
    // the old graph may still be in flight on the stream
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b);
    b->cfg = *cfg;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    return SCA_OK;
}

int sca_batch_get_config(const sca_batch* b, sca_batch_config* cfg)
{
    if (!b || !cfg) return SCA_EINVAL;
    *cfg = b->cfg;
    return SCA_OK;
}

int sca_batch_admit(sca_batch* b, const sca_req* reqs, int32_t n, int32_t* slots_out)
{
    if (!b || n < 0 || (n > 0 && (!reqs || !slots_out))) return SCA_EINVAL;
    if (b->failed) return SCA_ESTATE;
    for (int32_t i = 0; i < n; ++i)
        if (!valid_req(reqs[i])) return SCA_EINVAL;
    if ((size_t)n > b->free_slots.size()) return SCA_EBUSY;
    // all or nothing: place every state first
    std::vector<size_t> offs((size_t)n);
    int32_t placed = 0;
    for (; placed < n; ++placed) {
        if (!b->alloc.alloc(state_bytes(reqs[placed].X, reqs[placed].Y), &offs[(size_t)placed])) break;
    }
    if (placed < n) {
        for (int32_t i = 0; i < placed; ++i)
            b->alloc.release(offs[(size_t)i], state_bytes(reqs[i].X, reqs[i].Y));
        return SCA_EBUSY;
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return bfail(b);
    // the flat-init staging is free once the previous admission's copy has run
    if (b->flat_pending && hipEventSynchronize(b->flat_staged) != hipSuccess) return bfail(b);
    b->flat_pending = false;
    int32_t n_flat = 0;
    for (int32_t i = 0; i < n; ++i) {
        const sca_req& r = reqs[i];
        const int32_t slot = b->free_slots.back();
        b->free_slots.pop_back();
        SlotHost& s = b->slots[(size_t)slot];
        s.used = true;
        s.req = r;
        s.offset = offs[(size_t)i];
        s.bytes = state_bytes(r.X, r.Y);
        s.t = 0;
        s.W = (int32_t)(r.X >= 128 ? r.X / 128 : 1);
        s.nb = (int32_t)(r.X >= 128 ? 64 : r.X / 2);
        const ProbCode P = classify(r.p), Q = classify(r.q);
        const bool persite = (r.flags & SCA_FORCE_PERSITE) || !P.dyadic || !Q.dyadic;
        sca::BatchDesc& d = s.desc;
        d = sca::BatchDesc{};
        d.S = reinterpret_cast<uint64_t*>(b->arena + s.offset);
        d.plane = r.Y * s.W;
        d.h0 = reinterpret_cast<int64_t*>(d.S + 4 * d.plane);
        d.W = s.W;
        d.Y = (int32_t)r.Y;
        d.nb = s.nb;
        d.mode = persite ? 1 : 0;
        d.k0 = (uint32_t)r.seed;
        d.k1 = (uint32_t)(r.seed >> 32);
        d.all_p = P.all;
        d.all_q = Q.all;
        d.has_q = r.q > 0.0 ? 1 : 0;
        if (persite) {
            d.thr_p = P.thr;
            d.thr_q = Q.thr;
        } else {
            d.dig_p = P.digits;
            d.dig_q = Q.digits;
            d.ndraw = P.n > Q.n ? P.n : Q.n;
        }
        // states of up to 2^20 words share one launch (one workgroup per
        // state); larger ones get a launch of their own
        if (4 * d.plane <= ((int64_t)1 << 20)) {
            b->h_flat[n_flat++] = sca::flat_item(d.S, r.Y, s.W, s.nb, d.h0);
        } else if (sca::launch_flat_init(d.S, r.Y, s.W, s.nb, d.h0, b->stream) != hipSuccess) {
            return bfail(b);
        }
        slots_out[i] = slot;
    }
    if (n_flat > 0) {
        if (hipMemcpyAsync(b->d_flat, b->h_flat, sizeof(sca::FlatItem) * (size_t)n_flat, hipMemcpyHostToDevice,
                           b->stream) != hipSuccess ||
            hipEventRecord(b->flat_staged, b->stream) != hipSuccess ||
            sca::launch_flat_init_many(b->d_flat, n_flat, b->stream) != hipSuccess)
            return bfail(b);
        b->flat_pending = true;
    }
    return SCA_OK;
}

}  // extern "C"

namespace {

// One epoch in which slot s advances mcs_of(s) MCS (clamped to its budget).
template <typename F>
int batch_epoch(sca_batch* b, F mcs_of, int32_t* active_out)
{
    if (b->failed) return SCA_ESTATE;
    DeviceGuard dg(b->device);
    if (!dg.ok) return bfail(b);
    if (b->err_pending && hipEventQuery(b->err_copied) == hipSuccess) {
        b->err_pending = false;
        if (*b->h_err) return bfail(b);  // a split realization's barrier gave up: its state is not valid
    }
    // the staging buffers are free once the previous epoch's copies have run
    if (b->staged_pending && hipEventSynchronize(b->staged) != hipSuccess) return bfail(b);
    b->staged_pending = false;
    // The save areas and the depth of the captured graph decide which
    // realizations can run blocked, so the graph is made first.
    if (!b->exec && capture_epoch_graph(b) != hipSuccess) return bfail(b);
    const int32_t grid = b->num_cus * b->cfg.blocks_per_cu;
    const int32_t max_depth = b->save_words > 0 ? b->cfg.depth : 0;
    int32_t count = 0, hi = -1;
    std::vector<std::pair<int64_t, int32_t>> work;
    std::vector<int64_t> runs((size_t)b->max_slots, 0);
    int64_t total = 0;
    for (int32_t slot = 0; slot < b->max_slots; ++slot) {
        SlotHost& s = b->slots[(size_t)slot];
        if (!s.used) continue;
        const int64_t left = s.req.n_mcs - s.t;
        int64_t run = mcs_of(s);
        if (run > left) run = left;
        if (run < 0) run = 0;
        runs[(size_t)slot] = run;
        sca::BatchDesc d = s.desc;
        d.t = (uint32_t)s.t;
        d.n_run = (uint32_t)run;
        d.depth = 0;
        d.bands = 0;
        d.parts = 1;
        d.sync_idx = 0;
        d.save = nullptr;
        if (d.mode == 0 && run > 0)
            (void)sca::blocked_plan(s.W, (int)s.req.Y, max_depth, b->cfg.block_threads, 1, &d.depth, &d.bands);
        b->h_desc[slot] = d;
        hi = slot;
        if (run > 0) {
            work.emplace_back(run * s.req.X * s.req.Y, slot);
            total += run * s.req.X * s.req.Y;
        }
    }
    if (b->cfg.order == 0)
        std::stable_sort(work.begin(), work.end(),
                         [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                             return x.first > y.first;
                         });
    // Realizations that run as temporally blocked passes go first (the
    // persistent kernel takes them in a phase of their own), and among them
    // the split ones: a blocked realization with more work than the average
    // per persistent workgroup runs on parts = the smallest power of two that
    // brings its share under that average (at most max_parts, as the band
    // geometry allows), while the parts in all stay within the number of
    // persistent workgroups that the device runs at once, so that every part
    // is taken by a running workgroup's first pop.
    std::stable_partition(work.begin(), work.end(), [b](const std::pair<int64_t, int32_t>& w) {
        return b->h_desc[w.second].depth > 0;
    });
    const int64_t avg = total / grid;
    int32_t parts_used = 0, n_split = 0;
    std::vector<std::pair<int64_t, int32_t>> split, rest;
    for (const auto& w : work) {
        sca::BatchDesc& d = b->h_desc[w.second];
        const SlotHost& s = b->slots[(size_t)w.second];
        int32_t P = 1, K = d.depth, nb = d.bands;
        if (d.depth > 0 && b->cfg.order == 0)
            for (int32_t p2 = 2; p2 <= b->cfg.max_parts && w.first / (p2 / 2) > avg; p2 *= 2) {
                int32_t K2 = 0, nb2 = 0;
                if (parts_used + p2 > b->resident ||
                    !sca::blocked_plan(s.W, (int)s.req.Y, max_depth, b->cfg.block_threads, p2, &K2, &nb2))
                    break;
                P = p2;
                K = K2;
                nb = nb2;
            }
        if (P > 1) {
            d.parts = P;
            d.depth = K;
            d.bands = nb;
            d.sync_idx = n_split++;
            d.save = b->d_save + (size_t)b->save_words * (size_t)(grid + parts_used);
            parts_used += P;
            split.push_back(w);
        } else {
            rest.push_back(w);
        }
    }
    for (const auto& w : split)
        for (int32_t m = 0; m < b->h_desc[w.second].parts; ++m)
            b->h_order[count++] = w.second | (m << sca::kItemSlotBits);
    for (const auto& w : rest) b->h_order[count++] = w.second;
    if (active_out) *active_out = (int32_t)work.size();
    if (count == 0) return SCA_OK;
    *b->h_count = count;
    if (hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(sca::BatchDesc) * (size_t)(hi + 1), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_order, b->h_order, sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b->d_counters, b->h_count, sizeof(int32_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipEventRecord(b->staged, b->stream) != hipSuccess)
        return bfail(b);
    b->staged_pending = true;
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return bfail(b);
    if (n_split > 0 && !b->err_pending) {
        if (hipMemcpyAsync(b->h_err, b->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipEventRecord(b->err_copied, b->stream) != hipSuccess)
            return bfail(b);
        b->err_pending = true;
    }
    for (const auto& w : work) b->slots[(size_t)w.second].t += runs[(size_t)w.second];
    return SCA_OK;
}

}  // namespace

extern "C" {

int sca_batch_run(sca_batch* b, int64_t mcs_epoch, int32_t* active_out)
{
    if (!b || mcs_epoch < 0) return SCA_EINVAL;
    return batch_epoch(b, [mcs_epoch](const SlotHost&) { return mcs_epoch; }, active_out);
}

int sca_batch_run_work(sca_batch* b, int64_t site_updates, int32_t* active_out)
{
    if (!b || site_updates <= 0) return SCA_EINVAL;
    return batch_epoch(
        b,
        [site_updates](const SlotHost& s) {
            const int64_t q = site_updates / (s.req.X * s.req.Y);
            return q > 0 ? q : (int64_t)1;
        },
        active_out);
}

int sca_batch_slot(const sca_batch* b, int32_t slot, sca_slot_info* out)
{
    if (!b || !out || slot < 0 || slot >= b->max_slots || !b->slots[(size_t)slot].used) return SCA_EINVAL;
    const SlotHost& s = b->slots[(size_t)slot];
    out->X = s.req.X;
    out->Y = s.req.Y;
    out->t = s.t;
    out->n_mcs = s.req.n_mcs;
    out->seed = s.req.seed;
    out->slopes_dev = s.desc.S;
    out->h0_dev = s.desc.h0;
    return SCA_OK;
}

int sca_batch_roughness(sca_batch* b, int32_t slot, int64_t out3[3], double* w2)
{
    if (!b || !out3 || slot < 0 || slot >= b->max_slots || !b->slots[(size_t)slot].used) return SCA_EINVAL;
    if (b->failed) return SCA_ESTATE;
    DeviceGuard dg(b->device);
    if (!dg.ok) return bfail(b);
    const SlotHost& s = b->slots[(size_t)slot];
    const int rc = moments_of(s.desc.S, s.desc.h0, s.req.X, s.req.Y, s.W, s.nb, b->d_ws, b->stream, out3, w2);
    if (rc == SCA_EDEVICE) return bfail(b);
    // the stream is synchronized: a barrier that gave up in an earlier launch shows in d_err
    int32_t err = 0;
    if (hipMemcpy(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost) != hipSuccess || err) return bfail(b);
    return rc;
}

int sca_batch_release(sca_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[(size_t)slot].used) return SCA_EINVAL;
    SlotHost& s = b->slots[(size_t)slot];
    b->alloc.release(s.offset, s.bytes);
    s = SlotHost{};
    b->free_slots.push_back(slot);
    return SCA_OK;
}

void sca_batch_destroy(sca_batch* b)
{
    if (!b) return;
    {
        DeviceGuard dg(b->device);
        (void)hipStreamSynchronize(b->stream);
        batch_free(b);
    }
}

}  // extern "C"

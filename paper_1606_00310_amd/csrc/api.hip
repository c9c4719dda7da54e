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
#include <cstring>
#include <new>

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
    if (n_mcs < 0 || !valid_prob(p) || !valid_prob(q) || (flags & ~SCA_FORCE_PERSITE)) return SCA_EINVAL;
    if (c->t + n_mcs > (int64_t)UINT32_MAX) return SCA_EINVAL;
    if (n_mcs == 0) return SCA_OK;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);

    const ProbCode P = classify(p), Q = classify(q);
    const bool persite = (flags & SCA_FORCE_PERSITE) || !P.dyadic || !Q.dyadic;
    const bool has_q = (q > 0.0);
    sca::SweepArgs a{};
    a.S = c->S;
    a.plane = c->Y * c->W;
    a.W = c->W;
    a.Y = (int32_t)c->Y;
    a.nb = c->nb;
    a.k0 = (uint32_t)c->seed;
    a.k1 = (uint32_t)(c->seed >> 32);
    a.h0 = c->aux;
    a.all_p = P.all;
    a.all_q = Q.all;
    if (persite) {
        a.thr_p = P.thr;
        a.thr_q = Q.thr;
    } else {
        a.dig_p = P.digits;
        a.dig_q = Q.digits;
        a.ndraw = P.n > Q.n ? P.n : Q.n;
    }
    const sca::XiMode mode = persite ? sca::XiMode::PerSite : sca::XiMode::Mask;
    for (int64_t i = 0; i < n_mcs; ++i) {
        a.t = (uint32_t)(c->t + i);
        for (int parity = 0; parity < 2; ++parity) {
            a.parity = parity;
            if (sca::launch_halfstep(a, mode, has_q, c->stream) != hipSuccess) return fail(c);
        }
    }
    c->t += n_mcs;
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

int sca_roughness(sca_ctx* c, int64_t out3[3], double* w2)
{
    if (!c || !out3) return SCA_EINVAL;
    if (c->failed) return SCA_ESTATE;
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c);
    if (sca::launch_row_sums(c->S, nullptr, c->X, c->Y, c->W, c->nb, ws_rows(c), c->stream) != hipSuccess)
        return fail(c);
    if (sca::launch_combine(c->S, c->aux, nullptr, nullptr, c->X, c->Y, c->W, ws_rows(c), ws_col(c), ws_res(c),
                            c->stream) != hipSuccess)
        return fail(c);
    int64_t r[6];
    const int rc = read_back(c, ws_res(c), r, 6);
    if (rc != SCA_OK) return rc;
    const __int128 s1 = join128(r[0], r[1]), s2 = join128(r[2], r[3]);
    if (!fits64(s1) || !fits64(s2)) return SCA_EOVERFLOW;
    const __int128 N = (__int128)c->X * c->Y;
    out3[0] = (int64_t)N;
    out3[1] = (int64_t)s1;
    out3[2] = (int64_t)s2;
    if (w2) *w2 = (double)(N * s2 - s1 * s1) / ((double)N * (double)N);
    return SCA_OK;
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
    }
    delete c;
}

}  // extern "C"

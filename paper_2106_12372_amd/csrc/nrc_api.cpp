// C ABI of the radiance-cache library: argument validation, the layout of the
// caller-owned device workspaces, and the launch sequences of each entry point.
// The library allocates no device memory of its own.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "nrc_api_internal.h"
#include "nrc_internal.h"

using nrc::Geo;

namespace {

thread_local std::string g_err;

}  // namespace

namespace nrc {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return NRC_OK;
}

int device_fail(hipError_t e, const char* what) {
    return fail(NRC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int validate_config(const nrc_config* c) {
    if (!c) return fail(NRC_EINVAL, "config is NULL");
    if (c->width != 64 && c->width != 128) return fail(NRC_EINVAL, "width must be 64 or 128 (got %d)", c->width);
    if (c->n_hidden < 1 || c->n_hidden > 8) return fail(NRC_EINVAL, "n_hidden must be in 1..8 (got %d)", c->n_hidden);
    if (c->n_out != 3) return fail(NRC_EINVAL, "n_out must be 3 (got %d)", c->n_out);
    if (c->precision != NRC_FP32 && c->precision != NRC_FP16 && c->precision != NRC_BF16 &&
        c->precision != NRC_FP32_VALU)
        return fail(NRC_EINVAL, "unknown precision %d", c->precision);
    if (c->enc_preset != NRC_PRESET_CONFIG && c->enc_preset != NRC_PRESET_PAPER &&
        c->enc_preset != NRC_PRESET_PAPER_TRI && c->enc_preset != NRC_PRESET_PAPER_GAUSS)
        return fail(NRC_EINVAL, "unknown encoding preset %d", c->enc_preset);
    if (fp32_form(c->precision) && (c->width != 64 || c->n_hidden > 6))
        return fail(NRC_EINVAL, "the FP32 forms support width 64 and n_hidden <= 6");
    if (!fp32_form(c->precision) && c->width == 128 && c->n_hidden > 5)
        return fail(NRC_EINVAL, "width 128 supports n_hidden <= 5");
    if (!(c->lr > 0.0f) || !std::isfinite(c->lr)) return fail(NRC_EINVAL, "lr must be positive");
    if (!(c->beta1 >= 0.0f && c->beta1 < 1.0f) || !(c->beta2 >= 0.0f && c->beta2 < 1.0f))
        return fail(NRC_EINVAL, "Adam betas must be in [0, 1)");
    if (!(c->adam_eps >= 0.0f) || !std::isfinite(c->adam_eps)) return fail(NRC_EINVAL, "adam_eps must be >= 0");
    if (!(c->loss_eps > 0.0f) || !std::isfinite(c->loss_eps)) return fail(NRC_EINVAL, "loss_eps must be positive");
    if (!(c->loss_scale > 0.0f) || !std::isfinite(c->loss_scale)) return fail(NRC_EINVAL, "loss_scale must be positive");
    if (!(c->ema_alpha >= 0.0f && c->ema_alpha < 1.0f)) return fail(NRC_EINVAL, "ema_alpha must be in [0, 1)");
    if (c->factorize != 0 && c->factorize != 1) return fail(NRC_EINVAL, "factorize must be 0 or 1");
    return NRC_OK;
}

CacheLayout cache_layout(const nrc_config& c) {
    const Geo d(c.width, c.n_hidden);
    const size_t P = (size_t)d.n_params();
    CacheLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    L.w = take(P * 4);
    L.m = take(P * 4);
    L.v = take(P * 4);
    L.t = take(16);
    if (!fp32_form(c.precision)) {
        const size_t copies = (size_t)train_frag_copies(c.precision);
        L.ffr = take(copies * d.n_fwd_frags() * kFragElems * 2);
        L.bfr = take(copies * d.n_bwd_frags() * kFragElems * 2);
    } else {
        L.ffr = L.bfr = 0;
    }
    L.e = L.wbar = L.effr = 0;
    if (c.ema_alpha > 0.0f) {
        L.e = take(P * 4);
        L.wbar = take(P * 4);
        if (!fp32_form(c.precision)) L.effr = take((size_t)d.n_fwd_frags() * kFragElems * 2);
    }
    L.total = off;
    return L;
}

ScratchLayout scratch_layout(const nrc_config& c, int64_t n) {
    const Geo d(c.width, c.n_hidden);
    const size_t P = (size_t)d.n_params();
    const int ts = train_tile(c.precision, c.width);
    const size_t tiles = (size_t)((n + ts - 1) / ts);
    ScratchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    L.tiles = (int64_t)tiles;
    L.partials = take(tiles * P * 4);
    L.partials2 = take(tiles * P * 4);
    L.loss_part = take(tiles * 4);
    L.grad = take(P * 4);
    L.flags = take(tiles * 4);
    // the step's loss and skip flag side by side, so one 8-byte copy reads both
    L.loss = take(16);
    L.skipped = L.loss + 4;
    L.total = off;
    return L;
}

// Bytes of the autograd form's activation buffer: per training tile, h_1 .. h_H
// at the operand precision, then the network output of every record as four
// floats (see k_train_mfma / k_train_fp32).
size_t act_layout(const nrc_config& c, int64_t n) {
    const int ts = train_tile(c.precision, c.width);
    const size_t tiles = (size_t)((n + ts - 1) / ts);
    const size_t elem = fp32_form(c.precision) ? 4 : 2;
    return tiles * (size_t)c.n_hidden * (size_t)c.width * (size_t)ts * elem + tiles * (size_t)ts * 16;
}

// Network shape plus the reflectance-factorisation column the kernels use.
Geo kernel_geo(const nrc_config& c) {
    Geo d(c.width, c.n_hidden);
    d.F = c.factorize ? albedo_col(c.enc_preset) : 0;
    return d;
}

// Enqueue one training step (forward, loss, backward, reduction, Adam) on s.
int enqueue_train_step(nrc_cache* c, const void* enc, const float* target, const int32_t* idx,
                       int64_t n, char* scratch, float* loss_dev, int32_t* skipped_dev, hipStream_t s,
                       LcgGather lg, int raw_layout) {
    const nrc_config& cfg = c->cfg;
    const Geo d = kernel_geo(cfg);
    const ScratchLayout sl = scratch_layout(cfg, n);
    float* partials = (float*)(scratch + (c->parity ? sl.partials2 : sl.partials));
    float* loss_part = (float*)(scratch + sl.loss_part);
    int32_t* tile_bad = (int32_t*)(scratch + sl.flags);
    const float scale = cfg.loss_scale;
    const float grad_scale = (float)((double)scale / (3.0 * (double)n));
    hipError_t e;
    if (raw_layout >= 0) {
        const float* raw = (const float*)enc;
        if (cfg.precision == NRC_FP32_VALU)
            e = launch_train_fp32_valu_raw(d, cfg.enc_preset, raw_layout, c->w(), raw, target, idx, n, cfg.loss_eps,
                                           grad_scale, partials, loss_part, tile_bad, s, lg);
        else if (cfg.precision == NRC_FP32)
            e = launch_train_fp32_raw(d, cfg.enc_preset, raw_layout, c->w(), raw, target, idx, n, cfg.loss_eps,
                                      grad_scale, partials, loss_part, tile_bad, s, lg);
        else
            e = launch_train_mfma_raw(cfg.precision, d, cfg.enc_preset, raw_layout, c->ffr(), c->bfr(), raw, target,
                                      idx, n, cfg.loss_eps, grad_scale, partials, loss_part, tile_bad, s, lg);
    } else if (cfg.precision == NRC_FP32_VALU)
        e = launch_train_fp32_valu(d, c->w(), (const float*)enc, target, idx, n, false, cfg.loss_eps, grad_scale,
                                   partials, loss_part, tile_bad, nullptr, s, lg);
    else if (cfg.precision == NRC_FP32)
        e = launch_train_fp32(d, c->w(), (const float*)enc, target, idx, n, false, cfg.loss_eps, grad_scale,
                              partials, loss_part, tile_bad, nullptr, s, nullptr, lg);
    else
        e = launch_train_mfma(cfg.precision, d, c->ffr(), c->bfr(), enc, target, idx, n, false, cfg.loss_eps,
                              grad_scale, partials, loss_part, tile_bad, nullptr, s, nullptr, lg);
    if (e != hipSuccess) return device_fail(e, "training kernel launch");
    float* loss_out = loss_dev ? loss_dev : (float*)(scratch + sl.loss);
    int32_t* skipped_out = skipped_dev ? skipped_dev : (int32_t*)(scratch + sl.skipped);
    const AdamHyper hp{cfg.lr, cfg.beta1, cfg.beta2, cfg.adam_eps};
    const EmaArgs ema{c->ema() ? cfg.ema_alpha : 0.0f, c->e(), c->wbar(), c->effr()};
    e = launch_reduce_adam(cfg.precision, d, !fp32_form(cfg.precision), partials, (int)sl.tiles,
                           tile_bad, loss_part, (float)(1.0 / (3.0 * (double)n)), loss_out,
                           1.0f / scale, c->w(), c->m(), c->v(), c->tslots(), c->parity, hp, ema,
                           skipped_out, c->ffr(), c->bfr(), s);
    if (e != hipSuccess) return device_fail(e, "gradient reduction / Adam launch");
    c->parity ^= 1;
    return NRC_OK;
}

int enqueue_forward(nrc_cache* c, const void* enc, int64_t n, float* rgb, hipStream_t s) {
    const Geo d = kernel_geo(c->cfg);
    hipError_t e;
    if (c->cfg.precision == NRC_FP32_VALU)
        e = launch_fwd_fp32_valu(d, c->query_w(), (const float*)enc, n, rgb, s);
    else if (c->cfg.precision == NRC_FP32)
        e = launch_fwd_fp32(d, c->query_w(), (const float*)enc, n, rgb, s);
    else
        e = launch_fwd_mfma(c->cfg.precision, d, c->query_ffr(), enc, n, rgb, s);
    if (e != hipSuccess) return device_fail(e, "forward launch");
    return NRC_OK;
}

}  // namespace nrc

using namespace nrc;

extern "C" {

int nrc_config_default(nrc_config* cfg) {
    if (!cfg) return fail(NRC_EINVAL, "config is NULL");
    std::memset(cfg, 0, sizeof *cfg);
    cfg->width = 64;
    cfg->n_hidden = 5;
    cfg->n_out = 3;
    cfg->precision = NRC_FP16;
    cfg->enc_preset = NRC_PRESET_CONFIG;
    cfg->lr = 1e-2f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.99f;
    cfg->adam_eps = 1e-8f;
    cfg->loss_eps = 0.01f;
    cfg->loss_scale = 128.0f;
    cfg->ema_alpha = 0.0f;
    cfg->factorize = 0;
    cfg->seed = 0;
    return ok();
}

const char* nrc_last_error(void) { return g_err.c_str(); }

int64_t nrc_param_count(const nrc_config* cfg) {
    if (validate_config(cfg) != NRC_OK) return -1;
    ok();
    return Geo(cfg->width, cfg->n_hidden).n_params();
}

size_t nrc_cache_bytes(const nrc_config* cfg) {
    if (validate_config(cfg) != NRC_OK) return 0;
    ok();
    return cache_layout(*cfg).total;
}

size_t nrc_train_scratch_bytes(const nrc_config* cfg, int64_t n) {
    if (validate_config(cfg) != NRC_OK) return 0;
    if (n < 0 || n > ((int64_t)1 << 31)) { fail(NRC_EINVAL, "n must be in [0, 2^31]"); return 0; }
    ok();
    return scratch_layout(*cfg, n).total;
}

int nrc_enc_elem_bytes(const nrc_config* cfg) {
    if (validate_config(cfg) != NRC_OK) return NRC_EINVAL;
    ok();
    return fp32_form(cfg->precision) ? 4 : 2;
}

int nrc_cache_create(const nrc_config* cfg, void* dev_ws, size_t ws_bytes, void* stream,
                     nrc_cache** out) {
    if (!out) return fail(NRC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc != NRC_OK) return rc;
    if (!dev_ws) return fail(NRC_EINVAL, "workspace is NULL");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(NRC_EINVAL, "workspace must be 256-byte aligned");
    const CacheLayout L = cache_layout(*cfg);
    if (ws_bytes < L.total)
        return fail(NRC_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, L.total);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    nrc_cache* c = new (std::nothrow) nrc_cache();
    if (!c) return fail(NRC_ENOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->lay = L;
    c->ws = (char*)dev_ws;
    c->parity = 0;
    c->device = dev;
    e = hipMemsetAsync(dev_ws, 0, L.total, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        delete c;
        return device_fail(e, "workspace clear");
    }
    *out = c;
    return ok();
}

int nrc_cache_destroy(nrc_cache* cache) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    delete cache;
    return ok();
}

int nrc_cache_config(const nrc_cache* cache, nrc_config* out) {
    if (!cache || !out) return fail(NRC_EINVAL, "NULL argument");
    *out = cache->cfg;
    return ok();
}

// Rebuild the reduced-precision weight copies from the master weights and
// restart the EMA set at W_bar = W, E = 0 (enqueued on s).
static hipError_t reset_ema_and_frags(nrc_cache* c, hipStream_t s) {
    const Geo d(c->cfg.width, c->cfg.n_hidden);
    const size_t bytes = (size_t)d.n_params() * 4;
    hipError_t e = hipSuccess;
    if (c->ema()) {
        e = hipMemsetAsync(c->e(), 0, bytes, s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->wbar(), c->w(), bytes, hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess && !fp32_form(c->cfg.precision)) {
        const size_t copies = (size_t)train_frag_copies(c->cfg.precision);
        e = hipMemsetAsync(c->ffr(), 0, copies * d.n_fwd_frags() * kFragElems * 2, s);
        if (e == hipSuccess) e = hipMemsetAsync(c->bfr(), 0, copies * d.n_bwd_frags() * kFragElems * 2, s);
        if (e == hipSuccess && c->ema())
            e = hipMemsetAsync(c->effr(), 0, (size_t)d.n_fwd_frags() * kFragElems * 2, s);
        if (e == hipSuccess)
            e = launch_build_frags(c->cfg.precision, d, c->w(), c->ffr(), c->bfr(), c->effr(), s);
    }
    return e;
}

static int upload_state(nrc_cache* c, const float* w, const float* m, const float* v, int64_t t,
                        hipStream_t s) {
    const Geo d(c->cfg.width, c->cfg.n_hidden);
    const size_t bytes = (size_t)d.n_params() * 4;
    hipError_t e = hipMemcpyAsync(c->w(), w, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = m ? hipMemcpyAsync(c->m(), m, bytes, hipMemcpyHostToDevice, s) : hipMemsetAsync(c->m(), 0, bytes, s);
    if (e == hipSuccess)
        e = v ? hipMemcpyAsync(c->v(), v, bytes, hipMemcpyHostToDevice, s) : hipMemsetAsync(c->v(), 0, bytes, s);
    int32_t ts[4] = {(int32_t)t, (int32_t)t, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(c->tslots(), ts, sizeof ts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = reset_ema_and_frags(c, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "state upload");
    c->parity = 0;
    return ok();
}

int nrc_set_weights(nrc_cache* cache, const float* host_w, int64_t n, void* stream) {
    if (!cache || !host_w) return fail(NRC_EINVAL, "NULL argument");
    const int64_t P = Geo(cache->cfg.width, cache->cfg.n_hidden).n_params();
    if (n != P) return fail(NRC_EINVAL, "expected %lld weights, got %lld", (long long)P, (long long)n);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host_w[i])) return fail(NRC_EINVAL, "weight %lld is not finite", (long long)i);
    return upload_state(cache, host_w, nullptr, nullptr, 0, (hipStream_t)stream);
}

int nrc_set_weights_device(nrc_cache* cache, const float* dev_w, int64_t n, void* stream) {
    if (!cache || !dev_w) return fail(NRC_EINVAL, "NULL argument");
    if (((uintptr_t)dev_w & 3) != 0) return fail(NRC_EINVAL, "misaligned weights");
    const Geo d(cache->cfg.width, cache->cfg.n_hidden);
    if (n != d.n_params()) return fail(NRC_EINVAL, "expected %d weights, got %lld", d.n_params(), (long long)n);
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)d.n_params() * 4;
    hipError_t e = hipMemcpyAsync(cache->w(), dev_w, bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(cache->m(), 0, bytes, s);
    if (e == hipSuccess) e = hipMemsetAsync(cache->v(), 0, bytes, s);
    if (e == hipSuccess) e = hipMemsetAsync(cache->tslots(), 0, 16, s);
    if (e == hipSuccess) e = reset_ema_and_frags(cache, s);
    if (e != hipSuccess) return device_fail(e, "device weight upload");
    cache->parity = 0;
    return ok();
}

int nrc_get_weights(const nrc_cache* cache, float* host_w, int64_t n, void* stream) {
    if (!cache || !host_w) return fail(NRC_EINVAL, "NULL argument");
    const int64_t P = Geo(cache->cfg.width, cache->cfg.n_hidden).n_params();
    if (n != P) return fail(NRC_EINVAL, "expected %lld weights, got %lld", (long long)P, (long long)n);
    hipError_t e = hipMemcpyAsync(host_w, const_cast<nrc_cache*>(cache)->w(), (size_t)P * 4,
                                  hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "weight download");
    return ok();
}

int nrc_get_state(const nrc_cache* cache, float* host_w, float* host_m, float* host_v, int64_t n,
                  int64_t* t, void* stream) {
    if (!cache || !host_w || !host_m || !host_v || !t) return fail(NRC_EINVAL, "NULL argument");
    nrc_cache* c = const_cast<nrc_cache*>(cache);
    const int64_t P = Geo(c->cfg.width, c->cfg.n_hidden).n_params();
    if (n != P) return fail(NRC_EINVAL, "expected %lld weights, got %lld", (long long)P, (long long)n);
    hipStream_t s = (hipStream_t)stream;
    int32_t ts[4];
    hipError_t e = hipMemcpyAsync(host_w, c->w(), (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host_m, c->m(), (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host_v, c->v(), (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ts, c->tslots(), sizeof ts, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "state download");
    *t = ts[c->parity];
    return ok();
}

int nrc_set_state(nrc_cache* cache, const float* host_w, const float* host_m, const float* host_v,
                  int64_t n, int64_t t, void* stream) {
    if (!cache || !host_w || !host_m || !host_v) return fail(NRC_EINVAL, "NULL argument");
    const int64_t P = Geo(cache->cfg.width, cache->cfg.n_hidden).n_params();
    if (n != P) return fail(NRC_EINVAL, "expected %lld weights, got %lld", (long long)P, (long long)n);
    if (t < 0 || t > INT32_MAX) return fail(NRC_EINVAL, "step count out of range");
    return upload_state(cache, host_w, host_m, host_v, t, (hipStream_t)stream);
}

int nrc_get_ema(const nrc_cache* cache, float* host_w_bar, float* host_e, int64_t n, void* stream) {
    if (!cache || !host_w_bar || !host_e) return fail(NRC_EINVAL, "NULL argument");
    nrc_cache* c = const_cast<nrc_cache*>(cache);
    if (!c->ema()) return fail(NRC_EINVAL, "the cache keeps no EMA weights (ema_alpha = 0)");
    const int64_t P = Geo(c->cfg.width, c->cfg.n_hidden).n_params();
    if (n != P) return fail(NRC_EINVAL, "expected %lld weights, got %lld", (long long)P, (long long)n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(host_w_bar, c->wbar(), (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host_e, c->e(), (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "EMA download");
    return ok();
}

int nrc_set_ema(nrc_cache* cache, const float* host_w_bar, const float* host_e, int64_t n, void* stream) {
    if (!cache || !host_w_bar || !host_e) return fail(NRC_EINVAL, "NULL argument");
    if (!cache->ema()) return fail(NRC_EINVAL, "the cache keeps no EMA weights (ema_alpha = 0)");
    const Geo d(cache->cfg.width, cache->cfg.n_hidden);
    if (n != d.n_params()) return fail(NRC_EINVAL, "expected %d weights, got %lld", d.n_params(), (long long)n);
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)d.n_params() * 4;
    hipError_t e = hipMemcpyAsync(cache->wbar(), host_w_bar, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cache->e(), host_e, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !fp32_form(cache->cfg.precision))
        e = launch_build_frags(cache->cfg.precision, d, cache->wbar(), cache->effr(), nullptr, nullptr, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "EMA upload");
    return ok();
}

int nrc_encode(const nrc_cache* cache, const float* raw, int raw_layout, int64_t n, void* enc,
               void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (raw_layout != NRC_RAW14 && raw_layout != NRC_RAW16) return fail(NRC_EINVAL, "unknown raw layout %d", raw_layout);
    if (n < 0) return fail(NRC_EINVAL, "n must be >= 0");
    if (n == 0) return ok();
    if (!raw || !enc) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(raw) || !aligned16(enc)) return fail(NRC_EINVAL, "buffers must be 16-byte aligned");
    hipError_t e = launch_encode(cache->cfg.precision, cache->cfg.enc_preset, raw_layout, raw, n, enc,
                                 (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "encode launch");
    return ok();
}

int nrc_forward(nrc_cache* cache, const void* enc, int64_t n, float* rgb, void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 0) return fail(NRC_EINVAL, "n must be >= 0");
    if (n == 0) return ok();
    if (!enc || !rgb) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)rgb & 3)) return fail(NRC_EINVAL, "misaligned buffer");
    const int rc = enqueue_forward(cache, enc, n, rgb, (hipStream_t)stream);
    return rc == NRC_OK ? ok() : rc;
}

int nrc_forward_raw(nrc_cache* cache, const float* raw, int raw_layout, int64_t n, float* rgb,
                    void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (raw_layout != NRC_RAW14 && raw_layout != NRC_RAW16) return fail(NRC_EINVAL, "unknown raw layout %d", raw_layout);
    if (cache->cfg.width != 64) return fail(NRC_EINVAL, "the fused raw-record path supports width 64");
    if (n < 0) return fail(NRC_EINVAL, "n must be >= 0");
    if (n == 0) return ok();
    if (!raw || !rgb) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(raw) || ((uintptr_t)rgb & 3)) return fail(NRC_EINVAL, "misaligned buffer");
    const Geo d = kernel_geo(cache->cfg);
    hipError_t e;
    if (cache->cfg.precision == NRC_FP32_VALU)
        e = launch_fwd_raw_fp32_valu(d, cache->cfg.enc_preset, raw_layout, cache->query_w(), raw, n, rgb,
                                     (hipStream_t)stream);
    else if (cache->cfg.precision == NRC_FP32)
        e = launch_fwd_raw_fp32(d, cache->cfg.enc_preset, raw_layout, cache->query_w(), raw, n, rgb,
                                (hipStream_t)stream);
    else
        e = launch_fwd_raw_mfma(cache->cfg.precision, d, cache->cfg.enc_preset, raw_layout,
                                cache->query_ffr(), raw, n, rgb, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "fused forward launch");
    return ok();
}

int nrc_train_step(nrc_cache* cache, const void* enc, const float* target, int64_t n,
                   void* scratch, size_t scratch_bytes, float* loss_dev, int32_t* skipped_dev,
                   void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 1) return fail(NRC_EINVAL, "a training batch needs n >= 1");
    if (n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "training batch too large");
    if (!enc || !target || !scratch) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)target & 3) || ((uintptr_t)scratch & 255))
        return fail(NRC_EINVAL, "misaligned buffer (scratch must be 256-byte aligned)");
    if (((uintptr_t)loss_dev & 3) || ((uintptr_t)skipped_dev & 3)) return fail(NRC_EINVAL, "misaligned output");
    const size_t need = scratch_layout(cache->cfg, n).total;
    if (scratch_bytes < need)
        return fail(NRC_ENOMEM, "scratch of %zu bytes is smaller than the %zu bytes needed", scratch_bytes, need);
    const int rc = enqueue_train_step(cache, enc, target, nullptr, n, (char*)scratch, loss_dev, skipped_dev,
                                      (hipStream_t)stream);
    return rc == NRC_OK ? ok() : rc;
}

size_t nrc_act_ws_bytes(const nrc_config* cfg, int64_t n) {
    if (validate_config(cfg) != NRC_OK) return 0;
    if (n < 0 || n > ((int64_t)1 << 31)) { fail(NRC_EINVAL, "n must be in [0, 2^31]"); return 0; }
    ok();
    return act_layout(*cfg, n);
}

int nrc_forward_train(nrc_cache* cache, const void* enc, int64_t n, void* act_ws, size_t act_bytes, float* rgb,
                      void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 0 || n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "n must be in [0, 2^31]");
    if (n == 0) return ok();
    if (!enc || !act_ws || !rgb) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || !aligned16(act_ws) || ((uintptr_t)rgb & 3)) return fail(NRC_EINVAL, "misaligned buffer");
    if (cache->cfg.precision == NRC_FP32_VALU)
        return fail(NRC_EINVAL, "the vector-ALU FP32 form keeps no activation buffer (use nrc_forward)");
    const size_t need = act_layout(cache->cfg, n);
    if (act_bytes < need)
        return fail(NRC_ENOMEM, "activation buffer of %zu bytes is smaller than the %zu bytes needed", act_bytes, need);
    const Geo d = kernel_geo(cache->cfg);
    hipError_t e;
    if (cache->cfg.precision == NRC_FP32)
        e = launch_fwd_train_fp32(d, cache->w(), (const float*)enc, n, (float*)act_ws, rgb, (hipStream_t)stream);
    else
        e = launch_fwd_train_mfma(cache->cfg.precision, d, cache->ffr(), enc, n, act_ws, rgb, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "training forward launch");
    return ok();
}

int nrc_backward(nrc_cache* cache, const void* enc, const void* act_ws, const float* grad_rgb, int64_t n,
                 void* scratch, size_t scratch_bytes, float* grad_w, float* grad_enc, void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 1) return fail(NRC_EINVAL, "a backward batch needs n >= 1");
    if (n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "batch too large");
    if (!enc || !grad_rgb || !scratch || !grad_w) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)grad_rgb & 3) || ((uintptr_t)scratch & 255) ||
        ((uintptr_t)grad_w & 3) || (grad_enc && !aligned16(grad_enc)) || (act_ws && !aligned16(act_ws)))
        return fail(NRC_EINVAL, "misaligned buffer");
    const nrc_config& cfg = cache->cfg;
    const ScratchLayout sl = scratch_layout(cfg, n);
    if (scratch_bytes < sl.total)
        return fail(NRC_ENOMEM, "scratch of %zu bytes is smaller than the %zu bytes needed", scratch_bytes, sl.total);
    const Geo d = kernel_geo(cfg);
    char* sc = (char*)scratch;
    float* partials = (float*)(sc + sl.partials);
    float* loss_part = (float*)(sc + sl.loss_part);
    int32_t* tile_bad = (int32_t*)(sc + sl.flags);
    hipStream_t s = (hipStream_t)stream;
    // the upstream gradient is scaled by the loss scale before the backward
    // pass rounds it to FP16/BF16 and unscaled after the sums (a mean-reduced
    // loss over 2^16 records gives dL/dy near 1e-5, where FP16 is subnormal)
    const float scale = cfg.loss_scale;
    if (act_ws && cfg.precision == NRC_FP32_VALU)
        return fail(NRC_EINVAL, "the vector-ALU FP32 form keeps no activation buffer (pass NULL)");
    hipError_t e;
    if (cfg.precision == NRC_FP32_VALU)
        e = launch_train_fp32_valu(d, cache->w(), (const float*)enc, grad_rgb, nullptr, n, true, cfg.loss_eps,
                                   scale, partials, loss_part, tile_bad, grad_enc, s);
    else if (cfg.precision == NRC_FP32)
        e = launch_train_fp32(d, cache->w(), (const float*)enc, grad_rgb, nullptr, n, true, cfg.loss_eps, scale,
                              partials, loss_part, tile_bad, grad_enc, s, (const float*)act_ws);
    else
        e = launch_train_mfma(cfg.precision, d, cache->ffr(), cache->bfr(), enc, grad_rgb, nullptr, n, true,
                              cfg.loss_eps, scale, partials, loss_part, tile_bad, grad_enc, s, act_ws);
    if (e != hipSuccess) return device_fail(e, "backward kernel launch");
    e = launch_reduce(d, !fp32_form(cfg.precision), partials, (int)sl.tiles, 1.0f / scale, grad_w, loss_part,
                      1.0f, nullptr, s);
    if (e != hipSuccess) return device_fail(e, "gradient reduction launch");
    return ok();
}

// ---------------------------------------------------------------------------
// Training-record pipeline (Sec. 3.5 shuffle and batches, Sec. 3.2 self-training)
// ---------------------------------------------------------------------------
size_t nrc_shuffle_scratch_bytes(int64_t n) {
    if (n < 0) { fail(NRC_EINVAL, "n must be >= 0"); return 0; }
    ok();
    return shuffle_scratch_bytes();
}

int nrc_shuffle(int64_t n, uint64_t seed, int32_t* perm, void* scratch, size_t scratch_bytes,
                void* stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(NRC_EINVAL, "n must be in [0, 2^31)");
    if (n == 0) return ok();
    if (!perm || !scratch) return fail(NRC_EINVAL, "NULL buffer");
    if (((uintptr_t)perm & 3) || ((uintptr_t)scratch & 3)) return fail(NRC_EINVAL, "misaligned buffer");
    if (scratch_bytes < shuffle_scratch_bytes())
        return fail(NRC_ENOMEM, "shuffle scratch of %zu bytes is smaller than the %zu bytes needed",
                    scratch_bytes, shuffle_scratch_bytes());
    const hipError_t e = launch_shuffle(n, seed, perm, (int32_t*)scratch, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "shuffle launch");
    return ok();
}

int nrc_train_step_indexed(nrc_cache* cache, const void* enc, const float* target, const int32_t* idx,
                           int64_t n, void* scratch, size_t scratch_bytes, float* loss_dev,
                           int32_t* skipped_dev, void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (n < 1) return fail(NRC_EINVAL, "a training batch needs n >= 1");
    if (n > ((int64_t)1 << 31)) return fail(NRC_EINVAL, "training batch too large");
    if (!enc || !target || !idx || !scratch) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)target & 3) || ((uintptr_t)idx & 3) || ((uintptr_t)scratch & 255))
        return fail(NRC_EINVAL, "misaligned buffer (scratch must be 256-byte aligned)");
    if (((uintptr_t)loss_dev & 3) || ((uintptr_t)skipped_dev & 3)) return fail(NRC_EINVAL, "misaligned output");
    const size_t need = scratch_layout(cache->cfg, n).total;
    if (scratch_bytes < need)
        return fail(NRC_ENOMEM, "scratch of %zu bytes is smaller than the %zu bytes needed", scratch_bytes, need);
    const int rc = enqueue_train_step(cache, enc, target, idx, n, (char*)scratch, loss_dev, skipped_dev,
                                      (hipStream_t)stream);
    return rc == NRC_OK ? ok() : rc;
}

namespace {
// Frame scratch: the permutation, the shuffle's span counts, and one training
// step's scratch for the largest batch (the steps run one after another).
struct FrameLayout {
    size_t perm, counts, step, total;
    int64_t max_batch;
};

FrameLayout frame_layout(const nrc_config& c, int64_t n_records, int steps, int64_t batch) {
    FrameLayout L{};
    const int64_t used = n_records < steps * batch ? n_records : steps * batch;
    L.max_batch = (used + steps - 1) / steps;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    L.perm = take((size_t)n_records * 4);
    L.counts = take(shuffle_scratch_bytes());
    L.step = take(scratch_layout(c, L.max_batch).total);
    L.total = off;
    return L;
}

int check_frame_args(const nrc_config* cfg, int64_t n_records, int steps, int64_t batch) {
    if (steps < 1 || steps > 64) return fail(NRC_EINVAL, "steps must be in [1, 64]");
    if (batch < 1 || batch > ((int64_t)1 << 30)) return fail(NRC_EINVAL, "batch must be in [1, 2^30]");
    if (n_records < steps || n_records >= ((int64_t)1 << 31))
        return fail(NRC_EINVAL, "n_records must be in [steps, 2^31)");
    (void)cfg;
    return NRC_OK;
}
}  // namespace

size_t nrc_frame_scratch_bytes(const nrc_config* cfg, int64_t n_records, int steps, int64_t batch) {
    if (validate_config(cfg) != NRC_OK) return 0;
    if (check_frame_args(cfg, n_records, steps, batch) != NRC_OK) return 0;
    ok();
    return frame_layout(*cfg, n_records, steps, batch).total;
}

namespace {
// The frame's training steps on perm (validated arguments, scratch checked).
int enqueue_frame_steps(nrc_cache* cache, const void* enc, const float* target, const int32_t* perm,
                        int64_t n_records, int steps, int64_t batch, char* step_scratch, float* losses_dev,
                        int32_t* skipped_dev, hipStream_t s, int raw_layout = -1) {
    const int64_t used = n_records < steps * batch ? n_records : steps * batch;
    for (int k = 0; k < steps; ++k) {
        const int64_t lo = k * used / steps, hi = (k + 1) * used / steps;
        const int rc = enqueue_train_step(cache, enc, target, perm + lo, hi - lo, step_scratch, losses_dev + k,
                                          skipped_dev + k, s, LcgGather{}, raw_layout);
        if (rc != NRC_OK) return rc;
    }
    return ok();
}

int check_frame_buffers(nrc_cache* cache, const void* enc, const float* target, int64_t n_records, int steps,
                        int64_t batch, void* scratch, size_t scratch_bytes, float* losses_dev,
                        int32_t* skipped_dev, FrameLayout* L) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    const int rc0 = check_frame_args(&cache->cfg, n_records, steps, batch);
    if (rc0 != NRC_OK) return rc0;
    if (!enc || !target || !scratch || !losses_dev || !skipped_dev) return fail(NRC_EINVAL, "NULL buffer");
    if (!aligned16(enc) || ((uintptr_t)target & 3) || ((uintptr_t)scratch & 255) ||
        ((uintptr_t)losses_dev & 3) || ((uintptr_t)skipped_dev & 3))
        return fail(NRC_EINVAL, "misaligned buffer (scratch must be 256-byte aligned)");
    *L = frame_layout(cache->cfg, n_records, steps, batch);
    if (scratch_bytes < L->total)
        return fail(NRC_ENOMEM, "scratch of %zu bytes is smaller than the %zu bytes needed", scratch_bytes, L->total);
    return NRC_OK;
}
}  // namespace

namespace {
// nrc_train_frame's steps after validation; raw_layout >= 0: enc holds raw
// records the training kernels encode.
int enqueue_frame(nrc_cache* cache, const void* enc, const float* target, int64_t n_records, int steps,
                  int64_t batch, uint64_t seed, void* scratch, const FrameLayout& L, float* losses_dev,
                  int32_t* skipped_dev, void* stream, int raw_layout) {
    char* sc = (char*)scratch;
    hipStream_t s = (hipStream_t)stream;
    if ((n_records & (n_records - 1)) == 0) {
        // A power-of-two record count: the LCG's modulus is the record count,
        // the orbit skips nothing, and each step's kernel computes its records'
        // orbit positions itself (the same permutation nrc_shuffle writes).
        const uint32_t mask = (uint32_t)(n_records - 1);
        const Affine step{kLcgA, kLcgC};
        const uint32_t x0 = (uint32_t)(seed & mask);
        const int64_t used = n_records < steps * batch ? n_records : steps * batch;
        for (int k = 0; k < steps; ++k) {
            const int64_t lo = k * used / steps, hi = (k + 1) * used / steps;
            const LcgGather lg{step, apply(power(step, (uint64_t)lo), x0) & mask, mask};
            const int rc2 = enqueue_train_step(cache, enc, target, nullptr, hi - lo, sc + L.step, losses_dev + k,
                                               skipped_dev + k, s, lg, raw_layout);
            if (rc2 != NRC_OK) return rc2;
        }
        return ok();
    }
    int32_t* perm = (int32_t*)(sc + L.perm);
    hipError_t e = launch_shuffle(n_records, seed, perm, (int32_t*)(sc + L.counts), s);
    if (e != hipSuccess) return device_fail(e, "shuffle launch");
    return enqueue_frame_steps(cache, enc, target, perm, n_records, steps, batch, sc + L.step, losses_dev,
                               skipped_dev, s, raw_layout);
}
}  // namespace

int nrc_train_frame(nrc_cache* cache, const void* enc, const float* target, int64_t n_records, int steps,
                    int64_t batch, uint64_t seed, void* scratch, size_t scratch_bytes, float* losses_dev,
                    int32_t* skipped_dev, void* stream) {
    FrameLayout L;
    const int rc = check_frame_buffers(cache, enc, target, n_records, steps, batch, scratch, scratch_bytes,
                                       losses_dev, skipped_dev, &L);
    if (rc != NRC_OK) return rc;
    return enqueue_frame(cache, enc, target, n_records, steps, batch, seed, scratch, L, losses_dev, skipped_dev,
                         stream, -1);
}

int nrc_train_frame_raw(nrc_cache* cache, const float* raw, int raw_layout, const float* target,
                        int64_t n_records, int steps, int64_t batch, uint64_t seed, void* scratch,
                        size_t scratch_bytes, float* losses_dev, int32_t* skipped_dev, void* stream) {
    if (!cache) return fail(NRC_EINVAL, "cache is NULL");
    if (raw_layout != NRC_RAW14 && raw_layout != NRC_RAW16) return fail(NRC_EINVAL, "unknown raw layout %d", raw_layout);
    if (cache->cfg.width != 64) return fail(NRC_EINVAL, "the fused raw-record path supports width 64");
    FrameLayout L;
    const int rc = check_frame_buffers(cache, raw, target, n_records, steps, batch, scratch, scratch_bytes,
                                       losses_dev, skipped_dev, &L);
    if (rc != NRC_OK) return rc;
    return enqueue_frame(cache, raw, target, n_records, steps, batch, seed, scratch, L, losses_dev, skipped_dev,
                         stream, raw_layout);
}

int nrc_train_frame_indexed(nrc_cache* cache, const void* enc, const float* target, const int32_t* perm,
                            int64_t n_records, int steps, int64_t batch, void* scratch, size_t scratch_bytes,
                            float* losses_dev, int32_t* skipped_dev, void* stream) {
    FrameLayout L;
    const int rc = check_frame_buffers(cache, enc, target, n_records, steps, batch, scratch, scratch_bytes,
                                       losses_dev, skipped_dev, &L);
    if (rc != NRC_OK) return rc;
    if (!perm || ((uintptr_t)perm & 3)) return fail(NRC_EINVAL, "perm is NULL or misaligned");
    return enqueue_frame_steps(cache, enc, target, perm, n_records, steps, batch, (char*)scratch + L.step,
                               losses_dev, skipped_dev, (hipStream_t)stream);
}

int nrc_self_training_targets(const float* radiance, const float* throughput, const float* tail_rgb,
                              const int32_t* tail_index, int64_t n, int64_t n_tail, float* target,
                              void* stream) {
    if (n < 0 || n_tail < 0) return fail(NRC_EINVAL, "n and n_tail must be >= 0");
    if (n == 0) return ok();
    if (n_tail < 1) return fail(NRC_EINVAL, "records need at least one tail prediction");
    if (!radiance || !throughput || !tail_rgb || !tail_index || !target) return fail(NRC_EINVAL, "NULL buffer");
    if (((uintptr_t)radiance | (uintptr_t)throughput | (uintptr_t)tail_rgb | (uintptr_t)tail_index |
         (uintptr_t)target) & 3)
        return fail(NRC_EINVAL, "misaligned buffer");
    const hipError_t e = launch_self_train(radiance, throughput, tail_rgb, tail_index, n, n_tail, target,
                                           (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "self-training target launch");
    return ok();
}

size_t nrc_error_norms_scratch_bytes(int64_t n) {
    if (n < 0) { fail(NRC_EINVAL, "n must be >= 0"); return 0; }
    ok();
    return error_norms_scratch_bytes();
}

int nrc_error_norms(const float* got, const double* ref, int64_t n, void* scratch, size_t scratch_bytes,
                    double* out, void* stream) {
    if (n < 1 || n >= ((int64_t)1 << 40)) return fail(NRC_EINVAL, "n must be in [1, 2^40)");
    if (!got || !ref || !scratch || !out) return fail(NRC_EINVAL, "NULL buffer");
    if (((uintptr_t)got & 3) || ((uintptr_t)ref & 7) || ((uintptr_t)scratch & 7) || ((uintptr_t)out & 7))
        return fail(NRC_EINVAL, "misaligned buffer");
    if (scratch_bytes < error_norms_scratch_bytes())
        return fail(NRC_ENOMEM, "scratch of %zu bytes is smaller than the %zu bytes needed", scratch_bytes,
                    error_norms_scratch_bytes());
    const hipError_t e = launch_error_norms(got, ref, n, (double*)scratch, out, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "error-norm launch");
    return ok();
}

}  // extern "C"

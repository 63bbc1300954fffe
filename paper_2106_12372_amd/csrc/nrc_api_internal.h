// Host-side state of a cache and the layouts of the caller-owned device
// workspaces; shared by the C ABI and the serving loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nrc_internal.h"

namespace nrc {

// Byte offsets inside a cache workspace.
struct CacheLayout {
    size_t w, m, v, t, ffr, bfr, e, wbar, effr, total;
};

// Byte offsets inside the scratch of one training step / backward pass.
struct ScratchLayout {
    int64_t tiles;
    // partials: two regions of per-tile weight-gradient partials; consecutive
    // training steps of a cache alternate between them, so a step's kernel
    // never rewrites the lines the previous step's reduction has just read
    // (measured: that rewrite costs the training kernel ~3 us per step).
    size_t partials, partials2, loss_part, grad, flags, loss, skipped, total;
};

CacheLayout cache_layout(const nrc_config& c);
ScratchLayout scratch_layout(const nrc_config& c, int64_t n);
size_t act_layout(const nrc_config& c, int64_t n);
int validate_config(const nrc_config* c);
bool aligned16(const void* p);

int fail(int code, const char* fmt, ...);
int ok();
int device_fail(hipError_t e, const char* what);

}  // namespace nrc

struct nrc_cache {
    nrc_config cfg;
    nrc::CacheLayout lay;
    char* ws;
    int parity;  // which step-count slot holds the current count
    int device;
    float* w() { return (float*)(ws + lay.w); }
    float* m() { return (float*)(ws + lay.m); }
    float* v() { return (float*)(ws + lay.v); }
    int32_t* tslots() { return (int32_t*)(ws + lay.t); }
    void* ffr() { return nrc::fp32_form(cfg.precision) ? nullptr : (void*)(ws + lay.ffr); }
    void* bfr() { return nrc::fp32_form(cfg.precision) ? nullptr : (void*)(ws + lay.bfr); }
    bool ema() const { return cfg.ema_alpha > 0.0f; }
    float* e() { return ema() ? (float*)(ws + lay.e) : nullptr; }
    float* wbar() { return ema() ? (float*)(ws + lay.wbar) : nullptr; }
    void* effr() { return (ema() && !nrc::fp32_form(cfg.precision)) ? (void*)(ws + lay.effr) : nullptr; }
    // Weights the query entry points use: the EMA set when it is kept.
    const float* query_w() { return ema() ? wbar() : w(); }
    const void* query_ffr() { return ema() ? effr() : ffr(); }
};

namespace nrc {
// idx (may be NULL): the batch is records idx[0..n) of enc / target; lg (if
// its mask is set and idx is NULL): the batch is n records of the LCG orbit.
// raw_layout >= 0: enc holds raw records (FP32, that layout) that the
// training kernel encodes itself.
int enqueue_train_step(nrc_cache* c, const void* enc, const float* target, const int32_t* idx,
                       int64_t n, char* scratch, float* loss_dev, int32_t* skipped_dev, hipStream_t s,
                       LcgGather lg = LcgGather{}, int raw_layout = -1);
int enqueue_forward(nrc_cache* c, const void* enc, int64_t n, float* rgb, hipStream_t s);
}  // namespace nrc

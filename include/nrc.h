/*
 * nrc.h - C ABI of the MI355X neural radiance cache library.
 *
 * The cache is the network of Mueller et al., "Real-time Neural Radiance
 * Caching for Path Tracing" (arXiv 2106.12372): a bias-free ReLU MLP that maps
 * an encoded path vertex to cached scattered radiance (Sec. 3, Eq. 1), queried
 * once per terminal vertex and trained online from arrays of training records
 * (Sec. 3.5), with the input encodings of Sec. 3.6 / Table "parameters", the
 * architecture of Sec. 5, the relative L2 loss of Eq. 5 and Adam (Sec. 5).
 *
 * Conventions shared by every entry point:
 *  - Every call returns an int status (NRC_OK or a negative error code); no
 *    exception crosses the ABI.  nrc_last_error() gives a message for the last
 *    failing call on the calling thread.
 *  - Argument errors (null or misaligned pointers, negative sizes, bad enums,
 *    too-small workspaces) are reported before any device call is made.
 *  - The library never allocates device memory: the caller allocates and frees
 *    every device buffer (the cache workspace, scratch, inputs, outputs).
 *    Host-side handles are allocated by the library and freed by *_destroy.
 *    The one fixed device array the library holds is the scratch of
 *    nrc_train_step_noalloc (NRC_NOALLOC_SCRATCH_BYTES per GPU).
 *  - "stream" arguments are hipStream_t values passed as void*; NULL is the
 *    default stream.  Work is enqueued asynchronously; nothing synchronises
 *    the host unless stated.
 *  - Device pointers must be 16-byte aligned.  Row-major layouts throughout.
 *  - A cache handle must not be used from two threads at once; the serving
 *    entry points (nrc_serve_*) are thread-safe.
 */
#ifndef NRC_H
#define NRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define NRC_OK 0
#define NRC_PENDING 1
#define NRC_EINVAL (-1)
#define NRC_ENOMEM (-2)
#define NRC_EDEVICE (-3)
#define NRC_EBUSY (-4)
#define NRC_ENOTFOUND (-5)

/* Arithmetic of the layer products. */
#define NRC_FP32 0 /* FP32 products and sums (FP32 matrix cores), FP32 encoded input */
#define NRC_FP16 1 /* FP16 matrix-core products, FP32 accumulation and master weights */
#define NRC_BF16 2 /* BF16 matrix-core products, FP32 accumulation and master weights */
#define NRC_FP32_VALU 3 /* FP32 products and sums on the vector ALUs only, no matrix instructions: the
                           plain FP32 baseline (width 64, n_hidden <= 6; no activation buffer) */

/* Input encoding presets (Sec. 3.6, Table "parameters"). */
#define NRC_PRESET_CONFIG 0 /* 6 octaves sin+cos, roughness as is, zero pad */
#define NRC_PRESET_PAPER 1  /* 12 sines, one-blob of 1-exp(-r), pad with one */
#define NRC_PRESET_PAPER_TRI 2 /* as PAPER with the triangle wave of Sec. 5 in place of sin */
#define NRC_PRESET_PAPER_GAUSS 3 /* as PAPER with a Gaussian one-blob kernel (one bin wide), the
                                    kernel the quartic of Sec. 5 replaces */

/* Raw path-vertex record layouts (FP32, row-major). */
#define NRC_RAW14 0 /* pos 3 | dir (u,w) 2 | normal (u,w) 2 | roughness | diffuse 3 | specular 3 */
#define NRC_RAW16 1 /* pos 3 | dir xyz 3 | normal xyz 3 | roughness | diffuse 3 | specular 3 */

/* Width of the encoded input (62 features padded to 64, Sec. 3.6). */
#define NRC_ENC_WIDTH 64

/*
 * Cache configuration.  Architecture of Sec. 5: `n_hidden` hidden layers of
 * `width` ReLU neurons, no biases, a linear output of `n_out` (= 3, RGB).
 * Supported: width 64 or 128 (FP32 forms: 64 only); n_hidden 1..8 (FP32 forms: 1..6); n_out 3.
 * Adam (Sec. 5 Optimizer): lr, beta1, beta2, adam_eps; loss_eps is the eps of
 * Eq. 5; loss_scale multiplies the loss gradient before the reduced-precision
 * backward pass and is divided out before Adam (use 1 for FP32).
 * ema_alpha > 0 keeps the exponential moving average of the weights of Eq. 2
 * (Sec. 3.3), bias-corrected: W_bar_t = E_t / (1 - alpha^t) with
 * E_t = alpha E_{t-1} + (1 - alpha) W_t, advanced by every applied Adam step;
 * the query entry points (nrc_forward, nrc_forward_raw) then use W_bar, as the
 * paper does for rendering, while training and nrc_backward use W.  Before the
 * first step W_bar equals the weights that were set.
 */
typedef struct nrc_config {
    int32_t width;
    int32_t n_hidden;
    int32_t n_out;
    int32_t precision;  /* NRC_FP32 / NRC_FP16 / NRC_BF16 / NRC_FP32_VALU */
    int32_t enc_preset; /* NRC_PRESET_* */
    float lr;
    float beta1;
    float beta2;
    float adam_eps;
    float loss_eps;
    float loss_scale;
    float ema_alpha; /* EMA of the weights (Eq. 2); 0 disables, the paper uses 0.99 */
    int32_t factorize; /* 1: reflectance factorisation (Sec. 5): the prediction is the
                        * network output times (diffuse + specular albedo), per channel,
                        * both read from the encoded row (config preset: columns 53..55
                        * and 56..58; paper presets: 56..58 and 59..61).  Training,
                        * the loss and the gradients then act on the factorised value. */
    uint64_t seed;   /* reserved; weights are always set explicitly */
} nrc_config;

typedef struct nrc_cache nrc_cache;

/* Fills *cfg with the defaults: 64, 5, 3, FP16, CONFIG, 1e-2, 0.9, 0.99, 1e-8,
 * 0.01, 128, 0 (no EMA), 0 (no factorisation), 0.  Returns NRC_EINVAL on NULL. */
int nrc_config_default(nrc_config* cfg);

/* Message describing the last failure on the calling thread ("" if none).
 * Valid until the next nrc_* call on the same thread. */
const char* nrc_last_error(void);

/* Number of weights: width*64 + (n_hidden-1)*width^2 + 3*width (Sec. 5). */
int64_t nrc_param_count(const nrc_config* cfg);

/* Bytes of device workspace a cache needs (master weights, Adam moments, step
 * counter, reduced-precision weight copies).  0 on an invalid config. */
size_t nrc_cache_bytes(const nrc_config* cfg);

/* Bytes of device scratch one nrc_train_step / nrc_backward over n records
 * needs: two regions of per-tile weight-gradient partials (consecutive steps
 * of a cache alternate between them), loss partials and flags.  0 (with
 * NRC_EINVAL as the last error) on an invalid config or n outside [0, 2^31]. */
size_t nrc_train_scratch_bytes(const nrc_config* cfg, int64_t n);

/* Bytes per element of the encoded input at the cache precision (4 or 2). */
int nrc_enc_elem_bytes(const nrc_config* cfg);

/*
 * Creates a cache in the caller's device workspace `dev_ws` of at least
 * nrc_cache_bytes(cfg) bytes.  Weights start at zero; call nrc_set_weights.
 * Does not take ownership of dev_ws; nrc_cache_destroy does not free it.
 * `stream` is the stream used for the set-up copies.
 */
int nrc_cache_create(const nrc_config* cfg, void* dev_ws, size_t ws_bytes, void* stream,
                     nrc_cache** out);
int nrc_cache_destroy(nrc_cache* cache);
int nrc_cache_config(const nrc_cache* cache, nrc_config* out);

/*
 * Weights as one flat FP32 host array, matrices in layer order W_0 .. W_L,
 * each row-major [out][in] (Sec. 5 architecture; n = nrc_param_count).
 * set: also resets the Adam moments and step count; synchronises `stream`.
 * get: copies the FP32 master weights out; synchronises `stream`.
 */
int nrc_set_weights(nrc_cache* cache, const float* host_w, int64_t n, void* stream);
int nrc_get_weights(const nrc_cache* cache, float* host_w, int64_t n, void* stream);

/*
 * Same as nrc_set_weights with the weights in device memory (FP32, n floats):
 * enqueues the copy and the rebuild of the reduced-precision copies on
 * `stream` without synchronising.  Adam moments and step count are reset.
 * Used by the autograd wrapper, whose weights are a device tensor.
 */
int nrc_set_weights_device(nrc_cache* cache, const float* dev_w, int64_t n, void* stream);

/*
 * Full optimiser state for checkpoint/resume: weights, Adam first and second
 * moments (each n floats, host) and the step count t.  Synchronises `stream`.
 */
int nrc_get_state(const nrc_cache* cache, float* host_w, float* host_m, float* host_v,
                  int64_t n, int64_t* t, void* stream);
int nrc_set_state(nrc_cache* cache, const float* host_w, const float* host_m,
                  const float* host_v, int64_t n, int64_t t, void* stream);

/*
 * EMA weight set (caches with ema_alpha > 0): W_bar (the weights queries use)
 * and the running sum E, each n floats on the host, for inspection and
 * checkpoint/resume.  nrc_set_ema must follow nrc_set_state (which resets the
 * EMA to W_bar = W, E = 0).  Synchronises `stream`.
 */
int nrc_get_ema(const nrc_cache* cache, float* host_w_bar, float* host_e, int64_t n, void* stream);
int nrc_set_ema(nrc_cache* cache, const float* host_w_bar, const float* host_e, int64_t n,
                void* stream);

/*
 * Input encoding (Sec. 3.6, Table "parameters"): raw device records
 * [n][14] (NRC_RAW14) or [n][16] (NRC_RAW16) FP32 -> enc [n][64] at the cache
 * precision (FP32 for NRC_FP32, else FP16/BF16), using the cache's preset.
 * Position: frequency encoding; direction and normal: spherical coordinates
 * then one-blob with 4 quartic blobs; roughness, albedos as in the preset.
 * n == 0 is a no-op.
 */
int nrc_encode(const nrc_cache* cache, const float* raw, int raw_layout, int64_t n, void* enc,
               void* stream);

/*
 * Batched inference (Sec. 4, Fig. "fully-fused-illustration"): rgb[n][3]
 * (FP32, device) = network(enc[n][64]) with the current weights.  Any n >= 0.
 */
int nrc_forward(nrc_cache* cache, const void* enc, int64_t n, float* rgb, void* stream);

/*
 * Inference straight from raw records (Sec. 3.6 encodings + Sec. 4 network in
 * one kernel): rgb[n][3] = network(encode(raw[n][14 or 16])), the encoded
 * features never touching device memory.  Same result as nrc_encode followed by
 * nrc_forward (the features are rounded to the cache precision in both).
 * Width 64 only.  Any n >= 0.
 */
int nrc_forward_raw(nrc_cache* cache, const float* raw, int raw_layout, int64_t n, float* rgb,
                    void* stream);

/*
 * One optimisation step (Sec. 3.3 and 3.5, Eq. 5, Sec. 5): forward over the batch
 * enc[n][64] with targets target[n][3] (FP32), relative L2 loss, backward,
 * weight gradients summed over the batch, then one Adam update of the master
 * weights.  The loss (FP32 scalar) is written to *loss_dev and the skip flag
 * (1 if the gradient was not finite and the step was skipped, else 0) to
 * *skipped_dev, both device pointers (may be NULL).  `scratch` is device memory
 * of nrc_train_scratch_bytes(cfg, n) bytes.  n must be >= 1.
 */
int nrc_train_step(nrc_cache* cache, const void* enc, const float* target, int64_t n,
                   void* scratch, size_t scratch_bytes, float* loss_dev, int32_t* skipped_dev,
                   void* stream);

/*
 * nrc_train_step without a scratch argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The step's scratch is a fixed array inside the
 * library, NRC_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on a
 * GPU until the process ends; the call itself allocates nothing.  The result
 * equals nrc_train_step's bit for bit.  A batch whose scratch
 * (nrc_train_scratch_bytes(cfg, n)) exceeds the array is refused with
 * NRC_ENOMEM before any device call: at width 64 that is n up to about
 * 19,000 records, at width 128 about 2,700.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  Other arguments as for
 * nrc_train_step.
 */
#define NRC_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
int nrc_train_step_noalloc(nrc_cache* cache, const void* enc, const float* target, int64_t n,
                           float* loss_dev, int32_t* skipped_dev, void* stream);

/*
 * Autograd form (Sec. 4 "Training the fully fused neural network": the forward
 * pass keeps the activations that backpropagation reads).
 *
 * nrc_act_ws_bytes: bytes of the activation buffer for n records (0 with
 * NRC_EINVAL on an invalid config or n outside [0, 2^31]).
 *
 * nrc_forward_train: rgb[n][3] (FP32, device) = the prediction for enc[n][64]
 * with the training weights W (not the EMA set), and act_ws (device, 16-byte
 * aligned, act_bytes >= nrc_act_ws_bytes(cfg, n)) receives every hidden
 * layer's activations and the network outputs, for nrc_backward.  n == 0 is a
 * no-op.
 *
 * nrc_backward: given any upstream gradient grad_rgb[n][3] (FP32, device) of
 * the predictions for enc[n][64], writes grad_w (FP32, device, nrc_param_count
 * floats in the weight layout above, summed over the batch) and, if grad_enc
 * is not NULL, grad_enc[n][64] (FP32, device).  act_ws: the buffer
 * nrc_forward_train filled for the same enc, n and weights (its contents are
 * trusted, not checked), or NULL to recompute the forward pass inside the
 * kernel.  The upstream gradient is multiplied by the config's loss_scale
 * before the reduced-precision backward pass rounds it and divided out of
 * grad_w and grad_enc (grad_rgb * loss_scale must stay within FP16 range in
 * the FP16 form).  `scratch` as for nrc_train_step.  n must be >= 1.
 */
size_t nrc_act_ws_bytes(const nrc_config* cfg, int64_t n);
int nrc_forward_train(nrc_cache* cache, const void* enc, int64_t n, void* act_ws, size_t act_bytes, float* rgb,
                      void* stream);
int nrc_backward(nrc_cache* cache, const void* enc, const void* act_ws, const float* grad_rgb, int64_t n,
                 void* scratch, size_t scratch_bytes, float* grad_w, float* grad_enc, void* stream);

/* ------------------------------------------------------------------------- */
/* Training-record pipeline of one frame (Sec. 3.3 footnote, Sec. 3.5,       */
/* Sec. 3.2 self-training).                                                  */
/* ------------------------------------------------------------------------- */

/* Bytes of device scratch nrc_shuffle needs (a small constant, 4 KiB). */
size_t nrc_shuffle_scratch_bytes(int64_t n);

/*
 * Record shuffle of Sec. 3.5 ("shuffle all training records using a linear
 * congruential generator").  Writes perm[0..n) (int32, device), a permutation
 * of 0..n-1: the orbit x_0 = seed mod m, x_{i+1} = (a x_i + c) mod m of the
 * full-period LCG on m = the smallest power of two >= n, with values >= n
 * skipped; a = 1284865837 and c = 4150755663 (Knuth's MMIX multiplier and
 * increment reduced mod 2^32).  The same (n, seed) always gives the same
 * order.  scratch: device, 4-byte aligned, nrc_shuffle_scratch_bytes(n);
 * overwritten.  0 <= n < 2^31.  Asynchronous on `stream`.
 */
int nrc_shuffle(int64_t n, uint64_t seed, int32_t* perm, void* scratch, size_t scratch_bytes,
                void* stream);

/*
 * One training step (as nrc_train_step) on the records idx[0..n) of enc and
 * target: the batch is gathered inside the training kernel.  idx: device int32,
 * each entry a valid row of enc / target (not checked).  scratch as for
 * nrc_train_step with this n.
 */
int nrc_train_step_indexed(nrc_cache* cache, const void* enc, const float* target,
                           const int32_t* idx, int64_t n, void* scratch, size_t scratch_bytes,
                           float* loss_dev, int32_t* skipped_dev, void* stream);

/* Bytes of device scratch nrc_train_frame needs; 0 on invalid arguments. */
size_t nrc_frame_scratch_bytes(const nrc_config* cfg, int64_t n_records, int steps, int64_t batch);

/*
 * The cache update of one frame (Sec. 3.3 footnote, Sec. 3.5): shuffle the
 * n_records training records (nrc_shuffle with `seed`), take the first
 * used = min(n_records, steps * batch) of them, and run `steps` training
 * steps, step k on shuffled records [k used / steps, (k+1) used / steps)
 * (disjoint batches, exactly `batch` records each when n_records >= steps *
 * batch; the paper uses steps = 4, batch = 16384).  losses_dev[steps] and
 * skipped_dev[steps] (device) receive each step's loss and skip flag.
 * enc[n_records][64] at the cache precision, target[n_records][3] FP32, both
 * device.  steps in [1, 64], n_records in [steps, 2^31).  scratch: device,
 * 256-byte aligned, nrc_frame_scratch_bytes.  Everything is enqueued on
 * `stream`; nothing waits for the host.
 */
int nrc_train_frame(nrc_cache* cache, const void* enc, const float* target, int64_t n_records,
                    int steps, int64_t batch, uint64_t seed, void* scratch, size_t scratch_bytes,
                    float* losses_dev, int32_t* skipped_dev, void* stream);

/*
 * The training steps of nrc_train_frame on a permutation the caller has
 * already computed (for example nrc_shuffle with the frame's seed, enqueued on
 * another stream beside the frame's query pass: neither the shuffle nor the
 * records' encoding reads the weights, so only the training steps need to
 * follow the queries).  perm[n_records]: device int32, each entry a valid row
 * of enc / target (not checked); steps k runs on perm[k used / steps,
 * (k+1) used / steps) with used = min(n_records, steps * batch), exactly as
 * nrc_train_frame.  Other arguments and the scratch size
 * (nrc_frame_scratch_bytes) as for nrc_train_frame.  With perm from
 * nrc_shuffle(n_records, seed) the result equals nrc_train_frame(seed) bit for
 * bit.
 */
int nrc_train_frame_indexed(nrc_cache* cache, const void* enc, const float* target, const int32_t* perm,
                            int64_t n_records, int steps, int64_t batch, void* scratch,
                            size_t scratch_bytes, float* losses_dev, int32_t* skipped_dev, void* stream);

/*
 * nrc_train_frame on raw training records (the path-vertex records of Sec.
 * 3.6, Table "parameters", before the input encoding): the training kernels
 * encode each gathered record with the cache's preset, exactly as
 * nrc_encode would, so the result equals nrc_encode followed by
 * nrc_train_frame bit for bit, without the encoded copy of the records.
 * raw: device FP32 [n_records][14] (NRC_RAW14) or [n_records][16]
 * (NRC_RAW16), 16-byte aligned; raw_layout one of those.  Width 64 only
 * (NRC_EINVAL otherwise), as nrc_forward_raw.  Other arguments, the scratch
 * size (nrc_frame_scratch_bytes) and the errors as for nrc_train_frame.
 */
int nrc_train_frame_raw(nrc_cache* cache, const float* raw, int raw_layout, const float* target,
                        int64_t n_records, int steps, int64_t batch, uint64_t seed, void* scratch,
                        size_t scratch_bytes, float* losses_dev, int32_t* skipped_dev, void* stream);

/*
 * Self-training targets (Sec. 3.2, Sec. 6 "Self-training"): a training
 * record's target is the radiance gathered from its vertex to the end of its
 * path plus the throughput from its vertex to the path's tail times the
 * cache's prediction at the tail vertex (an nrc_forward / nrc_forward_raw of
 * the tail queries):
 *   target[i][c] = radiance[i][c] + throughput[i][c] * tail_rgb[tail_index[i]][c].
 * All arrays FP32 [.][3] (tail_index int32 [n]), device.  A tail_index outside
 * [0, n_tail) gives a NaN target, so the training step that uses it skips.
 */
int nrc_self_training_targets(const float* radiance, const float* throughput, const float* tail_rgb,
                              const int32_t* tail_index, int64_t n, int64_t n_tail, float* target,
                              void* stream);

/*
 * Validation: per-channel error norms of a batch of predictions against
 * reference values, reduced in FP64 on the device (the inputs of the
 * per-channel relative errors of the precision forms, normwise in the L2 and
 * the max norm).  got: device FP32 [n][3]; ref: device FP64 [n][3]; out:
 * device FP64 [3][4] with, for channel c,
 *   out[c][0] = sum_i (got_ic - ref_ic)^2,  out[c][1] = sum_i ref_ic^2,
 *   out[c][2] = max_i |got_ic - ref_ic|,    out[c][3] = max_i |ref_ic|.
 * scratch: device, 8-byte aligned, nrc_error_norms_scratch_bytes(n) bytes.
 * The summation order is fixed, so the result is bitwise reproducible.
 * n in [1, 2^40).
 */
size_t nrc_error_norms_scratch_bytes(int64_t n);
int nrc_error_norms(const float* got, const double* ref, int64_t n, void* scratch, size_t scratch_bytes,
                    double* out, void* stream);

/* ------------------------------------------------------------------------- */
/* Serving: continuous batching of inference and training requests over     */
/* several resident caches.                                                  */
/* ------------------------------------------------------------------------- */
#define NRC_REQ_INFER 0
#define NRC_REQ_TRAIN 1

typedef struct nrc_server nrc_server;

typedef struct nrc_serve_config {
    int32_t n_caches;        /* number of independent caches (1..64) */
    nrc_config cache_cfg;    /* configuration shared by all caches */
    void* arena;             /* device memory for caches and per-request scratch */
    size_t arena_bytes;
    int32_t n_streams;       /* HIP streams the scheduler launches on (1..16) */
    int32_t max_inflight;    /* requests on the device at once (>= 1) */
} nrc_serve_config;

typedef struct nrc_request {
    int32_t kind;            /* NRC_REQ_INFER or NRC_REQ_TRAIN */
    const void* enc;         /* device [n][64] at the cache precision */
    const float* target;     /* device [n][3] (training only) */
    float* rgb;              /* device [n][3] output (inference only) */
    int64_t n;
} nrc_request;

typedef struct nrc_result {
    int32_t status;          /* NRC_OK, NRC_PENDING or an error */
    int32_t skipped;         /* training: step skipped on a non-finite gradient */
    float loss;              /* training: loss of the step */
    double t_submit;         /* seconds, monotonic clock */
    double t_start;          /* seconds, when launched */
    double t_done;           /* seconds, when its completion was observed */
} nrc_result;

/* Creates the server: carves one cache workspace per cache out of the arena
 * and keeps the remainder for per-request scratch.  Weights start at zero. */
int nrc_serve_create(const nrc_serve_config* cfg, nrc_server** out);
/* Sets the weights of one cache (synchronous). */
int nrc_serve_set_weights(nrc_server* srv, int cache_id, const float* host_w, int64_t n);
int nrc_serve_get_weights(nrc_server* srv, int cache_id, float* host_w, int64_t n);
/* Queues a request and returns a ticket without blocking.  NRC_ENOMEM if the
 * request could never fit the arena.  Request buffers must stay valid until
 * nrc_serve_poll returns NRC_OK for the ticket.  Requests on one cache run in
 * submission order.  The server launches on its own non-blocking streams and
 * does not wait for device work the caller enqueued elsewhere: the request's
 * inputs must be complete, and nothing else may write its buffers, from the
 * call on (synchronise the producing stream first). */
int nrc_serve_submit(nrc_server* srv, int cache_id, const nrc_request* req, uint64_t* ticket);
/* NRC_PENDING until the request has finished, then NRC_OK and *res filled
 * (once; a finished ticket is then forgotten: NRC_ENOTFOUND afterwards). */
int nrc_serve_poll(nrc_server* srv, uint64_t ticket, nrc_result* res);
/* Blocks until every submitted request has finished. */
int nrc_serve_drain(nrc_server* srv);
/* NRC_EBUSY while requests are pending (call nrc_serve_drain first). */
int nrc_serve_destroy(nrc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* NRC_H */

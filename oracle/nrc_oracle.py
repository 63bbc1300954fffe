"""FP64 CPU oracle of the neural radiance cache hot path.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
definition that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library or its Python
binding: both sides only read the same seeded inputs (``synthdata``).

Everything is float64 NumPy, one step at a time in the order the paper states
it.  Citations name the section, equation or table of Mueller et al.,
"Real-time Neural Radiance Caching for Path Tracing" (arXiv 2106.12372).

Readings of points the paper leaves open (each also listed in the design
notes):

* Table "parameters" + Sec. 3.6 (Input Encoding): 14-float records carry the
  spherical coordinates already; 16-float records carry unit vectors that go
  through ``sph``.
* ``sph`` (Table "parameters"): u = arccos(z)/pi, w = (atan2(y, x) + pi)/(2 pi).
* Frequency encoding (Sec. 3.6): the "config" preset uses 6 octaves d = 0..5
  with both sin and cos of 2^d*pi*p (12 features per coordinate); the "paper"
  preset uses 12 sines, d = 0..11.  Order: coordinate, then octave, then
  (sin, cos).  The phase is reduced exactly, r = (2^d p) mod 2, before sin(pi r).
* One-blob (Sec. 3.6, Sec. 5 cheap primitives): k = 4 bins on [0,1]; the blob is
  the quartic kernel 15/16 (1-x^2)^2 of half-width one bin, centred at k*s, and
  each bin receives the kernel mass over it; the two edge bins also take the
  tails, so the k values sum to one.
* Padding (Sec. 3.6): the config preset pads with 0 (roughness enters as is);
  the paper preset encodes 1 - exp(-r) with one-blob and pads with 1.
* Cheap primitives (Sec. 5): the one-blob kernel is the quartic throughout;
  the "paper-tri" preset also replaces each sine sin(2^d pi p) by the triangle
  wave the paper defines in its figure "cheap_primitives",
  tri(x) = 2|x mod 2 - 1| - 1, evaluated at x = 2^d p.  Its period is 2, that
  of sin(pi x); its phase is the printed one (tri(0) = 1, tri(1) = -1, the
  phase of cos(pi x)), which the paper gives and the oracle keeps.  The
  "paper-gauss" preset keeps
  the sines and uses the kernel the quartic replaced, a Gaussian: the paper
  gives no width (it defers the one-blob encoding to its earlier work), read
  as a standard deviation of one bin, with the bin masses from the normal CDF
  Phi(u) = (1 + erf(u / sqrt 2)) / 2 and the edge bins again taking the tails.
* Architecture (Sec. 5 Architecture): 6 weight matrices, no biases, ReLU after
  each hidden layer, linear output.  ReLU'(0) = 0.
* Loss (Eq. 5, Sec. 5 Relative loss): per channel (y_hat - y)^2 / (lum^2 + eps)
  with lum the mean of the three predicted channels, held constant in the
  gradient; mean over all 3n terms; eps = 0.01.
* Adam (Sec. 5 Optimizer): Kingma-Ba with bias correction, eps added to
  sqrt(v_hat), no weight decay, first step t = 1.  A step whose gradient is not
  finite is skipped (t unchanged).
* Loss scaling is a rounding device of reduced-precision arithmetic; in FP64
  it cancels exactly, so the oracle has no scale.
* EMA of the weights (Eq. 2): as printed its two coefficients do not sum to
  one; it is read as the bias-corrected average
  W_bar_t = [(1 - a) W_t + a eta_{t-1} W_bar_{t-1}] / eta_t, eta_t = 1 - a^t,
  i.e. W_bar_t = E_t / eta_t with E_t = a E_{t-1} + (1 - a) W_t, E_0 = 0.  It
  advances only on steps that update the weights and never feeds back.
* Record shuffle (Sec. 3.5): the paper shuffles the training records with a
  linear congruential generator but gives no constants.  Read as the orbit of
  a full-period LCG x_{i+1} = (a x_i + c) mod m on m = 2^ceil(log2 n) (Hull and
  Dobell: c odd and a = 1 mod 4 give period m), started at x_0 = seed mod m,
  with values >= n skipped: a permutation of the n records.  a and c are
  Knuth's MMIX multiplier and increment reduced mod 2^32.  The frame uses the
  first min(n, s l) shuffled records, cut into s consecutive batches of
  near-equal size (exactly l each when n >= s l).
* Self-training (Sec. 3.2, Sec. 6 Self-training): a record's target is the
  radiance gathered from its vertex to the tail of its path plus the
  throughput to the tail times the cache's prediction at the tail vertex.
* Reflectance factorisation (Sec. 5): the cache's prediction is the network
  output times alpha + beta, per channel; alpha and beta are the identity-
  encoded diffuse and specular albedo columns of the network input itself, so
  the factor is a function of the input row.  The loss (Eq. 5, luminance of
  the factorised prediction) and its gradient act on the factorised value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Constants fixed by the paper
# ---------------------------------------------------------------------------
LOSS_EPS = 0.01        # Eq. 5
N_BLOBS = 4            # Sec. 3.6, k = 4
PAPER_OCTAVES = 12     # Sec. 3.6, frequencies 2^d, d = 0..11
CONFIG_OCTAVES = 6     # config preset: 6 octaves x (sin, cos)
ENC_WIDTH = 64         # Sec. 3.6: 62 features padded to 64

RAW14 = 0
RAW16 = 1
PRESET_CONFIG = 0
PRESET_PAPER = 1
PRESET_PAPER_TRI = 2   # paper preset with the triangle wave in place of sin (Sec. 5)
PRESET_PAPER_GAUSS = 3  # paper preset with a Gaussian one-blob kernel in place of the quartic (Sec. 5)
PAPER_PRESETS = (PRESET_PAPER, PRESET_PAPER_TRI, PRESET_PAPER_GAUSS)


def albedo_columns(preset: int):
    """Columns of the diffuse and specular albedo in the encoded row (Sec. 3.6
    concatenation order): after roughness at 52 (config), after the roughness
    one-blob at 52..55 (paper)."""
    return (56, 59) if preset in PAPER_PRESETS else (53, 56)


# ---------------------------------------------------------------------------
# Encodings (Sec. 3.6, Table "parameters", Sec. 5 high-performance primitives)
# ---------------------------------------------------------------------------
def sph(v: np.ndarray) -> np.ndarray:
    """Unit vector [n][3] -> spherical coordinates normalised to [0,1]^2 (Table "parameters")."""
    v = np.asarray(v, dtype=np.float64)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    return np.stack([theta / np.pi, (phi + np.pi) / (2.0 * np.pi)], axis=1)


def tri(x: np.ndarray) -> np.ndarray:
    """Triangle wave of Sec. 5 (figure "cheap_primitives"), the stand-in for the
    sine of the frequency encoding: 2 |x mod 2 - 1| - 1, period 2."""
    return 2.0 * np.abs(np.mod(x, 2.0) - 1.0) - 1.0


def freq(p: np.ndarray, preset: int = PRESET_CONFIG) -> np.ndarray:
    """Frequency encoding of positions [n][3] (Sec. 3.6): 12 features per coordinate."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    cols = []
    for c in range(3):
        if preset == PRESET_PAPER_TRI:
            # the sine of frequency 2^d replaced by the triangle wave of the same period
            for d in range(PAPER_OCTAVES):
                cols.append(tri(p[:, c] * 2.0 ** d))
        elif preset in (PRESET_PAPER, PRESET_PAPER_GAUSS):
            for d in range(PAPER_OCTAVES):
                r = np.mod(p[:, c] * 2.0 ** d, 2.0)
                cols.append(np.sin(np.pi * r))
        else:
            for d in range(CONFIG_OCTAVES):
                r = np.mod(p[:, c] * 2.0 ** d, 2.0)
                cols.append(np.sin(np.pi * r))
                cols.append(np.cos(np.pi * r))
    return np.stack(cols, axis=1).reshape(n, 36)


def quartic_cdf(u: np.ndarray) -> np.ndarray:
    """CDF of the quartic kernel 15/16 (1 - x^2)^2 on [-1, 1] (Sec. 5, cheap primitives)."""
    u = np.asarray(u, dtype=np.float64)
    uc = np.clip(u, -1.0, 1.0)
    inner = 0.5 + (15.0 / 16.0) * (uc - (2.0 / 3.0) * uc ** 3 + 0.2 * uc ** 5)
    return np.where(u <= -1.0, 0.0, np.where(u >= 1.0, 1.0, inner))


def gauss_cdf(u: np.ndarray) -> np.ndarray:
    """CDF of the standard normal kernel, (1 + erf(u / sqrt 2)) / 2."""
    u = np.asarray(u, dtype=np.float64)
    return 0.5 * (1.0 + np.vectorize(math.erf)(u / math.sqrt(2.0)))


def one_blob(s: np.ndarray, k: int = N_BLOBS, cdf=quartic_cdf) -> np.ndarray:
    """One-blob encoding of scalars in [0,1] into k bins (Sec. 3.6): kernel mass
    per bin, the kernel centred at k s in bin units, the edge bins taking the tails."""
    s = np.asarray(s, dtype=np.float64)
    c = k * s
    out = np.empty(s.shape + (k,), dtype=np.float64)
    for j in range(k):
        hi = np.ones_like(c) if j == k - 1 else cdf(j + 1 - c)
        lo = np.zeros_like(c) if j == 0 else cdf(j - c)
        out[..., j] = hi - lo
    return out


def encode(raw: np.ndarray, layout: int = RAW14, preset: int = PRESET_CONFIG) -> np.ndarray:
    """Raw path-vertex records -> 64-wide network input (Sec. 3.6, Table "parameters")."""
    raw = np.asarray(raw, dtype=np.float64)
    n = raw.shape[0]
    pos = raw[:, 0:3]
    if layout == RAW14:
        d_sph, n_sph, rest = raw[:, 3:5], raw[:, 5:7], raw[:, 7:14]
    elif layout == RAW16:
        d_sph, n_sph, rest = sph(raw[:, 3:6]), sph(raw[:, 6:9]), raw[:, 9:16]
    else:
        raise ValueError(f"unknown layout {layout}")
    rough, diffuse, specular = rest[:, 0:1], rest[:, 1:4], rest[:, 4:7]
    cdf = gauss_cdf if preset == PRESET_PAPER_GAUSS else quartic_cdf
    parts = [freq(pos, preset),
             one_blob(d_sph, cdf=cdf).reshape(n, 8),
             one_blob(n_sph, cdf=cdf).reshape(n, 8)]
    paper = preset in PAPER_PRESETS
    if paper:
        parts.append(one_blob(1.0 - np.exp(-rough[:, 0]), cdf=cdf).reshape(n, 4))
    else:
        parts.append(rough)
    parts += [diffuse, specular]
    body = np.concatenate(parts, axis=1)
    pad_value = 1.0 if paper else 0.0
    pad = np.full((n, ENC_WIDTH - body.shape[1]), pad_value)
    return np.concatenate([body, pad], axis=1)


# ---------------------------------------------------------------------------
# Network (Sec. 4, Sec. 5 Architecture)
# ---------------------------------------------------------------------------
def forward(mats, h0: np.ndarray):
    """Bias-free ReLU MLP. Returns (y_hat [n][n_out], [h_0, ..., h_L]) with h_l the input of W_l."""
    h = np.asarray(h0, dtype=np.float64)
    hs = [h]
    for l, w in enumerate(mats):
        z = h @ np.asarray(w, dtype=np.float64).T
        if l == len(mats) - 1:
            return z, hs
        h = np.maximum(z, 0.0)
        hs.append(h)
    raise ValueError("empty network")


def relative_l2(y_hat: np.ndarray, y: np.ndarray, eps: float = LOSS_EPS):
    """Relative L2 loss of Eq. 5 with luminance normalisation; returns (loss, dL/dy_hat).

    The denominator uses the prediction with its gradient stopped, so it is a
    constant in the derivative.  The loss is the mean over all 3n terms.
    """
    y_hat = np.asarray(y_hat, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = y_hat.shape[0]
    if n == 0:
        return 0.0, np.zeros_like(y_hat)
    lum = y_hat.mean(axis=1, keepdims=True)
    denom = lum * lum + eps
    diff = y_hat - y
    loss = float((diff * diff / denom).sum() / (3 * n))
    grad = 2.0 * diff / denom / (3 * n)
    return loss, grad


def backward(mats, hs, delta_out: np.ndarray):
    """Reverse pass of `forward` given dL/dy_hat: returns (dW list, dL/dh_0)."""
    grads = [None] * len(mats)
    delta = np.asarray(delta_out, dtype=np.float64)        # dL/dz of the current layer's output
    for l in range(len(mats) - 1, -1, -1):
        w = np.asarray(mats[l], dtype=np.float64)
        grads[l] = delta.T @ hs[l]                         # sum over the batch of delta h^T
        g_in = delta @ w                                   # dL/dh_l
        if l == 0:
            return grads, g_in
        delta = g_in * (hs[l] > 0.0)                       # through ReLU: h_l = max(z_l, 0)
    raise ValueError("empty network")


# ---------------------------------------------------------------------------
# Optimiser (Sec. 5 Optimizer)
# ---------------------------------------------------------------------------
@dataclass
class AdamConfig:
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.99
    eps: float = 1e-8


def adam(w: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, g: np.ndarray, cfg: AdamConfig):
    """One Adam update (Kingma & Ba) of flat float64 arrays; returns (w, m, v, t)."""
    t = t + 1
    m = cfg.beta1 * m + (1.0 - cfg.beta1) * g
    v = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
    m_hat = m / (1.0 - cfg.beta1 ** t)
    v_hat = v / (1.0 - cfg.beta2 ** t)
    w = w - cfg.lr * m_hat / (np.sqrt(v_hat) + cfg.eps)
    return w, m, v, t


# ---------------------------------------------------------------------------
# Cache state, training step, frame (Sec. 3.3 footnote, Sec. 3.5)
# ---------------------------------------------------------------------------
def layer_shapes(width: int, n_hidden: int, n_in: int = ENC_WIDTH, n_out: int = 3):
    return [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(n_out, width)]


@dataclass
class CacheState:
    """Flat float64 master weights, Adam moments and step count of one cache."""
    w: np.ndarray
    width: int = 64
    n_hidden: int = 5
    m: np.ndarray = None
    v: np.ndarray = None
    t: int = 0
    adam: AdamConfig = field(default_factory=AdamConfig)
    loss_eps: float = LOSS_EPS
    ema_alpha: float = 0.0      # Sec. 3.3 uses 0.99; 0 disables the EMA set
    w_bar: np.ndarray = None
    factorize: bool = False     # Sec. 5 reflectance factorisation
    preset: int = PRESET_CONFIG  # encoding preset: where the albedo columns sit

    def __post_init__(self):
        self.w = np.asarray(self.w, dtype=np.float64).copy()
        if self.m is None:
            self.m = np.zeros_like(self.w)
        if self.v is None:
            self.v = np.zeros_like(self.w)

    def mats(self):
        out, off = [], 0
        for o, i in layer_shapes(self.width, self.n_hidden):
            out.append(self.w[off:off + o * i].reshape(o, i))
            off += o * i
        return out


def reflectance(enc: np.ndarray, preset: int) -> np.ndarray:
    """alpha + beta per channel (Sec. 5 Reflectance factorization), [n][3]."""
    enc = np.asarray(enc, dtype=np.float64)
    a, b = albedo_columns(preset)
    return enc[:, a:a + 3] + enc[:, b:b + 3]


def predict(state: CacheState, enc: np.ndarray) -> np.ndarray:
    """Cache query: the network output, times alpha + beta when factorised."""
    out = forward(state.mats(), enc)[0]
    if state.factorize:
        out = out * reflectance(enc, state.preset)
    return out


def ema_step(w_bar_prev: np.ndarray, w: np.ndarray, t: int, alpha: float) -> np.ndarray:
    """One step of Eq. 2 (bias-corrected reading): W_bar_t from W_bar_{t-1} and W_t."""
    eta_t = 1.0 - alpha ** t
    eta_prev = 1.0 - alpha ** (t - 1)
    return ((1.0 - alpha) * w + alpha * eta_prev * w_bar_prev) / eta_t


def gradient(state: CacheState, enc: np.ndarray, y: np.ndarray):
    """Loss and flat weight gradient of one batch (Eq. 5 through the network).
    Factorised: y_hat = f * R with R = alpha + beta, so dL/df = dL/dy_hat * R."""
    mats = state.mats()
    f, hs = forward(mats, enc)
    r = reflectance(enc, state.preset) if state.factorize else 1.0
    loss, d_out = relative_l2(f * r, y, state.loss_eps)
    grads, _ = backward(mats, hs, d_out * r)
    return loss, np.concatenate([g.reshape(-1) for g in grads])


def query_gradient(state: CacheState, enc: np.ndarray, grad_out: np.ndarray):
    """Gradients of a scalar whose gradient with respect to the cache's
    prediction is `grad_out` [n][3]: (flat weight gradient, input gradient
    [n][64]).  Factorised, the input gradient also takes d(f R)/dR = f on each
    albedo column."""
    mats = state.mats()
    f, hs = forward(mats, enc)
    grad_out = np.asarray(grad_out, dtype=np.float64)
    if not state.factorize:
        grads, g_in = backward(mats, hs, grad_out)
    else:
        grads, g_in = backward(mats, hs, grad_out * reflectance(enc, state.preset))
        a, b = albedo_columns(state.preset)
        g_in[:, a:a + 3] += grad_out * f
        g_in[:, b:b + 3] += grad_out * f
    return np.concatenate([g.reshape(-1) for g in grads]), g_in


def train_step(state: CacheState, enc: np.ndarray, y: np.ndarray):
    """One optimisation step on one batch; returns (loss, skipped).  With
    state.ema_alpha > 0 the EMA weight set (Eq. 2) follows the new weights."""
    loss, g = gradient(state, enc, y)
    if not np.all(np.isfinite(g)):
        return loss, True
    state.w, state.m, state.v, state.t = adam(state.w, state.m, state.v, state.t, g, state.adam)
    if state.ema_alpha > 0.0:
        prev = state.w_bar if state.w_bar is not None else np.zeros_like(state.w)
        state.w_bar = ema_step(prev, state.w, state.t, state.ema_alpha)
    return loss, False


def predict_ema(state: CacheState, enc: np.ndarray) -> np.ndarray:
    """Cache query with the EMA weights (Sec. 3.3): the set used for rendering."""
    w = state.w_bar if state.w_bar is not None else state.w
    return predict(CacheState(w, width=state.width, n_hidden=state.n_hidden,
                              factorize=state.factorize, preset=state.preset), enc)


# ---------------------------------------------------------------------------
# Training-record pipeline (Sec. 3.5 shuffle, Sec. 3.2 self-training)
# ---------------------------------------------------------------------------
LCG_A = 6364136223846793005 % 2 ** 32   # = 5 (mod 8)
LCG_C = 1442695040888963407 % 2 ** 32   # odd


def lcg_modulus(n: int) -> int:
    m = 1
    while m < n:
        m *= 2
    return m


def lcg_permutation(n: int, seed: int) -> np.ndarray:
    """Shuffled record order: the LCG orbit from seed mod m with values >= n skipped."""
    m = lcg_modulus(n)
    x = seed % m
    out = []
    for _ in range(m):
        if x < n:
            out.append(x)
        x = (LCG_A * x + LCG_C) % m
    return np.array(out, dtype=np.int64)


def frame_batches(n: int, steps: int, batch: int, seed: int):
    """Record indices of each of the `steps` training batches of one frame."""
    perm = lcg_permutation(n, seed)
    used = min(n, steps * batch)
    return [perm[s * used // steps:(s + 1) * used // steps] for s in range(steps)]


def self_training_targets(radiance: np.ndarray, throughput: np.ndarray, tail_rgb: np.ndarray,
                          tail_index: np.ndarray) -> np.ndarray:
    """target_i = radiance_i + throughput_i * tail_rgb[tail_index_i], per channel."""
    radiance = np.asarray(radiance, dtype=np.float64)
    throughput = np.asarray(throughput, dtype=np.float64)
    tail_rgb = np.asarray(tail_rgb, dtype=np.float64)
    return radiance + throughput * tail_rgb[np.asarray(tail_index)]


def frame_shuffled(state: CacheState, query_enc: np.ndarray, record_enc: np.ndarray,
                   record_y: np.ndarray, steps: int = 4, batch: int = 16384, seed: int = 0):
    """One frame with the shuffle: queries with the start-of-frame weights, then one
    step per shuffled batch (Sec. 3.3 footnote, Sec. 3.5)."""
    rgb = predict(state, query_enc)
    losses, skips = [], []
    for idx in frame_batches(record_enc.shape[0], steps, batch, seed):
        if idx.size == 0:
            losses.append(0.0)
            skips.append(True)
            continue
        loss, skipped = train_step(state, record_enc[idx], record_y[idx])
        losses.append(loss)
        skips.append(skipped)
    return rgb, losses, skips


def frame(state: CacheState, query_enc: np.ndarray, record_enc: np.ndarray,
          record_y: np.ndarray, n_steps: int = 4):
    """One frame: queries with the start-of-frame weights, then `n_steps` steps on
    disjoint consecutive slices of the training records (Sec. 3.3 footnote, Sec. 3.5)."""
    rgb = predict(state, query_enc)
    n = record_enc.shape[0]
    per = n // n_steps
    losses = []
    for s in range(n_steps):
        sl = slice(s * per, (s + 1) * per)
        loss, _ = train_step(state, record_enc[sl], record_y[sl])
        losses.append(loss)
    return rgb, losses


def channel_rel_error(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Normwise relative error per channel: max_i |got-ref| / max_i |ref|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref), axis=0)
    den = np.where(den == 0.0, 1.0, den)
    return np.max(np.abs(got - ref), axis=0) / den


def flops_per_query(width: int = 64, n_hidden: int = 5) -> int:
    return 2 * sum(o * i for o, i in layer_shapes(width, n_hidden))


if __name__ == "__main__":  # pragma: no cover
    print("oracle flops/query", flops_per_query(), "pi", math.pi)

"""Seeded synthetic inputs for the radiance-cache hot path.

Shared by the oracle-side tests and the GPU path alike, so it holds none of
the method's arithmetic: no encoding, no network, no loss, no optimiser.  It
only draws path-vertex records, training targets, initial weights and serving
traces from fixed distributions with NumPy's PCG64 generator (drawn in float64,
handed out as float32 exactly as both sides consume them).

Distributions (stand-ins for the path vertices a renderer would produce; the
paper's scenes are not available):

* position ~ U[0,1]^3
* scattered direction and surface normal ~ uniform on the unit sphere.  In the
  14-float record they are drawn directly in normalised spherical coordinates:
  the polar coordinate (in [0,1]) is the inverse-CDF sample arccos(1-2*xi)/pi,
  the azimuthal one is U[0,1] (the law of a uniform direction).  In the
  16-float record they are unit vectors (normalised Gaussian triples).
* roughness, diffuse albedo, specular albedo ~ U[0,1]
* training target, all three channels: exp(sin(3*x) + cos(2*y)) with x, y the
  first two position coordinates.
* weights: Glorot-uniform, bound sqrt(6 / (fan_in + fan_out)).
"""
from __future__ import annotations

import numpy as np

# Seeds of the standard synthetic workload.
SEED_WEIGHTS = 0
SEED_QUERIES = 1
SEED_RECORDS = 2
SEED_HELDOUT = 3
SEED_SERVE = 4
SEED_FD = 5

RAW14 = 0  # pos 3 | dir (u,w) 2 | normal (u,w) 2 | roughness 1 | diffuse 3 | specular 3
RAW16 = 1  # pos 3 | dir xyz 3 | normal xyz 3 | roughness 1 | diffuse 3 | specular 3
RAW_WIDTH = {RAW14: 14, RAW16: 16}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    norm = np.sqrt((g * g).sum(axis=1, keepdims=True))
    norm[norm == 0.0] = 1.0
    return g / norm


def raw_records(n: int, seed: int, layout: int = RAW14) -> np.ndarray:
    """`n` path-vertex records, float32 `[n][14]` (RAW14) or `[n][16]` (RAW16)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = _rng(seed)
    pos = rng.random((n, 3))
    if layout == RAW14:
        xi = rng.random((n, 4))
        d_u = np.arccos(np.clip(1.0 - 2.0 * xi[:, 0], -1.0, 1.0)) / np.pi
        n_u = np.arccos(np.clip(1.0 - 2.0 * xi[:, 2], -1.0, 1.0)) / np.pi
        dirs = np.stack([d_u, xi[:, 1]], axis=1)
        nrms = np.stack([n_u, xi[:, 3]], axis=1)
    elif layout == RAW16:
        dirs = _unit_vectors(rng, n)
        nrms = _unit_vectors(rng, n)
    else:
        raise ValueError(f"unknown raw layout {layout}")
    rough = rng.random((n, 1))
    diffuse = rng.random((n, 3))
    specular = rng.random((n, 3))
    out = np.concatenate([pos, dirs, nrms, rough, diffuse, specular], axis=1)
    return np.ascontiguousarray(out.astype(np.float32))


def targets(raw: np.ndarray) -> np.ndarray:
    """Positive synthetic radiance exp(sin 3x + cos 2y) on all three channels, float32 `[n][3]`."""
    x = raw[:, 0].astype(np.float64)
    y = raw[:, 1].astype(np.float64)
    t = np.exp(np.sin(3.0 * x) + np.cos(2.0 * y))
    return np.ascontiguousarray(np.repeat(t[:, None], 3, axis=1).astype(np.float32))


def layer_shapes(width: int = 64, n_hidden: int = 5, n_in: int = 64, n_out: int = 3):
    """(out, in) of every weight matrix: input layer, n_hidden-1 hidden->hidden, output."""
    shapes = [(width, n_in)]
    shapes += [(width, width)] * (n_hidden - 1)
    shapes.append((n_out, width))
    return shapes


def n_params(width: int = 64, n_hidden: int = 5, n_in: int = 64, n_out: int = 3) -> int:
    return sum(o * i for o, i in layer_shapes(width, n_hidden, n_in, n_out))


def glorot_weights(width: int = 64, n_hidden: int = 5, seed: int = SEED_WEIGHTS,
                   n_in: int = 64, n_out: int = 3) -> np.ndarray:
    """Flat float32 weights, matrices in layer order, each row-major [out][in]."""
    rng = _rng(seed)
    parts = []
    for o, i in layer_shapes(width, n_hidden, n_in, n_out):
        bound = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-bound, bound, size=(o, i)).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def split_weights(flat: np.ndarray, width: int = 64, n_hidden: int = 5,
                  n_in: int = 64, n_out: int = 3):
    """Views of a flat weight vector as the list of [out][in] matrices."""
    mats, off = [], 0
    for o, i in layer_shapes(width, n_hidden, n_in, n_out):
        mats.append(flat[off:off + o * i].reshape(o, i))
        off += o * i
    if off != flat.size:
        raise ValueError(f"weight vector has {flat.size} entries, expected {off}")
    return mats


def gaussian(shape, seed: int) -> np.ndarray:
    """Standard normal float32 array (upstream gradients for finite-difference checks)."""
    return np.ascontiguousarray(_rng(seed).standard_normal(shape).astype(np.float32))


def uniform_features(n: int, width: int, seed: int) -> np.ndarray:
    """U[0,1) float32 `[n][width]`: generic non-negative network inputs."""
    return np.ascontiguousarray(_rng(seed).random((n, width)).astype(np.float32))


def serve_trace(n_requests: int, n_caches: int = 8, p_infer: float = 0.6,
                n_min: float = 1e3, n_max: float = 2e6, n_train: int = 16384,
                rate_per_s: float = 1000.0, seed: int = SEED_SERVE):
    """Poisson arrival trace mixing inference and training requests.

    Returns a list of dicts (t_arrive seconds, kind 'infer'|'train', cache id, n).
    Inference sizes are log-uniform on [n_min, n_max].
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    kinds = rng.random(n_requests) < p_infer
    caches = rng.integers(0, n_caches, size=n_requests)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_requests))
    out = []
    for k in range(n_requests):
        if kinds[k]:
            out.append(dict(t_arrive=float(t[k]), kind="infer", cache=int(caches[k]),
                            n=int(round(sizes[k]))))
        else:
            out.append(dict(t_arrive=float(t[k]), kind="train", cache=int(caches[k]), n=n_train))
    return out


# Special values of the edge-case records: exact integers and halves, the
# ends of the unit interval, large magnitudes and values just inside them.
EDGE_POSITIONS = (0.0, 1.0, -1.0, 0.5, -0.5, 0.25, 2.0, -2.0, 3.0, -4.0, 4.0 - 2.0 ** -20,
                  1.0 - 2.0 ** -24, 2.0 ** -30, -(2.0 ** -30), 1000.0, -1000.0, 1000.375, -999.625)
EDGE_ANGLES = (0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0, 2.0 ** -24, 1.0 - 2.0 ** -24)
EDGE_ROUGHNESS = (0.0, 1e-7, 0.5, 1.0, 20.0, 1000.0)
EDGE_ALBEDO = (0.0, 0.5, 1.0)
# Unit vectors on the axes, with the signed zeros that pick atan2's branch at
# the poles and on the negative x axis.
EDGE_VECTORS = ((0.0, 0.0, 1.0), (0.0, 0.0, -1.0), (-0.0, 0.0, 1.0), (-0.0, -0.0, 1.0),
                (0.0, -0.0, -1.0), (1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (-1.0, -0.0, 0.0),
                (0.0, 1.0, 0.0), (0.0, -1.0, 0.0), (1.0, -0.0, 0.0))


def edge_records(n_random: int, seed: int, layout: int = RAW14) -> np.ndarray:
    """Records at the edges of each field's range, then `n_random` records with
    positions U[-4, 4) (a third of them U[-1000, 1000)), roughness U[0, 20) and
    the other fields as in `raw_records`.

    The special part cycles every field through its special values (positions,
    spherical angles or axis unit vectors, roughness, albedos) with different
    strides, so each value meets many values of the other fields.  Signed
    zeros of the unit vectors survive the cast to float32.
    """
    w = RAW_WIDTH[layout]
    n_special = 3 * len(EDGE_POSITIONS) * len(EDGE_ANGLES)
    sp = np.zeros((n_special, w), dtype=np.float64)
    i = np.arange(n_special)
    P, A, V = len(EDGE_POSITIONS), len(EDGE_ANGLES), len(EDGE_VECTORS)
    pos = np.asarray(EDGE_POSITIONS)
    for c in range(3):
        sp[:, c] = pos[(i + 5 * c) % P]
    if layout == RAW14:
        ang = np.asarray(EDGE_ANGLES)
        for a in range(4):
            sp[:, 3 + a] = ang[(i * (a + 1) + 3 * a) % A]
        rest = 7
    else:
        vec = np.asarray(EDGE_VECTORS)
        sp[:, 3:6] = vec[i % V]
        sp[:, 6:9] = vec[(3 * i + 4) % V]
        rest = 9
    sp[:, rest] = np.asarray(EDGE_ROUGHNESS)[i % len(EDGE_ROUGHNESS)]
    alb = np.asarray(EDGE_ALBEDO)
    for j in range(6):
        sp[:, rest + 1 + j] = alb[(i + j) % len(alb)]
    rnd = raw_records(n_random, seed, layout).astype(np.float64)
    rng = _rng(seed + 1)
    rnd[:, 0:3] = rng.uniform(-4.0, 4.0, size=(n_random, 3))
    big = rng.random(n_random) < 1.0 / 3.0
    rnd[big, 0:3] = rng.uniform(-1000.0, 1000.0, size=(int(big.sum()), 3))
    rnd[:, rest] = rng.uniform(0.0, 20.0, size=n_random)
    return np.ascontiguousarray(np.concatenate([sp, rnd], axis=0).astype(np.float32))

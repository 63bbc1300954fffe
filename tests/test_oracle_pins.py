"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an exact hand-derived fixture, a brute-force loop, finite
differences, an invariant, or an independent library routine.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

import synthdata as sd
from oracle import nrc_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Encodings
# ----------------------------------------------------------------------------
def test_freq_matches_libm_closed_form():
    # Sec. 3.6: sin of 2^d * pi * x.  libm's sin on the unreduced argument is an
    # independent evaluation of the same closed form.
    x = sd.uniform_features(200, 3, seed=11).astype(np.float64)
    paper = O.freq(x, O.PRESET_PAPER)
    conf = O.freq(x, O.PRESET_CONFIG)
    for i in range(x.shape[0]):
        for c in range(3):
            for d in range(12):
                want = math.sin(2.0 ** d * math.pi * x[i, c])
                assert abs(paper[i, 12 * c + d] - want) < 1e-11
            for d in range(6):
                arg = 2.0 ** d * math.pi * x[i, c]
                assert abs(conf[i, 12 * c + 2 * d] - math.sin(arg)) < 1e-12
                assert abs(conf[i, 12 * c + 2 * d + 1] - math.cos(arg)) < 1e-12


def test_freq_dyadic_points_exact():
    # x = 1/2: sin(2^d pi/2) = 1 for d = 0 and 0 otherwise; cos = 0, then -1, then 1.
    p = np.full((1, 3), 0.5)
    paper = O.freq(p, O.PRESET_PAPER)[0]
    want = np.array([1.0] + [0.0] * 11)
    for c in range(3):
        assert np.allclose(paper[12 * c:12 * c + 12], want, atol=1e-15)
    conf = O.freq(p, O.PRESET_CONFIG)[0]
    sin_want = [1, 0, 0, 0, 0, 0]
    cos_want = [0, -1, 1, 1, 1, 1]
    for d in range(6):
        assert abs(conf[2 * d] - sin_want[d]) < 1e-15
        assert abs(conf[2 * d + 1] - cos_want[d]) < 1e-15
    # x = 1/4: sin(pi/4) = sqrt(2)/2, sin(pi/2) = 1, then 0.
    q = O.freq(np.full((1, 3), 0.25), O.PRESET_PAPER)[0]
    assert abs(q[0] - math.sqrt(0.5)) < 1e-15 and abs(q[1] - 1.0) < 1e-15
    assert np.all(np.abs(q[2:12]) < 1e-15)


def test_quartic_kernel_normalised_and_cdf_is_its_integral():
    # Sec. 5 cheap primitives: quartic(x) = 15/16 (1 - x^2)^2 on [-1, 1].
    kern = lambda x: 15.0 / 16.0 * (1.0 - x * x) ** 2
    total, _ = integrate.quad(kern, -1.0, 1.0)
    assert abs(total - 1.0) < 1e-13
    for u in [-1.0, -0.73, -0.25, 0.0, 0.1, 0.5, 0.99, 1.0]:
        want, _ = integrate.quad(kern, -1.0, u)
        assert abs(O.quartic_cdf(np.array(u)) - want) < 1e-13
    assert O.quartic_cdf(np.array(-3.0)) == 0.0 and O.quartic_cdf(np.array(7.0)) == 1.0


def _read_golden_one_blob():
    rows = []
    with open(os.path.join(GOLDEN, "one_blob_quartic_dyadic.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([Fraction(tok) for tok in line.split()])
    return rows


def test_one_blob_exact_dyadic_fixture():
    rows = _read_golden_one_blob()
    assert len(rows) == 9
    s = np.array([float(r[0]) for r in rows])
    got = O.one_blob(s)
    for i, r in enumerate(rows):
        for j in range(4):
            assert got[i, j] == pytest.approx(float(r[1 + j]), abs=1e-15)
            # every fixture value survives FP16 unchanged
            assert float(np.float16(float(r[1 + j]))) == float(r[1 + j])


def test_one_blob_invariants():
    s = np.concatenate([np.linspace(0.0, 1.0, 1001), sd.uniform_features(500, 1, 12)[:, 0]])
    e = O.one_blob(s)
    assert np.allclose(e.sum(axis=1), 1.0, atol=1e-14)           # telescoping partition of unity
    assert np.all(e >= -1e-15)
    assert np.all((np.abs(e) > 1e-15).sum(axis=1) <= 3)           # blob spans two bin widths
    mirrored = O.one_blob(1.0 - s)[:, ::-1]
    assert np.allclose(e, mirrored, atol=1e-14)                   # mirror symmetry
    # the bin holding the blob centre always carries the largest mass
    c = 4 * s
    inner = (s > 0.01) & (s < 0.99) & (np.abs(c - np.round(c)) > 1e-9)   # no two-way ties
    assert np.all(np.argmax(e[inner], axis=1) == np.minimum((4 * s[inner]).astype(int), 3))


def test_one_blob_matches_numerical_bin_integrals():
    # Brute force: integrate the quartic blob over each bin numerically.
    kern = lambda x: 15.0 / 16.0 * (1.0 - x * x) ** 2 if abs(x) < 1.0 else 0.0
    for s in [0.03, 0.2, 0.41, 0.5, 0.77, 0.96]:
        c = 4 * s
        want = []
        for j in range(4):
            lo = -np.inf if j == 0 else j
            hi = np.inf if j == 3 else j + 1
            lo_c, hi_c = max(lo - c, -1.0), min(hi - c, 1.0)
            want.append(integrate.quad(kern, lo_c, hi_c)[0] if hi_c > lo_c else 0.0)
        assert np.allclose(O.one_blob(np.array([s]))[0], want, atol=1e-12)


def test_gauss_one_blob_matches_numerical_bin_integrals():
    # Brute force: integrate the standard normal density (one bin per unit of
    # standard deviation) over each bin; the edge bins take the tails.
    pdf = lambda x: math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    for s in [0.0, 0.03, 0.2, 0.41, 0.5, 0.77, 0.96, 1.0]:
        c = 4 * s
        want = []
        for j in range(4):
            lo = -np.inf if j == 0 else j - c
            hi = np.inf if j == 3 else j + 1 - c
            want.append(integrate.quad(pdf, lo, hi, epsabs=1e-14, epsrel=1e-13)[0])
        got = O.one_blob(np.array([s]), cdf=O.gauss_cdf)[0]
        assert np.allclose(got, want, atol=1e-12), (s, got, want)


def test_gauss_one_blob_invariants():
    s = np.concatenate([np.linspace(0.0, 1.0, 401), sd.uniform_features(200, 1, 13)[:, 0]])
    e = O.one_blob(s, cdf=O.gauss_cdf)
    assert np.allclose(e.sum(axis=1), 1.0, atol=1e-14)           # telescoping partition of unity
    assert np.all(e > 0.0)                                        # a Gaussian reaches every bin
    assert np.allclose(e, O.one_blob(1.0 - s, cdf=O.gauss_cdf)[:, ::-1], atol=1e-14)   # mirror symmetry
    # the centre bin's mass: at s = 1/8 (centre of bin 0, half a bin from its
    # inner edge) it is Phi(1/2) of the whole tail-absorbing edge bin
    assert np.isclose(O.one_blob(np.array([0.125]), cdf=O.gauss_cdf)[0, 0], O.gauss_cdf(np.array(0.5)), atol=1e-15)


def test_encode_paper_gauss_preset_layout():
    raw = sd.raw_records(64, 91)
    a = O.encode(raw, preset=O.PRESET_PAPER)
    b = O.encode(raw, preset=O.PRESET_PAPER_GAUSS)
    r = raw.astype(np.float64)
    assert np.array_equal(a[:, :36], b[:, :36])                   # the same 12 sines per coordinate
    assert np.array_equal(a[:, 56:], b[:, 56:])                   # albedos and the padding of ones
    # dir (2 x 4 bins), normal (2 x 4), 1 - exp(-roughness) (4): Gaussian blobs
    for k, v in enumerate([r[:, 3], r[:, 4], r[:, 5], r[:, 6], 1.0 - np.exp(-r[:, 7])]):
        assert np.allclose(b[:, 36 + 4 * k:40 + 4 * k], O.one_blob(v, cdf=O.gauss_cdf), atol=1e-15)
    assert not np.allclose(a[:, 36:56], b[:, 36:56])


def test_sph_axes():
    v = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0], [0, -1, 0], [-1, 0, 1e-300]], dtype=np.float64)
    v[5] /= np.linalg.norm(v[5])
    got = O.sph(v)
    want = np.array([[0.0, 0.5], [1.0, 0.5], [0.5, 0.5], [0.5, 0.75], [0.5, 0.25], [0.5, 1.0]])
    assert np.allclose(got, want, atol=1e-15)
    # ranges on random unit vectors
    u = O.sph(sd.raw_records(1000, 7, sd.RAW16)[:, 3:6].astype(np.float64))
    assert np.all((u >= 0) & (u <= 1))


def test_sph_inverts_spherical_parametrisation():
    # Build unit vectors from known angles and recover them.
    rng = np.random.Generator(np.random.PCG64(21))
    th = rng.uniform(0.01, np.pi - 0.01, 300)
    ph = rng.uniform(-np.pi + 0.01, np.pi - 0.01, 300)
    v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    got = O.sph(v)
    assert np.allclose(got[:, 0], th / np.pi, atol=1e-13)
    assert np.allclose(got[:, 1], (ph + np.pi) / (2 * np.pi), atol=1e-13)


def test_encode_layout_config_preset():
    raw = sd.raw_records(64, 8)
    enc = O.encode(raw)
    assert enc.shape == (64, 64)
    r = raw.astype(np.float64)
    # position -> 36 frequency features (coordinate-major)
    for c in range(3):
        for d in range(6):
            assert np.allclose(enc[:, 12 * c + 2 * d], np.sin(2 ** d * np.pi * r[:, c]), atol=1e-12)
    # one-blob groups sum to one
    for g in range(4):
        assert np.allclose(enc[:, 36 + 4 * g:40 + 4 * g].sum(axis=1), 1.0, atol=1e-14)
    assert np.array_equal(enc[:, 52], r[:, 7])                 # roughness as is
    assert np.array_equal(enc[:, 53:56], r[:, 8:11])           # diffuse albedo, identity
    assert np.array_equal(enc[:, 56:59], r[:, 11:14])          # specular albedo, identity
    assert np.all(enc[:, 59:] == 0.0)                          # zero pad


def test_encode_layout_paper_preset():
    raw = sd.raw_records(64, 9)
    enc = O.encode(raw, preset=O.PRESET_PAPER)
    r = raw.astype(np.float64)
    for c in range(3):
        for d in range(12):
            assert np.allclose(enc[:, 12 * c + d], np.sin(2 ** d * np.pi * r[:, c]), atol=1e-11)
    # roughness enters as one-blob of 1 - exp(-r): its centre of mass tracks that value
    ob = enc[:, 52:56]
    assert np.allclose(ob.sum(axis=1), 1.0, atol=1e-14)
    assert np.array_equal(enc[:, 56:59], r[:, 8:11])
    assert np.array_equal(enc[:, 59:62], r[:, 11:14])
    assert np.all(enc[:, 62:] == 1.0)                          # pad with one (implicit bias)


def test_encode_raw16_equals_raw14_of_same_angles():
    raw16 = sd.raw_records(128, 10, sd.RAW16).astype(np.float64)
    # independent spherical coordinates via complex angles
    def angles(v):
        th = np.arccos(np.clip(v[:, 2], -1, 1)) / np.pi
        ph = np.angle(v[:, 0] + 1j * v[:, 1]) / (2 * np.pi) + 0.5
        return np.stack([th, ph], axis=1)
    raw14 = np.concatenate([raw16[:, 0:3], angles(raw16[:, 3:6]), angles(raw16[:, 6:9]), raw16[:, 9:16]], axis=1)
    assert np.allclose(O.encode(raw16, O.RAW16), O.encode(raw14, O.RAW14), atol=1e-12)


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------
def _brute_mlp(mats, x):
    """Scalar-loop evaluation of the bias-free ReLU network."""
    out = []
    for row in x:
        h = [float(v) for v in row]
        for l, w in enumerate(mats):
            z = [sum(float(w[o][i]) * h[i] for i in range(len(h))) for o in range(len(w))]
            h = z if l == len(mats) - 1 else [max(0.0, v) for v in z]
        out.append(h)
    return np.array(out)


def test_forward_brute_force_tiny():
    rng = np.random.Generator(np.random.PCG64(31))
    shapes = [(4, 5), (4, 4), (4, 4), (3, 4)]
    mats = [rng.standard_normal(s) for s in shapes]
    x = rng.standard_normal((8, 5))
    y, hs = O.forward(mats, x)
    assert np.allclose(y, _brute_mlp(mats, x), atol=1e-13)
    assert len(hs) == 4 and np.array_equal(hs[0], x)


def test_forward_linear_special_case():
    # Non-negative inputs and weights keep every ReLU in its identity branch, so
    # the network is the plain matrix product W_5 ... W_0 x.
    rng = np.random.Generator(np.random.PCG64(32))
    mats = [np.abs(rng.standard_normal(s)) for s in sd.layer_shapes()]
    x = rng.random((16, 64))
    chain = np.eye(64)
    for w in mats:
        chain = w @ chain
    assert np.allclose(O.forward(mats, x)[0], x @ chain.T, rtol=1e-12)


def test_forward_homogeneous_and_zero():
    w = sd.split_weights(sd.glorot_weights().astype(np.float64))
    x = O.encode(sd.raw_records(32, 4))
    y1 = O.forward(w, x)[0]
    assert np.array_equal(O.forward(w, 2.0 * x)[0], 2.0 * y1)    # positive homogeneity, exact
    assert np.all(O.forward(w, np.zeros_like(x))[0] == 0.0)
    assert np.all(O.forward([np.zeros_like(m) for m in w], x)[0] == 0.0)


# ----------------------------------------------------------------------------
# Loss (Eq. 5)
# ----------------------------------------------------------------------------
def test_loss_zero_at_target():
    y = sd.targets(sd.raw_records(10, 1)).astype(np.float64)
    loss, g = O.relative_l2(y, y)
    assert loss == 0.0 and np.all(g == 0.0)


def test_loss_single_sample_by_hand():
    # y_hat = (1, 2, 3), y = 0: luminance 2, denominator 4.01.
    loss, g = O.relative_l2(np.array([[1.0, 2.0, 3.0]]), np.zeros((1, 3)))
    assert loss == pytest.approx(14.0 / 4.01 / 3.0, rel=1e-15)
    assert np.allclose(g, np.array([[2.0, 4.0, 6.0]]) / 4.01 / 3.0, rtol=1e-15)


def test_loss_gradient_is_stop_gradient_derivative():
    rng = np.random.Generator(np.random.PCG64(33))
    yh = rng.random((5, 3)) * 4
    y = rng.random((5, 3)) * 4
    _, g = O.relative_l2(yh, y)
    den = yh.mean(axis=1, keepdims=True) ** 2 + 0.01           # frozen at the prediction
    h = 1e-4
    for i in range(5):
        for c in range(3):
            p, m = yh.copy(), yh.copy()
            p[i, c] += h
            m[i, c] -= h
            fd = (((p - y) ** 2 / den).sum() - ((m - y) ** 2 / den).sum()) / (2 * h) / 15
            assert g[i, c] == pytest.approx(fd, rel=1e-9, abs=1e-12)


# ----------------------------------------------------------------------------
# Backward: finite differences and torch autograd
# ----------------------------------------------------------------------------
def _frozen_loss(mats, x, y, den):
    yh = O.forward(mats, x)[0]
    return float(((yh - y) ** 2 / den).sum() / (3 * x.shape[0]))


def test_backward_central_differences_weights_and_inputs():
    rng = np.random.Generator(np.random.PCG64(34))
    shapes = [(8, 6), (8, 8), (8, 8), (3, 8)]
    mats = [rng.standard_normal(s) * 0.7 for s in shapes]
    x = rng.standard_normal((12, 6))
    y = rng.random((12, 3)) * 3
    yh, hs = O.forward(mats, x)
    _, d_out = O.relative_l2(yh, y)
    grads, g_in = O.backward(mats, hs, d_out)
    den = yh.mean(axis=1, keepdims=True) ** 2 + 0.01
    h = 1e-3

    def masks(ms, xx):
        return [hh > 0 for hh in O.forward(ms, xx)[1][1:]]

    base = masks(mats, x)
    checked = 0
    for l, w in enumerate(mats):
        for idx in np.ndindex(*w.shape):
            p = [m.copy() for m in mats]
            m_ = [m.copy() for m in mats]
            p[l][idx] += h
            m_[l][idx] -= h
            if any((a != b).any() for a, b in zip(masks(p, x), base)) or \
               any((a != b).any() for a, b in zip(masks(m_, x), base)):
                continue  # a ReLU kink lies inside [-h, h]
            fd = (_frozen_loss(p, x, y, den) - _frozen_loss(m_, x, y, den)) / (2 * h)
            assert grads[l][idx] == pytest.approx(fd, rel=1e-7, abs=1e-10)
            checked += 1
    assert checked >= 150
    for idx in np.ndindex(*x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        if any((a != b).any() for a, b in zip(masks(mats, xp), base)) or \
           any((a != b).any() for a, b in zip(masks(mats, xm), base)):
            continue
        fd = (_frozen_loss(mats, xp, y, den) - _frozen_loss(mats, xm, y, den)) / (2 * h)
        assert g_in[idx] == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_backward_matches_torch_autograd_fp64():
    torch = pytest.importorskip("torch")
    w = sd.split_weights(sd.glorot_weights().astype(np.float64))
    raw = sd.raw_records(256, 2)
    x = O.encode(raw)
    y = sd.targets(raw).astype(np.float64)
    yh, hs = O.forward(w, x)
    loss, d_out = O.relative_l2(yh, y)
    grads, g_in = O.backward(w, hs, d_out)

    tw = [torch.tensor(m, dtype=torch.float64, requires_grad=True) for m in w]
    tx = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    h = tx
    for l, m in enumerate(tw):
        h = h @ m.T
        if l < len(tw) - 1:
            h = torch.relu(h)
    lum = h.mean(dim=1, keepdim=True).detach()
    tl = ((h - torch.tensor(y)) ** 2 / (lum ** 2 + 0.01)).mean()
    tl.backward()
    assert tl.item() == pytest.approx(loss, rel=1e-13)
    for a, b in zip(grads, tw):
        assert np.allclose(a, b.grad.numpy(), rtol=1e-11, atol=1e-16)
    assert np.allclose(g_in, tx.grad.numpy(), rtol=1e-11, atol=1e-16)


# ----------------------------------------------------------------------------
# Adam
# ----------------------------------------------------------------------------
def test_adam_constant_gradient_closed_form():
    # With a constant gradient the bias-corrected moments are g and g^2 exactly,
    # so every step moves by -lr * g / (|g| + eps).
    cfg = O.AdamConfig()
    g = np.array([3.0, -0.5, 1e-3, 0.0, -7e-9])
    w = np.zeros_like(g)
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    t = 0
    for k in range(1, 6):
        w_prev = w
        w, m, v, t = O.adam(w, m, v, t, g, cfg)
        assert t == k
        assert np.allclose(w - w_prev, -cfg.lr * g / (np.abs(g) + cfg.eps), rtol=1e-12, atol=1e-18)


def test_adam_matches_torch_optim_fp64():
    torch = pytest.importorskip("torch")
    cfg = O.AdamConfig()
    rng = np.random.Generator(np.random.PCG64(35))
    w0 = rng.standard_normal(50)
    p = torch.tensor(w0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=cfg.lr, betas=(cfg.beta1, cfg.beta2), eps=cfg.eps)
    w, m, v, t = w0.copy(), np.zeros(50), np.zeros(50), 0
    for _ in range(6):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g)
        opt.step()
        w, m, v, t = O.adam(w, m, v, t, g, cfg)
        assert np.allclose(w, p.detach().numpy(), rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------------------------
# Training step and frame
# ----------------------------------------------------------------------------
def test_train_step_gradient_matches_finite_differences_of_state():
    st = O.CacheState(sd.glorot_weights(width=8, n_hidden=2), width=8, n_hidden=2)
    raw = sd.raw_records(16, 3)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    loss, g = O.gradient(st, x, y)
    den = O.predict(st, x).mean(axis=1, keepdims=True) ** 2 + 0.01
    h = 1e-3
    rng = np.random.Generator(np.random.PCG64(36))
    ok = 0
    for k in rng.choice(g.size, 60, replace=False):
        a = O.CacheState(st.w.copy(), width=8, n_hidden=2)
        b = O.CacheState(st.w.copy(), width=8, n_hidden=2)
        a.w[k] += h
        b.w[k] -= h
        ha = [hh > 0 for hh in O.forward(a.mats(), x)[1][1:]]
        hb = [hh > 0 for hh in O.forward(b.mats(), x)[1][1:]]
        if any((p != q).any() for p, q in zip(ha, hb)):
            continue
        fd = (_frozen_loss(a.mats(), x, y, den) - _frozen_loss(b.mats(), x, y, den)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-7, abs=1e-10)
        ok += 1
    assert ok > 30


@pytest.mark.filterwarnings("ignore:invalid value encountered:RuntimeWarning")
def test_train_step_skips_non_finite_gradient():
    st = O.CacheState(sd.glorot_weights())
    raw = sd.raw_records(32, 3)
    x = O.encode(raw)
    y = sd.targets(raw).astype(np.float64)
    y[3, 1] = np.inf
    w0 = st.w.copy()
    _, skipped = O.train_step(st, x, y)
    assert skipped and st.t == 0 and np.array_equal(st.w, w0)


def test_training_reduces_loss():
    st = O.CacheState(sd.glorot_weights())
    raw = sd.raw_records(4096, 2)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    losses = [O.train_step(st, x[:1024], y[:1024])[0] for _ in range(8)]
    assert losses[-1] < 0.1 * losses[0]


def test_frame_queries_use_start_of_frame_weights_and_disjoint_batches():
    st = O.CacheState(sd.glorot_weights())
    q = O.encode(sd.raw_records(64, 1))
    raw = sd.raw_records(1024, 2)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    before = O.predict(st, q)
    rgb, losses = O.frame(st, q, x, y)
    assert np.array_equal(rgb, before) and len(losses) == 4 and st.t == 4
    # shuffling records inside a quarter changes nothing but rounding; across quarters it does
    st_a = O.CacheState(sd.glorot_weights())
    perm = np.concatenate([np.random.Generator(np.random.PCG64(37)).permutation(256) + 256 * k for k in range(4)])
    O.frame(st_a, q, x[perm], y[perm])
    assert np.allclose(st_a.w, st.w, rtol=1e-9, atol=1e-12)
    st_b = O.CacheState(sd.glorot_weights())
    swap = np.arange(1024)
    swap[[0, 1023]] = swap[[1023, 0]]
    O.frame(st_b, q, x[swap], y[swap])
    assert not np.allclose(st_b.w, st.w, rtol=1e-9, atol=1e-12)


# ----------------------------------------------------------------------------
# EMA of the weights (Eq. 2)
# ----------------------------------------------------------------------------
def test_ema_matches_explicit_weighted_average():
    # Closed form of the bias-corrected average of W_1..W_t with weights
    # (1 - a) a^(t-i), normalised by their sum 1 - a^t.
    a = 0.99
    rng = np.random.Generator(np.random.PCG64(41))
    ws = [rng.standard_normal(7) for _ in range(12)]
    w_bar = np.zeros(7)
    for t in range(1, 13):
        w_bar = O.ema_step(w_bar, ws[t - 1], t, a)
        coef = np.array([(1 - a) * a ** (t - i) for i in range(1, t + 1)])
        want = (coef[:, None] * np.array(ws[:t])).sum(axis=0) / coef.sum()
        assert np.allclose(w_bar, want, rtol=1e-12, atol=1e-14)
        assert coef.sum() == pytest.approx(1 - a ** t, rel=1e-12)


def test_ema_first_step_and_constant_weights():
    w = np.array([0.3, -2.0, 5.0])
    assert np.allclose(O.ema_step(np.zeros(3), w, 1, 0.99), w, rtol=1e-14)
    w_bar = np.zeros(3)
    for t in range(1, 50):
        w_bar = O.ema_step(w_bar, w, t, 0.99)
        assert np.allclose(w_bar, w, rtol=1e-12)


def test_ema_does_not_feed_back_into_training():
    raw = sd.raw_records(2048, 3)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    plain = O.CacheState(sd.glorot_weights())
    ema = O.CacheState(sd.glorot_weights(), ema_alpha=0.99)
    for k in range(3):
        O.train_step(plain, x[k * 512:(k + 1) * 512], y[k * 512:(k + 1) * 512])
        O.train_step(ema, x[k * 512:(k + 1) * 512], y[k * 512:(k + 1) * 512])
    assert np.array_equal(plain.w, ema.w)
    assert not np.allclose(ema.w_bar, ema.w)
    assert np.allclose(O.predict_ema(plain, x[:8]), O.predict(plain, x[:8]))


# ----------------------------------------------------------------------------
# Triangle wave (Sec. 5, cheap primitives)
# ----------------------------------------------------------------------------
def test_triangle_wave_closed_form():
    # The triangle wave printed in Sec. 5 (figure "cheap_primitives"),
    # tri(x) = 2|x mod 2 - 1| - 1: period 2, tri(0) = 1, tri(1/2) = 0,
    # tri(1) = -1, tri(3/2) = 0, slope -2 on [0, 1] and +2 on [1, 2].
    x = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, -0.5, -1.0, 7.0, 7.5, 8.0])
    want = np.array([1.0, 0.5, 0.0, -0.5, -1.0, -0.5, 0.0, 0.5, 1.0, 0.0, 0.0, -1.0, -1.0, 0.0, 1.0])
    assert np.array_equal(O.tri(x), want)
    t = np.linspace(0.0, 1.0, 101)
    assert np.allclose(O.tri(t), 1.0 - 2.0 * t, atol=1e-14)          # falling edge
    assert np.allclose(O.tri(t + 1.0), -1.0 + 2.0 * t, atol=1e-14)    # rising edge
    # period 2 and even symmetry, at points where both sides are exact
    y = np.arange(-4096, 4096) / 256.0
    assert np.array_equal(O.tri(y + 2.0), O.tri(y))
    assert np.array_equal(O.tri(-y), O.tri(y))
    # range [-1, 1], zero mean over a period
    assert O.tri(y).min() == -1.0 and O.tri(y).max() == 1.0
    assert abs(np.mean(O.tri(np.arange(512) / 256.0))) < 1e-15
    # it meets cos(pi x) at every multiple of 1/2 and has its sign everywhere,
    # lying inside it in magnitude (a cosine half-wave lies above its chords)
    h = np.arange(-8, 9) * 0.5
    assert np.allclose(O.tri(h), np.round(np.cos(np.pi * h), 12), atol=1e-15)
    z = np.linspace(-3.0, 3.0, 6001)
    c = np.round(np.cos(np.pi * z), 12)
    assert np.array_equal(np.sign(np.round(O.tri(z), 12)), np.sign(c))
    assert np.all(np.abs(O.tri(z)) <= np.abs(c) + 1e-12)


def test_encode_paper_tri_preset_layout():
    raw = sd.raw_records(64, 90)
    a = O.encode(raw, preset=O.PRESET_PAPER)
    b = O.encode(raw, preset=O.PRESET_PAPER_TRI)
    r = raw.astype(np.float64)
    for c in range(3):
        for d in range(12):
            x = 2 ** d * r[:, c]
            # with k = floor(x): falling edge 1 - 2 (x - k) for even k, rising
            # edge -1 + 2 (x - k) for odd k
            k = np.floor(x)
            frac = x - k                               # in [0, 1)
            want = np.where(np.mod(k, 2) == 0, 1.0 - 2.0 * frac, -1.0 + 2.0 * frac)
            assert np.allclose(b[:, 12 * c + d], want, atol=1e-12)
    assert np.array_equal(a[:, 36:], b[:, 36:])          # everything after the position is shared


# ----------------------------------------------------------------------------
# Reflectance factorisation (Sec. 5): prediction = network output * (alpha + beta)
# ----------------------------------------------------------------------------
def _small_state(factorize, preset=O.PRESET_CONFIG, seed=0):
    return O.CacheState(sd.glorot_weights(width=8, n_hidden=2, seed=seed), width=8, n_hidden=2,
                        factorize=factorize, preset=preset)


def test_factorised_prediction_scales_by_raw_albedos():
    # The factor comes from the raw record's diffuse (fields 8..10) and specular
    # (11..13) albedo, whichever columns the preset puts them in.
    raw = sd.raw_records(64, 91)
    r = raw[:, 8:11].astype(np.float64) + raw[:, 11:14].astype(np.float64)
    for preset in (O.PRESET_CONFIG, O.PRESET_PAPER, O.PRESET_PAPER_TRI):
        x = O.encode(raw, preset=preset)
        plain = O.predict(_small_state(False, preset), x)
        fact = O.predict(_small_state(True, preset), x)
        assert np.allclose(fact, plain * r, rtol=1e-14, atol=0)
        assert np.array_equal(O.reflectance(x, preset), r)


def test_factorisation_with_unit_reflectance_is_the_identity():
    raw = sd.raw_records(32, 92).copy()
    raw[:, 8:11] = 0.25
    raw[:, 11:14] = 0.75
    x = O.encode(raw)
    y = sd.targets(raw).astype(np.float64)
    assert np.array_equal(O.predict(_small_state(True), x), O.predict(_small_state(False), x))
    la, ga = O.gradient(_small_state(True), x, y)
    lb, gb = O.gradient(_small_state(False), x, y)
    assert la == lb and np.array_equal(ga, gb)


def _masks(st, x):
    return [hh > 0 for hh in O.forward(st.mats(), x)[1][1:]]


def test_factorised_query_gradient_central_differences():
    # L = sum G * y_hat.  Along any one weight or input coordinate (ReLU masks
    # fixed) y_hat = f R is at most quadratic, so central differences are exact
    # up to rounding, albedo columns included.
    raw = sd.raw_records(12, 93)
    x = O.encode(raw)
    g_out = np.random.Generator(np.random.PCG64(94)).standard_normal((12, 3))
    st = _small_state(True)
    gw, gx = O.query_gradient(st, x, g_out)
    h = 1e-3
    base = _masks(st, x)

    def lossf(s, xx):
        return float((g_out * O.predict(s, xx)).sum())

    rng = np.random.Generator(np.random.PCG64(95))
    ok = 0
    for k in rng.choice(gw.size, 80, replace=False):
        a, b = _small_state(True), _small_state(True)
        a.w[k] += h
        b.w[k] -= h
        if any((p != q).any() for p, q in zip(_masks(a, x), base)) or \
           any((p != q).any() for p, q in zip(_masks(b, x), base)):
            continue
        assert gw[k] == pytest.approx((lossf(a, x) - lossf(b, x)) / (2 * h), rel=1e-7, abs=1e-10)
        ok += 1
    assert ok > 40
    cols = list(range(36, 64))   # one-blob, roughness, both albedos, padding
    ok = 0
    for i in range(12):
        for j in cols:
            xp, xm = x.copy(), x.copy()
            xp[i, j] += h
            xm[i, j] -= h
            if any((p != q).any() for p, q in zip(_masks(st, xp), base)) or \
               any((p != q).any() for p, q in zip(_masks(st, xm), base)):
                continue
            fd = (lossf(st, xp) - lossf(st, xm)) / (2 * h)
            assert gx[i, j] == pytest.approx(fd, rel=1e-7, abs=1e-10)
            ok += 1
    assert ok > 200


def test_factorised_train_gradient_central_differences():
    # Eq. 5 on the factorised prediction, denominator held at its unperturbed value.
    raw = sd.raw_records(16, 96)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    st = _small_state(True)
    loss, g = O.gradient(st, x, y)
    yh = O.predict(st, x)
    den = yh.mean(axis=1, keepdims=True) ** 2 + 0.01
    assert loss == pytest.approx(float(((yh - y) ** 2 / den).mean()), rel=1e-13)
    h = 1e-3
    base = _masks(st, x)

    def frozen(s):
        return float(((O.predict(s, x) - y) ** 2 / den).sum() / (3 * x.shape[0]))

    rng = np.random.Generator(np.random.PCG64(97))
    ok = 0
    for k in rng.choice(g.size, 60, replace=False):
        a, b = _small_state(True), _small_state(True)
        a.w[k] += h
        b.w[k] -= h
        if any((p != q).any() for p, q in zip(_masks(a, x), base)) or \
           any((p != q).any() for p, q in zip(_masks(b, x), base)):
            continue
        assert g[k] == pytest.approx((frozen(a) - frozen(b)) / (2 * h), rel=1e-7, abs=1e-10)
        ok += 1
    assert ok > 30


# ----------------------------------------------------------------------------
# Training-record shuffle (Sec. 3.5) and self-training targets (Sec. 3.2)
# ----------------------------------------------------------------------------
def _golden_lcg():
    rows = {}
    for line in open(os.path.join(GOLDEN, "lcg_orbit_m16.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *v = line.split()
            rows[k] = [int(t) for t in v]
    return rows


def test_lcg_orbit_matches_hand_derived_fixture():
    g = _golden_lcg()
    assert O.lcg_permutation(16, 0).tolist() == g["orbit"]
    assert O.lcg_permutation(10, 0).tolist() == g["n10"]
    assert O.lcg_permutation(10, 7).tolist() == g["n10s7"]
    assert O.lcg_permutation(10, 7 + 16).tolist() == g["n10s7"]     # the seed acts mod m


def test_lcg_full_period_and_permutation():
    # Hull-Dobell: c odd and a = 1 (mod 4) give the full period 2^k, so every
    # orbit is a permutation; skipping values >= n keeps one of [0, n).
    assert O.LCG_C % 2 == 1 and O.LCG_A % 4 == 1
    for k in range(0, 17):
        m = 2 ** k
        assert np.array_equal(np.sort(O.lcg_permutation(m, 12345)), np.arange(m))
    rng = np.random.Generator(np.random.PCG64(98))
    for n in [1, 2, 3, 5, 1000, 16385, 50000]:
        p = O.lcg_permutation(n, int(rng.integers(0, 2 ** 32)))
        assert p.size == n and np.array_equal(np.sort(p), np.arange(n))
    assert O.lcg_permutation(0, 5).size == 0


def test_frame_batches_are_disjoint_and_spread_over_the_records():
    n, steps, batch = 65536, 4, 16384
    bs = O.frame_batches(n, steps, batch, 2)
    assert [b.size for b in bs] == [batch] * steps
    allb = np.concatenate(bs)
    assert np.array_equal(np.sort(allb), np.arange(n))               # disjoint, cover all
    # not correlated with record position (image region): every batch draws
    # within 10% of its share from each sixteenth of the record range
    for b in bs:
        h = np.bincount(b // (n // 16), minlength=16)
        assert np.max(np.abs(h - batch / 16)) <= 0.1 * batch / 16
    # more records than s l: the first s l shuffled ones are used
    bs = O.frame_batches(70000, steps, batch, 2)
    assert [b.size for b in bs] == [batch] * steps
    assert np.array_equal(np.concatenate(bs), O.lcg_permutation(70000, 2)[:steps * batch])
    # fewer: near-equal batches of all of them
    bs = O.frame_batches(1001, steps, batch, 2)
    assert [b.size for b in bs] == [250, 250, 250, 251]
    assert np.array_equal(np.sort(np.concatenate(bs)), np.arange(1001))


def test_frame_shuffled_equals_frame_on_permuted_records():
    st_a = O.CacheState(sd.glorot_weights())
    st_b = O.CacheState(sd.glorot_weights())
    raw = sd.raw_records(4 * 256, 99)
    x, y = O.encode(raw), sd.targets(raw).astype(np.float64)
    q = O.encode(sd.raw_records(64, 100))
    rgb_a, la, sa = O.frame_shuffled(st_a, q, x, y, steps=4, batch=256, seed=9)
    p = O.lcg_permutation(x.shape[0], 9)
    rgb_b, lb = O.frame(st_b, q, x[p], y[p], n_steps=4)
    assert np.array_equal(rgb_a, rgb_b) and la == lb and not any(sa)
    assert np.array_equal(st_a.w, st_b.w)


def test_self_training_targets():
    rng = np.random.Generator(np.random.PCG64(101))
    L = rng.random((50, 3))
    T = rng.random((50, 3))
    tail = rng.random((7, 3))
    k = rng.integers(0, 7, 50)
    got = O.self_training_targets(L, T, tail, k)
    assert np.array_equal(O.self_training_targets(L, np.zeros_like(T), tail, k), L)   # no tail term
    assert np.array_equal(O.self_training_targets(np.zeros_like(L), np.ones_like(T), tail, k), tail[k])
    for i in range(50):                                                           # record by record
        for c in range(3):
            assert got[i, c] == L[i, c] + T[i, c] * tail[k[i], c]


# ----------------------------------------------------------------------------
# Positions anywhere in R^3 (Table "parameters": the position is a point of the
# scene, not a unit-cube coordinate)
# ----------------------------------------------------------------------------
def test_freq_far_from_the_unit_cube():
    # Beyond [0,1) the exact mod-2 reduction must still give sin/cos(2^d pi p):
    # checked against libm on the unreduced FP64 argument, whose rounding at
    # |2^d pi p| < 2^24 is below 1e-8.
    raw = sd.edge_records(2000, 31)
    p = raw[:, 0:3].astype(np.float64)
    f = O.freq(p, O.PRESET_CONFIG).reshape(-1, 3, 6, 2)
    for d in range(6):
        a = np.pi * 2.0 ** d * p
        assert np.max(np.abs(f[:, :, d, 0] - np.sin(a))) < 1e-8
        assert np.max(np.abs(f[:, :, d, 1] - np.cos(a))) < 1e-8
    g = O.freq(p, O.PRESET_PAPER).reshape(-1, 3, 12)
    for d in range(12):
        assert np.max(np.abs(g[:, :, d] - np.sin(np.pi * 2.0 ** d * p))) < 1e-8
    # the triangle wave is even and 2-periodic, so -p and p + 2 give the same
    # features as p, exactly
    t = O.freq(p, O.PRESET_PAPER_TRI)
    assert np.array_equal(O.freq(-p, O.PRESET_PAPER_TRI), t)
    assert np.array_equal(O.freq(p + 2.0, O.PRESET_PAPER_TRI), t)
    assert np.all(np.abs(t) <= 1.0)


def test_encode_edge_records_invariants():
    # Poles, signed zeros, bin edges, roughness 0 and 20: every one-blob group
    # sums to one, every value is in range, nothing is non-finite, and the
    # roughness one-blob takes its end values.
    for layout in (O.RAW14, O.RAW16):
        raw = sd.edge_records(500, 32, layout)
        for preset in (O.PRESET_CONFIG, O.PRESET_PAPER, O.PRESET_PAPER_TRI, O.PRESET_PAPER_GAUSS):
            e = O.encode(raw, layout, preset)
            assert np.all(np.isfinite(e))
            ob = e[:, 36:56 if preset != O.PRESET_CONFIG else 52].reshape(len(e), -1, 4)
            assert np.allclose(ob.sum(axis=2), 1.0, atol=1e-14)
            assert np.all(ob >= -1e-15) and np.all(ob <= 1.0 + 1e-15)
            assert np.all(np.abs(e[:, :36]) <= 1.0 + 1e-15)
        if layout == O.RAW16:
            # at the poles the polar angle is 0 or 1 exactly, so one-blob gives a unit vector
            s = O.sph(raw[:, 3:6])
            pole = raw[:, 5] == 1.0
            assert np.all(s[pole, 0] == 0.0)
            assert np.array_equal(O.one_blob(s[pole, 0]), np.tile([1.0, 0, 0, 0], (int(pole.sum()), 1)))
            # atan2's signed-zero branches (IEEE 754 / C99): the azimuth of
            # (-1, +0, 0) is 1, of (-1, -0, 0) is 0, of (+0, +0, 1) is 1/2 and of
            # (-0, -0, 1) is 0
            v = np.array([[-1.0, 0.0, 0.0], [-1.0, -0.0, 0.0], [0.0, 0.0, 1.0], [-0.0, -0.0, 1.0]])
            assert np.array_equal(O.sph(v)[:, 1], [1.0, 0.0, 0.5, 0.0])
    raw = sd.edge_records(0, 33, O.RAW14)
    e = O.encode(raw, O.RAW14, O.PRESET_PAPER)
    r = raw[:, 7]
    assert np.array_equal(e[r == 0.0, 52:56], np.tile([1.0, 0, 0, 0], (int((r == 0.0).sum()), 1)))
    assert np.allclose(e[r >= 20.0, 52:56], [0.0, 0.0, 0.0, 1.0], atol=1e-15)

"""Parity of the HIP path with the FP64 oracle, element by element, through the C ABI.

Tolerances (derived in the design notes):
* encode: FP32 output 2e-6 absolute (libm-grade sinpi/cospi, acos, atan2 in
  FP32); FP16/BF16 output additionally one rounding of the stored value
  (relative 2^-11 / 2^-8).
* forward, FP32: 1e-5 normwise per channel (max |err| / max |ref|).
* forward, FP16: 1e-2 normwise per channel.  BF16 on untrained Glorot weights:
  3e-2 (rounding 2^-8 per operand over six layers); 1e-2 after training.
* training, FP32: trained outputs 1e-5, loss 1e-5 relative; FP16/BF16: trained
  outputs 1e-2 (BF16 2e-2 for a single step from Glorot weights), loss 1%.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd
from oracle import nrc_oracle as O

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp16", "bf16"]
ENC_REL = {"fp32": 0.0, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
FWD_TOL = {"fp32": 1e-5, "fp16": 1e-2, "bf16": 3e-2}


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12372_amd.nrc as nrc
    return nrc


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def make_cache(N, prec, width=64, n_hidden=5, preset=0, weights=None, **kw):
    cfg = N.make_config(width=width, n_hidden=n_hidden, precision=prec, enc_preset=preset, **kw)
    c = N.Cache(cfg)
    w = sd.glorot_weights(width, n_hidden) if weights is None else weights
    c.set_weights(w)
    return c, w


def rounded_input(x, prec):
    """Device tensor at the cache precision and the exact values it holds (float64)."""
    t = dev(x, {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[prec])
    return t, t.float().cpu().numpy().astype(np.float64)


def state_of(w, width=64, n_hidden=5):
    return O.CacheState(w.astype(np.float64), width=width, n_hidden=n_hidden)


# ---------------------------------------------------------------------------
# Encoding (Sec. 3.6)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n", [4096, 1000, 129, 1])
def test_encode_matches_oracle(N, prec, preset, layout, n):
    c, _ = make_cache(N, prec, preset=preset)
    raw = sd.raw_records(n, 100 + n, layout)
    enc = N.nrc_encode(c, dev(raw), layout).float().cpu().numpy().astype(np.float64)
    ref = O.encode(raw, layout, preset)
    tol = 2e-6 + ENC_REL[prec] * np.abs(ref) * 1.0001
    err = np.abs(enc - ref)
    assert np.all(err <= tol), f"max excess {np.max(err - tol)} at {np.unravel_index(np.argmax(err - tol), err.shape)}"


def test_encode_empty_is_noop(N):
    c, _ = make_cache(N, "fp16")
    raw = torch.empty((0, 14), device="cuda")
    enc = N.nrc_encode(c, raw, 0)
    assert enc.shape == (0, 64)


def test_encode_dyadic_one_blob_exact(N):
    # One-blob values at dyadic coordinates are exact rationals representable in FP16.
    s = np.array([0, 1 / 8, 1 / 4, 3 / 8, 1 / 2, 5 / 8, 3 / 4, 7 / 8, 1.0])
    raw = np.zeros((9, 14), dtype=np.float32)
    raw[:, 3] = s
    for prec in PRECS:
        c, _ = make_cache(N, prec)
        enc = N.nrc_encode(c, dev(raw), 0).float().cpu().numpy().astype(np.float64)
        assert np.array_equal(enc[:, 36:40], O.one_blob(s)), prec


# ---------------------------------------------------------------------------
# Forward (Sec. 4, Sec. 5 architecture)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [4096, 4097, 1000, 65, 16, 1])
def test_forward_matches_oracle(N, prec, n):
    c, w = make_cache(N, prec)
    x, x64 = rounded_input(sd.uniform_features(n, 64, 7 + n), prec)
    rgb = N.nrc_forward(c, x).cpu().numpy()
    ref = O.predict(state_of(w), x64)
    err = O.channel_rel_error(rgb, ref)
    assert np.all(err <= FWD_TOL[prec]), err


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_forward_width128(N, prec):
    c, w = make_cache(N, prec, width=128)
    x, x64 = rounded_input(sd.uniform_features(3000, 64, 8), prec)
    rgb = N.nrc_forward(c, x).cpu().numpy()
    ref = O.predict(state_of(w, 128), x64)
    assert np.all(O.channel_rel_error(rgb, ref) <= FWD_TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_hidden", [1, 2, 3])
def test_forward_other_depths(N, prec, n_hidden):
    c, w = make_cache(N, prec, n_hidden=n_hidden)
    x, x64 = rounded_input(sd.uniform_features(777, 64, 9), prec)
    rgb = N.nrc_forward(c, x).cpu().numpy()
    ref = O.predict(state_of(w, 64, n_hidden), x64)
    assert np.all(O.channel_rel_error(rgb, ref) <= FWD_TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_forward_encoded_records_end_to_end(N, prec):
    c, w = make_cache(N, prec)
    raw = sd.raw_records(5000, sd.SEED_QUERIES)
    rgb = N.nrc_forward(c, N.nrc_encode(c, dev(raw), 0)).cpu().numpy()
    ref = O.predict(state_of(w), O.encode(raw))
    assert np.all(O.channel_rel_error(rgb, ref) <= FWD_TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_forward_positive_homogeneity(N, prec):
    # No biases and ReLU: f(2x) = 2 f(x).  Exact in FP32 and BF16 (no subnormals
    # in range); FP16 can round subnormal activations differently.
    c, _ = make_cache(N, prec)
    x, _ = rounded_input(sd.uniform_features(2048, 64, 10), prec)
    y1 = N.nrc_forward(c, x)
    y2 = N.nrc_forward(c, (x.float() * 2).to(x.dtype))
    if prec == "fp16":
        assert torch.allclose(y2, 2 * y1, rtol=1e-3, atol=1e-6)
    else:
        assert torch.equal(y2, 2 * y1)


def test_forward_zero_weights_give_zero(N):
    for prec in PRECS:
        c, _ = make_cache(N, prec, weights=np.zeros(sd.n_params(), dtype=np.float32))
        x, _ = rounded_input(sd.uniform_features(300, 64, 11), prec)
        assert torch.count_nonzero(N.nrc_forward(c, x)) == 0


def test_forward_empty(N):
    c, _ = make_cache(N, "fp16")
    assert N.nrc_forward(c, torch.empty((0, 64), dtype=torch.float16, device="cuda")).shape == (0, 3)


# ---------------------------------------------------------------------------
# Training (Eq. 5, Sec. 5 optimizer, Sec. 3.4-3.5 schedule)
# ---------------------------------------------------------------------------
def _train_parity(N, prec, n, steps, seed, out_tol, loss_tol, width=64):
    c, w = make_cache(N, prec, width=width)
    raw = sd.raw_records(n * steps, seed)
    enc = N.nrc_encode(c, dev(raw), 0)
    enc64 = enc.float().cpu().numpy().astype(np.float64)
    y = sd.targets(raw)
    yd = dev(y)
    st = state_of(w, width)
    for s in range(steps):
        sl = slice(s * n, (s + 1) * n)
        loss, skipped = N.nrc_train_step(c, enc[sl].contiguous(), yd[sl].contiguous())
        ref_loss, ref_skip = O.train_step(st, enc64[sl], y[sl].astype(np.float64))
        assert int(skipped.item()) == 0 and not ref_skip
        assert abs(loss.item() - ref_loss) <= loss_tol * abs(ref_loss), (s, loss.item(), ref_loss)
    q, q64 = rounded_input(O.encode(sd.raw_records(4096, sd.SEED_HELDOUT)), prec)
    got = N.nrc_forward(c, q).cpu().numpy()
    ref = O.predict(st, q64)
    err = O.channel_rel_error(got, ref)
    assert np.all(err <= out_tol), err
    wt = c.get_weights().astype(np.float64)
    rel_w = np.linalg.norm(wt - st.w) / np.linalg.norm(st.w)
    return err, rel_w


def test_train_fp32_one_step_config0(N):
    _, rel_w = _train_parity(N, "fp32", 1024, 1, sd.SEED_RECORDS, 1e-5, 1e-5)
    assert rel_w < 1e-5


def test_train_fp32_four_steps_frame_schedule(N):
    _, rel_w = _train_parity(N, "fp32", 16384, 4, sd.SEED_RECORDS, 1e-5, 1e-5)
    assert rel_w < 1e-5


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_train_mfma_one_step(N, prec):
    _train_parity(N, prec, 1024, 1, sd.SEED_RECORDS, 1e-2 if prec == "fp16" else 2e-2, 1e-2)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_train_mfma_four_steps_frame_schedule(N, prec):
    _, rel_w = _train_parity(N, prec, 16384, 4, sd.SEED_RECORDS, 1e-2, 1e-2)
    assert rel_w < 2e-2


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 63, 65, 1000])
def test_train_ragged_batches(N, prec, n):
    tol = 1e-5 if prec == "fp32" else 3e-2
    _train_parity(N, prec, n, 1, 40 + n, tol, 1e-5 if prec == "fp32" else 1e-2)


@pytest.mark.parametrize("prec", PRECS)
def test_train_skips_non_finite_gradient(N, prec):
    c, w = make_cache(N, prec)
    raw = sd.raw_records(512, 12)
    y = sd.targets(raw)
    y[17, 1] = np.inf
    enc = N.nrc_encode(c, dev(raw), 0)
    _, skipped = N.nrc_train_step(c, enc, dev(y))
    assert int(skipped.item()) == 1
    wt, m, v, t = c.get_state()
    assert t == 0 and np.array_equal(wt, w) and not m.any() and not v.any()
    # the next finite step proceeds as the first step
    _, skipped = N.nrc_train_step(c, enc, dev(sd.targets(raw)))
    assert int(skipped.item()) == 0
    assert c.get_state()[3] == 1


@pytest.mark.parametrize("prec", PRECS)
def test_train_is_deterministic_and_resumable(N, prec):
    raw = sd.raw_records(4 * 2048, 13)
    y = dev(sd.targets(raw))

    def run(c, steps, start=0):
        enc = N.nrc_encode(c, dev(raw), 0)
        for s in range(start, start + steps):
            N.nrc_train_step(c, enc[s * 2048:(s + 1) * 2048], y[s * 2048:(s + 1) * 2048])
        torch.cuda.synchronize()

    a, _ = make_cache(N, prec)
    run(a, 4)
    b, _ = make_cache(N, prec)
    run(b, 4)
    assert np.array_equal(a.get_weights(), b.get_weights())
    # checkpoint after 2 steps, restore into a fresh cache, continue: bitwise equal
    c, _ = make_cache(N, prec)
    run(c, 2)
    state = c.get_state()
    d, _ = make_cache(N, prec)
    d.set_state(*state)
    run(d, 2, start=2)
    wa, ma, va, ta = a.get_state()
    wd, md, vd, td = d.get_state()
    assert ta == td == 4
    assert np.array_equal(wa, wd) and np.array_equal(ma, md) and np.array_equal(va, vd)


# ---------------------------------------------------------------------------
# Backward with an upstream gradient (autograd form)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,width", [("fp32", 64), ("fp16", 64), ("bf16", 64), ("fp16", 128)])
def test_backward_matches_oracle(N, prec, width):
    c, w = make_cache(N, prec, width=width)
    n = 1000
    x, x64 = rounded_input(sd.uniform_features(n, 64, 14), prec)
    r = sd.gaussian((n, 3), sd.SEED_FD)
    gw, genc = N.nrc_backward(c, x, dev(r))
    st = state_of(w, width)
    y, hs = O.forward(st.mats(), x64)
    grads, gin = O.backward(st.mats(), hs, r.astype(np.float64))
    ref_w = np.concatenate([g.reshape(-1) for g in grads])
    gw = gw.cpu().numpy()
    tol = 1e-5 if prec == "fp32" else (1e-2 if prec == "fp16" else 3e-2)
    off = 0
    for l, g in enumerate(grads):
        sz = g.size
        e = np.max(np.abs(gw[off:off + sz] - ref_w[off:off + sz])) / np.max(np.abs(ref_w[off:off + sz]))
        assert e <= tol, (l, e)
        off += sz
    e_in = np.max(np.abs(genc.cpu().numpy() - gin)) / np.max(np.abs(gin))
    assert e_in <= tol, e_in


# ---------------------------------------------------------------------------
# Full frame size: sampled rows against the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", PRECS)
def test_full_frame_sampled(N, prec):
    n = 1920 * 1080
    c, w = make_cache(N, prec)
    raw = sd.raw_records(n, sd.SEED_QUERIES)
    rgb = N.nrc_forward(c, N.nrc_encode(c, dev(raw), 0))
    idx = np.random.Generator(np.random.PCG64(99)).choice(n, 4096, replace=False)
    idx = np.concatenate([idx, [0, n - 1]])
    got = rgb.cpu().numpy()[idx]
    ref = O.predict(state_of(w), O.encode(raw[idx]))
    assert np.all(O.channel_rel_error(got, ref) <= FWD_TOL[prec])

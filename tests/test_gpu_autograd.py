"""Differentiation form: the fused kernels behind torch.autograd.Function.

Widths 64 and 128, 5 hidden layers, batch 2^16, FP16 (and FP32 at width 64).
L = sum(R * network(enc)) with a seeded R ~ N(0,1), so dL/dy = R.  Gradients
of the weights and of the encoded inputs are compared with the FP64 oracle
(whose own gradients are pinned by central finite differences) and with the
rounding model; tolerances as in test_gpu_parity.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd
from oracle import nrc_oracle as O
from tests import rounding_model as RM
from tests.test_gpu_parity import BWD_TOL, FWD_TOL, MODEL_TOL, l2_err

pytestmark = pytest.mark.gpu


def _maxnorm(got, ref):
    """max_i |got - ref| / max_i |ref| (max-normwise relative error)."""
    return float(np.max(np.abs(np.asarray(got) - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def AG():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_12372_amd import autograd
    return autograd


@pytest.mark.parametrize("prec,width,n", [("fp16", 64, 65536), ("fp16", 128, 65536), ("fp32", 64, 4096),
                                          ("bf16", 64, 65536)])
def test_autograd_gradients(AG, prec, width, n):
    mod = AG.NRCModule(width=width, n_hidden=5, precision=prec)
    dt = mod.cache.enc_dtype
    x = torch.from_numpy(sd.uniform_features(n, 64, 51)).to("cuda").to(dt).requires_grad_(True)
    r = sd.gaussian((n, 3), sd.SEED_FD)
    if prec == "fp32":
        # records whose ReLU masks rounding decides (a pre-activation within
        # the FP32 dot-product error bound gamma_64 sum |w h| of zero, 12 of
        # 4096 here) take no upstream gradient, so the strict FP32 bound
        # compares only what the arithmetic fixes (with this seed, one unit
        # sits 1.4e-8 sum |w h| from zero and rounds the other way)
        st0 = O.CacheState(mod.weights.detach().cpu().numpy(), width=width)
        x0 = x.detach().float().cpu().numpy().astype(np.float64)
        r[RM.relu_undecided_rows(st0.mats(), x0)] = 0.0
    y = mod(x)
    (y * torch.from_numpy(r).to("cuda")).sum().backward()
    gw = mod.weights.grad.cpu().numpy().astype(np.float64)
    gx = x.grad.float().cpu().numpy().astype(np.float64)
    x64 = x.detach().float().cpu().numpy().astype(np.float64)
    w = mod.weights.detach().cpu().numpy()
    st = O.CacheState(w, width=width)
    yref, hs = O.forward(st.mats(), x64)
    assert np.all(l2_err(y.detach().cpu().numpy(), yref) <= FWD_TOL[prec])
    grads, gin = O.backward(st.mats(), hs, r.astype(np.float64))
    ref_w = np.concatenate([g.reshape(-1) for g in grads])
    assert np.linalg.norm(gw - ref_w) / np.linalg.norm(ref_w) <= BWD_TOL[prec]
    # grad_enc comes back in the input dtype, so compare it at that rounding
    q = RM.quantiser(prec)
    assert np.linalg.norm(gx - q(gin)) / np.linalg.norm(gin) <= BWD_TOL[prec]
    got_layers = sd.split_weights(gw.astype(np.float64), width, 5)
    if prec == "fp32":
        # element by element: every layer's max-normwise error within the FP32 bound
        for l, (a, b) in enumerate(zip(got_layers, grads)):
            assert _maxnorm(a, b) <= 1e-5, (l, _maxnorm(a, b))
        assert _maxnorm(gx, gin) <= 1e-5
        return
    _, mhs, qm = RM.forward(st.mats(), x64, q, RM.train_weight_quantiser(prec))
    mg, mgin = RM.backward(qm, mhs, r.astype(np.float64), q)
    mref = np.concatenate([g.reshape(-1) for g in mg])
    assert np.linalg.norm(gw - mref) / np.linalg.norm(mref) <= MODEL_TOL[prec]
    assert np.linalg.norm(gx - q(mgin)) / np.linalg.norm(mgin) <= MODEL_TOL[prec]
    # Layer by layer, in the L2 and the max norm: the distance to the oracle is
    # the format's own (the rounding model's distance, here 3-5% in FP16 and up
    # to 21% max-normwise in BF16 under random-sign upstream gradients) plus a
    # quarter, and the distance to the rounding model is the kernels' own
    # summation order.
    for l, (a, b, m) in enumerate(zip(got_layers, grads, mg)):
        fmt_l2 = np.linalg.norm(m - b) / np.linalg.norm(b)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1.25 * fmt_l2 + 1e-3, (l, "l2")
        assert _maxnorm(a, b) <= 1.25 * _maxnorm(m, b) + 1e-3, (l, "max", _maxnorm(a, b), _maxnorm(m, b))
        assert np.linalg.norm(a - m) / np.linalg.norm(m) <= MODEL_TOL[prec], (l, "model l2")
        assert _maxnorm(a, m) <= 2 * MODEL_TOL[prec], (l, "model max", _maxnorm(a, m))


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_autograd_factorised(AG, prec):
    # Reflectance factorisation: the input gradient also flows into the albedo
    # columns (d(f R)/dR = f).
    from paper_2106_12372_amd import nrc as N
    mod = AG.NRCModule(precision=prec, factorize=True)
    raw = sd.raw_records(8192, 53)
    x = N.nrc_encode(mod.cache, torch.from_numpy(raw).to("cuda")).requires_grad_(True)
    r = sd.gaussian((8192, 3), sd.SEED_FD)
    y = mod(x)
    (y * torch.from_numpy(r).to("cuda")).sum().backward()
    x64 = x.detach().float().cpu().numpy().astype(np.float64)
    st = O.CacheState(mod.weights.detach().cpu().numpy(), factorize=True)
    assert np.all(l2_err(y.detach().cpu().numpy(), O.predict(st, x64)) <= FWD_TOL[prec])
    ref_w, ref_in = O.query_gradient(st, x64, r.astype(np.float64))
    gw = mod.weights.grad.cpu().numpy().astype(np.float64)
    gx = x.grad.float().cpu().numpy().astype(np.float64)
    q = RM.quantiser(prec)
    assert np.linalg.norm(gw - ref_w) / np.linalg.norm(ref_w) <= BWD_TOL[prec]
    assert np.linalg.norm(gx - q(ref_in)) / np.linalg.norm(ref_in) <= BWD_TOL[prec]


def test_autograd_drives_torch_optimizer(AG):
    mod = AG.NRCModule(precision="fp16")
    raw = sd.raw_records(4096, 52)
    from paper_2106_12372_amd import nrc as N
    enc = N.nrc_encode(mod.cache, torch.from_numpy(raw).to("cuda"))
    y = torch.from_numpy(sd.targets(raw)).to("cuda")
    opt = torch.optim.Adam(mod.parameters(), lr=1e-2, betas=(0.9, 0.99))
    losses = []
    for _ in range(30):
        opt.zero_grad()
        pred = mod(enc)
        loss = ((pred - y) ** 2 / (pred.detach().mean(1, keepdim=True) ** 2 + 0.01)).mean()
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.05 * losses[0]


@pytest.mark.parametrize("prec,width", [("fp16", 64), ("fp16", 128), ("bf16", 64), ("fp32", 64)])
def test_backward_from_kept_activations(AG, prec, width):
    # nrc_forward_train keeps the activations; nrc_backward then reads them
    # instead of recomputing the forward pass.  The values are the ones the
    # recompute produces, so both gradients agree bit for bit, and both follow
    # the oracle's gradient (Sec. 4: the activations kept for backpropagation).
    from paper_2106_12372_amd import nrc as N
    n = 65536 if prec != "fp32" else 4097
    cfg = N.make_config(width=width, precision=prec)
    c = N.Cache(cfg)
    w = sd.glorot_weights(width, 5)
    c.set_weights(w)
    x = torch.from_numpy(sd.uniform_features(n, 64, 61)).to("cuda").to(c.enc_dtype)
    r = sd.gaussian((n, 3), sd.SEED_FD)
    if prec == "fp32":
        st0 = O.CacheState(w.astype(np.float64), width=width)
        r[RM.relu_undecided_rows(st0.mats(), x.float().cpu().numpy().astype(np.float64))] = 0.0
    rd = torch.from_numpy(r).to("cuda")
    rgb, act = N.nrc_forward_train(c, x)
    assert act.numel() == N.nrc_act_ws_bytes(cfg, n)
    if prec in ("fp16", "fp32"):
        assert torch.equal(rgb, N.nrc_forward(c, x))      # the same products in the same order
    gw_a, gx_a = N.nrc_backward(c, x, rd, act=act)
    gw_r, gx_r = N.nrc_backward(c, x, rd)
    assert torch.equal(gw_a, gw_r) and torch.equal(gx_a, gx_r)
    x64 = x.float().cpu().numpy().astype(np.float64)
    st = O.CacheState(w.astype(np.float64), width=width)
    assert np.all(l2_err(rgb.cpu().numpy(), O.predict(st, x64)) <= FWD_TOL[prec])
    ref_w, ref_in = O.query_gradient(st, x64, r.astype(np.float64))
    gw = gw_a.cpu().numpy().astype(np.float64)
    gx = gx_a.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gw - ref_w) / np.linalg.norm(ref_w) <= BWD_TOL[prec]
    assert np.linalg.norm(gx - ref_in) / np.linalg.norm(ref_in) <= BWD_TOL[prec]


@pytest.mark.parametrize("factorize", [False, True])
def test_autograd_mean_relative_loss_fp16_is_loss_scaled(AG, factorize):
    # A mean-reduced relative L2 loss (Eq. 5) over 2^16 records on targets
    # within a few percent of the prediction (a cache that fits) gives dL/dy
    # of order 1e-6, inside FP16's subnormal range (below 2^-14); the backward
    # pass scales it by the loss scale before rounding and divides the scale
    # out of the sums, so the gradients follow the oracle's at the FP16 bound.
    from paper_2106_12372_amd import nrc as N
    mod = AG.NRCModule(precision="fp16", factorize=factorize)
    n = 65536
    raw = sd.raw_records(n, 62)
    x = N.nrc_encode(mod.cache, torch.from_numpy(raw).to("cuda")).requires_grad_(True)
    st0 = O.CacheState(mod.weights.detach().cpu().numpy().astype(np.float64), factorize=factorize)
    near = O.predict(st0, x.detach().float().cpu().numpy().astype(np.float64))
    near = near * (1.0 + 0.05 * sd.gaussian((n, 3), 63).astype(np.float64))
    y = torch.from_numpy(near.astype(np.float32)).to("cuda")
    pred = mod(x)
    pred.retain_grad()
    lum = pred.detach().mean(1, keepdim=True)
    loss = ((pred - y) ** 2 / (lum ** 2 + 0.01)).mean()
    loss.backward()
    g_out = pred.grad.detach().cpu().numpy().astype(np.float64)
    assert np.median(np.abs(g_out)) < 2.0 ** -14           # the regime loss scaling is for
    x64 = x.detach().float().cpu().numpy().astype(np.float64)
    st = O.CacheState(mod.weights.detach().cpu().numpy().astype(np.float64), factorize=factorize)
    ref_w, ref_in = O.query_gradient(st, x64, g_out)
    gw = mod.weights.grad.cpu().numpy().astype(np.float64)
    gx = x.grad.float().cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gw - ref_w) / np.linalg.norm(ref_w) <= BWD_TOL["fp16"]
    assert np.linalg.norm(gx - RM.quantiser("fp16")(ref_in)) / np.linalg.norm(ref_in) <= BWD_TOL["fp16"]
    # per layer, too
    mats_ref = sd.split_weights(ref_w)
    mats_got = sd.split_weights(gw)
    for a, b in zip(mats_got, mats_ref):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= BWD_TOL["fp16"]

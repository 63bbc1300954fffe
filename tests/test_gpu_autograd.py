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
        # records whose ReLU masks rounding decides take no upstream gradient,
        # so the strict FP32 bound compares only what the arithmetic fixes
        # (with this seed, one unit of 4096 records sits 1.4e-8 from zero)
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
    if prec != "fp32":
        _, mhs, qm = RM.forward(st.mats(), x64, q)
        mg, mgin = RM.backward(qm, mhs, r.astype(np.float64), q)
        mref = np.concatenate([g.reshape(-1) for g in mg])
        assert np.linalg.norm(gw - mref) / np.linalg.norm(mref) <= MODEL_TOL[prec]
        assert np.linalg.norm(gx - q(mgin)) / np.linalg.norm(mgin) <= MODEL_TOL[prec]


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

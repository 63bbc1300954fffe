"""The training step that allocates nothing (nrc_train_step_noalloc), through
the C ABI: on two calls in a row, the second with a smaller batch, its loss,
skip flag and updated weights equal those of nrc_train_step with a caller
scratch buffer, bit for bit (the same kernels on the same inputs)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12372_amd.nrc as nrc
    return nrc


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_noalloc_step_equals_scratch_step(N, prec):
    cfg = N.make_config(precision=prec, ema_alpha=0.99)
    a, b = N.Cache(cfg), N.Cache(cfg)
    w = sd.glorot_weights()
    a.set_weights(w)
    b.set_weights(w)
    for n, seed in ((16384, 710), (1000, 711)):
        raw = sd.raw_records(n, seed)
        enc = N.nrc_encode(a, torch.from_numpy(raw).cuda())
        y = torch.from_numpy(sd.targets(raw)).cuda()
        print(f"step n={n} prec={prec}", flush=True)
        la, sa = N.nrc_train_step(a, enc, y)
        lb, sb = N.nrc_train_step_noalloc(b, enc, y)
        torch.cuda.synchronize()
        assert int(sa.item()) == 0 and int(sb.item()) == 0
        assert la.item() == lb.item(), (n, la.item(), lb.item())
        assert np.array_equal(a.get_weights(), b.get_weights()), n
        wa, ea = a.get_ema()
        wb, eb = b.get_ema()
        assert np.array_equal(wa, wb) and np.array_equal(ea, eb), n
        q = N.nrc_encode(a, torch.from_numpy(sd.raw_records(4096, 712)).cuda())
        assert torch.equal(N.nrc_forward(a, q), N.nrc_forward(b, q)), n


def test_noalloc_step_refuses_batches_beyond_its_array(N):
    cfg = N.make_config(precision="fp16")
    c = N.Cache(cfg)
    c.set_weights(sd.glorot_weights())
    n = 1
    while N.nrc_train_scratch_bytes(cfg, n) <= N.NRC_NOALLOC_SCRATCH_BYTES:
        n *= 2
    enc = torch.zeros((n, 64), dtype=torch.float16, device="cuda")
    y = torch.ones((n, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(N.NrcError) as e:
        N.nrc_train_step_noalloc(c, enc, y)
    assert e.value.code == N.NRC_ENOMEM
    assert "fixed scratch" in N.last_error()

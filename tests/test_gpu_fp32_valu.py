"""The plain FP32 form on the vector ALUs (NRC_FP32_VALU, no matrix
instructions): the baseline the matrix-core forms are compared with.  Same
oracle, same FP32 bounds as the FP32 matrix-core form (1e-5 normwise per
channel; loss 1e-5 relative)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd
from oracle import nrc_oracle as O
from tests import rounding_model as RM
from tests.test_gpu_parity import check_outputs, l2_err

pytestmark = pytest.mark.gpu
P = "fp32_valu"


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12372_amd.nrc as nrc
    return nrc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make(N, **kw):
    c = N.Cache(N.make_config(precision=P, **kw))
    w = sd.glorot_weights()
    c.set_weights(w)
    return c, w


@pytest.mark.parametrize("n", [1, 63, 1000, 4097])
def test_forward_matches_oracle(N, n):
    c, w = make(N)
    x = sd.uniform_features(n, 64, 700 + n)
    got = N.nrc_forward(c, dev(x)).cpu().numpy()
    check_outputs(got, O.predict(O.CacheState(w.astype(np.float64)), x.astype(np.float64)), 1e-5, 1e-5)


@pytest.mark.parametrize("preset", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
def test_forward_raw_equals_encode_then_forward(N, preset, layout):
    c, w = make(N, enc_preset=preset)
    raw = dev(sd.raw_records(3001, 710 + preset, layout))
    fused = N.nrc_forward_raw(c, raw, layout)
    assert torch.equal(fused, N.nrc_forward(c, N.nrc_encode(c, raw, layout)))
    ref = O.predict(O.CacheState(w.astype(np.float64)), O.encode(raw.cpu().numpy(), layout, preset))
    check_outputs(fused.cpu().numpy(), ref, 1e-5, 1e-5)


def test_frame_schedule_matches_oracle(N):
    # four 16,384-record steps on the shuffled records of one frame
    c, w = make(N)
    raw = sd.raw_records(65536, sd.SEED_RECORDS)
    enc = N.nrc_encode(c, dev(raw))
    y = sd.targets(raw)
    losses, skipped = N.nrc_train_frame(c, enc, dev(y), steps=4, batch=16384, seed=3)
    st = O.CacheState(w.astype(np.float64))
    q = O.encode(sd.raw_records(65536, sd.SEED_HELDOUT))
    _, ref_l, ref_skip = O.frame_shuffled(st, q[:0], enc.cpu().numpy().astype(np.float64), y.astype(np.float64),
                                          4, 16384, 3)
    got_losses = losses.cpu().numpy()
    assert int(skipped.sum().item()) == 0 and not any(ref_skip)
    assert np.allclose(got_losses, ref_l, rtol=1e-5), (got_losses, ref_l)
    got = N.nrc_forward(c, dev(q.astype(np.float32))).cpu().numpy()
    check_outputs(got, O.predict(st, q), 1e-5, 1e-5)


def test_backward_matches_oracle(N):
    c, w = make(N)
    n = 4096
    x = sd.uniform_features(n, 64, 720)
    r = sd.gaussian((n, 3), sd.SEED_FD)
    st = O.CacheState(w.astype(np.float64))
    r[RM.relu_undecided_rows(st.mats(), x.astype(np.float64))] = 0.0
    gw, gx = N.nrc_backward(c, dev(x), dev(r))
    ref_w, ref_in = O.query_gradient(st, x.astype(np.float64), r.astype(np.float64))
    gw = gw.cpu().numpy().astype(np.float64)
    for a, b in zip(sd.split_weights(gw), sd.split_weights(ref_w)):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-5
    assert np.linalg.norm(gx.cpu().numpy() - ref_in) / np.linalg.norm(ref_in) <= 1e-5


def test_no_activation_buffer(N):
    c, _ = make(N)
    x = dev(sd.uniform_features(100, 64, 730))
    with pytest.raises(N.NrcError) as e:
        N.nrc_forward_train(c, x, act=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.code == N.NRC_EINVAL

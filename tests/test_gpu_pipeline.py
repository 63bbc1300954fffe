"""Training-record pipeline of one frame (Sec. 3.3 footnote, Sec. 3.5, Sec. 3.2)
through the C ABI: the LCG shuffle (integer work: bit-exact against the
oracle), training on gathered batches, the whole frame update, and the
self-training targets.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd
from oracle import nrc_oracle as O
from tests import rounding_model as RM
from tests.test_gpu_parity import MODEL_TOL, check_fp32_adam_step, dev, l2_err, make_cache, rounded_input, state_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12372_amd.nrc as nrc
    return nrc


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 16384, 65536, 65537, 100003, (1 << 20) + 5])
@pytest.mark.parametrize("seed", [0, 1, (1 << 40) + 7])
def test_shuffle_matches_oracle_bitwise(N, n, seed):
    got = N.nrc_shuffle(n, seed).cpu().numpy()
    assert np.array_equal(got, O.lcg_permutation(n, seed))


def test_shuffle_empty(N):
    assert N.nrc_shuffle(0, 3).numel() == 0


@pytest.mark.parametrize("n", [(1 << 25) + 3, 1 << 24])
def test_shuffle_large_is_a_permutation_with_the_oracle_ends(N, n):
    # 2^25 + 3 (m = 2^26, the counting kernels, 256 rounds per workgroup) and
    # 2^24 (m = n, the single kernel, 64 rounds).  The whole orbit is too long
    # for the oracle's loop, so check that the result is a permutation and that
    # its first and last entries follow the orbit forwards from x_0 and
    # backwards from x_0 (the inverse map x -> a^-1 (x - c) mod m).
    seed = 12345
    perm = N.nrc_shuffle(n, seed)
    srt, _ = torch.sort(perm)
    assert torch.equal(srt, torch.arange(n, device="cuda", dtype=torch.int32))
    m = O.lcg_modulus(n)
    x, head = seed % m, []
    while len(head) < 1000:
        if x < n:
            head.append(x)
        x = (O.LCG_A * x + O.LCG_C) % m
    inv = pow(O.LCG_A, -1, m)
    x, tail = seed % m, []
    while len(tail) < 1000:
        x = (inv * (x - O.LCG_C)) % m
        if x < n:
            tail.append(x)
    p = perm.cpu().numpy()
    assert p[:1000].tolist() == head
    assert p[-1000:].tolist() == tail[::-1]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_indexed_step_equals_step_on_gathered_batch(N, prec):
    raw = sd.raw_records(5000, 81)
    y = dev(sd.targets(raw))
    idx = N.nrc_shuffle(5000, 4)[:1234].contiguous()
    a, _ = make_cache(N, prec, factorize=True)
    b, _ = make_cache(N, prec, factorize=True)
    enc = N.nrc_encode(a, dev(raw), 0)
    la, sa = N.nrc_train_step_indexed(a, enc, y, idx)
    il = idx.long()
    lb, sb = N.nrc_train_step(b, enc[il].contiguous(), y[il].contiguous())
    assert torch.equal(la, lb) and int(sa.item()) == int(sb.item()) == 0
    assert np.array_equal(a.get_weights(), b.get_weights())


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp32_valu"])
@pytest.mark.parametrize("preset", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n_records", [32768, 20001])
def test_raw_frame_equals_encode_then_frame(N, prec, preset, layout, n_records):
    # The training kernels encode each gathered raw record with the encoding
    # kernel's arithmetic and rounding, so a frame on raw records equals the
    # frame on their encoding bit for bit: losses, skip flags, weights, Adam
    # moments and step count.  32,768 records take the in-kernel LCG orbit,
    # 20,001 the shuffle's permutation (steps of 5,000 and 5,001 records,
    # ragged tiles).  Every other preset factorises by the reflectance, whose
    # albedo columns the kernels then read from the encoded row.
    raw = sd.raw_records(n_records, 90 + n_records, layout)
    y = dev(sd.targets(raw))
    fact = preset % 2 == 0
    a, _ = make_cache(N, prec, preset=preset, factorize=fact)
    b, _ = make_cache(N, prec, preset=preset, factorize=fact)
    la, sa = N.nrc_train_frame(a, N.nrc_encode(a, dev(raw), layout), y, steps=4, batch=8192, seed=11)
    lb, sb = N.nrc_train_frame_raw(b, dev(raw), y, layout=layout, steps=4, batch=8192, seed=11)
    assert torch.equal(la, lb) and torch.equal(sa, sb)
    assert int(sa.sum().item()) == 0
    for x, z in zip(a.get_state()[:3], b.get_state()[:3]):
        assert np.array_equal(x, z)
    assert a.get_state()[3] == b.get_state()[3] == 4


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp32_valu"])
def test_raw_frame_with_a_non_finite_record_skips_like_the_encoded_frame(N, prec):
    # A NaN position encodes to NaN features in both paths, so the step that
    # gathers that record has a non-finite gradient and is skipped; the other
    # steps go ahead.  Both paths agree bit for bit, skip flags included.
    raw = sd.raw_records(32768, 17)
    raw[12345, 0] = np.nan
    y = dev(sd.targets(np.nan_to_num(raw)))
    a, _ = make_cache(N, prec)
    b, _ = make_cache(N, prec)
    la, sa = N.nrc_train_frame(a, N.nrc_encode(a, dev(raw), 0), y, steps=4, batch=8192, seed=5)
    lb, sb = N.nrc_train_frame_raw(b, dev(raw), y, steps=4, batch=8192, seed=5)
    assert torch.equal(sa, sb) and int(sa.sum().item()) == 1
    assert torch.equal(la.isnan(), lb.isnan())
    assert torch.equal(la[~la.isnan()], lb[~lb.isnan()])
    assert np.array_equal(a.get_weights(), b.get_weights())


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp32_valu"])
@pytest.mark.parametrize("layout", [0, 1])
def test_raw_frame_on_edge_records_equals_encode_then_frame(N, prec, layout):
    # The method's edge inputs (positions far outside [0, 1), exact 0 and 1,
    # RAW16 poles, angles on bin edges, roughness 0 and large) through the
    # in-kernel encoding of the training step, against the encoding kernel.
    raw = sd.edge_records(8000, 77 + layout, layout)
    y = dev(sd.targets(raw))
    a, _ = make_cache(N, prec, preset=1)
    b, _ = make_cache(N, prec, preset=1)
    la, sa = N.nrc_train_frame(a, N.nrc_encode(a, dev(raw), layout), y, steps=4, batch=2048, seed=2)
    lb, sb = N.nrc_train_frame_raw(b, dev(raw), y, layout=layout, steps=4, batch=2048, seed=2)
    assert torch.equal(la, lb) and torch.equal(sa, sb)
    assert np.array_equal(a.get_weights(), b.get_weights())


def test_raw_frame_needs_width_64(N):
    c, _ = make_cache(N, "fp16", width=128)
    raw = sd.raw_records(4096, 5)
    with pytest.raises(N.NrcError):
        N.nrc_train_frame_raw(c, dev(raw), dev(sd.targets(raw)), steps=4, batch=1024)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("n_records", [65536, 50001, 70000])
def test_frame_steps_match_oracle_from_the_same_state(N, prec, n_records):
    # Each of the frame's steps against the oracle's step from the GPU's own
    # state before it (weights, Adam moments, t), on the oracle's shuffled
    # batch: the arithmetic of every step is checked without the rounding
    # differences of earlier steps compounding through Adam's sign-like
    # first update.
    c, w = make_cache(N, prec)
    raw = sd.raw_records(n_records, 82)
    enc = N.nrc_encode(c, dev(raw), 0)
    e64 = enc.float().cpu().numpy().astype(np.float64)
    y = sd.targets(raw)
    yd = dev(y)
    perm = N.nrc_shuffle(n_records, 77)
    batches = O.frame_batches(n_records, 4, 16384, 77)
    assert np.array_equal(perm.cpu().numpy()[:sum(b.size for b in batches)], np.concatenate(batches))
    tol = 1e-5 if prec == "fp32" else 1e-2
    lo = 0
    for k, idx in enumerate(batches):
        wt, m, v, t = c.get_state()
        st = O.CacheState(wt.astype(np.float64), m=m.astype(np.float64), v=v.astype(np.float64), t=t)
        st_before = O.CacheState(st.w.copy(), m=st.m.copy(), v=st.v.copy(), t=t)
        ref_loss, ref_skip = O.train_step(st, e64[idx], y[idx].astype(np.float64))
        loss, skipped = N.nrc_train_step_indexed(c, enc, yd, perm[lo:lo + idx.size].contiguous())
        lo += idx.size
        assert int(skipped.item()) == 0 and not ref_skip
        assert abs(loss.item() - ref_loss) <= tol * abs(ref_loss), (k, loss.item(), ref_loss)
        if prec == "fp32":
            check_fp32_adam_step(c.get_weights(), st_before, st.w, e64[idx], y[idx].astype(np.float64))


FRAME_MAX_TOL = {"fp16": 1e-2, "bf16": 1e-2}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_train_frame_matches_oracle_frame(N, prec):
    # The whole reduced-precision frame against the oracle's frame (4 x 16,384),
    # then per-channel error on 65,536 held-out queries through the trained
    # weights: normwise L2 and normwise max (max_i |got - ref| / max_i |ref|).
    c, w = make_cache(N, prec)
    raw = sd.raw_records(65536, 82)
    enc = N.nrc_encode(c, dev(raw), 0)
    e64 = enc.float().cpu().numpy().astype(np.float64)
    y = sd.targets(raw)
    losses, skipped = N.nrc_train_frame(c, enc, dev(y), steps=4, batch=16384, seed=77)
    st = state_of(w)
    q, q64 = rounded_input(O.encode(sd.raw_records(65536, sd.SEED_HELDOUT)), prec)
    _, ref_losses, ref_skips = O.frame_shuffled(st, q64, e64, y.astype(np.float64), 4, 16384, 77)
    assert skipped.cpu().tolist() == [0, 0, 0, 0] and not any(ref_skips)
    got_l = losses.cpu().numpy()
    assert np.all(np.abs(got_l - ref_losses) <= 1e-2 * np.abs(ref_losses)), (got_l, ref_losses)
    got_d = N.nrc_forward(c, q)
    got = got_d.cpu().numpy()
    ref = O.predict(st, q64)
    e2, em = l2_err(got, ref), O.channel_rel_error(got, ref)
    print(f"{prec} frame, 65,536 held-out queries: per-channel L2 {e2}, max {em}")
    # the same errors from the device's FP64 validation reduction
    nrm = N.nrc_error_norms(got_d, torch.from_numpy(ref).to("cuda")).cpu().numpy()
    assert np.allclose(np.sqrt(nrm[:, 0] / nrm[:, 1]), e2, rtol=1e-12)
    assert np.array_equal(nrm[:, 2] / nrm[:, 3], em)
    # L2 and max within 1e-2 in both formats.  BF16's training products take
    # each weight as a hi + lo pair of BF16 values: with one BF16 value per
    # weight, the rounding model of this frame reaches 1.14e-2 max-normwise,
    # 1.0e-2 of it from the weights training learns; with the pair it gives
    # 0.57-0.73e-2 (FP16: 2.3e-3).
    assert np.all(e2 <= 1e-2) and np.all(em <= FRAME_MAX_TOL[prec]), (e2, em)
    # the kernels against the rounding model of the same frame
    model = RM.TrainModel(w, prec, loss_scale=c.cfg.loss_scale)
    for idx in O.frame_batches(65536, 4, 16384, 77):
        model.step(e64[idx], y[idx].astype(np.float64))
    assert np.all(l2_err(got, model.predict(q64)) <= MODEL_TOL[prec])


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_train_frame_equals_shuffle_then_indexed_steps(N, prec):
    raw = sd.raw_records(70000, 83)
    y = dev(sd.targets(raw))
    a, _ = make_cache(N, prec)
    b, _ = make_cache(N, prec)
    enc = N.nrc_encode(a, dev(raw), 0)
    la, _ = N.nrc_train_frame(a, enc, y, steps=4, batch=16384, seed=5)
    perm = N.nrc_shuffle(70000, 5)
    lb = []
    for k in range(4):
        l, _ = N.nrc_train_step_indexed(b, enc, y, perm[k * 16384:(k + 1) * 16384].contiguous())
        lb.append(l.item())
    assert la.cpu().tolist() == lb
    assert np.array_equal(a.get_weights(), b.get_weights())


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("n_records", [65536, 70000, 50001])
def test_train_frame_indexed_on_a_side_stream_shuffle_equals_train_frame(N, prec, n_records):
    # The permutation comes from a shuffle enqueued on another stream (ordered
    # by an event), as a renderer overlaps it with the frame's query pass.
    raw = sd.raw_records(n_records, 86)
    y = dev(sd.targets(raw))
    a, _ = make_cache(N, prec)
    b, _ = make_cache(N, prec)
    enc = N.nrc_encode(a, dev(raw), 0)
    la, sa = N.nrc_train_frame(a, enc, y, steps=4, batch=16384, seed=9)
    side = torch.cuda.Stream()
    ready = torch.cuda.Event()
    with torch.cuda.stream(side):
        perm = N.nrc_shuffle(n_records, 9, stream=side.cuda_stream)
        ready.record(side)
    torch.cuda.current_stream().wait_event(ready)
    lb, sb = N.nrc_train_frame_indexed(b, enc, y, perm, steps=4, batch=16384)
    assert torch.equal(la, lb) and torch.equal(sa, sb)
    assert np.array_equal(a.get_weights(), b.get_weights())


def test_train_frame_indexed_rejects_bad_arguments(N):
    c, _ = make_cache(N, "fp16")
    enc = N.nrc_encode(c, dev(sd.raw_records(1000, 87)), 0)
    y = dev(sd.targets(sd.raw_records(1000, 87)))
    with pytest.raises(ValueError):
        N.nrc_train_frame_indexed(c, enc, y, torch.zeros(999, dtype=torch.int32, device="cuda"))
    with pytest.raises(N.NrcError):
        N.nrc_train_frame_indexed(c, enc, y, torch.zeros(1000, dtype=torch.int32, device="cuda"), steps=0)


def test_self_training_targets(N):
    rng = np.random.Generator(np.random.PCG64(84))
    n, nt = 10000, 777
    L = rng.random((n, 3)).astype(np.float32)
    T = rng.random((n, 3)).astype(np.float32)
    tail = rng.random((nt, 3)).astype(np.float32)
    k = rng.integers(0, nt, n).astype(np.int32)
    got = N.nrc_self_training_targets(dev(L), dev(T), dev(tail), dev(k, torch.int32)).cpu().numpy()
    ref = O.self_training_targets(L, T, tail, k)
    # one fused multiply-add in FP32: within one rounding of the exact value
    assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) * 1.0001)


def test_self_training_bad_tail_index_makes_the_step_skip(N):
    n = 256
    L = dev(np.ones((n, 3), np.float32))
    tail = dev(np.ones((4, 3), np.float32))
    k = np.zeros(n, np.int32)
    k[9] = 4                                               # out of range
    tgt = N.nrc_self_training_targets(L, L, tail, dev(k, torch.int32))
    assert torch.isnan(tgt[9]).all() and not torch.isnan(tgt[:9]).any() and not torch.isnan(tgt[10:]).any()
    c, w = make_cache(N, "fp16")
    enc = N.nrc_encode(c, dev(sd.raw_records(n, 85)), 0)
    _, skipped = N.nrc_train_step(c, enc, tgt)
    assert int(skipped.item()) == 1 and np.array_equal(c.get_weights(), w)

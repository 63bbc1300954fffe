"""Method-level properties the paper states, checked on synthetic data through
the C ABI (no scenes are available):

* Sec. 3.3, Eq. 2: queries through the exponential moving average of the
  weights flicker less from frame to frame than queries through the latest
  weights when the training targets are noisy (the paper's temporal-stability
  comparison, here on a static synthetic target with seeded multiplicative
  noise).
* Sec. 5, cheap primitives: replacing the sines of the frequency encoding by
  triangle waves leaves the quality of the fit essentially unchanged.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthdata as sd
from oracle import nrc_oracle as O
from tests.test_gpu_parity import dev, make_cache

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12372_amd.nrc as nrc
    return nrc


def _noisy_frames(n_frames, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    for f in range(n_frames):
        raw = sd.raw_records(n, seed * 1000 + f)
        y = sd.targets(raw) * rng.lognormal(0.0, 0.5, (n, 1)).astype(np.float32)   # per-record noise
        yield raw, y


def test_ema_reduces_frame_to_frame_flicker(N):
    # 160 frames of 4 steps: the bias-corrected average has forgotten the
    # initial fit (0.99^440 < 0.02 at the first measured frame), so what is
    # measured over the last 50 frames is the steady state, where the average
    # averages the per-frame noise of the weights over about 100 steps.
    frames, n, measured = 160, 4 * 2048, 50
    q_raw = dev(sd.raw_records(4096, sd.SEED_HELDOUT))
    flicker = {}
    for alpha in (0.0, 0.99):
        c, _ = make_cache(N, "fp16", ema_alpha=alpha)
        prev, diffs = None, []
        for f, (raw, y) in enumerate(_noisy_frames(frames, n, 5)):
            enc = N.nrc_encode(c, dev(raw))
            N.nrc_train_frame(c, enc, dev(y), steps=4, batch=2048, seed=f)
            if f >= frames - measured - 1:
                pred = N.nrc_forward_raw(c, q_raw).cpu().numpy().astype(np.float64)
                if prev is not None:
                    diffs.append(np.mean(np.abs(pred - prev)) / np.mean(np.abs(pred)))
                prev = pred
        flicker[alpha] = float(np.mean(diffs))
    assert flicker[0.99] < 0.5 * flicker[0.0], flicker


def test_triangle_wave_encoding_fits_as_well_as_sines(N):
    losses = {}
    for preset in (O.PRESET_PAPER, O.PRESET_PAPER_TRI):
        c, _ = make_cache(N, "fp16", preset=preset)
        for f in range(30):
            raw = sd.raw_records(4 * 4096, 700 + f)
            enc = N.nrc_encode(c, dev(raw))
            N.nrc_train_frame(c, enc, dev(sd.targets(raw)), steps=4, batch=4096, seed=f)
        held = sd.raw_records(8192, sd.SEED_HELDOUT)
        pred = N.nrc_forward_raw(c, dev(held)).cpu().numpy().astype(np.float64)
        losses[preset], _ = O.relative_l2(pred, sd.targets(held).astype(np.float64))
    assert losses[O.PRESET_PAPER_TRI] < 1.5 * losses[O.PRESET_PAPER] + 1e-3, losses


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_long_online_training_stays_finite_and_keeps_improving(N, prec):
    # 200 frames of online training (new records each frame, 4 x 16,384 shuffled
    # steps) with the static loss scale of 128: no step is skipped, the outputs
    # stay finite, and the held-out relative L2 after 200 frames is below 2% of
    # that after 10 (measured: 0.113 -> 0.00045 in both formats).
    c, _ = make_cache(N, prec)
    held = sd.raw_records(16384, sd.SEED_HELDOUT)
    held_d, held_y = dev(held), sd.targets(held).astype(np.float64)
    errs = {}
    skipped = 0
    for f in range(200):
        raw = sd.raw_records(65536, 5000 + f)
        enc = N.nrc_encode(c, dev(raw))
        _, sk = N.nrc_train_frame(c, enc, dev(sd.targets(raw)), steps=4, batch=16384, seed=f)
        skipped += int(sk.sum().item())
        if f + 1 in (10, 200):
            pred = N.nrc_forward_raw(c, held_d).cpu().numpy().astype(np.float64)
            assert np.all(np.isfinite(pred))
            errs[f + 1], _ = O.relative_l2(pred, held_y)
    print(f"{prec}: held-out relative L2 after 10 frames {errs[10]:.5f}, after 200 {errs[200]:.5f}")
    assert skipped == 0
    assert errs[200] <= 0.02 * errs[10], errs

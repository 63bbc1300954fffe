"""C ABI checks that need no GPU: exported symbols, configuration and size rules,
and argument validation, which happens before any device call."""
import ctypes
import os
import re

import pytest

import synthdata as sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nrc.h")


@pytest.fixture(scope="module")
def N():
    import paper_2106_12372_amd.nrc as nrc
    return nrc


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nrc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(N):
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(N.lib, name), f"{name} declared in nrc.h but not exported"
    assert sorted(N.EXPORTED) == names


def test_param_count_matches_architecture(N):
    for width, hidden in [(64, 5), (128, 5), (64, 1), (64, 8), (128, 2)]:
        cfg = N.make_config(width=width, n_hidden=hidden)
        assert N.nrc_param_count(cfg) == sd.n_params(width, hidden)
    assert sd.n_params() == 20672


def test_config_validation(N):
    bad = [dict(width=96), dict(n_hidden=0), dict(n_hidden=9), dict(precision=7),
           dict(enc_preset=4), dict(lr=-1.0), dict(beta1=1.0), dict(loss_eps=0.0),
           dict(loss_scale=0.0), dict(precision="fp32", width=128), dict(width=128, n_hidden=6)]
    raw_bad = N.make_config()
    raw_bad.factorize = 2                         # only 0 and 1 are defined
    for kw in bad + [raw_bad]:
        cfg = kw if isinstance(kw, N.nrc_config) else N.make_config(**kw)
        with pytest.raises(N.NrcError) as e:
            N.nrc_cache_bytes(cfg)
        assert e.value.code == N.NRC_EINVAL
        assert N.last_error() != ""


def test_workspace_and_scratch_sizes(N):
    cfg = N.make_config()
    P = 20672
    ws = N.nrc_cache_bytes(cfg)
    assert ws >= 3 * 4 * P + 2 * 42 * 1024
    s1 = N.nrc_train_scratch_bytes(cfg, 16384)
    assert s1 >= 256 * P * 4                      # one weight-gradient partial per 64-record tile
    assert N.nrc_train_scratch_bytes(cfg, 16385) > s1
    assert N.nrc_train_scratch_bytes(N.make_config(precision="fp32"), 1) > 0
    # beyond the largest training batch the size is refused, never wrapped
    assert N.lib.nrc_train_scratch_bytes(ctypes.byref(cfg), (1 << 31) + 1) == 0
    assert N.lib.nrc_train_scratch_bytes(ctypes.byref(cfg), 1 << 62) == 0


def test_create_rejects_bad_workspace_before_device_calls(N):
    cfg = N.make_config()
    h = ctypes.c_void_p()
    rc = N.lib.nrc_cache_create(ctypes.byref(cfg), None, 1 << 20, None, ctypes.byref(h))
    assert rc == N.NRC_EINVAL and "NULL" in N.last_error()
    rc = N.lib.nrc_cache_create(ctypes.byref(cfg), ctypes.c_void_p(4096 + 16), 1 << 20, None, ctypes.byref(h))
    assert rc == N.NRC_EINVAL and "aligned" in N.last_error()
    rc = N.lib.nrc_cache_create(ctypes.byref(cfg), ctypes.c_void_p(4096), 100, None, ctypes.byref(h))
    assert rc == N.NRC_ENOMEM
    rc = N.lib.nrc_cache_create(ctypes.byref(cfg), ctypes.c_void_p(4096), 1 << 20, None, None)
    assert rc == N.NRC_EINVAL


def test_entry_points_reject_null_cache(N):
    P = ctypes.c_void_p
    assert N.lib.nrc_forward(None, P(4096), 10, P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_encode(None, P(4096), 0, 10, P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_train_step(None, P(4096), P(4096), 10, P(4096), 1 << 30, None, None, None) == N.NRC_EINVAL
    assert N.lib.nrc_backward(None, P(4096), None, P(4096), 10, P(4096), 1 << 30, P(4096), None, None) == N.NRC_EINVAL
    assert N.lib.nrc_forward_train(None, P(4096), 10, P(4096), 1 << 30, P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_train_step_noalloc(None, P(4096), P(4096), 10, None, None, None) == N.NRC_EINVAL
    assert N.lib.nrc_cache_destroy(None) == N.NRC_EINVAL
    assert N.lib.nrc_config_default(None) == N.NRC_EINVAL


def test_record_pipeline_rejects_bad_arguments_before_device_calls(N):
    P = ctypes.c_void_p
    assert N.lib.nrc_shuffle_scratch_bytes(65536) == 4096
    assert N.lib.nrc_shuffle(-1, 0, P(4096), P(4096), 4096, None) == N.NRC_EINVAL
    assert N.lib.nrc_shuffle(1 << 31, 0, P(4096), P(4096), 4096, None) == N.NRC_EINVAL
    assert N.lib.nrc_shuffle(0, 0, None, None, 0, None) == N.NRC_OK           # empty: nothing to do
    assert N.lib.nrc_shuffle(10, 0, None, P(4096), 4096, None) == N.NRC_EINVAL
    assert N.lib.nrc_shuffle(10, 0, P(4096), P(4096), 16, None) == N.NRC_ENOMEM
    assert N.lib.nrc_train_step_indexed(None, P(4096), P(4096), P(4096), 10, P(4096), 1 << 30, None, None,
                                        None) == N.NRC_EINVAL
    cfg = N.make_config()
    sb = N.nrc_frame_scratch_bytes(cfg, 65536, 4, 16384)
    assert sb >= 65536 * 4 + N.nrc_train_scratch_bytes(cfg, 16384)
    assert N.nrc_frame_scratch_bytes(cfg, 70000, 4, 16384) > sb                  # the permutation grows
    for args in [(65536, 0, 16384), (65536, 65, 16384), (3, 4, 16384), (65536, 4, 0), (1 << 31, 4, 16384)]:
        assert N.lib.nrc_frame_scratch_bytes(ctypes.byref(cfg), *args) == 0
    assert N.lib.nrc_train_frame(None, P(4096), P(4096), 65536, 4, 16384, 0, P(4096), 1 << 30, P(4096),
                                 P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_train_frame_indexed(None, P(4096), P(4096), P(4096), 65536, 4, 16384, P(4096), 1 << 30,
                                         P(4096), P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_train_frame_raw(None, P(4096), N.NRC_RAW14, P(4096), 65536, 4, 16384, 0, P(4096), 1 << 30,
                                     P(4096), P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_self_training_targets(P(4096), P(4096), P(4096), P(4096), 10, 0, P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_self_training_targets(None, P(4096), P(4096), P(4096), 10, 5, P(4096), None) == N.NRC_EINVAL
    assert N.lib.nrc_self_training_targets(None, None, None, None, 0, 0, None, None) == N.NRC_OK


def test_activation_buffer_size(N):
    # per 64-record tile (32 at width 128 in the matrix-core forms): every
    # hidden layer's activations at the operand precision, plus four floats of
    # network output per record
    for prec, elem in (("fp16", 2), ("bf16", 2), ("fp32", 4)):
        cfg = N.make_config(precision=prec)
        assert N.nrc_act_ws_bytes(cfg, 65536) == 1024 * (5 * 64 * 64 * elem + 64 * 16)
        assert N.nrc_act_ws_bytes(cfg, 65) == 2 * (5 * 64 * 64 * elem + 64 * 16)
        assert N.nrc_act_ws_bytes(cfg, 0) == 0
    cfg = N.make_config(precision="fp16", width=128)
    assert N.nrc_act_ws_bytes(cfg, 64) == 2 * (5 * 128 * 32 * 2 + 32 * 16)
    assert N.lib.nrc_act_ws_bytes(ctypes.byref(cfg), -1) == 0

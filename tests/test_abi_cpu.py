"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the public header declares, validates configurations and
fails cleanly when no gfx950 device is present."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2202_05977_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wskp.h")


def _wskp():
    pytest.importorskip("torch")
    from paper_2202_05977_amd import wskp
    if not os.path.exists(wskp.LIB_PATH):
        pytest.skip("libwskp.so not built")
    return wskp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wskp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("wskp_create", "wskp_destroy", "wskp_denoise", "wskp_denoise_batch",
              "wskp_decode", "wskp_backward", "wskp_workspace_size", "wskp_num_weights"):
        assert n in names


def test_binding_constants_match_the_header():
    """The flag and enum values the binding passes are the header's."""
    wskp = _wskp()
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(WSKP_BATCH_[A-Z_]+)\s+(\d+)u", text))
    assert int(defs["WSKP_BATCH_REVERSE_TILES"]) == wskp.BATCH_REVERSE_TILES
    assert int(defs["WSKP_BATCH_GRAPH"]) == wskp.BATCH_GRAPH
    assert wskp.BATCH_REVERSE_TILES & wskp.BATCH_GRAPH == 0


def test_library_exports_every_declared_symbol():
    wskp = _wskp()
    lib = wskp.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_num_weights_matches_blob():
    wskp = _wskp()
    for cfg in synth.CONFIGS.values():
        assert wskp.wskp_num_weights(cfg) == synth.num_weights(cfg) == synth.make_weights(cfg).size


def test_config_validation():
    wskp = _wskp()
    import dataclasses
    bad = [
        dataclasses.replace(synth.SMALL, kernel_sizes=(3, 4)),       # even size
        dataclasses.replace(synth.SMALL, kernel_sizes=(17,)),        # too large
        dataclasses.replace(synth.SMALL, channels=(16, 24, 64)),     # not a multiple of 16
        dataclasses.replace(synth.SMALL, kernel_sizes=tuple(range(1, 19, 2))),  # M = 9
        dataclasses.replace(synth.SMALL, conv_size=4),               # conv size not 3 or 5
        dataclasses.replace(synth.SMALL, conv_size=7),
    ]
    for cfg in bad:
        assert wskp.wskp_num_weights(cfg) == 0
        with pytest.raises(wskp.WskpError) as ei:
            wskp.wskp_create(cfg, np.zeros(10, np.float32))
        assert ei.value.status == -1


def test_weight_count_mismatch_is_rejected():
    wskp = _wskp()
    blob = synth.make_weights(synth.SMALL)
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_create(synth.SMALL, blob[:-1])
    assert ei.value.status == -1


def test_status_strings():
    wskp = _wskp()
    lib = wskp.lib()
    for s in range(0, -9, -1):
        assert lib.wskp_status_string(s)
    assert lib.wskp_status_string(-99) == b"unknown status"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU driver is present")
def test_create_without_device_fails_cleanly():
    wskp = _wskp()
    blob = synth.make_weights(synth.SMALL)
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_create(synth.SMALL, blob)
    assert ei.value.status == -4


def test_host_e4m3_encoder_matches_library_cast():
    """The host e4m3 encoder (FP8 weights) rounds like torch's float8_e4m3fn
    cast inside the finite range and saturates at +-448 outside it."""
    wskp = _wskp()
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.normal(0, 1, 4000), rng.normal(0, 100, 2000), rng.uniform(-448, 448, 2000),
        np.ldexp(rng.uniform(1, 2, 1000), rng.integers(-12, -5, 1000)),   # subnormal range
        np.array([0.0, -0.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11, 448.0, -448.0,
                  1.0625, 1.1875, 17.0, 19.0, 240.0, 432.0, 440.0, 447.9])]).astype(np.float32)
    got = wskp.wskp_fp8_e4m3_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(got, ref)
    sat = wskp.wskp_fp8_e4m3_encode(np.array([500.0, -1e9, 449.0], np.float32))
    np.testing.assert_array_equal(sat, [0x7E, 0xFE, 0x7E])


def test_binding_rejects_head_with_wrong_channel_count():
    """wskp_decode / wskp_backward index the head record with the handle's
    2M channels; the binding rejects any other channel count before it
    reaches the library (checked here with a registered stand-in handle
    value: the check runs before any device call)."""
    import torch
    wskp = _wskp()
    fake = ctypes.c_void_p(0x1234)
    wskp._handle_M[fake.value] = 5
    try:
        head = torch.zeros(1, 8, 8, 6)
        c = torch.zeros(1, 8, 8, 3)
        with pytest.raises(ValueError, match="expected"):
            wskp.wskp_decode(fake, head, c, None, torch.zeros_like(c))
        with pytest.raises(ValueError, match="expected"):
            wskp.wskp_backward(fake, head, c, None, c, head, c, torch.zeros(16, dtype=torch.uint8))
        with pytest.raises(ValueError, match="unknown handle"):
            wskp.wskp_decode(ctypes.c_void_p(0x5678), torch.zeros(1, 8, 8, 10), c, None, c)
    finally:
        wskp._handle_M.pop(fake.value, None)


def test_fp8_with_5x5_convs_is_unsupported():
    """The FP8 plan runs 3x3 convs only; the check precedes any device use."""
    wskp = _wskp()
    cfg = synth.REPVGG
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_create(cfg, synth.make_weights(cfg), "fp8", act_scales=np.ones(9, np.float32))
    assert ei.value.status == -3


@pytest.mark.parametrize("ci,co,identity,absent", [(3, 3, True, ()), (4, 6, False, ()),
                                                   (5, 5, True, ("w5",)), (2, 3, False, ("w1", "w3"))])
def test_repvgg_merge_matches_the_oracle(ci, co, identity, absent):
    """The library's host-side merge (float32) against the oracle's (float64)
    on the same branch parameters, absent branches included."""
    wskp = _wskp()
    import oracle
    rng = np.random.default_rng(ci * 10 + co)
    br = {}
    for k in (1, 3, 5):
        if f"w{k}" in absent:
            continue
        br[f"w{k}"] = rng.normal(0, 0.5, size=(co, ci, k, k)).astype(np.float32)
        br[f"b{k}"] = rng.uniform(-0.1, 0.1, size=(co,)).astype(np.float32)
    br["identity"] = identity
    w, b = wskp.wskp_repvgg_merge(br, ci, co)
    wo, bo = oracle.repvgg_merge(br, ci, co)
    # at most three float32 terms per element: a few float32 ulps
    np.testing.assert_allclose(w, wo, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(b, bo, rtol=1e-6, atol=1e-7)


def test_repvgg_merge_rejects_bad_arguments():
    wskp = _wskp()
    br = {"w3": np.zeros((2, 3, 3, 3), np.float32), "b3": np.zeros(2, np.float32), "identity": True}
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_repvgg_merge(br, 3, 2)        # identity with cin != cout
    assert ei.value.status == -1
    with pytest.raises(ValueError):
        wskp.wskp_repvgg_merge({"w1": np.zeros((2, 2, 3, 3), np.float32),
                                "b1": np.zeros(2, np.float32)}, 2, 2)   # wrong branch shape
    with pytest.raises(ValueError):
        wskp.wskp_repvgg_merge({"w3": np.zeros((2, 2, 3, 3), np.float32)}, 2, 2)   # bias missing
    # the C entry point itself rejects a half-given branch
    w = np.zeros((2, 2, 3, 3), np.float32)
    out_w = np.empty((2, 2, 5, 5), np.float32)
    out_b = np.empty(2, np.float32)
    st = wskp.lib().wskp_repvgg_merge(2, 2, None, None, w.ctypes.data, None, None, None, 0,
                                      out_w.ctypes.data, out_b.ctypes.data)
    assert st == -1

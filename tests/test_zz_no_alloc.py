"""wskp_denoise_static (no workspace argument, no allocation) against
wskp_denoise through the C ABI: bitwise equal results on two calls in a row,
the second on a smaller frame, and the size limit of the static scratch."""
import numpy as np
import pytest

from paper_2202_05977_amd import synth
from _helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec,sizes", [("bf16", [(720, 1280), (360, 640)]),
                                        ("fp32", [(128, 160), (72, 104)])])
def test_static_scratch_equals_workspace_entry_point(prec, sizes):
    from paper_2202_05977_amd import wskp
    cfg = synth.HD if prec == "bf16" else synth.SMALL
    dn = wskp.Denoiser(cfg, synth.make_weights(cfg, 0), prec)
    for k, (H, W) in enumerate(sizes):
        f = to_dev(synth.make_frame(50 + k, H, W))
        ref = dn(f).clone()
        out = torch.full_like(ref, float("nan"))
        wskp.wskp_denoise_static(dn.h, f["radiance"], f["albedo"], f["normal"], f["depth"], out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (prec, H, W)
    dn.close()


def test_static_scratch_rejects_frames_that_do_not_fit():
    from paper_2202_05977_amd import wskp
    cfg = synth.HD
    dn = wskp.Denoiser(cfg, synth.make_weights(cfg, 0), "fp32")
    H, W = 720, 1280
    assert wskp.wskp_workspace_size(dn.h, [H], [W]) > wskp.wskp_static_scratch_bytes()
    f = to_dev(synth.make_frame(1, H, W))
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(wskp.WskpError) as ei:
        wskp.wskp_denoise_static(dn.h, f["radiance"], f["albedo"], f["normal"], f["depth"], out)
    assert ei.value.status == -6
    dn.close()

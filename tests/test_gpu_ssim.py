"""Structural similarity of the registration (the SSIM section 3 reports for
demons) on the GPU through the C ABI, against the FP64 oracle.  Needs an
MI355X; run with -m gpu.

Bars: the GPU's SSIM against the oracle's SSIM of the oracle-normalised
patterns with the test warped by the GPU's own final field: 2e-5 (FP32
window sums of z-scored values, ~1e-6 per pixel); against the oracle's whole
path 2e-3 (the two fields differ by ~1e-4 px RMS); an identical pair gives
exactly 1 on both sides.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("name,H,W", [("batch_256", 256, 256), ("odd", 180, 203)])
def test_ssim_matches_oracle(E, orc, name, H, W):
    from paper_1907_05993_amd import synth as S
    if name == "odd":
        specs = [S.make_spec(9, i, H, W, mis_deg=(0.0, 4.0)) for i in range(3)]
    else:
        specs = S.workload_specs(name, n=3)
    refs, tests = S.render_batch(specs)
    print(f"ssim: 3 pairs of {H} x {W}", flush=True)
    gp = E.Params(levels=3, iters=(15, 15, 15), roi_size=32)
    op = orc.make_params(levels=3, iters=15, roi_size=32, n_roi=20)
    g = E.Registrar(gp).register(cuda(refs), cuda(tests), want_ssim=True)
    torch.cuda.synchronize()
    gs = g["ssim"].cpu().numpy()
    gf = g["field"].cpu().numpy()
    o = orc.register_batch(refs, tests, op)
    for i in range(3):
        Rn, _ = orc.normalize(refs[i])
        Tn, _ = orc.normalize(tests[i])
        ref_val = orc.ssim(Rn, orc.warp(Tn, gf[i].astype(np.float64)))
        print("  pair %d: GPU %.7f, oracle on the GPU's field %.7f, oracle path %.7f"
              % (i, gs[i], ref_val, o["ssim"][i]))
        assert abs(gs[i] - ref_val) <= 2e-5
        assert abs(gs[i] - o["ssim"][i]) <= 2e-3


def test_ssim_identical_pair_and_xcf_first(E, orc):
    from paper_1907_05993_amd import synth as S
    spec = S.make_spec(98, 0, 128, 128, exact_angle=0.0, strain=0.0)
    ref, _ = S.render_pair(spec)
    print("ssim: identical pair, XCF first pass", flush=True)
    g = E.Registrar(E.Params(levels=3, iters=(10, 10, 10), roi_size=32)).register(
        cuda(ref[None]), cuda(ref[None]), want_ssim=True)
    torch.cuda.synchronize()
    assert g["ssim"].cpu().numpy()[0] == 1.0
    g = E.Registrar(E.Params(levels=3, iters=(10, 10, 10), roi_size=32, first_pass=1)).register(
        cuda(ref[None]), cuda(ref[None]), want_ssim=True)
    torch.cuda.synchronize()
    assert np.isnan(g["ssim"].cpu().numpy()[0])

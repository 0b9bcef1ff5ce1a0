"""Pyramids whose level sizes do not halve evenly, and the paper's own pattern
size and settings (section 3.1: 1244 x 1024 px, pattern centre (0.5, 0.5,
0.5), 7 levels x 25 iterations, no field smoothing), on the GPU against the
FP64 oracle.  Needs an MI355X; run with -m gpu.

Bars: restriction of odd sizes 1e-6 (as for even sizes); whole path with
smoothing: the field RMS 1e-3 px at 10 iterations per level, median / 95th
percentile 2e-3 / 0.05 px at 30, F from a common R_finite 1e-6 (the
pipeline bars for even sizes); without smoothing (the paper's setting) the
field's median only (unsmoothed demons amplify rounding differences in flat
regions by orders of magnitude) and F from a common R_finite to 1e-6.
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


@pytest.mark.parametrize("shape", [(7, 9), (25, 39), (311, 156), (5, 64)])
def test_stage_restrict_odd_sizes(E, orc, shape):
    x = np.random.default_rng(shape[0] * 7 + shape[1]).normal(size=(3,) + shape).astype(np.float32)
    print(f"restrict {shape}", flush=True)
    out = E.stage_restrict(cuda(x)).cpu().numpy()
    assert out.shape == (3, (shape[0] + 1) // 2, (shape[1] + 1) // 2)
    for i in range(3):
        np.testing.assert_allclose(out[i], orc.restrict(x[i].astype(np.float64)), atol=1e-6)


def field_stats(a, b):
    d = np.sqrt(((np.asarray(a, np.float64) - b) ** 2).sum(0))
    return float(np.sqrt((d ** 2).mean())), float(np.median(d)), float(np.percentile(d, 95)), float(d.max())


def _compare(E, orc, refs, tests, gp, op, strict, strips=None):
    reg = E.Registrar(gp)
    for (lh, lw), rows in (strips or {}).items():
        reg.set_strip_height(lh, lw, rows)
    g = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op)
    gf = g["field"].cpu().numpy()
    stats = [field_stats(gf[i], o["field"][i]) for i in range(refs.shape[0])]
    print("  field |du| (rms, median, p95, max):", [tuple("%.1e" % v for v in st) for st in stats])
    for rms, med, p95, mx in stats:
        if strict:
            assert rms <= 1e-3
        else:
            assert med <= 2e-3 and p95 <= 0.05
    assert np.array_equal(g["iters"].cpu().numpy(), o["iters"])
    o2 = orc.register_batch(refs, tests, op, rfin=g["R_finite"].cpu().numpy(), want_field=False)
    dF = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    print("  from the GPU's R_finite: max |dF| %.2e" % dF)
    assert dF <= 1e-6
    return g, o


@pytest.mark.parametrize("iters,strict", [(10, True), (30, False)])
def test_odd_level_sizes_match_oracle(E, orc, iters, strict):
    """200 x 156 px with 4 levels: 200/100/50/25 by 156/78/39/20.  As for even
    sizes, the field bar is the RMS at a depth where the FP32 and FP64
    iterations stay together (10 per level) and the median / 95th percentile
    at a depth where a few pixels drift apart (30 per level)."""
    from paper_1907_05993_amd import synth as S
    specs = [S.make_spec(8, i, 200, 156, mis_deg=(0.0, 4.0)) for i in range(3)]
    refs, tests = S.render_batch(specs)
    print(f"odd level sizes: 3 pairs of 200 x 156, 4 levels x {iters}", flush=True)
    gp = E.Params(levels=4, iters=(iters,) * 4, sigma_px=1.0, roi_size=32, n_roi=20)
    op = orc.make_params(levels=4, iters=iters, sigma=1.0, roi_size=32, n_roi=20)
    _compare(E, orc, refs, tests, gp, op, strict=strict)


@pytest.mark.parametrize("strip,tol", [(64, 0.0), (16, 0.0), (0, 0.0), (64, 0.05)])
def test_wide_level_segments_and_tiles_match_oracle(E, orc, strip, tol):
    """A 700 px wide level 0 (600 x 700 px, 3 levels): the row kernels cut it
    into three column segments of 256 lanes (each writing 238 columns), at
    strips of 64 and 16 rows, or the 2-D tile kernel runs it (strip height 0).
    Every variant meets the oracle's field to the 1e-3 px RMS bar at a depth
    where the FP32 and FP64 iterations stay together.  With a tolerance the
    stop decisions sum the squared update over strips and segments, and the
    iteration counts equal the oracle's."""
    from paper_1907_05993_amd import synth as S
    specs = [S.make_spec(9, i, 600, 700, mis_deg=(0.0, 3.0)) for i in range(2)]
    refs, tests = S.render_batch(specs)
    print(f"wide level: 2 pairs of 600 x 700, 3 levels x 10, level-0 strip height {strip}, tolerance {tol}",
          flush=True)
    gp = E.Params(levels=3, iters=(10,) * 3, sigma_px=1.0, tol_px=tol, roi_size=64, n_roi=20)
    op = orc.make_params(levels=3, iters=10, sigma=1.0, tol=tol, roi_size=64, n_roi=20)
    g, _ = _compare(E, orc, refs, tests, gp, op, strict=True, strips={(600, 700): strip})
    its = g["iters"].cpu().numpy()
    print("  iterations per level (finest first):", its.tolist())
    if tol > 0:
        # a stop on the segmented level itself (level 0), decided from the segment sums
        assert (its[:, 0] < 10).any()


@pytest.mark.parametrize("sigma,iters", [(1.0, 10), (0.0, 25)])
def test_paper_workload_matches_oracle(E, orc, sigma, iters):
    """One 10 deg pair at the paper's size, pattern centre and ROI count, 7
    levels.  With smoothing (10 iterations per level) the field meets the
    median / 95th-percentile bars.  With the paper's settings (no smoothing,
    25 iterations per level) unsmoothed demons is chaotic on these patterns:
    the oracle's own field moves by 0.29 px RMS (24 px at worst) when its
    input is perturbed by 1e-7 relative after only 10 iterations per level,
    so the field is judged against the envelope of FP32 rounding alone: the
    oracle's iteration with FP32 storage and arithmetic (tests/fp32_demons.py)
    on the same pair, whose median, 95th percentile and RMS of |du| against
    the FP64 oracle (two rounding orders, the larger) bound the GPU's median
    and 95th percentile to within 10 times (one pair: a single realisation of
    a chaotic difference; its RMS, set by the few pixels that diverged, is
    printed only);
    and the second pass from a common R_finite (1e-6)."""
    from paper_1907_05993_amd import synth as S
    w = S.WORKLOADS["paper_1244"]
    specs = S.workload_specs("paper_1244", n=1)
    refs, tests = S.render_batch(specs)
    print(f"paper size: 1 pair of 1244 x 1024, 7 levels x {iters}, sigma {sigma}, 101 ROIs of 128", flush=True)
    gp = E.Params(levels=7, iters=(iters,) * 7, sigma_px=sigma, roi_size=w["roi"], n_roi=w["n_roi"], pc=w["pc"])
    op = orc.make_params(levels=7, iters=iters, sigma=sigma, roi_size=w["roi"], n_roi=w["n_roi"], pc=w["pc"])
    g = E.Registrar(gp).register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op)
    rms, med, p95, mx = field_stats(g["field"].cpu().numpy()[0], o["field"][0])
    print("  field |du|: rms %.1e, median %.1e, p95 %.1e, max %.1e" % (rms, med, p95, mx))
    assert med <= 2e-3
    if sigma > 0:
        assert p95 <= 0.05
    else:
        import fp32_demons
        emed, ep95, erms = fp32_demons.envelope(refs, tests, o["field"], levels=7, iters=iters, sigma=0.0)[0]
        print("  FP32 envelope |du|: rms %.1e, median %.1e, p95 %.1e" % (erms, emed, ep95))
        assert med <= 10.0 * emed and p95 <= 10.0 * ep95
    assert np.array_equal(g["iters"].cpu().numpy(), o["iters"])
    o2 = orc.register_batch(refs, tests, op, rfin=g["R_finite"].cpu().numpy(), want_field=False)
    dF = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    print("  from the GPU's R_finite: max |dF| %.2e" % dF)
    assert dF <= 1e-6
    from scipy.spatial.transform import Rotation
    truth = Rotation.from_matrix(np.linalg.svd(specs[0].F)[0] @ np.linalg.svd(specs[0].F)[2]).as_rotvec()
    err = np.linalg.norm(g["rotvec"].cpu().numpy()[0] - truth)
    print("  rotation error %.2e rad (oracle %.2e)" % (err, np.linalg.norm(o["rotvec"][0] - truth)))

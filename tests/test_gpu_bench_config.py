"""The launch configuration the benchmark times, tested as it runs there.

* Two demons iterations per launch with 128-row strips on a batch of 1024
  pairs at 256 x 256 (2 strips per pair: 2048 workgroups per launch, more than
  the device holds at once, so the strips of one pair start at different
  times) equal one iteration per launch bit for bit, with tolerances that
  stop pairs after odd and after even iteration counts.  This is the
  regression test of the stop decision taken while a pair's other strips are
  still owed their recompute of the previous iteration.
* The benchmark's registrars (warm start with the fitted network field and
  the plain method; tolerance 1e-4 px, cap 150 per level, graph replay on,
  strip heights autotuned on the 1024-pair batch of exactly 10 degrees)
  against the FP64 oracle on 16 sampled pairs: the deformation gradient from
  a common R_finite to 1e-6, equal iteration counts, and the field.  At this
  depth (3 x 150) the iteration is chaotic in the noise-dominated pixels, so
  the field's difference is judged against what FP32 rounding alone does:
  the oracle's iteration in float32 (tests/fp32_demons.py, two rounding
  orders, the larger difference per statistic) on the same pairs from the
  same initial field.  Per statistic of |du| (median, 95th percentile, RMS)
  the median over the 16 pairs of the GPU's difference is at most 2 times
  the envelope's, and no pair's median or 95th percentile is above 10 times
  its own envelope's (a single pair's RMS is set by the few pixels where the
  iteration diverged and scatters by more than an order of magnitude between
  FP32 realisations, so it is compared over the pairs only).  The
  oracle starts from the same initial field as the GPU (the fitted network
  field, or zero where the GPU fell back).
Needs an MI355X.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = "paper_1907_05993_amd/weights/warm_cnn_256.bin"
SAMPLE = np.linspace(0, 1023, 16).round().astype(int)


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def params(E, tol, cap=150, warm=False):
    return E.Params(levels=3, iters=(cap,) * 3, sigma_px=1.0, tol_px=tol, roi_size=64, n_roi=20,
                    warm_start=2 if warm else 0, fallback_residual_px=0.5)


def test_fused_128_rows_equal_single_on_1024_pairs(E):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("batch_256", n=1024)
    refs, tests, _ = E.gen_pairs(specs, labels=False)
    seen = set()
    for tol in (0.1, 0.05):
        print(f"case: 1024 pairs 256^2, rows 128, tol {tol}", flush=True)
        outs = []
        for rows in (0, 128):
            reg = E.Registrar(params(E, tol))
            for l in range(3):
                reg.set_strip_height(256 >> l, 256 >> l, 128 >> l if rows == 0 else 128)
                reg.set_fused_height(256 >> l, 256 >> l, rows)
            outs.append({k: v.cpu().numpy() for k, v in reg.register(refs, tests).items() if hasattr(v, "cpu")})
            reg.close()
        a, b = outs
        its = a["iters"]
        print("iterations per level (mean):", its.mean(axis=0).tolist(),
              "odd stops per level:", ((its < 150) & (its % 2 == 1)).sum(axis=0).tolist(),
              "even stops per level:", ((its < 150) & (its % 2 == 0)).sum(axis=0).tolist(), flush=True)
        for v in its[its < 150].ravel():
            seen.add(int(v) % 2)
        for k in ("field", "iters", "status", "F", "q1", "q2", "R_finite"):
            assert np.array_equal(a[k], b[k]), k
    assert seen == {0, 1}


@pytest.fixture(scope="module")
def batch():
    """The benchmark's 1024-pair workload (256 x 256, exactly 10 degrees),
    rendered by the CPU generator so that the oracle's inputs do not come
    from the library."""
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("batch_256_10deg", n=1024)
    refs, tests = S.render_batch(specs)
    return refs, tests


@pytest.mark.parametrize("warm", [True, False])
def test_bench_registrar_matches_oracle_on_16_sampled_pairs(E, orc, batch, warm):
    from oracle import cnn
    refs, tests = batch
    print(f"case: bench registrar, warm={warm}, 1024 pairs, 16 sampled", flush=True)
    reg = E.Registrar(params(E, 1e-4, warm=warm))
    if warm:
        reg.load_model(WEIGHTS)
    reg.set_graphs(True)
    d_refs, d_tests = cuda(refs), cuda(tests)
    tuned = reg.autotune(d_refs, d_tests)
    fused = reg.fused_heights(256, 256)
    print("tuned strip rows:", tuned, "two-iteration strip rows:", fused, flush=True)
    reg.register(d_refs, d_tests, want_field=False)  # graph capture, as the benchmark's warm-up
    g = reg.register(d_refs, d_tests)
    torch.cuda.synchronize()
    st = g["status"].cpu().numpy()[SAMPLE]
    op = orc.make_params(levels=3, iters=150, sigma=1.0, tol=1e-4, roi_size=64, n_roi=20)
    if warm:
        H = W = 256
        pcs = (0.5 * W - 0.5, 0.5 * H - 0.5, 0.7 * W)
        wf = g["warm_field"].cpu().numpy()[SAMPLE].astype(np.float64)
        u0 = np.stack([cnn.warm_init_field(wf[i], H, W, pcs, 2, bool(st[i] & E.WARM_USED)) for i in range(16)])
        o = orc.register_batch(refs[SAMPLE], tests[SAMPLE], op, u_init=u0)
        print("warm used on", int((st & E.WARM_USED != 0).sum()), "of 16 sampled pairs", flush=True)
    else:
        u0 = None
        o = orc.register_batch(refs[SAMPLE], tests[SAMPLE], op)
    import fp32_demons
    gf = g["field"].cpu().numpy()[SAMPLE]
    env = fp32_demons.envelope(refs[SAMPLE], tests[SAMPLE], o["field"], u_init=u0, workers=8, iters=150, tol=1e-4)
    gs = np.array([fp32_demons.field_stats(gf[k], o["field"][k]) for k in range(16)])
    for k in range(16):
        print("pair %4d |du| median %.1e p95 %.1e rms %.1e;  FP32 envelope %.1e %.1e %.1e"
              % ((SAMPLE[k],) + tuple(gs[k]) + tuple(env[k])))
    print("median over pairs: GPU", np.median(gs, 0), "envelope", np.median(env, 0))
    assert np.all(np.median(gs, 0) <= 2.0 * np.median(env, 0))
    assert np.all(gs[:, :2] <= 10.0 * env[:, :2]), (gs / env).round(2).tolist()
    gi = g["iters"].cpu().numpy()[SAMPLE]
    assert np.array_equal(gi, o["iters"])
    rf = g["R_finite"].cpu().numpy()[SAMPLE]
    o2 = orc.register_batch(refs[SAMPLE], tests[SAMPLE], op, rfin=rf, want_field=False)
    dF = np.abs(g["F"].cpu().numpy()[SAMPLE] - o2["F"]).max()
    print("max |dF| from a common R_finite: %.2e" % dF)
    assert dF <= 1e-6
    reg.close()

"""Whole-path parity of the HIP library (through the C ABI) against the FP64
oracle, plus the edge cases of the path.  Needs an MI355X; run with -m gpu.

Bars (FP32 GPU vs FP64 oracle):
  * displacement field: RMS over all pixels <= 1e-3 px while the iteration is
    stable (3 levels x 20-30 iterations).  Deeper, Eq. (1) is chaotic in the
    noise-dominated pixels where |a| ~ |grad R| is small: two FP64 builds of
    the oracle that differ only in FMA contraction already disagree by ~5e-4 px
    RMS and 0.1 px max after 3 x 150 iterations at 256^2.  At full depth the
    tests therefore check (i) that every single step equals the oracle's step
    from the same state (test_gpu_stages.py, teacher forcing), (ii) robust
    field statistics (median and 95th percentile of |du|), and (iii) the
    unique downstream result;
  * deformation gradient: |dF_ij| <= 1e-6 when both second passes start from
    the same R_finite (the GPU's); end to end the difference is bounded by
    1e-4, except for pairs whose second pass is ill-conditioned (a failed
    first pass leaves spurious XCF peaks): there it is bounded by three times
    the oracle's own response to an R_finite change of the observed size;
  * integer outputs (iteration counts, status bits) exact in fixed-count mode.
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


def gen(name, n, start=0):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs(name, n=n, start=start)
    refs, tests = S.render_batch(specs)
    return refs, tests, specs


def params_pair(E, orc, levels=3, iters=100, sigma=1.0, roi=32, tol=0.0, n_roi=20):
    gp = E.Params(levels=levels, iters=(iters,) * levels, sigma_px=sigma, tol_px=tol, roi_size=roi,
                  n_roi=n_roi)
    op = orc.make_params(levels=levels, iters=iters, sigma=sigma, tol=tol, roi_size=roi, n_roi=n_roi)
    return gp, op


def _axis_rotation(axis, angle):
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(np.asarray(axis, np.float64) * angle).as_matrix()


def field_rms(a, b):
    return float(np.sqrt(((np.asarray(a, np.float64) - b) ** 2).mean()))


def field_stats(a, b):
    d = np.sqrt(((np.asarray(a, np.float64) - b) ** 2).sum(0))
    return float(np.sqrt((d ** 2).mean())), float(np.median(d)), float(np.percentile(d, 95)), float(d.max())


def compare(E, orc, refs, tests, gp, op, strict=True, F_tol=1e-6):
    """strict: field RMS <= 1e-3 px; otherwise (chaotic depth) median <= 2e-3
    px and 95th percentile <= 0.05 px."""
    reg = E.Registrar(gp)
    g = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op)
    n = refs.shape[0]
    gf = g["field"].cpu().numpy()
    stats = [field_stats(gf[i], o["field"][i]) for i in range(n)]
    print("field |du| (rms, median, p95, max) per pair:", [tuple("%.1e" % v for v in st) for st in stats])
    for rms, med, p95, mx in stats:
        if strict:
            assert rms <= 1e-3
        else:
            assert med <= 2e-3 and p95 <= 0.05
    assert np.array_equal(g["iters"].cpu().numpy(), o["iters"])
    # second pass from the same R_finite (the GPU's)
    rf = g["R_finite"].cpu().numpy()
    o2 = orc.register_batch(refs, tests, op, rfin=rf, want_field=False)
    dF = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    dq2 = np.abs(g["q2"].cpu().numpy() - o2["q2"]).max()
    print("second pass from GPU R_finite: max |dF| %.2e, max |dq2| %.2e px" % (dF, dq2))
    assert dF <= F_tol
    # end to end: the remaining difference comes from R_finite, whose own
    # difference comes from the (chaotic) demons field.  Bar: 1e-4, or, for a
    # pair whose second pass is ill-conditioned (spurious XCF peaks after a
    # failed first pass), three times the change the oracle's own second pass
    # shows for an R_finite change of the observed size about each axis.
    gF = g["F"].cpu().numpy()
    dF_e2e = np.abs(gF - o["F"]).max(axis=(1, 2))
    dR = np.abs(g["R_finite"].cpu().numpy() - o["Rfin"]).max(axis=(1, 2))
    print("end to end: max |dF| %.2e, max |dR_finite| %.2e" % (dF_e2e.max(), dR.max()))
    if (dF_e2e > 1e-4).any():
        base = orc.register_batch(refs, tests, op, rfin=o["Rfin"], want_field=False)["F"]
        sens = np.zeros(n)
        for ax in np.eye(3):
            rot = np.stack([_axis_rotation(ax, max(dR[i], 1e-9)) for i in range(n)])
            pert = orc.register_batch(refs, tests, op, rfin=np.einsum("nij,njk->nik", rot, o["Rfin"]),
                                      want_field=False)["F"]
            sens = np.maximum(sens, np.abs(pert - base).max(axis=(1, 2)))
        print("second-pass response to the R_finite difference:", ["%.1e" % v for v in sens])
        assert (dF_e2e <= np.maximum(1e-4, 3.0 * sens + 1e-6)).all()
    assert np.array_equal(g["status"].cpu().numpy().astype(np.uint32), o["status"])
    # Eq. (6): the rotation tensor of the GPU's own rotation vector, as the oracle forms it
    om = g["omega"].cpu().numpy()
    rv = g["rotvec"].cpu().numpy()
    for i in range(n):
        np.testing.assert_array_equal(om[i], orc.omega(rv[i]))
    return g, o


def test_single_pair_128_stable_depth(E, orc):
    """Single pair, 128^2, 3 levels x 20 iterations, sigma 1, 20 ROIs of 32^2: strict bar."""
    refs, tests, _ = gen("single_128", 1)
    gp, op = params_pair(E, orc, iters=20, roi=32)
    compare(E, orc, refs, tests, gp, op, strict=True)


def test_single_pair_128_full_depth(E, orc):
    """The single-pair workload as configured: 3 x 100 iterations."""
    refs, tests, _ = gen("single_128", 1)
    gp, op = params_pair(E, orc, iters=100, roi=32)
    compare(E, orc, refs, tests, gp, op, strict=False)


def test_batch_256_stable_depth(E, orc):
    """256^2 pairs (the batch workload's inputs), 3 x 15 iterations, ROIs of 64^2: strict bar."""
    refs, tests, _ = gen("batch_256", 4)
    gp, op = params_pair(E, orc, iters=15, roi=64)
    compare(E, orc, refs, tests, gp, op, strict=True)


def test_batch_256_full_depth(E, orc):
    """256^2 pairs, 3 x 150 (the batch workload's settings) on 4 pairs.

    At this depth the field's difference from the FP64 oracle is bounded by
    what FP32 rounding alone produces: the oracle's iteration with FP32
    storage and arithmetic (tests/fp32_demons.py, the same steps in the same
    order, two rounding orders, the larger difference per statistic) run on
    the same pairs gives the envelope.  Per statistic of |du| (median, 95th
    percentile, RMS over the pixels), the median over the pairs of the GPU's
    difference is at most 2 times the envelope's, and no pair's median or
    95th percentile is above 10 times its own envelope's (a single pair's RMS
    is set by the few pixels where the iteration diverged and scatters by
    more than an order of magnitude between FP32 realisations)."""
    import fp32_demons
    refs, tests, _ = gen("batch_256", 4)
    gp, op = params_pair(E, orc, iters=150, roi=64)
    g, o = compare(E, orc, refs, tests, gp, op, strict=False)
    gf = g["field"].cpu().numpy()
    es = fp32_demons.envelope(refs, tests, o["field"], workers=8, iters=150)
    gs = np.array([fp32_demons.field_stats(gf[i], o["field"][i]) for i in range(4)])
    for i in range(4):
        print("pair %d  |du| GPU vs FP64: median %.1e p95 %.1e rms %.1e;  FP32 envelope: median %.1e p95 %.1e "
              "rms %.1e" % ((i,) + tuple(gs[i]) + tuple(es[i])), flush=True)
    assert np.all(np.median(gs, axis=0) <= 2.0 * np.median(es, axis=0)), (np.median(gs, 0), np.median(es, 0))
    assert np.all(gs[:, :2] <= 10.0 * es[:, :2]), (gs / es).round(2).tolist()


def test_full_batch_1024_sampled(E, orc):
    """The full 1024-pair 256^2 batch in one call (the benchmark's launch
    configuration); 3 sampled pairs are checked against the oracle."""
    refs, tests, _ = gen("batch_256", 1024)
    gp, op = params_pair(E, orc, iters=150, roi=64)
    reg = E.Registrar(gp)
    g = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    idx = [0, 517, 1023]
    o = orc.register_batch(refs[idx], tests[idx], op)
    gf = g["field"][idx].cpu().numpy()
    for k in range(3):
        rms, med, p95, mx = field_stats(gf[k], o["field"][k])
        print("pair", idx[k], "field |du| rms %.1e median %.1e p95 %.1e max %.1e" % (rms, med, p95, mx))
        assert med <= 2e-3 and p95 <= 0.05
    rf = g["R_finite"][idx].cpu().numpy()
    o2 = orc.register_batch(refs[idx], tests[idx], op, rfin=rf, want_field=False)
    assert np.abs(g["F"][idx].cpu().numpy() - o2["F"]).max() <= 1e-6
    # properties that hold for every pair
    F = g["F"].cpu().numpy()
    assert np.allclose(np.linalg.det(F), 1.0, atol=1e-12)
    R = g["R"].cpu().numpy()
    assert np.allclose(np.einsum("nji,njk->nik", R, R), np.eye(3), atol=1e-12)
    assert np.all(g["iters"].cpu().numpy() == 150)


def test_identical_pair_is_exactly_zero(E, orc):
    refs, _, _ = gen("single_128", 2)
    gp, _ = params_pair(E, orc, iters=20)
    g = E.Registrar(gp).register(cuda(refs), cuda(refs))
    torch.cuda.synchronize()
    assert not g["field"].any().item()
    assert not g["q1"].any().item()
    eye = np.broadcast_to(np.eye(3), (2, 3, 3))
    np.testing.assert_allclose(g["F_first"].cpu().numpy(), eye, atol=1e-13)
    # the second pass sees FP32 FFT round-off (|q2| ~ 1e-6 px), i.e. F ~ I + 1e-8
    np.testing.assert_allclose(g["F"].cpu().numpy(), eye, atol=1e-7)
    assert np.abs(g["q2"].cpu().numpy()).max() < 1e-4
    assert np.abs(g["rotvec"].cpu().numpy()).max() < 1e-7
    np.testing.assert_allclose(g["peak_height"].cpu().numpy(), 1.0, atol=1e-5)


def test_degenerate_and_nonfinite_inputs(E, orc):
    refs, tests, _ = gen("single_128", 3)
    tests[1] = 5.0
    tests[2, 10, 10] = np.nan
    gp, _ = params_pair(E, orc, iters=5)
    g = E.Registrar(gp).register(cuda(refs), cuda(tests))
    st = g["status"].cpu().numpy()
    assert st[0] & (orc.DEGENERATE_INPUT | orc.NONFINITE_INPUT) == 0
    assert st[1] & orc.DEGENERATE_INPUT
    assert st[2] & orc.NONFINITE_INPUT
    assert torch.isfinite(g["field"]).all().item()


def test_mixed_sizes_match_separate_calls(E, orc):
    from paper_1907_05993_amd import synth as S
    a = [S.render_pair(S.make_spec(21, i, 128, 128, exact_angle=1.5)) for i in range(2)]
    b = [S.render_pair(S.make_spec(22, i, 160, 96, exact_angle=1.5)) for i in range(2)]
    gp, _ = params_pair(E, orc, iters=30, roi=32)
    reg = E.Registrar(gp)
    order = [a[0], b[0], a[1], b[1]]
    g = reg.register([cuda(p[0]) for p in order], [cuda(p[1]) for p in order])
    ga = reg.register(cuda(np.stack([p[0] for p in a])), cuda(np.stack([p[1] for p in a])))
    gb = reg.register(cuda(np.stack([p[0] for p in b])), cuda(np.stack([p[1] for p in b])))
    torch.cuda.synchronize()
    for k, (src, j) in enumerate([(ga, 0), (gb, 0), (ga, 1), (gb, 1)]):
        assert torch.equal(g["F"][k], src["F"][j])
        assert torch.equal(g["field"][k], src["field"][j])


def test_shared_reference_matches_unshared(E, orc):
    from paper_1907_05993_amd import synth as S
    spec0 = S.make_spec(23, 0, 128, 128, exact_angle=1.0)
    ref, _ = S.render_pair(spec0)
    tests = np.stack([S.render_pair(S.make_spec(23, i, 128, 128, exact_angle=1.0))[1] for i in range(3)])
    refs = np.stack([ref] * 3)
    gp, _ = params_pair(E, orc, iters=30, roi=32)
    reg = E.Registrar(gp)
    r_one = cuda(ref)
    shared = reg.register([r_one] * 3, list(cuda(tests).unbind(0)), ref_ids=[7, 7, 7])
    plain = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    assert torch.equal(shared["field"], plain["field"])
    assert torch.equal(shared["F"], plain["F"])


def test_deterministic(E, orc):
    refs, tests, _ = gen("single_128", 4)
    gp, _ = params_pair(E, orc, iters=40, roi=32, tol=1e-4)
    reg = E.Registrar(gp)
    a = reg.register(cuda(refs), cuda(tests))
    b = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    for k in ("field", "F", "q2", "iters", "status"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("tol", [0.15, 0.03])
def test_tolerance_mode(E, orc, tol):
    """Per-pair convergence.  The RMS update of Eq. (1) on noisy patterns
    plateaus near 1e-2 px (level 0) and 6e-2 px (level 2, full-res px), so
    tol = 0.15 stops every level early and tol = 0.03 stops some levels and
    caps others.  Iteration counts within one of the oracle's, status bits
    consistent with the counts."""
    refs, tests, _ = gen("batch_256", 3)
    gp, op = params_pair(E, orc, iters=150, roi=64, tol=tol)
    g = E.Registrar(gp).register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op)
    gi = g["iters"].cpu().numpy()
    print("iterations GPU", gi.tolist(), "oracle", o["iters"].tolist())
    assert np.abs(gi - o["iters"]).max() <= 1
    assert gi.min() < 150  # early stops happened
    st = g["status"].cpu().numpy().astype(np.uint32)
    for i in range(3):
        conv = np.all(gi[i] < 150)
        assert bool(st[i] & orc.CONVERGED) == conv or not np.array_equal(gi[i], o["iters"][i])
        assert bool(st[i] & orc.HIT_CAP) == (not bool(st[i] & orc.CONVERGED))
    if np.array_equal(gi, o["iters"]):
        assert np.array_equal(st, o["status"])


def test_second_pass_only_entry(E, orc):
    refs, tests, specs = gen("batch_256", 2)
    _, op = params_pair(E, orc, iters=150, roi=64)
    rf = np.stack([orc.polar(s.F) for s in specs])
    gp, _ = params_pair(E, orc, iters=150, roi=64)
    g = E.Registrar(gp).second_pass(cuda(refs), cuda(tests), torch.from_numpy(rf))
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op, rfin=rf, want_field=False)
    assert np.abs(g["F"].cpu().numpy() - o["F"]).max() <= 1e-6
    np.testing.assert_allclose(g["R_finite"].cpu().numpy(), rf, atol=0)


def test_zero_pairs_and_validation(E, orc):
    gp, _ = params_pair(E, orc, iters=5)
    reg = E.Registrar(gp)
    out = reg.register(torch.empty(0, 128, 128, device="cuda"), torch.empty(0, 128, 128, device="cuda"))
    assert out["F"].shape[0] == 0
    # sizes that do not halve evenly are accepted (130 -> 65 -> 33); a coarsest level under 4 px is not
    out = reg.register(cuda(np.zeros((1, 130, 128))), cuda(np.zeros((1, 130, 128))))
    torch.cuda.synchronize()
    assert out["F"].shape[0] == 1
    with pytest.raises(E.EbsdError) as ei:
        reg.register(cuda(np.zeros((1, 12, 128))), cuda(np.zeros((1, 12, 128))))
    assert ei.value.code == -2  # 12 -> 6 -> 3
    with pytest.raises(E.EbsdError) as ei:
        E.Registrar(E.Params(roi_size=128)).register(cuda(np.zeros((1, 128, 128))),
                                                     cuda(np.zeros((1, 128, 128))))
    assert ei.value.code == -3


def test_strip_height_does_not_change_results(E, orc):
    """The autotuner only changes the work decomposition: every strip height
    gives bitwise the same result."""
    refs, tests, _ = gen("batch_256", 2)
    gp, _ = params_pair(E, orc, iters=12, roi=64)
    outs = []
    for rows in (16, 32, 64, 128):
        reg = E.Registrar(gp)
        for l in range(3):
            reg.set_strip_height(256 >> l, 256 >> l, rows)
        outs.append(reg.register(cuda(refs), cuda(tests)))
    tuned = E.Registrar(gp)
    table = tuned.autotune(cuda(refs), cuda(tests))
    assert set(table.values()) <= {16, 32, 64, 128}
    outs.append(tuned.register(cuda(refs), cuda(tests)))
    torch.cuda.synchronize()
    for o in outs[1:]:
        for k in ("field", "F", "iters", "status"):
            assert torch.equal(o[k], outs[0][k]), k


def test_graph_replay_matches_eager(E, orc):
    """Captured-graph replays (new inputs and outputs every call, eager work and
    synchronisations in between) equal direct launches bit for bit."""
    sets = [gen("single_128", 2, start=2 * k) for k in range(3)]
    gp, _ = params_pair(E, orc, iters=25, roi=32, tol=0.03)
    eager = E.Registrar(gp)
    eager.set_graphs(False)
    graph = E.Registrar(gp)
    for rep in range(2):
        for refs, tests, _ in sets:
            a = graph.register(cuda(refs), cuda(tests))
            torch.cuda.synchronize()
            b = eager.register(cuda(refs), cuda(tests))
            torch.cuda.synchronize()
            for k in ("field", "F", "R", "q1", "q2", "peak_height", "iters", "status"):
                assert torch.equal(a[k], b[k]), (rep, k)


def test_tune_cache_file_written_whole_and_read_back(E, tmp_path, monkeypatch):
    """With EBSD_TUNE_CACHE set, an autotune writes the tuned table through a
    temporary file renamed over the cache (no partial file, no temporary left
    behind), and a handle created afterwards starts from that table."""
    from paper_1907_05993_amd import synth as S
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("EBSD_TUNE_CACHE", str(path))
    specs = S.workload_specs("batch_256_10deg", n=64)
    r, t, _ = E.gen_pairs(specs, labels=False)
    p = E.Params(levels=3, iters=(10,) * 3, sigma_px=1.0, roi_size=64, n_roi=20)
    print("case: tune cache, 64 pairs 256^2", flush=True)
    reg = E.Registrar(p)
    tuned = reg.autotune(r, t)
    fused = reg.fused_heights(256, 256)
    reg.close()
    lines = path.read_text().splitlines()
    print("cache:", lines, "tuned:", tuned, "fused:", fused, flush=True)
    assert lines and all(x.split()[0] == "gfx950" and len(x.split()) == 5 for x in lines)
    assert not [q.name for q in tmp_path.iterdir() if q.name != "tune.txt"]
    reg2 = E.Registrar(p)
    for (h, w), ty in tuned.items():
        assert E.lib().ebsd_get_strip_height(reg2._h, h, w) == ty, (h, w)
    assert reg2.fused_heights(256, 256) == fused
    reg2.close()


def test_autotune_on_mixed_sizes_leaves_results_unchanged(E):
    """An autotune over a batch of 128 x 128 and 256 x 256 pairs (two size
    buckets, every level of both timed) changes only the work decomposition:
    the registration afterwards equals an untuned handle's bit for bit."""
    from paper_1907_05993_amd import synth as S
    small = E.gen_pairs([S.make_spec(33, i, 128, 128, mis_deg=(0.0, 8.0)) for i in range(48)], labels=False)
    large = E.gen_pairs([S.make_spec(34, i, 256, 256, mis_deg=(0.0, 8.0)) for i in range(32)], labels=False)
    refs = [small[0][i] for i in range(48)] + [large[0][i] for i in range(32)]
    tests = [small[1][i] for i in range(48)] + [large[1][i] for i in range(32)]
    p = E.Params(levels=3, iters=(20,) * 3, sigma_px=1.0, tol_px=0.05, roi_size=32, n_roi=20)
    print("case: autotune on 48 x 128^2 + 32 x 256^2", flush=True)
    plain = E.Registrar(p)
    a = plain.register(refs, tests)
    tuned = E.Registrar(p)
    tuned.autotune(refs, tests)
    heights = {k: E.lib().ebsd_get_strip_height(tuned._h, *k) for k in [(128, 128), (64, 64), (32, 32), (256, 256)]}
    print("tuned strip heights:", heights, "two-iteration:", tuned.fused_heights(256, 256), tuned.fused_heights(128, 128),
          flush=True)
    b = tuned.register(refs, tests)
    torch.cuda.synchronize()
    for k in ("F", "R", "iters", "status", "q1", "q2", "R_finite"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
    for fa, fb in zip(a["field"], b["field"]):
        assert torch.equal(fa, fb)
    plain.close()
    tuned.close()

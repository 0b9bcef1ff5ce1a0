"""The scan-map and mixed-size stream configurations at their full sizes, in
one registrar each (the launch configuration of a production run): 4096
scan points at 400 x 400 with twelve shared references, and 16384 pairs of
128, 256 and 512 px (40/40/20 %) in uneven calls with the warm start.
Sampled pairs are checked against the FP64 oracle (second pass from the
GPU's R_finite, the deformation-gradient bar 1e-6); properties that hold
for every pair are checked on all of them.  Needs an MI355X."""
import time

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


def check_all(g, n, levels=3):
    """Properties of every pair: det F = 1, R orthonormal with det 1, the
    rotation vector of R, finite outputs, one of CONVERGED / HIT_CAP."""
    F = g["F"].cpu().numpy()
    R = g["R"].cpu().numpy()
    rv = g["rotvec"].cpu().numpy()
    st = g["status"].cpu().numpy().astype(np.uint32)
    assert F.shape == (n, 3, 3) and np.isfinite(F).all() and np.isfinite(rv).all()
    assert np.allclose(np.linalg.det(F), 1.0, atol=1e-12)
    assert np.allclose(np.einsum("nji,njk->nik", R, R), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-12)
    th = np.linalg.norm(rv, axis=1)
    assert np.all(th < 0.5)
    conv, cap = (st & 1) != 0, (st & 2) != 0
    assert np.all(conv ^ cap)
    its = g["iters"].cpu().numpy()
    assert its.shape == (n, levels) and its.min() >= 1 and its.max() <= 150


def test_scan_map_4096_full_size(E, orc):
    """c3: the whole 64 x 64 scan map at 400 x 400, references shared per
    grain, per-pair stopping at 1e-4 px, ROIs of 128."""
    from paper_1907_05993_amd import synth as S
    m = S.scan_map()
    n = m["size"] * m["size"]
    tests, refs, ref_ids = S.scan_specs(400, 400, list(range(n)), smap=m)
    print(f"case: scan map {n} points at 400x400", flush=True)
    _, d_tests, _ = E.gen_pairs(tests, labels=False)
    grains = sorted(refs)
    # the references and the sampled test patterns checked against the oracle come from the
    # CPU generator (the oracle's inputs never come from the library); the rest from the GPU's
    idx = [0, 1337, 2048, 4095]
    d_ref = cuda(np.stack([S.render_pair(refs[k])[0] for k in grains]))
    for i in idx:
        d_tests[i] = cuda(S.render_pair(tests[i])[1])
    slot = {gg: i for i, gg in enumerate(grains)}
    ref_list = [d_ref[slot[gg]] for gg in ref_ids]
    p = E.Params(levels=3, iters=(150,) * 3, sigma_px=1.0, tol_px=1e-4, roi_size=128, n_roi=20)
    reg = E.Registrar(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = reg.register(ref_list, list(d_tests), ref_ids=ref_ids, want_field=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"{n} pairs in {dt:.2f} s ({n / dt:.0f} pairs/s, first call incl. graph capture)")
    check_all(g, n)
    its = g["iters"].cpu().numpy()
    edges = [1, 2, 5, 10, 20, 50, 100, 150, 151]
    for l in range(its.shape[1]):
        hist, _ = np.histogram(its[:, l], bins=edges)
        print("iterations at level %d (bins %s): %s" % (l, edges, hist.tolist()))
    # rotation against the generator's intragranular rotation field
    truth = np.stack([t.extra["rotvec"] for t in tests])
    err = np.linalg.norm(g["rotvec"].cpu().numpy() - truth, axis=1)
    ang = np.degrees(np.linalg.norm(truth, axis=1))
    small = ang < 2.0
    print("rotation error (rad): median %.2e, p95 %.2e; below 2 deg: median %.2e (%d points)"
          % (np.median(err), np.percentile(err, 95), np.median(err[small]), small.sum()))
    assert np.median(err[small]) < 5e-3
    # sampled pairs against the oracle from the same R_finite
    r = np.stack([d_ref[slot[ref_ids[i]]].cpu().numpy() for i in idx])
    t = d_tests[idx].cpu().numpy()
    op = orc.make_params(levels=3, iters=150, sigma=1.0, tol=1e-4, roi_size=128, n_roi=20)
    o2 = orc.register_batch(r, t, op, rfin=g["R_finite"][idx].cpu().numpy(), want_field=False)
    dF = np.abs(g["F"][idx].cpu().numpy() - o2["F"]).max()
    print("sampled pairs %s: max |dF| from a common R_finite %.2e" % (idx, dF))
    assert dF <= 1e-6


def test_mixed_size_stream_16384(E, orc):
    """c5: 16384 pairs of 128, 256 and 512 px (40/40/20 %, 0-12 deg, strain
    +-2e-3) in three uneven calls of mixed sizes, warm start on (fitted
    field, fallback at 0.5 px), per-pair stopping at 1e-4 px, 20 ROIs of 32;
    64 sampled pairs against the oracle."""
    import os
    from paper_1907_05993_amd import synth as S
    rng = np.random.default_rng(55)
    n = 16384
    sizes = rng.choice([128, 256, 512], size=n, p=[0.4, 0.4, 0.2])
    specs = [S.make_spec(5, i, int(N), int(N), mis_deg=(0.0, 12.0), strain=2e-3) for i, N in enumerate(sizes)]
    print(f"case: mixed stream of {n} pairs", flush=True)
    refs = [None] * n
    tests = [None] * n
    for N in (128, 256, 512):
        idx = np.nonzero(sizes == N)[0]
        r, t, _ = E.gen_pairs([specs[i] for i in idx], labels=False)
        for k, i in enumerate(idx):
            refs[i] = r[k]
            tests[i] = t[k]
    # 64 sampled pairs (26 / 26 / 12 of 128 / 256 / 512 px, seeded) are checked against the
    # oracle below; they come from the CPU generator (the oracle's inputs never come from the
    # library)
    rs = np.random.default_rng(56)
    sampled = []
    for N, k in ((128, 26), (256, 26), (512, 12)):
        idx = sorted(rs.choice(np.nonzero(sizes == N)[0], size=k, replace=False).tolist())
        for i in idx:
            r1, t1 = S.render_pair(specs[i])
            refs[i], tests[i] = cuda(r1), cuda(t1)
        sampled.append((N, k, idx))
    weights = os.path.join(os.path.dirname(E.__file__), "weights", "warm_cnn_256.bin")
    p = E.Params(levels=3, iters=(150,) * 3, sigma_px=1.0, tol_px=1e-4, roi_size=32, n_roi=20, warm_start=2)
    reg = E.Registrar(p)
    reg.load_model(weights)
    calls = [(0, 4096), (4096, 11264), (11264, n)]
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in calls:
        outs.append(reg.register(refs[a:b], tests[a:b], want_field=False))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"{n} pairs in {dt:.2f} s ({n / dt:.0f} pairs/s, first calls incl. graph capture)")
    g = {k: torch.cat([o[k] for o in outs]) for k in ("F", "R", "rotvec", "R_finite", "status", "iters")}
    check_all(g, n)
    st = g["status"].cpu().numpy().astype(np.uint32)
    used = (st & 4) != 0
    assert np.all(used ^ ((st & 8) != 0))  # warm start used or fallen back, for every pair
    truth = np.stack([np.linalg.svd(s.F)[0] @ np.linalg.svd(s.F)[2] for s in specs])
    from scipy.spatial.transform import Rotation
    err = np.linalg.norm(g["rotvec"].cpu().numpy() - Rotation.from_matrix(truth).as_rotvec(), axis=1)
    for N in (128, 256, 512):
        e = err[sizes == N]
        print("N=%d: %d pairs, warm start used %.0f%%, rotation error median %.2e p95 %.2e"
              % (N, e.size, 100 * used[sizes == N].mean(), np.median(e), np.percentile(e, 95)))
    # 64 sampled pairs (26 / 26 / 12 of 128 / 256 / 512 px, seeded) against the oracle from the
    # same R_finite: the distribution of the deformation-gradient differences
    dFs = []
    for N, k, idx in sampled:
        r = np.stack([refs[i].cpu().numpy() for i in idx])
        t = np.stack([tests[i].cpu().numpy() for i in idx])
        op = orc.make_params(levels=3, iters=150, sigma=1.0, tol=1e-4, roi_size=32, n_roi=20)
        o2 = orc.register_batch(r, t, op, rfin=g["R_finite"][idx].cpu().numpy(), want_field=False)
        d = np.abs(g["F"][idx].cpu().numpy() - o2["F"]).max(axis=(1, 2))
        print("N=%d, %d sampled pairs: |dF| from a common R_finite median %.1e, max %.1e" % (N, k, np.median(d), d.max()))
        dFs.append(d)
    dFs = np.concatenate(dFs)
    print("64 sampled pairs: |dF| median %.1e, p95 %.1e, max %.1e"
          % (np.median(dFs), np.percentile(dFs, 95), dFs.max()))
    assert dFs.max() <= 1e-6

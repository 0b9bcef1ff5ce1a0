"""Per-pair convergence across launches: with a tolerance, a level's demons
launches go out in chunks and stop once no pair of the size bucket is left
iterating.  Results are bit-identical to issuing every launch to the cap
(graph replay and direct launches, one and two iterations per launch, one
and several size buckets), and the skipped launches are reported.  Needs an
MI355X."""
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


def run(E, refs, tests, tol, chunk, fused, graphs=True, cap=150):
    p = E.Params(levels=3, iters=(cap,) * 3, sigma_px=1.0, tol_px=tol, roi_size=64, n_roi=20)
    reg = E.Registrar(p)
    reg.set_graphs(graphs)
    reg.set_resident(False)
    reg.set_gating(chunk)
    H = refs[0].shape[-1]
    for l in range(3):
        reg.set_fused_height(H >> l, H >> l, fused)
    g = reg.register(refs, tests)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else [t.cpu().numpy() for t in v])
           for k, v in g.items() if torch.is_tensor(v) or k == "field"}
    issued, planned = reg.launch_counts()
    reg.close()
    return out, issued, planned


@pytest.mark.parametrize("fused,graphs", [(0, True), (64, True), (64, False)])
def test_gating_equals_full_sequence(E, fused, graphs):
    from paper_1907_05993_amd import synth as S
    print(f"case: gating, fused rows {fused}, graphs {graphs}", flush=True)
    specs = S.workload_specs("batch_256", n=64)
    refs, tests, _ = E.gen_pairs(specs, labels=False)
    for tol in (0.1, 0.05):
        a, ia, pa = run(E, refs, tests, tol, 0, fused, graphs)
        b, ib, pb = run(E, refs, tests, tol, 4, fused, graphs)
        print(f"  tol {tol}: launches issued {ib.tolist()} of {pb.tolist()} (ungated {ia.tolist()}); "
              f"max iterations per level {a['iters'].max(axis=0).tolist()}", flush=True)
        assert np.array_equal(ia, pa) and np.array_equal(pa, pb)
        for k in ("field", "iters", "status", "F", "q1", "q2", "R_finite"):
            assert np.array_equal(a[k], b[k]), k
        # the level stops within the chunk of its last pair's stop plus the two queued behind
        # that chunk's count: at most 3 chunks of 4 launches past the launch that recorded it
        per_launch = 2 if fused else 1
        last = a["iters"].max(axis=0)
        need = np.where(last < 150, -(-last // per_launch) + 1, pb)  # the launch that records the stop
        assert np.all(ib <= np.minimum(pb, need + 12))
        assert np.all(ib >= np.minimum(pb, need))
        assert (ib < pb).any()


def test_gating_with_several_buckets_and_no_tolerance(E):
    """Two size buckets in one call, each gated on its own pairs; without a
    tolerance every launch is issued."""
    from paper_1907_05993_amd import synth as S
    print("case: gating, two buckets", flush=True)
    a_specs = [S.make_spec(31, i, 128, 128, mis_deg=(0.0, 6.0)) for i in range(6)]
    b_specs = [S.make_spec(32, i, 256, 256, mis_deg=(0.0, 6.0)) for i in range(6)]
    ra, ta, _ = E.gen_pairs(a_specs, labels=False)
    rb, tb, _ = E.gen_pairs(b_specs, labels=False)
    refs = [ra[i] for i in range(6)] + [rb[i] for i in range(6)]
    tests = [ta[i] for i in range(6)] + [tb[i] for i in range(6)]
    p = E.Params(levels=3, iters=(80,) * 3, sigma_px=1.0, tol_px=0.1, roi_size=32, n_roi=20)
    outs = []
    for chunk in (0, 3):
        reg = E.Registrar(p)
        reg.set_resident(False)
        reg.set_gating(chunk)
        g = reg.register(refs, tests)
        torch.cuda.synchronize()
        outs.append((g, reg.launch_counts()))
    (g0, (i0, p0)), (g1, (i1, p1)) = outs
    print("  launches issued", i1.tolist(), "of", p1.tolist())
    for k in ("F", "iters", "status", "q2"):
        assert torch.equal(g0[k], g1[k]), k
    for f0, f1 in zip(g0["field"], g1["field"]):
        assert torch.equal(f0, f1)
    assert (i1 < p1).any() and np.array_equal(i0, p0)
    p0t = E.Params(levels=3, iters=(20,) * 3, sigma_px=1.0, tol_px=0.0, roi_size=32, n_roi=20)
    reg = E.Registrar(p0t)
    reg.set_resident(False)
    reg.register(refs, tests)
    torch.cuda.synchronize()
    ii, pp = reg.launch_counts()
    assert np.array_equal(ii, pp) and np.all(pp == 2 * 20)

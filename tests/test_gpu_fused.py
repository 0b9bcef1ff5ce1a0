"""Two demons iterations per launch (temporal blocking) against one per
launch: identical fields, iteration counts, status bits and deformation
gradients, bit for bit, with fixed iteration counts (odd and even caps) and
with tolerances that stop pairs on odd and on even iterations; and parity
with the FP64 oracle at stable depth.  Needs an MI355X."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def gen(name, n, start=0):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs(name, n=n, start=start)
    return S.render_batch(specs)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run(E, refs, tests, H, W, iters, tol, fused_rows, graphs=True):
    p = E.Params(levels=3, iters=(iters,) * 3, sigma_px=1.0, tol_px=tol, roi_size=64 if H >= 256 else 32, n_roi=20)
    reg = E.Registrar(p)
    reg.set_graphs(graphs)
    for l in range(3):
        if fused_rows != 8 or (W >> l) <= 128:  # 8-row strips on levels at most 128 px wide only
            reg.set_fused_height(H >> l, W >> l, fused_rows)
    out = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}


@pytest.mark.parametrize("name,H,iters,tol", [
    ("batch_256", 256, 7, 0.0), ("batch_256", 256, 8, 0.0),
    ("batch_256", 256, 150, 0.15), ("batch_256", 256, 150, 0.03), ("batch_256", 256, 20, 0.05),
    ("single_128", 128, 9, 0.0), ("single_128", 128, 100, 0.15)])
def test_fused_equals_single(E, name, H, iters, tol):
    print(f"case: fused vs single {name} {H} iters={iters} tol={tol}", flush=True)
    n = 4 if H == 256 else 1
    refs, tests = gen(name, n)
    a = run(E, refs, tests, H, H, iters, tol, 0)
    for rows in (8, 16, 32, 64, 128):
        b = run(E, refs, tests, H, H, iters, tol, rows)
        print("iters per level (single):", a["iters"].tolist(), "status", a["status"].tolist())
        for k in ("field", "iters", "status", "F", "q1", "q2", "R_finite"):
            assert np.array_equal(a[k], b[k]), (k, rows)
    # also without graph replay
    c = run(E, refs, tests, H, H, iters, tol, 64, graphs=False)
    assert np.array_equal(a["field"], c["field"]) and np.array_equal(a["iters"], c["iters"])


@pytest.mark.parametrize("N", [400, 512])
def test_fused_equals_single_wide(E, N):
    """Levels up to 512 px wide (eight wavefronts per row): two iterations
    per launch equal one per launch bit for bit, fixed count and tolerance."""
    from paper_1907_05993_amd import synth as S
    print(f"case: fused vs single {N} px", flush=True)
    specs = [S.make_spec(70, i, N, N, mis_deg=(0.0, 6.0)) for i in range(2)]
    refs, tests = S.render_batch(specs)
    for iters, tol in ((9, 0.0), (60, 0.1)):
        a = run(E, refs, tests, N, N, iters, tol, 0)
        for rows in (16, 64, 128):
            b = run(E, refs, tests, N, N, iters, tol, rows)
            for k in ("field", "iters", "status", "F", "q1", "q2", "R_finite"):
                assert np.array_equal(a[k], b[k]), (k, rows, iters)


def test_fused_stops_on_odd_and_even_iterations(E):
    """The tolerance cases above must include pairs that stop after an odd and
    after an even number of iterations on some level (so both decision paths
    of the two-iteration launch are taken)."""
    refs, tests = gen("batch_256", 4)
    seen = set()
    for tol in (0.15, 0.05, 0.03):
        a = run(E, refs, tests, 256, 256, 150, tol, 128)
        its = a["iters"]
        for v in its[its < 150].ravel():
            seen.add(int(v) % 2)
    print("stop parities seen:", seen)
    assert seen == {0, 1}


def test_fused_matches_oracle_stable_depth(E, orc):
    refs, tests = gen("batch_256", 2)
    g = run(E, refs, tests, 256, 256, 15, 0.0, 64)
    op = orc.make_params(levels=3, iters=15, sigma=1.0, roi_size=64, n_roi=20)
    o = orc.register_batch(refs, tests, op)
    for i in range(2):
        rms = float(np.sqrt(((g["field"][i] - o["field"][i]) ** 2).mean()))
        print("field rms vs oracle %.2e" % rms)
        assert rms <= 1e-3

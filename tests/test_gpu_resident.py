"""Level-resident demons (levels of at most 64 x 64 px iterated in one launch,
one workgroup per pair) against the launch-per-iteration path and the FP64
oracle.  Needs an MI355X; run with -m gpu.

Bars: with a fixed iteration count every output is bit-identical to the
launch-per-iteration path (the per-pixel arithmetic is the same); with a
tolerance, the iteration counts equal the oracle's (the stop decision sums
the squared update in another order, which matters only within rounding of
the tolerance).
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


def run(E, refs, tests, params, resident, graphs=True):
    reg = E.Registrar(params)
    reg.set_resident(resident)
    reg.set_graphs(graphs)
    g = reg.register(cuda(refs), cuda(tests))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in g.items() if not k.startswith("_")}


@pytest.mark.parametrize("name,n,sigma,iters", [("single_128", 1, 1.0, 100), ("batch_256", 6, 1.0, 40),
                                                ("batch_256", 3, 0.0, 25), ("batch_256", 3, 1.3, 30)])
def test_resident_levels_bit_identical(E, orc, name, n, sigma, iters):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs(name, n=n)
    refs, tests = S.render_batch(specs)
    roi = 32 if name == "single_128" else 64
    print(f"resident vs per-iteration launches: {n} pairs of {name}, sigma {sigma}, {iters} iterations", flush=True)
    p = E.Params(levels=3, iters=(iters,) * 3, sigma_px=sigma, roi_size=roi)
    a = run(E, refs, tests, p, True)
    b = run(E, refs, tests, p, False)
    for k in ("field", "F", "q1", "q2", "F_first", "iters", "status", "peak_height"):
        assert np.array_equal(a[k], b[k]), k


def test_resident_tolerance_matches_oracle(E, orc):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("single_128", n=1) + [S.make_spec(4, i, 128, 128, mis_deg=(0.0, 3.0)) for i in range(3)]
    refs, tests = S.render_batch(specs)
    for tol in (0.15, 0.03):
        print(f"resident levels with tolerance {tol}", flush=True)
        p = E.Params(levels=3, iters=(100,) * 3, sigma_px=1.0, tol_px=tol, roi_size=32)
        g = run(E, refs, tests, p, True)
        o = orc.register_batch(refs, tests, orc.make_params(levels=3, iters=100, sigma=1.0, tol=tol, roi_size=32,
                                                            n_roi=20))
        print("  iterations GPU", g["iters"].tolist(), "oracle", o["iters"].tolist())
        assert np.array_equal(g["iters"], o["iters"])
        assert np.array_equal(g["status"].astype(np.uint32), o["status"])


def test_resident_bucket_boundary_and_shared_references(E):
    """The resident levels serve buckets of at most 256 pairs: 257 pairs of
    128 px in one call (every level on the row kernels) against the same pairs
    as 256 + 1 (levels of 64 and 32 px resident), with references shared in
    groups of three (one pyramid per distinct reference) and a tolerance that
    stops some pairs early.  Fields, iteration counts, status and F agree bit
    for bit, except where a stop decision sits within rounding of the
    tolerance (the two paths sum the squared update in different orders):
    then only that pair's counts may differ by one, and there are none here."""
    from paper_1907_05993_amd import synth as S
    n = 257
    specs = S.workload_specs("single_128", n=n)
    ref, test, _ = E.gen_pairs(specs, labels=False)
    ref_ids = [i // 3 for i in range(n)]
    refs = [ref[3 * (i // 3)] for i in range(n)]
    tests = [test[i] for i in range(n)]
    p = E.Params(levels=3, iters=(60,) * 3, sigma_px=1.0, tol_px=0.05, roi_size=32)
    print(f"resident bucket boundary: {n} pairs of 128 px, references shared in threes", flush=True)

    def call(lo, hi):
        reg = E.Registrar(p)
        g = reg.register(refs[lo:hi], tests[lo:hi], ref_ids=ref_ids[lo:hi])
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in g.items() if torch.is_tensor(v)}

    whole = call(0, n)
    parts = [call(0, 256), call(256, n)]
    split = {k: np.concatenate([parts[0][k], parts[1][k]]) for k in whole}
    print("  mean iterations per level", whole["iters"].mean(axis=0).round(2).tolist(),
          "stopped early", int((whole["iters"] < 60).any(axis=1).sum()))
    assert (whole["iters"] < 60).any()
    for k in ("field", "iters", "status", "F", "q1", "q2"):
        assert np.array_equal(whole[k], split[k]), k

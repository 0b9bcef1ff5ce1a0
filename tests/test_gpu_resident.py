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

"""Pipelined registration (ebsd_pipeline_*): batches submitted in turn run on
two or three handles with their own streams, several batches in flight at
once.  Every output of every batch
equals a plain ebsd_register_batch call on the same batch bit for bit: the
warm-started path on the benchmark's patterns (256 x 256, 10 degrees, trained
network), and the plain path with a tolerance that stops pairs (gated level
launches, counts and stop decisions included), batches of two pattern sizes
(plain and warm-started), and scan batches whose grains share references.
Needs an MI355X."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = "paper_1907_05993_amd/weights/warm_cnn_256.bin"
KEYS = ("field", "F", "R", "rotvec", "R_finite", "F_first", "q1", "q2", "peak_height", "iters", "status",
        "mae_first", "mae", "omega", "warm_field", "warm_misfit")


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


@pytest.fixture(scope="module")
def batches(E):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("batch_256_10deg", n=3 * 192)
    refs, tests, _ = E.gen_pairs(specs, labels=False)
    return [(refs[k * 192:(k + 1) * 192].contiguous(), tests[k * 192:(k + 1) * 192].contiguous()) for k in range(3)]


def host(out):
    return {k: out[k].cpu().numpy() for k in KEYS if k in out}


@pytest.mark.parametrize("depth,warm,tol", [(2, True, 1e-4), (3, False, 0.1)])
def test_pipelined_batches_equal_single_calls(E, batches, depth, warm, tol):
    p = E.Params(levels=3, iters=(40,) * 3, sigma_px=1.0, tol_px=tol, roi_size=64, n_roi=20,
                 warm_start=2 if warm else 0, fallback_residual_px=1.0)
    print(f"case: pipeline depth {depth}, warm={warm}, tol {tol}, 3 batches of 192", flush=True)
    reg = E.Registrar(p)
    if warm:
        reg.load_model(WEIGHTS)
    want = [host(reg.register(r, t)) for r, t in batches]
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=depth)
    if warm:
        pl.load_model(WEIGHTS)
    for rep in range(2):  # the second round replays the captured graphs
        outs = [pl.submit(r, t) for r, t in batches]
        pl.wait()
        torch.cuda.synchronize()
        for k, o in enumerate(outs):
            got = host(o)
            assert got.keys() == want[k].keys()
            for key in got:
                assert np.array_equal(got[key], want[k][key], equal_nan=True), (rep, k, key)
    if tol > 0.01:
        its = np.concatenate([w["iters"] for w in want])
        print("pairs stopped before the cap per level:", (its < 40).sum(axis=0).tolist(), flush=True)
        assert (its < 40).any()
    pl.close()


@pytest.mark.parametrize("depth,warm,tol", [(2, False, 0.1), (3, True, 0.05)])
def test_pipelined_mixed_size_batches_equal_single_calls(E, depth, warm, tol):
    """Batches that each hold 128 x 128 and 256 x 256 pairs in an interleaved
    order (two size buckets per call, the warm start resampling the 128 px
    pairs), several in flight: every output equals a single call's."""
    from paper_1907_05993_amd import synth as S
    p = E.Params(levels=3, iters=(30,) * 3, sigma_px=1.0, tol_px=tol, roi_size=32, n_roi=20,
                 warm_start=2 if warm else 0, fallback_residual_px=1.0)
    print(f"case: pipeline depth {depth}, warm={warm}, tol {tol}, 3 mixed batches of 24 x 128^2 + 16 x 256^2",
          flush=True)
    small = E.gen_pairs([S.make_spec(31, i, 128, 128, mis_deg=(0.0, 12.0)) for i in range(72)], labels=False)
    large = E.gen_pairs([S.make_spec(32, i, 256, 256, mis_deg=(0.0, 12.0)) for i in range(48)], labels=False)
    batches = []
    ns = nl = 0
    for k in range(3):
        refs, tests = [], []
        for j in range(40):  # 3 small, 2 large, repeated
            if j % 5 < 3:
                src, i, ns = small, ns, ns + 1
            else:
                src, i, nl = large, nl, nl + 1
            refs.append(src[0][i])
            tests.append(src[1][i])
        batches.append((refs, tests))
    assert ns == 72 and nl == 48

    def host_mixed(out):
        got = {k: out[k].cpu().numpy() for k in KEYS if k in out and k != "field"}
        got["field"] = [f.cpu().numpy() for f in out["field"]]
        return got

    reg = E.Registrar(p)
    if warm:
        reg.load_model(WEIGHTS)
    want = [host_mixed(reg.register(r, t)) for r, t in batches]
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=depth)
    if warm:
        pl.load_model(WEIGHTS)
    outs = [pl.submit(r, t) for r, t in batches]
    pl.wait()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        got = host_mixed(o)
        assert got.keys() == want[k].keys()
        for key in got:
            if key == "field":
                assert len(got[key]) == 40
                for j in range(40):
                    assert np.array_equal(got[key][j], want[k][key][j]), (k, j)
            else:
                assert np.array_equal(got[key], want[k][key], equal_nan=True), (k, key)
    its = np.concatenate([w["iters"] for w in want])
    print("pairs stopped before the cap per level:", (its < 30).sum(axis=0).tolist(), flush=True)
    assert (its < 30).any()
    if warm:
        st = np.concatenate([w["status"] for w in want])
        print("warm start used on", int((st & E.WARM_USED != 0).sum()), "of", st.size, flush=True)
    pl.close()


def test_pipelined_scan_batches_with_shared_references_equal_single_calls(E):
    """Scan points at 400 x 400 whose grains share one reference each (ref_ids:
    one reference pyramid per grain), ROIs of 128, two batches in flight on two
    handles with a stopping tolerance: every output equals a single call's."""
    from paper_1907_05993_amd import synth as S
    m = S.scan_map()
    gid = m["gid"].ravel()
    batches = []
    for pick in ([0, 7, 19, 40], [1, 8, 20, 39]):
        idx = []
        for g in (0, 6, 9):
            idx += [int(i) for i in np.nonzero(gid == g)[0][pick]]
        tests, refs, ref_ids = S.scan_specs(400, 400, idx, smap=m)
        ref_img, test_img = S.render_scan(tests, refs, ref_ids)
        d_ref = {g: torch.from_numpy(r).cuda() for g, r in ref_img.items()}
        batches.append(([d_ref[g] for g in ref_ids], [torch.from_numpy(t).cuda() for t in test_img], list(ref_ids)))
    print("case: pipeline depth 2, 2 scan batches of 12 points at 400^2, 3 shared references each", flush=True)
    p = E.Params(levels=3, iters=(20,) * 3, sigma_px=1.0, tol_px=0.1, roi_size=128, n_roi=20)

    def host_list(out):
        got = {k: out[k].cpu().numpy() for k in KEYS if k in out and k != "field"}
        f = out["field"]
        got["field"] = f.cpu().numpy() if isinstance(f, torch.Tensor) else np.stack([x.cpu().numpy() for x in f])
        return got

    reg = E.Registrar(p)
    want = [host_list(reg.register(r, t, ref_ids=ids)) for r, t, ids in batches]
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=2)
    for rep in range(2):
        outs = [pl.submit(r, t, ref_ids=ids) for r, t, ids in batches]
        pl.wait()
        torch.cuda.synchronize()
        for k, o in enumerate(outs):
            got = host_list(o)
            assert got.keys() == want[k].keys()
            for key in got:
                assert np.array_equal(got[key], want[k][key], equal_nan=True), (rep, k, key)
    its = np.concatenate([w["iters"] for w in want])
    print("pairs stopped before the cap per level:", (its < 20).sum(axis=0).tolist(), flush=True)
    pl.close()


def test_pipelined_growing_batches_equal_single_calls(E, batches):
    """Batches of 8, 48, 192, 16 and 96 pairs in turn on two handles: each
    handle's workspace grows while the other captures and replays graphs for
    new batch sizes; every output equals a single call's."""
    r, t = batches[0]
    sizes = (8, 48, 192, 16, 96)
    p = E.Params(levels=3, iters=(12,) * 3, sigma_px=1.0, tol_px=0.05, roi_size=64, n_roi=20)
    print("case: pipeline depth 2, batches of", sizes, flush=True)
    reg = E.Registrar(p)
    want = [host(reg.register(r[:n].contiguous(), t[:n].contiguous())) for n in sizes]
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=2)
    outs = [pl.submit(r[:n].contiguous(), t[:n].contiguous()) for n in sizes]
    pl.wait()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        got = host(o)
        for key in got:
            assert np.array_equal(got[key], want[k][key], equal_nan=True), (sizes[k], key)
    pl.close()


def test_registrars_in_two_threads_equal_serial_calls(E, batches):
    """Two registrars used at once from two host threads, each on its own
    stream (first calls: workspace growth and graph capture in both threads
    at the same time); each thread's outputs equal a serial call's."""
    import threading
    p = E.Params(levels=3, iters=(15,) * 3, sigma_px=1.0, tol_px=0.05, roi_size=64, n_roi=20)
    print("case: two registrars in two threads, 3 calls each", flush=True)
    want = []
    reg = E.Registrar(p)
    for r, t in batches[:2]:
        want.append(host(reg.register(r, t)))
    torch.cuda.synchronize()
    reg.close()
    got = [[], []]
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            rg = E.Registrar(p)
            with torch.cuda.stream(s):
                for _ in range(3):
                    out = rg.register(*batches[k])
                    s.synchronize()
                    got[k].append(host(out))
            rg.close()
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not errors, errors
    for k in range(2):
        assert len(got[k]) == 3
        for rep, g in enumerate(got[k]):
            for key in g:
                assert np.array_equal(g[key], want[k][key], equal_nan=True), (k, rep, key)


@pytest.mark.parametrize("opts", [dict(first_pass=1), dict(bandpass=(1.0, 20.0), background=(1, 0.0)),
                                  dict(background=(0, 15.0), xcf_passes=2, remap_interp=1)])
def test_pipelined_options_equal_single_calls(E, batches, opts):
    """The path's options through the pipeline: the conventional XCF first pass,
    the pre-filter with the static background correction (the bucket's mean
    test pattern), the dynamic background with two bilinear remap passes."""
    p = E.Params(levels=3, iters=(12,) * 3, sigma_px=1.0, roi_size=64, n_roi=20, **opts)
    print("case: pipeline depth 2, options", opts, flush=True)
    bs = [(r[:64].contiguous(), t[:64].contiguous()) for r, t in batches]
    reg = E.Registrar(p)
    want = [host(reg.register(r, t)) for r, t in bs]
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=2)
    outs = [pl.submit(r, t) for r, t in bs]
    pl.wait()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        got = host(o)
        assert got.keys() == want[k].keys()
        for key in got:
            assert np.array_equal(got[key], want[k][key], equal_nan=True), (k, key)
    pl.close()


def test_pipeline_rejects_bad_batches_at_submission(E, batches):
    pl = E.Pipeline(E.Params(levels=3, iters=(5,) * 3), depth=2)
    r, t = batches[0]
    with pytest.raises(E.EbsdError):
        pl.submit(r[:, :3, :3].contiguous(), t[:, :3, :3].contiguous())  # coarsest level under 4 x 4
    out = pl.submit(r[:4], t[:4])
    empty = pl.submit(r[:0], t[:0])  # an empty batch is a no-op in the queue
    pl.wait()
    assert out["F"].shape == (4, 3, 3)
    assert empty["F"].shape[0] == 0
    pl.close()


def test_bench_pipeline_configuration_on_1024_pairs(E):
    """The headline's configuration: two handles, each autotuned on the 1024-pair
    batch (256 x 256, exactly 10 degrees), graph replay, warm start, 3 x 150
    iterations at 1e-4 px; four batches in flight equal one call at a time."""
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("batch_256_10deg", n=1024)
    refs, tests, _ = E.gen_pairs(specs, labels=False)
    p = E.Params(levels=3, iters=(150,) * 3, sigma_px=1.0, tol_px=1e-4, roi_size=64, n_roi=20, warm_start=2,
                 fallback_residual_px=1.0)
    print("case: pipeline depth 2, 1024 pairs, bench configuration", flush=True)
    reg = E.Registrar(p)
    reg.load_model(WEIGHTS)
    reg.set_graphs(True)
    reg.autotune(refs, tests)
    want = host(reg.register(refs, tests))
    torch.cuda.synchronize()
    reg.close()
    pl = E.Pipeline(p, depth=2)
    pl.load_model(WEIGHTS)
    pl.set_graphs(True)
    tuned = pl.autotune(refs, tests)
    print("strip heights per handle:", tuned, flush=True)
    outs = [pl.submit(refs, tests) for _ in range(4)]
    pl.wait()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        got = host(o)
        for key in got:
            assert np.array_equal(got[key], want[key], equal_nan=True), (k, key)
    pl.close()

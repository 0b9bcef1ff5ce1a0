"""GPU pattern generator (ebsd_gen_pairs) against the CPU generator
(paper_1907_05993_amd/synth.py) and the plain-Python noise references.
Needs an MI355X.

Bars: noise-free patterns within 2 fp32 units of the FP64 CPU rendering
(both render in FP64 and round once; transcendental last-bit differences
remain); labels within 1e-5 px of the exact field; Poisson draws equal to the
Philox4x32-10 + PTRS reference draw for draw (at most 1 in 1000 may differ,
for a uniform within a last-bit of a decision boundary); large samples with
Poisson mean, variance and histogram.
"""
import math
import time

import numpy as np
import pytest
import scipy.stats
import torch

import philox_ref as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def specs_for(n, H, W, cid=50, noise=False, mis=(0.0, 12.0)):
    from paper_1907_05993_amd import synth as S
    return [S.make_spec(cid, i, H, W, mis_deg=mis, strain=2e-3, noise=noise) for i in range(n)]


@pytest.mark.parametrize("H,W", [(256, 256), (128, 128), (64, 256)])
def test_noise_free_patterns_and_labels_match_cpu_generator(E, H, W):
    from paper_1907_05993_amd import synth as S
    print(f"case: gen noise-free {H}x{W}", flush=True)
    specs = specs_for(4, H, W)
    ref, test, label = E.gen_pairs(specs)
    ref, test, label = ref.cpu().numpy(), test.cpu().numpy(), label.cpu().numpy()
    worst = 0.0
    for i, s in enumerate(specs):
        r, t = S.render_pair(s)
        for g, c in ((ref[i], r), (test[i], t)):
            ulps = np.abs(g.astype(np.float64) - c) / np.spacing(np.abs(c).astype(np.float32))
            worst = max(worst, float(ulps.max()))
        geom = S.Geometry(H, W, s.pc)
        gy, gx = np.mgrid[0:H // 4, 0:W // 4].astype(np.float64)
        q = S.true_shift_field(s.F, geom, 4 * gx + 1.5, 4 * gy + 1.5)
        assert np.abs(label[i] - np.moveaxis(q, 0, -1)).max() <= 1e-5
    print("worst difference %.1f fp32 units" % worst)
    assert worst <= 2.0


def flat_specs(n, lam, key0=11):
    from paper_1907_05993_amd import synth as S
    out = []
    for i in range(n):
        s = S.PairSpec(H=32, W=32, G=np.eye(3), F=np.eye(3), gxy=(0.0, 0.0), counts=lam, noise=True,
                       seeds=(key0, i))
        out.append(s)
    return out


def gen_flat(E, specs):
    """Flat patterns (background only, no bands)."""
    from paper_1907_05993_amd import ebsd as Eb
    import ctypes as C
    n = len(specs)
    H, W = specs[0].H, specs[0].W
    arr = (Eb.CGenSpec * n)()
    for i, s in enumerate(specs):
        for j in range(9):
            arr[i].G[j] = float(np.eye(3).ravel()[j])
            arr[i].F[j] = float(np.eye(3).ravel()[j])
        arr[i].counts = s.counts
        arr[i].key[0], arr[i].key[1] = s.seeds
        arr[i].noise = 1
        arr[i].bands = 0
    ref = torch.empty(n, H, W, device="cuda")
    test = torch.empty(n, H, W, device="cuda")
    Eb._check(Eb.lib().ebsd_gen_pairs(arr, n, H, W, 0.5, 0.5, 0.7, Eb._ptr(ref), Eb._ptr(test), None,
                                      Eb._stream()), "ebsd_gen_pairs")
    return ref.cpu().numpy(), test.cpu().numpy()


@pytest.mark.parametrize("lam", [4.5, 37.0, 1e4])
def test_poisson_draws_equal_reference(E, lam):
    print(f"case: poisson exact lam={lam}", flush=True)
    specs = flat_specs(1, lam)
    ref, test = gen_flat(E, specs)
    key = specs[0].seeds
    exp_r = np.array([P.poisson(lam, p, 0, key) for p in range(32 * 32)]).reshape(32, 32)
    exp_t = np.array([P.poisson(lam, p, 1, key) for p in range(32 * 32)]).reshape(32, 32)
    mism = int((ref[0] != exp_r).sum() + (test[0] != exp_t).sum())
    print("mismatches %d of 2048" % mism)
    assert mism <= 2


def test_poisson_statistics_at_scale(E):
    print("case: poisson statistics", flush=True)
    from paper_1907_05993_amd import synth as S
    lam = 1e4
    specs = [S.PairSpec(H=256, W=256, G=np.eye(3), F=np.eye(3), counts=lam, noise=True, seeds=(12, i))
             for i in range(4)]
    ref, test = gen_flat(E, specs)
    x = np.concatenate([ref.ravel(), test.ravel()]).astype(np.float64)
    assert np.all(x == np.round(x))
    n = x.size
    assert abs(x.mean() - lam) <= 4.5 * math.sqrt(lam / n)
    assert abs(x.var() / lam - 1.0) <= 4.5 * math.sqrt(2.0 / n)
    edges = np.unique(np.linspace(lam - 3 * math.sqrt(lam), lam + 3 * math.sqrt(lam), 25).astype(int))
    obs = np.array([((x >= a) & (x < b)).sum() for a, b in zip(edges[:-1], edges[1:])])
    cdf = scipy.stats.poisson.cdf
    expc = np.array([cdf(b - 1, lam) - cdf(a - 1, lam) for a, b in zip(edges[:-1], edges[1:])]) * n
    chi2 = ((obs - expc) ** 2 / expc).sum()
    print("chi2 %.1f over %d bins" % (chi2, len(obs)))
    assert scipy.stats.chi2.sf(chi2, len(obs) - 1) > 1e-4
    # reference and test streams are independent
    a = ref.ravel() - lam
    b = test.ravel() - lam
    rho = float(np.corrcoef(a, b)[0, 1])
    assert abs(rho) <= 4.5 / math.sqrt(a.size)


def test_reproducible_and_keyed(E):
    specs = specs_for(2, 128, 128, noise=True)
    r1, t1, l1 = E.gen_pairs(specs)
    r2, t2, l2 = E.gen_pairs(specs)
    assert torch.equal(r1, r2) and torch.equal(t1, t2) and torch.equal(l1, l2)
    r3, _, _ = E.gen_pairs(specs_for(2, 128, 128, cid=51, noise=True))
    assert not torch.equal(r1, r3)
    # the first pair alone renders the same as inside a batch
    r4, t4, _ = E.gen_pairs(specs[:1])
    assert torch.equal(r4[0], r1[0]) and torch.equal(t4[0], t1[0])


def test_generation_speed(E):
    specs = specs_for(1024, 256, 256, cid=52, noise=True)
    E.gen_pairs(specs[:8])
    torch.cuda.synchronize()
    t = time.perf_counter()
    E.gen_pairs(specs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    print("generated 1024 pairs of 256^2 with labels in %.3f s (%.0f pairs/s)" % (dt, 1024 / dt))

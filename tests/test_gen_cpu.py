"""CPU pins of the generator's noise references (tests/philox_ref.py)."""
import math

import numpy as np
import scipy.stats

import philox_ref as P


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the Random123 library."""
    assert P.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert P.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                           0x6D5451FD)
    assert P.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_uniforms_are_uniform():
    u = np.array([P.uniforms2(p, 0, 0, (7, 9)) for p in range(4000)]).ravel()
    assert u.min() >= 0.0 and u.max() < 1.0
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3


def test_ptrs_reference_has_poisson_statistics():
    for lam in (3.7, 25.0, 1e4):
        x = np.array([P.poisson(lam, p, 1, (3, 5)) for p in range(6000)])
        assert abs(x.mean() - lam) <= 4.5 * math.sqrt(lam / x.size)
        assert abs(x.var() / lam - 1.0) <= 4.5 * math.sqrt(2.0 / x.size) + 1.0 / lam
        # goodness of fit on central bins
        lo, hi = int(max(0, lam - 3 * math.sqrt(lam))), int(lam + 3 * math.sqrt(lam)) + 1
        edges = np.linspace(lo, hi, 12).astype(int)
        edges = np.unique(edges)
        obs = np.array([((x >= a) & (x < b)).sum() for a, b in zip(edges[:-1], edges[1:])])
        exp = np.array([scipy.stats.poisson.cdf(b - 1, lam) - scipy.stats.poisson.cdf(a - 1, lam)
                        for a, b in zip(edges[:-1], edges[1:])]) * x.size
        chi2 = ((obs - exp) ** 2 / exp).sum()
        assert scipy.stats.chi2.sf(chi2, len(obs) - 1) > 1e-4

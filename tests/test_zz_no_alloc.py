"""The allocation-free pre-filter (ebsd_stage_bandpass_static) against the
allocating entry point (ebsd_stage_bandpass), through the C ABI: the same
kernels, so the outputs are equal bit for bit, on two calls in a row (the
second smaller, reusing the device's fixed buffer), and an input larger than
the fixed buffer is refused before anything runs.  Needs an MI355X."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def _patterns(n, H, W, seed):
    """Raw synthetic patterns (counts around 1e4) with a smooth background."""
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:H, 0:W] / max(H, W)
    base = 1e4 * (1.0 + 0.2 * xs - 0.1 * ys)
    return torch.from_numpy((rng.poisson(base[None] * rng.uniform(0.8, 1.2, (n, 1, 1)))).astype(np.float32)).cuda()


@pytest.mark.parametrize("order", ["static_first", "allocating_first"])
def test_static_bandpass_equals_allocating(E, order):
    L = E.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for k, (n, H, W, lo, hi) in enumerate([(6, 300, 256, 1.0, 8.0), (2, 128, 96, 0.0, 4.0)]):
        print(f"case: no-alloc bandpass {order}, call {k}: n={n} {H}x{W} lo={lo} hi={hi}", flush=True)
        x = _patterns(n, H, W, 10 + k)
        a = torch.full_like(x, np.nan)
        b = torch.full_like(x, np.nan)
        calls = [(L.ebsd_stage_bandpass, a), (L.ebsd_stage_bandpass_static, b)]
        if order == "static_first":
            calls.reverse()
        for fn, dst in calls:
            rc = fn(C.c_void_p(x.data_ptr()), n, H, W, C.c_float(lo), C.c_float(hi), C.c_void_p(dst.data_ptr()),
                    stream)
            assert rc == 0, rc
        torch.cuda.synchronize()
        assert torch.isfinite(b).all()
        assert torch.equal(a, b)


def test_static_bandpass_refuses_inputs_over_its_buffer(E):
    L = E.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    x = torch.zeros(17, 512, 512, device="cuda")  # 2 x 17 x 512 x 512 > 8 Mi floats
    out = torch.full_like(x, 7.0)
    rc = L.ebsd_stage_bandpass_static(C.c_void_p(x.data_ptr()), 17, 512, 512, C.c_float(1.0), C.c_float(8.0),
                                      C.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    assert rc == -10
    assert E.lib().ebsd_strerror(-10).decode().startswith("input larger")
    assert (out == 7.0).all()
    # the largest input that fits: 16 x 512 x 512 (2 n H W = 8 Mi floats)
    rc = L.ebsd_stage_bandpass_static(C.c_void_p(x.data_ptr()), 16, 512, 512, C.c_float(1.0), C.c_float(8.0),
                                      C.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    assert rc == 0
    assert (out[:16] == 0.0).all() and (out[16] == 7.0).all()

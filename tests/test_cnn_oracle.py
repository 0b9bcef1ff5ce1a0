"""Pins of the warm-start network oracle (oracle/cnn.py), CPU only.

The FP64 forward pass is compared with the same network assembled from
torch's library operators (conv2d, max_pool2d, nearest interpolation); the
backward pass with torch autograd and with central finite differences of the
oracle's own loss; bfloat16 rounding with torch's conversion; the Adam step
with torch.optim.Adam.  The fallback fit is pinned by fields that follow the
Eq. (2) model exactly and by fields that do not.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from oracle import cnn

TINY = (3, 4, 5, 6)


def tiny_net(seed=0, emulate=False):
    p = cnn.init_params(seed, widths=TINY)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(0, 0.1, size=p[k].shape)
    return cnn.Net(p, emulate=emulate)


def torch_forward(p, x):
    """The same network from torch operators (NCHW, float64)."""
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    h = t(x).permute(0, 3, 1, 2)

    def conv(name, h):
        w = t(p[name + ".w"]).permute(3, 2, 0, 1)  # [3,3,ci,co] -> [co,ci,3,3]
        return torch.relu(Fn.conv2d(h, w, t(p[name + ".b"]), padding=1))

    e1 = conv("c1b", conv("c1a", h))
    e2 = conv("c2b", conv("c2a", Fn.max_pool2d(e1, 2)))
    e3 = conv("c3b", conv("c3a", Fn.max_pool2d(e2, 2)))
    e4 = conv("c4b", conv("c4a", Fn.max_pool2d(e3, 2)))
    cat = torch.cat([Fn.interpolate(e4, scale_factor=2, mode="nearest"), e3], dim=1)
    d2 = conv("d2", conv("d1", cat))
    out = torch.einsum("nchw,co->nhwo", d2, t(p["head.w"])) + t(p["head.b"])
    return out


def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38]])
    # exact halfway cases in float32: low 16 bits = 0x8000, even and odd upper halves
    halves = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40490000 | 0x8000], np.uint32)
              .view(np.float32).astype(np.float64))
    x = np.concatenate([x, halves])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)
    assert cnn.bf16(halves[0]) == 1.0 and cnn.bf16(halves[1]) == np.float32(1.015625)


def test_conv3x3_and_its_gradients_match_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(3, 3, 3, 5))
    b = rng.normal(size=5)
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_()
    wt = torch.from_numpy(w).permute(3, 2, 0, 1).contiguous().requires_grad_()
    yt = Fn.conv2d(xt, wt, torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(cnn.conv3x3(x, w, b), yt.permute(0, 2, 3, 1).detach().numpy(),
                               atol=1e-12)
    g = rng.normal(size=(2, 7, 9, 5))
    yt.backward(torch.from_numpy(g).permute(0, 3, 1, 2))
    np.testing.assert_allclose(cnn.conv3x3_dgrad(g, w), xt.grad.permute(0, 2, 3, 1).numpy(),
                               atol=1e-12)
    np.testing.assert_allclose(cnn.conv3x3_wgrad(x, g), wt.grad.permute(2, 3, 1, 0).numpy(),
                               atol=1e-11)


def test_maxpool_upsample_and_their_gradients_match_torch():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 8, 3))
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_()
    yt = Fn.max_pool2d(xt, 2)
    y, idx = cnn.maxpool2(x)
    np.testing.assert_array_equal(y, yt.permute(0, 2, 3, 1).detach().numpy())
    g = rng.normal(size=y.shape)
    yt.backward(torch.from_numpy(g).permute(0, 3, 1, 2))
    np.testing.assert_array_equal(cnn.maxpool2_back(g, idx, x.shape), xt.grad.permute(0, 2, 3, 1).numpy())
    ut = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_()
    up = Fn.interpolate(ut, scale_factor=2, mode="nearest")
    np.testing.assert_array_equal(cnn.upsample2(x), up.permute(0, 2, 3, 1).detach().numpy())
    g2 = rng.normal(size=(2, 12, 16, 3))
    up.backward(torch.from_numpy(g2).permute(0, 3, 1, 2))
    np.testing.assert_allclose(cnn.upsample2_back(g2), ut.grad.permute(0, 2, 3, 1).numpy(), atol=1e-14)


def test_maxpool_ties_route_to_first_in_scan_order():
    x = np.zeros((1, 2, 2, 3))
    x[0, :, :, 0] = [[1, 1], [1, 1]]      # all tie -> (0,0)
    x[0, :, :, 1] = [[0, 2], [2, 2]]      # -> (0,1)
    x[0, :, :, 2] = [[0, 0], [3, 3]]      # -> (1,0)
    y, idx = cnn.maxpool2(x)
    assert idx[0, 0, 0].tolist() == [0, 1, 2]
    g = cnn.maxpool2_back(np.ones((1, 1, 1, 3)), idx, x.shape)
    assert g[0, 0, 0, 0] == 1 and g[0, 0, 1, 1] == 1 and g[0, 1, 0, 2] == 1 and g.sum() == 3


def test_network_forward_matches_torch_operators():
    net = tiny_net(3)
    x = np.random.default_rng(3).normal(size=(2, 16, 16, 2))
    out, _ = net.forward(x)
    ref = torch_forward(net.p, x).detach().numpy()
    assert out.shape == (2, 4, 4, 2)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_network_backward_matches_torch_autograd():
    net = tiny_net(4)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, 16, 16, 2))
    label = rng.normal(size=(2, 4, 4, 2))
    L, out, g = net.loss_and_grads(x, label)
    tp = {k: torch.from_numpy(v.copy()).requires_grad_() for k, v in net.p.items()}
    # rebuild torch_forward on tensors that carry gradients
    h = torch.from_numpy(x).permute(0, 3, 1, 2)

    def conv(name, h):
        return torch.relu(Fn.conv2d(h, tp[name + ".w"].permute(3, 2, 0, 1), tp[name + ".b"], padding=1))

    e1 = conv("c1b", conv("c1a", h))
    e2 = conv("c2b", conv("c2a", Fn.max_pool2d(e1, 2)))
    e3 = conv("c3b", conv("c3a", Fn.max_pool2d(e2, 2)))
    e4 = conv("c4b", conv("c4a", Fn.max_pool2d(e3, 2)))
    cat = torch.cat([Fn.interpolate(e4, scale_factor=2, mode="nearest"), e3], dim=1)
    d2 = conv("d2", conv("d1", cat))
    o = torch.einsum("nchw,co->nhwo", d2, tp["head.w"]) + tp["head.b"]
    lt = ((o - torch.from_numpy(label)) ** 2).sum(dim=3).mean()
    lt.backward()
    assert abs(L - lt.item()) <= 1e-12 * max(1.0, abs(L))
    for k in net.p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=k)


def test_network_gradients_match_central_differences():
    net = tiny_net(5)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(2, 16, 16, 2))
    label = rng.normal(size=(2, 4, 4, 2))
    _, _, g = net.loss_and_grads(x, label)
    h = 1e-6
    worst = 0.0
    for k in net.p:
        flat = net.p[k].reshape(-1)
        for i in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp = net.loss(net.forward(x)[0], label)[0]
            flat[i] = old - h
            lm = net.loss(net.forward(x)[0], label)[0]
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst < 1e-6


def test_emulated_network_rounds_where_stated():
    """With bf16 emulation the stored activations are bf16 values; the output
    stays within bf16-level error of the exact network."""
    p = cnn.init_params(6, widths=TINY)
    x = np.random.default_rng(6).normal(size=(1, 16, 16, 2))
    out_e, ce = cnn.Net(p, emulate=True).forward(x)
    out_x, _ = cnn.Net(p, emulate=False).forward(x)
    for name in ("e1", "e3", "dec"):
        np.testing.assert_array_equal(ce[name], cnn.bf16(ce[name]))
    rel = np.abs(out_e - out_x).max() / np.abs(out_x).max()
    assert 0 < rel < 0.05


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=50)
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.from_numpy(p0.copy()).requires_grad_()
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        cnn.adam_update(p, g, m, v, t)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)


def test_flatten_roundtrip_and_parameter_count():
    p = cnn.init_params(0)
    vec = cnn.flatten(p)
    assert vec.size == 1762306
    q = cnn.unflatten(vec)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])


def test_grid_points_are_level2_pixel_centres(orc):
    """Restricting a full-resolution ramp twice gives the ramp's value at the
    grid coordinates (the [1,3,3,1]/8 filter is exact on linear functions)."""
    H = W = 32
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    ramp = x + 100.0 * y
    r2 = orc.restrict(orc.restrict(ramp))
    gx, gy = cnn.grid_points(H, W)
    inner = (slice(1, -1), slice(1, -1))  # borders see the clamp
    np.testing.assert_allclose(r2[inner], (gx + 100.0 * gy)[inner], atol=1e-12)


def test_warm_fallback_accepts_model_fields_and_rejects_others():
    from paper_1907_05993_amd import synth as S
    H = W = 256
    pcs = (0.5 * W - 0.5, 0.5 * H - 0.5, 0.7 * W)
    ang = np.radians(7.0)
    F = np.array([[np.cos(ang), -np.sin(ang), 0.0], [np.sin(ang), np.cos(ang), 0.0], [0, 0, 1]])
    F = (np.eye(3) + 1e-3 * np.diag([1.0, -2.0, 1.0])) @ F
    geom = S.Geometry(H, W, (0.5, 0.5, 0.7))
    gx, gy = cnn.grid_points(H, W)
    q = S.true_shift_field(F, geom, gx, gy)          # [2, 64, 64]
    field = np.moveaxis(q, 0, -1)
    use, rms, Ff = cnn.warm_fallback(field, H, W, pcs)
    assert use and rms < 1e-9
    Fn_ = F / np.cbrt(np.linalg.det(F))
    np.testing.assert_allclose(Ff, Fn_, atol=1e-9)
    # independent N(0, s^2) noise on both components: the RMS endpoint misfit
    # is s*sqrt(2) (less a negligible share for the 8 fitted parameters); the
    # decision compares the misfit (full-resolution px) with the threshold
    noise = np.random.default_rng(8).normal(0, 1.0, size=field.shape)
    use2, rms2, _ = cnn.warm_fallback(field + 0.5 * noise, H, W, pcs)
    assert not use2 and abs(rms2 - 0.5 * np.sqrt(2)) < 0.03
    use3, rms3, _ = cnn.warm_fallback(field + 0.25 * noise, H, W, pcs)
    assert use3 and abs(rms3 - 0.25 * np.sqrt(2)) < 0.015
    assert not cnn.warm_fallback(field + 0.25 * noise, H, W, pcs, threshold=0.3)[0]
    # in a resampled frame the misfit is scaled to the registered pattern's px
    assert cnn.warm_fallback(field + 0.25 * noise, H, W, pcs, threshold=0.3, px_scale=0.5)[0]

"""FP64 NumPy oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Only the test suite and the benchmark's CPU leg use this module; the product
never imports it.

Network (the warm start of the demons registration): a 4-level convolutional
encoder-decoder mapping a stacked, normalised (reference, test) pair of
256 x 256 patterns to the displacement field on the 64 x 64 grid of the
coarsest demons level, in full-resolution px:

    enc1  conv3x3 2->32, ReLU, conv3x3 32->32, ReLU            @256^2  -> e1
          maxpool 2x2
    enc2  conv3x3 32->64, ReLU, conv3x3 64->64, ReLU            @128^2  -> e2
          maxpool 2x2
    enc3  conv3x3 64->128, ReLU, conv3x3 128->128, ReLU         @64^2   -> e3
          maxpool 2x2
    enc4  conv3x3 128->256, ReLU, conv3x3 256->256, ReLU        @32^2   -> e4
    dec   nearest upsample e4 to 64^2, concat [up(e4), e3] (384 ch),
          conv3x3 384->128, ReLU, conv3x3 128->128, ReLU, conv1x1 128->2

All 3x3 convolutions use zero padding 1.  Layout is NHWC.  Loss: mean over the
batch and the 64 x 64 grid of the squared endpoint error |u - label|^2.

Precision emulation (emulate=True) mirrors the GPU path: convolution operands
(activations, 3x3 weights, and in the backward pass the pre-activation
gradients) are rounded to bfloat16 (round to nearest even, via float32); all
sums, biases, the 1x1 head and the loss are exact (FP64 here, FP32
accumulation on the GPU).  With emulate=False the whole network is plain
FP64, which the finite-difference pins use.

Max-pooling routes the gradient to the first maximum of each 2 x 2 window in
the order (0,0), (0,1), (1,0), (1,1).
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128, 256)
CONV_NAMES = ("c1a", "c1b", "c2a", "c2b", "c3a", "c3b", "c4a", "c4b", "d1", "d2")


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_shapes(widths=WIDTHS, cin=2):
    """(cin, cout) of every 3x3 convolution, in CONV_NAMES order, and the head."""
    w1, w2, w3, w4 = widths
    convs = [(cin, w1), (w1, w1), (w1, w2), (w2, w2), (w2, w3), (w3, w3), (w3, w4), (w4, w4),
             (w4 + w3, w3), (w3, w3)]
    return dict(zip(CONV_NAMES, convs)), (w3, 2)


def init_params(seed=0, widths=WIDTHS, cin=2):
    """He-normal 3x3 weights [3, 3, cin, cout], zero biases, small head."""
    rng = np.random.default_rng(seed)
    convs, head = layer_shapes(widths, cin)
    p = {}
    for name, (ci, co) in convs.items():
        p[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(3, 3, ci, co))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = rng.normal(0.0, np.sqrt(1.0 / head[0]), size=head)
    p["head.b"] = np.zeros(head[1])
    return p


def conv3x3(x, w, b=None):
    """NHWC zero-padded 3x3 convolution: out[n,y,x,o] = sum w[ky,kx,c,o] x[n,y+ky-1,x+kx-1,c]."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    out = np.zeros((n, h, wd, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + h, kx:kx + wd, :] @ w[ky, kx]
    if b is not None:
        out += b
    return out


def conv3x3_wgrad(x, dz):
    """dW[ky,kx,c,o] = sum_{n,y,x} x[n,y+ky-1,x+kx-1,c] dz[n,y,x,o]."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    dw = np.zeros((3, 3, c, dz.shape[3]))
    dzf = dz.reshape(-1, dz.shape[3])
    for ky in range(3):
        for kx in range(3):
            dw[ky, kx] = xp[:, ky:ky + h, kx:kx + wd, :].reshape(-1, c).T @ dzf
    return dw


def conv3x3_dgrad(dz, w):
    """dX[n,y,x,c] = sum_{ky,kx,o} dz[n,y-ky+1,x-kx+1,o] w[ky,kx,c,o]."""
    n, h, wd, o = dz.shape
    dzp = np.zeros((n, h + 2, wd + 2, o))
    dzp[:, 1:-1, 1:-1, :] = dz
    dx = np.zeros((n, h, wd, w.shape[2]))
    for ky in range(3):
        for kx in range(3):
            # dz at (y - ky + 1) is dzp at (y - ky + 2)
            dx += dzp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + wd, :] @ w[ky, kx].T
    return dx


def maxpool2(x):
    """2x2 max pooling; also returns the index (0..3) of the first maximum."""
    n, h, w, c = x.shape
    v = np.stack([x[:, 0::2, 0::2], x[:, 0::2, 1::2], x[:, 1::2, 0::2], x[:, 1::2, 1::2]])
    idx = np.argmax(v, axis=0)  # first maximum in the order above
    return np.take_along_axis(v, idx[None], axis=0)[0], idx


def maxpool2_back(g, idx, shape):
    out = np.zeros(shape)
    for k, (dy, dx) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        out[:, dy::2, dx::2] += np.where(idx == k, g, 0.0)
    return out


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_back(g):
    return g[:, 0::2, 0::2] + g[:, 0::2, 1::2] + g[:, 1::2, 0::2] + g[:, 1::2, 1::2]


class Net:
    def __init__(self, params, emulate=True):
        self.p = params
        self.emulate = emulate

    def _r(self, x):
        return bf16(x) if self.emulate else np.asarray(x, np.float64)

    def _conv_relu(self, name, x, cache):
        w = self._r(self.p[name + ".w"])
        z = conv3x3(x, w, self.p[name + ".b"])
        a = self._r(np.maximum(z, 0.0))
        cache[name] = (x, w, a)
        return a

    def forward(self, inp):
        """inp: [n, H, W, 2] normalised (ref, test).  Returns (field [n, H/4, W/4, 2], cache)."""
        c = {}
        x = self._r(inp)
        e1 = self._conv_relu("c1b", self._conv_relu("c1a", x, c), c)
        p1, i1 = maxpool2(e1)
        e2 = self._conv_relu("c2b", self._conv_relu("c2a", p1, c), c)
        p2, i2 = maxpool2(e2)
        e3 = self._conv_relu("c3b", self._conv_relu("c3a", p2, c), c)
        p3, i3 = maxpool2(e3)
        e4 = self._conv_relu("c4b", self._conv_relu("c4a", p3, c), c)
        cat = np.concatenate([upsample2(e4), e3], axis=3)
        d2 = self._conv_relu("d2", self._conv_relu("d1", cat, c), c)
        out = d2 @ self.p["head.w"] + self.p["head.b"]
        c.update(i1=i1, i2=i2, i3=i3, e1=e1, e2=e2, e3=e3, e4=e4, dec=d2)
        return out, c

    @staticmethod
    def loss(out, label):
        """Mean squared endpoint error and its gradient w.r.t. out."""
        d = out - label
        m = out.shape[0] * out.shape[1] * out.shape[2]
        return float((d ** 2).sum() / m), 2.0 * d / m

    def _conv_back(self, name, g, grads):
        x, w, a = self.cache[name]
        dz = g * (a > 0)
        grads[name + ".b"] = dz.sum(axis=(0, 1, 2))
        dzr = self._r(dz)
        grads[name + ".w"] = conv3x3_wgrad(x, dzr)
        return conv3x3_dgrad(dzr, w)

    def backward(self, gout):
        """Gradients of all parameters for d(loss)/d(out) = gout."""
        c = self.cache
        g = {}
        d2 = c["dec"]
        g["head.w"] = d2.reshape(-1, d2.shape[3]).T @ gout.reshape(-1, gout.shape[3])
        g["head.b"] = gout.sum(axis=(0, 1, 2))
        gd2 = gout @ self.p["head.w"].T
        gcat = self._conv_back("d1", self._conv_back("d2", gd2, g), g)
        w4 = c["e4"].shape[3]
        ge4 = upsample2_back(gcat[..., :w4])
        ge3 = gcat[..., w4:]
        gp3 = self._conv_back("c4a", self._conv_back("c4b", ge4, g), g)
        ge3 = ge3 + maxpool2_back(gp3, c["i3"], c["e3"].shape)
        gp2 = self._conv_back("c3a", self._conv_back("c3b", ge3, g), g)
        ge2 = maxpool2_back(gp2, c["i2"], c["e2"].shape)
        gp1 = self._conv_back("c2a", self._conv_back("c2b", ge2, g), g)
        ge1 = maxpool2_back(gp1, c["i1"], c["e1"].shape)
        self._conv_back("c1a", self._conv_back("c1b", ge1, g), g)
        return g

    def loss_and_grads(self, inp, label):
        out, self.cache = self.forward(inp)
        L, gout = self.loss(out, label)
        return L, out, self.backward(gout)


# -- training step -----------------------------------------------------------------------

def adam_update(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) on arrays, in place; t counts from 1."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p -= lr * mhat / (np.sqrt(vhat) + eps)


def flat_names(widths=WIDTHS):
    """Parameter names in the order of the flat parameter vector."""
    names = []
    for n in CONV_NAMES:
        names += [n + ".w", n + ".b"]
    return names + ["head.w", "head.b"]


def flatten(p, widths=WIDTHS):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in flat_names(widths)])


def unflatten(vec, widths=WIDTHS, cin=2):
    convs, head = layer_shapes(widths, cin)
    shapes = {}
    for n, (ci, co) in convs.items():
        shapes[n + ".w"] = (3, 3, ci, co)
        shapes[n + ".b"] = (co,)
    shapes["head.w"] = head
    shapes["head.b"] = (head[1],)
    out, o = {}, 0
    for k in flat_names(widths):
        s = shapes[k]
        sz = int(np.prod(s))
        out[k] = np.asarray(vec[o:o + sz], np.float64).reshape(s)
        o += sz
    assert o == len(vec)
    return out


# -- warm-start field and its fallback rule ------------------------------------------------

def grid_points(H, W):
    """Full-resolution coordinates of the coarsest (H/4 x W/4) demons grid.

    With the [1,3,3,1]/8 restriction, pixel i of level l sits at full-resolution
    coordinate 2^l i + (2^l - 1)/2, i.e. 4i + 1.5 at level 2."""
    ys, xs = np.mgrid[0:H // 4, 0:W // 4].astype(np.float64)
    return 4.0 * xs + 1.5, 4.0 * ys + 1.5


def warm_fallback(field, H, W, pcs, radius_frac=0.3, threshold=0.5, px_scale=1.0):
    """Fit the Eq. (2) model to a predicted coarse field and decide its use.

    field: [H/4, W/4, 2] (x, y) shifts in full-resolution px at the grid points.
    The fit uses the grid points within radius_frac * W of the pattern centre
    and the Eq. (3) solver (DLT start, Gauss-Newton, det F = 1).  The RMS
    distance between the fitted model's shifts and the predicted shifts is
    the misfit (px of H x W); the field is used when the misfit in
    full-resolution px of the registered pattern (misfit x px_scale: the
    pattern's size over H when the fit runs in a resampled frame) is at most
    threshold.  Returns (use, rms_misfit_px, F).
    """
    import oracle
    xs, ys = grid_points(H, W)
    sel = (xs - pcs[0]) ** 2 + (ys - pcs[1]) ** 2 <= (radius_frac * W) ** 2
    cx, cy = xs[sel], ys[sel]
    q = np.asarray(field, np.float64)[sel]
    F, _ = oracle.solve_F(q, cx, cy, pcs)
    r = np.stack([cx - pcs[0], cy - pcs[1], np.full_like(cx, pcs[2])])
    v = F @ r
    px = pcs[0] + pcs[2] * v[0] / v[2]
    py = pcs[1] + pcs[2] * v[1] / v[2]
    d2 = (px - cx - q[:, 0]) ** 2 + (py - cy - q[:, 1]) ** 2
    rms = float(np.sqrt(d2.mean()))
    return rms * px_scale <= threshold, rms, F


def warm_init_field(field, H, W, pcs, mode, use, levels=3):
    """Coarsest-level initial field of the warm start (units: coarsest-level px).

    field: [H/4, W/4, 2] predicted shifts (full-resolution px); mode 1 starts
    demons from the prediction itself, mode 2 from the Eq. (2) model fitted to
    it (warm_fallback's F evaluated at the grid points); use = False gives the
    zero field of the fallback.  Returns [2, H/4, W/4].
    """
    f = np.asarray(field, np.float64)
    u0 = np.zeros((2, H // 4, W // 4))
    if not use:
        return u0
    if mode == 1:
        u0[:] = np.moveaxis(f, -1, 0)
    else:
        _, _, Ff = warm_fallback(f, H, W, pcs, threshold=np.inf)
        gx, gy = grid_points(H, W)
        r = np.stack([gx - pcs[0], gy - pcs[1], np.full_like(gx, pcs[2])])
        v = np.einsum("ij,jhw->ihw", Ff, r)
        u0[0] = pcs[0] + pcs[2] * v[0] / v[2] - gx
        u0[1] = pcs[1] + pcs[2] * v[1] / v[2] - gy
    return u0 / 2 ** (levels - 1)

"""The oracle's multi-resolution demons iteration with FP32 storage and FP32
arithmetic (NumPy float32).

Test infrastructure: the test suite and the benchmark's parity check use it;
the product never does.  It is kept apart from the FP64 oracle on purpose.

The FP64 oracle (oracle/ebsd_oracle.c) takes each step of section 1's
multi-resolution demons and Eq. (1) in the paper's order; this module takes
the same steps in the same order, but every image, field and intermediate is
a float32 and every operation rounds to float32 (normalisation statistics
excepted: they are FP64, as on the GPU).  It shares no code with the library.

Its purpose is the size of the difference that FP32 rounding alone makes after
many iterations: Eq. (1)'s update is ill-conditioned in noise-dominated pixels
(|R - T(x + u)| and |grad R| both small), so two correct implementations that
round differently drift apart with depth.  The GPU's difference from the FP64
oracle at full depth is judged against this module's difference from it.
"""
import os

import numpy as np

f32 = np.float32


def normalize(p):
    """z-score with FP64 statistics (population std), stored as float32."""
    d = np.asarray(p, np.float64)
    m = d.mean()
    sd = np.sqrt(((d - m) ** 2).mean())
    return ((d - m) / sd).astype(f32)


def restrict(img):
    """Factor-2 [1,3,3,1]/8 restriction with clamped borders (sizes halve rounding up)."""
    def along(a, axis):
        n = a.shape[axis]
        i = np.arange((n + 1) // 2)
        take = lambda k: np.take(a, np.clip(k, 0, n - 1), axis=axis)
        return (take(2 * i - 1) + f32(3) * take(2 * i) + f32(3) * take(2 * i + 1) + take(2 * i + 2)) / f32(8)
    return along(along(img, 1), 0)


def gradient(f):
    """Central differences, one-sided on the border (numpy.gradient's rule)."""
    gx = np.empty_like(f)
    gy = np.empty_like(f)
    gx[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / f32(2)
    gx[:, 0] = f[:, 1] - f[:, 0]
    gx[:, -1] = f[:, -1] - f[:, -2]
    gy[1:-1] = (f[2:] - f[:-2]) / f32(2)
    gy[0] = f[1] - f[0]
    gy[-1] = f[-1] - f[-2]
    return gx, gy


def bilinear(img, x, y):
    """Bilinear samples at (x, y), coordinates clamped to the image before the floor."""
    H, W = img.shape
    xc = np.clip(x, f32(0), f32(W - 1))
    yc = np.clip(y, f32(0), f32(H - 1))
    x0 = np.floor(xc).astype(np.int64)
    y0 = np.floor(yc).astype(np.int64)
    fx = xc - x0.astype(f32)
    fy = yc - y0.astype(f32)
    dx = (x0 + 1 < W).astype(np.int64)  # the right neighbour, clamped
    dy = np.where(y0 + 1 < H, W, 0)
    flat = img.ravel()
    i00 = y0 * W + x0
    one = f32(1)
    top = (one - fx) * flat.take(i00) + fx * flat.take(i00 + dx)
    bot = (one - fx) * flat.take(i00 + dy) + fx * flat.take(i00 + dy + dx)
    return (one - fy) * top + fy * bot


def taps(sigma):
    r = int(np.floor(3.0 * sigma + 0.5))
    w = np.exp(-np.arange(-r, r + 1, dtype=np.float64) ** 2 / (2.0 * sigma * sigma))
    return (w / w.sum()).astype(f32), r


def smooth(v, w, r, cols_first=False):
    """Separable Gaussian with replicated borders: rows, then columns (or the
    other way round: the same sum rounded in another order)."""
    H, W = v.shape

    def along(a, axis):
        # a[.., clamp(i + j), ..] for j = -r..r as slices of the edge-replicated array
        pad = [(0, 0), (0, 0)]
        pad[axis] = (r, r)
        ap = np.pad(a, pad, mode="edge")
        n = a.shape[axis]
        acc = np.zeros_like(a)
        for j in range(-r, r + 1):
            sl = ap[:, r + j:r + j + n] if axis == 1 else ap[r + j:r + j + n, :]
            acc = acc + w[j + r] * sl
        return acc

    if cols_first:
        return along(along(v, 0), 1)
    return along(along(v, 1), 0)


def demons_iter(R, T, gx, gy, u, w, r, cols_first=False):
    """One Eq. (1) step on the accumulated field, then its smoothing; returns
    (u_new, RMS of the update)."""
    H, W = R.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(f32)
    wv = bilinear(T, xs + u[0], ys + u[1])
    a = R - wv
    den = gx * gx + gy * gy + a * a
    ok = den > f32(1e-9)
    safe = np.where(ok, den, f32(1))
    dux = np.where(ok, a * gx / safe, f32(0))
    duy = np.where(ok, a * gy / safe, f32(0))
    v = np.stack([u[0] + dux, u[1] + duy])
    un = np.stack([smooth(v[0], w, r, cols_first), smooth(v[1], w, r, cols_first)]) if r > 0 else v
    d = (un - u).astype(np.float64)
    return un, float(np.sqrt((d ** 2).sum(axis=0).mean()))


def prolong(u, H, W):
    """x2 bilinear on the half-pixel map (fine i -> coarse (i - 0.5) / 2), values doubled."""
    ys, xs = np.mgrid[0:H, 0:W]
    x = (xs.astype(f32) - f32(0.5)) / f32(2)
    y = (ys.astype(f32) - f32(0.5)) / f32(2)
    return np.stack([f32(2) * bilinear(u[c], x, y) for c in range(2)])


def demons(ref, test, levels=3, iters=150, sigma=1.0, tol=0.0, u_init=None, cols_first=False):
    """Multi-resolution demons of one pair; returns (field [2, H, W] float32,
    iteration counts per level, finest first).  u_init: coarsest-level
    initial field [2, h, w] in that level's px.  cols_first: smooth columns
    before rows (another FP32 rounding order of the same iteration)."""
    R = [normalize(ref)]
    T = [normalize(test)]
    for _ in range(1, levels):
        R.append(restrict(R[-1]))
        T.append(restrict(T[-1]))
    w, r = taps(sigma) if sigma > 0 else (None, 0)
    hc, wc = R[-1].shape
    u = np.zeros((2, hc, wc), f32) if u_init is None else np.asarray(u_init, f32).copy()
    its = [0] * levels
    caps = [iters] * levels if np.isscalar(iters) else list(iters)
    for l in range(levels - 1, -1, -1):
        gx, gy = gradient(R[l])
        k = 0
        while k < caps[l]:
            u, rms = demons_iter(R[l], T[l], gx, gy, u, w, r, cols_first)
            k += 1
            if tol > 0 and (1 << l) * rms < tol:
                break
        its[l] = k
        if l > 0:
            u = prolong(u, *R[l - 1].shape)
    return u, its


def field_stats(a, b):
    """(median, 95th percentile, RMS) over the pixels of |a - b| (field vectors)."""
    d = np.sqrt(((np.asarray(a, np.float64) - b) ** 2).sum(0))
    return float(np.median(d)), float(np.percentile(d, 95)), float(np.sqrt((d ** 2).mean()))


def _cases(refs, tests, fields64, u_init, cases, kw):
    """field_stats of the FP32 run for each (pair, cols_first) case."""
    out = []
    for i, cf in cases:
        u, _ = demons(refs[i], tests[i], u_init=None if u_init is None else u_init[i], cols_first=bool(cf), **kw)
        out.append(field_stats(u, fields64[i]))
    return out


def _cases_in_processes(refs, tests, fields64, u_init, cases, kw, workers, timeout_s=900):
    """The cases split over `workers` child interpreters running this file,
    inputs and results through .npz/.npy files in a temporary folder; None when a
    child cannot be started or fails."""
    import json
    import shutil
    import subprocess
    import sys
    import tempfile
    d = tempfile.mkdtemp(prefix="fp32_envelope_")
    procs = []
    try:
        arrays = {"refs": np.asarray(refs), "tests": np.asarray(tests), "fields": np.asarray(fields64)}
        if u_init is not None:
            arrays["u_init"] = np.asarray(u_init)
        np.savez(os.path.join(d, "in.npz"), **arrays)
        for w in range(workers):
            mine = cases[w::workers]
            if not mine:
                continue
            job = os.path.join(d, "job%d.json" % w)
            with open(job, "w") as f:
                json.dump({"cases": [[int(i), bool(cf)] for i, cf in mine], "kw": kw}, f)
            procs.append((w, subprocess.Popen([sys.executable, os.path.abspath(__file__), d, job],
                                              stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)))
        stats = [None] * len(cases)
        for w, pr in procs:
            _, err = pr.communicate(timeout=timeout_s)
            if pr.returncode != 0:
                return None
            res = np.load(os.path.join(d, "job%d.npy" % w), allow_pickle=False)
            for k, j in enumerate(range(w, len(cases), workers)):
                stats[j] = tuple(res[k])
        return stats
    except (OSError, subprocess.SubprocessError):
        return None
    finally:
        for _, pr in procs:
            if pr.poll() is None:
                pr.kill()
                pr.wait()
        shutil.rmtree(d, ignore_errors=True)


def envelope(refs, tests, fields64, u_init=None, workers=1, **kw):
    """Per pair, the largest (median, p95, RMS) of |u32 - u64| over the two
    FP32 rounding orders (rows or columns smoothed first), against the FP64
    fields fields64 [n, 2, H, W].  Returns an [n, 3] array.  workers > 1
    runs the (pair, order) cases in that many child interpreters (falling
    back to this process if they cannot run); kw: demons() arguments."""
    n = len(refs)
    cases = [(i, cf) for i in range(n) for cf in (False, True)]
    stats = None
    if workers > 1 and len(cases) > 1:
        stats = _cases_in_processes(refs, tests, fields64, u_init, cases, kw, min(workers, len(cases)))
    if stats is None:
        stats = _cases(refs, tests, fields64, u_init, cases, kw)
    out = np.zeros((n, 3))
    for (i, _), st in zip(cases, stats):
        out[i] = np.maximum(out[i], st)
    return out


def _child(folder, job):
    import json
    with open(job) as f:
        spec = json.load(f)
    with np.load(os.path.join(folder, "in.npz"), allow_pickle=False) as z:
        u_init = z["u_init"] if "u_init" in z.files else None
        res = _cases(z["refs"], z["tests"], z["fields"], u_init, [tuple(c) for c in spec["cases"]], spec["kw"])
    np.save(job[:-5] + ".npy", np.array(res, dtype=np.float64))


if __name__ == "__main__":
    import sys
    _child(sys.argv[1], sys.argv[2])

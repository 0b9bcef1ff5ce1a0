"""Seeded synthetic Kikuchi-pattern generator (CPU, FP64, NumPy).

Stands in for the paper's EMsoft dynamical simulations of FCC nickel at 20 kV
and its experimental scans, which are not available here.  It produces input
pairs with the shapes, intensity statistics and geometry of the paper's
workload, and ground-truth labels.  It holds none of the registration
method's arithmetic: it renders patterns and reports the deformation that was
applied; both the HIP path and the CPU oracle consume its arrays unchanged.

Geometry
    Gnomonic projection.  Pixel (x, y) (x = column, y = row, centres at
    integers) sees direction r(x) = (x - x*, y - y*, Z*) with
    x* = pc_x W - 0.5, y* = pc_y H - 0.5, Z* = pc_z W (px).

Bands
    One band for each of the 25 distinct plane normals of the FCC families
    {111}, {200}, {220}, {311}.  For a unit normal n (detector frame) a
    direction d lies at angle phi = asin(n . d/|d|) from the plane; the band
    profile is (1 + cos(pi phi / theta_B)) / 2 for |phi| <= theta_B, where
    theta_B = asin((lambda / 2a) sqrt(h^2 + k^2 + l^2)) and lambda/a = 0.02438
    (20 kV electrons on nickel), so the width scales as 1/d.

Intensity
    I = 1 + 0.2 (g_x (x/(W-1) - 1/2) + g_y (y/(H-1) - 1/2)) + 0.5 sum(profiles),
    g ~ U(-1, 1) per pair; scaled to a mean of ``counts`` (1e4), Poisson
    noise (independent draws for reference and test), stored as float32.

Test pattern
    Rendered by pull-back: T(x') = bands(F^-1 r(x')) + the same background,
    with F = (I + eps) R_mis.  The exact shift field is then
    q(x) = pi(F r(x)) - x, pi(v) = (x* + Z* v_x/v_z, y* + Z* v_y/v_z), which is
    the projective model of the paper's Eq. (2).

Seeds
    numpy.random.SeedSequence([config_id, pair_index, stream]) with the
    streams below, so every pair is reproducible on its own.
"""
from __future__ import annotations

import itertools
import math
import os
from dataclasses import dataclass, field

import numpy as np

LAMBDA_OVER_A = 0.02438
FAMILIES = ((1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 1, 1))
# Higher-order FCC reflectors (all-odd or all-even hkl), used by the "rich"
# band set: narrower, weaker bands that real patterns show as well.
FAMILIES_RICH = FAMILIES + ((2, 2, 2), (4, 0, 0), (3, 3, 1), (4, 2, 0), (4, 2, 2), (5, 1, 1),
                            (3, 3, 3), (4, 4, 0), (5, 3, 1), (6, 0, 0), (6, 2, 0))

S_ORIENT, S_STRAIN, S_NOISE_REF, S_NOISE_TEST, S_BACKGROUND, S_MISORIENT = range(6)


def plane_normals(families=FAMILIES):
    """Distinct (up to sign) plane normals of the given families, with theta_B
    and the family's amplitude (1 for the four main families, falling as
    1/|g| beyond them)."""
    out = []
    g0 = math.sqrt(11.0)
    for fam in families:
        seen = set()
        for perm in set(itertools.permutations(fam)):
            for signs in itertools.product((1, -1), repeat=3):
                v = tuple(s * c for s, c in zip(signs, perm))
                if all(c == 0 for c in v):
                    continue
                # canonical representative of +-v
                first = next(c for c in v if c != 0)
                key = v if first > 0 else tuple(-c for c in v)
                seen.add(key)
        for hkl in sorted(seen):
            h, k, l = hkl
            g = math.sqrt(h * h + k * k + l * l)
            amp = 1.0 if fam in FAMILIES else g0 / g * 0.5
            out.append((hkl, math.asin(LAMBDA_OVER_A / 2.0 * g), amp))
    return out


_NORMALS = {"basic": plane_normals(FAMILIES), "rich": plane_normals(FAMILIES_RICH)}
assert len(_NORMALS["basic"]) == 25


def random_rotation(rng):
    """Uniform rotation on SO(3) from a uniform unit quaternion (Shoemake 1992)."""
    u1, u2, u3 = rng.random(3)
    a = math.sqrt(1.0 - u1)
    b = math.sqrt(u1)
    qw, qx, qy, qz = (a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
                      b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3))
    return quat_to_matrix(qw, qx, qy, qz)


def quat_to_matrix(w, x, y, z):
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def axis_angle_matrix(axis, angle):
    """Rodrigues' rotation formula."""
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def random_axis(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


@dataclass
class Geometry:
    H: int
    W: int
    pc: tuple = (0.5, 0.5, 0.7)

    @property
    def xs(self):
        return self.pc[0] * self.W - 0.5

    @property
    def ys(self):
        return self.pc[1] * self.H - 0.5

    @property
    def zs(self):
        return self.pc[2] * self.W

    def directions(self):
        """r(x) for every pixel, shape [3, H, W]."""
        y, x = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        return np.stack([x - self.xs, y - self.ys, np.full_like(x, self.zs)])

    def project(self, v):
        """pi(v) for v of shape [3, ...] -> (x, y)."""
        return self.xs + self.zs * v[0] / v[2], self.ys + self.zs * v[1] / v[2]


def render_bands(G, d, bands="basic"):
    """Sum of band profiles for crystal orientation G (crystal -> detector)
    seen along directions d [3, ...] (not necessarily unit)."""
    nl = _NORMALS[bands]
    dn = d / np.linalg.norm(d, axis=0, keepdims=True)
    flat = dn.reshape(3, -1)
    normals = np.array([np.array(hkl, np.float64) / np.linalg.norm(hkl) for hkl, _, _ in nl])
    thetas = np.array([t for _, t, _ in nl])
    amps = np.array([a for _, _, a in nl])
    s = (G @ normals.T).T @ flat  # [nb, P] = sin(phi)
    acc = np.zeros(flat.shape[1])
    for b in range(len(nl)):
        sb = s[b]
        m = np.abs(sb) <= math.sin(thetas[b])
        if not m.any():
            continue
        phi = np.arcsin(sb[m])
        acc[m] += amps[b] * 0.5 * (1.0 + np.cos(math.pi * phi / thetas[b]))
    return acc.reshape(d.shape[1:])


def background(geom, gxy):
    y, x = np.mgrid[0:geom.H, 0:geom.W].astype(np.float64)
    return 1.0 + 0.2 * (gxy[0] * (x / (geom.W - 1) - 0.5) + gxy[1] * (y / (geom.H - 1) - 0.5))


@dataclass
class PairSpec:
    """Everything that defines one reference/test pair."""
    H: int
    W: int
    G: np.ndarray                 # reference crystal orientation (crystal -> detector)
    F: np.ndarray                 # applied deformation gradient (detector frame)
    gxy: tuple = (0.0, 0.0)       # background gradient coefficients
    pc: tuple = (0.5, 0.5, 0.7)
    counts: float = 1e4
    noise: bool = True
    seeds: tuple = (0, 0)         # (config_id, pair_index) for the noise streams
    bands: str = "basic"          # "basic" = the four main families, "rich" = + higher orders
    extra: dict = field(default_factory=dict)


def render_pair(spec: PairSpec):
    """Render (ref, test) float32 [H, W] for one PairSpec."""
    geom = Geometry(spec.H, spec.W, spec.pc)
    r = geom.directions()
    bg = background(geom, spec.gxy)
    Iref = bg + 0.5 * render_bands(spec.G, r, spec.bands)
    Finv = np.linalg.inv(spec.F)
    d = np.einsum("ij,jhw->ihw", Finv, r)
    Itest = bg + 0.5 * render_bands(spec.G, d, spec.bands)
    ref = Iref * (spec.counts / Iref.mean())
    test = Itest * (spec.counts / Itest.mean())
    if spec.noise:
        cid, pid = spec.seeds
        rr = np.random.default_rng(np.random.SeedSequence([cid, pid, S_NOISE_REF]))
        rt = np.random.default_rng(np.random.SeedSequence([cid, pid, S_NOISE_TEST]))
        ref = rr.poisson(ref).astype(np.float64)
        test = rt.poisson(test).astype(np.float64)
    return ref.astype(np.float32), test.astype(np.float32)


def true_shift_field(F, geom: Geometry, xs=None, ys=None):
    """Label field q(x) = pi(F r(x)) - x at the given pixel positions
    (default: every pixel).  Returns [2, ...] (x shift, y shift)."""
    if xs is None:
        ys, xs = np.mgrid[0:geom.H, 0:geom.W].astype(np.float64)
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    r = np.stack([xs - geom.xs, ys - geom.ys, np.full_like(xs, geom.zs)])
    v = np.einsum("ij,j...->i...", np.asarray(F, np.float64), r)
    px, py = geom.project(v)
    return np.stack([px - xs, py - ys])


def strain_matrix(rng, bound):
    e = rng.uniform(-bound, bound, size=6)
    return np.array([[e[0], e[5], e[4]], [e[5], e[1], e[3]], [e[4], e[3], e[2]]])


def make_spec(config_id, pair_index, H, W, mis_deg=(0.0, 10.0), strain=2e-3, exact_angle=None,
              counts=1e4, noise=True, pc=(0.5, 0.5, 0.7), background_on=True):
    """Seeded PairSpec: uniform SO(3) orientation, misorientation with a
    uniform random axis and an angle uniform in mis_deg (or exact_angle deg),
    symmetric strain with components uniform in +-strain, F = (I + eps) R."""
    ss = lambda s: np.random.default_rng(np.random.SeedSequence([config_id, pair_index, s]))
    G = random_rotation(ss(S_ORIENT))
    rm = ss(S_MISORIENT)
    axis = random_axis(rm)
    ang = exact_angle if exact_angle is not None else rm.uniform(mis_deg[0], mis_deg[1])
    Rm = axis_angle_matrix(axis, math.radians(ang))
    eps = strain_matrix(ss(S_STRAIN), strain) if strain > 0 else np.zeros((3, 3))
    F = (np.eye(3) + eps) @ Rm
    gxy = tuple(ss(S_BACKGROUND).uniform(-1.0, 1.0, size=2)) if background_on else (0.0, 0.0)
    return PairSpec(H=H, W=W, G=G, F=F, gxy=gxy, pc=pc, counts=counts, noise=noise,
                    seeds=(config_id, pair_index),
                    extra={"axis": axis, "angle_deg": ang, "eps": eps, "Rmis": Rm})


def render_batch(specs, workers=None):
    """Render a list of PairSpec into (refs, tests) float32 [n, H, W] arrays.
    Serial by default (about 17 ms per 256^2 pair); workers > 1 uses a thread
    pool.  No processes are forked or spawned."""
    n = len(specs)
    H, W = specs[0].H, specs[0].W
    refs = np.empty((n, H, W), np.float32)
    tests = np.empty((n, H, W), np.float32)
    if workers is None:
        workers = 1

    def one(i):
        refs[i], tests[i] = render_pair(specs[i])

    if n >= 4 and workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(n)))
    else:
        for i in range(n):
            one(i)
    return refs, tests


# -- scan maps --------------------------------------------------------------------

def scan_map(config_id=3, size=64, grains=12, max_deg=10.0):
    """Seeded Voronoi scan map for the scan workload.

    Grain seeds are uniform in [0, size)^2; a scan point belongs to the nearest
    seed (ties to the lower index).  Each grain has a uniform SO(3) orientation,
    a background gradient, and a linear intragranular rotation field
    w(p) = K_g (p - seed_g) (rotation vector, rad) with K_g Gaussian 3 x 2,
    scaled so that the largest |w| over the grain's points is theta_g, uniform
    in (0, max_deg] degrees."""
    rng = np.random.default_rng(np.random.SeedSequence([config_id, 0, 100]))
    seeds = rng.uniform(0.0, size, size=(grains, 2))
    ys, xs = np.mgrid[0:size, 0:size]
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)
    gid = np.argmin(((pts[:, None, :] - seeds[None]) ** 2).sum(-1), axis=1)
    G, K, theta, gxy = [], [], [], []
    for g in range(grains):
        rg = np.random.default_rng(np.random.SeedSequence([config_id, g, 101]))
        G.append(random_rotation(rg))
        k = rg.normal(size=(3, 2))
        th = math.radians(rg.uniform(0.0, max_deg)) or math.radians(max_deg)
        d = pts[gid == g] - seeds[g]
        mx = np.linalg.norm(d @ k.T, axis=1).max() if d.size else 1.0
        K.append(k * (th / mx) if mx > 0 else k)
        theta.append(th)
        gxy.append(tuple(rg.uniform(-1.0, 1.0, size=2)))
    return dict(size=size, seeds=seeds, gid=gid.reshape(size, size), G=G, K=K, theta=theta, gxy=gxy)


def scan_specs(H, W, indices, config_id=3, counts=1e4, noise=True, smap=None):
    """PairSpecs of scan points (index = y * size + x) and the reference spec of
    each grain they use.  Returns (tests, refs, ref_ids): the test of point p
    is the grain's orientation under F = R(w(p)); refs[g] renders the grain's
    reference pattern (noise seeded per grain, so every point of a grain shares
    one reference); ref_ids[i] is the grain of point i."""
    m = smap or scan_map(config_id)
    size = m["size"]
    tests, ref_ids = [], []
    for idx in indices:
        x, y = idx % size, idx // size
        g = int(m["gid"][y, x])
        w = m["K"][g] @ (np.array([x, y], np.float64) - m["seeds"][g])
        ang = float(np.linalg.norm(w))
        F = axis_angle_matrix(w / ang, ang) if ang > 0 else np.eye(3)
        tests.append(PairSpec(H=H, W=W, G=m["G"][g], F=F, gxy=m["gxy"][g], counts=counts, noise=noise,
                              seeds=(config_id, int(idx)), extra={"grain": g, "rotvec": w}))
        ref_ids.append(g)
    refs = {g: PairSpec(H=H, W=W, G=m["G"][g], F=np.eye(3), gxy=m["gxy"][g], counts=counts, noise=noise,
                        seeds=(config_id, 1000000 + g)) for g in sorted(set(ref_ids))}
    return tests, refs, ref_ids


def render_scan(tests, refs, ref_ids):
    """(ref patterns per grain {g: [H, W]}, test patterns [n, H, W]) for scan_specs output."""
    ref_img = {g: render_pair(s)[0] for g, s in refs.items()}
    _, test_img = render_batch(tests)
    return ref_img, test_img


# -- workloads ------------------------------------------------------------------

WORKLOADS = {
    # single pair, 128^2, 2 deg random axis, 1e-3 strain, 3 levels x 100 it, 20 ROIs of 32^2
    "single_128": dict(config_id=1, n=1, H=128, W=128, exact_angle=2.0, strain=1e-3,
                       iters=100, roi=32),
    # batch of 1024 pairs, 256^2, misorientation U(0,10) deg, strain +-2e-3, 3 x 150, ROIs 64^2
    "batch_256": dict(config_id=2, n=1024, H=256, W=256, mis_deg=(0.0, 10.0), strain=2e-3,
                      iters=150, roi=64),
    # the headline: 1024 pairs at 256^2, misorientation exactly 10 deg
    "batch_256_10deg": dict(config_id=6, n=1024, H=256, W=256, exact_angle=10.0, strain=2e-3,
                            iters=150, roi=64),
    # scan map: 64 x 64 points at 400^2, 12 Voronoi grains with one reference each,
    # intragranular rotation up to 10 deg, per-pair stop at 1e-4 px, ROIs of 128^2
    # (patterns from scan_specs / render_scan)
    "scan_400": dict(config_id=3, n=4096, H=400, W=400, strain=0.0, iters=150, roi=128, tol=1e-4),
    # the paper's own pattern size and settings (section 3.1): 1244 x 1024 px (width x height),
    # pattern centre (0.5, 0.5, 0.5), 7 levels x 25 iterations, no field smoothing; 10 deg;
    # 100 ROIs of 256 x 256 on a ring plus one at the centre (the paper's test set 1)
    "paper_1244": dict(config_id=7, n=256, H=1024, W=1244, exact_angle=10.0, strain=2e-3, iters=25,
                       levels=7, sigma=0.0, roi=256, n_roi=101, pc=(0.5, 0.5, 0.5)),
}


def workload_specs(name, n=None, start=0):
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    kw = dict(mis_deg=w.get("mis_deg", (0.0, 10.0)), strain=w["strain"],
              exact_angle=w.get("exact_angle"), pc=w.get("pc", (0.5, 0.5, 0.7)))
    return [make_spec(w["config_id"], start + i, w["H"], w["W"], **kw) for i in range(n)]

"""Eq. (3) under the traction-free constraint with the sample-frame strain and
stress (Eq. (13)-(16), supplementary Part 2) on the GPU through the C ABI,
against the FP64 oracle.  Needs an MI355X; run with -m gpu.

Bars (both sides FP64 from the same fp32 shifts; the Lagrange-Newton steps
converge to |step| < 1e-14 on both):
  * F and eps_S: 1e-11; sigma_S: 1e-11 C11 (3 Pa for nickel);
  * against the constructed truth, exact shifts rounded to fp32 (~4e-6 px at
    60 px, 2e-8 of Z*): F to 1e-7, sigma to 1e-7 C11;
  * whole path on rendered noise-free pairs (one remap/XCF pass): the stress
    error against the constructed stress below 150 MPa (the oracle's own path
    gives 24-43 MPa on these pairs; the paper reports a phantom stress of
    ~35 MPa).
"""
import importlib.util
import math
import os

import numpy as np
import pytest
import scipy.linalg
import torch
from scipy.spatial.transform import Rotation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


@pytest.fixture(scope="module")
def pins():
    spec = importlib.util.spec_from_file_location(
        "pins", os.path.join(os.path.dirname(__file__), "test_oracle_pins.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def cases(pins, n, seed0):
    out = []
    r = np.random.default_rng(seed0)
    for k in range(n):
        g = Rotation.random(random_state=seed0 + k).as_matrix()
        inplane = r.uniform(-2e-3, 2e-3, size=3)
        eps_S = pins._traction_free_strain(tuple(inplane), g, pins.NI)
        V = np.real(scipy.linalg.sqrtm(np.eye(3) + 2 * eps_S))
        F_S = V @ Rotation.from_rotvec(r.normal(scale=0.03, size=3)).as_matrix()
        out.append((g, eps_S, F_S))
    return out


@pytest.mark.parametrize("second_pass_form", [False, True])
def test_traction_free_matches_oracle_and_truth(E, orc, pins, second_pass_form):
    cx, cy, pcs = pins._layout()
    S = pins._r_tilt(math.radians(70.0))
    cs = cases(pins, 48, 200 + int(second_pass_form))
    q, gs, Ms, Ftrue, eps_true = [], [], [], [], []
    r = np.random.default_rng(7)
    for g, eps_S, F_S in cs:
        F = S.T @ F_S @ S
        M = Rotation.from_rotvec(r.normal(scale=0.1, size=3)).as_matrix() if second_pass_form else np.eye(3)
        q.append(pins._project(F @ M.T, cx, cy, *pcs))
        gs.append(g)
        Ms.append(M)
        Ftrue.append(F)
        eps_true.append(eps_S)
    q = np.stack(q).astype(np.float32)
    print(f"traction-free solve, {len(cs)} cases, second-pass form {second_pass_form}", flush=True)
    g = E.traction_free(torch.from_numpy(q).cuda(), cx, cy, pcs, np.stack(gs), S, pins.NI,
                        M=np.stack(Ms) if second_pass_form else None)
    torch.cuda.synchronize()
    Fg, eg, sg = (g[k].cpu().numpy() for k in ("F", "eps_S", "sigma_S"))
    assert not g["status"].cpu().numpy().any()
    dF = de = ds = 0.0
    for i in range(len(cs)):
        Fo, eo, so, st = orc.solve_F_traction_free(q[i].astype(np.float64), cx, cy, pcs, S, gs[i], pins.NI,
                                                   M=Ms[i] if second_pass_form else None)
        assert st == 0
        dF = max(dF, np.abs(Fg[i] - Fo).max())
        de = max(de, np.abs(eg[i] - eo).max())
        ds = max(ds, np.abs(sg[i] - so).max())
    print("  vs oracle: max |dF| %.1e, |d eps| %.1e, |d sigma| %.1e Pa" % (dF, de, ds))
    assert dF <= 1e-11 and de <= 1e-11 and ds <= 1e-11 * pins.NI[0]
    tF = np.abs(Fg - np.stack(Ftrue)).max()
    sig_true = np.stack([pins._stress_tensor_route(e, gg, pins.NI) for e, gg in zip(eps_true, gs)])
    tS = np.abs(sg - sig_true).max()
    print("  vs truth (fp32 shifts): max |dF| %.1e, |d sigma| %.2f MPa; surface tractions <= %.1e Pa"
          % (tF, tS / 1e6, np.abs(sg[:, 2, :]).max()))
    assert tF <= 1e-7 and tS <= 1e-7 * pins.NI[0]
    assert np.abs(sg[:, 2, :]).max() <= 1e-11 * pins.NI[0]


def test_traction_free_whole_path(E, orc, pins):
    """A rendered noise-free pair (rich band set, 256 px) whose test is the
    reference seen through a traction-free F (2 deg): the path's q2 and
    R_finite, then the constrained solve; GPU against the oracle from the
    same inputs, and the stress against the constructed one."""
    from paper_1907_05993_amd import synth as S_
    S = pins._r_tilt(math.radians(70.0))
    refs, tests, gs, sig_true = [], [], [], []
    for k in range(4):
        r = np.random.default_rng(300 + k)
        G = S_.random_rotation(r)
        R_S = Rotation.from_rotvec(S_.random_axis(r) * math.radians(2.0)).as_matrix()
        R_det = S.T @ R_S @ S
        g = (S @ R_det @ G).T  # passive sample -> crystal of the test crystal
        eps_S = pins._traction_free_strain(tuple(r.uniform(-1e-3, 1e-3, size=3)), g, pins.NI)
        V = np.real(scipy.linalg.sqrtm(np.eye(3) + 2 * eps_S))
        F = S.T @ (V @ R_S) @ S
        spec = S_.PairSpec(H=256, W=256, G=G, F=F, gxy=(0.0, 0.0), noise=False, bands="rich")
        a, b = S_.render_pair(spec)
        refs.append(a)
        tests.append(b)
        gs.append(g)
        sig_true.append(pins._stress_tensor_route(eps_S, g, pins.NI))
    print("traction-free stress on the whole path, 4 noise-free pairs of 256", flush=True)
    reg = E.Registrar(E.Params(levels=3, iters=(50, 50, 50), roi_size=64))
    out = reg.register(torch.from_numpy(np.stack(refs)).cuda(), torch.from_numpy(np.stack(tests)).cuda(),
                       want_field=False)
    torch.cuda.synchronize()
    op = orc.make_params(roi_size=64, n_roi=20)
    cx, cy, _, _, _ = orc.roi_layout(256, 256, op)
    pcs = orc.pc_pixels(256, 256, op)
    g = E.traction_free(out["q2"], cx, cy, pcs, np.stack(gs), S, pins.NI, M=out["R_finite"])
    torch.cuda.synchronize()
    sg = g["sigma_S"].cpu().numpy()
    q2 = out["q2"].cpu().numpy()
    Rf = out["R_finite"].cpu().numpy()
    for i in range(4):
        Fo, eo, so, st = orc.solve_F_traction_free(q2[i].astype(np.float64), cx, cy, pcs, S, gs[i], pins.NI, M=Rf[i])
        assert np.abs(sg[i] - so).max() <= 1e-11 * pins.NI[0]
    err = np.abs(sg - np.stack(sig_true)).max(axis=(1, 2))
    print("  stress error per pair (MPa):", ["%.1f" % (e / 1e6) for e in err])
    assert (err < 1.5e8).all()

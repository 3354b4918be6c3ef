"""torch.autograd path through the HIP library, checked against central finite
differences of the renderer itself (common random numbers), and a short
optimisation run."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_03939_amd import scenes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03939_amd import binding
    binding.load()
    return binding


def _scene():
    rng = np.random.default_rng(31)
    V, F = S.noise_sphere(5, 0.2, noise_seed=8)
    floor = np.array([[-3, -1.25, -3], [3, -1.25, -3], [3, -1.25, 3], [-3, -1.25, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    env = S.gaussian_lobe_envmap(rng, 64, 32) + np.float32(0.3)
    return S.Scene(Vf, Ff, S.random_materials(Ff.shape[0], rng), np.zeros((0, 6), np.float32), env), nv


def test_renderfn_matches_library(B):
    _say("case RenderFn == library forward/backward")
    from paper_2012_03939_amd.autograd import render
    sc, _ = _scene()
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 0.6, 3.0), 32, 32)]
    V = torch.tensor(sc.V, device="cuda", requires_grad=True)
    M = torch.tensor(sc.mat, device="cuda", requires_grad=True)
    img = render(V, M, g, cams, 4, 2, seed=3)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    ref = g.render(cams, 4, 2, seed=3)
    dV, dM = g.backward(cams, 4, 2, w, seed=3)
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), ref)
    for a, b in ((V.grad, dV), (M.grad, dM)):
        rel = float((a - b).norm() / b.norm())
        assert rel < 1e-5, rel


def test_vertex_gradient_vs_central_differences(B):
    """E[dL/dV . delta] from the adjoint (interior + primary + secondary edges)
    against central differences of the same renderer with common random numbers,
    paired over seeds.  Environment lighting only: every visibility
    discontinuity is then covered by an edge term."""
    _say("case vertex gradient vs free CRN central differences, 24 seeds")
    sc, nobj = _scene()
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 0.6, 3.0), 48, 48)]
    spp, bounces = 32, 2
    rng = np.random.default_rng(4)
    w = torch.from_numpy(rng.uniform(0.5, 1.5, size=(48 * 48, 3)).astype(np.float32)).cuda()
    delta = np.zeros_like(sc.V)
    P = sc.V[:nobj].astype(np.float64)
    radial = P / np.linalg.norm(P, axis=1, keepdims=True)
    delta[:nobj] = radial * (1.0 + 0.5 * np.sin(3.0 * P[:, :1]) * np.cos(2.0 * P[:, 1:2]))
    delta /= np.abs(delta).max()
    V0 = torch.from_numpy(sc.V).cuda()
    dl = torch.from_numpy(delta.astype(np.float32)).cuda()
    h = 2e-3
    fd, ad = [], []
    for s in range(24):
        g.update(V=V0 + h * dl)
        lp = float((g.render(cams, spp, bounces, seed=s) * w).sum())
        g.update(V=V0 - h * dl)
        lm = float((g.render(cams, spp, bounces, seed=s) * w).sum())
        g.update(V=V0)
        dV, _ = g.backward(cams, spp, bounces, w, seed=s)
        fd.append((lp - lm) / (2 * h))
        ad.append(float((dV * dl).sum()))
    fd, ad = np.array(fd), np.array(ad)
    diff = fd - ad
    se = diff.std(ddof=1) / np.sqrt(len(diff))
    _say(f"  mean FD {fd.mean():.5g}  mean AD {ad.mean():.5g}  mean diff {diff.mean():.4g} +- {se:.3g}")
    assert abs(diff.mean()) < 4 * se + 0.02 * abs(ad.mean())
    assert abs(ad.mean()) > 4 * ad.std(ddof=1) / np.sqrt(len(ad))      # the derivative is resolved


def test_interior_only_misses_visibility(B):
    """Without the edge terms the vertex gradient is biased on a silhouette-heavy
    scene: the same central differences disagree with the interior-only adjoint."""
    _say("case interior-only adjoint vs CRN central differences")
    V, F = S.geodesic_sphere(4)
    mat = S.uniform_materials(F.shape[0], kd=0.8, ks=0.0, rough=0.3)
    sc = S.Scene(V.astype(np.float32), F, mat, np.zeros((0, 6), np.float32), np.ones((16, 32, 3), np.float32))
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.0, 0.0, 3.0), 48, 48)]
    V0 = torch.from_numpy(sc.V).cuda()
    dl = V0 / V0.norm(dim=1, keepdim=True)                 # inflate: silhouette moves outward
    w = torch.ones((48 * 48, 3), device="cuda")
    h = 2e-3
    fd, ai, aa = [], [], []
    for s in range(8):
        g.update(V=V0 + h * dl)
        lp = float(g.render(cams, 16, 1, seed=s).sum())
        g.update(V=V0 - h * dl)
        lm = float(g.render(cams, 16, 1, seed=s).sum())
        g.update(V=V0)
        fd.append((lp - lm) / (2 * h))
        ai.append(float((g.backward(cams, 16, 1, w, seed=s, flags=B.ST_GRAD_INTERIOR)[0] * dl).sum()))
        aa.append(float((g.backward(cams, 16, 1, w, seed=s)[0] * dl).sum()))
    fd, ai, aa = map(np.array, (fd, ai, aa))
    _say(f"  FD {fd.mean():.5g}  all terms {aa.mean():.5g}  interior only {ai.mean():.5g}")
    assert abs(aa.mean() - fd.mean()) < 0.1 * abs(fd.mean())
    assert abs(ai.mean() - fd.mean()) > 0.5 * abs(fd.mean())


def test_short_optimisation_reduces_loss(B):
    _say("case 25 optimisation steps, small views")
    from paper_2012_03939_amd.optimise import run
    r = run(steps=25, nviews=8, res=64, spp=4, bounces=2, target_spp=16)
    _say(f"  {r}")
    assert r["image_l2_last"] < 0.9 * r["image_l2_first"]


def test_optimisation_resumes_from_a_checkpoint(B):
    """3 steps with a checkpoint, then a resumed run to 6 steps, against 6 steps
    without interruption (same per-step seeds and Adam state).  The gradients
    are sums of float atomics from two streams (the adjoint beside the edge
    terms), whose order varies from run to run, and Adam's normalised steps
    carry that rounding into the vertices: the bar is 1e-4 of a vertex move of
    up to 6e-3; a resume that lost the Adam moments moves them ~1e-3 apart."""
    import os
    import tempfile
    from paper_2012_03939_amd.optimise import load_checkpoint, run
    print("case optimisation checkpoint: 3 steps + resume to 6 vs 6 uninterrupted", flush=True)
    kw = dict(nviews=4, res=48, spp=4, bounces=2, target_spp=8)
    path = os.path.join(tempfile.mkdtemp(), "opt.pt")
    run(steps=3, checkpoint=path, checkpoint_every=3, **kw)
    assert load_checkpoint(path)["step"] == 2
    resumed = run(steps=6, checkpoint=path, resume=True, return_params=True, **kw)
    plain = run(steps=6, return_params=True, **kw)
    dv = (resumed["V"] - plain["V"]).abs().max().item()
    dm = (resumed["M"] - plain["M"]).abs().max().item()
    print(f"  max |dV| {dv:.2e} max |dM| {dm:.2e}", flush=True)
    assert dv < 1e-4 and dm < 1e-4
    assert abs(resumed["image_l2_last"] - plain["image_l2_last"]) < 1e-4 * plain["image_l2_last"]

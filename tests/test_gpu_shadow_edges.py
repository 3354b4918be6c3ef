"""Point-light shadow boundaries (ST_EDGE_SHADOW) through the C ABI: the term
alone and with every other term against the FP64 oracle (flipped samples masked
out of both sides), the closed-form scene of the oracle pin, and a free
finite-difference check of the renderer for a cast shadow under a point light,
which the other edge terms alone cannot pass (there the adjoint without the
shadow term is exactly zero)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, GRAD_RTOL, rel_l2

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


def _sphere_on_floor(nlights=3, seed=14):
    rng = np.random.default_rng(seed)
    V, F = S.noise_sphere(6, 0.15, noise_seed=2)
    floor = np.array([[-3, -1.3, -3], [3, -1.3, -3], [3, -1.3, 3], [-3, -1.3, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    return S.Scene(Vf, Ff, S.random_materials(Ff.shape[0], rng), S.hemisphere_lights(nlights, rng), None), nv


def _parity(B, sc, cams, spp, bounces, flags, seed=0, ratio=1.0):
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    nl = sc.lights.shape[0] if flags & B.ST_EDGE_SHADOW else 0
    npath = B.num_pixels(cams) * spp
    ne = B.num_edge_samples(cams, spp, ratio, nl)
    d_img = np.random.default_rng(6).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    dt = torch.from_numpy(d_img).cuda()
    ph = torch.zeros(npath, dtype=torch.int32, device="cuda")
    eh = torch.zeros(max(ne, 1), dtype=torch.int32, device="cuda")
    g.backward(cams, spp, bounces, dt, seed, flags, ratio, debug_hash=ph, debug_edge_hash=eh)
    g.check_errors()
    _, _, oph, oeh = o.backward(cams, spp, bounces, d_img, seed, flags, ratio)
    gph = ph.cpu().numpy().view(np.uint32)
    geh = eh.cpu().numpy().view(np.uint32)[:ne]
    assert oeh.shape == (ne,)
    pmask = ~((gph != oph) & (oph != 0))
    emask = ~((geh != oeh) & (oeh != 0))
    dV, dM = g.backward(cams, spp, bounces, dt, seed, flags, ratio,
                        path_mask=torch.from_numpy(pmask.astype(np.uint8)).cuda(),
                        edge_mask=torch.from_numpy(emask.astype(np.uint8)).cuda())
    torch.cuda.synchronize()
    oV, oM, _, _ = o.backward(cams, spp, bounces, d_img, seed, flags, ratio, path_mask=pmask.astype(np.uint8),
                              edge_mask=emask.astype(np.uint8))
    return 1 - pmask.mean(), 1 - emask.mean(), rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM), oV


@pytest.mark.parametrize("flags", [8, 15])
def test_shadow_edges_parity(B, flags):
    _say(f"case shadow edges parity, noise sphere + floor, 3 lights, B=2, flags={flags}")
    sc, _ = _sphere_on_floor()
    cams = [S.look_at_origin((0.3, 0.9, 3.1), 40, 32), S.look_at_origin((-2.0, 1.5, 2.0), 32, 32)]
    pf, ef, rv, rm, oV = _parity(B, sc, cams, 4, 2, flags)
    _say(f"  path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert np.abs(oV).max() > 0 and rv < GRAD_RTOL
    if flags & 1:
        assert rm < GRAD_RTOL


def test_shadow_edges_closed_form_scene(B):
    _say("case shadow edges, floor + unseen occluder triangle (the oracle pin's scene)")
    floor = np.array([[-3, -3, 0], [3, -3, 0], [3, 3, 0], [-3, 3, 0]], np.float32)
    occ = np.array([[-1.2, -0.2, 1.0], [-0.8, -0.3, 1.05], [-1.0, 0.3, 0.95]], np.float32)
    V = np.concatenate([floor, occ])
    F = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6]], np.int32)
    mat = np.zeros((3, 7), np.float32)
    mat[:, :3] = 0.6
    mat[:, 6] = 0.5
    light = np.array([[-2.2, 0.0, 3.0, 10.0, 10.0, 10.0]], np.float32)
    sc = S.Scene(V, F, mat, light, None)
    cams = [S.Camera((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, 64, 64)]
    pf, ef, rv, rm, oV = _parity(B, sc, cams, 1, 1, 8, seed=3, ratio=8.0)
    _say(f"  edge flips {ef:.5f} relL2 dV {rv:.2e}")
    assert ef < FLIP_MAX and rv < GRAD_RTOL and np.abs(oV[4:7]).max() > 0


def test_point_light_vertex_gradient_vs_central_differences(B):
    """E[dL/dV . delta] from the adjoint against central differences of the
    renderer with common random numbers, paired over seeds, for the cast shadow
    of an occluder the camera does not see (floor + triangle under a point
    light): the image changes only through the shadow boundary, so the shadow
    term carries the whole derivative and without it the adjoint is zero."""
    _say("case point-light FD: cast shadow of an unseen occluder, 16 seeds x 64 spp")
    floor = np.array([[-3, -3, 0], [3, -3, 0], [3, 3, 0], [-3, 3, 0]], np.float32)
    occ = np.array([[-1.2, -0.2, 1.0], [-0.8, -0.3, 1.05], [-1.0, 0.3, 0.95]], np.float32)
    V = np.concatenate([floor, occ])
    F = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6]], np.int32)
    mat = np.zeros((3, 7), np.float32)
    mat[:, :3] = 0.6
    mat[:, 6] = 0.5
    light = np.array([[-2.2, 0.0, 3.0, 10.0, 10.0, 10.0]], np.float32)
    sc = S.Scene(V, F, mat, light, None)
    g = B.GPUScene.from_scene(sc)
    cams = [S.Camera((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, 64, 64)]
    spp, bounces = 64, 1
    w = torch.from_numpy(np.random.default_rng(4).uniform(0.5, 1.5, size=(64 * 64, 3)).astype(np.float32)).cuda()
    delta = np.zeros_like(V)
    delta[4:7] = np.random.default_rng(9).normal(size=(3, 3))
    V0 = torch.from_numpy(V).cuda()
    dl = torch.from_numpy(delta.astype(np.float32)).cuda()
    h = 5e-3
    fd, ad, an = [], [], []
    for s in range(16):
        g.update(V=V0 + h * dl)
        lp = float((g.render(cams, spp, bounces, seed=s) * w).sum())
        g.update(V=V0 - h * dl)
        lm = float((g.render(cams, spp, bounces, seed=s) * w).sum())
        g.update(V=V0)
        fd.append((lp - lm) / (2 * h))
        ad.append(float((g.backward(cams, spp, bounces, w, seed=s, flags=15, edge_ratio=4.0)[0] * dl).sum()))
        an.append(float((g.backward(cams, spp, bounces, w, seed=s, flags=7)[0] * dl).sum()))
    fd, ad, an = map(np.array, (fd, ad, an))
    se = (fd - ad).std(ddof=1) / np.sqrt(len(fd))
    _say(f"  FD {fd.mean():.5g} +- {fd.std(ddof=1) / 4:.3g}  all terms {ad.mean():.5g} (diff se {se:.3g})  "
         f"without shadow edges {an.mean():.5g}")
    assert abs(fd.mean()) > 4 * fd.std(ddof=1) / np.sqrt(len(fd))      # the derivative is resolved
    assert abs((fd - ad).mean()) < 4 * se + 0.03 * abs(fd.mean())
    assert np.abs(an).max() == 0.0

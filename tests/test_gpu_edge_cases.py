"""Degenerate and extreme inputs against the FP64 oracle, through the C ABI: a
single-triangle mesh (the traversal's one-leaf path and three boundary edges),
a mesh with zero-area faces, cameras that see nothing, the largest bounce count
(8), and a 1x1 image at 1 spp.  Same bars as the main parity tests."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, GRAD_RTOL
from test_gpu_parity import _backward_case, _forward_case

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


def _triangle_scene():
    rng = np.random.default_rng(21)
    V = np.array([[-1.0, -0.8, 0.0], [1.2, -0.6, 0.1], [0.1, 1.0, -0.2]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    return S.Scene(V, F, S.random_materials(1, rng), S.hemisphere_lights(1, rng), S.gaussian_lobe_envmap(rng, 32, 16))


def test_single_triangle_forward_and_backward(B):
    _say("case single triangle, one light + env, B=2: forward and all gradient terms")
    sc = _triangle_scene()
    cams = [S.look_at_origin((0.3, 0.2, 3.0), 40, 36), S.look_at_origin((-2.0, 0.5, 2.0), 24, 24)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 4, 2)
    _say(f"  forward flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0 and (ref > 0).any()
    d_img = np.random.default_rng(3).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, 7)
    _say(f"  backward path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX and np.abs(oV).max() > 0
    assert rv < GRAD_RTOL and rm < GRAD_RTOL


def test_zero_area_faces(B):
    """Two faces of a sphere collapsed to zero area (a vertex moved onto its
    neighbour): no hit on them, no NaN, parity in the forward and backward."""
    _say("case sphere with collapsed faces, 2 lights, B=2: forward and all gradient terms")
    rng = np.random.default_rng(22)
    V, F = S.noise_sphere(5, 0.1, noise_seed=4)
    V = V.astype(np.float32).copy()
    a, b = int(F[7, 0]), int(F[7, 1])
    V[b] = V[a]                                      # every face with both a and b has zero area
    sc = S.Scene(V, F, S.random_materials(F.shape[0], rng), S.hemisphere_lights(2, rng), None)
    cams = [S.look_at_origin(tuple(3.0 * V[a] / np.linalg.norm(V[a])), 32, 32)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 4, 2)
    _say(f"  forward flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert np.isfinite(img.cpu().numpy()).all()
    assert fr < FLIP_MAX and bad == 0
    d_img = np.random.default_rng(4).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, 7)
    _say(f"  backward path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert np.isfinite(oV).all()
    assert pf < FLIP_MAX and ef < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL


def test_cameras_that_see_nothing(B):
    """Every camera ray misses (the object is behind the camera): the masked image
    is zero and so are all gradients, on both sides."""
    _say("case cameras facing away from the object, env, B=3")
    wl = S.small_sphere()
    sc = S.Scene(wl.scenes[0].V, wl.scenes[0].F, wl.scenes[0].mat, wl.scenes[0].lights,
                 S.gaussian_lobe_envmap(np.random.default_rng(5), 32, 16))
    far = [S.Camera((0.0, 0.0, 3.0), (0.0, 0.0, 6.0), (0.0, 1.0, 0.0), 45.0, 16, 12)]
    g = B.GPUScene.from_scene(sc)
    img = g.render(far, 2, 3, seed=1)
    torch.cuda.synchronize()
    ref, _ = O.OracleScene.from_scene(sc).render(far, 2, 3, 1)
    assert float(img.abs().max()) == 0.0 and np.abs(ref).max() == 0.0
    d = torch.ones((B.num_pixels(far), 3), dtype=torch.float32, device="cuda")
    dV, dM = g.backward(far, 2, 3, d, seed=1, flags=7)
    torch.cuda.synchronize()
    g.check_errors()
    assert float(dV.abs().max()) == 0.0 and float(dM.abs().max()) == 0.0


def test_largest_bounce_count(B):
    _say("case torus env, 8 bounces (the largest allowed), forward and interior gradients")
    rng = np.random.default_rng(23)
    V, F = S.noise_torus(24, 12, 0.1, noise_seed=13)
    sc = S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), S.hemisphere_lights(1, rng),
                 S.gaussian_lobe_envmap(rng, 32, 16))
    cams = [S.look_at_origin((0.5, 2.0, 2.5), 24, 20)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 4, 8)
    _say(f"  forward flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0
    d_img = np.random.default_rng(6).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 8, d_img, 5)
    _say(f"  backward path flips {pf:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL


def test_one_pixel_one_sample(B):
    _say("case 1x1 image, 1 spp, sphere, point lights, B=2, all terms")
    wl = S.small_sphere()
    sc = wl.scenes[0]
    cams = [S.look_at_origin((0.0, 0.2, 3.0), 1, 1)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 1, 2)
    assert fr == 0 and bad == 0
    d_img = np.ones((1, 3), np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 1, 2, d_img, 7)
    _say(f"  backward path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf == 0 and (np.abs(oV).max() == 0 or rv < GRAD_RTOL)


def test_mesh_through_the_near_plane(B):
    """A tetrahedron with one vertex behind the eye, an envmap and a point light:
    the primary edges through that vertex are clipped at the near plane and to
    the image on both sides (fp64 candidate weights), and the camera paths of the
    forward see the part in front of the eye."""
    _say("case tetrahedron through the near plane, light + env, B=2: forward and all gradient terms")
    rng = np.random.default_rng(23)
    V = np.array([[-0.6, -0.5, 0.0], [0.5, -0.6, -0.3], [0.0, 0.6, 0.2], [1.2, 0.4, 4.2]], np.float32)
    F = np.array([[0, 1, 2], [0, 3, 1], [1, 3, 2], [2, 3, 0]], np.int32)
    sc = S.Scene(V, F, S.random_materials(4, rng), S.hemisphere_lights(1, rng), S.gaussian_lobe_envmap(rng, 32, 16))
    cams = [S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 48, 40)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 4, 2)
    _say(f"  forward flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0 and (ref > 0).any()
    d_img = np.random.default_rng(4).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, 2)
    _say(f"  backward (primary edges) edge flips {ef:.5f} relL2 dV {rv:.2e}")
    assert ef < FLIP_MAX and np.abs(oV[3]).max() > 0 and rv < GRAD_RTOL
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, 15)
    _say(f"  backward (all terms) path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL


def test_non_finite_gradient_sets_the_error_word(B):
    """A NaN in the row of d_image of a pixel that sees the mesh makes the
    backward's gradients non-finite;
    the final check of the backward records it and st_check_errors reports
    ST_ERR_DEVICE_FAULT (then the word is clear again)."""
    _say("case NaN in d_image -> ST_ERR_DEVICE_FAULT")
    sc = _triangle_scene()
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.3, 0.2, 3.0), 24, 20)]
    g.check_errors()
    img = g.render(cams, 2, 2, seed=0)
    d = torch.zeros((B.num_pixels(cams), 3), device="cuda")
    d[int(torch.argmax(img.sum(dim=1)))] = float("nan")     # a pixel whose paths hit the triangle
    g.backward(cams, 2, 2, d, 0, B.ST_ALL_GRADS)
    with pytest.raises(B.StError, match="error -5"):
        g.check_errors()
    g.check_errors()                             # cleared
    g.backward(cams, 2, 2, torch.ones_like(d), 0, B.ST_ALL_GRADS)
    g.check_errors()                             # finite input, no report


def test_max_workspace_bytes(B):
    """A cap below the call's workspace fails with ST_ERR_OOM before any launch
    (the output buffer is left untouched); a cap that leaves out only the hit
    records renders the same image, and the backward then traces again."""
    _say("case max_workspace_bytes: OOM before launch, records left out under a tight cap")
    sc = _triangle_scene()
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.3, 0.2, 3.0), 32, 32)]
    spp, bounces = 4, 2
    ref = g.render(cams, spp, bounces, seed=1).clone()
    out = torch.full_like(ref, 7.0)
    with pytest.raises(B.StError, match="error -3"):
        g.render(cams, spp, bounces, seed=1, out=out, max_workspace_bytes=1 << 20)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    d = torch.ones_like(ref)
    with pytest.raises(B.StError, match="error -3"):
        g.backward(cams, spp, bounces, d, 1, B.ST_ALL_GRADS, max_workspace_bytes=1 << 20)
    # the forward's own need (radiance, queues, spill stack) without the records
    # (4 (2B + 1) bytes per path sample)
    npath = B.num_pixels(cams) * spp
    big = 1 << 40
    g.render(cams, spp, bounces, seed=1, out=out, max_workspace_bytes=big)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)

    def adjoint_rays(seed, extra=0):
        g.read_work()
        g.backward(cams, spp, bounces, d, seed, B.ST_ALL_GRADS | B.ST_COUNT_WORK | extra)
        return g.read_work()["k_adjoint"][2]

    full = adjoint_rays(1, B.ST_BACKWARD_RETRACE)
    assert adjoint_rays(1) < full                 # records kept under a large cap
    # find the smallest cap the render accepts, then check it keeps no records:
    # its backward (another seed than the records held) traces every main path
    lo, hi = 1, big
    while hi - lo > 1:
        mid = (lo + hi) // 2
        try:
            g.render(cams, spp, bounces, seed=1, out=out, max_workspace_bytes=mid)
            hi = mid
        except B.StError:
            lo = mid
    g.render(cams, spp, bounces, seed=2, out=out, max_workspace_bytes=hi)
    full2 = adjoint_rays(2, B.ST_BACKWARD_RETRACE)
    assert adjoint_rays(2) == full2               # no records under the tight cap
    g.render(cams, spp, bounces, seed=2, out=out, max_workspace_bytes=hi + 4 * (2 * bounces + 1) * npath)
    assert adjoint_rays(2) < full2                # room for them again
    g.check_errors()


def test_hidden_triangle_primary_edges(B):
    """A triangle wholly behind a larger one under a point light on the camera
    side: every sampled point of its edges is hidden (both side rays meet the
    occluder), so the primary edge term gives its vertices exactly zero on both
    implementations, and the visible triangle's gradient matches the oracle."""
    _say("case hidden triangle behind an occluder, B=2: primary edge term")
    front = np.array([[-0.8, -0.7, 0.5], [0.9, -0.6, 0.4], [0.0, 0.9, 0.5]], np.float32)
    back = np.array([[-0.2, -0.2, -0.5], [0.25, -0.15, -0.6], [0.0, 0.25, -0.5]], np.float32)
    V = np.concatenate([front, back])
    F = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    lights = np.array([[0.3, 0.4, 2.5, 6.0, 6.0, 6.0]], np.float32)
    sc = S.Scene(V, F, S.random_materials(2, np.random.default_rng(23)), lights, None)
    cams = [S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 40, 40)]
    d_img = np.random.default_rng(5).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    g = B.GPUScene.from_scene(sc)
    dV, _ = g.backward(cams, 8, 2, torch.from_numpy(d_img).cuda(), seed=3, flags=B.ST_EDGE_PRIMARY)
    g.check_errors()
    gv = dV.cpu().numpy()
    assert np.all(gv[3:] == 0.0), gv[3:]
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 8, 2, d_img, 2)
    _say(f"  backward edge flips {ef:.5f} relL2 dV {rv:.2e}")
    assert ef < FLIP_MAX and rv < GRAD_RTOL
    assert np.all(oV[3:] == 0.0) and np.abs(oV[:3]).max() > 0

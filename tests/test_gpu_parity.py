"""GPU (HIP, float32) against the FP64 oracle, through the C ABI.

Forward radiance: per-pixel relative 1e-4 outside discrete-decision flips,
flips below 0.1 % of pixels.  Gradients: relative L2 1e-3 for dV and dmat with
flipped samples masked out of both sides.  Integer work (LBVH, edge list) is
bit-exact.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, GRAD_RTOL, RAD_RTOL, radiance_check, rel_l2, view_slices

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


def _flipped_pixels(gh, oh, spp):
    return (np.asarray(gh).reshape(-1, spp) != np.asarray(oh).reshape(-1, spp)).any(axis=1)


def _forward_case(B, sc, cams, spp, bounces, seed=0, flags=0, queue_capacity=0):
    g = B.GPUScene.from_scene(sc)
    npix = B.num_pixels(cams)
    hh = torch.zeros(npix * spp, dtype=torch.int32, device="cuda")
    img = g.render(cams, spp, bounces, seed, flags=flags, queue_capacity=queue_capacity, debug_hash=hh)
    g.check_errors()
    o = O.OracleScene.from_scene(sc)
    ref, oh = o.render(cams, spp, bounces, seed)
    gh = hh.cpu().numpy().view(np.uint32)
    fl = _flipped_pixels(gh, oh, spp)
    bad, checked, worst = radiance_check(img.cpu().numpy(), ref, fl, view_slices(cams))
    return fl.mean(), bad, checked, worst, img, ref


# --------------------------------------------------------------------------
# integer work: edge list and LBVH, bit-exact
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 4, 9, 22])
def test_lbvh_bit_exact(B, k):
    _say(f"case lbvh k={k}")
    V, F = S.noise_sphere(k, 0.1, noise_seed=3)
    sc = S.Scene(V.astype(np.float32), F, S.uniform_materials(F.shape[0]), np.zeros((0, 6), np.float32), None)
    g = B.GPUScene.from_scene(sc)
    keys, child, parent, aabb = g.lbvh()
    torch.cuda.synchronize()
    rk, rc, rp, ra = O.lbvh(sc.V, sc.F, treelet_rounds=O.TREELET_ROUNDS)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(child.cpu().numpy(), rc)
    assert np.array_equal(parent.cpu().numpy(), rp)
    assert np.array_equal(aabb.cpu().numpy().view(np.uint32), ra.view(np.uint32))


def test_lbvh_torus_and_rebuild(B):
    _say("case lbvh torus + update")
    wl = S.torus_envmap(res=8, nviews=1, spp=1)
    sc = wl.scenes[0]
    g = B.GPUScene.from_scene(sc)
    V2 = S.perturbed_vertices(sc.V, 0.01, 5)
    g.update(V=torch.from_numpy(V2).cuda())
    keys, child, parent, aabb = g.lbvh()
    torch.cuda.synchronize()
    rk, rc, rp, ra = O.lbvh(V2, sc.F, treelet_rounds=O.TREELET_ROUNDS)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(child.cpu().numpy(), rc)
    assert np.array_equal(parent.cpu().numpy(), rp)
    assert np.array_equal(aabb.cpu().numpy().view(np.uint32), ra.view(np.uint32))


def test_edges_match_oracle(B):
    _say("case edges")
    V, F = S.noise_sphere(6, 0.1, noise_seed=3)
    sc = S.Scene(V.astype(np.float32), F, S.uniform_materials(F.shape[0]), np.zeros((0, 6), np.float32), None)
    g = B.GPUScene.from_scene(sc)
    e = g.edges().cpu().numpy()
    assert np.array_equal(e, O.OracleScene.from_scene(sc).edges())


def test_bvh_closest_equals_brute_force(B):
    _say("case bvh vs brute")
    rng = np.random.default_rng(1)
    V, F = S.noise_sphere(12, 0.15, noise_seed=4)
    soup = rng.uniform(-0.8, 0.8, (300, 3, 3))
    V2 = np.concatenate([V, soup.reshape(-1, 3)]).astype(np.float32)
    F2 = np.concatenate([F, V.shape[0] + np.arange(900).reshape(300, 3)]).astype(np.int32)
    g = B.GPUScene(V2, F2, S.uniform_materials(F2.shape[0]))
    n = 200000
    o = rng.uniform(-2.5, 2.5, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    f1, t1 = g.trace(ot, dt, 1e-4, brute=False)
    f2, t2 = g.trace(ot, dt, 1e-4, brute=True)
    f1, f2, t1, t2 = (x.cpu().numpy() for x in (f1, f2, t1, t2))
    assert np.array_equal(f1, f2)
    hit = f1 >= 0
    assert np.array_equal(t1[hit], t2[hit])
    assert hit.mean() > 0.05


# --------------------------------------------------------------------------
# forward radiance
# --------------------------------------------------------------------------

def test_forward_small_sphere_point_light(B):
    _say("case forward sphere320 64x64 4spp B=1")
    wl = S.small_sphere()
    fr, bad, checked, worst, img, ref = _forward_case(B, wl.scenes[0], wl.cams, wl.spp, wl.bounces)
    _say(f"  flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0
    assert (ref[:, 0] > 0).mean() > 0.2


@pytest.mark.parametrize("mega", [False, True])
def test_forward_envmap_multibounce(B, mega):
    _say(f"case forward torus-env small B=3 mega={mega}")
    rng = np.random.default_rng(11)
    V, F = S.noise_torus(48, 24, 0.1, noise_seed=13)
    sc = S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), np.zeros((0, 6), np.float32),
                 S.gaussian_lobe_envmap(rng, 64, 32))
    cams = [S.look_at_origin(e, 40, 32) for e in 4.0 * S.fibonacci_sphere(3)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 4, 3,
                                                      flags=B.ST_FORWARD_MEGAKERNEL if mega else 0,
                                                      queue_capacity=3000)
    _say(f"  flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0


def test_forward_point_lights_two_bounces_ragged(B):
    _say("case forward noise sphere 3 lights B=2 ragged views")
    rng = np.random.default_rng(12)
    V, F = S.noise_sphere(8, 0.15, noise_seed=2)
    floor = np.array([[-3, -1.3, -3], [3, -1.3, -3], [3, -1.3, 3], [-3, -1.3, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    sc = S.Scene(Vf, Ff, S.random_materials(Ff.shape[0], rng), S.hemisphere_lights(3, rng), None)
    cams = [S.look_at_origin((0.3, 0.9, 3.1), 37, 29), S.look_at_origin((-2.5, 1.0, 1.5), 24, 40)]
    fr, bad, checked, worst, img, ref = _forward_case(B, sc, cams, 3, 2)
    _say(f"  flips {fr:.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0


# --------------------------------------------------------------------------
# backward
# --------------------------------------------------------------------------

def _backward_case(B, sc, cams, spp, bounces, d_img, flags, seed=0, edge_ratio=1.0):
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    npath = B.num_pixels(cams) * spp
    # primary edge samples, then (shadow-boundary term) as many per point light
    nl = int(sc.lights.shape[0]) if flags & B.ST_EDGE_SHADOW else 0
    ne = B.num_edge_samples(cams, spp, edge_ratio, nl)
    dt = torch.from_numpy(np.ascontiguousarray(d_img, np.float32)).cuda()
    ph = torch.zeros(npath, dtype=torch.int32, device="cuda")
    eh = torch.zeros(max(ne, 1), dtype=torch.int32, device="cuda")
    g.backward(cams, spp, bounces, dt, seed, flags, edge_ratio, debug_hash=ph, debug_edge_hash=eh)
    g.check_errors()
    oV, oM, oph, oeh = o.backward(cams, spp, bounces, d_img, seed, flags, edge_ratio)
    gph = ph.cpu().numpy().view(np.uint32)
    geh = eh.cpu().numpy().view(np.uint32)[:ne]
    pmask = ~((gph != oph) & (oph != 0))
    emask = ~((geh != oeh) & (oeh != 0))
    pflip = 1.0 - pmask.mean()
    eflip = 1.0 - emask.mean() if ne else 0.0
    pm = torch.from_numpy(pmask.astype(np.uint8)).cuda()
    em = torch.from_numpy(emask.astype(np.uint8)).cuda() if ne else None
    dV, dM = g.backward(cams, spp, bounces, dt, seed, flags, edge_ratio, path_mask=pm, edge_mask=em)
    torch.cuda.synchronize()
    oV, oM, _, _ = o.backward(cams, spp, bounces, d_img, seed, flags, edge_ratio, path_mask=pmask.astype(np.uint8),
                              edge_mask=emask.astype(np.uint8) if ne else None)
    return pflip, eflip, rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM), oV, oM


def _loss_grad(sc, cams, spp, bounces, seed=0):
    """d_image of the mean squared error against a target rendered from perturbed vertices (oracle renders)."""
    o = O.OracleScene.from_scene(sc)
    R, _ = o.render(cams, spp, bounces, seed)
    tgt = S.Scene(S.perturbed_vertices(sc.V, 0.01, 77), sc.F, sc.mat, sc.lights, sc.env, sc.scene_id)
    T, _ = O.OracleScene.from_scene(tgt).render(cams, spp, bounces, seed + 1)
    return (2.0 * (R - T) / R.size).astype(np.float32)


@pytest.mark.parametrize("flags", [1, 2, 7])
def test_backward_small_sphere(B, flags):
    _say(f"case backward sphere320 64x64 4spp B=1 flags={flags}")
    wl = S.small_sphere()
    sc = wl.scenes[0]
    d_img = _loss_grad(sc, wl.cams, wl.spp, wl.bounces)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, wl.cams, wl.spp, wl.bounces, d_img, flags)
    _say(f"  path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert np.abs(oV).max() > 0
    assert rv < GRAD_RTOL
    if flags & 1:
        assert rm < GRAD_RTOL


@pytest.mark.parametrize("flags", [1, 4, 7])
def test_backward_envmap_multibounce(B, flags):
    _say(f"case backward torus-env small B=2 flags={flags}")
    rng = np.random.default_rng(13)
    V, F = S.noise_torus(40, 20, 0.1, noise_seed=13)
    sc = S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), np.zeros((0, 6), np.float32),
                 S.gaussian_lobe_envmap(rng, 64, 32))
    cams = [S.look_at_origin(e, 32, 24) for e in 4.0 * S.fibonacci_sphere(2)]
    d_img = np.random.default_rng(5).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, flags)
    _say(f"  path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert rv < GRAD_RTOL
    if flags & 1:
        assert rm < GRAD_RTOL


def test_backward_point_lights_two_bounces(B):
    _say("case backward noise sphere + floor, 3 lights, B=2, all terms")
    rng = np.random.default_rng(14)
    V, F = S.noise_sphere(6, 0.15, noise_seed=2)
    floor = np.array([[-3, -1.3, -3], [3, -1.3, -3], [3, -1.3, 3], [-3, -1.3, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    sc = S.Scene(Vf, Ff, S.random_materials(Ff.shape[0], rng), S.hemisphere_lights(3, rng), None)
    cams = [S.look_at_origin((0.3, 0.9, 3.1), 40, 32)]
    d_img = np.random.default_rng(6).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    pf, ef, rv, rm, oV, oM = _backward_case(B, sc, cams, 4, 2, d_img, 7)
    _say(f"  path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert pf < FLIP_MAX and ef < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL

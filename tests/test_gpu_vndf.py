"""Visible-normal sampling of the specular lobe (ST_BSDF_SAMPLER_VNDF) through
the C ABI against the FP64 oracle with the same sampler: forward radiance per
pixel and gradients (flipped samples masked), on glossy materials where the
specular lobe matters; and the two samplers estimate the same image."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, GRAD_RTOL, radiance_check, rel_l2, view_slices

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


def _scene(seed=21):
    rng = np.random.default_rng(seed)
    V, F = S.noise_torus(40, 20, 0.1, noise_seed=13)
    mat = S.random_materials(F.shape[0], rng)
    mat[:, 3:6] = rng.uniform(0.3, 0.9, (F.shape[0], 3))        # strong specular
    mat[:, 6] = np.exp(rng.uniform(np.log(0.05), np.log(0.4), F.shape[0]))
    return S.Scene(V.astype(np.float32), F, mat.astype(np.float32), S.hemisphere_lights(2, rng),
                   S.gaussian_lobe_envmap(rng, 64, 32))


def _pair(B, sc):
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    g.set_bsdf_sampler(B.ST_BSDF_SAMPLER_VNDF)
    o.set_vndf(True)
    return g, o


def test_vndf_forward_parity(B):
    _say("case VNDF forward: glossy torus, 2 lights + env, B=3")
    g, o = _pair(B, _scene())
    cams = [S.look_at_origin(e, 40, 32) for e in 3.2 * S.fibonacci_sphere(2)]
    spp = 4
    hh = torch.zeros(B.num_pixels(cams) * spp, dtype=torch.int32, device="cuda")
    img = g.render(cams, spp, 3, seed=3, debug_hash=hh)
    g.check_errors()
    ref, oh = o.render(cams, spp, 3, seed=3)
    fl = (hh.cpu().numpy().view(np.uint32).reshape(-1, spp) != oh.reshape(-1, spp)).any(axis=1)
    bad, checked, worst = radiance_check(img.cpu().numpy(), ref, fl, view_slices(cams))
    _say(f"  flips {fl.mean():.5f} bad {bad}/{checked} worst {worst:.2e}")
    assert fl.mean() < FLIP_MAX and bad == 0


def test_vndf_backward_parity(B):
    _say("case VNDF backward flags=7")
    g, o = _pair(B, _scene())
    cams = [S.look_at_origin((0.4, 1.2, 3.0), 32, 28)]
    spp, bounces, seed, flags = 4, 2, 5, 7
    npath = B.num_pixels(cams) * spp
    ne = B.num_edge_samples(cams, spp, 1.0)
    d_img = np.random.default_rng(5).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    dt = torch.from_numpy(d_img).cuda()
    ph = torch.zeros(npath, dtype=torch.int32, device="cuda")
    eh = torch.zeros(max(ne, 1), dtype=torch.int32, device="cuda")
    g.backward(cams, spp, bounces, dt, seed, flags, debug_hash=ph, debug_edge_hash=eh)
    g.check_errors()
    _, _, oph, oeh = o.backward(cams, spp, bounces, d_img, seed, flags)
    gph = ph.cpu().numpy().view(np.uint32)
    geh = eh.cpu().numpy().view(np.uint32)[:ne]
    pmask = ~((gph != oph) & (oph != 0))
    emask = ~((geh != oeh) & (oeh != 0))
    dV, dM = g.backward(cams, spp, bounces, dt, seed, flags, path_mask=torch.from_numpy(pmask.astype(np.uint8)).cuda(),
                        edge_mask=torch.from_numpy(emask.astype(np.uint8)).cuda())
    torch.cuda.synchronize()
    oV, oM, _, _ = o.backward(cams, spp, bounces, d_img, seed, flags, path_mask=pmask.astype(np.uint8),
                              edge_mask=emask.astype(np.uint8))
    rv, rm = rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM)
    _say(f"  path flips {1 - pmask.mean():.5f} edge flips {1 - emask.mean():.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert 1 - pmask.mean() < FLIP_MAX and 1 - emask.mean() < FLIP_MAX
    assert rv < GRAD_RTOL and rm < GRAD_RTOL


def test_vndf_and_halfvector_estimate_the_same_image(B):
    """Both samplers are unbiased: at 1024 spp the two images of a glossy scene
    agree to within their Monte Carlo error (per-view means)."""
    _say("case VNDF vs half-vector sampler, image means at 1024 spp")
    sc = _scene(22)
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 1.2, 3.0), 32, 32)]
    a = g.render(cams, 1024, 3, seed=1).cpu().numpy().astype(np.float64)
    g.set_bsdf_sampler(B.ST_BSDF_SAMPLER_VNDF)
    b = g.render(cams, 1024, 3, seed=2).cpu().numpy().astype(np.float64)
    ma, mb = a.mean(0), b.mean(0)
    _say(f"  mean rgb half-vector {ma} vnds {mb}")
    assert np.all(np.abs(ma - mb) < 0.01 * np.maximum(ma, 1e-3))

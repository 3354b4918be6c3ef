"""Backward passes that take the main paths' hits and shadow occlusions from the
records of the matching forward pass instead of tracing them again: parity with
the FP64 oracle, agreement with the re-tracing backward (same decisions, same
gradients up to the last bits of the hit distance), and no use of records that
belong to another seed, another camera set or an older scene state."""
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


def _scene(seed=3, nl=2, env=True):
    rng = np.random.default_rng(seed)
    V, F = S.noise_torus(40, 20, 0.1, noise_seed=13)
    lights = S.hemisphere_lights(nl, rng) if nl else np.zeros((0, 6), np.float32)
    return S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), lights,
                   S.gaussian_lobe_envmap(rng, 64, 32) if env else None)


def _grads(B, g, cams, spp, bounces, d, seed, flags, hashes=False):
    npath = B.num_pixels(cams) * spp
    ph = torch.zeros(npath, dtype=torch.int32, device="cuda") if hashes else None
    dV, dM = g.backward(cams, spp, bounces, d, seed, flags, debug_hash=ph)
    torch.cuda.synchronize()
    return dV.cpu().numpy(), dM.cpu().numpy(), (ph.cpu().numpy().view(np.uint32) if hashes else None)


@pytest.mark.parametrize("nl,env", [(2, True), (0, True), (1, False)])
def test_records_match_retrace_and_oracle(B, nl, env):
    """With one shadow entry per shading point (environment only, or one light)
    the forward records occlusion from the shadow kernel itself."""
    _say(f"case hit records: torus 1600 faces, {nl} lights, env {env}, B=3, render then backward")
    sc = _scene(3, nl, env)
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 1.2, 3.0), 32, 28), S.look_at_origin((-2.0, 1.0, 2.2), 24, 24)]
    spp, bounces, seed, flags = 4, 3, 11, 7
    d_img = np.random.default_rng(5).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)
    dt = torch.from_numpy(d_img).cuda()
    g.render(cams, spp, bounces, seed=seed)
    g.read_work()
    g.backward(cams, spp, bounces, dt, seed, flags | B.ST_COUNT_WORK)
    rays_rec = g.read_work()["k_adjoint"][2]
    g.backward(cams, spp, bounces, dt, seed, flags | B.ST_COUNT_WORK | B.ST_BACKWARD_RETRACE)
    rays_retrace = g.read_work()["k_adjoint"][2]
    _say(f"  adjoint rays with records {rays_rec}, re-tracing {rays_retrace}")
    assert rays_rec < 0.5 * rays_retrace             # the main paths were not traced again
    dV_r, dM_r, h_r = _grads(B, g, cams, spp, bounces, dt, seed, flags, hashes=True)
    dV_t, dM_t, h_t = _grads(B, g, cams, spp, bounces, dt, seed, flags | B.ST_BACKWARD_RETRACE, hashes=True)
    assert np.array_equal(h_r, h_t)
    assert rel_l2(dV_r, dV_t) < 1e-5 and rel_l2(dM_r, dM_t) < 1e-5
    # against the oracle (flipped samples masked out of both sides); the records
    # serve the path replay (interior and secondary terms), so those are compared
    flags = 5
    dV_r, dM_r, h_r = _grads(B, g, cams, spp, bounces, dt, seed, flags, hashes=True)
    _, _, oph, _ = o.backward(cams, spp, bounces, d_img, seed, flags)
    pmask = ~((h_r != oph) & (oph != 0))
    g.render(cams, spp, bounces, seed=seed)              # records again for the masked pass
    dV, dM = g.backward(cams, spp, bounces, dt, seed, flags,
                        path_mask=torch.from_numpy(pmask.astype(np.uint8)).cuda())
    torch.cuda.synchronize()
    oV, oM, _, _ = o.backward(cams, spp, bounces, d_img, seed, flags, path_mask=pmask.astype(np.uint8))
    rv, rm = rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM)
    _say(f"  path flips {1 - pmask.mean():.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert 1 - pmask.mean() < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL


def test_records_not_used_across_calls(B):
    """With records of another seed, camera set or scene state the backward traces
    the main paths again (as many adjoint rays as with ST_BACKWARD_RETRACE)."""
    _say("case hit records invalidated by another seed, other cameras and a scene update")
    sc = _scene(4)
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 1.2, 3.0), 24, 24)]
    spp, bounces = 2, 2
    dt = torch.from_numpy(np.random.default_rng(6).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)).cuda()

    def rays(seed, extra=0):
        g.read_work()
        g.backward(cams, spp, bounces, dt, seed, 7 | B.ST_COUNT_WORK | extra)
        return g.read_work()["k_adjoint"][2]

    g.render(cams, spp, bounces, seed=1)
    full = rays(1, B.ST_BACKWARD_RETRACE)
    assert rays(1) < 0.5 * full                                   # matching records are used
    assert rays(2) == rays(2, B.ST_BACKWARD_RETRACE)              # other seed
    g.render([S.look_at_origin((0.5, 1.2, 3.0), 24, 24)], spp, bounces, seed=1)
    assert rays(1) == full                                        # other cameras
    g.render(cams, spp, bounces, seed=1)
    g.update(V=torch.from_numpy(S.perturbed_vertices(sc.V, 0.01, 3)).cuda())
    assert rays(1) == rays(1, B.ST_BACKWARD_RETRACE)              # scene changed

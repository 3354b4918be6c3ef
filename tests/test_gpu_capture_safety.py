"""Captured graphs against later eager calls, through the C ABI.

A graph keeps the device addresses it was captured with.  The library must not
free a workspace such a graph writes into when a later eager call needs a larger
one (the old allocation is retired and freed with the scene), and hit records
written by a graph replay must never be taken by an eager backward of another
forward pass (the key of the pass that wrote them lives in device memory next
to them, and names the buffer).  Each check compares with the re-tracing
backward (ST_BACKWARD_RETRACE) and counts the adjoint's rays to see whether the
records were used."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_03939_amd import scenes as S
from parity_util import rel_l2

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
    V, F = S.noise_torus(40, 20, 0.1, noise_seed=13)
    return S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), S.hemisphere_lights(1, rng),
                   S.gaussian_lobe_envmap(rng, 64, 32))


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                    # sizes the workspaces outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    torch.cuda.synchronize()
    return graph


def _backward_rays(B, g, cams, spp, bounces, d, seed, extra=0):
    g.read_work()
    dV, dM = g.backward(cams, spp, bounces, d, seed, 7 | B.ST_COUNT_WORK | extra)
    torch.cuda.synchronize()
    return dV.cpu().numpy(), dM.cpu().numpy(), g.read_work()["k_adjoint"][2]


def test_records_of_a_replay_are_not_taken_by_another_backward(B):
    _say("case capture render(seed 1), eager render(seed 2), replay, backward(seed 2) and backward(seed 1)")
    g = B.GPUScene.from_scene(_scene())
    cams = [S.look_at_origin((0.4, 1.2, 3.0), 32, 28)]
    spp, bounces = 4, 2
    img = torch.empty((B.num_pixels(cams), 3), device="cuda")
    d = torch.from_numpy(np.random.default_rng(2).normal(size=(B.num_pixels(cams), 3)).astype(np.float32)).cuda()
    graph = _capture(lambda: g.render(cams, spp, bounces, seed=1, out=img))
    g.render(cams, spp, bounces, seed=2)
    graph.replay()
    torch.cuda.synchronize()
    dV, dM, rays = _backward_rays(B, g, cams, spp, bounces, d, 2)
    rV, rM, rays_full = _backward_rays(B, g, cams, spp, bounces, d, 2, B.ST_BACKWARD_RETRACE)
    _say(f"  backward(seed 2) adjoint rays {rays} (re-tracing {rays_full}); relL2 vs re-trace dV "
         f"{rel_l2(dV, rV):.2e} dmat {rel_l2(dM, rM):.2e}")
    assert rays == rays_full
    assert rel_l2(dV, rV) < 1e-5 and rel_l2(dM, rM) < 1e-5
    # the replay's own records do serve the backward of its forward
    dV1, dM1, rays1 = _backward_rays(B, g, cams, spp, bounces, d, 1)
    rV1, rM1, _ = _backward_rays(B, g, cams, spp, bounces, d, 1, B.ST_BACKWARD_RETRACE)
    _say(f"  backward(seed 1) adjoint rays {rays1}; relL2 vs re-trace dV {rel_l2(dV1, rV1):.2e}")
    assert rays1 < 0.5 * rays_full
    assert rel_l2(dV1, rV1) < 1e-5 and rel_l2(dM1, rM1) < 1e-5
    g.check_errors()


def test_workspace_growth_keeps_captured_buffers(B):
    _say("case capture a small render, grow the workspaces with a larger eager render, replay the graph")
    g = B.GPUScene.from_scene(_scene())
    small = [S.look_at_origin((0.4, 1.2, 3.0), 24, 20)]
    large = [S.look_at_origin((0.4, 1.2, 3.0), 64, 64), S.look_at_origin((-2.0, 1.0, 2.2), 48, 48)]
    spp, bounces = 2, 2
    ref = g.render(small, spp, bounces, seed=5).clone()
    img = torch.empty_like(ref)
    graph = _capture(lambda: g.render(small, spp, bounces, seed=5, out=img))
    g.render(large, 4, bounces, seed=6)          # larger radiance, queue and record buffers
    torch.cuda.synchronize()
    for rep in range(3):
        img.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, ref), rep
    d = torch.from_numpy(np.random.default_rng(3).normal(size=(B.num_pixels(small), 3)).astype(np.float32)).cuda()
    dV, dM, rays = _backward_rays(B, g, small, spp, bounces, d, 5)
    rV, rM, rays_full = _backward_rays(B, g, small, spp, bounces, d, 5, B.ST_BACKWARD_RETRACE)
    _say(f"  after the replays: adjoint rays {rays} (re-tracing {rays_full})")
    # the replay wrote its records into the retired buffer: the scene's current
    # one holds the larger render's, so the backward traces again
    assert rays == rays_full
    assert rel_l2(dV, rV) < 1e-5 and rel_l2(dM, rM) < 1e-5
    g.check_errors()


def test_captured_backward_matches_eager(B):
    """Eagerly the adjoint runs on the scene's second stream beside the primary
    edges' side paths; under capture every kernel runs in order on the caller's
    stream.  Replays of a captured backward (records, all gradient terms), with
    eager work and synchronisation between them, equal the eager backward up to
    the order of float atomics."""
    _say("case captured backward (all terms) replayed 3 times against eager backwards")
    sc = _scene()
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.4, 1.2, 3.2), 64, 48), S.look_at_origin((-2.5, 0.8, 2.0), 48, 48)]
    spp, bounces, seed = 4, 2, 9
    img = g.render(cams, spp, bounces, seed).clone()
    d = torch.from_numpy(np.random.default_rng(3).normal(size=tuple(img.shape)).astype(np.float32)).cuda()
    dV = torch.empty((g.nv, 3), dtype=torch.float32, device="cuda")
    dM = torch.empty((g.nf, 7), dtype=torch.float32, device="cuda")

    def bwd():
        g.backward(cams, spp, bounces, d, seed, B.ST_ALL_GRADS, dV=dV, dmat=dM)

    graph = _capture(bwd)
    for rep in range(3):
        g.render(cams, spp, bounces, seed)          # eager work between replays (same records key)
        bwd()
        torch.cuda.synchronize()
        eV, eM = dV.cpu().numpy().copy(), dM.cpu().numpy().copy()
        graph.replay()
        torch.cuda.synchronize()
        rv, rm = rel_l2(dV.cpu().numpy(), eV), rel_l2(dM.cpu().numpy(), eM)
        _say(f"  replay {rep}: relL2 dV {rv:.2e} dmat {rm:.2e}")
        assert np.abs(eV).max() > 0 and rv < 1e-5 and rm < 1e-5
    g.check_errors()

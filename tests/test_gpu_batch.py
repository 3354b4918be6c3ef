"""Batched multi-scene rendering, HIP-graph capture and the autotuner, through the C ABI.

A batched render numbers each camera's random streams by its index among the
cameras of its own scene, so it must equal per-scene renders bit for bit, and
the oracle per scene within the parity tolerance.  Captured graphs are replayed
several times with eager work in between and every replay is checked against
the eager result.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, radiance_check, rel_l2, view_slices

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


def _small_batch():
    rng = np.random.default_rng(2003)
    scs, cams, cs = [], [], []
    for s, k in enumerate((3, 5, 8)):
        V, F = S.noise_sphere(k, 0.1, noise_seed=40 + s)
        mat = S.random_materials(F.shape[0], rng)
        if s % 2 == 0:
            sc = S.Scene(V.astype(np.float32), F, mat, S.hemisphere_lights(2, rng), None, s)
        else:
            sc = S.Scene(V.astype(np.float32), F, mat, np.zeros((0, 6), np.float32), S.gaussian_lobe_envmap(rng, 32, 16), s)
        scs.append(sc)
        for e in 3.0 * S.fibonacci_sphere(2):
            r = int(rng.choice([16, 24, 32]))
            cams.append(S.look_at_origin(e, r, r + 8))
            cs.append(s)
    order = np.random.default_rng(5).permutation(len(cams))      # interleave scenes
    return scs, [cams[i] for i in order], [cs[i] for i in order]


def test_batch_equals_per_scene_renders(B):
    _say("case batch == per-scene renders (3 scenes, 6 uneven views, B=2, 4 spp)")
    scs, cams, cs = _small_batch()
    gs = [B.GPUScene.from_scene(s) for s in scs]
    img = B.render_batch(gs, cams, cs, 4, 2, seed=3).cpu().numpy()
    sl = view_slices(cams)
    for s, g in enumerate(gs):
        idx = [i for i in range(len(cams)) if cs[i] == s]
        ref = g.render([cams[i] for i in idx], 4, 2, seed=3).cpu().numpy()
        got = np.concatenate([img[sl[i]] for i in idx])
        assert np.array_equal(got, ref), s


def test_batch_matches_oracle(B):
    _say("case batch vs oracle per scene")
    scs, cams, cs = _small_batch()
    gs = [B.GPUScene.from_scene(s) for s in scs]
    spp = 4
    hh = torch.zeros(B.num_pixels(cams) * spp, dtype=torch.int32, device="cuda")
    img = B.render_batch(gs, cams, cs, spp, 2, seed=3, debug_hash=hh).cpu().numpy()
    gh = hh.cpu().numpy().view(np.uint32).reshape(-1, spp)
    sl = view_slices(cams)
    for s, sc in enumerate(scs):
        idx = [i for i in range(len(cams)) if cs[i] == s]
        ref, oh = O.OracleScene.from_scene(sc).render([cams[i] for i in idx], spp, 2, seed=3)
        got = np.concatenate([img[sl[i]] for i in idx])
        ghs = np.concatenate([gh[sl[i]] for i in idx])
        flipped = (ghs != oh.reshape(-1, spp)).any(axis=1)
        bad, checked, worst = radiance_check(got, ref, flipped, view_slices([cams[i] for i in idx]))
        _say(f"  scene {s}: flips {flipped.mean():.5f} bad {bad}/{checked} worst {worst:.2e}")
        assert flipped.mean() < FLIP_MAX
        assert bad == 0


def test_graph_capture_replay(B):
    _say("case graph capture of update + render + backward, 3 replays")
    wl = S.small_sphere(res=32, spp=2)
    sc = wl.scenes[0]
    g = B.GPUScene.from_scene(sc)
    V = torch.from_numpy(sc.V).cuda()
    img = torch.empty((B.num_pixels(wl.cams), 3), device="cuda")
    d = torch.from_numpy(np.random.default_rng(1).normal(size=(B.num_pixels(wl.cams), 3)).astype(np.float32)).cuda()
    dV = torch.empty_like(V)
    dM = torch.empty((g.nf, 7), device="cuda")

    def step():
        g.update(V=V)
        g.render(wl.cams, wl.spp, 1, seed=7, out=img)
        g.backward(wl.cams, wl.spp, 1, d, seed=7, flags=B.ST_ALL_GRADS, dV=dV, dmat=dM)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                                   # sizes the workspace outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref_img, ref_dV, ref_dM = img.clone(), dV.clone(), dM.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        img.zero_(); dV.zero_(); dM.zero_()
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()     # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, ref_img), rep
        assert rel_l2(dV.cpu().numpy(), ref_dV.cpu().numpy()) < 1e-5, rep
        assert rel_l2(dM.cpu().numpy(), ref_dM.cpu().numpy()) < 1e-5, rep
    g.check_errors()


def test_autotune_and_cache(B):
    _say("case autotune + cache")
    scs, cams, cs = _small_batch()
    gs = [B.GPUScene.from_scene(s) for s in scs]
    before = B.render_batch(gs, cams, cs, 4, 2, seed=3).cpu().numpy()
    path = os.path.join(tempfile.mkdtemp(), "tune.jsonl")
    cap, grid = B.autotune(gs, cams, 4, 2, cam_scene=cs, cache_path=path)
    assert cap >= (1 << 20) and grid in (1024, 2048, 4096)
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 1 and '"queue_capacity": %d' % cap in lines[0]
    cap2, grid2 = B.autotune(gs, cams, 4, 2, cam_scene=cs, cache_path=path)
    assert (cap2, grid2) == (cap, grid) and len(open(path).read().strip().splitlines()) == 1
    after = B.render_batch(gs, cams, cs, 4, 2, seed=3).cpu().numpy()
    assert np.array_equal(before, after)

"""Traversal work counters (ST_COUNT_WORK): the wavefront closest-hit kernel and
the single-kernel forward trace the same camera rays through the same traversal
(direct light off, no environment, one bounce), so their node-visit, triangle-test
and ray counts agree exactly, and the per-ray figures are plausible for a 4-wide
BVH over a 40k-face mesh (a counter that reported, say, the iteration cap for
every ray would fail here)."""
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


def test_wavefront_and_megakernel_count_the_same_work(B):
    _say("case work counters: torus 40k faces, camera rays only, wavefront vs megakernel")
    rng = np.random.default_rng(4)
    V, F = S.noise_torus(200, 100, 0.1, noise_seed=13)
    sc = S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), np.zeros((0, 6), np.float32), None)
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.5, 2.5, 3.0), 96, 80), S.look_at_origin((-3.0, 0.4, 1.5), 64, 64)]
    spp = 2
    g.read_work()
    g.render(cams, spp, 1, seed=3, flags=B.ST_COUNT_WORK)
    torch.cuda.synchronize()
    w = g.read_work()
    g.render(cams, spp, 1, seed=3, flags=B.ST_COUNT_WORK | B.ST_FORWARD_MEGAKERNEL)
    torch.cuda.synchronize()
    m = g.read_work()
    g.check_errors()
    ext, mega = w["k_extend"], m["k_forward_mega"]
    npath = B.num_pixels(cams) * spp
    _say(f"  wavefront {ext}  megakernel {mega}  paths {npath}")
    assert ext == mega
    visits, tests, rays = ext
    assert rays == npath
    assert 1.0 <= visits / rays <= 64.0 and 0.0 < tests / rays <= 32.0


def test_paired_launch_counts_its_rays(B):
    """With an environment map every bounce's shadow rays are traced in one
    launch with the next bounce's extension rays: the paired launch's own rays
    are then all extension rays but the camera rays, plus every shadow ray,
    and its visits and tests are at most the two kinds' totals."""
    _say("case work counters: torus 40k faces, environment map, 2 bounces, paired launches")
    rng = np.random.default_rng(5)
    V, F = S.noise_torus(200, 100, 0.1, noise_seed=13)
    env = S.gaussian_lobe_envmap(rng, 64, 32)
    sc = S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), np.zeros((0, 6), np.float32), env)
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.5, 2.5, 3.0), 96, 80), S.look_at_origin((-3.0, 0.4, 1.5), 64, 64)]
    spp = 2
    g.read_work()
    g.render(cams, spp, 2, seed=3, flags=B.ST_COUNT_WORK)
    torch.cuda.synchronize()
    w = g.read_work()
    g.check_errors()
    ext, sh, pair = w["k_extend"], w["k_shadow"], w["k_trace_pair"]
    npath = B.num_pixels(cams) * spp
    _say(f"  extension {ext}  shadow {sh}  paired {pair}  paths {npath}")
    assert ext[2] > npath and sh[2] > 0
    assert pair[2] == ext[2] - npath + sh[2]
    assert pair[0] <= ext[0] + sh[0] and pair[1] <= ext[1] + sh[1]
    assert pair[0] >= sh[0]

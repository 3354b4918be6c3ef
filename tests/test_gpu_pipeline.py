"""Pipeline steps around the renderer (Sec. 3.2 "Subdivision"; the coarse-to-fine
schedule) through the C ABI: the GPU 1 -> 4 subdivision is bit-exact against the
oracle's definition-level subdivision, and a short coarse-to-fine optimisation
runs through three mesh resolutions with the loss going down."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
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


@pytest.mark.parametrize("which", ["sphere320", "torus40k_moved"])
def test_subdivide_bit_exact(B, which):
    _say(f"case subdivision {which}")
    if which == "sphere320":
        V, F = S.geodesic_sphere(4)
        V = V.astype(np.float32)
        sc = S.Scene(V, F, S.uniform_materials(F.shape[0]), np.zeros((0, 6), np.float32), None)
        g = B.GPUScene.from_scene(sc)
    else:
        wl = S.torus_envmap(res=64, nviews=1, spp=1, bounces=1)
        sc = wl.scenes[0]
        g = B.GPUScene.from_scene(sc)
        V = S.perturbed_vertices(sc.V, 0.01, 5)          # subdivision uses the updated vertices
        g.update(V=torch.from_numpy(V).cuda())
        F = sc.F
    Vg, Fg = g.subdivide()
    torch.cuda.synchronize()
    Vo, Fo = O.subdivide(V, F)
    assert np.array_equal(Fg.cpu().numpy(), Fo)
    assert np.array_equal(Vg.cpu().numpy().view(np.uint32), Vo.view(np.uint32))
    # the subdivided mesh is a valid scene again
    g2 = B.GPUScene(Vg, Fg, S.uniform_materials(Fg.shape[0]), None, np.ones((8, 16, 3), np.float32))
    assert g2.nf == 4 * F.shape[0]


def test_coarse_to_fine_optimisation(B):
    _say("case coarse-to-fine: 320 -> 1280 -> 5120 faces, 12 steps each, 8 views at 64^2")
    from paper_2012_03939_amd.optimise import run
    r = run(steps=12, nviews=8, res=64, spp=4, bounces=2, target_spp=16, subdivisions=2)
    _say(f"  {r}")
    assert r["faces_per_level"] == [320, 1280, 5120]
    assert r["image_l2_last"] < 0.9 * r["image_l2_first"]


def test_experiment_gi_planes(B):
    """Sec. 3.3: with global illumination the optimised floor albedo is close to the
    true white; the one-bounce renderer explains the light bled from the red and
    blue walls by a wrong floor albedo."""
    _say("case experiment: three planes, albedo from GI vs one-bounce renders")
    from paper_2012_03939_amd.experiments import gi_planes
    r = gi_planes(steps=80, res=64, spp=8)
    _say(f"  {r}")
    gi, ob = r["global_illumination"], r["one_bounce"]
    assert gi["floor"]["abs_error"] < 0.05
    assert ob["floor"]["abs_error"] > 2 * gi["floor"]["abs_error"]


def test_experiment_divot_shape_from_shading(B):
    """Sec. 3.2: a divot invisible in silhouette is pushed in from shading alone."""
    _say("case experiment: sphere with a divot, 5 cameras x 4 lights")
    from paper_2012_03939_amd.experiments import divot
    r = divot(steps=300, res=64, spp=32, k=16)
    _say(f"  {r}")
    assert r["recovered_fraction"] > 0.3
    assert r["silhouette_radius_change"] < 0.05
    assert r["image_l2_last"] < 0.5 * r["image_l2_first"]

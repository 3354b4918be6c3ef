"""The allocation-free render (st_render_noalloc) against st_render, through the
C ABI: the same image bit for bit on two calls in a row, the second with a
smaller input, free device memory unchanged across the calls, and the limits
rejected before any launch."""
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
    rng = np.random.default_rng(41)
    V, F = S.noise_sphere(10, 0.1, noise_seed=5)
    return S.Scene(V.astype(np.float32), F, S.random_materials(F.shape[0], rng), S.hemisphere_lights(2, rng),
                   S.gaussian_lobe_envmap(rng, 64, 32))


def test_noalloc_render_equals_render(B):
    _say("case st_render_noalloc vs st_render: 2 views 96x80 + 64x64 at 8 spp, then 1 view 40x32 at 2 spp")
    g = B.GPUScene.from_scene(_scene())
    first = [S.look_at_origin((0.3, 0.5, 3.0), 96, 80), S.look_at_origin((-2.0, 1.0, 2.0), 64, 64)]
    second = [S.look_at_origin((1.0, -0.5, 2.8), 40, 32)]
    out1 = torch.full((B.num_pixels(first), 3), -1.0, device="cuda")
    out2 = torch.full((B.num_pixels(second), 3), -1.0, device="cuda")
    g.render_noalloc(first, 8, 3, seed=1, out=out1)       # warm-up (the runtime's own launch resources)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    g.render_noalloc(first, 8, 3, seed=4, out=out1)
    g.render_noalloc(second, 2, 2, seed=9, out=out2)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _say(f"  free device memory before {free0} after {free1}")
    assert free1 == free0
    ref1 = g.render(first, 8, 3, seed=4)
    ref2 = g.render(second, 2, 2, seed=9)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    assert torch.equal(out2, ref2)
    assert float(ref1.max()) > 0
    g.check_errors()


def test_noalloc_render_single_kernel_forward_and_hashes(B):
    _say("case st_render_noalloc with the single-kernel forward and decision hashes")
    g = B.GPUScene.from_scene(_scene())
    cams = [S.look_at_origin((0.3, 0.5, 3.0), 48, 40)]
    n = B.num_pixels(cams) * 4
    h1 = torch.zeros(n, dtype=torch.int32, device="cuda")
    h2 = torch.zeros(n, dtype=torch.int32, device="cuda")
    a = g.render_noalloc(cams, 4, 2, seed=2, debug_hash=h1)
    b = g.render(cams, 4, 2, seed=2, debug_hash=h2)
    c = g.render_noalloc(cams, 4, 2, seed=2, flags=B.ST_FORWARD_MEGAKERNEL)
    d = g.render(cams, 4, 2, seed=2, flags=B.ST_FORWARD_MEGAKERNEL)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(h1, h2) and torch.equal(c, d)
    g.check_errors()


def test_noalloc_limits(B):
    _say("case st_render_noalloc limits: path samples and cameras")
    g = B.GPUScene.from_scene(_scene())
    with pytest.raises(B.StError, match="static scratch limit"):
        g.render_noalloc([S.look_at_origin((0.3, 0.5, 3.0), 512, 512)], 8, 2)
    with pytest.raises(B.StError, match="at most 64 cameras"):
        g.render_noalloc([S.look_at_origin((0.3, 0.5, 3.0), 4, 4)] * 65, 1, 1)
    g.check_errors()

"""Secondary-edge samples deferred to a job pass (the default when no decision
hashes are requested) against the inline form (used when they are): the same
side paths are traced and the gradients agree to float rounding, for the
secondary term alone, with the interior term, and with crease/material edges."""
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


@pytest.mark.parametrize("flags", [4, 5, 4 | 64, 4 | 256, 5 | 64 | 256])
def test_deferred_equals_inline(B, flags):
    _say(f"case secondary edges deferred vs inline, flags={flags}")
    rng = np.random.default_rng(12)
    V, F = S.noise_sphere(8, 0.15, noise_seed=2)
    floor = np.array([[-3, -1.3, -3], [3, -1.3, -3], [3, -1.3, 3], [-3, -1.3, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    sc = S.Scene(Vf, Ff, S.random_materials(Ff.shape[0], rng), S.hemisphere_lights(2, rng),
                 S.gaussian_lobe_envmap(rng, 64, 32))
    g = B.GPUScene.from_scene(sc)
    cams = [S.look_at_origin((0.3, 0.9, 3.1), 48, 48), S.look_at_origin((-2.0, 1.5, 2.0), 40, 40)]
    spp, bounces, seed = 8, 3, 4
    dt = torch.from_numpy(rng.normal(size=(B.num_pixels(cams), 3)).astype(np.float32)).cuda()
    hb = torch.zeros(B.num_pixels(cams) * spp, dtype=torch.int32, device="cuda")
    g.read_work()
    dV_i, dM_i = g.backward(cams, spp, bounces, dt, seed, flags | B.ST_COUNT_WORK, debug_hash=hb)   # inline
    torch.cuda.synchronize()
    rays_i = g.read_work()["k_adjoint"][2]
    dV_i, dM_i = dV_i.cpu().numpy().copy(), dM_i.cpu().numpy().copy()
    dV_d, dM_d = g.backward(cams, spp, bounces, dt, seed, flags | B.ST_COUNT_WORK)                  # deferred
    torch.cuda.synchronize()
    rays_d = g.read_work()["k_adjoint"][2]
    g.check_errors()
    rv, rm = rel_l2(dV_d.cpu().numpy(), dV_i), rel_l2(dM_d.cpu().numpy(), dM_i)
    _say(f"  adjoint rays inline {rays_i} deferred {rays_d}; relL2 dV {rv:.2e} dmat {rm:.2e}; |dV| {np.abs(dV_i).max():.3g}")
    assert np.abs(dV_i).max() > 0
    assert rv < 1e-5 and rm < 1e-5
    # the job pass replays each job's path up to its vertex again: the side-path rays
    # are the same, the replayed main-path rays come on top
    assert rays_d >= rays_i

"""Secondary edges at creases and material boundaries (ST_EDGE_SECONDARY_INTERIOR):
a glossy floor reflects a two-tone wall; moving the wall's interior vertex bends
the red/blue boundary, which the camera sees directly (primary edges) and in the
reflection (direction-space edges that are not silhouettes).  Free central
differences of the renderer agree with the adjoint only when those edges are
sampled; the option is also checked against the FP64 oracle."""
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


def _two_tone_wall_over_glossy_floor(res=48):
    fl = np.array([[-3, -3, 0], [3, -3, 0], [3, 3, 0], [-3, 3, 0]], np.float32)
    wv = np.array([[x, 1.5, z] for z in (0.2, 0.8, 1.4) for x in (-1.0, 0.0, 1.0)], np.float32)
    V = np.concatenate([fl, wv])
    F = [[0, 1, 2], [0, 2, 3]]
    for j in range(2):
        for i in range(2):
            a, b, c, d = 4 + 3 * j + i, 5 + 3 * j + i, 7 + 3 * j + i, 8 + 3 * j + i
            F += [[a, b, d], [a, d, c]]
    F = np.array(F, np.int32)
    mat = np.zeros((F.shape[0], 7), np.float32)
    mat[:2, :3], mat[:2, 3:6], mat[:2, 6] = 0.05, 0.9, 0.05            # glossy floor
    cen = V[F].mean(1)
    for f in range(2, F.shape[0]):
        mat[f, :3] = (0.9, 0.1, 0.1) if cen[f, 0] < 0 else (0.1, 0.1, 0.9)
        mat[f, 6] = 0.5
    sc = S.Scene(V, F, mat, np.zeros((0, 6), np.float32), np.ones((8, 16, 3), np.float32))
    cam = S.Camera((0.0, -1.2, 1.0), (0.0, 0.8, 0.0), (0, 0, 1), 50.0, res, res)
    delta = np.zeros_like(V)
    delta[8, 0] = 1.0                     # the wall's interior vertex, along the wall
    return sc, cam, delta


def test_secondary_interior_edges_vs_central_differences(B):
    _say("case crease/material secondary edges: FD vs adjoint with and without, 32 seeds x 64 spp")
    sc, cam, delta = _two_tone_wall_over_glossy_floor()
    g = B.GPUScene.from_scene(sc)
    w = torch.zeros((48 * 48, 3), device="cuda")
    w[:, 0] = 1.0                         # red channel: the two materials differ there
    V0 = torch.from_numpy(sc.V).cuda()
    dl = torch.from_numpy(delta).cuda()
    h, spp = 5e-3, 64
    fd, ad, an = [], [], []
    for s in range(32):
        g.update(V=V0 + h * dl)
        lp = float((g.render([cam], spp, 2, seed=s) * w).sum())
        g.update(V=V0 - h * dl)
        lm = float((g.render([cam], spp, 2, seed=s) * w).sum())
        g.update(V=V0)
        fd.append((lp - lm) / (2 * h))
        ad.append(float((g.backward([cam], spp, 2, w, seed=s, flags=15 | B.ST_EDGE_SECONDARY_INTERIOR)[0] * dl).sum()))
        an.append(float((g.backward([cam], spp, 2, w, seed=s, flags=15)[0] * dl).sum()))
    fd, ad, an = map(np.array, (fd, ad, an))
    se = (fd - ad).std(ddof=1) / np.sqrt(len(fd))
    sn = (fd - an).std(ddof=1) / np.sqrt(len(fd))
    _say(f"  FD {fd.mean():.2f}  with interior edges {ad.mean():.2f} (diff se {se:.2f})  without {an.mean():.2f}")
    assert abs((fd - ad).mean()) < 4 * se + 0.03 * abs(fd.mean())
    assert abs((fd - an).mean()) > 6 * sn


def test_secondary_interior_edges_parity(B):
    _say("case crease/material secondary edges vs oracle")
    sc, cam, _ = _two_tone_wall_over_glossy_floor(res=32)
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    flags = 1 | 4 | B.ST_EDGE_SECONDARY_INTERIOR
    spp, bounces = 8, 2
    d_img = np.random.default_rng(3).normal(size=(32 * 32, 3)).astype(np.float32)
    dt = torch.from_numpy(d_img).cuda()
    ph = torch.zeros(32 * 32 * spp, dtype=torch.int32, device="cuda")
    g.backward([cam], spp, bounces, dt, 2, flags, debug_hash=ph)
    g.check_errors()
    _, _, oph, _ = o.backward([cam], spp, bounces, d_img, 2, flags)
    pmask = ~((ph.cpu().numpy().view(np.uint32) != oph) & (oph != 0))
    dV, dM = g.backward([cam], spp, bounces, dt, 2, flags, path_mask=torch.from_numpy(pmask.astype(np.uint8)).cuda())
    torch.cuda.synchronize()
    oV, oM, _, _ = o.backward([cam], spp, bounces, d_img, 2, flags, path_mask=pmask.astype(np.uint8))
    rv, rm = rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM)
    _say(f"  path flips {1 - pmask.mean():.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert 1 - pmask.mean() < FLIP_MAX and rv < GRAD_RTOL and rm < GRAD_RTOL and np.abs(oV).max() > 0

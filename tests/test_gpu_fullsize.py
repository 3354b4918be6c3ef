"""Parity at the full workload sizes, in the launch configuration the benchmark
times (default options): the GPU renders / differentiates everything, the FP64
oracle computes sampled pixels one by one (forward) or the gradient of a loss
whose image gradient is non-zero on a sparse random pixel set (backward; the
oracle skips path and edge samples whose pixel has a zero image gradient, which
contribute exactly zero), and, for the 8-view point-light ring, on every pixel."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2012_03939_amd import scenes as S
from parity_util import FLIP_MAX, GRAD_RTOL, RAD_RTOL, rel_l2

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


def _pick_pixels(cams, n, seed):
    rng = np.random.default_rng(seed)
    off = np.cumsum([0] + [c.width * c.height for c in cams])
    g = np.sort(rng.choice(off[-1], size=n, replace=False))
    view = np.searchsorted(off, g, side="right") - 1
    return g, np.stack([view, g - off[view]], 1)


def _forward_sampled(B, wl, npix_check, seed=0):
    sc = wl.scenes[0]
    g = B.GPUScene.from_scene(sc)
    npix = B.num_pixels(wl.cams)
    hh = torch.zeros(npix * wl.spp, dtype=torch.int32, device="cuda")
    img = g.render(wl.cams, wl.spp, wl.bounces, seed, debug_hash=hh)
    g.check_errors()
    gidx, pix = _pick_pixels(wl.cams, npix_check, 123)
    o = O.OracleScene.from_scene(sc)
    rgb, oh = o.render_samples(wl.cams, wl.spp, wl.bounces, seed, pix=pix)
    ref = rgb.mean(axis=1)
    gh = hh.cpu().numpy().view(np.uint32).reshape(npix, wl.spp)[gidx]
    flipped = (gh != oh).any(axis=1)
    got = img.cpu().numpy()[gidx].astype(np.float64)
    floor = 1e-3 * np.maximum(ref.mean(axis=0), 1e-12)
    err = (np.abs(got - ref) / np.maximum(np.abs(ref), floor[None, :])).max(axis=1)
    return flipped.mean(), int((err[~flipped] > RAD_RTOL).sum()), float(err[~flipped].max()), ref


def test_fullsize_forward_noise_sphere_ring(B):
    _say("case fullsize forward: 9680-face noise sphere, 8x256^2, 16 spp, B=2, 3 point lights")
    wl = S.noise_sphere_ring()
    fr, bad, worst, ref = _forward_sampled(B, wl, 2000)
    _say(f"  flips {fr:.5f} bad {bad} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0
    assert (ref.max(axis=1) > 0).mean() > 0.2


def test_fullsize_forward_torus_bench_config(B):
    _say("case fullsize forward: 40k torus, env 512x256, 16x512^2, 16 spp, B=3")
    wl = S.torus_envmap(res=512, nviews=16, spp=16, bounces=3)
    fr, bad, worst, ref = _forward_sampled(B, wl, 1500)
    _say(f"  flips {fr:.5f} bad {bad} worst {worst:.2e}")
    assert fr < FLIP_MAX and bad == 0


def _backward_parity(B, wl, d_img, flags, seed=0):
    """GPU and oracle backward of the same image gradient, with every path and
    edge sample's decision hash compared; flipped samples (where the hashes
    differ) are masked out of both passes before the gradients are compared.
    When nothing flipped the first pass is already the masked one."""
    sc = wl.scenes[0]
    cams, spp, bounces = wl.cams, wl.spp, wl.bounces
    npix = B.num_pixels(cams)
    nl = int(sc.lights.shape[0]) if flags & B.ST_EDGE_SHADOW else 0
    ne = B.num_edge_samples(cams, spp, 1.0, nl)
    g = B.GPUScene.from_scene(sc)
    o = O.OracleScene.from_scene(sc)
    dt = torch.from_numpy(d_img).cuda()
    ph = torch.zeros(npix * spp, dtype=torch.int32, device="cuda")
    eh = torch.zeros(max(ne, 1), dtype=torch.int32, device="cuda")
    dV, dM = g.backward(cams, spp, bounces, dt, seed, flags, 1.0, debug_hash=ph, debug_edge_hash=eh)
    g.check_errors()
    _say("  gpu backward done")
    oV, oM, oph, oeh = o.backward(cams, spp, bounces, d_img, seed, flags, 1.0)
    _say("  oracle backward done")
    gph = ph.cpu().numpy().view(np.uint32)
    geh = eh.cpu().numpy().view(np.uint32)[:ne]
    assert oeh.shape == (ne,)
    pmask = ~((gph != oph) & (oph != 0))
    emask = ~((geh != oeh) & (oeh != 0))
    n_paths = int((oph != 0).sum())
    n_edges = int((oeh != 0).sum())
    pflip = float((~pmask).sum()) / max(n_paths, 1)
    eflip = float((~emask).sum()) / max(n_edges, 1)
    del ph, eh
    if not (pmask.all() and emask.all()):
        dV, dM = g.backward(cams, spp, bounces, dt, seed, flags, 1.0,
                            path_mask=torch.from_numpy(pmask.astype(np.uint8)).cuda(),
                            edge_mask=torch.from_numpy(emask.astype(np.uint8)).cuda())
        torch.cuda.synchronize()
        oV, oM, _, _ = o.backward(cams, spp, bounces, d_img, seed, flags, 1.0, path_mask=pmask.astype(np.uint8),
                                  edge_mask=emask.astype(np.uint8))
        _say("  masked passes done")
    return pflip, eflip, n_paths, n_edges, rel_l2(dV.cpu().numpy(), oV), rel_l2(dM.cpu().numpy(), oM), oV


def _sparse_d_image(B, cams, n_active):
    gidx, _ = _pick_pixels(cams, n_active, 321)
    d_img = np.zeros((B.num_pixels(cams), 3), np.float32)
    d_img[gidx] = np.random.default_rng(9).normal(size=(n_active, 3)).astype(np.float32)
    return d_img


def test_fullsize_backward_torus_bench_config(B):
    _say("case fullsize backward: 40k torus, env, 16x512^2, 16 spp, B=3, flags 15 (library default), "
         "200 active pixels")
    wl = S.torus_envmap(res=512, nviews=16, spp=16, bounces=3)
    pf, ef, npth, ned, rv, rm, _ = _backward_parity(B, wl, _sparse_d_image(B, wl.cams, 200), B.ST_ALL_GRADS)
    _say(f"  paths {npth} edges {ned} path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert npth > 1000 and ned > 10
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert rv < GRAD_RTOL and rm < GRAD_RTOL


def test_fullsize_backward_noise_sphere_ring(B):
    _say("case fullsize backward: 9680-face noise sphere ring, 8x256^2, 16 spp, B=2, 3 point lights, "
         "flags 15 (with shadow boundaries), 300 active pixels")
    wl = S.noise_sphere_ring()
    pf, ef, npth, ned, rv, rm, _ = _backward_parity(B, wl, _sparse_d_image(B, wl.cams, 300), B.ST_ALL_GRADS)
    _say(f"  paths {npth} edges {ned} path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert npth > 1000 and ned > 10
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert rv < GRAD_RTOL and rm < GRAD_RTOL


def test_fullsize_backward_noise_sphere_ring_dense(B):
    """Every pixel of the 8 views carries an image gradient: all 8,388,608 path
    samples, as many primary edge samples and 3 x as many shadow-boundary
    samples enter both gradients."""
    _say("case fullsize backward dense: 9680-face noise sphere ring, 8x256^2, 16 spp, B=2, 3 point lights, "
         "flags 15, d_image non-zero at every pixel")
    wl = S.noise_sphere_ring()
    npix = B.num_pixels(wl.cams)
    d_img = np.random.default_rng(10).normal(size=(npix, 3)).astype(np.float32)
    pf, ef, npth, ned, rv, rm, oV = _backward_parity(B, wl, d_img, B.ST_ALL_GRADS)
    _say(f"  paths {npth} edges {ned} path flips {pf:.5f} edge flips {ef:.5f} relL2 dV {rv:.2e} dmat {rm:.2e}")
    assert npth == npix * wl.spp
    assert pf < FLIP_MAX and ef < FLIP_MAX
    assert rv < GRAD_RTOL and rm < GRAD_RTOL
    assert (np.abs(oV).sum(axis=1) > 0).mean() > 0.5

"""torch.autograd binding of the renderer R(x, m, c_i) (Shape from Tracing, Sec. 3.2 and 3.3).

`render(V, mat, scene, cams, spp, bounces, seed)` returns the image and, on
backward, calls the library's adjoint with the image gradient.  The loss of
Sec. 3.2 (mean squared error against targets whose background is black) and the
smoothness prior are ordinary torch code on top of it.
"""
from __future__ import annotations

import torch

from . import binding as B


class RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, mat, scene: "B.GPUScene", cams, spp: int, bounces: int, seed: int, flags: int):
        V = V.detach().contiguous()
        mat = mat.detach().contiguous()
        scene.update(V=V, mat=mat)
        ctx.scene = scene
        ctx.args = (cams, spp, bounces, seed, flags)
        ctx.state = (V, mat)
        ctx.version = scene.version
        return scene.render(cams, spp, bounces, seed)

    @staticmethod
    def backward(ctx, d_img):
        scene = ctx.scene
        cams, spp, bounces, seed, flags = ctx.args
        if scene.version != ctx.version:          # the scene was re-rendered with other parameters since
            scene.update(V=ctx.state[0], mat=ctx.state[1])
        dV, dmat = scene.backward(cams, spp, bounces, d_img.contiguous(), seed, flags)
        return dV, dmat, None, None, None, None, None, None


def render(V, mat, scene, cams, spp: int, bounces: int, seed: int = 0, flags: int = B.ST_ALL_GRADS):
    return RenderFn.apply(V, mat, scene, cams, spp, bounces, seed, flags)


def vertex_neighbours(F: torch.Tensor, nv: int):
    """Undirected edge list (i, j) of a triangle mesh, both directions."""
    e = torch.cat([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0).long()
    e = torch.cat([e, e.flip(1)], 0)
    e = torch.unique(e, dim=0)
    return e[:, 0], e[:, 1]


def uniform_laplacian(V: torch.Tensor, src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """Mean squared norm of the uniform Laplacian: V_i minus the mean of its neighbours."""
    nv = V.shape[0]
    deg = torch.zeros(nv, device=V.device, dtype=V.dtype).index_add_(0, src, torch.ones_like(src, dtype=V.dtype))
    acc = torch.zeros_like(V).index_add_(0, src, V[dst])
    lap = V - acc / deg.clamp_min(1.0)[:, None]
    return (lap * lap).sum(1).mean()

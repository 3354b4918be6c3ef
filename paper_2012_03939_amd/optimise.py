"""Joint refinement of vertex positions and per-face materials by gradient descent
through the path tracer (Shape from Tracing, Sec. 3.2 "Vertex optimization" and
Sec. 3.3 "Material Optimization"; the loss is the mean squared error of Sec. 3.2
with a black background standing for the masks).

The synthetic problem: targets are 32 views at 256x256 of a 100,820-face noise
sphere with random per-face materials under an HDR environment map; the start is
a 5,120-face sphere with a uniform grey material.  Adam (lr 1e-3 vertices, 1e-2
materials), uniform-Laplacian smoothness weighted 0.1, 8 spp, 2 bounces.

With tex_res = r > 0 the materials are mesh colours of resolution r (Sec. 3.3
"Representation"), started from the grey material in every texel, and
spec_var_w > 0 adds the Sec. 3.3 specular variance penalty
spec_var_w * Var(m_s): the variance over texels of each specular channel,
summed over the three channels.  With subdivisions = s > 0 the schedule is
coarse to fine (Sec. 3.2 "Subdivision"): the start mesh is the k = 4 sphere
(320 faces), every `steps` iterations the current mesh is subdivided 1 -> 4 on
the GPU (st_scene_subdivide) into a new scene, and the materials restart from
the neutral grey (Sec. 3.3: re-optimised after every topology change), s times.

With checkpoint=PATH and checkpoint_every=n the state (vertices, faces,
materials, Adam moments, level, step, loss history) is written every n steps;
resume=True continues from it at the next step with the same per-step seeds
(a reconstruction runs for hours: Sec. 3.4 "Optimization Details" alternates
long material and geometry phases).

    python -m paper_2012_03939_amd.optimise --steps 200 [--checkpoint ckpt.pt --checkpoint-every 20 [--resume]]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import binding as B
from . import scenes as S
from .autograd import render, uniform_laplacian, vertex_neighbours


CHECKPOINT_FORMAT = 1


def _cpu(obj):
    if torch.is_tensor(obj):
        return obj.detach().cpu()
    if isinstance(obj, dict):
        return {k: _cpu(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return type(obj)(_cpu(v) for v in obj)
    return obj


def save_checkpoint(path: str, level: int, step: int, V, M, F, opt, history: dict) -> None:
    """Optimisation state after `step` of `level`: vertices, faces, material rows,
    the optimiser's state (Adam moments and step counts), the per-step losses and
    times so far.  Written to a temporary file, then renamed over `path`."""
    state = {"format": CHECKPOINT_FORMAT, "level": int(level), "step": int(step), "V": _cpu(V), "M": _cpu(M),
             "F": _cpu(F), "opt": _cpu(opt.state_dict()),
             "history": {k: [float(x) if not isinstance(x, int) else x for x in v] for k, v in history.items()}}
    tmp = path + ".tmp"
    torch.save(state, tmp)
    os.replace(tmp, path)


def load_checkpoint(path: str) -> dict:
    """The state save_checkpoint wrote (tensors on the CPU; loaded without
    executing anything from the file)."""
    state = torch.load(path, map_location="cpu", weights_only=True)
    if state.get("format") != CHECKPOINT_FORMAT:
        raise ValueError(f"{path}: not an optimisation checkpoint of format {CHECKPOINT_FORMAT}")
    return state


def run(steps: int = 200, nviews: int = 32, res: int = 256, spp: int = 8, bounces: int = 2, target_spp: int = 64,
        lr_v: float = 1e-3, lr_m: float = 1e-2, lap_w: float = 0.1, log_every: int = 0, tex_res: int = 0,
        spec_var_w: float = 0.0, subdivisions: int = 0, checkpoint: str | None = None, checkpoint_every: int = 0,
        resume: bool = False, return_params: bool = False) -> dict:
    dev = torch.device("cuda")
    target_sc, start_sc, cams = S.optimisation_problem(nviews, res)
    gt = B.GPUScene.from_scene(target_sc)
    T = gt.render(cams, target_spp, bounces, seed=12345).clone()
    gt.close()
    if subdivisions > 0:
        Vs, Fs = S.geodesic_sphere(4)
        start_sc = S.Scene(Vs.astype(np.float32), Fs, S.uniform_materials(Fs.shape[0]), start_sc.lights, start_sc.env,
                           start_sc.scene_id)
    times, l2, faces = [], [], []
    ck = load_checkpoint(checkpoint) if (resume and checkpoint and os.path.exists(checkpoint)) else None
    first_level = 0
    if ck is not None:
        first_level = ck["level"]
        times, l2 = list(ck["history"]["times"]), list(ck["history"]["l2"])
        faces = [int(x) for x in ck["history"]["faces"]]
    for level in range(first_level, subdivisions + 1):
        from_ck = ck is not None and level == first_level
        if from_ck:
            # the mesh and materials of the checkpoint (a per-face placeholder
            # material creates the scene; mesh colours replace it below)
            Fk = ck["F"].numpy().astype(np.int32)
            start_sc = S.Scene(ck["V"].numpy().astype(np.float32), Fk, S.uniform_materials(int(Fk.shape[0])),
                               start_sc.lights, start_sc.env, start_sc.scene_id)
            faces = faces[:-1]
        elif level > 0:
            with torch.no_grad():
                g.update(V=V.detach().contiguous())
                Vn, Fn = g.subdivide()
            grey = S.uniform_materials(int(Fn.shape[0]))
            start_sc = S.Scene(Vn.cpu().numpy(), Fn.cpu().numpy(), grey, start_sc.lights, start_sc.env,
                               start_sc.scene_id)
            g.close()
        g = B.GPUScene.from_scene(start_sc)
        # wavefront chunk size and traversal grid for this workload (timed renders)
        B.autotune([g], cams, spp, bounces)
        V = torch.tensor(start_sc.V, device=dev, requires_grad=True)
        mat0 = start_sc.mat
        if from_ck:
            mat0 = ck["M"].numpy().astype(np.float32)
        elif tex_res > 0:
            mat0 = np.repeat(start_sc.mat, (tex_res + 1) * (tex_res + 2) // 2, axis=0)
        if tex_res > 0:
            g.set_mesh_colors(tex_res, torch.from_numpy(mat0).to(dev))
        M = torch.tensor(mat0, device=dev, requires_grad=True)
        F = torch.from_numpy(start_sc.F).to(dev)
        src, dst = vertex_neighbours(F, V.shape[0])
        opt = torch.optim.Adam([{"params": [V], "lr": lr_v}, {"params": [M], "lr": lr_m}])
        first_it = 0
        if from_ck:
            opt.load_state_dict(ck["opt"])
            first_it = ck["step"] + 1
        faces.append(int(F.shape[0]))
        for it in range(first_it, steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            opt.zero_grad(set_to_none=True)
            img = render(V, M, g, cams, spp, bounces, seed=level * steps + it)
            img_l2 = ((img - T) ** 2).mean()
            loss = img_l2 + lap_w * uniform_laplacian(V, src, dst)
            if spec_var_w > 0.0:
                loss = loss + spec_var_w * M[:, 3:6].var(dim=0, unbiased=False).sum()
            loss.backward()
            opt.step()
            with torch.no_grad():
                M[:, :6].clamp_(0.0, 1.0)
                M[:, 6].clamp_(0.01, 1.0)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            l2.append(float(img_l2.detach()))
            if log_every and it % log_every == 0:
                print(json.dumps({"level": level, "step": it, "image_l2": l2[-1], "s": times[-1]}), flush=True)
            if checkpoint and checkpoint_every and (it + 1) % checkpoint_every == 0:
                save_checkpoint(checkpoint, level, it, V, M, F, opt, {"times": times, "l2": l2, "faces": faces})
    g.check_errors()
    warm = times[2:] if len(times) > 4 else times
    out = {"steps": steps * (subdivisions + 1), "s_per_step": float(np.median(warm)), "image_l2_first": l2[0],
           "image_l2_last": l2[-1], "faces_per_level": faces,
           "path_samples_per_step": B.num_pixels(cams) * spp, "views": nviews, "res": res, "spp": spp,
           "bounces": bounces, "target_faces": int(target_sc.F.shape[0]),
           "tex_res": tex_res, "material_rows": int(M.shape[0]), "faces": faces[-1]}
    if return_params:
        out["V"], out["M"] = V.detach(), M.detach()
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--log-every", type=int, default=20)
    ap.add_argument("--tex-res", type=int, default=0)
    ap.add_argument("--spec-var", type=float, default=0.0)
    ap.add_argument("--subdivisions", type=int, default=0)
    ap.add_argument("--checkpoint", default=None, help="state file written every --checkpoint-every steps")
    ap.add_argument("--checkpoint-every", type=int, default=0)
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint when it exists")
    a = ap.parse_args()
    out = run(a.steps, log_every=a.log_every, tex_res=a.tex_res, spec_var_w=a.spec_var, subdivisions=a.subdivisions,
              checkpoint=a.checkpoint, checkpoint_every=a.checkpoint_every, resume=a.resume)
    print(json.dumps(out))

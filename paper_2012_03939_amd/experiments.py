"""The paper's two synthetic experiments, run through the HIP renderer.

gi_planes: Sec. 3.3 "Effects of Global Illumination" — three intersecting planes
(red, blue, white diffuse albedo), geometry known, albedos optimised from a
rendered target once with global illumination (3 bounces) and once with
one-bounce light transport.  With GI the white floor comes back white; with one
bounce it absorbs the red and blue light bled onto it.

divot: Sec. 3.2 "Shape From Shading" — a sphere with a divot that leaves the
silhouette unchanged, 5 cameras each with 4 light positions, reconstructed from
a plain sphere: only shading can push the divot in.

    python -m paper_2012_03939_amd.experiments gi
    python -m paper_2012_03939_amd.experiments divot
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

from . import binding as B
from . import scenes as S
from .autograd import render, uniform_laplacian, vertex_neighbours


# --------------------------------------------------------------------------
# three planes: floor y = 0 (white), wall x = 0 (red), wall z = 0 (blue)
# --------------------------------------------------------------------------

def _grid_quad(origin, du, dv, n):
    """n x n grid of a planar quad origin + s du + t dv, s, t in [0, 1]; 2 n^2 faces."""
    s = np.linspace(0.0, 1.0, n + 1)
    P = origin[None, None, :] + s[:, None, None] * du[None, None, :] + s[None, :, None] * dv[None, None, :]
    V = P.reshape(-1, 3)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a, b, c, d = idx[:-1, :-1], idx[1:, :-1], idx[:-1, 1:], idx[1:, 1:]
    F = np.concatenate([np.stack([a, b, d], -1).reshape(-1, 3), np.stack([a, d, c], -1).reshape(-1, 3)])
    return V, F


ALBEDO = {"floor": (0.8, 0.8, 0.8), "red": (0.8, 0.1, 0.1), "blue": (0.1, 0.1, 0.8)}


def three_planes(n: int = 8):
    """Floor (white), left wall (red), back wall (blue), each 2 x 2 and 2 n^2 faces;
    the walls stand on the floor and meet along the corner line."""
    parts = [("floor", np.array([0.0, 0.0, 0.0]), np.array([2.0, 0, 0]), np.array([0, 0, 2.0])),
             ("red", np.array([0.0, 0.0, 0.0]), np.array([0, 0, 2.0]), np.array([0, 2.0, 0])),
             ("blue", np.array([0.0, 0.0, 0.0]), np.array([0, 2.0, 0]), np.array([2.0, 0, 0]))]
    Vs, Fs, labels = [], [], []
    off = 0
    for name, o, du, dv in parts:
        V, F = _grid_quad(o, du, dv, n)
        Vs.append(V)
        Fs.append(F + off)
        labels += [name] * F.shape[0]
        off += V.shape[0]
    V = np.concatenate(Vs).astype(np.float32) - np.array([0.7, 0.7, 0.7], np.float32)
    F = np.concatenate(Fs).astype(np.int32)
    mat = np.zeros((F.shape[0], 7), np.float32)
    for i, lab in enumerate(labels):
        mat[i, :3] = ALBEDO[lab]
    mat[:, 6] = 0.5
    return V, F, mat, np.array(labels)


def gi_planes(steps: int = 150, res: int = 96, spp: int = 16, lr: float = 0.02, n: int = 8, seed: int = 0) -> dict:
    dev = torch.device("cuda")
    V, F, mat_true, labels = three_planes(n)
    light = np.array([[0.9, 1.2, 0.9, 6.0, 6.0, 6.0]], np.float32)
    eyes = [(2.6, 1.6, 2.6), (2.9, 1.0, 1.6), (1.6, 1.0, 2.9), (2.4, 2.4, 2.0)]
    cams = [S.Camera(e, (0.0, -0.2, 0.0), (0, 1, 0), 50.0, res, res) for e in eyes]
    target_scene = S.Scene(V, F, mat_true, light, None)
    gt = B.GPUScene.from_scene(target_scene)
    T = gt.render(cams, 4 * spp, 3, seed=999).clone()
    gt.close()
    out = {}
    for name, bounces in (("global_illumination", 3), ("one_bounce", 1)):
        start = mat_true.copy()
        start[:, :3] = 0.5
        g = B.GPUScene.from_scene(S.Scene(V, F, start, light, None))
        Vt = torch.from_numpy(V).to(dev)
        kd = torch.tensor(start[:, :3], device=dev, requires_grad=True)
        rest = torch.from_numpy(start[:, 3:]).to(dev)
        opt = torch.optim.Adam([kd], lr=lr)
        for it in range(steps):
            opt.zero_grad(set_to_none=True)
            img = render(Vt, torch.cat([kd, rest], 1), g, cams, spp, bounces, seed=seed + it, flags=B.ST_GRAD_INTERIOR)
            loss = ((img - T) ** 2).mean()
            loss.backward()
            opt.step()
            with torch.no_grad():
                kd.clamp_(0.0, 1.0)
        g.check_errors()
        est = kd.detach().cpu().numpy()
        res_ = {}
        for lab in ALBEDO:
            m = labels == lab
            res_[lab] = {"albedo": est[m].mean(0).round(4).tolist(),
                         "abs_error": float(np.abs(est[m].mean(0) - np.array(ALBEDO[lab])).mean())}
        res_["final_image_l2"] = float(loss.detach())
        out[name] = res_
        g.close()
    return out


# --------------------------------------------------------------------------
# sphere with a divot, 5 cameras x 4 lights
# --------------------------------------------------------------------------

def divot_sphere(k: int = 24, depth: float = 0.25, width: float = 0.35):
    """Unit geodesic sphere pushed in around +z: r = 1 - depth exp(-theta^2 / (2 width^2)),
    theta the angle from +z.  The dent stays inside the silhouette of views along +z."""
    V, F = S.geodesic_sphere(k)
    th = np.arccos(np.clip(V[:, 2], -1.0, 1.0))
    r = 1.0 - depth * np.exp(-th ** 2 / (2.0 * width ** 2))
    return (V * r[:, None]).astype(np.float32), F


def divot(steps: int = 300, res: int = 96, spp: int = 32, k: int = 24, depth: float = 0.25, lr: float = 5e-3,
          lap_w: float = 0.5, seed: int = 0) -> dict:
    dev = torch.device("cuda")
    Vt, F = divot_sphere(k, depth)
    V0, _ = divot_sphere(k, 0.0)
    mat = S.uniform_materials(F.shape[0], kd=0.7, ks=0.0, rough=0.5)
    cams = [S.Camera(e, (0, 0, 0), (0, 1, 0), 40.0, res, res)
            for e in [(0, 0, 3.2), (0.8, 0.3, 3.1), (-0.8, 0.3, 3.1), (0.3, 0.9, 3.0), (-0.3, -0.8, 3.1)]]
    lights = [np.array([[x, y, 3.0, 9.0, 9.0, 9.0]], np.float32) for x, y in [(2, 2), (-2, 2), (2, -2), (-2, -2)]]
    targets, scenes = [], []
    for li, lt in enumerate(lights):
        gt = B.GPUScene(Vt, F, mat, lt, None, scene_id=li)
        targets.append(gt.render(cams, 4 * spp, 1, seed=999).clone())
        gt.close()
        scenes.append(B.GPUScene(V0, F, mat, lt, None, scene_id=li))
    V = torch.tensor(V0, device=dev, requires_grad=True)
    M = torch.from_numpy(mat).to(dev)
    src, dst = vertex_neighbours(torch.from_numpy(F).to(dev), V.shape[0])
    opt = torch.optim.Adam([V], lr=lr)
    l2 = []
    for it in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = 0.0
        for li, g in enumerate(scenes):
            img = render(V, M, g, cams, spp, 1, seed=seed + 7 * it + li)
            loss = loss + ((img - targets[li]) ** 2).mean()
        l2.append(float(loss.detach()))
        (loss + lap_w * uniform_laplacian(V, src, dst)).backward()
        opt.step()
    for g in scenes:
        g.check_errors()
        g.close()
    Vf = V.detach().cpu().numpy()
    # the dent as recovered: radial depression of every vertex against the unit
    # sphere, projected on the target's dent profile (1 = the full divot)
    th = np.arccos(np.clip(V0[:, 2], -1.0, 1.0))
    prof = np.exp(-th ** 2 / (2.0 * 0.35 ** 2))
    got_r = 1.0 - np.linalg.norm(Vf, axis=1)
    frac = float((prof * got_r).sum() / (depth * (prof * prof).sum()))
    pole = int(np.argmax(V0[:, 2]))
    rim = np.abs(th - math.pi / 2) < 0.05
    return {"target_depth": depth, "recovered_pole_depth": float(got_r[pole]), "recovered_fraction": frac,
            "silhouette_radius_change": float(np.abs(np.linalg.norm(Vf[rim], axis=1) - 1.0).mean()),
            "image_l2_first": l2[0], "image_l2_last": l2[-1], "steps": steps, "cameras": len(cams),
            "lights": len(lights), "faces": int(F.shape[0])}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["gi", "divot"])
    ap.add_argument("--steps", type=int, default=0, help="0: the experiment's default")
    a = ap.parse_args()
    kw = {"steps": a.steps} if a.steps else {}
    print(json.dumps(gi_planes(**kw) if a.which == "gi" else divot(**kw)))

#!/usr/bin/env python3
"""Throughput of one optimisation step of the differentiable path tracer.

Step = LBVH rebuild for the current vertices (st_scene_update) + forward render
(st_render) + image-loss gradient (torch) + adjoint with interior, primary-edge
and secondary-edge terms (st_render_backward).  Workload: 40,000-face
noise-displaced torus under a 512x256 six-lobe HDR environment map, 16 views at
512x512, 16 samples per pixel, 3 bounces (67,108,864 path samples per step).
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line.  --gpus N with N > 1 is refused: the method runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit (the roofline's count): a slab test of one box is
# about 15 FP32 operations, so a visit of a 4-wide BVH node (four child boxes)
# is 60; a ray-triangle test is about 30.
FLOPS_PER_VISIT = 60
FLOPS_PER_TEST = 30
# The same work counted from the operations the kernels issue: per box 6 sub +
# 6 mul + 12 min/max = 24 (96 per node); per triangle test 2 cross (18) + 4 dot
# (20) + 1 rcp + 3 sub + 3 mul = 45.
ISSUED_FLOPS_PER_VISIT = 96
ISSUED_FLOPS_PER_TEST = 45
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# library launch names of the queue-streaming kernels -> their rocprofv3 names
HBM_KERNELS = {"k_shade": "k_shade<false>", "k_adjoint<3>": "k_adjoint<3, false, 1>",
               "k_adjoint_sec<3>": "k_adjoint<3, true, 0>",
               "k_extend": "k_extend", "k_trace_pair": "k_trace_pair", "k_shadow": "k_shadow"}
# Work-counter rows (st_read_work) that belong to one launch name alone: the
# extension and shadow rows count those rays wherever they are traced, which
# is also inside k_trace_pair once it runs.
OWN_WORK = ("k_trace_pair", "k_adjoint", "k_forward_mega")


CU_COUNT, SIMDS_PER_CU, CLOCK_HZ = 256, 4, 2.4e9
VALU_CYCLES_PER_WAVE_INST = 4      # a 64-lane VALU instruction occupies a 16-lane SIMD for 4 cycles


def measured_counters(kernel: str):
    """From the committed rocprofv3 counter summary of `kernel`: HBM bytes per
    launch (FETCH_SIZE and WRITE_SIZE scaled by their plain-copy factors), the
    share of SIMD cycles spent issuing VALU instructions, and the share of lanes
    active in them; None when the kernel sources changed after the counters were
    taken."""
    from paper_2012_03939_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "pmc_traversal_kernels_torus40k_16x512sq_16spp.json")
    try:
        with open(path) as fh:
            pm = json.load(fh)
    except OSError:
        return None
    if pm.get("source_hash") != kernel_source_hash():
        return None
    k = pm["kernels"].get(kernel) or pm["kernels"].get(kernel.split("<")[0])
    if k is None:
        return None
    issue = None
    if k.get("sq_insts_valu_per_dispatch") and k.get("mean_dispatch_ms_under_counters"):
        simd_cycles = k["mean_dispatch_ms_under_counters"] * 1e-3 * CLOCK_HZ * CU_COUNT * SIMDS_PER_CU
        issue = k["sq_insts_valu_per_dispatch"] * VALU_CYCLES_PER_WAVE_INST / simd_cycles
    return {"traffic": k["hbm_bytes_per_dispatch"], "valu_issue_utilisation": issue,
            "valu_lane_utilisation": k.get("valu_lane_utilisation"),
            "ms_under_counters": k.get("mean_dispatch_ms_under_counters")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spp", type=int, default=16)
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--views", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--mesh-colors-res", type=int, default=4, help="mesh-colour step at this resolution (0 skips)")
    ap.add_argument("--opt-steps", type=int, default=200, help="optimisation-loop steps (0 skips)")
    ap.add_argument("--cpu-baseline-res", type=int, default=1024)
    ap.add_argument("--env-sampler", choices=["cdf", "alias"], default="cdf",
                    help="environment texel draw: row/column CDFs or the alias table (same distribution)")
    ap.add_argument("--bsdf-sampler", choices=["halfvector", "vndf"], default="halfvector",
                    help="specular half-vectors from D cos(theta_h) or from the visible normals")
    ap.add_argument("--edge-sampler", choices=["cdf", "hierarchy"], default="cdf",
                    help="secondary edges drawn by the length CDF or the importance hierarchy")
    ap.add_argument("--profile-only", action="store_true", help="one untimed step (for rocprofv3 runs)")
    ap.add_argument("--batched-trace", action="store_true",
                    help="one per-view pass, then one batched pass of the 4-scene workload, 0.3 s apart (for "
                         "rocprofv3 kernel traces)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip st_autotune (wavefront chunk size and traversal grid) before the warm-up")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON-lines cache of st_autotune: a workload found there is not timed again (profiling "
                         "runs reuse the choice of an earlier run)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only a plain 512 MiB device copy: the reference that scales the HBM byte counters")
    return ap.parse_args()


def progress(msg: str) -> None:
    """One line on stderr when a phase of the run ends (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_info():
    """Host CPU model and logical core count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_baseline(wl, res, spp, bounces):
    """The FP64 oracle on a bounded sample: the same torus scene, one view at
    res x res, same spp and bounces, full forward + adjoint (all three terms)."""
    import numpy as np
    import oracle as O
    from paper_2012_03939_amd import scenes as S
    sc = wl.scenes[0]
    cam = S.look_at_origin(wl.cams[0].eye, res, res)
    o = O.OracleScene.from_scene(sc)
    nt = O.default_threads()
    t0 = time.perf_counter()
    img, _ = o.render([cam], spp, bounces, seed=0, nthreads=nt)
    d = np.random.default_rng(0).normal(size=img.shape).astype(np.float32)
    o.backward([cam], spp, bounces, d, seed=0, flags=7, nthreads=nt)
    dt = time.perf_counter() - t0
    n = res * res * spp
    info = cpu_info()
    return {"value": n / dt, "unit": "path samples/s (fwd+adjoint)", "cores": nt, "kind": "oracle",
            "sample": f"same torus scene and envmap, 1 view at {res}x{res}, {spp} spp, {bounces} bounces, "
                      f"forward + adjoint (interior, primary and secondary edges): {n} path samples in {dt:.2f} s",
            "threads": nt, "nproc": info["nproc"], "cpu_model": info["cpu_model"],
            "threads_note": "std::thread workers = min(nproc, 16): one GPU's share of the host is 16 threads"}


def mesh_colors_step(B, S, torch, wl, r, steps=3):
    """The same optimisation step (update + render + adjoint, all terms) with the
    materials as mesh colours of resolution r (Sec. 3.3): 40,000 (r+1)(r+2)/2 texels."""
    import numpy as np
    sc = wl.scenes[0]
    g = B.GPUScene.from_scene(sc)
    tex = torch.from_numpy(S.mesh_color_texels(sc.mat, r, np.random.default_rng(8))).cuda()
    g.set_mesh_colors(r, tex)
    B.autotune([g], wl.cams, wl.spp, wl.bounces)
    npix = B.num_pixels(wl.cams)
    img = torch.empty((npix, 3), dtype=torch.float32, device="cuda")
    dV = torch.empty((g.nv, 3), dtype=torch.float32, device="cuda")
    dM = torch.empty((g.ntex, 7), dtype=torch.float32, device="cuda")
    V0 = torch.from_numpy(sc.V).cuda()
    target = g.render(wl.cams, wl.spp, wl.bounces, seed=1).clone()

    def step(i):
        g.update(V=V0)
        g.render(wl.cams, wl.spp, wl.bounces, seed=i, out=img)
        g.backward(wl.cams, wl.spp, wl.bounces, (img - target) * (2.0 / img.numel()), seed=i,
                   flags=B.ST_ALL_GRADS, dV=dV, dmat=dM)

    step(0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        step(10 + i)
    e1.record()
    torch.cuda.synchronize()
    g.check_errors()
    ms = e0.elapsed_time(e1) / steps
    n = npix * wl.spp
    return {"tex_res": r, "texels": g.ntex, "ms_per_step": ms, "value": n / (ms / 1e3), "unit": "path samples/s",
            "steps": steps}


def batched_vs_per_view(B, S, torch, reps=3):
    """Forward render of 4 scenes (2,000 / 8,000 / 20,480 / 60,500 faces) with 24 views
    of uneven resolution, 16 spp, 2 bounces: one batched pass against one call per view."""
    wl = S.batched_uneven()
    gs = [B.GPUScene.from_scene(s) for s in wl.scenes]
    npix = B.num_pixels(wl.cams)
    out = torch.empty((npix, 3), dtype=torch.float32, device="cuda")
    outs = [torch.empty((c.width * c.height, 3), dtype=torch.float32, device="cuda") for c in wl.cams]

    def batched():
        B.render_batch(gs, wl.cams, wl.cam_scene, wl.spp, wl.bounces, seed=0, out=out)

    def per_view():
        for i, c in enumerate(wl.cams):
            gs[wl.cam_scene[i]].render([c], wl.spp, wl.bounces, seed=0, out=outs[i])

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {}
    graphs = {}
    for name, fn in (("batched", batched), ("per_view", per_view)):
        fn()
        torch.cuda.synchronize()
        res[name + "_ms"] = timed(fn)
        # the same launches captured once and replayed as a graph
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        graphs[name] = g
        g.replay()
        torch.cuda.synchronize()
        res[name + "_graph_ms"] = timed(g.replay)
    res["speedup"] = res["per_view_ms"] / res["batched_ms"]
    res["speedup_graphs"] = res["per_view_graph_ms"] / res["batched_graph_ms"]
    res["speedup_batched_graph_vs_per_view"] = res["per_view_ms"] / res["batched_graph_ms"]
    res["path_samples"] = npix * wl.spp
    res["workload"] = wl.name
    return res


def batched_trace(B, S, torch):
    """The two modes of the batched comparison once each, separated by idle
    time so that a kernel trace splits into the two phases."""
    wl = S.batched_uneven()
    gs = [B.GPUScene.from_scene(s) for s in wl.scenes]
    out = torch.empty((B.num_pixels(wl.cams), 3), dtype=torch.float32, device="cuda")
    outs = [torch.empty((c.width * c.height, 3), dtype=torch.float32, device="cuda") for c in wl.cams]

    def per_view():
        for i, c in enumerate(wl.cams):
            gs[wl.cam_scene[i]].render([c], wl.spp, wl.bounces, seed=0, out=outs[i])

    def batched():
        B.render_batch(gs, wl.cams, wl.cam_scene, wl.spp, wl.bounces, seed=0, out=out)

    per_view()
    batched()                       # workspaces sized outside the traced phases
    torch.cuda.synchronize()
    for fn in (per_view, batched):
        time.sleep(0.3)
        fn()
        torch.cuda.synchronize()
    time.sleep(0.3)
    print(json.dumps({"batched_trace": wl.name, "phases": ["per_view", "batched"]}))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this path tracer runs on one GPU; multi-GPU runs are not supported "
                                   "(path samples would split by view, with one all-reduce of the "
                                   "gradients per step)"}))
        sys.exit(2)
    if args.copy_reference:
        from paper_2012_03939_amd.profiling import copy_reference
        copy_reference()
        return
    import numpy as np
    import torch
    from paper_2012_03939_amd import binding as B, scenes as S

    if args.batched_trace:
        batched_trace(B, S, torch)
        return
    wl = S.torus_envmap(res=args.res, nviews=args.views, spp=args.spp, bounces=3)
    sc = wl.scenes[0]
    g = B.GPUScene.from_scene(sc)
    g.set_env_sampler(B.ST_ENV_SAMPLER_ALIAS if args.env_sampler == "alias" else B.ST_ENV_SAMPLER_CDF)
    g.set_bsdf_sampler(B.ST_BSDF_SAMPLER_VNDF if args.bsdf_sampler == "vndf" else B.ST_BSDF_SAMPLER_HALFVECTOR)
    cams, spp, bounces = wl.cams, wl.spp, wl.bounces
    grads = B.ST_ALL_GRADS | (B.ST_EDGE_SECONDARY_HIERARCHY if args.edge_sampler == "hierarchy" else 0)
    npix = B.num_pixels(cams)
    n_paths = npix * spp
    dev = torch.device("cuda")
    V0 = torch.from_numpy(sc.V).to(dev)
    # target images from perturbed vertices (synthetic stand-in for captured views)
    g.update(V=torch.from_numpy(S.perturbed_vertices(sc.V, 0.01, 77)).to(dev))
    # (a profiling run renders the target with the single-kernel forward, so that its
    # trace holds the wavefront kernels of exactly one step)
    target = g.render(cams, spp, bounces, seed=1, flags=B.ST_FORWARD_MEGAKERNEL if args.profile_only else 0).clone()
    Vs = [V0 + 1e-4 * torch.randn_like(V0) for _ in range(2)]
    dV = torch.empty_like(V0)
    dM = torch.empty((g.nf, 7), dtype=torch.float32, device=dev)
    img = torch.empty((npix, 3), dtype=torch.float32, device=dev)
    scale = 2.0 / img.numel()

    def step(i, spp=spp, extra=0):
        g.update(V=Vs[i & 1])
        g.render(cams, spp, bounces, seed=i, out=img)
        d = (img - target) * scale
        g.backward(cams, spp, bounces, d, seed=i, flags=grads | extra, dV=dV, dmat=dM)

    def timed_steps(n, **kw):
        step(50, **kw)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(n):
            step(60 + i, **kw)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    # the library's autotuner picks the wavefront chunk size and the traversal
    # grid for this workload (timed renders, before the warm-up); later renders
    # and backward passes of the scene use them
    tuned = (None, None) if args.no_autotune else B.autotune([g], cams, spp, bounces, cache_path=args.autotune_cache)
    if args.profile_only:
        step(0)
        torch.cuda.synchronize()
        g.check_errors()
        print(json.dumps({"profile_only": True, "n_paths": n_paths}))
        return

    progress(f"autotuned queue capacity {tuned[0]}, trace grid {tuned[1]}")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    g.check_errors()
    progress(f"{args.warmup} warm-up steps done")
    B.profile_read()
    B.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        step(100 + i)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.profile_enable(False)
    prof = B.profile_read()
    g.check_errors()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    progress(f"{args.steps} timed steps: {ms_per_step:.2f} ms per step")
    value = n_paths * args.steps / (ms / 1e3)

    # the dominant traversal kernel and its algorithmic work, counted on device in
    # one extra (untimed) step; a kernel qualifies when a work-counter row is its own
    own = OWN_WORK if "k_trace_pair" in prof else OWN_WORK + ("k_extend", "k_shadow")
    dom_name, (dom_ms, dom_n) = max(((k, v) for k, v in prof.items() if k.split("<")[0] in own),
                                    key=lambda kv: kv[1][0])
    g.read_work()
    g.update(V=Vs[0])
    g.render(cams, spp, bounces, seed=100, out=img, flags=B.ST_COUNT_WORK)
    fwork = g.read_work()
    g.backward(cams, spp, bounces, (img - target) * scale, seed=100, flags=grads | B.ST_COUNT_WORK,
               dV=dV, dmat=dM)
    work = {k: tuple(a + b for a, b in zip(v, fwork[k])) for k, v in g.read_work().items()}
    # The same kernel in a forward render alone: in the step, the backward's
    # launches share the GPU with the adjoint on the second stream, which
    # lengthens their durations; a forward runs on one stream only.
    B.profile_read()
    B.profile_enable(True)
    for i in range(3):
        g.render(cams, spp, bounces, seed=100, out=img)
    B.profile_enable(False)
    fprof = B.profile_read()
    wkey = dom_name.split("<")[0]
    visits, tests, rays = work.get(wkey, (0, 0, 0))
    launches_per_step = dom_n / args.steps
    flops_per_launch = (visits * FLOPS_PER_VISIT + tests * FLOPS_PER_TEST) / max(launches_per_step, 1)
    issued_per_launch = (visits * ISSUED_FLOPS_PER_VISIT + tests * ISSUED_FLOPS_PER_TEST) / max(launches_per_step, 1)
    avg_ms = dom_ms / dom_n
    achieved = flops_per_launch / (avg_ms / 1e3) / 1e12
    achieved_issued = issued_per_launch / (avg_ms / 1e3) / 1e12
    alone = None
    if dom_name in fprof and fwork.get(wkey, (0, 0, 0))[2]:
        fms, fn = fprof[dom_name]
        fv, ft, fr = fwork[wkey]
        fper = fn / 3
        fflops = (fv * FLOPS_PER_VISIT + ft * FLOPS_PER_TEST) / fper
        alone = {"avg_launch_ms": fms / fn, "launches_per_render": fper, "node_visits_per_launch": fv / fper,
                 "tri_tests_per_launch": ft / fper, "rays_per_launch": fr / fper,
                 "achieved": fflops / (fms / fn / 1e3) / 1e12,
                 "frac": fflops / (fms / fn / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                 "note": "forward renders alone (one stream), 3 renders after the timed region"}
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps} for k, v in prof.items()}
    # every forward-style traversal launch of the step together (camera, extension
    # and shadow rays of the main paths and of the primary-edge side paths)
    trav_ms = sum(kernels[k]["ms_per_step"] for k in ("k_extend", "k_trace_pair", "k_shadow") if k in kernels)
    trav_flops = sum(work[k][0] * FLOPS_PER_VISIT + work[k][1] * FLOPS_PER_TEST for k in ("k_extend", "k_shadow"))
    traversal_all = {"kernels": ["k_extend", "k_trace_pair", "k_shadow"], "ms_per_step": trav_ms,
                     "achieved": trav_flops / (trav_ms / 1e3) / 1e12 if trav_ms else None,
                     "frac": trav_flops / (trav_ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS if trav_ms else None}
    # rays, node visits and triangle tests of one step: per ray kind (extension
    # and shadow rays wherever traced), and per launch name where the row is its
    # own (time and rate only there)
    traversal = {}
    for k, (kv, kt, kr) in work.items():
        if not kr:
            continue
        e = {"rays_per_step": kr, "node_visits_per_ray": kv / kr, "tri_tests_per_ray": kt / kr}
        if k in own:
            # (the adjoint's row covers its job pass, launched as k_adjoint_sec)
            kms = sum(v["ms_per_step"] for n, v in kernels.items() if n.split("<")[0].startswith(k))
            e.update({"ms_per_step": kms, "rays_per_s": kr / (kms / 1e3) if kms else None})
        traversal[{"k_extend": "extension_rays", "k_shadow": "shadow_rays"}.get(k, k)] = e
    mc = measured_counters(dom_name)
    # queue-streaming kernels: HBM bytes per launch (counters of these sources)
    # over their live mean launch time, against a measured streaming copy; and
    # the same bytes over the mean dispatch time in the counter run, where
    # rocprofv3 serialises the dispatches (no kernel shares the GPU with another,
    # as the adjoint and the side paths do in the step)
    copy_gbs = B.copy_bandwidth()
    hbm = {"copy_gbs": copy_gbs, "peak_gbs": PEAK_HBM_GBS, "kernels": {}}
    for lk, pk in HBM_KERNELS.items():
        if lk not in prof:
            continue
        kms, kn = prof[lk]
        c = measured_counters(pk)
        gbs = c["traffic"] / (kms / kn * 1e-3) / 1e9 if c else None
        hbm["kernels"][lk] = {"avg_launch_ms": kms / kn, "hbm_bytes_per_launch": c["traffic"] if c else None,
                              "gbs": gbs, "frac_of_copy": gbs / copy_gbs if gbs else None,
                              "frac_of_peak": gbs / PEAK_HBM_GBS if gbs else None}
        rms = c.get("ms_under_counters") if c else None
        if rms:
            rg = c["traffic"] / (rms * 1e-3) / 1e9
            hbm["kernels"][lk].update({"rocprof_ms": rms, "rocprof_gbs": rg, "rocprof_frac_of_copy": rg / copy_gbs,
                                       "rocprof_frac_of_peak": rg / PEAK_HBM_GBS})
    # the same step at the workload's own 32 spp, and with every main-path ray traced again in the adjoint
    ms32 = timed_steps(3, spp=2 * spp)
    progress(f"{2 * spp} spp step: {ms32:.2f} ms")
    ms_retrace = timed_steps(3, extra=B.ST_BACKWARD_RETRACE)
    progress(f"re-tracing step: {ms_retrace:.2f} ms")
    out = {
        "metric": "fwd+adjoint path samples/sec at 16 views 512^2 16spp; sec per optimisation step",
        "value": value,
        "unit": "path samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "faces": int(sc.F.shape[0]), "views": len(cams), "res": args.res,
                   "spp": spp, "bounces": bounces, "path_samples_per_step": n_paths,
                   "edge_samples_per_step": B.num_edge_samples(cams, spp, 1.0, int(sc.lights.shape[0])),
                   "envmap": "512x256", "env_sampler": args.env_sampler, "bsdf_sampler": args.bsdf_sampler,
                   "edge_sampler": args.edge_sampler, "autotuned_queue_capacity": tuned[0],
                   "autotuned_trace_grid": tuned[1]},
        "roofline": {"bound": "alu", "kernel": dom_name, "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": (mc or {}).get("traffic"),
                     "flops_per_node_visit": FLOPS_PER_VISIT, "flops_per_tri_test": FLOPS_PER_TEST,
                     "achieved_issued_count": achieved_issued,
                     "frac_issued_count": achieved_issued / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-scaled)",
                     "avg_launch_ms": avg_ms,
                     "valu_issue_utilisation": (mc or {}).get("valu_issue_utilisation"),
                     "valu_lane_utilisation": (mc or {}).get("valu_lane_utilisation"), "node_visits_per_launch": visits / max(launches_per_step, 1),
                     "tri_tests_per_launch": tests / max(launches_per_step, 1),
                     "rays_per_launch": rays / max(launches_per_step, 1),
                     "rays_per_s": rays / max(launches_per_step, 1) / (avg_ms / 1e3),
                     "forward_alone": alone, "traversal_all": traversal_all},
        "kernels": kernels,
        "traversal": traversal,
        "hbm": hbm,
        "spp32": {"spp": 2 * spp, "ms_per_step": ms32, "value": 2 * n_paths / (ms32 / 1e3),
                  "unit": "path samples/s", "steps": 3},
        "retrace": {"ms_per_step": ms_retrace, "value": n_paths / (ms_retrace / 1e3), "unit": "path samples/s",
                    "steps": 3, "note": "backward traces every main-path ray again (no hit records)"},
    }
    if args.mesh_colors_res > 0:
        out["mesh_colors"] = mesh_colors_step(B, S, torch, wl, args.mesh_colors_res)
        progress(f"mesh-colour step: {out['mesh_colors']['ms_per_step']:.2f} ms")
    if not args.no_batched:
        out["batched"] = batched_vs_per_view(B, S, torch)
        progress(f"batched speed-up {out['batched']['speedup']:.2f}")
    if args.opt_steps > 0:
        # second half of the metric: seconds per optimisation step (Adam through torch.autograd)
        from paper_2012_03939_amd.optimise import run as optimise
        out["optimisation"] = optimise(steps=args.opt_steps)
        progress("optimisation loop done")
    if not args.no_cpu_baseline:
        progress("oracle baseline on the host cores")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_baseline_res, spp, bounces)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

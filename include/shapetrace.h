/*
 * shapetrace: MI355X (gfx950) differentiable path tracer, C ABI.
 *
 * The operation is the rendering function R(x, m, c_i) of Shape from Tracing
 * (Sec. 3.2, "Vertex optimization": a physically based path tracer that also
 * returns gradients of the pixels with respect to the mesh vertices x) with the
 * per-facet Torrance-Sparrow materials m of Sec. 3.3 ("Representation": diffuse
 * albedo, specular colour, roughness; mesh colours at resolution 0, i.e. one
 * texel per triangle), global illumination (Sec. 3.3, "Effects of Global
 * Illumination"), and the two lighting inputs of Sec. 3.1: point lights or an
 * HDR environment map.  The loss of Sec. 3.2 (masked mean squared error) is left
 * to the caller: st_render_backward receives dLoss/dImage and returns dLoss/dV
 * and dLoss/dMaterial, including the silhouette-edge visibility terms.
 *
 * Conventions shared by every entry point:
 *  - Array arguments (V, F, materials, lights, envmap, images, gradients) are
 *    DEVICE pointers owned by the caller, row-major and contiguous.  Camera
 *    records, cam_scene and the options struct are HOST memory.
 *  - All work is enqueued on the given HIP stream and returns before it
 *    finishes; outputs are complete when the stream is.  st_scene_create also
 *    synchronises the stream (it validates the face indices on the host).
 *  - st_scene_create / st_scene_update copy their inputs; the caller may free
 *    them afterwards.  The library owns the BVH, CDFs, queues and workspace until
 *    st_scene_destroy.  Render calls may grow the library workspace (the first
 *    call with a larger shape allocates); identical later calls allocate nothing.
 *  - Graph capture: st_render, st_render_batch and st_render_backward may be
 *    captured (hipStreamBeginCapture / torch.cuda.graph) once an uncaptured call
 *    with the same shapes has sized the workspace; a call that would allocate
 *    under capture fails with ST_ERR_INVALID_ARG.  Memory a captured graph uses
 *    stays valid until st_scene_destroy: a workspace that later grows is retired,
 *    not freed, as are the material arrays st_scene_set_mesh_colors replaces.
 *    Destroying a scene invalidates every graph that uses it.  Calls on one scene
 *    (eager or replayed) must be ordered on one stream: they share its workspace.
 *  - Outputs are overwritten, never accumulated.
 *  - Return value 0 on success, a negative ST_ERR_* code otherwise; the message
 *    of the last failure on the calling thread is returned by st_last_error().
 *  - Limits: 1 <= spp < 65536, 1 <= bounces <= 8, 1 <= ncam < 65536, at most 16
 *    point lights, fewer than 2^31 path samples per call (the counter layout of
 *    the random streams needs these).
 */
#ifndef SHAPETRACE_H
#define SHAPETRACE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ST_OK 0
#define ST_ERR_INVALID_ARG (-1)
#define ST_ERR_HIP (-2)
#define ST_ERR_OOM (-3)
#define ST_ERR_QUEUE_OVERFLOW (-4)
#define ST_ERR_DEVICE_FAULT (-5)

/* gradient terms of st_render_backward, and forward-pass switches */
#define ST_GRAD_INTERIOR 1u        /* derivative of the estimator at fixed sampled directions */
#define ST_EDGE_PRIMARY 2u         /* screen-space silhouette / crease edges (camera visibility) */
#define ST_EDGE_SECONDARY 4u       /* direction-space silhouette edges at every path vertex */
#define ST_EDGE_SHADOW 8u          /* point-light shadow boundaries seen by the camera (image-space term) */
#define ST_FORWARD_MEGAKERNEL 16u  /* forward as one kernel per path sample instead of the wavefront */
#define ST_COUNT_WORK 32u          /* count BVH node visits, triangle tests and rays (st_read_work) */
#define ST_EDGE_SECONDARY_INTERIOR 64u  /* secondary edges: also creases and material boundaries seen from
                                           a path vertex, not only silhouettes (2 side paths per sample) */
#define ST_BACKWARD_RETRACE 128u   /* backward: trace every main-path ray again even when hit records of
                                      the matching forward pass are held (see st_render_backward) */
#define ST_EDGE_SECONDARY_HIERARCHY 256u  /* secondary edges drawn by an importance hierarchy instead of the
                                             length CDF (see st_scene_edge_tree) */

typedef struct st_scene st_scene;

/* Pinhole camera (the calibrated cameras c_i of Sec. 3.2): vertical field of
 * view in degrees, image row 0 at the top; width x height pixels. */
typedef struct {
    float eye[3], target[3], up[3];
    float fov_y_deg;
    int32_t width, height;
} st_camera;

typedef struct {
    uint32_t flags;                  /* ST_GRAD_* | ST_EDGE_* | ST_FORWARD_MEGAKERNEL */
    float edge_spp_ratio;            /* primary edge samples per (pixel x spp) of each view; with
                                        ST_EDGE_SHADOW as many shadow-edge samples per (view, light) */
    int64_t queue_capacity;          /* wavefront chunk size in path samples (0: the scene's autotuned value,
                                        else 2^24) */
    uint32_t* debug_decision_hash;   /* device, optional: one FNV-1a hash of the discrete decisions per
                                        path sample, index ((pixel offset of view + y*W + x) * spp + j) */
    uint32_t* debug_edge_hash;       /* device, optional (backward): one hash per primary edge sample,
                                        then (ST_EDGE_SHADOW) one per shadow-edge sample, sample i of
                                        (view v, light l) at N_e + nl eoff_v + l N_e(v) + i, N_e the
                                        primary total, eoff_v the primary offset of view v */
    float* debug_sample_radiance;    /* device, optional (forward): per path sample rgb, same index */
    const uint8_t* path_mask;        /* device, optional (backward): 0 skips a path sample */
    const uint8_t* edge_mask;        /* device, optional (backward): 0 skips an edge sample (same index) */
    int64_t max_workspace_bytes;     /* 0: no limit.  Otherwise a call whose library workspace (radiance
                                        buffer, wavefront queues, traversal spill stack; backward: edge
                                        tables, secondary-edge jobs, primary-edge side paths) would exceed
                                        it fails with ST_ERR_OOM before launching any kernel; a forward
                                        keeps no hit records when only they would exceed it */
} st_render_opts;

/* Default options: interior, primary and secondary edge terms and the
 * point-light shadow boundaries, one edge sample per pixel sample, default
 * queue capacity, no debug outputs. */
st_render_opts st_render_opts_default(void);

/* Create a scene (Sec. 3.2 triangle mesh x with faces; Sec. 3.3 per-face
 * material; Sec. 3.1 lights).
 *   V: float [nv,3] vertex positions.  F: int32 [nf,3] vertex indices
 *   (validated: 0 <= index < nv, else ST_ERR_INVALID_ARG).
 *   face_materials: float [nf,7] = kd rgb, ks rgb, roughness (roughness floor 1e-3).
 *   lights: float [nl,6] = position xyz, radiant intensity rgb (W/sr); NULL when nl == 0.
 *   envmap: float [he,we,3] equirectangular, +y up, row 0 looking along +y; NULL for none.
 *   scene_id: second word of the Philox key of this scene's random streams.
 *   out: receives the handle.  Allocates, copies, builds the BVH and CDFs, and
 *   synchronises stream s. */
int st_scene_create(const float* V, int32_t nv, const int32_t* F, int32_t nf, const float* face_materials,
                    const float* lights, int32_t nl, const float* envmap, int32_t he, int32_t we,
                    uint32_t scene_id, hipStream_t s, st_scene** out);

/* One gradient-descent step's new parameters (Sec. 3.2 "Vertex optimization":
 * the vertex positions x move every step; Sec. 3.3 "Material Optimization":
 * the material texels likewise), with the topology of the scene kept.  Replace
 * vertex positions (float [nv,3]) and/or materials (float [ntex,7], the
 * current material rows: one per face, or the mesh-colour texels); either may be
 * NULL.  Rebuilds the LBVH and edge CDF on the stream; allocates nothing. */
int st_scene_update(st_scene* scene, const float* V, const float* face_materials, hipStream_t s);

/* Switch the scene's materials to mesh colours (Sec. 3.3 "Representation") of
 * resolution r in [0, 64]: texels is a device float [ntex, 7] with
 * ntex = nf (r+1)(r+2)/2, same 7 parameters as per-face materials.  The point
 * with barycentric coordinates (alpha, beta) of face t (alpha weighs the face's
 * second vertex, beta its third) is shaded with texel
 * t (r+1)(r+2)/2 + i (2r - i + 3)/2 + j, (i, j) = floor(r (alpha, beta)) clamped
 * to 0 <= i <= r, 0 <= j <= r - i.  r = 0 is one texel per face (the
 * representation st_scene_create sets up).  Afterwards st_scene_update takes
 * [ntex,7] materials and st_render_backward writes d/d(texels) [ntex,7] (texel
 * lookup is piecewise constant, so texels receive the material gradient of the
 * points they shade; texel boundaries inside a face carry no edge term).
 * Allocates (not capturable) and synchronises s; ST_ERR_INVALID_ARG when
 * 7 ntex >= 2^31. */
int st_scene_set_mesh_colors(st_scene* scene, int32_t r, const float* texels, hipStream_t s);
/* 1 -> 4 subdivision of the scene's current mesh (Sec. 3.2 "Subdivision": every
 * edge split at its midpoint), for a coarse-to-fine schedule; the caller creates
 * a new scene from the result (topology changes need st_scene_create).
 *   out_V: device float [nv + ne, 3] = the vertices, then the midpoint
 *   (va + vb) / 2 of every edge in st_scene_edges order;
 *   out_F: device int32 [4 nf, 3]: face f becomes (v0, m01, m20), (v1, m12, m01),
 *   (v2, m20, m12), (m01, m12, m20) at rows 4f .. 4f+3, with mij the midpoint of
 *   edge (vi, vj) (orientation kept; a degenerate edge's midpoint is its vertex).
 * ne is entry 2 of st_scene_info (nv, nf, ne, nl, he, we).  Allocates nothing. */
int st_scene_subdivide(const st_scene* scene, float* out_V, int32_t* out_F, hipStream_t s);
/* Current mesh-colour resolution and number of material rows (either may be NULL). */
int st_scene_mesh_colors_info(const st_scene* scene, int32_t* r, int64_t* ntex);

/* How environment light samples pick their texel (Sec. 3.2: the map is sampled
 * in proportion to its texels' power).  Both give the same distribution, the
 * texel probability P_t = mean(rgb_t) * solid angle_t / sum over texels, and the
 * same pdf; only the draw differs:
 *   ST_ENV_SAMPLER_CDF (default): marginal row CDF on u0, then the row's
 *   conditional CDF on u1 (guided binary searches in fp64);
 *   ST_ENV_SAMPLER_ALIAS: Walker's alias method with Vose's construction, built
 *   on the host in fp64 from the P_t above: bin k = floor(u0 n) (n = he we),
 *   texel k if u1 < prob_k, else alias_k.  One 16-byte load per sample.
 * The position inside the texel uses u2, u3 in both.  The first ALIAS request
 * copies the map to the host, builds the table and allocates 16 n bytes (not
 * capturable); synchronises s.  ST_ERR_INVALID_ARG for an unknown method or a
 * scene without an environment map. */
#define ST_ENV_SAMPLER_CDF 0
#define ST_ENV_SAMPLER_ALIAS 1
int st_scene_set_env_sampler(st_scene* scene, int32_t method, hipStream_t s);
/* The alias table (host arrays of he*we entries: double prob, int32 alias), for
 * inspection; ST_ERR_INVALID_ARG before the table is built. */
int st_scene_env_alias_table(const st_scene* scene, double* prob, int32_t* alias);

/* How the specular lobe of the BRDF mixture (Sec. 3.3 Torrance-Sparrow; lobe
 * chosen with probability 1/2) draws its half-vector h:
 *   ST_BSDF_SAMPLER_HALFVECTOR (default): h ~ D(h) cos(theta_h);
 *   ST_BSDF_SAMPLER_VNDF: h ~ the normals visible from wo, G1(wo) max(0, wo.h)
 *   D(h) / cos(theta_o) (Heitz and d'Eon 2014, Beckmann: stretched slopes, the
 *   in-plane slope by bracketed Newton on its CDF, the other by erfinv).
 * Both are unbiased with their own pdf (used for the path weight and the MIS
 * weights); VNDF never samples back-facing microfacets.  Changes the scene's
 * state (hit records of earlier renders are dropped); synchronises s. */
#define ST_BSDF_SAMPLER_HALFVECTOR 0
#define ST_BSDF_SAMPLER_VNDF 1
int st_scene_set_bsdf_sampler(st_scene* scene, int32_t method, hipStream_t s);

/* Forward render (Sec. 3.2, R(x, c_i)).  cams: host array of ncam cameras.
 * out: device float [sum_i width_i*height_i, 3], views concatenated, each row-major;
 * every pixel is the mean of spp path samples with a one-pixel box filter.
 * bounces: number of surface vertices with next-event estimation (1 = direct light).
 * seed: first word of the Philox key.  opts may be NULL (defaults). */
int st_render(st_scene* scene, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed,
              const st_render_opts* opts, float* out, hipStream_t s);

/* st_render for callers that cannot allocate device memory: code under graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments and the same image (bit for bit) as st_render on one scene; every
 * workspace (camera table, per-sample radiance, wavefront queues, traversal
 * spill stack) lives in one static 64 MiB device array of the library, which
 * each GPU the library runs on holds until the process ends.  No hipMalloc,
 * hipFree or allocating call; the camera table goes to the device through
 * kernel arguments.  Limits: at most 64 cameras and 2^20 path samples
 * (sum of width x height x spp) per call, else ST_ERR_INVALID_ARG before any
 * launch.  Keeps no hit records (a later backward traces its main paths).
 * Every call on a GPU shares that array: calls that overlap on one GPU (other
 * streams, other threads, replays of graphs holding this call) race and must be
 * ordered by the caller.  Traversal uses 512 blocks per launch. */
int st_render_noalloc(st_scene* scene, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces,
                      uint32_t seed, const st_render_opts* opts, float* out, hipStream_t s);

/* Adjoint of st_render (Sec. 3.2 gradients w.r.t. geometry; Sec. 3.3 materials).
 * Must be called with the same (cams, spp, bounces, seed) as the forward pass
 * whose image gradient it receives; it replays every path from its random
 * counters.  Hit records: a single-scene wavefront st_render keeps, per path
 * sample, the face hit at every bounce and the occlusion of every shadow ray
 * (4 (2 bounces + 1) bytes per path sample, scene-owned, at most 16 GiB; scenes
 * with more than 30 point lights keep none).  When the backward's (cams, spp,
 * bounces, seed) equal those of the last such render executed on the stream
 * (eager or replayed from a graph) and the scene has not changed since
 * (st_scene_update, st_scene_set_mesh_colors, st_scene_set_env_sampler,
 * st_scene_set_bsdf_sampler), the replay takes hits and occlusions from the
 * records (the hit distance from the recorded face's plane) instead of tracing
 * the main path again; the render writes the key of its pass into device memory
 * beside the records and the adjoint compares it there, so a graph replay in
 * between is seen.  ST_BACKWARD_RETRACE in opts->flags disables the records.
 * The result is the same estimator either way.
 *   d_image: device float, same layout as st_render's out.
 *   out_dV: device float [nv,3]; out_dmat: device float [ntex,7] (ntex = nf unless the scene uses
 *   mesh colours, st_scene_set_mesh_colors); both overwritten. */
int st_render_backward(st_scene* scene, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces,
                       uint32_t seed, const st_render_opts* opts, const float* d_image, float* out_dV,
                       float* out_dmat, hipStream_t s);

/* Several independent scenes in one pass (Sec. 4.1 "Reconstructing Simulated
 * Objects" renders 32 calibrated views of each object per step; this renders
 * the views of several objects together): camera i renders scene cam_scene[i]
 * (host int32 [ncam]).  Each camera's random streams are numbered by its index
 * among the cameras of its own scene, so the result equals per-scene st_render
 * calls bit for bit.  Output layout as st_render over the concatenated views. */
int st_render_batch(st_scene* const* scenes, int32_t nscenes, const st_camera* cams, const int32_t* cam_scene,
                    int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed, const st_render_opts* opts,
                    float* out, hipStream_t s);

/* Autotuner: times st_render of this exact workload (same arguments as
 * st_render_batch; cam_scene may be NULL for one scene) over wavefront chunk
 * sizes {2^20..2^27} x traversal grids {1024, 2048, 4096} blocks and keeps the
 * fastest on every scene in the list (a smaller chunk or grid must be 3 %
 * faster than a larger one to be chosen); later renders and backward passes of
 * those scenes use it unless opts->queue_capacity is set.  cache_path (may be
 * NULL): JSON-lines file keyed by device and workload signature; a matching
 * line is used without timing, a new result is appended.  Synchronises s and
 * allocates a temporary image.  The chosen values are returned through the two
 * optional host pointers. */
int st_autotune(st_scene* const* scenes, int32_t nscenes, const st_camera* cams, const int32_t* cam_scene,
                int32_t ncam, int32_t spp, int32_t bounces, const char* cache_path, int64_t* out_queue_capacity,
                int32_t* out_trace_grid, hipStream_t s);

/* Wait for stream s and report what kernels of earlier calls on this scene
 * recorded in its device error word, then clear it: ST_ERR_QUEUE_OVERFLOW when a
 * wavefront queue reservation went past its capacity (the entries are dropped,
 * not written; the queues are sized so that this does not happen),
 * ST_ERR_DEVICE_FAULT for a traversal stack overflow or iteration cap, or a
 * non-finite value in a rendered image or in dV / dmat (checked after every
 * term of a backward), or several of these.  The message lists the bits. */
int st_check_errors(st_scene* scene, hipStream_t s);

/* Introspection for tests (device outputs, caller-allocated):
 *  st_scene_info: host int64 [6] = nv, nf, number of edges, nl, he, we.
 *  st_scene_edges: int32 [ne,4] = (va < vb, f1, f2 or -1), canonical order.
 *  st_scene_lbvh: keys uint64 [nf] (morton << 32 | face, ascending; 10 bits per
 *    axis over cubic cells, 1024 along the longest extent of the face-centre
 *    box), child int32 [nf-1,2] (bit 31 marks a leaf index), parent int32
 *    [2nf-1] (internal nodes, then leaves; -1 at the root), aabb float [2nf-1,6]
 *    (min xyz, max xyz).  The tree is the Karras radix tree over the keys after
 *    one bottom-up pass of treelet restructuring (7-entry treelets re-arranged
 *    to their least SAH cost, triangle cost = box area, internal node cost =
 *    1.2 x box area + children); leaves and the root box are those of the radix
 *    tree.  Deterministic: a function of the mesh alone.
 *  st_trace_rays: closest hit of n rays o,d (float [n,3]) with t > tmin, through
 *    the BVH or by brute force; out_face int32 [n] (-1 miss), out_t float [n]. */
int st_scene_info(const st_scene* scene, int64_t* out6);
/* Traversal work counted by calls made with ST_COUNT_WORK since the last read:
 * host uint64 [5][3] = for the extension rays and the shadow rays of the
 * wavefront forward (wherever launched), the adjoint replay kernel, the
 * single-kernel forward, and the paired launch that traces the extension rays
 * of one bounce with the shadow rays of the bounce before (its rays are also
 * in the first two rows): BVH node visits, triangle tests, rays traced.
 * Waits for s and resets the counters. */
int st_read_work(st_scene* scene, uint64_t* out3, hipStream_t s);
int st_scene_edges(st_scene* scene, int32_t* out_edges, hipStream_t s);
int st_scene_lbvh(st_scene* scene, uint64_t* keys, int32_t* child, int32_t* parent, float* aabb, hipStream_t s);
/* Secondary-edge importance hierarchy (ST_EDGE_SECONDARY_HIERARCHY; Li et al.
 * 2018 sample silhouette edges through a hierarchy, the paper relies on their
 * renderer): the radix tree (layout of st_scene_lbvh) over the edges' boxes,
 * key = morton << 32 | edge, every node with the float sum of the lengths below
 * it (a leaf: its edge's length, computed in double from the float endpoints).
 * Every node also holds the box of the unit normals of the faces beside its
 * edges (a boundary edge, always a silhouette, takes the cube [-1, 1]^3).  At a
 * shading point p with normal n the edge is drawn by descending the tree, each
 * child with probability proportional to its weight: zero when its box lies
 * wholly behind the tangent plane of p, or, unless ST_EDGE_SECONDARY_INTERIOR
 * is set, when the normal box proves that p sees every face below from the same
 * side (no silhouette there), both tests with a margin of 2^-16 of the box's
 * size plus distance; else its length sum times a cosine bound in (0, 1] over
 * (squared distance from p to the box centre + squared half diagonal); a fresh
 * uniform per level.  A node whose two children both weigh zero ends the draw
 * with no edge (the sample contributes nothing; no bias, since only edges that
 * cannot contribute are ever cut).  The point on the edge stays uniform and the
 * sample is weighted by length / probability.  The tree is built on the first
 * call that needs it after a scene change (allocates; not capturable).
 * Outputs: keys uint64 [ne], child int32 [ne-1,2], parent int32 [2ne-1], box
 * float [2ne-1,6], len float [2ne-1], nbox float [2ne-1,6] (normal box, lower
 * then upper corner); any may be NULL. */
int st_scene_edge_tree(st_scene* scene, uint64_t* keys, int32_t* child, int32_t* parent, float* box, float* len,
                       float* nbox, hipStream_t s);
int st_trace_rays(st_scene* scene, const float* o, const float* d, int32_t n, float tmin, int32_t brute,
                  int32_t* out_face, float* out_t, hipStream_t s);

/* Measurement reference: copies nbytes (a multiple of 16, 16-byte aligned
 * device pointers) from src to dst with a plain streaming kernel (non-temporal
 * 16-byte loads and stores), asynchronously on s.  Its bandwidth is the
 * achievable HBM rate the kernels' traffic is compared with. */
int st_stream_copy(void* dst, const void* src, int64_t nbytes, hipStream_t s);

/* Kernel timing for profiling harnesses: while enabled, every kernel the
 * library launches is bracketed by two HIP events recorded on its launch
 * stream.  st_profile_read waits for those events, writes the kernel names
 * (newline-separated, NUL-terminated, at most names_len bytes), the summed
 * milliseconds and the launch counts of up to max_kernels kernels in first-seen
 * order, clears the record, and returns the number of kernels (or < 0). */
int st_profile_enable(int on);
int st_profile_read(char* names, int32_t names_len, double* ms, int32_t* counts, int32_t max_kernels);

void st_scene_destroy(st_scene* scene);
const char* st_last_error(void);
int st_version(void);

#ifdef __cplusplus
}
#endif
#endif

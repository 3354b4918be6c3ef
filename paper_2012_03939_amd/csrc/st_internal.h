// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include "st_device.h"
#include "../../include/shapetrace.h"

#include <functional>

namespace st {

// optional per-kernel timing with HIP events recorded on the launch stream
void prof_begin(hipStream_t s, const char* name);
void prof_end(hipStream_t s);
extern bool g_prof_on;

#define ST_LAUNCH(name, kern, grid, block, shm, stream, ...)                   \
    do {                                                                        \
        if (st::g_prof_on) st::prof_begin(stream, name);                        \
        hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__);        \
        if (st::g_prof_on) st::prof_end(stream);                                \
    } while (0)

// every device allocation of one scene (library-owned)
constexpr int TREELET_ROUNDS = 1;   // bottom-up treelet-restructuring passes over the Karras tree (a second one
                                    // bought no measurable traversal time for its 1.9 ms)
constexpr int FACC = 16;   // gradient slots of one vertex: 3 corners x xyz, then the 7 material parameters
// Gradient accumulators are face-major, so that the slots one shading point adds
// to share a cache line: face f owns facc[16 f .. 16 f + 15] (corners in 0..8;
// without mesh colours its material in 9..15), and with mesh colours texel t owns
// macc[8 t .. 8 t + 6].
constexpr int FACC_STRIDE = 16, MACC_STRIDE = 8, FACC_MAT = 9;

struct SceneDev {
    int nv = 0, nf = 0, nl = 0, he = 0, we = 0, ne = 0;
    uint32_t scene_id = 0;
    bool has_env = false;
    float* V = nullptr;
    int* F = nullptr;
    int* vf_off = nullptr;                   // vertex -> (face, corner) CSR offsets [nv+1]
    int* fe = nullptr;                       // edge of face f from corner k to k+1 [3 nf] (-1: degenerate)
    int* vf_idx = nullptr;                   // entries 3 f + corner [3 nf]
    float* facc = nullptr;                   // per-face corner gradient accumulators [9, nf]
    float* macc = nullptr;                   // per-texel material gradient accumulators [7, ntex]
    int tex_res = 0;                         // mesh-colours resolution r
    int ntex = 0;                            // material rows: nf (r+1)(r+2)/2
    float* mat = nullptr;
    float* lights = nullptr;
    float* env = nullptr;
    // geometry build
    float4 *fnorm = nullptr, *bmin = nullptr, *bmax = nullptr, *cen = nullptr;
    float* bounds = nullptr;                 // lo[3], hi[3], scale[3]
    uint32_t* mkeys[2] = {nullptr, nullptr};
    uint32_t* mvals[2] = {nullptr, nullptr};
    uint32_t* rs_hist = nullptr;
    uint64_t* keys64 = nullptr;
    int* child = nullptr;                    // [2*(nf-1)]
    int* parent = nullptr;                   // [2*nf-1]
    float* aabb = nullptr;                   // [(2*nf-1)*6]
    int* refit_cnt = nullptr;
    float* tcost = nullptr;                  // [nf-1] SAH cost of every internal node's subtree
    // secondary-edge importance tree (built on demand): radix tree over the edge
    // boxes with per-node length sums; sorted leaf -> edge in evals_sorted
    float4 *ebmin = nullptr, *ebmax = nullptr, *ecen = nullptr;
    float* ebounds = nullptr;
    uint32_t* emkeys[2] = {nullptr, nullptr};
    uint32_t* emvals[2] = {nullptr, nullptr};
    uint32_t* ers_hist = nullptr;
    uint64_t* ekeys64 = nullptr;
    int *echild = nullptr, *eparent = nullptr, *ecnt = nullptr;
    float *eaabb = nullptr, *elen = nullptr, *enbox = nullptr;
    float4* enode = nullptr;                 // packed internal nodes of the edge tree (8 float4 each)
    const uint32_t* eleaf_edge = nullptr;    // points into emkeys/emvals after the sort
    int* tleaves = nullptr;                  // [nf-1] triangles below every internal node
    float4* nodes4 = nullptr;                // [(nf-1)*8] 4-wide nodes (at most nf-1 of them)
    int* flag4 = nullptr;                    // [nf-1] binary node starts a 4-wide node
    uint32_t* id4 = nullptr;                 // [nf-1] 4-wide node index of each such node
    float4* ccost = nullptr;                 // [nf-1] collapse cost of a subtree in 1..4 slots
    uint32_t* cdec = nullptr;                // [nf-1] collapse decisions (bit fields, see k_collapse_cost)
    float4* tri = nullptr;                   // [nf*3]
    int* fleaf = nullptr;                    // [nf] leaf index of each face
    // edges (topology fixed at creation)
    int4* edges = nullptr;
    double* edge_w = nullptr;
    int* eguide = nullptr;                   // guide table of ecdf
    int* mguide = nullptr;                   // guide table of the env marginal CDF
    int* cguide = nullptr;                   // guide tables of the env conditional CDFs
    double* ecdf = nullptr;
    double* etotal_d = nullptr;
    float* etotal_f = nullptr;
    // environment map
    double* row_dom = nullptr;               // [he] row solid angles
    float* rowcos = nullptr;                 // [he+1]
    double* cond = nullptr;
    double* marg = nullptr;
    double* env_rows = nullptr;
    double* env_total = nullptr;
    float* texpdf = nullptr;
    EnvAlias* ealias = nullptr;              // [he*we], built on the first request for alias sampling
    uint32_t* err = nullptr;                 // device error word
    unsigned long long* rec_key = nullptr;   // key of the forward pass whose hit records the scene holds (0: none)
    unsigned long long* work = nullptr;      // traversal work counters [3]
    DevScene* dscene = nullptr;              // device copy of the kernel view
    DevScene hscene;                         // host copy of the kernel view
};

// per-render workspace (grow-only)
struct Workspace {
    size_t bytes = 0;
    void* base = nullptr;
};

// columns of a ray queue (SoA, one float-sized word each): the ray and the state
// of the path it continues, copied along on compaction so that every kernel
// reads its queue entries coalesced
enum QCol {
    QOX, QOY, QOZ, QDX, QDY, QDZ,   // ray origin, direction
    QEXCL,                          // face the ray leaves (int), -1 for camera rays
    QPPREV,                         // BRDF pdf of the sampled direction (MIS at escape)
    QQ,                             // index of the path's radiance slot
    QC0, QC1,                       // Philox counter words c0, c1 of the path
    QVD,                            // camera index | stream domain << 16
    QBR, QBG, QBB,                  // throughput
    QHASH,                          // decision hash (debug outputs only)
    QNCOL
};

// queue and path-state arrays of one wavefront chunk (SoA)
constexpr int FETCH_INTS = 32 * FETCH_SLOT_INTS;   // slots k (shadow) and 16 + k (extension), k < 16

struct Queues {
    float* ray[2][QNCOL];    // queue of bounce k is ray[k & 1]
    float* ht;               // hit t
    int* hf;                 // hit face
    float* sx[3];            // shade record: hit point
    int* sface;              // shade record: face, -1 when no vertex
    uint32_t* sinfo;         // shade record: bit0 sampled, bit1 lobe, bit2 continued
    int* stex;               // shade record: env texel sampled
    int* snext;              // shade record: index of the continuation in the next queue, -1 if none
    float* sh[7];            // shadow entries [entry][i]: dir xyz, tmax, contrib rgb
    uint8_t* socc;           // shadow entry outcome [entry][i]: 0 no ray, 1 occluded, 2 unoccluded
    uint32_t* slist;         // shadow entries (l * cap + i) that carry a ray, compacted per bounce
    int* cnt;                // ray counts per bounce (k), shadow-ray counts per bounce (32 + k)
    int* fetch;              // fetch counters: slot k (shadow rays of bounce k), 16 + k (extension rays)
    uint32_t* spill;         // traversal stack spill
    float* L;                // per path sample radiance [total, 3] (processing order)
    int cap;                 // chunk capacity in paths
    int grid;                // blocks of the traversal kernels (<= TRACE_GRID)
    int nent;                // shadow entries per shading point (nl + env)
};

__device__ __forceinline__ uint32_t& qu(float* const* cols, int c, int i) { return ((uint32_t*)cols[c])[i]; }

// Queue streams (rays, hits, shading records, shadow entries) are written once
// and read once or twice per bounce, gigabytes per pass: with ST_QUEUE_NT they
// move with non-temporal hints, so that they do not evict the data the
// kernels do reuse from the caches (BVH nodes, triangles, materials, the
// environment map and its sampling tables).
#ifndef ST_QUEUE_NT
#define ST_QUEUE_NT 1
#endif
template <class T> __device__ __forceinline__ T qld(const T* p) {
#if ST_QUEUE_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <class T> __device__ __forceinline__ void qst(T* p, T v) {
#if ST_QUEUE_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}
__device__ __forceinline__ float qf(float* const* cols, int c, int i) { return qld(cols[c] + i); }
__device__ __forceinline__ uint32_t qu_ld(float* const* cols, int c, int i) { return qld((const uint32_t*)cols[c] + i); }
__device__ __forceinline__ void qf_st(float* const* cols, int c, int i, float v) { qst(cols[c] + i, v); }
__device__ __forceinline__ void qu_st(float* const* cols, int c, int i, uint32_t v) { qst((uint32_t*)cols[c] + i, v); }

struct FwdParams {
    const DevScene* scenes;
    const DevCam* cams;
    const long long* qoff;   // [ncam+1]
    int ncam, spp, B;
    uint32_t seed;
    uint32_t* dbg_hash;      // canonical order, optional
    uint32_t* err;
    unsigned long long* work;  // optional traversal counters
    uint32_t* hash_by_q;     // optional: final path hash stored at the path's radiance index
    int* rec_face;           // optional hit records of the main paths: face of bounce k at [(k-1) rec_n + path]
    uint32_t* rec_occ;       // occluded shadow entries (bit l) of bounce k at [(k-1) rec_n + path]
    long long rec_n;
    unsigned long long* rec_key_dev;  // with rec_face: the records' key word, cleared by the first camera kernel
};

void launch_scene_geometry(SceneDev& s, hipStream_t st);
void launch_edge_tree(SceneDev& s, hipStream_t st);
void launch_subdivide(const SceneDev& s, float* out_V, int32_t* out_F, hipStream_t st);
void launch_guide(const double* C, int n, size_t cstride, int rows, int* guide, int glog, hipStream_t st);
int guide_log2(int n);
void launch_env_build(SceneDev& s, hipStream_t st);

void launch_forward_wavefront(const FwdParams& p, Queues& q, long long total, int has_env_any, int nent,
                              hipStream_t st);
// an action run once, after the at-th launch of a sequence that ticks it
struct LaunchHook {
    int at = -1, count = 0;
    std::function<void()> fn;
    void tick() {
        if (++count == at && fn) fn();
    }
};
void launch_wavefront_bounces(const FwdParams& p, Queues& q, int n, int has_env_any, hipStream_t st,
                              LaunchHook* hook = nullptr);
void launch_forward_mega(const FwdParams& p, float* L, long long total, uint32_t* spill, int grid, hipStream_t st);
// key_dev (optional): receives key before the film is written (the forward is complete)
void launch_film(const DevCam* cams, const long long* pixoff, int ncam, int spp, const float* L,
                 long long npix, float* out, uint32_t* err, hipStream_t st, unsigned long long* key_dev = nullptr,
                 unsigned long long key = 0);
// sets ERR_NAN in *err when a[0..na) or b[0..nb) holds a non-finite value
void launch_check_finite(const float* a, long long na, const float* b, long long nb, uint32_t* err, hipStream_t st);
void launch_sample_radiance(const FwdParams& p, const float* L, long long total, float* out, hipStream_t st);

struct BwdParams {
    int rec_split;           // the main pass is split: a records-only pass, then one that traces if they are stale
    float* vrec;             // the adjoint's per-vertex replay records (adj_vrec_bytes)
    const DevScene* scenes;
    const DevCam* cams;
    const long long* qoff;   // [ncam+1] path offsets (processing order)
    const long long* eoff;   // [ncam+1] primary edge sample offsets
    int ncam, spp, B;
    uint32_t seed;
    uint32_t flags;
    const float* d_image;
    const uint8_t* path_mask;
    const uint8_t* edge_mask;
    float* dV;
    float* dmat;
    uint32_t* dbg_hash;
    uint32_t* dbg_edge_hash;
    uint32_t* err;
    unsigned long long* work;
    uint32_t* spill;
    double* pcdf;            // per-view primary edge CDF [ncam, ne+1]
    double* pw;              // per-view primary edge weights [ncam, ne]
    double* ptotal;          // [ncam]
    int* pguide;             // per-view guide tables of pcdf [ncam, 2^pglog]
    int pglog;
    double* pacc;            // per (view, edge): sums of c (1-t) and c t over its primary edge samples [ncam, ne, 2]
    int ne;
    double* lw;              // per-light shadow-edge weights [nl, ne]
    double* lcdf;            // per-light shadow-edge CDF [nl, ne+1]
    double* ltotal;          // [nl]
    int* lguide;             // per-light guide tables [nl, 2^pglog]
    float* facc;             // per-face corner accumulators [9, nf]: d/d(v0, v1, v2)
    float* macc;             // per-texel material accumulators [7, ntex]
    int ntex;
    const int* vf_off;       // vertex -> (face, corner) CSR of the scene
    const int* vf_idx;
    const int* rec_face;     // hit records held by the scene, or null (trace again)
    const uint32_t* rec_occ;
    long long rec_n;
    // the records are used only when the key the forward wrote next to them
    // (device word, stream-ordered, so also right after graph replays) equals the
    // key of this backward's cameras, spp, bounces, seed and scene version
    const unsigned long long* rec_key_dev;
    unsigned long long rec_key;
    // deferred secondary edges (null: traced inline): accepted vertices per path
    // (bit k), then the compacted (path, vertex) jobs and their count
    uint8_t* sec_mask;
    int2* sec_jobs;
    int* sec_njobs;
    // paths whose camera ray hit a face (the records pass of the adjoint walks
    // only these), or null
    uint32_t* adj_list;
    int* adj_n;
};

void launch_backward_prep(const BwdParams& p, int nf, long long total_paths, hipStream_t st);
void launch_backward(const BwdParams& p, int nv, int nf, long long total_paths, long long total_edges, int grid,
                     hipStream_t st);
void launch_face_gather(const BwdParams& p, int nv, hipStream_t st);
// bytes of the deferred secondary-edge workspace for total_paths paths of B bounces
size_t sec_workspace_bytes(long long total_paths, int B);
// the adjoint's path list: a counter (256 B) and one 32-bit path index per path
inline size_t adj_list_bytes(long long total_paths) { return 256 + sizeof(uint32_t) * (size_t)total_paths; }
void carve_sec_workspace(BwdParams& p, void* base, long long total_paths);
// primary edges with their side paths traced by the wavefront kernels
// point-light shadow boundaries (ST_EDGE_SHADOW); total_edges = primary edge samples
void launch_shadow_edges(const BwdParams& p, long long total_edges, int nl, hipStream_t st);
void launch_primary_edges(const BwdParams& p, const FwdParams& fp, Queues& q, float* Lside, uint32_t* hside,
                          long long total_edges, int has_env_any, hipStream_t st, LaunchHook* hook = nullptr);
void launch_fill_f32(float* p, long long n, float v, hipStream_t st);
void launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t st);
void launch_put_u64(unsigned long long* p, unsigned long long v, hipStream_t st);
void launch_stream_copy(float4* dst, const float4* src, long long n, hipStream_t st);
// copies nwords host words to dst through kernel arguments (no staging memory;
// a captured launch carries its own copy)
void launch_put_words(uint32_t* dst, const uint32_t* src, size_t nwords, hipStream_t st);
void launch_trace_debug(const DevScene* s, const float* o, const float* d, int n, float tmin, int brute,
                        int* out_face, float* out_t, uint32_t* spill, uint32_t* err, hipStream_t st);

constexpr int TRACE_BLOCK = 256;
static_assert(TRACE_BLOCK == TRAV_BLOCK, "traversal blocks size the LDS stack");
// largest grid of the traversal kernels; the spill stack has one column per thread of it
constexpr unsigned TRACE_GRID = 4096;
// the adjoint's per-vertex replay records: 27 slots per vertex of BM vertices
// for every thread of a grid of at most TRACE_GRID blocks of TRACE_BLOCK
constexpr int ADJ_VREC_SLOTS = 27;
inline int adj_bm(int B) { return B <= 1 ? 1 : B <= 2 ? 2 : B <= 3 ? 3 : 8; }
inline size_t adj_vrec_bytes(int B) {
    return sizeof(float) * (size_t)ADJ_VREC_SLOTS * adj_bm(B) * TRACE_GRID * TRACE_BLOCK;
}

} // namespace st

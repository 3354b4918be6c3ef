// Host side of the C ABI: validation, allocation, camera set-up, workspace
// management and kernel sequencing on the caller's stream.
#include "st_internal.h"
#include "../../include/shapetrace.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace st;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                                     \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return fail(ST_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// set while the current call's stream is being captured into a graph: no
// allocation may happen then
thread_local bool g_capturing = false;

// A grow-only device workspace.  Once a buffer has been handed to kernels
// recorded into a graph (stream capture), its memory must outlive that graph,
// which the library cannot see: a later growth then retires the allocation
// (freed with the scene) instead of freeing it.
struct GrowBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool captured = false;            // p was used by a captured launch
    std::vector<void*> retired;       // earlier allocations captured graphs may still use
    int ensure(size_t bytes) {
        if (bytes <= cap && p) {
            if (g_capturing) captured = true;
            return ST_OK;
        }
        if (g_capturing)
            return fail(ST_ERR_INVALID_ARG, "workspace would grow during graph capture: make one uncaptured call "
                                            "with the same shapes first");
        if (p) {
            if (captured) retired.push_back(p);
            else hipFree(p);
            p = nullptr;
            cap = 0;
            captured = false;
        }
        const size_t want = std::max<size_t>(bytes + bytes / 8, 256);
        if (hipMalloc(&p, want) != hipSuccess) { p = nullptr; return fail(ST_ERR_OOM, "device allocation failed"); }
        cap = want;
        return ST_OK;
    }
    void release() {
        if (p) hipFree(p);
        for (void* q : retired) hipFree(q);
        retired.clear();
        p = nullptr;
        cap = 0;
    }
};

// carve aligned sub-arrays out of one allocation
struct Carver {
    char* base;
    size_t off = 0;
    template <class T> T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* r = (T*)(base + off);
        off += n * sizeof(T);
        return r;
    }
};

template <class T> int dalloc(T** p, size_t n) {
    if (n == 0) n = 1;
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) { *p = nullptr; return fail(ST_ERR_OOM, "device allocation failed"); }
    return ST_OK;
}

// camera basis, written exactly like the specification (double precision)
struct D3 { double x, y, z; };
D3 sub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
double dotd(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
D3 scal(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
D3 crossd(D3 a, D3 b) { return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
D3 normd(D3 a) { double l = std::sqrt(dotd(a, a)); return scal(a, 1.0 / l); }

bool make_devcam(const st_camera& c, DevCam& o) {
    if (c.width < 1 || c.height < 1) return false;
    D3 eye{c.eye[0], c.eye[1], c.eye[2]}, tg{c.target[0], c.target[1], c.target[2]}, up{c.up[0], c.up[1], c.up[2]};
    D3 fv = sub(tg, eye);
    if (dotd(fv, fv) == 0.0 || dotd(up, up) == 0.0) return false;
    D3 f = normd(fv);
    D3 upn = normd(up);
    if (std::fabs(dotd(f, upn)) > 0.999) upn = D3{0, 0, 1};
    if (std::fabs(dotd(f, upn)) > 0.999) upn = D3{1, 0, 0};
    D3 r = normd(crossd(f, upn));
    D3 u = crossd(r, f);
    const double th = std::tan((double)c.fov_y_deg * 3.14159265358979323846 / 360.0);
    const double aspect = (double)c.width / (double)c.height;
    if (!(th > 0.0) || !std::isfinite(th)) return false;
    const double rs = th * aspect;
    o.eye[0] = c.eye[0]; o.eye[1] = c.eye[1]; o.eye[2] = c.eye[2];
    o.f[0] = (float)f.x; o.f[1] = (float)f.y; o.f[2] = (float)f.z;
    o.rs[0] = (float)(r.x * rs); o.rs[1] = (float)(r.y * rs); o.rs[2] = (float)(r.z * rs);
    o.us[0] = (float)(u.x * th); o.us[1] = (float)(u.y * th); o.us[2] = (float)(u.z * th);
    o.deye[0] = eye.x; o.deye[1] = eye.y; o.deye[2] = eye.z;
    o.df[0] = f.x; o.df[1] = f.y; o.df[2] = f.z;
    o.dr[0] = r.x; o.dr[1] = r.y; o.dr[2] = r.z;
    o.du[0] = u.x; o.du[1] = u.y; o.du[2] = u.z;
    o.dth = th;
    o.daspect = aspect;
    o.W = c.width;
    o.H = c.height;
    o.scene = 0;
    o.rngview = 0;
    return true;
}

} // namespace

// ---- per-kernel event profiler -------------------------------------------
namespace st {
bool g_prof_on = false;
}
namespace {
struct ProfRec { std::string name; hipEvent_t a, b; };
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_evpool;
hipEvent_t take_event() {
    if (!g_evpool.empty()) { hipEvent_t e = g_evpool.back(); g_evpool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}
} // namespace
void st::prof_begin(hipStream_t s, const char* name) {
    ProfRec r{name, take_event(), nullptr};
    hipEventRecord(r.a, s);
    g_prof.push_back(r);
}
void st::prof_end(hipStream_t s) {
    if (g_prof.empty()) return;
    g_prof.back().b = take_event();
    hipEventRecord(g_prof.back().b, s);
}

struct st_scene {
    SceneDev d;
    GrowBuf Lbuf, qbuf, spillbuf, primbuf, sidebuf, sidehash, secbuf;
    // immutable device tables of camera records, offsets and scene views, keyed
    // by content: written once by an uncaptured call, then reused (also by graphs)
    struct CamTable { uint64_t hash; std::vector<char> host; void* dev; void* pinned; };
    std::vector<CamTable> tables;
    long long tuned_cap = 0;           // autotuned wavefront chunk size (0: none)
    int tuned_grid = 0;                // autotuned traversal grid (0: none)
    // hit records of the last single-scene wavefront render, for its backward;
    // which forward they belong to is the device word d.rec_key
    GrowBuf recbuf;
    uint64_t version = 0;              // bumped by every change of geometry, materials or sampler
    uint64_t etree_version = ~0ull;    // scene version the edge importance tree was built for
    std::vector<void*> retired;        // replaced material arrays (captured graphs may still read them)
    // the adjoint of a backward runs on aux (forked from and joined back into the
    // caller's stream) while the primary edges' side paths run on the caller's
    // stream; its traversal stacks spill into spill_aux
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    GrowBuf spill_aux;
    GrowBuf adjbuf;                    // the adjoint's list of paths that have a vertex
    GrowBuf vrecbuf;                   // the adjoint's per-vertex replay records
};

namespace {

int check_scene(const st_scene* s) {
    if (!s) return fail(ST_ERR_INVALID_ARG, "scene is NULL");
    return ST_OK;
}

// stage camera records, offset tables and the scene table into device memory on stream s
struct CamSetup {
    DevCam* cams = nullptr;
    long long* qoff = nullptr;
    long long* pixoff = nullptr;
    long long* eoff = nullptr;
    DevScene* scenes = nullptr;
    long long total_paths = 0, total_pix = 0, total_edges = 0;
};

// camera records, offset tables and the scene table of a call, serialised on
// the host (each array 256-byte aligned) with their offsets in the blob
struct CamHost {
    std::vector<char> bytes;
    size_t o_cam = 0, o_q = 0, o_p = 0, o_e = 0, o_s = 0;
    long long total_paths = 0, total_pix = 0, total_edges = 0;
};

int build_cam_table(st_scene* const* scenes, int nscenes, const st_camera* cams, const int32_t* cam_scene,
                    int32_t ncam, int32_t spp, double ratio, CamHost& out) {
    if (!cams) return fail(ST_ERR_INVALID_ARG, "cams is NULL");
    if (ncam < 1 || ncam > 65535) return fail(ST_ERR_INVALID_ARG, "ncam must be in [1, 65535]");
    if (spp < 1 || spp > 65535) return fail(ST_ERR_INVALID_ARG, "spp must be in [1, 65535]");
    std::vector<DevCam> dc(ncam);
    std::vector<long long> qoff(ncam + 1), pix(ncam + 1), eoff(ncam + 1);
    std::vector<int> per_scene(nscenes, 0);
    long long q = 0, p = 0, e = 0;
    for (int i = 0; i < ncam; ++i) {
        if (!make_devcam(cams[i], dc[i])) return fail(ST_ERR_INVALID_ARG, "invalid camera " + std::to_string(i));
        const long long hw = (long long)cams[i].width * cams[i].height;
        if (hw >= (1ll << 31)) return fail(ST_ERR_INVALID_ARG, "image too large");
        dc[i].scene = cam_scene ? cam_scene[i] : 0;
        if (dc[i].scene < 0 || dc[i].scene >= nscenes) return fail(ST_ERR_INVALID_ARG, "cam_scene out of range");
        dc[i].rngview = per_scene[dc[i].scene]++;
        const long long ne = (long long)std::llround(ratio * (double)cams[i].width * (double)cams[i].height * (double)spp);
        dc[i].qoff = q; dc[i].pixoff = p; dc[i].eoff = e; dc[i].ne = ne;
        qoff[i] = q; pix[i] = p; eoff[i] = e;
        q += hw * spp; p += hw; e += ne;
    }
    qoff[ncam] = q; pix[ncam] = p; eoff[ncam] = e;
    if (q >= (1ll << 31)) return fail(ST_ERR_INVALID_ARG, "more than 2^31 path samples in one call");
    if (e >= (1ll << 40)) return fail(ST_ERR_INVALID_ARG, "too many edge samples");
    std::vector<char>& host = out.bytes;
    host.clear();
    size_t off = 0;
    auto put = [&](const void* src, size_t n) {
        const size_t at = off = (off + 255) & ~(size_t)255;
        off += n;
        host.resize(off);
        std::memcpy(host.data() + at, src, n);
        return at;
    };
    std::vector<DevScene> hs(nscenes);
    for (int i = 0; i < nscenes; ++i) hs[i] = scenes[i]->d.hscene;
    out.o_cam = put(dc.data(), sizeof(DevCam) * ncam);
    out.o_q = put(qoff.data(), sizeof(long long) * (ncam + 1));
    out.o_p = put(pix.data(), sizeof(long long) * (ncam + 1));
    out.o_e = put(eoff.data(), sizeof(long long) * (ncam + 1));
    out.o_s = put(hs.data(), sizeof(DevScene) * nscenes);
    out.total_paths = q;
    out.total_pix = p;
    out.total_edges = e;
    return ST_OK;
}

// device pointers of a serialised table placed at dev
void point_cams(const CamHost& h, char* dev, CamSetup& out) {
    out.cams = (DevCam*)(dev + h.o_cam);
    out.qoff = (long long*)(dev + h.o_q);
    out.pixoff = (long long*)(dev + h.o_p);
    out.eoff = (long long*)(dev + h.o_e);
    out.scenes = (DevScene*)(dev + h.o_s);
    out.total_paths = h.total_paths;
    out.total_pix = h.total_pix;
    out.total_edges = h.total_edges;
}

int setup_cams(st_scene* owner, st_scene* const* scenes, int nscenes, const st_camera* cams,
               const int32_t* cam_scene, int32_t ncam, int32_t spp, double ratio, hipStream_t s, CamSetup& out) {
    CamHost ch;
    int rc = build_cam_table(scenes, nscenes, cams, cam_scene, ncam, spp, ratio, ch);
    if (rc) return rc;
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(s, &cst));
    const bool capturing = cst != hipStreamCaptureStatusNone;
    g_capturing = capturing;
    // find or create the device copy of the table
    const std::vector<char>& host = ch.bytes;
    uint64_t hv = 1469598103934665603ull;      // FNV-1a 64 of the serialised table
    for (char c : host) { hv ^= (unsigned char)c; hv *= 1099511628211ull; }
    char* dev = nullptr;
    for (auto& t : owner->tables)
        if (t.hash == hv && t.host == host) { dev = (char*)t.dev; break; }
    if (!dev) {
        if (capturing)
            return fail(ST_ERR_INVALID_ARG, "cameras not staged: make one uncaptured call with the same cameras, "
                                            "spp and edge ratio before capturing");
        st_scene::CamTable t{hv, host, nullptr, nullptr};
        if (hipMalloc(&t.dev, host.size()) != hipSuccess) return fail(ST_ERR_OOM, "camera table allocation failed");
        if (hipHostMalloc(&t.pinned, host.size(), hipHostMallocDefault) != hipSuccess) {
            hipFree(t.dev);
            return fail(ST_ERR_OOM, "camera staging allocation failed");
        }
        std::memcpy(t.pinned, host.data(), host.size());
        HIPCHK(hipMemcpyAsync(t.dev, t.pinned, host.size(), hipMemcpyHostToDevice, s));
        owner->tables.push_back(std::move(t));
        dev = (char*)owner->tables.back().dev;
    }
    point_cams(ch, dev, out);
    return ST_OK;
}

// identity of a forward pass's main paths: cameras, spp, bounces, seed, the
// scene state and the record buffer written (a graph captured before the
// buffer grew writes its records into the retired one); never 0, which marks
// "no records"
uint64_t record_key(const st_scene* sc, const st_camera* cams, int ncam, int spp, int bounces, uint32_t seed,
                    const void* buf) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void* src, size_t n) {
        const unsigned char* b = (const unsigned char*)src;
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    mix(cams, sizeof(st_camera) * (size_t)ncam);
    const long long w[6] = {ncam, spp, bounces, (long long)seed, (long long)sc->version, (long long)(uintptr_t)buf};
    mix(w, sizeof(w));
    return h | 1ull;
}

constexpr size_t REC_MAX_BYTES = 16ull << 30;
// wavefront chunk (paths per pass of the bounce kernels) without tuning: each
// launch ends in a drain where its longest rays run alone, so larger chunks
// waste less; 2^24 paths hold about 3.3 GB of queues with one shadow entry
constexpr long long DEFAULT_QUEUE_CAP = 1ll << 24;

// chunk size for n items with at most cap per chunk: the same number of chunks,
// of equal size (rounded up to an even multiple of 256), so that no chunk is a
// small remainder paying a full set of launches
long long balanced_chunk(long long n, long long cap) {
    if (n <= cap) return std::max<long long>(n, 1);
    const long long chunks = (n + cap - 1) / cap;
    const long long c = ((n + chunks - 1) / chunks + 255) & ~255ll;
    return std::min(c, cap);
}


// wavefront chunk capacity actually used for a requested one (shadow entries
// are numbered l * n + i in a 32-bit index)
int queue_cap(long long cap, int nent) {
    return (int)std::min<long long>(cap, (0x7FFFFFFFll / std::max(nent, 1)) & ~1ll);
}

// bytes of the queue workspace of a chunk of cap paths with nent shadow entries each
size_t queue_bytes(int cap, int nent) {
    const size_t per = 256;
    const size_t words = 2 * QNCOL + 2 + 3 + 4 + 8 * (size_t)std::max(nent, 1);
    return (size_t)cap * 4 * words + (size_t)cap * std::max(nent, 1) + (words + 10) * per + 64 * 4 +
           FETCH_INTS * sizeof(int);
}

constexpr size_t SPILL_BYTES = (size_t)SPILL_STACK * TRACE_GRID * TRACE_BLOCK * sizeof(uint32_t);

int over_budget(const st_render_opts& o, size_t need) {
    if (o.max_workspace_bytes > 0 && need > (size_t)o.max_workspace_bytes)
        return fail(ST_ERR_OOM, "the call needs " + std::to_string(need) + " bytes of library workspace, more than "
                                "max_workspace_bytes = " + std::to_string((long long)o.max_workspace_bytes));
    return ST_OK;
}

int ensure_spill(st_scene* sc) {
    return sc->spillbuf.ensure(SPILL_BYTES);
}

// queue arrays of a chunk of cap paths (cap from queue_cap) carved out of base,
// which holds queue_bytes(cap, nent) bytes
void carve_queues(char* base, int cap, int nent, float* L, uint32_t* spill, Queues& q) {
    Carver c{base};
    for (int b = 0; b < 2; ++b)
        for (int i = 0; i < QNCOL; ++i) q.ray[b][i] = c.take<float>(cap);
    q.ht = c.take<float>(cap);
    q.hf = c.take<int>(cap);
    for (int i = 0; i < 3; ++i) q.sx[i] = c.take<float>(cap);
    q.sface = c.take<int>(cap);
    q.sinfo = c.take<uint32_t>(cap);
    q.stex = c.take<int>(cap);
    q.snext = c.take<int>(cap);
    for (int i = 0; i < 7; ++i) q.sh[i] = c.take<float>((size_t)cap * std::max(nent, 1));
    q.socc = c.take<uint8_t>((size_t)cap * std::max(nent, 1));
    q.slist = c.take<uint32_t>((size_t)cap * std::max(nent, 1));
    q.cnt = c.take<int>(64);
    q.fetch = c.take<int>(FETCH_INTS);
    q.spill = spill;
    q.L = L;
    q.cap = cap;
    q.grid = 0;
    q.nent = nent;
}

int make_queues(st_scene* sc, int cap, int nent, float* L, Queues& q) {
    cap = queue_cap(cap, nent);
    int rc = sc->qbuf.ensure(queue_bytes(cap, nent));
    if (rc) return rc;
    carve_queues((char*)sc->qbuf.p, cap, nent, L, (uint32_t*)sc->spillbuf.p, q);
    return ST_OK;
}

int render_impl(st_scene* owner, st_scene* const* scenes, int nscenes, const st_camera* cams, const int32_t* cam_scene,
                int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed, const st_render_opts* opts, float* out,
                hipStream_t s) {
    if (!out) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    if (bounces < 1 || bounces > 8) return fail(ST_ERR_INVALID_ARG, "bounces must be in [1, 8]");
    st_render_opts o = opts ? *opts : st_render_opts_default();
    CamSetup cs;
    int rc = setup_cams(owner, scenes, nscenes, cams, cam_scene, ncam, spp, 0.0, s, cs);
    if (rc) return rc;
    const DevScene* dscenes = cs.scenes;
    int nent = 0, has_env_any = 0;
    for (int i = 0; i < nscenes; ++i) {
        nent = std::max(nent, scenes[i]->d.nl + (scenes[i]->d.has_env ? 1 : 0));
        has_env_any |= scenes[i]->d.has_env ? 1 : 0;
    }
    // workspace of the call, checked against the caller's cap before any kernel
    const bool mega = (o.flags & ST_FORWARD_MEGAKERNEL) != 0;
    long long cap = o.queue_capacity > 0 ? o.queue_capacity : (owner->tuned_cap > 0 ? owner->tuned_cap : DEFAULT_QUEUE_CAP);
    cap = std::min<long long>(cap, 1ll << 28);
    cap = balanced_chunk(cs.total_paths, cap);
    const size_t need = (size_t)cs.total_paths * 3 * sizeof(float) + SPILL_BYTES +
                        (mega ? 0 : queue_bytes(queue_cap(cap, nent), nent));
    rc = over_budget(o, need);
    if (rc) return rc;
    rc = owner->Lbuf.ensure((size_t)cs.total_paths * 3 * sizeof(float));
    if (rc) return rc;
    rc = ensure_spill(owner);
    if (rc) return rc;
    FwdParams p;
    p.scenes = dscenes;
    p.cams = cs.cams;
    p.qoff = cs.qoff;
    p.ncam = ncam;
    p.spp = spp;
    p.B = bounces;
    p.seed = seed;
    p.dbg_hash = o.debug_decision_hash;
    p.err = owner->d.err;
    p.work = (o.flags & ST_COUNT_WORK) ? owner->d.work : nullptr;
    p.hash_by_q = nullptr;
    p.rec_face = nullptr;
    p.rec_occ = nullptr;
    p.rec_n = 0;
    // hit records for the backward of a single-scene wavefront render
    const size_t rec_bytes = (size_t)(2 * bounces + 1) * (size_t)cs.total_paths * sizeof(int);
    // (an optimisation of the backward: left out rather than exceed the cap)
    const bool want_rec = nscenes == 1 && !mega && scenes[0]->d.nl <= 30 && rec_bytes <= REC_MAX_BYTES &&
                          !(o.max_workspace_bytes > 0 && need + rec_bytes > (size_t)o.max_workspace_bytes);
    // the records' key (device word) is cleared by the first camera kernel of a
    // render that rewrites them and set by k_film once they are complete; a
    // render that keeps none leaves the records and their key as they are
    uint64_t rec_key = 0;
    p.rec_key_dev = nullptr;
    if (want_rec && !(g_capturing && owner->recbuf.cap < rec_bytes) && owner->recbuf.ensure(rec_bytes) == ST_OK) {
        p.rec_face = (int*)owner->recbuf.p;
        p.rec_occ = (uint32_t*)(p.rec_face + (size_t)(bounces + 1) * cs.total_paths);
        p.rec_n = cs.total_paths;
        p.rec_key_dev = owner->d.rec_key;
        rec_key = record_key(owner, cams, ncam, spp, bounces, seed, owner->recbuf.p);
    }
    float* L = (float*)owner->Lbuf.p;
    if (mega) {
        launch_forward_mega(p, L, cs.total_paths, (uint32_t*)owner->spillbuf.p, TRACE_GRID, s);
    } else {
        Queues q;
        rc = make_queues(owner, (int)cap, nent, L, q);
        if (rc) return rc;
        q.grid = owner->tuned_grid;
        launch_forward_wavefront(p, q, cs.total_paths, has_env_any, nent, s);
    }
    launch_film(cs.cams, cs.pixoff, ncam, spp, L, cs.total_pix, out, owner->d.err, s,
                rec_key ? owner->d.rec_key : nullptr, rec_key);
    if (o.debug_sample_radiance) launch_sample_radiance(p, L, cs.total_paths, o.debug_sample_radiance, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

// ---- the allocation-free render's scratch ----------------------------------
// One static device array per GPU (the code object holds it, so every device
// the library runs on keeps it until the process ends): camera table, traversal
// spill stack, per-sample radiance and the wavefront queues of
// st_render_noalloc.  Host code never uses the array's name as an address: the
// device address is looked up once per device with hipGetSymbolAddress.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
constexpr size_t NOALLOC_TABLE_BYTES = 32u << 10;
constexpr int NOALLOC_MAX_CAMS = 64;
constexpr long long NOALLOC_MAX_PATHS = 1ll << 20;
constexpr unsigned NOALLOC_TRACE_GRID = 512;      // traversal blocks: the spill stack has one column per thread
constexpr size_t NOALLOC_SPILL_BYTES = (size_t)SPILL_STACK * NOALLOC_TRACE_GRID * TRACE_BLOCK * sizeof(uint32_t);
constexpr int NOALLOC_MAX_DEVICES = 64;
static_assert(NOALLOC_TABLE_BYTES + NOALLOC_SPILL_BYTES + (size_t)NOALLOC_MAX_PATHS * 3 * sizeof(float) <
                  NOALLOC_SCRATCH_BYTES,
              "scratch layout");

static __device__ __align__(256) __attribute__((used)) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_addr[NOALLOC_MAX_DEVICES] = {};

// device address of the scratch array on the current device (looked up on the
// first request per device, with that device current)
int scratch_address(void** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(ST_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ST_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return ST_OK;
}

} // namespace

// The backward launches the adjoint on the scene's second stream after this many
// launches of the primary edges' side paths: after k_edge_camera, which then has
// the GPU to itself (2.7 ms) instead of waiting 11-12 ms for room beside the
// adjoint's first blocks; the adjoint overlaps the side paths' traversal instead.
constexpr int FORK_AFTER_LAUNCHES = 1;

extern "C" {

st_render_opts st_render_opts_default(void) {
    st_render_opts o;
    std::memset(&o, 0, sizeof(o));
    o.flags = ST_GRAD_INTERIOR | ST_EDGE_PRIMARY | ST_EDGE_SECONDARY | ST_EDGE_SHADOW;
    o.edge_spp_ratio = 1.0f;
    return o;
}

int st_version(void) { return 1; }

int st_profile_enable(int on) {
    g_prof_on = on != 0;
    return ST_OK;
}

int st_profile_read(char* names, int32_t names_len, double* ms, int32_t* counts, int32_t max_kernels) {
    // aggregate by kernel name in first-seen order; "name1\nname2\n..." into names
    std::vector<std::string> order;
    std::vector<double> tot;
    std::vector<int> cnt;
    for (auto& r : g_prof) {
        if (!r.b) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(ST_ERR_HIP, "event synchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(ST_ERR_HIP, "event elapsed failed");
        size_t k = 0;
        while (k < order.size() && order[k] != r.name) ++k;
        if (k == order.size()) { order.push_back(r.name); tot.push_back(0.0); cnt.push_back(0); }
        tot[k] += t;
        cnt[k] += 1;
    }
    for (auto& r : g_prof) { g_evpool.push_back(r.a); if (r.b) g_evpool.push_back(r.b); }
    g_prof.clear();
    std::string joined;
    const int n = std::min<int>((int)order.size(), max_kernels);
    for (int i = 0; i < n; ++i) {
        joined += order[i] + "\n";
        if (ms) ms[i] = tot[i];
        if (counts) counts[i] = cnt[i];
    }
    if (names && names_len > 0) {
        std::strncpy(names, joined.c_str(), names_len - 1);
        names[names_len - 1] = 0;
    }
    return n;
}

const char* st_last_error(void) { return g_err.c_str(); }

int st_scene_create(const float* V, int32_t nv, const int32_t* F, int32_t nf, const float* mat, const float* lights,
                    int32_t nl, const float* env, int32_t he, int32_t we, uint32_t scene_id, hipStream_t s,
                    st_scene** out) {
    if (!out) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!V || !F || !mat) return fail(ST_ERR_INVALID_ARG, "V, F and face_materials must be non-NULL");
    if (nv < 3 || nf < 1) return fail(ST_ERR_INVALID_ARG, "need nv >= 3 and nf >= 1");
    if (nl < 0 || nl > MAX_LIGHTS) return fail(ST_ERR_INVALID_ARG, "nl must be in [0, 16]");
    if (nl > 0 && !lights) return fail(ST_ERR_INVALID_ARG, "lights is NULL");
    if (env && (he < 1 || we < 1)) return fail(ST_ERR_INVALID_ARG, "envmap needs he, we >= 1");
    if (!env) he = we = 0;
    // topology on the host: validate indices and build the canonical edge list
    std::vector<int32_t> Fh(3 * (size_t)nf);
    HIPCHK(hipMemcpyAsync(Fh.data(), F, sizeof(int32_t) * Fh.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int32_t v : Fh)
        if (v < 0 || v >= nv) return fail(ST_ERR_INVALID_ARG, "face index out of range");
    // vertex -> (face, corner) incidence in CSR form, for the gather of per-face gradients
    std::vector<int32_t> vf_off((size_t)nv + 1, 0), vf_idx(3 * (size_t)nf);
    for (int32_t v : Fh) ++vf_off[(size_t)v + 1];
    for (int v = 0; v < nv; ++v) vf_off[(size_t)v + 1] += vf_off[v];
    {
        std::vector<int32_t> fill(vf_off.begin(), vf_off.end() - 1);
        for (int f = 0; f < nf; ++f)
            for (int k = 0; k < 3; ++k) vf_idx[fill[Fh[3 * f + k]]++] = 3 * f + k;
    }
    // half-edges (min vertex, max vertex, face, corner) sorted: equal edges are
    // adjacent; fe[3 f + k] = edge of face f from corner k to corner k+1
    std::vector<std::array<int, 4>> hes;
    hes.reserve(3 * (size_t)nf);
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            const int a = Fh[3 * f + k], b = Fh[3 * f + (k + 1) % 3];
            hes.push_back({std::min(a, b), std::max(a, b), f, k});
        }
    std::sort(hes.begin(), hes.end());
    std::vector<int4> edges;
    std::vector<int32_t> fe(3 * (size_t)nf, -1);
    for (size_t i = 0; i < hes.size();) {
        size_t j = i;
        while (j < hes.size() && hes[j][0] == hes[i][0] && hes[j][1] == hes[i][1]) ++j;
        if (hes[i][0] != hes[i][1]) {
            for (size_t m = i; m < j; ++m) fe[3 * (size_t)hes[m][2] + hes[m][3]] = (int32_t)edges.size();
            edges.push_back(make_int4(hes[i][0], hes[i][1], hes[i][2], j - i >= 2 ? hes[i + 1][2] : -1));
        }
        i = j;
    }

    st_scene* sc = new st_scene();
    if (hipStreamCreateWithFlags(&sc->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sc->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sc->ev_join, hipEventDisableTiming) != hipSuccess) {
        st_scene_destroy(sc);
        return fail(ST_ERR_HIP, "stream or event creation failed");
    }
    SceneDev& d = sc->d;
    d.nv = nv; d.nf = nf; d.nl = nl; d.he = he; d.we = we; d.ne = (int)edges.size(); d.scene_id = scene_id;
    d.tex_res = 0; d.ntex = nf;
    int rc = ST_OK;
    auto A = [&](int r) { if (r && !rc) rc = r; };
    A(dalloc(&d.V, 3 * (size_t)nv)); A(dalloc(&d.F, 3 * (size_t)nf)); A(dalloc(&d.mat, 7 * (size_t)nf));
    A(dalloc(&d.lights, 6 * (size_t)std::max(nl, 1)));
    A(dalloc(&d.fnorm, nf)); A(dalloc(&d.bmin, nf)); A(dalloc(&d.bmax, nf)); A(dalloc(&d.cen, nf));
    A(dalloc(&d.bounds, 16));
    for (int b = 0; b < 2; ++b) { A(dalloc(&d.mkeys[b], nf)); A(dalloc(&d.mvals[b], nf)); }
    A(dalloc(&d.rs_hist, 256 * (size_t)((nf + 1023) / 1024)));
    A(dalloc(&d.keys64, nf));
    A(dalloc(&d.child, 2 * (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.parent, 2 * (size_t)nf));
    A(dalloc(&d.aabb, 6 * (size_t)(2 * nf)));
    A(dalloc(&d.refit_cnt, (size_t)nf));
    A(dalloc(&d.tcost, (size_t)nf));
    A(dalloc(&d.tleaves, (size_t)nf));
    A(dalloc(&d.nodes4, 8 * (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.flag4, (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.id4, (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.ccost, (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.cdec, (size_t)std::max(nf - 1, 1)));
    A(dalloc(&d.tri, 3 * (size_t)nf));
    A(dalloc(&d.fleaf, (size_t)nf));
    A(dalloc(&d.vf_off, (size_t)nv + 1));
    A(dalloc(&d.fe, 3 * (size_t)nf));
    A(dalloc(&d.vf_idx, 3 * (size_t)nf));
    A(dalloc(&d.facc, FACC_STRIDE * (size_t)nf));
    A(dalloc(&d.macc, MACC_STRIDE));     // per-texel material slots exist only with mesh colours
    A(dalloc(&d.edges, edges.size()));
    A(dalloc(&d.edge_w, edges.size()));
    A(dalloc(&d.eguide, (size_t)1 << guide_log2((int)edges.size())));
    A(dalloc(&d.ecdf, edges.size() + 1));
    A(dalloc(&d.etotal_d, 1));
    A(dalloc(&d.etotal_f, 1));
    A(dalloc(&d.err, 1));
    A(dalloc(&d.rec_key, 1));
    A(dalloc(&d.work, 3 * WORK_SLOTS));
    A(dalloc(&d.dscene, 1));
    if (he > 0) {
        A(dalloc(&d.env, 3 * (size_t)he * we));
        A(dalloc(&d.row_dom, he));
        A(dalloc(&d.rowcos, 2 * (he + 1)));
        A(dalloc(&d.cond, (size_t)he * (we + 1)));
        A(dalloc(&d.marg, he + 1));
        A(dalloc(&d.env_rows, he));
        A(dalloc(&d.env_total, 1));
        A(dalloc(&d.texpdf, (size_t)he * we));
        A(dalloc(&d.mguide, (size_t)1 << guide_log2(he)));
        A(dalloc(&d.cguide, (size_t)he << guide_log2(we)));
    }
    if (rc) { st_scene_destroy(sc); return rc; }
    auto cleanup_fail = [&](int code, const std::string& m) { st_scene_destroy(sc); return fail(code, m); };
#define HIPCHK2(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return cleanup_fail(ST_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); } while (0)
    HIPCHK2(hipMemcpyAsync(d.V, V, sizeof(float) * 3 * nv, hipMemcpyDeviceToDevice, s));
    HIPCHK2(hipMemcpyAsync(d.F, F, sizeof(int) * 3 * nf, hipMemcpyDeviceToDevice, s));
    HIPCHK2(hipMemcpyAsync(d.mat, mat, sizeof(float) * 7 * nf, hipMemcpyDeviceToDevice, s));
    if (nl > 0) HIPCHK2(hipMemcpyAsync(d.lights, lights, sizeof(float) * 6 * nl, hipMemcpyDeviceToDevice, s));
    if (!edges.empty())
        HIPCHK2(hipMemcpyAsync(d.edges, edges.data(), sizeof(int4) * edges.size(), hipMemcpyHostToDevice, s));
    HIPCHK2(hipMemcpyAsync(d.vf_off, vf_off.data(), sizeof(int32_t) * vf_off.size(), hipMemcpyHostToDevice, s));
    HIPCHK2(hipMemcpyAsync(d.fe, fe.data(), sizeof(int32_t) * fe.size(), hipMemcpyHostToDevice, s));
    HIPCHK2(hipMemcpyAsync(d.vf_idx, vf_idx.data(), sizeof(int32_t) * vf_idx.size(), hipMemcpyHostToDevice, s));
    launch_fill_u32(d.err, 1, 0u, s);
    launch_put_u64(d.rec_key, 0ull, s);
    launch_fill_u32((uint32_t*)d.work, 6 * WORK_SLOTS, 0u, s);
    std::vector<double> dom(std::max(he, 1));
    std::vector<float> rowcos(2 * (he + 1));
    if (he > 0) {
        HIPCHK2(hipMemcpyAsync(d.env, env, sizeof(float) * 3 * (size_t)he * we, hipMemcpyDeviceToDevice, s));
        const double PI = 3.14159265358979323846;
        for (int r = 0; r < he; ++r) dom[r] = (2.0 * PI / we) * (std::cos(PI * r / he) - std::cos(PI * (r + 1) / he));
        for (int r = 0; r <= he; ++r) {
            const double h = 0.5 * PI * r / he;
            rowcos[r] = (float)(2.0 * std::sin(h) * std::sin(h));            // 1 - cos(pi r / he)
            rowcos[he + 1 + r] = (float)(2.0 * std::cos(h) * std::cos(h));   // 1 + cos(pi r / he)
        }
        HIPCHK2(hipMemcpyAsync(d.row_dom, dom.data(), sizeof(double) * he, hipMemcpyHostToDevice, s));
        HIPCHK2(hipMemcpyAsync(d.rowcos, rowcos.data(), sizeof(float) * 2 * (he + 1), hipMemcpyHostToDevice, s));
        launch_env_build(d, s);
    }
    launch_scene_geometry(d, s);
    HIPCHK2(hipGetLastError());
    double etot = 0.0;
    if (he > 0) HIPCHK2(hipMemcpyAsync(&etot, d.env_total, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK2(hipStreamSynchronize(s));
    d.has_env = he > 0 && etot > 0.0;
    DevScene& h = d.hscene;
    h.V = d.V; h.F = d.F; h.mat = d.mat; h.lights = d.lights; h.fnorm = d.fnorm; h.tri = d.tri; h.fleaf = d.fleaf; h.nodes4 = d.nodes4;
    h.env = d.env; h.marg = d.marg; h.cond = d.cond; h.texpdf = d.texpdf; h.rowcos = d.rowcos;
    h.edges = d.edges; h.ecdf = d.ecdf; h.etotal = d.etotal_f;
    h.eguide = d.eguide; h.mguide = d.mguide; h.cguide = d.cguide;
    h.eglog = guide_log2(d.ne); h.mglog = guide_log2(he); h.cglog = guide_log2(we);
    h.nv = nv; h.nf = nf; h.nl = nl; h.he = he; h.we = we; h.ne = d.ne; h.has_env = d.has_env ? 1 : 0;
    h.tex_res = 0;
    h.ealias = nullptr;
    h.env_alias = 0;
    h.vndf = 0;
    h.etchild = nullptr;
    h.etbox = nullptr;
    h.etlen = nullptr;
    h.etnbox = nullptr;
    h.etnode = nullptr;
    h.etedge = nullptr;
    h.scene_id = scene_id;
    HIPCHK2(hipMemcpyAsync(d.dscene, &h, sizeof(DevScene), hipMemcpyHostToDevice, s));
    HIPCHK2(hipStreamSynchronize(s));
#undef HIPCHK2
    // set-up of st_render_noalloc on this device, outside any capture (a failure
    // here is reported by st_render_noalloc itself, which looks again)
    void* scr = nullptr;
    if (scratch_address(&scr)) g_err.clear();
    *out = sc;
    return ST_OK;
}

int st_scene_update(st_scene* sc, const float* V, const float* mat, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (V) HIPCHK(hipMemcpyAsync(sc->d.V, V, sizeof(float) * 3 * sc->d.nv, hipMemcpyDeviceToDevice, s));
    if (mat) HIPCHK(hipMemcpyAsync(sc->d.mat, mat, sizeof(float) * 7 * (size_t)sc->d.ntex, hipMemcpyDeviceToDevice, s));
    if (V) launch_scene_geometry(sc->d, s);
    if (V || mat) ++sc->version;
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_scene_subdivide(const st_scene* sc, float* out_V, int32_t* out_F, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!out_V || !out_F) return fail(ST_ERR_INVALID_ARG, "out_V and out_F must be non-NULL");
    launch_subdivide(sc->d, out_V, out_F, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_scene_set_mesh_colors(st_scene* sc, int32_t r, const float* texels, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (r < 0 || r > 64) return fail(ST_ERR_INVALID_ARG, "mesh-colour resolution must be in [0, 64]");
    if (!texels) return fail(ST_ERR_INVALID_ARG, "texels is NULL");
    SceneDev& d = sc->d;
    const long long ntex = (long long)d.nf * ((r + 1) * (r + 2) / 2);
    if (7 * ntex >= (1ll << 31)) return fail(ST_ERR_INVALID_ARG, "too many texels (7 nf (r+1)(r+2)/2 must be < 2^31)");
    HIPCHK(hipStreamSynchronize(s));
    float *mat = nullptr, *macc = nullptr;
    if (dalloc(&mat, 7 * (size_t)ntex) || dalloc(&macc, MACC_STRIDE * (size_t)(r > 0 ? ntex : 1))) {
        if (mat) hipFree(mat);
        if (macc) hipFree(macc);
        return fail(ST_ERR_OOM, "texel arrays");
    }
    HIPCHK(hipMemcpyAsync(mat, texels, sizeof(float) * 7 * (size_t)ntex, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    sc->retired.push_back(d.mat);
    sc->retired.push_back(d.macc);
    d.mat = mat;
    d.macc = macc;
    d.tex_res = r;
    d.ntex = (int)ntex;
    d.hscene.mat = mat;
    d.hscene.tex_res = r;
    ++sc->version;
    HIPCHK(hipMemcpyAsync(d.dscene, &d.hscene, sizeof(DevScene), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return ST_OK;
}

// Texel probabilities of the environment map, as the CDFs and the pdf use them:
// mean of the three channels times the texel's solid angle, over the total;
// rows and the total summed in index order.  Then Vose's construction of the
// alias table: bins below their share on one stack, the rest on another, in
// index order; each step takes the top of both.
static void build_env_alias(const std::vector<float>& env, int he, int we, std::vector<EnvAlias>& out) {
    const double PI = 3.14159265358979323846;
    const size_t n = (size_t)he * we;
    std::vector<double> w(n), rows(he);
    for (int r = 0; r < he; ++r) {
        const double dom = (2.0 * PI / we) * (std::cos(PI * r / he) - std::cos(PI * (r + 1) / he));
        double rs = 0.0;
        for (int c = 0; c < we; ++c) {
            const float* t = &env[3 * ((size_t)r * we + c)];
            const double m = ((double)t[0] + (double)t[1] + (double)t[2]) / 3.0;
            w[(size_t)r * we + c] = m * dom;
            rs += m * dom;
        }
        rows[r] = rs;
    }
    double tot = 0.0;
    for (int r = 0; r < he; ++r) tot += rows[r];
    out.assign(n, EnvAlias{1.0, 0, 0});
    std::vector<double> share(n);
    std::vector<int> lo, hi;
    lo.reserve(n);
    hi.reserve(n);
    for (size_t i = 0; i < n; ++i) {
        out[i].alias = (int)i;
        share[i] = (w[i] / tot) * (double)n;
        (share[i] < 1.0 ? lo : hi).push_back((int)i);
    }
    while (!lo.empty() && !hi.empty()) {
        const int a = lo.back(), b = hi.back();
        lo.pop_back();
        hi.pop_back();
        out[a].prob = share[a];
        out[a].alias = b;
        share[b] = (share[b] + share[a]) - 1.0;
        (share[b] < 1.0 ? lo : hi).push_back(b);
    }
}

int st_scene_set_env_sampler(st_scene* sc, int32_t method, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    SceneDev& d = sc->d;
    if (method != ST_ENV_SAMPLER_CDF && method != ST_ENV_SAMPLER_ALIAS)
        return fail(ST_ERR_INVALID_ARG, "unknown environment sampler");
    if (!d.has_env) return fail(ST_ERR_INVALID_ARG, "scene has no environment map");
    HIPCHK(hipStreamSynchronize(s));
    if (method == ST_ENV_SAMPLER_ALIAS && !d.ealias) {
        const size_t n = (size_t)d.he * d.we;
        std::vector<float> env(3 * n);
        HIPCHK(hipMemcpyAsync(env.data(), d.env, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<EnvAlias> tab;
        build_env_alias(env, d.he, d.we, tab);
        if (dalloc(&d.ealias, n)) return fail(ST_ERR_OOM, "environment alias table");
        HIPCHK(hipMemcpyAsync(d.ealias, tab.data(), sizeof(EnvAlias) * n, hipMemcpyHostToDevice, s));
    }
    d.hscene.ealias = d.ealias;
    d.hscene.env_alias = method == ST_ENV_SAMPLER_ALIAS ? 1 : 0;
    ++sc->version;
    HIPCHK(hipMemcpyAsync(d.dscene, &d.hscene, sizeof(DevScene), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return ST_OK;
}

// the secondary-edge importance tree of the scene's current vertices (built,
// and its arrays allocated, on first use after a change)
static int ensure_edge_tree(st_scene* sc, hipStream_t s) {
    SceneDev& d = sc->d;
    if (d.ne <= 0 || sc->etree_version == sc->version) return ST_OK;
    if (!d.echild) {
        if (g_capturing) return fail(ST_ERR_INVALID_ARG, "edge tree not built: make one uncaptured call first");
        const size_t n = (size_t)d.ne;
        int rc = 0;
        auto A = [&](int r) { if (r && !rc) rc = r; };
        A(dalloc(&d.ebmin, n)); A(dalloc(&d.ebmax, n)); A(dalloc(&d.ecen, n)); A(dalloc(&d.ebounds, 16));
        for (int b = 0; b < 2; ++b) { A(dalloc(&d.emkeys[b], n)); A(dalloc(&d.emvals[b], n)); }
        A(dalloc(&d.ers_hist, 256 * ((n + 1023) / 1024)));
        A(dalloc(&d.ekeys64, n));
        A(dalloc(&d.echild, 2 * std::max<size_t>(n - 1, 1)));
        A(dalloc(&d.eparent, 2 * n - 1));
        A(dalloc(&d.ecnt, n));
        A(dalloc(&d.eaabb, 6 * (2 * n - 1)));
        A(dalloc(&d.elen, 2 * n - 1));
        A(dalloc(&d.enbox, 6 * (2 * n - 1)));
        A(dalloc(&d.enode, 8 * std::max<size_t>(n - 1, 1)));
        if (rc) return rc;
    }
    launch_edge_tree(d, s);
    d.hscene.etchild = d.echild;
    d.hscene.etbox = d.eaabb;
    d.hscene.etlen = d.elen;
    d.hscene.etnbox = d.enbox;
    d.hscene.etnode = d.enode;
    d.hscene.etedge = d.eleaf_edge;
    HIPCHK(hipMemcpyAsync(d.dscene, &d.hscene, sizeof(DevScene), hipMemcpyHostToDevice, s));
    HIPCHK(hipGetLastError());
    sc->etree_version = sc->version;
    return ST_OK;
}

int st_scene_edge_tree(st_scene* sc, uint64_t* keys, int32_t* child, int32_t* parent, float* box, float* len,
                       float* nbox, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    rc = ensure_edge_tree(sc, s);
    if (rc) return rc;
    const SceneDev& d = sc->d;
    const size_t n = (size_t)d.ne;
    if (n == 0) return ST_OK;
    if (keys) HIPCHK(hipMemcpyAsync(keys, d.ekeys64, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    if (child && n > 1) HIPCHK(hipMemcpyAsync(child, d.echild, sizeof(int) * 2 * (n - 1), hipMemcpyDeviceToDevice, s));
    if (parent) HIPCHK(hipMemcpyAsync(parent, d.eparent, sizeof(int) * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    if (box) HIPCHK(hipMemcpyAsync(box, d.eaabb, sizeof(float) * 6 * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    if (len) HIPCHK(hipMemcpyAsync(len, d.elen, sizeof(float) * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    if (nbox) HIPCHK(hipMemcpyAsync(nbox, d.enbox, sizeof(float) * 6 * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

int st_scene_set_bsdf_sampler(st_scene* sc, int32_t method, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (method != ST_BSDF_SAMPLER_HALFVECTOR && method != ST_BSDF_SAMPLER_VNDF)
        return fail(ST_ERR_INVALID_ARG, "unknown BRDF sampler");
    SceneDev& d = sc->d;
    d.hscene.vndf = method == ST_BSDF_SAMPLER_VNDF ? 1 : 0;
    ++sc->version;
    HIPCHK(hipMemcpyAsync(d.dscene, &d.hscene, sizeof(DevScene), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return ST_OK;
}

int st_scene_env_alias_table(const st_scene* sc, double* prob, int32_t* alias) {
    int rc = check_scene(sc);
    if (rc) return rc;
    const SceneDev& d = sc->d;
    if (!d.ealias) return fail(ST_ERR_INVALID_ARG, "no alias table (st_scene_set_env_sampler with ST_ENV_SAMPLER_ALIAS first)");
    const size_t n = (size_t)d.he * d.we;
    std::vector<EnvAlias> tab(n);
    HIPCHK(hipMemcpy(tab.data(), d.ealias, sizeof(EnvAlias) * n, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) {
        if (prob) prob[i] = tab[i].prob;
        if (alias) alias[i] = tab[i].alias;
    }
    return ST_OK;
}

int st_scene_mesh_colors_info(const st_scene* sc, int32_t* r, int64_t* ntex) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (r) *r = sc->d.tex_res;
    if (ntex) *ntex = sc->d.ntex;
    return ST_OK;
}

int st_render(st_scene* sc, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed,
              const st_render_opts* opts, float* out, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    st_scene* list[1] = {sc};
    return render_impl(sc, list, 1, cams, nullptr, ncam, spp, bounces, seed, opts, out, s);
}

int st_render_noalloc(st_scene* sc, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed,
                      const st_render_opts* opts, float* out, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!out) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    if (bounces < 1 || bounces > 8) return fail(ST_ERR_INVALID_ARG, "bounces must be in [1, 8]");
    if (ncam > NOALLOC_MAX_CAMS)
        return fail(ST_ERR_INVALID_ARG, "st_render_noalloc: at most " + std::to_string(NOALLOC_MAX_CAMS) + " cameras");
    st_render_opts o = opts ? *opts : st_render_opts_default();
    st_scene* list[1] = {sc};
    CamHost ch;
    rc = build_cam_table(list, 1, cams, nullptr, ncam, spp, 0.0, ch);
    if (rc) return rc;
    if (ch.total_paths > NOALLOC_MAX_PATHS)
        return fail(ST_ERR_INVALID_ARG, "st_render_noalloc: " + std::to_string(ch.total_paths) +
                                            " path samples exceed its static scratch limit of " +
                                            std::to_string(NOALLOC_MAX_PATHS));
    if (ch.bytes.size() > NOALLOC_TABLE_BYTES) return fail(ST_ERR_INVALID_ARG, "st_render_noalloc: camera table too large");
    void* scr = nullptr;
    rc = scratch_address(&scr);
    if (rc) return rc;
    // scratch layout: camera table | spill stack | radiance per path sample | queues
    char* const base = (char*)scr;
    uint32_t* const spill = (uint32_t*)(base + NOALLOC_TABLE_BYTES);
    float* const L = (float*)(base + NOALLOC_TABLE_BYTES + NOALLOC_SPILL_BYTES);
    const size_t lbytes = (((size_t)ch.total_paths * 3 * sizeof(float)) + 255) & ~(size_t)255;
    char* const qbase = (char*)L + lbytes;
    const size_t qroom = NOALLOC_SCRATCH_BYTES - NOALLOC_TABLE_BYTES - NOALLOC_SPILL_BYTES - lbytes;
    const int nent = sc->d.nl + (sc->d.has_env ? 1 : 0);
    const bool mega = (o.flags & ST_FORWARD_MEGAKERNEL) != 0;
    int cap = 0;
    if (!mega) {
        // the largest chunk whose queues fit the rest of the scratch
        const size_t words = 2 * QNCOL + 2 + 3 + 4 + 8 * (size_t)std::max(nent, 1);
        const size_t per = 4 * words + (size_t)std::max(nent, 1), fixed = queue_bytes(0, nent);
        long long c = qroom > fixed ? (long long)((qroom - fixed) / per) : 0;
        c = std::min<long long>(c, std::max<long long>(ch.total_paths, 1));
        if (o.queue_capacity > 0) c = std::min<long long>(c, o.queue_capacity);
        c = queue_cap(c, nent);
        while (c > 0 && queue_bytes((int)c, nent) > qroom) --c;
        if (c < 1) return fail(ST_ERR_INVALID_ARG, "st_render_noalloc: no room for the wavefront queues");
        cap = (int)c;
    }
    // the table goes in through kernel arguments (no staging memory)
    std::vector<uint32_t> words((ch.bytes.size() + 3) / 4, 0u);
    std::memcpy(words.data(), ch.bytes.data(), ch.bytes.size());
    launch_put_words((uint32_t*)base, words.data(), words.size(), s);
    CamSetup cs;
    point_cams(ch, base, cs);
    FwdParams p;
    p.scenes = cs.scenes;
    p.cams = cs.cams;
    p.qoff = cs.qoff;
    p.ncam = ncam;
    p.spp = spp;
    p.B = bounces;
    p.seed = seed;
    p.dbg_hash = o.debug_decision_hash;
    p.err = sc->d.err;
    p.work = (o.flags & ST_COUNT_WORK) ? sc->d.work : nullptr;
    p.hash_by_q = nullptr;
    p.rec_face = nullptr;        // no hit records: the scene's record buffer is not touched
    p.rec_occ = nullptr;
    p.rec_n = 0;
    p.rec_key_dev = nullptr;
    if (mega) {
        launch_forward_mega(p, L, cs.total_paths, spill, NOALLOC_TRACE_GRID, s);
    } else {
        Queues q;
        carve_queues(qbase, cap, nent, L, spill, q);
        q.grid = NOALLOC_TRACE_GRID;
        launch_forward_wavefront(p, q, cs.total_paths, sc->d.has_env ? 1 : 0, nent, s);
    }
    launch_film(cs.cams, cs.pixoff, ncam, spp, L, cs.total_pix, out, sc->d.err, s);
    if (o.debug_sample_radiance) launch_sample_radiance(p, L, cs.total_paths, o.debug_sample_radiance, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_render_batch(st_scene* const* scenes, int32_t nscenes, const st_camera* cams, const int32_t* cam_scene,
                    int32_t ncam, int32_t spp, int32_t bounces, uint32_t seed, const st_render_opts* opts,
                    float* out, hipStream_t s) {
    if (!scenes || nscenes < 1) return fail(ST_ERR_INVALID_ARG, "need at least one scene");
    for (int i = 0; i < nscenes; ++i)
        if (!scenes[i]) return fail(ST_ERR_INVALID_ARG, "scene is NULL");
    if (!cam_scene) return fail(ST_ERR_INVALID_ARG, "cam_scene is NULL");
    return render_impl(scenes[0], scenes, nscenes, cams, cam_scene, ncam, spp, bounces, seed, opts, out, s);
}

int st_render_backward(st_scene* sc, const st_camera* cams, int32_t ncam, int32_t spp, int32_t bounces,
                       uint32_t seed, const st_render_opts* opts, const float* d_image, float* out_dV,
                       float* out_dmat, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!d_image || !out_dV || !out_dmat) return fail(ST_ERR_INVALID_ARG, "d_image, out_dV and out_dmat must be non-NULL");
    if (bounces < 1 || bounces > 8) return fail(ST_ERR_INVALID_ARG, "bounces must be in [1, 8]");
    st_render_opts o = opts ? *opts : st_render_opts_default();
    if (!(o.edge_spp_ratio >= 0.0f) || o.edge_spp_ratio > 64.0f) return fail(ST_ERR_INVALID_ARG, "edge_spp_ratio must be in [0, 64]");
    if ((o.flags & ST_EDGE_SECONDARY) && (o.flags & ST_EDGE_SECONDARY_HIERARCHY)) {
        // before the camera table: it holds a copy of the scene view with the tree
        rc = ensure_edge_tree(sc, s);
        if (rc) return rc;
    }
    CamSetup cs;
    st_scene* list[1] = {sc};
    rc = setup_cams(sc, list, 1, cams, nullptr, ncam, spp, (double)o.edge_spp_ratio, s, cs);
    if (rc) return rc;
    const int ne = sc->d.ne;
    const int pglog = guide_log2(ne);
    const int nls = (o.flags & ST_EDGE_SHADOW) ? sc->d.nl : 0;     // lights with shadow-edge tables
    const size_t pbytes = sizeof(double) * ((size_t)ncam * ne + (size_t)ncam * (ne + 1) + ncam) +
                          sizeof(int) * ((size_t)ncam << pglog) + sizeof(double) * 2 * (size_t)ncam * ne +
                          sizeof(double) * ((size_t)nls * ne + (size_t)nls * (ne + 1) + nls) +
                          sizeof(int) * ((size_t)nls << pglog) + 9 * 256;
    // workspace of the call, checked against the caller's cap before any kernel:
    // spill stack, edge tables, deferred secondary-edge jobs and, for the primary
    // edges, the side paths' radiance (and hashes) and their wavefront queues
    const bool defer_sec = (o.flags & ST_EDGE_SECONDARY) && !o.debug_decision_hash && cs.total_paths > 0 && ne > 0;
    const bool prim = (o.flags & ST_EDGE_PRIMARY) && cs.total_edges > 0 && ne > 0;
    const int nent_side = sc->d.nl + (sc->d.has_env ? 1 : 0);
    long long side_cap = o.queue_capacity > 0 ? o.queue_capacity : (sc->tuned_cap > 0 ? sc->tuned_cap : DEFAULT_QUEUE_CAP);
    side_cap = std::min<long long>(side_cap, 1ll << 28);
    side_cap = balanced_chunk(2 * cs.total_edges, side_cap) & ~1ll;     // two side paths per edge sample
    if (prim && 2 * cs.total_edges >= (1ll << 32)) return fail(ST_ERR_INVALID_ARG, "too many primary edge samples");
    // hit records of this pass's forward, when the scene holds them in a buffer
    // large enough (the adjoint still checks on the device that they are this
    // pass's); with them and no inline secondary-edge side paths, the adjoint's
    // records pass walks a list of the paths that have a vertex (not with
    // decision hashes, which every path writes)
    const size_t rec_bytes = (size_t)(2 * bounces + 1) * (size_t)cs.total_paths * sizeof(int);
    const bool recs_fit = !(o.flags & ST_BACKWARD_RETRACE) && sc->recbuf.p && sc->recbuf.cap >= rec_bytes;
    const bool adj_listed = recs_fit && (defer_sec || !(o.flags & ST_EDGE_SECONDARY)) && !o.debug_decision_hash &&
                            cs.total_paths > 0 && cs.total_paths < (1ll << 31);
    {
        size_t need = SPILL_BYTES + pbytes + (defer_sec ? sec_workspace_bytes(cs.total_paths, bounces) : 0) +
                      (adj_listed ? adj_list_bytes(cs.total_paths) : 0) +
                      ((o.flags & 5u) && cs.total_paths > 0 ? adj_vrec_bytes(bounces) : 0);
        if (prim)
            need += (size_t)cs.total_edges * 6 * sizeof(float) +
                    (o.debug_edge_hash ? (size_t)cs.total_edges * 2 * sizeof(uint32_t) : 0) +
                    queue_bytes(queue_cap(side_cap, nent_side), nent_side);
        rc = over_budget(o, need);
        if (rc) return rc;
    }
    rc = ensure_spill(sc);
    if (rc) return rc;
    rc = sc->primbuf.ensure(pbytes);
    if (rc) return rc;
    Carver c{(char*)sc->primbuf.p};
    BwdParams p;
    p.scenes = cs.scenes;
    p.cams = cs.cams;
    p.qoff = cs.qoff;
    p.eoff = cs.eoff;
    p.ncam = ncam;
    p.spp = spp;
    p.B = bounces;
    p.seed = seed;
    p.flags = o.flags & (15u | ST_EDGE_SECONDARY_INTERIOR | ST_EDGE_SECONDARY_HIERARCHY);
    p.d_image = d_image;
    p.path_mask = o.path_mask;
    p.edge_mask = o.edge_mask;
    p.dV = out_dV;
    p.dmat = out_dmat;
    p.dbg_hash = o.debug_decision_hash;
    p.dbg_edge_hash = o.debug_edge_hash;
    p.err = sc->d.err;
    p.work = (o.flags & ST_COUNT_WORK) ? sc->d.work : nullptr;
    p.spill = (uint32_t*)sc->spillbuf.p;
    p.pw = c.take<double>((size_t)ncam * ne);
    p.pcdf = c.take<double>((size_t)ncam * (ne + 1));
    p.ptotal = c.take<double>(ncam);
    p.pguide = c.take<int>((size_t)ncam << pglog);
    p.pglog = pglog;
    p.pacc = c.take<double>(2 * (size_t)ncam * ne);
    p.lw = c.take<double>((size_t)nls * ne);
    p.lcdf = c.take<double>((size_t)nls * (ne + 1));
    p.ltotal = c.take<double>(nls);
    p.lguide = c.take<int>((size_t)nls << pglog);
    p.facc = sc->d.facc;
    p.macc = sc->d.macc;
    p.ntex = sc->d.ntex;
    p.vf_off = sc->d.vf_off;
    p.vf_idx = sc->d.vf_idx;
    p.ne = ne;
    // the records are offered when they can hold this pass's paths; the adjoint
    // takes them only if the key its forward wrote on the device matches
    const bool offer_rec = recs_fit && sc->recbuf.ensure(rec_bytes) == ST_OK;
    p.rec_face = offer_rec ? (const int*)sc->recbuf.p : nullptr;
    p.rec_occ = offer_rec ? (const uint32_t*)((const int*)sc->recbuf.p + (size_t)(bounces + 1) * cs.total_paths) : nullptr;
    p.rec_n = offer_rec ? cs.total_paths : 0;
    p.rec_key_dev = sc->d.rec_key;
    p.rec_key = record_key(sc, cams, ncam, spp, bounces, seed, sc->recbuf.p);
    // secondary edges deferred to a job pass (not when decision hashes are asked for:
    // those follow the inline order)
    p.sec_mask = nullptr;
    p.sec_jobs = nullptr;
    p.sec_njobs = nullptr;
    if (defer_sec) {
        rc = sc->secbuf.ensure(sec_workspace_bytes(cs.total_paths, bounces));
        if (rc) return rc;
        carve_sec_workspace(p, sc->secbuf.p, cs.total_paths);
    }
    // records offered and no inline secondary-edge side paths: the main pass of
    // the adjoint runs first without traversal (see k_adjoint)
    p.rec_split = p.rec_face != nullptr && (p.sec_mask != nullptr || !(p.flags & 4u)) ? 1 : 0;
    p.adj_list = nullptr;
    p.adj_n = nullptr;
    if (p.rec_split && adj_listed) {
        rc = sc->adjbuf.ensure(adj_list_bytes(cs.total_paths));
        if (rc) return rc;
        p.adj_n = (int*)sc->adjbuf.p;
        p.adj_list = (uint32_t*)((char*)sc->adjbuf.p + 256);
    }
    launch_fill_f32(out_dV, 3ll * sc->d.nv, 0.0f, s);
    launch_fill_f32(out_dmat, 7ll * sc->d.ntex, 0.0f, s);
    if (o.debug_decision_hash) launch_fill_u32(o.debug_decision_hash, cs.total_paths, 0u, s);
    if (o.debug_edge_hash) launch_fill_u32(o.debug_edge_hash, cs.total_edges * (1 + nls), 0u, s);
    // The adjoint (latency-bound: dependent gathers at four waves per SIMD) and the
    // primary edges' side paths (issue-bound traversal) share nothing but atomics
    // into dV, so outside graph capture the adjoint runs on the scene's second
    // stream, with its own traversal spill region, while the side paths run here;
    // the per-face gather into dV waits for both.
    const bool adjoint = (p.flags & 5u) && cs.total_paths > 0;
    const bool overlap = adjoint && prim && !g_capturing;
    p.vrec = nullptr;
    if (adjoint) {
        rc = sc->vrecbuf.ensure(adj_vrec_bytes(bounces));
        if (rc) return rc;
        p.vrec = (float*)sc->vrecbuf.p;
    }
    // every workspace first: between the fork and the join nothing may fail
    uint32_t* hside = nullptr;
    Queues q;
    if (prim) {
        rc = sc->sidebuf.ensure((size_t)cs.total_edges * 6 * sizeof(float));
        if (rc) return rc;
        if (o.debug_edge_hash) {
            rc = sc->sidehash.ensure((size_t)cs.total_edges * 2 * sizeof(uint32_t));
            if (rc) return rc;
            hside = (uint32_t*)sc->sidehash.p;
        }
        rc = make_queues(sc, (int)side_cap, nent_side, (float*)sc->sidebuf.p, q);
        if (rc) return rc;
        q.grid = sc->tuned_grid;
    }
    if (overlap) {
        rc = sc->spill_aux.ensure(SPILL_BYTES);
        if (rc) return rc;
    }
    // the adjoint's launch on the second stream, after the side paths' first
    // FORK_AFTER_LAUNCHES launches on this one (at once when there are none)
    bool forked = false;
    auto fork = [&]() {
        forked = true;
        BwdParams pa = p;
        pa.spill = (uint32_t*)sc->spill_aux.p;
        const hipError_t e = hipEventRecord(sc->ev_fork, s);
        // a record or wait that fails leaves aux unordered after s: the adjoint then runs here
        if (e == hipSuccess && hipStreamWaitEvent(sc->aux, sc->ev_fork, 0) == hipSuccess)
            launch_backward(pa, sc->d.nv, sc->d.nf, cs.total_paths, cs.total_edges, TRACE_GRID, sc->aux);
        else
            launch_backward(p, sc->d.nv, sc->d.nf, cs.total_paths, cs.total_edges, TRACE_GRID, s);
    };
    // the adjoint's preparation runs on this stream in either case, before any fork
    if (adjoint) launch_backward_prep(p, sc->d.nf, cs.total_paths, s);
    LaunchHook hook;
    if (overlap) {
        if (FORK_AFTER_LAUNCHES <= 0) fork();
        hook.at = FORK_AFTER_LAUNCHES;
        hook.fn = fork;
    } else if (adjoint) {
        launch_backward(p, sc->d.nv, sc->d.nf, cs.total_paths, cs.total_edges, TRACE_GRID, s);
    }
    if (prim) {
        // side paths of the primary edge samples run through the wavefront kernels
        FwdParams fp;
        fp.scenes = cs.scenes;
        fp.cams = cs.cams;
        fp.qoff = cs.qoff;
        fp.ncam = ncam;
        fp.spp = spp;
        fp.B = bounces;
        fp.seed = seed;
        fp.dbg_hash = nullptr;
        fp.err = sc->d.err;
        fp.work = p.work;
        fp.hash_by_q = hside;
        fp.rec_face = nullptr;
        fp.rec_occ = nullptr;
        fp.rec_n = 0;
        fp.rec_key_dev = nullptr;
        launch_primary_edges(p, fp, q, (float*)sc->sidebuf.p, hside, cs.total_edges, sc->d.has_env ? 1 : 0, s,
                             overlap && !forked ? &hook : nullptr);
    }
    if (overlap && !forked) fork();
    if (nls > 0) launch_shadow_edges(p, cs.total_edges, nls, s);
    if (overlap) {
        // the join (an event recorded on aux after its last kernel, waited on here)
        HIPCHK(hipEventRecord(sc->ev_join, sc->aux));
        HIPCHK(hipStreamWaitEvent(s, sc->ev_join, 0));
    }
    if (adjoint) launch_face_gather(p, sc->d.nv, s);
    // every term has been added: a non-finite gradient sets the error word
    launch_check_finite(out_dV, 3ll * sc->d.nv, out_dmat, 7ll * sc->d.ntex, sc->d.err, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_autotune(st_scene* const* scenes, int32_t nscenes, const st_camera* cams, const int32_t* cam_scene,
                int32_t ncam, int32_t spp, int32_t bounces, const char* cache_path, int64_t* out_queue_capacity,
                int32_t* out_trace_grid, hipStream_t s) {
    if (!scenes || nscenes < 1) return fail(ST_ERR_INVALID_ARG, "need at least one scene");
    for (int i = 0; i < nscenes; ++i)
        if (!scenes[i]) return fail(ST_ERR_INVALID_ARG, "scene is NULL");
    if (nscenes > 1 && !cam_scene) return fail(ST_ERR_INVALID_ARG, "cam_scene is NULL");
    if (!cams || ncam < 1 || spp < 1 || bounces < 1 || bounces > 8) return fail(ST_ERR_INVALID_ARG, "bad workload");
    // workload signature
    long long paths = 0, pix = 0, faces = 0;
    int env = 0, lights = 0;
    for (int i = 0; i < ncam; ++i) { pix += (long long)cams[i].width * cams[i].height; }
    paths = pix * spp;
    for (int i = 0; i < nscenes; ++i) { faces += scenes[i]->d.nf; env += scenes[i]->d.has_env; lights += scenes[i]->d.nl; }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    char sig[256];
    std::snprintf(sig, sizeof(sig), "scenes=%d faces=%lld views=%d paths=%lld bounces=%d env=%d lights=%d", nscenes,
                  faces, ncam, paths, bounces, env, lights);
    std::string device = std::string(prop.gcnArchName) + " cu=" + std::to_string(prop.multiProcessorCount);
    long long best_cap = 0;
    int best_grid = 0;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[1024];
            while (std::fgets(line, sizeof(line), f)) {
                std::string l(line);
                if (l.find("\"device\": \"" + device + "\"") == std::string::npos) continue;
                if (l.find("\"key\": \"" + std::string(sig) + "\"") == std::string::npos) continue;
                const size_t a0 = l.find("\"queue_capacity\": "), a1 = l.find("\"trace_grid\": ");
                if (a0 == std::string::npos || a1 == std::string::npos) continue;
                best_cap = std::atoll(l.c_str() + a0 + 18);
                best_grid = std::atoi(l.c_str() + a1 + 14);
            }
            std::fclose(f);
        }
    }
    if (best_cap <= 0) {
        float* out = nullptr;
        if (hipMalloc((void**)&out, sizeof(float) * 3 * (size_t)pix) != hipSuccess) return fail(ST_ERR_OOM, "autotune buffer");
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const long long caps[] = {1ll << 27, 1ll << 26, 1ll << 25, 1ll << 24, 1ll << 23, 1ll << 22, 1ll << 21, 1ll << 20};
        const int grids[] = {4096, 2048, 1024};
        float best_ms = 1e30f;
        st_render_opts o = st_render_opts_default();
        int rc = ST_OK;
        for (long long cap : caps) {
            if (cap > 2 * std::max(paths, 1ll) && cap != (1ll << 20)) continue;
            for (int grid : grids) {
                for (int i = 0; i < nscenes; ++i) { scenes[i]->tuned_cap = cap; scenes[i]->tuned_grid = grid; }
                float ms = 1e30f;
                for (int rep = 0; rep < 3 && rc == ST_OK; ++rep) {
                    HIPCHK(hipEventRecord(e0, s));
                    rc = render_impl(scenes[0], scenes, nscenes, cams, cam_scene, ncam, spp, bounces, 0, &o, out, s);
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    float t = 0.f;
                    HIPCHK(hipEventElapsedTime(&t, e0, e1));
                    if (rep > 0) ms = std::min(ms, t);     // the first run may allocate
                }
                if (rc) break;
                // candidates come largest chunk and grid first, and a later one must be 3 %
                // faster to replace the best: the forward alone barely separates the large
                // chunks, and the backward's primary-edge side paths (twice the forward's
                // paths) run in fewer chunks the larger they are
                if (ms < best_ms * 0.97f) { best_ms = ms; best_cap = cap; best_grid = grid; }
            }
            if (rc) break;
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipFree(out);
        if (rc) return rc;
        if (cache_path) {
            if (FILE* f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "{\"device\": \"%s\", \"key\": \"%s\", \"queue_capacity\": %lld, \"trace_grid\": %d, \"ms\": %.4f}\n",
                             device.c_str(), sig, best_cap, best_grid, best_ms);
                std::fclose(f);
            }
        }
    }
    for (int i = 0; i < nscenes; ++i) { scenes[i]->tuned_cap = best_cap; scenes[i]->tuned_grid = best_grid; }
    if (out_queue_capacity) *out_queue_capacity = best_cap;
    if (out_trace_grid) *out_trace_grid = best_grid;
    return ST_OK;
}

int st_stream_copy(void* dst, const void* src, int64_t nbytes, hipStream_t s) {
    if (nbytes < 0 || (nbytes > 0 && (!dst || !src))) return fail(ST_ERR_INVALID_ARG, "bad copy arguments");
    if ((nbytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15))
        return fail(ST_ERR_INVALID_ARG, "st_stream_copy needs 16-byte aligned pointers and size");
    launch_stream_copy((float4*)dst, (const float4*)src, nbytes / 16, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_check_errors(st_scene* sc, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    uint32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, sc->d.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (e) {
        launch_fill_u32(sc->d.err, 1, 0u, s);
        HIPCHK(hipStreamSynchronize(s));
        const std::string what = "device error word " + std::to_string(e) +
                                 " (1: traversal stack overflow, 2: non-finite image or gradient value, "
                                 "4: queue reservation past its capacity, 8: traversal iteration cap)";
        if (e == ERR_QUEUE) return fail(ST_ERR_QUEUE_OVERFLOW, what);
        return fail(ST_ERR_DEVICE_FAULT, what);
    }
    return ST_OK;
}

int st_read_work(st_scene* sc, uint64_t* out3, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!out3) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    HIPCHK(hipMemcpyAsync(out3, sc->d.work, 3 * WORK_SLOTS * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    launch_fill_u32((uint32_t*)sc->d.work, 6 * WORK_SLOTS, 0u, s);
    HIPCHK(hipStreamSynchronize(s));
    return ST_OK;
}

int st_scene_info(const st_scene* sc, int64_t* out6) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!out6) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    out6[0] = sc->d.nv; out6[1] = sc->d.nf; out6[2] = sc->d.ne; out6[3] = sc->d.nl; out6[4] = sc->d.he; out6[5] = sc->d.we;
    return ST_OK;
}

int st_scene_edges(st_scene* sc, int32_t* out, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (!out) return fail(ST_ERR_INVALID_ARG, "out is NULL");
    if (sc->d.ne > 0) HIPCHK(hipMemcpyAsync(out, sc->d.edges, sizeof(int4) * sc->d.ne, hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

int st_scene_lbvh(st_scene* sc, uint64_t* keys, int32_t* child, int32_t* parent, float* aabb, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    const size_t n = sc->d.nf;
    if (keys) HIPCHK(hipMemcpyAsync(keys, sc->d.keys64, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    if (child && n > 1) HIPCHK(hipMemcpyAsync(child, sc->d.child, sizeof(int) * 2 * (n - 1), hipMemcpyDeviceToDevice, s));
    if (parent) {
        if (n == 1) launch_fill_u32((uint32_t*)parent, 1, 0xFFFFFFFFu, s);
        else HIPCHK(hipMemcpyAsync(parent, sc->d.parent, sizeof(int) * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    }
    if (aabb) HIPCHK(hipMemcpyAsync(aabb, sc->d.aabb, sizeof(float) * 6 * (2 * n - 1), hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

int st_trace_rays(st_scene* sc, const float* o, const float* d, int32_t n, float tmin, int32_t brute, int32_t* of,
                  float* ot, hipStream_t s) {
    int rc = check_scene(sc);
    if (rc) return rc;
    if (n < 0 || (long long)n > (long long)TRACE_GRID * TRACE_BLOCK) return fail(ST_ERR_INVALID_ARG, "n out of range");
    if (n > 0 && (!o || !d || !of || !ot)) return fail(ST_ERR_INVALID_ARG, "NULL array");
    rc = ensure_spill(sc);
    if (rc) return rc;
    launch_trace_debug(sc->d.dscene, o, d, n, tmin, brute, of, ot, (uint32_t*)sc->spillbuf.p, sc->d.err, s);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

void st_scene_destroy(st_scene* sc) {
    if (!sc) return;
    hipDeviceSynchronize();
    SceneDev& d = sc->d;
    void* ptrs[] = {d.V, d.F, d.mat, d.lights, d.env, d.fnorm, d.bmin, d.bmax, d.cen, d.bounds, d.mkeys[0], d.mkeys[1],
                    d.mvals[0], d.mvals[1], d.rs_hist, d.keys64, d.child, d.parent, d.aabb, d.refit_cnt, d.tcost, d.tleaves, d.ebmin, d.ebmax, d.ecen, d.ebounds, d.emkeys[0], d.emkeys[1],
                    d.emvals[0], d.emvals[1], d.ers_hist, d.ekeys64, d.echild, d.eparent, d.ecnt, d.eaabb, d.elen, d.enbox, d.enode, d.nodes4, d.flag4, d.id4, d.ccost, d.cdec,
                    d.tri, d.fleaf, d.edges, d.edge_w, d.eguide, d.mguide, d.cguide, d.ecdf, d.etotal_d, d.etotal_f, d.row_dom, d.rowcos, d.cond, d.marg,
                    d.env_rows, d.env_total, d.texpdf, d.err, d.work, d.dscene, d.vf_off, d.vf_idx, d.facc, d.macc, d.fe,
                    d.ealias, d.rec_key};
    for (void* p : ptrs)
        if (p) hipFree(p);
    sc->Lbuf.release(); sc->qbuf.release(); sc->spillbuf.release(); sc->primbuf.release(); sc->recbuf.release();
    sc->sidebuf.release(); sc->sidehash.release(); sc->secbuf.release(); sc->spill_aux.release();
    sc->adjbuf.release();
    sc->vrecbuf.release();
    if (sc->ev_fork) hipEventDestroy(sc->ev_fork);
    if (sc->ev_join) hipEventDestroy(sc->ev_join);
    if (sc->aux) hipStreamDestroy(sc->aux);
    for (void* q : sc->retired) hipFree(q);
    for (auto& t : sc->tables) {
        if (t.dev) hipFree(t.dev);
        if (t.pinned) hipHostFree(t.pinned);
    }
    delete sc;
}

} // extern "C"

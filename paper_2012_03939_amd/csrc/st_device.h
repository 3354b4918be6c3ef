// Device-side building blocks of the gfx950 path tracer: vector math, Philox
// streams, decision hash, BVH traversal with LDS-staged stacks, the
// Torrance-Sparrow BRDF (evaluation, sampling, pdf and reverse-mode
// derivative), environment-map sampling, and the path estimator used by the
// adjoint replay and by the edge side paths.
//
// Method: Shape from Tracing, Sec. 3.2 (a differentiable physically based path
// tracer R(x, c_i) with gradients of pixels w.r.t. geometry) and Sec. 3.3
// (per-facet Torrance-Sparrow materials; global illumination).  The estimator is
// fixed by the library's stream and shading specification: point lights are
// all sampled at every vertex, one environment sample per vertex is combined
// with BRDF sampling by the balance heuristic, the BRDF is a Lambertian term
// plus a Beckmann / Smith microfacet lobe scaled by the specular colour.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

constexpr float PI_F = 3.14159265358979323846f;
constexpr float INV_PI_F = 0.318309886183790671538f;
constexpr float INV_SQRT_PI_F = 0.564189583547756286948f;
constexpr float TMIN = 1e-4f;
constexpr float SHADOW_SHRINK = 1e-4f;
constexpr float ALPHA_MIN = 1e-3f;
constexpr float LOBE_SPEC_P = 0.5f;
constexpr double EPS_PRIMARY = 1e-3;    // pixels
constexpr float EPS_SECONDARY = 1e-4f;  // radians
constexpr double ZNEAR = 1e-3;
constexpr float SEC_COS_MIN = 1e-5f;    // secondary edge points this close to the tangent plane are skipped
constexpr float BOX_GROW = 1.0000004f;  // 1 + 2*gamma(3): conservative slab exit distance
#ifndef ST_LDS_STACK
#define ST_LDS_STACK 16
#endif
constexpr int LDS_STACK = ST_LDS_STACK; // per-lane traversal stack entries held in LDS
constexpr int SPILL_STACK = 64 - LDS_STACK;  // further entries spilled to HBM (64 in all)
constexpr int TRAV_BLOCK = 256;              // threads of every block that traverses (LDS stack stride)
constexpr uint32_t LEAF_BIT = 0x80000000u;
constexpr int MAX_LIGHTS = 16;
// slots of the traversal work counters (node visits, triangle tests, rays each):
// extension rays and shadow rays wherever traced, the adjoint, the single-kernel
// forward, and (counted a second time) the rays of the paired launch
constexpr int WORK_EXTEND = 0, WORK_SHADOW = 1, WORK_ADJOINT = 2, WORK_MEGA = 3, WORK_PAIR = 4, WORK_SLOTS = 5;

// error word bits (device -> host)
constexpr uint32_t ERR_STACK = 1u;
constexpr uint32_t ERR_NAN = 2u;
constexpr uint32_t ERR_QUEUE = 4u;
constexpr uint32_t ERR_LOOP = 8u;
constexpr int TRAVERSAL_CAP = 1 << 22;   // node visits per ray before the traversal gives up

// ---------------------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 mk(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return V3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return V3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ V3 mul(V3 a, V3 b) { return V3{a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float len(V3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / len(a)); }
__device__ __forceinline__ float hsum(V3 a) { return a.x + a.y + a.z; }
__device__ __forceinline__ V3 ld3(const float* p) { return V3{p[0], p[1], p[2]}; }
__device__ __forceinline__ V3 xyz(float4 a) { return V3{a.x, a.y, a.z}; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}
__device__ __forceinline__ float unif(uint32_t r) { return (float)(r >> 8) * (1.0f / 16777216.0f); }

struct Ctr { uint32_t c0, c1, c2hi, c3; };
struct Key { uint32_t k0, k1; };

__device__ __forceinline__ float4 draw4(const Ctr& c, uint32_t bounce, uint32_t block, const Key& k) {
    uint4 r = philox(c.c0, c.c1, c.c2hi | (bounce << 8) | block, c.c3, k.k0, k.k1);
    return make_float4(unif(r.x), unif(r.y), unif(r.z), unif(r.w));
}

// FNV-1a over the little-endian bytes of 32-bit decision words
struct Hash {
    uint32_t h;
    bool on;
    __device__ void push(uint32_t w) {
        if (!on) return;
#pragma unroll
        for (int b = 0; b < 4; ++b) { h ^= (w >> (8 * b)) & 0xFFu; h *= 0x01000193u; }
    }
};
constexpr uint32_t FNV_INIT = 0x811C9DC5u;

// ---------------------------------------------------------------------------
// scene as the kernels see it
// ---------------------------------------------------------------------------
// one bin of the environment alias table: texel k of bin k is kept when the
// second uniform is below prob, otherwise the bin's alias texel is taken
struct __align__(16) EnvAlias {
    double prob;
    int alias;
    int pad;
};

struct DevScene {
    const float* V;       // [nv,3]
    const int* F;         // [nf,3]
    const float* mat;     // [nf,7]
    const float* lights;  // [nl,6]
    const float4* fnorm;  // [nf] unit geometric normal
    const float4* tri;    // [nf*3] leaf-ordered (v0, face bits) (e1) (e2)
    const int* fleaf;     // [nf] leaf index of each face
    const float4* nodes4; // 4-wide nodes, 8 float4 each: SoA child boxes + child codes
    const float* env;     // [he,we,3]
    const double* marg;   // [he+1]
    const double* cond;   // [he,we+1]
    const float* texpdf;  // [he*we] solid-angle pdf of each texel
    const float* rowcos;  // [2*(he+1)]: 1 - cos(pi r / he), then 1 + cos(pi r / he)
    const int4* edges;    // [ne] (va, vb, f1, f2)
    const double* ecdf;   // [ne+1] cumulative 3-D length / total
    const float* etotal;  // total 3-D edge length
    const int* eguide;    // guide table of ecdf, 2^eglog entries
    const int* mguide;    // guide table of the env marginal CDF, 2^mglog entries
    const int* cguide;    // guide tables of the env conditional CDFs, 2^cglog entries per row
    const int* etchild;   // secondary-edge importance tree: children [ne-1, 2]
    const float* etbox;   // node boxes [2ne-1, 6] (internal nodes, then leaves)
    const float* etlen;   // node length sums [2ne-1]
    const float* etnbox;  // node boxes of the adjacent faces' unit normals [2ne-1, 6]
    const float4* etnode; // per internal node, both children's box, length, normal box and code
                          // in one 128-B record (8 float4, layout of k_epack) [ne-1]
    const uint32_t* etedge; // sorted leaf -> edge
    const EnvAlias* ealias; // [he*we] alias table of the texel probabilities, used when env_alias
    int env_alias;
    int vndf;             // specular lobe sampled from the visible normals
    int eglog, mglog, cglog;
    int nv, nf, nl, he, we, ne, has_env;
    int tex_res;          // mesh-colours resolution r: mat has nf (r+1)(r+2)/2 rows
    uint32_t scene_id;
};

// per-lane traversal stack: LDS_STACK entries in LDS (lane-interleaved), the
// rest in a per-thread HBM spill region
// address-space-qualified views: loads through them compile to global_load /
// ds_read instead of generic flat accesses
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const vf4 gfloat4;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(3))) uint32_t lu32;

struct TravStack {
    lu32* lds;         // this lane's LDS stack column: entry i at lds[i * TRAV_BLOCK]
    gu32* spill;       // spill base; entry i of thread g at spill[i*gstride + g]
    uint32_t gstride, gid;
    uint32_t* err;
    unsigned long long* work;   // optional: node visits, triangle tests, rays
    unsigned long long* work2;  // optional: a second set of the same counters
    __device__ __forceinline__ void put(int i, uint32_t v) {
        if (i < LDS_STACK) lds[i * TRAV_BLOCK] = v;
        else spill[(i - LDS_STACK) * gstride + gid] = v;
    }
    __device__ __forceinline__ uint32_t get(int i) const {
        if (i < LDS_STACK) return lds[i * TRAV_BLOCK];
        return spill[(i - LDS_STACK) * gstride + gid];
    }
    // pushes m (0..3) entries: a, then b, then c; entries beyond the m-th are
    // written too when they stay in LDS (above the new top, so never read)
    __device__ __forceinline__ bool push3(int& sp, int m, uint32_t a, uint32_t b, uint32_t c) {
        if (sp + 3 <= LDS_STACK) {
            lds[sp * TRAV_BLOCK] = a;
            lds[(sp + 1) * TRAV_BLOCK] = b;
            lds[(sp + 2) * TRAV_BLOCK] = c;
            sp += m;
            return true;
        }
        if (sp + m > LDS_STACK + SPILL_STACK) return false;
        if (m > 0) put(sp++, a);
        if (m > 1) put(sp++, b);
        if (m > 2) put(sp++, c);
        return true;
    }
};

__device__ __forceinline__ TravStack make_trav_stack(uint32_t* lds, uint32_t* spill, uint32_t* err,
                                                     unsigned long long* work) {
    TravStack s;
    // the stack layout assumes TRAV_BLOCK threads per block
    if (blockDim.x != TRAV_BLOCK && threadIdx.x == 0) atomicOr(err, ERR_STACK);
    s.lds = (lu32*)lds + threadIdx.x;
    s.spill = (gu32*)spill;
    s.gstride = gridDim.x * blockDim.x;
    s.gid = blockIdx.x * blockDim.x + threadIdx.x;
    s.err = err;
    s.work = work;
    s.work2 = nullptr;
    return s;
}

// the geometry one traversal reads, held in registers for the whole traversal
struct TraceGeo {
    const gfloat4* nodes4;
    const gfloat4* tri;
    int nf;
};
__device__ __forceinline__ TraceGeo trace_geo(const DevScene& S) {
    return TraceGeo{(const gfloat4*)S.nodes4, (const gfloat4*)S.tri, S.nf};
}

// Moller-Trumbore, two-sided, on the leaf-ordered triangle record
__device__ __forceinline__ bool tri_test(const gfloat4* tri, uint32_t leaf, V3 o, V3 d, float tmin, float tmax,
                                         float& t, int& face) {
    const vf4 a = tri[3 * leaf], b = tri[3 * leaf + 1], c = tri[3 * leaf + 2];
    const V3 e1 = V3{b.x, b.y, b.z}, e2 = V3{c.x, c.y, c.z};
    const V3 p = cross(d, e2);
    const float det = dot(e1, p);
    if (det == 0.0f) return false;
    const float inv = 1.0f / det;
    const V3 s = o - V3{a.x, a.y, a.z};
    const float b1 = dot(s, p) * inv;
    if (b1 < 0.0f || b1 > 1.0f) return false;
    const V3 q = cross(s, e1);
    const float b2 = dot(d, q) * inv;
    if (b2 < 0.0f || b1 + b2 > 1.0f) return false;
    t = dot(e2, q) * inv;
    face = __float_as_int(a.w);
    return t > tmin && t < tmax;
}

// distance along o + t d to the plane of face f, with the arithmetic of the
// triangle test (the hit distance of a recorded hit)
__device__ __forceinline__ float face_hit_t(const DevScene& S, int f, V3 o, V3 d) {
    const V3 a = ld3(S.V + 3 * (size_t)S.F[3 * f]);
    const V3 e1 = ld3(S.V + 3 * (size_t)S.F[3 * f + 1]) - a, e2 = ld3(S.V + 3 * (size_t)S.F[3 * f + 2]) - a;
    const V3 p = cross(d, e2);
    const float inv = 1.0f / dot(e1, p);
    const V3 q = cross(o - a, e1);
    return dot(e2, q) * inv;
}

__device__ __forceinline__ V3 safe_inv(V3 d) {
    auto f = [](float v) { return 1.0f / (fabsf(v) > 1e-30f ? v : copysignf(1e-30f, v)); };
    return V3{f(d.x), f(d.y), f(d.z)};
}

// slab test of the 4 child boxes of a 4-wide node; entry distance per slot,
// +inf for a miss or an empty slot
__device__ __forceinline__ void node4_test(const gfloat4* nodes4, uint32_t node, V3 o, V3 inv, float tmin, float tmax,
                                           float t[4], uint32_t c[4]) {
    const gfloat4* n = nodes4 + 8 * (size_t)node;
    const vf4 x0 = n[0], x1 = n[1], y0 = n[2], y1 = n[3], z0 = n[4], z1 = n[5], cc = n[6];
    const float lx[4] = {x0.x, x0.y, x0.z, x0.w}, hx[4] = {x1.x, x1.y, x1.z, x1.w};
    const float ly[4] = {y0.x, y0.y, y0.z, y0.w}, hy[4] = {y1.x, y1.y, y1.z, y1.w};
    const float lz[4] = {z0.x, z0.y, z0.z, z0.w}, hz[4] = {z1.x, z1.y, z1.z, z1.w};
    c[0] = __float_as_uint(cc.x); c[1] = __float_as_uint(cc.y); c[2] = __float_as_uint(cc.z); c[3] = __float_as_uint(cc.w);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float ax = (lx[s] - o.x) * inv.x, bx = (hx[s] - o.x) * inv.x;
        const float ay = (ly[s] - o.y) * inv.y, by = (hy[s] - o.y) * inv.y;
        const float az = (lz[s] - o.z) * inv.z, bz = (hz[s] - o.z) * inv.z;
        const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tmin));
        const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tmax)) * BOX_GROW;
        t[s] = t0 <= t1 ? t0 : __int_as_float(0x7f800000);
    }
}

// leaf children of a visited node in slot order, kept in four registers: no
// lane-varying index into a register array (which the compiler would move to
// LDS), and one triangle-test site for all of them
struct LeafList {
    uint32_t l0 = 0, l1 = 0, l2 = 0, l3 = 0;
    int n = 0;
    __device__ __forceinline__ void add(uint32_t v) {
        l0 = n == 0 ? v : l0;
        l1 = n == 1 ? v : l1;
        l2 = n == 2 ? v : l2;
        l3 = n == 3 ? v : l3;
        ++n;
    }
    __device__ __forceinline__ uint32_t pop() {
        const uint32_t v = l0;
        l0 = l1; l1 = l2; l2 = l3;
        --n;
        return v;
    }
};

// moves the hit leaf children out of (t, c): their distance becomes +inf
__device__ __forceinline__ LeafList take_leaves(float t[4], const uint32_t c[4]) {
    LeafList L;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (t[s] < __int_as_float(0x7f800000) && (c[s] & LEAF_BIT)) {
            L.add(c[s] & ~LEAF_BIT);
            t[s] = __int_as_float(0x7f800000);
        }
    return L;
}

__device__ __forceinline__ void cswap(float& ta, uint32_t& ca, float& tb, uint32_t& cb) {
    if (tb < ta) {
        const float t = ta; ta = tb; tb = t;
        const uint32_t c = ca; ca = cb; cb = c;
    }
}

// closest hit with t in (tmin, inf) excluding one face; ties go to the smaller face id.
// (t0, f0): a hit already known (f0 >= 0, from the same triangle test), which
// only prunes the traversal: the result is the least (t, face) either way
__device__ int trace_closest(const DevScene& S, V3 o, V3 d, float tmin, int exclude, float& thit, TravStack& st,
                             float t0 = __int_as_float(0x7f800000), int f0 = -1) {
    const float INF = __int_as_float(0x7f800000);
    float tbest = t0;
    int best = f0;
    const TraceGeo G = trace_geo(S);
    if (G.nf <= 0) return -1;
    uint32_t tests = 0;
    auto leaf = [&](uint32_t l) {
        ++tests;
        float t; int f;
        if (tri_test(G.tri, l, o, d, tmin, INF, t, f) && f != exclude) {
            if (t < tbest || (t == tbest && f < best)) { tbest = t; best = f; }
        }
    };
    if (G.nf == 1) { leaf(0); thit = tbest; return best; }
    const V3 inv = safe_inv(d);
    uint32_t node = 0;
    int sp = 0;
    int iter = 0;
    for (;; ++iter) {
        if (iter >= TRAVERSAL_CAP) { atomicOr(st.err, ERR_LOOP); break; }
        float t[4];
        uint32_t c[4];
        node4_test(G.nodes4, node, o, inv, tmin, tbest, t, c);
        // hit leaf slots, tested in slot order at one site (a wave runs the
        // largest per-lane count of leaf tests, not one block per slot)
        LeafList lv = take_leaves(t, c);
        while (lv.n > 0) leaf(lv.pop());
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (t[s] > tbest) t[s] = INF;
        // nearest first: sort the 4 (distance, code) pairs
        cswap(t[0], c[0], t[1], c[1]); cswap(t[2], c[2], t[3], c[3]);
        cswap(t[0], c[0], t[2], c[2]); cswap(t[1], c[1], t[3], c[3]);
        cswap(t[1], c[1], t[2], c[2]);
        if (t[0] < INF) {
            // the hit slots come first: push slots m-1 .. 1 (farthest first)
            const bool h1 = t[1] < INF, h2 = t[2] < INF, h3 = t[3] < INF;
            const int m = (int)h1 + (int)h2 + (int)h3;
            const uint32_t a = h3 ? c[3] : (h2 ? c[2] : c[1]);
            const uint32_t b = h3 ? c[2] : c[1];
            if (!st.push3(sp, m, a, b, c[1])) { atomicOr(st.err, ERR_STACK); break; }
            node = c[0];
        } else {
            if (sp == 0) break;
            node = st.get(--sp);
        }
    }
    // node visits: one per iteration (the cap exit visits none)
    const uint32_t visits = (uint32_t)min(iter + 1, TRAVERSAL_CAP);
    for (unsigned long long* w : {st.work, st.work2})
        if (w) {
            atomicAdd(w, (unsigned long long)visits);
            atomicAdd(w + 1, (unsigned long long)tests);
            atomicAdd(w + 2, 1ull);
        }
    thit = tbest;
    return best;
}

__device__ bool trace_any_impl(const DevScene& S, V3 o, V3 d, float tmin, float tmax, int exclude, TravStack& st,
                               uint32_t& visits, uint32_t& tests) {
    const float INF = __int_as_float(0x7f800000);
    const TraceGeo G = trace_geo(S);
    if (G.nf <= 0) return false;
    auto leaf = [&](uint32_t l) -> bool {
        ++tests;
        float t; int f;
        return tri_test(G.tri, l, o, d, tmin, tmax, t, f) && f != exclude;
    };
    if (G.nf == 1) return leaf(0);
    const V3 inv = safe_inv(d);
    uint32_t node = 0;
    int sp = 0;
    for (int iter = 0;; ++iter) {
        if (iter >= TRAVERSAL_CAP) { atomicOr(st.err, ERR_LOOP); return false; }
        ++visits;
        float t[4];
        uint32_t c[4];
        node4_test(G.nodes4, node, o, inv, tmin, tmax, t, c);
        LeafList lv = take_leaves(t, c);
        while (lv.n > 0)
            if (leaf(lv.pop())) return true;
        // the first hit slot is visited next, the others are pushed in slot order
        bool have = false;
        uint32_t next = 0, q0 = 0, q1 = 0, q2 = 0;
        int m = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (t[s] < INF) {
                if (!have) { next = c[s]; have = true; }
                else {
                    q0 = m == 0 ? c[s] : q0;
                    q1 = m == 1 ? c[s] : q1;
                    q2 = m == 2 ? c[s] : q2;
                    ++m;
                }
            }
        }
        if (!st.push3(sp, m, q0, q1, q2)) { atomicOr(st.err, ERR_STACK); return false; }
        if (have) {
            node = next;
        } else {
            if (sp == 0) return false;
            node = st.get(--sp);
        }
    }
}

__device__ __forceinline__ bool trace_any(const DevScene& S, V3 o, V3 d, float tmin, float tmax, int exclude,
                                          TravStack& st) {
    uint32_t visits = 0, tests = 0;
    const bool r = trace_any_impl(S, o, d, tmin, tmax, exclude, st, visits, tests);
    for (unsigned long long* w : {st.work, st.work2})
        if (w) {
            atomicAdd(w, (unsigned long long)visits);
            atomicAdd(w + 1, (unsigned long long)tests);
            atomicAdd(w + 2, 1ull);
        }
    return r;
}

// ---------------------------------------------------------------------------
// Torrance-Sparrow BRDF: kd/pi + ks * D * G / (4 cos_i cos_o), Beckmann D,
// height-correlated Smith G of the Beckmann surface.
// ---------------------------------------------------------------------------
struct Mat { V3 kd, ks; float a; };
__device__ __forceinline__ Mat load_mat(const float* m) {
    Mat r;
    r.kd = V3{m[0], m[1], m[2]};
    r.ks = V3{m[3], m[4], m[5]};
    r.a = m[6];
    return r;
}
__device__ __forceinline__ float alpha_eff(float a) { return a > ALPHA_MIN ? a : ALPHA_MIN; }

// Material row of the point x on face f.  Mesh colours (Sec. 3.3
// "Representation"): at resolution r the point with barycentric coordinates
// (alpha of the second vertex, beta of the third) uses texel
// f (r+1)(r+2)/2 + i (2r - i + 3)/2 + j, (i, j) = floor(r (alpha, beta)),
// clamped to 0 <= i <= r, 0 <= j <= r - i; r = 0 is one row per face.
__device__ __forceinline__ int texel_of(const DevScene& S, int f, V3 x) {
    const int r = S.tex_res;
    if (r == 0) return f;
    const V3 v0 = ld3(S.V + 3 * S.F[3 * f]), v1 = ld3(S.V + 3 * S.F[3 * f + 1]), v2 = ld3(S.V + 3 * S.F[3 * f + 2]);
    const V3 e1 = v1 - v0, e2 = v2 - v0, q = x - v0;
    const V3 N = cross(e1, e2);
    const float nn = dot(N, N);
    float a = dot(cross(q, e2), N) / nn, b = dot(cross(e1, q), N) / nn;
    a = fminf(fmaxf(a, -1.0f), 2.0f);   // also maps NaN to -1
    b = fminf(fmaxf(b, -1.0f), 2.0f);
    int i = (int)floorf((float)r * a), j = (int)floorf((float)r * b);
    i = min(max(i, 0), r);
    j = min(max(j, 0), r - i);
    return (f * (r + 1) * (r + 2) + i * (2 * r - i + 3)) / 2 + j;
}

// Beckmann D with tan^2 taken from |n x h|^2 / (n.h)^2: 1 - (n.h)^2 cancels in
// float32 near the highlight, the cross product does not
__device__ __forceinline__ float beckmann_D(V3 n, V3 h, float ch, float a) {
    const float c2 = ch * ch;
    const V3 nh = cross(n, h);
    const float t2 = dot(nh, nh) / c2;
    return expf(-t2 / (a * a)) / (PI_F * a * a * c2 * c2);
}

__device__ __forceinline__ float smith_lambda(float c, float a) {
    if (c >= 1.0f) return 0.0f;
    const float s = sqrtf(1.0f - c * c);
    const float x = c / (a * s);
    return (expf(-x * x) * INV_SQRT_PI_F / x - erfcf(x)) * 0.5f;
}

__device__ __forceinline__ V3 brdf_eval(V3 wi, V3 wo, V3 n, const Mat& m) {
    const float ci = dot(n, wi), co = dot(n, wo);
    if (!(ci > 0.0f) || !(co > 0.0f)) return V3{0.f, 0.f, 0.f};
    const float a = alpha_eff(m.a);
    const V3 h = normalize(wi + wo);
    const float ch = dot(n, h);
    float spec = 0.0f;
    if (ch > 0.0f) {
        const float D = beckmann_D(n, h, ch, a);
        const float G = 1.0f / (1.0f + smith_lambda(ci, a) + smith_lambda(co, a));
        spec = D * G / (4.0f * ci * co);
    }
    return m.kd * INV_PI_F + m.ks * spec;
}

// pdf of the one-sample mixture: 1/2 cosine-weighted + 1/2 specular, whose
// half-vectors follow D(h) cos(theta_h), or with vndf the normals visible from
// wo, G1(wo) max(0, wo.h) D(h) / cos(theta_o) (Heitz and d'Eon 2014); either
// becomes a pdf of wi through 1 / (4 |wo.h|)
__device__ __forceinline__ float bsdf_pdf(V3 wi, V3 wo, V3 n, float alpha, bool vndf) {
    const float ci = dot(n, wi);
    if (!(ci > 0.0f)) return 0.0f;
    const float a = alpha_eff(alpha);
    const float pd = (1.0f - LOBE_SPEC_P) * ci * INV_PI_F;
    const V3 hv = wi + wo;
    const float hl = len(hv);
    float ps = 0.0f;
    if (hl > 0.0f) {
        const V3 h = hv * (1.0f / hl);
        const float ch = dot(n, h);
        if (!vndf) {
            const float oh = fabsf(dot(wo, h));
            if (ch > 0.0f && oh > 0.0f) ps = LOBE_SPEC_P * beckmann_D(n, h, ch, a) * ch / (4.0f * oh);
        } else {
            const float oh = dot(wo, h), co = dot(n, wo);
            if (ch > 0.0f && oh > 0.0f && co > 0.0f) {
                const float g1 = 1.0f / (1.0f + smith_lambda(co, a));
                ps = LOBE_SPEC_P * g1 * beckmann_D(n, h, ch, a) / (4.0f * co);
            }
        }
    }
    return pd + ps;
}

// Visible-normal sample of the Beckmann lobe in the local frame (z = normal):
// stretch wo by alpha; for the standard surface seen at cot(theta') = c the
// slope along the incident plane has density ~ (c - x) exp(-x^2) on x < c with
// integral F(x) = c sqrt(pi)/2 erfc(-x) + exp(-x^2)/2, inverted by bracketed
// Newton steps (from below on the lower half of u1, through F(c) - F(x) on the
// upper half); the other slope is erfinv(2 u2 - 1); rotate, unstretch.
constexpr float VNDF_COT_MAX = 1e4f;
constexpr float VNDF_Y_MAX = 1.0f - 1.0f / 8388608.0f;
constexpr float HALF_SQRT_PI_F = 0.886226925452758013649f;
__device__ __forceinline__ V3 vndf_normal(V3 wl, float a, float u1, float u2) {
    const V3 ws = normalize(V3{a * wl.x, a * wl.y, wl.z});
    const float st = sqrtf(ws.x * ws.x + ws.y * ws.y);
    const float cphi = st > 0.0f ? ws.x / st : 1.0f, sphi = st > 0.0f ? ws.y / st : 0.0f;
    const float c = st > 0.0f ? fminf(ws.z / st, VNDF_COT_MAX) : VNDF_COT_MAX;
    const bool upper = u1 > 0.5f;
    const float Fc = c * HALF_SQRT_PI_F * erfcf(-c) + 0.5f * expf(-c * c);
    const float target = (upper ? 1.0f - u1 : u1) * Fc;
    float lo = -8.0f, hi = fminf(c, 8.0f), x = fminf(0.0f, 0.5f * c);   // the root lies below 8
    for (int it = 0; it < 24; ++it) {
        const float ex = expf(-x * x);
        const float g = upper ? target - (c * HALF_SQRT_PI_F * (erfcf(x) - erfcf(c)) + 0.5f * (expf(-c * c) - ex))
                              : (c * HALF_SQRT_PI_F * erfcf(-x) + 0.5f * ex) - target;
        if (g > 0.0f) hi = x; else lo = x;
        const float dg = (c - x) * ex;
        float xn = dg > 0.0f ? x - g / dg : 0.5f * (lo + hi);
        if (!(xn >= lo && xn <= hi)) xn = 0.5f * (lo + hi);    // a converged step stays put
        x = xn;
    }
    const float y = erfinvf(fmaxf(-VNDF_Y_MAX, fminf(VNDF_Y_MAX, 2.0f * u2 - 1.0f)));
    const float sx = (cphi * x - sphi * y) * a, sy = (sphi * x + cphi * y) * a;
    return normalize(V3{-sx, -sy, 1.0f});
}

// orthonormal basis around n (Duff et al. 2017, branchless)
__device__ __forceinline__ void onb(V3 n, V3& t, V3& b) {
    const float sg = copysignf(1.0f, n.z);
    const float a = -1.0f / (sg + n.z);
    const float bb = n.x * n.y * a;
    t = V3{1.0f + sg * n.x * n.x * a, sg * bb, -sg * n.x};
    b = V3{bb, sg + n.y * n.y * a, -n.y};
}

__device__ __forceinline__ int bsdf_sample(float4 u, V3 wo, V3 n, float alpha, bool vndf, V3& wi) {
    V3 t, b;
    onb(n, t, b);
    const float a = alpha_eff(alpha);
    if (u.x < LOBE_SPEC_P && vndf) {
        const V3 hl = vndf_normal(V3{dot(wo, t), dot(wo, b), dot(wo, n)}, a, u.y, u.z);
        const V3 h = t * hl.x + b * hl.y + n * hl.z;
        wi = h * (2.0f * dot(wo, h)) - wo;
        return 0;
    }
    const float phi = 2.0f * PI_F * u.z;
    float sp, cp;
    sincosf(phi, &sp, &cp);
    if (u.x < LOBE_SPEC_P) {
        const float t2 = -a * a * logf(1.0f - u.y);
        const float ch = 1.0f / sqrtf(1.0f + t2);
        const float sh = sqrtf(t2 / (1.0f + t2));    // sin^2 = tan^2 / (1 + tan^2): no cancellation near the pole
        const V3 h = t * (sh * cp) + b * (sh * sp) + n * ch;
        wi = h * (2.0f * dot(wo, h)) - wo;
        return 0;
    }
    const float r = sqrtf(u.y);
    const float z = sqrtf(fmaxf(0.0f, 1.0f - u.y));
    wi = t * (r * cp) + b * (r * sp) + n * z;
    return 1;
}

// Secondary-edge importance hierarchy.  Node weight seen from the shading
// point p with normal nrm (contraction off, this operation order): zero when the
// node's box lies wholly behind the tangent plane of p (with a margin of 2^-16
// of the box's size plus distance, so that a box lying in the plane keeps its
// weight whatever the rounding of p), or (sil) when no edge in it can be a
// silhouette from p: the bound of N.(p - q) over q in the box and N in the
// node's box of face normals keeps one sign beyond the same margin; otherwise
// its length sum, times a cosine factor (reach + margin) / (L1 distance + half
// the box's edge sum + margin) in (0, 1], over (squared distance to the box
// centre + squared half diagonal).  The descent
// takes each child with probability proportional to its weight, by a fresh
// uniform per level (level l: component l % 4 of the draw of block 4 + l / 4 at
// vertex k); returns the edge and its probability pe, or -1 when all weights vanish.
__device__ __forceinline__ float edge_node_weight(const float* bx, float len, const float* nb, V3 p, V3 nrm,
                                                  bool sil) {
#pragma clang fp contract(off)
    const float dx = (bx[0] + bx[3]) * 0.5f - p.x, dy = (bx[1] + bx[4]) * 0.5f - p.y, dz = (bx[2] + bx[5]) * 0.5f - p.z;
    const float ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
    const float reach = (dx * nrm.x + dy * nrm.y + dz * nrm.z) +
                        0.5f * ((fabsf(nrm.x) * ex + fabsf(nrm.y) * ey) + fabsf(nrm.z) * ez);
    const float tol = 0x1p-16f * (((fabsf(dx) + fabsf(dy)) + fabsf(dz)) + ((ex + ey) + ez));
    if (!(reach > -tol)) return 0.0f;
    if (sil) {
        const float a0 = -nb[0] * dx, b0 = -nb[3] * dx, a1 = -nb[1] * dy, b1 = -nb[4] * dy;
        const float a2 = -nb[2] * dz, b2 = -nb[5] * dz;
        const float lo = ((0.0f + fminf(a0, b0)) + fminf(a1, b1)) + fminf(a2, b2);
        const float hi = ((0.0f + fmaxf(a0, b0)) + fmaxf(a1, b1)) + fmaxf(a2, b2);
        const float rad = ((0.0f + fmaxf(fabsf(nb[0]), fabsf(nb[3])) * (0.5f * ex)) +
                           fmaxf(fabsf(nb[1]), fabsf(nb[4])) * (0.5f * ey)) +
                          fmaxf(fabsf(nb[2]), fabsf(nb[5])) * (0.5f * ez);
        if (lo - rad > tol || hi + rad < -tol) return 0.0f;
    }
    const float dl1 = ((fabsf(dx) + fabsf(dy)) + fabsf(dz)) + 0.5f * ((ex + ey) + ez);
    const float cb = (reach + tol) / (dl1 + tol);
    return len * cb / ((dx * dx + dy * dy + dz * dz) + 0.25f * ((ex * ex + ey * ey) + ez * ez));
}

// child j (0, 1) of a packed record: box (6), length, normal box (6), code
__device__ __forceinline__ float edge_child_weight(const float4* rec, int j, V3 p, V3 nrm, bool sil, int& code) {
    const float4 a = rec[4 * j], b = rec[4 * j + 1], c = rec[4 * j + 2], d = rec[4 * j + 3];
    const float bx[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
    const float nb[6] = {b.w, c.x, c.y, c.z, c.w, d.x};
    code = __float_as_int(d.y);
    return edge_node_weight(bx, b.z, nb, p, nrm, sil);
}

__device__ __forceinline__ int edge_tree_sample(const DevScene& S, V3 p, V3 nrm, const Ctr& ctr, int k,
                                                const Key& key, bool sil, float& pe) {
#pragma clang fp contract(off)
    pe = 1.0f;
    if (S.ne <= 0) return -1;
    int code = S.ne == 1 ? (int)LEAF_BIT : 0;
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int level = 0; !(code & (int)LEAF_BIT); ++level) {
        if (level >= 128) return -1;
        if ((level & 3) == 0) u = draw4(ctr, k, 4 + (level >> 2), key);
        const float4* rec = S.etnode + 8 * (size_t)code;
        int c0, c1;
        const float w0 = edge_child_weight(rec, 0, p, nrm, sil, c0), w1 = edge_child_weight(rec, 1, p, nrm, sil, c1);
        const float tot = w0 + w1;
        if (!(tot > 0.0f)) return -1;
        const float p0 = w0 / tot;
        const float ul = (level & 3) == 0 ? u.x : (level & 3) == 1 ? u.y : (level & 3) == 2 ? u.z : u.w;
        if (ul < p0) { code = c0; pe *= p0; }
        else { code = c1; pe *= w1 / tot; }
    }
    if (S.ne == 1 && !(edge_node_weight(S.etbox, S.etlen[0], S.etnbox, p, nrm, sil) > 0.0f)) return -1;
    return (int)S.etedge[code & 0x7FFFFFFF];
}

// Reverse-mode derivative of f(wi, wo, n, m) contracted with gf (rgb):
// accumulates into gn, gwi (only needed when wi depends on the geometry) and gm[7].
__device__ __forceinline__ float dlambda_dc(float c, float a, float& dla) {
    // Lambda(x), x = c / (a sqrt(1-c^2)); dLambda/dx = -exp(-x^2) / (2 sqrt(pi) x^2)
    dla = 0.0f;
    if (c >= 1.0f) return 0.0f;
    const float s = sqrtf(1.0f - c * c);
    const float x = c / (a * s);
    if (x > 12.0f) return 0.0f;
    const float dldx = -expf(-x * x) * (0.5f * INV_SQRT_PI_F) / (x * x);
    dla = dldx * (-x / a);
    return dldx / (a * s * s * s);
}

__device__ __forceinline__ void brdf_backward(V3 wi, V3 wo, V3 n, const Mat& m, V3 gf, V3& gn, V3& gwi,
                                              float* gm) {
    const float ci = dot(n, wi), co = dot(n, wo);
    if (!(ci > 0.0f) || !(co > 0.0f)) return;
    gm[0] += gf.x * INV_PI_F; gm[1] += gf.y * INV_PI_F; gm[2] += gf.z * INV_PI_F;
    const float a = alpha_eff(m.a);
    const V3 hv = wi + wo;
    const float hl = len(hv);
    const V3 h = hv * (1.0f / hl);
    const float ch = dot(n, h);
    if (!(ch > 0.0f)) return;
    const float D = beckmann_D(n, h, ch, a);
    const float li = smith_lambda(ci, a), lo = smith_lambda(co, a);
    const float G = 1.0f / (1.0f + li + lo);
    const float K = D * G / (4.0f * ci * co);
    gm[3] += gf.x * K; gm[4] += gf.y * K; gm[5] += gf.z * K;
    const float glnK = dot(gf, m.ks) * K;       // gradient w.r.t. ln K
    const float c2 = ch * ch;
    const float dlnD_dch = 2.0f / (c2 * ch * a * a) - 4.0f / ch;
    const V3 nh = cross(n, h);
    const float dlnD_da = 2.0f * dot(nh, nh) / (c2 * a * a * a) - 2.0f / a;
    float dlia, dloa;
    const float dli = dlambda_dc(ci, a, dlia), dlo = dlambda_dc(co, a, dloa);
    if (m.a > ALPHA_MIN) gm[6] += glnK * (dlnD_da - G * (dlia + dloa));
    const float gci = glnK * (-G * dli - 1.0f / ci);
    const float gco = glnK * (-G * dlo - 1.0f / co);
    const float gch = glnK * dlnD_dch;
    gn = gn + wi * gci + wo * gco + h * gch;
    // through h = normalize(wi + wo) (wo is fixed)
    const V3 gh = n * gch;
    const V3 ghv = (gh - h * dot(h, gh)) * (1.0f / hl);
    gwi = gwi + n * gci + ghv;
}

// ---------------------------------------------------------------------------
// environment map: equirectangular, +y up, row 0 at theta = 0
// ---------------------------------------------------------------------------
// guide table of a CDF (cut-point method): guide[g] = largest i in [0, n-1] with
// C[i] <= g / G, G = 2^glog.  With g = floor(u G) the answer of cdf_find lies in
// [guide[g], guide[g + 1]], so a search of that (usually one- or two-entry)
// range returns exactly the index of the plain search.
__device__ __forceinline__ int cdf_guided(const double* C, int n, const int* guide, int glog, double u) {
    const int G = 1 << glog;
    int g = (int)(u * (double)G);
    g = g < G - 1 ? g : G - 1;
    int lo = guide[g];
    int hi = g + 1 < G ? guide[g + 1] : n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int cdf_find(const double* C, int n, double u) {
    // largest i in [0, n-1] with C[i] <= u (C[0] == 0 <= u)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int env_texel_of(const DevScene& S, V3 d) {
    const float y = fminf(1.0f, fmaxf(-1.0f, d.y));
    const float th = acosf(y);
    float ph = atan2f(d.x, d.z);
    if (ph < 0.0f) ph += 2.0f * PI_F;
    const int r = min((int)(th * (1.0f / PI_F) * S.he), S.he - 1);
    const int c = min((int)(ph * (0.5f / PI_F) * S.we), S.we - 1);
    return r * S.we + c;
}
__device__ __forceinline__ V3 env_rgb(const DevScene& S, int t) { return ld3(S.env + 3 * (size_t)t); }

__device__ __forceinline__ int env_sample(const DevScene& S, float4 u, V3& dir, float& pdf) {
    int r, c;
    if (S.env_alias) {
        // bin from the first uniform, the bin's texel or its alias from the second
        const int n = S.he * S.we;
        const int k = min((int)((double)u.x * (double)n), n - 1);
        const EnvAlias e = S.ealias[k];
        const int t = (double)u.y < e.prob ? k : e.alias;
        r = t / S.we;
        c = t - r * S.we;
    } else {
        r = cdf_guided(S.marg, S.he, S.mguide, S.mglog, (double)u.x);
        c = cdf_guided(S.cond + (size_t)r * (S.we + 1), S.we, S.cguide + ((size_t)r << S.cglog), S.cglog,
                       (double)u.y);
    }
    const float phi = 2.0f * PI_F * ((float)c + u.z) / (float)S.we;
    // cos(theta) uniform between the row's bounds; 1 -+ cos(theta) are taken
    // from the per-row tables of 1 - cos and 1 + cos so that sin(theta) keeps
    // full precision near both poles
    const float om0 = S.rowcos[r], om1 = S.rowcos[r + 1];                        // 1 - cos
    const float op0 = S.rowcos[S.he + 1 + r], op1 = S.rowcos[S.he + 2 + r];      // 1 + cos
    float a, b, cth;
    if (op0 + op1 >= om0 + om1) {       // upper half of the sphere: 1 - cos is the small one
        a = om0 + u.w * (om1 - om0);
        b = 2.0f - a;
        cth = 1.0f - a;
    } else {
        b = op0 - u.w * (op0 - op1);
        a = 2.0f - b;
        cth = b - 1.0f;
    }
    const float sth = sqrtf(fmaxf(0.0f, a * b));
    float sp, cp;
    sincosf(phi, &sp, &cp);
    dir = V3{sth * sp, cth, sth * cp};
    const int t = r * S.we + c;
    pdf = S.texpdf[t];
    return t;
}

// ---------------------------------------------------------------------------
// camera (precomputed basis; r and u already scaled by tan(fov/2) and aspect)
// ---------------------------------------------------------------------------
struct DevCam {
    float eye[3], f[3], rs[3], us[3];
    double deye[3], df[3], dr[3], du[3], dth, daspect;
    int W, H, scene;
    int rngview;         // view field of the random-stream counters: index among this scene's cameras
    long long qoff;      // processing-order path offset
    long long pixoff;    // canonical pixel offset
    long long eoff;      // primary edge sample offset
    long long ne;        // primary edge samples of this view
};

__device__ __forceinline__ V3 cam_dir(const DevCam& c, float sx, float sy) {
    const float nx = 2.0f * sx / (float)c.W - 1.0f, ny = 1.0f - 2.0f * sy / (float)c.H;
    const V3 d = ld3(c.f) + ld3(c.rs) * nx + ld3(c.us) * ny;
    return normalize(d);
}

// ---------------------------------------------------------------------------
// the path estimator (forward radiance only): used for the edge side paths and
// the single-kernel forward.  first_escape_full: a first-segment miss returns
// the environment radiance (secondary side rays) instead of black (camera).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void push_face(Hash& h, int f) { h.push(f < 0 ? 0xFFFFFFFFu : (uint32_t)f); }

__device__ V3 trace_estimator(const DevScene& S, V3 o, V3 d, int exclude, int nvert, bool first_escape_full,
                              const Ctr& ctr, const Key& key, Hash& hash, TravStack& st) {
    V3 L{0.f, 0.f, 0.f}, beta{1.f, 1.f, 1.f};
    float p_prev = 0.0f;
    for (int k = 1; k <= nvert + 1; ++k) {
        float t;
        const int f = trace_closest(S, o, d, TMIN, exclude, t, st);
        push_face(hash, f);
        if (f < 0) {
            if (S.has_env && (k > 1 || first_escape_full)) {
                const int tex = env_texel_of(S, d);
                hash.push((uint32_t)tex);
                const V3 Le = env_rgb(S, tex);
                float w = 1.0f;
                if (k > 1) { const float pe = S.texpdf[tex]; w = p_prev / (p_prev + pe); }
                L = L + mul(beta, Le) * w;
            }
            break;
        }
        if (k == nvert + 1) break;
        const V3 x = o + d * t;
        V3 n = xyz(S.fnorm[f]);
        const V3 wo = -d;
        if (dot(n, wo) < 0.0f) n = -n;
        const int tx = texel_of(S, f, x);
        if (S.tex_res) hash.push((uint32_t)tx);
        const Mat m = load_mat(S.mat + 7 * (size_t)tx);
        for (int l = 0; l < S.nl; ++l) {
            const float* lt = S.lights + 6 * l;
            const V3 dl = ld3(lt) - x;
            const float r2 = dot(dl, dl);
            uint32_t code = 0;
            if (r2 > 0.0f) {
                const float r = sqrtf(r2);
                const V3 wl = dl * (1.0f / r);
                const float c = dot(n, wl);
                if (c > 0.0f) {
                    const bool occ = trace_any(S, x, wl, TMIN, r * (1.0f - SHADOW_SHRINK), f, st);
                    code = occ ? 1u : 2u;
                    if (!occ) L = L + mul(beta, mul(ld3(lt + 3), brdf_eval(wl, wo, n, m))) * (c / r2);
                }
            }
            hash.push(code);
        }
        if (S.has_env) {
            const float4 u = draw4(ctr, k, 1, key);
            V3 we; float pe;
            const int tex = env_sample(S, u, we, pe);
            hash.push((uint32_t)tex);
            const float c = dot(n, we);
            uint32_t code = 0;
            if (c > 0.0f && pe > 0.0f) {
                const bool occ = trace_any(S, x, we, TMIN, __int_as_float(0x7f800000), f, st);
                code = occ ? 1u : 2u;
                if (!occ) {
                    const V3 fv = brdf_eval(we, wo, n, m);
                    const float den = pe + bsdf_pdf(we, wo, n, m.a, S.vndf);
                    L = L + mul(beta, mul(env_rgb(S, tex), fv)) * (c / den);
                }
            }
            hash.push(code);
        }
        if (!(k < nvert || S.has_env)) break;
        const float4 u = draw4(ctr, k, 2, key);
        V3 wi;
        const int lobe = bsdf_sample(u, wo, n, m.a, S.vndf, wi);
        const float ci = dot(n, wi);
        const float pb = bsdf_pdf(wi, wo, n, m.a, S.vndf);
        hash.push((uint32_t)lobe);
        if (!(ci > 0.0f) || !(pb > 0.0f)) { hash.push(0u); break; }
        hash.push(1u);
        beta = mul(beta, brdf_eval(wi, wo, n, m)) * (ci / pb);
        p_prev = pb;
        o = x; d = wi; exclude = f;
    }
    return L;
}

__device__ __forceinline__ uint64_t lanemask_lt64() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// processing order of path samples inside one view: sample-major, then 8x8
// pixel tiles (when the view is a multiple of 8 in both axes), then row-major
__device__ __forceinline__ void decode_path(const DevCam& c, long long local, int spp, int& x, int& y, int& j) {
    const long long hw = (long long)c.W * c.H;
    j = (int)(local / hw);
    const int p = (int)(local - (long long)j * hw);
    if ((c.W & 7) == 0 && (c.H & 7) == 0) {
        const int tile = p >> 6, within = p & 63, tw = c.W >> 3;
        x = (tile % tw) * 8 + (within & 7);
        y = (tile / tw) * 8 + (within >> 3);
    } else {
        x = p % c.W;
        y = p / c.W;
    }
    (void)spp;
}

__device__ __forceinline__ int find_view(const long long* off, int ncam, long long q) {
    // largest v with off[v] <= q
    int lo = 0, hi = ncam - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// prefix sums in double inside one block of 1024 threads (contiguous chunks per
// thread, then a serial scan of the 1024 partial sums): out[0] = 0,
// out[i+1] = out[i] + w[i], then optionally normalised by the total.
// ---------------------------------------------------------------------------
__device__ inline void block_scan_normalise(const double* w, int n, double* out, double* total_out) {
    __shared__ double part[1024];
    __shared__ double total_s;
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = t * per, e = min(n, b + per);
    double s = 0.0;
    for (int i = b; i < e; ++i) s += w[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double acc = 0.0;
        for (int i = 0; i < 1024; ++i) { const double v = part[i]; part[i] = acc; acc += v; }
        total_s = acc;
        *total_out = acc;
    }
    __syncthreads();
    const double tot = total_s;
    double acc = part[t];
    if (t == 0) out[0] = 0.0;
    for (int i = b; i < e; ++i) {
        acc += w[i];
        out[i + 1] = tot > 0.0 ? acc / tot : 0.0;
    }
}


// ---------------------------------------------------------------------------
// queue reservation with one atomic per block.  Atomics on one address are
// serialised by the memory system (about 11 ns apiece on this part), so one
// reservation per wave caps a compaction kernel at roughly 90 M waves/s;
// reserving per block of BS threads divides that cost by BS / 64.  Every thread
// of the block calls it (it synchronises the block); lanes with emit get M
// consecutive slots, the others -1.  lds holds BS / 64 + 1 ints.
// ---------------------------------------------------------------------------
template <int BS, int M>
__device__ __forceinline__ int block_reserve(bool emit, int* counter, int* lds) {
    const uint64_t mask = __ballot(emit);
    const int w = (int)(threadIdx.x >> 6);
    if (__lane_id() == 0) lds[w] = M * __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int j = 0; j < BS / 64; ++j) {
            const int c = lds[j];
            lds[j] = acc;
            acc += c;
        }
        lds[BS / 64] = acc > 0 ? atomicAdd(counter, acc) : 0;
    }
    __syncthreads();
    const int o = lds[BS / 64] + lds[w] + M * __popcll(mask & lanemask_lt64());
    __syncthreads();
    return emit ? o : -1;
}

// m (0 <= m < 2^BITS) consecutive slots per thread from *counter, in thread
// order within the block, with one atomic per block; every thread of the block
// calls it (it synchronises the block).  lds holds BS / 64 + 1 ints.
template <int BS, int BITS>
__device__ __forceinline__ int block_reserve_n(int m, int* counter, int* lds) {
    constexpr int NW = BS / 64;
    const uint64_t lt = lanemask_lt64();
    int pre = 0, tot = 0;
    for (int b = 0; b < BITS; ++b) {
        const uint64_t bm = __ballot((m >> b) & 1);
        pre += __popcll(bm & lt) << b;
        tot += __popcll(bm) << b;
    }
    const int w = (int)(threadIdx.x >> 6);
    if (__lane_id() == 0) lds[w] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int j = 0; j < NW; ++j) {
            const int x = lds[j];
            lds[j] = acc;
            acc += x;
        }
        lds[NW] = acc > 0 ? atomicAdd(counter, acc) : 0;
    }
    __syncthreads();
    const int o = lds[NW] + lds[w] + pre;
    __syncthreads();
    return o;
}

// Two reservations in one pass: one slot per thread with emit from *ca, and m
// (0 <= m < 32) consecutive slots per thread from *cb.  Returns (slot or -1,
// first of the m slots).  lds holds 2 (BS / 64 + 1) ints.
template <int BS>
__device__ __forceinline__ int2 block_reserve2(bool emit, int m, int* ca, int* cb, int* lds) {
    constexpr int NW = BS / 64;
    const uint64_t lt = lanemask_lt64();
    const uint64_t mask = __ballot(emit);
    int pre = 0, tot = 0;
    for (int b = 0; b < 5; ++b) {
        const uint64_t bm = __ballot((m >> b) & 1);
        pre += __popcll(bm & lt) << b;
        tot += __popcll(bm) << b;
    }
    const int w = (int)(threadIdx.x >> 6);
    if (__lane_id() == 0) {
        lds[w] = __popcll(mask);
        lds[NW + 1 + w] = tot;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        // lane 0 scans and reserves for ca, lane 1 for cb: one atomic
        // instruction, so the two round trips overlap
        const int base = threadIdx.x == 0 ? 0 : NW + 1;
        int acc = 0;
        for (int j = 0; j < NW; ++j) {
            const int x = lds[base + j];
            lds[base + j] = acc;
            acc += x;
        }
        int* const ctr = threadIdx.x == 0 ? ca : cb;
        lds[base + NW] = acc > 0 ? atomicAdd(ctr, acc) : 0;
    }
    __syncthreads();
    const int oa = lds[NW] + lds[w] + __popcll(mask & lt);
    const int ob = lds[2 * NW + 1] + lds[NW + 1 + w] + pre;
    __syncthreads();
    return make_int2(emit ? oa : -1, ob);
}

// Block index remapped so that each XCD works on one contiguous range of the
// grid: the hardware hands block b to XCD b % 8, so XCD x receives blocks
// x, x + 8, ...; they become x's consecutive share [x G/8, (x+1) G/8) (the
// first G % 8 XCDs one block more), and neighbouring work shares one L2.
constexpr unsigned NUM_XCD = 8;
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned per = G / NUM_XCD, rem = G % NUM_XCD, x = b % NUM_XCD, j = b / NUM_XCD;
    return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}
#ifndef ST_XCD_MAP
#define ST_XCD_MAP 1
#endif
// the block index the adjoint's grid-stride loop starts from (the traversal
// kernels keep the hardware order: contiguous shares per XCD made them slower,
// 69.8 -> 84.3 ms for k_extend, presumably because cheap and costly stretches
// of the queue then land on different XCDs)
__device__ __forceinline__ unsigned grid_block() { return ST_XCD_MAP ? xcd_block() : blockIdx.x; }

// ---------------------------------------------------------------------------
// persistent traversal of a ray queue with dynamic fetch: a wave refills its
// idle lanes whenever at least FETCH_MIN of them are idle, so a lane whose ray
// finished early takes the next ray instead of waiting for the slowest lane of
// its wave.  Each ray's outcome is that of trace_any (ANY) or trace_closest.
// ---------------------------------------------------------------------------
#ifndef ST_FETCH_MIN
#define ST_FETCH_MIN 16
#endif
#ifndef ST_FETCH_CHUNK
#define ST_FETCH_CHUNK 128
#endif
#ifndef ST_FETCH_NC
#define ST_FETCH_NC 8
#endif
constexpr int FETCH_MIN = ST_FETCH_MIN;      // idle lanes that trigger a refill
constexpr int FETCH_CHUNK = ST_FETCH_CHUNK;  // rays a wave takes from a counter at a time
constexpr int FETCH_NC = ST_FETCH_NC;        // counters, each owning a contiguous segment of the queue
constexpr int FETCH_SLOT_INTS = FETCH_NC * 32;   // one 128-byte line per counter

struct RayJob {
    V3 o, d;
    float tmax;   // any-hit: the ray is tested on (TMIN, tmax); closest hit: +inf
    int excl;     // face excluded from the test (the ray's origin face), -1 for none
    TraceGeo G;
};

// fetch(i, job) loads ray i and returns true, or stores ray i's outcome itself
// and returns false when it needs no traversal.  finish(i, face, t) stores the
// outcome: for ANY face is 1 when occluded and 0 otherwise; for the closest
// hit face is -1 and t = +inf on a miss.
template <bool ANY, class Fetch, class Finish>
__device__ __forceinline__ void trace_queue(int* counters, int n, TravStack& st, Fetch fetch, Finish finish) {
    const float INF = __int_as_float(0x7f800000);
    // a finished ray's outcome is stored when its lane is refilled (or at the
    // end), so that no store is in flight while the traversal waits on loads
    bool live = false, pend = false, drained = n <= 0;
    int idx = 0, sp = 0, iters = 0, best = -1;
    float tbest = INF;
    uint32_t node = 0;
    RayJob J;
    V3 inv{0.f, 0.f, 0.f};
    uint32_t visits = 0, tests = 0, rays = 0;
    // wave-uniform pool [cur, end) of rays taken from the counters; counter c
    // hands out chunks of segment [c seg, (c + 1) seg), starting at this
    // block's own counter and moving on to the others once it is used up
    int cur = 0, end = 0, tried = 0;
    const int seg = (int)(((long long)n + FETCH_NC - 1) / FETCH_NC);
    const int home = (int)(blockIdx.x % FETCH_NC);
    for (;;) {
        const uint64_t idle = __ballot(!live);
        const int nidle = __popcll(idle);
        if ((cur < end || !drained) && (nidle >= FETCH_MIN || nidle == (int)__builtin_amdgcn_wavefrontsize())) {
            const int leader = __ffsll((long long)idle) - 1;
            while (cur >= end && !drained) {
                const int c = (home + tried) % FETCH_NC;
                int b = 0;
                if ((int)__lane_id() == leader) b = atomicAdd(counters + 32 * c, FETCH_CHUNK);
                b = __builtin_amdgcn_readlane(b, leader);   // wave-uniform from here on
                const int s0 = c * seg, s1 = (int)min((long long)s0 + seg, (long long)n);
                if (b < s1 - s0) {
                    cur = s0 + b;
                    end = (int)min((long long)cur + FETCH_CHUNK, (long long)s1);
                } else if (++tried >= FETCH_NC) {
                    drained = true;
                }
            }
            if (pend) {
                finish(idx, best, tbest);
                pend = false;
            }
            const int take = min(nidle, end - cur);
            if (!live && take > 0) {
                const int rank = __popcll(idle & lanemask_lt64());
                if (rank < take) {
                    idx = cur + rank;
                    if (fetch(idx, J)) {
                        if (J.G.nf <= 0) {
                            finish(idx, ANY ? 0 : -1, INF);
                        } else if (J.G.nf == 1) {
                            float t; int f;
                            const bool h = tri_test(J.G.tri, 0, J.o, J.d, TMIN, J.tmax, t, f) && f != J.excl;
                            if (ANY) finish(idx, h ? 1 : 0, INF);
                            else finish(idx, h ? f : -1, h ? t : INF);
                        } else {
                            live = true;
                            ++rays;
                            inv = safe_inv(J.d);
                            node = 0; sp = 0; iters = 0; best = ANY ? 0 : -1; tbest = INF;
                        }
                    }
                }
            }
            if (take > 0) cur += take;
        }
        if (nidle == (int)__builtin_amdgcn_wavefrontsize() && drained && cur >= end) break;
        if (!live) continue;
        bool done = false;
        if (iters >= TRAVERSAL_CAP) {
            atomicOr(st.err, ERR_LOOP);
            done = true;
        } else {
            ++iters;
            ++visits;
            float t[4];
            uint32_t c[4];
            node4_test(J.G.nodes4, node, J.o, inv, TMIN, ANY ? J.tmax : tbest, t, c);
            LeafList lv = take_leaves(t, c);
            while (lv.n > 0) {
                ++tests;
                float th; int fh;
                if (tri_test(J.G.tri, lv.pop(), J.o, J.d, TMIN, J.tmax, th, fh) && fh != J.excl) {
                    if (ANY) { best = 1; break; }
                    if (th < tbest || (th == tbest && fh < best)) { tbest = th; best = fh; }
                }
            }
            if (ANY && best) {
                done = true;
            } else {
                bool have = false, overflow = false;
                uint32_t next = 0;
                if (ANY) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (t[s] < INF) {
                            if (!have) { next = c[s]; have = true; }
                            else if (sp >= LDS_STACK + SPILL_STACK) overflow = true;
                            else st.put(sp++, c[s]);
                        }
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (t[s] > tbest) t[s] = INF;
                    // nearest first: continue with the nearest child, stack the others farthest-first
                    cswap(t[0], c[0], t[1], c[1]); cswap(t[2], c[2], t[3], c[3]);
                    cswap(t[0], c[0], t[2], c[2]); cswap(t[1], c[1], t[3], c[3]);
                    cswap(t[1], c[1], t[2], c[2]);
                    if (t[0] < INF) {
                        next = c[0];
                        have = true;
#pragma unroll
                        for (int s = 3; s >= 1; --s) {
                            if (t[s] < INF) {
                                if (sp >= LDS_STACK + SPILL_STACK) overflow = true;
                                else st.put(sp++, c[s]);
                            }
                        }
                    }
                }
                if (overflow) {
                    atomicOr(st.err, ERR_STACK);
                    done = true;
                } else if (have) {
                    node = next;
                } else if (sp == 0) {
                    done = true;
                } else {
                    node = st.get(--sp);
                }
            }
        }
        if (done) {
            live = false;
            pend = true;
        }
    }
    if (pend) finish(idx, best, tbest);
    if (st.work && rays) {
        atomicAdd(st.work, (unsigned long long)visits);
        atomicAdd(st.work + 1, (unsigned long long)tests);
        atomicAdd(st.work + 2, (unsigned long long)rays);
    }
}

} // namespace st

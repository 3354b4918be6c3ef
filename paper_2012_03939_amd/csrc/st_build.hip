// Scene build on the GPU: per-face normals and bounds, the LBVH (30-bit Morton
// codes, stable LSD radix sort, Karras 2012 radix-tree hierarchy, bottom-up
// min/max refit), the leaf-ordered triangle records, the 3-D edge-length CDF of
// the secondary edge term, and the environment-map CDFs.
//
// The paper (Sec. 3.2, "Representation") relies on fast ray-surface
// intersection as the bulk of the cost without naming a structure; the LBVH is
// this library's choice.  Its integer part is bit-exact by specification:
// float32 centroids (min+max)*0.5, scale = float(1024 / (hi - lo)) evaluated in
// double, q = clamp(floor((c - lo) * s), 0, 1023), 10 bits per axis with x
// highest, key = morton << 32 | face, ascending.
#include "st_internal.h"

namespace st {

// ---------------------------------------------------------------------------
__global__ void k_face_prep(const float* __restrict__ V, const int* __restrict__ F, int nf, float4* fnorm,
                            float4* bmin, float4* bmax, float4* cen) {
#pragma clang fp contract(off)
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const V3 a = ld3(V + 3 * F[3 * f]), b = ld3(V + 3 * F[3 * f + 1]), c = ld3(V + 3 * F[3 * f + 2]);
    const V3 N = cross(b - a, c - a);
    const float l = len(N);
    const V3 n = l > 0.0f ? N * (1.0f / l) : V3{0.f, 0.f, 0.f};
    fnorm[f] = make_float4(n.x, n.y, n.z, 0.5f * l);
    const V3 mn{fminf(a.x, fminf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)), fminf(a.z, fminf(b.z, c.z))};
    const V3 mx{fmaxf(a.x, fmaxf(b.x, c.x)), fmaxf(a.y, fmaxf(b.y, c.y)), fmaxf(a.z, fmaxf(b.z, c.z))};
    bmin[f] = make_float4(mn.x, mn.y, mn.z, 0.f);
    bmax[f] = make_float4(mx.x, mx.y, mx.z, 0.f);
    const float cx = mn.x + mx.x, cy = mn.y + mx.y, cz = mn.z + mx.z;
    cen[f] = make_float4(cx * 0.5f, cy * 0.5f, cz * 0.5f, 0.f);
}

// single block: centroid bounds and the per-axis Morton scale
__global__ void k_bounds(const float4* __restrict__ cen, int nf, float* out /* lo[3], hi[3], s[3] */) {
    __shared__ float smin[3][1024], smax[3][1024];
    const int t = threadIdx.x;
    float lo[3] = {__int_as_float(0x7f800000), __int_as_float(0x7f800000), __int_as_float(0x7f800000)};
    float hi[3] = {-__int_as_float(0x7f800000), -__int_as_float(0x7f800000), -__int_as_float(0x7f800000)};
    for (int i = t; i < nf; i += blockDim.x) {
        const float4 c = cen[i];
        lo[0] = fminf(lo[0], c.x); lo[1] = fminf(lo[1], c.y); lo[2] = fminf(lo[2], c.z);
        hi[0] = fmaxf(hi[0], c.x); hi[1] = fmaxf(hi[1], c.y); hi[2] = fmaxf(hi[2], c.z);
    }
    for (int k = 0; k < 3; ++k) { smin[k][t] = lo[k]; smax[k][t] = hi[k]; }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < 3; ++k) {
                smin[k][t] = fminf(smin[k][t], smin[k][t + s]);
                smax[k][t] = fmaxf(smax[k][t], smax[k][t + s]);
            }
        __syncthreads();
    }
    if (t == 0) {
        // one scale for all axes (cubic cells): 1024 cells along the longest extent
        double ext = 0.0;
        for (int k = 0; k < 3; ++k) ext = fmax(ext, (double)smax[k][0] - (double)smin[k][0]);
        for (int k = 0; k < 3; ++k) {
            out[k] = smin[k][0];
            out[3 + k] = smax[k][0];
            out[6 + k] = ext > 0.0 ? (float)(1024.0 / ext) : 0.0f;
        }
    }
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(const float4* __restrict__ cen, int nf, const float* __restrict__ bnd, uint32_t* keys,
                         uint32_t* vals) {
#pragma clang fp contract(off)
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const float4 c = cen[f];
    const float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        const float d = cc[k] - bnd[k];
        const float p = d * bnd[6 + k];
        const int qi = (int)floorf(p);
        q[k] = (uint32_t)min(1023, max(0, qi));
    }
    keys[f] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[f] = (uint32_t)f;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u32 key, u32 value), 8-bit digits, tiles of 1024
// ---------------------------------------------------------------------------
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 4;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ void k_rs_hist(const uint32_t* __restrict__ keys, int n, int shift, uint32_t* hist, int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = base + r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of hist[256 * nblocks] (digit-major) in one block
__global__ void k_rs_scan(uint32_t* hist, int total) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (total + 1023) / 1024;
    const int b = t * per, e = min(total, b + per);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < 1024; ++i) { const uint32_t v = part[i]; part[i] = acc; acc += v; }
    }
    __syncthreads();
    uint32_t acc = part[t];
    for (int i = b; i < e; ++i) { const uint32_t v = hist[i]; hist[i] = acc; acc += v; }
}

__global__ void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* kout,
                             uint32_t* vout, int n, int shift, const uint32_t* __restrict__ hist, int nblocks) {
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t wcount[NW][256];
    __shared__ uint32_t running[256];
    __shared__ uint32_t gbase[256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    running[t] = 0;
    gbase[t] = hist[t * nblocks + blockIdx.x];
    for (int k = 0; k < NW; ++k) wcount[k][t] = 0;
    __syncthreads();
    const int base = blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = base + r * RS_THREADS + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t dg = (key >> shift) & 0xFFu;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcount[w][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        {   // per digit: offsets of each wave inside this round
            uint32_t acc = running[t];
            for (int k = 0; k < NW; ++k) { const uint32_t c = wcount[k][t]; wcount[k][t] = acc; acc += c; }
            running[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = gbase[dg] + wcount[w][dg] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        for (int k = 0; k < NW; ++k) wcount[k][t] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Karras 2012 hierarchy over the sorted 64-bit keys (morton << 32 | face)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int kdelta(const uint32_t* m, const uint32_t* fa, int n, int i, int j) {
    if (j < 0 || j > n - 1) return -1;
    const uint64_t a = ((uint64_t)m[i] << 32) | fa[i];
    const uint64_t b = ((uint64_t)m[j] << 32) | fa[j];
    return __clzll(a ^ b);
}

__global__ void k_karras(const uint32_t* __restrict__ m, const uint32_t* __restrict__ fa, int n, int* child,
                         int* parent) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = kdelta(m, fa, n, i, i + 1) > kdelta(m, fa, n, i, i - 1) ? 1 : -1;
    const int dmin = kdelta(m, fa, n, i, i - d);
    int lmax = 2;
    while (kdelta(m, fa, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (kdelta(m, fa, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = kdelta(m, fa, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(m, fa, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int split = i + s * d + min(d, 0);
    const int left = (min(i, j) == split) ? (int)(LEAF_BIT | (uint32_t)split) : split;
    const int right = (max(i, j) == split + 1) ? (int)(LEAF_BIT | (uint32_t)(split + 1)) : split + 1;
    child[2 * i] = left;
    child[2 * i + 1] = right;
    parent[(left & (int)LEAF_BIT) ? (n - 1) + (left & 0x7FFFFFFF) : left] = i;
    parent[(right & (int)LEAF_BIT) ? (n - 1) + (right & 0x7FFFFFFF) : right] = i;
    if (i == 0) parent[0] = -1;
}

__global__ void k_leaf_init(const uint32_t* __restrict__ sface, const float4* __restrict__ bmin,
                            const float4* __restrict__ bmax, const float* __restrict__ V, const int* __restrict__ F,
                            int n, float* aabb, float4* tri, int* fleaf, int* cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) cnt[i] = 0;
    if (i >= n) return;
    const int f = (int)sface[i];
    fleaf[f] = i;
    float* b = aabb + 6 * ((size_t)(n - 1) + i);
    const float4 mn = bmin[f], mx = bmax[f];
    b[0] = mn.x; b[1] = mn.y; b[2] = mn.z; b[3] = mx.x; b[4] = mx.y; b[5] = mx.z;
    const V3 a = ld3(V + 3 * F[3 * f]), bb = ld3(V + 3 * F[3 * f + 1]), c = ld3(V + 3 * F[3 * f + 2]);
    const V3 e1 = bb - a, e2 = c - a;
    tri[3 * i] = make_float4(a.x, a.y, a.z, __int_as_float(f));
    tri[3 * i + 1] = make_float4(e1.x, e1.y, e1.z, 0.f);
    tri[3 * i + 2] = make_float4(e2.x, e2.y, e2.z, 0.f);
}

__device__ __forceinline__ float aload(const float* p) {
    return __uint_as_float(__hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__global__ void k_refit(const int* __restrict__ parent, const int* __restrict__ child, int n, float* aabb,
                        int* cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int node = parent[(n - 1) + i];
    for (int depth = 0; node >= 0 && depth < 128; ++depth) {
        __threadfence();
        if (atomicAdd(&cnt[node], 1) == 0) return;    // the other child is not done yet
        __threadfence();
        float box[6];
        const int c0 = child[2 * node], c1 = child[2 * node + 1];
        const size_t i0 = (c0 & (int)LEAF_BIT) ? (size_t)(n - 1) + (c0 & 0x7FFFFFFF) : (size_t)c0;
        const size_t i1 = (c1 & (int)LEAF_BIT) ? (size_t)(n - 1) + (c1 & 0x7FFFFFFF) : (size_t)c1;
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(aload(aabb + 6 * i0 + k), aload(aabb + 6 * i1 + k));
            box[3 + k] = fmaxf(aload(aabb + 6 * i0 + 3 + k), aload(aabb + 6 * i1 + 3 + k));
        }
        for (int k = 0; k < 6; ++k)
            __hip_atomic_store((uint32_t*)(aabb + 6 * (size_t)node + k), __float_as_uint(box[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        node = parent[node];
    }
}

// ---------------------------------------------------------------------------
// Treelet restructuring of the Karras tree (Karras and Aila, HPG 2013), one
// bottom-up pass per launch.  Every internal node r with at least TL_LEAVES
// triangles below it, once both of its subtrees are final (second arrival at
// r's counter, as in the refit), becomes the root of a treelet of TL_LEAVES
// entries (smaller nodes only get their triangle count and SAH cost, each by
// the lane that reached it): starting from r's two children, the
// internal entry with the largest box area (first in list order on ties) is
// replaced by its two children, appended at the end of the list.  The entries
// are re-arranged into the binary tree of least SAH cost (a triangle leaf costs
// its box area, an internal node C_INNER * area + the costs of its children),
// found by dynamic programming over the 2^k - 1 subsets of entries; the
// treelet's internal nodes are reused (r stays the root, the others in
// ascending id order along the preorder of the new tree).  All comparisons are
// in float32 with contraction off, in a fixed order, so the tree is a function
// of the mesh alone, not of the wave schedule.
//
// One wave owns a treelet at a time: lane 0 forms it and writes the rebuilt
// nodes, the 64 lanes share the subset DP (subsets L and L + 64 per lane, one
// subset size per step).  Every access to tree data that another wave may
// write during the pass is an agent-scope atomic (coherent across the XCDs'
// L2s without flushing them), so the hand-off at a node's counter needs only
// the wave's own outstanding stores drained before the increment
// (handoff_release), not an L2 write-back and invalidate per level.
// ---------------------------------------------------------------------------
constexpr int TL_LEAVES = 7;
constexpr float TL_C_INNER = 1.2f;
constexpr int TL_BLOCK = 256;
constexpr int TL_WAVES = TL_BLOCK / 64;
constexpr int TL_GUARD = 1 << 16;

__device__ __forceinline__ int ald_i(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ast_i(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ast_f(float* p, float v) {
    __hip_atomic_store((uint32_t*)p, __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float tl_area(const float* b) {
#pragma clang fp contract(off)
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return 2.0f * ((dx * dy + dy * dz) + dz * dx);
}
__device__ __forceinline__ void handoff_release() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);     // no compiler motion across this point
    __builtin_amdgcn_s_waitcnt(0);               // every store of this wave has completed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct TreeletLds {
    float opt[128];
    int part[128];
    int ent[TL_LEAVES + 1];
    int ids[TL_LEAVES];
    float box[TL_LEAVES + 1][6];
    float cost[TL_LEAVES + 1];
    int leaves[TL_LEAVES + 1];
    int k;
};

__device__ void treelet_restructure(int r, int lane, TreeletLds& T, int* child, int* parent, float* aabb,
                                    float* tcost, int* tleaves, int n) {
#pragma clang fp contract(off)
    auto bidx = [n](int code) -> size_t {
        return (code & (int)LEAF_BIT) ? (size_t)(n - 1) + (code & 0x7FFFFFFF) : (size_t)code;
    };
    wave_sync_lds();
    if (lane == 0) {
        int ent[TL_LEAVES + 1], ids[TL_LEAVES];
        float box[TL_LEAVES + 1][6], area[TL_LEAVES + 1];
        int k = 2, ni = 1;
        ids[0] = r;
        for (int a = 0; a < 2; ++a) {
            ent[a] = ald_i(child + 2 * r + a);
            for (int q = 0; q < 6; ++q) box[a][q] = aload(aabb + 6 * bidx(ent[a]) + q);
            area[a] = tl_area(box[a]);
        }
        while (k < TL_LEAVES) {
            int bi = -1;
            float ba = -1.0f;
            for (int i = 0; i < k; ++i)
                if (!(ent[i] & (int)LEAF_BIT) && area[i] > ba) { ba = area[i]; bi = i; }
            if (bi < 0) break;
            const int c = ent[bi];
            ids[ni++] = c;
            for (int i = bi; i + 1 < k; ++i) {
                ent[i] = ent[i + 1];
                area[i] = area[i + 1];
                for (int q = 0; q < 6; ++q) box[i][q] = box[i + 1][q];
            }
            k -= 1;
            for (int a = 0; a < 2; ++a, ++k) {
                ent[k] = ald_i(child + 2 * c + a);
                for (int q = 0; q < 6; ++q) box[k][q] = aload(aabb + 6 * bidx(ent[k]) + q);
                area[k] = tl_area(box[k]);
            }
        }
        T.k = k;
        for (int i = 0; i < k; ++i) {
            T.ent[i] = ent[i];
            for (int q = 0; q < 6; ++q) T.box[i][q] = box[i][q];
            T.cost[i] = (ent[i] & (int)LEAF_BIT) ? area[i] : aload(tcost + ent[i]);
            T.leaves[i] = (ent[i] & (int)LEAF_BIT) ? 1 : ald_i(tleaves + ent[i]);
        }
        // the internal nodes other than r in ascending id order (insertion sort)
        for (int i = 2; i < ni; ++i) {
            const int v = ids[i];
            int j = i - 1;
            while (j >= 1 && ids[j] > v) { ids[j + 1] = ids[j]; --j; }
            ids[j + 1] = v;
        }
        for (int i = 0; i < ni; ++i) T.ids[i] = ids[i];
    }
    wave_sync_lds();
    const int k = T.k, full = (1 << k) - 1;
    // union-box areas of this lane's subsets, singletons' costs
    float sarea[2];
    int sset[2];
    for (int h = 0; h < 2; ++h) {
        const int S = lane + 64 * h;
        sset[h] = (S >= 1 && S <= full) ? S : 0;
        float u[6] = {__int_as_float(0x7f800000), __int_as_float(0x7f800000), __int_as_float(0x7f800000),
                      -__int_as_float(0x7f800000), -__int_as_float(0x7f800000), -__int_as_float(0x7f800000)};
        for (int j = 0; j < k; ++j)
            if (sset[h] >> j & 1)
                for (int q = 0; q < 3; ++q) {
                    u[q] = fminf(u[q], T.box[j][q]);
                    u[3 + q] = fmaxf(u[3 + q], T.box[j][3 + q]);
                }
        sarea[h] = sset[h] ? tl_area(u) : 0.0f;
        if (sset[h] && __popc(sset[h]) == 1) T.opt[sset[h]] = T.cost[__ffs(sset[h]) - 1];
    }
    wave_sync_lds();
    for (int size = 2; size <= k; ++size) {
        for (int h = 0; h < 2; ++h) {
            const int S = sset[h];
            if (!S || __popc(S) != size) continue;
            const int lb = S & -S, rest = S ^ lb;
            float best = __int_as_float(0x7f800000);
            int bp = 0;
            int sub = (rest - 1) & rest;
            for (;;) {
                const int P = lb | sub;
                const float c = T.opt[P] + T.opt[S ^ P];
                if (c < best) { best = c; bp = P; }
                if (sub == 0) break;
                sub = (sub - 1) & rest;
            }
            T.opt[S] = TL_C_INNER * sarea[h] + best;
            T.part[S] = bp;
        }
        wave_sync_lds();
    }
    if (lane == 0) {
        // preorder of the optimal tree's internal subsets
        int pre[TL_LEAVES], st[TL_LEAVES + 1];
        int np = 0, sp = 0;
        st[sp++] = full;
        while (sp > 0) {
            const int S = st[--sp];
            pre[np++] = S;
            const int P = T.part[S], Q = S ^ P;
            if (__popc(Q) > 1) st[sp++] = Q;
            if (__popc(P) > 1) st[sp++] = P;
        }
        auto code_of = [&](int X) -> int {
            if (__popc(X) == 1) return T.ent[__ffs(X) - 1];
            for (int i = 0; i < np; ++i)
                if (pre[i] == X) return T.ids[i];
            return -1;
        };
        for (int i = 0; i < np; ++i) {
            const int S = pre[i], id = T.ids[i], P = T.part[S], Q = S ^ P;
            const int a = code_of(P), c = code_of(Q);
            ast_i(child + 2 * id, a);
            ast_i(child + 2 * id + 1, c);
            ast_i(parent + bidx(a), id);
            ast_i(parent + bidx(c), id);
            ast_f(tcost + id, T.opt[S]);
            int cnt = 0;
            for (int j = 0; j < k; ++j)
                if (S >> j & 1) cnt += T.leaves[j];
            ast_i(tleaves + id, cnt);
            float u[6] = {__int_as_float(0x7f800000), __int_as_float(0x7f800000), __int_as_float(0x7f800000),
                          -__int_as_float(0x7f800000), -__int_as_float(0x7f800000), -__int_as_float(0x7f800000)};
            for (int j = 0; j < k; ++j)
                if (S >> j & 1)
                    for (int q = 0; q < 3; ++q) {
                        u[q] = fminf(u[q], T.box[j][q]);
                        u[3 + q] = fmaxf(u[3 + q], T.box[j][3 + q]);
                    }
            for (int q = 0; q < 6; ++q) ast_f(aabb + 6 * (size_t)id + q, u[q]);
        }
    }
}

// triangle count and SAH cost of a code (leaf: 1 and its box area)
__device__ __forceinline__ void code_stats(int code, const float* aabb, const float* tcost, const int* tleaves, int n,
                                           int& leaves, float& cost) {
    if (code & (int)LEAF_BIT) {
        float b[6];
        for (int q = 0; q < 6; ++q) b[q] = aload(aabb + 6 * ((size_t)(n - 1) + (code & 0x7FFFFFFF)) + q);
        leaves = 1;
        cost = tl_area(b);
    } else {
        leaves = ald_i(tleaves + code);
        cost = aload(tcost + code);
    }
}

__global__ __launch_bounds__(TL_BLOCK) void k_treelet(int* child, int* parent, float* aabb, float* tcost,
                                                      int* tleaves, int* cnt, int n, uint32_t* err) {
#pragma clang fp contract(off)
    __shared__ TreeletLds lds[TL_WAVES];
    const int lane = threadIdx.x & 63;
    TreeletLds& T = lds[threadIdx.x >> 6];
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = leaf < n;
    int node = active ? parent[(n - 1) + leaf] : -1;
    if (node < 0) active = false;
    int guard = 0;
    for (; guard < TL_GUARD; ++guard) {
        bool own = false, big = false;
        if (active) {
            handoff_release();
            if (atomicAdd(&cnt[node], 1) == 0) active = false;    // the other subtree is not done yet
            else own = true;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        if (own) {
            int l0, l1;
            float k0, k1;
            code_stats(ald_i(child + 2 * node), aabb, tcost, tleaves, n, l0, k0);
            code_stats(ald_i(child + 2 * node + 1), aabb, tcost, tleaves, n, l1, k1);
            big = l0 + l1 >= TL_LEAVES;
            if (!big) {
                float b[6];
                for (int q = 0; q < 6; ++q) b[q] = aload(aabb + 6 * (size_t)node + q);
                ast_i(tleaves + node, l0 + l1);
                ast_f(tcost + node, TL_C_INNER * tl_area(b) + (k0 + k1));
            }
        }
        uint64_t m = __ballot(big);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            treelet_restructure(__builtin_amdgcn_readlane(node, src), lane, T, child, parent, aabb, tcost, tleaves, n);
        }
        if (own) {
            const int p = ald_i(parent + node);
            if (p < 0) active = false;
            else node = p;
        }
        if (__ballot(active) == 0) break;
    }
    if (guard == TL_GUARD && active) atomicOr(err, ERR_LOOP);
}

// Collapse of the binary tree into 4-wide nodes with the least summed box area
// of the 4-wide nodes (under the surface-area measure, the expected number of
// node visits of a ray that meets the root box; every triangle stays one leaf
// slot, so triangle tests do not depend on the collapse).  Bottom-up, like the
// refit, every internal node x with children l, r gets
//   D[x][1] = A(x) + min over a, b >= 1, a + b <= 4 of D[l][a] + D[r][b]
//             (x heads a 4-wide node; as a slot of its parent it is one slot)
//   D[x][k] = min(D[x][k - 1], min over a + b = k of D[l][a] + D[r][b]),  k = 2..4
//             (x opened: its subtree fills up to k slots of the enclosing node)
// with D = 0 for a leaf.  Ties keep the first candidate in the order written,
// so the tree is a function of the binary tree alone.  cdec[x]: bits 0-1 and
// 2-3 hold a - 1 and b - 1 of the first line; bits 4 + 2 (k - 2), two per k,
// the a of the second line (0: k - 1 slots).
__device__ __forceinline__ float box_area(const float* b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return 2.0f * (dx * dy + dy * dz + dz * dx);
}

__global__ void k_collapse_cost(const int* __restrict__ parent, const int* __restrict__ child,
                                const float* __restrict__ aabb, int n, int* cnt, float* cost, uint32_t* dec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int node = parent[(n - 1) + i];
    for (int depth = 0; node >= 0 && depth < 128; ++depth) {
        __threadfence();
        if (atomicAdd(&cnt[node], 1) == 0) return;    // the other child is not done yet
        __threadfence();
        float D[2][5];
        for (int j = 0; j < 2; ++j) {
            const int c = child[2 * node + j];
            D[j][0] = 0.0f;
            for (int k = 1; k <= 4; ++k) D[j][k] = (c & (int)LEAF_BIT) ? 0.0f : aload(cost + 4 * (size_t)c + (k - 1));
        }
        float head = __int_as_float(0x7f800000);
        uint32_t d = 0;
        for (int a = 1; a <= 3; ++a)
            for (int b = 1; a + b <= 4; ++b)
                if (D[0][a] + D[1][b] < head) {
                    head = D[0][a] + D[1][b];
                    d = (uint32_t)(a - 1) | ((uint32_t)(b - 1) << 2);
                }
        float Dx[5];
        Dx[1] = box_area(aabb + 6 * (size_t)node) + head;
        for (int k = 2; k <= 4; ++k) {
            float v = Dx[k - 1];
            uint32_t choice = 0;
            for (int a = 1; a < k; ++a)
                if (D[0][a] + D[1][k - a] < v) {
                    v = D[0][a] + D[1][k - a];
                    choice = (uint32_t)a;
                }
            Dx[k] = v;
            d |= choice << (4 + 2 * (k - 2));
        }
        for (int k = 1; k <= 4; ++k)
            __hip_atomic_store((uint32_t*)(cost + 4 * (size_t)node + (k - 1)), __float_as_uint(Dx[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        dec[node] = d;
        node = parent[node];
    }
}

// the number of slots (1..k) that node x's subtree takes in the enclosing 4-wide
// node when offered k: fewer while its choice for k is "k - 1 slots"
__device__ __forceinline__ int collapse_slots(uint32_t dx, int k) {
    while (k >= 2 && ((dx >> (4 + 2 * (k - 2))) & 3u) == 0u) --k;
    return k;
}

// flag[x] = 1 when internal node x heads a 4-wide node: the choices of its
// ancestors, replayed from the root down, leave it one slot (the root heads the
// tree).  The path is read upwards into a bit string first.
__global__ void k_collapse_flag(const int* __restrict__ parent, const int* __restrict__ child,
                                const uint32_t* __restrict__ dec, int n, int* flag, uint32_t* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    uint64_t bits[2] = {0ull, 0ull};   // bit j: the node at depth j + 1 on the path is a right child
    int depth = 0;
    for (int x = i; parent[x] >= 0; x = parent[x]) {
        if (depth >= 128) {
            // deeper than any radix tree over 64-bit keys: head a node (fewer slots
            // for the parent, never more)
            atomicOr(err, ERR_LOOP);
            flag[i] = 1;
            return;
        }
        const int px = parent[x];
        const uint64_t right = child[2 * px + 1] == x ? 1ull : 0ull;
        bits[depth >> 6] |= right << (depth & 63);
        ++depth;
    }
    // bits hold the path from i upwards: bit depth - 1 is the root's child
    int v = 0, k = 1;      // node on the path and its slot budget (1: heads a 4-wide node)
    for (int lvl = depth - 1; lvl >= 0; --lvl) {
        const uint32_t dv = dec[v];
        int a, b;
        if (k == 1) {
            a = (int)(dv & 3u) + 1;
            b = (int)((dv >> 2) & 3u) + 1;
        } else {
            a = (int)((dv >> (4 + 2 * (k - 2))) & 3u);
            b = k - a;
        }
        const int right = (int)((bits[lvl >> 6] >> (lvl & 63)) & 1ull);
        const int c = child[2 * v + right];
        k = collapse_slots(dec[c], right ? b : a);
        v = c;
    }
    flag[i] = k == 1 ? 1 : 0;
}

// 4-wide node of a binary node x that heads one: its children, every internal
// one that does not head a node replaced by its own two children until only
// leaves and heads remain (at most 4 by the costs above), in tree order (8
// float4: min x, max x, min y, max y, min z, max z of the 4 slots, child codes,
// pad)
__global__ void k_pack4(const int* __restrict__ child, const float* __restrict__ aabb, const int* __restrict__ flag,
                        const uint32_t* __restrict__ id4, int n, float4* nodes4, uint32_t* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1 || !flag[i]) return;
    int sl[4] = {child[2 * i], child[2 * i + 1], 0, 0};
    int m = 2;
    for (int pass = 0; pass < 3; ++pass) {
        int at = -1;
        for (int s = 0; s < m; ++s)
            if (at < 0 && !(sl[s] & (int)LEAF_BIT) && !flag[sl[s]]) at = s;
        if (at < 0) break;
        if (m == 4) { atomicOr(err, ERR_LOOP); break; }   // cannot happen: the costs allow at most 4 slots
        const int x = sl[at];
        for (int s = m; s > at + 1; --s) sl[s] = sl[s - 1];
        sl[at] = child[2 * x];
        sl[at + 1] = child[2 * x + 1];
        ++m;
    }
    float v[6][4];
    int cc[4];
    for (int s = 0; s < 4; ++s) {
        if (s < m) {
            const int c = sl[s];
            const size_t bi = (c & (int)LEAF_BIT) ? (size_t)(n - 1) + (c & 0x7FFFFFFF) : (size_t)c;
            const float* bb = aabb + 6 * bi;
            v[0][s] = bb[0]; v[1][s] = bb[3]; v[2][s] = bb[1]; v[3][s] = bb[4]; v[4][s] = bb[2]; v[5][s] = bb[5];
            cc[s] = (c & (int)LEAF_BIT) ? c : (int)id4[c];
        } else {
            // an empty slot is a box at +infinity on every axis: its slab test
            // gives an entry distance of +inf or an empty interval, a miss either way
            v[0][s] = v[1][s] = v[2][s] = v[3][s] = v[4][s] = v[5][s] = __int_as_float(0x7f800000);
            cc[s] = -1;
        }
    }
    float4* o = nodes4 + 8 * (size_t)id4[i];
    for (int k = 0; k < 6; ++k) o[k] = make_float4(v[k][0], v[k][1], v[k][2], v[k][3]);
    o[6] = make_float4(__int_as_float(cc[0]), __int_as_float(cc[1]), __int_as_float(cc[2]), __int_as_float(cc[3]));
    o[7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_keys64(const uint32_t* __restrict__ m, const uint32_t* __restrict__ fa, int n, uint64_t* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = ((uint64_t)m[i] << 32) | fa[i];
}

__global__ void k_edge_len(const int4* __restrict__ edges, int ne, const float* __restrict__ V, double* w) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int4 E = edges[e];
    const double dx = (double)V[3 * E.y] - (double)V[3 * E.x];
    const double dy = (double)V[3 * E.y + 1] - (double)V[3 * E.x + 1];
    const double dz = (double)V[3 * E.y + 2] - (double)V[3 * E.x + 2];
    w[e] = sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ void k_edge_cdf(const double* w, int ne, double* cdf, double* total, float* ftotal) {
    block_scan_normalise(w, ne, cdf, total);
    if (threadIdx.x == 0) *ftotal = (float)*total;
}

// environment map: per-row texel weights (mean rgb times row solid angle) and
// conditional CDFs, summed serially per row; marginal over rows serially.
__global__ void k_env_rows(const float* __restrict__ env, int he, int we, const double* __restrict__ dom,
                           double* cond, double* rows) {
#pragma clang fp contract(off)
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= he) return;
    double acc = 0.0;
    double* C = cond + (size_t)r * (we + 1);
    C[0] = 0.0;
    for (int c = 0; c < we; ++c) {
        const float* t = env + 3 * ((size_t)r * we + c);
        const double m = ((double)t[0] + (double)t[1] + (double)t[2]) / 3.0;
        acc += m * dom[r];
        C[c + 1] = acc;
    }
    rows[r] = acc;
    for (int c = 0; c <= we; ++c) C[c] = acc > 0.0 ? C[c] / acc : (double)c / we;
}

__global__ void k_env_marg(const double* rows, int he, double* marg, double* total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    marg[0] = 0.0;
    for (int r = 0; r < he; ++r) { acc += rows[r]; marg[r + 1] = acc; }
    *total = acc;
    for (int r = 0; r <= he; ++r) marg[r] = acc > 0.0 ? marg[r] / acc : 0.0;
}

__global__ void k_env_pdf(const float* __restrict__ env, int he, int we, const double* __restrict__ dom,
                          const double* __restrict__ total, float* texpdf) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= he * we) return;
    const int r = i / we;
    const float* t = env + 3 * (size_t)i;
    const double m = ((double)t[0] + (double)t[1] + (double)t[2]) / 3.0;
    const double tot = *total;
    texpdf[i] = tot > 0.0 ? (float)((m * dom[r]) / tot / dom[r]) : 0.0f;
}

// guide tables: for CDF row y (blockIdx.y), guide[g] = largest i in [0, n-1]
// with C[i] <= g / 2^glog (C[0] == 0)
__global__ void k_guide(const double* __restrict__ C, int n, size_t cstride, int* guide, int glog) {
    const int G = 1 << glog;
    const double* Cr = C + cstride * blockIdx.y;
    int* gr = guide + ((size_t)blockIdx.y << glog);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x)
        gr[g] = cdf_find(Cr, n, (double)g / (double)G);
}

void launch_guide(const double* C, int n, size_t cstride, int rows, int* guide, int glog, hipStream_t st) {
    if (n <= 0 || rows <= 0) return;
    const int G = 1 << glog;
    ST_LAUNCH("k_guide", k_guide, dim3((G + 255) / 256 < 1024 ? (G + 255) / 256 : 1024, rows), dim3(256), 0, st, C, n,
              cstride, guide, glog);
}

int guide_log2(int n) {
    int l = 0;
    while ((1 << l) < n && l < 24) ++l;
    return l;
}

// 1 -> 4 subdivision (Sec. 3.2 "Subdivision": every edge split at its
// midpoint): vertices [V; midpoint of edge e at nv + e], face f ->
// (v0, m01, m20), (v1, m12, m01), (v2, m20, m12), (m01, m12, m20) at 4f.. 4f+3,
// which keeps every face's orientation
__global__ void k_subdivide(const float* __restrict__ V, const int* __restrict__ F, const int* __restrict__ fe,
                            const int4* __restrict__ edges, int nv, int nf, int ne, float* outV, int* outF) {
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += stride) outV[i] = V[i];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        const int4 E = edges[e];
        for (int c = 0; c < 3; ++c) outV[3 * (size_t)(nv + e) + c] = (V[3 * E.x + c] + V[3 * E.y + c]) * 0.5f;
    }
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += stride) {
        const int v0 = F[3 * f], v1 = F[3 * f + 1], v2 = F[3 * f + 2];
        // a degenerate edge (both ends one vertex) has that vertex as its midpoint
        const int m01 = fe[3 * f] >= 0 ? nv + fe[3 * f] : v0;
        const int m12 = fe[3 * f + 1] >= 0 ? nv + fe[3 * f + 1] : v1;
        const int m20 = fe[3 * f + 2] >= 0 ? nv + fe[3 * f + 2] : v2;
        int* o = outF + 12 * (size_t)f;
        o[0] = v0;  o[1] = m01; o[2] = m20;
        o[3] = v1;  o[4] = m12; o[5] = m01;
        o[6] = v2;  o[7] = m20; o[8] = m12;
        o[9] = m01; o[10] = m12; o[11] = m20;
    }
}


// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_subdivide(const SceneDev& s, float* out_V, int32_t* out_F, hipStream_t st) {
    const long long n = std::max<long long>(std::max<long long>(3ll * s.nv, s.ne), s.nf);
    ST_LAUNCH("k_subdivide", k_subdivide, dim3(nb(n, 256) < 4096 ? nb(n, 256) : 4096), dim3(256), 0, st, s.V, s.F,
              s.fe, s.edges, s.nv, s.nf, s.ne, out_V, out_F);
}


// ---------------------------------------------------------------------------
// secondary-edge importance tree: the same radix tree over the edges' boxes,
// each node also carrying the float sum of the edge lengths below it
// ---------------------------------------------------------------------------
__global__ void k_edge_prep(const float* __restrict__ V, const int4* __restrict__ edges, int ne, float4* bmin,
                            float4* bmax, float4* cen) {
#pragma clang fp contract(off)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int4 E = edges[e];
    const V3 a = ld3(V + 3 * E.x), c = ld3(V + 3 * E.y);
    const V3 mn{fminf(a.x, c.x), fminf(a.y, c.y), fminf(a.z, c.z)};
    const V3 mx{fmaxf(a.x, c.x), fmaxf(a.y, c.y), fmaxf(a.z, c.z)};
    bmin[e] = make_float4(mn.x, mn.y, mn.z, 0.f);
    bmax[e] = make_float4(mx.x, mx.y, mx.z, 0.f);
    const float cx = mn.x + mx.x, cy = mn.y + mx.y, cz = mn.z + mx.z;
    cen[e] = make_float4(cx * 0.5f, cy * 0.5f, cz * 0.5f, 0.f);
}

// unit normal of face f: the double cross product of the float edge vectors over
// its double length, rounded to float; false for a degenerate face
__device__ __forceinline__ bool unit_normal_d(const float* __restrict__ V, const int* __restrict__ F, int f,
                                              float* un) {
#pragma clang fp contract(off)
    double q[3][3];
    for (int a = 0; a < 3; ++a) {
        const int v = F[3 * f + a];
        for (int k = 0; k < 3; ++k) q[a][k] = (double)V[3 * v + k];
    }
    const double e1x = q[1][0] - q[0][0], e1y = q[1][1] - q[0][1], e1z = q[1][2] - q[0][2];
    const double e2x = q[2][0] - q[0][0], e2y = q[2][1] - q[0][1], e2z = q[2][2] - q[0][2];
    const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
    const double l = sqrt((cx * cx + cy * cy) + cz * cz);
    if (!(l > 0.0) || !isfinite(l)) return false;
    un[0] = (float)(cx / l); un[1] = (float)(cy / l); un[2] = (float)(cz / l);
    return true;
}

// leaves of the edge tree in sorted order: box, length (the double-precision
// length of the float endpoints, rounded to float) and the box of the adjacent
// faces' unit normals (the whole cube [-1, 1]^3, which never culls, for a
// boundary edge or a degenerate face); clears the refit counters
__global__ void k_eleaf_init(const uint32_t* __restrict__ sedge, const float4* __restrict__ bmin,
                             const float4* __restrict__ bmax, const int4* __restrict__ edges,
                             const float* __restrict__ V, const int* __restrict__ F, int n, float* aabb, float* len,
                             float* nbox, int* cnt) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) cnt[i] = 0;
    if (i >= n) return;
    const int e = (int)sedge[i];
    float* bx = aabb + 6 * ((size_t)(n - 1) + i);
    const float4 mn = bmin[e], mx = bmax[e];
    bx[0] = mn.x; bx[1] = mn.y; bx[2] = mn.z; bx[3] = mx.x; bx[4] = mx.y; bx[5] = mx.z;
    const int4 E = edges[e];
    const double dx = (double)V[3 * E.y] - (double)V[3 * E.x];
    const double dy = (double)V[3 * E.y + 1] - (double)V[3 * E.x + 1];
    const double dz = (double)V[3 * E.y + 2] - (double)V[3 * E.x + 2];
    len[(size_t)(n - 1) + i] = (float)sqrt((dx * dx + dy * dy) + dz * dz);
    float nb[6] = {-1.0f, -1.0f, -1.0f, 1.0f, 1.0f, 1.0f};
    float n1[3], n2[3];
    if (E.w >= 0 && unit_normal_d(V, F, E.z, n1) && unit_normal_d(V, F, E.w, n2))
        for (int k = 0; k < 3; ++k) {
            nb[k] = fminf(n1[k], n2[k]);
            nb[3 + k] = fmaxf(n1[k], n2[k]);
        }
    float* o = nbox + 6 * ((size_t)(n - 1) + i);
    for (int k = 0; k < 6; ++k) o[k] = nb[k];
}

// bottom-up boxes and length sums of the edge tree (second arrival at a node
// combines its two children, as in the refit)
__global__ void k_erefit(const int* __restrict__ parent, const int* __restrict__ child, int n, float* aabb,
                         float* len, float* nbox, int* cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int node = parent[(n - 1) + i];
    for (int depth = 0; node >= 0 && depth < 4096; ++depth) {
        __threadfence();
        if (atomicAdd(&cnt[node], 1) == 0) return;
        __threadfence();
        const int c0 = child[2 * node], c1 = child[2 * node + 1];
        const size_t i0 = (c0 & (int)LEAF_BIT) ? (size_t)(n - 1) + (c0 & 0x7FFFFFFF) : (size_t)c0;
        const size_t i1 = (c1 & (int)LEAF_BIT) ? (size_t)(n - 1) + (c1 & 0x7FFFFFFF) : (size_t)c1;
        float box[6];
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(aload(aabb + 6 * i0 + k), aload(aabb + 6 * i1 + k));
            box[3 + k] = fmaxf(aload(aabb + 6 * i0 + 3 + k), aload(aabb + 6 * i1 + 3 + k));
        }
        for (int k = 0; k < 6; ++k)
            __hip_atomic_store((uint32_t*)(aabb + 6 * (size_t)node + k), __float_as_uint(box[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(aload(nbox + 6 * i0 + k), aload(nbox + 6 * i1 + k));
            box[3 + k] = fmaxf(aload(nbox + 6 * i0 + 3 + k), aload(nbox + 6 * i1 + 3 + k));
        }
        for (int k = 0; k < 6; ++k)
            __hip_atomic_store((uint32_t*)(nbox + 6 * (size_t)node + k), __float_as_uint(box[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        const float l = aload(len + i0) + aload(len + i1);
        __hip_atomic_store((uint32_t*)(len + node), __float_as_uint(l), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        node = parent[node];
    }
}

// packed record of internal node i of the edge tree: for child j, float4s
// 4j..4j+3 hold its box (lower, upper), length, normal box (lower, upper) and code
__global__ void k_epack(const int* __restrict__ child, const float* __restrict__ aabb, const float* __restrict__ len,
                        const float* __restrict__ nbox, int n, float4* node) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    for (int j = 0; j < 2; ++j) {
        const int c = child[2 * i + j];
        const size_t k = (c & (int)LEAF_BIT) ? (size_t)(n - 1) + (c & 0x7FFFFFFF) : (size_t)c;
        const float* b = aabb + 6 * k;
        const float* nb = nbox + 6 * k;
        float4* o = node + 8 * (size_t)i + 4 * j;
        o[0] = make_float4(b[0], b[1], b[2], b[3]);
        o[1] = make_float4(b[4], b[5], len[k], nb[0]);
        o[2] = make_float4(nb[1], nb[2], nb[3], nb[4]);
        o[3] = make_float4(nb[5], __int_as_float(c), 0.0f, 0.0f);
    }
}

// Morton keys of n centres, stably sorted (4 LSD passes); returns the buffer
// index that holds the sorted (key, value) pairs
static int radix_sort_keys(const float4* cen, int n, float* bounds, uint32_t* const mk[2], uint32_t* const mv[2],
                           uint32_t* hist, hipStream_t st) {
    ST_LAUNCH("k_bounds", k_bounds, dim3(1), dim3(1024), 0, st, cen, n, bounds);
    ST_LAUNCH("k_morton", k_morton, dim3(nb(n, 256)), dim3(256), 0, st, cen, n, bounds, mk[0], mv[0]);
    const int nblocks = (n + RS_TILE - 1) / RS_TILE;
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        ST_LAUNCH("k_rs_hist", k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, st, mk[cur], n, shift, hist, nblocks);
        ST_LAUNCH("k_rs_scan", k_rs_scan, dim3(1), dim3(1024), 0, st, hist, 256 * nblocks);
        ST_LAUNCH("k_rs_scatter", k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, st, mk[cur], mv[cur], mk[cur ^ 1],
                  mv[cur ^ 1], n, shift, hist, nblocks);
        cur ^= 1;
    }
    return cur;
}

void launch_edge_tree(SceneDev& s, hipStream_t st) {
    const int n = s.ne;
    if (n <= 0) return;
    ST_LAUNCH("k_edge_prep", k_edge_prep, dim3(nb(n, 256)), dim3(256), 0, st, s.V, s.edges, n, s.ebmin, s.ebmax,
              s.ecen);
    const int cur = radix_sort_keys(s.ecen, n, s.ebounds, s.emkeys, s.emvals, s.ers_hist, st);
    const uint32_t* sm = s.emkeys[cur];
    const uint32_t* se = s.emvals[cur];
    s.eleaf_edge = se;
    ST_LAUNCH("k_keys64", k_keys64, dim3(nb(n, 256)), dim3(256), 0, st, sm, se, n, s.ekeys64);
    if (n > 1) ST_LAUNCH("k_karras", k_karras, dim3(nb(n - 1, 256)), dim3(256), 0, st, sm, se, n, s.echild, s.eparent);
    ST_LAUNCH("k_eleaf_init", k_eleaf_init, dim3(nb(n, 256)), dim3(256), 0, st, se, s.ebmin, s.ebmax, s.edges, s.V,
              s.F, n, s.eaabb, s.elen, s.enbox, s.ecnt);
    if (n > 1) {
        ST_LAUNCH("k_erefit", k_erefit, dim3(nb(n, 256)), dim3(256), 0, st, s.eparent, s.echild, n, s.eaabb, s.elen,
                  s.enbox, s.ecnt);
        ST_LAUNCH("k_epack", k_epack, dim3(nb(n - 1, 256)), dim3(256), 0, st, s.echild, s.eaabb, s.elen, s.enbox, n,
                  s.enode);
    }
}

void launch_scene_geometry(SceneDev& s, hipStream_t st) {
    const int nf = s.nf;
    if (nf <= 0) return;
    ST_LAUNCH("k_face_prep", k_face_prep, dim3(nb(nf, 256)), dim3(256), 0, st, s.V, s.F, nf, s.fnorm, s.bmin, s.bmax,
                       s.cen);
    ST_LAUNCH("k_bounds", k_bounds, dim3(1), dim3(1024), 0, st, s.cen, nf, s.bounds);
    ST_LAUNCH("k_morton", k_morton, dim3(nb(nf, 256)), dim3(256), 0, st, s.cen, nf, s.bounds, s.mkeys[0], s.mvals[0]);
    const int nblocks = (nf + RS_TILE - 1) / RS_TILE;
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        ST_LAUNCH("k_rs_hist", k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, st, s.mkeys[cur], nf, shift, s.rs_hist,
                           nblocks);
        ST_LAUNCH("k_rs_scan", k_rs_scan, dim3(1), dim3(1024), 0, st, s.rs_hist, 256 * nblocks);
        ST_LAUNCH("k_rs_scatter", k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, st, s.mkeys[cur], s.mvals[cur],
                           s.mkeys[cur ^ 1], s.mvals[cur ^ 1], nf, shift, s.rs_hist, nblocks);
        cur ^= 1;
    }
    // after 4 passes the sorted data is back in buffer 0
    const uint32_t* sm = s.mkeys[cur];
    const uint32_t* sf = s.mvals[cur];
    ST_LAUNCH("k_keys64", k_keys64, dim3(nb(nf, 256)), dim3(256), 0, st, sm, sf, nf, s.keys64);
    if (nf > 1)
        ST_LAUNCH("k_karras", k_karras, dim3(nb(nf - 1, 256)), dim3(256), 0, st, sm, sf, nf, s.child, s.parent);
    ST_LAUNCH("k_leaf_init", k_leaf_init, dim3(nb(nf, 256)), dim3(256), 0, st, sf, s.bmin, s.bmax, s.V, s.F, nf, s.aabb,
                       s.tri, s.fleaf, s.refit_cnt);
    if (nf > 1) {
        ST_LAUNCH("k_refit", k_refit, dim3(nb(nf, 256)), dim3(256), 0, st, s.parent, s.child, nf, s.aabb,
                           s.refit_cnt);
        for (int rd = 0; rd < TREELET_ROUNDS; ++rd) {
            launch_fill_u32((uint32_t*)s.refit_cnt, nf - 1, 0u, st);
            ST_LAUNCH("k_treelet", k_treelet, dim3(nb(nf, TL_BLOCK)), dim3(TL_BLOCK), 0, st, s.child, s.parent, s.aabb,
                      s.tcost, s.tleaves, s.refit_cnt, nf, s.err);
        }
        launch_fill_u32((uint32_t*)s.refit_cnt, nf - 1, 0u, st);
        ST_LAUNCH("k_collapse_cost", k_collapse_cost, dim3(nb(nf, 256)), dim3(256), 0, st, s.parent, s.child, s.aabb,
                  nf, s.refit_cnt, (float*)s.ccost, s.cdec);
        ST_LAUNCH("k_collapse_flag", k_collapse_flag, dim3(nb(nf - 1, 256)), dim3(256), 0, st, s.parent, s.child,
                  s.cdec, nf, s.flag4, s.err);
        hipMemcpyAsync(s.id4, s.flag4, sizeof(int) * (nf - 1), hipMemcpyDeviceToDevice, st);
        ST_LAUNCH("k_rs_scan", k_rs_scan, dim3(1), dim3(1024), 0, st, s.id4, nf - 1);
        ST_LAUNCH("k_pack4", k_pack4, dim3(nb(nf - 1, 256)), dim3(256), 0, st, s.child, s.aabb, s.flag4, s.id4, nf,
                  s.nodes4, s.err);
    }
    if (s.ne > 0) {
        ST_LAUNCH("k_edge_len", k_edge_len, dim3(nb(s.ne, 256)), dim3(256), 0, st, s.edges, s.ne, s.V, s.edge_w);
        ST_LAUNCH("k_edge_cdf", k_edge_cdf, dim3(1), dim3(1024), 0, st, s.edge_w, s.ne, s.ecdf, s.etotal_d,
                           s.etotal_f);
        launch_guide(s.ecdf, s.ne, 0, 1, s.eguide, guide_log2(s.ne), st);
    }
}

void launch_env_build(SceneDev& s, hipStream_t st) {
    if (s.he <= 0) return;
    ST_LAUNCH("k_env_rows", k_env_rows, dim3(nb(s.he, 64)), dim3(64), 0, st, s.env, s.he, s.we, s.row_dom, s.cond,
                       s.env_rows);
    ST_LAUNCH("k_env_marg", k_env_marg, dim3(1), dim3(64), 0, st, s.env_rows, s.he, s.marg, s.env_total);
    launch_guide(s.marg, s.he, 0, 1, s.mguide, guide_log2(s.he), st);
    launch_guide(s.cond, s.we, (size_t)(s.we + 1), s.he, s.cguide, guide_log2(s.we), st);
    ST_LAUNCH("k_env_pdf", k_env_pdf, dim3(nb((long long)s.he * s.we, 256)), dim3(256), 0, st, s.env, s.he, s.we,
                       s.row_dom, s.env_total, s.texpdf);
}

} // namespace st

// Forward rendering R(x, m, c_i) (Shape from Tracing, Sec. 3.2) as a wavefront
// path tracer: per bounce a closest-hit kernel over a compacted ray queue, a
// shading kernel (next-event estimation set-up, BRDF sampling, wave-ballot
// compaction of the surviving paths) and a per-path shadow kernel that traces
// the point-light and environment shadow rays and adds their contributions in a
// fixed order.  Queues are structure-of-arrays in HBM; per-sample radiance is
// kept for a final film pass that averages the samples of each pixel.
#include "st_internal.h"

namespace st {

// occupancy targets (waves per SIMD) the compiler fits the register budget to
#ifndef ST_SHADE_WAVES
#define ST_SHADE_WAVES 6
#endif
#ifndef ST_EXTEND_WAVES
#define ST_EXTEND_WAVES 8
#endif
#ifndef ST_SHADOW_WAVES
#define ST_SHADOW_WAVES 8
#endif
#define SHADE_OCC __attribute__((amdgpu_waves_per_eu(ST_SHADE_WAVES)))
#ifndef ST_SHADE_BLOCK
#define ST_SHADE_BLOCK 512
#endif
constexpr int SHADE_BLOCK = ST_SHADE_BLOCK;   // threads of a k_shade block (one queue reservation each)
#define EXTEND_OCC __attribute__((amdgpu_waves_per_eu(ST_EXTEND_WAVES)))
#define SHADOW_OCC __attribute__((amdgpu_waves_per_eu(ST_SHADOW_WAVES)))



// canonical path index of a (view, pixel, sample)
__device__ __forceinline__ long long canon(const DevCam& c, int x, int y, int j, int spp) {
    return (c.pixoff + (long long)y * c.W + x) * spp + j;
}

// final decision hash of a path: canonical debug slot, or the path's radiance slot
__device__ __forceinline__ void final_hash(const FwdParams& p, float* const* r, int i, uint32_t h) {
    if (p.hash_by_q) {
        p.hash_by_q[qu(r, QQ, i)] = h;
    } else if (p.dbg_hash) {
        const DevCam& c = p.cams[qu(r, QVD, i) & 0xFFFFu];
        p.dbg_hash[(c.pixoff + (long long)qu(r, QC0, i)) * p.spp + (qu(r, QC1, i) & 0xFFFFu)] = h;
    }
}

// ---------------------------------------------------------------------------
__global__ void k_camera(FwdParams p, Queues q, long long q0, int n) {
    const int stride = gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x < 64) q.cnt[threadIdx.x] = threadIdx.x == 1 ? n : 0;
    // the hit records are rewritten from here on: their key is cleared until k_film
    if (q0 == 0 && blockIdx.x == 0 && threadIdx.x == 0 && p.rec_key_dev) *p.rec_key_dev = 0ull;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < FETCH_INTS; j += stride) q.fetch[j] = 0;
    float* const* r = q.ray[1];
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const long long qq = q0 + s;
        const int v = find_view(p.qoff, p.ncam, qq);
        const DevCam& c = p.cams[v];
        const DevScene& S = p.scenes[c.scene];
        int x, y, j;
        decode_path(c, qq - c.qoff, p.spp, x, y, j);
        const Ctr ctr{(uint32_t)(y * c.W + x), ((uint32_t)c.rngview << 16) | (uint32_t)j, 0u, 0u};
        const float4 u = draw4(ctr, 0, 0, Key{p.seed, S.scene_id});
        const V3 d = cam_dir(c, (float)x + u.x, (float)y + u.y);
        // origin (the eye), previous pdf, throughput and hash of a camera ray are
        // constants that the bounce-1 kernels take from the camera themselves
        qf_st(r, QDX, s, d.x); qf_st(r, QDY, s, d.y); qf_st(r, QDZ, s, d.z);
        qu_st(r, QEXCL, s, 0xFFFFFFFFu);
        qu_st(r, QQ, s, (uint32_t)qq);
        qu_st(r, QC0, s, ctr.c0);
        qu_st(r, QC1, s, ctr.c1);
        qu_st(r, QVD, s, (uint32_t)v);
        q.L[3 * (size_t)qq] = 0.0f; q.L[3 * (size_t)qq + 1] = 0.0f; q.L[3 * (size_t)qq + 2] = 0.0f;
    }
}

// closest hit of queue entry i of bounce k
__device__ __forceinline__ void extend_one(const FwdParams& p, const Queues& q, int k, float* const* r, int i,
                                           TravStack& st) {
    const DevCam& cam = p.cams[qu_ld(r, QVD, i) & 0xFFFFu];
    const DevScene& S = p.scenes[cam.scene];
    const V3 o = k == 1 ? ld3(cam.eye) : V3{qf(r, QOX, i), qf(r, QOY, i), qf(r, QOZ, i)};
    const V3 d{qf(r, QDX, i), qf(r, QDY, i), qf(r, QDZ, i)};
    uint32_t ex = qu_ld(r, QEXCL, i);
    float t0 = __int_as_float(0x7f800000);
    int f0 = -1;
    if (k == 1 && ex != 0xFFFFFFFFu) {
        // a primary-edge side ray names its edge: the edge's faces are
        // tested first, so that the traversal starts with their hit
        const int4 E = S.edges[ex & 0x7FFFFFFFu];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int fe = j == 0 ? E.z : E.w;
            float th; int fh;
            if (fe >= 0 && tri_test((const gfloat4*)S.tri, (uint32_t)S.fleaf[fe], o, d, TMIN,
                                    __int_as_float(0x7f800000), th, fh) &&
                (th < t0 || (th == t0 && fh < f0))) {
                t0 = th;
                f0 = fh;
            }
        }
        ex = 0xFFFFFFFFu;
    }
    float t;
    const int f = trace_closest(S, o, d, TMIN, (int)ex, t, st, t0, f0);
    qst(q.ht + i, t);
    qst(q.hf + i, f);
}

// closest hit for every queued ray of bounce k (queue k & 1)
#ifndef ST_EXTEND_QUEUE
#define ST_EXTEND_QUEUE 0
#endif
__global__ void __launch_bounds__(TRACE_BLOCK) EXTEND_OCC k_extend(FwdParams p, Queues q, int k) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    TravStack st = make_trav_stack(lds, q.spill, p.err, p.work ? p.work + 3 * WORK_EXTEND : nullptr);
    const int n = q.cnt[k];
    float* const* r = q.ray[k & 1];
    if (ST_EXTEND_QUEUE) {
        // persistent waves refilled from the fetch counters of slot 16 + k
        trace_queue<false>(
            q.fetch + FETCH_SLOT_INTS * (16 + k), n, st,
            [&](int i, RayJob& J) {
                const DevCam& cam = p.cams[qu_ld(r, QVD, i) & 0xFFFFu];
                const DevScene& S = p.scenes[cam.scene];
                J.o = k == 1 ? ld3(cam.eye) : V3{qf(r, QOX, i), qf(r, QOY, i), qf(r, QOZ, i)};
                J.d = V3{qf(r, QDX, i), qf(r, QDY, i), qf(r, QDZ, i)};
                J.tmax = __int_as_float(0x7f800000);
                J.excl = (int)qu_ld(r, QEXCL, i);
                J.G = trace_geo(S);
                return true;
            },
            [&](int i, int f, float t) {
                q.ht[i] = t;
                q.hf[i] = f;
            });
        return;
    }
    // 64 consecutive queue entries per wave, traced in lockstep
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) extend_one(p, q, k, r, i, st);
}

#ifndef ST_SHADOW_QUEUE
#define ST_SHADOW_QUEUE 0
#endif
#ifndef ST_PAIR_TRACE
#define ST_PAIR_TRACE 1
#endif
// With one shadow entry per shading point and no decision hashes, k_shadow adds
// each unoccluded contribution itself and records occlusion in the hit records,
// and k_shadow_sum is not launched (the sum over one entry is that entry).
__host__ __device__ __forceinline__ bool shadow_fused(const FwdParams& p, const Queues& q) {
    return !ST_SHADOW_QUEUE && q.nent == 1 && !(p.dbg_hash || p.hash_by_q);
}

// shading of bounce k: escapes, next-event set-up and BRDF continuation.
// HASH: decision hashes are asked for (p.dbg_hash or p.hash_by_q); compiled
// apart, because the hash state alone made the compiler spill 11 more dwords.
template <bool HASH>
__global__ void __launch_bounds__(SHADE_BLOCK) SHADE_OCC k_shade(FwdParams p, Queues q, int k) {
    __shared__ int resv[2 * (SHADE_BLOCK / 64 + 1)];
    const int n = q.cnt[k];
    float* const* r = q.ray[k & 1];
    float* const* rn = q.ray[(k + 1) & 1];
    const int stride = gridDim.x * blockDim.x;
    constexpr bool hashing = HASH;
    // with the shadow sum fused into k_shadow, the shading record keeps only what
    // k_shadow reads (face, point)
    const bool fused = shadow_fused(p, q);
    // every thread of a block runs the same number of iterations: the
    // compaction below reserves queue slots per block
    for (int b0 = blockIdx.x * blockDim.x; b0 < n; b0 += stride) {
        const int i = b0 + (int)threadIdx.x;
        const bool active = i < n;
        bool emit = false;
        uint32_t rays = 0;          // shadow entries of this shading point that carry a ray
        V3 x{0.f, 0.f, 0.f}, wi{0.f, 0.f, 0.f}, beta{0.f, 0.f, 0.f};
        float pb = 0.0f;
        int f = -1;
        uint32_t hv = 0;
        // path identity (slot, counters, camera | domain), carried to the continuation
        uint32_t pq = 0, c0 = 0, c1 = 0, vd = 0;
        if (active) {
            pq = qu_ld(r, QQ, i);
            c0 = qu_ld(r, QC0, i);
            c1 = qu_ld(r, QC1, i);
            vd = qu_ld(r, QVD, i);
            const DevScene& S = p.scenes[p.cams[vd & 0xFFFFu].scene];
            const Key key{p.seed, S.scene_id};
            const Ctr ctr{c0, c1, 0u, vd >> 16};
            Hash h{hashing ? (k == 1 ? FNV_INIT : qu_ld(r, QHASH, i)) : 0u, hashing};
            beta = k == 1 ? V3{1.f, 1.f, 1.f} : V3{qf(r, QBR, i), qf(r, QBG, i), qf(r, QBB, i)};
            f = qld(q.hf + i);
            push_face(h, f);
            if (p.rec_face && (vd >> 16) == 0u) qst(p.rec_face + (size_t)(k - 1) * p.rec_n + pq, f);
            if (!fused) q.sface[i] = -1;
            const V3 d{qf(r, QDX, i), qf(r, QDY, i), qf(r, QDZ, i)};
            if (f < 0) {
                if (S.has_env && k > 1) {
                    const int tex = env_texel_of(S, d);
                    h.push((uint32_t)tex);
                    const float pp = qf(r, QPPREV, i);
                    const float w = pp / (pp + S.texpdf[tex]);
                    const V3 c = mul(beta, env_rgb(S, tex)) * w;
                    float* L = q.L + 3 * (size_t)pq;
                    L[0] += c.x; L[1] += c.y; L[2] += c.z;
                }
                if (hashing) final_hash(p, r, i, h.h);
            } else if (k > p.B) {
                if (hashing) final_hash(p, r, i, h.h);
            } else if (k == 1 && (vd >> 16) == 1u && qld(q.hf + (i ^ 1)) == f) {
                // the two side rays of a primary edge sample (queue slots 2j and
                // 2j + 1 at bounce 1) met the same face first: the edge point is
                // hidden behind it, there is no jump to measure, and both side
                // paths end here with zero radiance
                if (hashing) final_hash(p, r, i, h.h);
            } else {
                const V3 o = k == 1 ? ld3(p.cams[vd & 0xFFFFu].eye) : V3{qf(r, QOX, i), qf(r, QOY, i), qf(r, QOZ, i)};
                x = o + d * qld(q.ht + i);
                V3 n = xyz(S.fnorm[f]);
                const V3 wo = -d;
                if (dot(n, wo) < 0.0f) n = -n;
                const int tx = texel_of(S, f, x);
                if (S.tex_res) h.push((uint32_t)tx);
                const Mat m = load_mat(S.mat + 7 * (size_t)tx);
                for (int l = 0; l < S.nl; ++l) {
                    const float* lt = S.lights + 6 * l;
                    const V3 dl = ld3(lt) - x;
                    const float r2 = dot(dl, dl);
                    float tmax = -1.0f;
                    V3 wl{0.f, 0.f, 0.f}, ct{0.f, 0.f, 0.f};
                    if (r2 > 0.0f) {
                        const float rr = sqrtf(r2);
                        wl = dl * (1.0f / rr);
                        const float c = dot(n, wl);
                        if (c > 0.0f) {
                            tmax = rr * (1.0f - SHADOW_SHRINK);
                            ct = mul(beta, mul(ld3(lt + 3), brdf_eval(wl, wo, n, m))) * (c / r2);
                        }
                    }
                    // an entry is read only when it carries a ray (listed for k_shadow;
                    // k_shadow_sum reads the contribution of an unoccluded one)
                    const size_t e = (size_t)l * q.cap + i;
                    if (tmax >= 0.0f) {
                        qst(q.sh[0] + e, wl.x); qst(q.sh[1] + e, wl.y); qst(q.sh[2] + e, wl.z); qst(q.sh[3] + e, tmax);
                        qst(q.sh[4] + e, ct.x); qst(q.sh[5] + e, ct.y); qst(q.sh[6] + e, ct.z);
                        rays |= 1u << l;
                    } else if (!fused) {
                        q.socc[e] = 0;
                    }
                }
                int tex = 0;
                if (S.has_env) {
                    const float4 u = draw4(ctr, k, 1, key);
                    V3 we; float pe;
                    tex = env_sample(S, u, we, pe);
                    const float c = dot(n, we);
                    float tmax = -1.0f;
                    V3 ct{0.f, 0.f, 0.f};
                    if (c > 0.0f && pe > 0.0f) {
                        tmax = __int_as_float(0x7f800000);
                        const float den = pe + bsdf_pdf(we, wo, n, m.a, S.vndf);
                        ct = mul(beta, mul(env_rgb(S, tex), brdf_eval(we, wo, n, m))) * (c / den);
                    }
                    const size_t e = (size_t)S.nl * q.cap + i;
                    if (tmax >= 0.0f) {
                        qst(q.sh[0] + e, we.x); qst(q.sh[1] + e, we.y); qst(q.sh[2] + e, we.z); qst(q.sh[3] + e, tmax);
                        qst(q.sh[4] + e, ct.x); qst(q.sh[5] + e, ct.y); qst(q.sh[6] + e, ct.z);
                        rays |= 1u << S.nl;
                    } else if (!fused) {
                        q.socc[e] = 0;
                    }
                }
                uint32_t info = 0;
                if (k < p.B || S.has_env) {
                    const float4 u = draw4(ctr, k, 2, key);
                    const int lobe = bsdf_sample(u, wo, n, m.a, S.vndf, wi);
                    const float ci = dot(n, wi);
                    pb = bsdf_pdf(wi, wo, n, m.a, S.vndf);
                    info = 1u | ((uint32_t)lobe << 1);
                    if (ci > 0.0f && pb > 0.0f) {
                        info |= 4u;
                        emit = true;
                        beta = mul(beta, brdf_eval(wi, wo, n, m)) * (ci / pb);
                    }
                }
                // the shading record: the shadow rays' origin and excluded face (fused:
                // read only through the listed entries)
                if (!fused || rays) {
                    qst(q.sface + i, f);
                    qst(q.sx[0] + i, x.x); qst(q.sx[1] + i, x.y); qst(q.sx[2] + i, x.z);
                }
                if (!fused) q.sinfo[i] = info;
                if (shadow_fused(p, q) && p.rec_occ && (vd >> 16) == 0u)
                    p.rec_occ[(size_t)(k - 1) * p.rec_n + pq] = 0u;
                if (!fused) q.stex[i] = tex;
                if (!fused) q.snext[i] = -1;
            }
            hv = h.h;
        }
        // compaction of the continuing paths into the next queue, and of the
        // shadow entries that carry a ray (those of one shading point
        // consecutive) into the shadow list of this bounce
        const int2 oo = block_reserve2<SHADE_BLOCK>(emit, __popc(rays), &q.cnt[k + 1], &q.cnt[32 + k], resv);
        const int o = oo.x;
        // the next queue holds one continuation per path of the chunk and the
        // shadow list nent entries per shading point, so this never trips; a
        // reservation past either is reported (ST_ERR_QUEUE_OVERFLOW), not written
        if ((emit && o >= q.cap) || (rays && (long long)oo.y + __popc(rays) > (long long)q.cap * max(q.nent, 1))) {
            atomicOr(p.err, ERR_QUEUE);
            emit = false;
            rays = 0;
        }
        for (int so = oo.y; rays; rays &= rays - 1, ++so)
            qst(q.slist + so, (uint32_t)(__ffs(rays) - 1) * (uint32_t)q.cap + (uint32_t)i);
        {
            if (emit) {
                qf_st(rn, QOX, o, x.x); qf_st(rn, QOY, o, x.y); qf_st(rn, QOZ, o, x.z);
                qf_st(rn, QDX, o, wi.x); qf_st(rn, QDY, o, wi.y); qf_st(rn, QDZ, o, wi.z);
                qu_st(rn, QEXCL, o, (uint32_t)f);
                qf_st(rn, QPPREV, o, pb);
                qu_st(rn, QQ, o, pq);
                qu_st(rn, QC0, o, c0);
                qu_st(rn, QC1, o, c1);
                qu_st(rn, QVD, o, vd);
                qf_st(rn, QBR, o, beta.x); qf_st(rn, QBG, o, beta.y); qf_st(rn, QBB, o, beta.z);
                if (hashing) qu_st(rn, QHASH, o, hv);
                if (!fused) q.snext[i] = o;
            }
        }
        if (active && hashing) qu(r, QHASH, i) = hv;
    }
}

// shadow ray w of the list of bounce k: occlusion code, or (fused) the
// unoccluded contribution added and the occlusion recorded
__device__ __forceinline__ void shadow_one(const FwdParams& p, const Queues& q, int k, float* const* r, int w,
                                           bool fused, TravStack& st) {
    const uint32_t e = qld(q.slist + w);
    const int i = (int)(e % (uint32_t)q.cap);
    const int f = qld(q.sface + i);
    const DevScene& S = p.scenes[p.cams[qu_ld(r, QVD, i) & 0xFFFFu].scene];
    const float tmax = qld(q.sh[3] + e);
    const V3 o{qld(q.sx[0] + i), qld(q.sx[1] + i), qld(q.sx[2] + i)}, dd{qld(q.sh[0] + e), qld(q.sh[1] + e), qld(q.sh[2] + e)};
    const bool occluded = trace_any(S, o, dd, TMIN, tmax, f, st);
    if (fused) {
        if (occluded) {
            if (p.rec_occ && (qu_ld(r, QVD, i) >> 16) == 0u) p.rec_occ[(size_t)(k - 1) * p.rec_n + qu_ld(r, QQ, i)] = 1u;
        } else {
            float* L = q.L + 3 * (size_t)qu_ld(r, QQ, i);
            L[0] += qld(q.sh[4] + e); L[1] += qld(q.sh[5] + e); L[2] += qld(q.sh[6] + e);
        }
    } else {
        q.socc[e] = occluded ? 1 : 2;
    }
}

// shadow rays of bounce k: the entries listed by k_shade (entry l of shading
// point i is l * cap + i), one outcome code each (1 occluded, 2 unoccluded);
// k_shade wrote 0 (no ray) for the others
__global__ void __launch_bounds__(TRACE_BLOCK) SHADOW_OCC k_shadow(FwdParams p, Queues q, int k) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    TravStack st = make_trav_stack(lds, q.spill, p.err, p.work ? p.work + 3 * WORK_SHADOW : nullptr);
    const int items = q.cnt[32 + k];
    float* const* r = q.ray[k & 1];
    if (ST_SHADOW_QUEUE) {
        // persistent waves refilled from the fetch counters of slot k
        trace_queue<true>(
            q.fetch + FETCH_SLOT_INTS * k, items, st,
            [&](int w, RayJob& J) {
                const uint32_t e = q.slist[w];
                const int i = (int)(e % (uint32_t)q.cap);
                const DevScene& S = p.scenes[p.cams[qu_ld(r, QVD, i) & 0xFFFFu].scene];
                J.o = V3{q.sx[0][i], q.sx[1][i], q.sx[2][i]};
                J.d = V3{q.sh[0][e], q.sh[1][e], q.sh[2][e]};
                J.tmax = q.sh[3][e];
                J.excl = q.sface[i];
                J.G = trace_geo(S);
                return true;
            },
            [&](int w, int occ, float) { q.socc[q.slist[w]] = occ ? 1 : 2; });
        return;
    }
    const bool fused = shadow_fused(p, q);
    // 64 consecutive listed rays per wave, traced in lockstep
    const int stride = gridDim.x * blockDim.x;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < items; w += stride) shadow_one(p, q, k, r, w, fused, st);
}

// One launch for the extension rays of bounce k + 1 and the shadow rays of
// bounce k: both start at the shading points of bounce k and neither reads
// what the other writes (hits of the next queue; radiance, occlusion records
// or outcome codes of this bounce), so the two traversals share one grid and
// one drain at the end instead of two.  Waves take the listed shadow rays first
// (their count rounded up to whole waves), then the extension rays (this order
// measured 0.7 ms faster per step than the other).
__global__ void __launch_bounds__(TRACE_BLOCK) EXTEND_OCC k_trace_pair(FwdParams p, Queues q, int k) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    TravStack st = make_trav_stack(lds, q.spill, p.err, nullptr);
    st.work2 = p.work ? p.work + 3 * WORK_PAIR : nullptr;
    unsigned long long* const wext = p.work ? p.work + 3 * WORK_EXTEND : nullptr;
    unsigned long long* const wsh = p.work ? p.work + 3 * WORK_SHADOW : nullptr;
    const int n = q.cnt[k + 1];
    const int items = q.cnt[32 + k];
    float* const* rn = q.ray[(k + 1) & 1];
    float* const* r = q.ray[k & 1];
    const bool fused = shadow_fused(p, q);
    // unsigned: with many lights the two counts together can pass 2^31 (each is
    // below 2^31, the grid below 2^21, so the sum and the next index fit 32 bits)
    const uint32_t s64 = ((uint32_t)items + 63u) & ~63u;
    const uint32_t stride = gridDim.x * blockDim.x, all = s64 + (uint32_t)n;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < all; i += stride) {
        if (i < s64) {
            if (i < (uint32_t)items) {
                st.work = wsh;
                shadow_one(p, q, k, r, (int)i, fused, st);
            }
        } else {
            st.work = wext;
            extend_one(p, q, k + 1, rn, (int)(i - s64), st);
        }
    }
}

// shadow contributions of bounce k added per shading point in entry order
__global__ void k_shadow_sum(FwdParams p, Queues q, int k) {
    const int n = q.cnt[k];
    float* const* r = q.ray[k & 1];
    float* const* rn = q.ray[(k + 1) & 1];
    const int stride = gridDim.x * blockDim.x;
    const bool hashing = p.dbg_hash || p.hash_by_q;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int f = q.sface[i];
        if (f < 0) continue;
        const DevScene& S = p.scenes[p.cams[qu(r, QVD, i) & 0xFFFFu].scene];
        Hash h{hashing ? qu(r, QHASH, i) : 0u, hashing};
        V3 acc{0.f, 0.f, 0.f};
        const int nent = S.nl + (S.has_env ? 1 : 0);
        uint32_t occ = 0;
        for (int l = 0; l < nent; ++l) {
            const size_t e = (size_t)l * q.cap + i;
            if (l == S.nl) h.push((uint32_t)q.stex[i]);
            const uint32_t code = q.socc[e];
            if (code == 2u) acc = acc + V3{q.sh[4][e], q.sh[5][e], q.sh[6][e]};
            if (code == 1u) occ |= 1u << l;
            h.push(code);
        }
        if (p.rec_occ && (qu(r, QVD, i) >> 16) == 0u) p.rec_occ[(size_t)(k - 1) * p.rec_n + qu(r, QQ, i)] = occ;
        const uint32_t info = q.sinfo[i];
        if (info & 1u) {
            h.push((info >> 1) & 1u);
            h.push((info >> 2) & 1u);
        }
        float* L = q.L + 3 * (size_t)qu(r, QQ, i);
        L[0] += acc.x; L[1] += acc.y; L[2] += acc.z;
        if (hashing) {
            const int o = q.snext[i];
            if (o >= 0) qu(rn, QHASH, o) = h.h;
            else final_hash(p, r, i, h.h);
        }
    }
}

// single-kernel forward (one thread per path sample); same estimator
__global__ void __launch_bounds__(TRACE_BLOCK) k_forward_mega(FwdParams p, float* L, long long total,
                                                              uint32_t* spill) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    TravStack st = make_trav_stack(lds, spill, p.err, p.work ? p.work + 3 * WORK_MEGA : nullptr);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long qq = blockIdx.x * (long long)blockDim.x + threadIdx.x; qq < total; qq += stride) {
        const int v = find_view(p.qoff, p.ncam, qq);
        const DevCam& c = p.cams[v];
        const DevScene& S = p.scenes[c.scene];
        int x, y, j;
        decode_path(c, qq - c.qoff, p.spp, x, y, j);
        const Ctr ctr{(uint32_t)(y * c.W + x), ((uint32_t)c.rngview << 16) | (uint32_t)j, 0u, 0u};
        const Key key{p.seed, S.scene_id};
        const float4 u = draw4(ctr, 0, 0, key);
        const V3 d = cam_dir(c, (float)x + u.x, (float)y + u.y);
        Hash h{FNV_INIT, true};
        const V3 r = trace_estimator(S, ld3(c.eye), d, -1, p.B, false, ctr, key, h, st);
        L[3 * qq] = r.x; L[3 * qq + 1] = r.y; L[3 * qq + 2] = r.z;
        if (p.dbg_hash) p.dbg_hash[canon(c, x, y, j, p.spp)] = h.h;
    }
}

// film: average the spp samples of each pixel in sample order
__global__ void k_film(const DevCam* __restrict__ cams, const long long* __restrict__ pixoff, int ncam, int spp,
                       const float* __restrict__ L, long long npix, float* out, uint32_t* err,
                       unsigned long long* key_dev, unsigned long long key) {
    if (key_dev && blockIdx.x == 0 && threadIdx.x == 0) *key_dev = key;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < npix; g += stride) {
        const int v = find_view(pixoff, ncam, g);
        const DevCam& c = cams[v];
        const int p = (int)(g - c.pixoff);
        const int x = p % c.W, y = p / c.W;
        int pt;
        if ((c.W & 7) == 0 && (c.H & 7) == 0) pt = (((y >> 3) * (c.W >> 3) + (x >> 3)) << 6) | ((y & 7) << 3) | (x & 7);
        else pt = p;
        const long long hw = (long long)c.W * c.H;
        float a = 0.f, b = 0.f, cc = 0.f;
        for (int j = 0; j < spp; ++j) {
            const long long qq = c.qoff + (long long)j * hw + pt;
            a += qld(L + 3 * qq); b += qld(L + 3 * qq + 1); cc += qld(L + 3 * qq + 2);
        }
        const float inv = 1.0f / (float)spp;
        out[3 * g] = a * inv; out[3 * g + 1] = b * inv; out[3 * g + 2] = cc * inv;
        if (!isfinite(a + b + cc)) atomicOr(err, ERR_NAN);
    }
}

// per-sample radiance in canonical order (debug output)
__global__ void k_sample_radiance(FwdParams p, const float* __restrict__ L, long long total, float* out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long qq = blockIdx.x * (long long)blockDim.x + threadIdx.x; qq < total; qq += stride) {
        const int v = find_view(p.qoff, p.ncam, qq);
        const DevCam& c = p.cams[v];
        int x, y, j;
        decode_path(c, qq - c.qoff, p.spp, x, y, j);
        const long long g = canon(c, x, y, j, p.spp);
        out[3 * g] = L[3 * qq]; out[3 * g + 1] = L[3 * qq + 1]; out[3 * g + 2] = L[3 * qq + 2];
    }
}

__global__ void k_fill_f32(float* p, long long n, float v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, long long n, uint32_t v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// closest hit of caller-given rays (BVH, or brute force over all faces)
__global__ void __launch_bounds__(TRACE_BLOCK) k_trace_debug(const DevScene* sc, const float* o, const float* d,
                                                             int n, float tmin, int brute, int* of, float* ot,
                                                             uint32_t* spill, uint32_t* err) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    const DevScene& S = *sc;
    TravStack st = make_trav_stack(lds, spill, err, nullptr);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const V3 oo = ld3(o + 3 * i), dd = ld3(d + 3 * i);
    float tb = __int_as_float(0x7f800000);
    int fb = -1;
    if (brute) {
        for (int l = 0; l < S.nf; ++l) {
            float t; int f;
            if (tri_test((const gfloat4*)S.tri, (uint32_t)l, oo, dd, tmin, __int_as_float(0x7f800000), t, f))
                if (t < tb || (t == tb && f < fb)) { tb = t; fb = f; }
        }
    } else {
        fb = trace_closest(S, oo, dd, tmin, -1, tb, st);
    }
    of[i] = fb;
    ot[i] = tb;
}

// ---------------------------------------------------------------------------
static inline unsigned grid_for(long long n, int bs, unsigned cap) {
    long long g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (unsigned)(g < (long long)cap ? g : cap);
}


void launch_forward_wavefront(const FwdParams& p, Queues& q, long long total, int has_env_any, int nent,
                              hipStream_t st) {
    q.nent = nent;
    for (long long q0 = 0; q0 < total; q0 += q.cap) {
        const int n = (int)((total - q0) < q.cap ? (total - q0) : q.cap);
        ST_LAUNCH("k_camera", k_camera, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, st, p, q, q0, n);
        launch_wavefront_bounces(p, q, n, has_env_any, st);
    }
}

// extension / shading / shadow kernels of every bounce for a chunk whose first
// ray queue (queue 1) and count cnt[1] have been filled; n bounds the count
void launch_wavefront_bounces(const FwdParams& p, Queues& q, int n, int has_env_any, hipStream_t st,
                              LaunchHook* hook) {
    const unsigned gmax = (q.grid > 0 && (unsigned)q.grid < TRACE_GRID) ? (unsigned)q.grid : TRACE_GRID;
    const unsigned g = grid_for(n, TRACE_BLOCK, gmax);
    const int last = p.B + (has_env_any ? 1 : 0);
    const bool fused = shadow_fused(p, q);
    ST_LAUNCH("k_extend", k_extend, dim3(g), dim3(TRACE_BLOCK), 0, st, p, q, 1);
    if (hook) hook->tick();
    for (int k = 1; k <= last; ++k) {
        // bounce k is traced: shade it, then trace its shadow rays together with
        // the extension rays of bounce k + 1
        if (p.dbg_hash || p.hash_by_q)
            ST_LAUNCH("k_shade", k_shade<true>, dim3(grid_for(n, SHADE_BLOCK, gmax)), dim3(SHADE_BLOCK), 0, st, p, q, k);
        else
            ST_LAUNCH("k_shade", k_shade<false>, dim3(grid_for(n, SHADE_BLOCK, gmax)), dim3(SHADE_BLOCK), 0, st, p, q, k);
        if (hook) hook->tick();
        const bool shadow = k <= p.B, next = k < last;
        if (ST_PAIR_TRACE && shadow && next) {
            ST_LAUNCH("k_trace_pair", k_trace_pair, dim3(g), dim3(TRACE_BLOCK), 0, st, p, q, k);
            if (hook) hook->tick();
        } else {
            if (shadow) {
                ST_LAUNCH("k_shadow", k_shadow, dim3(g), dim3(TRACE_BLOCK), 0, st, p, q, k);
                if (hook) hook->tick();
            }
            if (next) {
                ST_LAUNCH("k_extend", k_extend, dim3(g), dim3(TRACE_BLOCK), 0, st, p, q, k + 1);
                if (hook) hook->tick();
            }
        }
        if (shadow && !fused)
            ST_LAUNCH("k_shadow_sum", k_shadow_sum, dim3(grid_for(n, 256, gmax)), dim3(256), 0, st, p, q, k);
    }
}

void launch_forward_mega(const FwdParams& p, float* L, long long total, uint32_t* spill, int grid,
                         hipStream_t st) {
    ST_LAUNCH("k_forward_mega", k_forward_mega, dim3(grid_for(total, TRACE_BLOCK, grid)), dim3(TRACE_BLOCK), 0, st, p, L,
                       total, spill);
}

void launch_film(const DevCam* cams, const long long* pixoff, int ncam, int spp, const float* L, long long npix,
                 float* out, uint32_t* err, hipStream_t st, unsigned long long* key_dev, unsigned long long key) {
    ST_LAUNCH("k_film", k_film, dim3(grid_for(npix, 256, 1u << 16)), dim3(256), 0, st, cams, pixoff, ncam, spp, L,
                       npix, out, err, key_dev, key);
}

void launch_sample_radiance(const FwdParams& p, const float* L, long long total, float* out, hipStream_t st) {
    ST_LAUNCH("k_sample_radiance", k_sample_radiance, dim3(grid_for(total, 256, 1u << 16)), dim3(256), 0, st, p, L, total,
                       out);
}

void launch_fill_f32(float* ptr, long long n, float v, hipStream_t st) {
    if (n > 0) ST_LAUNCH("k_fill_f32", k_fill_f32, dim3(grid_for(n, 256, 1u << 16)), dim3(256), 0, st, ptr, n, v);
}
// non-finite values among a[0..na) and b[0..nb) set ERR_NAN
__global__ void k_check_finite(const float* __restrict__ a, long long na, const float* __restrict__ b, long long nb,
                               uint32_t* err) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < na + nb; i += stride)
        bad |= !isfinite(i < na ? a[i] : b[i - na]);
    if (__ballot(bad) && __lane_id() == 0) atomicOr(err, ERR_NAN);
}

void launch_check_finite(const float* a, long long na, const float* b, long long nb, uint32_t* err, hipStream_t st) {
    if (na + nb > 0)
        ST_LAUNCH("k_check_finite", k_check_finite, dim3(grid_for(na + nb, 256, 1u << 12)), dim3(256), 0, st, a, na, b,
                  nb, err);
}

// streaming copy of n 16-byte words (the achievable-bandwidth reference of the
// measurements): each thread moves 4 words per step with non-temporal loads and
// stores, consecutive lanes on consecutive words
__global__ void __launch_bounds__(256) k_stream_copy(vf4* __restrict__ dst, const vf4* __restrict__ src, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const vf4 a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride);
        const vf4 c = __builtin_nontemporal_load(src + i + 2 * stride), d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

void launch_stream_copy(float4* dst, const float4* src, long long n, hipStream_t st) {
    if (n > 0)
        ST_LAUNCH("k_stream_copy", k_stream_copy, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, (vf4*)dst,
                  (const vf4*)src, n);
}

// up to WORD_CHUNK words passed by value (so a captured launch carries its own
// copy) written to dst
constexpr int WORD_CHUNK = 480;
struct WordChunk {
    uint32_t n;
    uint32_t w[WORD_CHUNK];
};
__global__ void k_put_words(uint32_t* dst, WordChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

void launch_put_words(uint32_t* dst, const uint32_t* src, size_t nwords, hipStream_t st) {
    for (size_t i = 0; i < nwords; i += WORD_CHUNK) {
        WordChunk c;
        c.n = (uint32_t)(nwords - i < (size_t)WORD_CHUNK ? nwords - i : (size_t)WORD_CHUNK);
        for (uint32_t j = 0; j < c.n; ++j) c.w[j] = src[i + j];
        ST_LAUNCH("k_put_words", k_put_words, dim3(1), dim3(256), 0, st, dst + i, c);
    }
}

__global__ void k_put_u64(unsigned long long* p, unsigned long long v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

void launch_put_u64(unsigned long long* ptr, unsigned long long v, hipStream_t st) {
    ST_LAUNCH("k_put_u64", k_put_u64, dim3(1), dim3(64), 0, st, ptr, v);
}

void launch_fill_u32(uint32_t* ptr, long long n, uint32_t v, hipStream_t st) {
    if (n > 0) ST_LAUNCH("k_fill_u32", k_fill_u32, dim3(grid_for(n, 256, 1u << 16)), dim3(256), 0, st, ptr, n, v);
}

void launch_trace_debug(const DevScene* s, const float* o, const float* d, int n, float tmin, int brute,
                        int* out_face, float* out_t, uint32_t* spill, uint32_t* err, hipStream_t st) {
    if (n > 0)
        ST_LAUNCH("k_trace_debug", k_trace_debug, dim3((n + TRACE_BLOCK - 1) / TRACE_BLOCK), dim3(TRACE_BLOCK), 0, st, s, o,
                           d, n, tmin, brute, out_face, out_t, spill, err);
}

} // namespace st

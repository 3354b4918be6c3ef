// Adjoint of the path tracer (Shape from Tracing, Sec. 3.2: gradients of the
// rendered pixels with respect to vertex positions, and Sec. 3.3 per-facet
// materials; the edge-sampled visibility terms follow the renderer the paper
// cites for geometry gradients).
//
// Interior term: every path sample is replayed from its Philox counters (no
// state is kept from the forward pass), its at most B vertices are recorded in
// registers, and a reverse sweep differentiates the estimator at fixed sampled
// directions with pdfs, MIS weights and visibility held constant; hit points
// move with the hit face's vertices and the previous vertex, point-light
// directions move with the hit point.
//
// Secondary edges: at each vertex one mesh edge is drawn in proportion to its
// length; if it is a silhouette seen from the shading point, two side rays
// bracket it and the jump of incoming radiance times the normal velocity of
// the edge on the sphere of directions is scattered to the edge endpoints and
// to the shading point.
//
// Primary edges: per view, edges are drawn in proportion to their projected
// length (candidates: boundary edges and edges with a front-facing face), a
// point on the edge gets two side camera paths, and the radiance jump times the
// screen-space normal velocity is scattered to the two endpoints.
#include "st_internal.h"

namespace st {


template <class T, int N> __device__ __forceinline__ T sel(const T (&a)[N], int k) {
    T r = a[0];
#pragma unroll
    for (int i = 1; i < N; ++i)
        if (i == k) r = a[i];
    return r;
}
template <class T, int N> __device__ __forceinline__ void put(T (&a)[N], int k, const T& v) {
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i == k) a[i] = v;
}

// Per-vertex records of a path replay, in a per-thread region of global memory:
// slot s of thread g at base[s * gstride + g] (a wave's 64 threads in 256
// consecutive bytes).  As private arrays they sat in scratch memory anyway (the
// sweep indexes them by a loop counter), and were cleared for every path; here
// an entry is written only when the replay reaches its vertex and read only
// then.  A field of type T for BM vertices takes BM * W slots from s0 on (W = 3
// for a vector).
struct RecMem {
    float* base;
    size_t gstride, gid;
    __device__ __forceinline__ float& at(int slot) const { return base[(size_t)slot * gstride + gid]; }
};
template <class T, int BM> struct RecField {
    const RecMem* m;
    int s0;
};
template <int BM> __device__ __forceinline__ V3 sel(const RecField<V3, BM>& f, int k) {
    const int s = f.s0 + 3 * k;
    return V3{f.m->at(s), f.m->at(s + 1), f.m->at(s + 2)};
}
template <int BM> __device__ __forceinline__ void put(const RecField<V3, BM>& f, int k, const V3& v) {
    const int s = f.s0 + 3 * k;
    f.m->at(s) = v.x; f.m->at(s + 1) = v.y; f.m->at(s + 2) = v.z;
}
template <int BM> __device__ __forceinline__ float sel(const RecField<float, BM>& f, int k) { return f.m->at(f.s0 + k); }
template <int BM> __device__ __forceinline__ void put(const RecField<float, BM>& f, int k, float v) { f.m->at(f.s0 + k) = v; }
template <class T, int BM> __device__ __forceinline__ T sel(const RecField<T, BM>& f, int k) {
    static_assert(sizeof(T) == 4, "32-bit fields");
    return (T)__float_as_uint(f.m->at(f.s0 + k));
}
template <class T, int BM> __device__ __forceinline__ void put(const RecField<T, BM>& f, int k, const T& v) {
    static_assert(sizeof(T) == 4, "32-bit fields");
    f.m->at(f.s0 + k) = __uint_as_float((uint32_t)v);
}

__device__ __forceinline__ void atomic_add3(float* p, V3 g) {
    atomicAdd(p, g.x);
    atomicAdd(p + 1, g.y);
    atomicAdd(p + 2, g.z);
}

// unnormalised face normal in double, fixed operation order
__device__ __forceinline__ void face_N_d(const DevScene& S, int f, double N[3], double v0[3]) {
#pragma clang fp contract(off)
    const float* a = S.V + 3 * S.F[3 * f];
    const float* b = S.V + 3 * S.F[3 * f + 1];
    const float* c = S.V + 3 * S.F[3 * f + 2];
    const double e1x = (double)b[0] - (double)a[0], e1y = (double)b[1] - (double)a[1], e1z = (double)b[2] - (double)a[2];
    const double e2x = (double)c[0] - (double)a[0], e2y = (double)c[1] - (double)a[1], e2z = (double)c[2] - (double)a[2];
    N[0] = e1y * e2z - e1z * e2y;
    N[1] = e1z * e2x - e1x * e2z;
    N[2] = e1x * e2y - e1y * e2x;
    v0[0] = a[0]; v0[1] = a[1]; v0[2] = a[2];
}

__device__ __forceinline__ bool silhouette(const DevScene& S, int4 E, V3 x) {
#pragma clang fp contract(off)
    if (E.w < 0) return true;
    const double xa[3] = {(double)x.x - (double)S.V[3 * E.x], (double)x.y - (double)S.V[3 * E.x + 1],
                          (double)x.z - (double)S.V[3 * E.x + 2]};
    double N1[3], N2[3], t[3];
    face_N_d(S, E.z, N1, t);
    face_N_d(S, E.w, N2, t);
    const double s1 = N1[0] * xa[0] + N1[1] * xa[1] + N1[2] * xa[2];
    const double s2 = N2[0] * xa[0] + N2[1] * xa[1] + N2[2] * xa[2];
    return (s1 > 0.0) != (s2 > 0.0);
}

constexpr uint32_t R_FLIP = 1u, R_ENV = 2u, R_CONT = 4u, R_ESC = 8u, R_SEC = 16u;

#ifndef ST_FACE_REDUCE
#define ST_FACE_REDUCE 1
#endif
constexpr bool FACE_REDUCE = ST_FACE_REDUCE != 0;   // wave-level reduction of the primary-vertex gradients

// material slots of texel tx on face f (face-major accumulators)
__device__ __forceinline__ float* mat_slots(float* facc, float* macc, bool texels, int f, int tx) {
    return texels ? macc + (size_t)MACC_STRIDE * tx : facc + (size_t)FACC_STRIDE * f + FACC_MAT;
}

// Adds vals to the accumulators of face f (slots 0..8: the three corners) and
// of its texel tx (slots 9..15: the material) with one atomic instruction per
// (texel, wave): every lane stores its 16 values in its own LDS row, then for
// each texel of the wave (one per round, the first pending lane's) the active
// lanes sum the 16 slots over the lanes of that texel (the r-th active lane
// slots r, r + n, ... of n active lanes: one slot each in a full wave) and add
// the sums with one atomic instruction.  Primary hits of a wave are
// neighbouring pixels, so few texels cover most lanes.  Lanes with !has
// contribute nothing; any subset of the wave's lanes may call it together.
// red: this wave's 64 x FACC floats of LDS.
__device__ __forceinline__ void face_reduce_add(bool has, int f, int tx, const float (&vals)[FACC], float* facc,
                                                float* macc, bool texels, float* red) {
    const int lane = (int)__lane_id();
    const uint64_t act = __ballot(true);
    const int nact = __popcll(act);
    const int rank = __popcll(act & lanemask_lt64());
    float4* const row = (float4*)(red + lane * FACC);
#pragma unroll
    for (int j = 0; j < FACC / 4; ++j) row[j] = make_float4(vals[4 * j], vals[4 * j + 1], vals[4 * j + 2], vals[4 * j + 3]);
    // the rows are read by other lanes of this wave: LDS accesses of one wave
    // complete in order; this keeps the compiler from moving the reads up
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    bool pending = has;
    for (;;) {
        const uint64_t m = __ballot(pending);
        if (!m) break;
        const int leader = __ffsll((long long)m) - 1;
        const int lt = __builtin_amdgcn_readlane(tx, leader);
        const int lf = __builtin_amdgcn_readlane(f, leader);
        const bool mine = pending && tx == lt;
        const uint64_t grp = __ballot(mine);
        for (int j = rank; j < FACC; j += nact) {
            float acc = 0.0f;
            for (uint64_t g = grp; g; g &= g - 1) acc += red[(__ffsll((long long)g) - 1) * FACC + j];
            float* const dst = j < FACC_MAT ? facc + (size_t)FACC_STRIDE * lf + j
                                            : mat_slots(facc, macc, texels, lf, lt) + (j - FACC_MAT);
            atomicAdd(dst, acc);
        }
        pending = pending && !mine;
    }
    // the next call rewrites the rows
    __builtin_amdgcn_wave_barrier();
}

// occupancy target of the adjoint (waves per SIMD): the register budget the
// compiler fits it to (4: measured fastest among 3 to 8)
#ifndef ST_ADJ_WAVES
#define ST_ADJ_WAVES 4
#endif
// JOBS = false: one thread per path sample (qq < total).  With p.sec_mask set,
// an accepted secondary edge sample only marks bit k of the path's mask; its
// side paths, its direct term and its pseudo term (propagated back along the
// path) are left to the JOBS = true pass, one thread per marked (path, vertex),
// which replays the path with the interior term off and processes that vertex
// alone.  Accepted samples are rare, so inline they would hold whole waves for
// one lane's side paths; as jobs they fill the lanes.
// RECM > 0: the main pass of a backward that holds the hit records of its
// forward and defers secondary edges, compiled without any traversal (which
// leaves the compiler far fewer values to spill; RECM = 1 also without the
// secondary-edge hierarchy's descent, RECM = 2 with it); it does nothing when
// the records turn out stale on the device, and the RECM = 0 pass launched after
// it then traces (that pass returns at once when the records pass ran).
template <int BM, bool JOBS, int RECM = 0>
__global__ void __launch_bounds__(TRACE_BLOCK) __attribute__((amdgpu_waves_per_eu(ST_ADJ_WAVES)))
k_adjoint(BwdParams p, long long total) {
    constexpr bool REC = RECM > 0;
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    __shared__ float red_s[TRACE_BLOCK / 64][64 * FACC];
    float* const red = red_s[threadIdx.x >> 6];
    TravStack st = make_trav_stack(lds, p.spill, p.err, p.work ? p.work + 3 * WORK_ADJOINT : nullptr);
    const RecMem rm{p.vrec, (size_t)gridDim.x * blockDim.x, (size_t)blockIdx.x * blockDim.x + threadIdx.x};
    const bool want_interior = !JOBS && (p.flags & 1u), want_secondary = p.flags & 4u;
    const bool sec_interior = p.flags & ST_EDGE_SECONDARY_INTERIOR;   // creases / material edges too
    const bool hier = RECM != 1 && (p.flags & ST_EDGE_SECONDARY_HIERARCHY);   // edges from the importance tree
    const bool defer = REC || (!JOBS && p.sec_mask != nullptr);
    // hit records only when they belong to this pass's forward (same on every lane)
    const bool recs = p.rec_face != nullptr && *p.rec_key_dev == p.rec_key;
    if (REC && !recs) return;
    if (!REC && !JOBS && p.rec_split && recs) return;
    const int* const rec_face = recs ? p.rec_face : nullptr;
    const uint32_t* const rec_occ = recs ? p.rec_occ : nullptr;
    const long long stride = (long long)gridDim.x * blockDim.x;
    // the records pass walks the list of paths that have a vertex when it is given
    const bool listed = REC && !JOBS && p.adj_list != nullptr;
    const long long count = JOBS ? (long long)*p.sec_njobs : listed ? (long long)*p.adj_n : total;
    // the main pass gives each XCD consecutive paths (their hits share that XCD's
    // L2: 18.1 -> 15.8 ms); the job pass keeps the hardware order
    const long long b0 = JOBS ? (long long)blockIdx.x : (long long)grid_block();
    for (long long it = b0 * blockDim.x + threadIdx.x; it < count; it += stride) {
        int ksel = -1;
        long long qq = it;
        if (JOBS) {
            const int2 jb = p.sec_jobs[it];
            qq = jb.x;
            ksel = jb.y;
        } else if (listed) {
            qq = (long long)p.adj_list[it];
        }
        const int vw = find_view(p.qoff, p.ncam, qq);
        const DevCam& c = p.cams[vw];
        const DevScene& S = p.scenes[c.scene];
        int x, y, j;
        decode_path(c, qq - c.qoff, p.spp, x, y, j);
        const long long g = (c.pixoff + (long long)y * c.W + x) * p.spp + j;
        if (p.path_mask && !p.path_mask[g]) continue;
        const float* di = p.d_image + 3 * (c.pixoff + (long long)y * c.W + x);
        if (di[0] == 0.0f && di[1] == 0.0f && di[2] == 0.0f) continue;
        const V3 w = V3{di[0], di[1], di[2]} * (1.0f / (float)p.spp);
        const Key key{p.seed, S.scene_id};
        const Ctr ctr{(uint32_t)(y * c.W + x), ((uint32_t)c.rngview << 16) | (uint32_t)j, 0u, 0u};
        const float4 u0 = draw4(ctr, 0, 0, key);
        const V3 d0 = cam_dir(c, (float)x + u0.x, (float)y + u0.y);
        Hash h{FNV_INIT, p.dbg_hash != nullptr};

        // ---- replay, recording each vertex --------------------------------
        // Entries of a vertex are written when the replay reaches it and read only
        // for k < nvtx under the flag that marks them (R_ENV: rwe, rden, rtex;
        // R_CONT: rwi, rpb; R_ESC: resc; R_SEC: rsecm, rsecc; rse >= 0: rte, rsw).
        const RecField<int, BM> rf{&rm, 0}, rtex{&rm, BM}, rse{&rm, 2 * BM};
        const RecField<uint32_t, BM> rfl{&rm, 3 * BM};
        const RecField<V3, BM> rx{&rm, 4 * BM}, rwe{&rm, 7 * BM}, rwi{&rm, 10 * BM}, resc{&rm, 13 * BM},
            rbeta{&rm, 16 * BM}, rsecm{&rm, 19 * BM};
        const RecField<float, BM> rden{&rm, 22 * BM}, rpb{&rm, 23 * BM}, rte{&rm, 24 * BM}, rsecc{&rm, 25 * BM},
            rsw{&rm, 26 * BM};
        int nvtx = 0;
        {
            V3 o = ld3(c.eye), d = d0, beta{1.f, 1.f, 1.f};
            int excl = -1;
            float pprev = 0.0f;
            for (int k = 1; k <= p.B + 1; ++k) {
                float t;
                const size_t ri = (size_t)(k - 1) * p.rec_n + qq;
                int f;
                if (REC || rec_face) {
                    f = qld(rec_face + ri);
                    t = f >= 0 ? face_hit_t(S, f, o, d) : __int_as_float(0x7f800000);
                } else {
                    f = trace_closest(S, o, d, TMIN, excl, t, st);
                }
                push_face(h, f);
                if (f < 0) {
                    if (S.has_env && k > 1) {
                        const int tex = env_texel_of(S, d);
                        h.push((uint32_t)tex);
                        const float wv = pprev / (pprev + S.texpdf[tex]);
                        put(resc, k - 2, env_rgb(S, tex) * wv);
                        put(rfl, k - 2, sel(rfl, k - 2) | R_ESC);
                    }
                    break;
                }
                if (k == p.B + 1) break;
                const V3 xh = o + d * t;
                V3 n = xyz(S.fnorm[f]);
                const V3 wo = -d;
                uint32_t fl = 0;
                if (dot(n, wo) < 0.0f) { n = -n; fl |= R_FLIP; }
                const int tx = texel_of(S, f, xh);
                if (S.tex_res) h.push((uint32_t)tx);
                const Mat m = load_mat(S.mat + 7 * (size_t)tx);
                const uint32_t rocc = (REC || rec_occ) ? qld(rec_occ + ri) : 0u;
                for (int l = 0; l < S.nl; ++l) {
                    const float* lt = S.lights + 6 * l;
                    const V3 dl = ld3(lt) - xh;
                    const float r2 = dot(dl, dl);
                    uint32_t code = 0;
                    if (r2 > 0.0f) {
                        const float rr = sqrtf(r2);
                        const V3 wl = dl * (1.0f / rr);
                        if (dot(n, wl) > 0.0f) {
                            const bool occ = (REC || rec_occ) ? ((rocc >> l) & 1u) != 0u
                                                       : trace_any(S, xh, wl, TMIN, rr * (1.0f - SHADOW_SHRINK), f, st);
                            code = occ ? 1u : 2u;
                            if (!occ) fl |= 1u << (8 + l);
                        }
                    }
                    h.push(code);
                }
                if (S.has_env) {
                    const float4 u = draw4(ctr, k, 1, key);
                    V3 we; float pe;
                    const int tex = env_sample(S, u, we, pe);
                    h.push((uint32_t)tex);
                    const float ce = dot(n, we);
                    uint32_t code = 0;
                    if (ce > 0.0f && pe > 0.0f) {
                        const bool occ = (REC || rec_occ) ? ((rocc >> S.nl) & 1u) != 0u
                                                   : trace_any(S, xh, we, TMIN, __int_as_float(0x7f800000), f, st);
                        code = occ ? 1u : 2u;
                        if (!occ) {
                            fl |= R_ENV;
                            put(rwe, k - 1, we);
                            put(rden, k - 1, pe + bsdf_pdf(we, wo, n, m.a, S.vndf));
                            put(rtex, k - 1, tex);
                        }
                    }
                    h.push(code);
                }
                const bool continues = (k < p.B) || S.has_env;
                put(rse, k - 1, -1);
                if (want_secondary && continues && S.ne > 0 && *S.etotal > 0.0f) {
                    const float4 u = draw4(ctr, k, 3, key);
                    // the edge (-2: the hierarchy found no edge in front of the tangent
                    // plane) and 1 / (density of the edge point per unit length)
                    int e;
                    float wsel;
                    if (hier) {
                        float pe;
                        e = edge_tree_sample(S, xh, n, ctr, k, key, !sec_interior, pe);
                        if (e >= 0) {
                            const int4 Eh = S.edges[e];
                            wsel = len(ld3(S.V + 3 * Eh.y) - ld3(S.V + 3 * Eh.x)) / pe;
                        } else {
                            e = -2;
                            wsel = 0.0f;
                        }
                    } else {
                        e = cdf_guided(S.ecdf, S.ne, S.eguide, S.eglog, (double)u.x);
                        wsel = *S.etotal;
                    }
                    put(rse, k - 1, e);
                    put(rte, k - 1, u.y);
                    put(rsw, k - 1, wsel);
                }
                put(rf, k - 1, f);
                put(rx, k - 1, xh);
                put(rbeta, k - 1, beta);
                nvtx = k;
                if (!continues) { put(rfl, k - 1, fl); break; }
                const float4 u = draw4(ctr, k, 2, key);
                V3 wi;
                const int lobe = bsdf_sample(u, wo, n, m.a, S.vndf, wi);
                const float ci = dot(n, wi);
                const float pb = bsdf_pdf(wi, wo, n, m.a, S.vndf);
                h.push((uint32_t)lobe);
                if (!(ci > 0.0f) || !(pb > 0.0f)) { h.push(0u); put(rfl, k - 1, fl); break; }
                h.push(1u);
                fl |= R_CONT;
                put(rfl, k - 1, fl);
                put(rwi, k - 1, wi);
                put(rpb, k - 1, pb);
                beta = mul(beta, brdf_eval(wi, wo, n, m)) * (ci / pb);
                pprev = pb;
                o = xh; d = wi; excl = f;
            }
        }

        // ---- secondary edge samples (side paths in their own stream) --------
        if (want_secondary) {
            uint32_t accepted = 0;
            for (int k = 0; k < nvtx; ++k) {
                const int e = sel(rse, k);
                if (e == -1 || (JOBS && k != ksel)) continue;
                if (e == -2) { h.push(0xFFFFFFFFu); h.push(0u); continue; }
                h.push((uint32_t)e);
                const int f = sel(rf, k);
                const V3 xh = sel(rx, k);
                const int4 E = S.edges[e];
                const V3 va = ld3(S.V + 3 * E.x), vb = ld3(S.V + 3 * E.y);
                const float te = sel(rte, k);
                const V3 yv = va + (vb - va) * te;
                const V3 wv = yv - xh;
                const float r2 = dot(wv, wv);
                // an edge of the shading face lies in the tangent plane: never a silhouette
                bool ok = E.z != f && E.w != f && (sec_interior || silhouette(S, E, xh)) && r2 > 0.0f;
                V3 n = xyz(S.fnorm[f]);
                if (sel(rfl, k) & R_FLIP) n = -n;
                V3 ud{0.f, 0.f, 0.f}, mv{0.f, 0.f, 0.f};
                float cv = 0.0f, ml = 0.0f;
                if (ok) {
                    ud = wv * (1.0f / sqrtf(r2));
                    cv = dot(n, ud);
                    mv = cross(ud, normalize(vb - va));
                    ml = len(mv);
                    ok = cv > SEC_COS_MIN && ml > 0.0f;
                }
                if (!ok) { h.push(0u); continue; }
                h.push(1u);
                if (defer) { accepted |= 1u << k; continue; }
                const V3 mm = mv * (1.0f / ml);
                const Ctr sc{ctr.c0, ctr.c1, (uint32_t)(k + 1) << 16, 2u};
                V3 Ls[2];
                for (int side = 0; side < 2; ++side) {
                    const V3 dir = normalize(ud + mm * (side == 0 ? -EPS_SECONDARY : EPS_SECONDARY));
                    Ls[side] = trace_estimator(S, xh, dir, f, p.B - (k + 1), true, sc, key, h, st);
                }
                const V3 dirk = k == 0 ? d0 : sel(rwi, k - 1);
                const Mat m = load_mat(S.mat + 7 * (size_t)texel_of(S, f, xh));
                const V3 fv = brdf_eval(ud, -dirk, n, m);
                const float cc = dot(mul(w, mul(sel(rbeta, k), fv)), Ls[0] - Ls[1]) * cv * (sel(rsw, k) / r2);
                put(rsecc, k, cc);
                put(rsecm, k, mv);
                put(rfl, k, sel(rfl, k) | R_SEC);
                atomic_add3(p.dV + 3 * (size_t)E.x, mv * (cc * (1.0f - te)));
                atomic_add3(p.dV + 3 * (size_t)E.y, mv * (cc * te));
            }
            if (defer && accepted) p.sec_mask[qq] = (uint8_t)accepted;
        }

        // ---- reverse sweep ------------------------------------------------
        // every lane runs BM rounds so that the primary vertices (k = 0) of
        // the wave are accumulated together
        {
            V3 Snext{0.f, 0.f, 0.f}, gxnext{0.f, 0.f, 0.f};
            for (int k = BM - 1; k >= 0; --k) {
                float vals[FACC];
                const bool has = k < nvtx;
                const int f = has ? sel(rf, k) : -1;
                const int tx = has ? texel_of(S, f, sel(rx, k)) : -1;
                if (has) {
                    const uint32_t fl = sel(rfl, k);
                    const V3 xh = sel(rx, k);
                    const V3 dir = k == 0 ? d0 : sel(rwi, k - 1);
                    const V3 wo = -dir;
                    const int i0 = S.F[3 * f], i1 = S.F[3 * f + 1], i2 = S.F[3 * f + 2];
                    const V3 v0 = ld3(S.V + 3 * i0), v1 = ld3(S.V + 3 * i1), v2 = ld3(S.V + 3 * i2);
                    const V3 e1 = v1 - v0, e2 = v2 - v0;
                    const V3 N = cross(e1, e2);
                    const float Nl = len(N);
                    const V3 nu = N * (1.0f / Nl);
                    const float sg = (fl & R_FLIP) ? -1.0f : 1.0f;
                    const V3 n = nu * sg;
                    const Mat m = load_mat(S.mat + 7 * (size_t)tx);
                    const V3 a = want_interior ? mul(w, sel(rbeta, k)) : V3{0.f, 0.f, 0.f};
                    V3 C{0.f, 0.f, 0.f}, gn{0.f, 0.f, 0.f}, gx = gxnext, gdummy{0.f, 0.f, 0.f};
                    float gm[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    for (int l = 0; l < S.nl; ++l) {
                        if (!((fl >> (8 + l)) & 1u)) continue;
                        const float* lt = S.lights + 6 * l;
                        const V3 I = ld3(lt + 3);
                        const V3 dl = ld3(lt) - xh;
                        const float r2 = dot(dl, dl);
                        const float rr = sqrtf(r2);
                        const V3 wl = dl * (1.0f / rr);
                        const float cl = dot(n, wl);
                        const V3 fv = brdf_eval(wl, wo, n, m);
                        const V3 If = mul(I, fv);
                        C = C + If * (cl / r2);
                        const V3 aI = mul(a, I);
                        const float gcl = dot(aI, fv) / r2;
                        const float gr2 = -dot(aI, fv) * cl / (r2 * r2);
                        V3 gwl{0.f, 0.f, 0.f};
                        brdf_backward(wl, wo, n, m, aI * (cl / r2), gn, gwl, gm);
                        gn = gn + wl * gcl;
                        gwl = gwl + n * gcl;
                        const V3 gd = (gwl - wl * dot(wl, gwl)) * (1.0f / rr) + dl * (2.0f * gr2);
                        gx = gx - gd;
                    }
                    if (fl & R_ENV) {
                        const V3 we = sel(rwe, k);
                        const float den = sel(rden, k);
                        const V3 Le = env_rgb(S, sel(rtex, k));
                        const float ce = dot(n, we);
                        const V3 fv = brdf_eval(we, wo, n, m);
                        C = C + mul(Le, fv) * (ce / den);
                        const V3 aL = mul(a, Le);
                        brdf_backward(we, wo, n, m, aL * (ce / den), gn, gdummy, gm);
                        gn = gn + we * (dot(aL, fv) / den);
                    }
                    V3 Sk = C;
                    if (fl & R_CONT) {
                        const V3 wi = sel(rwi, k);
                        const float pb = sel(rpb, k);
                        const V3 S1 = (fl & R_ESC) ? sel(resc, k) : Snext;
                        const float ci = dot(n, wi);
                        const V3 fv = brdf_eval(wi, wo, n, m);
                        const V3 uu = mul(a, S1);
                        brdf_backward(wi, wo, n, m, uu * (ci / pb), gn, gdummy, gm);
                        gn = gn + wi * (dot(uu, fv) / pb);
                        Sk = Sk + mul(fv, S1) * (ci / pb);
                    }
                    if (fl & R_SEC) gx = gx - sel(rsecm, k) * sel(rsecc, k);
                    // normal n = sg * N / |N|
                    const V3 gnu = gn * sg;
                    V3 gN = (gnu - nu * dot(nu, gnu)) * (1.0f / Nl);
                    // hit point x = o + t dir, t = ((v0 - o) . N) / (dir . N)
                    const float dN = dot(dir, N);
                    const float gt = dot(gx, dir) / dN;
                    const V3 go = gx - N * gt;
                    V3 gv0 = N * gt;
                    gN = gN + (v0 - xh) * gt;
                    const V3 ge1 = cross(e2, gN), ge2 = cross(gN, e1);
                    gv0 = gv0 - ge1 - ge2;
                    vals[0] = gv0.x; vals[1] = gv0.y; vals[2] = gv0.z;
                    vals[3] = ge1.x; vals[4] = ge1.y; vals[5] = ge1.z;
                    vals[6] = ge2.x; vals[7] = ge2.y; vals[8] = ge2.z;
    #pragma unroll
                    for (int i = 0; i < 7; ++i) vals[9 + i] = want_interior ? gm[i] : 0.0f;
                    Snext = Sk;
                    gxnext = go;
                }
                if (k == 0 && FACE_REDUCE) {
                    face_reduce_add(has, f, tx, vals, p.facc, p.macc, S.tex_res > 0, red);
                } else if (has) {
                    float* const fa = p.facc + (size_t)FACC_STRIDE * f;
                    float* const ma = mat_slots(p.facc, p.macc, S.tex_res > 0, f, tx);
#pragma unroll
                    for (int j = 0; j < 9; ++j) atomicAdd(fa + j, vals[j]);
#pragma unroll
                    for (int j = 0; j < 7; ++j) atomicAdd(ma + j, vals[9 + j]);
                }
            }
        }
        if (p.dbg_hash) p.dbg_hash[g] = h.h;
    }
}

// ---------------------------------------------------------------------------
// primary edges
// ---------------------------------------------------------------------------
__device__ __forceinline__ void project_d(const DevCam& c, double vx, double vy, double vz, double& sx, double& sy,
                                          double& z) {
#pragma clang fp contract(off)
    const double px = vx - c.deye[0], py = vy - c.deye[1], pz = vz - c.deye[2];
    z = px * c.df[0] + py * c.df[1] + pz * c.df[2];
    const double a = px * c.dr[0] + py * c.dr[1] + pz * c.dr[2];
    const double b = px * c.du[0] + py * c.du[1] + pz * c.du[2];
    sx = (a / (z * (c.dth * c.daspect)) + 1.0) * (0.5 * c.W);
    sy = (1.0 - b / (z * c.dth)) * (0.5 * c.H);
}

__device__ __forceinline__ bool front_facing_d(const DevScene& S, int f, const DevCam& c) {
#pragma clang fp contract(off)
    double N[3], v0[3];
    face_N_d(S, f, N, v0);
    const double wx = c.deye[0] - v0[0], wy = c.deye[1] - v0[1], wz = c.deye[2] - v0[2];
    return N[0] * wx + N[1] * wy + N[2] * wz > 0.0;
}

// The image of edge E in view c, as the primary edge term integrates over it:
// the part of the edge in front of the near plane (an endpoint at depth <=
// ZNEAR is replaced by the edge's point at depth ZNEAR; sa, sb = fraction of
// the edge cut away at its first, second vertex), projected to the image
// segment x(t) = A + t (B - A), and the range [t0, t1] of t inside the image
// rectangle [0, W] x [0, H] (Liang-Barsky, sides in a fixed order).  fp64 with
// a fixed operation order, so both implementations take the same candidates
// and weights.  False when nothing is left.
struct ScreenEdge {
    double ax, ay, bx, by;
    double sa, sb, t0, t1;
};

__device__ __forceinline__ bool screen_edge(const DevCam& c, const DevScene& S, int4 E, ScreenEdge& r) {
#pragma clang fp contract(off)
    const float* A = S.V + 3 * E.x;
    const float* B = S.V + 3 * E.y;
    const double a0 = A[0], a1 = A[1], a2 = A[2], b0 = B[0], b1 = B[1], b2 = B[2];
    double ax, ay, az, bx, by, bz;
    project_d(c, a0, a1, a2, ax, ay, az);
    project_d(c, b0, b1, b2, bx, by, bz);
    if (!(az > ZNEAR) && !(bz > ZNEAR)) return false;
    r.sa = 0.0;
    r.sb = 0.0;
    if (!(az > ZNEAR)) {
        r.sa = (ZNEAR - az) / (bz - az);
        project_d(c, a0 + (b0 - a0) * r.sa, a1 + (b1 - a1) * r.sa, a2 + (b2 - a2) * r.sa, ax, ay, az);
    }
    if (!(bz > ZNEAR)) {
        r.sb = (ZNEAR - bz) / (az - bz);
        project_d(c, b0 + (a0 - b0) * r.sb, b1 + (a1 - b1) * r.sb, b2 + (a2 - b2) * r.sb, bx, by, bz);
    }
    r.ax = ax; r.ay = ay; r.bx = bx; r.by = by;
    const double dx = bx - ax, dy = by - ay;
    const double P[4] = {-dx, dx, -dy, dy};
    const double Q[4] = {ax, (double)c.W - ax, ay, (double)c.H - ay};
    double t0 = 0.0, t1 = 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (P[i] == 0.0) {
            if (Q[i] < 0.0) return false;
            continue;
        }
        const double q = Q[i] / P[i];
        if (P[i] < 0.0) { if (q > t0) t0 = q; }
        else { if (q < t1) t1 = q; }
    }
    if (!(t0 < t1)) return false;
    r.t0 = t0;
    r.t1 = t1;
    return true;
}

__global__ void k_prim_weights(BwdParams p) {
#pragma clang fp contract(off)
    const int v = blockIdx.y;
    const DevCam& c = p.cams[v];
    const DevScene& S = p.scenes[c.scene];
    const int ne = S.ne;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        const int4 E = S.edges[e];
        double lenv = 0.0;
        const bool cand = E.w < 0 || front_facing_d(S, E.z, c) || front_facing_d(S, E.w, c);
        ScreenEdge se;
        if (cand && screen_edge(c, S, E, se)) {
            const double dx = se.bx - se.ax, dy = se.by - se.ay;
            lenv = (se.t1 - se.t0) * sqrt(dx * dx + dy * dy);
        }
        p.pw[(size_t)v * p.ne + e] = lenv;
    }
}

__global__ void k_prim_cdf(BwdParams p) {
    const int v = blockIdx.x;
    const DevScene& S = p.scenes[p.cams[v].scene];
    block_scan_normalise(p.pw + (size_t)v * p.ne, S.ne, p.pcdf + (size_t)v * (p.ne + 1), p.ptotal + v);
}

// ---------------------------------------------------------------------------
// primary edges through the wavefront: set-up of one edge sample, emission of
// its two side camera rays, and the gradient once their radiance is known
// ---------------------------------------------------------------------------
struct EdgeSample {
    int v, e, px, py;
    long long si;
    double t, xs, ys, nx, ny;
    bool inside;
};

// false when the sample is masked or its view has no candidate edge
__device__ __forceinline__ bool edge_setup(const BwdParams& p, long long ge, EdgeSample& es) {
    if (p.edge_mask && !p.edge_mask[ge]) return false;
    es.v = find_view(p.eoff, p.ncam, ge);
    const DevCam& c = p.cams[es.v];
    const DevScene& S = p.scenes[c.scene];
    if (!(p.ptotal[es.v] > 0.0)) return false;
    es.si = ge - c.eoff;
    const Ctr ctr{(uint32_t)es.si, (uint32_t)c.rngview << 16, 0u, 1u};
    const float4 u = draw4(ctr, 0, 3, Key{p.seed, S.scene_id});
    // stratified over the view's ne samples: sample si takes the CDF at (si + u0) / ne, so
    // consecutive samples walk along the CDF (coherent side rays and accumulators)
    es.e = cdf_guided(p.pcdf + (size_t)es.v * (p.ne + 1), S.ne, p.pguide + ((size_t)es.v << p.pglog), p.pglog,
                      ((double)es.si + (double)u.x) / (double)c.ne);
    ScreenEdge se;
    screen_edge(c, S, S.edges[es.e], se);     // true: only such edges have weight
    // the point is uniform on the visible part [t0, t1] of the image segment
    es.t = se.t0 + (double)u.y * (se.t1 - se.t0);
    const double ax = se.ax, ay = se.ay, bx = se.bx, by = se.by;
    es.xs = (1.0 - es.t) * ax + es.t * bx;
    es.ys = (1.0 - es.t) * ay + es.t * by;
    es.px = (int)floor(es.xs);
    es.py = (int)floor(es.ys);
    es.inside = es.xs >= 0.0 && es.ys >= 0.0 && es.px < c.W && es.py < c.H;
    const double dx = bx - ax, dy = by - ay;
    const double l = sqrt(dx * dx + dy * dy);
    es.nx = -dy / l;
    es.ny = dx / l;
    return true;
}

__device__ __forceinline__ V3 side_dir(const DevCam& c, const EdgeSample& es, int side) {
    const double sgn = side == 0 ? -1.0 : 1.0;
    const double sx = es.xs + sgn * EPS_PRIMARY * es.nx, sy = es.ys + sgn * EPS_PRIMARY * es.ny;
    const double ndx = 2.0 * sx / c.W - 1.0, ndy = 1.0 - 2.0 * sy / c.H;
    const double kx = ndx * c.dth * c.daspect, ky = ndy * c.dth;
    const double ddx = c.df[0] + c.dr[0] * kx + c.du[0] * ky;
    const double ddy = c.df[1] + c.dr[1] * kx + c.du[1] * ky;
    const double ddz = c.df[2] + c.dr[2] * kx + c.du[2] * ky;
    const double il = 1.0 / sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
    return V3{(float)(ddx * il), (float)(ddy * il), (float)(ddz * il)};
}

constexpr int EDGE_CAM_BLOCK = 1024;   // threads of a k_edge_camera block (one queue reservation each)

__global__ void __launch_bounds__(EDGE_CAM_BLOCK) k_edge_camera(BwdParams p, Queues q, long long e0, int n) {
    __shared__ int resv[EDGE_CAM_BLOCK / 64 + 1];
    const int stride = gridDim.x * blockDim.x;
    float* const* r = q.ray[1];
    for (int b0 = blockIdx.x * blockDim.x; b0 < n; b0 += stride) {
        const int i = b0 + (int)threadIdx.x;
        const long long ge = e0 + i;
        EdgeSample es;
        bool active = false;
        if (i < n && edge_setup(p, ge, es) && es.inside) {
            const DevCam& c = p.cams[es.v];
            const float* di = p.d_image + 3 * (c.pixoff + (long long)es.py * c.W + es.px);
            active = !(di[0] == 0.0f && di[1] == 0.0f && di[2] == 0.0f);
        }
        const int o0 = block_reserve<EDGE_CAM_BLOCK, 2>(active, &q.cnt[1], resv);
        if (!active) continue;
        if (o0 + 2 > q.cap) {               // the chunk holds both side rays of every sample
            atomicOr(p.err, ERR_QUEUE);
            continue;
        }
        const DevCam& c = p.cams[es.v];
        for (int side = 0; side < 2; ++side) {
            const int s = o0 + side;
            const V3 d = side_dir(c, es, side);
            // (origin, previous pdf, throughput and hash of a camera ray are
            // taken from the camera by the bounce-1 kernels)
            r[QDX][s] = d.x; r[QDY][s] = d.y; r[QDZ][s] = d.z;
            // a camera ray excludes no face: the slot carries the sampled edge
            // (top bit set), whose faces the extension tests before traversing
            qu(r, QEXCL, s) = 0x80000000u | (uint32_t)es.e;
            const uint32_t lq = (uint32_t)(2 * ge + side);
            qu(r, QQ, s) = lq;
            qu(r, QC0, s) = (uint32_t)es.si;
            qu(r, QC1, s) = (uint32_t)c.rngview << 16;
            qu(r, QVD, s) = (uint32_t)es.v | (1u << 16);
            q.L[3 * (size_t)lq] = 0.0f; q.L[3 * (size_t)lq + 1] = 0.0f; q.L[3 * (size_t)lq + 2] = 0.0f;
        }
    }
}

// sum of v over the lanes of the wave whose flag is set (every lane takes part)
__device__ __forceinline__ double wave_sum_masked(bool in, double v) {
    double s = in ? v : 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

__global__ void k_edge_grad(BwdParams p, const float* __restrict__ Ls, const uint32_t* __restrict__ hs,
                            long long total) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const int lane = (int)(threadIdx.x & 63u);
    // whole waves iterate together: the reduction below needs every lane
    for (long long w0 = blockIdx.x * (long long)blockDim.x + (threadIdx.x & ~63u); w0 < total; w0 += stride) {
        const long long ge = w0 + lane;
        EdgeSample es;
        bool has = false;
        double a0 = 0.0, a1 = 0.0;
        long long key = -1;
        if (ge < total && edge_setup(p, ge, es)) {
            const DevCam& c = p.cams[es.v];
            Hash h{FNV_INIT, p.dbg_edge_hash != nullptr};
            if (!es.inside) {
                h.push((uint32_t)es.e);
                h.push(0u);
                if (p.dbg_edge_hash) p.dbg_edge_hash[ge] = h.h;
            } else {
                const float* di = p.d_image + 3 * (c.pixoff + (long long)es.py * c.W + es.px);
                if (!(di[0] == 0.0f && di[1] == 0.0f && di[2] == 0.0f)) {
                    h.push((uint32_t)es.e);
                    h.push(1u);
                    if (p.dbg_edge_hash) {
                        h.push(hs[2 * ge]);
                        h.push(hs[2 * ge + 1]);
                        p.dbg_edge_hash[ge] = h.h;
                    }
                    const float* lm = Ls + 6 * ge;
                    float lv[6];
#pragma unroll
                    for (int m = 0; m < 6; ++m) lv[m] = qld(lm + m);
                    const double cc = ((double)di[0] * ((double)lv[0] - lv[3]) +
                                       (double)di[1] * ((double)lv[1] - lv[4]) +
                                       (double)di[2] * ((double)lv[2] - lv[5])) * (p.ptotal[es.v] / (double)c.ne);
                    a0 = cc * (1.0 - es.t);
                    a1 = cc * es.t;
                    key = (long long)es.v * p.ne + es.e;
                    has = true;
                }
            }
        }
        // the screen-space Jacobian and the edge normal depend on (view, edge) only:
        // the two endpoint weights are summed per (view, edge) here and applied once in
        // k_edge_finish; lanes of a wave that share a (view, edge) (consecutive
        // stratified samples mostly do) are summed first, one atomic pair per group
        bool pending = has;
        for (;;) {
            const uint64_t m = __ballot(pending);
            if (!m) break;
            const int leader = __ffsll((long long)m) - 1;
            const long long lk = ((long long)__builtin_amdgcn_readlane((int)(key >> 32), leader) << 32) |
                                 (unsigned int)__builtin_amdgcn_readlane((int)(key & 0xFFFFFFFFll), leader);
            const bool mine = pending && key == lk;
            const double s0 = wave_sum_masked(mine, a0), s1 = wave_sum_masked(mine, a1);
            if (lane == leader) {
                double* acc = p.pacc + 2 * (size_t)lk;
                atomicAdd(acc, s0);
                atomicAdd(acc + 1, s1);
            }
            pending = pending && !mine;
        }
    }
}

// d(x_s, y_s)/d(vertex) of the perspective projection, contracted with the
// screen-space edge normal and the accumulated endpoint weights of (view, edge).
// The image point is x = (1 - t) pi(a') + t pi(b') with the near-plane ends
// a' = va + sa (vb - va), b' = vb + sb (va - vb); t, sa and sb are held fixed
// (they only slide the point along the image line), so the Jacobians are taken
// at a' and b' and passed to the vertices with the weights (1 - sa, sa) and
// (sb, 1 - sb).
__global__ void k_edge_finish(BwdParams p) {
#pragma clang fp contract(off)
    const int v = blockIdx.y;
    const DevCam& c = p.cams[v];
    const DevScene& S = p.scenes[c.scene];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S.ne; e += gridDim.x * blockDim.x) {
        const double* acc = p.pacc + 2 * ((size_t)v * p.ne + e);
        const double w0 = acc[0], w1 = acc[1];
        if (w0 == 0.0 && w1 == 0.0) continue;
        const int4 E = S.edges[e];
        ScreenEdge se;
        if (!screen_edge(c, S, E, se)) continue;
        const double dx = se.bx - se.ax, dy = se.by - se.ay;
        const double l = sqrt(dx * dx + dy * dy);
        const double nx = -dy / l, ny = dx / l;
        const double pa[3] = {S.V[3 * E.x], S.V[3 * E.x + 1], S.V[3 * E.x + 2]};
        const double pb[3] = {S.V[3 * E.y], S.V[3 * E.y + 1], S.V[3 * E.y + 2]};
        double g[2][3];
        for (int end = 0; end < 2; ++end) {
            const double s0 = end == 0 ? se.sa : se.sb;
            const double* P0 = end == 0 ? pa : pb;
            const double* P1 = end == 0 ? pb : pa;
            const double wgt = end == 0 ? w0 : w1;
            const double qx = (P0[0] + (P1[0] - P0[0]) * s0) - c.deye[0];
            const double qy = (P0[1] + (P1[1] - P0[1]) * s0) - c.deye[1];
            const double qz = (P0[2] + (P1[2] - P0[2]) * s0) - c.deye[2];
            const double z = qx * c.df[0] + qy * c.df[1] + qz * c.df[2];
            const double aa = qx * c.dr[0] + qy * c.dr[1] + qz * c.dr[2];
            const double bb = qx * c.du[0] + qy * c.du[1] + qz * c.du[2];
            const double kx = (0.5 * c.W) / (c.dth * c.daspect) / (z * z);
            const double ky = -(0.5 * c.H) / c.dth / (z * z);
            for (int k3 = 0; k3 < 3; ++k3) {
                const double dsx = kx * (c.dr[k3] * z - aa * c.df[k3]);
                const double dsy = ky * (c.du[k3] * z - bb * c.df[k3]);
                g[end][k3] = wgt * (dsx * nx + dsy * ny);
            }
        }
        double ga[3], gb[3];
        for (int k3 = 0; k3 < 3; ++k3) {
            ga[k3] = (1.0 - se.sa) * g[0][k3] + se.sb * g[1][k3];
            gb[k3] = se.sa * g[0][k3] + (1.0 - se.sb) * g[1][k3];
        }
        atomic_add3(p.dV + 3 * (size_t)E.x, V3{(float)ga[0], (float)ga[1], (float)ga[2]});
        atomic_add3(p.dV + 3 * (size_t)E.y, V3{(float)gb[0], (float)gb[1], (float)gb[2]});
    }
}

// per-face corner accumulators (corner c of face f at facc[16 f + 3 c]) to dV
// (vertex gather over the incidence CSR, fixed order); material accumulators
// (per face, or per texel with mesh colours) to dmat [ntex, 7]
__global__ void k_face_gather(BwdParams p) {
    const DevScene& S = p.scenes[0];
    const int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < S.nv; v += stride) {
        float sx = 0.f, sy = 0.f, sz = 0.f;
        for (int j = p.vf_off[v]; j < p.vf_off[v + 1]; ++j) {
            const int e = p.vf_idx[j];
            const float* a = p.facc + (size_t)FACC_STRIDE * (e / 3) + 3 * (e % 3);
            sx += a[0]; sy += a[1]; sz += a[2];
        }
        p.dV[3 * (size_t)v] += sx;
        p.dV[3 * (size_t)v + 1] += sy;
        p.dV[3 * (size_t)v + 2] += sz;
    }
    const bool texels = S.tex_res > 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < p.ntex; t += stride) {
        const float* a = mat_slots(p.facc, p.macc, texels, t, t);
#pragma unroll
        for (int i = 0; i < 7; ++i) p.dmat[7 * (size_t)t + i] = a[i];
    }
}

// ---------------------------------------------------------------------------
// point-light shadow boundaries seen by the camera.  For light l an edge is a
// candidate when it is a boundary edge or its faces lie on opposite sides of the
// light (the fp64 side test of the secondary edges, at the light position);
// edges are drawn by 3-D length, t uniform.  The light ray through the edge
// point y continues to the receiver point z; if the camera sees z, the screen
// point s = pi(z) lies on the image of the shadow boundary.  With tau = ds/dt
// and n = perp(tau)/|tau| the receiver points under s -/+ 1e-3 px n take the
// light's visibility V-, V+, and the sample adds
// d_image(s) . (V- - V+) L_l(z) (n . ds/dtheta) |tau| W_l / (|vb - va| N_s)
// for theta = the edge's endpoints and the receiver face's vertices.
// ---------------------------------------------------------------------------
__global__ void k_light_weights(BwdParams p) {
#pragma clang fp contract(off)
    const int l = blockIdx.y;
    const DevScene& S = p.scenes[0];
    const V3 pl = ld3(S.lights + 6 * l);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S.ne; e += gridDim.x * blockDim.x) {
        const int4 E = S.edges[e];
        double w = 0.0;
        if (silhouette(S, E, pl)) {
            const double dx = (double)S.V[3 * E.y] - (double)S.V[3 * E.x];
            const double dy = (double)S.V[3 * E.y + 1] - (double)S.V[3 * E.x + 1];
            const double dz = (double)S.V[3 * E.y + 2] - (double)S.V[3 * E.x + 2];
            w = sqrt(dx * dx + dy * dy + dz * dz);
        }
        p.lw[(size_t)l * p.ne + e] = w;
    }
}

__global__ void k_light_cdf(BwdParams p) {
    const int l = blockIdx.x;
    block_scan_normalise(p.lw + (size_t)l * p.ne, p.ne, p.lcdf + (size_t)l * (p.ne + 1), p.ltotal + l);
}

// screen point of z and its Jacobian rows (d sx/dz, d sy/dz) for camera c
__device__ __forceinline__ void project_jac(const DevCam& c, const double z[3], double& sx, double& sy, double& depth,
                                            double jx[3], double jy[3]) {
#pragma clang fp contract(off)
    const double q[3] = {z[0] - c.deye[0], z[1] - c.deye[1], z[2] - c.deye[2]};
    depth = q[0] * c.df[0] + q[1] * c.df[1] + q[2] * c.df[2];
    const double a = q[0] * c.dr[0] + q[1] * c.dr[1] + q[2] * c.dr[2];
    const double b = q[0] * c.du[0] + q[1] * c.du[1] + q[2] * c.du[2];
    sx = (a / (depth * (c.dth * c.daspect)) + 1.0) * (0.5 * c.W);
    sy = (1.0 - b / (depth * c.dth)) * (0.5 * c.H);
    const double kx = (0.5 * c.W) / (c.dth * c.daspect) / (depth * depth);
    const double ky = -(0.5 * c.H) / c.dth / (depth * depth);
    for (int k = 0; k < 3; ++k) {
        jx[k] = kx * (c.dr[k] * depth - a * c.df[k]);
        jy[k] = ky * (c.du[k] * depth - b * c.df[k]);
    }
}

__device__ void shadow_edge_one(const BwdParams& p, const DevScene& S, const DevCam& c, int v, int l, long long si,
                                long long nsv, Hash& h, TravStack& st) {
#pragma clang fp contract(off)
    if (!(p.ltotal[l] > 0.0)) return;
    const Ctr ctr{(uint32_t)si, ((uint32_t)c.rngview << 16) | (uint32_t)l, 0u, 3u};
    const float4 u = draw4(ctr, 0, 3, Key{p.seed, S.scene_id});
    // stratified over the nsv samples of the (view, light) pair
    const int e = cdf_guided(p.lcdf + (size_t)l * (p.ne + 1), S.ne, p.lguide + ((size_t)l << p.pglog), p.pglog,
                             ((double)si + (double)u.x) / (double)nsv);
    const float t = u.y;
    h.push((uint32_t)e);
    const int4 E = S.edges[e];
    const float* lt = S.lights + 6 * l;
    const V3 pl = ld3(lt), va = ld3(S.V + 3 * E.x), vb = ld3(S.V + 3 * E.y);
    const V3 y = va + (vb - va) * t;
    const V3 w = normalize(y - pl);
    float tr;
    const int fr = trace_closest(S, y, w, TMIN, E.z, tr, st);
    h.push(fr < 0 ? 0xFFFFFFFFu : (uint32_t)fr);
    if (fr < 0 || fr == E.w) return;
    const V3 zt = y + w * tr;
    const V3 eye = ld3(c.eye);
    float tc;
    const int fc = trace_closest(S, eye, normalize(zt - eye), TMIN, -1, tc, st);
    const bool vis = fc == fr;
    h.push(vis ? 2u : 1u);
    if (!vis) return;
    // receiver point on the plane of fr along the light ray through y (fp64)
    double Nr[3], r0[3];
    face_N_d(S, fr, Nr, r0);
    const double yd[3] = {(double)y.x, (double)y.y, (double)y.z}, pd[3] = {(double)pl.x, (double)pl.y, (double)pl.z};
    const double D[3] = {yd[0] - pd[0], yd[1] - pd[1], yd[2] - pd[2]};
    const double Bd = Nr[0] * D[0] + Nr[1] * D[1] + Nr[2] * D[2];
    const double A = Nr[0] * (r0[0] - pd[0]) + Nr[1] * (r0[1] - pd[1]) + Nr[2] * (r0[2] - pd[2]);
    const double lam = A / Bd;
    const double z[3] = {pd[0] + D[0] * lam, pd[1] + D[1] * lam, pd[2] + D[2] * lam};
    double xs, ys, depth, jx[3], jy[3];
    project_jac(c, z, xs, ys, depth, jx, jy);
    const int px = (int)floor(xs), py = (int)floor(ys);
    const bool inside = depth > ZNEAR && xs >= 0.0 && ys >= 0.0 && px < c.W && py < c.H;
    h.push(inside ? 1u : 0u);
    if (!inside) return;
    const float* di = p.d_image + 3 * (c.pixoff + (long long)py * c.W + px);
    if (di[0] == 0.0f && di[1] == 0.0f && di[2] == 0.0f) return;
    // tau = ds/dt = J (dz/dy)(vb - va), dz/dy d = lam (d - D (Nr . d) / Bd)
    const double ed[3] = {(double)vb.x - (double)va.x, (double)vb.y - (double)va.y, (double)vb.z - (double)va.z};
    const double ne_ = (Nr[0] * ed[0] + Nr[1] * ed[1] + Nr[2] * ed[2]) / Bd;
    double dz[3];
    for (int k = 0; k < 3; ++k) dz[k] = lam * (ed[k] - D[k] * ne_);
    const double tx = jx[0] * dz[0] + jx[1] * dz[1] + jx[2] * dz[2];
    const double ty = jy[0] * dz[0] + jy[1] * dz[1] + jy[2] * dz[2];
    const double tl = sqrt(tx * tx + ty * ty);
    if (!(tl > 0.0)) return;
    const double nx = -ty / tl, ny = tx / tl;
    // light visibility on both sides, at the receiver plane under the side points
    int vsd[2];
    for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? -1.0 : 1.0;
        const double sxp = xs + sg * EPS_PRIMARY * nx, syp = ys + sg * EPS_PRIMARY * ny;
        const double ndx = 2.0 * sxp / c.W - 1.0, ndy = 1.0 - 2.0 * syp / c.H;
        const double kx = ndx * c.dth * c.daspect, ky = ndy * c.dth;
        double dd[3];
        for (int k = 0; k < 3; ++k) dd[k] = c.df[k] + c.dr[k] * kx + c.du[k] * ky;
        const double il = 1.0 / sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
        for (int k = 0; k < 3; ++k) dd[k] *= il;
        const double tp = (Nr[0] * (r0[0] - c.deye[0]) + Nr[1] * (r0[1] - c.deye[1]) + Nr[2] * (r0[2] - c.deye[2])) /
                          (Nr[0] * dd[0] + Nr[1] * dd[1] + Nr[2] * dd[2]);
        const double zs[3] = {c.deye[0] + dd[0] * tp, c.deye[1] + dd[1] * tp, c.deye[2] + dd[2] * tp};
        const double wl[3] = {pd[0] - zs[0], pd[1] - zs[1], pd[2] - zs[2]};
        const double r = sqrt(wl[0] * wl[0] + wl[1] * wl[1] + wl[2] * wl[2]);
        const V3 zf{(float)zs[0], (float)zs[1], (float)zs[2]};
        const V3 wf{(float)(wl[0] / r), (float)(wl[1] / r), (float)(wl[2] / r)};
        vsd[side] = trace_any(S, zf, wf, TMIN, (float)(r * (1.0 - (double)SHADOW_SHRINK)), fr, st) ? 0 : 1;
        h.push((uint32_t)vsd[side]);
    }
    if (vsd[0] == vsd[1]) return;
    // unshadowed radiance of the light at z toward the camera
    const V3 zf{(float)z[0], (float)z[1], (float)z[2]};
    const V3 wo = normalize(eye - zt);
    V3 n = normalize(V3{(float)Nr[0], (float)Nr[1], (float)Nr[2]});
    if (dot(n, wo) < 0.0f) n = -n;
    const V3 dl = pl - zt;
    const float r2 = dot(dl, dl);
    const V3 wl = dl * (1.0f / sqrtf(r2));
    const float cl = dot(n, wl);
    if (!(cl > 0.0f)) return;
    const Mat m = load_mat(S.mat + 7 * (size_t)texel_of(S, fr, zf));
    const V3 fv = brdf_eval(wl, wo, n, m);
    const V3 I = ld3(lt + 3);
    const double dv = (double)(vsd[0] - vsd[1]);
    double cc = ((double)di[0] * fv.x * I.x + (double)di[1] * fv.y * I.y + (double)di[2] * fv.z * I.z) * dv *
                (double)cl / (double)r2;
    cc *= tl * p.ltotal[l] / (p.lw[(size_t)l * p.ne + e] * (double)nsv);
    // reverse: g_z = J^T (cc n), then z = pl + lam (y - pl), lam = (Nr . (r0 - pl)) / (Nr . (y - pl))
    double gz[3];
    for (int k = 0; k < 3; ++k) gz[k] = cc * (nx * jx[k] + ny * jy[k]);
    const double glam = gz[0] * D[0] + gz[1] * D[1] + gz[2] * D[2];
    double gy[3], gN[3], gr0[3];
    for (int k = 0; k < 3; ++k) {
        gy[k] = lam * gz[k] - glam * lam * Nr[k] / Bd;
        gN[k] = glam * ((r0[k] - pd[k]) * Bd - A * D[k]) / (Bd * Bd);
        gr0[k] = glam * Nr[k] / Bd;
    }
    // N = e1 x e2 with e1 = r1 - r0, e2 = r2 - r0
    const int i0 = S.F[3 * fr], i1 = S.F[3 * fr + 1], i2 = S.F[3 * fr + 2];
    const double e1[3] = {(double)S.V[3 * i1] - r0[0], (double)S.V[3 * i1 + 1] - r0[1], (double)S.V[3 * i1 + 2] - r0[2]};
    const double e2[3] = {(double)S.V[3 * i2] - r0[0], (double)S.V[3 * i2 + 1] - r0[1], (double)S.V[3 * i2 + 2] - r0[2]};
    const double ge1[3] = {e2[1] * gN[2] - e2[2] * gN[1], e2[2] * gN[0] - e2[0] * gN[2], e2[0] * gN[1] - e2[1] * gN[0]};
    const double ge2[3] = {gN[1] * e1[2] - gN[2] * e1[1], gN[2] * e1[0] - gN[0] * e1[2], gN[0] * e1[1] - gN[1] * e1[0]};
    const float tt = t;
    atomic_add3(p.dV + 3 * (size_t)E.x, V3{(float)(gy[0] * (1.0 - tt)), (float)(gy[1] * (1.0 - tt)),
                                           (float)(gy[2] * (1.0 - tt))});
    atomic_add3(p.dV + 3 * (size_t)E.y, V3{(float)(gy[0] * tt), (float)(gy[1] * tt), (float)(gy[2] * tt)});
    atomic_add3(p.dV + 3 * (size_t)i0, V3{(float)(gr0[0] - ge1[0] - ge2[0]), (float)(gr0[1] - ge1[1] - ge2[1]),
                                          (float)(gr0[2] - ge1[2] - ge2[2])});
    atomic_add3(p.dV + 3 * (size_t)i1, V3{(float)ge1[0], (float)ge1[1], (float)ge1[2]});
    atomic_add3(p.dV + 3 * (size_t)i2, V3{(float)ge2[0], (float)ge2[1], (float)ge2[2]});
}

// one thread per shadow-edge sample; sample gs of (view v, light l, index i) is
// nl eoff[v] + l N_e(v) + i, and its hash / mask slot follows the primary edge samples
__global__ void __launch_bounds__(TRACE_BLOCK) k_shadow_edges(BwdParams p, long long total_edges, long long nsh) {
    __shared__ uint32_t lds[LDS_STACK * TRACE_BLOCK];
    TravStack st = make_trav_stack(lds, p.spill, p.err, nullptr);
    const DevScene& S = p.scenes[0];
    const long long nl = S.nl;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long gs = blockIdx.x * (long long)blockDim.x + threadIdx.x; gs < nsh; gs += stride) {
        int lo = 0, hi = p.ncam - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (nl * p.eoff[mid] <= gs) lo = mid; else hi = mid - 1;
        }
        const DevCam& c = p.cams[lo];
        const long long nsv = p.eoff[lo + 1] - p.eoff[lo];
        const long long rem = gs - nl * p.eoff[lo];
        const int l = (int)(rem / nsv);
        const long long si = rem - (long long)l * nsv;
        if (p.edge_mask && !p.edge_mask[total_edges + gs]) continue;
        Hash h{FNV_INIT, p.dbg_edge_hash != nullptr};
        shadow_edge_one(p, S, c, lo, l, si, nsv, h, st);
        if (p.dbg_edge_hash) p.dbg_edge_hash[total_edges + gs] = h.h;
    }
}


// ---------------------------------------------------------------------------
static inline unsigned gridb(long long n, int bs, int cap) {
    long long g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

void launch_primary_edges(const BwdParams& p, const FwdParams& fp, Queues& q, float* Lside, uint32_t* hside,
                          long long total_edges, int has_env_any, hipStream_t st, LaunchHook* hook) {
    if (total_edges <= 0 || p.ne <= 0) return;
    ST_LAUNCH("k_prim_weights", k_prim_weights, dim3(gridb(p.ne, 256, 1024), p.ncam), dim3(256), 0, st, p);
    ST_LAUNCH("k_prim_cdf", k_prim_cdf, dim3(p.ncam), dim3(1024), 0, st, p);
    launch_guide(p.pcdf, p.ne, (size_t)(p.ne + 1), p.ncam, p.pguide, p.pglog, st);
    const long long per = q.cap / 2;
    for (long long e0 = 0; e0 < total_edges; e0 += per) {
        const int n = (int)((total_edges - e0) < per ? (total_edges - e0) : per);
        launch_fill_u32((uint32_t*)q.cnt, 64, 0u, st);
        launch_fill_u32((uint32_t*)q.fetch, FETCH_INTS, 0u, st);
        ST_LAUNCH("k_edge_camera", k_edge_camera, dim3(gridb(n, EDGE_CAM_BLOCK, 1 << 20)), dim3(EDGE_CAM_BLOCK), 0, st,
                  p, q, e0, n);
        if (hook) hook->tick();
        launch_wavefront_bounces(fp, q, 2 * n, has_env_any, st, hook);
    }
    launch_fill_u32((uint32_t*)p.pacc, 4ll * p.ncam * p.ne, 0u, st);      // +0.0 doubles
    ST_LAUNCH("k_edge_grad", k_edge_grad, dim3(gridb(total_edges, 256, 1 << 16)), dim3(256), 0, st, p, Lside, hside,
              total_edges);
    ST_LAUNCH("k_edge_finish", k_edge_finish, dim3(gridb(p.ne, 256, 1024), p.ncam), dim3(256), 0, st, p);
}

// Paths whose camera ray hit a face, in path order within each block's span.
// A path whose camera ray escaped has no vertex: its adjoint adds nothing (the
// environment seen directly depends on neither the vertices nor the
// materials), and its lanes would idle through the replay of the others.  Each
// thread looks at 16 consecutive paths, so a block reserves list slots once per
// 4,096 paths: all blocks share the one counter, and a reservation per 256
// paths kept the kernel waiting on it.
constexpr int ADJ_LIST_PER = 16;
__global__ void __launch_bounds__(256) k_adj_list(const int* __restrict__ rec_face, long long total, uint32_t* list,
                                                  int* n) {
    __shared__ int resv[256 / 64 + 1];
    constexpr long long span = 256ll * ADJ_LIST_PER;
    for (long long b0 = (long long)blockIdx.x * span; b0 < total; b0 += (long long)gridDim.x * span) {
        const long long i0 = b0 + (long long)threadIdx.x * ADJ_LIST_PER;
        uint32_t m = 0;
        if (i0 + ADJ_LIST_PER <= total) {
            // rec_face is 256-B aligned and i0 a multiple of 16: four 16-B loads
            const int4* v = (const int4*)(rec_face + i0);
#pragma unroll
            for (int j = 0; j < ADJ_LIST_PER / 4; ++j) {
                const int4 a = v[j];
                m |= (uint32_t)(a.x >= 0) << (4 * j) | (uint32_t)(a.y >= 0) << (4 * j + 1) |
                     (uint32_t)(a.z >= 0) << (4 * j + 2) | (uint32_t)(a.w >= 0) << (4 * j + 3);
            }
        } else {
            for (int j = 0; j < ADJ_LIST_PER && i0 + j < total; ++j) m |= (uint32_t)(rec_face[i0 + j] >= 0) << j;
        }
        // every thread of the block calls it (it synchronises the block)
        int o = block_reserve_n<256, 5>(__popc(m), n, resv);
        for (; m; m &= m - 1, ++o) list[o] = (uint32_t)(i0 + __ffs(m) - 1);
    }
}

// (path, vertex) jobs of the marked secondary edge samples, in path and vertex
// order within each block's span: each thread reads the marks of 16
// consecutive paths (one 16-byte load), and a block reserves job slots once
// per 4,096 paths (all blocks share the one counter; a reservation per 256
// paths and bit kept the kernel waiting on it)
constexpr int SEC_JOBS_PER = 16;
__global__ void __launch_bounds__(256) k_sec_jobs(const uint8_t* __restrict__ mask, long long total, int B,
                                                 int2* jobs, int* njobs, uint32_t* err) {
    __shared__ int resv[256 / 64 + 1];
    constexpr long long span = 256ll * SEC_JOBS_PER;
    const uint32_t keep = 0x01010101u * ((1u << B) - 1u);     // the B vertex bits of each byte
    for (long long b0 = (long long)blockIdx.x * span; b0 < total; b0 += (long long)gridDim.x * span) {
        const long long i0 = b0 + (long long)threadIdx.x * SEC_JOBS_PER;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (i0 + SEC_JOBS_PER <= total) {
            // mask is 16-B aligned and i0 a multiple of 16
            const uint4 v = *(const uint4*)(mask + i0);
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
            for (int j = 0; j < SEC_JOBS_PER && i0 + j < total; ++j) w[j >> 2] |= (uint32_t)mask[i0 + j] << (8 * (j & 3));
        }
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[q] &= keep;
            cnt += __popc(w[q]);
        }
        // every thread of the block calls it (it synchronises the block); at most 16 x 8 jobs
        int o = block_reserve_n<256, 8>(cnt, njobs, resv);
        for (int j = 0; j < SEC_JOBS_PER; ++j) {
            for (uint32_t m = (w[j >> 2] >> (8 * (j & 3))) & 0xFFu; m; m &= m - 1, ++o) {
                if ((long long)o < total * B) jobs[o] = make_int2((int)(i0 + j), __ffs(m) - 1);   // at most B per path
                else atomicOr(err, ERR_QUEUE);
            }
        }
    }
}

size_t sec_workspace_bytes(long long total_paths, int B) {
    return 256 + (((size_t)total_paths + 255) & ~(size_t)255) + sizeof(int2) * (size_t)total_paths * B + 256;
}

void carve_sec_workspace(BwdParams& p, void* base, long long total_paths) {
    char* c = (char*)base;
    p.sec_njobs = (int*)c;
    p.sec_mask = (uint8_t*)(c + 256);
    p.sec_jobs = (int2*)(c + 256 + (((size_t)total_paths + 255) & ~(size_t)255));
}

template <int BM>
static void launch_adjoint(const BwdParams& p, long long total_paths, int grid, const char* name,
                           const char* name_jobs, hipStream_t st) {
    const dim3 gd(gridb(total_paths, TRACE_BLOCK, grid)), bd(TRACE_BLOCK);
    if (p.rec_split && (p.flags & ST_EDGE_SECONDARY_HIERARCHY))
        ST_LAUNCH(name, (k_adjoint<BM, false, 2>), gd, bd, 0, st, p, total_paths);
    else if (p.rec_split)
        ST_LAUNCH(name, (k_adjoint<BM, false, 1>), gd, bd, 0, st, p, total_paths);
    // (returns at once when the records pass above found its records valid)
    ST_LAUNCH(name, (k_adjoint<BM, false>), gd, bd, 0, st, p, total_paths);
    if (p.sec_mask) {
        ST_LAUNCH("k_sec_jobs", k_sec_jobs, dim3(gridb(total_paths, 256 * SEC_JOBS_PER, 1 << 12)), dim3(256), 0, st, p.sec_mask,
                  total_paths, p.B, p.sec_jobs, p.sec_njobs, p.err);
        // the job count stays on the device: a fixed grid strides over it
        ST_LAUNCH(name_jobs, (k_adjoint<BM, true>), dim3(1024), bd, 0, st, p, 0ll);
    }
}

// What the adjoint passes start from: cleared accumulators and job counters,
// and the list of paths with a vertex.  Small kernels, launched on the caller's
// stream before the adjoint forks to the second stream: there they would wait
// for room behind the side paths' traversal, and the adjoint with them.
void launch_backward_prep(const BwdParams& p, int nf, long long total_paths, hipStream_t st) {
    if (!((p.flags & 5u) && total_paths > 0)) return;
    launch_fill_u32((uint32_t*)p.facc, (long long)FACC_STRIDE * nf, 0u, st);
    if (p.ntex != nf) launch_fill_u32((uint32_t*)p.macc, (long long)MACC_STRIDE * p.ntex, 0u, st);
    if (p.sec_mask) {
        launch_fill_u32((uint32_t*)p.sec_njobs, 1, 0u, st);
        launch_fill_u32((uint32_t*)p.sec_mask, (total_paths + 3) / 4, 0u, st);
    }
    if (p.rec_split && p.adj_list) {
        launch_fill_u32((uint32_t*)p.adj_n, 1, 0u, st);
        ST_LAUNCH("k_adj_list", k_adj_list, dim3(gridb(total_paths, 256 * ADJ_LIST_PER, 1 << 12)), dim3(256), 0, st,
                  p.rec_face, total_paths, p.adj_list, p.adj_n);
    }
}

// the interior and secondary-edge terms into the per-face accumulators (and
// secondary-edge atomics into dV), after launch_backward_prep on the same
// stream or one ordered after it; launch_face_gather adds them to dV and dmat
void launch_backward(const BwdParams& p, int nv, int nf, long long total_paths, long long total_edges, int grid,
                     hipStream_t st) {
    (void)nv;
    (void)nf;
    (void)total_edges;
    if ((p.flags & 5u) && total_paths > 0) {
        if (p.B <= 1) launch_adjoint<1>(p, total_paths, grid, "k_adjoint<1>", "k_adjoint_sec<1>", st);
        else if (p.B <= 2) launch_adjoint<2>(p, total_paths, grid, "k_adjoint<2>", "k_adjoint_sec<2>", st);
        else if (p.B <= 3) launch_adjoint<3>(p, total_paths, grid, "k_adjoint<3>", "k_adjoint_sec<3>", st);
        else launch_adjoint<8>(p, total_paths, grid, "k_adjoint<8>", "k_adjoint_sec<8>", st);
    }
}

// dV += the per-face corner accumulators gathered per vertex (a plain add: after
// every other writer of dV), dmat = the material accumulators
void launch_face_gather(const BwdParams& p, int nv, hipStream_t st) {
    ST_LAUNCH("k_face_gather", k_face_gather, dim3(gridb(std::max<long long>(nv, p.ntex), 256, 4096)), dim3(256), 0, st,
              p);
}

void launch_shadow_edges(const BwdParams& p, long long total_edges, int nl, hipStream_t st) {
    if (total_edges <= 0 || p.ne <= 0 || nl <= 0) return;
    ST_LAUNCH("k_light_weights", k_light_weights, dim3(gridb(p.ne, 256, 1024), nl), dim3(256), 0, st, p);
    ST_LAUNCH("k_light_cdf", k_light_cdf, dim3(nl), dim3(1024), 0, st, p);
    launch_guide(p.lcdf, p.ne, (size_t)(p.ne + 1), nl, p.lguide, p.pglog, st);
    const long long nsh = total_edges * nl;
    ST_LAUNCH("k_shadow_edges", k_shadow_edges, dim3(gridb(nsh, TRACE_BLOCK, TRACE_GRID)), dim3(TRACE_BLOCK), 0, st, p,
              total_edges, nsh);
}

} // namespace st

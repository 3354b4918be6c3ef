// FP64 CPU oracle for the differentiable path tracer.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call this
// code: only the tests, the smoke check and the CPU-baseline leg of the bench do.
// It shares no code with the HIP library; the two agree only on the written
// specification of the estimator (random-number streams, shading, edge terms)
// and receive the same seeded float32 inputs.
//
// What it computes (Shape from Tracing, Sec. 3.2 "Vertex optimization" and
// Sec. 3.3 "Representation"): the path-traced rendering R(x, m, c_i) of a
// triangle mesh with per-face Torrance-Sparrow materials under point lights or
// an HDR environment map (Sec. 3.1), with global illumination (Sec. 3.3,
// "Effects of Global Illumination"), and the gradient of a loss on that image
// with respect to vertex positions and per-face materials, including the
// edge-sampled visibility terms of the renderer the paper relies on (Sec. 3.2,
// which cites Li et al. 2018 for gradients with respect to geometry).
//
// The image is a Monte Carlo estimate, so the oracle follows the estimator step
// by step in double precision with the same counter-based random numbers as the
// GPU.  Derivatives of the per-sample estimator are taken by forward-mode dual
// numbers on a replay of the recorded path (no hand-derived adjoint here).
//
// Parity status of each function is written in its comment; where none of the
// pins in the CPU test-suite reaches a choice, the comment says
// "parity unpinned".

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace orc {

static const double PI = 3.14159265358979323846;
static const double TMIN = 1e-4;            // ray epsilon (scene units)
static const double SHADOW_SHRINK = 1e-4;   // point-light shadow ray stops at r(1 - 1e-4)
static const double ALPHA_MIN = 1e-3;       // roughness floor
static const double LOBE_SPEC_P = 0.5;      // probability of sampling the specular lobe
static const double EPS_PRIMARY = 1e-3;     // primary edge side offset, pixels
static const double EPS_SECONDARY = 1e-4;   // secondary edge side offset, radians
static const double ZNEAR = 1e-3;           // primary edges are clipped at this depth
static const double SEC_COS_MIN = 1e-5;     // secondary edge points this close to the tangent plane are skipped

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, the key bumped
// between rounds by the Weyl constants.  Parity: pinned against numpy's
// Philox4x64-10 through a width-generic reference and bit-compared with it.
// --------------------------------------------------------------------------
struct U4 { uint32_t v[4]; };

static U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    U4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// 24-bit uniform in [0, 1 - 2^-24], exact in float and double.
static inline double unif(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }

struct Ctr { uint32_t c0, c1, c2hi, c3; };   // c2 = c2hi | (bounce << 8) | block

static inline void draw4(const Ctr& c, uint32_t bounce, uint32_t block, uint32_t k0, uint32_t k1,
                         double u[4]) {
    U4 r = philox(c.c0, c.c1, c.c2hi | (bounce << 8) | block, c.c3, k0, k1);
    for (int i = 0; i < 4; ++i) u[i] = unif(r.v[i]);
}

// FNV-1a over the little-endian bytes of 32-bit decision words.
struct Hash {
    uint32_t h = 0x811C9DC5u;
    bool on = true;
    std::vector<uint32_t>* buf = nullptr;   // when set, words are queued instead of hashed
    void push(uint32_t w) {
        if (!on) return;
        if (buf) { buf->push_back(w); return; }
        for (int b = 0; b < 4; ++b) { h ^= (w >> (8 * b)) & 0xFFu; h *= 0x01000193u; }
    }
};

// --------------------------------------------------------------------------
// scalar types: double, and a forward-mode dual number with N tangents
// --------------------------------------------------------------------------
template <int N> struct Dual {
    double v;
    double d[N];
    Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
    Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }
};
static inline double val(double x) { return x; }
template <int N> static inline double val(const Dual<N>& x) { return x.v; }

template <int N> static inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> static inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> static inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> static inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> static inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v / b.v; double ib = 1.0 / b.v;
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r; }
template <int N> static inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> static inline Dual<N> operator+(double b, const Dual<N>& a) { Dual<N> r = a; r.v += b; return r; }
template <int N> static inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> static inline Dual<N> operator-(double b, const Dual<N>& a) { Dual<N> r = -a; r.v += b; return r; }
template <int N> static inline Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> static inline Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> static inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> static inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> static inline Dual<N> chain(const Dual<N>& a, double fv, double dfv) {
    Dual<N> r; r.v = fv; for (int i = 0; i < N; ++i) r.d[i] = dfv * a.d[i]; return r; }
template <int N> static inline Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> static inline Dual<N> exp(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> static inline Dual<N> erfc(const Dual<N>& a) {
    return chain(a, std::erfc(a.v), -2.0 / std::sqrt(PI) * std::exp(-a.v * a.v)); }
using std::sqrt; using std::exp; using std::erfc;

template <class T> struct V3 {
    T x, y, z;
    V3() : x(0.0), y(0.0), z(0.0) {}
    V3(T a, T b, T c) : x(a), y(b), z(c) {}
    template <class S> explicit V3(const V3<S>& o) : x(o.x), y(o.y), z(o.z) {}
    T& operator[](int i) { return i == 0 ? x : (i == 1 ? y : z); }
    const T& operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
};
using D3 = V3<double>;
template <class T> static inline V3<T> operator+(const V3<T>& a, const V3<T>& b) { return V3<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> static inline V3<T> operator-(const V3<T>& a, const V3<T>& b) { return V3<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T> static inline V3<T> operator-(const V3<T>& a) { return V3<T>(-a.x, -a.y, -a.z); }
template <class T, class S> static inline V3<T> operator*(const V3<T>& a, const S& s) { return V3<T>(a.x * s, a.y * s, a.z * s); }
template <class T> static inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> static inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return V3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
template <class T> static inline T length(const V3<T>& a) { return sqrt(dot(a, a)); }
template <class T> static inline V3<T> normalize(const V3<T>& a) { T l = length(a); return a * (1.0 / l); }
template <int N> static inline V3<Dual<N>> normalize(const V3<Dual<N>>& a) {
    Dual<N> l = length(a); return V3<Dual<N>>(a.x / l, a.y / l, a.z / l); }
template <class T> static inline V3<T> lift(const D3& a) { return V3<T>(T(a.x), T(a.y), T(a.z)); }
static inline D3 vval(const D3& a) { return a; }
template <int N> static inline D3 vval(const V3<Dual<N>>& a) { return D3(a.x.v, a.y.v, a.z.v); }

// --------------------------------------------------------------------------
// scene
// --------------------------------------------------------------------------
struct Edge { int va, vb, f1, f2; };

struct BVHNode { double lo[3], hi[3]; int left, right, first, count; };

struct EdgeTree {
    int n = 0;                      // edges (leaves)
    std::vector<uint64_t> keys;     // sorted morton << 32 | edge
    std::vector<int> child, parent;
    std::vector<float> box, len;    // per node (internal nodes, then leaves)
    std::vector<float> nbox;        // per node: box of the unit normals of the edges' faces
};

struct Scene {
    int nv = 0, nf = 0, nl = 0, he = 0, we = 0;
    int tex_res = 0;               // mesh-colours resolution r; mat holds nf (r+1)(r+2)/2 texels
    uint32_t id = 0;
    std::vector<double> V, mat, lights, env;
    std::vector<int> F;
    std::vector<Edge> edges;
    std::vector<double> ecdf;     // cumulative 3-D edge length / total, size ne+1
    double elen_total = 0.0;
    bool has_env = false;
    std::vector<double> marg, cond, texp;   // env CDFs and texel probabilities
    double env_total = 0.0;
    bool env_alias = false;                 // texel chosen through the alias table instead of the CDFs
    bool vndf = false;                      // specular lobe sampled from the visible normals
    EdgeTree etree;                         // secondary-edge importance hierarchy
    std::vector<double> aprob;              // Walker/Vose alias table over the texels
    std::vector<int> alias;
    std::vector<BVHNode> nodes;
    std::vector<int> perm;

    D3 vert(int i) const { return D3(V[3 * i], V[3 * i + 1], V[3 * i + 2]); }
};

// Mesh colours (Sec. 3.3 "Representation"): the texel of the point with
// barycentric coordinates (alpha, beta) in triangle t at resolution r is
// entry t (r+1)(r+2)/2 + i (2r - i + 3)/2 + j of the texel array, with
// (i, j) = floor(r (alpha, beta)); alpha weighs the triangle's second vertex and
// beta its third.  Points on the boundary of the barycentric domain are
// clamped into it (0 <= i <= r, 0 <= j <= r - i).
static long long texel_index(int r, long long t, double alpha, double beta) {
    if (!(alpha == alpha) || !(beta == beta)) alpha = beta = 0.0;
    alpha = std::min(std::max(alpha, -1.0), 2.0);
    beta = std::min(std::max(beta, -1.0), 2.0);
    long long i = (long long)std::floor(r * alpha), j = (long long)std::floor(r * beta);
    i = std::min<long long>(std::max<long long>(i, 0), r);
    j = std::min<long long>(std::max<long long>(j, 0), r - i);
    return (t * (r + 1) * (r + 2) + i * (2 * r - i + 3)) / 2 + j;
}

// Barycentric coordinates (alpha of v1, beta of v2) of point x in the plane of face f.
static void barycentric(const Scene& s, int f, const D3& x, double& alpha, double& beta);

// Texel (material row) of the point x on face f.
static long long texel_of(const Scene& s, int f, const D3& x) {
    if (s.tex_res == 0) return f;
    double a, b;
    barycentric(s, f, x, a, b);
    return texel_index(s.tex_res, f, a, b);
}

// Unnormalised face normal (v1-v0)x(v2-v0), evaluated in a fixed operation order.
static D3 face_N(const Scene& s, int f) {
    D3 a = s.vert(s.F[3 * f]), b = s.vert(s.F[3 * f + 1]), c = s.vert(s.F[3 * f + 2]);
    return cross(b - a, c - a);
}

static void barycentric(const Scene& s, int f, const D3& x, double& alpha, double& beta) {
    D3 v0 = s.vert(s.F[3 * f]), e1 = s.vert(s.F[3 * f + 1]) - v0, e2 = s.vert(s.F[3 * f + 2]) - v0;
    D3 N = cross(e1, e2), q = x - v0;
    double nn = dot(N, N);
    alpha = dot(cross(q, e2), N) / nn;
    beta = dot(cross(e1, q), N) / nn;
}

// Edge list in canonical order: (va < vb) ascending, f1 the smaller face id.
static void build_edges(Scene& s) {
    std::vector<std::array<int, 3>> he;
    he.reserve(3 * s.nf);
    for (int f = 0; f < s.nf; ++f)
        for (int k = 0; k < 3; ++k) {
            int a = s.F[3 * f + k], b = s.F[3 * f + (k + 1) % 3];
            he.push_back({std::min(a, b), std::max(a, b), f});
        }
    std::sort(he.begin(), he.end());
    s.edges.clear();
    for (size_t i = 0; i < he.size();) {
        size_t j = i;
        while (j < he.size() && he[j][0] == he[i][0] && he[j][1] == he[i][1]) ++j;
        Edge e{he[i][0], he[i][1], he[i][2], (j - i >= 2) ? he[i + 1][2] : -1};
        s.edges.push_back(e);
        i = j;
    }
    const size_t ne = s.edges.size();
    s.ecdf.assign(ne + 1, 0.0);
    double acc = 0.0;
    std::vector<double> cum(ne + 1, 0.0);
    for (size_t e = 0; e < ne; ++e) {
        D3 d = s.vert(s.edges[e].vb) - s.vert(s.edges[e].va);
        acc += std::sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
        cum[e + 1] = acc;
    }
    s.elen_total = acc;
    for (size_t e = 0; e <= ne; ++e) s.ecdf[e] = acc > 0 ? cum[e] / acc : 0.0;
}

// Environment-map distribution (piecewise constant over equirectangular texels,
// each weighted by its mean RGB times its solid angle).  Parity: pinned by the
// normalisation, constant-map and histogram tests.
static void build_env(Scene& s) {
    s.has_env = false;
    if (s.he <= 0 || s.we <= 0 || s.env.empty()) return;
    const int H = s.he, W = s.we;
    std::vector<double> w((size_t)H * W), rows(H);
    for (int r = 0; r < H; ++r) {
        double dom = (2.0 * PI / W) * (std::cos(PI * r / H) - std::cos(PI * (r + 1) / H));
        double rs = 0.0;
        for (int c = 0; c < W; ++c) {
            const double* t = &s.env[3 * ((size_t)r * W + c)];
            double m = (t[0] + t[1] + t[2]) / 3.0;
            w[(size_t)r * W + c] = m * dom;
            rs += m * dom;
        }
        rows[r] = rs;
    }
    double tot = 0.0;
    s.marg.assign(H + 1, 0.0);
    for (int r = 0; r < H; ++r) { tot += rows[r]; s.marg[r + 1] = tot; }
    s.env_total = tot;
    if (!(tot > 0.0)) return;
    for (int r = 0; r <= H; ++r) s.marg[r] /= tot;
    s.cond.assign((size_t)H * (W + 1), 0.0);
    s.texp.assign((size_t)H * W, 0.0);
    for (int r = 0; r < H; ++r) {
        double* C = &s.cond[(size_t)r * (W + 1)];
        double acc = 0.0;
        C[0] = 0.0;
        for (int c = 0; c < W; ++c) { acc += w[(size_t)r * W + c]; C[c + 1] = acc; }
        for (int c = 0; c <= W; ++c) C[c] = rows[r] > 0 ? C[c] / rows[r] : (double)c / W;
        for (int c = 0; c < W; ++c) s.texp[(size_t)r * W + c] = w[(size_t)r * W + c] / tot;
    }
    s.has_env = true;
}

static inline double row_solid_angle(const Scene& s, int r) {
    return (2.0 * PI / s.we) * (std::cos(PI * r / s.he) - std::cos(PI * (r + 1) / s.he));
}

// largest i in [0, n-1] with C[i] <= u  (C[0] == 0 <= u)
static inline int cdf_find(const double* C, int n, double u) {
    return (int)(std::upper_bound(C, C + n, u) - C) - 1;
}

static int env_texel_of(const Scene& s, const D3& d) {
    double y = std::max(-1.0, std::min(1.0, d.y));
    double th = std::acos(y);
    double ph = std::atan2(d.x, d.z);
    if (ph < 0) ph += 2.0 * PI;
    int r = std::min((int)(th / PI * s.he), s.he - 1);
    int c = std::min((int)(ph / (2.0 * PI) * s.we), s.we - 1);
    return r * s.we + c;
}

static D3 env_rgb(const Scene& s, int texel) {
    return D3(s.env[3 * (size_t)texel], s.env[3 * (size_t)texel + 1], s.env[3 * (size_t)texel + 2]);
}

static double env_pdf_texel(const Scene& s, int texel) {
    int r = texel / s.we;
    return s.texp[texel] / row_solid_angle(s, r);
}

// Alias table of the texel probabilities (Walker 1977, Vose 1991): bin k keeps
// probability aprob[k] for texel k and gives the rest to texel alias[k].  Built
// with two stacks in index order, taking from their tops, in fp64.
static void build_alias(Scene& s) {
    const int n = s.he * s.we;
    s.aprob.assign(n, 1.0);
    s.alias.resize(n);
    std::vector<double> q(n);
    std::vector<int> small, large;
    for (int i = 0; i < n; ++i) {
        s.alias[i] = i;
        q[i] = s.texp[i] * n;
        if (q[i] < 1.0) small.push_back(i); else large.push_back(i);
    }
    while (!small.empty() && !large.empty()) {
        const int a = small.back(), l = large.back();
        small.pop_back();
        large.pop_back();
        s.aprob[a] = q[a];
        s.alias[a] = l;
        q[l] = (q[l] + q[a]) - 1.0;
        if (q[l] < 1.0) small.push_back(l); else large.push_back(l);
    }
}

static int env_sample(const Scene& s, const double u[4], D3& dir, double& pdf) {
    int r, c;
    if (s.env_alias) {
        // bin by u0, texel of the bin or its alias by u1
        const int n = s.he * s.we;
        int k = (int)(u[0] * n);
        if (k > n - 1) k = n - 1;
        const int texel = u[1] < s.aprob[k] ? k : s.alias[k];
        r = texel / s.we;
        c = texel % s.we;
    } else {
        r = cdf_find(s.marg.data(), s.he, u[0]);
        c = cdf_find(&s.cond[(size_t)r * (s.we + 1)], s.we, u[1]);
    }
    double phi = 2.0 * PI * (c + u[2]) / s.we;
    double ct = std::cos(PI * r / s.he), cb = std::cos(PI * (r + 1) / s.he);
    double cth = ct - u[3] * (ct - cb);
    double sth = std::sqrt(std::max(0.0, 1.0 - cth * cth));
    dir = D3(sth * std::sin(phi), cth, sth * std::cos(phi));
    int texel = r * s.we + c;
    pdf = env_pdf_texel(s, texel);
    return texel;
}

// --------------------------------------------------------------------------
// ray-triangle intersection (Moller-Trumbore, two-sided) and a median-split BVH.
// Parity: BVH closest/any hit pinned against brute force (exact face and t).
// --------------------------------------------------------------------------
static bool tri_hit(const Scene& s, int f, const D3& o, const D3& d, double tmin, double tmax, double& t) {
    D3 v0 = s.vert(s.F[3 * f]), v1 = s.vert(s.F[3 * f + 1]), v2 = s.vert(s.F[3 * f + 2]);
    D3 e1 = v1 - v0, e2 = v2 - v0;
    D3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    D3 sv = o - v0;
    double b1 = dot(sv, p) * inv;
    if (b1 < 0.0 || b1 > 1.0) return false;
    D3 q = cross(sv, e1);
    double b2 = dot(d, q) * inv;
    if (b2 < 0.0 || b1 + b2 > 1.0) return false;
    t = dot(e2, q) * inv;
    return t > tmin && t < tmax;
}

static void build_bvh(Scene& s) {
    s.nodes.clear();
    s.perm.resize(s.nf);
    for (int i = 0; i < s.nf; ++i) s.perm[i] = i;
    if (s.nf == 0) return;
    std::vector<D3> cen(s.nf), lo(s.nf), hi(s.nf);
    for (int f = 0; f < s.nf; ++f) {
        D3 a = s.vert(s.F[3 * f]), b = s.vert(s.F[3 * f + 1]), c = s.vert(s.F[3 * f + 2]);
        for (int k = 0; k < 3; ++k) {
            lo[f][k] = std::min(a[k], std::min(b[k], c[k]));
            hi[f][k] = std::max(a[k], std::max(b[k], c[k]));
            cen[f][k] = 0.5 * (lo[f][k] + hi[f][k]);
        }
    }
    struct Job { int node, first, count; };
    std::vector<Job> stack;
    s.nodes.push_back(BVHNode());
    stack.push_back({0, 0, s.nf});
    while (!stack.empty()) {
        Job j = stack.back(); stack.pop_back();
        BVHNode nd;
        for (int k = 0; k < 3; ++k) { nd.lo[k] = 1e300; nd.hi[k] = -1e300; }
        D3 clo(1e300, 1e300, 1e300), chi(-1e300, -1e300, -1e300);
        for (int i = j.first; i < j.first + j.count; ++i) {
            int f = s.perm[i];
            for (int k = 0; k < 3; ++k) {
                nd.lo[k] = std::min(nd.lo[k], lo[f][k]); nd.hi[k] = std::max(nd.hi[k], hi[f][k]);
                clo[k] = std::min(clo[k], cen[f][k]); chi[k] = std::max(chi[k], cen[f][k]);
            }
        }
        // widen by a relative margin so that the box test can never cull a hit
        for (int k = 0; k < 3; ++k) {
            double m = 1e-9 * (std::fabs(nd.lo[k]) + std::fabs(nd.hi[k]) + 1.0);
            nd.lo[k] -= m; nd.hi[k] += m;
        }
        if (j.count <= 4) {
            nd.left = nd.right = -1; nd.first = j.first; nd.count = j.count;
            s.nodes[j.node] = nd;
            continue;
        }
        int ax = 0;
        for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
        int mid = j.first + j.count / 2;
        std::nth_element(s.perm.begin() + j.first, s.perm.begin() + mid, s.perm.begin() + j.first + j.count,
                         [&](int a, int b) { return cen[a][ax] < cen[b][ax] || (cen[a][ax] == cen[b][ax] && a < b); });
        int l = (int)s.nodes.size(); s.nodes.push_back(BVHNode());
        int r = (int)s.nodes.size(); s.nodes.push_back(BVHNode());
        nd.left = l; nd.right = r; nd.first = j.first; nd.count = 0;
        s.nodes[j.node] = nd;
        stack.push_back({l, j.first, mid - j.first});
        stack.push_back({r, mid, j.first + j.count - mid});
    }
}

static bool box_hit(const BVHNode& n, const D3& o, const D3& d, double tmin, double tmax) {
    double t0 = tmin, t1 = tmax;
    for (int k = 0; k < 3; ++k) {
        double a = (n.lo[k] - o[k]) / d[k], b = (n.hi[k] - o[k]) / d[k];
        if (std::isnan(a) || std::isnan(b)) {        // d[k] == 0 and o on a slab plane
            if (o[k] < n.lo[k] || o[k] > n.hi[k]) return false;
            continue;
        }
        if (a > b) std::swap(a, b);
        t0 = std::max(t0, a); t1 = std::min(t1, b);
        if (t0 > t1) return false;
    }
    return true;
}

// closest hit with t in (tmin, inf); equal t resolved to the smaller face id
static int closest_hit(const Scene& s, const D3& o, const D3& d, double tmin, int exclude, double& tbest,
                       bool brute = false) {
    int best = -1;
    tbest = INFINITY;
    auto consider = [&](int f) {
        if (f == exclude) return;
        double t;
        if (tri_hit(s, f, o, d, tmin, INFINITY, t)) {
            if (t < tbest || (t == tbest && f < best)) { tbest = t; best = f; }
        }
    };
    if (brute || s.nodes.empty()) {
        for (int f = 0; f < s.nf; ++f) consider(f);
        return best;
    }
    int stack[128]; int sp = 0; stack[sp++] = 0;
    while (sp) {
        const BVHNode& n = s.nodes[stack[--sp]];
        if (!box_hit(n, o, d, tmin, tbest)) continue;
        if (n.left < 0) { for (int i = n.first; i < n.first + n.count; ++i) consider(s.perm[i]); }
        else { stack[sp++] = n.left; stack[sp++] = n.right; }
    }
    return best;
}

static bool any_hit(const Scene& s, const D3& o, const D3& d, double tmin, double tmax, int exclude,
                    bool brute = false) {
    if (brute || s.nodes.empty()) {
        for (int f = 0; f < s.nf; ++f) { double t; if (f != exclude && tri_hit(s, f, o, d, tmin, tmax, t)) return true; }
        return false;
    }
    int stack[128]; int sp = 0; stack[sp++] = 0;
    while (sp) {
        const BVHNode& n = s.nodes[stack[--sp]];
        if (!box_hit(n, o, d, tmin, tmax)) continue;
        if (n.left < 0) {
            for (int i = n.first; i < n.first + n.count; ++i) {
                int f = s.perm[i]; double t;
                if (f != exclude && tri_hit(s, f, o, d, tmin, tmax, t)) return true;
            }
        } else { stack[sp++] = n.left; stack[sp++] = n.right; }
    }
    return false;
}

// --------------------------------------------------------------------------
// camera: pinhole, vertical field of view, image row 0 at the top
// --------------------------------------------------------------------------
struct Cam {
    D3 eye, f, r, u;
    double th, aspect;
    int W, H;
};

static Cam make_cam(const double* row, int W, int H) {
    Cam c;
    c.eye = D3(row[0], row[1], row[2]);
    D3 tg(row[3], row[4], row[5]), up(row[6], row[7], row[8]);
    c.f = normalize(tg - c.eye);
    D3 upn = normalize(up);
    if (std::fabs(dot(c.f, upn)) > 0.999) upn = D3(0, 0, 1);
    if (std::fabs(dot(c.f, upn)) > 0.999) upn = D3(1, 0, 0);
    c.r = normalize(cross(c.f, upn));
    c.u = cross(c.r, c.f);
    c.th = std::tan(row[9] * PI / 360.0);
    c.aspect = (double)W / (double)H;
    c.W = W; c.H = H;
    return c;
}

static D3 cam_dir(const Cam& c, double sx, double sy) {
    double nx = 2.0 * sx / c.W - 1.0, ny = 1.0 - 2.0 * sy / c.H;
    return normalize(c.f + c.r * (nx * c.th * c.aspect) + c.u * (ny * c.th));
}

template <class T> static void project(const Cam& c, const V3<T>& v, T& sx, T& sy, T& z) {
    V3<T> p = v - lift<T>(c.eye);
    z = dot(p, lift<T>(c.f));
    T a = dot(p, lift<T>(c.r)), b = dot(p, lift<T>(c.u));
    sx = (a / (z * (c.th * c.aspect)) + 1.0) * (0.5 * c.W);
    sy = (1.0 - b / (z * c.th)) * (0.5 * c.H);
}

// --------------------------------------------------------------------------
// Torrance-Sparrow BRDF (Sec. 3.3 "Representation"): Lambertian kd/pi plus a
// microfacet lobe ks * D * G / (4 cos_i cos_o) with the Beckmann distribution
// and the height-correlated Smith masking of the Beckmann surface.  The
// specular colour ks plays the role of the Fresnel factor (no angular term).
// Parity: D normalisation, weak white furnace of D and Lambda, reciprocity and
// the pdf normalisation are pinned by quadrature; the choice of D/G/F itself is
// a reading of an unspecified model (parity unpinned beyond those invariants).
// --------------------------------------------------------------------------
template <class T> static T beckmann_D(const T& ch, const T& a) {
    T c2 = ch * ch;
    T t2 = (1.0 - c2) / c2;
    return exp(-t2 / (a * a)) / (PI * a * a * c2 * c2);
}

template <class T> static T smith_lambda(const T& c, const T& a) {
    if (val(c) >= 1.0) return T(0.0);
    T sn = sqrt(1.0 - c * c);
    T x = c / (a * sn);
    return (exp(-x * x) / (x * std::sqrt(PI)) - erfc(x)) * 0.5;
}

template <class T> static T alpha_eff(const T& a) { return val(a) > ALPHA_MIN ? a : T(ALPHA_MIN); }

// f(wi, wo) per channel; zero when either direction is below the surface
template <class T>
static V3<T> brdf(const V3<T>& wi, const V3<T>& wo, const V3<T>& n, const T* m) {
    T ci = dot(n, wi), co = dot(n, wo);
    if (!(val(ci) > 0.0) || !(val(co) > 0.0)) return V3<T>();
    T a = alpha_eff(m[6]);
    V3<T> h = normalize(wi + wo);
    T ch = dot(n, h);
    T spec(0.0);
    if (val(ch) > 0.0) {
        T D = beckmann_D(ch, a);
        T G = 1.0 / (1.0 + smith_lambda(ci, a) + smith_lambda(co, a));
        spec = D * G / (4.0 * ci * co);
    }
    return V3<T>(m[0] * (1.0 / PI) + m[3] * spec, m[1] * (1.0 / PI) + m[4] * spec, m[2] * (1.0 / PI) + m[5] * spec);
}

// pdf of the one-sample mixture: 1/2 cosine-weighted + 1/2 specular.  The
// specular half-vectors follow D(h) cos(theta_h) (classical), or with vndf the
// distribution of normals visible from wo, G1(wo) max(0, wo.h) D(h) / cos(theta_o)
// (Heitz and d'Eon 2014); either is turned into a pdf of wi by 1 / (4 |wo.h|).
static double bsdf_pdf(const D3& wi, const D3& wo, const D3& n, double alpha, bool vndf) {
    double ci = dot(n, wi);
    if (!(ci > 0.0)) return 0.0;
    double a = std::max(alpha, ALPHA_MIN);
    double pd = (1.0 - LOBE_SPEC_P) * ci / PI;
    D3 hv = wi + wo;
    double hl = length(hv);
    double ps = 0.0;
    if (hl > 0.0) {
        D3 h = hv * (1.0 / hl);
        double ch = dot(n, h), oh = dot(wo, h);
        if (!vndf) {
            oh = std::fabs(oh);
            if (ch > 0.0 && oh > 0.0) ps = LOBE_SPEC_P * beckmann_D(ch, a) * ch / (4.0 * oh);
        } else {
            double co = dot(n, wo);
            if (ch > 0.0 && oh > 0.0 && co > 0.0) {
                double g1 = 1.0 / (1.0 + smith_lambda(co, a));
                ps = LOBE_SPEC_P * g1 * beckmann_D(ch, a) / (4.0 * co);
            }
        }
    }
    return pd + ps;
}

// inverse error function: Winitzki's closed-form approximation (S. Winitzki,
// "A handy approximation for the error function and its inverse", 2008, a = 0.147)
// refined by Newton steps on erf in double precision
static double erfinv_d(double y) {
    const double a = 0.147;
    const double l = std::log((1.0 - y) * (1.0 + y));
    const double t = 2.0 / (PI * a) + 0.5 * l;
    double x = std::copysign(std::sqrt(std::sqrt(t * t - l / a) - t), y);
    for (int it = 0; it < 8; ++it) {
        // erf(x) - y, taken through erfc near |y| = 1 where erf(x) and y cancel
        const double r = y > 0.5 ? (1.0 - y) - std::erfc(x) : y < -0.5 ? std::erfc(-x) - (1.0 + y) : std::erf(x) - y;
        const double d = r / (2.0 / std::sqrt(PI) * std::exp(-x * x));
        x -= d;
        if (std::fabs(d) < 1e-16 * std::max(1.0, std::fabs(x))) break;
    }
    return x;
}

// Visible-normal sampling of the Beckmann lobe (Heitz and d'Eon 2014): stretch
// wo by alpha; for the standard surface seen at cot(theta') = c, the slope along
// the incident plane has density ~ (c - x) exp(-x^2) on x < c, whose integral
// F(x) = c sqrt(pi)/2 erfc(-x) + exp(-x^2) / 2 is inverted at u1 F(c); the
// other slope is erfinv(2 u2 - 1); rotate back, unstretch, normal from slopes.
static const double VNDF_COT_MAX = 1e4;         // cot(theta') at (near) normal incidence
static const double VNDF_Y_MAX = 1.0 - 1.0 / 8388608.0;   // |2 u2 - 1| kept below 1 (u2 = 0)

static double vndf_F(double x, double c) {
    return c * (0.5 * std::sqrt(PI)) * std::erfc(-x) + 0.5 * std::exp(-x * x);
}
// F(c) - F(x), without the cancellation of the difference near x = c
static double vndf_G(double x, double c) {
    return c * (0.5 * std::sqrt(PI)) * (std::erfc(x) - std::erfc(c)) + 0.5 * (std::exp(-c * c) - std::exp(-x * x));
}

static D3 vndf_normal(const D3& wo_l, double a, double u1, double u2) {
    D3 ws = normalize(D3(a * wo_l.x, a * wo_l.y, wo_l.z));
    double st = std::sqrt(ws.x * ws.x + ws.y * ws.y);
    double cphi = st > 0.0 ? ws.x / st : 1.0, sphi = st > 0.0 ? ws.y / st : 0.0;
    double c = st > 0.0 ? std::min(ws.z / st, VNDF_COT_MAX) : VNDF_COT_MAX;
    // bracketed Newton over (-8, c): F(x) = u1 F(c) on the lower half of u1,
    // F(c) - F(x) = (1 - u1) F(c) on the upper half
    const bool upper = u1 > 0.5;
    const double target = (upper ? 1.0 - u1 : u1) * vndf_F(c, c);
    // (the root lies below 8: F(8) equals F(c) to far below double rounding)
    double lo = -8.0, hi = std::min(c, 8.0), x = std::min(0.0, 0.5 * c);
    for (int it = 0; it < 100; ++it) {
        double g = upper ? target - vndf_G(x, c) : vndf_F(x, c) - target;    // increasing in x
        if (g > 0.0) hi = x; else lo = x;
        double dg = (c - x) * std::exp(-x * x);
        double xn = dg > 0.0 ? x - g / dg : 0.5 * (lo + hi);
        if (!(xn >= lo && xn <= hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) < 1e-15 * std::max(1.0, std::fabs(x))) { x = xn; break; }
        x = xn;
    }
    double yv = std::max(-VNDF_Y_MAX, std::min(VNDF_Y_MAX, 2.0 * u2 - 1.0));
    double y = erfinv_d(yv);
    double sx = (cphi * x - sphi * y) * a, sy = (sphi * x + cphi * y) * a;
    return normalize(D3(-sx, -sy, 1.0));
}

// orthonormal basis around n (Duff et al. 2017, JCGT 6(1), branchless construction)
static void onb(const D3& n, D3& t, D3& b) {
    double sg = std::copysign(1.0, n.z);
    double a = -1.0 / (sg + n.z);
    double bb = n.x * n.y * a;
    t = D3(1.0 + sg * n.x * n.x * a, sg * bb, -sg * n.x);
    b = D3(bb, sg + n.y * n.y * a, -n.y);
}

// returns lobe (0 specular, 1 diffuse) and the sampled world direction
static int bsdf_sample(const double u[4], const D3& wo, const D3& n, double alpha, bool vndf, D3& wi) {
    D3 t, b;
    onb(n, t, b);
    double a = std::max(alpha, ALPHA_MIN);
    double phi = 2.0 * PI * u[2];
    if (u[0] < LOBE_SPEC_P && vndf) {
        D3 hl = vndf_normal(D3(dot(wo, t), dot(wo, b), dot(wo, n)), a, u[1], u[2]);
        D3 h = t * hl.x + b * hl.y + n * hl.z;
        wi = h * (2.0 * dot(wo, h)) - wo;
        return 0;
    }
    if (u[0] < LOBE_SPEC_P) {
        double t2 = -a * a * std::log(1.0 - u[1]);
        double ch = 1.0 / std::sqrt(1.0 + t2);
        double sh = std::sqrt(std::max(0.0, 1.0 - ch * ch));
        D3 h = t * (sh * std::cos(phi)) + b * (sh * std::sin(phi)) + n * ch;
        wi = h * (2.0 * dot(wo, h)) - wo;
        return 0;
    }
    double r = std::sqrt(u[1]);
    double z = std::sqrt(std::max(0.0, 1.0 - u[1]));
    wi = t * (r * std::cos(phi)) + b * (r * std::sin(phi)) + n * z;
    return 1;
}

// --------------------------------------------------------------------------
// path estimator
// --------------------------------------------------------------------------
static const int MAXV = 8;
static const int MAXL = 16;

struct VRec {
    int face = -1, flip = 0;
    long long tex = -1;           // material texel of the vertex
    D3 wo;
    int lcode[MAXL];
    int ecode = 0; D3 we, Le; double eden = 0.0;
    int sec = 0; double sec_c = 0.0; D3 sec_m;
    int cont = 0; D3 wi; double pb = 0.0;
    int esc = 0; D3 esc_val;
};
struct PRec { int nv = 0; D3 o, d; VRec v[MAXV]; };

struct Grad {           // double accumulators for dV [nv*3] and dmat [nf*7]
    std::vector<double> dV, dM;
};

struct SecCtx {         // secondary-edge state of a main path (backward only)
    double w[3];        // loss weight per channel for this sample
    Grad* g;
    bool interior = false;  // also take edges that are not silhouettes from the shading point
                            // (creases and material boundaries seen in direction space)
    bool hier = false;      // edges drawn by the importance hierarchy instead of the length CDF
};

struct Key { uint32_t k0, k1; };

static int edge_tree_sample(const Scene& s, const D3& x, const D3& nn, const Ctr& ctr, int k, const Key& key,
                            bool sil, float& pe);

static void push_face(Hash& h, int f) { h.push(f < 0 ? 0xFFFFFFFFu : (uint32_t)f); }

// Hit point on the plane of face f along (o, d): the same point Moller-Trumbore
// returns, written so that its dependence on the vertices is explicit.
template <class T>
static V3<T> plane_hit(const V3<T>& o, const V3<T>& d, const V3<T>& v0, const V3<T>& v1, const V3<T>& v2) {
    V3<T> N = cross(v1 - v0, v2 - v0);
    T t = dot(v0 - o, N) / dot(d, N);
    return o + d * t;
}

static D3 L_in_side(const Scene& s, const D3& x, const D3& dir, int exclude, int budget, const Ctr& ctr,
                    const Key& key, Hash& hash);

// Secondary (direction-space) edge term at path vertex k: shading point x on
// face f, normal n flipped toward wo, material row m, path throughput beta.
// One edge is drawn (length CDF, or the importance hierarchy), a point y
// uniform on it; the edge is taken when it is a silhouette seen from x (a
// boundary edge, or its two faces on opposite sides of x) or, with
// sec.interior, any edge not of face f (creases and material boundaries).  Two
// side rays bracket the edge direction, their incoming radiance is estimated
// with the remaining vertex budget, and the jump times the BRDF, the cosine and
// the normal velocity of the edge on the sphere of directions is scattered to
// the edge's endpoints (dV) with the selection weight.  The decision words go
// to sech.
static void secondary_edge_sample(const Scene& s, const D3& x, const D3& n, const D3& wo, int f, const double* m,
                                  const D3& beta, int k, int budget, const Ctr& ctr, const Key& key,
                                  const SecCtx& sec, Hash& sech, VRec* vr) {
    double u[4];
    draw4(ctr, k, 3, key.k0, key.k1, u);
    int e;
    double wsel = 0.0;      // 1 / (probability density of the edge point per unit length)
    if (sec.hier) {
        float pe;
        e = edge_tree_sample(s, x, n, ctr, k, key, !sec.interior, pe);
        if (e >= 0) {
            const Edge& Es = s.edges[e];
            wsel = length(s.vert(Es.vb) - s.vert(Es.va)) / (double)pe;
        }
    } else {
        e = cdf_find(s.ecdf.data(), (int)s.edges.size(), u[0]);
        wsel = s.elen_total;
    }
    double te = u[1];
    if (e < 0) { sech.push(0xFFFFFFFFu); sech.push(0u); return; }
    sech.push((uint32_t)e);
    const Edge& E = s.edges[e];
    D3 va = s.vert(E.va), vb = s.vert(E.vb);
    // an edge of the shading face lies in the tangent plane (cos = 0):
    // its direction-space contribution vanishes, so it is never taken
    bool sil = E.f1 != f && E.f2 != f;
    if (sil && E.f2 >= 0 && !sec.interior) {
        double s1 = dot(face_N(s, E.f1), x - va), s2 = dot(face_N(s, E.f2), x - va);
        sil = (s1 > 0.0) != (s2 > 0.0);
    }
    D3 y = va + (vb - va) * te;
    D3 wv = y - x;
    double r2 = dot(wv, wv);
    if (sil && r2 > 0.0) {
        double r = std::sqrt(r2);
        D3 ud = wv * (1.0 / r);
        double cv = dot(n, ud);
        D3 eh = normalize(vb - va);
        D3 mv = cross(ud, eh);
        double ml = length(mv);
        if (cv > SEC_COS_MIN && ml > 0.0) {
            sech.push(1u);
            D3 mm = mv * (1.0 / ml);
            D3 wm = normalize(ud - mm * EPS_SECONDARY), wp = normalize(ud + mm * EPS_SECONDARY);
            Ctr sc{ctr.c0, ctr.c1, (uint32_t)k << 16, 2u};
            D3 Lm = L_in_side(s, x, wm, f, budget, sc, key, sech);
            D3 Lp = L_in_side(s, x, wp, f, budget, sc, key, sech);
            D3 fv = brdf(ud, wo, n, m);
            double cc = 0.0;
            for (int ch = 0; ch < 3; ++ch)
                cc += sec.w[ch] * beta[ch] * fv[ch] * cv * (Lm[ch] - Lp[ch]);
            cc *= wsel / r2;
            if (sec.g) {
                for (int k3 = 0; k3 < 3; ++k3) {
                    sec.g->dV[3 * E.va + k3] += cc * (1.0 - te) * mv[k3];
                    sec.g->dV[3 * E.vb + k3] += cc * te * mv[k3];
                }
            }
            if (vr) { vr->sec = 1; vr->sec_c = cc; vr->sec_m = mv; }
            return;
        }
    }
    sech.push(0u);
}

// Radiance estimate along a ray (Sec. 3.2: R is a physically based path tracer).
// first_escape_full: a miss on the very first segment returns the environment
// radiance (side rays of the secondary edge term); otherwise (camera rays) a
// first-segment miss is black, which is how the masks M^t, M^r of the loss are
// read (background zero).
static D3 trace_estimator(const Scene& s, D3 o, D3 d, int exclude, int nvert, bool first_escape_full,
                          const Ctr& ctr, const Key& key, Hash& hash, PRec* rec, SecCtx* sec) {
    D3 L(0, 0, 0), beta(1, 1, 1);
    double p_prev = 0.0;
    if (rec) { rec->nv = 0; rec->o = o; rec->d = d; }
    // decision words of the secondary edge samples follow all main-path words
    std::vector<uint32_t> secbuf;
    Hash sech;
    sech.on = hash.on;
    sech.buf = &secbuf;
    for (int k = 1; k <= nvert + 1; ++k) {
        double t;
        int f = closest_hit(s, o, d, TMIN, exclude, t);
        push_face(hash, f);
        if (f < 0) {
            if (s.has_env && (k > 1 || first_escape_full)) {
                int tex = env_texel_of(s, d);
                hash.push((uint32_t)tex);
                D3 Le = env_rgb(s, tex);
                double w = 1.0;
                if (k > 1) { double pe = env_pdf_texel(s, tex); w = p_prev / (p_prev + pe); }
                L = L + D3(beta.x * Le.x, beta.y * Le.y, beta.z * Le.z) * w;
                if (rec && k > 1) { rec->v[k - 2].esc = 1; rec->v[k - 2].esc_val = Le * w; }
            }
            break;
        }
        if (k == nvert + 1) break;
        VRec* vr = rec ? &rec->v[k - 1] : nullptr;
        D3 v0 = s.vert(s.F[3 * f]), v1 = s.vert(s.F[3 * f + 1]), v2 = s.vert(s.F[3 * f + 2]);
        D3 x = plane_hit(o, d, v0, v1, v2);
        D3 n = normalize(cross(v1 - v0, v2 - v0));
        D3 wo = -d;
        int flip = dot(n, wo) < 0.0;
        if (flip) n = -n;
        const long long tx = texel_of(s, f, x);
        if (s.tex_res > 0) hash.push((uint32_t)tx);
        const double* m = &s.mat[7 * tx];
        if (vr) { vr->face = f; vr->flip = flip; vr->wo = wo; vr->tex = tx; rec->nv = k; }
        // next-event estimation: every point light (Sec. 3.1 point-light input)
        for (int l = 0; l < s.nl; ++l) {
            const double* lt = &s.lights[6 * l];
            D3 dl = D3(lt[0], lt[1], lt[2]) - x;
            double r2 = dot(dl, dl);
            int code = 0;
            if (r2 > 0.0) {
                double r = std::sqrt(r2);
                D3 wl = dl * (1.0 / r);
                double c = dot(n, wl);
                if (c > 0.0) {
                    bool occ = any_hit(s, x, wl, TMIN, r * (1.0 - SHADOW_SHRINK), f);
                    code = occ ? 1 : 2;
                    if (!occ) {
                        D3 fv = brdf(wl, wo, n, m);
                        L = L + D3(beta.x * lt[3] * fv.x, beta.y * lt[4] * fv.y, beta.z * lt[5] * fv.z) * (c / r2);
                    }
                }
            }
            hash.push((uint32_t)code);
            if (vr) vr->lcode[l] = code;
        }
        // next-event estimation: one environment sample, balance-heuristic MIS
        if (s.has_env) {
            double u[4];
            draw4(ctr, k, 1, key.k0, key.k1, u);
            D3 we; double pe;
            int tex = env_sample(s, u, we, pe);
            hash.push((uint32_t)tex);
            double c = dot(n, we);
            int code = 0;
            if (c > 0.0 && pe > 0.0) {
                bool occ = any_hit(s, x, we, TMIN, INFINITY, f);
                code = occ ? 1 : 2;
                if (!occ) {
                    D3 fv = brdf(we, wo, n, m);
                    double pb = bsdf_pdf(we, wo, n, m[6], s.vndf);
                    double den = pe + pb;
                    D3 Le = env_rgb(s, tex);
                    L = L + D3(beta.x * Le.x * fv.x, beta.y * Le.y * fv.y, beta.z * Le.z * fv.z) * (c / den);
                    if (vr) { vr->we = we; vr->Le = Le; vr->eden = den; }
                }
            }
            hash.push((uint32_t)code);
            if (vr) vr->ecode = code;
        }
        const bool continues = (k < nvert) || s.has_env;
        // secondary (direction-space) silhouette edge term, backward only
        if (sec && continues && !s.edges.empty() && s.elen_total > 0.0)
            secondary_edge_sample(s, x, n, wo, f, m, beta, k, nvert - k, ctr, key, *sec, sech, vr);
        // continuation by sampling the BRDF mixture
        if (!continues) break;
        double u[4];
        draw4(ctr, k, 2, key.k0, key.k1, u);
        D3 wi;
        int lobe = bsdf_sample(u, wo, n, m[6], s.vndf, wi);
        double ci = dot(n, wi);
        double pb = bsdf_pdf(wi, wo, n, m[6], s.vndf);
        hash.push((uint32_t)lobe);
        if (!(ci > 0.0) || !(pb > 0.0)) { hash.push(0u); break; }
        hash.push(1u);
        D3 fv = brdf(wi, wo, n, m);
        beta = D3(beta.x * fv.x * ci / pb, beta.y * fv.y * ci / pb, beta.z * fv.z * ci / pb);
        if (vr) { vr->cont = 1; vr->wi = wi; vr->pb = pb; }
        p_prev = pb;
        o = x; d = wi; exclude = f;
    }
    for (uint32_t w : secbuf) hash.push(w);
    return L;
}

// incoming radiance along a secondary-edge side ray, estimated with the
// remaining vertex budget (its own counter domain, shared by both sides)
static D3 L_in_side(const Scene& s, const D3& x, const D3& dir, int exclude, int budget, const Ctr& ctr,
                    const Key& key, Hash& hash) {
    return trace_estimator(s, x, dir, exclude, budget, true, ctr, key, hash, nullptr, nullptr);
}

// --------------------------------------------------------------------------
// replay of a recorded main path with scalar type T (double or dual): the
// derivative of the per-sample estimator at fixed sampled directions, with
// pdfs, MIS weights and visibility held constant, point-light directions and
// hit points attached to the geometry.  Returns sum_c w_c L_c plus the
// secondary-edge pseudo term c * m . (-x_k) whose x-derivative carries the
// motion of the shading point.
// --------------------------------------------------------------------------
template <class T> struct DT { static const int N = 0, FB = 0, MV = 0, MF = 0; };
template <> struct DT<Dual<48>> { static const int N = 48, FB = 27, MV = 9, MF = 3; };
template <> struct DT<Dual<128>> { static const int N = 128, FB = 72, MV = 24, MF = 8; };

template <class T> static T seeded(double v, int slot) { (void)slot; return T(v); }
template <> Dual<48> seeded<Dual<48>>(double v, int slot) { Dual<48> r(v); if (slot >= 0) r.d[slot] = 1.0; return r; }
template <> Dual<128> seeded<Dual<128>>(double v, int slot) { Dual<128> r(v); if (slot >= 0) r.d[slot] = 1.0; return r; }

struct PView {                 // local parameters of one path: its vertices' texels and face vertices
    const Scene* s = nullptr;
    int nvs = 0, vids[3 * MAXV];
    int nts = 0;
    long long tids[MAXV];
    int vslot(int v) const { for (int i = 0; i < nvs; ++i) if (vids[i] == v) return i; return -1; }
    int tslot(long long t) const { for (int i = 0; i < nts; ++i) if (tids[i] == t) return i; return -1; }
    void add_vertex(int f, long long tex) {
        if (tslot(tex) < 0) tids[nts++] = tex;
        for (int k = 0; k < 3; ++k) { int v = s->F[3 * f + k]; if (vslot(v) < 0) vids[nvs++] = v; }
    }
};

struct Perturb { int kind = -1, index = -1; double delta = 0.0; };   // kind 0: V coord, 1: material

template <class T> static V3<T> pvert(const PView& P, int v, const Perturb& pt) {
    D3 p = P.s->vert(v);
    if (pt.kind == 0 && pt.index / 3 == v) p[pt.index % 3] += pt.delta;
    int sl = DT<T>::N ? P.vslot(v) : -1;
    if (sl < 0) return V3<T>(T(p.x), T(p.y), T(p.z));
    return V3<T>(seeded<T>(p.x, 3 * sl), seeded<T>(p.y, 3 * sl + 1), seeded<T>(p.z, 3 * sl + 2));
}

template <class T> static void pmat(const PView& P, long long tex, const Perturb& pt, T out[7]) {
    int sl = DT<T>::N ? P.tslot(tex) : -1;
    for (int c = 0; c < 7; ++c) {
        double v = P.s->mat[7 * tex + c];
        if (pt.kind == 1 && pt.index == 7 * tex + c) v += pt.delta;
        out[c] = sl < 0 ? T(v) : seeded<T>(v, DT<T>::FB + 7 * sl + c);
    }
}

template <class T>
static T replay(const Scene& s, const PRec& R, const double w[3], bool interior, bool secondary,
                const PView& P, const Perturb& pt) {
    V3<T> L, beta(T(1.0), T(1.0), T(1.0));
    V3<T> xprev = lift<T>(R.o);
    T extra(0.0);
    for (int k = 0; k < R.nv; ++k) {
        const VRec& vr = R.v[k];
        D3 dir = (k == 0) ? R.d : R.v[k - 1].wi;
        int f = vr.face;
        V3<T> v0 = pvert<T>(P, s.F[3 * f], pt), v1 = pvert<T>(P, s.F[3 * f + 1], pt),
              v2 = pvert<T>(P, s.F[3 * f + 2], pt);
        V3<T> x = plane_hit(xprev, lift<T>(dir), v0, v1, v2);
        V3<T> n = normalize(cross(v1 - v0, v2 - v0));
        if (vr.flip) n = -n;
        V3<T> wo = lift<T>(vr.wo);
        T m[7];
        pmat<T>(P, vr.tex, pt, m);
        V3<T> C;
        for (int l = 0; l < s.nl; ++l) {
            if (vr.lcode[l] != 2) continue;
            const double* lt = &s.lights[6 * l];
            V3<T> dl = V3<T>(T(lt[0]), T(lt[1]), T(lt[2])) - x;
            T r2 = dot(dl, dl);
            T r = sqrt(r2);
            V3<T> wl = dl * (1.0 / r);
            T c = dot(n, wl);
            V3<T> fv = brdf(wl, wo, n, m);
            T g = c / r2;
            C = C + V3<T>(fv.x * (lt[3] * g), fv.y * (lt[4] * g), fv.z * (lt[5] * g));
        }
        if (vr.ecode == 2) {
            V3<T> we = lift<T>(vr.we);
            V3<T> fv = brdf(we, wo, n, m);
            T g = dot(n, we) / vr.eden;
            C = C + V3<T>(fv.x * (vr.Le.x * g), fv.y * (vr.Le.y * g), fv.z * (vr.Le.z * g));
        }
        L = L + V3<T>(beta.x * C.x, beta.y * C.y, beta.z * C.z);
        if (secondary && vr.sec)
            extra = extra - (x.x * vr.sec_m.x + x.y * vr.sec_m.y + x.z * vr.sec_m.z) * vr.sec_c;
        if (vr.cont) {
            V3<T> wi = lift<T>(vr.wi);
            V3<T> fv = brdf(wi, wo, n, m);
            T g = dot(n, wi) / vr.pb;
            V3<T> Tk(fv.x * g, fv.y * g, fv.z * g);
            if (vr.esc)
                L = L + V3<T>(beta.x * Tk.x * vr.esc_val.x, beta.y * Tk.y * vr.esc_val.y, beta.z * Tk.z * vr.esc_val.z);
            beta = V3<T>(beta.x * Tk.x, beta.y * Tk.y, beta.z * Tk.z);
        }
        xprev = x;
    }
    T out = extra;
    if (interior) out = out + (L.x * w[0] + L.y * w[1] + L.z * w[2]);
    return out;
}

// scatter the tangents of a dual loss into the dense gradient
template <class T> static void scatter(const PView& P, const T& loss, Grad& g) {
    for (int i = 0; i < P.nvs; ++i)
        for (int c = 0; c < 3; ++c) g.dV[3 * P.vids[i] + c] += loss.d[3 * i + c];
    for (int i = 0; i < P.nts; ++i)
        for (int c = 0; c < 7; ++c) g.dM[7 * P.tids[i] + c] += loss.d[DT<T>::FB + 7 * i + c];
}

static void path_gradient(const Scene& s, const PRec& R, const double w[3], bool interior, bool secondary,
                          int bounces, Grad& g) {
    PView P; P.s = &s;
    for (int k = 0; k < R.nv; ++k) P.add_vertex(R.v[k].face, R.v[k].tex);
    if (bounces <= 3) {
        Perturb none;
        Dual<48> l = replay<Dual<48>>(s, R, w, interior, secondary, P, none);
        scatter(P, l, g);
    } else {
        Perturb none;
        Dual<128> l = replay<Dual<128>>(s, R, w, interior, secondary, P, none);
        scatter(P, l, g);
    }
}

// --------------------------------------------------------------------------
// sample enumeration shared with the GPU (canonical order for masks/hashes):
// path g = (pixel offset of view v + y*W + x) * spp + j ; primary edge samples
// of view v at offset sum_{u<v} N_e(u) with N_e = round(ratio * W*H*spp).
// --------------------------------------------------------------------------
struct Views {
    std::vector<Cam> cams;
    std::vector<int64_t> pixoff, eoff, ne;
};

static Views make_views(const double* cams, const int* res, int ncam, int spp, double ratio) {
    Views v;
    int64_t po = 0, eo = 0;
    for (int i = 0; i < ncam; ++i) {
        v.cams.push_back(make_cam(cams + 10 * i, res[2 * i], res[2 * i + 1]));
        v.pixoff.push_back(po);
        v.eoff.push_back(eo);
        int64_t n = (int64_t)std::llround(ratio * (double)res[2 * i] * (double)res[2 * i + 1] * (double)spp);
        v.ne.push_back(n);
        po += (int64_t)res[2 * i] * res[2 * i + 1];
        eo += n;
    }
    v.pixoff.push_back(po);
    v.eoff.push_back(eo);
    return v;
}

// main-path estimate for one (view, pixel, sample)
static D3 pixel_sample(const Scene& s, const Cam& c, int view, int px, int py, int j, int spp, int bounces,
                       const Key& key, Hash& h, PRec* rec, SecCtx* sec) {
    Ctr ctr{(uint32_t)(py * c.W + px), ((uint32_t)view << 16) | (uint32_t)j, 0u, 0u};
    double u[4];
    draw4(ctr, 0, 0, key.k0, key.k1, u);
    D3 d = cam_dir(c, px + u[0], py + u[1]);
    (void)spp;
    return trace_estimator(s, c.eye, d, -1, bounces, false, ctr, key, h, rec, sec);
}

template <class F> static void parallel_for(int64_t n, int nthreads, F fn) {
    if (nthreads <= 1 || n < 2) { for (int64_t i = 0; i < n; ++i) fn(i, 0); return; }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
        th.emplace_back([&, t]() {
            for (;;) {
                int64_t b = next.fetch_add(64);
                if (b >= n) break;
                for (int64_t i = b; i < std::min(n, b + 64); ++i) fn(i, t);
            }
        });
    for (auto& x : th) x.join();
}

// primary (screen-space) edge term of one view; see the header comment of
// or_backward for the estimator
struct EdgeView {
    std::vector<double> cdf;
    double total = 0.0;
};

static bool front_facing(const Scene& s, int f, const D3& eye) {
    D3 v0 = s.vert(s.F[3 * f]);
    D3 N = face_N(s, f);
    D3 w = eye - v0;
    return N.x * w.x + N.y * w.y + N.z * w.z > 0.0;
}

// The image of edge E in view c, as the primary edge term integrates over it.
// Near plane: the part of the edge with depth > ZNEAR is kept; an endpoint at
// or behind that depth is replaced by the point of the edge at depth ZNEAR,
// sa (sb) being the fraction of the edge cut away at va (vb).  The kept
// segment projects to the straight image segment x(t) = A + t (B - A),
// t in [0, 1]; only its part inside the image rectangle [0, W] x [0, H]
// (the range [t0, t1] of t, Liang-Barsky) can contribute, since points outside
// the image have no pixel.  ok is false when nothing is left.
struct ScreenEdge {
    bool ok = false;
    double ax = 0, ay = 0, bx = 0, by = 0;
    double sa = 0, sb = 0, t0 = 0, t1 = 1;
};

static ScreenEdge screen_edge(const Scene& s, const Cam& c, const Edge& E) {
    ScreenEdge r;
    D3 a = s.vert(E.va), b = s.vert(E.vb);
    double ax, ay, az, bx, by, bz;
    project<double>(c, a, ax, ay, az);
    project<double>(c, b, bx, by, bz);
    if (!(az > ZNEAR) && !(bz > ZNEAR)) return r;
    if (!(az > ZNEAR)) {
        r.sa = (ZNEAR - az) / (bz - az);
        D3 ac(a.x + (b.x - a.x) * r.sa, a.y + (b.y - a.y) * r.sa, a.z + (b.z - a.z) * r.sa);
        project<double>(c, ac, ax, ay, az);
    }
    if (!(bz > ZNEAR)) {
        r.sb = (ZNEAR - bz) / (az - bz);
        D3 bc(b.x + (a.x - b.x) * r.sb, b.y + (a.y - b.y) * r.sb, b.z + (a.z - b.z) * r.sb);
        project<double>(c, bc, bx, by, bz);
    }
    r.ax = ax; r.ay = ay; r.bx = bx; r.by = by;
    const double dx = bx - ax, dy = by - ay;
    // x(t) inside the rectangle: p t <= q for the four sides, in a fixed order
    double t0 = 0.0, t1 = 1.0;
    const double P[4] = {-dx, dx, -dy, dy};
    const double Q[4] = {ax, (double)c.W - ax, ay, (double)c.H - ay};
    for (int i = 0; i < 4; ++i) {
        if (P[i] == 0.0) {
            if (Q[i] < 0.0) return r;
            continue;
        }
        const double q = Q[i] / P[i];
        if (P[i] < 0.0) { if (q > t0) t0 = q; }
        else { if (q < t1) t1 = q; }
    }
    if (!(t0 < t1)) return r;
    r.t0 = t0; r.t1 = t1;
    r.ok = true;
    return r;
}

static EdgeView primary_cdf(const Scene& s, const Cam& c) {
    EdgeView ev;
    const size_t ne = s.edges.size();
    std::vector<double> cum(ne + 1, 0.0);
    double acc = 0.0;
    for (size_t e = 0; e < ne; ++e) {
        const Edge& E = s.edges[e];
        double len = 0.0;
        bool cand = E.f2 < 0 || front_facing(s, E.f1, c.eye) || front_facing(s, E.f2, c.eye);
        if (cand) {
            ScreenEdge se = screen_edge(s, c, E);
            if (se.ok) {
                double dx = se.bx - se.ax, dy = se.by - se.ay;
                len = (se.t1 - se.t0) * std::sqrt(dx * dx + dy * dy);
            }
        }
        acc += len;
        cum[e + 1] = acc;
    }
    ev.total = acc;
    ev.cdf.assign(ne + 1, 0.0);
    for (size_t e = 0; e <= ne; ++e) ev.cdf[e] = acc > 0 ? cum[e] / acc : 0.0;
    return ev;
}

static void primary_edge_sample(const Scene& s, const Cam& c, const EdgeView& ev, int view, int64_t si, int64_t ne,
                                int spp, int bounces, const Key& key, const float* d_img_view,
                                Hash& h, Grad& g, bool& computed) {
    (void)spp;
    computed = false;
    if (!(ev.total > 0.0)) return;
    double u[4];
    Ctr ctr{(uint32_t)si, (uint32_t)view << 16, 0u, 1u};
    draw4(ctr, 0, 3, key.k0, key.k1, u);
    // stratified over the view's ne samples: sample si takes the CDF at (si + u0) / ne
    int e = cdf_find(ev.cdf.data(), (int)s.edges.size(), ((double)si + u[0]) / (double)ne);
    const Edge& E = s.edges[e];
    const ScreenEdge se = screen_edge(s, c, E);     // ok: only such edges have weight
    // the point is uniform on the visible part [t0, t1] of the image segment
    double t = se.t0 + u[1] * (se.t1 - se.t0);
    double ax = se.ax, ay = se.ay, bx = se.bx, by = se.by;
    double xs = (1.0 - t) * ax + t * bx, ys = (1.0 - t) * ay + t * by;
    int px = (int)std::floor(xs), py = (int)std::floor(ys);
    bool inside = xs >= 0.0 && ys >= 0.0 && px < c.W && py < c.H;
    const float* dimg = inside ? d_img_view + 3 * ((int64_t)py * c.W + px) : nullptr;
    if (inside && dimg[0] == 0.0f && dimg[1] == 0.0f && dimg[2] == 0.0f) return;   // contributes zero
    computed = true;
    h.push((uint32_t)e);
    if (!inside) { h.push(0u); return; }
    h.push(1u);
    double dx = bx - ax, dy = by - ay;
    double l = std::sqrt(dx * dx + dy * dy);
    double nx = -dy / l, ny = dx / l;
    D3 dm = cam_dir(c, xs - EPS_PRIMARY * nx, ys - EPS_PRIMARY * ny);
    D3 dp = cam_dir(c, xs + EPS_PRIMARY * nx, ys + EPS_PRIMARY * ny);
    // each side path hashes its own decisions; the sample hash takes both results
    Hash hm, hp;
    hm.on = hp.on = h.on;
    // When the first surface both side rays meet is the same face, the edge
    // point is hidden behind it: the image has no jump there, and the two paths
    // would differ only by the smooth change of the integrand across 2 eps (plus
    // the noise of decisions that flip between them).  Both sides count as zero.
    double tm, tp;
    const int fm = closest_hit(s, c.eye, dm, TMIN, -1, tm), fp = closest_hit(s, c.eye, dp, TMIN, -1, tp);
    D3 Lm(0, 0, 0), Lp(0, 0, 0);
    if (fm == fp) {
        push_face(hm, fm);
        push_face(hp, fp);
    } else {
        Lm = trace_estimator(s, c.eye, dm, -1, bounces, false, ctr, key, hm, nullptr, nullptr);
        Lp = trace_estimator(s, c.eye, dp, -1, bounces, false, ctr, key, hp, nullptr, nullptr);
    }
    h.push(hm.h);
    h.push(hp.h);
    double cc = 0.0;
    for (int ch = 0; ch < 3; ++ch) cc += (double)dimg[ch] * (Lm[ch] - Lp[ch]);
    cc *= ev.total / (double)ne;
    // normal velocity of the image point x = (1 - t) pi(a') + t pi(b'), with the
    // (near-plane) segment ends a' = va + sa (vb - va), b' = vb + sb (va - vb) and
    // t, sa, sb held fixed (they only slide the point along the image line):
    // 6-tangent dual numbers, slots 0..2 the coordinates of va, 3..5 of vb
    typedef Dual<48> DD;
    D3 pa = s.vert(E.va), pb = s.vert(E.vb);
    V3<DD> A3(seeded<DD>(pa.x, 0), seeded<DD>(pa.y, 1), seeded<DD>(pa.z, 2));
    V3<DD> B3(seeded<DD>(pb.x, 3), seeded<DD>(pb.y, 4), seeded<DD>(pb.z, 5));
    V3<DD> ac = A3 + (B3 - A3) * se.sa, bc = B3 + (A3 - B3) * se.sb;
    DD sxa, sya, sza, sxb, syb, szb;
    project<DD>(c, ac, sxa, sya, sza);
    project<DD>(c, bc, sxb, syb, szb);
    DD X = sxa * (1.0 - t) + sxb * t, Y = sya * (1.0 - t) + syb * t;
    for (int k = 0; k < 3; ++k) {
        g.dV[3 * E.va + k] += cc * (X.d[k] * nx + Y.d[k] * ny);
        g.dV[3 * E.vb + k] += cc * (X.d[3 + k] * nx + Y.d[3 + k] * ny);
    }
}

// --------------------------------------------------------------------------
// point-light shadow boundaries seen directly by the camera (the image-space
// edge term of a shadow; the shadow of an occluder edge e under light l is the
// central projection of e from the light onto the receiving surface).
//
// Candidate edges for light l: boundary edges and edges whose two faces lie on
// opposite sides of the light position (fp64 test, fixed operation order).  An
// edge is chosen with probability proportional to its 3-D length, a point
// y = va + t (vb - va) on it with t uniform; the light ray through y continues
// to the receiver point z (first hit from y, the edge's faces excluded).  When
// z is seen by the camera, its screen point s = pi(z) lies on the image curve of
// the shadow boundary; with tau = ds/dt and n the screen normal perp(tau)/|tau|,
// the receiver points under s -/+ 1e-3 px n take the light's visibility V-, V+,
// and the sample adds d_image(pixel of s) . (V- - V+) L_l(z) (n . ds/dtheta)
// |tau| W_l / (|vb - va| N_s) to dLoss/dtheta, where L_l(z) is the unshadowed
// radiance of light l reflected at z toward the camera, W_l the total candidate
// length and N_s the number of samples of the (view, light) pair.  theta moves
// the edge's endpoints and the receiver face's vertices; the light is fixed.
// --------------------------------------------------------------------------
struct LightEdges {
    std::vector<double> cdf;
    double total = 0.0;
};

static LightEdges light_cdf(const Scene& s, int l) {
    LightEdges le;
    const size_t ne = s.edges.size();
    const double* lt = &s.lights[6 * l];
    D3 pl(lt[0], lt[1], lt[2]);
    std::vector<double> cum(ne + 1, 0.0);
    double acc = 0.0;
    for (size_t e = 0; e < ne; ++e) {
        const Edge& E = s.edges[e];
        D3 va = s.vert(E.va), vb = s.vert(E.vb);
        bool cand = E.f2 < 0;
        if (!cand) {
            double s1 = dot(face_N(s, E.f1), pl - va), s2 = dot(face_N(s, E.f2), pl - va);
            cand = (s1 > 0.0) != (s2 > 0.0);
        }
        acc += cand ? length(vb - va) : 0.0;
        cum[e + 1] = acc;
    }
    le.total = acc;
    le.cdf.assign(ne + 1, 0.0);
    for (size_t e = 0; e <= ne; ++e) le.cdf[e] = acc > 0 ? cum[e] / acc : 0.0;
    return le;
}

static void shadow_edge_sample(const Scene& s, const Cam& c, const LightEdges& le, int view, int l, int64_t si,
                               int64_t ns, const Key& key, const float* d_img_view, Hash& h, Grad& g) {
    if (!(le.total > 0.0)) return;
    double u[4];
    Ctr ctr{(uint32_t)si, ((uint32_t)view << 16) | (uint32_t)l, 0u, 3u};
    draw4(ctr, 0, 3, key.k0, key.k1, u);
    // stratified over the ns samples of the (view, light) pair
    const int e = cdf_find(le.cdf.data(), (int)s.edges.size(), ((double)si + u[0]) / (double)ns);
    const double t = u[1];
    h.push((uint32_t)e);
    const Edge& E = s.edges[e];
    const double* lt = &s.lights[6 * l];
    const D3 pl(lt[0], lt[1], lt[2]), I(lt[3], lt[4], lt[5]);
    const D3 va = s.vert(E.va), vb = s.vert(E.vb);
    const D3 y = va + (vb - va) * t;
    const D3 w = normalize(y - pl);
    double tr;
    const int fr = closest_hit(s, y, w, TMIN, E.f1, tr);
    push_face(h, fr);
    if (fr < 0 || fr == E.f2) return;
    const D3 z = y + w * tr;
    double tc;
    const int fc = closest_hit(s, c.eye, normalize(z - c.eye), TMIN, -1, tc);
    const bool vis = fc == fr;
    h.push(vis ? 2u : 1u);
    if (!vis) return;
    // the receiver point and its screen point as functions of (t, va, vb, r0, r1, r2)
    typedef Dual<48> T;
    const int rv[3] = {s.F[3 * fr], s.F[3 * fr + 1], s.F[3 * fr + 2]};
    V3<T> A(seeded<T>(va.x, 1), seeded<T>(va.y, 2), seeded<T>(va.z, 3));
    V3<T> Bv(seeded<T>(vb.x, 4), seeded<T>(vb.y, 5), seeded<T>(vb.z, 6));
    V3<T> R[3];
    for (int k = 0; k < 3; ++k) {
        D3 p = s.vert(rv[k]);
        R[k] = V3<T>(seeded<T>(p.x, 7 + 3 * k), seeded<T>(p.y, 8 + 3 * k), seeded<T>(p.z, 9 + 3 * k));
    }
    T tt = seeded<T>(t, 0);
    V3<T> yy = A + (Bv - A) * tt;
    V3<T> P = lift<T>(pl);
    V3<T> Nr = cross(R[1] - R[0], R[2] - R[0]);
    T lam = dot(Nr, R[0] - P) / dot(Nr, yy - P);
    V3<T> zz = P + (yy - P) * lam;
    T sx, sy, sz;
    project<T>(c, zz, sx, sy, sz);
    const double xs = sx.v, ys = sy.v;
    const int px = (int)std::floor(xs), py = (int)std::floor(ys);
    const bool inside = sz.v > ZNEAR && xs >= 0.0 && ys >= 0.0 && px < c.W && py < c.H;
    h.push(inside ? 1u : 0u);
    if (!inside) return;
    const float* dimg = d_img_view + 3 * ((int64_t)py * c.W + px);
    if (dimg[0] == 0.0f && dimg[1] == 0.0f && dimg[2] == 0.0f) return;
    const double tx = sx.d[0], ty = sy.d[0];
    const double tl = std::sqrt(tx * tx + ty * ty);
    if (!(tl > 0.0)) return;
    const double nx = -ty / tl, ny = tx / tl;
    // light visibility on both sides, at the receiver plane under the side points
    const D3 r0 = s.vert(rv[0]);
    const D3 Nd = face_N(s, fr);
    int vsd[2];
    for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? -1.0 : 1.0;
        const D3 dd = cam_dir(c, xs + sg * EPS_PRIMARY * nx, ys + sg * EPS_PRIMARY * ny);
        const D3 zs = c.eye + dd * (dot(Nd, r0 - c.eye) / dot(Nd, dd));
        const D3 wl = pl - zs;
        const double r = length(wl);
        vsd[side] = any_hit(s, zs, wl * (1.0 / r), TMIN, r * (1.0 - SHADOW_SHRINK), fr) ? 0 : 1;
        h.push((uint32_t)vsd[side]);
    }
    if (vsd[0] == vsd[1]) return;
    // unshadowed radiance of light l at z toward the camera
    const D3 wo = normalize(c.eye - z);
    D3 n = normalize(Nd);
    if (dot(n, wo) < 0.0) n = -n;
    const D3 dl = pl - z;
    const double r2 = dot(dl, dl);
    const D3 wl = dl * (1.0 / std::sqrt(r2));
    const double cl = dot(n, wl);
    if (!(cl > 0.0)) return;
    const double* m = &s.mat[7 * texel_of(s, fr, z)];
    const D3 fv = brdf(wl, wo, n, m);
    double cc = 0.0;
    for (int ch = 0; ch < 3; ++ch) cc += (double)dimg[ch] * (vsd[0] - vsd[1]) * fv[ch] * I[ch] * cl / r2;
    cc *= tl * le.total / (length(vb - va) * (double)ns);
    auto vn = [&](int slot) { return nx * sx.d[slot] + ny * sy.d[slot]; };
    for (int k = 0; k < 3; ++k) {
        g.dV[3 * E.va + k] += cc * vn(1 + k);
        g.dV[3 * E.vb + k] += cc * vn(4 + k);
        for (int q = 0; q < 3; ++q) g.dV[3 * rv[q] + k] += cc * vn(7 + 3 * q + k);
    }
}

// --------------------------------------------------------------------------
// LBVH reference (integer Morton codes, bit-exact spec shared with the GPU):
// float32 centroids and scale, 10 bits per axis (x highest), key = morton<<32 |
// face, ascending sort, Karras 2012 hierarchy, min/max refit.
// --------------------------------------------------------------------------
static inline uint32_t spread10(uint32_t v) {
    uint32_t r = 0;
    for (int i = 0; i < 10; ++i) r |= ((v >> i) & 1u) << (3 * i);
    return r;
}

static inline int clz64(uint64_t x) { return x ? __builtin_clzll(x) : 64; }

// Radix tree (Karras 2012) over n primitive boxes mn/mx (float [n,3]):
// centres (mn + mx) / 2, 30-bit Morton codes over cubic cells, keys
// morton << 32 | primitive, sorted; children, parents and refitted boxes.
static void radix_tree_of_boxes(const std::vector<float>& mn, const std::vector<float>& mx, int nf, uint64_t* keys,
                                int* child, int* parent, float* aabb) {
    std::vector<float> ce(3 * (size_t)nf);
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            volatile float sum = mn[3 * f + k] + mx[3 * f + k];
            float cc = sum * 0.5f;
            ce[3 * f + k] = cc;
            lo[k] = std::min(lo[k], cc); hi[k] = std::max(hi[k], cc);
        }
    // one scale for all three axes (cells are cubes): 1024 cells along the
    // longest extent of the centroid box
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, (double)hi[k] - (double)lo[k]);
    float sc[3];
    for (int k = 0; k < 3; ++k) sc[k] = ext > 0.0 ? (float)(1024.0 / ext) : 0.0f;
    std::vector<uint64_t> kv(nf);
    for (int f = 0; f < nf; ++f) {
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            volatile float dlt = ce[3 * f + k] - lo[k];
            volatile float pr = dlt * sc[k];
            float fl = std::floor((float)pr);
            int qi = (int)fl;
            q[k] = (uint32_t)std::max(0, std::min(1023, qi));
        }
        uint32_t morton = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        kv[f] = ((uint64_t)morton << 32) | (uint32_t)f;
    }
    std::sort(kv.begin(), kv.end());
    for (int i = 0; i < nf; ++i) keys[i] = kv[i];
    const int n = nf;
    const int LEAF = (int)0x80000000;
    auto delta = [&](int i, int j) -> int {
        if (j < 0 || j > n - 1) return -1;
        return clz64(kv[i] ^ kv[j]);
    };
    for (int i = 0; i < 2 * n - 1; ++i) parent[i] = -1;
    for (int i = 0; i < n - 1; ++i) {
        int d = delta(i, i + 1) > delta(i, i - 1) ? 1 : -1;
        int dmin = delta(i, i - d);
        int lmax = 2;
        while (delta(i, i + lmax * d) > dmin) lmax *= 2;
        int l = 0;
        for (int tt = lmax / 2; tt >= 1; tt /= 2)
            if (delta(i, i + (l + tt) * d) > dmin) l += tt;
        int j = i + l * d;
        int dnode = delta(i, j);
        int sp = 0, tt = l;
        do {
            tt = (tt + 1) / 2;
            if (delta(i, i + (sp + tt) * d) > dnode) sp += tt;
        } while (tt > 1);
        int split = i + sp * d + std::min(d, 0);
        int left = (std::min(i, j) == split) ? (LEAF | split) : split;
        int right = (std::max(i, j) == split + 1) ? (LEAF | (split + 1)) : split + 1;
        child[2 * i] = left; child[2 * i + 1] = right;
        parent[(left & LEAF) ? (n - 1) + (left & 0x7FFFFFFF) : left] = i;
        parent[(right & LEAF) ? (n - 1) + (right & 0x7FFFFFFF) : right] = i;
    }
    // leaves, then internal nodes by a post-order walk
    for (int i = 0; i < n; ++i) {
        int f = (int)(kv[i] & 0xFFFFFFFFu);
        float* b = aabb + 6 * ((n - 1) + i);
        for (int k = 0; k < 3; ++k) { b[k] = mn[3 * f + k]; b[3 + k] = mx[3 * f + k]; }
    }
    if (n < 2) return;
    std::vector<int> order, st{0};
    while (!st.empty()) {
        int i = st.back(); st.pop_back(); order.push_back(i);
        for (int c = 0; c < 2; ++c) if (!(child[2 * i + c] & LEAF)) st.push_back(child[2 * i + c]);
    }
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
        int i = *it;
        float* b = aabb + 6 * i;
        const float* cb[2];
        for (int c = 0; c < 2; ++c) {
            int ch = child[2 * i + c];
            cb[c] = aabb + 6 * ((ch & LEAF) ? (n - 1) + (ch & 0x7FFFFFFF) : ch);
        }
        for (int k = 0; k < 3; ++k) {
            b[k] = std::min(cb[0][k], cb[1][k]);
            b[3 + k] = std::max(cb[0][3 + k], cb[1][3 + k]);
        }
    }
}

static void lbvh_reference(const float* V, int nv, const int* F, int nf, uint64_t* keys, int* child,
                           int* parent, float* aabb) {
    (void)nv;
    std::vector<float> mn(3 * (size_t)nf), mx(3 * (size_t)nf);
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            float a = V[3 * F[3 * f] + k], b = V[3 * F[3 * f + 1] + k], c = V[3 * F[3 * f + 2] + k];
            mn[3 * f + k] = std::min(a, std::min(b, c));
            mx[3 * f + k] = std::max(a, std::max(b, c));
        }
    radix_tree_of_boxes(mn, mx, nf, keys, child, parent, aabb);
}

// Edge tree of the secondary-edge importance hierarchy: the radix tree over the
// edges' boxes, every node carrying the float sum of the lengths below it
// (a leaf: its edge's length rounded to float; a node: left + right).
static void build_edge_tree(Scene& s) {
    EdgeTree& T = s.etree;
    const int n = (int)s.edges.size();
    T.n = n;
    T.keys.assign(n, 0);
    T.child.assign(2 * (size_t)std::max(n - 1, 0), 0);
    T.parent.assign(2 * (size_t)n - (n > 0 ? 1 : 0), -1);
    T.box.assign(6 * T.parent.size(), 0.0f);
    T.len.assign(T.parent.size(), 0.0f);
    T.nbox.assign(6 * T.parent.size(), 0.0f);
    if (n == 0) return;
    std::vector<float> mn(3 * (size_t)n), mx(3 * (size_t)n);
    for (int e = 0; e < n; ++e)
        for (int k = 0; k < 3; ++k) {
            const float a = (float)s.V[3 * s.edges[e].va + k], c = (float)s.V[3 * s.edges[e].vb + k];
            mn[3 * e + k] = std::min(a, c);
            mx[3 * e + k] = std::max(a, c);
        }
    radix_tree_of_boxes(mn, mx, n, T.keys.data(), T.child.data(), T.parent.data(), T.box.data());
    for (int i = 0; i < n; ++i) {
        const Edge& E = s.edges[(int)(T.keys[i] & 0xFFFFFFFFu)];
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double d = (double)(float)s.V[3 * E.vb + k] - (double)(float)s.V[3 * E.va + k];
            d2 += d * d;
        }
        T.len[(n - 1) + i] = (float)std::sqrt(d2);
        // unit normals of the adjacent faces, from the float vertices in double,
        // rounded to float; a boundary edge (always a silhouette) or a degenerate
        // face takes the whole cube [-1, 1]^3, which never culls
        float* nb = &T.nbox[6 * ((size_t)(n - 1) + i)];
        for (int k = 0; k < 3; ++k) { nb[k] = -1.0f; nb[3 + k] = 1.0f; }
        if (E.f2 < 0) continue;
        float un[2][3];
        bool ok = true;
        for (int j = 0; j < 2; ++j) {
            const int f = j == 0 ? E.f1 : E.f2;
            double q[3][3];
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) q[a][k] = (double)(float)s.V[3 * s.F[3 * f + a] + k];
            const double e1[3] = {q[1][0] - q[0][0], q[1][1] - q[0][1], q[1][2] - q[0][2]};
            const double e2[3] = {q[2][0] - q[0][0], q[2][1] - q[0][1], q[2][2] - q[0][2]};
            const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                 e1[0] * e2[1] - e1[1] * e2[0]};
            const double l = std::sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
            if (!(l > 0.0) || !std::isfinite(l)) { ok = false; break; }
            for (int k = 0; k < 3; ++k) un[j][k] = (float)(c[k] / l);
        }
        if (!ok) continue;
        for (int k = 0; k < 3; ++k) {
            nb[k] = std::min(un[0][k], un[1][k]);
            nb[3 + k] = std::max(un[0][k], un[1][k]);
        }
    }
    if (n < 2) return;
    const int LEAF = (int)0x80000000;
    std::vector<int> order, st{0};
    while (!st.empty()) {
        int i = st.back(); st.pop_back(); order.push_back(i);
        for (int c = 0; c < 2; ++c) if (!(T.child[2 * i + c] & LEAF)) st.push_back(T.child[2 * i + c]);
    }
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
        const int i = *it;
        float l[2];
        size_t ci[2];
        for (int c = 0; c < 2; ++c) {
            const int ch = T.child[2 * i + c];
            ci[c] = (ch & LEAF) ? (size_t)(n - 1) + (ch & 0x7FFFFFFF) : (size_t)ch;
            l[c] = T.len[ci[c]];
        }
        T.len[i] = l[0] + l[1];
        for (int k = 0; k < 3; ++k) {
            T.nbox[6 * (size_t)i + k] = std::min(T.nbox[6 * ci[0] + k], T.nbox[6 * ci[1] + k]);
            T.nbox[6 * (size_t)i + 3 + k] = std::max(T.nbox[6 * ci[0] + 3 + k], T.nbox[6 * ci[1] + 3 + k]);
        }
    }
}

// Importance of a tree node seen from the shading point p with normal nrm
// (float, contraction off, this operation order on both implementations):
// zero when the node's box lies wholly behind the tangent plane of p (such
// edges contribute nothing), otherwise the node's length over the squared
// distance to the box centre plus the squared half diagonal.  The plane test
// keeps a margin of 2^-16 of the box's size plus distance, so that a box lying
// in the plane (edges coplanar with the shading point, as on a flat floor)
// keeps its weight whatever the rounding of p: the cut only ever keeps extra
// boxes, whose edges then contribute zero, and never drops a contributing one.
// With sil, the node is also zero when no edge in it can be a silhouette from
// p: an edge is one when p lies in front of one adjacent face plane and behind
// the other, so a node whose faces all have p on the same side (the bound
// N.(p - q) over q in the box and N in the node's normal box keeps one sign,
// beyond the same margin) holds none.
static float edge_node_weight(const EdgeTree& T, int code, const float p[3], const float nrm[3], bool sil) {
    const int idx = (code & (int)0x80000000) ? (T.n - 1) + (code & 0x7FFFFFFF) : code;
    const float* bx = &T.box[6 * (size_t)idx];
    const float dx = (bx[0] + bx[3]) * 0.5f - p[0], dy = (bx[1] + bx[4]) * 0.5f - p[1], dz = (bx[2] + bx[5]) * 0.5f - p[2];
    const float ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
    const float reach = (dx * nrm[0] + dy * nrm[1] + dz * nrm[2]) +
                        0.5f * ((std::fabs(nrm[0]) * ex + std::fabs(nrm[1]) * ey) + std::fabs(nrm[2]) * ez);
    const float tol = 0x1p-16f * (((std::fabs(dx) + std::fabs(dy)) + std::fabs(dz)) + ((ex + ey) + ez));
    if (!(reach > -tol)) return 0.0f;
    if (sil) {
        const float* nb = &T.nbox[6 * (size_t)idx];
        const float d[3] = {dx, dy, dz}, e[3] = {ex, ey, ez};
        float lo = 0.0f, hi = 0.0f, rad = 0.0f;
        for (int k = 0; k < 3; ++k) {
            const float a = -nb[k] * d[k], b = -nb[3 + k] * d[k];
            lo = lo + std::min(a, b);
            hi = hi + std::max(a, b);
            rad = rad + std::max(std::fabs(nb[k]), std::fabs(nb[3 + k])) * (0.5f * e[k]);
        }
        if (lo - rad > tol || hi + rad < -tol) return 0.0f;
    }
    const float dl1 = ((std::fabs(dx) + std::fabs(dy)) + std::fabs(dz)) + 0.5f * ((ex + ey) + ez);
    const float cb = (reach + tol) / (dl1 + tol);
    return T.len[idx] * cb / ((dx * dx + dy * dy + dz * dz) + 0.25f * ((ex * ex + ey * ey) + ez * ez));
}

// Stochastic descent of the edge tree: at every node the child is taken with
// probability proportional to its weight, by a fresh uniform per level (level l
// uses component l % 4 of the draw of block 4 + l / 4 at vertex k).  Returns the
// edge (canonical index) and its probability pe, or -1 when every weight is zero.
static int edge_tree_sample(const Scene& s, const D3& x, const D3& nn, const Ctr& ctr, int k, const Key& key,
                            bool sil, float& pe) {
    const EdgeTree& T = s.etree;
    pe = 1.0f;
    if (T.n <= 0) return -1;
    const float p[3] = {(float)x.x, (float)x.y, (float)x.z}, nrm[3] = {(float)nn.x, (float)nn.y, (float)nn.z};
    const int LEAF = (int)0x80000000;
    int code = T.n == 1 ? LEAF : 0;
    double u[4] = {0, 0, 0, 0};
    for (int level = 0; !(code & LEAF); ++level) {
        if (level >= 128) return -1;
        if ((level & 3) == 0) draw4(ctr, k, 4 + (level >> 2), key.k0, key.k1, u);
        const int c0 = T.child[2 * code], c1 = T.child[2 * code + 1];
        const float w0 = edge_node_weight(T, c0, p, nrm, sil), w1 = edge_node_weight(T, c1, p, nrm, sil);
        const float tot = w0 + w1;
        if (!(tot > 0.0f)) return -1;
        const float p0 = w0 / tot;
        if ((float)u[level & 3] < p0) { code = c0; pe *= p0; }
        else { code = c1; pe *= w1 / tot; }
    }
    if (T.n == 1 && !(edge_node_weight(T, LEAF, p, nrm, sil) > 0.0f)) return -1;
    return (int)(T.keys[code & 0x7FFFFFFF] & 0xFFFFFFFFu);
}

// --------------------------------------------------------------------------
// Treelet restructuring of the binary tree (Karras and Aila, HPG 2013: small
// treelets re-arranged into their SAH-optimal topology, bottom-up).  Stated
// here as a definition, in float32 like the tree's boxes, so that every
// comparison is taken in the same precision as on the GPU:
//  - SAH cost of a subtree: a triangle leaf costs the area of its box; an
//    internal node costs C_INNER * area(box) + cost(left) + cost(right);
//    area(b) = 2 ((dx dy + dy dz) + dz dx).
//  - Every internal node r is visited after both of its subtrees (post-order).
//    A node with fewer than TREELET_LEAVES triangles below it is left as it is
//    (its cost: C_INNER * area(box) + (cost(child0) + cost(child1))).
//    Otherwise its treelet: the list starts as (child0, child1); while the list has fewer
//    than TREELET_LEAVES entries and holds an internal node, the internal entry
//    of largest box area (first in list order on ties) is removed and its two
//    children appended.  The removed nodes, r first, are the treelet's
//    internal nodes.
//  - Over the k list entries (bit j of a subset = entry j), opt({j}) = cost of
//    entry j and, for |S| >= 2, opt(S) = C_INNER * area(union of S) +
//    min over P (opt(P) + opt(S \ P)), P = lowest bit of S plus a proper subset
//    `sub` of the rest, sub taken in the order (rest-1)&rest, (sub-1)&rest, ..., 0;
//    the first strict minimum wins.
//  - Rebuild: the internal subsets of the optimal tree in preorder (a stack:
//    pop S, record it, push S\P if internal, then P if internal) take the ids
//    r, then the other treelet internal nodes in ascending id order; node S
//    gets children (P, S \ P), box = union of its entries, cost = opt(S).
// Rounds repeat the whole bottom-up pass.
// --------------------------------------------------------------------------
static const float C_INNER = 1.2f;
static const int TREELET_LEAVES = 7;

static inline float box_area(const float* b) {
    float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return 2.0f * ((dx * dy + dy * dz) + dz * dx);
}

struct TreeRef {
    int n;
    int* child;
    int* parent;
    float* aabb;
    std::vector<float> cost;      // per internal node
    std::vector<int> leaves;      // triangles below each internal node
    static const int LEAF = (int)0x80000000;
    float* box(int code) { return aabb + 6 * ((code & LEAF) ? (size_t)(n - 1) + (code & 0x7FFFFFFF) : (size_t)code); }
    int pidx(int code) const { return (code & LEAF) ? (n - 1) + (code & 0x7FFFFFFF) : code; }
    float code_cost(int code) { return (code & LEAF) ? box_area(box(code)) : cost[code]; }
    int code_leaves(int code) const { return (code & LEAF) ? 1 : leaves[code]; }
};

static void treelet_node(TreeRef& T, int r) {
    const int LEAF = TreeRef::LEAF;
    const int c0 = T.child[2 * r], c1 = T.child[2 * r + 1];
    T.leaves[r] = T.code_leaves(c0) + T.code_leaves(c1);
    if (T.leaves[r] < TREELET_LEAVES) {
        T.cost[r] = C_INNER * box_area(T.box(r)) + (T.code_cost(c0) + T.code_cost(c1));
        return;
    }
    std::vector<int> ent = {c0, c1};
    std::vector<int> inner = {r};
    while ((int)ent.size() < TREELET_LEAVES) {
        int bi = -1;
        float ba = -1.0f;
        for (int i = 0; i < (int)ent.size(); ++i)
            if (!(ent[i] & LEAF)) {
                float a = box_area(T.box(ent[i]));
                if (a > ba) { ba = a; bi = i; }
            }
        if (bi < 0) break;
        int c = ent[bi];
        inner.push_back(c);
        ent.erase(ent.begin() + bi);
        ent.push_back(T.child[2 * c]);
        ent.push_back(T.child[2 * c + 1]);
    }
    const int k = (int)ent.size(), full = (1 << k) - 1;
    std::vector<float> opt(1 << k), area(1 << k);
    std::vector<int> part(1 << k, 0);
    for (int S = 1; S <= full; ++S) {
        float u[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int j = 0; j < k; ++j)
            if (S >> j & 1) {
                const float* bb = T.box(ent[j]);
                for (int q = 0; q < 3; ++q) { u[q] = std::min(u[q], bb[q]); u[3 + q] = std::max(u[3 + q], bb[3 + q]); }
            }
        area[S] = box_area(u);
    }
    for (int j = 0; j < k; ++j) opt[1 << j] = T.code_cost(ent[j]);
    for (int size = 2; size <= k; ++size)
        for (int S = 1; S <= full; ++S) {
            if (__builtin_popcount(S) != size) continue;
            const int lb = S & -S, rest = S ^ lb;
            float best = INFINITY;
            int bp = 0;
            int sub = (rest - 1) & rest;
            for (;;) {
                const int P = lb | sub;
                const float c = opt[P] + opt[S ^ P];
                if (c < best) { best = c; bp = P; }
                if (sub == 0) break;
                sub = (sub - 1) & rest;
            }
            opt[S] = C_INNER * area[S] + best;
            part[S] = bp;
        }
    // preorder of the optimal tree's internal subsets
    std::vector<int> pre, st = {full};
    while (!st.empty()) {
        int S = st.back();
        st.pop_back();
        pre.push_back(S);
        const int P = part[S], Q = S ^ P;
        if (__builtin_popcount(Q) > 1) st.push_back(Q);
        if (__builtin_popcount(P) > 1) st.push_back(P);
    }
    std::vector<int> ids(inner.begin() + 1, inner.end());
    std::sort(ids.begin(), ids.end());
    ids.insert(ids.begin(), r);
    auto code_of = [&](int X) -> int {
        if (__builtin_popcount(X) == 1) return ent[__builtin_ctz(X)];
        for (size_t i = 0; i < pre.size(); ++i) if (pre[i] == X) return ids[i];
        return -1;
    };
    for (size_t i = 0; i < pre.size(); ++i) {
        const int S = pre[i], id = ids[i], P = part[S], Q = S ^ P;
        const int a = code_of(P), c = code_of(Q);
        T.child[2 * id] = a;
        T.child[2 * id + 1] = c;
        T.parent[T.pidx(a)] = id;
        T.parent[T.pidx(c)] = id;
        T.cost[id] = opt[S];
        int cnt = 0;
        for (int j = 0; j < k; ++j) if (S >> j & 1) cnt += T.code_leaves(ent[j]);
        T.leaves[id] = cnt;
    }
    // boxes bottom-up over the rebuilt nodes (reverse preorder)
    for (size_t i = pre.size(); i-- > 0;) {
        const int id = ids[i];
        float* b = T.box(id);
        const float* b0 = T.box(T.child[2 * id]);
        const float* b1 = T.box(T.child[2 * id + 1]);
        for (int q = 0; q < 3; ++q) { b[q] = std::min(b0[q], b1[q]); b[3 + q] = std::max(b0[3 + q], b1[3 + q]); }
    }
}

static void treelet_rounds(int n, int* child, int* parent, float* aabb, int rounds) {
    if (n < 2) return;
    TreeRef T{n, child, parent, aabb, std::vector<float>(n - 1, 0.0f), std::vector<int>(n - 1, 0)};
    for (int rd = 0; rd < rounds; ++rd) {
        // post-order of the current tree
        std::vector<int> order, st{0};
        while (!st.empty()) {
            int i = st.back();
            st.pop_back();
            order.push_back(i);
            for (int c = 0; c < 2; ++c) if (!(child[2 * i + c] & TreeRef::LEAF)) st.push_back(child[2 * i + c]);
        }
        for (auto it = order.rbegin(); it != order.rend(); ++it) treelet_node(T, *it);
    }
}

} // namespace orc

// ==========================================================================
// C interface (ctypes)
// ==========================================================================
using namespace orc;

extern "C" {

void* or_scene_create(const float* V, int nv, const int* F, int nf, const float* mat, const float* lights,
                      int nl, const float* env, int he, int we, unsigned scene_id) {
    if (nl > MAXL) return nullptr;
    Scene* s = new Scene();
    s->nv = nv; s->nf = nf; s->nl = nl; s->id = scene_id;
    s->V.assign(V, V + 3 * (size_t)nv);
    s->F.assign(F, F + 3 * (size_t)nf);
    s->mat.assign(mat, mat + 7 * (size_t)nf);
    if (nl > 0) s->lights.assign(lights, lights + 6 * (size_t)nl);
    if (env && he > 0 && we > 0) { s->he = he; s->we = we; s->env.assign(env, env + 3 * (size_t)he * we); }
    build_edges(*s);
    build_edge_tree(*s);
    build_env(*s);
    build_bvh(*s);
    return s;
}

void or_scene_destroy(void* p) { delete (Scene*)p; }

// Switch the scene's materials to mesh colours of resolution r: texels holds
// nf (r+1)(r+2)/2 rows of 7 (r = 0: one row per face).  Returns the row count.
long long or_scene_set_texels(void* p, int r, const float* texels) {
    Scene* s = (Scene*)p;
    if (r < 0 || r > 64) return -1;
    s->tex_res = r;
    const size_t n = 7 * (size_t)s->nf * (size_t)((r + 1) * (r + 2) / 2);
    s->mat.assign(texels, texels + n);
    return (long long)(n / 7);
}

long long or_texel_index(int r, long long t, double alpha, double beta) { return texel_index(r, t, alpha, beta); }

// The secondary-edge importance tree: keys [n], child [n-1,2], parent [2n-1],
// box [2n-1,6], len [2n-1] (the layout of or_lbvh).
int or_edge_tree(void* p, unsigned long long* keys, int* child, int* parent, float* box, float* len, float* nbox) {
    const EdgeTree& T = ((Scene*)p)->etree;
    std::copy(T.keys.begin(), T.keys.end(), keys);
    std::copy(T.child.begin(), T.child.end(), child);
    std::copy(T.parent.begin(), T.parent.end(), parent);
    std::copy(T.box.begin(), T.box.end(), box);
    std::copy(T.len.begin(), T.len.end(), len);
    std::copy(T.nbox.begin(), T.nbox.end(), nbox);
    return T.n;
}

// One hierarchy draw from shading point x with normal n for the counters of
// sample i (vertex 1): the edge (or -1) and its probability.
int or_edge_tree_sample(void* p, const double* x, const double* n, long long i, unsigned seed, int sil, float* pe) {
    Scene* s = (Scene*)p;
    Ctr ctr{(uint32_t)i, 0u, 0u, 3u};
    return edge_tree_sample(*s, D3(x[0], x[1], x[2]), D3(n[0], n[1], n[2]), ctr, 1, Key{seed, s->id}, sil != 0, *pe);
}

// Specular lobe sampled from the visible normals (on) or from D cos(theta_h) (off, the default).
int or_scene_set_vndf(void* p, int on) {
    ((Scene*)p)->vndf = on != 0;
    return 0;
}

double or_erfinv(double y) { return erfinv_d(y); }

// Environment texels chosen through the alias table (on) or the CDFs (off, the default).
int or_scene_set_env_alias(void* p, int on) {
    Scene* s = (Scene*)p;
    if (!s->has_env) return -1;
    s->env_alias = on != 0;
    if (s->env_alias && s->aprob.empty()) build_alias(*s);
    return 0;
}

void or_env_alias_table(void* p, double* prob, int* alias) {
    Scene* s = (Scene*)p;
    if (s->aprob.empty()) build_alias(*s);
    for (size_t i = 0; i < s->aprob.size(); ++i) { prob[i] = s->aprob[i]; alias[i] = s->alias[i]; }
}

long long or_texel_of(void* p, int f, const double* x) { return texel_of(*(Scene*)p, f, D3(x[0], x[1], x[2])); }

int or_num_edges(void* p) { return (int)((Scene*)p)->edges.size(); }

void or_edges(void* p, int* out) {
    Scene* s = (Scene*)p;
    for (size_t e = 0; e < s->edges.size(); ++e) {
        out[4 * e] = s->edges[e].va; out[4 * e + 1] = s->edges[e].vb;
        out[4 * e + 2] = s->edges[e].f1; out[4 * e + 3] = s->edges[e].f2;
    }
}

double or_edge_total(void* p) { return ((Scene*)p)->elen_total; }

void or_philox(const unsigned* ctr, const unsigned* key, unsigned* out) {
    U4 r = philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

void or_brdf(const double* wi, const double* wo, const double* n, const double* m, double* out) {
    D3 r = brdf(D3(wi[0], wi[1], wi[2]), D3(wo[0], wo[1], wo[2]), D3(n[0], n[1], n[2]), m);
    out[0] = r.x; out[1] = r.y; out[2] = r.z;
}

double or_bsdf_pdf(const double* wi, const double* wo, const double* n, double alpha, int vndf) {
    return bsdf_pdf(D3(wi[0], wi[1], wi[2]), D3(wo[0], wo[1], wo[2]), D3(n[0], n[1], n[2]), alpha, vndf != 0);
}

int or_bsdf_sample(const double* u, const double* wo, const double* n, double alpha, int vndf, double* wi) {
    D3 w;
    int lobe = bsdf_sample(u, D3(wo[0], wo[1], wo[2]), D3(n[0], n[1], n[2]), alpha, vndf != 0, w);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
    return lobe;
}

double or_beckmann_D(double ch, double a) { return beckmann_D(ch, a); }
double or_smith_lambda(double c, double a) { return smith_lambda(c, a); }

int or_env_sample(void* p, const double* u, double* dir, double* pdf) {
    Scene* s = (Scene*)p;
    if (!s->has_env) return -1;
    D3 d;
    int t = env_sample(*s, u, d, *pdf);
    dir[0] = d.x; dir[1] = d.y; dir[2] = d.z;
    return t;
}

double or_env_pdf(void* p, const double* dir) {
    Scene* s = (Scene*)p;
    if (!s->has_env) return 0.0;
    return env_pdf_texel(*s, env_texel_of(*s, D3(dir[0], dir[1], dir[2])));
}

int or_env_texel(void* p, const double* dir) {
    Scene* s = (Scene*)p;
    return env_texel_of(*s, D3(dir[0], dir[1], dir[2]));
}

int or_closest(void* p, const double* o, const double* d, double tmin, int exclude, int brute, double* t) {
    return closest_hit(*(Scene*)p, D3(o[0], o[1], o[2]), D3(d[0], d[1], d[2]), tmin, exclude, *t, brute != 0);
}

int or_anyhit(void* p, const double* o, const double* d, double tmin, double tmax, int exclude, int brute) {
    return any_hit(*(Scene*)p, D3(o[0], o[1], o[2]), D3(d[0], d[1], d[2]), tmin, tmax, exclude, brute != 0) ? 1 : 0;
}

void or_camera_ray(const double* cam, int W, int H, double sx, double sy, double* o, double* d) {
    Cam c = make_cam(cam, W, H);
    D3 dd = cam_dir(c, sx, sy);
    o[0] = c.eye.x; o[1] = c.eye.y; o[2] = c.eye.z;
    d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
}

void or_project(const double* cam, int W, int H, const double* v, double* out) {
    Cam c = make_cam(cam, W, H);
    double sx, sy, z;
    project<double>(c, D3(v[0], v[1], v[2]), sx, sy, z);
    out[0] = sx; out[1] = sy; out[2] = z;
}

void or_lbvh(const float* V, int nv, const int* F, int nf, unsigned long long* keys, int* child, int* parent,
             float* aabb) {
    lbvh_reference(V, nv, F, nf, (uint64_t*)keys, child, parent, aabb);
}

// The Karras tree after `rounds` bottom-up treelet-restructuring passes.
void or_bvh_treelets(const float* V, int nv, const int* F, int nf, int rounds, unsigned long long* keys, int* child,
                     int* parent, float* aabb) {
    lbvh_reference(V, nv, F, nf, (uint64_t*)keys, child, parent, aabb);
    treelet_rounds(nf, child, parent, aabb, rounds);
}

// Forward render.  pix: npix pairs (view, y*W+x), or NULL for every pixel of
// every view in canonical order.  Writes per-sample radiance [npix, spp, 3] and
// the per-sample decision hash [npix, spp].
int or_render(void* p, const double* cams, const int* res, int ncam, int spp, int bounces, unsigned seed,
              const long long* pix, long long npix, double* out_rgb, unsigned* out_hash, int nthreads) {
    Scene* s = (Scene*)p;
    if (bounces < 1 || bounces > MAXV || spp < 1) return -1;
    Views vw = make_views(cams, res, ncam, spp, 0.0);
    if (!pix) npix = vw.pixoff[ncam];
    Key key{seed, s->id};
    parallel_for(npix * spp, nthreads, [&](int64_t idx, int) {
        int64_t q = idx / spp; int j = (int)(idx % spp);
        int view; int64_t local;
        if (pix) { view = (int)pix[2 * q]; local = pix[2 * q + 1]; }
        else {
            view = (int)(std::upper_bound(vw.pixoff.begin(), vw.pixoff.end(), q) - vw.pixoff.begin()) - 1;
            local = q - vw.pixoff[view];
        }
        const Cam& c = vw.cams[view];
        Hash h;
        D3 L = pixel_sample(*s, c, view, (int)(local % c.W), (int)(local / c.W), j, spp, bounces, key, h, nullptr,
                            nullptr);
        out_rgb[3 * idx] = L.x; out_rgb[3 * idx + 1] = L.y; out_rgb[3 * idx + 2] = L.z;
        if (out_hash) out_hash[idx] = h.h;
    });
    return 0;
}

// Backward.  flags: 1 interior, 2 primary edges, 4 secondary edges.
// d_image: float [sum W*H, 3], the loss gradient on the image (image = mean of
// the spp samples of each pixel).  Samples whose pixel has a zero d_image row
// contribute exactly zero and are skipped (their hash is left 0).  Masks (uint8,
// optional) switch off single path samples / primary edge samples.
int or_backward(void* p, const double* cams, const int* res, int ncam, int spp, int bounces, unsigned seed,
                unsigned flags, double ratio, const float* d_image, const unsigned char* path_mask,
                const unsigned char* edge_mask, double* dV, double* dmat, unsigned* path_hash,
                unsigned* edge_hash, int nthreads) {
    Scene* s = (Scene*)p;
    if (bounces < 1 || bounces > MAXV || spp < 1) return -1;
    Views vw = make_views(cams, res, ncam, spp, ratio);
    Key key{seed, s->id};
    int nt = std::max(1, nthreads);
    std::vector<Grad> G(nt);
    for (auto& g : G) { g.dV.assign(3 * (size_t)s->nv, 0.0); g.dM.assign(s->mat.size(), 0.0); }
    const bool interior = flags & 1, primary = flags & 2, secondary = flags & 4, shadow = flags & 8;
    const int64_t npath = vw.pixoff[ncam] * spp;
    if (path_hash) std::memset(path_hash, 0, sizeof(unsigned) * npath);
    if (interior || secondary) {
        parallel_for(npath, nt, [&](int64_t idx, int tid) {
            if (path_mask && !path_mask[idx]) return;
            int64_t q = idx / spp; int j = (int)(idx % spp);
            int view = (int)(std::upper_bound(vw.pixoff.begin(), vw.pixoff.end(), q) - vw.pixoff.begin()) - 1;
            int64_t local = q - vw.pixoff[view];
            const float* di = d_image + 3 * q;
            if (di[0] == 0.0f && di[1] == 0.0f && di[2] == 0.0f) return;
            const Cam& c = vw.cams[view];
            double w[3] = {di[0] / (double)spp, di[1] / (double)spp, di[2] / (double)spp};
            Hash h;
            PRec rec;
            SecCtx sc{{w[0], w[1], w[2]}, &G[tid], (flags & 64) != 0, (flags & 256) != 0};
            pixel_sample(*s, c, view, (int)(local % c.W), (int)(local / c.W), j, spp, bounces, key, h, &rec,
                         secondary ? &sc : nullptr);
            path_gradient(*s, rec, w, interior, secondary, bounces, G[tid]);
            if (path_hash) path_hash[idx] = h.h;
        });
    }
    const int64_t n_edge_all = vw.eoff[ncam] * (1 + ((flags & 8) ? (int64_t)s->nl : 0));
    if (edge_hash) std::memset(edge_hash, 0, sizeof(unsigned) * n_edge_all);
    if (primary) {
        for (int v = 0; v < ncam; ++v) {
            const Cam& c = vw.cams[v];
            EdgeView ev = primary_cdf(*s, c);
            const float* dv = d_image + 3 * vw.pixoff[v];
            parallel_for(vw.ne[v], nt, [&](int64_t si, int tid) {
                int64_t gi = vw.eoff[v] + si;
                if (edge_mask && !edge_mask[gi]) return;
                Hash h;
                bool comp;
                primary_edge_sample(*s, c, ev, v, si, vw.ne[v], spp, bounces, key, dv, h, G[tid], comp);
                if (edge_hash && comp) edge_hash[gi] = h.h;
            });
        }
    }
    if (shadow && s->nl > 0) {
        // point-light shadow boundaries: samples of (view v, light l) follow the
        // primary edge samples, at nl eoff[v] + l N_e(v) + i
        const int64_t ep = vw.eoff[ncam];
        for (int l = 0; l < s->nl; ++l) {
            LightEdges le = light_cdf(*s, l);
            for (int v = 0; v < ncam; ++v) {
                const Cam& c = vw.cams[v];
                const float* dv = d_image + 3 * vw.pixoff[v];
                const int64_t base = ep + (int64_t)s->nl * vw.eoff[v] + (int64_t)l * vw.ne[v];
                parallel_for(vw.ne[v], nt, [&](int64_t si, int tid) {
                    const int64_t gi = base + si;
                    if (edge_mask && !edge_mask[gi]) return;
                    Hash h;
                    shadow_edge_sample(*s, c, le, v, l, si, vw.ne[v], key, dv, h, G[tid]);
                    if (edge_hash) edge_hash[gi] = h.h;
                });
            }
        }
    }
    for (size_t i = 0; i < 3 * (size_t)s->nv; ++i) { double a = 0; for (auto& g : G) a += g.dV[i]; dV[i] = a; }
    for (size_t i = 0; i < s->mat.size(); ++i) { double a = 0; for (auto& g : G) a += g.dM[i]; dmat[i] = a; }
    return 0;
}

// One path sample's loss value L = sum_c w_c L_c (+ secondary pseudo term) under
// a single parameter perturbation, with every decision, sampled direction, pdf
// and MIS weight frozen at the unperturbed path (the finite-difference check of
// the dual-number derivative).  kind 0: dV index, 1: dmat index, -1: none.
double or_sample_frozen(void* p, const double* cams, const int* res, int ncam, int spp, int bounces,
                        unsigned seed, unsigned flags, int view, int px, int py, int j, const double* w,
                        int kind, int index, double delta) {
    Scene* s = (Scene*)p;
    Views vw = make_views(cams, res, ncam, spp, 0.0);
    Key key{seed, s->id};
    Hash h;
    PRec rec;
    Grad dummy; dummy.dV.assign(3 * (size_t)s->nv, 0.0); dummy.dM.assign(s->mat.size(), 0.0);
    SecCtx sc{{w[0], w[1], w[2]}, &dummy, (flags & 64) != 0, (flags & 256) != 0};
    pixel_sample(*s, vw.cams[view], view, px, py, j, spp, bounces, key, h, &rec, (flags & 4) ? &sc : nullptr);
    PView P; P.s = s;
    for (int k = 0; k < rec.nv; ++k) P.add_vertex(rec.v[k].face, rec.v[k].tex);
    Perturb pt; pt.kind = kind; pt.index = index; pt.delta = delta;
    return replay<double>(*s, rec, w, (flags & 1) != 0, (flags & 4) != 0, P, pt);
}

// The same sample's radiance from the recording pass (for the replay-equals-
// record check) and its dual-number gradient (dense dV, dmat).
double or_sample_grad(void* p, const double* cams, const int* res, int ncam, int spp, int bounces,
                      unsigned seed, unsigned flags, int view, int px, int py, int j, const double* w,
                      double* rgb, double* dV, double* dmat) {
    Scene* s = (Scene*)p;
    Views vw = make_views(cams, res, ncam, spp, 0.0);
    Key key{seed, s->id};
    Hash h;
    PRec rec;
    Grad g; g.dV.assign(3 * (size_t)s->nv, 0.0); g.dM.assign(s->mat.size(), 0.0);
    // flag 8: leave out the direct edge-endpoint terms (only the replay derivative)
    SecCtx sc{{w[0], w[1], w[2]}, (flags & 8) ? nullptr : &g, (flags & 64) != 0, (flags & 256) != 0};
    D3 L = pixel_sample(*s, vw.cams[view], view, px, py, j, spp, bounces, key, h, &rec,
                        (flags & 4) ? &sc : nullptr);
    rgb[0] = L.x; rgb[1] = L.y; rgb[2] = L.z;
    path_gradient(*s, rec, w, (flags & 1) != 0, (flags & 4) != 0, bounces, g);
    for (size_t i = 0; i < 3 * (size_t)s->nv; ++i) dV[i] = g.dV[i];
    for (size_t i = 0; i < s->mat.size(); ++i) dmat[i] = g.dM[i];
    PView P; P.s = s;
    for (int k = 0; k < rec.nv; ++k) P.add_vertex(rec.v[k].face, rec.v[k].tex);
    Perturb none;
    return replay<double>(*s, rec, w, true, false, P, none);
}

// Secondary edge term alone at a fixed shading point p (normal n, outgoing wo,
// material of face `face`, throughput 1, loss weight 1/3 per channel), averaged
// over nsamples edge samples drawn exactly as at the first vertex of a path
// (the function the backward calls); the shading point itself is held fixed,
// so only the edge endpoints receive gradient.  interior: also creases and
// material boundaries.  Used to pin the estimator against the closed-form
// projected solid angle of polygons.
void or_secondary_term(void* p, const double* pp, const double* nn, const double* wo, int face, int budget,
                       long long nsamples, unsigned seed, int hier, int interior, double* dV) {
    Scene* s = (Scene*)p;
    Grad g; g.dV.assign(3 * (size_t)s->nv, 0.0); g.dM.assign(s->mat.size(), 0.0);
    Key key{seed, s->id};
    D3 x(pp[0], pp[1], pp[2]), n(nn[0], nn[1], nn[2]), o(wo[0], wo[1], wo[2]);
    const double* m = &s->mat[7 * texel_of(*s, face, x)];
    SecCtx sc;
    for (int ch = 0; ch < 3; ++ch) sc.w[ch] = 1.0 / (3.0 * (double)nsamples);
    sc.g = &g;
    sc.interior = interior != 0;
    sc.hier = hier != 0;
    Hash h; h.on = false;
    if (!s->edges.empty() && s->elen_total > 0.0)
        for (long long i = 0; i < nsamples; ++i) {
            Ctr ctr{(uint32_t)i, 0u, 0u, 3u};
            secondary_edge_sample(*s, x, n, o, face, m, D3(1, 1, 1), 1, budget, ctr, key, sc, h, nullptr);
        }
    for (size_t i = 0; i < 3 * (size_t)s->nv; ++i) dV[i] = g.dV[i];
}

} // extern "C"

"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
numpy's Philox, quadrature identities of the microfacet model, the closed-form
radiance of a Lambertian plane under a point light, the white furnace, the
hemisphere integral of a plane under a non-constant environment, brute
force intersection, central finite differences, and closed-form edge
derivatives (projected triangle area, projected solid angle of a polygon).
CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2012_03939_amd import scenes as S
from philox_ref import philox, draw4, uniform24


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------

@pytest.mark.parametrize("key", [(0, 0), (5, 7), (0xFFFFFFFFFFFF, 123456789)])
def test_philox_generic_matches_numpy_4x64(key):
    bg = np.random.Philox(counter=0, key=list(key))
    raw = [int(x) for x in bg.random_raw(8)]
    # numpy advances the counter before producing a block
    assert raw[:4] == philox((1, 0, 0, 0), key, width=64)
    assert raw[4:] == philox((2, 0, 0, 0), key, width=64)


def test_philox_oracle_matches_reference_4x32():
    rng = np.random.default_rng(3)
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        assert list(O.philox4x32(c, k)) == philox(c, k, width=32)


def test_uniform24_chi2():
    from scipy import stats
    u = np.array([uniform24(r) for i in range(4000) for r in philox((i, 7, 2, 0), (11, 3))])
    assert u.min() >= 0.0 and u.max() <= 1.0 - 2 ** -24
    h, _ = np.histogram(u, bins=32, range=(0, 1))
    assert stats.chisquare(h).pvalue > 1e-3


# --------------------------------------------------------------------------
# Torrance-Sparrow BRDF (Beckmann D, Smith Lambda, specular colour)
# --------------------------------------------------------------------------

def _hemi_quad(n_t=400, n_p=64):
    th = (np.arange(n_t) + 0.5) * (0.5 * np.pi / n_t)
    ph = (np.arange(n_p) + 0.5) * (2 * np.pi / n_p)
    w = np.sin(th) * (0.5 * np.pi / n_t) * (2 * np.pi / n_p)
    return th, ph, w


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.5, 1.0])
def test_beckmann_D_normalised(alpha):
    # integral over the hemisphere of D(h) cos(theta_h) = 1 (phi-independent)
    n_t = 20000
    th = (np.arange(n_t) + 0.5) * (0.5 * np.pi / n_t)
    val = sum(O.beckmann_D(math.cos(t), alpha) * math.cos(t) * math.sin(t) for t in th)
    val *= (0.5 * np.pi / n_t) * 2 * np.pi
    assert abs(val - 1.0) < 2e-4
    assert abs(O.beckmann_D(1.0, alpha) - 1.0 / (np.pi * alpha * alpha)) < 1e-12 / alpha ** 2


@pytest.mark.parametrize("alpha,theta_o", [(0.1, 0.3), (0.3, 0.9), (0.5, 1.3), (0.8, 0.6)])
def test_smith_weak_white_furnace(alpha, theta_o):
    # Heitz 2014: integral of G1(wo) D(h) max(0, wo.h) / cos(theta_o) dh = 1
    wo = np.array([math.sin(theta_o), 0.0, math.cos(theta_o)])
    g1 = 1.0 / (1.0 + O.smith_lambda(math.cos(theta_o), alpha))
    n_t, n_p = 3000, 256
    th = (np.arange(n_t) + 0.5) * (0.5 * np.pi / n_t)
    ph = (np.arange(n_p) + 0.5) * (2 * np.pi / n_p)
    T, P = np.meshgrid(th, ph, indexing="ij")
    h = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    D = np.vectorize(lambda c: O.beckmann_D(c, alpha))(np.cos(th))[:, None]
    integrand = D * np.maximum(0.0, h @ wo) * np.sin(T)
    val = integrand.sum() * (0.5 * np.pi / n_t) * (2 * np.pi / n_p) * g1 / wo[2]
    assert abs(val - 1.0) < 2e-3


def test_lambda_limits():
    assert O.smith_lambda(1.0, 0.3) == 0.0
    # Lambda grows without bound toward grazing and vanishes toward normal incidence
    assert O.smith_lambda(0.01, 0.5) > 10.0
    assert O.smith_lambda(0.99, 0.05) < 1e-12


def _rand_dir_upper(rng):
    while True:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if d[2] > 0.05:
            return d


def test_brdf_reciprocity_and_lambert():
    rng = np.random.default_rng(5)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(50):
        wi, wo = _rand_dir_upper(rng), _rand_dir_upper(rng)
        m = np.concatenate([rng.uniform(0, 1, 3), rng.uniform(0, 1, 3), [rng.uniform(0.05, 0.8)]])
        assert np.allclose(O.brdf(wi, wo, n, m), O.brdf(wo, wi, n, m), rtol=1e-12, atol=0)
        mz = m.copy()
        mz[3:6] = 0
        assert np.allclose(O.brdf(wi, wo, n, mz), mz[:3] / np.pi, rtol=1e-15, atol=0)
        assert np.array_equal(O.brdf(-wi, wo, n, m), np.zeros(3))


@pytest.mark.parametrize("alpha", [0.1, 0.4])
def test_specular_energy_bounded(alpha):
    # single-scattering microfacet lobe with ks = 1 reflects at most all energy
    n = np.array([0.0, 0.0, 1.0])
    th, ph, w = _hemi_quad(300, 96)
    m = np.array([0, 0, 0, 1, 1, 1, alpha], float)
    for to in (0.2, 1.0):
        wo = np.array([math.sin(to), 0, math.cos(to)])
        tot = 0.0
        for t, wt in zip(th, w):
            for p in ph:
                wi = np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])
                tot += O.brdf(wi, wo, n, m)[0] * wi[2] * wt
        assert 0.5 < tot <= 1.0 + 1e-3


@pytest.mark.parametrize("vndf", [False, True])
@pytest.mark.parametrize("alpha,to", [(0.08, 0.4), (0.3, 1.0), (0.6, 0.2), (0.5, 1.45)])
def test_bsdf_sampling_matches_pdf(alpha, to, vndf):
    """Sampled directions against the mixture pdf (chi^2 over cos(theta) x phi bins,
    the mass below the surface as one more bin), classical and visible-normal."""
    from scipy import stats
    rng = np.random.default_rng(9)
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([math.sin(to), 0, math.cos(to)])
    N = 60000
    nb_c, nb_p = 8, 8
    counts = np.zeros((nb_c, nb_p))
    below = 0
    us = rng.random((N, 4))
    for u in us:
        _, wi = O.bsdf_sample(u, wo, n, alpha, vndf)
        if wi[2] <= 0:
            below += 1
            continue
        ic = min(int(wi[2] * nb_c), nb_c - 1)
        ip = min(int((math.atan2(wi[1], wi[0]) % (2 * np.pi)) / (2 * np.pi) * nb_p), nb_p - 1)
        counts[ic, ip] += 1
    # expected mass per (cos theta, phi) bin from the pdf by quadrature
    exp_mass = np.zeros((nb_c, nb_p))
    sub = 12
    for ic in range(nb_c):
        for ip in range(nb_p):
            acc = 0.0
            for a in range(sub):
                c = (ic + (a + 0.5) / sub) / nb_c
                s = math.sqrt(1 - c * c)
                for b in range(sub):
                    p = (ip + (b + 0.5) / sub) / nb_p * 2 * np.pi
                    wi = np.array([s * math.cos(p), s * math.sin(p), c])
                    acc += O.bsdf_pdf(wi, wo, n, alpha, vndf)
            exp_mass[ic, ip] = acc / sub ** 2 * (1.0 / nb_c) * (2 * np.pi / nb_p)
    upper = exp_mass.sum()
    assert upper <= 1.0 + 1e-3
    obs = np.append(counts.ravel(), below)
    exp = np.append(exp_mass.ravel(), max(1.0 - upper, 0.0)) * N
    keep = exp > 20
    obs_k, exp_k = obs[keep], exp[keep]
    exp_k = exp_k * obs_k.sum() / exp_k.sum()
    assert stats.chisquare(obs_k, exp_k).pvalue > 1e-4


# --------------------------------------------------------------------------
# environment map distribution
# --------------------------------------------------------------------------

def _tiny_scene(env=None):
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    return O.OracleScene(V, F, S.uniform_materials(1), None, env)


def test_env_pdf_normalised_and_constant_map_uniform():
    rng = np.random.default_rng(2)
    env = S.gaussian_lobe_envmap(rng, 64, 32)
    sc = _tiny_scene(env)
    he, we = env.shape[:2]
    tot = 0.0
    for r in range(he):
        dom = (2 * np.pi / we) * (math.cos(np.pi * r / he) - math.cos(np.pi * (r + 1) / he))
        th = np.pi * (r + 0.5) / he
        for c in range(we):
            ph = 2 * np.pi * (c + 0.5) / we
            d = [math.sin(th) * math.sin(ph), math.cos(th), math.sin(th) * math.cos(ph)]
            assert sc.env_texel(d) == r * we + c
            tot += sc.env_pdf(d) * dom
    assert abs(tot - 1.0) < 1e-12
    const = _tiny_scene(np.ones((16, 32, 3), np.float32))
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        assert abs(const.env_pdf(d) - 1.0 / (4 * np.pi)) < 1e-12


def test_env_sampling_histogram():
    from scipy import stats
    rng = np.random.default_rng(4)
    env = S.gaussian_lobe_envmap(rng, 32, 16)
    sc = _tiny_scene(env)
    he, we = env.shape[:2]
    w = env.astype(np.float64).mean(axis=2)
    dom = np.array([(2 * np.pi / we) * (math.cos(np.pi * r / he) - math.cos(np.pi * (r + 1) / he)) for r in range(he)])
    P = (w * dom[:, None]).ravel()
    P /= P.sum()
    N = 50000
    counts = np.zeros(he * we)
    for u in rng.random((N, 4)):
        t, d, pdf = sc.env_sample(u)
        counts[t] += 1
        r = t // we
        assert abs(pdf - P[t] / dom[r]) <= 1e-9 * pdf
    keep = P * N > 20
    exp = P[keep] * N
    obs = counts[keep]
    exp *= obs.sum() / exp.sum()
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_env_sample_direction_inside_texel():
    rng = np.random.default_rng(6)
    env = S.gaussian_lobe_envmap(rng, 64, 32)
    sc = _tiny_scene(env)
    misses = 0
    for u in rng.random((3000, 4)):
        t, d, _ = sc.env_sample(u)
        assert abs(np.linalg.norm(d) - 1.0) < 1e-12
        misses += sc.env_texel(d) != t
    assert misses <= 3    # only exact texel borders may round across


def _texel_probs(env):
    """Texel probabilities written out from their definition (power x solid angle)."""
    he, we = env.shape[:2]
    w = env.astype(np.float64).mean(axis=2)
    dom = np.array([(2 * np.pi / we) * (math.cos(np.pi * r / he) - math.cos(np.pi * (r + 1) / he)) for r in range(he)])
    P = (w * dom[:, None]).ravel()
    return P / P.sum(), dom


def test_env_alias_table_reproduces_texel_probabilities():
    """Walker's alias table: bin k keeps prob_k of its 1/n for texel k and hands
    1 - prob_k to alias_k, so summing the pieces over all bins must give back
    every texel's probability; a dropped leftover or a wrong stack update fails."""
    rng = np.random.default_rng(11)
    for he, we in [(16, 32), (7, 5), (1, 1), (64, 128)]:
        env = S.gaussian_lobe_envmap(rng, we, he) if he > 1 else np.full((1, 1, 3), 2.0, np.float32)
        sc = _tiny_scene(env)
        prob, alias = sc.env_alias_table()
        n = he * we
        P, _ = _texel_probs(env)
        assert ((prob >= 0) & (prob <= 1)).all() and ((alias >= 0) & (alias < n)).all()
        back = prob.copy()
        np.add.at(back, alias, 1.0 - prob)
        back -= np.where(alias == np.arange(n), 1.0 - prob, 0.0)    # a bin aliased to itself gives nothing away
        assert np.abs(back / n - P).max() < 1e-12 * max(P.max(), 1.0 / n)
        # a bin below its share is never the alias of another bin unless it was topped up first
        assert (prob[alias == np.arange(n)] == 1.0).all()


def test_env_alias_sampling_histogram_and_pdf():
    """With the alias table on, the texel histogram matches the texel
    probabilities, the pdf is the same, and directions stay inside their texel."""
    from scipy import stats
    rng = np.random.default_rng(4)
    env = S.gaussian_lobe_envmap(rng, 32, 16)
    sc = _tiny_scene(env)
    sc.set_env_alias(True)
    he, we = env.shape[:2]
    P, dom = _texel_probs(env)
    N = 50000
    counts = np.zeros(he * we)
    misses = 0
    for u in rng.random((N, 4)):
        t, d, pdf = sc.env_sample(u)
        counts[t] += 1
        assert abs(pdf - P[t] / dom[t // we]) <= 1e-9 * pdf
        misses += sc.env_texel(d) != t
    assert misses <= 20
    keep = P * N > 20
    exp = P[keep] * N
    obs = counts[keep]
    exp *= obs.sum() / exp.sum()
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_env_alias_exhaustive_two_by_two():
    """2 x 2 map: the probability of each texel over an exact grid of (u0, u1)
    equals its texel probability up to the grid step."""
    env = np.array([[[1, 1, 1], [3, 3, 3]], [[0.5, 0.5, 0.5], [6, 6, 6]]], np.float32)
    sc = _tiny_scene(env)
    sc.set_env_alias(True)
    P, _ = _texel_probs(env)
    G = 400
    hits = np.zeros(4)
    for i in range(G):
        for j in range(G):
            t, _, _ = sc.env_sample([(i + 0.5) / G, (j + 0.5) / G, 0.5, 0.5])
            hits[t] += 1
    assert np.abs(hits / G ** 2 - P).max() <= 2.0 / G


# --------------------------------------------------------------------------
# intersection and acceleration structure
# --------------------------------------------------------------------------

def test_bvh_equals_brute_force():
    rng = np.random.default_rng(8)
    V, F = S.noise_sphere(6, 0.15, noise_seed=3)
    # plus a soup of random triangles inside
    soup = rng.uniform(-0.8, 0.8, (60, 3, 3))
    V2 = np.concatenate([V, soup.reshape(-1, 3)])
    F2 = np.concatenate([F, V.shape[0] + np.arange(180).reshape(60, 3)]).astype(np.int32)
    sc = O.OracleScene(V2.astype(np.float32), F2, S.uniform_materials(F2.shape[0]))
    for _ in range(1500):
        o = rng.uniform(-2.5, 2.5, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ex = int(rng.integers(-1, F2.shape[0]))
        f1, t1 = sc.closest(o, d, 1e-4, ex, brute=False)
        f2, t2 = sc.closest(o, d, 1e-4, ex, brute=True)
        assert f1 == f2 and (f1 < 0 or t1 == t2)
        tmax = float(rng.uniform(0.1, 5))
        assert sc.anyhit(o, d, 1e-4, tmax, ex, False) == sc.anyhit(o, d, 1e-4, tmax, ex, True)


def test_triangle_hit_known_answer():
    V = np.array([[-1, -1, 2], [1, -1, 2], [0, 1, 2]], np.float32)
    sc = O.OracleScene(V, np.array([[0, 1, 2]], np.int32), S.uniform_materials(1))
    f, t = sc.closest([0.1, 0.2, -1.0], [0, 0, 1])
    assert f == 0 and t == 3.0
    f, t = sc.closest([0.1, 0.2, -1.0], [0, 0, -1])
    assert f == -1
    f, t = sc.closest([0.1, 0.2, -1.0], [0, 0, 1], exclude=0)
    assert f == -1
    assert not sc.anyhit([0.1, 0.2, -1.0], [0, 0, 1], 1e-4, 2.999)
    assert sc.anyhit([0.1, 0.2, -1.0], [0, 0, 1], 1e-4, 3.001)


# --------------------------------------------------------------------------
# camera model
# --------------------------------------------------------------------------

def _pinhole(cam, sx, sy):
    """The pinhole definition written out directly (vertical fov, row 0 at top)."""
    e = np.array(cam.eye, np.float32).astype(float)
    tg = np.array(cam.target, np.float32).astype(float)
    up = np.array(cam.up, np.float32).astype(float)
    f = (tg - e) / np.linalg.norm(tg - e)
    r = np.cross(f, up / np.linalg.norm(up))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(float(np.float32(cam.fov_y_deg)) * math.pi / 360)
    ndx = 2 * sx / cam.width - 1
    ndy = 1 - 2 * sy / cam.height
    d = f + ndx * th * cam.width / cam.height * r + ndy * th * u
    return e, d / np.linalg.norm(d)


def test_camera_rays_and_projection_agree():
    rng = np.random.default_rng(1)
    cam = S.Camera((0.3, 0.7, 2.9), (0.1, -0.2, 0.0), (0, 1, 0), 45.0, 96, 64)
    for _ in range(100):
        sx, sy = rng.uniform(0, 96), rng.uniform(0, 64)
        o, d = O.camera_ray(cam, sx, sy)
        e, dd = _pinhole(cam, sx, sy)
        assert np.allclose(o, e, atol=0) and np.allclose(d, dd, rtol=0, atol=1e-14)
        p = O.project(cam, o + 2.5 * d)
        assert abs(p[0] - sx) < 1e-9 and abs(p[1] - sy) < 1e-9 and p[2] > 0


# --------------------------------------------------------------------------
# closed-form radiance: Lambertian plane under a point light
# --------------------------------------------------------------------------

def test_lambertian_plane_point_light_closed_form():
    V = np.array([[-5, -5, 0], [5, -5, 0], [5, 5, 0], [-5, 5, 0]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    kd = np.array([0.3, 0.5, 0.7], np.float32)
    mat = np.zeros((2, 7), np.float32)
    mat[:, :3] = kd
    mat[:, 6] = 0.3
    light = np.array([[0.5, 0.3, 2.0, 10.0, 8.0, 6.0]], np.float32)
    sc = O.OracleScene(V, F, mat, light, None, scene_id=3)
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 16, 12)
    seed, spp = 9, 2
    rgb, _ = sc.render_samples([cam], spp, 1, seed)
    pl = light[0, :3].astype(float)
    I = light[0, 3:].astype(float)
    worst = 0.0
    for y in range(12):
        for x in range(16):
            for j in range(spp):
                u = draw4(y * 16 + x, j, 0, 0, seed, 3)
                o, d = _pinhole(cam, x + u[0], y + u[1])
                t = -o[2] / d[2]
                p = o + t * d
                wl = pl - p
                r2 = wl @ wl
                cos = wl[2] / math.sqrt(r2)
                expect = kd.astype(float) / np.pi * I * cos / r2
                got = rgb[y * 16 + x, j]
                worst = max(worst, np.abs(got - expect).max() / expect.max())
    assert worst < 1e-12


# --------------------------------------------------------------------------
# white furnace: convex Lambertian object under a constant environment
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bounces,kd", [(1, 1.0), (2, 1.0), (3, 0.5)])
def test_white_furnace(bounces, kd):
    V, F = S.geodesic_sphere(3)
    mat = S.uniform_materials(F.shape[0], kd=kd, ks=0.0, rough=0.3)
    sc = O.OracleScene(V.astype(np.float32), F, mat, None, np.full((16, 32, 3), 1.0, np.float32))
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 30.0, 24, 24)
    rgb, hsh = sc.render_samples([cam], 16, bounces, seed=1)
    hit = rgb.reshape(-1, 3)[:, 0] > 0
    vals = rgb.reshape(-1, 3)[hit]
    assert hit.sum() > 2000
    m = vals.mean(axis=0)
    se = vals.std(axis=0) / math.sqrt(vals.shape[0])
    assert np.all(np.abs(m - kd) < 4 * se + 1e-9), (m, se)


# --------------------------------------------------------------------------
# environment sample and BRDF sample combined (balance heuristic) under a
# non-constant map: one bounce off a plane that sees only the upper hemisphere.
# The expectation is the hemisphere integral of BRDF x map x cosine, so any
# weight or pdf that is off for some directions (a wrong texel, a missing
# Jacobian, weights not summing to one) biases the mean; the constant map of
# the furnace test cannot show that.
# --------------------------------------------------------------------------

def _sky_integral(env, wo, m, sub):
    """sum over the texels above the horizon of L * int f(wi, wo) cos dwi,
    midpoint rule on sub x sub cells of exact solid angle (rows at
    theta = pi r / he, columns at phi = 2 pi c / we, y up)."""
    he, we = env.shape[:2]
    n = np.array([0.0, 1.0, 0.0])
    dph = 2 * np.pi / we / sub
    tot = np.zeros(3)
    for r in range(he // 2):
        for i in range(sub):
            ta = np.pi * (r + i / sub) / he
            tb = np.pi * (r + (i + 1) / sub) / he
            th = 0.5 * (ta + tb)
            dom = dph * (math.cos(ta) - math.cos(tb))
            for c in range(we):
                for j in range(sub):
                    ph = 2 * np.pi * (c + (j + 0.5) / sub) / we
                    wi = np.array([math.sin(th) * math.sin(ph), math.cos(th), math.sin(th) * math.cos(ph)])
                    tot += env[r, c].astype(np.float64) * O.brdf(wi, wo, n, m) * wi[1] * dom
    return tot


@pytest.mark.parametrize("kind,sampler", [("lambert", ""), ("glossy", ""), ("glossy", "vndf"), ("lambert", "alias")])
def test_environment_estimator_matches_hemisphere_integral(kind, sampler):
    rng = np.random.default_rng(21)
    env = S.gaussian_lobe_envmap(rng, 16, 8, nlobes=8, base=0.1)
    he, we = env.shape[:2]
    sky = env[: he // 2].astype(np.float64).mean(axis=2)
    assert sky.max() > 5 * sky.min()     # the map varies where the plane looks
    if kind == "lambert":
        m = np.array([0.8, 0.6, 0.4, 0.0, 0.0, 0.0, 0.3])
        to = math.radians(20.0)
    else:
        m = np.array([0.05, 0.05, 0.05, 0.8, 0.6, 0.4, 0.25])
        to = math.radians(50.0)
    V = np.array([[-5, 0, -5], [5, 0, -5], [5, 0, 5], [-5, 0, 5]], np.float32)
    F = np.array([[0, 2, 1], [0, 3, 2]], np.int32)          # normal +y
    sc = O.OracleScene(V, F, np.tile(m.astype(np.float32), (2, 1)), None, env)
    sc.set_vndf(sampler == "vndf")
    sc.set_env_alias(sampler == "alias")
    # a narrow camera: every sample leaves the plane towards the same wo
    wo = np.array([0.0, math.cos(to), math.sin(to)])
    cam = S.Camera(tuple(3.0 * wo), (0, 0, 0), (0, 1, 0), 0.2, 4, 4)
    rgb, _ = sc.render_samples([cam], 65536, 1, seed=5)
    vals = rgb.reshape(-1, 3)
    mean = vals.mean(axis=0)
    se = vals.std(axis=0) / math.sqrt(vals.shape[0])
    if kind == "lambert":
        # closed form: kd / pi * sum L_t * int_texel cos = dphi (sin^2 tb - sin^2 ta) / 2
        thr = np.pi * np.arange(he // 2 + 1) / he
        w_row = (2 * np.pi / we) * 0.5 * (np.sin(thr[1:]) ** 2 - np.sin(thr[:-1]) ** 2)
        expect = m[:3] / np.pi * (env[: he // 2].astype(np.float64) * w_row[:, None, None]).sum(axis=(0, 1))
        assert np.allclose(_sky_integral(env, wo, m, 8), expect, rtol=1e-3, atol=0)
    else:
        expect = _sky_integral(env, wo, m, 12)
    assert np.all(se < 0.01 * expect), (se, expect)
    assert np.all(np.abs(mean - expect) < 4 * se), (mean, expect, se)


# --------------------------------------------------------------------------
# interior derivative: dual numbers vs central differences on the frozen path
# --------------------------------------------------------------------------

def _fd_check(sc, cams, spp, B, samples, flags, seed=0):
    rng = np.random.default_rng(12)
    checked = 0
    for (view, px, py, j) in samples:
        w = rng.uniform(0.2, 1.0, 3)
        loss, rgb, dV, dM = sc.sample_grad(cams, spp, B, view, px, py, j, w, seed, flags | 8)
        if flags & 1:
            assert abs(loss - (rgb @ w)) <= 1e-12 * max(1.0, abs(loss))   # replay == record
        base = sc.sample_frozen(cams, spp, B, view, px, py, j, w, -1, -1, 0.0, seed, flags)
        if flags == 1:
            assert abs(base - loss) <= 1e-12 * max(1.0, abs(loss))
        nz_v = np.argwhere(np.abs(dV.ravel()) > 0).ravel()
        nz_m = np.argwhere(np.abs(dM.ravel()) > 0).ravel()
        scale = max(np.abs(dV).max(initial=0), np.abs(dM).max(initial=0), 1e-12)
        h = 1e-6
        for kind, idxs, g in ((0, nz_v, dV.ravel()), (1, nz_m, dM.ravel())):
            for i in idxs:
                fp = sc.sample_frozen(cams, spp, B, view, px, py, j, w, kind, int(i), h, seed, flags)
                fm = sc.sample_frozen(cams, spp, B, view, px, py, j, w, kind, int(i), -h, seed, flags)
                fd = (fp - fm) / (2 * h)
                assert abs(fd - g[i]) <= 2e-6 * scale + 1e-6 * abs(g[i]), (kind, i, fd, g[i])
                checked += 1
    return checked


def test_fd_frozen_point_light_direct():
    wl = S.small_sphere(res=16, spp=2)
    sc = O.OracleScene.from_scene(wl.scenes[0])
    samples = [(0, x, y, j) for (x, y) in [(8, 8), (5, 9), (10, 4), (7, 12)] for j in range(2)]
    assert _fd_check(sc, wl.cams, 2, 1, samples, flags=1) > 50


def test_fd_frozen_envmap_multibounce():
    rng = np.random.default_rng(21)
    V, F = S.noise_sphere(4, 0.2, noise_seed=5)
    # a floor plane under the object so that continuation rays hit surfaces
    floor = np.array([[-3, -1.2, -3], [3, -1.2, -3], [3, -1.2, 3], [-3, -1.2, 3]], np.float32)
    Vf = np.concatenate([V, floor]).astype(np.float32)
    nv = V.shape[0]
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    mat = S.random_materials(Ff.shape[0], rng)
    env = S.gaussian_lobe_envmap(rng, 32, 16)
    lights = np.array([[1.0, 2.0, 1.5, 6, 6, 6]], np.float32)
    sc = O.OracleScene(Vf, Ff, mat, lights, env)
    cams = [S.Camera((0.0, 0.4, 3.2), (0, -0.2, 0), (0, 1, 0), 40.0, 20, 20)]
    samples = [(0, x, y, j) for (x, y) in [(10, 10), (6, 14), (13, 8), (9, 17), (4, 10)] for j in range(3)]
    assert _fd_check(sc, cams, 3, 3, samples, flags=1) > 100


def test_fd_frozen_secondary_pseudo_term():
    # the secondary edge pseudo term carries the shading-point motion; its
    # dual derivative must match finite differences of the frozen replay too
    rng = np.random.default_rng(22)
    V, F = S.noise_sphere(3, 0.3, noise_seed=9)
    floor = np.array([[-3, -1.3, -3], [3, -1.3, -3], [3, -1.3, 3], [-3, -1.3, 3]], np.float32)
    Vf = np.concatenate([V, floor]).astype(np.float32)
    nv = V.shape[0]
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    sc = O.OracleScene(Vf, Ff, S.random_materials(Ff.shape[0], rng), None, S.gaussian_lobe_envmap(rng, 32, 16))
    cams = [S.Camera((0.0, 0.5, 3.0), (0, -0.3, 0), (0, 1, 0), 45.0, 16, 16)]
    samples = [(0, x, y, j) for x in range(2, 14, 3) for y in range(2, 14, 3) for j in range(2)]
    assert _fd_check(sc, cams, 2, 2, samples, flags=5) > 50


# --------------------------------------------------------------------------
# primary edge term: closed-form derivative of the projected area of a triangle
# --------------------------------------------------------------------------

def _screen_area(cam, P):
    pts = []
    for v in P:
        e, f = None, None
        eye = np.array(cam.eye, np.float32).astype(float)
        tg = np.array(cam.target, np.float32).astype(float)
        up = np.array(cam.up, np.float32).astype(float)
        f = (tg - eye) / np.linalg.norm(tg - eye)
        r = np.cross(f, up / np.linalg.norm(up))
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        th = math.tan(float(np.float32(cam.fov_y_deg)) * math.pi / 360)
        p = v - eye
        z = p @ f
        sx = (p @ r / (z * th * cam.width / cam.height) + 1) * 0.5 * cam.width
        sy = (1 - p @ u / (z * th)) * 0.5 * cam.height
        pts.append((sx, sy))
    (ax, ay), (bx, by), (cx, cy) = pts
    return 0.5 * abs((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))


def test_primary_edges_projected_area_derivative():
    V = np.array([[-0.5, -0.4, 0.1], [0.6, -0.3, -0.2], [0.0, 0.55, 0.0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    mat = S.uniform_materials(1, kd=1.0, ks=0.0, rough=0.3)
    sc = O.OracleScene(V, F, mat, None, np.ones((8, 16, 3), np.float32))
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 48, 48)
    spp = 48
    d_img = np.ones((48 * 48, 3), np.float32)
    dV, dM, _, _ = sc.backward([cam], spp, 1, d_img, seed=4, flags=O.FLAG_PRIMARY)
    # closed form: sum of the image = L0 * (projected area in pixels); 3 channels
    Vd = V.astype(float)
    ref = np.zeros_like(Vd)
    h = 1e-6
    for i in range(3):
        for k in range(3):
            Vp, Vm = Vd.copy(), Vd.copy()
            Vp[i, k] += h
            Vm[i, k] -= h
            ref[i, k] = 3.0 * (_screen_area(cam, Vp) - _screen_area(cam, Vm)) / (2 * h)
    rel = np.linalg.norm(dV - ref) / np.linalg.norm(ref)
    assert rel < 0.04, (rel, dV, ref)
    assert np.all(dM == 0)


def test_primary_edges_hidden_triangle_contributes_nothing():
    """A triangle wholly behind a larger one, lit by a point light on the camera
    side: its edges are candidates (front-facing) and are sampled, but at every
    sampled point both side rays meet the occluder first, so the edge term gives
    its vertices exactly zero (what moving a hidden triangle does to the image).
    The two side paths would otherwise differ by the light's change over 2 eps on
    the occluder, an error that does not vanish with more samples.  The visible
    triangle's own edges still carry their jump."""
    front = np.array([[-0.8, -0.7, 0.5], [0.9, -0.6, 0.4], [0.0, 0.9, 0.5]], np.float32)
    back = np.array([[-0.2, -0.2, -0.5], [0.25, -0.15, -0.6], [0.0, 0.25, -0.5]], np.float32)
    V = np.concatenate([front, back])
    F = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    mat = S.uniform_materials(2, kd=1.0, ks=0.0, rough=0.3)
    lights = np.array([[0.3, 0.4, 2.5, 6.0, 6.0, 6.0]], np.float32)
    sc = O.OracleScene(V, F, mat, lights, None)
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 48, 48)
    # the back triangle projects inside the front one
    eye, fwd, r, u, th = _cam_frame(cam)

    def px(v):
        q = v.astype(float) - eye
        return np.array([q @ r / (q @ fwd), q @ u / (q @ fwd)])

    def inside(p, tri):
        a, b, c = (px(t) for t in tri)
        def cr(e, w):
            return e[0] * w[1] - e[1] * w[0]

        d = [cr(b - a, p - a), cr(c - b, p - b), cr(a - c, p - c)]
        return all(x > 0 for x in d) or all(x < 0 for x in d)

    assert all(inside(px(v), front) for v in back)
    d_img = np.ones((48 * 48, 3), np.float32)
    dV, _, _, eh = sc.backward([cam], 16, 1, d_img, seed=5, flags=O.FLAG_PRIMARY)
    assert np.all(dV[3:] == 0.0), dV[3:]
    assert np.linalg.norm(dV[:3]) > 1.0


# --------------------------------------------------------------------------
# primary edge term on closed meshes: per-face albedo under a constant
# environment, so that d(sum of the image)/dV is the derivative of the
# albedo-weighted projected area of the front faces (silhouette edges carry the
# object/background jump, interior edges the jump between face albedos), with
# the mesh clipped at the near plane when it reaches behind the eye
# --------------------------------------------------------------------------

ZNEAR = 1e-3


def _cam_frame(cam):
    eye = np.array(cam.eye, np.float32).astype(float)
    tg = np.array(cam.target, np.float32).astype(float)
    up = np.array(cam.up, np.float32).astype(float)
    f = (tg - eye) / np.linalg.norm(tg - eye)
    r = np.cross(f, up / np.linalg.norm(up))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(float(np.float32(cam.fov_y_deg)) * math.pi / 360)
    return eye, f, r, u, th


def _to_screen(cam, pts):
    eye, f, r, u, th = _cam_frame(cam)
    out = []
    for v in pts:
        p = v - eye
        z = p @ f
        out.append(((p @ r / (z * th * cam.width / cam.height) + 1) * 0.5 * cam.width,
                    (1 - p @ u / (z * th)) * 0.5 * cam.height))
    return out


def _clip_near(poly, cam):
    """Sutherland-Hodgman: the part of a 3-D polygon with depth > ZNEAR."""
    eye, f = _cam_frame(cam)[:2]
    d = [(v - eye) @ f - ZNEAR for v in poly]
    out = []
    for i in range(len(poly)):
        j = (i + 1) % len(poly)
        if d[i] > 0:
            out.append(poly[i])
        if (d[i] > 0) != (d[j] > 0):
            out.append(poly[i] + (poly[j] - poly[i]) * (d[i] / (d[i] - d[j])))
    return out


def _clip_image(poly, W, H):
    """Sutherland-Hodgman against the image rectangle [0, W] x [0, H]."""
    for k, lim, lower in ((0, 0.0, True), (0, float(W), False), (1, 0.0, True), (1, float(H), False)):
        out = []
        for i in range(len(poly)):
            a, b = poly[i], poly[(i + 1) % len(poly)]
            ia = a[k] >= lim if lower else a[k] <= lim
            ib = b[k] >= lim if lower else b[k] <= lim
            if ia:
                out.append(a)
            if ia != ib:
                t = (lim - a[k]) / (b[k] - a[k])
                out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
        poly = out
        if not poly:
            return []
    return poly


def _shoelace(poly):
    if len(poly) < 3:
        return 0.0
    return abs(sum(poly[i][0] * poly[(i + 1) % len(poly)][1] - poly[(i + 1) % len(poly)][0] * poly[i][1]
                   for i in range(len(poly)))) / 2


def _front_face_weighted_area(cam, V, F, w):
    """sum over faces facing the eye of w_f x (pixel area of the face's visible
    image).  From outside a convex body the front faces are exactly the visible
    surface and their images do not overlap; the visible image of a face is its
    part in front of the near plane, projected, inside the image."""
    eye = _cam_frame(cam)[0]
    tot = 0.0
    for fi, (a, b, c) in enumerate(F):
        if np.cross(V[b] - V[a], V[c] - V[a]) @ (eye - V[a]) <= 0:
            continue
        poly = _clip_near([V[a], V[b], V[c]], cam)
        if len(poly) >= 3:
            tot += w[fi] * _shoelace(_clip_image(_to_screen(cam, poly), cam.width, cam.height))
    return tot


def _outward(V, F):
    c = V.mean(0)
    F = F.copy()
    for i, (a, b, cc) in enumerate(F):
        if np.cross(V[b] - V[a], V[cc] - V[a]) @ (V[a] - c) < 0:
            F[i] = (a, cc, b)
    return F


def _primary_vs_closed_form(V, F, kd, cam, seeds, spp=16, ratio=4.0):
    mat = np.zeros((F.shape[0], 7), np.float32)
    mat[:, :3] = kd
    mat[:, 6] = 0.3
    sc = O.OracleScene(V, F, mat, None, np.ones((8, 16, 3), np.float32))
    d_img = np.ones((cam.width * cam.height, 3), np.float32)
    got = np.mean([sc.backward([cam], spp, 1, d_img, seed=s, flags=O.FLAG_PRIMARY, edge_ratio=ratio)[0]
                   for s in seeds], axis=0)
    # Lambertian kd, constant environment L0 = 1, one bounce, convex: every
    # visible point has expected radiance kd (per channel); d_image = 1 on
    # every channel sums the three albedos
    w = kd.astype(float).sum(axis=1)
    Vd = V.astype(float)
    ref = np.zeros_like(Vd)
    h = 1e-6
    for i in range(V.shape[0]):
        for k in range(3):
            Vp, Vm = Vd.copy(), Vd.copy()
            Vp[i, k] += h
            Vm[i, k] -= h
            ref[i, k] = (_front_face_weighted_area(cam, Vp, F, w) - _front_face_weighted_area(cam, Vm, F, w)) / (2 * h)
    return got, ref


def test_primary_edges_closed_convex_mesh_per_face_albedo():
    """Closed convex hull of 14 points, 24 faces with random albedos: exercises
    the candidate rule (an edge is sampled when one of its faces faces the eye:
    silhouettes and front interior edges, not back edges).  Silhouette-only
    candidates or a reversed facing test miss the interior jumps (12-13 %
    off); the estimator is within 1 % per seed."""
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(3)
    P = rng.normal(size=(14, 3))
    P = P / np.linalg.norm(P, axis=1, keepdims=True) * np.array([0.9, 0.7, 0.8])
    V = P.astype(np.float32)
    F = _outward(V.astype(float), ConvexHull(P).simplices.astype(np.int32))
    assert F.shape[0] == 24
    kd = np.random.default_rng(4).uniform(0.1, 0.9, size=(F.shape[0], 3)).astype(np.float32)
    cam = S.Camera((0.4, 0.5, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 64, 64)
    got, ref = _primary_vs_closed_form(V, F, kd, cam, seeds=(0, 1, 2))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel < 0.03, rel


def test_primary_edges_near_plane_clip():
    """A tetrahedron with one vertex behind the eye: its three edges through that
    vertex cross the near plane and are clipped there, then to the image; their
    visible images carry both the silhouette and the interior jumps, and the
    vertex behind the eye still moves them (dropping such edges is 69 % off)."""
    V = np.array([[-0.6, -0.5, 0.0], [0.5, -0.6, -0.3], [0.0, 0.6, 0.2], [1.2, 0.4, 4.2]], np.float32)
    F = _outward(V.astype(float), np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], np.int32))
    kd = np.array([[0.8, 0.8, 0.8], [0.3, 0.5, 0.7], [0.6, 0.2, 0.4], [0.9, 0.6, 0.1]], np.float32)
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 48, 48)
    eye, fwd = _cam_frame(cam)[:2]
    assert (V[3] - eye) @ fwd < 0 and all((V[i] - eye) @ fwd > 1 for i in range(3))
    got, ref = _primary_vs_closed_form(V, F, kd, cam, seeds=(0, 1, 2))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel < 0.03, rel
    assert np.linalg.norm(ref[3]) > 0.1 * np.linalg.norm(ref)
    assert np.linalg.norm(got[3] - ref[3]) < 0.05 * np.linalg.norm(ref[3])


# --------------------------------------------------------------------------
# secondary edge term: closed-form projected solid angle of an occluder
# --------------------------------------------------------------------------

def _psa(p, n, tri):
    """Projected solid angle of a spherical triangle seen from p (Lambert's formula)."""
    u = [(v - p) / np.linalg.norm(v - p) for v in tri]
    tot = 0.0
    for i in range(3):
        a, b = u[i], u[(i + 1) % 3]
        g = np.cross(a, b)
        g /= np.linalg.norm(g)
        tot += math.acos(np.clip(a @ b, -1, 1)) * (g @ n)
    return abs(tot) / 2


@pytest.mark.parametrize("hierarchy", [False, True])
def test_secondary_edges_polygon_irradiance_derivative(hierarchy):
    tri = np.array([[-0.3, 0.8, -0.2], [0.4, 0.9, -0.1], [0.05, 0.7, 0.45]], np.float32)
    floor = np.array([[-0.05, 0.0, -0.05], [0.05, 0.0, -0.05], [0.0, 0.0, 0.06]], np.float32)
    V = np.concatenate([floor, tri])
    F = np.array([[0, 2, 1], [3, 4, 5]], np.int32)
    mat = S.uniform_materials(2, kd=1.0, ks=0.0, rough=0.3)
    sc = O.OracleScene(V, F, mat, None, np.ones((8, 16, 3), np.float32))
    p = np.array([0.0, 0.0, 0.0])
    n = np.array([0.0, 1.0, 0.0])
    wo = np.array([0.3, 1.0, 0.2]) / np.linalg.norm([0.3, 1.0, 0.2])
    dV = sc.secondary_term(p, n, wo, face=0, budget=0, nsamples=400000, seed=2, hierarchy=hierarchy)
    # E(p) = kd/pi * L0 * (pi - PSA(triangle)), so dE/dv = -(1/pi) dPSA/dv
    T = tri.astype(float)
    ref = np.zeros((3, 3))
    h = 1e-6
    for i in range(3):
        for k in range(3):
            Tp, Tm = T.copy(), T.copy()
            Tp[i, k] += h
            Tm[i, k] -= h
            ref[i, k] = -(_psa(p, n, Tp) - _psa(p, n, Tm)) / (2 * h) / np.pi
    got = dV[3:]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel < 0.05, (rel, got, ref)
    assert np.abs(dV[:3]).max() == 0.0


@pytest.mark.parametrize("hierarchy", [False, True])
def test_secondary_edges_crease_between_two_albedos(hierarchy):
    """Creases and material boundaries (the interior option): a valley of two
    Lambertian faces of different albedo above a shading point, under a constant
    environment L0 = 1, convex as seen from below, so each face returns kd L0 in
    expectation.  The reflected radiance is
      I = kd_p/pi (pi - sum_faces (1 - kd_f) PSA_f),
    PSA the projected solid angle (Lambert's polygon formula).  The shared edge is
    no silhouette from the point, so its term (jump (kd_A - kd_B) L0) is sampled
    only with the option: with it the estimator meets the closed form, without it
    it is 32 % off."""
    wall = np.array([[-0.35, 0.55, -0.3], [0.3, 0.6, 0.35], [-0.5, 0.95, 0.4], [0.45, 0.9, -0.45]], np.float32)
    floor = np.array([[-1e-3, 0, -1e-3], [1e-3, 0, -1e-3], [0, 0, 1e-3]], np.float32)
    V = np.concatenate([floor, wall])
    F = np.array([[0, 2, 1], [3, 4, 5], [3, 6, 4]], np.int32)
    kdA, kdB = np.array([0.9, 0.6, 0.2]), np.array([0.1, 0.3, 0.8])
    mat = np.zeros((3, 7), np.float32)
    mat[0, :3], mat[1, :3], mat[2, :3] = 1.0, kdA, kdB
    mat[:, 6] = 0.3
    sc = O.OracleScene(V, F, mat, None, np.ones((8, 16, 3), np.float32))
    p, n = np.array([0.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    wo = np.array([0.3, 1.0, 0.2]) / np.linalg.norm([0.3, 1.0, 0.2])
    kdA32, kdB32 = mat[1, :3].astype(float), mat[2, :3].astype(float)

    def irradiance(W):
        A, B = W[[3, 4, 5]], W[[3, 6, 4]]
        return sum(np.pi - (1 - kdA32[c]) * _psa(p, n, A) - (1 - kdB32[c]) * _psa(p, n, B) for c in range(3)) / (3 * np.pi)

    Vd = V.astype(float)
    ref = np.zeros_like(Vd)
    h = 1e-6
    for i in range(3, 7):
        for k in range(3):
            Vp, Vm = Vd.copy(), Vd.copy()
            Vp[i, k] += h
            Vm[i, k] -= h
            ref[i, k] = (irradiance(Vp) - irradiance(Vm)) / (2 * h)
    with_int = sc.secondary_term(p, n, wo, face=0, budget=1, nsamples=400000, seed=2, hierarchy=hierarchy,
                                 interior=True)
    without = sc.secondary_term(p, n, wo, face=0, budget=1, nsamples=100000, seed=2, hierarchy=hierarchy,
                                interior=False)
    rel = np.linalg.norm(with_int - ref) / np.linalg.norm(ref)
    rel_without = np.linalg.norm(without - ref) / np.linalg.norm(ref)
    assert rel < 0.03, rel
    assert rel_without > 0.2, rel_without
    assert np.abs(with_int[:3]).max() == 0.0


# --------------------------------------------------------------------------
# edge list and LBVH reference
# --------------------------------------------------------------------------

def test_edge_list_canonical_closed_mesh():
    V, F = S.geodesic_sphere(4)
    sc = O.OracleScene(V.astype(np.float32), F, S.uniform_materials(F.shape[0]))
    E = sc.edges()
    assert E.shape[0] == 480
    assert np.all(E[:, 0] < E[:, 1])
    keys = E[:, 0].astype(np.int64) * 100000 + E[:, 1]
    assert np.all(np.diff(keys) > 0)
    assert np.all(E[:, 3] > E[:, 2])          # closed: two faces, f1 < f2
    for va, vb, f1, f2 in E[:50]:
        for f in (f1, f2):
            assert va in F[f] and vb in F[f]
    V32 = V.astype(np.float32).astype(np.float64)
    total = sum(np.linalg.norm(V32[b] - V32[a]) for a, b, _, _ in E)
    assert abs(sc.edge_total() - total) < 1e-9


def _spread(v):
    r = 0
    for i in range(10):
        r |= ((v >> i) & 1) << (3 * i)
    return r


@pytest.mark.parametrize("k", [1, 3, 9])
def test_lbvh_reference_definition(k):
    V, F = S.noise_sphere(k, 0.1, noise_seed=1)
    V = V.astype(np.float32)
    keys, child, parent, aabb = O.lbvh(V, F)
    n = F.shape[0]
    # Morton codes from the definition, in float32
    tri = V[F]
    mn, mx = tri.min(axis=1), tri.max(axis=1)
    c = ((mn + mx) * np.float32(0.5)).astype(np.float32)
    lo, hi = c.min(axis=0), c.max(axis=0)
    ext = max(float(h) - float(l) for l, h in zip(lo, hi))      # cubic cells: one scale for all axes
    s = np.full(3, np.float32(1024.0 / ext) if ext > 0 else np.float32(0), np.float32)
    q = np.clip(np.floor((c - lo).astype(np.float32) * s).astype(np.int64), 0, 1023)
    mort = np.array([(_spread(a) << 2) | (_spread(b) << 1) | _spread(cc) for a, b, cc in q], np.uint64)
    ref = np.sort((mort << np.uint64(32)) | np.arange(n, dtype=np.uint64))
    assert np.array_equal(keys, ref)
    LEAF = 0x80000000
    seen = np.zeros(n, int)

    def rng_of(code):
        if code & LEAF:
            i = code & 0x7FFFFFFF
            seen[i] += 1
            return i, i, aabb[n - 1 + i]
        a0, b0, box0 = rng_of(int(child[code, 0]) & 0xFFFFFFFF)
        a1, b1, box1 = rng_of(int(child[code, 1]) & 0xFFFFFFFF)
        assert b0 + 1 == a1                      # contiguous leaf ranges
        box = aabb[code]
        for bb in (box0, box1):
            assert np.all(box[:3] <= bb[:3]) and np.all(box[3:] >= bb[3:])
        assert np.array_equal(box[:3], np.minimum(box0[:3], box1[:3]))
        assert np.array_equal(box[3:], np.maximum(box0[3:], box1[3:]))
        # radix-tree property: the split sits at the first differing bit of the range
        pre = 64 - int(keys[a0] ^ keys[b1]).bit_length()
        assert 64 - int(keys[b0] ^ keys[a1]).bit_length() == pre
        return a0, b1, box

    if n > 1:
        a, b, _ = rng_of(0)
        assert (a, b) == (0, n - 1)
        assert parent[0] == -1
        for i in range(n - 1):
            for cc in child[i]:
                cc = int(cc) & 0xFFFFFFFF
                idx = (n - 1 + (cc & 0x7FFFFFFF)) if cc & LEAF else cc
                assert parent[idx] == i
    assert np.all(seen <= 1) and (n == 1 or np.all(seen == 1))
    for i in range(n):
        f = int(keys[i] & np.uint64(0xFFFFFFFF))
        assert np.array_equal(aabb[n - 1 + i, :3], mn[f]) and np.array_equal(aabb[n - 1 + i, 3:], mx[f])


# --------------------------------------------------------------------------
# mesh colours (Sec. 3.3 "Representation")
# --------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 8])
def test_mesh_color_layout_is_a_bijection_per_triangle(r):
    """The cells {(i, j): 0 <= i <= r, 0 <= j <= r - i} of every triangle map one to
    one onto that triangle's block of (r+1)(r+2)/2 texels, blocks in triangle
    order; r = 0 is one texel per triangle."""
    T = (r + 1) * (r + 2) // 2
    for t in (0, 1, 7, 1000):
        seen = set()
        for i in range(r + 1):
            for j in range(r - i + 1):
                # a point strictly inside cell (i, j) of the barycentric grid
                a, b = ((i + 0.25) / r, (j + 0.25) / r) if r else (0.25, 0.25)
                k = O.texel_index(r, t, a, b)
                assert t * T <= k < (t + 1) * T
                seen.add(k)
        assert len(seen) == T
    # the corners and the far edge of the domain stay inside the block
    for a, b in [(0, 0), (1, 0), (0, 1), (0.5, 0.5), (-1e-9, 0.3), (0.7, 0.3 + 1e-9)]:
        assert 5 * T <= O.texel_index(r, 5, a, b) < 6 * T


def _bary_numpy(p, v0, v1, v2):
    """(alpha, beta) with p = v0 + alpha (v1 - v0) + beta (v2 - v0), by least squares."""
    A = np.stack([v1 - v0, v2 - v0], 1)
    sol, *_ = np.linalg.lstsq(A, p - v0, rcond=None)
    return sol


def test_mesh_colors_lambertian_plane_point_light():
    """Per-sample radiance of a two-triangle plane textured with mesh colours at
    r = 4 (a different albedo per texel): kd of the hit point's texel / pi * I cos / r^2."""
    V = np.array([[-1.2, -1.2, 0], [1.2, -1.2, 0], [1.2, 1.2, 0], [-1.2, 1.2, 0]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    r = 4
    T = (r + 1) * (r + 2) // 2
    rng = np.random.default_rng(12)
    tex = np.zeros((2 * T, 7), np.float32)
    tex[:, :3] = rng.uniform(0.1, 0.9, (2 * T, 3))
    tex[:, 6] = 0.3
    light = np.array([[0.5, 0.3, 2.0, 10.0, 8.0, 6.0]], np.float32)
    sc = O.OracleScene(V, F, tex[:2], light, None, scene_id=3)
    sc.set_mesh_colors(r, tex)
    cam = S.Camera((0.0, 0.0, 3.0), (0, 0, 0), (0, 1, 0), 45.0, 16, 12)
    seed, spp = 9, 2
    rgb, _ = sc.render_samples([cam], spp, 1, seed)
    pl, I = light[0, :3].astype(float), light[0, 3:].astype(float)
    Vd = V.astype(float)
    worst, used = 0.0, set()
    for y in range(12):
        for x in range(16):
            for j in range(spp):
                u = draw4(y * 16 + x, j, 0, 0, seed, 3)
                o, d = _pinhole(cam, x + u[0], y + u[1])
                p = o + (-o[2] / d[2]) * d
                if max(abs(p[0]), abs(p[1])) > 1.2 - 1e-6:       # off the plane (or on its rim)
                    if max(abs(p[0]), abs(p[1])) > 1.2 + 1e-6:
                        assert not rgb[y * 16 + x, j].any()
                    continue
                # face of the quad containing p (diagonal v0-v2: x >= y is face 0)
                f = 0 if p[0] >= p[1] else 1
                a, b = _bary_numpy(p, *Vd[F[f]])
                k = O.texel_index(r, f, a, b)
                used.add(k)
                wl = pl - p
                r2 = wl @ wl
                expect = tex[k, :3].astype(float) / np.pi * I * (wl[2] / math.sqrt(r2)) / r2
                worst = max(worst, np.abs(rgb[y * 16 + x, j] - expect).max() / expect.max())
    assert worst < 1e-12
    assert len(used) > 15         # the view covers most of the 30 texels


def _textured_test_scene(r, constant_per_face):
    rng = np.random.default_rng(44)
    V, F = S.noise_sphere(4, 0.2, noise_seed=5)
    floor = np.array([[-3, -1.2, -3], [3, -1.2, -3], [3, -1.2, 3], [-3, -1.2, 3]], np.float32)
    nv = V.shape[0]
    Vf = np.concatenate([V, floor]).astype(np.float32)
    Ff = np.concatenate([F, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    mat = S.random_materials(Ff.shape[0], rng)
    T = (r + 1) * (r + 2) // 2
    tex = np.repeat(mat, T, axis=0) if constant_per_face else S.random_materials(Ff.shape[0] * T, rng)
    env = S.gaussian_lobe_envmap(rng, 32, 16)
    lights = np.array([[1.0, 2.0, 1.5, 6, 6, 6]], np.float32)
    return Vf, Ff, mat, tex, lights, env


def test_mesh_colors_constant_per_face_equal_per_face_materials():
    """Texels equal within every triangle render exactly like per-face materials,
    and the texel gradients of a triangle sum to its per-face gradient (all terms)."""
    r = 3
    Vf, Ff, mat, tex, lights, env = _textured_test_scene(r, True)
    cams = [S.look_at_origin((0.3, 0.9, 3.0), 12, 10)]
    a = O.OracleScene(Vf, Ff, mat, lights, env)
    b = O.OracleScene(Vf, Ff, mat, lights, env)
    b.set_mesh_colors(r, tex)
    ia, _ = a.render(cams, 4, 2, seed=5)
    ib, _ = b.render(cams, 4, 2, seed=5)
    assert np.array_equal(ia, ib)
    d = np.random.default_rng(3).normal(size=ia.shape).astype(np.float32)
    dVa, dMa, _, _ = a.backward(cams, 4, 2, d, seed=5, flags=7)
    dVb, dMb, _, _ = b.backward(cams, 4, 2, d, seed=5, flags=7)
    T = (r + 1) * (r + 2) // 2
    assert np.allclose(dVa, dVb, rtol=1e-12, atol=1e-15)
    assert np.allclose(dMb.reshape(-1, T, 7).sum(1), dMa, rtol=1e-10, atol=1e-14)
    assert np.abs(dMa).max() > 0


def test_fd_frozen_mesh_colors():
    """Dual-number derivative with respect to texels and vertices ≡ central
    differences of the frozen path, textured scene at r = 2, envmap + point light."""
    Vf, Ff, mat, tex, lights, env = _textured_test_scene(2, False)
    sc = O.OracleScene(Vf, Ff, mat, lights, env)
    sc.set_mesh_colors(2, tex)
    cams = [S.look_at_origin((0.3, 0.9, 3.0), 16, 16)]
    samples = [(0, x, y, j) for (x, y) in [(8, 8), (5, 9), (10, 4), (3, 13)] for j in range(2)]
    assert _fd_check(sc, cams, 2, 3, samples, flags=1) > 50


# --------------------------------------------------------------------------
# 1 -> 4 subdivision (Sec. 3.2 "Subdivision")
# --------------------------------------------------------------------------

def test_subdivide_single_triangle_by_hand():
    V = np.array([[0, 0, 0], [2, 0, 0], [0, 4, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    V2, F2 = O.subdivide(V, F)
    # edges in (min, max) order: (0,1) -> 3, (0,2) -> 4, (1,2) -> 5
    assert np.array_equal(V2, np.array([[0, 0, 0], [2, 0, 0], [0, 4, 0], [1, 0, 0], [0, 2, 0], [1, 2, 0]], np.float32))
    assert np.array_equal(F2, np.array([[0, 3, 4], [1, 5, 3], [2, 4, 5], [3, 5, 4]], np.int32))


@pytest.mark.parametrize("k", [1, 3])
def test_subdivide_invariants_closed_mesh(k):
    V, F = S.noise_sphere(k, 0.2, noise_seed=3)
    V = V.astype(np.float32)
    V2, F2 = O.subdivide(V, F)
    ne = 30 * k * k
    assert V2.shape == (V.shape[0] + ne, 3) and F2.shape == (4 * F.shape[0], 3)
    # Euler characteristic of a sphere, and every edge shared by exactly two faces
    e2 = {}
    for f in F2:
        for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            e2[(min(a, b), max(a, b))] = e2.get((min(a, b), max(a, b)), 0) + 1
    assert V2.shape[0] - len(e2) + F2.shape[0] == 2
    assert set(e2.values()) == {2}
    # the four children tile the parent: areas add up and normals keep their direction
    def area_normal(VV, FF):
        n = np.cross(VV[FF[:, 1]] - VV[FF[:, 0]], VV[FF[:, 2]] - VV[FF[:, 0]]).astype(np.float64)
        return n
    npar = area_normal(V.astype(np.float64), F)
    nch = area_normal(V2.astype(np.float64), F2).reshape(-1, 4, 3)
    assert np.allclose(nch.sum(1), npar, rtol=1e-5, atol=1e-7)
    assert (np.einsum("fcj,fj->fc", nch, npar) > 0).all()


# --------------------------------------------------------------------------
# point-light shadow boundaries (row NEXT-1)
# --------------------------------------------------------------------------

def _gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def test_shadow_edges_closed_form_polygon():
    """A Lambertian floor z = 0 seen straight down, lit by one point light and
    shadowed by a triangle that the camera does not see.  The image is zero
    inside the shadow polygon (the central projection of the triangle from the
    light) and L(x) = kd/pi I cos/r^2 outside, so d(sum of pixels)/d(occluder
    vertex) = - boundary integral of L times the polygon's outward normal
    velocity, evaluated here by Gauss-Legendre quadrature along the three edges
    of the projected polygon.  The shadow-edge estimator must match it."""
    floor = np.array([[-3, -3, 0], [3, -3, 0], [3, 3, 0], [-3, 3, 0]], np.float32)
    occ = np.array([[-1.2, -0.2, 1.0], [-0.8, -0.3, 1.05], [-1.0, 0.3, 0.95]], np.float32)
    V = np.concatenate([floor, occ])
    F = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6]], np.int32)
    kd = 0.6
    mat = np.zeros((3, 7), np.float32)
    mat[:, :3] = kd
    mat[:, 6] = 0.5
    light = np.array([[-2.2, 0.0, 3.0, 10.0, 10.0, 10.0]], np.float32)
    W = H = 64
    cam = S.Camera((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, W, H)
    sc = O.OracleScene(V, F, mat, light, None)
    d_img = np.ones((W * H, 3), np.float32)
    dV, _, _, eh = sc.backward([cam], 1, 1, d_img, seed=3, flags=8, edge_ratio=50.0)
    assert (eh[W * H * 50:] != 0).all()          # every shadow sample hashes its decisions
    est = dV[4:7]

    pl, I = light[0, :3].astype(float), float(light[0, 3])
    Vd = V.astype(float)

    def screen(X):                       # the camera's projection (pinhole looking down -z, up +y)
        e = np.array([0.0, 0.0, 2.5])
        f, r, u = np.array([0, 0, -1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
        th = math.tan(math.radians(22.5))
        p = X - e
        z = p @ f
        return np.array([(p @ r / (z * th) + 1.0) * 0.5 * W, (1.0 - p @ u / (z * th)) * 0.5 * H])

    def unscreen(s):                     # floor point under screen point s
        th = math.tan(math.radians(22.5))
        a = (2.0 * s[0] / W - 1.0) * th * 2.5
        b = (1.0 - 2.0 * s[1] / H) * th * 2.5
        return np.array([a, b, 0.0])

    def L(x):
        dl = pl - x
        r2 = dl @ dl
        return kd / math.pi * I * (dl[2] / math.sqrt(r2)) / r2

    def Q(v):                            # shadow of occluder vertex v on the floor
        lam = pl[2] / (pl[2] - v[2])
        return pl + lam * (v - pl)

    q = np.array([screen(Q(v)) for v in Vd[4:7]])
    area2 = (q[1, 0] - q[0, 0]) * (q[2, 1] - q[0, 1]) - (q[2, 0] - q[0, 0]) * (q[1, 1] - q[0, 1])
    uq, wq = _gauss_legendre(64)
    expect = np.zeros((3, 3))
    h = 1e-6
    for i in range(3):
        for k in range(3):
            vp, vm = Vd[4 + i].copy(), Vd[4 + i].copy()
            vp[k] += h
            vm[k] -= h
            qdot = (screen(Q(vp)) - screen(Q(vm))) / (2 * h)     # velocity of polygon vertex i
            tot = 0.0
            for a in range(3):
                b2 = (a + 1) % 3
                if i not in (a, b2):
                    continue
                d = q[b2] - q[a]
                ln = math.hypot(*d)
                nout = np.array([d[1], -d[0]]) / ln * (1.0 if area2 > 0 else -1.0)
                for uu, ww in zip(uq, wq):
                    s = q[a] + uu * d
                    wgt = (1.0 - uu) if i == a else uu
                    tot += ww * ln * L(unscreen(s)) * wgt * (qdot @ nout)
            expect[i, k] = -3.0 * tot         # three colour channels, d_image = 1 each
    scale = np.abs(expect).max()
    assert scale > 0
    assert np.abs(est - expect).max() < 0.03 * scale, (est, expect)


# --------------------------------------------------------------------------
# treelet restructuring of the Karras tree
# --------------------------------------------------------------------------

C_INNER = 1.2


def _area(b):
    d = np.maximum(np.asarray(b[3:], np.float64) - np.asarray(b[:3], np.float64), 0.0)
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0])


def _tree_check(child, parent, aabb, n):
    """Every leaf reached once from the root, parent links consistent, every box
    the exact union of its children's; returns the SAH cost in float64."""
    LEAF = 0x80000000
    seen = np.zeros(n, int)
    cost = 0.0
    stack = [0]
    assert parent[0] == -1
    while stack:
        i = stack.pop()
        cost += C_INNER * _area(aabb[i])
        boxes = []
        for c in child[i]:
            c = int(c) & 0xFFFFFFFF
            if c & LEAF:
                j = c & 0x7FFFFFFF
                seen[j] += 1
                assert parent[n - 1 + j] == i
                boxes.append(aabb[n - 1 + j])
                cost += _area(aabb[n - 1 + j])
            else:
                assert parent[c] == i
                boxes.append(aabb[c])
                stack.append(c)
        assert np.array_equal(aabb[i][:3], np.minimum(boxes[0][:3], boxes[1][:3]))
        assert np.array_equal(aabb[i][3:], np.maximum(boxes[0][3:], boxes[1][3:]))
    assert (seen == 1).all()
    return cost


@pytest.mark.parametrize("which", ["sphere80", "sphere720", "torus_small"])
def test_treelets_valid_and_lower_sah(which):
    if which == "torus_small":
        V, F = S.noise_torus(40, 20, 0.1, noise_seed=13)
    else:
        V, F = S.noise_sphere(2 if which == "sphere80" else 6, 0.1, noise_seed=1)
    V = V.astype(np.float32)
    n = F.shape[0]
    k0, c0, p0, a0 = O.lbvh(V, F)
    costs = [_tree_check(c0, p0, a0, n)]
    for rounds in (1, 2, 3):
        k, c, p, a = O.lbvh(V, F, treelet_rounds=rounds)
        assert np.array_equal(k, k0)                       # leaves (sorted keys) and their boxes are untouched
        assert np.array_equal(a[n - 1:], a0[n - 1:]) and np.array_equal(a[0], a0[0])
        costs.append(_tree_check(c, p, a, n))
    assert costs[1] < costs[0] and costs[2] <= costs[1] * (1 + 1e-6) and costs[3] <= costs[2] * (1 + 1e-6)
    assert costs[2] < 0.99 * costs[0]


def _all_trees(items):
    """Every full binary tree over the labelled leaves (nested pairs)."""
    if len(items) == 1:
        yield items[0]
        return
    first, rest = items[0], items[1:]
    m = len(rest)
    for mask in range(1 << m):
        if mask == (1 << m) - 1:
            continue
        left = [first] + [rest[i] for i in range(m) if mask >> i & 1]
        right = [rest[i] for i in range(m) if not mask >> i & 1]
        for a in _all_trees(left):
            for b in _all_trees(right):
                yield (a, b)


def _tree_cost(t, boxes):
    if not isinstance(t, tuple):
        return _area(boxes[t]), boxes[t]
    ca, ba = _tree_cost(t[0], boxes)
    cb, bb = _tree_cost(t[1], boxes)
    u = np.concatenate([np.minimum(ba[:3], bb[:3]), np.maximum(ba[3:], bb[3:])])
    return C_INNER * _area(u) + ca + cb, u


@pytest.mark.parametrize("n", [3, 6, 7])
def test_treelets_reach_brute_force_optimum_on_small_trees(n):
    """With exactly 7 triangles the root's treelet holds every leaf, so the
    restructured tree must cost what the best of all (2n-3)!! = 10395 binary
    trees costs; below 7 triangles no node qualifies and the tree is the radix tree."""
    rng = np.random.default_rng(20 + n)
    for trial in range(4 if n == 7 else 2):
        V = rng.uniform(-1, 1, size=(3 * n, 3)).astype(np.float32) * np.array([1.0, 0.2, 1.0], np.float32)
        V[3:] += rng.uniform(-0.5, 0.5, size=(1, 3)).astype(np.float32)
        F = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
        k, c, p, a = O.lbvh(V, F, treelet_rounds=1)
        if n < 7:
            k0, c0, p0, a0 = O.lbvh(V, F)
            assert np.array_equal(c, c0) and np.array_equal(p, p0) and np.array_equal(a, a0)
            continue
        got = _tree_check(c, p, a, n)
        boxes = [a[n - 1 + i].astype(np.float64) for i in range(n)]
        best = min(_tree_cost(t, boxes)[0] for t in _all_trees(list(range(n))))
        assert abs(got - best) <= 1e-5 * best, (trial, got, best)


# --------------------------------------------------------------------------
# visible-normal sampling of the specular lobe
# --------------------------------------------------------------------------

def test_erfinv_against_scipy():
    from scipy.special import erfinv
    for y in [-0.9999998, -0.999, -0.7, -0.1, 0.0, 1e-9, 0.3, 0.5, 0.95, 0.9999998]:
        assert abs(O.erfinv(y) - erfinv(y)) <= 1e-13 * max(1.0, abs(erfinv(y)))


@pytest.mark.parametrize("alpha", [0.05, 0.3, 0.8])
def test_vndf_pdf_at_normal_incidence_is_the_classical_pdf(alpha):
    """Seen along the normal every microfacet is visible (G1 = 1, wo.h = n.h), so
    the visible-normal pdf equals the D cos(theta_h) / (4 wo.h) one."""
    rng = np.random.default_rng(3)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(200):
        wi = rng.normal(size=3)
        wi[2] = abs(wi[2])
        wi /= np.linalg.norm(wi)
        a, b = O.bsdf_pdf(wi, n, n, alpha, True), O.bsdf_pdf(wi, n, n, alpha, False)
        assert abs(a - b) <= 1e-12 * max(a, 1e-300)


def test_vndf_samples_only_visible_normals():
    """Every sampled half-vector faces wo (wo.h > 0), at grazing angles too."""
    rng = np.random.default_rng(5)
    n = np.array([0.0, 0.0, 1.0])
    for to in (0.1, 1.2, 1.55):
        wo = np.array([math.sin(to), 0.0, math.cos(to)])
        for u in rng.random((3000, 4)):
            u[0] = 0.1                                   # specular lobe
            _, wi = O.bsdf_sample(u, wo, n, 0.4, True)
            h = wi + wo
            assert np.dot(wo, h / np.linalg.norm(h)) > 0.0


# --------------------------------------------------------------------------
# secondary-edge importance hierarchy
# --------------------------------------------------------------------------

def _node_weight(box, ln, nb, p, nrm, sil=True):
    """The node importance written out in float32 (box lower/upper corners, total
    length, box of the face normals)."""
    f = np.float32
    c = (box[:3] + box[3:]) * f(0.5) - p
    e = box[3:] - box[:3]
    reach = (c[0] * nrm[0] + c[1] * nrm[1] + c[2] * nrm[2]) + f(0.5) * ((abs(nrm[0]) * e[0] + abs(nrm[1]) * e[1])
                                                                       + abs(nrm[2]) * e[2])
    tol = f(2.0 ** -16) * (((abs(c[0]) + abs(c[1])) + abs(c[2])) + ((e[0] + e[1]) + e[2]))
    if not reach > -tol:
        return f(0.0)
    if sil:
        lo = hi = rad = f(0.0)
        for k in range(3):
            a, b = -nb[k] * c[k], -nb[3 + k] * c[k]
            lo, hi = lo + min(a, b), hi + max(a, b)
            rad = rad + max(abs(nb[k]), abs(nb[3 + k])) * (f(0.5) * e[k])
        if lo - rad > tol or hi + rad < -tol:
            return f(0.0)
    dl1 = ((abs(c[0]) + abs(c[1])) + abs(c[2])) + f(0.5) * ((e[0] + e[1]) + e[2])
    cb = (reach + tol) / (dl1 + tol)
    return f(ln * cb / ((c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) + f(0.25) * ((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2])))


def _all_edge_probs(tree, p, nrm, sil=True):
    """Probability of every edge under the descent, and of a dead end (a node
    whose children both weigh zero); the two add up to one."""
    keys, child, parent, box, ln, nb = tree
    n = keys.shape[0]
    LEAF = 0x80000000
    probs = np.zeros(n)
    dead = 0.0

    def idx(code):
        return n - 1 + (code & 0x7FFFFFFF) if code & LEAF else code

    stack = [(0, 1.0)]
    while stack:
        node, pr = stack.pop()
        c = [int(x) & 0xFFFFFFFF for x in child[node]]
        w = [_node_weight(box[idx(k)], ln[idx(k)], nb[idx(k)], p, nrm, sil) for k in c]
        tot = np.float32(w[0] + w[1])
        if not tot > 0:
            dead += pr
            continue
        for k, wk in zip(c, w):
            q = pr * float(np.float32(wk / tot))
            if q == 0:
                continue
            if k & LEAF:
                probs[int(keys[k & 0x7FFFFFFF]) & 0xFFFFFFFF] += q
            else:
                stack.append((k, q))
    assert abs(probs.sum() + dead - 1.0) < 1e-5
    return probs, dead


def test_edge_tree_valid():
    V, F = S.noise_sphere(4, 0.1, noise_seed=2)
    sc = O.OracleScene(V.astype(np.float32), F, S.uniform_materials(F.shape[0]), None, None)
    keys, child, parent, box, ln, nb = sc.edge_tree()
    E = sc.edges()
    n = E.shape[0]
    V32 = V.astype(np.float32)
    assert _tree_check(child, parent, box, n) > 0              # leaves once, boxes exact unions
    assert _tree_check(child, parent, nb, n) > 0               # normal boxes: exact unions too
    # a leaf's normal box holds the unit normals of both faces beside its edge
    Vd = V32.astype(np.float64)
    for i, key in enumerate(keys):
        e = int(key) & 0xFFFFFFFF
        for f in E[e, 2:]:
            nf = np.cross(Vd[F[f, 1]] - Vd[F[f, 0]], Vd[F[f, 2]] - Vd[F[f, 0]])
            nf /= np.linalg.norm(nf)
            assert np.all(nb[n - 1 + i, :3] <= nf + 1e-7) and np.all(nf <= nb[n - 1 + i, 3:] + 1e-7)
    leaf_len = np.sqrt(((V32[E[:, 1]].astype(np.float64) - V32[E[:, 0]].astype(np.float64)) ** 2).sum(1))
    order = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.array_equal(ln[n - 1:], leaf_len[order].astype(np.float32))
    LEAF = 0x80000000
    for i in range(n - 1):
        c = [int(x) & 0xFFFFFFFF for x in child[i]]
        l = [ln[n - 1 + (k & 0x7FFFFFFF)] if k & LEAF else ln[k] for k in c]
        assert ln[i] == np.float32(l[0] + l[1])
    assert abs(ln[0] - leaf_len.sum()) < 1e-5 * leaf_len.sum()


def test_edge_tree_sampling_matches_probabilities():
    """Sampled edges follow the product of the per-level probabilities (with the
    dead ends, where both children of a node weigh zero, as one more outcome);
    edges wholly behind the tangent plane are never drawn."""
    from scipy import stats
    Vs, Fs = S.noise_sphere(3, 0.1, noise_seed=5)
    floor = np.array([[-3, -1.5, -3], [3, -1.5, -3], [3, -1.5, 3], [-3, -1.5, 3]], np.float32)
    nv = Vs.shape[0]
    V = np.concatenate([Vs, floor]).astype(np.float32)
    F = np.concatenate([Fs, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    sc = O.OracleScene(V, F, S.uniform_materials(F.shape[0]), None, None)
    tree = sc.edge_tree()
    E = sc.edges()
    x = np.array([0.6, -1.5, 0.3])                      # on the floor, under the sphere
    nrm = np.array([0.1, 0.98, 0.15]) / np.linalg.norm([0.1, 0.98, 0.15])
    P, dead = _all_edge_probs(tree, x.astype(np.float32), nrm.astype(np.float32))
    N = 40000
    counts = np.zeros(E.shape[0] + 1)
    for i in range(N):
        e, pe = sc.edge_tree_sample(x, nrm, i, seed=3)
        assert e == -1 or abs(pe - P[e]) <= 1e-6 * P[e] + 1e-12
        counts[e] += 1
    P = np.append(P, dead)
    behind = np.array([(np.stack([V[a], V[b]]) - x) @ nrm for a, b in E[:, :2]]).max(axis=1) < -1e-3
    behind = np.append(behind, False)
    assert behind.any() and counts[behind].sum() == 0 and P[behind].sum() == 0
    keep = P * N > 15
    exp = P[keep] * N
    obs = counts[keep]
    exp *= obs.sum() / exp.sum()
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def _hier_scene():
    Vs, Fs = S.noise_sphere(4, 0.2, noise_seed=9)
    floor = np.array([[-3, -1.4, -3], [3, -1.4, -3], [3, -1.4, 3], [-3, -1.4, 3]], np.float32)
    nv = Vs.shape[0]
    V = np.concatenate([Vs, floor]).astype(np.float32)
    F = np.concatenate([Fs, [[nv, nv + 2, nv + 1], [nv, nv + 3, nv + 2]]]).astype(np.int32)
    return V, F, O.OracleScene(V, F, S.uniform_materials(F.shape[0]), None, None)


def _could_contribute(V, F, E, e, x, n, face, silhouettes):
    """Brute force, in float64: edge e can carry a secondary-edge sample at x when
    it is not an edge of the shading face, is a silhouette from x (one adjacent
    face plane with x in front, the other with x behind, or a boundary edge)
    unless silhouettes is off, and has a point seen above the tangent plane."""
    va, vb, f1, f2 = (int(t) for t in E[e])
    if face in (f1, f2):
        return False
    Vd = V.astype(np.float64)
    if silhouettes and f2 >= 0:
        s = [np.dot(np.cross(Vd[F[f, 1]] - Vd[F[f, 0]], Vd[F[f, 2]] - Vd[F[f, 0]]), x - Vd[va]) for f in (f1, f2)]
        if (s[0] > 0) == (s[1] > 0):
            return False
    y = Vd[va][None, :] + np.linspace(0, 1, 65)[:, None] * (Vd[vb] - Vd[va])[None, :]
    d = y - x
    r = np.linalg.norm(d, axis=1)
    return bool(((d @ n) > 1e-5 * r).any())


@pytest.mark.parametrize("silhouettes", [True, False])
def test_edge_tree_keeps_every_contributing_edge(silhouettes):
    """The hierarchy only ever zeroes edges that cannot contribute: at shading
    points on a bumpy sphere and on the floor under it, every edge that passes
    the brute-force test has a positive probability; with the silhouette bound on,
    more of the probability lands on such edges than under the length CDF."""
    V, F, sc = _hier_scene()
    tree = sc.edge_tree()
    E = sc.edges()
    Vd = V.astype(np.float64)
    rng = np.random.default_rng(4)
    points = []
    for f in rng.choice(F.shape[0] - 2, 6, replace=False):
        b = rng.dirichlet([2.0, 2.0, 2.0])
        x = b @ Vd[F[f]]
        n = np.cross(Vd[F[f, 1]] - Vd[F[f, 0]], Vd[F[f, 2]] - Vd[F[f, 0]])
        points.append((x, n / np.linalg.norm(n), int(f)))
    points.append((np.array([0.7, -1.4, 0.2]), np.array([0.0, 1.0, 0.0]), F.shape[0] - 1))
    points.append((np.array([-2.2, -1.4, 1.9]), np.array([0.0, 1.0, 0.0]), F.shape[0] - 2))
    useful = []
    for x, n, face in points:
        P, dead = _all_edge_probs(tree, x.astype(np.float32), n.astype(np.float32), silhouettes)
        ok = np.array([_could_contribute(V, F, E, e, x, n, face, silhouettes) for e in range(E.shape[0])])
        assert ok.any() and (P[ok] > 0).all()
        ln_e = np.linalg.norm(Vd[E[:, 1]] - Vd[E[:, 0]], axis=1)
        useful.append((P[ok].sum(), ln_e[ok].sum() / ln_e.sum()))
        for i in range(50):                              # the sampler draws from these probabilities
            e, pe = sc.edge_tree_sample(x, n, i, seed=8, silhouettes=silhouettes)
            assert e == -1 or abs(pe - P[e]) <= 1e-6 * P[e] + 1e-12
    if silhouettes:                                      # more useful draws than the length CDF makes
        h, c = np.array(useful).T
        assert h.mean() > 2.0 * c.mean(), useful

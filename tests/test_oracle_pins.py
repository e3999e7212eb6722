"""Pins of the FP64 oracle against closed forms, library routines, brute force
and invariants -- never against a retyping of its own formulas.

Each test names the passage of the paper the pinned part follows.
"""

import math

import numpy as np
import pytest
import scipy.integrate
import scipy.ndimage
import torch

from oracle import oracle
from workloads import camera, medium, weights

G_VALUES = (0.0, 0.5, 0.85, 0.9, 0.95, -0.6)


# --------------------------------------------------------------------------
# Henyey-Greenstein phase, Sec. III.B.3 eq. (5)

@pytest.mark.parametrize("g", G_VALUES)
def test_hg_normalises_over_the_sphere(g):
    # a phase function integrates to one over the sphere: 2 pi int_{-1}^{1} f dmu = 1
    val, _ = scipy.integrate.quad(lambda mu: oracle.hg(g, mu), -1.0, 1.0, limit=400,
                                  epsabs=1e-13, epsrel=1e-12)
    assert abs(2.0 * math.pi * val - 1.0) < 1e-9


@pytest.mark.parametrize("g", G_VALUES)
def test_hg_mean_cosine_is_g(g):
    # the asymmetry parameter is the mean scattering cosine (text after eq. 5)
    val, _ = scipy.integrate.quad(lambda mu: mu * oracle.hg(g, mu), -1.0, 1.0, limit=400,
                                  epsabs=1e-13, epsrel=1e-12)
    assert abs(2.0 * math.pi * val - g) < 1e-9


@pytest.mark.parametrize("g", G_VALUES)
def test_hg_forward_backward_closed_forms(g):
    assert oracle.hg(g, 1.0) == pytest.approx((1 + g) / (4 * math.pi * (1 - g) ** 2), rel=1e-12)
    assert oracle.hg(g, -1.0) == pytest.approx((1 - g) / (4 * math.pi * (1 + g) ** 2), rel=1e-12)


def test_hg_isotropic_special_case():
    # eq. (7): g = 0 is the isotropic phase 1/(4 pi)
    for mu in np.linspace(-1, 1, 11):
        assert oracle.hg(0.0, mu) == pytest.approx(1.0 / (4.0 * math.pi), rel=1e-15)


def test_hg_golden_table():
    # independently computed values of eq. (5) at mu = +1, -1, 0
    rows = np.loadtxt(oracle_golden("hg_values.txt"))
    for g, fwd, bwd, side in rows:
        assert oracle.hg(g, 1.0) == pytest.approx(fwd, rel=1e-5)
        assert oracle.hg(g, -1.0) == pytest.approx(bwd, rel=1e-5)
        assert oracle.hg(g, 0.0) == pytest.approx(side, rel=1e-5)


def oracle_golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


# --------------------------------------------------------------------------
# Density pyramid, Sec. III.B.1 (box filter down to 1^3)

def test_pyramid_level_count_and_box_mean():
    rho = medium.fbm_cloud(16, seed=3)
    M = oracle.Medium(rho)
    assert M.levels == 5                       # 16, 8, 4, 2, 1
    ref = rho.astype(np.float64)
    for m in range(1, M.levels):
        n = ref.shape[0] // 2
        ref = ref.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))
        np.testing.assert_allclose(M.level(m), ref, rtol=1e-13, atol=0)


def test_pyramid_conserves_mass():
    rho = medium.fbm_cloud(32, seed=5)
    M = oracle.Medium(rho)
    mass = [M.level(m).sum() * (2.0 ** m / 32) ** 3 for m in range(M.levels)]
    np.testing.assert_allclose(mass, mass[0], rtol=1e-12)


def test_pyramid_keeps_constant_grid_constant():
    M = oracle.Medium(medium.constant(8, 0.37))
    for m in range(M.levels):
        np.testing.assert_allclose(M.level(m), np.float32(0.37), rtol=1e-15)


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.Medium(np.zeros((12, 12, 12), np.float32))


# --------------------------------------------------------------------------
# Light frame and graded transmittance fields, eq. (1) and eq. (15)

def test_light_frame_dominant_axis_and_ties():
    M = oracle.Medium(medium.constant(4, 1.0))
    M.set_light((0.3, 0.9, 0.3))
    fr = M.light_frame()
    assert (fr["a"], fr["b"], fr["c"], fr["sigma"]) == (1, 0, 2, 1)
    assert fr["sb"] == pytest.approx(1.0 / 3.0, rel=1e-7)
    M.set_light((1.0, -1.0, 0.5))               # tie |x| = |y| -> lowest index
    fr = M.light_frame()
    assert (fr["a"], fr["b"], fr["c"], fr["sigma"]) == (0, 1, 2, 1)
    M.set_light((0.2, 0.1, -3.0))
    fr = M.light_frame()
    assert (fr["a"], fr["b"], fr["c"], fr["sigma"]) == (2, 0, 1, -1)
    with pytest.raises(ValueError):
        M.set_light((0.0, 0.0, 0.0))


@pytest.mark.parametrize("light", [(0.3, 0.9, 0.3), (-0.7, 0.2, 0.4), (0.1, -0.3, -0.95)])
def test_homogeneous_slab_path_density(light):
    # rho == c: inside the box every sample equals c * ds * (J + 1/2)
    c, n = float(np.float32(0.6)), 16          # the grid holds float32 values
    M = oracle.Medium(medium.constant(n, c))
    M.set_light(light)
    fr = M.light_frame()
    la = abs(fr["l"][fr["a"]])
    D, (ulo, uhi, vlo, vhi) = M.path_density(0)
    ds = (1.0 / n) / la
    for J in range(n):
        for V in range(vlo, vhi + 1):
            for U in range(ulo, uhi + 1):
                # the ray stays inside laterally for all slices up to J
                ok = all(-0.5 <= U - Jp * fr["sb"] <= n - 0.5 and -0.5 <= V - Jp * fr["sc"] <= n - 0.5
                         for Jp in range(J + 1))
                if ok:
                    assert D[J, V - vlo, U - ulo] == pytest.approx(c * ds * (J + 0.5), rel=1e-13)


@pytest.mark.parametrize("light", [(0.3, 0.9, 0.3), (0.2, -0.1, 0.8)])
def test_homogeneous_slab_transmittance_closed_form(light):
    # eq. (15) for a homogeneous medium: T = exp(-sigma_t c d), d the distance
    # from x to the light-facing face along l (rays that leave through that face)
    c, n, sigma_t = 0.5, 32, 8.0                # 0.5 is exact in float32
    M = oracle.Medium(medium.constant(n, c))
    M.set_light(light)
    fr = M.light_frame()
    l = fr["l"]
    rng = np.random.default_rng(0)
    checked = 0
    for x in rng.random((400, 3)) * 0.8 + 0.1:
        face = 1.0 if l[fr["a"]] > 0 else 0.0
        t = (face - x[fr["a"]]) / l[fr["a"]]
        exitp = (x + t * l)[[fr["b"], fr["c"]]]     # lateral exit coordinates
        if np.all((exitp >= 1.0 / n) & (exitp <= 1 - 1.0 / n)):
            d = t
            assert M.sample_D(0, x) == pytest.approx(c * d, rel=1e-12)
            f = M.features(sigma_t, 0.5, 1.0, x[None].astype(np.float32),
                           np.array([[0, 0, -1]], np.float32))
            # tp uses the float32-rounded point; compare with its own distance
            xf = x.astype(np.float32).astype(np.float64)
            tf = (face - xf[fr["a"]]) / l[fr["a"]]
            assert f["tp"][0] == pytest.approx(math.exp(-sigma_t * c * tf), rel=1e-12)
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("light,axis", [((0, 1, 0), 1), ((0, -1, 0), 1), ((1, 0, 0), 0),
                                        ((0, 0, -1), 2)])
def test_axis_aligned_light_reduces_to_cumsum(light, axis):
    # with zero shear each ray is one voxel column: D = ds (cumsum - own/2)
    rho = medium.fbm_cloud(16, seed=2)
    M = oracle.Medium(rho)
    M.set_light(light)
    sign = np.sign(sum(light))
    for m in range(M.levels):
        lev = M.level(m)
        nm = lev.shape[0]
        D, (ulo, uhi, vlo, vhi) = M.path_density(m)
        assert (ulo, uhi, vlo, vhi) == (-1, nm, -1, nm)
        # move the sweep axis first ([z][y][x] -> numpy axis 2 - axis), light side first
        col = np.moveaxis(lev, 2 - axis, 0)
        if sign > 0:
            col = col[::-1]
        ref = (np.cumsum(col, axis=0) - 0.5 * col) / nm
        # remaining numpy axes are (c, b) = ascending lateral axes reversed
        got = D[:, 1:nm + 1, 1:nm + 1]
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
        assert np.all(D[:, 0, :] == 0) and np.all(D[:, :, 0] == 0)


def _analytic_rho(x, y, z):
    return 0.55 + 0.25 * np.sin(2.1 * x + 0.7) * np.cos(1.7 * y - 0.3) + 0.15 * np.sin(2.9 * z + 1.1)


def _grid_of(fn, n):
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return fn(x, y, z).astype(np.float32)


def test_path_density_converges_to_ray_integral():
    # brute force: the continuous optical depth of a smooth field along the
    # ray to the light-facing face, by adaptive quadrature; the discrete
    # sheared trapezoid must approach it at second order
    light = np.array([0.3, 0.9, 0.3])
    l = light / np.linalg.norm(light)
    rng = np.random.default_rng(17)
    pts = np.column_stack([rng.uniform(0.25, 0.45, 16), rng.uniform(0.05, 0.6, 16),
                           rng.uniform(0.25, 0.45, 16)])
    ref = []
    for x in pts:
        t1 = (1.0 - x[1]) / l[1]
        f = lambda t: _analytic_rho(*(x + t * l))
        ref.append(scipy.integrate.quad(f, 0.0, t1, epsabs=1e-13, epsrel=1e-13)[0])
    ns = (8, 16, 32, 64)
    errs = []
    for n in ns:
        M = oracle.Medium(_grid_of(_analytic_rho, n))
        M.set_light(light)
        e = np.array([M.sample_D(0, x) - r for x, r in zip(pts, ref)])
        errs.append(np.sqrt(np.mean(e * e)))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert errs[-1] < 1e-4, errs
    assert slope > 1.8, (errs, slope)


# Sheared lights at the edges of the box (eq. 1 integrated along rays parallel
# to l).  Each pin is geometry worked out on the unit cube, by brute force over
# rays, slices or points: none retypes the oracle's ray-range or lookup formulas.
SHEARED_LIGHTS = [(0.3, 0.9, 0.3), (-0.7, 0.2, 0.4), (0.1, -0.3, -0.95), (0.5, 0.5, -0.45),
                  (0.9, -0.85, 0.2), (-0.35, -0.6, 0.58)]


def _frame_of(light):
    # the library and the oracle receive the direction as float32
    l = np.asarray(light, np.float32).astype(np.float64)
    l = l / np.linalg.norm(l)
    a = int(np.argmax(np.abs(l)))
    b, c = [i for i in range(3) if i != a]
    return l, a, b, c


@pytest.mark.parametrize("light", SHEARED_LIGHTS)
def test_stored_rays_cover_every_ray_that_meets_the_box(light):
    # With a density that is positive everywhere, a sheared ray has a non-zero
    # sample exactly when it crosses the box's lateral extent at some slice.
    # Every such ray must be stored strictly inside the stored range (its
    # first and last rays are margins that miss the box), the margin rays must
    # be zero at every slice, and every stored ray that meets the box must
    # carry a positive path density at the far end of the box.
    rho = (medium.fbm_cloud(16, seed=3) * 0.5 + 0.25).astype(np.float32)
    M = oracle.Medium(rho)
    M.set_light(light)
    fr = M.light_frame()
    for m in range(M.levels):
        nm = 16 >> m
        D, (ulo, uhi, vlo, vhi) = M.path_density(m)
        # brute force over a wide window of integer rays and every slice:
        # lateral index coordinate of ray U at slice J is U - J s
        def meets(r, s):
            return any(-0.5 <= r - J * s <= nm - 0.5 for J in range(nm))
        us = [U for U in range(-4 * nm - 4, 5 * nm + 5) if meets(U, fr["sb"])]
        vs = [V for V in range(-4 * nm - 4, 5 * nm + 5) if meets(V, fr["sc"])]
        assert ulo < min(us) and max(us) < uhi, (m, ulo, uhi, us[0], us[-1])
        assert vlo < min(vs) and max(vs) < vhi, (m, vlo, vhi, vs[0], vs[-1])
        assert np.all(D[:, :, 0] == 0) and np.all(D[:, :, -1] == 0)
        assert np.all(D[:, 0, :] == 0) and np.all(D[:, -1, :] == 0)
        for V in range(vlo, vhi + 1):
            for U in range(ulo, uhi + 1):
                hit = any(-0.5 <= U - J * fr["sb"] <= nm - 0.5 and -0.5 <= V - J * fr["sc"] <= nm - 0.5
                          for J in range(nm))
                assert (D[-1, V - vlo, U - ulo] > 0) == hit, (m, U, V)


def _slice_planes(nm, sigma):
    """World coordinates along the dominant axis of the voxel-centre planes of
    a level, ordered from the light side."""
    c = (np.arange(nm) + 0.5) / nm
    return c[::-1] if sigma > 0 else c


@pytest.mark.parametrize("light", SHEARED_LIGHTS)
def test_path_density_is_zero_beside_the_box(light):
    # A point whose line towards the light passes the box more than one voxel
    # away (laterally, at every slice plane between the light-facing face and
    # two slices beyond the point) sees no medium: the interpolated path
    # density is exactly zero, at every level.
    n, c = 16, 0.5
    M = oracle.Medium(medium.constant(n, c))
    M.set_light(light)
    l, a, b, cc = _frame_of(light)
    fr = M.light_frame()
    rng = np.random.default_rng(5)
    for m in range(M.levels):
        nm = n >> m
        h = 1.0 / nm
        pts = rng.uniform(-0.5 - 3 * h, 1.5 + 3 * h, (1500, 3))
        pts[:, a] = rng.uniform(0.0, 1.0, 1500)
        planes = _slice_planes(nm, fr["sigma"])
        checked = 0
        for x in pts:
            # planes from the light side up to two slices beyond the point
            beyond = x[a] - 2 * h if fr["sigma"] > 0 else x[a] + 2 * h
            use = planes[planes >= beyond] if fr["sigma"] > 0 else planes[planes <= beyond]
            clear = True
            for pa in use:
                t = (pa - x[a]) / l[a]
                yb, yc = x[b] + t * l[b], x[cc] + t * l[cc]
                if not (yb < -h or yb > 1 + h or yc < -h or yc > 1 + h):
                    clear = False
                    break
            if clear:
                assert M.sample_D(m, x) == 0.0, (m, x)
                checked += 1
        assert checked > 50, (m, checked)


@pytest.mark.parametrize("light", SHEARED_LIGHTS)
def test_path_density_beyond_the_faces_of_a_slab(light):
    # Homogeneous slab rho == c.  Beyond the light-facing face the lookup
    # clamps to the first slice, whose trapezoid value is half a step:
    # c h_m / (2 |l_a|).  Beyond the far face it clamps to the last slice:
    # c h_m (n_m - 1/2) / |l_a|.  Both hold where the line through the point
    # stays at least one voxel inside the box laterally on the slices involved.
    n, c = 16, 0.5
    M = oracle.Medium(medium.constant(n, c))
    M.set_light(light)
    l, a, b, cc = _frame_of(light)
    fr = M.light_frame()
    la = abs(l[a])
    rng = np.random.default_rng(9)
    far_total = 0
    for m in range(M.levels):
        nm = n >> m
        h = 1.0 / nm
        planes = _slice_planes(nm, fr["sigma"])
        near = far = 0
        for _ in range(600):
            x = rng.uniform(0.0, 1.0, 3)
            side = rng.integers(2)                    # 0: light side, 1: far side
            out = rng.uniform(0.01, 0.6)
            light_face = 1.0 if fr["sigma"] > 0 else 0.0
            far_face = 1.0 - light_face
            toward = 1.0 if fr["sigma"] > 0 else -1.0
            x[a] = light_face + toward * out if side == 0 else far_face - toward * out
            use = planes[:1] if side == 0 else planes
            inside = True
            for pa in use:
                t = (pa - x[a]) / l[a]
                yb, yc = x[b] + t * l[b], x[cc] + t * l[cc]
                if not (h <= yb <= 1 - h and h <= yc <= 1 - h):
                    inside = False
                    break
            if not inside:
                continue
            if side == 0:
                assert M.sample_D(m, x) == pytest.approx(c * h / (2 * la), rel=1e-12)
                near += 1
            else:
                assert M.sample_D(m, x) == pytest.approx(c * h * (nm - 0.5) / la, rel=1e-12)
                far += 1
        if nm >= 4:                                   # coarser levels have no interior
            assert near > 20, (m, near)
        far_total += far
    if max(abs(fr["sb"]), abs(fr["sc"])) < 0.8:       # steeper shears leave no full column
        assert far_total > 20, far_total


# --------------------------------------------------------------------------
# Template sampling, Sec. III.B.2-4 (light-aligned 12 x 5x5x9 lattice)

def _site_offsets(l):
    """Lattice offsets o_t in site order for light l (dominant axis a)."""
    a = int(np.argmax(np.abs(l)))
    b, c = [i for i in range(3) if i != a]
    out = []
    for q in range(-4, 5):
        for j in range(-2, 3):
            for i in range(-2, 3):
                o = q * l / abs(l[a])
                o = o.copy()
                o[b] += i
                o[c] += j
                out.append(o)
    return np.array(out)


def test_site_density_matches_scipy_trilinear():
    # site densities against scipy's linear map_coordinates with edge clamping
    rho = medium.fbm_cloud(32, seed=4)
    M = oracle.Medium(rho)
    l = np.array([0.35, -0.8, 0.45])
    l /= np.linalg.norm(l)
    M.set_light(l.astype(np.float32))
    lf = M.light_frame()["l"]
    pts, dirs = camera.random_points(6, seed=11, lo=0.2, hi=0.8)
    f = M.features(8.0, 0.7, 0.6, pts, dirs)
    offs = _site_offsets(lf)
    for p in range(len(pts)):
        for k in range(12):
            m = min(k, M.levels - 1)
            lev = M.level(m)
            nm = lev.shape[0]
            s = pts[p].astype(np.float64)[None, :] + (2.0 ** k / 32) * offs
            g = s * nm - 0.5
            vals = scipy.ndimage.map_coordinates(lev, [g[:, 2], g[:, 1], g[:, 0]], order=1,
                                                 mode="nearest", prefilter=False)
            inside = np.all((s >= 0) & (s <= 1), axis=1)
            np.testing.assert_allclose(f["rho"][p, k], np.where(inside, vals, 0.0),
                                       rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("light", [(0, 1, 0), (0, 0, -1)])
def test_axis_aligned_sites_hit_raw_voxels(light):
    # p at a level-m voxel centre, zero shear: the sites of layer m sit on
    # level-m voxel centres, so every feature is a raw array entry
    rho = medium.fbm_cloud(16, seed=9)
    M = oracle.Medium(rho)
    M.set_light(light)
    sigma_t, lam = 8.0, 0.6
    a = int(np.argmax(np.abs(light)))
    sgn = np.sign(sum(light))
    b, c = [i for i in range(3) if i != a]
    for m in range(3):
        nm = 16 >> m
        I = np.array([nm // 2 - 1, nm // 2, nm // 2 - 1 + (nm > 2)])
        p = ((I + 0.5) / nm).astype(np.float32)
        f = M.features(sigma_t, 0.5, lam, p[None], np.array([[1, 0, 0]], np.float32))
        D, (ulo, uhi, vlo, vhi) = M.path_density(m)
        lev = M.level(m)
        t = 0
        for q in range(-4, 5):
            for j in range(-2, 3):
                for i in range(-2, 3):
                    v = I.copy()
                    v[a] += int(q * sgn)
                    v[b] += i
                    v[c] += j
                    if np.all((v >= 0) & (v < nm)):
                        r = lev[v[2], v[1], v[0]]
                        J = nm - 1 - v[a] if sgn > 0 else v[a]
                        T = math.exp(-lam ** (m + 1) * sigma_t * D[J, v[c] - vlo, v[b] - ulo])
                        assert f["rho"][0, m, t] == pytest.approx(r, rel=1e-13, abs=1e-15)
                        assert f["tbar"][0, m, t] == pytest.approx(T, rel=1e-12)
                    t += 1


def test_phase_features_closed_forms():
    # sites on the light axis have d = +-l; lateral sites d = +-e_b, +-e_c
    M = oracle.Medium(medium.constant(8, 0.3))
    l = np.array([0.2, 0.3, 0.9])
    l /= np.linalg.norm(l)
    M.set_light(l.astype(np.float32))
    lf = M.light_frame()["l"]
    g = 0.8
    w = np.array([0.6, -0.48, 0.64], np.float32)
    wf = w.astype(np.float64) / np.linalg.norm(w.astype(np.float64))
    f = M.features(8.0, g, 0.6, np.array([[0.5, 0.5, 0.5]], np.float32), w[None])
    phi = f["phi"][0]
    hg = lambda mu: (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * mu) ** 1.5)
    site = lambda q, j, i: ((q + 4) * 5 + (j + 2)) * 5 + (i + 2)
    wl = float(wf @ lf)
    # toward the light: d = l, so P = HG(w.l) HG(1); away: d = -l, P = HG(-w.l) HG(-1)
    assert math.expm1(phi[site(2, 0, 0)]) == pytest.approx(hg(wl) * (1 + g) / (4 * math.pi * (1 - g) ** 2), rel=1e-12)
    assert math.expm1(phi[site(-3, 0, 0)]) == pytest.approx(hg(-wl) * (1 - g) / (4 * math.pi * (1 + g) ** 2), rel=1e-12)
    # centre site: the single-scatter phase HG(w.l)
    assert math.expm1(phi[site(0, 0, 0)]) == pytest.approx(hg(wl), rel=1e-12)
    # lateral site along +b (b = x for a = z): d = e_x
    assert math.expm1(phi[site(0, 0, 1)]) == pytest.approx(hg(wf[0]) * hg(lf[0]), rel=1e-12)
    assert math.expm1(phi[site(0, -1, 0)]) == pytest.approx(hg(-wf[1]) * hg(-lf[1]), rel=1e-12)
    # squeeze vector: alpha and g entries
    assert f["stats"][0, 0, 6] == g
    assert f["stats"][0, 0, 7] == pytest.approx(math.acos(wl), rel=1e-12)


# --------------------------------------------------------------------------
# Multi-lobe HG phase, Sec. III.A eq. (6): weights summing to one

MHG_PHASES = ([(0.7, 0.8), (0.3, -0.4)], [(0.5, 0.95), (0.3, 0.2), (0.2, -0.7)], [(1.0, 0.6)])


@pytest.mark.parametrize("phase", MHG_PHASES)
def test_mhg_normalises_and_mean_cosine_is_weighted(phase):
    val, _ = scipy.integrate.quad(lambda mu: oracle.mhg(phase, mu), -1.0, 1.0, limit=400,
                                  epsabs=1e-13, epsrel=1e-13)
    assert 2 * math.pi * val == pytest.approx(1.0, abs=1e-9)
    mc, _ = scipy.integrate.quad(lambda mu: mu * oracle.mhg(phase, mu), -1.0, 1.0, limit=400,
                                 epsabs=1e-13, epsrel=1e-13)
    assert 2 * math.pi * mc == pytest.approx(sum(w * g for w, g in phase), abs=1e-9)


def test_mhg_reduces_to_hg():
    for mu in (-1.0, -0.3, 0.0, 0.4, 1.0):
        # one lobe of weight 1 is plain HG, bit for bit; equal lobes add up to it
        assert oracle.mhg([(1.0, 0.7)], mu) == oracle.hg(0.7, mu)
        assert oracle.mhg([(0.25, 0.7), (0.75, 0.7)], mu) == pytest.approx(oracle.hg(0.7, mu), rel=1e-15)
        # forward and backward values of a two-lobe mixture, each lobe in closed form
        fw = 0.6 * (1 + 0.9) / (4 * math.pi * (1 - 0.9) ** 2) + 0.4 * (1 - 0.5) / (4 * math.pi * (1 + 0.5) ** 2)
        assert oracle.mhg([(0.6, 0.9), (0.4, -0.5)], 1.0) == pytest.approx(fw, rel=1e-13)


def test_mhg_phase_features_and_single_scatter():
    """With a two-lobe phase f, the centre site carries f(w.l), a site toward
    the light f(w.l) f(1), the squeeze vector the mean cosine, and the
    single-scatter term f(w.l) T(p); one lobe of weight 1 gives the HG
    features bit for bit."""
    phase = [(0.7, 0.8), (0.3, -0.4)]
    f = lambda mu: sum(w * (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * mu) ** 1.5) for w, g in phase)
    M = oracle.Medium(medium.fbm_cloud(16, seed=2))
    l = np.array([0.2, 0.3, 0.9])
    l /= np.linalg.norm(l)
    M.set_light(l.astype(np.float32))
    lf = M.light_frame()["l"]
    w = np.array([0.6, -0.48, 0.64], np.float32)
    wf = w.astype(np.float64) / np.linalg.norm(w.astype(np.float64))
    x = np.array([[0.45, 0.5, 0.55]], np.float32)
    r = M.features(8.0, phase, 0.6, x, w[None])
    wl = float(wf @ lf)
    site = lambda q, j, i: ((q + 4) * 5 + (j + 2)) * 5 + (i + 2)
    assert math.expm1(r["phi"][0, site(0, 0, 0)]) == pytest.approx(f(wl), rel=1e-12)
    assert math.expm1(r["phi"][0, site(2, 0, 0)]) == pytest.approx(f(wl) * f(1.0), rel=1e-12)
    assert r["stats"][0, 3, 6] == pytest.approx(0.7 * 0.8 - 0.3 * 0.4, rel=1e-15)
    assert r["f0"][0] == pytest.approx(f(wl) * r["tp"][0], rel=1e-12)
    one = M.features(8.0, [(1.0, 0.8)], 0.6, x, w[None])
    plain = M.features(8.0, 0.8, 0.6, x, w[None])
    for k in one:
        np.testing.assert_array_equal(one[k], plain[k])


# --------------------------------------------------------------------------
# Volume phase, Sec. III.A eq. (9): the phase averaged over the cone under
# which a template site is seen from the point


def _cone_mean_brute(phase, mu0, beta):
    """Mean of a phase over a cone of half-angle beta around d, w.d = mu0, by
    two-dimensional adaptive quadrature over the cone's polar and azimuthal
    angles (the definition, integrated numerically)."""
    lobes = [(1.0, phase)] if np.ndim(phase) == 0 else phase
    f = lambda mu: sum(w * (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * mu) ** 1.5) for w, g in lobes)
    s0 = math.sqrt(1 - mu0 * mu0)
    val, _ = scipy.integrate.dblquad(
        lambda psi, th: f(mu0 * math.cos(th) + s0 * math.sin(th) * math.cos(psi)) * math.sin(th),
        0.0, beta, 0.0, 2 * math.pi, epsabs=1e-14, epsrel=1e-12)
    return val / (2 * math.pi * (1 - math.cos(beta)))


@pytest.mark.parametrize("g,mu0,beta", [(0.9, 0.7, 0.3), (0.95, 0.99, 0.07), (0.95, -0.4, 0.5),
                                        (-0.6, 0.2, 0.25), (0.5, 1.0, 0.1), (0.8, -1.0, 0.2)])
def test_volume_phase_matches_brute_force_cone_quadrature(g, mu0, beta):
    assert oracle.hg_cone(g, mu0, beta) == pytest.approx(_cone_mean_brute(g, mu0, beta), rel=1e-10)


def test_volume_phase_limits():
    for g in (0.0, 0.6, -0.85):
        # the whole sphere: the normalisation 1/(4 pi) (the 64-point rule over the
        # whole of cos theta leaves ~2e-11 at g = -0.85; the lattice's cones are
        # at most 30 degrees wide); g = 0: isotropic for any cone
        assert oracle.hg_cone(g, 0.3, math.pi) == pytest.approx(1 / (4 * math.pi), rel=1e-9)
    assert oracle.hg_cone(0.0, -0.7, 0.4) == pytest.approx(1 / (4 * math.pi), rel=1e-14)
    # a vanishing cone: the point phase
    for g, mu0 in ((0.9, 0.5), (0.95, 0.999), (-0.5, -0.8)):
        assert oracle.hg_cone(g, mu0, 1e-5) == pytest.approx(oracle.hg(g, mu0), rel=1e-8)


def test_volume_phase_features():
    """With the volume phase a site's feature is the product of the two cone
    means (site seen as a ball of half the lattice spacing: half-angle
    asin(1 / (2 |o|))); the centre site keeps the point phase."""
    phase = [(0.7, 0.8), (0.3, -0.4)]
    M = oracle.Medium(medium.constant(8, 0.3))
    l = np.array([0.2, 0.3, 0.9])
    l /= np.linalg.norm(l)
    M.set_light(l.astype(np.float32))
    fr = M.light_frame()
    lf = fr["l"]
    w = np.array([0.6, -0.48, 0.64], np.float32)
    wf = w.astype(np.float64) / np.linalg.norm(w.astype(np.float64))
    x = np.array([[0.45, 0.5, 0.55]], np.float32)
    vol = M.features(8.0, phase, 0.6, x, w[None], volume=True)
    pnt = M.features(8.0, phase, 0.6, x, w[None])
    site = lambda q, j, i: ((q + 4) * 5 + (j + 2)) * 5 + (i + 2)
    assert vol["phi"][0, site(0, 0, 0)] == pnt["phi"][0, site(0, 0, 0)]
    # a lateral site: o = e_b (b = x for a = z), |o| = 1
    d = np.array([1.0, 0.0, 0.0])
    beta = math.asin(0.5)
    expect = _cone_mean_brute(phase, float(wf @ d), beta) * _cone_mean_brute(phase, float(d @ lf), beta)
    assert math.expm1(vol["phi"][0, site(0, 0, 1)]) == pytest.approx(expect, rel=1e-9)
    # a site toward the light, q = 2: o = 2 l / |l_a|, |o| = 2 / |l_a|
    on = 2 / abs(lf[2])
    beta = math.asin(0.5 / on)
    expect = _cone_mean_brute(phase, float(wf @ lf), beta) * _cone_mean_brute(phase, 1.0, beta)
    assert math.expm1(vol["phi"][0, site(2, 0, 0)]) == pytest.approx(expect, rel=1e-9)
    # everything but the phase features is unchanged
    for k in ("tbar", "rho", "tp", "f0"):
        np.testing.assert_array_equal(vol[k], pnt[k])


def test_isotropic_phase_features():
    M = oracle.Medium(medium.constant(8, 0.3))
    M.set_light((0.3, 0.9, 0.3))
    pts, dirs = camera.random_points(4, seed=1)
    f = M.features(8.0, 0.0, 0.6, pts, dirs)
    iso = 1.0 / (4 * math.pi)
    expect = np.full(225, math.log1p(iso * iso))
    expect[112] = math.log1p(iso)
    for p in range(4):
        np.testing.assert_allclose(f["phi"][p], expect, rtol=1e-14)


def test_squeeze_statistics_are_layer_means_and_maxima():
    M = oracle.Medium(medium.fbm_cloud(16, seed=8))
    M.set_light((0.5, 0.2, -0.8))
    pts, dirs = camera.random_points(3, seed=3, lo=0.3, hi=0.7)
    f = M.features(8.0, 0.6, 0.6, pts, dirs)
    st = f["stats"]
    np.testing.assert_allclose(st[:, :, 0], f["rho"].mean(axis=2), rtol=1e-13)
    np.testing.assert_allclose(st[:, :, 2], f["tbar"].mean(axis=2), rtol=1e-13)
    np.testing.assert_allclose(st[:, :, 3], f["rho"].max(axis=2), rtol=0)
    np.testing.assert_allclose(st[:, :, 5], f["tbar"].max(axis=2), rtol=0)
    np.testing.assert_allclose(st[:, :, 1], f["phi"].mean(axis=1)[:, None].repeat(12, 1), rtol=1e-13)
    np.testing.assert_allclose(st[:, :, 4], f["phi"].max(axis=1)[:, None].repeat(12, 1), rtol=0)


# --------------------------------------------------------------------------
# 3D-CNN (Fig. 3), squeeze-excitation (eq. 24-26) and backbone (Fig. 6)

def _torch_cnn_se(grp, lattice):
    x = torch.tensor(lattice, dtype=torch.float64).reshape(1, 1, 9, 5, 5)
    t = lambda k: torch.tensor(np.asarray(grp[k], np.float64))
    y = torch.relu(torch.nn.functional.conv3d(x, t("w1"), t("b1")))
    H = torch.relu(torch.nn.functional.conv3d(y, t("w2"), t("b2")))[0, :, :, 0, 0]   # [16][5]
    z = H.mean(dim=1)
    e = torch.sigmoid(t("s2") @ torch.relu(t("s1") @ z + t("c1")) + t("c2"))
    return (e[:, None] * H).reshape(-1).numpy()


def test_cnn_se_matches_torch_conv3d():
    params = weights.he_init(32, 3, seed=4, bias_scale=0.3)
    rng = np.random.default_rng(0)
    for group in ("diffuse", "highlight"):
        for _ in range(8):
            lat = rng.random(225)
            got = oracle.cnn_se(params, group, lat)
            ref = _torch_cnn_se(params["groups"][group], lat)
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_se_with_zero_excitation_halves_features():
    params = weights.he_init(32, 3, seed=4, bias_scale=0.3)
    grp = params["groups"]["diffuse"]
    for k in ("s1", "c1", "s2", "c2"):
        grp[k] = np.zeros_like(grp[k])
    lat = np.random.default_rng(1).random(225)
    x = torch.tensor(lat).reshape(1, 1, 9, 5, 5)
    t = lambda k: torch.tensor(np.asarray(grp[k], np.float64))
    H = torch.relu(torch.nn.functional.conv3d(torch.relu(torch.nn.functional.conv3d(
        x, t("w1"), t("b1"))), t("w2"), t("b2")))[0, :, :, 0, 0]
    np.testing.assert_allclose(oracle.cnn_se(params, "diffuse", lat), 0.5 * H.reshape(-1).numpy(),
                               rtol=1e-12, atol=1e-14)


def test_descriptor_layout_and_mlp_match_numpy():
    params = weights.he_init(24, 4, seed=6, bias_scale=0.2)
    rng = np.random.default_rng(2)
    tbar = rng.random((12, 225))
    stats = rng.random((12, 8))
    desc = oracle.descriptor(params, tbar, stats, 0.93)
    assert desc.shape == (1057,) and desc[-1] == 0.93
    for k in range(12):
        grp = params["groups"]["diffuse" if k < 8 else "highlight"]
        np.testing.assert_allclose(desc[k * 88:k * 88 + 80], _torch_cnn_se(grp, tbar[k]),
                                   rtol=1e-12, atol=1e-14)
        np.testing.assert_array_equal(desc[k * 88 + 80:k * 88 + 88], stats[k])
    h = desc
    for i, (A, b) in enumerate(zip(params["A"], params["beta"])):
        h = A.astype(np.float64) @ h + b.astype(np.float64)
        if i < len(params["A"]) - 1:
            h = np.maximum(h, 0.0)
    assert oracle.mlp(params, desc) == pytest.approx(h[0], rel=1e-12)


# --------------------------------------------------------------------------
# Whole query: eq. (19) single-scatter term, eq. (21) decode

def _small_setup(n=16, seed=0):
    rho = medium.fbm_cloud(n, seed=seed)
    M = oracle.Medium(rho)
    M.set_light((0.3, 0.9, 0.3))
    pts, dirs = camera.random_points(24, seed=21, lo=0.05, hi=0.95)
    return M, pts, dirs


def test_zero_weights_give_single_scatter_closed_form():
    M, pts, dirs = _small_setup()
    params = weights.zeros_like(weights.he_init(16, 3))
    out = M.query(params, pts, dirs, sigma_t=8.0, albedo=0.99, g=0.85, radiance=2.5)
    l = M.light_frame()["l"]
    for p in range(len(pts)):
        w = dirs[p].astype(np.float64)
        w /= np.linalg.norm(w)
        mu = float(w @ l)
        hg = (1 - 0.85 ** 2) / (4 * math.pi * (1 + 0.85 ** 2 - 2 * 0.85 * mu) ** 1.5)
        T = math.exp(-8.0 * M.sample_D(0, pts[p].astype(np.float64)))
        assert out["y"][p] == 0.0 and out["F"][p] == 0.0
        assert out["L"][p] == pytest.approx(2.5 * hg * T, rel=1e-12)


@pytest.mark.parametrize("entry", [0, 37, 79, 80, 85, 87, 88 * 5 + 12, 88 * 9 + 83, 88 * 11 + 87, 1056])
def test_selector_weights_return_one_descriptor_entry(entry):
    M, pts, dirs = _small_setup()
    params = weights.he_init(8, 4, seed=3)
    for A in params["A"]:
        A[:] = 0.0
    params["A"][0][0, entry] = 1.0
    params["A"][1][0, 0] = 1.0
    params["A"][2][0, 0] = 1.0
    params["A"][3][0, 0] = 1.0
    out = M.query(params, pts, dirs, sigma_t=8.0, albedo=0.99, g=0.85, want_desc=True)
    np.testing.assert_array_equal(out["y"], out["desc"][:, entry])
    np.testing.assert_allclose(out["F"], 0.99 ** 4 * np.expm1(out["y"]), rtol=1e-15)


def test_radiance_is_linear_in_light_intensity():
    M, pts, dirs = _small_setup()
    params = weights.he_init(16, 3, seed=2)
    a = M.query(params, pts, dirs, 8.0, 0.99, 0.85, radiance=1.0)["L"]
    b = M.query(params, pts, dirs, 8.0, 0.99, 0.85, radiance=4.0)["L"]
    np.testing.assert_array_equal(4.0 * a, b)


def test_mirroring_the_dominant_axis_is_invariant():
    # flip the grid along y, mirror the light and the points: same radiance
    rho = medium.fbm_cloud(16, seed=12)
    params = weights.he_init(16, 3, seed=2, bias_scale=0.1)
    rng = np.random.default_rng(5)
    pts = (np.floor(rng.random((20, 3)) * 2 ** 20) / 2 ** 20).astype(np.float32)
    dirs = rng.standard_normal((20, 3)).astype(np.float32)
    A = oracle.Medium(rho)
    A.set_light((0.3, 0.9, 0.3))
    B = oracle.Medium(np.ascontiguousarray(rho[:, ::-1, :]))
    B.set_light((0.3, -0.9, 0.3))
    pm, dm = pts.copy(), dirs.copy()
    pm[:, 1] = 1.0 - pm[:, 1]
    dm[:, 1] = -dm[:, 1]
    a = A.query(params, pts, dirs, 8.0, 0.99, 0.85)
    b = B.query(params, pm, dm, 8.0, 0.99, 0.85)
    np.testing.assert_allclose(a["L"], b["L"], rtol=1e-12)
    np.testing.assert_allclose(a["y"], b["y"], rtol=1e-12)


def test_batch_order_invariance():
    M, pts, dirs = _small_setup()
    params = weights.he_init(16, 3, seed=2)
    full = M.query(params, pts, dirs, 8.0, 0.99, 0.85)["L"]
    perm = np.random.default_rng(3).permutation(len(pts))
    part = M.query(params, pts[perm], dirs[perm], 8.0, 0.99, 0.85)["L"]
    np.testing.assert_array_equal(full[perm], part)


# ---- the paper's templates (Sec. III.B.2, eq. 2-4) ----------------------------

def test_template_counts():
    # the per-layer counts as printed: 6, 8, ..., 48 (sum 194, where the text
    # says 182) and 32, 16, 16, 8 (sum 72)
    c = oracle.tpl_counts()
    assert c[:8] == [6, 8, 12, 16, 24, 32, 48, 48] and sum(c[:8]) == 194
    assert c[8:] == [32, 16, 16, 8] and sum(c[8:]) == 72
    assert oracle.TPL_SITES == 266


def test_template_points_lie_in_their_regions():
    # layer 0: the centre and 5 points on the unit sphere; layers 1-7: the shell
    # 1/2 <= |u| <= 1; cone layer h: axial t in [h/4, (h+1)/4], radius <= t
    u0 = oracle.tpl_unit(0)
    assert np.all(u0[0] == 0.0) and np.all(np.linalg.norm(u0[1:], axis=1) > 0)
    assert np.all(np.linalg.norm(u0, axis=1) <= 1.0 + 1e-15)
    for k in range(1, 8):
        r = np.linalg.norm(oracle.tpl_unit(k), axis=1)
        assert np.all((r >= 0.5 - 1e-15) & (r <= 1.0 + 1e-15)), k
        assert len(np.unique(np.round(oracle.tpl_unit(k), 12), axis=0)) == len(r)   # distinct points
    for h in range(4):
        u = oracle.tpl_unit(8 + h)
        assert np.all((u[:, 0] >= h / 4) & (u[:, 0] <= (h + 1) / 4))
        assert np.all(np.hypot(u[:, 1], u[:, 2]) <= u[:, 0] + 1e-15)


def test_template_uniformity_measure_matches_nearest_neighbours():
    # eq. (3): D(S_i) is the mean nearest-neighbour distance (scipy's k-d tree)
    from scipy.spatial import cKDTree
    for k in range(12):
        u = oracle.tpl_unit(k)
        d, _ = cKDTree(u).query(u, k=2)
        assert oracle.tpl_D(k) == pytest.approx(d[:, 1].mean(), rel=1e-13), k


def test_templates_are_more_even_than_random_sets():
    # "evenly distributed": each layer's D(S_i) exceeds the 95th percentile
    # of D over 200 seeded sets of as many points drawn uniformly in the same
    # region (ball, shell, or the layer's frustum of the cone)
    from scipy.spatial import cKDTree
    r = np.random.default_rng(3)
    for k in range(12):
        n = oracle.tpl_counts()[k]
        vals = []
        for _ in range(200):
            if k < 8:
                v = r.standard_normal((n, 3))
                v /= np.linalg.norm(v, axis=1, keepdims=True)
                lo = 0.0 if k == 0 else 0.125
                v *= np.cbrt(r.uniform(lo, 1.0, (n, 1)))
            else:
                lo, hi = (k - 8) / 4, (k - 7) / 4
                t = np.cbrt(lo ** 3 + r.random(n) * (hi ** 3 - lo ** 3))
                rad = np.sqrt(r.random(n)) * t
                a = r.uniform(0, 2 * np.pi, n)
                v = np.stack([t, rad * np.cos(a), rad * np.sin(a)], axis=1)
            vals.append(cKDTree(v).query(v, k=2)[0][:, 1].mean())
        assert oracle.tpl_D(k) > np.percentile(vals, 95), k


def test_template_radii_follow_eq4():
    # r_i = 2^(i-1) xi_i / (2^8 D(S_i)), xi_i = 1 - 0.08 min(i, 5): the
    # layer's nearest-neighbour spacing is 2^(i-1) xi_i voxels of a 256^3 grid
    for i in range(8):
        xi = 1.0 - 0.08 * min(i, 5)
        assert oracle.tpl_radius(i) * oracle.tpl_D(i) * 256 == pytest.approx(2.0 ** (i - 1) * xi, rel=1e-14)
    r = [oracle.tpl_radius(i) for i in range(8)]
    assert all(b > a for a, b in zip(r, r[1:]))


def test_light_extent_closed_forms():
    s3 = 1 / np.sqrt(3)
    assert oracle.tpl_light_extent([0, 1, 0], [0.5, 0.5, 0.5]) == pytest.approx(0.5, rel=1e-15)
    assert oracle.tpl_light_extent([s3, s3, s3], [0.5, 0.5, 0.5]) == pytest.approx(0.5 * np.sqrt(3), rel=1e-14)
    assert oracle.tpl_light_extent([0, 0, -1], [0.2, 0.3, 0.9]) == pytest.approx(0.9, rel=1e-15)
    assert oracle.tpl_light_extent([1, 0, 0], [0.5, 1.5, 0.5]) == 0.0            # misses the cube
    assert oracle.tpl_light_extent([1, 0, 0], [0.5, 0.5, 0.5]) == pytest.approx(0.5)
    assert oracle.tpl_light_extent([1, 0, 0], [-0.5, 0.5, 0.5]) == pytest.approx(1.5)   # enters, far exit
    assert oracle.tpl_light_extent([-1, 0, 0], [-0.5, 0.5, 0.5]) == 0.0          # the cube is behind


def _expected_tpl_levels(n, L):
    # level whose voxel matches the layer's spacing: round(log2(spacing * n)),
    # clamped to [0, L-1]
    out = []
    for i in range(8):
        x = 2.0 ** (i - 1) * (1 - 0.08 * min(i, 5)) / 256 * n
        out.append(int(min(max(np.floor(np.log2(x) + 0.5), 0), L - 1)))
    return out


@pytest.mark.parametrize("light", [(0.3, 0.9, 0.3), (0.2, -0.1, 0.8)])
def test_template_features_homogeneous_medium(light):
    # rho == c: the density is c at every template point inside the closed
    # cube and 0 outside; the graded transmittance at a point whose ray to
    # the light leaves through the light face is exp(-lam^(m+1) sigma_t c d),
    # d its distance to that face, which also pins each layer's level m
    c, n, sigma_t, lam = 0.5, 32, 8.0, 0.6
    M = oracle.Medium(medium.constant(n, c))
    M.set_light(light)
    fr = M.light_frame()
    l = fr["l"]
    r = np.random.default_rng(1)
    pts = r.uniform(0.3, 0.7, (6, 3)).astype(np.float32)
    dirs = np.tile(np.array([[0, 0, -1]], np.float32), (6, 1))
    f = M.tpl_features(sigma_t, 0.5, lam, pts, dirs)
    counts = oracle.tpl_counts()
    first = np.cumsum([0] + counts)
    a = fr["a"]
    face = 1.0 if l[a] > 0 else 0.0
    levels = _expected_tpl_levels(n, M.levels)
    checked = 0
    for p in range(len(pts)):
        x = pts[p].astype(np.float64)
        dl = oracle.tpl_light_extent(l, x)
        for k in range(12):
            u = oracle.tpl_unit(k)
            if k < 8:
                s = x + oracle.tpl_radius(k) * u
                m = levels[k]
            else:
                e1, e2 = _duff_onb(l)
                s = x + dl * (u[:, :1] * l + u[:, 1:2] * e1 + u[:, 2:3] * e2)
                sp = oracle.tpl_D(k) * dl * n
                m = int(min(max(np.floor(np.log2(sp) + 0.5), 0), M.levels - 1)) if sp > 0 else 0
            inside = np.all((s >= 0) & (s <= 1), axis=1)
            got_r = f["rho"][p, first[k]:first[k + 1]]
            np.testing.assert_array_equal(got_r[~inside], 0.0)
            np.testing.assert_allclose(got_r[inside], c, rtol=1e-14)
            got_t = f["tbar"][p, first[k]:first[k + 1]]
            for j in range(counts[k]):
                t = (face - s[j, a]) / l[a]
                ex = s[j] + t * l
                lat = ex[[fr["b"], fr["c"]]]
                # (rays whose interpolation neighbours, a voxel of the level
                # to either side, stay inside too: two voxels of margin)
                mg = 2.0 / (n >> m)
                if inside[j] and np.all((lat >= mg) & (lat <= 1 - mg)) and mg <= s[j, a] <= 1 - mg:
                    assert got_t[j] == pytest.approx(math.exp(-lam ** (m + 1) * sigma_t * c * t), rel=1e-10)
                    checked += 1
    assert checked > 300


def _duff_onb(l):
    s = 1.0 if l[2] >= 0 else -1.0
    a = -1.0 / (s + l[2])
    b = l[0] * l[1] * a
    return (np.array([1.0 + s * l[0] * l[0] * a, s * b, -s * l[0]]),
            np.array([b, s + l[1] * l[1] * a, -l[1]]))


def test_duff_frame_is_orthonormal():
    for l in np.random.default_rng(2).standard_normal((50, 3)):
        l = l / np.linalg.norm(l)
        e1, e2 = _duff_onb(l)
        B = np.stack([l, e1, e2])
        np.testing.assert_allclose(B @ B.T, np.eye(3), atol=1e-14)


def test_template_phase_and_statistics():
    # the centre point (layer 0, point 0) carries f(w.l); at g = 0 every other
    # point carries log1p(1/(4 pi)^2); the squeeze vector holds each layer's
    # means and maxima, g and alpha
    n = 16
    M = oracle.Medium(medium.fbm_cloud(n, seed=2))
    M.set_light((0.3, 0.9, 0.3))
    l = M.light_frame()["l"]
    pts, dirs = camera.random_points(20, seed=4, lo=0.1, hi=0.9)
    for g in (0.0, 0.7):
        f = M.tpl_features(8.0, g, 0.6, pts, dirs)
        w = dirs.astype(np.float64)
        w /= np.linalg.norm(w, axis=1, keepdims=True)
        wl = w @ l
        for p in range(len(pts)):
            assert f["phi"][p, 0] == pytest.approx(math.log1p(oracle.hg(g, wl[p])), rel=1e-14)
            if g == 0.0:
                np.testing.assert_allclose(f["phi"][p, 1:], math.log1p(1 / (4 * np.pi) ** 2), rtol=1e-14)
        first = np.cumsum([0] + oracle.tpl_counts())
        for k in range(12):
            sl = slice(first[k], first[k + 1])
            v = f["stats"][:, k]
            for col, key, red in ((0, "rho", np.mean), (1, "phi", np.mean), (2, "tbar", np.mean),
                                  (3, "rho", np.max), (4, "phi", np.max), (5, "tbar", np.max)):
                np.testing.assert_allclose(v[:, col], red(f[key][:, sl], axis=1), rtol=1e-13)
            np.testing.assert_allclose(v[:, 6], g)
            np.testing.assert_allclose(v[:, 7], np.arccos(np.clip(wl, -1, 1)), rtol=1e-13)


def test_template_descriptor_layout_and_probes():
    # per layer: tbar, rho, phi (template order), then the squeeze vector;
    # zeros up to the albedo entry 1056.  Zero weights give the single-scatter
    # term; a selector network returns any chosen entry.
    n = 16
    d = medium.fbm_cloud(n, seed=3)
    M = oracle.Medium(d)
    M.set_light((0.3, 0.9, 0.3))
    pts, dirs = camera.random_points(12, seed=5, lo=0.05, hi=0.95)
    params = weights.he_init(16, 3, seed=1)
    f = M.tpl_features(8.0, 0.85, 0.6, pts, dirs)
    q = M.tpl_query(params, pts, dirs, 8.0, 0.9, 0.85, 1.0, want_desc=True)
    first = np.cumsum([0] + oracle.tpl_counts())
    for p in range(len(pts)):
        exp = []
        for k in range(12):
            sl = slice(first[k], first[k + 1])
            exp += list(f["tbar"][p, sl]) + list(f["rho"][p, sl]) + list(f["phi"][p, sl]) + list(f["stats"][p, k])
        assert len(exp) == 894
        np.testing.assert_allclose(q["desc"][p, :894], exp, rtol=1e-15)
        np.testing.assert_array_equal(q["desc"][p, 894:1056], 0.0)
        assert q["desc"][p, 1056] == 0.9
    z = weights.zeros_like(params)
    qz = M.tpl_query(z, pts, dirs, 8.0, 0.9, 0.85, 2.0)
    np.testing.assert_allclose(qz["L"], 2.0 * f["f0"], rtol=1e-14)
    for entry in (0, 17, 893, 1056):
        s = weights.zeros_like(params)
        s["A"][0][0, entry] = 1.0
        s["A"][1][0, 0] = 1.0
        s["A"][2][0, 0] = 1.0
        y = M.tpl_query(s, pts, dirs, 8.0, 0.9, 0.85, 1.0)["y"]
        np.testing.assert_allclose(y, np.maximum(q["desc"][:, entry], 0.0), rtol=1e-14)


# ---- the paper's backbone modules (Sec. III.C.2, Fig. 6) ---------------------

def _tpl_setup():
    d = medium.fbm_cloud(16, seed=4)
    M = oracle.Medium(d)
    M.set_light((0.3, 0.9, 0.3))
    pts, dirs = camera.random_points(10, seed=6, lo=0.1, hi=0.9)
    f = M.tpl_features(8.0, 0.85, 0.6, pts, dirs)
    params = weights.he_init(16, 3, seed=1)
    feats = M.tpl_query(params, pts, dirs, 8.0, 0.9, 0.85, 1.0, want_desc=True)["desc"]
    return M, pts, dirs, f, feats[:, :894]


def _layer_slice(k, tau):
    counts = oracle.tpl_counts()
    base = sum(3 * c + 8 for c in counts[:k])
    return slice(base + tau * counts[k], base + (tau + 1) * counts[k])


def test_modules_with_zero_weights_carry_the_last_layers():
    # zero weights: every step's FC-2 term vanishes, so a module ends with its
    # group's last layer features; a merge selecting entry j returns it
    M, pts, dirs, f, feats = _tpl_setup()
    mods = [np.zeros_like(a) for a in weights.he_init_modules(2)]
    for p in range(len(pts)):
        d0 = oracle.modules(mods, feats[p], 0.9)
        assert np.all(d0[:192] == 0.0) and d0[192] == feats[p, 3 * 6 + 6] and d0[193] == feats[p, 3 * 6 + 7]
        assert d0[1056] == 0.9 and np.all(d0[194:1056] == 0.0)
    sel = [np.zeros_like(a) for a in weights.he_init_modules(2)]
    merges = sel[-6:]
    for tau in range(3):
        Mt = merges[2 * tau]
        Mt[0, 5] = 1.0          # a diffuse entry of the last diffuse layer (48 points)
        Mt[1, 48 + 3] = 1.0     # a highlight entry of the last highlight layer (8 points)
    for p in range(len(pts)):
        d1 = oracle.modules(sel, feats[p], 0.9)
        for tau in range(3):
            assert d1[tau * 64] == pytest.approx(feats[p, _layer_slice(7, tau)][5], rel=1e-15)
            assert d1[tau * 64 + 1] == pytest.approx(feats[p, _layer_slice(11, tau)][3], rel=1e-15)


@pytest.mark.parametrize("isel,vsel", [(0, 2), (16, 5), (17, 0)])
def test_module_last_step_closed_form(isel, vsel):
    # last highlight step (layer 10 -> 11; a = 16 + 2, b = 8) of type 1 (density):
    # S1[0][vsel] = 1 and S2[isel][0] = 1 gate entry isel of u = [h; g; alpha]
    # by sigmoid(ReLU(v_vsel)); F1 sends it to output 0, F2 = I, so
    # h_0 = ReLU(x11_0 + gate * u_isel) + x11_0 and h_o = ReLU(x11_o) + x11_o
    M, pts, dirs, f, feats = _tpl_setup()
    mods = [np.zeros_like(a) for a in weights.he_init_modules(2)]
    # index of the last highlight step of type 1 in the flat list: 8 arrays per step
    steps_per_type = 7 + 3
    step = 1 * steps_per_type + 7 + 2
    S1, e1, S2, e2, F1, f1, F2, f2 = mods[8 * step: 8 * step + 8]
    assert S2.shape == (18, 2) and F1.shape == (8, 18) and F2.shape == (8, 8)
    S1[0, vsel] = 1.0
    S2[isel, 0] = 1.0
    F1[0, isel] = 1.0
    F2[:, :] = np.eye(8)
    merges = mods[-6:]
    for o in range(8):
        merges[2 * 1][o, 48 + o] = 1.0
    counts = oracle.tpl_counts()
    for p in range(len(pts)):
        d = oracle.modules(mods, feats[p], 0.9)
        x10 = feats[p, _layer_slice(10, 1)]
        x11 = feats[p, _layer_slice(11, 1)]
        v10 = feats[p, sum(3 * c + 8 for c in counts[:10]) + 3 * 16:][:8]
        u = np.r_[x10, v10[6], v10[7]]
        gate = 1.0 / (1.0 + math.exp(-max(v10[vsel], 0.0)))
        h = np.maximum(x11, 0.0) + x11
        h[0] = max(x11[0] + gate * u[isel], 0.0) + x11[0]
        np.testing.assert_allclose(d[64:72], np.maximum(h, 0.0), rtol=1e-14)


def test_modules_query_zero_weights_give_single_scatter():
    M, pts, dirs, f, feats = _tpl_setup()
    params = weights.zeros_like(weights.he_init(16, 3, seed=1))
    mods = [np.zeros_like(a) for a in weights.he_init_modules(2)]
    q = M.tpl_modules_query(params, mods, pts, dirs, 8.0, 0.9, 0.85, 2.0)
    np.testing.assert_allclose(q["L"], 2.0 * f["f0"], rtol=1e-14)

"""GPU parity of every stage of the hot path against the FP64 oracle, called
through the C ABI.  Tolerances (FP32 path): pyramid rel 1e-6; path density
rel 2e-6 of the field's maximum; site densities exactly zero where the oracle's
are (the in-cube decision) and 2e-6 absolute elsewhere; graded transmittance,
phase and statistics 2e-5; radiance rel-L2 <= 1e-4.  BF16 radiance rel-L2 <=
1e-2."""

import numpy as np
import pytest
import torch

from gpu_common import Scene, camera, configs, f32, medium, oracle, rel_l2, set_precision, small_points, weights

pytestmark = pytest.mark.gpu

LIGHTS = [(0.3, 0.9, 0.3), (0.0, 1.0, 0.0), (0.0, -1.0, 0.0), (1.0, 0.2, -0.3),
          (-0.7, 0.2, 0.4), (0.1, -0.3, -0.95), (1.0, 1.0, 1.0)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_14051_amd import nis
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = nis.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 2, 16, 32])
def test_pyramid_matches_oracle(ctx, n):
    print("pyramid n=%d" % n, flush=True)
    rho = medium.fbm_cloud(n, seed=n) if n > 2 else np.random.default_rng(n).random((n, n, n)).astype(np.float32)
    mid = ctx.load_medium(rho, 8.0, 0.99, 0.85)
    om = oracle.Medium(rho)
    got = ctx.pyramid(mid)
    assert len(got) == om.levels
    for m in range(om.levels):
        np.testing.assert_allclose(got[m], om.level(m), rtol=1e-6, atol=1e-7)
    ctx.unload_medium(mid)


# (n, light): every test light at two sizes; lights whose shear times a slice
# index lands a hair above an integer, so that the rows of neighbouring rays
# are not one apart at every magnitude (the sweep's row-sharing exception);
# and the frame's size, whose slices take two chunks of the sweep's segments.
SWEEP_CASES = ([(n, light) for n in (8, 32) for light in LIGHTS]
               + [(32, (-0.9583333134651184, 1.0, 0.375)), (32, (-0.9375, 1.0, 0.4375)),
                  (128, (0.3, 0.9, 0.3)), (256, (0.3, 0.9, 0.3)), (256, (1.0, 0.2, -0.3))])


@pytest.mark.parametrize("n,light", SWEEP_CASES)
def test_sweep_matches_oracle(ctx, n, light):
    print("sweep n=%d light=%s" % (n, light), flush=True)
    rho = medium.fbm_cloud(n, seed=3)
    s = Scene(ctx, rho, light)
    for m in range(s.om.levels):
        ref, rng = s.om.path_density(m)
        got, grng = ctx.path_density(s.mid, m)
        assert grng == rng
        assert got.shape == ref.shape
        scale = max(ref.max(), 1e-30)
        np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6 * scale)
        # the gather's pairs along V hold the same values, index-clamped
        pairs = ctx.path_pairs(s.mid, m)
        nv = got.shape[1]
        vp = np.arange(nv + 1)
        np.testing.assert_array_equal(pairs[..., 0], got[:, np.clip(vp - 1, 0, nv - 1), :])
        np.testing.assert_array_equal(pairs[..., 1], got[:, np.clip(vp, 0, nv - 1), :])
    s.close()


@pytest.mark.parametrize("light,g", [((0.3, 0.9, 0.3), 0.85), ((-0.7, 0.2, 0.4), 0.5),
                                     ((0.1, -0.3, -0.95), 0.95), ((1.0, 0.2, -0.3), 0.0),
                                     ((0.2, 0.3, -0.9), -0.9),
                                     # multi-lobe phases (eq. 6): two and three HG lobes
                                     ((0.3, 0.9, 0.3), [(0.7, 0.8), (0.3, -0.4)]),
                                     ((-0.7, 0.2, 0.4), [(0.5, 0.95), (0.3, 0.2), (0.2, -0.7)])])
def test_features_match_oracle(ctx, light, g):
    print("features light=%s g=%s" % (light, g), flush=True)
    d, pts, dirs = small_points()
    s = Scene(ctx, d, light, g=g)
    params = weights.he_init(16, 3, seed=1)
    ctx.set_weights(params)
    ref = s.oracle_features(params, pts, dirs)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in ctx.features(s.mid, dev(pts), dev(dirs)).items()}
    # the in-cube decision of every site is exact
    np.testing.assert_array_equal(got["rho"] == 0, ref["rho"] == 0)
    np.testing.assert_allclose(got["rho"], ref["rho"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(got["tbar"], ref["tbar"], rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(got["phi"], ref["phi"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(got["stats"], ref["stats"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(got["tp"], ref["tp"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(got["f0"], ref["f0"], rtol=2e-5, atol=1e-9)
    s.close()


def frame_size_points(n, seed):
    """Points for the frame-size checks: inside the cube, within two voxels
    of a face (each face, corners included), and outside it."""
    r = np.random.default_rng(seed)
    inner = r.uniform(0.02, 0.98, (n // 2, 3))
    near = r.uniform(0.0, 1.0, (n // 4, 3))
    axis = r.integers(0, 3, n // 4)
    side = r.integers(0, 2, n // 4)
    near[np.arange(n // 4), axis] = np.where(side == 1, 1.0 - r.uniform(0, 2.0 / 256, n // 4),
                                             r.uniform(0, 2.0 / 256, n // 4))
    near[:4] = [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.001, 0.999, 0.5], [0.999, 0.001, 0.001]]
    outside = r.uniform(-0.05, 1.05, (n - n // 2 - n // 4, 3))
    outside[:, 0] = np.where(r.random(len(outside)) < 0.5, r.uniform(-0.05, -0.001, len(outside)),
                             r.uniform(1.001, 1.05, len(outside)))
    pts = np.concatenate([inner, near, outside]).astype(np.float32)
    dirs = r.standard_normal((n, 3))
    dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    return pts, dirs


@pytest.fixture(scope="module")
def frame_cloud():
    return configs.FRAME.density()


@pytest.mark.parametrize("light", [configs.LIGHT_DIR, (1.0, 0.2, -0.3)])
def test_features_descriptor_and_y_at_frame_size(ctx, frame_cloud, light):
    """The 256^3 frame medium (9 levels, the brick and slab paths a 32^3 grid
    never takes at levels 0-4), with the frame light and an x-dominant light:
    every site's density, graded transmittance and phase, the statistics, the
    descriptor and y (FP32, the frame's 10 x 200 network) element by element
    against the oracle, at 256 points inside the cube, within two voxels of
    its faces and outside it."""
    print("frame-size features light=%s" % (light,), flush=True)
    w = configs.FRAME
    pts, dirs = frame_size_points(256, seed=31)
    s = Scene(ctx, frame_cloud, light, w.sigma_t, w.albedo, w.g, w.radiance)
    params = w.params()
    ctx.set_weights(params)
    ctx.set_precision("fp32")
    ref = s.oracle_features(params, pts, dirs)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in ctx.features(s.mid, dev(pts), dev(dirs)).items()}
    np.testing.assert_array_equal(got["rho"] == 0, ref["rho"] == 0)
    np.testing.assert_allclose(got["rho"], ref["rho"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(got["tbar"], ref["tbar"], rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(got["phi"], ref["phi"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(got["stats"], ref["stats"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(got["tp"], ref["tp"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(got["f0"], ref["f0"], rtol=2e-5, atol=1e-9)
    q = s.oracle_query(params, pts, dirs, want_desc=True)
    desc, y = ctx.network(s.mid, dev(pts), dev(dirs))
    np.testing.assert_allclose(desc.cpu().numpy().astype(np.float64), q["desc"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(y.cpu().numpy(), q["y"], rtol=0, atol=2e-5 * np.abs(q["y"]).max())
    s.close()


def test_descriptor_and_network_output_fp32(ctx):
    d, pts, dirs = small_points(extra_random=100)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(128, 6, seed=1, bias_scale=0.05)
    ctx.set_weights(params)
    ctx.set_precision("fp32")
    ref = s.oracle_query(params, pts, dirs, want_desc=True)
    desc, y = ctx.network(s.mid, dev(pts), dev(dirs))
    desc = desc.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(desc, ref["desc"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(y.cpu().numpy(), ref["y"], rtol=0, atol=2e-5 * np.abs(ref["y"]).max())
    s.close()


FP8_TARGET_MISS = pytest.mark.xfail(
    strict=True, reason="E4M3 keeps 3 mantissa bits: over these He-init backbones every scaling scheme "
                        "(static per-layer activation scales with per-channel power-of-two or MX-block weight "
                        "scales, per-row/per-column absmax, BF16 first and last layers) floors at a radiance "
                        "rel-L2 of about 0.04-0.05, above the 3e-2 target")


# FP8 regression bound on the small workload: a host emulation of the FP8
# scheme (static per-layer activation scales, per-channel power-of-two weight
# scales, E4M3 descriptor) on the oracle's descriptors gives radiance rel-L2
# 0.069 / 0.078 / 0.064 / 0.148 at g = 0 / 0.5 / 0.85 / 0.95 on this 6 x 128
# network; a layout or scale mistake gives errors of order one.
FP8_BOUND = 0.2


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2),
                                      pytest.param("fp8", 3e-2, marks=FP8_TARGET_MISS),
                                      ("fp8", FP8_BOUND)])
def test_query_small_workload(ctx, prec, tol):
    """The 32^3 / 64x64 / 6x128 workload end to end.  FP32 and BF16 meet their
    targets (1e-4, 1e-2).  FP8 is checked against its target (3e-2, recorded as
    not met) and against the bound it achieves, which guards regressions."""
    w = configs.SMALL
    d = w.density()
    pts, dirs, _ = w.points(d)
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    params = w.params()
    ctx.set_weights(params)
    set_precision(ctx, prec, s.mid, pts, dirs)
    ref = s.oracle_query(params, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    err = rel_l2(L, ref["L"])
    _, y = ctx.network(s.mid, dev(pts), dev(dirs), want_desc=False)
    Fg = f32(w.albedo) ** 4 * np.expm1(y.cpu().numpy().astype(np.float64))
    print("%s small: rel-L2(L) %.3g rel-L2(F) %.3g max|dy| %.3g" % (
        prec, err, rel_l2(Fg, ref["F"]), np.abs(y.cpu().numpy() - ref["y"]).max()), flush=True)
    assert err <= tol
    assert rel_l2(Fg, ref["F"]) <= tol
    ctx.set_precision("fp32")
    s.close()


@pytest.mark.parametrize("g", [0.0, 0.5, 0.95])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2), ("fp8", FP8_BOUND)])
def test_query_small_workload_g_sweep(ctx, g, prec, tol):
    """The small workload at the other HG asymmetries of the precision
    workload (0.85 is the test above): FP32 and BF16 within their targets, FP8
    within the bound it achieves."""
    w = configs.SMALL
    d = w.density()
    pts, dirs, _ = w.points(d)
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, g, w.radiance)
    params = w.params()
    ctx.set_weights(params)
    set_precision(ctx, prec, s.mid, pts, dirs)
    ref = s.oracle_query(params, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    ctx.set_precision("fp32")
    err = rel_l2(L, ref["L"])
    print("g=%s %s small: rel-L2(L) %.3g" % (g, prec, err), flush=True)
    assert err <= tol
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("width", [16, 24, 100, 200, 256])
def test_backbone_widths(ctx, width, prec):
    """Every padded backbone width, including widths whose padding is not a
    multiple of the MFMA K step.  FP32: radiance rel-L2 <= 1e-4.  BF16: these
    random networks put y near 0, where a relative radiance error says little,
    so the bound is on y itself: |dy| <= 0.04, about ten bfloat16 unit
    roundoffs (2^-8) for four layers with activations of order one."""
    d, pts, dirs = small_points(extra_random=100)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(width, 4, seed=width, bias_scale=0.05)
    ctx.set_weights(params)
    set_precision(ctx, prec, s.mid, pts, dirs)
    ref = s.oracle_query(params, pts, dirs)
    _, y = ctx.network(s.mid, dev(pts), dev(dirs), want_desc=False)
    L = ctx.query(s.mid, pts, dirs)
    ctx.set_precision("fp32")
    print("width %d %s: rel-L2(L) %.3g max|dy| %.3g" % (
        width, prec, rel_l2(L, ref["L"]), np.abs(y.cpu().numpy() - ref["y"]).max()), flush=True)
    assert np.all(np.isfinite(L))
    dy = np.abs(y.cpu().numpy() - ref["y"]).max()
    if prec == "fp32":
        assert rel_l2(L, ref["L"]) <= 1e-4
    elif prec == "bf16":
        assert dy <= 0.04
    else:
        # E4M3 unit roundoff is 2^-4 (6.25%); three quantised layers of
        # order-one activations, twice the worst case seen (0.38)
        assert dy <= 0.75
    s.close()


def test_multi_lobe_phase_query_and_single_lobe_identity(ctx):
    """FP32 radiance with a two-lobe phase meets the FP32 bound against the
    oracle; one lobe of weight 1 gives the plain-HG features bit for bit."""
    d, pts, dirs = small_points(extra_random=100)
    phase = [(0.6, 0.9), (0.4, -0.3)]
    s = Scene(ctx, d, (0.2, -0.5, 0.8), g=phase)
    params = weights.he_init(128, 6, seed=1, bias_scale=0.05)
    ctx.set_weights(params)
    ctx.set_precision("fp32")
    ref = s.oracle_query(params, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    assert rel_l2(L, ref["L"]) <= 1e-4
    ctx.set_phase_lobes(s.mid, [(1.0, 0.7)])
    one = ctx.features(s.mid, dev(pts), dev(dirs))
    ctx.set_medium_params(s.mid, 8.0, 0.99, 0.7)
    plain = ctx.features(s.mid, dev(pts), dev(dirs))
    for k in one:
        np.testing.assert_array_equal(one[k].cpu().numpy(), plain[k].cpu().numpy())
    s.close()


# The volume phase (eq. 9) is tabulated per light and phase over the angle
# between w and each site direction (2048 bins, linear interpolation): the
# interpolation error, about (h^2/8) max|d2f/dangle2| with h = pi/2047, is
# largest for the sharpest lobe and the narrowest cone (g = 0.95, the
# farthest sites); measured maxima of |dphi| are 1.4e-4 (g = 0.95),
# 3.8e-5 (g = -0.9), 1.9e-5 (g = 0.85), and fall as h^2 with the bin count.
VOLUME_PHI_ATOL = 3e-4


@pytest.mark.parametrize("light,g", [((0.3, 0.9, 0.3), 0.85), ((-0.7, 0.2, 0.4), 0.95),
                                     ((0.2, 0.3, -0.9), -0.9),
                                     ((0.1, -0.3, -0.95), [(0.7, 0.8), (0.3, -0.4)])])
def test_volume_phase_features_match_oracle(ctx, light, g):
    print("volume phase light=%s g=%s" % (light, g), flush=True)
    d, pts, dirs = small_points()
    s = Scene(ctx, d, light, g=g, volume=True)
    params = weights.he_init(16, 3, seed=1)
    ctx.set_weights(params)
    ref = s.oracle_features(params, pts, dirs)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in ctx.features(s.mid, dev(pts), dev(dirs)).items()}
    np.testing.assert_allclose(got["phi"], ref["phi"], rtol=0, atol=VOLUME_PHI_ATOL)
    np.testing.assert_allclose(got["stats"], ref["stats"], rtol=2e-5, atol=VOLUME_PHI_ATOL)
    # only the phase features change
    np.testing.assert_allclose(got["tbar"], ref["tbar"], rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(got["f0"], ref["f0"], rtol=2e-5, atol=1e-9)
    s.close()


def test_volume_phase_query_and_switching_back(ctx):
    """FP32 radiance with volume phases against the oracle; switching the
    volume phase off again restores the point-phase features bit for bit."""
    d, pts, dirs = small_points(extra_random=100)
    s = Scene(ctx, d, (0.2, -0.5, 0.8), g=0.9, volume=True)
    params = weights.he_init(128, 6, seed=1, bias_scale=0.05)
    ctx.set_weights(params)
    ctx.set_precision("fp32")
    ref = s.oracle_query(params, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    err = rel_l2(L, ref["L"])
    print("volume phase FP32 rel-L2 %.3g" % err, flush=True)
    # the tables' phase-feature error (|dphi| <= 3e-4) passes through the
    # network into y (measured 8.8e-7 here); the FP32 arithmetic alone stays
    # near 3e-7
    assert err <= 1e-5
    ctx.set_volume_phase(s.mid, False)
    off = ctx.features(s.mid, dev(pts), dev(dirs))
    fresh = Scene(ctx, d, (0.2, -0.5, 0.8), g=0.9)
    plain = ctx.features(fresh.mid, dev(pts), dev(dirs))
    for k in off:
        np.testing.assert_array_equal(off[k].cpu().numpy(), plain[k].cpu().numpy())
    fresh.close()
    s.close()


def test_zero_weights_reduce_to_single_scatter(ctx):
    d, pts, dirs = small_points()
    s = Scene(ctx, d, (0.2, -0.5, 0.8), radiance=2.5)
    params = weights.zeros_like(weights.he_init(16, 3))
    ctx.set_weights(params)
    L = ctx.query(s.mid, pts, dirs)
    feat = s.oracle_features(params, pts, dirs)
    np.testing.assert_allclose(L, 2.5 * feat["f0"], rtol=2e-5, atol=1e-9)
    s.close()


@pytest.mark.parametrize("entry", [0, 44, 79, 80, 81, 82, 83, 84, 85, 86, 87, 88 * 7 + 3, 88 * 8 + 50,
                                   88 * 11 + 85, 1056])
def test_selector_weights_reach_every_descriptor_part(ctx, entry):
    d, pts, dirs = small_points(extra_random=50)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(16, 3, seed=3)
    for A in params["A"]:
        A[:] = 0.0
    params["A"][0][0, entry] = 1.0
    params["A"][1][0, 0] = 1.0
    params["A"][2][0, 0] = 1.0
    ctx.set_weights(params)
    ref = s.oracle_query(params, pts, dirs, want_desc=True)
    _, y = ctx.network(s.mid, dev(pts), dev(dirs), want_desc=False)
    scale = max(np.abs(ref["desc"][:, entry]).max(), 1e-6)
    np.testing.assert_allclose(y.cpu().numpy(), ref["desc"][:, entry], rtol=2e-5, atol=2e-6 * scale)
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("count", [1, 31, 33, 127, 129, 1000])
def test_ragged_batches_and_batch_invariance(ctx, count, prec):
    d, pts, dirs = small_points()
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(128, 6, seed=1)
    ctx.set_weights(params)
    set_precision(ctx, prec, s.mid, pts, dirs)
    full = ctx.query(s.mid, pts, dirs)
    idx = np.random.default_rng(count).choice(len(pts), count, replace=False)
    part = ctx.query(s.mid, pts[idx], dirs[idx])
    np.testing.assert_array_equal(part, full[idx])          # points are independent
    again = ctx.query(s.mid, pts, dirs)
    np.testing.assert_array_equal(again, full)              # deterministic
    ctx.set_precision("fp32")
    s.close()


def test_fp8_needs_activation_scales(ctx):
    """FP8 is refused (NIS_E_UNSUPPORTED) until the backbone's static
    activation scales are known; scales from the weight blob are used as
    given (non-positive ones are refused), and calibration replaces them.
    A blob whose scales are 1 (codes = values) clips the descriptor's entries
    above 448 only, so its radiance stays within the FP8 bound."""
    from paper_2401_14051_amd import nis
    w = configs.SMALL
    d = w.density()
    pts, dirs, _ = w.points(d)
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    params = w.params()
    ctx.set_weights(params)
    with pytest.raises(nis.NisError) as e:
        ctx.set_precision("fp8")
    assert e.value.code == nis.NIS_E_UNSUPPORTED
    with pytest.raises(nis.NisError) as e:
        ctx.set_weights(params, fp8_scales=np.r_[1.0, 1.0, np.zeros(params["n_linear"])])
    assert e.value.code == nis.NIS_E_INVALID
    ref = s.oracle_query(params, pts, dirs)["L"]
    # calibrated scales
    set_precision(ctx, "fp8", s.mid, pts, dirs)
    cal = ctx.query(s.mid, pts, dirs)
    # weights without scales while FP8 is selected: queries are refused
    ctx.set_weights(params)
    with pytest.raises(nis.NisError) as e:
        ctx.query(s.mid, pts, dirs)
    assert e.value.code == nis.NIS_E_UNSUPPORTED
    # scales in the blob
    ctx.set_weights(params, fp8_scales=np.ones(2 + params["n_linear"]))
    ones = ctx.query(s.mid, pts, dirs)
    ctx.set_precision("fp32")
    print("fp8 calibrated %.3g, unit scales %.3g" % (rel_l2(cal, ref), rel_l2(ones, ref)), flush=True)
    assert rel_l2(cal, ref) <= FP8_BOUND
    assert np.all(np.isfinite(ones))
    s.close()


@pytest.mark.parametrize("n", [1, 2, 4])
def test_tiny_media(ctx, n):
    rho = np.random.default_rng(n).random((n, n, n)).astype(np.float32)
    pts, dirs = camera.random_points(200, seed=n, lo=-0.2, hi=1.2)
    s = Scene(ctx, rho, (0.4, -0.2, 0.7))
    params = weights.he_init(32, 3, seed=2, bias_scale=0.1)
    ctx.set_weights(params)
    ref = s.oracle_query(params, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    assert rel_l2(L, ref["L"]) <= 1e-4
    s.close()


def test_invalid_arguments_are_rejected(ctx):
    from paper_2401_14051_amd import nis
    rho = medium.fbm_cloud(8)
    with pytest.raises(nis.NisError) as e:
        ctx.load_medium(np.zeros((6, 6, 6), np.float32), 8.0, 0.9, 0.5)
    assert e.value.code == nis.NIS_E_INVALID
    for bad in [(-1.0, 0.9, 0.5), (8.0, 1.5, 0.5), (8.0, 0.9, 1.0), (np.nan, 0.9, 0.5)]:
        with pytest.raises(nis.NisError):
            ctx.load_medium(rho, *bad)
    bad_rho = rho.copy()
    bad_rho[1, 2, 3] = np.inf
    with pytest.raises(nis.NisError):
        ctx.load_medium(bad_rho, 8.0, 0.9, 0.5)
    mid = ctx.load_medium(rho, 8.0, 0.9, 0.5)
    with pytest.raises(nis.NisError) as e:
        ctx.set_light(mid, (0.0, 0.0, 0.0))
    assert e.value.code == nis.NIS_E_INVALID
    for lobes in ([], [(0.2, 0.1)] * 5, [(0.5, 0.3), (0.4, 0.2)], [(1.0, 1.0)], [(1.5, 0.2), (-0.5, 0.1)],
                  [(0.5, np.nan), (0.5, 0.1)]):
        with pytest.raises(nis.NisError) as e:
            ctx.set_phase_lobes(mid, lobes)
        assert e.value.code == nis.NIS_E_INVALID
    with pytest.raises(nis.NisError) as e:
        nis._check(nis._lib.nis_set_volume_phase(ctx.h, mid, 2))   # only 0 and 1
    assert e.value.code == nis.NIS_E_INVALID
    pts, dirs = camera.random_points(10, seed=1)
    with pytest.raises(nis.NisError) as e:
        ctx.query(mid, pts, dirs)
    assert e.value.code == nis.NIS_E_STATE                  # no light yet
    ctx.set_light(mid, (0.3, 0.9, 0.3))
    with pytest.raises(nis.NisError) as e:
        ctx.query(99999, pts, dirs)
    assert e.value.code == nis.NIS_E_STATE
    bad = pts.copy()
    bad[3, 1] = np.nan
    ctx.set_weights(weights.he_init(16, 3))
    with pytest.raises(nis.NisError) as e:
        ctx.query(mid, bad, dirs)
    assert e.value.code == nis.NIS_E_INVALID
    zd = dirs.copy()
    zd[2] = 0
    with pytest.raises(nis.NisError):
        ctx.query(mid, pts, zd)
    with pytest.raises(nis.NisError) as e:
        ctx.set_weights(blob=b"NISW" + b"\0" * 100)
    assert e.value.code == nis.NIS_E_INVALID
    with pytest.raises(nis.NisError) as e:
        ctx.set_precision(7)
    assert e.value.code == nis.NIS_E_INVALID
    assert nis.nis_query(ctx.h, mid, None, None, 0, None) == nis.NIS_E_INVALID
    ctx.unload_medium(mid)
    with pytest.raises(nis.NisError):
        ctx.unload_medium(mid)


def test_medium_params_change_without_resweep(ctx):
    d, pts, dirs = small_points(extra_random=50)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(32, 3, seed=4)
    ctx.set_weights(params)
    ctx.query(s.mid, pts, dirs)
    ctx.set_medium_params(s.mid, 5.0, 0.9, 0.3)
    s.sigma_t, s.albedo, s.g = 5.0, 0.9, 0.3
    ref = s.oracle_query(params, pts, dirs)
    assert rel_l2(ctx.query(s.mid, pts, dirs), ref["L"]) <= 1e-4
    s.close()


def test_mirroring_the_dominant_axis(ctx):
    rho = medium.fbm_cloud(32, seed=12)
    params = weights.he_init(32, 3, seed=2, bias_scale=0.1)
    ctx.set_weights(params)
    rng = np.random.default_rng(5)
    pts = (np.floor(rng.random((300, 3)) * 2 ** 20) / 2 ** 20).astype(np.float32)
    dirs = rng.standard_normal((300, 3)).astype(np.float32)
    a = ctx.load_medium(rho, 8.0, 0.99, 0.85)
    ctx.set_light(a, (0.3, 0.9, 0.3))
    b = ctx.load_medium(np.ascontiguousarray(rho[:, ::-1, :]), 8.0, 0.99, 0.85)
    ctx.set_light(b, (0.3, -0.9, 0.3))
    pm, dm = pts.copy(), dirs.copy()
    pm[:, 1] = 1.0 - pm[:, 1]
    dm[:, 1] = -dm[:, 1]
    np.testing.assert_allclose(ctx.query(a, pts, dirs), ctx.query(b, pm, dm), rtol=1e-5, atol=1e-7)
    ctx.unload_medium(a)
    ctx.unload_medium(b)


def test_device_query_on_a_torch_stream(ctx):
    d, pts, dirs = small_points()
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(128, 6, seed=1)
    ctx.set_weights(params)
    host = ctx.query(s.mid, pts, dirs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p, q = dev(pts), dev(dirs)
        out = torch.empty(len(pts), dtype=torch.float32, device="cuda")
        ctx.query_device(s.mid, p, q, out)
    stream.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), host)
    s.close()


@pytest.fixture(scope="module")
def diag512(ctx):
    """A 512^3 medium under a light along the cube's diagonal, loaded on both
    sides; its finest level's path-density pairs take 4.3 GB."""
    from paper_2401_14051_amd import nis
    light = (1.0, 1.0, 1.0)
    fp = nis.light_footprint(512, light)
    assert fp["levels"][0] >= 1 << 32
    print("diagonal light 512^3: level 0 pairs %d bytes" % fp["levels"][0], flush=True)
    s = Scene(ctx, configs.LARGE.density(), light)
    yield s, fp
    s.close()


def diag_points(n_face=384, n_any=128, seed=17):
    """Points near the face away from the light (1,1,1), whose lattices reach
    the finest level's last slices, and points anywhere in the cube."""
    r = np.random.default_rng(seed)
    pts = np.concatenate([np.column_stack([r.uniform(0.0, 0.012, n_face), r.uniform(0.05, 0.95, (n_face, 2))]),
                          r.uniform(0.0, 1.0, (n_any, 3))]).astype(np.float32)
    dirs = r.standard_normal((n_face + n_any, 3))
    dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    return pts, dirs


def test_diagonal_light_past_4gib_at_512(ctx, diag512):
    """The 512^3 medium under the diagonal light: its finest level's
    path-density pairs pass what one 32-bit buffer offset reaches.  The
    sweep's slices beyond the 4 GiB mark hold the oracle's path density (rel
    2e-6 of the maximum), and the gather reads them: features, FP32 radiance
    (rel-L2 1e-4) and the paper templates' FP32 radiance at points near the
    face away from the light, whose lattices reach those slices, match the
    oracle."""
    s, fp = diag512
    got, grng = ctx.path_density(s.mid, 0)
    ref, rng = s.om.path_density(0)
    assert grng == rng and got.shape == ref.shape
    row_bytes = (got.shape[2] + 4) * (got.shape[1] + 1) * 8
    assert row_bytes * 512 == fp["levels"][0]
    first = (1 << 32) // row_bytes             # the slice that straddles the mark
    assert first < 511
    scale = float(ref.max())
    for J in [0, 200] + list(range(first - 2, 512)):
        np.testing.assert_allclose(got[J], ref[J], rtol=0, atol=2e-6 * scale, err_msg="slice %d" % J)
    del got, ref
    print("diagonal light 512^3: path density ok (slices from %d)" % first, flush=True)
    # the light's dominant axis is x and points towards +x: slices of large J
    # lie at small x
    pts, dirs = diag_points()
    params = weights.he_init(16, 3, seed=1)
    ctx.set_weights(params)
    ref = s.oracle_features(params, pts, dirs)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in ctx.features(s.mid, dev(pts), dev(dirs)).items()}
    np.testing.assert_array_equal(got["rho"] == 0, ref["rho"] == 0)
    np.testing.assert_allclose(got["rho"], ref["rho"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(got["tbar"], ref["tbar"], rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(got["stats"], ref["stats"], rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(got["tp"], ref["tp"], rtol=2e-5, atol=1e-7)
    # the points' sites reach the slices past the mark
    assert ref["tbar"].min() < 0.99
    ctx.set_precision("fp32")
    L = ctx.query(s.mid, pts, dirs)
    err = rel_l2(L, s.oracle_query(params, pts, dirs)["L"])
    ctx.set_templates("paper")
    try:
        Lt = ctx.query(s.mid, pts, dirs)
    finally:
        ctx.set_templates("lattice")
    err_t = rel_l2(Lt, s.oracle_tpl_query(params, pts, dirs)["L"])
    print("diagonal light 512^3: rel-L2 lattice %.3g templates %.3g" % (err, err_t), flush=True)
    assert err <= 1e-4 and err_t <= 1e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_diagonal_light_512_in_batches_and_frames(ctx, diag512, prec):
    """The gather's 64-bit path inside shared launches: a query batch over the
    diagonal-light 512^3 medium and a 32^3 medium equals their single queries,
    and frames of both from the frame server with batch_gather (small frames
    admitted together share one gather) equal their synchronous renders, bit
    for bit."""
    s, _ = diag512
    print("diagonal light 512^3 in batches and frames %s" % prec, flush=True)
    params = weights.he_init(16, 3, seed=1)
    ctx.set_weights(params)
    set_precision(ctx, prec)
    small = ctx.load_medium(medium.fbm_cloud(32, seed=9), 8.0, 0.99, 0.85)
    ctx.set_light(small, (0.3, 0.9, 0.3), 1.0)
    try:
        pts, dirs = diag_points(96, 64, seed=23)
        qp, qd = dev(pts), dev(dirs)
        singles = []
        for m in (s.mid, small):
            out = torch.empty(len(pts), dtype=torch.float32, device="cuda")
            ctx.query_device(m, qp, qd, out)
            singles.append(out)
        outs = [torch.full((len(pts),), -1.0, device="cuda") for _ in range(2)]
        ctx.query_batch([(s.mid, qp, qd, outs[0]), (small, qp, qd, outs[1])])
        torch.cuda.synchronize()
        for a, b in zip(outs, singles):
            assert torch.equal(a, b)
        # frames of both media through the server
        from paper_2401_14051_amd import nis
        cam = nis.camera(96, 96, 45.0)
        reqs = [(s.mid, (1.0, 1.0, 1.0), 11), (small, (0.3, 0.9, 0.3), 12)]
        ctx.server_start(1 << 36, prec, 4, batch_gather=True)
        try:
            ids = [ctx.submit(m, cam, l, 1.0, 0.85, seed) for m, l, seed in reqs]
            served = []
            for fid in ids:
                r = ctx.wait(fid)
                assert r.status == 0, r.status
                served.append(ctx.frame_image(r).cpu().numpy())
                ctx.release(fid)
        finally:
            ctx.server_stop()
        for (m, l, seed), img in zip(reqs, served):
            ctx.set_light(m, l, 1.0)
            ref = ctx.render(m, cam, seed).cpu().numpy()
            assert np.count_nonzero(ref) > 100
            np.testing.assert_array_equal(img, ref)
    finally:
        ctx.set_precision("fp32")
        ctx.unload_medium(small)

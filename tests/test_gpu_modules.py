"""GPU parity of the paper's backbone modules (Sec. III.C.2, Fig. 6, eq.
24-26; nis_set_backbone) over the paper's templates against the FP64 oracle,
through the C ABI.

Tolerances.  The modules run in FP32 on template features that match the
oracle to about 2e-5 relative; pushing features perturbed by 2e-5 (relative,
uniform) through the oracle's modules moves a descriptor row by at most
1.6e-5 of its largest entry (He-initialised modules, biases 0.05), so the
descriptor is checked per row against 5e-5 of the row's largest magnitude;
y to 1e-4 of max |y|; radiance rel-L2 <= 1e-4.  Rounding the modules'
descriptor alone to bfloat16 moves y by up to 0.007 on the oracle, so BF16
is bounded as the template path's BF16 is, |dy| <= 0.04; FP8 |dy| <= 0.5."""

import numpy as np
import pytest
import torch

from gpu_common import Scene, configs, f32, oracle_params, rel_l2, set_precision, small_points, weights

pytestmark = pytest.mark.gpu

PARAMS = dict(width=128, n_linear=6, seed=1, bias_scale=0.05)


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_14051_amd import nis
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = nis.Context(0)
    c.set_templates("paper")
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def mods(seed=2, bias_scale=0.05):
    return weights.he_init_modules(seed=seed, bias_scale=bias_scale)


def check_desc_y(desc, y, ref):
    d = desc.cpu().numpy().astype(np.float64)
    rowmax = np.abs(ref["desc"]).max(axis=1, keepdims=True)
    err = np.abs(d - ref["desc"])
    worst = float((err / rowmax).max())
    print("modules descriptor: worst row-relative error %.3g" % worst, flush=True)
    assert np.all(err <= 5e-5 * rowmax + 1e-7)
    yy = y.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(yy, ref["y"], rtol=0, atol=1e-4 * np.abs(ref["y"]).max())


def set_paper(ctx, params, m):
    ctx.set_weights(params, modules=m)
    ctx.set_backbone("paper")


def test_modules_descriptor_and_y_fp32(ctx):
    d, pts, dirs = small_points(extra_random=200)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(**PARAMS)
    m = mods()
    set_paper(ctx, params, m)
    ctx.set_precision("fp32")
    ref = s.oracle_tpl_modules_query(params, m, pts, dirs, want_desc=True)
    desc, y = ctx.network(s.mid, dev(pts), dev(dirs))
    check_desc_y(desc, y, ref)
    ctx.set_backbone("mlp")
    s.close()


@pytest.mark.parametrize("light,g", [((-0.7, 0.2, 0.4), 0.5), ((1.0, 0.2, -0.3), [(0.7, 0.8), (0.3, -0.4)])])
def test_modules_other_lights_and_phases(ctx, light, g):
    d, pts, dirs = small_points(extra_random=100, seed=9)
    s = Scene(ctx, d, light, g=g)
    params = weights.he_init(**PARAMS)
    m = mods(seed=4)
    set_paper(ctx, params, m)
    ctx.set_precision("fp32")
    ref = s.oracle_tpl_modules_query(params, m, pts, dirs, want_desc=True)
    desc, y = ctx.network(s.mid, dev(pts), dev(dirs))
    check_desc_y(desc, y, ref)
    ctx.set_backbone("mlp")
    s.close()


def test_modules_at_frame_size(ctx):
    """The 256^3 frame medium and its 10 x 200 network: points inside, near the
    faces of and outside the cube."""
    from test_gpu_parity import frame_size_points
    w = configs.FRAME
    pts, dirs = frame_size_points(256, seed=43)
    s = Scene(ctx, w.density(), w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    params = weights.he_init(w.width, w.n_linear, seed=w.weight_seed, bias_scale=0.05)
    m = mods()
    set_paper(ctx, params, m)
    ctx.set_precision("fp32")
    ref = s.oracle_tpl_modules_query(params, m, pts, dirs, want_desc=True)
    desc, y = ctx.network(s.mid, dev(pts), dev(dirs))
    check_desc_y(desc, y, ref)
    ctx.set_backbone("mlp")
    s.close()


@pytest.mark.parametrize("prec,dy_tol", [("fp32", None), ("bf16", 0.04), ("fp8", 0.5)])
def test_modules_query_small_workload(ctx, prec, dy_tol):
    w = configs.SMALL
    d = w.density()
    pts, dirs, _ = w.points(d)
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    params = w.params()
    m = mods(bias_scale=0.0)
    set_paper(ctx, params, m)
    set_precision(ctx, prec, s.mid, pts, dirs)
    ref = s.oracle_tpl_modules_query(params, m, pts, dirs)
    L = ctx.query(s.mid, pts, dirs)
    _, y = ctx.network(s.mid, dev(pts), dev(dirs), want_desc=False)
    ctx.set_precision("fp32")
    ctx.set_backbone("mlp")
    err = rel_l2(L, ref["L"])
    dy = np.abs(y.cpu().numpy() - ref["y"]).max()
    print("modules %s small: rel-L2 %.3g max|dy| %.3g" % (prec, err, dy), flush=True)
    assert np.all(np.isfinite(L))
    if dy_tol is None:
        assert err <= 1e-4
    else:
        assert dy <= dy_tol
    s.close()


def test_modules_chunks(ctx):
    """More points than one module pass (65,536): the whole query equals, bit
    for bit, the queries of its two parts, and a sample matches the oracle."""
    from workloads import camera
    d, _, _ = small_points(extra_random=0)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(64, 4, seed=3, bias_scale=0.05)
    m = mods()
    set_paper(ctx, params, m)
    ctx.set_precision("bf16")
    pts, dirs = camera.random_points(70001, seed=17, lo=-0.1, hi=1.1)
    L = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    ctx.query_device(s.mid, dev(pts), dev(dirs), L)
    cut = 65536 + 123
    La = torch.empty(cut, dtype=torch.float32, device="cuda")
    Lb = torch.empty(len(pts) - cut, dtype=torch.float32, device="cuda")
    ctx.query_device(s.mid, dev(pts[:cut]), dev(dirs[:cut]), La)
    ctx.query_device(s.mid, dev(pts[cut:]), dev(dirs[cut:]), Lb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(L.cpu().numpy(), torch.cat([La, Lb]).cpu().numpy())
    ctx.set_precision("fp32")
    idx = np.random.default_rng(3).choice(len(pts), 300, replace=False)
    idx = np.concatenate([idx, [0, 65535, 65536, len(pts) - 1]])
    Lf = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    ctx.query_device(s.mid, dev(pts), dev(dirs), Lf)
    torch.cuda.synchronize()
    ref = s.oracle_tpl_modules_query(params, m, pts[idx], dirs[idx])["L"]
    assert rel_l2(Lf.cpu().numpy()[idx], ref) <= 1e-4
    ctx.set_backbone("mlp")
    s.close()


def test_modules_render_equals_query_of_frame_points(ctx):
    from paper_2401_14051_amd import nis
    from workloads import medium
    d = medium.fbm_cloud(32, seed=5)
    mid = ctx.load_medium(d, 8.0, 0.9, 0.7)
    ctx.set_light(mid, (0.3, 0.9, 0.3), 1.0)
    set_paper(ctx, weights.he_init(64, 4, seed=3, bias_scale=0.05), mods())
    ctx.set_precision("bf16")
    cam = nis.camera(101, 43, 40.0, eye=(1.6, 0.7, 1.2))
    img = ctx.render(mid, cam, 7).cpu().numpy().ravel()
    p, dd, pix = ctx.frame_points(mid, cam, 7)
    L = torch.empty(p.shape[0], dtype=torch.float32, device="cuda")
    ctx.query_device(mid, p, dd, L)
    torch.cuda.synchronize()
    exp = np.zeros(101 * 43, np.float32)
    exp[pix.cpu().numpy()] = np.float32(0.9) * L.cpu().numpy()
    np.testing.assert_array_equal(img, exp)
    ctx.set_precision("fp32")
    ctx.set_backbone("mlp")
    ctx.unload_medium(mid)


def test_modules_rgb_channels(ctx):
    """Per-channel albedo: each channel's radiance equals the grey query of a
    medium with that albedo (the modules do not read the albedo)."""
    d, pts, dirs = small_points(extra_random=50)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(**PARAMS)
    m = mods()
    set_paper(ctx, params, m)
    ctx.set_precision("fp32")
    rgb = (0.99, 0.9, 0.7)
    ctx.set_albedo_rgb(s.mid, rgb)
    L3 = ctx.query_rgb(s.mid, pts, dirs)
    for c in range(3):
        ref = s.om.tpl_modules_query(oracle_params(params), m, pts, dirs, f32(s.sigma_t), f32(rgb[c]),
                                     s.phase(), f32(s.radiance))["L"]
        assert rel_l2(L3[:, c], ref) <= 1e-4
    ctx.set_backbone("mlp")
    s.close()


def test_modules_errors(ctx):
    from paper_2401_14051_amd import nis
    d, pts, dirs = small_points(extra_random=10)
    s = Scene(ctx, d, configs.LIGHT_DIR)
    params = weights.he_init(16, 3, seed=1)
    ctx.set_weights(params)
    with pytest.raises(nis.NisError) as e:
        ctx.set_backbone(5)
    assert e.value.code == nis.NIS_E_INVALID
    with pytest.raises(nis.NisError) as e:   # weights without modules
        ctx.set_backbone("paper")
    assert e.value.code == nis.NIS_E_STATE
    set_paper(ctx, params, mods())
    ctx.set_weights(params)                  # replaced by weights without modules
    with pytest.raises(nis.NisError) as e:
        ctx.query(s.mid, pts, dirs)
    assert e.value.code == nis.NIS_E_STATE
    set_paper(ctx, params, mods())
    ctx.set_templates("lattice")
    with pytest.raises(nis.NisError) as e:   # the modules read the paper's templates
        ctx.query(s.mid, pts, dirs)
    assert e.value.code == nis.NIS_E_STATE
    ctx.set_templates("paper")
    out = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    with pytest.raises(nis.NisError) as e:
        ctx.query_device_noalloc(s.mid, dev(pts), dev(dirs), out)
    assert e.value.code == nis.NIS_E_UNSUPPORTED
    # malformed module blocks
    blob = bytearray(nis.pack_weights(params, modules=mods()))
    with pytest.raises(nis.NisError) as e:
        ctx.set_weights(blob=bytes(blob[:-4]))
    assert e.value.code == nis.NIS_E_INVALID
    blob[36:40] = (2).to_bytes(4, "little")   # has_modules
    with pytest.raises(nis.NisError) as e:
        ctx.set_weights(blob=bytes(blob))
    assert e.value.code == nis.NIS_E_INVALID
    # back to the plain MLP: the template path's results
    ctx.set_backbone("mlp")
    L = ctx.query(s.mid, pts, dirs)
    ref = s.oracle_tpl_query(params, pts, dirs)["L"]
    assert rel_l2(L, ref) <= 1e-4
    s.close()

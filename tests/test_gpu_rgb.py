"""A coloured albedo (Sec. III.C.2: one albedo per red, green and blue channel;
eq. 21 decodes channel c with albedo_c^gamma), called through the C ABI.

The oracle evaluates each channel as a grey query with that channel's albedo,
so channel c of the RGB path is held to the one-channel bounds (FP32 rel-L2
1e-4, BF16 1e-2).  The RGB path shares the features between the channels and
rewrites only the descriptor's albedo entry, so each channel also equals the
one-channel query at that albedo bit for bit, at every precision."""

import numpy as np
import pytest
import torch

from gpu_common import Scene, camera, configs, f32, rel_l2, set_precision, small_points, weights

pytestmark = pytest.mark.gpu

RGB = (0.95, 0.6, 0.3)


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_14051_amd import nis
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = nis.Context(0)
    yield c
    c.close()


def nis_mod():
    from paper_2401_14051_amd import nis
    return nis


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_rgb_query_matches_oracle_per_channel(ctx, prec, tol):
    print("rgb query %s" % prec, flush=True)
    d, pts, dirs = small_points(extra_random=100)
    s = Scene(ctx, d, (0.2, -0.5, 0.8))
    params = weights.he_init(128, 6, seed=1, bias_scale=0.05)
    ctx.set_weights(params)
    ctx.set_precision(prec)
    ctx.set_albedo_rgb(s.mid, RGB)
    L = ctx.query_rgb(s.mid, pts, dirs)
    assert L.shape == (pts.shape[0], 3)
    for c in range(3):
        s.albedo = RGB[c]
        ref = s.oracle_query(params, pts, dirs)["L"]
        err = rel_l2(L[:, c], ref)
        print("rgb query %s channel %d rel-L2 %.3e" % (prec, c, err), flush=True)
        assert err <= tol
    s.close()
    ctx.set_precision("fp32")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_rgb_channels_equal_grey_queries(ctx, prec):
    """Channel c of an RGB query equals the one-channel query with albedo_c,
    on the host and the device entry points; a grey medium's RGB query is
    three copies of its one-channel query."""
    print("rgb identity %s" % prec, flush=True)
    nis = nis_mod()
    d, pts, dirs = small_points(extra_random=100)
    s = Scene(ctx, d, (-0.7, 0.2, 0.4), albedo=0.8)
    ctx.set_weights(weights.he_init(128, 6, seed=2, bias_scale=0.05))
    set_precision(ctx, prec, s.mid, pts, dirs)
    grey = ctx.query(s.mid, pts, dirs)
    L3 = ctx.query_rgb(s.mid, pts, dirs)
    for c in range(3):
        np.testing.assert_array_equal(L3[:, c], grey)
    ctx.set_albedo_rgb(s.mid, RGB)
    L = ctx.query_rgb(s.mid, pts, dirs)
    out = torch.empty(pts.shape[0], 3, dtype=torch.float32, device="cuda")
    ctx.query_rgb_device(s.mid, dev(pts), dev(dirs), out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), L)
    # the one-channel calls refuse a coloured medium
    with pytest.raises(nis.NisError) as e:
        ctx.query(s.mid, pts, dirs)
    assert e.value.code == nis.NIS_E_STATE
    for c in range(3):
        ctx.set_medium_params(s.mid, 8.0, RGB[c], 0.85)
        np.testing.assert_array_equal(L[:, c], ctx.query(s.mid, pts, dirs))
    # three equal channels make the medium grey again
    ctx.set_albedo_rgb(s.mid, (0.8, 0.8, 0.8))
    np.testing.assert_array_equal(ctx.query(s.mid, pts, dirs), grey)
    s.close()
    ctx.set_precision("fp32")


def test_rgb_query_in_several_passes(ctx):
    """A device query of more points than one pass holds (2^21): each channel
    still equals the one-channel query at its albedo, bit for bit."""
    print("rgb multi-pass", flush=True)
    d, _, _ = small_points(extra_random=10)
    s = Scene(ctx, d, (0.3, 0.9, 0.3))
    ctx.set_weights(weights.he_init(64, 4, seed=6, bias_scale=0.05))
    ctx.set_precision("bf16")
    n = (1 << 21) + 1000
    p, q = camera.random_points(n, seed=21, lo=-0.1, hi=1.1)
    tp, tq = dev(p), dev(q)
    ctx.set_albedo_rgb(s.mid, RGB)
    out = torch.empty(n, 3, dtype=torch.float32, device="cuda")
    ctx.query_rgb_device(s.mid, tp, tq, out)
    one = torch.empty(n, dtype=torch.float32, device="cuda")
    for c in range(3):
        ctx.set_medium_params(s.mid, 8.0, RGB[c], 0.85)
        ctx.query_device(s.mid, tp, tq, one)
        torch.cuda.synchronize()
        assert torch.equal(out[:, c], one), c
    s.close()
    ctx.set_precision("fp32")


def test_rgb_render_small_workload(ctx):
    """FP32 RGB frame of the 64^2 orthographic workload against the oracle per
    channel; a grey medium's RGB frame is three copies of its grey frame."""
    print("rgb render", flush=True)
    nis = nis_mod()
    w = configs.SMALL
    d = w.density()
    params = w.params()
    ctx.set_weights(params)
    ctx.set_precision("fp32")
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    cam = nis.camera(64, 64, vfov_deg=0.0, ortho_z=1.0)
    grey = ctx.render(s.mid, cam, w.point_seed).cpu().numpy()
    img3 = ctx.render_rgb(s.mid, cam, w.point_seed).cpu().numpy()
    assert img3.shape == (64, 64, 3)
    for c in range(3):
        np.testing.assert_array_equal(img3[:, :, c], grey)
    ctx.set_albedo_rgb(s.mid, RGB)
    img = ctx.render_rgb(s.mid, cam, w.point_seed).cpu().numpy().reshape(-1, 3)
    o, dirs = camera.orthographic_rays(64)
    rp, rd, rpix = camera.delta_track(d, w.sigma_t, o, dirs, seed=w.point_seed)
    miss = np.ones(64 * 64, bool)
    miss[rpix] = False
    assert np.all(img[miss] == 0.0)
    for c in range(3):
        s.albedo = RGB[c]
        ref = f32(RGB[c]) * s.oracle_query(params, rp, rd)["L"]
        err = rel_l2(img[rpix, c], ref)
        print("rgb render channel %d rel-L2 %.3e over %d hits" % (c, err, rpix.size), flush=True)
        assert err <= 1e-4
    s.close()


def test_rgb_invalid_arguments(ctx):
    """Albedos out of range are refused; the one-channel calls refuse a
    coloured medium."""
    print("rgb invalid arguments", flush=True)
    nis = nis_mod()
    d, pts, dirs = small_points(extra_random=10)
    s = Scene(ctx, d, (0.2, -0.5, 0.8))
    ctx.set_weights(weights.he_init(16, 3, seed=1))
    for bad in [(1.5, 0.5, 0.5), (0.5, -0.1, 0.5), (0.5, 0.5, float("nan"))]:
        with pytest.raises(nis.NisError) as e:
            ctx.set_albedo_rgb(s.mid, bad)
        assert e.value.code == nis.NIS_E_INVALID
    ctx.set_albedo_rgb(s.mid, RGB)
    cam = nis.camera(16, 16, vfov_deg=0.0, ortho_z=1.0)
    with pytest.raises(nis.NisError) as e:
        ctx.render(s.mid, cam, 0)
    assert e.value.code == nis.NIS_E_STATE
    # the RGB calls work on it
    assert ctx.query_rgb(s.mid, pts, dirs).shape == (pts.shape[0], 3)
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_server_renders_coloured_media_in_rgb(ctx, prec):
    """Frames of a coloured medium through the frame server, in a mix with
    grey frames: each equals the synchronous render (RGB or grey) bit for bit."""
    print("server rgb %s" % prec, flush=True)
    nis = nis_mod()
    from workloads import medium
    ctx.set_weights(weights.he_init(64, 4, seed=4, bias_scale=0.05))
    ctx.set_precision(prec)
    grey = ctx.load_medium(medium.fbm_cloud(32, seed=1), 8.0, 0.9, 0.8)
    col = ctx.load_medium(medium.fbm_cloud(32, seed=2), 8.0, 0.9, 0.8)
    ctx.set_albedo_rgb(col, RGB)
    cams = [nis.camera(96, 40, 40.0, eye=(1.6, 0.7, 1.2)), nis.camera(64, 64, 35.0, eye=(0.4, 1.8, 0.9))]
    reqs = [(col, cams[0], (0.3, 0.9, 0.3), 0.85, 1), (grey, cams[1], (-0.5, 0.4, 0.7), 0.6, 2),
            (col, cams[1], (0.2, -0.6, 0.7), 0.3, 3), (grey, cams[0], (0.3, 0.9, 0.3), 0.9, 4)]
    ctx.server_start(1 << 32, prec, max_inflight=3)
    try:
        fids = [ctx.submit(m, cam, l, g=g, seed=sd) for m, cam, l, g, sd in reqs]
        imgs = []
        for fid in fids:
            r = ctx.wait(fid)
            imgs.append((r.channels, ctx.frame_image(r).cpu().numpy()))
            ctx.release(fid)
    finally:
        ctx.server_stop()
    for (m, cam, l, g, sd), (ch, img) in zip(reqs, imgs):
        ctx.set_light(m, l, 1.0)
        ctx.set_medium_params(m, 8.0, 0.9, g)
        if m == col:
            ctx.set_albedo_rgb(m, RGB)
            ref = ctx.render_rgb(m, cam, sd).cpu().numpy()
            assert ch == 3 and img.shape == (cam.height, cam.width, 3)
        else:
            ref = ctx.render(m, cam, sd).cpu().numpy()
            assert ch == 1 and img.shape == (cam.height, cam.width)
        np.testing.assert_array_equal(img, ref)
    ctx.unload_medium(grey)
    ctx.unload_medium(col)
    ctx.set_precision("fp32")

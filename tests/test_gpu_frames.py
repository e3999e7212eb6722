"""GPU tests of the frame driver and the frame server, through the C ABI.

Frame points: the device's camera rays and first-collision delta tracking
against ``workloads.camera``, which implements the same definition (the same
SplitMix64 hash, the same flight and acceptance draws) in float64 numpy: the
set of colliding pixels must be identical and the points agree to float32
rounding (2e-6 absolute).  Rendered images: albedo * L at the hit pixels
against the oracle evaluated at the numpy generator's points (fp32 rel-L2
1e-4, bf16 1e-2, as for point queries), exact zeros at the misses.  Server:
every frame is bit-identical whether rendered alone, in a mix of concurrent
requests, or through the synchronous call; admission under a budget that
holds one frame serialises the frames; requests larger than the budget fail
at submission."""

import numpy as np
import pytest
import torch

from gpu_common import Scene, camera, configs, f32, medium, rel_l2, set_precision, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_14051_amd import nis
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = nis.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def frame_density():
    return configs.FRAME.density()


def nis_mod():
    from paper_2401_14051_amd import nis
    return nis


def check_points(ctx, mid, density, sigma_t, cam, origins, dirs, seed):
    pts, dd, pix = ctx.frame_points(mid, cam, seed)
    rp, rd, rpix = camera.delta_track(density, sigma_t, origins, dirs, seed=seed)
    got_pix = pix.cpu().numpy().astype(np.int64)
    assert got_pix.size == rpix.size, (got_pix.size, rpix.size)
    np.testing.assert_array_equal(got_pix, rpix)
    np.testing.assert_allclose(pts.cpu().numpy(), rp, rtol=0, atol=2e-6)
    np.testing.assert_allclose(dd.cpu().numpy(), rd, rtol=0, atol=2e-7)
    return rp, rd, rpix


@pytest.mark.parametrize("seed", [0, 99])
def test_frame_points_orthographic(ctx, seed):
    print("frame points ortho seed=%d" % seed, flush=True)
    nis = nis_mod()
    w = configs.SMALL
    d = w.density()
    mid = ctx.load_medium(d, w.sigma_t, w.albedo, w.g)
    o, dirs = camera.orthographic_rays(64)
    check_points(ctx, mid, d, w.sigma_t, nis.camera(64, 64, vfov_deg=0.0, ortho_z=1.0), o, dirs, seed)
    ctx.unload_medium(mid)


@pytest.mark.parametrize("res,vfov,eye,up", [
    ((480, 270), 45.0, configs.FRAME_EYE, (0.0, 1.0, 0.0)),
    ((200, 100), 60.0, (1.8, 0.9, -0.6), (0.0, 1.0, 0.0)),
    ((77, 131), 30.0, (0.2, -1.1, 0.4), (0.0, 0.0, 1.0)),
])
def test_frame_points_pinhole(ctx, frame_density, res, vfov, eye, up):
    print("frame points pinhole res=%s eye=%s" % (res, eye), flush=True)
    nis = nis_mod()
    w = configs.FRAME
    mid = ctx.load_medium(frame_density, w.sigma_t, w.albedo, w.g)
    o, dirs = camera.pinhole_rays(res[0], res[1], vfov, eye=eye, up=up)
    check_points(ctx, mid, frame_density, w.sigma_t, nis.camera(res[0], res[1], vfov, eye=eye, up=up), o,
                 dirs, seed=5)
    ctx.unload_medium(mid)


def test_frame_points_full_1080p(ctx, frame_density):
    """The 1080p frame of the 256^3 cloud: 1,206,872 collisions, every one
    matching the generator."""
    print("frame points 1080p", flush=True)
    nis = nis_mod()
    w = configs.FRAME
    mid = ctx.load_medium(frame_density, w.sigma_t, w.albedo, w.g)
    o, dirs = w.rays()
    rp, _, _ = check_points(ctx, mid, frame_density, w.sigma_t, nis.camera(1920, 1080, 45.0, eye=w.eye), o,
                            dirs, seed=w.point_seed)
    assert rp.shape[0] == 1206872
    ctx.unload_medium(mid)


def test_frame_points_degenerate(ctx):
    """An empty medium, a camera looking away from the cube and a single
    pixel."""
    print("frame points degenerate", flush=True)
    nis = nis_mod()
    empty = ctx.load_medium(np.zeros((8, 8, 8), np.float32), 8.0, 0.9, 0.5)
    pts, _, _ = ctx.frame_points(empty, nis.camera(32, 16), 0)
    assert pts.shape[0] == 0
    d = medium.fbm_cloud(16, seed=2)
    mid = ctx.load_medium(d, 8.0, 0.9, 0.5)
    away = nis.camera(32, 16, 40.0, eye=(0.5, 0.5, 2.0), target=(0.5, 0.5, 3.0))
    pts, _, _ = ctx.frame_points(mid, away, 0)
    assert pts.shape[0] == 0
    o, dirs = camera.pinhole_rays(1, 1, 20.0, eye=(0.5, 0.5, 2.0))
    check_points(ctx, mid, d, 8.0, nis.camera(1, 1, 20.0), o, dirs, seed=3)
    ctx.unload_medium(mid)
    ctx.unload_medium(empty)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_render_small_workload(ctx, prec, tol):
    print("render small %s" % prec, flush=True)
    nis = nis_mod()
    w = configs.SMALL
    d = w.density()
    params = w.params()
    ctx.set_weights(params)
    ctx.set_precision(prec)
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    o, dirs = camera.orthographic_rays(64)
    rp, rd, rpix = camera.delta_track(d, w.sigma_t, o, dirs, seed=w.point_seed)
    img = ctx.render(s.mid, nis.camera(64, 64, vfov_deg=0.0, ortho_z=1.0), w.point_seed).cpu().numpy().ravel()
    L = s.oracle_query(params, rp, rd)["L"]
    ref = np.zeros(64 * 64)
    ref[rpix] = f32(w.albedo) * L
    miss = np.ones(64 * 64, bool)
    miss[rpix] = False
    assert np.all(img[miss] == 0.0)
    err = rel_l2(img[rpix], ref[rpix])
    print("render small %s rel-L2 %.3e over %d hits" % (prec, err, rpix.size), flush=True)
    assert err <= tol
    s.close()
    ctx.set_precision("fp32")


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_render_1080p_sampled(ctx, frame_density, prec, tol):
    """The 1080p frame in the launch configuration the benchmark times,
    checked against the oracle at 512 sampled hit pixels."""
    print("render 1080p %s" % prec, flush=True)
    nis = nis_mod()
    w = configs.FRAME
    params = w.params()
    ctx.set_weights(params)
    ctx.set_precision(prec)
    s = Scene(ctx, frame_density, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    o, dirs = w.rays()
    rp, rd, rpix = camera.delta_track(frame_density, w.sigma_t, o, dirs, seed=w.point_seed)
    img = ctx.render(s.mid, nis.camera(1920, 1080, 45.0, eye=w.eye), w.point_seed).cpu().numpy().ravel()
    miss = np.ones(img.size, bool)
    miss[rpix] = False
    assert np.all(img[miss] == 0.0)
    pick = np.random.default_rng(11).choice(rpix.size, 512, replace=False)
    L = s.oracle_query(params, rp[pick], rd[pick])["L"]
    err = rel_l2(img[rpix[pick]], f32(w.albedo) * L)
    print("render 1080p %s rel-L2 %.3e" % (prec, err), flush=True)
    assert err <= tol
    s.close()
    ctx.set_precision("fp32")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_render_equals_query_of_frame_points(ctx, prec):
    """A rendered frame walks its collisions in bands of rows, which changes
    only their order: its image equals, bit for bit, the query of the
    pixel-ordered collisions of nis_frame_points scattered to their pixels
    (a camera whose last band of rows is partial)."""
    print("render vs frame points %s" % prec, flush=True)
    nis = nis_mod()
    d = medium.fbm_cloud(32, seed=5)
    mid = ctx.load_medium(d, 8.0, 0.9, 0.7)
    ctx.set_light(mid, (0.3, 0.9, 0.3), 1.0)
    ctx.set_weights(weights.he_init(64, 4, seed=3, bias_scale=0.05))
    cp, cd = camera.random_points(2048, seed=9, lo=0.0, hi=1.0)
    set_precision(ctx, prec, mid, cp, cd)
    cam = nis.camera(101, 43, 40.0, eye=(1.6, 0.7, 1.2))
    img = ctx.render(mid, cam, 7).cpu().numpy().ravel()
    pts, dirs, pix = ctx.frame_points(mid, cam, 7)
    L = torch.empty(pts.shape[0], dtype=torch.float32, device="cuda")
    ctx.query_device(mid, pts.contiguous(), dirs.contiguous(), L)
    torch.cuda.synchronize()
    ctx.set_precision("fp32")
    ref = np.zeros(101 * 43, np.float32)
    ref[pix.cpu().numpy()] = np.float32(0.9) * L.cpu().numpy()
    assert pts.shape[0] > 500
    np.testing.assert_array_equal(img, ref)
    ctx.unload_medium(mid)


# ---- frame server ---------------------------------------------------------------

def _requests(m32, m64):
    nis = nis_mod()
    return [
        (m32, nis.camera(64, 64, vfov_deg=0.0), (0.3, 0.9, 0.3), 1.0, 0.85, 0),
        (m64, nis.camera(96, 80, 40.0, eye=(0.5, 0.5, 1.8)), (-0.7, 0.2, 0.4), 2.0, 0.5, 7),
        (m32, nis.camera(128, 72, 45.0, eye=(1.7, 0.6, 0.9)), (0.3, 0.9, 0.3), 1.0, 0.95, 3),
        (m64, nis.camera(50, 50, vfov_deg=0.0, ortho_z=1.2), (0.0, -1.0, 0.0), 0.5, 0.0, 11),
        (m32, nis.camera(64, 64, vfov_deg=0.0), (0.3, 0.9, 0.3), 1.0, 0.6, 1),
        (m64, nis.camera(33, 17, 60.0, eye=(0.5, 1.9, 0.5), up=(0.0, 0.0, 1.0)), (1.0, 1.0, 1.0), 1.0, 0.3, 5),
    ]


def _serve(ctx, reqs, max_inflight, budget=1 << 32, precision="bf16", batch_gather=False):
    ctx.server_start(budget, precision, max_inflight, batch_gather=batch_gather)
    try:
        ids = [ctx.submit(m, cam, l, rad, g, seed) for m, cam, l, rad, g, seed in reqs]
        out = []
        for fid in ids:
            r = ctx.wait(fid)
            assert r.status == 0, r.status
            out.append((ctx.frame_image(r).cpu().numpy(), r.n_points, (r.t_submit, r.t_start, r.t_done)))
            ctx.release(fid)
        return out
    finally:
        ctx.server_stop()


def test_server_frames_alone_and_in_a_mix_are_identical(ctx):
    print("server alone vs mix", flush=True)
    w = configs.SMALL
    ctx.set_weights(w.params())
    m32 = ctx.load_medium(w.density(), 8.0, 0.99, 0.85)
    m64 = ctx.load_medium(medium.fbm_cloud(64, seed=4), 6.0, 0.95, 0.85)
    reqs = _requests(m32, m64)
    alone = [_serve(ctx, [r], 1)[0] for r in reqs]
    mix = _serve(ctx, reqs, 4)
    for (a, na, _), (b, nb, _) in zip(alone, mix):
        assert na == nb
        np.testing.assert_array_equal(a, b)
    # the synchronous call renders the same frames
    ctx.set_precision("bf16")
    for (m, cam, l, rad, g, seed), (a, na, _) in zip(reqs, alone):
        sig, alb = (8.0, 0.99) if m == m32 else (6.0, 0.95)
        ctx.set_medium_params(m, sig, alb, g)
        ctx.set_light(m, l, rad)
        img = ctx.render(m, cam, seed).cpu().numpy()
        np.testing.assert_array_equal(img, a)
        assert np.count_nonzero(img) <= na
    ctx.set_precision("fp32")
    ctx.unload_medium(m64)
    ctx.unload_medium(m32)


@pytest.mark.parametrize("precision", ["bf16", "fp32", "fp8"])
def test_server_batch_gather_equals_frames_alone(ctx, precision):
    """With batch_gather, the frames admitted together share one gather
    launch; each image equals, bit for bit, the frame served alone without
    batching.  The mix includes volume phases and a frame too large to batch
    (1500 x 1500 pixels, more than 2^21), which runs on its own."""
    print("server batch gather %s" % precision, flush=True)
    nis = nis_mod()
    w = configs.SMALL
    ctx.set_weights(w.params())
    m32 = ctx.load_medium(w.density(), 8.0, 0.99, 0.85)
    m64 = ctx.load_medium(medium.fbm_cloud(64, seed=4), 6.0, 0.95, 0.85)
    ctx.set_volume_phase(m64, True)
    if precision == "fp8":
        p, d = camera.random_points(4096, seed=3)
        ctx.set_light(m32, (0.3, 0.9, 0.3), 1.0)
        ctx.calibrate_fp8(m32, torch.from_numpy(p).cuda(), torch.from_numpy(d).cuda())
    reqs = _requests(m32, m64) + [(m32, nis.camera(1500, 1500, 30.0, eye=(0.5, 0.5, 2.5)), (0.2, 0.9, -0.3),
                                   1.0, 0.8, 9)]
    alone = [_serve(ctx, [r], 1, budget=1 << 36, precision=precision)[0] for r in reqs]
    for inflight in (4, 7):
        mix = _serve(ctx, reqs, inflight, budget=1 << 36, precision=precision, batch_gather=True)
        for (a, na, _), (b, nb, _) in zip(alone, mix):
            assert na == nb
            np.testing.assert_array_equal(a, b)
    ctx.unload_medium(m64)
    ctx.unload_medium(m32)


def test_server_admission_under_a_one_frame_budget(ctx):
    """With room for one frame only, each frame is admitted after the previous
    one was released, and every frame still completes."""
    print("server one-frame budget", flush=True)
    nis = nis_mod()
    w = configs.SMALL
    ctx.set_weights(w.params())
    m = ctx.load_medium(w.density(), 8.0, 0.99, 0.85)
    cam = nis.camera(64, 64, vfov_deg=0.0)
    reqs = [(m, cam, (0.3, 0.9, 0.3), 1.0, 0.85, s) for s in range(4)]
    free = _serve(ctx, reqs, 4)
    # room for one frame and half of another
    need = ctx.frame_memory(m, cam, (0.3, 0.9, 0.3), "bf16")
    tight = _serve(ctx, reqs, 4, budget=need + need // 2)
    for (a, na, _), (b, nb, _) in zip(free, tight):
        assert na == nb
        np.testing.assert_array_equal(a, b)
    times = [t for _, _, t in tight]
    for prev, nxt in zip(times, times[1:]):
        assert nxt[1] >= prev[2], (prev, nxt)
    ctx.server_start(1 << 20, "bf16", 2)
    try:
        with pytest.raises(nis.NisError) as e:
            ctx.submit(m, nis.camera(1920, 1080, 45.0), (0.3, 0.9, 0.3))
        assert e.value.code == nis.NIS_E_NOMEM
    finally:
        ctx.server_stop()
    ctx.unload_medium(m)


def test_server_state_errors(ctx):
    print("server errors", flush=True)
    nis = nis_mod()
    w = configs.SMALL
    ctx.set_weights(w.params())
    m = ctx.load_medium(w.density(), 8.0, 0.99, 0.85)
    cam = nis.camera(16, 16, vfov_deg=0.0)
    with pytest.raises(nis.NisError) as e:
        ctx.submit(m, cam, (0.3, 0.9, 0.3))
    assert e.value.code == nis.NIS_E_STATE
    with pytest.raises(nis.NisError) as e:
        ctx.server_stop()
    assert e.value.code == nis.NIS_E_STATE
    ctx.server_start(1 << 30, "fp32", 2)
    try:
        with pytest.raises(nis.NisError) as e:
            ctx.server_start(1 << 30, "fp32", 2)
        assert e.value.code == nis.NIS_E_STATE
        with pytest.raises(nis.NisError) as e:
            ctx.set_weights(w.params())
        assert e.value.code == nis.NIS_E_STATE
        with pytest.raises(nis.NisError) as e:
            ctx.unload_medium(m)
        assert e.value.code == nis.NIS_E_STATE
        for bad in [dict(g=1.0), dict(light_dir=(0.0, 0.0, 0.0)), dict(medium=12345)]:
            args = dict(medium=m, cam=cam, light_dir=(0.3, 0.9, 0.3), g=0.5)
            args.update(bad)
            with pytest.raises(nis.NisError) as e:
                ctx.submit(**args)
            assert e.value.code in (nis.NIS_E_INVALID, nis.NIS_E_STATE)
        with pytest.raises(nis.NisError) as e:
            ctx.submit(m, nis.camera(0, 16, vfov_deg=0.0), (0.3, 0.9, 0.3))
        assert e.value.code == nis.NIS_E_INVALID
        with pytest.raises(nis.NisError) as e:
            ctx.poll(987654)
        assert e.value.code == nis.NIS_E_INVALID
        fid = ctx.submit(m, cam, (0.3, 0.9, 0.3), seed=2)
        r = ctx.wait(fid)
        assert r.status == 0 and r.t_submit <= r.t_start <= r.t_done
        assert ctx.poll(fid).status == 0
        ctx.release(fid)
        with pytest.raises(nis.NisError):
            ctx.release(fid)
    finally:
        ctx.server_stop()
    ctx.unload_medium(m)


# ---- the large workload -----------------------------------------------------------

@pytest.fixture(scope="module")
def large_scene(ctx):
    """The large workload (512^3, 4K) loaded on both sides, and the generator's
    collisions of 4096 seeded pixels of its frame."""
    w = configs.LARGE
    d = w.density()
    s = Scene(ctx, d, w.light, w.sigma_t, w.albedo, w.g, w.radiance)
    o, dirs = w.rays()
    pick = np.sort(np.random.default_rng(13).choice(o.shape[0], 4096, replace=False))
    rp, rd, rpix = camera.delta_track(d, w.sigma_t, o[pick], dirs[pick], seed=w.point_seed, pixels=pick)
    yield s, pick, rp, rd, rpix
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_render_4k_large_sampled(ctx, large_scene, prec, tol):
    """The large workload's 4K frame of the 512^3 cloud, checked against the
    oracle at the hits among 4096 sampled pixels; the sampled misses are
    exactly zero."""
    print("render 4K large %s" % prec, flush=True)
    nis = nis_mod()
    w = configs.LARGE
    s, pick, rp, rd, rpix = large_scene
    params = w.params()
    ctx.set_weights(params)
    ctx.set_precision(prec)
    img = ctx.render(s.mid, nis.camera(3840, 2160, 45.0, eye=w.eye), w.point_seed).cpu().numpy().ravel()
    ctx.set_precision("fp32")
    miss = np.setdiff1d(pick, rpix)
    assert np.all(img[miss] == 0.0)
    assert rpix.size > 1000
    L = s.oracle_query(params, rp, rd)["L"]
    err = rel_l2(img[rpix], f32(w.albedo) * L)
    print("render 4K large %s rel-L2 %.3e over %d hits" % (prec, err, rpix.size), flush=True)
    assert err <= tol

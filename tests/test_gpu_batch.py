"""Several queries in one launch (nis_query_batch): every query's radiance
equals, bit for bit, the single device query of the same points, at every
precision, over media of different sizes, lights (one dominated by x) and
phases (two lobes; volume phases), ragged and empty queries, a medium listed
twice; and the batch's error paths."""

import numpy as np
import pytest
import torch

from gpu_common import weights
from workloads import camera, medium

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2401_14051_amd import nis
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = nis.Context(0)
    ctx.set_weights(weights.he_init(64, 4, seed=3, bias_scale=0.05))
    a = ctx.load_medium(medium.fbm_cloud(32, seed=5), 8.0, 0.99, 0.85)
    ctx.set_light(a, (0.3, 0.9, 0.3), 1.0)
    b = ctx.load_medium(medium.fbm_cloud(16, seed=6), 6.0, 0.9, 0.5)
    ctx.set_light(b, (-0.7, 0.2, 0.4), 2.0)
    ctx.set_phase_lobes(b, [(0.7, 0.8), (0.3, -0.4)])
    c = ctx.load_medium(medium.fbm_cloud(64, seed=7), 10.0, 0.95, 0.7)
    ctx.set_light(c, (1.0, 0.2, -0.3), 1.5)
    ctx.set_volume_phase(c, True)
    yield nis, ctx, (a, b, c)
    ctx.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def queries(mids, sizes, seed=21):
    out = []
    for i, (m, n) in enumerate(zip(mids, sizes)):
        p, d = camera.random_points(max(n, 1), seed=seed + i, lo=-0.1, hi=1.1)
        out.append((m, dev(p[:n]), dev(d[:n])))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_batch_equals_single_queries(setup, prec):
    nis, ctx, (a, b, c) = setup
    qs = queries([a, b, c, a, b], [4129, 777, 5000, 1, 0])
    if prec == "fp8":
        ctx.calibrate_fp8(a, qs[0][1], qs[0][2])
    ctx.set_precision(prec)
    single = []
    for m, p, d in qs:
        o = torch.full((p.shape[0],), -1.0, dtype=torch.float32, device="cuda")
        if p.shape[0]:
            ctx.query_device(m, p, d, o)
        single.append(o)
    batch = [torch.full((p.shape[0],), -2.0, dtype=torch.float32, device="cuda") for _, p, _ in qs]
    ctx.query_batch([(m, p, d, o) for (m, p, d), o in zip(qs, batch)])
    torch.cuda.synchronize()
    ctx.set_precision("fp32")
    for s, t in zip(single, batch):
        np.testing.assert_array_equal(t.cpu().numpy(), s.cpu().numpy())
    assert np.all(np.isfinite(batch[2].cpu().numpy()))


def test_batch_of_many_small_queries(setup):
    """64 queries (the most a batch holds), every workgroup range in use."""
    nis, ctx, (a, b, c) = setup
    ctx.set_precision("bf16")
    qs = queries([(a, b, c)[i % 3] for i in range(64)], [(37 * i) % 301 + 1 for i in range(64)], seed=100)
    batch = [torch.empty(p.shape[0], dtype=torch.float32, device="cuda") for _, p, _ in qs]
    ctx.query_batch([(m, p, d, o) for (m, p, d), o in zip(qs, batch)])
    for (m, p, d), t in zip(qs, batch):
        o = torch.empty(p.shape[0], dtype=torch.float32, device="cuda")
        ctx.query_device(m, p, d, o)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(t.cpu().numpy(), o.cpu().numpy())
    ctx.set_precision("fp32")


def test_batch_errors(setup):
    nis, ctx, (a, b, c) = setup
    qs = queries([a], [10])
    o = torch.empty(10, dtype=torch.float32, device="cuda")
    with pytest.raises(nis.NisError) as e:
        ctx.query_batch([])
    assert e.value.code == nis.NIS_E_INVALID
    with pytest.raises(nis.NisError) as e:
        ctx.query_batch([(a, qs[0][1], qs[0][2], o)] * 65)
    assert e.value.code == nis.NIS_E_INVALID
    with pytest.raises(nis.NisError) as e:
        ctx.query_batch([(12345, qs[0][1], qs[0][2], o)])
    assert e.value.code == nis.NIS_E_STATE
    ctx.set_templates("paper")
    with pytest.raises(nis.NisError) as e:
        ctx.query_batch([(a, qs[0][1], qs[0][2], o)])
    assert e.value.code == nis.NIS_E_UNSUPPORTED
    ctx.set_templates("lattice")
    rgb = ctx.load_medium(medium.fbm_cloud(8, seed=9), 8.0, 0.9, 0.5)
    ctx.set_albedo_rgb(rgb, (0.9, 0.8, 0.7))
    ctx.set_light(rgb, (0.3, 0.9, 0.3), 1.0)
    with pytest.raises(nis.NisError) as e:
        ctx.query_batch([(rgb, qs[0][1], qs[0][2], o)])
    assert e.value.code == nis.NIS_E_STATE
    ctx.unload_medium(rgb)

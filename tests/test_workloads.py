"""Host-side input generators: tracking a subset of a frame's rays gives the
same collisions as tracking the whole frame (the large workload's parity test
tracks a sample of its pixels only)."""

import numpy as np

from workloads import camera, configs


def test_delta_track_subset_equals_full_frame():
    w = configs.SMALL
    d = w.density()
    o, dirs = w.rays()
    fp, fd, fpix = camera.delta_track(d, w.sigma_t, o, dirs, seed=w.point_seed)
    pick = np.sort(np.random.default_rng(3).choice(o.shape[0], 700, replace=False))
    sp, sd, spix = camera.delta_track(d, w.sigma_t, o[pick], dirs[pick], seed=w.point_seed, pixels=pick)
    want = np.isin(fpix, pick)
    np.testing.assert_array_equal(spix, fpix[want])
    np.testing.assert_array_equal(sp, fp[want])
    np.testing.assert_array_equal(sd, fd[want])
    assert spix.size > 100

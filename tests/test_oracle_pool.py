"""The GPU tests render large pixel sets with the oracle in a pool of
processes; the pooled result must equal the single-process oracle exactly
(same pixels, same arithmetic, only split into chunks)."""

import numpy as np

import gpu_helpers
from helpers import oracle_workload
from oracle import raycast as orc
from paper_2204_11762_amd import workloads as wl


def test_pooled_oracle_equals_direct():
    wk = wl.c1()
    pix = np.arange(128 * 128)
    assert len(pix) >= gpu_helpers.POOL_MIN_PIXELS
    pooled = gpu_helpers.oracle_on_pixels(wk, pix)
    M, cam, tf, prm = oracle_workload(wk)
    direct = orc.render_pixels(M, cam, tf, prm, pix)
    np.testing.assert_array_equal(pooled.rgba, direct.rgba)
    np.testing.assert_array_equal(pooled.samples, direct.samples)
    np.testing.assert_array_equal(pooled.n_nominal, direct.n_nominal)
    np.testing.assert_array_equal(pooled.near_threshold, direct.near_threshold)

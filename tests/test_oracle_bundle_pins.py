"""Pins of the oracle's dithered orbit bundles (Sec. 2.2.1): n realisations
per initial condition on a box of 0.1 kpc in position and 5% of the local
circular speed in velocity, consecutive in the library, and a bundle's row of
the orbit matrix the mean of its realisations' rows."""
import numpy as np
import pytest

import workloads as W
from oracle import ics as I


def test_zero_deviates_and_corners():
    rng = np.random.default_rng(1)
    ics = rng.normal(0, 100, (6, 5))
    vc = rng.uniform(100, 250, 5)
    out = I.dither(ics, vc, np.zeros((4, 6, 5)), 0.1, 0.05)
    assert np.array_equal(out, np.repeat(ics, 4, axis=1))
    corners = np.where(rng.random((4, 6, 5)) < 0.5, -0.5, 0.5)
    out = I.dither(ics, vc, corners, 0.1, 0.05)
    d = out - np.repeat(ics, 4, axis=1)
    assert np.allclose(np.abs(d[:3]), 0.05, rtol=0, atol=1e-12)
    assert np.allclose(np.abs(d[3:]), 0.025 * np.repeat(vc, 4)[None, :], rtol=1e-12, atol=1e-12)


def test_deviates_stay_in_the_box():
    u = W.dither_deviates(4, 1000, seed=3)
    assert u.min() >= -0.5 and u.max() < 0.5 and abs(u.mean()) < 0.01


def test_bundle_means_and_normalisation():
    rng = np.random.default_rng(2)
    A = rng.random((40, 17))
    A /= A.sum(1, keepdims=True)
    B = I.bundle_rows(A, 4)
    assert B.shape == (10, 17)
    assert np.allclose(B, A.reshape(10, 4, 17).mean(1), rtol=1e-15, atol=0)
    assert np.allclose(B.sum(1), 1.0, rtol=1e-14)
    same = I.bundle_rows(np.repeat(A[:10], 4, axis=0), 4)
    assert np.allclose(same, A[:10], rtol=2e-16, atol=0)
    assert np.array_equal(I.bundle_rows(A, 1), A)

"""Seeded synthetic inputs: determinism and the stated statistics."""
import math

import numpy as np

import workloads as W


def test_blobs_seeded_and_mean_free():
    a = W.gaussian_blobs(32, 16, seed=2).rho
    b = W.gaussian_blobs(32, 16, seed=2).rho
    assert np.array_equal(a, b)
    assert abs(a.mean()) < 1e-12
    assert not np.array_equal(a, W.gaussian_blobs(32, 16, seed=3).rho)


def test_blobs_periodic_minimum_image():
    # a blob near a corner wraps around: the field is smooth across the boundary
    rho = W.gaussian_blobs(64, 1, seed=0, sigma_range=(0.08, 0.08), subtract_mean=False).rho
    jump_x = np.abs(rho[:, :, 0] - rho[:, :, -1]).max()
    step_x = np.abs(np.diff(rho, axis=2)).max()
    assert jump_x <= step_x * 1.0001


def test_grf_unit_variance_zero_mean_and_spectrum():
    f = W.gaussian_random_field(64, seed=3).rho
    assert abs(f.mean()) < 1e-12 and abs(f.std() - 1.0) < 1e-12
    # power-law slope of the shell-averaged spectrum is about -3
    fh = np.abs(np.fft.rfftn(f)) ** 2
    k = np.fft.fftfreq(64, 1 / 64)
    kr = np.fft.rfftfreq(64, 1 / 64)
    K = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2)
    sel1 = (K > 3.5) & (K < 4.5)
    sel2 = (K > 15.5) & (K < 16.5)
    slope = math.log(fh[sel2].mean() / fh[sel1].mean()) / math.log(16 / 4)
    assert abs(slope + 3.0) < 0.3


def test_batch_sizes():
    ns = W.batch_grid_sizes(seed=4)
    assert len(ns) == 96 and set(ns) == {32, 48, 64, 96, 128}
    assert ns == W.batch_grid_sizes(seed=4)


def test_uniform_sphere_faces_are_point_mass_potential():
    p = W.uniform_sphere(32)
    mass = 4 * math.pi * 0.3 ** 3 / 3
    # x- face centre closest to the axis: (-1, -h/2, -h/2)
    h = 2 / 32
    r = math.sqrt(1 + 2 * (h / 2) ** 2)
    assert abs(p.faces[0][16, 16] + mass / r) < 1e-15
    assert p.rho.sum() > 0 and set(np.unique(p.rho)) == {0.0, 1.0}

"""The seeded input generators produce the workloads they describe."""
import math

import numpy as np

import lbm_inputs as inp


def test_seeded_and_deterministic():
    a = inp.taylor_green(32, 32, 0.1, 0.3, noise=1e-3, seed=5)
    b = inp.taylor_green(32, 32, 0.1, 0.3, noise=1e-3, seed=5)
    c = inp.taylor_green(32, 32, 0.1, 0.3, noise=1e-3, seed=6)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[1], c[1])


def test_taylor_green_noise_statistics():
    rho, ux, uy = inp.taylor_green(256, 256, 0.1, 0.3, noise=1e-3, seed=0)
    clean = inp.taylor_green(256, 256, 0.1, 0.3)
    d = np.concatenate([(ux - clean[1]).ravel(), (uy - clean[2]).ravel()])
    assert abs(d.std() - 1e-3) < 2e-5 and abs(d.mean()) < 1e-5
    assert np.array_equal(rho, clean[0])


def test_turbulence_spectrum_and_rms():
    n = 256
    rho, ux, uy = inp.random_phase_turbulence(n, 4, 64, 0.05, seed=1)
    assert abs(np.sqrt(0.5 * np.mean(ux ** 2 + uy ** 2)) - 0.05) < 1e-15
    assert np.allclose([np.sqrt(np.mean(ux ** 2)), np.sqrt(np.mean(uy ** 2))], 0.05, rtol=0.2)
    k = np.fft.fftfreq(n, 1.0 / n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    K = np.rint(np.sqrt(kx ** 2 + ky ** 2))
    E = np.abs(np.fft.fft2(ux)) ** 2 + np.abs(np.fft.fft2(uy)) ** 2
    assert E[(K < 4) | (K > 64)].sum() < 1e-20 * E.sum()
    div = np.fft.ifft2(1j * kx * np.fft.fft2(ux) + 1j * ky * np.fft.fft2(uy)).real
    assert np.max(np.abs(div)) < 1e-12
    # shell energy ~ K^(-5/3): fit the slope over the band
    shells = np.arange(6, 60)
    Es = np.array([E[K == s].sum() for s in shells])
    slope = np.polyfit(np.log(shells), np.log(Es), 1)[0]
    assert abs(slope + 5.0 / 3.0) < 0.25


def test_double_shear_layer_matches_definition():
    nx, ny = 64, 48
    rho, ux, uy = inp.double_shear_layer(nx, ny, 0.04, 80.0, 0.05)
    y, x = 10, 7
    assert ux[y, x] == 0.04 * math.tanh(80.0 * (y / ny - 0.25))
    y = 40
    assert ux[y, x] == 0.04 * math.tanh(80.0 * (0.75 - y / ny))
    assert uy[y, x] == 0.05 * 0.04 * math.sin(2 * math.pi * (x / nx + 0.25))
    assert np.all(rho == 1.0)


def test_rotated_shear_wave_is_periodic_shear():
    rho, ux, uy = inp.rotated_shear_wave(32, 1e-3, U=0.2)
    assert np.array_equal(ux, uy)
    assert np.allclose(np.roll(ux, 1, axis=(0, 1)), ux)  # constant along (1, 1): pure shear
    assert abs(ux.mean() - 0.2 / math.sqrt(2)) < 1e-15


def test_workloads_cover_the_configurations():
    w = inp.WORKLOADS
    assert (w["tg64"].nx, w["tg64"].steps, w["tg64"].theta) == (64, 1000, 1 / 3)
    assert (w["tg4096"].nx, w["tg4096"].theta, w["tg4096"].nu, w["tg4096"].steps) == (4096, 0.3, 0.005, 2000)
    assert (w["turb8192"].nx, w["turb8192"].nu, w["turb8192"].steps) == (8192, 1e-4, 5000)
    assert (w["shear1024"].nx, w["shear1024"].theta, w["shear1024"].steps) == (1024, 0.4, 500)
    assert (w["dsl16384"].nx, w["dsl16384"].ny, w["dsl16384"].nu) == (16384, 4096, 2e-4)

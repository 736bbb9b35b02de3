"""Pins for two later parts of the FP64 oracle, each against something other
than itself.

Colour from a vector field (Sect. 2.1: colour generated directly from a
vector input field instead of a scalar through a colour map): a single
particle's image against the closed-form kernel times brightness x intensity
x vector; linearity in the vector; equality with a one-entry palette of the
same colour; non-finite vectors drop the particle.

Expected flux (the FP64 conservation check: sum_p E_p kappa_p with kappa_p the
particle's sampled, truncated and clipped kernel): the closed form
kappa -> 1 - exp(-nu^2) for a well-sampled particle, half of it for a
particle centred on the image edge, and the per-pixel sum of the additive
image, which the oracle forms in another order."""
import math

import numpy as np
import pytest

from tests.helpers import axis_camera, flat_look, particles, rel_l2


def _render(R, ps, cam, mode, looks, **kw):
    return R.render(R.Particles(ps), cam, R.params(mode, R.Looks(looks), **kw))


def _vec_look(brightness=1.0):
    return dict(vector=1, brightness=brightness)


def test_vector_colour_single_particle_closed_form(oracle):
    """Pinhole camera on the z axis, 90 deg over 128 px (F = 64 px); a particle
    at (0.5, 0.25, 0) seen from 10 units sits at X = 64 + 3.2, Y = 64 - 1.6
    with rho = 64 h / 10.  Every pixel is beta I v exp(-d^2/sigma^2)/(pi
    sigma^2) inside R = 3 sigma and 0 outside."""
    cam = axis_camera(128, 128, dist=10.0, fov=90.0)
    v = np.array([0.2, 0.55, 0.9], np.float32).astype(np.float64)  # inputs are FP32
    h, I, beta = 0.75, 1.75, 0.625
    ps = particles([[0.5, 0.25, 0.0]], h=h, intensity=I, rgb=v)
    img = _render(oracle, ps, cam, oracle.ADD_RAW, [_vec_look(beta)])
    X, Y = 64.0 + 3.2, 64.0 - 1.6
    rho = 64.0 * h / 10.0
    s2 = (rho / 3.0) ** 2 + 0.25
    jj, ii = np.mgrid[0:128, 0:128]
    d2 = (ii + 0.5 - X) ** 2 + (jj + 0.5 - Y) ** 2
    tau = np.where(d2 <= 9.0 * s2, np.exp(-d2 / s2) / (math.pi * s2), 0.0)
    want = beta * I * v[None, None, :] * tau[:, :, None]
    np.testing.assert_allclose(img, want, rtol=1e-12, atol=1e-15)


def test_vector_colour_is_linear_and_matches_a_one_entry_palette(oracle):
    cam = axis_camera(48, 40, dist=4.0, fov=60.0)
    rng = np.random.Generator(np.random.PCG64(21))
    n = 200
    pts = rng.normal(0, 0.6, size=(n, 3))
    h = rng.uniform(0.02, 0.3, size=n)
    inten = rng.lognormal(0, 0.7, size=n)
    # multiples of 1/64, so that v1 + 2 v2 is exact in the FP32 inputs
    v1 = rng.integers(0, 64, size=(n, 3)) / 64.0
    v2 = rng.integers(0, 64, size=(n, 3)) / 64.0
    img1 = _render(oracle, particles(pts, h, inten, rgb=v1), cam, oracle.ADD_RAW, [_vec_look()])
    img2 = _render(oracle, particles(pts, h, inten, rgb=v2), cam, oracle.ADD_RAW, [_vec_look()])
    img12 = _render(oracle, particles(pts, h, inten, rgb=v1 + 2.0 * v2), cam, oracle.ADD_RAW,
                    [_vec_look()])
    assert rel_l2(img12, img1 + 2.0 * img2) < 1e-13
    # one colour for every particle: the same image as a one-entry palette
    c = np.array([0.3, 0.6, 0.1], np.float32)
    a = _render(oracle, particles(pts, h, inten, rgb=c), cam, oracle.ADD_AEQE, [_vec_look(0.8)])
    b = _render(oracle, particles(pts, h, inten), cam, oracle.ADD_AEQE,
                [flat_look(tuple(c), brightness=0.8)])
    assert rel_l2(a, b) < 1e-15


def test_vector_colour_species_mix_and_non_finite(oracle):
    """Species 0 through a palette, species 1 from its vectors; a particle with
    a NaN component is inactive, the rest are unchanged."""
    cam = axis_camera(40, 40, dist=4.0, fov=60.0)
    pts = [[-0.3, 0.0, 0.0], [0.3, 0.1, 0.0], [0.0, -0.3, 0.0]]
    v = np.array([[0.1, 0.2, 0.3], [0.9, 0.5, 0.1], [np.nan, 0.5, 0.5]], np.float32)
    ps = particles(pts, 0.1, 1.0, 0.5, species=[0, 1, 1], rgb=v)
    looks = [flat_look((1.0, 1.0, 1.0)), _vec_look()]
    P = oracle.Particles(ps)
    prm = oracle.params(oracle.ADD_RAW, oracle.Looks(looks))
    pr = oracle.project(P, cam, prm)
    assert [pr[k].active for k in range(3)] == [1, 1, 0]
    np.testing.assert_allclose(list(pr[1].E), [0.9, 0.5, 0.1], rtol=1e-7)
    np.testing.assert_allclose(list(pr[0].E), [1.0, 1.0, 1.0], rtol=0)
    # without the rgb array a vector-coloured species is an error
    ps.rgb = None
    with pytest.raises(RuntimeError):
        _render(oracle, ps, cam, oracle.ADD_RAW, looks)


def test_expected_flux_single_particle_closed_form(oracle):
    """sigma >= 2 px and nu = 6: the sampled kernel sums to 1 - e^-36 to far
    below 1e-9 (Poisson summation error ~exp(-pi^2 sigma^2)), so the expected
    flux is E (1 - e^-36); with nu = 3 it is E (1 - e^-9) up to the pixelated
    disc edge."""
    cam = axis_camera(256, 256, dist=10.0, fov=90.0)
    ps = particles([[1.0, -0.5, 0.0]], h=0.5, intensity=2.0)  # sigma^2 = 4.80
    look = [flat_look((0.25, 0.5, 1.0))]
    L = oracle.Looks(look)
    E = np.array([0.5, 1.0, 2.0])
    got6 = oracle.expected_flux(oracle.Particles(ps), cam, oracle.params(oracle.ADD_RAW, L, nu=6.0))
    np.testing.assert_allclose(got6, E * (1.0 - math.exp(-36.0)), rtol=1e-9)
    got3 = oracle.expected_flux(oracle.Particles(ps), cam, oracle.params(oracle.ADD_RAW, L))
    np.testing.assert_allclose(got3, E * (1.0 - math.exp(-9.0)), rtol=2e-3)


def test_expected_flux_of_a_particle_on_the_image_edge_is_half(oracle):
    """A particle centred on the left image edge (X = 0): its box is clipped at
    column 0 and, by the mirror symmetry of the sampled kernel about X = 0
    (pixel centres at +-1/2, +-3/2, ...), exactly half of the kernel's sum
    lands inside."""
    cam = axis_camera(128, 128, dist=10.0, fov=90.0)
    ps = particles([[-10.0, 0.25, 0.0]], h=1.2)  # X = 64 - 64 = 0, rho = 7.68 px
    L = oracle.Looks([flat_look()])
    prm = oracle.params(oracle.ADD_RAW, L, nu=6.0)
    got = oracle.expected_flux(oracle.Particles(ps), cam, prm)
    assert oracle.project(oracle.Particles(ps), cam, prm)[0].X == pytest.approx(0.0, abs=1e-12)
    np.testing.assert_allclose(got, 0.5 * (1.0 - math.exp(-36.0)), rtol=1e-9)


def test_expected_flux_equals_the_image_sum(oracle):
    """Many particles, some clipped by the image edges: the per-particle sums
    equal the per-pixel sum of the additive image (both exact in FP64 up to
    rounding order), and a particle's vector colour enters linearly."""
    cam = axis_camera(64, 48, dist=3.0, fov=70.0)
    rng = np.random.Generator(np.random.PCG64(23))
    n = 600
    pts = rng.normal(0, 1.0, size=(n, 3))
    h = rng.uniform(0.02, 0.4, size=n)
    inten = rng.lognormal(0, 0.7, size=n)
    v = rng.uniform(0, 1, size=(n, 3))
    ps = particles(pts, h, inten, rng.uniform(0, 1, size=n), rgb=v,
                   species=(rng.uniform(size=n) < 0.3).astype(np.uint8))
    looks = [dict(rgb=np.linspace(0.1, 1.0, 48).reshape(16, 3), brightness=0.7), _vec_look(1.3)]
    L = oracle.Looks(looks)
    prm = oracle.params(oracle.ADD_RAW, L)
    P = oracle.Particles(ps)
    img = oracle.render(P, cam, prm)
    exp_flux = oracle.expected_flux(P, cam, prm)
    np.testing.assert_allclose(exp_flux, img.reshape(-1, 3).sum(0), rtol=1e-12)
    # sorted mode has no such sum
    with pytest.raises(RuntimeError):
        oracle.expected_flux(P, cam, oracle.params(oracle.SORTED, L))

"""Pins of the oracle's Stage 2 (band, projection, weights) and Stage 4 area.

Each expected value is fixed by mathematics independent of the oracle: a brute-force
lattice count, the normalisation of the cosine weight (eq. cosine-kernel), and the
band-integrated area of a sphere, 4πR²(1 + c₂ε²/R²) with c₂ = 1/3 − 2/π² (every level
set at distance η carries area 4π(R+η)² and the cosine weight has second moment c₂ε²).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1709_08070_amd import synth

C2 = 1.0 / 3.0 - 2.0 / math.pi ** 2


def test_delta_normalisation_and_moments():
    for eps in (0.5, 1.0, 0.3):
        f = lambda t: oracle.delta(t, eps)
        assert integrate.quad(f, -eps, eps, epsabs=0, epsrel=1e-13)[0] == pytest.approx(1.0, rel=1e-12)
        assert integrate.quad(lambda t: t * f(t), -eps, eps)[0] == pytest.approx(0.0, abs=1e-14)
        m2 = integrate.quad(lambda t: t * t * f(t), -eps, eps, epsabs=0, epsrel=1e-13)[0]
        assert m2 == pytest.approx(C2 * eps * eps, rel=1e-11)
        assert oracle.delta(eps, eps) == 0.0 and oracle.delta(-1.5 * eps, eps) == 0.0
        assert oracle.delta(0.0, eps) == pytest.approx(1.0 / eps)


def _sphere(h, centre=(0.0123, 0.0456, 0.0789), R=2.0):
    atoms = synth.born_ion(R, 1.0, centre)
    return oracle.pipeline(atoms, h, ses=False)


@pytest.mark.parametrize("centre,expected", [((0.0, 0.0, 0.0), 3214), ((0.0123, 0.0456, 0.0789), 3281)])
def test_sphere_band_node_count_brute_force(centre, expected):
    h, R, eps = 0.25, 2.0, 0.5
    dims, origin, phi, nodes, gidx, prm = _sphere(h, centre, R)
    # independent count: every lattice point of hℤ³ with −ε < |x − c| − R < ε
    m = int(math.ceil((R + eps) / h)) + 2
    ax = np.arange(-m, m + 1) * h
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    d = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) - R
    assert len(nodes) == int(np.sum((d > -eps) & (d < eps))) == expected


def test_sphere_projection_and_normals():
    h, R = 0.25, 2.0
    c = np.array([0.0123, 0.0456, 0.0789])
    dims, origin, phi, nodes, gidx, prm = _sphere(h)
    rad = np.linalg.norm(nodes[:, :3] - c, axis=1)
    assert np.max(np.abs(rad - R)) < 0.02 * h          # central differences: O(h²) off the sphere
    radial = (nodes[:, :3] - c) / rad[:, None]
    assert np.min(np.sum(radial * nodes[:, 3:6], axis=1)) > 1 - 1e-3
    # band order is the lexicographic grid order
    assert np.all(np.diff(gidx) > 0)


@pytest.mark.parametrize("h", [0.5, 0.25, 0.125])
def test_sphere_area(h):
    R, eps = 2.0, 2 * h
    dims, origin, phi, nodes, gidx, prm = _sphere(h)
    A = oracle.area(nodes, h)
    rel = A / (4 * math.pi * R * R) - 1.0
    assert abs(rel - C2 * eps * eps / (R * R)) < 1e-3


def test_band_weights_and_order_on_globule():
    atoms = synth.globule(60, 11)
    dims, origin, phi, nodes, gidx, prm = oracle.pipeline(atoms, 0.5, ses=False)
    eps = prm[oracle.BAND]
    assert np.all(np.abs(nodes[:, 6]) < eps)
    np.testing.assert_allclose(nodes[:, 7], (1 + np.cos(np.pi * nodes[:, 6] / eps)) / (2 * eps), rtol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(nodes[:, 3:6], axis=1), 1.0, rtol=1e-14)
    # the band is exactly the set −ε < φ < ε
    assert len(nodes) == int(np.sum((phi > -eps) & (phi < eps)))

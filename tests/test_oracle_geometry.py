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


# ------------------------------------------------------- explicit Jacobian and WENO normals
# J = 1 − φΔφ + φ²⟨n, adj(∇²φ) n⟩ (section "Implicit boundary integral methods", with the
# adjugate reading). Fixed independently of the oracle by: a quadratic field, on which the
# central differences are exact and adj(B) = det(B)·B⁻¹ (numpy); the sphere, where J is the
# area ratio (R/ρ)²; the cylinder, where it is R/ρ (one curved direction: the φ² term must
# vanish); and the band-integrated area, which J makes exact up to quadrature error.


def test_jacobian_exact_on_quadratic_field():
    rng = np.random.default_rng(3)
    dims, h = (9, 10, 11), 0.25
    M = rng.normal(size=(3, 3))
    B = M + M.T + 3.0 * np.eye(3)  # symmetric, invertible, not diagonal
    a, c0 = rng.normal(size=3), 0.3
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    X = np.stack([i, j, k], -1).reshape(-1, 3) * h - 1.0
    phi = c0 + X @ a + 0.5 * np.einsum("ni,ij,nj->n", X, B, X)
    adjB = np.linalg.det(B) * np.linalg.inv(B)
    checked = 0
    for node in rng.choice(np.prod(dims), 200, replace=False):
        ii, jj, kk = np.unravel_index(node, dims)
        if min(ii, jj, kk) == 0 or ii == dims[0] - 1 or jj == dims[1] - 1 or kk == dims[2] - 1:
            continue
        g = a + B @ X[node]
        n = g / np.linalg.norm(g)
        f = phi[node]
        want = 1.0 - f * np.trace(B) + f * f * (n @ adjB @ n)
        got = oracle.jacobian(dims, h, phi, node, n)
        assert got == pytest.approx(want, rel=1e-11, abs=1e-11)
        checked += 1
    assert checked > 50


def test_jacobian_sphere_and_cylinder():
    R, c = 2.0, np.array([0.0123, 0.0456, 0.0789])
    errs = []
    for h in (0.25, 0.125):
        dims, origin, phi, nodes, gidx, prm = oracle.pipeline(synth.born_ion(R, 1.0, tuple(c)), h, ses=False,
                                                              jacobian=True)
        J = nodes[:, 7] / np.array([oracle.delta(f, 2 * h) for f in nodes[:, 6]])
        errs.append(np.max(np.abs(J - (R / (R + nodes[:, 6])) ** 2)))
    assert errs[1] < 1e-3 and errs[0] / errs[1] > 4.0  # at least second order
    # cylinder of radius R along z, sampled away from the z ends
    h = 0.125
    dims = (48, 48, 12)
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    x, y = i * h - 3.0 + c[0], j * h - 3.0 + c[1]
    rho = np.sqrt(x * x + y * y)
    phi = (rho - R).reshape(-1)
    sel = np.nonzero((np.abs(phi) < 2 * h) & (k.reshape(-1) == 6))[0]
    worst = 0.0
    for node in sel:
        ii, jj, _ = np.unravel_index(node, dims)
        n = np.array([x[ii, jj, 6], y[ii, jj, 6], 0.0]) / rho[ii, jj, 6]
        worst = max(worst, abs(oracle.jacobian(dims, h, phi, node, n) - R / rho[ii, jj, 6]))
    assert len(sel) > 100 and worst < 1e-3


@pytest.mark.parametrize("h", [0.25, 0.125])
def test_sphere_area_with_explicit_jacobian(h):
    R = 2.0
    dims, origin, phi, nodes, gidx, prm = oracle.pipeline(synth.born_ion(R), h, ses=False, jacobian=True)
    rel = abs(oracle.area(nodes, h) / (4 * math.pi * R * R) - 1.0)
    # J ≡ 1 leaves c₂ε²/R² (8.2e-3 at h = 0.25); the explicit J removes that term
    assert rel < 0.03 * C2 * (2 * h) ** 2 / R ** 2


def test_weno_average_gradient_normals():
    R, c, h = 2.0, np.array([0.0123, 0.0456, 0.0789]), 0.25
    worst = {}
    for gs in (oracle.GRAD_CENTRAL, oracle.GRAD_WENO):
        dims, origin, phi, nodes, gidx, prm = oracle.pipeline(synth.born_ion(R, 1.0, tuple(c)), h, ses=False,
                                                              grad_scheme=gs)
        rad = nodes[:, :3] - c
        radial = rad / np.linalg.norm(rad, axis=1)[:, None]
        worst[gs] = (np.max(np.linalg.norm(nodes[:, 3:6] - radial, axis=1)),
                     np.max(np.abs(np.linalg.norm(rad, axis=1) - R)))
    # fifth-order one-sided derivatives on a smooth distance function: far below the O(h²)
    # of central differences, and the projection lands on the sphere
    assert worst[1][0] < 0.05 * worst[0][0]
    assert worst[1][1] < 1e-8
    # on a quadratic field every WENO candidate stencil is exact, so the average is too
    dims, h = (12, 12, 12), 0.25
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    X = np.stack([i, j, k], -1).reshape(-1, 3) * h
    B = np.array([[1.0, 0.3, -0.2], [0.3, 0.5, 0.1], [-0.2, 0.1, 0.8]])
    a = np.array([0.4, -0.7, 0.2])
    phi = X @ a + 0.5 * np.einsum("ni,ij,nj->n", X, B, X)
    node = np.ravel_multi_index((6, 5, 7), dims)
    m, p = oracle.weno_grad(dims, h, phi, node)
    np.testing.assert_allclose((m + p) / 2, a + B @ X[node], rtol=0, atol=1e-12)


def test_surface_curvature_sphere_and_cylinder():
    """κ1 + κ2 at the projection: 2/R on a sphere (at every band node, both sides of the
    surface), 1/R on a cylinder; second order in h."""
    R, c = 2.0, np.array([0.0123, 0.0456, 0.0789])
    errs = []
    for h in (0.25, 0.125):
        dims, origin, phi, nodes, gidx, prm = oracle.pipeline(synth.born_ion(R, 1.0, tuple(c)), h, ses=False)
        curv = oracle.curvature(dims, h, phi, gidx, nodes)
        errs.append(np.max(np.abs(curv - 2.0 / R)))
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 3.5
    h, dims = 0.125, (48, 48, 12)
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    x, y = i * h - 3.0 + c[0], j * h - 3.0 + c[1]
    rho = np.sqrt(x * x + y * y)
    phi = (rho - R).reshape(-1)
    sel = np.nonzero((np.abs(phi) < 2 * h) & (k.reshape(-1) == 6))[0]
    nrm = [np.array([x.reshape(-1)[q], y.reshape(-1)[q], 0.0]) / rho.reshape(-1)[q] for q in sel]
    nodes = np.zeros((len(sel), 8))
    nodes[:, 3:6] = nrm
    curv = oracle.curvature(dims, h, phi, sel, nodes)
    assert np.max(np.abs(curv - 1.0 / R)) < 1e-3

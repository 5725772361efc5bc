"""Pins of the oracle's operator, right-hand side, GMRES and energy.

Closed forms used (all independent of the oracle's code):
  * Gauss's lemma for the Laplace double layer of a constant density: −1 at an interior
    point, 0 outside, −½ on the surface; with the regularization of the tangent disc of
    radius τ, the on-surface value becomes −½ + ½ sin(θ0/2), sin θ0 = τ/R (the cap
    contribution ∫ −1/(8πR|x−y|) over the cap is −½ sin(θ0/2)).
  * The Kirkwood single-ion solution (single-ion section): on the sphere
    ψ* = q/(4π ε_E (1+κR) R), ψ*_n = −q/(4π ε_I R²), and
    G* = q²/(8πR) (1/(ε_E(1+κR)) − 1/ε_I).
  * For a centred charge and the exact potential, every energy term is the same on the
    sphere, so the IBIM energy equals G* times the band area ratio.
  * GMRES is compared with dense LU of the same matrix.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1709_08070_amd import synth

C2 = 1.0 / 3.0 - 2.0 / math.pi ** 2
R, Q, EI, EE, KAP = 2.0, 1.0, 1.0, 80.0, 0.1257
CENTRE = np.array([0.0123, 0.0456, 0.0789])


def kirkwood_energy(R=R, q=Q, ei=EI, ee=EE, kappa=KAP):
    return q * q / (8 * math.pi * R) * (1.0 / (ee * (1 + kappa * R)) - 1.0 / ei)


@pytest.fixture(scope="module")
def c1():
    atoms = synth.born_ion(R, Q, tuple(CENTRE))
    return (atoms,) + oracle.pipeline(atoms, 0.25, ses=False)


def _double_layer(nodes, target, prm, h):
    """Σ_j h³ ω_j ∂G0(target, y_j)/∂n(y_j): the oracle's K11 with θ1 → 0."""
    p = prm.copy()
    p[oracle.EPS_OUT] = 1e-300
    s = 0.0
    for row in nodes:
        s += oracle.pair(target, [0, 0, 1.0], row[:3], row[3:6], p)[0] * h ** 3 * row[7]
    return s


def test_gauss_lemma_interior_and_exterior(c1):
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    h, eps = 0.25, 0.5
    fac = 1 + C2 * eps * eps / (R * R)
    assert _double_layer(nodes, CENTRE, prm, h) == pytest.approx(-fac, abs=2e-3)
    assert _double_layer(nodes, CENTRE + [0.7, -0.4, 0.3], prm, h) == pytest.approx(-fac, abs=3e-3)
    assert abs(_double_layer(nodes, CENTRE + [3 * R, 0.5, 0.2], prm, h)) < 1e-3


def test_gauss_lemma_on_surface_with_regularization(c1):
    """Row average of λ1·1 + (K11 part) applied to ψ = 1 with θ1 → 0 equals the
    regularized on-surface double layer."""
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    h, eps, tau = 0.25, 0.5, 0.25
    p = prm.copy()
    p[oracle.EPS_OUT] = 1e-300
    n = len(nodes)
    y = oracle.matvec(nodes, p, np.concatenate([np.ones(n), np.zeros(n)]))
    lam1 = 0.5
    dl = y[:n] - lam1
    theta0 = math.asin(tau / R)
    expected = -(1 + C2 * eps * eps / (R * R)) * (0.5 - 0.5 * math.sin(theta0 / 2))
    assert np.mean(dl) == pytest.approx(expected, abs=2e-3)
    assert np.max(np.abs(dl - expected)) < 0.03


def test_rhs_closed_form_on_sphere(c1):
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    n = len(nodes)
    g = oracle.rhs(nodes, atoms, prm)
    rad = np.linalg.norm(nodes[:, :3] - CENTRE, axis=1)
    np.testing.assert_allclose(g[:n], Q / (4 * math.pi * EI * rad), rtol=1e-13)
    np.testing.assert_allclose(g[n:], -Q / (4 * math.pi * EI * rad ** 2) * np.sum(
        (nodes[:, :3] - CENTRE) / rad[:, None] * nodes[:, 3:6], axis=1), rtol=1e-12)


def test_energy_quadrature_of_exact_potential(c1):
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    n, h = len(nodes), 0.25
    psi = Q / (4 * math.pi * EE * (1 + KAP * R) * R)
    psin = -Q / (4 * math.pi * EI * R * R)
    G, _ = oracle.energy(nodes, atoms, prm, np.concatenate([np.full(n, psi), np.full(n, psin)]))
    ratio = oracle.area(nodes, h) / (4 * math.pi * R * R)
    assert G / kirkwood_energy() == pytest.approx(ratio, rel=5e-5)


def test_kirkwood_residual_is_discretization_sized(c1):
    """The exact solution satisfies the discrete system up to the O(τ/R + ε²/R²) error."""
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    n = len(nodes)
    p = np.concatenate([np.full(n, Q / (4 * math.pi * EE * (1 + KAP * R) * R)), np.full(n, -Q / (4 * math.pi * EI * R * R))])
    res = oracle.matvec(nodes, prm, p) - oracle.rhs(nodes, atoms, prm)
    rel = np.linalg.norm(res) / np.linalg.norm(oracle.rhs(nodes, atoms, prm))
    assert 1e-3 < rel < 0.1


def test_gmres_matches_dense_lu(c1):
    atoms, dims, origin, phi, nodes, gidx, prm = c1
    g = oracle.rhs(nodes, atoms, prm)
    A = oracle.dense(nodes, prm)
    x_lu = np.linalg.solve(A, g)
    x, it, rr, ok = oracle.gmres(nodes, prm, g, tol=1e-10)
    assert ok and rr <= 1e-10
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-8
    # dense assembly and the matrix-free operator agree
    v = np.random.default_rng(1).normal(size=2 * len(nodes))
    np.testing.assert_allclose(A @ v, oracle.matvec(nodes, prm, v), rtol=1e-11, atol=1e-11 * np.abs(A @ v).max())


@pytest.mark.parametrize("tau_k,lo,hi", [(1.0, 0.0288, 0.0576), (0.5, 0.0159, 0.0318)])
def test_kirkwood_energy_born_ion(c1, tau_k, lo, hi):
    """C1 Born ion, h = 0.25, ε = 2h: the regularization error model predicts +2.88 %
    (τ = h) and +1.59 % (τ = h/2); accept 1×–2× the model with the model's sign."""
    atoms = c1[0]
    _, _, _, nodes, _, prm = oracle.pipeline(atoms, 0.25, ses=False, tau_k=tau_k)
    g = oracle.rhs(nodes, atoms, prm)
    x, it, rr, ok = oracle.gmres(nodes, prm, g, tol=1e-8)
    assert ok
    G, _ = oracle.energy(nodes, atoms, prm, x)
    err = (G - kirkwood_energy()) / kirkwood_energy()
    assert lo <= err <= hi


@pytest.mark.slow
def test_kirkwood_first_order_convergence():
    atoms = synth.born_ion(R, Q, tuple(CENTRE))
    errs = []
    for h in (0.5, 0.25, 0.125):
        _, _, _, nodes, _, prm = oracle.pipeline(atoms, h, ses=False)
        x, it, rr, ok = oracle.gmres(nodes, prm, oracle.rhs(nodes, atoms, prm), tol=1e-8)
        assert ok
        errs.append((oracle.energy(nodes, atoms, prm, x)[0] - kirkwood_energy()) / kirkwood_energy())
    assert errs[0] > errs[1] > errs[2] > 0
    assert 1.6 < errs[0] / errs[1] < 2.6 and 1.6 < errs[1] / errs[2] < 2.6


def _table2_rows(grid=64):
    """The printed rows of the single-ion table for one grid size."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_single_ion.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            row = [float(v) for v in line.split()]
            if int(row[0]) == grid:
                rows.append(row)
    return rows


@pytest.mark.slow
@pytest.mark.parametrize("row", _table2_rows(), ids=["tau=h", "tau=h/2"])
def test_replays_single_ion_table(row):
    """Replays the paper's 64³ single-ion rows (R = 8.31 Å reading, h = 25/64, ε = 2h,
    GMRES 1e-5). Node count, solution error and area error are reproduced closely; the
    energy error comes out smaller than printed (same order)."""
    _, _, tau_k, dof, _, sol_p, area_p, en_p = row
    Rr, h = 8.31, 25.0 / 64.0
    atoms = synth.born_ion(Rr, 1.0)
    _, _, _, nodes, _, prm = oracle.pipeline(atoms, h, ses=False, tau_k=tau_k)
    n = len(nodes)
    assert abs(n - dof) / dof < 0.01
    x, it, rr, ok = oracle.gmres(nodes, prm, oracle.rhs(nodes, atoms, prm), tol=1e-5)
    assert ok and it <= 8
    ps = 1 / (4 * math.pi * EE * (1 + KAP * Rr) * Rr)
    pn = -1 / (4 * math.pi * EI * Rr * Rr)
    w = nodes[:, 7]
    sol = math.sqrt(np.sum(w * ((x[:n] - ps) ** 2 + (x[n:] - pn) ** 2)) / np.sum(w * (ps ** 2 + pn ** 2)))
    area = abs(oracle.area(nodes, h) / (4 * math.pi * Rr * Rr) - 1)
    G, _ = oracle.energy(nodes, atoms, prm, x)
    en = abs(G / kirkwood_energy(Rr) - 1)
    assert sol == pytest.approx(sol_p, rel=0.1)
    assert area == pytest.approx(area_p, rel=0.15)
    assert 0.4 * en_p < en < 1.2 * en_p


def test_kirkwood_energy_curved_disc_averages(c1):
    """With the curvature-corrected disc averages the regularization error of the Born ion
    drops from first to second order in h (τ = h): under 0.5 % at h = 0.25 against +2.9 %
    with the paper's averages, and about 4× smaller per halving of h."""
    atoms = c1[0]
    errs = {}
    for h in (0.5, 0.25):
        dims, origin, phi, nodes, gidx, prm = oracle.pipeline(atoms, h, ses=False, avg=oracle.AVG_CURVED)
        curv = oracle.curvature(dims, h, phi, gidx, nodes)
        x, it, rr, ok = oracle.gmres(nodes, prm, oracle.rhs(nodes, atoms, prm), tol=1e-9, curv=curv)
        assert ok
        errs[h] = (oracle.energy(nodes, atoms, prm, x)[0] - kirkwood_energy()) / kirkwood_energy()
    assert 0.0 < errs[0.25] < 0.005
    assert errs[0.5] / errs[0.25] > 3.0

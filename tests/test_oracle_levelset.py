"""Pins of the oracle's Stage 1 (level set of the solvent excluded surface).

  * WENO5 one-sided derivatives are exact on linear data and fifth-order on smooth data.
  * The inward eikonal flow φ_t = |∇φ| has the Hopf–Lax solution
    φ(x, t) = max_{|c−x| ≤ t} φ0(c); started from φ_SAS = F − ρ0 and run to t = ρ0 it is the
    signed function of the SES (probe-ball closing). The oracle is compared with a brute-force
    maximum over a dense sample of the ball, for one and for two atoms.
  * The flow has a closed-form transient: from φ0 = (|x−c|² − R²)/(2R) the Hopf–Lax maximum
    is φ(x, t) = ((|x−c| + t)² − R²)/(2R), whose gradient grows in time, so a first-order
    time integrator in place of the third-order TVD Runge–Kutta scheme is off by about 0.1h.
  * A single atom's SES is the atom itself: after the whole Stage 1 the band values equal
    |x − z| − r.
  * A closed shell of atoms around a void larger than the probe: cavity removal deletes the
    inner surface, so no band node projects inside the shell.
  * Reinitialization (eqs. reinit and signum) turns a function that is not a distance
    function into one without moving its zero set: from φ0 = (|x−c|² − R²)/(2R) (zero set the
    sphere of radius R, |∇φ0| = |x−c|/R) it restores |x−c| − R in the band to a small
    fraction of h, |∇φ| to 1, and moves the zero crossings along grid edges by O(h²). The
    same checks fail on the input itself, i.e. on a Stage 1 with the reinitialization left
    out.
  * The whole Stage 1 on two atoms gives the signs of a brute-force probe closing away from
    the surface and a distance function in the band (|∇φ| → 1 at second order in h), which
    the closing function before reinitialization is not (its |∇φ| departs from 1 by about
    0.12 in the re-entrant groove at every h).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1709_08070_amd import synth


def test_weno_exact_on_linear_and_high_order_on_smooth():
    dims, h = (16, 17, 18), 0.1
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    lin = (0.3 * i - 0.7 * j + 1.1 * k).ravel() * h
    node = (8 * dims[1] + 8) * dims[2] + 9
    m, p = oracle.weno_grad(dims, h, lin, node)
    np.testing.assert_allclose(m, [0.3, -0.7, 1.1], rtol=1e-12)
    np.testing.assert_allclose(p, [0.3, -0.7, 1.1], rtol=1e-12)
    errs = []
    for hh in (0.1, 0.05):
        x = (i * hh).ravel()
        f = np.sin(1.3 * x)
        c = 8
        nd = (c * dims[1] + 8) * dims[2] + 9
        m, p = oracle.weno_grad(dims, hh, f, nd)
        errs.append(max(abs(m[0] - 1.3 * math.cos(1.3 * c * hh)), abs(p[0] - 1.3 * math.cos(1.3 * c * hh))))
    assert errs[0] / errs[1] > 20  # at least ~fourth/fifth order


def _hopf_lax_check(atoms, h, n_check, spacing, seed=0):
    rho = 1.4
    dims, origin = oracle.grid(atoms, h, oracle.grid_margin(atoms, h))
    phi0 = oracle.vdw(dims, origin, h, atoms) - rho
    phie = oracle.eikonal(dims, h, phi0, rho)
    idx = np.nonzero(np.abs(phie) < 2 * h)[0]
    sel = np.random.default_rng(seed).choice(idx, n_check, replace=False)
    k = sel % dims[2]
    j = (sel // dims[2]) % dims[1]
    i = sel // (dims[1] * dims[2])
    X = np.column_stack([origin[0] + h * i, origin[1] + h * j, origin[2] + h * k])
    g = np.arange(-rho, rho + 1e-9, spacing)
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    P = P[np.linalg.norm(P, axis=1) <= rho]
    ex = np.empty(len(X))
    for q, x in enumerate(X):
        c = x + P
        F = np.min(np.linalg.norm(c[:, None, :] - atoms[None, :, :3], axis=2) - atoms[None, :, 3], axis=1)
        ex[q] = F.max() - rho
    return phie[sel], ex


def test_eikonal_flow_is_hopf_lax_single_atom():
    atoms = np.array([[0.0123, 0.0456, 0.0789, 1.7, 1.0]])
    num, ex = _hopf_lax_check(atoms, 0.25, 60, 0.05)
    # brute force under-estimates the maximum by at most spacing·√3/2
    assert np.max(np.abs(num - ex)) < 0.2 * 0.25


def test_eikonal_flow_is_hopf_lax_two_atoms():
    atoms = np.array([[-1.1, 0.03, 0.01, 1.6, 0.5], [1.2, -0.02, 0.04, 1.5, -0.5]])
    h = 0.25
    num, ex = _hopf_lax_check(atoms, h, 120, 0.05)
    assert np.max(np.abs(num - ex)) < 0.25 * h
    far = np.abs(ex) > 0.3 * h
    assert np.all(np.sign(num[far]) == np.sign(ex[far]))


def test_eikonal_flow_exact_on_radial_quadratic():
    """Section "Inward eikonal flow": φ_t = |∇φ| from φ0 = (ρ² − R²)/(2R), ρ = |x − c|, has the
    solution ((ρ + t)² − R²)/(2R) (the maximum of φ0 over the t-ball sits at the far end of
    the radius). Checked at t = 1.4 on nodes with 1 < ρ < 2.5, more than 4 Å from the grid
    boundary (the reflected ghosts of the zero-Neumann boundary do not reach them)."""
    h, R, L, t = 0.25, 2.0, 6.5, 1.4
    n = int(round(2 * L / h)) + 1
    g = np.arange(n) * h - L
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    c = (0.0123, 0.0456, 0.0789)
    rho = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2).ravel()
    phi = oracle.eikonal((n, n, n), h, (rho ** 2 - R ** 2) / (2 * R), t)
    m = (rho > 1.0) & (rho < 2.5)
    exact = ((rho + t) ** 2 - R ** 2) / (2 * R)
    assert m.sum() > 3000
    assert np.max(np.abs(phi[m] - exact[m])) < 0.005 * h


def test_single_atom_ses_is_the_atom():
    atoms = np.array([[0.0123, 0.0456, 0.0789, 1.7, 1.0]])
    h = 0.25
    dims, origin, phi, nodes, gidx, prm = oracle.pipeline(atoms, h, ses=True)
    k = gidx % dims[2]
    j = (gidx // dims[2]) % dims[1]
    i = gidx // (dims[1] * dims[2])
    X = np.column_stack([origin[0] + h * i, origin[1] + h * j, origin[2] + h * k])
    exact = np.linalg.norm(X - atoms[0, :3], axis=1) - 1.7
    assert np.max(np.abs(nodes[:, 6] - exact)) < 0.01 * h


def test_cavity_removed_from_closed_shell():
    atoms = synth.shell(6.0, 1.6, 2.2)
    h = 0.5
    prm = oracle.params(h)
    dims, origin = oracle.grid(atoms, h, oracle.grid_margin(atoms, h))
    phi0 = oracle.vdw(dims, origin, h, atoms) - 1.4
    phie = oracle.eikonal(dims, h, phi0, 1.4)
    # the void is solvent-free after the flow: φ > 0 at the centre, unreachable from the boundary
    cidx = np.argmin(np.abs(np.arange(dims[0]) * h + origin[0]))
    cj = np.argmin(np.abs(np.arange(dims[1]) * h + origin[1]))
    ck = np.argmin(np.abs(np.arange(dims[2]) * h + origin[2]))
    c = (cidx * dims[1] + cj) * dims[2] + ck
    assert phie[c] > 0
    phic, outside, nset = oracle.cavity(dims, h, phie, prm[oracle.BAND])
    assert nset > 0 and outside[c] == 0 and phic[c] == -prm[oracle.BAND]
    assert outside[0] == 1
    phi, ncav = oracle.ses(dims, origin, atoms, prm)
    nodes, _ = oracle.band(dims, origin, h, phi, prm[oracle.BAND])
    assert np.min(np.linalg.norm(nodes[:, :3], axis=1)) > 6.0


def test_no_cavity_no_change():
    atoms = np.array([[-1.1, 0.03, 0.01, 1.6, 0.5], [1.2, -0.02, 0.04, 1.5, -0.5]])
    h = 0.5
    dims, origin = oracle.grid(atoms, h, oracle.grid_margin(atoms, h))
    phi0 = oracle.vdw(dims, origin, h, atoms) - 1.4
    phie = oracle.eikonal(dims, h, phi0, 1.4)
    phic, outside, nset = oracle.cavity(dims, h, phie, 2 * h)
    assert nset == 0
    np.testing.assert_array_equal(phic, phie)
    assert np.array_equal(outside.astype(bool), phie > 0)


def _box_sphere(h, R=2.0, c=(0.0123, 0.0456, 0.0789), L=4.0):
    """Cubic grid of spacing h on [−L, L]³ and the distance ρ of every node from c."""
    n = int(round(2 * L / h)) + 1
    g = np.arange(n) * h - L
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    rho = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2).ravel()
    return (n, n, n), rho


def _grad_norm(phi, dims, h):
    """|∇φ| by central differences at interior nodes (NaN on the grid boundary)."""
    p = phi.reshape(dims)
    gx = (p[2:, 1:-1, 1:-1] - p[:-2, 1:-1, 1:-1]) / (2 * h)
    gy = (p[1:-1, 2:, 1:-1] - p[1:-1, :-2, 1:-1]) / (2 * h)
    gz = (p[1:-1, 1:-1, 2:] - p[1:-1, 1:-1, :-2]) / (2 * h)
    out = np.full(dims, np.nan)
    out[1:-1, 1:-1, 1:-1] = np.sqrt(gx * gx + gy * gy + gz * gz)
    return out.ravel()


def _zero_crossings(phi, dims):
    """Per axis: the grid edges whose end values change sign, and the linear crossing point
    on each (fraction of the edge)."""
    p = phi.reshape(dims)
    out = []
    for ax in range(3):
        a = np.moveaxis(p, ax, 0)
        m = (a[:-1] < 0) != (a[1:] < 0)
        out.append((m, a[:-1][m] / (a[:-1][m] - a[1:][m])))
    return out


def _distance_defects(phi, phi_ref, dims, h, rho, R, eps):
    """(max band error of φ against |x−c| − R in units of h, max ||∇φ| − 1| in the band,
    max zero-crossing shift against phi_ref in units of h², or inf if the crossings changed
    edges)."""
    exact = rho - R
    band = np.abs(exact) < eps
    gn = _grad_norm(phi, dims, h)
    inner = band & ~np.isnan(gn)
    shift = 0.0
    for (m0, t0), (m1, t1) in zip(_zero_crossings(phi_ref, dims), _zero_crossings(phi, dims)):
        if not np.array_equal(m0, m1):
            return np.max(np.abs(phi[band] - exact[band])) / h, np.max(np.abs(gn[inner] - 1)), np.inf
        shift = max(shift, np.max(np.abs(t1 - t0)) * h / h ** 2)
    return np.max(np.abs(phi[band] - exact[band])) / h, np.max(np.abs(gn[inner] - 1)), shift


@pytest.mark.parametrize("shape", ["quadratic", "shallow"])
def test_reinit_restores_distance_of_non_distance_input(shape):
    """Section "Reinitialization", eqs. reinit and signum: the steady state of
    φ_t + sgn_h(φ0)(|∇φ| − 1) = 0 is the signed distance to the zero set of φ0. Inputs whose
    gradient is near 1 in the band, as Stage 1 produces them: the quadratic
    (|x−c|² − R²)/(2R) (|∇φ0| = 0.75..1.25 in the band at h = 0.25) and the shallow
    0.4(|x−c| − R). (Steep inputs, |∇φ0| ≥ 2, are outside this class: with sgn_h smoothed
    over h rather than |∇φ0|h the scheme moves their zero set by O(h).)"""
    R, shifts = 2.0, []
    for h in (0.25, 0.125):
        eps = 2 * h
        dims, rho = _box_sphere(h, R)
        phi0 = (rho ** 2 - R ** 2) / (2 * R) if shape == "quadratic" else 0.4 * (rho - R)
        steps = 2 * math.ceil((eps / h + 4) / 0.3 - 1e-9)  # the default step count
        phi = oracle.reinit(dims, h, phi0, steps)
        err, gdev, shift = _distance_defects(phi, phi0, dims, h, rho, R, eps)
        assert err < 0.02, (h, err)        # |φ − (|x−c| − R)| in the band, units of h
        assert gdev < 0.02, (h, gdev)      # ||∇φ| − 1| in the band
        assert shift < 0.15, (h, shift)    # zero crossings, units of h²
        shifts.append(shift * h * h)
        # the same checks on the input itself (a Stage 1 without reinitialization) fail
        err0, gdev0, _ = _distance_defects(phi0, phi0, dims, h, rho, R, eps)
        assert err0 > 0.1 and gdev0 > 0.1, (h, err0, gdev0)
    if shape == "quadratic":
        assert shifts[0] / shifts[1] > 3.0, shifts  # the zero set moves by O(h²)


def _stage1_steps(atoms, h, reinitialize=True):
    """Stage 1 composed from the oracle's own stages (vdW − ρ0, eikonal flow to ρ0, cavity
    removal, reinitialization with the default step count)."""
    prm = oracle.params(h)
    eps = prm[oracle.BAND]
    dims, origin = oracle.grid(atoms, h, oracle.grid_margin(atoms, h))
    phi = oracle.eikonal(dims, h, oracle.vdw(dims, origin, h, atoms) - 1.4, 1.4)
    phi, _, _ = oracle.cavity(dims, h, phi, eps)
    if reinitialize:
        phi = oracle.reinit(dims, h, phi, 2 * math.ceil((eps / h + 4) / 0.3 - 1e-9))
    return dims, origin, prm, phi


def test_two_atom_ses_signs_and_distance():
    """The whole Stage 1 on two atoms with a re-entrant groove: the signs agree with a
    brute-force probe closing (max over the ρ0-ball of F, minus ρ0) at nodes more than h from
    the surface, and φ is a distance function in the band, at second order in h. Without the
    reinitialization the band gradient check fails at every h."""
    atoms = np.array([[-1.15, 0.03, 0.01, 1.6, 0.5], [1.2, -0.02, 0.04, 1.5, -0.5]])
    rho, devs = 1.4, []
    for h in (0.25, 0.125):
        dims, origin, prm, phi = _stage1_steps(atoms, h)
        np.testing.assert_array_equal(phi, oracle.ses(dims, origin, atoms, prm)[0])
        eps = prm[oracle.BAND]
        gn = _grad_norm(phi, dims, h)
        band = (np.abs(phi) < eps) & ~np.isnan(gn)
        devs.append(np.max(np.abs(gn[band] - 1)))
        _, _, _, phi_nr = _stage1_steps(atoms, h, reinitialize=False)
        gn_nr = _grad_norm(phi_nr, dims, h)
        band_nr = (np.abs(phi_nr) < eps) & ~np.isnan(gn_nr)
        assert np.max(np.abs(gn_nr[band_nr] - 1)) > 0.08
        if h == 0.25:
            cand = np.nonzero(np.abs(phi) < 4 * h)[0]
            sel = np.random.default_rng(3).choice(cand, 150, replace=False)
            k, j, i = sel % dims[2], (sel // dims[2]) % dims[1], sel // (dims[1] * dims[2])
            X = np.column_stack([origin[0] + h * i, origin[1] + h * j, origin[2] + h * k])
            g = np.arange(-rho, rho + 1e-9, 0.05)
            P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
            P = P[np.linalg.norm(P, axis=1) <= rho]
            closing = np.empty(len(X))
            for q, x in enumerate(X):
                c = x + P
                F = np.min(np.linalg.norm(c[:, None, :] - atoms[None, :, :3], axis=2) - atoms[None, :, 3], axis=1)
                closing[q] = F.max() - rho
            far = np.abs(closing) > h
            assert far.sum() > 50
            assert np.all(np.sign(phi[sel][far]) == np.sign(closing[far]))
    assert devs[0] < 0.05 and devs[1] < 0.015 and devs[0] / devs[1] > 2.5, devs

"""Pins of the oracle's Stage 1 (level set of the solvent excluded surface).

  * WENO5 one-sided derivatives are exact on linear data and fifth-order on smooth data.
  * The inward eikonal flow φ_t = |∇φ| has the Hopf–Lax solution
    φ(x, t) = max_{|c−x| ≤ t} φ0(c); started from φ_SAS = F − ρ0 and run to t = ρ0 it is the
    signed function of the SES (probe-ball closing). The oracle is compared with a brute-force
    maximum over a dense sample of the ball, for one and for two atoms.
  * A single atom's SES is the atom itself: after the whole Stage 1 the band values equal
    |x − z| − r.
  * A closed shell of atoms around a void larger than the probe: cavity removal deletes the
    inner surface, so no band node projects inside the shell.
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

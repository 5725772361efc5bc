"""Pins of the oracle's pair kernels (regularization subsection, eq. IBIM-PBE).

The closed forms in the oracle are checked against high-precision numerical
derivatives of the two fundamental solutions G0 = 1/(4πr) and Gκ = e^{−κr}/(4πr),
computed here with mpmath (40 digits), so that a dropped term, a wrong sign or a
swapped normal in any of the four kernels fails.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import oracle

mp.mp.dps = 40
KAPPA = 0.1257


def _G(kappa):
    def g(x, y):
        r = mp.sqrt(sum((x[i] - y[i]) ** 2 for i in range(3)))
        return mp.exp(-kappa * r) / (4 * mp.pi * r)
    return g


def _fd_kernels(x, nx, y, ny, eps_in=1.0, eps_out=80.0, kappa=KAPPA):
    """K11, K12, K21, K22 from directional derivatives of G0 and Gκ (definition, not closed form)."""
    x, nx, y, ny = ([mp.mpf(float(v)) for v in a] for a in (x, nx, y, ny))
    G0, Gk = _G(0), _G(mp.mpf(kappa))
    th1, th2 = mp.mpf(eps_out) / eps_in, mp.mpf(eps_in) / eps_out

    def dny(G):
        return mp.diff(lambda t: G(x, [y[i] + t * ny[i] for i in range(3)]), 0)

    def dnx(G):
        return mp.diff(lambda t: G([x[i] + t * nx[i] for i in range(3)], y), 0)

    def dnxny(G):
        return mp.diff(lambda s, t: G([x[i] + s * nx[i] for i in range(3)], [y[i] + t * ny[i] for i in range(3)]),
                       (0, 0), (1, 1))

    K11 = dny(G0) - th1 * dny(Gk)
    K12 = G0(x, y) - Gk(x, y)
    K21 = dnxny(G0) - dnxny(Gk)
    K22 = dnx(G0) - th2 * dnx(Gk)
    return np.array([float(K11), float(K12), float(K21), float(K22)])


def _unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


CASES = [
    ([0, 0, 0], [0, 0, 1], [1, 0, 0], [0, 0, 1]),
    ([0, 0, 0], [0, 0, 1], [0.5, 0.25, -0.125], _unit([0.2, -0.1, 1.0])),
    ([1.9, 0.3, -0.2], _unit([1.9, 0.3, -0.2]), [-0.4, 1.7, 0.9], _unit([-0.4, 1.7, 0.9])),
    ([3.0, -1.0, 2.0], _unit([0.3, 0.5, -0.8]), [-2.5, 4.0, 0.7], _unit([-0.6, 0.1, 0.2])),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_kernels_match_derivatives_of_green_functions(case):
    x, nx, y, ny = CASES[case]
    prm = oracle.params(0.25, tau_k=1e-6)  # no regularization at these distances
    K = oracle.pair(x, _unit(nx), y, _unit(ny), prm)
    ref = _fd_kernels(x, _unit(nx), y, _unit(ny))
    np.testing.assert_allclose(K, ref, rtol=1e-12, atol=1e-15)


def test_kernels_other_dielectrics_and_kappa():
    x, nx, y, ny = CASES[3]
    prm = oracle.params(0.25, eps_in=2.0, eps_out=40.0, kappa=0.7, tau_k=1e-6)
    K = oracle.pair(x, nx, y, ny, prm)
    ref = _fd_kernels(x, nx, y, ny, eps_in=2.0, eps_out=40.0, kappa=0.7)
    np.testing.assert_allclose(K, ref, rtol=1e-12, atol=1e-15)


def test_kernel_symmetries():
    rng = np.random.default_rng(3)
    prm = oracle.params(0.25, tau_k=1e-6)
    swapped = oracle.params(0.25, eps_in=80.0, eps_out=1.0, tau_k=1e-6)
    for _ in range(20):
        x, y = rng.normal(size=3) * 2, rng.normal(size=3) * 2
        nx, ny = _unit(rng.normal(size=3)), _unit(rng.normal(size=3))
        Kxy = oracle.pair(x, nx, y, ny, prm)
        Kyx = oracle.pair(y, ny, x, nx, prm)
        assert Kxy[1] == pytest.approx(Kyx[1], rel=1e-14)
        assert Kxy[2] == pytest.approx(Kyx[2], rel=1e-12, abs=1e-16)
        # K22(y, x) is the adjoint double layer: equals K11(x, y) with θ1 replaced by θ2.
        assert Kyx[3] == pytest.approx(oracle.pair(x, nx, y, ny, swapped)[0], rel=1e-12, abs=1e-16)


def test_disc_average_of_k12():
    """K̄12 is the mean of G0 − Gκ over the tangent disc of radius τ (eq. reg-kernel-a)."""
    for kappa, tau in ((KAPPA, 0.25), (KAPPA, 0.125), (0.9, 0.3)):
        prm = oracle.params(1.0, kappa=kappa, tau_k=tau)
        K = oracle.pair([0, 0, 0], [0, 0, 1], [0, 0, 0], [0, 0, 1], prm)  # self pair: always regularized
        f = lambda rho: (1 - math.exp(-kappa * rho)) / (4 * math.pi * rho) * 2 * math.pi * rho
        avg = integrate.quad(f, 0, tau, epsabs=0, epsrel=1e-13)[0] / (math.pi * tau * tau)
        assert K[0] == 0 and K[2] == 0 and K[3] == 0
        assert K[1] == pytest.approx(avg, rel=1e-11)


def test_regularization_predicate_metrics():
    prm = oracle.params(1.0, tau_k=0.5)
    x, n = [0, 0, 0], [0, 0, 1]
    kbar = oracle.pair(x, n, x, n, prm)[1]
    # tangent distance 0.4 < τ, normal offset 0.1: regularized under every metric
    assert oracle.pair(x, n, [0.4, 0, 0.1], n, prm)[1] == kbar
    # tangent distance 0.6 > τ: not regularized
    assert oracle.pair(x, n, [0.6, 0, 0.0], n, prm)[1] != kbar
    # same normal line but 3 Å away: guarded and Euclidean keep the kernel, the literal metric averages it
    far = [0.0, 0.1, 3.0]
    assert oracle.pair(x, n, far, n, prm)[1] != kbar
    lit = prm.copy(); lit[oracle.METRIC] = oracle.METRIC_TANGENT
    assert oracle.pair(x, n, far, n, lit)[1] == kbar
    euc = prm.copy(); euc[oracle.METRIC] = oracle.METRIC_EUCLID
    assert oracle.pair(x, n, [0.3, 0, 0.3], n, euc)[1] == kbar      # r = 0.42 < τ
    assert oracle.pair(x, n, [0.45, 0, 0.25], n, euc)[1] != kbar    # r = 0.515 > τ
    assert oracle.pair(x, n, [0.45, 0, 0.25], n, prm)[1] == kbar    # tangent 0.45 < τ, r < 2τ


# ---------------------------------------------- curvature-corrected disc averages
# A regularized pair stands for the disc of radius τ around x*; its value times the disc's
# area should be the integral of the kernel over that part of the surface. Fixed here by
# quadrature of the oracle's own (pinned) kernels: over the spherical cap whose tangent-plane
# projection at the pole lies within τ (K11, K22: error O(τ²/R²), falling 4× per halving), and
# over the flat disc (K21: exact).

def _cap_integral(k, R, tau, prm):
    x, nx = np.array([0.0, 0.0, R]), np.array([0.0, 0.0, 1.0])
    th_max = math.asin(tau / R)

    def f(th):
        u = np.array([math.sin(th), 0.0, math.cos(th)])
        return oracle.pair(x, nx, R * u, u, prm)[k] * 2 * math.pi * R * R * math.sin(th)

    val, _ = integrate.quad(f, 0.0, th_max, limit=200, epsabs=0.0, epsrel=1e-9)
    return val, 2 * math.pi * R * R * (1 - math.cos(th_max))


@pytest.mark.parametrize("k", [0, 3], ids=["K11", "K22"])
def test_curved_disc_averages_of_the_double_layers(k):
    R = 2.0
    unreg = oracle.params(1.0, tau_k=1e-9)
    errs = []
    for tau in (0.5, 0.25, 0.125):
        integral, area = _cap_integral(k, R, tau, unreg)
        curved = oracle.params(1.0, tau_k=tau, avg=oracle.AVG_CURVED)
        kbar = oracle.pair([0, 0, R], [0, 0, 1], [0, 0, R], [0, 0, 1], curved, curv_x=2.0 / R)[k]
        errs.append(abs(kbar * area - integral) / abs(integral))
        # the paper's average is zero: it drops the whole integral
        assert oracle.pair([0, 0, R], [0, 0, 1], [0, 0, R], [0, 0, 1], oracle.params(1.0, tau_k=tau), 2.0 / R)[k] == 0
    assert errs[0] < 0.02 and errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


@pytest.mark.parametrize("kappa", [KAPPA, 0.7, 0.0])
def test_flat_disc_average_of_k21(kappa):
    z, ez = [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]
    unreg = oracle.params(1.0, kappa=kappa, tau_k=1e-9)
    for tau in (0.5, 0.25):
        integral, _ = integrate.quad(lambda r: oracle.pair(z, ez, [r, 0, 0], ez, unreg)[2] * 2 * math.pi * r,
                                     0.0, tau, epsabs=1e-15, epsrel=1e-12, limit=200)
        kbar = oracle.pair(z, ez, z, ez, oracle.params(1.0, kappa=kappa, tau_k=tau, avg=oracle.AVG_CURVED))[2]
        assert kbar * math.pi * tau * tau == pytest.approx(integral, rel=1e-8, abs=1e-15)

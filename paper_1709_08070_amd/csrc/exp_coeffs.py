"""Coefficients of the degree-11 polynomial for e^t on |t| ≤ ln2/2 used by exp_neg_f64
(fp64_math.hpp): the interpolant of e^t at the 12 Chebyshev nodes of the interval
(near-minimax), solved in the monomial basis in 60-digit arithmetic and rounded to doubles.
Prints the coefficients (t^0 first) and the largest relative error of their Horner
evaluation on a 4001-point grid, measured in 60-digit arithmetic (1.7e-17; the Taylor
series to degree 13 gives 5.2e-18, the FP64 rounding unit is 1.1e-16).

    python paper_1709_08070_amd/csrc/exp_coeffs.py
"""
import mpmath as mp

mp.mp.dps = 60
DEG = 11
L = mp.log(2) / 2
nodes = [L * mp.cos(mp.pi * (2 * k + 1) / (2 * (DEG + 1))) for k in range(DEG + 1)]
A = mp.matrix([[x ** j for j in range(DEG + 1)] for x in nodes])
c = mp.lu_solve(A, mp.matrix([mp.e ** x for x in nodes]))
coef = [float(c[j]) for j in range(DEG + 1)]
worst = mp.mpf(0)
for i in range(4001):
    t = -L + 2 * L * i / 4000
    p = mp.mpf(0)
    for cj in reversed(coef):
        p = p * t + mp.mpf(cj)
    worst = max(worst, abs(p / mp.e ** t - 1))
for j, v in enumerate(coef):
    print(f"c{j} = {v!r}")
print(f"max relative error {float(worst):.2e}")

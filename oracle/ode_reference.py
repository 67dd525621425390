"""Converged reference solutions of the kinetic ODE (test infrastructure only).

The explicit asymptotic method approximates the solution of Eq. (eq1.1),

    dY_i/dt = F+_i - F-_i,   F+_i = sum_{j: c_j = i} f_j,   F-_i = sum_{j: i in reac(j)} f_j,
    f_j = k_j Y_a (Y_b)      (mass action, constant rates over the interval),

whose exact solution conserves sum_i w_i Y_i when every reaction conserves the
weights.  This module integrates that ODE with scipy's Radau IIA (an implicit
fifth-order Runge-Kutta method with error control) at tight tolerances and an
analytic sparse Jacobian: the "converged reference" the final-abundance error
of the explicit integrator is measured against.  It shares nothing with the
explicit integrator of oracle.c or with the HIP path.

Pins (tests/test_oracle_pins.py): a linear network against the matrix
exponential, conservation of sum w Y, and the tiny nonlinear network of P7.
"""
from __future__ import annotations

import numpy as np
import scipy.integrate
import scipy.sparse as sp


def _incidence(net):
    a = np.asarray(net.reactant0, dtype=np.int64)
    b = np.asarray(net.reactant1, dtype=np.int64)
    c = np.asarray(net.product, dtype=np.int64)
    return a, b, c, b >= 0


def mass_action_rhs(net, k):
    """f(t, Y) = S f_j(Y) of Eq. (eq1.1) and its sparse Jacobian, for rates k [R]."""
    a, b, c, two = _incidence(net)
    N, R = net.n_species, len(a)
    k = np.asarray(k, dtype=np.float64)
    j_all = np.arange(R)
    # stoichiometry S [N][R]: +1 at the product, -1 at each reactant
    S = sp.csr_matrix((np.concatenate([np.ones(R), -np.ones(R), -np.ones(two.sum())]),
                       (np.concatenate([c, a, b[two]]),
                        np.concatenate([j_all, j_all, j_all[two]]))), shape=(N, R))
    bb = np.where(two, b, 0)

    def flux(Y):
        return k * Y[a] * np.where(two, Y[bb], 1.0)

    def rhs(t, Y):
        return S @ flux(Y)

    def jac(t, Y):
        # d f_j / d Y_a = k_j (Y_b or 1);  d f_j / d Y_b = k_j Y_a (two-body only)
        dfa = k * np.where(two, Y[bb], 1.0)
        dfb = (k * Y[a])[two]
        Jf = sp.csr_matrix((np.concatenate([dfa, dfb]),
                            (np.concatenate([j_all, j_all[two]]), np.concatenate([a, b[two]]))),
                           shape=(R, N))
        return (S @ Jf).tocsc()

    return rhs, jac


def radau(net, k, Y0, t_end, rtol=1e-10, atol=1e-30):
    """Y(t_end) of Eq. (eq1.1) from Y0 with rates k, by scipy Radau (tight tolerances)."""
    rhs, jac = mass_action_rhs(net, k)
    sol = scipy.integrate.solve_ivp(rhs, (0.0, float(t_end)), np.asarray(Y0, dtype=np.float64),
                                    method="Radau", rtol=rtol, atol=atol, jac=jac,
                                    jac_sparsity=None)
    if not sol.success:
        raise RuntimeError(f"Radau failed: {sol.message}")
    return sol.y[:, -1].copy(), int(sol.nfev), int(sol.t.size - 1)

"""Closed form of log det and its gradient for the arrow-free spatio-temporal
model exp(theta_1) kron(R_t, Q_s) + exp(theta_2) I, from the eigenvalues of
the path-graph Laplacians.  A pin for the tests (test infrastructure: the
product library never uses it)."""
from __future__ import annotations

import math
from typing import Tuple


def closed_form(nt: int, ns: int, kappa: float, theta) -> Tuple[float, Tuple[float, float]]:
    """log det and gradient of exp(theta_1) K + exp(theta_2) I (no arrow, no
    Z^T Z) from the eigenvalues of K: lambda_t mu_s with lambda_t = 2 - 2
    cos(pi t / n_t) and mu_s = (kappa^2 + 2 - 2 cos(pi s / n_s))^2."""
    import numpy as np
    lam = 2.0 - 2.0 * np.cos(np.pi * np.arange(nt) / nt)
    mu = (kappa ** 2 + 2.0 - 2.0 * np.cos(np.pi * np.arange(ns) / ns)) ** 2
    e1, e2 = math.exp(float(theta[0])), math.exp(float(theta[1]))
    ev = e1 * np.outer(lam, mu) + e2
    return float(np.log(ev).sum()), (float((e1 * np.outer(lam, mu) / ev).sum()), float((e2 / ev).sum()))

"""Pins of the gradient of log det A(theta) on the CPU: the oracle's log det
and its Jacobi-formula gradient, sum_ij Sigma_ij (dA/dtheta_i)_ij from the
oracle's selected inverse, against the closed form of the arrow-free model
(eigenvalues of a Kronecker product of path Laplacians) and against central
finite differences of the oracle's log det on the full model."""
import math

import numpy as np
import pytest

from closed_form import closed_form
from paper_2504_19171_amd import grad


def oracle_trace(oracle_mod, S, nb, w, ab, P, C):
    """sum_ij Sigma_ij B_ij for B symmetric in canonical band form (test-side sum)."""
    t = float(np.dot(S.Sb[0], ab[0]))
    for d in range(1, w + 1):
        t += 2.0 * float(np.dot(S.Sb[d, : nb - d], ab[d, : nb - d]))
    if P is not None and P.size:
        t += 2.0 * float(np.sum(S.SP * P)) + float(np.sum(S.SC * C))
    return t


def model_np(m, theta):
    ab, P, C = m.assemble(theta)
    return ab.numpy(), (P.numpy() if P is not None else None), (C.numpy() if C is not None else None)


def oracle_logdet_grad(oracle_mod, m, theta, b=64):
    ab, P, C = model_np(m, theta)
    Pz = P if P is not None else np.zeros((0, m.nb))
    Cz = C if C is not None else np.zeros((0, 0))
    f = oracle_mod.cholesky(ab, Pz, Cz)
    assert f.info == 0
    S = oracle_mod.selinv(f, b)
    g = []
    for dab, dP, dC in m.derivatives(theta):
        g.append(oracle_trace(oracle_mod, S, m.nb, m.w, dab.numpy(), None if dP is None else dP.numpy(),
                              None if dC is None else dC.numpy()))
    return f, g


@pytest.mark.parametrize("theta", [(0.4, -1.2), (-2.0, 0.5), (1.5, 1.5)])
def test_arrow_free_model_matches_closed_form(oracle_mod, theta):
    nt, ns, kappa = 4, 25, 0.5
    m = grad.SpatioTemporal(nt, ns, kappa, 0, seed=1, device="cpu", arrow=False, with_ztz=False)
    f, g = oracle_logdet_grad(oracle_mod, m, theta)
    ld, gc = closed_form(nt, ns, kappa, theta)
    scale = max(1.0, float(np.sum(np.abs(2.0 * np.log(f.diag())))))
    assert abs(f.logdet - ld) <= 1e-12 * scale
    for gi, ci in zip(g, gc):
        assert abs(gi - ci) <= 1e-10 * abs(ci)


def test_full_model_gradient_matches_central_differences(oracle_mod):
    m = grad.SpatioTemporal(3, 20, 0.5, 4, seed=7, device="cpu")
    theta = [0.2, -0.5]
    f, g = oracle_logdet_grad(oracle_mod, m, theta)
    h = 1e-5
    for i in range(2):
        tp = list(theta); tm = list(theta)
        tp[i] += h; tm[i] -= h
        ldp = oracle_mod.cholesky(*[x if x is not None else np.zeros((0, 0)) for x in model_np(m, tp)]).logdet
        ldm = oracle_mod.cholesky(*[x if x is not None else np.zeros((0, 0)) for x in model_np(m, tm)]).logdet
        fd = (ldp - ldm) / (2 * h)
        print(f"theta_{i + 1}: Jacobi {g[i]:.12e}  central difference {fd:.12e}")
        assert abs(g[i] - fd) <= 1e-6 * abs(g[i])


def test_trace_of_a_planted_mistake_is_caught(oracle_mod):
    """A dropped factor 2 on the off-diagonal terms of the test-side trace
    breaks the agreement with the closed form (so the pin can fail)."""
    nt, ns, kappa = 3, 15, 0.5
    m = grad.SpatioTemporal(nt, ns, kappa, 0, seed=1, device="cpu", arrow=False, with_ztz=False)
    theta = (0.3, -0.3)
    ab, _, _ = model_np(m, theta)
    f = oracle_mod.cholesky(ab, np.zeros((0, m.nb)), np.zeros((0, 0)))
    S = oracle_mod.selinv(f, 64)
    dab = m.derivatives(theta)[0][0].numpy()
    wrong = float(np.dot(S.Sb[0], dab[0])) + sum(float(np.dot(S.Sb[d, : m.nb - d], dab[d, : m.nb - d]))
                                                  for d in range(1, m.w + 1))
    _, gc = closed_form(nt, ns, kappa, theta)
    assert abs(wrong - gc[0]) > 1e-3 * abs(gc[0])

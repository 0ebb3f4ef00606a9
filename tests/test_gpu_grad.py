"""The gradient of log det A(theta) through the HIP path: the trace product
against the oracle's selected inverse, the autograd function against the
oracle gradient and central differences, and at the full size of the
spatio-temporal workload (n_t = 50, n_s = 2,000, tile 256) against the closed
form of the arrow-free model and central differences of the full model."""
import math

import numpy as np
import pytest

from closed_form import closed_form
from paper_2504_19171_amd import grad, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2504_19171_amd import stiles as st
    st.load()
    return torch


def test_trace_product_matches_oracle(torch_cuda, oracle_mod):
    from gpu_util import to_device
    from test_grad_oracle import oracle_trace
    from paper_2504_19171_amd import stiles as st
    nb, w, a, b = 900, 70, 20, 64
    M = inputs.arrowhead_spd(nb, w, a, seed=11)
    Bm = inputs.arrowhead_spd(nb, w, a, seed=12)      # any symmetric B on the pattern of A
    lay = st.layout(M.n, w, a, b)
    L, _, _ = st.factor(st.pack(*to_device(M, "cuda:0"), lay), lay)
    S, _ = st.selinv(L, lay)
    B = st.pack(*to_device(Bm, "cuda:0"), lay)
    t = float(st.trace_product(S, B, lay).item())
    So = oracle_mod.selinv(oracle_mod.cholesky(M.ab, M.P, M.C), b)
    ref = oracle_trace(oracle_mod, So, nb, w, Bm.ab, Bm.P, Bm.C)
    print(f"trace {t:.15e} oracle {ref:.15e}", flush=True)
    assert abs(t - ref) <= 1e-10 * abs(ref)
    # padding and the unused tiles are left out: tr(Sigma A) = n exactly up to rounding
    tA = float(st.trace_product(S, st.pack(*to_device(M, "cuda:0"), lay), lay).item())
    assert abs(tA - M.n) <= 1e-9 * M.n


def test_autograd_matches_oracle_and_differences(torch_cuda, oracle_mod):
    torch = torch_cuda
    from test_grad_oracle import oracle_logdet_grad
    m_cpu = grad.SpatioTemporal(4, 40, 0.5, 6, seed=5, device="cpu")
    m_gpu = grad.SpatioTemporal(4, 40, 0.5, 6, seed=5, device="cuda:0")
    m_gpu.X = m_cpu.X.to("cuda:0")   # the same covariates on both sides
    theta0 = [0.3, -0.8]
    f, g_or = oracle_logdet_grad(oracle_mod, m_cpu, theta0)
    fn = grad.LogDet(m_gpu, tile=64)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    ld = fn(theta)
    ld.backward()
    g = theta.grad.tolist()
    scale = max(1.0, float(np.sum(np.abs(2.0 * np.log(f.diag())))))
    print(f"log det {float(ld):.12e} oracle {f.logdet:.12e}; grad {g} oracle {g_or}", flush=True)
    assert abs(float(ld) - f.logdet) <= 1e-12 * scale
    for gi, oi in zip(g, g_or):
        assert abs(gi - oi) <= 1e-10 * abs(oi)
    h = 1e-5
    for i in range(2):
        tp = torch.tensor(theta0, dtype=torch.float64); tm = tp.clone()
        tp[i] += h; tm[i] -= h
        fd = (float(fn(tp)) - float(fn(tm))) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * abs(g[i])


def test_full_size_arrow_free_closed_form(torch_cuda):
    torch = torch_cuda
    nt, ns, kappa = 50, 2000, 0.5
    m = grad.SpatioTemporal(nt, ns, kappa, 0, seed=4, device="cuda:0", arrow=False, with_ztz=False)
    fn = grad.LogDet(m, tile=256)
    for theta0 in ([0.0, 0.0], [-3.0, -3.0]):
        theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
        print(f"full size arrow-free theta {theta0}: n = {m.n}, w = {m.w}", flush=True)
        ld = fn(theta)
        ld.backward()
        ref, gref = closed_form(nt, ns, kappa, theta0)
        g = theta.grad.tolist()
        print(f"  log det {float(ld):.13e} closed form {ref:.13e}; grad {g} closed form {gref}", flush=True)
        assert abs(float(ld) - ref) <= 1e-12 * max(1.0, abs(ref))
        for gi, ri in zip(g, gref):
            assert abs(gi - ri) <= 1e-10 * abs(ri)


def test_full_size_model_central_differences(torch_cuda):
    torch = torch_cuda
    m = grad.SpatioTemporal(50, 2000, 0.5, 50, seed=4, device="cuda:0")
    fn = grad.LogDet(m, tile=256)
    theta0 = [0.0, 0.0]
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    print(f"full model n = {m.n}, w = {m.w}, arrow {m.a}", flush=True)
    ld = fn(theta)
    ld.backward()
    g = theta.grad.tolist()
    h = 1e-5
    for i in range(2):
        tp = torch.tensor(theta0, dtype=torch.float64); tm = tp.clone()
        tp[i] += h; tm[i] -= h
        fd = (float(fn(tp)) - float(fn(tm))) / (2 * h)
        print(f"  theta_{i + 1}: Jacobi {g[i]:.12e} central difference {fd:.12e}", flush=True)
        assert abs(g[i] - fd) <= 1e-6 * abs(g[i])
    assert math.isfinite(float(ld))

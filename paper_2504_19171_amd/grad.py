"""Differentiation of log det A(theta): a torch.autograd.Function whose
forward is the library's factor (log det) and whose backward is Jacobi's
formula read off the selected inverse,

    d log det A / d theta_i = tr(A^{-1} dA/dtheta_i) = sum_ij Sigma_ij (dA/dtheta_i)_ij,

which needs Sigma only where dA/dtheta_i is non-zero, i.e. on the pattern of
A, inside the tile pattern of L (the use of selected inversion the paper's
INLA setting makes of it, Sec. I).  The product and its sum run in the
library (stiles_trace_product); this module only assembles the matrices.

The model (`SpatioTemporal`) is the precision matrix of a space-time field
plus fixed effects:
    A(theta) = blockdiag(exp(theta_1) K, 0) + exp(theta_2) I + Z^T Z,  Z = [I | X],
with K = kron(R_t, Q_s) in time-major order, R_t the random-walk-1 matrix of
a path of n_t times (the path-graph Laplacian: 1 at the ends, 2 inside, -1
off the diagonal), Q_s = (kappa^2 I + G)^2 with G the same Laplacian on a
chain of n_s sites, and X (n_t n_s x a) the fixed-effect covariates.  Z^T Z
puts I on the field block, X in the coupling rows (the arrow) and X^T X in
the corner.  So the band has half-bandwidth n_s + 2 and the arrow width a.
    dA/dtheta_1 = exp(theta_1) blockdiag(K, 0),   dA/dtheta_2 = exp(theta_2) I.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

from . import stiles as st


class SpatioTemporal:
    """A(theta) of the module docstring on one device, in canonical band form."""

    def __init__(self, nt: int, ns: int, kappa: float, a: int, seed: int, device, arrow: bool = True,
                 with_ztz: bool = True):
        import torch
        self.nt, self.ns, self.kappa, self.dev = int(nt), int(ns), float(kappa), device
        self.nb = self.nt * self.ns
        self.a = int(a) if arrow else 0
        self.w = self.ns + 2 if self.nt > 1 else 2
        self.with_ztz = with_ztz
        self.Kab = self._kron_band()
        g = torch.Generator(device=device)
        g.manual_seed(int(seed))
        self.X = (torch.randn((self.nb, self.a), generator=g, dtype=torch.float64, device=device)
                  if self.a else None)
        self._XtX = None     # X^T X, formed on first use (it does not depend on theta)

    @staticmethod
    def path_laplacian_diag(m: int):
        import torch
        d = torch.full((m,), 2.0, dtype=torch.float64)
        if m == 1:
            d[0] = 0.0
        else:
            d[0] = d[-1] = 1.0
        return d

    def _kron_band(self):
        """K = kron(R_t, Q_s) in canonical band form: ab[d, j] = K[j+d, j]."""
        import torch
        nt, ns, dev = self.nt, self.ns, self.dev
        r = self.path_laplacian_diag(nt)                          # R_t diagonal; off-diagonal -1
        m = self.kappa ** 2 + self.path_laplacian_diag(ns)        # M = kappa^2 I + G; off-diagonal -1
        # Q = M^2: Q[i,i] = m_i^2 + (#neighbours), Q[i+1,i] = -(m_i + m_{i+1}), Q[i+2,i] = 1
        q0 = m * m
        q0[1:] += 1.0
        q0[:-1] += 1.0
        q1 = -(m[:-1] + m[1:])
        q2 = torch.ones(max(ns - 2, 0), dtype=torch.float64)
        Q = [q0, q1, q2]
        ab = torch.zeros((self.w + 1, self.nb), dtype=torch.float64)
        for t in range(nt):
            c0 = t * ns
            for dd in range(3):                                    # same time, K[(t,s+dd),(t,s)]
                if ns - dd > 0:
                    ab[dd, c0:c0 + ns - dd] = r[t] * Q[dd]
            if t + 1 < nt:                                         # next time: R[t+1,t] = -1
                for e in range(-2, 3):                             # K[(t+1,s+e),(t,s)] = -Q[s+e,s]
                    d = ns + e
                    qe = Q[abs(e)]
                    if e >= 0:
                        ab[d, c0:c0 + ns - e] = -qe
                    else:
                        ab[d, c0 - e:c0 + ns] = -qe
        return ab.to(dev)

    @property
    def n(self) -> int:
        return self.nb + self.a

    def layout(self, tile: int) -> st.Layout:
        return st.layout(self.n, self.w, self.a, tile)

    def assemble(self, theta) -> Tuple[object, object, object]:
        """(ab, P, C) of A(theta) on the device."""
        import torch
        t1, t2 = float(theta[0]), float(theta[1])
        ab = math.exp(t1) * self.Kab
        ab[0] += math.exp(t2) + (1.0 if self.with_ztz else 0.0)
        if not self.a:
            return ab, None, None
        if self._XtX is None or self._XtX[0] is not self.X:
            self._XtX = (self.X, self.X.T @ self.X)
        P = self.X.T.contiguous()
        C = self._XtX[1] + math.exp(t2) * torch.eye(self.a, dtype=torch.float64, device=self.dev)
        return ab, P, C

    def derivatives(self, theta):
        """[(ab, P, C)] of dA/dtheta_1 and dA/dtheta_2 on the device."""
        import torch
        t1, t2 = float(theta[0]), float(theta[1])
        d1 = math.exp(t1) * self.Kab
        d2 = torch.zeros_like(self.Kab)
        d2[0] = math.exp(t2)
        out = []
        for ab, cdiag in ((d1, 0.0), (d2, math.exp(t2))):
            if self.a:
                P = torch.zeros((self.a, self.nb), dtype=torch.float64, device=self.dev)
                C = cdiag * torch.eye(self.a, dtype=torch.float64, device=self.dev)
                out.append((ab, P, C))
            else:
                out.append((ab, None, None))
        return out


def _check(info, where):
    v = int(info.item())
    if v != 0:
        raise st.StilesError(v, where)


class LogDet:
    """log det A(theta) as a differentiable function of theta (torch tensor of 2)."""

    def __init__(self, model: SpatioTemporal, tile: int = 256):
        import torch

        self.model, self.tile = model, int(tile)
        self.lay = model.layout(self.tile)
        outer = self

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta):
                ab, P, C = outer.model.assemble(theta.detach().cpu().tolist())
                A = st.pack(ab, P, C, outer.lay)
                L, ld, info = st.factor(A, outer.lay, out=A)
                _check(info, "stiles_factor")
                ctx.L = L
                ctx.theta = theta.detach().cpu().tolist()
                return ld.reshape(()).to(theta.device)

            @staticmethod
            def backward(ctx, g):
                S, sinfo = st.selinv(ctx.L, outer.lay)
                _check(sinfo, "stiles_selinv")
                tr = []
                for ab, P, C in outer.model.derivatives(ctx.theta):
                    B = st.pack(ab, P, C, outer.lay)
                    tr.append(st.trace_product(S, B, outer.lay))
                ctx.L = None
                return g * torch.cat(tr).to(g.device)

        self._f = _F

    def __call__(self, theta):
        return self._f.apply(theta)

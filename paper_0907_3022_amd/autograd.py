"""torch.autograd.Function around the GPU propagation and its adjoint.

ChebPropagate.apply(V, psi0, prop) returns psi after prop.K Chebyshev steps
of H(V) = H_0 + diag(V), where V is the on-site potential of a 1D
finite-difference chain or the on-site energies of a honeycomb ribbon.  Its
backward pass runs the library's reverse recursion (chebtd_adjoint) and
returns dL/dV and dL/dpsi0.  The spectral scale (a, b) is fixed by the
propagator, so the derivative is that of the exact propagator up to the
1e-15 truncation of the expansion.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .api import Context


class Propagator:
    """Geometry, step and spectral bounds of a differentiable propagation.

    kind: "chain" (needs dx) or "honeycomb" (needs width, length, edge, t).
    bounds: (emin, emax) enclosing the spectrum of H(V) for every V the
    caller will use (they fix H~ = (H - b)/a).
    adjoint_mode: L.ADJ_STEP, L.ADJ_SQRTM or L.ADJ_REVERSE; None picks
    L.ADJ_REVERSE (the fastest, three vectors per step) where the lattice
    allows it and L.ADJ_STEP elsewhere.
    """

    def __init__(self, kind, dt, K, bounds, *, dx=None, width=None, length=None, edge="zigzag",
                 t=1.0, alpha=0.01, tol=1e-15, adjoint_mode=None, context=None):
        if kind not in ("chain", "honeycomb"):
            raise ValueError("kind must be 'chain' or 'honeycomb'")
        if int(K) < 0:
            raise ValueError("K must be >= 0")
        self.kind, self.dt, self.K = kind, float(dt), int(K)
        self.bounds = (float(bounds[0]), float(bounds[1]))
        self.dx, self.width, self.length, self.edge, self.t = dx, width, length, edge, t
        self.alpha, self.tol, self.adjoint_mode = alpha, tol, adjoint_mode
        self.ctx = context or Context()
        self.M = None
        self.run = 0

    def _setup(self, V):
        if self.kind == "chain":
            self.ctx.chain1d(V, self.dx)
        else:
            self.ctx.honeycomb(self.width, self.length, V, edge=self.edge, t=self.t)
        self.ctx.set_bounds(*self.bounds, self.alpha)
        self.M = self.ctx.plan(self.dt, self.tol)

    def forward(self, V, psi0, keep=True):
        """psi after K steps; with keep, the trajectory is stored for one
        backward and self.run numbers that run."""
        self._setup(V)
        steps = max(self.K, 1)  # storage for at least one step (K = 0 stores none)
        if keep and self.adjoint_mode is None:
            try:
                self.ctx.reserve_adjoint(steps, L.ADJ_REVERSE)
            except L.ChebError as err:  # past the downward walk's offset limit
                if err.code != L.E_ARG:
                    raise
                self.ctx.reserve_adjoint(steps, L.ADJ_STEP)
        elif keep:
            self.ctx.reserve_adjoint(steps, self.adjoint_mode)
        psi = psi0.detach().clone().contiguous()
        self.ctx.propagate(psi, self.K, flags=L.KEEP_CHECKPOINTS if keep else 0)
        self.run = self.ctx.checkpoint_run() if keep else 0
        return psi

    def backward(self, gbar, V, psi0=None, run=None):
        """gbar: dL/dpsi_K (torch convention); returns (dL/dV, dL/dpsi_0).
        run: the checkpointing run of the forward pass this gradient belongs
        to.  If the context has stored another trajectory since (the same
        propagator applied again before this backward), the forward pass is
        run again from V and psi0 so the adjoint sees its own trajectory."""
        if run is not None and self.ctx.checkpoint_run() != run:
            if psi0 is None:
                raise RuntimeError("the stored trajectory belongs to another run and psi0 is unknown")
            self.forward(V, psi0, keep=True)
            run = self.run
        g = gbar.detach().clone().contiguous().to(torch.complex128)
        dV = torch.zeros_like(V, dtype=torch.float64)
        self.ctx.adjoint(g, dV, run=run)
        return dV, g


class ChebPropagate(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V, psi0, prop: Propagator):
        keep = V.requires_grad or psi0.requires_grad
        out = prop.forward(V.detach(), psi0, keep=keep)
        fctx.prop = prop
        fctx.run = prop.run
        fctx.save_for_backward(V, psi0)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        V, psi0 = fctx.saved_tensors
        dV, dpsi0 = fctx.prop.backward(grad_out, V.detach(), psi0.detach(), fctx.run)
        return dV, dpsi0, None

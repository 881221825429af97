"""Differentiable expectation values: the adjoint sweep behind torch.autograd.

    ev = Expectation(n, gates, obs)            # gates may hold rotations
    f = ev(theta)                              # theta: 1-D float tensor
    f.backward()                               # theta.grad <- df/dtheta

f(theta) = <0..0| U(theta)^dagger O U(theta) |0..0> with O a weighted sum of
Z strings: the cost function of a variational (parametrised-circuit)
algorithm.  The paper's simulator evaluates such circuits forward only; the
gradient here is the adjoint method of Jones and Gacon (arXiv:2009.02823).  The forward
pass runs the circuit with the fused tile passes and reduces O on the GPU;
the backward pass rewinds the stored state together with the co-state
O|psi> in one sweep (qsv_adjoint), so one backward costs about as much as a
few forward passes, independent of the number of parameters.

Every step runs in libqsv.so; this module only moves the angle vector and
the gradient between torch and the library.
"""
from __future__ import annotations

import numpy as np

from .qsv import FLAG_FORWARD, FLAG_FROM_ZERO, GROT, QSV_C128, Context, State, adjoint, marshal_gates

__all__ = ["Expectation"]


def _torch():
    import torch
    return torch


class Expectation:
    """A fixed circuit and observable, differentiable in the rotation angles.

    gates: gate list (see marshal_gates); rotation gates index into theta.
    obs:   [(qubits, weight), ...], a weighted sum of Z strings.
    The object owns two device states of 2^n amplitudes (the state and the
    co-state).  A forward call leaves U(theta)|0..0> in the first; the
    backward of the most recent call rewinds it in place.  The backward of
    an older call (or a second backward of the same call) recomputes the
    state from its saved angles first.
    """

    def __init__(self, n: int, gates, obs, dtype: int = QSV_C128, context: Context | None = None):
        self.n = n
        self.dtype = dtype
        self.obs = list(obs)
        self.ctx = context if context is not None else Context()
        self.g = marshal_gates(gates)
        self.nparams = int(max((int(r["param"]) + 1 for r in self.g if r["kind"] == GROT), default=0))
        self.psi = State(self.ctx, n, dtype)
        self.lam = State(self.ctx, n, dtype)
        self._version = 0          # bumped by every forward
        self._fresh = False        # psi holds the state of call _version

    def __call__(self, theta):
        return _ExpectationFn.apply(theta, self)

    def value(self, theta: np.ndarray) -> float:
        p = np.ascontiguousarray(theta, dtype=np.float64)
        self.psi.apply_circuit(None, p, flags=FLAG_FROM_ZERO, marshalled=self.g)
        self._version += 1
        self._fresh = True
        return self.psi.expect_z(self.obs)[1]

    def gradient(self, theta: np.ndarray, version: int) -> np.ndarray:
        p = np.ascontiguousarray(theta, dtype=np.float64)
        flags = 0 if (self._fresh and version == self._version) else FLAG_FORWARD
        self._fresh = False        # the sweep consumes psi
        _, grad = adjoint(self.psi, self.lam, None, p, self.obs, flags, marshalled=self.g)
        return grad


class _ExpectationFn:
    """Built lazily so that importing this module does not import torch."""
    _cls = None

    @classmethod
    def apply(cls, theta, ev: Expectation):
        if cls._cls is None:
            torch = _torch()

            class Fn(torch.autograd.Function):
                @staticmethod
                def forward(fctx, th, e):
                    p = th.detach().to("cpu", torch.float64).reshape(-1).numpy()
                    if p.size < e.nparams:
                        raise ValueError(f"circuit uses {e.nparams} angles, got {p.size}")
                    f = e.value(p)
                    fctx.e = e
                    fctx.version = e._version
                    fctx.save_for_backward(th.detach().to("cpu", torch.float64))
                    return torch.tensor(f, dtype=th.dtype, device=th.device)

                @staticmethod
                def backward(fctx, gout):
                    (th,) = fctx.saved_tensors
                    grad = fctx.e.gradient(th.reshape(-1).numpy(), fctx.version)
                    g = torch.from_numpy(grad).reshape(th.shape)
                    return g.to(gout.device, gout.dtype) * gout, None

            cls._cls = Fn
        return cls._cls.apply(theta, ev)

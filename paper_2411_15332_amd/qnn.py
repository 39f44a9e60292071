"""QNN layer on the state-vector engine: forward <Z_0> and the adjoint backward.

The circuit is the hardware-efficient ansatz: an RY(x_q) angle-encoding layer,
then L layers of RY(theta) on every qubit, RZ(theta) on every qubit and the
CNOT ring CNOT(q, (q+1) mod n). The parameter vector of one batch entry is
[x (n), theta (2nL)] with theta index (2l + {0: RY, 1: RZ}) n + q.

Both run in the HIP kernels behind the C ABI. When a gradient is needed, the
forward call itself is sv_adjoint_expect_z (one forward and one reverse sweep
over psi and lambda = Z_0 psi, with Im <lambda|P|psi> accumulated in FP64 at
every rotation), which returns <Z_0> and every gradient at once; backward
only scales the stored gradients by the incoming ones. Otherwise forward is
sv_apply_circuit + sv_expect_z. State handles (and the adjoint's work
buffers) are kept between calls, a few per shape.
"""
from __future__ import annotations

import threading
from collections import OrderedDict
from typing import List

import numpy as np
import torch

from .sv import GATE_DTYPE, StateVector

_CACHE_MAX = 4
_cache: "OrderedDict[tuple, StateVector]" = OrderedDict()
_cache_lock = threading.Lock()


def _handle(n: int, dtype: str, batch: int, device: int) -> StateVector:
    """A cached state handle of this shape (least recently used ones are
    released beyond a few)."""
    key = (n, dtype, batch, device)
    sv = _cache.pop(key, None)
    if sv is None:
        sv = StateVector(n, dtype, batch=batch, device=device)
    _cache[key] = sv
    while len(_cache) > _CACHE_MAX:
        _, old = _cache.popitem(last=False)
        old.close()
    return sv


def release_cache() -> None:
    """Free the cached state handles and their device memory."""
    with _cache_lock:
        while _cache:
            _, sv = _cache.popitem()
            sv.close()


_RY, _RZ, _CNOT = 10, 11, 13


def ansatz_gates(n: int, layers: int) -> np.ndarray:
    """sv_gate records of the ansatz with parameter references."""
    recs: List[tuple] = [(_RY, q, -1, q, 0.0, 0) for q in range(n)]
    for l in range(layers):
        recs += [(_RY, q, -1, n + (2 * l) * n + q, 0.0, 0) for q in range(n)]
        recs += [(_RZ, q, -1, n + (2 * l + 1) * n + q, 0.0, 0) for q in range(n)]
        if n >= 2:
            recs += [(_CNOT, q, (q + 1) % n, -1, 0.0, 0) for q in range(n)]
    return np.array(recs, dtype=GATE_DTYPE)


def _params(theta: torch.Tensor, x: torch.Tensor) -> np.ndarray:
    return np.ascontiguousarray(
        torch.cat([x.detach(), theta.detach()], dim=1).to("cpu", torch.float64).numpy())


class QNNFunction(torch.autograd.Function):
    """f_b = <Z_0> of the ansatz with parameters (x_b, theta_b).

    theta: [B, 2nL], x: [B, n]; returns [B] in theta's dtype and device.
    Gradients flow to theta and x.
    """

    @staticmethod
    def forward(ctx, theta, x, n: int, layers: int, dtype: str = "c128"):
        B = theta.shape[0]
        gates = ansatz_gates(n, layers)
        p = _params(theta, x)
        device = torch.cuda.current_device()
        need_grad = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        with _cache_lock:
            sv = _handle(n, dtype, B, device)
            if need_grad:
                z, g = sv.adjoint_expect_z(gates, p, qubit=0)   # <Z_0> and every gradient
            else:
                sv.set_basis(0)
                sv.apply(gates, p)
                z, g = sv.expect_z(0), None
        ctx.n = n
        ctx.grad = None if g is None else torch.as_tensor(g, dtype=theta.dtype, device=theta.device)
        return torch.as_tensor(z, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        n = ctx.n
        g = ctx.grad * grad_out[:, None]
        return g[:, n:], g[:, :n], None, None, None


def qnn_expect(theta, x, n: int, layers: int, dtype: str = "c128"):
    return QNNFunction.apply(theta, x, n, layers, dtype)

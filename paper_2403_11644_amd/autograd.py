"""Differentiation through the decomposition with hand-written adjoints.

decompose is linear: c = M vec(A) with M[P, (r, c)] = 2^-n P[c][r], so its
vector-Jacobian product (PyTorch's convention for complex tensors: the
gradient with respect to conj(A)) is M^H g = 2^-n sum_P g_P P -- the
reconstruction kernel with the PTD_ADJOINT scale.  Reconstruction
A = sum_P c_P P has adjoint 2^n M, i.e. the decomposition without its
2^-n scale (PTD_ADJOINT of pauli_decompose).
"""
from __future__ import annotations

import torch

from . import api


class PauliDecompose(torch.autograd.Function):
    """c = decompose(A) for a dense complex A; backward runs the adjoint
    reconstruction kernel."""

    @staticmethod
    def forward(ctx, A: torch.Tensor) -> torch.Tensor:
        return api.decompose(A.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor) -> torch.Tensor:
        return api.reconstruct(g.contiguous(), adjoint=True)


class PauliReconstruct(torch.autograd.Function):
    """A = reconstruct(c) for dense complex coefficients; backward runs the
    decomposition kernel without its 2^-n scale."""

    @staticmethod
    def forward(ctx, c: torch.Tensor) -> torch.Tensor:
        return api.reconstruct(c.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor) -> torch.Tensor:
        return api.decompose(g.contiguous(), adjoint=True)


def pauli_decompose(A: torch.Tensor) -> torch.Tensor:
    return PauliDecompose.apply(A)


def pauli_reconstruct(c: torch.Tensor) -> torch.Tensor:
    return PauliReconstruct.apply(c)

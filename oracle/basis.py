"""Orthonormal polynomials and the discrete equilibrium (oracle; test infrastructure only).

Sec. 5.2: starting from the generating set V = {1, p^a, p^a p^b, ...} the
Gram-Schmidt procedure with respect to the weight omega(p^0) yields
polynomials J^(k) orthonormal under int omega J_l J_k d^dp/p^0 (Eq.
mj-orthogonal-conditions).  The projection coefficients are
a^(k) = int f^eq J^(k) d^dp/p^0 (Eq. mj-projection-coefficients) and the
discrete equilibrium is f^eq_i = w_i sum_k a^(k) J^(k)(p_i) (Eq.
mj-discrete-feq).

The inner product is evaluated with the quadrature itself, which is exact for
degree <= 2N and therefore equals the continuum one.  Elements of V that are
linearly dependent on earlier ones on the mass shell (p^0 p^0 = m^2 + |p|^2)
are skipped.  The supplementary third-order polynomials that the paper does
not print are obtained this way; the projection onto the span is unique, so
the result does not depend on the basis chosen.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import torch

from . import mj
from .quadrature import Quadrature


def generating_set(d: int, order: int):
    """V as index tuples in the paper's order: degree by degree, a <= b <= c ..."""
    out = [()]
    for deg in range(1, order + 1):
        out.extend(itertools.combinations_with_replacement(range(d + 1), deg))
    return out


@dataclass
class Basis:
    quad: Quadrature
    gens: list            # kept generating monomials (index tuples)
    C: np.ndarray         # (K, len(gens)) J^(k) = sum_v C[k, v] * monomial_v
    J: np.ndarray         # (K, Q) J^(k)(p_i)


def monomial_values(quad: Quadrature, idx) -> np.ndarray:
    v = np.ones(quad.Q, dtype=np.longdouble)
    for a in idx:
        v = v * quad.p[:, a].astype(np.longdouble)
    return v


def gram_schmidt(quad: Quadrature, order: int, tol: float = 1e-10) -> Basis:
    """Modified Gram-Schmidt (with one re-orthogonalisation pass) in extended precision."""
    w = quad.w.astype(np.longdouble)

    def dot(a, b):
        return np.sum(w * a * b)

    gens_all = generating_set(quad.d, order)
    kept, rows_val, rows_coef = [], [], []
    for g in gens_all:
        val = monomial_values(quad, g)
        coef = np.zeros(len(gens_all), dtype=np.longdouble)
        coef[gens_all.index(g)] = 1.0
        norm0 = np.sqrt(dot(val, val))
        for _ in range(2):
            for jv, jc in zip(rows_val, rows_coef):
                proj = dot(val, jv)
                val = val - proj * jv
                coef = coef - proj * jc
        nrm = np.sqrt(dot(val, val))
        if nrm <= tol * norm0:
            continue                        # dependent on the mass shell
        rows_val.append(val / nrm)
        rows_coef.append(coef / nrm)
        kept.append(g)
    idx_kept = [gens_all.index(g) for g in kept]
    C = np.array(rows_coef)[:, idx_kept].astype(np.float64)
    # re-express each J^(k) over the kept monomials only (dependent ones never entered)
    J = np.array(rows_val).astype(np.float64)
    return Basis(quad, kept, C, J)


def projection_coefficients(basis: Basis, n, T, U):
    """a^(k) = int f^eq J^(k) d^dp/p^0 from the closed-form Maxwell-Juettner moments (App. B)."""
    quad = basis.quad
    n = torch.as_tensor(n, dtype=torch.float64)
    T = torch.as_tensor(T, dtype=torch.float64)
    U = torch.as_tensor(U, dtype=torch.float64)
    mom = torch.stack([torch.broadcast_to(torch.as_tensor(mj.mj_tensor_moment(g, n, T, U, quad.m, quad.d),
                                                          dtype=torch.float64), n.shape)
                       for g in basis.gens])
    C = torch.as_tensor(basis.C, dtype=torch.float64)
    return torch.einsum("kv,v...->k...", C, mom)


def equilibrium(basis: Basis, n, T, U):
    """f^eq_i = w_i sum_k a^(k) J^(k)(p_i)  (Eq. mj-discrete-feq); shape (Q, ...)."""
    a = projection_coefficients(basis, n, T, U)
    J = torch.as_tensor(basis.J, dtype=torch.float64)
    w = torch.as_tensor(basis.quad.w, dtype=torch.float64)
    feq = torch.einsum("kq,k...->q...", J, a)
    return w.reshape((-1,) + (1,) * (feq.dim() - 1)) * feq

"""Generating function of the bin counts and the wrapped distribution (oracle;
test infrastructure only).

By Eq. Lamb_lhaf_master multiplied by the vacuum probability (the step from
Eq. Lamb_lhaf_def to Eq. coarse_grained_prob), the probability generating
function of the bin counts b is

    G(w) = sum_b Pr(b) prod_l w_l^{b_l} = Pr(0) q(A, gamma, z(w)),

where z_i = w_l for every mode i in bin l (Eq. change_in_product) and z_i = 1
for a mode that is not measured (summing over its photon number), and q is the
closed form of Eq. q_d:

    q = exp(1/2 gamma^T [I - D X A]^-1 D X gamma) / sqrt(det[I - D X A]),
    D = diag(z) (+) diag(z).

The square root is the branch continuous from z = 0, where the determinant is 1.
Here it is fixed through the eigenvalues lambda_i of D X A: log det = sum_i
Log(1 - lambda_i) with principal logarithms.  For a physical state ||X A||_2 < 1
(X A = I - Sigma^-1 and Sigma > I/2), so for |z_i| <= 1 every |lambda_i| < 1,
each factor 1 - t lambda_i stays in the right half-plane along t in [0, 1], and
the principal logarithms are the continuous ones.

The coefficients are extracted with the finite-difference sieve of Sec. V
taking the nodes to be the G_l-th roots of unity (the node freedom stated
there): the explicit inverse DFT

    P_wrap(b) = (1 / prod_l G_l) sum_k G(w_k) prod_l w_{k,l}^{-b_l},
    w_{k,l} = exp(2 pi i k_l / G_l),

returns sum over m >= 0 of Pr(b + m o G), which is Pr(b) up to the probability
mass beyond the grid (the 'wrap').
"""
from __future__ import annotations

import itertools

import numpy as np

from . import state as st


def log_q(A, gamma, z) -> complex:
    """log q(A, gamma, z) of Eq. q_d with the continuous branch (eigenvalues)."""
    n2 = A.shape[0]
    X = st.xmat(n2 // 2)
    D = np.diag(np.concatenate([z, z]))
    DXA = D @ X @ A
    lam = np.linalg.eigvals(DXA)
    logdet = np.sum(np.log(1.0 - lam))
    expo = 0.5 * gamma @ np.linalg.solve(np.eye(n2) - DXA, D @ X @ gamma)
    return expo - 0.5 * logdet


def z_of_w(bins, w) -> np.ndarray:
    """Broadcast the bin variables to the fine modes (1 for unmeasured modes)."""
    w_ext = np.concatenate([np.asarray(w, dtype=np.complex128), [1.0 + 0j]])
    return w_ext[np.where(bins < 0, len(w), bins)]


def log_pgf(S, w) -> complex:
    """log G(w) for an assembled state S (see state.assemble)."""
    return np.log(S["pr0"]) + log_q(S["A"], S["gamma"], z_of_w(S["bins"], w))


def grid_values(S, grid) -> np.ndarray:
    """G(w_k) at every point of the roots-of-unity grid, shape tuple(grid)."""
    grid = [int(g) for g in grid]
    out = np.empty(grid, dtype=np.complex128)
    for k in itertools.product(*[range(g) for g in grid]):
        w = np.exp(2j * np.pi * np.array(k) / np.array(grid))
        out[k] = np.exp(log_pgf(S, w))
    return out


def inverse_dft(values, cutoff) -> np.ndarray:
    """P(b) = (1/prod G) sum_k values[k] prod_l exp(-2 pi i k_l b_l / G_l) for b in
    the box [0, cutoff_l]; one explicit DFT matrix per axis (a plain matrix
    product per axis).  Returns the complex result (its imaginary part is
    rounding noise for a real distribution)."""
    out = values.astype(np.complex128)
    for ax, (g, nmax) in enumerate(zip(values.shape, cutoff)):
        k = np.arange(g)
        b = np.arange(int(nmax) + 1)
        F = np.exp(-2j * np.pi * np.outer(b, k) / g) / g  # (N+1) x G
        out = np.moveaxis(np.tensordot(F, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def wrapped_distribution(inst, grid=None, return_imag=False):
    """P_wrap on the instance's grid (or `grid`), over the box [0, cutoff]."""
    S = st.assemble(inst)
    g = inst["grid"] if grid is None else grid
    P = inverse_dft(grid_values(S, g), inst["cutoff"])
    return (P.real, np.abs(P.imag).max()) if return_imag else P.real

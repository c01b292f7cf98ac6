"""Gradients of the wrapped distribution by torch autograd (oracle; test
infrastructure only).

The same formulas as state.py and pgf.py, written with torch complex128
tensors on the CPU so that autograd can differentiate the probabilities with
respect to the squeezing parameters r, the transfer matrix T, the
displacements alpha and the Schmidt weights lambda (each weight a free
variable: the state depends on them through lambda_k / lambda_0 only,
Eq. relation_between_sqz_par generalised to K modes), through Sec. II (Sigma,
A = X(I - Sigma^-1), gamma = X Sigma^-1 zbar, vacuum probability), Eq. q_d,
Eq. Lamb_lhaf_master and the explicit inverse DFT.

log det[I - D X A] is evaluated for its value through the eigenvalues (the
continuous branch, see pgf.py) and for its derivative through torch's
slogdet: the two differ by a constant 2 pi i m, which has no derivative.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

CT = torch.complex128


def _internal_r(r, schmidt):
    if schmidt is None:
        return r[:, None]
    lam = schmidt if isinstance(schmidt, torch.Tensor) else torch.as_tensor(np.asarray(schmidt), dtype=torch.float64)
    ratio = lam / lam[0]
    return torch.atanh(torch.sqrt(ratio)[None, :] * torch.tanh(r)[:, None])


def _xmat(n):
    Z = torch.zeros((n, n), dtype=CT)
    I = torch.eye(n, dtype=CT)
    return torch.cat([torch.cat([Z, I], 1), torch.cat([I, Z], 1)], 0)


def _state(T, r, alpha, schmidt):
    M = T.shape[0]
    rk = _internal_r(r, schmidt)
    K = rk.shape[1]
    Tf = torch.kron(T, torch.eye(K, dtype=CT))
    n_in = (torch.sinh(rk) ** 2).reshape(-1).to(CT)
    m_in = (torch.sinh(rk) * torch.cosh(rk)).reshape(-1).to(CT)
    N = Tf.conj() @ torch.diag(n_in) @ Tf.T
    Mm = Tf @ torch.diag(m_in) @ Tf.T
    a_in = torch.zeros(M * K, dtype=CT)
    if alpha is not None:
        idx = torch.arange(M) * K
        a_in = a_in.index_put((idx,), alpha)
    beta = Tf @ a_in
    n = M * K
    Sigma = torch.eye(2 * n, dtype=CT) + torch.cat([torch.cat([N.T, Mm], 1), torch.cat([Mm.conj(), N], 1)], 0)
    zbar = torch.cat([beta, beta.conj()])
    X = _xmat(n)
    Sinv = torch.linalg.inv(Sigma)
    A = X @ (torch.eye(2 * n, dtype=CT) - Sinv)
    gamma = X @ Sinv @ zbar
    B = torch.eye(2 * n, dtype=CT) - X @ A
    log_pr0 = -0.5 * gamma @ torch.linalg.solve(B, X @ gamma) + 0.5 * torch.logdet(B)
    return A, gamma, log_pr0, X


def wrapped_distribution_torch(T, r, alpha, inst, schmidt=None):
    """P_wrap for the instance's binning, differentiable in (T, r, alpha) and,
    when given as a tensor, in the Schmidt weights."""
    if schmidt is None:
        schmidt = inst.get("schmidt")
    A, gamma, log_pr0, X = _state(T, r, alpha, schmidt)
    M = T.shape[0]
    K = 1 if schmidt is None else len(schmidt)
    b = np.asarray(inst["bin_of"], dtype=np.int64)
    bins = b if inst.get("resolve_internal", 0) else np.repeat(b, K)
    grid = [int(g) for g in inst["grid"]]
    cutoff = [int(c) for c in inst["cutoff"]]
    n2 = A.shape[0]
    vals = []
    XA = X @ A
    for k in itertools.product(*[range(g) for g in grid]):
        w = np.exp(2j * np.pi * np.array(k) / np.array(grid))
        z = np.concatenate([w, [1.0]])[np.where(bins < 0, len(w), bins)]
        d = torch.as_tensor(np.concatenate([z, z]), dtype=CT)
        S = torch.eye(n2, dtype=CT) - d[:, None] * XA
        lam = np.linalg.eigvals(np.diag(np.concatenate([z, z])) @ XA.detach().numpy())
        branch = complex(np.sum(np.log(1.0 - lam)))
        sign, logabs = torch.linalg.slogdet(S)
        ld_grad = logabs.to(CT) + torch.log(sign)
        logdet = ld_grad + (branch - ld_grad.detach())
        expo = 0.5 * gamma @ torch.linalg.solve(S, d * (X @ gamma))
        vals.append(torch.exp(log_pr0 + expo - 0.5 * logdet))
    Gv = torch.stack(vals).reshape(grid)
    out = Gv
    for ax, (g, nmax) in enumerate(zip(grid, cutoff)):
        kk = np.arange(g)
        bb = np.arange(nmax + 1)
        F = torch.as_tensor(np.exp(-2j * np.pi * np.outer(bb, kk) / g) / g, dtype=CT)
        out = torch.movedim(torch.tensordot(F, torch.movedim(out, ax, 0), dims=([1], [0])), 0, ax)
    return out.real


def gradients_full(inst, dP):
    """Gradient of L = sum_b dP(b) P_wrap(b): dict with r (dL/dr), T and alpha
    (dL/dRe x + i dL/dIm x), schmidt (dL/dlambda_k, each weight free; None for
    K = 1) and P."""
    T = torch.tensor(np.asarray(inst["T"]), dtype=CT, requires_grad=True)
    r = torch.tensor(np.asarray(inst["r"]), dtype=torch.float64, requires_grad=True)
    alpha = None
    if inst.get("alpha") is not None:
        alpha = torch.tensor(np.asarray(inst["alpha"]), dtype=CT, requires_grad=True)
    lam = None
    if inst.get("schmidt") is not None:
        lam = torch.tensor(np.asarray(inst["schmidt"]), dtype=torch.float64, requires_grad=True)
    P = wrapped_distribution_torch(T, r, alpha, inst, schmidt=lam)
    L = (P * torch.as_tensor(np.asarray(dP), dtype=torch.float64)).sum()
    L.backward()
    return dict(r=r.grad.numpy(), T=T.grad.numpy(), alpha=None if alpha is None else alpha.grad.numpy(),
                schmidt=None if lam is None else lam.grad.numpy(), P=P.detach().numpy())


def gradients(inst, dP):
    """dL/dr, dL/dRe T + i dL/dIm T, dL/dRe alpha + i dL/dIm alpha for
    L = sum_b dP(b) P_wrap(b)."""
    g = gradients_full(inst, dP)
    return g["r"], g["T"], g["alpha"], g["P"]

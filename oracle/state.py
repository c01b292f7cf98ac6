"""Gaussian-state assembly (oracle; test infrastructure only).

Follows Sec. II of the paper: the mode vector zeta = (a_1..a_m, a_1^dag..a_m^dag),
the covariance matrix Sigma = Sigma^(s=-1) (Eq. covariance_matrix) in the valid
form I + [[N^T, M],[M^*, N]] with N_ij = <a_i^dag a_j>, M_ij = <a_i a_j> taken
about the means, the vector of means (Eq. vector_of_means), the adjacency matrix
A = X (I - Sigma^-1) (Eq. defA), the loop vector gamma = X Sigma^-1 zbar
(Eq. defgamma) and the vacuum probability (Eq. vacuum_probability).

Internal modes (Sec. VI B, Sec. VIII A): every external input j carries K
internal (Schmidt) modes, ordered external-major (index j*K + k,
Eq. internal_mode_detection_pattern); the interferometer acts identically on
each internal mode (T tensor I_K); only internal mode 0 is displaced.  The
squeezing of internal mode k follows the paper's two-mode relation
(Eq. relation_between_sqz_par) generalised to K modes:
tanh^2 r_jk = (lambda_k / lambda_0) tanh^2 r_j.

Fully distinguishable inputs (App. D: spectrally orthogonal single-mode
squeezed states interfering in the circuit): K = M internal modes, input j
squeezed by r_j in internal mode j only (r_jk = r_j delta_jk), instance key
"distinguishable".

Everything is dense complex128 over all 2MK quadrature indices; no block
structure is exploited here.
"""
from __future__ import annotations

import numpy as np


def squeezing_per_internal_mode(r: np.ndarray, schmidt) -> np.ndarray:
    """M x K squeezing parameters; column 0 is r itself."""
    r = np.asarray(r, dtype=np.float64)
    if schmidt is None:
        return r[:, None].copy()
    lam = np.asarray(schmidt, dtype=np.float64)
    ratio = lam / lam[0]
    return np.arctanh(np.sqrt(ratio)[None, :] * np.tanh(r)[:, None])


def n_internal(inst) -> int:
    """K of an instance: M for fully distinguishable inputs, else len(schmidt) (1 if none)."""
    if inst.get("distinguishable", 0):
        return np.asarray(inst["T"]).shape[0]
    return 1 if inst.get("schmidt") is None else len(inst["schmidt"])


def output_moments(T, r, alpha=None, schmidt=None, distinguishable=False):
    """Normally ordered moments of the output modes.

    Inputs are single-mode squeezed vacua S(r)|0> (S(xi) = exp[(xi a^dag^2 -
    xi^* a^2)/2], App. B) displaced by alpha on internal mode 0.  A passive
    lossy interferometer maps a_out = T a_in + (vacuum noise), so with
    n_in = <a^dag a> = sinh^2 r and m_in = <a a> = sinh r cosh r:
        N = <a^dag a>_out = T^* diag(n_in) T^T,  M = <a a>_out = T diag(m_in) T^T,
        beta = <a>_out = T alpha.
    Returns (N, M, beta) over the M*K output modes, external-major."""
    T = np.asarray(T, dtype=np.complex128)
    m = T.shape[0]
    if distinguishable:
        assert schmidt is None and alpha is None
        rk = np.diag(np.asarray(r, dtype=np.float64))  # r_jk = r_j delta_jk
    else:
        rk = squeezing_per_internal_mode(r, schmidt)
    K = rk.shape[1]
    Tfull = np.kron(T, np.eye(K))  # a_out[i*K+k] = sum_j T[i,j] a_in[j*K+k]
    n_in = np.sinh(rk).ravel() ** 2
    m_in = (np.sinh(rk) * np.cosh(rk)).ravel()
    N = Tfull.conj() @ np.diag(n_in) @ Tfull.T
    Mm = Tfull @ np.diag(m_in) @ Tfull.T
    a_in = np.zeros(m * K, dtype=np.complex128)
    if alpha is not None:
        a_in[0::K] = alpha
    beta = Tfull @ a_in
    return N, Mm, beta


def covariance_and_means(N, Mm, beta):
    """Sigma = I + [[N^T, M],[M^*, N]] and zbar = (beta, beta^*) (Sec. II)."""
    n = N.shape[0]
    Sigma = np.eye(2 * n, dtype=np.complex128) + np.block([[N.T, Mm], [Mm.conj(), N]])
    zbar = np.concatenate([beta, beta.conj()])
    return Sigma, zbar


def xmat(n: int) -> np.ndarray:
    """X = [[0, I],[I, 0]] for n modes (Eq. x_matrix_husimi_cov)."""
    Z = np.zeros((n, n))
    I = np.eye(n)
    return np.block([[Z, I], [I, Z]]).astype(np.complex128)


def adjacency(Sigma, zbar):
    """A = X (I - Sigma^-1), gamma = X Sigma^-1 zbar (Eqs. defA, defgamma)."""
    n2 = Sigma.shape[0]
    X = xmat(n2 // 2)
    Sinv = np.linalg.inv(Sigma)
    A = X @ (np.eye(n2) - Sinv)
    gamma = X @ Sinv @ zbar
    return A, gamma


def vacuum_probability(A, gamma) -> complex:
    """Pr(0) = exp(-1/2 gamma^T [I - X A]^-1 X gamma) sqrt(det(I - X A))
    (Eq. vacuum_probability).  Returned as a complex number whose imaginary part
    is rounding noise."""
    n2 = A.shape[0]
    X = xmat(n2 // 2)
    B = np.eye(n2) - X @ A
    expo = -0.5 * gamma @ np.linalg.solve(B, X @ gamma)
    return np.exp(expo) * np.sqrt(np.linalg.det(B))


def marginal(Sigma, zbar, keep):
    """Reduced Gaussian state of the modes in `keep` (partial trace of a
    Gaussian state keeps the corresponding rows/columns of Sigma and entries of
    zbar, in both the a and a^dag halves)."""
    n = Sigma.shape[0] // 2
    keep = np.asarray(keep, dtype=np.int64)
    idx = np.concatenate([keep, keep + n])
    return Sigma[np.ix_(idx, idx)], zbar[idx]


def fine_bins(inst) -> np.ndarray:
    """Bin index for each of the M*K fine (internal-resolved) modes."""
    M = inst["T"].shape[0]
    K = n_internal(inst)
    b = np.asarray(inst["bin_of"], dtype=np.int64)
    if inst.get("resolve_internal", 0):
        assert b.shape[0] == M * K
        return b.copy()
    assert b.shape[0] == M
    return np.repeat(b, K)


def assemble(inst):
    """Full dense state of an instance: dict with Sigma, zbar, A, gamma, pr0,
    and the per-fine-mode bin index."""
    N, Mm, beta = output_moments(inst["T"], inst["r"], inst.get("alpha"), inst.get("schmidt"),
                                 bool(inst.get("distinguishable", 0)))
    Sigma, zbar = covariance_and_means(N, Mm, beta)
    A, gamma = adjacency(Sigma, zbar)
    pr0 = vacuum_probability(A, gamma)
    return dict(Sigma=Sigma, zbar=zbar, A=A, gamma=gamma, pr0=pr0, N=N, M=Mm, beta=beta,
                bins=fine_bins(inst))

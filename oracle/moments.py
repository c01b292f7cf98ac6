"""Coarse-grained joint moments and cumulants (oracle; test infrastructure only).

Definitions (Sec. VI C, Eqs. CGmom and CGmom2, with the bin counts b_l raised
to powers p_l): the joint moment is E[prod_l b_l^{p_l}] = sum_b prod_l
b_l^{p_l} Pr(b), summed over the distribution itself; the joint cumulant of
the multiset of variables in which b_l appears p_l times follows from the
moments by the partition formula

    <<X_1 ... X_n>> = sum over set partitions pi of {1..n} of
                      (|pi| - 1)! (-1)^(|pi| - 1) prod_{B in pi} E[prod_{i in B} X_i].

Exact cumulants without summing over a distribution (cumulants_series): the
moment generating function of Eq. M, with one shared variable t_l per bin,

    log M(t) = -1/2 log det(I - G R) + 1/2 zbar^H (I - G R)^-1 G zbar,
    G = sum_l u_l P_l,  u_l = e^{t_l} - 1,  R = Sigma^(s=1),

(P_l the projector on the rows of bin l, both halves) expands as
1/2 sum_{k>=1} tr((G R)^k) / k + 1/2 sum_{k>=0} zbar^H (G R)^k G zbar, a power
series in u whose coefficients are sums over words of bin labels of
tr(P_l1 R ... P_lk R) and zbar^H P_l0 R P_l1 ... R P_lk zbar.  With
(e^t - 1)^m = sum_n m! S(n, m) t^n / n! (S the Stirling numbers of the second
kind), the cumulant of powers p is <<b^p>> = sum_q a_q prod_l S(p_l, q_l) q_l!.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import pgf


def oversampled_distribution(inst, G: int) -> np.ndarray:
    """Pr(b) for b_l < G on a G^L grid (the wrapped distribution, whose wrap is
    the mass at b_l >= G)."""
    x = dict(inst)
    L = len(inst["cutoff"])
    x["grid"] = np.full(L, G, np.int32)
    x["cutoff"] = np.full(L, G - 1, np.int32)
    return pgf.wrapped_distribution(x)


def joint_moments(P: np.ndarray, orders) -> np.ndarray:
    """E[prod_l b_l^{p_l}] for p_l in [0, orders_l], from a distribution P
    indexed by the bin counts."""
    out = np.zeros(tuple(int(o) + 1 for o in orders))
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in P.shape], indexing="ij")
    for p in itertools.product(*[range(int(o) + 1) for o in orders]):
        w = np.ones_like(P)
        for g, e in zip(grids, p):
            w = w * g ** e
        out[p] = float((w * P).sum())
    return out


def _set_partitions(items):
    """All partitions of a list into non-empty blocks."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        yield [[first]] + part
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]


def joint_cumulants(mom: np.ndarray) -> np.ndarray:
    """Joint cumulants <<prod_l b_l^{p_l}>> (each b_l repeated p_l times) from
    the joint moments of the same box, by the partition formula."""
    out = np.zeros_like(mom)
    L = mom.ndim
    for p in itertools.product(*[range(n) for n in mom.shape]):
        labels = [l for l in range(L) for _ in range(p[l])]
        if not labels:
            out[p] = 0.0
            continue
        total = 0.0
        for part in _set_partitions(list(range(len(labels)))):
            term = float((-1) ** (len(part) - 1) * math.factorial(len(part) - 1))
            for block in part:
                q = [0] * L
                for i in block:
                    q[labels[i]] += 1
                term *= mom[tuple(q)]
            total += term
        out[p] = total
    return out


def moments_from_cumulants(cum: np.ndarray) -> np.ndarray:
    """Inverse of joint_cumulants: E[X_1..X_n] = sum_pi prod_{B in pi} <<X_B>>."""
    out = np.zeros_like(cum)
    L = cum.ndim
    for p in itertools.product(*[range(n) for n in cum.shape]):
        labels = [l for l in range(L) for _ in range(p[l])]
        if not labels:
            out[p] = 1.0
            continue
        total = 0.0
        for part in _set_partitions(list(range(len(labels)))):
            term = 1.0
            for block in part:
                q = [0] * L
                for i in block:
                    q[labels[i]] += 1
                term *= cum[tuple(q)]
            total += term
        out[p] = total
    return out


def _stirling2(n: int, m: int) -> int:
    """Stirling number of the second kind S(n, m) (partitions of n items into m blocks)."""
    S = [[0] * (m + 1) for _ in range(n + 1)]
    S[0][0] = 1
    for i in range(1, n + 1):
        for j in range(1, min(i, m) + 1):
            S[i][j] = j * S[i - 1][j] + S[i - 1][j - 1]
    return S[n][m]


def cumulants_series(inst, orders) -> np.ndarray:
    """Joint cumulants <<prod_l b_l^{p_l}>> for p_l in [0, orders_l] from the
    series of log M (Eq. M); dense over all 2MK quadrature indices."""
    from . import state as st
    S = st.assemble(inst)
    Sigma, zbar, bins = S["Sigma"], S["zbar"], S["bins"]
    n2 = Sigma.shape[0]
    R = Sigma - np.eye(n2)
    rb = np.concatenate([bins, bins])
    L = len(inst["cutoff"])
    proj = [np.diag((rb == l).astype(np.float64)) for l in range(L)]
    PR = [Pl @ R for Pl in proj]
    orders = [int(o) for o in orders]
    pmax = sum(orders)
    a = np.zeros(tuple(o + 1 for o in orders), dtype=np.complex128)  # coefficients of u^q
    # words of length k over the bin labels with letter counts q (q <= orders)
    for k in range(1, pmax + 1):
        for word in itertools.product(range(L), repeat=k):
            q = [0] * L
            for l in word:
                q[l] += 1
            if any(qi > oi for qi, oi in zip(q, orders)):
                continue
            # 1/2 tr(P_l1 R ... P_lk R) / k
            Mw = np.eye(n2, dtype=np.complex128)
            for l in word:
                Mw = Mw @ PR[l]
            a[tuple(q)] += 0.5 * np.trace(Mw) / k
            # 1/2 zbar^H P_l1 R P_l2 R ... R P_lk zbar  (k letters, k - 1 factors R)
            v = proj[word[-1]] @ zbar
            for l in reversed(word[:-1]):
                v = PR[l] @ v
            a[tuple(q)] += 0.5 * (zbar.conj() @ v)
    out = np.zeros(a.shape)
    for p in itertools.product(*[range(o + 1) for o in orders]):
        tot = 0.0
        for q in itertools.product(*[range(pi + 1) for pi in p]):
            c = a[q].real
            if c == 0.0:
                continue
            f = 1.0
            for pi, qi in zip(p, q):
                f *= _stirling2(pi, qi) * math.factorial(qi)
            tot += c * f
        out[p] = tot
    return out

"""Heralded density matrices (Sec. VII) -- oracle; test infrastructure only.

Modes of an instance are the fine (internal-resolved) modes of state.py.
Each is a heralding mode in one of the L bins (bin index >= 0), traced out
(-1) or kept (KEEP = -2); the kept modes carry the heralded state.  For a
heralding pattern b~ in the box the unnormalised heralded state is the
partial trace of the projector onto every compatible fine pattern
(Eq. projector_onto_heralding_outcome, Eq. heralded_state_internal):

    <v| rho(b~) |u>  =  sum_{n~ in K(b~)} <n~, v| rho |n~, u>,

with u, v Fock patterns of the kept modes (instance order of the fine
modes), each entry in [0, N], N = fock_cutoff.  Modes traced out are removed
first: the partial trace of a Gaussian state is the Gaussian state of the
remaining modes, with their rows and columns of Sigma and entries of zbar
(state.marginal).  A matrix element of the remaining state is Eq. lhaf_offd,

    <m| rho |n>  =  Pr(0) lhaf(A_{n (+) m}, gamma_{n (+) m}) / prod_k sqrt(n_k! m_k!),

the first half of the indices carrying the ket pattern n and the second the
bra pattern m.  Output of every route: a complex array of shape
(N_1+1, ..., N_L+1, D, D), D = (N+1)^g, entry [b~][v][u] = <v|rho(b~)|u>,
the multi-indices u, v row-major over the kept modes (last one fastest).

Routes:
* density_brute: Eq. lhaf_heralded_offd_internal_1 term by term, the loop
  hafnians by the brute-force matching recursion of lhaf.c.  Tiny cases.
* density_taylor: every matrix element of the reduced state up to the
  photon numbers needed, as Taylor coefficients.  A loop hafnian of a matrix
  with repeated indices is the mixed derivative
      lhaf(A_s, gamma_s) = d^s / dc^s  exp(1/2 c^T A c + gamma^T c)  at c = 0
  (each term of the expansion of the exponential is one single-pair
  matching of the repeated indices), so the coefficient of c^s is
  lhaf(A_s, gamma_s) / s!.  taylor_coefficients solves
  d f / d c_0 = (gamma_0 + sum_j A_0j c_j) f order by order in c_0.
* density_pure: for a pure state (no loss, K = 1, nothing traced) the block
  A_{n(+)m} has no entries between the halves, the element factorises as
  psi_m conj(psi_n), and psi comes from the Taylor coefficients of the
  bra-side block alone (M indices instead of 2M).

All three are pinned in tests/test_oracle_density.py (closed forms, the
brute-force definition, the joint photon-number distribution of pgf.py).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import brute
from . import state as st

KEEP = -2
TRACED = -1


def taylor_coefficients(A, g, caps) -> np.ndarray:
    """Coefficients a[s] of exp(1/2 c^T A c + g^T c) (A symmetric) for
    0 <= s_i <= caps[i]; complex array of shape caps + 1.

    With f the exponential, df/dc_0 = (g_0 + sum_j A_0j c_j) f; comparing the
    coefficients of c_0^(t-1) c_rest^r on both sides,
        t a[t, r] = g_0 a[t-1, r] + A_00 a[t-2, r] + sum_{j>0} A_0j a[t-1, r - e_j],
    and a[0, :] is the same expansion with c_0 = 0 (one variable fewer)."""
    A = np.asarray(A, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    caps = [int(c) for c in caps]
    d = len(caps)
    if d == 0:
        return np.ones((), dtype=np.complex128)
    rest = taylor_coefficients(A[1:, 1:], g[1:], caps[1:])
    out = np.zeros((caps[0] + 1,) + rest.shape, dtype=np.complex128)
    out[0] = rest
    for t in range(1, caps[0] + 1):
        prev = out[t - 1]
        acc = g[0] * prev
        if t >= 2:
            acc = acc + A[0, 0] * out[t - 2]
        for j in range(1, d):
            if caps[j] == 0:
                continue
            shifted = np.zeros_like(prev)
            dst = [slice(None)] * (d - 1)
            src = [slice(None)] * (d - 1)
            dst[j - 1] = slice(1, caps[j] + 1)
            src[j - 1] = slice(0, caps[j])
            shifted[tuple(dst)] = prev[tuple(src)]
            acc = acc + A[0, j] * shifted
        out[t] = acc / t
    return out


def _reduced(inst):
    """Reduced state of the heralding and kept modes: (A, gamma, Pr(0), bins
    of the remaining fine modes)."""
    S = st.assemble(inst)
    bins = S["bins"]
    rem = np.nonzero(bins != TRACED)[0]
    Sig, zb = st.marginal(S["Sigma"], S["zbar"], rem)
    A, gamma = st.adjacency(Sig, zb)
    pr0 = st.vacuum_probability(A, gamma)
    return A, gamma, pr0, bins[rem]


def _heralding_patterns(bins, cutoff):
    """For every b~ in the box: the list of fine heralding patterns n~ (one
    count per heralding mode, in mode order) compatible with it."""
    her = np.nonzero(bins >= 0)[0]
    members = [np.nonzero(bins[her] == l)[0] for l in range(len(cutoff))]
    out = {}
    for b in itertools.product(*[range(int(c) + 1) for c in cutoff]):
        per_bin = [list(brute._compositions(b[l], len(members[l]))) if len(members[l]) else
                   ([()] if b[l] == 0 else []) for l in range(len(cutoff))]
        pats = []
        for combo in itertools.product(*per_bin):
            n = np.zeros(len(her), dtype=np.int64)
            for l in range(len(cutoff)):
                n[members[l]] = combo[l]
            pats.append(n)
        out[b] = pats
    return her, out


def _kept_patterns(g, N):
    return list(itertools.product(range(N + 1), repeat=g))


def density_brute(inst) -> np.ndarray:
    """Eq. lhaf_heralded_offd_internal_1 with brute-force loop hafnians."""
    N = int(inst["fock_cutoff"])
    cutoff = [int(c) for c in inst["cutoff"]]
    A, gamma, pr0, bins = _reduced(inst)
    keep = np.nonzero(bins == KEEP)[0]
    g = len(keep)
    D = (N + 1) ** g
    her, pats = _heralding_patterns(bins, cutoff)
    n_modes = len(bins)
    kp = _kept_patterns(g, N)
    out = np.zeros([c + 1 for c in cutoff] + [D, D], dtype=np.complex128)
    for b, plist in pats.items():
        for vi, v in enumerate(kp):
            for ui, u in enumerate(kp):
                acc = 0j
                for n in plist:
                    ket = np.zeros(n_modes, dtype=np.int32)
                    bra = np.zeros(n_modes, dtype=np.int32)
                    ket[her] = n
                    bra[her] = n
                    ket[keep] = u
                    bra[keep] = v
                    lh = brute.lhaf_multiset(A, gamma, np.concatenate([ket, bra]))
                    acc += lh / np.prod([math.factorial(int(x)) for x in n])
                fu = np.prod([math.factorial(x) for x in u])
                fv = np.prod([math.factorial(x) for x in v])
                out[b + (vi, ui)] = pr0 * acc / math.sqrt(fu * fv)
    return out


def density_taylor(inst) -> np.ndarray:
    """Every element <n~, v|rho|n~, u> from the Taylor coefficients of the
    generating function of the reduced state, summed over K(b~)."""
    N = int(inst["fock_cutoff"])
    cutoff = [int(c) for c in inst["cutoff"]]
    A, gamma, pr0, bins = _reduced(inst)
    n_modes = len(bins)
    keep = np.nonzero(bins == KEEP)[0]
    g = len(keep)
    D = (N + 1) ** g
    caps_half = [cutoff[b] if b >= 0 else N for b in bins]
    a = taylor_coefficients(A, gamma, caps_half + caps_half)
    her, pats = _heralding_patterns(bins, cutoff)
    fact = np.array([math.factorial(k) for k in range(N + 1)], dtype=np.float64)
    # sqrt(u! v!) over the kept multi-indices, [v][u]
    fk = np.ones([N + 1] * g)
    for j in range(g):
        shape = [1] * g
        shape[j] = N + 1
        fk = fk * fact.reshape(shape)
    sq = np.sqrt(np.outer(fk.ravel(), fk.ravel()))
    out = np.zeros([c + 1 for c in cutoff] + [D, D], dtype=np.complex128)
    for b, plist in pats.items():
        acc = np.zeros((D, D), dtype=np.complex128)
        for n in plist:
            idx = [slice(None)] * (2 * n_modes)
            for pos, cnt in zip(her, n):
                idx[pos] = int(cnt)
                idx[n_modes + pos] = int(cnt)
            sub = a[tuple(idx)]  # axes: kept ket modes, then kept bra modes
            ket_bra = sub.reshape(D, D)  # [u][v]
            # <n~,v|rho|n~,u> = Pr(0) lhaf / sqrt((n~,u)! (n~,v)!) = Pr(0) a n~! sqrt(u! v!)
            nf = np.prod([math.factorial(int(x)) for x in n])
            acc += ket_bra.T * nf
        out[b] = pr0 * acc * sq
    return out


def density_pure(inst) -> np.ndarray:
    """As density_taylor for a pure state, from the amplitudes
    psi_m = sqrt(Pr(0)) lhaf(A_bb m, gamma_b m) / sqrt(m!) of the bra-side
    block (the ket side is their complex conjugate, up to one common phase
    that cancels in psi_m conj(psi_n))."""
    N = int(inst["fock_cutoff"])
    cutoff = [int(c) for c in inst["cutoff"]]
    A, gamma, pr0, bins = _reduced(inst)
    n_modes = len(bins)
    cross = A[:n_modes, n_modes:]
    if np.abs(cross).max() > 1e-12 * max(1.0, np.abs(A).max()):
        raise ValueError("density_pure needs a pure state (A has entries between the halves)")
    keep = np.nonzero(bins == KEEP)[0]
    g = len(keep)
    D = (N + 1) ** g
    caps = [cutoff[b] if b >= 0 else N for b in bins]
    Ab = A[n_modes:, n_modes:]
    gb = gamma[n_modes:]
    a = taylor_coefficients(Ab, gb, caps)
    # psi = sqrt(Pr(0)) a sqrt(m!) (Pr(0) real positive)
    for j in range(n_modes):
        shape = [1] * n_modes
        shape[j] = caps[j] + 1
        a = a * np.sqrt(np.array([math.factorial(k) for k in range(caps[j] + 1)], dtype=np.float64)).reshape(shape)
    psi = math.sqrt(pr0.real) * a
    her, pats = _heralding_patterns(bins, cutoff)
    out = np.zeros([c + 1 for c in cutoff] + [D, D], dtype=np.complex128)
    for b, plist in pats.items():
        acc = np.zeros((D, D), dtype=np.complex128)
        for n in plist:
            idx = [slice(None)] * n_modes
            for pos, cnt in zip(her, n):
                idx[pos] = int(cnt)
            vec = psi[tuple(idx)].reshape(D)
            acc += np.outer(vec, vec.conj())  # [v][u] = psi_(n~,v) conj(psi_(n~,u))
        out[b] = acc
    return out

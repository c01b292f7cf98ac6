"""Exact box probabilities by brute force (oracle; test infrastructure only).

Pr(b) = sum over fine patterns s compatible with b of Pr(s)  (Eq. coarse_grained_prob,
first line; with internal modes Eq. prob_internal_modes), where each fine
probability is Eq. gbs_probability_distribution:

    Pr(s) = Pr(0) lhaf(filldiag(A_{s(+)s}, gamma_{s(+)s})) / prod_i s_i!.

Modes that are not measured are removed first by taking the marginal
(reduced) Gaussian state of the measured modes, so every sum here is finite.
Feasible only for small photon numbers (the loop hafnian is exponential).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess

import numpy as np

from . import state as st

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblhaf_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile lhaf.c with gcc into oracle/liblhaf_oracle.so."""
    src = os.path.join(_HERE, "lhaf.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", _SO, src])
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_lhaf_multiset.restype = ctypes.c_int
        lib.oracle_lhaf_multiset.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def lhaf_multiset(A, g, mult) -> complex:
    """lhaf(filldiag(A_mult, g_mult)) where vertex type t is repeated mult[t] times."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    g = np.ascontiguousarray(g, dtype=np.complex128)
    mult = np.ascontiguousarray(mult, dtype=np.int32)
    keep = np.nonzero(mult)[0]
    if keep.size == 0:
        return 1.0 + 0j
    A = np.ascontiguousarray(A[np.ix_(keep, keep)])
    g = np.ascontiguousarray(g[keep])
    mult = np.ascontiguousarray(mult[keep])
    out = np.zeros(2)
    rc = _load().oracle_lhaf_multiset(len(keep), A.ctypes.data, g.ctypes.data, mult.ctypes.data,
                                      out.ctypes.data)
    if rc != 0:
        raise ValueError("loop hafnian too large for the brute-force oracle")
    return complex(out[0], out[1])


def fock_probability(A, gamma, pr0, n) -> complex:
    """Eq. gbs_probability_distribution for a pattern n over the state's modes."""
    n = np.asarray(n, dtype=np.int32)
    mult = np.concatenate([n, n])
    return pr0 * lhaf_multiset(A, gamma, mult) / np.prod([math.factorial(int(x)) for x in n])


def _compositions(total: int, parts: int):
    """All tuples of `parts` non-negative integers summing to `total`."""
    if parts == 1:
        yield (total,)
        return
    for first in range(total + 1):
        for rest in _compositions(total - first, parts - 1):
            yield (first,) + rest


def box_probabilities(inst) -> np.ndarray:
    """Exact Pr(b) for every b in the box [0, cutoff_l], by enumerating fine
    patterns of the measured (internal-resolved) modes."""
    S = st.assemble(inst)
    bins = S["bins"]
    measured = np.nonzero(bins >= 0)[0]
    Sig, zb = st.marginal(S["Sigma"], S["zbar"], measured)
    A, gamma = st.adjacency(Sig, zb)
    pr0 = st.vacuum_probability(A, gamma)
    mbins = bins[measured]
    cutoff = [int(c) for c in inst["cutoff"]]
    L = len(cutoff)
    members = [np.nonzero(mbins == l)[0] for l in range(L)]
    out = np.zeros([c + 1 for c in cutoff])
    for b in itertools.product(*[range(c + 1) for c in cutoff]):
        total = 0j
        per_bin = [list(_compositions(b[l], len(members[l]))) if len(members[l]) else
                   ([()] if b[l] == 0 else []) for l in range(L)]
        for combo in itertools.product(*per_bin):
            n = np.zeros(len(measured), dtype=np.int32)
            for l in range(L):
                n[members[l]] = combo[l]
            total += fock_probability(A, gamma, pr0, n)
        out[b] = total.real
    return out

"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not against the oracle itself: closed forms, brute force, invariants and the
fidelities printed in Sec. VIII A."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute, pgf
from oracle import state as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Loop hafnian (Eq. lhaf_def)
# ---------------------------------------------------------------------------

def _haf_by_permutations(B):
    """Hafnian from its permutation-sum definition: (1/(m! 2^m)) sum over all
    permutations of prod_i B[s(2i), s(2i+1)]."""
    n = B.shape[0]
    if n == 0:
        return 1.0 + 0j
    m = n // 2
    tot = 0j
    for p in itertools.permutations(range(n)):
        prod = 1.0 + 0j
        for i in range(m):
            prod *= B[p[2 * i], p[2 * i + 1]]
        tot += prod
    return tot / (math.factorial(m) * 2 ** m)


def _lhaf_by_subsets(B):
    """Loop hafnian as the sum over the set S of looped vertices of
    prod_{i in S} B_ii times the hafnian of the rest."""
    n = B.shape[0]
    tot = 0j
    for k in range(n + 1):
        for S in itertools.combinations(range(n), k):
            rest = [i for i in range(n) if i not in S]
            if len(rest) % 2:
                continue
            tot += np.prod([B[i, i] for i in S]) * _haf_by_permutations(B[np.ix_(rest, rest)])
    return tot


def test_lhaf_2x2_hand():
    A = np.array([[9.0, 2.0 + 1j], [2.0 + 1j, 7.0]])
    g = np.array([3.0, -1j])
    # matchings of two vertices: {(0,1)} or two loops
    assert abs(brute.lhaf_multiset(A, g, [1, 1]) - ((2 + 1j) + 3 * (-1j))) < 1e-15


def test_hafnian_4x4_hand():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    A = A + A.T
    expect = A[0, 1] * A[2, 3] + A[0, 2] * A[1, 3] + A[0, 3] * A[1, 2]
    assert abs(brute.lhaf_multiset(A, np.zeros(4), [1, 1, 1, 1]) - expect) < 1e-13


def test_lhaf_all_ones_counts_involutions():
    # lhaf of the all-ones n x n matrix counts single-pair matchings with loops,
    # i.e. involutions of n points (OEIS A000085)
    involutions = [1, 1, 2, 4, 10, 26, 76, 232, 764, 2620, 9496]
    for n, cnt in enumerate(involutions):
        assert brute.lhaf_multiset(np.ones((1, 1)), np.ones(1), [n]) == pytest.approx(cnt)
    # the same count with the n vertices split over distinct types
    for split in ([2, 3], [1, 1, 1, 1, 1], [4, 0, 2]):
        n = sum(split)
        t = len(split)
        assert brute.lhaf_multiset(np.ones((t, t)), np.ones(t), split).real == pytest.approx(involutions[n])


def test_lhaf_repeated_rows_vs_permutation_definition():
    rng = np.random.default_rng(1)
    for mult in ([1, 2, 1], [3, 1], [2, 2], [0, 1, 2, 2]):
        t = len(mult)
        A = rng.standard_normal((t, t)) + 1j * rng.standard_normal((t, t))
        A = A + A.T
        g = rng.standard_normal(t) + 1j * rng.standard_normal(t)
        idx = np.repeat(np.arange(t), mult)
        B = A[np.ix_(idx, idx)].copy()
        B[np.diag_indices_from(B)] = g[idx]
        assert abs(brute.lhaf_multiset(A, g, mult) - _lhaf_by_subsets(B)) < 1e-11


def test_lhaf_scaling_and_permutation():
    # Eq. lhaf_scaling and Eq. lhafP on an explicit (non-repeated) matrix
    rng = np.random.default_rng(2)
    n = 6
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.T
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    one = np.ones(n, dtype=np.int32)
    base = brute.lhaf_multiset(A, g, one)
    scaled = brute.lhaf_multiset(np.diag(c) @ A @ np.diag(c), c * g, one)
    assert abs(scaled - np.prod(c) * base) < 1e-10 * abs(np.prod(c) * base)
    P = rng.permutation(n)
    assert abs(brute.lhaf_multiset(A[np.ix_(P, P)], g[P], one) - base) < 1e-11


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def _single_mode_squeezed_law(r, nmax):
    p = np.zeros(nmax + 1)
    for n in range(0, nmax + 1, 2):
        m = n // 2
        p[n] = math.factorial(n) / (4 ** m * math.factorial(m) ** 2) * np.tanh(r) ** n / np.cosh(r)
    return p


@pytest.mark.parametrize("r", [0.3, 0.8])
def test_single_mode_squeezed_vacuum_even_law(r):
    inst = W.make_instance(np.eye(1), [r], bin_of=[0], cutoff=[12], grid=[200])
    expect = _single_mode_squeezed_law(r, 12)
    assert np.abs(pgf.wrapped_distribution(inst) - expect).max() < 1e-14
    small = W.make_instance(np.eye(1), [r], bin_of=[0], cutoff=[8])
    assert np.abs(brute.box_probabilities(small) - expect[:9]).max() < 1e-14


def test_lossy_coherent_states_are_poisson_per_bin():
    rng = np.random.default_rng(3)
    M = 4
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    alpha = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    alpha *= 0.8
    bin_of = np.array([0, 1, 1, 0])
    inst = W.make_instance(T, np.zeros(M), alpha=alpha, bin_of=bin_of, cutoff=[6, 6], grid=[48, 48])
    beta = T @ alpha
    mu = [np.sum(np.abs(beta[bin_of == l]) ** 2) for l in range(2)]
    pois = [np.array([np.exp(-m) * m ** k / math.factorial(k) for k in range(7)]) for m in mu]
    expect = np.outer(pois[0], pois[1])
    assert np.abs(pgf.wrapped_distribution(inst) - expect).max() < 1e-14
    small = W.make_instance(T, np.zeros(M), alpha=alpha, bin_of=bin_of, cutoff=[3, 3])
    assert np.abs(brute.box_probabilities(small) - expect[:4, :4]).max() < 1e-14


@pytest.mark.parametrize("k", [1, 3])
def test_thermal_bin_is_negative_binomial(k):
    # A two-mode squeezed vacuum (two equal squeezers on the beamsplitter of
    # Eq. beam_splitter_unitary) leaves each output mode thermal with mean
    # sinh^2 r; tracing the partners and binning k such modes gives the
    # negative binomial law C(b+k-1, b) nbar^b / (1+nbar)^(b+k).
    r = 0.6
    U2 = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    T = np.kron(np.eye(k), U2)
    bin_of = np.tile([0, -1], k)
    inst = W.make_instance(T, np.full(2 * k, r), bin_of=bin_of, cutoff=[10], grid=[96])
    nbar = np.sinh(r) ** 2
    b = np.arange(11)
    expect = np.array([math.comb(x + k - 1, x) for x in b]) * nbar ** b / (1 + nbar) ** (b + k)
    assert np.abs(pgf.wrapped_distribution(inst) - expect).max() < 1e-14


def test_two_mode_squeezed_vacuum_diagonal_law():
    # Sec. VIII A: the beamsplitter of Eq. beam_splitter_unitary on two equal
    # squeezers gives amplitudes chi_n = i^n tanh^n(xi)/cosh(xi), so
    # P(n, m) = delta_nm (1 - x) x^n with x = tanh^2 xi.
    r = 0.7
    U2 = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    inst = W.make_instance(U2, [r, r], bin_of=[0, 1], cutoff=[8, 8], grid=[80, 80])
    x = np.tanh(r) ** 2
    expect = np.diag((1 - x) * x ** np.arange(9))
    assert np.abs(pgf.wrapped_distribution(inst) - expect).max() < 1e-14
    small = W.make_instance(U2, [r, r], bin_of=[0, 1], cutoff=[4, 4])
    assert np.abs(brute.box_probabilities(small) - expect[:5, :5]).max() < 1e-14


# ---------------------------------------------------------------------------
# Brute force vs generating function (whole chain)
# ---------------------------------------------------------------------------

def test_plain_m4_brute_force_matches_oversampled_grid():
    inst = W.plain_m4()
    exact = brute.box_probabilities(inst)
    wrapped = pgf.wrapped_distribution(inst, grid=[40, 40])
    assert np.abs(exact - wrapped).max() < 1e-15
    # on the stated 7x7 grid the result is the wrapped distribution, which
    # exceeds the exact one by at most the mass beyond the grid
    P7 = pgf.wrapped_distribution(inst)
    diff = P7 - exact
    assert diff.min() > -1e-15
    assert diff.max() < 1.0 - exact.sum() + 1e-15


def test_displaced_internal_modes_brute_force():
    rng = W.rng_for(99)
    M, K = 3, 2
    T = np.sqrt(0.6) * W.haar_unitary(M, rng)
    alpha = 0.4 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    inst = W.make_instance(T, rng.uniform(0.2, 0.5, M), alpha=alpha, schmidt=[0.7, 0.3],
                           bin_of=[0, 1, 1], cutoff=[3, 3])
    exact = brute.box_probabilities(inst)
    wrapped = pgf.wrapped_distribution(inst, grid=[40, 40])
    assert np.abs(exact - wrapped).max() < 1e-15


def test_unmeasured_modes_two_routes():
    # w = 1 on an unmeasured mode (generating function) vs the reduced state
    # (brute force on the marginal)
    rng = W.rng_for(98)
    M = 4
    T = np.sqrt(0.8) * W.haar_unitary(M, rng)
    inst = W.make_instance(T, rng.uniform(0.3, 0.6, M), bin_of=[0, -1, 1, -1], cutoff=[4, 4])
    exact = brute.box_probabilities(inst)
    wrapped = pgf.wrapped_distribution(inst, grid=[40, 40])
    assert np.abs(exact - wrapped).max() < 1e-15


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def test_normalisation_full_grid_box():
    # Eq. prob1: with the box equal to the whole grid, the wrapped
    # distribution sums to G(1) = 1
    inst = W.lossy_m16_k3(grid=[5, 5, 5, 5])
    inst["cutoff"] = np.array([4, 4, 4, 4], np.int32)
    P, imag = pgf.wrapped_distribution(inst, return_imag=True)
    assert abs(P.sum() - 1.0) < 1e-13
    assert imag < 1e-15


def _moment_instance():
    rng = W.rng_for(97)
    M, K = 4, 2
    T = np.sqrt(0.5) * W.haar_unitary(M, rng)
    alpha = 0.5 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    r = rng.uniform(0.2, 0.45, M)
    return T, r, alpha, np.array([0.75, 0.25]), np.array([0, 1, 1, 0])


def test_mean_photon_number_per_bin():
    # <b_l> = sum_{i in bin l} sum_k [ sum_j |T_ij|^2 sinh^2 r_jk + delta_k0 |(T alpha)_i|^2 ]
    T, r, alpha, lam, bin_of = _moment_instance()
    inst = W.make_instance(T, r, alpha=alpha, schmidt=lam, bin_of=bin_of, cutoff=[39, 39], grid=[40, 40])
    P = pgf.wrapped_distribution(inst)
    rk = np.arctanh(np.sqrt(lam / lam[0])[None, :] * np.tanh(r)[:, None])
    per_mode = (np.abs(T) ** 2 @ (np.sinh(rk) ** 2)).sum(1) + np.abs(T @ alpha) ** 2
    b = np.arange(40)
    means = [(P.sum(1) * b).sum(), (P.sum(0) * b).sum()]
    for l in range(2):
        assert means[l] == pytest.approx(per_mode[bin_of == l].sum(), abs=1e-12)


def test_second_moments_per_bin():
    # zero displacement, Wick: Cov(n_i, n_j) = |N_ij|^2 + |M_ij|^2 + delta_ij N_ii
    T, r, _, lam, bin_of = _moment_instance()
    inst = W.make_instance(T, r, schmidt=lam, bin_of=bin_of, cutoff=[39, 39], grid=[40, 40])
    P = pgf.wrapped_distribution(inst)
    rk = np.arctanh(np.sqrt(lam / lam[0])[None, :] * np.tanh(r)[:, None])
    M, K = T.shape[0], 2
    cov = np.zeros((2, 2))
    for k in range(K):
        Nk = T.conj() @ np.diag(np.sinh(rk[:, k]) ** 2) @ T.T
        Mk = T @ np.diag(np.sinh(rk[:, k]) * np.cosh(rk[:, k])) @ T.T
        C = np.abs(Nk) ** 2 + np.abs(Mk) ** 2 + np.diag(np.diag(Nk).real)
        for l, m in itertools.product(range(2), range(2)):
            cov[l, m] += C[np.ix_(bin_of == l, bin_of == m)].sum()
    b = np.arange(40)
    m0, m1 = (P.sum(1) * b).sum(), (P.sum(0) * b).sum()
    c00 = (P.sum(1) * b * b).sum() - m0 * m0
    c11 = (P.sum(0) * b * b).sum() - m1 * m1
    c01 = (P * np.outer(b, b)).sum() - m0 * m1
    assert np.allclose([c00, c01, c11], [cov[0, 0], cov[0, 1], cov[1, 1]], atol=1e-11)


def test_conjugation_and_within_bin_permutation_invariance():
    inst = W.plain_m4(grid=[9, 9])
    P = pgf.wrapped_distribution(inst)
    conj = dict(inst, T=inst["T"].conj())
    assert np.abs(pgf.wrapped_distribution(conj) - P).max() < 1e-15
    perm = [1, 0, 3, 2]  # relabel output modes inside each bin
    permd = dict(inst, T=inst["T"][perm])
    assert np.abs(pgf.wrapped_distribution(permd) - P).max() < 1e-15
    swap = dict(inst, bin_of=np.array([1, 1, 0, 0], np.int32))  # relabel bins
    assert np.abs(pgf.wrapped_distribution(swap) - P.T).max() < 1e-15


def test_hermitian_symmetry_and_real_axis():
    S = st.assemble(W.lossy_m16_k3())
    rng = np.random.default_rng(5)
    for _ in range(3):
        w = np.exp(2j * np.pi * rng.random(4))
        assert abs(np.exp(pgf.log_pgf(S, w.conj())) - np.exp(pgf.log_pgf(S, w)).conj()) < 1e-15
    # on [0,1]^L the generating function is a positive combination of monomials
    for t in (0.0, 0.3, 1.0):
        g = np.exp(pgf.log_pgf(S, np.full(4, t)))
        assert g.real > 0 and abs(g.imag) < 1e-15
    assert abs(np.exp(pgf.log_pgf(S, np.ones(4))) - 1.0) < 1e-13


# ---------------------------------------------------------------------------
# Printed numbers: Fock heralding with spectral impurity (Sec. VIII A)
# ---------------------------------------------------------------------------

def test_fock_heralding_fidelities_match_paper():
    gold = json.load(open(os.path.join(GOLDEN, "fock_heralding_fidelity.json")))
    for case in gold["cases"]:
        inst = W.fock_herald_instance(case["p"], case["eta"], xi=gold["xi"], cutoff=(3, 63), grid=[64, 64])
        P = pgf.wrapped_distribution(inst)
        for n, F_paper in zip((1, 2, 3), case["F"]):
            F = np.sqrt(P[n, n] / P[n].sum())
            assert abs(F - F_paper) <= 0.5 * 10 ** (-case["decimals"]) + 1e-12, (case, n, F)


def test_uniform_loss_total_photon_law_is_a_convolution():
    """One bin over all modes, T = sqrt(eta) U: the total photon number does not
    depend on U and is the sum of M independent single-mode lossy squeezed
    counts (a passive unitary conserves the total number; uniform loss commutes
    with it), so its law is the M-fold convolution of the single-mode law."""
    M, N, G = 4, 14, 64
    single = W.make_instance(np.array([[np.sqrt(0.36)]]), [0.89], bin_of=[0], cutoff=[G - 1], grid=[G])
    p1 = pgf.wrapped_distribution(single)
    law = np.zeros(1)
    law[0] = 1.0
    for _ in range(M):
        law = np.convolve(law, p1)
    for seed in (6, 7):
        U = W.haar_unitary(M, W.rng_for(seed, M))
        inst = W.make_instance(np.sqrt(0.36) * U, np.full(M, 0.89), bin_of=np.zeros(M), cutoff=[N], grid=[G])
        P = pgf.wrapped_distribution(inst)
        assert np.abs(P - law[:N + 1]).max() < 1e-13

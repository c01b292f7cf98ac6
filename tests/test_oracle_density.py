"""Pins of the heralded density-matrix oracle (Sec. VII) on the CPU: the
loop-hafnian definition, closed forms of coherent, squeezed and two-mode
squeezed states, the joint photon-number distribution of the PGF oracle,
and the structural invariants of a density matrix."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import brute, pgf
from oracle import density as od

KEEP = W.KEEP


def test_taylor_coefficients_are_loop_hafnians():
    """s! [c^s] exp(1/2 c^T A c + g^T c) = lhaf(A_s, g_s) (Eq. lhaf_def), for a
    symmetric A that is not a physical state's, on every s of a small box."""
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    A = Z + Z.T
    g = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    caps = (2, 1, 3, 1)
    a = od.taylor_coefficients(A, g, caps)
    worst = 0.0
    for s in np.ndindex(*[c + 1 for c in caps]):
        lh = brute.lhaf_multiset(A, g, np.array(s, np.int32))
        got = a[s] * np.prod([math.factorial(x) for x in s])
        worst = max(worst, abs(got - lh) / max(1.0, abs(lh)))
    assert worst <= 1e-12


def test_coherent_states_closed_form():
    """Coherent inputs on a lossy interferometer stay coherent (beta = T alpha):
    the herald count is Poisson and the kept mode is |beta_1><beta_1|,
    <v|rho|u> = exp(-|b|^2) b^v conj(b)^u / sqrt(v! u!)."""
    rng = W.rng_for(71)
    T = np.sqrt(0.8) * W.haar_unitary(2, rng)
    alpha = np.array([0.9 - 0.4j, -0.5 + 0.7j])
    x = W.make_instance(T, np.zeros(2), alpha=alpha, bin_of=[0, KEEP], cutoff=[3], fock_cutoff=4)
    beta = T @ alpha
    ref = np.zeros((4, 5, 5), complex)
    for b in range(4):
        pb = math.exp(-abs(beta[0]) ** 2) * abs(beta[0]) ** (2 * b) / math.factorial(b)
        for v in range(5):
            for u in range(5):
                ref[b, v, u] = (pb * math.exp(-abs(beta[1]) ** 2) * beta[1] ** v * np.conj(beta[1]) ** u
                                / math.sqrt(math.factorial(v) * math.factorial(u)))
    for route in (od.density_taylor, od.density_brute):
        assert np.abs(route(x) - ref).max() <= 1e-14, route.__name__


def test_squeezed_vacuum_closed_form():
    """S(r)|0> with S(xi) = exp[(xi a^dag^2 - xi^* a^2)/2] (App. B):
    psi_2k = tanh(r)^k sqrt((2k)!) / (2^k k!) / sqrt(cosh r), odd amplitudes 0;
    the second mode is vacuum, so only the herald pattern 0 occurs."""
    r = 0.7
    x = W.make_instance(np.eye(2), np.array([r, 0.0]), bin_of=[KEEP, 0], cutoff=[2], fock_cutoff=8)
    psi = np.zeros(9)
    for k in range(5):
        psi[2 * k] = math.tanh(r) ** k * math.sqrt(math.factorial(2 * k)) / (2 ** k * math.factorial(k))
    psi /= math.sqrt(math.cosh(r))
    got = od.density_taylor(x)
    assert np.abs(got[0] - np.outer(psi, psi)).max() <= 1e-14
    assert np.abs(got[1:]).max() <= 1e-15


@pytest.mark.parametrize("eta", [1.0, 0.6])
def test_two_mode_squeezed_vacuum_heralds_fock_states(eta):
    """Equal squeezers on [[1, i],[i, 1]]/sqrt(2) give a two-mode squeezed
    vacuum sum_n c_n |n, n>, |c_n|^2 = tanh^2n r / cosh^2 r.  Heralding n in
    port 0 leaves |n> in port 1, which loss eta turns into the binomial mixture
    sum_k C(n, k) eta^k (1 - eta)^(n-k) |k><k|."""
    r = 0.5
    U = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2.0)
    T = np.diag([1.0, math.sqrt(eta)]) @ U
    x = W.make_instance(T, np.full(2, r), bin_of=[0, KEEP], cutoff=[4], fock_cutoff=5)
    ref = np.zeros((5, 6, 6))
    for n in range(5):
        pn = math.tanh(r) ** (2 * n) / math.cosh(r) ** 2
        for k in range(n + 1):
            ref[n, k, k] = pn * math.comb(n, k) * eta ** k * (1 - eta) ** (n - k)
    got = od.density_taylor(x)
    assert np.abs(got - ref).max() <= 1e-14


def _tiny_cases():
    rng = W.rng_for(72)
    T3 = np.sqrt(0.7) * W.haar_unitary(3, rng)
    al = 0.3 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    return {
        "displaced_one_bin": W.make_instance(T3, [0.5, 0.4, 0.6], alpha=al, bin_of=[0, 0, KEEP], cutoff=[2],
                                             fock_cutoff=2),
        "internal_modes_traced": W.make_instance(T3, [0.5, 0.4, 0.6], alpha=al, schmidt=[0.75, 0.25],
                                                 bin_of=[0, 0, 1, -1, KEEP, -1], resolve_internal=1,
                                                 cutoff=[2, 1], fock_cutoff=2),
    }


@pytest.mark.parametrize("name", sorted(_tiny_cases()))
def test_taylor_route_matches_the_loop_hafnian_definition(name):
    x = _tiny_cases()[name]
    a, b = od.density_taylor(x), od.density_brute(x)
    assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max())


def _mixed_case():
    """Lossy, two spectral modes, two kept modes, one traced: small squeezing
    so that the PGF oracle's grid of 20 points per bin wraps below 1e-14
    (a squeezed mode's tail beyond 2k photons falls as tanh^2k r)."""
    rng = W.rng_for(73)
    T = np.sqrt(0.75) * W.haar_unitary(3, rng)
    al = 0.25 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    return W.make_instance(T, [0.18, 0.15, 0.2], alpha=al, schmidt=[0.8, 0.2],
                           bin_of=[0, 0, 1, -1, KEEP, KEEP], resolve_internal=1, cutoff=[2, 2], fock_cutoff=3)


def test_diagonal_is_the_joint_distribution_of_the_pgf_oracle():
    """<u|rho(b~)|u> = Pr(b~, u): the kept modes as one-mode bins of the PGF
    oracle (determinants and an inverse DFT, Eq. coarse_grained_prob)."""
    x = _mixed_case()
    rho = od.density_taylor(x)
    b = x["bin_of"].copy()
    b[b == KEEP] = [2, 3]
    y = W.make_instance(x["T"], x["r"], alpha=x["alpha"], schmidt=x["schmidt"], bin_of=b, resolve_internal=1,
                        cutoff=[2, 2, 3, 3], grid=[20, 20, 20, 20])
    P = pgf.wrapped_distribution(y)
    diag = np.einsum("abvv->abv", rho).reshape(3, 3, 4, 4)
    assert np.abs(diag.imag).max() <= 1e-15
    assert np.abs(diag.real - P).max() <= 1e-14


def test_hermitian_and_positive_semidefinite():
    """Each truncated rho(b~) is a principal submatrix of a positive operator."""
    rho = od.density_taylor(_mixed_case())
    for b in np.ndindex(*rho.shape[:2]):
        m = rho[b]
        assert np.abs(m - m.conj().T).max() <= 1e-16
        assert np.linalg.eigvalsh(0.5 * (m + m.conj().T)).min() >= -1e-16


def test_pure_route_matches_the_taylor_route():
    rng = W.rng_for(74)
    U = W.haar_unitary(3, rng)
    al = 0.4 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    x = W.make_instance(U, [0.6, 0.3, 0.8], alpha=al, bin_of=[0, 1, KEEP], cutoff=[2, 2], fock_cutoff=4)
    a, b = od.density_pure(x), od.density_taylor(x)
    assert np.abs(a - b).max() <= 1e-15
    with pytest.raises(ValueError):
        od.density_pure(_mixed_case())

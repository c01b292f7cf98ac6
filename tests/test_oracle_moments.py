"""Pins of the moment and cumulant oracle (oracle/moments.py) on the CPU.

joint_moments / joint_cumulants (the definitions) are fed closed-form
distributions (squeezed vacuum even law, Poisson, negative binomial) and must
return the closed-form cumulants; cumulants_series (the series of Eq. M) must
return the same closed forms from the states themselves, and agree with the
definitions applied to the oracle's own distribution at low order; moments and
cumulants round-trip."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import moments as om


def _squeezed_law(r, nmax):
    p = np.zeros(nmax + 1)
    for n in range(0, nmax + 1, 2):
        m = n // 2
        p[n] = math.factorial(n) / (4 ** m * math.factorial(m) ** 2) * np.tanh(r) ** n / np.cosh(r)
    return p


def _squeezed_cumulants(r):
    # M(t) = (cosh^2 r - sinh^2 r e^{2t})^{-1/2}; a = sinh^2 r
    a = np.sinh(r) ** 2
    return np.array([0.0, a, 2 * a * (1 + a), 4 * a * (1 + a) * (1 + 2 * a), 8 * a * (1 + a) * (1 + 6 * a + 6 * a * a)])


def _negbin_cumulants(n, k):
    return k * np.array([0.0, n, n * (1 + n), n * (1 + n) * (1 + 2 * n), n * (1 + n) * (1 + 6 * n + 6 * n * n)])


@pytest.mark.parametrize("r", [0.3, 0.7])
def test_definitions_on_the_closed_form_squeezed_law(r):
    cum = om.joint_cumulants(om.joint_moments(_squeezed_law(r, 600), [4]))
    expect = _squeezed_cumulants(r)
    assert np.abs(cum - expect).max() <= 1e-12 * expect.max()


def test_definitions_on_closed_form_poisson_and_negative_binomial():
    mu = (0.7, 1.9)
    b = np.arange(120)
    pois = [np.exp(-m) * m ** b.astype(float) / np.array([math.factorial(int(x)) for x in b], float) for m in mu]
    cum = om.joint_cumulants(om.joint_moments(np.outer(pois[0], pois[1]), [4, 4]))
    expect = np.zeros((5, 5))
    for j in range(1, 5):
        expect[j, 0], expect[0, j] = mu
    assert np.abs(cum - expect).max() <= 1e-10  # total order 8: cancellation in the partition sum
    n, k = np.sinh(0.5) ** 2, 3
    bb = np.arange(300)
    nb = np.array([math.comb(int(x) + k - 1, int(x)) for x in bb], float) * n ** bb / (1 + n) ** (bb + k)
    cum = om.joint_cumulants(om.joint_moments(nb, [4]))
    expect = _negbin_cumulants(n, k)
    assert np.abs(cum - expect).max() <= 1e-11 * expect.max()


@pytest.mark.parametrize("r", [0.3, 0.7])
def test_series_single_mode_squeezed_vacuum(r):
    inst = W.make_instance(np.eye(1), [r], bin_of=[0], cutoff=[4])
    expect = _squeezed_cumulants(r)
    assert np.abs(om.cumulants_series(inst, [4]) - expect).max() <= 1e-13 * expect.max()


def test_series_lossy_coherent_bins_are_poisson():
    rng = np.random.default_rng(3)
    M = 4
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    alpha = 0.6 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    bin_of = np.array([0, 1, 1, 0])
    inst = W.make_instance(T, np.zeros(M), alpha=alpha, bin_of=bin_of, cutoff=[3, 3])
    beta = T @ alpha
    mu = [np.sum(np.abs(beta[bin_of == l]) ** 2) for l in range(2)]
    expect = np.zeros((4, 4))
    for j in range(1, 4):
        expect[j, 0], expect[0, j] = mu
    assert np.abs(om.cumulants_series(inst, [3, 3]) - expect).max() <= 1e-13


def test_series_thermal_bin_is_negative_binomial():
    r, k = 0.5, 3
    U2 = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    inst = W.make_instance(np.kron(np.eye(k), U2), np.full(2 * k, r), bin_of=np.tile([0, -1], k), cutoff=[4])
    expect = _negbin_cumulants(np.sinh(r) ** 2, k)
    assert np.abs(om.cumulants_series(inst, [4]) - expect).max() <= 1e-13 * expect.max()


def test_series_agrees_with_the_definitions_on_the_oracle_distribution():
    # internal modes, displacement, an unmeasured mode; second order, where the
    # distribution's rounding noise is harmless
    rng = W.rng_for(55)
    M = 4
    T = np.sqrt(0.6) * W.haar_unitary(M, rng)
    alpha = 0.4 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    inst = W.make_instance(T, rng.uniform(0.2, 0.6, M), alpha=alpha, schmidt=[0.7, 0.3], bin_of=[0, 1, -1, 1],
                           cutoff=[2, 2])
    P = om.oversampled_distribution(inst, 48)
    defn = om.joint_cumulants(om.joint_moments(P, [2, 2]))
    ser = om.cumulants_series(inst, [2, 2])
    assert np.abs(defn - ser).max() <= 1e-9 * np.abs(ser).max()  # rounding of the DFT-computed distribution


def test_moments_and_cumulants_round_trip():
    rng = np.random.default_rng(9)
    cum = rng.standard_normal((3, 4, 2))
    cum[0, 0, 0] = 0.0
    mom = om.moments_from_cumulants(cum)
    assert mom[0, 0, 0] == 1.0
    assert np.abs(om.joint_cumulants(mom) - cum).max() < 1e-12
    assert abs(mom[1, 1, 0] - (cum[1, 1, 0] + cum[1, 0, 0] * cum[0, 1, 0])) < 1e-14
    assert math.isclose(mom[2, 0, 0], cum[2, 0, 0] + cum[1, 0, 0] ** 2, rel_tol=1e-14)

"""Pins of the oracle's fully distinguishable inputs (App. D: each input's
squeezed vacuum in its own internal mode, detectors blind to it): the
distribution is the convolution of the distributions of the inputs taken one
at a time, each a single squeezer (K = 1) through the same circuit; and the
brute-force loop-hafnian sum on a tiny instance."""
import numpy as np

import workloads as W
from oracle import brute, pgf


def _single_input(x, j):
    r = np.zeros_like(x["r"])
    r[j] = x["r"][j]
    return W.make_instance(x["T"], r, bin_of=x["bin_of"], cutoff=x["cutoff"], grid=x["grid"])


def _convolve_box(a, b):
    """(a * b)(c) for c in the box of a (both arrays over the same box)."""
    out = np.zeros_like(a)
    for idx in np.ndindex(*a.shape):
        acc = 0.0
        for jdx in np.ndindex(*[i + 1 for i in idx]):
            acc += a[jdx] * b[tuple(i - j for i, j in zip(idx, jdx))]
        out[idx] = acc
    return out


def test_distribution_is_the_convolution_of_the_single_inputs():
    # small squeezing and a 40-point grid: the wrap is below 1e-15
    x = W.distinguishable_instance(3, 2, [2, 1], cutoff=[3, 2], grid=[40, 40], eta=0.7, r_range=(0.2, 0.4))
    P = pgf.wrapped_distribution(x)
    conv = None
    for j in range(3):
        Pj = pgf.wrapped_distribution(_single_input(x, j))
        conv = Pj if conv is None else _convolve_box(conv, Pj)
    assert np.abs(P - conv).max() <= 1e-14
    # not the indistinguishable distribution of the same squeezers (K = 1)
    y = dict(x)
    y.pop("distinguishable")
    assert np.abs(P - pgf.wrapped_distribution(y)).max() > 1e-3


def test_tiny_instance_against_brute_force():
    x = W.distinguishable_instance(2, 3, [1, 1], cutoff=[2, 2], grid=[40, 40], eta=0.8, r_range=(0.2, 0.5))
    assert np.abs(pgf.wrapped_distribution(x) - brute.box_probabilities(x)).max() <= 1e-14

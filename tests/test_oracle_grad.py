"""The autograd gradient oracle against central finite differences of the
numpy oracle (an independent implementation of the same formulas)."""
import numpy as np

import workloads as W
from oracle import grad as og
from oracle import pgf


def _tiny():
    rng = W.rng_for(77)
    M = 3
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    alpha = 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    return W.make_instance(T, rng.uniform(0.3, 0.6, M), alpha=alpha, schmidt=[0.7, 0.3],
                           bin_of=[0, 1, -1], cutoff=[2, 3], grid=[5, 6])


def _loss(inst, dP):
    return float((pgf.wrapped_distribution(inst) * dP).sum())


def test_torch_oracle_forward_equals_numpy_oracle():
    inst = _tiny()
    rng = np.random.default_rng(1)
    dP = rng.standard_normal((3, 4))
    _, _, _, P = og.gradients(inst, dP)
    assert np.abs(P - pgf.wrapped_distribution(inst)).max() < 1e-15


def test_autograd_matches_central_differences():
    inst = _tiny()
    rng = np.random.default_rng(2)
    dP = rng.standard_normal((3, 4))
    gr, gT, ga, _ = og.gradients(inst, dP)
    h = 1e-6
    for j in range(3):
        p, m = dict(inst, r=inst["r"].copy()), dict(inst, r=inst["r"].copy())
        p["r"][j] += h
        m["r"][j] -= h
        assert abs((_loss(p, dP) - _loss(m, dP)) / (2 * h) - gr[j]) < 1e-8
    for (i, j) in [(0, 0), (1, 2), (2, 1)]:
        for unit, part in ((1.0, "re"), (1j, "im")):
            p, m = dict(inst, T=inst["T"].copy()), dict(inst, T=inst["T"].copy())
            p["T"][i, j] += unit * h
            m["T"][i, j] -= unit * h
            fd = (_loss(p, dP) - _loss(m, dP)) / (2 * h)
            ref = gT[i, j].real if part == "re" else gT[i, j].imag
            assert abs(fd - ref) < 1e-8, (i, j, part, fd, ref)
    for j in range(3):
        for unit, part in ((1.0, "re"), (1j, "im")):
            p, m = dict(inst, alpha=inst["alpha"].copy()), dict(inst, alpha=inst["alpha"].copy())
            p["alpha"][j] += unit * h
            m["alpha"][j] -= unit * h
            fd = (_loss(p, dP) - _loss(m, dP)) / (2 * h)
            ref = ga[j].real if part == "re" else ga[j].imag
            assert abs(fd - ref) < 1e-8, (j, part, fd, ref)


def test_schmidt_weight_gradient_matches_central_differences():
    """dL/dlambda_k with each weight free (the state depends on lambda_k /
    lambda_0 only, so sum_k lambda_k dL/dlambda_k = 0)."""
    rng = W.rng_for(78)
    M = 3
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    inst = W.make_instance(T, rng.uniform(0.3, 0.7, M), schmidt=[0.5, 0.3, 0.2], bin_of=[0, 1, 1],
                           cutoff=[2, 3], grid=[5, 6])
    dP = np.random.default_rng(4).standard_normal((3, 4))
    g = og.gradients_full(inst, dP)
    h = 1e-6
    for k in range(3):
        p, m = dict(inst, schmidt=inst["schmidt"].copy()), dict(inst, schmidt=inst["schmidt"].copy())
        p["schmidt"][k] += h
        m["schmidt"][k] -= h
        fd = (_loss(p, dP) - _loss(m, dP)) / (2 * h)
        assert abs(fd - g["schmidt"][k]) < 1e-8, (k, fd, g["schmidt"][k])
    assert abs(float(np.dot(inst["schmidt"], g["schmidt"]))) < 1e-12

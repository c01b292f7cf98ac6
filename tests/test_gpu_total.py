"""The paper's GBS total-photon-number workload (Sec. VIII C): M = 16 .. 256
equally squeezed inputs (xi = 0.89) on sqrt(0.36) x Haar, one bin over all
modes, cutoffs N_max = 27 .. 170.

Expected values: for M <= 64 the oracle's wrapped distribution on the stated
grid; for every M the M-fold convolution of the oracle's single-mode law
(uniform loss makes the total count a sum of M independent single-mode counts,
pinned on the CPU by test_uniform_loss_total_photon_law_is_a_convolution),
wrapped onto the same grid; and with an automatic grid, the exact law."""
import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W
from oracle import pgf

pytestmark = pytest.mark.gpu
MS = sorted(W.TOTAL_PHOTON_CUTOFF)


def _say(*a):
    print(*a, flush=True)


def _eval(insts, precision="fp64", tol=1e-9):
    import torch
    with cgd.Context(insts, precision=precision, tol=tol) as ctx:
        p = ctx.eval()
        torch.cuda.synchronize()
        grids, wrap = ctx.bounds()
        return [x.cpu().numpy().copy() for x in ctx.split(p)], grids, wrap


def _exact_law(M, length=4096):
    """Law of the total count up to `length` (the mass beyond is far below
    1e-30 for these means), from the oracle's single-mode law."""
    single = W.make_instance(np.array([[np.sqrt(0.36)]]), [0.89], bin_of=[0], cutoff=[511], grid=[512])
    p1 = pgf.wrapped_distribution(single)
    law = np.zeros(length)
    law[0] = 1.0
    for _ in range(M):
        law = np.convolve(law, p1)[:length]
    return law


def _wrapped(law, G, N):
    out = np.zeros(G)
    for s in range(0, len(law), G):
        chunk = law[s:s + G]
        out[:len(chunk)] += chunk
    return out[:N + 1]


def test_small_sizes_against_the_oracle():
    insts = [W.gbs_total(M) for M in MS if M <= 64]
    got, grids, _ = _eval(insts)
    for x, P in zip(insts, got):
        ref = pgf.wrapped_distribution(x)
        _say(f"  M = {x['T'].shape[0]}: max |gpu - oracle| = {np.abs(P - ref).max():.2e}")
        assert np.abs(P - ref).max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_all_sizes_against_the_convolution_law(precision):
    insts = [W.gbs_total(M) for M in MS]
    got, grids, wrap = _eval(insts, precision)
    for M, x, P, (G,) in zip(MS, insts, got, grids):
        N = int(x["cutoff"][0])
        law = _exact_law(M)
        ref = _wrapped(law, G, N)
        d = np.abs(P - ref).max()
        _say(f"  M = {M}, N_max = {N}: max |gpu - wrapped law| = {d:.2e}, tail beyond N_max "
             f"{law[N + 1:].sum():.2e}, reported wrap bound {wrap[MS.index(M)]:.2e}")
        assert d <= 1e-12
        assert law[G:].sum() <= wrap[MS.index(M)] * (1 + 1e-9) + 1e-300


def test_automatic_grid_gives_the_exact_law():
    insts = [W.gbs_total(M, grid=[0]) for M in (16, 256)]
    got, grids, wrap = _eval(insts)
    for M, P, (G,), wb in zip((16, 256), got, grids, wrap):
        law = _exact_law(M)
        _say(f"  M = {M}: automatic grid {G}, bound {wb:.2e}")
        assert wb <= 1e-10
        assert np.abs(P - law[:len(P)]).max() <= 1e-9

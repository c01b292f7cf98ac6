"""Low-rank blocks on the GPU: fully distinguishable inputs (App. D: input j
squeezed in its own internal mode j, every internal block of rank 2) and K = 1
or Schmidt instances with one or two squeezed inputs (rank 2 or 4), evaluated
by per-point r x r determinants instead of factorisations of order 2M.

Bars: FP64 within 1e-12 absolute per probability of the oracle (whose App. D
instances are pinned on the CPU by the convolution of the single-input
distributions and by brute force); the general factorisation of the same
blocks (CGD_FLAG_NO_LOWRANK) within 1e-12; the mixed path within its 1e-9
budget; at full size, grid values sampled against the oracle point by point
and every grid value against the general route."""
import sys

import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W
from oracle import moments as om
from oracle import pgf
from oracle import state as st

pytestmark = pytest.mark.gpu
TOL_FP64 = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cgd.lib()
    yield
    torch.cuda.synchronize()


def _cases():
    """name -> (instance, number of low-rank blocks expected)."""
    rng = W.rng_for(4242)
    U6 = W.haar_unitary(6, rng)
    U5 = W.haar_unitary(5, rng)
    U4 = W.haar_unitary(4, rng)
    traced = W.distinguishable_instance(8, 3, [3, 3, 2], [4, 4, 1])
    traced["bin_of"] = np.array([0, 0, 0, 1, 1, 1, -1, -1], np.int32)
    traced["cutoff"] = np.array([4, 4], np.int32)
    traced["grid"] = np.array([5, 5], np.int32)
    one_bin = W.distinguishable_instance(5, 4, [5], [7], grid=[12])
    return {
        "dist_m6_3bins": (W.distinguishable_instance(6, 1, [2, 2, 2], [3, 3, 3]), 6),
        "dist_m8_traced": (traced, 8),
        "dist_m5_one_bin_oversampled": (one_bin, 5),
        "k1_two_squeezers_rank4": (W.make_instance(np.sqrt(0.6) * U6, [0.6, 0, 0.4, 0, 0, 0],
                                                   bin_of=W.contiguous_bins([3, 3]), cutoff=[4, 4]), 1),
        "k1_one_squeezer_rank2": (W.make_instance(np.sqrt(0.8) * U5, [0, 0.7, 0, 0, 0],
                                                  bin_of=W.contiguous_bins([5]), cutoff=[6], grid=[9]), 1),
        "schmidt_k2_one_squeezer": (W.make_instance(np.sqrt(0.7) * U4, [0.5, 0, 0, 0], schmidt=[0.7, 0.3],
                                                    bin_of=W.contiguous_bins([2, 2]), cutoff=[3, 3]), 2),
    }


def _dists(insts, flags=0, precision="fp64", tol=1e-9):
    import torch
    with cgd.Context(insts, precision=precision, tol=tol, flags=flags) as ctx:
        err = torch.zeros(ctx.n_inst, dtype=torch.float64, device="cuda")
        p = ctx.eval(err=err)
        torch.cuda.synchronize()
        out = [x.cpu().numpy().copy() for x in ctx.split(p)]
        return out, err.cpu().numpy(), ctx.tuning()["lowrank_blocks"]


def _grid(insts, flags=0):
    import torch
    with cgd.Context(insts, flags=flags) as ctx:
        ctx.eval()
        g = ctx.grid_values()
        torch.cuda.synchronize()
        return g.cpu().numpy().copy(), ctx.tuning()["lowrank_blocks"]


@pytest.mark.parametrize("name", list(_cases()))
def test_lowrank_blocks_match_the_oracle(name):
    inst, nlow = _cases()[name]
    _say("low-rank vs oracle:", name)
    (P,), err, got = _dists([inst])
    assert got == nlow
    ref = pgf.wrapped_distribution(inst)
    assert np.abs(P - ref).max() <= TOL_FP64, np.abs(P - ref).max()
    assert np.all(err == 0.0)


def test_lowrank_route_equals_the_factorisation_batched():
    cases = _cases()
    insts = [c[0] for c in cases.values()] + [W.plain_m4()]
    _say("low-rank vs CGD_FLAG_NO_LOWRANK, batch of", len(insts))
    A, _, na = _dists(insts)
    B, _, nb = _dists(insts, cgd.FLAG_NO_LOWRANK)
    assert na == sum(c[1] for c in cases.values()) and nb == 0
    for a, b in zip(A, B):
        assert np.abs(a - b).max() <= TOL_FP64
    # the instance with no low-rank block is unaffected by the neighbours' route
    assert np.abs(A[-1] - pgf.wrapped_distribution(W.plain_m4())).max() <= TOL_FP64


def test_lowrank_on_the_mixed_path():
    cases = _cases()
    insts = [c[0] for c in cases.values()] + [W.lossy_m16_k3(grid=[5, 5, 5, 5])]
    insts[-1]["cutoff"] = np.array([4, 4, 4, 4], np.int32)
    _say("low-rank blocks on the mixed path, batch of", len(insts))
    P, err, _ = _dists(insts, precision="mixed", tol=1e-9)
    for x, p, e in zip(insts, P, err):
        d = np.abs(p - pgf.wrapped_distribution(x)).max()
        assert d <= 1e-9 and d <= e + TOL_FP64, (d, e)
    # instances with only low-rank blocks have no FP32 pass: error bound 0
    assert np.all(err[:-1] == 0.0)


def test_lowrank_moments_match_the_factorisation():
    x, _ = _cases()["dist_m6_3bins"]
    y = dict(x)
    y["grid"] = None
    _say("low-rank blocks in moments and cumulants mode")
    for flag in (cgd.FLAG_MOMENTS, cgd.FLAG_CUMULANTS):
        import torch
        out = []
        for extra in (0, cgd.FLAG_NO_LOWRANK):
            with cgd.Context([y], flags=flag | extra) as ctx:
                p = ctx.eval()
                torch.cuda.synchronize()
                out.append(ctx.split(p)[0].cpu().numpy().copy())
        # element by element at the moments tests' relative bar (orders up to 9
        # here: the circle's DFT amplifies rounding by about (1 / rho)^order)
        assert np.all(np.abs(out[0] - out[1]) <= 1e-9 * np.abs(out[1]) + 1e-13)


def test_full_size_distinguishable_sampled_points():
    """M = 20 distinguishable squeezers, three bins, cutoffs 8 (the
    workload's shape at a size the oracle evaluates point by point)."""
    inst = W.distinguishable_instance(20, 9, [7, 7, 6], [8, 8, 8], eta=0.5)
    _say("dist M=20 3 bins, 9^3 grid, sampled points")
    logg, nlow = _grid([inst])
    assert nlow == 20
    S = st.assemble(inst)
    G = np.asarray(inst["grid"], dtype=float)
    dims = [int(G[0]) // 2 + 1] + [int(g) for g in G[1:]]
    ks = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(11)
    for p in np.concatenate([[0, 1, len(logg) - 1], rng.choice(len(logg), 5, replace=False)]):
        lo = pgf.log_pgf(S, np.exp(2j * np.pi * ks[p] / G))
        assert abs(np.exp(logg[p]) - np.exp(lo)) <= TOL_FP64, (p, logg[p], lo)
        d = logg[p] - lo
        assert abs(complex(d.real, (d.imag + np.pi) % (2 * np.pi) - np.pi)) < 1e-8, (p, logg[p], lo)


def test_gbs144_distinguishable_every_grid_value_against_the_factorisation():
    """144 distinguishable squeezers (r ~ U[0.4, 1.2], eta = 0.3), three bins of
    48, cutoffs 12: every grid value of the low-rank route against the general
    factorisation of the same 144 blocks of order 288."""
    inst = W.distinguishable_instance(144, 0, [48, 48, 48], [12, 12, 12], eta=0.3, r_range=(0.4, 1.2))
    _say("dist M=144 3 bins, 13^3 grid, low-rank vs factorisation")
    a, na = _grid([inst])
    b, nb = _grid([inst], cgd.FLAG_NO_LOWRANK)
    assert na == 144 and nb == 0
    assert np.abs(np.exp(a) - np.exp(b)).max() <= TOL_FP64
    assert np.abs(a - b).max() <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lowrank_repeated_and_static_evaluations_are_bitwise_equal(precision):
    """The low-rank launch inside the captured evaluation: replays of cgd_eval
    and a cgd_eval_static call (no allocation) give the same bits, with a
    factorised instance in the batch."""
    import torch
    cases = _cases()
    insts = [cases["dist_m6_3bins"][0], cases["k1_two_squeezers_rank4"][0], W.plain_m4()]
    _say("low-rank blocks: eval replays and eval_static,", precision)
    with cgd.Context(insts, precision=precision, tol=1e-9, flags=cgd.FLAG_NO_AUTOTUNE) as ctx:
        first = ctx.eval().clone()
        for _ in range(3):
            again = ctx.eval()
            torch.cuda.synchronize()
            assert torch.equal(again, first)
        static = ctx.eval_static()
        torch.cuda.synchronize()
        assert torch.equal(static, first)
        P = [x.cpu().numpy() for x in ctx.split(first)]
    for x, p in zip(insts, P):
        assert np.abs(p - pgf.wrapped_distribution(x)).max() <= (TOL_FP64 if precision == "fp64" else 1e-9)


@pytest.mark.parametrize("M, bins", [(4, [2, 2]), (5, [2, 2, 1])])
def test_distinguishable_cumulants_and_moments_against_the_series(M, bins):
    """Joint moments and cumulants of fully distinguishable inputs (App. D, row
    f4) on the low-rank route against the oracle's series of log M (Eq. M), at
    the moments tests' relative bar."""
    import torch
    x = W.distinguishable_instance(M, 5 + M, bins, list(bins))
    x["grid"] = None
    ref = om.cumulants_series(x, x["cutoff"])
    _say("distinguishable cumulants and moments, M =", M)
    for flag, want in ((cgd.FLAG_CUMULANTS, ref), (cgd.FLAG_MOMENTS, om.moments_from_cumulants(ref))):
        with cgd.Context([x], flags=flag) as ctx:
            got = ctx.split(ctx.eval())[0].cpu().numpy().copy()
            torch.cuda.synchronize()
            assert ctx.tuning()["lowrank_blocks"] == M
        err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
        assert err.max() <= 1e-9, (flag, err.max())

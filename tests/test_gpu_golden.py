"""Full-size, element-wise parity of the HIP path with the CPU oracle.

Every probability of the box of every benchmark workload (the 8 heaviest
instances of the 512-instance batch) against the oracle's wrapped
distribution on the same grid, stored under tests/golden/ by
tests/golden/make_golden.py (which calls only oracle/ and workloads/).

Bars: FP64 path within 1e-12 absolute per probability; mixed path (tol =
1e-9) within 1e-9, and within its own reported bound plus the FP64 rounding
level.  The workloads are evaluated as bench.py evaluates them (the whole
batch in one context, default route choice)."""
import os
import sys

import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
import make_golden  # noqa: E402

TOL_FP64 = 1e-12
TOL_MIXED = 1e-9


def _say(*a):
    print(*a, flush=True)


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path)


def _eval(insts, precision, flags=0):
    import torch
    with cgd.Context(insts, precision=precision, tol=TOL_MIXED, flags=flags) as ctx:
        err = torch.full((ctx.n_inst,), -1.0, dtype=torch.float64, device="cuda")
        p = ctx.eval(err=err)
        torch.cuda.synchronize()
        return [x.cpu().numpy().copy() for x in ctx.split(p)], err.cpu().numpy()


def _check(name, insts, which, precision, flags=0):
    g = _golden(name)
    got, err = _eval(insts, precision, flags)
    worst = 0.0
    for j, i in enumerate(which):
        ref = g[f"P_{j}"]
        assert got[i].shape == ref.shape, (name, i)
        assert np.array_equal(g[f"grid_{j}"], insts[i]["grid"])
        d = float(np.abs(got[i] - ref).max())
        worst = max(worst, d)
        if precision == "fp64":
            assert err[i] == 0.0
            assert d <= TOL_FP64, (name, i, d)
        else:
            assert 0.0 <= err[i] <= TOL_MIXED, (name, i, err[i])
            assert d <= TOL_MIXED, (name, i, d)
            assert d <= err[i] + TOL_FP64, (name, i, d, err[i])
    _say(f"{name} {precision} flags {flags}: max |P_gpu - P_oracle| = {worst:.3e}, bound {err.max():.3e}")


SINGLE = ["lossy16_k3", "gbs144_2bins", "gbs144_3bins"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", SINGLE)
def test_single_instance_workloads_every_probability(name, precision):
    _check(name, make_golden.CASES[name](), [0], precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gbs144_2bins_per_point_route_every_probability(precision):
    # the default takes the Hessenberg route here; the factorisation per point
    # must give the same box
    _check("gbs144_2bins", make_golden.CASES["gbs144_2bins"](), [0], precision, flags=cgd.FLAG_NO_HESSENBERG)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mesh32_k4_all_64_sets_every_probability(precision):
    insts = make_golden.CASES["mesh32_k4"]()
    _check("mesh32_k4", insts, list(range(len(insts))), precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uneven512_heaviest_instances_every_probability(precision):
    # the whole batch in one context (as bench.py runs it); the 8 instances with
    # the most factorisation work are compared probability by probability
    insts = W.uneven_batch()
    which = [int(i) for i in _golden("uneven512_heavy")["index"]]
    assert which == make_golden.UNEVEN_HEAVY
    _check("uneven512_heavy", insts, which, precision)


def test_gbs144_2bins_routes_agree_at_every_grid_point():
    """log G at all 7381 evaluated points: Hessenberg route against the
    factorisation per point (both FP64)."""
    import torch
    inst = W.gbs_m144(2)
    vals = {}
    for flags in (cgd.FLAG_HESSENBERG, cgd.FLAG_NO_HESSENBERG):
        with cgd.Context([inst], flags=flags) as ctx:
            ctx.eval()
            vals[flags] = ctx.grid_values().cpu().numpy()
            torch.cuda.synchronize()
    a, b = vals[cgd.FLAG_HESSENBERG], vals[cgd.FLAG_NO_HESSENBERG]
    assert a.shape == b.shape == (7381,)
    dG = np.abs(np.exp(a) - np.exp(b))
    _say(f"routes: max |G_hess - G_point| = {dG.max():.3e}")
    assert dG.max() <= 1e-13
    big = np.exp(b.real) > 1e-6
    dphase = np.angle(np.exp(1j * (a.imag - b.imag)))
    assert np.abs(a.real - b.real)[big].max() <= 1e-9
    assert np.abs(dphase)[big].max() <= 1e-9


def _shape_counts(insts, precision):
    with cgd.Context(insts, precision=precision, tol=TOL_MIXED, flags=cgd.FLAG_NO_HESSENBERG) as ctx:
        rep = ctx.tuning()
    return {c["class"]: (len(c["fp64_ms"]), len(c["fp32_ms"]) if c["precision"] == "fp32+fp64" else 0)
            for c in rep["classes"] if c["class"] < 3}


def _shape_cases():
    # the 8 heaviest batch instances hold blocks of orders 33..96 (classes 1, 2);
    # the mesh sets blocks of order 32 (class 0)
    batch = W.uneven_batch()
    which = [int(i) for i in _golden("uneven512_heavy")["index"]]
    return {"uneven512_heavy": ([batch[i] for i in which], {1, 2}),
            "mesh32_k4": (make_golden.CASES["mesh32_k4"](), {0})}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["uneven512_heavy", "mesh32_k4"])
def test_every_kernel_shape_of_classes_0_to_2(case, precision):
    """Each FP64 shape (register kernel and FP64 MFMA) and, on the mixed path,
    each FP32 MFMA shape of the size classes <= 96, pinned in turn with
    cgd_set_kernel_shape, against the oracle's boxes (factorisation per
    point): the 8 heaviest instances of the batch (classes 1, 2) and the 64
    mesh sets (class 0)."""
    import torch
    insts, classes = _shape_cases()[case]
    g = _golden(case)
    counts = _shape_counts(insts, precision)
    assert classes <= set(counts), counts
    for cls in sorted(classes):
        n64, n32 = counts[cls]
        for kind, n in (("fp64", n64), ("fp32", n32)):
            for v in range(n):
                with cgd.Context(insts, precision=precision, tol=TOL_MIXED, flags=cgd.FLAG_NO_HESSENBERG) as ctx:
                    ctx.set_kernel_shape(cls, v if kind == "fp64" else -1, v if kind == "fp32" else -1)
                    rep = {c["class"]: c for c in ctx.tuning()["classes"]}
                    name = list(rep[cls][f"{kind}_ms"])[v]
                    err = torch.full((ctx.n_inst,), -1.0, dtype=torch.float64, device="cuda")
                    p = ctx.eval(err=err)
                    torch.cuda.synchronize()
                    got = [x.cpu().numpy() for x in ctx.split(p)]
                    err = err.cpu().numpy()
                worst = max(float(np.abs(got[j] - g[f"P_{j}"]).max()) for j in range(len(insts)))
                _say(f"  {case} {precision} class {cls} {name}: max |P - P_oracle| {worst:.2e}, bound {err.max():.2e}")
                if precision == "fp64":
                    assert worst <= TOL_FP64 and err.max() == 0.0, (name, worst)
                else:
                    assert worst <= TOL_MIXED and err.max() <= TOL_MIXED and worst <= err.max() + TOL_FP64, name

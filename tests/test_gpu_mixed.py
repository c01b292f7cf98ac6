"""Mixed path (complex FP32 factorisations + FP64 re-factorisation of the grid
points whose value can matter) against the FP64 path.

Bar: every probability of every instance within 1e-9 of the FP64 path, and
within the per-instance error bound the library reports."""
import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _say(*a):
    print(*a, flush=True)


def _run(instances, precision, tol=TOL, flags=cgd.FLAG_NO_HESSENBERG):
    # the FP32 path is what is tested here: the Hessenberg route (FP64 in both
    # precisions) is switched off unless a test asks for it
    import torch
    with cgd.Context(instances, precision=precision, tol=tol, flags=flags) as ctx:
        err = torch.full((ctx.n_inst,), -1.0, dtype=torch.float64, device="cuda")
        p = ctx.eval(err=err)
        torch.cuda.synchronize()
        stats = ctx.mixed_stats() if precision == "mixed" else None
        return np.concatenate([x.cpu().numpy().ravel() for x in ctx.split(p)]), err.cpu().numpy(), stats, \
            ctx.prob_offsets.copy()


def _per_instance_maxdiff(a, b, offs):
    return np.array([np.abs(a[offs[i]:offs[i + 1]] - b[offs[i]:offs[i + 1]]).max() for i in range(len(offs) - 1)])


CASES = {
    "plain4": lambda: [W.plain_m4()],
    "lossy16_k3": lambda: [W.lossy_m16_k3()],
    "gbs144_2bins": lambda: [W.gbs_m144(2)],
    "mesh32_k4": lambda: W.mesh_batch(16),
    "uneven512": lambda: W.uneven_batch(96),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_error_model_holds(name):
    """With nothing re-evaluated (tol huge) the reported bound must still cover
    the actual deviation from FP64: this checks the assumed FP32 error."""
    _say("fp32-only vs fp64:", name)
    insts = CASES[name]()
    p64, _, _, offs = _run(insts, "fp64")
    p32, err, (nfix, ntot), _ = _run(insts, "mixed", tol=1e300)
    assert nfix == 0
    d = _per_instance_maxdiff(p32, p64, offs)
    _say("  max |P32 - P64| =", d.max(), " bound =", err.max(), " ratio max", (d / err).max())
    assert np.all(d <= err)


@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_matches_fp64_within_1e9(name):
    _say("mixed vs fp64:", name)
    insts = CASES[name]()
    p64, err64, _, offs = _run(insts, "fp64")
    pm, errm, (nfix, ntot), _ = _run(insts, "mixed")
    d = _per_instance_maxdiff(pm, p64, offs)
    _say(f"  max |Pmixed - P64| = {d.max():.3e}, bound {errm.max():.3e}, refactorised {nfix}/{ntot}")
    assert np.all(err64 == 0.0)
    assert np.all(errm <= TOL)
    assert np.all(d <= np.maximum(errm, 1e-15))
    assert d.max() <= TOL


def test_mixed_order_192_class_and_elimination_off():
    # order 192 (three bins of 48, one eliminated) takes the 8-wave MFMA class;
    # the dense no-Schur lossy instance (order 97) the order-128 class
    _say("mixed gbs144_3bins / no-Schur lossy16_k3")
    for insts, flags in (([W.gbs_m144(3)], 0), ([W.lossy_m16_k3()], cgd.FLAG_NO_SCHUR | cgd.FLAG_DENSE_INTERNAL)):
        flags |= cgd.FLAG_NO_HESSENBERG
        p64, _, _, offs = _run(insts, "fp64", flags=flags)
        pm, errm, _, _ = _run(insts, "mixed", flags=flags)
        assert np.abs(pm - p64).max() <= TOL
        assert np.all(errm <= TOL)


def test_mixed_with_hessenberg_route_matches_fp64():
    # the two-bin GBS instance takes the Hessenberg route by itself (FP64 in
    # both precisions): no FP32 factorisation, a zero bound, and the FP64 values
    _say("mixed, automatic route: gbs144_2bins")
    insts = [W.gbs_m144(2)]
    p64, _, _, _ = _run(insts, "fp64", flags=0)
    pm, errm, (nfix, ntot), _ = _run(insts, "mixed", flags=0)
    assert nfix == 0 and ntot == 0
    assert np.all(errm == 0.0)
    assert np.abs(pm - p64).max() <= 1e-14

"""Heralded density matrices (Sec. VII) on the GPU through the C ABI, against
closed forms, the oracle's loop-hafnian definition (tiny cases), its Taylor
and pure-state routes (moderate and full GKP-like sizes), the PGF oracle's
joint distribution (the diagonal at full size), and the library's own
probability path.  Grids are automatic (tail bound <= tol / 10), so the wrapped
output is compared with exact values within the reported wrap bound."""
import math

import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W
from oracle import density as od
from oracle import pgf

pytestmark = pytest.mark.gpu
KEEP = W.KEEP
ATOL = 1e-12


def _say(*a):
    print(*a, flush=True)


def _auto(x):
    y = dict(x)
    y["grid"] = np.zeros(len(x["cutoff"]), np.int32)
    return y


def _gpu(insts, flags=0, tol=1e-13, static=False):
    import torch
    with cgd.Context(insts, flags=flags, tol=tol) as ctx:
        p = ctx.eval_static() if static else ctx.eval()
        torch.cuda.synchronize()
        _, wrap = ctx.bounds()
        return [x.cpu().numpy().copy() for x in ctx.split(p)], wrap


def _check(got, ref, wrap, what):
    d = np.abs(got - ref).max()
    _say(f"  {what}: max |gpu - ref| = {d:.2e} (wrap bound {wrap:.1e}, max |ref| {np.abs(ref).max():.2e})")
    assert d <= ATOL + wrap, (what, d)


def test_coherent_and_squeezed_closed_forms():
    rng = W.rng_for(71)
    T = np.sqrt(0.8) * W.haar_unitary(2, rng)
    alpha = np.array([0.9 - 0.4j, -0.5 + 0.7j])
    coh = W.make_instance(T, np.zeros(2), alpha=alpha, bin_of=[0, KEEP], cutoff=[3], fock_cutoff=4)
    r = 0.7
    sq = W.make_instance(np.eye(2), np.array([r, 0.0]), bin_of=[KEEP, 0], cutoff=[2], fock_cutoff=8)
    (gc, gs), wrap = _gpu([_auto(coh), _auto(sq)])
    beta = T @ alpha
    ref = np.zeros((4, 5, 5), complex)
    for b in range(4):
        pb = math.exp(-abs(beta[0]) ** 2) * abs(beta[0]) ** (2 * b) / math.factorial(b)
        for v in range(5):
            for u in range(5):
                ref[b, v, u] = (pb * math.exp(-abs(beta[1]) ** 2) * beta[1] ** v * np.conj(beta[1]) ** u
                                / math.sqrt(math.factorial(v) * math.factorial(u)))
    _check(gc, ref, wrap[0], "coherent")
    psi = np.zeros(9)
    for k in range(5):
        psi[2 * k] = math.tanh(r) ** k * math.sqrt(math.factorial(2 * k)) / (2 ** k * math.factorial(k))
    psi /= math.sqrt(math.cosh(r))
    ref = np.zeros((3, 9, 9))
    ref[0] = np.outer(psi, psi)
    _check(gs, ref, wrap[1], "squeezed vacuum")


@pytest.mark.parametrize("eta", [1.0, 0.6])
def test_two_mode_squeezed_vacuum_heralds_fock_states(eta):
    r = 0.5
    U = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2.0)
    T = np.diag([1.0, math.sqrt(eta)]) @ U
    x = W.make_instance(T, np.full(2, r), bin_of=[0, KEEP], cutoff=[4], fock_cutoff=5)
    (g,), wrap = _gpu([_auto(x)])
    ref = np.zeros((5, 6, 6))
    for n in range(5):
        pn = math.tanh(r) ** (2 * n) / math.cosh(r) ** 2
        for k in range(n + 1):
            ref[n, k, k] = pn * math.comb(n, k) * eta ** k * (1 - eta) ** (n - k)
    _check(g, ref, wrap[0], f"TMSV heralding, eta {eta}")


def _tiny():
    rng = W.rng_for(72)
    T3 = np.sqrt(0.7) * W.haar_unitary(3, rng)
    al = 0.3 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    return {
        "displaced_one_bin": W.make_instance(T3, [0.5, 0.4, 0.6], alpha=al, bin_of=[0, 0, KEEP], cutoff=[2],
                                             fock_cutoff=2),
        "internal_modes_traced": W.make_instance(T3, [0.5, 0.4, 0.6], alpha=al, schmidt=[0.75, 0.25],
                                                 bin_of=[0, 0, 1, -1, KEEP, -1], resolve_internal=1,
                                                 cutoff=[2, 1], fock_cutoff=2),
        "kept_external_mode_all_internal": W.make_instance(T3, [0.5, 0.4, 0.6], schmidt=[0.75, 0.25],
                                                           bin_of=[0, 1, KEEP], cutoff=[2, 1], fock_cutoff=1),
    }


@pytest.mark.parametrize("name", sorted(_tiny()))
def test_tiny_cases_against_the_loop_hafnian_definition(name):
    x = _tiny()[name]
    (g,), wrap = _gpu([_auto(x)])
    _check(g, od.density_brute(x), wrap[0], name)


def _moderate():
    rng = W.rng_for(73)
    T = np.sqrt(0.75) * W.haar_unitary(3, rng)
    al = 0.25 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    return {
        "two_kept_modes_displaced": W.make_instance(T, [0.5, 0.45, 0.6], alpha=al, schmidt=[0.8, 0.2],
                                                    bin_of=[0, 0, 1, -1, KEEP, KEEP], resolve_internal=1,
                                                    cutoff=[2, 2], fock_cutoff=3),
        "fock_heralding": W.fock_herald_density(0.9, 0.85, herald=3, fock_cutoff=6),
        "gkp_shape_small_pattern": W.gkp_like(0.85, 0.9, herald=(2, 3), fock_cutoff=8),
    }


@pytest.mark.parametrize("flags", [0, cgd.FLAG_NO_SCHUR, cgd.FLAG_DENSE_INTERNAL])
@pytest.mark.parametrize("name", sorted(_moderate()))
def test_moderate_cases_against_the_taylor_oracle(name, flags):
    x = _moderate()[name]
    (g,), wrap = _gpu([_auto(x)], flags=flags)
    _check(g, od.density_taylor(x), wrap[0], f"{name} flags {flags}")


def test_pure_gkp_shape_full_size_elementwise():
    """K = 1, lossless: heralding pattern (5, 7), Fock cutoff 26 -- every
    element against the oracle's pure-state route."""
    x = W.gkp_like(1.0, 1.0)
    (g,), wrap = _gpu([_auto(x)])
    _check(g, od.density_pure(x), wrap[0], "pure GKP shape (5, 7), N = 26")


def test_mixed_gkp_shape_full_size_properties_and_diagonal():
    """Two spectral modes and loss at the full GKP shape: each rho(b~) is
    Hermitian and positive semidefinite, and its diagonal is the joint
    distribution of (heralding bins, kept mode) -- from the PGF oracle on the
    same heralding grid, and from the library's probability path.  The kept
    mode's own axis is exact on the density side, so the probability side
    takes 200 points for it (its tail beyond 200 photons is below 1e-16)."""
    x = W.gkp_like(0.85, 0.9)
    (g,), _ = _gpu([x])  # the stated grid (6, 8): wrapped values on both sides
    for b in np.ndindex(*g.shape[:2]):
        m = g[b]
        assert np.abs(m - m.conj().T).max() <= 1e-15
        ev = np.linalg.eigvalsh(0.5 * (m + m.conj().T))
        assert ev.min() >= -1e-14 * max(1.0, ev.max()), (b, ev.min())
    y = dict(x)
    bo = x["bin_of"].copy()
    bo[bo == KEEP] = 2
    y.update(bin_of=bo, cutoff=np.array([5, 7, 26], np.int32), grid=np.array([6, 8, 200], np.int32))
    y.pop("fock_cutoff")
    diag = np.einsum("abvv->abv", g)
    assert np.abs(diag.imag).max() <= 1e-15
    ref = pgf.wrapped_distribution(y)
    d1 = np.abs(diag.real - ref).max()
    (P,), _ = _gpu([y])
    d2 = np.abs(diag.real - P).max()
    _say(f"  diagonal vs PGF oracle {d1:.2e}, vs the library's probabilities {d2:.2e}")
    assert d1 <= ATOL and d2 <= ATOL


def test_batch_with_probability_instances_and_static_entry_point():
    """Density and probability instances in one context (odd offsets before a
    density instance), cgd_eval and cgd_eval_static, each instance as alone."""
    mod = _moderate()
    insts = [W.plain_m4(), mod["two_kept_modes_displaced"], W.lossy_m16_k3(),
             mod["fock_heralding"], _tiny()["displaced_one_bin"]]
    # bitwise equality needs the same kernel shapes in every context: the
    # autotuner, timing a different mix of work, may pick others
    fl = cgd.FLAG_NO_AUTOTUNE
    got, _ = _gpu(insts, flags=fl)
    got_s, _ = _gpu(insts, flags=fl, static=True)
    for i, x in enumerate(insts):
        (alone,), _ = _gpu([x], flags=fl)
        assert np.array_equal(got[i], alone), i
        assert np.array_equal(got_s[i], alone), i
    assert got[1].shape == (3, 3, 16, 16) and got[3].shape == (4, 7, 7)
    _check(got[0], pgf.wrapped_distribution(insts[0]), 0.0, "plain_m4 in the batch")


def test_graph_replays_match_eager_evaluation():
    import torch
    x = _moderate()["gkp_shape_small_pattern"]
    with cgd.Context([x]) as ctx:
        ctx.set_timing(True)
        ref = ctx.eval().clone()
        torch.cuda.synchronize()
        t = ctx.stage_times()
        assert t["density"] > 0, t
        ctx.set_timing(False)
        out = torch.empty_like(ref)
        for _ in range(3):
            ctx.eval(out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)

"""Gradients from the adjoint kernels (through the C ABI) against the autograd
oracle and central finite differences of the GPU forward."""
import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W
from oracle import grad as og

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _gpu_grad(insts, dP_list, flags=0):
    import torch
    with cgd.Context(insts, flags=cgd.FLAG_GRAD | flags) as ctx:
        P = ctx.eval()
        dP = torch.tensor(np.concatenate([d.ravel() for d in dP_list]), dtype=torch.float64, device="cuda")
        dr, dT, da = ctx.grad(dP)
        torch.cuda.synchronize()
        return dr.cpu().numpy(), dT.cpu().numpy(), da.cpu().numpy(), P.cpu().numpy()


def _small_instances():
    rng = W.rng_for(76)
    out = []
    M = 3
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    alpha = 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    out.append(W.make_instance(T, rng.uniform(0.3, 0.6, M), alpha=alpha, schmidt=[0.7, 0.3],
                               bin_of=[0, 1, -1], cutoff=[2, 3], grid=[5, 6]))
    M = 4
    T = np.sqrt(0.6) * W.haar_unitary(M, rng)
    out.append(W.make_instance(T, rng.uniform(0.2, 0.7, M), bin_of=[0, 0, 1, 1], cutoff=[4, 4], grid=[8, 7]))
    T = np.sqrt(0.8) * W.haar_unitary(M, rng)
    alpha = 0.4 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    out.append(W.make_instance(T, rng.uniform(0.2, 0.5, M), alpha=alpha, bin_of=[0, 0, 0, 0], cutoff=[6], grid=[9]))
    return out


def test_adjoint_matches_autograd_oracle():
    _say("adjoint vs autograd oracle (batched small instances)")
    insts = _small_instances()
    rng = np.random.default_rng(3)
    dPs = [rng.standard_normal(tuple(int(c) + 1 for c in x["cutoff"])) for x in insts]
    dr, dT, da, _ = _gpu_grad(insts, dPs)
    ro = to = 0
    for x, dP in zip(insts, dPs):
        M = x["T"].shape[0]
        gr, gT, ga, _ = og.gradients(x, dP)
        assert np.abs(dr[ro:ro + M] - gr).max() < 1e-11, (dr[ro:ro + M], gr)
        assert np.abs(dT[to:to + M * M].reshape(M, M) - gT).max() < 1e-11
        if ga is not None:
            assert np.abs(da[ro:ro + M] - ga).max() < 1e-11
        else:
            assert np.abs(da[ro:ro + M]).max() == 0.0
        ro += M
        to += M * M


def test_mesh_gradients_wrt_r_eta_theta_vs_finite_differences():
    """Config 5 shape (M=32, K=4, 2 bins of 16, cutoff 12) on a few parameter
    sets: d(loss)/d(r, eta, theta) through the autograd wrapper against central
    differences (h = 1e-6) of the GPU forward."""
    import torch
    _say("mesh_batch gradients vs central differences")
    p = W.mesh_params(2)
    spec = dict(schmidt=p["schmidt"], bin_of=p["bin_of"], cutoff=p["cutoff"])
    rng = np.random.default_rng(5)
    wgt = torch.tensor(rng.standard_normal((2, 13, 13)), dtype=torch.float64, device="cuda")

    def loss_of(r, eta, theta):
        T = torch.stack([W.mesh_transfer(eta[b], theta[b], p["phases"], p["M"]) for b in range(2)])
        P = cgd.distribution(r, T, None, spec)
        return (P * wgt).sum()

    r = torch.tensor(np.stack([s["r"] for s in p["sets"]]), requires_grad=True)
    eta = torch.tensor(np.stack([s["eta"] for s in p["sets"]]), requires_grad=True)
    theta = torch.tensor(np.stack([s["theta"] for s in p["sets"]]), requires_grad=True)
    L = loss_of(r, eta, theta)
    L.backward()
    h = 1e-6
    checks = [("r", r, (0, 3)), ("r", r, (1, 30)), ("eta", eta, (0, 7)), ("eta", eta, (1, 16)),
              ("theta", theta, (0, 0)), ("theta", theta, (1, 250)), ("theta", theta, (0, 495))]
    for name, var, idx in checks:
        with torch.no_grad():
            base = [r.detach().clone(), eta.detach().clone(), theta.detach().clone()]
            k = {"r": 0, "eta": 1, "theta": 2}[name]
            plus = [b.clone() for b in base]
            minus = [b.clone() for b in base]
            plus[k][idx] += h
            minus[k][idx] -= h
            fd = (loss_of(*plus).item() - loss_of(*minus).item()) / (2 * h)
        g = var.grad[idx].item()
        _say(f"  d/d{name}{idx}: adjoint {g:.10e}  fd {fd:.10e}")
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx, g, fd)


def test_gradient_is_bitwise_reproducible():
    import torch
    insts = _small_instances()
    dPs = [np.ones(tuple(int(c) + 1 for c in x["cutoff"])) for x in insts]
    # two contexts run the same kernels only with the shapes pinned (the
    # autotuner times each context's own work)
    a = _gpu_grad(insts, dPs, cgd.FLAG_NO_AUTOTUNE)
    b = _gpu_grad(insts, dPs, cgd.FLAG_NO_AUTOTUNE)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_schmidt_weight_gradient_matches_autograd_oracle():
    """d_dschmidt (each Schmidt weight free) against the autograd oracle, on a
    displaced two-weight instance and a three-weight one with an unmeasured
    mode; and the scaling invariance sum_k lambda_k dL/dlambda_k = 0."""
    import torch
    rng = W.rng_for(79)
    M = 3
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    alpha = 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    insts = [_small_instances()[0],
             W.make_instance(T, rng.uniform(0.3, 0.7, M), alpha=alpha, schmidt=[0.5, 0.3, 0.2],
                             bin_of=[0, -1, 1], cutoff=[3, 2], grid=[6, 5])]
    dPs = [np.random.default_rng(6 + i).standard_normal(tuple(int(c) + 1 for c in x["cutoff"]))
           for i, x in enumerate(insts)]
    with cgd.Context(insts, flags=cgd.FLAG_GRAD) as ctx:
        ctx.eval()
        dP = torch.tensor(np.concatenate([d.ravel() for d in dPs]), dtype=torch.float64, device="cuda")
        dr, dT, da, ds = ctx.grad(dP, schmidt=True)
        torch.cuda.synchronize()
        ds = ds.cpu().numpy()
    off = 0
    for x, d in zip(insts, dPs):
        K = len(x["schmidt"])
        g = og.gradients_full(x, d)
        _say(f"  dL/dlambda gpu {ds[off:off + K]} oracle {g['schmidt']}")
        assert np.abs(ds[off:off + K] - g["schmidt"]).max() < 1e-11
        assert abs(float(np.dot(x["schmidt"], ds[off:off + K]))) < 1e-11
        off += K


def test_mesh_gradient_matches_autograd_oracle_at_full_shape():
    """One parameter set of the differentiation workload (M = 32, K = 4, two
    bins of 16, cutoff 12): dL/dr, dL/dT and dL/dlambda from the adjoint
    against the autograd oracle (dense 256 x 256 per grid point)."""
    import torch
    x = W.mesh_batch(1)[0]
    dP = np.random.default_rng(8).standard_normal((13, 13))
    with cgd.Context([x], flags=cgd.FLAG_GRAD) as ctx:
        ctx.eval()
        dr, dT, da, ds = ctx.grad(torch.tensor(dP.ravel(), dtype=torch.float64, device="cuda"), schmidt=True)
        torch.cuda.synchronize()
    g = og.gradients_full(x, dP)
    M = 32
    er = np.abs(dr.cpu().numpy() - g["r"]).max() / np.abs(g["r"]).max()
    eT = np.abs(dT.cpu().numpy().reshape(M, M) - g["T"]).max() / np.abs(g["T"]).max()
    es = np.abs(ds.cpu().numpy() - g["schmidt"]).max() / np.abs(g["schmidt"]).max()
    _say(f"  mesh set 0: relative max error r {er:.2e}, T {eT:.2e}, lambda {es:.2e}")
    assert er < 1e-9 and eT < 1e-9 and es < 1e-9


def test_adjoint_above_order_96_matches_autograd_oracle():
    """Blocks of order 98 to 105 (M = 49..52, two bins, one displaced) take the
    blocked adjoint (Gauss-Jordan inverse in an HBM workspace), batched with a
    small instance on the register kernel: dL/dr, dL/dT, dL/dalpha and
    dL/dlambda against the autograd oracle."""
    import torch
    rng = W.rng_for(81)
    insts = []
    M = 52
    T = np.sqrt(0.6) * W.haar_unitary(M, rng)
    alpha = 0.2 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    insts.append(W.make_instance(T, rng.uniform(0.2, 0.6, M), alpha=alpha, bin_of=W.contiguous_bins([26, 26]),
                                 cutoff=[2, 2], grid=[3, 3]))
    M = 49
    T = np.sqrt(0.7) * W.haar_unitary(M, rng)
    insts.append(W.make_instance(T, rng.uniform(0.2, 0.6, M), schmidt=[0.7, 0.3], bin_of=W.contiguous_bins([24, 25]),
                                 cutoff=[2, 3], grid=[3, 4]))
    insts.append(_small_instances()[1])
    dPs = [np.random.default_rng(11 + i).standard_normal(tuple(int(c) + 1 for c in x["cutoff"]))
           for i, x in enumerate(insts)]
    _say("adjoint above order 96 vs autograd oracle")
    with cgd.Context(insts, flags=cgd.FLAG_GRAD) as ctx:
        ctx.eval()
        dP = torch.tensor(np.concatenate([d.ravel() for d in dPs]), dtype=torch.float64, device="cuda")
        dr, dT, da, ds = ctx.grad(dP, schmidt=True)
        torch.cuda.synchronize()
        dr, dT, da, ds = (t.cpu().numpy() for t in (dr, dT, da, ds))
    ro = to = so = 0
    for x, d in zip(insts, dPs):
        M = x["T"].shape[0]
        K = 1 if x.get("schmidt") is None else len(x["schmidt"])
        g = og.gradients_full(x, d)

        def rel(a, b):
            return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)

        er = rel(dr[ro:ro + M], g["r"])
        eT = rel(dT[to:to + M * M].reshape(M, M), g["T"])
        _say(f"  M = {M}: relative max error r {er:.2e}, T {eT:.2e}")
        assert er < 1e-9 and eT < 1e-9
        if g["alpha"] is not None:
            assert rel(da[ro:ro + M], g["alpha"]) < 1e-9
        else:
            assert np.abs(da[ro:ro + M]).max() == 0.0
        if g["schmidt"] is not None:
            assert rel(ds[so:so + K], g["schmidt"]) < 1e-9
        ro += M
        to += M * M
        so += K


def test_adjoint_at_order_243_matches_autograd_oracle():
    """A displaced 121-mode instance (bordered order 243: fifteen full
    16-column steps of the blocked inverse and a last one of 3) against the
    autograd oracle."""
    import torch
    rng = W.rng_for(82)
    M = 121
    T = np.sqrt(0.5) * W.haar_unitary(M, rng)
    alpha = 0.1 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    x = W.make_instance(T, rng.uniform(0.1, 0.4, M), alpha=alpha, bin_of=W.contiguous_bins([60, 61]),
                        cutoff=[1, 2], grid=[2, 3])
    d = np.random.default_rng(13).standard_normal((2, 3))
    _say("adjoint at order 243 vs autograd oracle")
    with cgd.Context([x], flags=cgd.FLAG_GRAD) as ctx:
        ctx.eval()
        dr, dT, da = (t.cpu().numpy() for t in ctx.grad(torch.tensor(d.ravel(), dtype=torch.float64, device="cuda")))
        torch.cuda.synchronize()
    g = og.gradients_full(x, d)
    for name, a, b in (("r", dr, g["r"]), ("T", dT.reshape(M, M), g["T"]), ("alpha", da, g["alpha"])):
        e = np.abs(a - b).max() / np.abs(b).max()
        _say(f"  {name}: relative max error {e:.2e}")
        assert e < 1e-9, name

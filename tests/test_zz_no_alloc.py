"""cgd_eval_static, the evaluation entry point that allocates nothing (its
per-evaluation buffers live in a static device array), against cgd_eval on
the same contexts: identical probabilities and error bounds, for two calls in
a row whose second has a smaller input, in both precisions; oversized
contexts are refused with a clear error."""
import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _big():
    edge = W.make_instance(np.sqrt(0.7) * W.haar_unitary(5, W.rng_for(123)), np.full(5, 0.4),
                           alpha=0.2 * np.ones(5, np.complex128), schmidt=[0.6, 0.3, 0.1],
                           bin_of=[2, 0, -1, 1, 0], cutoff=[3, 2, 4], grid=[6, 5, 7])
    # per-point factorisations (FP32 and FP64 classes), the Hessenberg route
    # (two-bin GBS state) and a displaced instance with an unmeasured mode
    return [W.lossy_m16_k3(), W.gbs_m144(2), W.plain_m4(), edge] + W.uneven_batch(24)


def _small():
    return [W.plain_m4(grid=[9, 8])]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_matches_eval_on_two_calls_second_smaller(precision):
    import torch
    torch.cuda.set_device(0)
    ctxs = [cgd.Context(_big(), precision=precision), cgd.Context(_small(), precision=precision)]
    try:
        ref = []
        for ctx in ctxs:
            err = torch.full((ctx.n_inst,), -1.0, dtype=torch.float64, device="cuda")
            p = ctx.eval(err=err).clone()
            ref.append((p, err.clone()))
        torch.cuda.synchronize()
        got = []
        for ctx in ctxs:  # the second call has the smaller input
            _say(f"cgd_eval_static {precision}: {ctx.n_inst} instances, {ctx.n_points} points")
            p = torch.full((ctx.n_probs,), float("nan"), dtype=torch.float64, device="cuda")
            err = torch.full((ctx.n_inst,), -1.0, dtype=torch.float64, device="cuda")
            ctx.eval_static(p, err)
            torch.cuda.synchronize()
            got.append((p, err))
        for (pr, er), (pg, eg) in zip(ref, got):
            assert torch.equal(pr, pg), float((pr - pg).abs().max())
            assert torch.equal(er, eg)
        # a regular evaluation after the static ones still agrees
        p = ctxs[0].eval().clone()
        torch.cuda.synchronize()
        assert torch.equal(p, ref[0][0])
    finally:
        for ctx in ctxs:
            ctx.close()


def test_static_refuses_oversized_context():
    import torch
    # 2049 x 2048 evaluated points: its buffers need far more than the static array
    inst = W.make_instance(np.sqrt(0.5) * W.haar_unitary(2, W.rng_for(7)), np.full(2, 0.3),
                           bin_of=[0, 1], cutoff=[4, 4], grid=[4096, 2048])
    with cgd.Context([inst]) as ctx:
        with pytest.raises(cgd.CgdError) as e:
            ctx.eval_static()
        assert e.value.status == cgd.CGD_ERR_ARG and "bytes" in str(e.value)
        torch.cuda.synchronize()


def test_diagnostics_need_a_regular_evaluation_after_static():
    import torch
    with cgd.Context(_small()) as ctx:
        ctx.eval_static()
        torch.cuda.synchronize()
        with pytest.raises(cgd.CgdError) as e:
            ctx.grid_values()
        assert e.value.status == cgd.CGD_ERR_STATE
        ctx.eval()
        ctx.grid_values()
        torch.cuda.synchronize()

"""Write the full-box expected distributions of the benchmark workloads.

Test infrastructure.  Every stored number comes from the CPU oracle
(oracle/pgf.py, oracle/state.py) on the seeded inputs of workloads/: for each
instance, G(w) at every point of the whole roots-of-unity grid (no Hermitian
half grid: the oracle does not use that symmetry) by eigenvalues of D(w)XA
plus a dense solve, then the explicit inverse DFT over the box.  That is the
wrapped distribution P(b) = sum_{m >= 0} Pr(b + m o G) of Eq.
coarse_grained_prob on the stated grid, the quantity the library returns.

The per-point oracle calls are spread over worker processes (one BLAS thread
each); the arithmetic of each point is the oracle's, unchanged.

Usage (from the repository root):
    python tests/golden/make_golden.py [--workers 6] [name ...]
Names: lossy16_k3 gbs144_2bins gbs144_3bins mesh32_k4 uneven512_heavy.
Writes tests/golden/<name>.npz with, per instance i: P_i (the box, float64),
imag_i (max |Im| of the inverse DFT, a rounding witness), grid_i, cutoff_i;
uneven512_heavy also stores `index`, the instance numbers in the batch.
"""
from __future__ import annotations

import argparse
import itertools
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import pgf  # noqa: E402
from oracle import state as st  # noqa: E402

# The eight instances of the 512-instance batch with the most factorisation
# work on the device (grid points x K x (2M)^3): they take the largest size
# classes and dominate its evaluation time.
UNEVEN_HEAVY = [299, 236, 159, 151, 411, 350, 430, 246]

CASES = {
    "lossy16_k3": lambda: [W.lossy_m16_k3()],
    "gbs144_2bins": lambda: [W.gbs_m144(2)],
    "gbs144_3bins": lambda: [W.gbs_m144(3)],
    "mesh32_k4": lambda: W.mesh_batch(64),
    "uneven512_heavy": lambda: [W.uneven_instance(i) for i in UNEVEN_HEAVY],
}

_STATE = {}


def _init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _points(args):
    key, ks = args
    S, grid = _STATE[key]
    g = np.asarray(grid, dtype=float)
    return [np.exp(pgf.log_pgf(S, np.exp(2j * np.pi * np.asarray(k) / g))) for k in ks]


def oracle_box(inst, pool, key, chunk=64):
    """The oracle's wrapped distribution of one instance on its stated grid."""
    grid = [int(g) for g in inst["grid"]]
    ks = list(itertools.product(*[range(g) for g in grid]))
    tasks = [(key, ks[i:i + chunk]) for i in range(0, len(ks), chunk)]
    vals = np.empty(len(ks), dtype=np.complex128)
    pos = 0
    for part in pool.imap(_points, tasks):
        vals[pos:pos + len(part)] = part
        pos += len(part)
    P = pgf.inverse_dft(vals.reshape(grid), inst["cutoff"])
    return P.real, float(np.abs(P.imag).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(CASES))
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    for name in args.names:
        insts = CASES[name]()
        for i, inst in enumerate(insts):
            _STATE[(name, i)] = (st.assemble(inst), [int(g) for g in inst["grid"]])
        out = {}
        t0 = time.time()
        # fork after the states exist, so the workers inherit them
        with mp.get_context("fork").Pool(args.workers, initializer=_init) as pool:
            for i, inst in enumerate(insts):
                P, im = oracle_box(inst, pool, (name, i))
                out[f"P_{i}"] = P
                out[f"imag_{i}"] = np.float64(im)
                out[f"grid_{i}"] = np.asarray(inst["grid"], np.int32)
                out[f"cutoff_{i}"] = np.asarray(inst["cutoff"], np.int32)
                print(f"{name}[{i}] box {P.shape} sum {P.sum():.15f} max|Im| {im:.2e} "
                      f"({time.time() - t0:.0f} s)", flush=True)
        if name == "uneven512_heavy":
            out["index"] = np.asarray(UNEVEN_HEAVY, np.int32)
        np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
        for i in range(len(insts)):
            _STATE.pop((name, i))


if __name__ == "__main__":
    main()

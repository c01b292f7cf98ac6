"""Seeded synthetic inputs for coarse-grained photon-number workloads.

This module only draws random numbers and builds input objects (Haar unitaries,
beamsplitter meshes, bin partitions, parameter draws).  It contains none of the
arithmetic of the method itself, so both the CPU oracle and the GPU path can
take their inputs from here without sharing any computation.

An *instance* is a plain dict:

    T                M x M complex128 transfer matrix, a_out = T a_in
    r                M float64 squeezing parameters of Schmidt mode 0
    alpha            M complex128 displacements of Schmidt mode 0, or None
    schmidt          K float64 Schmidt weights (sum 1, descending) or None (K=1)
    bin_of           int32 bin index per measured mode, -1 = not measured
                     (traced out), KEEP = -2 = kept (the heralded modes whose
                     density matrix is returned); length M (bins over external
                     modes) or M*K when resolve_internal is 1 (index i*K + k)
    resolve_internal 0 or 1
    cutoff           int32 per bin: output box b_l in [0, cutoff_l]
    grid             int32 per bin: roots-of-unity grid extent G_l >= cutoff_l+1
    fock_cutoff      (only with kept modes) Fock cutoff N of every kept mode:
                     density matrix elements <v|rho|u> for u, v in [0, N]

Workload shapes follow the paper's physical settings: single-mode squeezed
inputs on a lossy interferometer (Sec. II, Sec. VIII C), internal Schmidt
modes (Sec. VI B, Sec. VIII A) and binned detection (Sec. VI A).
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = (2412, 17742)
KEEP = -2  # bin_of value of a kept (heralded) mode


def rng_for(stream: int, inst: int = 0) -> np.random.Generator:
    """Counter-style seeding: one independent PCG64 stream per (workload stream, instance)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([*SEED_ROOT, stream, inst])))


def haar_unitary(m: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random m x m unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri's recipe)."""
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def contiguous_bins(sizes) -> np.ndarray:
    """bin_of for consecutive blocks of the given sizes."""
    return np.concatenate([np.full(s, l, dtype=np.int32) for l, s in enumerate(sizes)])


def schmidt_geometric(K: int, ratio: float) -> np.ndarray | None:
    if K == 1:
        return None
    w = ratio ** np.arange(K, dtype=np.float64)
    return w / w.sum()


def make_instance(T, r, alpha=None, schmidt=None, bin_of=None, cutoff=None, grid=None,
                  resolve_internal=0, fock_cutoff=None, distinguishable=0) -> dict:
    T = np.ascontiguousarray(T, dtype=np.complex128)
    M = T.shape[0]
    cutoff = np.asarray(cutoff, dtype=np.int32)
    grid = cutoff + 1 if grid is None else np.asarray(grid, dtype=np.int32)
    extra = {} if fock_cutoff is None else {"fock_cutoff": int(fock_cutoff)}
    if distinguishable:
        extra["distinguishable"] = 1
    return dict(**extra,
        T=T,
        r=np.ascontiguousarray(r, dtype=np.float64),
        alpha=None if alpha is None else np.ascontiguousarray(alpha, dtype=np.complex128),
        schmidt=None if schmidt is None else np.ascontiguousarray(schmidt, dtype=np.float64),
        bin_of=np.ascontiguousarray(bin_of if bin_of is not None else np.zeros(M), dtype=np.int32),
        resolve_internal=int(resolve_internal),
        cutoff=cutoff,
        grid=np.ascontiguousarray(grid, dtype=np.int32),
    )


def n_internal(inst: dict) -> int:
    if inst.get("distinguishable", 0):
        return inst["T"].shape[0]
    return 1 if inst["schmidt"] is None else len(inst["schmidt"])


def distinguishable_instance(M, seed, bins, cutoff, grid=None, eta=0.6, r_range=(0.3, 0.9)) -> dict:
    """M single-mode squeezed vacua in mutually orthogonal spectral modes
    (fully distinguishable, App. D) on sqrt(eta) x Haar: input j squeezed
    (r_j ~ U[r_range]) in its own internal mode j; contiguous bins of the
    given sizes, detectors blind to the internal mode."""
    rng = rng_for(7000 + seed)
    U = haar_unitary(M, rng)
    r = rng.uniform(r_range[0], r_range[1], M)
    return make_instance(np.sqrt(eta) * U, r, bin_of=contiguous_bins(bins), cutoff=cutoff, grid=grid,
                         distinguishable=1)


# ---------------------------------------------------------------------------
# The benchmark workloads: seeded synthetic inputs with the shapes and value
# distributions of the paper's settings (lossy interferometers, Schmidt
# modes, GBS scale, uneven batches, parameter meshes).
# ---------------------------------------------------------------------------

def plain_m4(grid=None) -> dict:
    """M=4 single-mode squeezed vacua (r=0.5) on sqrt(0.5)*Haar, K=1, no
    displacement, bins {0,1},{2,3}, cutoff 6 (grid 7x7 unless overridden)."""
    rng = rng_for(1)
    U = haar_unitary(4, rng)
    return make_instance(np.sqrt(0.5) * U, np.full(4, 0.5), bin_of=contiguous_bins([2, 2]),
                         cutoff=[6, 6], grid=grid)


def lossy_m16_k3(grid=None) -> dict:
    """M=16, K=3 (weights ~0.6^k), r~U[0.3,0.9], T=sqrt(0.4)*Haar, alpha~CN(0,0.1)
    on a seeded half of the inputs, 4 contiguous bins of 4, cutoff 10."""
    rng = rng_for(2)
    M = 16
    r = rng.uniform(0.3, 0.9, M)
    U = haar_unitary(M, rng)
    alpha = np.zeros(M, dtype=np.complex128)
    idx = rng.choice(M, M // 2, replace=False)
    # CN(0, 0.1): E|alpha|^2 = 0.1, i.e. real and imaginary parts ~ N(0, 0.05)
    alpha[idx] = np.sqrt(0.05) * (rng.standard_normal(M // 2) + 1j * rng.standard_normal(M // 2))
    return make_instance(np.sqrt(0.4) * U, r, alpha=alpha, schmidt=schmidt_geometric(3, 0.6),
                         bin_of=contiguous_bins([4, 4, 4, 4]), cutoff=[10] * 4, grid=grid)


def uneven_instance(i: int) -> dict:
    """One of the 512 uneven batching instances."""
    rng = rng_for(3, i)
    M = int(rng.integers(8, 65))
    K = int(rng.integers(1, 5))
    L = int(min(rng.integers(1, 5), M))
    cuts = np.sort(rng.choice(np.arange(1, M), L - 1, replace=False)) if L > 1 else np.array([], int)
    sizes = np.diff(np.concatenate([[0], cuts, [M]]))
    cutoff = rng.integers(4, 13, L)
    r = rng.uniform(0.2, 1.0, M)
    t = rng.uniform(0.2, 0.9)
    U = haar_unitary(M, rng)
    return make_instance(np.sqrt(t) * U, r, schmidt=schmidt_geometric(K, 0.6),
                         bin_of=contiguous_bins(sizes), cutoff=cutoff)


def uneven_batch(n: int = 512) -> list[dict]:
    return [uneven_instance(i) for i in range(n)]


def gbs_m144(bins: int = 2) -> dict:
    """GBS scale: M=144, K=1, r~U[0.4,1.2], T=sqrt(0.3)*Haar, no displacement.
    bins=2: 2 bins of 72, cutoff 120; bins=3: 3 bins of 48, cutoff 40."""
    if bins not in (2, 3):
        raise ValueError("gbs_m144 has 2 or 3 bins")
    rng = rng_for(4)
    M = 144
    r = rng.uniform(0.4, 1.2, M)
    U = haar_unitary(M, rng)
    if bins == 2:
        return make_instance(np.sqrt(0.3) * U, r, bin_of=contiguous_bins([72, 72]), cutoff=[120, 120])
    return make_instance(np.sqrt(0.3) * U, r, bin_of=contiguous_bins([48, 48, 48]), cutoff=[40, 40, 40])


def dist_m144(cutoff: int = 40) -> dict:
    """The circuit and squeezers of gbs_m144(3) with the 144 inputs fully
    distinguishable (App. D: input j in its own internal mode j, K = M = 144):
    3 bins of 48, the given cutoff per bin."""
    x = gbs_m144(3)
    return make_instance(x["T"], x["r"], bin_of=x["bin_of"], cutoff=[cutoff] * 3, distinguishable=1)


# --- total photon number of a GBS setup (the paper's Sec. VIII C) ----------

# cutoffs N_max the paper uses for M = 16 .. 256 (Fig. total_probs_time_comparison)
TOTAL_PHOTON_CUTOFF = {16: 27, 32: 45, 64: 71, 128: 109, 256: 170}


def gbs_total(M: int, cutoff: int | None = None, grid=None) -> dict:
    """M spectrally pure single-mode squeezed vacua with equal squeezing
    xi = 0.89 on T = sqrt(0.36) U, U Haar, no displacement, one bin over all
    modes (total photon number), cutoff N_max from the paper's list."""
    rng = rng_for(6, M)
    U = haar_unitary(M, rng)
    N = TOTAL_PHOTON_CUTOFF.get(M, 2 * M) if cutoff is None else cutoff
    return make_instance(np.sqrt(0.36) * U, np.full(M, 0.89), bin_of=np.zeros(M, np.int32), cutoff=[N],
                         grid=grid)


# --- workload 5: differentiable state-preparation parameters -----------------

def mesh_layout(M: int):
    """Rectangular (Clements-style) mesh: M layers alternating even/odd
    nearest-neighbour pairs; returns a list of (layer, mode) for each of the
    M(M-1)/2 beamsplitters."""
    pairs = []
    for layer in range(M):
        for i in range(layer % 2, M - 1, 2):
            pairs.append((layer, i))
    assert len(pairs) == M * (M - 1) // 2
    return pairs


def mesh_unitary(theta, phases, M: int):
    """U(theta): product of real beamsplitters [[cos, -sin],[sin, cos]] on
    adjacent modes, each preceded by a fixed phase exp(i*phi) on its first mode.
    Works on numpy arrays and on torch tensors (differentiable in theta)."""
    try:
        import torch
        is_torch = isinstance(theta, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_torch = False
    if is_torch:
        import torch
        U = torch.eye(M, dtype=torch.complex128)
        ph = torch.as_tensor(np.exp(1j * np.asarray(phases)), dtype=torch.complex128)
        c, s = torch.cos(theta).to(torch.complex128), torch.sin(theta).to(torch.complex128)
        for b, (_, i) in enumerate(mesh_layout(M)):
            row_i = ph[b] * U[i]
            row_j = U[i + 1]
            U = U.clone()
            U[i] = c[b] * row_i - s[b] * row_j
            U[i + 1] = s[b] * row_i + c[b] * row_j
        return U
    U = np.eye(M, dtype=np.complex128)
    ph = np.exp(1j * np.asarray(phases))
    c, s = np.cos(theta), np.sin(theta)
    for b, (_, i) in enumerate(mesh_layout(M)):
        row_i = ph[b] * U[i]
        row_j = U[i + 1].copy()
        U[i] = c[b] * row_i - s[b] * row_j
        U[i + 1] = s[b] * row_i + c[b] * row_j
    return U


def mesh_params(n_sets: int = 64):
    """Parameter sets for the differentiation workload: M=32, K=4 (weights
    ~0.5^k), r~U[0.3,1.0], loss~U[0.1,0.5] per mode (eta = 1-loss), 496 mesh
    angles, fixed phase screen shared by all sets."""
    M = 32
    prng = rng_for(5, 10_000)
    phases = prng.uniform(0, 2 * np.pi, M * (M - 1) // 2)
    sets = []
    for s in range(n_sets):
        rng = rng_for(5, s)
        sets.append(dict(r=rng.uniform(0.3, 1.0, M), eta=1.0 - rng.uniform(0.1, 0.5, M),
                         theta=rng.uniform(0, 2 * np.pi, M * (M - 1) // 2)))
    return dict(M=M, K=4, schmidt=schmidt_geometric(4, 0.5), phases=phases,
                bin_of=contiguous_bins([16, 16]), cutoff=np.array([12, 12], np.int32), sets=sets)


def mesh_transfer(eta, theta, phases, M=32):
    """T = diag(sqrt(eta)) U(theta); numpy or torch (differentiable)."""
    U = mesh_unitary(theta, phases, M)
    try:
        import torch
        if isinstance(eta, torch.Tensor):
            return torch.sqrt(eta).to(torch.complex128)[:, None] * U
    except ImportError:  # pragma: no cover
        pass
    return np.sqrt(eta)[:, None] * U


def mesh_batch(n_sets: int = 64) -> list[dict]:
    p = mesh_params(n_sets)
    out = []
    for s in p["sets"]:
        T = mesh_transfer(s["eta"], s["theta"], p["phases"], p["M"])
        out.append(make_instance(T, s["r"], schmidt=p["schmidt"], bin_of=p["bin_of"], cutoff=p["cutoff"]))
    return out


# --- paper's Fock-heralding setup (Sec. VIII A) -----------------------------

def fock_herald_instance(p: float, eta: float, xi: float = 1.1, cutoff=(3, 3), grid=None) -> dict:
    """Two equally squeezed inputs (xi) on the balanced beamsplitter
    U = [[1, i],[i, 1]]/sqrt(2) with uniform transmission eta, two internal
    (spectral) modes with weights (p, 1-p).  Bins over internal-resolved modes:
    bin 0 = port 0 (both spectral modes, the herald), bin 1 = port 1 spectral
    mode 0 (the heralded mode); port 1 spectral mode 1 is traced out."""
    U = np.array([[1, 1j], [1j, 1]], dtype=np.complex128) / np.sqrt(2.0)
    T = np.sqrt(eta) * U
    if p >= 1.0:
        schmidt = None
        bin_of = np.array([0, 1], np.int32)
    else:
        schmidt = np.array([p, 1 - p])
        bin_of = np.array([0, 0, 1, -1], np.int32)  # index i*K + k
    return make_instance(T, np.full(2, xi), schmidt=schmidt, bin_of=bin_of, cutoff=list(cutoff),
                         grid=grid, resolve_internal=1)


def gkp_like(p: float, eta: float, seed: int = 0, herald=(5, 7), fock_cutoff: int = 26) -> dict:
    """The shape of the approximate-GKP heralding setup of Sec. VIII B: three
    squeezed inputs on sqrt(eta) x a 3 x 3 unitary, two spectral modes with
    weights (p, 1 - p) (one mode for p >= 1), the first two output ports
    measured (one bin each, both spectral modes; cutoffs = the heralding
    pattern (5, 7)), spectral mode 0 of port 2 kept with Fock cutoff 26 and
    its spectral mode 1 traced out.  The paper takes the squeezing and the
    unitary from a reference that is not available here; these are seeded
    draws (r ~ U[0.6, 1.2], Haar U) of the same shape."""
    rng = rng_for(70, seed)
    U = haar_unitary(3, rng)
    r = rng.uniform(0.6, 1.2, 3)
    if p >= 1.0:
        schmidt, bin_of = None, [0, 1, KEEP]
    else:
        schmidt, bin_of = np.array([p, 1.0 - p]), [0, 0, 1, 1, KEEP, -1]
    return make_instance(np.sqrt(eta) * U, r, schmidt=schmidt, bin_of=bin_of, cutoff=list(herald),
                         resolve_internal=1, fock_cutoff=fock_cutoff)


def gkp_like_map(n: int = 50, seed: int = 0) -> list[dict]:
    """n x n grid of gkp_like states over p in [0.7, 0.99] and eta in [0.8, 1.0]
    (the parameter ranges of the paper's GKP fidelity map), same unitary and
    squeezing for all; p runs slowest."""
    return [gkp_like(p, eta, seed) for p in np.linspace(0.7, 0.99, n) for eta in np.linspace(0.8, 1.0, n)]


def fock_herald_density(p: float, eta: float, xi: float = 1.1, herald: int = 3, fock_cutoff: int = 6) -> dict:
    """fock_herald_instance with port 1, spectral mode 0 kept instead of
    binned: the heralded state's density matrix for the pattern `herald` in
    port 0 (and every smaller one)."""
    inst = fock_herald_instance(p, eta, xi, cutoff=(herald, 0))
    b = inst["bin_of"].copy()
    b[b == 1] = KEEP
    return make_instance(inst["T"], inst["r"], schmidt=inst["schmidt"], bin_of=b, cutoff=[herald],
                         resolve_internal=1, fock_cutoff=fock_cutoff)

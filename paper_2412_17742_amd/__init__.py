"""Coarse-grained photon-number distributions of Gaussian states on MI355X.

Thin Python binding over the C ABI of libcgd.so (include/cgd.h): argument
marshalling only.  Every step of the evaluation runs in the library's HIP
kernels; PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the library is missing, importing the binding succeeds but every
call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgd.so")

CGD_OK, CGD_ERR_ARG, CGD_ERR_NONPHYSICAL, CGD_ERR_NUMERIC, CGD_ERR_DEVICE, CGD_ERR_NOMEM, CGD_ERR_STATE = range(7)
STATUS_NAMES = ["CGD_OK", "CGD_ERR_ARG", "CGD_ERR_NONPHYSICAL", "CGD_ERR_NUMERIC", "CGD_ERR_DEVICE",
                "CGD_ERR_NOMEM", "CGD_ERR_STATE"]
PREC_FP64, PREC_MIXED = 0, 1
FLAG_DENSE_INTERNAL = 1
FLAG_NO_SCHUR = 2
FLAG_GRAD = 4
FLAG_HESSENBERG = 8
FLAG_NO_HESSENBERG = 16
FLAG_NO_AUTOTUNE = 32
FLAG_MOMENTS = 64
FLAG_CUMULANTS = 128
FLAG_NO_LOWRANK = 256
KEEP = -2  # bin_of value of a kept mode (heralded density matrices)
# launch stages of one evaluation (per-stage timing); LU stages are order buckets
STAGES = ["schur", "lu_le32", "lu_le64", "lu_le96", "lu_le128", "lu_le144", "lu_gt144", "combine", "dft", "fix",
          "hess", "hess_det", "pair", "density"]
# the kernels behind each LU bucket: (FP64 path, FP32 first pass of the mixed path)
LU_KERNELS = {
    "lu_le32": ("lu_reg<double,8,8,4,4>", "lu_mfma_f32<2,1,2>"),
    "lu_le64": ("lu_reg<double,16,16,4,4>", "lu_mfma_f32<4,1,2,4>"),
    "lu_le96": ("lu_reg<double,16,32,6,3>", "lu_mfma_f32<6,2,2,3>"),
    "lu_le128": ("lu_reg<double,16,32,8,4>", "lu_mfma_f32<8,2,4>"),
    "lu_le144": ("lu_reg<double,16,48,9,3>", "lu_mfma_f32<9,3,4>"),
    "lu_gt144": ("lu_big_f64", "lu_mfma_f32<12,2,4> (orders <= 192)"),
}


class CgdError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {message}")


class CgdInstance(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("K", ctypes.c_int32), ("L", ctypes.c_int32),
        ("T", ctypes.c_void_p), ("r", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
        ("schmidt", ctypes.c_void_p), ("bin_of", ctypes.c_void_p),
        ("resolve_internal", ctypes.c_int32),
        ("cutoff", ctypes.c_void_p), ("grid", ctypes.c_void_p),
        ("fock_cutoff", ctypes.c_int32), ("distinguishable", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcgd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2412_17742_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.cgd_create.restype = i32
    L.cgd_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(CgdInstance), i32, i32, ctypes.c_double,
                             ctypes.c_uint32, vp]
    L.cgd_layout.restype = i32
    L.cgd_layout.argtypes = [vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64)]
    L.cgd_eval.restype = i32
    L.cgd_eval.argtypes = [vp, vp, vp]
    L.cgd_eval_static.restype = i32
    L.cgd_eval_static.argtypes = [vp, vp, vp]
    L.cgd_points.restype = i64
    L.cgd_points.argtypes = [vp]
    L.cgd_grid_values.restype = i32
    L.cgd_grid_values.argtypes = [vp, vp]
    L.cgd_grad.restype = i32
    L.cgd_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    L.cgd_set_timing.restype = i32
    L.cgd_set_timing.argtypes = [vp, i32]
    L.cgd_stage_times.restype = i32
    L.cgd_stage_times.argtypes = [vp, vp]
    L.cgd_stage_work.restype = i32
    L.cgd_stage_work.argtypes = [vp, vp, vp]
    L.cgd_mixed_stats.restype = i32
    L.cgd_mixed_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.cgd_bounds.restype = i32
    L.cgd_bounds.argtypes = [vp, vp, vp]
    L.cgd_set_kernel_shape.restype = i32
    L.cgd_set_kernel_shape.argtypes = [vp, i32, i32, i32]
    L.cgd_tuning.restype = ctypes.c_char_p
    L.cgd_tuning.argtypes = [vp]
    L.cgd_destroy.restype = None
    L.cgd_destroy.argtypes = [vp]
    L.cgd_last_error.restype = ctypes.c_char_p
    L.cgd_last_error.argtypes = []
    _lib = L
    return L


def _check(status: int):
    if status != CGD_OK:
        raise CgdError(status, lib().cgd_last_error().decode())


def _as(arr, dtype):
    return None if arr is None else np.ascontiguousarray(arr, dtype=dtype)


def _internal_modes(inst: dict) -> int:
    """K: M for fully distinguishable inputs, else the number of Schmidt weights (1 if none)."""
    if inst.get("distinguishable", 0):
        return int(np.asarray(inst["T"]).shape[0])
    return 1 if inst.get("schmidt") is None else len(inst["schmidt"])


def _marshal(inst: dict, keep: list) -> CgdInstance:
    T = _as(inst["T"], np.complex128)
    M = T.shape[0]
    K = _internal_modes(inst)
    arrays = dict(
        T=T, r=_as(inst["r"], np.float64), alpha=_as(inst.get("alpha"), np.complex128),
        schmidt=_as(inst.get("schmidt"), np.float64), bin_of=_as(inst["bin_of"], np.int32),
        cutoff=_as(inst["cutoff"], np.int32), grid=_as(inst.get("grid"), np.int32),
    )
    keep.append(arrays)
    ptr = {k: (None if v is None else v.ctypes.data) for k, v in arrays.items()}
    return CgdInstance(M, K, len(arrays["cutoff"]), ptr["T"], ptr["r"], ptr["alpha"], ptr["schmidt"],
                       ptr["bin_of"], int(inst.get("resolve_internal", 0)), ptr["cutoff"], ptr["grid"],
                       int(inst.get("fock_cutoff", 0)), int(inst.get("distinguishable", 0)))


def _density_dim(inst: dict):
    """D = (fock_cutoff + 1)^g for an instance with g kept modes, else None."""
    b = np.asarray(inst["bin_of"])
    K = _internal_modes(inst)
    g = int((b == KEEP).sum()) * (1 if inst.get("resolve_internal", 0) else K)
    return (int(inst.get("fock_cutoff", 0)) + 1) ** g if g else None


class Context:
    """A batch of instances prepared on the device (cgd_create)."""

    def __init__(self, instances, precision: str = "fp64", tol: float = 1e-9, flags: int = 0, stream=None):
        import torch
        if isinstance(instances, dict):
            instances = [instances]
        L = lib()
        keep: list = []
        arr = (CgdInstance * len(instances))(*[_marshal(x, keep) for x in instances])
        prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        _check(L.cgd_create(ctypes.byref(handle), arr, len(instances), prec, float(tol), int(flags),
                            ctypes.c_void_p(stream.cuda_stream)))
        self._h = handle
        self.n_inst = len(instances)
        n = ctypes.c_int64()
        ng = ctypes.c_int64()
        offs = np.zeros(self.n_inst + 1, dtype=np.int64)
        _check(L.cgd_layout(self._h, ctypes.byref(n), offs.ctypes.data, ctypes.byref(ng)))
        self.n_probs = n.value
        self.prob_offsets = offs
        self.n_grid = ng.value
        self.n_points = L.cgd_points(self._h)
        self.shapes = [tuple(int(c) + 1 for c in x["cutoff"]) for x in instances]
        self.density_dims = [_density_dim(x) for x in instances]
        self._M = [np.asarray(x["T"]).shape[0] for x in instances]
        self._K = [_internal_modes(x) for x in instances]

    def eval(self, probs=None, err=None):
        """Wrapped distributions of all instances, concatenated (device float64)."""
        import torch
        if probs is None:
            probs = torch.empty(self.n_probs, dtype=torch.float64, device="cuda")
        assert probs.dtype == torch.float64 and probs.is_cuda and probs.numel() >= self.n_probs
        assert probs.is_contiguous()
        if err is not None:
            assert err.dtype == torch.float64 and err.is_cuda and err.numel() >= self.n_inst
        _check(lib().cgd_eval(self._h, ctypes.c_void_p(probs.data_ptr()),
                              None if err is None else ctypes.c_void_p(err.data_ptr())))
        return probs

    def eval_static(self, probs=None, err=None):
        """As eval(), through cgd_eval_static: no device allocation inside the
        library call (its per-evaluation buffers are a static device array)."""
        import torch
        if probs is None:
            probs = torch.empty(self.n_probs, dtype=torch.float64, device="cuda")
        assert probs.dtype == torch.float64 and probs.is_cuda and probs.numel() >= self.n_probs
        assert probs.is_contiguous()
        if err is not None:
            assert err.dtype == torch.float64 and err.is_cuda and err.numel() >= self.n_inst
        _check(lib().cgd_eval_static(self._h, ctypes.c_void_p(probs.data_ptr()),
                                     None if err is None else ctypes.c_void_p(err.data_ptr())))
        return probs

    def split(self, probs):
        """Split the concatenated output into one array per instance: reshaped to
        the box, or for an instance with kept modes a complex view of shape
        box + (D, D) holding <v|rho(b~)|u> at [b~][v][u]."""
        import torch
        out = []
        for i in range(self.n_inst):
            lo = int(self.prob_offsets[i])  # a density instance's offset is even; a double of
            D = self.density_dims[i]         # padding before it ends the previous range
            nb = int(np.prod(self.shapes[i]))
            if D is None:
                out.append(probs[lo:lo + nb].reshape(self.shapes[i]))
            else:
                seg = probs[lo:lo + 2 * D * D * nb]
                out.append(torch.view_as_complex(seg.view(-1, 2)).reshape(self.shapes[i] + (D, D)))
        return out

    def grid_values(self):
        """log G at the evaluated grid points (complex128 device tensor)."""
        import torch
        out = torch.empty(2 * self.n_points, dtype=torch.float64, device="cuda")
        _check(lib().cgd_grid_values(self._h, ctypes.c_void_p(out.data_ptr())))
        return torch.view_as_complex(out.view(-1, 2))

    def grad(self, dprobs, schmidt=False):
        """Gradient of L with dL/dP = dprobs (device float64, n_probs): returns
        (dL/dr, dL/dRe T + i dL/dIm T, dL/dRe alpha + i dL/dIm alpha) as device
        tensors (instances concatenated; T flattened row-major), and with
        schmidt=True also dL/dlambda (each Schmidt weight free, instances
        concatenated)."""
        import torch
        assert dprobs.dtype == torch.float64 and dprobs.is_cuda and dprobs.is_contiguous()
        nM = int(sum(self._M))
        nT = int(sum(m * m for m in self._M))
        dr = torch.zeros(nM, dtype=torch.float64, device="cuda")
        dT = torch.zeros(2 * nT, dtype=torch.float64, device="cuda")
        da = torch.zeros(2 * nM, dtype=torch.float64, device="cuda")
        ds = torch.zeros(int(sum(self._K)), dtype=torch.float64, device="cuda")
        _check(lib().cgd_grad(self._h, ctypes.c_void_p(dprobs.data_ptr()), ctypes.c_void_p(dr.data_ptr()),
                              ctypes.c_void_p(dT.data_ptr()), ctypes.c_void_p(da.data_ptr()),
                              ctypes.c_void_p(ds.data_ptr())))
        out = (dr, torch.view_as_complex(dT.view(-1, 2)), torch.view_as_complex(da.view(-1, 2)))
        return out + (ds,) if schmidt else out

    def set_timing(self, enable: bool = True):
        _check(lib().cgd_set_timing(self._h, int(enable)))

    def stage_times(self):
        """ms per stage of the last evaluation (-1: stage had no work); waits for it."""
        ms = np.zeros(len(STAGES))
        _check(lib().cgd_stage_times(self._h, ms.ctypes.data))
        return dict(zip(STAGES, ms))

    def stage_work(self):
        """(flops, bytes) per stage and evaluation, algorithmic counts."""
        f = np.zeros(len(STAGES))
        b = np.zeros(len(STAGES))
        _check(lib().cgd_stage_work(self._h, f.ctypes.data, b.ctypes.data))
        return dict(zip(STAGES, f)), dict(zip(STAGES, b))

    def mixed_stats(self):
        """(factorisations repeated in FP64 by the last mixed evaluation, total per evaluation)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().cgd_mixed_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def bounds(self):
        """(grid extents per instance with automatic entries resolved, wrap-tail
        bound per instance: 0 <= P_wrap(b) - Pr(b) <= bound for every b in the box)."""
        nL = sum(len(s) for s in self.shapes)
        g = np.zeros(nL, np.int32)
        w = np.zeros(self.n_inst, np.float64)
        _check(lib().cgd_bounds(self._h, g.ctypes.data, w.ctypes.data))
        out, off = [], 0
        for s in self.shapes:
            out.append(tuple(int(x) for x in g[off:off + len(s)]))
            off += len(s)
        return out, w

    def set_kernel_shape(self, size_class: int, fp64_shape: int = -1, fp32_shape: int = -1):
        """Pin a size class's FP64 and/or FP32 kernel shape (indices into the
        tuning report's per-class timing lists; -1 keeps the current one)."""
        _check(lib().cgd_set_kernel_shape(self._h, int(size_class), int(fp64_shape), int(fp32_shape)))

    def tuning(self):
        """The autotuner's report (dict): per size class, the timed kernels and the choice."""
        import json
        return json.loads(lib().cgd_tuning(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().cgd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def binned_distribution(instances, precision: str = "fp64", tol: float = 1e-9, flags: int = 0):
    """Evaluate and return one float64 device tensor per instance."""
    with Context(instances, precision, tol, flags) as ctx:
        probs = ctx.eval()
        import torch
        torch.cuda.current_stream().synchronize()
        return [p.clone() for p in ctx.split(probs)]


class _Distribution:
    """torch.autograd.Function over a batch of instances that share their
    binning: forward = cgd_eval, backward = cgd_grad."""

    @staticmethod
    def make():
        import torch

        class Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, r, T, alpha, schmidt, spec):
                B, M = r.shape
                insts = []
                for b in range(B):
                    lam = spec.get("schmidt") if schmidt is None else schmidt[b].detach().cpu().numpy()
                    insts.append(dict(
                        T=T[b].detach().cpu().numpy(), r=r[b].detach().cpu().numpy(),
                        alpha=None if alpha is None else alpha[b].detach().cpu().numpy(),
                        schmidt=lam, bin_of=spec["bin_of"], cutoff=spec["cutoff"],
                        grid=spec.get("grid"), resolve_internal=spec.get("resolve_internal", 0)))
                c = Context(insts, flags=FLAG_GRAD)
                P = c.eval().clone()
                ctx.c = c
                ctx.B, ctx.M = B, M
                ctx.has_alpha = alpha is not None
                ctx.has_schmidt = schmidt is not None
                ctx.devices = (r.device, T.device, None if alpha is None else alpha.device,
                               None if schmidt is None else schmidt.device)
                shape = tuple(int(x) + 1 for x in spec["cutoff"])
                return P.view(B, *shape)

            @staticmethod
            def backward(ctx, gP):
                dr, dT, da, ds = ctx.c.grad(gP.contiguous().view(-1).to(torch.float64), schmidt=True)
                ctx.c.close()
                B, M = ctx.B, ctx.M
                dr = dr.view(B, M).to(ctx.devices[0])
                dT = dT.view(B, M, M).to(ctx.devices[1])
                da = da.view(B, M).to(ctx.devices[2]) if ctx.has_alpha else None
                ds = ds.view(B, -1).to(ctx.devices[3]) if ctx.has_schmidt else None
                return dr, dT, da, ds, None

        return Fn


_fn = None


def distribution(r, T, alpha, spec, schmidt=None):
    """Differentiable binned distributions of a batch of states with one binning.

    r: (B, M) float64, T: (B, M, M) complex128, alpha: (B, M) complex128 or None,
    schmidt: (B, K) float64 Schmidt weights or None (then spec["schmidt"] for
    every instance, not differentiated) (torch tensors, any device); spec: dict
    with schmidt, bin_of, cutoff and optionally grid and resolve_internal.
    Returns a (B, N_1+1, ..., N_L+1) float64 CUDA tensor; backward runs the
    library's adjoint (gradients with respect to r, T, alpha and schmidt, each
    Schmidt weight a free variable)."""
    global _fn
    if _fn is None:
        _fn = _Distribution.make()
    return _fn.apply(r, T, alpha, schmidt, spec)

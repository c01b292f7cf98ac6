"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every function include/cgd.h declares, and rejects invalid arguments
before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2412_17742_amd as cgd
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "cgd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert {"cgd_create", "cgd_eval", "cgd_grad", "cgd_destroy", "cgd_layout", "cgd_last_error"} <= set(names)
    L = ctypes.CDLL(cgd.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def _create(inst, **kw):
    keep = []
    arr = (cgd.CgdInstance * 1)(cgd._marshal(inst, keep))
    h = ctypes.c_void_p()
    st = cgd.lib().cgd_create(ctypes.byref(h), arr, 1, kw.get("prec", 0), kw.get("tol", 1e-9), kw.get("flags", 0), None)
    return st, h, cgd.lib().cgd_last_error().decode()


@pytest.mark.parametrize("mutate, status", [
    (lambda x: x.update(T=2.0 * x["T"]), cgd.CGD_ERR_NONPHYSICAL),
    (lambda x: x.update(r=-x["r"]), cgd.CGD_ERR_NONPHYSICAL),
    (lambda x: x["r"].__setitem__(0, np.nan), cgd.CGD_ERR_NONPHYSICAL),
    (lambda x: x.update(bin_of=np.array([0, 0, 2, 1], np.int32)), cgd.CGD_ERR_ARG),
    (lambda x: x.update(cutoff=np.array([-1, 6], np.int32)), cgd.CGD_ERR_ARG),
    (lambda x: x.update(grid=np.array([6, 7], np.int32)), cgd.CGD_ERR_ARG),
    (lambda x: x.update(schmidt=np.array([0.5, 0.4])), cgd.CGD_ERR_NONPHYSICAL),
    (lambda x: x.update(schmidt=np.array([0.3, 0.7])), cgd.CGD_ERR_NONPHYSICAL),
])
def test_create_rejects_invalid_instances(mutate, status):
    inst = W.plain_m4()
    mutate(inst)
    st, h, msg = _create(inst)
    assert st == status, msg
    assert h.value is None
    assert msg


def test_create_rejects_bad_call_arguments():
    L = cgd.lib()
    h = ctypes.c_void_p()
    assert L.cgd_create(ctypes.byref(h), None, 1, 0, 1e-9, 0, None) == cgd.CGD_ERR_ARG
    keep = []
    arr = (cgd.CgdInstance * 1)(cgd._marshal(W.plain_m4(), keep))
    assert L.cgd_create(ctypes.byref(h), arr, 1, 7, 1e-9, 0, None) == cgd.CGD_ERR_ARG
    assert L.cgd_create(ctypes.byref(h), arr, 1, cgd.PREC_MIXED, 0.0, 0, None) == cgd.CGD_ERR_ARG
    assert L.cgd_create(ctypes.byref(h), arr, 1, 0, 1e-9, 1 << 20, None) == cgd.CGD_ERR_ARG
    both = cgd.FLAG_HESSENBERG | cgd.FLAG_NO_HESSENBERG
    assert L.cgd_create(ctypes.byref(h), arr, 1, 0, 1e-9, both, None) == cgd.CGD_ERR_ARG
    assert L.cgd_eval(None, None, None) == cgd.CGD_ERR_ARG
    assert L.cgd_grad(None, None, None, None, None, None) == cgd.CGD_ERR_ARG
    L.cgd_destroy(None)


def test_automatic_grid_needs_a_finite_tolerance():
    # grid entry 0 asks for an automatic grid from the tail bound, which needs tol
    inst = W.plain_m4()
    inst["grid"] = np.array([0, 7], np.int32)
    for tol in (0.0, float("inf")):
        st, h, msg = _create(inst, tol=tol)
        assert st == cgd.CGD_ERR_ARG and "tol" in msg, msg
    inst["grid"] = np.array([0, 5], np.int32)  # the explicit entry is still checked
    st, h, msg = _create(inst, tol=1e-9)
    assert st == cgd.CGD_ERR_ARG and "grid" in msg, msg


def test_density_mode_arguments_are_checked_before_the_device():
    """Kept modes (bin CGD_KEEP): FP64 only, no gradient or moments flags,
    valid bin codes and Fock cutoffs, at most 2^22 matrix elements per point."""
    base = W.gkp_like(0.9, 0.95)
    bad = [
        (dict(prec=cgd.PREC_MIXED), "FP64"),
        (dict(flags=cgd.FLAG_GRAD), "FP64"),
        (dict(flags=cgd.FLAG_MOMENTS), "FP64"),
    ]
    for kw, word in bad:
        st, h, msg = _create(base, **kw)
        assert st == cgd.CGD_ERR_ARG and word in msg, msg
        assert h.value is None
    for mutate, word in [
        (lambda x: x["bin_of"].__setitem__(0, -3), "bin index"),
        (lambda x: x.update(fock_cutoff=-1), "fock_cutoff"),
        (lambda x: x.update(fock_cutoff=4095), "2^22"),
        (lambda x: x.update(bin_of=np.full(6, cgd.KEEP, np.int32)), "kept modes"),  # 2g = 12 but N = 26
    ]:
        x = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        mutate(x)
        st, h, msg = _create(x)
        assert st == cgd.CGD_ERR_ARG and (word in msg or "2^22" in msg), msg


def test_set_kernel_shape_checks_its_arguments():
    L = cgd.lib()
    assert L.cgd_set_kernel_shape(None, 0, 0, -1) == cgd.CGD_ERR_ARG


def test_distinguishable_instances_are_checked_before_the_device():
    """Fully distinguishable inputs (App. D): K == M, no Schmidt weights, no
    displacement, no gradient; an unknown flag bit is still refused."""
    base = W.distinguishable_instance(4, 0, [2, 2], [3, 3])
    assert W.n_internal(base) == 4 and base["distinguishable"] == 1
    for mutate in [
        lambda x: x.update(schmidt=np.full(4, 0.25)),
        lambda x: x.update(alpha=np.full(4, 0.1 + 0.0j)),
    ]:
        x = dict(base)
        mutate(x)
        st, h, msg = _create(x)
        assert st == cgd.CGD_ERR_ARG and "distinguishable" in msg, msg
        assert h.value is None
    keep = []
    one = cgd._marshal(base, keep)
    one.K = 3
    arr = (cgd.CgdInstance * 1)(one)
    h = ctypes.c_void_p()
    assert cgd.lib().cgd_create(ctypes.byref(h), arr, 1, 0, 1e-9, 0, None) == cgd.CGD_ERR_ARG
    assert "distinguishable" in cgd.lib().cgd_last_error().decode()
    st, h, msg = _create(base, flags=cgd.FLAG_GRAD)
    assert st == cgd.CGD_ERR_ARG and "distinguishable" in msg, msg
    st, h, msg = _create(base, flags=1 << 9)
    assert st == cgd.CGD_ERR_ARG and "flags" in msg, msg

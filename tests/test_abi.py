"""The C interface without a GPU: the library loads, exports every entry
point that include/pn.h declares, and rejects invalid arguments before it
touches a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pn_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_0908_3889_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpn.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"pn_integrate", "pn_rhs", "pn_observables", "pn_strerror"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_0908_3889_amd import _lib
    assert set(_lib.EXPORTS) == set(_declared())


def test_strerror_and_version(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.pn_strerror(code).decode().startswith("PN_")
    assert lib.pn_version().decode()


def test_opts_struct_layout_matches_header():
    from paper_0908_3889_amd._lib import PnOpts
    # 3 doubles, one int64, seven int32 padded to 8 bytes, two pointers
    assert C.sizeof(PnOpts) == 3 * 8 + 8 + 7 * 4 + 4 + 2 * 8
    assert PnOpts.order.offset == 64 and PnOpts.packed.offset == 72
    names = [f[0] for f in PnOpts._fields_]
    src = open(os.path.join(ROOT, "include", "pn.h")).read()
    body = src[src.index("typedef struct pn_opts"):src.index("} pn_opts;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    assert re.findall(r"\b(\w+);", body) == names


def test_invalid_arguments_return_einval_without_a_device(lib):
    from paper_0908_3889_amd._lib import PnOpts, PN_EINVAL, PN_OK
    z = C.c_void_p(0)
    fake = C.c_void_p(0x1000)       # never dereferenced: validation fails first
    o = PnOpts()
    call = lambda n, ld, tol=1e-8, wf=0.05, ptr=fake, opt=o: lib.pn_integrate(
        n, ld, ptr, ptr, ptr, ptr, wf, tol, C.byref(opt), ptr, ptr, ptr, ptr, z, z)
    assert call(-1, 0) == PN_EINVAL
    assert call(10, 5) == PN_EINVAL
    assert call(10, 10, ptr=z) == PN_EINVAL
    assert call(10, 10, tol=0.0) == PN_EINVAL
    assert call(10, 10, tol=float("nan")) == PN_EINVAL
    assert call(10, 10, wf=-1.0) == PN_EINVAL
    bad = PnOpts(); bad.block = 96
    assert call(10, 10, opt=bad) == PN_EINVAL
    bad = PnOpts(); bad.schedule = 7
    assert call(10, 10, opt=bad) == PN_EINVAL
    bad = PnOpts(); bad.h_fixed = -1.0
    assert call(10, 10, opt=bad) == PN_EINVAL
    bad = PnOpts(); bad.terms = 64
    assert call(10, 10, opt=bad) == PN_EINVAL
    bad = PnOpts(); bad.precision = 3
    assert call(10, 10, opt=bad) == PN_EINVAL
    bad = PnOpts(); bad.packed = C.c_void_p(0x1008)  # input records must be 16-byte aligned
    assert call(10, 10, opt=bad) == PN_EINVAL
    assert call(0, 0) == PN_OK                       # empty batch: nothing to do
    ph = lambda n, ld, out, tol=1e-8: lib.pn_integrate_phase(
        n, ld, fake, fake, fake, fake, 0.05, tol, C.byref(o), fake, fake, fake, fake, z, out, z)
    assert ph(10, 10, z) == PN_EINVAL                # the phase output is required
    assert ph(10, 10, fake, tol=-1.0) == PN_EINVAL
    assert ph(10, 5, fake) == PN_EINVAL
    assert ph(0, 0, z) == PN_OK
    d1, d2 = C.c_double(0.0), C.c_double(0.0)
    assert lib.pn_fma_rate(0, 100, C.byref(d1), C.byref(d2), z) == PN_EINVAL
    assert lib.pn_fma_rate(9, 100, C.byref(d1), C.byref(d2), z) == PN_EINVAL
    assert lib.pn_fma_rate(8, 0, C.byref(d1), C.byref(d2), z) == PN_EINVAL
    assert lib.pn_fma_rate(8, 100, None, C.byref(d2), z) == PN_EINVAL
    big = 1 << 36                                    # PN_MAX_N
    assert call(big + 1, big + 1) == PN_EINVAL
    assert call(10, big + 1) == PN_EINVAL
    assert lib.pn_adjoint_workspace_bytes(big + 1, 16) == 0
    assert lib.pn_ks_workspace_bytes(big + 1) == 0
    assert lib.pn_rhs(-1, 0, fake, fake, fake, None, z) == PN_EINVAL
    assert lib.pn_observables(5, 4, fake, fake, z) == PN_EINVAL
    assert lib.pn_observables(0, 0, fake, fake, z) == PN_OK


def test_cost_order_argument_checks_without_a_device(lib):
    from paper_0908_3889_amd._lib import PN_EINVAL, PN_OK
    fake = C.c_void_p(0x1000)       # never dereferenced: validation fails first
    z = C.c_void_p(0)
    assert lib.pn_cost_order_workspace_bytes(0) == 0
    assert lib.pn_cost_order_workspace_bytes(-1) == 0
    assert lib.pn_cost_order_workspace_bytes(1 << 31) == 0
    call = lambda n, ld, ptr=fake, ws=1 << 20, wf=0.05, packed=z: lib.pn_cost_order(
        n, ld, ptr, ptr, ptr, ptr, wf, ptr, ptr, ws, packed, z)
    assert call(-1, 0) == PN_EINVAL
    assert call(10, 5) == PN_EINVAL
    assert call(1 << 31, 1 << 31) == PN_EINVAL
    assert call(10, 10, wf=float("nan")) == PN_EINVAL
    assert call(10, 10, ptr=z) == PN_EINVAL
    assert call(10, 10, packed=C.c_void_p(0x1008)) == PN_EINVAL   # misaligned records
    assert call(0, 0, ptr=z) == PN_OK


def test_replay_and_tape_size_checks_without_a_device(lib):
    from paper_0908_3889_amd._lib import PN_EINVAL, PN_OK, PN_PREC_FP32_SPLIT, PnOpts
    fake = C.c_void_p(0x1000)       # never dereferenced: validation fails first
    z = C.c_void_p(0)
    assert lib.pn_ckpt_bytes(1000, 1024, 16) == 1000 * lib.pn_tape_stride(1024, 16) * 8
    assert lib.pn_ckpt_bytes(0, 1024, 16) == 0
    assert lib.pn_ckpt_bytes(-1, 1024, 16) == 0
    assert lib.pn_ckpt_bytes(10, 0, 16) == 0
    assert lib.pn_ckpt_bytes(10, 1024, 0) == 0

    def call(n, ld, ptr=fake, wf=0.05, cap=1024, K=16, opt=None):
        return lib.pn_integrate_replay(n, ld, ptr, ptr, ptr, ptr, wf, opt, ptr, cap, K, None, ptr, ptr, z)
    assert call(-1, 0) == PN_EINVAL
    assert call(10, 5) == PN_EINVAL
    assert call(10, 10, ptr=z) == PN_EINVAL
    assert call(10, 10, wf=0.0) == PN_EINVAL
    assert call(10, 10, wf=float("nan")) == PN_EINVAL
    assert call(10, 10, cap=0) == PN_EINVAL
    assert call(10, 10, K=0) == PN_EINVAL
    o = PnOpts()
    o.precision = PN_PREC_FP32_SPLIT
    assert call(10, 10, opt=C.byref(o)) == PN_EINVAL
    o = PnOpts()
    o.h_fixed = 10.0
    assert call(10, 10, opt=C.byref(o)) == PN_EINVAL
    assert call(0, 0, ptr=z) == PN_OK


def test_fma_lanes_argument_checks_without_a_device(lib):
    from paper_0908_3889_amd._lib import PN_EINVAL
    d = C.c_double()
    assert lib.pn_fma_lanes(-1, 10, C.byref(d), C.byref(d), None) == PN_EINVAL
    assert lib.pn_fma_lanes(65, 10, C.byref(d), C.byref(d), None) == PN_EINVAL
    assert lib.pn_fma_lanes(8, 0, C.byref(d), C.byref(d), None) == PN_EINVAL
    assert lib.pn_fma_lanes(8, 10, None, C.byref(d), None) == PN_EINVAL

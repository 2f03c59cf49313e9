"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/pic.h declares, and rejects bad configurations on the host
(validation runs before any HIP call)."""
import ctypes as C
import os
import re

import pytest

from paper_1310_0930_amd import pic as P
from paper_1310_0930_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = _declared()
    assert "pic_push_deposit" in names and "pic_field_advance" in names and "pic_step" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps the same entry points under the same names
    for name in names:
        if name != "pic_strerror":
            assert hasattr(P, name), name


def test_strerror_names_every_status():
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert P.strerror(st) and "unknown" not in P.strerror(st)
    assert "unknown" in P.strerror(12345)


def _create(cfg):
    h = C.c_void_p()
    st = P.lib().pic_create(C.byref(cfg), C.byref(h))
    if st == P.PIC_OK:
        P.lib().pic_destroy(h)
    return st


def _good(**kw):
    w = I.WORKLOADS["w3d_128_quadratic"]
    args = dict(dims=3, n=w.n3, dx=w.dx3, dt=w.dt, order=2, real_bytes=4, bc=(0, 0, 0))
    args.update(kw)
    return P.make_config(**args)


@pytest.mark.parametrize("kw,expect", [
    (dict(dims=1), P.PIC_EINVAL),
    (dict(order=5), P.PIC_EINVAL),
    (dict(order=0), P.PIC_EINVAL),
    (dict(real_bytes=2), P.PIC_EINVAL),
    (dict(n=(1, 128, 128)), P.PIC_EINVAL),
    (dict(n=(128, 3, 128), bc=(0, 1, 0)), P.PIC_EINVAL),
    (dict(dx=(0.2, 0.0, 0.2)), P.PIC_EINVAL),
    (dict(dx=(0.2, float("nan"), 0.2)), P.PIC_EINVAL),
    (dict(dt=0.0), P.PIC_EINVAL),
    (dict(dt=0.2), P.PIC_ECOURANT),
    (dict(dt=1.0001 / (3 ** 0.5) * 0.2), P.PIC_ECOURANT),
    (dict(bc=(0, 2, 0)), P.PIC_EINVAL),
    (dict(sort_every=0), P.PIC_EINVAL),
    (dict(tile=(5, 8, 8)), P.PIC_EINVAL),
    (dict(dims=2, n=(64, 64, 4), dx=(0.2, 0.2, 1.0), dt=0.05), P.PIC_EINVAL),
])
def test_create_rejects_bad_config(kw, expect):
    assert _create(_good(**kw)) == expect


def test_create_accepts_courant_limit_or_reports_no_device():
    """A valid configuration passes validation; without a GPU the first HIP
    call fails with PIC_EHIP (never a crash)."""
    dt = 0.2 / 3 ** 0.5
    st = _create(_good(dt=dt))
    assert st in (P.PIC_OK, P.PIC_EHIP)


def test_null_arguments():
    lib = P.lib()
    assert lib.pic_create(None, None) == P.PIC_EINVAL
    h = C.c_void_p()
    assert lib.pic_create(None, C.byref(h)) == P.PIC_EINVAL and not h.value
    assert lib.pic_destroy(None) == P.PIC_OK
    b = C.c_size_t()
    assert lib.pic_workspace_bytes(None, 10, C.byref(b)) == P.PIC_EINVAL
    assert lib.pic_sort(None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_push_deposit(None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_field_advance(None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_step(None, None, None, 1, None, None) == P.PIC_EINVAL
    assert lib.pic_deposit_rho(None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_diagnostics(None, None, None, None, None, None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_read_flags(None, None, 0, None, None, None) == P.PIC_EINVAL
    assert lib.pic_read_push_counts(None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_push_deposit_add(None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_deposit_rho_add(None, None, None, None, None) == P.PIC_EINVAL
    assert lib.pic_step_species(0, None, None, None, None, 1, None) == P.PIC_EINVAL
    assert lib.pic_step_species(1, None, None, None, None, 1, None) == P.PIC_EINVAL
    assert lib.pic_diagnostics_species(0, None, None, None, None, None, None, None, None, None,
                                       None) == P.PIC_EINVAL


def test_product_path_does_not_touch_the_oracle():
    """The HIP binding never imports or loads the oracle: no CPU fallback."""
    pat = re.compile(r"(import\s+oracle|from\s+oracle|liboracle|oracle\.h|pic_oracle)")
    pkg = os.path.join(ROOT, "paper_1310_0930_amd")
    files = [os.path.join(pkg, f) for f in os.listdir(pkg) if f.endswith(".py")]
    files += [os.path.join(pkg, "csrc", f) for f in os.listdir(os.path.join(pkg, "csrc"))]
    for fn in files:
        assert not pat.search(open(fn).read()), fn

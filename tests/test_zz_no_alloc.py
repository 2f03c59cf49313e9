"""The no-allocation field advance (pic_field_advance_static) through the C
ABI: the same result as pic_field_advance with a workspace, on two calls in a
row (the second on a smaller grid), with open faces so that its static
scratch (the saved E planes next to open faces) is used."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fields(n, real, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    ncell = n[0] * n[1] * n[2]
    return [torch.randn((3, ncell), generator=g, device="cuda", dtype=real) for _ in range(3)]


@pytest.mark.parametrize("rb", [8, 4])
def test_static_field_advance_equals_workspace_form(rb):
    from paper_1310_0930_amd import pic as P
    real = torch.float64 if rb == 8 else torch.float32
    cases = [((40, 28, 24), (0.1, 0.2, 0.2), (P.PIC_BC_OPEN, P.PIC_BC_OPEN, P.PIC_BC_OPEN)),
             ((20, 12, 9), (0.2, 0.2, 0.25), (P.PIC_BC_PERIODIC, P.PIC_BC_OPEN, P.PIC_BC_OPEN))]
    for k, (n, dx, bc) in enumerate(cases):  # the second call has the smaller grid
        dt = 0.5 / np.sqrt(sum(1.0 / d ** 2 for d in dx))
        cfg = P.make_config(3, n, dx, dt, 2, real_bytes=rb, bc=bc)
        ctx = P.pic_create(cfg)
        try:
            E, B, J = _fields(n, real, 100 + k)
            E2, B2, J2 = E.clone(), B.clone(), J.clone()
            ws = torch.zeros(P.pic_workspace_bytes(ctx, 0), dtype=torch.uint8, device="cuda")
            for _ in range(3):
                P.pic_field_advance(ctx, P.fields_struct(E, B, J), ws.data_ptr())
                P.pic_field_advance_static(ctx, P.fields_struct(E2, B2, J2))
            torch.cuda.synchronize()
            assert torch.equal(E, E2) and torch.equal(B, B2), (rb, n)
            assert float(E.abs().max()) > 0
        finally:
            P.pic_destroy(ctx)


def test_static_field_advance_rejects_grids_beyond_its_scratch():
    """4 n_a n_b reals per open axis must fit 16 MiB: a 1024 x 1024 face in
    double precision needs 32 MiB, and the call returns PIC_ESCRATCH before
    any launch (no field arrays are touched)."""
    from paper_1310_0930_amd import pic as P
    cfg = P.make_config(3, (4, 1024, 1024), (0.2, 0.2, 0.2), 0.05, 1, real_bytes=8,
                        bc=(P.PIC_BC_OPEN, P.PIC_BC_PERIODIC, P.PIC_BC_PERIODIC))
    ctx = P.pic_create(cfg)
    try:
        dummy = torch.zeros(1, device="cuda", dtype=torch.float64)
        f = P.PicFields((C.c_void_p * 3)(*[dummy.data_ptr()] * 3), (C.c_void_p * 3)(*[dummy.data_ptr()] * 3),
                        (C.c_void_p * 3)(*[dummy.data_ptr()] * 3))
        st = P.lib().pic_field_advance_static(ctx, C.byref(f), None)
        assert st == P.PIC_ESCRATCH
    finally:
        P.pic_destroy(ctx)

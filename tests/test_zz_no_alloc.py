"""sg_step_noalloc through the C ABI against sg_step: two calls in a row on
plans that were never given a workspace, the second smaller than the first,
each bitwise equal to sg_step on the same fields; a size beyond the scratch
maximum is refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

from paper_1206_3215_amd import inputs
from tests.gpuutil import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
D = inputs.PAPER_DOMAIN


def raw_plan(b, n_x, n_y, prec, batch):
    """A plan made through the C ABI with no workspace handed to it."""
    h = C.c_void_p()
    b.check(b.lib.fft2d_plan(n_x, n_y, b.PST_R2C, prec, batch, None, C.byref(h)), "fft2d_plan")
    return h


@pytest.mark.parametrize("calls", [[(512, 512, 0, 2, 7), (128, 64, 1, 1, 5)]])
def test_noalloc_matches_sg_step_on_consecutive_calls(calls):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    for nx, ny, prec, batch, steps in calls:
        dt_ = torch.float64 if prec else torch.float32
        u0 = np.stack([inputs.sg_gaussian(nx, ny, D, seed=s)[0] for s in range(batch)])
        v0 = 0.2 * np.stack([inputs.noise(nx, ny, 50 + s) for s in range(batch)])
        ref_plan = b.Plan(nx, ny, b.PST_R2C, prec, batch)
        up, uc = torch.empty(batch, ny, nx, dtype=dt_, device="cuda"), torch.empty(batch, ny, nx, dtype=dt_,
                                                                                 device="cuda")
        ref_plan.sg_start(to_dev(u0, torch, dt_), to_dev(v0, torch, dt_), up, uc, D, 0.01)
        ap, ac = up.clone(), uc.clone()
        ref_plan.sg_step(up, uc, D, 0.01, steps)
        h = raw_plan(b, nx, ny, prec, batch)
        try:
            p = b.SgParams(b.domain(D), 0.01)
            b.check(b.lib.sg_step_noalloc(h, C.c_void_p(ap.data_ptr()), C.c_void_p(ac.data_ptr()), C.byref(p),
                                          steps), "sg_step_noalloc")
            st = C.c_int()
            b.check(b.lib.pst_sync_status(h, C.byref(st)), "pst_sync_status")
            assert st.value == b.PST_OK
        finally:
            b.lib.fft2d_destroy(h)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(ap), to_host(up)), (nx, ny, prec)
        assert np.array_equal(to_host(ac), to_host(uc)), (nx, ny, prec)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    h = raw_plan(b, 4096, 4096, b.PST_FP32, 1)            # 3 half spectra of 4096 x 2049 complex64: 201 MB
    try:
        u = torch.zeros(1, 4096, 4096, dtype=torch.float32, device="cuda")
        w = torch.zeros_like(u)
        p = b.SgParams(b.domain(D), 0.01)
        st = b.lib.sg_step_noalloc(h, C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()), C.byref(p), 3)
        assert st == b.PST_ERR_INVALID and "maximum" in b.lib.pst_last_error().decode()
        assert float(w.abs().max()) == 0.0                  # nothing ran
    finally:
        b.lib.fft2d_destroy(h)

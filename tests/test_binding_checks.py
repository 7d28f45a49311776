"""Host-side argument checks of the Python binding: dtype, size and kind
errors raise ValueError before any pointer crosses the C ABI (the kernels
trust the sizes they are given).  Runs without a GPU: the tensors are on the
CPU and the checks fire before the device check."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1206_3215_amd", "libpst.so")

torch = pytest.importorskip("torch")
if not os.path.exists(LIB):
    pytest.skip("libpst.so not built", allow_module_level=True)
from paper_1206_3215_amd import binding as b  # noqa: E402
from paper_1206_3215_amd import inputs  # noqa: E402

D = inputs.PAPER_DOMAIN


def fake_plan(nx, ny, kind, prec, batch):
    """A Plan object with its shape attributes but no device plan (the
    checks under test run before the handle is used)."""
    p = b.Plan.__new__(b.Plan)
    p.nx, p.ny, p.kind, p.prec, p.batch, p.handle = nx, ny, kind, prec, batch, None
    return p


def test_nls_step_rejects_real_and_wrong_size_fields():
    p = fake_plan(32, 16, b.PST_C2C, b.PST_FP32, 2)
    with pytest.raises(ValueError, match="dtype"):
        p.nls_step(torch.zeros(2, 16, 32, dtype=torch.float32), D, 1e-3, 1.0, 1)
    with pytest.raises(ValueError, match="dtype"):
        p.nls_step(torch.zeros(2, 16, 32, dtype=torch.complex128), D, 1e-3, 1.0, 1)
    with pytest.raises(ValueError, match="elements"):
        p.nls_step(torch.zeros(1, 16, 32, dtype=torch.complex64), D, 1e-3, 1.0, 1)
    with pytest.raises(ValueError, match="GPU"):                 # right dtype and size: the device check
        p.nls_step(torch.zeros(2, 16, 32, dtype=torch.complex64), D, 1e-3, 1.0, 1)


def test_solver_kind_must_match_plan():
    c2c = fake_plan(16, 16, b.PST_C2C, b.PST_FP64, 1)
    r2c = fake_plan(16, 16, b.PST_R2C, b.PST_FP64, 1)
    w = torch.zeros(1, 16, 16, dtype=torch.float64)
    with pytest.raises(ValueError, match="R2C"):
        c2c.ns_step(w, inputs.NS_DOMAIN, 1e-3, 1e-3, 1)
    with pytest.raises(ValueError, match="C2C"):
        r2c.nls_step(torch.zeros(1, 16, 16, dtype=torch.complex128), D, 1e-3, 1.0, 1)


def test_sg_and_ns_field_checks():
    p = fake_plan(16, 8, b.PST_R2C, b.PST_FP32, 3)
    good = torch.zeros(3, 8, 16, dtype=torch.float32)
    with pytest.raises(ValueError, match="u_curr"):
        p.sg_step(good, torch.zeros(2, 8, 16, dtype=torch.float32), D, 0.01, 1)
    with pytest.raises(ValueError, match="v0"):
        p.sg_start(good, torch.zeros(3, 8, 16, dtype=torch.float64), good, good, D, 0.01)
    with pytest.raises(ValueError, match="dev_iters"):
        p.ns_step(good, inputs.NS_DOMAIN, 1e-3, 1e-3, 4, dev_iters=torch.zeros(11, dtype=torch.int32))
    with pytest.raises(ValueError, match="dev_iters"):
        p.ns_step(good, inputs.NS_DOMAIN, 1e-3, 1e-3, 4, dev_iters=torch.zeros(12, dtype=torch.int64))
    with pytest.raises(ValueError, match="f1"):
        p.conserved_quantities("sg", good, None, d=D, dt=0.01)


def test_fft_exec_half_spectrum_sizes():
    p = fake_plan(16, 8, b.PST_R2C, b.PST_FP64, 1)
    real = torch.zeros(1, 8, 16, dtype=torch.float64)
    with pytest.raises(ValueError, match="out"):
        p.fft2d_exec(real, torch.zeros(1, 8, 8, dtype=torch.complex128), -1)   # needs 8 x 9
    with pytest.raises(ValueError, match="in"):
        p.fft2d_exec(torch.zeros(1, 8, 9, dtype=torch.complex64), real, 1)


def test_solve_batch_request_checks():
    nls = b.make_params("nls", D, 1e-3)
    sg = b.make_params("sg", D, 0.01)
    z = torch.zeros(16, 16, dtype=torch.complex64)
    r = torch.zeros(16, 16, dtype=torch.float32)
    cases = [
        ({"eq": "nls", "f0": r, "params": nls, "nsteps": 1}, "dtype"),
        ({"eq": "ns", "f0": z, "params": b.make_params("ns", D, 1e-3), "nsteps": 1}, "dtype"),
        ({"eq": "sg", "f0": r, "f1": None, "params": sg, "nsteps": 1}, "f1"),
        ({"eq": "sg", "f0": r, "f1": torch.zeros(16, 16, dtype=torch.float64), "params": sg, "nsteps": 1}, "f1"),
        ({"eq": "nls", "f0": torch.zeros(2, 16, 16, dtype=torch.complex64), "params": nls, "nsteps": 1}, "one"),
        ({"eq": "nls", "f0": z, "params": sg, "nsteps": 1}, "NlsParams"),
        ({"eq": "nls", "f0": z, "params": nls, "nsteps": 1,
          "dev_status": torch.zeros(1, dtype=torch.int64)}, "dev_status"),
        ({"eq": "heat", "f0": z, "params": nls, "nsteps": 1}, "unknown"),
    ]
    for req, msg in cases:
        with pytest.raises(ValueError, match=msg):
            b.solve_batch([req])

"""2D FFT through the C ABI vs the oracle's FP64 transform."""
import math

import numpy as np
import pytest

from oracle import spectral as sp
from tests.gpuutil import need_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 1), (8, 16, 2), (16, 8, 1), (32, 64, 3), (64, 64, 1), (128, 32, 2), (256, 512, 1),
          (1024, 1024, 1), (2048, 64, 1), (64, 4096, 1), (4096, 4096, 1), (8192, 16, 1), (16, 8192, 1)]
# relative error per log2(points): FP32 at its rounding level; FP64 at 5x the largest error
# measured (4.3e-17 per log2 at 4096^2, as large as numpy's own FP64 round trip), the
# O(eps log N) level of a double-precision FFT
TOL = {0: 1e-5, 1: 2e-16}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx,ny,batch", SHAPES)
def test_c2c_forward_inverse(nx, ny, batch, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    rng = np.random.default_rng(nx * 7 + ny + batch)
    x = rng.standard_normal((batch, ny, nx)) + 1j * rng.standard_normal((batch, ny, nx))
    plan = b.Plan(nx, ny, b.PST_C2C, prec, batch)
    xd = to_dev(x, torch, plan.complex_dtype)
    yd = torch.empty_like(xd)
    plan.fft2d_exec(xd, yd, -1)
    ref = np.stack([sp.fft2(x[i]) for i in range(batch)])
    assert rel_err(to_host(yd), ref) < TOL[prec] * math.log2(nx * ny)
    plan.fft2d_exec(yd, yd, +1)                     # in place inverse
    assert rel_err(to_host(yd), x) < TOL[prec] * math.log2(nx * ny)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx,ny,batch", [(4, 4, 1), (8, 8, 3), (16, 64, 1), (64, 32, 2), (256, 256, 1),
                                         (1024, 512, 1), (2048, 2048, 1), (4096, 128, 1)])
def test_r2c_c2r(nx, ny, batch, prec):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    rng = np.random.default_rng(nx + 3 * ny + batch)
    x = rng.standard_normal((batch, ny, nx))
    plan = b.Plan(nx, ny, b.PST_R2C, prec, batch)
    xd = to_dev(x, torch, plan.real_dtype)
    yd = torch.empty((batch, ny, nx // 2 + 1), dtype=plan.complex_dtype, device="cuda")
    plan.fft2d_exec(xd, yd, -1)
    ref = np.stack([sp.rfft2(x[i]) for i in range(batch)])
    assert rel_err(to_host(yd), ref) < TOL[prec] * math.log2(nx * ny)
    zd = torch.empty_like(xd)
    plan.fft2d_exec(yd, zd, +1)
    assert rel_err(to_host(zd), x) < TOL[prec] * math.log2(nx * ny)
    assert to_host(yd).shape == (batch, ny, nx // 2 + 1)


def test_c2r_ignores_imaginary_dc_and_nyquist():
    # numpy's inverse real transform drops Im of the self-conjugate modes.
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    nx = ny = 16
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1, ny, nx // 2 + 1)) + 1j * rng.standard_normal((1, ny, nx // 2 + 1))
    plan = b.Plan(nx, ny, b.PST_R2C, 1, 1)
    out = torch.empty((1, ny, nx), dtype=torch.float64, device="cuda")
    plan.fft2d_exec(to_dev(X, torch, torch.complex128), out, +1)
    assert rel_err(to_host(out)[0], sp.irfft2(X[0], (ny, nx))) < 1e-13


@pytest.mark.parametrize("eq,kind,n", [("nls", 0, 4096), ("nls", 0, 256), ("sg", 1, 2048), ("ns", 1, 1024)])
def test_autotune_picks_a_compiled_variant(eq, kind, n):
    need_gpu()
    from paper_1206_3215_amd import binding as b
    plan = b.Plan(n, n, kind, b.PST_FP32, 1)
    v = plan.autotune(eq)
    assert 0 <= v < len(plan.column_variants())


@pytest.mark.parametrize("prec,n,batch", [(0, 4096, 1), (0, 8192, 1), (1, 4096, 1), (1, 8192, 1), (0, 1024, 3),
                                          (0, 64, 2)])
def test_column_variants_agree(prec, n, batch):
    # every variant runs the same radix schedule with the same twiddles;
    # variants with the same values per thread give bit-identical results,
    # others may differ by where the compiler fuses multiply-adds (FP32
    # rounding level after three steps)
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    from paper_1206_3215_amd import inputs
    d = inputs.PAPER_DOMAIN
    psi0 = np.stack([inputs.nls_gaussian(n, n, d, seed=s) for s in range(batch)])
    cdt = torch.complex64 if prec == b.PST_FP32 else torch.complex128
    plan = b.Plan(n, n, b.PST_C2C, prec, batch)
    variants = plan.column_variants()
    if prec == b.PST_FP32 and n >= 4096:
        assert len(variants) == 5 and variants[1][1] == 32 and variants[1][2] == 1
    if prec == b.PST_FP64 and n >= 4096:
        assert len(variants) == 6 and variants[2][1] == 32 and variants[5][3] == 8
    ref = None
    for v, (_, vpt, _, radix) in enumerate(variants):
        plan.set_column_variant(v)
        a = to_dev(psi0, torch, cdt)
        plan.nls_step(a, d, 1e-3, 1.0, 3)
        f = to_dev(psi0, torch, cdt)
        plan.fft2d_exec(f, f, -1)
        got = (to_host(a), to_host(f))
        if ref is None:
            ref = got
            continue
        e = (rel_err(got[0], ref[0]), rel_err(got[1], ref[1]))
        print(f"variant {v} {variants[v]}: rel diff nls {e[0]:.2e} fft {e[1]:.2e}")
        if vpt == variants[0][1] and radix == variants[0][3]:
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), f"variant {v}"
        else:
            bar = 2e-6 if prec == b.PST_FP32 else 1e-13
            assert e[0] < bar and e[1] < bar, f"variant {v}"
    with pytest.raises(b.PstError):
        plan.set_column_variant(len(variants))

"""NLS split-step through the C ABI vs the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import nls as onls
from paper_1206_3215_amd import inputs
from tests.gpuutil import need_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

# Stated tolerances: max relative error vs the FP64 oracle.
TOL = {0: 1e-4, 1: 1e-11}


def run_gpu(psi0, d, dt, g, nsteps, prec, chunk=None, diag=False, variant=0, row_variant=0):
    torch = need_gpu()
    from paper_1206_3215_amd import binding as b
    batch = psi0.shape[0] if psi0.ndim == 3 else 1
    ny, nx = psi0.shape[-2:]
    plan = b.Plan(nx, ny, b.PST_C2C, prec, batch)
    plan.set_column_variant(variant)
    plan.set_row_variant(row_variant)
    psi = to_dev(psi0.reshape(batch, ny, nx), torch, plan.complex_dtype)
    diags = []
    chunk = chunk or nsteps
    done = 0
    if diag:
        diags.append(plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g))
    while done < nsteps:
        k = min(chunk, nsteps - done)
        plan.nls_step(psi, d, dt, g, k)
        done += k
        if diag:
            diags.append(plan.conserved_quantities("nls", psi, d=d, dt=dt, g=g))
    torch.cuda.synchronize()
    return to_host(psi).reshape(psi0.shape), diags


@pytest.mark.parametrize("prec", [1, 0])
def test_small_workload_matches_oracle(prec):
    # 64^2 on [-8pi,8pi)^2, seeded noise, dt 0.0025, 200 steps, diagnostics every 20.
    d = inputs.NLS_SMALL_DOMAIN
    psi0 = inputs.nls_gaussian(64, 64, d, seed=0)
    ref, rdiag = onls.run(psi0, d.lx, d.ly, 0.0025, 1.0, 200, diag_every=20)
    got, gdiag = run_gpu(psi0, d, 0.0025, 1.0, 200, prec, chunk=20, diag=True)
    assert rel_err(got, ref) < TOL[prec]
    gm = np.array([x[0, 0] for x in gdiag])
    ge = np.array([x[0, 1] for x in gdiag])
    rm = np.array([x[1] for x in rdiag])
    re_ = np.array([x[2] for x in rdiag])
    if prec == 1:
        assert np.max(np.abs(gm / rm - 1)) < 1e-12
        assert np.max(np.abs(ge / re_ - 1)) < 1e-12
        assert np.max(np.abs(gm / gm[0] - 1)) < 1e-12   # mass to rounding (paper's Results)
    else:
        # FP32 reading: each step applies unit-modulus factors rounded once,
        # so the mass drifts by at most one single-precision rounding unit per
        # step; the energy follows the field (FP32 tolerance class)
        steps = 20 * np.arange(len(gm))
        assert np.all(np.abs(gm / gm[0] - 1) <= 2.0 ** -23 * np.maximum(steps, 1))
        assert np.max(np.abs(ge / re_ - 1)) < TOL[0]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("nx,ny,batch", [(16, 8, 1), (32, 32, 3), (128, 64, 2), (4, 4, 1)])
def test_ragged_shapes_and_batches(nx, ny, batch, prec):
    d = inputs.Domain(7.0, 5.0, -3.5, -2.5)
    psi0 = np.stack([inputs.nls_gaussian(nx, ny, d, seed=s) for s in range(batch)]) * 1.7
    got, _ = run_gpu(psi0, d, 0.01, -1.0, 7, prec)
    for i in range(batch):
        ref, _ = onls.run(psi0[i], d.lx, d.ly, 0.01, -1.0, 7)
        assert rel_err(got[i], ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_strong_nonlinear_phase_against_oracle(prec):
    # per-step nonlinear phase dt g |psi|^2 up to ~0.4, beyond the small-angle
    # series: the rotation takes the half angle's sine and cosine
    d = inputs.Domain(12.0, 12.0, -6.0, -6.0)
    psi0 = inputs.nls_gaussian(64, 64, d, seed=3) * 6.0
    assert 0.05 * np.max(np.abs(psi0)) ** 2 > 0.3
    got, _ = run_gpu(psi0, d, 0.05, 1.0, 20, prec)
    ref, _ = onls.run(psi0, d.lx, d.ly, 0.05, 1.0, 20)
    assert rel_err(got, ref) < TOL[prec]


def test_zero_and_one_step():
    d = inputs.PAPER_DOMAIN
    psi0 = inputs.nls_gaussian(64, 64, d, seed=1)
    got0, _ = run_gpu(psi0, d, 1e-3, 1.0, 0, 1)
    assert np.array_equal(got0, psi0)
    got1, _ = run_gpu(psi0, d, 1e-3, 1.0, 1, 1)
    ref1, _ = onls.run(psi0, d.lx, d.ly, 1e-3, 1.0, 1)
    assert rel_err(got1, ref1) < 1e-12


@pytest.mark.parametrize("prec", [1, 0])
def test_plane_wave_closed_form_full_size(prec):
    # Property at the headline size 4096^2 (any size): a plane wave is
    # reproduced exactly by the split step for any dt.
    n, L, A, dt, steps = 4096, 10 * math.pi, 0.3, 1e-3, 100
    X, Y = inputs.grid(n, n, inputs.Domain(L, L, 0, 0))
    k = 2 * math.pi * np.array([5, -3]) / L
    psi0 = A * np.exp(1j * (k[0] * X + k[1] * Y))
    got, _ = run_gpu(psi0, inputs.Domain(L, L, 0, 0), dt, 1.0, steps, prec)
    exact = psi0 * np.exp(-1j * (k @ k + A * A) * dt * steps)
    assert rel_err(got, exact) < TOL[prec]


@pytest.fixture(scope="module")
def oracle_4096_10():
    d = inputs.PAPER_DOMAIN
    psi0 = inputs.nls_gaussian(4096, 4096, d, seed=0)
    ref, _ = onls.run(psi0, d.lx, d.ly, 1e-3, 1.0, 10)
    return psi0, ref


@pytest.mark.parametrize("prec,variant", [(0, v) for v in range(5)] + [(1, v) for v in range(6)])
def test_headline_size_against_oracle_short(prec, variant, oracle_4096_10):
    # 4096^2 on [-5pi,5pi)^2, 10 steps, in every column variant (the
    # benchmark runs the one the autotuner picks).
    d = inputs.PAPER_DOMAIN
    psi0, ref = oracle_4096_10
    got, _ = run_gpu(psi0, d, 1e-3, 1.0, 10, prec, variant=variant)
    assert rel_err(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec,row", [(p, r) for p in (0, 1) for r in range(4)])
def test_headline_size_row_variants(prec, row, oracle_4096_10):
    # every row variant of the in-place row pass at 4096 (split exchange,
    # radix 8), with the radix-8 column variant in FP64
    d = inputs.PAPER_DOMAIN
    psi0, ref = oracle_4096_10
    got, _ = run_gpu(psi0, d, 1e-3, 1.0, 10, prec, variant=5 if prec else 0, row_variant=row)
    assert rel_err(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("n", [64, 1024, 2048])
def test_pair_row_variants_bitwise_equal(prec, n):
    # the row-pair pass in each pairs-per-block variant: same arithmetic, so
    # bit-identical to the default, and within tolerance of the oracle
    from paper_1206_3215_amd import binding as b
    d = inputs.PAPER_DOMAIN
    psi0 = np.stack([inputs.nls_gaussian(n, n // 2, d, seed=s) for s in range(3)])
    base, _ = run_gpu(psi0, d, 1e-3, 1.0, 4, prec)
    for r in range(1, len(b.row_variants(prec, n))):
        got, _ = run_gpu(psi0, d, 1e-3, 1.0, 4, prec, row_variant=r)
        assert np.array_equal(got, base), r
    ref, _ = onls.run(psi0[1], d.lx, d.ly, 1e-3, 1.0, 4)
    assert rel_err(base[1], ref) < TOL[prec]


@pytest.mark.parametrize("prec,variant,row", [(0, 1, 0), (0, 4, 2), (1, 0, 0), (1, 2, 1), (1, 4, 3), (1, 5, 2)])
def test_plane_wave_closed_form_8192(prec, variant, row):
    # the largest compiled line length (32 values per thread and the split
    # exchange in rows and in FP32 columns; FP64 columns in variants 0 and 2;
    # radix 8 and the wide split tiles)
    n, L, A, dt, steps = 8192, 10 * math.pi, 0.3, 1e-3, 20
    X, Y = inputs.grid(n, n, inputs.Domain(L, L, 0, 0))
    k = 2 * math.pi * np.array([-7, 4]) / L
    psi0 = A * np.exp(1j * (k[0] * X + k[1] * Y))
    got, _ = run_gpu(psi0, inputs.Domain(L, L, 0, 0), dt, 1.0, steps, prec, variant=variant, row_variant=row)
    exact = psi0 * np.exp(-1j * (k @ k + A * A) * dt * steps)
    assert rel_err(got, exact) < TOL[prec]


@pytest.fixture(scope="module")
def oracle_1024_1000():
    d = inputs.PAPER_DOMAIN
    psi0 = inputs.nls_gaussian(1024, 1024, d, seed=0)
    ref, diags = onls.run(psi0, d.lx, d.ly, 1e-3, 1.0, 1000, diag_every=1000)
    return psi0, ref, diags


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [0, 1])
def test_1024_thousand_steps_against_oracle(prec, oracle_1024_1000):
    # Headline configuration at its 1024^2 grid: [-5pi,5pi)^2, dt 1e-3, 1000 steps.
    d = inputs.PAPER_DOMAIN
    psi0, ref, rdiag = oracle_1024_1000
    got, gdiag = run_gpu(psi0, d, 1e-3, 1.0, 1000, prec, diag=True)
    err = rel_err(got, ref)
    print(f"prec={prec} rel_err={err:.3e} mass drift={gdiag[-1][0,0]/gdiag[0][0,0]-1:.3e}")
    assert err < TOL[prec]
    assert abs(gdiag[-1][0, 0] / rdiag[-1][1] - 1) < (1e-12 if prec else 1e-4)


@pytest.mark.parametrize("n,variant", [(4096, 1), (2048, 1)])
def test_batched_fields_equal_single_field_runs(n, variant):
    # several fields per plan at the long-line sizes (one line per block in
    # the in-place row pass, field index per block): each field bitwise equal
    # to its own single-field run
    torch = need_gpu()
    d = inputs.PAPER_DOMAIN
    psi0 = np.stack([inputs.nls_gaussian(n, n, d, seed=s) for s in (0, 5)])
    got, _ = run_gpu(psi0, d, 1e-3, 1.0, 3, 0, variant=variant)
    for i in range(2):
        one, _ = run_gpu(psi0[i:i + 1], d, 1e-3, 1.0, 3, 0, variant=variant)
        assert np.array_equal(got[i], one[0])

"""GPU parity of the expanded encoding operators (FP32 form) against the FP64
oracle: whole-output comparisons at small sizes that span several tiles and
ragged tails, the adjoint identity, and
bitwise determinism.  Tolerance: relative l2 error <= 1e-5 (FP32 form)."""
import numpy as np
import pytest

import synth
from oracle import encoding
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _ee():
    import paper_2211_07532_amd as ee
    return ee


def test_sh_basis_matches_oracle():
    import torch
    ee = _ee()
    for n, ny, fov, z0, nb in ((32, 32, 0.222, 0.0, 9), (148, 148, 0.222, 0.003, 16), (13, 7, 0.1, -0.006, 16)):
        b = ee.sh_basis(n, ny, fov, fov * ny / n, z0, nb, device="cuda").cpu().numpy()
        ref = encoding.sh_basis(n, fov, z0, nb, ny=ny, fov_y=fov * ny / n)
        assert np.max(np.abs(b - ref)) <= 1e-15 * np.max(np.abs(ref)) + 1e-300


@pytest.mark.parametrize("sh", [False, True], ids=["maps", "sh"])
@pytest.mark.parametrize("name", ["tiny", "ragged", "onecoil-nofield", "40coils"])
def test_forward_adjoint_whole_output(name, sh):
    import torch
    ee = _ee()
    if name == "tiny":
        w = synth.TINY
        case = Case(w, sh=sh)
        batch = 2
    elif name == "ragged":
        w = synth.Workload("ragged", 13, 0.1, 5, 333, 3e-6, 2.0, 16, 120.0, 20.0, 5, "haar", 1, 21)
        case = Case(w, z0=0.004, sh=sh)
        batch = 3
    elif name == "onecoil-nofield":
        w = synth.Workload("c1", 24, 0.2, 1, 600, 2e-6, 2.0, 3, 0.0, 20.0, 5, "haar", 1, 22)
        case = Case(w, with_dw0=False, nbasis=0, sh=sh)
        batch = 1
    else:
        w = synth.Workload("c40", 20, 0.2, 40, 700, 2e-6, 2.0, 9, 80.0, 20.0, 5, "haar", 1, 23)
        case = Case(w, sh=sh)
        batch = 1
    print(f"[case] {name} n={w.n} T={w.nsamples} C={case.smaps.shape[0]} L={case.coef.shape[1]} B={batch}",
          flush=True)
    x = c64(synth.random_complex((batch, w.npix), 31))
    x[0] = case.x_noisy
    y_ref = encoding.forward(x, *case.oracle_args())
    y = ee.forward(case.to_dev(x), case.op).cpu().numpy()
    assert y.shape == y_ref.shape
    assert rel(y, y_ref) <= TOL
    g = c64(synth.random_complex(y_ref.shape, 32))
    x_ref = encoding.adjoint(g, *case.oracle_args())
    xa = ee.adjoint(case.to_dev(g), case.op).cpu().numpy()
    assert rel(xa, x_ref) <= TOL
    # adjoint identity on the GPU results
    for b in range(batch):
        lhs = np.vdot(g[b], y[b])
        rhs = np.vdot(xa[b], x[b])
        assert abs(lhs - rhs) / (np.linalg.norm(y[b]) * np.linalg.norm(g[b])) <= 1e-6
    torch.cuda.synchronize()


def test_bitwise_determinism():
    ee = _ee()
    case = Case(synth.TINY)
    x = case.to_dev(case.x_noisy)
    y1 = ee.forward(x, case.op).cpu().numpy()
    y2 = ee.forward(x, case.op).cpu().numpy()
    assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))
    g = case.to_dev(y1)
    a1 = ee.adjoint(g, case.op).cpu().numpy()
    a2 = ee.adjoint(g, case.op).cpu().numpy()
    assert np.array_equal(a1.view(np.uint32), a2.view(np.uint32))


def test_invalid_arguments_raise():
    import torch
    ee = _ee()
    case = Case(synth.TINY)
    bad = torch.zeros(5, dtype=torch.complex64, device="cuda")
    with pytest.raises((ValueError, RuntimeError)):
        ee.forward(bad, case.op)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("shape", [(1, 1, 1, 1, 1, 1), (1, 7, 17, 3, 4, 2), (5, 3, 300, 2, 0, 1),
                                   (17, 2, 5, 17, 2, 1)],
                         ids=["1x1-T1-C1", "1x7-T17-C3-B2", "5x3-nofield", "17x2-T5-C17"])
def test_degenerate_shapes(shape, prec):
    """Degenerate geometries against the oracle: a single pixel and sample,
    a one-column image, no field terms, more coils than samples (basis given
    as maps, so any nx x ny)."""
    import torch
    ee = _ee()
    nx, ny, T, C, L, B = shape
    R = nx * ny
    rng = np.random.default_rng(7 + nx + 10 * ny + T)
    smaps = c64(synth.random_complex((C, R), 41 + C))
    coef = rng.normal(0.0, 2.0, (T, L))
    basis = rng.uniform(-1.0, 1.0, (L, R))
    time = np.arange(T, dtype=np.float64) * 2e-6
    dw0 = rng.uniform(-600.0, 600.0, R)
    x = c64(synth.random_complex((B, R), 43))
    dev = torch.device("cuda")
    op = ee.Operator(nx, ny, torch.from_numpy(smaps.astype(np.complex64)).to(dev), torch.from_numpy(coef).to(dev),
                     torch.from_numpy(time).to(dev), torch.from_numpy(basis).to(dev), torch.from_numpy(dw0).to(dev))
    print(f"[case] degenerate {nx}x{ny} T={T} C={C} L={L} B={B} {prec}", flush=True)
    bar = TOL if prec == "fp32" else 1e-3
    y_ref = encoding.forward(x, smaps, coef, time, basis, dw0)
    y = ee.forward(torch.from_numpy(x.astype(np.complex64)).to(dev), op, precision=prec).cpu().numpy()
    assert y.shape == y_ref.shape and rel(y, y_ref) <= bar
    g = c64(synth.random_complex(y_ref.shape, 44))
    xa = ee.adjoint(torch.from_numpy(g.astype(np.complex64)).to(dev), op, precision=prec).cpu().numpy()
    x_ref = encoding.adjoint(g, smaps, coef, time, basis, dw0)
    assert xa.shape == x_ref.shape and rel(xa, x_ref) <= bar


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("shape", [(1, 1, 1, 1, 1), (3, 17, 40, 2, 1), (17, 3, 33, 5, 2), (33, 20, 100, 4, 1)],
                         ids=["1x1-T1", "3x17", "17x3-B2", "33x20"])
def test_degenerate_shapes_sh(shape, prec):
    """The solid-harmonic kind (the library evaluates the basis from the grid
    geometry and, in the split forms, runs the polynomial kernels) on
    degenerate and non-square grids with rectangular fields of view, 16 terms
    and dB0, against the oracle's basis on the same geometry."""
    import torch
    ee = _ee()
    nx, ny, T, C, B = shape
    fx, fy, z0, L = 0.1, 0.07, 0.003, 16
    R = nx * ny
    rng = np.random.default_rng(100 + nx + 10 * ny + T)
    basis = encoding.sh_basis(nx, fx, z0, L, ny=ny, fov_y=fy)
    scale = 3.0 / np.maximum(np.abs(basis).max(axis=1), 1e-12)   # a few radians per term at most
    coef = rng.normal(0.0, 1.0, (T, L)) * scale[None, :]
    time = np.arange(T, dtype=np.float64) * 2e-6
    dw0 = rng.uniform(-600.0, 600.0, R)
    smaps = c64(synth.random_complex((C, R), 51 + C))
    x = c64(synth.random_complex((B, R), 52))
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    op = ee.Operator(nx, ny, t(smaps.astype(np.complex64)), t(coef), t(time), None, t(dw0), sh_grid=(fx, fy, z0))
    print(f"[case] degenerate sh {nx}x{ny} T={T} C={C} B={B} {prec}", flush=True)
    bar = TOL if prec == "fp32" else 1e-3
    y_ref = encoding.forward(x, smaps, coef, time, basis, dw0)
    y = ee.forward(t(x.astype(np.complex64)), op, precision=prec).cpu().numpy()
    assert y.shape == y_ref.shape and rel(y, y_ref) <= bar
    g = c64(synth.random_complex(y_ref.shape, 53))
    xa = ee.adjoint(t(g.astype(np.complex64)), op, precision=prec).cpu().numpy()
    x_ref = encoding.adjoint(g, smaps, coef, time, basis, dw0)
    assert xa.shape == x_ref.shape and rel(xa, x_ref) <= bar

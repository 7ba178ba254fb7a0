"""GPU parity of receiver pre-whitening and coil compression against the FP64
oracle.  Eigenvectors are unique only up to a phase per column, so the
compression is compared through what is unique: the eigenvalues, the
projector V_k V_k^H onto the kept subspace, the data and maps mapped back
through V_k^H, and the compressed data against the forward model with the
virtual maps.  Bars: 1e-6 relative (whitening), 1e-6 (eigenvalues), 1e-5
(subspace quantities; FP32 inputs and outputs)."""
import numpy as np
import pytest

import synth
from oracle import coils, encoding
from tests.gpu_common import Case, c64, rel

pytestmark = pytest.mark.gpu


def _dev(a, dtype=np.complex64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


def _psi(C, seed):
    rng = np.random.default_rng(seed)
    m = (rng.standard_normal((C, C)) + 1j * rng.standard_normal((C, C))) / np.sqrt(2) + 2.0 * np.eye(C)
    return m @ m.conj().T


@pytest.mark.parametrize("C", [1, 5, 8, 32])
def test_prewhiten_matches_oracle(C):
    import paper_2211_07532_amd as ee
    rng = np.random.default_rng(40 + C)
    y = c64((rng.standard_normal((777, C)) + 1j * rng.standard_normal((777, C))))
    s = c64((rng.standard_normal((C, 300)) + 1j * rng.standard_normal((C, 300))))
    psi = _psi(C, 50 + C)
    yw_ref, sw_ref = coils.prewhiten(psi, y, s)
    yd, sd = _dev(y), _dev(s)
    ee.prewhiten(_dev(psi, np.complex128), yd, sd)
    e1, e2 = rel(yd.cpu().numpy(), yw_ref), rel(sd.cpu().numpy(), sw_ref)
    print(f"[case] prewhiten C={C}: data {e1:.2e} maps {e2:.2e}", flush=True)
    assert e1 <= 1e-6 and e2 <= 1e-6


def _compare_compression(y, s, nv, bar=1e-5):
    import paper_2211_07532_amd as ee
    yv_ref, sv_ref, w_ref, vk_ref = coils.compress(y, s, nv)
    yv, sv, w, v = ee.coil_compress(_dev(y), nv, _dev(s))
    w = w.cpu().numpy()
    v = v.cpu().numpy()
    vk = v[:, :nv]
    ew = np.max(np.abs(w - w_ref)) / w_ref[0]
    eo = np.max(np.abs(v.conj().T @ v - np.eye(v.shape[0])))
    # energy kept: sum of the kept eigenvalues, valid for any choice inside a
    # degenerate cluster
    ee_ = abs(np.sum(np.abs(yv.cpu().numpy()) ** 2) - np.sum(w_ref[:nv])) / np.sum(w_ref)
    gap = (w_ref[nv - 1] - w_ref[nv]) / w_ref[0] if nv < len(w_ref) else 1.0
    print(f"  eigenvalues {ew:.2e} orthonormality {eo:.2e} kept energy {ee_:.2e} gap {gap:.1e}", flush=True)
    assert ew <= 1e-6 and eo <= 1e-12 and ee_ <= bar
    if gap > 1e-6:
        # a separated subspace is unique: compare its projector and the data and
        # maps mapped back through it
        ep = rel(vk @ vk.conj().T, vk_ref @ vk_ref.conj().T)
        ey = rel(yv.cpu().numpy() @ vk.conj().T, yv_ref @ vk_ref.conj().T)
        es = rel(vk.conj() @ sv.cpu().numpy(), vk_ref.conj() @ sv_ref)
        print(f"  projector {ep:.2e} data {ey:.2e} maps {es:.2e}", flush=True)
        assert ep <= bar and ey <= bar and es <= bar
    return yv, sv


@pytest.mark.parametrize("C,nv", [(3, 2), (8, 4), (17, 9), (32, 16)])
def test_compress_random_data_matches_oracle(C, nv):
    rng = np.random.default_rng(60 + C)
    # distinct, well separated singular values
    u = np.linalg.qr(rng.standard_normal((900, C)) + 1j * rng.standard_normal((900, C)))[0]
    q = np.linalg.qr(rng.standard_normal((C, C)) + 1j * rng.standard_normal((C, C)))[0]
    y = c64(u @ np.diag(np.geomspace(10.0, 0.1, C)) @ q.conj().T)
    s = c64(rng.standard_normal((C, 200)) + 1j * rng.standard_normal((C, 200)))
    print(f"[case] compress random C={C} nv={nv}", flush=True)
    _compare_compression(y, s, nv)


@pytest.mark.parametrize("nv", [8, 16, 20])
def test_compress_full_size_data_follows_virtual_model(nv):
    """1.5 mm workload: 32 physical coils compressed to nv virtual coils; the
    compressed data equal the GPU forward model with the virtual maps."""
    import paper_2211_07532_amd as ee
    from oracle import solve
    w = synth.MM15
    case = Case(w, sh=True)
    y = c64(solve.Operator(case.smaps, case.coef, case.time, case.basis_np, case.dw0, w.n).A(case.x_noisy))
    print(f"[case] compress 1.5 mm 32 -> {nv}", flush=True)
    yv, sv = _compare_compression(y, case.smaps, nv)
    op_v = ee.Operator(w.n, w.n, sv, case.t_coef, case.t_time, None, case.t_dw0, sh_grid=(w.fov, w.fov, case.z0))
    y2 = ee.forward(case.to_dev(case.x_noisy), op_v).cpu().numpy()
    assert rel(yv.cpu().numpy(), y2) <= 1e-5

"""Pins of the oracle's wavelet transform and soft-threshold: the defining
identities of the Daubechies filter, perfect reconstruction, Parseval,
the Haar closed form, vanishing moments on polynomial images, and the
proximal optimality condition of the soft-threshold."""
import math

import numpy as np
import pytest

import synth
from oracle import wavelet


def test_db4_filter_identities():
    h = wavelet.daubechies_filter(4)
    assert len(h) == 8
    assert h.sum() == pytest.approx(math.sqrt(2), abs=1e-14)
    assert np.sum(h * h) == pytest.approx(1.0, abs=1e-14)
    for m in (1, 2, 3):
        assert abs(np.sum(h[:-2 * m] * h[2 * m:])) < 1e-14
    k = np.arange(8)
    for p in range(4):
        assert abs(np.sum((-1.0) ** k * k ** p * h)) < 1e-11 * max(1, 8 ** p)
    # extremal phase: zeros of H(z) = sum h[n] z^-n other than z=-1 lie inside |z|<1
    zeros = np.roots(h)
    inner = zeros[np.abs(zeros + 1) > 1e-2]
    assert len(inner) == 3 and np.all(np.abs(inner) < 1)
    # the 4-fold zero at z = -1 (p vanishing moments)
    assert np.sum(np.abs(zeros + 1) < 1e-2) == 4


def test_haar_filter_and_closed_form():
    h = wavelet.haar_filter()
    np.testing.assert_allclose(h, [1 / math.sqrt(2)] * 2)
    x = np.array([[1.0, 2.0], [3.0, 4.0]])
    w = wavelet.dwt2(x, 1, "haar")
    # LL = sum/2, HL = row difference, LH = column difference, HH = diagonal
    np.testing.assert_allclose(w.real, [[5.0, -1.0], [-2.0, 0.0]], atol=1e-15)


@pytest.mark.parametrize("name,levels,shape", [("haar", 2, (32, 32)), ("db4", 3, (152, 152)),
                                               ("db4", 4, (208, 208)), ("db4", 2, (16, 24)),
                                               ("haar", 3, (8, 8))])
def test_perfect_reconstruction_and_parseval(name, levels, shape):
    x = synth.random_complex(shape, 3)
    w = wavelet.dwt2(x, levels, name)
    assert np.linalg.norm(w) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    xr = wavelet.idwt2(w, levels, name)
    assert np.max(np.abs(xr - x)) < 1e-13 * np.max(np.abs(x))
    # inverse is the adjoint: <W x, v> = <x, W^H v>
    v = synth.random_complex(shape, 4)
    assert abs(np.vdot(v, w) - np.vdot(wavelet.idwt2(v, levels, name), x)) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(v)


def test_analysis_matrix_orthogonal():
    for name in ("haar", "db4"):
        for n in (8, 12, 38):
            m = wavelet.analysis_matrix(n, wavelet.filters(name))
            np.testing.assert_allclose(m @ m.T, np.eye(n), atol=1e-14)


def test_db4_details_vanish_on_cubic_image():
    n = 64
    u = np.arange(n, dtype=float)
    yy, xx = np.meshgrid(u, u, indexing="ij")
    img = 0.3 + 0.2 * xx - 0.01 * yy + 1e-3 * xx * yy + 2e-4 * xx ** 3 - 1e-4 * yy ** 2 * xx
    w = wavelet.dwt2(img, 1, "db4")
    # away from the periodic wrap (last 3 outputs of each half depend on it)
    hl = w[:n // 2, n // 2:][: n // 2 - 4, : n // 2 - 4]
    lh = w[n // 2:, :n // 2][: n // 2 - 4, : n // 2 - 4]
    hh = w[n // 2:, n // 2:][: n // 2 - 4, : n // 2 - 4]
    scale = np.max(np.abs(img))
    assert np.max(np.abs(hl)) < 1e-10 * scale
    assert np.max(np.abs(lh)) < 1e-10 * scale
    assert np.max(np.abs(hh)) < 1e-10 * scale


def test_soft_threshold_is_the_prox():
    rng = np.random.default_rng(0)
    w = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    tau = 0.9
    levels = 2
    u = wavelet.soft_threshold(w, tau, levels)
    det = wavelet.detail_mask(16, 16, levels)
    # LL passes through
    np.testing.assert_array_equal(u[~det], w[~det])
    # optimality: 0 in (u - w) + tau * d|u|  on every detail coefficient
    for a, b in zip(u[det], w[det]):
        if a != 0:
            assert abs((a - b) + tau * a / abs(a)) < 1e-14
        else:
            assert abs(b) <= tau
    # ties and zeros map to zero
    z = np.zeros((4, 4), complex)
    z[2, 2] = tau
    z[3, 3] = 0
    assert wavelet.soft_threshold(z, tau, 1)[2, 2] == 0
    # prox minimises 1/2|u - w|^2 + tau|u| : compare against perturbations
    for a, b in zip(u[det][:20], w[det][:20]):
        f0 = 0.5 * abs(a - b) ** 2 + tau * abs(a)
        for d in (1e-3, -1e-3, 1e-3j, -1e-3j):
            assert f0 <= 0.5 * abs(a + d - b) ** 2 + tau * abs(a + d) + 1e-15


def test_detail_mask_counts():
    m = wavelet.detail_mask(152, 152, 3)
    assert (~m).sum() == 19 * 19
    m = wavelet.detail_mask(208, 208, 4)
    assert (~m).sum() == 13 * 13


@pytest.mark.parametrize("name,levels", [("haar", 3), ("db4", 2)])
def test_constant_image_lands_in_coarsest_lowpass(name, levels):
    # each level maps a constant c to c*2 in LL (sum h = sqrt 2 per axis) and 0 elsewhere
    x = np.full((32, 48), 0.75 + 0.25j)
    w = wavelet.dwt2(x, levels, name)
    ll = w[: 32 >> levels, : 48 >> levels]
    np.testing.assert_allclose(ll, (0.75 + 0.25j) * 2 ** levels, rtol=1e-13)
    det = wavelet.detail_mask(32, 48, levels)
    assert np.max(np.abs(w[det])) < 1e-13

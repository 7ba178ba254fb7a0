"""Pins of the coil pre-whitening and compression oracle (CPU).

* whitening: closed form for a diagonal covariance; whitened correlated noise
  has identity covariance (statistical, many samples); the model keeps its
  form with the whitened maps (L^{-1} (A x) = A_{L^{-1} S} x);
* compression: eigenvalues = squared singular values of the data (a library
  SVD); eigenvectors orthonormal and ordered; nv = C keeps the normal operator
  A^H A and the data norm; exactly rank-k data are reproduced from k virtual
  coils; compressed data = the forward model with the virtual maps."""
import numpy as np

import synth
from oracle import coils, encoding


def _rng(s):
    return np.random.default_rng(s)


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def test_whitening_diagonal_closed_form():
    rng = _rng(1)
    d = rng.uniform(0.5, 3.0, 6)
    y = _crandn(rng, 40, 6)
    s = _crandn(rng, 6, 25)
    yw, sw = coils.prewhiten(np.diag(d), y, s)
    assert np.allclose(yw, y / np.sqrt(d)[None, :], atol=1e-14)
    assert np.allclose(sw, s / np.sqrt(d)[:, None], atol=1e-14)


def test_whitened_noise_is_white():
    rng = _rng(2)
    C, n = 8, 200000
    m = _crandn(rng, C, C) + 2.0 * np.eye(C)
    psi = m @ m.conj().T
    noise = _crandn(rng, n, C) @ m.T                 # rows n_t = m z_t, covariance m m^H
    nw, _ = coils.prewhiten(psi, noise, np.zeros((C, 1)))
    cov = nw.T @ nw.conj() / n
    assert np.max(np.abs(cov - np.eye(C))) <= 6.0 / np.sqrt(n) * 3
    # an un-whitened covariance is far from the identity
    cov0 = noise.T @ noise.conj() / n
    assert np.max(np.abs(cov0 - np.eye(C))) > 0.5


def test_whitening_keeps_the_model():
    w = synth.TINY
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, 0.0, w.nbasis)
    rng = _rng(3)
    m = _crandn(rng, w.ncoils, w.ncoils) + 3.0 * np.eye(w.ncoils)
    psi = m @ m.conj().T
    y = encoding.forward(p.x_noisy, p.smaps, p.coef, p.time, basis, p.dw0)
    yw, sw = coils.prewhiten(psi, y, p.smaps)
    y2 = encoding.forward(p.x_noisy, sw, p.coef, p.time, basis, p.dw0)
    assert np.linalg.norm(yw - y2) <= 1e-12 * np.linalg.norm(y2)


def test_compression_eigenvalues_are_squared_singular_values():
    rng = _rng(4)
    y = _crandn(rng, 300, 10) @ _crandn(rng, 10, 10)
    w, v = coils.compression_matrix(y)
    sv = np.linalg.svd(y, compute_uv=False)
    assert np.allclose(w, sv ** 2, rtol=1e-10)
    assert np.all(np.diff(w) <= 0)
    assert np.allclose(v.conj().T @ v, np.eye(10), atol=1e-12)


def test_full_compression_keeps_normal_operator_and_norm():
    w = synth.TINY
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, 0.0, w.nbasis)
    args = (p.coef, p.time, basis, p.dw0)
    y = encoding.forward(p.x_noisy, p.smaps, *args)
    yv, sv, _, _ = coils.compress(y, p.smaps, w.ncoils)
    assert abs(np.linalg.norm(yv) - np.linalg.norm(y)) <= 1e-12 * np.linalg.norm(y)
    x = _crandn(_rng(5), w.npix)
    n1 = encoding.adjoint(encoding.forward(x, p.smaps, *args), p.smaps, *args)
    n2 = encoding.adjoint(encoding.forward(x, sv, *args), sv, *args)
    assert np.linalg.norm(n1 - n2) <= 1e-11 * np.linalg.norm(n1)


def test_rank_k_data_compress_losslessly():
    rng = _rng(6)
    T, C, k = 200, 12, 5
    y = _crandn(rng, T, k) @ _crandn(rng, k, C)
    yv, _, w, vk = coils.compress(y, np.zeros((C, 3)), k)
    assert np.linalg.norm(yv @ vk.conj().T - y) <= 1e-11 * np.linalg.norm(y)
    assert np.all(w[k:] <= 1e-9 * w[0])


def test_compressed_data_follow_the_virtual_model():
    w = synth.TINY
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, 0.0, w.nbasis)
    args = (p.coef, p.time, basis, p.dw0)
    y = encoding.forward(p.x_noisy, p.smaps, *args)
    yv, sv, _, _ = coils.compress(y, p.smaps, 4)
    y2 = encoding.forward(p.x_noisy, sv, *args)
    assert np.linalg.norm(yv - y2) <= 1e-12 * np.linalg.norm(y2)

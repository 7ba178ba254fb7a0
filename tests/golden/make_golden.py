"""Writes the FP64 oracle's reference reconstruction of the 1.5 mm workload
(148 x 148, 32 coils, T = 16384, 3rd-order field + dB0; 50 FISTA iterations
with a 3-level db4 wavelet; L from 20 power steps from the seeded start
vector; lambda = 1e-3 max|A^H y|) to mm15_fista.npz.  Calls only the oracle
and the seeded input generator.  Takes several minutes on 8 cores.

    python tests/golden/make_golden.py            # FISTA golden (mm15_fista.npz)
    python tests/golden/make_golden.py balanced   # balanced-FISTA golden (mm15_balanced.npz)
    python tests/golden/make_golden.py mm11       # 1.1 mm FISTA golden (mm11_fista.npz; ~1 h on 8 cores)
    python tests/golden/make_golden.py diff       # unrolled-FISTA gradients, differentiation workload
                                                  # (diff_unrolled.npz)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import encoding, solve  # noqa: E402


def c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def main():
    w = synth.MM15
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, w.z0, w.nbasis)
    op = solve.Operator(c64(p.smaps), p.coef, p.time, basis, p.dw0, w.n)
    t0 = time.time()
    y = c64(op.A(c64(p.x_noisy)))
    v0 = c64(synth.power_start(w.npix, 7))
    L = solve.power_lipschitz(op, v0, 20)
    lam = solve.lambda_rule(op, y)
    x = solve.fista(op, y, L, lam, w.n_iter, w.levels, w.wavelet, w.n_pad)
    np.savez_compressed(os.path.join(HERE, "mm15_fista.npz"), x_hat=x.astype(np.complex128), lipschitz=L,
                        lam=lam, n_iter=w.n_iter, n_power=20, power_seed=7)
    print(f"wrote mm15_fista.npz: L={L:.6e} lambda={lam:.6e} ({time.time() - t0:.0f} s)")


def main_mm11():
    """The 1.1 mm workload (200 x 200, 32 coils, T = 40000, 3rd-order field
    + dB0, diffusion-weighted phantom): 100 FISTA iterations with a 4-level
    db4 wavelet on the 208 x 208 grid, L from 20 power steps from the seeded
    start vector, lambda = 1e-3 max|A^H y|."""
    w = synth.MM11
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, w.z0, w.nbasis)
    op = solve.Operator(c64(p.smaps), p.coef, p.time, basis, p.dw0, w.n)
    t0 = time.time()
    y = c64(op.A(c64(p.x_noisy)))
    v0 = c64(synth.power_start(w.npix, 7))
    L = solve.power_lipschitz(op, v0, 20)
    lam = solve.lambda_rule(op, y)
    print(f"L={L:.6e} lambda={lam:.6e} ({time.time() - t0:.0f} s)", flush=True)
    x = solve.fista(op, y, L, lam, w.n_iter, w.levels, w.wavelet, w.n_pad)
    np.savez_compressed(os.path.join(HERE, "mm11_fista.npz"), x_hat=x.astype(np.complex128), lipschitz=L,
                        lam=lam, n_iter=w.n_iter, n_power=20, power_seed=7)
    print(f"wrote mm11_fista.npz: L={L:.6e} lambda={lam:.6e} ({time.time() - t0:.0f} s)")


def main_balanced():
    """The paper's regulariser on the same problem: undecimated db4 with one
    level, sigma/2 weights from W A^H y, balanced FISTA with kappa = L_A,
    50 iterations; L_A from the FISTA golden file."""
    from oracle import balanced as bal
    w = synth.MM15
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, w.z0, w.nbasis)
    op = solve.Operator(c64(p.smaps), p.coef, p.time, basis, p.dw0, w.n)
    t0 = time.time()
    y = c64(op.A(c64(p.x_noisy)))
    L_A = float(np.load(os.path.join(HERE, "mm15_fista.npz"))["lipschitz"])
    lam = bal.sigma_weights(bal.swt2(op.AH(y).reshape(w.n, w.n), 1, "db4"), 1)
    x = bal.fista(op, y, L_A, L_A, lam, 50, 1, "db4")
    np.savez_compressed(os.path.join(HERE, "mm15_balanced.npz"), x_hat=x.astype(np.complex128), lipschitz=L_A,
                        lam=lam, n_iter=50, levels=1)
    print(f"wrote mm15_balanced.npz: L_A={L_A:.6e} lambda={lam} ({time.time() - t0:.0f} s)")


def main_diff():
    """The differentiation workload (128 x 128, 16 coils, T = 12000, 3rd-order
    field + dB0): loss ||x_hat - x_true||^2 of 10 unrolled FISTA iterations
    (db4 J = 3, fixed L and lambda) on y = A x_in, x_in the noisy phantom, and
    its gradients with respect to x_in, k_l(t) and dB0 by the oracle's
    reverse pass.  L = 1.01 x the estimate of 30 power steps from the seeded
    start vector; lambda = 1e-3 max|A^H y|."""
    from oracle import unrolled
    w = synth.DIFF
    p = synth.make_problem(w)
    basis = encoding.sh_basis(w.n, w.fov, w.z0, w.nbasis)
    smaps = c64(p.smaps)
    op = solve.Operator(smaps, p.coef, p.time, basis, p.dw0, w.n)
    t0 = time.time()
    x_in = c64(p.x_noisy)
    L = 1.01 * solve.power_lipschitz(op, c64(synth.power_start(w.npix, 9)), 30)
    lam = solve.lambda_rule(op, op.A(x_in))
    print(f"L={L:.6e} lambda={lam:.6e} ({time.time() - t0:.0f} s)", flush=True)
    loss, gx, gc, gd = unrolled.reverse_loss_and_grads(x_in, c64(p.x_true), smaps, p.coef, p.time, basis, p.dw0, L,
                                                       lam, w.n_iter, w.levels, w.wavelet, w.n, w.n_pad)
    np.savez_compressed(os.path.join(HERE, "diff_unrolled.npz"), loss=loss, grad_x=gx.astype(np.complex64),
                        grad_coef=gc.astype(np.float32), grad_dw0=gd.astype(np.float32), lipschitz=L, lam=lam,
                        n_iter=w.n_iter, levels=w.levels, n_power=30, power_seed=9)
    print(f"wrote diff_unrolled.npz: loss={loss:.6e} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "balanced":
        main_balanced()
    elif len(sys.argv) > 1 and sys.argv[1] == "mm11":
        main_mm11()
    elif len(sys.argv) > 1 and sys.argv[1] == "diff":
        main_diff()
    else:
        main()

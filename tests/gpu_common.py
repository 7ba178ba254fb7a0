"""Shared helpers of the GPU parity tests: seeded inputs as torch device
tensors (for the HIP path) and as rounded numpy arrays (for the oracle)."""
from __future__ import annotations

import numpy as np

import synth


def c64(a: np.ndarray) -> np.ndarray:
    """Round to complex64 and back, so both sides see identical inputs."""
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


class Case:
    """One problem: numpy inputs for the oracle, device tensors for the GPU."""

    def __init__(self, w: synth.Workload, z0: float | None = None, ncoils: int | None = None,
                 with_dw0: bool = True, nbasis: int | None = None, sh: bool = False):
        import torch
        from oracle import encoding
        import paper_2211_07532_amd as ee

        self.w = w
        p = synth.make_problem(w)
        nb = w.nbasis if nbasis is None else nbasis
        self.z0 = w.z0 if z0 is None else z0
        self.smaps = c64(p.smaps if ncoils is None else synth.coil_maps(w, ncoils))
        self.coef = p.coef[:, :nb].copy()
        self.time = p.time
        self.dw0 = p.dw0 if with_dw0 else None
        self.x_true = c64(p.x_true)
        self.x_noisy = c64(p.x_noisy)
        self.basis_np = encoding.sh_basis(w.n, w.fov, self.z0, nb)
        dev = torch.device("cuda")
        self.dev = dev
        self.t_smaps = torch.from_numpy(self.smaps.astype(np.complex64)).to(dev)
        self.t_coef = torch.from_numpy(self.coef).to(dev)
        self.t_time = torch.from_numpy(self.time).to(dev)
        self.t_dw0 = None if self.dw0 is None else torch.from_numpy(self.dw0).to(dev)
        # the GPU evaluates its own basis from the grid geometry
        self.t_basis = ee.sh_basis(w.n, w.n, w.fov, w.fov, self.z0, nb, device=dev)
        if sh and nb > 0:
            # the basis declared as solid harmonics on the grid: the library evaluates it itself
            self.op = ee.Operator(w.n, w.n, self.t_smaps, self.t_coef, self.t_time, None, self.t_dw0,
                                  sh_grid=(w.fov, w.fov, self.z0))
        else:
            self.op = ee.Operator(w.n, w.n, self.t_smaps, self.t_coef, self.t_time, self.t_basis, self.t_dw0)

    def oracle_args(self):
        return (self.smaps, self.coef, self.time, self.basis_np, self.dw0)

    def to_dev(self, a: np.ndarray):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(self.dev)


def emulated_split_errors(case, x, g, ts, rs, kind, y_norm=None, x_norm=None):
    """Relative errors that the round-to-nearest-even emulation of the split
    arithmetic (oracle.splitemu: phase tile rounded to FP32, both operands
    split hi/lo, three products) shows for the forward (input image x [R])
    and the adjoint (input data g [T][C], coil combination in FP64), against
    exact FP64 sums, evaluated on the sample rows ts and pixels rs.  With all
    rows / pixels these are the whole outputs' errors.  With a uniform random
    subset, pass the exact norms of the whole outputs (y_norm, x_norm): the
    error energy of the subset, scaled by T/len(ts) (R/len(rs)), then
    estimates the whole output's (the error is spread evenly over the
    outputs while their energy is not)."""
    from oracle import encoding, splitemu
    coef, time, basis, dw0, smaps = case.coef, case.time, case.basis_np, case.dw0, case.smaps
    z = (smaps * x[None, :]).T                                    # [R][C]
    ph = encoding.phase(coef[ts], time[ts], basis, dw0)           # [len(ts)][R]
    e32 = np.exp(1j * ph).astype(np.complex64).astype(np.complex128)
    y_ex = np.exp(1j * ph) @ z
    d_y = np.linalg.norm(splitemu.split_cmatmul(e32, c64(z), kind) - y_ex)
    ph = encoding.phase(coef, time, basis[:, rs], None if dw0 is None else dw0[rs])  # [T][len(rs)]
    e32 = np.exp(1j * ph).astype(np.complex64).astype(np.complex128)
    u = splitemu.split_cmatmul(np.conj(e32).T, g, kind)           # [len(rs)][C]
    x_emu = np.sum(np.conj(smaps[:, rs]).T * u, axis=1)
    x_ex = np.sum(np.conj(smaps[:, rs]).T * (np.conj(np.exp(1j * ph)).T @ g), axis=1)
    d_x = np.linalg.norm(x_emu - x_ex)
    if y_norm is None:
        fwd = d_y / np.linalg.norm(y_ex)
    else:
        fwd = d_y * np.sqrt(len(time) / len(ts)) / y_norm
    if x_norm is None:
        adj = d_x / np.linalg.norm(x_ex)
    else:
        adj = d_x * np.sqrt(smaps.shape[1] / len(rs)) / x_norm
    return float(fwd), float(adj)

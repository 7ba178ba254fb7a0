"""Round-to-nearest-even emulation of bf16 / fp16 hi-lo split products.
Test infrastructure only.

A value v (already rounded to float32) is split as hi = rnd(v),
lo = rnd(v - hi); a product a*b is then taken as
hi_a*hi_b + hi_a*lo_b + lo_a*hi_b (the lo*lo term dropped), each product
exact and the sum accumulated in higher precision.  With p mantissa bits
(8 for bf16, 11 for fp16) the relative error per product is about
3 * 2^(-2p), which is the error level the split-precision operators are
expected to show.  Used on tiny sizes only.
"""
from __future__ import annotations

import numpy as np


def round_bf16(v: np.ndarray) -> np.ndarray:
    """float32 -> nearest bf16 (ties to even), returned as float64."""
    f = np.asarray(v, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def round_fp16(v: np.ndarray) -> np.ndarray:
    return np.asarray(v, dtype=np.float32).astype(np.float16).astype(np.float64)


def split(v: np.ndarray, kind: str):
    rnd = round_bf16 if kind == "bf16" else round_fp16
    v32 = np.asarray(v, dtype=np.float32)
    hi = rnd(v32)
    lo = rnd((v32.astype(np.float64) - hi).astype(np.float32))
    return hi, lo


def split_matmul(a: np.ndarray, b: np.ndarray, kind: str) -> np.ndarray:
    """Real a @ b with both operands split; three products."""
    ah, al = split(a, kind)
    bh, bl = split(b, kind)
    return ah @ bh + ah @ bl + al @ bh


def split_cmatmul(a: np.ndarray, b: np.ndarray, kind: str) -> np.ndarray:
    """Complex a @ b through four real split products."""
    ar, ai = a.real, a.imag
    br, bi = b.real, b.imag
    re = split_matmul(ar, br, kind) - split_matmul(ai, bi, kind)
    im = split_matmul(ar, bi, kind) + split_matmul(ai, br, kind)
    return re + 1j * im

"""Oracle emulation of the reduced-precision operators (test infrastructure).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Mixed precision is not in the paper; these are this project's definitions of
the FP32 and BF16 local operators, evaluated with numpy in the stated
precisions so the GPU results can be bounded against them:

* FP32: u, D, G, B in float32, every product and sum in float32.
* BF16: u, D, G, B rounded to bfloat16 (round to nearest even); the
  derivative contractions sum exact BF16 x BF16 products in float32; the
  G-combination is float32 and its three results are rounded to BF16; the
  transposed contractions sum in float32 and the r, s, t contributions are
  added in that order; the Helmholtz term h2 B u is float32.
* BF16 split: G and B are stored in IEEE half precision with one
  power-of-two scale per element and array (``f16_scaled_storage``); u, D and
  the intermediate fluxes enter the matrix cores as hi + lo BF16 pairs
  (three products per contraction, FP32 sums).  Its reference is the exact
  operator with the stored G and B (``ax_bf16_split_reference``); the split
  reproduces that to about 2^-16 relative.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nonfinite = ~np.isfinite(x)
    out = np.where(nonfinite, x, out)
    return out.reshape(np.shape(a))


def _contract(D, u, axis_letter, transpose):
    """Apply D (or D^T) along one tensor direction of u[E, k, j, i] in the
    dtype of the inputs."""
    Dm = D.T if transpose else D
    if axis_letter == "r":
        return np.einsum("im,ekjm->ekji", Dm, u)
    if axis_letter == "s":
        return np.einsum("jm,ekmi->ekji", Dm, u)
    return np.einsum("km,emji->ekji", Dm, u)


def ax_lowp(mesh, u, h1, h2, precision):
    """Local operator in 'f32' or 'bf16' (see module docstring); returns float64."""
    f32 = np.float32
    if precision == "f32":
        D = mesh.D.astype(f32)
        G = mesh.G.astype(f32)
        B = mesh.B.astype(f32)
        uu = np.asarray(u).astype(f32)
        rnd = lambda a: a
    elif precision == "bf16":
        D = bf16_round(mesh.D.astype(f32))
        G = bf16_round(mesh.G.astype(f32))
        B = bf16_round(mesh.B.astype(f32))
        uu = bf16_round(np.asarray(u).astype(f32))
        rnd = bf16_round
    else:
        raise ValueError(precision)
    ur = _contract(D, uu, "r", False).astype(f32)
    us = _contract(D, uu, "s", False).astype(f32)
    ut = _contract(D, uu, "t", False).astype(f32)
    wr = rnd(G[0] * ur + G[1] * us + G[2] * ut)
    ws = rnd(G[1] * ur + G[3] * us + G[4] * ut)
    wt = rnd(G[2] * ur + G[4] * us + G[5] * ut)
    w = _contract(D, wr, "r", True).astype(f32)
    w = w + _contract(D, ws, "s", True).astype(f32)
    w = w + _contract(D, wt, "t", True).astype(f32)
    w = f32(h1) * w + f32(h2) * B * uu
    return w.astype(np.float64)


def bf16_storage(a):
    """Geometric factors as the BF16 operators store them (float32, then RNE
    to bfloat16), returned as float64."""
    return bf16_round(np.asarray(a).astype(np.float32)).astype(np.float64)


def f16_scale_exponents(a, elem_axis):
    """Per-element exponent k of the half-precision storage: the largest
    magnitude of the element's values divided by 2^k lies in [2^14, 2^15),
    the top binade below the half-precision maximum (k = 0 for an element of
    zeros)."""
    a = np.asarray(a, dtype=np.float64)
    axes = tuple(d for d in range(a.ndim) if d != elem_axis)
    m = np.max(np.abs(a), axis=axes)
    _, x = np.frexp(m)            # m = f 2^x with f in [0.5, 1)
    return np.where(m > 0, x - 15, 0).astype(np.int64)


def f16_scaled_storage(a, elem_axis):
    """Values as the split-BF16 operator stores them: per element, a / 2^k
    rounded to IEEE half (ties to even, straight from float64), times 2^k,
    as float64.  The scaling by a power of two is exact, so the only error is
    the half rounding, at most 2^-11 relative (or 2^-39 of the element's
    largest magnitude for values that fall below the half normal range)."""
    a = np.asarray(a, dtype=np.float64)
    k = f16_scale_exponents(a, elem_axis)
    shape = [1] * a.ndim
    shape[elem_axis] = -1
    k = k.reshape(shape)
    h = np.ldexp(a, -k).astype(np.float16)
    return np.ldexp(h.astype(np.float64), k)


def ax_bf16_split_reference(mesh, u, h1, h2):
    """Exact (FP64) local operator with G [6, E, ...] and B [E, ...] as the
    split-BF16 operator stores them (half precision, per-element scale)."""
    return mesh.ax(u, h1, h2, G=f16_scaled_storage(mesh.G, 1), B=f16_scaled_storage(mesh.B, 0))

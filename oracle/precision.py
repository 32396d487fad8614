"""16-bit storage formats of the mixed-precision path (oracle, test infrastructure).

The paper runs in double precision throughout; storing fields and operators
in 16 bits with FP32 arithmetic is an implementation choice for the
preconditioner, where only the outer FGCR's true residual (computed in FP64)
decides convergence.  These functions define the storage format exactly, so
that the GPU's conversion can be compared bit for bit and its 16-bit
kernels can be compared with the FP64 oracle applied to the same stored
values.

Definitions (every rounding is round-to-nearest-even):

* ``round_f32``: FP64 -> FP32.
* ``round_16(x32, kind)``: FP32 -> FP16 (``numpy.float16``) or BF16 (the top
  16 bits of the FP32 pattern after adding ``0x7FFF`` plus the lowest kept
  bit), returned as exact FP32 values.
* fine field (per site and right-hand side): ``x32 = round_f32(psi)``;
  ``s = max |real component|`` over the site's 24 reals (FP32);
  ``inv = fl32(1 / s)``; stored ``q = round_16(fl32(x32 * inv))``; read back as
  ``fl32(s * q)``.  A site with ``s`` below the smallest normal FP32 number
  reads back as zero.
* prolongator columns: ``round_16(round_f32(v))``, no scale.
* SU(3) links: the first two rows as prolongator columns; the third row is
  not stored but rebuilt as ``conj(row0 x row1)`` from the stored rows (for
  a unitary matrix with determinant 1 this is the third row), here in FP64.
* coarse-operator blocks: as a fine site, with the whole (2Nv x 2Nv) block in
  place of the site's 24 reals.

Parity pinned by the tests of this module: exactly representable values are
unchanged, ties go to the even neighbour, the largest component of a site
maps to exactly +-1, and the read-back error is at most half a unit in the
last place of the 16-bit format times the scale.
"""
from __future__ import annotations

import numpy as np

FLT_MIN = np.float32(np.finfo(np.float32).tiny)
# half a unit in the last place of values in [0.5, 1) (the worst case of a
# value scaled into [-1, 1])
HALF_ULP = {"f16": 2.0 ** -12, "bf16": 2.0 ** -9}


def round_f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x).astype(np.complex64 if np.iscomplexobj(x) else np.float32)


def _bf16_bits(x32: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    return (rounded << 16).astype(np.uint32)


def round_16(x32: np.ndarray, kind: str) -> np.ndarray:
    """FP32 (real array) -> nearest 16-bit value of ``kind``, as FP32."""
    x32 = np.asarray(x32, dtype=np.float32)
    if kind == "f16":
        return x32.astype(np.float16).astype(np.float32)
    if kind == "bf16":
        if not np.all(np.isfinite(x32)):
            raise ValueError("bf16 rounding is defined here for finite values only")
        return _bf16_bits(x32).view(np.float32).reshape(x32.shape)
    raise ValueError(kind)


def _re_im(z32: np.ndarray) -> np.ndarray:
    return np.stack([z32.real, z32.imag], axis=-1)


def quantise_groups(z: np.ndarray, kind: str, ngroup_axes: int):
    """Scale-and-round every group formed by the last ``ngroup_axes`` axes.

    Returns ``(scale, q, readback)``: FP32 scales of shape ``z.shape[:-ngroup_axes]``,
    stored values ``q`` (complex64, exact 16-bit numbers) and the FP32 read-back."""
    z32 = round_f32(np.asarray(z, dtype=np.complex128))
    parts = _re_im(z32)                                  # [..., group..., 2] float32
    axes = tuple(range(z32.ndim - ngroup_axes, z32.ndim + 1))
    s = np.max(np.abs(parts), axis=axes).astype(np.float32)
    zero = s < FLT_MIN
    with np.errstate(divide="ignore"):
        inv = np.where(zero, np.float32(0), np.float32(1) / np.where(zero, np.float32(1), s)).astype(np.float32)
    inv_b = inv.reshape(inv.shape + (1,) * (ngroup_axes + 1))
    q = round_16((parts * inv_b).astype(np.float32), kind)
    s = np.where(zero, np.float32(0), s).astype(np.float32)
    s_b = s.reshape(s.shape + (1,) * (ngroup_axes + 1))
    back = (s_b * q).astype(np.float32)
    qz = (q[..., 0] + 1j * q[..., 1]).astype(np.complex64)
    bz = (back[..., 0] + 1j * back[..., 1]).astype(np.complex64)
    return s, qz, bz


def store_fine(psi: np.ndarray, kind: str) -> np.ndarray:
    """Read-back of a canonical fine field ``[..., 4, 3]`` after 16-bit storage."""
    return quantise_groups(psi, kind, 2)[2]


def store_links(u: np.ndarray, kind: str) -> np.ndarray:
    """Links (or any unscaled operator entries) after 16-bit storage, complex64."""
    z32 = round_f32(np.asarray(u, dtype=np.complex128))
    return (round_16(z32.real, kind) + 1j * round_16(z32.imag, kind)).astype(np.complex64)


def store_su3_links(u: np.ndarray, kind: str) -> np.ndarray:
    """SU(3) links ``[..., 3, 3]`` as the 16-bit path uses them (complex128):
    rows 0 and 1 rounded, row 2 rebuilt from them."""
    r = store_links(np.asarray(u)[..., :2, :], kind).astype(np.complex128)
    row2 = np.conj(np.cross(r[..., 0, :], r[..., 1, :]))
    return np.concatenate([r, row2[..., None, :]], axis=-2)

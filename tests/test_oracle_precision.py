"""Pins of the 16-bit storage formats (oracle.precision) against brute force and
the defining properties of round-to-nearest-even scaling."""
import numpy as np
import pytest

import synthetic
from oracle import precision


def _neighbours_bf16(x):
    """The two bf16 values around float32 x (truncation and the next one up in magnitude)."""
    bits = np.float32(x).view(np.uint32)
    lo = np.uint32(bits & 0xFFFF0000)
    hi = np.uint32(lo + 0x10000)
    return lo.view(np.float32), hi.view(np.float32)


def test_bf16_rounding_is_nearest_even_by_brute_force():
    rng = np.random.default_rng(0)
    xs = (rng.standard_normal(4000) * 10.0 ** rng.uniform(-20, 20, 4000)).astype(np.float32)
    got = precision.round_16(xs, "bf16")
    for x, g in zip(xs, got):
        lo, hi = _neighbours_bf16(x)
        dlo, dhi = abs(float(x) - float(lo)), abs(float(x) - float(hi))
        if dlo < dhi:
            want = lo
        elif dhi < dlo:
            want = hi
        else:  # tie: even last kept bit
            want = lo if (int(np.float32(lo).view(np.uint32)) >> 16) % 2 == 0 else hi
        assert np.float32(g).view(np.uint32) == np.float32(want).view(np.uint32), (x, g, want)


def test_f16_rounding_is_nearest_even_by_brute_force():
    rng = np.random.default_rng(1)
    xs = (rng.uniform(-1, 1, 4000) * 2.0 ** rng.integers(-20, 15, 4000)).astype(np.float32)
    got = precision.round_16(xs, "f16")
    grid = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float64)  # all finite >= 0
    for x, g in zip(xs, got):
        a = abs(float(x))
        i = np.searchsorted(grid, a)
        cands = [grid[j] for j in (i - 1, i) if 0 <= j < len(grid)]
        d = [abs(a - cc) for cc in cands]
        best = [cc for cc, dd in zip(cands, d) if dd == min(d)]
        if len(best) == 2:  # tie: even mantissa
            best = [cc for cc in best if np.float16(cc).view(np.uint16) % 2 == 0]
        assert abs(float(g)) == best[0] and (g == 0 or np.sign(g) == np.sign(x)), (x, g, best)


@pytest.mark.parametrize("kind,tie,down,up", [
    ("f16", 1 + 2.0 ** -11, 1.0, 1 + 2.0 ** -10),        # ties to the even 1.0
    ("f16", 1 + 3 * 2.0 ** -11, 1 + 2.0 ** -10, 1 + 2.0 ** -9),
    ("bf16", 1 + 2.0 ** -8, 1.0, 1 + 2.0 ** -7),
    ("bf16", 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, 1 + 2.0 ** -6),
])
def test_ties_round_to_even(kind, tie, down, up):
    """A value halfway between two neighbours goes to the one with an even last bit:
    1 (mantissa ...0) below, and the upper neighbour when the lower one is odd."""
    got = float(precision.round_16(np.float32(tie), kind))
    assert got in (down, up)
    lower_is_even = tie in (1 + 2.0 ** -11, 1 + 2.0 ** -8)
    assert got == (down if lower_is_even else up)


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_fine_storage_properties(kind):
    dims = (2, 2, 2, 4)
    psi = synthetic.gaussian_spinor(dims, seed=3, nrhs=2)
    rng = np.random.default_rng(4)
    psi = psi * 10.0 ** rng.uniform(-6, 6, size=psi.shape[:-2])[..., None, None]
    s, q, back = precision.quantise_groups(psi, kind, 2)
    parts = np.stack([q.real, q.imag], -1)
    # every stored value lies in [-1, 1] and each site's largest one is exactly +-1
    assert np.abs(parts).max() <= 1.0
    assert np.all(np.abs(parts).max(axis=(-3, -2, -1)) == 1.0)
    # read-back error: half an ulp of the 16-bit format times the scale (plus FP32 rounding)
    p32 = psi.astype(np.complex64).astype(np.complex128)
    err = np.maximum(np.abs((back - p32).real), np.abs((back - p32).imag)).max(axis=(-2, -1))
    assert np.all(err <= precision.HALF_ULP[kind] * s * (1 + 2.0 ** -20))
    # power-of-two rescaling commutes with storage (scales are exact)
    back2 = precision.store_fine(psi * 2.0 ** 7, kind)
    assert np.array_equal(back2, (back.astype(np.complex128) * 2.0 ** 7).astype(np.complex64))
    # exactly representable fields are unchanged
    exact = np.zeros_like(psi)
    exact[..., 0, 0] = 1.0
    exact[..., 1, 2] = -0.5 + 0.25j
    assert np.array_equal(precision.store_fine(exact, kind), exact.astype(np.complex64))
    # a zero site stays zero
    assert np.all(precision.store_fine(np.zeros_like(psi), kind) == 0)


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_su3_link_storage(kind):
    u = synthetic.gauge_field((2, 2, 2, 2), 0.4, 11)
    us = precision.store_su3_links(u, kind)
    # rows 0 and 1 are the rounded rows; row 2 is rebuilt and stays close to unitary
    assert np.array_equal(us[..., :2, :], precision.store_links(u[..., :2, :], kind).astype(np.complex128))
    tol = {"f16": 2e-3, "bf16": 1.5e-2}[kind]
    assert np.abs(us - u).max() < tol
    # unit links are exact in every format
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), u.shape)
    assert np.array_equal(precision.store_su3_links(one, kind), one)

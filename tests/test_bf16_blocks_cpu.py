"""The arithmetic facts the matrix-core collision rests on, checked on the
host from the paper's M (the oracle's FP64 construction of Eq. 5) and from
the IEEE formats, independently of the library's own tables:

* after the per-group butterflies, M is block diagonal (the 4x4 blocks of
  the conserved/even moments, of the x-odd and y-odd moments, and the two
  2x2 quadrupole blocks), and every block entry is a number with at most 8
  significant bits -- exact in BF16 -- once the diagonal groups' columns of
  the x and y blocks are divided by sqrt 2;
* an FP32 value splits exactly into three BF16 parts by round-to-nearest-
  even and exact remainders (hi + mid + lo = x); the first remainder is at
  most 2^-8 |x| and the second 2^-17 |x| (8 significant bits per part).
"""
import math

import numpy as np

from oracle import core

# moments (0-based rows of M) of each block, over the butterfly outputs:
# columns 0..3 A of the four velocity groups, 4..7 X, 8..11 Y, 12..15 Q
BLOCKS = [((0, 3, 10, 11), (0, 1, 2, 3)), ((1, 6, 8, 14), (4, 5, 6, 7)),
          ((2, 7, 9, 15), (8, 9, 10, 11)), ((4, 12), (12, 13)), ((5, 13), (14, 15))]


def butterfly():
    """The per-group sums and differences of the populations: groups of four
    consecutive velocities, the axis groups ordered (+,0), (0,+), (-,0),
    (0,-) and the diagonal groups (+,+), (-,+), (-,-), (+,-)."""
    F = np.zeros((16, 16))
    for g in range(4):
        b = 4 * g
        F[g, b:b + 4] = [1, 1, 1, 1]
        F[12 + g, b:b + 4] = [1, -1, 1, -1]
        if g < 2:
            F[4 + g, [b, b + 2]] = [1, -1]
            F[8 + g, [b + 1, b + 3]] = [1, -1]
        else:
            F[4 + g, b:b + 4] = [1, -1, -1, 1]
            F[8 + g, b:b + 4] = [1, 1, -1, -1]
    return F


def bf16_exact(w, tol=1e-12):
    if w == 0.0:
        return True
    m, _ = math.frexp(w)
    t = m * 256.0
    return abs(t - round(t)) <= tol * 256.0


def test_velocity_groups_are_the_butterflys():
    v = core.model().v
    axis = np.array([(1, 0), (0, 1), (-1, 0), (0, -1)], dtype=float)
    diag = np.array([(1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
    for g, pattern in enumerate((axis, axis, diag, diag)):
        dirs = v[4 * g:4 * g + 4]
        dirs = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
        np.testing.assert_allclose(dirs, pattern / np.linalg.norm(pattern, axis=1, keepdims=True), atol=1e-14)


def test_forward_transform_is_block_diagonal_and_exact_in_bf16():
    M = core.model().M
    B = M @ np.linalg.inv(butterfly())
    scale = np.max(np.abs(B))
    mask = np.zeros_like(B, dtype=bool)
    for rows, cols in BLOCKS:
        mask[np.ix_(rows, cols)] = True
    assert np.max(np.abs(B[~mask])) <= 1e-12 * scale
    for bi, (rows, cols) in enumerate(BLOCKS):
        for i in rows:
            for c in cols:
                w = B[i, c]
                if bi in (1, 2) and c % 4 >= 2:   # diagonal groups of the x and y blocks
                    assert not bf16_exact(w) or w == 0.0, (i, c, w)
                    w = w / math.sqrt(2.0)
                assert bf16_exact(w, tol=1e-9), (bi, i, c, B[i, c])


def bf16(x32):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP32."""
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def test_three_way_split_is_exact_and_remainders_within_their_bounds():
    rng = np.random.default_rng(11)
    mant = rng.uniform(1.0, 2.0, 400000)
    expo = rng.integers(-40, 40, mant.size)
    sign = rng.choice([-1.0, 1.0], mant.size)
    x = (sign * mant * np.exp2(expo)).astype(np.float32)
    edge = np.array([1.0, -1.0, np.nextafter(np.float32(2.0), np.float32(0.0)), 1.0 + 2.0 ** -23,
                     1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 3.0 * 2.0 ** -20, 1.00390625 + 2.0 ** -23],
                    dtype=np.float32)
    x = np.concatenate([x, edge, -edge])
    hi = bf16(x)
    r = x - hi                                  # FP32 arithmetic
    assert np.array_equal(r.astype(np.float64), x.astype(np.float64) - hi.astype(np.float64))
    mid = bf16(r)
    lo = bf16((r - mid).astype(np.float32))
    total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, x.astype(np.float64))
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(r.astype(np.float64)) <= 2.0 ** -8 * ax)
    resid = np.abs(r.astype(np.float64) - mid.astype(np.float64))   # the two-part split's remainder
    assert np.all(resid <= 2.0 ** -17 * ax)
    assert np.max(resid / ax) > 2.0 ** -18                           # and the bound is not loose by 2

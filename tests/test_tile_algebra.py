"""Index algebra of the float32 matrix-core tile bodies, checked on the CPU
with an exact model of the 16x16x4 matrix instruction (no GPU, no oracle).

The model: A is 16 x 4 (lane l supplies A[l % 16][l // 16]), B is 4 x 16
(lane l supplies B[l // 16][l % 16]), and lane l's result register v holds
row 4 (l // 16) + v, column l % 16 of A B + C.  The kernels feed lane li the
channels of block row 4 (li % 4) + li // 4 in the horizontal product, take
result register v of a ring block as the vertical step's B operand, build
the vertical Toeplitz slice of step j = 4 d + v as tap(4 j + lane // 16 - r -
lane % 16), and issue only the steps j < SH = ceil((16 + 2r) / 4).  Under
that model the vertical pass must equal the truncated convolution of
eq. (1)'s spatial kernel over the ring's rows, for every radius the kernels
take, and every skipped step must carry only zero taps."""
import numpy as np
import pytest


def hrow_of_lane(li):
    return 4 * (li % 4) + li // 4


def mfma_16x16x4(a_lanes, b_lanes, c):
    """c (16 x 16) += A B with A, B given per lane as the instruction reads
    them."""
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for lane in range(64):
        A[lane % 16, lane // 16] = a_lanes[lane]
        B[lane // 16, lane % 16] = b_lanes[lane]
    return c + A @ B


def result_register(D, v):
    """Per-lane value of result register v: row 4 (l // 16) + v, column
    l % 16."""
    return np.array([D[4 * (lane // 16) + v, lane % 16] for lane in range(64)])


@pytest.mark.parametrize("r", list(range(1, 49)))
def test_vertical_steps_equal_the_banded_convolution(r):
    rng = np.random.default_rng(r)
    g = np.concatenate([[1.0], rng.uniform(0.1, 1.0, r)])

    def tap(d):
        return g[abs(d)] if abs(d) <= r else 0.0

    SH = (16 + 2 * r + 3) // 4
    DV = (16 + 2 * r + 15) // 16
    # H rows of the ring: DV blocks of 16 rows x 16 columns
    Hrows = rng.standard_normal((16 * DV, 16))
    # each ring block is a horizontal product's result; with the identity
    # as B its result row m is the A row lane m fed: block row hrow_of_lane(m)
    ring = []
    eye = np.eye(4)
    for d in range(DV):
        blk = Hrows[16 * d:16 * d + 16]
        regs = []
        for v in range(4):
            # column-by-column: the result's column n is H row (of the lane's
            # A row) at column n; build it with 4 products of k-slices
            D = np.zeros((16, 16))
            for kk in range(4):
                a = [blk[hrow_of_lane(lane % 16), 4 * kk + lane // 16] for lane in range(64)]
                b = [eye[lane // 16][(lane % 16) - 4 * kk] if 0 <= (lane % 16) - 4 * kk < 4
                     else 0.0 for lane in range(64)]
                D = mfma_16x16x4(a, b, D)
            regs.append(result_register(D, v))
        ring.append(regs)
    # register v of block d holds block row 4 v + lane // 16
    for d in range(DV):
        for v in range(4):
            want = [Hrows[16 * d + 4 * v + lane // 16, lane % 16] for lane in range(64)]
            assert np.array_equal(ring[d][v], want)
    # vertical pass: steps j < SH only; the rest must be all-zero slices
    out = np.zeros((16, 16))
    for j in range(4 * DV):
        at = [tap(4 * j + lane // 16 - r - lane % 16) for lane in range(64)]
        if j >= SH:
            assert not any(at), (r, j)
            continue
        out = mfma_16x16x4(at, ring[j // 4][j % 4], out)
    # output row m of the block is window row m + r of the ring
    want = np.zeros((16, 16))
    for m in range(16):
        for h in range(16 * DV):
            want[m] += tap(h - r - m) * Hrows[h]
    assert np.allclose(out, want, rtol=0, atol=1e-12)
    # and every non-zero tap of the window is met: rows m .. m + 2r
    assert 4 * SH >= 16 + 2 * r and 4 * (SH - 1) <= 15 + 2 * r

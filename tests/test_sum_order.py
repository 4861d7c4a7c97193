"""The summation order of the heat-bath cumulative weights moves draws only at rounding level.

The oracle adds the weights one value at a time in value order (the plain reading of the
inverse-CDF draw of Sec. 3.3.2).  Kernels that split the range over the 64 lanes of a
wavefront add them in another order: value j belongs to block j // c (c = ceil(W / 64)); the
block sums are combined by a scan over four rows of 16 blocks (strides 1, 2, 4, 8 inside a row,
then the last entry of rows 0 and 2 into rows 1 and 3, then the last entry of row 1 into rows 2
and 3), and C_v is the preceding blocks' scan plus the running sum inside v's block.  The two
orders give cumulative weights that differ by a few units in the last place, so a draw can part
only when U * total falls within that distance of a cumulative weight.  This test runs both
orders on the same chains (same start states, same uniform numbers) of a sparse QUIO problem
shaped like the N = 10^4 Erdos-Renyi workload (mean degree 8, W = 101) and checks that at least
99.9 % of the reads end identical, and that the orders' cumulative weights agree to rounding.
"""
import numpy as np

import oracle
from paper_2511_17245_amd import inputs as I


def _blocked_cumulative(w):
    """C_v in the blocked order (rows of reads, columns of values)."""
    R, W = w.shape
    c = -(-W // 64)
    pad = np.zeros((R, 64 * c))
    pad[:, :W] = w
    blocks = pad.reshape(R, 64, c)
    run = np.add.accumulate(blocks, axis=2)          # running sum inside each block, left to right
    incl = run[:, :, -1].copy()                      # block sums
    for stride in (1, 2, 4, 8):
        prev = incl.copy()
        for b in range(64):
            if b % 16 >= stride:
                incl[:, b] = prev[:, b] + prev[:, b - stride]
    incl[:, 16:32] += incl[:, 15:16]
    incl[:, 48:64] += incl[:, 47:48]
    incl[:, 32:64] += incl[:, 31:32]
    before = np.concatenate([np.zeros((R, 1)), incl[:, :63]], axis=1)
    C = (before[:, :, None] + run).reshape(R, 64 * c)[:, :W]
    return C, incl[:, 63]


def _plain_cumulative(w):
    C = np.add.accumulate(w, axis=1)                 # sequential, value order
    return C, C[:, -1]


def _draw(C, total, U):
    thr = U * total
    passed = C > thr[:, None]
    idx = np.argmax(passed, axis=1)
    idx[~passed.any(axis=1)] = C.shape[1] - 1
    return idx


def test_blocked_and_value_order_agree_on_almost_every_read():
    rng = np.random.Generator(np.random.PCG64(2511))
    n, lo, hi, reads, sweeps = 200, -50, 50, 512, 30
    p = I.erdos_renyi_quio(n, 8.0, lo, hi, 10, 20, rng)
    J = np.zeros((n, n), np.int64)
    h = np.zeros(n, np.int64)
    for c, vs in p.terms():
        if len(vs) == 1:
            h[vs[0]] += c
        else:
            i, j = vs
            J[i, j] += c
            J[j, i] += c
    beta, _, _ = oracle.Poly(p).schedule(sweeps)
    W = hi - lo + 1
    vals = np.arange(lo, hi + 1, dtype=np.int64)
    z0 = rng.integers(lo, hi + 1, size=(reads, n))
    za, zb = z0.copy(), z0.copy()
    parted = 0
    worst = 0.0
    for s in range(sweeps):
        U = rng.random((n, reads))
        for k in range(n):
            for z, order in ((za, _plain_cumulative), (zb, _blocked_cumulative)):
                a1 = z @ J[k] + h[k]                                    # dE(v) = a1 (v - z_k)
                d = a1[:, None] * (vals[None, :] - z[:, k][:, None])
                w = np.exp(-(beta[s] * (d - d.min(axis=1, keepdims=True)).astype(np.float64)))
                C, total = order(w)
                z[:, k] = lo + _draw(C, total, U[k])
            if s % 10 == 0 and k % 50 == 0:
                same = np.all(za == zb, axis=1)
                a1 = za[same] @ J[k] + h[k]
                d = a1[:, None] * (vals[None, :] - za[same][:, k][:, None])
                w = np.exp(-(beta[s] * (d - d.min(axis=1, keepdims=True)).astype(np.float64)))
                Ca, ta = _plain_cumulative(w)
                Cb, tb = _blocked_cumulative(w)
                worst = max(worst, float(np.max(np.abs(Ca - Cb) / ta[:, None])))
        parted = int(np.sum(np.any(za != zb, axis=1)))
    assert parted <= reads // 1000, parted
    # the two orders' cumulative weights differ only by rounding (a few units of 2^-53)
    assert worst < 64 * 2.0 ** -53, worst

"""Why the pair kernels' sources are sorted along a Hilbert curve (host-side
check of the design choice, independent of the HIP sort): on the uniform
dilute field of 16384 vortices, chunks of 64 consecutive sources in Hilbert
order are far more compact than in Morton (Z) order, whose jumps across
quadrant edges make chunks straddle distant clumps.  The radius of a chunk
(about its centre) bounds how close a target may be for the chunk's multipole
expansion to converge, so compact chunks send more far chunks through their
expansions.  Both curves here follow their textbook constructions on a
16-bit grid with one scale for both axes, as the kernel does."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def grid16(x):
    lo = x.min(0)
    span = (x.max(0) - lo).max()
    return np.floor((x - lo) / span * 65535).astype(np.int64)


def morton(q):
    def spread(v):
        v = v & 0xFFFF
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        return (v | (v << 1)) & 0x55555555
    return spread(q[:, 0]) | (spread(q[:, 1]) << 1)


def hilbert(q):
    q1, q2 = q[:, 0].copy(), q[:, 1].copy()
    d = np.zeros(len(q), np.int64)
    s = 1 << 15
    while s > 0:
        r1 = ((q1 & s) > 0).astype(np.int64)
        r2 = ((q2 & s) > 0).astype(np.int64)
        d += s * s * ((3 * r1) ^ r2)
        flip = (r2 == 0) & (r1 == 1)
        q1[flip] = 65535 - q1[flip]
        q2[flip] = 65535 - q2[flip]
        sw = r2 == 0
        q1[sw], q2[sw] = q2[sw].copy(), q1[sw].copy()
        s >>= 1
    return d


def chunk_radii(x, key):
    xs = x[np.argsort(key, kind="stable")]
    n = len(xs) // 64
    c = xs[: n * 64].reshape(n, 64, 2)
    return np.sqrt(((c - c.mean(1, keepdims=True)) ** 2).sum(2).max(1))


def test_hilbert_curve_is_continuous():
    """Consecutive cells of a 256 x 256 sub-grid along the curve are neighbours."""
    i, j = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    q = np.stack([i.ravel() << 8, j.ravel() << 8], 1).astype(np.int64)
    d = hilbert(q)
    assert len(np.unique(d)) == len(d)
    o = np.argsort(d)
    assert (np.abs(np.diff(i.ravel()[o])) + np.abs(np.diff(j.ravel()[o]))).max() == 1


def test_hilbert_chunks_are_more_compact_than_morton():
    from paper_1010_2475_amd import workloads as wl
    w = wl.dilute_multi(N=16384, M=4)
    q = grid16(w.x)
    rh = chunk_radii(w.x, hilbert(q)).mean()
    rm = chunk_radii(w.x, morton(q)).mean()
    print("mean chunk radius: Hilbert %.1f, Morton %.1f (mean spacing 2)" % (rh, rm))
    assert rh < 0.7 * rm

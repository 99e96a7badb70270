"""The flip kernels find a local root's cell inside the thread's tile from
the cell offset dc = dz L^2 + dy L + dx between the root's cell and the
thread's own (|dx| < TX, |dy| < TY, |dz| < TZ), by two float32 roundings:
dz = rint(dc * (1/L^2)), then dy = rint((dc - dz L^2) * (1/L)), and
dx = the rest (TileIdx::local_key_near).  This is only claimed for L at
least twice the largest tile edge; the test replays the float32 arithmetic
for every tile shape and every such L up to the largest lattice (406) and
every offset, and also shows that the claim fails below that bound."""
import numpy as np

SHAPES = [(8, 8, 4), (8, 4, 4), (4, 4, 4), (8, 8, 8), (16, 8, 8)]
L_MAX = 406


def decode(dc, L):
    inv_LL = np.float32(1.0) / np.float32(L * L)
    inv_L = np.float32(1.0) / np.float32(L)
    dz = np.rint(dc.astype(np.float32) * inv_LL).astype(np.int64)
    r1 = dc - dz * L * L
    dy = np.rint(r1.astype(np.float32) * inv_L).astype(np.int64)
    dx = r1 - dy * L
    return dz, dy, dx


def offsets(tx, ty, tz):
    dx, dy, dz = np.meshgrid(np.arange(-tx + 1, tx), np.arange(-ty + 1, ty), np.arange(-tz + 1, tz), indexing="ij")
    return dx.ravel(), dy.ravel(), dz.ravel()


def test_rounding_decode_exact_from_twice_the_tile_edge():
    for tx, ty, tz in SHAPES:
        dx, dy, dz = offsets(tx, ty, tz)
        for L in range(2 * max(tx, ty, tz), L_MAX + 1):
            dc = dz * L * L + dy * L + dx
            gz, gy, gx = decode(dc, L)
            assert np.array_equal(gz, dz) and np.array_equal(gy, dy) and np.array_equal(gx, dx), (tx, ty, tz, L)


def test_rounding_decode_fails_below_the_bound():
    """At L = tile edge the offsets are ambiguous (dx = L - 1 and dx = -1 of
    the next row give the same dc): the bound is needed."""
    tx, ty, tz = 8, 8, 8
    dx, dy, dz = offsets(tx, ty, tz)
    L = 8
    gz, gy, gx = decode(dz * L * L + dy * L + dx, L)
    assert not (np.array_equal(gz, dz) and np.array_equal(gy, dy) and np.array_equal(gx, dx))

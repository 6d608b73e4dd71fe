"""Host-side check of the candidate-row bound of the tile gathers.

A tile kernel lists the cell-list rows (a run of x bins at one (y, z) bin, at most two
runs per row when the x range crosses the periodic seam) of every ion that can reach its
nodes; the rows go to a fixed LDS buffer of MAXR entries.  This test counts the rows the
way the kernels do, for every tile start of grids up to 64 cells across and every tile,
halo and kernel-width configuration built, and checks the count against the buffer sizes
(the kernels also check the same bound at compile time and raise a sticky capacity flag
if it were ever exceeded at run time)."""
import itertools

import pytest

BIN = 2


def floordiv(a, b):
    return a // b


def rows(nx, ny, nz, x0, y0, z0, tx, ty, tz, hlo, hhi):
    nbx, nby = nx // BIN, ny // BIN
    lo, hi = floordiv(x0 - hlo, BIN), floordiv(x0 + tx - 1 + hhi, BIN)
    if hi - lo + 1 >= nbx:
        nseg = 1
    else:
        nseg = 1 if lo % nbx <= hi % nbx else 2
    ylo, yhi = floordiv(y0 - hlo, BIN), floordiv(y0 + ty - 1 + hhi, BIN)
    if yhi - ylo + 1 >= nby:
        ylo, yhi = 0, nby - 1
    czlo, czhi = max(z0 - hlo, 0), min(z0 + tz - 1 + hhi, nz - 1)
    nzb = max(czhi // BIN - czlo // BIN + 1, 0)
    return nzb * (yhi - ylo + 1) * nseg


def bound(ty, tz, hlo, hhi):
    nb = lambda t: (t - 1 + hhi) // BIN + (hlo + BIN - 1) // BIN + 1
    return 2 * nb(ty) * nb(tz)


# (name, tile edge in x and y, tile depth in z, z depth passed, halo below, halo above, MAXR)
CONFIGS = [
    ("charge spread 16^3", 16, 16, 16, 2, 2, 256),
    ("charge spread 8^3 (batch)", 8, 8, 8, 2, 2, 256),
    ("adjoint transposed gather 16x16x8", 16, 8, 8, 2, 2, 256),
    ("face spread, Peskin, with RFD", 16, 16, 16, 3, 2, 256),
    ("face spread, Peskin, no RFD", 16, 16, 16, 2, 2, 256),
    ("face spread, windows of 4 nodes, with RFD", 16, 16, 16, 3, 2, 256),
    ("face spread, windows of 8 nodes, with RFD", 16, 16, 16, 5, 4, 512),
    ("face spread, windows of 8 nodes, no RFD", 16, 16, 16, 4, 4, 512),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_tile_rows_fit_the_buffer(cfg):
    _, T, TZ, tzp, hlo, hhi, maxr = cfg
    assert bound(T, tzp, hlo, hhi) <= maxr
    worst = 0
    for nx, ny, nz in itertools.product((8, 16, 32, 64), (8, 16, 64), (8, 9, 17, 40)):
        tx, ty = min(T, nx), min(T, ny)
        for x0 in range(0, nx, tx):
            for y0 in range(0, ny, ty):
                for z0 in range(0, nz + 1, TZ):
                    # the z-face grid has nz + 1 levels; the kernels pass at most
                    # min(tz, nz - z0 + 1) levels of node depth
                    tz = min(tzp, nz + 1 - z0, nz - z0 + 1)
                    if tz <= 0:
                        continue
                    r = rows(nx, ny, nz, x0, y0, z0, tx, ty, tz, hlo, hhi)
                    assert r <= bound(T, tzp, hlo, hhi), (nx, ny, nz, x0, y0, z0, r)
                    worst = max(worst, r)
    assert worst <= maxr

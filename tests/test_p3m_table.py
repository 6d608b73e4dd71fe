"""The near-field pair-force table (F^P of eq LC, Sec. II.B.1) from two independent
builders: the library's host builder (discos_p3m_table, C++ with its own FFT) and the
oracle's tool, which wrote the committed table.  Both take the same seeded placements;
they must agree to rounding.  Host computation only (no GPU work)."""
import numpy as np
import pytest

from paper_2204_14167_amd import workloads


def _lib():
    from paper_2204_14167_amd import discos
    return discos


def test_library_table_matches_the_committed_table():
    discos = _lib()
    src, dirs = workloads.p3m_placements()
    g, dr = discos.p3m_table(workloads.P3M_BOX, workloads.P3M_DRHO, src, dirs)
    ref, rdr = workloads.load_p3m_table()
    assert dr == rdr and g.shape == ref.shape
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    # the Coulomb limit: g(rho) rho^2 -> 1 far from the kernel's support
    k = int(round(4.0 / dr))
    assert abs(g[k] * 16.0 - 1.0) < 1e-3


def test_library_table_rejects_bad_arguments():
    discos = _lib()
    src = np.zeros((2, 3))
    dirs = np.ones((2, 3, 5))
    for n in (7, 12, 512):
        with pytest.raises(discos.DiscosError):
            discos.p3m_table(n, 0.25, src, dirs)
    with pytest.raises(discos.DiscosError):
        discos.p3m_table(16, 0.0, src, dirs)
    with pytest.raises(ValueError):
        discos.p3m_table(16, 0.25, src, np.ones((3, 3, 5)))


def test_oracle_tool_reproduces_the_committed_table():
    """The committed table is exactly what the oracle's tool writes from the seeded
    placements (bitwise)."""
    from oracle import make_tables
    rho, g = make_tables.p3m_table()
    ref, dr = workloads.load_p3m_table()
    assert dr == make_tables.DRHO
    assert np.array_equal(rho, np.arange(len(ref)) * dr)
    assert np.array_equal(g, ref)

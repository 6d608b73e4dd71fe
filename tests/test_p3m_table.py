"""The near-field pair-force table (F^P of eq LC, Sec. II.B.1) is a stored input of
the method that both sides read.  The committed file is exactly what the oracle's
offline tool writes from the seeded placements, and it has the Coulomb limit the
paper's construction implies.  Host computation only (no GPU work)."""
import numpy as np

import workloads


def test_oracle_tool_reproduces_the_committed_table():
    """The committed table is exactly what the oracle's tool writes from the seeded
    placements (bitwise)."""
    from oracle import make_tables
    rho, g = make_tables.p3m_table()
    ref, dr = workloads.load_p3m_table()
    assert dr == make_tables.DRHO
    assert np.array_equal(rho, np.arange(len(ref)) * dr)
    assert np.array_equal(g, ref)


def test_committed_table_limits():
    """g(0) = 0 by symmetry, and g(rho) rho^2 -> 1 once the kernels of the two charges
    stop overlapping (4 cells apart and beyond)."""
    g, dr = workloads.load_p3m_table()
    assert g[0] == 0.0
    for rho in (4.0, 5.0, 6.0):
        k = int(round(rho / dr))
        assert abs(g[k] * rho * rho - 1.0) < 2e-3, (rho, g[k] * rho * rho)

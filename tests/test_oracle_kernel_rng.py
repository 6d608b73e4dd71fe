"""Pins of the oracle's kernel and random-number generator (CPU only).

The Peskin kernel is pinned by the moment conditions it was built from
(App. B, eq peskin1d: partition of unity, zero first moment, even/odd sums 1/2,
sum of squares 3/8) and by its values at the nodes; Philox4x32-10 by the
known-answer vectors published with its definition (Salmon et al., SC'11).
"""
import numpy as np
import pytest

from oracle.peskin import node_weights, phi_pe
from oracle.rng import ion_normals, normal_pair, philox4x32_10

pytestmark = pytest.mark.filterwarnings("ignore")


def test_peskin_node_values():
    assert phi_pe(np.array([0.0]))[0] == 0.5
    assert phi_pe(np.array([1.0]))[0] == 0.25
    assert phi_pe(np.array([-1.0]))[0] == 0.25
    assert phi_pe(np.array([2.0]))[0] == 0.0
    assert phi_pe(np.array([2.5]))[0] == 0.0
    # continuity across the branch boundary r = 1
    e = 1e-9
    assert abs(phi_pe(np.array([1.0 - e]))[0] - phi_pe(np.array([1.0 + e]))[0]) < 1e-8


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_peskin_moments(seed):
    zeta = np.random.default_rng(seed).uniform(-0.5, 0.5, 1000)
    j = np.arange(-4, 5)
    w = phi_pe(zeta[:, None] - j[None, :])
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=4e-16)
    np.testing.assert_allclose((w * (zeta[:, None] - j)).sum(axis=1), 0.0, atol=1e-15)
    np.testing.assert_allclose(w[:, j % 2 == 0].sum(axis=1), 0.5, atol=4e-16)
    np.testing.assert_allclose(w[:, j % 2 == 1].sum(axis=1), 0.5, atol=4e-16)
    np.testing.assert_allclose((w * w).sum(axis=1), 3.0 / 8.0, atol=1e-15)


def test_node_weights_cover_support():
    x = np.random.default_rng(3).uniform(0, 16, 500)
    for off in (0.0, 0.5):
        n, w = node_weights(x, 1.0, off)
        np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=4e-16)
        assert np.all((w == 0).sum(axis=1) >= 1)
        # weight of node n is phi(x - (n + off))
        np.testing.assert_array_equal(w, phi_pe(x[:, None] - (n + off)))


def test_philox_known_answers():
    f = 0xFFFFFFFF
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((f, f, f, f), (f, f), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, expect in cases:
        out = philox4x32_10(*ctr, *key)
        assert tuple(int(v) for v in out) == expect


def test_normals_statistics():
    ids = np.arange(200_000)
    a, b = normal_pair(1234, 7, 1, 0, ids)
    for v in (a, b):
        assert abs(v.mean()) < 0.01
        assert abs(v.var() - 1.0) < 0.01
        assert abs(((v ** 4).mean()) - 3.0) < 0.05
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01
    w = ion_normals(1234, 7, 1, ids[:1000])
    assert w.shape == (3, 1000)
    np.testing.assert_array_equal(w[0], a[:1000])
    # distinct steps and tags give independent streams
    c, _ = normal_pair(1234, 8, 1, 0, ids)
    d, _ = normal_pair(1234, 7, 2, 0, ids)
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.01
    assert abs(np.corrcoef(a, d)[0, 1]) < 0.01

"""Pins of the oracle's solid harmonics and expansions: the Legendre
addition theorem, geometric convergence of truncated multipole and local
expansions to the direct sum (Section 2.3: ME valid far from the cluster,
LE valid inside a sub-domain), and the packing layout."""
import numpy as np
import pytest

from oracle import harmonics as H


def test_addition_theorem():
    rng = np.random.default_rng(1)
    y = rng.normal(size=(6, 3)) * 0.25
    x = rng.normal(size=(6, 3))
    x *= (2.0 / np.linalg.norm(x, axis=1))[:, None]
    tot = np.zeros(6, complex)
    for n in range(45):
        for m in range(-n, n + 1):
            tot += np.conj(H.R(n, m, y)) * H.I(n, m, x)
    np.testing.assert_allclose(tot.real, 1.0 / np.linalg.norm(x - y, axis=1), rtol=1e-13)
    assert np.abs(tot.imag).max() < 1e-13


def test_special_values():
    r = np.array([[0.3, -0.2, 0.5]])
    assert H.R(0, 0, r)[0] == pytest.approx(1.0)
    assert H.R(1, 0, r)[0] == pytest.approx(0.5)          # z
    # R_1^1 = -(x + i y)/2 with the Condon-Shortley phase
    assert H.R(1, 1, r)[0] == pytest.approx(-(0.3 - 0.2j) / 2)
    rr = np.linalg.norm(r)
    assert H.I(0, 0, r)[0] == pytest.approx(1.0 / rr)
    assert H.I(1, 0, r)[0] == pytest.approx(0.5 / rr ** 3)  # z / r^3


@pytest.mark.parametrize("p", [4, 8, 10])
def test_me_and_le_converge(p):
    rng = np.random.default_rng(2)
    s = 1.0
    X = np.array([0.1, 0.2, -0.3])
    y = X + rng.uniform(-0.5, 0.5, size=(30, 3)) * s
    w = rng.normal(size=30)
    tgt = X + np.array([[4.0, 0.5, 0.2], [0.0, -3.5, 1.0]])
    direct = (w[None, :] / np.linalg.norm(tgt[:, None, :] - y[None, :, :], axis=2)).sum(axis=1)
    me = H.p2m(y, w, X, s, p)
    err_me = np.abs(H.eval_me(me, X, s, p, tgt) - direct).max() / np.abs(direct).max()
    # local expansion about a far centre, evaluated near it
    Xt = X + np.array([4.0, 0.0, 0.0])
    xt = Xt + rng.uniform(-0.5, 0.5, size=(5, 3))
    direct_t = (w[None, :] / np.linalg.norm(xt[:, None, :] - y[None, :, :], axis=2)).sum(axis=1)
    le = H.p2l(y, w, Xt, s, p)
    err_le = np.abs(H.eval_le(le, Xt, s, p, xt) - direct_t).max() / np.abs(direct_t).max()
    bound = 3.0 * (np.sqrt(3) / 2 / 3.5) ** p
    assert err_me < bound and err_le < bound


def test_pack_roundtrip():
    rng = np.random.default_rng(3)
    p = 6
    v = rng.normal(size=p * p)
    c = H.unpack(v, p)
    np.testing.assert_array_equal(H.pack({k: c[k] for k in c if k[1] >= 0}, p), v)
    assert H.index(3, 0) == 9 and H.index(3, 1, "re") == 10 and H.index(3, 1, "im") == 11
    assert H.index(3, 3, "im") == 15 and H.index(4, 0) == 16

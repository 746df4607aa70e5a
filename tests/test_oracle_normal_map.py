"""Pins of the oracle's normal-mapped heightfield (the normal-mapped glass
panel of the paper's attached validation, Sec. 6.1).

  * a normal map equal to the heights' own central-difference slopes gives
    the very same paths and image as no normal map;
  * the chain rule across the two parameterisations: with that normal map,
    the heights gradient of the plain heightfield equals the normal-map
    run's heights gradient (geometry only) plus the central-difference
    operator's transpose applied to its normal-map gradient;
  * central finite differences of the loss in the normal-map slopes, with
    equal decision signatures at +h and -h;
  * detached passes leave the normal map alone.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_32920_amd import scenes


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _central_slopes(h, G, dx):
    """The slopes the heightfield's shading uses: central differences, one
    sided on the border; returns the map and the linear operator D with
    map = D h."""
    D = np.zeros((G * G * 2, G * G))
    for j in range(G):
        for i in range(G):
            a, b = max(i - 1, 0), min(i + 1, G - 1)
            D[2 * (j * G + i), j * G + b] += 1.0 / ((b - a) * dx)
            D[2 * (j * G + i), j * G + a] -= 1.0 / ((b - a) * dx)
            c, d = max(j - 1, 0), min(j + 1, G - 1)
            D[2 * (j * G + i) + 1, d * G + i] += 1.0 / ((d - c) * dx)
            D[2 * (j * G + i) + 1, c * G + i] -= 1.0 / ((d - c) * dx)
    hh = h.reshape(G, G)
    nm = np.zeros((G, G, 2))
    for j in range(G):
        for i in range(G):
            a, b = max(i - 1, 0), min(i + 1, G - 1)
            nm[j, i, 0] = (hh[j, b] - hh[j, a]) / ((b - a) * dx)
            c, d = max(j - 1, 0), min(j + 1, G - 1)
            nm[j, i, 1] = (hh[d, i] - hh[c, i]) / ((d - c) * dx)
    return nm.reshape(-1), D


def test_central_difference_map_reproduces_the_heightfield():
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    nm, _ = _central_slopes(sc["heights"], 8, sc["hf"]["dx"])
    r0 = O.render(sc, 5, 4096, 4, per_path=True, threads=1)
    r1 = O.render(sc, 5, 4096, 4, per_path=True, normal_map=nm, threads=1)
    assert np.array_equal(r0["sig"], r1["sig"])
    assert np.array_equal(r0["image"], r1["image"])


def test_chain_rule_between_heights_and_normal_map():
    sc = scenes.caustic_scene(G=8, width=32, height=32)
    nm, D = _central_slopes(sc["heights"], 8, sc["hf"]["dx"])
    dI = np.random.default_rng(3).normal(size=(32, 32, 3))
    g0 = O.gradient(sc, 7, 4096, 4, dI, flags=O.ATTACHED)
    g1 = O.gradient(sc, 7, 4096, 4, dI, flags=O.ATTACHED, normal_map=nm)
    assert np.count_nonzero(g1["normal_map"]) > 20
    lhs = g0["heights"]
    rhs = g1["heights"] + D.T @ g1["normal_map"]
    np.testing.assert_allclose(rhs, lhs, rtol=1e-9, atol=1e-9 * np.abs(lhs).max())


def test_finite_differences_normal_map_attached():
    sc = scenes.glass_panel_scene(G=8, width=32, height=32)
    seed, n, D = 5, 4096, 4
    T = O.render(sc, 99, n, D, normal_map=sc["normal_map_target"])["image"]
    r0 = O.render(sc, seed, n, D, per_path=True)
    _, dI = O.loss_and_adjoint(r0["image"], T)
    g = O.gradient(sc, seed, n, D, dI, flags=O.ATTACHED)["normal_map"]
    assert np.count_nonzero(g) > 20
    m0 = sc["normal_map"].copy()
    eps = 1e-7
    checked = 0
    for k in np.argsort(-np.abs(g))[:12]:
        mp, mm = m0.copy(), m0.copy()
        mp[k] += eps
        mm[k] -= eps
        rp = O.render(sc, seed, n, D, normal_map=mp, per_path=True)
        rm = O.render(sc, seed, n, D, normal_map=mm, per_path=True)
        if not (np.array_equal(rp["sig"], r0["sig"]) and np.array_equal(rm["sig"], r0["sig"])):
            continue
        fd = (O.loss_and_adjoint(rp["image"], T)[0] - O.loss_and_adjoint(rm["image"], T)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-5 * np.abs(g).max(), (k, fd, g[k])
        checked += 1
    assert checked >= 8
    # detached: geometry and shading are held fixed
    assert not np.any(O.gradient(sc, seed, n, D, dI)["normal_map"])

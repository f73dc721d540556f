"""Pins of the oracle's general periodic cell (App. A, eq. L-distance_def
with period vectors L_i that need not be orthogonal).

Reading: voxel k of the cell {sum_i alpha_i L_i} is centred at
x_a = sum_i (k_i + 1/2) (L_ia / n_i); the squared distance to a site is the
minimum over integer translations k of the folded squared length of
d_a = (s_a - x_a) + sum_i k_i L_ia.  Pinned against:
- the orthogonal oracle, bit for bit, when the period matrix is diagonal;
- the orthogonal oracle up to rounding after a rotation of the whole problem;
- an independent numpy minimum over a wide box of translations, on sheared,
  hexagonal and strongly skewed cells in 2D, 3D and 4D;
- validation of singular or non-finite period matrices.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2201_13234_amd import inputs as I


def kind_param(rng, kind, ns):
    if kind == O.LAGUERRE:
        return rng.uniform(0, 4, ns)
    if kind == O.JOHNSON_MEHL:
        return rng.uniform(0, 2, ns)
    return None


def voxel_centres(n, P):
    """Cartesian voxel centres [nvox, d] in memory order (axis 0 fastest)."""
    d = len(n)
    idx = np.meshgrid(*[np.arange(v) for v in reversed(n)], indexing="ij")[::-1]
    alpha = [((idx[i] + 0.5) / n[i]).ravel() for i in range(d)]
    return np.stack([sum(alpha[i] * P[i][a] for i in range(d)) for a in range(d)], axis=1)


def numpy_keys(n, P, coords, param, kind, growth, reach):
    d = len(n)
    X = voxel_centres(n, P)
    P = np.asarray(P, dtype=np.float64)
    shifts = np.array(np.meshgrid(*([np.arange(-reach, reach + 1)] * d), indexing="ij")).reshape(d, -1).T
    offs = shifts @ P                                   # [nimg, d] Cartesian translations
    ks = []
    for s in range(len(coords)):
        diff = coords[s][None, None, :] + offs[None, :, :] - X[:, None, :]
        q = (diff ** 2).sum(-1).min(axis=1)
        if kind == O.LAGUERRE:
            q = q - param[s]
        elif kind == O.JOHNSON_MEHL:
            q = param[s] + np.sqrt(q) / growth
        ks.append(q.reshape(tuple(reversed(n))))
    return np.stack(ks)


def check_against(K, lab, keys, rtol=1e-11):
    kmin = K.min(axis=0)
    np.testing.assert_allclose(keys, kmin, rtol=rtol, atol=1e-9)
    picked = np.take_along_axis(K, lab[None].astype(np.int64), 0)[0]
    np.testing.assert_allclose(picked, kmin, rtol=rtol, atol=1e-9)
    agree = lab == K.argmin(axis=0)
    if K.shape[0] > 1:
        srt = np.sort(K, axis=0)
        near_tie = (srt[1] - srt[0]) <= 1e-8 * (1 + np.abs(srt[0]))
    else:
        near_tie = np.zeros_like(agree)
    assert np.all(agree | near_tie)


@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_diagonal_periods_equal_the_orthogonal_reading(kind, d):
    rng = np.random.default_rng(1200 + 10 * d + kind)
    n = {1: (57,), 2: (23, 17), 3: (11, 9, 8), 4: (6, 5, 4, 5)}[d]
    L = [float(v) * float(rng.uniform(0.6, 1.6)) for v in n]
    ns = 25
    coords = I.uniform_sites(rng, ns, L)
    coords[:3] = (np.floor(coords[:3] / (np.array(L) / n)) + 0.5) * (np.array(L) / n)   # on centres
    param = kind_param(rng, kind, ns)
    lab, key = O.brute(O.problem(n, L, kind, True, 0.9), coords, param, want_keys=True)
    P = np.diag(L)
    lab2, key2, _ = O.tessellate(O.problem(n, L, kind, True, 0.9, periods=P), coords, param, want_keys=True)
    np.testing.assert_array_equal(lab2, lab)
    np.testing.assert_array_equal(key2.view(np.int64), key.view(np.int64))


def rotation(d, rng):
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
@pytest.mark.parametrize("d", [2, 3])
def test_rotated_orthogonal_cell(kind, d):
    rng = np.random.default_rng(1300 + 10 * d + kind)
    n = (19, 15) if d == 2 else (9, 8, 7)
    L = [float(v) for v in n]
    ns = 20
    coords = I.uniform_sites(rng, ns, L)
    param = kind_param(rng, kind, ns)
    lab, key = O.brute(O.problem(n, L, kind, True, 1.1), coords, param, want_keys=True)
    R = rotation(d, rng)
    P = (R * np.array(L)).T                 # row i = R e_i L_i
    lab2, key2, _ = O.tessellate(O.problem(n, L, kind, True, 1.1, periods=P), coords @ R.T, param,
                                 want_keys=True)
    np.testing.assert_allclose(key2, key, rtol=1e-11, atol=1e-10)
    K = numpy_keys(n, np.diag(L), coords, param, kind, 1.1, 1)
    check_against(K, lab2, key2)


CELLS = {
    "hex2": [[6.0, 0.0], [3.0, 3.0 * math.sqrt(3.0)]],
    "shear2": [[7.0, 0.0], [5.5, 3.0]],
    "skew2": [[9.0, 0.4], [-2.0, 2.5]],
    "tri3": [[6.0, 0.0, 0.0], [2.0, 5.0, 0.0], [1.5, -1.0, 4.5]],
    "shear4": [[4.0, 0.0, 0.0, 0.0], [1.0, 3.5, 0.0, 0.0], [0.0, 1.2, 3.0, 0.5], [0.7, 0.0, -0.9, 3.2]],
}


@pytest.mark.parametrize("cell", sorted(CELLS))
@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
def test_general_cell_matches_image_sum(cell, kind):
    rng = np.random.default_rng(1400 + kind + 7 * sorted(CELLS).index(cell))
    P = np.array(CELLS[cell])
    d = P.shape[0]
    n = {2: (21, 16), 3: (9, 8, 7), 4: (5, 4, 5, 4)}[d]
    ns = 12
    alpha = rng.random((ns, d)) + rng.integers(-2, 3, (ns, d))       # some sites outside the cell
    coords = alpha @ P
    param = kind_param(rng, kind, ns)
    lab, keys, _ = O.tessellate(O.problem(n, [1.0] * d, kind, True, 0.8, periods=P), coords, param,
                                want_keys=True)
    check_against(numpy_keys(n, P, coords, param, kind, 0.8, 5 if d < 4 else 4), lab, keys)


def test_label_points_general_cell():
    rng = np.random.default_rng(15)
    P = np.array(CELLS["tri3"])
    n = (7, 6, 5)
    coords = rng.random((10, 3)) @ P
    p = O.problem(n, [1.0] * 3, O.VORONOI, True, periods=P)
    full, keys = O.brute(p, coords, want_keys=True)
    vox = np.stack([rng.integers(0, v, 40) for v in n], axis=1)
    lab, k = O.label_points(p, coords, None, vox)
    idx = tuple(vox[:, a] for a in reversed(range(3)))
    np.testing.assert_array_equal(lab, full[idx])
    np.testing.assert_array_equal(k, keys[idx])


def test_general_cell_validation():
    good = np.array([[0.5, 0.5], [1.0, 2.0]])
    P = np.array([[3.0, 0.0], [1.0, 2.0]])
    assert O.validate(O.problem((4, 4), [1, 1], O.VORONOI, True, periods=P), good) == O.OK
    assert O.validate(O.problem((4, 4), [1, 1], O.VORONOI, True, periods=P), good + 100.0) == O.OK
    bad = good.copy()
    bad[1, 1] = np.nan
    assert O.validate(O.problem((4, 4), [1, 1], O.VORONOI, True, periods=P), bad) == O.ERR_INPUT
    for Pbad in ([[1.0, 2.0], [2.0, 4.0]], [[1.0, np.inf], [0.0, 1.0]], [[0.0, 0.0], [0.0, 0.0]]):
        assert O.validate(O.problem((4, 4), [1, 1], O.VORONOI, True, periods=Pbad), good) == O.ERR_INVALID
    p = O.problem((4, 4), [1, 1], O.VORONOI, True, periods=P)
    p.periodic = 0
    assert O.validate(p, good) == O.ERR_INVALID

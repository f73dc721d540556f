"""Pins of the oracle's general-dimension and periodic-coordinate readings.

The paper states the method for any dimension (Sec. 3, problem statement)
and defines the L-periodic distance for points anywhere in space (App. A,
eq. L-distance_def).  The oracle reads q in d dimensions as
d0*d0 + T with T = d1*d1, T + d2*d2, ... (the 2D and 3D forms are its first
cases) and brings a periodic site into the unit cell by an exact fmod.  These
tests pin both readings to things other than the oracle itself:

- embedding: an extra axis of one voxel with every site on its centre adds
  an exact zero to T, so a (d+1)-dimensional problem must reproduce the
  d-dimensional labels and keys bit for bit (the 2D and 3D oracle are pinned
  by the other oracle tests);
- lattice sites in 4D give boxes, with exact squared distances as keys;
- 1D Voronoi labels from sorted sites and exact midpoints (rational
  arithmetic, no distance formula);
- an independent numpy image sum (App. A, eq. d') in 1D, 4D and 5D, and for
  sites several periods outside the cell;
- translation of every site by whole periods (exact on dyadic coordinates)
  and the roll symmetry in 4D;
- the two-step algorithm equals brute force in 1D, 4D, 5D and 6D at any level.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2201_13234_amd import inputs as I


def prob(n, kind=O.VORONOI, periodic=True, growth=1.0, L=None):
    return O.problem(n, L if L is not None else [float(v) for v in n], kind, periodic, growth)


def kind_param(rng, kind, ns):
    if kind == O.LAGUERRE:
        return rng.uniform(0, 6, ns)
    if kind == O.JOHNSON_MEHL:
        return rng.uniform(0, 3, ns)
    return None


def all_taus(p, coords, param):
    rng = np.random.default_rng(len(coords))
    star = O.choose_tau(p, coords, param)
    return [float("nan"), -math.inf, math.inf, star * rng.uniform(0.05, 0.6),
            star * rng.uniform(1.5, 4.0)]


# ------------------------------------------------------------------ embedding

@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_extra_axis_of_one_voxel(kind, periodic, d):
    rng = np.random.default_rng(500 + 10 * d + kind + 3 * periodic)
    n = tuple(int(v) for v in rng.integers(3, 14 if d <= 3 else 6, d))
    L = [float(v) * float(rng.uniform(0.5, 2.0)) for v in n]
    ns = int(rng.integers(1, 30))
    coords = I.uniform_sites(rng, ns, L)
    param = kind_param(rng, kind, ns)
    lab, key = O.brute(O.problem(n, L, kind, periodic, 0.7), coords, param, want_keys=True)
    Le = float(rng.uniform(0.5, 3.0))
    ce = np.concatenate([coords, np.full((ns, 1), 0.5 * Le)], axis=1)   # on the voxel centre
    p1 = O.problem(n + (1,), L + [Le], kind, periodic, 0.7)
    for tau in all_taus(p1, ce, param):
        lab1, key1, _ = O.tessellate(p1, ce, param, tau=tau, want_keys=True)
        np.testing.assert_array_equal(lab1[0], lab)
        np.testing.assert_array_equal(key1[0].view(np.int64), key.view(np.int64))


# -------------------------------------------------------------------- lattice

@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
def test_lattice_gives_boxes_4d(periodic, kind):
    m, c = (2, 3, 2, 2), (3, 2, 3, 4)
    n = tuple(m[a] * c[a] for a in range(4))
    grids = np.meshgrid(*[np.arange(v) for v in m], indexing="ij")        # site index a0 fastest
    centres = np.stack([(g.ravel(order="F") + 0.5) * c[a] for a, g in enumerate(grids)], axis=1)
    ns = len(centres)
    param = None if kind == O.VORONOI else np.full(ns, 1.25)
    p = prob(n, kind, periodic, growth=0.5)
    vi = np.meshgrid(*[np.arange(v) for v in reversed(n)], indexing="ij")[::-1]   # x0 .. x3
    expect = np.zeros(tuple(reversed(n)), dtype=np.int64)
    stride = 1
    for a in range(4):
        expect += (vi[a] // c[a]) * stride
        stride *= m[a]
    for tau in all_taus(p, centres, param):
        lab, keys, _ = O.tessellate(p, centres, param, tau=tau, want_keys=True)
        np.testing.assert_array_equal(lab, expect)
    if kind == O.VORONOI:
        d2 = sum(((vi[a] % c[a]) + 0.5 - 0.5 * c[a]) ** 2 for a in range(4))
        np.testing.assert_array_equal(keys, d2)


# ------------------------------------------------------------ 1D closed form

@pytest.mark.parametrize("periodic", [False, True])
def test_1d_voronoi_from_midpoints(periodic):
    rng = np.random.default_rng(77)
    n = 97
    L = 24.0
    ns = 11
    coords = np.sort(rng.integers(0, 96 * 8, ns)) / 32.0        # dyadic, may repeat
    coords = coords[rng.permutation(ns)]                          # indices not in order
    lab = O.brute(O.problem([n], [L], O.VORONOI, periodic), coords[:, None])
    h = Fraction(L) / n
    for i in range(n):
        x = (i + Fraction(1, 2)) * h
        dist = []
        for s in range(ns):
            d = abs(Fraction(coords[s]) - x)
            if periodic:
                d = min(d, Fraction(L) - d)
            dist.append(d)
        best = min(dist)
        assert lab[i] == dist.index(best), i                      # lowest index on ties


# -------------------------------------------------- independent image sum

def image_sum_keys(n, L, coords, param, kind, periodic, growth, reach=1):
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) * (L[a] / n[a]) for a in range(d)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")[::-1]
    shifts = range(-reach, reach + 1) if periodic else (0,)
    images = np.array(np.meshgrid(*([list(shifts)] * d), indexing="ij")).reshape(d, -1).T
    ks = []
    for s in range(len(coords)):
        best = None
        for img in images:
            q = sum((coords[s, a] + img[a] * L[a] - grids[a]) ** 2 for a in range(d))
            best = q if best is None else np.minimum(best, q)
        if kind == O.LAGUERRE:
            best = best - param[s]
        elif kind == O.JOHNSON_MEHL:
            best = param[s] + np.sqrt(best) / growth
        ks.append(best)
    return np.stack(ks)


def check_against(K, lab, keys):
    kmin = K.min(axis=0)
    np.testing.assert_allclose(keys, kmin, rtol=1e-11, atol=1e-9)
    picked = np.take_along_axis(K, lab[None].astype(np.int64), 0)[0]
    np.testing.assert_allclose(picked, kmin, rtol=1e-11, atol=1e-9)
    agree = lab == K.argmin(axis=0)
    if K.shape[0] > 1:
        srt = np.sort(K, axis=0)
        near_tie = (srt[1] - srt[0]) <= 1e-9 * (1 + np.abs(srt[0]))
    else:
        near_tie = np.zeros_like(agree)
    assert np.all(agree | near_tie)


@pytest.mark.parametrize("seed", range(9))
def test_matches_image_sum_in_other_dimensions(seed):
    rng = np.random.default_rng(600 + seed)
    d = (1, 4, 5)[seed % 3]
    n = tuple(int(v) for v in rng.integers(2, 40 if d == 1 else 6, d))
    L = [float(v) * float(rng.uniform(0.6, 1.7)) for v in n]
    kind = (seed // 3) % 3
    periodic = seed % 2 == 0
    ns = int(rng.integers(1, 16))
    coords = I.uniform_sites(rng, ns, L)
    param = kind_param(rng, kind, ns)
    lab, keys, _ = O.tessellate(O.problem(n, L, kind, periodic, 0.8), coords, param, want_keys=True)
    check_against(image_sum_keys(n, L, coords, param, kind, periodic, 0.8), lab, keys)


@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
@pytest.mark.parametrize("d", [2, 3])
def test_sites_outside_the_cell_match_image_sum(kind, d):
    rng = np.random.default_rng(700 + kind + 5 * d)
    n = (23, 17) if d == 2 else (11, 9, 8)
    L = [float(v) * 0.9 for v in n]
    ns = 14
    coords = I.uniform_sites(rng, ns, L) + rng.integers(-3, 4, (ns, d)) * np.array(L)
    coords[0, 0] = -1e-300            # rounds onto the cell origin
    param = kind_param(rng, kind, ns)
    lab, keys, _ = O.tessellate(O.problem(n, L, kind, True, 1.3), coords, param, want_keys=True)
    check_against(image_sum_keys(n, L, coords, param, kind, True, 1.3, reach=4), lab, keys)


# ------------------------------------------------------- whole-period shifts

@pytest.mark.parametrize("kind", [O.VORONOI, O.LAGUERRE, O.JOHNSON_MEHL])
@pytest.mark.parametrize("d", [1, 3, 4])
def test_whole_period_shift_changes_nothing(kind, d):
    rng = np.random.default_rng(800 + kind + 7 * d)
    n = {1: (37,), 3: (9, 8, 7), 4: (5, 4, 6, 3)}[d]
    L = [float(v) for v in n]
    ns = 12
    coords = np.stack([rng.integers(0, v * 256, ns) / 256.0 for v in n], axis=1)
    param = kind_param(rng, kind, ns)
    p = O.problem(n, L, kind, True, 0.9)
    base, bkeys, _ = O.tessellate(p, coords, param, want_keys=True)
    for k in range(3):
        shift = rng.integers(-5, 6, (ns, d)) * np.array(L)     # exact on these coordinates
        lab, keys, _ = O.tessellate(p, coords + shift, param, want_keys=True)
        np.testing.assert_array_equal(lab, base)
        np.testing.assert_array_equal(keys.view(np.int64), bkeys.view(np.int64))


def test_negative_zero_and_tiny_coordinates():
    # cell reading: fmod keeps -1e-300 below 0, the sum -1e-300 + L rounds to
    # L, which is the origin of the next period; -0.0 is the origin itself.
    n, L = (16, 12), [16.0, 12.0]
    base = np.array([[0.0, 3.25], [7.5, 0.0], [12.0, 9.0]])
    p = O.problem(n, L, O.VORONOI, True)
    ref = O.brute(p, base)
    for v in (-1e-300, -0.0, 16.0, -16.0, 32.0):
        c = base.copy()
        c[0, 0] = v
        np.testing.assert_array_equal(O.brute(p, c), ref)
    c = base.copy()
    c[0, 0] = -0.25                      # exactly 15.75
    c2 = base.copy()
    c2[0, 0] = 15.75
    np.testing.assert_array_equal(O.brute(p, c), O.brute(p, c2))


@pytest.mark.parametrize("kind", [O.VORONOI, O.JOHNSON_MEHL])
def test_roll_symmetry_4d(kind):
    rng = np.random.default_rng(900 + kind)
    n = (6, 5, 4, 5)
    ns = 15
    coords = np.stack([rng.integers(0, v * 512, ns) / 512.0 for v in n], axis=1)
    param = kind_param(rng, kind, ns)
    p = prob(n, kind, True)
    base, _, _ = O.tessellate(p, coords, param)
    for k in ((1, 0, 0, 0), (0, 2, 0, 3), (5, 4, 3, 2)):
        shifted = np.stack([(coords[:, a] + k[a]) % n[a] for a in range(4)], axis=1)
        lab, _, _ = O.tessellate(p, shifted, param)
        np.testing.assert_array_equal(lab, np.roll(base, shift=tuple(reversed(k)), axis=(0, 1, 2, 3)))


# ------------------------------------------- two steps equal brute force

@pytest.mark.parametrize("seed", range(12))
def test_two_step_equals_brute_force_nd(seed):
    rng = np.random.default_rng(1000 + seed)
    d = (1, 4, 5, 6)[seed % 4]
    top = {1: 200, 4: 7, 5: 5, 6: 4}[d]
    n = tuple(int(v) for v in rng.integers(1, top, d))
    L = [float(v) * float(rng.uniform(0.5, 2.0)) for v in n]
    kind = (seed // 4) % 3
    periodic = seed % 2 == 0
    ns = int(rng.integers(1, 40))
    coords = I.uniform_sites(rng, ns, L)
    if seed % 3 == 0:      # sites on voxel centres and duplicates
        h = np.array(L) / np.array(n)
        coords[: ns // 2] = (np.floor(coords[: ns // 2] / h) + 0.5) * h
        coords[-1] = coords[0]
    if periodic:
        coords = coords + rng.integers(-2, 3, coords.shape) * np.array(L)
    param = kind_param(rng, kind, ns)
    p = O.problem(n, L, kind, periodic, float(rng.uniform(0.3, 3.0)))
    ref, refk = O.brute(p, coords, param, want_keys=True)
    for tau in all_taus(p, coords, param):
        for threads in (1, 3):
            lab, keys, _ = O.tessellate(p, coords, param, tau=tau, nthreads=threads, want_keys=True)
            np.testing.assert_array_equal(lab, ref, err_msg=f"tau={tau}")
            np.testing.assert_array_equal(keys, refk)


def test_label_points_in_5d():
    rng = np.random.default_rng(5)
    n = (4, 5, 3, 4, 6)
    L = [float(v) for v in n]
    coords = I.uniform_sites(rng, 20, L)
    p = O.problem(n, L, O.VORONOI, True)
    full, keys = O.brute(p, coords, want_keys=True)
    vox = np.stack([rng.integers(0, v, 50) for v in n], axis=1)
    lab, k = O.label_points(p, coords, None, vox)
    idx = tuple(vox[:, a] for a in reversed(range(5)))
    np.testing.assert_array_equal(lab, full[idx])
    np.testing.assert_array_equal(k, keys[idx])

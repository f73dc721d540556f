"""Property tests of the oracle on tiny grids drawn by hypothesis, with
adversarial structure: sites on voxel centres (exact ties), duplicates,
sites on the domain faces, a single site, equal parameters.

- The two-step ball algorithm (Sec. 3.2.2 and 3.3.2) returns exactly the
  brute-force argmin (the definition, Sec. 2) at any level tau: its
  second step covers every voxel the first leaves open.
- Brute force agrees with an independent numpy evaluation of the keys that
  takes the periodic distance as a minimum over images (App. A) instead of
  the conditional wrap, up to rounding of the two formulas.
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle as O
from test_oracle_pins import numpy_keys


@st.composite
def problems(draw, max_side=10, max_sites=30):
    d = draw(st.sampled_from([2, 3]))
    n = tuple(draw(st.integers(1, max_side if d == 3 else 3 * max_side)) for _ in range(d))
    kind = draw(st.integers(0, 2))
    periodic = draw(st.booleans())
    ns = draw(st.integers(1, max_sites))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    mode = draw(st.sampled_from(["uniform", "centres", "duplicates", "faces", "mixed"]))
    rng = np.random.default_rng(seed)
    L = np.array([float(v) for v in n])
    coords = rng.uniform(0.0, 1.0, (ns, d)) * L
    if mode == "centres":          # every site on a voxel centre: many exact ties
        coords = np.floor(coords) + 0.5
    elif mode == "duplicates":     # repeated sites: the lowest index must win
        coords = coords[rng.integers(0, max(1, ns // 3), ns)]
    elif mode == "faces":          # sites on the faces at 0 (inside [0, L))
        coords[:, rng.integers(0, d)] = 0.0
    elif mode == "mixed":
        k = ns // 2
        coords[:k] = np.floor(coords[:k]) + 0.5
    param = None
    if kind == O.LAGUERRE:
        param = (rng.uniform(-4.0, 9.0, ns) if draw(st.booleans())
                 else np.full(ns, float(draw(st.integers(0, 5)))))
    elif kind == O.JOHNSON_MEHL:
        param = (rng.uniform(0.0, 6.0, ns) if draw(st.booleans())
                 else np.full(ns, 1.5))
    growth = draw(st.sampled_from([1.0, 0.5, 2.0, 0.7]))
    return n, kind, periodic, coords, param, growth


SETTINGS = settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(problems(), st.sampled_from(["star", "-inf", "inf", "small", "large"]))
def test_two_step_equals_brute_force_any_level(prob, level):
    n, kind, periodic, coords, param, growth = prob
    p = O.problem(n, [float(v) for v in n], kind, periodic, growth)
    star = O.choose_tau(p, coords, param)
    tau = {"star": float("nan"), "-inf": -math.inf, "inf": math.inf,
           "small": 0.2 * star, "large": 3.0 * star}[level]
    ref, refk = O.brute(p, coords, param, want_keys=True)
    lab, keys, _ = O.tessellate(p, coords, param, tau=tau, want_keys=True)
    np.testing.assert_array_equal(lab, ref)
    np.testing.assert_array_equal(keys.view(np.int64), refk.view(np.int64))


@SETTINGS
@given(problems(max_side=8, max_sites=12))
def test_brute_force_matches_image_minimum(prob):
    n, kind, periodic, coords, param, growth = prob
    p = O.problem(n, [float(v) for v in n], kind, periodic, growth)
    lab, keys = O.brute(p, coords, param, want_keys=True)
    K = numpy_keys(n, coords, param, kind, periodic, growth)
    kmin = K.min(axis=0)
    np.testing.assert_allclose(keys, kmin, rtol=1e-12, atol=1e-9)
    picked = np.take_along_axis(K, lab[None].astype(np.int64), 0)[0]
    np.testing.assert_allclose(picked, kmin, rtol=1e-12, atol=1e-9)
    # where no other key is within rounding, the label is the unique argmin
    srt = np.sort(K, axis=0)
    clear = (srt[1] - srt[0]) > 1e-9 * (1 + np.abs(srt[0])) if len(coords) > 1 else np.ones(lab.shape, bool)
    assert np.all((lab == K.argmin(axis=0)) | ~clear)

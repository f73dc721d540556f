"""Parity of the general path (vt_tessellate_nd: 1 to 6 axes) and of periodic
sites outside the unit cell with the oracle, voxel by voxel, bit for bit:
labels and the winning keys.

Sizes span several tiles with ragged tails on every axis; the edge cases are
one site, duplicates, sites on voxel centres, axes of one voxel, more sites
than voxels, clusters that overflow one staging round of the kernel, and bad
input.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13234_amd import inputs as I
from gpu_util import describe_mismatch, run_device, run_oracle, to_dev, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2201_13234_amd import vtess
    assert torch.cuda.is_available()
    c = vtess.Context(0)
    yield c
    c.close()


def run_nd(ctx, w, generic=False, keys=True):
    import torch
    job = to_dev(w)
    if keys:
        job.keys = torch.full(tuple(reversed(w.n)), -7.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda:0")
    print(f"[nd] {w.name} n={w.n} ns={len(w.coords)} kind={w.kind} periodic={w.periodic} "
          f"generic={generic}", flush=True)
    ctx.tessellate_nd(job, status=st, generic=generic)
    torch.cuda.synchronize()
    return job.labels.cpu().numpy(), (job.keys.cpu().numpy() if keys else None), int(st.item())


def oracle_keys(w):
    p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
    lab, key, _ = oracle.tessellate(p, w.coords, w.param, want_keys=True)
    return lab, key


def check(ctx, w, generic=False):
    lab_ref, key_ref = oracle_keys(w)
    lab, key, st = run_nd(ctx, w, generic)
    assert st == 0
    assert np.array_equal(lab, lab_ref), f"{w.name}: " + describe_mismatch(lab, lab_ref)
    assert np.array_equal(key.view(np.int64), key_ref.view(np.int64)), f"{w.name}: keys differ"


def random_nd(seed, d, kind=None, periodic=None, outside=False):
    rng = np.random.default_rng(3000 + seed)
    top = {1: 3000, 2: 90, 3: 30, 4: 14, 5: 9, 6: 6}[d]
    n = tuple(int(v) for v in rng.integers(1, top, d))
    if np.prod(n) < 64:
        n = tuple(max(v, 3) for v in n)
    L = tuple(float(v) * float(rng.uniform(0.5, 2.0)) for v in n)
    kind = int(rng.integers(0, 3)) if kind is None else kind
    periodic = bool(rng.integers(0, 2)) if periodic is None else periodic
    ns = int(rng.integers(1, 300))
    coords = I.uniform_sites(rng, ns, L)
    if outside and periodic:
        coords = coords + rng.integers(-3, 4, coords.shape) * np.array(L)
    sp = (np.prod(L) / ns) ** (1.0 / d)
    param = None
    if kind == I.LAGUERRE:
        param = I.lognormal_weights(rng, ns, 0.5 * sp, 0.3)
    elif kind == I.JOHNSON_MEHL:
        param = rng.uniform(0.0, 1.92 * sp, ns)
    growth = float(rng.choice([1.0, 0.5, 0.7, 2.0]))
    return workload(n, kind, periodic, coords, param, growth, L=L, name=f"nd{d}_{seed}")


# ------------------------------------------------------------- other dimensions

@pytest.mark.parametrize("seed", range(24))
def test_nd_random(ctx, seed):
    d = (1, 4, 5, 6)[seed % 4]
    check(ctx, random_nd(seed, d, kind=(seed // 4) % 3, periodic=seed % 8 < 4))


@pytest.mark.parametrize("seed", range(12))
def test_general_kernel_in_2d_and_3d(ctx, seed):
    # the general kernel on 2 and 3 axes must give the tuned path's results
    d = 2 + seed % 2
    w = random_nd(100 + seed, d, kind=(seed // 2) % 3, periodic=seed % 4 < 2)
    check(ctx, w, generic=True)


@pytest.mark.parametrize("d", [2, 3])
def test_nd_entry_routes_2d_3d_to_the_tuned_path(ctx, d):
    w = random_nd(200 + d, d, kind=0, periodic=True)
    lab_ref, key_ref = oracle_keys(w)
    lab, key, st = run_nd(ctx, w, generic=False)
    assert st == 0 and np.array_equal(lab, lab_ref)
    assert np.array_equal(key.view(np.int64), key_ref.view(np.int64))


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_nd_1d_long_line(ctx, kind):
    # 1D: many tiles of 256 voxels, ragged end
    rng = np.random.default_rng(40 + kind)
    n = (200_003,)
    L = (1000.0,)
    ns = 5000
    coords = I.uniform_sites(rng, ns, L)
    param = None if kind == 0 else rng.uniform(0, 0.3, ns)
    check(ctx, workload(n, kind, kind != 1, coords, param, 0.9, L=L, name=f"line{kind}"))


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_nd_4d_several_thousand_sites(ctx, kind):
    rng = np.random.default_rng(50 + kind)
    n = (21, 18, 17, 13)
    L = tuple(float(v) for v in n)
    ns = 4000
    coords = I.uniform_sites(rng, ns, L)
    sp = (np.prod(L) / ns) ** 0.25
    param = None
    if kind == 1:
        param = I.lognormal_weights(rng, ns, 0.5 * sp, 0.3)
    elif kind == 2:
        param = rng.uniform(0, 1.92 * sp, ns)
    check(ctx, workload(n, kind, True, coords, param, 1.0, L=L, name=f"4d{kind}"))


# --------------------------------------------------------------------- edge cases

@pytest.mark.parametrize("d", [1, 4, 6])
def test_nd_single_site(ctx, d):
    n = {1: (77,), 4: (5, 6, 7, 3), 6: (3, 4, 2, 3, 2, 3)}[d]
    w = workload(n, 2, False, np.full((1, d), 0.37), np.array([1.5]), 0.8, name=f"one{d}")
    check(ctx, w)


@pytest.mark.parametrize("d", [1, 4, 5])
def test_nd_duplicates_and_voxel_centres(ctx, d):
    rng = np.random.default_rng(60 + d)
    n = {1: (300,), 4: (9, 8, 7, 6), 5: (6, 5, 7, 4, 5)}[d]
    ns = 120
    idx = np.stack([rng.integers(0, v, ns) for v in n], axis=1)
    coords = idx + 0.5                                   # on voxel centres (L = n)
    coords[ns // 2:] = coords[: ns - ns // 2]            # duplicates: lower index wins
    for periodic in (True, False):
        check(ctx, workload(n, 0, periodic, coords, name=f"dup{d}{periodic}"))


def test_nd_axes_of_one_voxel(ctx):
    rng = np.random.default_rng(7)
    n = (1, 13, 1, 9, 1)
    L = (0.7, 13.0, 2.0, 9.0, 1.0)
    coords = I.uniform_sites(rng, 40, L)
    for kind in (0, 1, 2):
        param = None if kind == 0 else rng.uniform(0, 2, 40)
        check(ctx, workload(n, kind, kind != 2, coords, param, 1.3, L=L, name=f"flat{kind}"))


def test_nd_more_sites_than_voxels(ctx):
    rng = np.random.default_rng(8)
    n = (4, 5, 3, 4)
    L = tuple(float(v) for v in n)
    coords = I.uniform_sites(rng, 2000, L)
    check(ctx, workload(n, 0, True, coords, L=L, name="dense4d"))


@pytest.mark.parametrize("kind", [0, 2])
def test_nd_cluster_overflows_staging(ctx, kind):
    # 3000 sites inside one small region: a tile's candidates exceed one LDS
    # staging round (512) several times over.
    rng = np.random.default_rng(9 + kind)
    n = (12, 12, 10, 10)
    L = tuple(float(v) for v in n)
    coords = 5.0 + rng.random((3000, 4)) * 0.8
    param = None if kind == 0 else rng.uniform(0, 0.01, 3000)
    check(ctx, workload(n, kind, False, coords, param, 1.0, L=L, name=f"cluster{kind}"))


def test_nd_bad_input(ctx):
    rng = np.random.default_rng(10)
    n = (7, 6, 5, 4)
    L = tuple(float(v) for v in n)
    coords = I.uniform_sites(rng, 30, L)
    for periodic, bad in ((False, 7.0), (False, -0.5), (True, np.nan), (True, np.inf)):
        c = coords.copy()
        c[11, 0] = bad
        lab, key, st = run_nd(ctx, workload(n, 0, periodic, c, L=L, name="bad"))
        assert st == 5 and np.all(lab == -1) and np.all(np.isnan(key))
    # a bad parameter
    lab, key, st = run_nd(ctx, workload(n, 1, True, coords, np.where(np.arange(30) == 3, np.nan, 1.0),
                                        L=L, name="badw"))
    assert st == 5 and np.all(lab == -1)


def test_nd_scalar_errors(ctx):
    import torch
    from paper_2201_13234_amd import vtess
    w = random_nd(300, 4, kind=0)
    job = to_dev(w)
    job.n = (3,) * 7
    with pytest.raises(ValueError):
        ctx.tessellate_nd(job)
    job = to_dev(w)
    job.L = (1.0, -1.0, 1.0, 1.0)
    with pytest.raises(vtess.VtError) as e:
        ctx.tessellate_nd(job)
    assert e.value.code == vtess.ERR_INVALID
    torch.cuda.synchronize()


# --------------------------------------------- periodic sites outside the cell

@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_tuned_path_sites_outside_the_cell(ctx, d, kind):
    w = random_nd(400 + 3 * d + kind, d, kind=kind, periodic=True, outside=True)
    w.coords[0, 0] = -1e-300
    lab_ref, key_ref = oracle_keys(w)
    lab, st = run_device(ctx, w, status=True)
    assert st == 0 and np.array_equal(lab, lab_ref), describe_mismatch(lab, lab_ref)
    # the batch path bins with the same kernels
    import torch
    job = to_dev(w)
    job.keys = torch.zeros(tuple(reversed(w.n)), dtype=torch.float64, device="cuda:0")
    ctx.tessellate_batch([job])
    torch.cuda.synchronize()
    assert np.array_equal(job.labels.cpu().numpy(), lab_ref)
    assert np.array_equal(job.keys.cpu().numpy().view(np.int64), key_ref.view(np.int64))


@pytest.mark.parametrize("d", [1, 4, 5])
def test_nd_sites_outside_the_cell(ctx, d):
    for kind in (0, 1, 2):
        check(ctx, random_nd(500 + 3 * d + kind, d, kind=kind, periodic=True, outside=True))


# ------------------------------------------------------ general period vectors

CELLS = {
    "hex2": [[6.0, 0.0], [3.0, 3.0 * np.sqrt(3.0)]],
    "shear2": [[7.0, 0.0], [5.5, 3.0]],
    "skew2": [[9.0, 0.4], [-2.0, 2.5]],
    "tri3": [[6.0, 0.0, 0.0], [2.0, 5.0, 0.0], [1.5, -1.0, 4.5]],
    "shear4": [[4.0, 0.0, 0.0, 0.0], [1.0, 3.5, 0.0, 0.0], [0.0, 1.2, 3.0, 0.5], [0.7, 0.0, -0.9, 3.2]],
}


def lattice_case(cell, kind, seed, far=2, ns=None):
    rng = np.random.default_rng(seed)
    P = np.array(CELLS[cell])
    d = P.shape[0]
    n = {2: (61, 47), 3: (19, 17, 15), 4: (9, 8, 7, 6)}[d]
    ns = ns or {2: 70, 3: 90, 4: 60}[d]
    alpha = rng.random((ns, d)) + rng.integers(-far, far + 1, (ns, d))
    coords = alpha @ P
    vol = abs(np.linalg.det(P))
    sp = (vol / ns) ** (1.0 / d)
    param = None
    if kind == 1:
        param = I.lognormal_weights(rng, ns, 0.5 * sp, 0.3)
    elif kind == 2:
        param = rng.uniform(0.0, 1.92 * sp, ns)
    w = workload(n, kind, True, coords, param, 0.8, L=[1.0] * d, name=f"lat_{cell}_{kind}")
    return w, P


def run_lattice(ctx, w, P):
    import torch
    job = to_dev(w)
    job.periods = P.tolist()
    job.keys = torch.full(tuple(reversed(w.n)), -7.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda:0")
    print(f"[lattice] {w.name} n={w.n} ns={len(w.coords)}", flush=True)
    ctx.tessellate_nd(job, status=st)
    torch.cuda.synchronize()
    return job.labels.cpu().numpy(), job.keys.cpu().numpy(), int(st.item())


def lattice_oracle(w, P):
    p = oracle.problem(w.n, w.L, w.kind, True, w.growth, periods=P)
    return oracle.brute(p, w.coords, w.param, want_keys=True)


@pytest.mark.parametrize("cell", sorted(CELLS))
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_lattice_cells(ctx, cell, kind):
    w, P = lattice_case(cell, kind, 700 + kind + 10 * sorted(CELLS).index(cell))
    lab_ref, key_ref = lattice_oracle(w, P)
    lab, key, st = run_lattice(ctx, w, P)
    assert st == 0
    assert np.array_equal(lab, lab_ref), w.name + ": " + describe_mismatch(lab, lab_ref)
    assert np.array_equal(key.view(np.int64), key_ref.view(np.int64)), w.name + ": keys"


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lattice_diagonal_equals_orthogonal(ctx, d):
    # a diagonal period matrix is the orthogonal cell: same labels and keys
    w = random_nd(800 + d, d, kind=d % 3, periodic=True)
    lab_ref, key_ref = oracle_keys(w)
    lab, key, st = run_lattice(ctx, w, np.diag(w.L))
    assert st == 0 and np.array_equal(lab, lab_ref), describe_mismatch(lab, lab_ref)
    assert np.array_equal(key.view(np.int64), key_ref.view(np.int64))


def test_lattice_sites_far_outside(ctx):
    w, P = lattice_case("tri3", 0, 900, far=40)
    lab_ref, key_ref = lattice_oracle(w, P)
    lab, key, st = run_lattice(ctx, w, P)
    assert st == 0 and np.array_equal(lab, lab_ref), describe_mismatch(lab, lab_ref)
    assert np.array_equal(key.view(np.int64), key_ref.view(np.int64))


@pytest.mark.parametrize("kind", [0, 2])
def test_lattice_larger_sampled(ctx, kind):
    # many tiles: 64^3 voxels of a triclinic cell, 3,000 sites; sampled voxels
    rng = np.random.default_rng(910 + kind)
    P = np.array(CELLS["tri3"]) * 8.0
    n = (64, 64, 64)
    ns = 3000
    coords = rng.random((ns, 3)) @ P
    param = None if kind == 0 else rng.uniform(0, 6.0, ns)
    w = workload(n, kind, True, coords, param, 1.0, L=[1.0] * 3, name=f"lat_big_{kind}")
    lab, key, st = run_lattice(ctx, w, P)
    assert st == 0
    vox = np.stack([rng.integers(0, v, 3000) for v in n], axis=1)
    p = oracle.problem(n, w.L, kind, True, 1.0, periods=P)
    ref, refk = oracle.label_points(p, w.coords, w.param, vox)
    idx = tuple(vox[:, a] for a in reversed(range(3)))
    assert np.array_equal(lab[idx], ref)
    assert np.array_equal(key[idx].view(np.int64), refk.view(np.int64))


@pytest.mark.parametrize("case", ["2d_ragged", "3d_laguerre", "3d_jm", "4d_sampled"])
def test_two_voxels_per_thread(ctx, case):
    """Grids large enough for the general kernel to give each thread two
    voxels along axis 0 (orthogonal periods, 2 to 4 axes, axis 0 at least
    eight thread widths long, 8,192 or more doubled tiles), with ragged tails
    on every axis: labels and keys against the oracle."""
    rng = np.random.default_rng(940 + len(case))
    if case == "2d_ragged":
        w = workload((2007, 2100), 0, True, I.uniform_sites(rng, 20000, [2007.0, 2100.0]), name=case)
    elif case == "3d_laguerre":
        n = (200, 190, 180)
        c = I.uniform_sites(rng, 8000, [float(v) for v in n])
        w = workload(n, 1, False, c, I.lognormal_weights(rng, 8000, 3.0, 0.3), name=case)
    elif case == "3d_jm":
        n = (160, 170, 176)
        c = I.uniform_sites(rng, 5000, [float(v) for v in n])
        w = workload(n, 2, True, c, rng.uniform(0.0, 15.0, 5000), 0.7, name=case)
    else:
        n = (56, 40, 44, 48)
        c = I.uniform_sites(rng, 9000, [float(v) for v in n])
        w = workload(n, 0, True, c, name=case)
        lab, key, st = run_nd(ctx, w)
        assert st == 0
        vox = np.stack([rng.integers(0, v, 20000) for v in n], axis=1)
        vox[:4] = [[55, 39, 43, 47], [54, 0, 0, 0], [0, 39, 43, 47], [7, 20, 30, 40]]  # tails, both halves
        p = oracle.problem(n, w.L, 0, True, 1.0)
        ref, refk = oracle.label_points(p, w.coords, None, vox)
        idx = tuple(vox[:, a] for a in reversed(range(4)))
        assert np.array_equal(lab[idx], ref)
        assert np.array_equal(key[idx].view(np.int64), refk.view(np.int64))
        return
    check(ctx, w, generic=True)


def test_nd_many_bins(ctx):
    # 80,000 sites in 4D: tens of thousands of bins, a multi-block bin scan
    rng = np.random.default_rng(950)
    n = (20, 18, 22, 16)
    w = workload(n, 0, True, I.uniform_sites(rng, 80_000, [float(v) for v in n]), name="nd_many_bins")
    check(ctx, w)


def test_lattice_errors(ctx):
    from paper_2201_13234_amd import vtess
    w, P = lattice_case("hex2", 0, 920)
    job = to_dev(w)
    job.periods = [[1.0, 2.0], [2.0, 4.0]]
    with pytest.raises(vtess.VtError) as e:
        ctx.tessellate_nd(job)
    assert e.value.code == vtess.ERR_INVALID
    w.periodic = False
    job = to_dev(w)
    job.periods = P.tolist()
    with pytest.raises(vtess.VtError) as e:
        ctx.tessellate_nd(job)
    assert e.value.code == vtess.ERR_INVALID
    w.periodic = True
    w.coords = w.coords.copy()
    w.coords[5, 1] = np.nan
    lab, key, st = run_lattice(ctx, w, P)
    assert st == 5 and np.all(lab == -1) and np.all(np.isnan(key))


def test_scale_bounds_on_the_device(ctx):
    """Weights and times beyond 2^200, and site coordinates beyond it with
    period vectors, are bad site data (status 5, labels -1); lengths or growth
    rates outside [2^-200, 2^200] are refused before any launch."""
    import torch
    from paper_2201_13234_amd import vtess
    big = vtess.SCALE_MAX
    rng = np.random.default_rng(77)
    n = (12, 10, 8)
    pts = I.uniform_sites(rng, 20, [float(v) for v in n])
    for kind, ok_val, bad_val in ((1, -big, 2 * big), (2, big, -2 * big)):
        prm = np.zeros(20)
        prm[4] = ok_val
        lab, st = run_device(ctx, workload(n, kind, True, pts, prm), status=True)
        assert st == 0
        ref = run_oracle(workload(n, kind, True, pts, prm))
        assert np.array_equal(lab, ref)
        prm[4] = bad_val
        lab, st = run_device(ctx, workload(n, kind, True, pts, prm), status=True)
        assert st == 5 and np.all(lab == -1)
        # the general path checks the same bound
        lab, key, st = run_nd(ctx, workload(n + (1,), kind, True, np.c_[pts, np.full(20, 0.5)], prm,
                                            name="scale_nd"))
        assert st == 5 and np.all(lab == -1)
    for bad in (dict(L=(2 * big, 10.0, 8.0)), dict(growth=2 * big)):
        w = workload(n, 2, True, pts, np.zeros(20), growth=bad.get("growth", 1.0), L=bad.get("L"))
        with pytest.raises(vtess.VtError) as e:
            ctx.tessellate(to_dev(w))
        assert e.value.code == vtess.ERR_INVALID
    w, P = lattice_case("hex2", 0, 921)
    w.coords = w.coords.copy()
    w.coords[3, 0] = 2 * big
    lab, key, st = run_lattice(ctx, w, P)
    assert st == 5 and np.all(lab == -1)
    torch.cuda.synchronize()

"""Many obstacle boxes (Section V-B's obstacle-count rows of Table III: one
forest described by 150 to 5000 boxes): queries with more than 64 boxes
build a uniform grid of per-cell box lists on the device and check every
point against its cell's boxes only.  Culling never changes a decision, so
trees must equal the oracle's (which tests every box): bit for bit for the
Euclidean cost, tree for tree on decisive runs for the Dubins airplane and
the double integrator.  Also: the batch and no-allocation paths with grids,
boxes far larger than a cell, and the box-count limit."""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1705_02403_amd import gmt


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def forest_roadmap():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    gmt.use_torch_allocator()
    s = I.dubins_samples(0, 5000)
    tab = O.neighbors(s, O.DUBINS, I.DUBINS_RADIUS, I.DUBINS_TURN)
    rm = gmt.gmt_build_neighbors(torch.from_numpy(s).cuda(), gmt.GMT_COST_DUBINS_AIRPLANE, I.DUBINS_RADIUS,
                                 turn_radius=I.DUBINS_TURN)
    yield s, tab, rm
    rm.free()


def goal_of(p):
    return gmt.make_goal(p.goal_center, p.goal_radius, p.pdim)


def tree_equal(res, ref, exact):
    assert res.status == ref.status and res.iters == ref.iters
    np.testing.assert_array_equal(res.parent.cpu().numpy(), ref.parent)
    np.testing.assert_array_equal(res.group_iter.cpu().numpy(), ref.group_iter)
    np.testing.assert_array_equal(res.added_iter.cpu().numpy(), ref.added_iter)
    c = res.cost.cpu().numpy()
    fin = np.isfinite(ref.cost)
    np.testing.assert_array_equal(np.isfinite(c), fin)
    if exact:
        np.testing.assert_array_equal(c[fin], ref.cost[fin])
    else:
        np.testing.assert_allclose(c[fin], ref.cost[fin], rtol=1e-12, atol=0)
    if ref.status == O.OK:
        assert list(res.path) == list(ref.path)


@pytest.mark.parametrize("m,seeds", [(150, (0, 1)), (500, (0, 2)), (1500, (1,)), (5000, (2,))])
def test_forest_resolution_dubins(forest_roadmap, m, seeds):
    s, tab, rm = forest_roadmap
    for seed in seeds:
        p = I.dubins_forest_problem(seed, s, m)
        say("forest m=%d seed %d" % (m, seed))
        ref = O.plan(p, p.r, tab)
        res = gmt.gmt_plan(rm, p.x_init, goal_of(p), p.boxes, p.lam, gmt.make_opts(edge_step=p.step))
        assert O.decisive(ref, O.DUBINS, rel=1e-9, collide_abs=1e-9)
        tree_equal(res, ref, exact=False)
        assert ref.status == O.OK


@pytest.mark.parametrize("dim,n,m,side,seed", [(2, 2000, 600, (0.01, 0.04), 0), (3, 4096, 1000, (0.01, 0.05), 1),
                                               (3, 4096, 8192, (0.005, 0.02), 2)])
def test_many_boxes_euclidean_bit_exact(dim, n, m, side, seed):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    say("euclid %dD n=%d m=%d" % (dim, n, m))
    p = I.geometric_problem(seed, dim, n, m, side[0], side[1], step=0.005 if dim == 2 else 0.002)
    # Theorem 1's radius with the obstacle-free volume (the exact union volume
    # of thousands of boxes is too costly to compute here)
    r = O.radius(dim, 1.0, n)
    rm = gmt.gmt_build_neighbors(torch.from_numpy(p.samples).cuda(), gmt.GMT_COST_EUCLIDEAN, r)
    res = gmt.gmt_plan(rm, p.x_init, goal_of(p), p.boxes, p.lam, gmt.make_opts(edge_step=p.step))
    ref = O.plan(p, r)
    tree_equal(res, ref, exact=True)
    # one workgroup per query (the batch shape) gives the same tree
    out = gmt.gmt_plan_batch([gmt.BatchQuery(rm, p.x_init, goal_of(p), p.boxes, p.lam, p.step)],
                             gmt.make_opts(edge_step=p.step, threads=1024), outputs=True)
    tree_equal(out[0], ref, exact=True)
    rm.free()


def test_many_boxes_double_integrator():
    """300 boxes (the cave rows' count), n = 4096: at least 3 trees compared."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    n = 4096
    r = 1.75 * (16384.0 / n) ** (1.0 / 6.0)
    s = I.di_samples(4, n)
    tab = O.neighbors(s, O.DI, r)
    rm = gmt.gmt_build_neighbors(torch.from_numpy(s).cuda(), gmt.GMT_COST_DOUBLE_INTEGRATOR, r)
    compared = 0
    for seed in range(12):
        p = I.di_problem(300 + seed, s, m=300, smin=0.02, smax=0.08, r=r)
        ref = O.plan(p, r, tab)
        res = gmt.gmt_plan(rm, p.x_init, goal_of(p), p.boxes, p.lam, gmt.make_opts(traj_points=16))
        if O.decisive(ref, O.DI, rel=1e-9, collide_abs=1e-9):
            tree_equal(res, ref, exact=False)
            compared += 1
        else:
            assert res.status == ref.status
        if compared >= 3:
            break
    say("DI m=300: %d trees compared" % compared)
    assert compared >= 3
    rm.free()


def test_grid_paths_agree(forest_roadmap):
    """Large boxes spanning many cells; batch of grid and non-grid queries;
    the no-allocation entry point with a grid: all equal to gmt_plan."""
    s, tab, rm = forest_roadmap
    base = I.dubins_forest_problem(3, s, 500)
    big = I.from_grid(I.to_grid(np.array([[0.3, 0.3, 0.0, 0.7, 0.7, 0.45], [0.0, 0.6, 0.8, 1.0, 0.65, 1.0]])))
    p_big = dataclasses.replace(base, boxes=np.ascontiguousarray(np.vstack([base.boxes, big]).astype(np.float32)))
    ref = O.plan(p_big, p_big.r, tab)
    res = gmt.gmt_plan(rm, p_big.x_init, goal_of(p_big), p_big.boxes, p_big.lam, gmt.make_opts(edge_step=p_big.step))
    if O.decisive(ref, O.DUBINS, rel=1e-9, collide_abs=1e-9):
        tree_equal(res, ref, exact=False)
    else:
        assert res.status == ref.status
    small = I.dubins_problem(5, s)  # 150 trunks, and one with 40 (no grid)
    few = dataclasses.replace(small, boxes=np.ascontiguousarray(small.boxes[:40]))
    qs = [p_big, base, small, few]
    singles = [gmt.gmt_plan(rm, q.x_init, goal_of(q), q.boxes, q.lam, gmt.make_opts(edge_step=q.step)) for q in qs]
    out = gmt.gmt_plan_batch([gmt.BatchQuery(rm, q.x_init, goal_of(q), q.boxes, q.lam, q.step) for q in qs],
                             gmt.make_opts(edge_step=0.005))
    for got, want in zip(out, singles):
        assert got.status == want.status and got.iters == want.iters and list(got.path) == list(want.path)
        assert got.path_cost == want.path_cost
    N1 = s.shape[1] + 1
    dev = torch.device("cuda", 0)
    arrays = (torch.empty(N1, dtype=torch.int32, device=dev), torch.empty(N1, dtype=torch.float64, device=dev),
              torch.empty(N1, dtype=torch.int32, device=dev), torch.empty(N1, dtype=torch.int32, device=dev))
    a = gmt.gmt_plan_noalloc(rm, p_big.x_init, goal_of(p_big), p_big.boxes, p_big.lam,
                             gmt.make_opts(edge_step=p_big.step), *arrays)
    assert a.status == res.status and list(a.path) == list(res.path) and a.path_cost == res.path_cost
    np.testing.assert_array_equal(a.parent.cpu().numpy(), res.parent.cpu().numpy())


def test_box_limit(forest_roadmap):
    s, tab, rm = forest_roadmap
    p = I.dubins_problem(0, s)
    many = np.ascontiguousarray(np.repeat(p.boxes[:1], 8193, axis=0))
    with pytest.raises(gmt.GmtError) as e:
        gmt.gmt_plan(rm, p.x_init, goal_of(p), many, p.lam, gmt.make_opts(edge_step=p.step))
    assert e.value.status == gmt.GMT_EINVAL

"""Full-size parity (6D double integrator, n = 16384, r = 1.75) in the launch
configurations the benchmark times, and host-forced failure paths.

A batch of queries runs with one 1024-thread workgroup per query (state and
costs-to-come in LDS, lanes 8); queries whose oracle run is decisive are
compared tree for tree, and every tree of the batch is checked on sampled
nodes against properties that hold at any size: each sampled node's cost is
its parent's plus the oracle's cost of that edge, the edge passes the
oracle's lazy check, and the parent was added earlier.  Single plans run
with the default and the tuned team shapes."""

import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1705_02403_amd import gmt

N, R = 16384, 1.75


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def world():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    gmt.use_torch_allocator()
    sets = {}
    for ss in (0, 1):
        s = I.di_samples(ss, N)
        rm = gmt.gmt_build_neighbors(torch.from_numpy(s).cuda(), gmt.GMT_COST_DOUBLE_INTEGRATOR, R)
        tab = O.neighbors(s, O.DI, R)
        # the GPU-built table holds exactly the oracle's pairs (costs to 1e-12)
        rp, col, cost, tau = rm.export()
        np.testing.assert_array_equal(rp, tab.row_ptr)
        np.testing.assert_array_equal(col, tab.col)
        np.testing.assert_allclose(cost, tab.cost, rtol=1e-12, atol=0)
        sets[ss] = (s, rm, tab)
    yield sets
    for _, rm, _ in sets.values():
        rm.free()


def goal_of(p):
    return gmt.make_goal(p.goal_center, p.goal_radius, 3)


def check_tree_sampled(p, res, tab, rng, count=150):
    par = res.parent.cpu().numpy()
    cost = res.cost.cpu().numpy()
    ai = res.added_iter.cpu().numpy()
    n = p.n
    in_tree = np.flatnonzero((par >= 0) & (np.arange(n + 1) < n))
    assert np.all(np.isfinite(cost[in_tree]))
    for x in rng.choice(in_tree, size=min(count, in_tree.size), replace=False):
        y = int(par[x])
        src = p.x_init if y == n else p.samples[:, y]
        J, tau = O.di_cost(src, p.samples[:, x])
        assert J < R
        assert abs(cost[x] - (cost[y] + J)) <= 1e-12 * cost[x], (x, y)
        free, _ = O.edge_free(p, y, int(x), tau)
        assert free, (x, y)
        assert ai[y] < ai[x] or y == n


def test_batch_full_size_bench_shape(world):
    say("full-size batch, lanes 8, 1024 threads")
    rng = np.random.default_rng(0)
    probs, qs = [], []
    for k in range(48):
        ss = k % 2
        s, rm, _ = world[ss]
        p = I.di_problem(5_000 + k, s, r=R, sample_seed=ss)
        probs.append(p)
        qs.append(gmt.BatchQuery(rm, p.x_init, goal_of(p), p.boxes, p.lam))
    out = gmt.gmt_plan_batch(qs, gmt.make_opts(traj_points=16, lanes=8, threads=1024), outputs=True)
    compared = tried = 0
    for p, res in zip(probs, out):
        tab = world[p.sample_seed][2]
        if compared < 8:
            ref = O.plan(p, R, tab)
            tried += 1
            assert res.status == ref.status
            if O.decisive(ref, O.DI, rel=1e-9, collide_abs=1e-9):
                fin = np.isfinite(ref.cost)
                np.testing.assert_array_equal(res.parent.cpu().numpy(), ref.parent)
                np.testing.assert_array_equal(res.group_iter.cpu().numpy(), ref.group_iter)
                np.testing.assert_array_equal(res.added_iter.cpu().numpy(), ref.added_iter)
                np.testing.assert_array_equal(np.isfinite(res.cost.cpu().numpy()), fin)
                np.testing.assert_allclose(res.cost.cpu().numpy()[fin], ref.cost[fin], rtol=1e-12, atol=0)
                if ref.status == O.OK:
                    assert list(res.path) == list(ref.path)
                compared += 1
            elif ref.status == O.OK:
                assert abs(res.path_cost - ref.path_cost) <= 1e-5 * ref.path_cost
        if res.status == gmt.GMT_OK:
            check_tree_sampled(p, res, tab, rng)
    say("full-size batch: %d of %d oracle runs compared tree for tree" % (compared, tried))
    assert compared >= 6


@pytest.mark.parametrize("team_wgs,threads,lanes", [(0, 0, 0), (64, 256, 32), (32, 1024, 32)])
def test_single_full_size(world, team_wgs, threads, lanes):
    say("full-size single plan %d x %d, lanes %d" % (team_wgs, threads, lanes))
    s, rm, tab = world[1]
    p = I.di_problem(6_001, s, r=R, sample_seed=1)
    res = gmt.gmt_plan(rm, p.x_init, goal_of(p), p.boxes, p.lam,
                       gmt.make_opts(traj_points=16, team_wgs=team_wgs, threads=threads, lanes=lanes))
    ref = O.plan(p, R, tab)
    assert res.status == ref.status
    if ref.status == O.OK:
        assert abs(res.path_cost - ref.path_cost) <= 1e-12 * ref.path_cost
        check_tree_sampled(p, res, tab, np.random.default_rng(1))


def test_forced_failures(world):
    say("forced failures")
    s, rm, _ = world[0]
    p = I.di_problem(7_000, s, r=R)
    o = gmt.make_opts(traj_points=16)
    # non-finite start
    bad = p.x_init.copy()
    bad[0] = np.nan
    with pytest.raises(gmt.GmtError) as e:
        gmt.gmt_plan(rm, bad, goal_of(p), p.boxes, p.lam, o)
    assert e.value.status == gmt.GMT_EINVAL
    # an allocator that fails: the build reports GMT_ENOMEM and nothing leaks
    @C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
    def no_alloc(nbytes, ctx, stream):
        return None

    @C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
    def no_free(ptr, ctx, stream):
        pass

    a = gmt.gmt_allocator(no_alloc, no_free, None)
    assert gmt.lib().gmt_set_allocator(C.byref(a)) == gmt.GMT_OK
    try:
        with pytest.raises(gmt.GmtError) as e:
            gmt.gmt_build_neighbors(torch.from_numpy(s[:, :1024].copy()).cuda(), gmt.GMT_COST_DOUBLE_INTEGRATOR, 2.5)
        assert e.value.status == gmt.GMT_ENOMEM
    finally:
        gmt.use_torch_allocator()
    # the library still works afterwards
    res = gmt.gmt_plan(rm, p.x_init, goal_of(p), p.boxes, p.lam, o, outputs=False)
    assert res.status in (gmt.GMT_OK, gmt.GMT_NO_PATH)


@pytest.mark.parametrize("kind", ["euclid", "di"])
def test_build_failure_frees_everything(kind):
    """An allocator that fails after k successful allocations: every build
    reports GMT_ENOMEM and returns each buffer it obtained (the live set is
    empty afterwards), for every k until the build succeeds."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    say("build failure paths (%s)" % kind)
    if kind == "euclid":
        s = I.problem_3d(2, n=3000).samples
        ck, r = gmt.GMT_COST_EUCLIDEAN, 0.2
    else:
        s = I.di_samples(5, 1024)
        ck, r = gmt.GMT_COST_DOUBLE_INTEGRATOR, 2.5
    d = torch.from_numpy(s).cuda()
    live, budget = {}, [0]

    @C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
    def counted_alloc(nbytes, ctx, stream):
        if budget[0] <= 0:
            return None
        budget[0] -= 1
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    @C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
    def counted_free(ptr, ctx, stream):
        live.pop(int(ptr))

    a = gmt.gmt_allocator(counted_alloc, counted_free, None)
    assert gmt.lib().gmt_set_allocator(C.byref(a)) == gmt.GMT_OK
    try:
        for k in range(0, 40):
            budget[0] = k
            try:
                rm = gmt.gmt_build_neighbors(d, ck, r)
            except gmt.GmtError as e:
                assert e.status == gmt.GMT_ENOMEM, (k, e.status)
                torch.cuda.synchronize()
                assert not live, (k, len(live))
                continue
            assert rm.nnz > 0
            rm.free()
            torch.cuda.synchronize()
            assert not live
            break
        else:
            raise AssertionError("the build never succeeded")
    finally:
        gmt.use_torch_allocator()

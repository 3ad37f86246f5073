"""Halton sample sets on the GPU (Section V-A: the planner samples the
deterministic, low-dispersion Halton sequence) against the oracle's sets,
bit for bit; plans on Halton roadmaps against the oracle's plans.

Generator cases: 2D/3D/6D, with and without boxes, n = 1, ragged n, a start
index past 1, a second call continuing where the first stopped, n = 0, and a
3D set of 2^20 points (compared whole: the oracle's vectorised path is exact
integer arithmetic pinned to the definition).  Plans: Euclidean trees are
exact on both sides, so parent / group / added iteration / cost / path are
compared bit for bit; the double integrator on a Halton set is compared tree
for tree where the oracle's run is decisive."""

import dataclasses

import numpy as np
import pytest

from oracle import halton as H
from oracle import oracle as O
from paper_1705_02403_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1705_02403_amd import gmt


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    gmt.use_torch_allocator()
    yield
    torch.cuda.synchronize()


def kind_of(dim):
    return gmt.GMT_COST_DOUBLE_INTEGRATOR if dim == 6 else gmt.GMT_COST_EUCLIDEAN


BOX3 = I.from_grid(I.to_grid(np.array([[0.1, 0.1, 0.1, 0.5, 0.6, 0.7], [0.4, 0.0, 0.2, 0.9, 0.3, 0.8]])))
CASES = [(1, 2, None, 1), (2000, 2, "2d", 1), (2001, 2, None, 77), (16384, 3, "3d", 1), (3001, 3, BOX3, 5),
         (1, 6, None, 1), (4096, 6, None, 1), (16384, 6, "di", 1), (5003, 6, BOX3, 1000)]


def boxes_of(spec):
    if spec is None:
        return None
    if isinstance(spec, np.ndarray):
        return spec
    if spec == "2d":
        return I.problem_2d(0).boxes
    if spec == "3d":
        return I.problem_3d(1, n=64).boxes
    return I.di_problem(0, I.di_samples(0, 16)).boxes


@pytest.mark.parametrize("n,dim,spec,first", CASES)
def test_halton_set_bit_exact(n, dim, spec, first):
    say("halton n=%d dim=%d first=%d" % (n, dim, first))
    bx = boxes_of(spec)
    want, k_want = H.halton_samples(n, dim, dim == 6, bx, first)
    got, k_got = gmt.gmt_sample_halton(n, dim, kind_of(dim), first, bx)
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    assert k_got == k_want


def test_halton_continues_and_empty():
    say("halton continuation")
    a, k1 = gmt.gmt_sample_halton(1000, 6, gmt.GMT_COST_DOUBLE_INTEGRATOR, 1, BOX3)
    b, k2 = gmt.gmt_sample_halton(777, 6, gmt.GMT_COST_DOUBLE_INTEGRATOR, k1, BOX3)
    whole, kw = H.halton_samples(1777, 6, True, BOX3)
    np.testing.assert_array_equal(np.concatenate([a.cpu().numpy(), b.cpu().numpy()], axis=1), whole)
    assert k2 == kw
    e, k = gmt.gmt_sample_halton(0, 3, gmt.GMT_COST_EUCLIDEAN, 9)
    assert k == 9 and e.numel() == 0
    for bad in [(10, 3, gmt.GMT_COST_EUCLIDEAN, 0), (10, 6, gmt.GMT_COST_EUCLIDEAN, 1),
                (10, 4, gmt.GMT_COST_DOUBLE_INTEGRATOR, 1), (10, 2, gmt.GMT_COST_EUCLIDEAN, 1 << 31)]:
        with pytest.raises(gmt.GmtError) as ex:
            gmt.gmt_sample_halton(*bad)
        assert ex.value.status == gmt.GMT_EINVAL
    # the index range ends at 2^31 - 1: asking past it is an error, not a wrap
    with pytest.raises(gmt.GmtError) as ex:
        gmt.gmt_sample_halton(100, 2, gmt.GMT_COST_EUCLIDEAN, (1 << 31) - 50)
    assert ex.value.status == gmt.GMT_EINVAL


def test_halton_million_points():
    say("halton 3D n=2^20")
    n = 1 << 20
    want, k_want = H.halton_samples(n, 3)
    got, k_got = gmt.gmt_sample_halton(n, 3, gmt.GMT_COST_EUCLIDEAN)
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    assert k_got == k_want == n + 1


def halton_problem(prob, r_rule="halton"):
    s = H.halton_samples(prob.n, prob.dim, False, prob.boxes)[0]
    p = dataclasses.replace(prob, samples=s)
    mu = O.free_volume(p.pdim, p.boxes)
    r = H.halton_radius(p.dim, mu, p.n) if r_rule == "halton" else O.radius(p.dim, mu, p.n)
    return p, r


def plan_gpu(p, r, samples_dev):
    rm = gmt.gmt_build_neighbors(samples_dev, gmt.GMT_COST_EUCLIDEAN, r)
    res = gmt.gmt_plan(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, p.pdim), p.boxes, p.lam,
                       gmt.make_opts(edge_step=p.step))
    rm.free()
    return res


def compare_exact(res, ref):
    assert res.status == ref.status
    assert res.iters == ref.iters
    np.testing.assert_array_equal(res.parent.cpu().numpy(), ref.parent)
    np.testing.assert_array_equal(res.group_iter.cpu().numpy(), ref.group_iter)
    np.testing.assert_array_equal(res.added_iter.cpu().numpy(), ref.added_iter)
    c = res.cost.cpu().numpy()
    fin = np.isfinite(ref.cost)
    np.testing.assert_array_equal(np.isfinite(c), fin)
    np.testing.assert_array_equal(c[fin], ref.cost[fin])
    if ref.status == O.OK:
        assert list(res.path) == list(ref.path) and res.path_cost == ref.path_cost


@pytest.mark.parametrize("dim,seed,rule", [(2, 0, "halton"), (2, 1, "halton"), (2, 2, "theorem1"),
                                           (3, 0, "halton"), (3, 1, "theorem1")])
def test_plan_on_halton_roadmap_bit_exact(dim, seed, rule):
    """The GPU draws the Halton set rejected from the query's boxes, builds its
    table and plans; the oracle does the same from its own set."""
    say("halton plan %dD seed %d radius %s" % (dim, seed, rule))
    prob = I.problem_2d(seed) if dim == 2 else I.problem_3d(seed)
    p, r = halton_problem(prob, rule)
    dev, _ = gmt.gmt_sample_halton(p.n, dim, gmt.GMT_COST_EUCLIDEAN, 1, p.boxes)
    np.testing.assert_array_equal(dev.cpu().numpy(), p.samples)
    res = plan_gpu(p, r, dev)
    ref = O.plan(p, r)
    compare_exact(res, ref)
    assert ref.status == O.OK


def test_plan_di_on_halton_set():
    """Double integrator on a Halton set of 4096 states (velocity in the unit
    ball), GPU-built table: the table equals the oracle's and at least 6
    trees are compared node for node."""
    n = 4096
    r = 1.75 * (16384.0 / n) ** (1.0 / 6.0)
    s = H.halton_samples(n, 6, True)[0]
    tab = O.neighbors(s, O.DI, r)
    dev, _ = gmt.gmt_sample_halton(n, 6, gmt.GMT_COST_DOUBLE_INTEGRATOR)
    np.testing.assert_array_equal(dev.cpu().numpy(), s)
    rm = gmt.gmt_build_neighbors(dev, gmt.GMT_COST_DOUBLE_INTEGRATOR, r)
    rp, col, cost, _ = rm.export()
    np.testing.assert_array_equal(rp, tab.row_ptr)
    np.testing.assert_array_equal(col, tab.col)
    np.testing.assert_allclose(cost, tab.cost, rtol=1e-12, atol=0)
    compared = tried = 0
    for seed in range(30):
        prob = I.di_problem(200 + seed, s, r=r)
        ref = O.plan(prob, r, tab)
        res = gmt.gmt_plan(rm, prob.x_init, gmt.make_goal(prob.goal_center, prob.goal_radius, 3), prob.boxes,
                           prob.lam, gmt.make_opts(traj_points=16))
        tried += 1
        if O.decisive(ref, O.DI, rel=1e-9, collide_abs=1e-9):
            compare_exact_di(res, ref)
            compared += 1
        else:
            assert res.status == ref.status
            if ref.status == O.OK:
                assert abs(res.path_cost - ref.path_cost) <= 1e-5 * ref.path_cost
        if compared >= 6:
            break
    say("halton DI: %d of %d trees compared" % (compared, tried))
    assert compared >= 6
    rm.free()


def compare_exact_di(res, ref):
    assert res.status == ref.status and res.iters == ref.iters
    np.testing.assert_array_equal(res.parent.cpu().numpy(), ref.parent)
    np.testing.assert_array_equal(res.group_iter.cpu().numpy(), ref.group_iter)
    np.testing.assert_array_equal(res.added_iter.cpu().numpy(), ref.added_iter)
    c = res.cost.cpu().numpy()
    fin = np.isfinite(ref.cost)
    np.testing.assert_array_equal(np.isfinite(c), fin)
    np.testing.assert_allclose(c[fin], ref.cost[fin], rtol=1e-12, atol=0)
    if ref.status == O.OK:
        assert list(res.path) == list(ref.path)

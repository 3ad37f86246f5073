"""Learned sampler on the GPU: the BF16 MFMA GEMM against FP64 products of
the same BF16 operands; one CVAE training step (loss, every gradient tensor,
Adam) and decoding against the FP64 oracle; the output map bit-exact against
the oracle; and training on plain-GMT* paths lowering the loss and the path
cost of the plain planner at equal n."""

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1705_02403_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1705_02403_amd import gmt, radius, sampler as S


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    gmt.use_torch_allocator()
    return torch.device("cuda", 0)


def bf16(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev).to(torch.bfloat16)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    return float(np.dot(a, b) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("ta,tb", [(False, True), (False, False), (True, False), (True, True)])
@pytest.mark.parametrize("M_,N_,K_", [(72, 40, 48), (8, 8, 8), (200, 264, 136), (16, 256, 4096), (130, 16, 256)])
def test_gemm_against_fp64(dev, ta, tb, M_, N_, K_):
    if ta and M_ % 8:
        # a transposed A is read along M in 8-element vectors: M must be a multiple of 8
        with pytest.raises(gmt.GmtError):
            S.gemm_bf16(bf16(np.ones((K_, M_)), dev), bf16(np.ones((K_, N_)), dev), True, False)
        M_ += 8 - M_ % 8
    say("gemm ta=%d tb=%d M=%d N=%d K=%d" % (ta, tb, M_, N_, K_))
    rng = np.random.default_rng(M_ * 7 + N_ * 3 + K_ + 11 * ta + 5 * tb)
    A = rng.normal(size=(K_, M_) if ta else (M_, K_))
    B = rng.normal(size=(N_, K_) if tb else (K_, N_))
    bias = rng.normal(size=N_).astype(np.float32)
    At, Bt = bf16(A, dev), bf16(B, dev)
    a = At.float().cpu().numpy().astype(np.float64)
    b = Bt.float().cpu().numpy().astype(np.float64)
    a = a.T if ta else a
    b = b.T if tb else b
    for relu, use_bias in [(False, False), (True, True)]:
        ref = a @ b + (bias.astype(np.float64) if use_bias else 0.0)
        if relu:
            ref = np.maximum(ref, 0.0)
        Cf, Cb = S.gemm_bf16(At, Bt, ta, tb, torch.from_numpy(bias).to(dev) if use_bias else None, relu,
                             out_f32=True, out_bf16=True)
        cf = Cf.cpu().numpy().astype(np.float64)
        # exact BF16 products, FP32 sums: one rounding per 32-term MFMA step
        # and per bias add, at most (K/32 + 2) u sum|a||b|; twice that allowed
        scale = np.abs(a) @ np.abs(b) + np.abs(bias.astype(np.float64))
        tol = 2.0 * (K_ / 32 + 2) * 2.0 ** -24 * scale
        assert np.all(np.abs(cf - ref) <= tol), np.max(np.abs(cf - ref) / scale)
        cb = Cb.float().cpu().numpy().astype(np.float64)
        assert np.all(np.abs(cb - ref) <= 2.0 ** -8 * np.abs(ref) + tol)


def test_gemm_strided_operand(dev):
    """The decoder's first layer reads the z columns of W1 in place (row
    stride 416): op(B) is an 8-column slice of a wider matrix."""
    say("gemm strided")
    rng = np.random.default_rng(3)
    W = bf16(rng.normal(size=(256, 416)), dev)
    Z = bf16(rng.normal(size=(1000, 8)), dev)
    Cf, _ = S.gemm_bf16(Z, W[:, 0:8], False, True)
    ref = Z.float().cpu().numpy().astype(np.float64) @ W[:, 0:8].float().cpu().numpy().astype(np.float64).T
    assert np.max(np.abs(Cf.cpu().numpy() - ref)) <= 1e-4


def training_case(seed, P=16, W=64):
    rng = np.random.default_rng(seed)
    cond = I.bf16_round(rng.uniform(0, 1, size=(P, 396)))
    targ = I.bf16_round(rng.normal(size=(W, 6)))
    owner = rng.integers(0, P, size=W).astype(np.int32)
    rows = np.arange(W, dtype=np.int32)
    eps = I.normal_draws(seed, W)
    return cond, targ, owner, rows, eps


def tensors(flat):
    return {"%s.%s" % (net, k): v.ravel() for net, d in zip(("enc", "dec"), M.unpack(flat)) for k, v in d.items()}


def test_training_step_gradients_match_oracle(dev):
    say("sampler: gradients vs oracle")
    params = I.sampler_params(3, out_scale=1.0)
    cond, targ, owner, rows, eps = training_case(1)
    w, beta = 1.0, 0.5
    smp = S.Sampler(params)
    smp.set_data(cond, targ, owner)
    loss = torch.zeros(2, dtype=torch.float32, device=dev)
    smp.train_step(rows, torch.from_numpy(eps).to(dev), S.train_opts(lr=0.0, recon_weight=w, kl_weight=beta), loss)
    g = smp.grads().astype(np.float64)
    assert np.array_equal(smp.params(), params)  # lr 0 keeps the parameters
    _, rec, kl, gref = M.cvae_loss(params.astype(np.float64), targ[rows], cond[owner[rows]], eps, w, beta)
    r_gpu, k_gpu = loss.cpu().numpy()
    assert abs(r_gpu - rec) <= 1e-2 * abs(rec) and abs(k_gpu - kl) <= 1e-2 * abs(kl) + 1e-6
    got, ref = tensors(g), tensors(gref)
    for name in ref:
        if np.linalg.norm(ref[name]) == 0.0:
            assert np.all(got[name] == 0.0), name
            continue
        assert rel_l2(got[name], ref[name]) <= 2e-2, (name, rel_l2(got[name], ref[name]))
        assert cosine(got[name], ref[name]) >= 0.999, (name, cosine(got[name], ref[name]))
    smp.close()


def test_adam_step_matches_oracle(dev):
    say("sampler: adam")
    params = I.sampler_params(4, out_scale=1.0)
    cond, targ, owner, rows, eps = training_case(2)
    opts = S.train_opts(lr=1e-2, adam_eps=1.0)  # eps 1: the step is close to linear in the gradient
    smp = S.Sampler(params)
    smp.set_data(cond, targ, owner)
    smp.train_step(rows, torch.from_numpy(eps).to(dev), opts)
    dp = smp.params().astype(np.float64) - params
    _, _, _, gref = M.cvae_loss(params.astype(np.float64), targ[rows], cond[owner[rows]], eps, 1.0, 1.0)
    p1, _, _ = M.adam(params.astype(np.float64), gref, 0.0, 0.0, 1, 1e-2, 0.9, 0.999, 1.0)
    assert rel_l2(dp, p1 - params) <= 3e-2
    smp.close()


def test_decode_matches_oracle(dev):
    say("sampler: decode vs oracle")
    params = I.sampler_params(5, out_scale=1.0)
    s = I.di_samples(0, 256)
    prob = I.di_problem(7, s)
    c = S.condition(prob)
    eps = I.normal_draws(9, 777)
    smp = S.Sampler(params)
    raw = smp.decode(c, torch.from_numpy(eps).to(dev)).cpu().numpy().astype(np.float64)
    ref = M.decode(params.astype(np.float64), c, eps)
    assert rel_l2(raw, ref) <= 2e-2
    smp.close()


@pytest.mark.parametrize("count", [1, 4097])
def test_finish_bit_exact(dev, count):
    say("sampler: finish count=%d" % count)
    prob = I.di_problem(11, I.di_samples(0, 64))
    raw = (I.normal_draws(13, count) * 2.0).astype(np.float32)
    if count > 1:
        raw[5, 2] = np.nan
        raw[6, 3:6] = 1e30
    fb = I.di_samples(17, count)
    out, rej = S.finish(torch.from_numpy(raw).to(dev), prob.boxes, torch.from_numpy(fb).to(dev))
    ref, rej_ref = M.finish(raw.astype(np.float64), prob.boxes, fb)
    assert rej == rej_ref
    assert np.array_equal(out.cpu().numpy(), ref)


def test_generate_is_decode_then_finish(dev):
    say("sampler: generate composition")
    params = I.sampler_params(6, out_scale=1.0)
    prob = I.di_problem(12, I.di_samples(0, 64))
    c = S.condition(prob)
    eps = torch.from_numpy(I.normal_draws(21, 3000)).to(dev)
    fb = torch.from_numpy(I.di_samples(22, 3000)).to(dev)
    smp = S.Sampler(params)
    raw = smp.decode(c, eps)
    a, ra = S.finish(raw, prob.boxes, fb)
    big = torch.zeros((6, 5000), dtype=torch.float32, device=dev)
    rb = smp.generate(c, eps, prob.boxes, fb, big[:, 1000:4000])
    assert ra == rb and torch.equal(big[:, 1000:4000], a)
    assert torch.count_nonzero(big[:, :1000]) == 0 and torch.count_nonzero(big[:, 4000:]) == 0
    smp.close()


def test_learned_half_lowers_path_cost(dev):
    """Train on waypoints of plain GMT* paths (n = 8192) and compare the plain
    planner at n = 2048 with uniform samples against the same n with half of
    the samples from the network: the mean path cost must drop."""
    say("sampler: benefit")
    n_train, n_eval = 8192, 2048
    r_tr = radius.di_radius(n_train)
    opts = gmt.make_opts(traj_points=16)
    samples, rms = {}, {}
    for ss in range(4):
        samples[ss] = I.di_samples(ss, n_train)
        rms[ss] = gmt.gmt_build_neighbors(torch.from_numpy(samples[ss]).to(dev), gmt.GMT_COST_DOUBLE_INTEGRATOR, r_tr)
    probs = [I.di_problem(100_000 + k, samples[k % 4], r=r_tr, sample_seed=k % 4) for k in range(1500)]
    data = S.path_dataset(probs, rms, samples, opts)
    for rm in rms.values():
        rm.free()
    say("  %d/%d training problems solved, %d waypoints" % (data.solved, data.problems, data.targets.shape[0]))
    smp = S.Sampler(I.sampler_params(0))
    hist = S.train(smp, data, steps=800, batch=1024, seed=1, opts=S.train_opts(lr=2e-3, kl_weight=0.5),
                   log_every=100)
    say("  loss %s" % [(s, round(r, 3), round(k, 3)) for s, r, k in hist])
    assert hist[-1][1] < 0.6 * hist[0][1]
    r_ev = radius.di_radius(n_eval)
    costs = {False: [], True: []}
    ok = {False: 0, True: 0}
    for k in range(48):
        p = I.di_problem(900_000 + k, I.di_samples(0, 16), r=r_ev)
        for learned in (False, True):
            x, _ = S.mixed_samples(smp, p, n_eval, seed=k, learned=learned)
            rm = gmt.gmt_build_neighbors(x, gmt.GMT_COST_DOUBLE_INTEGRATOR, r_ev)
            res = gmt.gmt_plan(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam,
                               opts, outputs=False)
            rm.free()
            costs[learned].append(res.path_cost if res.status == gmt.GMT_OK else np.inf)
            ok[learned] += res.status == gmt.GMT_OK
    both = [(a, b) for a, b in zip(costs[False], costs[True]) if np.isfinite(a) and np.isfinite(b)]
    plain = np.mean([a for a, _ in both])
    mixed = np.mean([b for _, b in both])
    say("  solved plain %d learned %d of 48; mean cost plain %.4f learned %.4f over %d"
        % (ok[False], ok[True], plain, mixed, len(both)))
    assert ok[True] >= ok[False] - 2
    assert mixed < plain
    smp.close()

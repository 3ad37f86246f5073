"""Benchmark: GMT* plans/s and single-plan p50/p99 latency on the 6D double
integrator at n = 16384 (40 boxes, lambda 0.5, r = 1.75, 16 trajectory
points), with path costs checked against the FP64 oracle.

A step is one gmt_plan_batch call over --batch queries on resident roadmaps
(8 sample sets of 16384 samples, built once with gmt_build_neighbors before
timing, as the method precomputes its roadmap offline).  Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6  # MI355X vector FP64

# HBM-side bytes per k_plan launch from rocprofv3 counter runs (FETCH_SIZE x 2.00
# and WRITE_SIZE x 1.00, the factors a 1 GiB copy gives; medians of six
# launches), for the kernel sources with this digest, by launch shape (lanes
# per candidate, threads per workgroup); reported only while both match
TRAFFIC = {"sources_sha256": "09142274bfdf39a333cef8ccef16a254ff3fd10b99db7ef9f7df586eb960a60c",
           "batch": 4096,
           "by_shape": {(8, 1024): int((2.0 * 51233252 + 5657746) * 1024),
                        (16, 1024): int((2.0 * 61386686 + 5627096) * 1024),
                        (4, 1024): int((2.0 * 46127507 + 5575959) * 1024)}}
# the same for the Euclidean row kernel k_eu_rows building the 3D table at
# n = 1048576 with tile shape 2 (medians of eight builds)
EU_TRAFFIC = {"sources_sha256": "90ec443b3e4cc5aa71b57d2c8d3f8d52075c01bd93d7903ae2ad93c1174e5a58", "n": 1048576,
              "tile": 2,
              "bytes_per_launch": int((2.0 * 62061.8 + 2966571.0) * 1024)}


def say(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(msg, file=sys.stderr, flush=True)


def kernel_digest(files=("gmt_plan.hpp", "gmt_dev.hpp")):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1705_02403_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--sample-sets", type=int, default=8)
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--latency-warmup", type=int, default=20)
    ap.add_argument("--oracle-checks", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--server-requests", type=int, default=4096)
    ap.add_argument("--server-rate", type=float, default=20000.0)
    ap.add_argument("--server-slots", type=int, default=4)
    ap.add_argument("--server-low-requests", type=int, default=512,
                    help="requests of the low-load server run (0: skip)")
    ap.add_argument("--server-low-rate", type=float, default=500.0)
    ap.add_argument("--server-max-batch", type=int, default=256)
    ap.add_argument("--server-threads", type=int, default=0,
                    help="threads per workgroup for the server's batches (0: library choice)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape instead of tuning it first")
    ap.add_argument("--lanes", type=int, default=0, help="force lanes per candidate (skips tuning)")
    ap.add_argument("--threads", type=int, default=0, help="force threads per workgroup (skips tuning)")
    ap.add_argument("--only-throughput", action="store_true",
                    help="time the batches only (for counter runs): no latency, server, build or oracle sections")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB buffer 5 times (calibrates HBM byte counters)")
    ap.add_argument("--euclid-sizes", default="16384,65536,262144,1048576",
                    help="sample counts of the 3D Euclidean table builds reported (empty: none)")
    ap.add_argument("--mixed-requests", type=int, default=512,
                    help="mixed 2D/3D/6D replanning stream (0: skip)")
    ap.add_argument("--mixed-rate", type=float, default=2000.0)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the learned sampler and its comparison with plain GMT* at n=32768")
    ap.add_argument("--learned-train", type=int, default=100000)
    ap.add_argument("--learned-steps", type=int, default=3000)
    ap.add_argument("--learned-test", type=int, default=200)
    ap.add_argument("--dubins-queries", type=int, default=512)
    ap.add_argument("--dubins-latency", type=int, default=100)
    ap.add_argument("--forest-queries", type=int, default=12)
    ap.add_argument("--halton-queries", type=int, default=8)
    ap.add_argument("--replan-scenarios", type=int, default=64)
    ap.add_argument("--cpu-2d", type=int, default=200, help="single-core oracle latency: 2D problems")
    ap.add_argument("--cpu-3d", type=int, default=200, help="single-core oracle latency: 3D problems")
    ap.add_argument("--cpu-di", type=int, default=200, help="single-core oracle latency: 6D problems")
    ap.add_argument("--cpu-mixed", type=int, default=64,
                    help="oracle throughput over the first requests of the mixed 2D/3D/6D set (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the Dubins, Halton and replanning sections")
    return ap.parse_args()


def plan_bytes(w, in_edge=24):
    """Algorithmic bytes of planning work: 4 B per out-edge walked (index),
    `in_edge` B per in-edge scanned, 16 B per node added, 12 B per open-list
    entry partitioned.  24 B per in-edge is the unit the method must move
    (8 B index + FP32 edge cost, 16 B of node state gathered); the table as
    built stores FP64 edge costs in 12-byte records, 28 B per in-edge."""
    return (4 * w["out_edges"] + in_edge * w["in_edges"] + 16 * w["commits"] + 12 * w["open_entries"])


def euclid_build_bytes(n, dim, edges, per_edge=8):
    """Algorithmic bytes of a Euclidean table: samples read (4 B per
    coordinate), row pointers, and per edge an index plus an FP32 cost (8 B).
    The table as built writes one 8-byte (squared distance, column) record
    per edge, the row pointers and the row lengths (4 B per sample more)."""
    return 4 * dim * n + 4 * (n + 1) + per_edge * edges


def di_build_flops(tested, solved):
    """Algorithmic flops of a double-integrator table: about 150 per pair whose
    arrival-time quartic is solved, 10 per pair the lower bound rejects."""
    return 150 * solved + 10 * (tested - solved)


def learned_report(args, torch, gmt, I):
    """Learned sampler (configuration 5): train on waypoints of plain GMT*
    paths at n=32768, then compare the 50/50 learned mix at n in {1k, 2k, 4k, 8k}
    with plain GMT* at n=32768 on held-out queries."""
    from paper_1705_02403_amd import radius, sampler as S
    dev = torch.device("cuda", 0)
    opts = gmt.make_opts(traj_points=16)
    n_big = 32768
    r_big = radius.di_radius(n_big)
    sets = 8
    samples, rms, build_ms = {}, {}, []
    for ss in range(sets):
        samples[ss] = I.di_samples(ss, n_big)
        d = torch.from_numpy(samples[ss]).to(dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rms[ss] = gmt.gmt_build_neighbors(d, gmt.GMT_COST_DOUBLE_INTEGRATOR, r_big)
        torch.cuda.synchronize()
        build_ms.append((time.perf_counter() - t) * 1e3)
    t = time.perf_counter()
    train_probs = [I.di_problem(1_000_000 + k, samples[k % sets], r=r_big, sample_seed=k % sets)
                   for k in range(args.learned_train)]
    data = S.path_dataset(train_probs, rms, samples, opts)
    data_s = time.perf_counter() - t
    smp = S.Sampler(I.sampler_params(0))
    t = time.perf_counter()
    hist = S.train(smp, data, steps=args.learned_steps, batch=1024, seed=0,
                   opts=S.train_opts(lr=1e-3, kl_weight=0.5), log_every=max(args.learned_steps // 10, 1))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    tests = [I.di_problem(2_000_000 + k, samples[k % sets], r=r_big, sample_seed=k % sets)
             for k in range(args.learned_test)]
    # plain GMT* at n = 32768 gets its own tuned single-plan shape too
    p0 = tests[0]
    tuned_plain = gmt.gmt_autotune([gmt.BatchQuery(rms[p0.sample_seed], p0.x_init,
                                                   gmt.make_goal(p0.goal_center, p0.goal_radius, 3),
                                                   p0.boxes, p0.lam)], opts, single=True, reps=3)
    ref_cost, ref_ms = [], []
    for p in tests:
        res, ms = timed(lambda: gmt.gmt_plan(rms[p.sample_seed], p.x_init,
                                             gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam,
                                             opts, outputs=False))
        ref_cost.append(res.path_cost if res.status == gmt.GMT_OK else np.inf)
        ref_ms.append(ms)
    ref_cost = np.array(ref_cost)
    plain_p50 = float(np.percentile(ref_ms, 50))
    # Sample sets of n < 32768 at three edge rules: the radius rule r(n) with
    # 16 trajectory points (edges grow as n shrinks), the same radius with the
    # trajectory points scaled by r(n) / r(32768) (the checked points stay as
    # dense along an edge as at n = 32768), and plain's own radius r(32768)
    # with 16 points (the same edges as plain; only the samples differ).
    rows, tuned_single = {}, {}
    for n in (1024, 2048, 4096, 8192):
        r_n = radius.di_radius(n)
        k_scaled = int(math.ceil(16.0 * r_n / r_big))
        n_l = n // 2
        # query-independent draws stay resident: `sets` pools, query k uses pool k % sets
        uni = [torch.from_numpy(I.di_samples(7_000 + ss, n - n_l)).to(dev) for ss in range(sets)]
        fb = [torch.from_numpy(I.di_samples(8_000 + ss, n_l)).to(dev) for ss in range(sets)]
        eps = [torch.from_numpy(I.normal_draws(9_000 + ss, n_l)).to(dev) for ss in range(sets)]
        uni_full = [torch.from_numpy(I.di_samples(7_000 + ss, n)).to(dev) for ss in range(sets)]
        rules = (("", r_n, 16), ("_points_scaled", r_n, k_scaled), ("_equal_r", r_big, 16))
        for tag, rr, kp in rules:
            opts_k = gmt.make_opts(traj_points=kp)
            # single-plan launch shape for this set size and edge rule, tuned on a uniform set
            rm_t = gmt.gmt_build_neighbors(torch.from_numpy(I.di_samples(7_000, n)).to(dev),
                                           gmt.GMT_COST_DOUBLE_INTEGRATOR, rr)
            p0 = tests[0]
            tuned_single["n%d%s" % (n, tag)] = gmt.gmt_autotune(
                [gmt.BatchQuery(rm_t, p0.x_init, gmt.make_goal(p0.goal_center, p0.goal_radius, 3), p0.boxes,
                                p0.lam)], opts_k, single=True, reps=3)
            rm_t.free()
            for learned in ((True, False) if tag != "_points_scaled" else (True,)):
                costs, lat, rej, parts = [], [], 0, []
                for k, p in enumerate(tests):
                    goal = gmt.make_goal(p.goal_center, p.goal_radius, 3)
                    ss = k % sets

                    def run():
                        t0 = time.perf_counter()
                        if learned:
                            x, rj = S.mixed_samples(smp, p, n, 0, True, uniform=uni[ss], fallback=fb[ss],
                                                    eps=eps[ss])
                        else:
                            x, rj = uni_full[ss], 0
                        torch.cuda.synchronize()
                        t1 = time.perf_counter()
                        rm = gmt.gmt_build_neighbors(x, gmt.GMT_COST_DOUBLE_INTEGRATOR, rr)
                        t2 = time.perf_counter()
                        res = gmt.gmt_plan(rm, p.x_init, goal, p.boxes, p.lam, opts_k, outputs=False)
                        t3 = time.perf_counter()
                        rm.free()
                        parts.append((t1 - t0, t2 - t1, t3 - t2))
                        return res, rj
                    (res, rj), ms = timed(run)
                    rej += rj
                    costs.append(res.path_cost if res.status == gmt.GMT_OK else np.inf)
                    lat.append(ms)
                costs = np.array(costs)
                both = np.isfinite(costs) & np.isfinite(ref_cost)
                ratio = costs[both] / ref_cost[both]
                e2e = float(np.percentile(lat, 50))
                rows["%s%s_n%d" % ("learned" if learned else "uniform", tag, n)] = {
                    "n": n, "r": round(rr, 4), "traj_points": kp,
                    "solved": int(np.isfinite(costs).sum()),
                    "median_cost_ratio_vs_plain_n32768": round(float(np.median(ratio)), 4) if both.any() else None,
                    "mean_cost_ratio_vs_plain_n32768": round(float(np.mean(ratio)), 4) if both.any() else None,
                    "p50_ms_end_to_end": round(e2e, 3),
                    "p99_ms_end_to_end": round(float(np.percentile(lat, 99)), 3),
                    "faster_than_plain_resident": bool(e2e < plain_p50),
                    "p50_ms_sampler": round(float(np.median([a for a, _, _ in parts])) * 1e3, 3),
                    "p50_ms_build": round(float(np.median([b for _, b, _ in parts])) * 1e3, 3),
                    "p50_ms_plan": round(float(np.median([c for _, _, c in parts])) * 1e3, 3),
                    "rejected_per_query": round(rej / len(tests), 1)}
        say("learned n=%d done" % n)
    for rm in rms.values():
        rm.free()
    smp.close()
    return {"train_problems": args.learned_train, "train_solved": data.solved,
            "waypoints": int(data.targets.shape[0]), "dataset_s": round(data_s, 1),
            "train_steps": args.learned_steps, "train_s": round(train_s, 2),
            "loss_first_last": [[round(v, 4) for v in hist[0][1:]], [round(v, 4) for v in hist[-1][1:]]],
            "test_problems": len(tests),
            "plain_n32768": {"solved": int(np.isfinite(ref_cost).sum()), "r": round(r_big, 4),
                             "p50_ms_plan_resident": round(plain_p50, 3),
                             "build_ms": round(float(np.median(build_ms)), 3),
                             "single_plan_shape": {kk: tuned_plain[kk] for kk in
                                                   ("lanes", "team_wgs", "threads", "ms", "default_ms")}},
            "mixes": rows,
            "single_plan_shape": {k: {kk: v[kk] for kk in ("lanes", "team_wgs", "threads", "ms", "default_ms")}
                                  for k, v in tuned_single.items()},
            "note": "end-to-end = sampler inference + neighbour build + plan, synchronised, per query; uniform "
                    "draws, fallbacks and noise are query-independent and resident (8 pools per n); edge rules: "
                    "r(n) = 1.75 (16384/n)^(1/6) with 16 trajectory points; r(n) with ceil(16 r(n)/r(32768)) "
                    "points (_points_scaled); plain's r(32768) with 16 points (_equal_r)"}


def lat_stats(ms):
    ms = np.asarray(ms, np.float64)
    return {"p50_ms": round(float(np.percentile(ms, 50)), 3), "p99_ms": round(float(np.percentile(ms, 99)), 3)}


def single_latency(torch, gmt, rm, probs, opts, warm=5):
    """Wall time of gmt_plan (entry to path on the host) per query."""
    out, ms = [], []
    for k, p in enumerate(list(probs[:warm]) + list(probs)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = gmt.gmt_plan(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, p.pdim), p.boxes, p.lam,
                           opts, outputs=False)
        dt = (time.perf_counter() - t) * 1e3
        if k >= warm:
            ms.append(dt)
            out.append(res)
    return out, ms


def batch_rate(torch, gmt, queries, opts, reps=3):
    """plans/s of one prepared batch (median of `reps` timed runs after one warm-up)."""
    pb = gmt.PreparedBatch(queries, opts)
    pb.run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        pb.run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return len(queries) / float(np.median(ts)), pb.results()


def dubins_report(args, torch, gmt, I):
    """Dubins airplane (Section V-A's third workload): n = 5000 samples, forests
    of 150 trunks: single-plan latency and batch plans/s; then one forest described by 150 .. 5000 boxes (Table III's obstacle rows)."""
    dev = torch.device("cuda", 0)
    n, sets = 5000, 4
    samples, rms, bms = {}, {}, []
    gmt.gmt_profile_enable(True)
    for ss in range(sets):
        samples[ss] = I.dubins_samples(ss, n)
        rms[ss] = gmt.gmt_build_neighbors(torch.from_numpy(samples[ss]).to(dev), gmt.GMT_COST_DUBINS_AIRPLANE,
                                          I.DUBINS_RADIUS, turn_radius=I.DUBINS_TURN)
        bms.append(gmt.gmt_last_build())
    gmt.gmt_profile_enable(False)
    gmt.gmt_profile_read()
    opts = gmt.make_opts(edge_step=I.DUBINS_STEP)
    probs = [I.dubins_problem(k, samples[k % sets], sample_seed=k % sets) for k in range(args.dubins_queries)]
    lat, lres = [], []
    for ss in range(sets):
        sub = [p for p in probs if p.sample_seed == ss][:max(args.dubins_latency // sets, 1)]
        o, m = single_latency(torch, gmt, rms[ss], sub, opts)
        lat += m
        lres += o
    qs = [gmt.BatchQuery(rms[p.sample_seed], p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam,
                         p.step) for p in probs]
    rate, bres = batch_rate(torch, gmt, qs, opts)
    sweep = []
    for m in (150, 500, 1500, 5000):
        fp = [I.dubins_forest_problem(k, samples[0], m) for k in range(args.forest_queries)]
        o, ms = single_latency(torch, gmt, rms[0], fp, opts, warm=2)
        fq = [gmt.BatchQuery(rms[0], p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam, p.step)
              for p in fp]
        frate, _ = batch_rate(torch, gmt, fq * max(1, 256 // len(fq)), opts, reps=2)
        costs = [x.path_cost for x in o if x.status == gmt.GMT_OK]
        sweep.append(dict(boxes=m, solved="%d/%d" % (len(costs), len(o)), **lat_stats(ms),
                          batch_plans_per_s=round(frate, 1),
                          median_cost=round(float(np.median(costs)), 4) if costs else None))
    for rm in rms.values():
        rm.free()
    bk = [b["kernel_ms"] for b in bms[1:]] or [bms[0]["kernel_ms"]]
    return {"workload": "Dubins airplane n=%d, 150 trunks, turning radius %.2f, r=%.2f, step %.3f, lambda 0.5"
                        % (n, I.DUBINS_TURN, I.DUBINS_RADIUS, I.DUBINS_STEP),
            "roadmap_edges": int(bms[0]["edges"]), "build_kernel_ms": round(float(np.median(bk)), 3),
            "single": dict(queries=len(lat), solved=sum(r.status == gmt.GMT_OK for r in lres), **lat_stats(lat)),
            "batch": {"queries": len(qs), "plans_per_s": round(rate, 1),
                      "solved": sum(r.status == gmt.GMT_OK for r in bres)},
            "obstacle_sweep": sweep,
            "paper_context": "Table III forest rows on a GTX 980 at n = 5k: 150 / 500 / 1500 / 5000 boxes in "
                             "7 / 14 / 18 / 26 ms (different forest and hardware)"}


def halton_report(args, torch, gmt, I):
    """Halton sample sets (Section V-A) against uniform ones: 3D workload at
    n = 16384 (Halton radius vs Theorem 1's), and the double integrator."""
    from paper_1705_02403_amd import radius as RAD
    dev = torch.device("cuda", 0)
    rows = {}
    probs = [I.problem_3d(k) for k in range(args.halton_queries)]
    for mode in ("uniform", "halton"):
        lat, costs, ok, edges, gen_ms = [], [], 0, [], []
        for p in probs:
            mu = RAD.free_volume(3, p.boxes)
            if mode == "halton":
                torch.cuda.synchronize()
                t = time.perf_counter()
                x, _ = gmt.gmt_sample_halton(p.n, 3, gmt.GMT_COST_EUCLIDEAN, 1, p.boxes)
                torch.cuda.synchronize()
                gen_ms.append((time.perf_counter() - t) * 1e3)
                r = RAD.halton_radius(3, mu, p.n)
            else:
                x = torch.from_numpy(p.samples).to(dev)
                r = RAD.theorem1_radius(3, mu, p.n)
            rm = gmt.gmt_build_neighbors(x, gmt.GMT_COST_EUCLIDEAN, r)
            edges.append(rm.nnz)
            o, ms = single_latency(torch, gmt, rm, [p], gmt.make_opts(edge_step=p.step), warm=1)
            lat += ms
            if o[0].status == gmt.GMT_OK:
                ok += 1
                costs.append(o[0].path_cost)
            rm.free()
        rows[mode] = dict(solved="%d/%d" % (ok, len(probs)), mean_edges=int(np.mean(edges)),
                          median_cost=round(float(np.median(costs)), 4) if costs else None, **lat_stats(lat))
        if gen_ms:
            rows[mode]["sample_ms"] = round(float(np.median(gen_ms)), 3)
    return {"workload": "3D, n=16384, 60 boxes: uniform samples at Theorem 1's radius vs Halton samples at "
                        "the Halton radius (twice a dispersion bound)", "rows": rows}


def replan_report(args, torch, gmt, I):
    """Replanning in a collapsing world (Section V-C): scenarios on one resident
    double-integrator roadmap, all replanned every 10 ms of world time."""
    from paper_1705_02403_amd import replan as RP
    dev = torch.device("cuda", 0)
    s = I.di_samples(0, 16384)
    rm = gmt.gmt_build_neighbors(torch.from_numpy(s).to(dev), gmt.GMT_COST_DOUBLE_INTEGRATOR, I.DI_RADIUS)
    ec = RP.EdgeCosts(rm)
    plan = RP.library_planner(rm, gmt.make_opts(traj_points=16), 3)
    out = []
    for rate in (0.0, 20.0, 50.0):
        scen = []
        for k in range(args.replan_scenarios):
            p = I.di_problem(500 + k, s)
            scen.append(RP.Scenario(p.x_init, p.goal_center, p.goal_radius, p.boxes,
                                    I.collapse_schedule(k, rate, 4.0), p.lam))
        st = RP.Replanner(s, ec, plan, scen, pdim=3, dt=0.01, speed=2.0, t_max=4.0).run()
        st["boxes_per_s"] = rate
        out.append(st)
    rm.free()
    return {"workload": "6D double integrator n=16384, 40 boxes plus a Poisson collapse, %d scenarios, "
                        "10 ms ticks, robots fly 2 cost units per second" % args.replan_scenarios, "runs": out}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _run_pool(jobs, cores):
    """Run the callables in `jobs` on `cores` threads (the oracle's C calls
    release the GIL, so each thread keeps one core busy); returns each job's
    wall time in ms, in job order, and the makespan in s."""
    ms = [0.0] * len(jobs)
    nxt = [0]
    lock = threading.Lock()

    def worker():
        while True:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            if k >= len(jobs):
                return
            t = time.perf_counter()
            jobs[k]()
            ms[k] = (time.perf_counter() - t) * 1e3
    ths = [threading.Thread(target=worker) for _ in range(max(1, cores))]
    t = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    return ms, time.perf_counter() - t


def cpu_latency_report(args, cores):
    """Single-core oracle latency (the serial FP64 C oracle, one thread per
    plan) per workload: the 2D, 3D and 6D configurations, their neighbour
    tables built beforehand (excluded, as the GPU's roadmaps are resident).
    Problems run `cores` at a time, one per thread."""
    from oracle import oracle as O
    from paper_1705_02403_amd import inputs as I
    out = {}
    for name, make, count in (("2d_n2000", lambda k: I.problem_2d(k), args.cpu_2d),
                              ("3d_n16384", lambda k: I.problem_3d(k), args.cpu_3d),
                              ("di_n16384", None, args.cpu_di)):
        if count <= 0:
            continue
        jobs = []
        t = time.perf_counter()
        if make is None:
            s = I.di_samples(0, 16384)
            tab = O.neighbors(s, O.DI, I.DI_RADIUS)
            for k in range(count):
                p = I.di_problem(k, s)
                jobs.append(lambda p=p: O.plan(p, p.r, tab))
        else:
            for k in range(count):
                p = make(k)
                r = O.euclid_radius(p)
                tab = O.neighbors(p.samples, O.EUCLID, r)
                jobs.append(lambda p=p, r=r, tab=tab: O.plan(p, r, tab))
        tables_s = time.perf_counter() - t
        ms, _ = _run_pool(jobs, cores)
        out[name] = dict(problems=count, tables_s=round(tables_s, 1), **lat_stats(ms))
    return out


def cpu_mixed_report(args, cores):
    """Oracle throughput on the mixed 2D/3D/6D set (configuration 4): the
    first --cpu-mixed requests in arrival order, one worker thread per core,
    all at t = 0; tables of their shared sample sets built beforehand."""
    from oracle import oracle as O
    from paper_1705_02403_amd import inputs as I, radius
    specs = I.batch_specs(512)[:args.cpu_mixed]
    tabs, samples = {}, {}
    t = time.perf_counter()
    for sp in specs:
        key = (sp["dim"], sp["n"], sp["sample_seed"])
        if key in tabs:
            continue
        x = (I.di_samples(sp["sample_seed"], sp["n"]) if sp["dim"] == 6
             else I.uniform_samples(sp["dim"], sp["n"], sp["sample_seed"]))
        samples[key] = x
        rr = radius.shared_roadmap_radius(sp["dim"], sp["n"])
        tabs[key] = (rr, O.neighbors(x, O.DI if sp["dim"] == 6 else O.EUCLID, rr))
    tables_s = time.perf_counter() - t
    jobs = []
    for sp in specs:
        key = (sp["dim"], sp["n"], sp["sample_seed"])
        p = I.mixed_problem(sp, samples[key])
        rr, tab = tabs[key]
        jobs.append(lambda p=p, rr=rr, tab=tab: O.plan(p, rr, tab))
    ms, wall = _run_pool(jobs, cores)
    return {"value": round(len(jobs) / wall, 2), "unit": "plans/s", "cores": cores, "problems": len(jobs),
            "roadmaps": len(tabs), "tables_s": round(tables_s, 1), "makespan_s": round(wall, 2),
            "dims": {str(d): sum(sp["dim"] == d for sp in specs) for d in (2, 3, 6)},
            "sample": "the first %d of the 512 mixed requests (arrival order), all at t = 0, one oracle "
                      "thread per core" % len(jobs)}


def mixed_report(args, torch, gmt, I):
    """Batched replanning (configuration 4): mixed 2D/3D/6D queries, n
    log-uniform in [1k, 32k], 10-100 boxes, on shared resident roadmaps keyed
    by (dim, n, sample seed); Poisson arrivals, then all at once."""
    from paper_1705_02403_amd import radius, server
    dev = torch.device("cuda", 0)
    specs = I.batch_specs(args.mixed_requests)
    samples, rms = {}, {}
    t = time.perf_counter()
    for sp in specs:
        key = (sp["dim"], sp["n"], sp["sample_seed"])
        if key in rms:
            continue
        x = (I.di_samples(sp["sample_seed"], sp["n"]) if sp["dim"] == 6
             else I.uniform_samples(sp["dim"], sp["n"], sp["sample_seed"]))
        samples[key] = x
        kind = gmt.GMT_COST_DOUBLE_INTEGRATOR if sp["dim"] == 6 else gmt.GMT_COST_EUCLIDEAN
        rms[key] = gmt.gmt_build_neighbors(torch.from_numpy(x).to(dev), kind,
                                           radius.shared_roadmap_radius(sp["dim"], sp["n"]))
    build_s = time.perf_counter() - t
    probs = [(sp, I.mixed_problem(sp, samples[(sp["dim"], sp["n"], sp["sample_seed"])])) for sp in specs]

    def make(p):
        return lambda rm: gmt.BatchQuery(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, p.pdim),
                                         p.boxes, p.lam, p.step)

    arr = I.poisson_arrivals(len(probs), args.mixed_rate, seed=7)
    reqs = [server.Request(float(a), (sp["dim"], sp["n"], sp["sample_seed"]), make(p), tag=k)
            for k, (a, (sp, p)) in enumerate(zip(arr, probs))]
    srv = server.ReplanServer(lambda key: rms[key], gmt.make_opts(traj_points=16), engine_budget=16 << 30,
                              roadmap_budget=1 << 40, slots=4, max_batch=256)
    srv.serve(reqs[:64], realtime=False)  # warm streams and workspaces
    rep = srv.serve(reqs)
    sat = srv.serve(reqs, realtime=False)
    srv.engine.close()
    for rm in rms.values():
        rm.free()
    solved = sum(s.status == gmt.GMT_OK for s in rep.served)
    return {"requests": len(reqs), "roadmaps": len(rms), "roadmap_build_s": round(build_s, 2),
            "dims": {str(d): sum(sp["dim"] == d for sp in specs) for d in (2, 3, 6)},
            "arrival_rate_hz": args.mixed_rate, "p50_ms": round(rep.p50_ms, 3), "p99_ms": round(rep.p99_ms, 3),
            "plans_per_s": round(rep.plans_per_s, 1), "solved": solved,
            "all_at_once_plans_per_s": round(sat.plans_per_s, 1),
            "all_at_once_p50_ms": round(sat.p50_ms, 3), "batches": rep.engine.get("batches")}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the planner shards by query, and this build measures "
              "one device (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1705_02403_amd import gmt, inputs as I

    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_copy": 1 << 30, "copies": 5}), flush=True)
        return
    gmt.use_torch_allocator()
    stream = torch.cuda.current_stream()
    n = args.n
    r = I.DI_RADIUS

    # ---- resident roadmaps (untimed; the method precomputes them) ----
    samples = {ss: I.di_samples(ss, n) for ss in range(args.sample_sets)}
    rms, build_ms, di_builds = {}, [], []
    gmt.gmt_profile_enable(True)
    for ss in range(args.sample_sets):
        d = torch.from_numpy(samples[ss]).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rms[ss] = gmt.gmt_build_neighbors(d, gmt.GMT_COST_DOUBLE_INTEGRATOR, r)
        torch.cuda.synchronize()
        build_ms.append((time.perf_counter() - t0) * 1e3)
        di_builds.append(gmt.gmt_last_build())
    gmt.gmt_profile_enable(False)
    gmt.gmt_profile_read()
    nnz = [rms[ss].nnz for ss in rms]
    # the first build of the process also pays module loading: median of the rest
    dib = di_builds[1:] if len(di_builds) > 1 else di_builds
    di_kms = float(np.median([b["kernel_ms"] for b in dib]))
    di_flops = float(np.median([di_build_flops(b["pairs_tested"], b["pairs_solved"]) for b in dib]))
    di_build_line = {"workload": "6D double integrator n=%d, r=%.3f" % (n, r), "bound": "fp64-valu",
                     "kernel_ms": round(di_kms, 4),
                     "pairs_tested": int(np.median([b["pairs_tested"] for b in dib])),
                     "pairs_solved": int(np.median([b["pairs_solved"] for b in dib])),
                     "flops": int(di_flops), "achieved": round(di_flops / (di_kms * 1e-3) / 1e12, 2),
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(di_flops / (di_kms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4),
                     "flop_model": "150 per solved pair + 10 per prefiltered pair",
                     "wall_ms": round(float(np.median(build_ms[1:] or build_ms)), 3)}

    probs = [I.di_problem(k, samples[k % args.sample_sets], sample_seed=k % args.sample_sets)
             for k in range(args.batch)]

    def query(p):
        return gmt.BatchQuery(rms[p.sample_seed], p.x_init,
                              gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam)

    queries = [query(p) for p in probs]
    opts = gmt.make_opts(traj_points=16, lanes=args.lanes, threads=args.threads)
    if args.lanes or args.threads:
        args.no_autotune = True
    # launch shape: the autotuner times every candidate on this batch and on
    # one single query, checks they give identical results, caches the fastest
    tuned = None
    if not args.no_autotune:
        tuned = {"batch": gmt.gmt_autotune(queries, opts, single=False, reps=2),
                 "single": gmt.gmt_autotune(queries[:1], opts, single=True, reps=3)}
        say("tuned batch shape: lanes %(lanes)d, team_wgs %(team_wgs)d, workgroups %(workgroups)d, "
            "threads %(threads)d" % tuned["batch"])
    # ---- eager steps: each one gmt_plan_batch call on host-side query
    # descriptors (staging and descriptor upload inside every step; PCIe-
    # inclusive); their HIP events give the kernel's duration ----
    batch = gmt.PreparedBatch(queries, opts)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    gmt.gmt_profile_enable(True)
    gmt.gmt_profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    eager_elapsed = time.perf_counter() - t0
    kernel_ms, launches = gmt.gmt_profile_read()
    gmt.gmt_profile_enable(False)
    work = gmt.gmt_last_work()
    out = batch.results()
    say("eager steps: %.3f ms per step" % (eager_elapsed * 1e3 / args.steps))

    # ---- timed steps (the headline): the batch staged and uploaded once,
    # each step a replay of its captured launch (queue reset, planning
    # kernel, results copied back), inputs resident in HBM ----
    gb = gmt.GraphBatch(queries, opts)
    for _ in range(args.warmup):
        gb.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gb.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(a.status == b.status and a.path_cost == b.path_cost for a, b in zip(gb.results(), out))
    gb.close()
    inputs_resident = (tuned["batch"]["team_wgs"] if tuned else 1) == 1
    ok = sum(o.status == gmt.GMT_OK for o in out)
    plans = args.steps * args.batch
    value = plans / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    avg_kernel_ms = kernel_ms / max(launches, 1)
    bytes_per_launch = plan_bytes(work)  # one launch plans the whole batch
    achieved = bytes_per_launch / (avg_kernel_ms * 1e-3) / 1e9
    bytes_as_built = plan_bytes(work, in_edge=28)
    shape = (tuned["batch"] if tuned else {"lanes": args.lanes, "threads": args.threads})
    traffic = None
    if kernel_digest() == TRAFFIC["sources_sha256"] and args.batch == TRAFFIC["batch"]:
        traffic = TRAFFIC["by_shape"].get((shape.get("lanes"), shape.get("threads")))

    # ---- latency: single queries, the whole GPU on one plan ----
    lat = []
    n_lat = 0 if args.only_throughput else args.latency_warmup + args.latency_samples
    for k in range(n_lat):
        p = probs[k % len(probs)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = gmt.gmt_plan(rms[p.sample_seed], p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3),
                           p.boxes, p.lam, opts, outputs=False)
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[args.latency_warmup:]) if len(lat) > args.latency_warmup else None

    # ---- replanning server: Poisson arrivals through the continuous-batching engine ----
    srv_line = None
    if args.server_requests > 0 and not args.only_throughput:
        from paper_1705_02403_amd import server
        arr = I.poisson_arrivals(args.server_requests, args.server_rate, seed=11)
        reqs = [server.Request(float(t), probs[k % len(probs)].sample_seed,
                               (lambda q: lambda rm: q)(queries[k % len(queries)]), tag=k)
                for k, t in enumerate(arr)]
        sopts = gmt.make_opts(traj_points=16, threads=args.server_threads)
        srv = server.ReplanServer(lambda key: rms[key], sopts, engine_budget=8 << 30,
                                  roadmap_budget=1 << 40, slots=args.server_slots,
                                  max_batch=args.server_max_batch)
        srv.serve(reqs[:256])  # warm the streams and workspaces
        rep = srv.serve(reqs)
        srv.engine.close()
        by_tag = {s.tag: s for s in rep.served}
        same = sum(by_tag[k].path_cost == out[k % len(out)].path_cost for k in by_tag)
        srv_line = {"arrival_rate_hz": args.server_rate, "requests": len(rep.served),
                    "slots": args.server_slots, "max_batch": args.server_max_batch,
                    "threads": args.server_threads,
                    "plans_per_s": round(rep.plans_per_s, 1), "p50_ms": round(rep.p50_ms, 3),
                    "p99_ms": round(rep.p99_ms, 3), "batches": rep.engine.get("batches"),
                    "lone_launches": rep.engine.get("lone_launches"),
                    "peak_inflight_requests": rep.engine.get("peak_inflight_requests"),
                    "identical_to_batch": "%d/%d" % (same, len(rep.served))}
        # low load: requests often find the device idle and run in the
        # single-plan launch shape
        if args.server_low_requests > 0:
            arr = I.poisson_arrivals(args.server_low_requests, args.server_low_rate, seed=12)
            lreqs = [server.Request(float(t), probs[k % len(probs)].sample_seed,
                                    (lambda q: lambda rm: q)(queries[k % len(queries)]), tag=k)
                     for k, t in enumerate(arr)]
            srv = server.ReplanServer(lambda key: rms[key], sopts, engine_budget=8 << 30,
                                      roadmap_budget=1 << 40, slots=args.server_slots,
                                      max_batch=args.server_max_batch)
            srv.serve(lreqs[:32])
            low = srv.serve(lreqs)
            srv.engine.close()
            by_tag = {s.tag: s for s in low.served}
            same = sum(by_tag[k].path_cost == out[k % len(out)].path_cost for k in by_tag)
            srv_line["low_load"] = {"arrival_rate_hz": args.server_low_rate, "requests": len(low.served),
                                    "plans_per_s": round(low.plans_per_s, 1), "p50_ms": round(low.p50_ms, 3),
                                    "p99_ms": round(low.p99_ms, 3), "batches": low.engine.get("batches"),
                                    "lone_launches": low.engine.get("lone_launches"),
                                    "identical_to_batch": "%d/%d" % (same, len(low.served))}

    # ---- Euclidean neighbour table builds, 3D (the 3D workload and larger n) ----
    # bytes the build must move: samples read, row pointers, an index and a
    # cost per edge; as built: one 8-byte record per edge and the row lengths
    build_line = None
    if not args.only_throughput and args.euclid_sizes:
        from paper_1705_02403_amd import radius as RAD
        build_line = []
        for n3 in [int(x) for x in args.euclid_sizes.split(",")]:
            p3 = I.problem_3d(0, n=n3)
            r3 = RAD.problem_radius(p3)
            d3 = torch.from_numpy(p3.samples).cuda()
            # the tuner's tile shape for this (dim, n) bucket, then builds with it
            btuned = gmt.gmt_autotune_build(d3, r3, reps=3)
            bt, kt = [], []
            gmt.gmt_profile_enable(True)
            for k in range(5):
                torch.cuda.synchronize()
                t = time.perf_counter()
                rm3 = gmt.gmt_build_neighbors(d3, gmt.GMT_COST_EUCLIDEAN, r3)
                torch.cuda.synchronize()
                bt.append((time.perf_counter() - t) * 1e3)
                lb = gmt.gmt_last_build()
                kt.append(lb["kernel_ms"])
                e3 = rm3.nnz
                held = rm3.device_bytes
                rm3.free()
            gmt.gmt_profile_enable(False)
            gmt.gmt_profile_read()
            bt = float(np.median(bt[1:]))
            kms = float(np.median(kt[1:]))
            nbytes = euclid_build_bytes(n3, 3, e3)
            built = euclid_build_bytes(n3, 3, e3) + 4 * n3
            eu_traffic = None
            if (n3 == EU_TRAFFIC["n"] and lb["tile"] == EU_TRAFFIC["tile"] and
                    kernel_digest(("gmt_build.hpp", "gmt_dev.hpp")) == EU_TRAFFIC["sources_sha256"]):
                eu_traffic = EU_TRAFFIC["bytes_per_launch"]
            build_line.append({"workload": "3D Euclidean n=%d, r=%.4f" % (n3, r3), "edges": int(e3),
                               "device_bytes": int(held),
                               "kernel_ms": round(kms, 4), "wall_ms": round(bt, 3), "bytes": int(nbytes),
                               "achieved": round(nbytes / (kms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(nbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "bytes_as_built": int(built),
                               "frac_as_built": round(built / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "traffic_k_eu_rows": eu_traffic, "tile": int(lb["tile"]),
                               "tuner": {"tile": btuned["tile"], "ms": round(btuned["ms"], 4),
                                         "default_ms": round(btuned["default_ms"], 4),
                                         "rejected": btuned["rejected"]}})
            say("euclid build n=%d: %.3f ms wall, %.3f ms kernels, tile %d" % (n3, bt, kms, lb["tile"]))
            del d3

    learned = None
    if not args.no_learned and not args.only_throughput:
        say("learned sampler")
        learned = learned_report(args, torch, gmt, I)
    extra = {}
    if not args.no_extra and not args.only_throughput:
        say("dubins airplane")
        extra["dubins"] = dubins_report(args, torch, gmt, I)
        say("halton")
        extra["halton"] = halton_report(args, torch, gmt, I)
        say("replanning")
        extra["replanning"] = replan_report(args, torch, gmt, I)
    mixed = (mixed_report(args, torch, gmt, I)
             if args.mixed_requests > 0 and not args.only_throughput else None)

    # ---- cost against the FP64 oracle (sample set 0) and CPU baseline ----
    check = {}
    cpu = None
    if (args.oracle_checks > 0 or not args.no_cpu) and not args.only_throughput:
        from oracle import oracle as O
        t = time.perf_counter()
        tab = O.neighbors(samples[0], O.DI, r)
        oracle_build_s = time.perf_counter() - t
        sel = [p for p in probs if p.sample_seed == 0][:max(args.oracle_checks, 1)]
        rel, same_path = [], 0
        by_seed = {p.seed: o for p, o in zip(probs, out)}
        for p in sel[:args.oracle_checks]:
            ref = O.plan(p, r, tab)
            g = by_seed[p.seed]
            if ref.status == O.OK and g.status == gmt.GMT_OK:
                rel.append(abs(g.path_cost - ref.path_cost) / ref.path_cost)
                same_path += int(list(g.path) == list(ref.path))
            elif ref.status != g.status:
                rel.append(float("inf"))
        check = {"problems": len(sel[:args.oracle_checks]),
                 "max_rel_cost_diff": (max(rel) if rel else None),
                 "identical_paths": same_path, "oracle_table_s": round(oracle_build_s, 2)}
        if not args.no_cpu:
            cores = os.cpu_count() or 1
            lock = threading.Lock()
            done = [0]
            stop = time.perf_counter() + args.cpu_seconds
            pool_probs = [p for p in probs if p.sample_seed == 0]

            def worker(w):
                k = w
                while time.perf_counter() < stop:
                    O.plan(pool_probs[k % len(pool_probs)], r, tab)
                    with lock:
                        done[0] += 1
                    k += cores
            ths = [threading.Thread(target=worker, args=(w,)) for w in range(cores)]
            t = time.perf_counter()
            for th in ths:
                th.start()
            for th in ths:
                th.join()
            dt = time.perf_counter() - t
            say("cpu latency")
            cpu = {"value": round(done[0] / dt, 2), "unit": "plans/s", "cores": cores,
                   "kind": "oracle",
                   "sample": "%d FP64 oracle plans (Algorithm 1, serial C) of the same 6D DI n=%d "
                             "queries on sample set 0, one thread per core (%d) for %.1f s; its "
                             "neighbour table (%.1f s, OpenMP) built beforehand like the GPU roadmaps"
                             % (done[0], n, cores, dt, oracle_build_s),
                   "cpu_model": cpu_model(), "nproc": cores,
                   "single_core_latency": cpu_latency_report(args, cores),
                   "latency_note": "serial C oracle, one thread per plan, %d plans at a time; tables "
                                   "precomputed (excluded, as the roadmap is)" % cores,
                   "mixed_set": cpu_mixed_report(args, cores) if args.cpu_mixed > 0 else None}

    line = {
        "metric": "plans/s + p50/p99 plan latency, 6D double-integrator n=16k; cost vs FP64 oracle",
        "value": round(value, 1),
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "6D double integrator, n=16384 samples, 40 boxes U[0.05,0.2], "
                               "lambda=0.5, r=1.75, 16 trajectory points",
                   "batch_queries": args.batch, "sample_sets": args.sample_sets},
        "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat is not None else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat is not None else None,
        "solved": "%d/%d" % (ok, args.batch),
        "inputs_resident": inputs_resident,
        "eager_ms_per_step": round(eager_elapsed * 1e3 / args.steps, 3),
        "eager_plans_per_s": round(plans / eager_elapsed, 1),
        "launch_shape": tuned,
        "roadmap_build_ms": round(float(np.median(build_ms)), 3),
        "roadmap_nnz": int(np.median(nnz)),
        "work_per_plan": {k: round(v / args.batch, 1) for k, v in work.items()},
        "oracle_check": check,
        "server": srv_line,
        "mixed_stream": mixed,
        "learned": learned,
        "dubins": extra.get("dubins"),
        "halton": extra.get("halton"),
        "replanning": extra.get("replanning"),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_plan<1> (one launch per batch)",
                     "avg_kernel_ms": round(avg_kernel_ms, 3),
                     "bytes_per_launch": int(bytes_per_launch),
                     "bytes_model": "4 B per out-edge + 24 B per scanned in-edge + 16 B per commit "
                                    "+ 12 B per open entry",
                     "as_built": {"bytes_per_launch": int(bytes_as_built),
                                  "frac": round(bytes_as_built / (avg_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "note": "28 B per in-edge: 12-byte FP64-cost record + 16 B node state"},
                     "traffic_frac": (round(traffic / (avg_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None)},
        "build_rooflines": {"di": di_build_line, "euclid_3d": build_line},
        "cpu_baseline": cpu,
    }
    for rm in rms.values():
        rm.free()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

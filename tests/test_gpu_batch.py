"""Batches of independent runs (lb_batch_*) and the continuous-batching
request loop.

The batched kernel runs the tile step of LB_PATH_TILE on every live slot, so
each slot's result must equal the same run alone bit for bit, on any path
(the single-run paths agree bit for bit with each other), whatever else is
in the batch, whenever it joined, whichever kernel configuration the
autotuner picked, and whether its steps came from graph replays or direct
launches."""
import numpy as np
import pytest

import lbinputs as LI
from gpu_helpers import TOL, run_gpu, run_oracle, run_oracle_f16s_budget

pytestmark = pytest.mark.gpu


def mixed_runs(storage="f32"):
    """Runs of different boxes (ragged against every tile shape), N and
    parameters."""
    runs = []
    for k, (L, ny, n, steps) in enumerate([(64, 64, 2, 60), (70, 33, 3, 45), (96, 130, 2, 80), (130, 97, 3, 30),
                                           (150, 64, 2, 75), (200, 41, 3, 52)]):
        if n == 2:
            p = LI.params("D2Q9", 2, (L, ny), tau=0.9 + 0.05 * k, kappa=0.01,
                          chi=np.array([[0.0, 2.3 + 0.1 * k], [2.3 + 0.1 * k, 0.0]]))
            r = LI.noisy_uniform(p, [0.5, 0.5], 0.01, 300 + k)
        else:
            chi = np.full((3, 3), 3.1 + 0.03 * k)
            np.fill_diagonal(chi, 0.0)
            p = LI.params("D2Q9", 3, (L, ny), tau=1.1 - 0.03 * k, kappa=0.008, chi=chi)
            r = LI.noisy_uniform(p, [1 / 3] * 3, 0.01, 300 + k)
        runs.append((p, r, steps))
    return runs


def solo(cfg, rho0, steps, storage, path):
    return run_gpu(cfg, rho0, steps, storage=storage, path=path, fields=True)


def drain(batch, slots, max_calls=10000, chunk=7):
    """Step until every slot in `slots` has finished; returns their moments."""
    out = {}
    for _ in range(max_calls):
        batch.step(chunk)
        counts = batch.poll(0)
        for s, target in slots.items():
            if s not in out and counts[s] == target:
                out[s] = batch.moments(s)
        if len(out) == len(slots):
            return out
    raise AssertionError("slots did not finish")


@pytest.mark.parametrize("storage", ["f32", "f64", "f16s"])
def test_batch_equals_each_run_alone(storage):
    from paper_0704_3444_amd import Batch

    runs = mixed_runs()
    b = Batch(storage=storage, max_comp=3, max_slots=16, arena_bytes=256 << 20, graph_steps=8)
    slots = {b.add(p, r, steps): steps for (p, r, steps) in runs}
    out = drain(b, slots)
    b.close()
    for (s, steps), (p, r, _) in zip(slots.items(), runs):
        for path in ("tile", "split"):
            ref = solo(p, r, steps, storage, path)
            print(f"[batch] {storage} slot {s} {p['shape']} N={p['n_comp']} {steps} steps vs {path}", flush=True)
            assert out[s]["step"] == steps
            assert np.array_equal(out[s]["rho"], ref["rho"]), (s, path)
            assert np.array_equal(out[s]["U"], ref["U"]), (s, path)
            assert np.array_equal(out[s]["mass"], ref["mass"]), (s, path)


def test_batch_graph_replays_match_direct_launches():
    """Copies of one run with targets 8, 16, ..., 40: each replay of an
    8-step graph finishes one of them; between replays the program does its
    own eager work and synchronises.  Every finished copy equals the run
    alone with that many steps, and the batch stepped by direct launches
    only (graph longer than any call)."""
    import torch
    from paper_0704_3444_amd import Batch

    p, r, _ = mixed_runs()[1]
    outs = []
    for gs in (8, 1000):
        b = Batch(storage="f32", max_comp=3, max_slots=8, arena_bytes=64 << 20, graph_steps=gs)
        slots = {b.add(p, r, 8 * k): 8 * k for k in range(1, 6)}
        res = {}
        for k in range(1, 6):
            b.step(8)
            x = torch.ones(1000, device="cuda").cumsum(0)  # unrelated eager work between replays
            torch.cuda.synchronize()
            assert float(x[-1]) == 1000.0
            counts = b.poll(0)
            for s, target in slots.items():
                if target == 8 * k:
                    assert counts[s] == target
                    res[target] = b.moments(s)["rho"]
                else:
                    assert counts[s] == min(8 * k, target)
        b.close()
        outs.append(res)
    for target in outs[0]:
        ref = solo(p, r, target, "f32", "tile")
        assert np.array_equal(outs[0][target], ref["rho"]), target
        assert np.array_equal(outs[1][target], ref["rho"]), target


def test_batch_join_and_leave_midrun():
    """Slots join while others are half way and leave when done; a slot
    removed before it finished is stopped; its arena range is reused."""
    from paper_0704_3444_amd import Batch

    runs = mixed_runs()
    b = Batch(storage="f32", max_comp=3, max_slots=4, arena_bytes=128 << 20, graph_steps=5)
    a = b.add(*runs[0])
    b.step(23)
    c = b.add(*runs[2])
    d = b.add(*runs[5])
    b.step(11)
    b.remove(d)  # stopped early
    e = b.add(*runs[3])
    out = drain(b, {a: runs[0][2], c: runs[2][2], e: runs[3][2]})
    b.close()
    for s, (p, r, steps) in ((a, runs[0]), (c, runs[2]), (e, runs[3])):
        ref = solo(p, r, steps, "f32", "tile")
        assert np.array_equal(out[s]["rho"], ref["rho"]), s


def test_batch_admission_by_footprint():
    from paper_0704_3444_amd import Batch, LBError, lb

    p, r, steps = mixed_runs()[2]
    probe = Batch(storage="f32", max_comp=3, max_slots=4, arena_bytes=1 << 20)
    fp = probe.footprint(p)
    probe.close()
    need = lb.lb_workspace_bytes(lb.make_params(p, storage="f32"))
    assert fp == (need + 255) // 256 * 256
    b = Batch(storage="f32", max_comp=3, max_slots=4, arena_bytes=2 * fp + 1000)
    s1 = b.add(p, r, steps)
    s2 = b.add(p, r, steps)
    assert b.try_add(p, r, steps) is None  # arena full
    with pytest.raises(LBError) as ei:
        b.add(p, r, steps)
    assert ei.value.code == lb.LB_ENOMEM
    out = drain(b, {s1: steps, s2: steps})
    b.remove(s1)
    s3 = b.try_add(p, r, steps)
    assert s3 is not None
    out3 = drain(b, {s3: steps})
    b.close()
    assert np.array_equal(out[s1]["rho"], out3[s3]["rho"])


def test_batch_autotuner_and_configurations():
    """Every configuration gives the same result; the tuner times them all,
    keeps the fastest, and the runs keep progressing correctly."""
    from paper_0704_3444_amd import Batch, lb_batch_config_count

    runs = mixed_runs()
    count = lb_batch_config_count("f32", 3)
    p, r, steps = runs[3]
    ref = solo(p, r, steps, "f32", "tile")["rho"]
    for config in range(count):
        b = Batch(storage="f32", max_comp=3, max_slots=2, arena_bytes=64 << 20, config=config, graph_steps=4)
        s = b.add(p, r, steps)
        out = drain(b, {s: steps})
        b.close()
        assert np.array_equal(out[s]["rho"], ref), config
    b = Batch(storage="f32", max_comp=3, max_slots=8, arena_bytes=256 << 20, graph_steps=4)
    long_steps = 400
    slots = {b.add(p2, r2, long_steps): long_steps for (p2, r2, _) in runs}
    best, ms = b.tune(3)
    print(f"[tune] best {best}, ms/step {np.round(ms, 4).tolist()}", flush=True)
    assert 0 <= best < count and np.all(ms > 0) and ms[best] == ms.min()
    out = drain(b, slots, chunk=50)
    b.close()
    p0, r0, _ = runs[0]
    first = min(slots)
    assert np.array_equal(out[first]["rho"], solo(p0, r0, long_steps, "f32", "tile")["rho"])


def test_batch_rejects_what_it_cannot_run():
    from paper_0704_3444_amd import Batch, LBError

    b = Batch(storage="f32", max_comp=2, max_slots=2, arena_bytes=64 << 20)
    p3, r3, _ = mixed_runs()[1]
    with pytest.raises(LBError) as ei:
        b.add(p3, r3, 10)  # N = 3 > max_comp
    assert ei.value.code == -3
    cfg, rho0 = LI.ternary_d3q19(8, chi=3.0)
    with pytest.raises(LBError):
        b.add(cfg, rho0, 10)
    p2, r2, _ = mixed_runs()[0]
    s = b.add(p2, r2, 50)
    with pytest.raises(LBError) as ei:
        b.moments(s)  # not finished
    assert ei.value.code == -1
    b.close()


@pytest.mark.parametrize("storage,tol", [("f32", TOL["f32"]), ("f16s", None)])
def test_serving_loop_each_result_same_alone_and_in_mix(storage, tol):
    """Continuous batching of a Poisson mix: every request completes, and
    its densities equal the same run alone (bit for bit) and the oracle
    within the storage's bar (shifted FP16: the rounding budget of the run,
    f16s_check)."""
    from paper_0704_3444_amd import serve

    reqs = LI.serving_mix(12, seed=77, rate_hz=400.0, side=(64, 160), steps=150)
    recs, summary = serve.serve_batched(reqs, storage=storage, max_slots=6, arena_bytes=96 << 20, chunk=20,
                                        graph_steps=10, keep_fields=True)
    print(f"[serve] {storage} {summary}", flush=True)
    assert summary["requests"] == 12 and summary["p99_ms"] >= summary["p50_ms"] > 0
    by_id = {x["id"]: x for x in recs}
    for r in reqs:
        rec = by_id[r["id"]]
        assert rec["status"] == 0 and rec["step"] == r["nsteps"]
        alone = solo(r["cfg"], r["rho0"], r["nsteps"], storage, "auto")
        assert np.array_equal(rec["rho"], alone["rho"]), r["id"]
    r = reqs[0]
    if storage == "f16s":
        o, budget = run_oracle_f16s_budget(r["cfg"], r["rho0"], r["nsteps"])
        d = (np.abs(by_id[r["id"]]["rho"] - o["rho"]) / o["rho"]).max(axis=1)
        ratio = float(np.max(d / (budget["rel"] + 1e-5)))
        print(f"[serve] f16s request {r['id']} density error / rounding bar {ratio:.3f}", flush=True)
        assert ratio < 1.0, ratio
        return
    o = run_oracle(r["cfg"], r["rho0"], r["nsteps"])
    err = float(np.max(np.abs(by_id[r["id"]]["rho"] - o["rho"]) / o["rho"]))
    print(f"[serve] {storage} request {r['id']} vs oracle {err:.2e}", flush=True)
    assert err < tol, err

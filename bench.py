"""Benchmark: per-edge typed 3/4-node graphlet counting on one MI355X.

One step = one tg_count call over the whole resident graph: preprocessing,
scheduling, typed triangles, node tables, typed 4-cycles, per-edge orbits and
graphlets (per-edge rows for every edge) and global counts (Eq. 17).  Inputs
are seeded synthetic graphs already in HBM when timing starts.

Prints one JSON line (see the design notes for every field).
"""
import argparse
import hashlib
import json
import os
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "edges/s and typed graphlets/s (k≤4) at 1 GPU; % HBM peak; learned vs plain schedule"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources whose change invalidates a stored HBM-traffic measurement of the
# combine phase (the kernel itself, its device helpers and its launch code).
_COMBINE_SOURCES = ("paper_1901_10026_amd/csrc/tg_combine.hip", "paper_1901_10026_amd/csrc/tg_device.h",
                    "paper_1901_10026_amd/csrc/tg_internal.h", "paper_1901_10026_amd/csrc/tg_api.hip")
_TRAFFIC_FILE = "profiles/combine_cl-1m_hbm_traffic.txt"


def combine_source_hash():
    h = hashlib.sha256()
    for rel in _COMBINE_SOURCES:
        with open(os.path.join(_ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(workload):
    """HBM bytes per combine phase from the committed rocprofv3 counter
    summary, or None when it is absent, is for another workload, or was
    taken on different kernel sources."""
    path = os.path.join(_ROOT, _TRAFFIC_FILE)
    if workload != "cl-1m" or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != combine_source_hash():
        return None
    try:
        return int(float(vals["traffic_bytes_per_phase"]))
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE
    and WRITE_SIZE counters."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def graph_stats(g):
    """Per-edge structural quantities used for algorithmic byte counts."""
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    n = g.n
    d = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int64), d)
    up = ci > src
    ei, ej = src[up], ci[up]
    return dict(n=n, m=len(ei), nnz=len(ci), deg=d, ei=ei, ej=ej)


# bytes of the common-neighbour lists the library keeps (12 B per entry of
# the bound, the shorter row's length, summed over the edges)
TLIST_BUDGET = 16 << 30


def keeps_lists(st):
    d = st["deg"]
    return 12 * int(np.minimum(d[st["ei"]], d[st["ej"]]).sum()) <= TLIST_BUDGET


def combine_bytes(st, L, tau_sum, lists):
    """Algorithmic bytes of the per-edge combine kernel (one launch = every
    edge): edge endpoints (8 B), row offsets of both ends (16 B), typed
    degree and node tables of both endpoints (2 x (4L + 16 L^2) B), the
    edge's own typed triangle counts (4L B) and typed 4-cycle counts (8P B),
    per member of T_ij its type (1 B), the typed triangle counts of (i,k) and
    (j,k) and the typed degree of k (12L B), and the written row (8R B).
    T_ij itself is either found by intersecting both CSR rows (4 B per id of
    either row) or, with the lists the tau pass keeps, read from that list
    (its offset, 8 B per edge, and 12 B per member: the id and two edge
    ids)."""
    P = L * (L + 1) // 2
    R = 2 * L + 6 * P
    d = st["deg"]
    per_edge_fixed = 8 + 16 + 2 * (4 * L + 16 * L * L) + 4 * L + 8 * P + 8 * R
    if lists:
        tset = 8 * st["m"] + 12 * tau_sum
    else:
        tset = 4 * (d[st["ei"]] + d[st["ej"]]).sum()
    return int(st["m"] * per_edge_fixed + tset + tau_sum * (1 + 12 * L))


def cpu_baseline(g, seconds, threads):
    """The oracle as it stands on a uniform random sample of edges, for a
    bounded time; returns edges/s over the sampled edges."""
    import oracle
    oracle.build(force=False)
    st = graph_stats(g)
    rng = np.random.default_rng(12345)
    done, t_used = 0, 0.0
    batch = 256
    while t_used < seconds:
        idx = rng.integers(0, st["m"], size=batch)
        t0 = time.perf_counter()
        oracle.count_edges(g.row_ptr, g.col_idx, g.types, g.L, st["ei"][idx].astype(np.int32),
                           st["ej"][idx].astype(np.int32), nthreads=threads)
        t_used += time.perf_counter() - t0
        done += batch
    return dict(value=done / t_used, unit="edges/s", cores=threads, kind="oracle",
                sample=f"{done} edges drawn uniformly (seed 12345) from the same graph, counted by the oracle's "
                       f"per-edge method (all rows) in {t_used:.1f} s on {threads} host threads")


def time_count(tg, g, rp, ci, ty, out_g, out_e, steps, per_edge=True, **kw):
    import torch
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    s0.record(stream)
    for _ in range(steps):
        tg.count(rp, ci, ty, g.L, per_edge=per_edge, out_global=out_g, out_edges=out_e, **kw)
    s1.record(stream)
    torch.cuda.synchronize()
    return s0.elapsed_time(s1) / steps


def compare_schedules(tg, g, rp, ci, ty, out_g, out_e, steps=5):
    """No cost order, the degree-product schedule and the learned schedule
    (MLP trained on a 1% edge sample), each with the default launch shapes,
    then degree and learned autotuned; the counts are the same in every
    case."""
    import torch
    res = {}
    res["none_ms"] = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="none")
    log(f"no cost order: {res['none_ms']:.1f} ms")
    res["degree_ms"] = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="degree")
    log(f"degree schedule: {res['degree_ms']:.1f} ms")
    t_deg, _ = tg.autotune(rp, ci, ty, g.L, out_g, out_e, schedule="degree")
    res["degree_autotuned_ms"] = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="degree", tuning=t_deg)
    res["degree_tuning"] = t_deg.as_dict()
    log(f"degree schedule, autotuned: {res['degree_autotuned_ms']:.1f} ms")
    model = tg.CostModel(seed=55)
    torch.cuda.synchronize()
    t0 = time.time()
    hist = model.train(rp, ci, ty, g.L, sample_frac=0.01, seed=56, epochs=15)
    res["mlp_train_ms"] = (time.time() - t0) * 1e3
    res["mlp_loss_first_last"] = [hist[0], hist[-1]]
    res["learned_ms"] = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="learned", model=model)
    log(f"learned schedule: {res['learned_ms']:.1f} ms")
    t_l, _ = tg.autotune(rp, ci, ty, g.L, out_g, out_e, schedule="learned", model=model)
    res["learned_autotuned_ms"] = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="learned",
                                             model=model, tuning=t_l)
    res["learned_tuning"] = t_l.as_dict()
    log(f"learned schedule, autotuned: {res['learned_autotuned_ms']:.1f} ms (training {res['mlp_train_ms']:.0f} ms)")
    return res


def outputs_leg(tg, g, rp, ci, ty, out_g, out_e, steps=3):
    """The two extra per-edge outputs on the same graph: orbit rows (g1..g12
    per type or type pair) written beside the graphlet rows, and the sparse
    (key, count) form of the graphlet rows."""
    import torch
    dev = rp.device
    W = tg.edge_orbit_width(g.L)
    orb = torch.empty((g.m, W), dtype=torch.uint64, device=dev)
    tg.count(rp, ci, ty, g.L, out_global=out_g, out_edges=out_e, out_orbits=orb)
    orbit_ms = time_count(tg, g, rp, ci, ty, out_g, out_e, steps, out_orbits=orb)
    del orb
    log(f"graphlet + orbit rows: {orbit_ms:.1f} ms")
    _, _, ends = tg.count(rp, ci, ty, g.L, out_global=out_g, out_edges=out_e, endpoints=True)
    off, keys, cnts = tg.rows_sparse(out_e, ends, ty, g.L)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(steps):
        off, keys, cnts = tg.rows_sparse(out_e, ends, ty, g.L)
    s1.record()
    torch.cuda.synchronize()
    sparse_ms = s0.elapsed_time(s1) / steps
    pairs = int(keys.numel())
    per_edge = torch.diff(off)
    res = {"orbit_width": W, "count_with_orbits_ms": orbit_ms, "sparse_ms": sparse_ms, "sparse_pairs": pairs,
           "sparse_pairs_per_edge_mean": pairs / g.m, "sparse_pairs_per_edge_max": int(per_edge.max().item()),
           "sparse_bytes": pairs * 12 + (g.m + 1) * 8, "dense_row_bytes": g.m * out_e.shape[1] * 8}
    log(f"sparse rows: {pairs} pairs ({pairs / g.m:.1f} per edge), {sparse_ms:.1f} ms")
    return res


def global_leg(tg, g, rp, ci, ty, out_g, steps=3):
    """Global counts alone on the same graph: tg_count_global (each instance
    counted a fixed number of times) against tg_count without per-edge rows;
    both must give the global vector of the timed step."""
    import torch
    want = out_g.clone()
    glob = torch.empty_like(out_g)
    tg.count_global(rp, ci, ty, g.L, out=glob)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    phases = {}
    s0.record()
    for _ in range(steps):
        ph = {}
        tg.count_global(rp, ci, ty, g.L, out=glob, phase_ms=ph)
        for k, v in ph.items():
            phases[k] = phases.get(k, 0.0) + v / steps
    s1.record()
    torch.cuda.synchronize()
    once_ms = s0.elapsed_time(s1) / steps
    same = bool(torch.equal(glob.view(torch.int64), want.view(torch.int64)))
    per_edge_ms = time_count(tg, g, rp, ci, ty, glob, None, steps, per_edge=False)
    same = same and bool(torch.equal(glob.view(torch.int64), want.view(torch.int64)))
    log(f"global only: counted once {once_ms:.1f} ms, per-edge path without rows {per_edge_ms:.1f} ms, equal={same}")
    return {"count_global_ms": once_ms, "count_global_edges_per_s": g.m / (once_ms * 1e-3),
            "count_global_phase_ms": phases, "per_edge_path_global_only_ms": per_edge_ms, "equal": same}


def null_leg(tg, g, rp, ci, ty, permutations=100, seed=2024):
    """Type-permutation null model on the same graph: global counts under
    `permutations` seeded random permutations of the node types (one
    tg_count_global_types call) and their mean; the first two permutations
    are checked against separate tg_count_global calls."""
    import torch
    perms = tg.type_permutations(g.types, permutations, seed)
    tv = torch.from_numpy(perms).to(rp.device)
    counts, mean = tg.count_global_types(rp, ci, tv[:2].contiguous(), g.L)   # warm-up
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    counts, mean = tg.count_global_types(rp, ci, tv, g.L)
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1)
    same = all(bool(torch.equal(counts[b].view(torch.int64),
                                tg.count_global(rp, ci, tv[b].contiguous(), g.L).view(torch.int64)))
               for b in range(2))
    actual = tg.count_global(rp, ci, ty, g.L).cpu().numpy().view(np.uint64).astype(np.float64)
    mu = mean.cpu().numpy()
    # keys that occur under the real types but never in any permutation, and
    # the reverse (the paper's "forbidden" typed motifs)
    occurs = counts.view(torch.int64).ne(0).any(dim=0).cpu().numpy()
    log(f"null model: {permutations} permutations in {ms:.0f} ms ({ms / permutations:.1f} ms each), equal={same}")
    return {"permutations": permutations, "seed": seed, "ms": ms, "ms_per_permutation": ms / permutations,
            "equal_to_single_calls": same, "keys_only_in_real": int(((actual > 0) & ~occurs).sum()),
            "keys_only_in_permuted": int(((actual == 0) & occurs).sum()),
            "keys_nonzero_real": int((actual > 0).sum()), "keys_nonzero_mean": int((mu > 0).sum())}


def directed_leg(tg, g, rp, ci, ty, steps=3):
    """Directed typed 3-node graphlets on the same graph oriented by a seeded
    draw (20% of edges reciprocal, the rest one arc in a random direction):
    per-edge rows (15 L columns) and global counts."""
    import torch

    import graphgen
    sd = torch.from_numpy(graphgen.orient(g.row_ptr, g.col_idx, 99, 0.2)).to(rp.device)
    K = tg.directed3_num_keys(g.L)
    glob, rows, _ = tg.count_directed3(rp, ci, sd, ty, g.L)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    phases = {}
    s0.record()
    for _ in range(steps):
        ph = {}
        tg.count_directed3(rp, ci, sd, ty, g.L, phase_ms=ph)
        for k, v in ph.items():
            phases[k] = phases.get(k, 0.0) + v / steps
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / steps
    log(f"directed 3-node: {ms:.1f} ms ({K} keys, rows of {15 * g.L})")
    del rows
    return {"orientation": "seed 99, 20% reciprocal", "keys": K, "row_width": 15 * g.L, "ms": ms,
            "edges_per_s": g.m / (ms * 1e-3), "phase_ms": {k: v for k, v in phases.items() if v > 0}}


def giant_schedules_leg(tg, dev, frac=0.01, seed=31):
    """The 20M-node skewed graph: per-edge rows of a seeded uniform edge
    sample (rows only; its rows for all edges would not fit) under the
    degree-product schedule and the learned one (MLP trained on a 1% edge
    sample of the same graph), with identical rows."""
    import torch

    import graphgen
    t0 = time.time()
    g = graphgen.workload("cl-20m")
    log(f"cl-20m: n={g.n} m={g.m} ({time.time() - t0:.0f} s to generate)")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ty = torch.from_numpy(g.types).to(dev)
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(g.m, size=int(g.m * frac), replace=False)).astype(np.int64)
    d_ids = torch.from_numpy(ids).to(dev)
    model = tg.CostModel(seed=57)
    torch.cuda.synchronize()
    t0 = time.time()
    model.train(rp, ci, ty, g.L, sample_frac=0.01, seed=58, epochs=15)
    train_ms = (time.time() - t0) * 1e3
    res = {"workload": "cl-20m", "sample_edges": len(ids), "mlp_train_ms": train_ms}
    rows = {}
    for sched in ("degree", "learned"):
        ph = {}
        torch.cuda.synchronize()
        t0 = time.time()
        _, r, _ = tg.count(rp, ci, ty, g.L, edge_ids=d_ids, global_counts=False, schedule=sched,
                           model=model if sched == "learned" else None, phase_ms=ph)
        torch.cuda.synchronize()
        res[sched] = {"ms": (time.time() - t0) * 1e3, "phase_ms": ph}
        rows[sched] = r
        log(f"cl-20m sample, {sched} schedule: " + " ".join(f"{k}={v:.0f}ms" for k, v in ph.items()))
    res["equal"] = bool(torch.equal(rows["degree"].view(torch.int64), rows["learned"].view(torch.int64)))
    log(f"cl-20m rows identical under both schedules: {res['equal']}")
    return res


def giant_global_leg(tg, dev):
    """The 20M-node skewed graph counted in full for its global counts alone
    (tg_count_global), with its 8 types and again with one type: the typed
    counts of each shape must add up to the untyped one."""
    import torch

    import graphgen
    g = graphgen.workload("cl-20m")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ty = torch.from_numpy(g.types).to(dev)
    res = {"workload": "cl-20m", "n": g.n, "m": g.m, "L": g.L}
    out = {}
    for label, types, L in (("typed", ty, g.L), ("untyped", torch.zeros_like(ty), 1)):
        ph = {}
        torch.cuda.synchronize()
        t0 = time.time()
        glob = tg.count_global(rp, ci, types, L, phase_ms=ph)
        torch.cuda.synchronize()
        res[label] = {"ms": (time.time() - t0) * 1e3, "phase_ms": ph}
        out[label] = glob.cpu().numpy().view(np.uint64)
        log(f"cl-20m global counts, {label}: {res[label]['ms']:.0f} ms (" +
            " ".join(f"{k}={v:.0f}" for k, v in ph.items()) + ")")
    per_shape = {}
    for k in range(len(out["typed"])):
        sh = tg.key_decode(g.L, k)[0]
        per_shape[sh] = per_shape.get(sh, 0) + int(out["typed"][k])
    res["per_shape"] = [per_shape.get(sh, 0) for sh in range(8)]
    res["untyped"]["counts"] = [int(x) for x in out["untyped"]]
    res["partition_holds"] = res["per_shape"] == res["untyped"]["counts"]
    log(f"cl-20m typed counts add up to the untyped ones per shape: {res['partition_holds']}")
    return res


def batch_leg(tg, dev, steps=3):
    """100,000 small typed graphs (n log-uniform in [10, 500], density
    U(0.02, 0.3), L uniform in 2..8) counted by tg_count_batch, autotuned."""
    import torch

    import graphgen
    b = graphgen.batch_gnp(100_000, 10, 500, 0.02, 0.3, 2, 8, 4)
    key_off = tg.key_offsets(b.L)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    args = (t(b.node_off, np.int64), t(b.slot_off, np.int64), t(b.row_ptr, np.int32), t(b.col_idx, np.int32),
            t(b.types, np.uint8), t(b.L, np.uint8), t(key_off, np.int64))
    out = torch.empty(int(key_off[-1]), dtype=torch.uint64, device=dev)
    tg.count_batch(*args, out=out)
    tuning, _ = tg.autotune_batch(*args, out)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(steps):
        tg.count_batch(*args, out=out, tuning=tuning)
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / steps
    m = int(b.slot_off[-1]) // 2
    log(f"batch: {b.G} graphs, {m} edges, {ms:.1f} ms")
    return {"workload": "gnp-batch-100k", "graphs": b.G, "edges": m, "ms_per_call": ms,
            "graphs_per_s": b.G / (ms * 1e-3), "edges_per_s": m / (ms * 1e-3), "tuning": tuning.as_dict()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl-1m")
    ap.add_argument("--schedule", default="degree", choices=["none", "degree", "learned"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the schedule comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-small-graphs leg")
    ap.add_argument("--no-outputs", action="store_true", help="skip the orbit-row and sparse-row leg")
    ap.add_argument("--no-global", action="store_true", help="skip the global-counts-only leg")
    ap.add_argument("--no-null", action="store_true", help="skip the type-permutation null-model leg")
    ap.add_argument("--no-directed", action="store_true", help="skip the directed 3-node leg")
    ap.add_argument("--giant-global", action="store_true",
                    help="also count the 20M-node graph's global counts in full, typed and untyped (minutes)")
    ap.add_argument("--giant-schedules", action="store_true",
                    help="also compare the degree and learned schedules on a 1%% edge sample of the 20M-node graph "
                         "(several minutes)")
    ap.add_argument("--permutations", type=int, default=100, help="permutations of the null-model leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (edges would shard by range, "
              "with one all-reduce of the global key vector); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch

    import graphgen
    import paper_1901_10026_amd as tg

    graphgen.build(force=False)
    dev = torch.device("cuda:0")
    t0 = time.time()
    g = graphgen.workload(args.workload)
    log(f"workload {g.name}: n={g.n} m={g.m} L={g.L} max_deg={int(np.diff(g.row_ptr).max())} "
        f"({time.time() - t0:.1f} s to generate)")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ty = torch.from_numpy(g.types).to(dev)
    K, R = tg.num_keys(g.L), tg.edge_row_width(g.L)
    out_g = torch.empty(K, dtype=torch.uint64, device=dev)
    out_e = torch.empty((g.m, R), dtype=torch.uint64, device=dev)
    torch.cuda.synchronize()

    def step(phases=None):
        tg.count(rp, ci, ty, g.L, per_edge=True, schedule=args.schedule, out_global=out_g, out_edges=out_e,
                 phase_ms=phases)

    for w in range(args.warmup):
        step()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    phase_acc = {}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        ph = {}
        step(ph)
        for k, v in ph.items():
            phase_acc[k] = phase_acc.get(k, 0.0) + v
        log(f"step {s + 1}/{args.steps}: " + " ".join(f"{k}={v:.2f}ms" for k, v in ph.items()))
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end) / args.steps
    phases = {k: v / args.steps for k, v in phase_acc.items()}
    glob = out_g.cpu().numpy().view(np.uint64)
    total_graphlets = int(sum(int(x) for x in glob))
    # |T_ij| summed over edges = 3 x number of triangles
    tri_keys = [k for k in range(K) if tg.key_decode(g.L, k)[0] == 1]
    tau_sum = 3 * int(sum(int(glob[k]) for k in tri_keys))
    st = graph_stats(g)
    lists = keeps_lists(st)
    cb = combine_bytes(st, g.L, tau_sum, lists)
    comb_ms = phases.get("combine", 0.0)
    achieved = cb / (comb_ms * 1e-3) / 1e9 if comb_ms > 0 else 0.0
    traffic = stored_traffic(g.name)
    # the counters' HBM bytes over this run's phase time (the counters come
    # from a separate profiled run of the same sources)
    traffic_gbs = traffic / (comb_ms * 1e-3) / 1e9 if traffic and comb_ms > 0 else None
    rec = {
        "metric": METRIC,
        "value": g.m / (ms * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "m": g.m, "L": g.L, "schedule": args.schedule,
                   "model": g.meta.get("model"), "gamma": g.meta.get("gamma"), "wmax": g.meta.get("wmax"),
                   "types": g.meta.get("types")},
        "typed_graphlets_per_s": total_graphlets / (ms * 1e-3),
        "typed_graphlets": total_graphlets,
        "phase_ms": phases,
        "roofline": {"bound": "hbm",
                     "kernel": "combine phase: gather kernels k_combine<16>, k_combine<64>, k_combine<256> and "
                               "their k_combine_rows launches, together every edge once",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes": cb, "phase_ms": comb_ms, "traffic": traffic,
                     "traffic_gbs": traffic_gbs,
                     "traffic_frac": traffic_gbs / HBM_PEAK_GBS if traffic_gbs else None,
                     "t_ij_from": "kept lists" if lists else "row intersection"},
    }
    if not args.no_compare:
        rec["schedules"] = compare_schedules(tg, g, rp, ci, ty, out_g, out_e)
    if not args.no_global:
        rec["global_only"] = global_leg(tg, g, rp, ci, ty, out_g)
    if not args.no_null:
        rec["null_model"] = null_leg(tg, g, rp, ci, ty, permutations=args.permutations)
    if not args.no_directed:
        rec["directed3"] = directed_leg(tg, g, rp, ci, ty)
    if not args.no_outputs:
        rec["outputs"] = outputs_leg(tg, g, rp, ci, ty, out_g, out_e)
    if args.giant_global:
        rec["giant_global"] = giant_global_leg(tg, dev)
    if args.giant_schedules:
        rec["giant_schedules"] = giant_schedules_leg(tg, dev)
    if not args.no_batch:
        rec["batch"] = batch_leg(tg, dev)
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"cpu baseline: oracle for ~{args.cpu_seconds:.0f} s on {threads} threads")
        rec["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds, threads)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

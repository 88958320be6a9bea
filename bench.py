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


# Sources whose change invalidates a stored traffic measurement: the device
# code of tg_count's kernels and their helpers (the host launch code in
# tg_api.hip is not hashed).
_KERNEL_SOURCES = ("paper_1901_10026_amd/csrc/tg_combine.hip", "paper_1901_10026_amd/csrc/tg_clique.hip",
                   "paper_1901_10026_amd/csrc/tg_c4part.hip", "paper_1901_10026_amd/csrc/tg_kernels.hip",
                   "paper_1901_10026_amd/csrc/tg_device.h", "paper_1901_10026_amd/csrc/tg_internal.h")
_TRAFFIC_FILE = "profiles/tg_count_cl-1m_l2_traffic.txt"
# kernels of each timed phase of tg_count (rocprofv3 kernel-name prefixes)
PHASE_KERNELS = {
    "cycles": ("k_c4_hash", "k_c4_group", "k_c4_bwalk", "k_c4_bcount", "k_c4_slot_wedges", "k_c4_fold", "k_fill_u32",
               "k_fill_u64"),
    "cliques": ("k_k4_low", "k_k4_tier", "k_k4_zero", "k_max_tsum_all"),
    "combine": ("k_combine",),
}


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in _KERNEL_SOURCES:
        with open(os.path.join(_ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(workload):
    """L2-egress bytes per call of each phase (FETCH_SIZE and WRITE_SIZE
    counters, scaled by a plain copy) from the committed rocprofv3 summary,
    as {phase: bytes}; None when it is absent, is for another workload, or
    was taken on different kernel sources."""
    path = os.path.join(_ROOT, _TRAFFIC_FILE)
    if workload != "cl-1m" or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    out = {}
    for ph in PHASE_KERNELS:
        try:
            out[ph] = int(float(vals[f"traffic_bytes.{ph}"]))
        except (KeyError, ValueError):
            pass
    return out or None


def _kernel_name(full):
    """'void tg::k_x<1, int>(args...)' -> 'k_x<1, int>'."""
    name = full[5:] if full.startswith("void ") else full
    name = name.replace("tg::", "").replace("(anonymous namespace)::", "")
    return name.split("(", 1)[0].strip()


def _read_counter_csv(path, counter):
    """Per kernel-name (template arguments cut) sums of one rocprofv3 counter
    (KiB) and dispatch counts, from its counter_collection.csv."""
    import csv
    sums, calls = {}, {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = _kernel_name(row["Kernel_Name"])
            sums[name] = sums.get(name, 0.0) + float(row["Counter_Value"])
            calls[name] = calls.get(name, 0) + 1
    return sums, calls


def summarize_trace(stats_csv, calls_per_run):
    """Prints a per-kernel summary of a rocprofv3 --kernel-trace --stats run
    (its kernel_stats.csv): calls, total and per-tg_count-call milliseconds,
    and the phase totals."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"{'kernel':60s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'ms_per_call':>11s} {'pct':>6s}")
    per_phase = {ph: 0.0 for ph in PHASE_KERNELS}
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = _kernel_name(r["Name"])
        t = float(r["TotalDurationNs"]) / 1e6
        print(f"{name[:60]:60s} {int(r['Calls']):6d} {t:10.3f} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{t / calls_per_run:11.3f} {100 * t * 1e6 / total:6.2f}")
        for ph, prefixes in PHASE_KERNELS.items():
            if any(name.startswith(pf) for pf in prefixes):
                per_phase[ph] += t / calls_per_run
    for ph, t in per_phase.items():
        print(f"# phase {ph} (kernels {', '.join(PHASE_KERNELS[ph])}): {t:.3f} ms per tg_count call")


def summarize_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, calls_per_run):
    """Prints the L2-egress summary from four rocprofv3 --pmc runs (FETCH_SIZE
    and WRITE_SIZE of tg_count, then of a plain device copy of copy_bytes
    bytes done 3 times), per kernel and per phase, with the source hash."""
    f, fc = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    w, _ = _read_counter_csv(write_csv, "WRITE_SIZE")
    cf, cfc = _read_counter_csv(copy_fetch_csv, "FETCH_SIZE")
    cw, cwc = _read_counter_csv(copy_write_csv, "WRITE_SIZE")
    ck = max(cf, key=lambda k: cf[k])
    fetch_scale = copy_bytes / (cf[ck] / cfc[ck] * 1024.0)
    write_scale = copy_bytes / (cw[ck] / cwc[ck] * 1024.0)
    print(f"# copy kernel {ck}: FETCH_SIZE {cf[ck] / cfc[ck]:.1f} KiB and WRITE_SIZE {cw[ck] / cwc[ck]:.1f} KiB "
          f"per copy of {copy_bytes} bytes")
    print(f"# scale factors (bytes moved / counter bytes): fetch {fetch_scale:.4f}, write {write_scale:.4f}")
    print("# L2 egress (requests leaving L2, MALL hits included), per call of tg_count")
    print(f"{'kernel':60s} {'calls':>6s} {'FETCH_KiB':>14s} {'WRITE_KiB':>14s} {'scaled_GB':>10s}")
    per_phase = {ph: 0.0 for ph in PHASE_KERNELS}
    for k in sorted(f, key=lambda k: -(f[k] * fetch_scale + w.get(k, 0.0) * write_scale)):
        fk, wk = f[k] / calls_per_run, w.get(k, 0.0) / calls_per_run
        b = (fk * fetch_scale + wk * write_scale) * 1024.0
        print(f"{k[:60]:60s} {fc[k] / calls_per_run:6.0f} {fk:14.1f} {wk:14.1f} {b / 1e9:10.2f}")
        for ph, prefixes in PHASE_KERNELS.items():
            if any(k.startswith(pf) for pf in prefixes):
                per_phase[ph] += b
    for ph, b in per_phase.items():
        print(f"# phase {ph}: kernels {', '.join(PHASE_KERNELS[ph])}")
        print(f"traffic_bytes.{ph}: {int(b)}")
    print(f"source_sha256: {kernel_source_hash()}")


LDS_COUNTERS = ("SQ_INSTS_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_ADDR_CONFLICT",
                "SQ_ACTIVE_INST_LDS", "SQ_WAVES", "GRBM_GUI_ACTIVE")


def summarize_lds(csv_path, calls_per_run, cus=256):
    """Prints per-kernel LDS figures from one rocprofv3 --pmc run of the LDS
    counters: LDS instructions, the fraction of CU-cycles in which the LDS
    served indexed accesses (SQ_LDS_IDX_ACTIVE over GRBM_GUI_ACTIVE x CUs,
    the share of the LDS's peak rate in use), and the share of those cycles
    stalled by bank conflicts."""
    vals = {c: _read_counter_csv(csv_path, c)[0] for c in LDS_COUNTERS}
    calls = _read_counter_csv(csv_path, "SQ_INSTS_LDS")[1]
    print(f"{'kernel':60s} {'calls':>6s} {'lds_insts':>12s} {'lds_busy':>9s} {'bank_confl':>10s} {'waves':>10s}")
    for k in sorted(calls, key=lambda k: -vals["SQ_LDS_IDX_ACTIVE"].get(k, 0.0)):
        gui = vals["GRBM_GUI_ACTIVE"].get(k, 0.0)
        act = vals["SQ_LDS_IDX_ACTIVE"].get(k, 0.0)
        if act <= 0 or gui <= 0:
            continue
        busy = act / (gui * cus)
        conf = vals["SQ_LDS_BANK_CONFLICT"].get(k, 0.0) / act
        print(f"{k[:60]:60s} {calls[k] / calls_per_run:6.0f} {vals['SQ_INSTS_LDS'].get(k, 0.0) / calls_per_run:12.4g} "
              f"{busy:9.4f} {conf:10.4f} {vals['SQ_WAVES'].get(k, 0.0) / calls_per_run:10.4g}")
    print(f"source_sha256: {kernel_source_hash()}")


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
    """Per-edge structural quantities used for algorithmic byte counts:
    canonical edges, degrees, and out-degrees d+ in the degree order (u
    before v when (d_u, u) < (d_v, v))."""
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    n = g.n
    d = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int64), d)
    up = ci > src
    ei, ej = src[up], ci[up]
    rank = np.empty(n, dtype=np.int64)
    rank[np.lexsort((np.arange(n), d))] = np.arange(n)
    higher = rank[ci] > rank[src]
    dplus = np.bincount(src[higher], minlength=n).astype(np.int64)
    return dict(n=n, m=len(ei), nnz=len(ci), deg=d, ei=ei, ej=ej, src=src, col=ci, rank=rank, dplus=dplus,
                higher=higher)


def cycle_wedges(st):
    """Wedges x-u-w of the 4-cycle pass, x the highest-ranked node: scanned
    (every w of u's row, for every higher neighbour x of u: sum of
    d_u d+_u) and oriented (w below x as well)."""
    d, dplus = st["deg"], st["dplus"]
    scanned = int((d * dplus).sum())
    # slot (u, x) with x above u: the w of u's row below x are the slots of
    # u's row that sort before x by rank
    src, rank = st["src"], st["rank"]
    order = np.lexsort((rank[st["col"]], src))
    rp = np.concatenate([[0], np.cumsum(d)])
    pos = np.arange(len(order), dtype=np.int64) - rp[src[order]]
    oriented = int(pos[st["higher"][order]].sum())
    return scanned, oriented


# bytes of the common-neighbour lists the library keeps (12 B per entry of
# the bound, the shorter row's length, summed over the edges)
TLIST_BUDGET = 16 << 30


def keeps_lists(st):
    d = st["deg"]
    return 12 * int(np.minimum(d[st["ei"]], d[st["ej"]]).sum()) <= TLIST_BUDGET


def combine_bytes(st, L, tau_sum, lists, k4_width=0, probes=0):
    """Algorithmic bytes of the per-edge combine phase (gather and row
    kernels, every edge once): edge endpoints (8 B), row offsets of both ends
    (16 B), typed degree and node tables of both endpoints (2 x (4L + 16 L^2)
    B), the edge's own typed triangle counts (4L B) and typed 4-cycle counts
    (8P B), per member of T_ij its type (1 B), the typed triangle counts of
    (i,k) and (j,k) and the typed degree of k (12L B), and the written row
    (8R B).  T_ij itself is either found by intersecting both CSR rows (4 B
    per id of either row) or, with the lists the tau pass keeps, read from
    that list (its offset, 8 B per edge, and 12 B per member: the id and two
    slots).  The typed 4-cliques of the edge are either read from the clique
    pass's counters (k4_width B for each of the P type pairs) or, with
    k4_width = 0, found by out-list probes: the out-list offsets of every
    member (8 B) and 4 B per probe (`probes` = sum over edges of the
    out-degrees of T_ij's members)."""
    P = L * (L + 1) // 2
    R = 2 * L + 6 * P
    d = st["deg"]
    per_edge_fixed = 8 + 16 + 2 * (4 * L + 16 * L * L) + 4 * L + 8 * P + 8 * R
    if lists:
        tset = 8 * st["m"] + 12 * tau_sum
    else:
        tset = 4 * (d[st["ei"]] + d[st["ej"]]).sum()
    if k4_width:
        cliques = st["m"] * P * k4_width
    else:
        cliques = 8 * tau_sum + 4 * probes
    return int(st["m"] * per_edge_fixed + tset + tau_sum * (1 + 12 * L) + cliques)


def clique_probes(st, tri):
    """Out-list probes of the per-edge 4-clique search: the out-degrees of
    T_ij's members summed over the edges, i.e. sum over nodes k of d+_k
    times the number of triangles at k (tri)."""
    return int((st["dplus"] * np.asarray(tri, dtype=np.int64)).sum())


def cycles_bytes(st, L, scanned, oriented, c4_width):
    """Algorithmic bytes of the typed 4-cycle phase: per scanned wedge the
    far end's id and degree in the counting and in the crediting walk (16 B),
    per oriented wedge one 16-bit count update (4 B), a read of the far end's
    count row (16-bit per type, 2L B) and its type (1 B), and per edge the
    fold of its two slot rows into one (3 P counters of c4_width B).  The
    credit atomics, whose number depends on the cycles found, are left out:
    a lower bound."""
    P = L * (L + 1) // 2
    return int(16 * scanned + oriented * (4 + 2 * L + 1) + 3 * st["m"] * P * c4_width)


def clique_bytes(st, L, k4_width):
    """Algorithmic bytes of the clique pass: per node its out-list ids and
    types (5 B each), per member b of a node's out-list b's out-list offsets
    (8 B) and out-list, read in both passes (8 d+_b B): sum over b of
    d-_b (8 + 8 d+_b) with d-_b = d_b - d+_b lower neighbours, and the
    per-edge counters cleared and flushed (2 P k4_width B per edge).  The
    credits of the edges inside each out-list (data-dependent) are left out:
    a lower bound."""
    P = L * (L + 1) // 2
    d, dplus = st["deg"], st["dplus"]
    dminus = d - dplus
    return int(5 * st["m"] + (dminus * (8 + 8 * dplus)).sum() + 2 * st["m"] * P * k4_width)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
    return dict(value=done / t_used, unit="edges/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
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
    # three more of each, interleaved, for the run-to-run spread
    dr, lr = [res["degree_autotuned_ms"]], [res["learned_autotuned_ms"]]
    for _ in range(3):
        dr.append(time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="degree", tuning=t_deg))
        lr.append(time_count(tg, g, rp, ci, ty, out_g, out_e, steps, schedule="learned", model=model, tuning=t_l))
    res["degree_autotuned_runs_ms"], res["learned_autotuned_runs_ms"] = dr, lr
    spread = max(dr) - min(dr)
    gain = float(np.mean(dr) - np.mean(lr))
    res["degree_autotuned_spread_ms"] = spread
    res["learned_gain_ms"] = gain
    res["learned_gain_over_spread"] = gain / spread if spread > 0 else None
    log(f"autotuned, 4 runs each: degree {np.mean(dr):.1f} ms (spread {spread:.2f}), learned {np.mean(lr):.1f} ms")
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


def directed4_leg(tg, dev, steps=3):
    """Directed typed 4-node graphlets on the 2000-node Chung-Lu graph (L = 3)
    oriented by a seeded draw (20% of edges reciprocal): per-edge rows over
    every directed typed 4-node key and global counts."""
    import torch

    import graphgen
    g = graphgen.chung_lu_small()
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ty = torch.from_numpy(g.types).to(dev)
    sd = torch.from_numpy(graphgen.orient(g.row_ptr, g.col_idx, 23, 0.2)).to(dev)
    glob, rows, _ = tg.count_directed4(rp, ci, sd, ty, g.L, per_edge=True)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(steps):
        tg.count_directed4(rp, ci, sd, ty, g.L, per_edge=True)
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / steps
    K = tg.directed4_num_keys(g.L)
    sets = int(glob.view(torch.int64).sum().item())
    log(f"directed 4-node (cl-2k oriented): {ms:.2f} ms, {K} keys, {sets} sets")
    return {"workload": "cl-2k", "orientation": "seed 23, 20% reciprocal", "L": g.L, "keys": K, "ms": ms,
            "edges_per_s": g.m / (ms * 1e-3), "directed_sets": sets,
            "nonzero_keys": int(glob.view(torch.int64).ne(0).sum().item())}


def partite_leg(tg, dev, steps=3):
    """The two part-structured graphs (bipartite 50M edges, L = 2;
    3-partite 30M edges, L = 3): per-edge rows for every edge and global
    counts, per call, with the phase times."""
    import torch

    import graphgen
    res = {}
    for name in ("bip-50m", "tri-30m"):
        t0 = time.time()
        g = graphgen.workload(name)
        gen_s = time.time() - t0
        rp = torch.from_numpy(g.row_ptr).to(dev)
        ci = torch.from_numpy(g.col_idx).to(dev)
        ty = torch.from_numpy(g.types).to(dev)
        out_g = torch.empty(tg.num_keys(g.L), dtype=torch.uint64, device=dev)
        out_e = torch.empty((g.m, tg.edge_row_width(g.L)), dtype=torch.uint64, device=dev)
        tg.count(rp, ci, ty, g.L, out_global=out_g, out_edges=out_e)
        ms = time_count(tg, g, rp, ci, ty, out_g, out_e, steps)
        ph = {}
        tg.count(rp, ci, ty, g.L, out_global=out_g, out_edges=out_e, phase_ms=ph)
        torch.cuda.synchronize()
        res[name] = {"n": g.n, "m": g.m, "L": g.L, "max_degree": int(np.diff(g.row_ptr).max()), "generate_s": gen_s,
                     "ms": ms, "edges_per_s": g.m / (ms / 1e3), "phase_ms": ph}
        log(f"{name}: m={g.m} {ms:.1f} ms per call ({g.m / (ms / 1e3) / 1e6:.1f} M edges/s)")
        del rp, ci, ty, out_g, out_e
        tg.release_scratch()
    return res


def giant_per_edge_leg(tg, dev, rows_edges=100_000, repeats=1, learned=True):
    """The 20M-node skewed graph (300M edges, L = 8) through the whole
    per-edge path: one tg_count over every edge, with global counts from the
    per-edge sums (Eq. 17) and per-edge rows for the first `rows_edges`
    canonical edges, under the degree-product schedule and under the learned
    one (MLP trained on a 1% edge sample of the same graph).  Counts and rows
    must be identical; each call is timed with HIP events on the stream, and
    the degree call is repeated `repeats` times for its spread."""
    import torch

    import graphgen
    t0 = time.time()
    g = graphgen.workload("cl-20m")
    gen_s = time.time() - t0
    d = np.diff(g.row_ptr)
    log(f"cl-20m: n={g.n} m={g.m} max_deg={int(d.max())} ({gen_s:.0f} s to generate)")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    ty = torch.from_numpy(g.types).to(dev)
    K, R = tg.num_keys(g.L), tg.edge_row_width(g.L)
    res = {"workload": "cl-20m", "n": g.n, "m": g.m, "L": g.L, "max_degree": int(d.max()),
           "rows_for_edges": rows_edges, "generate_s": gen_s}
    outs = {}

    def one(sched, model=None):
        out_g = torch.empty(K, dtype=torch.uint64, device=dev)
        out_e = torch.empty((rows_edges, R), dtype=torch.uint64, device=dev)
        ph = {}
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        tg.count(rp, ci, ty, g.L, per_edge=True, edge_range=(0, rows_edges), schedule=sched, model=model,
                 out_global=out_g, out_edges=out_e, phase_ms=ph)
        s1.record()
        torch.cuda.synchronize()
        ms = s0.elapsed_time(s1)
        free, total_mem = torch.cuda.mem_get_info()
        res["device_bytes_used_after_call"] = int(total_mem - free)
        return ms, ph, out_g, out_e

    runs = []
    for r in range(max(1, repeats)):
        ms, ph, og, oe = one("degree")
        runs.append(ms)
        log(f"cl-20m per-edge path, degree schedule: {ms / 1e3:.1f} s (" +
            " ".join(f"{k}={v / 1e3:.1f}s" for k, v in ph.items() if v > 0) + ")")
        outs["degree"] = (og, oe)
        res["degree"] = {"ms": ms, "phase_ms": ph}
    res["degree"]["ms_runs"] = runs
    tg.release_scratch()
    if not learned:
        return res
    model = tg.CostModel(seed=57)
    torch.cuda.synchronize()
    t0 = time.time()
    model.train(rp, ci, ty, g.L, sample_frac=0.01, seed=58, epochs=15)
    res["mlp_train_ms"] = (time.time() - t0) * 1e3
    ms, ph, og, oe = one("learned", model)
    outs["learned"] = (og, oe)
    res["learned"] = {"ms": ms, "phase_ms": ph}
    log(f"cl-20m per-edge path, learned schedule: {ms / 1e3:.1f} s (" +
        " ".join(f"{k}={v / 1e3:.1f}s" for k, v in ph.items() if v > 0) + f"), training {res['mlp_train_ms']:.0f} ms")
    res["equal"] = bool(torch.equal(outs["degree"][0].view(torch.int64), outs["learned"][0].view(torch.int64)) and
                        torch.equal(outs["degree"][1].view(torch.int64), outs["learned"][1].view(torch.int64)))
    glob = outs["degree"][0].cpu().numpy().view(np.uint64)
    total = int(sum(int(x) for x in glob))
    res["typed_graphlets"] = total
    # the phases a schedule decides: the edge order of the combine step and
    # the ordering itself (the other phases do the same work under both)
    res["scheduled_phases_ms"] = {k: res[k]["phase_ms"].get("schedule", 0.0) + res[k]["phase_ms"].get("combine", 0.0)
                                  for k in ("degree", "learned")}
    res["learned_gain_scheduled_phases"] = 1.0 - res["scheduled_phases_ms"]["learned"] / res["scheduled_phases_ms"][
        "degree"]
    log(f"cl-20m schedule + combine phases: degree {res['scheduled_phases_ms']['degree'] / 1e3:.2f} s, learned "
        f"{res['scheduled_phases_ms']['learned'] / 1e3:.2f} s")
    res["edges_per_s"] = {k: g.m / (res[k]["ms"] * 1e-3) for k in ("degree", "learned")}
    res["typed_graphlets_per_s"] = {k: total / (res[k]["ms"] * 1e-3) for k in ("degree", "learned")}
    log(f"cl-20m: rows and global counts identical under both schedules: {res['equal']}")
    del outs, rp, ci, ty
    tg.release_scratch()
    torch.cuda.empty_cache()
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


def phase_rooflines(tg, g, out_e, tau_sum, phases):
    """Roofline objects of the three largest phases of tg_count (4-cycles,
    4-cliques, per-edge combine): algorithmic bytes (the byte models above,
    with the launch decisions the library takes on this graph) over the
    phase time measured with HIP events on the call's stream, against the
    HBM peak; `traffic` is the committed counter summary's L2-egress bytes
    for the phase's kernels when it matches the kernel sources."""
    import torch
    L = g.L
    P = L * (L + 1) // 2
    st = graph_stats(g)
    lists = keeps_lists(st)
    tuning = tg.Tuning.default()
    pass_used = bool(tuning.clique_pass) and int(st["dplus"].max()) <= 4096
    # |T_e| per edge from the rows, for the widest clique counter and the
    # probe count of the out-list path
    tsz = out_e.view(torch.int64)[:, L:2 * L].sum(1)
    max_t = int(tsz.max().item()) if tsz.numel() else 0
    k4_width = (8 if max_t * max(max_t - 1, 0) // 2 >= (1 << 32) else 4) if pass_used else 0
    probes = 0
    if not pass_used:
        tri2 = torch.zeros(g.n, dtype=torch.int64, device=out_e.device)
        tri2.index_add_(0, torch.from_numpy(st["ei"]).to(out_e.device), tsz)
        tri2.index_add_(0, torch.from_numpy(st["ej"]).to(out_e.device), tsz)
        probes = clique_probes(st, (tri2 // 2).cpu().numpy())
    dmax = int(st["deg"].max())
    c4_width = 8 if (dmax - 1) * (dmax - 1) >= (1 << 32) else 4
    scanned, oriented = cycle_wedges(st)
    models = {
        "cycles": (cycles_bytes(st, L, scanned, oriented, c4_width),
                   "typed 4-cycle phase: k_c4_hash tiers, k_c4_bwalk/k_c4_bcount bucketed counts, "
                   "k_c4_group count/credit/clear, k_c4_fold",
                   f"{scanned} scanned and {oriented} oriented wedges; credits left out"),
        "cliques": (clique_bytes(st, L, k4_width) if pass_used else 0,
                    "typed 4-clique pass: k_k4_low over every node with 3 or more higher-ranked neighbours",
                    "out-lists of every node's out-list members read twice; credits left out"),
        "combine": (combine_bytes(st, L, tau_sum, lists, k4_width=k4_width, probes=probes),
                    "per-edge combine: gather kernels k_combine<16|64|256> and their k_combine_rows launches",
                    f"T_ij from {'kept lists' if lists else 'row intersection'}, 4-cliques from "
                    f"{'the clique pass' if pass_used else f'{probes} out-list probes'}"),
    }
    traffic = stored_traffic(g.name) or {}
    out = {}
    for ph, (b, kern, note) in models.items():
        ms = phases.get(ph, 0.0)
        if ms <= 0 or b <= 0:
            continue
        achieved = b / (ms * 1e-3) / 1e9
        tr = traffic.get(ph)
        out[ph] = {"bound": "hbm", "kernel": kern, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": b, "phase_ms": ms, "model": note,
                   "traffic": tr, "traffic_source": "L2 egress: FETCH_SIZE and WRITE_SIZE scaled by a plain copy "
                                                    "(MALL hits included), from " + _TRAFFIC_FILE,
                   "traffic_gbs": tr / (ms * 1e-3) / 1e9 if tr else None}
    return out


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
    ap.add_argument("--no-partite", action="store_true", help="skip the bipartite and 3-partite graphs")
    ap.add_argument("--no-giant", action="store_true",
                    help="skip the 20M-node graph's per-edge leg (every edge counted under the degree and the "
                         "learned schedule, several minutes)")
    ap.add_argument("--giant-repeats", type=int, default=1, help="degree-schedule calls of the 20M-node leg")
    ap.add_argument("--giant-only", action="store_true",
                    help="only run the 20M-node per-edge leg and print its object (for profiling)")
    ap.add_argument("--giant-degree-only", action="store_true",
                    help="with --giant-only: the degree schedule only")
    ap.add_argument("--permutations", type=int, default=100, help="permutations of the null-model leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                             "COPY_WRITE_CSV"),
                    help="only print the L2-egress summary of rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of the "
                         "benchmark step and of --copy-calibration (counter_collection.csv files) and exit")
    ap.add_argument("--summarize-lds", metavar="COUNTER_CSV",
                    help="print per-kernel LDS figures of a rocprofv3 --pmc run of the LDS counters and exit")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="only print the per-kernel summary of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the calibration copy (--summarize-counters)")
    ap.add_argument("--calls", type=int, default=1, help="tg_count calls in the profiled run (--summarize-counters)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.calls)
        return
    if args.summarize_lds:
        summarize_lds(args.summarize_lds, args.calls)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, copy_bytes=args.copy_mib << 20, calls_per_run=args.calls)
        return
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
    if args.giant_only:
        # the 20M-node per-edge leg alone (for profiling it), as its own line
        print(json.dumps({"giant_per_edge": giant_per_edge_leg(tg, dev, repeats=args.giant_repeats,
                                                               learned=not args.giant_degree_only)}), flush=True)
        return
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
    rooflines = phase_rooflines(tg, g, out_e, tau_sum, phases)
    main_phase = max(rooflines, key=lambda ph: rooflines[ph]["phase_ms"])
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
        "roofline": rooflines[main_phase],
        "roofline_phases": {ph: r for ph, r in rooflines.items() if ph != main_phase},
    }
    if not args.no_compare:
        rec["schedules"] = compare_schedules(tg, g, rp, ci, ty, out_g, out_e)
    if not args.no_global:
        rec["global_only"] = global_leg(tg, g, rp, ci, ty, out_g)
    if not args.no_null:
        rec["null_model"] = null_leg(tg, g, rp, ci, ty, permutations=args.permutations)
    if not args.no_directed:
        rec["directed3"] = directed_leg(tg, g, rp, ci, ty)
        rec["directed4"] = directed4_leg(tg, dev)
    if not args.no_outputs:
        rec["outputs"] = outputs_leg(tg, g, rp, ci, ty, out_g, out_e)
    if not args.no_partite:
        try:
            rec["partite"] = partite_leg(tg, dev)
        except Exception as ex:  # reported in the line; the rest of the run still counts
            log(f"partite leg failed: {ex}")
            rec["partite"] = {"error": str(ex)}
    if args.giant_global:
        rec["giant_global"] = giant_global_leg(tg, dev)
    if not args.no_giant:
        # the 20M-node graph needs most of the device: drop this graph's
        # buffers and the library's cached scratch first
        del out_e
        tg.release_scratch()
        torch.cuda.empty_cache()
        try:
            rec["giant_per_edge"] = giant_per_edge_leg(tg, dev, repeats=args.giant_repeats)
        except Exception as ex:  # reported in the line; the rest of the run still counts
            log(f"cl-20m per-edge leg failed: {ex}")
            rec["giant_per_edge"] = {"error": str(ex)}
    if not args.no_batch:
        rec["batch"] = batch_leg(tg, dev)
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"cpu baseline: oracle for ~{args.cpu_seconds:.0f} s on {threads} threads")
        rec["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds, threads)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

"""Throughput of the NN-Descent K-NN graph build on one MI355X.

A step is one whole build (random init, iterations until changes < delta*N*K,
write-out) of the image-shaped workload: N=60000 points of d=784 integer
intensities 0..255 (~80% zeros), K=20, rho=1, delta=0.001, seed 1, at most
30 iterations. Inputs are resident in HBM before the timed region.

Prints one JSON line: evals/s (sum of e_t over the build / build time), the
time to tie-aware recall 0.99, the roofline of the local-join kernel (its
algorithmic bytes per launch -- member rows gathered per owner without reuse,
member metadata and emitted proposals -- over its event-timed average launch,
against HBM; its MFMA flop rate e_t * 2d beside it), and the FP64 oracle timed
on a bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
WORKLOADS = {
    # the headline workload (default)
    "image60k_d784": dict(workload="image60k_d784", N=60000, d=784, K=20, rho=1.0, delta=0.001, max_iters=30,
                          seed=1, gen=lambda: __import__("synth").image_like(60000, 1)),
    "gauss2k_d8": dict(workload="gauss2k_d8", N=2000, d=8, K=10, rho=1.0, delta=0.001, max_iters=20, seed=0,
                       gen=lambda: __import__("synth").workload("gauss2k_d8")[0]),
    # points in random memory order; the graph-ordered permutation after iteration 6 (measured best of
    # t_p = 1..8) makes the later iterations gather nearby records
    "blobs4m_d3": dict(workload="blobs4m_d3", N=4_000_000, d=3, K=15, rho=0.5, delta=0.001, max_iters=30, seed=2,
                       reorder=6, gen=lambda: __import__("synth").lowd_blobs(4_000_000, 2)),
    "batch512": dict(workload="batch512", N=None, d=None, K=15, rho=1.0, delta=0.001, max_iters=30, seed=4,
                     gen=lambda: __import__("synth").batched_datasets(512, 4)),
    # the paper's selection-step workload (Sec. 4: Synthetic Gaussian Dataset, n = 16384, d = 8)
    "gauss16k_d8": dict(workload="gauss16k_d8", N=16384, d=8, K=20, rho=1.0, delta=0.001, max_iters=30, seed=6,
                        gen=lambda: __import__("synth").synthetic_gaussian(16384, 8, 6)),
    # the paper's reordering workload (Sec. 4, Fig. 5: Synthetic Clustered Dataset, 16384 points, 16 clusters, d = 8)
    "clustered16k_d8": dict(workload="clustered16k_d8", N=16384, d=8, K=20, rho=1.0, delta=0.001, max_iters=30,
                            seed=4, gen=lambda: __import__("synth").clustered_labels(16384, 8, 16, 4)[0]),
    # the paper's roofline workloads (Sec. 4, Fig. 3: Synthetic Gaussian Dataset, n = 131072, d = 8 and 256)
    "gauss131k_d8": dict(workload="gauss131k_d8", N=131072, d=8, K=20, rho=1.0, delta=0.001, max_iters=30, seed=8,
                         gen=lambda: __import__("synth").synthetic_gaussian(131072, 8, 8)),
    "gauss131k_d256": dict(workload="gauss131k_d256", N=131072, d=256, K=20, rho=1.0, delta=0.001, max_iters=30,
                           seed=8, gen=lambda: __import__("synth").synthetic_gaussian(131072, 256, 8)),
    # audio-shaped stand-in (Sec. 4: Audio dataset, 54387 x 192)
    "audio54k_d192": dict(workload="audio54k_d192", N=54387, d=192, K=20, rho=1.0, delta=0.001, max_iters=30,
                          seed=7, gen=lambda: __import__("synth").audio_like(54387, 192, 7)),
    # the three split planes (1.15 GB) exceed the 256 MB last-level cache: the graph-ordered permutation
    # after iteration 2 pays here (measured)
    "aniso200k_d960": dict(workload="aniso200k_d960", N=200_000, d=960, K=20, rho=0.5, delta=0.001, max_iters=30,
                           seed=3, reorder=2, gen=lambda: __import__("synth").anisotropic_clusters(200_000, 960, 3)),
}
WORKLOAD = WORKLOADS["image60k_d784"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("knng_kernels.hip", "knng_api.hip", "knng_impl.h"):
        h.update(open(os.path.join(ROOT, "paper_2112_06630_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def exact_kth(X, K, rows):
    """Exact K-th neighbour distance (FP64, self excluded) and the exact
    neighbour ids of the query rows, on the GPU with torch (evaluation only,
    not the method's path)."""
    import torch
    Xd = X.double()
    n = (Xd * Xd).sum(1)
    out = torch.empty(len(rows), dtype=torch.float64, device=X.device)
    ids = torch.empty((len(rows), K), dtype=torch.int64, device=X.device)
    step = max(1, min(4096, (1 << 28) // X.shape[0]))
    for s in range(0, len(rows), step):
        r = rows[s:s + step]
        D = n[r, None] + n[None, :] - 2.0 * (Xd[r] @ Xd.T)
        D[torch.arange(len(r), device=X.device), r] = float("inf")
        tk = torch.topk(D, K, dim=1, largest=False)
        out[s:s + step] = tk.values[:, -1]
        ids[s:s + step] = tk.indices
    return out, ids


def plain_recall(ids, exact_ids, rows):
    """Plain intersection recall |found ∩ exact| / K over the query rows (ties
    at the K-th distance count against it)."""
    import torch
    found = ids[rows].long()
    hit = (found[:, :, None] == exact_ids[:, None, :]).any(-1)
    return float(hit.float().mean())


def dist_error(X, ids, dists, rows):
    """Stored FP32 distances of the query rows against an FP64 recomputation
    (torch on the GPU; evaluation only): max absolute error and max error
    relative to the distance."""
    Xd = X.double()
    abs_max, rel_max = 0.0, 0.0
    for s in range(0, len(rows), 2048):
        r = rows[s:s + 2048]
        diff = Xd[ids[r].long()] - Xd[r, None, :]
        D = (diff * diff).sum(-1)
        e = (dists[r].double() - D).abs()
        abs_max = max(abs_max, float(e.max()))
        rel_max = max(rel_max, float((e / D.clamp_min(1e-30)).max()))
    return abs_max, rel_max


def recall_of(X, ids, tau, rows, rel=1e-5):
    """Tie-aware recall over the query rows: a found id counts when its FP64
    distance is within rel of the exact K-th distance."""
    Xd = X.double()
    good = 0
    for s in range(0, len(rows), 2048):
        r = rows[s:s + 2048]
        diff = Xd[ids[r].long()] - Xd[r, None, :]
        D = (diff * diff).sum(-1)
        good += int((D <= tau[s:s + 2048, None] * (1 + rel) + 1e-9).sum())
    return good / (len(rows) * ids.shape[1])


def cpu_baseline(Xnp, w, budget_s=20.0, sampling="weighted", threads=0, blocks=0):
    """FP64 oracle on the host: init + iterations 1, 2, ... of the same workload
    (same sampling rule) until ~budget_s of CPU work; evals/s over the
    iterations run."""
    import oracle
    oracle.build(force=False)
    if threads:
        oracle.set_num_threads(threads)
    C = oracle.cap(w["K"], w["rho"])
    t0 = time.perf_counter()
    st = oracle.init(Xnp, w["K"], w["seed"])
    ev = 0
    iters = 0
    thr = w["delta"] * Xnp.shape[0] * w["K"]
    stopped = False
    while time.perf_counter() - t0 < budget_s and iters < w["max_iters"]:
        st, e, c = oracle.iterate(Xnp, st, w["K"], C, w["seed"], sampling, max(1, blocks))
        ev += e
        iters += 1
        if c < thr:   # the build's own stop rule (Sec. 2: changes below delta*N*K)
            stopped = True
            break
    dt = time.perf_counter() - t0
    how = "stop rule met" if stopped else ("iteration cap" if iters >= w["max_iters"] else "time budget")
    return {"value": ev / dt, "unit": "distance evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, full {w['workload']} input, init + iterations 1..{iters} ({how}; "
                      f"{ev} evals in {dt:.1f} s)"}


def traffic_path(workload: str) -> str:
    """Counter summary of a workload: profiles/traffic.json for the headline
    workload, profiles/traffic_<workload>.json for the others."""
    name = "traffic.json" if workload == WORKLOAD["workload"] else f"traffic_{workload}.json"
    return os.path.join(ROOT, "profiles", name)


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs of the
    workload, if they were taken on the current kernel source; else None."""
    p = traffic_path(workload)
    if not os.path.exists(p):
        return None
    rec = json.load(open(p)).get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def reorder_of(args, w) -> int:
    """The permutation point t_p of a run: --reorder if given, else the
    workload's own setting (0: off)."""
    return int(args.reorder) if args.reorder is not None else int(w.get("reorder", 0))


def member_counts_and_graphs(X, w, args, iters, keep_graphs):
    """Replays the build through the step API (deterministic: the same
    trajectory as the timed builds): per iteration, the members gathered by
    the join (sum over owners with a new member of n_new + n_old) and, if
    asked, the graph G_t."""
    import paper_2112_06630_amd as knng
    ctx = knng.Context(X, w["K"], w["rho"], w["delta"], w["max_iters"], w["seed"], reorder_of(args, w),
                       path=args.path, precision=args.precision, sampling=args.sampling, blocks=args.blocks)
    ctx.init()
    members, graphs = [], []
    for _ in range(iters):
        ctx.iterate()
        cnt = ctx.samples()[2].long()
        members.append(int((cnt.sum(1) * (cnt[:, 0] > 0)).sum().item()))
        if keep_graphs:
            graphs.append(ctx.export().ids)
    ctx.close()
    return members, graphs


def bench_batch(args, w):
    """512 independent datasets in one captured graph vs 512 sequential builds."""
    import numpy as np
    import torch
    import paper_2112_06630_amd as knng
    data = w["gen"]()
    dev = torch.device("cuda:0")
    Xs = [torch.from_numpy(X).to(dev) for X, _ in data]
    seeds = [s for _, s in data]
    t0 = time.perf_counter()
    b = knng.Batch(Xs, seeds, w["K"], w["rho"], w["delta"], w["max_iters"])
    plan_s = time.perf_counter() - t0
    b.capture()
    for _ in range(args.warmup):
        b.launch()
    b.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(b.stream)
    for _ in range(args.steps):
        b.launch()
    ev1.record(b.stream)
    b.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    st = b.stats()
    evals = int(sum(sum(e) for e in st["evals"]))
    entries = {d: r.partition("@")[0] for d, r in (e.split(":") for e in b.tuning.split(","))}   # path per d
    # the same builds one dataset at a time (same join paths)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_ids = []
    for X, s in zip(Xs, seeds):
        seq_ids.append(knng.build(X, w["K"], w["rho"], w["delta"], w["max_iters"], s,
                                  path=entries[str(X.shape[1])])[0])
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    identical = all(torch.equal(a, c) for a, c in zip(b.ids, seq_ids))
    rec = None
    if not args.no_recall:
        tot, good = 0, 0.0
        for X, ids in zip(Xs, b.ids):
            rows = torch.arange(X.shape[0], device=dev)
            tau, _ = exact_kth(X, w["K"], rows)
            good += recall_of(X, ids, tau, rows) * X.shape[0]
            tot += X.shape[0]
        rec = good / tot
    out = {
        "metric": "distance evals/sec", "value": round(evals / (ms_per_step / 1e3), 1), "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch512", "datasets": len(data), "N_total": int(sum(X.shape[0] for X in Xs)),
                   "dims": sorted({int(X.shape[1]) for X in Xs}), "K": w["K"], "rho": w["rho"],
                   "delta": w["delta"], "max_iters": w["max_iters"], "tuning": b.tuning},
        "evals_per_build": evals, "recall": rec, "sequential_ms": round(seq_ms, 3),
        "speedup_vs_sequential": round(seq_ms / ms_per_step, 2), "identical_to_sequential": identical,
        "graph_device_ms": round(ev0.elapsed_time(ev1) / args.steps, 3), "plan_and_tune_s": round(plan_s, 3),
        "iters_max": int(max(st["iters"])), "converged": int(sum(st["converged"])),
    }
    b.close()
    print(json.dumps(out), flush=True)


def summarize_pmc(fetch_csv, write_csv, copy_mib, command, workload):
    """Writes the workload's counter summary (traffic_path): HBM bytes per launch of each knng kernel
    from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the counter reads for the plain copy of
    copy_mib MiB that bench.py --copy-probe-mib issues in the same run.
    Dispatches of the iteration a build enqueues ahead of its stop decision
    return at once; those (fetch below 1% of the kernel's largest) are left
    out of the per-launch figures."""
    import csv
    import collections

    def per_kernel(path, counter):
        rows = list(csv.DictReader(open(path)))
        agg = collections.defaultdict(list)
        probe = None
        for r in rows:
            if r.get("Counter_Name", counter) != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("knng::", "").replace("void ", "").split("<")[0]
            kib = float(r["Counter_Value"])
            if "copyBuffer" in name and int(r["Grid_Size"]) >= (copy_mib << 7):
                probe = kib
            agg[name].append(kib)
        return agg, probe

    fetch, fprobe = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wprobe = per_kernel(write_csv, "WRITE_SIZE")
    if not fprobe or not wprobe:
        raise SystemExit("copy probe not found in the counter runs")
    f_scale = copy_mib * 1024.0 / fprobe   # a copy reads copy_mib MiB
    w_scale = copy_mib * 1024.0 / wprobe   # and writes copy_mib MiB
    out = {"_scale": {"fetch": f_scale, "write": w_scale, "copy_mib": copy_mib,
                      "probe_fetch_kib": fprobe, "probe_write_kib": wprobe}, "_command": command}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("k_"):
            continue
        fl, wl = fetch.get(k, []), write.get(k, [])
        keep_f = [x for x in fl if x >= 0.01 * max(fl)] if fl else []
        keep_w = [y for x, y in zip(fl, wl) if x >= 0.01 * max(fl)] if fl and len(fl) == len(wl) else wl
        fb = sum(keep_f) / max(1, len(keep_f)) * 1024 * f_scale
        wb = sum(keep_w) / max(1, len(keep_w)) * 1024 * w_scale
        out[k] = {"source_hash": kernel_source_hash(), "bytes_per_launch": int(fb + wb),
                  "fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
                  "launches": len(keep_f), "early_exits": len(fl) - len(keep_f)}
    path = traffic_path(workload)
    json.dump(out, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps({k: out[k] for k in out if not k.startswith("_")}, indent=1))


def run_sweep(args):
    """The paper's scaling sweeps (Sec. 4): dimension d = 8, 72, ..., 3144 at
    n = 16384 on its Synthetic Single Gaussian Dataset, or size n = 2^10 ..
    2^20 at d = 256 on its Synthetic Gaussian Dataset (one Gaussian per basis
    vector); covariance 2 I; K = 20, rho = 1, delta = 0.001, T = 30.
    "lowd": d = 8, 16, ..., 96 at n = 16384, where the direct-form (VALU) join
    still fits its LDS stage, to place the VALU / matrix-core crossover.
    Every join path the plan accepts at a point is timed (wall clock of whole
    builds, inputs resident); one JSON line per (point, path)."""
    import numpy as np
    import torch
    import synth
    import paper_2112_06630_amd as knng

    dev = torch.device("cuda:0")
    K, rho, delta, T, seed = 20, 1.0, 0.001, 30, 5
    if args.sweep == "d":
        pts = [(16384, d) for d in range(8, 3145, 64)]
    elif args.sweep == "lowd":
        pts = [(16384, d) for d in range(8, 97, 8)]
    else:
        pts = [(1 << e, 256) for e in range(10, 21)]
    for N, d in pts:
        gen = synth.synthetic_gaussian if args.sweep == "n" else synth.single_gaussian
        X = torch.from_numpy(gen(N, d, seed)).to(dev)
        for path in ("valu", "mfma", "bf16x3"):
            try:
                p = knng.make_params(K, rho, delta, T, seed, False, path=path, sampling=args.sampling)
                ws = torch.empty(knng.workspace_bytes(N, d, p), dtype=torch.uint8, device=dev)
            except Exception:
                continue   # the path does not take this shape (VALU: rows must fit the LDS stage)
            if ws.numel() == 0:
                continue
            ids = torch.empty((N, K), dtype=torch.int32, device=dev)
            dists = torch.empty((N, K), dtype=torch.float32, device=dev)
            run = lambda: knng.build(X, K, rho, delta, T, seed, False, path=path, workspace=ws, out=(ids, dists),
                                     sampling=args.sampling)
            for _ in range(max(1, args.warmup)):
                run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = [run()[2] for _ in range(args.steps)]
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            st = sts[-1]
            ev = sum(st["evals"])
            join = float(sum(st["join_ms"]))
            print(json.dumps({"sweep": args.sweep, "N": N, "d": d, "path": path, "sampling": args.sampling,
                              "ms_per_build": round(ms, 3),
                              "iters": st["iters"], "evals": ev, "evals_per_s": round(ev / (ms / 1e3), 1),
                              "paper_gflops": round(ev * (3 * d - 1) / (ms / 1e3) / 1e9, 2),
                              "alg_tflops": round(ev * 2 * d / (ms / 1e3) / 1e12, 3),
                              "join_ms": round(join, 3), "planes": st.get("planes")}), flush=True)
            del ws, ids, dists
        del X


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reorder", type=int, default=None,
                    help="graph-ordered permutation once after iteration t_p (0: off); default: the workload's "
                         "(after iteration 2 on aniso200k_d960 and 6 on blobs4m_d3, where it pays; off elsewhere)")
    ap.add_argument("--workload", default="image60k_d784", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--path", default="auto", choices=["auto", "valu", "mfma", "bf16x3"])
    ap.add_argument("--delta", type=float, default=None, help="override the workload's stop threshold")
    ap.add_argument("--sampling", default="weighted", choices=["weighted", "turbo"],
                    help="selection-step rule (Sec. 3.1): bounded heaps or turbosampling")
    ap.add_argument("--recall-rows", type=int, default=100000,
                    help="query rows for recall (all rows when N is smaller; a seeded sample otherwise)")
    ap.add_argument("--blocks", type=int, default=0,
                    help="block-asynchronous iterations over this many blocks of owners (0: synchronous)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU oracle baseline (0: all host cores)")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="headline workload only (by default the low-d blobs4m_d3 build is timed beside it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the builds, copy this many MiB once (device to device) so that "
                         "HBM counters can be scaled by a kernel of known traffic")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarize two rocprofv3 counter runs of --workload into its profiles/traffic*.json "
                         "and exit")
    ap.add_argument("--pmc-command", default="", help="the command the counter runs used (recorded)")
    ap.add_argument("--sweep", choices=["d", "n", "lowd"], default=None,
                    help="the paper's dimension (n = 16384) or size (d = 256) sweep on a single Gaussian: "
                         "one JSON line per point and join path, no headline line")
    args = ap.parse_args()
    if args.pmc_summary:
        summarize_pmc(args.pmc_summary[0], args.pmc_summary[1], args.copy_probe_mib or 1024, args.pmc_command,
                      args.workload)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.sweep:
        run_sweep(args)
        return

    w = dict(WORKLOADS[args.workload])
    if args.workload == "batch512":
        if args.delta is not None:
            w["delta"] = args.delta
        bench_batch(args, w)
        return
    out = measure(args, w, args.steps, args.warmup, args.recall_rows, not args.no_cpu)
    if args.workload == WORKLOAD["workload"] and not args.no_secondary:
        # the low-d gather-bound workload beside the headline, so that every
        # default run also times it (fewer steps: one build is ~0.1 s)
        lw = dict(WORKLOADS["blobs4m_d3"])
        sec = measure(args, lw, max(3, min(args.steps, 10)), max(1, min(args.warmup, 2)), 2000, False)
        out["secondary"] = {lw["workload"]: {k: sec[k] for k in (
            "value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config", "iters", "evals_per_build",
            "recall", "recall_rows", "ms_to_recall_0.99", "device_ms_per_build", "phase_ms", "reorder_ms",
            "roofline")}}
    print(json.dumps(out), flush=True)


def join_kernel_name(knng, s0, precision):
    if precision == "bf16":
        return "k_join_bf16"
    return {knng.PATH_MFMA: "k_join_mfma", knng.PATH_MFMA_BF16X3: "k_join_split"}.get(s0["path"], "k_join_valu")


def member_encoding(kernel, s0, dpad):
    """(row bytes, all bytes) the join reads per member as the library stores
    them: byte rows (8-bit data) or the split-BF16 planes it reads, with the
    member's sample entry (8 B), snapshot K-th key (8 B) and squared norm (4 B,
    8 B in FP64 on inexact data); the precision form's BF16 copy, its
    staged FP32 row and the copy's two norms (8 B); the direct form's FP32
    row with the sample entry and the K-th key, which share one 32-byte
    record with a 4-float row."""
    norm = 8 if s0.get("accurate") else 4
    if kernel == "k_join_split":
        row = dpad if s0.get("u8") else 2 * dpad * max(1, s0["planes"])
        return row, row + 16 + norm
    if kernel == "k_join_mfma":
        return 4 * dpad, 4 * dpad + 16 + norm
    if kernel == "k_join_bf16":
        return 6 * dpad, 6 * dpad + 16 + 8
    if dpad == 4:
        return 16, 32 + 8
    return 4 * dpad, 4 * dpad + 16


def join_roofline(knng, w, s0, stats, members, precision):
    """Roofline of the local join from its event-timed launches.

    Algorithmic bytes per launch follow the per-unit figures of the method's
    byte model: every member row gathered once per owner in FP32
    (4 * d_pad bytes, no reuse across owners), its sample entry read (8 B),
    and one 8-byte key written per emitted proposal. ``encoding`` prices the
    rows as the kernel actually stores them, with the member metadata it
    reads (member_encoding): on 8-bit data (byte rows) this is about a
    quarter of the FP32 figure, and the FP32-model fraction can then exceed 1
    without the kernel moving more than the memory system delivers. ``traffic`` is the counter-measured
    L2-to-memory traffic of the same kernel (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled by a copy of known size), when the committed counter
    summary was taken on the current source."""
    import numpy as np
    kernel = join_kernel_name(knng, s0, precision)
    join_ms = [float(np.median([s["join_ms"][i] for s in stats])) for i in range(s0["iters"])]
    dpad = s0["dpad"]
    alg = [m * (4 * dpad + 8) + 8 * pr for m, pr in zip(members, s0["proposals"])]
    enc_row, enc_member = member_encoding(kernel, s0, dpad)
    enc = [m * enc_member + 8 * pr for m, pr in zip(members, s0["proposals"])]
    flops = [e * 2 * w["d"] for e in s0["evals"]]
    sec = sum(join_ms) / 1e3
    ach = sum(alg) / sec / 1e9
    ach_enc = sum(enc) / sec / 1e9
    ach_fl = sum(flops) / sec / 1e12
    n = len(join_ms)
    traffic = traffic_record(kernel, w["workload"])
    peak_fl = PEAK_BF16_MFMA_TFLOPS if kernel in ("k_join_bf16", "k_join_split") else PEAK_FP32_MFMA_TFLOPS
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": kernel,
            "avg_launch_ms": round(sum(join_ms) / n, 4), "launches": n,
            "bytes_per_launch": int(sum(alg) / n), "members_per_launch": int(sum(members) / n),
            "proposals_per_launch": int(sum(s0["proposals"]) / n),
            "encoding": {"row_bytes": enc_row, "member_bytes": enc_member, "bytes_per_launch": int(sum(enc) / n),
                         "achieved": round(ach_enc, 1), "frac": round(ach_enc / PEAK_HBM_GBS, 4)},
            "mfma": {"achieved": round(ach_fl, 3), "peak": peak_fl, "unit": "TFLOP/s",
                     "frac": round(ach_fl / peak_fl, 4), "flops_per_launch": int(sum(flops) / n)}}
    if traffic:
        roof["traffic_achieved"] = round(traffic * n / sec / 1e9, 1)
    if roof["frac"] > 1:
        roof["note"] = ("the FP32 row model exceeds the HBM peak: the kernel reads a lossless "
                        f"{enc_row / dpad:g}-byte-per-dimension encoding of the rows (see encoding)")
    return roof


def measure(args, w, steps, warmup, recall_rows, with_cpu):
    """Times `steps` whole builds of workload `w` (inputs resident in HBM)
    after `warmup` untimed ones; returns the result line as a dict."""
    import numpy as np
    import torch
    import paper_2112_06630_amd as knng

    w = dict(w)
    if args.delta is not None:
        w["delta"] = args.delta
    Xnp = w["gen"]()
    dev = torch.device("cuda:0")
    X = torch.from_numpy(Xnp).to(dev)
    p = knng.make_params(w["K"], w["rho"], w["delta"], w["max_iters"], w["seed"], reorder_of(args, w),
                         path=args.path, precision=args.precision, sampling=args.sampling, blocks=args.blocks)
    ws = torch.empty(knng.workspace_bytes(w["N"], w["d"], p), dtype=torch.uint8, device=dev)
    ids = torch.empty((w["N"], w["K"]), dtype=torch.int32, device=dev)
    dists = torch.empty((w["N"], w["K"]), dtype=torch.float32, device=dev)
    run = lambda: knng.build(X, w["K"], w["rho"], w["delta"], w["max_iters"], w["seed"], reorder_of(args, w),
                             path=args.path, workspace=ws, out=(ids, dists), precision=args.precision,
                             sampling=args.sampling, blocks=args.blocks)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(run()[2])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps
    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    evals = sum(stats[0]["evals"])
    for s in stats[1:]:
        assert s["evals"] == stats[0]["evals"] and s["changes"] == stats[0]["changes"], "non-deterministic build"
    value = evals / (ms_per_step / 1e3)

    s0 = stats[len(stats) // 2]
    no_recall = args.no_recall or recall_rows <= 0
    # per-iteration member counts (and graphs) from a step-API replay of the
    # same deterministic trajectory (untimed)
    members, curve_ids = member_counts_and_graphs(X, w, args, s0["iters"], not no_recall)
    roof = join_roofline(knng, w, s0, stats, members, args.precision)
    kernel = roof["kernel"]

    # time to recall 0.99: per-iteration graphs from the same step-API replay
    rec = t99 = rcurve = derr = rec_plain = None
    if not no_recall:
        N = w["N"]
        if N <= recall_rows:
            rows = torch.arange(N, device=dev)
        else:
            rows = torch.from_numpy(np.sort(np.random.default_rng(12345).choice(N, recall_rows,
                                                                                replace=False))).to(dev)
        tau, exact_ids = exact_kth(X, w["K"], rows)
        curve = [recall_of(X, ids_t, tau, rows) for ids_t in curve_ids]
        rec_plain = plain_recall(ids, exact_ids, rows)
        rec = curve[-1]
        derr = dist_error(X, ids, dists, rows)
        cum = s0["init_ms"] + s0["reorder_ms"]
        rcurve = []
        for t, r in enumerate(curve):
            cum += float(np.median([s["iter_ms"][t] for s in stats]))
            rcurve.append([round(cum, 4), round(r, 6)])
            if r >= 0.99 and t99 is None:
                t99 = cum
    # context: a plain device-to-device copy of 1 GiB (1 GiB read + 1 GiB written)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    cpu = cpu_baseline(Xnp, w, sampling=args.sampling, threads=args.cpu_threads, blocks=args.blocks) \
        if with_cpu else None
    if cpu is not None and args.precision != "fp32":
        cpu["sample"] += " (the oracle computes FP64 distances)"
    if kernel == "k_join_split":
        dtype = "u8+f32" if s0.get("u8") else ("f32" if s0["planes"] == 3 else f"bf16x{s0['planes']}+f32")
    else:
        dtype = {"k_join_bf16": "bf16+f32"}.get(kernel, "f32")

    del ws, ids, dists, X
    return {
        "metric": "distance evals/sec", "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # split form: the BF16 planes the join reads (all three carry FP32 values exactly)
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w["workload"], "N": w["N"], "d": w["d"], "K": w["K"], "rho": w["rho"],
                   "delta": w["delta"], "max_iters": w["max_iters"], "seed": w["seed"],
                   "reorder": reorder_of(args, w),
                   "path": {knng.PATH_MFMA: "mfma", knng.PATH_MFMA_BF16X3: "bf16x3"}.get(s0["path"], "valu"),
                   "precision": args.precision, "sampling": args.sampling, "blocks": args.blocks},
        "iters": s0["iters"], "evals_per_build": evals, "recall": rec, "recall_plain": rec_plain,
        "ms_to_recall_0.99": t99,
        "recall_rows": None if no_recall else int(min(w["N"], recall_rows)),
        "recall_curve": rcurve,   # [device ms since the build began, recall of G_t] per iteration
        # stored FP32 distances of the recall rows vs FP64: max absolute and max relative error
        "dist_err_vs_fp64": None if derr is None else {"abs": derr[0], "rel": derr[1]},
        "evals_per_iter": [int(e) for e in s0["evals"]],
        "iter_ms": [round(float(np.median([s["iter_ms"][t] for s in stats])), 4) for t in range(s0["iters"])],
        "rescored_per_build": int(sum(s0.get("rescored", []))),
        "reorder_ms": round(float(s0["reorder_ms"]), 3), "init_ms": round(float(s0["init_ms"]), 3),
        "device_ms_per_build": round(float(np.median([s["total_ms"] for s in stats])), 3),
        "phase_ms": {k: round(float(sum(s0[k])), 3) for k in ("sample_ms", "join_ms", "merge_ms")},
        "roofline": roof, "cpu_baseline": cpu,
        # context: e*(3d-1) flop/s (the paper's convention: d differences, d
        # products, d-1 additions per evaluation) and a measured copy bandwidth
        "paper_gflops": round(evals * (3 * w["d"] - 1) / (ms_per_step / 1e3) / 1e9, 1),
        "copy_GBps": round(copy_gbs, 1),
    }


if __name__ == "__main__":
    main()

"""Benchmark: the estimator's hot path on the R-MAT scale-20 workload.

One step = one pass of the whole path over the workload: for both
f = exp(beta A), beta = 1/d_max, and f = (I - gamma A)^-1, gamma =
0.85/lambda_max (50 power iterations), the full diagonal diag(f(A)) and the
full action f(A) 1, each with K = 40 and N = 256 walks per start row, FP64.
Inputs are resident in device memory before the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "walk steps/s + HBM GB/s; queries/s & p99 latency vs plain at equal error"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20, help="R-MAT scale")
    ap.add_argument("--walks", type=int, default=256)
    ap.add_argument("--K", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=float, default=3e7,
                    help="walk steps per query in the oracle's timed sample")
    ap.add_argument("--only", choices=["all", "action", "diag"], default="all")
    ap.add_argument("--copy-probe-bytes", type=int, default=0,
                    help="after timing, run one device copy of this many bytes (counter calibration)")
    ap.add_argument("--summarize", metavar="DIR[,DIR...]",
                    help="print a markdown summary of rocprofv3 CSV output in the directories and exit")
    ap.add_argument("--record-sources", metavar="PATH",
                    help="write the hashes of the timed kernels' sources to PATH (for --summarize)")
    ap.add_argument("--probe-bytes", type=int, default=0,
                    help="with --summarize: size of the calibration copy in that run")
    ap.add_argument("--workload", choices=["hotpath", "batch", "serve", "fp32"], default="hotpath",
                    help="hotpath: the R-MAT workload above (default); batch: 64 uneven requests "
                         "batched vs one at a time; serve: Poisson arrivals on resident graphs, "
                         "served vs sequential; fp32: FP32 vs FP64 walk weights on the "
                         "4M-node Barabasi-Albert graph")
    ap.add_argument("--requests", type=int, default=0, help="batch/serve: number of requests")
    ap.add_argument("--qps", type=float, default=0.0,
                    help="serve: arrival rate (0: the sequential path's measured capacity)")
    ap.add_argument("--seed", type=int, default=7, help="batch/serve: workload seed")
    ap.add_argument("--batch-n-max", type=int, default=1024,
                    help="batch: largest walks per start row the pilot may choose (the pilot asks "
                         "up to 65536 for the grid and ER requests)")
    ap.add_argument("--serve-scales", default="19,20,21,22,23,24,25,26",
                    help="serve: R-MAT scales of the resident graphs (native generator)")
    ap.add_argument("--no-compact", action="store_true",
                    help="hotpath: skip the compact batched/served legs")
    ap.add_argument("--tune", metavar="CACHE",
                    help="hotpath: autotune the walk kernels first (mcmf_tune, outside the timed "
                         "region), caching the choice in the JSON file CACHE")
    return ap.parse_args()


def algorithmic_bytes(kind, st, atomics=0):
    """Bytes the method itself must move through HBM, per kernel (the
    per-unit figures of the measurement plan):
    action walk: 12 B per transition (the current row's record, 8 B, and the
                 picked column, 4 B) + 8 B per recorded state (r at that state);
    diag walk:   12 B per transition (Q_k itself accumulates on chip);
    gather:      4 B per probed column entry + 8 B per FP64 atomic into d
                 (one per requested neighbour of each start row)."""
    steps = st["walk_steps"]
    transitions = steps - st["walks"]
    if kind == "action_walk":
        return 12 * transitions + 8 * steps
    if kind == "diag_walk":
        return 12 * transitions
    if kind == "diag_gather":
        return 4 * st["gather_probes"] + 8 * atomics
    raise ValueError(kind)


def layout_bytes(kind, st):
    """Bytes this implementation's data layout moves beyond the algorithmic
    ones: the diagonal's visit records (12 B per recorded state, written by
    the walk and read back by the gather) and the 4 B more of a 16-byte edge
    record than the 12 B of row record and column per transition.  The wide
    hub masks the diagonal walk reads under the WIDE layout are left out:
    the call does not count them (the FETCH_SIZE traffic includes them)."""
    steps = st["walk_steps"]
    transitions = steps - st["walks"]
    if kind == "diag_walk":
        return 12 * steps + 4 * transitions
    if kind == "diag_gather":
        return 12 * steps
    return 0


# Kernel name fragment -> (roofline name, source file whose hash tags counter data).
KERNELS = {"k_diag_gather": ("diag_gather", "gather.hip+gather_core.hpp"),
           "k_diag_walk": ("diag_walk", "walk.hip+walk_core.hpp"),
           "k_action_walk": ("action_walk", "walk.hip+walk_core.hpp")}
# Calibration: an elementwise kernel that reads and writes a known byte count
# (device-to-device memcpy may run on a DMA engine and show no kernel).
COPY_KERNEL = "neg_kernel"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rmat20.md")
CHUNK_KEY = "visit_chunk_bytes"


def source_sha(fnames):
    """Hash of the '+'-separated source files a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for fname in fnames.split("+"):
        h.update(open(os.path.join(ROOT, "paper_2308_01037_amd", "csrc", fname), "rb").read())
    return h.hexdigest()[:16]


def kernel_label(name):
    """Short kernel name: the library's k_* kernels with their template
    arguments, other kernels up to their parameter list."""
    import re
    m = re.search(r"(k_\w+(?:<[^()]*>)?)", name)
    if m:
        return m.group(1)
    return name.replace("void ", "").split("(")[0][:60]


def summarize(directory, probe_bytes):
    """Markdown summary of rocprofv3 --kernel-trace/--pmc CSV files."""
    import csv
    import glob
    lines = []
    traces, counters = [], []
    for d in directory.split(","):
        traces += glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
        counters += glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if traces:
        per = {}
        for path in traces:
            for r in csv.DictReader(open(path)):
                ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                k = per.setdefault(kernel_label(r["Kernel_Name"]), [0, 0])
                k[0] += 1
                k[1] += ns
        lines.append("| kernel | launches | total ms | avg ms |")
        lines.append("|---|---|---|---|")
        for name, (cnt, ns) in sorted(per.items(), key=lambda kv: -kv[1][1])[:20]:
            lines.append(f"| `{name}` | {cnt} | {ns / 1e6:.2f} | {ns / cnt / 1e6:.3f} |")
    if counters:
        agg = {}
        for path in counters:
            for r in csv.DictReader(open(path)):
                full = r["Kernel_Name"]
                name = COPY_KERNEL if COPY_KERNEL in full else kernel_label(full)
                key = (name, r["Counter_Name"])
                a = agg.setdefault(key, [0.0, set()])
                a[0] += float(r["Counter_Value"])
                a[1].add(r["Dispatch_Id"])
        lines.append("")
        # FETCH_SIZE and WRITE_SIZE read in KiB; the SQ_ counters are counts.
        if all(c in ("FETCH_SIZE", "WRITE_SIZE") for _, c in agg):
            lines.append("| kernel | counter | dispatches | KiB per dispatch |")
        else:
            lines.append("| kernel | counter | dispatches | per dispatch (KiB for FETCH_SIZE, WRITE_SIZE) |")
        lines.append("|---|---|---|---|")
        for (name, ctr), (tot, disp) in sorted(agg.items()):
            if any(f in name for f in list(KERNELS) + [COPY_KERNEL]):
                lines.append(f"| `{name}` | {ctr} | {len(disp)} | {tot / len(disp):.1f} |")
        # Source hashes recorded by the profiled run itself (--record-sources).
        recorded = {}
        for d in directory.split(","):
            try:
                recorded.update(json.load(open(os.path.join(d, "sources.json"))))
            except OSError:
                pass
        traffic = {}
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            copy = [(tot, disp) for (name, c), (tot, disp) in agg.items()
                    if c == ctr and COPY_KERNEL in name]
            if not copy or not probe_bytes:
                continue
            # The calibration copy is the largest copy in the run.
            tot, disp = max(copy, key=lambda t: t[0] / len(t[1]))
            factor = probe_bytes / (tot / len(disp) * 1024.0)
            lines.append(f"\n{ctr}: copy of {probe_bytes} bytes reads {tot / len(disp):.1f} KiB "
                         f"per dispatch -> factor {factor:.4f}")
            for frag, (kname, src) in KERNELS.items():
                hits = [(tot2, d2) for (name, c), (tot2, d2) in agg.items() if c == ctr and frag in name]
                if hits:
                    tot2 = sum(h[0] for h in hits)
                    nd = sum(len(h[1]) for h in hits)
                    if src not in recorded:
                        continue  # no record of the sources this run was built from
                    t = traffic.setdefault(kname, {"source": src, "sha": recorded[src]})
                    if kname.startswith("diag"):
                        t[CHUNK_KEY] = recorded.get(CHUNK_KEY)
                    t[ctr.lower() + "_bytes_per_launch"] = tot2 / nd * 1024.0 * factor
        if traffic:
            lines.append("")
            lines.append("traffic: " + json.dumps(traffic))
    return "\n".join(lines)


def visit_chunk_bytes(torch):
    """The library's diagonal visit buffer: MCMF_DIAG_CHUNK_BYTES, else 1/16
    of device memory within [256 MiB, 16 GiB] (it sets the start rows one
    diagonal walk and gather launch take)."""
    return int(os.environ.get("MCMF_DIAG_CHUNK_BYTES", "0")) or min(
        16 << 30, max(256 << 20, torch.cuda.get_device_properties(0).total_memory // 16))


def load_traffic(kernel, chunk_bytes=None):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none, the kernel's source changed since it was taken,
    or (diagonal kernels) the visit buffer, hence the work per launch, differs."""
    try:
        for line in open(TRAFFIC_FILE):
            if line.startswith("traffic: "):
                t = json.loads(line[len("traffic: "):]).get(kernel)
                if not t or t["sha"] != source_sha(t["source"]):
                    return None
                if kernel.startswith("diag") and t.get(CHUNK_KEY) != chunk_bytes:
                    return None
                if "fetch_size_bytes_per_launch" in t and "write_size_bytes_per_launch" in t:
                    return t["fetch_size_bytes_per_launch"] + t["write_size_bytes_per_launch"]
    except OSError:
        pass
    return None


def host_cpu():
    """Model of the host CPU (lscpu's model name, with the family, model,
    stepping and clock from /proc/cpuinfo, since a virtual machine may report
    a bare vendor name), and the logical CPUs this process may use."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if not line.strip():
                    break  # the first processor's block is enough
                key, _, value = line.partition(":")
                info[key.strip()] = value.strip()
    except OSError:
        pass
    model = model or info.get("model name", "")
    extra = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    if "cpu MHz" in info:
        extra.append(f"{float(info['cpu MHz']):.0f} MHz")
    if extra:
        model = f"{model} ({', '.join(extra)})"
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(csr, queries, target_steps, K, N):
    """The oracle, single-threaded and pinned to one core, on a bounded
    sample: each query evaluated at random non-isolated output rows (its walks
    start from their neighbourhoods), rows added until one query's walks make
    about `target_steps` steps.  Then the Erdos-Renyi G(1000, 0.01) workload
    (exp(A), K = 30, N = 1000, full diagonal and full action) end to end.
    Returns walk steps per second and the details."""
    import graphgen as G
    import oracle
    rng = np.random.default_rng(123)
    cand = rng.permutation(np.nonzero(csr.deg > 0)[0])
    starts, picked = set(), []
    per_start = N * (K - 1)
    for r in cand:
        nb = csr.col[csr.row_ptr[r]:csr.row_ptr[r + 1]]
        grown = len(starts.union(nb.tolist()))
        if grown * per_start > 1.5 * target_steps:
            continue  # a hub neighbourhood alone would overshoot
        starts.update(nb.tolist())
        picked.append(r)
        if len(starts) * per_start >= target_steps:
            break
    sample = np.sort(np.array(picked, dtype=np.int32))
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})  # one core for the oracle (single thread)
    try:
        total_steps, total_s = 0, 0.0
        for kind, fn, scale in queries:
            t0 = time.perf_counter()
            if kind == "action":
                r = oracle.action(csr, fn, np.ones(csr.n), N=N, K=K, scale=scale, seed=1, rows=sample)
            else:
                r = oracle.diag(csr, fn, N=N, K=K, scale=scale, seed=1, rows=sample,
                                assume_symmetric=True)
            dt = time.perf_counter() - t0
            total_steps += r["steps"]
            total_s += dt
            log(f"oracle {kind} fn={fn}: {r['steps']} steps in {dt:.2f} s")
        er = G.erdos_renyi_dense(1000, 0.01, seed=0)
        t0 = time.perf_counter()
        ra = oracle.action(er, oracle.FN_EXP, np.ones(er.n), N=1000, K=30, scale=1.0, seed=1)
        t1 = time.perf_counter()
        rd = oracle.diag(er, oracle.FN_EXP, N=1000, K=30, scale=1.0, seed=1, assume_symmetric=True)
        t2 = time.perf_counter()
        log(f"oracle ER(1000, 0.01): action {t1 - t0:.2f} s, diag {t2 - t1:.2f} s")
    finally:
        os.sched_setaffinity(0, before)
    er1000 = {"action_s": t1 - t0, "diag_s": t2 - t1,
              "walk_steps_per_query": ra["steps"], "walk_steps_per_s": (ra["steps"] + rd["steps"]) / (t2 - t0)}
    return total_steps / total_s, total_steps, total_s, sample.size, core, er1000


# ------------------------------------------------------------------ batch / serve

TARGET_SE = 1e-3  # target standard error of every estimate, relative to its rms value


class Query:
    """One request of the batch / serve workloads and its device buffers."""

    def __init__(self, M, torch, graph, csr, kind, fn, scale, K, rows=None, v=None, seed=1, rid=0):
        self.M, self.torch = M, torch
        self.graph, self.csr, self.kind, self.fn, self.scale, self.K = graph, csr, kind, fn, scale, K
        self.rows = None if rows is None else torch.as_tensor(np.asarray(rows, np.int32), device="cuda")
        self.v = None if v is None else torch.as_tensor(np.asarray(v, np.float64), device="cuda")
        self.count = csr.n if (kind == M.MCMF_REQ_ACTION or rows is None) else len(rows)
        self.seed, self.rid, self.N = seed, rid, 16
        self.out = torch.empty(max(self.count, 1), dtype=torch.float64, device="cuda")

    def request(self, rid=None, out=None):
        M = self.M
        return M.make_request(self.kind, self.graph.handle, M.make_fn(self.fn, self.scale), self.K,
                              self.N, self.out if out is None else out, rows=self.rows, v=self.v,
                              seed=self.seed, request_id=self.rid if rid is None else rid)

    def single(self, stream):
        M = self.M
        opts = M.make_opts(seed=self.seed, request_id=self.rid, stream=stream)
        f = M.make_fn(self.fn, self.scale)
        if self.kind == M.MCMF_REQ_ACTION:
            M.mcmf_action(self.graph.handle, f, self.v, self.N, self.K, opts, self.out)
        else:
            M.mcmf_diag(self.graph.handle, f, self.rows, 0 if self.rows is None else len(self.rows),
                        self.N, self.K, opts, self.out)


def pick_walks(M, torch, queries, n0=16, n_min=32, n_max=65536):
    """Walks per start row from a pilot: two independent estimates with n0
    walks each (32 pilot walks per start row in all, on request ids apart from
    the production ones) give the estimator's spread se0 (relative to the
    estimate's rms); N = n0 (se0 / target)^2, clamped to [n_min, n_max]."""
    for q in queries:
        q.N = n0
    outs = [[torch.empty_like(q.out) for q in queries] for _ in range(2)]
    for k in range(2):
        M.mcmf_batch([q.request(rid=(1 << 30) + 2 * i + k, out=outs[k][i]) for i, q in enumerate(queries)])
    torch.cuda.synchronize()
    for i, q in enumerate(queries):
        a = outs[0][i][:q.count].cpu().numpy()
        b = outs[1][i][:q.count].cpu().numpy()
        rms = float(np.sqrt(np.mean(a ** 2))) if q.count else 0.0
        se0 = float(np.sqrt(np.mean((a - b) ** 2) / 2.0)) / rms if rms > 0 else 0.0
        q.N_pilot = int(max(n_min, np.ceil(n0 * (se0 / TARGET_SE) ** 2)))
        q.N = int(min(n_max, q.N_pilot))


def bench_batch(args):
    """64 uneven requests over ER / R-MAT / grid graphs of 1e4..1e6 nodes:
    one batched launch (eager and hipGraph) against one call per request."""
    import torch
    import graphgen as G
    from paper_2308_01037_amd import mcmf as M
    rng = np.random.default_rng(args.seed)
    t0 = time.time()
    specs = [("er1e4", lambda: G.erdos_renyi_gnm(10_000, 50_000, seed=1)),
             ("er1e5", lambda: G.erdos_renyi_gnm(100_000, 500_000, seed=2)),
             ("er1e6", lambda: G.erdos_renyi_gnm(1_000_000, 5_000_000, seed=3)),
             ("rmat14", lambda: G.rmat(14, seed=4)),
             ("rmat17", lambda: G.rmat(17, seed=5)),
             ("rmat20", lambda: G.rmat(20, seed=6)),
             ("grid1000", lambda: G.grid2d(1000, 1000))]
    graphs = []
    for name, make in specs:
        csr = make()
        graphs.append((name, csr, M.Graph.from_csr(csr), G.lambda_max(csr, 50)))
    log(f"graphs ready ({time.time() - t0:.1f} s)")
    n_req = args.requests or 64
    queries = []
    for i in range(n_req):
        name, csr, g, lam = graphs[rng.integers(len(graphs))]
        fn = M.MCMF_FN_EXP if rng.random() < 0.5 else M.MCMF_FN_RESOLVENT
        scale = 1.0 / csr.d_max if fn == M.MCMF_FN_EXP else 0.85 / lam
        if rng.random() < 0.5:
            frac = rng.uniform(0.01, 0.05)
            rows = np.sort(rng.choice(csr.n, max(1, int(frac * csr.n)), replace=False))
            queries.append(Query(M, torch, g, csr, M.MCMF_REQ_DIAG, fn, scale, args.K, rows=rows,
                                 seed=args.seed, rid=i))
        else:
            queries.append(Query(M, torch, g, csr, M.MCMF_REQ_ACTION, fn, scale, args.K,
                                 v=rng.random(csr.n), seed=args.seed, rid=i))
    pick_walks(M, torch, queries, n_max=args.batch_n_max)
    log("walks per row: " + " ".join(str(q.N) for q in queries))
    stream = torch.cuda.current_stream().cuda_stream
    reqs = [q.request() for q in queries]

    def plain():
        for q in queries:
            q.single(stream)
        torch.cuda.synchronize()

    def batched(use_graph):
        o = M.mcmf_batch_opts()
        o.stream = stream
        o.use_graph = 1 if use_graph else 0
        M.mcmf_batch(reqs, o)
        torch.cuda.synchronize()

    times = {}
    results = {}
    for name, fn in (("plain", plain), ("batched", lambda: batched(False)),
                     ("batched_graph", lambda: batched(True))):
        fn()  # warm-up
        log(f"{name}: warm-up done")
        ts = []
        for _ in range(max(1, args.steps)):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
            log(f"{name}: {ts[-1] * 1e3:.1f} ms")
        times[name] = float(np.median(ts))
        results[name] = [q.out[:q.count].cpu().numpy().copy() for q in queries]
        log(f"{name}: {times[name] * 1e3:.1f} ms for {n_req} requests")
    worst = 0.0
    for a, b in zip(results["plain"], results["batched_graph"]):
        if a.size:
            worst = max(worst, float(np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-300))))
    steps = sum(r.walk_steps for r in reqs)
    return {
        "metric": "queries/s, batched vs plain one-request-at-a-time, equal walks per request",
        "value": n_req / times["batched_graph"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "higher_is_better": True, "data": "synthetic", "dtype": "f64",
        "config": {"workload": f"{n_req} requests: diag on 1-5% row subsets or f(A)v with v~U(0,1), "
                               "exp(A/d_max) or (I-0.85A/lambda_max)^-1, over ER (avg degree 10) "
                               "n=1e4/1e5/1e6, R-MAT 14/17/20 (ef 16), grid 1000x1000; "
                               f"K={args.K}; N per request from a pilot for std error {TARGET_SE}",
                   "walks_per_row": [q.N for q in queries],
                   "walks_per_row_asked_by_pilot": [q.N_pilot for q in queries],
                   "walks_per_row_cap": args.batch_n_max},
        "queries_per_s": {k: n_req / v for k, v in times.items()},
        "ms": {k: v * 1e3 for k, v in times.items()},
        "speedup_vs_plain": times["plain"] / times["batched_graph"],
        "walk_steps": steps,
        "max_rel_diff_batched_vs_plain": worst,
    }


def bench_fp32(args):
    """The Barabasi-Albert configuration (n = 4,000,000, m = 8): exp(A/d_max),
    K = 40, N = 256, the full action with v = 1 and the diagonal on 1% of the
    rows, each timed with FP64 walk weights and with FP32 walk weights (FP64
    sums) on the same walks.  Reports walk steps/s of both, the per-kernel
    device time from the library's HIP events, and the largest FP32-FP64
    difference over the stated rounding bound 2 K 2^-24 sum|terms|: the terms
    are non-negative here, so sum|terms| is the Monte Carlo part, the result
    less c_0 v + c_1 s A v (exp: c_0 = c_1 = 1)."""
    import torch
    import graphgen as G
    from paper_2308_01037_amd import mcmf as M
    assert torch.cuda.is_available(), "needs a GPU"
    K, N = args.K, args.walks
    t0 = time.time()
    csr = G.barabasi_albert(4_000_000, 8, seed=0)
    rows = G.random_rows(csr.n, csr.n // 100, seed=0)
    s = 1.0 / csr.d_max
    log(f"BA n={csr.n} nnz={csr.nnz} d_max={csr.d_max} ({time.time() - t0:.1f} s)")
    g = M.Graph.from_csr(csr)
    stream = torch.cuda.current_stream().cuda_stream
    v = torch.ones(csr.n, dtype=torch.float64, device="cuda")
    y = torch.empty(csr.n, dtype=torch.float64, device="cuda")
    d = torch.empty(len(rows), dtype=torch.float64, device="cuda")
    rt = torch.as_tensor(rows, dtype=torch.int32, device="cuda")
    f = M.make_fn(M.MCMF_FN_EXP, s)

    def query(what, precision, req):
        st = M.mcmf_stats()
        opts = M.make_opts(seed=1, request_id=req, precision=precision, stream=stream)
        if what == "action":
            M.mcmf_action(g.handle, f, v, N, K, opts, y, st)
        else:
            M.mcmf_diag(g.handle, f, rt, len(rows), N, K, opts, d, st)
        return st.as_dict()

    out = {}
    results = {}
    for pname, prec in (("fp64", M.MCMF_PRECISION_FP64), ("fp32_weights", M.MCMF_PRECISION_FP32_WEIGHTS)):
        for what in ("action", "diag"):
            query(what, prec, 1000)
            torch.cuda.synchronize()
            sts = []
            t = time.perf_counter()
            for i in range(max(1, args.steps)):
                sts.append(query(what, prec, 0))
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t) / len(sts)
            steps = sts[0]["walk_steps"]
            out.setdefault(pname, {})[what] = {
                "ms": wall * 1e3, "walk_steps": steps, "walk_steps_per_s": steps / wall,
                "ms_walk": float(np.mean([x["ms_walk"] for x in sts])),
                "ms_gather": float(np.mean([x["ms_gather"] for x in sts])),
                "ms_spmv": float(np.mean([x["ms_spmv"] for x in sts]))}
            results[(pname, what)] = (y if what == "action" else d).cpu().numpy().copy()
            log(f"{pname} {what}: {wall * 1e3:.1f} ms, {steps / wall:.3e} steps/s")
    bound_use = {}
    for what, h in (("action", 1.0 + s * csr.deg), ("diag", np.ones(len(rows)))):
        x64, x32 = results[("fp64", what)], results[("fp32_weights", what)]
        bound = 2 * K * 2.0 ** -24 * np.abs(x64 - h) + 4 * np.finfo(np.float64).eps * np.abs(x64) + 1e-30
        bound_use[what] = float(np.max(np.abs(x32 - x64) / bound))
    g.close()
    total = {p: sum(q["walk_steps"] for q in out[p].values()) / sum(q["ms"] for q in out[p].values()) * 1e3
             for p in out}
    return {
        "metric": "walk steps/s, FP32 walk weights (FP64 sums) vs FP64, same walks",
        "value": total["fp32_weights"], "unit": "walk-steps/s", "n_gpus": 1, "steps": args.steps,
        "higher_is_better": True, "data": "synthetic", "dtype": "f32 weights, f64 sums",
        "config": {"workload": f"Barabasi-Albert n=4e6 m=8 (seed K_9): exp(A/d_max), K={K}, N={N}/row; "
                               f"full f(A)1 and diag on 1% of rows ({len(rows)})",
                   "n": csr.n, "nnz": csr.nnz, "d_max": csr.d_max},
        "walk_steps_per_s": total,
        "speedup_fp32_vs_fp64": total["fp32_weights"] / total["fp64"],
        "queries": out,
        "max_diff_over_bound": bound_use,
    }


def lambda_max_device(M, torch, g, n, iters=50):
    """Largest eigenvalue by power iteration from 1/sqrt(n) * 1, every product
    A x taken by the library itself (mcmf_action with K = 1 and coefficients
    (0, 1) returns A x): x <- A x / ||A x|| for iters - 1 steps, then
    lambda = ||A x||_2."""
    stream = torch.cuda.current_stream().cuda_stream
    coeffs = np.array([0.0, 1.0])
    f = M.make_fn(M.MCMF_FN_COEFFS, 1.0, coeffs=coeffs)
    opts = M.make_opts(stream=stream)
    x = torch.full((n,), 1.0 / np.sqrt(n), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(iters - 1):
        M.mcmf_action(g.handle, f, x, 1, 1, opts, y)
        x = y / torch.linalg.norm(y)
    M.mcmf_action(g.handle, f, x, 1, 1, opts, y)
    return float(torch.linalg.norm(y))


class GraphInfo:
    """A resident graph of the serve workload: its handle and sizes (the host
    CSR is dropped once the library holds its copy)."""

    def __init__(self, name, scale, csr, g, lam):
        self.name, self.scale, self.g, self.lam = name, scale, g, lam
        self.n, self.nnz, self.d_max = csr.n, csr.nnz, csr.d_max


def serve_requests(M, torch, graphs, n_req, rng, K, N, seed):
    """The serve workload's request stream.  Each request is, with
    probability 0.8, the diagonal on a row subset of a uniformly chosen graph
    (row count log-uniform in [1, 1e5], rows uniform without repetition);
    0.1, f(A)v with v ~ U(0,1) on a graph of scale <= 21; 0.1, the full
    diagonal of a graph of scale <= 20.  f is exp(A/d_max) or
    (I - 0.85 A/lambda_max)^-1 with probability 1/2 each."""
    import types
    full_ok = [g for g in graphs if g.scale <= 20] or graphs[:1]
    act_ok = [g for g in graphs if g.scale <= 21] or graphs[:1]
    queries, kinds = [], []
    for i in range(n_req):
        u = rng.random()
        pool = full_ok if u < 0.1 else (act_ok if u < 0.2 else graphs)
        gi = pool[rng.integers(len(pool))]
        fn = M.MCMF_FN_EXP if rng.random() < 0.5 else M.MCMF_FN_RESOLVENT
        scale = 1.0 / gi.d_max if fn == M.MCMF_FN_EXP else 0.85 / gi.lam
        shape = types.SimpleNamespace(n=gi.n)
        if u < 0.1:
            q = Query(M, torch, gi.g, shape, M.MCMF_REQ_DIAG, fn, scale, K, seed=seed, rid=i)
            kinds.append(f"full diag rmat{gi.scale}")
        elif u < 0.2:
            q = Query(M, torch, gi.g, shape, M.MCMF_REQ_ACTION, fn, scale, K, v=rng.random(gi.n),
                      seed=seed, rid=i)
            kinds.append(f"f(A)v rmat{gi.scale}")
        else:
            count = int(min(gi.n, np.floor(np.exp(rng.uniform(0.0, np.log(1e5))))))
            rows = np.sort(rng.choice(gi.n, max(1, count), replace=False))
            q = Query(M, torch, gi.g, shape, M.MCMF_REQ_DIAG, fn, scale, K, rows=rows, seed=seed,
                      rid=i)
            kinds.append(f"{len(rows)} rows rmat{gi.scale}")
        q.N = N
        queries.append(q)
    return queries, kinds


def serve_run(M, torch, queries, loads, rng, opts):
    """Each offered load: Poisson arrivals; the requests one at a time in
    arrival order (plain), then the same arrivals through the server.
    Latency is arrival to result; both paths run the same walks."""
    import threading
    n_req = len(queries)
    stream = torch.cuda.current_stream().cuda_stream
    pct = lambda xs, p: float(np.percentile(xs, p) * 1e3)
    runs, worst = [], 0.0
    for qps in loads:
        arrivals = np.cumsum(rng.exponential(1.0 / qps, n_req))
        lat_plain = []
        start = time.perf_counter()
        for q, a in zip(queries, arrivals):
            now = time.perf_counter() - start
            if now < a:
                time.sleep(a - now)
            q.single(stream)
            torch.cuda.synchronize()
            lat_plain.append(time.perf_counter() - start - a)
            if len(lat_plain) % 20 == 0:
                log(f"plain at {qps:.2f}/s: {len(lat_plain)}/{n_req} requests")
        span_plain = time.perf_counter() - start
        plain_out = [q.out[:q.count].cpu().numpy().copy() for q in queries]
        srv = M.mcmf_server_create(opts)
        reqs = [q.request() for q in queries]
        tickets = [None] * n_req
        submitted = [0.0] * n_req
        infos = [None] * n_req
        start = time.perf_counter()

        def waiter():
            for i in range(n_req):
                while tickets[i] is None:
                    time.sleep(0.0002)
                infos[i] = M.mcmf_server_wait(srv, tickets[i])
                if (i + 1) % 20 == 0:
                    log(f"served at {qps:.2f}/s: {i + 1}/{n_req} requests")

        th = threading.Thread(target=waiter)
        th.start()
        for i, a in enumerate(arrivals):
            now = time.perf_counter() - start
            if now < a:
                time.sleep(a - now)
            submitted[i] = time.perf_counter() - start
            tickets[i] = M.mcmf_server_submit(srv, reqs[i])
        th.join()
        span_srv = time.perf_counter() - start
        st = M.mcmf_server_query(srv)
        M.mcmf_server_destroy(srv)
        torch.cuda.synchronize()
        # Served latency: arrival -> end of the request's batch (the server's
        # own clock from submission on).
        lat_srv = [(sub - a) + (inf.queue_ms + inf.run_ms) * 1e-3
                   for sub, a, inf in zip(submitted, arrivals, infos)]
        for q, p in zip(queries, plain_out):
            x = q.out[:q.count].cpu().numpy()
            if x.size:
                worst = max(worst, float(np.max(np.abs(x - p) / np.maximum(np.abs(p), 1e-300))))
        run = {"offered_qps": qps,
               "served": {"requests_per_s": n_req / span_srv, "p50_ms": pct(lat_srv, 50),
                          "p99_ms": pct(lat_srv, 99), "batches": st["batches"],
                          "largest_batch": st["largest_batch"],
                          "peak_batches_in_flight": st["peak_batches_in_flight"],
                          "peak_bytes_in_flight": st["peak_bytes_in_flight"]},
               "plain": {"requests_per_s": n_req / span_plain, "p50_ms": pct(lat_plain, 50),
                         "p99_ms": pct(lat_plain, 99)}}
        log(f"offered {qps:.2f}/s: served {run['served']['requests_per_s']:.2f}/s p50 "
            f"{run['served']['p50_ms']:.0f} ms p99 {run['served']['p99_ms']:.0f} ms | plain "
            f"{run['plain']['requests_per_s']:.2f}/s p50 {run['plain']['p50_ms']:.0f} ms p99 "
            f"{run['plain']['p99_ms']:.0f} ms")
        runs.append(run)
    return runs, worst


def server_opts(M, torch, reserve_bytes=0):
    o = M.mcmf_server_opts()
    o.n_streams = 4
    o.max_batch = 32
    free_b, _ = torch.cuda.mem_get_info()
    o.hbm_budget_bytes = int(max(1 << 30, (free_b - reserve_bytes) * 0.6))
    o.visit_chunk_bytes = 1 << 30
    return o


def mean_service(torch, queries):
    """Each request alone (also the warm-up); mean seconds per request."""
    stream = torch.cuda.current_stream().cuda_stream
    svc = []
    for i, q in enumerate(queries):
        t = time.perf_counter()
        q.single(stream)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t)
        if (i + 1) % 10 == 0:
            log(f"service times: {i + 1}/{len(queries)} requests")
    return float(np.mean(svc)), svc


def bench_serve(args):
    """Resident R-MAT graphs (scales 19..26 by default), Poisson arrivals of
    mixed requests (serve_requests), offered at 0.25 / 0.5 / 0.75 / 0.9 of
    the plain path's capacity: the server (continuous batching, budget
    admission) against one request at a time in arrival order."""
    import torch
    import graphgen as G
    from paper_2308_01037_amd import mcmf as M
    rng = np.random.default_rng(args.seed)
    scales = [int(x) for x in args.serve_scales.split(",")]
    graphs, csr_bytes = [], 0
    t0 = time.time()
    for i, sc in enumerate(scales):
        t1 = time.time()
        csr = G.rmat_native(sc, seed=100 + i)
        gen_s = time.time() - t1
        g = M.Graph.from_csr(csr, device=False)
        lam = lambda_max_device(M, torch, g, csr.n)
        csr_bytes += csr.nnz * 4 + (csr.n + 1) * 8
        graphs.append(GraphInfo(f"rmat{sc}", sc, csr, g, lam))
        log(f"rmat{sc}: n={csr.n} nnz={csr.nnz} d_max={csr.d_max} lambda_max={lam:.1f} "
            f"(generated in {gen_s:.1f} s, resident after {time.time() - t1:.1f} s)")
        del csr
    free_b, total_b = torch.cuda.mem_get_info()
    log(f"{len(graphs)} graphs resident: {csr_bytes / 2**30:.1f} GiB of CSR (int64 row_ptr, int32 col), "
        f"{(total_b - free_b) / 2**30:.1f} GiB of device memory in use ({time.time() - t0:.0f} s)")
    K, N = args.K, args.walks
    n_req = args.requests or 80
    queries, kinds = serve_requests(M, torch, graphs, n_req, rng, K, N, args.seed)
    mean_svc, svc = mean_service(torch, queries)
    cap = 1.0 / mean_svc
    log(f"plain capacity {cap:.2f} requests/s (mean service {mean_svc * 1e3:.1f} ms, "
        f"p50 {np.percentile(svc, 50) * 1e3:.1f} ms, max {max(svc) * 1e3:.0f} ms)")
    fracs = [0.25, 0.5, 0.75, 0.9, 2.0] if not args.qps else [args.qps / cap]
    o = server_opts(M, torch)
    runs, worst = serve_run(M, torch, queries, [f * cap for f in fracs], rng, o)
    for run, f in zip(runs, fracs):
        run["offered_fraction_of_capacity"] = f
    for gi in graphs:
        gi.g.close()
    return {
        "metric": "served requests/s and p50/p99 latency vs plain sequential, equal walks per request",
        "value": max(r["served"]["requests_per_s"] for r in runs), "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "f64",
        "config": {"workload": f"{len(scales)} resident R-MAT graphs (scales {scales}, ef 16, "
                               f"{csr_bytes / 2**30:.1f} GiB CSR); {n_req} requests: 80% diag on "
                               "row subsets (log-uniform in [1, 1e5] rows), 10% f(A)v (scale <= 21), "
                               "10% full diag (scale <= 20); exp(A/d_max) or (I-0.85A/lambda_max)^-1; "
                               f"K={K}, N={N}; Poisson arrivals",
                   "request_kinds": kinds,
                   "plain_capacity_rps": cap, "mean_sequential_service_ms": mean_svc * 1e3,
                   "server": {"n_streams": o.n_streams, "max_batch": o.max_batch,
                              "hbm_budget_bytes": o.hbm_budget_bytes,
                              "visit_chunk_bytes": o.visit_chunk_bytes}},
        "runs": runs,
        "max_rel_diff_served_vs_plain": worst,
    }


def compact_batch_and_serve(M, torch, G, g20, csr20, lam20, K, N, seed):
    """The batched and served paths against the plain one, at a size that fits
    the default run: 16 requests batched (one launch, hipGraph) vs one call
    each; 48 requests served at 0.75 of the plain capacity vs one at a time.
    The graphs: R-MAT 16, 17 and 18 (numpy generator, seeds 100..102) and the
    R-MAT 20 graph of the main workload; N and K as there."""
    rng = np.random.default_rng(seed)
    graphs = []
    for i, sc in enumerate((16, 17, 18)):
        csr = G.rmat(sc, seed=100 + i)
        g = M.Graph.from_csr(csr)
        graphs.append(GraphInfo(f"rmat{sc}", sc, csr, g, G.lambda_max(csr, 50)))
    graphs.append(GraphInfo("rmat20", 20, csr20, g20, lam20))
    stream = torch.cuda.current_stream().cuda_stream
    # Batched vs plain, 16 requests of the serve mix.
    bq, _ = serve_requests(M, torch, graphs, 16, rng, K, N, seed)
    reqs = [q.request() for q in bq]

    def plain():
        for q in bq:
            q.single(stream)
        torch.cuda.synchronize()

    def batched():
        o = M.mcmf_batch_opts()
        o.stream = stream
        o.use_graph = 1
        M.mcmf_batch(reqs, o)
        torch.cuda.synchronize()

    bt = {}
    outs = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        fn()
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        bt[name] = float(np.median(ts))
        outs[name] = [q.out[:q.count].cpu().numpy().copy() for q in bq]
    bdiff = max((float(np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-300)))
                 for a, b in zip(outs["plain"], outs["batched"]) if a.size), default=0.0)
    log(f"compact batch: plain {bt['plain'] * 1e3:.0f} ms, batched {bt['batched'] * 1e3:.0f} ms")
    # Served vs plain at 0.75 of the plain capacity.
    sq, _ = serve_requests(M, torch, graphs, 48, rng, K, N, seed)
    mean_svc, _ = mean_service(torch, sq)
    runs, sdiff = serve_run(M, torch, sq, [0.75 / mean_svc], rng, server_opts(M, torch))
    for gi in graphs[:3]:
        gi.g.close()
    r = runs[0]
    return {
        "batched": {"workload": "16 requests (80% diag on row subsets of 1..1e5 rows, 10% f(A)v, 10% "
                                "full diag) over R-MAT 16/17/18/20, one hipGraph-launched batch vs one "
                                "call per request, equal walks",
                    "queries_per_s": 16 / bt["batched"], "plain_queries_per_s": 16 / bt["plain"],
                    "speedup_vs_plain": bt["plain"] / bt["batched"], "max_rel_diff_vs_plain": bdiff},
        "served": {"workload": "48 requests of the same mix, Poisson arrivals at 0.75 of the plain "
                               "capacity, server (4 streams, budget admission) vs one at a time",
                   "offered_qps": r["offered_qps"],
                   "queries_per_s": r["served"]["requests_per_s"], "p50_ms": r["served"]["p50_ms"],
                   "p99_ms": r["served"]["p99_ms"],
                   "plain_queries_per_s": r["plain"]["requests_per_s"],
                   "plain_p50_ms": r["plain"]["p50_ms"], "plain_p99_ms": r["plain"]["p99_ms"],
                   "max_rel_diff_vs_plain": sdiff},
    }


def main():
    args = parse()
    if args.summarize:
        print(summarize(args.summarize, args.probe_bytes))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the estimator's "
              "multi-GPU sharding is a design note, not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "fp32":
        print(json.dumps(bench_fp32(args)), flush=True)
        return

    import torch
    import graphgen as G
    from paper_2308_01037_amd import mcmf as M

    if args.record_sources:
        # The kernels' source hashes and the diagonal's visit-buffer size
        # (which sets how much work one launch does), for --summarize.
        os.makedirs(os.path.dirname(os.path.abspath(args.record_sources)), exist_ok=True)
        rec = {src: source_sha(src) for _, src in KERNELS.values()}
        rec[CHUNK_KEY] = visit_chunk_bytes(torch)
        with open(args.record_sources, "w") as fh:
            json.dump(rec, fh)

    def oracle_fn_kind(fname):
        import oracle
        return oracle.FN_EXP if fname == "exp" else oracle.FN_RESOLVENT

    assert torch.cuda.is_available(), "needs a GPU"
    K, N = args.K, args.walks
    t0 = time.time()
    csr = G.rmat(args.scale, edge_factor=16, seed=0)
    log(f"R-MAT scale {args.scale}: n={csr.n} nnz={csr.nnz} d_max={csr.d_max} "
        f"({time.time() - t0:.1f} s)")
    lam = G.lambda_max(csr, 50)
    beta, gamma = 1.0 / csr.d_max, 0.85 / lam
    log(f"lambda_max={lam:.2f} beta={beta:.4e} gamma={gamma:.4e}")

    g = M.Graph.from_csr(csr)
    n = csr.n
    tuned = None
    if args.tune:
        from paper_2308_01037_amd import tuning
        tuned = tuning.autotune(g, csr, M.make_fn(M.MCMF_FN_EXP, beta), N, K, args.tune)
        log(f"tuning: {tuned}")
    stream = torch.cuda.current_stream().cuda_stream
    v = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    queries = []
    for fname, kind, scale in (("exp", M.MCMF_FN_EXP, beta), ("resolvent", M.MCMF_FN_RESOLVENT, gamma)):
        if args.only in ("all", "action"):
            queries.append(("action", fname, kind, scale))
        if args.only in ("all", "diag"):
            queries.append(("diag", fname, kind, scale))

    def step(req):
        out = []
        for qi, (what, fname, kind, scale) in enumerate(queries):
            st = M.mcmf_stats()
            opts = M.make_opts(seed=1, request_id=req, stream=stream)
            f = M.make_fn(kind, scale)
            tq = time.perf_counter()
            if what == "action":
                M.mcmf_action(g.handle, f, v, N, K, opts, y, st)
            else:
                M.mcmf_diag(g.handle, f, None, 0, N, K, opts, d, st)
            out.append((what, fname, st.as_dict(), time.perf_counter() - tq))
        return out

    for w in range(args.warmup):
        step(1000 + w)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    records = []
    for s in range(args.steps):
        records.extend(step(s))
        log(f"step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    total_steps = sum(r[2]["walk_steps"] for r in records)
    value = total_steps / elapsed
    lat = np.array([r[3] for r in records]) * 1e3
    # Launches per query: one action walk; per diagonal query one walk and one
    # gather launch per visit-buffer chunk.
    chunk_bytes = visit_chunk_bytes(torch)

    def launches_of(what, st):
        if what == "action":
            return 1
        rows_per_chunk = max(1, (chunk_bytes // 12) // (N * (K - 1)))
        return -(-st["start_rows"] // rows_per_chunk)

    # Per-kernel device time (HIP events on the call's stream, summed by the
    # library), launches and bytes over the timed region.  A full diagonal
    # makes one FP64 atomic per requested neighbour of each start row: nnz.
    kernels = {}
    for what, fname, st, _ in records:
        parts = [("action_walk", st["ms_walk"])] if what == "action" else \
            [("diag_walk", st["ms_walk"]), ("diag_gather", st["ms_gather"])]
        for kind, ms in parts:
            k = kernels.setdefault(kind, {"ms": 0.0, "bytes": 0, "layout": 0, "launches": 0})
            k["ms"] += ms
            k["bytes"] += algorithmic_bytes(kind, st, atomics=csr.nnz)
            k["layout"] += layout_bytes(kind, st)
            k["launches"] += launches_of(what, st)
    for kind, k in kernels.items():
        k["gbs"] = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
        k["traffic"] = load_traffic(kind, chunk_bytes)  # counter bytes per launch, None if stale
        k["per_launch"] = k["bytes"] / k["launches"]
        k["ms_per_launch"] = k["ms"] / k["launches"]
        log(f"{kind}: {k['ms'] / args.steps:.1f} ms/step, {k['launches']} launches, "
            f"{k['gbs']:.1f} GB/s algorithmic ({k['gbs'] / HBM_PEAK_GBS:.3f} of peak)")
    # The diagonal query as a whole, with the method's own bytes per query:
    # 4 B for every column entry of every requested neighbour of every start
    # row (sum of deg(i)^2 over the requested rows: the probes the gather
    # would make with no hub sums), 8 B per atomic into d and 12 B per walk
    # transition, over the query's walk and gather time.  Hub sums done by the
    # walk and summed hub columns skipped by the gather count here at the
    # method's price, which the per-kernel figures leave out.
    diag_recs = [st for what, _, st, _ in records if what == "diag"]
    diag_query = None
    if diag_recs:
        deg = csr.deg.astype(np.float64)
        method_bytes = 4.0 * float(np.dot(deg, deg)) + 8.0 * csr.nnz
        per_q = [(method_bytes + 12.0 * (st["walk_steps"] - st["walks"]),
                  st["ms_walk"] + st["ms_gather"]) for st in diag_recs]
        b_q = sum(b for b, _ in per_q) / len(per_q)
        ms_q = sum(ms for _, ms in per_q) / len(per_q)
        diag_query = {"method_bytes_per_query": b_q, "ms_per_query": ms_q,
                      "gbs_method": b_q / (ms_q * 1e-3) / 1e9,
                      "frac": b_q / (ms_q * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"diag query: {ms_q:.1f} ms walk + gather, {b_q / 1e9:.1f} GB method bytes, "
            f"{diag_query['gbs_method']:.1f} GB/s ({diag_query['frac']:.3f} of peak)")
    dominant = max(kernels, key=lambda kk: kernels[kk]["ms"])
    dk = kernels[dominant]
    alg_total = sum(k["bytes"] for k in kernels.values())
    if args.copy_probe_bytes:
        src = torch.ones(args.copy_probe_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_probe_bytes} bytes done")

    compact = None
    if not args.no_compact and args.only == "all" and not args.copy_probe_bytes:
        t_c = time.time()
        compact = compact_batch_and_serve(M, torch, G, g, csr, lam, K, N, args.seed)
        log(f"compact batched/served legs: {time.time() - t_c:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        oq = [(what, oracle_fn_kind(fname), beta if fname == "exp" else gamma)
              for what, fname, _, _ in queries]
        rate, steps_c, secs, nrows, core, er1000 = cpu_baseline(csr, oq, args.cpu_steps, K, N)
        model, allowed, logical = host_cpu()
        cpu = {"value": rate, "unit": "walk-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"each of the {len(oq)} queries evaluated at {nrows} random non-isolated "
                         f"rows (walks from their neighbourhoods): {steps_c} walk steps in "
                         f"{secs:.1f} s, single thread pinned to logical CPU {core}",
               "host_cpu": model, "host_logical_cpus": logical, "cpus_allowed": allowed,
               "er1000_end_to_end": er1000}

    def frac(k):
        return k["gbs"] / HBM_PEAK_GBS

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"rmat{args.scale}-ef16 (a,b,c)=(.57,.19,.19) symmetrised: full diag and "
                        f"f(A)1 for exp(A/d_max) and (I-0.85A/lambda_max)^-1, K={K}, N={N}/row",
            "n": csr.n, "nnz": csr.nnz, "d_max": csr.d_max, "lambda_max": lam,
            "K": K, "walks_per_row": N, "queries_per_step": len(queries),
        },
        "queries_per_s": len(records) / elapsed,
        "query_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "hbm_gbs_algorithmic": alg_total / elapsed / 1e9,
        "kernels": {k: {"ms_per_step": v_["ms"] / args.steps,
                        "launches_per_step": v_["launches"] / args.steps,
                        "ms_per_launch": v_["ms_per_launch"],
                        "algorithmic_bytes_per_launch": v_["per_launch"],
                        "layout_bytes_per_launch": v_["layout"] / v_["launches"],
                        "gbs_algorithmic": v_["gbs"], "frac": frac(v_),
                        "traffic_bytes_per_launch": v_["traffic"],
                        "traffic_over_algorithmic": (v_["traffic"] / v_["per_launch"]
                                                     if v_["traffic"] else None)}
                    for k, v_ in kernels.items()},
        "diag_query": diag_query,
        "roofline": {
            "kernel": dominant,
            "bound": "hbm",
            "achieved": dk["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": frac(dk),
            "traffic": dk["traffic"],
            "bytes_per_launch": dk["per_launch"],
            "ms_per_launch": dk["ms_per_launch"],
            "launches": dk["launches"],
        },
        "cpu_baseline": cpu,
    }
    if compact is not None:
        result.update(compact)
    if tuned is not None:
        result["tuning"] = tuned
    g.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

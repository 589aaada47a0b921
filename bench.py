#!/usr/bin/env python3
"""Benchmark: GB/s of text recognized by chunked RI-DFA speculation (RID)
against all-states DFA speculation, bit-exact, with p50/p99 per call.

One step = one recognition of the whole text: reach kernels, join kernels
and finalize kernel, with the text already resident in HBM.  The value is
K steps queued back to back on one stream (ri_recognize_async, results left
on the device and checked after the final wait); p50/p99 are per-call times
of the synchronous ri_recognize_ex, which also reads the result back.
Default workload: the structured log lines (about 1 GiB, minimal DFA of
302 states, interface of 227 starts).  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload log|motif|tiny|batch|serve|sweep]
                  [--chunks C] [--seed S] [--algos rid,dfa] [--no-cpu-baseline]

Besides RID and the all-states minimal DFA, the single-text workloads time
the all-states powerset (subset) DFA of the position NFA, and the tiny
(a|b)*a(a|b)^3 workload at exactly 64 chunks (the paper's chunk count) and
at the tuned chunk count.  The CPU leg times the oracle's serial scan on one
core (`cpu_baseline.value`) and the paper's own CPU scheme, one thread per
chunk on every usable core, for RID and the DFA on a 64 MiB prefix.

--workload batch: 4096 texts (1 KiB - 4 MiB, log-uniform, about 2 GB) over
16 random expressions, recognized by one captured graph launch of a batch
(ri_batch_*, one launch sequence per automaton), RID and all-states DFA,
against the same batch with the long runs of every automaton in one
work-queue launch (RI_BATCH_QUEUE) and against one ri_recognize_ex call per
text.

--workload sweep: the regexp family (a|b)*a(a|b)^k for k = 3..12 (minimal
DFA 2^(k+1) states, interface k+2): GB/s of RID and of the all-states DFA,
converging and plain reach, on 64 MiB texts; the CPU leg times the oracle's
chunked recognizers on a 64 KiB sample and reports their transition counts
(NFA, DFA and RID chunk automata).

--workload serve: a pool of 64 resident keyword-union automata
.*(k1|...|kn).* (n in 200..2000), requests with log-normal text lengths
(median 64 KiB, sigma 1, cap 64 MiB), a keyword planted in half of them;
capacity (all requests at once), then Poisson arrivals at fractions of it:
p50/p99 latency and GB/s, RID and all-states DFA.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="log", choices=["log", "motif", "tiny", "batch", "serve", "sweep"])
    ap.add_argument("--algos", default="rid,dfa",
                    help="single-text workloads: algorithms to time (rid first; 'rid' alone for profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the subset-DFA baseline and the tiny workload at 64 chunks")
    ap.add_argument("--cpu-prefix-mib", type=int, default=64,
                    help="CPU leg: text prefix recognized by the threaded CPU scheme")
    ap.add_argument("--ks", default="3,4,5,6,7,8,9,10,11,12", help="sweep workload: k values")
    ap.add_argument("--sweep-mib", type=int, default=64, help="sweep workload: text MiB per k")
    ap.add_argument("--automata", type=int, default=64, help="serve workload: automata in the pool")
    ap.add_argument("--requests", type=int, default=2000, help="serve workload: requests per run")
    ap.add_argument("--loads", default="0.25,0.5,0.8", help="serve workload: offered loads (fractions of capacity)")
    ap.add_argument("--texts", type=int, default=4096, help="batch workload: number of texts")
    ap.add_argument("--procs", type=int, default=8, help="batch workload: text generator processes")
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="skip ri_autotune (the chunk count is then the library default)")
    ap.add_argument("--tune-rid", metavar="TARGET:WARM:RUNS[:CONVERGE]",
                    help="use these reach settings for RID instead of ri_autotune")
    ap.add_argument("--tune-dfa", metavar="TARGET:WARM:RUNS[:CONVERGE]",
                    help="use these reach settings for the DFA instead of ri_autotune")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the paper-literal (non-merging) reach comparison")
    ap.add_argument("--calib-copy", action="store_true",
                    help="one 256 MiB device-to-device copy before timing (known-size kernel "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn two rocprofv3 --pmc counter CSVs into the traffic record "
                         "under profiles/ and exit")
    return ap.parse_args()


# sources of the reach kernels (the long-run kernel and its helpers)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2412_14975_amd", "csrc", f)
               for f in ("k_reach.hip", "device.hpp", "kernels.hpp")]
CALIB_BYTES = 256 << 20


def kernel_source_hash():
    """Hash of the reach kernels' code: comments and layout are left out,
    so that only a change of the code itself drops the traffic record."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def traffic_record_path(workload_name):
    return os.path.join(ROOT, "profiles", f"traffic_long_kernel_{workload_name}.json")


def summarize_traffic(fetch_csv, write_csv, workload_name):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the RID long-run kernel,
    scaled by the same counters read on the known-size calibration copy."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        by_dispatch = {}
        for r in rows:
            by_dispatch.setdefault((r["Dispatch_Id"], r["Kernel_Name"]), 0.0)
            by_dispatch[(r["Dispatch_Id"], r["Kernel_Name"])] += float(r["Counter_Value"])
        return by_dispatch

    out = {"kernel_source_sha256": kernel_source_hash(), "workload": workload_name}
    for counter, path, key in (("FETCH_SIZE", fetch_csv, "fetch"), ("WRITE_SIZE", write_csv, "write")):
        d = per_kernel(path, counter)
        copies = [v for (i, k), v in d.items() if "copyBuffer" in k]
        longs = [v for (i, k), v in d.items() if "long_kernel<unsigned short" in k]
        calib = max(copies)                      # the 256 MiB copy is the largest copy
        factor = CALIB_BYTES / (calib * 1024.0)
        med = float(np.median(longs))
        out[key] = {"kib_per_dispatch_raw": med, "calib_copy_kib_raw": calib,
                    "scale": factor, "bytes_per_dispatch": med * 1024.0 * factor,
                    "dispatches": len(longs)}
    out["traffic_bytes_per_launch"] = out["fetch"]["bytes_per_dispatch"] + out["write"]["bytes_per_dispatch"]
    with open(traffic_record_path(workload_name), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def load_traffic(workload_name):
    p = traffic_record_path(workload_name)
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None    # kernels changed since the counters were taken
    return rec


def workload(name, seed):
    from workloads import gen
    if name == "motif":
        rx, motifs = gen.c2_regex_and_motifs(seed)
        x, _ = gen.c2_texts(seed, motifs=motifs)
        return rx, x, "motif-union-ACGT-256MiB"
    if name == "log":
        rx = gen.c3_regex()
        x, _, _ = gen.c3_texts(seed)
        return rx, x, "log-lines-1GiB"
    rx = gen.c1_regex()
    x, _ = gen.c1_texts(seed)
    return rx, x, "regexp-k3-1MiB"


def apply_setting(rec, setting):
    """setting: dict with chunk_target / warmup_bytes / runs_per_lane, or None
    (keep what ri_autotune stored in the handle)."""
    if setting:
        for k in ("chunk_target", "warmup_bytes", "runs_per_lane", "converge"):
            if k in setting:
                rec.set_option(k, setting[k])


def time_algo(torch, rec, t, algo, chunks, steps, warmup, want, setting=None):
    """Returns dict with per-call times (s), whole-run time and kernel timings."""
    apply_setting(rec, setting)
    for _ in range(warmup):
        r = rec.recognize(t, algo=algo, chunks=chunks)
    torch.cuda.synchronize()
    rec.set_profiling(True)
    per_call, reach_ms, join_ms, kern_ms, warm_ms, exact = [], [], [], [], [], True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c0 = time.perf_counter()
        r = rec.recognize(t, algo=algo, chunks=chunks)
        per_call.append(time.perf_counter() - c0)
        ms = rec.last_timings()
        reach_ms.append(ms[0])
        join_ms.append(ms[1])
        kern_ms.append(ms[3])
        warm_ms.append(ms[4])
        exact &= (r["accept"], r["final_state"]) == want
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    rec.set_profiling(False)
    # the same steps back to back on one stream: each call enqueues the whole
    # path and leaves its result on the device, one wait at the end
    res = torch.full((steps, 2), -7, dtype=torch.int32, device="cuda")
    rec.recognize_async(t, res[0], algo=algo, chunks=chunks)
    torch.cuda.synchronize()
    q0 = time.perf_counter()
    for i in range(steps):
        rec.recognize_async(t, res[i], algo=algo, chunks=chunks)
    torch.cuda.synchronize()
    queued = time.perf_counter() - q0
    exact &= all((bool(a), int(f)) == want for a, f in res.cpu().numpy())
    return dict(per_call=np.array(per_call), total=total, queued=queued, reach_ms=np.array(reach_ms),
                join_ms=np.array(join_ms), kern_ms=np.array(kern_ms), warm_ms=np.array(warm_ms),
                result=r, exact=exact)



# ---------------------------------------------------------------------------
# batched workload
# ---------------------------------------------------------------------------

BATCH_SEED = 21


def _batch_texts(job):
    """Worker: texts [i0, i1) of the batched workload."""
    from workloads import gen
    spec, lengths, i0, i1 = job
    seed = spec["seed"]
    trees = {}
    out = []
    for i in range(i0, i1):
        k = i % len(spec["expressions"])
        if k not in trees:
            _, tree, alphabet = gen.c4_candidate(seed, spec["expressions"][k]["index"])
            trees[k] = (tree, alphabet)
        x, changed = gen.c4_text(BATCH_SEED, i, trees[k][0], trees[k][1], int(lengths[i]))
        out.append((k, x, changed))
    return out


def batch_workload(count, procs):
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    from workloads import gen
    spec = json.load(open(os.path.join(ROOT, "tests", "golden", "c4_regexes.json")))
    lengths = gen.c4_lengths(BATCH_SEED, count=count)
    step = 32
    jobs = [(spec, lengths, i, min(count, i + step)) for i in range(0, count, step)]
    items = []
    # generated before the GPU is touched (fork of a process without a device context)
    with ProcessPoolExecutor(max_workers=max(1, procs), mp_context=mp.get_context("fork")) as ex:
        for part in ex.map(_batch_texts, jobs):
            items.extend(part)
    regexes = [gen.c4_candidate(spec["seed"], e["index"])[0] for e in spec["expressions"]]
    return spec, regexes, items


def main_batch(args):
    t_gen = time.perf_counter()
    spec, regexes, items = batch_workload(args.texts, args.procs)
    total = sum(len(x) for _, x, _ in items)
    print(f"# batch workload: {len(items)} texts, {total} bytes, {len(regexes)} expressions "
          f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)

    import torch
    import paper_2412_14975_amd as ri
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(2)

    # expected results: the oracle's minimal DFAs and serial scans (threads:
    # the C scan runs without the interpreter lock)
    refs = []
    for rx in regexes:
        d = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(rx)))
        refs.append((d, oracle.dense_table(d.n, d.delta)))
    with ThreadPoolExecutor(max_workers=max(1, args.procs)) as ex:
        want = list(ex.map(lambda it: oracle.serial(refs[it[0]][0], it[1], refs[it[0]][1]), items))
    print(f"# oracle results: {sum(w[0] for w in want)} of {len(want)} accepted", file=sys.stderr, flush=True)

    # texts packed at 16-byte aligned offsets in one device buffer
    offs, pos = [], 0
    for _, x, _ in items:
        offs.append(pos)
        pos += (len(x) + 15) // 16 * 16
    host = torch.empty(max(pos, 16), dtype=torch.uint8, pin_memory=True)
    hv = host.numpy()
    for (_, x, _), o in zip(items, offs):
        hv[o:o + len(x)] = x
    buf = host.to("cuda")
    views = [buf[o:o + len(x)] for (_, x, _), o in zip(items, offs)]
    recs = [ri.Recognizer(rx) for rx in regexes]
    torch.cuda.synchronize()

    res, res_pg, res_auto = {}, {}, {}
    # the grouped plan (one launch sequence per automaton), the long runs of
    # every automaton in one work-queue launch, and the automatic mode, whose
    # autotune picks one of the two
    for mode, algo in (("grouped", "rid"), ("grouped", "dfa"), ("queue", "rid"), ("queue", "dfa"),
                       ("auto", "rid"), ("auto", "dfa")):
        t0 = time.perf_counter()
        b = ri.Batch([(recs[k], v, algo) for (k, _, _), v in zip(items, views)], mode=mode)
        tun = b.autotune()
        b.capture()
        setup_s = time.perf_counter() - t0
        for _ in range(args.warmup):
            b.launch()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record(st)
            b.launch(st)
            e1.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
        got = b.results[: 2 * len(items)].view(-1, 2).cpu().numpy()
        exact = all((bool(g[0]), int(g[1])) == w for g, w in zip(got, want))
        info = b.info()
        groups = [b.group(g) for g in range(info["groups"])]
        b.close()
        dest = {"grouped": res, "queue": res_pg, "auto": res_auto}[mode]
        dest[algo] = dict(
                         gbps=total * args.steps / wall / 1e9, ms_per_step=wall / args.steps * 1e3,
                         p50_ms=float(np.percentile(ms, 50)), p99_ms=float(np.percentile(ms, 99)),
                         gbps_p50=total / (np.percentile(ms, 50) * 1e-3) / 1e9,
                         gbps_p99=total / (np.percentile(ms, 99) * 1e-3) / 1e9,
                         bitexact=bool(exact), setup_s=setup_s, chunks=int(info["slots"]),
                         kernels=int(info["kernels"]), device_bytes=int(info["device_bytes"]),
                         tuning=dict(trials=tun["trials"], best_ms=tun["best_ms"],
                                     chunk_bytes=sorted({g["chunk_bytes"] for g in groups}),
                                     warmup_bytes=sorted({g["warmup_bytes"] for g in groups})))
        if mode == "auto":
            dest[algo]["plan"] = "fused" if info["fused"] else "queue" if info["queue"] else "grouped"
        m = dest[algo]
        print(f"# batch {mode} {algo}: {m['gbps']:.1f} GB/s exact={exact}", file=sys.stderr, flush=True)

    # one ri_recognize_ex call per text (each call enqueues its kernels and
    # waits for its result), same texts, same automata
    per_text = {}
    for algo in ("rid", "dfa"):
        for k, v in zip(range(64), views):    # warm the per-stream workspaces
            recs[items[k][0]].recognize(v, algo=algo)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        exact = True
        for (k, _, _), v, w in zip(items, views, want):
            r = recs[k].recognize(v, algo=algo)
            exact &= (r["accept"], r["final_state"]) == w
        wall = time.perf_counter() - w0
        per_text[algo] = dict(gbps=total / wall / 1e9, ms=wall * 1e3, bitexact=bool(exact))
        print(f"# per-text {algo}: {per_text[algo]['gbps']:.1f} GB/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        # oracle serial scans, one host core, texts in order until about --cpu-seconds
        c0, nbytes, ntexts = time.perf_counter(), 0, 0
        while time.perf_counter() - c0 < args.cpu_seconds:
            k, x, _ = items[ntexts % len(items)]
            oracle.serial(refs[k][0], x, refs[k][1])
            nbytes += len(x)
            ntexts += 1
        dt = time.perf_counter() - c0
        cpu = dict(value=round(nbytes / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                   sample=f"oracle serial minimal-DFA scans of the first {ntexts} texts "
                          f"({nbytes} bytes, {dt:.1f} s)")

    r = res["rid"]
    achieved = total / (r["p50_ms"] * 1e-3) / 1e9
    out = {
        "metric": "GB/s of text recognized, RI-DFA vs all-states DFA speculation (bit-exact); p50/p99",
        "value": round(r["gbps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"batched-{len(items)}-texts-16-expressions", "n_bytes": total,
                   "texts": len(items), "expressions": len(regexes), "text_seed": BATCH_SEED,
                   "expression_seed": spec["seed"], "launch": "one captured hipGraph per step"},
        "p50_ms": round(r["p50_ms"], 4),
        "p99_ms": round(r["p99_ms"], 4),
        "bitexact": all(v["bitexact"] for v in res.values()) and all(v["bitexact"] for v in per_text.values())
        and all(v["bitexact"] for v in res_pg.values()) and all(v["bitexact"] for v in res_auto.values()),
        "batch": {a: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()} for a, m in res.items()},
        "batch_work_queue": {a: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()}
                             for a, m in res_pg.items()},
        "speedup_work_queue_vs_grouped": round(res_pg["rid"]["gbps"] / res["rid"]["gbps"], 4),
        "batch_auto": {a: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()}
                       for a, m in res_auto.items()},
        "per_text_calls": {a: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()}
                           for a, m in per_text.items()},
        "speedup_rid_vs_dfa": round(res["rid"]["gbps"] / res["dfa"]["gbps"], 4),
        "speedup_batch_vs_per_text": round(res["rid"]["gbps"] / per_text["rid"]["gbps"], 4),
        "command": " ".join(["python", "bench.py"] + sys.argv[1:]),
        "roofline": dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                         kernel="whole batch graph (text bytes / p50 graph time)",
                         algorithmic_bytes=int(total)),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for rc in recs:
        rc.close()


# ---------------------------------------------------------------------------
# serving workload
# ---------------------------------------------------------------------------

SERVE_SEED = 11


def main_serve(args):
    import torch
    import paper_2412_14975_amd as ri
    from concurrent.futures import ThreadPoolExecutor
    from workloads import gen
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(2)
    t0 = time.perf_counter()
    autos = [gen.c5_automaton(SERVE_SEED, i) for i in range(args.automata)]
    with ThreadPoolExecutor(max_workers=max(1, args.procs)) as ex:   # ri_build runs without the interpreter lock
        recs = list(ex.map(lambda a: ri.Recognizer(a[0]), autos))
    infos = [r.info() for r in recs]
    print(f"# {len(recs)} automata built ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    reqs = [(k, x) for _, k, x in gen.c5_requests(args.requests, [a[1] for a in autos], seed=SERVE_SEED)]
    total = sum(len(x) for _, x in reqs)
    # the oracle's results for this request stream (tests/golden/c5_serving.json,
    # written by tests/golden/make_c5_goldens.py from the oracle alone)
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "c5_serving.json")
    if os.path.exists(gpath) and args.automata == 64:
        g = json.load(open(gpath))
        rows = {r[0]: r for r in g["requests"]}
        if g["seed"] == SERVE_SEED and all(i in rows for i in range(len(reqs))):
            golden = {i: (bool(rows[i][3]), int(rows[i][4])) for i in range(len(reqs))}
            assert all(rows[i][1] == reqs[i][0] and rows[i][2] == len(reqs[i][1]) for i in range(len(reqs)))
    print(f"# {len(reqs)} requests, {total} bytes", file=sys.stderr, flush=True)
    loads = [float(v) for v in args.loads.split(",") if v]
    # device only: every text resident, one fused batch, timed with events
    dev_texts, device = [], {}
    for _, x in reqs:
        dev_texts.append(torch.from_numpy(x).to("cuda"))
    for algo in ("rid", "dfa"):
        b = ri.Batch([(recs[k], t, algo) for (k, _), t in zip(reqs, dev_texts)], mode="fused")
        try:
            tun = b.autotune()
            b.run()
            torch.cuda.synchronize()
            got = b.results[: 2 * len(reqs)].view(-1, 2).cpu().numpy()
            dev_exact = None if golden is None else all(
                (bool(got[i][0]), int(got[i][1])) == golden[i] for i in range(len(reqs)))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                b.run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            g0 = b.group(0)
            device[algo] = dict(gbps=total / (ms * 1e-3) / 1e9, ms=ms, bitexact_vs_oracle=dev_exact,
                                chunk_bytes=g0["chunk_bytes"],
                                warmup_bytes=g0["warmup_bytes"], tuning_trials=tun["trials"],
                                slots=int(b.info()["slots"]))
        finally:
            b.close()
        print(f"# device {algo}: {device[algo]['gbps']:.1f} GB/s", file=sys.stderr, flush=True)
    del dev_texts
    out_algo, results_by_algo = {}, {}
    for algo in ("rid", "dfa"):
        srv = ri.serve.Server(recs, algo=algo, slots=3, hbm_budget=32 << 30)
        try:
            # capacity: every request present at once
            c0 = time.perf_counter()
            for k, x in reqs:
                srv.submit(k, x, arrival=c0)
            done = srv.drain()
            wall = time.perf_counter() - c0
            results_by_algo[algo] = {d["id"]: (d["accept"], d["final_state"]) for d in done}
            cap_rps = len(reqs) / wall
            entry = dict(capacity=dict(gbps=total / wall / 1e9, req_per_s=cap_rps, wall_s=wall, steps=srv.steps))
            # Poisson arrivals at fractions of the capacity
            for frac in loads:
                qps = frac * cap_rps
                t, sched = 0.0, []
                prng = gen.PCG(SERVE_SEED + 2)
                for k, x in reqs:
                    t += float(prng.exponential(1.0 / qps))
                    sched.append((t, k, x))
                steps0 = srv.steps
                done, wall = ri.serve.run_open_loop(srv, sched)
                lat = np.array([d["latency"] for d in done])
                same = all((d["accept"], d["final_state"]) == results_by_algo[algo][d["id"] - len(reqs) * (1 + loads.index(frac))]
                           for d in done)
                entry[f"load_{frac:g}"] = dict(offered_req_per_s=qps, gbps=total / wall / 1e9,
                                               p50_ms=float(np.percentile(lat, 50) * 1e3),
                                               p99_ms=float(np.percentile(lat, 99) * 1e3),
                                               steps=srv.steps - steps0, same_results=bool(same))
                print(f"# serve {algo} load {frac}: p50 {entry[f'load_{frac:g}']['p50_ms']:.2f} ms "
                      f"p99 {entry[f'load_{frac:g}']['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
            entry["max_device_bytes_in_flight"] = srv.max_used
        finally:
            srv.close()
        out_algo[algo] = entry
    # every request: RID and DFA agree, and a sample agrees with single-text calls
    agree = all(results_by_algo["rid"][i] == results_by_algo["dfa"][i] for i in range(len(reqs)))
    alone_ok = True
    for i in range(0, len(reqs), max(1, len(reqs) // 50)):
        k, x = reqs[i]
        if len(x) == 0:
            continue
        r = recs[k].recognize(torch.from_numpy(x).to("cuda"), algo="rid")
        alone_ok &= (r["accept"], r["final_state"]) == results_by_algo["rid"][i]
    rid = out_algo["rid"]
    out = {
        "metric": "GB/s of text recognized, RI-DFA vs all-states DFA speculation (bit-exact); p50/p99",
        "value": round(device["rid"]["gbps"], 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": 5,
        "warmup": 1,
        "ms_per_step": round(device["rid"]["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"serving-{len(recs)}-keyword-automata", "requests": len(reqs), "n_bytes": total,
                   "keyword_seed": SERVE_SEED, "interface_states": [min(i["interface_states"] for i in infos),
                                                                     max(i["interface_states"] for i in infos)],
                   "min_dfa_states": [min(i["min_dfa_states"] for i in infos), max(i["min_dfa_states"] for i in infos)],
                   "slots": 3, "loads": loads},
        "bitexact": bool(agree and alone_ok) if golden is None else bool(
            all(results_by_algo[a][i] == golden[i] for a in ("rid", "dfa") for i in range(len(reqs)))
            and all(device[a]["bitexact_vs_oracle"] for a in ("rid", "dfa"))),
        "bitexact_against": "GPU self-consistency only (no oracle results for this request stream)"
        if golden is None else "oracle results of every request (tests/golden/c5_serving.json): serving "
                               "loop and device-only fused batch, RID and DFA",
        "serve": {a: {k: ({kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          if isinstance(v, dict) else v) for k, v in e.items()} for a, e in out_algo.items()},
        "serving_speedup_rid_vs_dfa": round(rid["capacity"]["gbps"] / out_algo["dfa"]["capacity"]["gbps"], 4),
        "note": "value: one fused batch of every request with the texts resident in HBM; serve.*: the "
                "serving loop with texts arriving in host memory (staging and PCIe included)",
        "device_only": {a: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()}
                        for a, m in device.items()},
        "device_speedup_rid_vs_dfa": round(device["rid"]["gbps"] / device["dfa"]["gbps"], 4),
        "command": " ".join(["python", "bench.py"] + sys.argv[1:]),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    for r in recs:
        r.close()


# ---------------------------------------------------------------------------
# regexp-family sweep
# ---------------------------------------------------------------------------

def main_sweep(args):
    import torch
    import paper_2412_14975_amd as ri
    from workloads import gen
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(2)
    import oracle
    ks = [int(v) for v in args.ks.split(",") if v]
    rows = []
    for k in ks:
        rx = gen.regexp_family(k)
        x, rej = gen.c1_texts(100 + k, n=args.sweep_mib << 20)
        # expected result: the oracle's minimal DFA, serial scan
        d = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(rx)))
        owant = oracle.serial(d, x, oracle.dense_table(d.n, d.delta))
        t = torch.from_numpy(x).to("cuda")
        rec = ri.Recognizer(rx)
        info = rec.info()
        row = dict(k=k, min_dfa_states=info["min_dfa_states"], interface_states=info["interface_states"],
                   ridfa_states=info["ridfa_states"], nfa_states=info["nfa_states"], bitexact=True)
        for algo in ("rid", "dfa"):
            tun = rec.autotune(t, algo=algo)
            want = owant
            for conv in (1, 0):
                rec.set_option("converge", conv)
                if conv:
                    rec.set_option("chunk_target", tun["chunk_target"])
                    rec.set_option("warmup_bytes", tun["warmup_bytes"])
                    rec.set_option("runs_per_lane", tun["runs_per_lane"])
                else:
                    rec.set_option("chunk_target", 65536)
                r = rec.recognize(t, algo=algo)
                torch.cuda.synchronize()
                c0 = time.perf_counter()
                for _ in range(args.steps):
                    r = rec.recognize(t, algo=algo)
                dt = (time.perf_counter() - c0) / args.steps
                row[f"{algo}_{'conv' if conv else 'plain'}_gbps"] = round(len(x) / dt / 1e9, 2)
                row["bitexact"] &= (r["accept"], r["final_state"]) == want
            row[f"{algo}_accept"] = bool(want[0])
        # the NFA device (position NFA over sets of states)
        tun = rec.autotune(t, algo="nfa")
        rec.set_option("chunk_target", tun["chunk_target"])
        r = rec.recognize(t, algo="nfa")
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(args.steps):
            r = rec.recognize(t, algo="nfa")
        dt = (time.perf_counter() - c0) / args.steps
        row["bitexact"] &= (r["accept"], r["final_state"]) == owant
        row["nfa_gbps"] = round(len(x) / dt / 1e9, 2)
        row["rid_over_nfa"] = round(row["rid_conv_gbps"] / row["nfa_gbps"], 2)
        rec.close()
        del t
        torch.cuda.empty_cache()
        rows.append(row)
        print(f"# k={k}: {row}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's chunked recognizers on a 64 KiB sample with 64 chunks:
        # their time and their transition counts (NFA, DFA and RID chunk automata)
        import oracle
        counts = []
        c0 = time.perf_counter()
        for k in ks:
            b = oracle.build(gen.regexp_family(k))
            x, _ = gen.c1_texts(100 + k, n=1 << 16)
            bounds = oracle.even_bounds(len(x), 64)
            d = oracle.csdpa(b.dfa, x, bounds)
            r = oracle.rid(b.Bq, x, bounds)
            nfa_t = oracle.nfa_csdpa_transitions(b.nfa, x, bounds)
            counts.append(dict(k=k, dfa=d["transitions"], rid=r["transitions"], nfa=nfa_t,
                               dfa_over_rid=round(d["transitions"] / max(1, r["transitions"]), 2)))
        dt = time.perf_counter() - c0
        cpu = dict(value=round(len(ks) * (1 << 16) * 3 / dt / 1e9, 6), unit="GB/s", cores=1, kind="oracle",
                   sample=f"oracle CSDPA (DFA), RID and NFA chunked recognition of a 64 KiB text with 64 "
                          f"chunks for each k ({dt:.1f} s)", transitions=counts)
    best = max(rows, key=lambda r: r["k"])
    out = {
        "metric": "GB/s of text recognized, RI-DFA vs all-states DFA speculation (bit-exact); p50/p99",
        "value": best["rid_conv_gbps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"regexp-family-sweep-{args.sweep_mib}MiB", "ks": ks},
        "sweep": rows,
        "bitexact": all(r["bitexact"] for r in rows),
        "command": " ".join(["python", "bench.py"] + sys.argv[1:]),
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload == "sweep" and not args.traffic_from:
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py: this recognizer runs on one GPU only; --gpus must be 1", file=sys.stderr)
            sys.exit(2)
        main_sweep(args)
        return
    if args.workload == "serve" and not args.traffic_from:
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py: this recognizer runs on one GPU only; --gpus must be 1", file=sys.stderr)
            sys.exit(2)
        main_serve(args)
        return
    if args.workload == "batch" and not args.traffic_from:
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py: this recognizer runs on one GPU only; --gpus must be 1", file=sys.stderr)
            sys.exit(2)
        main_batch(args)
        return
    if args.traffic_from:
        names = {"motif": "motif-union-ACGT-256MiB", "log": "log-lines-1GiB", "tiny": "regexp-k3-1MiB"}
        summarize_traffic(args.traffic_from[0], args.traffic_from[1], names[args.workload])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this recognizer runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2412_14975_amd as ri

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(2)

    rx, x, wname = workload(args.workload, args.seed)
    n = len(x)
    algos = [a for a in args.algos.split(",") if a]
    if not algos or any(a not in ("rid", "dfa") for a in algos) or len(set(algos)) != len(algos):
        print("bench.py: --algos names rid and/or dfa", file=sys.stderr)
        sys.exit(2)
    # the line's value is the first named algorithm's (rid unless profiling the DFA alone)
    prim = algos[0]
    print(f"# workload {wname}: n={n} bytes", file=sys.stderr, flush=True)

    # expected result from the oracle (serial scan, host)
    import oracle
    ref = oracle.build(rx)
    table = oracle.dense_table(ref.dfa.n, ref.dfa.delta)
    want = oracle.serial(ref.dfa, x, table)
    print(f"# oracle result {want}", file=sys.stderr, flush=True)

    rec = ri.Recognizer(rx)
    info = rec.info()
    t = torch.from_numpy(x).to("cuda")
    torch.cuda.synchronize()
    if args.calib_copy:
        src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tuning, fixed = {}, {}
    for algo, spec in (("rid", args.tune_rid), ("dfa", args.tune_dfa)):
        if spec:
            vals = [int(v) for v in spec.split(":")]
            fixed[algo] = dict(chunk_target=vals[0], warmup_bytes=vals[1], runs_per_lane=vals[2],
                               converge=vals[3] if len(vals) > 3 else 1)
            tuning[algo] = dict(fixed[algo], trials=0, source="given")
    if not args.no_tune and args.chunks == 0:
        # setup, outside the timed region: pick chunk target / warm-up / runs
        # per lane for each algorithm on this text (same grid for both)
        for algo in algos:
            if algo in fixed:
                continue
            tuning[algo] = rec.autotune(t, algo=algo)
            tuning[algo]["source"] = "ri_autotune"
            print(f"# tuned {algo}: {tuning[algo]}", file=sys.stderr, flush=True)
            fixed[algo] = {k: tuning[algo][k] for k in ("chunk_target", "warmup_bytes", "runs_per_lane", "converge")}

    timed = {}
    for algo in algos:
        timed[algo] = time_algo(torch, rec, t, algo, args.chunks, args.steps, args.warmup, want, fixed.get(algo))
        print(f"# {algo} done", file=sys.stderr, flush=True)
    rid = timed[prim]

    def summary(m, steps):
        p50 = float(np.percentile(m["per_call"], 50))
        p99 = float(np.percentile(m["per_call"], 99))
        return dict(gbps=n * steps / m["queued"] / 1e9, ms_per_step=m["queued"] / steps * 1e3,
                    sync_gbps=n * steps / m["total"] / 1e9,
                    p50_ms=p50 * 1e3, p99_ms=p99 * 1e3, gbps_p50=n / p50 / 1e9, gbps_p99=n / p99 / 1e9,
                    reach_ms=float(m["reach_ms"].mean()), join_ms=float(m["join_ms"].mean()),
                    long_ms=float(m["kern_ms"].mean()), warm_ms=float(m["warm_ms"].mean()),
                    chunks=m["result"]["chunks"], chunk_size=m["result"]["chunk_size"],
                    bitexact=bool(m["exact"]))

    def rounded(d):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}

    s_rid = summary(rid, args.steps)
    s_dfa = summary(timed["dfa"], args.steps) if "dfa" in timed and prim != "dfa" else None

    plain = None
    if not args.no_plain and "dfa" in timed:
        # the paper-literal reach (every run to the chunk end or its death, no
        # merging), RID vs all-states DFA at the RID chunk count
        c_rid = rid["result"]["chunks"]
        apply_setting(rec, fixed.get("rid"))
        rec.set_option("converge", 0)
        plain = {}
        for algo in ("rid", "dfa"):
            m = time_algo(torch, rec, t, algo, c_rid, 5, 1, want)
            plain[algo] = dict(gbps=round(n * 5 / m["queued"] / 1e9, 2),
                               ms_per_step=round(m["queued"] / 5 * 1e3, 4),
                               reach_ms=round(float(m["reach_ms"].mean()), 4),
                               chunks=m["result"]["chunks"], bitexact=bool(m["exact"]))
        plain["speedup_rid_vs_dfa"] = round(plain["rid"]["gbps"] / plain["dfa"]["gbps"], 4)
        rec.set_option("converge", 1)
        print(f"# plain done", file=sys.stderr, flush=True)

    extras = None
    if not args.no_extras:
        extras = {}
        # the all-states powerset DFA of the position NFA (the second
        # baseline; for the motif union the minimal DFA has one state)
        st = rec.autotune(t, algo="subset")
        m = time_algo(torch, rec, t, "subset", 0, max(3, args.steps // 3), 2, want,
                      {k: st[k] for k in ("chunk_target", "warmup_bytes", "runs_per_lane", "converge")})
        extras["all_states_subset_dfa"] = dict(rounded(summary(m, max(3, args.steps // 3))),
                                               states=info["subset_dfa_states"],
                                               speedup_rid_vs_subset=round(s_rid["gbps"] / (n * max(3, args.steps // 3) / m["queued"] / 1e9), 4))
        print(f"# subset done", file=sys.stderr, flush=True)
        # RID with every start stepping from the first byte of its chunk (no
        # walk of the starts' transformation automaton), at the tuned setting
        if info["prefix_depth"][0]:
            k = max(3, args.steps // 3)
            rec.set_option("prefix", 0)
            m = time_algo(torch, rec, t, "rid", args.chunks, k, 2, want, fixed.get("rid"))
            rec.set_option("prefix", 1)
            extras["rid_without_prefix_walk"] = dict(rounded(summary(m, k)), prefix_depth=info["prefix_depth"][0],
                                                     prefix_states=info["prefix_states"][0])
            print(f"# no-prefix done", file=sys.stderr, flush=True)
        # the NFA device of Sect. 2: the position NFA as chunk automaton,
        # every NFA state speculated, runs as sets of states
        if info["starts"][3] <= 256:
            nt = rec.autotune(t, algo="nfa")
            k = 3
            m = time_algo(torch, rec, t, "nfa", 0, k, 1, want, {"chunk_target": nt["chunk_target"]})
            nfa_gbps = n * k / m["queued"] / 1e9
            extras["nfa_device"] = dict(rounded(summary(m, k)), nfa_states=info["starts"][3],
                                        speedup_rid_vs_nfa=round(s_rid["gbps"] / nfa_gbps, 4))
            print(f"# nfa done", file=sys.stderr, flush=True)
        # the tiny workload at the paper's chunk count (64) and tuned
        from workloads import gen
        trx = gen.c1_regex()
        tx, _ = gen.c1_texts(args.seed)
        tref = oracle.build(trx)
        twant = oracle.serial(tref.dfa, tx)
        trec = ri.Recognizer(trx)
        tt = torch.from_numpy(tx).to("cuda")
        tiny = {}
        for algo in ("rid", "dfa"):
            tiny[algo] = {}
            for label, chunks in (("c64", 64), ("tuned", 0)):
                if chunks == 0:
                    tun = trec.autotune(tt, algo=algo)
                    setting = {k: tun[k] for k in ("chunk_target", "warmup_bytes", "runs_per_lane", "converge")}
                else:
                    setting = None
                m = time_algo(torch, trec, tt, algo, chunks, 20, 3, twant, setting)
                tiny[algo][label] = dict(gbps=round(len(tx) * 20 / m["queued"] / 1e9, 3),
                                         p50_ms=round(float(np.percentile(m["per_call"], 50)) * 1e3, 4),
                                         p99_ms=round(float(np.percentile(m["per_call"], 99)) * 1e3, 4),
                                         chunks=m["result"]["chunks"], bitexact=bool(m["exact"]))
        tiny["speedup_rid_vs_dfa_c64"] = round(tiny["rid"]["c64"]["gbps"] / tiny["dfa"]["c64"]["gbps"], 4)
        extras["tiny_regexp_k3_1MiB"] = tiny
        trec.close()
        del tt
        print(f"# tiny done", file=sys.stderr, flush=True)
        # the class-join fallback at scale: counting a's modulo 9 keeps 9 runs
        # per chunk (more than a hit-matrix row holds), so every call redoes
        # the join as a class join (queued: gated on the hit join's flag)
        frx = b"((b*a){9})*b*"
        fx = gen.random_text(gen.PCG(31), b"ab", 256 << 20)
        fref = oracle.build(frx)
        fwant = oracle.serial(fref.dfa, fx)
        frec = ri.Recognizer(frx)
        ft = torch.from_numpy(fx).to("cuda")
        fb = {}
        for chunks in (131072,):
            m = time_algo(torch, frec, ft, "rid", chunks, 10, 2, fwant, {"warmup_bytes": 16, "converge": 1})
            fb[f"c{chunks}"] = dict(gbps=round(len(fx) * 10 / m["queued"] / 1e9, 2),
                                    ms_per_step=round(m["queued"] / 10 * 1e3, 4),
                                    join_ms=round(float(m["join_ms"].mean()), 4),
                                    sync_p50_ms=round(float(np.percentile(m["per_call"], 50)) * 1e3, 4),
                                    chunks=m["result"]["chunks"], bitexact=bool(m["exact"]))
        extras["class_join_fallback_mod9_256MiB"] = fb
        frec.close()
        del ft
        print(f"# fallback done", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: the long-run kernel of the converging
    # reach.  Algorithmic bytes per launch = the text bytes it must read, i.e.
    # every chunk after its warm-up prefix (the merged runs of one chunk read
    # the same bytes; the run records, 12 B per run, are < 2% and left out).
    L = info["starts"][0 if prim == "rid" else 1]
    cs, c = s_rid["chunk_size"], s_rid["chunks"]
    conv_rid = fixed[prim].get("converge", 1) if prim in fixed else rec.get_option("converge")
    warm = (fixed[prim]["warmup_bytes"] if prim in fixed else rec.get_option("warmup_bytes")) if conv_rid else 0
    long_bytes = sum(max(0, min(cs, n - i * cs) - warm) for i in range(c)) if c < 5_000_000 else n
    achieved = long_bytes / (s_rid["long_ms"] * 1e-3) / 1e9
    trec_t = load_traffic(wname)
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=(round(trec_t["traffic_bytes_per_launch"]) if trec_t else None),
                kernel="long_kernel" if conv_rid else "plain_kernel", algorithmic_bytes=int(long_bytes),
                kernel_ms=round(s_rid["long_ms"], 4),
                reach_phase_gbps=round(n / (s_rid["reach_ms"] * 1e-3) / 1e9, 1),
                whole_path_gbps=round(s_rid["gbps"], 1),
                whole_path_frac=round(s_rid["gbps"] / HBM_PEAK_GBS, 4))

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's serial recognizer (plain C scan), one host core, whole text
        # repeated until about --cpu-seconds have passed
        reps, c0 = 0, time.perf_counter()
        while True:
            oracle.serial(ref.dfa, x, table)
            reps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - c0
        cpu = dict(value=round(n * reps / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                   sample=f"{reps} serial scans of the whole {n}-byte text by the oracle's "
                          f"minimal-DFA scan ({dt:.1f} s)")
        cpu["threaded_csdpa"] = threaded_cpu(oracle, ref, x, table, args.cpu_prefix_mib << 20)

    out = {
        "metric": "GB/s of text recognized, RI-DFA vs all-states DFA speculation (bit-exact); p50/p99",
        "value": round(s_rid["gbps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s_rid["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wname, "n_bytes": n, "seed": args.seed, "algo": prim,
                   "chunks": s_rid["chunks"], "chunk_size": s_rid["chunk_size"],
                   "interface_starts": L, "min_dfa_states": info["min_dfa_states"],
                   "ridfa_states": info["ridfa_states"]},
        "p50_ms": round(s_rid["p50_ms"], 4),
        "p99_ms": round(s_rid["p99_ms"], 4),
        "gbps_p50": round(s_rid["gbps_p50"], 2),
        "gbps_p99": round(s_rid["gbps_p99"], 2),
        "bitexact": all(m["exact"] for m in timed.values()) and (
            plain is None or (plain["rid"]["bitexact"] and plain["dfa"]["bitexact"])) and (
            extras is None or (extras["all_states_subset_dfa"]["bitexact"] and all(
                v["bitexact"] for a in ("rid", "dfa") for v in extras["tiny_regexp_k3_1MiB"][a].values())
                and all(v["bitexact"] for v in extras["class_join_fallback_mod9_256MiB"].values())
                and extras.get("nfa_device", {}).get("bitexact", True)
                and extras.get("rid_without_prefix_walk", {}).get("bitexact", True))),
        "rid": rounded(s_rid) if prim == "rid" else None,
        "all_states_dfa": rounded(s_dfa) if s_dfa else (rounded(s_rid) if prim == "dfa" else None),
        "speedup_rid_vs_dfa": round(s_rid["gbps"] / s_dfa["gbps"], 4) if s_dfa else None,
        "tuning": {k: rounded(v) for k, v in tuning.items()},
        "command": " ".join(["python", "bench.py"] + sys.argv[1:]),
        "plain_reach": plain,
        "extras": extras,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    rec.close()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def threaded_cpu(oracle, ref, x, table, prefix):
    """The paper's CPU scheme (one thread per chunk, serial join) for the
    all-states minimal DFA and for RID on the first `prefix` bytes, with as
    many chunks as usable cores; checked against the oracle's serial scan of
    the same prefix."""
    from oracle import baseline
    cores = len(os.sched_getaffinity(0))
    xp = np.ascontiguousarray(x[:prefix])
    want = oracle.serial(ref.dfa, xp, table)
    tq = oracle.dense_table(ref.Bq.n, ref.Bq.delta)
    d = baseline.csdpa_dfa(ref.dfa, xp, cores, table)
    r = baseline.csdpa_rid(ref.Bq, xp, cores, tq)
    end, _ = oracle.run(tq, ref.Bq.initial[0], xp, 0, len(xp))
    exact = (d["accept"], d["final_state"]) == want and r["accept"] == want[0] and (
        r["S"] == (ref.Bq.content[end] if end >= 0 else frozenset()))
    return dict(cpu_model=cpu_model(), cores=cores, threads=cores, chunks=cores, bytes=int(len(xp)),
                dfa_gbps=round(len(xp) / d["seconds"] / 1e9, 4), rid_gbps=round(len(xp) / r["seconds"] / 1e9, 4),
                speedup_rid_vs_dfa=round(d["seconds"] / r["seconds"], 4),
                dfa_transitions=d["transitions"], rid_transitions=r["transitions"],
                transitions_dfa_over_rid=round(d["transitions"] / max(1, r["transitions"]), 4),
                bitexact=bool(exact),
                note="reported baseline: the paper's scheme (Sect. 4), one thread per chunk, on the host cores")


if __name__ == "__main__":
    main()

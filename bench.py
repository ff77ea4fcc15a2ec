#!/usr/bin/env python3
"""Benchmark: input GB/s scanned, bit-exact, on one MI355X.

Workload (one step = one launch over the whole batch): one seeded ~200-node
expression over bytes (literals a-z, 8 classes, concat, alternation, star,
plus, optional) searched as .*(e).*, against 1,000,000 strings of exactly
256 bytes of uniform a-z with 10% planted members of the language.  Inputs
are resident in HBM before timing starts; the timed steps rotate over
several copies of the input so the 256 MB Infinity Cache cannot hold them.

Prints one JSON line with the metric, a roofline report for the matching
kernel and the CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def kernel_id(p, launch_desc: str) -> str:
    """Identity of the timed kernel: its generated source and launch variant."""
    import hashlib

    src = p.jit_source() if p.jit_stats()["ready"] else "table-form"
    # the default staging mode and the form it runs (other modes do not run here)
    st = p.jit_staging() if p.jit_stats()["ready"] else [0] * 7
    form = f"mode={st[0]}/{st[st[0]]}"
    return hashlib.sha256((src + "|" + launch_desc + "|" + form).encode()).hexdigest()[:16]


def recorded_traffic(kid: str):
    """HBM bytes per launch measured with rocprofv3 PMC counters for this exact kernel, or None."""
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".txt"):
            continue
        fields = {}
        for line in open(os.path.join(PROFILES, name)):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("kernel_id") == kid and "traffic_bytes_per_launch" in fields:
            return int(fields["traffic_bytes_per_launch"])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--strings", type=int, default=1_000_000)
    ap.add_argument("--length", type=int, default=256)
    ap.add_argument("--copies", type=int, default=4, help="input copies rotated across steps")
    ap.add_argument("--variant", type=int, default=0,
                    help="kernel variant: 0 = library default (sliced circuit when compiled), 1 lane, 2 wave, 3 sliced")
    ap.add_argument("--layout", choices=["fixed", "offsets"], default="fixed",
                    help="fixed: strings of equal length back to back (rx_match_fixed); offsets: rx_match")
    ap.add_argument("--no-jit", action="store_true", help="do not compile the bit-sliced circuit")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--serving", type=int, default=2000, help="requests per serving load point (0 = skip)")
    ap.add_argument("--copy-only", action="store_true", help="only run the stream-copy probe (counter calibration)")
    ap.add_argument("--serving-only", action="store_true", help="only run the serving comparison")
    ap.add_argument("--workload", choices=["single", "small", "multi", "pathological", "long"], default="single",
                    help="single is the benchmark; the others measure the remaining configurations")
    ap.add_argument("--multi-lines", type=int, default=4_000_000)
    ap.add_argument("--no-table", action="store_true", help="multi: time only the plane form (profiling runs)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 28)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(strings shard trivially across GPUs, but no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1108_3126_amd import rx
    from paper_1108_3126_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_only:
        print(json.dumps(copy_probe(torch, rx, dev, args.copy_bytes, reps=max(args.steps, 1))), flush=True)
        return
    if args.serving_only:
        print(json.dumps(run_serving(args, torch)), flush=True)
        return
    if args.workload != "single":
        fn = {"small": run_small, "multi": run_multi, "pathological": run_pathological,
              "long": run_long}[args.workload]
        print(json.dumps(fn(args, torch, dev)), flush=True)
        return
    t0 = time.time()
    prog = W.single_program(1)
    strings, planted = W.single_strings(prog, seed=1, n=args.strings, length=args.length)
    log(f"workload generated in {time.time() - t0:.1f}s: {prog.n_nodes} AST nodes, {strings.n} strings")

    p = rx.compile(prog.ast, prog.root, prog.classes, search=True).upload(dev)
    info = p.info
    log(f"program: m={info.m} L={info.n_leaves} words={info.words} table_bytes={info.table_bytes}")
    if not args.no_jit:
        j0 = time.time()
        p.jit()
        log(f"bit-sliced circuit compiled in {time.time() - j0:.2f}s: {p.jit_stats()}, staging {p.jit_staging()}")
    offs = torch.from_numpy(strings.offsets).to(dev)
    copies = [torch.from_numpy(strings.data).to(dev)]
    for _ in range(1, max(1, args.copies)):
        copies.append(copies[0].clone())
    out = torch.empty(strings.n, dtype=torch.uint8, device=dev)
    launch = None
    if args.variant or args.block or args.grid or args.unroll:
        launch = (args.variant, args.block, args.grid, args.unroll)

    def step(i):
        if args.layout == "fixed":
            rx.match_fixed(p, copies[i % len(copies)], args.length, strings.n, out=out, launch=launch)
        else:
            rx.match(p, copies[i % len(copies)], offs, out=out, launch=launch)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    got_warm = out.cpu().numpy()
    planted_ok = bool(got_warm[planted].all()) if len(planted) else True

    # The timed region: K launches back to back on the launch stream, one HIP
    # event before and one after (an event between launches costs several us
    # of wall time per step).  The average launch duration is the region's
    # event time over K, gaps between launches included.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        step(args.warmup + i)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    got_last = out.cpu().numpy()   # the results of the last timed step
    avg_kernel_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    input_bytes = int(strings.offsets[-1])
    value = input_bytes / (ms_per_step * 1e-3) / 1e9
    algo_bytes = input_bytes + strings.n + (8 * (strings.n + 1) if args.layout == "offsets" else 0)
    achieved = algo_bytes / (avg_kernel_ms * 1e-3) / 1e9
    # spread of single launches (after the timed region; not used for the figures)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(10)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(10)]
    for i in range(10):
        starts[i].record()
        step(i)
        ends[i].record()
    torch.cuda.synchronize()
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    log(f"timed region: {avg_kernel_ms:.4f} ms per launch (events), wall {ms_per_step:.4f} ms/step; "
        f"single launches: median {np.median(kern_ms):.4f} min {min(kern_ms):.4f}")

    # Correctness of the timed configuration: the oracle over every string of the batch, compared
    # with the last timed step's results.  The same run, timed, is the CPU baseline.
    threads = oracle.default_threads()
    c0 = time.perf_counter()
    want = oracle.match(prog.ast, prog.root, prog.classes, True, strings.data, strings.offsets, threads=threads)
    cdt = time.perf_counter() - c0
    mismatches = int(np.count_nonzero(got_last != want)) + int(np.count_nonzero(got_warm != want))
    bit_exact = mismatches == 0
    log(f"check: all {strings.n} strings against the oracle: mismatches {mismatches}, planted all matched "
        f"{planted_ok}, accepted {int(got_last.sum())}/{strings.n}")
    cpu = {"value": round(input_bytes / cdt / 1e9, 6), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"all {strings.n} strings of the batch ({input_bytes} bytes), {cdt:.1f} s"}
    log(f"cpu oracle: {cpu}")

    copy = copy_probe(torch, rx, dev, 1 << 28, reps=10)
    log(f"copy probe: {copy}")
    serving = run_serving(args, torch) if args.serving > 0 else None
    if serving:
        log(f"serving: {serving}")

    kid = kernel_id(p, f"layout={args.layout};variant={args.variant};unroll={args.unroll};block={args.block};"
                       f"grid={args.grid}")
    traffic = recorded_traffic(kid)
    log(f"kernel id {kid}; recorded traffic per launch: {traffic}")
    variant_name = {0: "auto", 1: "lane", 2: "wave", 3: "sliced"}[args.variant]
    if args.variant == 0:
        # offsets: a layout check on the device sends equal-length consecutive strings to the sliced kernel
        variant_name = ("sliced" if args.layout == "fixed" else "layout check + sliced") if not args.no_jit else "lane"
    rec = {
        "metric": "input GB/s scanned (bit-exact)",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "bit_exact": bit_exact and planted_ok,
        "checked_strings": int(strings.n),
        "config": {
            "workload": "single program: ~200-node regex searched as .*(e).* over 1M x 256 B lowercase strings, "
                        "10% planted",
            "strings": strings.n,
            "length": args.length,
            "ast_nodes": int(prog.n_nodes),
            "leaves": int(info.n_leaves),
            "kernel": variant_name,
            "input_copies": len(copies),
            "layout": args.layout,
            "kernel_id": kid,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic,
        },
        "cpu_baseline": cpu,
        "copy_probe": copy,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


def run_small(args, torch, dev):
    """The small configuration: one anchored expression over {a,b}, 1,000 strings; launch-bound."""
    import oracle
    from paper_1108_3126_amd import rx
    from paper_1108_3126_amd import workloads as W

    prog, s = W.small_program(0), W.small_strings(0)
    p = rx.compile(prog.ast, prog.root, prog.classes, False).upload(dev)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    out = torch.empty(s.n, dtype=torch.uint8, device=dev)
    for _ in range(20):
        rx.match(p, d, o, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(200)]
    for a, e in ev:
        a.record()
        rx.match(p, d, o, out=out)
        e.record()
    torch.cuda.synchronize()
    us = sorted(a.elapsed_time(e) * 1e3 for a, e in ev)
    want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets)
    ok = bool(np.array_equal(out.cpu().numpy(), want))
    # the paper's node-per-thread machine on the same batch
    nout = torch.empty(s.n, dtype=torch.uint8, device=dev)
    for _ in range(20):
        rx.match_nodes(p, d, o, out=nout)
    torch.cuda.synchronize()
    for a, e in ev:
        a.record()
        rx.match_nodes(p, d, o, out=nout)
        e.record()
    torch.cuda.synchronize()
    nus = sorted(a.elapsed_time(e) * 1e3 for a, e in ev)
    nok = bool(np.array_equal(nout.cpu().numpy(), want))
    return {"metric": "us per call", "workload": "small: 1 expression over {a,b}, 1,000 strings of length 0..32",
            "median_us": round(us[len(us) // 2], 2), "p99_us": round(us[int(len(us) * 0.99)], 2), "bit_exact": ok,
            "node_machine": {"median_us": round(nus[len(nus) // 2], 2), "p99_us": round(nus[int(len(nus) * 0.99)], 2),
                             "bit_exact": nok}}


def run_multi(args, torch, dev):
    """16 programs against 4M log-normal Zipf lines in one batched launch."""
    import oracle
    from paper_1108_3126_amd import autotune, rx
    from paper_1108_3126_amd import workloads as W

    t0 = time.time()
    progs = W.multi_programs(seed=2)
    lines = W.multi_lines(seed=2, n=args.multi_lines)
    log(f"multi: {len(progs)} programs, {lines.n} lines, {lines.offsets[-1] / 1e6:.0f} MB in {time.time() - t0:.1f}s")
    ps = [rx.compile(p.ast, p.root, p.classes, True).upload(dev) for p in progs]
    d, o = torch.from_numpy(lines.data).to(dev), torch.from_numpy(lines.offsets).to(dev)
    if args.no_table:
        cfg, tinfo = None, None
    else:
        cfg, tinfo = autotune.tune_multi(ps, d, o, budget_runs=40, use_cache=False)
        log(f"multi tuned: {tinfo}")

    def timed(config, reps=3, dd=d, oo=o):
        cfg_ = config if config is not None else rx.multi_config()
        if cfg_.form == rx.FORM_PLANES:
            cfg_ = rx.multi_config(form=rx.FORM_PLANES, max_bytes=dd.numel(), graph=cfg_.graph)
        need = rx.lib().rx_match_multi_workspace(oo.numel() - 1, len(ps), rx.ctypes.byref(cfg_))
        work = torch.empty(int(need) + 256, dtype=torch.uint8, device=dev)
        res = rx.match_multi(ps, dd, oo, config=cfg_, work=work)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            rx.match_multi(ps, dd, oo, out=res, config=cfg_, work=work)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, res.cpu().numpy()

    ms_table, got_table = timed(cfg) if cfg is not None else (None, None)
    # plane form: each program's bit-sliced circuit over length-sorted slabs
    j0 = time.time()
    rx.prepare_multi(ps)
    jit_s = time.time() - j0
    pcfg = rx.multi_config(form=rx.FORM_PLANES, max_bytes=int(lines.offsets[-1]))
    ms_planes, got = timed(pcfg)
    log(f"multi: table form {ms_table} ms, plane form {ms_planes:.3f} ms (circuits compiled in {jit_s:.1f} s)")
    ok = got_table is None or bool(np.array_equal(got, got_table))
    # the same launches replayed from a captured graph, on the whole batch and on a small one (20,000
    # lines), where the launch path is a larger share of a call
    gcfg = rx.multi_config(form=rx.FORM_PLANES, max_bytes=int(lines.offsets[-1]), graph=True)
    ms_graph, got_graph = timed(gcfg)
    graph_ok = bool(np.array_equal(got_graph, got))
    small_n = min(20000, lines.n)
    ds, os_ = d[:int(lines.offsets[small_n])], o[:small_n + 1]
    small = {"lines": small_n}
    for name, c in (("planes", rx.multi_config(form=rx.FORM_PLANES)),
                    ("planes_graph", rx.multi_config(form=rx.FORM_PLANES, graph=True)),
                    ("table", rx.multi_config()), ("table_graph", rx.multi_config(graph=True))):
        ms_s, got_s = timed(c, reps=50, dd=ds, oo=os_)
        small[name + "_ms"] = round(ms_s, 4)
        graph_ok = graph_ok and bool(np.array_equal(got_s, got[:, :small_n]))
    log(f"multi: graph replay {ms_graph:.3f} ms; 20,000 lines: {small}; graph results equal: {graph_ok}")
    rng = np.random.default_rng(7)
    for k, pr in enumerate(progs):
        idx = np.unique(rng.choice(lines.n, size=150, replace=False)).astype(np.int64)
        want = oracle.match(pr.ast, pr.root, pr.classes, True, lines.data, lines.offsets, index=idx)
        ok = ok and bool(np.array_equal(got[k][idx], want))
    nbytes = int(lines.offsets[-1])
    ms = ms_planes
    return {"metric": "unique input GB/s, all programs per line", "workload": "multi: 16 programs x 4M lines",
            "form": "planes", "ms": round(ms, 3), "input_GBs": round(nbytes / (ms * 1e-3) / 1e9, 2),
            "byte_program_steps_per_s": round(nbytes * len(progs) / (ms * 1e-3), 0),
            "graph_ms": round(ms_graph, 3), "small_batch": small, "graph_equal_direct": graph_ok,
            "table_form_ms": round(ms_table, 3) if ms_table else None,
            "speedup_vs_table": round(ms_table / ms, 2) if ms_table else None,
            "accepted_per_program": got.sum(axis=1).tolist(), "table_config": tinfo,
            "bit_exact_sample": ok, "planes_equal_table": None if got_table is None else bool(np.array_equal(got, got_table))}


def run_pathological(args, torch, dev):
    """4,096-node nested-star programs on a^n strings: time per n and linearity ratios."""
    import oracle
    from paper_1108_3126_amd import rx
    from paper_1108_3126_amd import workloads as W

    res = {"metric": "ms per launch (256 strings of length n)", "workload": "pathological", "families": {}}
    for family, k in (("nested", 819), ("altstar", 585)):
        prog = W.pathological_program(family, k)
        p = rx.compile(prog.ast, prog.root).upload(dev)
        fam = {}
        for n_len in (1000, 10000, 100000):
            s = W.pathological_strings(family, n_len, count=256)
            d = torch.from_numpy(s.data).to(dev)
            out = rx.match_fixed(p, d, n_len, s.n)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rx.match_fixed(p, d, n_len, s.n, out=out)
            e1.record()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            closed = bool(got[:128].sum() == 0 and got[128:].all())  # a* t
            entry = {"ms": round(e0.elapsed_time(e1), 3), "closed_form_ok": closed}
            if n_len == 1000:
                idx = np.array([0, 1, 127, 128, 200, 255], np.int64)
                want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets, index=idx)
                entry["oracle_ok"] = bool(np.array_equal(got[idx], want))
            fam[str(n_len)] = entry
            log(f"pathological {family} n={n_len}: {entry}")
        fam["ratio_1e4_1e3"] = round(fam["10000"]["ms"] / fam["1000"]["ms"], 2)
        fam["ratio_1e5_1e4"] = round(fam["100000"]["ms"] / fam["10000"]["ms"], 2)
        # program size: k repetitions at n = 10^4 (time should grow with the set width)
        scale = {}
        s = W.pathological_strings(family, 10000, count=256)
        d = torch.from_numpy(s.data).to(dev)
        for kk in (1, 8, 64, k):
            pk = W.pathological_program(family, kk)
            pp = rx.compile(pk.ast, pk.root).upload(dev)
            out = rx.match_fixed(pp, d, 10000, s.n)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rx.match_fixed(pp, d, 10000, s.n, out=out)
            e1.record()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            scale[str(kk)] = {"nodes": int(len(pk.ast)), "words": int(pp.info.words), "ms": round(e0.elapsed_time(e1), 3),
                              "closed_form_ok": bool(got[:128].sum() == 0 and got[128:].all())}
        fam["k_scaling_n1e4"] = scale
        log(f"pathological {family} k scaling at n=1e4: {scale}")
        # the paper's node-per-thread machine (one workgroup per string, one thread per node)
        nm = {}
        for n_len in (1000, 10000, 100000):
            s = W.pathological_strings(family, n_len, count=256)
            d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
            out = rx.match_nodes(p, d, o)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rx.match_nodes(p, d, o, out=out)
            e1.record()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            nm[str(n_len)] = {"ms": round(e0.elapsed_time(e1), 3),
                              "closed_form_ok": bool(got[:128].sum() == 0 and got[128:].all())}
            log(f"pathological {family} node machine n={n_len}: {nm[str(n_len)]}")
            if nm[str(n_len)]["ms"] > 2000:
                break
        if "100000" in nm:
            nm["ratio_1e5_1e4"] = round(nm["100000"]["ms"] / nm["10000"]["ms"], 2)
        nm["ratio_1e4_1e3"] = round(nm["10000"]["ms"] / nm["1000"]["ms"], 2)
        fam["node_machine"] = nm
        # the compiled circuit (here one or two state words: every 'a' leaf holds the same word) run
        # chunk-parallel: one wavefront per string, 2,048 chunks, each a map of the circuit's states
        pj = rx.compile(prog.ast, prog.root).upload(dev).jit()
        ck = {"state_words": pj.jit_stats()["state_words"]}
        for n_len in (1000, 10000, 100000):
            s = W.pathological_strings(family, n_len, count=256)
            d = torch.from_numpy(s.data).to(dev)
            launch = (rx.VARIANT_CHUNKS, 0, 0, 0)
            out = rx.match_fixed(pj, d, n_len, s.n, launch=launch)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                rx.match_fixed(pj, d, n_len, s.n, out=out, launch=launch)
            e1.record()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            entry = {"ms": round(e0.elapsed_time(e1) / 5, 4),
                     "closed_form_ok": bool(got[:128].sum() == 0 and got[128:].all())}
            if n_len == 1000:
                idx = np.array([0, 1, 127, 128, 200, 255], np.int64)
                want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets, index=idx)
                entry["oracle_ok"] = bool(np.array_equal(got[idx], want))
            ck[str(n_len)] = entry
        log(f"pathological {family} chunk-parallel circuit: {ck}")
        fam["chunk_parallel_circuit"] = ck
        res["families"][family] = fam
    return res


def run_long(args, torch, dev):
    """One long string: the lockstep run over the whole string (one lane or one wavefront) against the
    chunk-parallel run (rx_match_long), for the ~200-node searched expression and the 4,096-node families."""
    from paper_1108_3126_amd import rx
    from paper_1108_3126_amd import workloads as W

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, int(r.cpu().numpy()[0])

    res = {"metric": "ms per string", "workload": "long: one string", "cases": []}
    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    # text with no match: a 256-byte piece that the expression rejects, also when doubled, repeated
    pieces, _ = W.single_strings(prog, seed=30, n=4096, length=256, plant_frac=0.0)
    pd = torch.from_numpy(pieces.data).to(dev)
    bits = rx.match_fixed(p, pd, 256, pieces.n).cpu().numpy()
    piece = None
    for i in np.nonzero(bits == 0)[0][:64]:
        w = pieces.data[i * 256:(i + 1) * 256]
        two = torch.from_numpy(np.concatenate([w, w])).to(dev)
        if int(rx.match_fixed(p, two, 512, 1).cpu().numpy()[0]) == 0:
            piece = w
            break
    member, _ = W.single_strings(prog, seed=31, n=1, length=256, plant_frac=1.0)
    pj = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    for mb in (4, 64):
        n_bytes = mb << 20
        data = np.tile(piece, n_bytes // 256)
        base_bit = int(rx.match_long(p, torch.from_numpy(data).to(dev), data.size).cpu().numpy()[0])
        data[-256:] = member.data   # a member in the last 256 bytes: every chunk matters
        d = torch.from_numpy(data).to(dev)
        o = torch.tensor([0, data.size], dtype=torch.int64, device=dev)
        entry = {"case": f"~200-node expression searched, one {mb} MiB string, one member in its last 256 bytes",
                 "bit_without_member": base_bit}
        if mb <= 4:
            entry["serial_ms"], entry["serial_bit"] = timed(lambda: rx.match(p, d, o), reps=1)
            entry["GBs_serial"] = round(data.size / (entry["serial_ms"] * 1e-3) / 1e9, 3)
        entry["chunked_ms"], entry["chunked_bit"] = timed(lambda: rx.match_long(p, d, data.size))
        entry["first_chunked_ms"], entry["first_chunked"] = timed(lambda: rx.match_first_long(p, d, data.size))
        entry["chunks"] = min(int(round((data.size / 2) ** 0.5)), 4096)
        entry["GBs_chunked"] = round(data.size / (entry["chunked_ms"] * 1e-3) / 1e9, 2)
        # the compiled circuit (17 words) as chunks: each chunk an affine map of the state words
        entry["circuit_chunks_ms"], entry["circuit_chunks_bit"] = timed(lambda: rx.match_long(pj, d, data.size))
        entry["GBs_circuit_chunks"] = round(data.size / (entry["circuit_chunks_ms"] * 1e-3) / 1e9, 2)
        log(f"long: {entry}")
        res["cases"].append(entry)
    for family, k in (("nested", 819), ("altstar", 585)):
        pk = W.pathological_program(family, k)
        pp = rx.compile(pk.ast, pk.root).upload(dev)
        n_len = 100_000
        s = W.pathological_strings(family, n_len, count=2)
        acc = torch.from_numpy(s.data[n_len:].copy()).to(dev)
        entry = {"case": f"{family} 4,096 nodes, one string a^(n-1)t, n = 1e5"}
        entry["serial_ms"], entry["serial_bit"] = timed(lambda: rx.match_fixed(pp, acc, n_len, 1), reps=1)
        for ch in (16, 64):
            entry[f"chunked_{ch}_ms"], entry[f"chunked_{ch}_bit"] = timed(lambda: rx.match_long(pp, acc, n_len, ch),
                                                                       reps=1)
        pc = rx.compile(pk.ast, pk.root).upload(dev).jit()
        entry["circuit_chunks_ms"], entry["circuit_chunks_bit"] = timed(lambda: rx.match_long(pc, acc, n_len))
        log(f"long: {entry}")
        res["cases"].append(entry)
    return res


def copy_probe(torch, rx, dev, nbytes, reps=10):
    """Practical streaming ceiling: a coalesced device copy (read + write bytes per second)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(2)]
    a.fill_(1)
    rx.stream_copy(b[0], a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        rx.stream_copy(b[i & 1], a if i % 2 == 0 else b[0])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes": nbytes, "ms": round(ms, 4), "read_write_GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def run_serving(args, torch):
    """Batched server against the per-request plain path on the same requests and Poisson rate."""
    import threading
    import queue

    import oracle
    from paper_1108_3126_amd import server
    from paper_1108_3126_amd import workloads as W

    R = args.serving
    t0 = time.time()
    reqs = [W.serving_request(3, i) for i in range(R)]
    total_bytes = sum(int(s.offsets[-1]) for _, s in reqs)
    log(f"serving: {R} requests, {total_bytes / 1e6:.1f} MB, generated in {time.time() - t0:.1f}s")
    # warm up both paths (first-touch costs) on a few requests
    for p, s in reqs[:3]:
        server.plain_match(p, s.data, s.offsets)
    # capacity of the plain path: serial, back to back
    c0 = time.perf_counter()
    plain_out = [server.plain_match(p, s.data, s.offsets) for p, s in reqs]
    plain_cap = R / (time.perf_counter() - c0)
    # the plain path with its stream and device buffers made once (no per-request allocation)
    pre = server.PlainContext(max(int(s.offsets[-1] - s.offsets[0]) for _, s in reqs), max(s.n for _, s in reqs))
    for p, s in reqs[:3]:
        pre.match(p, s.data, s.offsets)
    c0 = time.perf_counter()
    pre_out = [pre.match(p, s.data, s.offsets) for p, s in reqs]
    pre_cap = R / (time.perf_counter() - c0)
    srv = server.Server(use_graph=True)
    for p, s in reqs[:3]:
        srv.wait(srv.submit(p, s.data, s.offsets))
    srv.reset_stats()
    c0 = time.perf_counter()
    ids = [srv.submit(p, s.data, s.offsets) for p, s in reqs]
    srv_out = [srv.wait(r) for r in ids]
    srv_cap = R / (time.perf_counter() - c0)
    st_cap = srv.stats()
    exact = all(np.array_equal(a, b) and np.array_equal(a, c) for a, b, c in zip(plain_out, srv_out, pre_out))
    # oracle on a sample of every 25th request, 20 strings each
    for k in range(0, R, 25):
        p, s = reqs[k]
        if s.n == 0:
            continue
        idx = np.unique(np.linspace(0, s.n - 1, min(20, s.n)).astype(np.int64))
        want = oracle.match(p.ast, p.root, p.classes, p.search, s.data, s.offsets, index=idx)
        exact = exact and bool(np.array_equal(srv_out[k][idx], want))

    def run_plain_at_rate(rate, fn):
        arrivals = W.poisson_arrivals(3, R, rate)
        q, lat = queue.Queue(), []

        def worker():
            while True:
                item = q.get()
                if item is None:
                    return
                t_arr, (p, s) = item
                fn(p, s.data, s.offsets)
                lat.append(time.perf_counter() - t_arr)

        th = threading.Thread(target=worker)
        th.start()
        start = time.perf_counter()
        for t, r in zip(arrivals, reqs):
            d = start + t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            q.put((time.perf_counter(), r))
        q.put(None)
        th.join()
        lat = np.array(lat) * 1e3
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3)}

    def run_server_at_rate(rate):
        arrivals = W.poisson_arrivals(3, R, rate)
        srv.reset_stats()
        ids = queue.Queue()

        def waiter():
            while True:
                r = ids.get()
                if r is None:
                    return
                srv.wait(r)

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        for t, (p, s) in zip(arrivals, reqs):
            d = start + t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ids.put(srv.submit(p, s.data, s.offsets))
        ids.put(None)
        th.join()
        st = srv.stats()
        return {"p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
                "steps": int(st["steps"])}

    # Poisson load points: half and 90% of each path's capacity.  The plain path
    # cannot sustain the server's rates (its queue would grow without bound),
    # so it is measured at its own two points only.
    points = []
    plain_fns = {"plain": server.plain_match, "plain_prealloc": pre.match}
    for who, cap in (("plain", plain_cap), ("plain_prealloc", pre_cap), ("batched", srv_cap)):
        for frac in (0.5, 0.9):
            rate = frac * cap
            pt = {"load": f"{frac} x {who} capacity", "rate_req_per_s": round(rate, 1),
                  "batched": run_server_at_rate(rate)}
            if who in plain_fns:
                pt[who] = run_plain_at_rate(rate, plain_fns[who])
            points.append(pt)
            log(f"serving point: {pt}")
    srv.close()
    pre.close()
    at = points[1]   # 0.9 x plain capacity: both paths at the same rate
    at_pre = points[3]   # 0.9 x the preallocated plain path's capacity
    return {
        "requests": R,
        "mb": round(total_bytes / 1e6, 1),
        "plain_req_per_s": round(plain_cap, 1),
        "plain_prealloc_req_per_s": round(pre_cap, 1),
        "batched_req_per_s": round(srv_cap, 1),
        "throughput_ratio": round(srv_cap / plain_cap, 2),
        "throughput_ratio_vs_prealloc": round(srv_cap / pre_cap, 2),
        "batched_GBs": round(total_bytes / (R / srv_cap) / 1e9, 3),
        "rate_req_per_s": at["rate_req_per_s"],
        "plain_p50_ms": at["plain"]["p50_ms"],
        "plain_p99_ms": at["plain"]["p99_ms"],
        "batched_p50_ms": at["batched"]["p50_ms"],
        "batched_p99_ms": at["batched"]["p99_ms"],
        "prealloc_rate_req_per_s": at_pre["rate_req_per_s"],
        "plain_prealloc_p50_ms": at_pre["plain_prealloc"]["p50_ms"],
        "plain_prealloc_p99_ms": at_pre["plain_prealloc"]["p99_ms"],
        "batched_at_prealloc_rate_p50_ms": at_pre["batched"]["p50_ms"],
        "batched_at_prealloc_rate_p99_ms": at_pre["batched"]["p99_ms"],
        "points": points,
        "steps_at_capacity": int(st_cap["steps"]),
        "capacity_pack_ms": round(st_cap["pack_ms"], 2),
        "capacity_device_ms": round(st_cap["device_ms"], 2),
        "graph_steps": int(st_cap["graph_steps"]),
        "bit_exact": bool(exact),
    }


if __name__ == "__main__":
    main()

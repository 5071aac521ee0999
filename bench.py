#!/usr/bin/env python3
"""Benchmark of the guest-memory translate-and-copy path on one MI355X.

Metric: GB/s copied + Mreq/s translated; p50/p99 latency, batched vs
per-request.  Default workload: one guest with 4 GiB of guest-physical
memory, 70/30 4 KiB/2 MiB pages, 16 memslots, 5% not-present leaves,
1e6 requests with log-uniform lengths 64 B - 64 KiB, 50/50 direction.

A step is one batched submission of every request (all epochs): translate
each page, set A/D bits, copy, build the ordered fault list.  Inputs are
resident in HBM before timing; between steps (untimed) the page-table frames
are restored (A/D bits cleared again) and the caches flushed by writing
1 GiB.  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB/s copied + Mreq/s translated; p50/p99 latency, batched vs per-request"
HBM_PEAK_GBS = 8000.0
ROOF_STEPS = 3  # profiled steps the roofline is measured over
WORKLOADS = {
    "C2": "one guest, 4 GiB guest memory, 4-level paging, 70/30 4KiB/2MiB pages, 16 memslots, "
          "5% not-present, 1e6 requests log-uniform 64B-64KiB, 50/50 direction",
    "C1": "one guest, 64 MiB, 8192 4KiB pages, 10% not-present, 4 memslots, 256 requests uniform 8-4096B",
    "C3": "16 VMs x 4 processes, 2 GiB each, 80/20 4KiB/2MiB, 4e6 requests log-uniform 16B-4MiB",
    "C5": "64 VMs x 2 GiB, 5-level paging, 60/35/5 4KiB/2MiB/1GiB, 3% not-present, 1e7 requests 16B-1MiB",
    "C2-PAE": "C2 under 32-bit PAE paging (4-entry root table, 32-bit addresses): one guest, 4 GiB, "
              "70/30 4KiB/2MiB, 16 memslots, 5% not-present, 1e6 requests log-uniform 64B-64KiB",
    "C2-EPT": "C2 with its guest-physical space behind a 4-level EPT (a second software walk instead of "
              "memslots; EPT leaves 2 MiB where aligned, else 4 KiB): one guest, 4 GiB, 70/30 4KiB/2MiB, "
              "5% not-present, 1e6 requests log-uniform 64B-64KiB",
}


def workload_spec(name):
    from workload import gen
    if name == "C2-PAE":
        return gen.spec("C2", levels=3, seed=1006)
    if name == "C2-EPT":
        return gen.spec("C2", ept=True, seed=1007)
    return gen.spec(name)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(a, q)) if len(a) else None


def restore_tables(ctx, wl):
    """Write every page-table frame back (clears the A/D bits a step set)."""
    from workload import gen
    for v in wl.vms:
        hpa = gen.gpa_to_arena(v.slots, v.pt_gfn << np.uint64(12))
        order = np.argsort(hpa)
        hs = hpa[order]
        data = v.pt_data[order]
        # merge runs of adjacent frames into one write
        i = 0
        while i < len(hs):
            j = i + 1
            while j < len(hs) and hs[j] == hs[j - 1] + 4096:
                j += 1
            blk = np.ascontiguousarray(data[i:j]).view(np.uint8).reshape(-1)
            ctx.vm_write(v.vm, int(hs[i]), blk, blk.size)
            i = j


def kernel_hash():
    """Hash of the kernel source (kernels.hip, dv_internal.h) with comments and
    blank lines removed: it changes when the compiled kernels can change."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "dv_internal.h"):
        with open(os.path.join(ROOT, "paper_1304_3771_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per copy-kernel launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"copy_traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads for the oracle's parallel leg: the cores this process may run
    on, at most 16 (one GPU's share of its host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(wl, seconds, name, max_vms=8):
    """Time the oracle on the host cores, restricted to the first `max_vms`
    VMs (the oracle keeps every arena it touches in host memory): one thread
    on request prefixes in index order, then N threads (each epoch's requests
    split over them, epochs in order) on whole passes over the requests,
    each leg until `seconds` of oracle time have passed."""
    from oracle import Oracle
    nvm = min(len(wl.vms), max_vms)
    log(f"cpu baseline: building host state for {nvm} of {len(wl.vms)} VMs")

    def fresh():
        arenas = [wl.arena_image(v) for v in range(nvm)]
        arenas += [np.zeros(4096, np.uint8) for _ in range(nvm, len(wl.vms))]
        return Oracle(arenas, [v.slots for v in wl.vms], [(p.vm, p.cr3, p.levels) for p in wl.procs],
                      wl.pool_image(), ept=[v.ept_root if v.vm < nvm else None for v in wl.vms])

    vm_of = np.array([p.vm for p in wl.procs])
    idx = np.nonzero(vm_of[wl.requests["asid"]] < nvm)[0]
    reqs = wl.requests[idx]
    ends = np.unique(np.searchsorted(idx, wl.epoch_end.astype(np.int64), side="left").astype(np.uint64))
    what = f"{len(reqs)} requests of VMs 0-{nvm - 1}" if nvm < len(wl.vms) else f"{len(reqs)} requests"
    # one thread
    o = fresh()
    tot_t, tot_b, done, passes = 0.0, 0, 0, 0
    chunk = 4096
    i = 0
    while tot_t < seconds and passes < 20:
        if i >= len(reqs):
            i = 0
            passes += 1
            if passes >= 20:
                break
        part = reqs[i:i + chunk]
        t0 = time.perf_counter()
        r, _ = o.batch(part)
        dt = time.perf_counter() - t0
        tot_t += dt
        tot_b += int(r["bytes_done"].sum())
        done += len(part)
        i += len(part)
        if dt < 0.2:
            chunk *= 2
    del o
    one = {"value": round(tot_b / tot_t / 1e9, 3), "unit": "GB/s", "cores": 1,
           "mreq_s": round(done / tot_t / 1e6, 4),
           "sample": f"{done} requests: {name}'s {what} in index order, {done / len(reqs):.2f} passes, "
                     f"{tot_t:.1f} s"}
    # N threads
    nt = host_threads()
    o = fresh()
    tot_t, tot_b, npass = 0.0, 0, 0
    while tot_t < seconds and npass < 20:
        t0 = time.perf_counter()
        r, _ = o.batch_mt(reqs, ends, threads=nt)
        tot_t += time.perf_counter() - t0
        tot_b += int(r["bytes_done"].sum())
        npass += 1
    del o
    model = cpu_model()
    return {"value": round(tot_b / tot_t / 1e9, 3), "unit": "GB/s", "cores": nt, "kind": "oracle",
            "mreq_s": round(npass * len(reqs) / tot_t / 1e6, 4), "cpu_model": model,
            "host_cores_visible": os.cpu_count(),
            "sample": f"{npass} passes over {name}'s {what}, each epoch's requests split over {nt} threads, "
                      f"epochs in order, {tot_t:.1f} s on {model}",
            "single_thread": one}


def translate_rate(ctx, wl, n, reps=3):
    """devirt_translate on n addresses of the first process (90% in its mapped
    leaves, 10% anywhere in the user range), READ, no A/D: addresses per
    microsecond (M/s), the median of reps timed calls after one untimed."""
    import torch
    rng = np.random.default_rng(7)
    p0 = wl.procs[0]
    k_map = int(n * 0.9)
    sel = rng.integers(0, len(p0.leaf_va), k_map)
    size = np.uint64(1) << (np.uint64(12) + np.uint64(9) * (p0.leaf_level[sel].astype(np.uint64) - np.uint64(1)))
    g = p0.leaf_va[sel] + rng.integers(0, 1 << 62, k_map, dtype=np.uint64) % size
    user_limit = {3: 1 << 32, 4: 1 << 47, 5: 1 << 56}[p0.levels]
    g = np.concatenate([g, rng.integers(0, user_limit, n - k_map, dtype=np.uint64)])
    rng.shuffle(g)
    dg = torch.from_numpy(g.view(np.int64)).cuda()
    xo = torch.empty(n * 24, dtype=torch.uint8, device="cuda")
    ctx.translate(p0.asid, dg, n, 0, xo)
    ctx.sync()
    xt = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.translate(p0.asid, dg, n, 0, xo)
        ctx.sync()
        xt.append(time.perf_counter() - t0)
    return n / float(np.median(xt)) / 1e6


def translate_only(args):
    """Only the translate-only rate of one workload, one JSON line."""
    import paper_1304_3771_amd as dv
    from workload import device, gen
    wl = gen.make_workload(workload_spec(args.workload), requests=False)
    ctx = dv.Context(0)
    device.load(ctx, wl)
    mreq = translate_rate(ctx, wl, args.xlat_n, reps=args.steps)
    ctx.close()
    log(f"translate: {mreq:.1f} Mreq/s")
    print(json.dumps({"metric": "Mreq/s translated", "value": round(mreq, 1), "unit": "Mreq/s", "n_gpus": 1,
                      "steps": args.steps, "data": "synthetic", "dtype": "int64",
                      "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                                 "addresses": args.xlat_n}}))


def parse_set(text: str) -> dict:
    """Launch config overrides written as key=value,key=value."""
    return {k: int(v) for k, v in (kv.split("=") for kv in text.split(","))}


SERVING_WORKLOAD = ("C4: 8 VMs x 4 GiB, 4 processes x 64 guest threads each, Poisson arrivals, "
                    "60% 24B / 25% 4KiB / 14% 16-256KiB / 1% 4147200B")


def serving(args):
    """C4: Poisson arrivals through the serving loop, one JSON line."""
    out_rates = serving_rates(args, [float(x) for x in args.rates.split(",")], args.serve_plain_ops)
    print(json.dumps({"metric": "serving p50/p99 latency and throughput, C4", "unit": "us", "n_gpus": 1,
                      "data": "synthetic", "dtype": "u8", "config": serving_config(args), "rates": out_rates}))


def serving_config(args):
    return {"workload": SERVING_WORKLOAD, "max_inflight": args.max_inflight, "pool_gib": args.pool_gib,
            "max_batch": args.max_batch, "streams": args.streams, "completion": args.completion,
            "launch_config": args.set or "default"}


def serving_rates(args, rates, plain_ops, seconds=None, min_ops=None):
    """Each arrival rate's p50/p99 latency and throughput through the serving
    loop on C4, over max(rate x seconds, min_ops) arrivals (and, for
    plain_ops > 0, the per-request path at that rate)."""
    seconds = args.serve_seconds if seconds is None else seconds
    min_ops = args.serve_min_ops if min_ops is None else min_ops
    import torch
    import paper_1304_3771_amd as dv
    from workload import device, gen

    sp = gen.spec("C4")
    log("serving: generating C4 (8 VMs x 4 GiB)")
    wl = gen.make_workload(sp, requests=False)
    ctx = dv.Context(0)
    if args.set:
        ctx.set_config(**parse_set(args.set))
    dw = device.load(ctx, wl)
    log("serving: uploaded")
    out_rates = []
    pool = None
    for lam in rates:
        n_ops = int(max(lam * seconds, min_ops))
        tr = gen.make_serving_trace(wl, n_ops, lam)
        if pool is None or pool.numel() < tr.pool_bytes:
            pool = torch.empty(tr.pool_bytes, dtype=torch.uint8, device="cuda")
        reqs = tr.requests.copy()
        reqs["host"] += np.uint64(pool.data_ptr())
        srv = ctx.server_start(max_inflight=args.max_inflight, pool_bytes=args.pool_gib << 30,
                               max_batch=args.max_batch, streams=args.streams, completion=args.completion)
        comps = []
        pbuf = np.empty(1 << 14, dv.COMPLETION_DTYPE)
        t0 = time.monotonic_ns()
        i = 0
        polls = 0
        t_sub = t_poll = 0
        arrival = tr.arrival_ns.astype(np.int64)  # same dtype as `now`: no per-call cast of the whole array
        try:
            while i < n_ops:
                now = np.int64(time.monotonic_ns() - t0)
                j = int(np.searchsorted(arrival, now, side="right"))
                if j > i:
                    ta = time.monotonic_ns()
                    srv.submit(reqs[i:j])
                    t_sub += time.monotonic_ns() - ta
                    i = j
                polls += 1
                if polls % 16 == 0:
                    ta = time.monotonic_ns()
                    c = srv.poll(1 << 14, pbuf)
                    t_poll += time.monotonic_ns() - ta
                    if len(c):
                        comps.append(c)
            srv.drain()
            sst = srv.stats()
            while True:
                c = srv.poll(1 << 20)
                if not len(c):
                    break
                comps.append(c)
        finally:
            srv.stop()
        c = np.concatenate(comps)
        c = c[np.argsort(c["ticket"])]
        lat = (c["t_done_ns"].astype(np.int64) - (t0 + tr.arrival_ns.astype(np.int64))) / 1e3
        span = (c["t_done_ns"].max() - t0) / 1e9
        nbytes = int(c["bytes_done"].sum())
        wait = (c["t_admit_ns"].astype(np.int64) - (t0 + tr.arrival_ns.astype(np.int64))) / 1e3
        lag = (c["t_submit_ns"].astype(np.int64) - (t0 + tr.arrival_ns.astype(np.int64))) / 1e3
        run = (c["t_done_ns"].astype(np.int64) - c["t_admit_ns"].astype(np.int64)) / 1e3
        launches = len(np.unique(c["t_admit_ns"]))  # operations admitted together share the stamp
        rec = {"rate_mreq_s": lam / 1e6, "ops": n_ops, "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
               "throughput_mreq_s": n_ops / span / 1e6, "gbs": nbytes / span / 1e9,
               "submit_lag_us": {"p50": pct(lag, 50), "p99": pct(lag, 99)},
               "admission_wait_us": {"p50": pct(wait, 50), "p99": pct(wait, 99)},
               "in_flight_us": {"p50": pct(run, 50), "p99": pct(run, 99)},
               "launches": launches, "ops_per_launch": round(n_ops / max(1, launches), 1),
               "server_thread": sst}
        log(f"  driver: {polls} iterations, {t_sub / 1e9:.3f} s in submit, {t_poll / 1e9:.3f} s in poll")
        log(f"  server thread over {span:.2f} s: inbox {sst['ns_inbox'] / 1e9:.3f} s, completions "
            f"{sst['ns_complete'] / 1e9:.3f} s, admission {sst['ns_admit'] / 1e9:.3f} s, launches "
            f"{sst['ns_launch'] / 1e9:.3f} s ({sst['launches']} launches, {sst['direct_launches']} direct, "
            f"{sst['loops']} loops)")
        # the plain per-request path at the same arrival rate (bounded sample)
        m = min(n_ops, plain_ops)
        if m == 0:
            out_rates.append(rec)
            log(f"lambda {lam / 1e6:.2f} M/s: served p50 {rec['p50_us']:.0f} us p99 {rec['p99_us']:.0f} us "
                f"(submit lag p50 {pct(lag, 50):.0f}, wait p50 {pct(wait, 50):.0f}, in flight p50 {pct(run, 50):.0f} p99 {pct(run, 99):.0f}; "
                f"{launches} launches, {rec['ops_per_launch']} ops each), {rec['throughput_mreq_s']:.3f} Mreq/s")
            continue
        stream = torch.cuda.current_stream()
        res = torch.zeros(m * 24, dtype=torch.uint8, device="cuda")
        done = np.zeros(m, np.int64)
        t0p = time.monotonic_ns()
        for k in range(m):
            while time.monotonic_ns() - t0p < int(tr.arrival_ns[k]):
                pass
            q = reqs[k]
            f = ctx.copy_to_guest if int(q["dir"]) == 1 else ctx.copy_from_guest
            f(int(q["asid"]), int(q["gva"]), int(q["host"]), int(q["len"]), res.data_ptr() + 24 * k, stream)
            stream.synchronize()
            done[k] = time.monotonic_ns()
        plat = (done - (t0p + tr.arrival_ns[:m].astype(np.int64))) / 1e3
        rec["per_request"] = {"ops": m, "p50_us": pct(plat, 50), "p99_us": pct(plat, 99),
                              "throughput_mreq_s": m / ((done[-1] - t0p) / 1e9) / 1e6}
        log(f"lambda {lam / 1e6:.2f} M/s: served p50 {rec['p50_us']:.0f} us p99 {rec['p99_us']:.0f} us "
            f"(submit lag p50 {pct(lag, 50):.0f}, wait p50 {pct(wait, 50):.0f}, in flight p50 {pct(run, 50):.0f} p99 {pct(run, 99):.0f}; "
            f"{launches} launches, {rec['ops_per_launch']} ops each), "
            f"{rec['throughput_mreq_s']:.3f} Mreq/s, {rec['gbs']:.1f} GB/s; per-request p50 "
            f"{rec['per_request']['p50_us']:.0f} us p99 {rec['per_request']['p99_us']:.0f} us")
        out_rates.append(rec)
    ctx.close()
    return out_rates


def free_guest_frames(wl, vm):
    """GPAs of the guest frames that no table and no mapped page of the encoded
    map uses (the frames a frontend could set aside for new tables)."""
    v = wl.vms[vm]
    nfr = v.mem_bytes >> 12
    cover = np.zeros(nfr + 1, np.int64)
    np.add.at(cover, v.pt_gfn.astype(np.int64), 1)
    np.add.at(cover, v.pt_gfn.astype(np.int64) + 1, -1)
    for p in wl.procs:
        if p.vm != vm:
            continue
        base = (p.leaf_frame >> np.uint64(12)).astype(np.int64)
        span = np.int64(1) << (9 * (p.leaf_level.astype(np.int64) - 1))
        np.add.at(cover, base, 1)
        np.add.at(cover, np.minimum(base + span, nfr), -1)
    return np.nonzero(np.cumsum(cover[:nfr]) == 0)[0].astype(np.uint64) << np.uint64(12)


def map_fresh_batch(rng, n, lim, mem_frames, dtype, write_flag):
    """n maps in runs of 16-4096 contiguous pages (log-uniform), like mmaps of
    device buffers, at random 2 MiB-aligned GVAs in the upper half of the user
    range [0, lim); frames uniform over the guest's memory."""
    g = []
    left = n
    while left:
        run = min(left, int(16 * 256 ** rng.random()))
        base = int(rng.integers(lim >> 22, (lim >> 21) - 8)) << 21  # the run ends below the limit
        g.append(np.uint64(base) + (np.arange(run, dtype=np.uint64) << np.uint64(12)))
        left -= run
    m = np.zeros(n, dtype)
    m["gva"] = np.concatenate(g)
    m["gpa"] = rng.integers(0, mem_frames, n).astype(np.uint64) << np.uint64(12)
    m["flags"] = write_flag
    return m


def map_remap_batch(rng, n, proc, mem_frames, dtype):
    """n maps onto pages the process's tables already map with 4 KiB leaves."""
    va = proc.leaf_va[proc.leaf_level == 1]
    m = np.zeros(n, dtype)
    m["gva"] = va[rng.integers(0, len(va), n)]
    m["gpa"] = rng.integers(0, mem_frames, n).astype(np.uint64) << np.uint64(12)
    m["flags"] = rng.integers(0, 2, n)
    return m


def map_bench(args):
    """Mapping pages (the guest-table writer), timed per call with HIP events."""
    import torch
    import paper_1304_3771_amd as dv
    from workload import device, gen

    sp = workload_spec(args.workload)
    log(f"map: generating {args.workload}")
    wl = gen.make_workload(sp, requests=False)
    ctx = dv.Context(0)
    dw = device.load(ctx, wl)
    p = wl.procs[0]
    free = free_guest_frames(wl, p.vm)  # ascending
    rng = np.random.default_rng(77)
    n = args.map_n
    lim = {3: 1 << 32, 4: 1 << 47, 5: 1 << 56}[p.levels]
    log(f"map: {len(free)} free guest frames, {n} maps per call")

    mem_frames = wl.vms[p.vm].mem_bytes >> 12

    def fresh_batch():
        return map_fresh_batch(rng, n, lim, mem_frames, dv.MAP_DTYPE, dv.MAP_WRITE)

    def remap_batch():
        return map_remap_batch(rng, n, p, mem_frames, dv.MAP_DTYPE)

    res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
    used = torch.zeros(1, dtype=torch.int64, device="cuda")
    # timing events made (and recorded once) up front: a torch event is created
    # lazily at its first record, which would otherwise land inside the timing
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    b.record()
    torch.cuda.synchronize()
    pool_per_call = args.map_pool
    out = {}
    calls = args.warmup + args.steps
    for kind, make in (("fresh", fresh_batch), ("remap", remap_batch)):
        # every batch made and uploaded first, each fresh call with a pool
        # slice of its own: the timed calls then run back to back
        dms = [torch.from_numpy(make().view(np.uint8).copy()).cuda() for _ in range(calls)]
        base = 0 if kind == "fresh" else calls * pool_per_call
        torch.cuda.synchronize()
        times, walls, hosts, tables = [], [], [], []
        bad = torch.zeros((), dtype=torch.int64, device="cuda")  # failed maps over all calls, counted on the GPU
        for it in range(calls):
            pool = free[base + it * pool_per_call:base + (it + 1) * pool_per_call]
            torch.cuda.synchronize()
            a.record()
            t0 = time.perf_counter()
            ctx.map_pages(0, dms[it], n, pool, res, used)
            host = (time.perf_counter() - t0) * 1e3
            b.record()
            b.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            bad += (res.view(n, 24)[:, 16:20] != 0).any(dim=1).sum()
            if it >= args.warmup:
                times.append(a.elapsed_time(b))
                walls.append(wall)
                hosts.append(host)
                tables.append(int(used.item()))
        if int(bad.item()):
            raise RuntimeError(f"map bench: {int(bad.item())} maps failed")
        del dms
        ms = float(np.mean(times))
        out[kind] = {"ms_per_call": round(ms, 4), "maps_per_s": round(n / ms * 1e3, 1),
                     "wall_ms_per_call": round(float(np.mean(walls)), 4),
                     "host_ms_in_call": round(float(np.mean(hosts)), 4),
                     "new_tables_per_call": int(np.mean(tables)), "calls": len(times)}
        log(f"map {kind}: {ms:.3f} ms per call of {n} maps, {n / ms / 1e3:.2f} Mmaps/s, "
            f"{int(np.mean(tables))} new tables per call")
    ctx.close()
    # algorithmic bytes of a fresh call: per map the record read, the result
    # written, the leaf entry written and a page-set slot (key + index); per
    # new table its 4 KiB zeroed (table-entry reads are left out: the walks
    # share them through the caches)
    alg = n * (24 + 24 + 8 + 16) + out["fresh"]["new_tables_per_call"] * 4096
    achieved = alg / (out["fresh"]["ms_per_call"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "devirt_map_pages (whole call)",
            "alg_bytes_per_call": alg}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        log("map: cpu baseline (oracle, fresh batches)")
        o = Oracle.from_workload(wl)
        nxt, tot, calls = 0, 0.0, 0
        while tot < args.cpu_seconds and calls < 80:
            m = fresh_batch()
            t0 = time.perf_counter()
            r, u = o.map_pages(0, m, free[nxt:nxt + pool_per_call])
            tot += time.perf_counter() - t0
            nxt += u
            calls += 1
        cpu = {"value": round(calls * n / tot, 1), "unit": "maps/s", "cores": 1, "kind": "oracle",
               "sample": f"{calls} fresh batches of {n} maps on {args.workload}'s tables, sequential, "
                         f"{tot:.1f} s on one of {os.cpu_count()} host cores"}
        log(f"map: cpu baseline {cpu['value'] / 1e6:.2f} Mmaps/s")
    print(json.dumps({"metric": "maps/s (guest-table writer)", "value": out["fresh"]["maps_per_s"], "unit": "maps/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                      "data": "synthetic", "dtype": "int64",
                      "config": {"workload": f"{args.workload} tables, {n} 4 KiB maps per call; fresh: runs of "
                                             "16-4096 pages at new 2 MiB-aligned GVAs; remap: mapped 4 KiB pages"},
                      "fresh": out["fresh"], "remap": out["remap"], "roofline": roof, "cpu_baseline": cpu}))


TUNE_CACHE = os.path.join(ROOT, "paper_1304_3771_amd", "tuning_cache.jsonl")


def tune(ctx, wl, name, dw, res, faults, nf, args):
    """The launch configuration: the tuning cache's entry for this workload on
    this device, else a tuning run (stored in the cache).  --retune tunes
    afresh and appends the new entry."""
    from workload import gen
    key = gen.workload_key(wl, name)
    n = wl.n_requests
    reps = 3 if n <= 2_000_000 else 1
    t0 = time.time()
    if args.retune:
        tmp = args.tune_cache + ".new"
        if os.path.exists(tmp):
            os.remove(tmp)
        best, ms, hit = ctx.autotune_cached(tmp, key, dw.reqs, n, res, wl.epoch_end, faults, nf, reps=reps)
        with open(tmp) as f, open(args.tune_cache, "a") as g:
            g.write(f.read())
        os.remove(tmp)
    else:
        best, ms, hit = ctx.autotune_cached(args.tune_cache, key, dw.reqs, n, res, wl.epoch_end, faults, nf,
                                            reps=reps)
    src = "tuning cache" if hit else "tuned now"
    log(f"{name}: launch config from the {src} in {time.time() - t0:.1f}s: {best} ({ms:.3f} ms)")
    return {"key": key, "source": src, "tuned_ms": round(ms, 4)}


class Batched:
    """Timed steps of one batched workload: between steps (untimed) the
    page-table frames are restored and 1 GiB is written to flush the caches."""

    def __init__(self, ctx, wl, dw, res, faults, nf, flush):
        self.ctx, self.wl, self.dw, self.res, self.faults, self.nf, self.flush = ctx, wl, dw, res, faults, nf, flush

    def reset(self):
        import torch
        restore_tables(self.ctx, self.wl)
        self.flush.fill_(1)
        torch.cuda.synchronize()

    def step(self, t_done=None):
        self.ctx.submit_batch(self.dw.reqs, self.wl.n_requests, self.res, self.wl.epoch_end, self.faults, self.nf,
                              t_done)

    def warm(self, k):
        for _ in range(k):
            self.reset()
            self.step()
            self.ctx.sync()
        log(f"warmup done ({k})")

    def profiled_steps(self, k, counters=False):
        """k steps with HIP events around every kernel launch (no graphs); summed stats.
        Device counters (which add atomics of their own) only when asked for."""
        tot = None
        for _ in range(k):
            self.reset()
            self.ctx.set_profiling(True, counters=counters)
            self.ctx.reset_stats()
            self.step()
            self.ctx.sync()
            st = self.ctx.get_stats()
            self.ctx.set_profiling(False)
            tot = st if tot is None else {key: tot[key] + st[key] for key in st}
        return tot

    def measure(self, warmup, steps, name, roof_steps=ROOF_STEPS):
        """Timed steps, the copy kernel's roofline (overlapped, then alone) and
        one step of device counters."""
        import torch
        import paper_1304_3771_amd as dv
        ctx = self.ctx
        self.warm(warmup)
        times = []
        for _ in range(steps):
            self.reset()
            t0 = time.perf_counter()
            self.step()
            ctx.sync()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        r = self.res.cpu().numpy().view(dv.RESULT_DTYPE)
        copied = int(r["bytes_done"].sum())
        ms_step = 1e3 * float(np.mean(times))
        gbs = copied / (ms_step * 1e-3) / 1e9
        nfaults = int(self.nf.item())
        log(f"{name} batched: {ms_step:.3f} ms/step, {gbs:.1f} GB/s copied, {nfaults} faults")
        # roofline of the dominant kernel (copy): HIP events around each launch
        # on its stream, over roof_steps steps of the same batch and config
        st = self.profiled_steps(roof_steps)
        copy_launches = max(1, st["copy_launches"])
        copy_ms = st["copy_ms"]
        alg_copy = 2 * copied * roof_steps  # every copied byte is read once and written once
        achieved = (alg_copy / copy_launches) / (copy_ms / copy_launches * 1e-3) / 1e9 if copy_ms > 0 else None
        roof = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": measured_traffic(name), "kernel": "k_copy", "launches": copy_launches,
                "avg_launch_ms": round(copy_ms / copy_launches, 4), "alg_bytes_per_launch": alg_copy // copy_launches}
        # the copy kernel alone on the GPU: translation not overlapped
        tuned = ctx.get_config()
        ctx.set_config(**{**tuned, "overlap": 0, "xlat_wgs_per_cu": 3})
        st_alone = self.profiled_steps(roof_steps)
        ctx.set_config(**tuned)
        alone_ms = st_alone["copy_ms"] / max(1, st_alone["copy_launches"])
        alone = (alg_copy / copy_launches) / (alone_ms * 1e-3) / 1e9 if alone_ms > 0 else None
        roof_alone = {"bound": "hbm", "achieved": round(alone, 1) if alone else None, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(alone / HBM_PEAK_GBS, 4) if alone else None,
                      "kernel": "k_copy", "avg_launch_ms": round(alone_ms, 4), "config": "overlap off"}
        log(f"{name} copy kernel alone (no overlap): {alone_ms:.4f} ms/launch, {alone:.1f} GB/s algorithmic")
        ps = self.profiled_steps(1, counters=True)  # device counters, in a step of their own
        cnt = {k: ps[k] for k in ("pages_walked", "cache_hits", "cache_misses", "segments", "inline_segments",
                                  "spilled_groups", "ad_atomics")}
        lookups = cnt["cache_hits"] + cnt["cache_misses"]
        cnt["cache_hit_rate"] = round(cnt["cache_hits"] / lookups, 4) if lookups else None
        log(f"{name} copy kernel: {copy_launches // roof_steps} launches/step, {copy_ms / roof_steps:.3f} ms/step, "
            f"{achieved:.1f} GB/s algorithmic; translate kernel: {st['xlat_ms'] / roof_steps:.3f} ms/step; "
            f"per step: {cnt}")
        return {"ms_per_step": ms_step, "gbs": gbs, "bytes_copied_per_step": copied, "faults": nfaults,
                "req_per_s": self.wl.n_requests / (ms_step * 1e-3), "roofline": roof,
                "roofline_copy_alone": roof_alone, "translate_ms_per_step": round(st["xlat_ms"] / roof_steps, 4),
                "counters": cnt, "launch": ctx.get_config()}


def fifo_leg(ctx, wl, args):
    """Per-request launches of a locality trace (each process revisits a few
    buffers) with the per-process FIFO translation cache of `args.fifo_entries`
    entries and without it: hit rate, throughput and latency."""
    import torch
    import paper_1304_3771_amd as dv
    from workload import gen
    reqs, pool_bytes = gen.make_locality_trace(wl, args.fifo_ops)
    pool = torch.zeros(pool_bytes, dtype=torch.uint8, device="cuda")
    reqs["host"] += np.uint64(pool.data_ptr())
    res = torch.zeros(len(reqs) * 24, dtype=torch.uint8, device="cuda")
    base = res.data_ptr()
    stream = torch.cuda.current_stream()
    calls = [(ctx.copy_to_guest if int(q["dir"]) == 1 else ctx.copy_from_guest, int(q["asid"]), int(q["gva"]),
              int(q["host"]), int(q["len"])) for q in reqs]
    tuned = ctx.get_config()
    out = {"trace": f"{len(reqs)} operations, 4 hot buffers of 16 B-4 KiB per process hit with p=0.95, "
                    "else 16 B-16 KiB anywhere in the process's VMAs", "entries": args.fifo_entries}
    for label, entries in (("cache", args.fifo_entries), ("no_cache", 0)):
        ctx.set_config(**{**tuned, "fifo_entries": entries})
        ctx.fifo_flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (f, a, g, h, ln) in enumerate(calls):
            f(a, g, h, ln, base + 24 * i, stream)
        ctx.sync(stream)
        dt = time.perf_counter() - t0
        ls = min(args.lat_sample, len(calls))
        lats = np.zeros(ls)
        for i in range(ls):
            f, a, g, h, ln = calls[i]
            t1 = time.perf_counter()
            f(a, g, h, ln, base + 24 * i, stream)
            stream.synchronize()
            lats[i] = (time.perf_counter() - t1) * 1e6
        d = {"req_per_s": round(len(calls) / dt, 1), "latency_us": {"p50_us": pct(lats, 50), "p99_us": pct(lats, 99)}}
        if entries:
            hm = np.array([ctx.fifo_counts(p.asid) for p in wl.procs], np.float64).sum(axis=0)
            d["hits"], d["misses"] = int(hm[0]), int(hm[1])
            d["hit_rate"] = round(hm[0] / max(1.0, hm.sum()), 4)
        out[label] = d
    ctx.set_config(**tuned)
    r = res.cpu().numpy().view(dv.RESULT_DTYPE)
    out["bytes_copied"] = int(r["bytes_done"].sum())
    log(f"per-request with a {args.fifo_entries}-entry FIFO translation cache: hit rate {out['cache']['hit_rate']}, "
        f"{out['cache']['req_per_s']:.0f} req/s (without: {out['no_cache']['req_per_s']:.0f}); p50 "
        f"{out['cache']['latency_us']['p50_us']:.1f} us (without: {out['no_cache']['latency_us']['p50_us']:.1f})")
    return out


def extra_workload(name, args):
    """Another batched workload measured in the same run (its own context):
    tuned launch, timed steps, copy-kernel roofline and counters."""
    import torch
    import paper_1304_3771_amd as dv
    from workload import device, gen
    t0 = time.time()
    log(f"{name}: generating")
    wl = gen.make_workload(workload_spec(name))
    n = wl.n_requests
    ctx = dv.Context(0)
    try:
        dw = device.load(ctx, wl)
        log(f"{name}: {n} requests, {len(wl.epoch_end)} epochs, loaded in {time.time() - t0:.1f}s")
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        tuning = tune(ctx, wl, name, dw, res, faults, nf, args)
        m = Batched(ctx, wl, dw, res, faults, nf, flush).measure(1, args.extra_steps, name, roof_steps=2)
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    return {"workload": f"{name}: {WORKLOADS[name]}", "requests": n, "epochs": int(len(wl.epoch_end)),
            "ms_per_step": round(m["ms_per_step"], 3), "value": round(m["gbs"], 2), "unit": "GB/s",
            "req_per_s": round(m["req_per_s"], 1), "bytes_copied_per_step": m["bytes_copied_per_step"],
            "faults": m["faults"], "roofline": m["roofline"], "roofline_copy_alone": m["roofline_copy_alone"],
            "translate_ms_per_step": m["translate_ms_per_step"], "counters": m["counters"],
            "launch": m["launch"], "tuning": tuning, "steps": args.extra_steps}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-sample", type=int, default=20000, help="requests timed on the per-request path")
    ap.add_argument("--lat-sample", type=int, default=2000, help="per-request latencies sampled")
    ap.add_argument("--fifo-ops", type=int, default=20000, help="operations of the translation-cache trace")
    ap.add_argument("--fifo-entries", type=int, default=10, help="entries of the per-process FIFO cache")
    ap.add_argument("--xlat-n", type=int, default=16_000_000, help="addresses for the translate-only rate")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="skip autotuning the batch launch")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="tuning cache (JSON lines) to read and extend")
    ap.add_argument("--retune", action="store_true", help="tune afresh and append the result to the cache")
    ap.add_argument("--extra", default=None,
                    help="more batched workloads measured after the main one (default: C3,C5 after C2)")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of each extra workload")
    ap.add_argument("--profile-only", action="store_true", help="only run K timed steps (for rocprofv3)")
    ap.add_argument("--set", default="", help="launch config overrides, e.g. seg_chunks=64,nontemporal=1")
    ap.add_argument("--serving", action="store_true", help="run the C4 serving sweep instead")
    ap.add_argument("--translate-only", action="store_true",
                    help="only the translate-only rate of the workload (devirt_translate, --xlat-n addresses)")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave out the short C4 serving leg (1 and 5 M req/s) of the default C2 run")
    ap.add_argument("--map", action="store_true", help="time mapping pages (the guest-table writer) instead")
    ap.add_argument("--map-n", type=int, default=1 << 19, help="maps per call")
    ap.add_argument("--map-pool", type=int, default=4096, help="free guest frames handed to each call")
    ap.add_argument("--rates", default="1e5,2.5e5,5e5,1e6,2e6,5e6")
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--serve-min-ops", type=int, default=200000)
    ap.add_argument("--serve-plain-ops", type=int, default=20000)
    ap.add_argument("--max-inflight", type=int, default=8192)
    ap.add_argument("--pool-gib", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=4096)
    ap.add_argument("--streams", type=int, default=3)
    ap.add_argument("--completion", default="poll", choices=["poll", "notify", "blocking"],
                    help="how the serving loop learns that a batch finished")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1304_3771_amd as dv
    from workload import device, gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dv.lib()
    if args.serving:
        return serving(args)
    if args.map:
        return map_bench(args)
    if args.translate_only:
        return translate_only(args)

    t_gen = time.time()
    sp = workload_spec(args.workload)
    log(f"generating {args.workload}")
    wl = gen.make_workload(sp)
    n = wl.n_requests
    log(f"generated {n} requests, {len(wl.epoch_end)} epochs in {time.time() - t_gen:.1f}s; uploading")
    ctx = dv.Context(0)
    if args.set:
        ctx.set_config(**parse_set(args.set))
    dw = device.load(ctx, wl)
    log(f"uploaded; launch config {ctx.get_config()}")
    res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
    faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    tuning = None
    if not args.no_autotune and not args.set:
        tuning = tune(ctx, wl, args.workload, dw, res, faults, nf, args)

    n_epochs = int(len(wl.epoch_end))
    B = Batched(ctx, wl, dw, res, faults, nf, flush)
    if args.profile_only:
        B.warm(args.warmup)
        # the steps the roofline is measured on, for rocprofv3 to trace
        st = B.profiled_steps(args.steps)
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        copied = int(r["bytes_done"].sum())
        # a plain copy-like kernel of known size (1 GiB read + 1 GiB written) to scale HBM counters
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        for _ in range(3):
            torch.add(a, 1, out=b)
        torch.cuda.synchronize()
        avg = st["copy_ms"] / max(1, st["copy_launches"])
        log(f"profiled steps: copy kernel {st['copy_launches']} launches, average {avg:.4f} ms (HIP events)")
        print(json.dumps({"workload": args.workload, "steps": args.steps,
                          "copy_launches": st["copy_launches"], "copy_avg_ms_hip_events": avg,
                          "copy_launches_per_step": int(len(wl.epoch_end)),
                          "alg_copy_bytes_per_step": 2 * copied, "calibration_bytes_each_way": 1 << 30}))
        return
    m = B.measure(args.warmup, args.steps, args.workload)
    ms_step, gbs, copied = m["ms_per_step"], m["gbs"], m["bytes_copied_per_step"]
    roof, roof_alone, counters = m["roofline"], m["roofline_copy_alone"], m["counters"]
    path_alg = 2 * copied + 56 * n + 8 * counters["pages_walked"] + 24 * int(nf.item())
    path_frac = path_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    # ---- batched per-request completion latency (device clock)
    B.reset()
    td = torch.zeros(n, dtype=torch.int64, device="cuda")
    B.step(td)
    ctx.sync()
    tdn = td.cpu().numpy() / 1e3
    lat_batched = {"p50_us": pct(tdn, 50), "p99_us": pct(tdn, 99), "max_us": float(tdn.max())}
    log(f"batched latency p50 {lat_batched['p50_us']:.1f} us p99 {lat_batched['p99_us']:.1f} us")

    # ---- plain per-request launches (throughput over a sample, then latency)
    B.reset()
    ps = min(args.plain_sample, n)
    hreq = dw.reqs_host
    pres = torch.zeros(ps * 24, dtype=torch.uint8, device="cuda")
    base = pres.data_ptr()
    stream = torch.cuda.current_stream()
    calls = [(ctx.copy_to_guest if int(q["dir"]) == 1 else ctx.copy_from_guest, int(q["asid"]), int(q["gva"]),
              int(q["host"]), int(q["len"])) for q in hreq[:ps]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (f, a, g, h, ln) in enumerate(calls):
        f(a, g, h, ln, base + 24 * i, stream)
    ctx.sync(stream)
    t_plain = time.perf_counter() - t0
    pr = pres.cpu().numpy().view(dv.RESULT_DTYPE)
    plain_bytes = int(pr["bytes_done"].sum())
    plain = {"sample_requests": ps, "req_per_s": ps / t_plain, "gbs": plain_bytes / t_plain / 1e9}
    ls = min(args.lat_sample, ps)
    lats = np.zeros(ls)
    for i in range(ls):
        f, a, g, h, ln = calls[i]
        t0 = time.perf_counter()
        f(a, g, h, ln, base + 24 * i, stream)
        stream.synchronize()
        lats[i] = (time.perf_counter() - t0) * 1e6
    lat_plain = {"p50_us": pct(lats, 50), "p99_us": pct(lats, 99)}
    batched_req_s = n / (ms_step * 1e-3)
    log(f"plain: {plain['req_per_s']:.0f} req/s, {plain['gbs']:.2f} GB/s; latency p50 {lat_plain['p50_us']:.1f} "
        f"p99 {lat_plain['p99_us']:.1f} us")

    # ---- the per-request path with the paper's per-process FIFO translation cache
    fifo = fifo_leg(ctx, wl, args)

    # ---- translate-only rate (Mreq/s), READ, no A/D
    mreq = translate_rate(ctx, wl, args.xlat_n)
    log(f"translate: {mreq:.1f} Mreq/s")

    launch = ctx.get_config()
    ctx.close()
    del dw, res, faults, nf, flush, B, td, pres
    torch.cuda.empty_cache()

    # ---- CPU baseline: the oracle, one thread and N threads, on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_seconds, args.workload)
        log(f"cpu baseline: {cpu['value']} GB/s on {cpu['cores']} threads, {cpu['single_thread']['value']} GB/s "
            f"on one ({cpu['sample']})")
    del wl

    # ---- the other batched workloads, measured in the same run
    extra = {}
    extra_names = args.extra if args.extra is not None else ("C3,C5" if args.workload == "C2" else "")
    for name in [x for x in extra_names.split(",") if x and x != args.workload]:
        extra[name] = extra_workload(name, args)

    # ---- the serving loop on C4 at two arrival rates (the full sweep: --serving)
    serve = None
    if args.workload == "C2" and not args.no_serving and not args.profile_only:
        serve = {"config": serving_config(args),
                 "rates": serving_rates(args, [1e6, 5e6], 0, seconds=0.4, min_ops=200000)}

    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "requests": n,
                   "epochs": n_epochs, "bytes_copied_per_step": copied, "launch": launch, "tuning": tuning},
        "translate_mreq_s": round(mreq, 2),
        "batched": {"req_per_s": round(batched_req_s, 1), "latency_us": lat_batched,
                    "latency_clock": "device wall clock, from the start of the submission"},
        "per_request_fifo": fifo,
        "per_request": {**{k: round(v, 3) for k, v in plain.items()}, "latency_us": lat_plain,
                        "latency_clock": "host, launch to stream sync"},
        "roofline": roof,
        "roofline_copy_alone": roof_alone,
        "path_roofline_frac": round(path_frac, 4),
        "counters": counters,
        "cpu_baseline": cpu,
        "workloads": extra,
        "serving": serve,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

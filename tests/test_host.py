"""Host-side logic of the benchmark (no GPU): its refusal of several GPUs,
the free-frame finder against a brute-force set, the map batches it times
(every map must succeed), its workload names, and the kernel-source hash
that ties the committed HBM counters to the kernels they were taken on."""
import os
import subprocess
import sys

import numpy as np
import pytest

import pins
from oracle import Oracle
from oracle.oracle import MAP_DTYPE
from workload import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_free_guest_frames_brute_force():
    import bench
    w = gen.make_workload(pins.small_specs()["mix2m"])
    v = w.vms[0]
    used = set(int(x) for x in v.pt_gfn)
    for p in w.procs:
        if p.vm != 0:
            continue
        for lv, fr in zip(p.leaf_level, p.leaf_frame):
            b = int(fr) >> 12
            used.update(range(b, b + (1 << (9 * (int(lv) - 1)))))
    exp = sorted(set(range(v.mem_bytes >> 12)) - used)
    got = [int(x) >> 12 for x in bench.free_guest_frames(w, 0)]
    assert got == exp


@pytest.mark.parametrize("name", ["mix2m", "lvl5", "pae"])
def test_map_bench_batches_all_succeed(name):
    import bench
    w = gen.make_workload(pins.small_specs()[name])
    p = w.procs[0]
    lim = {3: 1 << 32, 4: 1 << 47, 5: 1 << 56}[p.levels]
    mem = w.vms[p.vm].mem_bytes >> 12
    free = bench.free_guest_frames(w, p.vm)
    rng = np.random.default_rng(1)
    o = Oracle.from_workload(w)
    nxt = 0
    makers = (lambda: bench.map_fresh_batch(rng, 4096, lim, mem, MAP_DTYPE, 1),
              lambda: bench.map_remap_batch(rng, 4096, p, mem, MAP_DTYPE))
    for make in makers:
        for _ in range(2):
            r, used = o.map_pages(0, make(), free[nxt:nxt + 2048])
            assert np.all(r["code"] == 0), np.bincount(r["code"])
            nxt += used


def test_bench_workloads_resolve():
    import bench
    for name in bench.WORKLOADS:
        sp = bench.workload_spec(name)
        assert sp.n_requests > 0 and sp.levels in (3, 4, 5)
    assert bench.workload_spec("C2-EPT").ept and bench.workload_spec("C2-PAE").levels == 3


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    """The hash that ties committed HBM counters to the kernels changes with
    the code but not with comments or blank lines."""
    import shutil
    import bench
    src = os.path.join(ROOT, "paper_1304_3771_amd", "csrc")
    dst = tmp_path / "paper_1304_3771_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("kernels.hip", "dv_internal.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_hash()
    with open(dst / "kernels.hip", "a") as f:
        f.write("\n// a comment\n/* and a\n   block comment */\n\n")
    assert bench.kernel_hash() == h0
    with open(dst / "dv_internal.h", "a") as f:
        f.write("\nconstexpr int kUnused = 1;\n")
    assert bench.kernel_hash() != h0


@pytest.mark.parametrize("workload", ["C2", "C3", "C5", "C2-EPT"])
def test_committed_counters_match_the_kernels(workload):
    """The committed rocprofv3 HBM counters of each workload's copy kernel were
    taken on the current kernel source (else the bench reports no traffic)."""
    import bench
    t = bench.measured_traffic(workload)
    assert t is not None and t > 0, f"profiles/copy_traffic_{workload}.json is stale or missing"

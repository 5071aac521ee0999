"""devirt_copy_static, the per-request copy that allocates nothing (its
scratch is a static device array), against the per-request calls it varies,
devirt_copy_from_guest and devirt_copy_to_guest: the same calls in the same
order on two contexts holding the same world must leave identical results,
guest memory (A/D bits included) and host buffers, bit for bit.  Two calls in
a row, the second smaller, in each direction; then a request past the size
limit is refused with nothing done."""
import numpy as np
import pytest

import pins
from gpu_util import log, new_ctx
from workload import device, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _host_image(nbytes: int, key: int) -> np.ndarray:
    out = np.empty(nbytes, np.uint8)
    return gen.fill_bytes(out, 97, key)


def _present_runs(p):
    """(gva, bytes) of the longest runs of present leaves, longest first."""
    order = np.argsort(p.leaf_va)
    va = p.leaf_va[order].astype(np.int64)
    size = (np.int64(1) << (12 + 9 * (p.leaf_level[order].astype(np.int64) - 1)))
    ok = p.leaf_present[order]
    runs, start, end = [], None, None
    for v, n, good in zip(va, size, ok):
        if good and start is not None and v == end:
            end = v + n
            continue
        if start is not None:
            runs.append((start, end - start))
        start, end = (v, v + n) if good else (None, None)
    if start is not None:
        runs.append((start, end - start))
    return sorted(runs, key=lambda r: -r[1])


def test_static_copy_matches_per_request_calls():
    import torch
    import paper_1304_3771_amd as dv
    w = gen.make_workload(pins.small_specs()["mix2m"])
    p = w.procs[0]
    runs = _present_runs(p)
    (g0, n0), (g1, n1) = runs[0], runs[1]
    KiB = 1 << 10
    assert n0 > 2048 * KiB and n1 > 256 * KiB
    # (gva, len, dir, host offset): a long call (queued segments) then a
    # smaller one, in each direction, offsets and lengths unaligned on both
    # sides; the last one runs past its run into a not-present page and
    # stops there (prefix semantics)
    calls = [
        (g0 + 123, min(n0 - 123, 5 * 1024 * KiB + 777), dv.TO_GUEST, 37),
        (g1 + 999, 96 * KiB + 5, dv.TO_GUEST, 64 * 1024 * KiB + 11),
        (g0 + 4096 + 5, min(n0 - 4101, 3 * 1024 * KiB + 1), dv.FROM_GUEST, 7 * 1024 * KiB + 3),
        (g1 + n1 - 150 * KiB - 9, 200 * KiB, dv.FROM_GUEST, 80 * 1024 * KiB + 60),
    ]
    host_bytes = 96 * 1024 * KiB
    img = _host_image(host_bytes, 5)
    got = {}
    for mode in ("per_request", "static"):
        ctx = new_ctx()
        try:
            dw = device.load(ctx, w)
            host = torch.from_numpy(img.copy()).cuda()
            res = torch.zeros(24 * len(calls), dtype=torch.uint8, device="cuda")
            snaps = []
            for k, (gva, n, d, off) in enumerate(calls):
                log(f"{mode}: call {k} gva {gva:#x} len {n} dir {d} host+{off}")
                h = host.data_ptr() + off
                r = res.data_ptr() + 24 * k
                if mode == "static":
                    ctx.copy_static(p.asid, gva, h, n, d, r)
                elif d == dv.TO_GUEST:
                    ctx.copy_to_guest(p.asid, gva, h, n, r)
                else:
                    ctx.copy_from_guest(p.asid, gva, h, n, r)
                ctx.sync()
                torch.cuda.synchronize()
                snaps.append((res.cpu().numpy().copy(), device.read_arenas(ctx, dw)[0], host.cpu().numpy()))
            if mode == "static":
                # past the limit (16,384 pages): refused on the host, nothing done
                with pytest.raises(dv.DevirtError):
                    ctx.copy_static(p.asid, g0, host.data_ptr(), 65 * 1024 * KiB, dv.FROM_GUEST,
                                    res.data_ptr())
                ctx.sync()
                torch.cuda.synchronize()
                assert np.array_equal(host.cpu().numpy(), snaps[-1][2])
                assert np.array_equal(device.read_arenas(ctx, dw)[0], snaps[-1][1])
            got[mode] = snaps
        finally:
            ctx.close()
    for k in range(len(calls)):
        ra, aa, ha = got["per_request"][k]
        rb, ab, hb = got["static"][k]
        rr = ra.view(dv.RESULT_DTYPE)[k]
        log(f"call {k}: code {int(rr['code'])} bytes_done {int(rr['bytes_done'])}")
        assert np.array_equal(ra, rb), f"results differ after call {k}"
        assert np.array_equal(aa, ab), f"guest memory differs after call {k}"
        assert np.array_equal(ha, hb), f"host buffer differs after call {k}"
    # every call copied more than the inline limit (16 pages), so the copy
    # kernel ran on the queued segments; the last one faulted on its way
    r = got["static"][-1][0].view(dv.RESULT_DTYPE)
    assert np.all(r["bytes_done"] > 16 * 4096)
    assert np.all(r["code"][:3] == 0) and r["code"][3] == dv.CODES["NOT_PRESENT"]

"""Full-size parity: the one-guest 4 GiB workload with 1e6 requests (64 B - 64 KiB,
70/30 4 KiB/2 MiB pages, 16 memslots, 5% not present), run exactly as the
benchmark times it (default launch configuration, HIP graph, all epochs),
compared with the oracle on every result, every fault record, every arena
byte (A/D bits included) and every host-buffer byte."""
import numpy as np
import pytest

from gpu_util import log, new_ctx
from oracle import Oracle
from workload import device, gen

pytestmark = pytest.mark.gpu


def test_full_c2_bit_exact():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_3771_amd as dv
    log("full C2: generating")
    wl = gen.make_workload(gen.spec("C2"))
    n = wl.n_requests
    ctx = new_ctx()
    try:
        dw = device.load(ctx, wl)
        log("full C2: uploaded, running the batch")
        res = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        faults = torch.zeros(n * 24, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.submit_batch(dw.reqs, n, res, wl.epoch_end, faults, nf)
        ctx.sync()
        r = res.cpu().numpy().view(dv.RESULT_DTYPE)
        k = int(nf.item())
        f = faults.cpu().numpy()[:24 * k].view(dv.FAULT_DTYPE)
        arena = device.read_arenas(ctx, dw)[0]
        log("full C2: running the oracle")
        o = Oracle.from_workload(wl)
        er, ef = o.batch(wl.requests)
        assert np.array_equal(r.view(np.uint8), er.view(np.uint8)), "results differ"
        assert np.array_equal(f.view(np.uint8), ef.view(np.uint8)), "fault lists differ"
        bad = np.count_nonzero(arena != o.arenas[0])
        assert bad == 0, f"{bad} arena bytes differ"
        del arena
        chunk = 1 << 30
        for off in range(0, wl.pool_bytes, chunk):
            m = min(chunk, wl.pool_bytes - off)
            got = dw.pool[off:off + m].cpu().numpy()
            assert np.array_equal(got, o.pool[off:off + m]), f"pool differs in [{off}, {off + m})"
        log(f"full C2: bit-exact ({n} requests, {k} faults, {int(r['bytes_done'].sum())} bytes)")
    finally:
        ctx.close()

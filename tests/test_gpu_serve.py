"""GPU tests of the continuous-batching server: every result is the same
alone and in the mix; the budget admits, queues and rejects."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_00238_amd import synth

pytestmark = pytest.mark.gpu

TIGHT = 1e-3


def _inputs(W, H, seed, kind):
    img = synth.synth_image(W, H, seed=seed)
    if kind == "blocks":
        mask = synth.mask_blocks(W, H, 4, 0.2, seed=seed + 1)
    else:
        mask = synth.mask_blocks_and_pixels(W, H, 4, 0.25, 0.01, seed=seed + 1)
    return img, mask


def test_results_same_alone_and_in_the_mix():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    cases = [(96, 80, 61, "blocks"), (200, 136, 63, "pixels"), (128, 128, 65, "blocks"), (64, 200, 67, "pixels"),
             (150, 93, 69, "blocks"), (256, 160, 71, "pixels")]
    p = fse.fse_params_default(classes=((4, 14, 60),))
    alone = []
    tens = []
    for (W, H, sd, kind) in cases:
        img, mask = _inputs(W, H, sd, kind)
        ti = torch.from_numpy(img).to(dev)
        tm = torch.from_numpy(mask).to(dev)
        o = torch.empty_like(ti)
        fse.fse_extrapolate(ti, tm, p, o)
        torch.cuda.synchronize()
        alone.append(o.cpu().numpy())
        tens.append((ti, tm, torch.full_like(ti, -1.0), img, mask))
    srv = fse.fse_serve_create(hbm_budget_bytes=1 << 30, max_slots=3)
    try:
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for (ti, tm, o, _, _) in tens]
        stats = [fse.fse_serve_wait(srv, t, 60_000_000) for t in tickets]
    finally:
        fse.fse_serve_destroy(srv)
    for (ti, tm, o, img, mask), a, st in zip(tens, alone, stats):
        got = o.cpu().numpy()
        assert np.array_equal(got, a), "served result differs from the alone result"
        assert st["t_done_ms"] >= st["t_admit_ms"] >= st["t_submit_ms"] > 0
    # one of them against the oracle as well
    img, mask = tens[0][3], tens[0][4]
    ref = O.image(img, mask, ((4, 14, 60),))
    assert np.abs(alone[0] - ref)[mask.astype(bool)].max() <= TIGHT


def test_budget_queues_and_rejects():
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    p = fse.fse_params_default(classes=((4, 14, 20),))
    img, mask = _inputs(256, 256, 81, "blocks")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    torch.cuda.synchronize()  # inputs complete before the server's streams read them
    # budget fits about one request at a time: the rest must queue, not fail
    srv = fse.fse_serve_create(hbm_budget_bytes=256 * 256 * 14, max_slots=2)
    try:
        outs = [torch.empty_like(ti) for _ in range(4)]
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for o in outs]
        stats = [fse.fse_serve_wait(srv, t, 60_000_000) for t in tickets]
        ref = outs[0].cpu().numpy()
        for o in outs[1:]:
            assert np.array_equal(o.cpu().numpy(), ref)
        # admitted one after another
        admits = sorted(s["t_admit_ms"] for s in stats)
        dones = sorted(s["t_done_ms"] for s in stats)
        assert admits[1] >= dones[0] - 1e-3
        big = torch.zeros((2048, 2048), dtype=torch.float32, device=dev)
        bm = torch.zeros((2048, 2048), dtype=torch.uint8, device=dev)
        with pytest.raises(fse.FseError) as ei:
            fse.fse_serve_submit(srv, big, bm, p, torch.empty_like(big))
        assert ei.value.status == fse.FSE_ERR_BUDGET
    finally:
        fse.fse_serve_destroy(srv)


def test_destroy_frees_slot_workspaces():
    # each slot's device tables (128 MiB of FP64 reconstructed values alone
    # for a 4096x4096 request) go back to the device when the server is destroyed
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    img, mask = _inputs(4096, 4096, 81, "blocks")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    outs = [torch.empty_like(ti) for _ in range(3)]
    torch.cuda.synchronize()  # inputs complete before the server's streams read them
    p = fse.fse_params_default(classes=((4, 14, 10),))

    def cycle():
        srv = fse.fse_serve_create(hbm_budget_bytes=1 << 30, max_slots=3)
        try:
            tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for o in outs]
            for t in tickets:
                fse.fse_serve_wait(srv, t, 60_000_000)
        finally:
            fse.fse_serve_destroy(srv)
        torch.cuda.synchronize()

    cycle()  # first use: runtime state that stays for the process
    free0 = torch.cuda.mem_get_info()[0]
    cycle()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < 64 << 20, f"{(free0 - free1) >> 20} MiB not returned"
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_cancel_a_queued_request():
    # the budget admits one 2048x2048 request at a time: of three submitted
    # together, the third is still queued when it is withdrawn
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    img, mask = _inputs(2048, 2048, 85, "pixels")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    outs = [torch.full_like(ti, -3.0) for _ in range(3)]
    torch.cuda.synchronize()
    p = fse.fse_params_default(classes=((4, 14, 30),))
    srv = fse.fse_serve_create(hbm_budget_bytes=2048 * 2048 * 12, max_slots=2)
    try:
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for o in outs]
        assert fse.fse_serve_cancel(srv, tickets[2])
        with pytest.raises(fse.FseError) as ei:
            fse.fse_serve_wait(srv, tickets[2], 60_000_000)
        assert ei.value.status == fse.FSE_ERR_CANCELLED
        for t in tickets[:2]:
            fse.fse_serve_wait(srv, t, 60_000_000)
        with pytest.raises(fse.FseError) as ei:  # collected tickets are gone
            fse.fse_serve_cancel(srv, tickets[0])
        assert ei.value.status == fse.FSE_ERR_NOT_FOUND
    finally:
        fse.fse_serve_destroy(srv)
    assert torch.equal(outs[0], outs[1])
    assert (outs[2] == -3.0).all()  # the withdrawn request never ran


def test_mixed_parameters_in_one_server():
    # requests with different parameters (K, tiling) never share a launch;
    # each result equals the same request alone
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    pa = fse.fse_params_default(classes=((4, 14, 60),))
    pb = fse.fse_params_default(classes=((4, 14, 20),))
    pc = fse.fse_params_default(classes=((4, 14, 60),), tiling=fse.FSE_TILED, n_tiles=4, overlap=16, align=4)
    cases = []
    for i, p in enumerate([pa, pb, pc, pa, pb, pc]):
        img, mask = _inputs(96 + 8 * i, 80, 101 + i, "pixels")
        ti = torch.from_numpy(img).to(dev)
        tm = torch.from_numpy(mask).to(dev)
        alone = torch.empty_like(ti)
        fse.fse_extrapolate(ti, tm, p, alone)
        cases.append((ti, tm, p, alone, torch.full_like(ti, -1.0)))
    torch.cuda.synchronize()
    srv = fse.fse_serve_create(hbm_budget_bytes=1 << 30, max_slots=3)
    try:
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for (ti, tm, p, _, o) in cases]
        for t in tickets:
            fse.fse_serve_wait(srv, t, 60_000_000)
    finally:
        fse.fse_serve_destroy(srv)
    for k, (_, _, _, alone, o) in enumerate(cases):
        assert torch.equal(alone, o), f"request {k}: served differs from alone"


def test_wait_limit_error_fails_the_served_request(monkeypatch):
    # a launch whose dependency wait hits its (host-forced, zero) time limit
    # reports its error word; the server fails that request with
    # FSE_ERR_DEVICE instead of serving the invalid result, and a request
    # served afterwards with the normal limit is clean
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    img, mask = _inputs(256, 192, 91, "pixels")
    ti = torch.from_numpy(img).to(dev)
    tm = torch.from_numpy(mask).to(dev)
    p = fse.fse_params_default(classes=((4, 14, 30),), workgroups=256)
    o = torch.full_like(ti, -1.0)
    torch.cuda.synchronize()
    monkeypatch.setenv("FSE_WAIT_LIMIT_US", "0")
    srv = fse.fse_serve_create(hbm_budget_bytes=1 << 30, max_slots=2)
    try:
        t = fse.fse_serve_submit(srv, ti, tm, p, o)
        with pytest.raises(fse.FseError) as ei:
            fse.fse_serve_wait(srv, t, 60_000_000)
        assert ei.value.status == fse.FSE_ERR_DEVICE
        monkeypatch.delenv("FSE_WAIT_LIMIT_US")
        o2 = torch.full_like(ti, -1.0)
        t2 = fse.fse_serve_submit(srv, ti, tm, p, o2)
        fse.fse_serve_wait(srv, t2, 60_000_000)
    finally:
        fse.fse_serve_destroy(srv)
    ref = O.image(img, mask, ((4, 14, 30),))
    m = mask.astype(bool)
    assert np.abs(o2.cpu().numpy() - ref)[m].max() <= TIGHT


def test_trace_requests_against_the_oracle():
    # seeded requests of the serving trace (Poisson arrivals, square sides of
    # 512..4096, two mask kinds): the first 512 x 512 requests of the trace,
    # each with its own image and mask, served together with a 1024 x 1024
    # request of the same trace, every 512 x 512 result within the parity bar
    # of the FP64 oracle (its level-parallel form, bitwise the raster oracle)
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    trace = synth.poisson_trace(200.0, 2.0, seed=31)
    small = [r for r in trace if r["side"] == 512][:3]
    big = [r for r in trace if r["side"] == 1024][:1]
    assert len(small) == 3 and len(big) == 1
    cls = ((4, 14, 100),)
    p = fse.fse_params_default(classes=cls)
    reqs = []
    for r in small + big:
        img, mask = synth.request_inputs(r)
        ti = torch.from_numpy(img).to(dev)
        tm = torch.from_numpy(mask).to(dev)
        reqs.append((r, img, mask, ti, tm, torch.full_like(ti, -1.0)))
    torch.cuda.synchronize()
    srv = fse.fse_serve_create(hbm_budget_bytes=4 << 30, max_slots=2)
    try:
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for (_, _, _, ti, tm, o) in reqs]
        for t in tickets:
            fse.fse_serve_wait(srv, t, 120_000_000)
    finally:
        fse.fse_serve_destroy(srv)
    for (r, img, mask, _, _, o) in reqs[:3]:
        print("request", r["image_seed"], r["kind"], flush=True)
        ref, _, _ = O.image_levels(img, mask, cls)
        got = o.cpu().numpy()
        m = mask.astype(bool)
        assert np.array_equal(got[~m], img[~m])
        assert np.abs(got.astype(np.float64) - ref)[m].max() <= TIGHT


def test_sixteen_slots_each_result_as_alone():
    # the largest server: sixteen slots (each a stream with a hardware queue of
    # its own and a planning thread), requests submitted one by one so that
    # many groups are planned and in flight at once; every result bitwise the
    # request alone
    import torch
    from paper_2207_00238_amd import fse
    dev = torch.device("cuda:0")
    p = fse.fse_params_default(classes=((4, 14, 40),))
    reqs = []
    for i in range(24):
        W, H = 64 + 16 * (i % 5), 48 + 16 * (i % 3)
        img, mask = _inputs(W, H, 1200 + 2 * i, "blocks" if i % 2 else "pixels")
        ti = torch.from_numpy(img).to(dev)
        tm = torch.from_numpy(mask).to(dev)
        alone = torch.empty_like(ti)
        fse.fse_extrapolate(ti, tm, p, alone)
        reqs.append((ti, tm, torch.full_like(ti, -1.0), alone))
    torch.cuda.synchronize()
    srv = fse.fse_serve_create(hbm_budget_bytes=1 << 30, max_slots=16)
    try:
        tickets = [fse.fse_serve_submit(srv, ti, tm, p, o) for (ti, tm, o, _) in reqs]
        for t in tickets:
            fse.fse_serve_wait(srv, t, 60_000_000)
    finally:
        fse.fse_serve_destroy(srv)
    for (_, _, o, alone) in reqs:
        assert torch.equal(o, alone)

"""The serving loop on the GPU: every result is bitwise the same alone and in
the mix; admission against the HBM budget; error paths."""
import time

import numpy as np
import pytest

from paper_2506_04489_amd import densities as D
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def _wait(sv, tickets, timeout=120.0):
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            done, res, lat = sv.poll(t)
            if done:
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise TimeoutError("requests not done: %d" % len(pending))
        time.sleep(0.001)


def test_served_results_equal_alone():
    import torch
    reqs = D.serving_workload(count=24, rate=1000.0, seed=D.SERVE_SEED)
    sv = B.Server(hbm_budget_bytes=200 << 30, max_slots=16)
    rhos, us, tickets = [], [], []
    for r in reqs:
        td = torch.float64 if r.tier == "f64" else torch.float32
        rho = D.request_density(r, xp=torch, device="cuda").to(td).contiguous()
        torch.cuda.synchronize()
        u = torch.empty_like(rho)
        rhos.append(rho)
        us.append(u)
        tickets.append(sv.submit(r.n, r.h, 40, r.tier, rho, u))
    _wait(sv, tickets)
    lats = []
    for t in tickets:
        done, res, lat = sv.poll(t)
        assert done and res == 0
        lats.append(lat)
    st = sv.stats()
    assert st["completed"] == len(reqs)
    assert st["cache_misses"] >= 1 and st["cache_hits"] >= 1
    print("latency p50 %.2f ms p99 %.2f ms, peak %.2f GB" % (np.percentile(lats, 50), np.percentile(lats, 99),
                                                              st["bytes_peak"] / 2 ** 30))
    sv.close()
    plans = {}
    for r, rho, u in zip(reqs, rhos, us):
        key = (r.n, r.tier)
        if key not in plans:
            plans[key] = B.Plan(r.n, r.h, 40, dtype=r.tier).precompute()
        alone = plans[key].solve(rho)
        torch.cuda.synchronize()
        assert torch.equal(u, alone), key


def test_small_budget_queues_and_completes():
    import torch
    # room for one n = 64 request at a time: the rest wait in the queue
    n, h = 64, 2.0 / 64
    p = B.Plan(n, h, 40)
    one = p.workspace_bytes() + p.spectrum_bytes()
    sv = B.Server(hbm_budget_bytes=int(one * 1.5), max_slots=4)
    rho = D.gaussian(n, h, -1.0, 0.15, xp=torch, device="cuda").contiguous()
    us = [torch.empty_like(rho) for _ in range(6)]
    tickets = [sv.submit(n, h, 40, "f64", rho, u) for u in us]
    _wait(sv, tickets)
    st = sv.stats()
    assert st["bytes_peak"] <= int(one * 1.5)
    ref = p.precompute().solve(rho)
    torch.cuda.synchronize()
    for u in us:
        assert torch.equal(u, ref)
    sv.close()


def test_submit_errors():
    import torch
    sv = B.Server(hbm_budget_bytes=1 << 20, max_slots=2)
    rho = torch.zeros((64,) * 3, dtype=torch.float64, device="cuda")
    u = torch.empty_like(rho)
    with pytest.raises(B.PspError) as ei:
        sv.submit(64, 2 / 64, 40, "f64", rho, u)          # larger than the whole budget
    assert B.STATUS[ei.value.status] == "PSP_ENOMEM"
    with pytest.raises(B.PspError) as ei:
        sv.submit(63, 2 / 63, 40, "f64", rho, u)
    assert B.STATUS[ei.value.status] == "PSP_EUNSUPPORTED"
    with pytest.raises(B.PspError) as ei:
        sv.poll(123456)
    assert B.STATUS[ei.value.status] == "PSP_EINVAL"
    sv.close()


def test_cancel_queued_requests():
    """With room for one n = 64 request at a time, most of a burst waits in
    the queue: those canceled there finish with PSP_ECANCELED and leave u
    untouched; the others (and any already admitted) complete normally."""
    import torch
    n, h = 64, 2.0 / 64
    p = B.Plan(n, h, 40)
    one = p.workspace_bytes() + p.spectrum_bytes()
    sv = B.Server(hbm_budget_bytes=int(one * 1.5), max_slots=1)
    rho = D.gaussian(n, h, -1.0, 0.15, xp=torch, device="cuda").contiguous()
    torch.cuda.synchronize()
    us = [torch.full_like(rho, 7.0) for _ in range(12)]
    torch.cuda.synchronize()
    tickets = [sv.submit(n, h, 40, "f64", rho, u) for u in us]
    canceled = [t for t in tickets[4:] if sv.cancel(t)]
    assert len(canceled) >= 1
    _wait(sv, tickets)
    ref = p.precompute().solve(rho)
    torch.cuda.synchronize()
    for t, u in zip(tickets, us):
        done, res, _ = sv.poll(t)
        assert done
        if t in canceled:
            assert B.STATUS[res] == "PSP_ECANCELED"
            assert torch.all(u == 7.0)
        else:
            assert res == 0
            assert torch.equal(u, ref)
    with pytest.raises(B.PspError):
        sv.cancel(tickets[0])              # finished
    sv.close()


def test_tight_budget_with_cache_misses_stays_within_budget():
    """Room for one spectrum and two workspaces at a time, requests of
    several sizes (every one a spectrum-cache miss on arrival): admission
    evicts idle spectra and pooled workspaces but never holds more than the
    budget, and every request completes with the result of psp_solve."""
    import torch
    sizes = [64, 48, 64, 32, 48, 64, 32]
    big = B.Plan(64, 2.0 / 64, 40)
    budget = big.spectrum_bytes() + 2 * big.workspace_bytes() + (1 << 20)
    sv = B.Server(hbm_budget_bytes=budget, max_slots=4)
    rhos, us, tickets = [], [], []
    for i, n in enumerate(sizes):
        rho = D.gaussian(n, 2.0 / n, -1.0, 0.15, xp=torch, device="cuda").contiguous()
        torch.cuda.synchronize()
        u = torch.empty_like(rho)
        rhos.append(rho)
        us.append(u)
        tickets.append(sv.submit(n, 2.0 / n, 40, "f64", rho, u))
    _wait(sv, tickets)
    st = sv.stats()
    print("budget %d, peak %d, misses %d" % (budget, st["bytes_peak"], st["cache_misses"]))
    assert st["bytes_peak"] <= budget
    assert st["completed"] == len(sizes)
    sv.close()
    for n, rho, u in zip(sizes, rhos, us):
        alone = B.Plan(n, 2.0 / n, 40).precompute().solve(rho)
        torch.cuda.synchronize()
        assert torch.equal(u, alone), n


def test_served_results_match_the_oracle():
    """Served requests of both tiers and density families against the
    oracle's whole-grid solve (n <= 96): FP64 <= 1e-12, FP32 <= 1e-5."""
    import torch
    from oracle import psp_oracle as O
    from tests.gpu_util import rel_max_err
    reqs = [r for r in D.serving_workload(count=200, rate=1000.0, seed=D.SERVE_SEED) if r.n <= 96][:8]
    sv = B.Server(hbm_budget_bytes=64 << 30, max_slots=8)
    items = []
    for r in reqs:
        td = torch.float64 if r.tier == "f64" else torch.float32
        rho64 = D.request_density(r, xp=torch, device="cuda").contiguous()
        rho = rho64.to(td).contiguous()
        torch.cuda.synchronize()
        u = torch.empty_like(rho)
        # rho (the tier's copy) must live until the request is done
        items.append((r, rho64, u, sv.submit(r.n, r.h, 40, r.tier, rho, u), rho))
    _wait(sv, [it[3] for it in items])
    sv.close()
    for r, rho64, u, _, _ in items:
        want = O.solve(rho64.cpu().numpy(), r.h, 40)
        e = rel_max_err(u.double().cpu().numpy(), want)
        print("served n=%d %s %s E_par=%.2e" % (r.n, r.tier, r.kind, e))
        assert e <= (1e-12 if r.tier == "f64" else 1e-5)


def test_small_requests_do_not_wait_behind_large_ones():
    """Large requests (n = 384) and then small ones (n = 64) arrive
    together: the small ones run on the small class's streams, so the first
    of them completes before the last large one."""
    import torch
    sv = B.Server(hbm_budget_bytes=200 << 30, max_slots=32)
    big = [D.gaussian(384, 2.0 / 384, -1.0, 0.15, xp=torch, device="cuda").contiguous() for _ in range(1)]
    small = D.gaussian(64, 2.0 / 64, -1.0, 0.15, xp=torch, device="cuda").contiguous()
    torch.cuda.synchronize()
    # warm both spectra and workspaces
    w = [sv.submit(384, 2.0 / 384, 40, "f64", big[0], torch.empty_like(big[0])),
         sv.submit(64, 2.0 / 64, 40, "f64", small, torch.empty_like(small))]
    _wait(sv, w)
    ub = [torch.empty_like(big[0]) for _ in range(6)]
    us = [torch.empty_like(small) for _ in range(6)]
    tb = [sv.submit(384, 2.0 / 384, 40, "f64", big[0], u) for u in ub]
    ts = [sv.submit(64, 2.0 / 64, 40, "f64", small, u) for u in us]
    _wait(sv, tb + ts)
    lat_b = [sv.poll(t)[2] for t in tb]
    lat_s = [sv.poll(t)[2] for t in ts]
    print("large latencies %s ms, small %s ms" % (["%.2f" % v for v in lat_b], ["%.2f" % v for v in lat_s]))
    assert min(lat_s) < max(lat_b)
    sv.close()

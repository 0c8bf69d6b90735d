"""Continuous-batching server: every request's maps are bitwise those of
pdiv_lcp on the same divergence Gaussians, alone or in a mixed stream; the
HBM budget is never exceeded; failures stay with their own requests."""

import os

import numpy as np
import pytest
import torch

import paper_2510_01190_amd as P
import synth

pytestmark = pytest.mark.gpu

OK, INVALID, DEVICE, BUSY = 0, 1, 4, 5


def _field(ny, nx, seed):
    f = synth.gen_moments(ny, nx, seed, n_features=max(1, ny * nx // 4000))
    return [f[k].astype(np.float32) for k in ("mean_u", "var_u", "mean_v", "var_v")]


def _alone(planes, iso, dx=1.0, dy=1.0):
    ts = [torch.from_numpy(p).cuda() for p in planes]
    dm, dv = P.divergence_gaussian(*ts, dx=dx, dy=dy)
    return P.lcp(dm, dv, iso)


def test_results_equal_alone_in_a_mixed_stream():
    rng = np.random.default_rng(1)
    srv = P.Server(hbm_budget=4 << 30, n_streams=3)
    sizes = [(2, 2), (64, 80), (300, 257), (513, 700), (40, 1000)]
    fields = {}
    tickets = []
    for fid, (ny, nx) in enumerate(sizes):
        planes = _field(ny, nx, 100 + fid)
        fields[fid] = planes
        tickets.append(("new", fid, srv.put_field(fid, *planes, dx=1.0 + 0.25 * fid)))
    reqs = []
    for r in range(120):  # submitted without waiting: they queue behind the uploads
        fid = int(rng.integers(0, len(sizes)))
        k = int(rng.integers(1, 17))
        iso = rng.uniform(-0.1, 0.1, k).astype(np.float32)
        ny, nx = sizes[fid]
        out = torch.empty((k, ny - 1, nx - 1), device="cuda")
        reqs.append((fid, iso, out, srv.submit_lcp(fid, iso, out)))
    for _, _, t in tickets:
        assert srv.wait(t) == OK
    for fid, iso, out, t in reqs:
        assert srv.wait(t) == OK
    torch.cuda.synchronize()
    for fid, iso, out, t in reqs:
        assert torch.equal(out, _alone(fields[fid], iso, dx=1.0 + 0.25 * fid))
    st = srv.stats()
    assert st["done"] == len(reqs) + len(sizes) and st["failed"] == 0
    assert st["launches"] >= 1 and st["launches"] <= len(reqs)
    assert st["p99_us"] >= st["p50_us"] > 0
    assert st["peak_bytes"] <= 4 << 30
    srv.close()


def test_budget_is_never_exceeded_and_lru_evicts():
    planes = [_field(512, 512, 200 + i) for i in range(6)]
    n = 512 * 512
    slots = 2 * 2 * 512 * (128 + 16 * 4)  # descriptor slots of a 2-stream server
    budget = slots + 2 * 8 * n + 16 * n + (1 << 20)  # two resident fields + one upload
    srv = P.Server(hbm_budget=budget, n_streams=2)
    iso = np.array([0.0, 0.02], np.float32)
    for fid, pl in enumerate(planes):
        assert srv.wait(srv.put_field(fid, *pl)) == OK
        out = torch.empty((2, 511, 511), device="cuda")
        assert srv.wait(srv.submit_lcp(fid, iso, out)) == OK
        torch.cuda.synchronize()
        assert torch.equal(out, _alone(pl, iso))
    st = srv.stats()
    assert st["peak_bytes"] <= budget
    with pytest.raises(P.PdivError) as e:  # the oldest field has been evicted
        srv.submit_lcp(0, iso, torch.empty((2, 511, 511), device="cuda"))
    assert e.value.status == INVALID
    srv.close()


def test_field_that_can_never_fit_is_refused():
    srv = P.Server(hbm_budget=64 << 20, n_streams=1)
    pl = _field(2048, 2048, 3)
    with pytest.raises(P.PdivError) as e:
        srv.put_field(7, *pl)
    assert e.value.status == BUSY
    srv.close()


def test_invalid_requests():
    srv = P.Server(hbm_budget=1 << 30, n_streams=1)
    out = torch.empty((1, 3, 3), device="cuda")
    with pytest.raises(P.PdivError) as e:
        srv.submit_lcp(99, [0.0], out)
    assert e.value.status == INVALID
    pl = _field(4, 4, 4)
    assert srv.wait(srv.put_field(1, *pl)) == OK
    with pytest.raises(P.PdivError):
        srv.put_field(1, *pl)  # id in use
    with pytest.raises(P.PdivError):
        srv.submit_lcp(1, np.zeros(17, np.float32), out)
    with pytest.raises(P.PdivError):
        srv.wait(123456)
    srv.close()


def test_forced_launch_failure_stays_with_its_requests(monkeypatch):
    # the second slider launch is refused on the host before anything is
    # enqueued; only the requests of that launch fail
    monkeypatch.setenv("PDIV_FAULT", "server_launch:2")
    srv = P.Server(hbm_budget=1 << 30, n_streams=1)
    monkeypatch.delenv("PDIV_FAULT")
    pl = _field(100, 120, 5)
    assert srv.wait(srv.put_field(1, *pl)) == OK
    iso = np.array([0.01], np.float32)
    results = []
    for r in range(3):
        out = torch.empty((1, 99, 119), device="cuda")
        results.append((srv.wait(srv.submit_lcp(1, iso, out)), out))
    assert [s for s, _ in results] == [OK, DEVICE, OK]
    torch.cuda.synchronize()
    assert torch.equal(results[2][1], _alone(pl, iso))
    st = srv.stats()
    assert st["failed"] == 1
    srv.close()


def test_reserved_staging_pool_is_reused_under_back_pressure():
    # Two staging buffers for eight 1024x1024 fields submitted back to back:
    # put_field must wait for uploads to hand buffers back (the copies run on
    # several threads at this size), and every field still comes out right.
    srv = P.Server(hbm_budget=2 << 30, n_streams=2)
    srv.reserve_staging(1024 * 1024, 2)
    planes = [_field(1024, 1024, 300 + i) for i in range(8)]
    tickets = [srv.put_field(fid, *pl) for fid, pl in enumerate(planes)]
    for t in tickets:
        assert srv.wait(t) == OK
    iso = np.array([-0.01, 0.0, 0.015], np.float32)
    for fid, pl in enumerate(planes):
        out = torch.empty((3, 1023, 1023), device="cuda")
        assert srv.wait(srv.submit_lcp(fid, iso, out)) == OK
        torch.cuda.synchronize()
        assert torch.equal(out, _alone(pl, iso))
    srv.close()

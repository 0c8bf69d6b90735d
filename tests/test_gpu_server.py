"""Continuous-batching server: every request's maps are bitwise those of
pdiv_lcp on the same divergence Gaussians, alone or in a mixed stream, and
within 1e-5 of the FP64 oracle of Eq. 2-3 and the closed-form LCP on the
stored host planes; the HBM budget is never exceeded; failures stay with
their own requests."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth

pytestmark = pytest.mark.gpu

OK, INVALID, DEVICE, BUSY = 0, 1, 4, 5
TOL = 1e-5  # float32 storage: LCP max abs error against the FP64 oracle


def _field(ny, nx, seed):
    f = synth.gen_moments(ny, nx, seed, n_features=max(1, ny * nx // 4000))
    return [f[k].astype(np.float32) for k in ("mean_u", "var_u", "mean_v", "var_v")]


def _alone(planes, iso, dx=1.0, dy=1.0):
    ts = [torch.from_numpy(p).cuda() for p in planes]
    dm, dv = P.divergence_gaussian(*ts, dx=dx, dy=dy)
    return P.lcp(dm, dv, iso)


class _Oracle:
    """FP64 oracle maps of a field's stored host planes (its divergence
    Gaussians computed once per field)."""

    def __init__(self):
        self.div = {}

    def __call__(self, key, planes, iso, dx=1.0, dy=1.0):
        if key not in self.div:
            self.div[key] = O.divergence_gaussian(*[np.asarray(p, np.float64) for p in planes],
                                                  dx, dy)
        return O.lcp(*self.div[key], np.asarray(iso, np.float32))


def _check_oracle(out, ref):
    err = float(np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref))) if ref.size else 0.0
    assert err <= TOL, err


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
    orc = _Oracle()
    for fid, iso, out, t in reqs:
        assert torch.equal(out, _alone(fields[fid], iso, dx=1.0 + 0.25 * fid))
        _check_oracle(out, orc(fid, fields[fid], iso, dx=1.0 + 0.25 * fid))
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
    orc = _Oracle()
    for fid, pl in enumerate(planes):
        assert srv.wait(srv.put_field(fid, *pl)) == OK
        out = torch.empty((2, 511, 511), device="cuda")
        assert srv.wait(srv.submit_lcp(fid, iso, out)) == OK
        torch.cuda.synchronize()
        assert torch.equal(out, _alone(pl, iso))
        _check_oracle(out, orc(fid, pl, iso))
    # a field evicted and put again comes back with the same maps
    assert srv.wait(srv.put_field(100, *planes[0])) == OK
    out = torch.empty((2, 511, 511), device="cuda")
    assert srv.wait(srv.submit_lcp(100, iso, out)) == OK
    torch.cuda.synchronize()
    _check_oracle(out, orc(0, planes[0], iso))
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
    with pytest.raises(P.PdivError):  # 17 isovalues: more than a slider request takes
        srv.submit_lcp(1, np.zeros(17, np.float32), torch.empty((17, 3, 3), device="cuda"))
    with pytest.raises(P.PdivError):
        srv.wait(123456)
    srv.close()


def test_binding_rejects_outputs_and_planes_that_do_not_match():
    """The C call takes no size for out; the binding checks it against the
    field's grid, and put_field checks that the four planes agree."""
    srv = P.Server(hbm_budget=1 << 30, n_streams=1)
    pl = _field(6, 9, 8)
    assert srv.wait(srv.put_field(3, *pl)) == OK
    iso = [0.0, 0.01]
    for bad in (torch.empty((2, 5, 7), device="cuda"),              # wrong shape
                torch.empty((1, 5, 8), device="cuda"),              # wrong isovalue count
                torch.empty((2, 5, 8), device="cuda", dtype=torch.float16),
                torch.empty((2, 5, 8)),                             # host tensor
                torch.empty((2, 5, 16), device="cuda")[:, :, :8]):  # padded view
        with pytest.raises(ValueError):
            srv.submit_lcp(3, iso, bad)
    with pytest.raises(ValueError):
        srv.put_field(4, pl[0], pl[1], pl[2][:, :8], pl[3])
    with pytest.raises(ValueError):
        srv.put_field(4, pl[0], pl[1].astype(np.float16), pl[2], pl[3])
    with pytest.raises(ValueError):
        srv.put_field(4, *[torch.from_numpy(p).cuda() for p in pl])
    out = torch.empty((2, 5, 8), device="cuda")
    assert srv.wait(srv.submit_lcp(3, iso, out)) == OK
    torch.cuda.synchronize()
    _check_oracle(out, _Oracle()(3, pl, iso))
    srv.close()


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_16bit_host_planes_match_the_oracle_on_the_stored_values(dt):
    """put_field from 16-bit host planes: the upload, Eq. 2-3 and the slider
    LCP against the FP64 oracle on the 16-bit values as stored (float16 from
    numpy, bfloat16 as a torch CPU tensor)."""
    srv = P.Server(hbm_budget=1 << 30, n_streams=2)
    pl = _field(257, 301, 21)
    if dt == "f16":
        host = [p.astype(np.float16) for p in pl]
        stored = [h.astype(np.float64) for h in host]
    else:
        host = [torch.from_numpy(p).to(torch.bfloat16) for p in pl]
        stored = [h.float().numpy().astype(np.float64) for h in host]
    assert srv.wait(srv.put_field(9, *host, dx=0.5, dy=2.0)) == OK
    iso = np.array([-0.02, 0.0, 0.01, 0.05], np.float32)
    out = torch.empty((4, 256, 300), device="cuda")
    assert srv.wait(srv.submit_lcp(9, iso, out)) == OK
    torch.cuda.synchronize()
    _check_oracle(out, _Oracle()(9, stored, iso, dx=0.5, dy=2.0))
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
    _check_oracle(results[0][1], _Oracle()(1, pl, iso))
    st = srv.stats()
    assert st["failed"] == 1
    srv.close()


def test_forced_upload_failure_stays_with_its_field(monkeypatch):
    # the second new field's upload is refused on the host before anything is
    # allocated or enqueued: that put_field and the sliders on its field fail,
    # the other fields and their sliders are served and correct
    monkeypatch.setenv("PDIV_FAULT", "server_launch:0,server_upload:2")
    srv = P.Server(hbm_budget=1 << 30, n_streams=2)
    monkeypatch.delenv("PDIV_FAULT")
    planes = [_field(90, 110, 30 + i) for i in range(3)]
    puts = [srv.put_field(i, *planes[i]) for i in range(3)]
    assert [srv.wait(t) for t in puts] == [OK, DEVICE, OK]
    iso = np.array([-0.01, 0.02], np.float32)
    outs = [torch.empty((2, 89, 109), device="cuda") for _ in range(3)]
    status = [srv.wait(srv.submit_lcp(i, iso, outs[i])) for i in range(3)]
    assert status == [OK, DEVICE, OK]
    torch.cuda.synchronize()
    orc = _Oracle()
    for i in (0, 2):
        _check_oracle(outs[i], orc(i, planes[i], iso))
    st = srv.stats()
    assert st["failed"] == 2 and st["peak_bytes"] <= 1 << 30
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
    orc = _Oracle()
    for fid, pl in enumerate(planes):
        out = torch.empty((3, 1023, 1023), device="cuda")
        assert srv.wait(srv.submit_lcp(fid, iso, out)) == OK
        torch.cuda.synchronize()
        assert torch.equal(out, _alone(pl, iso))
        _check_oracle(out, orc(fid, pl, iso))
    srv.close()

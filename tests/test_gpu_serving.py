"""Continuous-batching server on the GPU: every request's results in a mix of
concurrent requests equal, bit for bit, the same request served alone and
the same points evaluated by the request's session (the server and every
evaluation path split the elements into the same segments and add them in
the same order); served values agree with the oracle's evaluation (Eqs.
Potential/Field) on sampled points; admission by HBM budget queues what does
not fit, oversized requests are refused."""
import numpy as np
import pytest

import oracle
from synth import gem_cell, parallel_plates, serve_requests, uniform_points

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def nb():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2606_24154_amd as nb
    return nb


def _geometries():
    # plates: one element segment; the small GEM cell with +-10 copies:
    # 688 elements x 441 copies, three segments of ~1e5 interactions per point
    return [parallel_plates(),
            gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2),
            gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=10)]


def _sessions(nb, precision, geoms):
    return [nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=precision) for g in geoms]


def _alone(nb, ses, pts):
    cols = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(DEV) for k in range(3)]
    out = ses.eval_points(*cols)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _rel_errors(got, ref):
    """pointwise relative errors of phi and |E| on points whose reference
    magnitude is at least 1e-3 of the sample's largest"""
    ap = np.abs(ref[:, 0])
    sel = ap >= 1e-3 * ap.max()
    ephi = np.max(np.abs(got[sel, 0] - ref[sel, 0]) / ap[sel])
    en = np.linalg.norm(ref[:, 1:], axis=1)
    sel = en >= 1e-3 * en.max()
    eE = np.max(np.linalg.norm(got[sel, 1:] - ref[sel, 1:], axis=1) / en[sel])
    return ephi, eE


@pytest.mark.parametrize("precision", [0, 1])
def test_mix_equals_alone_and_admission(nb, precision):
    from paper_2606_24154_amd.serving import replay
    geoms = _geometries()
    ses = _sessions(nb, precision, geoms)
    # tight budget: only a few mid-size requests fit at once (the 3-segment
    # geometry needs 8 + 4 x 3 doubles per point)
    srv = nb.Server(ses, hbm_budget=(8 + 4 * 3) * 8 * 12000, batch_interactions=2e8)
    reqs = serve_requests(40, rate_hz=400.0, n_geometries=3, seed=9, n_min=64, n_max=8000)
    # one request on the multi-segment geometry above the sorting threshold
    reqs[5] = (reqs[5][0], 2, 6000, reqs[5][3])
    assert sum(1 for r in reqs if r[1] == 2) >= 5

    def make_points(g, n, sd):
        return uniform_points(geoms[g].box_lo, geoms[g].box_hi, n, sd)

    run = replay(srv, reqs, make_points)
    assert not run["errors"]
    c = srv.counters()
    assert c.points_done == sum(r[2] for r in reqs) and c.launches >= 2
    checked = 0
    sigmas = [x.sigma().cpu().numpy() for x in ses]
    # the same requests one at a time through the same server, and through
    # the request's session
    for k, (_, g, n, sd) in enumerate(reqs):
        t = srv.submit(g, run["points_in"][k])
        alone, _ = srv.wait(t)
        out = run["results"][k]
        ref = _alone(nb, ses[g], run["points_in"][k])
        for name, r in zip(("phi", "ex", "ey", "ez"), ref):
            assert np.array_equal(out[name], alone[name]), (k, name)
            assert np.array_equal(out[name], r), (k, name, "session")
        # every request's served values against the oracle with the
        # session's sigma, on 8 sampled points (FP64 bar / mixed bar)
        checked += 1
        pts = run["points_in"][k]
        idx = np.random.default_rng(k).choice(len(pts), min(8, len(pts)), replace=False)
        want = oracle.eval_points(geoms[g], sigmas[g], pts[idx])
        got = np.column_stack([out[name][idx] for name in ("phi", "ex", "ey", "ez")])
        ephi, eE = _rel_errors(got, want)
        tol = 1e-10 if precision == 0 else 1e-6
        assert ephi < tol and eE < tol, (k, g, ephi, eE)
    assert checked == len(reqs)
    assert run["p99_s"] >= run["p50_s"] > 0
    srv.close()
    for x in ses:
        x.close()


def test_oversized_request_refused(nb):
    geoms = _geometries()[:1]
    ses = _sessions(nb, 0, geoms)
    srv = nb.Server(ses, hbm_budget=(8 + 4) * 8 * 1000)  # plates: one element segment
    with pytest.raises(nb.NebemError) as e:
        srv.submit(0, uniform_points(geoms[0].box_lo, geoms[0].box_hi, 2000, 1))
    assert e.value.code == nb.NEBEM_EBUSY
    t = srv.submit(0, uniform_points(geoms[0].box_lo, geoms[0].box_hi, 900, 2))
    out, st = srv.wait(t)
    assert st.points == 900 and np.all(np.isfinite(out["phi"]))
    srv.close()
    for x in ses:
        x.close()


def test_small_request_passes_blocked_head(nb):
    """A large request that does not fit beside an active one blocks the head
    of the line; a small request submitted after it is admitted past it and
    finishes first, with results still bit-equal to the session's."""
    geoms = _geometries()
    ses = _sessions(nb, 0, [geoms[0], geoms[2]])
    per_pt = (8 + 4 * 3) * 8  # the three-segment geometry's staging per point
    # one launch = one round of work items, so the first request (12 288
    # items) stays active over several launches
    srv = nb.Server(ses, hbm_budget=per_pt * 300000, batch_interactions=1.0)
    big = uniform_points(geoms[2].box_lo, geoms[2].box_hi, 262144, 31)
    blocked = uniform_points(geoms[2].box_lo, geoms[2].box_hi, 65536, 32)
    small = uniform_points(geoms[0].box_lo, geoms[0].box_hi, 200, 33)
    ta = srv.submit(1, big)
    tb = srv.submit(1, blocked)
    tc = srv.submit(0, small)
    out_c, st_c = srv.wait(tc)
    out_b, st_b = srv.wait(tb)
    out_a, st_a = srv.wait(ta)
    assert srv.counters().backfilled >= 1
    assert st_c.t_admit < st_b.t_admit and st_c.t_done < st_b.t_admit
    assert st_b.t_admit >= st_a.t_done - 1e-3
    for out, g, pts in ((out_c, 0, small), (out_b, 1, blocked)):
        ref = _alone(nb, ses[g], pts)
        for name, r in zip(("phi", "ex", "ey", "ez"), ref):
            assert np.array_equal(out[name], r), (g, name)
    srv.close()
    for x in ses:
        x.close()


def test_large_request_cap(nb):
    """With at most one large request active, a second large one waits at
    the head of the line until the first finishes while a small one passes
    it; results bit-equal to the session's."""
    geoms = _geometries()
    ses = _sessions(nb, 0, [geoms[0], geoms[2]])
    srv = nb.Server(ses, batch_interactions=1.0, large_interactions=1e9, max_large=1)
    big = uniform_points(geoms[2].box_lo, geoms[2].box_hi, 262144, 41)
    big2 = uniform_points(geoms[2].box_lo, geoms[2].box_hi, 20000, 42)
    small = uniform_points(geoms[0].box_lo, geoms[0].box_hi, 300, 43)
    # 688 x 441 interactions per point: both GEM requests are large, the
    # plates one (512 per point) is not
    ta = srv.submit(1, big)
    tb = srv.submit(1, big2)
    tc = srv.submit(0, small)
    out_c, st_c = srv.wait(tc)
    out_b, st_b = srv.wait(tb)
    out_a, st_a = srv.wait(ta)
    assert st_b.t_admit >= st_a.t_done - 1e-3
    assert st_c.t_done < st_a.t_done
    for out, g, pts in ((out_a, 1, big), (out_b, 1, big2), (out_c, 0, small)):
        ref = _alone(nb, ses[g], pts)
        for name, r in zip(("phi", "ex", "ey", "ez"), ref):
            assert np.array_equal(out[name], r), (g, name)
    srv.close()
    for x in ses:
        x.close()

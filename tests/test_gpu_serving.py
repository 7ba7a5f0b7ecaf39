"""Continuous-batching server on the GPU: every request's results in a mix of
concurrent requests equal, bit for bit, the same request served alone;
they agree with a plain session evaluation to rounding (the server sums the
elements in fixed segments); admission by HBM budget queues what does not
fit, oversized requests are refused."""
import numpy as np
import pytest

from synth import gem_cell, parallel_plates, serve_requests, uniform_points

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def nb():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2606_24154_amd as nb
    return nb


def _sessions(nb, precision):
    geoms = [parallel_plates(), gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)]
    ses = [nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=precision) for g in geoms]
    return geoms, ses


def _alone(nb, ses, pts):
    cols = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(DEV) for k in range(3)]
    out = ses.eval_points(*cols)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("precision", [0, 1])
def test_mix_equals_alone_and_admission(nb, precision):
    from paper_2606_24154_amd.serving import replay
    geoms, ses = _sessions(nb, precision)
    # tight budget: only a few mid-size requests fit at once
    srv = nb.Server(ses, hbm_budget=(8 + 4 * 2) * 8 * 12000, batch_interactions=2e8)
    reqs = serve_requests(40, rate_hz=400.0, n_geometries=2, seed=9, n_min=64, n_max=8000)

    def make_points(g, n, sd):
        return uniform_points(geoms[g].box_lo, geoms[g].box_hi, n, sd)

    run = replay(srv, reqs, make_points)
    assert not run["errors"]
    c = srv.counters()
    assert c.points_done == sum(r[2] for r in reqs) and c.launches >= 2
    # the same requests one at a time through the same server
    for k, (_, g, n, sd) in enumerate(reqs):
        t = srv.submit(g, run["points_in"][k])
        alone, _ = srv.wait(t)
        out = run["results"][k]
        for name in ("phi", "ex", "ey", "ez"):
            assert np.array_equal(out[name], alone[name]), (k, name)
        ref = _alone(nb, ses[g], run["points_in"][k])
        for name, r in zip(("phi", "ex", "ey", "ez"), ref):
            scale = np.abs(r).max()
            assert np.max(np.abs(out[name] - r)) <= 1e-11 * scale, (k, name)
    assert run["p99_s"] >= run["p50_s"] > 0
    srv.close()


def test_oversized_request_refused(nb):
    geoms, ses = _sessions(nb, 0)
    srv = nb.Server(ses, hbm_budget=(8 + 4) * 8 * 1000)  # plates: one element segment
    with pytest.raises(nb.NebemError) as e:
        srv.submit(0, uniform_points(geoms[0].box_lo, geoms[0].box_hi, 2000, 1))
    assert e.value.code == nb.NEBEM_EBUSY
    t = srv.submit(0, uniform_points(geoms[0].box_lo, geoms[0].box_hi, 900, 2))
    out, st = srv.wait(t)
    assert st.points == 900 and np.all(np.isfinite(out["phi"]))
    srv.close()

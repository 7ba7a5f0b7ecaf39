"""The allocation-free session evaluation (nebem_session_eval_noalloc)
against nebem_session_eval, through the C-ABI: bit-for-bit equal results on
two calls in a row, the first large enough to be taken in several chunks of
the fixed scratch, the second smaller; device memory use unchanged by the
calls; argument errors."""
import ctypes

import numpy as np
import pytest

from synth import gem_cell, uniform_points

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def nb():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2606_24154_amd as nb
    return nb


def _cols(pts):
    return [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(DEV) for k in range(3)]


def _call(nb, fn, ses, pts, out):
    px, py, pz = _cols(pts)
    stream = torch.cuda.current_stream().cuda_stream
    code = fn(ses.handle, px.data_ptr(), py.data_ptr(), pz.data_ptr(), len(pts), *(t.data_ptr() for t in out),
              ctypes.c_void_p(stream))
    torch.cuda.synchronize()
    return code


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_session_eval(nb, precision):
    # 688 elements x 441 copies: three element segments; 600 000 points need
    # about 100 MB of workspace, so the 64 MiB scratch takes them in chunks
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=10)
    ses = nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=precision)
    # the library's scratch is device memory of its own, held from its first
    # use; a first call loads it
    warm = uniform_points(g.box_lo, g.box_hi, 64, 9)
    assert _call(nb, nb.lib.nebem_session_eval_noalloc, ses, warm,
                 [torch.empty(64, dtype=torch.float64, device=DEV) for _ in range(4)]) == nb.NEBEM_OK
    for m, seed in ((600_000, 1), (5_000, 2)):
        pts = uniform_points(g.box_lo, g.box_hi, m, seed)
        ref = [torch.empty(m, dtype=torch.float64, device=DEV) for _ in range(4)]
        got = [torch.full((m,), np.nan, dtype=torch.float64, device=DEV) for _ in range(4)]
        assert _call(nb, nb.lib.nebem_session_eval, ses, pts, ref) == nb.NEBEM_OK
        torch.cuda.synchronize()
        before = torch.cuda.mem_get_info()[0]
        assert _call(nb, nb.lib.nebem_session_eval_noalloc, ses, pts, got) == nb.NEBEM_OK
        assert torch.cuda.mem_get_info()[0] == before
        for a, b in zip(got, ref):
            assert torch.equal(a, b), m
    # a component left out is not written
    pts = uniform_points(g.box_lo, g.box_hi, 300, 3)
    px, py, pz = _cols(pts)
    phi = torch.full((300,), 7.0, dtype=torch.float64, device=DEV)
    ex = torch.empty(300, dtype=torch.float64, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert nb.lib.nebem_session_eval_noalloc(ses.handle, px.data_ptr(), py.data_ptr(), pz.data_ptr(), 300, None,
                                             ex.data_ptr(), None, None, stream) == nb.NEBEM_OK
    torch.cuda.synchronize()
    assert torch.all(phi == 7.0) and torch.isfinite(ex).all()
    ses.close()


def test_noalloc_argument_errors(nb):
    assert nb.lib.nebem_session_eval_noalloc(None, None, None, None, 10, None, None, None, None,
                                             None) == nb.NEBEM_EINVAL
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)
    ses = nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=0)
    assert nb.lib.nebem_session_eval_noalloc(ses.handle, None, None, None, -1, None, None, None, None,
                                             None) == nb.NEBEM_EINVAL
    assert nb.lib.nebem_session_eval_noalloc(ses.handle, None, None, None, 10, None, None, None, None,
                                             None) == nb.NEBEM_EINVAL
    assert nb.lib.nebem_session_eval_noalloc(ses.handle, None, None, None, 0, None, None, None, None,
                                             None) == nb.NEBEM_OK
    ses.close()

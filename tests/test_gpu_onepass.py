"""The single-pass sketch sweep (Remark 4.2) through the C ABI: Omega bit-exact with the
oracle's generator, G and H against the oracle's products G = A Omega, H = A^T G within the
bounds of the two-pass sweep (FP64 dot products of length n and m), and against the library's
two-pass sweep; the panel sum of H has a fixed order, so repeated calls agree bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rng as ORNG

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 5


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("m,n,l,col0,panel", [
    (1000, 800, 200, 0, 128),     # 8 panels, ragged tiles
    (1000, 800, 200, 3, 333),     # ragged last panel, odd Omega offset
    (4097, 33, 16, 0, 1000),      # tall and narrow, 5 panels
    (257, 129, 33, 5, 0),         # default panel height: one panel
])
def test_onepass_vs_oracle(qb, m, n, l, col0, panel):
    _log(f"onepass {m}x{n} l={l} col0={col0} panel={panel}")
    A = W.gaussian_dense(m, n, 9)
    om, g, h = qb.qb_sketch_onepass(A.cuda(), SEED, col0, l, panel_rows=panel)
    An = A.numpy()
    Om = ORNG.gaussian_matrix(SEED, n, l, 0, col0)
    assert np.array_equal(om.cpu().numpy().view(np.int64), Om.view(np.int64))
    Gr = An @ Om
    Hr = An.T @ Gr
    gg, hh = g.cpu().numpy(), h.cpu().numpy()
    assert np.max(np.abs(gg - Gr)) <= 1e-13 * np.sqrt(n) * np.max(np.abs(An)) * np.max(np.abs(Om)) * 4
    assert np.linalg.norm(gg - Gr) <= 1e-14 * np.linalg.norm(Gr) * np.sqrt(n)
    assert np.linalg.norm(hh - Hr) <= 1e-14 * np.linalg.norm(Hr) * np.sqrt(m * n) + 1e-300
    om2, g2, h2 = qb.qb_sketch_onepass(A.cuda(), SEED, col0, l, panel_rows=panel)
    assert torch.equal(g, g2) and torch.equal(h, h2)


def test_onepass_full_size_matches_two_pass(qb):
    """The 20000 x 15000 workload at the headline's chunk width, default panels."""
    A = W.C2.make(device="cuda")
    om1, g1, h1 = qb.qb_sketch_dense(A, SEED, 0, 1024)
    om2, g2, h2 = qb.qb_sketch_onepass(A, SEED, 0, 1024)
    assert torch.equal(om1, om2)
    dg = (torch.linalg.matrix_norm(g1 - g2) / torch.linalg.matrix_norm(g1)).item()
    dh = (torch.linalg.matrix_norm(h1 - h2) / torch.linalg.matrix_norm(h1)).item()
    _log(f"onepass full size: rel |dG| {dg:.3e} rel |dH| {dh:.3e}")
    assert dg <= 1e-13 and dh <= 1e-13


def test_onepass_rejections(qb):
    A = W.gaussian_dense(50, 40, 1).cuda()
    with pytest.raises(qb.QBError):
        qb.qb_sketch_onepass(A, SEED, 0, 0)
    with pytest.raises(qb.QBError):
        qb.qb_sketch_onepass(A, SEED, 0, 8, panel_rows=-1)
    with pytest.raises(ValueError):
        qb.qb_sketch_onepass(A.float(), SEED, 0, 8)

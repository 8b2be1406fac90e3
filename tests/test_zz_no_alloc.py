"""The allocation-free entry point qb_fp_dense_noalloc against qb_fp_dense (the same
randQB_FP, Algorithm 4, with a caller-owned workspace), through the C ABI.

Two calls in a row on the library's static scratch array, the second on a smaller matrix
(so that stale contents of the larger call sit in the array), each compared with the
workspace entry point on the same input to the FP64 parity bar: same rank, status, passes
and chunks; |E - E_ref| <= 1e-10 ||A||^2; ||B - B_ref||_F <= 1e-10 ||A||_F;
max |Q - Q_ref| <= 1e-10.  (The scratch layout may give the block products fewer K splits,
so the two agree to rounding, not bit for bit.)"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _compare(r, ref):
    assert r.rank == ref.rank and r.status == ref.status
    assert r.passes == ref.passes and r.chunks == ref.chunks and r.blocks == ref.blocks
    assert abs(r.E - ref.E) <= 1e-10 * ref.normA2
    assert r.normA2 == ref.normA2
    nb = float(torch.linalg.matrix_norm(r.B - ref.B))
    assert nb <= 1e-10 * ref.normA2 ** 0.5, nb
    assert float((r.Q - ref.Q).abs().max()) <= 1e-10


@pytest.mark.parametrize("l_tilde", [0, -1])
def test_noalloc_two_calls_match_workspace_entry(qb, l_tilde):
    dev = torch.device("cuda:0")
    seed = W.SEED_OMEGA | 21
    cases = [(1000, 800, 20, 1e-2, "poly2"), (600, 400, 16, 1e-2, "exp20")]
    for m, n, b, tol, law in cases:
        print(f"noalloc {m}x{n} b={b} tol={tol} law={law} l_tilde={l_tilde}", flush=True)
        A = W.lowrank_dense(m, n, W.sigma_law(law, min(m, n)), 31).to(dev)
        r = qb.qb_fp_dense_noalloc(A, tol, b, seed, l_tilde=l_tilde)
        torch.cuda.synchronize()
        ref = qb.qb_fp_dense(A, tol, b, seed, l_tilde=l_tilde)
        torch.cuda.synchronize()
        _compare(r, ref)
        assert r.rank > 0 and r.status == qb.QB_OK
        # every phase timer stays zero: the call records no events
        assert all(t == 0.0 for t in r.ms)


def test_noalloc_rejects_a_problem_beyond_the_scratch(qb):
    A = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda:0")
    with pytest.raises(qb.QBError) as e:
        qb.qb_fp_dense_noalloc(A, 1e-2, 64, 1)
    assert e.value.status == qb.QB_ERR_WORKSPACE

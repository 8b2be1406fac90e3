"""GPU tests of the COO input path: the library's COO -> CSR conversion and randQB_FP /
randQB_EI on COO triplets, through the C ABI.

The triplets come from the seeded power-law CSR generator, shuffled by a seeded
permutation, with some entries split into two halves at the same (row, col) (exactly
representable parts, so every summation order gives the same value).  The conversion is
index work and is compared bit for bit with SciPy's COO -> CSR (sorted columns, duplicates
summed); the method is compared with the oracle on SciPy's CSR, to the FP64 path's
tolerances, and with the library's own CSR path on the original arrays (identical CSR
arrays, so identical results)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import randqb as R
from test_gpu_parity import _compare

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 8


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


def _triplets(csr, split_every=7, seed=81):
    """Shuffled COO triplets of csr with every split_every-th entry split in two halves."""
    S = csr.to_scipy().tocoo()
    row, col, val = S.row.astype(np.int32), S.col.astype(np.int32), S.data.astype(np.float64)
    sel = np.arange(0, len(val), split_every)
    half = val[sel] * 0.5
    val = val.copy()
    val[sel] = half
    row = np.concatenate([row, row[sel]])
    col = np.concatenate([col, col[sel]])
    val = np.concatenate([val, half])
    perm = np.random.default_rng(seed).permutation(len(val))
    return row[perm], col[perm], val[perm]


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def test_coo_to_csr_bit_exact(qb):
    csr = W.powerlaw_csr(3000, 1200, 30000, 82)
    row, col, val = _triplets(csr)
    rp, ci, va = qb.coo_to_csr(csr.m, csr.n, *_dev(row, col, val))
    ref = sp.coo_matrix((val, (row, col)), shape=(csr.m, csr.n)).tocsr()
    ref.sort_indices()
    _log(f"coo -> csr: {len(val)} triplets -> {ref.nnz} entries")
    assert np.array_equal(rp.cpu().numpy(), ref.indptr.astype(np.int64))
    assert np.array_equal(ci.cpu().numpy(), ref.indices.astype(np.int32))
    assert np.array_equal(va.cpu().numpy().view(np.int64), ref.data.view(np.int64))
    # the generator's own CSR is the same matrix
    assert np.array_equal(rp.cpu().numpy(), csr.rowptr) and np.array_equal(ci.cpu().numpy(), csr.colind)


def test_coo_edge_cases(qb):
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    rp, ci, va = qb.coo_to_csr(5, 4, e32, e32, torch.empty(0, dtype=torch.float64, device="cuda"))
    assert rp.cpu().tolist() == [0] * 6 and ci.numel() == 0
    r, c, v = _dev(np.array([0, 4, 4, 4], np.int32), np.array([3, 0, 0, 1], np.int32),
                   np.array([1.0, 2.0, 3.0, 4.0]))
    rp, ci, va = qb.coo_to_csr(5, 4, r, c, v)
    assert rp.cpu().tolist() == [0, 1, 1, 1, 1, 3]
    assert ci.cpu().tolist() == [3, 0, 1] and va.cpu().tolist() == [1.0, 5.0, 4.0]
    bad_r, bad_c, bad_v = _dev(np.array([0, 5], np.int32), np.array([0, 0], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(qb.QBError) as e:
        qb.coo_to_csr(5, 4, bad_r, bad_c, bad_v)
    assert e.value.status == qb.QB_ERR_ARG
    with pytest.raises(qb.QBError) as e:
        qb.qb_fp_coo(5, 4, bad_r, bad_c, bad_v, 0.5, 2, SEED)
    assert e.value.status == qb.QB_ERR_ARG


@pytest.mark.parametrize("algo,power", [("fp", 0), ("fp", 1), ("ei", 0)])
def test_coo_method_parity(qb, algo, power):
    wl = W.C3_SMALL
    csr = wl.make()
    row, col, val = _triplets(csr, split_every=5, seed=83)
    r, c, v = _dev(row, col, val)
    S = sp.coo_matrix((val, (row, col)), shape=(csr.m, csr.n)).tocsr()
    _log(f"coo {algo} P={power} {wl.name}")
    rp, ci, va = _dev(csr.rowptr, csr.colind, csr.val)
    if algo == "fp":
        res = qb.qb_fp_coo(csr.m, csr.n, r, c, v, wl.tol, wl.b, SEED, power=power)
        ora = R.randqb_fp(S, wl.tol, wl.b, SEED, power=power)
        via_csr = qb.qb_fp_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, SEED, power=power)
    else:
        res = qb.qb_ei_coo(csr.m, csr.n, r, c, v, wl.tol, wl.b, SEED)
        ora = R.randqb_ei(S, wl.tol, wl.b, SEED)
        via_csr = qb.qb_ei_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, SEED)
    _log(f"  conversion {res.ms[7]:.2f} ms")
    _compare(res, ora, S, f"coo {algo}")
    assert res.rank == via_csr.rank and res.E == via_csr.E
    assert torch.equal(res.Q, via_csr.Q) and torch.equal(res.B, via_csr.B)

"""Block (BSR) input at the C ABI: mgr_csr with block = 2 or 3.
  * the FP64 BSR SpMV against SciPy, entrywise within 1e-13 (|A| |x|)_i, on ragged block
    rows (empty ones, rows longer than a streamed window, which take the direct path);
  * mgr_setup on a BSR3 matrix builds the same hierarchy, bit for bit, as on its scalar
    expansion (the CSR with every entry of every block, zeros included);
  * FGMRES with the BSR3 outer matrix converges like the CSR one (iterations within one,
    true residual at the target)."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.helpers import device_workload
from workloads import poromech as pm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")


def to_bsr(A: sp.csr_matrix, b: int):
    B = sp.bsr_matrix(A, blocksize=(b, b))
    B.sort_indices()
    return B.indptr.astype(np.int64), B.indices.astype(np.int32), B.data


def expand(indptr, indices, blocks):
    """The scalar CSR with every entry of every block (zeros kept), columns sorted."""
    b = blocks.shape[1]
    nbr = len(indptr) - 1
    rows, cols, vals = [], [], []
    for br in range(nbr):
        for r in range(b):
            for e in range(indptr[br], indptr[br + 1]):
                for c in range(b):
                    rows.append(br * b + r)
                    cols.append(indices[e] * b + c)
                    vals.append(blocks[e, r, c])
    rows = np.array(rows, dtype=np.int64)
    ip = np.zeros(nbr * b + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nbr * b), out=ip[1:])
    return ip, np.array(cols, dtype=np.int64), np.array(vals)


def random_bsr(rng, nbr, b, lens):
    indptr = np.zeros(nbr + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    cols = np.concatenate([np.sort(rng.choice(nbr, size=L, replace=False)) for L in lens])
    blocks = rng.standard_normal((indptr[-1], b, b))
    blocks[rng.random(blocks.shape) < 0.2] = 0.0
    return indptr, cols.astype(np.int32), blocks


@pytest.mark.parametrize("b", [2, 3])
def test_bsr_spmv_matches_scipy(b):
    rng = np.random.default_rng(b)
    nbr = 900
    lens = rng.integers(0, 30, size=nbr)
    lens[[3, 4]] = 0
    # block rows longer than a window: 2x2 windows stage 576 blocks, the 3x3 kernel's 768
    lens[[100, 500]] = [300, 450]
    lens[[600, 700]] = [800, 890]
    lens[[200, 201]] = [26, 27]
    indptr, cols, blocks = random_bsr(rng, nbr, b, lens)
    A = m.Matrix.bsr_from_host(indptr, cols, blocks)
    S = sp.bsr_matrix((blocks, cols, indptr), shape=(nbr * b, nbr * b)).tocsr()
    x = rng.standard_normal(nbr * b)
    y = A.spmv(torch.as_tensor(x).cuda()).cpu().numpy()
    ref = S @ x
    bound = 1e-13 * (abs(S) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(y - ref) <= bound)
    # an empty matrix of blocks
    Z = m.Matrix.bsr_from_host(np.zeros(5, dtype=np.int64), np.zeros(0, dtype=np.int32),
                               np.zeros((0, b, b)))
    yz = Z.spmv(torch.ones(4 * b, dtype=torch.float64, device="cuda"))
    assert torch.count_nonzero(yz) == 0


def small_amg(opts, coarse_size=48):
    opts.amg_frelax = m.AMG(coarse_size=coarse_size)
    opts.amg_coarse = m.AMG(coarse_size=coarse_size)
    return opts


EXPORTS = [m.X_LEVEL_A, m.X_F, m.X_C, m.X_WP, m.X_ACOR, m.X_G]


def test_bsr3_setup_equals_expanded_csr():
    w = pm.three_phase(6, 5, 4, 3)
    indptr, cols, blocks = to_bsr(w.scipy(), 3)
    Ab = m.Matrix.bsr_from_host(indptr, cols, blocks)
    ip, ci, v = expand(indptr, cols, blocks)
    Ac = m.Matrix.from_host(ip, ci, v)
    labels = torch.as_tensor(w.labels).cuda()
    opts = small_amg(m.paper_plan("three"))
    opts.keep_setup = True
    Pb = m.Preconditioner(Ab, labels, opts)
    Pc = m.Preconditioner(Ac, labels, opts)
    nl = len(opts.levels)
    for l in range(nl):
        for what in EXPORTS:
            eb, ec = Pb.export(what, l), Pc.export(what, l)
            if isinstance(eb, tuple):
                for a, c in zip(eb[:3], ec[:3]):
                    assert np.array_equal(a, c), (l, what)
                    assert np.array_equal(np.signbit(a), np.signbit(c)) if a.dtype.kind == "f" \
                        else True
            else:
                assert np.array_equal(eb, ec), (l, what)
    cb, cc = Pb.export(m.X_LEVEL_A, nl), Pc.export(m.X_LEVEL_A, nl)
    for a, c in zip(cb[:3], cc[:3]):
        assert np.array_equal(a, c)
    v0 = torch.as_tensor(np.random.default_rng(1).standard_normal(w.n)).cuda()
    assert torch.equal(Pb.apply(v0), Pc.apply(v0))
    Pb.close()
    Pc.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bsr3_outer_fgmres(prec):
    w = pm.three_phase(10, 9, 8, 3)
    A, labels, b = device_workload(w)
    indptr, cols, blocks = to_bsr(w.scipy(), 3)
    Ab = m.Matrix.bsr_from_host(indptr, cols, blocks)
    P = m.Preconditioner(A, labels, small_amg(m.paper_plan("three", precision=prec)))
    x1, i1 = m.fgmres(A, b, M=P, restart=30, rtol=1e-6, maxit=400)
    x2, i2 = m.fgmres(Ab, b, M=P, restart=30, rtol=1e-6, maxit=400)
    rel = np.linalg.norm(w.b - w.scipy() @ x2.cpu().numpy()) / np.linalg.norm(w.b)
    print(f"  three 10x9x8 {prec}: CSR {i1['iters']} BSR3 {i2['iters']} true relres {rel:.2e}",
          flush=True)
    assert i2["converged"] and rel <= 1e-6 * 1.0000001
    assert abs(i1["iters"] - i2["iters"]) <= 1
    P.close()


def test_bsr_argument_errors():
    w = pm.three_phase(3, 3, 3, 3)
    indptr, cols, blocks = to_bsr(w.scipy(), 3)
    Ab = m.Matrix.bsr_from_host(indptr, cols, blocks)
    labels = torch.as_tensor(w.labels).cuda()
    Ab.c.block = 4
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(Ab, labels, m.paper_plan("three"))
    assert e.value.status == m.MGR_ERR_ARG
    Ab.c.block = 3
    Ab.c.reserved = 1
    b = torch.ones(w.n, dtype=torch.float64, device="cuda")
    with pytest.raises(m.MgrError) as e:
        m.fgmres(Ab, b, maxit=2)
    assert e.value.status == m.MGR_ERR_ARG


def cell_matrix(rng, ncell, br, long_cells, bc=None, ngroup=None):
    """CSR over ncell cells of br rows and ngroup column groups of bc: each cell draws a set
    of column groups and each of its rows a random subset of their columns (rows empty,
    rows sharing none of their blocks, explicit zeros); `long_cells` maps cell -> block
    count (those cells' rows take every column of their groups)."""
    bc = br if bc is None else bc
    ngroup = ncell if ngroup is None else ngroup
    indptr, cols = [0], []
    for I in range(ncell):
        nbk = long_cells.get(I, int(rng.integers(0, 14)))
        bks = np.sort(rng.choice(ngroup, size=min(nbk, ngroup), replace=False))
        for r in range(br):
            dens = 1.0 if I in long_cells else rng.choice([0.0, 0.3, 0.9, 1.0])
            keep = rng.random(len(bks) * bc) < dens
            cs = (bks[:, None] * bc + np.arange(bc)[None, :]).reshape(-1)[keep]
            cols.append(cs)
            indptr.append(indptr[-1] + len(cs))
    cols = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    vals = rng.standard_normal(len(cols))
    vals[rng.random(len(cols)) < 0.05] = 0.0
    return np.array(indptr, dtype=np.int64), cols, vals, ngroup * bc


def bsr_by_definition(indptr, cols, vals, br, bc=None):
    bc = br if bc is None else bc
    nbr = (len(indptr) - 1) // br
    brp, bci, blocks = [0], [], []
    for I in range(nbr):
        e0, e1 = indptr[I * br], indptr[I * br + br]
        bk = np.unique(cols[e0:e1] // bc)
        where = {c: k for k, c in enumerate(bk)}
        blk = np.zeros((len(bk), br, bc))
        for r in range(br):
            for e in range(indptr[I * br + r], indptr[I * br + r + 1]):
                blk[where[cols[e] // bc], r, cols[e] % bc] = vals[e]
        bci.append(bk)
        blocks.append(blk)
        brp.append(brp[-1] + len(bk))
    return (np.array(brp), np.concatenate(bci) if bci else np.zeros(0),
            np.concatenate(blocks) if blocks else np.zeros((0, br, bc)))


@pytest.mark.parametrize("br,bc", [(2, 2), (3, 3), (2, 3)])
def test_csr_to_bsr_matches_definition(br, bc):
    """The cell-block storage of the block-Jacobi sweeps and of A_CF, bit for bit: block
    columns, row pointers and every value (absent entries zero, explicit zeros kept), on
    cells of 0 .. 13 blocks, full cells of 25, 40, 60, 90 and 170 blocks (below and beyond the
    256 entries staged in LDS; beyond are merged from global memory) and ragged, empty and
    one-row cells; (2, 3) on a rectangular matrix."""
    rng = np.random.default_rng(40 + 10 * br + bc)
    ncell = 700
    ngroup = 700 if br == bc else 560
    ip, ci, v, m_cols = cell_matrix(rng, ncell, br, {5: 90, 6: 170, 7: 25, 300: 40, 699: 60}, bc, ngroup)
    A = m.Matrix.from_host(ip, ci, v, ncols=m_cols)
    brp, bci, bv = m.csr_to_bsr(A, br, bc)
    erp, eci, ev = bsr_by_definition(ip, ci, v, br, bc)
    assert np.array_equal(brp.cpu().numpy(), erp)
    assert np.array_equal(bci.cpu().numpy(), eci)
    assert np.array_equal(bv.cpu().numpy(), ev)


def test_csr_to_bsr_errors():
    import ctypes as C
    ip, ci, v, n = cell_matrix(np.random.default_rng(1), 5, 2, {})
    A = m.Matrix.from_host(ip, ci, v)          # 10 x 10
    for br, bc in ((1, 1), (3, 3), (4, 4), (3, 2), (2, 3)):   # shapes; 10 not a multiple of 3
        with pytest.raises(m.MgrError):
            m.csr_to_bsr(A, br, bc)
    brp, bci, bv = m.csr_to_bsr(A, 2)
    k = int(bci.numel())
    assert k > 0
    nb = C.c_int64()
    st = m.lib().mgr_csr_to_bsr(C.byref(A.c), 2, 2, brp.data_ptr(), bci.data_ptr(),
                                bv.data_ptr(), k - 1, C.byref(nb), None)
    assert st != 0 and nb.value == k          # capacity below the block count

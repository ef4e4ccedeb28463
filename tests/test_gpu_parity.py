"""GPU parity: the HIP library against the FP64 CPU oracle, through the C ABI.

Bars (from the method and its arithmetic):
  * integer/index work (C/F split, aggregates, every sparsity pattern) - bit-exact;
  * setup values (W_p, A_cor, G, coarse operators, AMG P and Galerkin products) - bit-exact:
    both sides take every product and sum in the same order with separate roundings;
  * preconditioner application in FP64 - relative 2-norm difference <= 1e-12 over the whole
    vector, and within every unknown type (displacement, each saturation, pressure)
    separately <= max(1e-12, 16 x the spread of the oracle against itself), so that an error
    confined to a block that carries little of the vector's norm is still seen.  The spread
    is the block's difference between the oracle and the same oracle with every row summed
    in the opposite order: the rounding noise of the method on that block (a saturation
    block is formed by residuals and corrections that nearly cancel: spreads up to 3.6e-12
    on the channelised case, 1e-12 on the two-phase ones, 1e-14 and less elsewhere);
  * preconditioner application with the FP32 hierarchy - within every unknown type, at most
    16 times the error of the oracle's own algorithm run in single precision (every stored
    value and every operation in float32), and never below 16 unit roundoffs (2^-24);
  * FGMRES - iteration count within +-1 of the oracle (CGS2 on the GPU, MGS in the oracle),
    true FP64 relative residual <= rtol.
"""
import numpy as np
import pytest

from oracle import amg as oamg
from oracle import krylov as okry
from oracle import mgr as omgr
from oracle.sparse import CSR
from tests.helpers import (assert_csr_equal, block_errors, device_workload, fp32_copy,
                           oracle_csr, oracle_plan, row_reversed_copy)
from workloads import poromech as pm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")


def log(*a):
    print(*a, flush=True)


def small_amg(opts, coarse_size=48):
    opts.amg_frelax = m.AMG(coarse_size=coarse_size)
    opts.amg_coarse = m.AMG(coarse_size=coarse_size)
    return opts


def tol_plan(tol, model="two"):
    """The paper plan with the tolerance form of G on the displacement level."""
    opts = m.paper_plan(model)
    opts.levels[0].nmax = -1
    opts.levels[0].drop_tol = tol
    return opts


def ilu_plan(model, level, steps, tri=3, sweeps=3):
    """The paper plan with the fine-grained ILU(level) global smoother on the levels that
    hold only cell unknowns."""
    opts = m.paper_plan(model, global_smoother="ilu", global_sweeps=steps)
    for L in opts.levels:
        if L.global_smoother == "ilu":
            L.ilu_level, L.ilu_sweeps, L.ilu_tri_sweeps = level, sweeps, tri
    return opts


def variant_plan(model, restrict=None, dff=None, **kw):
    """The paper plan with the Jacobi restriction and / or block D_FF on the given levels."""
    opts = m.paper_plan(model, **kw)
    for l, r in (restrict or {}).items():
        opts.levels[l].restrict = r
    for l, b in (dff or {}).items():
        opts.levels[l].dff_block = b
    return opts


def galerkin_plan(model, coarse):
    """The paper plan with no dropping on the displacement level (N_max = -1)."""
    opts = m.paper_plan(model, coarse=coarse) if model == "biot1" else m.paper_plan(model)
    opts.levels[0].nmax = -1
    return opts


CASES = [
    ("biot_8x8x8_paper_dense", lambda: pm.biot_single_phase(8, 8, 8, 0),
     lambda: small_amg(m.paper_plan("biot1", coarse="dense"))),
    ("biot_8x8x8_galerkin_dense", lambda: pm.biot_single_phase(8, 8, 8, 0),
     lambda: small_amg(galerkin_plan("biot1", "dense"))),
    ("biot_8x8x8_galerkin_amg", lambda: pm.biot_single_phase(8, 8, 8, 0),
     lambda: small_amg(galerkin_plan("biot1", "amg"))),
    ("biot_8x8x8_paper_amg", lambda: pm.biot_single_phase(8, 8, 8, 0),
     lambda: small_amg(m.paper_plan("biot1", coarse="amg"))),
    ("two_9x7x6_paper", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(m.paper_plan("two"))),
    ("two_9x7x6_paper_one_sweep", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(m.paper_plan("two", global_sweeps=1))),
    ("two_9x7x6_satfirst", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(m.saturation_first_plan("two"))),
    ("three_6x5x4_paper", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(m.paper_plan("three"))),
    ("two_9x7x6_quasi_impes", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(m.paper_plan("two", quasi_impes=True, global_sweeps=3))),
    ("two_9x7x6_drop_tol", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(tol_plan(0.05))),
    ("three_6x5x4_drop_tol", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(tol_plan(0.2, "three"))),
    ("two_9x7x6_block_gs", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(m.paper_plan("two", global_smoother="block_gs", global_sweeps=2))),
    ("three_6x5x4_block_gs", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(m.paper_plan("three", global_smoother="block_gs", global_sweeps=1))),
    ("channels_12x10x6_quasi_impes", lambda: pm.two_phase_channels(12, 10, 6, 2),
     lambda: small_amg(m.paper_plan("two", quasi_impes=True, global_sweeps=3))),
    ("three_6x5x4_quasi_impes", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(m.paper_plan("three", quasi_impes=True, global_sweeps=2))),
    ("two_9x7x6_ilu1", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(ilu_plan("two", level=1, steps=1))),
    ("two_9x7x6_ilu0_two_steps", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(ilu_plan("two", level=0, steps=2, tri=2))),
    ("three_6x5x4_ilu1", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(ilu_plan("three", level=1, steps=1))),
    ("channels_12x10x6_ilu1", lambda: pm.two_phase_channels(12, 10, 6, 2),
     lambda: small_amg(ilu_plan("two", level=1, steps=1, tri=4))),
    ("two_9x7x6_jacobi_restriction", lambda: pm.two_phase(9, 7, 6, 1),
     lambda: small_amg(variant_plan("two", restrict={0: "jacobi", 1: "jacobi"}))),
    ("biot_8x8x8_block_dff", lambda: pm.biot_single_phase(8, 8, 8, 0),
     lambda: small_amg(variant_plan("biot1", dff={0: 3}, coarse="dense"))),
    ("three_6x5x4_block_dff_jacobi_restriction", lambda: pm.three_phase(6, 5, 4, 3),
     lambda: small_amg(variant_plan("three", dff={0: 3}, restrict={0: "jacobi", 2: "jacobi"}))),
]


def compare_amg(P, level, H: oamg.AMGHierarchy, tag):
    nlev = P.amg_levels(level)
    assert nlev == len(H.levels), (tag, nlev, len(H.levels))
    for k, L in enumerate(H.levels):
        assert_csr_equal(P.export(m.X_AMG_A, level, k), L.A, f"{tag} AMG A[{k}]")
        if k + 1 < nlev:
            agg = P.export(m.X_AMG_AGG, level, k)
            assert np.array_equal(agg, L.agg), f"{tag} aggregates[{k}]"
            assert_csr_equal(P.export(m.X_AMG_P, level, k), L.P, f"{tag} AMG P[{k}]")


def compare_hierarchy(P, H: omgr.Hierarchy, tag):
    for l, L in enumerate(H.levels):
        log(f"  {tag}: level {l} n={L.A.shape[0]} nF={len(L.F)} nC={len(L.C)}")
        assert np.array_equal(P.export(m.X_F, l), L.F), f"{tag} F[{l}]"
        assert np.array_equal(P.export(m.X_C, l), L.C), f"{tag} C[{l}]"
        assert_csr_equal(P.export(m.X_LEVEL_A, l), L.A, f"{tag} A[{l}]")
        assert_csr_equal(P.export(m.X_WP, l), L.Wp, f"{tag} W_p[{l}]")
        assert_csr_equal(P.export(m.X_ACOR, l), L.Acor, f"{tag} A_cor[{l}]")
        assert_csr_equal(P.export(m.X_G, l), L.G, f"{tag} G[{l}]")
        if L.Wr is not None:
            assert_csr_equal(P.export(m.X_WR, l), L.Wr, f"{tag} W_r[{l}]")
        if L.amg is not None:
            compare_amg(P, l, L.amg, f"{tag} F-AMG[{l}]")
        if L.colors is not None:
            col = P.export(m.X_GS_COLOR, l)
            assert np.array_equal(col, L.colors), f"{tag} block Gauss-Seidel colours[{l}]"
    nl = len(H.levels)
    assert_csr_equal(P.export(m.X_LEVEL_A, nl), H.coarse_A, f"{tag} coarse A")
    if H.coarse_amg is not None:
        compare_amg(P, nl, H.coarse_amg, f"{tag} coarse AMG")


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    tag, make_w, make_o = request.param
    log(f"[case] {tag}")
    w = make_w()
    opts = make_o()
    opts.keep_setup = True
    A, labels, b = device_workload(w)
    P = m.Preconditioner(A, labels, opts)
    H = omgr.setup(oracle_csr(w), w.labels, oracle_plan(opts))
    yield tag, w, opts, A, labels, b, P, H
    P.close()


def test_setup_bit_exact(case):
    tag, w, opts, A, labels, b, P, H = case
    compare_hierarchy(P, H, tag)


def test_ilu_smoother_factors(case):
    """ILU global smoother: the factors on the ILU(k) pattern of D_B^{-1} A_l, bit for bit
    (closed-form block inverses, the pinned-order product, synchronous sweeps with the
    component sums in ascending order on both sides)."""
    tag, w, opts, A, labels, b, P, H = case
    levels = [l for l, L in enumerate(H.levels) if L.ilu is not None]
    if not levels:
        pytest.skip("no ILU smoother in this plan")
    for l in levels:
        S = H.levels[l].ilu.S
        log(f"  {tag}: ILU factors of level {l}: {S.nnz} entries")
        assert_csr_equal(P.export(m.X_ILU, l), S, f"{tag} ILU[{l}]")


# Cases whose coarsest grid is solved densely and is ill-conditioned: two FP64 direct
# solvers (the GPU's Gauss-Jordan inverse, the oracle's LAPACK LU) each have forward error
# up to about kappa(S_c) u, and differ by that much (for the Galerkin 8^3 pressure grid,
# kappa_2 = 4.1e6: Gauss-Jordan and an unblocked LU both differ from LAPACK's LU by 2e-11 in
# the oracle's own arithmetic).  Their bar is max(1e-12, 32 kappa_2(S_c) u).
KAPPA_BAR = {"biot_8x8x8_galerkin_dense"}


def apply_bar(tag, H):
    """Whole-vector bar (the block bars come from the oracle's own spread)."""
    if tag not in KAPPA_BAR:
        return 1e-12
    kappa = np.linalg.cond(H.coarse_A.to_dense())
    return max(1e-12, 32.0 * kappa * np.finfo(np.float64).eps)


def test_apply_fp64_matches_oracle(case):
    tag, w, opts, A, labels, b, P, H = case
    bar = apply_bar(tag, H)
    Hr = row_reversed_copy(H)
    rng = np.random.default_rng(5)
    for trial in range(3):
        v = rng.standard_normal(w.n) * np.where(w.labels == 0, 1e7, 1e-3)
        z_ref = omgr.apply(H, v)
        z = P.apply(torch.as_tensor(v).cuda()).cpu().numpy()
        err = np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref)
        blk = block_errors(z, z_ref, w.labels)
        spread = block_errors(omgr.apply(Hr, v), z_ref, w.labels)
        log(f"  {tag}: apply rel err {err:.3e}; per unknown type (gpu / oracle spread) "
            + " ".join(f"{t}:{e:.2e}/{spread[t]:.1e}" for t, e in blk.items()))
        assert err <= bar
        for t, e in blk.items():
            bar_t = max(bar, 16.0 * spread[t])
            assert e <= bar_t, (tag, t, e, bar_t)


U32 = 2.0 ** -24


def test_apply_fp32_matches_oracle(case):
    """The FP32 hierarchy (values cast after the FP64 setup, FP32 vectors and arithmetic
    inside the apply) against the FP64 oracle, per unknown type."""
    tag, w, opts, A, labels, b, P, H = case
    import copy
    o32 = copy.deepcopy(opts)
    o32.precision = "fp32"
    P32 = m.Preconditioner(A, labels, o32)
    H32 = fp32_copy(H)
    rng = np.random.default_rng(15)
    for trial in range(3):
        v = rng.standard_normal(w.n) * np.where(w.labels == 0, 1e7, 1e-3)
        z_ref = omgr.apply(H, v)
        z_o32 = omgr.apply(H32, v.astype(np.float32)).astype(np.float64)
        z = P32.apply(torch.as_tensor(v).cuda()).cpu().numpy()
        got = block_errors(z, z_ref, w.labels)
        ref = block_errors(z_o32, z_ref, w.labels)
        log(f"  {tag}: FP32 apply per unknown type (gpu / oracle in float32) "
            + " ".join(f"{t}:{got[t]:.2e}/{ref[t]:.2e}" for t in got))
        for t in got:
            assert got[t] <= 16.0 * max(ref[t], U32), (tag, t, got[t], ref[t])
    P32.close()


# the channelized case stalls above 1e-8 (in the oracle too); it is compared at 1e-6
FGMRES_RTOL = {"channels_12x10x6_quasi_impes": 1e-6, "channels_12x10x6_ilu1": 1e-6}


def test_fgmres_matches_oracle(case):
    tag, w, opts, A, labels, b, P, H = case
    rtol = FGMRES_RTOL.get(tag, 1e-8)
    Ao = oracle_csr(w)
    ref = okry.fgmres(Ao.matvec, lambda v: omgr.apply(H, v), w.b, restart=30, rtol=rtol,
                      maxit=400)
    x, info = m.fgmres(A, b, M=P, restart=30, rtol=rtol, maxit=400)
    xs = x.cpu().numpy()
    true = np.linalg.norm(w.b - w.scipy() @ xs) / np.linalg.norm(w.b)
    log(f"  {tag}: iters gpu {info['iters']} oracle {ref.iters}; true relres {true:.2e}")
    assert ref.converged and info["converged"]
    assert abs(info["iters"] - ref.iters) <= 1
    assert true <= rtol * 1.0000001
    assert info["true_relres"] == pytest.approx(true, rel=1e-6, abs=1e-14)
    errx = np.linalg.norm(xs - ref.x) / np.linalg.norm(ref.x)
    assert errx <= 1e-5


def test_graph_replays_match_eager(case):
    tag, w, opts, A, labels, b, P, H = case
    import copy
    o2 = copy.deepcopy(opts)
    o2.use_graph = False
    P2 = m.Preconditioner(A, labels, o2)
    rng = np.random.default_rng(6)
    for _ in range(3):
        v = torch.as_tensor(rng.standard_normal(w.n)).cuda()
        z1 = P.apply(v)
        torch.cuda.synchronize()
        z2 = P2.apply(v)
        torch.cuda.synchronize()
        assert torch.equal(z1, z2)
    P2.close()


def random_system(rng, labels, density, diag_ff):
    n = len(labels)
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    if diag_ff:
        f = np.flatnonzero(labels == 0)
        D[np.ix_(f, f)] = 0.0
    D[np.arange(n), np.arange(n)] = 3.0 * (np.abs(D).sum(axis=1) + 1.0)
    return D


def test_exactness_pin_one_iteration():
    """A_FF diagonal + one Jacobi sweep (omega = 1) + no dropping + exact coarse solve gives
    M^{-1} = A^{-1}: FGMRES converges in one iteration on the GPU."""
    rng = np.random.default_rng(7)
    labels = np.sort(rng.integers(0, 2, size=300)).astype(np.int8)[::-1].copy()
    labels = rng.permutation(labels).astype(np.int8)
    D = random_system(rng, labels, 0.03, True)
    Ao = CSR.from_dense(D)
    A = m.Matrix.from_host(Ao.indptr, Ao.indices, Ao.data)
    lab = torch.as_tensor(labels).cuda()
    opts = m.Options(levels=[m.Level((0,), nmax=-1, frelax="jacobi")], coarse="dense")
    P = m.Preconditioner(A, lab, opts)
    bb = torch.as_tensor(rng.standard_normal(300)).cuda()
    x, info = m.fgmres(A, bb, M=P, restart=30, rtol=1e-10)
    assert info["iters"] == 1
    v = rng.standard_normal(300)
    z = P.apply(torch.as_tensor(v).cuda()).cpu().numpy()
    assert np.linalg.norm(D @ z - v) / np.linalg.norm(v) <= 1e-12
    P.close()


@pytest.mark.parametrize("model", ["two", "three"])
def test_fp32_hierarchy_iterations_within_one(model):
    """FP32 hierarchy inside FP64 FGMRES against the FP64 hierarchy and the FP64 oracle:
    iterations within one, true FP64 residual at the target, and the solution error against
    the oracle's solution reported per unknown type.  Two solutions that meet the same
    residual tolerance on these Jacobians can differ by as much as either differs from the
    exact solution (the oracle's own x is 12% / 8% from x_true at rtol 1e-6); the FP32
    solution must be at least ten times closer to the oracle's than that."""
    w = pm.two_phase(12, 11, 10, 4) if model == "two" else pm.three_phase(10, 9, 8, 3)
    A, labels, b = device_workload(w)
    opts = small_amg(m.paper_plan(model))
    H = omgr.setup(oracle_csr(w), w.labels, oracle_plan(opts))
    ref = okry.fgmres(oracle_csr(w).matvec, lambda v: omgr.apply(H, v), w.b, restart=30,
                      rtol=1e-6, maxit=400)
    assert ref.converged
    ref_err = np.linalg.norm(ref.x - w.x_true) / np.linalg.norm(w.x_true)
    res = {}
    for prec in ("fp64", "fp32"):
        P = m.Preconditioner(A, labels, small_amg(m.paper_plan(model, precision=prec)))
        x, info = m.fgmres(A, b, M=P, restart=30, rtol=1e-6, maxit=400)
        xs = x.cpu().numpy()
        true = np.linalg.norm(w.b - w.scipy() @ xs) / np.linalg.norm(w.b)
        err = np.linalg.norm(xs - ref.x) / np.linalg.norm(ref.x)
        blk = block_errors(xs, ref.x, w.labels)
        res[prec] = (info["iters"], true, err)
        log(f"  {model} {prec}: iters {info['iters']} (oracle {ref.iters}) true relres "
            f"{true:.2e}; ||x - x_oracle||/||x_oracle|| {err:.2e}; per unknown type "
            + " ".join(f"{t}:{e:.2e}" for t, e in blk.items()))
        assert true <= 1e-6 * 1.0000001
        P.close()
    assert abs(res["fp64"][0] - res["fp32"][0]) <= 1
    assert abs(res["fp64"][0] - ref.iters) <= 1
    log(f"  {model}: ||x_oracle - x_true||/||x_true|| {ref_err:.2e}")
    assert res["fp32"][2] <= 0.1 * ref_err


def test_spmv_ragged_matches_scipy():
    import scipy.sparse as sp
    rng = np.random.default_rng(8)
    for n, dens in ((1, 1.0), (37, 0.2), (1000, 0.01), (4099, 0.003)):
        S = sp.random(n, n, density=dens, random_state=rng, format="csr")
        S.sort_indices()
        A = m.Matrix.from_host(S.indptr, S.indices, S.data)
        x = rng.standard_normal(n)
        y = A.spmv(torch.as_tensor(x).cuda()).cpu().numpy()
        ref = S @ x
        assert np.allclose(y, ref, rtol=1e-13, atol=1e-13 * (np.abs(ref).max() + 1e-300))


def test_spmv_long_and_empty_rows():
    """Rows longer than a streamed block, rows just over the staged-window slack (257 and
    300 entries), empty rows, and a single row."""
    import scipy.sparse as sp
    rng = np.random.default_rng(9)
    n = 3000
    lens = rng.integers(0, 40, size=n)
    lens[[5, 6, 2000]] = [2900, 5000 if n > 5000 else 2999, 2500]
    lens[[700, 1500, 2600]] = [257, 300, 256]
    lens[100:110] = 0
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = np.sort(rng.choice(n, size=min(L, n), replace=False))
        rows.append(np.full(c.size, i)); cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    S = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n))
    S.sort_indices()
    A = m.Matrix.from_host(S.indptr, S.indices, S.data)
    x = rng.standard_normal(n)
    y = A.spmv(torch.as_tensor(x).cuda()).cpu().numpy()
    assert np.allclose(y, S @ x, rtol=1e-12, atol=1e-12)
    bb = torch.as_tensor(S @ x).cuda()
    xs, info = m.fgmres(A, bb, restart=5, rtol=1e-30, maxit=2, raise_on_fail=False)
    assert info["iters"] == 2


def test_repeated_setups_reuse_cached_blocks():
    # setup and destroy of the same problem, the F-relaxation AMG built on a second stream:
    # the blocks freed by one setup serve the next, so the cache stops growing
    w = pm.biot_single_phase(6, 6, 6, 0)
    A, labels, b = device_workload(w)
    opts = small_amg(m.paper_plan("biot1"), coarse_size=24)
    L = m.lib()
    sizes = []
    for _ in range(5):
        P = m.Preconditioner(A, labels, opts)
        P.close()
        torch.cuda.synchronize()
        sizes.append(L.mgr_cached_bytes())
    assert sizes[2] == sizes[3] == sizes[4], sizes


def test_error_paths():
    w = pm.biot_single_phase(3, 3, 3, 0)
    A, labels, b = device_workload(w)
    bad = labels.clone()
    bad[5] = 9
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(A, bad, m.paper_plan("biot1"))
    assert e.value.status == m.MGR_ERR_ARG
    # a zero on the diagonal of A_FF
    data = w.data.copy()
    r = 4
    for q in range(w.indptr[r], w.indptr[r + 1]):
        if w.indices[q] == r:
            data[q] = 0.0
    Az = m.Matrix.from_host(w.indptr, w.indices, data)
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(Az, labels, m.Options(levels=[m.Level((0,))], coarse="dense"))
    assert e.value.status == m.MGR_ERR_ZERO_PIVOT
    # an empty C set
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(A, labels, m.Options(levels=[m.Level((0, 2))], coarse="dense"))
    assert e.value.status == m.MGR_ERR_ARG
    # both forms of G on one level
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(A, labels, m.Options(levels=[m.Level((0,), nmax=4, drop_tol=0.1)],
                                              coarse="dense"))
    assert e.value.status == m.MGR_ERR_ARG
    # an F block without full 3x3 node blocks: the nodal AMG, built on a second host thread
    # and stream, fails there and the error reaches the caller
    odd = labels.clone()
    odd[1] = 2
    with pytest.raises(m.MgrError) as e:
        m.Preconditioner(A, odd, small_amg(m.paper_plan("biot1"), coarse_size=24))
    assert e.value.status == m.MGR_ERR_UNSUPPORTED
    # the library stays usable afterwards
    P = m.Preconditioner(A, labels, m.paper_plan("biot1", coarse="dense"))
    P.close()
    # maxit reached: NOT_CONVERGED with the last iterate
    x, info = m.fgmres(A, b, M=None, restart=5, rtol=1e-14, maxit=3, raise_on_fail=False)
    assert info["status"] == m.MGR_ERR_NOT_CONVERGED and info["iters"] == 3


def test_setup_numeric_same_pattern_equals_fresh_setup():
    w1 = pm.two_phase(7, 6, 5, 11)
    w2 = pm.two_phase(7, 6, 5, 12)     # same pattern, other values
    A1, labels, b1 = device_workload(w1)
    A2, _, b2 = device_workload(w2)
    opts = small_amg(m.paper_plan("two"))
    P = m.Preconditioner(A1, labels, opts)
    P.setup_numeric(A2)
    Pf = m.Preconditioner(A2, labels, opts)
    v = torch.as_tensor(np.random.default_rng(1).standard_normal(w1.n)).cuda()
    assert torch.equal(P.apply(v), Pf.apply(v))
    w3 = pm.two_phase(7, 6, 6, 11)
    A3, l3, _ = device_workload(w3)
    with pytest.raises(m.MgrError) as e:
        P.setup_numeric(A3)
    assert e.value.status == m.MGR_ERR_PATTERN
    # same size and entry count, one column index moved by one place: the fingerprint of
    # the pattern differs
    ind = w1.indices.copy()
    r = w1.n // 2
    lo, hi = w1.indptr[r], w1.indptr[r + 1]
    q = next(q for q in range(hi - 1, lo - 1, -1)
             if ind[q] + 1 < w1.n and (q + 1 == hi or ind[q + 1] != ind[q] + 1))
    ind[q] += 1
    A4 = m.Matrix.from_host(w1.indptr, ind, w1.data)
    with pytest.raises(m.MgrError) as e:
        P.setup_numeric(A4)
    assert e.value.status == m.MGR_ERR_PATTERN
    P.close()
    Pf.close()


def test_setup_is_deterministic():
    w = pm.two_phase(8, 8, 8, 2)
    A, labels, b = device_workload(w)
    opts = small_amg(m.paper_plan("two", precision="fp32"))
    v = torch.as_tensor(np.random.default_rng(2).standard_normal(w.n)).cuda()
    outs = []
    for _ in range(2):
        P = m.Preconditioner(A, labels, opts)
        outs.append(P.apply(v))
        P.close()
    assert torch.equal(outs[0], outs[1])

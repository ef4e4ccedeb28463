"""GPU residual / Jacobian assembly and Newton time steps of the two-phase model
(mgr_poro_*), against the oracle (oracle/assembly.py, oracle/newton.py):
  * the library's Jacobian pattern equals the input generator's pattern of the same grid
    (independently written), labels included;
  * F(x) within 1e-12 (|A| |x|)_i of the oracle's per row, and every Jacobian entry within
    1e-13 of its row's largest, at random states with wells, Dirichlet dofs and nonzero
    displacement, on grids whose node and cell counts leave ragged last blocks;
  * the residual in state units (norms) against the oracle's;
  * a Newton time step: the same iteration count as the oracle's Newton with exact solves,
    and the same converged state, at tight tolerances; the owned Jacobian unchanged by the
    row scaling of the solves;
  * quadratic convergence and the smoother options on a channelised line drive;
  * at 64x64x16 cells, the Jacobian along a random direction against central differences
    of the GPU residual (a property at any size);
  * time-step cuts;
  * argument errors."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assembly as asm
from oracle import newton as onew
from workloads import poromech as pm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")
poro = pytest.importorskip("paper_1904_05960_amd.poro")


def random_case(nx, ny, nz, seed, u_scale=1e-4, p_noise=2e5, dt=86400.0):
    rng = np.random.default_rng(seed)
    prm = asm.Params(nx, ny, nz, dt=dt)
    nc = prm.ncell
    perm = 10.0 ** rng.uniform(-14.0, -12.0, nc)
    young = rng.uniform(5e9, 2e10, nc)
    nd = np.arange(prm.nnode)
    ix = nd % (nx + 1)
    iy = (nd // (nx + 1)) % (ny + 1)
    iz = nd // ((nx + 1) * (ny + 1))
    fx = np.zeros((prm.nnode, 3), dtype=bool)
    fx[iz == 0, :] = True
    fx[(ix == 0) | (ix == nx), 0] = True
    fx[(iy == 0) | (iy == ny), 1] = True
    props = asm.Props(perm, young, fx.ravel())
    props.qw[0] = 0.01
    props.qw[nc // 3] = 0.004
    props.wi[nc - 1] = 2e-12
    props.pbhp[nc - 1] = prm.p_ref - 2e5
    props.wi[nc // 2] = 1e-12
    props.pbhp[nc // 2] = prm.p_ref + 1e5
    props.qo[nc // 2] = 0.003
    x = np.zeros(prm.n)
    x[: prm.nu_dofs] = rng.normal(0.0, u_scale, prm.nu_dofs)
    x[: prm.nu_dofs][props.fixed] = 0.0
    x[prm.nu_dofs::2] = rng.uniform(0.15, 0.85, nc)
    x[prm.nu_dofs + 1::2] = prm.p_ref + rng.normal(0.0, p_noise, nc)
    x_old = x.copy()
    x_old[prm.nu_dofs::2] = np.clip(x_old[prm.nu_dofs::2] + rng.normal(0, 0.02, nc), 0.05, 0.95)
    x_old[prm.nu_dofs + 1::2] += rng.normal(0.0, 1e4, nc)
    x_old[: prm.nu_dofs] += rng.normal(0.0, 0.2 * u_scale, prm.nu_dofs)
    x_old[: prm.nu_dofs][props.fixed] = 0.0
    return prm, props, x, x_old


def gpu_model(prm, props, fixed_raw=None):
    p = poro.default_params(prm.nx, prm.ny, prm.nz, nu=prm.nu, dt=prm.dt, phi0=prm.phi0,
                            biot=prm.biot, grav=prm.grav, p_ref=prm.p_ref,
                            rho_solid=prm.rho_solid, rho0=prm.rho0, comp=prm.comp,
                            visc=prm.visc)
    return poro.Model(p, props.perm, props.young, props.fixed if fixed_raw is None else fixed_raw,
                      props.wi, props.pbhp, props.qw, props.qo)


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 3, 3), (7, 5, 4)])
def test_pattern_equals_generator(dims):
    nx, ny, nz = dims
    w = pm.two_phase(nx, ny, nz, seed=1, corr_len=2.0)
    prm = asm.Params(nx, ny, nz)
    props = asm.Props(w.meta["perm"], w.meta["young"], w.fixed.copy())
    M = gpu_model(prm, props)
    rp, ci, _, lab = M.export()
    assert np.array_equal(rp, w.indptr)
    assert np.array_equal(ci, w.indices)
    assert np.array_equal(lab, w.labels)
    M.close()


def compare_assembly(prm, props, x, x_old):
    M = gpu_model(prm, props)
    F = M.assemble(dev(x), dev(x_old)).cpu().numpy()
    rp, ci, val, _ = M.export()
    M.close()
    Fo = asm.residual(prm, props, x, x_old)
    Jo = asm.jacobian(prm, props, x).tocsr()
    absJx = abs(Jo) @ np.abs(x)
    assert np.all(np.abs(F - Fo) <= 1e-12 * absJx + 1e-300), \
        float(np.max(np.abs(F - Fo) / np.maximum(absJx, 1e-300)))
    rows = np.repeat(np.arange(prm.n), np.diff(rp))
    cols = np.array(ci, dtype=np.int64)
    ref = np.asarray(Jo[rows, cols]).ravel()
    rowmax = np.maximum.reduceat(np.abs(ref), rp[:-1])
    assert np.all(np.abs(val - ref) <= 1e-13 * rowmax[rows]), \
        float(np.max(np.abs(val - ref) / rowmax[rows]))
    # no derivative entry falls outside the pattern
    P = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(prm.n, prm.n))
    assert Jo.multiply(P).count_nonzero() == Jo.count_nonzero()
    return F, Fo


@pytest.mark.parametrize("dims,seed", [((3, 2, 2), 0), ((6, 5, 4), 1), ((12, 10, 6), 2)])
def test_residual_and_jacobian_match_oracle(dims, seed):
    prm, props, x, x_old = random_case(*dims, seed)
    compare_assembly(prm, props, x, x_old)


def test_assembly_without_wells_and_norms():
    prm, props, x, x_old = random_case(5, 4, 3, 3)
    props = asm.Props(props.perm, props.young, props.fixed)
    M = poro.Model(poro.default_params(prm.nx, prm.ny, prm.nz), props.perm, props.young,
                   props.fixed)
    F, nr = M.assemble(dev(x), dev(x_old), norms=True)
    M.close()
    Fo = asm.residual(prm, props, x, x_old)
    _, parts = asm.normalised(prm, props, Fo)
    for (ss, mx), (ss_o, mx_o) in zip(nr, parts):
        assert ss == pytest.approx(ss_o, rel=1e-10)
        assert mx == pytest.approx(mx_o, rel=1e-10)


def test_newton_step_matches_oracle():
    """Strict tolerances, so that both runs reach the same root: the same Newton iteration
    count as the oracle's Newton with exact linear solves, the same step lengths, and the
    same converged state."""
    prm, props, x, _ = random_case(4, 3, 3, 4, p_noise=2e4, dt=3600.0)
    nop = onew.NewtonOpts(tol_flow=1e-10, tol_mech=1e-13)
    xo, st_o = onew.time_step(prm, props, x, nop)
    assert st_o.converged
    M = gpu_model(prm, props)
    xg = dev(x)
    xold = dev(x)
    opts = m.paper_plan("two", precision="fp64")
    st = M.newton(xg, xold, opts, rtol=1e-12, maxit=200,
                  nopts=poro.newton_opts(tol_flow=1e-10, tol_mech=1e-13))
    # the solves use a row-scaled copy: the owned Jacobian (whose displacement block is
    # written once, at creation) still equals the oracle's after a re-assembly
    M.assemble(xg, xold)
    rp, ci, val, _ = M.export()
    M.close()
    xf = xg.cpu().numpy()
    Jo = asm.jacobian(prm, props, xf).tocsr()
    rows = np.repeat(np.arange(prm.n), np.diff(rp))
    ref = np.asarray(Jo[rows, np.array(ci, dtype=np.int64)]).ravel()
    rowmax = np.maximum.reduceat(np.abs(ref), rp[:-1])
    assert np.all(np.abs(val - ref) <= 1e-13 * rowmax[rows])
    assert st["converged"]
    assert st["newton_iters"] == st_o.newton_iters
    assert np.allclose(st["lambdas"], st_o.lambdas, rtol=0, atol=0)
    xg = xg.cpu().numpy()
    nu = prm.nu_dofs
    assert np.max(np.abs(xg[:nu] - xo[:nu])) <= 1e-9 * np.max(np.abs(xo[:nu]))
    assert np.max(np.abs(xg[nu::2] - xo[nu::2])) <= 1e-9
    assert np.max(np.abs(xg[nu + 1::2] - xo[nu + 1::2])) <= 1e-9 * np.max(np.abs(xo[nu + 1::2]))
    assert st["merit"][0] == pytest.approx(st_o.merit[0], rel=1e-10)


@pytest.mark.parametrize("kind", ["block_jacobi", "block_gs", "ilu"])
def test_line_drive_converges(kind):
    """Three time steps of the channelised line drive: every step converges, Newton
    converges quadratically at the end, and the linear solves reach their tolerance."""
    res = pm.channel_reservoir(16, 12, 4, seed=7)
    M = poro.model_from_reservoir(res)
    x, rec = poro.simulate(M, res["x0"], 3, poro.smoother_options(kind, "fp32"), rtol=1e-6)
    nu = M.nu
    M.close()
    assert all(r["converged"] for r in rec), rec
    assert all(r["linear_failures"] == 0 for r in rec)
    assert rec[0]["setups"] == 1 and all(r["setups"] == 0 for r in rec[1:])
    last = rec[-1]["merit"]
    assert rec[-1]["newton_iters"] >= 1 and last[-1] < 1e-2 * last[0]
    s = x.cpu().numpy()[nu::2]
    assert s.min() > 0.0 and s.max() < 1.0


def test_jacobian_directional_derivative_at_size():
    """At a size the oracle cannot assemble quickly (64x64x16 cells, 346,275 unknowns), a
    property that holds at any size: the assembled Jacobian times a random direction equals
    the central difference of the GPU residual along it, within the truncation and
    rounding of the difference (momentum, wetting and non-wetting rows separately)."""
    res = pm.channel_reservoir(64, 64, 16, seed=3)
    M = poro.model_from_reservoir(res)
    x = dev(res["x0"])
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    nu = M.nu
    x[:nu] = 1e-4 * torch.randn(nu, generator=g, device="cuda", dtype=torch.float64)
    x[:nu] *= dev(~res["fixed"])
    x[nu::2] = 0.15 + 0.7 * torch.rand(M.ncell, generator=g, device="cuda", dtype=torch.float64)
    x[nu + 1::2] += 1e5 * torch.randn(M.ncell, generator=g, device="cuda", dtype=torch.float64)
    x_old = x.clone()
    x_old[nu + 1::2] += 1e4
    M.assemble(x, x_old)
    d = torch.randn(M.n, generator=g, device="cuda", dtype=torch.float64)
    d[:nu] *= 1e-6 * dev(~res["fixed"])
    d[nu::2] *= 1e-3
    d[nu + 1::2] *= 1e2
    Jd = torch.empty_like(d)
    m._check(m.lib().mgr_spmv(C.byref(M.csr), m._ptr(d), m._ptr(Jd), m._stream()))
    h = 1e-3
    Fp = M.assemble(x + h * d, x_old, jacobian=False)
    Fm = M.assemble(x - h * d, x_old, jacobian=False)
    fd = (Fp - Fm) / (2 * h)
    M.close()
    for sl in (slice(0, nu), slice(nu, None, 2), slice(nu + 1, None, 2)):
        a, b = Jd[sl], fd[sl]
        assert float(torch.linalg.norm(a - b) / torch.linalg.norm(a)) < 1e-6


def test_time_step_control():
    """With few Newton iterations allowed, a long step fails and is retried with dt halved;
    the accepted steps still cover the whole interval and each converged."""
    res = pm.channel_reservoir(16, 12, 4, seed=7)
    res["dt"] = 20 * 86400.0
    M = poro.model_from_reservoir(res)
    x, rec = poro.simulate(M, res["x0"], 1, poro.smoother_options("ilu", "fp32"), rtol=1e-6,
                           nopts=poro.newton_opts(max_newton=4))
    dt_after = M.params.dt
    M.close()
    assert all(r["converged"] for r in rec)
    assert sum(r["cuts"] for r in rec) >= 1
    assert sum(r["dt"] for r in rec) == pytest.approx(20 * 86400.0, rel=1e-12)
    assert dt_after == 20 * 86400.0


def test_argument_errors():
    p = poro.default_params(0, 2, 2)
    z = np.zeros(4)
    with pytest.raises(m.MgrError) as e:
        poro.Model(p, z, z + 1e10, np.zeros(3 * 27, dtype=np.uint8))
    assert e.value.status == m.MGR_ERR_ARG
    p = poro.default_params(2, 2, 1)
    with pytest.raises(m.MgrError):
        poro.Model(p, np.ones(4) * 1e-13, np.ones(4) * 1e10, np.zeros(3 * 18, dtype=np.uint8),
                   wi=np.zeros(4))          # well index without bottom-hole pressures
    p = poro.default_params(2, 2, 1, dt=-1.0)
    with pytest.raises(m.MgrError):
        poro.Model(p, np.ones(4) * 1e-13, np.ones(4) * 1e10, np.zeros(3 * 18, dtype=np.uint8))
    p = poro.default_params(2, 2, 1)
    with pytest.raises(m.MgrError):
        poro.Model(p, np.ones(4) * 1e-13, np.zeros(4), np.zeros(3 * 18, dtype=np.uint8))

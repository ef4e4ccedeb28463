"""Pins of the oracle's residual / Jacobian of the two-phase model (Sec. 2-4) and of its
Newton time step (Sec. 4, eq. newton): finite differences, conservation, hydrostatics,
closed-form Biot loads, the rigid-body null space of the element stiffness, and an
independently written assembly of the same model (the input generator) at u = 0."""
import math

import numpy as np
import pytest

from oracle import assembly as asm
from oracle import newton as onew
from workloads import poromech as pm


def random_case(nx, ny, nz, seed, wells=True, fixed=True, u_scale=1e-4, p_noise=2e5, **kw):
    rng = np.random.default_rng(seed)
    prm = asm.Params(nx, ny, nz, **kw)
    nc = prm.ncell
    perm = 10.0 ** rng.uniform(-14.0, -12.0, nc)
    young = rng.uniform(5e9, 2e10, nc)
    fx = np.zeros(prm.nu_dofs, dtype=bool)
    if fixed:
        nd = np.arange(prm.nnode)
        ix = nd % (nx + 1)
        iy = (nd // (nx + 1)) % (ny + 1)
        iz = nd // ((nx + 1) * (ny + 1))
        fx[3 * nd[iz == 0] + 0] = True
        fx[3 * nd[iz == 0] + 1] = True
        fx[3 * nd[iz == 0] + 2] = True
        fx[3 * nd[(ix == 0) | (ix == nx)] + 0] = True
        fx[3 * nd[(iy == 0) | (iy == ny)] + 1] = True
    props = asm.Props(perm, young, fx)
    if wells:
        props.qw[0] = 0.01
        props.wi[nc - 1] = 2e-12
        props.pbhp[nc - 1] = prm.p_ref - 2e5
        props.qo[nc // 2] = 0.003
    x = np.zeros(prm.n)
    x[: prm.nu_dofs] = rng.normal(0.0, u_scale, prm.nu_dofs)
    x[: prm.nu_dofs][fx] = 0.0
    x[prm.nu_dofs::2] = rng.uniform(0.15, 0.85, nc)
    x[prm.nu_dofs + 1::2] = prm.p_ref + rng.normal(0.0, p_noise, nc)
    return prm, props, x


# ---------------------------------------------------------------------------------------
# Element matrices
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("nu", [0.25, 0.3])
def test_stiffness_matches_voigt_construction(nu):
    """The index-form stiffness equals the input generator's B^T D B construction."""
    K = asm.unit_stiffness(nu)
    Kg = pm.q1_unit_stiffness(nu)
    assert np.allclose(K, Kg, rtol=0, atol=1e-15 * np.abs(Kg).max())


def test_stiffness_null_space_is_rigid_motions():
    K = asm.unit_stiffness(0.25)
    assert np.allclose(K, K.T, atol=1e-15)
    X = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
    modes = []
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1.0
        modes.append(t.ravel())
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3))
        r[:, i] = -X[:, j]
        r[:, j] = X[:, i]
        modes.append(r.ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-14
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10) == 18 and ev.min() > -1e-14


def test_grad_integral_closed_form():
    G = asm.grad_integral()
    for a in range(8):
        for i in range(3):
            assert G[a, i] == pytest.approx(0.25 if (a >> i) & 1 else -0.25, abs=1e-16)


# ---------------------------------------------------------------------------------------
# Jacobian = dF/dx
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,stiff_comp", [(0, False), (1, True)])
def test_jacobian_matches_finite_differences(seed, stiff_comp):
    """Central differences of the residual, column by column.  With exaggerated
    compressibilities the small density terms (d rho / dp in the weight, the averaged
    density in the potential, the accumulation) carry weight the comparison can see."""
    kw = dict(comp=(2e-6, 5e-6)) if stiff_comp else {}
    prm, props, x = random_case(3, 2, 3, seed, **kw)
    rng = np.random.default_rng(seed + 10)
    x_old = x.copy()
    x_old[prm.nu_dofs + 1::2] += rng.normal(0, 1e4, prm.ncell)
    J = asm.jacobian(prm, props, x).toarray()
    h = np.empty(prm.n)
    h[: prm.nu_dofs] = 1e-9
    h[prm.nu_dofs::2] = 1e-6
    h[prm.nu_dofs + 1::2] = 1.0
    Jfd = np.zeros_like(J)
    for j in range(prm.n):
        e = np.zeros(prm.n)
        e[j] = h[j]
        Jfd[:, j] = (asm.residual(prm, props, x + e, x_old)
                     - asm.residual(prm, props, x - e, x_old)) / (2 * h[j])
    rowmax = np.abs(J).max(axis=1, keepdims=True)
    err = np.abs(J - Jfd)
    assert np.all(err <= 1e-6 * rowmax + 1e-7 * np.abs(J)), float((err / rowmax).max())


def test_jacobian_of_fixed_dofs_is_eliminated():
    prm, props, x = random_case(2, 2, 2, 3)
    J = asm.jacobian(prm, props, x).tocsr()
    K = asm.unit_stiffness(prm.nu)
    kd = asm.stiffness_diagonal(prm, props, K)
    for d in np.flatnonzero(props.fixed):
        row = J.getrow(d)
        assert row.nnz == 1 and row.indices[0] == d and row.data[0] == pytest.approx(kd[d])
        col = J.getcol(d)
        assert col.nnz == 1


# ---------------------------------------------------------------------------------------
# Conservation, hydrostatics, Biot load
# ---------------------------------------------------------------------------------------
def test_fluxes_telescope():
    """With x_old = x and no wells the accumulation vanishes and every face flux enters two
    cells with opposite signs: the mass residuals of each phase sum to zero."""
    prm, props, x = random_case(4, 3, 3, 4, wells=False)
    F = asm.residual(prm, props, x, x)
    for ph in (0, 1):
        f = F[prm.nu_dofs + ph::2]
        assert abs(f.sum()) <= 1e-12 * np.abs(f).max()
        assert np.abs(f).max() > 0


def test_wells_enter_the_global_balance():
    prm, props, x = random_case(4, 3, 3, 5, wells=True)
    F = asm.residual(prm, props, x, x)
    c = prm.ncell - 1
    for ph, q in ((0, props.qw), (1, props.qo)):
        r0 = prm.rho0[ph] * math.exp(prm.comp[ph] * (x[asm.p_dof(prm, c)] - prm.p_ref))
        S = x[asm.s_dof(prm, c)] if ph == 0 else 1.0 - x[asm.s_dof(prm, c)]
        prod = props.wi[c] * r0 * S * S / prm.visc[ph] * (x[asm.p_dof(prm, c)] - props.pbhp[c])
        total = F[prm.nu_dofs + ph::2].sum()
        assert total == pytest.approx(-q.sum() + prod, rel=1e-9)


@pytest.mark.parametrize("mobile", [0, 1])
def test_hydrostatic_column_has_no_flow(mobile):
    """Only one phase mobile (s = 1 or s = 0), its pressure in discrete hydrostatic balance
    p_K = p_L + (rho(p_K) + rho(p_L)) g / 2 for K below L, and x_old = x: every mass
    residual vanishes."""
    prm, props, x = random_case(2, 2, 5, 6, wells=False)
    s = 1.0 if mobile == 0 else 0.0
    x[prm.nu_dofs::2] = s
    for cy in range(prm.ny):
        for cx in range(prm.nx):
            p = prm.p_ref
            for cz in range(prm.nz - 1, -1, -1):
                c = asm.cell_index(prm, cx, cy, cz)
                if cz < prm.nz - 1:
                    pl = p
                    for _ in range(60):     # fixed point for the implicit density average
                        p = pl + 0.5 * (prm.rho0[mobile] * math.exp(prm.comp[mobile] * (p - prm.p_ref))
                                        + prm.rho0[mobile] * math.exp(prm.comp[mobile] * (pl - prm.p_ref))) * prm.grav
                x[asm.p_dof(prm, c)] = p
    F = asm.residual(prm, props, x, x)
    flow = F[prm.nu_dofs:]
    T = props.perm.max()
    scale = T * prm.rho0[mobile] / prm.visc[mobile] * 1e5
    assert np.abs(flow).max() <= 1e-12 * scale
    # the same state with gravity's sign flipped is far from balance
    x2 = x.copy()
    prm.grav = -prm.grav
    F2 = asm.residual(prm, props, x2, x2)
    assert np.abs(F2[prm.nu_dofs:]).max() > 1e3 * 1e-12 * scale


def test_uniform_pressure_biot_load():
    """u = 0, no gravity, uniform p, no Dirichlet dofs: the momentum residual is
    -(div eta, b p): zero at interior nodes, +b p (face area share) at nodes of the
    x = 0 face in x, -b p at nodes of the x = nx face."""
    prm, props, x = random_case(3, 3, 2, 7, wells=False, fixed=False, u_scale=0.0, grav=0.0)
    p0 = 2.0e7
    x[prm.nu_dofs + 1::2] = p0
    F = asm.residual(prm, props, x, x)
    Fu = F[: prm.nu_dofs].reshape(-1, 3)
    nd = np.arange(prm.nnode)
    ix = nd % (prm.nx + 1)
    iy = (nd // (prm.nx + 1)) % (prm.ny + 1)
    iz = nd // ((prm.nx + 1) * (prm.ny + 1))
    interior = (ix > 0) & (ix < prm.nx) & (iy > 0) & (iy < prm.ny) & (iz > 0) & (iz < prm.nz)
    assert np.abs(Fu[interior]).max() <= 1e-9 * p0
    face_mid = (ix == 0) & (iy > 0) & (iy < prm.ny) & (iz > 0) & (iz < prm.nz)
    assert np.allclose(Fu[face_mid, 0], prm.biot * p0, rtol=1e-14)
    face_mid = (ix == prm.nx) & (iy > 0) & (iy < prm.ny) & (iz > 0) & (iz < prm.nz)
    assert np.allclose(Fu[face_mid, 0], -prm.biot * p0, rtol=1e-14)
    assert np.allclose(Fu.sum(axis=0), 0.0, atol=1e-9 * p0)


# ---------------------------------------------------------------------------------------
# Against the independently written generator assembly (same model at u = 0)
# ---------------------------------------------------------------------------------------
def generator_case(nx=4, ny=3, nz=3, seed=11):
    w = pm.two_phase(nx, ny, nz, seed=seed, corr_len=2.0)
    prm = asm.Params(nx, ny, nz)
    props = asm.Props(w.meta["perm"], w.meta["young"], w.fixed.copy())
    x = np.zeros(prm.n)
    x[prm.nu_dofs::2] = w.meta["state"]["S_w"]
    x[prm.nu_dofs + 1::2] = w.meta["state"]["p"]
    return w, prm, props, x


def test_jacobian_matches_generator_at_zero_displacement():
    """The input generator assembles the same model's Jacobian with the density's pressure
    derivative left out of the mixture weight and of the averaged density in the
    potential.  Every other entry must agree to rounding; those two entry classes (momentum
    z rows x pressure columns, mass rows x pressure columns) agree to their size."""
    w, prm, props, x = generator_case()
    J = asm.jacobian(prm, props, x).toarray()
    G = w.scipy().toarray()
    # pattern: every nonzero of the derivative is structural in the generator
    Gs = w.scipy()
    struct = np.zeros_like(J, dtype=bool)
    for r in range(prm.n):
        struct[r, Gs.indices[Gs.indptr[r]:Gs.indptr[r + 1]]] = True
    assert not np.any((J != 0) & ~struct)
    nu = prm.nu_dofs
    pcol = np.zeros(prm.n, dtype=bool)
    pcol[nu + 1::2] = True
    zrow = np.zeros(prm.n, dtype=bool)
    zrow[2:nu:3] = True
    frow = np.zeros(prm.n, dtype=bool)
    frow[nu:] = True
    loose = (zrow[:, None] & pcol[None, :]) | (frow[:, None] & pcol[None, :])
    rowmax = np.abs(G).max(axis=1, keepdims=True)
    err = np.abs(J - G)
    assert np.all(err[~loose] <= 1e-13 * np.broadcast_to(rowmax, J.shape)[~loose])
    assert np.all(err[loose] <= 1e-5 * np.abs(G[loose]) + 1e-13 * np.broadcast_to(rowmax, J.shape)[loose])
    # and the loose classes really differ a little (the terms are present)
    assert err[loose].max() > 0


# ---------------------------------------------------------------------------------------
# Newton time step
# ---------------------------------------------------------------------------------------
def test_newton_converges_quadratically():
    prm, props, x = random_case(3, 3, 2, 8, p_noise=2e4, dt=3600.0)
    x_old = x.copy()
    st = None
    x1, st = onew.time_step(prm, props, x_old, onew.NewtonOpts(tol_flow=1e-12, tol_mech=1e-15,
                                                               max_newton=10))
    assert st.converged
    m = st.merit
    # once close, the merit falls at least quadratically (up to a constant)
    tail = [v for v in m if v < 1e-2 * m[0]]
    for a, b in zip(tail, tail[1:]):
        if b > 1e-13:
            assert b <= 50.0 * a * a / m[0] + 1e-13, m
    F = asm.residual(prm, props, x1, x_old)
    _, parts = asm.normalised(prm, props, F)
    assert parts[1][1] <= 1e-12 and parts[2][1] <= 1e-12


def test_newton_step_conserves_injected_mass():
    """After a converged step, the mass gained by each phase equals dt times the net
    source (wells) up to the Newton tolerance."""
    prm, props, x = random_case(3, 3, 2, 9, p_noise=2e4, dt=3600.0)
    x1, st = onew.time_step(prm, props, x, onew.NewtonOpts(tol_flow=1e-11, tol_mech=1e-14))
    assert st.converged
    F = asm.residual(prm, props, x1, x)
    # residual summed over cells = mass change / dt - net source; it is ~0 at convergence
    for ph in (0, 1):
        total = F[prm.nu_dofs + ph::2].sum() * prm.dt / (prm.phi0 * prm.rho0[ph])
        assert abs(total) <= 1e-9

"""Residual F(x) and Jacobian A(x) = dF/dx of two-phase poromechanics on unit cubes.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle; see the package docstring.

What is computed: the fully discrete nonlinear system of Sec. 3 (eq. IBVP_G, written as
F(x_n) = 0 in eq. IBVP_G_res) for the displacement / wetting-saturation / pressure model
of Sec. 2 (no capillarity, so both phases share p), and its exact Jacobian (Sec. 4,
eq. newton and eq. block_linear_system).  The space discretisation is the one Sec. 3
names: continuous trilinear (Q1) displacement, cell-wise constant s and p, two-point flux
approximation with first-order upwinding, backward Euler in time.  The constitutive
choices the paper leaves open are this model's own:

  * cells are unit cubes (x fastest, then y, then z); gravity points along -z;
  * Q1 element stiffness of an isotropic cell (Young's modulus E_c, Poisson ratio nu) by
    2x2x2 Gauss quadrature (`unit_stiffness`);
  * porosity phi = phi0 + b * eps_v(u), eps_v the integral of div u over the cell;
  * mixture weight rho g of eq. momentumBalanceS with the reference porosity:
    rho_mix = (1 - phi0) rho_s + phi0 (rho_w s + rho_nw (1 - s));
  * rho_l(p) = rho0_l exp(c_l (p - p_ref)), constant viscosities, Corey exponent 2:
    k_rw = max(s, 0)^2, k_rnw = max(1 - s, 0)^2, lambda_l = k_rl / mu_l;
  * face transmissibility T = 2 k_K k_L / (k_K + k_L) (unit area and distance); phase
    potential difference dPhi = p_K - p_L + (rho_K + rho_L)/2 g (z_K - z_L); the upwind
    cell is K when dPhi >= 0 (K the lower cell index), else L;
  * wells: fixed mass injection per cell and phase, and pressure-controlled producers
    q_l = -WI rho_l lambda_l (p - p_bhp) (both optional per cell);
  * a mass-balance row is accumulation + outflow - source (the sign convention of a
    residual whose Newton correction solves A dx = -F);
  * Dirichlet displacement dofs are fixed at zero: every residual uses the displacement
    with those dofs zeroed, and the row of a fixed dof is K_dd u_d with K_dd the assembled
    stiffness diagonal (so the Jacobian has that row and column eliminated, diagonal kept).

Unknown order: every displacement dof (node-major, x/y/z interleaved), then (s, p) per
cell.  Rows: momentum balance per displacement dof, then per cell the wetting-phase mass
balance (eq. IBVP_Gw) and the non-wetting-phase mass balance (eq. IBVP_Gnw).

Pins (tests/test_oracle_assembly.py): the stiffness against an independent Voigt-form
construction and its rigid-body null space; the Jacobian against central finite
differences of the residual; telescoping of the fluxes (global mass balance); a discrete
hydrostatic state with zero flow residual; the momentum residual of a uniform pressure;
and the Jacobian against an independently written assembly of the same model at u = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Params:
    """Grid and physical constants (SI units)."""
    nx: int
    ny: int
    nz: int
    nu: float = 0.25
    phi0: float = 0.2
    biot: float = 1.0
    grav: float = 9.81
    p_ref: float = 1.0e7
    rho_solid: float = 2650.0
    rho0: tuple = (1000.0, 800.0)      # wetting, non-wetting
    comp: tuple = (4.5e-10, 1.0e-9)
    visc: tuple = (1.0e-3, 5.0e-3)
    dt: float = 86400.0

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    @property
    def nnode(self):
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def nu_dofs(self):
        return 3 * self.nnode

    @property
    def n(self):
        return self.nu_dofs + 2 * self.ncell


@dataclass
class Props:
    """Per-cell permeability (m^2) and Young's modulus (Pa), fixed displacement dofs, and
    the wells (arrays of ncell; zero means no well)."""
    perm: np.ndarray
    young: np.ndarray
    fixed: np.ndarray
    wi: np.ndarray = None
    pbhp: np.ndarray = None
    qw: np.ndarray = None
    qo: np.ndarray = None

    def __post_init__(self):
        nc = self.perm.shape[0]
        for name in ("wi", "pbhp", "qw", "qo"):
            if getattr(self, name) is None:
                setattr(self, name, np.zeros(nc))


# ----------------------------------------------------------------------------------------
# Element matrices
# ----------------------------------------------------------------------------------------
def _shape_grad(a, xi):
    """Gradient of the trilinear shape function of local node a = ax + 2 ay + 4 az at the
    point xi of the unit cube."""
    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
    f = [xi[d] if (ax, ay, az)[d] else 1.0 - xi[d] for d in range(3)]
    s = [1.0 if (ax, ay, az)[d] else -1.0 for d in range(3)]
    return np.array([s[0] * f[1] * f[2], f[0] * s[1] * f[2], f[0] * f[1] * s[2]])


def unit_stiffness(nu):
    """24x24 Q1 stiffness of the unit cube for E = 1: with Lame constants lam, mu,
    K[3a+i, 3b+j] = sum over the 8 Gauss points (weight 1/8) of
    lam dN_a/dx_i dN_b/dx_j + mu dN_a/dx_j dN_b/dx_i + mu delta_ij grad N_a . grad N_b."""
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    g = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
    K = np.zeros((24, 24))
    for gz in g:
        for gy in g:
            for gx in g:
                G = [_shape_grad(a, (gx, gy, gz)) for a in range(8)]
                for a in range(8):
                    for b in range(8):
                        dot = float(G[a] @ G[b])
                        for i in range(3):
                            for j in range(3):
                                v = lam * G[a][i] * G[b][j] + mu * G[a][j] * G[b][i]
                                if i == j:
                                    v += mu * dot
                                K[3 * a + i, 3 * b + j] += 0.125 * v
    return K


def grad_integral():
    """Gint[a, i] = integral over the unit cube of dN_a/dx_i, by the same quadrature."""
    g = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
    G = np.zeros((8, 3))
    for gz in g:
        for gy in g:
            for gx in g:
                for a in range(8):
                    G[a] += 0.125 * _shape_grad(a, (gx, gy, gz))
    return G


# ----------------------------------------------------------------------------------------
# Grid helpers
# ----------------------------------------------------------------------------------------
def cell_index(prm, cx, cy, cz):
    return cx + prm.nx * (cy + prm.ny * cz)


def node_index(prm, ix, iy, iz):
    return ix + (prm.nx + 1) * (iy + (prm.ny + 1) * iz)


def cell_coords(prm, c):
    return c % prm.nx, (c // prm.nx) % prm.ny, c // (prm.nx * prm.ny)


def cell_nodes(prm, c):
    """The 8 nodes of cell c in local order a = ax + 2 ay + 4 az."""
    cx, cy, cz = cell_coords(prm, c)
    return [node_index(prm, cx + (a & 1), cy + ((a >> 1) & 1), cz + ((a >> 2) & 1))
            for a in range(8)]


def faces(prm):
    """Interior faces as (K, L, z_K - z_L) with K < L."""
    out = []
    for c in range(prm.ncell):
        cx, cy, cz = cell_coords(prm, c)
        if cx + 1 < prm.nx:
            out.append((c, c + 1, 0.0))
        if cy + 1 < prm.ny:
            out.append((c, c + prm.nx, 0.0))
        if cz + 1 < prm.nz:
            out.append((c, c + prm.nx * prm.ny, -1.0))
    return out


def s_dof(prm, c):
    return prm.nu_dofs + 2 * c


def p_dof(prm, c):
    return prm.nu_dofs + 2 * c + 1


# ----------------------------------------------------------------------------------------
# Constitutive functions
# ----------------------------------------------------------------------------------------
def density(prm, ph, p):
    """rho_l(p) and d rho_l / dp."""
    r = prm.rho0[ph] * math.exp(prm.comp[ph] * (p - prm.p_ref))
    return r, prm.comp[ph] * r


def phase_sat(ph, s):
    """Saturation of phase ph (0 wetting, 1 non-wetting) and its derivative in s."""
    return (s, 1.0) if ph == 0 else (1.0 - s, -1.0)


def mobility(prm, ph, s):
    """lambda_l = max(S_l, 0)^2 / mu_l and d lambda_l / ds."""
    S, dS = phase_sat(ph, s)
    Sp = max(S, 0.0)
    return Sp * Sp / prm.visc[ph], 2.0 * Sp * dS / prm.visc[ph]


def transmissibility(kK, kL):
    return 2.0 * kK * kL / (kK + kL)


def _masked_u(prm, props, x):
    u = np.array(x[: prm.nu_dofs], dtype=np.float64)
    u[props.fixed] = 0.0
    return u


def vol_strain(prm, u, c, Gint):
    nodes = cell_nodes(prm, c)
    return sum(Gint[a, i] * u[3 * nodes[a] + i] for a in range(8) for i in range(3))


def stiffness_diagonal(prm, props, K):
    d = np.zeros(prm.nu_dofs)
    for c in range(prm.ncell):
        for a, nd in enumerate(cell_nodes(prm, c)):
            for i in range(3):
                d[3 * nd + i] += props.young[c] * K[3 * a + i, 3 * a + i]
    return d


# ----------------------------------------------------------------------------------------
# Residual
# ----------------------------------------------------------------------------------------
def residual(prm: Params, props: Props, x, x_old):
    """F(x) for the time step from x_old to x (eq. IBVP_G_res)."""
    K = unit_stiffness(prm.nu)
    Gint = grad_integral()
    F = np.zeros(prm.n)
    u = _masked_u(prm, props, x)
    u_old = _masked_u(prm, props, x_old)

    # momentum balance (eq. IBVP_Gu): elastic + Biot + mixture weight, element by element
    for c in range(prm.ncell):
        nodes = cell_nodes(prm, c)
        dofs = [3 * nd + i for nd in nodes for i in range(3)]
        F[dofs] += props.young[c] * (K @ u[dofs])
        s, p = x[s_dof(prm, c)], x[p_dof(prm, c)]
        rw, _ = density(prm, 0, p)
        ro, _ = density(prm, 1, p)
        rho_mix = (1.0 - prm.phi0) * prm.rho_solid + prm.phi0 * (rw * s + ro * (1.0 - s))
        for a in range(8):
            for i in range(3):
                F[3 * nodes[a] + i] += -prm.biot * Gint[a, i] * p
                if i == 2:
                    F[3 * nodes[a] + i] += prm.grav * rho_mix / 8.0
    kdiag = stiffness_diagonal(prm, props, K)
    F[: prm.nu_dofs][props.fixed] = kdiag[props.fixed] * np.asarray(x[: prm.nu_dofs])[props.fixed]

    # mass balances (eq. IBVP_Gw, IBVP_Gnw): accumulation
    for c in range(prm.ncell):
        s, p = x[s_dof(prm, c)], x[p_dof(prm, c)]
        so, po = x_old[s_dof(prm, c)], x_old[p_dof(prm, c)]
        phi = prm.phi0 + prm.biot * vol_strain(prm, u, c, Gint)
        phi_o = prm.phi0 + prm.biot * vol_strain(prm, u_old, c, Gint)
        for ph in (0, 1):
            r, _ = density(prm, ph, p)
            ro_, _ = density(prm, ph, po)
            S, _ = phase_sat(ph, s)
            So, _ = phase_sat(ph, so)
            F[prm.nu_dofs + 2 * c + ph] += (phi * r * S - phi_o * ro_ * So) / prm.dt
    # outflow across interior faces
    for K_, L_, dz in faces(prm):
        T = transmissibility(props.perm[K_], props.perm[L_])
        pK, pL = x[p_dof(prm, K_)], x[p_dof(prm, L_)]
        sK, sL = x[s_dof(prm, K_)], x[s_dof(prm, L_)]
        for ph in (0, 1):
            rK, _ = density(prm, ph, pK)
            rL, _ = density(prm, ph, pL)
            dphi = pK - pL + 0.5 * (rK + rL) * prm.grav * dz
            if dphi >= 0.0:
                lam, _ = mobility(prm, ph, sK)
                flux = T * rK * lam * dphi
            else:
                lam, _ = mobility(prm, ph, sL)
                flux = T * rL * lam * dphi
            F[prm.nu_dofs + 2 * K_ + ph] += flux
            F[prm.nu_dofs + 2 * L_ + ph] -= flux
    # sources
    for c in range(prm.ncell):
        s, p = x[s_dof(prm, c)], x[p_dof(prm, c)]
        for ph, qinj in ((0, props.qw[c]), (1, props.qo[c])):
            q = qinj
            if props.wi[c] != 0.0:
                r, _ = density(prm, ph, p)
                lam, _ = mobility(prm, ph, s)
                q -= props.wi[c] * r * lam * (p - props.pbhp[c])
            F[prm.nu_dofs + 2 * c + ph] -= q
    return F


# ----------------------------------------------------------------------------------------
# Jacobian
# ----------------------------------------------------------------------------------------
def jacobian(prm: Params, props: Props, x):
    """A(x) = dF/dx as a scipy CSR matrix holding only the entries the derivative makes
    nonzero (the structural pattern is the caller's concern)."""
    K = unit_stiffness(prm.nu)
    Gint = grad_integral()
    u = _masked_u(prm, props, x)
    J = {}

    def add(r, c, v):
        J[(r, c)] = J.get((r, c), 0.0) + v

    for c in range(prm.ncell):
        nodes = cell_nodes(prm, c)
        dofs = [3 * nd + i for nd in nodes for i in range(3)]
        E = props.young[c]
        for al in range(24):
            for be in range(24):
                add(dofs[al], dofs[be], E * K[al, be])
        s, p = x[s_dof(prm, c)], x[p_dof(prm, c)]
        rw, drw = density(prm, 0, p)
        ro, dro = density(prm, 1, p)
        d_rho_mix_dp = prm.phi0 * (drw * s + dro * (1.0 - s))
        d_rho_mix_ds = prm.phi0 * (rw - ro)
        for a in range(8):
            for i in range(3):
                row = 3 * nodes[a] + i
                vp = -prm.biot * Gint[a, i]
                if i == 2:
                    vp += prm.grav * d_rho_mix_dp / 8.0
                    add(row, s_dof(prm, c), prm.grav * d_rho_mix_ds / 8.0)
                add(row, p_dof(prm, c), vp)
        # accumulation
        phi = prm.phi0 + prm.biot * vol_strain(prm, u, c, Gint)
        for ph in (0, 1):
            row = prm.nu_dofs + 2 * c + ph
            r, dr = density(prm, ph, p)
            S, dS = phase_sat(ph, s)
            for a in range(8):
                for i in range(3):
                    add(row, 3 * nodes[a] + i, prm.biot * Gint[a, i] * r * S / prm.dt)
            add(row, p_dof(prm, c), phi * dr * S / prm.dt)
            add(row, s_dof(prm, c), phi * r * dS / prm.dt)
    # fluxes
    for K_, L_, dz in faces(prm):
        T = transmissibility(props.perm[K_], props.perm[L_])
        pK, pL = x[p_dof(prm, K_)], x[p_dof(prm, L_)]
        sK, sL = x[s_dof(prm, K_)], x[s_dof(prm, L_)]
        for ph in (0, 1):
            rK, drK = density(prm, ph, pK)
            rL, drL = density(prm, ph, pL)
            dphi = pK - pL + 0.5 * (rK + rL) * prm.grav * dz
            ddphi_dpK = 1.0 + 0.5 * drK * prm.grav * dz
            ddphi_dpL = -1.0 + 0.5 * drL * prm.grav * dz
            if dphi >= 0.0:
                lam, dlam = mobility(prm, ph, sK)
                m = T * rK * lam
                d = {p_dof(prm, K_): m * ddphi_dpK + T * drK * lam * dphi,
                     p_dof(prm, L_): m * ddphi_dpL,
                     s_dof(prm, K_): T * rK * dlam * dphi}
            else:
                lam, dlam = mobility(prm, ph, sL)
                m = T * rL * lam
                d = {p_dof(prm, K_): m * ddphi_dpK,
                     p_dof(prm, L_): m * ddphi_dpL + T * drL * lam * dphi,
                     s_dof(prm, L_): T * rL * dlam * dphi}
            for col, v in d.items():
                add(prm.nu_dofs + 2 * K_ + ph, col, v)
                add(prm.nu_dofs + 2 * L_ + ph, col, -v)
    # producers
    for c in range(prm.ncell):
        if props.wi[c] == 0.0:
            continue
        s, p = x[s_dof(prm, c)], x[p_dof(prm, c)]
        for ph in (0, 1):
            r, dr = density(prm, ph, p)
            lam, dlam = mobility(prm, ph, s)
            dp = p - props.pbhp[c]
            row = prm.nu_dofs + 2 * c + ph
            add(row, p_dof(prm, c), props.wi[c] * (dr * lam * dp + r * lam))
            add(row, s_dof(prm, c), props.wi[c] * r * dlam * dp)
    # Dirichlet elimination: fixed rows keep only the diagonal, fixed columns are dropped
    fixed = np.zeros(prm.n, dtype=bool)
    fixed[: prm.nu_dofs] = props.fixed
    rows, cols, vals = [], [], []
    for (r, c), v in J.items():
        if (fixed[r] or fixed[c]) and r != c:
            continue
        rows.append(r)
        cols.append(c)
        vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(prm.n, prm.n))


# ----------------------------------------------------------------------------------------
# Normalised residual norms
# ----------------------------------------------------------------------------------------
def normalised(prm: Params, props: Props, F):
    """The residual in state units: momentum rows divided by the largest Young's modulus
    (a displacement), mass rows of phase l multiplied by dt / (phi0 rho0_l) (a saturation
    change).  Returns (vector, [sum of squares, max |.|] for u, wetting and non-wetting
    rows)."""
    Fh = np.array(F, dtype=np.float64)
    Fh[: prm.nu_dofs] /= float(np.max(props.young))
    for ph in (0, 1):
        Fh[prm.nu_dofs + ph::2] *= prm.dt / (prm.phi0 * prm.rho0[ph])
    parts = [Fh[: prm.nu_dofs], Fh[prm.nu_dofs::2], Fh[prm.nu_dofs + 1::2]]
    return Fh, [(float(np.sum(v * v)), float(np.max(np.abs(v))) if v.size else 0.0)
                for v in parts]

"""Seeded synthetic Jacobians of fully implicit multiphase poromechanics.

This module only produces inputs.  It assembles, at a random state, the monolithic
displacement / saturation / pressure Jacobian that the multigrid-reduction method is
applied to, following the model of the paper's Sec. 2-4: quasi-static linear momentum
balance with Biot coupling and the mixture self-weight, one mass balance per fluid phase
(no capillarity, so all phases share the pressure p), Q1 trilinear finite elements for the
displacement, piecewise-constant cell unknowns with a two-point flux approximation and
first-order upwinding, backward Euler in time, and the 3x3 block structure of the
`block_linear_system` equation.  It holds none of the preconditioner's arithmetic.

The detailed sub-block expressions of the paper's simulator are published elsewhere and
are not reproduced; the choices below (unit cubes, rate-form mass balances, Corey
exponent 2, harmonic transmissibility, the boundary conditions) are this generator's own
recipe.

Unknown ordering: every displacement dof first (node-major, x/y/z interleaved), then the
cell unknowns interleaved per cell, e.g. (s, p) for two phases.  Labels:
0 = displacement, 1 = (water) saturation, 2 = pressure, 3 = gas saturation.

Equations: the row of a saturation unknown is the mass balance of that saturation's phase
and the pressure row is the mass balance of the remaining phase (the non-wetting phase
for two phases, oil for three phases), as in the `IBVP_Gw` / `IBVP_Gnw` equations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GRAV = 9.81            # m/s^2, gravity points in -z
P_REF = 1.0e7          # Pa
PHI0 = 0.2             # reference porosity
BIOT = 1.0             # Biot coefficient
DT = 86400.0           # one day, s

PHASE = {
    "w": dict(rho0=1000.0, c=4.5e-10, mu=1.0e-3),
    "o": dict(rho0=800.0, c=1.0e-9, mu=5.0e-3),
    "g": dict(rho0=200.0, c=1.0e-7, mu=2.0e-5),
}

LABEL_U, LABEL_S, LABEL_P, LABEL_SG = 0, 1, 2, 3

# Cell-unknown models: slot labels, equation phases (one per slot, in slot order), and
# dS_phase/d(slot) for every phase (pressure slot has zero entries).
MODELS = {
    # single-phase Biot: one pressure unknown per cell, water mass balance, k_r = 1
    "biot1": dict(slots=[LABEL_P], eq_phase=["w"], dS={"w": [0.0]}, sat={"w": "one"},
                  gravity=False),
    # two-phase water/oil: (s_w, p); rows = water mass, oil mass
    "two": dict(slots=[LABEL_S, LABEL_P], eq_phase=["w", "o"],
                dS={"w": [1.0, 0.0], "o": [-1.0, 0.0]}, sat=None, gravity=True),
    # three-phase water/gas/oil: (s_w, s_g, p); rows = water, gas, oil mass
    "three": dict(slots=[LABEL_S, LABEL_SG, LABEL_P], eq_phase=["w", "g", "o"],
                  dS={"w": [1.0, 0.0, 0.0], "g": [0.0, 1.0, 0.0], "o": [-1.0, -1.0, 0.0]},
                  sat=None, gravity=True),
}


@dataclass
class Workload:
    """A Jacobian in CSR form plus the per-row unknown-type labels."""
    name: str
    nx: int
    ny: int
    nz: int
    model: str
    indptr: np.ndarray     # int64, n+1
    indices: np.ndarray    # int32, nnz, sorted and unique within a row
    data: np.ndarray       # float64, nnz
    labels: np.ndarray     # int8, n
    b: np.ndarray          # float64 right-hand side = A @ x_true
    x_true: np.ndarray     # float64
    fixed: np.ndarray      # bool over displacement dofs (Dirichlet)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


# ----------------------------------------------------------------------------------------
# Mechanics: Q1 element stiffness of a unit cube (E = 1), 2x2x2 Gauss quadrature
# ----------------------------------------------------------------------------------------
def q1_unit_stiffness(nu: float) -> np.ndarray:
    """24x24 stiffness of the unit cube for E = 1; dof 3a+i = (local node a, component i),
    local node a = ax + 2 ay + 4 az."""
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    g = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    K = np.zeros((24, 24))
    for gz in g:
        for gy in g:
            for gx in g:
                B = np.zeros((6, 24))
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    lx = gx if ax else 1.0 - gx
                    ly = gy if ay else 1.0 - gy
                    lz = gz if az else 1.0 - gz
                    dx = (1.0 if ax else -1.0) * ly * lz
                    dy = lx * (1.0 if ay else -1.0) * lz
                    dz = lx * ly * (1.0 if az else -1.0)
                    c = 3 * a
                    B[0, c] = dx
                    B[1, c + 1] = dy
                    B[2, c + 2] = dz
                    B[3, c + 1], B[3, c + 2] = dz, dy
                    B[4, c], B[4, c + 2] = dz, dx
                    B[5, c], B[5, c + 1] = dy, dx
                K += 0.125 * B.T @ D @ B
    return K


def q1_unit_grad_integral() -> np.ndarray:
    """G[a, i] = integral over the unit cube of dN_a/dx_i (exactly +-1/4)."""
    G = np.zeros((8, 3))
    for a in range(8):
        for i in range(3):
            G[a, i] = 0.25 if (a >> i) & 1 else -0.25
    return G


# ----------------------------------------------------------------------------------------
# Random fields
# ----------------------------------------------------------------------------------------
def gaussian_field(rng: np.random.Generator, shape, corr_len: float) -> np.ndarray:
    """Unit-variance stationary Gaussian field with exponential covariance exp(-r/corr_len)
    (r in cells), by spectral synthesis on a periodic grid padded 2x, then cropped."""
    pad = tuple(2 * s for s in shape)
    axes = [np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64) for n in pad]
    r2 = axes[0][:, None, None] ** 2 + axes[1][None, :, None] ** 2 + axes[2][None, None, :] ** 2
    cov = np.exp(-np.sqrt(r2) / corr_len)
    del r2
    lam = np.maximum(np.fft.rfftn(cov).real, 0.0)
    del cov
    white = rng.standard_normal(pad)
    f = np.fft.irfftn(np.fft.rfftn(white) * np.sqrt(lam), s=pad, axes=(0, 1, 2))
    return np.ascontiguousarray(f[: shape[0], : shape[1], : shape[2]])


def channel_field(rng: np.random.Generator, shape, width: int = 4, fraction: float = 0.25,
                  max_amp: float = 16.0) -> np.ndarray:
    """Binary channel indicator (1 inside a channel): channels run along x and meander in y
    (sinusoidal centreline, random phase and amplitude), `width` cells wide, spaced so about
    `fraction` of the cells are channel, with a random y-offset per z-layer."""
    nz, ny, nx = shape
    spacing = max(width + 1, int(round(width / fraction)))
    nchan = max(1, ny // spacing)
    ind = np.zeros(shape, dtype=bool)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    for k in range(nz):
        yoff = rng.uniform(0.0, spacing)
        for c in range(nchan):
            amp = rng.uniform(0.0, max_amp)
            phase = rng.uniform(0.0, 2.0 * math.pi)
            wavelength = rng.uniform(0.5, 1.5) * nx
            yc = (yoff + c * spacing + amp * np.sin(2.0 * math.pi * x / wavelength + phase)) % ny
            d = np.abs(y[:, None] - yc[None, :])
            d = np.minimum(d, ny - d)
            ind[k] |= d < 0.5 * width
    return ind


# ----------------------------------------------------------------------------------------
# Assembly
# ----------------------------------------------------------------------------------------
def _phase_props(name, p):
    ph = PHASE[name]
    rho = ph["rho0"] * np.exp(ph["c"] * (p - P_REF))
    return rho, ph["c"], ph["mu"]


def assemble(name, nx, ny, nz, model, logk10, E, nu, rng, sat_ranges=None,
             dirichlet=True) -> Workload:
    """Assemble the Jacobian at a random state.  `logk10` and `E` are cell arrays of shape
    (nz, ny, nx); `nu` is a scalar.  Draws from `rng`: pressure noise, saturations, x_true."""
    M = MODELS[model]
    slots = M["slots"]
    nf = len(slots)
    p_slot = slots.index(LABEL_P)
    sat_slots = [e for e in range(nf) if e != p_slot]
    grav = GRAV if M["gravity"] else 0.0
    nnx, nny, nnz_ = nx + 1, ny + 1, nz + 1
    nnode = nnx * nny * nnz_
    ncell = nx * ny * nz
    Nu = 3 * nnode
    N = Nu + nf * ncell

    # ---- state ---------------------------------------------------------------------
    kk = np.arange(nz, dtype=np.float64)[:, None, None] + 0.5          # cell-centre height
    zc = np.broadcast_to(kk, (nz, ny, nx))
    p = P_REF + rng.normal(0.0, 1.0e5, size=(nz, ny, nx))
    if grav:
        p = p + PHASE["w"]["rho0"] * grav * (nz - zc)
    S = {}
    if model == "two":
        lo, hi = (sat_ranges or {}).get("s", (0.2, 0.8))
        s = rng.uniform(lo, hi, size=(nz, ny, nx))
        S["w"], S["o"] = s, 1.0 - s
    elif model == "three":
        lo, hi = (sat_ranges or {}).get("sw", (0.2, 0.5))
        sw = rng.uniform(lo, hi, size=(nz, ny, nx))
        lo, hi = (sat_ranges or {}).get("sg", (0.05, 0.3))
        sg = rng.uniform(lo, hi, size=(nz, ny, nx))
        S["w"], S["g"], S["o"] = sw, sg, 1.0 - sw - sg
    else:
        S["w"] = np.ones((nz, ny, nx))
    phases = list(M["dS"].keys())
    rho = {}
    comp = {}
    mu = {}
    for ph in phases:
        rho[ph], comp[ph], mu[ph] = _phase_props(ph, p)

    k = 10.0 ** logk10
    Kref = q1_unit_stiffness(nu)
    Gint = q1_unit_grad_integral()

    # ---- displacement-displacement blocks per (node, neighbour offset) ---------------
    blocks = np.zeros((nnz_, nny, nnx, 27, 3, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        for bb in range(8):
            bx, by, bz = bb & 1, (bb >> 1) & 1, (bb >> 2) & 1
            off = (bz - az + 1) * 9 + (by - ay + 1) * 3 + (bx - ax + 1)
            blocks[az:az + nz, ay:ay + ny, ax:ax + nx, off] += (
                E[..., None, None] * Kref[3 * a:3 * a + 3, 3 * bb:3 * bb + 3])
    blocks = blocks.reshape(nnode, 27, 3, 3)

    iz, iy, ix = np.meshgrid(np.arange(nnz_), np.arange(nny), np.arange(nnx), indexing="ij")
    iz, iy, ix = iz.ravel(), iy.ravel(), ix.ravel()
    node = np.arange(nnode)

    # neighbour nodes (27 offsets in ascending global index order)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    nb_valid = np.zeros((nnode, 27), dtype=bool)
    nb_idx = np.zeros((nnode, 27), dtype=np.int64)
    for o, (dx, dy, dz) in enumerate(offs):
        jx, jy, jz = ix + dx, iy + dy, iz + dz
        nb_valid[:, o] = (jx >= 0) & (jx < nnx) & (jy >= 0) & (jy < nny) & (jz >= 0) & (jz < nnz_)
        nb_idx[:, o] = jx + nnx * (jy + nny * jz)
    # u-u part of displacement rows: (node, i, o, j)
    uu_cols = (3 * nb_idx[:, None, :, None] + np.arange(3)[None, None, None, :])
    uu_cols = np.broadcast_to(uu_cols, (nnode, 3, 27, 3)).reshape(Nu, 81)
    uu_vals = blocks.transpose(0, 2, 1, 3).reshape(Nu, 81)
    uu_mask = np.broadcast_to(nb_valid[:, None, :, None], (nnode, 3, 27, 3)).reshape(Nu, 81)
    del blocks

    # cells adjacent to a node, ascending cell index: (dz, dy, dx) in {-1, 0}^3
    coffs = [(dx, dy, dz) for dz in (-1, 0) for dy in (-1, 0) for dx in (-1, 0)]
    uf_cols = np.zeros((nnode, 3, 8, nf), dtype=np.int64)
    uf_vals = np.zeros((nnode, 3, 8, nf))
    uf_mask = np.zeros((nnode, 3, 8, nf), dtype=bool)
    rho_mix_ds = {}
    for e in sat_slots:       # d(mixture density)/d(saturation slot e) / phi
        rho_mix_ds[e] = sum(rho[ph] * M["dS"][ph][e] for ph in phases)
    for c, (dx, dy, dz) in enumerate(coffs):
        cx, cy, cz = ix + dx, iy + dy, iz + dz
        valid = (cx >= 0) & (cx < nx) & (cy >= 0) & (cy < ny) & (cz >= 0) & (cz < nz)
        cell = np.where(valid, cx + nx * (cy + ny * cz), 0)
        a = (-dx) + 2 * (-dy) + 4 * (-dz)           # local index of this node in that cell
        for i in range(3):
            for e in range(nf):
                uf_cols[:, i, c, e] = Nu + nf * cell + e
            uf_vals[:, i, c, p_slot] = -BIOT * Gint[a, i]
            uf_mask[:, i, c, p_slot] = valid
            if grav and i == 2:
                for e in sat_slots:
                    rmd = rho_mix_ds[e].ravel()[cell]
                    uf_vals[:, i, c, e] = grav * PHI0 * rmd / 8.0
                    uf_mask[:, i, c, e] = valid
    uf_cols = uf_cols.reshape(Nu, 8 * nf)
    uf_vals = uf_vals.reshape(Nu, 8 * nf)
    uf_mask = uf_mask.reshape(Nu, 8 * nf)

    u_cols = np.concatenate([uu_cols, uf_cols], axis=1)
    u_vals = np.concatenate([uu_vals, uf_vals], axis=1)
    u_mask = np.concatenate([uu_mask, uf_mask], axis=1)
    del uu_cols, uu_vals, uu_mask, uf_cols, uf_vals, uf_mask

    # ---- flow: accumulation + TPFA upwind fluxes ---------------------------------------
    # blk7[cell, slot, eq, unknown]; slots -z,-y,-x,self,+x,+y,+z
    blk7 = np.zeros((nz, ny, nx, 7, nf, nf))
    eqs = M["eq_phase"]
    for r, ph in enumerate(eqs):
        for e in range(nf):
            if e == p_slot:
                blk7[..., 3, r, e] += PHI0 * comp[ph] * rho[ph] * S[ph] / DT
            else:
                blk7[..., 3, r, e] += PHI0 * rho[ph] * M["dS"][ph][e] / DT

    def lam_and_dlam(ph, sl):
        mu_ = mu[ph]
        if model == "biot1":
            return np.full(S[ph][sl].shape, 1.0 / mu_), [np.zeros(S[ph][sl].shape)] * nf
        sv = S[ph][sl]
        lam = sv * sv / mu_
        dl = [2.0 * sv / mu_ * M["dS"][ph][e] for e in range(nf)]
        return lam, dl

    dirs = [  # (slice K, slice L, slot of L seen from K, slot of K seen from L, dz)
        ((slice(None), slice(None), slice(0, nx - 1)), (slice(None), slice(None), slice(1, nx)), 4, 2, 0.0),
        ((slice(None), slice(0, ny - 1), slice(None)), (slice(None), slice(1, ny), slice(None)), 5, 1, 0.0),
        ((slice(0, nz - 1), slice(None), slice(None)), (slice(1, nz), slice(None), slice(None)), 6, 0, -1.0),
    ]
    for sK, sL, slotL, slotK, dzKL in dirs:
        kK, kL = k[sK], k[sL]
        T = 2.0 * kK * kL / (kK + kL)
        for r, ph in enumerate(eqs):
            rhoK, rhoL = rho[ph][sK], rho[ph][sL]
            dphi = (p[sK] - p[sL]) + 0.5 * (rhoK + rhoL) * grav * dzKL
            upK = dphi >= 0.0             # tie: the lower cell index (K) is upwind
            lamK, dlK = lam_and_dlam(ph, sK)
            lamL, dlL = lam_and_dlam(ph, sL)
            mob = np.where(upK, rhoK * lamK, rhoL * lamL) * T
            dK = [None] * nf
            dL = [None] * nf
            for e in range(nf):
                if e == p_slot:
                    dK[e] = mob + np.where(upK, comp[ph] * rhoK * lamK * T * dphi, 0.0)
                    dL[e] = -mob + np.where(upK, 0.0, comp[ph] * rhoL * lamL * T * dphi)
                else:
                    dK[e] = np.where(upK, rhoK * dlK[e] * T * dphi, 0.0)
                    dL[e] = np.where(upK, 0.0, rhoL * dlL[e] * T * dphi)
            for e in range(nf):
                blk7[sK + (3, r, e)] += dK[e]
                blk7[sK + (slotL, r, e)] += dL[e]
                blk7[sL + (slotK, r, e)] -= dK[e]
                blk7[sL + (3, r, e)] -= dL[e]

    cz_, cy_, cx_ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cz_, cy_, cx_ = cz_.ravel(), cy_.ravel(), cx_.ravel()
    cells = np.arange(ncell)
    # u part of flow rows: 8 nodes of the cell ascending, 3 components
    fu_cols = np.zeros((ncell, 8, 3), dtype=np.int64)
    fu_g = np.zeros((8, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        nd = (cx_ + ax) + nnx * ((cy_ + ay) + nny * (cz_ + az))
        for i in range(3):
            fu_cols[:, a, i] = 3 * nd + i
            fu_g[a, i] = Gint[a, i]
    fu_cols = fu_cols.reshape(ncell, 24)
    fcols = np.zeros((ncell, nf, 24 + 7 * nf), dtype=np.int64)
    fvals = np.zeros((ncell, nf, 24 + 7 * nf))
    fmask = np.zeros((ncell, nf, 24 + 7 * nf), dtype=bool)
    for r, ph in enumerate(eqs):
        coef = (rho[ph] * S[ph]).ravel() * BIOT / DT
        fcols[:, r, :24] = fu_cols
        fvals[:, r, :24] = coef[:, None] * fu_g.reshape(1, 24)
        fmask[:, r, :24] = True
    nbr = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    b7 = blk7.reshape(ncell, 7, nf, nf)
    for sl, (dx, dy, dz) in enumerate(nbr):
        jx, jy, jz = cx_ + dx, cy_ + dy, cz_ + dz
        valid = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny) & (jz >= 0) & (jz < nz)
        nc = np.where(valid, jx + nx * (jy + ny * jz), 0)
        for r in range(nf):
            for e in range(nf):
                col = 24 + sl * nf + e
                fcols[:, r, col] = Nu + nf * nc + e
                fvals[:, r, col] = b7[:, sl, r, e]
                fmask[:, r, col] = valid
    fcols = fcols.reshape(ncell * nf, 24 + 7 * nf)
    fvals = fvals.reshape(ncell * nf, 24 + 7 * nf)
    fmask = fmask.reshape(ncell * nf, 24 + 7 * nf)
    del blk7, b7

    # ---- Dirichlet displacement constraints -----------------------------------------------
    fixed = np.zeros((nnode, 3), dtype=bool)
    if dirichlet:
        fixed[iz == 0, :] = True                       # bottom: u = 0
        fixed[(ix == 0) | (ix == nx), 0] = True        # x-faces: u_x = 0
        fixed[(iy == 0) | (iy == ny), 1] = True        # y-faces: u_y = 0
    fixed = fixed.ravel()
    urow = np.arange(Nu)[:, None]
    colfix = (u_cols < Nu) & fixed[np.minimum(u_cols, Nu - 1)] & (u_cols != urow)
    rowfix = fixed[:, None] & (u_cols != urow)
    u_vals = np.where(colfix | rowfix, 0.0, u_vals)
    fcolfix = (fcols < Nu) & fixed[np.minimum(fcols, Nu - 1)]
    fvals = np.where(fcolfix, 0.0, fvals)

    # ---- compact to CSR -----------------------------------------------------------
    cnt = np.concatenate([u_mask.sum(axis=1), fmask.sum(axis=1)])
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(cnt, out=indptr[1:])
    indices = np.concatenate([u_cols[u_mask], fcols[fmask]]).astype(np.int32)
    data = np.concatenate([u_vals[u_mask], fvals[fmask]])
    del u_cols, u_vals, u_mask, fcols, fvals, fmask

    labels = np.empty(N, dtype=np.int8)
    labels[:Nu] = LABEL_U
    labels[Nu:] = np.tile(np.array(slots, dtype=np.int8), ncell)

    # ---- manufactured solution -------------------------------------------------------
    sig = {LABEL_U: 1.0e-3, LABEL_P: 1.0e5, LABEL_S: 1.0e-2, LABEL_SG: 1.0e-2}
    x_true = np.empty(N)
    xu = rng.normal(0.0, sig[LABEL_U], size=Nu)
    xu[fixed] = 0.0
    x_true[:Nu] = xu
    xf = rng.standard_normal(ncell * nf) * np.tile(np.array([sig[s] for s in slots]), ncell)
    x_true[Nu:] = xf

    import scipy.sparse as sp
    A = sp.csr_matrix((data, indices, indptr), shape=(N, N))
    b = A @ x_true

    meta = dict(nnode=nnode, ncell=ncell, Nu=Nu, nf=nf, slots=list(slots), model=model,
                nu=nu, gravity=bool(grav),
                # the state the Jacobian was taken at, and the cell properties
                state=dict(p=p.ravel().copy(), **{"S_" + ph: S[ph].ravel().copy() for ph in S}),
                perm=k.ravel().copy(), young=np.asarray(E, dtype=np.float64).ravel().copy())
    return Workload(name=name, nx=nx, ny=ny, nz=nz, model=model, indptr=indptr,
                    indices=indices, data=data, labels=labels, b=b, x_true=x_true,
                    fixed=fixed, meta=meta)


# ----------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------
def biot_single_phase(nx=8, ny=8, nz=8, seed=0) -> Workload:
    """Single-phase Biot: log10 k iid N(-13, 0.5^2) m^2, E = 10 GPa, nu = 0.25, dt = 1 day."""
    rng = np.random.default_rng(seed)
    logk = -13.0 + 0.5 * rng.standard_normal((nz, ny, nx))
    E = np.full((nz, ny, nx), 10.0e9)
    return assemble(f"biot1p_{nx}x{ny}x{nz}", nx, ny, nz, "biot1", logk, E, 0.25, rng)


def two_phase(nx=64, ny=64, nz=64, seed=1, corr_len=8.0) -> Workload:
    """Two-phase water/oil: log10 k ~ N(-13, 1) with exponential correlation `corr_len` cells,
    Corey exponent 2, s ~ U[0.2, 0.8], E = 10 GPa, nu = 0.25."""
    rng = np.random.default_rng(seed)
    logk = -13.0 + gaussian_field(rng, (nz, ny, nx), corr_len)
    E = np.full((nz, ny, nx), 10.0e9)
    return assemble(f"twophase_{nx}x{ny}x{nz}", nx, ny, nz, "two", logk, E, 0.25, rng)


def two_phase_channels(nx=128, ny=128, nz=64, seed=2) -> Workload:
    """Two-phase, high-contrast channels: binary channels 4 cells wide with permeability
    ratio 1e4 plus log10 N(0, 2^2) noise; nu = 0.3, E ~ U[1, 50] GPa per z-layer."""
    rng = np.random.default_rng(seed)
    ch = channel_field(rng, (nz, ny, nx))
    logk = np.where(ch, -11.0, -15.0) + 2.0 * rng.standard_normal((nz, ny, nx))
    Elayer = rng.uniform(1.0e9, 50.0e9, size=nz)
    E = np.broadcast_to(Elayer[:, None, None], (nz, ny, nx)).copy()
    return assemble(f"twophase_channels_{nx}x{ny}x{nz}", nx, ny, nz, "two", logk, E, 0.3, rng)


def three_phase(nx=96, ny=96, nz=96, seed=3) -> Workload:
    """Three-phase water/gas/oil: ln k ~ N(ln 1e-13, 1.5^2) with correlation length 12 cells,
    s_w ~ U[0.2, 0.5], s_g ~ U[0.05, 0.3], E = 10 GPa, nu = 0.25."""
    rng = np.random.default_rng(seed)
    lnk = math.log(1.0e-13) + 1.5 * gaussian_field(rng, (nz, ny, nx), 12.0)
    logk = lnk / math.log(10.0)
    E = np.full((nz, ny, nx), 10.0e9)
    return assemble(f"threephase_{nx}x{ny}x{nz}", nx, ny, nz, "three", logk, E, 0.25, rng)


def closed_form_nnz(nx, ny, nz, model) -> int:
    """Structural nonzero count of the Jacobian pattern this generator emits."""
    nf = len(MODELS[model]["slots"])
    nsat = nf - 1
    grav = MODELS[model]["gravity"]
    su = lambda n: 2 + 2 + (n - 1) * 3 if n >= 1 else 1   # noqa: E731  neighbours per axis
    pairs_uu = su(nx) * su(ny) * su(nz)
    ncell = nx * ny * nz
    node_cell = 8 * ncell
    faces = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    uu = 9 * pairs_uu
    uf = node_cell * (3 + (nsat if grav else 0))        # p on 3 rows, saturations on z rows
    fu = node_cell * 3 * nf
    ff = (ncell + 2 * faces) * nf * nf
    return uu + uf + fu + ff


# ----------------------------------------------------------------------------------------
# Time-stepping inputs: a channelised reservoir with a water line drive
# ----------------------------------------------------------------------------------------
def channel_reservoir(nx=32, ny=32, nz=8, seed=5, width=4, k_channel=-12.0,
                      k_background=-14.5, noise=0.3, days_to_half_pv=100.0):
    """Cell properties and the initial state of a two-phase time-stepping problem.

    Permeability: binary channels (`channel_field`) with log10 k = k_channel inside and
    k_background outside, plus N(0, noise^2) in log10.  Young's modulus U[5, 30] GPa per
    z-layer, Poisson ratio 0.25.  Bottom fixed, lateral faces on rollers.  Wells: water
    injected on the x = 0 column of cells at a total mass rate that puts half a pore volume
    in over `days_to_half_pv` days, split in proportion to k; producers on the x = nx - 1
    column with well index 2 k and bottom-hole pressure 0.2 MPa below the initial pressure.
    Initial state: u = 0, s = 0.15, p = p_ref + rho_o g (depth of the cell centre).
    Returns a dict of flat arrays in the model's unknown order."""
    rng = np.random.default_rng(seed)
    ch = channel_field(rng, (nz, ny, nx), width=width, fraction=0.3, max_amp=max(2.0, ny / 8))
    logk = np.where(ch, k_channel, k_background) + noise * rng.standard_normal((nz, ny, nx))
    k = 10.0 ** logk
    Elayer = rng.uniform(5.0e9, 30.0e9, size=nz)
    E = np.broadcast_to(Elayer[:, None, None], (nz, ny, nx)).copy()
    nnx, nny, nnz_ = nx + 1, ny + 1, nz + 1
    nnode = nnx * nny * nnz_
    iz, iy, ix = np.meshgrid(np.arange(nnz_), np.arange(nny), np.arange(nnx), indexing="ij")
    iz, iy, ix = iz.ravel(), iy.ravel(), ix.ravel()
    fixed = np.zeros((nnode, 3), dtype=bool)
    fixed[iz == 0, :] = True
    fixed[(ix == 0) | (ix == nx), 0] = True
    fixed[(iy == 0) | (iy == ny), 1] = True
    ncell = nx * ny * nz
    cx = np.arange(ncell) % nx
    inj = cx == 0
    prod = cx == nx - 1
    pv = PHI0 * ncell
    q_total = 0.5 * pv * PHASE["w"]["rho0"] / (days_to_half_pv * DT)
    kf = k.ravel()
    qw = np.zeros(ncell)
    qw[inj] = q_total * kf[inj] / kf[inj].sum()
    zc = (np.arange(ncell) // (nx * ny)).astype(np.float64) + 0.5
    p0 = P_REF + PHASE["o"]["rho0"] * GRAV * (nz - zc)
    wi = np.zeros(ncell)
    wi[prod] = 2.0 * kf[prod]
    pbhp = np.where(prod, p0 - 2.0e5, 0.0)
    x0 = np.zeros(3 * nnode + 2 * ncell)
    x0[3 * nnode::2] = 0.15
    x0[3 * nnode + 1::2] = p0
    return dict(nx=nx, ny=ny, nz=nz, perm=kf.copy(), young=E.ravel().copy(),
                fixed=fixed.ravel(), wi=wi, pbhp=pbhp, qw=qw, qo=np.zeros(ncell), x0=x0,
                nu=0.25, dt=DT)

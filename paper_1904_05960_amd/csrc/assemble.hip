// Residual F(x) and Jacobian A(x) = dF/dx of two-phase poromechanics on a grid of unit
// cubes (Sec. 2-3, eq. IBVP_G and IBVP_G_res), and Newton's method with backtracking for
// one time step (Sec. 4, eq. newton) with the MGR-preconditioned FGMRES as linear solver.
//
// Discretisation: trilinear displacement (2x2x2 Gauss stiffness of a unit cube scaled by
// the cell's Young's modulus), cell-wise constant (s, p), two-point fluxes with harmonic
// transmissibility and first-order upwinding on the phase potential, backward Euler.
// Constitutive choices: porosity phi0 + b eps_v(u); mixture weight with the reference
// porosity; exponential densities; Corey exponent 2; fixed-rate injectors and
// pressure-controlled producers; Dirichlet displacement dofs fixed at zero.
//
// The library builds the Jacobian's pattern itself (rows of the displacement dofs node-major
// with x/y/z interleaved, then (s, p) per cell; columns sorted) and keeps it: every value
// position follows from the grid, so assembly writes each entry at a computed offset.
//   displacement row (node n, component i): the 27 neighbour nodes of n present in the grid
//     (ascending node index) x 3 components, then the cells around n (ascending) with the
//     (s, p) pair on z rows and p alone on x and y rows;
//   mass-balance row (cell c, phase e): the 8 nodes of c (ascending) x 3 components, then
//     the cells -z, -y, -x, c, +x, +y, +z present in the grid, each with (s, p).
// One thread per node computes the three momentum rows (element stiffness staged in LDS);
// one thread per cell computes both mass balances, computing each face flux on both sides
// with the same operations, so no atomics are needed and the result is deterministic.
#include <chrono>
#include <cmath>
#include <memory>

#include "common.hpp"

namespace mgr {
namespace {

struct PoroK {   // kernel-side copy of the parameters
  int nx, ny, nz;
  int64_t ncell, nnode, nu, n;
  double phi0, biot, grav, p_ref, rho_s, dt;
  double rho0[2], comp[2], visc[2];
};

__device__ __forceinline__ double gint(int a, int i) { return ((a >> i) & 1) ? 0.25 : -0.25; }

__device__ __forceinline__ void density(const PoroK &P, int ph, double p, double &r, double &dr) {
  r = P.rho0[ph] * exp(P.comp[ph] * (p - P.p_ref));
  dr = P.comp[ph] * r;
}

__device__ __forceinline__ void mobility(const PoroK &P, int ph, double s, double &l, double &dl) {
  const double S = ph == 0 ? s : 1.0 - s;
  const double dS = ph == 0 ? 1.0 : -1.0;
  const double Sp = S > 0.0 ? S : 0.0;
  l = Sp * Sp / P.visc[ph];
  dl = 2.0 * Sp * dS / P.visc[ph];
}

__device__ __forceinline__ int64_t node_id(const PoroK &P, int ix, int iy, int iz) {
  return ix + int64_t(P.nx + 1) * (iy + int64_t(P.ny + 1) * iz);
}
__device__ __forceinline__ int64_t cell_id(const PoroK &P, int cx, int cy, int cz) {
  return cx + int64_t(P.nx) * (cy + int64_t(P.ny) * cz);
}

// ---------------------------------------------------------------------------------------
// pattern
__global__ void k_row_len(PoroK P, int64_t *len) {
  const int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (r >= P.n) return;
  if (r < P.nu) {
    const int64_t nd = r / 3;
    const int i = int(r % 3);
    const int ix = int(nd % (P.nx + 1)), iy = int((nd / (P.nx + 1)) % (P.ny + 1));
    const int iz = int(nd / (int64_t(P.nx + 1) * (P.ny + 1)));
    const int nbx = 1 + (ix > 0) + (ix < P.nx), nby = 1 + (iy > 0) + (iy < P.ny);
    const int nbz = 1 + (iz > 0) + (iz < P.nz);
    const int ncx = (ix > 0) + (ix < P.nx), ncy = (iy > 0) + (iy < P.ny);
    const int ncz = (iz > 0) + (iz < P.nz);
    len[r] = 3 * nbx * nby * nbz + (i == 2 ? 2 : 1) * ncx * ncy * ncz;
  } else {
    const int64_t c = (r - P.nu) / 2;
    const int cx = int(c % P.nx), cy = int((c / P.nx) % P.ny), cz = int(c / (int64_t(P.nx) * P.ny));
    const int nb = 1 + (cx > 0) + (cx < P.nx - 1) + (cy > 0) + (cy < P.ny - 1) + (cz > 0) +
                   (cz < P.nz - 1);
    len[r] = 24 + 2 * nb;
  }
}

__global__ void k_fill_pattern(PoroK P, const int64_t *rp, int *ci, int8_t *labels) {
  const int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (r >= P.n) return;
  int64_t pos = rp[r];
  if (r < P.nu) {
    labels[r] = 0;
    const int64_t nd = r / 3;
    const int i = int(r % 3);
    const int ix = int(nd % (P.nx + 1)), iy = int((nd / (P.nx + 1)) % (P.ny + 1));
    const int iz = int(nd / (int64_t(P.nx + 1) * (P.ny + 1)));
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
          if (jx < 0 || jx > P.nx || jy < 0 || jy > P.ny || jz < 0 || jz > P.nz) continue;
          const int64_t m = node_id(P, jx, jy, jz);
          for (int j = 0; j < 3; ++j) ci[pos++] = int(3 * m + j);
        }
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int cx = ix + dx, cy = iy + dy, cz = iz + dz;
          if (cx < 0 || cx >= P.nx || cy < 0 || cy >= P.ny || cz < 0 || cz >= P.nz) continue;
          const int64_t c = cell_id(P, cx, cy, cz);
          if (i == 2) ci[pos++] = int(P.nu + 2 * c);
          ci[pos++] = int(P.nu + 2 * c + 1);
        }
  } else {
    const int64_t c = (r - P.nu) / 2;
    labels[r] = ((r - P.nu) & 1) ? 2 : 1;
    const int cx = int(c % P.nx), cy = int((c / P.nx) % P.ny), cz = int(c / (int64_t(P.nx) * P.ny));
    for (int a = 0; a < 8; ++a) {
      const int64_t m = node_id(P, cx + (a & 1), cy + ((a >> 1) & 1), cz + ((a >> 2) & 1));
      for (int j = 0; j < 3; ++j) ci[pos++] = int(3 * m + j);
    }
    const int off[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0},
                           {1, 0, 0},  {0, 1, 0},  {0, 0, 1}};
    for (int sl = 0; sl < 7; ++sl) {
      const int jx = cx + off[sl][0], jy = cy + off[sl][1], jz = cz + off[sl][2];
      if (jx < 0 || jx >= P.nx || jy < 0 || jy >= P.ny || jz < 0 || jz >= P.nz) continue;
      const int64_t nc = cell_id(P, jx, jy, jz);
      ci[pos++] = int(P.nu + 2 * nc);
      ci[pos++] = int(P.nu + 2 * nc + 1);
    }
  }
}

// ---------------------------------------------------------------------------------------
// constant displacement-displacement block and the stiffness diagonal
__global__ void k_uu_values(PoroK P, const int64_t *rp, const double *young, const double *K,
                            const uint8_t *fixed, double *val, double *kdiag) {
  const int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (r >= P.nu) return;
  const int64_t nd = r / 3;
  const int i = int(r % 3);
  const int ix = int(nd % (P.nx + 1)), iy = int((nd / (P.nx + 1)) % (P.ny + 1));
  const int iz = int(nd / (int64_t(P.nx + 1) * (P.ny + 1)));
  int64_t pos = rp[r];
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        if (jx < 0 || jx > P.nx || jy < 0 || jy > P.ny || jz < 0 || jz > P.nz) continue;
        const int64_t m = node_id(P, jx, jy, jz);
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          // cells holding both nodes, ascending cell index
          for (int cz = max(iz, jz) - 1; cz <= min(iz, jz); ++cz) {
            if (cz < 0 || cz >= P.nz) continue;
            for (int cy = max(iy, jy) - 1; cy <= min(iy, jy); ++cy) {
              if (cy < 0 || cy >= P.ny) continue;
              for (int cx = max(ix, jx) - 1; cx <= min(ix, jx); ++cx) {
                if (cx < 0 || cx >= P.nx) continue;
                const int a = (ix - cx) + 2 * (iy - cy) + 4 * (iz - cz);
                const int b = (jx - cx) + 2 * (jy - cy) + 4 * (jz - cz);
                v += young[cell_id(P, cx, cy, cz)] * K[(3 * a + i) * 24 + 3 * b + j];
              }
            }
          }
          const int64_t col = 3 * m + j;
          if (col == r) kdiag[r] = v;
          else if (fixed[r] || fixed[col]) v = 0.0;
          val[pos++] = v;
        }
      }
}

// ---------------------------------------------------------------------------------------
// momentum balance rows: residual and the (s, p) columns of the Jacobian
constexpr int kNodeThreads = 128;

__global__ void __launch_bounds__(kNodeThreads)
k_momentum(PoroK P, const double *x, const int64_t *rp, const double *young, const double *K,
           const uint8_t *fixed, const double *kdiag, double *F, double *val, int with_jac) {
  __shared__ double sK[576];
  for (int t = threadIdx.x; t < 576; t += blockDim.x) sK[t] = K[t];
  __syncthreads();
  const int64_t nd = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (nd >= P.nnode) return;
  const int ix = int(nd % (P.nx + 1)), iy = int((nd / (P.nx + 1)) % (P.ny + 1));
  const int iz = int(nd / (int64_t(P.nx + 1) * (P.ny + 1)));
  const int nbx = 1 + (ix > 0) + (ix < P.nx), nby = 1 + (iy > 0) + (iy < P.ny);
  const int nbz = 1 + (iz > 0) + (iz < P.nz);
  const int nuu = 3 * nbx * nby * nbz;   // u entries at the head of each of the three rows
  double f[3] = {0.0, 0.0, 0.0};
  int rank = 0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int cx = ix + dx, cy = iy + dy, cz = iz + dz;
        if (cx < 0 || cx >= P.nx || cy < 0 || cy >= P.ny || cz < 0 || cz >= P.nz) continue;
        const int64_t c = cell_id(P, cx, cy, cz);
        const int a = -dx - 2 * dy - 4 * dz;
        const double E = young[c];
        double e[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < 8; ++b) {
          const int64_t m = node_id(P, cx + (b & 1), cy + ((b >> 1) & 1), cz + ((b >> 2) & 1));
          for (int j = 0; j < 3; ++j) {
            const double uj = fixed[3 * m + j] ? 0.0 : x[3 * m + j];
            for (int i = 0; i < 3; ++i) e[i] += sK[(3 * a + i) * 24 + 3 * b + j] * uj;
          }
        }
        const double s = x[P.nu + 2 * c], p = x[P.nu + 2 * c + 1];
        double rw, drw, ro, dro;
        density(P, 0, p, rw, drw);
        density(P, 1, p, ro, dro);
        const double rho_mix = (1.0 - P.phi0) * P.rho_s + P.phi0 * (rw * s + ro * (1.0 - s));
        for (int i = 0; i < 3; ++i) {
          f[i] += E * e[i];
          f[i] += -P.biot * gint(a, i) * p;
        }
        f[2] += P.grav * rho_mix / 8.0;
        if (with_jac) {
          const double drm_dp = P.phi0 * (drw * s + dro * (1.0 - s));
          const double drm_ds = P.phi0 * (rw - ro);
          for (int i = 0; i < 3; ++i) {
            const int64_t r = 3 * nd + i;
            const bool fx = fixed[r] != 0;
            if (i < 2) {
              val[rp[r] + nuu + rank] = fx ? 0.0 : -P.biot * gint(a, i);
            } else {
              double vp = -P.biot * gint(a, 2);
              vp += P.grav * drm_dp / 8.0;
              val[rp[r] + nuu + 2 * rank] = fx ? 0.0 : P.grav * drm_ds / 8.0;
              val[rp[r] + nuu + 2 * rank + 1] = fx ? 0.0 : vp;
            }
          }
        }
        ++rank;
      }
  for (int i = 0; i < 3; ++i) {
    const int64_t r = 3 * nd + i;
    F[r] = fixed[r] ? kdiag[r] * x[r] : f[i];
  }
}

// ---------------------------------------------------------------------------------------
// mass-balance rows
struct Wells {
  const double *wi, *pbhp, *qw, *qo;   // any may be null (no well of that kind)
};

constexpr int kCellThreads = 128;

__global__ void __launch_bounds__(kCellThreads)
k_mass(PoroK P, const double *x, const double *xo, const int64_t *rp, const double *perm,
       const uint8_t *fixed, Wells W, double *F, double *val, int with_jac) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= P.ncell) return;
  const int cx = int(c % P.nx), cy = int((c / P.nx) % P.ny), cz = int(c / (int64_t(P.nx) * P.ny));
  const double s = x[P.nu + 2 * c], p = x[P.nu + 2 * c + 1];
  const double so = xo[P.nu + 2 * c], po = xo[P.nu + 2 * c + 1];
  int64_t nodes[8];
  double eps = 0.0, eps_o = 0.0;
  for (int a = 0; a < 8; ++a) {
    nodes[a] = node_id(P, cx + (a & 1), cy + ((a >> 1) & 1), cz + ((a >> 2) & 1));
    for (int i = 0; i < 3; ++i) {
      const int64_t d = 3 * nodes[a] + i;
      const bool fx = fixed[d] != 0;
      eps += gint(a, i) * (fx ? 0.0 : x[d]);
      eps_o += gint(a, i) * (fx ? 0.0 : xo[d]);
    }
  }
  const double phi = P.phi0 + P.biot * eps;
  const double phi_o = P.phi0 + P.biot * eps_o;
  double r[2], dr[2], lam[2], dlam[2], res[2];
  // Jacobian of the two rows: [phase][slot][unknown], slots -z,-y,-x,self,+x,+y,+z
  double J[2][7][2];
  for (int ph = 0; ph < 2; ++ph) {
    density(P, ph, p, r[ph], dr[ph]);
    mobility(P, ph, s, lam[ph], dlam[ph]);
    double ro_, dro_;
    density(P, ph, po, ro_, dro_);
    const double S = ph == 0 ? s : 1.0 - s, dS = ph == 0 ? 1.0 : -1.0;
    const double So = ph == 0 ? so : 1.0 - so;
    res[ph] = (phi * r[ph] * S - phi_o * ro_ * So) / P.dt;
    for (int sl = 0; sl < 7; ++sl) J[ph][sl][0] = J[ph][sl][1] = 0.0;
    J[ph][3][1] = phi * dr[ph] * S / P.dt;
    J[ph][3][0] = phi * r[ph] * dS / P.dt;
  }
  const int off[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0},
                         {1, 0, 0},  {0, 1, 0},  {0, 0, 1}};
  bool present[7];
  const double kc = perm[c];
  for (int sl = 0; sl < 7; ++sl) {
    const int jx = cx + off[sl][0], jy = cy + off[sl][1], jz = cz + off[sl][2];
    present[sl] = !(jx < 0 || jx >= P.nx || jy < 0 || jy >= P.ny || jz < 0 || jz >= P.nz);
    if (sl == 3 || !present[sl]) continue;
    const int64_t L = cell_id(P, jx, jy, jz);
    const double sL = x[P.nu + 2 * L], pL = x[P.nu + 2 * L + 1];
    const double kL = perm[L];
    const double T = 2.0 * kc * kL / (kc + kL);
    const double dz = double(-off[sl][2]);      // z_self - z_L
    const bool self_lower = sl > 3;
    for (int ph = 0; ph < 2; ++ph) {
      double rL, drL, lL, dlL;
      density(P, ph, pL, rL, drL);
      mobility(P, ph, sL, lL, dlL);
      const double dphi = p - pL + 0.5 * (r[ph] + rL) * P.grav * dz;
      const double dd_self = 1.0 + 0.5 * dr[ph] * P.grav * dz;
      const double dd_L = -1.0 + 0.5 * drL * P.grav * dz;
      // upwind: the lower-index cell of the face when the potential difference is zero
      const bool up_self = self_lower ? (dphi >= 0.0) : (dphi > 0.0);
      if (up_self) {
        const double m = T * r[ph] * lam[ph];
        res[ph] += T * r[ph] * lam[ph] * dphi;
        J[ph][3][1] += m * dd_self + T * dr[ph] * lam[ph] * dphi;
        J[ph][sl][1] += m * dd_L;
        J[ph][3][0] += T * r[ph] * dlam[ph] * dphi;
      } else {
        const double m = T * rL * lL;
        res[ph] += T * rL * lL * dphi;
        J[ph][3][1] += m * dd_self;
        J[ph][sl][1] += m * dd_L + T * drL * lL * dphi;
        J[ph][sl][0] += T * rL * dlL * dphi;
      }
    }
  }
  const double wi = W.wi ? W.wi[c] : 0.0;
  for (int ph = 0; ph < 2; ++ph) {
    double q = ph == 0 ? (W.qw ? W.qw[c] : 0.0) : (W.qo ? W.qo[c] : 0.0);
    if (wi != 0.0) {
      const double dp = p - W.pbhp[c];
      q -= wi * r[ph] * lam[ph] * dp;
      J[ph][3][1] += wi * (dr[ph] * lam[ph] * dp + r[ph] * lam[ph]);
      J[ph][3][0] += wi * r[ph] * dlam[ph] * dp;
    }
    res[ph] -= q;
    F[P.nu + 2 * c + ph] = res[ph];
  }
  if (!with_jac) return;
  for (int ph = 0; ph < 2; ++ph) {
    const int64_t row = P.nu + 2 * c + ph;
    double *v = val + rp[row];
    const double S = ph == 0 ? s : 1.0 - s;
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i) {
        const int64_t d = 3 * nodes[a] + i;
        v[3 * a + i] = fixed[d] ? 0.0 : P.biot * gint(a, i) * r[ph] * S / P.dt;
      }
    int k = 24;
    for (int sl = 0; sl < 7; ++sl) {
      if (!present[sl]) continue;
      v[k++] = J[ph][sl][0];
      v[k++] = J[ph][sl][1];
    }
  }
}

// ---------------------------------------------------------------------------------------
// residual norms in state units and the Newton update
constexpr int kNormBlocks = 256;
constexpr int kNormThreads = 256;

// partial[b * 6 + 2 t] = sum of squares, partial[b * 6 + 2 t + 1] = max |.| of type t
// (0: momentum rows / max Young's modulus, 1: wetting mass rows * dt / (phi0 rho0_w),
// 2: non-wetting mass rows * dt / (phi0 rho0_nw)).
__global__ void __launch_bounds__(kNormThreads)
k_norms(const double *F, int64_t nu, int64_t n, double emax, double fw, double fo,
        double *partial) {
  double ss[3] = {0.0, 0.0, 0.0}, mx[3] = {0.0, 0.0, 0.0};
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n;
       r += int64_t(gridDim.x) * blockDim.x) {
    int t;
    double v;
    if (r < nu) { t = 0; v = F[r] / emax; }
    else if (((r - nu) & 1) == 0) { t = 1; v = F[r] * fw; }
    else { t = 2; v = F[r] * fo; }
    ss[t] += v * v;
    mx[t] = fmax(mx[t], fabs(v));
  }
  __shared__ double red[6][kNormThreads];
  for (int t = 0; t < 3; ++t) {
    red[2 * t][threadIdx.x] = ss[t];
    red[2 * t + 1][threadIdx.x] = mx[t];
  }
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int t = 0; t < 3; ++t) {
        red[2 * t][threadIdx.x] += red[2 * t][threadIdx.x + w];
        red[2 * t + 1][threadIdx.x] = fmax(red[2 * t + 1][threadIdx.x], red[2 * t + 1][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// max |d| over the saturation unknowns
__global__ void __launch_bounds__(kNormThreads)
k_max_ds(const double *d, int64_t nu, int64_t ncell, double *partial) {
  double mx = 0.0;
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x)
    mx = fmax(mx, fabs(d[nu + 2 * c]));
  __shared__ double red[kNormThreads];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Row scaling of the Newton system to state units (momentum rows / the largest Young's
// modulus, mass rows of phase l * dt / (phi0 rho0_l)): sval = D val (a copy; the owned
// Jacobian stays unscaled) and F = D F in place.  MGR is unchanged by it (each reduction
// and smoother is invariant to row scaling); the FGMRES residual norm becomes one in which
// displacement and mass residuals weigh alike.
// One wavefront per row, its lanes striding the row's entries (coalesced).
constexpr int kScaleThreads = 256;
__global__ void __launch_bounds__(kScaleThreads)
k_scale_rows(const int64_t *rp, const double *val, double *sval, double *F, int64_t nu,
             int64_t n, double emax, double fw, double fo) {
  const int64_t r = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / 64;
  const int l = threadIdx.x & 63;
  if (r >= n) return;
  const int64_t e0 = rp[r], e1 = rp[r + 1];
  if (r < nu) {
    for (int64_t e = e0 + l; e < e1; e += 64) sval[e] = val[e] / emax;
    if (l == 0) F[r] = F[r] / emax;
  } else {
    const double f = ((r - nu) & 1) ? fo : fw;
    for (int64_t e = e0 + l; e < e1; e += 64) sval[e] = val[e] * f;
    if (l == 0) F[r] = F[r] * f;
  }
}

// xt = x - lambda d   (d solves A d = F, so -d is the Newton correction)
__global__ void k_step(const double *x, const double *d, double lambda, double *xt, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) xt[i] = x[i] + lambda * (-d[i]);
}

// Element stiffness of the unit cube for E = 1 (index form of the isotropic bilinear form
// lam div u div v + 2 mu eps(u) : eps(v), 2x2x2 Gauss points of weight 1/8).
void unit_stiffness(double nu, double *K) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int t = 0; t < 576; ++t) K[t] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {g[qx], g[qy], g[qz]};
        double G[8][3];
        for (int a = 0; a < 8; ++a) {
          const int bit[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
          double f[3], sg[3];
          for (int d = 0; d < 3; ++d) {
            f[d] = bit[d] ? xi[d] : 1.0 - xi[d];
            sg[d] = bit[d] ? 1.0 : -1.0;
          }
          G[a][0] = sg[0] * f[1] * f[2];
          G[a][1] = f[0] * sg[1] * f[2];
          G[a][2] = f[0] * f[1] * sg[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            const double dot = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                double v = lam * G[a][i] * G[b][j] + mu * G[a][j] * G[b][i];
                if (i == j) v += mu * dot;
                K[(3 * a + i) * 24 + 3 * b + j] += 0.125 * v;
              }
          }
      }
}

}  // namespace
}  // namespace mgr

using namespace mgr;

struct mgr_poro {
  mgr_poro_params prm{};
  PoroK k{};
  hipStream_t s = nullptr;
  DArr<int64_t> rp;
  DArr<int> ci;
  DArr<double> val;
  DArr<int8_t> labels;
  DArr<double> perm, young, wi, pbhp, qw, qo, K, kdiag;
  DArr<uint8_t> fixed;
  double emax = 0.0;
  bool has_wi = false, has_qw = false, has_qo = false;
  // Newton work
  DArr<double> F, d, xt, partial, sval;
  DArr<char> work;
  size_t work_bytes = 0;
};

namespace {
mgr_status pfail(const Error &e) {
  set_last_error(e.what());
  return e.st;
}

Wells wells_of(const mgr_poro *P) {
  return Wells{P->has_wi ? P->wi.p : nullptr, P->has_wi ? P->pbhp.p : nullptr,
               P->has_qw ? P->qw.p : nullptr, P->has_qo ? P->qo.p : nullptr};
}

// residual (and Jacobian) at x; norms [host, 6] when not null (synchronises)
void assemble(mgr_poro *P, const double *x, const double *xo, double *F, bool jac,
              double *norms, hipStream_t s) {
  const PoroK &k = P->k;
  const int jf = jac ? 1 : 0;
  hipLaunchKernelGGL(k_momentum, dim3(grid_for(k.nnode, kNodeThreads)), dim3(kNodeThreads), 0, s,
                     k, x, P->rp.p, P->young.p, P->K.p, P->fixed.p, P->kdiag.p, F, P->val.p, jf);
  KCHK();
  hipLaunchKernelGGL(k_mass, dim3(grid_for(k.ncell, kCellThreads)), dim3(kCellThreads), 0, s, k,
                     x, xo, P->rp.p, P->perm.p, P->fixed.p, wells_of(P), F, P->val.p, jf);
  KCHK();
  if (!norms) return;
  if (!P->partial.p) P->partial.alloc(kNormBlocks * 6, s);
  const double fw = k.dt / (k.phi0 * k.rho0[0]);
  const double fo = k.dt / (k.phi0 * k.rho0[1]);
  hipLaunchKernelGGL(k_norms, dim3(kNormBlocks), dim3(kNormThreads), 0, s, F, k.nu, k.n, P->emax,
                     fw, fo, P->partial.p);
  KCHK();
  std::vector<double> h(kNormBlocks * 6);
  HIPCHK(hipMemcpyAsync(h.data(), P->partial.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int t = 0; t < 6; ++t) norms[t] = 0.0;
  for (int b = 0; b < kNormBlocks; ++b)
    for (int t = 0; t < 3; ++t) {
      norms[2 * t] += h[b * 6 + 2 * t];
      norms[2 * t + 1] = std::max(norms[2 * t + 1], h[b * 6 + 2 * t + 1]);
    }
}

PoroK kernel_params(const mgr_poro_params &p) {
  PoroK k{};
  k.nx = p.nx;
  k.ny = p.ny;
  k.nz = p.nz;
  k.ncell = int64_t(p.nx) * p.ny * p.nz;
  k.nnode = int64_t(p.nx + 1) * (p.ny + 1) * (p.nz + 1);
  k.nu = 3 * k.nnode;
  k.n = k.nu + 2 * k.ncell;
  k.phi0 = p.phi0;
  k.biot = p.biot;
  k.grav = p.grav;
  k.p_ref = p.p_ref;
  k.rho_s = p.rho_solid;
  k.dt = p.dt;
  for (int i = 0; i < 2; ++i) {
    k.rho0[i] = p.rho0[i];
    k.comp[i] = p.comp[i];
    k.visc[i] = p.visc[i];
  }
  return k;
}

void check_params(const mgr_poro_params &p) {
  require(p.nx >= 1 && p.ny >= 1 && p.nz >= 1, MGR_ERR_ARG, "grid dimensions must be >= 1");
  const int64_t ncell = int64_t(p.nx) * p.ny * p.nz;
  const int64_t nnode = int64_t(p.nx + 1) * (p.ny + 1) * (p.nz + 1);
  // row lengths are at most 81 + 16 (momentum) and 38 (mass): bound nnz by 97 per row
  require((3 * nnode + 2 * ncell) * 97 < (int64_t(1) << 31), MGR_ERR_UNSUPPORTED,
          "grid too large for int32 column indices");
  require(p.nu > -1.0 && p.nu < 0.5, MGR_ERR_ARG, "Poisson ratio must lie in (-1, 0.5)");
  require(p.dt > 0.0, MGR_ERR_ARG, "dt must be positive");
  require(p.phi0 > 0.0 && p.phi0 < 1.0, MGR_ERR_ARG, "phi0 must lie in (0, 1)");
  for (int i = 0; i < 2; ++i)
    require(p.rho0[i] > 0.0 && p.visc[i] > 0.0 && p.comp[i] >= 0.0, MGR_ERR_ARG,
            "densities and viscosities must be positive, compressibilities >= 0");
  require(p.reserved == 0, MGR_ERR_ARG, "reserved must be 0");
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

extern "C" {

void mgr_poro_default_params(mgr_poro_params *p, int32_t nx, int32_t ny, int32_t nz) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->nu = 0.25;
  p->phi0 = 0.2;
  p->biot = 1.0;
  p->grav = 9.81;
  p->p_ref = 1.0e7;
  p->rho_solid = 2650.0;
  p->rho0[0] = 1000.0;
  p->rho0[1] = 800.0;
  p->comp[0] = 4.5e-10;
  p->comp[1] = 1.0e-9;
  p->visc[0] = 1.0e-3;
  p->visc[1] = 5.0e-3;
  p->dt = 86400.0;
}

void mgr_newton_default_opts(mgr_newton_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_newton = 12;
  o->max_backtracks = 6;
  o->tol_flow = 1.0e-6;
  o->tol_mech = 1.0e-10;
  o->max_ds = 0.2;
  o->armijo = 1.0e-4;
}

mgr_status mgr_poro_create(const mgr_poro_params *prm, const double *perm, const double *young,
                           const uint8_t *fixed, const double *well_index,
                           const double *well_pbhp, const double *inj_w, const double *inj_nw,
                           void *stream, mgr_poro **out) {
  if (!prm || !perm || !young || !fixed || !out) {
    set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  if ((well_index == nullptr) != (well_pbhp == nullptr)) {
    set_last_error("well_index and well_pbhp are given together");
    return MGR_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    check_params(*prm);
    auto P = std::make_unique<mgr_poro>();
    P->prm = *prm;
    P->k = kernel_params(*prm);
    P->s = s;
    const PoroK &k = P->k;
    auto copy_in = [&](DArr<double> &dst, const double *src, int64_t n) {
      dst.alloc(n, s);
      HIPCHK(hipMemcpyAsync(dst.p, src, n * sizeof(double), hipMemcpyDefault, s));
    };
    copy_in(P->perm, perm, k.ncell);
    copy_in(P->young, young, k.ncell);
    P->fixed.alloc(k.nu, s);
    HIPCHK(hipMemcpyAsync(P->fixed.p, fixed, k.nu, hipMemcpyDefault, s));
    if (well_index) {
      copy_in(P->wi, well_index, k.ncell);
      copy_in(P->pbhp, well_pbhp, k.ncell);
      P->has_wi = true;
    }
    if (inj_w) { copy_in(P->qw, inj_w, k.ncell); P->has_qw = true; }
    if (inj_nw) { copy_in(P->qo, inj_nw, k.ncell); P->has_qo = true; }
    std::vector<double> Kh(576);
    unit_stiffness(prm->nu, Kh.data());
    copy_in(P->K, Kh.data(), 576);
    P->emax = reduce_max_f64(P->young.p, k.ncell, s);
    require(P->emax > 0.0, MGR_ERR_ARG, "Young's moduli must be positive");
    // pattern
    DArr<int64_t> len(k.n, s);
    hipLaunchKernelGGL(k_row_len, dim3(grid_for(k.n, 256)), dim3(256), 0, s, k, len.p);
    KCHK();
    P->rp.alloc(k.n + 1, s);
    const int64_t nnz = exclusive_scan_i64(len.p, P->rp.p, k.n, s);
    P->ci.alloc(nnz, s);
    P->val.alloc(nnz, s);
    P->labels.alloc(k.n, s);
    hipLaunchKernelGGL(k_fill_pattern, dim3(grid_for(k.n, 256)), dim3(256), 0, s, k, P->rp.p,
                       P->ci.p, P->labels.p);
    KCHK();
    fill<double>(P->val.p, 0.0, nnz, s);
    P->kdiag.alloc(k.nu, s);
    hipLaunchKernelGGL(k_uu_values, dim3(grid_for(k.nu, 256)), dim3(256), 0, s, k, P->rp.p,
                       P->young.p, P->K.p, P->fixed.p, P->val.p, P->kdiag.p);
    KCHK();
    P->F.alloc(k.n, s);
    P->d.alloc(k.n, s);
    P->xt.alloc(k.n, s);
    HIPCHK(hipStreamSynchronize(s));
    *out = P.release();
  } catch (const Error &e) {
    return pfail(e);
  }
  return MGR_OK;
}

mgr_status mgr_poro_set_dt(mgr_poro *P, double dt) {
  if (!P || !(dt > 0.0)) {
    set_last_error("null handle or non-positive dt");
    return MGR_ERR_ARG;
  }
  P->prm.dt = dt;
  P->k.dt = dt;
  return MGR_OK;
}

mgr_status mgr_poro_matrix(const mgr_poro *P, mgr_csr *A, const int8_t **labels) {
  if (!P || !A) {
    set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  std::memset(A, 0, sizeof(*A));
  A->nrows = A->ncols = P->k.n;
  A->row_ptr = P->rp.p;
  A->col = P->ci.p;
  A->val = P->val.p;
  if (labels) *labels = P->labels.p;
  return MGR_OK;
}

mgr_status mgr_poro_export(const mgr_poro *P, int64_t *row_ptr, int32_t *col, double *val,
                           int8_t *labels, void *stream) {
  if (!P) {
    set_last_error("null handle");
    return MGR_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    const PoroK &k = P->k;
    const int64_t nnz = int64_t(P->ci.n);
    if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, P->rp.p, (k.n + 1) * sizeof(int64_t), hipMemcpyDefault, s));
    if (col) HIPCHK(hipMemcpyAsync(col, P->ci.p, nnz * sizeof(int32_t), hipMemcpyDefault, s));
    if (val) HIPCHK(hipMemcpyAsync(val, P->val.p, nnz * sizeof(double), hipMemcpyDefault, s));
    if (labels) HIPCHK(hipMemcpyAsync(labels, P->labels.p, k.n, hipMemcpyDefault, s));
    HIPCHK(hipStreamSynchronize(s));
  } catch (const Error &e) {
    return pfail(e);
  }
  return MGR_OK;
}

mgr_status mgr_poro_sizes(const mgr_poro *P, int64_t sizes[4]) {
  if (!P || !sizes) {
    set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  sizes[0] = P->k.n;
  sizes[1] = int64_t(P->ci.n);
  sizes[2] = P->k.nu;
  sizes[3] = P->k.ncell;
  return MGR_OK;
}

mgr_status mgr_poro_assemble(mgr_poro *P, const double *x, const double *x_old, double *F,
                             int32_t with_jacobian, double *norms, void *stream) {
  if (!P || !x || !x_old || !F) {
    set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  try {
    assemble(P, x, x_old, F, with_jacobian != 0, norms, static_cast<hipStream_t>(stream));
  } catch (const Error &e) {
    return pfail(e);
  }
  return MGR_OK;
}

mgr_status mgr_poro_newton(mgr_poro *P, mgr_handle **h, const mgr_opts *mo,
                           const fgmres_opts *fo, double *x, const double *x_old,
                           const mgr_newton_opts *no, mgr_newton_stats *st, void *stream) {
  if (!P || !h || !fo || !x || !x_old || !no || !st || (!*h && !mo)) {
    set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::memset(st, 0, sizeof(*st));
  try {
    require(no->max_newton >= 0 && no->max_newton <= MGR_NEWTON_MAX_RECORD, MGR_ERR_ARG,
            "max_newton must lie in [0, 32]");
    require(no->max_backtracks >= 0 && no->max_backtracks <= 60, MGR_ERR_ARG,
            "max_backtracks must lie in [0, 60]");
    require(no->max_ds > 0.0 && no->tol_flow > 0.0 && no->tol_mech > 0.0, MGR_ERR_ARG,
            "tolerances and max_ds must be positive");
    const PoroK &k = P->k;
    mgr_csr A;
    const int8_t *lab = nullptr;
    mgr_poro_matrix(P, &A, &lab);
    if (!P->sval.p) P->sval.alloc(P->val.n, s);
    A.val = P->sval.p;                       // the solves see the row-scaled Jacobian
    const size_t need = fgmres_workspace_bytes(k.n, fo->restart);
    if (P->work_bytes < need) {
      P->work.alloc(need, s);
      P->work_bytes = need;
    }
    auto merit_of = [&](const double *nr, bool &ok) {
      ok = nr[1] <= no->tol_mech && std::max(nr[3], nr[5]) <= no->tol_flow;
      return std::sqrt(nr[0] + nr[2] + nr[4]);
    };
    const double scale_w = k.dt / (k.phi0 * k.rho0[0]);
    const double scale_nw = k.dt / (k.phi0 * k.rho0[1]);
    auto scale_system = [&]() {
      hipLaunchKernelGGL(k_scale_rows, dim3(grid_for(k.n * 64, kScaleThreads)),
                         dim3(kScaleThreads), 0, s, P->rp.p,
                         P->val.p, P->sval.p, P->F.p, k.nu, k.n, P->emax, scale_w, scale_nw);
      KCHK();
    };
    double nr[6];
    double t0 = now_ms();
    assemble(P, x, x_old, P->F.p, true, nr, s);
    scale_system();
    st->assemble_ms += now_ms() - t0;
    bool ok = false;
    double m = merit_of(nr, ok);
    st->merit[0] = m;
    std::vector<double> hp(kNormBlocks);
    while (!ok && st->newton_iters < no->max_newton) {
      const int it = st->newton_iters;
      t0 = now_ms();
      mgr_status rc;
      if (!*h) {
        rc = mgr_setup(&A, lab, mo, stream, h);
        st->setups += 1;
      } else {
        rc = mgr_setup_numeric(*h, &A, stream);
      }
      if (rc != MGR_OK) return rc;
      st->setup_ms += now_ms() - t0;
      t0 = now_ms();
      fill<double>(P->d.p, 0.0, k.n, s);
      fgmres_result fr{};
      rc = fgmres_solve(&A, *h, P->F.p, P->d.p, fo, P->work.p, P->work_bytes, &fr, stream);
      st->solve_ms += now_ms() - t0;
      if (rc == MGR_ERR_NOT_CONVERGED) st->linear_failures += 1;
      else if (rc != MGR_OK) return rc;
      st->lin_iters[it] = fr.iters;
      st->linear_iters += fr.iters;
      st->newton_iters = it + 1;
      // step length: cap the saturation change, then halve until the merit decreases
      hipLaunchKernelGGL(k_max_ds, dim3(kNormBlocks), dim3(kNormThreads), 0, s, P->d.p, k.nu,
                         k.ncell, P->partial.p);
      KCHK();
      HIPCHK(hipMemcpyAsync(hp.data(), P->partial.p, kNormBlocks * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double dsmax = 0.0;
      for (double v : hp) dsmax = std::max(dsmax, v);
      double lam = 1.0;
      if (dsmax * lam > no->max_ds) lam = no->max_ds / dsmax;
      double mt = m;
      bool okt = false;
      t0 = now_ms();
      for (int bt = 0; bt <= no->max_backtracks; ++bt) {
        hipLaunchKernelGGL(k_step, dim3(grid_for(k.n, 256)), dim3(256), 0, s, x, P->d.p, lam,
                           P->xt.p, k.n);
        KCHK();
        assemble(P, P->xt.p, x_old, P->F.p, false, nr, s);
        mt = merit_of(nr, okt);
        if (mt <= (1.0 - no->armijo * lam) * m || bt == no->max_backtracks) break;
        lam *= 0.5;
        st->backtracks += 1;
      }
      st->lambda[it] = lam;
      HIPCHK(hipMemcpyAsync(x, P->xt.p, k.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      m = mt;
      ok = okt;
      st->merit[it + 1] = m;
      if (!ok && st->newton_iters < no->max_newton) {
        assemble(P, x, x_old, P->F.p, true, nullptr, s);   // Jacobian at the accepted point
        scale_system();
      }
      st->assemble_ms += now_ms() - t0;
    }
    HIPCHK(hipStreamSynchronize(s));
    st->converged = ok ? 1 : 0;
  } catch (const Error &e) {
    return pfail(e);
  }
  return MGR_OK;
}

void mgr_poro_destroy(mgr_poro *P) {
  if (!P) return;
  if (P->s) (void)hipStreamSynchronize(P->s);
  delete P;
}

}  // extern "C"

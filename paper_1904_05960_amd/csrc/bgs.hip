// Multicolour block Gauss-Seidel global smoother: the hybrid block Gauss-Seidel the paper
// uses as the global smoother of the flow levels (Sec. 5.3 remarks), in a colour order
// that lets every cell of one colour update at once.
//
// Cells are the same-cell blocks of a level whose rows are interleaved cell by cell (cell
// e = rows e*nb .. e*nb+nb-1).  Setup: the cell graph is the symmetrised block pattern of
// A (cells e != f adjacent when A couples a row of e with a row of f in either direction),
// coloured by Jones-Plassmann rounds: an uncoloured cell whose (priority, index) exceeds
// that of every uncoloured neighbour takes the smallest colour not used by its neighbours
// coloured in earlier rounds (SplitMix64 priorities of the cell index with a fixed salt).
// Apply: per sweep, per colour in ascending order, every cell of the colour computes the
// residual of its rows with the current x and adds D_e^{-1} times it; cells of one colour
// share no entry, so their updates are independent.
#include <algorithm>

#include "common.hpp"

namespace mgr {
namespace {

constexpr unsigned long long BGS_GOLDEN = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ unsigned long long bgs_splitmix64(unsigned long long seed) {
  unsigned long long z = seed + BGS_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_cell_prio(int64_t ncell, unsigned long long salt,
                            unsigned long long *__restrict__ prio, int *__restrict__ color) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  prio[e] = bgs_splitmix64((unsigned long long)e ^ salt);
  color[e] = -1;
}

// cell-of-row maps as CSR: Rc (ncell x n) row e = rows of cell e; Bc (n x ncell) row r =
// cell r / nb
__global__ void k_cell_maps(int64_t n, int nb, int *__restrict__ rc_rp, int *__restrict__ rc_ci,
                            double *__restrict__ rc_v, int *__restrict__ bc_rp,
                            int *__restrict__ bc_ci, double *__restrict__ bc_v) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r > n) return;
  bc_rp[r] = (int)r;
  if (r % nb == 0) rc_rp[r / nb] = (int)r;
  if (r == n) return;
  rc_ci[r] = (int)r;
  rc_v[r] = 1.0;
  bc_ci[r] = (int)(r / nb);
  bc_v[r] = 1.0;
}

// one Jones-Plassmann round (colours read from cold, written to cnew)
__global__ void k_jp_round(int64_t ncell, const int *__restrict__ gp, const int *__restrict__ gc,
                           const unsigned long long *__restrict__ prio,
                           const int *__restrict__ cold, int *__restrict__ cnew,
                           int *__restrict__ nunc, int *__restrict__ over) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const int ce = cold[e];
  if (ce >= 0) {
    cnew[e] = ce;
    return;
  }
  const unsigned long long pe = prio[e];
  bool win = true;
  unsigned long long used = 0ull;
  for (int q = gp[e]; q < gp[e + 1]; ++q) {
    const int f = gc[q];
    if (f == (int)e) continue;
    const int cf = cold[f];
    if (cf < 0) {
      const unsigned long long pf = prio[f];
      if (pf > pe || (pf == pe && f > (int)e)) win = false;
    } else if (cf < 64) {
      used |= 1ull << cf;
    }
  }
  if (win) {
    if (used == ~0ull) {          // all 64 colours taken around e
      atomicOr(over, 1);
      cnew[e] = 63;
      return;
    }
    cnew[e] = __ffsll((long long)~used) - 1;
  } else {
    cnew[e] = -1;
    atomicAdd(nunc, 1);
  }
}

__global__ void k_color_count(int64_t ncell, const int *__restrict__ color,
                              int *__restrict__ cnt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < ncell) atomicAdd(&cnt[color[e]], 1);
}

// cells grouped by colour (the order inside a colour does not matter: its cells are
// independent)
__global__ void k_color_fill(int64_t ncell, const int *__restrict__ color,
                             int *__restrict__ cursor, int *__restrict__ cells) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < ncell) cells[atomicAdd(&cursor[color[e]], 1)] = (int)e;
}

// the cells of one colour: G lanes per cell form the residuals of its NB rows, lane 0 adds
// D_e^{-1} r_e (row-major NB x NB inverse)
template <class T, int NB, int G>
__global__ void __launch_bounds__(256) k_bgs_color(int ncells, const int *__restrict__ cells,
                                                   const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const T *__restrict__ v,
                                                   const T *__restrict__ binv,
                                                   const T *__restrict__ b, T *__restrict__ x) {
  const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (g >= ncells) return;
  const int64_t e = cells[g];
  T r[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int64_t row = e * NB + t;
    T acc = 0;
    for (int q = rp[row] + l; q < rp[row + 1]; q += G) acc += v[q] * x[ci[q]];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    r[t] = b[row] - acc;
  }
  if (l != 0) return;
  const T *Di = binv + e * NB * NB;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    T s = 0;
#pragma unroll
    for (int u = 0; u < NB; ++u) s += Di[t * NB + u] * r[u];
    x[e * NB + t] += s;
  }
}

}  // namespace

void bgs_setup(const Csr &A, int nb, std::vector<int> &color_ptr, DArr<int> &cells,
               DArr<int> &color, hipStream_t s, int *dflag) {
  const int64_t n = A.n;
  require(nb >= 1 && n % nb == 0, MGR_ERR_UNSUPPORTED, "block Gauss-Seidel: rows not in cells");
  const int64_t ncell = n / nb;
  // cell graph: pattern of Rc A Bc, symmetrised
  Csr Rc, Bc, C1, C2, C2t, U;
  Rc.n = ncell; Rc.m = n; Rc.nnz = n;
  Bc.n = n; Bc.m = ncell; Bc.nnz = n;
  Rc.rp.alloc(ncell + 1, s); Rc.ci.alloc(std::max<int64_t>(n, 1), s);
  Rc.v.alloc(std::max<int64_t>(n, 1), s);
  Bc.rp.alloc(n + 1, s); Bc.ci.alloc(std::max<int64_t>(n, 1), s);
  Bc.v.alloc(std::max<int64_t>(n, 1), s);
  k_cell_maps<<<grid_for(n + 1, 256), 256, 0, s>>>(n, nb, Rc.rp.p, Rc.ci.p, Rc.v.p, Bc.rp.p,
                                                   Bc.ci.p, Bc.v.p);
  KCHK();
  spgemm(Rc, A, C1, s, dflag);
  Rc = Csr();
  spgemm(C1, Bc, C2, s, dflag);
  C1 = Csr();
  Bc = Csr();
  transpose(C2, C2t, false, s);
  merge_drop(C2, C2t, nullptr, -1, nullptr, U, false, s, dflag);
  check_flags(dflag, s, "block Gauss-Seidel cell graph");
  // Jones-Plassmann rounds
  DArr<unsigned long long> prio(ncell, s);
  DArr<int> c0(ncell, s), c1(ncell, s), nunc(1, s), over(1, s);
  fill<int>(over.p, 0, 1, s);
  color.alloc(ncell, s);
  k_cell_prio<<<grid_for(ncell, 256), 256, 0, s>>>(ncell, BGS_GOLDEN * 977ull, prio.p, c0.p);
  KCHK();
  int *cur = c0.p, *nxt = c1.p;
  for (int round = 0;; ++round) {
    require(round < 100000, MGR_ERR_HIP, "colouring did not finish");
    fill<int>(nunc.p, 0, 1, s);
    k_jp_round<<<grid_for(ncell, 256), 256, 0, s>>>(ncell, U.rp.p, U.ci.p, prio.p, cur, nxt,
                                                    nunc.p, over.p);
    KCHK();
    std::swap(cur, nxt);
    if (read_flag(nunc.p, s) == 0) break;
  }
  require(read_flag(over.p, s) == 0, MGR_ERR_UNSUPPORTED,
          "block Gauss-Seidel: the cell graph needs more than 64 colours");
  HIPCHK(hipMemcpyAsync(color.p, cur, ncell * sizeof(int), hipMemcpyDeviceToDevice, s));
  // cells grouped by colour
  DArr<int> cnt(64, s);
  fill<int>(cnt.p, 0, 64, s);
  k_color_count<<<grid_for(ncell, 256), 256, 0, s>>>(ncell, color.p, cnt.p);
  KCHK();
  int hc[64];
  d2h_sync(hc, cnt.p, sizeof(hc), s);
  int ncol = 0;
  for (int c = 0; c < 64; ++c)
    if (hc[c] > 0) ncol = c + 1;
  color_ptr.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) color_ptr[c + 1] = color_ptr[c] + hc[c];
  DArr<int> cursor(64, s);
  HIPCHK(hipMemcpyAsync(cursor.p, color_ptr.data(), ncol * sizeof(int), hipMemcpyHostToDevice, s));
  cells.alloc(std::max<int64_t>(ncell, 1), s);
  k_color_fill<<<grid_for(ncell, 256), 256, 0, s>>>(ncell, color.p, cursor.p, cells.p);
  KCHK();
  HIPCHK(hipStreamSynchronize(s));
}

template <class T>
void bgs_color_sweep(const CsrV<T> &A, int nb, const int *cells, int ncells, const T *binv,
                     const T *b, T *x, hipStream_t s) {
  if (ncells <= 0) return;
  const double avg = A.n ? (double)A.nnz / (double)A.n : 0.0;
#define BGS(NBV, GG)                                                                          \
  k_bgs_color<T, NBV, GG><<<grid_for((int64_t)ncells * GG, 256), 256, 0, s>>>(ncells, cells, A.rp, \
                                                                               A.ci, A.v, binv, b, x)
  if (nb == 2) {
    if (avg > 24) BGS(2, 16); else BGS(2, 8);
  } else if (nb == 3) {
    if (avg > 24) BGS(3, 16); else BGS(3, 8);
  } else {
    throw Error(MGR_ERR_UNSUPPORTED, "block Gauss-Seidel: 2 or 3 unknowns per cell");
  }
#undef BGS
  KCHK();
}
template void bgs_color_sweep<float>(const CsrV<float> &, int, const int *, int, const float *,
                                     const float *, float *, hipStream_t);
template void bgs_color_sweep<double>(const CsrV<double> &, int, const int *, int, const double *,
                                      const double *, double *, hipStream_t);

}  // namespace mgr

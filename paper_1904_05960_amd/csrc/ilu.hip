// Fine-grained ILU(k) global smoother (the pointwise ILU(1) of the Sec. 5.3 remarks and
// Sec. 6, computed by the fixed-point method of Chow and Patel), k = 0 or 1.
//
// Setup, on the level matrix A_l whose rows are interleaved cell by cell:
//  * As = D_B^{-1} A_l, D_B the same-cell diagonal blocks (their inverses are those of the
//    block-Jacobi smoother), by the pinned-order sparse product;
//  * the ILU(k) pattern S: As itself (k = 0), or As united with the pattern of
//    strict_lower(As) * strict_upper(As) (k = 1: the level-1 fill), values of As on it and
//    +0.0 on the fill;
//  * the factors as the fixed point of (LU)_ij = a_ij on S, by synchronous sweeps from
//    l_ij = a_ij / a_jj, u_ij = a_ij:
//        s_ij = a_ij - sum_{m < min(i,j)} l_im u_mj     (ascending m, one product and one
//                                                       subtraction at a time)
//        l_ij = s_ij / u_jj (i > j),  u_ij = s_ij (i <= j),
//    every component computed from the previous iterate.  A group of lanes owns a row i:
//    the row's columns and accumulators are staged in LDS, the pivots m of the row are taken
//    in ascending order, and the lanes split the strictly upper entries (m, j) of row m,
//    each locating j in row i by binary search.  Distinct j of one step land in distinct
//    accumulators, and a wave's LDS operations execute in issue order, so the steps of one
//    accumulator happen in ascending m;
//  * apply copies: L - I and U - D_U as CSR-stream matrices and 1 / u_ii.
// Apply: c = D_B^{-1} r; y from L y = c by Jacobi sweeps y <- c - (L - I) y from y = c;
// z from U z = y by z <- D_U^{-1} (y - (U - D_U) z) from z = D_U^{-1} y.
#include <climits>

#include "common.hpp"

namespace mgr {
namespace {

constexpr int ILU_MAXR = 256;   // longest row of the ILU pattern handled by the sweep kernel

// rows of the block-diagonal D_B^{-1}: row i holds the nb entries of its cell's inverse row
__global__ void k_blockdiag_pattern(int64_t n, int nb, int *rp, int *ci) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  rp[i] = (int)(i * nb);
  if (i == n) return;
  const int64_t c0 = (i / nb) * nb;
  for (int t = 0; t < nb; ++t) ci[i * nb + t] = (int)(c0 + t);
}

// MODE 0: strictly lower entries, 1: strictly upper entries; count pass (out_rp == nullptr
// writes counts into cnt) or fill pass
template <int MODE>
__global__ void k_split_count(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                              int *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) c += MODE == 0 ? (ci[e] < i) : (ci[e] > i);
  cnt[i] = c;
}
template <int MODE>
__global__ void k_split_fill(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ v, const int *__restrict__ orp,
                             int *__restrict__ oci, double *__restrict__ ov) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = orp[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const bool take = MODE == 0 ? (ci[e] < i) : (ci[e] > i);
    if (take) {
      oci[o] = ci[e];
      if (ov) ov[o] = v ? v[e] : 0.0;
      ++o;
    }
  }
}

// union of the patterns of A and B per row (both sorted), values of A, +0.0 where only B
__global__ void k_union_count(int64_t n, const int *__restrict__ arp, const int *__restrict__ aci,
                              const int *__restrict__ brp, const int *__restrict__ bci,
                              int *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = arp[i], pe = arp[i + 1], q = brp[i], qe = brp[i + 1], c = 0;
  while (p < pe || q < qe) {
    const int ca = p < pe ? aci[p] : INT_MAX, cb = q < qe ? bci[q] : INT_MAX;
    if (ca <= cb) ++p;
    if (cb <= ca) ++q;
    ++c;
  }
  cnt[i] = c;
}
__global__ void k_union_fill(int64_t n, const int *__restrict__ arp, const int *__restrict__ aci,
                             const double *__restrict__ av, const int *__restrict__ brp,
                             const int *__restrict__ bci, const int *__restrict__ orp,
                             int *__restrict__ oci, double *__restrict__ ov) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = arp[i], pe = arp[i + 1], q = brp[i], qe = brp[i + 1], o = orp[i];
  while (p < pe || q < qe) {
    const int ca = p < pe ? aci[p] : INT_MAX, cb = q < qe ? bci[q] : INT_MAX;
    if (ca <= cb) {
      oci[o] = ca;
      ov[o] = av[p];
      ++p;
      if (cb == ca) ++q;
    } else {
      oci[o] = cb;
      ov[o] = 0.0;
      ++q;
    }
    ++o;
  }
}

// position of the diagonal of every row; a missing or zero diagonal raises ZERO_PIVOT, a row
// longer than the sweep kernel's LDS rows raises UNSUPPORTED
__global__ void k_diag_pos(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ v, int *__restrict__ dpos, int *flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = -1;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) d = e;
  dpos[i] = d;
  if (d < 0 || !(v[d] != 0.0 && v[d] == v[d])) atomicOr(flag, FLAG_ZERO_PIVOT);
  if (rp[i + 1] - rp[i] > ILU_MAXR) atomicOr(flag, FLAG_ROW_TOO_LONG);
}

// starting iterate: l_ij = a_ij / a_jj below the diagonal, u_ij = a_ij on and above
__global__ void k_ilu_init(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ a, const int *__restrict__ dpos,
                           double *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int j = ci[e];
    x[e] = j < i ? a[e] / a[dpos[j]] : a[e];
  }
}

// one synchronous sweep: G lanes (16 or 32, a divisor of the wavefront) per row
template <int G>
__global__ void __launch_bounds__(256) k_ilu_sweep(int64_t n, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const double *__restrict__ a,
                                                   const int *__restrict__ dpos,
                                                   const double *__restrict__ old,
                                                   double *__restrict__ nw) {
  constexpr int NG = 256 / G;
  __shared__ int scol[NG][ILU_MAXR];
  __shared__ double sacc[NG][ILU_MAXR];
  const int g = threadIdx.x / G, l = threadIdx.x % G;
  const int64_t i = blockIdx.x * (int64_t)NG + g;
  if (i >= n) return;            // whole groups leave; no block-wide barrier below
  const int s0 = rp[i];
  const int len = rp[i + 1] - s0;  // <= ILU_MAXR (checked at setup)
  int *col = scol[g];
  double *acc = sacc[g];
  for (int q = l; q < len; q += G) {
    col[q] = ci[s0 + q];
    acc[q] = a[s0 + q];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int p = 0; p < len; ++p) {
    const int m = col[p];
    if (m >= (int)i) break;                      // columns ascend: the pivots m < i first
    const double lim = old[s0 + p];
    const int q1 = rp[m + 1];
    for (int q = dpos[m] + 1 + l; q < q1; q += G) {   // entries (m, j), j > m
      const int j = ci[q];
      int lo = 0, hi = len;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      if (lo < len && col[lo] == j) acc[lo] = acc[lo] - lim * old[q];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  for (int q = l; q < len; q += G) {
    const int j = col[q];
    nw[s0 + q] = j < (int)i ? acc[q] / old[dpos[j]] : acc[q];
  }
}

__global__ void k_inv_diag(int64_t n, const int *__restrict__ dpos, const double *__restrict__ v,
                           double *__restrict__ dinv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dinv[i] = 1.0 / v[dpos[i]];
}

template <class T>
__global__ void k_axpy(int64_t n, T alpha, const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = y[i] + alpha * x[i];
}
template <class T>
__global__ void k_scatter_axpy(const int *__restrict__ idx, int64_t n, T alpha,
                               const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[idx[i]] = y[idx[i]] + alpha * x[i];
}
__global__ void k_scale_cols_div(int64_t nnz, const int *__restrict__ ci,
                                 const double *__restrict__ d, double *__restrict__ v) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nnz) v[e] = v[e] / d[ci[e]];
}

template <int MODE>
void split_part(const Csr &S, Csr &out, hipStream_t s) {
  const int64_t n = S.n;
  out.n = n;
  out.m = S.m;
  out.rp.alloc(n + 1, s);
  if (n > 0) {
    k_split_count<MODE><<<grid_for(n, 256), 256, 0, s>>>(n, S.rp.p, S.ci.p, out.rp.p);
    KCHK();
  }
  out.nnz = exclusive_scan_i32(out.rp.p, out.rp.p, n, s);
  out.ci.alloc(std::max<int64_t>(out.nnz, 1), s);
  out.v.alloc(std::max<int64_t>(out.nnz, 1), s);
  if (n > 0) {
    k_split_fill<MODE><<<grid_for(n, 256), 256, 0, s>>>(n, S.rp.p, S.ci.p, S.v.p, out.rp.p,
                                                         out.ci.p, out.v.p);
    KCHK();
  }
}

}  // namespace

void ilu_pattern_values(const Csr &As, int level, Csr &S, hipStream_t s, int *dflag) {
  require(level == 0 || level == 1, MGR_ERR_UNSUPPORTED, "ILU level must be 0 or 1");
  if (level == 0) {
    copy_csr(As, S, s);
    return;
  }
  Csr Ls, Us, F;
  split_part<0>(As, Ls, s);
  split_part<1>(As, Us, s);
  spgemm(Ls, Us, F, s, dflag);
  const int64_t n = As.n;
  S.n = n;
  S.m = As.m;
  S.rp.alloc(n + 1, s);
  if (n > 0) {
    k_union_count<<<grid_for(n, 256), 256, 0, s>>>(n, As.rp.p, As.ci.p, F.rp.p, F.ci.p, S.rp.p);
    KCHK();
  }
  S.nnz = exclusive_scan_i32(S.rp.p, S.rp.p, n, s);
  S.ci.alloc(std::max<int64_t>(S.nnz, 1), s);
  S.v.alloc(std::max<int64_t>(S.nnz, 1), s);
  if (n > 0) {
    k_union_fill<<<grid_for(n, 256), 256, 0, s>>>(n, As.rp.p, As.ci.p, As.v.p, F.rp.p, F.ci.p,
                                                  S.rp.p, S.ci.p, S.v.p);
    KCHK();
  }
}

void ilu_factor(Csr &S, int sweeps, DArr<int> &dpos, hipStream_t s, int *dflag) {
  const int64_t n = S.n;
  dpos.alloc(std::max<int64_t>(n, 1), s);
  if (n == 0) return;
  k_diag_pos<<<grid_for(n, 256), 256, 0, s>>>(n, S.rp.p, S.ci.p, S.v.p, dpos.p, dflag);
  KCHK();
  check_flags(dflag, s, "ILU pattern (zero or missing diagonal, or a row longer than 256)");
  DArr<double> a(std::max<int64_t>(S.nnz, 1), s), other(std::max<int64_t>(S.nnz, 1), s);
  if (S.nnz) HIPCHK(hipMemcpyAsync(a.p, S.v.p, S.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  k_ilu_init<<<grid_for(n, 256), 256, 0, s>>>(n, S.rp.p, S.ci.p, a.p, dpos.p, S.v.p);
  KCHK();
  const double avg = (double)S.nnz / (double)n;
  for (int k = 0; k < sweeps; ++k) {
    if (avg <= 24.0)
      k_ilu_sweep<16><<<grid_for(n, 256 / 16), 256, 0, s>>>(n, S.rp.p, S.ci.p, a.p, dpos.p,
                                                             S.v.p, other.p);
    else
      k_ilu_sweep<32><<<grid_for(n, 256 / 32), 256, 0, s>>>(n, S.rp.p, S.ci.p, a.p, dpos.p,
                                                             S.v.p, other.p);
    KCHK();
    std::swap(S.v, other);
  }
}

void block_diag_pattern(int64_t n, int nb, int *rp, int *ci, hipStream_t s) {
  k_blockdiag_pattern<<<grid_for(n + 1, 256), 256, 0, s>>>(n, nb, rp, ci);
  KCHK();
}

void block_scale(const Csr &A, int nb, const double *binv, Csr &As, hipStream_t s, int *dflag) {
  const int64_t n = A.n;
  Csr Bd;
  Bd.n = Bd.m = n;
  Bd.nnz = n * nb;
  Bd.rp.alloc(n + 1, s);
  Bd.ci.alloc(std::max<int64_t>(Bd.nnz, 1), s);
  Bd.v.alloc(std::max<int64_t>(Bd.nnz, 1), s);
  k_blockdiag_pattern<<<grid_for(n + 1, 256), 256, 0, s>>>(n, nb, Bd.rp.p, Bd.ci.p);
  KCHK();
  if (Bd.nnz)
    HIPCHK(hipMemcpyAsync(Bd.v.p, binv, Bd.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  spgemm(Bd, A, As, s, dflag);
}

void ilu_split(const Csr &S, const DArr<int> &dpos, Csr &Lo, Csr &Up, DArr<double> &dinv,
               hipStream_t s) {
  split_part<0>(S, Lo, s);
  split_part<1>(S, Up, s);
  dinv.alloc(std::max<int64_t>(S.n, 1), s);
  if (S.n > 0) {
    k_inv_diag<<<grid_for(S.n, 256), 256, 0, s>>>(S.n, dpos.p, S.v.p, dinv.p);
    KCHK();
  }
}

template <class T>
void axpy(int64_t n, T alpha, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return;
  k_axpy<T><<<grid_for(n, 256), 256, 0, s>>>(n, alpha, x, y);
  KCHK();
}
template void axpy<float>(int64_t, float, const float *, float *, hipStream_t);
template void axpy<double>(int64_t, double, const double *, double *, hipStream_t);

template <class T>
void scatter_axpy(const int *idx, int64_t n, T alpha, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_axpy<T><<<grid_for(n, 256), 256, 0, s>>>(idx, n, alpha, x, y);
  KCHK();
}
template void scatter_axpy<float>(const int *, int64_t, float, const float *, float *,
                                  hipStream_t);
template void scatter_axpy<double>(const int *, int64_t, double, const double *, double *,
                                   hipStream_t);

void scale_cols_div(Csr &M, const double *d, hipStream_t s) {
  if (M.nnz <= 0) return;
  k_scale_cols_div<<<grid_for(M.nnz, 256), 256, 0, s>>>(M.nnz, M.ci.p, d, M.v.p);
  KCHK();
}

}  // namespace mgr

// Dense solves for the coarsest grids: the matrix is expanded to a dense row-major array
// and inverted once at setup (Gauss-Jordan with partial pivoting, FP64, one workgroup);
// each coarse solve in the V-cycle is then a dense matrix-vector product.
#include "common.hpp"

namespace mgr {
namespace {

__global__ void k_scatter_dense(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                                const double *__restrict__ v, double *__restrict__ D) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) D[i * n + ci[e]] = v[e];
}

constexpr int GJ_THREADS = 1024;

// In-place Gauss-Jordan inversion with partial pivoting (first row of largest |a| in the
// column); column interchanges undone at the end.
__global__ void __launch_bounds__(GJ_THREADS) k_gauss_jordan(double *__restrict__ A, int n,
                                                            int *__restrict__ piv,
                                                            double *__restrict__ colk,
                                                            int *flag) {
  __shared__ double s_val[GJ_THREADS];
  __shared__ int s_idx[GJ_THREADS];
  __shared__ int s_fail;
  const int t = threadIdx.x;
  if (t == 0) s_fail = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot search
    double best = -1.0;
    int bi = n;
    for (int i = k + t; i < n; i += GJ_THREADS) {
      const double a = fabs(A[(int64_t)i * n + k]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    s_val[t] = best;
    s_idx[t] = bi;
    __syncthreads();
    for (int o = GJ_THREADS / 2; o > 0; o >>= 1) {
      if (t < o) {
        const double a = s_val[t + o];
        const int ia = s_idx[t + o];
        if (a > s_val[t] || (a == s_val[t] && ia < s_idx[t])) { s_val[t] = a; s_idx[t] = ia; }
      }
      __syncthreads();
    }
    const int p = s_idx[0];
    const double pv = s_val[0];
    if (!(pv > 0.0)) {   // zero, or only NaN left in the column
      if (t == 0) s_fail = 1;
      __syncthreads();
      break;
    }
    if (t == 0) piv[k] = p;
    if (p != k) {
      for (int j = t; j < n; j += GJ_THREADS) {
        const double x = A[(int64_t)k * n + j];
        A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
        A[(int64_t)p * n + j] = x;
      }
    }
    __syncthreads();
    const double pivot = A[(int64_t)k * n + k];
    __syncthreads();
    for (int j = t; j < n; j += GJ_THREADS)
      A[(int64_t)k * n + j] = (j == k ? 1.0 : A[(int64_t)k * n + j]) / pivot;
    for (int i = t; i < n; i += GJ_THREADS) colk[i] = A[(int64_t)i * n + k];
    __syncthreads();
    for (int64_t q = t; q < (int64_t)n * n; q += GJ_THREADS) {
      const int i = (int)(q / n), j = (int)(q % n);
      if (i == k) continue;
      const double base = (j == k) ? 0.0 : A[q];
      A[q] = base - colk[i] * A[(int64_t)k * n + j];
    }
    __syncthreads();
  }
  if (s_fail) {
    if (t == 0) atomicOr(flag, FLAG_ZERO_PIVOT);
    return;
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int i = t; i < n; i += GJ_THREADS) {
        const double x = A[(int64_t)i * n + k];
        A[(int64_t)i * n + k] = A[(int64_t)i * n + p];
        A[(int64_t)i * n + p] = x;
      }
    }
    __syncthreads();
  }
}

// The same elimination for n <= GJ_LDS_N with the matrix held in LDS (rows padded to an odd
// stride so that a column is read without bank conflicts): one pivot step is four barriers
// and LDS traffic only; the pivot search is done by the first wavefront.
constexpr int GJ_LDS_N = 128;
__global__ void __launch_bounds__(GJ_THREADS) k_gauss_jordan_lds(double *__restrict__ A, int n,
                                                                int *flag) {
  __shared__ double sA[GJ_LDS_N * (GJ_LDS_N + 1)];
  __shared__ double s_colk[GJ_LDS_N];
  __shared__ int s_piv[GJ_LDS_N];
  __shared__ int s_p;
  __shared__ double s_pv;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  constexpr int NW = GJ_THREADS / 64;
  const int ld = n | 1;
  for (int i = w; i < n; i += NW)
    for (int j = lane; j < n; j += 64) sA[i * ld + j] = A[(int64_t)i * n + j];
  __syncthreads();
  bool fail = false;
  for (int k = 0; k < n; ++k) {
    if (w == 0) {   // first row of largest |a| in column k
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        const double a = fabs(sA[i * ld + k]);
        if (a > best) { best = a; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        s_p = bi;
        s_pv = best;
      }
    }
    __syncthreads();
    const int p = s_p;
    const double pv = s_pv;
    if (!(pv > 0.0)) {   // zero, or only NaN left in the column
      fail = true;
      break;
    }
    if (t == 0) s_piv[k] = p;
    if (p != k && t < n) {
      const double x = sA[k * ld + t];
      sA[k * ld + t] = sA[p * ld + t];
      sA[p * ld + t] = x;
    }
    __syncthreads();
    const double pivot = sA[k * ld + k];
    double rk = 0.0, ck = 0.0;
    if (t < n) {
      rk = (t == k ? 1.0 : sA[k * ld + t]) / pivot;
      ck = sA[t * ld + k];
    }
    __syncthreads();
    if (t < n) {
      sA[k * ld + t] = rk;
      s_colk[t] = ck;
    }
    __syncthreads();
    for (int i = w; i < n; i += NW) {
      if (i == k) continue;
      const double ci = s_colk[i];
      for (int j = lane; j < n; j += 64) {
        const double base = (j == k) ? 0.0 : sA[i * ld + j];
        sA[i * ld + j] = base - ci * sA[k * ld + j];
      }
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) atomicOr(flag, FLAG_ZERO_PIVOT);
    return;
  }
  // undo the interchanges: columns k and piv[k], last step first
  for (int k = n - 1; k >= 0; --k) {
    const int p = s_piv[k];
    if (p != k && t < n) {
      const double x = sA[t * ld + k];
      sA[t * ld + k] = sA[t * ld + p];
      sA[t * ld + p] = x;
    }
    __syncthreads();
  }
  for (int i = w; i < n; i += NW)
    for (int j = lane; j < n; j += 64) A[(int64_t)i * n + j] = sA[i * ld + j];
}

// Blocked form of the same elimination for GJ_LDS_N < n <= GJB_MAXN, one workgroup.  The
// columns are taken in panels of GJB columns: a panel (all n rows) is eliminated in LDS by
// the steps above, with the same pivot rule; that leaves its pivot rows holding
// Q1 = A11^{-1} and its other rows Q2 = -A21 A11^{-1} (A11: the panel's pivot-row block,
// A21: the rest of its columns, both as they stood before the panel).  The panel's row
// interchanges are then applied to every other column X, and X is updated as one block:
// X_R1 <- Q1 X_R1, X_R2 <- X_R2 + Q2 X_R1 (R1 the panel's pivot rows).  The matrix is read
// and written once per panel instead of once per column.
constexpr int GJB = 16;
constexpr int GJB_MAXN = 512;
__global__ void __launch_bounds__(GJ_THREADS) k_gauss_jordan_blocked(double *__restrict__ A, int n,
                                                                    int *__restrict__ piv,
                                                                    int *flag) {
  __shared__ double sP[GJB][GJB_MAXN + 1];   // panel, column l at sP[l][row]
  __shared__ double s_c[GJB_MAXN];           // multipliers of the current step
  __shared__ double s_rk[GJB];               // normalised pivot row within the panel
  __shared__ int s_piv[GJB];
  __shared__ int s_p;
  __shared__ double s_pv;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // column-parallel mapping of the block update: NP >= n columns, R threads per column
  const int NP = n <= 256 ? 256 : 512;
  const int R = GJ_THREADS / NP;
  const int col = t % NP, rgrp = t / NP;
  bool fail = false;
  for (int k0 = 0; k0 < n && !fail; k0 += GJB) {
    const int bw = min(GJB, n - k0);
    // 1. the panel into LDS (16 lanes read a row's panel segment)
    for (int q = t; q < n * GJB; q += GJ_THREADS) {
      const int i = q / GJB, l = q % GJB;
      if (l < bw) sP[l][i] = A[(int64_t)i * n + k0 + l];
    }
    __syncthreads();
    // 2. eliminate the panel's columns
    for (int j = 0; j < bw; ++j) {
      const int k = k0 + j;
      if (w == 0) {   // first row of largest |a| in column k, rows k..n-1
        double best = -1.0;
        int bi = n;
        for (int i = k + lane; i < n; i += 64) {
          const double a = fabs(sP[j][i]);
          if (a > best) { best = a; bi = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) {
          s_p = bi;
          s_pv = best;
        }
      }
      __syncthreads();
      const int p = s_p;
      if (!(s_pv > 0.0)) {   // zero, or only NaN left in the column
        fail = true;
        break;
      }
      if (t == 0) {
        s_piv[j] = p;
        piv[k] = p;
      }
      if (p != k && t < bw) {
        const double x = sP[t][k];
        sP[t][k] = sP[t][p];
        sP[t][p] = x;
      }
      __syncthreads();
      const double pivot = sP[j][k];
      if (t < bw) s_rk[t] = (t == j ? 1.0 : sP[t][k]) / pivot;
      for (int i = t; i < n; i += GJ_THREADS) s_c[i] = sP[j][i];
      __syncthreads();
      if (t < bw) sP[t][k] = s_rk[t];
      for (int i = t; i < n; i += GJ_THREADS) {
        if (i == k) continue;
        const double ci = s_c[i];
        for (int l = 0; l < bw; ++l) {
          const double base = (l == j) ? 0.0 : sP[l][i];
          sP[l][i] = base - ci * s_rk[l];
        }
      }
      __syncthreads();
    }
    if (fail) break;
    // 3. the panel's interchanges on the other columns (one thread per column, in order)
    const bool mine = col < n && (col < k0 || col >= k0 + bw);
    if (rgrp == 0 && mine) {
      for (int j = 0; j < bw; ++j) {
        const int k = k0 + j, p = s_piv[j];
        if (p != k) {
          const double x = A[(int64_t)k * n + col];
          A[(int64_t)k * n + col] = A[(int64_t)p * n + col];
          A[(int64_t)p * n + col] = x;
        }
      }
    }
    __syncthreads();
    // 4. block update of the other columns
    double y[GJB];
#pragma unroll
    for (int l = 0; l < GJB; ++l) y[l] = (mine && l < bw) ? A[(int64_t)(k0 + l) * n + col] : 0.0;
    __syncthreads();
    if (mine) {
      for (int i = rgrp; i < n; i += R) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < GJB; ++l)
          if (l < bw) acc += sP[l][i] * y[l];
        if (i >= k0 && i < k0 + bw) A[(int64_t)i * n + col] = acc;
        else A[(int64_t)i * n + col] = A[(int64_t)i * n + col] + acc;
      }
    }
    // the panel's columns back
    for (int q = t; q < n * GJB; q += GJ_THREADS) {
      const int i = q / GJB, l = q % GJB;
      if (l < bw) A[(int64_t)i * n + k0 + l] = sP[l][i];
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) atomicOr(flag, FLAG_ZERO_PIVOT);
    return;
  }
  // undo the interchanges: columns k and piv[k], last step first; a thread swaps within
  // its own rows only, in that order, so the steps need no barrier
  for (int i = t; i < n; i += GJ_THREADS)
    for (int k = n - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        const double x = A[(int64_t)i * n + k];
        A[(int64_t)i * n + k] = A[(int64_t)i * n + p];
        A[(int64_t)i * n + p] = x;
      }
    }
}

}  // namespace

void csr_to_dense(const Csr &A, double *D, hipStream_t s) {
  fill<double>(D, 0.0, A.n * A.n, s);
  if (A.n == 0) return;
  k_scatter_dense<<<grid_for(A.n, 256), 256, 0, s>>>(A.n, A.rp.p, A.ci.p, A.v.p, D);
  KCHK();
}

void dense_inverse(double *D, double *Inv, int n, int *dflag, hipStream_t s) {
  require(n >= 1 && n <= 4096, MGR_ERR_UNSUPPORTED, "dense solve limited to 4096 unknowns");
  HIPCHK(hipMemcpyAsync(Inv, D, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (n <= GJ_LDS_N) {
    k_gauss_jordan_lds<<<1, GJ_THREADS, 0, s>>>(Inv, n, dflag);
    KCHK();
  } else if (n <= GJB_MAXN) {
    DArr<int> piv(n, s);
    k_gauss_jordan_blocked<<<1, GJ_THREADS, 0, s>>>(Inv, n, piv.p, dflag);
    KCHK();
  } else {
    DArr<int> piv(n, s);
    DArr<double> colk(n, s);
    k_gauss_jordan<<<1, GJ_THREADS, 0, s>>>(Inv, n, piv.p, colk.p, dflag);
    KCHK();
  }
  check_flags(dflag, s, "dense inverse");
}

}  // namespace mgr

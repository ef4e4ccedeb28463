// Kernels of the preconditioner application (Algorithm 2 and the AMG V-cycles inside it),
// for FP32 or FP64 hierarchies.  All of them are HBM-bandwidth bound:
//  * CSR rows are processed by G lanes of a 64-wide wavefront (G from the mean row length),
//    so that each group streams a contiguous run of column indices and values;
//  * 3x3 block rows (nodal elasticity AMG) store the nine block entries in nine planes
//    (entry k of block e at v[k * nnzb + e]), so lane-consecutive blocks give unit-stride
//    loads; one lane handles one block and the three row sums are reduced over the group;
//  * the l1-Jacobi smoothing sweeps are fused with the residual they need: the presweep
//    from zero (x = D^{-1} b) and the residual b - A x are one pass over A, the postsweep
//    y = x + D^{-1}(b - A x) is one pass.
#include "common.hpp"

namespace mgr {
namespace {

enum { M_RESID = 0, M_SPMV = 1, M_SPMV_ADD = 2, M_L1PRE = 3, M_L1POST = 4 };
// restriction that also forms the next level's first smoothing iterate: out = A x,
// out2 = D^{-1} out with the next level's D (the product the separate pass would form)
enum { M_SPMV_DX = 6 };
// scaled residual out = D^{-1} (b - A x) (Jacobi sweeps on a triangular factor)
enum { M_RESID_SCALE = 7 };

template <class T, int G>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// One kernel for the CSR variants.  Work item t uses matrix row rows[t] (or t); the right
// side is indexed by bidx[t] (or t).
template <class T, int G, int MODE>
__global__ void __launch_bounds__(256) k_csr(int64_t nw, const int *__restrict__ rows,
                                             const int *__restrict__ bidx,
                                             const int *__restrict__ rp, const int *__restrict__ ci,
                                             const T *__restrict__ v, const T *__restrict__ x,
                                             const T *__restrict__ b, const T *__restrict__ dinv,
                                             T *__restrict__ out, T *__restrict__ out2) {
  const int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (t >= nw) return;
  const int row = rows ? rows[t] : (int)t;
  T acc = 0;
  const int e1 = rp[row + 1];
  for (int e = rp[row] + l; e < e1; e += G) {
    const int c = ci[e];
    if (MODE == M_L1PRE) acc += v[e] * (dinv[c] * b[c]);
    else acc += v[e] * x[c];
  }
  acc = group_sum<T, G>(acc);
  if (l != 0) return;
  if (MODE == M_RESID) {
    out[t] = b[bidx ? bidx[t] : t] - acc;
  } else if (MODE == M_SPMV) {
    out[t] = acc;
  } else if (MODE == M_SPMV_ADD) {
    out[t] += acc;
  } else if (MODE == M_L1PRE) {
    const T bi = b[t];
    out2[t] = dinv[t] * bi;       // x
    out[t] = bi - acc;            // r
  } else if (MODE == M_RESID_SCALE) {
    out[t] = dinv[t] * (b[t] - acc);
  } else {                        // M_L1POST: y = x + D^{-1}(b - A x)
    out[t] = x[t] + dinv[t] * (b[t] - acc);
  }
}

// CSR-stream variant (matrices with row blocks): block k owns rows [rb[k], rb[k+1]) whose
// entries start in the k-th window of SNNZ entries.  The window's products are formed with
// coalesced loads, PER independent loads in flight per thread, staged in LDS, and each row
// is summed from LDS by 8 lanes; a block whose rows hold more than scap<T> entries sums
// each row directly.  The FP64 window keeps 256 entries of slack (18 KB of LDS, 8 blocks per
// CU); the FP32 one 2048 (16 KB).  Row t of the matrix is work item t; `bidx` indexes b (RESID) and `oidx`
// the output (INTERP: z[oidx[t]] (+)= [eF[t]] + acc).
constexpr int SB = 256;
constexpr int SNNZ = 2048;
template <class T>
constexpr int scap = sizeof(T) == 4 ? 2 * SNNZ : SNNZ + 256;
enum { M_INTERP = 5 };

template <class T, int MODE>
__device__ __forceinline__ void csr_epilogue(int row, T acc, const int *__restrict__ bidx,
                                             const int *__restrict__ oidx,
                                             const T *__restrict__ x, const T *__restrict__ b,
                                             const T *__restrict__ dinv, T *__restrict__ out,
                                             T *__restrict__ out2, int accumulate) {
  if (MODE == M_RESID) {
    out[row] = b[bidx ? bidx[row] : row] - acc;
  } else if (MODE == M_SPMV) {
    out[row] = acc;
  } else if (MODE == M_SPMV_ADD) {
    out[row] += acc;
  } else if (MODE == M_L1PRE) {
    const T bi = b[row];
    out2[row] = dinv[row] * bi;
    out[row] = bi - acc;
  } else if (MODE == M_L1POST) {
    out[row] = x[row] + dinv[row] * (b[row] - acc);
  } else if (MODE == M_SPMV_DX) {
    out[row] = acc;
    out2[row] = dinv[row] * acc;
  } else if (MODE == M_RESID_SCALE) {
    out[row] = dinv[row] * (b[row] - acc);
  } else {  // M_INTERP: x = eF (may be null), out = z
    const int i = oidx[row];
    const T base = accumulate ? out[i] : (x ? x[row] : (T)0);
    out[i] = base + acc;
  }
}

// Row-local operands of a row's epilogue, loaded before the block's barrier so that their
// latency overlaps the window's gathers instead of following the LDS sums.
template <class T>
struct RowPre {
  int s = 0, e = 0, oi = 0;
  T bv = 0, dv = 0, xv = 0, ov = 0;
};
template <class T, int MODE>
__device__ __forceinline__ void row_prefetch(int row, int base, const int *__restrict__ rp,
                                             const int *__restrict__ bidx,
                                             const int *__restrict__ oidx,
                                             const T *__restrict__ x, const T *__restrict__ b,
                                             const T *__restrict__ dinv, const T *out,
                                             int accumulate, RowPre<T> &p) {
  p.s = rp[row] - base;
  p.e = rp[row + 1] - base;
  if (MODE == M_RESID) p.bv = b[bidx ? bidx[row] : row];
  if (MODE == M_L1PRE || MODE == M_L1POST || MODE == M_RESID_SCALE) p.bv = b[row];
  if (MODE == M_L1PRE || MODE == M_L1POST || MODE == M_SPMV_DX || MODE == M_RESID_SCALE)
    p.dv = dinv[row];
  if (MODE == M_L1POST) p.xv = x[row];
  if (MODE == M_SPMV_ADD) p.ov = out[row];
  if (MODE == M_INTERP) {
    p.oi = oidx[row];
    p.ov = accumulate ? out[p.oi] : (x ? x[row] : (T)0);
  }
}
// the same results as csr_epilogue, from prefetched operands
template <class T, int MODE>
__device__ __forceinline__ void csr_epilogue_pre(int row, T acc, const RowPre<T> &p,
                                                 T *__restrict__ out, T *__restrict__ out2) {
  if (MODE == M_RESID) {
    out[row] = p.bv - acc;
  } else if (MODE == M_SPMV) {
    out[row] = acc;
  } else if (MODE == M_SPMV_ADD) {
    out[row] = p.ov + acc;
  } else if (MODE == M_L1PRE) {
    out2[row] = p.dv * p.bv;
    out[row] = p.bv - acc;
  } else if (MODE == M_L1POST) {
    out[row] = p.xv + p.dv * (p.bv - acc);
  } else if (MODE == M_SPMV_DX) {
    out[row] = acc;
    out2[row] = p.dv * acc;
  } else if (MODE == M_RESID_SCALE) {
    out[row] = p.dv * (p.bv - acc);
  } else {  // M_INTERP
    out[p.oi] = p.ov + acc;
  }
}

template <class T, int MODE, int G>
__global__ void __launch_bounds__(SB) k_csr_stream(const int *__restrict__ rb,
                                                   const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const T *__restrict__ v,
                                                   const T *__restrict__ xin,
                                                   const T *__restrict__ x,
                                                   const T *__restrict__ b,
                                                   const T *__restrict__ dinv,
                                                   const int *__restrict__ bidx,
                                                   const int *__restrict__ oidx,
                                                   T *__restrict__ out, T *__restrict__ out2,
                                                   int accumulate) {
  // xin: the vector the products gather (x, or for L1PRE b scaled by dinv on the fly)
  __shared__ T prod[scap<T>];
  const int r0 = rb[blockIdx.x], r1 = rb[blockIdx.x + 1];
  if (r0 >= r1) return;
  const int base = rp[r0];
  const int cnt = rp[r1] - base;
  const int t = threadIdx.x;
  if (cnt <= scap<T>) {
    constexpr int PER = SNNZ / SB;
    // this thread's first row of the sum phase and its epilogue operands
    const int prow = r0 + t / G;
    RowPre<T> pre;
    if (prow < r1)
      row_prefetch<T, MODE>(prow, base, rp, bidx, oidx, x, b, dinv, out, accumulate, pre);
    for (int e0 = 0; e0 < cnt; e0 += PER * SB) {
      int c[PER];
      T vv[PER], xv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        c[u] = 0;
        vv[u] = 0;
        if (e < cnt) {
          c[u] = ci[base + e];
          vv[u] = v[base + e];
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        if (MODE == M_L1PRE) xv[u] = (e < cnt) ? dinv[c[u]] * b[c[u]] : (T)0;
        else xv[u] = (e < cnt) ? xin[c[u]] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        if (e < cnt) prod[e] = vv[u] * xv[u];
      }
    }
    __syncthreads();
    // G lanes per row (G ~ mean row length / 8, so that the block's rows take about one
    // pass of its 256 threads)
    const int l = t & (G - 1);
    for (int row = prow; row < r1; row += SB / G) {
      RowPre<T> p;
      if (row == prow) p = pre;
      else row_prefetch<T, MODE>(row, base, rp, bidx, oidx, x, b, dinv, out, accumulate, p);
      T acc = 0;
      for (int e = p.s + l; e < p.e; e += G) acc += prod[e];
      if (G > 1) acc = group_sum<T, G>(acc);
      if (l == 0) csr_epilogue_pre<T, MODE>(row, acc, p, out, out2);
    }
    return;
  }
  __shared__ T part[SB / 64];
  for (int row = r0; row < r1; ++row) {
    T acc = 0;
    for (int e = rp[row] + t; e < rp[row + 1]; e += SB) {
      const int c = ci[e];
      acc += v[e] * (MODE == M_L1PRE ? dinv[c] * b[c] : xin[c]);
    }
    acc = group_sum<T, 64>(acc);
    if ((t & 63) == 0) part[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      const T tot = (part[0] + part[1]) + (part[2] + part[3]);
      csr_epilogue<T, MODE>(row, tot, bidx, oidx, x, b, dinv, out, out2, accumulate);
    }
    __syncthreads();
  }
}

template <class T, int MODE>
void launch_csr_stream(const CsrV<T> &A, const T *xin, const T *x, const T *b, const T *dinv,
                       const int *bidx, const int *oidx, T *out, T *out2, int accumulate,
                       hipStream_t s) {
  if (A.nblk <= 0) return;
  const double avg = A.n ? (double)A.nnz / (double)A.n : 0.0;
#define LST(GG)                                                                            \
  k_csr_stream<T, MODE, GG><<<(unsigned)A.nblk, SB, 0, s>>>(A.rb, A.rp, A.ci, A.v, xin, x, b, \
                                                            dinv, bidx, oidx, out, out2,      \
                                                            accumulate)
  if (avg < 12) LST(1);
  else if (avg < 24) LST(2);
  else if (avg < 48) LST(4);
  else LST(8);
#undef LST
  KCHK();
}

// z_C (+)= e_C
template <class T>
__global__ void k_scatter_c(const int *__restrict__ C, int64_t nC, const T *__restrict__ eC,
                            T *__restrict__ z, int accumulate) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nC) return;
  const int i = C[k];
  z[i] = accumulate ? z[i] + eC[k] : eC[k];
}

__global__ void k_rowblocks32(int64_t n, const int *__restrict__ rp, int64_t K,
                              int *__restrict__ rb) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k > K) return;
  if (k == K) { rb[k] = (int)n; return; }
  const int64_t target = k * SNNZ;
  int64_t lo = 0, hi = n;          // first row whose start is >= target
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] < target) lo = mid + 1; else hi = mid;
  }
  rb[k] = (int)lo;
}

template <class T, int MODE>
void launch_csr(const CsrV<T> &A, int64_t nw, const int *rows, const int *bidx, const T *x,
                const T *b, const T *dinv, T *out, T *out2, hipStream_t s) {
  if (nw <= 0) return;
  const double avg = A.n ? (double)A.nnz / (double)A.n : 0.0;
#define LCSR(GG)                                                                          \
  k_csr<T, GG, MODE><<<grid_for(nw * GG, 256), 256, 0, s>>>(nw, rows, bidx, A.rp, A.ci, A.v, \
                                                             x, b, dinv, out, out2)
  if (avg > 48) LCSR(64);
  else if (avg > 24) LCSR(32);
  else if (avg > 12) LCSR(16);
  else if (avg > 6) LCSR(8);
  else LCSR(4);
#undef LCSR
  KCHK();
}

// BSR3 variants; G lanes per block row, block values in nine planes
template <class T, int G, int MODE>
__global__ void __launch_bounds__(256) k_bsr3(int64_t nb, const int *__restrict__ rp,
                                              const int *__restrict__ ci, int64_t nnzb,
                                              const T *__restrict__ v, const T *__restrict__ x,
                                              const T *__restrict__ b, const T *__restrict__ dinv,
                                              T *__restrict__ out, T *__restrict__ out2) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (I >= nb) return;
  T a0 = 0, a1 = 0, a2 = 0;
  const int e1 = rp[I + 1];
  for (int e = rp[I] + l; e < e1; e += G) {
    const int64_t c3 = 3 * (int64_t)ci[e];
    T x0, x1, x2;
    if (MODE == M_L1PRE) {
      x0 = dinv[c3] * b[c3];
      x1 = dinv[c3 + 1] * b[c3 + 1];
      x2 = dinv[c3 + 2] * b[c3 + 2];
    } else {
      x0 = x[c3];
      x1 = x[c3 + 1];
      x2 = x[c3 + 2];
    }
    const T *vb = v + e;
    a0 += vb[0] * x0 + vb[nnzb] * x1 + vb[2 * nnzb] * x2;
    a1 += vb[3 * nnzb] * x0 + vb[4 * nnzb] * x1 + vb[5 * nnzb] * x2;
    a2 += vb[6 * nnzb] * x0 + vb[7 * nnzb] * x1 + vb[8 * nnzb] * x2;
  }
  a0 = group_sum<T, G>(a0);
  a1 = group_sum<T, G>(a1);
  a2 = group_sum<T, G>(a2);
  if (l != 0) return;
  const int64_t r = 3 * I;
  if (MODE == M_SPMV) {
    out[r] = a0; out[r + 1] = a1; out[r + 2] = a2;
  } else if (MODE == M_SPMV_DX) {
    out[r] = a0; out[r + 1] = a1; out[r + 2] = a2;
    out2[r] = dinv[r] * a0; out2[r + 1] = dinv[r + 1] * a1; out2[r + 2] = dinv[r + 2] * a2;
  } else if (MODE == M_SPMV_ADD) {
    out[r] += a0; out[r + 1] += a1; out[r + 2] += a2;
  } else if (MODE == M_RESID) {
    out[r] = b[r] - a0; out[r + 1] = b[r + 1] - a1; out[r + 2] = b[r + 2] - a2;
  } else if (MODE == M_L1PRE) {
    const T b0 = b[r], b1 = b[r + 1], b2 = b[r + 2];
    out2[r] = dinv[r] * b0; out2[r + 1] = dinv[r + 1] * b1; out2[r + 2] = dinv[r + 2] * b2;
    out[r] = b0 - a0; out[r + 1] = b1 - a1; out[r + 2] = b2 - a2;
  } else {
    out[r] = x[r] + dinv[r] * (b[r] - a0);
    out[r + 1] = x[r + 1] + dinv[r + 1] * (b[r + 1] - a1);
    out[r + 2] = x[r + 2] + dinv[r + 2] * (b[r + 2] - a2);
  }
}

template <class T, int MODE>
void launch_bsr3(const Bsr3V<T> &A, const T *x, const T *b, const T *dinv, T *out, T *out2,
                 hipStream_t s) {
  if (A.n <= 0) return;
  const double avg = (double)A.nnzb / (double)A.n;
#define LB(GG)                                                                         \
  k_bsr3<T, GG, MODE><<<grid_for(A.n * GG, 256), 256, 0, s>>>(A.n, A.rp, A.ci, A.nnzb, A.v, \
                                                               x, b, dinv, out, out2)
  // lanes per block row ~ its mean length / 1.5, up to a wave (the restrictions of the
  // coarse levels have rows of a hundred blocks and more)
  if (avg > 96) LB(64);
  else if (avg > 48) LB(32);
  else if (avg > 12) LB(16);
  else if (avg > 6) LB(8);
  else LB(4);
#undef LB
  KCHK();
}

// interpolation and correction: z_F (+)= [eF] + W_p e_C, z_C (+)= e_C.  8 lanes per row.
template <class T>
__global__ void k_interp(int64_t n, const int *__restrict__ map, const int *__restrict__ wrp,
                         const int *__restrict__ wci, const T *__restrict__ wv,
                         const T *__restrict__ eC, const T *__restrict__ eF, T *__restrict__ z,
                         int accumulate) {
  constexpr int G = 8;
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (i >= n) return;
  const int m = map[i];
  if (m >= 0) {
    T acc = 0;
    for (int e = wrp[m] + l; e < wrp[m + 1]; e += G) acc += wv[e] * eC[wci[e]];
    acc = group_sum<T, G>(acc);
    if (l == 0) {
      const T base = accumulate ? z[i] : (eF ? eF[m] : (T)0);
      z[i] = base + acc;
    }
  } else if (l == 0) {
    const T e = eC[-m - 1];
    z[i] = accumulate ? z[i] + e : e;
  }
}

// dense y = M x, one wavefront per row
template <class T>
__global__ void k_gemv(const T *__restrict__ M, int n, const T *__restrict__ x, T *__restrict__ y) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  T acc = 0;
  const T *mr = M + row * (int64_t)n;
  for (int j = l; j < n; j += 64) acc += mr[j] * x[j];
  acc = group_sum<T, 64>(acc);
  if (l == 0) y[row] = acc;
}

template <class T>
__global__ void k_gather(const int *__restrict__ idx, int64_t n, const T *__restrict__ x,
                         T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[idx[t]];
}
template <class T>
__global__ void k_scatter_add(const int *__restrict__ idx, int64_t n, const T *__restrict__ x,
                              T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[idx[t]] += x[t];
}
template <class T>
__global__ void k_jacobi_update(const int *__restrict__ F, int64_t nF, const T *__restrict__ dinv,
                                T omega, const T *__restrict__ r, T *__restrict__ z) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < nF) z[F[t]] += omega * (dinv[t] * r[t]);
}
template <class T>
__global__ void k_jacobi_first(int64_t n, const int *__restrict__ map, const T *__restrict__ dinv,
                               T omega, const T *__restrict__ v, T *__restrict__ z) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = map[i];
  z[i] = m >= 0 ? omega * (dinv[m] * v[i]) : (T)0;
}
// z = D_B^{-1} v, or z += omega D_B^{-1} v, over consecutive nb x nb blocks
template <class T>
__global__ void k_block_jacobi(int64_t nblk, int nb, const T *__restrict__ inv,
                               const T *__restrict__ v, T omega, T *__restrict__ z, int acc) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nblk) return;
  const T *B = inv + e * nb * nb;
  const int64_t r0 = e * nb;
  T vv[3];
  for (int c = 0; c < nb; ++c) vv[c] = v[r0 + c];
  for (int r = 0; r < nb; ++r) {
    T s = 0;
    for (int c = 0; c < nb; ++c) s += B[r * nb + c] * vv[c];
    z[r0 + r] = acc ? z[r0 + r] + omega * s : s;
  }
}
// Products of a cell-blocked matrix (BR x BC row-major blocks over cells of BR rows) with
// one of two epilogues per cell:
//   CB_SWEEP (BR = BC): one block-Jacobi sweep zout = zin + omega D_B^{-1} (rhs - A zin);
//   CB_RESID: out = rhs[bidx] - A x (rhs gathered through bidx when given).
// Block k of the grid owns the block rows (cells) whose first block lies in the k-th window
// of 512 blocks.  One lane per block, two blocks per lane at a time (each block's values
// read as one record, its block column and x entries, all loads before any use), each
// block's BR row partials into LDS; then BG lanes per cell sum its rows and apply the
// epilogue, so a sweep's residual never goes to memory.  Windows holding more than PCAPB
// blocks (a cell with hundreds of neighbours) sum each cell directly with the whole
// workgroup.
constexpr int PCAPB = 768;
enum { CB_SWEEP = 0, CB_RESID = 1 };
template <class T, int BR, int BC, int MODE>
__device__ inline void cell_epilogue(int64_t I, const T (&acc)[BR], const T *__restrict__ zin,
                                     const T *__restrict__ rhs, const int *__restrict__ bidx,
                                     const T *__restrict__ inv, T omega, T *__restrict__ zout) {
  const int64_t row = I * BR;
  T res[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r) res[r] = rhs[bidx ? (int64_t)bidx[row + r] : row + r] - acc[r];
  if (MODE == CB_RESID) {
#pragma unroll
    for (int r = 0; r < BR; ++r) zout[row + r] = res[r];
    return;
  }
  const T *Bi = inv + I * BR * BR;
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    T sr = 0;
#pragma unroll
    for (int c = 0; c < BR; ++c) sr += Bi[r * BR + c] * res[c];
    zout[row + r] = zin[row + r] + omega * sr;
  }
}

template <class T, int BR, int BC, int BG, int MODE>
__global__ void __launch_bounds__(256) k_bsr_cell(const int *__restrict__ rb,
                                                  const int *__restrict__ rp,
                                                  const int *__restrict__ ci,
                                                  const T *__restrict__ v,
                                                  const T *__restrict__ zin,
                                                  const T *__restrict__ rhs,
                                                  const int *__restrict__ bidx,
                                                  const T *__restrict__ inv, T omega,
                                                  T *__restrict__ zout) {
  constexpr int BB = BR * BC;
  __shared__ T part[PCAPB * BR];
  const int r0 = rb[blockIdx.x], r1 = rb[blockIdx.x + 1];
  if (r0 >= r1) return;
  const int base = rp[r0];
  const int nblk = rp[r1] - base;
  const int t = threadIdx.x;
  if (nblk <= PCAPB) {
    constexpr int BPL = 2;
    for (int q0 = 0; q0 < nblk; q0 += BPL * 256) {
      T a[BPL][BB], xx[BPL][BC];
      int cc[BPL];
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * 256 + t;
        cc[h] = 0;
        if (e < nblk) {
          const T *bv = v + (int64_t)(base + e) * BB;
#pragma unroll
          for (int u = 0; u < BB; ++u) a[h][u] = bv[u];
          cc[h] = ci[base + e];
        } else {
#pragma unroll
          for (int u = 0; u < BB; ++u) a[h][u] = 0;
        }
      }
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * 256 + t;
#pragma unroll
        for (int c = 0; c < BC; ++c) xx[h][c] = (e < nblk) ? zin[(int64_t)cc[h] * BC + c] : (T)0;
      }
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * 256 + t;
        if (e < nblk) {
#pragma unroll
          for (int r = 0; r < BR; ++r) {
            T pr = a[h][r * BC] * xx[h][0];
#pragma unroll
            for (int c = 1; c < BC; ++c) pr += a[h][r * BC + c] * xx[h][c];
            part[e * BR + r] = pr;
          }
        }
      }
    }
    __syncthreads();
    const int l = t & (BG - 1);
    for (int I = r0 + t / BG; I < r1; I += 256 / BG) {
      const int s0 = rp[I] - base, len = rp[I + 1] - rp[I];
      T acc[BR];
#pragma unroll
      for (int r = 0; r < BR; ++r) acc[r] = 0;
      for (int k = l; k < len; k += BG)
#pragma unroll
        for (int r = 0; r < BR; ++r) acc[r] += part[(s0 + k) * BR + r];
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int o = BG / 2; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, BG);
      if (l == 0) cell_epilogue<T, BR, BC, MODE>(I, acc, zin, rhs, bidx, inv, omega, zout);
    }
    return;
  }
  __shared__ T fpart[4][BR];
  for (int I = r0; I < r1; ++I) {
    const int e0 = rp[I], len = rp[I + 1] - e0;
    T acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0;
    for (int k = t; k < len; k += 256) {
      const T *bv = v + (int64_t)(e0 + k) * BB;
      const int64_t c0 = (int64_t)ci[e0 + k] * BC;
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int c = 0; c < BC; ++c) acc[r] += bv[r * BC + c] * zin[c0 + c];
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      acc[r] = group_sum<T, 64>(acc[r]);
      if ((t & 63) == 0) fpart[t >> 6][r] = acc[r];
    }
    __syncthreads();
    if (t == 0) {
      T tot[BR];
#pragma unroll
      for (int r = 0; r < BR; ++r) tot[r] = (fpart[0][r] + fpart[1][r]) + (fpart[2][r] + fpart[3][r]);
      cell_epilogue<T, BR, BC, MODE>(I, tot, zin, rhs, bidx, inv, omega, zout);
    }
    __syncthreads();
  }
}

template <class T>
__global__ void k_fillv(T *p, T val, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}
template <class A, class B>
__global__ void k_cast(const A *__restrict__ a, B *__restrict__ b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (B)a[i];
}

}  // namespace

template <class T>
void VecOps<T>::resid(const CsrV<T> &A, int64_t nw, const int *rows, const int *bidx, const T *x,
                      const T *b, T *out, hipStream_t s) {
  if (!rows && A.rb && nw == A.n)
    launch_csr_stream<T, M_RESID>(A, x, x, b, nullptr, bidx, nullptr, out, nullptr, 0, s);
  else
    launch_csr<T, M_RESID>(A, nw, rows, bidx, x, b, nullptr, out, nullptr, s);
}
template <class T>
void VecOps<T>::spmv(const CsrV<T> &A, const T *x, T *y, bool accumulate, hipStream_t s) {
  if (A.rb) {
    if (accumulate)
      launch_csr_stream<T, M_SPMV_ADD>(A, x, x, nullptr, nullptr, nullptr, nullptr, y, nullptr, 0, s);
    else
      launch_csr_stream<T, M_SPMV>(A, x, x, nullptr, nullptr, nullptr, nullptr, y, nullptr, 0, s);
    return;
  }
  if (accumulate) launch_csr<T, M_SPMV_ADD>(A, A.n, nullptr, nullptr, x, nullptr, nullptr, y, nullptr, s);
  else launch_csr<T, M_SPMV>(A, A.n, nullptr, nullptr, x, nullptr, nullptr, y, nullptr, s);
}
template <class T>
void VecOps<T>::interp_fc(int64_t n, const int *map, const int *F, int64_t nF, const int *C,
                          int64_t nC, const CsrV<T> &Wp, const T *eC, const T *eF, T *z,
                          bool accumulate, hipStream_t s) {
  if (!Wp.rb) {
    interp(n, map, Wp, eC, eF, z, accumulate, s);
    return;
  }
  launch_csr_stream<T, M_INTERP>(Wp, eC, eF, nullptr, nullptr, nullptr, F, z, nullptr,
                                 accumulate ? 1 : 0, s);
  if (nC > 0) {
    k_scatter_c<T><<<grid_for(nC, 256), 256, 0, s>>>(C, nC, eC, z, accumulate ? 1 : 0);
    KCHK();
  }
}
template <class T>
void VecOps<T>::interp(int64_t n, const int *map, const CsrV<T> &Wp, const T *eC, const T *eF,
                       T *z, bool accumulate, hipStream_t s) {
  if (n <= 0) return;
  k_interp<T><<<grid_for(n * 8, 256), 256, 0, s>>>(n, map, Wp.rp, Wp.ci, Wp.v, eC, eF, z,
                                                   accumulate ? 1 : 0);
  KCHK();
}
// First l1-Jacobi sweep from zero and its residual: x = D^{-1} b in one pass, then
// r = b - A x with one gather per entry (gathering d^{-1} and b at every entry costs twice
// the gathers; the products and sums are the same)
template <class T>
__global__ void k_vmul(const T *__restrict__ a, const T *__restrict__ b, T *__restrict__ y,
                       int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] * b[i];
}
template <class T>
void VecOps<T>::l1_pre(const CsrV<T> &A, const T *dinv, const T *b, T *x, T *r, hipStream_t s) {
  if (A.rb) {
    if (A.n > 0) {
      k_vmul<T><<<grid_for(A.n, 256), 256, 0, s>>>(dinv, b, x, A.n);
      KCHK();
    }
    launch_csr_stream<T, M_RESID>(A, x, x, b, nullptr, nullptr, nullptr, r, nullptr, 0, s);
  } else {
    launch_csr<T, M_L1PRE>(A, A.n, nullptr, nullptr, nullptr, b, dinv, r, x, s);
  }
}
// restriction y = R r and the next level's x = D^{-1} y in one pass (matrices with row
// blocks; otherwise two)
template <class T>
void VecOps<T>::spmv_dx(const CsrV<T> &R, const T *r, const T *dinv_next, T *y, T *x_next,
                        hipStream_t s) {
  if (R.rb) {
    launch_csr_stream<T, M_SPMV_DX>(R, r, r, nullptr, dinv_next, nullptr, nullptr, y, x_next, 0,
                                    s);
    return;
  }
  spmv(R, r, y, false, s);
  if (R.n > 0) {
    k_vmul<T><<<grid_for(R.n, 256), 256, 0, s>>>(dinv_next, y, x_next, R.n);
    KCHK();
  }
}
template <class T>
void VecOps<T>::b_spmv_dx(const Bsr3V<T> &R, const T *r, const T *dinv_next, T *y, T *x_next,
                          hipStream_t s) {
  launch_bsr3<T, M_SPMV_DX>(R, r, nullptr, dinv_next, y, x_next, s);
}
// the first sweep's residual when x = D^{-1} b was formed by the restriction above
template <class T>
void VecOps<T>::l1_pre_given(const CsrV<T> &A, const T *b, const T *x, T *r, hipStream_t s) {
  if (A.rb) launch_csr_stream<T, M_RESID>(A, x, x, b, nullptr, nullptr, nullptr, r, nullptr, 0, s);
  else launch_csr<T, M_RESID>(A, A.n, nullptr, nullptr, x, b, nullptr, r, nullptr, s);
}
template <class T>
void VecOps<T>::b_l1_pre_given(const Bsr3V<T> &A, const T *b, const T *x, T *r, hipStream_t s) {
  launch_bsr3<T, M_RESID>(A, x, b, nullptr, r, nullptr, s);
}
template <class T>
void VecOps<T>::l1_post(const CsrV<T> &A, const T *dinv, const T *b, const T *x, T *y,
                        hipStream_t s) {
  if (A.rb)
    launch_csr_stream<T, M_L1POST>(A, x, x, b, dinv, nullptr, nullptr, y, nullptr, 0, s);
  else
    launch_csr<T, M_L1POST>(A, A.n, nullptr, nullptr, x, b, dinv, y, nullptr, s);
}
template <class T>
void VecOps<T>::b_spmv(const Bsr3V<T> &A, const T *x, T *y, bool accumulate, hipStream_t s) {
  if (accumulate) launch_bsr3<T, M_SPMV_ADD>(A, x, nullptr, nullptr, y, nullptr, s);
  else launch_bsr3<T, M_SPMV>(A, x, nullptr, nullptr, y, nullptr, s);
}
template <class T>
void VecOps<T>::b_l1_pre(const Bsr3V<T> &A, const T *dinv, const T *b, T *x, T *r, hipStream_t s) {
  if (A.n > 0) {
    k_vmul<T><<<grid_for(3 * A.n, 256), 256, 0, s>>>(dinv, b, x, 3 * A.n);
    KCHK();
  }
  launch_bsr3<T, M_RESID>(A, x, b, nullptr, r, nullptr, s);
}
template <class T>
void VecOps<T>::b_l1_post(const Bsr3V<T> &A, const T *dinv, const T *b, const T *x, T *y,
                          hipStream_t s) {
  launch_bsr3<T, M_L1POST>(A, x, b, dinv, y, nullptr, s);
}
template <class T>
void VecOps<T>::gemv(const T *M, int n, const T *x, T *y, hipStream_t s) {
  k_gemv<T><<<grid_for((int64_t)n * 64, 256), 256, 0, s>>>(M, n, x, y);
  KCHK();
}
template <class T>
void VecOps<T>::gather(const int *idx, int64_t n, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return;
  k_gather<T><<<grid_for(n, 256), 256, 0, s>>>(idx, n, x, y);
  KCHK();
}
template <class T>
void VecOps<T>::scatter_add(const int *idx, int64_t n, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_add<T><<<grid_for(n, 256), 256, 0, s>>>(idx, n, x, y);
  KCHK();
}
template <class T>
void VecOps<T>::jacobi_update(const int *F, int64_t nF, const T *dinv, T omega, const T *r, T *z,
                              hipStream_t s) {
  if (nF <= 0) return;
  k_jacobi_update<T><<<grid_for(nF, 256), 256, 0, s>>>(F, nF, dinv, omega, r, z);
  KCHK();
}
template <class T>
void VecOps<T>::jacobi_first(int64_t n, const int *map, const T *dinv, T omega, const T *v, T *z,
                             hipStream_t s) {
  if (n <= 0) return;
  k_jacobi_first<T><<<grid_for(n, 256), 256, 0, s>>>(n, map, dinv, omega, v, z);
  KCHK();
}
template <class T>
void VecOps<T>::block_jacobi(int64_t nblk, int nb, const T *inv, const T *v, T omega, T *z,
                             bool accumulate, hipStream_t s) {
  if (nblk <= 0) return;
  k_block_jacobi<T><<<grid_for(nblk, 256), 256, 0, s>>>(nblk, nb, inv, v, omega, z,
                                                        accumulate ? 1 : 0);
  KCHK();
}

template <class T>
void VecOps<T>::bsr_gs_sweep(const BsrBV<T> &A, const T *zin, const T *b, const T *inv, T omega,
                             T *zout, hipStream_t s) {
  if (A.nbr <= 0) return;
  require(A.br == A.bc && (A.br == 2 || A.br == 3), MGR_ERR_UNSUPPORTED, "sweep needs 2x2 or 3x3 blocks");
  if (A.nwin <= 0) {   // no blocks at all: zout = zin + omega D_B^{-1} b
    HIPCHK(hipMemcpyAsync(zout, zin, A.nbr * A.br * sizeof(T), hipMemcpyDeviceToDevice, s));
    block_jacobi(A.nbr, A.br, inv, b, omega, zout, true, s);
    return;
  }
  const double avg = (double)A.nblk / (double)A.nbr;
  const unsigned g = (unsigned)A.nwin;
#define GSL(BSZ, GG)                                                                        \
  k_bsr_cell<T, BSZ, BSZ, GG, CB_SWEEP><<<g, 256, 0, s>>>(A.rb, A.rp, A.ci, A.v, zin, b,   \
                                                          nullptr, inv, omega, zout)
  if (A.br == 2) {
    if (avg < 12) GSL(2, 4); else GSL(2, 8);
  } else {
    if (avg < 12) GSL(3, 4); else GSL(3, 8);
  }
#undef GSL
  KCHK();
}
template <class T>
void VecOps<T>::bsr_resid(const BsrBV<T> &A, const T *x, const T *b, const int *bidx, T *out,
                          hipStream_t s) {
  if (A.nbr <= 0) return;
  const int shape = A.br * 10 + A.bc;
  require(shape == 22 || shape == 33 || shape == 23, MGR_ERR_UNSUPPORTED, "unsupported cell block");
  if (A.nwin <= 0) {   // no blocks at all: out = b[bidx]
    if (bidx) gather(bidx, A.nbr * A.br, b, out, s);
    else HIPCHK(hipMemcpyAsync(out, b, A.nbr * A.br * sizeof(T), hipMemcpyDeviceToDevice, s));
    return;
  }
  const double avg = (double)A.nblk / (double)A.nbr;
  const unsigned g = (unsigned)A.nwin;
#define RSL(R, C, GG)                                                                     \
  k_bsr_cell<T, R, C, GG, CB_RESID><<<g, 256, 0, s>>>(A.rb, A.rp, A.ci, A.v, x, b, bidx,  \
                                                      nullptr, (T)0, out)
  if (shape == 22) {
    if (avg < 12) RSL(2, 2, 4); else RSL(2, 2, 8);
  } else if (shape == 33) {
    if (avg < 12) RSL(3, 3, 4); else RSL(3, 3, 8);
  } else {
    if (avg < 12) RSL(2, 3, 4); else RSL(2, 3, 8);
  }
#undef RSL
  KCHK();
}
template <class T>
void VecOps<T>::fill(T *p, T val, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fillv<T><<<grid_for(n, 256), 256, 0, s>>>(p, val, n);
  KCHK();
}

template <class T>
void VecOps<T>::resid_scale(const CsrV<T> &A, const T *dinv, const T *x, const T *b, T *out,
                            hipStream_t s) {
  if (A.rb)
    launch_csr_stream<T, M_RESID_SCALE>(A, x, x, b, dinv, nullptr, nullptr, out, nullptr, 0, s);
  else
    launch_csr<T, M_RESID_SCALE>(A, A.n, nullptr, nullptr, x, b, dinv, out, nullptr, s);
}
template <class T>
void VecOps<T>::vmul(const T *a, const T *b, T *y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_vmul<T><<<grid_for(n, 256), 256, 0, s>>>(a, b, y, n);
  KCHK();
}

template struct VecOps<float>;
template struct VecOps<double>;

void cast_to(const double *in, float *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<double, float><<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  KCHK();
}
void cast_to(const double *in, double *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<double, double><<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  KCHK();
}
void cast_from(const float *in, double *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<float, double><<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  KCHK();
}
void cast_from(const double *in, double *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<double, double><<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  KCHK();
}

void make_rowblocks(Csr &M, hipStream_t s) {
  // at least one block when there are rows, so that every row gets its epilogue
  const int64_t K = std::max<int64_t>((M.nnz + SNNZ - 1) / SNNZ, M.n > 0 ? 1 : 0);
  M.nblk = K;
  M.rb.alloc(K + 1, s);
  k_rowblocks32<<<grid_for(K + 1, 256), 256, 0, s>>>(M.n, M.rp.p, K, M.rb.p);
  KCHK();
}

}  // namespace mgr

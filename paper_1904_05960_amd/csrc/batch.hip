// Batched solve of many small independent systems.  The systems are placed on the diagonal
// of one block-diagonal matrix: one MGR setup and one preconditioned FGMRES serve them all,
// so every kernel launch of the setup, the V-cycle, the SpMV and the Gram-Schmidt passes
// covers every system at once.  Small systems are bound by launch latency, not by memory
// traffic; batching divides the number of launches per system by the batch size.
//
// The hierarchy of the union is the union of the systems' hierarchies: the C/F split, D_FF,
// W_p, the coarse product and the dropping are row-local (Sec. 5.2), and no strength edge
// (hence no aggregate) of the AMG crosses two systems.  Only the AMG's random priorities
// (hashed on the row index of the union) and its coarsest dense level differ from separate
// setups; both are still a valid preconditioner for every system.
//
// The Krylov process is kept per system (a single process over the union would need the
// residual polynomial to be small on all spectra at once, several times the iterations):
// each system has its own basis coefficients, Hessenberg matrix, Givens rotations, restart
// and convergence test, with its right-hand side scaled to unit norm.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace mgr {
namespace {

struct SysDesc {
  const int64_t *rp;
  const int *ci;
  const double *v;
  const int8_t *lab;
  const double *b;
  double *x;
  int64_t n, r0, e0;
};

__global__ void k_sys_nnz(const SysDesc *__restrict__ d, int k, int64_t *__restrict__ nnz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) nnz[i] = d[i].rp[d[i].n];
}

// system blockIdx.y: rows [r0, r0 + n) and entries [e0, e0 + nnz) of the union
__global__ void k_cat(const SysDesc *__restrict__ d, const int64_t *__restrict__ nnz,
                      int64_t *__restrict__ rp, int *__restrict__ ci, double *__restrict__ v,
                      int8_t *__restrict__ lab) {
  const SysDesc D = d[blockIdx.y];
  const int64_t m = nnz[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < D.n; i += stride) {
    rp[D.r0 + i] = D.rp[i] + D.e0;
    lab[D.r0 + i] = D.lab[i];
  }
  for (int64_t e = t0; e < m; e += stride) {
    ci[D.e0 + e] = D.ci[e] + (int)D.r0;
    v[D.e0 + e] = D.v[e];
  }
}

// out[k] = sum of squares of segment k (of a, or of a - c when c is given); one block per
// system, fixed reduction order
__global__ void k_seg_norm2(const SysDesc *__restrict__ d, const double *__restrict__ a,
                            const double *__restrict__ c, double *__restrict__ out) {
  __shared__ double sh[256];
  const SysDesc D = d[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < D.n; i += blockDim.x) {
    const double t = a ? (c ? a[D.r0 + i] - c[D.r0 + i] : a[D.r0 + i]) : D.b[i];
    s += t * t;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// bc = b / |b|, xc = x / |b| per segment (both 0 where |b| = 0)
__global__ void k_seg_scale_in(const SysDesc *__restrict__ d, const double *__restrict__ inv,
                               double *__restrict__ bc, double *__restrict__ xc) {
  const SysDesc D = d[blockIdx.y];
  const double w = inv[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bc[D.r0 + i] = D.b[i] * w;
    xc[D.r0 + i] = w != 0.0 ? D.x[i] * w : 0.0;
  }
}

// x = xc |b| per segment
__global__ void k_seg_scale_out(const SysDesc *__restrict__ d, const double *__restrict__ nrm,
                                const double *__restrict__ xc) {
  const SysDesc D = d[blockIdx.y];
  const double w = nrm[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D.n;
       i += (int64_t)gridDim.x * blockDim.x)
    D.x[i] = w != 0.0 ? xc[D.r0 + i] * w : 0.0;
}

// ---- FGMRES with one Arnoldi process per system ---------------------------------------
// The preconditioner and the SpMV act on the union (they are block diagonal), but every
// system keeps its own basis coefficients, Hessenberg matrix, Givens rotations and
// convergence test: its iterates are those of FGMRES on that system alone (up to the
// order of floating-point sums).  A system that has converged freezes: its next basis
// vectors are zero, which the block-diagonal operators keep zero.
constexpr int SKS = 72;        // stride of per-system coefficient arrays (>= restart + 1)
constexpr int SM = 64;         // largest restart

struct Seg {
  int64_t r0, n;
};

__device__ inline double seg_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum of acc over the 256 threads of a block, written to out[0] by thread 0 (fixed order)
__device__ inline void seg_block_sum(double v, double *out) {
  __shared__ double sh[4];
  v = seg_wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
}

// partial[(k * gridDim.x + blockIdx.x) * SKS + j] = V_j . w over the block's rows of
// system k = blockIdx.y (j < nv)
template <int NVB>
__global__ void __launch_bounds__(256) k_seg_multidot(const double *__restrict__ V, int64_t N,
                                                      int nv, const double *__restrict__ w,
                                                      const Seg *__restrict__ segs,
                                                      double *__restrict__ partial) {
  const Seg S = segs[blockIdx.y];
  double acc[NVB];
#pragma unroll
  for (int j = 0; j < NVB; ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256) {
    const int64_t gi = S.r0 + i;
    const double wi = w[gi];
#pragma unroll
    for (int j = 0; j < NVB; ++j)
      if (j < nv) acc[j] += V[(int64_t)j * N + gi] * wi;
  }
  double *out = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * SKS;
#pragma unroll
  for (int j = 0; j < NVB; ++j)
    if (j < nv) seg_block_sum(acc[j], out + j);
}

// w -= sum_j h_k[j] V_j on system k = blockIdx.y, then the partial dots of the new w with
// every V_j (norm_only = 0) or its squared norm (norm_only = 1, into slot 0)
template <int NVB>
__global__ void __launch_bounds__(256) k_seg_update(const double *__restrict__ V, int64_t N,
                                                    int nv, const double *__restrict__ h,
                                                    double *__restrict__ w,
                                                    const Seg *__restrict__ segs,
                                                    double *__restrict__ partial,
                                                    int norm_only) {
  const Seg S = segs[blockIdx.y];
  const double *hk = h + (int64_t)blockIdx.y * SKS;
  double acc[NVB];
#pragma unroll
  for (int j = 0; j < NVB; ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256) {
    const int64_t gi = S.r0 + i;
    double t[NVB];
#pragma unroll
    for (int j = 0; j < NVB; ++j) t[j] = j < nv ? V[(int64_t)j * N + gi] : 0.0;
    double wi = w[gi];
#pragma unroll
    for (int j = 0; j < NVB; ++j)
      if (j < nv) wi -= hk[j] * t[j];
    w[gi] = wi;
    if (norm_only) {
      acc[0] += wi * wi;
    } else {
#pragma unroll
      for (int j = 0; j < NVB; ++j) acc[j] += t[j] * wi;
    }
  }
  double *out = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * SKS;
  const int cnt = norm_only ? 1 : nv;
#pragma unroll
  for (int j = 0; j < NVB; ++j)
    if (j < cnt) seg_block_sum(acc[j], out + j);
}

// out[k * SKS + j] = sum over the nb blocks of system k (blockIdx.y) of partial j
// (j = blockIdx.x), in block order
__global__ void k_seg_reduce(const double *__restrict__ partial, int nb,
                             double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  const int k = blockIdx.y, j = blockIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[((int64_t)k * nb + b) * SKS + j];
  out[(int64_t)k * SKS + j] = s;
}

// Givens update of step j for every active system (one block each): as in the single
// solve, then the system stops (act = 0) when |g_{j+1}| <= tol or h_{j+1,j} = 0.
// scal[k] = 1 / h_{j+1,j} for the next basis vector, 0 once the system has stopped.
__global__ void k_seg_givens(double *__restrict__ H, double *__restrict__ cs,
                             double *__restrict__ sn, double *__restrict__ g,
                             const double *__restrict__ h1, const double *__restrict__ h2,
                             const double *__restrict__ hn2, int j, int m, double tol,
                             int *__restrict__ act, int *__restrict__ kseg,
                             double *__restrict__ scal, double *__restrict__ est) {
  const int k = blockIdx.x;
  if (threadIdx.x != 0) return;
  if (!act[k]) {
    scal[k] = 0.0;
    return;
  }
  const int ldh = m + 1;
  double *col = H + ((int64_t)k * m + j) * ldh;
  double *c = cs + (int64_t)k * m, *sv = sn + (int64_t)k * m, *gk = g + (int64_t)k * (m + 1);
  const double *a1 = h1 + (int64_t)k * SKS, *a2 = h2 + (int64_t)k * SKS;
  for (int i = 0; i <= j; ++i) col[i] = a1[i] + a2[i];
  const double hn = sqrt(hn2[(int64_t)k * SKS]);
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double u = c[i] * col[i] + sv[i] * col[i + 1];
    col[i + 1] = -sv[i] * col[i] + c[i] * col[i + 1];
    col[i] = u;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  c[j] = r != 0.0 ? a / r : 1.0;
  sv[j] = r != 0.0 ? b / r : 0.0;
  col[j] = r;
  col[j + 1] = 0.0;
  const double gj = gk[j];
  gk[j + 1] = -sv[j] * gj;
  gk[j] = c[j] * gj;
  kseg[k] = j + 1;
  est[k] = fabs(gk[j + 1]);
  const bool stop = !(fabs(gk[j + 1]) > tol) || !(hn > 0.0);
  if (stop) act[k] = 0;
  scal[k] = stop ? 0.0 : 1.0 / hn;
}

// v = w * scal[k] on each system
__global__ void k_seg_scale(const double *__restrict__ w, const double *__restrict__ scal,
                            double *__restrict__ v, const Seg *__restrict__ segs) {
  const Seg S = segs[blockIdx.y];
  const double a = scal[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[S.r0 + i] = w[S.r0 + i] * a;
}

// start of a cycle: v_0 = r / beta_k and g_k = (beta_k, 0, ...) for active systems; zero
// for the others
__global__ void k_seg_start(const double *__restrict__ r, const double *__restrict__ beta,
                            const int *__restrict__ act, double *__restrict__ V0,
                            double *__restrict__ g, int m, const Seg *__restrict__ segs) {
  const Seg S = segs[blockIdx.y];
  const int k = blockIdx.y;
  const double bk = act[k] ? beta[k] : 0.0;
  const double inv = bk > 0.0 ? 1.0 / bk : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)gridDim.x * blockDim.x)
    V0[S.r0 + i] = r[S.r0 + i] * inv;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[(int64_t)k * (m + 1) + i] = i == 0 ? bk : 0.0;
}

// y_k = H_k(1:kseg, 1:kseg)^{-1} g_k(1:kseg) by back substitution (one block per system)
__global__ void k_seg_trisolve(const double *__restrict__ H, const double *__restrict__ g,
                               const int *__restrict__ kseg, int m, double *__restrict__ y) {
  if (threadIdx.x != 0) return;
  const int k = blockIdx.x, kk = kseg[k];
  const int ldh = m + 1;
  const double *Hk = H + (int64_t)k * m * ldh;
  const double *gk = g + (int64_t)k * (m + 1);
  double *yk = y + (int64_t)k * SM;
  for (int i = kk - 1; i >= 0; --i) {
    double s = gk[i];
    for (int c = i + 1; c < kk; ++c) s -= Hk[(int64_t)c * ldh + i] * yk[c];
    yk[i] = s / Hk[(int64_t)i * ldh + i];
  }
}

// x += Z y_k on each system
__global__ void k_seg_xupdate(const double *__restrict__ Z, int64_t N,
                              const double *__restrict__ y, const int *__restrict__ kseg,
                              double *__restrict__ x, const Seg *__restrict__ segs) {
  const Seg S = segs[blockIdx.y];
  const int kk = kseg[blockIdx.y];
  const double *yk = y + (int64_t)blockIdx.y * SM;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gi = S.r0 + i;
    double s = x[gi];
    for (int c = 0; c < kk; ++c) s += Z[(int64_t)c * N + gi] * yk[c];
    x[gi] = s;
  }
}

// squared norm of each system's part of r (one block per system, fixed order)
__global__ void k_seg_sumsq(const double *__restrict__ r, const Seg *__restrict__ segs,
                            double *__restrict__ out) {
  const Seg S = segs[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < S.n; i += blockDim.x) {
    const double t = r[S.r0 + i];
    s += t * t;
  }
  seg_block_sum(s, out + blockIdx.x);
}


template <int NVB>
void seg_dots(const double *V, int64_t N, int nv, const double *w, const Seg *segs, int K,
              int bx, double *part, double *out, hipStream_t s) {
  k_seg_multidot<NVB><<<dim3(bx, K), 256, 0, s>>>(V, N, nv, w, segs, part);
  KCHK();
  k_seg_reduce<<<dim3(nv, K), 64, 0, s>>>(part, bx, out);
  KCHK();
}
template <int NVB>
void seg_upd(const double *V, int64_t N, int nv, const double *h, double *w, const Seg *segs,
             int K, int bx, double *part, double *out, bool norm_only, hipStream_t s) {
  k_seg_update<NVB><<<dim3(bx, K), 256, 0, s>>>(V, N, nv, h, w, segs, part, norm_only ? 1 : 0);
  KCHK();
  k_seg_reduce<<<dim3(norm_only ? 1 : nv, K), 64, 0, s>>>(part, bx, out);
  KCHK();
}

// FGMRES(m) over the union with one Arnoldi process per system (see above).  tol is the
// absolute residual each (unit-norm) system must reach.  Returns the final residual norm
// and the number of iterations of every system, and the number of steps taken.
mgr_status seg_fgmres(const mgr_csr &U, int64_t nnz, mgr_handle *h, const double *bc,
                      double *xc, const std::vector<Seg> &hsegs, int m, int maxit, double tol,
                      std::vector<double> &relres, std::vector<int> &iters, int &steps,
                      hipStream_t s) {
  const int K = (int)hsegs.size();
  const int64_t N = U.nrows;
  int64_t nmax = 1;
  for (const Seg &g : hsegs) nmax = std::max(nmax, g.n);
  const int bx = (int)std::min<int64_t>(64, std::max<int64_t>(1, (nmax + 1023) / 1024));
  const unsigned gv = (unsigned)std::min<int64_t>(1024, (nmax + 255) / 256);
  DArr<Seg> segs(K, s);
  HIPCHK(hipMemcpyAsync(segs.p, hsegs.data(), K * sizeof(Seg), hipMemcpyHostToDevice, s));
  DArr<int> rb(stream_blocks(nnz) + 1, s);
  rowblocks64(U, nnz, rb.p, s);
  DArr<double> V((size_t)(m + 1) * N, s), Z((size_t)m * N, s), w(N, s), r(N, s);
  DArr<double> H((size_t)K * m * (m + 1), s), cs((size_t)K * m, s), sn((size_t)K * m, s),
      g((size_t)K * (m + 1), s), y((size_t)K * SM, s);
  DArr<double> h1((size_t)K * SKS, s), h2((size_t)K * SKS, s), hn2((size_t)K * SKS, s),
      part((size_t)K * bx * SKS, s), scal(K, s), est(K, s), sq(K, s), beta(K, s);
  DArr<int> act(K, s), kseg(K, s);
  std::vector<int> hact(K), prev(K);
  std::vector<double> hsq(K), hbeta(K);
  relres.assign(K, 0.0);
  iters.assign(K, 0);
  steps = 0;
  for (;;) {
    spmv64_stream(U, nnz, rb.p, xc, bc, r.p, s);   // r = b - A x
    k_seg_sumsq<<<K, 256, 0, s>>>(r.p, segs.p, sq.p);
    KCHK();
    HIPCHK(hipMemcpyAsync(hsq.data(), sq.p, K * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool any = false;
    for (int k = 0; k < K; ++k) {
      hbeta[k] = std::sqrt(hsq[k]);
      relres[k] = hbeta[k];
      hact[k] = hbeta[k] > tol && std::isfinite(hbeta[k]);
      any = any || hact[k];
    }
    if (!any || steps >= maxit) break;
    HIPCHK(hipMemcpyAsync(act.p, hact.data(), K * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(beta.p, hbeta.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
    fill<int>(kseg.p, 0, K, s);
    k_seg_start<<<dim3(gv, K), 256, 0, s>>>(r.p, beta.p, act.p, V.p, g.p, m, segs.p);
    KCHK();
    for (int j = 0; j < m; ++j) {
      double *vj = V.p + (int64_t)j * N, *zj = Z.p + (int64_t)j * N;
      const mgr_status st = mgr_apply(h, vj, zj, s);
      if (st != MGR_OK) return st;
      spmv64_stream(U, nnz, rb.p, zj, nullptr, w.p, s);
      const int nv = j + 1;
#define SEGS(F, ...)                                   \
  if (nv <= 16) F<16>(__VA_ARGS__);                    \
  else if (nv <= 32) F<32>(__VA_ARGS__);               \
  else F<64>(__VA_ARGS__);
      SEGS(seg_dots, V.p, N, nv, w.p, segs.p, K, bx, part.p, h1.p, s)
      SEGS(seg_upd, V.p, N, nv, h1.p, w.p, segs.p, K, bx, part.p, h2.p, false, s)
      SEGS(seg_upd, V.p, N, nv, h2.p, w.p, segs.p, K, bx, part.p, hn2.p, true, s)
#undef SEGS
      k_seg_givens<<<K, 64, 0, s>>>(H.p, cs.p, sn.p, g.p, h1.p, h2.p, hn2.p, j, m, tol, act.p,
                                    kseg.p, scal.p, est.p);
      KCHK();
      prev = hact;
      HIPCHK(hipMemcpyAsync(hact.data(), act.p, K * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      ++steps;
      any = false;
      for (int k = 0; k < K; ++k) {
        iters[k] += prev[k];
        any = any || hact[k];
      }
      if (!any || j + 1 == m || steps >= maxit) break;
      k_seg_scale<<<dim3(gv, K), 256, 0, s>>>(w.p, scal.p, V.p + (int64_t)(j + 1) * N, segs.p);
      KCHK();
    }
    k_seg_trisolve<<<K, 64, 0, s>>>(H.p, g.p, kseg.p, m, y.p);
    KCHK();
    k_seg_xupdate<<<dim3(gv, K), 256, 0, s>>>(Z.p, N, y.p, kseg.p, xc, segs.p);
    KCHK();
  }
  return MGR_OK;
}

mgr_status bfail(const Error &e) {
  set_last_error(e.what());
  return e.st;
}

struct HandleGuard {
  mgr_handle *h = nullptr;
  ~HandleGuard() {
    if (h) mgr_destroy(h);
  }
};

}  // namespace
}  // namespace mgr

using namespace mgr;

extern "C" mgr_status mgr_batch_solve(int32_t k, const mgr_csr *A, const int8_t *const *labels,
                                      const double *const *b, double *const *x,
                                      const mgr_opts *opts, const fgmres_opts *o,
                                      double *relres, int32_t *iters, fgmres_result *res,
                                      void *stream) {
  set_last_error("");
  if (k <= 0 || k > 65535 || !A || !labels || !b || !x || !opts || !o || !relres) {
    set_last_error("mgr_batch_solve: null argument or k outside 1..65535");
    return MGR_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    std::vector<SysDesc> hd(k);
    int64_t N = 0;
    for (int i = 0; i < k; ++i) {
      const mgr_csr &M = A[i];
      require(M.block <= 1, MGR_ERR_ARG,
              "mgr_batch_solve: system " + std::to_string(i) + " is not a CSR matrix");
      require(M.nrows > 0 && M.nrows == M.ncols && M.row_ptr && M.col && M.val && labels[i] &&
                  b[i] && x[i],
              MGR_ERR_ARG, "mgr_batch_solve: system " + std::to_string(i) +
                               " is not a square non-empty matrix with labels, b and x");
      hd[i] = SysDesc{M.row_ptr, M.col, M.val, labels[i], b[i], x[i], M.nrows, N, 0};
      N += M.nrows;
    }
    require(N < ((int64_t)1 << 31), MGR_ERR_UNSUPPORTED, "mgr_batch_solve: too many rows");
    DArr<SysDesc> dd(k, s);
    DArr<int64_t> dnnz(k, s);
    HIPCHK(hipMemcpyAsync(dd.p, hd.data(), k * sizeof(SysDesc), hipMemcpyHostToDevice, s));
    k_sys_nnz<<<grid_for(k, 256), 256, 0, s>>>(dd.p, k, dnnz.p);
    KCHK();
    std::vector<int64_t> nnz(k);
    HIPCHK(hipMemcpyAsync(nnz.data(), dnnz.p, k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t E = 0, nmax = 0;
    for (int i = 0; i < k; ++i) {
      require(nnz[i] >= 0, MGR_ERR_ARG, "mgr_batch_solve: bad row pointers");
      hd[i].e0 = E;
      E += nnz[i];
      nmax = std::max(nmax, std::max(hd[i].n, nnz[i]));
    }
    require(E < ((int64_t)1 << 31), MGR_ERR_UNSUPPORTED, "mgr_batch_solve: too many entries");
    HIPCHK(hipMemcpyAsync(dd.p, hd.data(), k * sizeof(SysDesc), hipMemcpyHostToDevice, s));

    DArr<int64_t> rp(N + 1, s);
    DArr<int> ci(std::max<int64_t>(E, 1), s);
    DArr<double> v(std::max<int64_t>(E, 1), s), bc(N, s), xc(N, s), dn(k, s), dw(k, s);
    DArr<int8_t> lab(N, s);
    const int64_t gx = std::min<int64_t>((nmax + 255) / 256, 1024);
    k_cat<<<dim3((unsigned)gx, (unsigned)k), 256, 0, s>>>(dd.p, dnnz.p, rp.p, ci.p, v.p, lab.p);
    KCHK();
    HIPCHK(hipMemcpyAsync(rp.p + N, &E, sizeof(int64_t), hipMemcpyHostToDevice, s));

    // right-hand side norms; scale into the union
    k_seg_norm2<<<k, 256, 0, s>>>(dd.p, nullptr, nullptr, dn.p);
    KCHK();
    std::vector<double> nrm(k), inv(k);
    HIPCHK(hipMemcpyAsync(nrm.data(), dn.p, k * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int knz = 0;
    for (int i = 0; i < k; ++i) {
      nrm[i] = std::sqrt(nrm[i]);
      require(std::isfinite(nrm[i]), MGR_ERR_ARG,
              "mgr_batch_solve: right-hand side " + std::to_string(i) + " is not finite");
      inv[i] = nrm[i] > 0.0 ? 1.0 / nrm[i] : 0.0;
      knz += nrm[i] > 0.0;
    }
    HIPCHK(hipMemcpyAsync(dw.p, inv.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dn.p, nrm.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    const int64_t gv = std::min<int64_t>((nmax + 255) / 256, 1024);
    k_seg_scale_in<<<dim3((unsigned)gv, (unsigned)k), 256, 0, s>>>(dd.p, dw.p, bc.p, xc.p);
    KCHK();

    fgmres_result fr{};
    std::vector<double> rel;
    std::vector<int> its;
    int steps = 0;
    if (o->restart < 1 || o->restart > SM) {
      set_last_error("mgr_batch_solve: restart must lie in 1..64");
      return MGR_ERR_ARG;
    }
    if (knz > 0) {
      const mgr_csr U{N, N, rp.p, ci.p, v.p};
      HandleGuard g;
      const mgr_status st = mgr_setup(&U, lab.p, opts, stream, &g.h);
      if (st != MGR_OK) return st;
      std::vector<Seg> segs(k);
      for (int i = 0; i < k; ++i) segs[i] = Seg{hd[i].r0, hd[i].n};
      const mgr_status sf = seg_fgmres(U, E, g.h, bc.p, xc.p, segs, o->restart, o->maxit,
                                       o->rtol, rel, its, steps, s);
      if (sf != MGR_OK) return sf;
    } else {
      rel.assign(k, 0.0);
      its.assign(k, 0);
    }
    for (int i = 0; i < k; ++i) {
      relres[i] = nrm[i] > 0.0 ? rel[i] : 0.0;
      if (iters) iters[i] = its[i];
    }
    k_seg_scale_out<<<dim3((unsigned)gv, (unsigned)k), 256, 0, s>>>(dd.p, dn.p, xc.p);
    KCHK();
    HIPCHK(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int i = 0; i < k; ++i) worst = std::max(worst, relres[i]);
    fr.true_relres = worst;
    fr.converged = worst <= o->rtol ? 1 : 0;
    fr.iters = steps;
    if (res) {
      fr.history = res->history;
      fr.history_cap = res->history_cap;
      *res = fr;
    }
    if (!fr.converged) {
      set_last_error("mgr_batch_solve: not converged");
      return MGR_ERR_NOT_CONVERGED;
    }
    return MGR_OK;
  } catch (const Error &e) {
    return bfail(e);
  }
}

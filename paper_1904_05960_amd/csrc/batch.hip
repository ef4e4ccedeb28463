// Batched solve of many small independent systems.  The systems are placed on the diagonal
// of one block-diagonal matrix and solved as one: one MGR setup, one FGMRES, so every kernel
// launch of the setup, the V-cycle and the Krylov steps serves all of them at once.  Small
// systems are bound by launch latency, not by memory traffic; batching them divides the
// number of launches per system by the batch size.
//
// The hierarchy of the union is the union of the systems' hierarchies: the C/F split, D_FF,
// W_p, the coarse product and the dropping are row-local (Sec. 5.2), and no strength edge
// (hence no aggregate) of the AMG crosses two systems.  Only the AMG's random priorities
// (hashed on the row index of the union) and its coarsest dense level differ from separate
// setups; both are still a valid preconditioner for every system.
//
// Each right-hand side is scaled to unit norm before the solve and the union is solved to
// the absolute residual rtol: since the squared residual norms of the systems add up, each
// system then meets its own relative tolerance.  The solutions are scaled back.
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
                                      double *relres, fgmres_result *res, void *stream) {
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
    DArr<double> v(std::max<int64_t>(E, 1), s), bc(N, s), xc(N, s), y(N, s), dn(k, s),
        dw(k, s);
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
    if (res) {
      fr.history = res->history;
      fr.history_cap = res->history_cap;
    }
    mgr_status st = MGR_OK;
    if (knz > 0) {
      const mgr_csr U{N, N, rp.p, ci.p, v.p};
      HandleGuard g;
      st = mgr_setup(&U, lab.p, opts, stream, &g.h);
      if (st != MGR_OK) return st;
      fgmres_opts o2 = *o;
      o2.rtol = o->rtol / std::sqrt((double)knz);
      st = fgmres_solve(&U, g.h, bc.p, xc.p, &o2, nullptr, 0, &fr, stream);
      if (st != MGR_OK && st != MGR_ERR_NOT_CONVERGED) return st;
      // per-system residuals of the scaled systems (relative residuals of the originals)
      const mgr_status sp = mgr_spmv(&U, xc.p, y.p, stream);
      if (sp != MGR_OK) return sp;
      k_seg_norm2<<<k, 256, 0, s>>>(dd.p, bc.p, y.p, dw.p);
      KCHK();
      std::vector<double> r2(k);
      HIPCHK(hipMemcpyAsync(r2.data(), dw.p, k * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < k; ++i) relres[i] = nrm[i] > 0.0 ? std::sqrt(r2[i]) : 0.0;
    } else {
      for (int i = 0; i < k; ++i) relres[i] = 0.0;
    }
    k_seg_scale_out<<<dim3((unsigned)gv, (unsigned)k), 256, 0, s>>>(dd.p, dn.p, xc.p);
    KCHK();
    HIPCHK(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int i = 0; i < k; ++i) worst = std::max(worst, relres[i]);
    fr.true_relres = worst;
    fr.converged = worst <= o->rtol ? 1 : 0;
    if (res) *res = fr;
    if (st == MGR_ERR_NOT_CONVERGED || !fr.converged) {
      set_last_error("mgr_batch_solve: not converged");
      return MGR_ERR_NOT_CONVERGED;
    }
    return MGR_OK;
  } catch (const Error &e) {
    return bfail(e);
  }
}

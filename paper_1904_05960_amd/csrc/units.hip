// C-ABI access to the setup building blocks (sparse product with pinned order, transpose,
// drop/merge, strength + MIS(2) aggregation), so each can be checked on its own.
#include <memory>

#include "common.hpp"

struct mgr_owned_csr {
  mgr::Csr M;
  hipStream_t s = nullptr;
};

namespace mgr {
namespace {
mgr_status ufail(const Error &e) {
  set_last_error(e.what());
  return e.st;
}

void sizes_of(const Csr &M, int64_t out[3]) {
  out[0] = M.n;
  out[1] = M.m;
  out[2] = M.nnz;
}
}  // namespace
}  // namespace mgr

using namespace mgr;

extern "C" {

mgr_status mgr_spgemm(const mgr_csr *A, const mgr_csr *B, mgr_owned_csr **C, int64_t sizes[3],
                      void *stream) {
  if (!A || !B || !C || !sizes) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a, b;
    import_csr(A, a, s, flag.p);
    import_csr(B, b, s, flag.p);
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    spgemm(a, b, out->M, s, flag.p);
    check_flags(flag.p, s, "spgemm");
    sizes_of(out->M, sizes);
    *C = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_spgemm_grouped(const mgr_csr *A, const mgr_csr *B, int32_t group,
                              mgr_owned_csr **C, int64_t sizes[3], void *stream) {
  if (!A || !B || !C || !sizes || group < 1 || group > 3) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a, b;
    import_csr(A, a, s, flag.p);
    import_csr(B, b, s, flag.p);
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    spgemm(a, b, out->M, s, flag.p, group);
    check_flags(flag.p, s, "spgemm");
    sizes_of(out->M, sizes);
    *C = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_spgemm_b3(const mgr_csr *A, const mgr_csr *B, int32_t diag_b, mgr_owned_csr **C,
                         int64_t sizes[3], void *stream) {
  if (!A || !B || !C || !sizes) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a, b;
    import_csr(A, a, s, flag.p);
    import_csr(B, b, s, flag.p);
    require(a.m == b.n, MGR_ERR_ARG, "inner dimensions differ");
    Bsr3 ab, bb, cb;
    csr_to_bsr3(a, ab, s, flag.p, "A");
    csr_to_bsr3(b, bb, s, flag.p, "B");
    spgemm_b3(ab, bb, diag_b != 0, cb, s, flag.p);
    check_flags(flag.p, s, "block spgemm");
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    bsr3_to_csr(cb, out->M, s);
    HIPCHK(hipStreamSynchronize(s));
    sizes_of(out->M, sizes);
    *C = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_transpose(const mgr_csr *A, mgr_owned_csr **T, int64_t sizes[3], void *stream) {
  if (!A || !T || !sizes) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a;
    import_csr(A, a, s, flag.p);
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    transpose(a, out->M, true, s);
    HIPCHK(hipStreamSynchronize(s));
    sizes_of(out->M, sizes);
    *T = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_merge_drop(const mgr_csr *A, const mgr_csr *B, const double *w, int32_t nmax,
                          const int8_t *labels_c, mgr_owned_csr **S, int64_t sizes[3],
                          void *stream) {
  if (!A || !B || !S || !sizes) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a, b;
    import_csr(A, a, s, flag.p);
    import_csr(B, b, s, flag.p);
    DArr<int> rank;
    if (nmax >= 0) {
      require(labels_c != nullptr, MGR_ERR_ARG, "labels needed for dropping");
      label_rank(labels_c, b.n, rank, s);
    }
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    merge_drop(a, b, w, nmax, rank.p, out->M, true, s, flag.p);
    check_flags(flag.p, s, "merge/drop");
    sizes_of(out->M, sizes);
    *S = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_ilu(const mgr_csr *A, int32_t level, int32_t sweeps, mgr_owned_csr **F,
                   int64_t sizes[3], void *stream) {
  if (!A || !F || !sizes) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    require(sweeps >= 0 && sweeps <= 100000, MGR_ERR_ARG, "sweeps out of range");
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a;
    import_csr(A, a, s, flag.p);
    require(a.n == a.m, MGR_ERR_ARG, "A must be square");
    auto out = std::make_unique<mgr_owned_csr>();
    out->s = s;
    ilu_pattern_values(a, level, out->M, s, flag.p);
    DArr<int> dpos;
    ilu_factor(out->M, sweeps, dpos, s, flag.p);
    check_flags(flag.p, s, "ILU");
    HIPCHK(hipStreamSynchronize(s));
    sizes_of(out->M, sizes);
    *F = out.release();
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_dense_inverse(const double *D, double *Inv, int32_t n, void *stream) {
  if (!D || !Inv) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    require(n >= 1 && n <= 4096, MGR_ERR_ARG, "n must lie in [1, 4096]");
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    dense_inverse(const_cast<double *>(D), Inv, n, flag.p, s);
    HIPCHK(hipStreamSynchronize(s));
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_csr_to_bsr(const mgr_csr *A, int32_t br, int32_t bc, int32_t *brow_ptr,
                          int32_t *bcol, double *bval, int64_t capacity, int64_t *nblk,
                          void *stream) {
  if (!A || !nblk) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    const int shape = br * 10 + bc;
    require(shape == 22 || shape == 33 || shape == 23, MGR_ERR_ARG,
            "block shape must be 2x2, 3x3 or 2x3");
    require(A->nrows % br == 0 && A->ncols % bc == 0, MGR_ERR_ARG,
            "rows must be a multiple of br and columns of bc");
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a;
    import_csr(A, a, s, flag.p);
    check_flags(flag.p, s, "bsr import");
    BsrB B;
    csr_to_bsr_fill(a, br, bc, B, s);
    HIPCHK(hipStreamSynchronize(s));
    *nblk = B.nblk;
    if (bcol) {
      require(brow_ptr && bval, MGR_ERR_ARG, "brow_ptr and bval needed with bcol");
      require(capacity >= B.nblk, MGR_ERR_ARG, "capacity below the block count");
      HIPCHK(hipMemcpyAsync(brow_ptr, B.rp.p, (B.nbr + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
      if (B.nblk) {
        HIPCHK(hipMemcpyAsync(bcol, B.ci.p, B.nblk * sizeof(int), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(bval, B.v.p, B.nblk * br * bc * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      }
      HIPCHK(hipStreamSynchronize(s));
    }
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_aggregate(const mgr_csr *A, int32_t bs, double theta, int32_t level,
                         int32_t *agg, int64_t *nagg, void *stream) {
  if (!A || !agg || !nagg) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DArr<int> flag(1, s);
    clear_flag(flag.p, s);
    Csr a;
    import_csr(A, a, s, flag.p);
    AmgGraph G;
    strength_graph(a, bs, theta, G, s, flag.p);
    DArr<int> ag;
    int64_t na = 0;
    mis2_aggregate(G, level, ag, na, s);
    HIPCHK(hipMemcpyAsync(agg, ag.p, (a.n / bs) * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    *nagg = na;
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

mgr_status mgr_owned_export(const mgr_owned_csr *C, int64_t *row_ptr, int32_t *col, double *val,
                            void *stream) {
  if (!C) return MGR_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    const Csr &M = C->M;
    if (row_ptr) rowptr32_to_64(M.rp.p, row_ptr, M.n + 1, s);
    if (col && M.nnz)
      HIPCHK(hipMemcpyAsync(col, M.ci.p, M.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (val && M.nnz && M.v.p)
      HIPCHK(hipMemcpyAsync(val, M.v.p, M.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } catch (const Error &e) {
    return ufail(e);
  }
  return MGR_OK;
}

void mgr_owned_free(mgr_owned_csr *C) {
  if (C) {
    (void)hipStreamSynchronize(C->s);
    delete C;
  }
}

}  // extern "C"

// Internal declarations shared by the HIP translation units of libmgr355.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgr355.h"

namespace mgr {

// ------------------------------------------------------------------------------------
// errors
struct Error : std::runtime_error {
  mgr_status st;
  Error(mgr_status s, const std::string &m) : std::runtime_error(m), st(s) {}
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw ::mgr::Error(MGR_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define KCHK() HIPCHK(hipGetLastError())

inline void require(bool ok, mgr_status st, const std::string &msg) {
  if (!ok) throw Error(st, msg);
}

// device error flags raised by kernels (atomicOr on a device int)
enum : int {
  FLAG_ZERO_PIVOT = 1,
  FLAG_BAD_LABEL = 2,
  FLAG_ROW_TOO_LONG = 4,
  FLAG_NOT_BLOCKED = 8,
  FLAG_PATTERN = 16,
  FLAG_OVERFLOW = 32,
};

// ------------------------------------------------------------------------------------
// allocation (caller hook or stream-ordered hipMallocAsync)
void *dalloc(size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);

template <class T>
struct DArr {
  T *p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  bool own = true;   // false: a caller's array, read during one call and never freed here
  DArr() = default;
  DArr(size_t n_, hipStream_t s_) { alloc(n_, s_); }
  DArr(const DArr &) = delete;
  DArr &operator=(const DArr &) = delete;
  DArr(DArr &&o) noexcept : p(o.p), n(o.n), s(o.s), own(o.own) {
    o.p = nullptr;
    o.n = 0;
    o.own = true;
  }
  DArr &operator=(DArr &&o) noexcept {
    if (this != &o) {
      reset();
      p = o.p; n = o.n; s = o.s; own = o.own;
      o.p = nullptr; o.n = 0; o.own = true;
    }
    return *this;
  }
  ~DArr() { reset(); }
  void alloc(size_t n_, hipStream_t s_) {
    reset();
    s = s_;
    n = n_;
    p = n_ ? static_cast<T *>(dalloc(n_ * sizeof(T), s_)) : nullptr;
  }
  void borrow(T *q, size_t n_, hipStream_t s_) {
    reset();
    p = q;
    n = n_;
    s = s_;
    own = false;
  }
  void reset() {
    if (p && own) dfree(p, s);
    p = nullptr;
    n = 0;
    own = true;
  }
  size_t bytes() const { return own ? n * sizeof(T) : 0; }
  T *get() const { return p; }
};

// ------------------------------------------------------------------------------------
// matrices
// Device CSR with int32 row pointers (nnz < 2^31) and FP64 values, owning its arrays.
struct Csr {
  int64_t n = 0, m = 0, nnz = 0;
  DArr<int> rp, ci;
  DArr<double> v;
  DArr<int> rb;              // CSR-stream row blocks of apply matrices (nblk + 1), or empty
  int64_t nblk = 0;
  size_t bytes() const { return rp.bytes() + ci.bytes() + v.bytes() + rb.bytes(); }
};

// 3x3 block CSR with row-major blocks (9 doubles per block, entry (r, s) at 3r + s), used
// by the nodal AMG setup products.
struct Bsr3 {
  int64_t nb = 0, mb = 0, nnzb = 0;
  DArr<int> rp, ci;
  DArr<double> v;
};

// Read-only views used by apply kernels (T = float or double).
template <class T>
struct CsrV {
  int64_t n = 0, m = 0, nnz = 0;
  const int *rp = nullptr, *ci = nullptr;
  const T *v = nullptr;
  const int *rb = nullptr;   // CSR-stream row blocks (nblk + 1) when set
  int64_t nblk = 0;
};
// 3x3 block CSR: n, m in block rows/cols, values row-major per block (9 per block).
template <class T>
struct Bsr3V {
  int64_t n = 0, m = 0, nnzb = 0;
  const int *rp = nullptr, *ci = nullptr;
  const T *v = nullptr;
};

// br x bc block CSR of a matrix whose rows come in groups of br (the unknowns of a cell)
// and whose columns come in groups of bc: block row I = rows br I .. br I + br - 1, a block
// for every column group c / bc any of them touches, values row-major per block (zeros
// stored), and the stream windows of its apply kernels.
struct BsrB {
  int64_t nbr = 0, nblk = 0, nwin = 0;
  int br = 0, bc = 0;
  DArr<int> rp, ci, rb;
  DArr<double> v;
  size_t bytes() const { return rp.bytes() + ci.bytes() + rb.bytes() + v.bytes(); }
};
template <class T>
struct BsrBV {
  int64_t nbr = 0, nblk = 0, nwin = 0;
  int br = 0, bc = 0;
  const int *rp = nullptr, *ci = nullptr, *rb = nullptr;
  const T *v = nullptr;
};

// ------------------------------------------------------------------------------------
// launch geometry
inline unsigned grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return static_cast<unsigned>(g);
}

// ------------------------------------------------------------------------------------
// primitives (prims.hip)
int64_t exclusive_scan_i32(const int *in, int *out, int64_t n, hipStream_t s);   // out[n]=total
int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// no readback; the 64-bit total goes to *total64 (device) when given
void exclusive_scan_i32_async(const int *in, int *out, int64_t n, hipStream_t s,
                              int64_t *total64 = nullptr);
template <class T> void fill(T *p, T val, int64_t n, hipStream_t s);
int64_t reduce_max_i64(const int64_t *p, int64_t n, hipStream_t s);
int64_t reduce_sum_i32(const int *p, int64_t n, hipStream_t s);
double reduce_max_f64(const double *p, int64_t n, hipStream_t s);
void cast_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t s);
void cast_f32_to_f64(const float *in, double *out, int64_t n, hipStream_t s);
void negate_f64(double *p, int64_t n, hipStream_t s);
void rowptr64_to_32(const int64_t *in, int *out, int64_t n1, int *flag, hipStream_t s);
void rowptr32_to_64(const int *in, int64_t *out, int64_t n1, hipStream_t s);
void stream_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);
int read_flag(const int *dflag, hipStream_t s);      // synchronises
void *pinned_scratch();                               // 256 pinned host bytes per thread
void d2h_sync(void *dst, const void *src, size_t bytes, hipStream_t s);  // <= 256 bytes, waits
struct D2HPart {
  void *dst;
  const void *src;
  size_t bytes;
};
void d2h_sync_parts(const D2HPart *parts, int np, hipStream_t s);  // one wait for all parts
void clear_flag(int *dflag, hipStream_t s);
// throws the error that the raised device flags describe (synchronises)
void check_flags(const int *dflag, hipStream_t s, const char *where);

// ------------------------------------------------------------------------------------
// sparse setup kernels (spgemm.hip, setup.hip, amg_setup.hip)
// `group` > 1: rows of A in groups of that many rows (2 or 3) that likely share one column
// pattern; verified, and the groups then share their symbolic work, loads and hash tables
void spgemm(const Csr &A, const Csr &B, Csr &C, hipStream_t s, int *dflag, int group = 1);
void transpose(const Csr &A, Csr &T, bool values, hipStream_t s);
// S = A - diag(w) * B restricted to entries of B kept by the drop rule.
//   keep rule: nmax < 0 keeps all of B; otherwise per row the entries whose column c has
//   lrank[c] == lrank[row] plus the nmax largest |b| (ties: smaller column).
//   tol >= 0 replaces the nmax rule: the lrank entries plus the nonzero entries with
//   |b| >= tol * (largest |b| of the row).
//   w may be null (w = 1).  If values == false, only the union pattern is formed.
void merge_drop(const Csr &A, const Csr &B, const double *w, int nmax, const int *lrank,
                Csr &S, bool values, hipStream_t s, int *dflag, double tol = -1.0);
void drop_only(const Csr &B, int nmax, const int *lrank, Csr &G, hipStream_t s, int *dflag,
               double tol = -1.0);

struct CfSplit {
  int64_t n = 0, nF = 0, nC = 0;
  DArr<int> F, C;         // index lists (ascending)
  DArr<int> map;          // map[i] = F index if F point, else -(C index) - 1
};
void cf_split(const int8_t *labels, int64_t n, uint32_t fmask, CfSplit &cf, hipStream_t s,
              int *dflag);
// rank[x] = number of points before x with the label of x; `present` = mask of the labels
// that occur (others are skipped)
void label_rank(const int8_t *labels, int64_t n, DArr<int> &rank, hipStream_t s,
                uint32_t present = 0xffu);
// mask of the labels that occur (ARG error for labels outside [0, 7]); synchronises
uint32_t label_mask(const int8_t *labels, int64_t n, hipStream_t s);
// true when labels[i] == labels[i % p] for all i; synchronises
bool labels_periodic(const int8_t *labels, int64_t n, int p, hipStream_t s);
void gather_labels(const int8_t *labels, const int *idx, int64_t n, int8_t *out,
                   hipStream_t s);
// A_FF, A_FC, A_CF, A_CC of A under cf; dFF = diag(A_FF) (0 where missing).
// Entries (i, k) of A_CF with rank[C[i]] == rank[F[k]] (same entity), order kept.
void same_entity_filter(const Csr &Acf, const int *C, const int *F, const int *rank, Csr &out,
                        hipStream_t s);
void extract_blocks(const Csr &A, const CfSplit &cf, Csr *Aff, Csr &Afc, Csr &Acf, Csr &Acc,
                    double *dFF, hipStream_t s);
// M = D^{-1} A_FC (values a/d), in place on a copy.
void scale_rows_div(Csr &M, const double *d, hipStream_t s);
void check_nonzero(const double *d, int64_t n, int *dflag, hipStream_t s);
void copy_csr(const Csr &A, Csr &B, hipStream_t s);
// `borrow`: a scalar CSR's column and value arrays are used in place (the caller's arrays
// must outlive B); otherwise copied
void import_csr(const mgr_csr *A, Csr &B, hipStream_t s, int *dflag, bool borrow = false);
uint64_t pattern_hash(const Csr &A, hipStream_t s);

// AMG setup
struct AmgGraph {
  int64_t n = 0;
  DArr<int> rp, ci;
};
// bs = 3: `blocks`, when given, is the 3x3 block form of A (its node pattern is used)
void strength_graph(const Csr &A, int bs, double theta, AmgGraph &G, hipStream_t s,
                    int *dflag, const Bsr3 *blocks = nullptr);
void mis2_aggregate(const AmgGraph &G, int level, DArr<int> &agg, int64_t &nagg,
                    hipStream_t s);
void tentative(const DArr<int> &agg, int64_t nnode, int bs, int64_t nagg, Csr &T,
               hipStream_t s);
double gershgorin_rho(const Csr &A, hipStream_t s, int *dflag);
// d = diag(A), l1inv = 1 / (sum_j |a_ij|) in ascending order; returns
// max_i sum_j |a_ij| / |a_ii| (ZERO_PIVOT on a zero diagonal); synchronises
double row_stats(const Csr &A, double *d, double *l1inv, hipStream_t s, int *dflag);
void diag_of(const Csr &A, double *d, hipStream_t s);
void omega_over_diag(const double *d, double omega, double *w, int64_t n, hipStream_t s);
void l1_inverse(const Csr &A, double *dinv, hipStream_t s);

// dense (dense.hip)
void csr_to_dense(const Csr &A, double *D, hipStream_t s);
void dense_inverse(double *D, double *Inv, int n, int *dflag, hipStream_t s);

// BSR3 conversion: scalar CSR with full 3x3 blocks -> block CSR
// Symbolic sparse product: crp (n + 1, caller-allocated) gets the row pointers of the
// pattern of A B (A: n rows; B: bn x bm), cnnz its size; ub_out, when given, receives the
// number of products of every row (sum of the lengths of the rows of B it selects).
// Optional bucketing of the output rows run right after the row pointers are formed
// (`launch` zeroes and fills `counts` on the stream, given the per-row product bounds); the
// counts are then read back together with the symbolic totals into `host`.
struct SymBucket {
  std::function<void(const int64_t *ub)> launch;
  const int *counts = nullptr;
  int *host = nullptr;
  int nc = 0;
};
void spgemm_symbolic(int64_t n, const int *arp, const int *aci, int64_t annz, const int *brp,
                     const int *bci, int64_t bn, int64_t bm, int64_t bnnz, int *crp,
                     int64_t &cnnz, hipStream_t s, int *dflag, DArr<int64_t> *ub_out = nullptr,
                     const SymBucket *bk = nullptr);
// C = A B on 3x3 block matrices: the scalar product of their expansions, bit for bit (B's
// blocks diagonal when diagb).
void spgemm_b3(const Bsr3 &A, const Bsr3 &B, bool diagb, Bsr3 &C, hipStream_t s, int *dflag);
// CSR-stream row blocks of M (block k owns the rows whose entries start in the k-th window
// of the stream kernels); kept with the matrix for the apply kernels.
void make_rowblocks(Csr &M, hipStream_t s);
// rows `rows` (ascending, nr of them) of A as a CSR matrix of its own (columns unchanged)
void gather_rows(const Csr &A, const int *rows, int64_t nr, Csr &out, hipStream_t s);
// windows of 512 blocks over a block row pointer: rb[k] = first block row whose first block
// is at or beyond 512 k, rb[nwin] = nbr; returns nwin (0 without blocks)
int64_t make_block_windows(const int *rp, int64_t nbr, int64_t nblk, DArr<int> &rb,
                           hipStream_t s);
// (br, bc) = (2, 2), (3, 3) or (2, 3); with the windows of the apply kernels
void csr_to_bsr_fill(const Csr &A, int br, int bc, BsrB &B, hipStream_t s);
void csr_to_bsr3(const Csr &A, Bsr3 &B, hipStream_t s, int *dflag, const char *what);
void bsr3_to_csr(const Bsr3 &B, Csr &C, hipStream_t s);
// R = P^T (block pattern transposed, each block transposed)
void bsr3_transpose(const Bsr3 &P, Bsr3 &R, hipStream_t s);
// tentative prolongator of a nodal aggregation: block (node, agg(node)) = I3
void tentative_b3(const DArr<int> &agg, int64_t nnode, int64_t nagg, Bsr3 &T, hipStream_t s);
void csr_to_bsr3(const Csr &A, DArr<int> &rp, DArr<int> &ci, DArr<double> &v, int64_t &nb,
                 int64_t &mb, int64_t &nnzb, hipStream_t s, int *dflag, const char *what);
// setup trace on stderr when MGR355_TRACE is set
void trace(const std::string &msg);
// message returned by mgr_last_error() on this thread
void set_last_error(const std::string &msg);
// block-Jacobi inverses over consecutive nb x nb diagonal blocks (nb = 2 or 3)
void block_diag_inverse(const Csr &A, int nb, double *inv, hipStream_t s, int *dflag);
// fine-grained ILU(k) global smoother (ilu.hip)
void block_scale(const Csr &A, int nb, const double *binv, Csr &As, hipStream_t s, int *dflag);
// row pointers and columns of the block-diagonal n x n matrix of nb x nb blocks
void block_diag_pattern(int64_t n, int nb, int *rp, int *ci, hipStream_t s);
void ilu_pattern_values(const Csr &As, int level, Csr &S, hipStream_t s, int *dflag);
void ilu_factor(Csr &S, int sweeps, DArr<int> &dpos, hipStream_t s, int *dflag);
void ilu_split(const Csr &S, const DArr<int> &dpos, Csr &Lo, Csr &Up, DArr<double> &dinv,
               hipStream_t s);
template <class T> void axpy(int64_t n, T alpha, const T *x, T *y, hipStream_t s);
// y[idx[i]] += alpha * x[i]
template <class T>
void scatter_axpy(const int *idx, int64_t n, T alpha, const T *x, T *y, hipStream_t s);
// M_ik /= d_k (column scaling by division, IEEE rounding)
void scale_cols_div(Csr &M, const double *d, hipStream_t s);
// multicolour block Gauss-Seidel (bgs.hip): colouring of the cells of nb interleaved rows
// (color_ptr: host offsets per colour into `cells`; color: colour of every cell) and one
// colour's update x_e += D_e^{-1} (b - A x)_e for its cells
void bgs_setup(const Csr &A, int nb, std::vector<int> &color_ptr, DArr<int> &cells,
               DArr<int> &color, hipStream_t s, int *dflag);
template <class T>
void bgs_color_sweep(const CsrV<T> &A, int nb, const int *cells, int ncells, const T *binv,
                     const T *b, T *x, hipStream_t s);

// ------------------------------------------------------------------------------------
// apply kernels (apply.hip), T = float or double
template <class T>
struct VecOps {
  static void resid(const CsrV<T> &A, int64_t nw, const int *rows, const int *bidx,
                    const T *x, const T *b, T *out, hipStream_t s);
  static void spmv(const CsrV<T> &A, const T *x, T *y, bool accumulate, hipStream_t s);
  static void interp(int64_t n, const int *map, const CsrV<T> &Wp, const T *eC,
                     const T *eF, T *z, bool accumulate, hipStream_t s);
  // the same with the F and C lists: z_F (+)= [eF] + W_p e_C, z_C (+)= e_C
  static void interp_fc(int64_t n, const int *map, const int *F, int64_t nF, const int *C,
                        int64_t nC, const CsrV<T> &Wp, const T *eC, const T *eF, T *z,
                        bool accumulate, hipStream_t s);
  static void l1_pre(const CsrV<T> &A, const T *dinv, const T *b, T *x, T *r,
                     hipStream_t s);
  static void l1_post(const CsrV<T> &A, const T *dinv, const T *b, const T *x, T *y,
                      hipStream_t s);
  static void b_spmv(const Bsr3V<T> &A, const T *x, T *y, bool accumulate, hipStream_t s);
  static void b_l1_pre(const Bsr3V<T> &A, const T *dinv, const T *b, T *x, T *r,
                       hipStream_t s);
  static void b_l1_post(const Bsr3V<T> &A, const T *dinv, const T *b, const T *x, T *y,
                        hipStream_t s);
  // restriction y = R r that also writes the next level's first iterate D^{-1} y
  static void spmv_dx(const CsrV<T> &R, const T *r, const T *dinv_next, T *y, T *x_next,
                      hipStream_t s);
  static void b_spmv_dx(const Bsr3V<T> &R, const T *r, const T *dinv_next, T *y, T *x_next,
                        hipStream_t s);
  // first sweep's residual r = b - A x with x = D^{-1} b already formed
  static void l1_pre_given(const CsrV<T> &A, const T *b, const T *x, T *r, hipStream_t s);
  static void b_l1_pre_given(const Bsr3V<T> &A, const T *b, const T *x, T *r, hipStream_t s);
  static void gemv(const T *M, int n, const T *x, T *y, hipStream_t s);
  static void gather(const int *idx, int64_t n, const T *x, T *y, hipStream_t s);
  static void scatter_add(const int *idx, int64_t n, const T *x, T *y, hipStream_t s);
  static void jacobi_update(const int *F, int64_t nF, const T *dinv, T omega, const T *r,
                            T *z, hipStream_t s);
  static void jacobi_first(int64_t n, const int *map, const T *dinv, T omega, const T *v,
                           T *z, hipStream_t s);
  static void block_jacobi(int64_t nblk, int nb, const T *inv, const T *v, T omega, T *z,
                           bool accumulate, hipStream_t s);
  // one block-Jacobi sweep on a cell-blocked level: zout = zin + omega D_B^{-1} (b - A zin)
  static void bsr_gs_sweep(const BsrBV<T> &A, const T *zin, const T *b, const T *inv, T omega,
                           T *zout, hipStream_t s);
  // out_i = b[bidx ? bidx[i] : i] - (A x)_i on a cell-blocked matrix (any block shape)
  static void bsr_resid(const BsrBV<T> &A, const T *x, const T *b, const int *bidx, T *out,
                        hipStream_t s);
  static void fill(T *p, T val, int64_t n, hipStream_t s);
  // out = dinv .* (b - A x)
  static void resid_scale(const CsrV<T> &A, const T *dinv, const T *x, const T *b, T *out,
                          hipStream_t s);
  static void vmul(const T *a, const T *b, T *y, int64_t n, hipStream_t s);
};
void cast_to(const double *in, float *out, int64_t n, hipStream_t s);
void cast_to(const double *in, double *out, int64_t n, hipStream_t s);
void cast_from(const float *in, double *out, int64_t n, hipStream_t s);
void cast_from(const double *in, double *out, int64_t n, hipStream_t s);

// ------------------------------------------------------------------------------------
// FP64 Krylov kernels (krylov.hip)
void spmv64(const mgr_csr &A, const double *x, double *y, hipStream_t s);
void resid64(const mgr_csr &A, const double *x, const double *b, double *r, hipStream_t s);
int krylov_partials_blocks();
// The *_partials functions write one partial sum per block and return the number of
// blocks; reduce_partials adds those in a fixed order.
// partial[blk * KS + k] = sum over the rows of blk of V_k . w  (k < nv)
int multidot_partials(const double *V, int64_t n, int nv, const double *w, double *partial,
                      hipStream_t s);
// w -= sum_k h[k] V_k ; partial dots of the updated w with V_k (k < nv) or its norm^2
int cgs_update_partials(const double *V, int64_t n, int nv, const double *h, double *w,
                        double *partial, bool norm_only, hipStream_t s);
void reduce_partials(const double *partial, int nblk, int nv, double *out, bool add,
                     hipStream_t s);
void givens_step(double *H, double *cs, double *sn, double *g, const double *h1,
                 const double *h2, const double *hn2, int j, int ldh, double *scal,
                 double *unused, hipStream_t s);
void scale_vec(const double *w, const double *scale, double *v, int64_t n, hipStream_t s);
// v = w * scale[0], with a copy of v in float or double (the preconditioner's input)
void scale_vec_copy(const double *w, const double *scale, double *v, float *vf, int64_t n,
                    hipStream_t s);
void scale_vec_copy(const double *w, const double *scale, double *v, double *vd, int64_t n,
                    hipStream_t s);
void tri_solve_and_update(const double *H, const double *g, int k, int ldh, const double *Z,
                          int64_t n, double *x, double *y, hipStream_t s);
int norm2_partials(const double *r, int64_t n, double *partial, hipStream_t s);
int dot_partials(const double *a, const double *b, int64_t n, double *partial,
                  hipStream_t s);
void start_cycle_host_beta(const double *r, double beta, double *V0, double *g, int64_t n,
                           int mp1, hipStream_t s);
void spmv64_avg(const mgr_csr &A, const double *x, const double *b, double *y, double avg,
                hipStream_t s);
// CSR-stream SpMV (FP64, int64 row pointers): row blocks of about 2048 entries
int64_t stream_blocks(int64_t nnz);
int64_t bsr_stream_blocks(int64_t nnzb, int bs);
void bsr_rowblocks64(const mgr_csr &A, int64_t nnzb, int *rb, hipStream_t s);
void bsr_spmv64_stream(const mgr_csr &A, int64_t nnzb, const int *rb, const double *x,
                       const double *b, double *y, hipStream_t s);
// scalar rows of a CSR or BSR descriptor
inline int64_t scalar_rows(const mgr_csr &A) { return A.nrows * (A.block > 1 ? A.block : 1); }
void rowblocks64(const mgr_csr &A, int64_t nnz, int *rb, hipStream_t s);
void spmv64_stream(const mgr_csr &A, int64_t nnz, const int *rb, const double *x, const double *b,
                   double *y, hipStream_t s);

// ------------------------------------------------------------------------------------
// profiling hooks (abi.hip)
struct Prof {
  static bool on(int family);
  static void begin(int family, hipStream_t s);
  static void end(int family, hipStream_t s, double bytes);
};

}  // namespace mgr

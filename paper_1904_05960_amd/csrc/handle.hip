// Host orchestration of libmgr355: allocation, the MGR hierarchy (Sec. 5.2), the AMG
// hierarchies, the V-cycle of Algorithm 2, flexible GMRES, and the C ABI of mgr355.h.
#include <algorithm>
#include <atomic>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <thread>

#include "common.hpp"

namespace mgr {

// ===================================================================================
// allocation
// Default: a caching allocator.  Blocks are rounded up to size bins and kept, after free,
// on a free list of the stream they were freed on; a later allocation on the same stream
// reuses them in stream order (work queued on that stream before the free completes before
// anything queued after the reuse).  Blocks are obtained with hipMalloc; when it fails the
// cache is released (after a device synchronisation) and the allocation retried.
static void *(*g_alloc)(size_t, void *, void *) = nullptr;
static void (*g_free)(void *, void *, void *) = nullptr;
static void *g_ctx = nullptr;

namespace {
struct CacheKey {
  hipStream_t s;
  size_t bin;
  bool operator<(const CacheKey &o) const {
    return s < o.s || (s == o.s && bin < o.bin);
  }
};
std::mutex g_cache_mu;
// Held while a V-cycle is captured into a graph.  A device-wide wait or a hipFree in one
// thread while another thread captures invalidates that capture, so the paths that return
// cached blocks to HIP take it first (always after g_cache_mu; a capture allocates nothing).
std::mutex g_capture_mu;
std::map<CacheKey, std::vector<void *>> g_cache;  // free blocks
std::map<void *, size_t> g_live;                  // block -> bin size
size_t g_cached_bytes = 0;
size_t g_live_bytes = 0, g_peak_bytes = 0;        // bytes handed out (hook-less path)
long g_misses = 0;                                // hipMalloc calls (for the setup trace)
double g_miss_us = 0.0;

size_t bin_of(size_t bytes) {
  if (bytes <= 512) return 512;
  // powers of two up to 1 MiB, then multiples of 1/8 of the next power of two
  size_t p = 1;
  while (p < bytes) p <<= 1;
  if (p <= ((size_t)1 << 20)) return p;
  const size_t step = p / 8;
  return (bytes + step - 1) / step * step;
}

void release_cache_locked() {
  for (auto &kv : g_cache)
    for (void *q : kv.second) {
      (void)hipFree(q);
    }
  g_cache.clear();
  g_cached_bytes = 0;
}
}  // namespace

void *dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  if (g_alloc) {
    void *p = g_alloc(bytes, s, g_ctx);
    if (!p) throw Error(MGR_ERR_ALLOC, "allocator hook returned NULL");
    return p;
  }
  const size_t bin = bin_of(bytes);
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto it = g_cache.find(CacheKey{s, bin});
  if (it != g_cache.end() && !it->second.empty()) {
    void *p = it->second.back();
    it->second.pop_back();
    g_cached_bytes -= bin;
    g_live[p] = bin;
    g_live_bytes += bin;
    g_peak_bytes = std::max(g_peak_bytes, g_live_bytes);
    return p;
  }
  void *p = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e = hipMalloc(&p, bin);
  ++g_misses;
  g_miss_us += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> cg(g_capture_mu);
    (void)hipDeviceSynchronize();
    release_cache_locked();
    e = hipMalloc(&p, bin);
  }
  if (e != hipSuccess || !p)
    throw Error(MGR_ERR_ALLOC, std::string("hipMalloc(") + std::to_string(bin) + "): " +
                                   hipGetErrorString(e));
  g_live[p] = bin;
  g_live_bytes += bin;
  g_peak_bytes = std::max(g_peak_bytes, g_live_bytes);
  return p;
}

void dfree(void *p, hipStream_t s) {
  if (!p) return;
  if (g_free) {
    g_free(p, s, g_ctx);
    return;
  }
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  const size_t bin = it->second;
  g_live.erase(it);
  g_live_bytes -= bin;
  g_cache[CacheKey{s, bin}].push_back(p);
  g_cached_bytes += bin;
}

// lines of the setup's second host thread (the F-relaxation AMG) carry the tag "F"
thread_local const char *t_trace_tag = " ";

void trace(const std::string &msg) {
  static const bool on = std::getenv("MGR355_TRACE") != nullptr;
  if (!on) return;
  static auto t0 = std::chrono::steady_clock::now();
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::fprintf(stderr, "[mgr355 %10.3f ms %s] %s\n", ms, t_trace_tag, msg.c_str());
}

// ===================================================================================
// profiling: HIP events around launches of a kernel family
namespace {
struct ProfFamily {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<double> bytes;
  size_t used = 0;
};
ProfFamily g_prof[2];
std::mutex g_prof_mu;
}  // namespace

bool Prof::on(int f) { return g_prof[f].on; }
void Prof::begin(int f, hipStream_t s) {
  ProfFamily &P = g_prof[f];
  if (P.used == P.ev.size()) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    P.ev.emplace_back(a, b);
    P.bytes.push_back(0.0);
  }
  HIPCHK(hipEventRecord(P.ev[P.used].first, s));
}
void Prof::end(int f, hipStream_t s, double bytes) {
  ProfFamily &P = g_prof[f];
  HIPCHK(hipEventRecord(P.ev[P.used].second, s));
  P.bytes[P.used] = bytes;
  ++P.used;
}

// ===================================================================================
// hierarchy structures
struct AmgLevel {
  Csr A, P, R;               // FP64 scalar CSR (A of the last level is the dense-solved one)
  DArr<int> agg;
  int64_t nagg = 0;
  double omega = 0.0;
  DArr<double> dinv;         // l1 row sums inverted
  // nodal (3x3 block) forms: FP64 row-major blocks during the setup products
  std::unique_ptr<Bsr3> Ab64, Pb64, Rb64;
  // nodal (3x3 block) copies for the V-cycle
  DArr<int> Ab_rp, Ab_ci, Pb_rp, Pb_ci, Rb_rp, Rb_ci;
  int64_t nb = 0, ncb = 0, Ab_nnzb = 0, Pb_nnzb = 0, Rb_nnzb = 0;
  // apply-precision values (bytes of float or double)
  DArr<char> tA, tP, tR, tdinv;
  // work vectors (apply precision)
  DArr<char> x, r, b, y;
};

struct Amg {
  int bs = 1;
  std::vector<std::unique_ptr<AmgLevel>> lv;
  int nc = 0;                // coarsest size (dense)
  DArr<double> cinv64;
  DArr<char> tcinv;
};

struct MgrLevel {
  Csr A;                     // level matrix A_l (FP64)
  DArr<int8_t> labels;
  CfSplit cf;
  bool f_prefix = false;     // F = 0..nF-1
  bool needs_A = true;       // the V-cycle reads A_l
  DArr<double> dFF;
  Csr Acf, Wp, Acor, G;      // Acor / G only with keep_setup
  Csr AF, AC;                // rows F and rows C of A_l (residuals of uncompacted levels)
  int nb_gs = 0;             // global smoother block size
  bool gsb_pending = false;  // gsb still to be built from A
  DArr<double> binv64;
  BsrB gsb;                  // A_l as cell blocks for the block-Jacobi sweeps (FP64 values)
  DArr<char> tgsb;           // their values in the apply precision
  BsrB cfb;                  // A_CF as cell x F-group blocks for the compacted residual
  DArr<char> tcfb;           // (when its blocks are mostly full), values as tgsb
  bool cfb_pending = false;
  std::vector<int> gs_ptr;   // block Gauss-Seidel: cells of colour c are gs_cells[ptr[c]..)
  DArr<int> gs_cells, gs_color;
  Amg amg;                   // F-relaxation AMG
  DArr<double> ffinv64;      // dense F-relaxation inverse
  Csr Wr;                    // W_r = -A_CF D_FF^{-1} (Jacobi restriction)
  int dffb = 1;              // D_FF block size
  DArr<double> dffinv64;     // block D_FF: inverses of the F-row blocks
  Csr iluS;                  // ILU smoother: factors on the ILU(k) pattern (keep_setup)
  Csr iluL, iluU;            // strictly lower / upper parts of the factors
  DArr<double> ilu_dinv64;   // 1 / u_ii
  int nF = 0;
  // apply-precision copies
  DArr<char> tA, tAcf, tWp, tdinvF, tbinv, tffinv, tAF, tAC, tiluL, tiluU, tilu_dinv, tWr,
      tdffinv;
  // work vectors
  DArr<char> v, z, rF, eF, rfull, ilu_w;
};

template <class T> struct Ptr {
  static T *of(const DArr<char> &d) { return reinterpret_cast<T *>(d.p); }
};

}  // namespace mgr

struct mgr_handle {
  mgr_opts opts;
  hipStream_t s = nullptr;
  int64_t n = 0;
  std::vector<std::unique_ptr<mgr::MgrLevel>> lv;
  mgr::Csr coarseA;
  mgr::DArr<int8_t> coarse_labels;
  mgr::Amg coarse_amg;
  mgr::DArr<double> cdense64;
  mgr::DArr<char> tcdense;
  int ncd = 0;
  mgr::DArr<int> dflag;
  mgr::DArr<int8_t> labels0;
  uint64_t pattern = 0;
  mgr::DArr<char> v0, z0;    // apply-precision level-0 vectors
  hipStream_t cap = nullptr; // private capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t used_ev = nullptr; // recorded after every apply, on the caller's stream
  bool valid = true;            // false after a failed mgr_setup_numeric
  ~mgr_handle();
};

namespace mgr {
namespace {
thread_local std::string t_err;
}
void set_last_error(const std::string &msg) { t_err = msg; }
namespace {

size_t esz(const mgr_opts &o) { return o.precision == MGR_PREC_FP32 ? 4 : 8; }

void cast_values(const double *src, DArr<char> &dst, int64_t n, size_t sz, hipStream_t s) {
  dst.alloc(std::max<int64_t>(n, 1) * sz, s);
  if (n <= 0) return;
  if (sz == 4) cast_to(src, reinterpret_cast<float *>(dst.p), n, s);
  else cast_to(src, reinterpret_cast<double *>(dst.p), n, s);
}

__global__ void k_planes(const double *__restrict__ blk, int64_t nnzb, float *f, double *d) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnzb) return;
  for (int k = 0; k < 9; ++k) {
    const double x = blk[9 * e + k];
    if (f) f[k * nnzb + e] = (float)x;
    else d[k * nnzb + e] = x;
  }
}
void to_planes(const DArr<double> &blk, int64_t nnzb, DArr<char> &dst, size_t sz, hipStream_t s) {
  dst.alloc(std::max<int64_t>(nnzb, 1) * 9 * sz, s);
  if (nnzb <= 0) return;
  k_planes<<<grid_for(nnzb, 256), 256, 0, s>>>(
      blk.p, nnzb, sz == 4 ? reinterpret_cast<float *>(dst.p) : nullptr,
      sz == 8 ? reinterpret_cast<double *>(dst.p) : nullptr);
  KCHK();
}

mgr_amg_opts amg_defaults(mgr_amg_opts o) {
  if (!(o.theta0 > 0)) o.theta0 = 0.08;
  if (o.max_levels <= 0) o.max_levels = 10;
  if (o.coarse_size <= 0) o.coarse_size = 256;
  return o;
}

// AMG hierarchy on A (moved in); bs = 1 or 3
void amg_setup(Csr &&A, int bs, mgr_amg_opts o, Amg &H, const mgr_opts &mo, hipStream_t s,
               int *dflag) {
  o = amg_defaults(o);
  require(o.coarse_size <= 4096, MGR_ERR_ARG, "coarse_size above 4096");
  H.bs = bs;
  H.lv.clear();
  auto L0 = std::make_unique<AmgLevel>();
  L0->A = std::move(A);
  H.lv.push_back(std::move(L0));
  for (int k = 0;; ++k) {
    AmgLevel &L = *H.lv.back();
    const int64_t n = L.A.n;
    if (n <= o.coarse_size || k + 1 >= o.max_levels) break;
    trace("amg level " + std::to_string(k) + " n=" + std::to_string(n) + " nnz=" +
          std::to_string(L.A.nnz) + " bs=" + std::to_string(bs));
    AmgGraph G;
    if (bs == 3 && !L.Ab64) {
      // the block form serves the strength graph and the products of this level
      L.Ab64 = std::make_unique<Bsr3>();
      csr_to_bsr3(L.A, *L.Ab64, s, dflag, "AMG A");
    }
    strength_graph(L.A, bs, o.theta0 * std::ldexp(1.0, -k), G, s, dflag, L.Ab64.get());
    trace("  strength done");
    int64_t nagg = 0;
    DArr<int> agg;
    mis2_aggregate(G, k, agg, nagg, s);
    const int64_t nc = nagg * bs;
    trace("  aggregates " + std::to_string(nagg) + ", strong edges " + std::to_string(G.ci.n));
    if (nc == 0 || (double)nc > 0.8 * (double)n) break;
    Csr T;
    tentative(agg, n / bs, bs, nagg, T, s);
    DArr<double> d(n, s), w(n, s);
    L.dinv.alloc(n, s);
    const double rho = row_stats(L.A, d.p, L.dinv.p, s, dflag);
    const double omega = (4.0 / 3.0) / rho;
    omega_over_diag(d.p, omega, w.p, n, s);
    Csr AT;
    trace("  T, rho done");
    auto N = std::make_unique<AmgLevel>();
    if (bs == 3) {
      // the products on 3x3 blocks (same values as the scalar products, bit for bit)
      if (!L.Ab64) {
        L.Ab64 = std::make_unique<Bsr3>();
        csr_to_bsr3(L.A, *L.Ab64, s, dflag, "AMG A");
      }
      Bsr3 Tb, ATb;
      tentative_b3(agg, n / 3, nagg, Tb, s);
      spgemm_b3(*L.Ab64, Tb, true, ATb, s, dflag);
      bsr3_to_csr(ATb, AT, s);
      trace("  AT done");
      merge_drop(T, AT, w.p, -1, nullptr, L.P, true, s, dflag);
      L.Pb64 = std::make_unique<Bsr3>();
      csr_to_bsr3(L.P, *L.Pb64, s, dflag, "AMG P");
      L.Rb64 = std::make_unique<Bsr3>();
      bsr3_transpose(*L.Pb64, *L.Rb64, s);
      trace("  P, R done");
      Bsr3 APb;
      spgemm_b3(*L.Ab64, *L.Pb64, false, APb, s, dflag);
      trace("  AP done");
      N->Ab64 = std::make_unique<Bsr3>();
      spgemm_b3(*L.Rb64, APb, false, *N->Ab64, s, dflag);
      bsr3_to_csr(*N->Ab64, N->A, s);
      trace("  RAP done");
    } else {
      spgemm(L.A, T, AT, s, dflag);
      trace("  AT done");
      merge_drop(T, AT, w.p, -1, nullptr, L.P, true, s, dflag);
      transpose(L.P, L.R, true, s);
      trace("  P, R done");
      Csr AP;
      spgemm(L.A, L.P, AP, s, dflag);
      trace("  AP done");
      spgemm(L.R, AP, N->A, s, dflag);
      trace("  RAP done");
    }
    L.agg = std::move(agg);
    L.nagg = nagg;
    L.omega = omega;
    H.lv.push_back(std::move(N));
  }
  // coarsest: dense inverse
  trace("  levels done");
  AmgLevel &C = *H.lv.back();
  require(C.A.n <= 4096, MGR_ERR_UNSUPPORTED,
          "AMG coarsest level above 4096 unknowns (coarsening stalled)");
  H.nc = (int)C.A.n;
  DArr<double> D((size_t)H.nc * H.nc, s);
  H.cinv64.alloc((size_t)H.nc * H.nc, s);
  csr_to_dense(C.A, D.p, s);
  dense_inverse(D.p, H.cinv64.p, H.nc, dflag, s);
  // apply copies
  const size_t sz = esz(mo);
  for (size_t k = 0; k + 1 < H.lv.size(); ++k) {
    AmgLevel &L = *H.lv[k];
    cast_values(L.dinv.p, L.tdinv, L.A.n, sz, s);
    if (bs == 3) {
      // block forms from the setup products; the block index arrays move to the V-cycle
      if (!L.Ab64) {
        L.Ab64 = std::make_unique<Bsr3>();
        csr_to_bsr3(L.A, *L.Ab64, s, dflag, "AMG A");
      }
      L.nb = L.Ab64->nb;
      L.ncb = L.Ab64->mb;
      L.Ab_nnzb = L.Ab64->nnzb;
      L.Pb_nnzb = L.Pb64->nnzb;
      L.Rb_nnzb = L.Rb64->nnzb;
      to_planes(L.Ab64->v, L.Ab_nnzb, L.tA, sz, s);
      to_planes(L.Pb64->v, L.Pb_nnzb, L.tP, sz, s);
      to_planes(L.Rb64->v, L.Rb_nnzb, L.tR, sz, s);
      L.Ab_rp = std::move(L.Ab64->rp);
      L.Ab_ci = std::move(L.Ab64->ci);
      L.Pb_rp = std::move(L.Pb64->rp);
      L.Pb_ci = std::move(L.Pb64->ci);
      L.Rb_rp = std::move(L.Rb64->rp);
      L.Rb_ci = std::move(L.Rb64->ci);
      L.Ab64.reset();
      L.Pb64.reset();
      L.Rb64.reset();
    } else {
      make_rowblocks(L.A, s);
      make_rowblocks(L.P, s);
      make_rowblocks(L.R, s);
      cast_values(L.A.v.p, L.tA, L.A.nnz, sz, s);
      cast_values(L.P.v.p, L.tP, L.P.nnz, sz, s);
      cast_values(L.R.v.p, L.tR, L.R.nnz, sz, s);
    }
    L.x.alloc(L.A.n * sz, s);
    L.r.alloc(L.A.n * sz, s);
    L.y.alloc(L.A.n * sz, s);
    L.b.alloc(L.A.n * sz, s);
  }
  {
    AmgLevel &Lc = *H.lv.back();
    Lc.Ab64.reset();      // the coarsest level is solved densely
    Lc.y.alloc(std::max<int64_t>(Lc.A.n, 1) * sz, s);
    Lc.b.alloc(std::max<int64_t>(Lc.A.n, 1) * sz, s);
  }
  cast_values(H.cinv64.p, H.tcinv, (int64_t)H.nc * H.nc, sz, s);
  trace("  apply copies done");
  // buffers released below may have been allocated on another stream (the level matrix)
  HIPCHK(hipStreamSynchronize(s));
  if (!mo.keep_setup) {
    // the V-cycle only needs the apply copies (scalar levels still share the CSR pattern)
    for (size_t k = 0; k < H.lv.size(); ++k) {
      AmgLevel &L = *H.lv[k];
      L.A.v.reset();
      L.P.v.reset();
      L.R.v.reset();
      L.dinv.reset();
      if (bs == 3 || k + 1 == H.lv.size()) {
        L.A.rp.reset(); L.A.ci.reset();
        L.P.rp.reset(); L.P.ci.reset();
        L.R.rp.reset(); L.R.ci.reset();
      }
    }
    H.cinv64.reset();
  }
}

// ------------------------------------------------------------------------------------
template <class T>
CsrV<T> view(const Csr &M, const DArr<char> &tv) {
  CsrV<T> v;
  v.n = M.n; v.m = M.m; v.nnz = M.nnz;
  v.rp = M.rp.p; v.ci = M.ci.p;
  v.v = reinterpret_cast<const T *>(tv.p);
  v.rb = M.nblk ? M.rb.p : nullptr;
  v.nblk = M.nblk;
  return v;
}
template <class T>
CsrV<T> view64(const Csr &M) {
  CsrV<T> v;
  v.n = M.n; v.m = M.m; v.nnz = M.nnz;
  v.rp = M.rp.p; v.ci = M.ci.p;
  v.v = reinterpret_cast<const T *>(M.v.p);
  v.rb = M.nblk ? M.rb.p : nullptr;
  v.nblk = M.nblk;
  return v;
}
template <class T>
Bsr3V<T> bview(int64_t n, int64_t m, int64_t nnzb, const DArr<int> &rp, const DArr<int> &ci,
               const DArr<char> &tv) {
  Bsr3V<T> v;
  v.n = n; v.m = m; v.nnzb = nnzb;
  v.rp = rp.p; v.ci = ci.p;
  v.v = reinterpret_cast<const T *>(tv.p);
  return v;
}

// V-cycle from x = 0: y = V(b); y must not alias b.  `xready`: the level's first smoothing
// iterate x = D^{-1} b was formed by the restriction that produced b.
template <class T>
void vcycle(const Amg &H, size_t k, const T *b, T *y, hipStream_t s, bool xready = false) {
  using V = VecOps<T>;
  if (k + 1 == H.lv.size()) {
    V::gemv(Ptr<T>::of(H.tcinv), H.nc, b, y, s);
    return;
  }
  const AmgLevel &L = *H.lv[k];
  const AmgLevel &N = *H.lv[k + 1];
  T *x = Ptr<T>::of(L.x), *r = Ptr<T>::of(L.r);
  T *bc = Ptr<T>::of(N.b), *yc = Ptr<T>::of(N.y);
  const T *dinv = Ptr<T>::of(L.tdinv);
  if (H.bs == 3) {
    auto A = bview<T>(L.nb, L.nb, L.Ab_nnzb, L.Ab_rp, L.Ab_ci, L.tA);
    auto P = bview<T>(L.nb, L.ncb, L.Pb_nnzb, L.Pb_rp, L.Pb_ci, L.tP);
    auto R = bview<T>(N.A.n / 3, L.nb, L.Rb_nnzb, L.Rb_rp, L.Rb_ci, L.tR);
    const double sweep_bytes =
        (double)L.Ab_nnzb * (9 * sizeof(T) + 4) + (double)(L.nb + 1) * 4 + (double)L.A.n * sizeof(T) * 4;
    const bool prof = k == 0 && Prof::on(0);
    if (prof) Prof::begin(0, s);
    if (xready) V::b_l1_pre_given(A, b, x, r, s);
    else V::b_l1_pre(A, dinv, b, x, r, s);
    if (prof) Prof::end(0, s, sweep_bytes + (double)L.A.n * sizeof(T));
    const bool next_smooths = k + 2 < H.lv.size();   // the next level is not the coarsest
    if (next_smooths)
      V::b_spmv_dx(R, r, Ptr<T>::of(N.tdinv), bc, Ptr<T>::of(N.x), s);
    else
      V::b_spmv(R, r, bc, false, s);
    vcycle<T>(H, k + 1, bc, yc, s, next_smooths);
    V::b_spmv(P, yc, x, true, s);
    if (prof) Prof::begin(0, s);
    V::b_l1_post(A, dinv, b, x, y, s);
    if (prof) Prof::end(0, s, sweep_bytes + (double)L.A.n * sizeof(T));
  } else {
    auto A = view<T>(L.A, L.tA);
    auto P = view<T>(L.P, L.tP);
    auto R = view<T>(L.R, L.tR);
    if (xready) V::l1_pre_given(A, b, x, r, s);
    else V::l1_pre(A, dinv, b, x, r, s);
    const bool next_smooths = k + 2 < H.lv.size();   // the next level is not the coarsest
    if (next_smooths)
      V::spmv_dx(R, r, Ptr<T>::of(N.tdinv), bc, Ptr<T>::of(N.x), s);
    else
      V::spmv(R, r, bc, false, s);
    vcycle<T>(H, k + 1, bc, yc, s, next_smooths);
    V::spmv(P, yc, x, true, s);
    V::l1_post(A, dinv, b, x, y, s);
  }
}

}  // namespace

// Algorithm 2 at level l: z = M_l^{-1} v
template <class T>
void apply_level(mgr_handle *h, size_t l, const T *v, T *z, hipStream_t s) {
  using V = VecOps<T>;
  if (l == h->lv.size()) {
    if (h->opts.coarse == MGR_COARSE_DENSE) V::gemv(Ptr<T>::of(h->tcdense), h->ncd, v, z, s);
    else vcycle<T>(h->coarse_amg, 0, v, z, s);
    return;
  }
  MgrLevel &L = *h->lv[l];
  const mgr_level_opts &o = h->opts.level[l];
  MgrLevel *N = (l + 1 < h->lv.size()) ? h->lv[l + 1].get() : nullptr;
  const int64_t n = L.A.n, nF = L.cf.nF, nC = L.cf.nC;
  const bool fp64 = sizeof(T) == 8;
  CsrV<T> A = fp64 ? view64<T>(L.A) : view<T>(L.A, L.tA);
  CsrV<T> Acf = fp64 ? view64<T>(L.Acf) : view<T>(L.Acf, L.tAcf);
  CsrV<T> Wp = fp64 ? view64<T>(L.Wp) : view<T>(L.Wp, L.tWp);
  CsrV<T> AF = fp64 ? view64<T>(L.AF) : view<T>(L.AF, L.tAF);
  CsrV<T> AC = fp64 ? view64<T>(L.AC) : view<T>(L.AC, L.tAC);
  const bool sub = L.AF.n == nF && L.AC.n == nC && (nF + nC) > 0 && L.AF.rp.p && L.AC.rp.p;
  T *rF = Ptr<T>::of(L.rF), *eF = Ptr<T>::of(L.eF);
  // the next level's input/output vectors (the coarsest grid uses this level's buffer)
  T *rC = N ? Ptr<T>::of(N->v) : Ptr<T>::of(L.rfull);
  T *eC = N ? Ptr<T>::of(N->z) : Ptr<T>::of(L.rfull) + nC;
  bool zero_z = true;
  // global relaxation (block Jacobi over same-cell blocks)
  if (o.global_smoother == MGR_GSMOOTH_BLOCK_JACOBI) {
    // z = D_B^{-1} v, then z <- z + omega D_B^{-1} (v - A z) on the cell blocks of A_l, one
    // kernel per sweep, alternating between z and a work vector so that the last lands in z
    const T *binv = Ptr<T>::of(L.tbinv);
    const int extra = o.global_sweeps - 1;
    T *tmp = Ptr<T>::of(L.rfull) + 2 * nC;
    T *cur = (extra % 2 == 0) ? z : tmp;
    V::block_jacobi(n / L.nb_gs, L.nb_gs, binv, v, (T)1, cur, false, s);
    if (extra > 0) {
      BsrBV<T> G;
      G.nbr = L.gsb.nbr;
      G.nblk = L.gsb.nblk;
      G.nwin = L.gsb.nwin;
      G.br = G.bc = L.gsb.br;
      G.rp = L.gsb.rp.p;
      G.ci = L.gsb.ci.p;
      G.rb = L.gsb.rb.p;
      G.v = fp64 ? reinterpret_cast<const T *>(L.gsb.v.p) : Ptr<T>::of(L.tgsb);
      for (int sw = 0; sw < extra; ++sw) {
        T *nxt = (cur == z) ? tmp : z;
        V::bsr_gs_sweep(G, cur, v, binv, (T)o.global_omega, nxt, s);
        cur = nxt;
      }
    }
    zero_z = false;
  } else if (o.global_smoother == MGR_GSMOOTH_ILU) {
    const T *binv = Ptr<T>::of(L.tbinv);
    CsrV<T> Lo = fp64 ? view64<T>(L.iluL) : view<T>(L.iluL, L.tiluL);
    CsrV<T> Up = fp64 ? view64<T>(L.iluU) : view<T>(L.iluU, L.tiluU);
    const T *dU = fp64 ? reinterpret_cast<const T *>(L.ilu_dinv64.p) : Ptr<T>::of(L.tilu_dinv);
    T *w = Ptr<T>::of(L.ilu_w);
    T *c = w, *ya = w + n, *yb = w + 2 * n, *za = w + 3 * n, *zb = w + 4 * n;
    const int t = o.ilu_tri_sweeps;
    // out = (LU)^{-1} D_B^{-1} r with t Jacobi sweeps per triangular factor; out may be r
    auto smooth = [&](const T *r, T *out) {
      V::block_jacobi(n / L.nb_gs, L.nb_gs, binv, r, (T)1, c, false, s);
      const T *y = c;
      for (int k = 0; k < t; ++k) {
        T *dst = (k & 1) ? yb : ya;
        V::resid(Lo, n, nullptr, nullptr, y, c, dst, s);
        y = dst;
      }
      if (t == 0) {
        V::vmul(dU, y, out, n, s);
        return;
      }
      V::vmul(dU, y, za, n, s);
      const T *zp = za;
      for (int k = 0; k < t; ++k) {
        T *dst = k + 1 == t ? out : ((k & 1) ? za : zb);
        V::resid_scale(Up, dU, zp, y, dst, s);
        zp = dst;
      }
    };
    smooth(v, z);
    for (int sw = 1; sw < o.global_sweeps; ++sw) {
      T *r = Ptr<T>::of(L.rfull) + 2 * nC;
      V::resid(A, n, nullptr, nullptr, z, v, r, s);
      smooth(r, r);
      axpy<T>(n, (T)o.global_omega, r, z, s);
    }
    zero_z = false;
  } else if (o.global_smoother == MGR_GSMOOTH_BLOCK_GS) {
    const T *binv = Ptr<T>::of(L.tbinv);
    V::fill(z, (T)0, n, s);
    for (int sw = 0; sw < o.global_sweeps; ++sw)
      for (size_t c = 0; c + 1 < L.gs_ptr.size(); ++c)
        bgs_color_sweep<T>(A, L.nb_gs, L.gs_cells.p + L.gs_ptr[c], L.gs_ptr[c + 1] - L.gs_ptr[c],
                           binv, v, z, s);
    zero_z = false;
  }
  bool compactF = false;  // z_F held in eF, z otherwise untouched (z_C = 0)
  const T *dinvF = Ptr<T>::of(L.tdinvF);
  if (o.frelax == MGR_FRELAX_JACOBI && L.dffb > 1) {
    // block D_FF: z_F += omega D_FF^{-1} (v - A z)_F with the F-row blocks' inverses
    const T *dfi = Ptr<T>::of(L.tdffinv);
    for (int sw = 0; sw < o.frelax_sweeps; ++sw) {
      if (zero_z) {
        V::fill(z, (T)0, n, s);
        V::gather(L.cf.F.p, nF, v, rF, s);
        zero_z = false;
      } else if (sub) {
        V::resid(AF, nF, nullptr, L.cf.F.p, z, v, rF, s);
      } else {
        V::resid(A, nF, L.cf.F.p, L.cf.F.p, z, v, rF, s);
      }
      V::block_jacobi(nF / L.dffb, L.dffb, dfi, rF, (T)1, eF, false, s);
      scatter_axpy<T>(L.cf.F.p, nF, (T)o.frelax_omega, eF, z, s);
    }
  } else if (o.frelax == MGR_FRELAX_JACOBI) {
    int sw0 = 0;
    if (zero_z) {
      V::jacobi_first(n, L.cf.map.p, dinvF, (T)o.frelax_omega, v, z, s);
      sw0 = 1;
      zero_z = false;
    }
    for (int sw = sw0; sw < o.frelax_sweeps; ++sw) {
      if (sub) V::resid(AF, nF, nullptr, L.cf.F.p, z, v, rF, s);
      else V::resid(A, nF, L.cf.F.p, L.cf.F.p, z, v, rF, s);
      V::jacobi_update(L.cf.F.p, nF, dinvF, (T)o.frelax_omega, rF, z, s);
    }
  } else {
    const T *rin;
    if (zero_z) {
      if (L.f_prefix) rin = v;
      else { V::gather(L.cf.F.p, nF, v, rF, s); rin = rF; }
    } else {
      if (sub) V::resid(AF, nF, nullptr, L.cf.F.p, z, v, rF, s);
      else V::resid(A, nF, L.cf.F.p, L.cf.F.p, z, v, rF, s);
      rin = rF;
    }
    if (o.frelax == MGR_FRELAX_AMG) vcycle<T>(L.amg, 0, rin, eF, s);
    else V::gemv(Ptr<T>::of(L.tffinv), L.nF, rin, eF, s);
    if (zero_z) compactF = true;
    else V::scatter_add(L.cf.F.p, nF, eF, z, s);
  }
  if (o.restrict_ == MGR_RESTRICT_JACOBI) {
    // restrict by R~ = [W_r I]: r_C + W_r r_F of the full residual
    if (compactF) {
      V::fill(z, (T)0, n, s);
      V::scatter_add(L.cf.F.p, nF, eF, z, s);
      compactF = false;
    }
    CsrV<T> Wr = fp64 ? view64<T>(L.Wr) : view<T>(L.Wr, L.tWr);
    if (sub) {
      V::resid(AF, nF, nullptr, L.cf.F.p, z, v, rF, s);
      V::resid(AC, nC, nullptr, L.cf.C.p, z, v, rC, s);
    } else {
      V::resid(A, nF, L.cf.F.p, L.cf.F.p, z, v, rF, s);
      V::resid(A, nC, L.cf.C.p, L.cf.C.p, z, v, rC, s);
    }
    V::spmv(Wr, rF, rC, true, s);
  }
  // restrict the residual by injection
  else if (compactF && L.cfb.nbr > 0) {
    BsrBV<T> B;
    B.nbr = L.cfb.nbr;
    B.nblk = L.cfb.nblk;
    B.nwin = L.cfb.nwin;
    B.br = L.cfb.br;
    B.bc = L.cfb.bc;
    B.rp = L.cfb.rp.p;
    B.ci = L.cfb.ci.p;
    B.rb = L.cfb.rb.p;
    B.v = fp64 ? reinterpret_cast<const T *>(L.cfb.v.p) : Ptr<T>::of(L.tcfb);
    V::bsr_resid(B, eF, v, L.cf.C.p, rC, s);
  }
  else if (compactF) V::resid(Acf, nC, nullptr, L.cf.C.p, eF, v, rC, s);
  else if (sub) V::resid(AC, nC, nullptr, L.cf.C.p, z, v, rC, s);
  else V::resid(A, nC, L.cf.C.p, L.cf.C.p, z, v, rC, s);
  apply_level<T>(h, l + 1, rC, eC, s);
  // interpolate and correct
  V::interp_fc(n, L.cf.map.p, L.cf.F.p, nF, L.cf.C.p, nC, Wp, eC, compactF ? eF : nullptr, z,
               !compactF, s);
}

namespace {

// z = M^{-1} v; with input_ready the caller has already written v, in T, to h->v0
template <class T>
void apply_typed(mgr_handle *h, const double *v, double *z, hipStream_t s,
                 bool input_ready = false) {
  T *v0 = Ptr<T>::of(h->v0), *z0 = Ptr<T>::of(h->z0);
  if (!input_ready) cast_to(v, v0, h->n, s);
  const bool prof = Prof::on(0);
  if (h->opts.use_graph && !prof) {
    if (!h->gexec) {
      if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
      std::lock_guard<std::mutex> cg(g_capture_mu);
      HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
      try {
        apply_level<T>(h, 0, v0, z0, h->cap);
      } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(h->cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(h->cap, &h->graph));
      HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(h->gexec, s));
  } else {
    apply_level<T>(h, 0, v0, z0, s);
  }
  cast_from(z0, z, h->n, s);
  // the last stream that read the hierarchy: destroy and refresh wait for it
  if (!h->used_ev) HIPCHK(hipEventCreateWithFlags(&h->used_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(h->used_ev, s));
}

void wait_uses(mgr_handle *h) {
  if (h->s) HIPCHK(hipStreamSynchronize(h->s));
  if (h->used_ev) HIPCHK(hipEventSynchronize(h->used_ev));
}

void destroy_graph(mgr_handle *h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
}

// the hierarchy is built into the job (not into the level, which an exception on the
// building thread may destroy first) and moved into the level after the join
struct AsyncAmg {
  std::thread th;
  std::exception_ptr err;
  Amg amg;
  MgrLevel *level = nullptr;
};
// joins every setup thread on scope exit (also when the building thread throws)
struct Jobs {
  std::vector<std::unique_ptr<AsyncAmg>> v;
  void join() {
    for (auto &j : v)
      if (j->th.joinable()) j->th.join();
  }
  void rethrow() {
    for (auto &j : v)
      if (j->err) std::rethrow_exception(j->err);
  }
  ~Jobs() { join(); }
};

// Streams for the F-relaxation AMG setups built concurrently with the coarser levels, kept
// in a pool per device and reused by later setups: the caching allocator keeps freed blocks
// per stream, so blocks obtained on a pooled stream are found again by the next setup.
// Pooled streams live until the process ends.
std::mutex g_helper_mu;
std::map<int, std::vector<hipStream_t>> g_helper_pool;

struct HelperStream {
  hipStream_t s = nullptr;
  int dev = 0;
  void acquire() {
    HIPCHK(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> g(g_helper_mu);
      auto &v = g_helper_pool[dev];
      if (!v.empty()) {
        s = v.back();
        v.pop_back();
        return;
      }
    }
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  }
  ~HelperStream() {
    if (!s) return;
    (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> g(g_helper_mu);
    g_helper_pool[dev].push_back(s);
  }
};

// The cell-block copies of the levels (the block-Jacobi sweeps' level matrices, A_CF of a
// compacted level), read only by the apply.  A_CF's blocks are kept when at least 70 % of
// their entries are entries of A_CF (FP32 blocks take 4 br bc + 4 bytes against 8 per CSR
// entry).
void convert_cell_blocks(const std::vector<MgrLevel *> &lv, size_t sz, hipStream_t s) {
  for (MgrLevel *L : lv)
    if (L->gsb_pending) {
      const int nb = L->nb_gs;
      csr_to_bsr_fill(L->A, nb, nb, L->gsb, s);
      if (sz == 4) cast_values(L->gsb.v.p, L->tgsb, L->gsb.nblk * nb * nb, sz, s);
      L->gsb_pending = false;
    }
  for (MgrLevel *L : lv)
    if (L->cfb_pending) {
      const int br = L->cfb.br, bc = L->cfb.bc;
      csr_to_bsr_fill(L->Acf, br, bc, L->cfb, s);
      const double slots = (double)L->cfb.nblk * br * bc;
      if (slots > 0 && (double)L->Acf.nnz >= 0.7 * slots) {
        if (sz == 4) cast_values(L->cfb.v.p, L->tcfb, L->cfb.nblk * br * bc, sz, s);
      } else {
        L->cfb = BsrB();
      }
      L->cfb_pending = false;
    }
}

void build(mgr_handle *h, const mgr_csr *Ain, const int8_t *labels_in) {
  hipStream_t s = h->s;
  std::vector<hipEvent_t> events;
  struct EventGuard {
    std::vector<hipEvent_t> &e;
    ~EventGuard() { for (auto x : e) (void)hipEventDestroy(x); }
  } event_guard{events};
  HelperStream helper;       // the stream of the concurrent F-relaxation AMG setups
  HelperStream conv;         // the stream of the cell-block copies (built with the coarse grid)
  Jobs jobs;                 // declared last: joined before the events and the stream go
  int *flag = h->dflag.p;
  const mgr_opts &o = h->opts;
  const size_t sz = esz(o);
  Csr cur;
  // The caller's column and value arrays are read in place when nothing reads A after the
  // setup (which ends with a synchronisation): level 0 keeps A only for the ILU and block
  // Gauss-Seidel smoothers or with keep_setup, and without MGR levels the AMG owns it.
  const bool borrow_A = o.nlevels > 0 && !o.keep_setup &&
                        o.level[0].global_smoother != MGR_GSMOOTH_ILU &&
                        o.level[0].global_smoother != MGR_GSMOOTH_BLOCK_GS;
  import_csr(Ain, cur, s, flag, borrow_A);
  require(cur.n == cur.m, MGR_ERR_ARG, "A must be square");
  h->n = cur.n;
  h->pattern = pattern_hash(cur, s);
  DArr<int8_t> lab(std::max<int64_t>(cur.n, 1), s);
  if (cur.n) HIPCHK(hipMemcpyAsync(lab.p, labels_in, cur.n, hipMemcpyDeviceToDevice, s));
  for (int l = 0; l < o.nlevels; ++l) {
    const mgr_level_opts &lo = o.level[l];
    trace("mgr level " + std::to_string(l) + " n=" + std::to_string(cur.n) + " nnz=" +
          std::to_string(cur.nnz));
    auto L = std::make_unique<MgrLevel>();
    L->A = std::move(cur);
    L->labels = std::move(lab);
    const int64_t n = L->A.n;
    const uint32_t present = label_mask(L->labels.p, n, s);
    cf_split(L->labels.p, n, lo.f_label_mask, L->cf, s, flag);
    L->nF = (int)L->cf.nF;
    {
      int last = -1;
      d2h_sync(&last, L->cf.F.p + L->cf.nF - 1, sizeof(int), s);
      L->f_prefix = last == L->cf.nF - 1;
    }
    const int64_t nC = L->cf.nC;
    DArr<int8_t> labC(nC, s);
    gather_labels(L->labels.p, L->cf.C.p, nC, labC.p, s);
    DArr<int> lrankC;
    const bool dropping = lo.nmax_drop >= 0 || lo.drop_tol >= 0.0;
    if (dropping) label_rank(labC.p, nC, lrankC, s, present & ~lo.f_label_mask);
    const bool jac_r = lo.restrict_ == MGR_RESTRICT_JACOBI;
    const bool need_ff = lo.frelax != MGR_FRELAX_JACOBI || jac_r || lo.dff_block > 1;
    Csr Aff, Afc, Acc;
    L->dFF.alloc(L->cf.nF, s);
    extract_blocks(L->A, L->cf, need_ff ? &Aff : nullptr, Afc, L->Acf, Acc, L->dFF.p, s);
    check_nonzero(L->dFF.p, L->cf.nF, flag, s);
    check_flags(flag, s, "D_FF");
    // block D_FF: closed-form inverses of the diagonal blocks of dff_block consecutive F rows
    L->dffb = lo.dff_block;
    if (lo.dff_block > 1) {
      require(L->cf.nF % lo.dff_block == 0, MGR_ERR_ARG, "F rows not in blocks of dff_block");
      L->dffinv64.alloc(L->cf.nF * lo.dff_block, s);
      block_diag_inverse(Aff, lo.dff_block, L->dffinv64.p, s, flag);
    }
    // A_FF for the Jacobi restriction's triple product (the F-relaxation AMG takes Aff)
    Csr AffR;
    if (jac_r) copy_csr(Aff, AffR, s);
    // F-relaxation AMG: A_FF is ready
    if (lo.frelax == MGR_FRELAX_AMG) {
      require(lo.frelax_block == 1 || lo.frelax_block == 3, MGR_ERR_ARG, "frelax_block must be 1 or 3");
      // built on a second stream by a second host thread while this thread goes on with the
      // coarser levels (both are bound by sparse products and host synchronisation)
      if (!helper.s) helper.acquire();
      hipEvent_t ev;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIPCHK(hipEventRecord(ev, s));
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      auto job = std::make_unique<AsyncAmg>();
      AsyncAmg *J = job.get();
      J->level = L.get();
      const int bs = lo.frelax_block;
      hipStream_t s2 = helper.s;
      job->th = std::thread([J, bs, dev, ev, s2, o, A = std::move(Aff)]() mutable {
        try {
          HIPCHK(hipSetDevice(dev));
          t_trace_tag = "F";
          HIPCHK(hipStreamWaitEvent(s2, ev, 0));
          DArr<int> f2(1, s2);
          clear_flag(f2.p, s2);
          amg_setup(std::move(A), bs, o.amg_frelax, J->amg, o, s2, f2.p);
          HIPCHK(hipStreamSynchronize(s2));
        } catch (...) {
          J->err = std::current_exception();
        }
      });
      jobs.v.push_back(std::move(job));
      events.push_back(ev);
    }
    // W_p = -D_FF^{-1} A_FC (eq. injective_rp); M = -W_p
    Csr M;
    if (lo.interp == MGR_INTERP_JACOBI && lo.dff_block > 1) {
      block_scale(Afc, lo.dff_block, L->dffinv64.p, M, s, flag);   // block D_FF^{-1} A_FC
    } else if (lo.interp == MGR_INTERP_JACOBI) {
      M = jac_r ? Csr() : std::move(Afc);
      if (jac_r) copy_csr(Afc, M, s);
      scale_rows_div(M, L->dFF.p, s);
    } else {
      M.n = L->cf.nF;
      M.m = nC;
      M.nnz = 0;
      M.rp.alloc(M.n + 1, s);
      fill<int>(M.rp.p, 0, M.n + 1, s);
    }
    trace("  split/extract done");
    // the C-F block of the coarse product: all of A_CF, or its same-entity entries
    Csr AcfQ;
    if (lo.coupling == MGR_COUPLING_QUASI_IMPES) {
      DArr<int> rankL;
      label_rank(L->labels.p, n, rankL, s, present);
      same_entity_filter(L->Acf, L->cf.C.p, L->cf.F.p, rankL.p, AcfQ, s);
    }
    Csr Acor;
    // the C rows of a cell (one per C label) select the same F columns: the product
    // shares their work when their patterns agree
    spgemm(lo.coupling == MGR_COUPLING_QUASI_IMPES ? AcfQ : L->Acf, M, Acor, s, flag,
           __builtin_popcount(present & ~lo.f_label_mask));
    if (jac_r) {
      // N = A_CF D_FF^{-1}; correction A_CF M + N A_FC - N A_FF M (Jacobi restriction)
      Csr N;
      if (lo.dff_block > 1) {
        // A_CF (block D_FF^{-1}) as the pinned-order product with the block-diagonal matrix
        Csr Bd;
        Bd.n = Bd.m = L->cf.nF;
        Bd.nnz = L->cf.nF * lo.dff_block;
        Bd.rp.alloc(Bd.n + 1, s);
        Bd.ci.alloc(std::max<int64_t>(Bd.nnz, 1), s);
        Bd.v.alloc(std::max<int64_t>(Bd.nnz, 1), s);
        block_diag_pattern(Bd.n, lo.dff_block, Bd.rp.p, Bd.ci.p, s);
        if (Bd.nnz)
          HIPCHK(hipMemcpyAsync(Bd.v.p, L->dffinv64.p, Bd.nnz * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        spgemm(L->Acf, Bd, N, s, flag);
      } else {
        copy_csr(L->Acf, N, s);
        scale_cols_div(N, L->dFF.p, s);
      }
      Csr NAfc, NAff, T3, B1, B2;
      spgemm(N, Afc, NAfc, s, flag);
      DArr<double> minus1(std::max<int64_t>(nC, 1), s);
      fill<double>(minus1.p, -1.0, nC, s);
      merge_drop(Acor, NAfc, minus1.p, -1, nullptr, B1, true, s, flag);   // A_CF M + N A_FC
      spgemm(N, AffR, NAff, s, flag);
      spgemm(NAff, M, T3, s, flag);
      merge_drop(B1, T3, nullptr, -1, nullptr, B2, true, s, flag);       // - N A_FF M
      Acor = std::move(B2);
      negate_f64(N.v.p, N.nnz, s);
      L->Wr = std::move(N);
    }
    trace("  A_cor done");
    Csr S;
    merge_drop(Acc, Acor, nullptr, lo.nmax_drop, lrankC.p, S, true, s, flag, lo.drop_tol);
    trace("  S done");
    if (o.keep_setup) {
      if (dropping) drop_only(Acor, lo.nmax_drop, lrankC.p, L->G, s, flag, lo.drop_tol);
      else copy_csr(Acor, L->G, s);
      L->Acor = std::move(Acor);
    }
    negate_f64(M.v.p, M.nnz, s);
    L->Wp = std::move(M);
    // F-relaxation solvers (the AMG one is already under way)
    if (lo.frelax == MGR_FRELAX_DENSE) {
      require(L->cf.nF <= 4096, MGR_ERR_UNSUPPORTED, "dense F-relaxation limited to 4096 rows");
      DArr<double> D(L->cf.nF * L->cf.nF, s);
      L->ffinv64.alloc(L->cf.nF * L->cf.nF, s);
      csr_to_dense(Aff, D.p, s);
      dense_inverse(D.p, L->ffinv64.p, (int)L->cf.nF, flag, s);
      cast_values(L->ffinv64.p, L->tffinv, L->cf.nF * L->cf.nF, sz, s);
    }
    // global smoother
    if (lo.global_smoother != MGR_GSMOOTH_NONE) {
      // rows interleaved cell by cell: labels periodic with the present labels distinct
      const int nb = __builtin_popcount(present);
      const bool ok = nb >= 2 && nb <= 3 && n % nb == 0 && labels_periodic(L->labels.p, n, nb, s) &&
                      (label_mask(L->labels.p, nb, s) == present);
      require(ok, MGR_ERR_UNSUPPORTED,
              "block-Jacobi smoother needs rows interleaved cell by cell (2 or 3 unknowns)");
      L->nb_gs = nb;
      L->binv64.alloc(n * nb, s);
      block_diag_inverse(L->A, nb, L->binv64.p, s, flag);
      cast_values(L->binv64.p, L->tbinv, n * nb, sz, s);
      // cell blocks for the fused sweeps: built after the coarser levels (below)
      L->gsb_pending = lo.global_smoother == MGR_GSMOOTH_BLOCK_JACOBI && lo.global_sweeps > 1;
      if (lo.global_smoother == MGR_GSMOOTH_BLOCK_GS)
        bgs_setup(L->A, nb, L->gs_ptr, L->gs_cells, L->gs_color, s, flag);
      if (lo.global_smoother == MGR_GSMOOTH_ILU) {
        Csr As, S;
        block_scale(L->A, nb, L->binv64.p, As, s, flag);
        ilu_pattern_values(As, lo.ilu_level, S, s, flag);
        DArr<int> dpos;
        ilu_factor(S, lo.ilu_sweeps, dpos, s, flag);
        ilu_split(S, dpos, L->iluL, L->iluU, L->ilu_dinv64, s);
        make_rowblocks(L->iluL, s);
        make_rowblocks(L->iluU, s);
        if (sz == 4) {
          cast_values(L->iluL.v.p, L->tiluL, L->iluL.nnz, sz, s);
          cast_values(L->iluU.v.p, L->tiluU, L->iluU.nnz, sz, s);
          cast_values(L->ilu_dinv64.p, L->tilu_dinv, n, sz, s);
        }
        L->ilu_w.alloc(std::max<int64_t>(5 * n, 1) * sz, s);
        if (o.keep_setup) L->iluS = std::move(S);
        trace("  ILU(" + std::to_string(lo.ilu_level) + ") smoother: " +
              std::to_string(L->iluL.nnz + L->iluU.nnz + n) + " factor entries");
      }
    }
    // apply copies and work vectors
    DArr<double> dinvF(L->cf.nF, s);
    omega_over_diag(L->dFF.p, 1.0, dinvF.p, L->cf.nF, s);  // 1 / d_F
    cast_values(dinvF.p, L->tdinvF, L->cf.nF, sz, s);
    // the level matrix itself is read by the V-cycle unless the F-relaxation is a solve that
    // starts from z = 0 (then the residual uses A_CF only)
    // the V-cycle reads A_l itself only in the ILU and block Gauss-Seidel smoothers: the
    // block-Jacobi sweeps read its cell blocks, and every residual of the F-relaxation and
    // the restriction reads the F rows and C rows gathered below (AF, AC) or A_CF
    const bool needs_A = lo.global_smoother == MGR_GSMOOTH_ILU ||
                         lo.global_smoother == MGR_GSMOOTH_BLOCK_GS;
    L->needs_A = needs_A;
    // rows F and rows C of A_l for the residuals of levels that are not compacted
    const bool need_sub = lo.frelax == MGR_FRELAX_JACOBI || lo.global_smoother != MGR_GSMOOTH_NONE ||
                          jac_r;
    if (need_sub) {
      gather_rows(L->A, L->cf.F.p, L->cf.nF, L->AF, s);
      gather_rows(L->A, L->cf.C.p, nC, L->AC, s);
      make_rowblocks(L->AF, s);
      make_rowblocks(L->AC, s);
    }
    if (needs_A) make_rowblocks(L->A, s);
    make_rowblocks(L->Acf, s);
    make_rowblocks(L->Wp, s);
    {
      // the compacted residual r_C = v_C - A_CF e_F runs when the F-relaxation starts from
      // z = 0 and the restriction is injection; cells of br C rows, groups of bc F columns
      const bool compact = lo.global_smoother == MGR_GSMOOTH_NONE &&
                           (lo.frelax == MGR_FRELAX_AMG || lo.frelax == MGR_FRELAX_DENSE) && !jac_r;
      const int br = __builtin_popcount(present & ~lo.f_label_mask);
      // F columns in groups: the nodal triples of a 3x3-block F-relaxation, else one of
      // each F label
      const int bc = lo.frelax_block > 1 ? lo.frelax_block
                                         : __builtin_popcount(present & lo.f_label_mask);
      const int shape = br * 10 + bc;
      L->cfb_pending = compact && (shape == 22 || shape == 33 || shape == 23) && nC % br == 0 &&
                       L->cf.nF % bc == 0 && L->Acf.nnz > 0;
      L->cfb.br = br;
      L->cfb.bc = bc;
    }
    if (jac_r) make_rowblocks(L->Wr, s);
    if (lo.dff_block > 1) cast_values(L->dffinv64.p, L->tdffinv, L->cf.nF * lo.dff_block, sz, s);
    if (sz == 4) {
      if (needs_A) cast_values(L->A.v.p, L->tA, L->A.nnz, sz, s);
      cast_values(L->Acf.v.p, L->tAcf, L->Acf.nnz, sz, s);
      cast_values(L->Wp.v.p, L->tWp, L->Wp.nnz, sz, s);
      if (jac_r) cast_values(L->Wr.v.p, L->tWr, L->Wr.nnz, sz, s);
      if (need_sub) {
        cast_values(L->AF.v.p, L->tAF, L->AF.nnz, sz, s);
        cast_values(L->AC.v.p, L->tAC, L->AC.nnz, sz, s);
      }
    }
    L->rF.alloc(std::max<int64_t>(L->cf.nF, 1) * sz, s);
    L->eF.alloc(std::max<int64_t>(L->cf.nF, 1) * sz, s);
    L->v.alloc(std::max<int64_t>(n, 1) * sz, s);
    L->z.alloc(std::max<int64_t>(n, 1) * sz, s);
    L->rfull.alloc(std::max<int64_t>(2 * nC + n, 1) * sz, s);
    cur = std::move(S);
    lab = std::move(labC);
    h->lv.push_back(std::move(L));
  }
  // The cell-block copies are built by a thread of their own on a pooled stream while this
  // thread sets up the coarse grid: the levels are complete, and the coarse-grid AMG (small
  // kernels and read-backs) leaves most of the GPU free.
  {
    bool any = false;
    for (auto &L : h->lv) any = any || L->gsb_pending || L->cfb_pending;
    if (any) {
      conv.acquire();
      hipEvent_t ev;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      events.push_back(ev);
      HIPCHK(hipEventRecord(ev, s));
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      std::vector<MgrLevel *> lvs;
      for (auto &L : h->lv) lvs.push_back(L.get());
      auto job = std::make_unique<AsyncAmg>();   // no hierarchy: `level` stays null
      AsyncAmg *J = job.get();
      hipStream_t s3 = conv.s;
      job->th = std::thread([J, lvs, sz, dev, ev, s3]() {
        try {
          HIPCHK(hipSetDevice(dev));
          t_trace_tag = "B";
          HIPCHK(hipStreamWaitEvent(s3, ev, 0));
          convert_cell_blocks(lvs, sz, s3);
          HIPCHK(hipStreamSynchronize(s3));
        } catch (...) {
          J->err = std::current_exception();
        }
      });
      jobs.v.push_back(std::move(job));
    }
  }
  // coarsest grid
  trace("mgr levels done");
  const int64_t nc = cur.n;
  if (o.coarse == MGR_COARSE_DENSE) {
    require(nc <= 4096, MGR_ERR_UNSUPPORTED, "dense coarse solve limited to 4096 unknowns");
    h->ncd = (int)nc;
    DArr<double> D(nc * nc, s);
    h->cdense64.alloc(nc * nc, s);
    csr_to_dense(cur, D.p, s);
    dense_inverse(D.p, h->cdense64.p, (int)nc, flag, s);
    cast_values(h->cdense64.p, h->tcdense, nc * nc, sz, s);
    if (o.keep_setup) h->coarseA = std::move(cur);
  } else {
    Csr keep;
    if (o.keep_setup) copy_csr(cur, keep, s);
    amg_setup(std::move(cur), 1, o.amg_coarse, h->coarse_amg, o, s, flag);
    if (o.keep_setup) h->coarseA = std::move(keep);
  }
  h->coarse_labels = std::move(lab);
  jobs.join();
  jobs.rethrow();
  for (auto &j : jobs.v)
    if (j->level) j->level->amg = std::move(j->amg);
  trace("  F-relaxation AMG joined");
  h->v0.alloc(std::max<int64_t>(h->n, 1) * sz, s);
  h->z0.alloc(std::max<int64_t>(h->n, 1) * sz, s);
  // level 0 input / output are the handle vectors; release what apply does not need
  if (!o.keep_setup) {
    for (auto &L : h->lv) {
      if (!L->needs_A) {
        L->A.rp.reset();
        L->A.ci.reset();
        L->A.v.reset();
      }
      if (sz == 4) {
        L->A.v.reset();
        L->Acf.v.reset();
        L->Wp.v.reset();
        L->AF.v.reset();
        L->AC.v.reset();
        L->binv64.reset();
        L->gsb.v.reset();
        L->cfb.v.reset();
        L->ffinv64.reset();
        L->iluL.v.reset();
        L->iluU.v.reset();
        L->ilu_dinv64.reset();
        L->Wr.v.reset();
        L->dffinv64.reset();
      }
      L->dFF.reset();
      if (L->cfb.nbr > 0) {   // the compacted residual reads the cell blocks only
        L->Acf.rp.reset();
        L->Acf.ci.reset();
        L->Acf.v.reset();
        L->tAcf.reset();
      }
    }
    if (sz == 4) h->cdense64.reset();
  }
  HIPCHK(hipStreamSynchronize(s));
  check_flags(flag, s, "setup");
  {
    long misses;
    double us;
    {
      std::lock_guard<std::mutex> g(g_cache_mu);
      misses = g_misses;
      us = g_miss_us;
    }
    trace("setup done (allocator: " + std::to_string(misses) + " hipMalloc calls so far, " +
          std::to_string(us / 1000.0) + " ms)");
  }
}

void validate_opts(const mgr_opts &o) {
  require(o.nlevels >= 0 && o.nlevels <= MGR_MAX_LEVELS, MGR_ERR_ARG, "nlevels out of range");
  require(o.precision == MGR_PREC_FP64 || o.precision == MGR_PREC_FP32, MGR_ERR_ARG, "precision");
  require(o.coarse == MGR_COARSE_AMG || o.coarse == MGR_COARSE_DENSE, MGR_ERR_ARG, "coarse");
  for (int l = 0; l < o.nlevels; ++l) {
    const mgr_level_opts &lo = o.level[l];
    require(lo.f_label_mask != 0 && (lo.f_label_mask >> 8) == 0, MGR_ERR_ARG, "f_label_mask");
    require(lo.interp == MGR_INTERP_JACOBI || lo.interp == MGR_INTERP_ZERO, MGR_ERR_ARG, "interp");
    require(lo.frelax >= 0 && lo.frelax <= 2, MGR_ERR_ARG, "frelax");
    require(lo.frelax_sweeps >= 1 && lo.frelax_sweeps <= 100, MGR_ERR_ARG, "frelax_sweeps");
    require(lo.global_smoother >= 0 && lo.global_smoother <= 3, MGR_ERR_ARG, "global_smoother");
    require(lo.ilu_level == 0 || lo.ilu_level == 1, MGR_ERR_ARG, "ilu_level must be 0 or 1");
    require(lo.ilu_sweeps >= 0 && lo.ilu_sweeps <= 100, MGR_ERR_ARG, "ilu_sweeps");
    require(lo.ilu_tri_sweeps >= 0 && lo.ilu_tri_sweeps <= 100, MGR_ERR_ARG, "ilu_tri_sweeps");
    require(lo.restrict_ == MGR_RESTRICT_INJECTION || lo.restrict_ == MGR_RESTRICT_JACOBI,
            MGR_ERR_ARG, "restrict_");
    require(lo.restrict_ == MGR_RESTRICT_INJECTION ||
                (lo.coupling == MGR_COUPLING_FULL && lo.interp == MGR_INTERP_JACOBI),
            MGR_ERR_ARG, "Jacobi restriction needs full coupling and Jacobi interpolation");
    require(lo.dff_block >= 1 && lo.dff_block <= 3, MGR_ERR_ARG, "dff_block must be 1, 2 or 3");
    require(lo.reserved1 == 0, MGR_ERR_ARG, "reserved1 must be 0");
    require(lo.global_sweeps >= 1 && lo.global_sweeps <= 100, MGR_ERR_ARG, "global_sweeps");
    require(lo.coupling == MGR_COUPLING_FULL || lo.coupling == MGR_COUPLING_QUASI_IMPES, MGR_ERR_ARG,
            "coupling");
    require(!(lo.drop_tol >= 0.0 && lo.nmax_drop >= 0), MGR_ERR_ARG,
            "drop_tol and nmax_drop select two forms of G: set one");
    require(!(lo.drop_tol != lo.drop_tol), MGR_ERR_ARG, "drop_tol is NaN");
  }
}

size_t handle_bytes(const mgr_handle *h) {
  size_t b = 0;
  auto csr = [&](const Csr &M) { b += M.bytes(); };
  auto amg = [&](const Amg &H) {
    for (auto &L : H.lv) {
      csr(L->A); csr(L->P); csr(L->R);
      b += L->agg.bytes() + L->dinv.bytes() + L->Ab_rp.bytes() + L->Ab_ci.bytes() +
           L->Pb_rp.bytes() + L->Pb_ci.bytes() + L->Rb_rp.bytes() + L->Rb_ci.bytes() +
           L->tA.bytes() + L->tP.bytes() + L->tR.bytes() + L->tdinv.bytes() + L->x.bytes() +
           L->r.bytes() + L->b.bytes() + L->y.bytes();
    }
    b += H.cinv64.bytes() + H.tcinv.bytes();
  };
  for (auto &L : h->lv) {
    csr(L->A); csr(L->Acf); csr(L->Wp); csr(L->Acor); csr(L->G); csr(L->AF); csr(L->AC);
    b += L->labels.bytes() + L->cf.F.bytes() + L->cf.C.bytes() + L->cf.map.bytes() +
         L->dFF.bytes() + L->binv64.bytes() + L->gs_cells.bytes() + L->gs_color.bytes() +
         L->gsb.bytes() + L->tgsb.bytes() + L->cfb.bytes() + L->tcfb.bytes() +
         L->ffinv64.bytes() + L->tA.bytes() +
         L->tAcf.bytes() + L->tWp.bytes() + L->tdinvF.bytes() + L->tbinv.bytes() +
         L->tAF.bytes() + L->tAC.bytes() +
         L->tffinv.bytes() + L->v.bytes() + L->z.bytes() + L->rF.bytes() + L->eF.bytes() +
         L->rfull.bytes() + L->Wr.bytes() + L->dffinv64.bytes() + L->tWr.bytes() +
         L->tdffinv.bytes() + L->iluS.bytes() + L->iluL.bytes() + L->iluU.bytes() +
         L->ilu_dinv64.bytes() + L->tiluL.bytes() + L->tiluU.bytes() + L->tilu_dinv.bytes() +
         L->ilu_w.bytes();
    amg(L->amg);
  }
  csr(h->coarseA);
  amg(h->coarse_amg);
  b += h->cdense64.bytes() + h->tcdense.bytes() + h->v0.bytes() + h->z0.bytes() +
       h->coarse_labels.bytes() + h->labels0.bytes();
  return b;
}

mgr_status fail(const Error &e) {
  t_err = e.what();
  return e.st;
}

}  // namespace
}  // namespace mgr

mgr_handle::~mgr_handle() {
  if (s) (void)hipStreamSynchronize(s);
  if (used_ev) {
    (void)hipEventSynchronize(used_ev);
    (void)hipEventDestroy(used_ev);
  }
  mgr::destroy_graph(this);
  if (cap) (void)hipStreamDestroy(cap);
  // the hierarchy's buffers return to the allocator (every stream they were taken on is
  // synchronised: the caller's above, the pooled setup streams at the end of the setup)
  lv.clear();
  coarse_amg.lv.clear();
}

// ===================================================================================
// FGMRES
namespace mgr {
namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct FgWork {
  double *V, *Z, *w, *r, *partial, *H, *cs, *sn, *g, *h1, *h2, *hn2, *scal, *y, *red;
  int *rb;  // SpMV row blocks
};

size_t fg_layout(int64_t n, int m, char *base, FgWork *w) {
  size_t off = 0;
  auto take = [&](double **p, size_t count) {
    if (w) *p = reinterpret_cast<double *>(base + off);
    off += align256(count * sizeof(double));
  };
  FgWork tmp;
  FgWork *W = w ? w : &tmp;
  take(&W->V, (size_t)(m + 1) * n);
  take(&W->Z, (size_t)m * n);
  take(&W->w, n);
  take(&W->r, n);
  take(&W->partial, (size_t)krylov_partials_blocks());
  take(&W->H, (size_t)(m + 1) * m);
  take(&W->cs, m + 1);
  take(&W->sn, m + 1);
  take(&W->g, m + 2);
  take(&W->h1, 80);
  take(&W->h2, 80);
  take(&W->hn2, 8);
  take(&W->scal, 8);
  take(&W->y, m + 1);
  take(&W->red, 8);
  // row blocks: at most n + 2 entries (one block per 2048 entries, never more than rows)
  if (w) W->rb = reinterpret_cast<int *>(base + off);
  off += align256((size_t)(n + 2) * sizeof(int));
  return off;
}

// `hostv`: pinned or pageable host memory for the read-back
double host_norm(const double *r, int64_t n, FgWork &W, double *hostv, hipStream_t s) {
  const int nb = norm2_partials(r, n, W.partial, s);
  reduce_partials(W.partial, nb, 1, W.red, false, s);
  HIPCHK(hipMemcpyAsync(hostv, W.red, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return std::sqrt(*hostv);
}

// `noalloc`: the caller's workspace is used and nothing is allocated or created: the
// read-backs land in pageable memory on the host stack and the host waits on the stream
// instead of on events (the launches, their order and the results are those of the
// pipelined default path).
mgr_status fgmres_impl(const mgr_csr *A, mgr_handle *M, const double *b, double *x,
                       const fgmres_opts *o, void *work, size_t work_bytes, fgmres_result *res,
                       hipStream_t s, bool noalloc = false) {
  require(A && b && x && o, MGR_ERR_ARG, "null argument");
  require(A->block >= 0 && A->block <= 3 && A->reserved == 0, MGR_ERR_ARG,
          "matrix block size must be 0..3 and reserved 0");
  const int bs = A->block > 1 ? A->block : 1;
  const int64_t n = scalar_rows(*A);
  const int m = o->restart;
  require(m >= 1 && m <= 64, MGR_ERR_ARG, "restart must be in [1, 64]");
  require(o->maxit >= 1, MGR_ERR_ARG, "maxit must be positive");
  require(!M || M->n == n, MGR_ERR_ARG, "preconditioner size differs from A");
  require(!M || M->valid, MGR_ERR_ARG,
          "the preconditioner holds no setup: its last mgr_setup_numeric failed");
  if (noalloc && M)
    require(M->used_ev && (M->gexec || !M->opts.use_graph), MGR_ERR_ARG,
            "the preconditioner has not been applied yet (its first application captures "
            "its graph and creates its event): call mgr_apply or fgmres_solve with it once");
  const size_t need = fg_layout(n, m, nullptr, nullptr);
  DArr<char> own;
  char *base = static_cast<char *>(work);
  require(base || !noalloc, MGR_ERR_ARG, "no workspace");
  if (!base) {
    own.alloc(need, s);
    base = own.p;
  } else {
    require(work_bytes >= need, MGR_ERR_ARG, "fgmres workspace too small");
  }
  FgWork W;
  fg_layout(n, m, base, &W);
  // entries (blocks when bs > 1)
  int64_t nnz = 0;
  if (n) {
    HIPCHK(hipMemcpyAsync(&nnz, A->row_ptr + A->nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  // row blocks fit the workspace unless rows average more than 2048 entries; such CSR
  // matrices use the lanes-per-row kernel (BSR windows always fit: one per >= 227 values)
  const int64_t K = bs > 1 ? bsr_stream_blocks(nnz, bs) : stream_blocks(nnz);
  const bool streamed = K + 1 <= n + 2;
  require(bs == 1 || streamed, MGR_ERR_UNSUPPORTED, "BSR block rows longer than supported");
  if (streamed) {
    if (bs > 1) bsr_rowblocks64(*A, nnz, W.rb, s);
    else rowblocks64(*A, nnz, W.rb, s);
  }
  const double avg = n ? (double)nnz / (double)n : 0.0;
  // algorithmic bytes: values and column indices, row pointers, x and y once
  const double spmv_bytes =
      bs > 1 ? (double)nnz * (8.0 * bs * bs + 4.0) + (double)A->nrows * 8.0 + (double)n * 16.0
             : (double)nnz * 12.0 + (double)n * (8.0 + 8.0 + 8.0);
  auto matvec = [&](const double *xx, const double *bb, double *yy) {
    const bool prof = Prof::on(1);
    if (prof) Prof::begin(1, s);
    if (bs > 1) bsr_spmv64_stream(*A, nnz, W.rb, xx, bb, yy, s);
    else if (streamed) spmv64_stream(*A, nnz, W.rb, xx, bb, yy, s);
    else spmv64_avg(*A, xx, bb, yy, avg, s);
    if (prof) Prof::end(1, s, spmv_bytes + (bb ? (double)n * 8.0 : 0.0));
  };
  double host_buf[32];
  double *hb = noalloc ? host_buf : static_cast<double *>(pinned_scratch());
  const double bnorm = host_norm(b, n, W, hb, s);
  // a zero initial guess makes the first residual b itself (b - A 0 = b exactly), so the
  // first cycle starts without a product with A
  bool x_zero = host_norm(x, n, W, hb, s) == 0.0;
  fgmres_result R{};
  if (res) { R.history = res->history; R.history_cap = res->history_cap; }
  auto push = [&](double v) {
    if (R.history && R.history_len < R.history_cap) R.history[R.history_len++] = v;
  };
  if (bnorm == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    R.converged = 1;
    if (res) *res = R;
    return MGR_OK;
  }
  const double tol = o->rtol * bnorm;
  const int ldh = m + 1;
  int its = 0;
  bool first = true;
  // per-step residual estimates land in two pinned slots, each with its completion event
  double *slot[2] = {hb + 8, hb + 16};
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{ev};
  if (!noalloc)
    for (int i = 0; i < 2; ++i) HIPCHK(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  for (;;) {
    double beta = bnorm;
    if (x_zero) {
      HIPCHK(hipMemcpyAsync(W.r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      x_zero = false;
    } else {
      matvec(x, b, W.r);  // r = b - A x
      beta = host_norm(W.r, n, W, hb, s);
    }
    R.true_relres = beta / bnorm;
    push(beta / bnorm);
    if (beta <= tol) { R.converged = 1; break; }
    if (its >= o->maxit || !std::isfinite(beta)) break;
    if (!first) ++R.restarts;
    first = false;
    start_cycle_host_beta(W.r, beta, W.V, W.g, n, m + 1, s);
    // Arnoldi steps are software-pipelined by one: step j+1 (whose basis vector comes from
    // step j's device-side scalars) is enqueued before the host waits for step j's
    // residual estimate, so the GPU never idles on the host's convergence check.  When
    // step j ends the cycle, step j+1 has only written column j+1 of H, g[j+1..j+2] and
    // Z[j+1], none of which the update with k = j+1 reads.
    // step j of the cycle; `ready`: v_j was also written into the preconditioner's input
    auto step = [&](int j, bool ready) {
      double *vj = W.V + (int64_t)j * n;
      double *zj = W.Z + (int64_t)j * n;
      if (M) {
        if (M->opts.precision == MGR_PREC_FP32) apply_typed<float>(M, vj, zj, s, ready);
        else apply_typed<double>(M, vj, zj, s, ready);
      } else {
        HIPCHK(hipMemcpyAsync(zj, vj, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      matvec(zj, nullptr, W.w);
      // classical Gram-Schmidt, twice
      int nb = multidot_partials(W.V, n, j + 1, W.w, W.partial, s);
      reduce_partials(W.partial, nb, j + 1, W.h1, false, s);
      nb = cgs_update_partials(W.V, n, j + 1, W.h1, W.w, W.partial, false, s);
      reduce_partials(W.partial, nb, j + 1, W.h2, false, s);
      nb = cgs_update_partials(W.V, n, j + 1, W.h2, W.w, W.partial, true, s);
      reduce_partials(W.partial, nb, 1, W.hn2, false, s);
      givens_step(W.H, W.cs, W.sn, W.g, W.h1, W.h2, W.hn2, j, ldh, W.scal, nullptr, s);
      HIPCHK(hipMemcpyAsync(slot[j & 1], W.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
      if (!noalloc) HIPCHK(hipEventRecord(ev[j & 1], s));
    };
    int k = 0;
    step(0, false);
    for (int j = 0; j < m; ++j) {
      const bool ahead = j + 1 < m && its + 1 < o->maxit;
      if (ahead) {
        double *vn = W.V + (int64_t)(j + 1) * n;
        if (!M) scale_vec(W.w, W.scal + 2, vn, n, s);
        else if (M->opts.precision == MGR_PREC_FP32)
          scale_vec_copy(W.w, W.scal + 2, vn, Ptr<float>::of(M->v0), n, s);
        else
          scale_vec_copy(W.w, W.scal + 2, vn, Ptr<double>::of(M->v0), n, s);
        step(j + 1, M != nullptr);
      }
      if (noalloc) HIPCHK(hipStreamSynchronize(s));
      else HIPCHK(hipEventSynchronize(ev[j & 1]));
      ++its;
      const double *sc = slot[j & 1];
      R.est_relres = sc[0] / bnorm;
      push(R.est_relres);
      k = j + 1;
      if (sc[0] <= tol || sc[1] == 0.0 || its >= o->maxit || !std::isfinite(sc[0])) break;
    }
    tri_solve_and_update(W.H, W.g, k, ldh, W.Z, n, x, W.y, s);
  }
  R.iters = its;
  HIPCHK(hipStreamSynchronize(s));
  if (res) {
    double *hist = res->history;
    int cap = res->history_cap;
    *res = R;
    res->history = hist;
    res->history_cap = cap;
  }
  if (!R.converged) {
    t_err = "fgmres: not converged";
    return MGR_ERR_NOT_CONVERGED;
  }
  return MGR_OK;
}
}  // namespace
}  // namespace mgr

// ===================================================================================
// C ABI
using namespace mgr;

extern "C" {

void mgr_default_opts(mgr_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nlevels = 0;
  o->coarse = MGR_COARSE_AMG;
  o->amg_frelax = mgr_amg_opts{0.08, 10, 256};
  o->amg_coarse = mgr_amg_opts{0.08, 10, 256};
  o->precision = MGR_PREC_FP64;
  o->use_graph = 1;
  o->keep_setup = 0;
  for (int l = 0; l < MGR_MAX_LEVELS; ++l) {
    mgr_level_opts &L = o->level[l];
    L.f_label_mask = 0;
    L.interp = MGR_INTERP_JACOBI;
    L.nmax_drop = -1;
    L.frelax = MGR_FRELAX_JACOBI;
    L.frelax_sweeps = 1;
    L.frelax_omega = 1.0;
    L.frelax_block = 1;
    L.global_smoother = MGR_GSMOOTH_NONE;
    L.global_sweeps = 1;
    L.global_omega = 1.0;
    L.coupling = MGR_COUPLING_FULL;
    L.drop_tol = -1.0;
    L.ilu_level = 1;
    L.ilu_sweeps = 3;
    L.ilu_tri_sweeps = 3;
    L.restrict_ = MGR_RESTRICT_INJECTION;
    L.dff_block = 1;
    L.reserved1 = 0;
  }
}

mgr_status mgr_setup(const mgr_csr *A, const int8_t *labels, const mgr_opts *opts, void *stream,
                     mgr_handle **out) {
  t_err.clear();
  if (!A || !labels || !opts || !out) { t_err = "null argument"; return MGR_ERR_ARG; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_ptr<mgr_handle> h(new mgr_handle());
  try {
    validate_opts(*opts);
    require(A->nrows >= 1, MGR_ERR_ARG, "empty matrix");
    require(A->block >= 0 && A->block <= 3 && A->reserved == 0, MGR_ERR_ARG,
            "matrix block size must be 0..3 and reserved 0");
    const int64_t n = scalar_rows(*A);
    h->opts = *opts;
    h->s = s;
    h->dflag.alloc(1, s);
    clear_flag(h->dflag.p, s);
    h->labels0.alloc(n, s);
    HIPCHK(hipMemcpyAsync(h->labels0.p, labels, n, hipMemcpyDeviceToDevice, s));
    build(h.get(), A, labels);
  } catch (const Error &e) {
    (void)hipStreamSynchronize(s);   // nothing in flight reads the caller's arrays
    return fail(e);
  } catch (const std::exception &e) {
    (void)hipStreamSynchronize(s);
    t_err = e.what();
    return MGR_ERR_HIP;
  }
  *out = h.release();
  return MGR_OK;
}

mgr_status mgr_setup_numeric(mgr_handle *h, const mgr_csr *A, void *stream) {
  t_err.clear();
  if (!h || !A) { t_err = "null argument"; return MGR_ERR_ARG; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    require(A->block >= 0 && A->block <= 3 && A->reserved == 0, MGR_ERR_ARG,
            "matrix block size must be 0..3 and reserved 0");
    require(scalar_rows(*A) == h->n, MGR_ERR_PATTERN, "size differs from the original matrix");
    {
      Csr tmp;   // read in place: the hash is read back before the arrays are let go
      import_csr(A, tmp, s, h->dflag.p, A->block <= 1);
      require(pattern_hash(tmp, s) == h->pattern, MGR_ERR_PATTERN,
              "sparsity pattern differs from the original matrix");
    }
    wait_uses(h);
    h->valid = false;
    destroy_graph(h);
    h->lv.clear();
    h->coarseA = Csr();
    h->coarse_amg = Amg();
    h->cdense64.reset();
    h->tcdense.reset();
    h->s = s;
    clear_flag(h->dflag.p, s);
    DArr<int8_t> lab(h->n, s);
    HIPCHK(hipMemcpyAsync(lab.p, h->labels0.p, h->n, hipMemcpyDeviceToDevice, s));
    build(h, A, lab.p);
    HIPCHK(hipStreamSynchronize(s));
    h->valid = true;
  } catch (const Error &e) {
    (void)hipStreamSynchronize(s);   // nothing in flight reads the caller's arrays
    return fail(e);
  } catch (const std::exception &e) {
    (void)hipStreamSynchronize(s);
    t_err = e.what();
    return MGR_ERR_HIP;
  }
  return MGR_OK;
}

mgr_status mgr_apply(mgr_handle *h, const double *v, double *z, void *stream) {
  t_err.clear();
  if (!h || !v || !z) { t_err = "null argument"; return MGR_ERR_ARG; }
  try {
    require(h->valid, MGR_ERR_ARG, "the handle holds no setup: its last mgr_setup_numeric failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->opts.precision == MGR_PREC_FP32) apply_typed<float>(h, v, z, s);
    else apply_typed<double>(h, v, z, s);
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

size_t fgmres_workspace_bytes(int64_t n, int32_t restart) {
  return fg_layout(n, restart, nullptr, nullptr);
}

mgr_status fgmres_solve(const mgr_csr *A, mgr_handle *M, const double *b, double *x,
                        const fgmres_opts *o, void *work, size_t work_bytes, fgmres_result *res,
                        void *stream) {
  t_err.clear();
  try {
    return fgmres_impl(A, M, b, x, o, work, work_bytes, res, static_cast<hipStream_t>(stream));
  } catch (const Error &e) {
    return fail(e);
  }
}

}  // extern "C"

// Workspace of fgmres_solve_noalloc: one array per device, held from the library's load on
// that device until the process ends.  Host code never passes `scratch` itself (in host
// code the name is a host-side stand-in, not a device address): it uses the device address
// that hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

void *scratch_on_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  require(dev >= 0 && dev < kMaxDevices, MGR_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(MGR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

size_t fgmres_noalloc_max_bytes(void) { return kNoAllocBytes; }

mgr_status fgmres_solve_noalloc(const mgr_csr *A, mgr_handle *M, const double *b, double *x,
                                const fgmres_opts *o, fgmres_result *res, void *stream) {
  t_err.clear();
  try {
    require(A && o, MGR_ERR_ARG, "null argument");
    require(o->restart >= 1 && o->restart <= 64, MGR_ERR_ARG, "restart must be in [1, 64]");
    const size_t need = fgmres_workspace_bytes(scalar_rows(*A), o->restart);
    if (need > kNoAllocBytes)
      throw Error(MGR_ERR_ARG, "fgmres_solve_noalloc: the system needs " + std::to_string(need) +
                                   " bytes of workspace; the static workspace holds " +
                                   std::to_string(kNoAllocBytes));
    void *ws = scratch_on_current_device();
    return fgmres_impl(A, M, b, x, o, ws, kNoAllocBytes, res, static_cast<hipStream_t>(stream),
                       true);
  } catch (const Error &e) {
    return fail(e);
  }
}

void mgr_destroy(mgr_handle *h) { delete h; }

mgr_status mgr_footprint(const mgr_handle *h, size_t *bytes) {
  if (!h || !bytes) { t_err = "null argument"; return MGR_ERR_ARG; }
  *bytes = handle_bytes(h);
  return MGR_OK;
}

mgr_status mgr_estimate_footprint(int64_t n, int64_t nnz, const mgr_opts *opts, size_t *bytes) {
  if (!opts || !bytes || n < 0 || nnz < 0) { t_err = "bad argument"; return MGR_ERR_ARG; }
  // peak of setup: the imported copy of A, the level blocks and products, the AMG
  // hierarchies, their sparse-product temporaries and the row-split copies of levels that
  // are not compacted stay below five FP64 CSR copies of A,
  // plus 64 level vectors and the dense coarsest inverses (size-binned by the allocator)
  const double a = (double)nnz * 12.0 + (double)(n + 1) * 4.0;
  const double cs = std::max(opts->amg_frelax.coarse_size, opts->amg_coarse.coarse_size);
  const double dense = (opts->coarse == MGR_COARSE_DENSE ? 4096.0 * 4096.0 : 0.0) + cs * cs;
  double est = 5.0 * a + 64.0 * 8.0 * (double)n + 4.0 * 8.0 * dense + (double)(16 << 20);
  *bytes = (size_t)est;
  return MGR_OK;
}

void mgr_set_allocator(void *(*alloc_fn)(size_t, void *, void *),
                       void (*free_fn)(void *, void *, void *), void *ctx) {
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    std::lock_guard<std::mutex> cg(g_capture_mu);
    (void)hipDeviceSynchronize();
    release_cache_locked();
  }
  g_alloc = alloc_fn;
  g_free = free_fn;
  g_ctx = ctx;
}

const char *mgr_last_error(void) { return t_err.c_str(); }

mgr_status mgr_release_cache(void) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  std::lock_guard<std::mutex> cg(g_capture_mu);
  (void)hipDeviceSynchronize();
  release_cache_locked();
  return MGR_OK;
}

size_t mgr_cached_bytes(void) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  return g_cached_bytes;
}

void mgr_alloc_stats(size_t *live, size_t *peak, int32_t reset_peak) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  if (live) *live = g_live_bytes;
  if (peak) *peak = g_peak_bytes;
  if (reset_peak) g_peak_bytes = g_live_bytes;
}

mgr_status mgr_query(const mgr_handle *h, int32_t what, int32_t level, int32_t sub, int64_t out[3]) {
  t_err.clear();
  if (!h || !out) { t_err = "null argument"; return MGR_ERR_ARG; }
  try {
    const int nl = (int)h->lv.size();
    require(level >= 0 && level <= nl, MGR_ERR_ARG, "level out of range");
    const Amg *amg = nullptr;
    if (what >= MGR_X_AMG_A && what <= MGR_X_AMG_NLEV) {
      amg = level == nl ? &h->coarse_amg : &h->lv[level]->amg;
      require(!amg->lv.empty(), MGR_ERR_ARG, "no AMG hierarchy at this level");
      if (what == MGR_X_AMG_NLEV) { out[0] = (int64_t)amg->lv.size(); out[1] = out[2] = 0; return MGR_OK; }
      require(sub >= 0 && sub < (int)amg->lv.size(), MGR_ERR_ARG, "AMG level out of range");
    } else {
      require(level < nl || what == MGR_X_LEVEL_A, MGR_ERR_ARG, "level out of range");
    }
    auto csr = [&](const Csr &M) {
      require(M.v.p != nullptr || M.nnz == 0, MGR_ERR_ARG, "object not kept (set keep_setup)");
      out[0] = M.n; out[1] = M.m; out[2] = M.nnz;
    };
    switch (what) {
      case MGR_X_LEVEL_A: csr(level == nl ? h->coarseA : h->lv[level]->A); break;
      case MGR_X_F: out[0] = h->lv[level]->cf.nF; out[1] = 0; out[2] = out[0]; break;
      case MGR_X_C: out[0] = h->lv[level]->cf.nC; out[1] = 0; out[2] = out[0]; break;
      case MGR_X_GS_COLOR:
        require(h->lv[level]->gs_color.n > 0, MGR_ERR_ARG, "no block Gauss-Seidel at this level");
        out[0] = (int64_t)h->lv[level]->gs_color.n; out[1] = 0; out[2] = out[0];
        break;
      case MGR_X_WP: csr(h->lv[level]->Wp); break;
      case MGR_X_ACOR: csr(h->lv[level]->Acor); break;
      case MGR_X_G: csr(h->lv[level]->G); break;
      case MGR_X_ILU:
        require(h->lv[level]->iluS.rp.p != nullptr, MGR_ERR_ARG,
                "no ILU smoother kept at this level (set keep_setup)");
        csr(h->lv[level]->iluS);
        break;
      case MGR_X_WR:
        require(h->lv[level]->Wr.rp.p != nullptr, MGR_ERR_ARG,
                "no Jacobi restriction at this level");
        csr(h->lv[level]->Wr);
        break;
      case MGR_X_COARSE: csr(level + 1 == nl ? h->coarseA : h->lv[level + 1]->A); break;
      case MGR_X_AMG_A: csr(amg->lv[sub]->A); break;
      case MGR_X_AMG_P:
        require(sub + 1 < (int)amg->lv.size(), MGR_ERR_ARG, "coarsest AMG level has no P");
        csr(amg->lv[sub]->P);
        break;
      case MGR_X_AMG_AGG:
        require(sub + 1 < (int)amg->lv.size(), MGR_ERR_ARG, "coarsest AMG level has no aggregates");
        out[0] = amg->lv[sub]->A.n / amg->bs; out[1] = amg->lv[sub]->nagg; out[2] = out[0];
        break;
      default: throw Error(MGR_ERR_ARG, "unknown object");
    }
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

mgr_status mgr_export(const mgr_handle *h, int32_t what, int32_t level, int32_t sub,
                      int64_t *row_ptr, int32_t *col, double *val, void *stream) {
  int64_t sz[3];
  mgr_status st = mgr_query(h, what, level, sub, sz);
  if (st != MGR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    const int nl = (int)h->lv.size();
    auto ints = [&](const int *src, int64_t n) {
      if (col && n) HIPCHK(hipMemcpyAsync(col, src, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    };
    auto csr = [&](const Csr &M) {
      if (row_ptr) rowptr32_to_64(M.rp.p, row_ptr, M.n + 1, s);
      ints(M.ci.p, M.nnz);
      if (val && M.nnz)
        HIPCHK(hipMemcpyAsync(val, M.v.p, M.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    };
    const Amg *amg = (what >= MGR_X_AMG_A && what <= MGR_X_AMG_NLEV)
                         ? (level == nl ? &h->coarse_amg : &h->lv[level]->amg)
                         : nullptr;
    switch (what) {
      case MGR_X_LEVEL_A: csr(level == nl ? h->coarseA : h->lv[level]->A); break;
      case MGR_X_F: ints(h->lv[level]->cf.F.p, sz[0]); break;
      case MGR_X_C: ints(h->lv[level]->cf.C.p, sz[0]); break;
      case MGR_X_GS_COLOR: ints(h->lv[level]->gs_color.p, sz[0]); break;
      case MGR_X_WP: csr(h->lv[level]->Wp); break;
      case MGR_X_ACOR: csr(h->lv[level]->Acor); break;
      case MGR_X_G: csr(h->lv[level]->G); break;
      case MGR_X_ILU:
        require(h->lv[level]->iluS.rp.p != nullptr, MGR_ERR_ARG,
                "no ILU smoother kept at this level (set keep_setup)");
        csr(h->lv[level]->iluS);
        break;
      case MGR_X_WR:
        require(h->lv[level]->Wr.rp.p != nullptr, MGR_ERR_ARG,
                "no Jacobi restriction at this level");
        csr(h->lv[level]->Wr);
        break;
      case MGR_X_COARSE: csr(level + 1 == nl ? h->coarseA : h->lv[level + 1]->A); break;
      case MGR_X_AMG_A: csr(amg->lv[sub]->A); break;
      case MGR_X_AMG_P: csr(amg->lv[sub]->P); break;
      case MGR_X_AMG_AGG: ints(amg->lv[sub]->agg.p, sz[0]); break;
      default: break;
    }
    HIPCHK(hipStreamSynchronize(s));
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

mgr_status mgr_spmv(const mgr_csr *A, const double *x, double *y, void *stream) {
  t_err.clear();
  if (!A || !x || !y) { t_err = "null argument"; return MGR_ERR_ARG; }
  try {
    spmv64(*A, x, y, static_cast<hipStream_t>(stream));
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

mgr_status mgr_stream_copy(const double *src, double *dst, int64_t n, void *stream) {
  t_err.clear();
  try {
    stream_copy_f64(src, dst, n, static_cast<hipStream_t>(stream));
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

mgr_status mgr_profile_enable(int32_t family, int32_t enable) {
  if (family < 0 || family > 1) { t_err = "family"; return MGR_ERR_ARG; }
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof[family].on = enable != 0;
  g_prof[family].used = 0;
  return MGR_OK;
}

mgr_status mgr_profile_read(int32_t family, int64_t *launches, double *total_ms, double *bytes) {
  if (family < 0 || family > 1) { t_err = "family"; return MGR_ERR_ARG; }
  try {
    ProfFamily &P = g_prof[family];
    double ms = 0.0, by = 0.0;
    for (size_t i = 0; i < P.used; ++i) {
      HIPCHK(hipEventSynchronize(P.ev[i].second));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, P.ev[i].first, P.ev[i].second));
      ms += t;
      by += P.bytes[i];
    }
    if (launches) *launches = (int64_t)P.used;
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
  } catch (const Error &e) {
    return fail(e);
  }
  return MGR_OK;
}

}  // extern "C"

// Smoothed-aggregation AMG setup kernels: strength graph (scalar or 3x3 nodal), SplitMix64
// priorities, synchronous MIS(2) rounds, aggregation passes and the tentative
// prolongator.  Every decision is integer logic on values computed with single IEEE
// operations in a fixed order, so the hierarchy does not depend on thread scheduling.
#include "common.hpp"

namespace mgr {
namespace {

constexpr unsigned long long GOLDEN = 0x9E3779B97F4A7C15ull;
enum : int8_t { UNDECIDED = 0, SELECTED = 1, REMOVED = 2, ISOLATED = 3 };

__device__ __forceinline__ unsigned long long splitmix64_first(unsigned long long seed) {
  unsigned long long z = seed + GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// scalar strength: count pass (MODE 0) and fill pass (MODE 1); G lanes per row take the
// row G entries at a time, and the strong ones of a chunk are placed in column order by
// their rank among the group's ballot bits
template <int G, int MODE>
__global__ void k_strength_scalar(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                                  const double *__restrict__ v, const double *__restrict__ d,
                                  double th2, int *__restrict__ cnt, const int *__restrict__ srp,
                                  int *__restrict__ sci) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  const int gbase = (threadIdx.x & 63) & ~(G - 1);     // first lane of the group in the wave
  if (i >= n) return;
  const double di = d[i];
  int c = 0;
  const int o = MODE ? srp[i] : 0;
  const int e1 = rp[i + 1];
  for (int e0 = rp[i]; e0 < e1; e0 += G) {
    const int e = e0 + l;
    bool strong = false;
    int j = 0;
    if (e < e1) {
      j = ci[e];
      const double a = v[e];
      strong = j != (int)i && a != 0.0 &&
               __dmul_rn(a, a) >= __dmul_rn(th2, fabs(__dmul_rn(di, d[j])));
    }
    const uint64_t wave = __ballot(strong);
    const uint64_t grp = (wave >> gbase) & ((G == 64) ? ~0ull : ((1ull << G) - 1));
    if (MODE && strong) sci[o + c + __popcll(grp & ((1ull << l) - 1))] = j;
    c += __popcll(grp);
  }
  if (!MODE && l == 0) cnt[i] = c;
}

// node blocks of a scalar CSR with full 3x3 blocks: squared Frobenius norm of every block,
// summed row by row, left to right, from +0.0; G lanes per node, one block per lane
template <int G>
__global__ void k_node_norms(int64_t nn, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ v, const int *__restrict__ nrp,
                             int *__restrict__ nci, double *__restrict__ f) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (I >= nn) return;
  const int nb = nrp[I + 1] - nrp[I];
  for (int q = l; q < nb; q += G) {
    double acc = 0.0;
    for (int r = 0; r < 3; ++r) {
      const int s = rp[3 * I + r] + 3 * q;
      for (int c = 0; c < 3; ++c) acc = __dadd_rn(acc, __dmul_rn(v[s + c], v[s + c]));
    }
    if (nci) nci[nrp[I] + q] = ci[rp[3 * I] + 3 * q] / 3;
    f[nrp[I] + q] = acc;
  }
}
// 16 lanes per node row; the lane that holds the diagonal entry hands it to the others
constexpr int NG = 16;
__global__ void k_node_diag(int64_t nn, const int *__restrict__ nrp, const int *__restrict__ nci,
                            const double *__restrict__ f, double *__restrict__ fd) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / NG;
  const int l = threadIdx.x & (NG - 1);
  if (I >= nn) return;
  double x = 0.0;
  int found = 0;
  for (int e = nrp[I] + l; e < nrp[I + 1]; e += NG)
    if (nci[e] == I) {
      x = f[e];
      found = 1;
    }
#pragma unroll
  for (int o = NG / 2; o > 0; o >>= 1) {
    const double ox = __shfl_xor(x, o, NG);
    const int of = __shfl_xor(found, o, NG);
    if (of && !found) {
      x = ox;
      found = 1;
    }
  }
  if (l == 0) fd[I] = x;
}
// 16 lanes per node row, the row taken 16 entries at a time; strong entries are written in
// row order (each lane's place from a ballot of its group)
template <int MODE>
__global__ void k_strength_nodal(int64_t nn, const int *__restrict__ nrp, const int *__restrict__ nci,
                                 const double *__restrict__ f, const double *__restrict__ fd,
                                 double th4, int *__restrict__ cnt, const int *__restrict__ srp,
                                 int *__restrict__ sci) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / NG;
  const int l = threadIdx.x & (NG - 1);
  if (I >= nn) return;
  const double fi = fd[I];
  int c = 0;
  const int o = MODE ? srp[I] : 0;
  const int e0 = nrp[I], e1 = nrp[I + 1];
  for (int c0 = e0; c0 < e1; c0 += NG) {
    const int e = c0 + l;
    bool strong = false;
    int J = 0;
    if (e < e1) {
      J = nci[e];
      if (J != I) {
        const double x = f[e];
        strong = x != 0.0 && __dmul_rn(x, x) >= __dmul_rn(th4, __dmul_rn(fi, fd[J]));
      }
    }
    const uint64_t b = __ballot(strong);
    const int base = (int)(threadIdx.x & 63) & ~(NG - 1);
    const uint32_t gb = (uint32_t)((b >> base) & ((1ull << NG) - 1));
    if (MODE && strong) sci[o + c + __popc(gb & ((1u << l) - 1))] = J;
    c += __popc(gb);
  }
  if (!MODE && l == 0) cnt[I] = c;
}

__global__ void k_prio(int64_t n, unsigned long long salt, unsigned long long *__restrict__ prio,
                       const int *__restrict__ grp, int8_t *__restrict__ state) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  prio[i] = splitmix64_first((unsigned long long)i ^ salt);
  state[i] = (grp[i + 1] == grp[i]) ? ISOLATED : UNDECIDED;
}

// The graph kernels below take G lanes per node (G = 1 for short rows, 16 for the long rows
// of the coarse levels); maxima, ORs and the first best neighbour do not depend on how a
// row is split among lanes.
// out[i] = max(val[i], max over neighbours) where val = prio masked to undecided nodes (MODE 0)
// or a previous max (MODE 1)
template <int MODE, int G>
__global__ void k_rowmax(int64_t n, const int *__restrict__ grp, const int *__restrict__ gci,
                         const unsigned long long *__restrict__ prio,
                         const int8_t *__restrict__ state, const unsigned long long *__restrict__ in,
                         unsigned long long *__restrict__ out) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (i >= n) return;
  auto val = [&](int64_t j) -> unsigned long long {
    if (MODE == 0) return state[j] == UNDECIDED ? prio[j] : 0ull;
    return in[j];
  };
  unsigned long long m = l == 0 ? val(i) : 0ull;
  for (int e = grp[i] + l; e < grp[i + 1]; e += G) {
    unsigned long long x = val(gci[e]);
    m = x > m ? x : m;
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(m, o, G);
    m = x > m ? x : m;
  }
  if (l == 0) out[i] = m;
}
__global__ void k_select(int64_t n, const unsigned long long *__restrict__ prio,
                         const unsigned long long *__restrict__ m2, int8_t *__restrict__ state,
                         int *__restrict__ isnew) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool sel = state[i] == UNDECIDED && prio[i] == m2[i];
  if (sel) state[i] = SELECTED;
  isnew[i] = sel;
}
template <int G>
__global__ void k_rowany(int64_t n, const int *__restrict__ grp, const int *__restrict__ gci,
                         const int *__restrict__ in, int *__restrict__ out) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (i >= n) return;
  int a = l == 0 ? in[i] : 0;
  for (int e = grp[i] + l; e < grp[i + 1] && !a; e += G) a = in[gci[e]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) a |= __shfl_xor(a, o, G);
  if (l == 0) out[i] = a != 0;
}
__global__ void k_remove(int64_t n, const int *__restrict__ near, int8_t *__restrict__ state,
                         int *__restrict__ und) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool left = false;
  if (state[i] == UNDECIDED) {
    if (near[i]) state[i] = REMOVED;
    else left = true;
  }
  // one counter update per wavefront
  const unsigned long long w = __ballot(left);
  if (w && (int)(threadIdx.x & 63) == __ffsll((long long)w) - 1) atomicAdd(und, __popcll(w));
}

__global__ void k_is_state(int64_t n, const int8_t *__restrict__ state, int8_t s,
                           int *__restrict__ fl) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) fl[i] = state[i] == s;
}
__global__ void k_root_ids(int64_t n, const int8_t *__restrict__ state, const int *__restrict__ pos,
                           int *__restrict__ agg) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) agg[i] = state[i] == SELECTED ? pos[i] : -1;
}
// best neighbour by priority among candidates; PASS 1: candidates are roots, PASS 2:
// candidates are nodes aggregated after pass 1 (agg1)
// (the first neighbour in row order among those of the largest priority)
template <int PASS, int G>
__global__ void k_agg_pass(int64_t n, const int *__restrict__ grp, const int *__restrict__ gci,
                           const unsigned long long *__restrict__ prio,
                           const int8_t *__restrict__ state, const int *__restrict__ agg1,
                           int *__restrict__ agg) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (i >= n) return;
  if (state[i] == ISOLATED || agg1[i] >= 0) return;   // uniform over the node's lanes
  int best = -1, be = 0x7fffffff;
  unsigned long long bp = 0;
  for (int e = grp[i] + l; e < grp[i + 1]; e += G) {
    const int j = gci[e];
    const bool cand = (PASS == 1) ? state[j] == SELECTED : agg1[j] >= 0;
    if (cand && (best < 0 || prio[j] > bp)) { best = j; bp = prio[j]; be = e; }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const int ob = __shfl_xor(best, o, G), oe = __shfl_xor(be, o, G);
    const unsigned long long op = __shfl_xor(bp, o, G);
    if (ob >= 0 && (best < 0 || op > bp || (op == bp && oe < be))) {
      best = ob;
      bp = op;
      be = oe;
    }
  }
  if (l == 0 && best >= 0) agg[i] = agg1[best];
}
__global__ void k_leftover_flags(int64_t n, const int8_t *__restrict__ state,
                                 const int *__restrict__ agg, int *__restrict__ fl) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) fl[i] = state[i] != ISOLATED && agg[i] < 0;
}
__global__ void k_leftover_ids(int64_t n, const int *__restrict__ fl, const int *__restrict__ pos,
                               int base, int *__restrict__ agg) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && fl[i]) agg[i] = base + pos[i];
}

__global__ void k_tent_count(int64_t nrows, int bs, const int *__restrict__ agg,
                             int *__restrict__ cnt) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < nrows) cnt[r] = agg[r / bs] >= 0;
}
__global__ void k_tent_fill(int64_t nrows, int bs, const int *__restrict__ agg,
                            const int *__restrict__ rp, int *__restrict__ ci,
                            double *__restrict__ v) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int a = agg[r / bs];
  if (a >= 0) {
    ci[rp[r]] = a * bs + (int)(r % bs);
    v[rp[r]] = 1.0;
  }
}

}  // namespace

void strength_graph(const Csr &A, int bs, double theta, AmgGraph &G, hipStream_t s,
                    int *dflag, const Bsr3 *blocks) {
  Csr S;  // directed strong graph, pattern only
  const double th2 = theta * theta;
  if (bs == 1) {
    const int64_t n = A.n;
    DArr<double> d(n, s);
    diag_of(A, d.p, s);
    DArr<int> cnt(n + 1, s);
    k_strength_scalar<16, 0><<<grid_for(n * 16, 256), 256, 0, s>>>(n, A.rp.p, A.ci.p, A.v.p, d.p,
                                                                   th2, cnt.p, nullptr, nullptr);
    KCHK();
    S.n = S.m = n;
    S.rp.alloc(n + 1, s);
    S.nnz = exclusive_scan_i32(cnt.p, S.rp.p, n, s);
    S.ci.alloc(S.nnz, s);
    k_strength_scalar<16, 1><<<grid_for(n * 16, 256), 256, 0, s>>>(n, A.rp.p, A.ci.p, A.v.p, d.p,
                                                                   th2, nullptr, S.rp.p, S.ci.p);
    KCHK();
  } else {
    require(bs == 3, MGR_ERR_ARG, "AMG block size must be 1 or 3");
    // node pattern: that of the level's 3x3 block form when the caller has it
    DArr<int> own_rp, own_ci;
    int64_t nn, nnzb;
    if (blocks) {
      nn = blocks->nb;
      nnzb = blocks->nnzb;
    } else {
      DArr<double> bv_unused;
      int64_t mn;
      csr_to_bsr3(A, own_rp, own_ci, bv_unused, nn, mn, nnzb, s, dflag, "strength A");
    }
    const int *nrp = blocks ? blocks->rp.p : own_rp.p;
    const int *nci = blocks ? blocks->ci.p : own_ci.p;
    DArr<double> f(nnzb, s), fd(nn, s);
    k_node_norms<16><<<grid_for(nn * 16, 256), 256, 0, s>>>(nn, A.rp.p, A.ci.p, A.v.p, nrp,
                                                            nullptr, f.p);
    KCHK();
    k_node_diag<<<grid_for(nn * NG, 256), 256, 0, s>>>(nn, nrp, nci, f.p, fd.p);
    KCHK();
    const double th4 = th2 * th2;
    DArr<int> cnt(nn + 1, s);
    k_strength_nodal<0><<<grid_for(nn * NG, 256), 256, 0, s>>>(nn, nrp, nci, f.p, fd.p, th4, cnt.p,
                                                         nullptr, nullptr);
    KCHK();
    S.n = S.m = nn;
    S.rp.alloc(nn + 1, s);
    S.nnz = exclusive_scan_i32(cnt.p, S.rp.p, nn, s);
    S.ci.alloc(S.nnz, s);
    k_strength_nodal<1><<<grid_for(nn * NG, 256), 256, 0, s>>>(nn, nrp, nci, f.p, fd.p, th4,
                                                         nullptr, S.rp.p, S.ci.p);
    KCHK();
  }
  // symmetrise by union with the transpose
  Csr St, U;
  transpose(S, St, false, s);
  merge_drop(S, St, nullptr, -1, nullptr, U, false, s, dflag);
  G.n = U.n;
  G.rp = std::move(U.rp);
  G.ci = std::move(U.ci);
}

void mis2_aggregate(const AmgGraph &G, int level, DArr<int> &agg, int64_t &nagg, hipStream_t s) {
  const int64_t n = G.n;
  const unsigned gs = grid_for(n, 256);
  DArr<unsigned long long> prio(n, s), m1(n, s), m2(n, s);
  DArr<int8_t> state(n, s);
  DArr<int> a(n, s), b(n, s), und(1, s);
  const unsigned long long salt = GOLDEN * (unsigned long long)(level + 1);
  k_prio<<<gs, 256, 0, s>>>(n, salt, prio.p, G.rp.p, state.p);
  KCHK();
  // 16 lanes per node for the long rows of the coarse levels' graphs
  const bool wide = n > 0 && (double)G.ci.n > 16.0 * (double)n;
  const unsigned gw = grid_for(n * 16, 256);
  for (int round = 0; round < 100000; ++round) {
    if (wide) {
      k_rowmax<0, 16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, nullptr, m1.p);
      KCHK();
      k_rowmax<1, 16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, m1.p, m2.p);
      KCHK();
    } else {
      k_rowmax<0, 1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, nullptr, m1.p);
      KCHK();
      k_rowmax<1, 1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, m1.p, m2.p);
      KCHK();
    }
    k_select<<<gs, 256, 0, s>>>(n, prio.p, m2.p, state.p, a.p);
    KCHK();
    if (wide) {
      k_rowany<16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, a.p, b.p);
      KCHK();
      k_rowany<16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, b.p, a.p);
      KCHK();
    } else {
      k_rowany<1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, a.p, b.p);
      KCHK();
      k_rowany<1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, b.p, a.p);
      KCHK();
    }
    fill<int>(und.p, 0, 1, s);
    k_remove<<<gs, 256, 0, s>>>(n, a.p, state.p, und.p);
    KCHK();
    // the count is read after every second round: a round with no undecided node left
    // changes nothing, so the rounds run past the last useful one are harmless
    if ((round & 1) && read_flag(und.p, s) == 0) break;
  }
  // roots numbered in node order
  DArr<int> fl(n, s), pos(n + 1, s);
  k_is_state<<<gs, 256, 0, s>>>(n, state.p, SELECTED, fl.p);
  KCHK();
  const int64_t nroots = exclusive_scan_i32(fl.p, pos.p, n, s);
  DArr<int> agg1(n, s);
  k_root_ids<<<gs, 256, 0, s>>>(n, state.p, pos.p, agg1.p);
  KCHK();
  agg.alloc(n, s);
  HIPCHK(hipMemcpyAsync(agg.p, agg1.p, n * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (wide) k_agg_pass<1, 16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, agg1.p, agg.p);
  else k_agg_pass<1, 1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, agg1.p, agg.p);
  KCHK();
  HIPCHK(hipMemcpyAsync(agg1.p, agg.p, n * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (wide) k_agg_pass<2, 16><<<gw, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, agg1.p, agg.p);
  else k_agg_pass<2, 1><<<gs, 256, 0, s>>>(n, G.rp.p, G.ci.p, prio.p, state.p, agg1.p, agg.p);
  KCHK();
  k_leftover_flags<<<gs, 256, 0, s>>>(n, state.p, agg.p, fl.p);
  KCHK();
  const int64_t nleft = exclusive_scan_i32(fl.p, pos.p, n, s);
  if (nleft) {
    k_leftover_ids<<<gs, 256, 0, s>>>(n, fl.p, pos.p, (int)nroots, agg.p);
    KCHK();
  }
  nagg = nroots + nleft;
}

void tentative(const DArr<int> &agg, int64_t nnode, int bs, int64_t nagg, Csr &T, hipStream_t s) {
  const int64_t nr = nnode * bs;
  T.n = nr;
  T.m = nagg * bs;
  DArr<int> cnt(nr + 1, s);
  k_tent_count<<<grid_for(nr, 256), 256, 0, s>>>(nr, bs, agg.p, cnt.p);
  KCHK();
  T.rp.alloc(nr + 1, s);
  T.nnz = exclusive_scan_i32(cnt.p, T.rp.p, nr, s);
  T.ci.alloc(T.nnz, s);
  T.v.alloc(T.nnz, s);
  k_tent_fill<<<grid_for(nr, 256), 256, 0, s>>>(nr, bs, agg.p, T.rp.p, T.ci.p, T.v.p);
  KCHK();
}

}  // namespace mgr

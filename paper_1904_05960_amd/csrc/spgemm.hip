// Sparse matrix product C = A B with a pinned summation order, for the coarse-grid
// correction A_CF (D_FF^{-1} A_FC) of the MGR setup (Sec. 5.2) and the Galerkin products
// A T, A P and R (A P) of the AMG setup.
//
// c_ij is the sum over the entries a_ik of row i taken in ascending k, each product
// a_ik * b_kj rounded on its own and added to an accumulator that starts at +0.0 (no fused
// multiply-add).  The result pattern is symbolic: every (i, j) reached by a product, also
// when the value cancels.  With this order the values (and every decision later taken on
// them: dropping, strength, aggregation) do not depend on thread scheduling.
//
// Symbolic phase: one 64-lane workgroup per row inserts the column of every product into
// an LDS open-addressing table (flat over products, order irrelevant); rows whose distinct
// count would overflow the LDS table are redone with a table in global memory.
// Numeric phase: one workgroup per row walks the row of A in order; for each a_ik the
// lanes take the entries of row k of B (distinct columns, so no two lanes touch the same
// slot), find or insert the column and add the product; a barrier separates consecutive
// k.  The occupied slots are then compacted and placed by rank (columns are unique), which
// writes the row sorted by column.
#include "common.hpp"

namespace mgr {
namespace {

constexpr int SYM_HT = 4096;       // second-pass LDS symbolic table size (int keys)

__device__ __forceinline__ unsigned hslot(int key, unsigned mask) {
  return ((unsigned)key * 2654435761u) & mask;
}

__device__ __forceinline__ int next_pow2_dev(int64_t v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// ub[i] = number of products of row i (sum of the lengths of the rows of B it selects)
__global__ void k_upper_bound(int64_t n, const int *__restrict__ arp, const int *__restrict__ aci,
                              const int *__restrict__ brp, int64_t *__restrict__ ub) {
  constexpr int G = 16;
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (i >= n) return;
  int64_t s = 0;
  for (int e = arp[i] + l; e < arp[i + 1]; e += G) {
    const int k = aci[e];
    s += brp[k + 1] - brp[k];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  if (l == 0) ub[i] = s;
}

// Inserts `key` (>= 0) into the table; returns 1 if it was new, 0 if present, -1 if the
// probe wrapped around a full table.
__device__ __forceinline__ int table_insert(int *keys, unsigned mask, int key) {
  unsigned slot = hslot(key, mask);
  for (unsigned probe = 0; probe <= mask; ++probe) {
    int old = atomicCAS(&keys[slot], -1, key);
    if (old == -1) return 1;
    if (old == key) return 0;
    slot = (slot + 1) & mask;
  }
  return -1;
}

// Returns the slot of `key`, inserting it if absent; mask + 1 (out of range) if the table is
// full, which the sizing rules out (tables hold at least twice the row's distinct count,
// the grouped coarse product's at least four thirds of it).
__device__ __forceinline__ unsigned table_find_or_insert(int *keys, unsigned mask, int key) {
  unsigned slot = hslot(key, mask);
  for (unsigned probe = 0; probe <= mask; ++probe) {
    int cur = keys[slot];
    if (cur == key) return slot;
    if (cur == -1) {
      int old = atomicCAS(&keys[slot], -1, key);
      if (old == -1 || old == key) return slot;
    }
    slot = (slot + 1) & mask;
  }
  return mask + 1;
}

// Orders the table updates of consecutive steps between the lanes of one wave.  A table in
// LDS needs no wait: a wave's LDS operations execute in issue order, so a wavefront-scope
// fence (a compiler barrier) suffices and loads already in flight for later steps stay in
// flight.  A table in global memory takes a workgroup-scope fence.
template <bool LDS_TABLE>
__device__ __forceinline__ void table_step_fence() {
  if (LDS_TABLE) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Symbolic count of one row by a group of G lanes with a table of `ht` slots; returns -1
// if more than 3/4 of the table would be needed.  Products are taken flat (their order does
// not matter here): the entries of the row of A are read G at a time and the lanes walk the
// concatenated rows of B they select.
template <int G>
__device__ __forceinline__ int sym_row(int row, const int *__restrict__ arp, const int *__restrict__ aci,
                       const int *__restrict__ brp, const int *__restrict__ bci, int *keys,
                       int ht, int *s_count, int *s_excl, int *s_start) {
  const int l = threadIdx.x & (G - 1);
  const unsigned mask = (unsigned)ht - 1;
  for (int s = l; s < ht; s += G) keys[s] = -1;
  if (l == 0) *s_count = 0;
  __builtin_amdgcn_wave_barrier();
  const int limit = (ht / 4) * 3;
  const int as = arp[row], ae = arp[row + 1];
  int over = 0;
  for (int c0 = as; c0 < ae; c0 += G) {
    const int e = c0 + l;
    int len = 0, st = 0;
    if (e < ae) {
      const int k = aci[e];
      st = brp[k];
      len = brp[k + 1] - st;
    }
    int inc = len;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int t = __shfl_up(inc, o, G);
      if (l >= o) inc += t;
    }
    s_excl[l] = inc - len;
    s_start[l] = st;
    const int total = __shfl(inc, G - 1, G);
    __builtin_amdgcn_wave_barrier();
    const int nent = min(G, ae - c0);
    constexpr int PU = 4;
    for (int p0 = 0; p0 < total; p0 += PU * G) {
      int jj[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int p = p0 + u * G + l;
        jj[u] = -1;
        if (p < total) {
          int lo = 0, hi = nent - 1;        // entry t with s_excl[t] <= p < s_excl[t+1]
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_excl[mid] <= p) lo = mid; else hi = mid - 1;
          }
          jj[u] = bci[s_start[lo] + (p - s_excl[lo])];
        }
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        if (jj[u] < 0) continue;
        const int r = table_insert(keys, mask, jj[u]);
        if (r == 1) {
          if (atomicAdd(s_count, 1) >= limit) over = 1;
        } else if (r < 0) {
          over = 1;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) over |= __shfl_xor(over, o, G);
    if (over) return -1;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  return *s_count;
}

// rows of `rows` (or all rows when rows == nullptr), 64 / G per 64-lane workgroup, tables of
// at most HT slots (smaller for rows with few products); overflowing rows go to `retry`
template <int G, int HT>
__global__ void __launch_bounds__(64) k_sym_lds(int64_t nrows, const int *__restrict__ rows,
                                                const int64_t *__restrict__ ub,
                                                const int *__restrict__ arp,
                                                const int *__restrict__ aci,
                                                const int *__restrict__ brp,
                                                const int *__restrict__ bci,
                                                int *__restrict__ cnt, int *__restrict__ retry,
                                                int *__restrict__ nretry) {
  constexpr int NR = 64 / G;
  __shared__ int keys[NR][HT];
  __shared__ int s_count[NR], s_excl[NR][G], s_start[NR][G];
  const int g = threadIdx.x / G;
  const int64_t idx = (int64_t)blockIdx.x * NR + g;
  if (idx >= nrows) return;
  const int row = rows ? rows[idx] : (int)idx;
  const int64_t u = ub[row];
  const int ht = u > HT / 2 ? HT : next_pow2_dev(u < 16 ? 32 : 2 * u);
  const int c = sym_row<G>(row, arp, aci, brp, bci, keys[g], ht, &s_count[g], s_excl[g],
                           s_start[g]);
  if ((threadIdx.x & (G - 1)) == 0) {
    if (c < 0) {
      cnt[row] = 0;
      retry[atomicAdd(nretry, 1)] = row;
    } else {
      cnt[row] = c;
    }
  }
}

__global__ void __launch_bounds__(64) k_sym_global(int nrows, const int *__restrict__ rows, int ht,
                                                   const int *__restrict__ arp,
                                                   const int *__restrict__ aci,
                                                   const int *__restrict__ brp,
                                                   const int *__restrict__ bci,
                                                   int *__restrict__ cnt,
                                                   int *__restrict__ scratch,
                                                   int *__restrict__ flag) {
  __shared__ int s_count, s_excl[64], s_start[64];
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  int *keys = scratch + (int64_t)blockIdx.x * ht;
  const int c = sym_row<64>(row, arp, aci, brp, bci, keys, ht, &s_count, s_excl, s_start);
  if (threadIdx.x == 0) {
    if (c < 0) { atomicOr(flag, FLAG_ROW_TOO_LONG); cnt[row] = 0; }
    else cnt[row] = c;
  }
}

template <int G, bool LDS_TABLE>
__device__ __forceinline__ void num_row_g(int row, const int *__restrict__ arp, const int *__restrict__ aci,
                          const double *__restrict__ av, const int *__restrict__ brp,
                          const int *__restrict__ bci, const double *__restrict__ bv,
                          const int *__restrict__ crp, int *__restrict__ cci,
                          double *__restrict__ cv, int *keys, double *vals, int *lk, double *lv,
                          int ht, int *s_n, int *flag) {
  const int l = threadIdx.x & (G - 1);
  const unsigned mask = (unsigned)ht - 1;
  for (int s = l; s < ht; s += G) {
    keys[s] = -1;
    vals[s] = 0.0;
  }
  if (l == 0) *s_n = 0;
  __builtin_amdgcn_wave_barrier();
  const int as = arp[row], ae = arp[row + 1];
  for (int c0 = as; c0 < ae; c0 += G) {
    const int e = c0 + l;
    int k = 0, b0 = 0, b1 = 0;
    double a = 0.0;
    if (e < ae) {
      k = aci[e];
      a = av[e];
      b0 = brp[k];
      b1 = brp[k + 1];
    }
    const int cnt = min(G, ae - c0);
    // PF steps at a time: the first G entries of each selected row of B are loaded into
    // registers for all PF steps before they are applied, in ascending k
    constexpr int PF = 8;
    for (int t0 = 0; t0 < cnt; t0 += PF) {
      int jj[PF], qa[PF], qb[PF];
      double bb[PF], at[PF];
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int tt = (t0 + u < cnt) ? t0 + u : 0;
        at[u] = __shfl(a, tt, G);
        qa[u] = __shfl(b0, tt, G);
        qb[u] = (t0 + u < cnt) ? __shfl(b1, tt, G) : qa[u];
        const int q = qa[u] + l;
        const bool ok = q < qb[u];
        jj[u] = ok ? bci[q] : -1;
        bb[u] = ok ? bv[q] : 0.0;
      }
      // slots of the PF steps first, independent of each other: the home slots are read
      // together and only keys not found there take the probing path
      unsigned sl[PF];
      int seen[PF];
#pragma unroll
      for (int u = 0; u < PF; ++u) sl[u] = hslot(jj[u] >= 0 ? jj[u] : 0, mask);
#pragma unroll
      for (int u = 0; u < PF; ++u) seen[u] = jj[u] >= 0 ? keys[sl[u]] : -1;
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (jj[u] >= 0 && seen[u] != jj[u]) {
          sl[u] = table_find_or_insert(keys, mask, jj[u]);
          if (sl[u] > mask) atomicOr(flag, FLAG_PATTERN);
        }
      }
      // then the products, added in ascending k
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (t0 + u < cnt) {
          if (jj[u] >= 0 && sl[u] <= mask)
            vals[sl[u]] = __dadd_rn(vals[sl[u]], __dmul_rn(at[u], bb[u]));
          for (int q = qa[u] + G + l; q < qb[u]; q += G) {   // rows of B longer than G
            const unsigned slot = table_find_or_insert(keys, mask, bci[q]);
            if (slot > mask) { atomicOr(flag, FLAG_PATTERN); continue; }
            vals[slot] = __dadd_rn(vals[slot], __dmul_rn(at[u], bv[q]));
          }
        }
        table_step_fence<LDS_TABLE>();
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  for (int s = l; s < ht; s += G) {
    const int key = keys[s];
    if (key != -1) {
      const int t = atomicAdd(s_n, 1);
      if (t < ht / 2) {
        lk[t] = key;
        lv[t] = vals[s];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int m = *s_n;
  const int base = crp[row];
  if (m > ht / 2 || m != crp[row + 1] - base) {
    if (l == 0) atomicOr(flag, FLAG_PATTERN);
    return;
  }
  for (int t = l; t < m; t += G) {
    const int key = lk[t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += (lk[u] < key);
    cci[base + rank] = key;
    cv[base + rank] = lv[t];
  }
}

// one 64-lane workgroup = 64 / G rows, each with its own table of HT slots
template <int G, int HT>
__global__ void __launch_bounds__(64) k_num_lds(int nrows, const int *__restrict__ rows,
                                                const int *__restrict__ arp,
                                                const int *__restrict__ aci,
                                                const double *__restrict__ av,
                                                const int *__restrict__ brp,
                                                const int *__restrict__ bci,
                                                const double *__restrict__ bv,
                                                const int *__restrict__ crp, int *__restrict__ cci,
                                                double *__restrict__ cv, int *flag) {
  constexpr int NR = 64 / G;
  __shared__ int keys[NR][HT];
  __shared__ double vals[NR][HT];
  __shared__ int lk[NR][HT / 2];
  __shared__ double lv[NR][HT / 2];
  __shared__ int s_n[NR];
  const int g = threadIdx.x / G;
  const int idx = blockIdx.x * NR + g;
  if (idx >= nrows) return;
  num_row_g<G, true>(rows[idx], arp, aci, av, brp, bci, bv, crp, cci, cv, keys[g], vals[g], lk[g], lv[g],
               HT, &s_n[g], flag);
}

__global__ void __launch_bounds__(64) k_num_global(int nrows, const int *__restrict__ rows, int ht,
                                                   const int *__restrict__ arp,
                                                   const int *__restrict__ aci,
                                                   const double *__restrict__ av,
                                                   const int *__restrict__ brp,
                                                   const int *__restrict__ bci,
                                                   const double *__restrict__ bv,
                                                   const int *__restrict__ crp,
                                                   int *__restrict__ cci, double *__restrict__ cv,
                                                   int *scratch_i, double *scratch_d, int *flag) {
  __shared__ int s_n;
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  int *keys = scratch_i + (int64_t)blockIdx.x * (ht + ht / 2);
  int *lk = keys + ht;
  double *vals = scratch_d + (int64_t)blockIdx.x * (ht + ht / 2);
  double *lv = vals + ht;
  num_row_g<64, false>(row, arp, aci, av, brp, bci, bv, crp, cci, cv, keys, vals, lk, lv, ht, &s_n, flag);
}

// block-product row buckets by output blocks: <= 12, <= 24, <= 32 (16 lanes), <= 64 (32),
// <= 128, <= 256 (64), longer (global tables); then the first four again for rows whose
// steps carry many items (wide: 64 lanes, the same tables)
constexpr int NBUCKET = 11;
constexpr int B_GLOBAL = 6;
constexpr int B_WIDE = 7;

__global__ void k_max_len(int nrows, const int *__restrict__ rows, const int *__restrict__ crp,
                          int *__restrict__ out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  int r = rows[t];
  atomicMax(out, crp[r + 1] - crp[r]);
}

__global__ void k_max_ub(int nrows, const int *__restrict__ rows, const int64_t *__restrict__ ub,
                         unsigned long long *__restrict__ out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  atomicMax(out, (unsigned long long)ub[rows[t]]);
}

// Products with few output columns (coarse AMG levels, m <= DMAX): the row is accumulated
// in a dense LDS array indexed by column instead of a hash table; one 64-lane workgroup (one
// wavefront) per row.  Symbolic: a bit per column, the products walked flat as in sym_row.
// Numeric: the entries of the row of A are read 64 at a time, then PF steps at a time the
// selected rows of B are loaded into registers before they are added in ascending k (the
// same pinned order); the flagged columns are written in ascending order.
constexpr int DMAX = 8192;   // largest dense row: 72 KB of LDS per workgroup

// Products with at most TINY_M output columns (the last coarse levels, where a few output
// rows carry most of the work): B is expanded to a dense row-major array with a presence
// mask per row, and one lane per output column walks the row of A in ascending k, adding
// a_ik b_kj wherever (k, j) is an entry of B: the same products, rounded and added in the
// same order as in the accumulating forms, with every lane busy.
constexpr int TINY_M = 128;

__global__ void k_tiny_expand(int64_t nb, int m, const int *__restrict__ brp,
                              const int *__restrict__ bci, const double *__restrict__ bv,
                              double *__restrict__ bd, unsigned long long *__restrict__ bmask) {
  const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
  const int l = threadIdx.x & 63;
  if (k >= nb) return;
  unsigned long long m0 = 0ull, m1 = 0ull;
  for (int q = brp[k] + l; q < brp[k + 1]; q += 64) {
    const int j = bci[q];
    bd[k * m + j] = bv[q];
    if (j < 64) m0 |= 1ull << j;
    else m1 |= 1ull << (j - 64);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m0 |= __shfl_xor(m0, o, 64);
    m1 |= __shfl_xor(m1, o, 64);
  }
  if (l == 0) {
    bmask[2 * k] = m0;
    bmask[2 * k + 1] = m1;
  }
}

// output pattern of a row: the union of the masks of the rows of B it selects
__global__ void k_tiny_sym(int64_t n, const int *__restrict__ arp, const int *__restrict__ aci,
                           const unsigned long long *__restrict__ bmask,
                           unsigned long long *__restrict__ rmask, int *__restrict__ cnt) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  unsigned long long m0 = 0ull, m1 = 0ull;
  for (int e = arp[row] + l; e < arp[row + 1]; e += 64) {
    const int k = aci[e];
    m0 |= bmask[2 * k];
    m1 |= bmask[2 * k + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m0 |= __shfl_xor(m0, o, 64);
    m1 |= __shfl_xor(m1, o, 64);
  }
  if (l == 0) {
    rmask[2 * row] = m0;
    rmask[2 * row + 1] = m1;
    cnt[row] = __popcll(m0) + __popcll(m1);
  }
}

template <int MW>
__global__ void __launch_bounds__(MW) k_tiny_num(int64_t n, int m, const int *__restrict__ arp,
                                                 const int *__restrict__ aci,
                                                 const double *__restrict__ av,
                                                 const double *__restrict__ bd,
                                                 const unsigned long long *__restrict__ bmask,
                                                 const unsigned long long *__restrict__ rmask,
                                                 const int *__restrict__ crp,
                                                 int *__restrict__ cci, double *__restrict__ cv) {
  const int64_t row = blockIdx.x;
  if (row >= n) return;
  const int j = threadIdx.x, word = j >> 6, bit = j & 63;
  const int as = arp[row], ae = arp[row + 1];
  double acc = 0.0;
  constexpr int U = 8;   // the loads of U steps are issued before they are added in order
  for (int e0 = as; e0 < ae; e0 += U) {
    int kk[U];
    double aa[U], bb[U];
    unsigned long long mm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e0 + u < ae;
      kk[u] = ok ? aci[e0 + u] : 0;
      aa[u] = ok ? av[e0 + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e0 + u < ae;
      mm[u] = ok ? bmask[2 * (int64_t)kk[u] + word] : 0ull;
      bb[u] = (ok && j < m) ? bd[(int64_t)kk[u] * m + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if ((mm[u] >> bit) & 1ull) acc = __dadd_rn(acc, __dmul_rn(aa[u], bb[u]));
  }
  const unsigned long long r = rmask[2 * row + word];
  if (j < m && ((r >> bit) & 1ull)) {
    const int pos = crp[row] + (word ? __popcll(rmask[2 * row]) : 0) +
                    __popcll(r & ((1ull << bit) - 1ull));
    cci[pos] = j;
    cv[pos] = acc;
  }
}

template <int DM>
__global__ void __launch_bounds__(64) k_sym_dense(int64_t n, int m, const int *__restrict__ arp,
                                                  const int *__restrict__ aci,
                                                  const int *__restrict__ brp,
                                                  const int *__restrict__ bci,
                                                  int *__restrict__ cnt) {
  __shared__ unsigned bits[DM / 32];
  __shared__ int s_excl[64], s_start[64];
  const int64_t row = blockIdx.x;
  if (row >= n) return;
  const int l = threadIdx.x;
  for (int w = l; w < (m + 31) / 32; w += 64) bits[w] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int c = 0;
  const int as = arp[row], ae = arp[row + 1];
  for (int c0 = as; c0 < ae; c0 += 64) {
    const int e = c0 + l;
    int len = 0, st = 0;
    if (e < ae) {
      const int k = aci[e];
      st = brp[k];
      len = brp[k + 1] - st;
    }
    int inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(inc, o, 64);
      if (l >= o) inc += t;
    }
    s_excl[l] = inc - len;
    s_start[l] = st;
    const int total = __shfl(inc, 63, 64);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int nent = min(64, ae - c0);
    constexpr int PU = 4;
    for (int p0 = 0; p0 < total; p0 += PU * 64) {
      int jj[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int p = p0 + u * 64 + l;
        jj[u] = -1;
        if (p < total) {
          int lo = 0, hi = nent - 1;        // entry t with s_excl[t] <= p < s_excl[t+1]
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_excl[mid] <= p) lo = mid; else hi = mid - 1;
          }
          jj[u] = bci[s_start[lo] + (p - s_excl[lo])];
        }
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        if (jj[u] < 0) continue;
        const unsigned bit = 1u << (jj[u] & 31);
        c += (atomicOr(&bits[jj[u] >> 5], bit) & bit) == 0u;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (l == 0) cnt[row] = c;
}

template <int DM>
__global__ void __launch_bounds__(64) k_num_dense(int64_t n, int m, const int *__restrict__ arp,
                                                  const int *__restrict__ aci,
                                                  const double *__restrict__ av,
                                                  const int *__restrict__ brp,
                                                  const int *__restrict__ bci,
                                                  const double *__restrict__ bv,
                                                  const int *__restrict__ crp,
                                                  int *__restrict__ cci, double *__restrict__ cv,
                                                  int *flagp) {
  __shared__ double acc[DM];
  __shared__ unsigned char flag[DM];
  const int64_t row = blockIdx.x;
  if (row >= n) return;
  const int l = threadIdx.x;
  for (int j = l; j < m; j += 64) {
    acc[j] = 0.0;
    flag[j] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int as = arp[row], ae = arp[row + 1];
  for (int c0 = as; c0 < ae; c0 += 64) {
    const int e = c0 + l;
    int k = 0, b0 = 0, b1 = 0;
    double a = 0.0;
    if (e < ae) {
      k = aci[e];
      a = av[e];
      b0 = brp[k];
      b1 = brp[k + 1];
    }
    const int cnt = min(64, ae - c0);
    constexpr int PF = 8;
    for (int t0 = 0; t0 < cnt; t0 += PF) {
      int jj[PF], qa[PF], qb[PF];
      double bb[PF], at[PF];
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int tt = (t0 + u < cnt) ? t0 + u : 0;
        at[u] = __shfl(a, tt, 64);
        qa[u] = __shfl(b0, tt, 64);
        qb[u] = (t0 + u < cnt) ? __shfl(b1, tt, 64) : qa[u];
        const int q = qa[u] + l;
        const bool ok = q < qb[u];
        jj[u] = ok ? bci[q] : -1;
        bb[u] = ok ? bv[q] : 0.0;
      }
      // ascending k; the columns of one step are distinct
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (t0 + u < cnt) {
          if (jj[u] >= 0) {
            acc[jj[u]] = __dadd_rn(acc[jj[u]], __dmul_rn(at[u], bb[u]));
            flag[jj[u]] = 1;
          }
          for (int q = qa[u] + 64 + l; q < qb[u]; q += 64) {   // rows of B longer than 64
            const int j = bci[q];
            acc[j] = __dadd_rn(acc[j], __dmul_rn(at[u], bv[q]));
            flag[j] = 1;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  int o = crp[row];
  const int end = crp[row + 1];
  for (int j0 = 0; j0 < m; j0 += 64) {
    const int j = j0 + l;
    const bool f = j < m && flag[j];
    const uint64_t mask = __ballot(f);
    if (f) {
      const int pos = o + __popcll(mask & ((1ull << l) - 1));
      if (pos < end) {
        cci[pos] = j;
        cv[pos] = acc[j];
      }
    }
    o += __popcll(mask);
  }
  if (l == 0 && o != end) atomicOr(flagp, FLAG_PATTERN);
}

// scalar numeric pass: rows by output length, tables of 128 .. 4096 slots in LDS (up to
// 72 KB per workgroup on gfx950), longer rows in global memory
constexpr int NBS = 7;
__global__ void k_bucket_s(int64_t n, const int *__restrict__ crp, int *__restrict__ lists,
                           int *__restrict__ counts, int64_t stride) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int b = -1;
  if (i < n) {
    const int len = crp[i + 1] - crp[i];
    if (len > 0)
      b = len <= 64 ? 0 : len <= 128 ? 1 : len <= 256 ? 2 : len <= 512 ? 3 : len <= 1024 ? 4
        : len <= 2048 ? 5 : 6;
  }
  for (int k = 0; k < NBS; ++k) {
    const uint64_t m = __ballot(b == k);
    if (m == 0) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[k], __popcll(m));
    base = __shfl(base, leader, 64);
    if (b == k) lists[k * stride + base + __popcll(m & ((1ull << lane) - 1))] = (int)i;
  }
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace

namespace {
template <int G, int HT>
void launch_num(int nrows, const int *rows, const Csr &A, const Csr &B, Csr &C, int *dflag,
                hipStream_t s) {
  constexpr int NR = 64 / G;
  k_num_lds<G, HT><<<(nrows + NR - 1) / NR, 64, 0, s>>>(nrows, rows, A.rp.p, A.ci.p, A.v.p, B.rp.p,
                                                        B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p,
                                                        dflag);
  KCHK();
}

// table HT for rows of at most HT/2 outputs; G lanes per row, raised so that the tables of
// one workgroup stay within 36 KB of LDS
void dispatch_num(int bucket, int g0, int nrows, const int *rows, const Csr &A, const Csr &B,
                  Csr &C, int *dflag, hipStream_t s) {
  const int HT = 128 << bucket;
  int G = std::min(64, std::max(g0, HT / 32));
#define NUMCASE(GG, HH)                                          \
  if (G == GG && HT == HH) {                                     \
    launch_num<GG, HH>(nrows, rows, A, B, C, dflag, s);          \
    return;                                                      \
  }
  NUMCASE(8, 128) NUMCASE(16, 128) NUMCASE(32, 128) NUMCASE(64, 128)
  NUMCASE(8, 256) NUMCASE(16, 256) NUMCASE(32, 256) NUMCASE(64, 256)
  NUMCASE(16, 512) NUMCASE(32, 512) NUMCASE(64, 512)
  NUMCASE(32, 1024) NUMCASE(64, 1024) NUMCASE(64, 2048) NUMCASE(64, 4096)
#undef NUMCASE
  throw Error(MGR_ERR_HIP, "spgemm: no numeric kernel for this bucket");
}

int lanes_for(double mean) { return mean > 48 ? 64 : mean > 24 ? 32 : mean > 6 ? 16 : 8; }
}  // namespace

void spgemm_symbolic(int64_t n, const int *arp, const int *aci, int64_t annz, const int *brp,
                     const int *bci, int64_t bn, int64_t bm, int64_t bnnz, int *crp,
                     int64_t &cnnz, hipStream_t s, int *dflag, DArr<int64_t> *ub_out,
                     const SymBucket *bk) {
  DArr<int64_t> ub(n, s);
  k_upper_bound<<<grid_for(n * 16, 256), 256, 0, s>>>(n, arp, aci, brp, ub.p);
  KCHK();
  DArr<int> cnt(n + 1, s), retry(n, s);
  // read back together: the retry counts of passes 1 and 2 (two ints) and the total
  DArr<int64_t> rbk(2, s);
  int *nretry_p = reinterpret_cast<int *>(rbk.p);
  fill<int>(nretry_p, 0, 2, s);
  // symbolic pass 1: tables of <= 512 slots, 64 / G rows per workgroup
  const double meanA = (double)annz / (double)std::max<int64_t>(n, 1);
  const double meanB = (double)bnnz / (double)std::max<int64_t>(bn, 1);
  const double prods = meanA * meanB;
  if (prods > 256) {
    k_sym_lds<64, 512><<<(unsigned)n, 64, 0, s>>>(n, nullptr, ub.p, arp, aci, brp, bci, cnt.p,
                                                  retry.p, nretry_p);
  } else if (prods > 64) {
    k_sym_lds<32, 512><<<(unsigned)((n + 1) / 2), 64, 0, s>>>(n, nullptr, ub.p, arp, aci, brp,
                                                              bci, cnt.p, retry.p, nretry_p);
  } else {
    k_sym_lds<16, 512><<<(unsigned)((n + 3) / 4), 64, 0, s>>>(n, nullptr, ub.p, arp, aci, brp,
                                                              bci, cnt.p, retry.p, nretry_p);
  }
  KCHK();
  // the scan assumes that pass 1 counted every row; it is repeated when some did not fit
  exclusive_scan_i32_async(cnt.p, crp, n, s, rbk.p + 1);
  if (bk) bk->launch(ub.p);
  int64_t hb[2];
  const D2HPart parts[2] = {{hb, rbk.p, sizeof(hb)},
                            {bk ? bk->host : nullptr, bk ? bk->counts : nullptr,
                             bk ? bk->nc * sizeof(int) : 0}};
  d2h_sync_parts(parts, 2, s);
  const int hretry = reinterpret_cast<const int *>(hb)[0];
  if (hretry == 0) {
    require(hb[1] <= 0x7fffffffLL, MGR_ERR_UNSUPPORTED,
            "prefix sum exceeds 2^31 (matrix too large)");
    cnnz = hb[1];
    if (ub_out) *ub_out = std::move(ub);
    return;
  }
  {
    // pass 2: 4096-slot tables, one row per workgroup
    DArr<int> retry2(hretry, s);
    k_sym_lds<64, SYM_HT><<<(unsigned)hretry, 64, 0, s>>>(hretry, retry.p, ub.p, arp, aci, brp,
                                                          bci, cnt.p, retry2.p, nretry_p + 1);
    KCHK();
    const int hretry2 = read_flag(nretry_p + 1, s);
    if (hretry2 > 0) {
      // pass 3: tables in global memory sized by the largest row
      DArr<unsigned long long> mub(1, s);
      fill<unsigned long long>(mub.p, 0ull, 1, s);
      k_max_ub<<<grid_for(hretry2, 256), 256, 0, s>>>(hretry2, retry2.p, ub.p, mub.p);
      KCHK();
      unsigned long long hm = 0;
      d2h_sync(&hm, mub.p, sizeof(hm), s);
      const int64_t cap = std::min<int64_t>((int64_t)hm, bm);
      const int64_t ht = next_pow2(2 * std::max<int64_t>(cap, 32));
      require(ht <= (int64_t)1 << 22, MGR_ERR_UNSUPPORTED,
              "spgemm: a product row exceeds the supported length");
      const int64_t batch = std::max<int64_t>(1, ((int64_t)64 << 20) / (ht * 4));
      DArr<int> scratch(std::min<int64_t>(batch, hretry2) * ht, s);
      for (int64_t b0 = 0; b0 < hretry2; b0 += batch) {
        const int nb = (int)std::min<int64_t>(batch, hretry2 - b0);
        k_sym_global<<<nb, 64, 0, s>>>(nb, retry2.p + b0, (int)ht, arp, aci, brp, bci, cnt.p,
                                       scratch.p, dflag);
        KCHK();
      }
    }
  }
  cnnz = exclusive_scan_i32(cnt.p, crp, n, s);
  if (bk) {
    bk->launch(ub.p);
    d2h_sync(bk->host, bk->counts, bk->nc * sizeof(int), s);
  }
  if (ub_out) *ub_out = std::move(ub);
}

// ---------------------------------------------------------------------------------
// Products whose rows of A come in groups of R rows with one column pattern (the rows of a
// cell in A_CF): the rows of a group select the same rows of B, so they share the symbolic
// count, the loads of B and the hash table of output columns; each row keeps its own
// accumulators, summed in the same ascending k as the scalar kernels, so C is the same to
// the bit.
namespace {
template <int R>
__global__ void k_group_same(int64_t ng, const int *__restrict__ arp, const int *__restrict__ aci,
                             int *__restrict__ flag) {
  const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 16;
  const int l = threadIdx.x & 15;
  if (g >= ng) return;
  const int64_t r0 = g * R;
  const int s0 = arp[r0], len = arp[r0 + 1] - s0;
  bool bad = false;
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const int sr = arp[r0 + r];
    if (arp[r0 + r + 1] - sr != len) bad = true;
    else
      for (int e = l; e < len; e += 16) bad |= aci[sr + e] != aci[s0 + e];
  }
  if (bad) atomicOr(flag, 1);
}
// the first row of every group; upper bounds of their products
__global__ void k_group_rows(int64_t ng, int R, const int *__restrict__ arp,
                             const int *__restrict__ aci, const int *__restrict__ brp,
                             int *__restrict__ rows, int64_t *__restrict__ ub) {
  constexpr int G = 16;
  const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (g >= ng) return;
  const int64_t i = g * R;
  int64_t sum = 0;
  for (int e = arp[i] + l; e < arp[i + 1]; e += G) {
    const int k = aci[e];
    sum += brp[k + 1] - brp[k];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, G);
  if (l == 0) {
    rows[g] = (int)i;
    ub[i] = sum;
  }
}
__global__ void k_group_bcast(int64_t ng, int R, int *__restrict__ cnt, int *__restrict__ mx) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const int c = cnt[g * R];
  for (int r = 1; r < R; ++r) cnt[g * R + r] = c;
  atomicMax(mx, c);
}

template <int G, int R>
__device__ __forceinline__ void num_group_g(int r0, const int *__restrict__ arp,
                                            const int *__restrict__ aci,
                                            const double *__restrict__ av,
                                            const int *__restrict__ brp,
                                            const int *__restrict__ bci,
                                            const double *__restrict__ bv,
                                            const int *__restrict__ crp, int *__restrict__ cci,
                                            double *__restrict__ cv, int *keys, double *vals,
                                            int *lk, int *ls, int ht, int *s_n, int *flag) {
  const int l = threadIdx.x & (G - 1);
  const unsigned mask = (unsigned)ht - 1;
  for (int q = l; q < ht; q += G) {
    keys[q] = -1;
#pragma unroll
    for (int r = 0; r < R; ++r) vals[r * ht + q] = 0.0;
  }
  if (l == 0) *s_n = 0;
  __builtin_amdgcn_wave_barrier();
  const int as = arp[r0], ae = arp[r0 + 1];
  int aoff[R];
#pragma unroll
  for (int r = 0; r < R; ++r) aoff[r] = arp[r0 + r] - as;
  for (int c0 = as; c0 < ae; c0 += G) {
    const int e = c0 + l;
    int k = 0, b0 = 0, b1 = 0;
    double a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = 0.0;
    if (e < ae) {
      k = aci[e];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = av[e + aoff[r]];
      b0 = brp[k];
      b1 = brp[k + 1];
    }
    const int cnt = min(G, ae - c0);
    constexpr int PF = 8;
    for (int t0 = 0; t0 < cnt; t0 += PF) {
      int jj[PF], qa[PF], qb[PF];
      double bb[PF], at[PF][R];
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int tt = (t0 + u < cnt) ? t0 + u : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) at[u][r] = __shfl(a[r], tt, G);
        qa[u] = __shfl(b0, tt, G);
        qb[u] = (t0 + u < cnt) ? __shfl(b1, tt, G) : qa[u];
        const int q = qa[u] + l;
        const bool ok = q < qb[u];
        jj[u] = ok ? bci[q] : -1;
        bb[u] = ok ? bv[q] : 0.0;
      }
      unsigned sl[PF];
      int seen[PF];
#pragma unroll
      for (int u = 0; u < PF; ++u) sl[u] = hslot(jj[u] >= 0 ? jj[u] : 0, mask);
#pragma unroll
      for (int u = 0; u < PF; ++u) seen[u] = jj[u] >= 0 ? keys[sl[u]] : -1;
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (jj[u] >= 0 && seen[u] != jj[u]) {
          sl[u] = table_find_or_insert(keys, mask, jj[u]);
          if (sl[u] > mask) atomicOr(flag, FLAG_PATTERN);
        }
      }
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (t0 + u < cnt) {
          if (jj[u] >= 0 && sl[u] <= mask) {
#pragma unroll
            for (int r = 0; r < R; ++r)
              vals[r * ht + sl[u]] = __dadd_rn(vals[r * ht + sl[u]], __dmul_rn(at[u][r], bb[u]));
          }
          for (int q = qa[u] + G + l; q < qb[u]; q += G) {   // rows of B longer than G
            const unsigned slot = table_find_or_insert(keys, mask, bci[q]);
            if (slot > mask) { atomicOr(flag, FLAG_PATTERN); continue; }
            const double bq = bv[q];
#pragma unroll
            for (int r = 0; r < R; ++r)
              vals[r * ht + slot] = __dadd_rn(vals[r * ht + slot], __dmul_rn(at[u][r], bq));
          }
        }
        table_step_fence<true>();
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  for (int q = l; q < ht; q += G) {
    const int key = keys[q];
    if (key != -1) {
      const int t = atomicAdd(s_n, 1);
      if (t < (3 * ht) / 4) {
        lk[t] = key;
        ls[t] = q;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int m = *s_n;
  bool bad = m > (3 * ht) / 4;
#pragma unroll
  for (int r = 0; r < R; ++r) bad |= m != crp[r0 + r + 1] - crp[r0 + r];
  if (bad) {
    if (l == 0) atomicOr(flag, FLAG_PATTERN);
    return;
  }
  for (int t = l; t < m; t += G) {
    const int key = lk[t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += (lk[u] < key);
    const int q = ls[t];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = crp[r0 + r] + rank;
      cci[pos] = key;
      cv[pos] = vals[r * ht + q];
    }
  }
}

// one 64-lane workgroup = 64 / G groups, each with its key table of HT slots and R value
// tables
template <int G, int HT, int R>
__global__ void __launch_bounds__(64) k_num_grp(int ngrp, const int *__restrict__ rows,
                                                const int *__restrict__ arp,
                                                const int *__restrict__ aci,
                                                const double *__restrict__ av,
                                                const int *__restrict__ brp,
                                                const int *__restrict__ bci,
                                                const double *__restrict__ bv,
                                                const int *__restrict__ crp,
                                                int *__restrict__ cci, double *__restrict__ cv,
                                                int *flag) {
  constexpr int NR = 64 / G;
  __shared__ int keys[NR][HT];
  __shared__ double vals[NR][R * HT];
  __shared__ int lk[NR][3 * HT / 4], ls[NR][3 * HT / 4];
  __shared__ int s_n[NR];
  const int g = threadIdx.x / G;
  const int idx = blockIdx.x * NR + g;
  if (idx >= ngrp) return;
  num_group_g<G, R>(rows[idx], arp, aci, av, brp, bci, bv, crp, cci, cv, keys[g], vals[g],
                    lk[g], ls[g], HT, &s_n[g], flag);
}

// C = A B by groups of R rows when every group of A shares one column pattern and every
// output row fits a table of 512 slots; false (nothing written to C) otherwise
bool spgemm_grouped(const Csr &A, const Csr &B, Csr &C, int R, hipStream_t s, int *dflag) {
  const int64_t n = A.n, ng = n / R;
  if (R < 2 || R > 3 || n % R != 0 || ng == 0 || ng > 0x7fffffffLL) return false;
  DArr<int> f(1, s);
  fill<int>(f.p, 0, 1, s);
  if (R == 2) k_group_same<2><<<grid_for(ng * 16, 256), 256, 0, s>>>(ng, A.rp.p, A.ci.p, f.p);
  else k_group_same<3><<<grid_for(ng * 16, 256), 256, 0, s>>>(ng, A.rp.p, A.ci.p, f.p);
  KCHK();
  if (read_flag(f.p, s) != 0) return false;
  DArr<int> rows(ng, s), cnt(n + 1, s), retry(ng, s), mx(1, s);
  DArr<int64_t> ub(n, s);
  k_group_rows<<<grid_for(ng * 16, 256), 256, 0, s>>>(ng, R, A.rp.p, A.ci.p, B.rp.p, rows.p, ub.p);
  KCHK();
  fill<int>(f.p, 0, 1, s);
  fill<int>(mx.p, 0, 1, s);
  const double meanA = (double)A.nnz / (double)std::max<int64_t>(n, 1);
  const double meanB = (double)B.nnz / (double)std::max<int64_t>(B.n, 1);
  const double prods = meanA * meanB;
  if (prods > 256)
    k_sym_lds<64, 512><<<(unsigned)ng, 64, 0, s>>>(ng, rows.p, ub.p, A.rp.p, A.ci.p, B.rp.p,
                                                   B.ci.p, cnt.p, retry.p, f.p);
  else if (prods > 64)
    k_sym_lds<32, 512><<<(unsigned)((ng + 1) / 2), 64, 0, s>>>(ng, rows.p, ub.p, A.rp.p, A.ci.p,
                                                               B.rp.p, B.ci.p, cnt.p, retry.p, f.p);
  else
    k_sym_lds<16, 512><<<(unsigned)((ng + 3) / 4), 64, 0, s>>>(ng, rows.p, ub.p, A.rp.p, A.ci.p,
                                                               B.rp.p, B.ci.p, cnt.p, retry.p, f.p);
  KCHK();
  k_group_bcast<<<grid_for(ng, 256), 256, 0, s>>>(ng, R, cnt.p, mx.p);
  KCHK();
  int hb[2];
  const D2HPart parts[2] = {{&hb[0], f.p, sizeof(int)}, {&hb[1], mx.p, sizeof(int)}};
  d2h_sync_parts(parts, 2, s);
  if (hb[0] != 0 || hb[1] > 256) return false;   // a row needs a larger table
  C.nnz = exclusive_scan_i32(cnt.p, C.rp.p, n, s);
  C.ci.alloc(std::max<int64_t>(C.nnz, 1), s);
  C.v.alloc(std::max<int64_t>(C.nnz, 1), s);
  if (C.nnz == 0) return true;
  // tables filled up to three quarters: half the LDS of a half-full table, so twice the
  // groups share a CU (the kernel waits on its loads; the longer probe runs cost less)
  const int ht = hb[1] <= 96 ? 128 : hb[1] <= 192 ? 256 : 512;
  // lanes per group: 16 while the rows of B average at most 16 entries (longer rows take a
  // second pass), else 32 or 64
  const int G = meanB > 48 ? 64 : meanB > 16 ? 32 : 16;
#define GRP(GG, HH, RR)                                                                        \
  if (G == GG && ht == HH && R == RR) {                                                        \
    k_num_grp<GG, HH, RR><<<(unsigned)((ng + 64 / GG - 1) / (64 / GG)), 64, 0, s>>>(           \
        (int)ng, rows.p, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p,   \
        dflag);                                                                                \
    KCHK();                                                                                    \
    return true;                                                                               \
  }
  GRP(16, 128, 2) GRP(16, 256, 2) GRP(32, 128, 2) GRP(32, 256, 2) GRP(64, 128, 2) GRP(64, 256, 2)
  GRP(16, 128, 3) GRP(16, 256, 3) GRP(32, 128, 3) GRP(32, 256, 3) GRP(64, 128, 3) GRP(64, 256, 3)
  GRP(16, 512, 2) GRP(32, 512, 2) GRP(64, 512, 2) GRP(32, 512, 3) GRP(64, 512, 3)
#undef GRP
  // no instance for this shape (16 lanes with three 512-slot value tables would need 64 KB
  // of LDS): the scalar path (C's row pointers are rebuilt there)
  C.ci.reset();
  C.v.reset();
  return false;
}
}  // namespace

void spgemm(const Csr &A, const Csr &B, Csr &C, hipStream_t s, int *dflag, int group) {
  require(A.m == B.n, MGR_ERR_ARG, "spgemm: inner dimensions differ");
  const int64_t n = A.n;
  C.n = n;
  C.m = B.m;
  C.rp.alloc(n + 1, s);
  if (n == 0) {
    fill<int>(C.rp.p, 0, 1, s);
    C.nnz = 0;
    return;
  }
  const double meanB = (double)B.nnz / (double)std::max<int64_t>(B.n, 1);
  const double meanA = (double)A.nnz / (double)std::max<int64_t>(A.n, 1);
  const bool tiny_or_dense = B.m <= DMAX && meanA * meanB >= 64.0 &&
                             (B.m <= TINY_M || (double)B.m <= (B.m > 4096 ? 8.0 : 64.0) *
                                                               meanA * meanB);
  if (group > 1 && !tiny_or_dense && spgemm_grouped(A, B, C, group, s, dflag)) return;
  if (B.m <= TINY_M && meanA * meanB >= 64.0 && B.n * B.m <= ((int64_t)1 << 24)) {
    const int mm = (int)B.m;
    DArr<double> bd(std::max<int64_t>(B.n * mm, 1), s);
    DArr<unsigned long long> bmask(2 * std::max<int64_t>(B.n, 1), s), rmask(2 * n, s);
    DArr<int> cnt(n + 1, s);
    if (B.n > 0) {
      k_tiny_expand<<<grid_for(B.n * 64, 256), 256, 0, s>>>(B.n, mm, B.rp.p, B.ci.p, B.v.p, bd.p,
                                                            bmask.p);
      KCHK();
    }
    k_tiny_sym<<<grid_for(n * 64, 256), 256, 0, s>>>(n, A.rp.p, A.ci.p, bmask.p, rmask.p, cnt.p);
    KCHK();
    C.nnz = exclusive_scan_i32(cnt.p, C.rp.p, n, s);
    C.ci.alloc(std::max<int64_t>(C.nnz, 1), s);
    C.v.alloc(std::max<int64_t>(C.nnz, 1), s);
    if (C.nnz > 0) {
      if (mm <= 64)
        k_tiny_num<64><<<(unsigned)n, 64, 0, s>>>(n, mm, A.rp.p, A.ci.p, A.v.p, bd.p, bmask.p,
                                                  rmask.p, C.rp.p, C.ci.p, C.v.p);
      else
        k_tiny_num<128><<<(unsigned)n, 128, 0, s>>>(n, mm, A.rp.p, A.ci.p, A.v.p, bd.p, bmask.p,
                                                    rmask.p, C.rp.p, C.ci.p, C.v.p);
      KCHK();
    }
    return;
  }
  // dense accumulation pays when a row's products cover a good part of its columns; the
  // widest tables (beyond 4096 columns, 72 KB of LDS: two workgroups per CU) only when the
  // products are at least an eighth of the columns
  const double dense_ratio = B.m > 4096 ? 8.0 : 64.0;
  if (B.m <= DMAX && meanA * meanB >= 64.0 && (double)B.m <= dense_ratio * meanA * meanB) {
    // few output columns and many products per row: dense accumulation
    // tables sized to the column count: small ones leave room for several workgroups per CU
    DArr<int> cnt(n + 1, s);
    const int mm = (int)B.m;
#define DSYM(DM) k_sym_dense<DM><<<(unsigned)n, 64, 0, s>>>(n, mm, A.rp.p, A.ci.p, B.rp.p, B.ci.p, cnt.p)
    if (mm <= 128) DSYM(128);
    else if (mm <= 512) DSYM(512);
    else if (mm <= 2048) DSYM(2048);
    else if (mm <= 4096) DSYM(4096);
    else DSYM(DMAX);
#undef DSYM
    KCHK();
    C.nnz = exclusive_scan_i32(cnt.p, C.rp.p, n, s);
    C.ci.alloc(std::max<int64_t>(C.nnz, 1), s);
    C.v.alloc(std::max<int64_t>(C.nnz, 1), s);
    if (C.nnz > 0) {
#define DNUM(DM)                                                                           \
  k_num_dense<DM><<<(unsigned)n, 64, 0, s>>>(n, mm, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, \
                                             B.v.p, C.rp.p, C.ci.p, C.v.p, dflag)
      if (mm <= 128) DNUM(128);
      else if (mm <= 512) DNUM(512);
      else if (mm <= 2048) DNUM(2048);
      else if (mm <= 4096) DNUM(4096);
      else DNUM(DMAX);
#undef DNUM
      KCHK();
    }
    return;
  }
  // rows bucketed by output length for the numeric phase (read back with the symbolic totals)
  DArr<int> lists((size_t)NBS * n, s), counts(NBS, s);
  int hc[NBS] = {};
  SymBucket bk;
  bk.launch = [&](const int64_t *) {
    fill<int>(counts.p, 0, NBS, s);
    k_bucket_s<<<grid_for(n, 256), 256, 0, s>>>(n, C.rp.p, lists.p, counts.p, n);
    KCHK();
  };
  bk.counts = counts.p;
  bk.host = hc;
  bk.nc = NBS;
  spgemm_symbolic(n, A.rp.p, A.ci.p, A.nnz, B.rp.p, B.ci.p, B.n, B.m, B.nnz, C.rp.p, C.nnz, s,
                  dflag, nullptr, &bk);
  C.ci.alloc(C.nnz, s);
  C.v.alloc(C.nnz, s);
  if (C.nnz == 0) return;
  const int g0 = lanes_for(meanB);
  for (int b = 0; b < NBS - 1; ++b)
    if (hc[b] > 0) dispatch_num(b, g0, hc[b], lists.p + (size_t)b * n, A, B, C, dflag, s);
  const int nbig = hc[NBS - 1];
  if (nbig > 0) {
    const int *big = lists.p + (size_t)(NBS - 1) * n;
    DArr<int> mx(1, s);
    fill<int>(mx.p, 0, 1, s);
    k_max_len<<<grid_for(nbig, 256), 256, 0, s>>>(nbig, big, C.rp.p, mx.p);
    KCHK();
    const int hm = read_flag(mx.p, s);
    const int64_t ht = next_pow2(2 * (int64_t)hm);
    require(ht <= (int64_t)1 << 22, MGR_ERR_UNSUPPORTED,
            "spgemm: a product row exceeds the supported length");
    const int64_t per = ht + ht / 2;
    const int64_t batch = std::max<int64_t>(1, ((int64_t)128 << 20) / (per * 12));
    const int64_t nb0 = std::min<int64_t>(batch, nbig);
    DArr<int> si(nb0 * per, s);
    DArr<double> sd(nb0 * per, s);
    for (int64_t b0 = 0; b0 < nbig; b0 += batch) {
      const int nb = (int)std::min<int64_t>(batch, nbig - b0);
      k_num_global<<<nb, 64, 0, s>>>(nb, big + b0, (int)ht, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p,
                                     B.v.p, C.rp.p, C.ci.p, C.v.p, si.p, sd.p, dflag);
      KCHK();
    }
  }
}


// ---------------------------------------------------------------------------------------
// 3x3 block products for the nodal AMG (A T, A P and R (A P) of matrices whose patterns
// consist of full 3x3 blocks).  Scalar entry (3I+r, 3J+s) of C = A B is the sum over the
// scalar columns k = 3K+c of row 3I+r, in ascending k; walking the blocks K of block row I
// in ascending order and c = 0, 1, 2 inside each block visits the same k in the same order,
// so every entry gets the same products, rounded the same way, added in the same order as
// in the scalar product above: the values agree bit for bit, with 1/9 of the index work.
// With `diagb` the blocks of B are diagonal (the tentative prolongator): only c = s
// contributes, exactly the products the scalar form takes.
namespace {

template <int G, bool DIAGB, bool LDS_TABLE>
__device__ __forceinline__ void num_row_b3(int row, const int *__restrict__ arp, const int *__restrict__ aci,
                           const double *__restrict__ av, const int *__restrict__ brp,
                           const int *__restrict__ bci, const double *__restrict__ bv,
                           const int *__restrict__ crp, int *__restrict__ cci,
                           double *__restrict__ cv, int *keys, double *vals, int *lk, int *ls,
                           int ht, int cap, int *s_n, int *flag) {
  const int l = threadIdx.x & (G - 1);
  const unsigned mask = (unsigned)ht - 1;
  for (int q = l; q < ht; q += G) keys[q] = -1;
  for (int q = l; q < 9 * ht; q += G) vals[q] = 0.0;
  if (l == 0) *s_n = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int as = arp[row], ae = arp[row + 1];
  // The column and B-row bounds of G blocks of the row are loaded at once, one per lane, and
  // handed to the steps by shuffles.  The work of a step is split into units of at most one
  // item per lane; the loads of PB units are issued together, then the units update the
  // table in order, so one memory latency is paid per PB units.  Updates of consecutive
  // steps are ordered by a fence.
  constexpr int PB = 8;
  for (int c0 = as; c0 < ae; c0 += G) {
    int kb0 = 0, kb1 = 0;
    if (c0 + l < ae) {
      const int kk = aci[c0 + l];
      kb0 = brp[kk];
      kb1 = brp[kk + 1];
    }
    const int cnt = min(G, ae - c0);
    if (DIAGB) {
      // unit = one step; lane t < 9 owns entry t = 3r + s of the output block and takes the
      // products a_rs * b_ss; the first block of each step's row of B is prefetched
      const int s3 = l % 3;
      for (int st0 = 0; st0 < cnt; st0 += PB) {
        double a[PB], bd[PB];
        int key[PB], q0[PB], q1[PB];
#pragma unroll
        for (int j = 0; j < PB; ++j) {
          const int st = st0 + j < cnt ? st0 + j : cnt - 1;
          q0[j] = __shfl(kb0, st, G);
          q1[j] = __shfl(kb1, st, G);
          a[j] = 0.0;
          bd[j] = 0.0;
          key[j] = -1;
          if (st0 + j < cnt) {
            if (l < 9) a[j] = av[9 * (int64_t)(c0 + st) + l];
            if (q0[j] < q1[j]) {
              key[j] = bci[q0[j]];
              if (l < 9) bd[j] = bv[9 * (int64_t)q0[j] + 4 * s3];
            }
          }
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
          if (st0 + j >= cnt) break;
          for (int q = q0[j]; q < q1[j]; ++q) {
            const int kq = q == q0[j] ? key[j] : bci[q];
            const double bq = q == q0[j] ? bd[j] : (l < 9 ? bv[9 * (int64_t)q + 4 * s3] : 0.0);
            const unsigned slot = table_find_or_insert(keys, mask, kq);
            if (slot > mask) {
              atomicOr(flag, FLAG_PATTERN);
              continue;
            }
            if (l < 9) {
              double *c = vals + 9 * slot + l;
              *c = __dadd_rn(*c, __dmul_rn(a[j], bq));
            }
          }
          table_step_fence<LDS_TABLE>();
        }
      }
    } else {
      // unit = (step, items i0 .. i0 + G - 1); item it = 3 (q - b0) + r: the output block
      // row r of the block product with block q of B, three entries of one block row
      int st = 0, i0 = 0;
      int b0 = __shfl(kb0, 0, G), b1 = __shfl(kb1, 0, G);
      while (st < cnt) {
        int key[PB], r[PB], ust[PB];
        double a0[PB], a1[PB], a2[PB], b[PB][9];
#pragma unroll
        for (int j = 0; j < PB; ++j) {
          key[j] = -1;
          ust[j] = -1;
          r[j] = 0;
          if (st < cnt) {
            ust[j] = st;
            const int it = i0 + l;
            if (it < 3 * (b1 - b0)) {
              const int e = c0 + st;
              const int q = b0 + it / 3;
              r[j] = it - 3 * (it / 3);
              a0[j] = av[9 * (int64_t)e + 3 * r[j]];
              a1[j] = av[9 * (int64_t)e + 3 * r[j] + 1];
              a2[j] = av[9 * (int64_t)e + 3 * r[j] + 2];
#pragma unroll
              for (int t = 0; t < 9; ++t) b[j][t] = bv[9 * (int64_t)q + t];
              key[j] = bci[q];
            }
            i0 += G;
            if (i0 >= 3 * (b1 - b0)) {
              ++st;
              i0 = 0;
              const int ss = st < cnt ? st : cnt - 1;
              b0 = __shfl(kb0, ss, G);
              b1 = __shfl(kb1, ss, G);
            }
          }
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
          if (ust[j] < 0) break;
          if (j > 0 && ust[j] != ust[j - 1]) table_step_fence<LDS_TABLE>();
          if (key[j] >= 0) {
            const unsigned slot = table_find_or_insert(keys, mask, key[j]);
            if (slot > mask) {
              atomicOr(flag, FLAG_PATTERN);
            } else {
              double *c = vals + 9 * slot + 3 * r[j];
#pragma unroll
              for (int t = 0; t < 3; ++t) {
                double x = c[t];
                x = __dadd_rn(x, __dmul_rn(a0[j], b[j][0 + t]));
                x = __dadd_rn(x, __dmul_rn(a1[j], b[j][3 + t]));
                x = __dadd_rn(x, __dmul_rn(a2[j], b[j][6 + t]));
                c[t] = x;
              }
            }
          }
        }
        table_step_fence<LDS_TABLE>();
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  for (int q = l; q < ht; q += G) {
    const int key = keys[q];
    if (key != -1) {
      const int t = atomicAdd(s_n, 1);
      if (t < cap) {
        lk[t] = key;
        ls[t] = q;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int m = *s_n;
  const int base = crp[row];
  if (m > cap || m != crp[row + 1] - base) {
    if (l == 0) atomicOr(flag, FLAG_PATTERN);
    return;
  }
  for (int t = l; t < m; t += G) {
    const int key = lk[t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += (lk[u] < key);
    cci[base + rank] = key;
    const double *c = vals + 9 * ls[t];
#pragma unroll
    for (int q = 0; q < 9; ++q) cv[9 * (int64_t)(base + rank) + q] = c[q];
  }
}

template <int G, int HT, bool DIAGB>
__global__ void __launch_bounds__(64) k_num_b3(int nrows, const int *__restrict__ rows,
                                               const int *__restrict__ arp,
                                               const int *__restrict__ aci,
                                               const double *__restrict__ av,
                                               const int *__restrict__ brp,
                                               const int *__restrict__ bci,
                                               const double *__restrict__ bv,
                                               const int *__restrict__ crp, int *__restrict__ cci,
                                               double *__restrict__ cv, int *flag) {
  constexpr int NR = 64 / G;
  // tables filled up to three quarters (rows of at most 3 HT / 4 blocks)
  constexpr int CAP = 3 * HT / 4;
  __shared__ int keys[NR][HT];
  __shared__ double vals[NR][9 * HT];
  __shared__ int lk[NR][CAP], ls[NR][CAP];
  __shared__ int s_n[NR];
  const int g = threadIdx.x / G;
  const int idx = blockIdx.x * NR + g;
  if (idx >= nrows) return;
  num_row_b3<G, DIAGB, true>(rows[idx], arp, aci, av, brp, bci, bv, crp, cci, cv, keys[g], vals[g],
                       lk[g], ls[g], HT, CAP, &s_n[g], flag);
}

template <bool DIAGB>
__global__ void __launch_bounds__(64) k_num_b3_global(
    int nrows, const int *__restrict__ rows, int ht, const int *__restrict__ arp,
    const int *__restrict__ aci, const double *__restrict__ av, const int *__restrict__ brp,
    const int *__restrict__ bci, const double *__restrict__ bv, const int *__restrict__ crp,
    int *__restrict__ cci, double *__restrict__ cv, int *scratch_i, double *scratch_d,
    int *flag) {
  __shared__ int s_n;
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  int *keys = scratch_i + (int64_t)blockIdx.x * 2 * ht;
  int *lk = keys + ht;
  int *ls = lk + ht / 2;
  double *vals = scratch_d + (int64_t)blockIdx.x * 9 * ht;
  num_row_b3<64, DIAGB, false>(row, arp, aci, av, brp, bci, bv, crp, cci, cv, keys, vals, lk, ls, ht,
                        ht / 2, &s_n, flag);
}

// block rows by output block count: <= 32, <= 64, <= 128, <= 256, longer.  A row of the
// first two classes whose steps average more items (3 per block of B) than two per lane of
// its group goes to the wide class of the same table size, one 64-lane group per row.
__global__ void k_bucket_b3(int64_t n, const int *__restrict__ crp, const int *__restrict__ arp,
                            const int64_t *__restrict__ ub, int diagb, int *__restrict__ lists,
                            int *__restrict__ counts, int64_t stride) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int b = -1;
  if (i < n) {
    const int len = crp[i + 1] - crp[i];
    if (len > 0)
      b = len <= 12 ? 0 : len <= 24 ? 1 : len <= 32 ? 2 : len <= 64 ? 3 : len <= 128 ? 4
        : len <= 256 ? 5 : B_GLOBAL;
    if (!diagb && b >= 0 && b <= 3) {
      const int64_t items = 3 * ub[i], steps = arp[i + 1] - arp[i];
      if (items > (b <= 2 ? 32 : 64) * steps) b += B_WIDE;
    }
  }
  for (int k = 0; k < NBUCKET; ++k) {
    const uint64_t m = __ballot(b == k);
    if (m == 0) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[k], __popcll(m));
    base = __shfl(base, leader, 64);
    if (b == k) lists[k * stride + base + __popcll(m & ((1ull << lane) - 1))] = (int)i;
  }
}

template <int G, int HT>
void launch_num_b3(bool diagb, int nrows, const int *rows, const Bsr3 &A, const Bsr3 &B,
                   Bsr3 &C, int *dflag, hipStream_t s) {
  constexpr int NR = 64 / G;
  const unsigned grid = (unsigned)((nrows + NR - 1) / NR);
  if (diagb)
    k_num_b3<G, HT, true><<<grid, 64, 0, s>>>(nrows, rows, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p,
                                              B.v.p, C.rp.p, C.ci.p, C.v.p, dflag);
  else
    k_num_b3<G, HT, false><<<grid, 64, 0, s>>>(nrows, rows, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p,
                                               B.v.p, C.rp.p, C.ci.p, C.v.p, dflag);
  KCHK();
}

}  // namespace

void spgemm_b3(const Bsr3 &A, const Bsr3 &B, bool diagb, Bsr3 &C, hipStream_t s, int *dflag) {
  require(A.mb == B.nb, MGR_ERR_ARG, "block spgemm: inner dimensions differ");
  const int64_t n = A.nb;
  C.nb = n;
  C.mb = B.mb;
  C.rp.alloc(n + 1, s);
  if (n == 0) {
    fill<int>(C.rp.p, 0, 1, s);
    C.nnzb = 0;
    return;
  }
  DArr<int64_t> ub;
  // rows by output block count; LDS tables of twice it, or of four thirds of it for rows of
  // up to 24 blocks (the short rows of A T take 16-slot tables, 5 KB per 64-lane workgroup,
  // so that three times as many workgroups share a CU as with 64 slots), rows beyond 256
  // blocks in global memory (read back with the symbolic totals)
  DArr<int> lists((size_t)NBUCKET * n, s), counts(NBUCKET, s);
  int hc[NBUCKET] = {};
  SymBucket bk;
  bk.launch = [&](const int64_t *ubp) {
    fill<int>(counts.p, 0, NBUCKET, s);
    k_bucket_b3<<<grid_for(n, 256), 256, 0, s>>>(n, C.rp.p, A.rp.p, ubp, diagb ? 1 : 0, lists.p,
                                                  counts.p, n);
    KCHK();
  };
  bk.counts = counts.p;
  bk.host = hc;
  bk.nc = NBUCKET;
  spgemm_symbolic(n, A.rp.p, A.ci.p, A.nnzb, B.rp.p, B.ci.p, B.nb, B.mb, B.nnzb, C.rp.p, C.nnzb,
                  s, dflag, &ub, &bk);
  C.ci.alloc(std::max<int64_t>(C.nnzb, 1), s);
  C.v.alloc(std::max<int64_t>(9 * C.nnzb, 1), s);
  if (C.nnzb == 0) return;
  const int *lp = lists.p;
  const size_t N = (size_t)n;
  if (hc[0] > 0) launch_num_b3<16, 16>(diagb, hc[0], lp, A, B, C, dflag, s);
  if (hc[1] > 0) launch_num_b3<16, 32>(diagb, hc[1], lp + N, A, B, C, dflag, s);
  if (hc[2] > 0) launch_num_b3<16, 64>(diagb, hc[2], lp + 2 * N, A, B, C, dflag, s);
  if (hc[3] > 0) launch_num_b3<32, 128>(diagb, hc[3], lp + 3 * N, A, B, C, dflag, s);
  if (hc[4] > 0) launch_num_b3<64, 256>(diagb, hc[4], lp + 4 * N, A, B, C, dflag, s);
  if (hc[5] > 0) launch_num_b3<64, 512>(diagb, hc[5], lp + 5 * N, A, B, C, dflag, s);
  if (hc[B_WIDE] > 0) launch_num_b3<64, 16>(diagb, hc[B_WIDE], lp + 7 * N, A, B, C, dflag, s);
  if (hc[B_WIDE + 1] > 0) launch_num_b3<64, 32>(diagb, hc[B_WIDE + 1], lp + 8 * N, A, B, C, dflag, s);
  if (hc[B_WIDE + 2] > 0) launch_num_b3<64, 64>(diagb, hc[B_WIDE + 2], lp + 9 * N, A, B, C, dflag, s);
  if (hc[B_WIDE + 3] > 0) launch_num_b3<64, 128>(diagb, hc[B_WIDE + 3], lp + 10 * N, A, B, C, dflag, s);
  if (hc[B_GLOBAL] > 0) {
    const int nbig = hc[B_GLOBAL];
    const int *big = lists.p + (size_t)B_GLOBAL * n;
    DArr<int> mx(1, s);
    fill<int>(mx.p, 0, 1, s);
    k_max_len<<<grid_for(nbig, 256), 256, 0, s>>>(nbig, big, C.rp.p, mx.p);
    KCHK();
    const int hm = read_flag(mx.p, s);
    const int64_t ht = next_pow2(2 * (int64_t)hm);
    require(ht <= (int64_t)1 << 20, MGR_ERR_UNSUPPORTED,
            "block spgemm: a product row exceeds the supported length");
    const int64_t per = 2 * ht * 4 + 9 * ht * 8;
    const int64_t batch = std::max<int64_t>(1, ((int64_t)256 << 20) / per);
    const int64_t nb0 = std::min<int64_t>(batch, nbig);
    DArr<int> si(nb0 * 2 * ht, s);
    DArr<double> sd(nb0 * 9 * ht, s);
    for (int64_t b0 = 0; b0 < nbig; b0 += batch) {
      const int nb = (int)std::min<int64_t>(batch, nbig - b0);
      if (diagb)
        k_num_b3_global<true><<<nb, 64, 0, s>>>(nb, big + b0, (int)ht, A.rp.p, A.ci.p, A.v.p,
                                                B.rp.p, B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p,
                                                si.p, sd.p, dflag);
      else
        k_num_b3_global<false><<<nb, 64, 0, s>>>(nb, big + b0, (int)ht, A.rp.p, A.ci.p, A.v.p,
                                                 B.rp.p, B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p,
                                                 si.p, sd.p, dflag);
      KCHK();
    }
  }
}

}  // namespace mgr

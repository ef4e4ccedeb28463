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

constexpr int WG = 64;
constexpr int SYM_HT = 4096;       // LDS symbolic table size (int keys)
constexpr int NUM_HT_SMALL = 128;  // rows with <= 64 entries
constexpr int NUM_HT_MID = 1024;   // rows with <= 512 entries

__device__ __forceinline__ unsigned hslot(int key, unsigned mask) {
  return ((unsigned)key * 2654435761u) & mask;
}

__device__ __forceinline__ int next_pow2_dev(int64_t v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

__global__ void k_upper_bound(int64_t n, const int *__restrict__ arp, const int *__restrict__ aci,
                              const int *__restrict__ brp, int64_t *__restrict__ ub) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t s = 0;
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    int k = aci[e];
    s += brp[k + 1] - brp[k];
  }
  ub[i] = s;
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
// full, which the sizing rules out (tables hold at least twice the row's distinct count).
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

// Symbolic count of one row with a table of `ht` slots; returns -1 if more than 3/4 of the
// table would be needed.  All 64 lanes of the workgroup call it.
__device__ int sym_row(int row, const int *__restrict__ arp, const int *__restrict__ aci,
                       const int *__restrict__ brp, const int *__restrict__ bci, int *keys,
                       int ht, int *s_count, int *s_excl, int *s_start) {
  const int lane = threadIdx.x;
  const unsigned mask = (unsigned)ht - 1;
  for (int s = lane; s < ht; s += WG) keys[s] = -1;
  if (lane == 0) *s_count = 0;
  __syncthreads();
  const int limit = (ht / 4) * 3;
  const int as = arp[row], ae = arp[row + 1];
  bool over = false;
  for (int c0 = as; c0 < ae; c0 += WG) {
    // per chunk of 64 A entries: exclusive prefix of B row lengths
    int e = c0 + lane;
    int len = 0, st = 0;
    if (e < ae) {
      int k = aci[e];
      st = brp[k];
      len = brp[k + 1] - st;
    }
    int inc = len;
#pragma unroll
    for (int o = 1; o < WG; o <<= 1) {
      int t = __shfl_up(inc, o, WG);
      if (lane >= o) inc += t;
    }
    s_excl[lane] = inc - len;
    s_start[lane] = st;
    const int total = __shfl(inc, WG - 1, WG);
    __syncthreads();
    const int nent = min(WG, ae - c0);
    for (int p = lane; p < total; p += WG) {
      // entry t with s_excl[t] <= p < s_excl[t+1]
      int lo = 0, hi = nent - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s_excl[mid] <= p) lo = mid; else hi = mid - 1;
      }
      int j = bci[s_start[lo] + (p - s_excl[lo])];
      int r = table_insert(keys, mask, j);
      if (r == 1) {
        int c = atomicAdd(s_count, 1);
        if (c >= limit) over = true;
      } else if (r < 0) {
        over = true;
      }
    }
    __syncthreads();
    if (__syncthreads_or(over)) return -1;
  }
  __syncthreads();
  return *s_count;
}

__global__ void k_sym_lds(int64_t n, const int64_t *__restrict__ ub, const int *__restrict__ arp,
                          const int *__restrict__ aci, const int *__restrict__ brp,
                          const int *__restrict__ bci, int *__restrict__ cnt,
                          int *__restrict__ retry, int *__restrict__ nretry) {
  __shared__ int keys[SYM_HT];
  __shared__ int s_count, s_excl[WG], s_start[WG];
  const int row = blockIdx.x;
  if (row >= n) return;
  const int64_t u = ub[row];
  const int ht = u > SYM_HT / 2 ? SYM_HT : next_pow2_dev(u < 32 ? 64 : 2 * u);
  int c = sym_row(row, arp, aci, brp, bci, keys, ht, &s_count, s_excl, s_start);
  if (threadIdx.x == 0) {
    if (c < 0) {
      cnt[row] = 0;
      retry[atomicAdd(nretry, 1)] = row;
    } else {
      cnt[row] = c;
    }
  }
}

__global__ void k_sym_global(int nrows, const int *__restrict__ rows, int ht,
                             const int *__restrict__ arp, const int *__restrict__ aci,
                             const int *__restrict__ brp, const int *__restrict__ bci,
                             int *__restrict__ cnt, int *__restrict__ scratch,
                             int *__restrict__ flag) {
  __shared__ int s_count, s_excl[WG], s_start[WG];
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  int *keys = scratch + (int64_t)blockIdx.x * ht;
  int c = sym_row(row, arp, aci, brp, bci, keys, ht, &s_count, s_excl, s_start);
  if (threadIdx.x == 0) {
    if (c < 0) { atomicOr(flag, FLAG_ROW_TOO_LONG); cnt[row] = 0; }
    else cnt[row] = c;
  }
}

// Numeric phase for one row: keys/vals table of `ht` slots plus a compaction list of ht/2.
__device__ void num_row(int row, const int *__restrict__ arp, const int *__restrict__ aci,
                        const double *__restrict__ av, const int *__restrict__ brp,
                        const int *__restrict__ bci, const double *__restrict__ bv,
                        const int *__restrict__ crp, int *__restrict__ cci,
                        double *__restrict__ cv, int *keys, double *vals, int *lk, double *lv,
                        int ht, int *s_n, int *flag) {
  const int lane = threadIdx.x;
  const unsigned mask = (unsigned)ht - 1;
  for (int s = lane; s < ht; s += WG) {
    keys[s] = -1;
    vals[s] = 0.0;
  }
  if (lane == 0) *s_n = 0;
  __syncthreads();
  const int as = arp[row], ae = arp[row + 1];
  for (int e = as; e < ae; ++e) {          // ascending k: the pinned order
    const int k = aci[e];
    const double a = av[e];
    const int bs = brp[k], be = brp[k + 1];
    for (int q = bs + lane; q < be; q += WG) {
      const unsigned slot = table_find_or_insert(keys, mask, bci[q]);
      if (slot > mask) { atomicOr(flag, FLAG_PATTERN); continue; }
      vals[slot] = __dadd_rn(vals[slot], __dmul_rn(a, bv[q]));
    }
    __syncthreads();
  }
  for (int s = lane; s < ht; s += WG) {
    const int key = keys[s];
    if (key != -1) {
      const int t = atomicAdd(s_n, 1);
      if (t < ht / 2) {
        lk[t] = key;
        lv[t] = vals[s];
      }
    }
  }
  __syncthreads();
  const int m = *s_n;
  if (m > ht / 2) {
    if (lane == 0) atomicOr(flag, FLAG_PATTERN);
    return;
  }
  const int base = crp[row];
  if (lane == 0 && m != crp[row + 1] - base) atomicOr(flag, FLAG_PATTERN);
  if (m != crp[row + 1] - base) return;
  for (int t = lane; t < m; t += WG) {
    const int key = lk[t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += (lk[u] < key);
    cci[base + rank] = key;
    cv[base + rank] = lv[t];
  }
}

template <int HT>
__global__ void k_num_lds(int nrows, const int *__restrict__ rows, const int *__restrict__ arp,
                          const int *__restrict__ aci, const double *__restrict__ av,
                          const int *__restrict__ brp, const int *__restrict__ bci,
                          const double *__restrict__ bv, const int *__restrict__ crp,
                          int *__restrict__ cci, double *__restrict__ cv, int *flag) {
  __shared__ int keys[HT];
  __shared__ double vals[HT];
  __shared__ int lk[HT / 2];
  __shared__ double lv[HT / 2];
  __shared__ int s_n;
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  num_row(row, arp, aci, av, brp, bci, bv, crp, cci, cv, keys, vals, lk, lv, HT, &s_n, flag);
}

__global__ void k_num_global(int nrows, const int *__restrict__ rows, int ht,
                             const int *__restrict__ arp, const int *__restrict__ aci,
                             const double *__restrict__ av, const int *__restrict__ brp,
                             const int *__restrict__ bci, const double *__restrict__ bv,
                             const int *__restrict__ crp, int *__restrict__ cci,
                             double *__restrict__ cv, int *scratch_i, double *scratch_d,
                             int *flag) {
  __shared__ int s_n;
  if ((int)blockIdx.x >= nrows) return;
  const int row = rows[blockIdx.x];
  int *keys = scratch_i + (int64_t)blockIdx.x * (ht + ht / 2);
  int *lk = keys + ht;
  double *vals = scratch_d + (int64_t)blockIdx.x * (ht + ht / 2);
  double *lv = vals + ht;
  num_row(row, arp, aci, av, brp, bci, bv, crp, cci, cv, keys, vals, lk, lv, ht, &s_n, flag);
}

// rows by output length: bucket 0 (<= 64), 1 (<= 512), 2 (larger); empty rows skipped
__global__ void k_bucket(int64_t n, const int *__restrict__ crp, int *__restrict__ lists,
                         int *__restrict__ counts, int64_t stride) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int len = crp[i + 1] - crp[i];
  if (len == 0) return;
  int b = len <= NUM_HT_SMALL / 2 ? 0 : (len <= NUM_HT_MID / 2 ? 1 : 2);
  int pos = atomicAdd(&counts[b], 1);
  lists[b * stride + pos] = (int)i;
}

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

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace

void spgemm(const Csr &A, const Csr &B, Csr &C, hipStream_t s, int *dflag) {
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
  DArr<int64_t> ub(n, s);
  k_upper_bound<<<grid_for(n, 256), 256, 0, s>>>(n, A.rp.p, A.ci.p, B.rp.p, ub.p);
  KCHK();
  DArr<int> cnt(n + 1, s), retry(n, s), nretry(1, s);
  fill<int>(nretry.p, 0, 1, s);
  k_sym_lds<<<(unsigned)n, WG, 0, s>>>(n, ub.p, A.rp.p, A.ci.p, B.rp.p, B.ci.p, cnt.p, retry.p,
                                       nretry.p);
  KCHK();
  int hretry = 0;
  HIPCHK(hipMemcpyAsync(&hretry, nretry.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hretry > 0) {
    DArr<unsigned long long> mub(1, s);
    HIPCHK(hipMemsetAsync(mub.p, 0, sizeof(unsigned long long), s));
    k_max_ub<<<grid_for(hretry, 256), 256, 0, s>>>(hretry, retry.p, ub.p, mub.p);
    KCHK();
    unsigned long long hm = 0;
    HIPCHK(hipMemcpyAsync(&hm, mub.p, sizeof(hm), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t cap = std::min<int64_t>((int64_t)hm, B.m);
    int64_t ht = next_pow2(2 * std::max<int64_t>(cap, 32));
    require(ht <= (int64_t)1 << 22, MGR_ERR_UNSUPPORTED,
            "spgemm: a product row exceeds the supported length");
    int64_t batch = std::max<int64_t>(1, ((int64_t)64 << 20) / (ht * 4));
    DArr<int> scratch(std::min<int64_t>(batch, hretry) * ht, s);
    for (int64_t b0 = 0; b0 < hretry; b0 += batch) {
      int nb = (int)std::min<int64_t>(batch, hretry - b0);
      k_sym_global<<<nb, WG, 0, s>>>(nb, retry.p + b0, (int)ht, A.rp.p, A.ci.p, B.rp.p, B.ci.p,
                                     cnt.p, scratch.p, dflag);
      KCHK();
    }
  }
  C.nnz = exclusive_scan_i32(cnt.p, C.rp.p, n, s);
  require(read_flag(dflag, s) == 0, MGR_ERR_UNSUPPORTED, "spgemm: product row too long");
  C.ci.alloc(C.nnz, s);
  C.v.alloc(C.nnz, s);
  if (C.nnz == 0) return;
  // numeric phase by output row length
  DArr<int> lists(3 * n, s), counts(3, s);
  fill<int>(counts.p, 0, 3, s);
  k_bucket<<<grid_for(n, 256), 256, 0, s>>>(n, C.rp.p, lists.p, counts.p, n);
  KCHK();
  int hc[3];
  HIPCHK(hipMemcpyAsync(hc, counts.p, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hc[0] > 0) {
    k_num_lds<NUM_HT_SMALL><<<hc[0], WG, 0, s>>>(hc[0], lists.p, A.rp.p, A.ci.p, A.v.p, B.rp.p,
                                                B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p, dflag);
    KCHK();
  }
  if (hc[1] > 0) {
    k_num_lds<NUM_HT_MID><<<hc[1], WG, 0, s>>>(hc[1], lists.p + n, A.rp.p, A.ci.p, A.v.p, B.rp.p,
                                              B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p, dflag);
    KCHK();
  }
  if (hc[2] > 0) {
    DArr<int> mx(1, s);
    fill<int>(mx.p, 0, 1, s);
    k_max_len<<<grid_for(hc[2], 256), 256, 0, s>>>(hc[2], lists.p + 2 * n, C.rp.p, mx.p);
    KCHK();
    int hm = 0;
    HIPCHK(hipMemcpyAsync(&hm, mx.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t ht = next_pow2(2 * (int64_t)hm);
    require(ht <= (int64_t)1 << 22, MGR_ERR_UNSUPPORTED,
            "spgemm: a product row exceeds the supported length");
    int64_t per = ht + ht / 2;
    int64_t batch = std::max<int64_t>(1, ((int64_t)128 << 20) / (per * 12));
    int64_t nb0 = std::min<int64_t>(batch, hc[2]);
    DArr<int> si(nb0 * per, s);
    DArr<double> sd(nb0 * per, s);
    for (int64_t b0 = 0; b0 < hc[2]; b0 += batch) {
      int nb = (int)std::min<int64_t>(batch, hc[2] - b0);
      k_num_global<<<nb, WG, 0, s>>>(nb, lists.p + 2 * n + b0, (int)ht, A.rp.p, A.ci.p, A.v.p,
                                     B.rp.p, B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p, si.p, sd.p,
                                     dflag);
      KCHK();
    }
  }
  require(read_flag(dflag, s) == 0, MGR_ERR_HIP, "spgemm: numeric pattern mismatch");
}

}  // namespace mgr

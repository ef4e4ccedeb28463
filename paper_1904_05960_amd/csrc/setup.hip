// MGR setup kernels (Sec. 5.1-5.2): C/F split by label, extraction of A_FF, A_FC, A_CF,
// A_CC, Jacobi interpolation, the dropping operator G with the merge
// S = A_CC - G(A_CF D_FF^{-1} A_FC), transposition, and format conversions.
// Floating-point steps are single IEEE operations (no contraction), matching the
// summation and rounding order the setup is specified with.
#include "common.hpp"

namespace mgr {
namespace {

__device__ __forceinline__ uint64_t group_bits(bool p, int G) {
  uint64_t b = __ballot(p);
  if (G == 64) return b;
  const int lane = threadIdx.x & 63;
  const int base = lane & ~(G - 1);
  return (b >> base) & ((1ull << G) - 1);
}
__device__ __forceinline__ int lane_in_group(int G) { return threadIdx.x & (G - 1); }

// ---------------------------------------------------------------------------------
// C/F split
__global__ void k_cf_flags(const int8_t *__restrict__ lab, int64_t n, uint32_t fmask,
                           int *__restrict__ isF, int *flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int t = lab[i];
  if (t < 0 || t > 7) { atomicOr(flag, FLAG_BAD_LABEL); t = 0; }
  isF[i] = (fmask >> t) & 1u;
}
__global__ void k_cf_fill(int64_t n, const int *__restrict__ isF, const int *__restrict__ fpos,
                          int *__restrict__ F, int *__restrict__ C, int *__restrict__ map) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = fpos[i];
  if (isF[i]) { F[f] = (int)i; map[i] = f; }
  else { int c = (int)i - f; C[c] = (int)i; map[i] = -c - 1; }
}
__global__ void k_label_eq(const int8_t *__restrict__ lab, int64_t n, int t, int *__restrict__ fl) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) fl[i] = lab[i] == t;
}
__global__ void k_label_rank_set(const int8_t *__restrict__ lab, int64_t n, int t,
                                 const int *__restrict__ pos, int *__restrict__ rank) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && lab[i] == t) rank[i] = pos[i];
}
// bit t of *mask set when label t occurs; *bad set when a label lies outside [0, 7]
__global__ void k_label_mask(const int8_t *__restrict__ lab, int64_t n, unsigned *__restrict__ mask,
                             int *__restrict__ bad) {
  unsigned m = 0;
  int b = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int t = lab[i];
    if (t < 0 || t > 7) b = 1;
    else m |= 1u << t;
  }
  for (int o = 32; o > 0; o >>= 1) {
    m |= __shfl_xor(m, o, 64);
    b |= __shfl_xor(b, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (m) atomicOr(mask, m);
    if (b) atomicOr(bad, 1);
  }
}
// *bad set unless lab[i] == lab[i % p] for every i
__global__ void k_label_period(const int8_t *__restrict__ lab, int64_t n, int p,
                               int *__restrict__ bad) {
  int b = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (lab[i] != lab[i % p]) b = 1;
  if (b) atomicOr(bad, 1);
}
__global__ void k_gather_i8(const int8_t *__restrict__ a, const int *__restrict__ idx, int64_t n,
                            int8_t *__restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[idx[i]];
}

// ---------------------------------------------------------------------------------
// block extraction; G lanes per row
template <int G>
__global__ void k_extract_count(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                                const int *__restrict__ map, int *__restrict__ cFF,
                                int *__restrict__ cFC, int *__restrict__ cCF,
                                int *__restrict__ cCC) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = lane_in_group(G);
  if (row >= n) return;
  int nf = 0, nc = 0;
  for (int e = rp[row] + l; e < rp[row + 1]; e += G) {
    if (map[ci[e]] >= 0) ++nf; else ++nc;
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    nf += __shfl_xor(nf, o, G);
    nc += __shfl_xor(nc, o, G);
  }
  if (l == 0) {
    int r = map[row];
    if (r >= 0) { if (cFF) cFF[r] = nf; cFC[r] = nc; }
    else { cCF[-r - 1] = nf; cCC[-r - 1] = nc; }
  }
}

template <int G>
__global__ void k_extract_fill(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                               const double *__restrict__ v, const int *__restrict__ map,
                               const int *__restrict__ pFF, int *__restrict__ ciFF,
                               double *__restrict__ vFF, const int *__restrict__ pFC,
                               int *__restrict__ ciFC, double *__restrict__ vFC,
                               const int *__restrict__ pCF, int *__restrict__ ciCF,
                               double *__restrict__ vCF, const int *__restrict__ pCC,
                               int *__restrict__ ciCC, double *__restrict__ vCC,
                               double *__restrict__ dFF) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = lane_in_group(G);
  const bool active = row < n;
  const int r = active ? map[row] : 0;
  const bool isFrow = r >= 0;
  const int rr = isFrow ? r : -r - 1;
  int oF = 0, oC = 0;
  if (active) {
    if (isFrow) { oF = pFF ? pFF[rr] : 0; oC = pFC[rr]; }
    else { oF = pCF[rr]; oC = pCC[rr]; }
  }
  const int s = active ? rp[row] : 0, e = active ? rp[row + 1] : 0;
  const int len = e - s;
  // the group loops until its row is done; groups in one wave differ in trip count, so
  // ballots are taken by every lane of the wave in every round
  int maxlen = len;
  for (int o = 32; o > 0; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o, 64));
  for (int c0 = 0; c0 < maxlen; c0 += G) {
    const int q = c0 + l;
    const bool has = q < len;
    int col = 0, m = 0;
    double val = 0.0;
    if (has) { col = ci[s + q]; val = v[s + q]; m = map[col]; }
    const bool toF = has && m >= 0;
    const bool toC = has && m < 0;
    const uint64_t bF = group_bits(toF, G), bC = group_bits(toC, G);
    const uint64_t below = (1ull << l) - 1;
    const int pf = __popcll(bF & below), pc = __popcll(bC & below);
    if (toF) {
      if (isFrow) {
        if (ciFF) { ciFF[oF + pf] = m; vFF[oF + pf] = val; }
        if (m == rr) dFF[rr] = val;
      } else { ciCF[oF + pf] = m; vCF[oF + pf] = val; }
    } else if (toC) {
      if (isFrow) { ciFC[oC + pc] = -m - 1; vFC[oC + pc] = val; }
      else { ciCC[oC + pc] = -m - 1; vCC[oC + pc] = val; }
    }
    oF += __popcll(bF);
    oC += __popcll(bC);
  }
}

// 8 lanes per row
__global__ void k_scale_rows_div(int64_t n, const int *__restrict__ rp, double *__restrict__ v,
                                 const double *__restrict__ d) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 8;
  const int l = threadIdx.x & 7;
  if (i >= n) return;
  const double di = d[i];
  for (int e = rp[i] + l; e < rp[i + 1]; e += 8) v[e] = __ddiv_rn(v[e], di);
}

__global__ void k_check_nonzero(const double *__restrict__ d, int64_t n, int *flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !(d[i] != 0.0 && d[i] == d[i])) atomicOr(flag, FLAG_ZERO_PIVOT);
}

// ---------------------------------------------------------------------------------
// merge with dropping: S = A - diag(w) keep(B).
// keep flags (only when dropping): G lanes per row of B; an entry off the sub-block
// diagonals is kept when fewer than nmax other off-diagonal entries beat it (larger |b|,
// or equal |b| and a smaller column).  Rows of up to G * MAXCH entries are held in the
// lanes' registers (chunk c of lane l = entry c * G + l).  For nmax <= KTOP the lanes
// reduce their candidates to the row's KTOP best by a butterfly over sorted lists, and an
// entry is kept when it is among the first nmax of them: the same set as counting (the
// order is total, and an entry whose |b| is NaN beats none and is beaten by none, so it
// has rank 0); for larger nmax every entry counts the entries that beat it through
// shuffles.  Longer rows compare against global memory.
constexpr int KTOP = 4;
__device__ __forceinline__ bool drop_beats(double a, int ca, double b, int cb) {
  return a > b || (a == b && ca < cb);
}
// insert (v, c) into the sorted list (best first) of KTOP entries, dropping the last
__device__ __forceinline__ void top_insert(double (&tv)[KTOP], int (&tc)[KTOP], double v, int c) {
#pragma unroll
  for (int k = 0; k < KTOP; ++k) {
    if (drop_beats(v, c, tv[k], tc[k])) {
      const double sv = tv[k];
      const int sc = tc[k];
      tv[k] = v;
      tc[k] = c;
      v = sv;
      c = sc;
    }
  }
}
template <int G, int MAXCH>
__global__ void k_drop_keep(int64_t n, const int *__restrict__ brp, const int *__restrict__ bci,
                            const double *__restrict__ bv, int nmax,
                            const int *__restrict__ lrank, unsigned char *__restrict__ keep) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (row >= n) return;
  const int bs = brp[row], be = brp[row + 1];
  const int len = be - bs;
  const int myrank = lrank[row];
  if (len <= G * MAXCH) {
    const int nch = (len + G - 1) / G;
    double av[MAXCH];
    int cc[MAXCH], rk[MAXCH];
    bool el[MAXCH];
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
      const int t = bs + c * G + l;
      const bool in = c < nch && t < be;
      cc[c] = in ? bci[t] : 0x7fffffff;
      av[c] = in ? fabs(bv[t]) : 0.0;
      el[c] = in && lrank[cc[c]] != myrank;
      rk[c] = 0;
    }
    if (nmax <= KTOP) {
      // the lane's best KTOP candidates (|b| >= 0 > -1 marks an empty place), then the
      // row's by merging the lists of lane groups of 2, 4, ..., G
      double tv[KTOP];
      int tc[KTOP];
#pragma unroll
      for (int k = 0; k < KTOP; ++k) {
        tv[k] = -1.0;
        tc[k] = 0x7fffffff;
      }
#pragma unroll
      for (int c = 0; c < MAXCH; ++c)
        if (el[c] && av[c] == av[c]) top_insert(tv, tc, av[c], cc[c]);
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) {
        double ov[KTOP];
        int oc[KTOP];
#pragma unroll
        for (int k = 0; k < KTOP; ++k) {
          ov[k] = __shfl_xor(tv[k], o, G);
          oc[k] = __shfl_xor(tc[k], o, G);
        }
#pragma unroll
        for (int k = 0; k < KTOP; ++k) top_insert(tv, tc, ov[k], oc[k]);
      }
      // the nmax-th best (when the row has that many candidates) is the last one kept
      const bool all = nmax > 0 && tv[nmax - 1] < 0.0;
      const double thv = nmax > 0 ? tv[nmax - 1] : 0.0;
      const int thc = nmax > 0 ? tc[nmax - 1] : 0;
#pragma unroll
      for (int c = 0; c < MAXCH; ++c) {
        const int t = bs + c * G + l;
        if (c < nch && t < be) {
          const bool nan = !(av[c] == av[c]);
          const bool top = nmax > 0 && (all || nan || !drop_beats(thv, thc, av[c], cc[c]));
          keep[t] = !el[c] || top;
        }
      }
      return;
    }
#pragma unroll
    for (int c2 = 0; c2 < MAXCH; ++c2) {
      if (c2 >= nch) break;
      for (int j = 0; j < G; ++j) {
        const double au = __shfl(av[c2], j, G);
        const int cu = __shfl(cc[c2], j, G);
        const bool eu = __shfl((int)el[c2], j, G) != 0;
        if (!eu) continue;
#pragma unroll
        for (int c1 = 0; c1 < MAXCH; ++c1)
          rk[c1] += (au > av[c1]) || (au == av[c1] && cu < cc[c1]);
      }
    }
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
      const int t = bs + c * G + l;
      if (c < nch && t < be) keep[t] = !el[c] || rk[c] < nmax;
    }
    return;
  }
  for (int t = bs + l; t < be; t += G) {
    const int ct = bci[t];
    bool k = true;
    if (lrank[ct] != myrank) {
      const double at = fabs(bv[t]);
      int rk = 0;
      for (int u = bs; u < be && rk < nmax; ++u) {
        const int cu = bci[u];
        if (lrank[cu] == myrank) continue;
        const double au = fabs(bv[u]);
        rk += (au > at) || (au == at && cu < ct);
      }
      k = rk < nmax;
    }
    keep[t] = k;
  }
}

// keep flags of the tolerance form of G: G lanes per row take the largest |b| of the row
// (a maximum, exact in any order), then an entry is kept when it lies on a sub-block
// diagonal, or is nonzero with |b| >= tol * max
template <int G>
__global__ void k_drop_tol(int64_t n, const int *__restrict__ brp, const int *__restrict__ bci,
                           const double *__restrict__ bv, double tol,
                           const int *__restrict__ lrank, unsigned char *__restrict__ keep) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (row >= n) return;
  const int bs = brp[row], be = brp[row + 1];
  double mx = 0.0;
  for (int t = bs + l; t < be; t += G) mx = fmax(mx, fabs(bv[t]));
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, G));
  const double thr = __dmul_rn(tol, mx);
  const int myrank = lrank[row];
  for (int t = bs + l; t < be; t += G) {
    const double a = fabs(bv[t]);
    keep[t] = lrank[bci[t]] == myrank || (a > 0.0 && a >= thr);
  }
}

// Merge of row `row` of A with the kept entries of row `row` of B (S = A - w B, see
// merge_drop); MODE 0 counts, MODE 1 writes columns (and values when sv != null).
// Two-pointer form, for rows longer than the LDS staging below.
template <int MODE>
__device__ void merge_row_serial(int64_t row, const int *__restrict__ arp,
                                 const int *__restrict__ aci, const double *__restrict__ av,
                                 const int *__restrict__ brp, const int *__restrict__ bci,
                                 const double *__restrict__ bv,
                                 const unsigned char *__restrict__ keep,
                                 const double *__restrict__ w, int *__restrict__ cnt,
                                 const int *__restrict__ srp, int *__restrict__ sci,
                                 double *__restrict__ sv) {
  int pa = arp ? arp[row] : 0;
  const int ea = arp ? arp[row + 1] : 0;
  int pb = brp[row];
  const int eb = brp[row + 1];
  const double wr = w ? w[row] : 1.0;
  int o = MODE ? srp[row] : 0;
  int c = 0;
  for (;;) {
    while (pb < eb && keep && !keep[pb]) ++pb;
    const bool ha = pa < ea, hb = pb < eb;
    if (!ha && !hb) break;
    const int ca = ha ? aci[pa] : 0x7fffffff;
    const int cb = hb ? bci[pb] : 0x7fffffff;
    if (MODE) {
      if (ca < cb) {
        sci[o] = ca;
        if (sv) sv[o] = av[pa];
      } else {
        const double b = w ? __dmul_rn(wr, bv[pb]) : bv[pb];
        sci[o] = cb;
        if (sv) sv[o] = (ca == cb) ? __dsub_rn(av[pa], b) : -b;
      }
      ++o;
    } else {
      ++c;
    }
    if (ca < cb) ++pa;
    else if (cb < ca) ++pb;
    else { ++pa; ++pb; }
  }
  if (!MODE) cnt[row] = c;
}

// The same merge by G lanes per row with both rows staged in LDS (up to 128 entries each:
// 25 KB per 256-thread workgroup for 16 lanes per row, 12.5 KB for 32, so that a CU holds
// its full 32 wavefronts of the 32-lane form).
// An entry's output position is its rank in the union: an entry of A is preceded by the
// entries of A before it and by the entries of B that are kept, not in A and of smaller
// column; a kept entry of B that is not in A, by the entries of A of smaller column and
// those entries of B before it (ob: prefix count over B).  The values are formed exactly as
// in the two-pointer form.
template <int MODE, int G>
__global__ void __launch_bounds__(256) k_merge_rows(int64_t n, const int *__restrict__ arp,
                                                    const int *__restrict__ aci,
                                                    const double *__restrict__ av,
                                                    const int *__restrict__ brp,
                                                    const int *__restrict__ bci,
                                                    const double *__restrict__ bv,
                                                    const unsigned char *__restrict__ keep,
                                                    const double *__restrict__ w,
                                                    int *__restrict__ cnt,
                                                    const int *__restrict__ srp,
                                                    int *__restrict__ sci,
                                                    double *__restrict__ sv) {
  constexpr int RPB = 256 / G, MCAP = 128;
  __shared__ int s_a[RPB][MCAP], s_b[RPB][MCAP], s_ob[RPB][MCAP + 1];
  const int g = threadIdx.x / G, l = threadIdx.x & (G - 1);
  const int64_t row = blockIdx.x * (int64_t)RPB + g;
  if (row >= n) return;   // whole groups leave; the groups never wait for each other
  const int a0 = arp ? arp[row] : 0, la = arp ? arp[row + 1] - a0 : 0;
  const int b0 = brp[row], lb = brp[row + 1] - b0;
  if (la > MCAP || lb > MCAP) {
    if (l == 0)
      merge_row_serial<MODE>(row, arp, aci, av, brp, bci, bv, keep, w, cnt, srp, sci, sv);
    return;
  }
  int *sa = s_a[g], *sb = s_b[g], *ob = s_ob[g];
  for (int t = l; t < la; t += G) sa[t] = aci[a0 + t];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // columns of B, and ob[t] = number of kept entries of B before t whose column is not in A
  int carry = 0;
  for (int t0 = 0; t0 < lb; t0 += G) {
    const int t = t0 + l;
    int only = 0;
    if (t < lb) {
      const int cb = bci[b0 + t];
      sb[t] = cb;
      if (!keep || keep[b0 + t]) {
        int lo = 0, hi = la;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sa[mid] < cb) lo = mid + 1; else hi = mid;
        }
        only = !(lo < la && sa[lo] == cb);
      }
    }
    int inc = only;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int y = __shfl_up(inc, o, G);
      if (l >= o) inc += y;
    }
    if (t < lb) ob[t] = carry + inc - only;
    carry += __shfl(inc, G - 1, G);
  }
  if (l == 0) ob[lb] = carry;
  if (!MODE) {
    if (l == 0) cnt[row] = la + carry;
    return;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double wr = w ? w[row] : 1.0;
  const int obase = srp[row];
  for (int t = l; t < la; t += G) {
    const int ca = sa[t];
    int lo = 0, hi = lb;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sb[mid] < ca) lo = mid + 1; else hi = mid;
    }
    const int pos = obase + t + ob[lo];
    sci[pos] = ca;
    if (sv) {
      if (lo < lb && sb[lo] == ca && (!keep || keep[b0 + lo])) {
        const double b = w ? __dmul_rn(wr, bv[b0 + lo]) : bv[b0 + lo];
        sv[pos] = __dsub_rn(av[a0 + t], b);
      } else {
        sv[pos] = av[a0 + t];
      }
    }
  }
  for (int t = l; t < lb; t += G) {
    if (ob[t + 1] == ob[t]) continue;   // dropped, or merged into an entry of A
    const int cb = sb[t];
    int lo = 0, hi = la;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sa[mid] < cb) lo = mid + 1; else hi = mid;
    }
    const int pos = obase + lo + ob[t];
    sci[pos] = cb;
    if (sv) sv[pos] = -(w ? __dmul_rn(wr, bv[b0 + t]) : bv[b0 + t]);
  }
}

// ---------------------------------------------------------------------------------
// transpose: column counts, scatter, per-row ordering by source row
__global__ void k_col_count(int64_t nnz, const int *__restrict__ ci, int *__restrict__ cnt) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}
// 16 lanes per source row; the order of the entries within a row of the transpose is
// fixed afterwards by k_rank_sort_rows
__global__ void k_transpose_scatter(int64_t n, const int *__restrict__ rp,
                                    const int *__restrict__ ci, const double *__restrict__ v,
                                    const int *__restrict__ trp, int *__restrict__ fillpos,
                                    int *__restrict__ tmp_r, double *__restrict__ tmp_v) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 16;
  const int l = threadIdx.x & 15;
  if (i >= n) return;
  for (int e = rp[i] + l; e < rp[i + 1]; e += 16) {
    const int c = ci[e];
    const int pos = trp[c] + atomicAdd(&fillpos[c], 1);
    tmp_r[pos] = (int)i;
    if (tmp_v) tmp_v[pos] = v[e];
  }
}
// keys are unique within a row: the output position of an entry is its rank.  One
// wavefront per row; rows of up to RS_LDS keys are compared from LDS.
constexpr int RS_LDS = 2048;
__global__ void __launch_bounds__(64) k_rank_sort_rows(int64_t n, const int *__restrict__ rp,
                                                       const int *__restrict__ tk,
                                                       const double *__restrict__ tv,
                                                       int *__restrict__ ok,
                                                       double *__restrict__ ov) {
  __shared__ int sk[RS_LDS];
  const int64_t row = blockIdx.x;
  if (row >= n) return;
  const int s = rp[row], m = rp[row + 1] - s;
  if (m <= RS_LDS) {
    for (int t = threadIdx.x; t < m; t += 64) sk[t] = tk[s + t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int t = threadIdx.x; t < m; t += 64) {
      const int key = sk[t];
      int rank = 0;
      for (int u = 0; u < m; ++u) rank += sk[u] < key;
      ok[s + rank] = key;
      if (tv) ov[s + rank] = tv[s + t];
    }
    return;
  }
  for (int t = threadIdx.x; t < m; t += 64) {
    const int key = tk[s + t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += tk[s + u] < key;
    ok[s + rank] = key;
    if (tv) ov[s + rank] = tv[s + t];
  }
}

// ---------------------------------------------------------------------------------
// 16 lanes per row; the lane that holds the diagonal entry hands it to the others
__global__ void k_diag(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                       const double *__restrict__ v, double *__restrict__ d) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 16;
  const int l = threadIdx.x & 15;
  if (i >= n) return;
  double x = 0.0;
  int found = 0;
  for (int e = rp[i] + l; e < rp[i + 1]; e += 16)
    if (ci[e] == i) {
      x = v[e];
      found = 1;
    }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    const double ox = __shfl_xor(x, o, 16);
    const int of = __shfl_xor(found, o, 16);
    if (of && !found) {
      x = ox;
      found = 1;
    }
  }
  if (l == 0) d[i] = x;
}
// rs_i / |a_ii| with rs_i summed in ascending column order
__global__ void k_gershgorin(int64_t n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ v, double *__restrict__ q, int *flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double rs = 0.0, d = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    rs = __dadd_rn(rs, fabs(v[e]));
    if (ci[e] == i) d = v[e];
  }
  if (d == 0.0) { atomicOr(flag, FLAG_ZERO_PIVOT); q[i] = 0.0; return; }
  q[i] = __ddiv_rn(rs, fabs(d));
}
// per row, one pass in ascending column order: the diagonal d_i, 1 / sum_j |a_ij| (the l1
// smoother) and the Gershgorin ratio sum_j |a_ij| / |a_ii|
// G lanes per row load the row coalesced, G entries at a time, into LDS; the first lane of
// the group then adds them in ascending column order (the order of the sum is the row's,
// not the lanes').
template <int G>
__global__ void __launch_bounds__(256) k_row_stats(int64_t n, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const double *__restrict__ v,
                                                   double *__restrict__ d,
                                                   double *__restrict__ q,
                                                   double *__restrict__ l1inv, int *flag) {
  __shared__ double s_abs[256];
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  const int base = threadIdx.x - l;
  if (i >= n) return;   // whole groups leave; the groups never wait for each other
  double rs = 0.0, di = 0.0;
  int found = 0;
  const int e0 = rp[i], e1 = rp[i + 1];
  for (int c0 = e0; c0 < e1; c0 += G) {
    const int e = c0 + l;
    double x = 0.0;
    if (e < e1) {
      x = v[e];
      if (ci[e] == (int)i) {
        di = x;
        found = 1;
      }
    }
    s_abs[threadIdx.x] = fabs(x);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (l == 0) {
      const int cnt = min(G, e1 - c0);
      for (int t = 0; t < cnt; ++t) rs = __dadd_rn(rs, s_abs[base + t]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // the diagonal from the lane that held it
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const double od = __shfl_xor(di, o, G);
    const int of = __shfl_xor(found, o, G);
    if (of && !found) {
      di = od;
      found = 1;
    }
  }
  if (l != 0) return;
  d[i] = di;
  l1inv[i] = rs != 0.0 ? 1.0 / rs : 0.0;
  if (di == 0.0) {
    atomicOr(flag, FLAG_ZERO_PIVOT);
    q[i] = 0.0;
  } else {
    q[i] = __ddiv_rn(rs, fabs(di));
  }
}
__global__ void k_l1_inv(int64_t n, const int *__restrict__ rp, const double *__restrict__ v,
                         double *__restrict__ dinv) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double rs = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) rs = __dadd_rn(rs, fabs(v[e]));
  dinv[i] = rs != 0.0 ? 1.0 / rs : 0.0;
}
__global__ void k_omega_over(const double *__restrict__ d, double omega, double *__restrict__ w,
                             int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) w[i] = __ddiv_rn(omega, d[i]);
}

// ---------------------------------------------------------------------------------
// scalar CSR with full 3x3 blocks -> BSR3; G lanes per node, lanes over blocks
template <int G>
__global__ void k_bsr3_count(int64_t nb, const int *__restrict__ rp, const int *__restrict__ ci,
                             int *__restrict__ cnt, int *flag, int *first_bad) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (I >= nb) return;
  const int s0 = rp[3 * I], s1 = rp[3 * I + 1], s2 = rp[3 * I + 2], s3 = rp[3 * I + 3];
  const int L = s1 - s0;
  bool ok = (L % 3 == 0) && (s2 - s1 == L) && (s3 - s2 == L);
  if (ok) {
    for (int q = 3 * l; q < L && ok; q += 3 * G) {
      const int c = ci[s0 + q];
      ok = (c % 3 == 0) && ci[s0 + q + 1] == c + 1 && ci[s0 + q + 2] == c + 2 &&
           ci[s1 + q] == c && ci[s1 + q + 1] == c + 1 && ci[s1 + q + 2] == c + 2 &&
           ci[s2 + q] == c && ci[s2 + q + 1] == c + 1 && ci[s2 + q + 2] == c + 2;
    }
  }
  // group AND
  int bad = !ok;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, G);
  if (l == 0) {
    if (bad) {
      atomicOr(flag, FLAG_NOT_BLOCKED);
      atomicMin(first_bad, (int)I);
    }
    cnt[I] = bad ? 0 : L / 3;
  }
}
template <int G>
__global__ void k_bsr3_fill(int64_t nb, const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ v, const int *__restrict__ brp,
                            int *__restrict__ bci, double *__restrict__ bv) {
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (I >= nb) return;
  const int b0 = brp[I], nbk = brp[I + 1] - b0;
  const int r0 = rp[3 * I], r1 = rp[3 * I + 1], r2 = rp[3 * I + 2];
  for (int q = l; q < nbk; q += G) {
    const int blk = b0 + q;
    bci[blk] = ci[r0 + 3 * q] / 3;
    double *o = bv + 9 * (int64_t)blk;
    o[0] = v[r0 + 3 * q]; o[1] = v[r0 + 3 * q + 1]; o[2] = v[r0 + 3 * q + 2];
    o[3] = v[r1 + 3 * q]; o[4] = v[r1 + 3 * q + 1]; o[5] = v[r1 + 3 * q + 2];
    o[6] = v[r2 + 3 * q]; o[7] = v[r2 + 3 * q + 1]; o[8] = v[r2 + 3 * q + 2];
  }
}

// inverses of consecutive nb x nb diagonal blocks (nb = 2 or 3), row-major
__global__ void k_block_inv(int64_t nblk, int nb, const int *__restrict__ rp,
                            const int *__restrict__ ci, const double *__restrict__ v,
                            double *__restrict__ inv, int *flag) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nblk) return;
  double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int r0 = (int)(e * nb);
  for (int r = 0; r < nb; ++r)
    for (int q = rp[r0 + r]; q < rp[r0 + r + 1]; ++q) {
      const int c = ci[q] - r0;
      if (c >= 0 && c < nb) B[r * nb + c] = v[q];
    }
  double *o = inv + (int64_t)e * nb * nb;
  if (nb == 2) {
    const double det = B[0] * B[3] - B[1] * B[2];
    if (det == 0.0 || det != det) { atomicOr(flag, FLAG_ZERO_PIVOT); return; }
    o[0] = B[3] / det; o[1] = -B[1] / det; o[2] = -B[2] / det; o[3] = B[0] / det;
  } else {
    const double c00 = B[4] * B[8] - B[5] * B[7], c01 = B[5] * B[6] - B[3] * B[8],
                 c02 = B[3] * B[7] - B[4] * B[6];
    const double det = B[0] * c00 + B[1] * c01 + B[2] * c02;
    if (det == 0.0 || det != det) { atomicOr(flag, FLAG_ZERO_PIVOT); return; }
    o[0] = c00 / det;
    o[1] = (B[2] * B[7] - B[1] * B[8]) / det;
    o[2] = (B[1] * B[5] - B[2] * B[4]) / det;
    o[3] = c01 / det;
    o[4] = (B[0] * B[8] - B[2] * B[6]) / det;
    o[5] = (B[2] * B[3] - B[0] * B[5]) / det;
    o[6] = c02 / det;
    o[7] = (B[1] * B[6] - B[0] * B[7]) / det;
    o[8] = (B[0] * B[4] - B[1] * B[3]) / det;
  }
}

// Pattern fingerprint (detects a changed pattern when values are updated): the sum over
// i of two 32-bit finalizer mixes (the MurmurHash3 fmix32 steps) of (a[i], i), one per
// half of a 64-bit word.  32-bit arithmetic only; sums in any order are equal.
__device__ __forceinline__ uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ unsigned long long hash_pair(uint32_t v, uint32_t i, uint32_t salt) {
  const uint32_t lo = fmix32(v ^ fmix32(i ^ salt));
  const uint32_t hi = fmix32(v + 0x9e3779b9u * (i + 1u) + salt);
  return ((unsigned long long)hi << 32) | lo;
}
// per-block partial sums (no atomics), then one block adds them to *out
__global__ void __launch_bounds__(256) k_hash(int64_t n, const int *__restrict__ a,
                                              unsigned long long salt,
                                              unsigned long long *__restrict__ part) {
  __shared__ unsigned long long sw[4];
  unsigned long long acc = 0;
  const uint32_t s32 = (uint32_t)salt;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += hash_pair((uint32_t)a[i], (uint32_t)i, s32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}
__global__ void __launch_bounds__(256) k_hash_sum(const unsigned long long *__restrict__ part,
                                                  int np, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long sw[4];
  unsigned long long acc = 0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out += (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

}  // namespace

// ===================================================================================
void cf_split(const int8_t *labels, int64_t n, uint32_t fmask, CfSplit &cf, hipStream_t s,
              int *dflag) {
  cf.n = n;
  DArr<int> isF(n, s), fpos(n + 1, s);
  k_cf_flags<<<grid_for(n, 256), 256, 0, s>>>(labels, n, fmask, isF.p, dflag);
  KCHK();
  cf.nF = exclusive_scan_i32(isF.p, fpos.p, n, s);
  cf.nC = n - cf.nF;
  check_flags(dflag, s, "C/F split");
  require(cf.nF > 0 && cf.nC > 0, MGR_ERR_ARG, "a reduction level has an empty F or C set");
  cf.F.alloc(cf.nF, s);
  cf.C.alloc(cf.nC, s);
  cf.map.alloc(n, s);
  k_cf_fill<<<grid_for(n, 256), 256, 0, s>>>(n, isF.p, fpos.p, cf.F.p, cf.C.p, cf.map.p);
  KCHK();
}

uint32_t label_mask(const int8_t *labels, int64_t n, hipStream_t s) {
  DArr<int> buf(2, s);
  fill<int>(buf.p, 0, 2, s);
  if (n > 0) {
    k_label_mask<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(
        labels, n, reinterpret_cast<unsigned *>(buf.p), buf.p + 1);
    KCHK();
  }
  int h[2];
  d2h_sync(h, buf.p, sizeof(h), s);
  require(h[1] == 0, MGR_ERR_ARG, "labels must lie in [0, 7]");
  return (uint32_t)h[0];
}

bool labels_periodic(const int8_t *labels, int64_t n, int p, hipStream_t s) {
  DArr<int> bad(1, s);
  fill<int>(bad.p, 0, 1, s);
  if (n > 0) {
    k_label_period<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(labels, n, p, bad.p);
    KCHK();
  }
  return read_flag(bad.p, s) == 0;
}

void label_rank(const int8_t *labels, int64_t n, DArr<int> &rank, hipStream_t s,
                uint32_t present) {
  rank.alloc(n, s);
  DArr<int> fl(n, s), pos(n + 1, s);
  for (int t = 0; t < 8; ++t) {
    if (!((present >> t) & 1u)) continue;
    k_label_eq<<<grid_for(n, 256), 256, 0, s>>>(labels, n, t, fl.p);
    KCHK();
    if (exclusive_scan_i32(fl.p, pos.p, n, s) == 0) continue;
    k_label_rank_set<<<grid_for(n, 256), 256, 0, s>>>(labels, n, t, pos.p, rank.p);
    KCHK();
  }
}

void gather_labels(const int8_t *labels, const int *idx, int64_t n, int8_t *out, hipStream_t s) {
  if (n <= 0) return;
  k_gather_i8<<<grid_for(n, 256), 256, 0, s>>>(labels, idx, n, out);
  KCHK();
}

void extract_blocks(const Csr &A, const CfSplit &cf, Csr *Aff, Csr &Afc, Csr &Acf, Csr &Acc,
                    double *dFF, hipStream_t s) {
  const int64_t n = A.n, nF = cf.nF, nC = cf.nC;
  constexpr int G = 16;
  DArr<int> cFF, cFC(nF + 1, s), cCF(nC + 1, s), cCC(nC + 1, s);
  if (Aff) cFF.alloc(nF + 1, s);
  k_extract_count<G><<<grid_for(n * G, 256), 256, 0, s>>>(n, A.rp.p, A.ci.p, cf.map.p, cFF.p,
                                                         cFC.p, cCF.p, cCC.p);
  KCHK();
  auto finish = [&](Csr &M, DArr<int> &cnt, int64_t rows, int64_t cols) {
    M.n = rows;
    M.m = cols;
    M.rp.alloc(rows + 1, s);
    M.nnz = exclusive_scan_i32(cnt.p, M.rp.p, rows, s);
    M.ci.alloc(M.nnz, s);
    M.v.alloc(M.nnz, s);
  };
  if (Aff) finish(*Aff, cFF, nF, nF);
  finish(Afc, cFC, nF, nC);
  finish(Acf, cCF, nC, nF);
  finish(Acc, cCC, nC, nC);
  fill<double>(dFF, 0.0, nF, s);
  k_extract_fill<G><<<grid_for(n * G, 256), 256, 0, s>>>(
      n, A.rp.p, A.ci.p, A.v.p, cf.map.p, Aff ? Aff->rp.p : nullptr, Aff ? Aff->ci.p : nullptr,
      Aff ? Aff->v.p : nullptr, Afc.rp.p, Afc.ci.p, Afc.v.p, Acf.rp.p, Acf.ci.p, Acf.v.p,
      Acc.rp.p, Acc.ci.p, Acc.v.p, dFF);
  KCHK();
}

// ---- same-entity filter of A_CF (quasi-IMPES coupling) ----------------------------
namespace {
__global__ void k_same_entity_count(int64_t n, const int *__restrict__ rp,
                                    const int *__restrict__ ci, const int *__restrict__ C,
                                    const int *__restrict__ F, const int *__restrict__ rank,
                                    int *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ri = rank[C[i]];
  int c = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) c += rank[F[ci[e]]] == ri;
  cnt[i] = c;
}
__global__ void k_same_entity_fill(int64_t n, const int *__restrict__ rp,
                                   const int *__restrict__ ci, const double *__restrict__ v,
                                   const int *__restrict__ C, const int *__restrict__ F,
                                   const int *__restrict__ rank, const int *__restrict__ orp,
                                   int *__restrict__ oci, double *__restrict__ ov) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ri = rank[C[i]];
  int o = orp[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    if (rank[F[ci[e]]] != ri) continue;
    oci[o] = ci[e];
    ov[o] = v[e];
    ++o;
  }
}
}  // namespace

void same_entity_filter(const Csr &Acf, const int *C, const int *F, const int *rank, Csr &out,
                        hipStream_t s) {
  out.n = Acf.n;
  out.m = Acf.m;
  out.rp.alloc(Acf.n + 1, s);
  DArr<int> cnt(std::max<int64_t>(Acf.n, 1), s);
  if (Acf.n) {
    k_same_entity_count<<<grid_for(Acf.n, 256), 256, 0, s>>>(Acf.n, Acf.rp.p, Acf.ci.p, C, F,
                                                              rank, cnt.p);
    KCHK();
  }
  out.nnz = exclusive_scan_i32(cnt.p, out.rp.p, Acf.n, s);
  out.ci.alloc(std::max<int64_t>(out.nnz, 1), s);
  out.v.alloc(std::max<int64_t>(out.nnz, 1), s);
  if (Acf.n) {
    k_same_entity_fill<<<grid_for(Acf.n, 256), 256, 0, s>>>(Acf.n, Acf.rp.p, Acf.ci.p, Acf.v.p, C,
                                                             F, rank, out.rp.p, out.ci.p, out.v.p);
    KCHK();
  }
}

void scale_rows_div(Csr &M, const double *d, hipStream_t s) {
  if (M.n == 0) return;
  k_scale_rows_div<<<grid_for(M.n * 8, 256), 256, 0, s>>>(M.n, M.rp.p, M.v.p, d);
  KCHK();
}

void check_nonzero(const double *d, int64_t n, int *dflag, hipStream_t s) {
  if (n == 0) return;
  k_check_nonzero<<<grid_for(n, 256), 256, 0, s>>>(d, n, dflag);
  KCHK();
}

void merge_drop(const Csr &A, const Csr &B, const double *w, int nmax, const int *lrank, Csr &S,
                bool values, hipStream_t s, int *dflag, double tol) {
  (void)dflag;
  const int64_t n = B.n;
  S.n = n;
  S.m = B.m;
  S.rp.alloc(n + 1, s);
  DArr<int> cnt(n + 1, s);
  DArr<unsigned char> keep;
  if (tol >= 0.0 && B.nnz > 0) {
    require(lrank != nullptr, MGR_ERR_ARG, "dropping needs per-label ranks");
    keep.alloc(B.nnz, s);
    constexpr int G = 16;
    k_drop_tol<G><<<grid_for(n * G, 256), 256, 0, s>>>(n, B.rp.p, B.ci.p, B.v.p, tol, lrank,
                                                       keep.p);
    KCHK();
  } else if (nmax >= 0 && B.nnz > 0) {
    require(lrank != nullptr, MGR_ERR_ARG, "dropping needs per-label ranks");
    keep.alloc(B.nnz, s);
    constexpr int G = 16;
    k_drop_keep<G, 8><<<grid_for(n * G, 256), 256, 0, s>>>(n, B.rp.p, B.ci.p, B.v.p, nmax, lrank,
                                                           keep.p);
    KCHK();
  }
  const int *arp = A.n ? A.rp.p : nullptr;
  const unsigned char *kp = keep.p;
  // 16 lanes per row for short rows, 32 for longer ones
  const bool wide = n > 0 && (double)(A.nnz + B.nnz) > 24.0 * (double)n;
#define MERGE(MODE, G, ...)                                                           \
  k_merge_rows<MODE, G><<<(unsigned)((n + 256 / G - 1) / (256 / G)), 256, 0, s>>>(__VA_ARGS__)
  if (n > 0) {
    if (wide)
      MERGE(0, 32, n, arp, A.ci.p, nullptr, B.rp.p, B.ci.p, nullptr, kp, nullptr, cnt.p, nullptr,
            nullptr, nullptr);
    else
      MERGE(0, 16, n, arp, A.ci.p, nullptr, B.rp.p, B.ci.p, nullptr, kp, nullptr, cnt.p, nullptr,
            nullptr, nullptr);
    KCHK();
  }
  S.nnz = exclusive_scan_i32(cnt.p, S.rp.p, n, s);
  S.ci.alloc(S.nnz, s);
  if (values) S.v.alloc(S.nnz, s);
  if (n > 0) {
    if (wide)
      MERGE(1, 32, n, arp, A.ci.p, values ? A.v.p : nullptr, B.rp.p, B.ci.p,
            values ? B.v.p : nullptr, kp, w, nullptr, S.rp.p, S.ci.p, values ? S.v.p : nullptr);
    else
      MERGE(1, 16, n, arp, A.ci.p, values ? A.v.p : nullptr, B.rp.p, B.ci.p,
            values ? B.v.p : nullptr, kp, w, nullptr, S.rp.p, S.ci.p, values ? S.v.p : nullptr);
    KCHK();
  }
#undef MERGE
}

void drop_only(const Csr &B, int nmax, const int *lrank, Csr &G, hipStream_t s, int *dflag,
               double tol) {
  Csr empty;
  merge_drop(empty, B, nullptr, nmax, lrank, G, true, s, dflag, tol);
  negate_f64(G.v.p, G.nnz, s);
}

void transpose(const Csr &A, Csr &T, bool values, hipStream_t s) {
  T.n = A.m;
  T.m = A.n;
  T.nnz = A.nnz;
  T.rp.alloc(T.n + 1, s);
  DArr<int> cnt(T.n + 1, s), fillpos(T.n, s);
  fill<int>(cnt.p, 0, T.n + 1, s);
  fill<int>(fillpos.p, 0, T.n, s);
  if (A.nnz) {
    k_col_count<<<grid_for(A.nnz, 256), 256, 0, s>>>(A.nnz, A.ci.p, cnt.p);
    KCHK();
  }
  exclusive_scan_i32_async(cnt.p, T.rp.p, T.n, s);   // the total is A.nnz
  T.ci.alloc(T.nnz, s);
  if (values) T.v.alloc(T.nnz, s);
  if (A.nnz == 0) return;
  DArr<int> tr(A.nnz, s);
  DArr<double> tv;
  if (values) tv.alloc(A.nnz, s);
  k_transpose_scatter<<<grid_for(A.n * 16, 256), 256, 0, s>>>(A.n, A.rp.p, A.ci.p, A.v.p, T.rp.p,
                                                         fillpos.p, tr.p, values ? tv.p : nullptr);
  KCHK();
  k_rank_sort_rows<<<(unsigned)T.n, 64, 0, s>>>(T.n, T.rp.p, tr.p, values ? tv.p : nullptr,
                                                T.ci.p, values ? T.v.p : nullptr);
  KCHK();
}

void diag_of(const Csr &A, double *d, hipStream_t s) {
  if (A.n == 0) return;
  k_diag<<<grid_for(A.n * 16, 256), 256, 0, s>>>(A.n, A.rp.p, A.ci.p, A.v.p, d);
  KCHK();
}

double row_stats(const Csr &A, double *d, double *l1inv, hipStream_t s, int *dflag) {
  DArr<double> q(std::max<int64_t>(A.n, 1), s);
  if (A.n > 0) {
    k_row_stats<16><<<grid_for(A.n * 16, 256), 256, 0, s>>>(A.n, A.rp.p, A.ci.p, A.v.p, d, q.p,
                                                           l1inv, dflag);
    KCHK();
  }
  const double r = reduce_max_f64(q.p, A.n, s);
  check_flags(dflag, s, "AMG diagonal");
  return r;
}

double gershgorin_rho(const Csr &A, hipStream_t s, int *dflag) {
  DArr<double> q(A.n, s);
  k_gershgorin<<<grid_for(A.n, 256), 256, 0, s>>>(A.n, A.rp.p, A.ci.p, A.v.p, q.p, dflag);
  KCHK();
  double r = reduce_max_f64(q.p, A.n, s);
  check_flags(dflag, s, "AMG diagonal");
  return r;
}

void omega_over_diag(const double *d, double omega, double *w, int64_t n, hipStream_t s) {
  if (n == 0) return;
  k_omega_over<<<grid_for(n, 256), 256, 0, s>>>(d, omega, w, n);
  KCHK();
}

void l1_inverse(const Csr &A, double *dinv, hipStream_t s) {
  if (A.n == 0) return;
  k_l1_inv<<<grid_for(A.n, 256), 256, 0, s>>>(A.n, A.rp.p, A.v.p, dinv);
  KCHK();
}

void copy_csr(const Csr &A, Csr &B, hipStream_t s) {
  B.n = A.n;
  B.m = A.m;
  B.nnz = A.nnz;
  B.rp.alloc(A.n + 1, s);
  B.ci.alloc(A.nnz, s);
  B.v.alloc(A.nnz, s);
  HIPCHK(hipMemcpyAsync(B.rp.p, A.rp.p, (A.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (A.nnz) {
    HIPCHK(hipMemcpyAsync(B.ci.p, A.ci.p, A.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(B.v.p, A.v.p, A.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
}

// BSR (b x b row-major blocks, block rows and columns) to scalar CSR: scalar row br*b + r
// holds, for every block of block row br in order, the b entries of the block's row r
// (zeros included), so the columns stay sorted
__global__ void k_bsr_rowptr(int64_t nbr, int bs, const int64_t *__restrict__ brp,
                             int *__restrict__ rp, int *flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > nbr * bs) return;
  const int64_t br = i / bs, r = i % bs;
  const int64_t v = i == nbr * bs ? brp[nbr] * bs * bs
                                  : brp[br] * bs * bs + r * (brp[br + 1] - brp[br]) * bs;
  if (v < 0 || v > 0x7fffffffLL) atomicOr(flag, FLAG_OVERFLOW);
  rp[i] = (int)v;
}
__global__ void k_bsr_expand(int64_t nbr, int bs, const int64_t *__restrict__ brp,
                             const int *__restrict__ bci, const double *__restrict__ bv,
                             const int *__restrict__ rp, int *__restrict__ ci,
                             double *__restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // scalar row
  if (i >= nbr * bs) return;
  const int64_t br = i / bs;
  const int r = (int)(i % bs);
  int o = rp[i];
  for (int64_t e = brp[br]; e < brp[br + 1]; ++e)
    for (int c = 0; c < bs; ++c) {
      ci[o] = bci[e] * bs + c;
      v[o] = bv[e * bs * bs + r * bs + c];
      ++o;
    }
}

void import_csr(const mgr_csr *A, Csr &B, hipStream_t s, int *dflag, bool borrow) {
  require(A->block >= 0 && A->block <= 3, MGR_ERR_ARG, "matrix block size must be 0..3");
  if (A->block > 1) {
    const int bs = A->block;
    int64_t nnzb = 0;
    HIPCHK(hipMemcpyAsync(&nnzb, A->row_ptr + A->nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t nnz = nnzb * bs * bs;
    require(nnzb >= 0 && nnz < 0x7fffffffLL, MGR_ERR_UNSUPPORTED, "nnz must be below 2^31");
    B.n = A->nrows * bs;
    B.m = A->ncols * bs;
    B.nnz = nnz;
    B.rp.alloc(B.n + 1, s);
    B.ci.alloc(std::max<int64_t>(nnz, 1), s);
    B.v.alloc(std::max<int64_t>(nnz, 1), s);
    k_bsr_rowptr<<<grid_for(B.n + 1, 256), 256, 0, s>>>(A->nrows, bs, A->row_ptr, B.rp.p, dflag);
    KCHK();
    if (B.n > 0) {
      k_bsr_expand<<<grid_for(B.n, 256), 256, 0, s>>>(A->nrows, bs, A->row_ptr, A->col, A->val,
                                                      B.rp.p, B.ci.p, B.v.p);
      KCHK();
    }
    check_flags(dflag, s, "block matrix import");
    return;
  }
  int64_t nnz = 0;
  HIPCHK(hipMemcpyAsync(&nnz, A->row_ptr + A->nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  require(nnz >= 0 && nnz < 0x7fffffffLL, MGR_ERR_UNSUPPORTED, "nnz must be below 2^31");
  B.n = A->nrows;
  B.m = A->ncols;
  B.nnz = nnz;
  B.rp.alloc(B.n + 1, s);
  rowptr64_to_32(A->row_ptr, B.rp.p, B.n + 1, dflag, s);
  if (borrow) {
    B.ci.borrow(const_cast<int *>(A->col), nnz, s);
    B.v.borrow(const_cast<double *>(A->val), nnz, s);
  } else {
    B.ci.alloc(nnz, s);
    B.v.alloc(nnz, s);
    if (nnz) {
      HIPCHK(hipMemcpyAsync(B.ci.p, A->col, nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(B.v.p, A->val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  check_flags(dflag, s, "matrix import");
}

uint64_t pattern_hash(const Csr &A, hipStream_t s) {
  constexpr unsigned NB = 2048;
  DArr<unsigned long long> h(1, s), part(NB, s);
  fill<unsigned long long>(h.p, 0ull, 1, s);
  const unsigned g0 = std::min<unsigned>(grid_for(A.n + 1, 256), NB);
  k_hash<<<g0, 256, 0, s>>>(A.n + 1, A.rp.p, 0x1234567ull, part.p);
  KCHK();
  k_hash_sum<<<1, 256, 0, s>>>(part.p, (int)g0, h.p);
  KCHK();
  if (A.nnz) {
    const unsigned g1 = std::min<unsigned>(grid_for(A.nnz, 256), NB);
    k_hash<<<g1, 256, 0, s>>>(A.nnz, A.ci.p, 0x9876543ull, part.p);
    KCHK();
    k_hash_sum<<<1, 256, 0, s>>>(part.p, (int)g1, h.p);
    KCHK();
  }
  unsigned long long r = 0;
  d2h_sync(&r, h.p, sizeof(r), s);
  return r;
}

void csr_to_bsr3(const Csr &A, DArr<int> &rp, DArr<int> &ci, DArr<double> &v, int64_t &nb,
                 int64_t &mb, int64_t &nnzb, hipStream_t s, int *dflag, const char *what) {
  require(A.n % 3 == 0 && A.m % 3 == 0, MGR_ERR_UNSUPPORTED, "BSR3 needs sizes divisible by 3");
  nb = A.n / 3;
  mb = A.m / 3;
  DArr<int> cnt(nb + 1, s), bad(1, s);
  fill<int>(bad.p, 0x7fffffff, 1, s);
  k_bsr3_count<16><<<grid_for(nb * 16, 256), 256, 0, s>>>(nb, A.rp.p, A.ci.p, cnt.p, dflag, bad.p);
  KCHK();
  rp.alloc(nb + 1, s);
  nnzb = exclusive_scan_i32(cnt.p, rp.p, nb, s);
  const int f = read_flag(dflag, s);
  if (f & FLAG_NOT_BLOCKED) {
    const int I = read_flag(bad.p, s);
    int r[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(r, A.rp.p + 3 * (int64_t)I, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    throw Error(MGR_ERR_UNSUPPORTED,
                std::string("nodal level without full 3x3 blocks (") + what + " " +
                    std::to_string(A.n) + "x" + std::to_string(A.m) + ", node " +
                    std::to_string(I) + ", row lengths " + std::to_string(r[1] - r[0]) + "/" +
                    std::to_string(r[2] - r[1]) + "/" + std::to_string(r[3] - r[2]) + ")");
  }
  check_flags(dflag, s, "block conversion");
  ci.alloc(nnzb, s);
  v.alloc(nnzb * 9, s);
  k_bsr3_fill<16><<<grid_for(nb * 16, 256), 256, 0, s>>>(nb, A.rp.p, A.ci.p, A.v.p, rp.p, ci.p, v.p);
  KCHK();
}

void csr_to_bsr3(const Csr &A, Bsr3 &B, hipStream_t s, int *dflag, const char *what) {
  csr_to_bsr3(A, B.rp, B.ci, B.v, B.nb, B.mb, B.nnzb, s, dflag, what);
}

namespace {
__global__ void k_b3_rowptr(int64_t nb, const int *__restrict__ brp, int *__restrict__ rp) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // scalar row
  if (t > 3 * nb) return;
  if (t == 3 * nb) {
    rp[t] = 9 * brp[nb];
    return;
  }
  const int64_t I = t / 3, r = t % 3;
  rp[t] = 9 * brp[I] + 3 * (int)r * (brp[I + 1] - brp[I]);
}
__global__ void k_b3_expand(int64_t nb, const int *__restrict__ brp, const int *__restrict__ bci,
                            const double *__restrict__ bv, const int *__restrict__ rp,
                            int *__restrict__ ci, double *__restrict__ v) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // (scalar row, block)
  if (t >= 3 * (int64_t)brp[nb]) return;
  const int64_t e = t / 3;
  const int r = (int)(t % 3);
  // block row of entry e: binary search in brp
  int64_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (brp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  const int64_t I = lo;
  const int64_t pos = rp[3 * I + r] + 3 * (e - brp[I]);
  const int J = bci[e];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ci[pos + c] = 3 * J + c;
    v[pos + c] = bv[9 * e + 3 * r + c];
  }
}
__global__ void k_iota_f64(int64_t n, double *__restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) v[i] = (double)i;
}
__global__ void k_b3_gather_t(int64_t nnzb, const double *__restrict__ idx,
                              const double *__restrict__ pv, double *__restrict__ rv) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nnzb) return;
  const int64_t q = (int64_t)idx[e];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[9 * e + 3 * r + c] = pv[9 * q + 3 * c + r];
}
__global__ void k_tent_b3(int64_t nnode, const int *__restrict__ agg, const int *__restrict__ rp,
                          int *__restrict__ ci, double *__restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nnode || agg[i] < 0) return;
  const int e = rp[i];
  ci[e] = agg[i];
#pragma unroll
  for (int q = 0; q < 9; ++q) v[9 * (int64_t)e + q] = (q % 4 == 0) ? 1.0 : 0.0;
}
__global__ void k_tent_b3_count(int64_t nnode, const int *__restrict__ agg, int *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nnode) cnt[i] = agg[i] >= 0 ? 1 : 0;
}
}  // namespace

void bsr3_to_csr(const Bsr3 &B, Csr &C, hipStream_t s) {
  C.n = 3 * B.nb;
  C.m = 3 * B.mb;
  require(9 * B.nnzb < ((int64_t)1 << 31), MGR_ERR_UNSUPPORTED, "matrix too large");
  C.nnz = 9 * B.nnzb;
  C.rp.alloc(C.n + 1, s);
  C.ci.alloc(std::max<int64_t>(C.nnz, 1), s);
  C.v.alloc(std::max<int64_t>(C.nnz, 1), s);
  k_b3_rowptr<<<grid_for(C.n + 1, 256), 256, 0, s>>>(B.nb, B.rp.p, C.rp.p);
  KCHK();
  if (B.nnzb == 0) return;
  k_b3_expand<<<grid_for(3 * B.nnzb, 256), 256, 0, s>>>(B.nb, B.rp.p, B.ci.p, B.v.p, C.rp.p,
                                                        C.ci.p, C.v.p);
  KCHK();
}

void bsr3_transpose(const Bsr3 &P, Bsr3 &R, hipStream_t s) {
  // transpose the block pattern carrying each block's index, then gather transposed blocks
  Csr Pp;
  Pp.n = P.nb;
  Pp.m = P.mb;
  Pp.nnz = P.nnzb;
  Pp.rp.alloc(P.nb + 1, s);
  HIPCHK(hipMemcpyAsync(Pp.rp.p, P.rp.p, (P.nb + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  Pp.ci.alloc(std::max<int64_t>(P.nnzb, 1), s);
  if (P.nnzb)
    HIPCHK(hipMemcpyAsync(Pp.ci.p, P.ci.p, P.nnzb * sizeof(int), hipMemcpyDeviceToDevice, s));
  Pp.v.alloc(std::max<int64_t>(P.nnzb, 1), s);
  if (P.nnzb) {
    k_iota_f64<<<grid_for(P.nnzb, 256), 256, 0, s>>>(P.nnzb, Pp.v.p);
    KCHK();
  }
  Csr Rp;
  transpose(Pp, Rp, true, s);
  R.nb = P.mb;
  R.mb = P.nb;
  R.nnzb = P.nnzb;
  R.rp = std::move(Rp.rp);
  R.ci = std::move(Rp.ci);
  R.v.alloc(std::max<int64_t>(9 * P.nnzb, 1), s);
  if (P.nnzb) {
    k_b3_gather_t<<<grid_for(P.nnzb, 256), 256, 0, s>>>(P.nnzb, Rp.v.p, P.v.p, R.v.p);
    KCHK();
  }
}

void tentative_b3(const DArr<int> &agg, int64_t nnode, int64_t nagg, Bsr3 &T, hipStream_t s) {
  T.nb = nnode;
  T.mb = nagg;
  T.rp.alloc(nnode + 1, s);
  DArr<int> cnt(nnode + 1, s);
  k_tent_b3_count<<<grid_for(nnode, 256), 256, 0, s>>>(nnode, agg.p, cnt.p);
  KCHK();
  T.nnzb = exclusive_scan_i32(cnt.p, T.rp.p, nnode, s);
  T.ci.alloc(std::max<int64_t>(T.nnzb, 1), s);
  T.v.alloc(std::max<int64_t>(9 * T.nnzb, 1), s);
  k_tent_b3<<<grid_for(nnode, 256), 256, 0, s>>>(nnode, agg.p, T.rp.p, T.ci.p, T.v.p);
  KCHK();
}

namespace {
__global__ void k_rows_count(int64_t nr, const int *__restrict__ rows, const int *__restrict__ rp,
                             int *__restrict__ cnt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < nr) cnt[t] = rp[rows[t] + 1] - rp[rows[t]];
}
template <int G>
__global__ void k_rows_copy(int64_t nr, const int *__restrict__ rows, const int *__restrict__ rp,
                            const int *__restrict__ ci, const double *__restrict__ v,
                            const int *__restrict__ orp, int *__restrict__ oci,
                            double *__restrict__ ov) {
  const int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (t >= nr) return;
  const int r = rows[t], s0 = rp[r], len = rp[r + 1] - s0, o = orp[t];
  for (int e = l; e < len; e += G) {
    oci[o + e] = ci[s0 + e];
    ov[o + e] = v[s0 + e];
  }
}
}  // namespace

void gather_rows(const Csr &A, const int *rows, int64_t nr, Csr &out, hipStream_t s) {
  out.n = nr;
  out.m = A.m;
  out.rp.alloc(nr + 1, s);
  DArr<int> cnt(std::max<int64_t>(nr, 1), s);
  if (nr > 0) {
    k_rows_count<<<grid_for(nr, 256), 256, 0, s>>>(nr, rows, A.rp.p, cnt.p);
    KCHK();
  }
  out.nnz = exclusive_scan_i32(cnt.p, out.rp.p, nr, s);
  out.ci.alloc(std::max<int64_t>(out.nnz, 1), s);
  out.v.alloc(std::max<int64_t>(out.nnz, 1), s);
  if (nr > 0 && out.nnz > 0) {
    k_rows_copy<16><<<grid_for(nr * 16, 256), 256, 0, s>>>(nr, rows, A.rp.p, A.ci.p, A.v.p,
                                                          out.rp.p, out.ci.p, out.v.p);
    KCHK();
  }
}

// ---------------------------------------------------------------------------------
// CSR -> B x BC block CSR over cells of B rows (every touched block stored whole)
namespace {
constexpr int kBsrWin = 512;   // blocks per stream window of the cell-block kernels

// The block columns of block row I (a cell) are the distinct c / BC of its B rows.  G lanes
// per cell stage the cell's column indices (one contiguous range of the CSR arrays) in LDS.
// An entry represents its block column when it is the first entry of that block column in
// its row and no earlier row of the cell holds the block column (binary searches in the
// sorted rows); representatives are marked in a bit mask.  Every block column has exactly
// one representative, so the position of block column bc among the cell's blocks is the
// number of representatives left of bc's lower bound in each row: popcounts of the mask.
// The count pass writes the number of representatives; the fill pass scatters every value
// into its block (the blocks are zeroed beforehand) and the representatives write the
// block columns.  No lane works serially over a cell.  Cells beyond BCAP entries are
// merged from global memory by one lane (256 staged entries: 17 KB per workgroup, so that a
// CU holds 32 wavefronts; the cells of 7-point flow levels and of A_CF hold at most 72).
constexpr int BG_LANES = 16;
constexpr int BCAP = 256;

// first position in s[lo, hi) whose value is >= key
__device__ inline int lds_lower_bound(const int *s, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// number of set bits of mask in positions [a, b)
__device__ inline int popc_range(const unsigned *mask, int a, int b) {
  int n = 0;
  for (int w = a >> 5; a < b && w <= (b - 1) >> 5; ++w) {
    const int lo = max(a - w * 32, 0), hi = min(b - w * 32, 32);
    const unsigned m = (hi == 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
    n += __popc(mask[w] & m);
  }
  return n;
}

template <int B, int BC, bool FILL>
__global__ void __launch_bounds__(256) k_bsrb_rows(int64_t nbr, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const double *__restrict__ v,
                                                   int *__restrict__ cnt,
                                                   const int *__restrict__ brp,
                                                   int *__restrict__ bci,
                                                   double *__restrict__ bv) {
  constexpr int NGR = 256 / BG_LANES;
  constexpr int NW = BCAP / 32;
  __shared__ int s_c[NGR][BCAP];
  __shared__ unsigned s_f[NGR][NW];
  const int g = threadIdx.x / BG_LANES, l = threadIdx.x & (BG_LANES - 1);
  const int64_t I = blockIdx.x * (int64_t)NGR + g;
  if (I >= nbr) return;   // whole groups leave together
  int rs[B + 1];
  const int e0 = rp[I * B];
#pragma unroll
  for (int r = 0; r <= B; ++r) rs[r] = rp[I * B + r] - e0;
  const int ne = rs[B];
  const int o = FILL ? brp[I] : 0;
  if (ne > BCAP) {   // long cell: merge from global memory by one lane
    if (l == 0) {
      int grs[B + 1];
#pragma unroll
      for (int r = 0; r <= B; ++r) grs[r] = rs[r] + e0;
      int p[B];
#pragma unroll
      for (int r = 0; r < B; ++r) p[r] = grs[r];
      int nb = 0;
      for (;;) {
        int mc = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < B; ++r)
          if (p[r] < grs[r + 1]) mc = min(mc, ci[p[r]] / BC);
        if (mc == 0x7fffffff) break;
        if (FILL) bci[o + nb] = mc;
#pragma unroll
        for (int r = 0; r < B; ++r)
          while (p[r] < grs[r + 1] && ci[p[r]] / BC == mc) {
            if (FILL) bv[(int64_t)(o + nb) * B * BC + r * BC + ci[p[r]] % BC] = v[p[r]];
            ++p[r];
          }
        ++nb;
      }
      if (!FILL) cnt[I] = nb;
    }
    return;
  }
  for (int k = l; k < ne; k += BG_LANES) s_c[g][k] = ci[e0 + k];
  for (int w = l; w < NW; w += BG_LANES) s_f[g][w] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int k = l; k < ne; k += BG_LANES) {
    int r = 0;
#pragma unroll
    for (int q = 1; q < B; ++q) r += (k >= rs[q]);
    const int bc = s_c[g][k] / BC;
    bool rep = (k == rs[r]) || (s_c[g][k - 1] / BC != bc);
#pragma unroll
    for (int q = 0; q < B - 1; ++q)
      if (rep && q < r) {
        const int lb = lds_lower_bound(s_c[g], rs[q], rs[q + 1], bc * BC);
        if (lb < rs[q + 1] && s_c[g][lb] < (bc + 1) * BC) rep = false;
      }
    if (rep) atomicOr(&s_f[g][k >> 5], 1u << (k & 31));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (!FILL) {
    if (l == 0) cnt[I] = popc_range(s_f[g], 0, ne);
    return;
  }
  for (int k = l; k < ne; k += BG_LANES) {
    int r = 0;
#pragma unroll
    for (int q = 1; q < B; ++q) r += (k >= rs[q]);
    const int c = s_c[g][k], bc = c / BC;
    int pos = 0;
#pragma unroll
    for (int q = 0; q < B; ++q)
      pos += popc_range(s_f[g], rs[q], lds_lower_bound(s_c[g], rs[q], rs[q + 1], bc * BC));
    bv[(int64_t)(o + pos) * B * BC + r * BC + (c - bc * BC)] = v[e0 + k];
    if (s_f[g][k >> 5] & (1u << (k & 31))) bci[o + pos] = bc;
  }
}

__global__ void k_bsrb_windows(int64_t nbr, const int *__restrict__ brp, int64_t K,
                               int *__restrict__ rb) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k > K) return;
  if (k == K) { rb[k] = (int)nbr; return; }
  const int64_t target = k * (int64_t)kBsrWin;
  int64_t lo = 0, hi = nbr;          // first block row whose first block is >= target
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (brp[mid] < target) lo = mid + 1; else hi = mid;
  }
  rb[k] = (int)lo;
}
}  // namespace

void csr_to_bsr_fill(const Csr &A, int br, int bc, BsrB &B, hipStream_t s) {
  const int shape = br * 10 + bc;
  require(shape == 22 || shape == 33 || shape == 23, MGR_ERR_ARG,
          "cell blocks must be 2x2, 3x3 or 2x3");
  require(A.n % br == 0 && A.m % bc == 0, MGR_ERR_ARG,
          "block matrix: sizes not divisible by the block shape");
  B.br = br;
  B.bc = bc;
  B.nbr = A.n / br;
  B.rp.alloc(B.nbr + 1, s);
  DArr<int> cnt(std::max<int64_t>(B.nbr, 1), s);
  const unsigned gr = grid_for(B.nbr * BG_LANES, 256);
#define BSRB_ROWS(R, C, F, cntp, brpp, bcip, bvp)                                           \
  k_bsrb_rows<R, C, F><<<gr, 256, 0, s>>>(B.nbr, A.rp.p, A.ci.p, F ? A.v.p : nullptr, cntp, \
                                          brpp, bcip, bvp)
  if (B.nbr > 0) {
    if (shape == 22) BSRB_ROWS(2, 2, false, cnt.p, nullptr, nullptr, nullptr);
    else if (shape == 33) BSRB_ROWS(3, 3, false, cnt.p, nullptr, nullptr, nullptr);
    else BSRB_ROWS(2, 3, false, cnt.p, nullptr, nullptr, nullptr);
    KCHK();
  }
  B.nblk = exclusive_scan_i32(cnt.p, B.rp.p, B.nbr, s);
  B.ci.alloc(std::max<int64_t>(B.nblk, 1), s);
  B.v.alloc(std::max<int64_t>(B.nblk * br * bc, 1), s);
  fill<double>(B.v.p, 0.0, B.nblk * br * bc, s);   // entries absent from A stay zero
  if (B.nbr > 0) {
    if (shape == 22) BSRB_ROWS(2, 2, true, nullptr, B.rp.p, B.ci.p, B.v.p);
    else if (shape == 33) BSRB_ROWS(3, 3, true, nullptr, B.rp.p, B.ci.p, B.v.p);
    else BSRB_ROWS(2, 3, true, nullptr, B.rp.p, B.ci.p, B.v.p);
    KCHK();
  }
#undef BSRB_ROWS
  B.nwin = make_block_windows(B.rp.p, B.nbr, B.nblk, B.rb, s);
}

int64_t make_block_windows(const int *rp, int64_t nbr, int64_t nblk, DArr<int> &rb,
                           hipStream_t s) {
  const int64_t nwin = nblk > 0 ? (nblk + kBsrWin - 1) / kBsrWin : 0;
  rb.alloc(nwin + 1, s);
  k_bsrb_windows<<<grid_for(nwin + 1, 256), 256, 0, s>>>(nbr, rp, nwin, rb.p);
  KCHK();
  return nwin;
}

void block_diag_inverse(const Csr &A, int nb, double *inv, hipStream_t s, int *dflag) {
  require(A.n % nb == 0, MGR_ERR_UNSUPPORTED, "block smoother: size not divisible by block");
  const int64_t nblk = A.n / nb;
  k_block_inv<<<grid_for(nblk, 256), 256, 0, s>>>(nblk, nb, A.rp.p, A.ci.p, A.v.p, inv, dflag);
  KCHK();
  check_flags(dflag, s, "same-cell blocks");
}

}  // namespace mgr

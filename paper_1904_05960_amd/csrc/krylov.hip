// FP64 kernels of flexible GMRES: outer SpMV (int64 row pointers), classical Gram-Schmidt
// with one re-orthogonalisation fused into streaming passes over the Krylov basis, norms,
// the Givens update of the Hessenberg least-squares problem, and x = x0 + Z y.
// Reductions are two-stage with a fixed tree (per-block partials, then one block per
// output), so results are identical from run to run.
#include <map>
#include <mutex>

#include "common.hpp"

namespace mgr {
namespace {

constexpr int NB = 1024;     // partial-sum blocks
constexpr int KS = 72;       // partial stride (>= restart + 1)
constexpr int KC = 16;       // basis vectors per register chunk

template <int G>
__global__ void __launch_bounds__(256) k_spmv64(int64_t n, const int64_t *__restrict__ rp,
                                                const int *__restrict__ ci,
                                                const double *__restrict__ v,
                                                const double *__restrict__ x,
                                                const double *__restrict__ b,
                                                double *__restrict__ y) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x & (G - 1);
  if (row >= n) return;
  double acc = 0.0;
  const int64_t e1 = rp[row + 1];
  for (int64_t e = rp[row] + l; e < e1; e += G) acc += v[e] * x[ci[e]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (l == 0) y[row] = b ? b[row] - acc : acc;
}

void launch_spmv64(const mgr_csr &A, const double *x, const double *b, double *y, hipStream_t s,
                   double avg) {
#define L64(GG)                                                                         \
  k_spmv64<GG><<<grid_for(A.nrows * GG, 256), 256, 0, s>>>(A.nrows, A.row_ptr, A.col, A.val, \
                                                           x, b, y)
  if (avg > 48) L64(64);
  else if (avg > 24) L64(32);
  else if (avg > 12) L64(16);
  else L64(8);
#undef L64
  KCHK();
}

// ---------------------------------------------------------------------------------
// CSR-stream SpMV: block k owns rows [rb[k], rb[k+1]) whose entries start in
// [k * SNNZ, (k+1) * SNNZ).  The block's products v[e] * x[ci[e]] are written to LDS with
// coalesced loads, then every row is summed from LDS by 8 lanes.  A block whose rows hold
// more than SCAP entries (only possible with a row longer than SCAP - SNNZ = 256) sums each
// row directly.  SCAP is kept just above SNNZ: 18 KB of LDS per block lets 8 blocks (32
// waves) share a CU, where a 32 KB window held 5.
constexpr int SB = 256;
constexpr int SNNZ = 2048;
constexpr int SCAP = SNNZ + 256;

__global__ void k_rowblocks(int64_t n, const int64_t *__restrict__ rp, int64_t K,
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

__global__ void __launch_bounds__(SB) k_spmv_stream(const int *__restrict__ rb,
                                                    const int64_t *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const double *__restrict__ v,
                                                    const double *__restrict__ x,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ y) {
  __shared__ double prod[SCAP];
  const int r0 = rb[blockIdx.x], r1 = rb[blockIdx.x + 1];
  if (r0 >= r1) return;
  const int64_t base = rp[r0];
  const int64_t cnt = rp[r1] - base;
  const int t = threadIdx.x;
  if (cnt <= SCAP) {
    constexpr int G = 8;
    // the first row of this thread's sum phase: its extent and b entry are loaded now, so
    // that their latency overlaps the gathers
    const int prow = r0 + t / G;
    int ps = 0, pe = 0;
    double pb = 0.0;
    if (prow < r1) {
      ps = (int)(rp[prow] - base);
      pe = (int)(rp[prow + 1] - base);
      if (b) pb = b[prow];
    }
    // all loads of a thread issued before any gather is consumed: PER independent chains
    constexpr int PER = SNNZ / SB;
    for (int e0 = 0; e0 < cnt; e0 += PER * SB) {
      int c[PER];
      double vv[PER], xv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        c[u] = 0;
        vv[u] = 0.0;
        if (e < cnt) {
          c[u] = ci[base + e];
          vv[u] = v[base + e];
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        xv[u] = (e < cnt) ? x[c[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = e0 + u * SB + t;
        if (e < cnt) prod[e] = vv[u] * xv[u];
      }
    }
    __syncthreads();
    const int l = t & (G - 1);
    for (int row = prow; row < r1; row += SB / G) {
      int s = ps, e1 = pe;
      double bv = pb;
      if (row != prow) {
        s = (int)(rp[row] - base);
        e1 = (int)(rp[row + 1] - base);
        bv = b ? b[row] : 0.0;
      }
      double acc = 0.0;
      for (int e = s + l; e < e1; e += G) acc += prod[e];
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
      if (l == 0) y[row] = b ? bv - acc : acc;
    }
    return;
  }
  static_assert(SB == 256, "the fallback sums four wave partials");
  __shared__ double part[SB / 64];
  for (int row = r0; row < r1; ++row) {
    double acc = 0.0;
    for (int64_t e = rp[row] + t; e < rp[row + 1]; e += SB) acc += v[e] * x[ci[e]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((t & 63) == 0) part[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      const double tot = (part[0] + part[1]) + (part[2] + part[3]);
      y[row] = b ? b[row] - tot : tot;
    }
    __syncthreads();
  }
}

// BSR variant (b x b row-major blocks; used for b = 2): block k owns the block rows whose
// first block lies in the k-th window of SNNZ / b^2 blocks; the window's b^2 values per
// block are read as one contiguous, coalesced stream, each multiplied by the x entry of
// its block column and staged in LDS; then every scalar row (br, r) sums the b entries of
// its row in each block from LDS with 8 lanes.  A window whose block rows hold more than
// SCAP values (a block row longer than (SCAP - SNNZ) / b^2 + 1 blocks) sums each scalar row
// directly.
template <int WB>
__global__ void k_bsr_rowblocks(int64_t nbr, const int64_t *__restrict__ rp, int64_t K,
                                int *__restrict__ rb) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k > K) return;
  if (k == K) { rb[k] = (int)nbr; return; }
  const int64_t target = k * WB;
  int64_t lo = 0, hi = nbr;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] < target) lo = mid + 1; else hi = mid;
  }
  rb[k] = (int)lo;
}

template <int B>
__global__ void __launch_bounds__(SB) k_bsr_stream(const int *__restrict__ rb,
                                                   const int64_t *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ y) {
  constexpr int BB = B * B;
  __shared__ double prod[SCAP];
  const int r0 = rb[blockIdx.x], r1 = rb[blockIdx.x + 1];
  if (r0 >= r1) return;
  const int64_t base = rp[r0];                 // first block of the window
  const int64_t cnt = (rp[r1] - base) * BB;    // values of the window
  const int t = threadIdx.x;
  if (cnt <= SCAP) {
    constexpr int G = 8;
    // the first scalar row of this thread's sum phase: block-row extent and b entry now
    const int nsr = (r1 - r0) * B;
    const int psr = t / G;
    int ps = 0, plen = 0;
    double pb = 0.0;
    if (psr < nsr) {
      const int br = r0 + psr / B;
      ps = (int)(rp[br] - base);
      plen = (int)(rp[br + 1] - rp[br]) * B;
      if (b) pb = b[(int64_t)br * B + psr % B];
    }
    constexpr int PER = SNNZ / SB;
    const double *vb = v + base * BB;
    for (int e0 = 0; e0 < cnt; e0 += PER * SB) {
      int c[PER];
      double vv[PER], xv[PER];
      // raw loads first (block column and value), all in flight together; the column
      // arithmetic waits for them in the gather loop
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int q = e0 + u * SB + t;
        c[u] = 0;
        vv[u] = 0.0;
        if (q < cnt) {
          c[u] = ci[base + q / BB];
          vv[u] = vb[q];
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int q = e0 + u * SB + t;
        xv[u] = (q < cnt) ? x[(int64_t)c[u] * B + (q % BB) % B] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int q = e0 + u * SB + t;
        if (q < cnt) prod[q] = vv[u] * xv[u];
      }
    }
    __syncthreads();
    const int l = t & (G - 1);
    for (int sr = psr; sr < nsr; sr += SB / G) {
      const int br = r0 + sr / B, r = sr % B;
      int s0 = ps, len = plen;
      double bv = pb;
      if (sr != psr) {
        s0 = (int)(rp[br] - base);
        len = (int)(rp[br + 1] - rp[br]) * B;
        bv = b ? b[(int64_t)br * B + r] : 0.0;
      }
      double acc = 0.0;
      for (int k = l; k < len; k += G) {
        const int e = s0 + k / B;
        acc += prod[e * BB + r * B + k % B];
      }
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
      if (l == 0) y[(int64_t)br * B + r] = b ? bv - acc : acc;
    }
    return;
  }
  static_assert(SB == 256, "the fallback sums four wave partials");
  __shared__ double part[SB / 64];
  for (int br = r0; br < r1; ++br) {
    const int64_t e0 = rp[br], len = (rp[br + 1] - e0) * B;
    for (int r = 0; r < B; ++r) {
      double acc = 0.0;
      for (int64_t k = t; k < len; k += SB) {
        const int64_t e = e0 + k / B;
        const int c = (int)(k % B);
        acc += v[e * BB + r * B + c] * x[(int64_t)ci[e] * B + c];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((t & 63) == 0) part[t >> 6] = acc;
      __syncthreads();
      if (t == 0) {
        const double tot = (part[0] + part[1]) + (part[2] + part[3]);
        const int64_t row = (int64_t)br * B + r;
        y[row] = b ? b[row] - tot : tot;
      }
      __syncthreads();
    }
  }
}

// 3x3 blocks, one lane per block: block k of the grid owns the block rows whose first block
// lies in the k-th window of WB3 = 512 blocks.  Each lane takes two blocks of the window at
// a time (its own nine values read as one 72-byte record, the block column, the three x
// entries), issuing every load of both before using any, and forms each block's three row
// partials (v_r0 x_0 + v_r1 x_1) + v_r2 x_2 into LDS; every scalar row then sums its blocks'
// partials with 8 lanes.  One lane per block needs 13 memory instructions per wave and 64
// blocks where a lane per value needs 27 (nine values, nine block columns, nine x
// entries); its per-lane records are gathered through L1 at the full streaming rate.
// Windows whose block rows hold more than PCAP3 blocks sum each scalar row directly.
constexpr int WB3 = 2 * SB;
constexpr int PCAP3 = 3 * SB;
__global__ void __launch_bounds__(SB) k_bsr3_lane(const int *__restrict__ rb,
                                                  const int64_t *__restrict__ rp,
                                                  const int *__restrict__ ci,
                                                  const double *__restrict__ v,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ y) {
  __shared__ double part[PCAP3 * 3];
  const int r0 = rb[blockIdx.x], r1 = rb[blockIdx.x + 1];
  if (r0 >= r1) return;
  const int64_t base = rp[r0];
  const int nblk = (int)(rp[r1] - base);
  const int t = threadIdx.x;
  if (nblk <= PCAP3) {
    constexpr int G = 8;
    // the first scalar row of this thread's sum phase: block-row extent and b entry now
    const int nsr = (r1 - r0) * 3;
    const int psr = t / G;
    int ps = 0, plen = 0;
    double pb = 0.0;
    if (psr < nsr) {
      const int br = r0 + psr / 3;
      ps = (int)(rp[br] - base);
      plen = (int)(rp[br + 1] - rp[br]);
      if (b) pb = b[(int64_t)br * 3 + psr % 3];
    }
    constexpr int BPL = 2;
    for (int q0 = 0; q0 < nblk; q0 += BPL * SB) {
      double a[BPL][9];
      int cc[BPL];
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * SB + t;
        cc[h] = 0;
        if (e < nblk) {
          const double *bv = v + (base + e) * 9;
#pragma unroll
          for (int u = 0; u < 9; ++u) a[h][u] = bv[u];
          cc[h] = ci[base + e];
        } else {
#pragma unroll
          for (int u = 0; u < 9; ++u) a[h][u] = 0.0;
        }
      }
      double xx[BPL][3];
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * SB + t;
        xx[h][0] = xx[h][1] = xx[h][2] = 0.0;
        if (e < nblk) {
          const double *xc = x + (int64_t)cc[h] * 3;
          xx[h][0] = xc[0];
          xx[h][1] = xc[1];
          xx[h][2] = xc[2];
        }
      }
#pragma unroll
      for (int h = 0; h < BPL; ++h) {
        const int e = q0 + h * SB + t;
        if (e < nblk) {
          part[e * 3 + 0] = a[h][0] * xx[h][0] + a[h][1] * xx[h][1] + a[h][2] * xx[h][2];
          part[e * 3 + 1] = a[h][3] * xx[h][0] + a[h][4] * xx[h][1] + a[h][5] * xx[h][2];
          part[e * 3 + 2] = a[h][6] * xx[h][0] + a[h][7] * xx[h][1] + a[h][8] * xx[h][2];
        }
      }
    }
    __syncthreads();
    const int l = t & (G - 1);
    for (int sr = psr; sr < nsr; sr += SB / G) {
      const int br = r0 + sr / 3, r = sr % 3;
      int s0 = ps, len = plen;
      double bvv = pb;
      if (sr != psr) {
        s0 = (int)(rp[br] - base);
        len = (int)(rp[br + 1] - rp[br]);
        bvv = b ? b[(int64_t)br * 3 + r] : 0.0;
      }
      double acc = 0.0;
      for (int k = l; k < len; k += G) acc += part[(s0 + k) * 3 + r];
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
      if (l == 0) y[(int64_t)br * 3 + r] = b ? bvv - acc : acc;
    }
    return;
  }
  static_assert(SB == 256, "the fallback sums four wave partials");
  __shared__ double fpart[SB / 64];
  for (int br = r0; br < r1; ++br) {
    const int64_t e0 = rp[br], len = (rp[br + 1] - e0) * 3;
    for (int r = 0; r < 3; ++r) {
      double acc = 0.0;
      for (int64_t k = t; k < len; k += SB) {
        const int64_t e = e0 + k / 3;
        const int c = (int)(k % 3);
        acc += v[e * 9 + r * 3 + c] * x[(int64_t)ci[e] * 3 + c];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((t & 63) == 0) fpart[t >> 6] = acc;
      __syncthreads();
      if (t == 0) {
        const double tot = (fpart[0] + fpart[1]) + (fpart[2] + fpart[3]);
        const int64_t row = (int64_t)br * 3 + r;
        y[row] = b ? b[row] - tot : tot;
      }
      __syncthreads();
    }
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-level reduction of KC values per thread into partial[blockIdx * KS + k0 + k]
__device__ inline void block_store(double (&acc)[KC], int kn, int k0, double *partial) {
  __shared__ double sh[4][KC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    double t = wave_sum(acc[k]);
    if (lane == 0) sh[w][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < kn) {
    const int k = threadIdx.x;
    partial[blockIdx.x * KS + k0 + k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_multidot(const double *__restrict__ V, int64_t n, int nv,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ partial) {
  for (int k0 = 0; k0 < nv; k0 += KC) {
    const int kn = min(KC, nv - k0);
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double wi = w[i];
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k < kn) acc[k] += V[(int64_t)(k0 + k) * n + i] * wi;
    }
    block_store(acc, kn, k0, partial);
  }
}

// w -= sum_k h[k] V_k; then partial dots of the new w with every V_k, or its norm^2
// all nv <= NVB dot products of one pass in registers: V and w are read once, and each
// block reduces its nv sums once
template <int NVB>
__global__ void __launch_bounds__(256) k_multidot_reg(const double *__restrict__ V, int64_t n,
                                                      int nv, const double *__restrict__ w,
                                                      double *__restrict__ partial) {
  double acc[NVB];
#pragma unroll
  for (int k = 0; k < NVB; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
    double t[NVB];
#pragma unroll
    for (int k = 0; k < NVB; ++k) t[k] = k < nv ? V[(int64_t)k * n + i] : 0.0;
#pragma unroll
    for (int k = 0; k < NVB; ++k) acc[k] += t[k] * wi;
  }
#pragma unroll
  for (int k0 = 0; k0 < NVB; k0 += KC) {
    if (k0 >= nv) break;
    double a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) a[k] = acc[k0 + k];
    block_store(a, min(KC, nv - k0), k0, partial);
  }
}

__global__ void __launch_bounds__(256) k_cgs_update(const double *__restrict__ V, int64_t n, int nv,
                                                    const double *__restrict__ h,
                                                    double *__restrict__ w,
                                                    double *__restrict__ partial, int norm_only) {
  __shared__ double sh_h[KS];
  for (int k = threadIdx.x; k < nv; k += blockDim.x) sh_h[k] = h[k];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double nacc = 0.0;
  for (int64_t i = i0; i < n; i += stride) {
    double wi = w[i];
    int k = 0;
    for (; k + 8 <= nv; k += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = V[(int64_t)(k + u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) wi -= sh_h[k + u] * t[u];
    }
    for (; k < nv; ++k) wi -= sh_h[k] * V[(int64_t)k * n + i];
    w[i] = wi;
    nacc += wi * wi;
  }
  if (norm_only) {
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    acc[0] = nacc;
    block_store(acc, 1, 0, partial);
    return;
  }
  for (int k0 = 0; k0 < nv; k0 += KC) {
    const int kn = min(KC, nv - k0);
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    for (int64_t i = i0; i < n; i += stride) {
      const double wi = w[i];
#pragma unroll
      for (int k = 0; k < KC; ++k)
        if (k < kn) acc[k] += V[(int64_t)(k0 + k) * n + i] * wi;
    }
    block_store(acc, kn, k0, partial);
  }
}

// First correction of CGS2 in one pass: w -= sum_k h[k] V_k and, with the same V_k(i)
// values still in registers, the partial dots of the new w with every V_k (the second
// projection).  NVB >= nv basis vectors per thread; the arithmetic and its order are those
// of k_cgs_update, which re-reads V for the dots.
// The rows are walked from the last one down: the pass before (the first projection)
// walked them upwards, so the rows it read last, still held by the memory-side cache, are
// read first.
template <int NVB>
__global__ void __launch_bounds__(256) k_cgs_fused(const double *__restrict__ V, int64_t n, int nv,
                                                   const double *__restrict__ h,
                                                   double *__restrict__ w,
                                                   double *__restrict__ partial) {
  __shared__ double sh_h[KS];
  for (int k = threadIdx.x; k < nv; k += blockDim.x) sh_h[k] = h[k];
  __syncthreads();
  double acc[NVB];
#pragma unroll
  for (int k = 0; k < NVB; ++k) acc[k] = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = n - 1 - r;
    double t[NVB];
#pragma unroll
    for (int k = 0; k < NVB; ++k) t[k] = k < nv ? V[(int64_t)k * n + i] : 0.0;
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < NVB; ++k)
      if (k < nv) wi -= sh_h[k] * t[k];
    w[i] = wi;
#pragma unroll
    for (int k = 0; k < NVB; ++k) acc[k] += t[k] * wi;
  }
#pragma unroll
  for (int k0 = 0; k0 < NVB; k0 += KC) {
    if (k0 >= nv) break;
    double a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) a[k] = acc[k0 + k];
    block_store(a, min(KC, nv - k0), k0, partial);
  }
}

__global__ void k_norm_partials(const double *__restrict__ r, int64_t n, double *__restrict__ partial) {
  double acc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc[0] += r[i] * r[i];
  block_store(acc, 1, 0, partial);
}
__global__ void k_dot_partials(const double *__restrict__ a, const double *__restrict__ b,
                               int64_t n, double *__restrict__ partial) {
  double acc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc[0] += a[i] * b[i];
  block_store(acc, 1, 0, partial);
}

// out[k] (+)= sum over blocks of partial[blk * KS + k]; one block per k, fixed order
__global__ void k_reduce_partials(const double *__restrict__ partial, int nblk,
                                  double *__restrict__ out, int add) {
  __shared__ double sh[256];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[b * KS + k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = add ? out[k] + sh[0] : sh[0];
}

// H column-major with leading dimension ldh; scal[0] = |g_{j+1}|, scal[1] = h_{j+1,j},
// scal[2] = 1 / h_{j+1,j} (0 at breakdown)
__global__ void k_givens(double *__restrict__ H, double *__restrict__ cs, double *__restrict__ sn,
                         double *__restrict__ g, const double *__restrict__ h1,
                         const double *__restrict__ h2, const double *__restrict__ hn2, int j,
                         int ldh, double *__restrict__ scal) {
  // the column and the earlier rotations are gathered by the whole block; one lane then
  // applies the rotations in order
  __shared__ double col[KS + 1], c[KS], sv[KS];
  const int t = threadIdx.x;
  for (int i = t; i <= j; i += blockDim.x) col[i] = h1[i] + h2[i];
  for (int i = t; i < j; i += blockDim.x) {
    c[i] = cs[i];
    sv[i] = sn[i];
  }
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(hn2[0]);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double u = c[i] * col[i] + sv[i] * col[i + 1];
      col[i + 1] = -sv[i] * col[i] + c[i] * col[i + 1];
      col[i] = u;
    }
    const double a = col[j], b = col[j + 1];
    const double r = hypot(a, b);
    cs[j] = r != 0.0 ? a / r : 1.0;
    sn[j] = r != 0.0 ? b / r : 0.0;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sn[j] * gj;
    g[j] = cs[j] * gj;
    scal[0] = fabs(g[j + 1]);
    scal[1] = hn;
    scal[2] = hn > 0.0 ? 1.0 / hn : 0.0;
  }
  __syncthreads();
  double *out = H + (int64_t)j * ldh;
  for (int i = t; i <= j + 1; i += blockDim.x) out[i] = col[i];
}

__global__ void k_scale(const double *__restrict__ w, const double *__restrict__ sc,
                        double *__restrict__ v, int64_t n) {
  const double a = sc[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * a;
}
// the same, also writing the new basis vector in the preconditioner's precision
template <class T>
__global__ void k_scale_copy(const double *__restrict__ w, const double *__restrict__ sc,
                             double *__restrict__ v, T *__restrict__ vt, int64_t n) {
  const double a = sc[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double u = w[i] * a;
    v[i] = u;
    vt[i] = static_cast<T>(u);
  }
}

__global__ void k_start(const double *__restrict__ r, double inv_beta, double beta,
                        double *__restrict__ V0, double *__restrict__ g, int64_t n, int mp1) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    V0[i] = r[i] * inv_beta;
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < mp1; k += blockDim.x) g[k] = k == 0 ? beta : 0.0;
}

__global__ void k_trisolve(const double *__restrict__ H, const double *__restrict__ g, int k,
                           int ldh, double *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= H[(int64_t)c * ldh + i] * y[c];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

__global__ void k_xupdate(const double *__restrict__ Z, int64_t n, int k,
                          const double *__restrict__ y, double *__restrict__ x) {
  __shared__ double sy[KS];
  for (int c = threadIdx.x; c < k; c += blockDim.x) sy[c] = y[c];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
    int c = 0;
    for (; c + 8 <= k; c += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = Z[(int64_t)(c + u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += t[u] * sy[c + u];
    }
    for (; c < k; ++c) s += Z[(int64_t)c * n + i] * sy[c];
    x[i] = s;
  }
}

unsigned sgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1u : (unsigned)g;
}

}  // namespace

int64_t stream_blocks(int64_t nnz) { return (nnz + SNNZ - 1) / SNNZ; }

void rowblocks64(const mgr_csr &A, int64_t nnz, int *rb, hipStream_t s) {
  const int64_t K = stream_blocks(nnz);
  k_rowblocks<<<grid_for(K + 1, 256), 256, 0, s>>>(A.nrows, A.row_ptr, K, rb);
  KCHK();
}

void spmv64_stream(const mgr_csr &A, int64_t nnz, const int *rb, const double *x, const double *b,
                   double *y, hipStream_t s) {
  const int64_t K = stream_blocks(nnz);
  if (K == 0) {
    if (A.nrows) launch_spmv64(A, x, b, y, s, 0.0);
    return;
  }
  k_spmv_stream<<<(unsigned)K, SB, 0, s>>>(rb, A.row_ptr, A.col, A.val, x, b, y);
  KCHK();
}

// BSR: windows of SNNZ / b^2 blocks (nnzb = number of blocks)
int64_t bsr_stream_blocks(int64_t nnzb, int bs) {
  const int64_t wb = bs == 3 ? WB3 : SNNZ / (bs * bs);
  return (nnzb + wb - 1) / wb;
}

void bsr_rowblocks64(const mgr_csr &A, int64_t nnzb, int *rb, hipStream_t s) {
  const int64_t K = bsr_stream_blocks(nnzb, A.block);
  if (A.block == 2)
    k_bsr_rowblocks<SNNZ / 4><<<grid_for(K + 1, 256), 256, 0, s>>>(A.nrows, A.row_ptr, K, rb);
  else
    k_bsr_rowblocks<WB3><<<grid_for(K + 1, 256), 256, 0, s>>>(A.nrows, A.row_ptr, K, rb);
  KCHK();
}

void bsr_spmv64_stream(const mgr_csr &A, int64_t nnzb, const int *rb, const double *x,
                       const double *b, double *y, hipStream_t s) {
  const int64_t K = bsr_stream_blocks(nnzb, A.block);
  if (K == 0) {   // no blocks: y = b (or 0)
    const int64_t n = A.nrows * A.block;
    if (n == 0) return;
    if (b) HIPCHK(hipMemcpyAsync(y, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemsetAsync(y, 0, n * sizeof(double), s));
    return;
  }
  if (A.block == 2)
    k_bsr_stream<2><<<(unsigned)K, SB, 0, s>>>(rb, A.row_ptr, A.col, A.val, x, b, y);
  else
    k_bsr3_lane<<<(unsigned)K, SB, 0, s>>>(rb, A.row_ptr, A.col, A.val, x, b, y);
  KCHK();
}

void spmv64(const mgr_csr &A, const double *x, double *y, hipStream_t s) {
  int64_t nnz = 0;
  if (A.nrows) {
    HIPCHK(hipMemcpyAsync(&nnz, A.row_ptr + A.nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (A.block > 1) {
    DArr<int> rb(bsr_stream_blocks(nnz, A.block) + 1, s);
    bsr_rowblocks64(A, nnz, rb.p, s);
    bsr_spmv64_stream(A, nnz, rb.p, x, nullptr, y, s);
    return;
  }
  DArr<int> rb(stream_blocks(nnz) + 1, s);
  rowblocks64(A, nnz, rb.p, s);
  spmv64_stream(A, nnz, rb.p, x, nullptr, y, s);
}

int krylov_partials_blocks() { return NB * KS; }

// Blocks of 256 threads of `kernel` that are resident on the device at once (at most NB):
// a grid of that size runs in a single round, without a partly filled last one.
static int resident_grid(const void *kernel) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, int> cache;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({dev, kernel});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int g = std::max(1, std::min(NB, per_cu * cus));
  cache[{dev, kernel}] = g;
  return g;
}

int multidot_partials(const double *V, int64_t n, int nv, const double *w, double *partial,
                      hipStream_t s) {
#define MDR(NVB)                                                                       \
  {                                                                                    \
    const int g = resident_grid(reinterpret_cast<const void *>(&k_multidot_reg<NVB>)); \
    k_multidot_reg<NVB><<<g, 256, 0, s>>>(V, n, nv, w, partial);                        \
    KCHK();                                                                            \
    return g;                                                                          \
  }
  if (nv <= 16) MDR(16)
  if (nv <= 32) MDR(32)
  if (nv <= 48) MDR(48)
  if (nv <= 64) MDR(64)
#undef MDR
  k_multidot<<<NB, 256, 0, s>>>(V, n, nv, w, partial);
  KCHK();
  return NB;
}
int cgs_update_partials(const double *V, int64_t n, int nv, const double *h, double *w,
                        double *partial, bool norm_only, hipStream_t s) {
  // the fused pass holds nv basis values per thread; beyond 48 they would not fit the
  // register file, and the two-pass form is used
  if (!norm_only && nv <= 48) {
#define CGF(NVB)                                                                    \
  {                                                                                 \
    const int g = resident_grid(reinterpret_cast<const void *>(&k_cgs_fused<NVB>)); \
    k_cgs_fused<NVB><<<g, 256, 0, s>>>(V, n, nv, h, w, partial);                     \
    KCHK();                                                                         \
    return g;                                                                       \
  }
    if (nv <= 16) CGF(16)
    if (nv <= 32) CGF(32)
    CGF(48)
#undef CGF
  }
  k_cgs_update<<<NB, 256, 0, s>>>(V, n, nv, h, w, partial, norm_only ? 1 : 0);
  KCHK();
  return NB;
}
void reduce_partials(const double *partial, int nblk, int nv, double *out, bool add,
                     hipStream_t s) {
  k_reduce_partials<<<nv, 256, 0, s>>>(partial, nblk, out, add ? 1 : 0);
  KCHK();
}
void givens_step(double *H, double *cs, double *sn, double *g, const double *h1, const double *h2,
                 const double *hn2, int j, int ldh, double *scal, double *unused, hipStream_t s) {
  (void)unused;
  k_givens<<<1, 64, 0, s>>>(H, cs, sn, g, h1, h2, hn2, j, ldh, scal);
  KCHK();
}
void scale_vec(const double *w, const double *scale, double *v, int64_t n, hipStream_t s) {
  k_scale<<<sgrid(n), 256, 0, s>>>(w, scale, v, n);
  KCHK();
}
void scale_vec_copy(const double *w, const double *scale, double *v, float *vf, int64_t n,
                    hipStream_t s) {
  k_scale_copy<float><<<sgrid(n), 256, 0, s>>>(w, scale, v, vf, n);
  KCHK();
}
void scale_vec_copy(const double *w, const double *scale, double *v, double *vd, int64_t n,
                    hipStream_t s) {
  k_scale_copy<double><<<sgrid(n), 256, 0, s>>>(w, scale, v, vd, n);
  KCHK();
}
void tri_solve_and_update(const double *H, const double *g, int k, int ldh, const double *Z,
                          int64_t n, double *x, double *y, hipStream_t s) {
  if (k <= 0) return;
  k_trisolve<<<1, 64, 0, s>>>(H, g, k, ldh, y);
  KCHK();
  k_xupdate<<<sgrid(n), 256, 0, s>>>(Z, n, k, y, x);
  KCHK();
}
int norm2_partials(const double *r, int64_t n, double *partial, hipStream_t s) {
  k_norm_partials<<<NB, 256, 0, s>>>(r, n, partial);
  KCHK();
  return NB;
}
int dot_partials(const double *a, const double *b, int64_t n, double *partial, hipStream_t s) {
  k_dot_partials<<<NB, 256, 0, s>>>(a, b, n, partial);
  KCHK();
  return NB;
}
void start_cycle_host_beta(const double *r, double beta, double *V0, double *g, int64_t n, int mp1,
                           hipStream_t s) {
  k_start<<<sgrid(n), 256, 0, s>>>(r, 1.0 / beta, beta, V0, g, n, mp1);
  KCHK();
}
void resid64(const mgr_csr &A, const double *x, const double *b, double *r, hipStream_t s) {
  launch_spmv64(A, x, b, r, s, 1e9);
}
void spmv64_avg(const mgr_csr &A, const double *x, const double *b, double *y, double avg,
                hipStream_t s) {
  launch_spmv64(A, x, b, y, s, avg);
}

}  // namespace mgr

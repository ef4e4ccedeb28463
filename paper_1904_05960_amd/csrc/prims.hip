// Device primitives: exclusive scans, reductions, fills, casts, streaming copy.
#include <mutex>

#include "common.hpp"

namespace mgr {

namespace {
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive scan over the 256 threads of a block; *total receives the block sum
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *total) {
  __shared__ int64_t sh[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_BLOCK / 64; ++i) {
    if (i < w) off += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

template <class T>
__global__ void k_tile_sum(const T *__restrict__ in, int64_t n, int64_t *__restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += (int64_t)in[base + k];
  int64_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ void k_tile_scan(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                            const int64_t *__restrict__ tile_base,
                            int64_t *__restrict__ total64 = nullptr) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t vals[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    vals[k] = (base + k < n) ? (int64_t)in[base + k] : 0;
    s += vals[k];
  }
  int64_t tot;
  int64_t off = block_excl_scan(s, &tot) + (tile_base ? tile_base[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = (T)off;
    off += vals[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) {
    out[n] = (T)off;
    if (total64) *total64 = off;
  }
}

// in-place-safe scan of int64 tile sums into an exclusive prefix (recursive)
void scan_i64_impl(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (ntiles <= 1) {
    k_tile_scan<int64_t><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, nullptr);
    KCHK();
    return;
  }
  DArr<int64_t> sums(ntiles + 1, s);
  k_tile_sum<int64_t><<<ntiles, SCAN_BLOCK, 0, s>>>(in, n, sums.p);
  KCHK();
  scan_i64_impl(sums.p, sums.p, ntiles, s);
  k_tile_scan<int64_t><<<ntiles, SCAN_BLOCK, 0, s>>>(in, out, n, sums.p);
  KCHK();
}

template <class T>
int64_t scan_generic(const T *in, T *out, int64_t n, hipStream_t s) {
  if (n == 0) {
    T z = 0;
    HIPCHK(hipMemcpyAsync(out, &z, sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
  }
  const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  DArr<int64_t> sums(ntiles + 1, s);
  k_tile_sum<T><<<ntiles, SCAN_BLOCK, 0, s>>>(in, n, sums.p);
  KCHK();
  scan_i64_impl(sums.p, sums.p, ntiles, s);
  k_tile_scan<T><<<ntiles, SCAN_BLOCK, 0, s>>>(in, out, n, sums.p);
  KCHK();
  // the true total in 64 bits (the output type may be narrower)
  int64_t h = 0;
  d2h_sync(&h, sums.p + ntiles, sizeof(int64_t), s);
  return h;
}

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T, class Op>
__global__ void k_reduce(const T *__restrict__ p, int64_t n, T init, T *__restrict__ out,
                         Op op) {
  __shared__ T sh[256];
  T acc = init;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc = op(acc, p[i]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

struct MaxOp {
  template <class T> __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct SumOp {
  template <class T> __device__ T operator()(T a, T b) const { return a + b; }
};

template <class T, class Op>
T reduce_generic(const T *p, int64_t n, T init, Op op, hipStream_t s) {
  const int blocks = 512;
  DArr<T> part(blocks, s);
  k_reduce<T, Op><<<blocks, 256, 0, s>>>(p, n, init, part.p, op);
  KCHK();
  DArr<T> fin(1, s);
  k_reduce<T, Op><<<1, 256, 0, s>>>(part.p, blocks, init, fin.p, op);
  KCHK();
  T h;
  d2h_sync(&h, fin.p, sizeof(T), s);
  return h;
}

__global__ void k_cast_d2f(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}
__global__ void k_cast_f2d(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}
__global__ void k_neg(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = -p[i];
}
__global__ void k_rp64to32(const int64_t *__restrict__ a, int *__restrict__ b, int64_t n,
                           int *flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = a[i];
    if (v < 0 || v > 0x7fffffffLL) atomicOr(flag, FLAG_OVERFLOW);
    b[i] = (int)v;
  }
}
__global__ void k_rp32to64(const int *__restrict__ a, int64_t *__restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
// dst = src, 16 bytes per lane per iteration
__global__ void k_stream_copy(const double2 *__restrict__ a, double2 *__restrict__ b,
                              int64_t n2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void k_copy_tail(const double *a, double *b, int64_t from, int64_t n) {
  int64_t i = from + threadIdx.x;
  if (i < n) b[i] = a[i];
}

unsigned stride_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  return g < 1 ? 1u : (unsigned)g;
}
}  // namespace

void *pinned_scratch();
int64_t exclusive_scan_i32(const int *in, int *out, int64_t n, hipStream_t s) {
  int64_t t = scan_generic<int>(in, out, n, s);
  require(t <= 0x7fffffffLL, MGR_ERR_UNSUPPORTED, "prefix sum exceeds 2^31 (matrix too large)");
  return t;
}
// the same scan with nothing read back: out[n] is written, and the total in 64 bits into
// *total64 (device memory) when given
void exclusive_scan_i32_async(const int *in, int *out, int64_t n, hipStream_t s,
                              int64_t *total64) {
  if (n == 0) {
    fill<int>(out, 0, 1, s);
    if (total64) fill<int64_t>(total64, 0, 1, s);
    return;
  }
  const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  DArr<int64_t> sums(ntiles + 1, s);
  k_tile_sum<int><<<ntiles, SCAN_BLOCK, 0, s>>>(in, n, sums.p);
  KCHK();
  scan_i64_impl(sums.p, sums.p, ntiles, s);
  k_tile_scan<int><<<ntiles, SCAN_BLOCK, 0, s>>>(in, out, n, sums.p, total64);
  KCHK();
}
int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  return scan_generic<int64_t>(in, out, n, s);
}

template <class T>
void fill(T *p, T val, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill<T><<<stride_grid(n), 256, 0, s>>>(p, val, n);
  KCHK();
}
template void fill<int>(int *, int, int64_t, hipStream_t);
template void fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template void fill<double>(double *, double, int64_t, hipStream_t);
template void fill<float>(float *, float, int64_t, hipStream_t);
template void fill<int8_t>(int8_t *, int8_t, int64_t, hipStream_t);
template void fill<uint64_t>(uint64_t *, uint64_t, int64_t, hipStream_t);
template void fill<unsigned long long>(unsigned long long *, unsigned long long, int64_t, hipStream_t);
template void fill<unsigned char>(unsigned char *, unsigned char, int64_t, hipStream_t);

int64_t reduce_max_i64(const int64_t *p, int64_t n, hipStream_t s) {
  return reduce_generic<int64_t>(p, n, INT64_MIN, MaxOp(), s);
}
int64_t reduce_sum_i32(const int *p, int64_t n, hipStream_t s) {
  // sum as int per block is safe for the small counts this is used on
  return (int64_t)reduce_generic<int>(p, n, 0, SumOp(), s);
}
double reduce_max_f64(const double *p, int64_t n, hipStream_t s) {
  return reduce_generic<double>(p, n, -1.0 / 0.0, MaxOp(), s);
}

void cast_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_d2f<<<stride_grid(n), 256, 0, s>>>(in, out, n);
  KCHK();
}
void cast_f32_to_f64(const float *in, double *out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_f2d<<<stride_grid(n), 256, 0, s>>>(in, out, n);
  KCHK();
}
void negate_f64(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_neg<<<stride_grid(n), 256, 0, s>>>(p, n);
  KCHK();
}
void rowptr64_to_32(const int64_t *in, int *out, int64_t n1, int *flag, hipStream_t s) {
  k_rp64to32<<<stride_grid(n1), 256, 0, s>>>(in, out, n1, flag);
  KCHK();
}
void rowptr32_to_64(const int *in, int64_t *out, int64_t n1, hipStream_t s) {
  k_rp32to64<<<stride_grid(n1), 256, 0, s>>>(in, out, n1);
  KCHK();
}
void stream_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    // one 16-byte element per thread: on this device a grid-stride copy with fewer,
    // longer-lived threads moves 15-20 % less per second
    int64_t g = (n2 + 255) / 256;
    if (g > 0x7fffffff) g = 0x7fffffff;
    k_stream_copy<<<(unsigned)g, 256, 0, s>>>(reinterpret_cast<const double2 *>(src),
                                              reinterpret_cast<double2 *>(dst), n2);
    KCHK();
  }
  if (n & 1) {
    k_copy_tail<<<1, 64, 0, s>>>(src, dst, 2 * n2, n);
    KCHK();
  }
}
// small pinned host buffer for the scalar reads of a solve loop (one per calling thread)
void *pinned_scratch() {
  thread_local void *buf = nullptr;
  if (!buf) HIPCHK(hipHostMalloc(&buf, 256, hipHostMallocDefault));
  return buf;
}

// Reads of a few bytes that the host needs before it can go on (sizes, counts, flags: the
// setup makes a few hundred of them, one after another).  The copy lands in a pinned buffer
// taken from a pool shared by all host threads (the setup's helper threads come and go),
// and the host polls the copy's completion event instead of blocking in the runtime: a
// blocking wait is woken some tens of microseconds after the GPU is done, a poll within a
// few.
namespace {
struct PinnedRead {
  void *p = nullptr;
  hipEvent_t ev = nullptr;
  int dev = -1;
};
std::mutex g_pin_mu;
std::vector<PinnedRead> g_pin_pool;   // kept until the process ends
}  // namespace

void d2h_sync(void *dst, const void *src, size_t bytes, hipStream_t s) {
  const D2HPart part{dst, src, bytes};
  d2h_sync_parts(&part, 1, s);
}

void d2h_sync_parts(const D2HPart *parts, int np, hipStream_t s) {
  size_t total = 0;
  for (int i = 0; i < np; ++i) total += (parts[i].bytes + 15) / 16 * 16;
  require(total <= 256, MGR_ERR_ARG, "d2h_sync: at most 256 bytes");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  PinnedRead b;
  {
    std::lock_guard<std::mutex> g(g_pin_mu);
    for (size_t i = 0; i < g_pin_pool.size(); ++i)
      if (g_pin_pool[i].dev == dev) {
        b = g_pin_pool[i];
        g_pin_pool[i] = g_pin_pool.back();
        g_pin_pool.pop_back();
        break;
      }
  }
  struct Back {
    PinnedRead &b;
    ~Back() {
      if (!b.p) return;
      std::lock_guard<std::mutex> g(g_pin_mu);
      g_pin_pool.push_back(b);
    }
  } back{b};
  if (!b.p) {
    b.dev = dev;
    HIPCHK(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    HIPCHK(hipHostMalloc(&b.p, 256, hipHostMallocDefault));
  }
  size_t off = 0;
  for (int i = 0; i < np; ++i) {
    if (parts[i].bytes)
      HIPCHK(hipMemcpyAsync(static_cast<char *>(b.p) + off, parts[i].src, parts[i].bytes,
                            hipMemcpyDeviceToHost, s));
    off += (parts[i].bytes + 15) / 16 * 16;
  }
  HIPCHK(hipEventRecord(b.ev, s));
  for (;;) {
    const hipError_t e = hipEventQuery(b.ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) HIPCHK(e);
  }
  off = 0;
  for (int i = 0; i < np; ++i) {
    if (parts[i].bytes) std::memcpy(parts[i].dst, static_cast<char *>(b.p) + off, parts[i].bytes);
    off += (parts[i].bytes + 15) / 16 * 16;
  }
}

int read_flag(const int *dflag, hipStream_t s) {
  int h = 0;
  d2h_sync(&h, dflag, sizeof(int), s);
  return h;
}
void clear_flag(int *dflag, hipStream_t s) { fill<int>(dflag, 0, 1, s); }

void check_flags(const int *dflag, hipStream_t s, const char *where) {
  const int f = read_flag(dflag, s);
  if (f == 0) return;
  const std::string w = std::string(" (") + where + ")";
  if (f & FLAG_BAD_LABEL) throw Error(MGR_ERR_ARG, "labels must lie in [0, 7]" + w);
  if (f & FLAG_OVERFLOW) throw Error(MGR_ERR_ARG, "row pointers out of range" + w);
  if (f & FLAG_ZERO_PIVOT)
    throw Error(MGR_ERR_ZERO_PIVOT, "zero or missing pivot (D_FF, AMG diagonal, block or dense inverse)" + w);
  if (f & FLAG_NOT_BLOCKED) throw Error(MGR_ERR_UNSUPPORTED, "nodal level without full 3x3 blocks" + w);
  if (f & FLAG_ROW_TOO_LONG) throw Error(MGR_ERR_UNSUPPORTED, "a product row exceeds the supported length" + w);
  throw Error(MGR_ERR_HIP, "internal consistency check failed (flag " + std::to_string(f) + ")" + w);
}

}  // namespace mgr

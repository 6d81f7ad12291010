// Device-wide scans and the stable radix sort used by the Morton grid.
//
// The check-point sort of Alg. 1 (step 2) must be stable: equal Morton IDs
// keep ascending global check-point index (Sec. 3.3.1, Table 3).  An LSD
// radix sort with stable per-digit scatter gives exactly that.
#include "stiv_common.h"

namespace stiv {

namespace {

constexpr int kScanThreads = 1024;

// Block-wide inclusive scan of one value per thread (1024 threads): a
// shuffle scan inside each wavefront, the 16 wavefront totals scanned by
// the first wavefront, two workgroup barriers in all.  sh needs 16 entries.
template <typename T>
__device__ T block_inclusive_scan(T v, T *sh) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    T w = lane < kScanThreads / 64 ? sh[lane] : T(0);
#pragma unroll
    for (int off = 1; off < kScanThreads / 64; off <<= 1) {
      const T u = __shfl_up(w, off, 64);
      if (lane >= off) w += u;
    }
    if (lane < kScanThreads / 64) sh[lane] = w;
  }
  __syncthreads();
  const T r = v + (wave ? sh[wave - 1] : T(0));
  __syncthreads();  // sh may be reused by the caller's next scan
  return r;
}

template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_excl(const TIn *in, int64_t *out,
                                                            const unsigned long long *n_dev, int64_t n_host) {
  __shared__ int64_t sh[kScanThreads];
  // n = n_host, or min(*n_dev, n_host) when a device count is given
  int64_t n = n_host;
  if (n_dev) n = (int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host;
  const int t = threadIdx.x;
  const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)t * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += (int64_t)in[i];
  int64_t inc = block_inclusive_scan<int64_t>(s, sh);
  int64_t base = inc - s;
  for (int64_t i = lo; i < hi; ++i) {
    int64_t v = (int64_t)in[i];
    out[i] = base;
    base += v;
  }
  if (t == kScanThreads - 1) out[n] = inc;
}

// Single-workgroup LSD radix sort, 4-bit digits, stable.  Each thread owns a
// contiguous chunk, so the scatter order within a digit follows input order.
__global__ __launch_bounds__(kScanThreads) void k_radix_1wg(uint64_t *keys, uint32_t *vals, uint64_t *tk,
                                                            uint32_t *tv, const unsigned long long *n_dev,
                                                            int64_t n_host, int key_bits) {
  __shared__ int32_t cnt[16 * kScanThreads];
  __shared__ int64_t sh[kScanThreads];
  int64_t n = n_host;
  if (n_dev) n = (int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host;
  const int t = threadIdx.x;
  const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)t * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  // only the bits below the largest key need passes
  {
    __shared__ unsigned long long kmax;
    if (t == 0) kmax = 0;
    __syncthreads();
    uint64_t m = 0;
    for (int64_t i = lo; i < hi; ++i) m = keys[i] > m ? keys[i] : m;
    if (m) atomicMax(&kmax, (unsigned long long)m);
    __syncthreads();
    const int used = kmax ? 64 - __clzll((long long)kmax) : 0;
    key_bits = used < key_bits ? used : key_bits;
    __syncthreads();
  }
  uint64_t *sk = keys, *dk = tk;
  uint32_t *sv = vals, *dv = tv;
  int passes = 0;
  for (int shift = 0; shift < key_bits; shift += 4, ++passes) {
    for (int dgt = 0; dgt < 16; ++dgt) cnt[dgt * kScanThreads + t] = 0;
    for (int64_t i = lo; i < hi; ++i) cnt[(int)((sk[i] >> shift) & 15u) * kScanThreads + t]++;
    __syncthreads();
    // exclusive scan in flat (digit, thread) order; thread t covers 16 entries
    int32_t loc[16];
    int64_t s = 0;
    for (int k = 0; k < 16; ++k) {
      loc[k] = cnt[t * 16 + k];
      s += loc[k];
    }
    int64_t inc = block_inclusive_scan<int64_t>(s, sh);
    int64_t base = inc - s;
    for (int k = 0; k < 16; ++k) {
      int32_t v = loc[k];
      cnt[t * 16 + k] = (int32_t)base;
      base += v;
    }
    __syncthreads();
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t k = sk[i];
      int dgt = (int)((k >> shift) & 15u);
      int32_t pos = cnt[dgt * kScanThreads + t]++;
      dk[pos] = k;
      dv[pos] = sv[i];
    }
    __threadfence_block();
    __syncthreads();
    uint64_t *xk = sk; sk = dk; dk = xk;
    uint32_t *xv = sv; sv = dv; dv = xv;
  }
  if (passes & 1) {
    for (int64_t i = t; i < n; i += kScanThreads) {
      keys[i] = sk[i];
      vals[i] = sv[i];
    }
  }
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_iota_u32(uint32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

void launch_scan_i64(const int64_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                     hipStream_t st) {
  k_scan_excl<int64_t><<<1, kScanThreads, 0, st>>>(in, out, n_dev, n_host);
}
void launch_scan_i32_to_i64(const int32_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                            hipStream_t st) {
  k_scan_excl<int32_t><<<1, kScanThreads, 0, st>>>(in, out, n_dev, n_host);
}
void launch_radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *tk, uint32_t *tv,
                           const unsigned long long *n_dev, int64_t n_host, int key_bits, hipStream_t st) {
  k_radix_1wg<<<1, kScanThreads, 0, st>>>(keys, vals, tk, tv, n_dev, n_host, key_bits);
}
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill_u64<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
}
void launch_iota_u32(uint32_t *p, int64_t n, hipStream_t st) {
  if (n > 0) k_iota_u32<<<grid_for(n, 256), 256, 0, st>>>(p, n);
}
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill_i32<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
}

}  // namespace stiv

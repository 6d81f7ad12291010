// Device-wide scans and the stable radix sort used by the Morton grid.
//
// The check-point sort of Alg. 1 (step 2) must be stable: equal Morton IDs
// keep ascending global check-point index (Sec. 3.3.1, Table 3).  An LSD
// radix sort with stable per-digit scatter gives exactly that.
#include "stiv_common.h"

namespace stiv {

namespace {

constexpr int kScanThreads = 1024;

// Block-wide inclusive scan of one value per thread (NT threads, at most
// 4096): a shuffle scan inside each wavefront, the wavefront totals scanned
// by the first wavefront, two workgroup barriers in all.  sh needs NT / 64
// entries.
template <typename T, int NT = kScanThreads>
__device__ T block_inclusive_scan(T v, T *sh) {
  static_assert(NT % 64 == 0 && NT / 64 <= 64, "whole wavefronts, totals in one wavefront");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  if (wave == 0) {
    T w = lane < NT / 64 ? sh[lane] : T(0);
#pragma unroll
    for (int off = 1; off < NT / 64; off <<= 1) {
      const T u = __shfl_up(w, off, 64);
      if (lane >= off) w += u;
    }
    if (lane < NT / 64) sh[lane] = w;
  }
  __syncthreads();
  const T r = v + (wave ? sh[wave - 1] : T(0));
  __syncthreads();  // sh may be reused by the caller's next scan
  return r;
}

constexpr int kScanItems = 8, kScanChunk = kScanThreads * kScanItems;

// Exclusive scan in one workgroup: tiles of kScanChunk elements (each thread
// owns kScanItems consecutive ones), a block scan per tile and a running
// carry between tiles; out[n] gets the total.
template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_excl(const TIn *in, int64_t *out,
                                                            const unsigned long long *n_dev, int64_t n_host) {
  __shared__ int64_t sh[kScanThreads / 64];
  __shared__ int64_t tile_total;
  // n = n_host, or min(*n_dev, n_host) when a device count is given
  int64_t n = n_host;
  if (n_dev) n = (int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host;
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < n; t0 += kScanChunk) {
    const int64_t i0 = t0 + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = (i0 + j < n) ? (int64_t)in[i0 + j] : 0;
      s += v[j];
    }
    const int64_t inc = block_inclusive_scan<int64_t>(s, sh);
    int64_t base = carry + inc - s;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (i0 + j < n) out[i0 + j] = base;
      base += v[j];
    }
    if (threadIdx.x == kScanThreads - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// --------------------------------------------------------------------------
// Multi-workgroup stable LSD radix sort, 8-bit digits.  A workgroup of 256
// threads owns a tile of 2048 consecutive keys, laid out [wavefront][round]
// [lane]: per pass, (1) a digit histogram per tile, written digit-major;
// (2) an exclusive scan of it, which is the first output position of each
// (digit, tile); (3) every key's rank among the equal digits before it in
// its tile -- matched across the wavefront by ballots on the 8 digit bits,
// carried across rounds and wavefronts in LDS -- gives its output position.
// Up to kRsFusedMaxBlocks tiles, (2) and (3) are one launch (k_rs_pass: each
// workgroup sums the histogram itself), so a pass costs two launches; there,
// a pass whose digit is the same for every key moves nothing.  Which of the
// two buffers holds a pass's input is kept on the device (the key count is
// read there too), and a last launch copies the result to buffer 0 if needed.
// Equal keys keep their input order (stable), as Alg. 1 requires.
// --------------------------------------------------------------------------
constexpr int kRsThreads = 256, kRsItems = 8, kRsTile = kRsThreads * kRsItems, kRsWaves = kRsThreads / 64;
static_assert(kRsThreads == 256, "one thread per digit in the histogram and offset steps");

__device__ inline int64_t rs_count(const unsigned long long *n_dev, int64_t n_host) {
  return n_dev ? ((int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host) : n_host;
}

// The two key / value buffers of the sort; which one holds the input of pass p
// is par[p] (device memory, written by the pass before; pass 0 reads buffer 0).
struct RsBufs {
  uint64_t *k[2];
  uint32_t *v[2];
};
__device__ inline int rs_cur(const int64_t *par, int p) { return p > 0 ? (int)par[p] : 0; }
// The digit at shift is the same in every key (bits: OR of the keys, OR of
// their complements; a bit that varies is set in both).
__device__ inline bool rs_digit_constant(const unsigned long long *bits, int shift) {
  return bits && (((bits[0] & bits[1]) >> shift) & 255ull) == 0;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(RsBufs B, const int64_t *par, int p,
                                                        const unsigned long long *n_dev, int64_t n_host, int shift,
                                                        int32_t *hist, int nblk, bool full_only,
                                                        const unsigned long long *bits) {
  __shared__ int h[256];
  if (rs_digit_constant(bits, shift)) return;  // the pass moves nothing and reads no histogram
  const uint64_t *keys = B.k[rs_cur(par, p)];
  const int64_t n = rs_count(n_dev, n_host);
  const int t = threadIdx.x, b = blockIdx.x;
  // with full_only, tiles past the count are never read (k_rs_pass stops at the
  // last tile that holds keys); the multi-launch scan reads every tile
  if (full_only && (int64_t)b * kRsTile >= n) return;
  h[t] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)b * kRsTile;
  for (int k = t; k < kRsTile; k += kRsThreads) {
    const int64_t e = e0 + k;
    if (e < n) atomicAdd(&h[(int)((keys[e] >> shift) & 255u)], 1);
  }
  __syncthreads();
  hist[(int64_t)t * nblk + b] = h[t];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(RsBufs B, int64_t *par, int p,
                                                           const unsigned long long *n_dev, int64_t n_host, int shift,
                                                           const int64_t *hoff, int nblk,
                                                           const unsigned long long *bits) {
  __shared__ int wcnt[kRsWaves][256];
  __shared__ int woff[kRsWaves][256];
  const int64_t n = rs_count(n_dev, n_host);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, b = blockIdx.x;
  const int cur = rs_cur(par, p);
  const uint64_t *sk = B.k[cur];
  const uint32_t *sv = B.v[cur];
  uint64_t *dk = B.k[cur ^ 1];
  uint32_t *dv = B.v[cur ^ 1];
  if (rs_digit_constant(bits, shift)) {
    if (b == 0 && t == 0) par[p + 1] = cur;
    return;
  }
  if (b == 0 && t == 0) par[p + 1] = cur ^ 1;
  for (int k = t; k < kRsWaves * 256; k += kRsThreads) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t base = (int64_t)b * kRsTile + (int64_t)w * (kRsItems * 64);
  uint64_t key[kRsItems];
  uint32_t val[kRsItems];
  int dg[kRsItems], rank[kRsItems];
#pragma unroll
  for (int j = 0; j < kRsItems; ++j) {
    const int64_t e = base + j * 64 + lane;
    const bool valid = e < n;
    key[j] = valid ? sk[e] : 0ull;
    val[j] = valid ? sv[e] : 0u;
    const int d = valid ? (int)((key[j] >> shift) & 255u) : 0;
    dg[j] = valid ? d : -1;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1;
      const unsigned long long m = __ballot(on);
      peers &= on ? m : ~m;
    }
    int pre = 0;
    if (valid) pre = wcnt[w][d];
    rank[j] = pre + __popcll(peers & lt);
    // the last lane of each group of equal digits advances the wavefront's count
    if (valid && (peers >> lane) == 1ull) wcnt[w][d] = pre + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    int run = 0;
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) {
      woff[ww][t] = run;
      run += wcnt[ww][t];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRsItems; ++j) {
    if (dg[j] < 0) continue;
    const int64_t dst = hoff[(int64_t)dg[j] * nblk + b] + woff[w][dg[j]] + rank[j];
    dk[dst] = key[j];
    dv[dst] = val[j];
  }
}

// Offsets and scatter of one pass in one launch, for inputs of at most
// kRsFusedMaxBlocks tiles: each workgroup finds the output position of its
// tile's first key of every digit from the whole histogram of the pass
// (counts of all smaller digits in every tile, plus this digit in the tiles
// before), then ranks and scatters its keys as k_rs_scatter does.  This
// replaces the scan launches between the histogram and the scatter.
constexpr int kRsFusedMaxBlocks = 256;
__global__ __launch_bounds__(kRsThreads) void k_rs_pass(RsBufs B, int64_t *par, int p,
                                                        const unsigned long long *n_dev, int64_t n_host, int shift,
                                                        const int32_t *hin, int nblk, const unsigned long long *bits) {
  __shared__ int wcnt[kRsWaves][256];
  __shared__ int woff[kRsWaves][256];
  __shared__ int64_t dbase[256];
  __shared__ int64_t sh[kRsWaves];
  __shared__ int s_const;
  const int64_t n = rs_count(n_dev, n_host);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, b = blockIdx.x;
  const int cur = rs_cur(par, p);
  const uint64_t *sk = B.k[cur];
  const uint32_t *sv = B.v[cur];
  uint64_t *dk = B.k[cur ^ 1];
  uint32_t *dv = B.v[cur ^ 1];
  if (n == 0 || rs_digit_constant(bits, shift)) {
    if (b == 0 && t == 0) par[p + 1] = cur;
    return;
  }
  // tiles that hold keys (the grid is sized for the capacity, the count is
  // read on the device); the others have nothing to place
  const int nfull = (int)((n + kRsTile - 1) / kRsTile);
  if (b >= nfull) return;
  if (t == 0) s_const = 0;
  __syncthreads();
  {
    // thread t: digit t
    int64_t tot = 0, before = 0;
    const int32_t *row = hin + (int64_t)t * nblk;
    for (int bb = 0; bb < nfull; ++bb) {
      const int c = row[bb];
      tot += c;
      before += bb < b ? c : 0;
    }
    if (tot == n) s_const = 1;  // every key has digit t
    const int64_t inc = block_inclusive_scan<int64_t, kRsThreads>(tot, sh);
    dbase[t] = inc - tot + before;
  }
  __syncthreads();
  // a digit shared by all keys leaves the order as it is (the sort is
  // stable): nothing moves and the next pass reads the same buffer.  Keys
  // of a few levels of the Morton grid leave their high digits constant.
  const bool constant = s_const != 0;
  if (b == 0 && t == 0) par[p + 1] = constant ? cur : cur ^ 1;
  if (constant) return;
  for (int k = t; k < kRsWaves * 256; k += kRsThreads) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t base = (int64_t)b * kRsTile + (int64_t)w * (kRsItems * 64);
  uint64_t key[kRsItems];
  uint32_t val[kRsItems];
  int dg[kRsItems], rank[kRsItems];
#pragma unroll
  for (int j = 0; j < kRsItems; ++j) {
    const int64_t e = base + j * 64 + lane;
    const bool valid = e < n;
    key[j] = valid ? sk[e] : 0ull;
    val[j] = valid ? sv[e] : 0u;
    const int d = valid ? (int)((key[j] >> shift) & 255u) : 0;
    dg[j] = valid ? d : -1;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1;
      const unsigned long long m = __ballot(on);
      peers &= on ? m : ~m;
    }
    int pre = 0;
    if (valid) pre = wcnt[w][d];
    rank[j] = pre + __popcll(peers & lt);
    if (valid && (peers >> lane) == 1ull) wcnt[w][d] = pre + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    int run = 0;
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) {
      woff[ww][t] = run;
      run += wcnt[ww][t];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRsItems; ++j) {
    if (dg[j] < 0) continue;
    const int64_t dst = dbase[dg[j]] + woff[w][dg[j]] + rank[j];
    dk[dst] = key[j];
    dv[dst] = val[j];
  }
}

// The sorted keys to buffer 0 when the last pass left them in buffer 1.
__global__ void k_rs_copy(RsBufs B, const int64_t *par, int passes, const unsigned long long *n_dev, int64_t n_host) {
  if (rs_cur(par, passes) == 0) return;
  const int64_t n = rs_count(n_dev, n_host);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    B.k[0][i] = B.k[1][i];
    B.v[0][i] = B.v[1][i];
  }
}

// --------------------------------------------------------------------------
// Multi-workgroup exclusive scan (reduce, scan the workgroup sums, scan each
// chunk with its offset) for long inputs; the single-workgroup kernel above
// serves short ones.
// --------------------------------------------------------------------------
template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const TIn *in, const unsigned long long *n_dev,
                                                            int64_t n_host, int64_t *sums) {
  __shared__ int64_t sh[kScanThreads / 64];
  const int64_t n = n_dev ? ((int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host) : n_host;
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  int64_t s = 0;
  for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads) {
    const int64_t i = c0 + k;
    if (i < n) s += (int64_t)in[i];
  }
  const int64_t inc = block_inclusive_scan<int64_t>(s, sh);
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = inc;
}

template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const TIn *in, int64_t *out,
                                                              const unsigned long long *n_dev, int64_t n_host,
                                                              const int64_t *soff, int nblk) {
  __shared__ int64_t sh[kScanThreads / 64];
  const int64_t n = n_dev ? ((int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host) : n_host;
  // each thread owns kScanItems consecutive elements of the chunk
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (i0 + j < n) ? (int64_t)in[i0 + j] : 0;
    s += v[j];
  }
  const int64_t inc = block_inclusive_scan<int64_t>(s, sh);
  int64_t base = soff[blockIdx.x] + inc - s;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (i0 + j < n) out[i0 + j] = base;
    base += v[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = soff[nblk];
}

// Several fills in one launch: workgroup row y fills job y.
__global__ void k_fill_multi(FillJobs J) {
  const FillJob f = J.job[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < f.n; i += (int64_t)gridDim.x * blockDim.x) {
    if (f.bytes == 8)
      reinterpret_cast<uint64_t *>(f.p)[i] = f.v;
    else
      reinterpret_cast<uint32_t *>(f.p)[i] = (uint32_t)f.v;
  }
}

// Two single-workgroup scans in one launch (workgroup 0: the first array).
template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_excl2(const TIn *in0, int64_t *out0, const TIn *in1,
                                                             int64_t *out1, const unsigned long long *n_dev,
                                                             int64_t n_host) {
  __shared__ int64_t sh[kScanThreads / 64];
  __shared__ int64_t tile_total;
  const TIn *in = blockIdx.x ? in1 : in0;
  int64_t *out = blockIdx.x ? out1 : out0;
  int64_t n = n_host;
  if (n_dev) n = (int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host;
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < n; t0 += kScanChunk) {
    const int64_t i0 = t0 + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = (i0 + j < n) ? (int64_t)in[i0 + j] : 0;
      s += v[j];
    }
    const int64_t inc = block_inclusive_scan<int64_t>(s, sh);
    int64_t base = carry + inc - s;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (i0 + j < n) out[i0 + j] = base;
      base += v[j];
    }
    if (threadIdx.x == kScanThreads - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
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

// Longest input scanned by one workgroup (8 tiles); longer ones use the
// three multi-workgroup kernels.
constexpr int64_t kScanSingleMax = 8 * (int64_t)kScanChunk;

int64_t scan_scratch_elems(int64_t n_host) { return 2 * ((n_host + kScanChunk - 1) / kScanChunk) + 2; }

template <typename TIn>
static void scan_any(const TIn *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host, int64_t *tmp,
                     hipStream_t st) {
  if (!tmp || n_host <= kScanSingleMax) {
    k_scan_excl<TIn><<<1, kScanThreads, 0, st>>>(in, out, n_dev, n_host);
    return;
  }
  const int nblk = (int)((n_host + kScanChunk - 1) / kScanChunk);
  int64_t *sums = tmp, *soff = tmp + nblk + 1;
  k_scan_sums<TIn><<<nblk, kScanThreads, 0, st>>>(in, n_dev, n_host, sums);
  k_scan_excl<int64_t><<<1, kScanThreads, 0, st>>>(sums, soff, nullptr, nblk);
  k_scan_chunks<TIn><<<nblk, kScanThreads, 0, st>>>(in, out, n_dev, n_host, soff, nblk);
}

void launch_scan_i64(const int64_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                     int64_t *tmp, hipStream_t st) {
  scan_any<int64_t>(in, out, n_dev, n_host, tmp, st);
}
void launch_scan_i32_to_i64(const int32_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                            int64_t *tmp, hipStream_t st) {
  scan_any<int32_t>(in, out, n_dev, n_host, tmp, st);
}
int64_t radix_scratch_blocks(int64_t n_host) { return (n_host + kRsTile - 1) / kRsTile; }
constexpr int kRsMaxPasses = 8;  // 64-bit keys
int64_t radix_offset_elems(int64_t n_host) {
  const int64_t h = 256 * radix_scratch_blocks(n_host);
  return h + 1 + scan_scratch_elems(h) + kRsMaxPasses + 1;  // offsets, scan scratch, buffer parity
}

void launch_radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *tk, uint32_t *tv,
                           const unsigned long long *n_dev, int64_t n_host, int key_bits, int32_t *hist,
                           int64_t *hoff, hipStream_t st, const unsigned long long *bits_dev) {
  if (n_host <= 0 || key_bits <= 0) return;
  const int nblk = (int)radix_scratch_blocks(n_host);
  const int64_t h = (int64_t)256 * nblk;
  int64_t *par = hoff + h + 1 + scan_scratch_elems(h);  // par[p]: buffer holding pass p's input
  const RsBufs B = {{keys, tk}, {vals, tv}};
  int passes = 0;
  for (int shift = 0; shift < key_bits && passes < kRsMaxPasses; shift += 8, ++passes) {
    k_rs_hist<<<nblk, kRsThreads, 0, st>>>(B, par, passes, n_dev, n_host, shift, hist, nblk,
                                           nblk <= kRsFusedMaxBlocks, bits_dev);
    if (nblk <= kRsFusedMaxBlocks) {
      k_rs_pass<<<nblk, kRsThreads, 0, st>>>(B, par, passes, n_dev, n_host, shift, hist, nblk, bits_dev);
    } else {
      scan_any<int32_t>(hist, hoff, nullptr, h, hoff + h + 1, st);
      k_rs_scatter<<<nblk, kRsThreads, 0, st>>>(B, par, passes, n_dev, n_host, shift, hoff, nblk, bits_dev);
    }
  }
  k_rs_copy<<<grid_for(n_host, 256), 256, 0, st>>>(B, par, passes, n_dev, n_host);
}
void launch_fill_multi(const FillJobs &J, hipStream_t st) {
  int64_t nmax = 0;
  for (int k = 0; k < J.count; ++k) nmax = J.job[k].n > nmax ? J.job[k].n : nmax;
  if (J.count <= 0 || nmax <= 0) return;
  k_fill_multi<<<dim3(grid_for(nmax, 256), J.count), 256, 0, st>>>(J);
}
void launch_scan2_i32_to_i64(const int32_t *in0, int64_t *out0, const int32_t *in1, int64_t *out1,
                             const unsigned long long *n_dev, int64_t n_host, int64_t *tmp, hipStream_t st) {
  if (n_host <= kScanSingleMax) {
    k_scan_excl2<int32_t><<<2, kScanThreads, 0, st>>>(in0, out0, in1, out1, n_dev, n_host);
    return;
  }
  scan_any<int32_t>(in0, out0, n_dev, n_host, tmp, st);
  scan_any<int32_t>(in1, out1, n_dev, n_host, tmp, st);
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

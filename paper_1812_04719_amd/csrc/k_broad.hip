// K1: vesicle broad phase on an implicit Morton-ordered grid (Alg. 1).
//
//   1. h_m = average diagonal of the scene's boxes (Alg. 1, first step); the
//      uniform octree has depth ceil(log2(L / h_m)) (Sec. 3.3.1).
//   2. Check points: per box and axis, points from lo to hi (both faces
//      included) with spacing no larger than the cell edge, so every cell
//      the box overlaps holds at least one of its points.  Each point is
//      keyed by the Morton ID of its cell (wrapped on periodic axes) with the
//      scene index in the high bits.
//   3. Stable sort of the keys (ties keep the global check-point order,
//      Table 3).
//   4. For every run of equal keys, all pairs of distinct boxes are tested;
//      every periodic image shift sigma with an overlap is inserted into a
//      hash set (Alg. 1's "unique").
//   5. The unique pairs are bucketed by their first vesicle and sorted
//      inside each bucket, giving the canonical (a, b, sigma) order.
// The overlap test is the exact FP64 closed-interval test on boxes shifted
// by sigma * L; the grid only decides which pairs get tested.
#include "stiv_common.h"

namespace stiv {

namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ inline uint64_t spread3(uint32_t x) {
  uint64_t v = x & 0x3ffu;
  v = (v | (v << 16)) & 0x30000ffull;
  v = (v | (v << 8)) & 0x300f00full;
  v = (v | (v << 4)) & 0x30c30c3ull;
  v = (v | (v << 2)) & 0x9249249ull;
  return v;
}

__device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

__device__ inline uint64_t pack_pair(int a, int b, const int s[3]) {
  return ((uint64_t)(uint32_t)a << 36) | ((uint64_t)(uint32_t)b << 12) | ((uint64_t)(s[0] + 8) << 8) |
         ((uint64_t)(s[1] + 8) << 4) | (uint64_t)(s[2] + 8);
}

__device__ inline uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Insert a key into the open-addressing set (linear probing).  The set is
// listed afterwards by k_hash_list, so an insertion touches only its own
// slots (no shared counter).
__device__ void hash_insert(uint64_t key, uint64_t *hash, int64_t cap, Counters *cnt) {
  uint64_t h = mix64(key) & (uint64_t)(cap - 1);
  for (int64_t probe = 0; probe < cap; ++probe) {
    // most insertions repeat a pair already present: look before the atomic
    const uint64_t seen = __hip_atomic_load((unsigned long long *)&hash[h], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    if (seen == key) return;
    if (seen != kEmpty) {
      h = (h + 1) & (uint64_t)(cap - 1);
      continue;
    }
    uint64_t prev = atomicCAS((unsigned long long *)&hash[h], (unsigned long long)kEmpty,
                              (unsigned long long)key);
    if (prev == kEmpty || prev == key) return;
    h = (h + 1) & (uint64_t)(cap - 1);
  }
  atomicAdd(&cnt->hash_overflow, 1ull);
}

__device__ inline bool box_overlap_shifted(const double *A, const double *B, const double sh[3]) {
  for (int c = 0; c < 3; ++c) {
    double blo = B[c] + sh[c], bhi = B[3 + c] + sh[c];
    if (!(A[c] <= bhi && blo <= A[3 + c])) return false;
  }
  return true;
}

// Insert every image shift of (a, b) whose shifted boxes overlap.
__device__ void test_pair_all_shifts(int a, int b, const double *A, const double *B, const double *L,
                                     uint64_t *hash, int64_t cap, Counters *cnt) {
  // candidate shifts per axis: (A.lo - B.hi)/L <= sigma <= (A.hi - B.lo)/L, widened
  // by 1e-6 against rounding; each one is then tested exactly
  int lo[3], hi[3];
  for (int c = 0; c < 3; ++c) {
    if (L[c] > 0.0) {
      lo[c] = (int)ceil((A[c] - B[3 + c]) / L[c] - 1e-6);
      hi[c] = (int)floor((A[3 + c] - B[c]) / L[c] + 1e-6);
      if (lo[c] < -kMaxShift || hi[c] > kMaxShift) {
        atomicAdd(&cnt->shift_overflow, 1ull);
        lo[c] = lo[c] < -kMaxShift ? -kMaxShift : lo[c];
        hi[c] = hi[c] > kMaxShift ? kMaxShift : hi[c];
      }
    } else {
      lo[c] = hi[c] = 0;
    }
  }
  int s[3];
  for (s[0] = lo[0]; s[0] <= hi[0]; ++s[0])
    for (s[1] = lo[1]; s[1] <= hi[1]; ++s[1])
      for (s[2] = lo[2]; s[2] <= hi[2]; ++s[2]) {
        if (a == b) {
          // own image: keep sigma > 0 lexicographically
          bool pos = s[0] > 0 || (s[0] == 0 && (s[1] > 0 || (s[1] == 0 && s[2] > 0)));
          if (!pos) continue;
        }
        double sh[3];
        for (int c = 0; c < 3; ++c) sh[c] = (double)s[c] * L[c];
        if (box_overlap_shifted(A, B, sh)) hash_insert(pack_pair(a, b, s), hash, cap, cnt);
      }
}

// Scene of each vesicle: binary search of scene_off (one thread per vesicle).
// Number of check points of a box on one axis; full = every cell of a
// periodic axis (box at least one period long).
__device__ inline int axis_points(const SceneGrid &g, int c, double lo, double hi, bool *full) {
  const double e = (hi - lo) + 2.0 * g.tiny;
  const int ncell = 1 << g.depth;
  *full = false;
  if (g.periodic[c] && e >= g.w[c] * ncell) {
    *full = true;
    return ncell;
  }
  int n = (int)ceil(e / g.w[c]) + 1;
  if (n < 2) n = 2;
  if (n > ncell + 2) n = ncell + 2;
  return n;
}

__device__ inline uint32_t axis_cell(const SceneGrid &g, int c, double lo, double hi, int k, int n, bool full) {
  const int ncell = 1 << g.depth;
  if (full) return (uint32_t)k;
  const double a = lo - g.tiny, e = (hi - lo) + 2.0 * g.tiny;
  const double x = (k == n - 1) ? (hi + g.tiny) : a + e * ((double)k / (double)(n - 1));
  long long ci = (long long)floor((x - g.org[c]) / g.w[c]);
  if (g.periodic[c]) {
    ci %= ncell;
    if (ci < 0) ci += ncell;
  } else {
    ci = ci < 0 ? 0 : (ci >= ncell ? ncell - 1 : ci);
  }
  return (uint32_t)ci;
}

// One workgroup per scene: the scene's grid (Alg. 1, first steps), then the
// number of check points of each of its vesicles' boxes.  With cp_off (a
// single scene) the workgroup also scans the counts into the check points'
// offsets (cp_off[n] = their number), which saves the scan's launch.
constexpr int kGridU = 4;
__global__ __launch_bounds__(256) void k_scene_grid(DevScene S, const double *box, SceneGrid *grid,
                                                    int64_t *cp_cnt, int64_t *cp_off) {
  __shared__ double sh_sum[256], sh_lo[3][256], sh_hi[3][256];
  __shared__ int64_t sh_wave[4];
  __shared__ SceneGrid sg;
  for (int sc = blockIdx.x; sc < S.n_scenes; sc += gridDim.x) {
    const int v0 = S.scene_off[sc], v1 = S.scene_off[sc + 1];
    double sum = 0.0, lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    // kGridU boxes per thread at a time, loaded before any is used
    for (int v0u = v0 + threadIdx.x; v0u < v1; v0u += kGridU * blockDim.x) {
      double Bv[kGridU][6];
#pragma unroll
      for (int u = 0; u < kGridU; ++u) {
        const int v = v0u + u * blockDim.x;
#pragma unroll
        for (int c = 0; c < 6; ++c) Bv[u][c] = v < v1 ? box[6 * (int64_t)v + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGridU; ++u) {
        if (v0u + u * (int)blockDim.x >= v1) break;
        const double *B = Bv[u];
        double dx = B[3] - B[0], dy = B[4] - B[1], dz = B[5] - B[2];
        sum += sqrt(dx * dx + dy * dy + dz * dz);
        for (int c = 0; c < 3; ++c) { lo[c] = fmin(lo[c], B[c]); hi[c] = fmax(hi[c], B[3 + c]); }
      }
    }
    sh_sum[threadIdx.x] = sum;
    for (int c = 0; c < 3; ++c) { sh_lo[c][threadIdx.x] = lo[c]; sh_hi[c][threadIdx.x] = hi[c]; }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        sh_sum[threadIdx.x] += sh_sum[threadIdx.x + off];
        for (int c = 0; c < 3; ++c) {
          sh_lo[c][threadIdx.x] = fmin(sh_lo[c][threadIdx.x], sh_lo[c][threadIdx.x + off]);
          sh_hi[c][threadIdx.x] = fmax(sh_hi[c][threadIdx.x], sh_hi[c][threadIdx.x + off]);
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      SceneGrid g;
      const int n = v1 - v0;
      const double hm = n > 0 ? sh_sum[0] / n : 1.0;
      double ext[3], lmax = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double L = S.box_len[3 * sc + c];
        g.periodic[c] = L > 0.0;
        if (L > 0.0) {
          g.org[c] = 0.0;
          ext[c] = L;
        } else {
          g.org[c] = n > 0 ? sh_lo[c][0] : 0.0;
          ext[c] = n > 0 ? sh_hi[c][0] - sh_lo[c][0] : 1.0;
        }
        lmax = fmax(lmax, ext[c]);
      }
      int depth = 0;
      if (hm > 0.0 && lmax > hm) depth = (int)ceil(log2(lmax / hm));
      depth = depth < 0 ? 0 : (depth > 10 ? 10 : depth);
      g.depth = depth;
      g.tiny = 1e-9 * fmax(lmax, 1.0);
      for (int c = 0; c < 3; ++c) g.w[c] = fmax(ext[c], g.tiny) / (double)(1 << depth);
      g.pad = 0;
      grid[sc] = g;
      sg = g;
    }
    __syncthreads();
    for (int v0u = v0 + threadIdx.x; v0u < v1; v0u += kGridU * blockDim.x) {
      double Bv[kGridU][6];
#pragma unroll
      for (int u = 0; u < kGridU; ++u) {
        const int v = v0u + u * blockDim.x;
#pragma unroll
        for (int c = 0; c < 6; ++c) Bv[u][c] = v < v1 ? box[6 * (int64_t)v + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGridU; ++u) {
        const int v = v0u + u * blockDim.x;
        if (v >= v1) break;
        int64_t tot = 1;
        for (int c = 0; c < 3; ++c) {
          bool full;
          tot *= axis_points(sg, c, Bv[u][c], Bv[u][3 + c], &full);
        }
        cp_cnt[v] = tot;
      }
    }
    __syncthreads();
    if (cp_off) {
      // exclusive scan: each thread a contiguous run of vesicles, the runs'
      // sums scanned within each wavefront by shuffles, then across them
      const int n = v1 - v0;
      const int chunk = (n + (int)blockDim.x - 1) / (int)blockDim.x;
      const int lo = v0 + (int)threadIdx.x * chunk, hi = lo + chunk < v1 ? lo + chunk : v1;
      int64_t run = 0;
      for (int v = lo; v < hi; ++v) run += cp_cnt[v];
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      int64_t incl = run;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      if (lane == 63) sh_wave[wave] = incl;
      __syncthreads();
      for (int w = 0; w < wave; ++w) incl += sh_wave[w];
      int64_t at = incl - run;
      for (int v = lo; v < hi; ++v) {
        const int64_t c = cp_cnt[v];
        cp_off[v] = at;
        at += c;
      }
      if (threadIdx.x == blockDim.x - 1) cp_off[v1] = incl;
      __syncthreads();
    }
  }
}

// kCpLanes threads per vesicle, each emitting every kCpLanes-th of its check
// points (index (kx * n_y + ky) * n_z + kz, as one thread would in order).
constexpr int kCpLanes = 8;
__global__ void k_cp_emit(DevScene S, const double *box, const int *ves_scene, const SceneGrid *grid,
                          const int64_t *cp_off, uint64_t *keys, uint32_t *vals, int64_t cap, Counters *cnt) {
  const int64_t nt = (int64_t)S.n_ves * kCpLanes;
  // which key bits vary: OR of the keys and of their complements (the sort
  // skips digits that are the same in every key: a shallow grid leaves the
  // high Morton digits zero)
  uint64_t k_or = 0, k_nor = 0;
  for (int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gid < nt; gid += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(gid / kCpLanes), part = (int)(gid % kCpLanes);
    const int sc = ves_scene[v];
    const SceneGrid g = grid[sc];
    const double *B = box + 6 * (int64_t)v;
    int n[3];
    bool full[3];
    for (int c = 0; c < 3; ++c) n[c] = axis_points(g, c, B[c], B[3 + c], &full[c]);
    const int64_t o0 = cp_off[v];
    const int total = n[0] * n[1] * n[2];
    for (int idx = part; idx < total; idx += kCpLanes) {
      const int kx = idx / (n[1] * n[2]), ky = (idx / n[2]) % n[1], kz = idx % n[2];
      const uint32_t cx = axis_cell(g, 0, B[0], B[3], kx, n[0], full[0]);
      const uint32_t cy = axis_cell(g, 1, B[1], B[4], ky, n[1], full[1]);
      const uint32_t cz = axis_cell(g, 2, B[2], B[5], kz, n[2], full[2]);
      const int64_t o = o0 + idx;
      if (o < cap) {
        const uint64_t key = ((uint64_t)sc << 30) | morton3(cx, cy, cz);
        keys[o] = key;
        vals[o] = (uint32_t)v;
        k_or |= key;
        k_nor |= ~key;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    k_or |= __shfl_xor(k_or, off, 64);
    k_nor |= __shfl_xor(k_nor, off, 64);
  }
  if ((threadIdx.x & 63) == 0 && (k_or | k_nor)) {
    atomicOr(&cnt->cp_key_bits[0], (unsigned long long)k_or);
    atomicOr(&cnt->cp_key_bits[1], (unsigned long long)k_nor);
  }
}

// One wavefront per check point i that starts its box's stretch in a cell
// (a box's check points in one cell are consecutive in the stable order, so
// each box is taken once per cell); lane l takes the l-th following check
// point of the same cell, 64 at a time, and tests the box pair if that point
// starts its own box's stretch.
__global__ __launch_bounds__(256) void k_cell_pairs(DevScene S, const double *box, const int *ves_scene,
                                                    const uint64_t *keys, const uint32_t *vals,
                                                    const unsigned long long *n_cp, int64_t cap_cp, uint64_t *hash,
                                                    int64_t cap, Counters *cnt) {
  int64_t n = (int64_t)*n_cp;
  n = n < cap_cp ? n : cap_cp;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n; i += nwaves) {
    const uint64_t k = keys[i];
    const int vi = (int)vals[i];
    if (i > 0 && keys[i - 1] == k && (int)vals[i - 1] == vi) continue;
    for (int64_t j0 = i + 1; j0 < n; j0 += 64) {
      const int64_t j = j0 + lane;
      // equal keys are contiguous: the lanes still in the cell are a prefix
      const bool in = j < n && keys[j] == k;
      if (in) {
        const int vj = (int)vals[j];
        if (vi != vj && (int)vals[j - 1] != vj) {
          const int a = vi < vj ? vi : vj, b = vi < vj ? vj : vi;
          const double *L = S.box_len + 3 * ves_scene[a];
          test_pair_all_shifts(a, b, box + 6 * (int64_t)a, box + 6 * (int64_t)b, L, hash, cap, cnt);
        }
      }
      if (!(__ballot(in) >> 63)) break;
    }
  }
  // each vesicle against its own periodic images (no cell needed)
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < S.n_ves; v += gridDim.x * blockDim.x) {
    const double *L = S.box_len + 3 * ves_scene[v];
    if (!(L[0] > 0.0 || L[1] > 0.0 || L[2] > 0.0)) continue;
    const double *A = box + 6 * (int64_t)v;
    test_pair_all_shifts(v, v, A, A, L, hash, cap, cnt);
  }
}

// List the keys of the set: each workgroup compacts a contiguous range of
// slots and reserves its output range with one atomic; n_pairs ends as the
// number of keys (the list order is settled by the bucket sort that follows).
constexpr int kListThreads = 256;
template <int kListItems>
__global__ __launch_bounds__(kListThreads) void k_hash_list(const uint64_t *hash, int64_t cap, uint64_t *uniq,
                                                            int64_t uniq_cap, int32_t *cnt_a, Counters *cnt) {
  __shared__ int wsum[kListThreads / 64];
  __shared__ unsigned long long base_sh;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t r0 = (int64_t)blockIdx.x * kListThreads * kListItems; r0 < cap;
       r0 += (int64_t)gridDim.x * kListThreads * kListItems) {
    // slots r0 + (w * kListItems + j) * 64 + lane: each wavefront a contiguous stretch
    uint64_t key[kListItems];
    int cnt_w = 0;
#pragma unroll
    for (int j = 0; j < kListItems; ++j) {
      const int64_t e = r0 + ((int64_t)(w * kListItems + j) << 6) + lane;
      key[j] = e < cap ? hash[e] : kEmpty;
      cnt_w += __popcll(__ballot(key[j] != kEmpty));
    }
    if (lane == 0) wsum[w] = cnt_w;
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int k = 0; k < kListThreads / 64; ++k) tot += wsum[k];
      base_sh = tot ? atomicAdd(&cnt->n_pairs, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    unsigned long long o = base_sh;
    for (int k = 0; k < w; ++k) o += (unsigned long long)wsum[k];
#pragma unroll
    for (int j = 0; j < kListItems; ++j) {
      const bool keep = key[j] != kEmpty;
      const unsigned long long m = __ballot(keep);
      if (keep) {
        const unsigned long long idx = o + __popcll(m & lt);
        if ((int64_t)idx < uniq_cap) {
          uniq[idx] = key[j];
          atomicAdd(&cnt_a[(int)(key[j] >> 36)], 1);  // pairs per first vesicle (bucket sizes)
        }
      }
      o += __popcll(m);
    }
    __syncthreads();
  }
}

__global__ void k_bucket_scatter(const uint64_t *uniq, int64_t uniq_cap, const int64_t *off_a, int32_t *cursor,
                                 uint64_t *sorted, const Counters *cnt) {
  int64_t n = (int64_t)cnt->n_pairs;
  n = n < uniq_cap ? n : uniq_cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = uniq[i];
    const int a = (int)(k >> 36);
    const int pos = atomicAdd(&cursor[a], 1);
    sorted[off_a[a] + pos] = k;
  }
}

constexpr int kBucketRegs = 16;

// One canonical pair record from its key (a, b, shift digits).
__device__ inline void emit_pair(uint64_t k, int64_t i, const double L[3], PairRec *pairs, int32_t *pair_ab,
                                 int32_t *pair_shift, int64_t cap_pairs) {
  PairRec r;
  r.a = (int)(k >> 36);
  r.b = (int)((k >> 12) & 0xffffffull);
  r.s[0] = (int)((k >> 8) & 15u) - 8;
  r.s[1] = (int)((k >> 4) & 15u) - 8;
  r.s[2] = (int)(k & 15u) - 8;
  r.pad = 0;
  for (int c = 0; c < 3; ++c) r.sh[c] = (double)r.s[c] * L[c];
  pairs[i] = r;
  if (i < cap_pairs) {
    pair_ab[2 * i] = r.a;
    pair_ab[2 * i + 1] = r.b;
    for (int c = 0; c < 3; ++c) pair_shift[3 * i + c] = r.s[c];
  }
}

__global__ void k_bucket_sort_emit(DevScene S, const int *ves_scene, const int64_t *off_a, uint64_t *sorted,
                                   int n_ves, PairRec *pairs, int32_t *pair_ab, int32_t *pair_shift,
                                   int64_t cap_pairs) {
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < n_ves; a += gridDim.x * blockDim.x) {
    const int64_t p0 = off_a[a], p1 = off_a[a + 1];
    const double *Lp = S.box_len + 3 * ves_scene[a];
    const double L[3] = {Lp[0], Lp[1], Lp[2]};
    if (p1 - p0 <= kBucketRegs) {
      // the usual case (a handful of pairs): all loads at once, an odd-even
      // transposition network in registers, the records written from there
      // (keys are distinct and below the ~0 padding)
      uint64_t v[kBucketRegs];
#pragma unroll
      for (int k = 0; k < kBucketRegs; ++k) v[k] = p0 + k < p1 ? sorted[p0 + k] : ~0ull;
#pragma unroll
      for (int r = 0; r < kBucketRegs; ++r)
#pragma unroll
        for (int k = r & 1; k + 1 < kBucketRegs; k += 2) {
          const uint64_t x = v[k], y = v[k + 1];
          v[k] = x < y ? x : y;
          v[k + 1] = x < y ? y : x;
        }
#pragma unroll
      for (int k = 0; k < kBucketRegs; ++k)
        if (p0 + k < p1) emit_pair(v[k], p0 + k, L, pairs, pair_ab, pair_shift, cap_pairs);
    } else {
      for (int64_t i = p0 + 1; i < p1; ++i) {  // insertion sort in place
        uint64_t k = sorted[i];
        int64_t j = i - 1;
        while (j >= p0 && sorted[j] > k) {
          sorted[j + 1] = sorted[j];
          --j;
        }
        sorted[j + 1] = k;
      }
      for (int64_t i = p0; i < p1; ++i) emit_pair(sorted[i], i, L, pairs, pair_ab, pair_shift, cap_pairs);
    }
  }
}

int grid1d(int64_t n, int threads, int maxg = 2048) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

}  // namespace

void launch_scene_grid(const DevScene &S, const double *ves_box, SceneGrid *grid, int64_t *cp_cnt, int64_t *cp_off,
                       hipStream_t st) {
  int g = S.n_scenes < 1024 ? S.n_scenes : 1024;
  if (g < 1) return;
  k_scene_grid<<<g, 256, 0, st>>>(S, ves_box, grid, cp_cnt, S.n_scenes == 1 ? cp_off : nullptr);
}
void launch_cp_emit(const DevScene &S, const double *ves_box, const int *ves_scene, const SceneGrid *grid,
                    const int64_t *cp_off, uint64_t *keys, uint32_t *vals, int64_t cap, Counters *cnt,
                    hipStream_t st) {
  k_cp_emit<<<grid1d((int64_t)S.n_ves * kCpLanes, 256, 4096), 256, 0, st>>>(S, ves_box, ves_scene, grid, cp_off,
                                                                              keys, vals, cap, cnt);
}
void launch_cell_pairs(const DevScene &S, const double *ves_box, const int *ves_scene, const uint64_t *keys,
                       const uint32_t *vals, const unsigned long long *n_cp, int64_t n_cp_cap, uint64_t *hash,
                       int64_t hash_cap, Counters *cnt, hipStream_t st) {
  // one wavefront per check point (grid-stride beyond 4096 x 4 wavefronts)
  k_cell_pairs<<<grid1d(n_cp_cap, 4, 4096), 256, 0, st>>>(S, ves_box, ves_scene, keys, vals, n_cp, n_cp_cap, hash,
                                                          hash_cap, cnt);
}
void launch_hash_list(const uint64_t *hash, int64_t hash_cap, uint64_t *uniq, int64_t uniq_cap, int32_t *cnt_a,
                      Counters *cnt, hipStream_t st) {
  // a small set is spread over more workgroups (4 slots per thread: 0.117 against 0.121 ms
  // for the vesicle broad phase at 1440 vesicles, 131K slots); a large one keeps 16 per thread
  // (2M slots in the 256-scene batch: 4 per thread costs 13 us there)
  if (hash_cap <= (int64_t)1 << 18)
    k_hash_list<4><<<grid1d(hash_cap, kListThreads * 4, 1024), kListThreads, 0, st>>>(hash, hash_cap, uniq,
                                                                                      uniq_cap, cnt_a, cnt);
  else
    k_hash_list<16><<<grid1d(hash_cap, kListThreads * 16, 1024), kListThreads, 0, st>>>(hash, hash_cap, uniq,
                                                                                         uniq_cap, cnt_a, cnt);
}
void launch_pair_bucket_scatter(const uint64_t *uniq, int64_t uniq_cap, const int64_t *off_a, int32_t *cursor_a,
                                uint64_t *sorted, Counters *cnt, hipStream_t st) {
  k_bucket_scatter<<<grid1d(uniq_cap, 256), 256, 0, st>>>(uniq, uniq_cap, off_a, cursor_a, sorted, cnt);
}
void launch_pair_bucket_sort_emit(const DevScene &S, const int *ves_scene, const int64_t *off_a, uint64_t *sorted,
                                  int n_ves, PairRec *pairs, int32_t *pair_ab, int32_t *pair_shift,
                                  int64_t cap_pairs, hipStream_t st) {
  k_bucket_sort_emit<<<grid1d(n_ves, 64), 64, 0, st>>>(S, ves_scene, off_a, sorted, n_ves, pairs, pair_ab,
                                                       pair_shift, cap_pairs);
}

}  // namespace stiv

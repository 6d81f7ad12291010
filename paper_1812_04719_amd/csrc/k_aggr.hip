// K5: canonical ordering and aggregation of contacts (Sec. 3.1.2: V = sum of
// the vertex-triangle volumes V_k; Sec. 3.3.2: the Jacobian J = dV/dX1 is
// stored per (volume, vertex)).
//
// Contacts arrive in arbitrary order from the narrow phase.  They are
// bucketed by vesicle pair (count, scan, scatter), then one workgroup per
// pair sorts its bucket by (kind, i, j) with a bitonic network in LDS (in a
// global scratch slice when the bucket is larger than LDS), writes the
// contacts in canonical order, sums V in that order, and forms the J rows by
// sorting the 4 per-contact vertex contributions by (vertex, contact order)
// and adding each run in order.  Sums therefore follow one fixed order and
// repeated runs are bit-identical (no floating-point atomics).
#include "stiv_common.h"

namespace stiv {

namespace {

constexpr int kAggThreads = 256;
constexpr int kLdsSort = 2048;

// Adds each lane's 1 to ctr[key] with one atomic per distinct key of the
// wavefront (contacts of a wavefront mostly share a pair, and one atomic per
// contact on the same counter serialized); returns the lane's old value
// (its position among the lanes of its key in lane order, after the value the
// counter had).  Lanes with key < 0 take no part.
__device__ inline int wave_grouped_add(int32_t *ctr, int key) {
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  unsigned long long todo = __ballot(key >= 0);
  int mine = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int k0 = __shfl(key, leader, 64);
    const unsigned long long grp = __ballot(key == k0) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&ctr[k0], __popcll(grp));
    base = __shfl(base, leader, 64);
    if ((grp >> lane) & 1ull) mine = base + __popcll(grp & lt);
    todo &= ~grp;
  }
  return mine;
}

__global__ void k_ct_pair_count(const Cand *ct, int64_t ct_cap, const Counters *cnt, int32_t *pair_cnt) {
  int64_t n = (int64_t)cnt->n_ct;
  n = n < ct_cap ? n : ct_cap;
  // whole wavefronts run every iteration (the grouped add is a wavefront operation)
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    (void)wave_grouped_add(pair_cnt, i < n ? ct[i].pair : -1);
  }
}

__global__ void k_ct_scatter(const Cand *ct, int64_t ct_cap, const Counters *cnt, const int64_t *pair_off,
                             int32_t *cursor, int32_t *perm) {
  int64_t n = (int64_t)cnt->n_ct;
  n = n < ct_cap ? n : ct_cap;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const int p = i < n ? ct[i].pair : -1;
    const int pos = wave_grouped_add(cursor, p);
    if (p >= 0) perm[pair_off[p] + pos] = (int32_t)i;
  }
}

// Ascending bitonic sort of (key, idx) pairs in place; n_pow2 >= n is a power of
// two and entries [n, n_pow2) are padded by the caller with key = ~0.  Inlined
// at each call, so that a call on the LDS arrays compiles to LDS accesses (a
// pointer that may be either LDS or global memory makes every access a
// generic one); GLOBAL adds the fence that the global-memory slices need.
template <bool GLOBAL>
__device__ __forceinline__ void bitonic(uint64_t *key, int32_t *idx, int n_pow2) {
  for (int size = 2; size <= n_pow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n_pow2 >> 1); t += blockDim.x) {
        // i = 2 * stride * (t / stride) + t % stride, stride a power of two
        const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
        const int j = i + stride;
        const bool asc = (i & size) == 0;
        const uint64_t ki = key[i], kj = key[j];
        if ((ki > kj) == asc) {
          key[i] = kj;
          key[j] = ki;
          const int32_t x = idx[i];
          idx[i] = idx[j];
          idx[j] = x;
        }
      }
      if (GLOBAL) __threadfence_block();
      __syncthreads();
    }
  }
}

__device__ inline int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__global__ __launch_bounds__(kAggThreads) void k_ct_sort_aggregate(
    DevScene S, DevTopo T, const PairRec *pairs, const Counters *cnt, const int64_t *pair_off, const int32_t *perm,
    const Cand *ct, const double *ct_s, const double *ct_vol, const double *ct_grad, double dt, uint64_t *gkeys,
    int32_t *gidx, int32_t *out_key, double *out_tau, double *out_s, double *out_vol, double *out_grad,
    int64_t cap_ct, double *pair_V, int32_t *pair_hasvt, int32_t *pair_rows, int32_t *row_vtx_tmp, double *row_g_tmp,
    int64_t pairs_cap) {
  __shared__ uint64_t skey[kLdsSort];
  __shared__ int32_t sidx[kLdsSort];
  __shared__ int s_nvt;
  __shared__ double s_part[kAggThreads];
  __shared__ int s_cnt[kAggThreads];
  int64_t np = (int64_t)cnt->n_pairs;
  np = np < pairs_cap ? np : pairs_cap;
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    const int64_t off = pair_off[p];
    const int n = (int)(pair_off[p + 1] - off);
    if (n == 0) {
      if (threadIdx.x == 0) { pair_hasvt[p] = 0; pair_rows[p] = 0; pair_V[p] = 0.0; }
      continue;
    }
    // ---- sort the pair's contacts by (kind, i, j)
    const int n2 = pow2_ceil(n);
    uint64_t *key = skey;
    int32_t *idx = sidx;
    if (n2 > kLdsSort) { key = gkeys + 8 * off; idx = gidx + 8 * off; }  // slice of 8*n >= n2 entries
    for (int k = threadIdx.x; k < n2; k += blockDim.x) {
      if (k < n) {
        const int32_t c = perm[off + k];
        const Cand cd = ct[c];
        key[k] = ((uint64_t)cd.kind << 42) | ((uint64_t)cd.i << 21) | (uint64_t)cd.j;
        idx[k] = c;
      } else {
        key[k] = ~0ull;
        idx[k] = -1;
      }
    }
    __threadfence_block();
    __syncthreads();
    if (n2 <= kLdsSort)
      bitonic<false>(skey, sidx, n2);
    else
      bitonic<true>(key, idx, n2);
    if (threadIdx.x == 0) s_nvt = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const int32_t c = idx[k];
      const Cand cd = ct[c];
      const int64_t o = off + k;
      if (cd.kind < 2) atomicAdd(&s_nvt, 1);
      if (o < cap_ct) {
        out_key[4 * o] = (int32_t)p;
        out_key[4 * o + 1] = cd.kind;
        out_key[4 * o + 2] = cd.i;
        out_key[4 * o + 3] = cd.j;
        out_tau[o] = ct_s[c] * dt;
        if (out_s) out_s[o] = ct_s[c];
        out_vol[o] = ct_vol[c];
        for (int q = 0; q < 12; ++q) out_grad[12 * o + q] = ct_grad[12 * (int64_t)c + q];
      }
    }
    __syncthreads();
    const int nvt = s_nvt;  // VT contacts come first (kind 0, 1 before 2)
    // ---- V = sum of V_k: each thread adds a contiguous run of the sorted VT
    // contacts, then the partial sums are added in thread order (a fixed
    // order, so repeated runs give the same bits)
    {
      const int chunk = (nvt + kAggThreads - 1) / kAggThreads;
      const int lo = threadIdx.x * chunk, hi = min(nvt, lo + chunk);
      double part = 0.0;
      for (int k = lo; k < hi; ++k) part += ct_vol[idx[k]];
      s_part[threadIdx.x] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        // the partial sums past the last non-empty run are +0 and would not
        // change the bits (V_k >= 0)
        const int nparts = chunk ? (nvt + chunk - 1) / chunk : 0;
        double V = 0.0;
        for (int k = 0; k < nparts; ++k) V += s_part[k];
        pair_V[p] = V;
        pair_hasvt[p] = nvt > 0;
        if (nvt == 0) pair_rows[p] = 0;
      }
      __syncthreads();
    }
    if (nvt == 0) continue;
    // ---- J rows: 4 contributions per VT contact keyed by (global vertex, order)
    const PairRec pr = pairs[p];
    const int nj = 4 * nvt;
    const int nj2 = pow2_ceil(nj);
    uint64_t *jkey = skey;
    int32_t *jidx = sidx;
    if (!(nj2 <= kLdsSort && n2 <= kLdsSort)) {
      // global slices of 8*n >= nj2 entries
      jkey = gkeys + 8 * off;
      jidx = gidx + 8 * off;
    }
    // Keep the sorted VT contact order aside (the sort buffers are reused
    // below); the slice of row_vtx_tmp is free until the rows are written.
    int32_t *ord = row_vtx_tmp + 4 * off;
    for (int k = threadIdx.x; k < nvt; k += blockDim.x) ord[k] = idx[k];
    __threadfence_block();
    __syncthreads();
    for (int e = threadIdx.x; e < nj2; e += blockDim.x) {
      if (e < nj) {
        const int k = e >> 2, role = e & 3;
        const Cand cd = ct[ord[k]];
        const int vv = cd.kind ? pr.b : pr.a, vt = cd.kind ? pr.a : pr.b;
        int64_t gid;
        if (role == 0) {
          gid = S.vtx_off[vv] + cd.i;
        } else {
          const int tt = S.topo_id[vt];
          gid = S.vtx_off[vt] + T.tri[3 * ((int64_t)T.tri_off[tt] + cd.j) + (role - 1)];
        }
        jkey[e] = ((uint64_t)gid << 24) | (uint64_t)e;
        jidx[e] = ord[k] * 4 + role;
      } else {
        jkey[e] = ~0ull;
        jidx[e] = -1;
      }
    }
    __threadfence_block();
    __syncthreads();
    if (jkey == skey)
      bitonic<false>(skey, sidx, nj2);
    else
      bitonic<true>(jkey, jidx, nj2);
    // segments of equal vertex: each thread owns a contiguous chunk of entries,
    // counts the segment starts in it, and after a scan of those counts writes
    // the rows that start in its chunk (adding the segment in entry order)
    {
      const int chunk = (nj + kAggThreads - 1) / kAggThreads;
      const int lo = threadIdx.x * chunk, hi = min(nj, lo + chunk);
      int starts = 0;
      for (int e = lo; e < hi; ++e) starts += (e == 0 || (jkey[e] >> 24) != (jkey[e - 1] >> 24));
      s_cnt[threadIdx.x] = starts;
      __syncthreads();
      for (int offs = 1; offs < kAggThreads; offs <<= 1) {
        const int add = threadIdx.x >= offs ? s_cnt[threadIdx.x - offs] : 0;
        __syncthreads();
        s_cnt[threadIdx.x] += add;
        __syncthreads();
      }
      int row = s_cnt[threadIdx.x] - starts;
      for (int e = lo; e < hi; ++e) {
        const uint64_t gv = jkey[e] >> 24;
        if (!(e == 0 || gv != (jkey[e - 1] >> 24))) continue;
        double g[3] = {0.0, 0.0, 0.0};
        for (int f = e; f < nj && (jkey[f] >> 24) == gv; ++f) {
          const int32_t c4 = jidx[f];
          const int64_t c = c4 >> 2;
          const int role = c4 & 3;
          for (int q = 0; q < 3; ++q) g[q] += ct_grad[12 * c + 3 * role + q];
        }
        row_vtx_tmp[4 * off + row] = (int32_t)gv;
        for (int q = 0; q < 3; ++q) row_g_tmp[3 * (4 * off + row) + q] = g[q];
        ++row;
      }
      if (threadIdx.x == kAggThreads - 1) pair_rows[p] = s_cnt[kAggThreads - 1];
      __syncthreads();
    }
  }
}

// Volumes and J rows to the caller's arrays; workgroup 0 also stores the
// final counts (check points, volumes, J rows) for the host.
__global__ void k_write_volumes(Counters *cnt, const int64_t *pair_off, const int64_t *vol_off,
                                const int64_t *row_off, const int32_t *pair_hasvt, const double *pair_V,
                                const int32_t *pair_rows, const int32_t *row_vtx_tmp, const double *row_g_tmp,
                                int32_t *vol_pair, double *vol_V, int64_t cap_vol, int32_t *j_vol, int32_t *j_vtx,
                                double *j_g, int64_t cap_jrow, int64_t pairs_cap, const int64_t *cp_total) {
  int64_t np = (int64_t)cnt->n_pairs;
  np = np < pairs_cap ? np : pairs_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cnt->n_cp = (unsigned long long)*cp_total;
    cnt->n_vol = (unsigned long long)vol_off[np];
    cnt->n_jrow = (unsigned long long)row_off[np];
  }
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    if (!pair_hasvt[p]) continue;
    const int64_t v = vol_off[p];
    if (threadIdx.x == 0 && v < cap_vol) {
      vol_pair[v] = (int32_t)p;
      vol_V[v] = pair_V[p];
    }
    const int64_t r0 = row_off[p];
    const int64_t src = 4 * pair_off[p];
    for (int r = threadIdx.x; r < pair_rows[p]; r += blockDim.x) {
      const int64_t o = r0 + r;
      if (o < cap_jrow) {
        j_vol[o] = (int32_t)v;
        j_vtx[o] = row_vtx_tmp[src + r];
        for (int q = 0; q < 3; ++q) j_g[3 * o + q] = row_g_tmp[3 * (src + r) + q];
      }
    }
  }
}

int g1(int64_t n, int t) {
  int64_t g = (n + t - 1) / t;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

void launch_ct_pair_count(const Cand *ct, int64_t ct_cap, const Counters *cnt, int32_t *pair_cnt, hipStream_t st) {
  k_ct_pair_count<<<g1(ct_cap, 256), 256, 0, st>>>(ct, ct_cap, cnt, pair_cnt);
}
void launch_ct_scatter(const Cand *ct, int64_t ct_cap, const Counters *cnt, const int64_t *pair_off,
                       int32_t *cursor, int32_t *perm, hipStream_t st) {
  k_ct_scatter<<<g1(ct_cap, 256), 256, 0, st>>>(ct, ct_cap, cnt, pair_off, cursor, perm);
}
void launch_ct_sort_aggregate(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                              const Counters *cnt, const int64_t *pair_off, const int32_t *perm, const Cand *ct,
                              const double *ct_s, const double *ct_vol, const double *ct_grad, double dt,
                              uint64_t *gkeys, int32_t *gidx, int32_t *out_key, double *out_tau, double *out_s,
                              double *out_vol, double *out_grad, int64_t cap_ct, double *pair_V, int32_t *pair_hasvt,
                              int32_t *pair_rows, int32_t *row_vtx_tmp, double *row_g_tmp, hipStream_t st) {
  k_ct_sort_aggregate<<<g1(pairs_cap, 1), kAggThreads, 0, st>>>(
      S, T, pairs, cnt, pair_off, perm, ct, ct_s, ct_vol, ct_grad, dt, gkeys, gidx, out_key, out_tau, out_s, out_vol,
      out_grad, cap_ct, pair_V, pair_hasvt, pair_rows, row_vtx_tmp, row_g_tmp, pairs_cap);
}
void launch_write_volumes(Counters *cnt, int64_t pairs_cap, const int64_t *pair_off, const int64_t *vol_off,
                          const int64_t *row_off, const int32_t *pair_hasvt, const double *pair_V,
                          const int32_t *pair_rows, const int32_t *row_vtx_tmp, const double *row_g_tmp,
                          int32_t *vol_pair, double *vol_V, int64_t cap_vol, int32_t *j_vol, int32_t *j_vtx,
                          double *j_g, int64_t cap_jrow, const int64_t *cp_total, hipStream_t st) {
  k_write_volumes<<<g1(pairs_cap, 1), 64, 0, st>>>(cnt, pair_off, vol_off, row_off, pair_hasvt, pair_V, pair_rows,
                                                   row_vtx_tmp, row_g_tmp, vol_pair, vol_V, cap_vol, j_vol, j_vtx,
                                                   j_g, cap_jrow, pairs_cap, cp_total);
}
}  // namespace stiv

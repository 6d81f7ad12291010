// K5: canonical ordering and aggregation of contacts (Sec. 3.1.2: V = sum of
// the vertex-triangle volumes V_k; Sec. 3.3.2: the Jacobian J = dV/dX1 is
// stored per (volume, vertex)).
//
// Contacts arrive in arbitrary order from the narrow phase, which also counts
// them per vesicle pair.  They are bucketed by pair (scan, scatter), then one
// workgroup per pair sorts its bucket by (kind, i, j) with a bitonic network
// in LDS (in a global scratch slice when the bucket is larger than LDS), writes the
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

// Bucketing: contact i goes to its pair's bucket (workgroup `blk` of `nblk`).
__device__ void ct_scatter(const Cand *ct, int64_t ct_cap, const Counters *cnt, const int64_t *pair_off,
                           int32_t *cursor, int32_t *perm, int blk, int nblk) {
  int64_t n = (int64_t)cnt->n_ct;
  n = n < ct_cap ? n : ct_cap;
  for (int64_t i0 = blk * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)nblk * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const int p = i < n ? ct[i].pair : -1;
    const int pos = wave_grouped_add(cursor, p);
    if (p >= 0) perm[pair_off[p] + pos] = (int32_t)i;
  }
}

// Ascending bitonic sort of (key, idx) pairs in a global-memory slice (pairs
// whose bucket does not fit in LDS); n_pow2 >= n is a power of two and entries
// [n, n_pow2) are padded by the caller with key = ~0.
__device__ void bitonic_global(uint64_t *key, int32_t *idx, int n_pow2) {
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
      __threadfence_block();
      __syncthreads();
    }
  }
}

// LDS sort buffers hold one pad entry after every 8, so that the 8 entries
// a thread exchanges in registers (below) lie in different banks for the
// threads of a half-wavefront whatever the stride between them.
__device__ __forceinline__ int kp(int i) { return i + (i >> 3); }

// Compare-exchange: the smaller key to x (the larger with desc).
__device__ __forceinline__ void cex(uint64_t &x, uint64_t &y, bool desc) {
  const bool sw = (x > y) != desc;
  const uint64_t a = sw ? y : x, b = sw ? x : y;
  x = a;
  y = b;
}

// M consecutive stages (strides 2^(lo+M-1) down to 2^lo) of the bitonic merge
// of `size`: the 2^M entries whose indices differ only in those M bits are
// exchanged only among themselves, so each thread loads one such group, runs
// the M stages on it in registers and stores it back.
template <int M>
__device__ __forceinline__ void sort_pass(uint64_t *key, int n2, int size, int lo) {
  const int groups = n2 >> M;
  for (int t = threadIdx.x; t < groups; t += kAggThreads) {
    const int b = ((t >> lo) << (lo + M)) | (t & ((1 << lo) - 1));
    const bool desc = (b & size) != 0;
    uint64_t v[1 << M];
#pragma unroll
    for (int a = 0; a < (1 << M); ++a) v[a] = key[kp(b + (a << lo))];
#pragma unroll
    for (int r = M - 1; r >= 0; --r)
#pragma unroll
      for (int a = 0; a < (1 << M); ++a)
        if (!(a & (1 << r))) cex(v[a], v[a | (1 << r)], desc);
#pragma unroll
    for (int a = 0; a < (1 << M); ++a) key[kp(b + (a << lo))] = v[a];
  }
  __syncthreads();
}

// Ascending bitonic sort of n2 (a power of two, at most kLdsSort) distinct
// 64-bit keys in a padded LDS buffer, three stages per pass (one barrier per
// pass).  The exchanges are those of the plain network, so is the result.
__device__ void sort_keys_lds(uint64_t *key, int n2) {
  const int mmax = 3;
  for (int size = 2; size <= n2; size <<= 1) {
    int sb = __ffs(size) - 2;  // bit of the first stride, size / 2
    while (sb >= 0) {
      const int m = sb + 1 < mmax ? sb + 1 : mmax;
      const int lo = sb - m + 1;
      if (m == 3)
        sort_pass<3>(key, n2, size, lo);
      else if (m == 2)
        sort_pass<2>(key, n2, size, lo);
      else
        sort_pass<1>(key, n2, size, lo);
      sb -= m;
    }
  }
}

__device__ inline int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Rows of J from the (vertex, entry)-sorted contributions: each thread owns a
// contiguous chunk of entries, counts the segment starts in it, and after a
// scan of those counts writes the rows that start in its chunk, adding each
// segment in entry order (gathers of up to four entries issued together).
// vtx(e) is the vertex of sorted entry e, con(e) its contribution (contact * 4
// + role).
template <class VTX, class CON>
__device__ __forceinline__ void write_rows(int nj, VTX vtx, CON con, int *s_cnt, const double *__restrict__ ct_grad,
                                           int32_t *__restrict__ row_vtx, double *__restrict__ row_g,
                                           int32_t *pair_rows_p) {
  const int chunk = (nj + kAggThreads - 1) / kAggThreads;
  const int lo = threadIdx.x * chunk, hi = min(nj, lo + chunk);
  int starts = 0;
  for (int e = lo; e < hi; ++e) starts += (e == 0 || vtx(e) != vtx(e - 1));
  // inclusive scan of the counts: within each wavefront by shuffles, then
  // the totals of the wavefronts before it
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = starts;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_cnt[wave] = incl;
  __syncthreads();
  for (int w = 0; w < wave; ++w) incl += s_cnt[w];
  int row = incl - starts;
  for (int e = lo; e < hi; ++e) {
    const uint64_t gv = vtx(e);
    if (!(e == 0 || gv != vtx(e - 1))) continue;
    double g[3] = {0.0, 0.0, 0.0};
    bool more = true;
    for (int f0 = e; more; f0 += 4) {
      int32_t c4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int f = f0 + u;
        more = more && f < nj && vtx(f) == gv;
        c4[u] = more ? con(f) : -1;
      }
      double v[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (c4[u] >= 0)
#pragma unroll
          for (int q = 0; q < 3; ++q) v[u][q] = ct_grad[12 * (int64_t)(c4[u] >> 2) + 3 * (c4[u] & 3) + q];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (c4[u] >= 0)
#pragma unroll
          for (int q = 0; q < 3; ++q) g[q] += v[u][q];
    }
    row_vtx[row] = (int32_t)gv;
#pragma unroll
    for (int q = 0; q < 3; ++q) row_g[3 * row + q] = g[q];
    ++row;
  }
  if (threadIdx.x == kAggThreads - 1) *pair_rows_p = incl;
  __syncthreads();
}

// Vesicle pairs with contacts, listed for the sort-aggregate kernel: pairs of
// at least kBigPair contacts from the front of `order`, the others from its
// back, so that the workgroups dispatched first take the largest buckets (the
// largest bucket is that kernel's critical path).  Pairs without contacts get
// their empty results here.  The order within each list is that of the
// atomics; it decides only which workgroup takes a pair, not any result.
constexpr int kBigPair = 128;

__device__ void pair_order(Counters *cnt, int64_t pairs_cap, const int64_t *pair_off, int32_t *order,
                           double *pair_V, int32_t *pair_hasvt, int32_t *pair_rows, int blk, int nblk) {
  int64_t np = (int64_t)cnt->n_pairs;
  np = np < pairs_cap ? np : pairs_cap;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  // whole wavefronts run every iteration (the appends are wavefront operations)
  for (int64_t p0 = blk * (int64_t)blockDim.x; p0 < np; p0 += (int64_t)nblk * blockDim.x) {
    const int64_t p = p0 + threadIdx.x;
    int cls = -1;
    if (p < np) {
      const int64_t n = pair_off[p + 1] - pair_off[p];
      if (n == 0) {
        pair_hasvt[p] = 0;
        pair_rows[p] = 0;
        pair_V[p] = 0.0;
      } else {
        cls = n >= kBigPair ? 0 : 1;
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const unsigned long long m = __ballot(cls == c);
      if (!m) continue;
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long b = 0;
      if (lane == leader) b = atomicAdd(&cnt->n_pair_order[c], (unsigned long long)__popcll(m));
      b = __shfl(b, leader, 64);
      if (cls == c) {
        const int64_t slot = (int64_t)(b + __popcll(m & lt));
        order[c == 0 ? slot : pairs_cap - 1 - slot] = (int32_t)p;
      }
    }
  }
}

// Both steps after the scan of the per-pair counts, in one launch: the first
// n_scatter workgroups bucket the contacts, the others list the pairs.
__global__ void k_ct_scatter_order(const Cand *ct, int64_t ct_cap, Counters *cnt, const int64_t *pair_off,
                                   int32_t *cursor, int32_t *perm, int64_t pairs_cap, int32_t *order, double *pair_V,
                                   int32_t *pair_hasvt, int32_t *pair_rows, int n_scatter) {
  if ((int)blockIdx.x < n_scatter)
    ct_scatter(ct, ct_cap, cnt, pair_off, cursor, perm, blockIdx.x, n_scatter);
  else
    pair_order(cnt, pairs_cap, pair_off, order, pair_V, pair_hasvt, pair_rows, blockIdx.x - n_scatter,
               gridDim.x - n_scatter);
}

// One workgroup per vesicle pair with contacts (grid-stride over the list of
// pair_order, large buckets first).  Buckets of up to kLdsSort
// contacts (J entries) are sorted in LDS as single 64-bit keys carrying the
// entry's position in their low bits; larger ones as (key, index) pairs in a
// global slice.  Every gather phase issues a thread's loads before its stores.
__global__ __launch_bounds__(kAggThreads) void k_ct_sort_aggregate(
    DevScene S, DevTopo T, const PairRec *__restrict__ pairs, const Counters *__restrict__ cnt,
    const int32_t *__restrict__ order, const int64_t *__restrict__ pair_off, const int32_t *__restrict__ perm, const Cand *__restrict__ ct,
    const double *__restrict__ ct_s, const double *__restrict__ ct_vol, const double *__restrict__ ct_grad, double dt,
    uint64_t *__restrict__ gkeys, int32_t *__restrict__ gidx, int32_t *__restrict__ out_key,
    double *__restrict__ out_tau, double *__restrict__ out_s, double *__restrict__ out_vol,
    double *__restrict__ out_grad, int64_t cap_ct, double *__restrict__ pair_V, int32_t *__restrict__ pair_hasvt,
    int32_t *__restrict__ pair_rows, int32_t *__restrict__ row_vtx_tmp, double *__restrict__ row_g_tmp,
    int64_t pairs_cap) {
  __shared__ uint64_t skey[kLdsSort + kLdsSort / 8];
  __shared__ int32_t sidx[kLdsSort];
  __shared__ int32_t sord[kLdsSort / 4];
  __shared__ int s_nvt;
  __shared__ double s_part[kAggThreads];
  __shared__ int s_cnt[kAggThreads];
  const int64_t n_big = (int64_t)cnt->n_pair_order[0], n_list = n_big + (int64_t)cnt->n_pair_order[1];
  for (int64_t w = blockIdx.x; w < n_list; w += gridDim.x) {
    const int64_t p = order[w < n_big ? w : pairs_cap - 1 - (w - n_big)];
    const int64_t off = pair_off[p];
    const int n = (int)(pair_off[p + 1] - off);
    // ---- sort the pair's contacts by (kind, i, j); afterwards idx[k] is the
    // contact of rank k
    const int n2 = pow2_ceil(n);
    const bool lds = n2 <= kLdsSort;
    int32_t *idx = lds ? sidx : gidx + 8 * off;  // global slice of 8*n >= n2 entries
    if (threadIdx.x == 0) s_nvt = 0;
    if (lds) {
      // key (kind, i, j) << 11 | k: distinct, and k < 2048 finds the contact
      for (int k0 = threadIdx.x; k0 < n2; k0 += 2 * kAggThreads) {
        int32_t c[2];
        Cand cd[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = k0 + u * kAggThreads;
          c[u] = k < n ? perm[off + k] : -1;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (c[u] >= 0) cd[u] = ct[c[u]];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = k0 + u * kAggThreads;
          if (k >= n2) break;
          skey[kp(k)] = c[u] >= 0 ? (((uint64_t)cd[u].kind << 42 | (uint64_t)cd[u].i << 21 | (uint64_t)cd[u].j) << 11) |
                                        (uint64_t)k
                                  : ~0ull;
          if (k < n) sidx[k] = c[u];
        }
      }
      __syncthreads();
      sort_keys_lds(skey, n2);
      // contact of each rank: read all, then overwrite sidx in rank order
      int32_t cr[kLdsSort / kAggThreads];
#pragma unroll
      for (int u = 0; u < kLdsSort / kAggThreads; ++u) {
        const int k = threadIdx.x + u * kAggThreads;
        cr[u] = k < n ? sidx[(int)(skey[kp(k)] & 2047u)] : -1;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kLdsSort / kAggThreads; ++u) {
        const int k = threadIdx.x + u * kAggThreads;
        if (k < n) sidx[k] = cr[u];
      }
      __syncthreads();
    } else {
      uint64_t *key = gkeys + 8 * off;
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
      bitonic_global(key, idx, n2);
    }
    // contacts in canonical order.  The stores go to the caller's arrays,
    // which need only the alignment of their element type; the loads come from
    // the library's own (256-byte aligned) buffers.
    for (int k = threadIdx.x; k < n; k += kAggThreads) {
      const int32_t c = idx[k];
      const Cand cd = ct[c];
      const double sv = ct_s[c], vv = ct_vol[c];
      const double2 *gsrc = reinterpret_cast<const double2 *>(ct_grad + 12 * (int64_t)c);
      double2 gg[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) gg[q] = gsrc[q];
      if (cd.kind < 2) atomicAdd(&s_nvt, 1);
      const int64_t o = off + k;
      if (o < cap_ct) {
        out_key[4 * o] = (int32_t)p;
        out_key[4 * o + 1] = cd.kind;
        out_key[4 * o + 2] = cd.i;
        out_key[4 * o + 3] = cd.j;
        out_tau[o] = sv * dt;
        if (out_s) out_s[o] = sv;
        out_vol[o] = vv;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          out_grad[12 * o + 2 * q] = gg[q].x;
          out_grad[12 * o + 2 * q + 1] = gg[q].y;
        }
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
    // ---- J rows: 4 contributions per VT contact keyed by (global vertex,
    // entry), entry e = 4 k + role for the VT contact of rank k (role 0 its
    // vertex, 1-3 the triangle's corners)
    const PairRec pr = pairs[p];
    const int nj = 4 * nvt;
    const int nj2 = pow2_ceil(nj);
    const int64_t voff[2] = {S.vtx_off[pr.a], S.vtx_off[pr.b]};
    const int64_t toff[2] = {T.tri_off[S.topo_id[pr.a]], T.tri_off[S.topo_id[pr.b]]};
    if (nj2 <= kLdsSort) {
      // nvt <= 512: the VT contacts in rank order stay in LDS, and the sort
      // key (vertex << 24 | e) alone finds each contribution
      for (int k = threadIdx.x; k < nvt; k += kAggThreads) sord[k] = idx[k];
      __syncthreads();
      for (int k = threadIdx.x; k < nj2 / 4; k += kAggThreads) {
        uint64_t kk[4] = {~0ull, ~0ull, ~0ull, ~0ull};
        if (k < nvt) {
          const Cand cd = ct[sord[k]];
          const int sv = cd.kind ? 1 : 0, st = 1 - sv;  // kind 0: vertex of a, triangle of b
          const int *tc = T.tri + 3 * (toff[st] + cd.j);
          const int t0 = tc[0], t1 = tc[1], t2 = tc[2];
          const int64_t gid[4] = {voff[sv] + cd.i, voff[st] + t0, voff[st] + t1, voff[st] + t2};
#pragma unroll
          for (int role = 0; role < 4; ++role) kk[role] = ((uint64_t)gid[role] << 24) | (uint64_t)(4 * k + role);
        }
#pragma unroll
        for (int role = 0; role < 4; ++role) skey[kp(4 * k + role)] = kk[role];
      }
      __syncthreads();
      sort_keys_lds(skey, nj2);
      write_rows(
          nj, [&](int e) { return skey[kp(e)] >> 24; },
          [&](int e) {
            const int x = (int)(skey[kp(e)] & 0xffffffu);
            return sord[x >> 2] * 4 + (x & 3);
          },
          s_cnt, ct_grad, row_vtx_tmp + 4 * off, row_g_tmp + 3 * (4 * off), pair_rows + p);
    } else {
      // global slices of 8*n >= nj2 entries; the sorted VT order is kept aside
      // first (the slices are reused), in the row slice, free until the rows
      // are written
      uint64_t *jkey = gkeys + 8 * off;
      int32_t *jidx = gidx + 8 * off;
      int32_t *ord = row_vtx_tmp + 4 * off;
      for (int k = threadIdx.x; k < nvt; k += blockDim.x) ord[k] = idx[k];
      __threadfence_block();
      __syncthreads();
      for (int k = threadIdx.x; k < nj2 / 4; k += kAggThreads) {
        if (k < nvt) {
          const int32_t c = ord[k];
          const Cand cd = ct[c];
          const int sv = cd.kind ? 1 : 0, st = 1 - sv;
          const int *tc = T.tri + 3 * (toff[st] + cd.j);
          const int t0 = tc[0], t1 = tc[1], t2 = tc[2];
          const int64_t gid[4] = {voff[sv] + cd.i, voff[st] + t0, voff[st] + t1, voff[st] + t2};
#pragma unroll
          for (int role = 0; role < 4; ++role) {
            jkey[4 * k + role] = ((uint64_t)gid[role] << 24) | (uint64_t)(4 * k + role);
            jidx[4 * k + role] = c * 4 + role;
          }
        } else {
#pragma unroll
          for (int role = 0; role < 4; ++role) {
            jkey[4 * k + role] = ~0ull;
            jidx[4 * k + role] = -1;
          }
        }
      }
      __threadfence_block();
      __syncthreads();
      bitonic_global(jkey, jidx, nj2);
      write_rows(
          nj, [&](int e) { return jkey[e] >> 24; }, [&](int e) { return jidx[e]; }, s_cnt, ct_grad,
          row_vtx_tmp + 4 * off, row_g_tmp + 3 * (4 * off), pair_rows + p);
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

void launch_ct_scatter_order(const Cand *ct, int64_t ct_cap, Counters *cnt, const int64_t *pair_off,
                             int32_t *cursor, int32_t *perm, int64_t pairs_cap, int32_t *order, double *pair_V,
                             int32_t *pair_hasvt, int32_t *pair_rows, hipStream_t st) {
  const int ns = g1(ct_cap, 256), no = g1(pairs_cap, 256);
  k_ct_scatter_order<<<ns + no, 256, 0, st>>>(ct, ct_cap, cnt, pair_off, cursor, perm, pairs_cap, order, pair_V,
                                              pair_hasvt, pair_rows, ns);
}
void launch_ct_sort_aggregate(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                              const Counters *cnt, const int32_t *order, const int64_t *pair_off, const int32_t *perm,
                              const Cand *ct,
                              const double *ct_s, const double *ct_vol, const double *ct_grad, double dt,
                              uint64_t *gkeys, int32_t *gidx, int32_t *out_key, double *out_tau, double *out_s,
                              double *out_vol, double *out_grad, int64_t cap_ct, double *pair_V, int32_t *pair_hasvt,
                              int32_t *pair_rows, int32_t *row_vtx_tmp, double *row_g_tmp, hipStream_t st) {
  k_ct_sort_aggregate<<<g1(pairs_cap, 1), kAggThreads, 0, st>>>(
      S, T, pairs, cnt, order, pair_off, perm, ct, ct_s, ct_vol, ct_grad, dt, gkeys, gidx, out_key, out_tau, out_s, out_vol,
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

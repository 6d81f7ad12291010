// Sparse LCP matrix B = J M J^T of the contact volumes (Sec. 3.3.3, Alg. 3):
// B(j,k) = sum over vesicles i of g_j,i . M_i g_k,i, where g_j,i is row j
// of the contact-volume Jacobian restricted to the points of vesicle i and
// M_i is the vesicle's block of the operator (A_ii^-1 G_ii in the paper;
// supplied by the caller).  Only the points that appear in J matter, so M_i
// is given on the vesicle's active points: a dense [3 a_i][3 a_i] row-major
// block, point-major with x, y, z inside, in the order of the active list.
//
// Layout: flag the active points, count and list them per vesicle (one
// workgroup per vesicle), offsets of the blocks.  Assembly: list the volumes
// of every vesicle, then one workgroup per vesicle forms z_j = g_j^T M_i for
// each of its volumes and the dots z_j . g_k; contributions of different
// vesicles to the same (j,k) are merged after a stable sort by (j,k) (so
// every sum runs in vesicle order: deterministic).
#include "stiv_common.h"

namespace stiv {

namespace {

constexpr int kLcpThreads = 256;

__device__ inline int ves_of_vertex(const int *vtx_off, int n_ves, int v) {
  int lo = 0, hi = n_ves - 1;  // last i with vtx_off[i] <= v
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (vtx_off[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_lcp_flag(const int *j_vtx, int64_t n, int32_t *flag) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    flag[j_vtx[r]] = 1;
}

// Exclusive scan of one int per thread over the workgroup; returns the total.
__device__ inline int block_excl(int v, int *sh, int *out) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kLcpThreads; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  *out = sh[t] - v;
  const int tot = sh[kLcpThreads - 1];
  __syncthreads();
  return tot;
}

// a_i = number of active points of vesicle i; m9[i] = 9 a_i^2.
__global__ __launch_bounds__(kLcpThreads) void k_lcp_count_act(const int *vtx_off, int n_ves, const int32_t *flag,
                                                               int32_t *a, int64_t *m9) {
  __shared__ int sh[kLcpThreads];
  for (int i = blockIdx.x; i < n_ves; i += gridDim.x) {
    int c = 0;
    for (int v = vtx_off[i] + threadIdx.x; v < vtx_off[i + 1]; v += blockDim.x) c += flag[v];
    int ex;
    const int tot = block_excl(c, sh, &ex);
    if (threadIdx.x == 0) {
      a[i] = tot;
      m9[i] = 9ll * tot * tot;
    }
  }
}

__global__ __launch_bounds__(kLcpThreads) void k_lcp_emit_act(const int *vtx_off, int n_ves, const int32_t *flag,
                                                              const int64_t *act_off, int32_t *act_vtx) {
  __shared__ int sh[kLcpThreads];
  for (int i = blockIdx.x; i < n_ves; i += gridDim.x) {
    int64_t base = act_off[i];
    for (int v0 = vtx_off[i]; v0 < vtx_off[i + 1]; v0 += blockDim.x) {
      const int v = v0 + threadIdx.x;
      const int f = v < vtx_off[i + 1] ? flag[v] : 0;
      int ex;
      const int tot = block_excl(f, sh, &ex);
      if (f) act_vtx[base + ex] = v;
      base += tot;
    }
  }
}

// Volumes touching each vesicle (a volume belongs to the pair (a, b)).
__global__ void k_lcp_vcount(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, int32_t *vcnt) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_vol; j += (int64_t)gridDim.x * blockDim.x) {
    const int p = vol_pair[j];
    const int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
    atomicAdd(&vcnt[a], 1);
    if (b != a) atomicAdd(&vcnt[b], 1);
  }
}

__global__ void k_lcp_vscatter(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, const int64_t *voff,
                               int32_t *vcur, int32_t *vlist) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_vol; j += (int64_t)gridDim.x * blockDim.x) {
    const int p = vol_pair[j];
    const int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
    vlist[voff[a] + atomicAdd(&vcur[a], 1)] = (int)j;
    if (b != a) vlist[voff[b] + atomicAdd(&vcur[b], 1)] = (int)j;
  }
}

__global__ void k_lcp_c2(const int64_t *voff, int n_ves, int64_t *c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ves; i += gridDim.x * blockDim.x) {
    const int64_t m = voff[i + 1] - voff[i];
    c2[i] = m * m;
  }
}

// first index in [lo, hi) with a[idx] >= key (a ascending)
__device__ inline int64_t lower_i32(const int32_t *a, int64_t lo, int64_t hi, int key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

constexpr int kLcpMaxVol = 128;   // volumes per vesicle
constexpr int kLcpMaxAct = 2048;  // active points per vesicle

struct LcpLds {
  int vol[kLcpMaxVol];
  int64_t rs[kLcpMaxVol], re[kLcpMaxVol];  // rows of each volume on this vesicle
  double z[3 * kLcpMaxAct];
  double red[kLcpThreads];
};

// One workgroup per vesicle: contributions g_j^T M_i g_k of all its volume pairs.
__global__ __launch_bounds__(kLcpThreads) void k_lcp_block(const int *vtx_off, int n_ves, const int64_t *act_off,
                                                           const int64_t *m_off, const int32_t *act_vtx,
                                                           const double *M, const int64_t *voff,
                                                           const int32_t *vlist, const int32_t *j_vol,
                                                           const int32_t *j_vtx, const double *j_g, int64_t n_jrow,
                                                           const int64_t *coff, uint64_t *ckey, double *cval,
                                                           unsigned long long *overflow) {
  __shared__ LcpLds L;
  const int t = threadIdx.x;
  for (int i = blockIdx.x; i < n_ves; i += gridDim.x) {
    const int m = (int)(voff[i + 1] - voff[i]);
    const int64_t a0 = act_off[i];
    const int na = (int)(act_off[i + 1] - a0);
    if (m == 0) continue;
    if (m > kLcpMaxVol || na > kLcpMaxAct) {
      if (t == 0) atomicAdd(overflow, 1ull);
      continue;
    }
    if (t == 0) {
      // volumes in ascending order (the scatter order is arbitrary)
      for (int q = 0; q < m; ++q) {
        const int v = vlist[voff[i] + q];
        int r = q;
        while (r > 0 && L.vol[r - 1] > v) { L.vol[r] = L.vol[r - 1]; --r; }
        L.vol[r] = v;
      }
    }
    __syncthreads();
    if (t < m) {
      const int j = L.vol[t];
      const int64_t r0 = lower_i32(j_vol, 0, n_jrow, j), r1 = lower_i32(j_vol, r0, n_jrow, j + 1);
      // rows of a volume are sorted by vertex: the vesicle's points form one run
      L.rs[t] = lower_i32(j_vtx, r0, r1, vtx_off[i]);
      L.re[t] = lower_i32(j_vtx, r0, r1, vtx_off[i + 1]);
    }
    __syncthreads();
    const double *Mi = M + m_off[i];
    const int n3 = 3 * na;
    for (int jj = 0; jj < m; ++jj) {
      // z = g_j^T M_i (row-major M_i: coalesced along columns)
      for (int c = t; c < n3; c += blockDim.x) {
        double s = 0.0;
        for (int64_t r = L.rs[jj]; r < L.re[jj]; ++r) {
          const int64_t loc = lower_i32(act_vtx, a0, a0 + na, j_vtx[r]) - a0;
          for (int al = 0; al < 3; ++al) s += j_g[3 * r + al] * Mi[(3 * loc + al) * (int64_t)n3 + c];
        }
        L.z[c] = s;
      }
      __syncthreads();
      for (int kk = 0; kk < m; ++kk) {
        // B(j,k) contribution = z . g_k over the rows of k on this vesicle
        double s = 0.0;
        for (int64_t r = L.rs[kk] + t; r < L.re[kk]; r += blockDim.x) {
          const int64_t loc = lower_i32(act_vtx, a0, a0 + na, j_vtx[r]) - a0;
          for (int be = 0; be < 3; ++be) s += L.z[3 * loc + be] * j_g[3 * r + be];
        }
        L.red[t] = s;
        __syncthreads();
        for (int off = kLcpThreads / 2; off > 0; off >>= 1) {
          if (t < off) L.red[t] += L.red[t + off];
          __syncthreads();
        }
        if (t == 0) {
          const int64_t o = coff[i] + (int64_t)jj * m + kk;
          ckey[o] = ((uint64_t)(uint32_t)L.vol[jj] << 32) | (uint32_t)L.vol[kk];
          cval[o] = L.red[0];
        }
        __syncthreads();
      }
    }
  }
}

__global__ void k_lcp_runs(const uint64_t *key, int64_t n, int32_t *start) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
    start[s] = (s == 0 || key[s] != key[s - 1]) ? 1 : 0;
}

// Sum every run of equal keys in sorted (vesicle) order.
__global__ void k_lcp_reduce(const uint64_t *key, const uint32_t *idx, const double *cval, int64_t n,
                             const int32_t *start, const int64_t *pos, int32_t *b_row, int32_t *b_col, double *b_val,
                             int64_t cap) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    if (!start[s]) continue;
    double v = 0.0;
    int64_t e = s;
    while (e < n && key[e] == key[s]) v += cval[idx[e++]];
    const int64_t o = pos[s];
    if (o < cap) {
      b_row[o] = (int32_t)(key[s] >> 32);
      b_col[o] = (int32_t)(key[s] & 0xffffffffu);
      b_val[o] = v;
    }
  }
}

int grid1(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

void launch_lcp_layout(const int *vtx_off, int n_ves, const int32_t *j_vtx, int64_t n_jrow, int32_t *flag,
                       int32_t *a, int64_t *m9, hipStream_t st) {
  if (n_jrow > 0) k_lcp_flag<<<grid1(n_jrow), 256, 0, st>>>(j_vtx, n_jrow, flag);
  if (n_ves > 0) k_lcp_count_act<<<n_ves < 4096 ? n_ves : 4096, kLcpThreads, 0, st>>>(vtx_off, n_ves, flag, a, m9);
}

void launch_lcp_emit(const int *vtx_off, int n_ves, const int32_t *flag, const int64_t *act_off, int32_t *act_vtx,
                     hipStream_t st) {
  if (n_ves > 0) k_lcp_emit_act<<<n_ves < 4096 ? n_ves : 4096, kLcpThreads, 0, st>>>(vtx_off, n_ves, flag, act_off, act_vtx);
}

void launch_lcp_vcount(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, int32_t *vcnt, hipStream_t st) {
  if (n_vol > 0) k_lcp_vcount<<<grid1(n_vol), 256, 0, st>>>(vol_pair, pair_ab, n_vol, vcnt);
}

void launch_lcp_vscatter(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, const int64_t *voff,
                         int32_t *vcur, int32_t *vlist, int n_ves, int64_t *c2, hipStream_t st) {
  if (n_vol > 0) k_lcp_vscatter<<<grid1(n_vol), 256, 0, st>>>(vol_pair, pair_ab, n_vol, voff, vcur, vlist);
  if (n_ves > 0) k_lcp_c2<<<grid1(n_ves), 256, 0, st>>>(voff, n_ves, c2);
}

void launch_lcp_block(const int *vtx_off, int n_ves, const int64_t *act_off, const int64_t *m_off,
                      const int32_t *act_vtx, const double *M, const int64_t *voff, const int32_t *vlist,
                      const int32_t *j_vol, const int32_t *j_vtx, const double *j_g, int64_t n_jrow,
                      const int64_t *coff, uint64_t *ckey, double *cval, unsigned long long *overflow,
                      hipStream_t st) {
  if (n_ves > 0)
    k_lcp_block<<<n_ves < 4096 ? n_ves : 4096, kLcpThreads, 0, st>>>(vtx_off, n_ves, act_off, m_off, act_vtx, M, voff,
                                                                   vlist, j_vol, j_vtx, j_g, n_jrow, coff, ckey, cval,
                                                                   overflow);
}

void launch_lcp_runs(const uint64_t *key, int64_t n, int32_t *start, hipStream_t st) {
  if (n > 0) k_lcp_runs<<<grid1(n), 256, 0, st>>>(key, n, start);
}

void launch_lcp_reduce(const uint64_t *key, const uint32_t *idx, const double *cval, int64_t n, const int32_t *start,
                       const int64_t *pos, int32_t *b_row, int32_t *b_col, double *b_val, int64_t cap,
                       hipStream_t st) {
  if (n > 0) k_lcp_reduce<<<grid1(n), 256, 0, st>>>(key, idx, cval, n, start, pos, b_row, b_col, b_val, cap);
}

}  // namespace stiv

// Backward pass (adjoint) of the contact volumes and their gradients.
//
// The forward produces V per contact volume and the Jacobian rows
// G = dV/dX1 per (volume, vertex).  Given cotangents dL/dV and dL/dG this
// computes dL/dX0 and dL/dX1.  For every vertex-triangle contact k of a
// volume, with gV = dL/dV and w = the dL/dG rows of its four vertices,
//   dL/dX += gV grad V_k + d/de [grad V_k](X1 + e w)
// (the Hessian of V_k applied to w; Hessians are symmetric), where grad is
// the full gradient with respect to X0 and X1 including the dependence of
// the contact time on the positions.  The directional derivative is taken
// in forward mode with dual numbers (narrow_math.h).  Contributions are
// summed per (volume, vertex) in canonical contact order, as the forward
// forms J rows, into that J row's slot; the rows are then sorted by vertex
// (stably, so volumes stay in order) and each vertex adds its rows in that
// order and is written once.  No floating-point atomics: repeated calls give
// the same bits.
#include <mutex>

#include "narrow_math.h"

namespace stiv {

namespace {

// Scratch of stiv_backward_static: one array per GPU, held by the process
// for as long as it runs.  Host code never passes `scratch` itself to a
// kernel (on the host that name is not a device address): it passes the
// address hipGetSymbolAddress reports for the current device.
constexpr size_t kBwdStaticBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kBwdStaticBytes];

constexpr int kBwdThreads = 256;
constexpr int kBwdLds = 2048;

__device__ int64_t lower_bound_i32(const int32_t *a, int64_t n, int32_t v, int stride) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid * stride] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ void bitonic_sort(uint64_t *key, int32_t *idx, int n_pow2) {
  for (int size = 2; size <= n_pow2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n_pow2 >> 1); t += blockDim.x) {
        const int i = 2 * stride * (t / stride) + (t % stride);
        const int j = i + stride;
        const bool asc = (i & size) == 0;
        const uint64_t ki = key[i], kj = key[j];
        if ((ki > kj) == asc) {
          key[i] = kj; key[j] = ki;
          const int32_t x = idx[i]; idx[i] = idx[j]; idx[j] = x;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
}

__global__ __launch_bounds__(kBwdThreads) void k_bwd_volume(
    DevScene S, DevTopo T, double d, double eps, double dt, int64_t n_ct, const int32_t *ct_key,
    const double *ct_tau, const int32_t *pair_ab, const int32_t *pair_shift, int64_t n_vol, const int32_t *vol_pair,
    int64_t n_jrow, const int32_t *j_vol, const int32_t *j_vtx, const double *dV, const double *dG, double *contrib,
    uint64_t *gkeys, int32_t *gidx, const double *ct_s, double *rowc) {
  __shared__ uint64_t skey[kBwdLds];
  __shared__ int32_t sidx[kBwdLds];
  const int64_t NV = S.n_vtx;
  for (int64_t v = blockIdx.x; v < n_vol; v += gridDim.x) {
    const int p = vol_pair[v];
    const int64_t c0 = lower_bound_i32(ct_key, n_ct, p, 4);
    const int64_t c1 = lower_bound_i32(ct_key, n_ct, p + 1, 4);
    int64_t nvt = 0;
    while (c0 + nvt < c1 && ct_key[4 * (c0 + nvt) + 1] < 2) ++nvt;  // VT contacts come first
    const int64_t r0 = lower_bound_i32(j_vol, n_jrow, (int32_t)v, 1);
    const int64_t r1 = lower_bound_i32(j_vol, n_jrow, (int32_t)v + 1, 1);
    const int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
    // image shift of b: sigma * L of the pair's scene
    int lo_s = 0, hi_s = S.n_scenes;
    while (hi_s - lo_s > 1) {
      const int mid = (lo_s + hi_s) >> 1;
      if (S.scene_off[mid] <= a) lo_s = mid; else hi_s = mid;
    }
    double sh[3];
    for (int c = 0; c < 3; ++c) sh[c] = (double)pair_shift[3 * p + c] * S.box_len[3 * lo_s + c];
    const double gV = dV ? dV[v] : 0.0;
    const int nj = (int)(4 * nvt);
    int nj2 = 1;
    while (nj2 < nj) nj2 <<= 1;
    uint64_t *key = skey;
    int32_t *idx = sidx;
    if (nj2 > kBwdLds) { key = gkeys + 8 * c0; idx = gidx + 8 * c0; }
    for (int64_t k = threadIdx.x; k < nvt; k += blockDim.x) {
      const int32_t *kk = ct_key + 4 * (c0 + k);
      const int kind = kk[1];
      const int vv = kind ? b : a, vt = kind ? a : b;
      const int *tri = T.tri + 3 * ((int64_t)T.tri_off[S.topo_id[vt]] + kk[3]);
      int64_t gid[4];
      gid[0] = S.vtx_off[vv] + kk[2];
      for (int r = 0; r < 3; ++r) gid[1 + r] = S.vtx_off[vt] + tri[r];
      nm::V3<double> X0[4], X1[4];
      double w[12];
      for (int r = 0; r < 4; ++r) {
        const bool shifted = (r == 0) ? (kind == 1) : (kind == 0);
        const double sx = shifted ? sh[0] : 0.0, sy = shifted ? sh[1] : 0.0, sz = shifted ? sh[2] : 0.0;
        X0[r] = nm::V3<double>{S.x0[gid[r]] + sx, S.x0[NV + gid[r]] + sy, S.x0[2 * NV + gid[r]] + sz};
        X1[r] = nm::V3<double>{S.x1[gid[r]] + sx, S.x1[NV + gid[r]] + sy, S.x1[2 * NV + gid[r]] + sz};
        // the J row of this vertex in this volume (rows are sorted by vertex)
        int64_t lo = r0, hi = r1;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (j_vtx[mid] < gid[r]) lo = mid + 1; else hi = mid;
        }
        const bool found = lo < r1 && j_vtx[lo] == gid[r];
        for (int c = 0; c < 3; ++c) w[3 * r + c] = (dG && found) ? dG[3 * lo + c] : 0.0;
      }
      const double s = ct_s ? ct_s[c0 + k] : ct_tau[c0 + k] / dt;
      double g0[12], g1[12];
      nm::vt_vjp(X0, X1, s, d, eps, dt, s == 0.0, gV, w, g0, g1);
      for (int r = 0; r < 4; ++r) {
        double *dst = contrib + 6 * (4 * (c0 + k) + r);
        for (int c = 0; c < 3; ++c) { dst[c] = g0[3 * r + c]; dst[3 + c] = g1[3 * r + c]; }
        const int e = (int)(4 * k + r);
        key[e] = ((uint64_t)gid[r] << 24) | (uint64_t)e;
        idx[e] = (int32_t)(4 * (c0 + k) + r);
      }
    }
    for (int e = nj + threadIdx.x; e < nj2; e += blockDim.x) { key[e] = ~0ull; idx[e] = -1; }
    __threadfence_block();
    __syncthreads();
    bitonic_sort(key, idx, nj2);
    // one thread per run of equal vertices adds the run in contact order and
    // stores the sum in the slot of that vertex's J row of this volume (every
    // vertex of a vertex-triangle contact has one: the rows are sorted by
    // vertex inside the volume)
    for (int e = threadIdx.x; e < nj; e += blockDim.x) {
      const uint64_t gv = key[e] >> 24;
      if (e > 0 && (key[e - 1] >> 24) == gv) continue;
      double acc[6] = {0, 0, 0, 0, 0, 0};
      for (int f = e; f < nj && (key[f] >> 24) == gv; ++f)
        for (int c = 0; c < 6; ++c) acc[c] += contrib[6 * (int64_t)idx[f] + c];
      int64_t lo = r0, hi = r1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((uint64_t)j_vtx[mid] < gv) lo = mid + 1; else hi = mid;
      }
      if (lo < r1 && (uint64_t)j_vtx[lo] == gv)
        for (int c = 0; c < 6; ++c) rowc[6 * lo + c] = acc[c];
    }
    __syncthreads();
  }
}

__global__ void k_zero(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Row sums start at zero (a row whose vertices have no vertex-triangle
// contact in its volume cannot occur, but a zero keeps every slot defined);
// sort keys are the rows' vertices, values the row indices.
__global__ void k_bwd_rows_init(const int32_t *j_vtx, int64_t n_jrow, double *rowc, uint64_t *rkey, uint32_t *rval) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_jrow; i += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < 6; ++c) rowc[6 * i + c] = 0.0;
    rkey[i] = (uint64_t)(uint32_t)j_vtx[i];
    rval[i] = (uint32_t)i;
  }
}

// Rows sorted by vertex (stable: volumes in order): the first entry of each
// run adds the run in order and writes its vertex once.
__global__ void k_bwd_vertex_sum(const uint64_t *rkey, const uint32_t *rval, int64_t n_jrow, const double *rowc,
                                 int64_t NV, double *dX0, double *dX1) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_jrow; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t gv = rkey[e];
    if (e > 0 && rkey[e - 1] == gv) continue;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t f = e; f < n_jrow && rkey[f] == gv; ++f)
      for (int c = 0; c < 6; ++c) acc[c] += rowc[6 * (int64_t)rval[f] + c];
    for (int c = 0; c < 3; ++c) {
      if (dX0) dX0[c * NV + (int64_t)gv] = acc[c];
      if (dX1) dX1[c * NV + (int64_t)gv] = acc[3 + c];
    }
  }
}

}  // namespace

size_t backward_static_bytes() { return kBwdStaticBytes; }

// Device address of `scratch` on `device`, looked up once per device with
// that device current and kept for the life of the process.
hipError_t backward_static_scratch(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) {
      e = hipSetDevice(device);
      if (e != hipSuccess) return e;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

BwdLayout backward_layout(int64_t n_ct, int64_t n_jrow) {
  BwdLayout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t nc = (size_t)(n_ct + 1), nj = (size_t)(n_jrow + 1);
  L.contrib = take(6 * 8 * 4 * nc);
  L.gkeys = take(8 * 8 * nc);
  L.gidx = take(4 * 8 * nc);
  L.rowc = take(6 * 8 * nj);
  L.rkey = take(8 * nj);
  L.rval = take(4 * nj);
  L.tk = take(8 * nj);
  L.tv = take(4 * nj);
  L.hist = take(4 * (size_t)(256 * radix_scratch_blocks((int64_t)nj)));
  L.hoff = take(8 * (size_t)radix_offset_elems((int64_t)nj));
  L.total = at;
  return L;
}

void launch_backward(const DevScene &S, const DevTopo &T, double d, double eps, double dt, int64_t n_ct,
                     const int32_t *ct_key, const double *ct_tau, const int32_t *pair_ab, const int32_t *pair_shift,
                     int64_t n_vol, const int32_t *vol_pair, int64_t n_jrow, const int32_t *j_vol,
                     const int32_t *j_vtx, const double *dV, const double *dG, const double *ct_s, double *contrib,
                     uint64_t *gkeys, int32_t *gidx, double *rowc, uint64_t *rkey, uint32_t *rval, uint64_t *tk,
                     uint32_t *tv, int32_t *hist, int64_t *hoff, double *dX0, double *dX1, hipStream_t st) {
  const int64_t n3 = 3 * (int64_t)S.n_vtx;
  int64_t gz = (n3 + 255) / 256;
  gz = gz > 4096 ? 4096 : (gz < 1 ? 1 : gz);
  if (dX0) k_zero<<<(int)gz, 256, 0, st>>>(dX0, n3);
  if (dX1) k_zero<<<(int)gz, 256, 0, st>>>(dX1, n3);
  if (n_vol <= 0 || n_jrow <= 0) return;
  int64_t gr = (n_jrow + 255) / 256;
  gr = gr > 4096 ? 4096 : gr;
  k_bwd_rows_init<<<(int)gr, 256, 0, st>>>(j_vtx, n_jrow, rowc, rkey, rval);
  int64_t g = n_vol < 8192 ? n_vol : 8192;
  k_bwd_volume<<<(int)g, kBwdThreads, 0, st>>>(S, T, d, eps, dt, n_ct, ct_key, ct_tau, pair_ab, pair_shift, n_vol,
                                               vol_pair, n_jrow, j_vol, j_vtx, dV, dG, contrib, gkeys, gidx, ct_s,
                                               rowc);
  launch_radix_sort_u64(rkey, rval, tk, tv, nullptr, n_jrow, 32, hist, hoff, st);
  k_bwd_vertex_sum<<<(int)gr, 256, 0, st>>>(rkey, rval, n_jrow, rowc, (int64_t)S.n_vtx, dX0, dX1);
}

}  // namespace stiv

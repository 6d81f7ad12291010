// Host side of libstiv: context, topology tiling, scratch arena, the detect
// pipeline and the C ABI declared in include/stiv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/stiv.h"
#include "stiv_common.h"

using namespace stiv;

namespace {

// ---------------------------------------------------------------------------
// Device buffer helper
// ---------------------------------------------------------------------------
struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

hipError_t ensure(Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return hipSuccess;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

template <typename T>
T *P(Buf &b) {
  return reinterpret_cast<T *>(b.p);
}

int64_t pow2_at_least(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

}  // namespace

struct stiv_ctx {
  int device = 0;
  std::string err;
  bool have_topo = false;
  // topology (device)
  Buf t_nv, t_nt, t_ne, t_tri_off, t_edge_off, t_tri, t_edge, t_patch_off, t_ptri_off, t_ptri, t_ptri_slot,
      t_pvtx_off, t_pvtx, t_pvtx_slot, t_pedge_off, t_pedge, t_pedge_slot, t_pref_off, t_pref, t_vbase, t_vp_off,
      t_vp, t_vp4, t_blob, t_tri_rec;
  DevTopo topo{};
  std::vector<int> h_npatch;  // patches per topology
  int max_patches = 0;
  int tile = 64;            // triangles per patch (16, 32 or 64)
  int prim_blocks = 4096;   // workgroups of the primitive-candidate kernel (1440 vesicles: 2048 1.25 ms
                            // per step, 4096 1.21, 8192 1.23, 16384 1.29)
  int narrow_blocks = 8192; // upper bound on workgroups of the root-search kernel
  // arena
  Buf counters, ves_box, ves_scene, grid, cp_cnt, cp_off, cp_keys, cp_vals, cp_tk, cp_tv, hash, uniq, sorted,
      cnt_a, cursor_a, off_a, pairs, ves_patch_cnt, ves_patch_off, patch_box, patch_dop, work, cand, hard, cand_list,
      ct,
      ct_s, ct_vol,
      ct_grad, pair_cnt, pair_cursor, pair_off, perm, gkeys, gidx, pair_V, pair_hasvt, pair_rows, vol_off,
      row_off, row_vtx, row_g, sort_tk, sort_tv, bwd_scratch, hard_geo, rs_hist, rs_off, scan_tmp;
  // learned contact-time bracket: FP32 parameters on the device, width in units of sd
  Buf toi_params, toi_packed, mlp_part;
  // LCP matrix assembly scratch
  Buf lcp_flag, lcp_a, lcp_m9, lcp_vcnt, lcp_vcur, lcp_voff, lcp_vlist, lcp_c2, lcp_coff, lcp_ckey, lcp_cval,
      lcp_cidx, lcp_tk, lcp_tv, lcp_start, lcp_pos, lcp_ovf;
  bool have_model = false;
  float toi_kwidth = 3.0f;
  int64_t cap_cp = 0, cap_pairs = 0, cap_work = 0, cap_cand = 0, cap_ct = 0, cap_patch = 0, cap_list = 0;
  int64_t arena_n_ves = 0, arena_max_patches = 0;
  Counters *h_cnt = nullptr;  // pinned
  // last structurally validated scene (pointers + sizes); see check_structure
  const void *val_ptr[4] = {};
  int64_t val_size[3] = {-1, -1, -1};
  hipEvent_t ev[9] = {};  // ev[8] marks the start, ev[0..7] stage boundaries
  // a second stream (default priority) on which the patch supports overlap the
  // vesicle broad phase, joined back into the call's stream by events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  float stage_ms[8] = {};
};

namespace {

// Histogram and offset scratch of the radix sort for up to n keys.
hipError_t ensure_sort_scratch(stiv_ctx *ctx, int64_t n) {
  const int64_t nb = radix_scratch_blocks(n > 0 ? n : 1);
  hipError_t e = ensure(ctx->rs_hist, 4 * (size_t)(256 * nb));
  if (e != hipSuccess) return e;
  return ensure(ctx->rs_off, 8 * (size_t)radix_offset_elems(n > 0 ? n : 1));
}

stiv_status fail(stiv_ctx *c, stiv_status s, const std::string &m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(ctx, STIV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <typename T>
hipError_t upload(Buf &b, const std::vector<T> &v) {
  hipError_t e = ensure(b, std::max<size_t>(v.size() * sizeof(T), 16));
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

extern "C" {

stiv_status stiv_create(stiv_ctx **out, int dev) {
  if (!out) return STIV_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || dev < 0 || dev >= n) return STIV_E_ARG;
  if (hipSetDevice(dev) != hipSuccess) return STIV_E_HIP;
  stiv_ctx *ctx = new stiv_ctx();
  ctx->device = dev;
  if (hipHostMalloc((void **)&ctx->h_cnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return STIV_E_HIP;
  }
  for (auto &e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      stiv_destroy(ctx);
      return STIV_E_HIP;
    }
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) != hipSuccess) {
    stiv_destroy(ctx);
    return STIV_E_HIP;
  }
  // the device address of stiv_backward_static's scratch, once per device
  void *scratch_addr = nullptr;
  if (backward_static_scratch(dev, &scratch_addr) != hipSuccess) {
    stiv_destroy(ctx);
    return STIV_E_HIP;
  }
  *out = ctx;
  return STIV_OK;
}

stiv_status stiv_destroy(stiv_ctx *ctx) {
  if (!ctx) return STIV_E_ARG;
  (void)hipSetDevice(ctx->device);
  Buf *all[] = {&ctx->t_nv, &ctx->t_nt, &ctx->t_ne, &ctx->t_tri_off, &ctx->t_edge_off, &ctx->t_tri, &ctx->t_edge,
                &ctx->t_patch_off, &ctx->t_ptri_off, &ctx->t_ptri, &ctx->t_ptri_slot, &ctx->t_pvtx_off,
                &ctx->t_pvtx, &ctx->t_pvtx_slot, &ctx->t_pedge_off, &ctx->t_pedge, &ctx->t_pedge_slot,
                &ctx->t_pref_off, &ctx->t_pref, &ctx->t_vbase, &ctx->t_vp_off, &ctx->t_vp, &ctx->t_vp4,
                &ctx->t_blob, &ctx->t_tri_rec, &ctx->hard_geo, &ctx->rs_hist, &ctx->rs_off, &ctx->scan_tmp, &ctx->counters, &ctx->ves_box, &ctx->ves_scene, &ctx->grid,
                &ctx->cp_cnt, &ctx->cp_off, &ctx->cp_keys, &ctx->cp_vals, &ctx->cp_tk, &ctx->cp_tv, &ctx->hash,
                &ctx->uniq, &ctx->sorted, &ctx->cnt_a, &ctx->cursor_a, &ctx->off_a, &ctx->pairs,
                &ctx->ves_patch_cnt, &ctx->ves_patch_off, &ctx->patch_box, &ctx->patch_dop, &ctx->work, &ctx->cand, &ctx->hard,
                &ctx->cand_list, &ctx->ct,
                &ctx->toi_params, &ctx->toi_packed, &ctx->mlp_part, &ctx->lcp_flag, &ctx->lcp_a, &ctx->lcp_m9, &ctx->lcp_vcnt,
                &ctx->lcp_vcur, &ctx->lcp_voff, &ctx->lcp_vlist, &ctx->lcp_c2, &ctx->lcp_coff, &ctx->lcp_ckey,
                &ctx->lcp_cval, &ctx->lcp_cidx, &ctx->lcp_tk, &ctx->lcp_tv, &ctx->lcp_start, &ctx->lcp_pos,
                &ctx->lcp_ovf,
                &ctx->ct_s, &ctx->ct_vol, &ctx->ct_grad, &ctx->pair_cnt, &ctx->pair_cursor, &ctx->pair_off,
                &ctx->perm, &ctx->gkeys, &ctx->gidx, &ctx->pair_V, &ctx->pair_hasvt, &ctx->pair_rows,
                &ctx->vol_off, &ctx->row_off, &ctx->row_vtx, &ctx->row_g, &ctx->sort_tk, &ctx->sort_tv,
                &ctx->bwd_scratch};
  for (Buf *b : all)
    if (b->p) (void)hipFree(b->p);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->h_cnt) (void)hipHostFree(ctx->h_cnt);
  delete ctx;
  return STIV_OK;
}

const char *stiv_last_error(const stiv_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ---------------------------------------------------------------------------
// Topology: copy and tile into patches of neighbouring triangles.
// ---------------------------------------------------------------------------
stiv_status stiv_set_topology(stiv_ctx *ctx, const stiv_topology *tp) {
  if (!ctx || !tp || tp->n_topo <= 0 || !tp->nv || !tp->tri || !tp->tri_off || !tp->edge || !tp->edge_off)
    return fail(ctx, STIV_E_ARG, "set_topology: null or empty topology");
  HIPCHK(hipSetDevice(ctx->device));
  const int nt_topo = tp->n_topo;
  std::vector<int> nv(nt_topo), ntv(nt_topo), nev(nt_topo), tri_off(nt_topo + 1), edge_off(nt_topo + 1);
  for (int t = 0; t <= nt_topo; ++t) { tri_off[t] = tp->tri_off[t]; edge_off[t] = tp->edge_off[t]; }
  std::vector<int> tri(3 * (size_t)tri_off[nt_topo]), edge(2 * (size_t)edge_off[nt_topo]);
  std::memcpy(tri.data(), tp->tri, tri.size() * sizeof(int));
  std::memcpy(edge.data(), tp->edge, edge.size() * sizeof(int));
  std::vector<int> patch_off(1, 0), ptri_off(1, 0), ptri, pvtx_off(1, 0), pvtx, pedge_off(1, 0), pedge,
      pref_off(1, 0), pref;
  std::vector<uint8_t> ptri_slot, pvtx_slot, pedge_slot;
  std::vector<int> vbase, vp_off(1, 0), vp, vp4;
  std::vector<int> tri_rec;  // per triangle in patch order: its three local vertex ids, its local patch
  int max_nv = 0;
  ctx->h_npatch.assign(nt_topo, 0);
  ctx->max_patches = 0;
  for (int t = 0; t < nt_topo; ++t) {
    nv[t] = tp->nv[t];
    ntv[t] = tri_off[t + 1] - tri_off[t];
    nev[t] = edge_off[t + 1] - edge_off[t];
    const int NT = ntv[t], NE = nev[t], NV = nv[t];
    if (NV <= 0 || NT <= 0 || NE <= 0) return fail(ctx, STIV_E_ARG, "set_topology: empty mesh");
    const int *T3 = tri.data() + 3 * (size_t)tri_off[t];
    const int *E2 = edge.data() + 2 * (size_t)edge_off[t];
    std::map<std::pair<int, int>, int> eid;
    for (int e = 0; e < NE; ++e) {
      int a = E2[2 * e], b = E2[2 * e + 1];
      if (a < 0 || b < 0 || a >= NV || b >= NV || a >= b)
        return fail(ctx, STIV_E_ARG, "set_topology: edges must be (lo, hi) local ids");
      eid[{a, b}] = e;
    }
    std::vector<int> tri_edges(3 * (size_t)NT);
    std::vector<std::vector<int>> edge_tris(NE);
    for (int k = 0; k < NT; ++k)
      for (int r = 0; r < 3; ++r) {
        int a = T3[3 * k + r], b = T3[3 * k + (r + 1) % 3];
        if (a < 0 || b < 0 || a >= NV || b >= NV) return fail(ctx, STIV_E_ARG, "set_topology: bad triangle");
        auto it = eid.find({std::min(a, b), std::max(a, b)});
        if (it == eid.end()) return fail(ctx, STIV_E_ARG, "set_topology: triangle edge missing from edge list");
        tri_edges[3 * k + r] = it->second;
        edge_tris[it->second].push_back(k);
      }
    for (int e = 0; e < NE; ++e)
      if (edge_tris[e].empty()) return fail(ctx, STIV_E_ARG, "set_topology: edge not on any triangle");
    std::vector<char> vref(NV, 0);
    for (int k = 0; k < 3 * NT; ++k) vref[T3[k]] = 1;
    for (int v = 0; v < NV; ++v)
      if (!vref[v]) return fail(ctx, STIV_E_ARG, "set_topology: vertex not on any triangle");
    // greedy breadth-first patches of up to 7/8 of `tile` neighbouring
    // triangles (a triangle is not added when the patch would exceed its
    // vertex or edge capacity for this patch size); the growth leaves small
    // islands behind, which are then merged into a neighbouring patch that
    // still has room (up to `tile` triangles within the capacities)
    int cap_ref = TileCaps<64>::ref, cap_edge = TileCaps<64>::owne;
    if (ctx->tile == 16) { cap_ref = TileCaps<16>::ref; cap_edge = TileCaps<16>::owne; }
    if (ctx->tile == 32) { cap_ref = TileCaps<32>::ref; cap_edge = TileCaps<32>::owne; }
    const int grow = ctx->tile - ctx->tile / 8;
    std::vector<int> tpatch(NT, -1);
    std::vector<std::vector<int>> patches;
    for (int seed = 0; seed < NT; ++seed) {
      if (tpatch[seed] >= 0) continue;
      std::vector<int> members, queue{seed};
      std::vector<int> verts, edges;
      size_t qh = 0;
      tpatch[seed] = (int)patches.size();
      while (qh < queue.size() && (int)members.size() < grow) {
        int k = queue[qh++];
        std::vector<int> nv2 = verts, ne2 = edges;
        for (int r = 0; r < 3; ++r) {
          if (std::find(nv2.begin(), nv2.end(), T3[3 * k + r]) == nv2.end()) nv2.push_back(T3[3 * k + r]);
          if (std::find(ne2.begin(), ne2.end(), tri_edges[3 * k + r]) == ne2.end()) ne2.push_back(tri_edges[3 * k + r]);
        }
        if ((int)nv2.size() > cap_ref || (int)ne2.size() > cap_edge) {
          tpatch[k] = -1;
          continue;
        }
        verts.swap(nv2);
        edges.swap(ne2);
        members.push_back(k);
        for (int r = 0; r < 3; ++r)
          for (int k2 : edge_tris[tri_edges[3 * k + r]])
            if (tpatch[k2] < 0) {
              tpatch[k2] = (int)patches.size();
              queue.push_back(k2);
            }
      }
      for (size_t q = qh; q < queue.size(); ++q) tpatch[queue[q]] = -1;  // release unvisited
      for (int k : members) tpatch[k] = (int)patches.size();
      patches.push_back(members);
    }
    {
      // islands of fewer than tile / 4 triangles join the smallest
      // edge-adjacent patch that can take them, until none can
      auto fits = [&](const std::vector<int> &tris) {
        if ((int)tris.size() > ctx->tile) return false;
        std::vector<int> vs, es;
        for (int k : tris)
          for (int r = 0; r < 3; ++r) {
            vs.push_back(T3[3 * k + r]);
            es.push_back(tri_edges[3 * k + r]);
          }
        std::sort(vs.begin(), vs.end());
        std::sort(es.begin(), es.end());
        const int nv = (int)(std::unique(vs.begin(), vs.end()) - vs.begin());
        const int ne = (int)(std::unique(es.begin(), es.end()) - es.begin());
        return nv <= cap_ref && ne <= cap_edge;
      };
      for (bool changed = true; changed;) {
        changed = false;
        for (size_t f = 0; f < patches.size(); ++f) {
          if (patches[f].empty() || (int)patches[f].size() >= ctx->tile / 4) continue;
          std::vector<int> nb;
          for (int k : patches[f])
            for (int r = 0; r < 3; ++r)
              for (int k2 : edge_tris[tri_edges[3 * k + r]])
                if (tpatch[k2] != (int)f) nb.push_back(tpatch[k2]);
          std::sort(nb.begin(), nb.end());
          nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
          std::stable_sort(nb.begin(), nb.end(),
                           [&](int a, int b) { return patches[a].size() < patches[b].size(); });
          for (int g : nb) {
            std::vector<int> tris = patches[g];
            tris.insert(tris.end(), patches[f].begin(), patches[f].end());
            if (!fits(tris)) continue;
            for (int k : patches[f]) tpatch[k] = g;
            patches[g].swap(tris);
            patches[f].clear();
            changed = true;
            break;
          }
        }
      }
      std::vector<std::vector<int>> kept;
      for (auto &pt : patches)
        if (!pt.empty()) kept.push_back(std::move(pt));
      patches.swap(kept);
      for (size_t pi = 0; pi < patches.size(); ++pi)
        for (int k : patches[pi]) tpatch[k] = (int)pi;
    }
    const int np = (int)patches.size();
    if (np > kMaxPatchesPerVes) return fail(ctx, STIV_E_ARG, "set_topology: mesh too large for the patch table");
    ctx->h_npatch[t] = np;
    ctx->max_patches = std::max(ctx->max_patches, np);
    max_nv = std::max(max_nv, NV);
    // the triangles' local vertex ids in patch order (the order of the patch
    // table's triangle lists), for the face-diagonal supports of each patch
    for (int pi = 0; pi < np; ++pi)
      for (int k : patches[pi]) tri_rec.insert(tri_rec.end(), {T3[3 * k], T3[3 * k + 1], T3[3 * k + 2], pi});
    {
      std::vector<std::vector<int>> vpl(NV);
      for (int pi = 0; pi < np; ++pi)
        for (int k : patches[pi])
          for (int r = 0; r < 3; ++r) {
            auto &l = vpl[T3[3 * k + r]];
            if (l.empty() || l.back() != pi) l.push_back(pi);
          }
      vbase.push_back((int)vp_off.size() - 1);
      for (int v = 0; v < NV; ++v) {
        std::sort(vpl[v].begin(), vpl[v].end());
        vpl[v].erase(std::unique(vpl[v].begin(), vpl[v].end()), vpl[v].end());
        for (int q : vpl[v]) vp.push_back(q);
        vp_off.push_back((int)vp.size());
        const int nq = (int)vpl[v].size();
        for (int k = 0; k < 4; ++k) vp4.push_back(nq > 4 ? (k < 3 ? vpl[v][k] : -2) : (k < nq ? vpl[v][k] : -1));
      }
    }
    std::vector<char> vown(NV, 0), eown(NE, 0);
    for (int pi = 0; pi < np; ++pi) {
      const auto &mem = patches[pi];
      std::vector<int> refs;
      for (int k : mem)
        for (int r = 0; r < 3; ++r) refs.push_back(T3[3 * k + r]);
      std::sort(refs.begin(), refs.end());
      refs.erase(std::unique(refs.begin(), refs.end()), refs.end());
      auto slot_of = [&](int v) { return (uint8_t)(std::lower_bound(refs.begin(), refs.end(), v) - refs.begin()); };
      for (int v : refs) pref.push_back(v);
      pref_off.push_back((int)pref.size());
      for (int k : mem) {
        ptri.push_back(k);
        for (int r = 0; r < 3; ++r) ptri_slot.push_back(slot_of(T3[3 * k + r]));
      }
      ptri_off.push_back((int)ptri.size());
      int nown_v = 0, nown_e = 0;
      for (int k : mem)
        for (int r = 0; r < 3; ++r) {
          int v = T3[3 * k + r];
          if (!vown[v]) {
            vown[v] = 1;
            pvtx.push_back(v);
            pvtx_slot.push_back(slot_of(v));
            ++nown_v;
          }
          int e = tri_edges[3 * k + r];
          if (!eown[e]) {
            eown[e] = 1;
            pedge.push_back(e);
            pedge_slot.push_back(slot_of(E2[2 * e]));
            pedge_slot.push_back(slot_of(E2[2 * e + 1]));
            ++nown_e;
          }
        }
      if (nown_v > cap_ref || nown_e > cap_edge || (int)refs.size() > cap_ref)
        return fail(ctx, STIV_E_ARG, "set_topology: patch exceeds tile limits");
      pvtx_off.push_back((int)pvtx.size());
      pedge_off.push_back((int)pedge.size());
    }
    patch_off.push_back(patch_off.back() + np);
  }
  // fixed-stride patch blobs for the current tile size
  int bs = 0;
  {
    auto build_blobs = [&](auto layout_tag) {
      using Lay = decltype(layout_tag);
      const int n_ptab = (int)ptri_off.size() - 1;
      std::vector<int> blob((size_t)n_ptab * Lay::stride, 0);
      for (int P = 0; P < n_ptab; ++P) {
        int *B = blob.data() + (size_t)P * Lay::stride;
        const int r0 = pref_off[P], nr = pref_off[P + 1] - r0;
        const int v0 = pvtx_off[P], nvx = pvtx_off[P + 1] - v0;
        const int t0 = ptri_off[P], ntr = ptri_off[P + 1] - t0;
        const int e0 = pedge_off[P], ned = pedge_off[P + 1] - e0;
        B[Lay::hdr + 0] = nr; B[Lay::hdr + 1] = nvx; B[Lay::hdr + 2] = ntr; B[Lay::hdr + 3] = ned;
        uint8_t *vs = reinterpret_cast<uint8_t *>(B + Lay::vslot);
        uint8_t *ts = reinterpret_cast<uint8_t *>(B + Lay::tslot);
        uint8_t *es = reinterpret_cast<uint8_t *>(B + Lay::eslot);
        for (int k = 0; k < nr; ++k) B[Lay::pref + k] = pref[r0 + k];
        for (int k = 0; k < nvx; ++k) { B[Lay::pvtx + k] = pvtx[v0 + k]; vs[k] = pvtx_slot[v0 + k]; }
        for (int k = 0; k < ntr; ++k) {
          B[Lay::ptri + k] = ptri[t0 + k];
          for (int r = 0; r < 3; ++r) ts[3 * k + r] = ptri_slot[3 * (size_t)(t0 + k) + r];
        }
        for (int k = 0; k < ned; ++k) {
          B[Lay::pedge + k] = pedge[e0 + k];
          es[2 * k] = pedge_slot[2 * (size_t)(e0 + k)];
          es[2 * k + 1] = pedge_slot[2 * (size_t)(e0 + k) + 1];
        }
      }
      bs = Lay::stride;
      return upload(ctx->t_blob, blob);
    };
    hipError_t e = ctx->tile == 16 ? build_blobs(BlobLayout<16>{})
                   : ctx->tile == 32 ? build_blobs(BlobLayout<32>{})
                                     : build_blobs(BlobLayout<64>{});
    HIPCHK(e);
  }
  HIPCHK(upload(ctx->t_nv, nv));
  HIPCHK(upload(ctx->t_nt, ntv));
  HIPCHK(upload(ctx->t_ne, nev));
  HIPCHK(upload(ctx->t_tri_off, tri_off));
  HIPCHK(upload(ctx->t_edge_off, edge_off));
  HIPCHK(upload(ctx->t_tri, tri));
  HIPCHK(upload(ctx->t_edge, edge));
  HIPCHK(upload(ctx->t_patch_off, patch_off));
  HIPCHK(upload(ctx->t_ptri_off, ptri_off));
  HIPCHK(upload(ctx->t_ptri, ptri));
  HIPCHK(upload(ctx->t_ptri_slot, ptri_slot));
  HIPCHK(upload(ctx->t_pvtx_off, pvtx_off));
  HIPCHK(upload(ctx->t_pvtx, pvtx));
  HIPCHK(upload(ctx->t_pvtx_slot, pvtx_slot));
  HIPCHK(upload(ctx->t_pedge_off, pedge_off));
  HIPCHK(upload(ctx->t_pedge, pedge));
  HIPCHK(upload(ctx->t_pedge_slot, pedge_slot));
  HIPCHK(upload(ctx->t_pref_off, pref_off));
  HIPCHK(upload(ctx->t_pref, pref));
  HIPCHK(upload(ctx->t_vbase, vbase));
  HIPCHK(upload(ctx->t_vp_off, vp_off));
  HIPCHK(upload(ctx->t_vp, vp));
  HIPCHK(upload(ctx->t_vp4, vp4));
  HIPCHK(upload(ctx->t_tri_rec, tri_rec));
  DevTopo &D = ctx->topo;
  D.n_topo = nt_topo;
  D.nv = P<int>(ctx->t_nv); D.nt = P<int>(ctx->t_nt); D.ne = P<int>(ctx->t_ne);
  D.tri_off = P<int>(ctx->t_tri_off); D.edge_off = P<int>(ctx->t_edge_off);
  D.tri = P<int>(ctx->t_tri); D.edge = P<int>(ctx->t_edge);
  D.patch_off = P<int>(ctx->t_patch_off);
  D.ptri_off = P<int>(ctx->t_ptri_off); D.ptri = P<int>(ctx->t_ptri); D.ptri_slot = P<uint8_t>(ctx->t_ptri_slot);
  D.pvtx_off = P<int>(ctx->t_pvtx_off); D.pvtx = P<int>(ctx->t_pvtx); D.pvtx_slot = P<uint8_t>(ctx->t_pvtx_slot);
  D.pedge_off = P<int>(ctx->t_pedge_off); D.pedge = P<int>(ctx->t_pedge);
  D.pedge_slot = P<uint8_t>(ctx->t_pedge_slot);
  D.pref_off = P<int>(ctx->t_pref_off); D.pref = P<int>(ctx->t_pref);
  D.vbase = P<int>(ctx->t_vbase); D.vp_off = P<int>(ctx->t_vp_off); D.vp = P<int>(ctx->t_vp);
  D.vp4 = P<int4>(ctx->t_vp4);
  D.blob = P<int>(ctx->t_blob);
  D.blob_stride = bs;
  D.tri_rec = P<int4>(ctx->t_tri_rec);
  D.max_nv = max_nv;
  ctx->have_topo = true;
  return STIV_OK;
}

// ---------------------------------------------------------------------------
// Arena
// ---------------------------------------------------------------------------
static stiv_status arena(stiv_ctx *ctx, const stiv_scene *s) {
  const int64_t N = s->n_ves;
  const int64_t S = s->n_scenes;
  if (ctx->cap_cp == 0) ctx->cap_cp = std::max<int64_t>(64 * N, 4096);
  if (ctx->cap_pairs == 0) ctx->cap_pairs = std::max<int64_t>(16 * N, 4096);
  if (ctx->cap_work == 0) ctx->cap_work = std::max<int64_t>(64 * ctx->cap_pairs, 1 << 16);
  if (ctx->cap_cand == 0) ctx->cap_cand = std::max<int64_t>(4 * ctx->cap_work, 1 << 20);
  if (ctx->cap_ct == 0) ctx->cap_ct = std::max<int64_t>(ctx->cap_cand / 8, 1 << 18);
  ctx->cap_patch = N * std::max(ctx->max_patches, 1);
  if (ctx->cap_patch >= INT32_MAX) return fail(ctx, STIV_E_ARG, "detect: too many patches for 32-bit work records");
  const int64_t hash_cap = pow2_at_least(4 * ctx->cap_pairs);
  HIPCHK(ensure(ctx->counters, sizeof(Counters)));
  HIPCHK(ensure(ctx->ves_box, 6 * 8 * (N + 1)));
  HIPCHK(ensure(ctx->ves_scene, 4 * (N + 1)));
  HIPCHK(ensure(ctx->grid, sizeof(SceneGrid) * (S + 1)));
  HIPCHK(ensure(ctx->cp_cnt, 8 * (N + 1)));
  HIPCHK(ensure(ctx->cp_off, 8 * (N + 2)));
  HIPCHK(ensure(ctx->cp_keys, 8 * ctx->cap_cp));
  HIPCHK(ensure(ctx->cp_vals, 4 * ctx->cap_cp));
  HIPCHK(ensure(ctx->cp_tk, 8 * ctx->cap_cp));
  HIPCHK(ensure_sort_scratch(ctx, ctx->cap_cp));
  HIPCHK(ensure(ctx->scan_tmp, 8 * (size_t)scan_scratch_elems(std::max<int64_t>(N, ctx->cap_pairs))));
  HIPCHK(ensure(ctx->cp_tv, 4 * ctx->cap_cp));
  HIPCHK(ensure(ctx->hash, 8 * hash_cap));
  HIPCHK(ensure(ctx->uniq, 8 * ctx->cap_pairs));
  HIPCHK(ensure(ctx->sorted, 8 * ctx->cap_pairs));
  HIPCHK(ensure(ctx->cnt_a, 4 * (N + 1)));
  HIPCHK(ensure(ctx->cursor_a, 4 * (N + 1)));
  HIPCHK(ensure(ctx->off_a, 8 * (N + 2)));
  HIPCHK(ensure(ctx->pairs, sizeof(PairRec) * ctx->cap_pairs));
  HIPCHK(ensure(ctx->ves_patch_cnt, 8 * (N + 1)));
  HIPCHK(ensure(ctx->ves_patch_off, 8 * (N + 2)));
  HIPCHK(ensure(ctx->patch_box, 6 * 8 * (ctx->cap_patch + 1)));
  HIPCHK(ensure(ctx->patch_dop, kDopVals * 4 * (ctx->cap_patch + 1)));
  HIPCHK(ensure(ctx->work, sizeof(WorkRec) * ctx->cap_work));
  HIPCHK(ensure(ctx->cand, sizeof(Cand) * ctx->cap_cand));
  HIPCHK(ensure(ctx->hard_geo, 24 * sizeof(double) * ctx->cap_cand));
  HIPCHK(ensure(ctx->ct, sizeof(Cand) * ctx->cap_ct));
  HIPCHK(ensure(ctx->ct_s, 8 * ctx->cap_ct));
  HIPCHK(ensure(ctx->ct_vol, 8 * ctx->cap_ct));
  HIPCHK(ensure(ctx->ct_grad, 12 * 8 * ctx->cap_ct));
  HIPCHK(ensure(ctx->pair_cnt, 4 * (ctx->cap_pairs + 1)));
  HIPCHK(ensure(ctx->pair_cursor, 4 * (ctx->cap_pairs + 1)));
  HIPCHK(ensure(ctx->pair_off, 8 * (ctx->cap_pairs + 2)));
  HIPCHK(ensure(ctx->perm, 4 * ctx->cap_ct));
  HIPCHK(ensure(ctx->gkeys, 8 * 8 * ctx->cap_ct));
  HIPCHK(ensure(ctx->gidx, 4 * 8 * ctx->cap_ct));
  HIPCHK(ensure(ctx->pair_V, 8 * (ctx->cap_pairs + 1)));
  HIPCHK(ensure(ctx->pair_hasvt, 4 * (ctx->cap_pairs + 1)));
  HIPCHK(ensure(ctx->pair_rows, 4 * (ctx->cap_pairs + 1)));
  HIPCHK(ensure(ctx->vol_off, 8 * (ctx->cap_pairs + 2)));
  HIPCHK(ensure(ctx->row_off, 8 * (ctx->cap_pairs + 2)));
  HIPCHK(ensure(ctx->row_vtx, 4 * 4 * ctx->cap_ct));
  HIPCHK(ensure(ctx->row_g, 3 * 8 * 4 * ctx->cap_ct));
  ctx->arena_n_ves = std::max<int64_t>(ctx->arena_n_ves, N);
  ctx->arena_max_patches = ctx->max_patches;
  return STIV_OK;
}

static stiv_status check_args(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p) {
  if (!s || !p) return fail(ctx, STIV_E_ARG, "null scene or params");
  if (!ctx->have_topo) return fail(ctx, STIV_E_STATE, "stiv_set_topology has not been called");
  if (!(p->d >= 0.0) || !std::isfinite(p->d)) return fail(ctx, STIV_E_ARG, "d must be finite and >= 0");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(ctx, STIV_E_ARG, "eps must be finite and > 0");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(ctx, STIV_E_ARG, "dt must be finite and > 0");
  if (s->n_ves < 0 || s->n_vtx < 0 || s->n_scenes < 1) return fail(ctx, STIV_E_ARG, "bad scene sizes");
  if (s->n_ves >= (1 << 24)) return fail(ctx, STIV_E_ARG, "at most 2^24 - 1 vesicles");
  if (s->n_ves > 0 && (!s->vtx_off || !s->topo_id || !s->scene_off || !s->box_len || !s->x0 || !s->x1))
    return fail(ctx, STIV_E_ARG, "null scene array");
  if ((p->flags & STIV_LEARNED_BRACKET) && !ctx->have_model)
    return fail(ctx, STIV_E_STATE, "STIV_LEARNED_BRACKET needs a model (stiv_set_toi_model)");
  return STIV_OK;
}

// Validate the small structural arrays (device) on the host before any
// kernel indexes with them.  The result is cached per (pointers, sizes);
// stiv_reserve clears the cache, so callers that rewrite these arrays in
// place call stiv_reserve first.
static stiv_status check_structure(stiv_ctx *ctx, const stiv_scene *s) {
  const void *ptrs[4] = {s->vtx_off, s->topo_id, s->scene_off, s->box_len};
  const int64_t sizes[3] = {s->n_ves, s->n_vtx, s->n_scenes};
  if (std::memcmp(ptrs, ctx->val_ptr, sizeof ptrs) == 0 && std::memcmp(sizes, ctx->val_size, sizeof sizes) == 0)
    return STIV_OK;
  std::vector<int32_t> vo(s->n_ves + 1), tid(s->n_ves), so(s->n_scenes + 1);
  std::vector<double> bl(3 * (size_t)s->n_scenes);
  HIPCHK(hipMemcpy(vo.data(), s->vtx_off, vo.size() * 4, hipMemcpyDeviceToHost));
  if (s->n_ves) HIPCHK(hipMemcpy(tid.data(), s->topo_id, tid.size() * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(so.data(), s->scene_off, so.size() * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bl.data(), s->box_len, bl.size() * 8, hipMemcpyDeviceToHost));
  if (vo[0] != 0 || vo[s->n_ves] != s->n_vtx) return fail(ctx, STIV_E_ARG, "vtx_off must run from 0 to n_vtx");
  std::vector<int> nv_topo(ctx->topo.n_topo);
  {
    std::vector<int> tmp(ctx->topo.n_topo);
    HIPCHK(hipMemcpy(tmp.data(), ctx->topo.nv, tmp.size() * 4, hipMemcpyDeviceToHost));
    nv_topo = tmp;
  }
  for (int v = 0; v < s->n_ves; ++v) {
    if (tid[v] < 0 || tid[v] >= ctx->topo.n_topo) return fail(ctx, STIV_E_ARG, "topo_id out of range");
    if (vo[v + 1] - vo[v] != nv_topo[tid[v]])
      return fail(ctx, STIV_E_ARG, "vtx_off does not match the vertex count of the vesicle's topology");
  }
  if (so[0] != 0 || so[s->n_scenes] != s->n_ves) return fail(ctx, STIV_E_ARG, "scene_off must run from 0 to n_ves");
  for (int k = 0; k < s->n_scenes; ++k)
    if (so[k + 1] < so[k]) return fail(ctx, STIV_E_ARG, "scene_off must be non-decreasing");
  for (double L : bl)
    if (!(L >= 0.0) || !std::isfinite(L)) return fail(ctx, STIV_E_ARG, "box_len must be finite and >= 0");
  std::memcpy(ctx->val_ptr, ptrs, sizeof ptrs);
  std::memcpy(ctx->val_size, sizes, sizeof sizes);
  return STIV_OK;
}

stiv_status stiv_reserve(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p) {
  if (!ctx) return STIV_E_ARG;
  stiv_status st = check_args(ctx, s, p);
  if (st != STIV_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  for (auto &q : ctx->val_ptr) q = nullptr;
  st = check_structure(ctx, s);
  if (st != STIV_OK) return st;
  return arena(ctx, s);
}

constexpr int kSupportGrid = 384;         // workgroups of the supports beside the broad phase
constexpr int64_t kSplitMaxVesicles = 4096;  // larger scenes: supports inside the box kernel

static void run_pipeline(stiv_ctx *ctx, const DevScene &S, const stiv_params *p, stiv_result *out, hipStream_t st,
                         bool timed) {
  const double h = 0.5 * p->d;
  const int64_t N = S.n_ves;
  Counters *cnt = P<Counters>(ctx->counters);
  const DevTopo &T = ctx->topo;
  const int64_t hash_cap = pow2_at_least(4 * ctx->cap_pairs);
  if (timed) (void)hipEventRecord(ctx->ev[8], st);
  {
    // every buffer this call clears, in one launch
    FillJobs J;
    J.add(cnt, 0ull, (int64_t)(sizeof(Counters) / 8), 8);
    J.add(P<uint64_t>(ctx->hash), ~0ull, hash_cap, 8);
    J.add(P<int32_t>(ctx->cnt_a), 0ull, N + 1, 4);
    J.add(P<int32_t>(ctx->cursor_a), 0ull, N + 1, 4);
    J.add(P<int32_t>(ctx->pair_cnt), 0ull, ctx->cap_pairs + 1, 4);
    J.add(P<int32_t>(ctx->pair_cursor), 0ull, ctx->cap_pairs + 1, 4);
    launch_fill_multi(J, st);
  }
  if (!launch_ves_tables(S, T, P<int64_t>(ctx->ves_patch_cnt), P<int>(ctx->ves_scene), P<int64_t>(ctx->ves_patch_off),
                         st))
    launch_scan_i64(P<int64_t>(ctx->ves_patch_cnt), P<int64_t>(ctx->ves_patch_off), nullptr, N, P<int64_t>(ctx->scan_tmp),
                    st);
  // ---- K0 boxes.  The patches' face-diagonal supports need only the
  // positions: up to kSplitMaxVesicles vesicles they run on the side stream
  // after the boxes, beside the vesicle broad phase (latency-bound, it leaves
  // most compute units idle), on a grid of a few workgroups per compute unit,
  // and are joined before the patch pairs; larger scenes compute them in the
  // box kernel (their supports would outlast the broad phase).
  const bool has_sup = boxes_have_supports(T, ctx->max_patches);
  const bool supports = has_sup && N <= kSplitMaxVesicles;
  if (timed) (void)hipEventRecord(ctx->ev[0], st);
  launch_boxes(S, T, h, P<int64_t>(ctx->ves_patch_off), P<double>(ctx->ves_box), P<double>(ctx->patch_box),
               P<float>(ctx->patch_dop), ctx->max_patches,
               supports ? kBoxParts : (has_sup ? (kBoxParts | kSupportParts) : (kBoxParts | kNoSupportParts)), 8192,
               cnt, st);
  if (supports) {
    (void)hipEventRecord(ctx->fork, st);
    (void)hipStreamWaitEvent(ctx->side, ctx->fork, 0);
    launch_boxes(S, T, h, P<int64_t>(ctx->ves_patch_off), P<double>(ctx->ves_box), P<double>(ctx->patch_box),
                 P<float>(ctx->patch_dop), ctx->max_patches, kSupportParts, kSupportGrid, cnt, ctx->side);
    (void)hipEventRecord(ctx->join, ctx->side);
  }
  if (timed) (void)hipEventRecord(ctx->ev[1], st);
  // ---- K1 vesicle broad phase
  launch_scene_grid(S, P<double>(ctx->ves_box), P<SceneGrid>(ctx->grid), P<int64_t>(ctx->cp_cnt),
                    P<int64_t>(ctx->cp_off), st);
  if (S.n_scenes != 1)
    launch_scan_i64(P<int64_t>(ctx->cp_cnt), P<int64_t>(ctx->cp_off), nullptr, N, P<int64_t>(ctx->scan_tmp), st);
  launch_cp_emit(S, P<double>(ctx->ves_box), P<int>(ctx->ves_scene), P<SceneGrid>(ctx->grid),
                 P<int64_t>(ctx->cp_off), P<uint64_t>(ctx->cp_keys), P<uint32_t>(ctx->cp_vals), ctx->cap_cp, cnt, st);
  const unsigned long long *n_cp = reinterpret_cast<const unsigned long long *>(P<int64_t>(ctx->cp_off) + N);
  int scene_bits = 0;
  while ((1ll << scene_bits) < S.n_scenes) ++scene_bits;
  launch_radix_sort_u64(P<uint64_t>(ctx->cp_keys), P<uint32_t>(ctx->cp_vals), P<uint64_t>(ctx->cp_tk),
                        P<uint32_t>(ctx->cp_tv), n_cp, ctx->cap_cp, 30 + scene_bits, P<int32_t>(ctx->rs_hist),
                        P<int64_t>(ctx->rs_off), st, cnt->cp_key_bits);
  launch_cell_pairs(S, P<double>(ctx->ves_box), P<int>(ctx->ves_scene), P<uint64_t>(ctx->cp_keys),
                    P<uint32_t>(ctx->cp_vals), n_cp, ctx->cap_cp, P<uint64_t>(ctx->hash), hash_cap, cnt, st);
  launch_hash_list(P<uint64_t>(ctx->hash), hash_cap, P<uint64_t>(ctx->uniq), ctx->cap_pairs, P<int32_t>(ctx->cnt_a),
                   cnt, st);
  launch_scan_i32_to_i64(P<int32_t>(ctx->cnt_a), P<int64_t>(ctx->off_a), nullptr, N, P<int64_t>(ctx->scan_tmp), st);
  launch_pair_bucket_scatter(P<uint64_t>(ctx->uniq), ctx->cap_pairs, P<int64_t>(ctx->off_a),
                             P<int32_t>(ctx->cursor_a), P<uint64_t>(ctx->sorted), cnt, st);
  launch_pair_bucket_sort_emit(S, P<int>(ctx->ves_scene), P<int64_t>(ctx->off_a), P<uint64_t>(ctx->sorted), (int)N,
                               P<PairRec>(ctx->pairs), out->pair_ab, out->pair_shift, out->cap_pairs, st);
  if (timed) (void)hipEventRecord(ctx->ev[2], st);
  // ---- K2 primitive broad phase (after the supports)
  if (supports) (void)hipStreamWaitEvent(st, ctx->join, 0);
  launch_patch_pairs(S, T, P<PairRec>(ctx->pairs), ctx->cap_pairs, P<double>(ctx->ves_box),
                     P<int64_t>(ctx->ves_patch_off), P<double>(ctx->patch_box), P<float>(ctx->patch_dop),
                     P<WorkRec>(ctx->work), ctx->cap_work, ctx->max_patches, cnt, st);
  if (timed) (void)hipEventRecord(ctx->ev[3], st);
  const bool emit = (p->flags & STIV_EMIT_CANDIDATES) != 0;
  launch_prim_cand(ctx->tile, ctx->prim_blocks, S, T, P<PairRec>(ctx->pairs), P<WorkRec>(ctx->work),
                   ctx->cap_work, P<double>(ctx->patch_box), p->d, P<Cand>(ctx->cand), P<double>(ctx->hard_geo), ctx->cap_cand, emit ? P<Cand>(ctx->cand_list) : nullptr,
                   emit ? ctx->cap_list : 0, cnt, st);
  if (timed) (void)hipEventRecord(ctx->ev[4], st);
  // ---- K3 + K4 root search, volumes and gradients
  launch_narrow(ctx->narrow_blocks, S, T, P<PairRec>(ctx->pairs), P<Cand>(ctx->cand), P<double>(ctx->hard_geo),
                ctx->cap_cand, p->d, p->eps,
                p->dt,
                P<Cand>(ctx->ct), P<double>(ctx->ct_s), P<double>(ctx->ct_vol), P<double>(ctx->ct_grad), ctx->cap_ct,
                P<int32_t>(ctx->pair_cnt), (p->flags & STIV_LEARNED_BRACKET) ? ctx->toi_packed.p : nullptr,
                ctx->toi_kwidth, cnt, st);
  if (timed) (void)hipEventRecord(ctx->ev[5], st);
  // ---- K5 aggregation
  // (the root search counted the contacts of each pair into pair_cnt)
  const unsigned long long *n_pairs_dev = &cnt->n_pairs;
  launch_scan_i32_to_i64(P<int32_t>(ctx->pair_cnt), P<int64_t>(ctx->pair_off), n_pairs_dev, ctx->cap_pairs, P<int64_t>(ctx->scan_tmp), st);
  // the per-pair counts are consumed by the scan: their buffer holds the list of pairs with contacts
  launch_ct_scatter_order(P<Cand>(ctx->ct), ctx->cap_ct, cnt, P<int64_t>(ctx->pair_off), P<int32_t>(ctx->pair_cursor),
                          P<int32_t>(ctx->perm), ctx->cap_pairs, P<int32_t>(ctx->pair_cnt), P<double>(ctx->pair_V),
                          P<int32_t>(ctx->pair_hasvt), P<int32_t>(ctx->pair_rows), st);
  launch_ct_sort_aggregate(S, T, P<PairRec>(ctx->pairs), ctx->cap_pairs, cnt, P<int32_t>(ctx->pair_cnt),
                           P<int64_t>(ctx->pair_off),
                           P<int32_t>(ctx->perm), P<Cand>(ctx->ct), P<double>(ctx->ct_s), P<double>(ctx->ct_vol),
                           P<double>(ctx->ct_grad), p->dt, P<uint64_t>(ctx->gkeys), P<int32_t>(ctx->gidx),
                           out->ct_key, out->ct_tau, out->ct_s, out->ct_vol, out->ct_grad, out->cap_ct, P<double>(ctx->pair_V),
                           P<int32_t>(ctx->pair_hasvt), P<int32_t>(ctx->pair_rows), P<int32_t>(ctx->row_vtx),
                           P<double>(ctx->row_g), st);
  launch_scan2_i32_to_i64(P<int32_t>(ctx->pair_hasvt), P<int64_t>(ctx->vol_off), P<int32_t>(ctx->pair_rows),
                          P<int64_t>(ctx->row_off), n_pairs_dev, ctx->cap_pairs, P<int64_t>(ctx->scan_tmp), st);
  launch_write_volumes(cnt, ctx->cap_pairs, P<int64_t>(ctx->pair_off), P<int64_t>(ctx->vol_off),
                       P<int64_t>(ctx->row_off), P<int32_t>(ctx->pair_hasvt), P<double>(ctx->pair_V),
                       P<int32_t>(ctx->pair_rows), P<int32_t>(ctx->row_vtx), P<double>(ctx->row_g), out->vol_pair,
                       out->vol_V, out->cap_vol, out->j_vol, out->j_vtx, out->j_g, out->cap_jrow,
                       P<int64_t>(ctx->cp_off) + N, st);
  if (timed) (void)hipEventRecord(ctx->ev[6], st);
}

// Counts of the last pipeline run into *out; STIV_E_CAPACITY when an internal
// buffer or a caller array was too small.
static stiv_status read_counts(stiv_ctx *ctx, const stiv_params *p, stiv_result *out, bool *internal_overflow) {
  const Counters &c = *ctx->h_cnt;
  *internal_overflow = (int64_t)c.n_cp > ctx->cap_cp || (int64_t)c.n_pairs > ctx->cap_pairs || c.hash_overflow ||
                       (int64_t)c.n_work > ctx->cap_work || (int64_t)hard_total(c.n_hard_vt_ee) > ctx->cap_cand ||
                       (int64_t)c.n_ct > ctx->cap_ct ||
                       ((p->flags & STIV_EMIT_CANDIDATES) && (int64_t)c.n_cand_list > ctx->cap_list);
  if (c.nonfinite) return fail(ctx, STIV_E_NUMERIC, "a position is NaN or infinite");
  if (c.shift_overflow) return fail(ctx, STIV_E_ARG, "periodic box too small: image shifts beyond +-7 box lengths");
  out->n_pairs = (int64_t)c.n_pairs;
  out->n_cand_vt = (int64_t)c.n_cand_vt;
  out->n_cand_ee = (int64_t)c.n_cand_ee;
  out->n_ct_vt = (int64_t)c.n_ct_vt;
  out->n_ct_ee = (int64_t)c.n_ct_ee;
  out->n_vol = (int64_t)c.n_vol;
  out->n_jrow = (int64_t)c.n_jrow;
  out->n_initially_within_d = (int64_t)c.within_d;
  out->n_degenerate_skipped = (int64_t)c.degenerate;
  out->n_search_exhausted = (int64_t)c.search_exhausted;
  return STIV_OK;
}

// A root search that ran out of its budget may have missed contacts: the
// outputs are written, but the call reports it.
static stiv_status check_exhausted(stiv_ctx *ctx, const stiv_result *out) {
  if (out->n_search_exhausted > 0)
    return fail(ctx, STIV_E_NUMERIC,
                std::to_string(out->n_search_exhausted) +
                    " root search(es) exhausted their interval budget; contacts of those candidates may be missing");
  return STIV_OK;
}

stiv_status stiv_detect(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, stiv_result *out, void *stream) {
  if (!ctx) return STIV_E_ARG;
  if (!out) return fail(ctx, STIV_E_ARG, "null result");
  stiv_status st0 = check_args(ctx, s, p);
  if (st0 != STIV_OK) return st0;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (s->n_ves == 0) {
    out->n_pairs = out->n_cand_vt = out->n_cand_ee = out->n_ct_vt = out->n_ct_ee = out->n_vol = out->n_jrow = 0;
    out->n_initially_within_d = out->n_degenerate_skipped = out->n_search_exhausted = 0;
    return STIV_OK;
  }
  stiv_status sv = check_structure(ctx, s);
  if (sv != STIV_OK) return sv;
  DevScene S;
  S.n_ves = s->n_ves; S.n_vtx = s->n_vtx; S.n_scenes = s->n_scenes;
  S.vtx_off = s->vtx_off; S.topo_id = s->topo_id; S.scene_off = s->scene_off;
  S.box_len = s->box_len; S.x0 = s->x0; S.x1 = s->x1;
  for (int attempt = 0; attempt < 4; ++attempt) {
    stiv_status sa = arena(ctx, s);
    if (sa != STIV_OK) return sa;
    if (p->flags & STIV_EMIT_CANDIDATES) {
      if (ctx->cap_list == 0) ctx->cap_list = 4 * ctx->cap_cand;
      HIPCHK(ensure(ctx->cand_list, sizeof(Cand) * ctx->cap_list));
    }
    run_pipeline(ctx, S, p, out, st, true);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->h_cnt, ctx->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const Counters &c = *ctx->h_cnt;
    bool grow = false;
    if (c.nonfinite) return fail(ctx, STIV_E_NUMERIC, "a position is NaN or infinite");
    if (c.shift_overflow)
      return fail(ctx, STIV_E_ARG, "periodic box too small: image shifts beyond +-7 box lengths");
    const int64_t need_cp = (int64_t)c.n_cp;
    if (need_cp > ctx->cap_cp) { ctx->cap_cp = need_cp + need_cp / 4; grow = true; }
    if ((int64_t)c.n_pairs > ctx->cap_pairs || c.hash_overflow) {
      ctx->cap_pairs = (int64_t)c.n_pairs * 2 + 1024;
      grow = true;
    }
    if ((int64_t)c.n_work > ctx->cap_work) { ctx->cap_work = (int64_t)c.n_work + c.n_work / 4 + 1024; grow = true; }
    if ((int64_t)hard_total(c.n_hard_vt_ee) > ctx->cap_cand) {
      const int64_t nh = (int64_t)hard_total(c.n_hard_vt_ee);
      ctx->cap_cand = nh + nh / 4 + 1024;
      grow = true;
    }
    if ((p->flags & STIV_EMIT_CANDIDATES) && (int64_t)c.n_cand_list > ctx->cap_list) {
      ctx->cap_list = (int64_t)c.n_cand_list + c.n_cand_list / 4 + 1024;
      grow = true;
    }
    if ((int64_t)c.n_ct > ctx->cap_ct) { ctx->cap_ct = (int64_t)c.n_ct + c.n_ct / 4 + 1024; grow = true; }
    if (grow) continue;
    bool internal = false;
    stiv_status sr = read_counts(ctx, p, out, &internal);
    if (sr != STIV_OK) return sr;
    float ms[8] = {};
    for (int k = 0; k < 6; ++k) (void)hipEventElapsedTime(&ms[k], ctx->ev[k], ctx->ev[k + 1]);
    (void)hipEventElapsedTime(&ms[6], ctx->ev[8], ctx->ev[6]);
    std::memcpy(ctx->stage_ms, ms, sizeof ms);
    const int64_t n_cand = out->n_cand_vt + out->n_cand_ee;
    if ((p->flags & STIV_EMIT_CANDIDATES) && out->cand) {
      const int64_t n = std::min(n_cand, out->cap_cand);
      if (n > 0) {
        HIPCHK(hipMemcpyAsync(out->cand, ctx->cand_list.p, (size_t)n * sizeof(Cand), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
      }
    }
    const bool over = out->n_pairs > out->cap_pairs || out->n_ct_vt + out->n_ct_ee > out->cap_ct ||
                      out->n_vol > out->cap_vol || out->n_jrow > out->cap_jrow ||
                      ((p->flags & STIV_EMIT_CANDIDATES) && n_cand > out->cap_cand);
    if (over) return fail(ctx, STIV_E_CAPACITY, "an output array is too small; n_* hold the required sizes");
    return check_exhausted(ctx, out);
  }
  return fail(ctx, STIV_E_CAPACITY, "internal buffers did not converge after growing");
}

stiv_status stiv_detect_async(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, stiv_result *out,
                              void *stream) {
  if (!ctx) return STIV_E_ARG;
  if (!out) return fail(ctx, STIV_E_ARG, "null result");
  stiv_status st0 = check_args(ctx, s, p);
  if (st0 != STIV_OK) return st0;
  if (p->flags & STIV_EMIT_CANDIDATES) return fail(ctx, STIV_E_ARG, "candidate lists need the synchronous stiv_detect");
  const void *ptrs[4] = {s->vtx_off, s->topo_id, s->scene_off, s->box_len};
  const int64_t sizes[3] = {s->n_ves, s->n_vtx, s->n_scenes};
  if (std::memcmp(ptrs, ctx->val_ptr, sizeof ptrs) != 0 || std::memcmp(sizes, ctx->val_size, sizeof sizes) != 0)
    return fail(ctx, STIV_E_STATE, "stiv_detect_async needs a prior stiv_detect or stiv_reserve on this scene");
  if (ctx->cap_cp == 0 || !ctx->counters.p || ctx->arena_n_ves < s->n_ves ||
      ctx->arena_max_patches < ctx->max_patches)
    return fail(ctx, STIV_E_STATE, "the arena is not sized: call stiv_detect once first");
  if (s->n_ves == 0) return STIV_OK;
  DevScene S;
  S.n_ves = s->n_ves; S.n_vtx = s->n_vtx; S.n_scenes = s->n_scenes;
  S.vtx_off = s->vtx_off; S.topo_id = s->topo_id; S.scene_off = s->scene_off;
  S.box_len = s->box_len; S.x0 = s->x0; S.x1 = s->x1;
  run_pipeline(ctx, S, p, out, reinterpret_cast<hipStream_t>(stream), false);
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

stiv_status stiv_collect(stiv_ctx *ctx, const stiv_params *p, stiv_result *out, void *stream) {
  if (!ctx || !p || !out) return STIV_E_ARG;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(ctx->h_cnt, ctx->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool internal = false;
  stiv_status sr = read_counts(ctx, p, out, &internal);
  if (sr != STIV_OK) return sr;
  if (internal)
    return fail(ctx, STIV_E_CAPACITY, "internal buffers overflowed: run stiv_detect to grow them, then capture again");
  const bool over = out->n_pairs > out->cap_pairs || out->n_ct_vt + out->n_ct_ee > out->cap_ct ||
                    out->n_vol > out->cap_vol || out->n_jrow > out->cap_jrow;
  if (over) return fail(ctx, STIV_E_CAPACITY, "an output array is too small; n_* hold the required sizes");
  return check_exhausted(ctx, out);
}

stiv_status stiv_set_patch_size(stiv_ctx *ctx, int tri_per_patch);

stiv_status stiv_set_option(stiv_ctx *ctx, int option, int64_t value) {
  if (!ctx) return STIV_E_ARG;
  switch (option) {
    case STIV_OPT_PATCH_TRI:
      return stiv_set_patch_size(ctx, (int)value);
    case STIV_OPT_PRIM_BLOCKS:
      if (value < 256 || value > 65536) return fail(ctx, STIV_E_ARG, "prim blocks out of range [256, 65536]");
      ctx->prim_blocks = (int)value;
      return STIV_OK;
    case STIV_OPT_NARROW_BLOCKS:
      if (value < 256 || value > 65536) return fail(ctx, STIV_E_ARG, "narrow blocks out of range [256, 65536]");
      ctx->narrow_blocks = (int)value;
      return STIV_OK;
    case STIV_OPT_QUEUE_CAPACITY:
      if (value < 64 || value > (int64_t)INT32_MAX)
        return fail(ctx, STIV_E_ARG, "queue capacity out of range [64, 2^31)");
      ctx->cap_cand = value;  // the buffers only grow: a smaller capacity uses part of them
      return STIV_OK;
    default:
      return fail(ctx, STIV_E_ARG, "unknown option");
  }
}

stiv_status stiv_get_stage_times(stiv_ctx *ctx, float *ms, int n) {
  if (!ctx || !ms) return STIV_E_ARG;
  for (int k = 0; k < n && k < 7; ++k) ms[k] = ctx->stage_ms[k];
  return STIV_OK;
}

static stiv_status check_backward_args(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p,
                                       const stiv_result *res) {
  if (!res) return fail(ctx, STIV_E_ARG, "null result");
  stiv_status st0 = check_args(ctx, s, p);
  if (st0 != STIV_OK) return st0;
  const int64_t n_ct = res->n_ct_vt + res->n_ct_ee;
  if (res->n_pairs > res->cap_pairs || n_ct > res->cap_ct || res->n_vol > res->cap_vol || res->n_jrow > res->cap_jrow)
    return fail(ctx, STIV_E_ARG, "backward needs a complete detect result (no capacity overflow)");
  if (n_ct > 0 && (!res->ct_key || !res->ct_tau || !res->pair_ab || !res->pair_shift))
    return fail(ctx, STIV_E_ARG, "backward needs the contact and pair arrays of the detect result");
  if (res->n_vol > 0 && (!res->vol_pair || !res->j_vol || !res->j_vtx))
    return fail(ctx, STIV_E_ARG, "backward needs the volume and Jacobian arrays of the detect result");
  return STIV_OK;
}

static DevScene dev_scene(const stiv_scene *s) {
  DevScene S;
  S.n_ves = s->n_ves; S.n_vtx = s->n_vtx; S.n_scenes = s->n_scenes;
  S.vtx_off = s->vtx_off; S.topo_id = s->topo_id; S.scene_off = s->scene_off;
  S.box_len = s->box_len; S.x0 = s->x0; S.x1 = s->x1;
  return S;
}

// The backward kernels on scratch at `base` (layout L).
static void run_backward(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, const stiv_result *res,
                         const double *dL_dV, const double *dL_dG, double *dL_dX0, double *dL_dX1, char *base,
                         const BwdLayout &L, hipStream_t st) {
  const int64_t n_ct = res->n_ct_vt + res->n_ct_ee;
  launch_backward(dev_scene(s), ctx->topo, p->d, p->eps, p->dt, n_ct, res->ct_key, res->ct_tau, res->pair_ab,
                  res->pair_shift, res->n_vol, res->vol_pair, res->n_jrow, res->j_vol, res->j_vtx, dL_dV, dL_dG,
                  res->ct_s, reinterpret_cast<double *>(base + L.contrib), reinterpret_cast<uint64_t *>(base + L.gkeys),
                  reinterpret_cast<int32_t *>(base + L.gidx), reinterpret_cast<double *>(base + L.rowc),
                  reinterpret_cast<uint64_t *>(base + L.rkey), reinterpret_cast<uint32_t *>(base + L.rval),
                  reinterpret_cast<uint64_t *>(base + L.tk), reinterpret_cast<uint32_t *>(base + L.tv),
                  reinterpret_cast<int32_t *>(base + L.hist), reinterpret_cast<int64_t *>(base + L.hoff), dL_dX0,
                  dL_dX1, st);
}

stiv_status stiv_backward(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, const stiv_result *res,
                          const double *dL_dV, const double *dL_dG, double *dL_dX0, double *dL_dX1, void *stream) {
  if (!ctx) return STIV_E_ARG;
  stiv_status sa = check_backward_args(ctx, s, p, res);
  if (sa != STIV_OK) return sa;
  HIPCHK(hipSetDevice(ctx->device));
  stiv_status sv = check_structure(ctx, s);
  if (sv != STIV_OK) return sv;
  const BwdLayout L = backward_layout(res->n_ct_vt + res->n_ct_ee, res->n_jrow);
  HIPCHK(ensure(ctx->bwd_scratch, L.total));
  run_backward(ctx, s, p, res, dL_dV, dL_dG, dL_dX0, dL_dX1, P<char>(ctx->bwd_scratch), L,
               reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

stiv_status stiv_backward_static(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, const stiv_result *res,
                                 const double *dL_dV, const double *dL_dG, double *dL_dX0, double *dL_dX1,
                                 void *stream) {
  if (!ctx) return STIV_E_ARG;
  stiv_status sa = check_backward_args(ctx, s, p, res);
  if (sa != STIV_OK) return sa;
  // no host copies here: the scene's structural arrays must be the ones a
  // previous stiv_detect (or stiv_reserve) on this context validated
  const void *ptrs[4] = {s->vtx_off, s->topo_id, s->scene_off, s->box_len};
  const int64_t sizes[3] = {s->n_ves, s->n_vtx, s->n_scenes};
  if (std::memcmp(ptrs, ctx->val_ptr, sizeof ptrs) != 0 || std::memcmp(sizes, ctx->val_size, sizeof sizes) != 0)
    return fail(ctx, STIV_E_STATE, "stiv_backward_static needs a prior stiv_detect or stiv_reserve on this scene");
  const BwdLayout L = backward_layout(res->n_ct_vt + res->n_ct_ee, res->n_jrow);
  if (L.total > backward_static_bytes())
    return fail(ctx, STIV_E_CAPACITY,
                "stiv_backward_static: " + std::to_string(res->n_ct_vt + res->n_ct_ee) + " contacts and " +
                    std::to_string(res->n_jrow) + " Jacobian rows need " + std::to_string(L.total) +
                    " bytes of scratch, more than its static " + std::to_string(backward_static_bytes()) +
                    " (use stiv_backward)");
  HIPCHK(hipSetDevice(ctx->device));
  void *base = nullptr;
  HIPCHK(backward_static_scratch(ctx->device, &base));
  run_backward(ctx, s, p, res, dL_dV, dL_dG, dL_dX0, dL_dX1, static_cast<char *>(base), L,
               reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

stiv_status stiv_set_patch_size(stiv_ctx *ctx, int tri_per_patch) {
  if (!ctx) return STIV_E_ARG;
  if (tri_per_patch != 16 && tri_per_patch != 32 && tri_per_patch != 64)
    return fail(ctx, STIV_E_ARG, "patch size must be 16, 32 or 64 triangles");
  if (ctx->tile != tri_per_patch) {
    ctx->tile = tri_per_patch;
    ctx->have_topo = false;  // the tiling depends on the patch size: set the topology again
  }
  return STIV_OK;
}

stiv_status stiv_get_stats(stiv_ctx *ctx, int64_t *vals, int n) {
  if (!ctx || !vals) return STIV_E_ARG;
  const Counters &c = *ctx->h_cnt;
  const int64_t v[10] = {(int64_t)c.n_cp,      (int64_t)c.n_pairs,   (int64_t)c.n_work,
                         (int64_t)c.n_pre,     (int64_t)c.n_cand_vt, (int64_t)c.n_cand_ee,
                         (int64_t)hard_total(c.n_hard_vt_ee), (int64_t)c.n_ct,      (int64_t)c.n_tests,
                         (int64_t)c.n_bracket_ok};
  for (int k = 0; k < n && k < 10; ++k) vals[k] = v[k];
  return STIV_OK;
}

stiv_status stiv_sort_pairs_u64(stiv_ctx *ctx, uint64_t *keys, uint32_t *vals, int64_t n, void *stream) {
  if (!ctx || n < 0 || (n > 0 && (!keys || !vals))) return fail(ctx, STIV_E_ARG, "bad sort arguments");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(ensure(ctx->sort_tk, 8 * (size_t)(n + 1)));
  HIPCHK(ensure(ctx->sort_tv, 4 * (size_t)(n + 1)));
  HIPCHK(ensure_sort_scratch(ctx, n));
  launch_radix_sort_u64(keys, vals, P<uint64_t>(ctx->sort_tk), P<uint32_t>(ctx->sort_tv), nullptr, n, 64,
                        P<int32_t>(ctx->rs_hist), P<int64_t>(ctx->rs_off), st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return STIV_OK;
}

static stiv_status check_lcp_args(stiv_ctx *ctx, const stiv_scene *s, const stiv_result *res) {
  if (!ctx) return STIV_E_ARG;
  if (!s || !res) return fail(ctx, STIV_E_ARG, "null scene or result");
  if (s->n_ves < 0 || s->n_vtx < 0 || (s->n_ves > 0 && !s->vtx_off)) return fail(ctx, STIV_E_ARG, "bad scene");
  if (res->n_vol < 0 || res->n_jrow < 0 || res->n_vol > res->cap_vol || res->n_jrow > res->cap_jrow ||
      res->n_pairs > res->cap_pairs)
    return fail(ctx, STIV_E_ARG, "result counts exceed its capacities (not a complete stiv_detect result)");
  if (res->n_jrow > 0 && (!res->j_vol || !res->j_vtx || !res->j_g))
    return fail(ctx, STIV_E_ARG, "null Jacobian arrays");
  if (res->n_vol > 0 && (!res->vol_pair || !res->pair_ab)) return fail(ctx, STIV_E_ARG, "null volume arrays");
  if (res->n_vol >= (1ll << 31)) return fail(ctx, STIV_E_ARG, "too many volumes");
  return STIV_OK;
}

stiv_status stiv_lcp_layout(stiv_ctx *ctx, const stiv_scene *s, const stiv_result *res, int64_t *act_off,
                            int64_t *m_off, int32_t *act_vtx, int64_t cap_act, int64_t *n_act, int64_t *n_m,
                            void *stream) {
  stiv_status stc = check_lcp_args(ctx, s, res);
  if (stc != STIV_OK) return stc;
  if (!act_off || !m_off || !n_act || !n_m || cap_act < 0 || (cap_act > 0 && !act_vtx))
    return fail(ctx, STIV_E_ARG, "bad layout outputs");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nv = s->n_ves;
  HIPCHK(ensure(ctx->lcp_flag, 4 * (size_t)(s->n_vtx + 1)));
  HIPCHK(ensure(ctx->lcp_a, 4 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_m9, 8 * (size_t)(nv + 1)));
  launch_fill_i32(P<int32_t>(ctx->lcp_flag), 0, s->n_vtx + 1, st);
  launch_lcp_layout(s->vtx_off, nv, res->j_vtx, res->n_jrow, P<int32_t>(ctx->lcp_flag), P<int32_t>(ctx->lcp_a),
                    P<int64_t>(ctx->lcp_m9), st);
  launch_scan_i32_to_i64(P<int32_t>(ctx->lcp_a), act_off, nullptr, nv, nullptr, st);
  launch_scan_i64(P<int64_t>(ctx->lcp_m9), m_off, nullptr, nv, nullptr, st);
  HIPCHK(hipGetLastError());
  int64_t tot[2];
  HIPCHK(hipMemcpyAsync(&tot[0], act_off + nv, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&tot[1], m_off + nv, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *n_act = tot[0];
  *n_m = tot[1];
  if (tot[0] > cap_act) return fail(ctx, STIV_E_CAPACITY, "act_vtx capacity too small");
  launch_lcp_emit(s->vtx_off, nv, P<int32_t>(ctx->lcp_flag), act_off, act_vtx, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return STIV_OK;
}

stiv_status stiv_form_lcp(stiv_ctx *ctx, const stiv_scene *s, const stiv_result *res, const int64_t *act_off,
                          const int64_t *m_off, const int32_t *act_vtx, const double *M, int32_t *b_row,
                          int32_t *b_col, double *b_val, int64_t cap_b, int64_t *n_b, void *stream) {
  stiv_status stc = check_lcp_args(ctx, s, res);
  if (stc != STIV_OK) return stc;
  if (!act_off || !m_off || !n_b || cap_b < 0 || (cap_b > 0 && (!b_row || !b_col || !b_val)))
    return fail(ctx, STIV_E_ARG, "bad LCP outputs");
  if (res->n_jrow > 0 && (!act_vtx || !M)) return fail(ctx, STIV_E_ARG, "null active list or operator blocks");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nv = s->n_ves;
  const int64_t n_vol = res->n_vol;
  HIPCHK(ensure(ctx->lcp_vcnt, 4 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_vcur, 4 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_voff, 8 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_c2, 8 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_coff, 8 * (size_t)(nv + 1)));
  HIPCHK(ensure(ctx->lcp_vlist, 4 * (size_t)(2 * n_vol + 1)));
  HIPCHK(ensure(ctx->lcp_ovf, 8));
  launch_fill_i32(P<int32_t>(ctx->lcp_vcnt), 0, nv + 1, st);
  launch_fill_i32(P<int32_t>(ctx->lcp_vcur), 0, nv + 1, st);
  launch_fill_u64(P<uint64_t>(ctx->lcp_ovf), 0ull, 1, st);
  launch_lcp_vcount(res->vol_pair, res->pair_ab, n_vol, P<int32_t>(ctx->lcp_vcnt), st);
  launch_scan_i32_to_i64(P<int32_t>(ctx->lcp_vcnt), P<int64_t>(ctx->lcp_voff), nullptr, nv, nullptr, st);
  launch_lcp_vscatter(res->vol_pair, res->pair_ab, n_vol, P<int64_t>(ctx->lcp_voff), P<int32_t>(ctx->lcp_vcur),
                      P<int32_t>(ctx->lcp_vlist), nv, P<int64_t>(ctx->lcp_c2), st);
  launch_scan_i64(P<int64_t>(ctx->lcp_c2), P<int64_t>(ctx->lcp_coff), nullptr, nv, nullptr, st);
  HIPCHK(hipGetLastError());
  int64_t nc = 0;
  HIPCHK(hipMemcpyAsync(&nc, P<int64_t>(ctx->lcp_coff) + nv, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (nc >= (1ll << 32)) return fail(ctx, STIV_E_CAPACITY, "too many LCP contributions");
  HIPCHK(ensure(ctx->lcp_ckey, 8 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_cval, 8 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_cidx, 4 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_tk, 8 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_tv, 4 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_start, 4 * (size_t)(nc + 1)));
  HIPCHK(ensure(ctx->lcp_pos, 8 * (size_t)(nc + 1)));
  launch_lcp_block(s->vtx_off, nv, act_off, m_off, act_vtx, M, P<int64_t>(ctx->lcp_voff), P<int32_t>(ctx->lcp_vlist),
                   res->j_vol, res->j_vtx, res->j_g, res->n_jrow, P<int64_t>(ctx->lcp_coff),
                   P<uint64_t>(ctx->lcp_ckey), P<double>(ctx->lcp_cval), P<unsigned long long>(ctx->lcp_ovf), st);
  launch_iota_u32(P<uint32_t>(ctx->lcp_cidx), nc, st);
  HIPCHK(ensure_sort_scratch(ctx, nc));
  launch_radix_sort_u64(P<uint64_t>(ctx->lcp_ckey), P<uint32_t>(ctx->lcp_cidx), P<uint64_t>(ctx->lcp_tk),
                        P<uint32_t>(ctx->lcp_tv), nullptr, nc, 64, P<int32_t>(ctx->rs_hist), P<int64_t>(ctx->rs_off),
                        st);
  launch_lcp_runs(P<uint64_t>(ctx->lcp_ckey), nc, P<int32_t>(ctx->lcp_start), st);
  launch_scan_i32_to_i64(P<int32_t>(ctx->lcp_start), P<int64_t>(ctx->lcp_pos), nullptr, nc, nullptr, st);
  launch_lcp_reduce(P<uint64_t>(ctx->lcp_ckey), P<uint32_t>(ctx->lcp_cidx), P<double>(ctx->lcp_cval), nc,
                    P<int32_t>(ctx->lcp_start), P<int64_t>(ctx->lcp_pos), b_row, b_col, b_val, cap_b, st);
  HIPCHK(hipGetLastError());
  int64_t nb = 0;
  unsigned long long ovf = 0;
  HIPCHK(hipMemcpyAsync(&nb, P<int64_t>(ctx->lcp_pos) + nc, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&ovf, ctx->lcp_ovf.p, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *n_b = nb;
  if (ovf) return fail(ctx, STIV_E_CAPACITY, "a vesicle has more than 128 volumes or 2048 active points");
  if (nb > cap_b) return fail(ctx, STIV_E_CAPACITY, "B capacity too small");
  return STIV_OK;
}

int stiv_mlp_nparam(void) { return mlp_nparam(); }

stiv_status stiv_set_toi_model(stiv_ctx *ctx, const float *params, int n, float kwidth) {
  if (!ctx) return STIV_E_ARG;
  if (!params) {
    ctx->have_model = false;
    return STIV_OK;
  }
  if (n != mlp_nparam()) return fail(ctx, STIV_E_ARG, "model must have stiv_mlp_nparam() parameters");
  if (!(kwidth > 0.0f) || !std::isfinite(kwidth)) return fail(ctx, STIV_E_ARG, "bracket width must be finite and > 0");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(ctx, STIV_E_ARG, "model parameters must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(ensure(ctx->toi_params, sizeof(float) * (size_t)n));
  HIPCHK(hipMemcpy(ctx->toi_params.p, params, sizeof(float) * (size_t)n, hipMemcpyHostToDevice));
  HIPCHK(ensure(ctx->toi_packed, mlp_packed_bytes()));
  launch_mlp_pack(P<float>(ctx->toi_params), ctx->toi_packed.p, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  ctx->toi_kwidth = kwidth;
  ctx->have_model = true;
  return STIV_OK;
}

stiv_status stiv_mlp_forward(stiv_ctx *ctx, const float *params, const float *x, int64_t n, float *out, void *stream) {
  if (!ctx || n < 0 || !params || (n > 0 && (!x || !out))) return fail(ctx, STIV_E_ARG, "bad mlp_forward arguments");
  HIPCHK(hipSetDevice(ctx->device));
  launch_mlp_forward(params, x, n, out, reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

stiv_status stiv_mlp_grad(stiv_ctx *ctx, const float *params, const float *x, const float *target, int64_t n,
                          float *grad, float *loss, void *stream) {
  if (!ctx || n < 0 || !params || !grad || (n > 0 && (!x || !target)))
    return fail(ctx, STIV_E_ARG, "bad mlp_grad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t need = sizeof(float) * (size_t)mlp_grad_blocks(n) * (size_t)(mlp_nparam() + 1);
  HIPCHK(ensure(ctx->mlp_part, need));
  launch_mlp_grad(params, x, target, n, P<float>(ctx->mlp_part), grad, loss, reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

stiv_status stiv_mlp_adam(stiv_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                          float beta1, float beta2, float eps, void *stream) {
  if (!ctx || !params || !grad || !m || !v || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(ctx, STIV_E_ARG, "bad adam arguments");
  HIPCHK(hipSetDevice(ctx->device));
  launch_adam(params, grad, m, v, step, lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return STIV_OK;
}

}  // extern "C"

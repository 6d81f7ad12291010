// Internal declarations shared by the HIP translation units of libstiv.
// Not part of the public ABI (see include/stiv.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stiv {

// ---------------------------------------------------------------------------
// Tiling limits.  A patch is a set of neighbouring triangles of one topology
// together with the vertices and edges it owns (every vertex and edge of the
// mesh is owned by exactly one patch), so a (patch, patch) work item yields
// every primitive pair exactly once.
// ---------------------------------------------------------------------------
// Patch sizes (triangles per patch) the kernels are built for, and the LDS
// capacities each size needs.  The host tiling stops growing a patch before
// any capacity would be exceeded.
template <int TILE>
struct TileCaps;
template <>
struct TileCaps<16> {
  static constexpr int ref = 24, ownv = 24, owne = 40;
};
template <>
struct TileCaps<32> {
  static constexpr int ref = 40, ownv = 40, owne = 64;
};
template <>
struct TileCaps<64> {
  static constexpr int ref = 64, ownv = 64, owne = 128;
};
// Per-patch blob: everything the primitive kernel needs about one patch in
// one contiguous, fixed-stride block of ints.  Layout (ints): header (number
// of referenced vertices, owned vertices, triangles, owned edges); byte
// arrays packed four to an int: slot (index into the referenced list) of
// every owned vertex, of the three corners of every triangle and of the two
// ends of every owned edge; the owned vertex, triangle and owned edge ids;
// then the referenced vertices' local ids.  The first `stage` ints (header,
// slots and ids) are what a work item keeps in LDS; the referenced ids only
// address the positions it loads.
template <int TILE>
struct BlobLayout {
  static constexpr int ref = TileCaps<TILE>::ref, ownv = TileCaps<TILE>::ownv, owne = TileCaps<TILE>::owne;
  static constexpr int hdr = 0, vslot = 4, tslot = vslot + ownv / 4, eslot = tslot + 3 * TILE / 4,
                       lds = (eslot + 2 * owne / 4 + 3) / 4 * 4, pvtx = lds, ptri = pvtx + ownv, pedge = ptri + TILE,
                       pref = pedge + owne, stage = pref, used = pref + ref, stride = (used + 63) / 64 * 64;
  static_assert(ownv % 4 == 0 && (3 * TILE) % 4 == 0 && (2 * owne) % 4 == 0, "byte arrays fill whole ints");
  static_assert(stage % 4 == 0 && stage / 4 <= 128, "the staged part is at most two int4 per lane");
};

// Patch-pair work item: pair index, global patch-table indices of the two
// patches, the first global vertex of each vesicle and the slots of the two
// patches in the per-call patch-box array.
struct __align__(16) WorkRec {
  int p, pa, pb, base_a;
  int base_b, box_a, box_b, pad;
};

constexpr int kMaxPatchTri = 64;   // largest supported patch
constexpr int kMaxPatchRef = 64;
constexpr int kMaxPatchesPerVes = 1024;
constexpr int kMaxShift = 7;       // |sigma_c| bound for periodic images (pair key packing)

// Device copy of the topology tables (all arrays indexed by topology or by
// global patch-table index).
struct DevTopo {
  int n_topo;
  const int *nv, *nt, *ne;             // [n_topo]
  const int *tri_off, *edge_off;       // [n_topo+1]
  const int *tri;                      // [sum nt][3]
  const int *edge;                     // [sum ne][2]
  const int *patch_off;                // [n_topo+1] patch-table range of each topology
  const int *ptri_off;                 // [n_ptab+1]
  const int *ptri;                     // triangle ids (local to the topology)
  const uint8_t *ptri_slot;            // [..][3] ref-slot of each corner
  const int *pvtx_off, *pvtx;          // owned vertices (local ids)
  const uint8_t *pvtx_slot;            // ref-slot of each owned vertex
  const int *pedge_off, *pedge;        // owned edges (edge ids)
  const uint8_t *pedge_slot;           // [..][2]
  const int *pref_off, *pref;          // referenced vertices (local ids)
  const int *vbase;                    // [n_topo] first row of each topology in vp_off
  const int *vp_off, *vp;              // vertex -> patches (local patch index) referencing it
  const int4 *vp4;                     // [rows] the same, up to 4 per vertex, -1 padded; .w == -2:
                                       // more than 4, read vp_off / vp
  const int *blob;                     // [n_ptab][blob_stride] patch blobs (BlobLayout of the current tile)
  int blob_stride;
  const int4 *tri_rec;                 // [sum nt] (three local vertex ids, local patch index) of every
                                       // triangle, in patch order: patch P's from ptri_off[P] on
  int max_nv;                          // largest vertex count of the topologies
};

// Patch bounds beyond the axis-aligned box: the support of the patch's
// triangles' space-time boxes along the six face diagonals of the cube,
// (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1) (a 9-DOP together
// with the box).  Per patch 12 floats, [direction][low, high], rounded
// outward (computed by the box kernel from FP32 vertex boxes).
constexpr int kDopDirs = 6;
constexpr int kDopVals = 2 * kDopDirs;

struct DevScene {
  int n_ves, n_vtx, n_scenes;
  const int *vtx_off, *topo_id, *scene_off;
  const double *box_len, *x0, *x1;
};

// Per-scene implicit Morton grid (Alg. 1): origin, cell widths, depth.
struct SceneGrid {
  double org[3], w[3], tiny;
  int depth, periodic[3], pad;
};

// One candidate vesicle pair, canonical order.
struct PairRec {
  int a, b;
  int s[3];
  int pad;
  double sh[3];  // sigma * L, FP64
};

// Device counters read back once per detect.
struct Counters {
  unsigned long long n_cp;         // check points
  unsigned long long n_raw_pairs;  // pair insertions (with duplicates)
  unsigned long long n_pairs;
  unsigned long long n_work;       // patch-pair work items
  unsigned long long n_pre;        // FP32 pre-candidates (superset of the exact candidates)
  unsigned long long n_cand_vt, n_cand_ee;  // exact FP64 candidates
  unsigned long long n_hard_vt_ee;  // root-search queue: vertex-triangle (low 32 bits) and edge-edge
                                    // (high 32 bits) candidates, from its front and from its back
  unsigned long long n_cand_list;  // candidates written to the optional list
  unsigned long long n_ct, n_ct_vt, n_ct_ee;
  unsigned long long n_vol, n_jrow;
  unsigned long long within_d, degenerate;
  unsigned long long hash_overflow, shift_overflow, nonfinite, lds_fallback;
  unsigned long long n_tests;      // primitive box-pair tests of the candidate sweep
  unsigned long long n_bracket_ok;  // root searches whose predicted bracket was certified
  unsigned long long work_claimed;  // work-item chunks handed out by the primitive kernel
  unsigned long long search_exhausted;  // root searches stopped by their budget of intervals
  unsigned long long cp_key_bits[2];    // OR of the check-point keys, OR of their complements
  unsigned long long n_pair_order[2];   // vesicle pairs with contacts: large buckets, the others
};

// Candidates queued for the root search (both kinds).
__host__ __device__ inline unsigned long long hard_total(unsigned long long vt_ee) {
  return (vt_ee & 0xffffffffull) + (vt_ee >> 32);
}

// Narrow-phase candidate record.
struct Cand {
  int pair, kind, i, j;
};

// ---------------------------------------------------------------------------
// Launchers (host side), one per kernel.  Where a count lives on the device
// (`*_dev`), the kernel reads it at run time and clamps it to the given
// capacity, so the host never waits for an intermediate count.
// ---------------------------------------------------------------------------
// scan / sort / fill.  With n_dev != nullptr the length is min(*n_dev, n_host).
// Exclusive scans: out[0 .. n] with out[n] the total; n = min(*n_dev, n_host)
// when a device count is given.  tmp: scan_scratch_elems(n_host) int64
// (NULL: one workgroup, for short inputs).
int64_t scan_scratch_elems(int64_t n_host);
void launch_scan_i64(const int64_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                     int64_t *tmp, hipStream_t st);
void launch_scan_i32_to_i64(const int32_t *in, int64_t *out, const unsigned long long *n_dev, int64_t n_host,
                            int64_t *tmp, hipStream_t st);
// Stable sort of n keys (device count n_dev clamped to n_host, or n_host)
// by their low key_bits bits, values moved along; tk, tv: n_host scratch;
// hist: 256 * radix_scratch_blocks(n_host) ints, hoff: radix_offset_elems(n_host) int64.
// bits_dev (optional, device): the OR of the keys and the OR of their
// complements; a digit where every key has the same bits is skipped at once.
int64_t radix_scratch_blocks(int64_t n_host);
int64_t radix_offset_elems(int64_t n_host);
void launch_radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *tk, uint32_t *tv,
                           const unsigned long long *n_dev, int64_t n_host, int key_bits, int32_t *hist,
                           int64_t *hoff, hipStream_t st, const unsigned long long *bits_dev = nullptr);
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st);
// Up to 8 fills (4- or 8-byte elements) in one launch.
struct FillJob {
  void *p;
  uint64_t v;
  int64_t n;
  int bytes;
};
struct FillJobs {
  FillJob job[8];
  int count = 0;
  void add(void *p, uint64_t v, int64_t n, int bytes) {
    if (n > 0) job[count++] = FillJob{p, v, n, bytes};
  }
};
void launch_fill_multi(const FillJobs &J, hipStream_t st);
// Two exclusive scans of the same length (one launch when short enough).
void launch_scan2_i32_to_i64(const int32_t *in0, int64_t *out0, const int32_t *in1, int64_t *out1,
                             const unsigned long long *n_dev, int64_t n_host, int64_t *tmp, hipStream_t st);
void launch_iota_u32(uint32_t *p, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);

// K0
// Per vesicle: its patch count and scene index; for scenes of up to a few
// thousand vesicles also the scan of the counts into patch_off (returns
// true), which is otherwise left to launch_scan_i64.
bool launch_ves_tables(const DevScene &S, const DevTopo &T, int64_t *patch_cnt, int *ves_scene, int64_t *patch_off,
                       hipStream_t st);
// patch_dop: every patch's face-diagonal supports (kDopVals floats per patch
// slot).
// Parts of the box kernel: vesicle and patch boxes; the patches' supports
// along the face diagonals; or, with the boxes, supports that never cull
// (for topologies without supports, see boxes_have_supports).  At most
// grid_max workgroups.
constexpr int kBoxParts = 1, kSupportParts = 2, kNoSupportParts = 4;
bool boxes_have_supports(const DevTopo &T, int max_patches);
void launch_boxes(const DevScene &S, const DevTopo &T, double h, const int64_t *ves_patch_off, double *ves_box,
                  double *patch_box, float *patch_dop, int max_patches, int parts, int grid_max, Counters *cnt,
                  hipStream_t st);

// K1
// With a single scene, also the check points' offsets (cp_off, the scan of
// cp_cnt); otherwise cp_off is left to launch_scan_i64.
void launch_scene_grid(const DevScene &S, const double *ves_box, SceneGrid *grid, int64_t *cp_cnt, int64_t *cp_off,
                       hipStream_t st);
// Also ORs every written key and its complement into cnt->cp_key_bits.
void launch_cp_emit(const DevScene &S, const double *ves_box, const int *ves_scene, const SceneGrid *grid,
                    const int64_t *cp_off, uint64_t *keys, uint32_t *vals, int64_t cap, Counters *cnt,
                    hipStream_t st);
void launch_cell_pairs(const DevScene &S, const double *ves_box, const int *ves_scene, const uint64_t *keys,
                       const uint32_t *vals, const unsigned long long *n_cp, int64_t n_cp_cap, uint64_t *hash,
                       int64_t hash_cap, Counters *cnt, hipStream_t st);
void launch_hash_list(const uint64_t *hash, int64_t hash_cap, uint64_t *uniq, int64_t uniq_cap, int32_t *cnt_a,
                      Counters *cnt, hipStream_t st);
void launch_pair_bucket_scatter(const uint64_t *uniq, int64_t uniq_cap, const int64_t *off_a,
                                int32_t *cursor_a, uint64_t *sorted, Counters *cnt, hipStream_t st);
void launch_pair_bucket_sort_emit(const DevScene &S, const int *ves_scene, const int64_t *off_a,
                                  uint64_t *sorted, int n_ves, PairRec *pairs, int32_t *pair_ab,
                                  int32_t *pair_shift, int64_t cap_pairs, hipStream_t st);

// K2
void launch_patch_pairs(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                        const double *ves_box, const int64_t *ves_patch_off, const double *patch_box,
                        const float *patch_dop, WorkRec *work, int64_t work_cap, int max_patches, Counters *cnt,
                        hipStream_t st);
// hard_geo: geometry of the queued candidates for the root search, SoA
// [24][hard_cap]: X0 (shifted) x, y, z of vertices 0..3, then D = X1 - X0.
void launch_prim_cand(int tile, int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs,
                      const WorkRec *work, int64_t work_cap, const double *patch_box, double d, Cand *hard,
                      double *hard_geo,
                      int64_t hard_cap, Cand *list, int64_t list_cap, Counters *cnt, hipStream_t st);

// K3 + K4: root search on the queued candidates, volumes and gradients
void launch_narrow(int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *hard,
                   const double *hard_geo, int64_t hard_cap,
                   double d, double eps, double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                   int64_t ct_cap, int32_t *pair_cnt, const void *mlp_packed, float kwidth, Counters *cnt,
                   hipStream_t st);

// LCP matrix assembly (Alg. 3)
void launch_lcp_layout(const int *vtx_off, int n_ves, const int32_t *j_vtx, int64_t n_jrow, int32_t *flag,
                       int32_t *a, int64_t *m9, hipStream_t st);
void launch_lcp_emit(const int *vtx_off, int n_ves, const int32_t *flag, const int64_t *act_off, int32_t *act_vtx,
                     hipStream_t st);
void launch_lcp_vcount(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, int32_t *vcnt, hipStream_t st);
void launch_lcp_vscatter(const int32_t *vol_pair, const int32_t *pair_ab, int64_t n_vol, const int64_t *voff,
                         int32_t *vcur, int32_t *vlist, int n_ves, int64_t *c2, hipStream_t st);
void launch_lcp_block(const int *vtx_off, int n_ves, const int64_t *act_off, const int64_t *m_off,
                      const int32_t *act_vtx, const double *M, const int64_t *voff, const int32_t *vlist,
                      const int32_t *j_vol, const int32_t *j_vtx, const double *j_g, int64_t n_jrow,
                      const int64_t *coff, uint64_t *ckey, double *cval, unsigned long long *overflow,
                      hipStream_t st);
void launch_lcp_runs(const uint64_t *key, int64_t n, int32_t *start, hipStream_t st);
void launch_lcp_reduce(const uint64_t *key, const uint32_t *idx, const double *cval, int64_t n, const int32_t *start,
                       const int64_t *pos, int32_t *b_row, int32_t *b_col, double *b_val, int64_t cap,
                       hipStream_t st);

// Learned contact-time bracket (perceptron kernels)
int mlp_nparam();
size_t mlp_packed_bytes();
void launch_mlp_pack(const float *params, void *packed, hipStream_t st);
void launch_mlp_forward(const float *params, const float *x, int64_t n, float *out, hipStream_t st);
int mlp_grad_blocks(int64_t n);
void launch_mlp_grad(const float *params, const float *x, const float *target, int64_t n, float *part, float *grad,
                     float *loss, hipStream_t st);
void launch_adam(float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2, float eps,
                 hipStream_t st);

// K5
// Buckets the contacts by vesicle pair (perm), and lists the pairs with
// contacts in `order` (cap_pairs entries; large buckets first) while writing
// the empty results of the others.
void launch_ct_scatter_order(const Cand *ct, int64_t ct_cap, Counters *cnt, const int64_t *pair_off,
                             int32_t *cursor, int32_t *perm, int64_t pairs_cap, int32_t *order, double *pair_V,
                             int32_t *pair_hasvt, int32_t *pair_rows, hipStream_t st);
void launch_ct_sort_aggregate(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                              const Counters *cnt, const int32_t *order, const int64_t *pair_off, const int32_t *perm,
                              const Cand *ct,
                              const double *ct_s, const double *ct_vol, const double *ct_grad, double dt,
                              uint64_t *gkeys, int32_t *gidx, int32_t *out_key, double *out_tau, double *out_s,
                              double *out_vol, double *out_grad, int64_t cap_ct, double *pair_V, int32_t *pair_hasvt,
                              int32_t *pair_rows, int32_t *row_vtx_tmp, double *row_g_tmp, hipStream_t st);
void launch_write_volumes(Counters *cnt, int64_t pairs_cap, const int64_t *pair_off, const int64_t *vol_off,
                          const int64_t *row_off, const int32_t *pair_hasvt, const double *pair_V,
                          const int32_t *pair_rows, const int32_t *row_vtx_tmp, const double *row_g_tmp,
                          int32_t *vol_pair, double *vol_V, int64_t cap_vol, int32_t *j_vol, int32_t *j_vtx,
                          double *j_g, int64_t cap_jrow, const int64_t *cp_total, hipStream_t st);
// Backward pass.  Its scratch, carved from one buffer at these byte offsets
// (256-aligned) for n_ct contacts and n_jrow Jacobian rows.
struct BwdLayout {
  size_t contrib, gkeys, gidx, rowc, rkey, rval, tk, tv, hist, hoff, total;
};
BwdLayout backward_layout(int64_t n_ct, int64_t n_jrow);
// The static scratch of stiv_backward_static: its size, and its device
// address on `device` (looked up once per device).
size_t backward_static_bytes();
hipError_t backward_static_scratch(int device, void **ptr);
void launch_backward(const DevScene &S, const DevTopo &T, double d, double eps, double dt, int64_t n_ct,
                     const int32_t *ct_key, const double *ct_tau, const int32_t *pair_ab, const int32_t *pair_shift,
                     int64_t n_vol, const int32_t *vol_pair, int64_t n_jrow, const int32_t *j_vol,
                     const int32_t *j_vtx, const double *dV, const double *dG, const double *ct_s, double *contrib,
                     uint64_t *gkeys, int32_t *gidx, double *rowc, uint64_t *rkey, uint32_t *rval, uint64_t *tk,
                     uint32_t *tv, int32_t *hist, int64_t *hoff, double *dX0, double *dX1, hipStream_t st);

}  // namespace stiv

/*
 * stiv.h -- C ABI of the MI355X (gfx950) contact-detection library.
 *
 * Computes, for vesicle surface meshes at t_n (X0) and at the candidate
 * position t_{n+1} (X1), following Lu, Rahimian & Zorin, "Parallel
 * contact-aware simulations of deformable particles in 3D Stokes flow":
 *
 *   - space-time bounding boxes of every vesicle (Sec. 3.3.1; Alg. 2,
 *     getBoundingBox), inflated by d/2 per side;
 *   - candidate vesicle pairs through a Morton-ordered implicit grid of check
 *     points (Alg. 1: average box diagonal, check points, stable sort by
 *     Morton ID, per-cell pair test, unique);
 *   - primitive candidates inside each vesicle pair (vertex-triangle both
 *     ways, edge-edge) whose space-time boxes intersect;
 *   - the narrow phase: earliest s in [0,1] where a vertex comes within d of
 *     a triangle's plane with its projection inside the triangle (Eq. 3.1,
 *     linear trajectories), and the edge-edge analogue;
 *   - each vertex-triangle contact's space-time interference volume
 *     (Eq. 3.2, App. A) and its gradient with respect to X1 of the four
 *     vertices, including the contact time's dependence on X1;
 *   - one contact volume per vesicle pair, V = sum of V_k, and the rows of
 *     the Jacobian J = dV/dX1 per (volume, vertex) (Sec. 3.1.2, 3.3.2).
 *
 * Conventions
 *   - Every array pointer in stiv_scene and stiv_result is a DEVICE pointer
 *     owned by the caller.  stiv_topology holds HOST pointers, copied by
 *     stiv_set_topology.  The library owns only its context's scratch arena.
 *   - Positions are FP64 SoA [3][n_vtx].  The narrow phase, volumes and
 *     gradients are FP64; FP32 appears only in conservative pre-filters.
 *   - Periodic image shifts sigma in Z^3 translate vesicle b by sigma*L.
 *     Pairs are (a, b, sigma) with a < b, or a == b and sigma > 0
 *     lexicographically (a vesicle against its own image).
 *   - Sign: the exported volume is the nonnegative interference magnitude of
 *     Eq. 3.2; the constraint of Eq. 2.5 / 3.4 is -V >= 0.
 *   - Edge-edge contacts are detected and reported with their time but add
 *     nothing to V or J (the paper sums vertex-triangle volumes only).
 *   - Outputs are written in canonical order: pairs by (a, b, sigma),
 *     contacts by (pair, kind, i, j), volumes by pair, J rows by (volume,
 *     vertex).  Two runs on the same input are bit-identical.
 *   - Errors: every entry point returns a stiv_status; stiv_last_error gives
 *     a message.  On STIV_E_CAPACITY the n_* fields hold the required sizes
 *     and the arrays are incomplete; reallocate and call again.
 */
#ifndef STIV_H
#define STIV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stiv_ctx stiv_ctx;

typedef enum {
  STIV_OK = 0,
  STIV_E_ARG = -1,      /* bad argument: d < 0, eps <= 0, dt <= 0, box_len < 0, bad offsets, no topology */
  STIV_E_CAPACITY = -2, /* a caller-provided output array is too small (see n_* for the sizes needed) */
  STIV_E_HIP = -3,      /* a HIP runtime call failed */
  STIV_E_NUMERIC = -4,  /* a position is NaN or infinite, or a root search ran out of its budget */
  STIV_E_STATE = -5     /* call order violated (e.g. detect before set_topology) */
} stiv_status;

/* Per-order mesh topology (HOST pointers), shared by all vesicles using it.
 * Triangles are local vertex ids, oriented outward (counter-clockwise seen
 * from outside); edges are (lo, hi) local ids.  Topology t owns triangles
 * tri[tri_off[t] .. tri_off[t+1]) and edges edge[edge_off[t] .. edge_off[t+1]). */
typedef struct {
  int32_t n_topo;
  const int32_t *nv;       /* [n_topo] vertices per vesicle of this topology */
  const int32_t *tri;      /* [sum nt][3] */
  const int32_t *tri_off;  /* [n_topo+1] */
  const int32_t *edge;     /* [sum ne][2] */
  const int32_t *edge_off; /* [n_topo+1] */
} stiv_topology;

/* A batch of independent scenes (DEVICE pointers).  Vesicle v owns global
 * vertices [vtx_off[v], vtx_off[v+1]) and uses topology topo_id[v]; scene s
 * owns vesicles [scene_off[s], scene_off[s+1]); pairs never cross scenes.
 * box_len[s][c] > 0 makes axis c of scene s periodic with that period;
 * 0 means free space on that axis.  Image shifts are limited to |sigma_c| <=
 * 7 (a vesicle box may span at most about 7 periods): beyond that stiv_detect
 * returns STIV_E_ARG.  At most 2^24 - 1 vesicles per call. */
typedef struct {
  int32_t n_ves, n_vtx, n_scenes;
  const int32_t *vtx_off;   /* [n_ves+1] */
  const int32_t *topo_id;   /* [n_ves] */
  const int32_t *scene_off; /* [n_scenes+1] */
  const double *box_len;    /* [n_scenes][3] */
  const double *x0;         /* [3][n_vtx] positions at t_n */
  const double *x1;         /* [3][n_vtx] candidate positions at t_{n+1} */
} stiv_scene;

/* d: minimum separation of the triangle meshes, (1 + 2 alpha) d_m (Sec. 3.1.2);
 * eps: velocity scale of the space-time metric (App. A), > 0; dt: time step, > 0. */
/* flags: STIV_EMIT_CANDIDATES also writes the list of primitive candidates;
 * STIV_LEARNED_BRACKET searches each root first inside the bracket predicted
 * by the model set with stiv_set_toi_model (same contacts, see there). */
enum { STIV_EMIT_CANDIDATES = 1u, STIV_LEARNED_BRACKET = 2u };
typedef struct {
  double d, eps, dt;
  uint32_t flags;
} stiv_params;

/* Outputs.  The caller sets cap_* and the array pointers (DEVICE memory);
 * the library writes the n_* counts (always the true count, also when it
 * exceeds the capacity).
 *   pair_ab [cap_pairs][2], pair_shift [cap_pairs][3]
 *   cand    [cap_cand][4] = (pair, kind, i, j), written only with
 *           STIV_EMIT_CANDIDATES (order unspecified)
 *   ct_key  [cap_ct][4] = (pair, kind, i, j); kind 0: vertex i of a vs
 *           triangle j of b; kind 1: vertex i of b vs triangle j of a;
 *           kind 2: edge i of a vs edge j of b (local ids)
 *   ct_tau  [cap_ct]    contact time tau = s* dt
 *   ct_vol  [cap_ct]    V_k (0 for edge-edge)
 *   ct_grad [cap_ct][12] dV_k/dX1 of (vertex, triangle corner 0, 1, 2)
 *   vol_pair, vol_V [cap_vol]: contact volumes (pairs with >= 1 VT contact)
 *   j_vol, j_vtx, j_g [cap_jrow] ([cap_jrow][3] for j_g): Jacobian rows
 *           (volume index, global vertex id, dV/dX1 of that vertex)
 *   ct_s    [cap_ct] optional (NULL: not written): the contact parameter
 *           s* in [0,1] itself (tau = s* dt); stiv_backward uses it when
 *           given, so that it differentiates at the forward's own root
 * Diagnostics (counts over the whole call):
 *   n_initially_within_d   contacts at s* = 0 (vertex already within d and
 *                          inside its triangle at t_n)
 *   n_degenerate_skipped   candidates skipped because F vanishes
 *                          identically or the normal vanishes at a root
 *   n_search_exhausted     root searches (Eq. 3.1) that examined their
 *                          whole budget of 4096 Bernstein intervals without
 *                          settling; their contacts may be missing, so a
 *                          nonzero count makes stiv_detect / stiv_collect
 *                          return STIV_E_NUMERIC (all outputs are still
 *                          written) */
typedef struct {
  int64_t cap_pairs, n_pairs;
  int32_t *pair_ab;
  int32_t *pair_shift;
  int64_t cap_cand, n_cand_vt, n_cand_ee;
  int32_t *cand;
  int64_t cap_ct, n_ct_vt, n_ct_ee;
  int32_t *ct_key;
  double *ct_tau, *ct_vol, *ct_grad;
  int64_t cap_vol, n_vol;
  int32_t *vol_pair;
  double *vol_V;
  int64_t cap_jrow, n_jrow;
  int32_t *j_vol, *j_vtx;
  double *j_g;
  int64_t n_initially_within_d, n_degenerate_skipped;
  double *ct_s;
  int64_t n_search_exhausted;
} stiv_result;

/* Create a context on a HIP device.  *ctx is NULL on failure. */
stiv_status stiv_create(stiv_ctx **ctx, int hip_device);
stiv_status stiv_destroy(stiv_ctx *ctx);

/* Copy the mesh topologies and build the library's patch tiling of each
 * (groups of neighbouring triangles with their owned vertices and edges). */
stiv_status stiv_set_topology(stiv_ctx *ctx, const stiv_topology *topo);

/* Triangles per patch of the primitive broad phase: 16, 32 or 64 (default
 * 64).  Changing it discards the topology tiling, so call stiv_set_topology
 * afterwards.  Results do not depend on it; speed does (see the autotuner). */
stiv_status stiv_set_patch_size(stiv_ctx *ctx, int tri_per_patch);

/* Tuning options (results never depend on them): STIV_OPT_PATCH_TRI
 * (16/32/64, as stiv_set_patch_size), STIV_OPT_PRIM_BLOCKS and
 * STIV_OPT_NARROW_BLOCKS (workgroups of the persistent primitive and
 * root-search kernels, 256..65536), STIV_OPT_QUEUE_CAPACITY (the number of
 * candidates the root-search queue holds before it grows, 64..2^31; detect
 * grows it and runs again when a step needs more, so a small value only
 * exercises that path). */
enum { STIV_OPT_PATCH_TRI = 1, STIV_OPT_PRIM_BLOCKS = 2, STIV_OPT_NARROW_BLOCKS = 3, STIV_OPT_QUEUE_CAPACITY = 4 };
stiv_status stiv_set_option(stiv_ctx *ctx, int option, int64_t value);

/* Pre-size the scratch arena for scenes of this shape (optional; detect
 * grows it on demand). */
stiv_status stiv_reserve(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p);

/* Run the whole path on `stream` (a hipStream_t; NULL = default stream).
 * All kernels are enqueued on the stream without host synchronisation; the
 * call then synchronises the stream once to read the counts into *out. */
stiv_status stiv_detect(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, stiv_result *out,
                        void *stream);

/* Graph-capturable detect.  Enqueues the same pipeline as stiv_detect on
 * `stream` with no host synchronisation, no allocation, no host copies and
 * no event records, so it can be captured into a hipGraph and replayed.
 * Requires a prior stiv_detect (or stiv_reserve) on a scene with the same
 * structural arrays, which sizes the arena; the counts stay on the device
 * until stiv_collect.  Candidate lists (STIV_EMIT_CANDIDATES) are not
 * available here. */
stiv_status stiv_detect_async(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, stiv_result *out,
                              void *stream);

/* Synchronise `stream` and read the counts of the last stiv_detect_async (or
 * graph replay) into *out.  STIV_E_CAPACITY if an internal buffer or an
 * output array was too small (run stiv_detect once to grow the arena, then
 * capture again). */
stiv_status stiv_collect(stiv_ctx *ctx, const stiv_params *p, stiv_result *out, void *stream);

/* Backward pass (adjoint) of a detect.  `res` is the complete result of a
 * stiv_detect on the same scene and parameters (its device arrays must be
 * unchanged).  With cotangents dL_dV [n_vol] of the contact volumes and
 * dL_dG [n_jrow][3] of the Jacobian rows (either may be NULL = zero), writes
 * dL_dX0 and dL_dX1 [3][n_vtx] (overwritten; either may be NULL):
 *   dL/dX = sum over VT contacts k of  gV grad V_k + H_k w,
 * grad over X0 and X1 including the contact time's dependence on them
 * (Eq. 3.1-3.2), H_k the Hessian of V_k, w the dL_dG rows of its vertices.
 * Edge-edge contacts contribute nothing (they add nothing to V).  The
 * contact parameter of each contact is res->ct_s when given, else
 * ct_tau / dt.  Enqueued on `stream`, no synchronisation.  Every vertex's
 * sum runs in one fixed order (contacts in canonical order, then volumes in
 * order), so repeated calls are bit-identical. */
stiv_status stiv_backward(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, const stiv_result *res,
                          const double *dL_dV, const double *dL_dG, double *dL_dX0, double *dL_dX1, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): stiv_backward with all of its scratch in one static device
 * array of STIV_BACKWARD_STATIC_BYTES per GPU, owned by the library and held
 * until the process ends.  Same arguments, kernels, results and summation
 * order as stiv_backward (bit-identical outputs).  It allocates nothing, makes
 * no host copy and does not synchronise: the scene's structural arrays
 * (vtx_off, topo_id, scene_off, box_len and the sizes) must be the ones a
 * previous stiv_detect or stiv_reserve on this context validated
 * (STIV_E_STATE otherwise).  Scratch needed: about 288 bytes per contact
 * (n_ct_vt + n_ct_ee) plus 72 bytes per Jacobian row, rounded up;
 * STIV_E_CAPACITY with a message giving the need when it exceeds the array
 * (the 1440-vesicle workload, 196K contacts and 55K rows, fits).  All calls
 * on one GPU share the array and each call writes every part of it it reads:
 * calls that overlap in time on one GPU (other streams, other contexts,
 * other threads) race and must be serialised by the caller. */
#define STIV_BACKWARD_STATIC_BYTES (64ull << 20)
stiv_status stiv_backward_static(stiv_ctx *ctx, const stiv_scene *s, const stiv_params *p, const stiv_result *res,
                                 const double *dL_dV, const double *dL_dG, double *dL_dX0, double *dL_dX1,
                                 void *stream);

/* Milliseconds of the last detect, measured with HIP events on the call's
 * stream: 0 box kernel, 1 vesicle broad phase (Morton grid), 2 patch-pair
 * cull, 3 primitive candidates, 4 narrow phase with volumes and gradients,
 * 5 aggregation, 6 whole call on the device.  Fills min(n, 7) values. */
stiv_status stiv_get_stage_times(stiv_ctx *ctx, float *ms, int n);

/* Work counts of the last detect (diagnostics, tuning): 0 check points,
 * 1 candidate vesicle pairs, 2 patch-pair work items, 3 FP32 pre-candidates
 * (a superset of the candidates), 4 vertex-triangle candidates, 5 edge-edge
 * candidates, 6 candidates that needed a root search (F may vanish on [0,1]
 * and the closest-point test may pass somewhere on [0,1]), 7 contacts,
 * 8 primitive box-pair tests made by the candidate sweep, 9 root searches
 * whose learned bracket was certified (STIV_LEARNED_BRACKET).
 * Fills min(n, 10) values. */
stiv_status stiv_get_stats(stiv_ctx *ctx, int64_t *vals, int n);

/* Device pointers to the library's internal Morton sort (tests only need
 * it for the worked example of Alg. 1 / Table 3): stable sort of n 64-bit
 * keys with 32-bit values, ascending, equal keys keep input order. */
stiv_status stiv_sort_pairs_u64(stiv_ctx *ctx, uint64_t *keys, uint32_t *vals, int64_t n, void *stream);

/* ---------------------------------------------------------------------------
 * LCP matrix (Sec. 3.3.3, Alg. 3).  B = J M J^T over the contact volumes of
 * a stiv_detect result: B(j,k) = sum over vesicles i of g_j,i . M_i g_k,i,
 * with g_j,i the Jacobian row of volume j restricted to the points of
 * vesicle i and M_i the vesicle's block of the operator (A_ii^-1 G_ii in the
 * paper's time stepping; supplied by the caller).  Only points that appear in
 * J enter, so M_i is given on the vesicle's ACTIVE points.
 * ------------------------------------------------------------------------- */

/* Active points of every vesicle.  res: the (complete, device) output of
 * stiv_detect on scene s.  Writes act_off [n_ves+1] (int64, DEVICE): the
 * active list of vesicle i is act_vtx[act_off[i] .. act_off[i+1]) (global
 * vertex ids, ascending); m_off [n_ves+1] (int64, DEVICE): offsets, in
 * doubles, of the blocks M_i in the operator array, each M_i being
 * [3 a_i][3 a_i] row-major with a_i = act_off[i+1] - act_off[i], rows and
 * columns point-major (x, y, z of active point 0, then point 1, ...).
 * *n_act, *n_m (HOST): totals.  E_CAPACITY (counts still written) when
 * n_act > cap_act.  Synchronous on stream. */
stiv_status stiv_lcp_layout(stiv_ctx *ctx, const stiv_scene *s, const stiv_result *res, int64_t *act_off,
                            int64_t *m_off, int32_t *act_vtx, int64_t cap_act, int64_t *n_act, int64_t *n_m,
                            void *stream);

/* Assemble B (Alg. 3) from res and the operator blocks M (DEVICE doubles in
 * the stiv_lcp_layout layout).  Output: the structural nonzeros of B (every
 * (j,k) whose volumes share a vesicle) as COO b_row, b_col (int32), b_val
 * (FP64), sorted by (row, col), DEVICE arrays of capacity cap_b; *n_b (HOST)
 * their number.  Sums over vesicles run in vesicle order (reproducible).
 * E_CAPACITY when n_b > cap_b (*n_b still written) or when a vesicle has
 * more than 128 volumes or 2048 active points.  Synchronous on stream. */
stiv_status stiv_form_lcp(stiv_ctx *ctx, const stiv_scene *s, const stiv_result *res, const int64_t *act_off,
                          const int64_t *m_off, const int32_t *act_vtx, const double *M, int32_t *b_row,
                          int32_t *b_col, double *b_val, int64_t cap_b, int64_t *n_b, void *stream);

/* ---------------------------------------------------------------------------
 * Learned contact-time bracket (a learned heuristic on top of the root search
 * of Eq. 3.1, not part of the paper's method; it never changes results).
 *
 * Model: perceptron 18 -> 64 -> 64 -> 2 with ReLU, evaluated with bf16
 * weights and activations and FP32 accumulation.  Parameters, FP32, flat:
 * W1[18][64] b1[64] W2[64][64] b2[64] W3[64][2] b3[2] (y = x W + b).
 * Input features of a candidate: the other three vertices relative to the
 * first vertex of the triangle (vertex-triangle: b - a, c - a, p - a) or of
 * the first edge (edge-edge: b - a, c - a, e - a), at t_n then at t_{n+1}
 * (images shifted by sigma L), divided by the mean edge length of the two
 * primitives at t_n.  Outputs o: predicted first root mu = sigmoid(o0) in
 * [0,1] and spread sd = softplus(o1) + 1e-3.  Training loss per sample with
 * first root s: 0.5 ((s - mu) / sd)^2 + log sd (Gaussian negative
 * log-likelihood), averaged over the samples.
 * ------------------------------------------------------------------------- */

/* Number of model parameters (5506). */
int stiv_mlp_nparam(void);

/* Install (copy from HOST memory) the model used with STIV_LEARNED_BRACKET;
 * params NULL removes it.  The search of a candidate then starts in
 * [mu - kwidth sd, mu + kwidth sd] clipped to [0,1]: when the Bernstein
 * coefficients of F on [0, lo] all have one strict sign there is no root
 * before lo and the earliest valid root is the first found in [lo, hi], else
 * in [hi, 1]; otherwise all of [0,1] is searched.  Contacts, their times (up
 * to the final rounding of the refinement) and all other outputs are those
 * of the search without the model.  E_ARG: n != stiv_mlp_nparam(), kwidth
 * <= 0 or a non-finite parameter. */
stiv_status stiv_set_toi_model(stiv_ctx *ctx, const float *params, int n, float kwidth);

/* Model outputs o [n][2] (raw, before the head) for features x [n][18];
 * all DEVICE pointers, asynchronous on stream. */
stiv_status stiv_mlp_forward(stiv_ctx *ctx, const float *params, const float *x, int64_t n, float *out, void *stream);

/* Gradient of the mean training loss over n samples (features x [n][18],
 * targets [n] in [0,1]) with respect to the parameters, into grad
 * [stiv_mlp_nparam()]; the mean loss into *loss (may be NULL).  Backward
 * products also run on bf16 tiles with FP32 accumulation; the cross-workgroup
 * sum is in a fixed order.  DEVICE pointers, asynchronous on stream; uses a
 * scratch buffer owned by ctx (calls on one ctx must not overlap). */
stiv_status stiv_mlp_grad(stiv_ctx *ctx, const float *params, const float *x, const float *target, int64_t n,
                          float *grad, float *loss, void *stream);

/* One Adam step (bias-corrected, step >= 1) on params with moments m, v,
 * all [stiv_mlp_nparam()] FP32 DEVICE arrays, asynchronous on stream. */
stiv_status stiv_mlp_adam(stiv_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                          float beta1, float beta2, float eps, void *stream);

/* Message of the last error on this context (never NULL). */
const char *stiv_last_error(const stiv_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* STIV_H */

/* 2D variant of the stencil-scaling operator (arXiv 1709.06793, Sec. 4.1:
 * the pre-asymptotic modification is fully specified in 2D).
 *
 * A context holds a triangular macro mesh refined `level` times uniformly
 * (each refinement splits a triangle into four), one slot lattice per macro
 * triangle (nodes on macro edges and vertices have a copy in every triangle
 * holding them), Dirichlet nodes = nodes on macro edges held by one triangle.
 * Vectors are device slot vectors of hhg2d_sizes().n_slots entries (FP64 or
 * FP32) in which all copies of a node hold the same value and Dirichlet
 * entries are 0; canonical vectors list the nodes in the order of
 * hhg2d_node_coords.  Errors: the hhg_status codes of hhg.h, message by
 * hhg2d_last_error.  Not thread-safe per context.
 */
#ifndef HHG2D_H
#define HHG2D_H

#include "hhg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhg2d_ctx_s *hhg2d_ctx;

/* hhg2d_apply_scaled without the MA2 modification */
#define HHG2D_FLAG_NO_MODIFICATION 1u

/* xy: n_vert x 2 macro vertex coordinates; tri: n_tri x 3 vertex ids (any
 * orientation, n_tri <= 65535); level 0..13.  Host memory, copied.  HHG_EINVAL for bad sizes,
 * HHG_EMESH for a degenerate triangle or bad ids.  *out is NULL on failure. */
hhg_status hhg2d_create(const double *xy, int32_t n_vert, const int32_t *tri, int32_t n_tri, int32_t level,
                        uint32_t flags, hhg2d_ctx *out);
hhg_status hhg2d_destroy(hhg2d_ctx ctx);
const char *hhg2d_last_error(hhg2d_ctx ctx);
/* slot vector length, canonical node count, unknowns (non-Dirichlet nodes),
 * and after hhg2d_set_coefficient the number of lattice edges whose factor
 * MA2 replaced (any pointer may be NULL) */
hhg_status hhg2d_sizes(hhg2d_ctx ctx, int64_t *n_slots, int64_t *n_nodes, int64_t *n_unknowns,
                       int64_t *n_modified);
/* canonical node coordinates (n_nodes x 2) and Dirichlet flags (n_nodes),
 * host buffers owned by the caller (either may be NULL) */
hhg_status hhg2d_node_coords(hhg2d_ctx ctx, double *xy, uint8_t *dirichlet);
/* k > 0 at every canonical node (host, n_nodes values).  Builds the merged
 * rows of nodes on shared macro edges and vertices and, unless
 * HHG2D_FLAG_NO_MODIFICATION, the MA2 replacements (Sec. 4.1): for a lattice
 * edge e of macro triangle T whose element-matrix entry a^T > 0 (only in
 * triangles with an obtuse angle), with k_{e;min} the least edge average
 * (k_a + k_b)/2 over the edges of the elements of T holding e and
 * lambda_min^T the smallest non-degenerate eigenvalue of
 * A_T x = lambda [[2,-1,-1],[-1,2,-1],[-1,-1,2]] x: if
 * (k_e - k_{e;min}) a^T > k_{e;min} lambda_min^T, e's factor k_e becomes
 * k_{e;min} (1 + lambda_min^T / a^T).  HHG_ECOEF for k <= 0 or non-finite. */
hhg_status hhg2d_set_coefficient(hhg2d_ctx ctx, const double *k);
/* v_slots = copies of v_canon (device buffers; padding slots 0) and back */
hhg_status hhg2d_from_canonical(hhg2d_ctx ctx, hhg_dtype dtype, const void *v_canon, void *v_slots,
                                void *stream);
hhg_status hhg2d_to_canonical(hhg2d_ctx ctx, hhg_dtype dtype, const void *v_slots, void *v_canon,
                              void *stream);
/* y = A u with stencil scaling (eq. (meshdep), M = 1; Lemma 3.2: edge factor
 * (k_a + k_b)/2, zero row sums) and MA2; Dirichlet rows of y are 0.  u, y:
 * distinct device slot vectors; HHG_ESTATE before a coefficient is set. */
hhg_status hhg2d_apply_scaled(hhg2d_ctx ctx, hhg_dtype dtype, const void *u, void *y, void *stream);
/* y = A~ u with nodal integration (eq. (standardfe)): element t contributes
 * the mean of k over its vertices times its element matrix. */
hhg_status hhg2d_apply_nodal(hhg2d_ctx ctx, hhg_dtype dtype, const void *u, void *y, void *stream);

#ifdef __cplusplus
}
#endif

#endif

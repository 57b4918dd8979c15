/*
 * hhg.h -- C ABI of the stencil-scaling operator library for MI355X (gfx950).
 *
 * The library applies the variable-coefficient P1 Darcy operator -div(k grad u)
 * with homogeneous Dirichlet data on hierarchical hybrid grids: a tetrahedral
 * macro mesh refined uniformly (Bey's rule, Sec. 2.1 of Bauer et al.,
 * "A stencil scaling approach for accelerating matrix-free finite element
 * implementations", arXiv 1709.06793).  Two discrete operators are offered:
 *   - the scaled-stencil operator a_h of eq. (discrete): off-diagonal stencil
 *     entry (k_i + k_j)/2 times the constant-coefficient reference entry, the
 *     diagonal as minus the row sum (Sec. 2.1, Sec. 6.1), optionally with the
 *     pre-asymptotic modification of Sec. 4.1 (read for 3D, see flags);
 *   - the classical nodal-integration operator of eq. (standardfe), assembled
 *     on the fly from six element matrices per macro tet (Sec. 6.2).
 * Around them: residual with norm, Jacobi / Chebyshev smoothing, geometric
 * multigrid V-cycles, FP32 V-cycles inside FP64 iterative refinement, and a
 * learned smoothing correction.
 *
 * Conventions for every call
 *   - Return value: hhg_status, 0 on success, < 0 on error (nothing is
 *     launched then), > 0 a warning.  hhg_last_error() gives the message.
 *     No C++ exception crosses this ABI.
 *   - Vectors: device pointers (hipMalloc / PyTorch CUDA memory) in the
 *     context's SLOT layout, owned by the caller.  One slot array per level:
 *     for each macro tet t (input order) a closed tetrahedral lattice of
 *     (n+1)(n+2)(n+3)/6 slots, n = 2^level, padded to a multiple of 64 slots,
 *     slot of lattice point (i,j,k) (i,j,k >= 0, i+j+k <= n) inside tet t:
 *       S(n) - S(n-k) + (i+j)(i+j+1)/2 + i,  S(m) = (m+1)(m+2)(m+3)/6,
 *     where (i,j,k) are the barycentric weights of t's vertices 1,2,3 times n
 *     (planes k in turn, inside a plane the anti-diagonals i+j in turn).
 *     A node on a macro face/edge/vertex appears in every tet holding it; input
 *     vectors must hold the same value in all copies ("consistent"), and all
 *     outputs are consistent.  Dirichlet slots (nodes on the domain boundary)
 *     must hold 0 in inputs and are written 0 in outputs; padding slots are
 *     never read.  hhg_to_canonical / hhg_from_canonical convert to and from
 *     the canonical unique-node order (from_canonical writes the 0s).
 *   - dtype selects double or float buffers (HHG_F64 / HHG_F32).
 *   - Streams: `stream` is a hipStream_t (NULL = the context's stream).  Calls
 *     are asynchronous and stream-ordered unless they return a host scalar
 *     (then they synchronise that stream).
 *   - The context owns all internal device memory; it allocates at creation
 *     and in hhg_set_coefficient only.  Calls on one context must not overlap
 *     (they share work vectors).
 *
 * Canonical node order (unique nodes, including Dirichlet nodes):
 *   1. macro vertices used by some tet, by increasing vertex id;
 *   2. macro edges {a<b} in lexicographic order, nodes by the weight s of b,
 *      s = 1..n-1;
 *   3. macro faces {a<b<c} in lexicographic order, nodes with weights
 *      (n-s-t, s, t) on (a,b,c), s,t >= 1, s+t <= n-1, t outer, s inner;
 *   4. macro tets in input order, interior nodes (i,j,k >= 1, i+j+k <= n-1),
 *      k outer, then j, then i.
 */
#ifndef HHG_H
#define HHG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hhg_status;
#define HHG_OK          0
#define HHG_EINVAL     (-1)   /* bad argument: level, dtype, null pointer, size */
#define HHG_EMESH      (-2)   /* degenerate tet, non-manifold or non-conforming macro mesh */
#define HHG_ECOEF      (-3)   /* coefficient not positive / not finite */
#define HHG_EHIP       (-4)   /* a HIP runtime call failed (message kept) */
#define HHG_ESTATE     (-5)   /* call needs state that is not there (no coefficient, no weights) */
#define HHG_ENOMEM     (-6)   /* device allocation failed */
#define HHG_WFALLBACK   1     /* warning: the learned smoother fell back to the plain one */

typedef struct hhg_ctx_s *hhg_ctx;

typedef enum { HHG_F64 = 0, HHG_F32 = 1 } hhg_dtype;
typedef enum { HHG_JACOBI = 0, HHG_CHEBYSHEV = 1, HHG_LEARNED = 2 } hhg_smoother;
typedef enum { HHG_SOLVE_F64 = 0, HHG_SOLVE_MIXED = 1, HHG_SOLVE_LEARNED = 2 } hhg_solve_mode;
/* scalar operator of hhg_solve_form */
typedef enum { HHG_FORM_SCALED = 0, HHG_FORM_NODAL = 1, HHG_FORM_MIXED = 2 } hhg_form;

/* flags of hhg_create_macro */
#define HHG_FLAG_NO_MODIFICATION 1u  /* disable the Sec. 4.1 modification (on by default) */
/* coarse-level scalar coefficients as geometric full-weighting averages of
 * the next finer level's, k_c = exp(sum_f P_fc log k_f / sum_f P_fc) with P
 * the P1 interpolation, instead of k at the coarse nodes (the default); for
 * rough coefficients given at the finest nodes only */
#define HHG_FLAG_COARSE_K_GEOMETRIC 2u

/* Build the context for a macro mesh (Sec. 2.1: macro triangulation T_H refined
 * uniformly up to max_level, 0 <= max_level <= 10).
 *   vert_xyz  host, n_vert x 3 doubles (row-major).
 *   tet_vert  host, n_tet x 4 vertex ids.  The ORDER inside a tet matters: the
 *             refinement cuts each octahedron along the line through the
 *             midpoints of edges (v0,v2) and (v1,v3) (the "gray" edge of Fig. 5).
 *   flags     HHG_FLAG_* bits.
 *   hip_stream the context's default stream (NULL = null stream).
 *   out       receives the context; NULL on failure.
 * Errors: HHG_EINVAL (null pointers, n_tet <= 0, ids out of range, level),
 * HHG_EMESH (zero-volume tet, a face shared by more than two tets,
 * a non-conforming mesh: two vertex ids at one point, a vertex on an edge or
 * face of a tet that does not hold it, overlapping coplanar boundary faces),
 * HHG_ENOMEM / HHG_EHIP.  Host setup computes, per macro tet and level, the
 * 15 primitive reference stencils (Sec. 2.2, Remark 2.1), the six element
 * matrices of the nodal kernel (Sec. 6.2) and the inter-tet node tables. */
hhg_status hhg_create_macro(const double *vert_xyz, int32_t n_vert,
                            const int32_t *tet_vert, int32_t n_tet,
                            int32_t max_level, uint32_t flags,
                            void *hip_stream, hhg_ctx *out);
hhg_status hhg_destroy(hhg_ctx ctx);
/* Message of the last error on this context (or of the last failed create when
 * ctx is NULL).  Owned by the library; valid until the next call. */
const char *hhg_last_error(hhg_ctx ctx);

/* Sizes at a level: n_slots = length of a slot vector (elements),
 * n_unknowns = non-Dirichlet unique nodes, n_nodes = all unique nodes
 * (length of a canonical vector).  Any pointer may be NULL. */
hhg_status hhg_vector_size(hhg_ctx ctx, int32_t level, int64_t *n_slots,
                           int64_t *n_unknowns, int64_t *n_nodes);
/* Coordinates of all unique nodes in canonical order into host memory
 * (n_nodes x 3 doubles), and (if not NULL) a Dirichlet flag per node. */
hhg_status hhg_node_coords(hhg_ctx ctx, int32_t level, double *xyz, uint8_t *dirichlet);

/* Convert between slot layout and canonical order at a level (device to
 * device, dtype elements).  from_canonical fills every copy of a node and
 * writes 0 to Dirichlet slots; to_canonical reads one copy per node. */
hhg_status hhg_to_canonical(hhg_ctx ctx, int32_t level, hhg_dtype dtype,
                            const void *v_slots, void *v_canon, void *stream);
hhg_status hhg_from_canonical(hhg_ctx ctx, int32_t level, hhg_dtype dtype,
                              const void *v_canon, void *v_slots, void *stream);

/* Nodal coefficient k > 0 at the finest level (max_level), canonical order,
 * double; on_device = 1 for a device pointer, 0 for host memory.  Coarser
 * levels sample k at their own nodes (the nested nodes, Sec. 2.2: k is stored
 * per node), or average it geometrically with HHG_FLAG_COARSE_K_GEOMETRIC.  Computes per level: FP32 copies, the Jacobi diagonal, the
 * Chebyshev bound, the modification corrections and the coarse-grid inverse.
 * Synchronises the stream.  Errors: HHG_ECOEF (k <= 0 or not finite). */
hhg_status hhg_set_coefficient(hhg_ctx ctx, const double *k_canonical, int on_device,
                               void *stream);

/* Coarsest multigrid level (default: the largest level with at most 4096
 * unknowns if it lies at least four levels below max_level, else the largest
 * with at most 1000; at most 4096 unknowns).  Recomputes the coarse inverse
 * (dense, FP64; on the device above 512 unknowns) if a coefficient is set. */
hhg_status hhg_set_coarse_level(hhg_ctx ctx, int32_t level);
/* Per-level solver data: Chebyshev bound of D^{-1}A (Gershgorin), number of
 * modification corrections (edges whose factor was replaced), coarse level. */
hhg_status hhg_level_info(hhg_ctx ctx, int32_t level, double *lambda_max,
                          int64_t *n_modified_edges, int32_t *coarse_level);

/* y = A u with the scaled-stencil operator (eq. (discrete), Sec. 6.1:
 * s_ij = (k_i + k_j)/2 shat_ij, s_ii = -sum_j s_ij; plus the modification of
 * Sec. 4.1 where triggered).  u, y: device slot vectors of dtype; u != y. */
hhg_status hhg_apply_scaled(hhg_ctx ctx, int32_t level, hhg_dtype dtype,
                            const void *u, void *y, void *stream);
/* Instrumentation (not part of the method): while enabled, every
 * hhg_apply_scaled times its stencil kernels with a pair of HIP events that
 * the launches themselves stamp (hipExtLaunchKernel on its stream: the start
 * at the first kernel's dispatch, the stop at the last kernel's completion;
 * the Sec. 4.1 correction kernel, if any, is outside the pair; a level without
 * stencil kernels gives an empty window).  hhg_read_timing synchronises on the
 * recorded events and returns the summed start-to-end times in ms (the stencil
 * kernels' durations, whatever else the stream runs between applies) and the
 * number of timed applies, and clears the record.  Enabling or disabling also
 * clears it.  Not for applies issued concurrently from several host threads
 * on one context. */
/* enable != 0: V-cycles inside hhg_solve, hhg_solve_form and
 * hhg_solve_tensor run as captured HIP graphs on a stream of the context
 * (each distinct level, cycle shape, operator, precision and vector pair is
 * captured once and replayed; a new coefficient, tensor coefficient or coarse
 * level starts new captures).  Cycles with the learned smoother always run
 * eagerly.  Default 0: every cycle runs eagerly on the caller's stream.  The
 * results are identical either way. */
hhg_status hhg_set_graphs(hhg_ctx ctx, int32_t enable);
hhg_status hhg_set_timing(hhg_ctx ctx, int32_t enable);
/* Tuning and tests (not part of the method): selects the variant of the
 * interior marching kernels for every context of the process; 0 (the
 * default, initial value from the environment variable HHG_MARCH_VARIANT)
 * chooses per precision and working-set size, 1..10 force one variant
 * (10: the LDS-staged FP64 scaled apply where a level fits it).  Results of
 * all variants agree to rounding.  HHG_EINVAL outside 0..10.  Not
 * thread-safe against concurrent applies. */
hhg_status hhg_set_kernel_variant(int32_t variant);
hhg_status hhg_read_timing(hhg_ctx ctx, double *ms_total, int64_t *launches);
/* y = A~ u with the nodal-integration operator (eq. (standardfe), Sec. 6.2). */
hhg_status hhg_apply_nodal(hhg_ctx ctx, int32_t level, hhg_dtype dtype,
                           const void *u, void *y, void *stream);
/* Tensor coefficient (Sec. 2.1 eq. (integral)): a(v,w) = sum_m int k_m (D_m v)(D_m w)
 * with six components D_m = c_m.grad, c_m = e_x, e_y, e_z, e_x+e_y, e_x+e_z,
 * e_y+e_z; for a symmetric K, k_i = K_ii - sum_{j!=i} K_ij (D = d/dx_i) and
 * k_ij = K_ij (D = d/dx_i + d/dx_j) give grad v . K grad w.  k6: 6 x n_nodes
 * values (component-major, canonical node order of the finest level; any
 * sign), host or device memory as for hhg_set_coefficient; coarser levels
 * take the values at their nodes.  Independent of the scalar coefficient. */
hhg_status hhg_set_tensor_coefficient(hhg_ctx ctx, const double *k6, int on_device, void *stream);
/* y = A_K u with every component scaled as the scalar operator (no Sec. 4.1
 * modification, which the paper defines for a scalar k only): row of node i =
 * sum_m sum_j (k_m(x_i) + k_m(x_j))/2 (s^m_i)_j (u_j - u_i).  Same vector
 * rules as hhg_apply_scaled; HHG_ESTATE before hhg_set_tensor_coefficient. */
hhg_status hhg_apply_tensor(hhg_ctx ctx, int32_t level, hhg_dtype dtype, const void *u, void *y,
                            void *stream);
/* y = A~_K u, the comparison form of hhg_apply_tensor: every component
 * nodally integrated (eq. (standardfe) applied to each a_m): element t
 * contributes (mean of k_m over t's vertices) times its element matrix of
 * a_m, summed over m.  Same vector rules and state requirement as
 * hhg_apply_tensor. */
hhg_status hhg_apply_tensor_nodal(hhg_ctx ctx, int32_t level, hhg_dtype dtype, const void *u, void *y,
                                  void *stream);
/* Stored stencils: the memory-bound baseline that stencil scaling avoids
 * (Sec. 6.4, the stored-stencil load model: 15 values per node).  Allocates
 * (first call; 15 FP64 + 15 FP32 values per slot of `level`) and fills the
 * rows of the interior nodes of every macro tet with the scaled operator's
 * coefficients w_d (k_i + k_{i+d}) and the centre -sum of them; the coefficient
 * must be set, and hhg_set_coefficient refreshes stored levels.  HHG_ENOMEM
 * if the allocation fails (nothing is kept then). */
hhg_status hhg_store_stencils(hhg_ctx ctx, int32_t level);
/* y = A u with the stored stencils of `level` on the interior rows (plain
 * 15-term products; inter-tet rows, Dirichlet zeros and the modification as
 * in hhg_apply_scaled).  HHG_EINVAL if the level's stencils are not stored. */
hhg_status hhg_apply_stored(hhg_ctx ctx, int32_t level, hhg_dtype dtype, const void *u, void *y,
                            void *stream);
/* y = A_I u with the primitive-mixed operator a_{h;I} (Sec. 5 eq. (modst)):
 * the row of a node on a macro primitive of a kind selected in
 * nodal_primitives (bit 0 vertices, bit 1 edges, bit 2 faces: I = W_V u W_E
 * is 3, I = W is 7) is its nodal-integration row (eq. (standardfe)); every
 * other row (tet interiors and unselected primitives) is the stencil-scaling
 * row, with the Sec. 4.1 modification where it is triggered (unless the
 * context was created with HHG_FLAG_NO_MODIFICATION).  0 gives
 * hhg_apply_scaled's result.  Same vector layout and rules as
 * hhg_apply_scaled; HHG_EINVAL for nodal_primitives outside 0..7. */
hhg_status hhg_apply_mixed(hhg_ctx ctx, int32_t level, hhg_dtype dtype, int32_t nodal_primitives,
                           const void *u, void *y, void *stream);
/* r = f - A u (scaled operator).  If norm2_out is not NULL it receives the
 * Euclidean norm of r over the unknowns (each unique node once, accumulated
 * in double) and the stream is synchronised.  r may alias neither f nor u. */
hhg_status hhg_residual(hhg_ctx ctx, int32_t level, hhg_dtype dtype, const void *f,
                        const void *u, void *r, double *norm2_out, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as hhg_residual (scaled operator, r = f - A u and the optional norm),
 * with the norm's per-block partials and its reduced value kept in a static
 * device array of the library (8 MiB per GPU, held until the process ends)
 * instead of the context's buffers.  Allocates nothing.  The context must
 * have been created with its device current (hhg_create_macro looks up that
 * device's copy of the array).  HHG_EINVAL when the level's reduction needs
 * more than the array holds (more than about 1M blocks: beyond a 48-tet mesh
 * at level 8).  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (different streams or threads) race and must not be
 * issued.  Nothing in the array needs clearing between calls. */
hhg_status hhg_residual_noalloc(hhg_ctx ctx, int32_t level, hhg_dtype dtype, const void *f,
                                const void *u, void *r, double *norm2_out, void *stream);
/* In-place smoothing of A u = f: `sweeps` steps of weighted Jacobi
 * u <- u + omega D^{-1}(f - A u) (HHG_JACOBI), or a Chebyshev polynomial of
 * degree `sweeps` in D^{-1}A on [0.1, 1] x lambda_max (HHG_CHEBYSHEV; omega
 * ignored), or `sweeps` learned steps (HHG_LEARNED, FP32 only, needs
 * weights): r = f - A u, then u <- u + D^{-1}(2/3 r + s c) with the network
 * output c and scale s of each macro-tet interior node (c = 0 elsewhere, so
 * other rows take the damped Jacobi step; omega ignored).  f, u: device slot
 * vectors. */
hhg_status hhg_smooth(hhg_ctx ctx, int32_t level, hhg_dtype dtype, hhg_smoother smoother,
                      int32_t sweeps, double omega, const void *f, void *u, void *stream);
/* One V(pre,post) cycle from `level` down to the coarse level: smoothing,
 * residual, restriction (transpose of P1 interpolation), exact coarse solve
 * (FP64), interpolation, smoothing; rediscretised coarse operators.  u is
 * updated in place.  rel_res_out (nullable): |f - A u| / |f| afterwards. */
hhg_status hhg_vcycle(hhg_ctx ctx, int32_t level, hhg_dtype dtype, int32_t pre, int32_t post,
                      hhg_smoother smoother, const void *f, void *u, double *rel_res_out,
                      void *stream);

typedef struct {
    int32_t iterations;        /* V-cycles performed (at most max_iter) */
    int32_t fallback;          /* learned smoother fell back (1) or not (0) */
    double rel_residual;       /* final |f - A u| / |f| in FP64 */
    double rho;                /* rate per V-cycle from the first FP64 residual after five
                                  cycles to the last, or the mean rate */
    double seconds;            /* wall time of the solve loop */
} hhg_solve_stats;

/* Solve A u = f at `level` to |f - A u| / |f| <= tol (FP64 residual, checked
 * after every refinement step):
 *   HHG_SOLVE_F64     FP64 V(pre,post) Chebyshev cycles;
 *   HHG_SOLVE_MIXED   FP64 residual, two FP32 V-cycles on the correction,
 *                     FP64 update (iterative refinement);
 *   HHG_SOLVE_LEARNED FP64 residual, one FP32 V-cycle with the learned smoother
 *                     on the finest level, FP64 update; falls back to Chebyshev
 *                     when the contraction worsens.
 * f, u: FP64 device slot vectors; u holds the start value and the result.
 * A residual that is not finite ends the solve (stats->rel_residual holds it).
 * Returns HHG_WFALLBACK (> 0) if the learned smoother fell back. */
hhg_status hhg_solve(hhg_ctx ctx, int32_t level, hhg_solve_mode mode, int32_t pre, int32_t post,
                     double tol, int32_t max_iter, const double *f, double *u,
                     hhg_solve_stats *stats, void *stream);

/* The same solve for the tensor-coefficient operator (Sec. 2.1 eq.
 * (integral)) of hhg_set_tensor_coefficient on every level of the cycle:
 * form 0 every component scaled (hhg_apply_tensor), form 1 every component
 * nodally integrated (hhg_apply_tensor_nodal), as the comparison of Sec. 7.
 * Chebyshev smoothing on D^{-1} A over [0.1, 1] x its Gershgorin bound, the
 * scalar solve's transfers, and a dense coarse inverse of the form (built
 * with the form's diagonals on the first call after a new tensor coefficient
 * or coarse level).  mode: HHG_SOLVE_F64 or HHG_SOLVE_MIXED (HHG_EINVAL
 * otherwise); HHG_ESTATE before hhg_set_tensor_coefficient.  The scalar
 * coefficient is not needed. */
hhg_status hhg_solve_tensor(hhg_ctx ctx, int32_t level, int32_t form, hhg_solve_mode mode, int32_t pre,
                            int32_t post, double tol, int32_t max_iter, const double *f, double *u,
                            hhg_solve_stats *stats, void *stream);

/* hhg_solve with the scalar coefficient on another discretisation of the
 * same problem on every level of the cycle (the comparison of Sec. 7):
 *   HHG_FORM_SCALED  exactly hhg_solve (all modes);
 *   HHG_FORM_NODAL   the nodal-integration operator (eq. (standardfe));
 *   HHG_FORM_MIXED   the primitive-mixed a_{h;I} of Sec. 5 eq. (modst), nodal
 *                    rows on the primitives in nodal_primitives (1 vertices,
 *                    2 edges, 4 faces; the paper's "scale Vol+Face" is 1|2).
 * The nodal and mixed forms take HHG_SOLVE_F64 or HHG_SOLVE_MIXED, smooth
 * with Chebyshev on their own diagonal and Gershgorin bound and build their
 * dense coarse inverse on first use (again after a new coefficient, coarse
 * level or primitive set).  HHG_EINVAL for other forms, modes or bits. */
hhg_status hhg_solve_form(hhg_ctx ctx, int32_t level, int32_t form, int32_t nodal_primitives,
                          hhg_solve_mode mode, int32_t pre, int32_t post, double tol, int32_t max_iter,
                          const double *f, double *u, hhg_solve_stats *stats, void *stream);

/* Learned smoothing correction (not in the paper).  Per interior node i of a
 * macro tet, a network maps the 15-point neighbourhood features
 * x_p = r_p * (1/s_i) (reciprocal rounded to FP32) and x_{15+p} = L_p - L_i
 * (p = 0: the node, p = 1..14: the neighbours in the tet-local lattice
 * directions (1,0,0), (0,1,0), (0,0,1),
 * (1,-1,0), (1,0,-1), (0,1,-1), (1,-1,1) and their negatives, in that order;
 * s_i = max_p |r_p| + 1e-30; L = log k rounded to FP32; x_30 = x_31 = 0)
 * through h1 = bf16(relu(W1 bf16(x) + b1)), h2 = relu(W2 h1 + b2),
 * c = w3 . h2 + b3 (BF16 parameters, FP32 accumulation on the matrix cores).
 * Nodes on macro faces/edges/vertices and Dirichlet nodes get c = 0.
 * A learned smoothing step is u <- u + D^{-1}(omega r + s c), omega = 2/3.
 * Parameter layout (FP32, rounded to BF16 inside):
 * W1[16][32], b1[16], W2[16][16], b2[16], w3[16], b3 (817 values).
 * The learned calls take FP32 slot vectors. */
#define HHG_LEARNED_NPARAM 817
hhg_status hhg_learned_set_weights(hhg_ctx ctx, const float *w_host, int64_t n);
/* When a learned solve (HHG_SOLVE_LEARNED) falls back to Chebyshev smoothing
 * for the rest of the solve.  A learned cycle is rejected when its residual
 * ratio is not finite, exceeds max_rate (default 1), or exceeds
 * plain_margin x the plain cycle's ratio (default 1.05; 0 turns this test
 * off).  The plain ratio is measured once per solve: at cycle 2 a Chebyshev
 * cycle runs from the same iterate as the learned one (one extra cycle); if
 * the learned cycle then loses, the solve keeps the plain cycle's result,
 * otherwise a rejected cycle's result is discarded.  HHG_EINVAL for
 * max_rate <= 0 or a negative or non-finite margin. */
hhg_status hhg_learned_set_fallback(hhg_ctx ctx, double max_rate, double plain_margin);
/* c_out[slot] = network output c_i (consistent FP32 slot vector). */
hhg_status hhg_learned_forward(hhg_ctx ctx, int32_t level, const float *r, float *c_out,
                               void *stream);
/* Gradient of sum_i g_i c_i with respect to the 817 parameters into host
 * memory dw_host (BF16 roundings of x and h1 taken as identities); g is an
 * FP32 slot vector.  Synchronises the stream. */
hhg_status hhg_learned_backward(hhg_ctx ctx, int32_t level, const float *r, const float *g,
                                float *dw_host, void *stream);
/* One training sample (r = A e): loss L = e1^T A e1 / e^T A e of the error
 * e1 = e - D^{-1}(omega r + s c) after one learned step, and dL/dparameters
 * into dw_host.  Synchronises the stream. */
hhg_status hhg_learned_loss_grad(hhg_ctx ctx, int32_t level, const float *r, const float *e,
                                 double *loss_out, float *dw_host, void *stream);
/* r_out = (float)(f - A u), e_out = (float)(u_star - u): a training pair from
 * FP64 slot vectors. */
hhg_status hhg_training_pair(hhg_ctx ctx, int32_t level, const double *f, const double *u,
                             const double *u_star, float *r_out, float *e_out, void *stream);
/* Host-side Adam step (Kingma and Ba) on n parameters: w, m, v updated in
 * place from gradient g at step t >= 1. */
hhg_status hhg_adam_update(float *w, float *m, float *v, const float *g, int64_t n, int32_t t,
                           double lr, double beta1, double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif /* HHG_H */

// hhg_internal.h -- device-side views of one refinement level and the kernel
// launchers the host driver calls.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hhg {

constexpr int BLOCK = 256;
constexpr int KIND_STRIDE = 16;                // entries per (tet, kind) stencil row
constexpr int TET_STENCIL = 16 * KIND_STRIDE;  // 16 kinds (15 used) per tet
constexpr int TET_EMAT = 6 * 16;               // six 4x4 element matrices per tet

// Everything a kernel needs about one level, for one precision T.
template <typename T>
struct LevelView {
    int n;          // intervals per macro edge (2^level)
    int n_tet;
    int S;          // slots of one closed tet lattice
    int64_t Spad;   // slots per tet in memory (multiple of 64)
    int bpt;        // 256-slot blocks per tet (flat kernels)
    // interior rows by column marching: wave work items (first in-plane
    // offset, k0 | k1 << 16), 4 per block; boundary slots (slot << 4 | kind)
    const uint2 *items;
    int n_items;
    int vpt;        // marching blocks per tet
    // the same for the two-rows-per-lane kernel (first row offset of 126)
    const uint2 *items2;
    int n_items2;
    int vpt2;
    // block items of the LDS-staged kernel (8 waves: first row offset of
    // 1008 consecutive offsets, k0 | k1 << 16); 0 when the level is too large
    const uint2 *itemsL;
    int n_itemsL;
    const uint32_t *bnd;
    int n_bnd;
    int bpt2;       // boundary blocks per tet
    const T *sten;          // [tet][16 kinds][16]: entries 0..13 = half reference entry per direction
    const T *emat;          // [tet][6 types][4][4]: element matrices / 4 (nodal kernel)
    const T *rstw;          // [tet][16 kinds][16]: restriction weights (0..13 dirs, 14 centre)
    const uint16_t *dmask;  // [tet]: bit = kind is on the Dirichlet boundary
    const uint16_t *smask;  // [tet]: bit = kind is shared with another tet (not Dirichlet)
    const T *kap;           // nodal coefficient, slot layout
    // unique nodes on inter-tet primitives: copies of node q are
    // sh_copy[sh_off[q] .. sh_off[q+1]) (packed tet, kind, i, j, k)
    int n_shared;
    const int32_t *sh_off;
    const uint64_t *sh_copy;
    // rows of the shared nodes as merged neighbour lists (ELL, entry m of
    // node q at m * n_shared + q; padding entries: coefficient 0, neighbour
    // = the node itself): row_q = sum_m c_m (u[sh_nb] - u[sh_self])
    int sh_w;
    const int64_t *sh_nb;     // global slot (tet * Spad + slot) of the neighbour
    const int64_t *sh_self;   // global slot of the node's first copy
    const int64_t *sh_cslot;  // global slot of every copy (sh_off order)
    // the same three (and sh_nbs below) as 32-bit slots when every global
    // slot of the level fits (null otherwise): the row kernel then streams 4
    // instead of 8 bytes per index
    const uint32_t *sh_nb32, *sh_self32, *sh_cslot32, *sh_nbs32;
    const T *sh_cs;           // scaled-operator coefficients
    const T *sh_cn;           // nodal-operator coefficients
    const uint8_t *sh_prim;   // macro primitive of node q: 1 vertex, 2 edge, 4 face
    // the scaled operator alone: the entries of the pattern above whose
    // scaled weight is not negligible (on Kuhn meshes 6 of the 14 entries
    // of a face node), same layout, with that operator's coefficients
    int sh_ws;
    const int64_t *sh_nbs;
    const T *sh_css;
    // tensor operator: its own (wider) pattern sh_wt / sh_nbt in the same
    // layout, coefficients with every component scaled (sh_ct) or nodally
    // integrated (sh_ctn)
    int sh_wt;
    const int64_t *sh_nbt;
    const T *sh_ct;
    const T *sh_ctn;
    // tensor operator: [tet][6 components][16 kinds][16] half reference entries
    // of the components D_m = c_m.grad, and the six coefficient fields
    // (component m at kt + m * n_tet * Spad), null until set
    const T *tsten;
    const T *kt;
    // the same operator's interior rows as seven direction-pair fields per
    // slot, K_p = sum_m w^m_p k_m with the tet's interior weights (pair p =
    // directions p and p + 7, whose interior weights agree): pair p at
    // kp + p * n_tet * Spad
    const T *kp;
    // [tet][6 components][6 types][4][4]: element matrices of the components / 4
    // (nodal-integration tensor operator)
    const T *temat;
};

// sparse corrections of the modification (Sec. 4.1) at one level
template <typename T>
struct CorrView {
    int n_rows;               // corrected unique rows
    const int32_t *c_off;     // corrections of row q: [c_off[q], c_off[q+1])
    const int64_t *c_self;    // slot of the row's node in the edge's tet
    const int64_t *c_nb;      // slot of the other end of the edge
    const T *c_delta;         // (k_mod - k_e) * reference entry of the edge in that tet
    const double *c_base;     // unmodified entry (k_e * reference entry), FP64
    const uint8_t *c_nbdir;   // 1 if the other end is a Dirichlet node
    const int32_t *p_off;     // copies of row q: [p_off[q], p_off[q+1])
    const int64_t *p_slot;
    const uint8_t *c_prim;    // macro primitive of the row's node (1/2/4 as sh_prim; 0 tet interior)
};

// kernel launchers (hhg_kernels.hip); every launcher returns hipGetLastError()
enum ApplyMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_CHEB = 2 };

// one fused Chebyshev sweep: with r = f - A u (modification included),
// d <- c_old d + c_r D^{-1} r (d taken as 0 when `first`) and u_new = u + d
template <typename T>
struct ChebArgs {
    // direction of the fused sweep: read only at a row's own slot (interior
    // rows) or at the first copy of a shared node (the inter-tet and
    // modification rows both take sh_off order), so a shared node's other
    // copies of d are not kept up to date
    T *d = nullptr;
    const T *invd = nullptr;
    T c_old = T(0), c_r = T(0);
    int first = 0;
};

template <typename T>
hipError_t launch_scaled(const LevelView<T> &L, int mode, const T *u, const T *f, T *y,
                         double *partial, int *n_partial, hipStream_t st);
template <typename T>
hipError_t launch_nodal(const LevelView<T> &L, const T *u, T *y, hipStream_t st);
// stored stencils (the baseline the method avoids: 15 weights per interior
// row, weight-major per tet, st[(tet * 15 + d) * Spad + slot], d < 14 the
// directions, 14 the centre) from the scaled operator's coefficients, and the
// apply that streams them
template <typename T>
hipError_t launch_store_stencils(const LevelView<double> &L, T *st, hipStream_t strm);
template <typename T>
hipError_t launch_stored(const LevelView<T> &L, const CorrView<T> &C, const T *st, const T *u, T *y,
                         hipStream_t strm);
// direction-pair fields K_p of the tensor operator from its component fields
hipError_t launch_tensor_pairs(const LevelView<double> &L, double *kp, hipStream_t st);
// merged shared-row coefficients of both tensor forms
hipError_t launch_tensor_shared_coef(const LevelView<double> &L, const int8_t *map, double *cs, double *cn,
                                     hipStream_t st);
// tensor-coefficient operator (Sec. 2.1 eq. (integral)) with every component
// scaled (form 0) or nodally integrated (form 1, eq. (standardfe) per
// component): interior rows, inter-tet rows (merged coefficients) and
// Dirichlet zeros.  mode MODE_APPLY: y = A u; MODE_RESID: y = f - A u with
// per-block sums of squares in partial[0 .. *n_partial)
template <typename T>
hipError_t launch_tensor(const LevelView<T> &L, int form, int mode, const T *u, const T *f, T *y, double *partial,
                         int *n_partial, hipStream_t st);
// partial entries launch_tensor (MODE_RESID) and launch_tensor_diag produce
int tensor_partial_count(int n, int n_tet, int n_shared);
// diagonal of a form (0 scaled tensor, 1 nodal tensor, 2 scalar nodal: all
// interior and shared rows; 3: only the shared rows on the primitives in
// mask, with nodal coefficients) and per-block Gershgorin maxima of D^{-1} A
// in partial[0 .. *n_partial); other slots untouched
hipError_t launch_form_diag(const LevelView<double> &L, int form, int mask, double *diag, double *partial,
                            int *n_partial, hipStream_t st);
// one fused Chebyshev sweep (as launch_cheb_sweep) of the primitive-mixed form
template <typename T>
hipError_t launch_cheb_sweep_mixed(const LevelView<T> &L, const CorrView<T> &C, int nodal_mask, const T *u,
                                   const T *f, T *u_new, const ChebArgs<T> &cb, hipStream_t st);
// the scalar nodal form (form 1) or the primitive-mixed form (form 2) in
// MODE_APPLY or MODE_RESID (per-block sums of squares in partial)
template <typename T>
hipError_t launch_scalar_form(const LevelView<T> &L, const CorrView<T> &C, int form, int mode, int nodal_mask,
                              const T *u, const T *f, T *y, double *partial, int *n_partial, hipStream_t st);
// the primitive-mixed operator (Sec. 5 eq. (modst)): nodal-integration rows
// for the nodes of the primitives in nodal_mask (1 vertices, 2 edges, 4
// faces), scaled rows (with their modification corrections) elsewhere
template <typename T>
hipError_t launch_mixed(const LevelView<T> &L, const CorrView<T> &C, const T *u, T *y, int nodal_mask,
                        hipStream_t st);
// fused Chebyshev sweep (interior march, shared rows, modification rows):
// reads u, f, d, D^{-1}; writes d and u_new (every slot of u_new: rows,
// copies, Dirichlet zeros).  u_new must not alias u.
template <typename T>
hipError_t launch_cheb_sweep(const LevelView<T> &L, const CorrView<T> &C, const T *u, const T *f, T *u_new,
                             const ChebArgs<T> &cb, hipStream_t st);
template <typename T>
hipError_t launch_correction(const LevelView<T> &L, const CorrView<T> &C, int mode, const T *u,
                             T *y, double *partial, hipStream_t st);
// D (diagonal, not inverted) into d; per-slot Gershgorin absolute row sums
// into asum (nullable); block maxima of the volume rows' ratios into partial
// (n_partial of them); (asum, D) per shared node into gabs
template <typename T>
hipError_t launch_diag(const LevelView<T> &L, T *d, double *asum, double *partial, double *gabs,
                       int *n_partial, hipStream_t st);
hipError_t launch_reduce(const double *partial, int n, int op_max, double *out, hipStream_t st);

template <typename T>
hipError_t launch_invert_diag(T *d, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_jacobi_update(T *u, const T *r, const T *invd, T omega, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_cheb_update(T *u, T *dvec, const T *r, const T *invd, T c_old, T c_r,
                              int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_restrict(const LevelView<T> &Lc, const LevelView<T> &Lf, const T *rf, T *rc,
                           hipStream_t st);
template <typename T>
hipError_t launch_prolong_add(const LevelView<T> &Lc, const LevelView<T> &Lf, const T *uc, T *uf,
                              hipStream_t st);
template <typename T>
hipError_t launch_coarse_solve(const double *ainv, int nu, const int64_t *gather,
                               const int32_t *copy_off, const int64_t *copy_slot, const T *f, T *u,
                               double *fc, hipStream_t st);
template <typename T>
hipError_t launch_fill(T *x, T v, int64_t n, hipStream_t st);
template <typename Ti, typename To>
hipError_t launch_convert(const Ti *in, To *out, int64_t n, hipStream_t st);
// kernel variant of the interior marches (0 = default policy); -1 if out of range
int set_march_variant(int v);
// the interior kernels' variant in force (0 = per precision and size)
int march_variant_now();
// timed applies: the stencil launches of the calling thread take these
// events (start at the first kernel's dispatch, stop at the last kernel's
// completion) until they are cleared with nullptrs; true while the start
// event has not been taken by a launch
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_unused();
// merged coefficients of the shared rows for the current k (scaled and nodal)
hipError_t launch_shared_coef(const LevelView<double> &L, const int8_t *map, double *cs, double *cn,
                              hipStream_t st);
hipError_t launch_shared_coef_scaled(const LevelView<double> &L, const int8_t *map, double *cs, hipStream_t st);
// inverse of the n x n matrix in the left half of work ([A | I], n x 2n,
// row-major; overwritten) into ainv; iscr: 2 ints (iscr[1] = 1 afterwards if
// A is singular; the caller clears it), dscr: n + 1 doubles
hipError_t launch_dense_inverse(double *work, int n, double *ainv, int *iscr, double *dscr, hipStream_t st);
hipError_t launch_add_f32_to_f64(double *u, const float *c, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_inject(const T *kf, int nf, T *kc, int nc, int n_tet, int64_t Spad_f,
                         int64_t Spad_c, hipStream_t st);
// coarse k as geometric full-weighting averages of the finer level's k
// (macro-tet interior nodes from the tet's own fine lattice, the n_list
// nodes on macro primitives from their support lists)
hipError_t launch_coarsen(const double *kf, int nf, double *kc, int nc, int n_tet, int64_t Spad_f, int64_t Spad_c,
                          int n_list, const int32_t *off, const int64_t *fslot, const double *w,
                          const int32_t *coff, const int64_t *cslot, hipStream_t st);
template <typename T>
hipError_t launch_from_canonical(const T *canon, const int32_t *slot2canon, T *slots, int64_t n,
                                 int keep_dirichlet, int S, int64_t Spad, hipStream_t st);
template <typename T>
hipError_t launch_to_canonical(const T *slots, const int64_t *canon2slot, T *canon, int64_t n,
                               hipStream_t st);
hipError_t launch_positive_check(const double *k, int64_t n, int *bad, hipStream_t st);

}  // namespace hhg

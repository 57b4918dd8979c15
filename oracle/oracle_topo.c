/*
 * oracle_topo.c -- topology half of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file (through oracle/oracle.py).  The product
 * library shares no code, header or table with it.
 *
 * What it does (and nothing more): refine every macro tetrahedron of a
 * simplicial macro mesh uniformly by Bey's rule (the refinement the paper's
 * section 2.1 cites for the 3D case) and give every node of the refined mesh a
 * canonical number.  All arithmetic of the method (element matrices, the
 * scaled and nodal forms, solvers) lives in oracle.py; this file is integer
 * only, so the refined mesh is exact.
 *
 * Node representation.  A node of macro tet t at refinement level L (N = 2^L)
 * is the integer barycentric 4-vector w (w_0+..+w_3 = N) with respect to t's
 * vertices in the order the caller gave them.  Two representations of the same
 * point in different macro tets are identified through the macro vertices with
 * non-zero weight, so the numbering is exact and independent of the tet.
 *
 * Canonical order (the interface shared with the product library; both sides
 * implement it independently):
 *   1. macro vertices that some tet uses, by increasing vertex id;
 *   2. macro edges {a<b} in lexicographic order; nodes by the weight s of b,
 *      s = 1..N-1;
 *   3. macro faces {a<b<c} in lexicographic order; nodes with weights
 *      (N-s-t, s, t) on (a, b, c), s,t >= 1, s+t <= N-1, t outer, s inner;
 *   4. macro tets in input order; interior nodes with tet-local lattice
 *      coordinates (i,j,k) = (w_1,w_2,w_3), i,j,k >= 1, i+j+k <= N-1, k outer,
 *      then j, then i.
 * A node is a Dirichlet node iff it lies on a macro face that belongs to one
 * tet only (the domain boundary), including edges and vertices of such faces.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nv, nt, L, N;
    double *X;            /* nv*3 vertex coordinates */
    int *tet;             /* nt*4 vertex ids, caller's order */
    int nvu;              /* number of used vertices */
    int *vpos;            /* vertex id -> canonical index or -1 */
    int ne;
    int *edge;            /* ne*2, a<b, sorted */
    int nf;
    int *face;            /* nf*3, a<b<c, sorted */
    int *face_ntet;
    uint8_t *v_bnd, *e_bnd, *f_bnd;
    int64_t EN, FN, TN;   /* interior nodes per edge / face / tet */
    int64_t off_e, off_f, off_t, n_nodes;
    int64_t *plane_off;   /* tet-interior prefix counts per k plane */
} OMesh;

/* ------------------------------------------------------------------ */
static int cmp_int2(const void *a, const void *b)
{
    const int *x = a, *y = b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}
static int cmp_int3(const void *a, const void *b)
{
    const int *x = a, *y = b;
    for (int i = 0; i < 3; ++i)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}
static void sort_small(int *v, int *w, int c)
{
    for (int i = 1; i < c; ++i)
        for (int j = i; j > 0 && v[j - 1] > v[j]; --j) {
            int t = v[j]; v[j] = v[j - 1]; v[j - 1] = t;
            if (w) { t = w[j]; w[j] = w[j - 1]; w[j - 1] = t; }
        }
}
static int find_edge(const OMesh *m, int a, int b)
{
    int key[2] = {a, b};
    int *p = bsearch(key, m->edge, m->ne, 2 * sizeof(int), cmp_int2);
    return p ? (int)((p - m->edge) / 2) : -1;
}
static int find_face(const OMesh *m, int a, int b, int c)
{
    int key[3] = {a, b, c};
    int *p = bsearch(key, m->face, m->nf, 3 * sizeof(int), cmp_int3);
    return p ? (int)((p - m->face) / 3) : -1;
}

/* ------------------------------------------------------------------ */
void om_destroy(OMesh *m)
{
    if (!m) return;
    free(m->X); free(m->tet); free(m->vpos); free(m->edge); free(m->face);
    free(m->face_ntet); free(m->v_bnd); free(m->e_bnd); free(m->f_bnd);
    free(m->plane_off); free(m);
}

OMesh *om_create(const double *X, int nv, const int *tet, int nt, int L)
{
    if (nv <= 0 || nt <= 0 || L < 0 || L > 12) return NULL;
    OMesh *m = calloc(1, sizeof(OMesh));
    m->nv = nv; m->nt = nt; m->L = L; m->N = 1 << L;
    m->X = malloc(sizeof(double) * 3 * nv);
    memcpy(m->X, X, sizeof(double) * 3 * nv);
    m->tet = malloc(sizeof(int) * 4 * nt);
    memcpy(m->tet, tet, sizeof(int) * 4 * nt);
    for (int i = 0; i < 4 * nt; ++i)
        if (tet[i] < 0 || tet[i] >= nv) { om_destroy(m); return NULL; }

    /* used vertices */
    m->vpos = malloc(sizeof(int) * nv);
    for (int i = 0; i < nv; ++i) m->vpos[i] = -1;
    for (int i = 0; i < 4 * nt; ++i) m->vpos[tet[i]] = 1;
    m->nvu = 0;
    for (int i = 0; i < nv; ++i)
        if (m->vpos[i] == 1) m->vpos[i] = m->nvu++;

    /* edges and faces with duplicates, then sort + unique */
    int *E = malloc(sizeof(int) * 12 * nt), *F = malloc(sizeof(int) * 12 * nt);
    static const int ep[6][2] = {{0,1},{0,2},{0,3},{1,2},{1,3},{2,3}};
    static const int fp[4][3] = {{1,2,3},{0,2,3},{0,1,3},{0,1,2}};
    for (int t = 0; t < nt; ++t) {
        for (int e = 0; e < 6; ++e) {
            int v[2] = {tet[4*t+ep[e][0]], tet[4*t+ep[e][1]]};
            sort_small(v, NULL, 2);
            E[12*t+2*e] = v[0]; E[12*t+2*e+1] = v[1];
        }
        for (int f = 0; f < 4; ++f) {
            int v[3] = {tet[4*t+fp[f][0]], tet[4*t+fp[f][1]], tet[4*t+fp[f][2]]};
            sort_small(v, NULL, 3);
            memcpy(F + 12*t + 3*f, v, sizeof v);
        }
    }
    qsort(E, 6 * nt, 2 * sizeof(int), cmp_int2);
    qsort(F, 4 * nt, 3 * sizeof(int), cmp_int3);
    m->edge = malloc(sizeof(int) * 12 * nt);
    m->ne = 0;
    for (int i = 0; i < 6 * nt; ++i)
        if (i == 0 || cmp_int2(E + 2*i, E + 2*(i-1)) != 0) {
            memcpy(m->edge + 2*m->ne, E + 2*i, 2 * sizeof(int)); m->ne++;
        }
    m->face = malloc(sizeof(int) * 12 * nt);
    m->face_ntet = calloc(4 * nt, sizeof(int));
    m->nf = 0;
    for (int i = 0; i < 4 * nt; ++i) {
        if (i == 0 || cmp_int3(F + 3*i, F + 3*(i-1)) != 0) {
            memcpy(m->face + 3*m->nf, F + 3*i, 3 * sizeof(int)); m->nf++;
        }
        m->face_ntet[m->nf - 1]++;
    }
    free(E); free(F);
    for (int f = 0; f < m->nf; ++f)
        if (m->face_ntet[f] > 2) { om_destroy(m); return NULL; }  /* non-manifold */

    /* boundary flags: faces with one tet, and their edges / vertices */
    m->v_bnd = calloc((size_t)nv, 1);
    m->e_bnd = calloc((size_t)(m->ne > 0 ? m->ne : 1), 1);
    m->f_bnd = calloc((size_t)(m->nf > 0 ? m->nf : 1), 1);
    for (int f = 0; f < m->nf; ++f) {
        if (m->face_ntet[f] != 1) continue;
        m->f_bnd[f] = 1;
        const int *v = m->face + 3*f;
        for (int a = 0; a < 3; ++a) {
            m->v_bnd[v[a]] = 1;
            for (int b = a + 1; b < 3; ++b) m->e_bnd[find_edge(m, v[a], v[b])] = 1;
        }
    }

    int64_t N = m->N;
    m->EN = N - 1;
    m->FN = (N - 1) * (N - 2) / 2;
    m->TN = (N - 1) * (N - 2) * (N - 3) / 6;
    m->off_e = m->nvu;
    m->off_f = m->off_e + (int64_t)m->ne * m->EN;
    m->off_t = m->off_f + (int64_t)m->nf * m->FN;
    m->n_nodes = m->off_t + (int64_t)nt * m->TN;

    /* plane_off[k] = number of tet-interior nodes with plane index < k */
    m->plane_off = calloc(N + 2, sizeof(int64_t));
    for (int64_t k = 1; k <= N; ++k) {
        int64_t M = N - 1 - k;            /* i+j <= M with i,j >= 1 */
        int64_t cnt = (k <= N - 3 && M >= 2) ? (M - 1) * M / 2 : 0;
        m->plane_off[k + 1] = m->plane_off[k] + cnt;
    }
    return m;
}

int64_t om_n_nodes(const OMesh *m) { return m->n_nodes; }
int om_level(const OMesh *m) { return m->L; }

/* canonical index of the node with barycentric weights w in macro tet t */
static int64_t canon(const OMesh *m, int t, const int w[4])
{
    int vid[4], ww[4], c = 0;
    for (int a = 0; a < 4; ++a)
        if (w[a] > 0) { vid[c] = m->tet[4*t + a]; ww[c] = w[a]; ++c; }
    if (c == 4) {
        int64_t i = w[1], j = w[2], k = w[3], M = m->N - 1 - k;
        int64_t loc = m->plane_off[k];
        for (int64_t jj = 1; jj < j; ++jj) loc += M - jj;
        return m->off_t + (int64_t)t * m->TN + loc + (i - 1);
    }
    sort_small(vid, ww, c);
    if (c == 1) return m->vpos[vid[0]];
    if (c == 2) {
        int e = find_edge(m, vid[0], vid[1]);
        return m->off_e + (int64_t)e * m->EN + (ww[1] - 1);
    }
    /* c == 3 */
    int f = find_face(m, vid[0], vid[1], vid[2]);
    int64_t s = ww[1], tt = ww[2];
    int64_t loc = (tt - 1) * (m->N - 1) - (tt - 1) * tt / 2 + (s - 1);
    return m->off_f + (int64_t)f * m->FN + loc;
}

/* coordinates and Dirichlet flag of every node, in canonical order */
void om_node_info(const OMesh *m, double *xyz, uint8_t *dirichlet)
{
    const int N = m->N;
    for (int t = 0; t < m->nt; ++t) {
        const int *tv = m->tet + 4*t;
        for (int k = 0; k <= N; ++k)
            for (int j = 0; j + k <= N; ++j)
                for (int i = 0; i + j + k <= N; ++i) {
                    int w[4] = {N - i - j - k, i, j, k};
                    int64_t c = canon(m, t, w);
                    for (int d = 0; d < 3; ++d) {
                        double s = 0.0;
                        for (int a = 0; a < 4; ++a)
                            s += (double)w[a] / (double)N * m->X[3*tv[a] + d];
                        xyz[3*c + d] = s;
                    }
                    /* which primitive: count non-zero weights */
                    int vid[4], c0 = 0;
                    for (int a = 0; a < 4; ++a) if (w[a] > 0) vid[c0++] = tv[a];
                    sort_small(vid, NULL, c0);
                    uint8_t b = 0;
                    if (c0 == 1) b = m->v_bnd[vid[0]];
                    else if (c0 == 2) b = m->e_bnd[find_edge(m, vid[0], vid[1])];
                    else if (c0 == 3) b = m->f_bnd[find_face(m, vid[0], vid[1], vid[2])];
                    dirichlet[c] = b;
                }
    }
}

/* ---------------- Bey refinement ---------------- */
typedef struct {
    const OMesh *m;
    int t;
    int64_t count, cap;
    int32_t *conn;        /* emitted elements: canonical vertex ids */
    int32_t *macro;
    int32_t *bary;        /* optional: emitted barycentric vertex vectors (16 ints) */
    int restrict_on;      /* only keep elements whose closure holds point p */
    int p[4];
    int fine_index;       /* if set, emit canonical ids of a mesh at level L+1 */
    const OMesh *fine;
} Emit;

/* exact closed-containment test of lattice point p in tet q (integer bary) */
static int64_t det3(const int64_t a[3], const int64_t b[3], const int64_t c[3])
{
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
         + a[2] * (b[0] * c[1] - b[1] * c[0]);
}
static int contains(const int q[4][4], const int p[4])
{
    int64_t c1[3], c2[3], c3[3], r[3];
    for (int d = 0; d < 3; ++d) {
        c1[d] = q[1][d + 1] - q[0][d + 1];
        c2[d] = q[2][d + 1] - q[0][d + 1];
        c3[d] = q[3][d + 1] - q[0][d + 1];
        r[d]  = p[d + 1] - q[0][d + 1];
    }
    int64_t D = det3(c1, c2, c3);
    if (D == 0) return 0;
    int64_t d1 = det3(r, c2, c3), d2 = det3(c1, r, c3), d3 = det3(c1, c2, r);
    int64_t s = D > 0 ? 1 : -1;
    return s * d1 >= 0 && s * d2 >= 0 && s * d3 >= 0 && s * (D - d1 - d2 - d3) >= 0;
}

static void emit(Emit *E, int q[4][4])
{
    if (E->count >= E->cap) { E->count++; return; }
    for (int a = 0; a < 4; ++a) E->conn[4 * E->count + a] = (int32_t)canon(E->m, E->t, q[a]);
    if (E->macro) E->macro[E->count] = E->t;
    if (E->bary)
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) E->bary[16 * E->count + 4 * a + c] = q[a][c];
    E->count++;
}

/* Bey's rule: children of [x0,x1,x2,x3] with xab the edge midpoints are
 * [x0,x01,x02,x03], [x01,x1,x12,x13], [x02,x12,x2,x23], [x03,x13,x23,x3],
 * and the octahedron cut along x02-x13:
 * [x01,x02,x03,x13], [x01,x02,x12,x13], [x02,x03,x13,x23], [x02,x12,x13,x23]. */
static void refine(Emit *E, int q[4][4], int depth)
{
    if (E->restrict_on && !contains((const int (*)[4])q, E->p)) return;
    if (depth == E->m->L) { emit(E, q); return; }
    int x[4][4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) x[a][b][c] = (q[a][c] + q[b][c]) / 2;
    static const int ch[8][4][2] = {
        {{0,0},{0,1},{0,2},{0,3}}, {{0,1},{1,1},{1,2},{1,3}},
        {{0,2},{1,2},{2,2},{2,3}}, {{0,3},{1,3},{2,3},{3,3}},
        {{0,1},{0,2},{0,3},{1,3}}, {{0,1},{0,2},{1,2},{1,3}},
        {{0,2},{0,3},{1,3},{2,3}}, {{0,2},{1,2},{1,3},{2,3}}};
    for (int c = 0; c < 8; ++c) {
        int qc[4][4];
        for (int a = 0; a < 4; ++a) memcpy(qc[a], x[ch[c][a][0]][ch[c][a][1]], sizeof qc[a]);
        refine(E, qc, depth + 1);
    }
}

static void run_all(Emit *E)
{
    const int N = E->m->N;
    for (int t = 0; t < E->m->nt; ++t) {
        int q[4][4] = {{N,0,0,0},{0,N,0,0},{0,0,N,0},{0,0,0,N}};
        E->t = t;
        refine(E, q, 0);
    }
}

int64_t om_n_elements(const OMesh *m)
{
    return (int64_t)m->nt << (3 * m->L);
}

/* all elements of the refined mesh: canonical vertex ids and the macro tet */
int64_t om_elements(const OMesh *m, int32_t *conn, int32_t *macro)
{
    Emit E = {0};
    E.m = m; E.conn = conn; E.macro = macro; E.cap = om_n_elements(m);
    run_all(&E);
    return E.count;
}

/* same, also returning the integer barycentric vertex vectors (16 per element) */
int64_t om_elements_bary(const OMesh *m, int32_t *conn, int32_t *macro, int32_t *bary)
{
    Emit E = {0};
    E.m = m; E.conn = conn; E.macro = macro; E.bary = bary; E.cap = om_n_elements(m);
    run_all(&E);
    return E.count;
}

/* one (macro tet, barycentric) representation of canonical node c */
static int node_repr(const OMesh *m, int64_t c, int *t_out, int w[4])
{
    const int N = m->N;
    int vid[4], ww[4], cnt = 0;
    if (c < 0 || c >= m->n_nodes) return -1;
    if (c < m->off_e) {
        for (int v = 0; v < m->nv; ++v)
            if (m->vpos[v] == c) { vid[0] = v; ww[0] = N; cnt = 1; break; }
    } else if (c < m->off_f) {
        int64_t e = (c - m->off_e) / m->EN, s = (c - m->off_e) % m->EN + 1;
        vid[0] = m->edge[2*e]; vid[1] = m->edge[2*e+1];
        ww[0] = N - (int)s; ww[1] = (int)s; cnt = 2;
    } else if (c < m->off_t) {
        int64_t f = (c - m->off_f) / m->FN, loc = (c - m->off_f) % m->FN;
        int64_t tt = 1;
        while (loc >= (N - 1 - tt)) { loc -= (N - 1 - tt); ++tt; }
        int64_t s = loc + 1;
        vid[0] = m->face[3*f]; vid[1] = m->face[3*f+1]; vid[2] = m->face[3*f+2];
        ww[0] = N - (int)s - (int)tt; ww[1] = (int)s; ww[2] = (int)tt; cnt = 3;
    } else {
        int64_t t = (c - m->off_t) / m->TN, loc = (c - m->off_t) % m->TN;
        int64_t k = 1;
        while (m->plane_off[k + 1] <= loc) ++k;
        loc -= m->plane_off[k];
        int64_t M = N - 1 - k, j = 1;
        while (loc >= M - j) { loc -= M - j; ++j; }
        int64_t i = loc + 1;
        *t_out = (int)t;
        w[0] = N - (int)(i + j + k); w[1] = (int)i; w[2] = (int)j; w[3] = (int)k;
        return 0;
    }
    /* find a tet holding all vertices of the primitive */
    for (int t = 0; t < m->nt; ++t) {
        int ok = 1, loc[4];
        for (int a = 0; a < cnt && ok; ++a) {
            loc[a] = -1;
            for (int b = 0; b < 4; ++b) if (m->tet[4*t+b] == vid[a]) loc[a] = b;
            if (loc[a] < 0) ok = 0;
        }
        if (!ok) continue;
        *t_out = t;
        w[0] = w[1] = w[2] = w[3] = 0;
        for (int a = 0; a < cnt; ++a) w[loc[a]] = ww[a];
        return 0;
    }
    return -1;
}

/* every element of the refined mesh whose closure holds node c (restricted
 * refinement: only children containing the point are refined further).
 * Returns the number found (may exceed cap; then only cap are stored). */
int64_t om_incident(const OMesh *m, int64_t c, int32_t *conn, int32_t *macro, int64_t cap)
{
    int t0, w0[4];
    if (node_repr(m, c, &t0, w0) != 0) return -1;
    /* the physical point, as macro vertices with weights */
    int vid[4], ww[4], cnt = 0;
    for (int a = 0; a < 4; ++a)
        if (w0[a] > 0) { vid[cnt] = m->tet[4*t0+a]; ww[cnt] = w0[a]; ++cnt; }
    Emit E = {0};
    E.m = m; E.conn = conn; E.macro = macro; E.cap = cap; E.restrict_on = 1;
    const int N = m->N;
    for (int t = 0; t < m->nt; ++t) {
        int w[4] = {0, 0, 0, 0}, ok = 1;
        for (int a = 0; a < cnt && ok; ++a) {
            int l = -1;
            for (int b = 0; b < 4; ++b) if (m->tet[4*t+b] == vid[a]) l = b;
            if (l < 0) ok = 0; else w[l] = ww[a];
        }
        if (!ok) continue;
        memcpy(E.p, w, sizeof w);
        E.t = t;
        int q[4][4] = {{N,0,0,0},{0,N,0,0},{0,0,N,0},{0,0,0,N}};
        refine(&E, q, 0);
    }
    return E.count;
}

/* canonical index at level L+1 (mesh `fine`) of every canonical node of `m` */
void om_coarse_to_fine(const OMesh *m, const OMesh *fine, int64_t *map)
{
    const int N = m->N;
    for (int t = 0; t < m->nt; ++t)
        for (int k = 0; k <= N; ++k)
            for (int j = 0; j + k <= N; ++j)
                for (int i = 0; i + j + k <= N; ++i) {
                    int w[4] = {N - i - j - k, i, j, k};
                    int w2[4] = {2 * w[0], 2 * w[1], 2 * w[2], 2 * w[3]};
                    map[canon(m, t, w)] = canon(fine, t, w2);
                }
}

/* P1 prolongation from level L (`m`) to level L+1 (`fine`) as triplets
 * (fine row, coarse col, weight): coarse vertices keep their value, the
 * midpoint of every coarse edge takes half of each end.  Duplicates (the same
 * pair found through several coarse elements) are emitted again; the caller
 * keeps one.  Returns the number of triplets written (16 per element). */
int64_t om_prolongation(const OMesh *m, const OMesh *fine, int64_t *rows, int64_t *cols, double *vals)
{
    int64_t ne = om_n_elements(m);
    int32_t *conn = malloc(sizeof(int32_t) * 4 * ne);
    int32_t *macro = malloc(sizeof(int32_t) * ne);
    int32_t *bary = malloc(sizeof(int32_t) * 16 * ne);
    om_elements_bary(m, conn, macro, bary);
    int64_t n = 0;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *q = bary + 16 * e;
        int t = macro[e];
        for (int a = 0; a < 4; ++a) {
            int w2[4];
            for (int c = 0; c < 4; ++c) w2[c] = 2 * q[4*a + c];
            rows[n] = canon(fine, t, w2); cols[n] = conn[4*e + a]; vals[n] = 1.0; ++n;
        }
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                int wm[4];
                for (int c = 0; c < 4; ++c) wm[c] = q[4*a + c] + q[4*b + c];
                int64_t f = canon(fine, t, wm);
                rows[n] = f; cols[n] = conn[4*e + a]; vals[n] = 0.5; ++n;
                rows[n] = f; cols[n] = conn[4*e + b]; vals[n] = 0.5; ++n;
            }
    }
    free(conn); free(macro); free(bary);
    return n;
}

/* number of macro tets that hold all given vertices (a primitive's valence) */
int om_valence(const OMesh *m, const int *vids, int cnt)
{
    int v = 0;
    for (int t = 0; t < m->nt; ++t) {
        int ok = 1;
        for (int a = 0; a < cnt && ok; ++a) {
            int f = 0;
            for (int b = 0; b < 4; ++b) if (m->tet[4*t+b] == vids[a]) f = 1;
            ok = f;
        }
        v += ok;
    }
    return v;
}

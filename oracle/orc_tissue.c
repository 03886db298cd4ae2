/* Tissue part of the FP64 oracle: geometry, the cell-centred finite-volume
 * diffusion operator, the explicit time step, stimulus and detection.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The operator follows Sec. 3.2 of the paper step by step:
 *   (a) node values v_n: inverse-distance weighted mean of the cells that
 *       share the node (weights 1/d_k, d_k = node-to-cell-centre distance);
 *   (b) face values v_f: mean of the three node values of the face;
 *   (c) cell gradients by Gauss-Green: grad v_c = (1/V_c) sum_j v_fj S_fj n_fj;
 *   (d) face gradient: alpha-weighted mean of the two cell gradients,
 *       alpha from the position of the face centroid between the centres;
 *   (e) the stabilised face gradient of eq. gra2bis, which replaces the
 *       component along the centre-to-centre unit vector e by the two-point
 *       difference (v_c' - v_c)/d;
 *   (f) flux A_f (M_f grad v_f).n_f through every interior face; boundary
 *       faces carry no flux; the cell balance of eq. electro2_3dmono gives
 *       dv_c/dt = sum_f flux / (chi Cm V_c) - I_ion - I_stim.
 * Every loop writes only its own entries and sums in a fixed order, so the
 * result does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"
#include "orc_models.h"

typedef struct {
    int32_t *ids;
    int64_t n;
    int64_t n0, ndur, nper;
    int32_t count;
    double amp;
} orc_stim;

struct orc_sim {
    int64_t nn, nc;
    double *xyz;
    int32_t *tet;
    double *fib, *scale;
    uint8_t *model;
    double sigma_l, sigma_t, dt, chi, cm;
    /* geometry */
    double *vol, *cen, *S;      /* S[(c*4+j)*3+k] outward area vector      */
    double *Sf;                 /* the area vector of the face's flux       */
    int32_t *nbr;               /* nbr[c*4+j], -1 boundary                 */
    int64_t *inc_off;           /* node -> cells                           */
    int32_t *inc_cell;
    double *inc_w;
    /* state */
    double *y;                  /* y[c*ORC_MAX_SLOTS + slot]               */
    double *vn, *g, *L;
    double *istim;
    /* detection */
    uint8_t *status;
    double *t_act, *v_max, *t_rep, *v_rest;
    double thr, repol;
    orc_stim *stims;
    int n_stims;
    double gscale[4];
    int64_t step;
    int ab2;                    /* non-gating states by Adams-Bashforth 2 */
    int rl2;                    /* gates at midpoint predictions (second order) */
    double *hist;               /* per cell: v rate, then the model's rates */
    /* Purkinje graph */
    int64_t np;
    double *pxyz;
    int64_t *padj_off;          /* node -> incident (neighbour, length) */
    int32_t *padj_nbr;
    double *padj_len;
    double *padj_scale;         /* conductivity multiplier of the segment */
    double *pell;               /* control length l_i */
    double *phist;              /* Adams-Bashforth history per node: ORC_HIST_SLOTS */
    double psigma;
    int pmodel;
    int32_t n_sub;
    int32_t n_sub_given;        /* <= 0: from the stability bound */
    double pdtmax;              /* forward-Euler bound of the graph operator */
    double *py;                 /* py[i*ORC_MAX_SLOTS + slot] */
    double *pistim;
    uint8_t *pstatus;
    double *pt_act;
    orc_stim *pstims;
    int n_pstims;
    /* per-medium time step: the 2D medium (triangles) takes n_sub2
     * substeps of dt / n_sub2 per tissue step (1: none) */
    int32_t n_sub2;
    /* junctions */
    int n_pmj;
    struct orc_pmj *pmj;
    /* bidomain: extracellular conductivities, potential and its solver */
    int bido;
    double sel, set;
    int restart, max_iter;
    double tol;
    double *phi;
    int64_t last_iters, total_iters;
    double last_relres;
};

struct orc_pmj {
    int32_t node;               /* graph node of the source, or -1 */
    int32_t src_cell;           /* cell of the source (2D-3D coupling), or -1 */
    int32_t *cells;
    int64_t n_cells;
    int64_t delay_o, delay_a, ndur;
    int two_way;
    double amp;
    int64_t fire_o, fire_a;     /* first step of the pending stimuli */
};

/* ------------------------------------------------------------- models -- */
int orc_model_n_slots(int model)
{
    switch (model) {
    case ORC_TP06_ENDO: case ORC_TP06_MID: case ORC_TP06_EPI: return 19;
    case ORC_CRN: return 21;
    case ORC_STEWART: return 20;
    case ORC_PASSIVE: return 1;
    default: return 0;
    }
}

const char *orc_model_slot_name(int model, int slot)
{
    switch (model) {
    case ORC_TP06_ENDO: case ORC_TP06_MID: case ORC_TP06_EPI:
        return orc_tp06_slot_name(slot);
    case ORC_CRN: return orc_crn_slot_name(slot);
    case ORC_STEWART: return orc_stewart_slot_name(slot);
    case ORC_PASSIVE: return slot == 0 ? "V" : NULL;
    default: return NULL;
    }
}

void orc_model_init(int model, double *y)
{
    for (int i = 0; i < ORC_MAX_SLOTS; ++i) y[i] = 0.0;
    switch (model) {
    case ORC_TP06_ENDO: case ORC_TP06_MID: case ORC_TP06_EPI:
        orc_tp06_init(y); break;
    case ORC_CRN: orc_crn_init(y); break;
    case ORC_STEWART: orc_stewart_init(y); break;
    default: y[0] = -86.2; break;   /* PASSIVE: any constant works */
    }
}

static double model_step(int model, double *y, double dt, double istim,
                         const double *gscale, orc_hist *h, const orc_mid *mid)
{
    switch (model) {
    case ORC_TP06_ENDO: case ORC_TP06_MID: case ORC_TP06_EPI:
        return orc_tp06_step(model, y, dt, istim, gscale, h, mid);
    case ORC_CRN: return orc_crn_step(y, dt, istim, gscale, h, mid);
    case ORC_STEWART: return orc_stewart_step(y, dt, istim, gscale, h, mid);
    default: return 0.0;
    }
}

double orc_model_step(int model, double *y, double dt, double istim,
                      const double *gscale)
{
    return model_step(model, y, dt, istim, gscale, NULL, NULL);
}

#define ORC_HIST_SLOTS 7   /* v, then at most 6 non-gating model states */

/* the potential's rate under the configured scheme (see orc_rate) */
static double v_rate(const orc_sim *s, double *hv, int first, double F)
{
    if (!s->ab2) return F;
    const double prev = first ? F : *hv;
    *hv = F;
    return 1.5 * F - 0.5 * prev;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ----------------------------------------------------------- geometry -- */
static void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

static int tet_has_node(const int32_t *t, int32_t n)
{
    return t[0] == n || t[1] == n || t[2] == n || t[3] == n;
}

/* vertices of cell c: 4 for a tetrahedron, 3 for a triangle of a 2D medium
 * (fourth node -1) */
static int nverts(const orc_sim *s, int64_t c) { return s->tet[4 * c + 3] < 0 ? 3 : 4; }

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Triangle c of a 2D medium (the paper's cell-centred FV on triangles,
 * Sec. 3.2): area, and per edge j (opposite vertex j) the in-plane outward
 * normal scaled by the edge length, the 2D counterpart of a face area
 * vector. */
static void triangle_geometry(orc_sim *s, int64_t c, const double *p[3])
{
    double u[3], v[3], N[3];
    sub3(p[1], p[0], u);
    sub3(p[2], p[0], v);
    cross3(u, v, N);
    const double twice = norm3(N);
    s->vol[c] = 0.5 * twice;
    for (int a = 0; a < 3; ++a) N[a] /= twice;
    for (int j = 0; j < 3; ++j) {
        const double *a0 = p[(j + 1) % 3], *a1 = p[(j + 2) % 3];
        double t[3], S[3], out[3];
        sub3(a1, a0, t);
        cross3(t, N, S);                     /* |S| = |t|, in the plane */
        sub3(a0, p[j], out);
        const double sg = dot3(S, out) > 0.0 ? 1.0 : -1.0;
        for (int a = 0; a < 3; ++a) s->S[(c * 4 + j) * 3 + a] = sg * S[a];
    }
    for (int a = 0; a < 3; ++a) s->S[(c * 4 + 3) * 3 + a] = 0.0;
}

static void build_geometry(orc_sim *s)
{
    const int64_t nc = s->nc, nn = s->nn;
    /* node -> incident cells (cells listed in increasing id order) */
    s->inc_off = calloc((size_t)nn + 1, sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < nverts(s, c); ++k) s->inc_off[s->tet[4 * c + k] + 1]++;
    for (int64_t n = 0; n < nn; ++n) s->inc_off[n + 1] += s->inc_off[n];
    s->inc_cell = malloc(sizeof(int32_t) * (size_t)(4 * nc));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)nn);
    memcpy(fill, s->inc_off, sizeof(int64_t) * (size_t)nn);
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < nverts(s, c); ++k) s->inc_cell[fill[s->tet[4 * c + k]]++] = (int32_t)c;
    free(fill);

    s->vol = malloc(sizeof(double) * (size_t)nc);
    s->cen = malloc(sizeof(double) * (size_t)nc * 3);
    s->S = malloc(sizeof(double) * (size_t)nc * 12);
    s->Sf = malloc(sizeof(double) * (size_t)nc * 12);
    s->nbr = malloc(sizeof(int32_t) * (size_t)nc * 4);

    /* triangles: geometry and edge neighbours (the other triangle holding
     * both edge vertices) */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        if (nverts(s, c) != 3) continue;
        const int32_t *t = s->tet + 4 * c;
        const double *p[3];
        for (int k = 0; k < 3; ++k) p[k] = s->xyz + 3 * (int64_t)t[k];
        for (int a = 0; a < 3; ++a) s->cen[3 * c + a] = (p[0][a] + p[1][a] + p[2][a]) / 3.0;
        triangle_geometry(s, c, p);
        for (int j = 0; j < 3; ++j) {
            const int32_t na = t[(j + 1) % 3], nb = t[(j + 2) % 3];
            int32_t found = -1;
            for (int64_t i = s->inc_off[na]; i < s->inc_off[na + 1]; ++i) {
                const int32_t k = s->inc_cell[i];
                if (k == (int32_t)c || nverts(s, k) != 3) continue;
                const int32_t *tk = s->tet + 4 * (int64_t)k;
                if (tk[0] == nb || tk[1] == nb || tk[2] == nb) { found = k; break; }
            }
            s->nbr[4 * c + j] = found;
        }
        s->nbr[4 * c + 3] = -1;
    }

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        if (nverts(s, c) != 4) continue;
        const int32_t *t = s->tet + 4 * c;
        const double *p[4];
        for (int k = 0; k < 4; ++k) p[k] = s->xyz + 3 * (int64_t)t[k];
        /* centroid: mean of the four vertices */
        for (int a = 0; a < 3; ++a)
            s->cen[3 * c + a] = 0.25 * (p[0][a] + p[1][a] + p[2][a] + p[3][a]);
        /* volume |det[x1-x0, x2-x0, x3-x0]| / 6 */
        double e1[3], e2[3], e3[3], cr[3];
        sub3(p[1], p[0], e1); sub3(p[2], p[0], e2); sub3(p[3], p[0], e3);
        cr[0] = e2[1] * e3[2] - e2[2] * e3[1];
        cr[1] = e2[2] * e3[0] - e2[0] * e3[2];
        cr[2] = e2[0] * e3[1] - e2[1] * e3[0];
        s->vol[c] = fabs(dot3(e1, cr)) / 6.0;
        /* faces: face j is the triangle opposite local vertex j */
        for (int j = 0; j < 4; ++j) {
            int q[3], m = 0;
            for (int k = 0; k < 4; ++k) if (k != j) q[m++] = k;
            double u[3], v[3], A[3], out[3];
            sub3(p[q[1]], p[q[0]], u);
            sub3(p[q[2]], p[q[0]], v);
            A[0] = 0.5 * (u[1] * v[2] - u[2] * v[1]);
            A[1] = 0.5 * (u[2] * v[0] - u[0] * v[2]);
            A[2] = 0.5 * (u[0] * v[1] - u[1] * v[0]);
            /* outward: away from the opposite vertex */
            sub3(p[q[0]], p[j], out);
            const double sg = dot3(A, out) > 0.0 ? 1.0 : -1.0;
            for (int a = 0; a < 3; ++a) s->S[(c * 4 + j) * 3 + a] = sg * A[a];
            /* neighbour: the other cell holding all three face vertices */
            int32_t na = t[q[0]], nb = t[q[1]], nd = t[q[2]];
            int32_t found = -1;
            for (int64_t i = s->inc_off[na]; i < s->inc_off[na + 1]; ++i) {
                int32_t k = s->inc_cell[i];
                if (k == (int32_t)c) continue;
                const int32_t *tk = s->tet + 4 * (int64_t)k;
                if (tet_has_node(tk, nb) && tet_has_node(tk, nd)) { found = k; break; }
            }
            s->nbr[4 * c + j] = found;
        }
    }

    /* flux area vectors: a tetrahedron's own; across an edge between two
     * triangles (not coplanar on a curved surface) the edge length times the
     * unit bisector of the two outward in-plane normals, shared with opposite
     * signs so that the flux is conservative */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        for (int j = 0; j < 4; ++j)
            for (int a = 0; a < 3; ++a) s->Sf[(c * 4 + j) * 3 + a] = s->S[(c * 4 + j) * 3 + a];
        if (nverts(s, c) != 3) continue;
        const int32_t *t = s->tet + 4 * c;
        for (int j = 0; j < 3; ++j) {
            const int32_t c2 = s->nbr[4 * c + j];
            if (c2 < 0) continue;
            /* the neighbour's edge with the same two vertices */
            const int32_t *t2 = s->tet + 4 * (int64_t)c2;
            int j2 = 0;
            for (int k = 0; k < 3; ++k)
                if (t2[k] != t[(j + 1) % 3] && t2[k] != t[(j + 2) % 3]) j2 = k;
            const double *S1 = s->S + (c * 4 + j) * 3, *S2 = s->S + (c2 * 4 + j2) * 3;
            const double l = norm3(S1), l2 = norm3(S2);
            double b[3];
            for (int a = 0; a < 3; ++a) b[a] = S1[a] / l - S2[a] / l2;
            const double nb = norm3(b);
            for (int a = 0; a < 3; ++a) s->Sf[(c * 4 + j) * 3 + a] = l * b[a] / nb;
        }
    }

    /* inverse-distance node weights */
    s->inc_w = malloc(sizeof(double) * (size_t)(4 * nc));
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < nn; ++n) {
        double sum = 0.0;
        for (int64_t i = s->inc_off[n]; i < s->inc_off[n + 1]; ++i) {
            double r[3];
            sub3(s->xyz + 3 * n, s->cen + 3 * (int64_t)s->inc_cell[i], r);
            s->inc_w[i] = 1.0 / norm3(r);
            sum += s->inc_w[i];
        }
        for (int64_t i = s->inc_off[n]; i < s->inc_off[n + 1]; ++i) s->inc_w[i] /= sum;
    }
}

/* conductivity tensor of a cell: scale * (s_t I + (s_l - s_t) f f^T) */
static void cell_tensor_of(const orc_sim *s, int64_t c, double sl, double st, double M[3][3])
{
    const double *f = s->fib + 3 * c;
    const double sc = s->scale ? s->scale[c] : 1.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            M[a][b] = sc * ((a == b ? st : 0.0) + (sl - st) * f[a] * f[b]);
}

/* ------------------------------------------------------------ operator -- */
void orc_node_values(const orc_sim *s, const double *v, double *vn)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nn; ++n) {
        double acc = 0.0;
        for (int64_t i = s->inc_off[n]; i < s->inc_off[n + 1]; ++i)
            acc += s->inc_w[i] * v[s->inc_cell[i]];
        vn[n] = acc;
    }
}

static void gradients_from_nodes(const orc_sim *s, const double *vn, double *g)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->nc; ++c) {
        const int32_t *t = s->tet + 4 * c;
        const int nv = nverts(s, c);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < nv; ++j) {
            /* face (edge) value: mean of its vertices' node values */
            double vf = 0.0;
            for (int k = 0; k < nv; ++k) if (k != j) vf += vn[t[k]];
            vf /= (double)(nv - 1);
            for (int a = 0; a < 3; ++a) acc[a] += vf * s->S[(c * 4 + j) * 3 + a];
        }
        for (int a = 0; a < 3; ++a) g[3 * c + a] = acc[a] / s->vol[c];
    }
}

void orc_cell_gradients(const orc_sim *s, const double *v, double *g)
{
    double *vn = malloc(sizeof(double) * (size_t)s->nn);
    orc_node_values(s, v, vn);
    gradients_from_nodes(s, vn, g);
    free(vn);
}

/* the face-flux sum sum_f A_f (M_f grad v_f).n_f of one cell for the tensor
 * with conductivities (sl, st) (Sec. 3.2, eq. electro2_3d) */
static double flux_sum(const orc_sim *s, int64_t c, const double *v, const double *g,
                       double sl, double st)
{
    double Mc[3][3];
    cell_tensor_of(s, c, sl, st, Mc);
    const int32_t *t = s->tet + 4 * c;
    const int nv = nverts(s, c);
    double total = 0.0;
    for (int j = 0; j < nv; ++j) {
        const int32_t c2 = s->nbr[4 * c + j];
        if (c2 < 0) continue;                      /* no-flux boundary */
        /* face centroid (edge midpoint) */
        double xf[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < nv; ++k)
            if (k != j)
                for (int a = 0; a < 3; ++a) xf[a] += s->xyz[3 * (int64_t)t[k] + a] / (double)(nv - 1);
        const double *x1 = s->cen + 3 * c, *x2 = s->cen + 3 * (int64_t)c2;
        double r1[3], r2[3], dd[3];
        sub3(x1, xf, r1); sub3(x2, xf, r2); sub3(x2, x1, dd);
        const double alpha = norm3(r2) / (norm3(r1) + norm3(r2));
        const double dist = norm3(dd);
        double e[3] = {dd[0] / dist, dd[1] / dist, dd[2] / dist};
        /* interpolated face gradient */
        double gb[3];
        for (int a = 0; a < 3; ++a)
            gb[a] = alpha * g[3 * c + a] + (1.0 - alpha) * g[3 * (int64_t)c2 + a];
        /* stabilised face gradient (eq. gra2bis) */
        const double corr = (v[c2] - v[c]) / dist - dot3(gb, e);
        double gf[3];
        for (int a = 0; a < 3; ++a) gf[a] = gb[a] + corr * e[a];
        /* face tensor and flux */
        double M2[3][3];
        cell_tensor_of(s, c2, sl, st, M2);
        const double *Sf = s->Sf + (c * 4 + j) * 3;
        double flux = 0.0;
        for (int a = 0; a < 3; ++a) {
            double Mg = 0.0;
            for (int b = 0; b < 3; ++b)
                Mg += (alpha * Mc[a][b] + (1.0 - alpha) * M2[a][b]) * gf[b];
            flux += Mg * Sf[a];
        }
        total += flux;
    }
    return total;
}

/* monodomain: the flux sum with M, divided by chi Cm V_c (mV/ms) */
static double cell_flux_sum(const orc_sim *s, int64_t c, const double *v,
                            const double *g)
{
    return flux_sum(s, c, v, g, s->sigma_l, s->sigma_t) / (s->chi * s->cm * s->vol[c]);
}

/* y = the flux sums of field x for conductivities (sl, st) */
static void apply_flux(const orc_sim *s, const double *x, double sl, double st, double *y)
{
    double *xn = malloc(sizeof(double) * (size_t)s->nn);
    double *g = malloc(sizeof(double) * (size_t)s->nc * 3);
    orc_node_values(s, x, xn);
    gradients_from_nodes(s, xn, g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->nc; ++c) y[c] = flux_sum(s, c, x, g, sl, st);
    free(xn);
    free(g);
}

void orc_apply_diffusion(const orc_sim *s, const double *v, double *L)
{
    double *vn = malloc(sizeof(double) * (size_t)s->nn);
    double *g = malloc(sizeof(double) * (size_t)s->nc * 3);
    orc_node_values(s, v, vn);
    gradients_from_nodes(s, vn, g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->nc; ++c) L[c] = cell_flux_sum(s, c, v, g);
    free(vn);
    free(g);
}

void orc_geometry(const orc_sim *s, double *vol, double *area_vec, int32_t *nbr)
{
    if (vol) memcpy(vol, s->vol, sizeof(double) * (size_t)s->nc);
    if (area_vec) memcpy(area_vec, s->S, sizeof(double) * (size_t)s->nc * 12);
    if (nbr) memcpy(nbr, s->nbr, sizeof(int32_t) * (size_t)s->nc * 4);
}

/* ---------------------------------------------------------- lifecycle -- */
orc_sim *orc_create(int64_t n_nodes, const double *xyz, int64_t n_tets,
                    const int32_t *tets, const double *fibre, double sigma_l,
                    double sigma_t, const double *scale, const uint8_t *model,
                    double dt, double chi, double cm)
{
    orc_sim *s = calloc(1, sizeof(orc_sim));
    s->nn = n_nodes; s->nc = n_tets;
    s->n_sub2 = 1;
    s->xyz = malloc(sizeof(double) * (size_t)n_nodes * 3);
    memcpy(s->xyz, xyz, sizeof(double) * (size_t)n_nodes * 3);
    s->tet = malloc(sizeof(int32_t) * (size_t)n_tets * 4);
    memcpy(s->tet, tets, sizeof(int32_t) * (size_t)n_tets * 4);
    s->fib = malloc(sizeof(double) * (size_t)n_tets * 3);
    memcpy(s->fib, fibre, sizeof(double) * (size_t)n_tets * 3);
    if (scale) {
        s->scale = malloc(sizeof(double) * (size_t)n_tets);
        memcpy(s->scale, scale, sizeof(double) * (size_t)n_tets);
    }
    s->model = malloc((size_t)n_tets);
    memcpy(s->model, model, (size_t)n_tets);
    s->sigma_l = sigma_l; s->sigma_t = sigma_t;
    s->dt = dt; s->chi = chi; s->cm = cm;
    s->thr = 0.0; s->repol = 0.9;
    for (int i = 0; i < 4; ++i) s->gscale[i] = 1.0;
    build_geometry(s);

    s->y = malloc(sizeof(double) * (size_t)n_tets * ORC_MAX_SLOTS);
    s->vn = malloc(sizeof(double) * (size_t)n_nodes);
    s->g = malloc(sizeof(double) * (size_t)n_tets * 3);
    s->L = malloc(sizeof(double) * (size_t)n_tets);
    s->istim = malloc(sizeof(double) * (size_t)n_tets);
    s->status = calloc((size_t)n_tets, 1);
    s->t_act = malloc(sizeof(double) * (size_t)n_tets);
    s->v_max = malloc(sizeof(double) * (size_t)n_tets);
    s->t_rep = malloc(sizeof(double) * (size_t)n_tets);
    s->v_rest = malloc(sizeof(double) * (size_t)n_tets);
    for (int64_t c = 0; c < n_tets; ++c) {
        orc_model_init(model[c], s->y + c * ORC_MAX_SLOTS);
        s->v_rest[c] = s->y[c * ORC_MAX_SLOTS];
        s->t_act[c] = NAN; s->t_rep[c] = NAN; s->v_max[c] = NAN;
    }
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->xyz); free(s->tet); free(s->fib); free(s->scale); free(s->model); free(s->Sf);
    free(s->vol); free(s->cen); free(s->S); free(s->nbr);
    free(s->inc_off); free(s->inc_cell); free(s->inc_w);
    free(s->y); free(s->vn); free(s->g); free(s->L); free(s->istim);
    free(s->status); free(s->t_act); free(s->v_max); free(s->t_rep);
    free(s->v_rest);
    for (int i = 0; i < s->n_stims; ++i) free(s->stims[i].ids);
    free(s->stims);
    free(s->pxyz); free(s->padj_off); free(s->padj_nbr); free(s->padj_len);
    free(s->padj_scale);
    free(s->hist); free(s->phist);
    free(s->pell); free(s->py); free(s->pistim); free(s->pstatus); free(s->pt_act);
    for (int i = 0; i < s->n_pstims; ++i) free(s->pstims[i].ids);
    free(s->pstims);
    for (int k = 0; k < s->n_pmj; ++k) free(s->pmj[k].cells);
    free(s->pmj);
    free(s->phi);
    free(s);
}

void orc_set_ionic_scale(orc_sim *s, const double gscale[4])
{
    for (int i = 0; i < 4; ++i) s->gscale[i] = gscale[i];
}

void orc_set_detection(orc_sim *s, double threshold, double repol_frac)
{
    s->thr = threshold;
    s->repol = repol_frac;
}

int orc_add_stimulus(orc_sim *s, int64_t n_ids, const int32_t *ids, double t0,
                     double dur, double amp, double period, int32_t count)
{
    s->stims = realloc(s->stims, sizeof(orc_stim) * (size_t)(s->n_stims + 1));
    orc_stim *st = &s->stims[s->n_stims++];
    st->ids = malloc(sizeof(int32_t) * (size_t)(n_ids > 0 ? n_ids : 1));
    memcpy(st->ids, ids, sizeof(int32_t) * (size_t)n_ids);
    st->n = n_ids;
    /* the Heaviside window of eq. stimulus, on whole steps */
    st->n0 = llround(t0 / s->dt);
    st->ndur = llround(dur / s->dt);
    st->nper = period > 0.0 ? llround(period / s->dt) : 0;
    st->count = count < 1 ? 1 : count;
    st->amp = amp;
    return s->n_stims - 1;
}

static int stim_active(const orc_stim *st, int64_t n)
{
    const int64_t k = n - st->n0;
    if (k < 0) return 0;
    if (st->nper <= 0) return k < st->ndur;
    return (k / st->nper) < st->count && (k % st->nper) < st->ndur;
}

/* ------------------------------------------------------------ Purkinje -- */
static double region_mean(const struct orc_pmj *J, const double *v)
{
    double acc = 0.0;
    for (int64_t q = 0; q < J->n_cells; ++q) acc += v[J->cells[q]];
    return acc / (double)J->n_cells;
}

/* Events of junction J after step n: the source potential went from a to b
 * (an upward threshold crossing schedules the pulse on the region); with
 * two-way coupling an upward crossing of the region's mean schedules the
 * pulse on the source.  v_old holds the tissue at level n, the cells level
 * n+1. */
static void junction_event(orc_sim *s, struct orc_pmj *J, double a, double b, const double *v_old)
{
    const int64_t n = s->step;
    if (a <= s->thr && b > s->thr) J->fire_o = n + 1 + J->delay_o;
    if (J->two_way) {
        const double m0 = region_mean(J, v_old);
        double m1 = 0.0;
        for (int64_t q = 0; q < J->n_cells; ++q) m1 += s->y[(int64_t)J->cells[q] * ORC_MAX_SLOTS];
        m1 /= (double)J->n_cells;
        if (m0 <= s->thr && m1 > s->thr) J->fire_a = n + 1 + J->delay_a;
    }
}

/* n_sub substeps of the graph over tissue step n, then junction events;
 * v_old is the tissue potential at level n (the cells hold level n+1). */
static void purkinje_step(orc_sim *s, const double *v_old)
{
    const int64_t n = s->step, np = s->np;
    const double dtp = s->dt / s->n_sub;
    double *vp = malloc(sizeof(double) * (size_t)np);
    double *vp0 = malloc(sizeof(double) * (size_t)np);
    for (int64_t i = 0; i < np; ++i) vp0[i] = s->py[i * ORC_MAX_SLOTS];
    /* stimuli of the graph during this tissue step */
    memset(s->pistim, 0, sizeof(double) * (size_t)np);
    for (int i = 0; i < s->n_pstims; ++i) {
        const orc_stim *st = &s->pstims[i];
        if (!stim_active(st, n)) continue;
        for (int64_t q = 0; q < st->n; ++q) s->pistim[st->ids[q]] += st->amp;
    }
    for (int k = 0; k < s->n_pmj; ++k) {
        const struct orc_pmj *J = &s->pmj[k];
        if (J->src_cell < 0 && J->two_way && n >= J->fire_a && n < J->fire_a + J->ndur)
            s->pistim[J->node] += J->amp;
    }
    for (int sub = 0; sub < s->n_sub; ++sub) {
        for (int64_t i = 0; i < np; ++i) vp[i] = s->py[i * ORC_MAX_SLOTS];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < np; ++i) {
            double *y = s->py + i * ORC_MAX_SLOTS;
            double flux = 0.0;
            for (int64_t e = s->padj_off[i]; e < s->padj_off[i + 1]; ++e)
                flux += s->padj_scale[e] * (vp[s->padj_nbr[e]] - vp[i]) / s->padj_len[e];
            const double L = s->psigma * flux / (s->chi * s->cm * s->pell[i]);
            double *hc = s->ab2 ? s->phist + i * ORC_HIST_SLOTS : NULL;
            const int first = n == 0 && sub == 0;
            orc_hist h = {hc ? hc + 1 : NULL, first};
            const orc_mid mid = {L - s->pistim[i]};
            const double iion = model_step(s->pmodel, y, dtp, s->pistim[i], s->gscale,
                                           hc ? &h : NULL, s->rl2 ? &mid : NULL);
            const double vnew = vp[i] + dtp * v_rate(s, hc, first, L - iion - s->pistim[i]);
            y[0] = vnew;
            if (!s->pstatus[i] && vp[i] <= s->thr && vnew > s->thr) {
                s->pt_act[i] = ((double)(n * s->n_sub + sub) +
                                (s->thr - vp[i]) / (vnew - vp[i])) * dtp;
                s->pstatus[i] = 1;
            }
        }
    }
    /* junction events: upward crossings during this step fire later */
    for (int k = 0; k < s->n_pmj; ++k) {
        struct orc_pmj *J = &s->pmj[k];
        if (J->src_cell >= 0) continue;
        junction_event(s, J, vp0[J->node], s->py[(int64_t)J->node * ORC_MAX_SLOTS], v_old);
    }
    free(vp);
    free(vp0);
}

/* Substeps per tissue step: as given, else the smallest count within 90 %
 * of the stability bound: dtmax for forward Euler, dtmax / 2 for
 * Adams-Bashforth 2 (its interval on the negative real axis is half as
 * long). */
static int32_t graph_substeps(const orc_sim *s)
{
    if (s->n_sub_given > 0) return s->n_sub_given;
    const double lim = (s->ab2 ? 0.45 : 0.9) * s->pdtmax;
    int32_t k = 1;
    while (s->dt / k > lim) ++k;
    return k;
}

int orc_set_purkinje(orc_sim *s, int64_t n, const double *xyz, int64_t n_edges,
                     const int32_t *edges, const double *edge_scale, double sigma,
                     int model, int32_t n_sub)
{
    if (n <= 0 || n_edges < 0 || !(sigma > 0)) return -1;
    for (int64_t e = 0; e < 2 * n_edges; ++e)
        if (edges[e] < 0 || edges[e] >= n) return -1;
    if (edge_scale)
        for (int64_t e = 0; e < n_edges; ++e)
            if (!(edge_scale[e] >= 0.0) || !isfinite(edge_scale[e])) return -1;
    s->np = n;
    s->pxyz = malloc(sizeof(double) * (size_t)n * 3);
    memcpy(s->pxyz, xyz, sizeof(double) * (size_t)n * 3);
    s->psigma = sigma;
    s->pmodel = model;
    s->padj_off = calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < n_edges; ++e) {
        s->padj_off[edges[2 * e] + 1]++;
        s->padj_off[edges[2 * e + 1] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) s->padj_off[i + 1] += s->padj_off[i];
    s->padj_nbr = malloc(sizeof(int32_t) * (size_t)(2 * n_edges + 1));
    s->padj_len = malloc(sizeof(double) * (size_t)(2 * n_edges + 1));
    s->padj_scale = malloc(sizeof(double) * (size_t)(2 * n_edges + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)n);
    memcpy(fill, s->padj_off, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t a = edges[2 * e], b = edges[2 * e + 1];
        double d[3];
        sub3(xyz + 3 * (int64_t)a, xyz + 3 * (int64_t)b, d);
        const double len = norm3(d), sc = edge_scale ? edge_scale[e] : 1.0;
        s->padj_nbr[fill[a]] = b; s->padj_scale[fill[a]] = sc; s->padj_len[fill[a]++] = len;
        s->padj_nbr[fill[b]] = a; s->padj_scale[fill[b]] = sc; s->padj_len[fill[b]++] = len;
    }
    free(fill);
    s->pell = calloc((size_t)n, sizeof(double));
    double dtmax = 1e300;
    for (int64_t i = 0; i < n; ++i) {
        double inv = 0.0;
        for (int64_t e = s->padj_off[i]; e < s->padj_off[i + 1]; ++e) {
            s->pell[i] += 0.5 * s->padj_len[e];
            inv += s->padj_scale[e] / s->padj_len[e];
        }
        if (inv > 0.0) {
            const double lim = s->chi * s->cm * s->pell[i] / (sigma * inv);
            if (lim < dtmax) dtmax = lim;
        }
    }
    s->n_sub_given = n_sub;
    s->pdtmax = dtmax;
    s->n_sub = graph_substeps(s);
    s->py = malloc(sizeof(double) * (size_t)n * ORC_MAX_SLOTS);
    s->pistim = calloc((size_t)n, sizeof(double));
    s->pstatus = calloc((size_t)n, 1);
    s->pt_act = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        orc_model_init(model, s->py + i * ORC_MAX_SLOTS);
        s->pt_act[i] = NAN;
    }
    return 0;
}

/* Muscle region of a junction at point x: the cells whose centroid lies
 * within the radius, else the cells sharing a node with the cell of nearest
 * centroid; only cells with `kind` vertices count (0: any). */
static void junction_region(orc_sim *s, struct orc_pmj *J, const double *x, double radius,
                            int kind)
{
    int64_t cnt = 0, best = -1;
    double bestd = 1e300;
    for (int64_t c = 0; c < s->nc; ++c) {
        if (kind && nverts(s, c) != kind) continue;
        double r[3];
        sub3(s->cen + 3 * c, x, r);
        const double d = norm3(r);
        if (d <= radius) cnt++;
        if (d < bestd) { bestd = d; best = c; }
    }
    if (cnt > 0) {
        J->cells = malloc(sizeof(int32_t) * (size_t)cnt);
        for (int64_t c = 0; c < s->nc; ++c) {
            if (kind && nverts(s, c) != kind) continue;
            double r[3];
            sub3(s->cen + 3 * c, x, r);
            if (norm3(r) <= radius) J->cells[J->n_cells++] = (int32_t)c;
        }
    } else {
        const int32_t *t = s->tet + 4 * best;
        J->cells = malloc(sizeof(int32_t) * (size_t)s->nc);
        for (int64_t c = 0; c < s->nc; ++c) {
            const int32_t *u = s->tet + 4 * c;
            int share = 0;
            for (int a = 0; a < nverts(s, best); ++a)
                for (int b = 0; b < nverts(s, c); ++b) share |= (t[a] == u[b]);
            if (share) J->cells[J->n_cells++] = (int32_t)c;
        }
    }
}

static void junction_timing(orc_sim *s, struct orc_pmj *J, double delay_ortho,
                            double delay_anti, int two_way, double amp, double dur)
{
    J->delay_o = llround(delay_ortho / s->dt);
    J->delay_a = llround(delay_anti / s->dt);
    J->ndur = llround(dur / s->dt);
    J->two_way = two_way;
    J->amp = amp;
    J->fire_o = J->fire_a = INT64_MIN / 2;
}

int orc_add_cell_junction(orc_sim *s, int32_t cell, double radius, double delay_ortho,
                          double delay_anti, int two_way, double amp, double dur)
{
    if (cell < 0 || cell >= s->nc) return -1;
    s->pmj = realloc(s->pmj, sizeof(struct orc_pmj) * (size_t)(s->n_pmj + 1));
    struct orc_pmj *J = &s->pmj[s->n_pmj++];
    memset(J, 0, sizeof(*J));
    J->node = -1;
    J->src_cell = cell;
    /* the region lies in the other medium (a triangle couples to tets) */
    junction_region(s, J, s->cen + 3 * (int64_t)cell, radius, nverts(s, cell) == 3 ? 4 : 3);
    if (J->n_cells == 0) { s->n_pmj--; free(J->cells); return -1; }
    junction_timing(s, J, delay_ortho, delay_anti, two_way, amp, dur);
    return s->n_pmj - 1;
}

int orc_add_pmj(orc_sim *s, int32_t node, double radius, double delay_ortho,
                double delay_anti, int two_way, double amp, double dur)
{
    if (node < 0 || node >= s->np) return -1;
    s->pmj = realloc(s->pmj, sizeof(struct orc_pmj) * (size_t)(s->n_pmj + 1));
    struct orc_pmj *J = &s->pmj[s->n_pmj++];
    memset(J, 0, sizeof(*J));
    J->node = node;
    J->src_cell = -1;
    junction_region(s, J, s->pxyz + 3 * (int64_t)node, radius, 0);
    junction_timing(s, J, delay_ortho, delay_anti, two_way, amp, dur);
    return s->n_pmj - 1;
}

int orc_add_purkinje_stimulus(orc_sim *s, int64_t n_ids, const int32_t *ids, double t0,
                              double dur, double amp, double period, int32_t count)
{
    s->pstims = realloc(s->pstims, sizeof(orc_stim) * (size_t)(s->n_pstims + 1));
    orc_stim *st = &s->pstims[s->n_pstims++];
    st->ids = malloc(sizeof(int32_t) * (size_t)(n_ids > 0 ? n_ids : 1));
    memcpy(st->ids, ids, sizeof(int32_t) * (size_t)n_ids);
    st->n = n_ids;
    st->n0 = llround(t0 / s->dt);
    st->ndur = llround(dur / s->dt);
    st->nper = period > 0.0 ? llround(period / s->dt) : 0;
    st->count = count < 1 ? 1 : count;
    st->amp = amp;
    return s->n_pstims - 1;
}

int32_t orc_purkinje_n_sub(const orc_sim *s) { return s->n_sub; }

void orc_get_purkinje_vm(const orc_sim *s, double *out)
{
    for (int64_t i = 0; i < s->np; ++i) out[i] = s->py[i * ORC_MAX_SLOTS];
}

void orc_get_purkinje_activation(const orc_sim *s, double *out)
{
    for (int64_t i = 0; i < s->np; ++i) out[i] = s->pstatus[i] ? s->pt_act[i] : NAN;
}

int64_t orc_get_pmj_region(const orc_sim *s, int k, int32_t *out, int64_t cap)
{
    if (k < 0 || k >= s->n_pmj) return -1;
    const struct orc_pmj *J = &s->pmj[k];
    for (int64_t q = 0; q < J->n_cells && q < cap; ++q) out[q] = J->cells[q];
    return J->n_cells;
}

/* ---------------------------------------------------------- bidomain -- */
static double dot_n(const double *a, const double *b, int64_t n)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/* Restarted GMRES (Arnoldi with modified Gram-Schmidt, Givens rotations;
 * Trefethen & Bau, lecture 35) for A x = b, A = the flux sums with the
 * conductivities (sl, st), starting from x.  Stops when the residual norm is
 * at most tol ||b|| or after max_iter Arnoldi steps; returns the steps. */
static int64_t gmres(orc_sim *s, const double *b, double *x, double sl, double st,
                     int m, double tol, int64_t max_iter, double *relres)
{
    const int64_t n = s->nc;
    const double bnorm = sqrt(dot_n(b, b, n));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        *relres = 0.0;
        return 0;
    }
    double *V = malloc(sizeof(double) * (size_t)n * (size_t)(m + 1));
    double *H = calloc((size_t)(m + 1) * (size_t)m, sizeof(double));   /* H[i*m + j] */
    double *cs = malloc(sizeof(double) * (size_t)m), *sn = malloc(sizeof(double) * (size_t)m);
    double *g = malloc(sizeof(double) * (size_t)(m + 1)), *y = malloc(sizeof(double) * (size_t)m);
    double *w = malloc(sizeof(double) * (size_t)n);
    int64_t it = 0;
    for (;;) {
        apply_flux(s, x, sl, st, w);
        for (int64_t i = 0; i < n; ++i) w[i] = b[i] - w[i];
        const double beta = sqrt(dot_n(w, w, n));
        *relres = beta / bnorm;
        if (beta <= tol * bnorm || it >= max_iter) break;
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < max_iter; ++j) {
            double *vj = V + (size_t)j * (size_t)n;
            apply_flux(s, vj, sl, st, w);
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * (size_t)n;
                const double h = dot_n(w, vi, n);
                H[i * m + j] = h;
                for (int64_t q = 0; q < n; ++q) w[q] -= h * vi[q];
            }
            const double hn = sqrt(dot_n(w, w, n));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {           /* earlier rotations */
                const double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double den = hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = den > 0.0 ? H[j * m + j] / den : 1.0;
            sn[j] = den > 0.0 ? H[(j + 1) * m + j] / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (fabs(g[j + 1]) <= tol * bnorm || hn == 0.0) break;
            double *vn1 = V + (size_t)(j + 1) * (size_t)n;
            for (int64_t q = 0; q < n; ++q) vn1[q] = w[q] / hn;
        }
        for (int i = k - 1; i >= 0; --i) {          /* R y = g */
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= H[i * m + l] * y[l];
            y[i] = acc / H[i * m + i];
        }
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * (size_t)n;
            for (int64_t q = 0; q < n; ++q) x[q] += y[i] * vi[q];
        }
    }
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(w);
    return it;
}

/* the extracellular potential of zero volume-weighted mean (the elliptic
 * equation fixes it up to a constant) */
static void zero_mean(const orc_sim *s, double *x)
{
    double num = 0.0, den = 0.0;
    for (int64_t c = 0; c < s->nc; ++c) { num += s->vol[c] * x[c]; den += s->vol[c]; }
    const double m = num / den;
    for (int64_t c = 0; c < s->nc; ++c) x[c] -= m;
}

/* v^{n+1} known: solve sum_f A_f ((Mi+Me) grad phi).n = -sum_f A_f (Mi grad v).n
 * for phi^{n+1}, starting from phi^n (Sec. 3.2) */
static void bidomain_solve(orc_sim *s)
{
    const int64_t nc = s->nc;
    double *v = malloc(sizeof(double) * (size_t)nc);
    double *b = malloc(sizeof(double) * (size_t)nc);
    for (int64_t c = 0; c < nc; ++c) v[c] = s->y[c * ORC_MAX_SLOTS];
    apply_flux(s, v, s->sigma_l, s->sigma_t, b);
    for (int64_t c = 0; c < nc; ++c) b[c] = -b[c];
    s->last_iters = gmres(s, b, s->phi, s->sigma_l + s->sel, s->sigma_t + s->set, s->restart,
                          s->tol, s->max_iter, &s->last_relres);
    s->total_iters += s->last_iters;
    zero_mean(s, s->phi);
    free(v);
    free(b);
}

int orc_set_bidomain(orc_sim *s, double sigma_el, double sigma_et, int restart, double tol,
                     int max_iter)
{
    if (!(sigma_el >= 0) || !(sigma_et >= 0) || restart < 1 || !(tol > 0) || max_iter < 1)
        return -1;
    s->bido = 1;
    s->sel = sigma_el;
    s->set = sigma_et;
    s->restart = restart;
    s->tol = tol;
    s->max_iter = max_iter;
    free(s->phi);
    s->phi = calloc((size_t)s->nc, sizeof(double));   /* exact for a uniform v^0 */
    s->last_iters = s->total_iters = 0;
    s->last_relres = 0.0;
    return 0;
}

void orc_get_phi_e(const orc_sim *s, double *out)
{
    for (int64_t c = 0; c < s->nc; ++c) out[c] = s->phi ? s->phi[c] : 0.0;
}

int64_t orc_bidomain_iterations(const orc_sim *s, int64_t *total, double *relres)
{
    if (total) *total = s->total_iters;
    if (relres) *relres = s->last_relres;
    return s->last_iters;
}

void orc_apply_flux(const orc_sim *s, const double *x, double sl, double st, double *y)
{
    apply_flux(s, x, sl, st, y);
}

int64_t orc_gmres(orc_sim *s, const double *b, double *x, double sl, double st, int restart,
                  double tol, int max_iter, double *relres)
{
    return gmres(s, b, x, sl, st, restart, tol, max_iter, relres);
}

/* ---------------------------------------------------------- time step -- */
/* Activation time (first upward crossing of the threshold) and APD90 of
 * cell c over one update vold -> vnew that starts at time t0 * h and lasts h:
 * the crossing instants are interpolated linearly inside the update. */
static void detect(orc_sim *s, int64_t c, double vold, double vnew, double t0, double h)
{
    if (s->status[c] == 0) {
        if (vold <= s->thr && vnew > s->thr) {
            s->t_act[c] = (t0 + (s->thr - vold) / (vnew - vold)) * h;
            s->v_max[c] = vnew;
            s->status[c] = 1;
        }
    } else if (s->status[c] == 1) {
        if (vnew > s->v_max[c]) s->v_max[c] = vnew;
        const double v90 = s->v_max[c] - s->repol * (s->v_max[c] - s->v_rest[c]);
        if (vold >= v90 && vnew < v90) {
            s->t_rep[c] = (t0 + (vold - v90) / (vold - vnew)) * h;
            s->status[c] = 2;
        }
    }
}

/* The 2D medium over tissue step n with a time step of its own (the paper
 * integrates its Purkinje shell of triangles at a far smaller step than the
 * myocardium, Sec. 4): n_sub2 explicit substeps of dt / n_sub2, each the
 * whole monodomain update of the triangles (node values, gradients, face
 * fluxes, cell model, v, detection) from the substep's own potentials.  The
 * stimulus currents are those of step n throughout.  Nodes belong to one
 * medium, so the node values of triangles depend on triangles only. */
static void medium2_substeps(orc_sim *s, int64_t n)
{
    const int64_t nc = s->nc;
    const int32_t m = s->n_sub2;
    const double h = s->dt / m;
    double *u = malloc(sizeof(double) * (size_t)nc);
    for (int32_t q = 0; q < m; ++q) {
        for (int64_t c = 0; c < nc; ++c) u[c] = s->y[c * ORC_MAX_SLOTS];
        orc_node_values(s, u, s->vn);
        gradients_from_nodes(s, s->vn, s->g);
        const int first = n == 0 && q == 0;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            if (nverts(s, c) != 3) continue;
            double *y = s->y + c * ORC_MAX_SLOTS;
            const double L = cell_flux_sum(s, c, u, s->g);
            double *hc = s->ab2 ? s->hist + c * ORC_HIST_SLOTS : NULL;
            orc_hist hh = {hc ? hc + 1 : NULL, first};
            const orc_mid mid = {L - s->istim[c]};
            const double iion = model_step(s->model[c], y, h, s->istim[c], s->gscale,
                                           hc ? &hh : NULL, s->rl2 ? &mid : NULL);
            const double vnew = u[c] + h * v_rate(s, hc, first, L - iion - s->istim[c]);
            y[0] = vnew;
            detect(s, c, u[c], vnew, (double)(n * m + q), h);
        }
    }
    free(u);
}

/* Forward-Euler bound of the 2D medium's operator from its two-point part:
 * cell c couples to each edge neighbour with sigma_max |S_f| / (d_f chi Cm
 * V_c) (sigma_max the larger conductivity times the cell's scale, |S_f| the
 * edge length, d_f the centroid distance), so by Gershgorin the spectrum
 * lies in [-2 r_c, 0] with r_c the sum of these couplings and explicit
 * steps up to 1 / max_c r_c are stable. */
static double medium2_dtmax(const orc_sim *s)
{
    double rmax = 0.0;
    const double smax = s->sigma_l > s->sigma_t ? s->sigma_l : s->sigma_t;
    for (int64_t c = 0; c < s->nc; ++c) {
        if (nverts(s, c) != 3) continue;
        double r = 0.0;
        for (int j = 0; j < 3; ++j) {
            const int32_t k = s->nbr[4 * c + j];
            if (k < 0) continue;
            double d[3];
            sub3(s->cen + 3 * (int64_t)k, s->cen + 3 * c, d);
            r += norm3(s->S + (c * 4 + j) * 3) / norm3(d);
        }
        r *= smax * (s->scale ? s->scale[c] : 1.0) / (s->chi * s->cm * s->vol[c]);
        if (r > rmax) rmax = r;
    }
    return rmax > 0.0 ? 1.0 / rmax : HUGE_VAL;
}

int orc_set_medium_substeps(orc_sim *s, int32_t n_sub)
{
    if (s->step != 0) return -1;
    if (n_sub > 0) {
        s->n_sub2 = n_sub;
        return 0;
    }
    const double lim = (s->ab2 ? 0.45 : 0.9) * medium2_dtmax(s);
    int32_t k = 1;
    while (s->dt / k > lim) ++k;
    s->n_sub2 = k;
    return 0;
}

int32_t orc_medium_substeps(const orc_sim *s) { return s->n_sub2; }

static void one_step(orc_sim *s)
{
    const int64_t nc = s->nc, n = s->step;
    const double dt = s->dt;
    if (s->ab2 && !s->hist) s->hist = calloc((size_t)nc * ORC_HIST_SLOTS, sizeof(double));
    if (s->ab2 && s->np > 0 && !s->phist)
        s->phist = calloc((size_t)s->np * ORC_HIST_SLOTS, sizeof(double));
    double *v = malloc(sizeof(double) * (size_t)nc);
    for (int64_t c = 0; c < nc; ++c) v[c] = s->y[c * ORC_MAX_SLOTS];

    /* stimulus currents at level n (protocol stimuli, then junctions) */
    memset(s->istim, 0, sizeof(double) * (size_t)nc);
    for (int i = 0; i < s->n_stims; ++i) {
        const orc_stim *st = &s->stims[i];
        if (!stim_active(st, n)) continue;
        for (int64_t q = 0; q < st->n; ++q) s->istim[st->ids[q]] += st->amp;
    }
    for (int k = 0; k < s->n_pmj; ++k) {
        const struct orc_pmj *J = &s->pmj[k];
        if (n >= J->fire_o && n < J->fire_o + J->ndur)
            for (int64_t q = 0; q < J->n_cells; ++q) s->istim[J->cells[q]] += J->amp;
        if (J->src_cell >= 0 && J->two_way && n >= J->fire_a && n < J->fire_a + J->ndur)
            s->istim[J->src_cell] += J->amp;
    }

    /* diffusion at level n; bidomain: the intracellular flux of v + phi_e */
    if (s->bido) {
        double *u = malloc(sizeof(double) * (size_t)nc);
        for (int64_t c = 0; c < nc; ++c) u[c] = v[c] + s->phi[c];
        orc_node_values(s, u, s->vn);
        gradients_from_nodes(s, s->vn, s->g);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c)
            s->L[c] = flux_sum(s, c, u, s->g, s->sigma_l, s->sigma_t) / (s->chi * s->cm * s->vol[c]);
        free(u);
    } else {
        orc_node_values(s, v, s->vn);
        gradients_from_nodes(s, s->vn, s->g);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) s->L[c] = cell_flux_sum(s, c, v, s->g);
    }

    /* cells: ionic update, v update, detection (with a time step of its
     * own the 2D medium follows below) */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        if (s->n_sub2 > 1 && nverts(s, c) == 3) continue;
        double *y = s->y + c * ORC_MAX_SLOTS;
        const double vold = v[c];
        double *hc = s->ab2 ? s->hist + c * ORC_HIST_SLOTS : NULL;
        orc_hist h = {hc ? hc + 1 : NULL, n == 0};
        const orc_mid mid = {s->L[c] - s->istim[c]};
        const double iion = model_step(s->model[c], y, dt, s->istim[c], s->gscale,
                                       hc ? &h : NULL, s->rl2 ? &mid : NULL);
        const double vnew = vold + dt * v_rate(s, hc, n == 0, s->L[c] - iion - s->istim[c]);
        y[0] = vnew;
        detect(s, c, vold, vnew, (double)n, dt);
    }
    if (s->n_sub2 > 1) medium2_substeps(s, n);
    if (s->np > 0) purkinje_step(s, v);
    for (int k = 0; k < s->n_pmj; ++k) {
        struct orc_pmj *J = &s->pmj[k];
        if (J->src_cell >= 0)
            junction_event(s, J, v[J->src_cell], s->y[(int64_t)J->src_cell * ORC_MAX_SLOTS], v);
    }
    if (s->bido) bidomain_solve(s);
    free(v);
    s->step++;
}

int orc_set_time_scheme(orc_sim *s, int scheme)
{
    if (scheme < 0 || scheme > 2 || s->step != 0) return -1;
    s->ab2 = scheme >= 1;
    s->rl2 = scheme == 2;
    if (s->np > 0) s->n_sub = graph_substeps(s);
    return 0;
}

void orc_step(orc_sim *s, int64_t n_steps)
{
    for (int64_t i = 0; i < n_steps; ++i) one_step(s);
}

int64_t orc_get_step(const orc_sim *s) { return s->step; }
void orc_set_step(orc_sim *s, int64_t step) { s->step = step; }

void orc_get_vm(const orc_sim *s, double *out)
{
    for (int64_t c = 0; c < s->nc; ++c) out[c] = s->y[c * ORC_MAX_SLOTS];
}

void orc_get_activation(const orc_sim *s, double *out)
{
    for (int64_t c = 0; c < s->nc; ++c) out[c] = s->status[c] ? s->t_act[c] : NAN;
}

void orc_get_apd90(const orc_sim *s, double *out)
{
    for (int64_t c = 0; c < s->nc; ++c)
        out[c] = s->status[c] == 2 ? s->t_rep[c] - s->t_act[c] : NAN;
}

double orc_mean_vm(const orc_sim *s)
{
    double num = 0.0, den = 0.0;
    for (int64_t c = 0; c < s->nc; ++c) {
        num += s->vol[c] * s->y[c * ORC_MAX_SLOTS];
        den += s->vol[c];
    }
    return num / den;
}

void orc_get_states(const orc_sim *s, double *out)
{
    for (int slot = 0; slot < ORC_MAX_SLOTS; ++slot)
        for (int64_t c = 0; c < s->nc; ++c)
            out[slot * s->nc + c] = slot < orc_model_n_slots(s->model[c])
                                        ? s->y[c * ORC_MAX_SLOTS + slot] : NAN;
}

void orc_set_states(orc_sim *s, const double *in)
{
    for (int slot = 0; slot < ORC_MAX_SLOTS; ++slot)
        for (int64_t c = 0; c < s->nc; ++c)
            if (slot < orc_model_n_slots(s->model[c]))
                s->y[c * ORC_MAX_SLOTS + slot] = in[slot * s->nc + c];
}

/* Detection state of every cell as 4 rows of n_tets: status (0 before
 * activation, 1 activated, 2 repolarised), activation time, running maximum
 * of V, repolarisation time.  With the states and the step counter this is
 * all a monodomain run without graph or bidomain carries from step to step,
 * so a long run can be stopped and resumed. */
void orc_get_detect_state(const orc_sim *s, double *out)
{
    for (int64_t c = 0; c < s->nc; ++c) {
        out[c] = (double)s->status[c];
        out[s->nc + c] = s->t_act[c];
        out[2 * s->nc + c] = s->v_max[c];
        out[3 * s->nc + c] = s->t_rep[c];
    }
}

void orc_set_detect_state(orc_sim *s, const double *in)
{
    for (int64_t c = 0; c < s->nc; ++c) {
        s->status[c] = (uint8_t)in[c];
        s->t_act[c] = in[s->nc + c];
        s->v_max[c] = in[2 * s->nc + c];
        s->t_rep[c] = in[3 * s->nc + c];
    }
}

/* ---------------------------------------------------------- detection -- */
void orc_detect_waveform(const double *v, int64_t n, double dt,
                         double threshold, double repol_frac, double *t_act,
                         double *apd90)
{
    int status = 0;
    double ta = NAN, vmax = NAN, tr = NAN;
    const double vrest = n > 0 ? v[0] : NAN;
    for (int64_t i = 0; i + 1 < n; ++i) {
        const double a = v[i], b = v[i + 1];
        if (status == 0) {
            if (a <= threshold && b > threshold) {
                ta = ((double)i + (threshold - a) / (b - a)) * dt;
                vmax = b;
                status = 1;
            }
        } else if (status == 1) {
            if (b > vmax) vmax = b;
            const double v90 = vmax - repol_frac * (vmax - vrest);
            if (a >= v90 && b < v90) {
                tr = ((double)i + (a - v90) / (a - b)) * dt;
                status = 2;
            }
        }
    }
    *t_act = status ? ta : NAN;
    *apd90 = status == 2 ? tr - ta : NAN;
}

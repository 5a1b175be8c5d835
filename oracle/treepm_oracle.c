/*
 * FP64 CPU oracle for the short-range (PP) part of the TreePM force of Ishiyama, Fukushige &
 * Makino, "GreeM: Massively Parallel TreePM Code for Large Cosmological N-body Simulations"
 * (PASJ 2009, arXiv:0910.0121).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the library never does, and it shares no code, header, table or helper
 * with the library.
 *
 * Everything is IEEE FP64, round to nearest, compiled without FMA contraction, and summed
 * in the order stated at each function.
 *
 * What it computes, with the passage each part follows:
 *  - orc_g_p3m: the cutoff function g_P3M(R) of eq. (2) (Section 2.1), as printed.
 *  - orc_direct_brute / orc_direct_cells: the exact short-range force, i.e. the pair law of
 *    eq. (1) (Section 2.1) with Plummer softening (Section 2.4) summed over every other
 *    particle, minimum image in the periodic box (Section 1: the tree part differs from a
 *    non-periodic treecode only by the force law and the handling of images).  Two
 *    independent pair enumerations (all pairs; cell list with cell side >= r_cut).
 *  - orc_tree_*: the reference tree of Section 2.2 steps 2 and 5 -- Morton keys, stable key
 *    sort, octree with the N_leaf stopping rule (Section 3.1.2), node mass and centre of
 *    mass, Barnes' grouping with N_crit (Section 3.1.2), one shared interaction list per
 *    group under opening angle theta with cutoff pruning (Section 2.2 step 3 measures both
 *    from the surface of the receiving region), and the list force summed in FP64.
 *
 * Readings taken where the paper is silent (each also listed in the design notes):
 *  - softening: Plummer denominator (r^2+eps^2)^(3/2), g evaluated at the unsoftened r;
 *  - a pair with r == 0 (the self term, or coincident particles) contributes nothing;
 *  - keys: q = min(2^21-1, floor(x * (2^21/L))) per axis, interleaved x above y above z;
 *  - sort ties keep input order;
 *  - a node is subdivided iff count >= n_leaf and level < 21; children are the nonempty
 *    octants in octant order, no path compression;
 *  - a group is a maximal node that has count <= n_crit or is a leaf;
 *  - x_g (the coordinate origin of the FP32 kernel) is the group node's cube centre;
 *  - prune: periodic gap between the node cube and the group bbox >= r_cut;
 *  - accept: l^2 < theta^2 * d^2, d = distance from the node's centre of mass to the group
 *    bbox, and the node cube does not touch the bbox (gap > 0); a tie opens the node.
 *  - quadrupole cells (Section 4.1), when selected: a cell entry adds the second-order term
 *    of the expansion of the cut-off pair law about its centre of mass (pair_quad), with the
 *    node's second moment taken directly from its particles;
 *  - distance-dependent opening (Section 4.1, eq. 12), when selected: theta is replaced by
 *    theta(d) = min(theta_max, theta_0 / sqrt(R g_P3M(R))), R = d / eta -- the distance is
 *    measured in units of eta so that theta_0 is dimensionless, d is the same distance as in
 *    the fixed test, and theta(d) = theta_max where R g(R) = 0 (the upper limit the paper
 *    asks for, since the unlimited angle diverges at both ends of the range).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXLEVEL 21

/* ---------------------------------------------------------------- pair law (eq. 1, 2) */

/* Cutoff function g_P3M(R), eq. (2), written out as printed. */
double orc_g_p3m(double R)
{
    if (R < 0.0) return 1.0; /* R = r/eta >= 0 always; guard only */
    double R2 = R * R, R3 = R2 * R, R4 = R3 * R, R5 = R4 * R, R6 = R5 * R, R7 = R6 * R,
           R8 = R7 * R;
    if (R < 1.0)
        return 1.0 - (224.0 * R3 - 224.0 * R5 + 70.0 * R6 + 48.0 * R7 - 21.0 * R8) / 140.0;
    if (R < 2.0)
        return 1.0 - (12.0 - 224.0 * R2 + 896.0 * R3 - 840.0 * R4 + 224.0 * R5 + 70.0 * R6 -
                      48.0 * R7 + 7.0 * R8) / 140.0;
    return 0.0;
}

/* Minimum image of a coordinate difference v in (-L, L): result in [-L/2, L/2). */
static double wrap(double v, double L)
{
    double h = 0.5 * L;
    if (v >= h) return v - L;
    if (v < -h) return v + L;
    return v;
}

/* Distance-dependent opening angle of Section 4.1, eq. (12): the uniform-density error of
 * a node at distance r scales as r theta^2 g(r/eta), so theta_0 / sqrt(R g(R)) spreads it
 * evenly.  R = r / eta (distance in units of eta), capped at theta_max; where R g(R) = 0
 * (r = 0, r >= r_cut) the cap is the angle. */
double orc_theta_r(double r, double eta, double theta0, double theta_max)
{
    double R = r / eta;
    double s = R * orc_g_p3m(R);
    if (!(s > 0.0)) return theta_max;
    double th = theta0 / sqrt(s);
    return th < theta_max ? th : theta_max;
}

/* Acceleration at the field point from a source of mass m displaced by d (source minus
 * field point), eq. (1) with Plummer softening:  m d g(|d|/eta) / (|d|^2+eps^2)^(3/2).
 * Adds into acc[3].  A pair at zero separation contributes nothing. */
static void pair_acc(const double d[3], double m, double eta, double eps2, double acc[3])
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double g = orc_g_p3m(r / eta);
    if (g == 0.0) return;
    double s2 = r2 + eps2;
    double f = m * g / (s2 * sqrt(s2));
    acc[0] += f * d[0];
    acc[1] += f * d[1];
    acc[2] += f * d[2];
}

/* First and second derivatives of g_P3M(R) of eq. (2), differentiated term by term. */
void orc_g_p3m_derivs(double R, double *g1, double *g2)
{
    double R2 = R * R, R3 = R2 * R, R4 = R3 * R, R5 = R4 * R, R6 = R5 * R, R7 = R6 * R;
    if (R < 1.0) {
        *g1 = -(672.0 * R2 - 1120.0 * R4 + 420.0 * R5 + 336.0 * R6 - 168.0 * R7) / 140.0;
        *g2 = -(1344.0 * R - 4480.0 * R3 + 2100.0 * R4 + 2016.0 * R5 - 1176.0 * R6) / 140.0;
    } else if (R < 2.0) {
        *g1 = -(-448.0 * R + 2688.0 * R2 - 3360.0 * R3 + 1120.0 * R4 + 420.0 * R5 -
                336.0 * R6 + 56.0 * R7) / 140.0;
        *g2 = -(-448.0 + 5376.0 * R - 10080.0 * R2 + 4480.0 * R3 + 2100.0 * R4 - 2016.0 * R5 +
                392.0 * R6) / 140.0;
    } else {
        *g1 = 0.0;
        *g2 = 0.0;
    }
}

/* Second-order (quadrupole) term of a cell whose particles have second moment Q about its
 * centre of mass, at displacement d = com - field point (Section 4.1: the expansion of the
 * cut-off force must carry the derivatives of the cutoff function).  With the pair law
 * F(d) = d h(r), h = g(r/eta) (r^2+eps^2)^(-3/2), the sum over the cell's particles of
 * F(d + s_j), sum m_j s_j = 0, is M F(d) plus
 *     (1/2) Q_ab d_a d_b F_c = (Q d)_c u + (1/2) tr(Q) d_c u + (1/2) (d.Q.d) d_c w,
 *     u = h'/r,  w = (h'/r)'/r,
 * to second order in the particles' offsets s_j.  Adds into acc[3]. */
static void pair_quad(const double d[3], const double Q[6], double eta, double eps2,
                      double acc[3])
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2), R = r / eta;
    if (R >= 2.0) return;
    double g = orc_g_p3m(R), g1, g2;
    orc_g_p3m_derivs(R, &g1, &g2);
    double s2 = r2 + eps2, s1 = sqrt(s2);
    double q = 1.0 / (s2 * s1);         /* (r^2+eps^2)^(-3/2) */
    double p = q / s2;                  /* (r^2+eps^2)^(-5/2) */
    double s7 = p / s2;                 /* (r^2+eps^2)^(-7/2) */
    double u = g1 * q / (eta * r) - 3.0 * g * p;
    double w = g2 * q / (eta * eta * r2) - g1 * q / (eta * r2 * r) - 6.0 * g1 * p / (eta * r) +
               15.0 * g * s7;
    double Qd[3] = {Q[0] * d[0] + Q[3] * d[1] + Q[4] * d[2],
                    Q[3] * d[0] + Q[1] * d[1] + Q[5] * d[2],
                    Q[4] * d[0] + Q[5] * d[1] + Q[2] * d[2]};
    double trQ = Q[0] + Q[1] + Q[2];
    double dQd = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
    for (int a = 0; a < 3; ++a) acc[a] += Qd[a] * u + 0.5 * trQ * d[a] * u + 0.5 * dQd * d[a] * w;
}

/* Public: acceleration at xi from a cell of mass M, centre of mass com and second moment Q
 * (order 1: monopole only; order 2: with the quadrupole term), minimum image in box L. */
void orc_cell_acc(const double xi[3], const double com[3], double M, const double Q[6],
                  double L, double r_cut, double eps, int order, double out[3])
{
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = wrap(com[a] - xi[a], L);
    out[0] = out[1] = out[2] = 0.0;
    pair_acc(d, M, 0.5 * r_cut, eps * eps, out);
    if (order >= 2) pair_quad(d, Q, 0.5 * r_cut, eps * eps, out);
}

/* |pair force| of the same pair, and the same magnitude without the cutoff factor g, for
 * condition-aware tolerances: adds into *mag and *newt.  The expanded polynomial of eq. (2)
 * sums terms up to ~300 in size near R = 2, so its rounding error is a few 1e-14 of the
 * uncut magnitude, not of |f|. */
static void pair_mag(const double d[3], double m, double eta, double eps2, double *mag,
                     double *newt)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double s2 = r2 + eps2;
    double nm = m * r / (s2 * sqrt(s2));
    *mag += orc_g_p3m(r / eta) * nm;
    *newt += nm;
}

/* Public single-pair evaluation (tests): acceleration at (xi) from (xj, m) in box L. */
void orc_pair(const double xi[3], const double xj[3], double m, double L, double r_cut,
              double eps, double out[3])
{
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = wrap(xj[a] - xi[a], L);
    out[0] = out[1] = out[2] = 0.0;
    pair_acc(d, m, 0.5 * r_cut, eps * eps, out);
}

/* ---------------------------------------------------------------- exact short-range sums */

/* O(N^2): a_i = sum over j != i, j in input order, of the pair law with minimum image. */
int orc_direct_brute(int64_t n, const double *x, const double *y, const double *z,
                     const double *m, double L, double r_cut, double eps, double *ax,
                     double *ay, double *az, int nthreads)
{
    double eta = 0.5 * r_cut, eps2 = eps * eps;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {wrap(x[j] - x[i], L), wrap(y[j] - y[i], L), wrap(z[j] - z[i], L)};
            pair_acc(d, m[j], eta, eps2, acc);
        }
        ax[i] = acc[0];
        ay[i] = acc[1];
        az[i] = acc[2];
    }
    return 0;
}

/* Same pair set through a cell list: nc = floor(L / r_cut) cells per side (side >= r_cut),
 * so every pair closer than r_cut is in the 27-cell neighbourhood.  Requires nc >= 3 so the
 * 27 neighbour cells are distinct.  Returns -1 if nc < 3. */
int orc_direct_cells(int64_t n, const double *x, const double *y, const double *z,
                     const double *m, double L, double r_cut, double eps, double *ax,
                     double *ay, double *az, int nthreads)
{
    int64_t nc = (int64_t)floor(L / r_cut);
    if (nc < 3) return -1;
    if (nc > 512) nc = 512;
    int64_t ncell = nc * nc * nc;
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *members = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cell_of || !head || !members) {
        free(cell_of); free(head); free(members);
        return -2;
    }
    memset(head, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        double p[3] = {x[i], y[i], z[i]};
        for (int a = 0; a < 3; ++a) {
            c[a] = (int64_t)floor(p[a] / L * (double)nc);
            if (c[a] < 0) c[a] = 0;
            if (c[a] >= nc) c[a] = nc - 1;
        }
        cell_of[i] = (c[0] * nc + c[1]) * nc + c[2];
        head[cell_of[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        memcpy(fill, head, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) members[fill[cell_of[i]]++] = i;
        free(fill);
    }
    double eta = 0.5 * r_cut, eps2 = eps * eps;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int64_t ci = cell_of[i];
        int64_t cx = ci / (nc * nc), cy = (ci / nc) % nc, cz = ci % nc;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t qx = (cx + dx + nc) % nc, qy = (cy + dy + nc) % nc,
                            qz = (cz + dz + nc) % nc;
                    int64_t q = (qx * nc + qy) * nc + qz;
                    for (int64_t k = head[q]; k < head[q + 1]; ++k) {
                        int64_t j = members[k];
                        if (j == i) continue;
                        double d[3] = {wrap(x[j] - x[i], L), wrap(y[j] - y[i], L),
                                       wrap(z[j] - z[i], L)};
                        pair_acc(d, m[j], eta, eps2, acc);
                    }
                }
        ax[i] = acc[0];
        ay[i] = acc[1];
        az[i] = acc[2];
    }
    free(cell_of); free(head); free(members);
    return 0;
}

/* ---------------------------------------------------------------- reference tree */

typedef struct {
    uint64_t code;      /* (1 << 3*level) | key prefix of length 3*level bits          */
    int level;
    uint32_t ix, iy, iz; /* integer cube coordinates at this level                     */
    int64_t first, count; /* range in key-sorted particle order                        */
    int64_t child_first; /* index of first child in the node array, -1 for a leaf     */
    int nchild;
    double mass, S[3], com[3];
    double Q[6];        /* second moment about com: xx, yy, zz, xy, xz, yz (quadrupole)  */
} onode;

typedef struct {
    int64_t node, first, count;
    double lo[3], hi[3], cg[3], hg[3], xg[3];
} ogroup;

typedef struct {
    /* parameters */
    double L, r_cut, eps, theta;
    int n_leaf, n_crit;
    int opening;        /* 0: fixed theta; 1: theta(d) of eq. (12), theta = theta_0        */
    double theta_max;   /* upper limit of theta(d) (opening 1)                           */
    int quadrupole;     /* cell entries also carry their second-order term (Section 4.1) */
    /* particles */
    int64_t n;
    uint64_t *key;      /* sorted keys                                                  */
    int64_t *idx;       /* input index of the k-th particle in key order                */
    double *px, *py, *pz, *pm; /* sorted FP64 positions and masses                      */
    /* tree */
    onode *nodes;
    int64_t n_nodes, cap_nodes;
    /* groups and lists */
    ogroup *groups;
    int64_t n_groups, cap_groups;
    int64_t *list_off;  /* n_groups + 1                                                 */
    int64_t *list;      /* entry: node index (cell) or sorted particle index (particle) */
    uint8_t *list_is_cell;
    int64_t n_entries, cap_entries;
    int walked;
} otree;

static uint64_t key_of(double x, double y, double z, double L)
{
    double s = 2097152.0 / L; /* 2^21 / L */
    double p[3] = {x, y, z};
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        double f = floor(p[a] * s);
        uint64_t v = (f <= 0.0) ? 0 : (uint64_t)f;
        if (v > 2097151u) v = 2097151u;
        q[a] = v;
    }
    uint64_t k = 0;
    for (int b = 0; b < 21; ++b) {
        k |= ((q[0] >> b) & 1u) << (3 * b + 2);
        k |= ((q[1] >> b) & 1u) << (3 * b + 1);
        k |= ((q[2] >> b) & 1u) << (3 * b);
    }
    return k;
}

typedef struct {
    uint64_t key;
    int64_t idx;
} kpair;

static int cmp_kpair(const void *a, const void *b)
{
    const kpair *p = (const kpair *)a, *q = (const kpair *)b;
    if (p->key < q->key) return -1;
    if (p->key > q->key) return 1;
    /* equal keys: input order (makes the sort stable) */
    return (p->idx < q->idx) ? -1 : (p->idx > q->idx) ? 1 : 0;
}

static int64_t push_node(otree *t)
{
    if (t->n_nodes == t->cap_nodes) {
        int64_t nc = t->cap_nodes ? 2 * t->cap_nodes : 1024;
        onode *p = (onode *)realloc(t->nodes, sizeof(onode) * (size_t)nc);
        if (!p) return -1;
        t->nodes = p;
        t->cap_nodes = nc;
    }
    memset(&t->nodes[t->n_nodes], 0, sizeof(onode));
    return t->n_nodes++;
}

/* Subdivide node u (already allocated) if count >= n_leaf and level < 21: its children are
 * the nonempty octants, in octant order, stored contiguously; then recurse into each. */
static int build_rec(otree *t, int64_t u)
{
    onode nd = t->nodes[u];
    if (nd.count < t->n_leaf || nd.level >= ORC_MAXLEVEL) {
        t->nodes[u].child_first = -1;
        t->nodes[u].nchild = 0;
        return 0;
    }
    int shift = 3 * (ORC_MAXLEVEL - (nd.level + 1));
    int64_t start[8], cnt[8];
    for (int o = 0; o < 8; ++o) { start[o] = -1; cnt[o] = 0; }
    for (int64_t k = nd.first; k < nd.first + nd.count; ++k) {
        int o = (int)((t->key[k] >> shift) & 7u);
        if (start[o] < 0) start[o] = k;
        cnt[o]++;
    }
    int nchild = 0;
    for (int o = 0; o < 8; ++o) nchild += (cnt[o] > 0);
    int64_t cf = t->n_nodes;
    for (int o = 0; o < 8; ++o) {
        if (!cnt[o]) continue;
        int64_t c = push_node(t);
        if (c < 0) return -1;
        onode *ch = &t->nodes[c];
        ch->level = nd.level + 1;
        ch->code = (nd.code << 3) | (uint64_t)o;
        ch->ix = 2u * nd.ix + (uint32_t)((o >> 2) & 1);
        ch->iy = 2u * nd.iy + (uint32_t)((o >> 1) & 1);
        ch->iz = 2u * nd.iz + (uint32_t)(o & 1);
        ch->first = start[o];
        ch->count = cnt[o];
    }
    t->nodes[u].child_first = cf;
    t->nodes[u].nchild = nchild;
    for (int c = 0; c < nchild; ++c)
        if (build_rec(t, cf + c)) return -1;
    return 0;
}

/* Node mass and centre of mass, bottom up.  Leaf: M = sum m_k and S = sum m_k x_k over its
 * particles in key order; internal node: M and S summed over its children in octant order;
 * com = S / M. */
static void moments_rec(otree *t, int64_t u)
{
    onode *nd = &t->nodes[u];
    double M = 0.0, S[3] = {0.0, 0.0, 0.0};
    if (nd->nchild == 0) {
        for (int64_t k = nd->first; k < nd->first + nd->count; ++k) {
            double mk = t->pm[k];
            M += mk;
            S[0] += mk * t->px[k];
            S[1] += mk * t->py[k];
            S[2] += mk * t->pz[k];
        }
    } else {
        for (int c = 0; c < nd->nchild; ++c) {
            moments_rec(t, nd->child_first + c);
            onode *ch = &t->nodes[nd->child_first + c];
            M += ch->mass;
            S[0] += ch->S[0];
            S[1] += ch->S[1];
            S[2] += ch->S[2];
        }
        nd = &t->nodes[u];
    }
    nd->mass = M;
    for (int a = 0; a < 3; ++a) {
        nd->S[a] = S[a];
        nd->com[a] = S[a] / M;
    }
}

static int push_group(otree *t, int64_t u)
{
    if (t->n_groups == t->cap_groups) {
        int64_t nc = t->cap_groups ? 2 * t->cap_groups : 256;
        ogroup *p = (ogroup *)realloc(t->groups, sizeof(ogroup) * (size_t)nc);
        if (!p) return -1;
        t->groups = p;
        t->cap_groups = nc;
    }
    onode *nd = &t->nodes[u];
    ogroup *g = &t->groups[t->n_groups++];
    g->node = u;
    g->first = nd->first;
    g->count = nd->count;
    double lo[3] = {t->px[nd->first], t->py[nd->first], t->pz[nd->first]};
    double hi[3] = {lo[0], lo[1], lo[2]};
    for (int64_t k = nd->first; k < nd->first + nd->count; ++k) {
        double p[3] = {t->px[k], t->py[k], t->pz[k]};
        for (int a = 0; a < 3; ++a) {
            if (p[a] < lo[a]) lo[a] = p[a];
            if (p[a] > hi[a]) hi[a] = p[a];
        }
    }
    double l = ldexp(t->L, -nd->level);
    uint32_t ic[3] = {nd->ix, nd->iy, nd->iz};
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = lo[a];
        g->hi[a] = hi[a];
        g->cg[a] = (lo[a] + hi[a]) * 0.5;
        g->hg[a] = (hi[a] - lo[a]) * 0.5;
        g->xg[a] = ((double)ic[a] + 0.5) * l;
    }
    return 0;
}

/* Groups: walking down from the root, the first node on each path that is a leaf or holds at
 * most n_crit particles.  Visited in octant order, so groups come out in key order. */
static int groups_rec(otree *t, int64_t u)
{
    onode *nd = &t->nodes[u];
    if (nd->nchild == 0 || nd->count <= t->n_crit) return push_group(t, u);
    int64_t cf = nd->child_first;
    int nc = nd->nchild;
    for (int c = 0; c < nc; ++c)
        if (groups_rec(t, cf + c)) return -1;
    return 0;
}

otree *orc_tree_build(int64_t n, const double *x, const double *y, const double *z,
                      const double *m, double L, double r_cut, double eps, double theta,
                      int n_leaf, int n_crit)
{
    if (n < 1 || n_leaf < 2 || n_crit < 1 || !(L > 0.0)) return NULL;
    otree *t = (otree *)calloc(1, sizeof(otree));
    if (!t) return NULL;
    t->L = L; t->r_cut = r_cut; t->eps = eps; t->theta = theta;
    t->n_leaf = n_leaf; t->n_crit = n_crit; t->n = n;
    kpair *kp = (kpair *)malloc(sizeof(kpair) * (size_t)n);
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    t->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t->px = (double *)malloc(sizeof(double) * (size_t)n);
    t->py = (double *)malloc(sizeof(double) * (size_t)n);
    t->pz = (double *)malloc(sizeof(double) * (size_t)n);
    t->pm = (double *)malloc(sizeof(double) * (size_t)n);
    if (!kp || !t->key || !t->idx || !t->px || !t->py || !t->pz || !t->pm) goto fail;
    for (int64_t i = 0; i < n; ++i) {
        kp[i].key = key_of(x[i], y[i], z[i], L);
        kp[i].idx = i;
    }
    qsort(kp, (size_t)n, sizeof(kpair), cmp_kpair);
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = kp[k].idx;
        t->key[k] = kp[k].key;
        t->idx[k] = i;
        t->px[k] = x[i];
        t->py[k] = y[i];
        t->pz[k] = z[i];
        t->pm[k] = m[i];
    }
    free(kp);
    kp = NULL;
    {
        int64_t r = push_node(t);
        if (r < 0) goto fail;
        t->nodes[r].code = 1;
        t->nodes[r].level = 0;
        t->nodes[r].first = 0;
        t->nodes[r].count = n;
        if (build_rec(t, 0)) goto fail;
    }
    moments_rec(t, 0);
    if (groups_rec(t, 0)) goto fail;
    return t;
fail:
    free(kp);
    free(t->key); free(t->idx); free(t->px); free(t->py); free(t->pz); free(t->pm);
    free(t->nodes); free(t->groups);
    free(t);
    return NULL;
}

void orc_tree_free(otree *t)
{
    if (!t) return;
    free(t->key); free(t->idx); free(t->px); free(t->py); free(t->pz); free(t->pm);
    free(t->nodes); free(t->groups);
    free(t->list_off); free(t->list); free(t->list_is_cell);
    free(t);
}

/* Second moments of every node about its centre of mass, from its particles directly:
 * Q = sum_k m_k (x_k - com)(x_k - com)^T over the node's range in key order (a node is a
 * sub-cube of [0, L), so no image is needed). */
static void second_moments(otree *t)
{
    for (int64_t u = 0; u < t->n_nodes; ++u) {
        onode *nd = &t->nodes[u];
        double Q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t k = nd->first; k < nd->first + nd->count; ++k) {
            double dx = t->px[k] - nd->com[0], dy = t->py[k] - nd->com[1],
                   dz = t->pz[k] - nd->com[2], m = t->pm[k];
            Q[0] += m * dx * dx;
            Q[1] += m * dy * dy;
            Q[2] += m * dz * dz;
            Q[3] += m * dx * dy;
            Q[4] += m * dx * dz;
            Q[5] += m * dy * dz;
        }
        for (int a = 0; a < 6; ++a) nd->Q[a] = Q[a];
    }
}

/* Cell entries with (1) or without (0) their quadrupole term in the list force.  The lists
 * do not change.  Returns 0, or -1 for an invalid value. */
int orc_tree_set_quadrupole(otree *t, int on)
{
    if (!t || on < 0 || on > 1) return -1;
    if (on && !t->quadrupole) second_moments(t);
    t->quadrupole = on;
    return 0;
}

/* Second moments of the nodes (n_nodes x 6: xx, yy, zz, xy, xz, yz), node array order. */
void orc_tree_nodes_q(otree *t, double *Q)
{
    second_moments(t);
    for (int64_t u = 0; u < t->n_nodes; ++u)
        for (int a = 0; a < 6; ++a) Q[6 * u + a] = t->nodes[u].Q[a];
}

/* Select the opening criterion: 0 = fixed theta (the build's theta); 1 = theta(d) of
 * eq. (12) with theta_0 = the build's theta and the cap theta_max.  Drops earlier lists.
 * Returns 0, or -1 for an invalid choice. */
int orc_tree_set_opening(otree *t, int opening, double theta_max)
{
    if (!t || opening < 0 || opening > 1 || !(theta_max >= 0.0)) return -1;
    t->opening = opening;
    t->theta_max = theta_max;
    free(t->list_off); free(t->list); free(t->list_is_cell);
    t->list_off = NULL; t->list = NULL; t->list_is_cell = NULL;
    t->n_entries = 0;
    t->walked = 0;
    return 0;
}

/* Replace the opening angle theta (theta_0 under the distance-dependent opening); the tree and
 * groups do not depend on it.  Drops earlier lists.  Returns 0, or -1 for theta outside
 * [0, 1]. */
int orc_tree_set_theta(otree *t, double theta)
{
    if (!t || !(theta >= 0.0 && theta <= 1.0)) return -1;
    t->theta = theta;
    free(t->list_off); free(t->list); free(t->list_is_cell);
    t->list_off = NULL; t->list = NULL; t->list_is_cell = NULL;
    t->n_entries = 0;
    t->walked = 0;
    return 0;
}

/* ------------------------------------------------ walk: one interaction list per group */

typedef struct {
    int64_t *e;
    uint8_t *c;
    int64_t n, cap;
} elist;

static int elist_push(elist *l, int64_t v, uint8_t is_cell)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 1024;
        int64_t *pe = (int64_t *)realloc(l->e, sizeof(int64_t) * (size_t)nc);
        if (!pe) return -1;
        l->e = pe;
        uint8_t *pc = (uint8_t *)realloc(l->c, (size_t)nc);
        if (!pc) return -1;
        l->c = pc;
        l->cap = nc;
    }
    l->e[l->n] = v;
    l->c[l->n] = is_cell;
    l->n++;
    return 0;
}

/* Visit node u for group g, in depth-first octant order:
 *   prune  : gap_a = max(0, |wrap(cn_a - cg_a)| - (l/2 + hg_a)),  sum gap^2 >= r_cut^2
 *   accept : dc_a  = max(0, |wrap(com_a - cg_a)| - hg_a),   l^2 < theta^2 sum dc^2, gap^2 > 0
 *            (theta = theta(d), d = sqrt(sum dc^2), under the distance-dependent opening)
 *   leaf   : one particle entry per particle, key order
 *   else   : visit the children. */
static int walk_rec(const otree *t, const ogroup *g, int64_t u, double rc2, double th2,
                    elist *out)
{
    const onode *nd = &t->nodes[u];
    double l = ldexp(t->L, -nd->level);
    double half = l * 0.5;
    uint32_t ic[3] = {nd->ix, nd->iy, nd->iz};
    double gap[3], dc[3];
    for (int a = 0; a < 3; ++a) {
        double cn = ((double)ic[a] + 0.5) * l;
        double v = fabs(wrap(cn - g->cg[a], t->L)) - (half + g->hg[a]);
        gap[a] = v > 0.0 ? v : 0.0;
    }
    double G = gap[0] * gap[0] + gap[1] * gap[1] + gap[2] * gap[2];
    if (G >= rc2) return 0;
    for (int a = 0; a < 3; ++a) {
        double v = fabs(wrap(nd->com[a] - g->cg[a], t->L)) - g->hg[a];
        dc[a] = v > 0.0 ? v : 0.0;
    }
    double D = dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2];
    if (t->opening) {
        double th = orc_theta_r(sqrt(D), 0.5 * t->r_cut, t->theta, t->theta_max);
        th2 = th * th;
    }
    if (l * l < th2 * D && G > 0.0) return elist_push(out, u, 1);
    if (nd->nchild == 0) {
        for (int64_t k = nd->first; k < nd->first + nd->count; ++k)
            if (elist_push(out, k, 0)) return -1;
        return 0;
    }
    for (int c = 0; c < nd->nchild; ++c)
        if (walk_rec(t, g, nd->child_first + c, rc2, th2, out)) return -1;
    return 0;
}

/* Build the interaction list of every group.  Returns total entries, or -1. */
int64_t orc_tree_walk(otree *t)
{
    if (!t) return -1;
    if (t->walked) return t->n_entries;
    double rc2 = t->r_cut * t->r_cut, th2 = t->theta * t->theta;
    elist all = {0};
    t->list_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(t->n_groups + 1));
    if (!t->list_off) return -1;
    t->list_off[0] = 0;
    for (int64_t gi = 0; gi < t->n_groups; ++gi) {
        if (walk_rec(t, &t->groups[gi], 0, rc2, th2, &all)) {
            free(all.e); free(all.c);
            return -1;
        }
        t->list_off[gi + 1] = all.n;
    }
    t->list = all.e;
    t->list_is_cell = all.c;
    t->n_entries = all.n;
    t->walked = 1;
    return all.n;
}

/* Source position and mass of a list entry. */
static void entry_source(const otree *t, int64_t e, uint8_t is_cell, double p[3], double *m)
{
    if (is_cell) {
        const onode *nd = &t->nodes[e];
        p[0] = nd->com[0]; p[1] = nd->com[1]; p[2] = nd->com[2];
        *m = nd->mass;
    } else {
        p[0] = t->px[e]; p[1] = t->py[e]; p[2] = t->pz[e];
        *m = t->pm[e];
    }
}

/* Walk one group into a private list and sum its force (used by the sampled timing path,
 * which does not keep lists).  Returns entries, or -1. */
static int64_t group_force(const otree *t, int64_t gi, const int64_t *ent, const uint8_t *isc,
                           int64_t ne, double *ax, double *ay, double *az)
{
    const ogroup *g = &t->groups[gi];
    double eta = 0.5 * t->r_cut, eps2 = t->eps * t->eps;
    for (int64_t k = g->first; k < g->first + g->count; ++k) {
        double xi[3] = {t->px[k], t->py[k], t->pz[k]};
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t q = 0; q < ne; ++q) {
            double p[3], mj;
            entry_source(t, ent[q], isc[q], p, &mj);
            double d[3] = {wrap(p[0] - xi[0], t->L), wrap(p[1] - xi[1], t->L),
                           wrap(p[2] - xi[2], t->L)};
            pair_acc(d, mj, eta, eps2, acc);
            if (t->quadrupole && isc[q]) pair_quad(d, t->nodes[ent[q]].Q, eta, eps2, acc);
        }
        int64_t i = t->idx[k];
        ax[i] = acc[0];
        ay[i] = acc[1];
        az[i] = acc[2];
    }
    return ne;
}

/* Sum over each particle's list of the pair-force magnitudes, sum_j |f_ij|, and of the same
 * magnitudes without g (input order): the scales of rounding error in the list force, for
 * condition-aware comparisons. */
int orc_tree_force_mag(otree *t, double *mag, double *newt, int nthreads)
{
    if (!t) return -1;
    if (orc_tree_walk(t) < 0) return -1;
    double eta = 0.5 * t->r_cut, eps2 = t->eps * t->eps;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t gi = 0; gi < t->n_groups; ++gi) {
        const ogroup *g = &t->groups[gi];
        for (int64_t k = g->first; k < g->first + g->count; ++k) {
            double s = 0.0, sn = 0.0;
            for (int64_t q = t->list_off[gi]; q < t->list_off[gi + 1]; ++q) {
                double p[3], mj;
                entry_source(t, t->list[q], t->list_is_cell[q], p, &mj);
                double d[3] = {wrap(p[0] - t->px[k], t->L), wrap(p[1] - t->py[k], t->L),
                               wrap(p[2] - t->pz[k], t->L)};
                pair_mag(d, mj, eta, eps2, &s, &sn);
            }
            mag[t->idx[k]] = s;
            newt[t->idx[k]] = sn;
        }
    }
    return 0;
}

/* List force for every particle (output in input order), from the lists of orc_tree_walk.
 * Each particle's sum runs over its group's list in list order. */
int orc_tree_force(otree *t, double *ax, double *ay, double *az, int nthreads)
{
    if (!t) return -1;
    if (orc_tree_walk(t) < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t gi = 0; gi < t->n_groups; ++gi) {
        int64_t o = t->list_off[gi];
        group_force(t, gi, t->list + o, t->list_is_cell + o, t->list_off[gi + 1] - o, ax, ay,
                    az);
    }
    return 0;
}

/* Walk and list force for the groups gi = offset, offset+stride, ... only (a stratified
 * sample in key order), each group's list built privately.  Forces of sampled particles are
 * written (input order); others are untouched.  If mag and newt are non-NULL they receive,
 * for the sampled particles, sum_j |f_ij| and the same sum without g (see
 * orc_tree_force_mag).  Returns the number of pair interactions (sum over sampled groups of
 * count * list length), or -1. */
int64_t orc_tree_walk_force_sample(otree *t, int64_t stride, int64_t offset, double *ax,
                                   double *ay, double *az, int nthreads,
                                   int64_t *particles_out, double *mag, double *newt)
{
    if (!t || stride < 1 || offset < 0) return -1;
    double rc2 = t->r_cut * t->r_cut, th2 = t->theta * t->theta;
    double eta = 0.5 * t->r_cut, eps2 = t->eps * t->eps;
    int64_t inter = 0, parts = 0;
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : inter, parts)
#endif
    for (int64_t gi = offset; gi < t->n_groups; gi += stride) {
        elist l = {0};
        if (walk_rec(t, &t->groups[gi], 0, rc2, th2, &l)) {
            fail = 1;
        } else {
            group_force(t, gi, l.e, l.c, l.n, ax, ay, az);
            inter += l.n * t->groups[gi].count;
            parts += t->groups[gi].count;
            if (mag && newt) {
                const ogroup *g = &t->groups[gi];
                for (int64_t k = g->first; k < g->first + g->count; ++k) {
                    double s = 0.0, sn = 0.0;
                    for (int64_t q = 0; q < l.n; ++q) {
                        double p[3], mj;
                        entry_source(t, l.e[q], l.c[q], p, &mj);
                        double d[3] = {wrap(p[0] - t->px[k], t->L), wrap(p[1] - t->py[k], t->L),
                                       wrap(p[2] - t->pz[k], t->L)};
                        pair_mag(d, mj, eta, eps2, &s, &sn);
                    }
                    mag[t->idx[k]] = s;
                    newt[t->idx[k]] = sn;
                }
            }
        }
        free(l.e);
        free(l.c);
    }
    if (particles_out) *particles_out = parts;
    return fail ? -1 : inter;
}

/* ---------------------------------------------------------------- exports for the tests */

int64_t orc_tree_n_nodes(const otree *t) { return t ? t->n_nodes : -1; }
int64_t orc_tree_n_groups(const otree *t) { return t ? t->n_groups : -1; }
int64_t orc_tree_n_entries(otree *t) { return orc_tree_walk(t); }

/* Sorted keys and the input index of each sorted particle. */
void orc_tree_sorted(const otree *t, uint64_t *key, int64_t *idx)
{
    memcpy(key, t->key, sizeof(uint64_t) * (size_t)t->n);
    memcpy(idx, t->idx, sizeof(int64_t) * (size_t)t->n);
}

/* Node arrays (depth-first allocation order): code, first, count, nchild, mass, com. */
void orc_tree_nodes(const otree *t, uint64_t *code, int64_t *first, int64_t *count,
                    int32_t *nchild, double *mass, double *comx, double *comy, double *comz)
{
    for (int64_t u = 0; u < t->n_nodes; ++u) {
        const onode *nd = &t->nodes[u];
        code[u] = nd->code;
        first[u] = nd->first;
        count[u] = nd->count;
        nchild[u] = nd->nchild;
        mass[u] = nd->mass;
        comx[u] = nd->com[0];
        comy[u] = nd->com[1];
        comz[u] = nd->com[2];
    }
}

/* Groups in key order: node code, first, count, and bbox/centres (3 doubles each). */
void orc_tree_groups(const otree *t, uint64_t *code, int64_t *first, int64_t *count,
                     double *lo, double *hi, double *xg)
{
    for (int64_t g = 0; g < t->n_groups; ++g) {
        const ogroup *gr = &t->groups[g];
        code[g] = t->nodes[gr->node].code;
        first[g] = gr->first;
        count[g] = gr->count;
        for (int a = 0; a < 3; ++a) {
            lo[3 * g + a] = gr->lo[a];
            hi[3 * g + a] = gr->hi[a];
            xg[3 * g + a] = gr->xg[a];
        }
    }
}

/* Lists in canonical form: offsets[n_groups+1]; per entry is_cell and value, where a cell
 * entry's value is the node code and a particle entry's value is the particle's input
 * index. */
int orc_tree_lists(otree *t, int64_t *offsets, uint8_t *is_cell, uint64_t *value)
{
    if (orc_tree_walk(t) < 0) return -1;
    for (int64_t g = 0; g <= t->n_groups; ++g) offsets[g] = t->list_off[g];
    for (int64_t q = 0; q < t->n_entries; ++q) {
        is_cell[q] = t->list_is_cell[q];
        value[q] = t->list_is_cell[q] ? t->nodes[t->list[q]].code
                                      : (uint64_t)t->idx[t->list[q]];
    }
    return 0;
}

/* Interaction count: sum over groups of count * list length. */
int64_t orc_tree_interactions(otree *t)
{
    if (orc_tree_walk(t) < 0) return -1;
    int64_t s = 0;
    for (int64_t g = 0; g < t->n_groups; ++g)
        s += t->groups[g].count * (t->list_off[g + 1] - t->list_off[g]);
    return s;
}

/* Morton key of one position (tests). */
uint64_t orc_key(double x, double y, double z, double L) { return key_of(x, y, z, L); }

/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the angular-momentum-conserving
 * Fast Multipole force evaluation of Korobkin et al., "Conservation of Angular
 * Momentum in the Fast Multipole Method" (arXiv:2107.07166).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the solver never does, and
 * nothing here is shared with the GPU path.
 *
 * What it computes, in the paper's notation (Sec. 2):
 *   nodes A, B with centres of mass Z_A, Z_B; R = Z_A - Z_B;
 *   particle a in A at X_a, x_a = X_a - Z_A; particle b in B at Y_b,
 *   y_b = Y_b - Z_B; delta = x_a - y_b, so X_a - Y_b = R + delta.
 *
 * The softened kernel is phi(r) = -(|r|^2 + eps^2)^(-1/2) (G factored out),
 * whose gradient is r g(r) with g(r) = (|r|^2 + eps^2)^(-3/2).
 *
 * Far-field pair acceleration of a due to b, for a node pair accepted by the
 * multipole acceptance criterion (Eq. mac_criterion), with the Taylor series
 * of Eq. taylor truncated at total degree p in delta:
 *   standard  : a = -m_b grad_delta T_p[phi](R; delta)
 *             = -m_b ( R T_{p-1}[g](R; delta) + delta T_{p-2}[g](R; delta) )
 *   conserving: the standard force projected onto n_ab (Eq. realign) with the
 *               projection scalar (a . u)/|u|^2, u = X_a - Y_b, expanded in
 *               delta (Eqs. nab-expansion, abnab-expansion) and truncated at
 *               degree p-1, the force's own degree; this is exactly
 *             = -m_b T_{p-1}[g](R; delta) (R + delta)
 *               which is central and antisymmetric, so pair torques vanish.
 *   conserving with the scalar kept to a higher degree K > p-1 (Sec. 3.2
 *               allows more terms of the expansion of the scalar): along
 *               delta -> t delta the standard force a(t) and u(t) = R + t delta
 *               are polynomials in t, 1/|u(t)|^2 a power series; the scalar's
 *               series is their product, summed to t^K at t = 1:
 *             = (sum_{n<=K} [t^n] (a(t).u(t)) / |u(t)|^2) (R + delta).
 *               The standard force's own truncation error enters the scalar
 *               from degree p on, so this is not the order K+1 force.
 *   conserving_r2 (zeroth order only, p = 1): the magnitude of the zeroth-
 *               order acceleration along n_ab (Eq. realign2), with n_ab
 *               expanded to first order in delta / |R| as in Eq.
 *               nab-expansion (the sum over b gives Eq. aaB0):
 *             = -m_b |grad phi(R)| (1 - n_R . delta / |R|)(n_R + delta / |R|)
 *             = -m_b (R.R + eps^2)^(-3/2) (1 - R . delta / |R|^2) (R + delta)
 *               with |grad phi(R)| = |R| (R.R + eps^2)^(-3/2), the softened
 *               zeroth-order magnitude (the paper writes the unsoftened
 *               1 / |R|^2); also central and antisymmetric.
 * T_k[f](R; delta) is the Taylor polynomial of total degree k of f about R,
 * evaluated at R + delta.  Its degree-n part is the coefficient of t^n in
 * f(R + t delta) = (c0 + c1 t + c2 t^2)^alpha with c0 = R.R + eps^2,
 * c1 = 2 R.delta, c2 = delta.delta, alpha = -3/2 for g (-1/2 for phi).  Those
 * univariate coefficients obey the power-of-a-series recurrence used in
 * orc_series.
 *
 * The near field (pairs of leaves the criterion rejects) is the exact softened
 * pair force, the gradient of Eq. jia.  Every unordered particle pair is
 * covered exactly once, either by a near pair of leaves or by one accepted
 * node pair, so theta = 0 reproduces the direct sum.
 *
 * Tree, keys and walk (the paper is silent on these; readings adopted):
 *   keys  : 21 bits per axis, q_d = min(2^21 - 1, floor((X_d - lo_d) * scale)),
 *           scale = 2^21 / ext, ext = max_d(hi_d - lo_d) (1 if zero);
 *           key bit 3i+2 = bit i of q_x, 3i+1 of q_y, 3i of q_z.
 *   order : stable sort by key (ties keep the input order).
 *   octree: node (level l, prefix = key >> 3(21-l)); a node with more than
 *           n_leaf particles and l < 21 gets its non-empty octants as
 *           children in digit order; nodes are numbered level by level, each
 *           level in Morton order.
 *   geometry (FP64, this exact operation order; no contraction):
 *           leaf: M = sum m, S = sum m X left to right over its particles;
 *           inner node: M, S summed over children in digit order; Z = S / M;
 *           r_max = sqrt(max over the node's particles of
 *                        ((dx*dx + dy*dy) + dz*dz)), d = X - Z.
 *   walk  : mutual dual-tree walk from (root, root).  Self pair: a leaf gives
 *           a near pair with itself, else children pairs (c_i, c_j), i <= j.
 *           Distinct pair: R = sqrt(same-order |Z_A - Z_B|^2); accepted
 *           (far pair) iff R > 0 and r_A + r_B <= theta * R (theta is
 *           tan(theta_MAC) of Eq. mac_criterion); else two leaves give a near
 *           pair; else split one node: the non-leaf if one is a leaf, else the
 *           larger r_max, then the lower level, then the lower node index.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.  OpenMP runs over
 * target particles only and every particle's sum has a fixed order, so the
 * results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LEVELS 21
#define ORC_QMAX ((1u << ORC_LEVELS) - 1u)

enum { ORC_STANDARD = 0, ORC_CONSERVING = 1, ORC_CONSERVING_R2 = 2 };

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated summation                                            */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double nsum_get(const nsum *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Direct sum: the gradient of Eq. jia with Plummer softening.               */
/* ------------------------------------------------------------------------ */
int orc_direct(int64_t n, const double *pos, const double *mass, double eps,
               double G, double *force, double *pot)
{
    if (n < 1 || !pos || !mass || !force) return -1;
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n; ++a) {
        nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, ph = {0, 0};
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double dx = pos[3 * a + 0] - pos[3 * b + 0];
            double dy = pos[3 * a + 1] - pos[3 * b + 1];
            double dz = pos[3 * a + 2] - pos[3 * b + 2];
            double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
            if (r2 == 0.0) continue; /* coincident and unsoftened: no force */
            double r = sqrt(r2);
            double w = mass[b] / (r2 * r);
            nsum_add(&fx, -w * dx);
            nsum_add(&fy, -w * dy);
            nsum_add(&fz, -w * dz);
            nsum_add(&ph, -mass[b] / r);
        }
        double s = G * mass[a];
        force[3 * a + 0] = s * nsum_get(&fx);
        force[3 * a + 1] = s * nsum_get(&fy);
        force[3 * a + 2] = s * nsum_get(&fz);
        if (pot) pot[a] = G * nsum_get(&ph);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Univariate Taylor coefficients of (c0 + c1 t + c2 t^2)^alpha.             */
/* With u(t) = c0 + c1 t + c2 t^2 and w = u^alpha, u w' = alpha u' w gives,  */
/* at t^(n-1):                                                               */
/*   n c0 w_n = (alpha - (n-1)) c1 w_{n-1} + (2 alpha - (n-2)) c2 w_{n-2}.    */
/* ------------------------------------------------------------------------ */
int orc_series(double c0, double c1, double c2, double alpha, int nmax, double *w)
{
    if (nmax < 0 || !w || !(c0 > 0.0)) return -1;
    w[0] = pow(c0, alpha);
    for (int n = 1; n <= nmax; ++n) {
        double v = (alpha - (double)(n - 1)) * c1 * w[n - 1];
        if (n >= 2) v += (2.0 * alpha - (double)(n - 2)) * c2 * w[n - 2];
        w[n] = v / ((double)n * c0);
    }
    return 0;
}

#define ORC_PMAX 8
#define ORC_KMAX 12 /* largest degree of the conserving projection scalar */

/* Degree of the conserving projection scalar: 0 selects the default p-1;
 * otherwise p-1 <= K <= ORC_KMAX, conserving variant only.  Returns -1 if
 * the combination is invalid. */
static int scalar_degree(int p, int variant, int kdeg)
{
    if (kdeg == 0) return p - 1;
    if (variant != ORC_CONSERVING || kdeg < p - 1 || kdeg > ORC_KMAX) return -1;
    return kdeg;
}

/* Truncated far-field acceleration of particle a due to particle b (unit G),
 * R = Z_A - Z_B, d = delta = x_a - y_b; kdeg = degree of the conserving
 * projection scalar (already validated, p-1 by default).  Optionally the
 * truncated potential -m_b T_p[(.)^(-1/2)] (standard expansion of Eq. taylor). */
static void pair_far(const double R[3], const double d[3], double mb, int p, int kdeg,
                     double eps2, int variant, double acc[3], double *pot)
{
    double c0 = (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]) + eps2;
    double c1 = 2.0 * (R[0] * d[0] + R[1] * d[1] + R[2] * d[2]);
    double c2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double gam[ORC_PMAX + 1];
    orc_series(c0, c1, c2, -1.5, p - 1, gam);
    double t_hi = 0.0, t_lo = 0.0; /* T_{p-1}[g], T_{p-2}[g] */
    for (int n = 0; n <= p - 1; ++n) {
        if (n <= p - 2) t_lo += gam[n];
        t_hi += gam[n];
    }
    if (variant == ORC_CONSERVING_R2) {
        /* scalar (R.R + eps^2)^(-3/2) (1 - R.delta / |R|^2) along R + delta */
        double rr = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
        double rd = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
        double sc = gam[0] * (1.0 - rd / rr);
        for (int k = 0; k < 3; ++k) acc[k] = -mb * ((R[k] + d[k]) * sc);
    } else if (variant == ORC_CONSERVING && kdeg > p - 1) {
        /* Eq. realign: project the standard pair force a onto u = X_a - Y_b,
         * the scalar (a . u)/|u|^2 expanded along delta -> t delta (Eqs.
         * nab-expansion, abnab-expansion) and kept to degree kdeg.
         * -a(t)/m_b = R sum_{n<=p-1} gam_n t^n + delta sum_{n<=p-2} gam_n t^(n+1);
         * num = coefficients of (-a(t)/m_b) . (R + t delta), degree <= p+1. */
        double rr = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
        double rd = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
        double num[ORC_PMAX + 2] = {0.0};
        for (int n = 0; n <= p - 1; ++n) {
            num[n] += gam[n] * rr;
            num[n + 1] += gam[n] * rd;
        }
        for (int n = 0; n <= p - 2; ++n) {
            num[n + 1] += gam[n] * rd;
            num[n + 2] += gam[n] * c2;
        }
        /* 1/|u(t)|^2 = (R.R + 2 R.delta t + delta.delta t^2)^(-1), no softening */
        double h[ORC_KMAX + 1];
        orc_series(rr, 2.0 * rd, c2, -1.0, kdeg, h);
        double sc = 0.0;
        for (int n = 0; n <= kdeg; ++n)
            for (int j = 0; j <= n && j <= p + 1; ++j) sc += num[j] * h[n - j];
        for (int k = 0; k < 3; ++k) acc[k] = -mb * ((R[k] + d[k]) * sc);
    } else if (variant == ORC_CONSERVING) {
        for (int k = 0; k < 3; ++k) acc[k] = -mb * ((R[k] + d[k]) * t_hi);
    } else {
        for (int k = 0; k < 3; ++k) acc[k] = -mb * (R[k] * t_hi + d[k] * t_lo);
    }
    if (pot) {
        double w[ORC_PMAX + 1];
        orc_series(c0, c1, c2, -0.5, p, w);
        double s = 0.0;
        for (int n = 0; n <= p; ++n) s += w[n];
        *pot = -mb * s;
    }
}

/* Exact softened pair acceleration of a due to b; returns 0 if coincident
 * and unsoftened (no force). */
static int pair_near(const double *Xa, const double *Xb, double mb, double eps2,
                     double acc[3], double *pot)
{
    double dx = Xa[0] - Xb[0], dy = Xa[1] - Xb[1], dz = Xa[2] - Xb[2];
    double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
    if (r2 == 0.0) return 0;
    double r = sqrt(r2);
    double w = mb / (r2 * r);
    acc[0] = -w * dx;
    acc[1] = -w * dy;
    acc[2] = -w * dz;
    if (pot) *pot = -mb / r;
    return 1;
}

/* Exported single-pair evaluation (for the pin tests). */
int orc_pair_far(const double *R, const double *x, const double *y, double mb,
                 int p, int kdeg, double eps, int variant, double *acc, double *pot)
{
    if (p < 1 || p > ORC_PMAX || !R || !x || !y || !acc) return -1;
    int K = scalar_degree(p, variant, kdeg);
    if (K < 0) return -1;
    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    pair_far(R, d, mb, p, K, eps * eps, variant, acc, pot);
    return 0;
}

/* Far-field acceleration (unit G) on nt targets at absolute positions Xt in a
 * node with centre ZA, due to ns sources Ys (masses ms) in a node with centre
 * ZB: the sum over b of the truncated pair accelerations. */
int orc_cluster_far(int64_t nt, const double *Xt, const double *ZA, int64_t ns,
                    const double *Ys, const double *ms, const double *ZB, int p, int kdeg,
                    double eps, int variant, double *acc, double *pot)
{
    if (p < 1 || p > ORC_PMAX || nt < 0 || ns < 0) return -1;
    int K = scalar_degree(p, variant, kdeg);
    if (K < 0) return -1;
    double R[3] = {ZA[0] - ZB[0], ZA[1] - ZB[1], ZA[2] - ZB[2]};
    double eps2 = eps * eps;
    for (int64_t a = 0; a < nt; ++a) {
        nsum s[3] = {{0, 0}, {0, 0}, {0, 0}}, sp = {0, 0};
        double x[3] = {Xt[3 * a] - ZA[0], Xt[3 * a + 1] - ZA[1], Xt[3 * a + 2] - ZA[2]};
        for (int64_t b = 0; b < ns; ++b) {
            double y[3] = {Ys[3 * b] - ZB[0], Ys[3 * b + 1] - ZB[1], Ys[3 * b + 2] - ZB[2]};
            double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
            double f[3], ph = 0.0;
            pair_far(R, d, ms[b], p, K, eps2, variant, f, pot ? &ph : NULL);
            for (int k = 0; k < 3; ++k) nsum_add(&s[k], f[k]);
            nsum_add(&sp, ph);
        }
        for (int k = 0; k < 3; ++k) acc[3 * a + k] = nsum_get(&s[k]);
        if (pot) pot[a] = nsum_get(&sp);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tree                                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, n_leaf;
    double theta;
    const double *pos_src; /* not owned; only used during build */
    double bbox[5];        /* lo_x, lo_y, lo_z, ext, scale */
    uint64_t *keys;        /* original order */
    int64_t *order;        /* sorted position -> original index */
    double *X;             /* sorted positions, 3 per particle */
    double *m;             /* sorted masses */
    /* nodes, level-major, Morton order within a level */
    int64_t nn, cap;
    int32_t *level;
    uint64_t *prefix;
    int64_t *first, *count, *child_first, *parent;
    int32_t *nchild;
    double *M, *Z, *rmax;
    /* interaction pairs, canonical (min id, max id) */
    int64_t n_m2l, cap_m2l, n_p2p, cap_p2p;
    int64_t *m2l, *p2p;
    /* per-node partner lists, built lazily for force evaluation */
    int64_t *m2l_off, *m2l_adj, *p2p_off, *p2p_adj, *leaf_of;
} orc_tree;

typedef struct { uint64_t key; int64_t idx; } keyidx;

static int keyidx_cmp(const void *pa, const void *pb)
{
    const keyidx *a = (const keyidx *)pa, *b = (const keyidx *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

static uint64_t spread3(uint32_t q)
{
    uint64_t v = 0;
    for (int i = 0; i < ORC_LEVELS; ++i)
        if (q & (1u << i)) v |= (uint64_t)1 << (3 * i);
    return v;
}

static int node_push(orc_tree *t, int32_t lvl, uint64_t pre, int64_t first,
                     int64_t count, int64_t parent)
{
    if (t->nn == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
#define GROW(f) do { void *q = realloc(t->f, (size_t)nc * sizeof(*t->f)); if (!q) return -1; t->f = q; } while (0)
        GROW(level); GROW(prefix); GROW(first); GROW(count); GROW(child_first);
        GROW(parent); GROW(nchild); GROW(M); GROW(rmax);
        {
            void *q = realloc(t->Z, (size_t)nc * 3 * sizeof(double));
            if (!q) return -1;
            t->Z = q;
        }
#undef GROW
        t->cap = nc;
    }
    int64_t i = t->nn++;
    t->level[i] = lvl;
    t->prefix[i] = pre;
    t->first[i] = first;
    t->count[i] = count;
    t->child_first[i] = -1;
    t->nchild[i] = 0;
    t->parent[i] = parent;
    return 0;
}

static int pair_push(int64_t **arr, int64_t *n, int64_t *cap, int64_t a, int64_t b)
{
    if (*n == *cap) {
        int64_t nc = *cap ? 2 * *cap : 4096;
        void *q = realloc(*arr, (size_t)nc * 2 * sizeof(int64_t));
        if (!q) return -1;
        *arr = q;
        *cap = nc;
    }
    (*arr)[2 * *n] = a < b ? a : b;
    (*arr)[2 * *n + 1] = a < b ? b : a;
    ++*n;
    return 0;
}

static int is_leaf(const orc_tree *t, int64_t i) { return t->nchild[i] == 0; }

/* Node to split for a distinct pair that the criterion rejects. */
static int64_t split_choice(const orc_tree *t, int64_t A, int64_t B)
{
    if (is_leaf(t, A)) return B;
    if (is_leaf(t, B)) return A;
    if (t->rmax[A] > t->rmax[B]) return A;
    if (t->rmax[B] > t->rmax[A]) return B;
    if (t->level[A] < t->level[B]) return A;
    if (t->level[B] < t->level[A]) return B;
    return A < B ? A : B;
}

static int interact(orc_tree *t, int64_t A, int64_t B)
{
    if (A == B) {
        if (is_leaf(t, A)) return pair_push(&t->p2p, &t->n_p2p, &t->cap_p2p, A, A);
        int64_t c0 = t->child_first[A], nc = t->nchild[A];
        for (int64_t i = 0; i < nc; ++i)
            for (int64_t j = i; j < nc; ++j)
                if (interact(t, c0 + i, c0 + j)) return -1;
        return 0;
    }
    const double *za = &t->Z[3 * A], *zb = &t->Z[3 * B];
    double dx = za[0] - zb[0], dy = za[1] - zb[1], dz = za[2] - zb[2];
    double R = sqrt((dx * dx + dy * dy) + dz * dz);
    if (R > 0.0 && t->rmax[A] + t->rmax[B] <= t->theta * R)
        return pair_push(&t->m2l, &t->n_m2l, &t->cap_m2l, A, B);
    if (is_leaf(t, A) && is_leaf(t, B))
        return pair_push(&t->p2p, &t->n_p2p, &t->cap_p2p, A, B);
    int64_t S = split_choice(t, A, B), O = (S == A) ? B : A;
    int64_t c0 = t->child_first[S], nc = t->nchild[S];
    for (int64_t i = 0; i < nc; ++i)
        if (interact(t, c0 + i, O)) return -1;
    return 0;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->keys); free(t->order); free(t->X); free(t->m);
    free(t->level); free(t->prefix); free(t->first); free(t->count);
    free(t->child_first); free(t->parent); free(t->nchild);
    free(t->M); free(t->Z); free(t->rmax);
    free(t->m2l); free(t->p2p);
    free(t->m2l_off); free(t->m2l_adj); free(t->p2p_off); free(t->p2p_adj);
    free(t->leaf_of);
    free(t);
}

orc_tree *orc_tree_build(int64_t n, const double *pos, const double *mass,
                         int64_t n_leaf, double theta)
{
    if (n < 1 || !pos || !mass || n_leaf < 1 || !(theta >= 0.0) || !(theta < 1.0))
        return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) return NULL;
    t->n = n;
    t->n_leaf = n_leaf;
    t->theta = theta;

    /* bounding cube and keys */
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = pos[d];
    for (int64_t a = 1; a < n; ++a)
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * a + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    if (ext == 0.0) ext = 1.0;
    double scale = 2097152.0 / ext;
    t->bbox[0] = lo[0]; t->bbox[1] = lo[1]; t->bbox[2] = lo[2];
    t->bbox[3] = ext; t->bbox[4] = scale;

    t->keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    keyidx *ki = (keyidx *)malloc((size_t)n * sizeof(keyidx));
    if (!t->keys || !ki) { free(ki); orc_tree_free(t); return NULL; }
    for (int64_t a = 0; a < n; ++a) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            double f = floor((pos[3 * a + d] - lo[d]) * scale);
            q[d] = (f >= (double)ORC_QMAX) ? ORC_QMAX : (uint32_t)f;
        }
        uint64_t k = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        t->keys[a] = k;
        ki[a].key = k;
        ki[a].idx = a;
    }
    qsort(ki, (size_t)n, sizeof(keyidx), keyidx_cmp);

    t->order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    t->X = (double *)malloc((size_t)n * 3 * sizeof(double));
    t->m = (double *)malloc((size_t)n * sizeof(double));
    uint64_t *sk = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!t->order || !t->X || !t->m || !sk) { free(ki); free(sk); orc_tree_free(t); return NULL; }
    for (int64_t s = 0; s < n; ++s) {
        int64_t a = ki[s].idx;
        t->order[s] = a;
        sk[s] = ki[s].key;
        for (int d = 0; d < 3; ++d) t->X[3 * s + d] = pos[3 * a + d];
        t->m[s] = mass[a];
    }
    free(ki);

    /* octree, level by level */
    if (node_push(t, 0, 0, 0, n, -1)) { free(sk); orc_tree_free(t); return NULL; }
    int64_t lvl_begin = 0, lvl_end = 1;
    for (int lvl = 0; lvl < ORC_LEVELS && lvl_begin < lvl_end; ++lvl) {
        int shift = 3 * (ORC_LEVELS - 1 - lvl);
        for (int64_t i = lvl_begin; i < lvl_end; ++i) {
            if (t->count[i] <= n_leaf) continue;
            int64_t s = t->first[i], e = s + t->count[i];
            t->child_first[i] = t->nn;
            while (s < e) {
                uint64_t dig = (sk[s] >> shift) & 7u;
                int64_t r = s + 1;
                while (r < e && ((sk[r] >> shift) & 7u) == dig) ++r;
                if (node_push(t, lvl + 1, (t->prefix[i] << 3) | dig, s, r - s, i)) {
                    free(sk); orc_tree_free(t); return NULL;
                }
                t->nchild[i]++;
                s = r;
            }
        }
        lvl_begin = lvl_end;
        lvl_end = t->nn;
    }
    free(sk);

    /* geometry, children before parents (children have larger indices) */
    for (int64_t i = t->nn - 1; i >= 0; --i) {
        double M = 0.0, S[3] = {0.0, 0.0, 0.0};
        if (is_leaf(t, i)) {
            for (int64_t s = t->first[i]; s < t->first[i] + t->count[i]; ++s) {
                M += t->m[s];
                for (int d = 0; d < 3; ++d) S[d] += t->m[s] * t->X[3 * s + d];
            }
        } else {
            for (int64_t c = t->child_first[i]; c < t->child_first[i] + t->nchild[i]; ++c) {
                M += t->M[c];
                /* inner nodes carry S in Z temporarily until all parents done */
                for (int d = 0; d < 3; ++d) S[d] += t->Z[3 * c + d];
            }
        }
        t->M[i] = M;
        for (int d = 0; d < 3; ++d) t->Z[3 * i + d] = S[d]; /* S for now */
    }
    for (int64_t i = 0; i < t->nn; ++i)
        for (int d = 0; d < 3; ++d) t->Z[3 * i + d] = t->Z[3 * i + d] / t->M[i];
    for (int64_t i = 0; i < t->nn; ++i) {
        double best = 0.0;
        const double *z = &t->Z[3 * i];
        for (int64_t s = t->first[i]; s < t->first[i] + t->count[i]; ++s) {
            double dx = t->X[3 * s] - z[0], dy = t->X[3 * s + 1] - z[1], dz = t->X[3 * s + 2] - z[2];
            double d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 > best) best = d2;
        }
        t->rmax[i] = sqrt(best);
    }

    /* walk */
    if (interact(t, 0, 0)) { orc_tree_free(t); return NULL; }
    return t;
}

/* sizes: n, nodes, far pairs, near pairs */
void orc_tree_sizes(const orc_tree *t, int64_t *out)
{
    out[0] = t->n;
    out[1] = t->nn;
    out[2] = t->n_m2l;
    out[3] = t->n_p2p;
}

void orc_tree_bbox(const orc_tree *t, double *out) { memcpy(out, t->bbox, sizeof(t->bbox)); }

/* keys (original particle order) and the sorted order (sorted position ->
 * original index) */
void orc_tree_keys(const orc_tree *t, uint64_t *keys, int64_t *order)
{
    if (keys) memcpy(keys, t->keys, (size_t)t->n * sizeof(uint64_t));
    if (order) memcpy(order, t->order, (size_t)t->n * sizeof(int64_t));
}

void orc_tree_nodes(const orc_tree *t, int32_t *level, uint64_t *prefix, int64_t *first,
                    int64_t *count, int64_t *child_first, int32_t *nchild, int64_t *parent,
                    double *M, double *Z, double *rmax)
{
    size_t nn = (size_t)t->nn;
    if (level) memcpy(level, t->level, nn * sizeof(int32_t));
    if (prefix) memcpy(prefix, t->prefix, nn * sizeof(uint64_t));
    if (first) memcpy(first, t->first, nn * sizeof(int64_t));
    if (count) memcpy(count, t->count, nn * sizeof(int64_t));
    if (child_first) memcpy(child_first, t->child_first, nn * sizeof(int64_t));
    if (nchild) memcpy(nchild, t->nchild, nn * sizeof(int32_t));
    if (parent) memcpy(parent, t->parent, nn * sizeof(int64_t));
    if (M) memcpy(M, t->M, nn * sizeof(double));
    if (Z) memcpy(Z, t->Z, nn * 3 * sizeof(double));
    if (rmax) memcpy(rmax, t->rmax, nn * sizeof(double));
}

/* canonical unordered pairs (lower node index first), in walk order */
void orc_tree_lists(const orc_tree *t, int64_t *m2l, int64_t *p2p)
{
    if (m2l && t->n_m2l > 0) memcpy(m2l, t->m2l, (size_t)t->n_m2l * 2 * sizeof(int64_t));
    if (p2p && t->n_p2p > 0) memcpy(p2p, t->p2p, (size_t)t->n_p2p * 2 * sizeof(int64_t));
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Per-node partner lists, each sorted by partner index. */
static int build_adjacency(orc_tree *t)
{
    if (t->m2l_off) return 0;
    int64_t nn = t->nn;
    t->m2l_off = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    t->p2p_off = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    t->leaf_of = (int64_t *)malloc((size_t)t->n * sizeof(int64_t));
    if (!t->m2l_off || !t->p2p_off || !t->leaf_of) return -1;
    for (int64_t k = 0; k < t->n_m2l; ++k) {
        t->m2l_off[t->m2l[2 * k] + 1]++;
        t->m2l_off[t->m2l[2 * k + 1] + 1]++;
    }
    for (int64_t k = 0; k < t->n_p2p; ++k) {
        int64_t a = t->p2p[2 * k], b = t->p2p[2 * k + 1];
        t->p2p_off[a + 1]++;
        if (b != a) t->p2p_off[b + 1]++;
    }
    for (int64_t i = 0; i < nn; ++i) {
        t->m2l_off[i + 1] += t->m2l_off[i];
        t->p2p_off[i + 1] += t->p2p_off[i];
    }
    t->m2l_adj = (int64_t *)malloc((size_t)(t->m2l_off[nn] + 1) * sizeof(int64_t));
    t->p2p_adj = (int64_t *)malloc((size_t)(t->p2p_off[nn] + 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)nn, sizeof(int64_t));
    if (!t->m2l_adj || !t->p2p_adj || !fill) { free(fill); return -1; }
    for (int64_t k = 0; k < t->n_m2l; ++k) {
        int64_t a = t->m2l[2 * k], b = t->m2l[2 * k + 1];
        t->m2l_adj[t->m2l_off[a] + fill[a]++] = b;
        t->m2l_adj[t->m2l_off[b] + fill[b]++] = a;
    }
    memset(fill, 0, (size_t)nn * sizeof(int64_t));
    for (int64_t k = 0; k < t->n_p2p; ++k) {
        int64_t a = t->p2p[2 * k], b = t->p2p[2 * k + 1];
        t->p2p_adj[t->p2p_off[a] + fill[a]++] = b;
        if (b != a) t->p2p_adj[t->p2p_off[b] + fill[b]++] = a;
    }
    free(fill);
    for (int64_t i = 0; i < nn; ++i) {
        qsort(t->m2l_adj + t->m2l_off[i], (size_t)(t->m2l_off[i + 1] - t->m2l_off[i]),
              sizeof(int64_t), cmp_i64);
        qsort(t->p2p_adj + t->p2p_off[i], (size_t)(t->p2p_off[i + 1] - t->p2p_off[i]),
              sizeof(int64_t), cmp_i64);
        if (is_leaf(t, i))
            for (int64_t s = t->first[i]; s < t->first[i] + t->count[i]; ++s) t->leaf_of[s] = i;
    }
    return 0;
}

/*
 * FMM forces on the given targets (original indices; NULL = all, in original
 * order): F_a = G m_a (near + far), near over the near pairs of a's leaf,
 * far over the accepted pairs of a's leaf and of every ancestor, each summed
 * particle by particle with the truncated pair expression.  pot (optional)
 * gets G times the potential with the far part from the standard Taylor
 * expansion of Eq. taylor.
 */
int orc_fmm_forces(orc_tree *t, int p, int kdeg, double eps, double G, int variant,
                   int64_t n_targets, const int64_t *targets, double *force, double *pot)
{
    if (!t || p < 1 || p > ORC_PMAX || !(eps >= 0.0) || !force) return -1;
    if (variant != ORC_STANDARD && variant != ORC_CONSERVING && variant != ORC_CONSERVING_R2) return -1;
    if (variant == ORC_CONSERVING_R2 && p != 1) return -1;
    int K = scalar_degree(p, variant, kdeg);
    if (K < 0) return -1;
    if (build_adjacency(t)) return -2;
    int64_t nt = targets ? n_targets : t->n;
    int64_t *pos_of = (int64_t *)malloc((size_t)t->n * sizeof(int64_t));
    if (!pos_of) return -2;
    for (int64_t s = 0; s < t->n; ++s) pos_of[t->order[s]] = s;
    double eps2 = eps * eps;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t ia = targets ? targets[k] : k;
        if (ia < 0 || ia >= t->n) { bad = 1; continue; }
        int64_t sa = pos_of[ia];
        const double *Xa = &t->X[3 * sa];
        nsum f[3] = {{0, 0}, {0, 0}, {0, 0}}, ph = {0, 0};
        double acc[3], pp = 0.0;
        int64_t leaf = t->leaf_of[sa];
        for (int64_t q = t->p2p_off[leaf]; q < t->p2p_off[leaf + 1]; ++q) {
            int64_t B = t->p2p_adj[q];
            for (int64_t sb = t->first[B]; sb < t->first[B] + t->count[B]; ++sb) {
                if (sb == sa) continue;
                if (!pair_near(Xa, &t->X[3 * sb], t->m[sb], eps2, acc, pot ? &pp : NULL)) continue;
                for (int d = 0; d < 3; ++d) nsum_add(&f[d], acc[d]);
                if (pot) nsum_add(&ph, pp);
            }
        }
        for (int64_t A = leaf; A >= 0; A = t->parent[A]) {
            const double *ZA = &t->Z[3 * A];
            double x[3] = {Xa[0] - ZA[0], Xa[1] - ZA[1], Xa[2] - ZA[2]};
            for (int64_t q = t->m2l_off[A]; q < t->m2l_off[A + 1]; ++q) {
                int64_t B = t->m2l_adj[q];
                const double *ZB = &t->Z[3 * B];
                double R[3] = {ZA[0] - ZB[0], ZA[1] - ZB[1], ZA[2] - ZB[2]};
                for (int64_t sb = t->first[B]; sb < t->first[B] + t->count[B]; ++sb) {
                    const double *Yb = &t->X[3 * sb];
                    double y[3] = {Yb[0] - ZB[0], Yb[1] - ZB[1], Yb[2] - ZB[2]};
                    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
                    pair_far(R, d, t->m[sb], p, K, eps2, variant, acc, pot ? &pp : NULL);
                    for (int dd = 0; dd < 3; ++dd) nsum_add(&f[dd], acc[dd]);
                    if (pot) nsum_add(&ph, pp);
                }
            }
        }
        double s = G * t->m[sa];
        for (int d = 0; d < 3; ++d) force[3 * k + d] = s * nsum_get(&f[d]);
        if (pot) pot[k] = G * nsum_get(&ph);
    }
    free(pos_of);
    return bad ? -1 : 0;
}

/*
 * Momentum diagnostics (FP64, compensated), Eqs. netforce and total_torque
 * summed over all particles, about the system centre of mass:
 *  out[0..2]  sum F            out[3]     sum |F|
 *  out[4..6]  sum (X-Xcm) x F  out[7]     sum |X-Xcm| |F|
 *  out[8..10] P = sum m v      out[11..13] L = sum m (X-Xcm) x v
 *  out[14]    sum m            out[15..17] Xcm
 *  out[18]    |sum F| / sum |F|           out[19] |sum (X-Xcm) x F| / sum |X-Xcm||F|
 */
int orc_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass,
                    const double *force, double *out)
{
    if (n < 1 || !pos || !mass || !force || !out) return -1;
    nsum M = {0, 0}, S[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t a = 0; a < n; ++a) {
        nsum_add(&M, mass[a]);
        for (int d = 0; d < 3; ++d) nsum_add(&S[d], mass[a] * pos[3 * a + d]);
    }
    double Mt = nsum_get(&M), cm[3];
    for (int d = 0; d < 3; ++d) cm[d] = nsum_get(&S[d]) / Mt;
    nsum F[3] = {{0, 0}, {0, 0}, {0, 0}}, T[3] = {{0, 0}, {0, 0}, {0, 0}};
    nsum P[3] = {{0, 0}, {0, 0}, {0, 0}}, L[3] = {{0, 0}, {0, 0}, {0, 0}};
    nsum Fn = {0, 0}, Tn = {0, 0};
    for (int64_t a = 0; a < n; ++a) {
        const double *f = &force[3 * a];
        double r[3] = {pos[3 * a] - cm[0], pos[3 * a + 1] - cm[1], pos[3 * a + 2] - cm[2]};
        double fn = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int d = 0; d < 3; ++d) nsum_add(&F[d], f[d]);
        nsum_add(&T[0], r[1] * f[2] - r[2] * f[1]);
        nsum_add(&T[1], r[2] * f[0] - r[0] * f[2]);
        nsum_add(&T[2], r[0] * f[1] - r[1] * f[0]);
        nsum_add(&Fn, fn);
        nsum_add(&Tn, rn * fn);
        if (vel) {
            const double *v = &vel[3 * a];
            for (int d = 0; d < 3; ++d) nsum_add(&P[d], mass[a] * v[d]);
            nsum_add(&L[0], mass[a] * (r[1] * v[2] - r[2] * v[1]));
            nsum_add(&L[1], mass[a] * (r[2] * v[0] - r[0] * v[2]));
            nsum_add(&L[2], mass[a] * (r[0] * v[1] - r[1] * v[0]));
        }
    }
    for (int d = 0; d < 3; ++d) {
        out[d] = nsum_get(&F[d]);
        out[4 + d] = nsum_get(&T[d]);
        out[8 + d] = nsum_get(&P[d]);
        out[11 + d] = nsum_get(&L[d]);
        out[15 + d] = cm[d];
    }
    out[3] = nsum_get(&Fn);
    out[7] = nsum_get(&Tn);
    out[14] = Mt;
    double fs = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
    double ts = sqrt(out[4] * out[4] + out[5] * out[5] + out[6] * out[6]);
    out[18] = out[3] > 0 ? fs / out[3] : 0.0;
    out[19] = out[7] > 0 ? ts / out[7] : 0.0;
    return 0;
}

int orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * Driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_oracle_sanitize.py on the CPU).  It calls every
 * exported oracle function on random and degenerate inputs: direct sums,
 * series, single pairs and clusters (every variant, the scalar-degree knob),
 * trees with their keys, nodes and lists, forces with potentials on all and on
 * some particles, diagnostics with and without velocities, and the argument
 * checks.  Any invalid memory access or undefined behaviour aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_tree orc_tree;
int orc_direct(int64_t n, const double *pos, const double *mass, double eps, double G, double *force, double *pot);
int orc_series(double c0, double c1, double c2, double alpha, int nmax, double *w);
int orc_pair_far(const double *R, const double *x, const double *y, double mb, int p, int kdeg, double eps,
                 int variant, double *acc, double *pot);
int orc_cluster_far(int64_t nt, const double *Xt, const double *ZA, int64_t ns, const double *Ys, const double *ms,
                    const double *ZB, int p, int kdeg, double eps, int variant, double *acc, double *pot);
orc_tree *orc_tree_build(int64_t n, const double *pos, const double *mass, int64_t n_leaf, double theta);
void orc_tree_free(orc_tree *t);
void orc_tree_sizes(const orc_tree *t, int64_t *out);
void orc_tree_bbox(const orc_tree *t, double *out);
void orc_tree_keys(const orc_tree *t, uint64_t *keys, int64_t *order);
void orc_tree_nodes(const orc_tree *t, int32_t *level, uint64_t *prefix, int64_t *first, int64_t *count,
                    int64_t *child_first, int32_t *nchild, int64_t *parent, double *M, double *Z, double *rmax);
void orc_tree_lists(const orc_tree *t, int64_t *m2l, int64_t *p2p);
int orc_fmm_forces(orc_tree *t, int p, int kdeg, double eps, double G, int variant, int64_t n_targets,
                   const int64_t *targets, double *force, double *pot);
int orc_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass, const double *force,
                    double *out);
int orc_set_threads(int nthreads);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static void run_tree(int64_t n, const double *pos, const double *mass, int64_t n_leaf, double theta)
{
    orc_tree *t = orc_tree_build(n, pos, mass, n_leaf, theta);
    CHECK(t != NULL);
    if (!t) return;
    int64_t sz[4];
    orc_tree_sizes(t, sz);
    double bb[5];
    orc_tree_bbox(t, bb);
    uint64_t *keys = malloc((size_t)n * sizeof(uint64_t));
    int64_t *order = malloc((size_t)n * sizeof(int64_t));
    orc_tree_keys(t, keys, order);
    int64_t nn = sz[1];
    int32_t *level = malloc((size_t)nn * sizeof(int32_t)), *nchild = malloc((size_t)nn * sizeof(int32_t));
    uint64_t *prefix = malloc((size_t)nn * sizeof(uint64_t));
    int64_t *first = malloc((size_t)nn * 8), *count = malloc((size_t)nn * 8), *cf = malloc((size_t)nn * 8),
            *parent = malloc((size_t)nn * 8);
    double *M = malloc((size_t)nn * 8), *Z = malloc((size_t)nn * 24), *rmax = malloc((size_t)nn * 8);
    orc_tree_nodes(t, level, prefix, first, count, cf, nchild, parent, M, Z, rmax);
    int64_t *m2l = malloc((size_t)(sz[2] + 1) * 16), *p2p = malloc((size_t)(sz[3] + 1) * 16);
    orc_tree_lists(t, m2l, p2p);
    const int64_t rows = n > 3 ? n : 3; /* the target subset below has 3 rows */
    double *f = malloc((size_t)rows * 24), *pot = malloc((size_t)rows * 8);
    for (int p = 1; p <= 8; p += 3) {
        CHECK(orc_fmm_forces(t, p, 0, 1e-3, 1.0, 0, n, NULL, f, pot) == 0);
        CHECK(orc_fmm_forces(t, p, 0, 0.0, 1.0, 1, n, NULL, f, NULL) == 0);
        CHECK(orc_fmm_forces(t, p, p + 1, 1e-3, 1.0, 1, n, NULL, f, pot) == 0);
    }
    CHECK(orc_fmm_forces(t, 1, 0, 1e-3, 1.0, 2, n, NULL, f, pot) == 0);
    int64_t tg[3] = {0, n - 1, n / 2};
    CHECK(orc_fmm_forces(t, 4, 0, 1e-3, 2.0, 1, 3, tg, f, pot) == 0);
    int64_t bad[1] = {n};
    CHECK(orc_fmm_forces(t, 4, 0, 1e-3, 1.0, 1, 1, bad, f, NULL) != 0);
    CHECK(orc_fmm_forces(t, 9, 0, 1e-3, 1.0, 1, n, NULL, f, NULL) != 0);
    CHECK(orc_fmm_forces(t, 2, 0, 1e-3, 1.0, 2, n, NULL, f, NULL) != 0);
    CHECK(orc_fmm_forces(t, 4, 2, 1e-3, 1.0, 1, n, NULL, f, NULL) != 0);
    free(keys); free(order); free(level); free(nchild); free(prefix); free(first); free(count); free(cf);
    free(parent); free(M); free(Z); free(rmax); free(m2l); free(p2p); free(f); free(pot);
    orc_tree_free(t);
}

int main(void)
{
    orc_set_threads(2);
    const int64_t n = 700;
    double *pos = malloc((size_t)n * 24), *vel = malloc((size_t)n * 24), *mass = malloc((size_t)n * 8);
    double *f = malloc((size_t)n * 24), *pot = malloc((size_t)n * 8), out[20];
    for (int64_t a = 0; a < n; ++a) {
        for (int d = 0; d < 3; ++d) {
            pos[3 * a + d] = urand() * urand() - 0.25;
            vel[3 * a + d] = urand() - 0.5;
        }
        mass[a] = 0.5 + urand();
    }
    /* duplicates and a coplanar slab */
    for (int64_t a = 100; a < 160; ++a)
        for (int d = 0; d < 3; ++d) pos[3 * a + d] = pos[3 * 7 + d];
    for (int64_t a = 200; a < 300; ++a) pos[3 * a + 2] = 0.125;

    CHECK(orc_direct(n, pos, mass, 1e-3, 1.0, f, pot) == 0);
    CHECK(orc_direct(n, pos, mass, 0.0, 1.0, f, NULL) == 0);
    CHECK(orc_diagnostics(n, pos, vel, mass, f, out) == 0);
    CHECK(orc_diagnostics(n, pos, NULL, mass, f, out) == 0);

    double w[13];
    CHECK(orc_series(2.0, 0.3, 0.1, -1.5, 12, w) == 0);
    CHECK(orc_series(0.0, 0.3, 0.1, -1.5, 4, w) != 0);
    double R[3] = {1.5, -0.3, 0.7}, x[3] = {0.1, 0.2, -0.1}, y[3] = {-0.2, 0.05, 0.1}, acc[3], ph;
    for (int p = 1; p <= 8; ++p)
        for (int v = 0; v < 3; ++v) CHECK(orc_pair_far(R, x, y, 1.0, p, 0, 1e-3, v, acc, &ph) == 0);
    for (int p = 1; p <= 8; ++p)
        for (int k = p; k <= 12; ++k) CHECK(orc_pair_far(R, x, y, 1.0, p, k, 0.0, 1, acc, &ph) == 0);
    CHECK(orc_pair_far(R, x, y, 1.0, 4, 13, 0.0, 1, acc, &ph) != 0);
    double Xt[6] = {2.0, 0.1, 0.0, 2.1, -0.1, 0.05}, ZA[3] = {2.05, 0.0, 0.025}, ZB[3] = {0.0, 0.0, 0.0};
    double Ys[9] = {0.1, 0.0, 0.0, -0.1, 0.05, 0.0, 0.0, -0.05, 0.02}, ms[3] = {1.0, 2.0, 0.5}, ca[6], cp[2];
    CHECK(orc_cluster_far(2, Xt, ZA, 3, Ys, ms, ZB, 5, 6, 1e-3, 1, ca, cp) == 0);
    CHECK(orc_cluster_far(2, Xt, ZA, 3, Ys, ms, ZB, 5, 0, 1e-3, 0, ca, cp) == 0);

    run_tree(n, pos, mass, 8, 0.5);
    run_tree(n, pos, mass, 1, 0.0);
    run_tree(n, pos, mass, 64, 0.9);
    run_tree(1, pos, mass, 4, 0.5);
    run_tree(2, pos, mass, 1, 0.5);
    /* all particles at one point */
    for (int64_t a = 0; a < 50; ++a)
        for (int d = 0; d < 3; ++d) pos[3 * a + d] = 0.5;
    run_tree(50, pos, mass, 4, 0.5);
    CHECK(orc_tree_build(0, pos, mass, 4, 0.5) == NULL);
    CHECK(orc_tree_build(10, pos, mass, 4, 1.0) == NULL);

    free(pos); free(vel); free(mass); free(f); free(pot);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle sanitize driver ok\n");
    return 0;
}

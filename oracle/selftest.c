/*
 * selftest.c -- a standalone run of every oracle entry point on a small
 * synthetic scene, for builds with AddressSanitizer and UndefinedBehavior
 * Sanitizer (test infrastructure, like the oracle itself).  It checks only
 * invariants that hold whatever the data (conservation of photons by the
 * compaction, counts and depths inside their ranges, finite values); the
 * oracle's arithmetic is pinned by the Python tests.
 *
 *   gcc -fsanitize=address,undefined -fno-sanitize-recover=all -g -O1 \
 *       oracle/selftest.c oracle/rt3d_oracle.c -lm -o selftest && ./selftest
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rt3d_oracle.h"

static const double SQRT_2PI = 2.5066282746310002;
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double uniform(void) /* xorshift64*, in (0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return ((double)((rng_state * 2685821657736338717ull) >> 11) + 0.5) / 9007199254740992.0;
}

static int poisson(double mean) /* Knuth's product method; small means only */
{
    const double L = exp(-mean);
    double p = 1.0;
    int k = 0;
    do {
        ++k;
        p *= uniform();
    } while (p > L);
    return k - 1;
}

static void fail(const char* what)
{
    fprintf(stderr, "selftest: %s\n", what);
    exit(1);
}

static void params_default(or_params* p)
{
    memset(p, 0, sizeof *p);
    p->n_iter = 3;
    p->k_max = 4;
    p->k_init = 3;
    p->p_xy = 1.0;
    p->dz = 0.1;
    p->h_apss = 2.0;
    p->h_int = 2.0;
    p->beta_t = 0.5;
    p->beta_r = 1.0;
    p->beta_b = 1.0;
    p->r_min = 1.0;
    p->sigma_b = 2.0;
    p->b_min = 1e-8;
    p->sbr_guess = 1.0;
    p->r_init = 1;
    p->n_min = 2;
    p->kappa = 3.0;
    p->m_min = 3;
    p->use_apss = 1;
}

static void check_state(const or_params* p, int64_t P, int T, const double* t, const double* r, const int* cnt,
                        const double* b)
{
    for (int64_t q = 0; q < P; ++q) {
        if (cnt[q] < 0 || cnt[q] > p->k_max) fail("point count out of range");
        if (!(b[q] >= 0.0) || !isfinite(b[q])) fail("background not finite and >= 0");
        for (int k = 0; k < cnt[q]; ++k) {
            const double tk = t[q * p->k_max + k], rk = r[q * p->k_max + k];
            if (!(tk >= 0.0 && tk <= T - 1)) fail("depth outside [0, T - 1]");
            if (!(rk >= 0.0) || !isfinite(rk)) fail("intensity not finite and >= 0");
        }
    }
}

int main(void)
{
    enum { F = 2, ROWS = 12, COLS = 10, T = 200, L = 19, S = 2 };
    const int64_t P = (int64_t)F * ROWS * COLS;
    double irf[L];
    for (int k = 0; k < L; ++k) irf[k] = exp(-0.5 * (k - 9) * (k - 9) / (1.5 * 1.5));
    or_model* m = or_model_new(irf, L, -1, T);
    if (!m) fail("model");

    /* two planes in depth, the nearer one over half of each frame */
    uint16_t* Z = calloc((size_t)P * T, sizeof *Z);
    double sum_z = 0.0;
    for (int64_t q = 0; q < P; ++q) {
        const int i = (int)((q / COLS) % ROWS), j = (int)(q % COLS);
        for (int t = 0; t < T; ++t) {
            double lam = 0.02;
            const double d0 = 120.0 + 0.5 * i, d1 = 60.0 + 0.3 * j;
            lam += 8.0 * exp(-0.5 * (t - d0) * (t - d0) / 2.25) / (1.5 * SQRT_2PI);
            if (j < COLS / 2) lam += 6.0 * exp(-0.5 * (t - d1) * (t - d1) / 2.25) / (1.5 * SQRT_2PI);
            Z[q * T + t] = (uint16_t)poisson(lam);
            sum_z += Z[q * T + t];
        }
    }
    uint32_t* off = malloc(sizeof(uint32_t) * (P + 1));
    uint32_t* ent = malloc(sizeof(uint32_t) * (size_t)P * T);
    const int64_t E = or_compact(Z, P, T, off, ent);
    double sum_e = 0.0;
    for (int64_t e = 0; e < E; ++e) sum_e += (double)(ent[e] & 0xffffu);
    if (sum_e != sum_z || (int64_t)off[P] != E) fail("compaction does not conserve the photons");

    or_params p;
    params_default(&p);
    const int K = p.k_max;
    double* g = malloc(sizeof(double) * P);
    double* t = calloc((size_t)P * K, sizeof(double));
    double* r = calloc((size_t)P * K, sizeof(double));
    double* n = calloc((size_t)P * K * 3, sizeof(double));
    int* cnt = calloc((size_t)P, sizeof(int));
    double* b = calloc((size_t)P, sizeof(double));
    for (int64_t q = 0; q < P; ++q) g[q] = (q % 17 == 5) ? 0.0 : 1.0;   /* a few dead pixels */

    double tau[5] = {-3.0, 0.0, 0.25, 9.5, 30.0}, h[5], hp[5], s[5], sp[5];
    or_h(m, 5, tau, h, hp);
    or_S(m, 5, tau, s, sp);
    int64_t q_lmf[L];
    or_lmf_table(m, 1.0, q_lmf);

    or_init(m, &p, F, ROWS, COLS, off, ent, g, t, r, n, cnt, b);
    or_init_normals(&p, F, ROWS, COLS, t, cnt, n);
    check_state(&p, P, T, t, r, cnt, b);
    const double nll0 = or_nll(m, P, off, ent, K, t, r, cnt, b, g);
    double* gt = calloc((size_t)P * K, sizeof(double));
    double* gr = calloc((size_t)P * K, sizeof(double));
    double* gb = calloc((size_t)P, sizeof(double));
    double* at = calloc((size_t)P * K, sizeof(double));
    double* ar = calloc((size_t)P * K, sizeof(double));
    double* ab = calloc((size_t)P, sizeof(double));
    or_grad(m, P, off, ent, K, t, r, cnt, b, g, gt, gr, gb, at, ar, ab);
    int64_t nb[64];
    or_apss_neighbours(&p, F, ROWS, COLS, t, cnt, P / 2, 1, nb, 64);
    or_iterate(m, &p, F, ROWS, COLS, off, ent, g, t, r, n, cnt, b);
    check_state(&p, P, T, t, r, cnt, b);
    or_reconstruct(m, &p, F, ROWS, COLS, off, ent, g, t, r, n, cnt, b);
    check_state(&p, P, T, t, r, cnt, b);
    const double nll1 = or_nll(m, P, off, ent, K, t, r, cnt, b, g);
    if (!isfinite(nll0) || !isfinite(nll1)) fail("negative log-likelihood not finite");

    /* the pinhole camera and the box divisor of the intensity low-pass */
    p.persp = 0.02;
    p.ilp_box = 1;
    or_reconstruct(m, &p, F, ROWS, COLS, off, ent, g, t, r, n, cnt, b);
    check_state(&p, P, T, t, r, cnt, b);

    /* super-resolution: 2 x 2 point-grid pixels per lidar pixel */
    p.persp = 0.0;
    p.ilp_box = 0;
    const int64_t Pf = P * S * S;
    double* tf = calloc((size_t)Pf * K, sizeof(double));
    double* rf = calloc((size_t)Pf * K, sizeof(double));
    double* nf = calloc((size_t)Pf * K * 3, sizeof(double));
    int* cf = calloc((size_t)Pf, sizeof(int));
    double* bf = calloc((size_t)P, sizeof(double));
    or_sr_reconstruct(m, &p, S, F, ROWS, COLS, off, ent, g, tf, rf, nf, cf, bf);
    for (int64_t q = 0; q < Pf; ++q)
        if (cf[q] < 0 || cf[q] > K) fail("super-resolved point count out of range");
    const double nll2 = or_sr_nll(m, S, F, ROWS, COLS, off, ent, K, tf, rf, cf, bf, g);
    if (!isfinite(nll2)) fail("super-resolved negative log-likelihood not finite");

    or_model_free(m);
    free(Z), free(off), free(ent), free(g), free(t), free(r), free(n), free(cnt), free(b);
    free(gt), free(gr), free(gb), free(at), free(ar), free(ab), free(tf), free(rf), free(nf), free(cf), free(bf);
    printf("selftest: %lld entries, %d frames of %d x %d, all oracle entry points ran\n", (long long)E, F, ROWS,
           COLS);
    return 0;
}

/*
 * rt3d_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Written from the paper (Tachella et al., real-time 3D reconstruction from
 * single-photon lidar data with plug-and-play point cloud denoisers):
 *   - Results, "Observation model": Poisson likelihood of the lidar cube and
 *     its negative log-likelihood g(t, r, b);
 *   - Results, "Reconstruction algorithm" (and its block diagram figure):
 *     PALM-style proximal gradient steps on the blocks t, r, b, each gradient
 *     step followed by a denoiser playing the role of the proximal operator;
 *     APSS for depth, a nearest-neighbour low-pass plus a minimum-intensity
 *     threshold for intensity, identity or an FFT-style image filter for
 *     background;
 *   - Methods, "3D Reconstruction algorithm": per-pixel initialisation and
 *     gradient steps, cost linear in the number of active (non-zero) bins;
 *   - Results, dynamic scenes (and Discussion): the super-resolution map f,
 *     several point-grid pixels per lidar pixel.
 * APSS (algebraic point set surfaces) is the sphere fit of the cited APSS
 * work, derived here from its least-squares definition.
 *
 * Every quantity is double precision, every loop is the direct definition,
 * single threaded, in the order the steps are stated.  No blocking, fusion or
 * reordering.  The readings chosen where the paper is silent are documented
 * beside each function.
 */
#include "rt3d_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* IRF model                                                                 */
/* ------------------------------------------------------------------------ */

struct or_model {
    int     L, o, T;
    double* hbar;   /* normalised IRF samples, sum 1 */
    double  hmax;   /* largest sample */
    double  sigma2; /* IRF variance in bins^2 */
    double  fisher; /* shift Fisher information per photon, 1/bins^2 */
    int     wl, wr; /* peak window half widths (5% / 95% cumulative mass) */
    /* per-pixel IRFs (or_model_set_classes): pixel p uses cls_m[cls[p]]
     * (class numbers >= ncls count as 0); no table: this model everywhere */
    int                ncls;
    or_model* const*   cls_m;
    const uint8_t*     cls;
};

/* The IRF of pixel pix (Observation model: h_ij is known per pixel). */
static const or_model* pm(const or_model* m, int64_t pix)
{
    if (!m->cls) return m;
    int k = m->cls[pix];
    return m->cls_m[k < m->ncls ? k : 0];
}

static void h_eval(const or_model* m, double tau, double* h, double* hp);

static double hb(const or_model* m, int k) { return (k >= 0 && k < m->L) ? m->hbar[k] : 0.0; }

/* Uniform Catmull-Rom cubic between p1 (s = 0) and p2 (s = 1), and its
 * derivative in s. */
static double catmull_rom(double p0, double p1, double p2, double p3, double s)
{
    return 0.5 * (2.0 * p1 + (-p0 + p2) * s + (2.0 * p0 - 5.0 * p1 + 4.0 * p2 - p3) * s * s
                  + (-p0 + 3.0 * p1 - 3.0 * p2 + p3) * s * s * s);
}

static double catmull_rom_ds(double p0, double p1, double p2, double p3, double s)
{
    return 0.5 * ((-p0 + p2) + 2.0 * (2.0 * p0 - 5.0 * p1 + 4.0 * p2 - p3) * s
                  + 3.0 * (-p0 + 3.0 * p1 - 3.0 * p2 + p3) * s * s);
}

/* The IRF h is "known" per pixel (Observation model).  Reading: samples
 * irf[0..L-1] at integer lags, normalised to unit sum, origin `origin`
 * (argmax when negative, smallest index on ties).  The continuous h(tau) is the
 * Catmull-Rom interpolant of the samples (zero beyond them, clamped at zero),
 * so h and h' are continuous between and across samples. */
or_model* or_model_new(const double* irf, int L, int origin, int T)
{
    if (L <= 0 || T <= 0 || L > T) return NULL;
    double sum = 0.0;
    for (int k = 0; k < L; ++k) {
        if (!(irf[k] >= 0.0) || !isfinite(irf[k])) return NULL;
        sum += irf[k];
    }
    if (!(sum > 0.0)) return NULL;
    or_model* m = (or_model*)calloc(1, sizeof(or_model));
    m->L = L; m->T = T;
    m->hbar = (double*)malloc(sizeof(double) * L);
    for (int k = 0; k < L; ++k) m->hbar[k] = irf[k] / sum;
    if (origin < 0) {
        int best = 0;
        for (int k = 1; k < L; ++k) if (m->hbar[k] > m->hbar[best]) best = k;
        origin = best;
    }
    m->o = origin;
    m->hmax = 0.0;
    for (int k = 0; k < L; ++k) m->hmax = m->hbar[k] > m->hmax ? m->hbar[k] : m->hmax;
    double mu = 0.0;
    for (int k = 0; k < L; ++k) mu += k * m->hbar[k];
    double var = 0.0;
    for (int k = 0; k < L; ++k) var += m->hbar[k] * (k - mu) * (k - mu);
    m->sigma2 = var;
    /* Fisher information of one photon about the shift of h (no background),
     * averaged over 32 sub-bin phases: mean_j sum_lag h'(lag + j/32)^2 / h(..),
     * over the lags where h is at least 1e-3 of the largest sample. */
    {
        double acc = 0.0;
        for (int j = 0; j < 32; ++j)
            for (int l = -origin - 1; l <= L - origin; ++l) {
                double h, hp;
                h_eval(m, l + j / 32.0, &h, &hp);
                if (h >= 1e-3 * m->hmax) acc += hp * hp / h;
            }
        m->fisher = acc / 32.0;
    }
    /* Peak window: lags where the cumulative IRF mass first reaches 5% / 95%. */
    double c = 0.0;
    int klo = -1, khi = -1;
    for (int k = 0; k < L; ++k) {
        c += m->hbar[k];
        if (klo < 0 && c >= 0.05) klo = k;
        if (khi < 0 && c >= 0.95) khi = k;
    }
    if (klo < 0) klo = 0;
    if (khi < 0) khi = L - 1;
    m->wl = origin - klo > 0 ? origin - klo : 0;
    m->wr = khi - origin > 0 ? khi - origin : 0;
    return m;
}

void or_model_free(or_model* m)
{
    if (!m) return;
    free(m->hbar); free(m);
}
/* Per-pixel IRFs: pixel p of every later call uses models[cls[p]] (n models,
 * models[0] normally m itself; numbers >= n use models[0]); cls == NULL
 * restores m everywhere.  The arrays are the caller's and must outlive the
 * calls.  All models share T. */
void or_model_set_classes(or_model* m, int n, or_model* const* models, const uint8_t* cls)
{
    m->ncls = cls ? n : 0;
    m->cls_m = cls ? models : NULL;
    m->cls = cls;
}

int    or_model_origin(const or_model* m) { return m->o; }
double or_model_sigma2(const or_model* m) { return m->sigma2; }
double or_model_fisher(const or_model* m) { return m->fisher; }
void   or_model_window(const or_model* m, int* wl, int* wr) { *wl = m->wl; *wr = m->wr; }

/* h(tau) and dh/dtau: the Catmull-Rom segment holding sample position
 * x = tau + origin; zero where the cubic is negative or beyond the samples. */
static void h_eval(const or_model* m, double tau, double* h, double* hp)
{
    double x = tau + m->o;
    *h = 0.0;
    *hp = 0.0;
    if (!(x > -1.0) || !(x < m->L)) return;
    int k = (int)floor(x);
    double s = x - k;
    double p0 = hb(m, k - 1), p1 = hb(m, k), p2 = hb(m, k + 1), p3 = hb(m, k + 2);
    double v = catmull_rom(p0, p1, p2, p3, s);
    if (v <= 0.0) return;
    *h = v;
    *hp = catmull_rom_ds(p0, p1, p2, p3, s);
}

void or_h(const or_model* m, int n, const double* tau, double* h, double* hp)
{
    for (int i = 0; i < n; ++i) h_eval(m, tau[i], &h[i], &hp[i]);
}

/* S(tau) = sum over all bins t of h(t - tau): the expected photon count of a
 * unit-intensity point at depth tau (Observation model, summed over t).
 * S'(tau) = dS/dtau = -sum_t h'(t - tau).  Direct summation over the support. */
static void S_eval(const or_model* m, double tau, double* S, double* Sp)
{
    int t0 = (int)floor(tau - m->o - 1.0);
    int t1 = (int)ceil(tau + m->L - m->o);
    if (t0 < 0) t0 = 0;
    if (t1 > m->T - 1) t1 = m->T - 1;
    double s = 0.0, sp = 0.0;
    for (int t = t0; t <= t1; ++t) {
        double h, hp;
        h_eval(m, t - tau, &h, &hp);
        s += h;
        sp -= hp;
    }
    *S = s; *Sp = sp;
}

void or_S(const or_model* m, int n, const double* tau, double* S, double* Sp)
{
    for (int i = 0; i < n; ++i) S_eval(m, tau[i], &S[i], &Sp[i]);
}

/* Log-matched-filter weights log((h + eps)/eps), eps = 1/(sbr_guess*T), in
 * fixed point with 16 fractional bits so that the filter score is an exact
 * integer and its argmax does not depend on summation order. */
void or_lmf_table(const or_model* m, double sbr_guess, int64_t* q)
{
    double inv_eps = sbr_guess * (double)m->T;
    for (int k = 0; k < m->L; ++k) q[k] = llround(log1p(m->hbar[k] * inv_eps) * 65536.0);
}

/* ------------------------------------------------------------------------ */
/* Histogram -> photon list                                                  */
/* ------------------------------------------------------------------------ */

/* Active bins of each pixel (bins with one or more photons, Methods), in
 * ascending bin order; the cost of every later step is linear in them. */
int64_t or_compact(const uint16_t* Z, int64_t npix, int T, uint32_t* off, uint32_t* ent)
{
    int64_t e = 0;
    for (int64_t p = 0; p < npix; ++p) {
        off[p] = (uint32_t)e;
        for (int t = 0; t < T; ++t) {
            uint16_t z = Z[p * T + t];
            if (z) ent[e++] = ((uint32_t)t << 16) | z;
        }
    }
    off[npix] = (uint32_t)e;
    return e;
}

static inline int ent_t(uint32_t e) { return (int)(e >> 16); }
static inline int ent_z(uint32_t e) { return (int)(e & 0xffffu); }

/* ------------------------------------------------------------------------ */
/* Likelihood                                                                */
/* ------------------------------------------------------------------------ */

/* Poisson intensity at bin t of pixel p: g*(sum_n r_n h(t - t_n) + b). */
static double lambda_at(const or_model* m, int k_max, const double* t, const double* r,
                        int cnt, double b, double g, int tb)
{
    double s = 0.0;
    for (int k = 0; k < cnt; ++k) {
        double h, hp;
        h_eval(m, tb - t[k], &h, &hp);
        s += r[k] * h;
    }
    (void)k_max;
    return g * (s + b);
}

/* NLL = sum_p [ g(sum_n r_n S(t_n) + T b) - sum_{active (t,z)} z log lambda_t
 *              + sum log z! ].  Exact, since sum_t lambda_t = g(sum r S + T b). */
double or_nll(const or_model* m, int64_t npix, const uint32_t* off, const uint32_t* ent,
              int k_max, const double* t, const double* r, const int* cnt,
              const double* b, const double* g)
{
    double total = 0.0;
    for (int64_t p = 0; p < npix; ++p) {
        if (!(g[p] > 0.0)) continue;
        const or_model* mp = pm(m, p);
        const double* tp = t + p * k_max;
        const double* rp = r + p * k_max;
        double sumS = 0.0;
        for (int k = 0; k < cnt[p]; ++k) {
            double S, Sp;
            S_eval(mp, tp[k], &S, &Sp);
            sumS += rp[k] * S;
        }
        double term = g[p] * (sumS + m->T * b[p]);
        for (uint32_t e = off[p]; e < off[p + 1]; ++e) {
            int tb = ent_t(ent[e]), z = ent_z(ent[e]);
            double lam = lambda_at(mp, k_max, tp, rp, cnt[p], b[p], g[p], tb);
            term -= z * log(lam);
            term += lgamma(z + 1.0);
        }
        total += term;
    }
    return total;
}

double or_nll_dense(const or_model* m, int64_t npix, const uint16_t* Z,
                    int k_max, const double* t, const double* r, const int* cnt,
                    const double* b, const double* g)
{
    double total = 0.0;
    for (int64_t p = 0; p < npix; ++p) {
        if (!(g[p] > 0.0)) continue;
        for (int tb = 0; tb < m->T; ++tb) {
            double lam = lambda_at(pm(m, p), k_max, t + p * k_max, r + p * k_max, cnt[p], b[p], g[p], tb);
            int z = Z[p * m->T + tb];
            total += lam - z * log(lam) + lgamma(z + 1.0);
        }
    }
    return total;
}

/* Partial derivatives of the NLL:
 *   d/dt_n = g r_n [ S'(t_n) + sum z h'(t - t_n)/lambda_t ]
 *   d/dr_n = g     [ S(t_n)  - sum z h(t - t_n)/lambda_t  ]
 *   d/db   = g     [ T       - sum z / lambda_t           ]
 * and the sums of the absolute values of their terms (tolerance scale). */
void or_grad(const or_model* m, int64_t npix, const uint32_t* off, const uint32_t* ent,
             int k_max, const double* t, const double* r, const int* cnt,
             const double* b, const double* g,
             double* gt, double* gr, double* gb,
             double* at, double* ar, double* ab)
{
    for (int64_t p = 0; p < npix; ++p) {
        const or_model* mp = pm(m, p);
        const double* tp = t + p * k_max;
        const double* rp = r + p * k_max;
        double G = g[p];
        double st[64], sr[64], ast[64], asr[64];
        double sb = 0.0;
        int c = cnt[p];
        for (int k = 0; k < c; ++k) st[k] = sr[k] = ast[k] = asr[k] = 0.0;
        if (G > 0.0) {
            for (uint32_t e = off[p]; e < off[p + 1]; ++e) {
                int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                double lam = lambda_at(mp, k_max, tp, rp, c, b[p], G, tb);
                for (int k = 0; k < c; ++k) {
                    double h, hp;
                    h_eval(mp, tb - tp[k], &h, &hp);
                    st[k] += z * hp / lam;
                    ast[k] += z * fabs(hp) / lam;
                    sr[k] += z * h / lam;
                    asr[k] += z * h / lam;
                }
                sb += z / lam;
            }
        }
        for (int k = 0; k < k_max; ++k) {
            gt[p * k_max + k] = gr[p * k_max + k] = 0.0;
            at[p * k_max + k] = ar[p * k_max + k] = 0.0;
        }
        for (int k = 0; k < c; ++k) {
            double S, Sp;
            S_eval(mp, tp[k], &S, &Sp);
            /* S' is itself a sum over bins: its terms count in the scale */
            double asp = 0.0;
            for (int t = 0; t < m->T; ++t) {
                double h, hp;
                h_eval(mp, t - tp[k], &h, &hp);
                asp += fabs(hp);
            }
            gt[p * k_max + k] = G * rp[k] * (Sp + st[k]);
            at[p * k_max + k] = G * fabs(rp[k]) * (asp + ast[k]);
            gr[p * k_max + k] = G * (S - sr[k]);
            ar[p * k_max + k] = G * (S + asr[k]);
        }
        gb[p] = G * (m->T - sb);
        ab[p] = G * (m->T + sb);
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbourhoods in world coordinates                                       */
/* ------------------------------------------------------------------------ */

/* Squared world distance between slot ka of pixel (fa, ia, ja) and slot kb of
 * pixel (fb, ib, jb): X = j p_xy, Y = i p_xy, Z = t dz (orthographic). */
/* The map f from (pixel, depth) to world coordinates (Observation model: the
 * camera parameters, such as the focal length, enter f).  persp = 0:
 * orthographic, X = j p_xy, Y = i p_xy, Z = t dz.  persp > 0 (reading): a
 * pinhole camera at the origin looking along +Z; pixel (i, j) of a rows x cols
 * frame sees along the unit ray v of (persp (j - cx), persp (i - cy), 1),
 * cx = (cols - 1)/2, cy = (rows - 1)/2 (persp: the tangent of one pixel's
 * angle), and depth t is the range t dz along that ray (time of flight), so
 * the point is t dz v. */
static void ray(const or_params* p, int rows, int cols, int i, int j, double v[3])
{
    if (!(p->persp > 0.0)) { v[0] = 0.0; v[1] = 0.0; v[2] = 1.0; return; }
    double u = p->persp * (j - 0.5 * (cols - 1)), w = p->persp * (i - 0.5 * (rows - 1));
    double nrm = sqrt(u * u + w * w + 1.0);
    v[0] = u / nrm; v[1] = w / nrm; v[2] = 1.0 / nrm;
}

/* World position of point (ib, jb, tb) relative to point (ia, ja, ta). */
static void rel(const or_params* p, int rows, int cols, int ia, int ja, double ta, int ib, int jb, double tb,
                double y[3])
{
    if (!(p->persp > 0.0)) {
        y[0] = (jb - ja) * p->p_xy; y[1] = (ib - ia) * p->p_xy; y[2] = (tb - ta) * p->dz;
        return;
    }
    double va[3], vb[3];
    ray(p, rows, cols, ia, ja, va);
    ray(p, rows, cols, ib, jb, vb);
    for (int c = 0; c < 3; ++c) y[c] = (tb * vb[c] - ta * va[c]) * p->dz;
}

static double dist2(const or_params* p, int rows, int cols, int ia, int ja, double ta, int ib, int jb, double tb)
{
    double y[3];
    rel(p, rows, cols, ia, ja, ta, ib, jb, tb, y);
    return y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
}

static int apss_radius(const or_params* p) { return (int)ceil(p->h_apss / p->p_xy); }

/* Points of the same frame closer than h_apss to point q (itself included),
 * searched either in the (2R+1)^2 pixel window or over the whole frame.
 * Returns the neighbour count; indices (pixel*k_max + slot) go to out. */
static int neighbours(const or_params* p, int F, int rows, int cols, const double* t,
                      const int* cnt, int64_t q, int brute, int64_t* out, int cap)
{
    (void)F;
    int K = p->k_max;
    int64_t pix = q / K;
    int64_t fr = pix / ((int64_t)rows * cols);
    int i = (int)((pix / cols) % rows), j = (int)(pix % cols);
    double h2 = p->h_apss * p->h_apss;
    int R = brute ? (rows > cols ? rows : cols) : apss_radius(p);
    int n = 0;
    for (int i2 = i - R; i2 <= i + R; ++i2) {
        if (i2 < 0 || i2 >= rows) continue;
        for (int j2 = j - R; j2 <= j + R; ++j2) {
            if (j2 < 0 || j2 >= cols) continue;
            int64_t pp = (fr * rows + i2) * cols + j2;
            for (int k = 0; k < cnt[pp]; ++k) {
                if (dist2(p, rows, cols, i, j, t[q], i2, j2, t[pp * K + k]) < h2) {
                    if (n < cap) out[n] = pp * K + k;
                    ++n;
                }
            }
        }
    }
    return n;
}

void or_apss_neighbours(const or_params* p, int F, int rows, int cols,
                        const double* t, const int* cnt, int64_t q,
                        int brute_force, int64_t* out, int cap)
{
    int n = neighbours(p, F, rows, cols, t, cnt, q, brute_force, out + 1, cap - 1);
    out[0] = n;
}

/* Compact-support kernel of the APSS fit: (1 - d^2/h^2)^4 for d < h. */
static double apss_weight(double d2, double h2)
{
    double a = 1.0 - d2 / h2;
    return a * a * a * a;
}

/* ------------------------------------------------------------------------ */
/* Initialisation (Methods: each pixel independently)                        */
/* ------------------------------------------------------------------------ */

/* Reading (the paper's initialisation is in its supplement): a log-matched
 * filter per pixel.  Photons of the (2 r_init + 1)^2 window are pooled; the
 * score L(tau) = sum z log((h(t - tau) + eps)/eps) is evaluated at every
 * integer tau; peaks are taken greedily (largest score, smallest tau on ties),
 * each suppressing |tau - tau*| <= w_nms, while the photons in the peak window
 * exceed the background expectation by kappa standard deviations (and n_min).
 * The window spans the lags holding 5%..95% of the IRF mass.  An accepted
 * peak claims the bins of its window; later peaks are scored on unclaimed
 * photons only and count only unclaimed bins (matching pursuit).  Intensity from the pixel's own photons in
 * the peak's bins minus background; background from the photons outside the
 * accepted windows.  Peaks with no excess photons are dropped. */
void or_init(const or_model* m, const or_params* p, int F, int rows, int cols,
             const uint32_t* off, const uint32_t* ent, const double* g,
             double* t, double* r, double* n, int* cnt, double* b)
{
    int T = m->T, K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    int64_t* q = (int64_t*)malloc(sizeof(int64_t) * T);
    int64_t* agg = (int64_t*)malloc(sizeof(int64_t) * T);
    int64_t* score = (int64_t*)malloc(sizeof(int64_t) * T);
    char* supp = (char*)malloc(T);
    char* claimed = (char*)malloc(T);   /* bin -> 1 + index of the accepted peak owning it */
    int Ri = p->r_init;
    const or_model* mq = NULL;          /* the model q was built for */
    for (int64_t pix = 0; pix < npix; ++pix) {
        /* the pixel's IRF scores its window's pooled photons */
        const or_model* mm = pm(m, pix);
        int L = mm->L, o = mm->o;
        int wnms = p->w_nms > 0 ? p->w_nms : (int)ceil(fmax(1.0, 2.0 * sqrt(mm->sigma2)));
        if (mm != mq) {
            or_lmf_table(mm, p->sbr_guess, q);
            mq = mm;
        }
        for (int k = 0; k < K; ++k) {
            t[pix * K + k] = 0.0; r[pix * K + k] = 0.0;
            n[(pix * K + k) * 3 + 0] = 0.0; n[(pix * K + k) * 3 + 1] = 0.0; n[(pix * K + k) * 3 + 2] = -1.0;
        }
        cnt[pix] = 0;
        double G = g[pix];
        if (!(G > 0.0)) { b[pix] = p->b_min; continue; }
        int64_t fr = pix / ((int64_t)rows * cols);
        int i = (int)((pix / cols) % rows), j = (int)(pix % cols);
        /* pooled photons of the window */
        for (int tb = 0; tb < T; ++tb) agg[tb] = 0;
        for (int i2 = i - Ri; i2 <= i + Ri; ++i2) {
            if (i2 < 0 || i2 >= rows) continue;
            for (int j2 = j - Ri; j2 <= j + Ri; ++j2) {
                if (j2 < 0 || j2 >= cols) continue;
                int64_t pp = (fr * rows + i2) * cols + j2;
                for (uint32_t e = off[pp]; e < off[pp + 1]; ++e) agg[ent_t(ent[e])] += ent_z(ent[e]);
            }
        }
        int64_t ntot = 0;
        for (int tb = 0; tb < T; ++tb) ntot += agg[tb];
        for (int tau = 0; tau < T; ++tau) { supp[tau] = 0; claimed[tau] = 0; }
        /* greedy peaks */
        int pk[64], lo[64], hi[64];
        int npk = 0;
        for (int it = 0; it < p->k_init && it < 64; ++it) {
            /* score over the photons no accepted peak has claimed yet */
            for (int tau = 0; tau < T; ++tau) score[tau] = 0;
            for (int tb = 0; tb < T; ++tb) {
                if (!agg[tb] || claimed[tb]) continue;
                for (int k = 0; k < L; ++k) {
                    int tau = tb - k + o;
                    if (tau >= 0 && tau < T) score[tau] += agg[tb] * q[k];
                }
            }
            int best = -1;
            int64_t bestv = 0;
            for (int tau = 0; tau < T; ++tau) {
                if (supp[tau]) continue;
                if (best < 0 || score[tau] > bestv) { best = tau; bestv = score[tau]; }
            }
            if (best < 0) break;
            int a = best - mm->wl < 0 ? 0 : best - mm->wl;
            int c = best + mm->wr > T - 1 ? T - 1 : best + mm->wr;
            /* the window's bins not already claimed by an accepted peak */
            int win = 0;
            int64_t nwin = 0;
            for (int tb = a; tb <= c; ++tb)
                if (!claimed[tb]) { ++win; nwin += agg[tb]; }
            double bw = (double)ntot * (double)win / (double)T;
            double d = (double)nwin - bw;
            int accept = win > 0 && nwin >= p->n_min && d >= 0.0
                         && d * d >= (p->kappa * p->kappa) * bw;
            int s0 = best - wnms < 0 ? 0 : best - wnms;
            int s1 = best + wnms > T - 1 ? T - 1 : best + wnms;
            for (int tau = s0; tau <= s1; ++tau) supp[tau] = 1;
            if (!accept) break;
            pk[npk] = best; lo[npk] = a; hi[npk] = c; ++npk;
            for (int tb = a; tb <= c; ++tb) if (!claimed[tb]) claimed[tb] = (char)npk;   /* peak index + 1 */
        }
        /* intensities and background from the pixel's own photons */
        int64_t zp = 0;
        for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) zp += ent_z(ent[e]);
        int64_t nown[64];
        int64_t sum_n = 0, sum_w = 0;
        int64_t wk[64];
        for (int k = 0; k < npk; ++k) {
            nown[k] = 0;
            wk[k] = 0;
            for (int tb = lo[k]; tb <= hi[k]; ++tb) if (claimed[tb] == k + 1) ++wk[k];
            for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
                int tb = ent_t(ent[e]);
                if (claimed[tb] == k + 1) nown[k] += ent_z(ent[e]);
            }
            sum_n += nown[k];
            sum_w += wk[k];
        }
        int64_t num = zp - sum_n;
        if (num < 0) num = 0;
        int64_t den = (int64_t)T - sum_w;
        /* keep the peaks with a positive background-corrected count */
        int kept_t[64];
        double kept_r[64];
        int nk = 0;
        for (int k = 0; k < npk; ++k) {
            int64_t win = wk[k];
            int keep = den > 0 ? (nown[k] * den > num * win) : (nown[k] > 0);
            double H = 0.0;
            for (int tb = lo[k]; tb <= hi[k]; ++tb)
                if (claimed[tb] == k + 1) H += hb(mm, tb - pk[k] + o);
            if (!keep || !(H > 0.0)) continue;
            double excess = den > 0 ? (double)nown[k] - (double)num * (double)win / (double)den
                                    : (double)nown[k];
            kept_t[nk] = pk[k];
            kept_r[nk] = excess / (G * H);
            ++nk;
        }
        /* ascending depth (peaks are distinct) */
        for (int a = 1; a < nk; ++a)
            for (int c = a; c > 0 && kept_t[c] < kept_t[c - 1]; --c) {
                int tt = kept_t[c]; kept_t[c] = kept_t[c - 1]; kept_t[c - 1] = tt;
                double rr = kept_r[c]; kept_r[c] = kept_r[c - 1]; kept_r[c - 1] = rr;
            }
        if (nk > K) nk = K;
        for (int k = 0; k < nk; ++k) { t[pix * K + k] = kept_t[k]; r[pix * K + k] = kept_r[k]; }
        cnt[pix] = nk;
        double bown = den > 0 ? (double)num / (double)den : 0.0;
        double b0 = bown / G;
        b[pix] = b0 > p->b_min ? b0 : p->b_min;
    }
    free(q); free(agg); free(score); free(supp); free(claimed);
}

/* Initial normals (reading; APSS needs oriented normals): weighted
 * least-squares plane Z = a + c1 X + c2 Y over the APSS neighbourhood, in
 * coordinates local to the point; n = (c1, c2, -1)/|.| faces the sensor.
 * Fewer than 3 neighbours or a near-singular system give n = (0, 0, -1). */
void or_init_normals(const or_params* p, int F, int rows, int cols,
                     const double* t, const int* cnt, double* n)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    double h2 = p->h_apss * p->h_apss;
    int cap = 4096;
    int64_t* nb = (int64_t*)malloc(sizeof(int64_t) * cap);
    for (int64_t pix = 0; pix < npix; ++pix) {
        int i = (int)((pix / cols) % rows), j = (int)(pix % cols);
        for (int k = 0; k < cnt[pix]; ++k) {
            int64_t q = pix * K + k;
            int nn = neighbours(p, F, rows, cols, t, cnt, q, 0, nb, cap);
            double* nq = n + q * 3;
            nq[0] = 0.0; nq[1] = 0.0; nq[2] = -1.0;
            if (nn < 3) continue;
            double M[3][3] = {{0}}, v[3] = {0};
            double W = 0.0;
            for (int a = 0; a < nn && a < cap; ++a) {
                int64_t pm = nb[a] / K;
                int i2 = (int)((pm / cols) % rows), j2 = (int)(pm % cols);
                double yv[3];
                rel(p, rows, cols, i, j, t[q], i2, j2, t[nb[a]], yv);
                double x = yv[0], y = yv[1], z = yv[2];
                double w = apss_weight(x * x + y * y + z * z, h2);
                double basis[3] = {1.0, x, y};
                for (int r0 = 0; r0 < 3; ++r0) {
                    for (int c0 = 0; c0 < 3; ++c0) M[r0][c0] += w * basis[r0] * basis[c0];
                    v[r0] += w * basis[r0] * z;
                }
                W += w;
            }
            double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                       - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                       + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            double scale = W * W * W * h2 * h2;
            if (!(det > 1e-9 * scale)) continue;
            /* Cramer's rule for the two slopes */
            double d1 = M[0][0] * (v[1] * M[2][2] - M[1][2] * v[2])
                      - v[0] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                      + M[0][2] * (M[1][0] * v[2] - v[1] * M[2][0]);
            double d2 = M[0][0] * (M[1][1] * v[2] - v[1] * M[2][1])
                      - M[0][1] * (M[1][0] * v[2] - v[1] * M[2][0])
                      + v[0] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            double c1 = d1 / det, c2 = d2 / det;
            double nrm = sqrt(c1 * c1 + c2 * c2 + 1.0);
            nq[0] = c1 / nrm; nq[1] = c2 / nrm; nq[2] = -1.0 / nrm;
            /* facing the sensor: against the pixel's ray.  Reading for the
             * pinhole camera: a plane containing the line of sight (within
             * 1e-6, e.g. two points of one pixel among three neighbours) has
             * no side facing the sensor; its point takes n = -v. */
            double vr[3];
            ray(p, rows, cols, i, j, vr);
            double nv = nq[0] * vr[0] + nq[1] * vr[1] + nq[2] * vr[2];
            if (p->persp > 0.0 && fabs(nv) <= 1e-6)
                for (int c = 0; c < 3; ++c) nq[c] = -vr[c];
            else if (nv > 0.0)
                for (int c = 0; c < 3; ++c) nq[c] = -nq[c];
        }
    }
    free(nb);
}

/* ------------------------------------------------------------------------ */
/* Depth block                                                               */
/* ------------------------------------------------------------------------ */

/* Gradient step on t (Reconstruction algorithm, depth update).  Reading of
 * the step size: the inverse of the expected curvature g r I_h, I_h the
 * IRF's shift Fisher information per photon (a 1/Lipschitz step), i.e.
 *   t_n <- clamp(t_n - (beta_t / I_h) [S'(t_n) + sum z h'(t - t_n)/lambda_t],
 * with the move clipped to |dmax| and t kept in [0, T-1].  All points of a
 * pixel use lambda from before the step (Jacobi).  Dead pixels and points of
 * zero intensity do not move. */
void or_depth_step(const or_model* m, const or_params* p, int64_t npix,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   double* t, const double* r, const int* cnt, const double* b)
{
    int K = p->k_max;
    double* t0 = (double*)malloc(sizeof(double) * K);
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        int c = cnt[pix];
        if (!(G > 0.0) || c == 0) continue;
        const or_model* mp = pm(m, pix);
        double dmax = p->dmax > 0.0 ? p->dmax : fmax(0.5, 1.0 / sqrt(mp->fisher));
        double* tp = t + pix * K;
        const double* rp = r + pix * K;
        for (int k = 0; k < c; ++k) t0[k] = tp[k];
        for (int k = 0; k < c; ++k) {
            if (!(rp[k] > 0.0)) continue;
            double acc = 0.0;
            for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
                int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                double lam = lambda_at(mp, K, t0, rp, c, b[pix], G, tb);
                double h, hp;
                h_eval(mp, tb - t0[k], &h, &hp);
                acc += z * hp / lam;
            }
            double S, Sp;
            S_eval(mp, t0[k], &S, &Sp);
            double step = -p->beta_t * (Sp + acc) / mp->fisher;
            if (step > dmax) step = dmax;
            if (step < -dmax) step = -dmax;
            double tn = t0[k] + step;
            if (tn < 0.0) tn = 0.0;
            if (tn > m->T - 1) tn = m->T - 1;
            tp[k] = tn;
        }
    }
    free(t0);
}

/* APSS denoising of the point cloud (Reconstruction algorithm, depth update;
 * algebraic sphere fit of the cited APSS work).  For each point q, with
 * neighbours y_m = x_m - x_q closer than h and weights w_m = (1 - d^2/h^2)^4,
 * the algebraic sphere s(y) = u0 + ul.y + u4 |y|^2 minimises
 * sum w |grad s(y_m) - n_m|^2 (which gives u4 and ul) and then
 * sum w s(y_m)^2 over u0:
 *   W = sum w, P = sum w y, N = sum w n, PN = sum w y.n, PP = sum w y.y,
 *   u4 = (PN - P.N/W) / (2 (PP - P.P/W)),  ul = (N - 2 u4 P)/W,
 *   u0 = -(ul.P + u4 PP)/W.
 * Reading: q is projected onto the sphere along its own line of sight (only
 * its depth moves), to the root nearest to it; its normal becomes the
 * normalised gradient there, oriented towards the sensor (negative Z).  One
 * fit per iteration, all points read the pre-step cloud (Jacobi).  Points with
 * fewer than m_min neighbours, a degenerate spread, or a line of sight tangent
 * to the sphere are left unchanged; the move is clipped to [-h, h]. */
void or_apss(const or_params* p, int F, int rows, int cols, int T,
             double* t, double* n, const int* cnt)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    int64_t nslot = npix * K;
    double* t0 = (double*)malloc(sizeof(double) * nslot);
    double* n0 = (double*)malloc(sizeof(double) * nslot * 3);
    memcpy(t0, t, sizeof(double) * nslot);
    memcpy(n0, n, sizeof(double) * nslot * 3);
    double h = p->h_apss, h2 = h * h;
    int cap = 4096;
    int64_t* nb = (int64_t*)malloc(sizeof(int64_t) * cap);
    for (int64_t pix = 0; pix < npix; ++pix) {
        int i = (int)((pix / cols) % rows), j = (int)(pix % cols);
        for (int k = 0; k < cnt[pix]; ++k) {
            int64_t q = pix * K + k;
            int nn = neighbours(p, F, rows, cols, t0, cnt, q, 0, nb, cap);
            if (nn < p->m_min) continue;
            double W = 0.0, P[3] = {0, 0, 0}, N[3] = {0, 0, 0}, PN = 0.0, PP = 0.0;
            for (int a = 0; a < nn && a < cap; ++a) {
                int64_t pm = nb[a] / K;
                int i2 = (int)((pm / cols) % rows), j2 = (int)(pm % cols);
                double y[3];
                rel(p, rows, cols, i, j, t0[q], i2, j2, t0[nb[a]], y);
                const double* nm = n0 + nb[a] * 3;
                double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
                double w = apss_weight(yy, h2);
                W += w;
                for (int c = 0; c < 3; ++c) { P[c] += w * y[c]; N[c] += w * nm[c]; }
                PN += w * (y[0] * nm[0] + y[1] * nm[1] + y[2] * nm[2]);
                PP += w * yy;
            }
            double PdP = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
            double PdN = P[0] * N[0] + P[1] * N[1] + P[2] * N[2];
            double D = PP - PdP / W;
            if (!(D > 1e-12 * W * h2)) continue;
            double u4 = 0.5 * (PN - PdN / W) / D;
            double ul[3];
            for (int c = 0; c < 3; ++c) ul[c] = (N[c] - 2.0 * u4 * P[c]) / W;
            double u0 = -(ul[0] * P[0] + ul[1] * P[1] + ul[2] * P[2] + u4 * PP) / W;
            /* the query moves along its own line of sight v: y = s v */
            double v[3];
            ray(p, rows, cols, i, j, v);
            double bz = ul[0] * v[0] + ul[1] * v[1] + ul[2] * v[2];
            double nul = sqrt(ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2]);
            if (!(fabs(bz) > 1e-6 * nul)) continue;
            double disc = bz * bz - 4.0 * u4 * u0;
            double s;
            if (disc < 0.0) s = -bz / (2.0 * u4);
            else s = -2.0 * u0 / (bz + (bz > 0.0 ? 1.0 : -1.0) * sqrt(disc));
            if (s > h) s = h;
            if (s < -h) s = -h;
            double tn = t0[q] + s / p->dz;
            if (tn < 0.0) tn = 0.0;
            if (tn > T - 1) tn = T - 1;
            t[q] = tn;
            double gr[3] = {ul[0] + 2.0 * u4 * s * v[0], ul[1] + 2.0 * u4 * s * v[1], ul[2] + 2.0 * u4 * s * v[2]};
            double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
            double gv = gr[0] * v[0] + gr[1] * v[1] + gr[2] * v[2];
            if (p->persp > 0.0 && fabs(gv) <= 1e-6 * gn) {
                /* pinhole camera, gradient perpendicular to the line of sight
                 * (the vertex of a missed sphere): the normal faces the sensor */
                for (int c = 0; c < 3; ++c) n[q * 3 + c] = -v[c];
            } else if (gn > 0.0) {
                double sg = gv > 0.0 ? -1.0 : 1.0;
                for (int c = 0; c < 3; ++c) n[q * 3 + c] = sg * gr[c] / gn;
            }
        }
    }
    free(nb); free(t0); free(n0);
}

/* Reading (not in the paper): two points of one pixel closer than d_merge bins
 * describe one surface; they are merged in ascending depth order into one
 * point at the intensity-weighted depth with the summed intensity and the
 * intensity-weighted normal. */
void or_merge(const or_model* m, const or_params* p, int64_t npix,
              double* t, double* r, double* n, int* cnt)
{
    int K = p->k_max;
    for (int64_t pix = 0; pix < npix; ++pix) {
        int c = cnt[pix];
        if (c < 2) continue;
        double dm = p->d_merge > 0.0 ? p->d_merge : fmax(1.0, sqrt(pm(m, pix)->sigma2));
        double* tp = t + pix * K;
        double* rp = r + pix * K;
        double* np = n + pix * K * 3;
        /* stable insertion sort by depth */
        for (int a = 1; a < c; ++a)
            for (int b = a; b > 0 && tp[b] < tp[b - 1]; --b) {
                double x = tp[b]; tp[b] = tp[b - 1]; tp[b - 1] = x;
                x = rp[b]; rp[b] = rp[b - 1]; rp[b - 1] = x;
                for (int q = 0; q < 3; ++q) { x = np[b * 3 + q]; np[b * 3 + q] = np[(b - 1) * 3 + q]; np[(b - 1) * 3 + q] = x; }
            }
        int a = 0;
        while (a + 1 < c) {
            if (tp[a + 1] - tp[a] < dm) {
                double ra = rp[a], rb = rp[a + 1];
                double tt = (ra + rb > 0.0) ? (ra * tp[a] + rb * tp[a + 1]) / (ra + rb) : 0.5 * (tp[a] + tp[a + 1]);
                double nn[3], nrm = 0.0;
                for (int q = 0; q < 3; ++q) { nn[q] = ra * np[a * 3 + q] + rb * np[(a + 1) * 3 + q]; nrm += nn[q] * nn[q]; }
                nrm = sqrt(nrm);
                if (nrm > 0.0) for (int q = 0; q < 3; ++q) np[a * 3 + q] = nn[q] / nrm;
                tp[a] = tt;
                rp[a] = ra + rb;
                for (int b = a + 1; b + 1 < c; ++b) {
                    tp[b] = tp[b + 1]; rp[b] = rp[b + 1];
                    for (int q = 0; q < 3; ++q) np[b * 3 + q] = np[(b + 1) * 3 + q];
                }
                --c;
                tp[c] = 0.0; rp[c] = 0.0; np[c * 3 + 0] = 0.0; np[c * 3 + 1] = 0.0; np[c * 3 + 2] = -1.0;
            } else {
                ++a;
            }
        }
        cnt[pix] = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Intensity block                                                           */
/* ------------------------------------------------------------------------ */

/* Gradient step on r (Reconstruction algorithm, intensity update).  Reading of
 * the step: the variable metric r/(g S(t_n)), which makes the step
 *   r_n <- max(0, r_n [(1 - beta_r) + beta_r sum z h(t - t_n)/(lambda_t S(t_n))])
 * (expectation-maximisation at beta_r = 1).  lambda uses the new depths and
 * the old intensities and background (Jacobi). */
void or_intensity_step(const or_model* m, const or_params* p, int64_t npix,
                       const uint32_t* off, const uint32_t* ent, const double* g,
                       const double* t, double* r, const int* cnt, const double* b)
{
    int K = p->k_max;
    double* r0 = (double*)malloc(sizeof(double) * K);
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        int c = cnt[pix];
        if (!(G > 0.0) || c == 0) continue;
        const or_model* mp = pm(m, pix);
        const double* tp = t + pix * K;
        double* rp = r + pix * K;
        for (int k = 0; k < c; ++k) r0[k] = rp[k];
        for (int k = 0; k < c; ++k) {
            double S, Sp;
            S_eval(mp, tp[k], &S, &Sp);
            if (!(S > 0.0)) continue;
            double acc = 0.0;
            for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
                int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                double lam = lambda_at(mp, K, tp, r0, c, b[pix], G, tb);
                double h, hp;
                h_eval(mp, tb - tp[k], &h, &hp);
                acc += z * h / lam;
            }
            double v = r0[k] * ((1.0 - p->beta_r) + p->beta_r * acc / S);
            rp[k] = v > 0.0 ? v : 0.0;
        }
    }
    free(r0);
}

/* Intensity denoiser (Reconstruction algorithm, intensity update): a low-pass
 * over nearest neighbours in the manifold the points define, which only
 * correlates points lying on one surface.  Reading: for each of the 8
 * surrounding pixels the single point nearest in world space (lowest slot on
 * ties) is a neighbour if closer than h_int.  The new intensity is the mean
 * over the point and its neighbours on its surface,
 * (r_n + sum of neighbour intensities) / (1 + number of neighbours found)
 * (Jacobi), so a pixel holding no point of that surface takes no part in the
 * mean.  Option ilp_box = 1 divides by 1 + the number of surrounding pixels
 * inside the image instead (a 3 x 3 box in which a missing neighbour counts
 * as zero intensity, which attenuates isolated points).  Points then below
 * r_min are removed (minimum admissible intensity) and the slots are
 * compacted in depth order. */
void or_intensity_filter(const or_params* p, int F, int rows, int cols,
                         double* t, double* r, double* n, int* cnt)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    double* rn = (double*)malloc(sizeof(double) * npix * K);
    double hi2 = p->h_int * p->h_int;
    for (int64_t pix = 0; pix < npix; ++pix) {
        int64_t fr = pix / ((int64_t)rows * cols);
        int i = (int)((pix / cols) % rows), j = (int)(pix % cols);
        for (int k = 0; k < cnt[pix]; ++k) {
            int64_t q = pix * K + k;
            double sum = r[q];
            int deg = 0, nside = 0;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    if (di == 0 && dj == 0) continue;
                    int i2 = i + di, j2 = j + dj;
                    if (i2 < 0 || i2 >= rows || j2 < 0 || j2 >= cols) continue;
                    ++nside;
                    int64_t pp = (fr * rows + i2) * cols + j2;
                    int best = -1;
                    double bd = 0.0;
                    for (int k2 = 0; k2 < cnt[pp]; ++k2) {
                        double d2 = dist2(p, rows, cols, i, j, t[q], i2, j2, t[pp * K + k2]);
                        if (best < 0 || d2 < bd) { best = k2; bd = d2; }
                    }
                    if (best >= 0 && bd < hi2) { sum += r[pp * K + best]; ++deg; }
                }
            rn[q] = sum / (1 + (p->ilp_box ? nside : deg));
        }
    }
    for (int64_t pix = 0; pix < npix; ++pix) {
        int c = 0;
        for (int k = 0; k < cnt[pix]; ++k) {
            int64_t q = pix * K + k;
            if (rn[q] < p->r_min) continue;
            int64_t d = pix * K + c;
            t[d] = t[q]; r[d] = rn[q];
            for (int a = 0; a < 3; ++a) n[d * 3 + a] = n[q * 3 + a];
            ++c;
        }
        for (int k = c; k < K; ++k) {
            int64_t d = pix * K + k;
            t[d] = 0.0; r[d] = 0.0; n[d * 3 + 0] = 0.0; n[d * 3 + 1] = 0.0; n[d * 3 + 2] = -1.0;
        }
        cnt[pix] = c;
    }
    free(rn);
}

/* ------------------------------------------------------------------------ */
/* Background block                                                          */
/* ------------------------------------------------------------------------ */

/* Gradient step on b (Reconstruction algorithm, background update), with the
 * variable metric b/(g T):  b <- max(b_min, b [(1 - beta_b) + beta_b sum z/(lambda_t T)]),
 * lambda from the new depths and intensities. */
void or_bg_step(const or_model* m, const or_params* p, int64_t npix,
                const uint32_t* off, const uint32_t* ent, const double* g,
                const double* t, const double* r, const int* cnt, double* b)
{
    int K = p->k_max;
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        if (!(G > 0.0)) continue;
        double acc = 0.0;
        for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
            int tb = ent_t(ent[e]), z = ent_z(ent[e]);
            double lam = lambda_at(pm(m, pix), K, t + pix * K, r + pix * K, cnt[pix], b[pix], G, tb);
            acc += z / lam;
        }
        double v = b[pix] * ((1.0 - p->beta_b) + p->beta_b * acc / m->T);
        b[pix] = v > p->b_min ? v : p->b_min;
    }
}

/* Background denoiser: the paper uses an FFT-based image filter for arrays and
 * monostatic scanners, the identity for bistatic ones.  Reading: circular
 * convolution of each frame's background image with a normalised sampled
 * Gaussian of sigma_b pixels truncated at ceil(4 sigma_b) (what an FFT filter
 * computes), rows then columns; sigma_b = 0 is the identity.  Floor at b_min. */
void or_bg_filter(const or_params* p, int F, int rows, int cols, double* b)
{
    int64_t npf = (int64_t)rows * cols;
    if (p->sigma_b > 0.0) {
        int rb = (int)ceil(4.0 * p->sigma_b);
        double* w = (double*)malloc(sizeof(double) * (2 * rb + 1));
        double s = 0.0;
        for (int d = -rb; d <= rb; ++d) { w[d + rb] = exp(-(double)d * d / (2.0 * p->sigma_b * p->sigma_b)); s += w[d + rb]; }
        for (int d = 0; d <= 2 * rb; ++d) w[d] /= s;
        double* tmp = (double*)malloc(sizeof(double) * npf);
        for (int f = 0; f < F; ++f) {
            double* bf = b + f * npf;
            for (int i = 0; i < rows; ++i)
                for (int j = 0; j < cols; ++j) {
                    double a = 0.0;
                    for (int d = -rb; d <= rb; ++d) {
                        int jj = ((j + d) % cols + cols) % cols;
                        a += w[d + rb] * bf[(int64_t)i * cols + jj];
                    }
                    tmp[(int64_t)i * cols + j] = a;
                }
            for (int i = 0; i < rows; ++i)
                for (int j = 0; j < cols; ++j) {
                    double a = 0.0;
                    for (int d = -rb; d <= rb; ++d) {
                        int ii = ((i + d) % rows + rows) % rows;
                        a += w[d + rb] * tmp[(int64_t)ii * cols + j];
                    }
                    bf[(int64_t)i * cols + j] = a;
                }
        }
        free(tmp); free(w);
    }
    for (int64_t q = 0; q < (int64_t)F * npf; ++q) if (b[q] < p->b_min) b[q] = p->b_min;
}

/* ------------------------------------------------------------------------ */
/* Whole loop                                                                */
/* ------------------------------------------------------------------------ */

/* One iteration of the block diagram: depth (gradient step, APSS), intensity
 * (gradient step, merge of coincident points first, low-pass, threshold),
 * background (gradient step, filter).  Parity unpinned as a whole: it is
 * checked against the GPU path, while each step has its own pins. */
void or_iterate(const or_model* m, const or_params* p, int F, int rows, int cols,
                const uint32_t* off, const uint32_t* ent, const double* g,
                double* t, double* r, double* n, int* cnt, double* b)
{
    int64_t npix = (int64_t)F * rows * cols;
    or_depth_step(m, p, npix, off, ent, g, t, r, cnt, b);
    if (p->use_apss) or_apss(p, F, rows, cols, m->T, t, n, cnt);
    or_merge(m, p, npix, t, r, n, cnt);
    or_intensity_step(m, p, npix, off, ent, g, t, r, cnt, b);
    or_intensity_filter(p, F, rows, cols, t, r, n, cnt);
    or_bg_step(m, p, npix, off, ent, g, t, r, cnt, b);
    or_bg_filter(p, F, rows, cols, b);
}

void or_reconstruct(const or_model* m, const or_params* p, int F, int rows, int cols,
                    const uint32_t* off, const uint32_t* ent, const double* g,
                    double* t, double* r, double* n, int* cnt, double* b)
{
    or_init(m, p, F, rows, cols, off, ent, g, t, r, n, cnt, b);
    or_init_normals(p, F, rows, cols, t, cnt, n);
    for (int it = 0; it < p->n_iter; ++it) or_iterate(m, p, F, rows, cols, off, ent, g, t, r, n, cnt, b);
}

/* ------------------------------------------------------------------------ */
/* Super-resolution (Results, dynamic scenes; Discussion)                    */
/* ------------------------------------------------------------------------ */

/* The map f may undersample: the point cloud lives on a grid s times finer
 * than the lidar pixels, frame f holding (rows s) x (cols s) point-grid pixels,
 * and the s x s point-grid pixels (i s + u, j s + v), 0 <= u, v < s, all map
 * to lidar pixel (i, j).  Gain and background stay per lidar pixel; the
 * lidar pixel's Poisson intensity adds the points of all its s^2 point-grid
 * pixels:
 *   lambda_{p,t} = g_p ( sum_{q -> p} sum_{n in q} r_n h(t - t_n) + b_p ).
 * Point arrays (t, r, n, cnt) are indexed by point-grid pixel, b and g by
 * lidar pixel; rows and cols below are the lidar frame's. */

/* Point-grid pixel of sub-position u (row-major in the s x s block) of lidar
 * pixel p. */
static int64_t sr_sub(int s, int rows, int cols, int64_t p, int u)
{
    int64_t fr = p / ((int64_t)rows * cols);
    int64_t i = (p / cols) % rows, j = p % cols;
    int64_t fi = i * s + u / s, fj = j * s + u % s;
    return (fr * rows * s + fi) * ((int64_t)cols * s) + fj;
}

static double sr_lambda(const or_model* m, int s, int rows, int cols, int K, int64_t p,
                        const double* t, const double* r, const int* cnt, double b, double g, int tb)
{
    double acc = 0.0;
    for (int u = 0; u < s * s; ++u) {
        int64_t q = sr_sub(s, rows, cols, p, u);
        for (int k = 0; k < cnt[q]; ++k) {
            double h, hp;
            h_eval(m, tb - t[q * K + k], &h, &hp);
            acc += r[q * K + k] * h;
        }
    }
    return g * (acc + b);
}

/* NLL of the super-resolved model (the same active-bin identity as or_nll:
 * sum_t lambda_t = g (sum over the lidar pixel's points r S(t_n) + T b)). */
double or_sr_nll(const or_model* m, int s, int F, int rows, int cols, const uint32_t* off,
                 const uint32_t* ent, int K, const double* t, const double* r, const int* cnt,
                 const double* b, const double* g)
{
    double total = 0.0;
    int64_t npix = (int64_t)F * rows * cols;
    for (int64_t p = 0; p < npix; ++p) {
        if (!(g[p] > 0.0)) continue;
        double sumS = 0.0;
        for (int u = 0; u < s * s; ++u) {
            int64_t q = sr_sub(s, rows, cols, p, u);
            for (int k = 0; k < cnt[q]; ++k) {
                double S, Sp;
                S_eval(m, t[q * K + k], &S, &Sp);
                sumS += r[q * K + k] * S;
            }
        }
        double term = g[p] * (sumS + m->T * b[p]);
        for (uint32_t e = off[p]; e < off[p + 1]; ++e) {
            int tb = ent_t(ent[e]), z = ent_z(ent[e]);
            term -= z * log(sr_lambda(m, s, rows, cols, K, p, t, r, cnt, b[p], g[p], tb));
            term += lgamma(z + 1.0);
        }
        total += term;
    }
    return total;
}

/* Partial derivatives: a point n of point-grid pixel q -> p sees its lidar
 * pixel's lambda,
 *   d/dt_n = g_p r_n [ S'(t_n) + sum_{E_p} z h'(t - t_n)/lambda_{p,t} ]
 *   d/dr_n = g_p     [ S(t_n)  - sum_{E_p} z h(t - t_n)/lambda_{p,t}  ]
 *   d/db_p = g_p     [ T       - sum_{E_p} z / lambda_{p,t}           ]
 * with the sums of the absolute values of the terms (at, ar, ab) as in or_grad.
 * gt, gr, at, ar: [point-grid pixels][K]; gb, ab: [lidar pixels]. */
void or_sr_grad(const or_model* m, int s, int F, int rows, int cols, const uint32_t* off,
                const uint32_t* ent, int K, const double* t, const double* r, const int* cnt,
                const double* b, const double* g, double* gt, double* gr, double* gb,
                double* at, double* ar, double* ab)
{
    int64_t npix = (int64_t)F * rows * cols;
    for (int64_t p = 0; p < npix; ++p) {
        double G = g[p], sb = 0.0;
        for (int u = 0; u < s * s; ++u) {
            int64_t q = sr_sub(s, rows, cols, p, u);
            for (int k = 0; k < K; ++k) {
                int64_t x = q * K + k;
                gt[x] = gr[x] = at[x] = ar[x] = 0.0;
            }
        }
        if (G > 0.0)
            for (uint32_t e = off[p]; e < off[p + 1]; ++e) {
                int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                sb += z / sr_lambda(m, s, rows, cols, K, p, t, r, cnt, b[p], G, tb);
            }
        for (int u = 0; u < s * s && G > 0.0; ++u) {
            int64_t q = sr_sub(s, rows, cols, p, u);
            for (int k = 0; k < cnt[q]; ++k) {
                int64_t x = q * K + k;
                double st = 0.0, ast = 0.0, sr = 0.0;
                for (uint32_t e = off[p]; e < off[p + 1]; ++e) {
                    int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                    double lam = sr_lambda(m, s, rows, cols, K, p, t, r, cnt, b[p], G, tb);
                    double h, hp;
                    h_eval(m, tb - t[x], &h, &hp);
                    st += z * hp / lam;
                    ast += z * fabs(hp) / lam;
                    sr += z * h / lam;
                }
                double S, Sp, asp = 0.0;
                S_eval(m, t[x], &S, &Sp);
                for (int tt = 0; tt < m->T; ++tt) {
                    double h, hp;
                    h_eval(m, tt - t[x], &h, &hp);
                    asp += fabs(hp);
                }
                gt[x] = G * r[x] * (Sp + st);
                at[x] = G * fabs(r[x]) * (asp + ast);
                gr[x] = G * (S - sr);
                ar[x] = G * (S + sr);
            }
        }
        gb[p] = G > 0.0 ? G * (m->T - sb) : 0.0;
        ab[p] = G > 0.0 ? G * (m->T + sb) : 0.0;
    }
}

/* The three gradient steps of or_depth_step / or_intensity_step / or_bg_step
 * under the super-resolved lambda (same step sizes; Jacobi: every point of a
 * lidar pixel sees lambda from before the step). */
void or_sr_depth_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                      const uint32_t* off, const uint32_t* ent, const double* g,
                      double* t, const double* r, const int* cnt, const double* b)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols, nfine = npix * s * s;
    double dmax = p->dmax > 0.0 ? p->dmax : fmax(0.5, 1.0 / sqrt(m->fisher));
    double* t0 = (double*)malloc(sizeof(double) * nfine * K);
    memcpy(t0, t, sizeof(double) * nfine * K);
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        if (!(G > 0.0)) continue;
        for (int u = 0; u < s * s; ++u) {
            int64_t q = sr_sub(s, rows, cols, pix, u);
            for (int k = 0; k < cnt[q]; ++k) {
                int64_t x = q * K + k;
                if (!(r[x] > 0.0)) continue;
                double acc = 0.0;
                for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
                    int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                    double lam = sr_lambda(m, s, rows, cols, K, pix, t0, r, cnt, b[pix], G, tb);
                    double h, hp;
                    h_eval(m, tb - t0[x], &h, &hp);
                    acc += z * hp / lam;
                }
                double S, Sp;
                S_eval(m, t0[x], &S, &Sp);
                double step = -p->beta_t * (Sp + acc) / m->fisher;
                if (step > dmax) step = dmax;
                if (step < -dmax) step = -dmax;
                double tn = t0[x] + step;
                if (tn < 0.0) tn = 0.0;
                if (tn > m->T - 1) tn = m->T - 1;
                t[x] = tn;
            }
        }
    }
    free(t0);
}

void or_sr_intensity_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                          const uint32_t* off, const uint32_t* ent, const double* g,
                          const double* t, double* r, const int* cnt, const double* b)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols, nfine = npix * s * s;
    double* r0 = (double*)malloc(sizeof(double) * nfine * K);
    memcpy(r0, r, sizeof(double) * nfine * K);
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        if (!(G > 0.0)) continue;
        for (int u = 0; u < s * s; ++u) {
            int64_t q = sr_sub(s, rows, cols, pix, u);
            for (int k = 0; k < cnt[q]; ++k) {
                int64_t x = q * K + k;
                double S, Sp;
                S_eval(m, t[x], &S, &Sp);
                if (!(S > 0.0)) continue;
                double acc = 0.0;
                for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
                    int tb = ent_t(ent[e]), z = ent_z(ent[e]);
                    double lam = sr_lambda(m, s, rows, cols, K, pix, t, r0, cnt, b[pix], G, tb);
                    double h, hp;
                    h_eval(m, tb - t[x], &h, &hp);
                    acc += z * h / lam;
                }
                double v = r0[x] * ((1.0 - p->beta_r) + p->beta_r * acc / S);
                r[x] = v > 0.0 ? v : 0.0;
            }
        }
    }
    free(r0);
}

void or_sr_bg_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   const double* t, const double* r, const int* cnt, double* b)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    for (int64_t pix = 0; pix < npix; ++pix) {
        double G = g[pix];
        if (!(G > 0.0)) continue;
        double acc = 0.0;
        for (uint32_t e = off[pix]; e < off[pix + 1]; ++e) {
            int tb = ent_t(ent[e]), z = ent_z(ent[e]);
            acc += z / sr_lambda(m, s, rows, cols, K, pix, t, r, cnt, b[pix], G, tb);
        }
        double v = b[pix] * ((1.0 - p->beta_b) + p->beta_b * acc / m->T);
        b[pix] = v > p->b_min ? v : p->b_min;
    }
}

/* Initial point-grid state (reading; the paper does not say how the finer
 * cloud starts): every point-grid pixel takes the points its lidar pixel's
 * initialisation found (tc, rc, cntc, lidar-pixel arrays), with the intensity
 * shared equally over the s^2 point-grid pixels so that lambda is unchanged.
 * Normals face the sensor until or_init_normals fits them on the point grid. */
void or_sr_expand(int K, int s, int F, int rows, int cols, const double* tc, const double* rc,
                  const int* cntc, double* t, double* r, double* n, int* cnt)
{
    int64_t npix = (int64_t)F * rows * cols;
    for (int64_t p = 0; p < npix; ++p)
        for (int u = 0; u < s * s; ++u) {
            int64_t q = sr_sub(s, rows, cols, p, u);
            cnt[q] = cntc[p];
            for (int k = 0; k < K; ++k) {
                int live = k < cntc[p];
                t[q * K + k] = live ? tc[p * K + k] : 0.0;
                r[q * K + k] = live ? rc[p * K + k] / ((double)s * s) : 0.0;
                n[(q * K + k) * 3 + 0] = 0.0;
                n[(q * K + k) * 3 + 1] = 0.0;
                n[(q * K + k) * 3 + 2] = -1.0;
            }
        }
}

/* One iteration with the super-resolved data term: the depth, intensity and
 * background gradient steps see lidar pixels; APSS, the merge and the
 * intensity low-pass act on the point grid; the background filter on the
 * lidar grid. */
void or_sr_iterate(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   double* t, double* r, double* n, int* cnt, double* b)
{
    int64_t nfine = (int64_t)F * rows * cols * s * s;
    or_sr_depth_step(m, p, s, F, rows, cols, off, ent, g, t, r, cnt, b);
    if (p->use_apss) or_apss(p, F, rows * s, cols * s, m->T, t, n, cnt);
    or_merge(m, p, nfine, t, r, n, cnt);
    or_sr_intensity_step(m, p, s, F, rows, cols, off, ent, g, t, r, cnt, b);
    or_intensity_filter(p, F, rows * s, cols * s, t, r, n, cnt);
    or_sr_bg_step(m, p, s, F, rows, cols, off, ent, g, t, r, cnt, b);
    or_bg_filter(p, F, rows, cols, b);
}

/* Initialisation on the lidar grid (or_init), expansion to the point grid,
 * normals there, then n_iter iterations. */
void or_sr_reconstruct(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                       const uint32_t* off, const uint32_t* ent, const double* g,
                       double* t, double* r, double* n, int* cnt, double* b)
{
    int K = p->k_max;
    int64_t npix = (int64_t)F * rows * cols;
    double* tc = (double*)calloc((size_t)npix * K, sizeof(double));
    double* rc = (double*)calloc((size_t)npix * K, sizeof(double));
    double* nc = (double*)calloc((size_t)npix * K * 3, sizeof(double));
    int* cntc = (int*)calloc((size_t)npix, sizeof(int));
    or_init(m, p, F, rows, cols, off, ent, g, tc, rc, nc, cntc, b);
    or_sr_expand(K, s, F, rows, cols, tc, rc, cntc, t, r, n, cnt);
    or_init_normals(p, F, rows * s, cols * s, t, cnt, n);
    for (int it = 0; it < p->n_iter; ++it) or_sr_iterate(m, p, s, F, rows, cols, off, ent, g, t, r, n, cnt, b);
    free(tc); free(rc); free(nc); free(cntc);
}

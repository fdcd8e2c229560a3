/*
 * rt3d_oracle.h -- FP64 CPU oracle for the plug-and-play point-cloud
 * reconstruction of single-photon lidar data (Tachella et al., "Real-time 3D
 * reconstruction from single-photon lidar data using plug-and-play point
 * cloud denoisers").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Conventions used throughout (readings of points the paper leaves open):
 *   - bins t = 0..T-1; pixel p = (f*rows + i)*cols + j (frame, row, column);
 *   - depth is in bins, as a real number; it is the position of the IRF
 *     origin (sample index `origin` of the given IRF);
 *   - world coordinates are orthographic, X = j*p_xy, Y = i*p_xy, Z = t*dz,
 *     or (persp > 0) those of a pinhole camera: t*dz along the pixel's ray;
 *   - per-pixel point state is pixel-major with stride k_max:
 *       t[p*k_max + k], r[p*k_max + k], n[(p*k_max + k)*3 + c],
 *     cnt[p] live points in slots 0..cnt-1, ascending depth;
 *   - b[p] background (photons/bin), g[p] gain (0 = dead pixel).
 *
 * Functions whose result is pinned only by GPU-versus-oracle agreement (no
 * closed form, example or brute force fixes them) say "parity unpinned".
 */
#ifndef RT3D_ORACLE_H
#define RT3D_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_params {
    int    n_iter;      /* PALM iterations */
    int    k_max;       /* slot capacity per pixel */
    int    k_init;      /* peaks sought per pixel at initialisation */
    double p_xy;        /* world units per pixel */
    double dz;          /* world units per bin */
    double h_apss;      /* APSS kernel support (world units) */
    double h_int;       /* intensity-graph radius (world units) */
    double beta_t;      /* depth step scale (Fisher units) */
    double dmax;        /* depth step clip (bins); <= 0: max(0.5, 1/sqrt(Fisher)) */
    double beta_r;      /* intensity step scale */
    double beta_b;      /* background step scale */
    double r_min;       /* minimum admissible intensity (photons) */
    double d_merge;     /* in-pixel merge distance (bins); <= 0: max(1, sigma_h) */
    double sigma_b;     /* background Gaussian (pixels); 0 = identity */
    double b_min;       /* background floor */
    double sbr_guess;   /* log-matched-filter floor eps = 1/(sbr_guess*T) */
    int    r_init;      /* log-matched-filter aggregation radius (pixels) */
    int    n_min;       /* minimum photons in a peak window */
    double kappa;       /* peak acceptance: sigmas above background */
    int    w_nms;       /* non-maximum suppression half width; <= 0: auto */
    int    m_min;       /* minimum APSS neighbours */
    int    use_apss;    /* 1 = APSS depth denoiser, 0 = none */
    double persp;       /* 0: orthographic map f; > 0: pinhole camera, tangent of one pixel's angle,
                           depth = range along the pixel's ray (see rel() in the source) */
    int    ilp_box;     /* intensity low-pass divisor: 0 = 1 + same-surface neighbours found
                           (the mean over the point's surface), 1 = 1 + surrounding pixels inside
                           the image (a 3 x 3 box in which a missing neighbour counts as zero) */
} or_params;

typedef struct or_model or_model;

/* IRF model: normalised samples, Catmull-Rom interpolant, sigma_h^2, shift Fisher information. */
or_model* or_model_new(const double* irf, int L, int origin, int T);
void      or_model_free(or_model* m);
/* Per-pixel IRFs h_ij (Observation model): pixel p of every later call on m
 * uses models[cls[p]] (cls[p] >= n: models[0]); cls = NULL: m everywhere.
 * The super-resolved functions (or_sr_*) use m alone. */
void      or_model_set_classes(or_model* m, int n, or_model* const* models, const uint8_t* cls);
int       or_model_origin(const or_model* m);
double    or_model_sigma2(const or_model* m);
double    or_model_fisher(const or_model* m);
void      or_model_window(const or_model* m, int* wl, int* wr);
void      or_h(const or_model* m, int n, const double* tau, double* h, double* hp);
void      or_S(const or_model* m, int n, const double* tau, double* S, double* Sp);
void      or_lmf_table(const or_model* m, double sbr_guess, int64_t* q);

/* Histogram -> photon list (CSR, ascending bin, packed (t<<16)|z). */
int64_t or_compact(const uint16_t* Z, int64_t npix, int T, uint32_t* off, uint32_t* ent);

/* Negative log-likelihood of the Poisson observation model. */
double or_nll(const or_model* m, int64_t npix, const uint32_t* off, const uint32_t* ent,
              int k_max, const double* t, const double* r, const int* cnt,
              const double* b, const double* g);
/* Dense form of the same sum over every bin (cross-check, small T only). */
double or_nll_dense(const or_model* m, int64_t npix, const uint16_t* Z,
                    int k_max, const double* t, const double* r, const int* cnt,
                    const double* b, const double* g);
/* Partial derivatives and their sums of absolute terms. */
void or_grad(const or_model* m, int64_t npix, const uint32_t* off, const uint32_t* ent,
             int k_max, const double* t, const double* r, const int* cnt,
             const double* b, const double* g,
             double* gt, double* gr, double* gb,
             double* at, double* ar, double* ab);

/* Steps of one PALM iteration; all operate in place. */
void or_init(const or_model* m, const or_params* p, int F, int rows, int cols,
             const uint32_t* off, const uint32_t* ent, const double* g,
             double* t, double* r, double* n, int* cnt, double* b);
void or_init_normals(const or_params* p, int F, int rows, int cols,
                     const double* t, const int* cnt, double* n);
void or_depth_step(const or_model* m, const or_params* p, int64_t npix,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   double* t, const double* r, const int* cnt, const double* b);
void or_apss(const or_params* p, int F, int rows, int cols, int T,
             double* t, double* n, const int* cnt);
void or_apss_neighbours(const or_params* p, int F, int rows, int cols,
                        const double* t, const int* cnt, int64_t q,
                        int brute_force, int64_t* out, int cap);
void or_merge(const or_model* m, const or_params* p, int64_t npix,
              double* t, double* r, double* n, int* cnt);
void or_intensity_step(const or_model* m, const or_params* p, int64_t npix,
                       const uint32_t* off, const uint32_t* ent, const double* g,
                       const double* t, double* r, const int* cnt, const double* b);
void or_intensity_filter(const or_params* p, int F, int rows, int cols,
                         double* t, double* r, double* n, int* cnt);
void or_bg_step(const or_model* m, const or_params* p, int64_t npix,
                const uint32_t* off, const uint32_t* ent, const double* g,
                const double* t, const double* r, const int* cnt, double* b);
void or_bg_filter(const or_params* p, int F, int rows, int cols, double* b);
void or_iterate(const or_model* m, const or_params* p, int F, int rows, int cols,
                const uint32_t* off, const uint32_t* ent, const double* g,
                double* t, double* r, double* n, int* cnt, double* b);
void or_reconstruct(const or_model* m, const or_params* p, int F, int rows, int cols,
                    const uint32_t* off, const uint32_t* ent, const double* g,
                    double* t, double* r, double* n, int* cnt, double* b);

/* Super-resolution (Results, dynamic scenes): s x s point-grid pixels per
 * lidar pixel.  rows, cols are the lidar frame's; t, r, n, cnt (and gt, gr,
 * at, ar) are indexed by point-grid pixel of the (rows s) x (cols s) frames,
 * b and g (and gb, ab) by lidar pixel.  s = 1 is the plain model. */
double or_sr_nll(const or_model* m, int s, int F, int rows, int cols, const uint32_t* off,
                 const uint32_t* ent, int K, const double* t, const double* r, const int* cnt,
                 const double* b, const double* g);
void or_sr_grad(const or_model* m, int s, int F, int rows, int cols, const uint32_t* off,
                const uint32_t* ent, int K, const double* t, const double* r, const int* cnt,
                const double* b, const double* g, double* gt, double* gr, double* gb,
                double* at, double* ar, double* ab);
void or_sr_depth_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                      const uint32_t* off, const uint32_t* ent, const double* g,
                      double* t, const double* r, const int* cnt, const double* b);
void or_sr_intensity_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                          const uint32_t* off, const uint32_t* ent, const double* g,
                          const double* t, double* r, const int* cnt, const double* b);
void or_sr_bg_step(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   const double* t, const double* r, const int* cnt, double* b);
void or_sr_expand(int K, int s, int F, int rows, int cols, const double* tc, const double* rc,
                  const int* cntc, double* t, double* r, double* n, int* cnt);
/* parity unpinned as a whole (like or_iterate / or_reconstruct) */
void or_sr_iterate(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                   const uint32_t* off, const uint32_t* ent, const double* g,
                   double* t, double* r, double* n, int* cnt, double* b);
void or_sr_reconstruct(const or_model* m, const or_params* p, int s, int F, int rows, int cols,
                       const uint32_t* off, const uint32_t* ent, const double* g,
                       double* t, double* r, double* n, int* cnt, double* b);

#ifdef __cplusplus
}
#endif
#endif

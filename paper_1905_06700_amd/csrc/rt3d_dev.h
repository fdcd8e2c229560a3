// rt3d_dev.h -- device-side structures, helpers and kernel launchers shared by
// the HIP translation units of librt3d.so (internal; not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rt3d.h"

namespace rt3d {

constexpr int KM = RT3D_K_MAX;

// Observation model tables on the device (built on the host in FP64).
struct DevModel {
    const float4*  cr;    // Catmull-Rom segment k-1 (samples k..k+1): cubic coefficients (c0, c1, c2, c3)
    const int32_t* q;     // log-matched-filter weights, 16 fractional bits
    const int32_t* qst;   // range-maximum table of q: qst[l * L + k] = max q[k .. k + 2^l - 1]
    const double*  hbar;  // normalised IRF samples
    int   T, L, o;
    int   wl, wr;         // peak window half widths
    int   wnms;           // peak suppression half width
    float sigma2;         // IRF variance
    float fisher_inv;     // 1 / (shift Fisher information per photon)
    // S and S' of a point whose IRF support lies inside [0, T): all L + 1
    // segments take part, and their sum clamped at zero is a piecewise cubic
    // in the shared local parameter s.  s_tab holds the s_np + 1 breakpoints
    // (0 = b_0 < ... < b_np = 1), then per piece the coefficients c0..c3 of
    // c0 + c1 s + c2 s^2 + c3 s^3; s_v0 / s_d0 and s_v1 / s_d1 are the value
    // and slope at s = 0 and s = 1 (segments not positive there drop out).
    // s_np = 0: direct summation.
    int           s_np;
    const double* s_tab;
    double        s_v0, s_d0, s_v1, s_d1;
    // Per-pixel IRFs: cls[pix] is the pixel's class and a launch with this
    // model (class cls_id of n_cls) touches only the pixels of its class
    // (numbers >= n_cls count as 0); cls = nullptr: every pixel.
    const uint8_t* cls;
    int            cls_id, n_cls;
    // Optional per-class pixel lists (launch_class_lists): the per-pixel
    // steps then take lane group i to pixel lst[lst_meta[cls_id] + i] and
    // leave past lst_meta[cls_id + 1] - lst_meta[cls_id] pixels.
    const uint32_t* lst;
    const uint32_t* lst_meta;
};

// Whether pixel pix belongs to the launch's IRF class.
__device__ __forceinline__ bool in_class(const DevModel& m, long long pix)
{
    if (!m.cls) return true;
    const int k = m.cls[pix];
    return (k < m.n_cls ? k : 0) == m.cls_id;
}

// Parameters as the kernels use them.
struct DevParams {
    int    k_max, k_init, r_init, n_min, m_min, apss_R;
    int    apss_Rs;   // halo the orthographic APSS tile stages (rings beyond it are farther than h)
    int    lpp;       // lanes per pixel of the gradient steps: 4 or 8
    int    ilp_box;   // intensity low-pass divisor: 0 = 1 + neighbours found, 1 = 1 + surrounding pixels
    double p_xy, dz, h_apss, h_int;
    double beta_t, dmax, beta_r, beta_b, r_min, d_merge, b_min, kappa;
    double persp;   // 0: orthographic map f; > 0: pinhole camera (see ray_dir)
};

// Unit viewing ray of pixel (i, j) of a rows x cols frame under the pinhole
// camera: (persp (j - cx), persp (i - cy), 1) normalised, cx = (cols - 1)/2,
// cy = (rows - 1)/2; a point at depth t lies at t dz along it.
__device__ __forceinline__ void ray_dir(double persp, int rows, int cols, int i, int j, double (&v)[3])
{
    const double u = persp * (j - 0.5 * (cols - 1)), w = persp * (i - 0.5 * (rows - 1));
    // 1/sqrt(q): the FP32 estimate and one Newton step in FP64 (relative error
    // ~1e-14, without FP64 division and square root)
    const double q = u * u + w * w + 1.0;
    const double y0 = (double)__frsqrt_rn((float)q);
    const double inv = y0 * (1.5 - 0.5 * q * y0 * y0);
    v[0] = u * inv;
    v[1] = w * inv;
    v[2] = inv;
}

// Point state, slot-major structure of arrays (see rt3d_state).
struct DevState {
    double*  t;
    float*   r;
    float*   n;     // [3][KM][P]
    uint8_t* cnt;
    float*   b;
};

// F frames of rows x cols pixels, P = F * rows * cols.  S is the stride of the
// state's slot planes: P when the state holds these pixels alone, more when
// they are one group of a batch of unevenly sized frames (the state pointers
// then point at the group's first pixel).
struct Shape {
    int F, rows, cols;
    long long P;
    long long S;
};

// The state of a group of a batch: every array advanced to its first pixel.
__host__ __device__ inline DevState state_at(DevState s, long long base)
{
    s.t += base;
    s.r += base;
    s.n += base;
    s.cnt += base;
    s.b += base;
    return s;
}

// Groups of equally sized frames that one launch of a tiled kernel covers
// (the kernels that read neighbouring pixels work on 16 x 16 pixel tiles of
// one frame): group g holds F[g] frames of rows[g] x cols[g] pixels from pixel
// base[g] on, and owns tiles tile0[g] .. tile0[g + 1] - 1 of the grid.
constexpr int TILE = 16;
constexpr int TILE_GROUPS = 16;
struct Tiles {
    int n;
    long long S;                       // slot stride of the state
    long long base[TILE_GROUPS];
    int F[TILE_GROUPS], rows[TILE_GROUPS], cols[TILE_GROUPS];
    int tile0[TILE_GROUPS + 1];
};

// Group of a tile (wave-uniform: the tile is the workgroup's).
__device__ __forceinline__ int tile_group(const Tiles& tg, int tile)
{
    int g = 0;
    while (g + 1 < tg.n && tile >= tg.tile0[g + 1]) ++g;
    return g;
}

__host__ __device__ inline Shape group_shape(const Tiles& tg, int g)
{
    Shape sh;
    sh.F = tg.F[g];
    sh.rows = tg.rows[g];
    sh.cols = tg.cols[g];
    sh.P = (long long)sh.F * sh.rows * sh.cols;
    sh.S = tg.S;
    return sh;
}

// Appends group (base, sh) to tg; false when tg is full.
inline bool tiles_add(Tiles& tg, long long base, const Shape& sh)
{
    if (tg.n == 0) tg.tile0[0] = 0;
    if (tg.n >= TILE_GROUPS) return false;
    const int g = tg.n++;
    tg.base[g] = base;
    tg.F[g] = sh.F;
    tg.rows[g] = sh.rows;
    tg.cols[g] = sh.cols;
    tg.S = sh.S;
    const long long nt = (long long)sh.F * ((sh.rows + TILE - 1) / TILE) * ((sh.cols + TILE - 1) / TILE);
    tg.tile0[g + 1] = tg.tile0[g] + (int)nt;
    return true;
}

// One group: the whole shape from pixel 0.
inline Tiles tiles_of(const Shape& sh)
{
    Tiles tg{};
    tiles_add(tg, 0, sh);
    return tg;
}

// ---------------------------------------------------------------------------
// Model evaluation in FP32 local coordinates.

// Catmull-Rom segment value and slope at local parameter s, clamped at zero.
__device__ __forceinline__ void cr_segment(const float4 c, float s, float& h, float& hp)
{
    h = fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x);
    hp = fmaf(fmaf(3.f * c.w, s, 2.f * c.z), s, c.y);
    if (!(h > 0.f)) {
        h = 0.f;
        hp = 0.f;
    }
}

// h(tb - t) and dh/dtau for an integer bin tb and a point at depth t held as
// integer anchor a = floor(t) plus fraction f = t - a.  h is the Catmull-Rom
// interpolant of the IRF samples (continuous value and slope).
// The lag's sample position x = tb - a + o - f falls in segment
// idx = floor(x) + 1 at local parameter s = x - floor(x): with f > 0 that is
// idx = tb - a + o and s = 1 - f, with f = 0 idx = tb - a + o + 1 and s = 0.
// Only idx depends on the bin, so a loop over bins for one point keeps s and
// the offset; segments exist for -1 < x < L, i.e. idx in [1 - sh, L].
__device__ __forceinline__ void irf_eval_t(const float4* __restrict__ cr, int L, int o, int tb, int a, float f,
                                           float& h, float& hp)
{
    const int sh = f > 0.f ? 1 : 0;
    const float s = sh ? 1.f - f : 0.f;
    const int lo = 1 - sh;
    const int idx = tb - a + o + lo;
    h = 0.f;
    hp = 0.f;
    if ((unsigned)(idx - lo) <= (unsigned)(L - lo)) cr_segment(cr[idx], s, h, hp);
}

__device__ __forceinline__ void irf_eval(const DevModel& m, int tb, int a, float f, float& h, float& hp)
{
    irf_eval_t(m.cr, m.L, m.o, tb, a, f, h, hp);
}

// S(t) = sum over bins of h(tb - t) and dS/dt = -sum h'(tb - t) (every lag
// shares the local parameter s).  Inside the domain, for an IRF whose segments
// never dip below zero, the closed-form cubic of all segments; else by direct
// summation over the segments that fall inside [0, T).
// Lane `part` of `parts` sums the segments k0 + part, k0 + part + parts, ...
// (parts = 1: the whole sum).
// tab: the piecewise cubic's table (m.s_tab, or a copy of it in LDS).
__device__ __forceinline__ void s_eval_tab(const DevModel& m, const double* tab, double t, float& S, float& Sp,
                                           int part = 0, int parts = 1)
{
    const double fl = floor(t);
    const int a = (int)fl;
    const float f = (float)(t - fl);
    const int sh = f > 0.f ? 1 : 0;
    const float s = sh ? 1.f - f : 0.f;
    // segment k holds bin tb = k + a - o + sh; keep 0 <= tb <= T - 1
    const int k0 = max(-1, m.o - a - sh), k1 = min(m.L - 1, m.T - 1 + m.o - a - sh);
    if (m.s_np > 0 && k0 == -1 && k1 == m.L - 1) {   // every segment: the piecewise cubic (by part 0)
        S = 0.f;
        Sp = 0.f;
        if (part == 0) {
            if (s == 0.f) {
                S = (float)m.s_v0;
                Sp = (float)(-m.s_d0);
            } else if (s == 1.f) {
                S = (float)m.s_v1;
                Sp = (float)(-m.s_d1);
            } else {
                const double sd = (double)s;
                int i = 0;
                while (i + 1 < m.s_np && sd >= tab[i + 1]) ++i;
                const double* c = tab + (m.s_np + 1) + 4 * i;
                S = (float)(((c[3] * sd + c[2]) * sd + c[1]) * sd + c[0]);
                Sp = (float)(-((3.0 * c[3] * sd + 2.0 * c[2]) * sd + c[1]));
            }
        }
        return;
    }
    float acc = 0.f, accp = 0.f;
#pragma unroll 4
    for (int k = k0 + part; k <= k1; k += parts) {
        float h, hp;
        cr_segment(m.cr[k + 1], s, h, hp);
        acc += h;
        accp -= hp;
    }
    S = acc;
    Sp = accp;
}

__device__ __forceinline__ void s_eval(const DevModel& m, double t, float& S, float& Sp, int part = 0,
                                       int parts = 1)
{
    s_eval_tab(m, m.s_tab, t, S, Sp, part, parts);
}

__device__ __forceinline__ int ent_bin(uint32_t e) { return (int)(e >> 16); }

// Live slot count of a pixel, clamped to the slot capacity.
__device__ __forceinline__ int load_cnt(const uint8_t* cnt, long long pix)
{
    int c = cnt[pix];
    return c < KM ? c : KM;
}
__device__ __forceinline__ int ent_cnt(uint32_t e) { return (int)(e & 0xffffu); }

// In-pixel merge of c points (reading; the paper does not say how duplicate
// points of one pixel are treated): a stable insertion sort by depth, then,
// in depth order, a point closer than dm bins to the next merges with it into
// the intensity-weighted depth (the plain mean when both intensities are 0),
// the summed intensity and the intensity-weighted normal, normalised (the
// first point's normal when the weighted sum vanishes); the merged point is
// compared with the next.  c drops by one per merge.
__device__ __forceinline__ void merge_points(double (&t)[KM], float (&r)[KM], float (&nx)[KM], float (&ny)[KM],
                                             float (&nz)[KM], int& c, double dm)
{
    for (int a = 1; a < c; ++a)
        for (int b = a; b > 0 && t[b] < t[b - 1]; --b) {
            double x = t[b]; t[b] = t[b - 1]; t[b - 1] = x;
            float y = r[b]; r[b] = r[b - 1]; r[b - 1] = y;
            y = nx[b]; nx[b] = nx[b - 1]; nx[b - 1] = y;
            y = ny[b]; ny[b] = ny[b - 1]; ny[b - 1] = y;
            y = nz[b]; nz[b] = nz[b - 1]; nz[b - 1] = y;
        }
    int a = 0;
    while (a + 1 < c) {
        if (t[a + 1] - t[a] < dm) {
            const double ra = r[a], rb = r[a + 1];
            const double tt = (ra + rb > 0.0) ? (ra * t[a] + rb * t[a + 1]) / (ra + rb) : 0.5 * (t[a] + t[a + 1]);
            const float mx = r[a] * nx[a] + r[a + 1] * nx[a + 1];
            const float my = r[a] * ny[a] + r[a + 1] * ny[a + 1];
            const float mz = r[a] * nz[a] + r[a + 1] * nz[a + 1];
            const float nrm = sqrtf(mx * mx + my * my + mz * mz);
            if (nrm > 0.f) {
                nx[a] = mx / nrm;
                ny[a] = my / nrm;
                nz[a] = mz / nrm;
            }
            t[a] = tt;
            r[a] = (float)(ra + rb);
            for (int b = a + 1; b + 1 < c; ++b) {
                t[b] = t[b + 1]; r[b] = r[b + 1];
                nx[b] = nx[b + 1]; ny[b] = ny[b + 1]; nz[b] = nz[b + 1];
            }
            --c;
        } else {
            ++a;
        }
    }
}

// Sphere fit from the moments and projection of the query along its line of
// sight: updates depth t (bins) and normal n when the fit is usable.  ray:
// the unit line of sight under the pinhole camera (nullptr: +Z, the
// orthographic map); the normal faces the sensor (against the ray).
__device__ __forceinline__ void apss_project(bool ok, float W, float Px, float Py, float Pz, float Nx, float Ny,
                                             float Nz, float PN, float PP, float h, float h2, double dz, double tmax,
                                             double& t, float (&n)[3], const float* ray = nullptr)
{
    if (!ok) return;
    const float invW = 1.f / W;
    const float PdP = Px * Px + Py * Py + Pz * Pz;
    const float PdN = Px * Nx + Py * Ny + Pz * Nz;
    const float D = PP - PdP * invW;
    if (!(D > 1e-12f * W * h2)) return;
    const float u4 = 0.5f * (PN - PdN * invW) / D;
    const float ulx = (Nx - 2.f * u4 * Px) * invW;
    const float uly = (Ny - 2.f * u4 * Py) * invW;
    const float ulz = (Nz - 2.f * u4 * Pz) * invW;
    const float u0 = -(ulx * Px + uly * Py + ulz * Pz + u4 * PP) * invW;
    const float nul = sqrtf(ulx * ulx + uly * uly + ulz * ulz);
    const float bz = ray ? ulx * ray[0] + uly * ray[1] + ulz * ray[2] : ulz;   // ul along the line of sight
    if (!(fabsf(bz) > 1e-6f * nul)) return;
    const float disc = bz * bz - 4.f * u4 * u0;
    float sroot;
    if (disc < 0.f) sroot = -bz / (2.f * u4);
    else sroot = -2.f * u0 / (bz + copysignf(sqrtf(disc), bz));
    sroot = fminf(fmaxf(sroot, -h), h);
    double tn = t + (double)sroot / dz;
    t = tn < 0.0 ? 0.0 : (tn > tmax ? tmax : tn);
    float gx = ulx, gy = uly, gz = ulz + 2.f * u4 * sroot, gv = gz;
    if (ray) {
        gx = ulx + 2.f * u4 * sroot * ray[0];
        gy = uly + 2.f * u4 * sroot * ray[1];
        gz = ulz + 2.f * u4 * sroot * ray[2];
        gv = gx * ray[0] + gy * ray[1] + gz * ray[2];
    }
    const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
    if (ray && fabsf(gv) <= 1e-6f * gn) {
        // pinhole camera, gradient perpendicular to the line of sight (the
        // vertex of a missed sphere): the normal faces the sensor
        n[0] = -ray[0];
        n[1] = -ray[1];
        n[2] = -ray[2];
    } else if (gn > 0.f) {
        const float inv = (gv > 0.f ? -1.f : 1.f) / gn;
        n[0] = gx * inv;
        n[1] = gy * inv;
        n[2] = gz * inv;
    }
}

// Detector gain of pixel p (Results, "Observation model": g, 0 for a dead
// pixel); a gain that is not a finite non-negative number also counts as
// dead (rt3d_reconstruct reports it as E_INVALID).
__device__ __forceinline__ float gain_at(const float* __restrict__ gain, long long p)
{
    const float g = gain ? gain[p] : 1.f;
    return (g > 0.f && g <= 3.402823466e38f) ? g : 0.f;
}

struct PixPoints {
    int    c;
    int    a[KM];    // floor(t)
    float  f[KM];    // t - floor(t)
    float  r[KM];
    double t[KM];
};

// Anchor of a slot at or beyond the count: far below every bin, so that no
// IRF support reaches any entry.
constexpr int PT_ABSENT = -(1 << 28);

// Every slot is read whatever the count (the state holds KM slots per pixel),
// so that no load waits on another; slots at or beyond the count hold t = 0,
// r = 0 and the anchor PT_ABSENT.
__device__ __forceinline__ void load_points(const DevState& s, long long P, long long pix, PixPoints& q)
{
    double tv[KM];
    float rv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        tv[k] = s.t[k * P + pix];
        rv[k] = s.r[k * P + pix];
    }
    q.c = load_cnt(s.cnt, pix);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const bool on = k < q.c;
        const double t = on ? tv[k] : 0.0;
        const double fl = floor(t);
        q.t[k] = t;
        q.a[k] = on ? (int)fl : PT_ABSENT;
        q.f[k] = (float)(t - fl);
        q.r[k] = on ? rv[k] : 0.f;
    }
}

// The step updates of one point / pixel (readings of the step sizes):
// depth: t - (beta_t / I_h) (S' + sum z h'/lambda), clipped to dmax, clamped
// to [0, T-1]; intensity (for S > 0): r [(1 - beta_r) + beta_r sum z h /
// (lambda S)], at least 0; background: b [(1 - beta_b) + beta_b sum z /
// (lambda T)], at least b_min.
__device__ __forceinline__ double depth_next(const DevModel& m, const DevParams& p, double t, float Sp, float shp)
{
    const float scale = (float)p.beta_t * m.fisher_inv;
    const float dmax = (float)p.dmax;
    const double tmax = (double)(m.T - 1);
    float step = -scale * (Sp + shp);
    step = fminf(fmaxf(step, -dmax), dmax);
    const double tn = t + (double)step;
    return tn < 0.0 ? 0.0 : (tn > tmax ? tmax : tn);
}

__device__ __forceinline__ float intensity_next(const DevParams& p, float r, float S, float shh)
{
    const float br = (float)p.beta_r;
    return fmaxf(r * ((1.f - br) + br * shh / S), 0.f);
}

__device__ __forceinline__ float background_next(const DevModel& m, const DevParams& p, float bb, float sz)
{
    const float bt = (float)p.beta_b;
    return fmaxf(bb * ((1.f - bt) + bt * sz / (float)m.T), (float)p.b_min);
}

// Writes a pixel's c points to its KM slots (empty slots: zero depth and
// intensity, normal facing the sensor) and its count.
__device__ __forceinline__ void store_points(const DevState& s, long long P, long long pix, const double (&t)[KM],
                                             const float (&r)[KM], const float (&nx)[KM], const float (&ny)[KM],
                                             const float (&nz)[KM], int c)
{
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const bool live = k < c;
        s.t[k * P + pix] = live ? t[k] : 0.0;
        s.r[k * P + pix] = live ? r[k] : 0.f;
        s.n[(0 * KM + k) * P + pix] = live ? nx[k] : 0.f;
        s.n[(1 * KM + k) * P + pix] = live ? ny[k] : 0.f;
        s.n[(2 * KM + k) * P + pix] = live ? nz[k] : -1.f;
    }
    s.cnt[pix] = (uint8_t)c;
}


// Wave-level helpers (wave64).
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }


// Cross-lane moves inside small aligned lane groups on the VALU (DPP), with
// no LDS traffic.  Every lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over each aligned group of 4 lanes (every lane ends with its group's sum):
// quad permutations [1,0,3,2] and [2,3,0,1].
__device__ __forceinline__ float quad_sum(float v)
{
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    return v;
}

__device__ __forceinline__ uint32_t quad_sum_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    return v;
}

// Sum over each aligned group of 8 lanes: the quad sums, then the half-row
// mirror (lane i of 8 meets lane 7 - i, which holds the other quad's sum).
__device__ __forceinline__ float oct_sum(float v)
{
    v = quad_sum(v);
    v += dpp_move<0x141>(v);
    return v;
}

// Workgroups are dispatched to the chip's 8 XCDs (each with its own L2) in
// turn: block b runs on XCD b % 8.  For kernels that read neighbouring
// pixels, remap so that each XCD takes one contiguous range of the work and
// neighbouring pixels meet in the same L2.  A bijection of [0, nblocks).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks)
{
    const unsigned q = nblocks / 8, r = nblocks % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Value of another lane by a DPP move, or 0 where the move has no source lane
// or the lane's row is outside ROW_MASK.  Every lane must be active.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// Inclusive prefix sum over the 64 lanes on the VALU: shifts by 1, 2, 4 and 8
// lanes inside each row of 16, then row 0's total into row 1 and row 2's into
// row 3 (broadcast of lane 15), then lane 31's prefix into rows 2 and 3.
// Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += dpp_or_zero<0x111>(v);
    v += dpp_or_zero<0x112>(v);
    v += dpp_or_zero<0x114>(v);
    v += dpp_or_zero<0x118>(v);
    v += dpp_or_zero<0x142, 0xA>(v);
    v += dpp_or_zero<0x143, 0xC>(v);
    return v;
}

// Sums over the 64 lanes (every lane gets the total, read from lane 63 of
// the inclusive scan), on the VALU with no LDS traffic.  Every lane must be
// active.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ unsigned long long dpp_or_zero_u64(unsigned long long v)
{
    const uint32_t lo = dpp_or_zero<CTRL, ROW_MASK>((uint32_t)v), hi = dpp_or_zero<CTRL, ROW_MASK>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long readlane63_u64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// The same scan on 64-bit integers (exact) and on doubles (a DPP move with no
// source lane gives the bits of +0.0).
__device__ __forceinline__ long long wave_sum(long long v)
{
    unsigned long long u = (unsigned long long)v;
    u += dpp_or_zero_u64<0x111>(u);
    u += dpp_or_zero_u64<0x112>(u);
    u += dpp_or_zero_u64<0x114>(u);
    u += dpp_or_zero_u64<0x118>(u);
    u += dpp_or_zero_u64<0x142, 0xA>(u);
    u += dpp_or_zero_u64<0x143, 0xC>(u);
    return (long long)readlane63_u64(u);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_sum_u32(v); }
__device__ __forceinline__ int wave_sum(int v) { return (int)wave_sum_u32((uint32_t)v); }

__device__ __forceinline__ double wave_sum(double v)
{
    auto step = [](double x, unsigned long long bits) { return x + __longlong_as_double((long long)bits); };
    v = step(v, dpp_or_zero_u64<0x111>((unsigned long long)__double_as_longlong(v)));
    v = step(v, dpp_or_zero_u64<0x112>((unsigned long long)__double_as_longlong(v)));
    v = step(v, dpp_or_zero_u64<0x114>((unsigned long long)__double_as_longlong(v)));
    v = step(v, dpp_or_zero_u64<0x118>((unsigned long long)__double_as_longlong(v)));
    v = step(v, dpp_or_zero_u64<0x142, 0xA>((unsigned long long)__double_as_longlong(v)));
    v = step(v, dpp_or_zero_u64<0x143, 0xC>((unsigned long long)__double_as_longlong(v)));
    return __longlong_as_double((long long)readlane63_u64((unsigned long long)__double_as_longlong(v)));
}

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All enqueue on `st` and return the
// launch status.

hipError_t launch_scan(const uint32_t* in, uint32_t* out, long long n, uint32_t* partial,
                       uint64_t cap, int32_t* err, hipStream_t st);
size_t scan_partial_elems(long long n);

// Entries of a pixel the compaction stages per pixel (workspace: P x CP_STAGE);
// pixels with more read their histogram a second time.
constexpr int CP_STAGE = 128;

hipError_t launch_compact(const uint16_t* Z, long long P, int T, uint32_t* off, uint32_t* ent,
                          uint64_t cap, uint32_t* counts, uint32_t* partial, uint32_t* stage, int32_t* err,
                          hipStream_t st);

// The same lists with no device allocation and no workspace: counts and scan
// prefixes in the library's fixed per-GPU array (P <= noalloc_max_pixels(),
// noalloc_scratch_bytes() bytes), nothing staged; err: E_CAPACITY sink or null.
long long noalloc_max_pixels();
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(uint32_t** ptr);
hipError_t launch_compact_noalloc(const uint16_t* Z, long long P, int T, uint32_t* off, uint32_t* ent,
                                  uint64_t cap, int32_t* err, hipStream_t st);

hipError_t launch_compact_events(const uint32_t* pix, const uint16_t* bin, uint64_t n, long long P, int T,
                                 uint32_t* evoff, uint32_t* scratch, uint32_t* off, uint32_t* ent, uint64_t cap,
                                 uint32_t* counts, uint32_t* partial, int32_t* err, hipStream_t st);

// wide: P + 1 words of workspace (a count and a pixel list) for pools too
// large for the first kernel's registers, or null (they take the HBM path).
hipError_t launch_init(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                       const uint32_t* ent, const float* gain, DevState s, uint32_t* wide,
                       hipStream_t st);
hipError_t launch_init_normals(const DevParams& p, const Shape& sh, DevState s, hipStream_t st);

hipError_t launch_depth_step(const DevModel& m, const DevParams& p, const Shape& sh,
                             const uint32_t* off, const uint32_t* ent, const float* gain,
                             DevState s, hipStream_t st);
// merge: the in-pixel merge first, fused (the loop's order)
hipError_t launch_intensity_step(const DevModel& m, const DevParams& p, const Shape& sh,
                                 const uint32_t* off, const uint32_t* ent, const float* gain,
                                 DevState s, bool merge, hipStream_t st);
// bdst: where the new background goes (nullptr: the state's own b)
hipError_t launch_bg_step(const DevModel& m, const DevParams& p, const Shape& sh,
                          const uint32_t* off, const uint32_t* ent, const float* gain, DevState s,
                          float* bdst, hipStream_t st);
// Pixel lists of the n IRF classes of map cls over P pixels (list: P entries;
// meta: CLASS_META words, meta[k] .. meta[k+1] - 1 the list positions of class k).
constexpr int CLASS_META = 2 * (RT3D_MAX_IRFS + 1);
hipError_t launch_class_lists(const uint8_t* cls, long long P, int n, uint32_t* list, uint32_t* meta,
                              hipStream_t st);
hipError_t launch_gradients(const DevModel& m, const DevParams& p, const Shape& sh,
                            const uint32_t* off, const uint32_t* ent, const float* gain,
                            DevState s, float* gt, float* gr, float* gb, hipStream_t st);

// only_above >= 0: pixels with at most that many points are copied, not fitted;
// carry: `out` also receives the counts, backgrounds and intensities (else only
// the depths and normals of the live slots)
hipError_t launch_apss_tiles(const DevModel& m, const DevParams& p, const Tiles& tg, DevState in, DevState out,
                             int only_above, bool carry, hipStream_t st);
// The halo the orthographic APSS tile stages for support h_apss, pitch p_xy
// and window radius R = ceil(h_apss / p_xy).
int apss_staged_halo(double h_apss, double p_xy, int R);
// LDS bytes of the APSS tile kernel for window radius R (the perspective camera needs it to fit 64 KB)
size_t apss_lds_bytes(int R);
hipError_t launch_ifilter_tiles(const DevParams& p, const Tiles& tg, DevState in, DevState out, hipStream_t st);
// dst = the filtered src floored at b_min, per group (src, dst, tmp: the batch's arrays)
hipError_t launch_bfilter_tiles(const float* w, int rb, const Tiles& tg, float b_min, const float* src, float* dst,
                                float* tmp, hipStream_t st);
hipError_t launch_apss(const DevModel& m, const DevParams& p, const Shape& sh, DevState in,
                       DevState out, int only_above, hipStream_t st);
hipError_t launch_merge(const DevModel& m, const DevParams& p, const Shape& sh, DevState s, hipStream_t st);
hipError_t launch_ifilter(const DevParams& p, const Shape& sh, DevState in, DevState out,
                          hipStream_t st);
// dst = the filtered src floored at b_min (src and dst distinct; tmp: P floats
// for filters too wide for the tiled kernel)
hipError_t launch_bfilter(const float* w, int rb, const Shape& sh, float b_min, const float* src, float* dst,
                          float* tmp, hipStream_t st);
hipError_t launch_copy_state(const Shape& sh, DevState in, DevState out, hipStream_t st);

// Every iteration in one launch for frames of at most LOOP_MAX_PIX pixels:
// state A in and out, B the second buffer, bt a P-float background scratch,
// w the 2 rb + 1 background filter taps (rb <= 0: the floor only).
constexpr int LOOP_MAX_PIX = 4096;
hipError_t launch_loop(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                       const uint32_t* ent, const float* gain, DevState A, DevState B, float* bt, const float* w,
                       int rb, int n_iter, hipStream_t st);

// n_bg: background values written (sh.P, or the lidar pixels under super-resolution)
hipError_t launch_output(const Shape& sh, DevState s, rt3d_output* out, uint32_t* counts,
                         uint32_t* partial, int32_t* err, long long n_bg, hipStream_t st);
// E_INVALID into *err when a gain of gain[0 .. P-1] is not a finite
// non-negative number.
hipError_t launch_check_gain(const float* gain, long long P, int32_t* err, hipStream_t st);
// World Z of the packed points of the group of frames g whose first pixel is
// `base` (out->world_z non-null), after launch_output.
hipError_t launch_world_z(const Shape& g, long long base, DevState s, const rt3d_output* out, double dz,
                          double persp, hipStream_t st);

// Super-resolution: s x s point-grid pixels per lidar pixel.  lid: the lidar
// frames; the state's point arrays have slot stride Pf (point-grid pixels),
// its b[0 .. lid.P - 1] is the lidar background.  step: RT3D_STEP_DEPTH,
// _INTENSITY or _BKG (bdst: where the new background goes, nullptr: st.b).
constexpr int SR_MAX = 4;
hipError_t launch_sr_step(int step, const DevModel& m, const DevParams& p, const Shape& lid, int s, long long Pf,
                          const uint32_t* off, const uint32_t* ent, const float* gain, DevState st, float* bdst,
                          hipStream_t stream);
// gt, gr: [KM][Pf], gb: [lid.P]
hipError_t launch_sr_gradients(const DevModel& m, const DevParams& p, const Shape& lid, int s, long long Pf,
                               const uint32_t* off, const uint32_t* ent, const float* gain, DevState st, float* gt,
                               float* gr, float* gb, hipStream_t stream);
// lid (slot stride lid.P) spread over the point grid into out (stride Pf)
hipError_t launch_sr_expand(const Shape& lsh, int s, long long Pf, DevState lid, DevState out, hipStream_t stream);

}  // namespace rt3d

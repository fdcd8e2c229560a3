// k_steps.hip -- the likelihood gradient steps on depth, intensity and
// background (Results, "Reconstruction algorithm": each block update is a
// gradient step on the Poisson negative log-likelihood of the "Observation
// model"), and the raw gradients.
//
// For pixel p with active entries (t, z), points (t_n, r_n), background b and
// gain g, lambda_t = g (sum_n r_n h(t - t_n) + b) and
//   dNLL/dt_n = g r_n [S'(t_n) + sum z h'(t - t_n) / lambda_t]
//   dNLL/dr_n = g     [S(t_n)  - sum z h(t - t_n) / lambda_t]
//   dNLL/db   = g     [T       - sum z / lambda_t]
// Steps (readings of the unstated step sizes):
//   depth:      t_n -= (beta_t / I_h) [S' + sum z h'/lambda], clipped to dmax,
//               clamped to [0, T-1]; I_h is the shift Fisher information of
//               one photon, so g r I_h is the expected curvature (PALM-style
//               1/Lipschitz scaling, damped by beta_t);
//   intensity:  r_n <- max(0, r_n [(1-beta_r) + beta_r sum z h/(lambda S)]);
//   background: b <- max(b_min, b [(1-beta_b) + beta_b sum z/(lambda T)]).
// Within a pixel every point uses lambda from before the step (Jacobi).
//
// Mapping: one lane per pixel; the lane streams its pixel's active entries
// (cost linear in active bins, as in the paper's Methods) and keeps the
// pixel's <= 4 points in registers.  Depth is held in FP64 state and
// evaluated in FP32 around an integer anchor, so the IRF lookup error stays
// at FP32 rounding of the local offset whatever T is.
#include "rt3d_dev.h"

namespace rt3d {

struct PixPoints {
    int    c;
    int    a[KM];    // floor(t)
    float  f[KM];    // t - floor(t)
    float  r[KM];
    double t[KM];
};

__device__ __forceinline__ void load_points(const DevState& s, long long P, long long pix, PixPoints& q)
{
    q.c = load_cnt(s.cnt, pix);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        q.t[k] = 0.0;
        q.r[k] = 0.f;
        q.a[k] = 0;
        q.f[k] = 0.f;
        if (k < q.c) {
            double t = s.t[k * P + pix];
            double fl = floor(t);
            q.t[k] = t;
            q.a[k] = (int)fl;
            q.f[k] = (float)(t - fl);
            q.r[k] = s.r[k * P + pix];
        }
    }
}

// Accumulates over the pixel's entries: sz = sum z/lambda, sh[k] = sum z h_k/lambda,
// shp[k] = sum z h'_k/lambda (and the absolute-term sums when ABS).
template <bool ABS>
__device__ __forceinline__ void accumulate(const DevModel& m, const PixPoints& q, float bb, float G,
                                           const uint32_t* __restrict__ ent, uint32_t e0, uint32_t e1,
                                           float& sz, float (&sh)[KM], float (&shp)[KM], float (&ahp)[KM])
{
    sz = 0.f;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        sh[k] = 0.f;
        shp[k] = 0.f;
        ahp[k] = 0.f;
    }
    auto one = [&](uint32_t v) {
        const int tb = ent_bin(v);
        const float z = (float)ent_cnt(v);
        float h[KM], hp[KM];
        float lam = bb;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            h[k] = 0.f;
            hp[k] = 0.f;
            if (k < q.c) {
                irf_eval(m, tb, q.a[k], q.f[k], h[k], hp[k]);
                lam = fmaf(q.r[k], h[k], lam);
            }
        }
        const float zl = z * __builtin_amdgcn_rcpf(lam * G);
        sz += zl;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < q.c) {
                sh[k] = fmaf(zl, h[k], sh[k]);
                shp[k] = fmaf(zl, hp[k], shp[k]);
                if (ABS) ahp[k] = fmaf(zl, fabsf(hp[k]), ahp[k]);
            }
        }
    };
    // eight entries in flight per lane, then the tail
    uint32_t e = e0;
    for (; e + 8 <= e1; e += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ent[e + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) one(v[u]);
    }
    for (; e < e1; ++e) one(ent[e]);
}

__global__ __launch_bounds__(256) void k_depth_step(DevModel m, DevParams p, Shape sh,
                                                    const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ ent,
                                                    const float* __restrict__ gain, DevState s)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const float G = gain ? gain[pix] : 1.f;
    PixPoints q;
    load_points(s, P, pix, q);
    if (q.c == 0 || !(G > 0.f)) return;
    float sz, shh[KM], shp[KM], ahp[KM];
    accumulate<false>(m, q, s.b[pix], G, ent, off[pix], off[pix + 1], sz, shh, shp, ahp);
    const float scale = (float)p.beta_t * m.fisher_inv;
    const float dmax = (float)p.dmax;
    const double tmax = (double)(m.T - 1);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < q.c && q.r[k] > 0.f) {
            float S, Sp;
            s_eval(m, q.t[k], S, Sp);
            float step = -scale * (Sp + shp[k]);
            step = fminf(fmaxf(step, -dmax), dmax);
            double tn = q.t[k] + (double)step;
            tn = tn < 0.0 ? 0.0 : (tn > tmax ? tmax : tn);
            s.t[k * P + pix] = tn;
        }
    }
}

__global__ __launch_bounds__(256) void k_intensity_step(DevModel m, DevParams p, Shape sh,
                                                        const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ ent,
                                                        const float* __restrict__ gain, DevState s)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const float G = gain ? gain[pix] : 1.f;
    PixPoints q;
    load_points(s, P, pix, q);
    if (q.c == 0 || !(G > 0.f)) return;
    float sz, shh[KM], shp[KM], ahp[KM];
    accumulate<false>(m, q, s.b[pix], G, ent, off[pix], off[pix + 1], sz, shh, shp, ahp);
    const float br = (float)p.beta_r;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < q.c) {
            float S, Sp;
            s_eval(m, q.t[k], S, Sp);
            if (S > 0.f) {
                float v = q.r[k] * ((1.f - br) + br * shh[k] / S);
                s.r[k * P + pix] = fmaxf(v, 0.f);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_bg_step(DevModel m, DevParams p, Shape sh,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ ent,
                                                 const float* __restrict__ gain, DevState s)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const float G = gain ? gain[pix] : 1.f;
    if (!(G > 0.f)) return;
    PixPoints q;
    load_points(s, P, pix, q);
    float sz, shh[KM], shp[KM], ahp[KM];
    const float bb = s.b[pix];
    accumulate<false>(m, q, bb, G, ent, off[pix], off[pix + 1], sz, shh, shp, ahp);
    const float bt = (float)p.beta_b;
    const float v = bb * ((1.f - bt) + bt * sz / (float)m.T);
    s.b[pix] = fmaxf(v, (float)p.b_min);
}

__global__ __launch_bounds__(256) void k_gradients(DevModel m, Shape sh, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ ent,
                                                   const float* __restrict__ gain, DevState s,
                                                   float* __restrict__ gt, float* __restrict__ gr,
                                                   float* __restrict__ gb)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const float G = gain ? gain[pix] : 1.f;
    PixPoints q;
    load_points(s, P, pix, q);
    float sz = 0.f, shh[KM] = {0, 0, 0, 0}, shp[KM] = {0, 0, 0, 0}, ahp[KM];
    if (G > 0.f) accumulate<false>(m, q, s.b[pix], G, ent, off[pix], off[pix + 1], sz, shh, shp, ahp);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        float vt = 0.f, vr = 0.f;
        if (k < q.c && G > 0.f) {
            float S, Sp;
            s_eval(m, q.t[k], S, Sp);
            vt = G * q.r[k] * (Sp + shp[k]);
            vr = G * (S - shh[k]);
        }
        gt[k * P + pix] = vt;
        gr[k * P + pix] = vr;
    }
    gb[pix] = G > 0.f ? G * ((float)m.T - sz) : 0.f;
}

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_depth_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                             const uint32_t* ent, const float* gain, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_depth_step, dim3(blocks_for(sh.P, 256)), dim3(256), 0, st, m, p, sh, off, ent, gain, s);
    return hipGetLastError();
}

hipError_t launch_intensity_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                                 const uint32_t* ent, const float* gain, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_intensity_step, dim3(blocks_for(sh.P, 256)), dim3(256), 0, st, m, p, sh, off, ent, gain,
                       s);
    return hipGetLastError();
}

hipError_t launch_bg_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                          const uint32_t* ent, const float* gain, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bg_step, dim3(blocks_for(sh.P, 256)), dim3(256), 0, st, m, p, sh, off, ent, gain, s);
    return hipGetLastError();
}

hipError_t launch_gradients(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                            const uint32_t* ent, const float* gain, DevState s, float* gt, float* gr, float* gb,
                            hipStream_t st)
{
    (void)p;
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gradients, dim3(blocks_for(sh.P, 256)), dim3(256), 0, st, m, sh, off, ent, gain, s, gt,
                       gr, gb);
    return hipGetLastError();
}

}  // namespace rt3d

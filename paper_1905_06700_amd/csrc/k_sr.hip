// k_sr.hip -- the super-resolved data term (Results, dynamic scenes, and
// Discussion: the map f may undersample).  The point cloud lives on a grid s
// times finer than the lidar pixels; the s x s point-grid pixels
// (i s + u, j s + v) all map to lidar pixel (i, j), whose Poisson intensity
// adds their points:
//   lambda_{p,t} = g_p (sum_{q -> p} sum_{n in q} r_n h(t - t_n) + b_p).
// Gain and background stay per lidar pixel.  Each point's gradient is that of
// the plain model with its lidar pixel's lambda:
//   dNLL/dt_n = g r_n [S'(t_n) + sum z h'(t - t_n)/lambda]
//   dNLL/dr_n = g     [S(t_n)  - sum z h(t - t_n)/lambda]
//   dNLL/db_p = g     [T       - sum z/lambda]
// and the steps are those of k_steps.hip (depth_next, intensity_next,
// background_next), Jacobi over the whole block.
//
// State: point arrays (t, r, n, cnt) on the point grid with slot stride Pf;
// the lidar pixels' background in b[0 .. P - 1] of the same state.
//
// Mapping: sixteen lanes per lidar pixel, four lidar pixels per wavefront.
// Lane u holds the points of the block's point-grid pixel u in registers
// (s <= 4, so s^2 <= 16 lanes); the block's points are also staged in LDS.
// The pixel's entries go through 16 at a time, one per lane: a lane
// evaluates lambda of its entry over the staged points and leaves
// z/(g lambda) and the bin in LDS; then every lane adds the batch's
// z h'/lambda and z h/lambda to each of its points.  The background's
// sum z/lambda is a sum over the sixteen lanes.
#include "rt3d_dev.h"

namespace rt3d {

// Lanes per lidar pixel (one per point-grid pixel of its block, s <= 4) and
// lidar pixels per workgroup.
constexpr int SR_GROUP = 16;
constexpr int SR_GROUPS = 16;

// What a launch of k_sr_step computes.
enum SrWork { SR_DEPTH, SR_INTENSITY, SR_BKG, SR_GRADIENTS };

// Orders a wavefront's LDS writes before its reads (and reads before the next writes).
__device__ __forceinline__ void sr_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Point-grid pixel of sub-position u (row-major in the s x s block) of lidar
// pixel p, for frames of rows x cols lidar pixels.
__device__ __forceinline__ long long sr_fine(long long p, int u, int s, int rows, int cols)
{
    const long long npf = (long long)rows * cols;
    const long long f = p / npf;
    const long long rem = p - f * npf;
    const long long i = rem / cols, j = rem - i * cols;
    const long long fi = i * s + u / s, fj = j * s + u % s;
    return (f * rows * s + fi) * ((long long)cols * s) + fj;
}

template <SrWork WHICH>
__global__ __launch_bounds__(SR_GROUP * SR_GROUPS) void k_sr_step(DevModel m, DevParams p, Shape lid, int s,
                                                                 long long Pf, const uint32_t* __restrict__ off,
                                                                 const uint32_t* __restrict__ ent,
                                                                 const float* __restrict__ gain, DevState st,
                                                                 float* __restrict__ bdst, float* __restrict__ gt,
                                                                 float* __restrict__ gr, float* __restrict__ gb)
{
    __shared__ int s_a[SR_GROUPS][SR_GROUP * KM];
    __shared__ float s_f[SR_GROUPS][SR_GROUP * KM];
    __shared__ float s_r[SR_GROUPS][SR_GROUP * KM];
    __shared__ float s_w[SR_GROUPS][SR_GROUP];
    __shared__ int s_tb[SR_GROUPS][SR_GROUP];
    const int g = (int)(threadIdx.x / SR_GROUP), u = (int)(threadIdx.x % SR_GROUP);
    const long long pix = (long long)blockIdx.x * SR_GROUPS + g;
    const bool valid = pix < lid.P;                 // the whole group
    const long long pq = valid ? pix : 0;
    // lane u: point-grid pixel u of the block, its points in registers
    const bool in_block = valid && u < s * s;
    const long long q = in_block ? sr_fine(pq, u, s, lid.rows, lid.cols) : 0;
    PixPoints pts;
    load_points(st, Pf, q, pts);
    if (!in_block) pts.c = 0;
    const float G = valid ? gain_at(gain, pq) : 0.f;
    const float bb = st.b[pq];
    const bool live = G > 0.f;                      // group-uniform
    // the block's points staged in LDS, lane after lane (prefix of the counts in the group)
    int before = 0, np = 0;
    for (int v = 0; v < SR_GROUP; ++v) {
        const int cv = __shfl(pts.c, (int)(threadIdx.x & ~(SR_GROUP - 1)) + v, 64);
        before += v < u ? cv : 0;
        np += cv;
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < pts.c) {
            s_a[g][before + k] = pts.a[k];
            s_f[g][before + k] = pts.f[k];
            s_r[g][before + k] = pts.r[k];
        }
    sr_sync();
    float sh[KM], shp[KM], sz = 0.f;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        sh[k] = 0.f;
        shp[k] = 0.f;
    }
    const uint32_t e0 = live ? off[pq] : 0u, e1 = live ? off[pq + 1] : 0u;
    const float invG = live ? 1.f / G : 0.f;
    for (uint32_t eb = e0; eb < e1; eb += SR_GROUP) {   // the same trip count on the group's lanes
        const uint32_t x = eb + (uint32_t)u;
        const bool on = x < e1;
        const uint32_t v = on ? ent[x] : 0u;
        const int tb = ent_bin(v);
        float lam = bb;
        for (int n = 0; n < np; ++n) {
            float h, hp;
            irf_eval(m, tb, s_a[g][n], s_f[g][n], h, hp);
            lam = fmaf(s_r[g][n], h, lam);
        }
        const float w = on ? (float)ent_cnt(v) * invG * __builtin_amdgcn_rcpf(lam) : 0.f;
        sz += w;
        if (WHICH != SR_BKG) {
            s_w[g][u] = w;
            s_tb[g][u] = tb;
            sr_sync();
            const int nb = (int)min((uint32_t)SR_GROUP, e1 - eb);
            for (int y = 0; y < nb; ++y) {
                const float wy = s_w[g][y];
                const int ty = s_tb[g][y];
#pragma unroll
                for (int k = 0; k < KM; ++k)
                    if (k < pts.c) {
                        float h, hp;
                        irf_eval(m, ty, pts.a[k], pts.f[k], h, hp);
                        sh[k] = fmaf(wy, h, sh[k]);
                        shp[k] = fmaf(wy, hp, shp[k]);
                    }
            }
            sr_sync();                              // reads done before the next batch's writes
        }
    }
    if (WHICH == SR_BKG || WHICH == SR_GRADIENTS) {
#pragma unroll
        for (int d = SR_GROUP / 2; d >= 1; d >>= 1) sz += __shfl_xor(sz, d, 64);
    }
    if (WHICH == SR_DEPTH) {
        if (live)
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (k < pts.c && pts.r[k] > 0.f) {
                    float S, Sp;
                    s_eval(m, pts.t[k], S, Sp);
                    st.t[(long long)k * Pf + q] = depth_next(m, p, pts.t[k], Sp, shp[k]);
                }
    } else if (WHICH == SR_INTENSITY) {
        if (live)
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (k < pts.c) {
                    float S, Sp;
                    s_eval(m, pts.t[k], S, Sp);
                    if (S > 0.f) st.r[(long long)k * Pf + q] = intensity_next(p, pts.r[k], S, sh[k]);
                }
    } else if (WHICH == SR_BKG) {
        if (valid && u == 0) bdst[pix] = live ? background_next(m, p, bb, sz) : bb;
    } else {   // raw gradients: every slot of the block's point-grid pixels, and gb
        if (in_block)
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                float vt = 0.f, vr = 0.f;
                if (live && k < pts.c) {
                    float S, Sp;
                    s_eval(m, pts.t[k], S, Sp);
                    vt = G * pts.r[k] * (Sp + shp[k]);
                    vr = G * (S - sh[k]);
                }
                gt[(long long)k * Pf + q] = vt;
                gr[(long long)k * Pf + q] = vr;
            }
        if (valid && u == 0) gb[pix] = live ? G * ((float)m.T - sz) : 0.f;
    }
}

// The lidar-grid initialisation (lid: stride lid.P) spread over the point
// grid (out: stride Pf): every point-grid pixel takes its lidar pixel's
// points with 1/s^2 of the intensity (lambda unchanged), normals facing the
// sensor until they are fitted; the lidar background goes to out.b[0 .. P-1].
__global__ __launch_bounds__(256) void k_sr_expand(Shape lsh, int s, long long Pf, DevState lid, DevState out)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Pf) return;
    const long long R = (long long)lsh.rows * s, C = (long long)lsh.cols * s;
    const long long f = q / (R * C);
    const long long rem = q - f * R * C;
    const long long fi = rem / C, fj = rem - fi * C;
    const long long P = lsh.P;
    const long long pix = (f * lsh.rows + fi / s) * lsh.cols + fj / s;
    const int c = load_cnt(lid.cnt, pix);
    const float share = 1.f / (float)(s * s);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const bool on = k < c;
        out.t[(long long)k * Pf + q] = on ? lid.t[(long long)k * P + pix] : 0.0;
        out.r[(long long)k * Pf + q] = on ? lid.r[(long long)k * P + pix] * share : 0.f;
        out.n[(long long)(0 * KM + k) * Pf + q] = 0.f;
        out.n[(long long)(1 * KM + k) * Pf + q] = 0.f;
        out.n[(long long)(2 * KM + k) * Pf + q] = -1.f;
    }
    out.cnt[q] = (uint8_t)c;
    if (q < P) out.b[q] = lid.b[q];
}

template <SrWork WHICH>
static hipError_t sr_launch(const DevModel& m, const DevParams& p, const Shape& lid, int s, long long Pf,
                            const uint32_t* off, const uint32_t* ent, const float* gain, DevState st, float* bdst,
                            float* gt, float* gr, float* gb, hipStream_t stream)
{
    if (lid.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sr_step<WHICH>, dim3((unsigned)((lid.P + SR_GROUPS - 1) / SR_GROUPS)),
                       dim3(SR_GROUP * SR_GROUPS), 0, stream, m, p, lid, s, Pf, off, ent, gain, st, bdst, gt, gr, gb);
    return hipGetLastError();
}

hipError_t launch_sr_step(int step, const DevModel& m, const DevParams& p, const Shape& lid, int s, long long Pf,
                          const uint32_t* off, const uint32_t* ent, const float* gain, DevState st, float* bdst,
                          hipStream_t stream)
{
    switch (step) {
    case RT3D_STEP_DEPTH:
        return sr_launch<SR_DEPTH>(m, p, lid, s, Pf, off, ent, gain, st, nullptr, nullptr, nullptr, nullptr, stream);
    case RT3D_STEP_INTENSITY:
        return sr_launch<SR_INTENSITY>(m, p, lid, s, Pf, off, ent, gain, st, nullptr, nullptr, nullptr, nullptr,
                                       stream);
    case RT3D_STEP_BKG:
        return sr_launch<SR_BKG>(m, p, lid, s, Pf, off, ent, gain, st, bdst ? bdst : st.b, nullptr, nullptr, nullptr,
                                 stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_sr_gradients(const DevModel& m, const DevParams& p, const Shape& lid, int s, long long Pf,
                               const uint32_t* off, const uint32_t* ent, const float* gain, DevState st, float* gt,
                               float* gr, float* gb, hipStream_t stream)
{
    return sr_launch<SR_GRADIENTS>(m, p, lid, s, Pf, off, ent, gain, st, nullptr, gt, gr, gb, stream);
}

hipError_t launch_sr_expand(const Shape& lsh, int s, long long Pf, DevState lid, DevState out, hipStream_t stream)
{
    if (Pf == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sr_expand, dim3((unsigned)((Pf + 255) / 256)), dim3(256), 0, stream, lsh, s, Pf, lid, out);
    return hipGetLastError();
}

}  // namespace rt3d

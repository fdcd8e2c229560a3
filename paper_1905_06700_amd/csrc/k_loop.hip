// k_loop.hip -- every iteration of the reconstruction loop (Results,
// "Reconstruction algorithm": depth step and APSS, in-pixel merge, intensity
// step and its low-pass and threshold, background step and its filter) in one
// launch, for batches of small frames.
//
// Mapping: one workgroup per frame (up to LOOP_MAX_PIX pixels) keeps running
// for all iterations; each step is a loop of the workgroup's threads over the
// frame's pixels (one pixel per thread at a time) and the steps are separated
// by workgroup barriers instead of kernel boundaries, so a call on a batch of
// small frames is one launch instead of seven per iteration.  The frame's point
// state, entries and background stay in the caches between steps.  Each step
// computes what the corresponding kernel of k_steps.hip, k_apss.hip and
// k_filter.hip computes (the same readings, the same update functions); sums
// over a pixel's entries run on one thread here, so their FP32 rounding order
// differs from the four-lane kernels.
#include "rt3d_dev.h"

namespace rt3d {

constexpr int LOOP_THREADS = 1024;

// Sums over one pixel's entries e0 .. e1 - 1, on one thread: sz = sum z/lambda,
// sh[k] = sum z h_k/lambda, shp[k] = sum z h'_k/lambda (entries outside the
// points' support have lambda = g b).
__device__ __forceinline__ void accumulate_1(const DevModel& m, const PixPoints& q, float bb, float G,
                                             const uint32_t* __restrict__ ent, uint32_t e0, uint32_t e1, float& sz,
                                             float (&sh)[KM], float (&shp)[KM])
{
    sz = 0.f;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        sh[k] = 0.f;
        shp[k] = 0.f;
    }
    const float invG = 1.f / G;
    int lo = 0x7fffffff, hi = -0x7fffffff;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < q.c) {
            lo = min(lo, q.a[k] - m.o - 1);
            hi = max(hi, q.a[k] - m.o + m.L);
        }
    int zout = 0;
    for (uint32_t x = e0; x < e1; ++x) {
        const uint32_t v = ent[x];
        const int tb = ent_bin(v);
        if (tb < lo || tb > hi) {
            zout += ent_cnt(v);
            continue;
        }
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
        const float zl = z * invG * __builtin_amdgcn_rcpf(lam);
        sz += zl;
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < q.c) {
                sh[k] = fmaf(zl, h[k], sh[k]);
                shp[k] = fmaf(zl, hp[k], shp[k]);
            }
    }
    sz += (float)zout * invG * __builtin_amdgcn_rcpf(bb);
}

// Depth step of pixel pix (state s, slot stride S).
__device__ __forceinline__ void depth_1(const DevModel& m, const DevParams& p, long long S, const uint32_t* off,
                                        const uint32_t* ent, const float* gain, const DevState& s, long long pix)
{
    PixPoints q;
    load_points(s, S, pix, q);
    const float G = gain_at(gain, pix);
    if (q.c == 0 || !(G > 0.f)) return;
    float sz, shh[KM], shp[KM];
    accumulate_1(m, q, s.b[pix], G, ent, off[pix], off[pix + 1], sz, shh, shp);
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < q.c && q.r[k] > 0.f) {
            float Sv, Spv;
            s_eval(m, q.t[k], Sv, Spv);
            s.t[k * S + pix] = depth_next(m, p, q.t[k], Spv, shp[k]);
        }
}

// In-pixel merge, then the intensity step, of pixel pix.
__device__ __forceinline__ void intensity_1(const DevModel& m, const DevParams& p, long long S, const uint32_t* off,
                                            const uint32_t* ent, const float* gain, const DevState& s,
                                            long long pix)
{
    PixPoints q;
    load_points(s, S, pix, q);
    bool need = false;
#pragma unroll
    for (int k = 1; k < KM; ++k)
        if (k < q.c && (q.t[k] < q.t[k - 1] || q.t[k] - q.t[k - 1] < p.d_merge)) need = true;
    if (need) {
        double t[KM];
        float r[KM], nx[KM], ny[KM], nz[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            t[k] = q.t[k];
            r[k] = q.r[k];
            nx[k] = s.n[(0 * KM + k) * S + pix];
            ny[k] = s.n[(1 * KM + k) * S + pix];
            nz[k] = s.n[(2 * KM + k) * S + pix];
        }
        int c = q.c;
        merge_points(t, r, nx, ny, nz, c, p.d_merge);
        store_points(s, S, pix, t, r, nx, ny, nz, c);
        load_points(s, S, pix, q);
    }
    const float G = gain_at(gain, pix);
    if (q.c == 0 || !(G > 0.f)) return;
    float sz, shh[KM], shp[KM];
    accumulate_1(m, q, s.b[pix], G, ent, off[pix], off[pix + 1], sz, shh, shp);
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < q.c) {
            float Sv, Spv;
            s_eval(m, q.t[k], Sv, Spv);
            if (Sv > 0.f) s.r[k * S + pix] = intensity_next(p, q.r[k], Sv, shh[k]);
        }
}

// Background step of pixel pix into bdst (dead pixels keep their b).
__device__ __forceinline__ void background_1(const DevModel& m, const DevParams& p, long long S, const uint32_t* off,
                                             const uint32_t* ent, const float* gain, const DevState& s, float* bdst,
                                             long long pix)
{
    PixPoints q;
    load_points(s, S, pix, q);
    const float G = gain_at(gain, pix);
    const float bb = s.b[pix];
    if (!(G > 0.f)) {
        bdst[pix] = bb;
        return;
    }
    float sz, shh[KM], shp[KM];
    accumulate_1(m, q, bb, G, ent, off[pix], off[pix + 1], sz, shh, shp);
    bdst[pix] = background_next(m, p, bb, sz);
}

// APSS of the points of pixel (i, j) of the frame starting at pixel fb: reads
// `in`, writes `out` (the neighbour loop is the one of k_apss_tile).
__device__ __forceinline__ void apss_1(const DevModel& m, const DevParams& p, const Shape& sh, const DevState& in,
                                       const DevState& out, long long fb, int i, int j)
{
    const long long S = sh.S;
    const long long pix = fb + (long long)i * sh.cols + j;
    const int c = load_cnt(in.cnt, pix);
    out.cnt[pix] = (uint8_t)c;
    out.b[pix] = in.b[pix];
#pragma unroll
    for (int k = 0; k < KM; ++k) out.r[k * S + pix] = in.r[k * S + pix];
    const int R = p.apss_R;
    const float h = (float)p.h_apss, h2 = h * h, inv_h2 = 1.f / h2;
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const double tmax = (double)(m.T - 1);
    for (int k = 0; k < c; ++k) {
        const double tq = in.t[k * S + pix];
        float W = 0.f, Px = 0.f, Py = 0.f, Pz = 0.f, Nx = 0.f, Ny = 0.f, Nz = 0.f, PN = 0.f, PP = 0.f, nn = 0.f;
        for (int di = -R; di <= R; ++di) {
            const float yy = (float)di * pxy;
            for (int dj = -R; dj <= R; ++dj) {
                const float yx = (float)dj * pxy;
                const float dl = fmaf(yx, yx, yy * yy);
                if (!(dl < h2)) continue;
                const int i2 = i + di, j2 = j + dj;
                if (i2 < 0 || i2 >= sh.rows || j2 < 0 || j2 >= sh.cols) continue;
                const long long pp = fb + (long long)i2 * sh.cols + j2;
                const int cc = load_cnt(in.cnt, pp);
                for (int k2 = 0; k2 < cc; ++k2) {
                    const float yz = (float)((in.t[k2 * S + pp] - tq) * dz);
                    const float d2 = fmaf(yz, yz, dl);
                    if (!(d2 < h2)) continue;
                    float a = 1.f - d2 * inv_h2;
                    a = a * a;
                    const float w = a * a;
                    const float nx = in.n[(0 * KM + k2) * S + pp];
                    const float ny = in.n[(1 * KM + k2) * S + pp];
                    const float nz = in.n[(2 * KM + k2) * S + pp];
                    W += w;
                    Px = fmaf(w, yx, Px);
                    Py = fmaf(w, yy, Py);
                    Pz = fmaf(w, yz, Pz);
                    Nx = fmaf(w, nx, Nx);
                    Ny = fmaf(w, ny, Ny);
                    Nz = fmaf(w, nz, Nz);
                    PN = fmaf(w, yx * nx + yy * ny + yz * nz, PN);
                    PP = fmaf(w, d2, PP);
                    nn += 1.f;
                }
            }
        }
        double tn = tq;
        float on[3] = {in.n[(0 * KM + k) * S + pix], in.n[(1 * KM + k) * S + pix], in.n[(2 * KM + k) * S + pix]};
        apss_project(nn >= (float)p.m_min, W, Px, Py, Pz, Nx, Ny, Nz, PN, PP, h, h2, dz, tmax, tn, on);
        out.t[k * S + pix] = tn;
#pragma unroll
        for (int a = 0; a < 3; ++a) out.n[(a * KM + k) * S + pix] = on[a];
    }
}

// Intensity low-pass and threshold of pixel (i, j): reads `in`, writes `out`
// (the neighbour loop is the one of k_ifilter_tile).
__device__ __forceinline__ void ifilter_1(const DevParams& p, const Shape& sh, const DevState& in,
                                          const DevState& out, long long fb, int i, int j)
{
    const long long S = sh.S;
    const long long pix = fb + (long long)i * sh.cols + j;
    const int c = load_cnt(in.cnt, pix);
    const float hi2 = (float)(p.h_int * p.h_int);
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const float rmin = (float)p.r_min;
    int nside = 0;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
            if (!(di == 0 && dj == 0) && i + di >= 0 && i + di < sh.rows && j + dj >= 0 && j + dj < sh.cols) ++nside;
    int nk = 0;
    for (int k = 0; k < c; ++k) {
        const double tq = in.t[k * S + pix];
        float sum = in.r[k * S + pix];
        int deg = 0;
        for (int di = -1; di <= 1; ++di) {
            const float dy = (float)di * pxy;
            for (int dj = -1; dj <= 1; ++dj) {
                if (di == 0 && dj == 0) continue;
                const float dx = (float)dj * pxy;
                const int i2 = i + di, j2 = j + dj;
                if (i2 < 0 || i2 >= sh.rows || j2 < 0 || j2 >= sh.cols) continue;
                const long long pp = fb + (long long)i2 * sh.cols + j2;
                const int cc = load_cnt(in.cnt, pp);
                int best = -1;
                float bd = 0.f;
                for (int k2 = 0; k2 < cc; ++k2) {
                    const float ddz = (float)((in.t[k2 * S + pp] - tq) * dz);
                    const float d2 = dx * dx + dy * dy + ddz * ddz;
                    if (best < 0 || d2 < bd) {
                        best = k2;
                        bd = d2;
                    }
                }
                if (best >= 0 && bd < hi2) {
                    sum += in.r[best * S + pp];
                    ++deg;
                }
            }
        }
        const float rn = sum / (float)(1 + (p.ilp_box ? nside : deg));
        if (rn < rmin) continue;
        out.t[nk * S + pix] = tq;
        out.r[nk * S + pix] = rn;
#pragma unroll
        for (int a = 0; a < 3; ++a) out.n[(a * KM + nk) * S + pix] = in.n[(a * KM + k) * S + pix];
        ++nk;
    }
    for (int k = nk; k < KM; ++k) {
        out.t[k * S + pix] = 0.0;
        out.r[k * S + pix] = 0.f;
        out.n[(0 * KM + k) * S + pix] = 0.f;
        out.n[(1 * KM + k) * S + pix] = 0.f;
        out.n[(2 * KM + k) * S + pix] = -1.f;
    }
    out.cnt[pix] = (uint8_t)nk;
    out.b[pix] = in.b[pix];
}

__device__ __forceinline__ int wrap_n(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// n_iter iterations on frames of sh (one workgroup per frame, at most
// LOOP_MAX_PIX pixels each): state A in and out, B the second buffer, bt the
// background scratch (P floats), w the 2 rb + 1 filter taps.
__global__ __launch_bounds__(LOOP_THREADS) void k_loop(DevModel m, DevParams p, Shape sh,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ ent,
                                                       const float* __restrict__ gain, DevState A, DevState B,
                                                       float* __restrict__ bt, const float* __restrict__ w, int rb,
                                                       int n_iter)
{
    __shared__ float rowpass[LOOP_MAX_PIX];
    const int N = sh.rows * sh.cols;
    const long long fb = (long long)blockIdx.x * N;
    const long long S = sh.S;
    const float b_min = (float)p.b_min;
    for (int it = 0; it < n_iter; ++it) {
        for (int x = threadIdx.x; x < N; x += blockDim.x) depth_1(m, p, S, off, ent, gain, A, fb + x);
        __syncthreads();
        for (int x = threadIdx.x; x < N; x += blockDim.x) apss_1(m, p, sh, A, B, fb, x / sh.cols, x % sh.cols);
        __syncthreads();
        for (int x = threadIdx.x; x < N; x += blockDim.x) intensity_1(m, p, S, off, ent, gain, B, fb + x);
        __syncthreads();
        for (int x = threadIdx.x; x < N; x += blockDim.x) ifilter_1(p, sh, B, A, fb, x / sh.cols, x % sh.cols);
        __syncthreads();
        for (int x = threadIdx.x; x < N; x += blockDim.x) background_1(m, p, S, off, ent, gain, A, bt, fb + x);
        __syncthreads();
        if (rb > 0) {
            // circular row pass into LDS, then the column pass with the floor
            // (taps in the order of k_bfilter_rows / k_bfilter_cols)
            for (int x = threadIdx.x; x < N; x += blockDim.x) {
                const int i = x / sh.cols, j = x % sh.cols;
                const float* row = bt + fb + (long long)i * sh.cols;
                float a = 0.f;
                for (int d = -rb; d <= rb; ++d) a = fmaf(w[d + rb], row[wrap_n(j + d, sh.cols)], a);
                rowpass[x] = a;
            }
            __syncthreads();
            for (int x = threadIdx.x; x < N; x += blockDim.x) {
                const int i = x / sh.cols, j = x % sh.cols;
                float a = 0.f;
                for (int d = -rb; d <= rb; ++d) a = fmaf(w[d + rb], rowpass[wrap_n(i + d, sh.rows) * sh.cols + j], a);
                A.b[fb + x] = fmaxf(a, b_min);
            }
        } else {
            for (int x = threadIdx.x; x < N; x += blockDim.x) A.b[fb + x] = fmaxf(bt[fb + x], b_min);
        }
        __syncthreads();
    }
}

hipError_t launch_loop(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                       const uint32_t* ent, const float* gain, DevState A, DevState B, float* bt, const float* w,
                       int rb, int n_iter, hipStream_t st)
{
    if (sh.P == 0 || n_iter <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_loop, dim3((unsigned)sh.F), dim3(LOOP_THREADS), 0, st, m, p, sh, off, ent, gain, A, B, bt, w,
                       rb, n_iter);
    return hipGetLastError();
}

}  // namespace rt3d

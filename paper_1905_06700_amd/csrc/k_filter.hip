// k_filter.hip -- the intensity denoiser and threshold, the background image
// filter, state copies and output packing.
//
// Intensity (Results, "Reconstruction algorithm", intensity update: a
// low-pass over nearest neighbours on the manifold the points define, then
// removal of points below the minimum admissible intensity).  Reading: for
// each of the 8 surrounding pixels inside the image the single point nearest
// in world space (lowest slot on ties) is a neighbour when closer than h_int;
// r_new = (r + sum of neighbour r) / (1 + number of surrounding pixels in the
// image), Jacobi; then points with r_new < r_min are removed and the slots
// compacted in depth order.
//
// Background (intensity update's sibling: an FFT-based image denoiser for
// arrays, the identity for bistatic scanners).  Reading: circular
// convolution with a normalised sampled Gaussian of sigma_b pixels truncated
// at ceil(4 sigma_b), row pass then column pass, floor b_min.
#include "rt3d_dev.h"

namespace rt3d {

__global__ __launch_bounds__(256) void k_ifilter(DevParams p, Shape sh, DevState in, DevState out)
{
    const long long P = sh.P;
    const long long pix = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = load_cnt(in.cnt, pix);
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pix / per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);
    const float hi2 = (float)(p.h_int * p.h_int);
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const float rmin = (float)p.r_min;
    int nk = 0;
    for (int k = 0; k < KM; ++k) {
        if (k >= c) break;
        const double tq = in.t[k * P + pix];
        const float rq = in.r[k * P + pix];
        float sum = rq;
        int nside = 0;
        for (int di = -1; di <= 1; ++di) {
            const int i2 = i + di;
            if (i2 < 0 || i2 >= sh.rows) continue;
            const float dy = (float)di * pxy;
            for (int dj = -1; dj <= 1; ++dj) {
                const int j2 = j + dj;
                if ((di == 0 && dj == 0) || j2 < 0 || j2 >= sh.cols) continue;
                ++nside;
                const float dx = (float)dj * pxy;
                const long long pp = (fr * sh.rows + i2) * sh.cols + j2;
                const int cc = load_cnt(in.cnt, pp);
                int best = -1;
                float bd = 0.f;
                for (int k2 = 0; k2 < cc; ++k2) {
                    const float ddz = (float)((in.t[k2 * P + pp] - tq) * dz);
                    const float d2 = dx * dx + dy * dy + ddz * ddz;
                    if (best < 0 || d2 < bd) {
                        best = k2;
                        bd = d2;
                    }
                }
                if (best >= 0 && bd < hi2) sum += in.r[best * P + pp];
            }
        }
        const float rn = sum / (float)(1 + nside);
        if (rn < rmin) continue;
        out.t[nk * P + pix] = tq;
        out.r[nk * P + pix] = rn;
#pragma unroll
        for (int a = 0; a < 3; ++a) out.n[(a * KM + nk) * P + pix] = in.n[(a * KM + k) * P + pix];
        ++nk;
    }
    for (int k = nk; k < KM; ++k) {
        out.t[k * P + pix] = 0.0;
        out.r[k * P + pix] = 0.f;
        out.n[(0 * KM + k) * P + pix] = 0.f;
        out.n[(1 * KM + k) * P + pix] = 0.f;
        out.n[(2 * KM + k) * P + pix] = -1.f;
    }
    out.cnt[pix] = (uint8_t)nk;
    out.b[pix] = in.b[pix];
}

// Row pass: tmp[f][i][j] = sum_d w[d] b[f][i][(j + d) mod cols].
__global__ __launch_bounds__(256) void k_bfilter_rows(const float* __restrict__ w, int rb, Shape sh,
                                                      const float* __restrict__ b, float* __restrict__ tmp)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    const int j = (int)(pix % sh.cols);
    const long long rowbase = pix - j;
    float a = 0.f;
    for (int d = -rb; d <= rb; ++d) {
        int jj = (j + d) % sh.cols;
        if (jj < 0) jj += sh.cols;
        a = fmaf(w[d + rb], b[rowbase + jj], a);
    }
    tmp[pix] = a;
}

// Column pass with the floor: b[f][i][j] = max(b_min, sum_d w[d] tmp[f][(i + d) mod rows][j]).
__global__ __launch_bounds__(256) void k_bfilter_cols(const float* __restrict__ w, int rb, Shape sh, float b_min,
                                                      const float* __restrict__ tmp, float* __restrict__ b)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    const int per_frame = sh.rows * sh.cols;
    const long long fbase = pix - pix % per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);
    float a = 0.f;
    for (int d = -rb; d <= rb; ++d) {
        int ii = (i + d) % sh.rows;
        if (ii < 0) ii += sh.rows;
        a = fmaf(w[d + rb], tmp[fbase + (long long)ii * sh.cols + j], a);
    }
    b[pix] = fmaxf(a, b_min);
}

__global__ __launch_bounds__(256) void k_bfloor(Shape sh, float b_min, float* __restrict__ b)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    b[pix] = fmaxf(b[pix], b_min);
}

__global__ __launch_bounds__(256) void k_copy_state(Shape sh, DevState in, DevState out)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    out.cnt[pix] = in.cnt[pix];
    out.b[pix] = in.b[pix];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        out.t[k * P + pix] = in.t[k * P + pix];
        out.r[k * P + pix] = in.r[k * P + pix];
#pragma unroll
        for (int a = 0; a < 3; ++a) out.n[(a * KM + k) * P + pix] = in.n[(a * KM + k) * P + pix];
    }
}

__global__ __launch_bounds__(256) void k_out_count(Shape sh, const uint8_t* __restrict__ cnt, uint32_t* __restrict__ counts)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    counts[pix] = cnt[pix];
}

__global__ __launch_bounds__(256) void k_out_pack(Shape sh, DevState s, const uint32_t* __restrict__ pt_off,
                                                  uint32_t capacity, double* __restrict__ depth,
                                                  float* __restrict__ inten, float* __restrict__ normal,
                                                  float* __restrict__ bg, int32_t* __restrict__ err)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = load_cnt(s.cnt, pix);
    const uint32_t base = pt_off[pix];
    bool overflow = false;
    for (int k = 0; k < c; ++k) {
        const uint64_t at = (uint64_t)base + k;
        if (at >= capacity) {
            overflow = true;
            continue;
        }
        depth[at] = s.t[k * P + pix];
        inten[at] = s.r[k * P + pix];
        if (normal) {
#pragma unroll
            for (int a = 0; a < 3; ++a) normal[at * 3 + a] = s.n[(a * KM + k) * P + pix];
        }
    }
    bg[pix] = s.b[pix];
    if (overflow) *err = RT3D_E_CAPACITY;
}

static inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_ifilter(const DevParams& p, const Shape& sh, DevState in, DevState out, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ifilter, dim3(nblk(sh.P)), dim3(256), 0, st, p, sh, in, out);
    return hipGetLastError();
}

hipError_t launch_bfilter(const float* w, int rb, const Shape& sh, float b_min, float* b, float* tmp, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    if (rb <= 0) {
        hipLaunchKernelGGL(k_bfloor, dim3(nblk(sh.P)), dim3(256), 0, st, sh, b_min, b);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bfilter_rows, dim3(nblk(sh.P)), dim3(256), 0, st, w, rb, sh, b, tmp);
    hipLaunchKernelGGL(k_bfilter_cols, dim3(nblk(sh.P)), dim3(256), 0, st, w, rb, sh, b_min, tmp, b);
    return hipGetLastError();
}

hipError_t launch_copy_state(const Shape& sh, DevState in, DevState out, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_state, dim3(nblk(sh.P)), dim3(256), 0, st, sh, in, out);
    return hipGetLastError();
}

hipError_t launch_output(const Shape& sh, DevState s, rt3d_output* out, uint32_t* counts, uint32_t* partial,
                         int32_t* err, hipStream_t st)
{
    if (sh.P > 0)
        hipLaunchKernelGGL(k_out_count, dim3(nblk(sh.P)), dim3(256), 0, st, sh, s.cnt, counts);
    hipError_t e = launch_scan(counts, out->pt_off, sh.P, partial, out->capacity, err, st);
    if (e != hipSuccess) return e;
    if (sh.P > 0)
        hipLaunchKernelGGL(k_out_pack, dim3(nblk(sh.P)), dim3(256), 0, st, sh, s, out->pt_off, out->capacity,
                           out->depth, out->intensity, out->normal, out->background, err);
    return hipGetLastError();
}

}  // namespace rt3d

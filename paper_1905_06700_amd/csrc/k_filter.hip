// k_filter.hip -- the intensity denoiser and threshold, the background image
// filter, state copies and output packing.
//
// Intensity (Results, "Reconstruction algorithm", intensity update: a
// low-pass over nearest neighbours on the manifold the points define, which
// correlates only points of one surface, then removal of points below the
// minimum admissible intensity).  Reading: for each of the 8 surrounding
// pixels inside the image the single point nearest in world space (lowest
// slot on ties) is a neighbour when closer than h_int; r_new = (r + sum of
// neighbour r) / (1 + number of neighbours found), Jacobi (p.ilp_box = 1:
// divided by 1 + the number of surrounding pixels in the image instead); then
// points with r_new < r_min are removed and the slots compacted in depth
// order.
//
// Background (intensity update's sibling: an FFT-based image denoiser for
// arrays, the identity for bistatic scanners).  Reading: circular
// convolution with a normalised sampled Gaussian of sigma_b pixels truncated
// at ceil(4 sigma_b), row pass then column pass, floor b_min.
#include "rt3d_dev.h"

namespace rt3d {

// Intensity filter and threshold on 16 x 16 pixel tiles of one frame: the
// tile's depths, intensities and counts with a one-pixel halo are staged in
// LDS, then one thread per pixel filters its points.
constexpr int IFT = TILE;
constexpr int IFS = IFT + 2;

// PERSP: world distances of the pinhole camera (t dz along each pixel's ray).
// The orthographic variant fits 74 VGPRs: six workgroups per CU.
template <bool PERSP>
__global__ __launch_bounds__(IFT * IFT, PERSP ? 1 : 6) void k_ifilter_tile(DevParams p, Tiles tg, DevState in, DevState out)
{
    __shared__ double tl[KM][IFS * IFS];
    __shared__ float rl[KM][IFS * IFS];
    __shared__ int cl[IFS * IFS];
    const int tile0 = (int)xcd_block(blockIdx.x, gridDim.x);
    const int g = tile_group(tg, tile0);
    const Shape sh = group_shape(tg, g);
    in = state_at(in, tg.base[g]);
    out = state_at(out, tg.base[g]);
    const long long S = sh.S;
    const int tile = tile0 - tg.tile0[g];
    const int tiles_x = (sh.cols + IFT - 1) / IFT, tiles_y = (sh.rows + IFT - 1) / IFT;
    const int tpf = tiles_x * tiles_y;
    const int fr = tile / tpf, tr = tile % tpf;
    const int i0 = (tr / tiles_x) * IFT, j0 = (tr % tiles_x) * IFT;
    const long long fbase = (long long)fr * sh.rows * sh.cols;
    for (int x = threadIdx.x; x < IFS * IFS; x += IFT * IFT) {
        const int i2 = i0 - 1 + x / IFS, j2 = j0 - 1 + x % IFS;
        int c = 0;
        if (i2 >= 0 && i2 < sh.rows && j2 >= 0 && j2 < sh.cols) {
            const long long pp = fbase + (long long)i2 * sh.cols + j2;
            c = load_cnt(in.cnt, pp);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                tl[k][x] = in.t[k * S + pp];
                rl[k][x] = in.r[k * S + pp];
            }
        }
        cl[x] = c;
    }
    // Normals and background move with their own pixel only.  In place (the
    // iteration's planes) a kept point's normal moves only when an earlier
    // point of the pixel was dropped, and the background stays; into another
    // state they are copied, loaded here with the tile (the output loop would
    // otherwise wait on them once per kept point; the pinhole variant, short
    // of registers, reads the normals there).
    const bool n_inplace = in.n == out.n, b_inplace = in.b == out.b;
    const int ty = threadIdx.x / IFT, tx = threadIdx.x % IFT;
    const int i = i0 + ty, j = j0 + tx;
    const bool inside = i < sh.rows && j < sh.cols;
    const long long pix = fbase + (long long)(inside ? i : 0) * sh.cols + (inside ? j : 0);
    float nq[3][KM];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < KM; ++k)
            nq[a][k] = !PERSP && !n_inplace && inside ? in.n[(a * KM + k) * S + pix] : 0.f;
    const float bq = !b_inplace && inside ? in.b[pix] : 0.f;
    __syncthreads();
    if (!inside) return;
    const int xc = (ty + 1) * IFS + tx + 1;
    const int c = cl[xc];
    const float hi2 = (float)(p.h_int * p.h_int);
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const float rmin = (float)p.r_min;
    int nside = 0;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
            if (!(di == 0 && dj == 0) && i + di >= 0 && i + di < sh.rows && j + dj >= 0 && j + dj < sh.cols) ++nside;
    int nk = 0;
    double vq[3] = {0.0, 0.0, 1.0};
    if (PERSP) ray_dir(p.persp, sh.rows, sh.cols, i, j, vq);
    for (int k = 0; k < c; ++k) {
        const double tq = tl[k][xc];
        float sum = rl[k][xc];
        int deg = 0;
        for (int di = -1; di <= 1; ++di) {
            const float dy = (float)di * pxy;
            for (int dj = -1; dj <= 1; ++dj) {
                if (di == 0 && dj == 0) continue;
                const float dx = (float)dj * pxy;
                const int x = xc + di * IFS + dj;
                const int cc = cl[x];                   // 0 outside the image
                double v2[3] = {0.0, 0.0, 1.0};
                if (PERSP && cc > 0) ray_dir(p.persp, sh.rows, sh.cols, i + di, j + dj, v2);
                int best = -1;
                float bd = 0.f;
                for (int k2 = 0; k2 < cc; ++k2) {
                    float d2;
                    if (PERSP) {
                        const double t2 = tl[k2][x];
                        const float ex = (float)((t2 * v2[0] - tq * vq[0]) * dz);
                        const float ey = (float)((t2 * v2[1] - tq * vq[1]) * dz);
                        const float ez = (float)((t2 * v2[2] - tq * vq[2]) * dz);
                        d2 = ex * ex + ey * ey + ez * ez;
                    } else {
                        const float ddz = (float)((tl[k2][x] - tq) * dz);
                        d2 = dx * dx + dy * dy + ddz * ddz;
                    }
                    if (best < 0 || d2 < bd) {
                        best = k2;
                        bd = d2;
                    }
                }
                if (best >= 0 && bd < hi2) {
                    sum += rl[best][x];
                    ++deg;
                }
            }
        }
        const float rn = sum / (float)(1 + (p.ilp_box ? nside : deg));
        if (rn < rmin) continue;
        out.t[nk * S + pix] = tq;
        out.r[nk * S + pix] = rn;
        if (n_inplace) {
            // slot k moves down to nk < k: its reads come before any write to it
            if (nk != k)
#pragma unroll
                for (int a = 0; a < 3; ++a) out.n[(a * KM + nk) * S + pix] = in.n[(a * KM + k) * S + pix];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float v = nq[a][0];
#pragma unroll
                for (int k2 = 1; k2 < KM; ++k2) v = k == k2 ? nq[a][k2] : v;
                out.n[(a * KM + nk) * S + pix] = PERSP ? in.n[(a * KM + k) * S + pix] : v;
            }
        }
        ++nk;
    }
    // slots past the new count: cleared where they held a point; in the
    // iteration (normals in place) slots past the old count keep what they
    // hold, as every reader of a slot checks the count
    for (int k = nk; k < KM; ++k) {
        if (n_inplace && k >= c) break;
        out.t[k * S + pix] = 0.0;
        out.r[k * S + pix] = 0.f;
        out.n[(0 * KM + k) * S + pix] = 0.f;
        out.n[(1 * KM + k) * S + pix] = 0.f;
        out.n[(2 * KM + k) * S + pix] = -1.f;
    }
    out.cnt[pix] = (uint8_t)nk;
    if (!b_inplace) out.b[pix] = bq;
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

__global__ __launch_bounds__(256) void k_bfloor(Shape sh, float b_min, const float* __restrict__ src,
                                                float* __restrict__ dst)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    dst[pix] = fmaxf(src[pix], b_min);
}

// Both passes on 16 x 16 output tiles of one frame: the source region with an
// rb-pixel circular halo is staged in LDS, the row pass fills the halo rows'
// columns of the tile, the column pass writes the tile.  Per output the sums
// run over the taps in the same order as the two separate passes, so the
// result is the same to the bit.
constexpr int BFT = TILE;

inline size_t bfilter_tile_floats(int rb)
{
    const size_t S = BFT + 2 * (size_t)rb;
    return S * S + S * BFT + 2 * (size_t)rb + 1;
}

__device__ __forceinline__ int wrap_index(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

__global__ __launch_bounds__(BFT * BFT) void k_bfilter_tile(const float* __restrict__ w, int rb, Tiles tg,
                                                            float b_min, const float* __restrict__ src,
                                                            float* __restrict__ dst)
{
    extern __shared__ float bf_lds[];
    const int S = BFT + 2 * rb;
    float* reg = bf_lds;              // [S][S]: rows i0 - rb .., columns j0 - rb .. (circular)
    float* tmp = reg + S * S;         // [S][BFT]: row pass
    float* wl = tmp + S * BFT;        // [2 rb + 1] taps
    const int tile0 = (int)xcd_block(blockIdx.x, gridDim.x);
    const int g = tile_group(tg, tile0);
    const Shape sh = group_shape(tg, g);
    src += tg.base[g];
    dst += tg.base[g];
    const int tile = tile0 - tg.tile0[g];
    const int tiles_x = (sh.cols + BFT - 1) / BFT, tiles_y = (sh.rows + BFT - 1) / BFT;
    const int tpf = tiles_x * tiles_y;
    const int fr = tile / tpf, tr = tile % tpf;
    const int i0 = (tr / tiles_x) * BFT, j0 = (tr % tiles_x) * BFT;
    const long long fbase = (long long)fr * sh.rows * sh.cols;
    for (int k = threadIdx.x; k < 2 * rb + 1; k += BFT * BFT) wl[k] = w[k];
    // the region by rows and columns of the thread's place in the tile (one
    // wrap per row and per column, no division by S)
    {
        const int ry = threadIdx.x / BFT, rx = threadIdx.x % BFT;
        for (int r = ry; r < S; r += BFT) {
            const long long row = fbase + (long long)wrap_index(i0 - rb + r, sh.rows) * sh.cols;
            for (int c = rx; c < S; c += BFT) reg[r * S + c] = src[row + wrap_index(j0 - rb + c, sh.cols)];
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < S * BFT; x += BFT * BFT) {
        const int r = x / BFT, c = x % BFT;
        const float* row = reg + r * S + c + rb;
        float a = 0.f;
        for (int d = -rb; d <= rb; ++d) a = fmaf(wl[d + rb], row[d], a);
        tmp[x] = a;
    }
    __syncthreads();
    const int ty = threadIdx.x / BFT, tx = threadIdx.x % BFT;
    const int i = i0 + ty, j = j0 + tx;
    if (i >= sh.rows || j >= sh.cols) return;
    float a = 0.f;
    for (int d = -rb; d <= rb; ++d) a = fmaf(wl[d + rb], tmp[(ty + rb + d) * BFT + tx], a);
    dst[fbase + (long long)i * sh.cols + j] = fmaxf(a, b_min);
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

// Packs the slots into the caller's point lists; a non-finite depth,
// intensity or background sets E_NONFINITE (overflow of the caller's
// capacity sets E_CAPACITY).
__global__ __launch_bounds__(256) void k_out_pack(Shape sh, DevState s, const uint32_t* __restrict__ pt_off,
                                                  uint32_t capacity, double* __restrict__ depth,
                                                  float* __restrict__ inten, float* __restrict__ normal,
                                                  float* __restrict__ bg, long long n_bg, int32_t* __restrict__ err)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = load_cnt(s.cnt, pix);
    const uint32_t base = pt_off[pix];
    bool overflow = false, nonfinite = false;
    for (int k = 0; k < c; ++k) {
        const uint64_t at = (uint64_t)base + k;
        const double t = s.t[k * P + pix];
        const float r = s.r[k * P + pix];
        nonfinite |= !isfinite(t) || !isfinite(r);
        if (at >= capacity) {
            overflow = true;
            continue;
        }
        depth[at] = t;
        inten[at] = r;
        if (normal) {
#pragma unroll
            for (int a = 0; a < 3; ++a) normal[at * 3 + a] = s.n[(a * KM + k) * P + pix];
        }
    }
    if (pix < n_bg) {
        const float b = s.b[pix];
        nonfinite |= !isfinite(b);
        bg[pix] = b;
    }
    if (overflow) *err = RT3D_E_CAPACITY;
    if (nonfinite) *err = RT3D_E_NONFINITE;
}

// A gain that is not a finite non-negative number sets E_INVALID (the
// kernels treat such a pixel as dead).
__global__ __launch_bounds__(256) void k_check_gain(const float* __restrict__ gain, long long P,
                                                    int32_t* __restrict__ err)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const float g = gain[pix];
    if (!(g >= 0.f && g <= 3.402823466e38f)) *err = RT3D_E_INVALID;
}

// World Z of the packed points of one group of equal-size frames (the map f
// of the observation model): depth x dz, times the z component of the
// pixel's unit ray under the pinhole camera.  s is the group's state, pt_off
// the group's first pixel's entry of the output offsets.
__global__ __launch_bounds__(256) void k_out_world_z(Shape sh, DevState s, const uint32_t* __restrict__ pt_off,
                                                     uint32_t capacity, double dz, double persp,
                                                     double* __restrict__ wz)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    const int c = load_cnt(s.cnt, pix);
    if (c == 0) return;
    double scale = dz;
    if (persp > 0.0) {
        const long long q = pix % ((long long)sh.rows * sh.cols);
        double v[3];
        ray_dir(persp, sh.rows, sh.cols, (int)(q / sh.cols), (int)(q % sh.cols), v);
        scale = dz * v[2];
    }
    const uint32_t base = pt_off[pix];
    for (int k = 0; k < c; ++k) {
        const uint64_t at = (uint64_t)base + k;
        if (at < capacity) wz[at] = s.t[k * sh.S + pix] * scale;
    }
}

static inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_ifilter_tiles(const DevParams& p, const Tiles& tg, DevState in, DevState out, hipStream_t st)
{
    if (tg.n == 0 || tg.tile0[tg.n] == 0) return hipSuccess;
    if (p.persp > 0.0)
        hipLaunchKernelGGL(k_ifilter_tile<true>, dim3((unsigned)tg.tile0[tg.n]), dim3(IFT * IFT), 0, st, p, tg, in,
                           out);
    else
        hipLaunchKernelGGL(k_ifilter_tile<false>, dim3((unsigned)tg.tile0[tg.n]), dim3(IFT * IFT), 0, st, p, tg, in,
                           out);
    return hipGetLastError();
}

hipError_t launch_ifilter(const DevParams& p, const Shape& sh, DevState in, DevState out, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    return launch_ifilter_tiles(p, tiles_of(sh), in, out, st);
}

hipError_t launch_bfilter_tiles(const float* w, int rb, const Tiles& tg, float b_min, const float* src, float* dst,
                                float* tmp, hipStream_t st)
{
    if (tg.n == 0 || tg.tile0[tg.n] == 0) return hipSuccess;
    const size_t lds = sizeof(float) * bfilter_tile_floats(rb);
    if (rb > 0 && lds <= 49152) {
        hipLaunchKernelGGL(k_bfilter_tile, dim3((unsigned)tg.tile0[tg.n]), dim3(BFT * BFT), lds, st, w, rb, tg, b_min,
                           src, dst);
        return hipGetLastError();
    }
    for (int g = 0; g < tg.n; ++g) {
        const Shape sh = group_shape(tg, g);
        const long long b = tg.base[g];
        if (rb <= 0) {
            hipLaunchKernelGGL(k_bfloor, dim3(nblk(sh.P)), dim3(256), 0, st, sh, b_min, src + b, dst + b);
        } else {
            // wide filters: the row pass into tmp, the column pass into dst
            hipLaunchKernelGGL(k_bfilter_rows, dim3(nblk(sh.P)), dim3(256), 0, st, w, rb, sh, src + b, tmp + b);
            hipLaunchKernelGGL(k_bfilter_cols, dim3(nblk(sh.P)), dim3(256), 0, st, w, rb, sh, b_min, tmp + b, dst + b);
        }
    }
    return hipGetLastError();
}

hipError_t launch_bfilter(const float* w, int rb, const Shape& sh, float b_min, const float* src, float* dst,
                          float* tmp, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    return launch_bfilter_tiles(w, rb, tiles_of(sh), b_min, src, dst, tmp, st);
}

hipError_t launch_copy_state(const Shape& sh, DevState in, DevState out, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_state, dim3(nblk(sh.P)), dim3(256), 0, st, sh, in, out);
    return hipGetLastError();
}

hipError_t launch_output(const Shape& sh, DevState s, rt3d_output* out, uint32_t* counts, uint32_t* partial,
                         int32_t* err, long long n_bg, hipStream_t st)
{
    if (sh.P > 0)
        hipLaunchKernelGGL(k_out_count, dim3(nblk(sh.P)), dim3(256), 0, st, sh, s.cnt, counts);
    hipError_t e = launch_scan(counts, out->pt_off, sh.P, partial, out->capacity, err, st);
    if (e != hipSuccess) return e;
    if (sh.P > 0)
        hipLaunchKernelGGL(k_out_pack, dim3(nblk(sh.P)), dim3(256), 0, st, sh, s, out->pt_off, out->capacity,
                           out->depth, out->intensity, out->normal, out->background, n_bg, err);
    return hipGetLastError();
}

hipError_t launch_check_gain(const float* gain, long long P, int32_t* err, hipStream_t st)
{
    if (!gain || P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_gain, dim3(nblk(P)), dim3(256), 0, st, gain, P, err);
    return hipGetLastError();
}

hipError_t launch_world_z(const Shape& g, long long base, DevState s, const rt3d_output* out, double dz,
                          double persp, hipStream_t st)
{
    if (g.P == 0 || !out->world_z) return hipSuccess;
    hipLaunchKernelGGL(k_out_world_z, dim3(nblk(g.P)), dim3(256), 0, st, g, state_at(s, base), out->pt_off + base,
                       out->capacity, dz, persp, out->world_z);
    return hipGetLastError();
}

}  // namespace rt3d

// k_cnn.hip -- the learned depth denoiser that can replace APSS in the depth
// block (the paper treats the denoiser as interchangeable: Results,
// "Reconstruction algorithm"; Discussion, other denoisers trade quality for
// speed).  Reading (not in the paper): a four-layer 3x3 convolutional network
// on per-pixel slot maps (features of the first three slots: depth relative
// to the mean of the same-surface neighbours -- points of the 5x5 window
// within 3 sigma_h -- in sigma_h units, log(1 + r), valid flag, neighbour
// count) predicting each slot's depth correction in sigma_h units; pixels
// with four points keep APSS.
//
// Every convolution is an implicit GEMM on the matrix cores:
// v_mfma_f32_16x16x16_f16 (FP16 inputs, FP32 accumulation).  Activations are
// FP16 NHWC with 16 or 32 channels (64 B per pixel at 32), weights FP16.
//   forward:         Y[p][co]   = b[co] + sum_{tap, ci} X[p + tap][ci] W[tap][ci][co]
//   backward data:   dX[p][ci]  = sum_{tap, co} dY[p + tap][co] W'[tap][co][ci],
//                    W' the tap-flipped transpose, gated by the ReLU of X
//   backward weight: dW[tap][ci][co] = sum_p X[p + tap][ci] dY[p][co],
//                    per-workgroup partials reduced in a fixed order
// A forward / backward-data workgroup owns 64 consecutive pixels of CR = 4
// image rows (one row per wavefront, four 16-pixel MFMA row tiles each) and
// stages the CR + 2 halo rows and the layer's weights in LDS, rows padded so
// that a fragment read meets no bank conflict: every weight fragment read
// from LDS feeds four row tiles, and the staged weights serve 256 pixels.
// The weight-gradient workgroup owns 64 pixels of one row at a time.
#include "rt3d_dev.h"
#include "rt3d_cnn.h"

#include <hip/hip_fp16.h>

namespace rt3d {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int CT = 64;   // output pixels per workgroup row (one row segment)
constexpr int CR = 4;    // image rows per forward / backward-data workgroup (one per wavefront)
// LDS row padding (halves) of the forward / backward-data halo pixels and
// weight rows: strides of 4 mod 32 words put the 16 lanes of a fragment read
// on distinct banks
constexpr int CPAD = 4;

__device__ __forceinline__ float4_t mfma16(half4_t a, half4_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// Stages rows y-1..y+NR-2, columns x0-1..x0+CT of one frame (zero outside
// the image) into LDS as [NR][CT+2][C + PAD] halves.
template <int C, int NR = 3, int PAD = 0>
__device__ __forceinline__ void stage_halo(const __half* __restrict__ X, int F, int H, int W, int f, int y,
                                           int x0, __half* __restrict__ halo)
{
    constexpr int VPP = C / 8;                       // 16-byte vectors per pixel
    const int nvec = NR * (CT + 2) * VPP;
    for (int v = threadIdx.x; v < nvec; v += blockDim.x) {
        const int c8 = v % VPP;
        const int px = (v / VPP) % (CT + 2);
        const int ry = v / (VPP * (CT + 2));
        const int yy = y + ry - 1, xx = x0 + px - 1;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            val = reinterpret_cast<const uint4*>(X + (((long long)f * H + yy) * W + xx) * C)[c8];
        if (PAD == 0) {
            reinterpret_cast<uint4*>(halo)[v] = val;
        } else {   // 8-byte aligned rows
            uint2* d = reinterpret_cast<uint2*>(halo + (ry * (CT + 2) + px) * (C + PAD) + 8 * c8);
            d[0] = make_uint2(val.x, val.y);
            d[1] = make_uint2(val.z, val.w);
        }
    }
    (void)F;
}

// Forward / backward-data convolution.  Wt: FP16 [COUT][9 * CIN] (k = tap * CIN + ci,
// tap = ky * 3 + kx).  MODE 0: + bias, ReLU; 1: + bias (last layer); 2: gate by
// (G > 0) (backward data, G = the layer input's activation), no bias.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(64 * CR) void k_conv3x3(const __half* __restrict__ X, const __half* __restrict__ Wt,
                                                 const float* __restrict__ bias, const __half* __restrict__ Gate,
                                                 __half* __restrict__ Y, int F, int H, int W)
{
    constexpr int K = 9 * CIN;
    constexpr int NT = COUT / 16;
    constexpr int MT = CT / 16;                      // row tiles per wavefront
    constexpr int HS = CIN + CPAD, WS = K + CPAD;    // LDS strides (halves) of a halo pixel, a weight row
    __shared__ __align__(16) __half halo[(CR + 2) * (CT + 2) * HS];
    __shared__ __align__(16) __half wsh[COUT * WS];
    const int segs = (W + CT - 1) / CT;
    const int bands = (H + CR - 1) / CR;
    const int seg = blockIdx.x % segs;
    const int y0 = ((blockIdx.x / segs) % bands) * CR;
    const int f = blockIdx.x / (segs * bands);
    const int x0 = seg * CT;
    stage_halo<CIN, CR + 2, CPAD>(X, F, H, W, f, y0, x0, halo);
    for (int v = threadIdx.x; v < COUT * K / 8; v += blockDim.x) {
        const uint4 val = reinterpret_cast<const uint4*>(Wt)[v];
        const int row = v / (K / 8), c8 = v % (K / 8);
        uint2* d = reinterpret_cast<uint2*>(wsh + row * WS + 8 * c8);
        d[0] = make_uint2(val.x, val.y);
        d[1] = make_uint2(val.z, val.w);
    }
    __syncthreads();

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;   // wavefront wv: image row y0 + wv
    const int i = lane & 15, g = lane >> 4;
    float4_t acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[mt][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap % 3;
        const __half* arow = halo + (((wv + ky) * (CT + 2)) + i + kx) * HS;
#pragma unroll
        for (int cc = 0; cc < CIN / 16; ++cc) {
            const int k = tap * CIN + cc * 16 + 4 * g;
            half4_t b[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) b[n] = *reinterpret_cast<const half4_t*>(wsh + (n * 16 + i) * WS + k);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const half4_t a = *reinterpret_cast<const half4_t*>(arow + mt * 16 * HS + cc * 16 + 4 * g);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[mt][n] = mfma16(a, b[n], acc[mt][n]);
            }
        }
    }
    // D[row = 4 g + r][col = i] of row tile mt: pixel x0 + 16 mt + 4 g + r of row y, channel 16 n + i
    const int y = y0 + wv;
    if (y >= H) return;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + i;
        const float bco = (MODE != 2) ? bias[co] : 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = x0 + mt * 16 + 4 * g + r;
                if (x >= W) continue;
                const long long pix = ((long long)f * H + y) * W + x;
                float v = acc[mt][n][r] + bco;
                if (MODE == 0) v = fmaxf(v, 0.f);
                if (MODE == 2 && !(__half2float(Gate[pix * COUT + co]) > 0.f)) v = 0.f;
                Y[pix * COUT + co] = __float2half(v);
            }
    }
}

// Weight gradient partials: each workgroup reduces its row segment over
// ROWS_PER_WG consecutive rows (same frame) into part[wg][9 * CIN][COUT] and
// bias partials bpart[wg][COUT].
constexpr int WG_ROWS = 8;

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const __half* __restrict__ X, const __half* __restrict__ dY,
                                                       float* __restrict__ part, float* __restrict__ bpart,
                                                       int F, int H, int W)
{
    constexpr int K9 = 9 * CIN;
    constexpr int MT = K9 / 16;                  // row tiles of (tap, ci)
    constexpr int NT = COUT / 16;
    constexpr int TILES = MT * NT;
    constexpr int TPW = (TILES + 3) / 4;         // tiles per wavefront
    __shared__ __align__(16) __half halo[3 * (CT + 2) * CIN];
    __shared__ __align__(16) __half dys[CT * COUT];
    const int segs = (W + CT - 1) / CT;
    const int rblocks = (H + WG_ROWS - 1) / WG_ROWS;
    const int seg = blockIdx.x % segs;
    const int rb = (blockIdx.x / segs) % rblocks;
    const int f = blockIdx.x / (segs * rblocks);
    const int x0 = seg * CT;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    float4_t acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = (float4_t){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int yr = 0; yr < WG_ROWS; ++yr) {
        const int y = rb * WG_ROWS + yr;
        if (y >= H) break;
        __syncthreads();
        stage_halo<CIN>(X, F, H, W, f, y, x0, halo);
        for (int v = threadIdx.x; v < CT * COUT / 8; v += blockDim.x) {
            const int px = v / (COUT / 8), c8 = v % (COUT / 8);
            const int x = x0 + px;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (x < W) val = reinterpret_cast<const uint4*>(dY + (((long long)f * H + y) * W + x) * COUT)[c8];
            reinterpret_cast<uint4*>(dys)[v] = val;
        }
        __syncthreads();
        if (threadIdx.x < COUT)
            for (int px = 0; px < CT; ++px) bsum += __half2float(dys[px * COUT + threadIdx.x]);
        // K dimension: the segment's 64 pixels in 4 steps of 16
#pragma unroll
        for (int ks = 0; ks < CT / 16; ++ks) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int tile = wv * TPW + t;
                if (tile >= TILES) continue;
                const int mt = tile / NT, nt = tile % NT;
                const int row = mt * 16 + i;                  // (tap, ci) of this lane's A row
                const int tap = row / CIN, ci = row % CIN;
                const int ky = tap / 3, kx = tap % 3;
                half4_t a, b;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int px = ks * 16 + 4 * g + r;        // reduction index = pixel
                    a[r] = (_Float16)halo[((ky * (CT + 2)) + px + kx) * CIN + ci];
                    b[r] = (_Float16)dys[px * COUT + nt * 16 + i];
                }
                acc[t] = mfma16(a, b, acc[t]);
            }
        }
    }
    float* out = part + (size_t)blockIdx.x * K9 * COUT;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int tile = wv * TPW + t;
        if (tile >= TILES) continue;
        const int mt = tile / NT, nt = tile % NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(mt * 16 + 4 * g + r) * COUT + nt * 16 + i] = acc[t][r];
    }
    if (threadIdx.x < COUT) bpart[(size_t)blockIdx.x * COUT + threadIdx.x] = bsum;
}

// Sums weight-gradient partials over workgroups in a fixed order and writes
// the FP32 gradient of the flat master-weight layout (scaled by 1/count).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ bpart,
                                                      int nwg, int cin_store, int cout_store, int cin, int cout,
                                                      const float* __restrict__ count, float* __restrict__ grad)
{
    const int n_w = 9 * cin * cout;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_w + cout) return;
    const float inv = 1.f / fmaxf(count[0], 1.f);
    float s = 0.f;
    if (idx < n_w) {
        const int co = idx % cout, ci = (idx / cout) % cin, tap = idx / (cout * cin);
        const int row = tap * cin_store + ci;
        for (int wg = 0; wg < nwg; ++wg) s += part[((size_t)wg * 9 * cin_store + row) * cout_store + co];
    } else {
        const int co = idx - n_w;
        for (int wg = 0; wg < nwg; ++wg) s += bpart[(size_t)wg * cout_store + co];
    }
    grad[idx] = s * inv;
}

// Features of the first three slots, FP16 [P][16].
// Features of slots k < min(cnt, 3): the neighbours of slot k are the points
// (any slot) of the 5x5 window (same frame, inside the image, itself
// included) within CNN_GATE sigma_h of t_k; channels 4k .. 4k+3 hold
// (t_k - their mean) / sigma_h clipped to [-8, 8], log(1 + r_k), 1 and their
// number / 25.  The other channels are zero.
// Features of 16 x 16 pixel tiles: the tile's depths and counts with a
// 2-pixel halo (the 5 x 5 windows) staged in LDS, one thread per pixel.
constexpr int PKT = 16, PKS = PKT + 4;
__global__ __launch_bounds__(PKT * PKT) void k_cnn_pack(Shape sh, DevState s, float sigma_h, __half* __restrict__ x)
{
    __shared__ double tl[KM][PKS * PKS];
    __shared__ int cl[PKS * PKS];
    const long long S = sh.S;   // slot stride (the whole batch's pixels when sh is one group of it)
    const int tiles_x = (sh.cols + PKT - 1) / PKT, tiles_y = (sh.rows + PKT - 1) / PKT;
    const int tpf = tiles_x * tiles_y;
    const int fr = (int)(blockIdx.x / tpf), tr = (int)(blockIdx.x % tpf);
    const int i0 = (tr / tiles_x) * PKT, j0 = (tr % tiles_x) * PKT;
    const long long fbase = (long long)fr * sh.rows * sh.cols;
    for (int xx = threadIdx.x; xx < PKS * PKS; xx += PKT * PKT) {
        const int i2 = i0 - 2 + xx / PKS, j2 = j0 - 2 + xx % PKS;
        int c2 = 0;
        if (i2 >= 0 && i2 < sh.rows && j2 >= 0 && j2 < sh.cols) {
            const long long pp = fbase + (long long)i2 * sh.cols + j2;
            c2 = load_cnt(s.cnt, pp);
#pragma unroll
            for (int k = 0; k < KM; ++k) tl[k][xx] = s.t[k * S + pp];
        }
        cl[xx] = c2;                                  // 0 outside the image
    }
    __syncthreads();
    const int ty = threadIdx.x / PKT, tx = threadIdx.x % PKT;
    const int i = i0 + ty, j = j0 + tx;
    if (i >= sh.rows || j >= sh.cols) return;
    const long long pix = fbase + (long long)i * sh.cols + j;
    const int xc = (ty + 2) * PKS + tx + 2;
    const int c = min(cl[xc], 3);
    const double gate = CNN_GATE * (double)sigma_h;
    double tk[3], sum[3] = {0.0, 0.0, 0.0};
    int n[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) tk[k] = k < c ? tl[k][xc] : 0.0;
    // each window point is read once and added to every slot it gates in
    // (per slot, the terms arrive in window order: rows, then columns, then slots)
    for (int di = -2; di <= 2; ++di)
        for (int dj = -2; dj <= 2; ++dj) {
            const int xx = xc + di * PKS + dj;
            const int c2 = cl[xx];
            for (int k2 = 0; k2 < c2; ++k2) {
                const double tm = tl[k2][xx];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < c && fabs(tm - tk[k]) <= gate) {
                        sum[k] += tm;
                        ++n[k];
                    }
            }
        }
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= c) continue;
        const double mean = sum[k] / n[k];
        v[4 * k] = fminf(fmaxf((float)((tk[k] - mean) / (double)sigma_h), -8.f), 8.f);
        v[4 * k + 1] = log1pf(s.r[k * S + pix]);
        v[4 * k + 2] = 1.f;
        v[4 * k + 3] = (float)n[k] / 25.f;
    }
    // the pixel's 16 halves as two 16-byte stores
    uint4 o[2];
    uint32_t* ow = reinterpret_cast<uint32_t*>(o);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t lo = __half_as_ushort(__float2half(v[2 * q]));
        const uint32_t hi = __half_as_ushort(__float2half(v[2 * q + 1]));
        ow[q] = lo | (hi << 16);
    }
    reinterpret_cast<uint4*>(x + pix * 16)[0] = o[0];
    reinterpret_cast<uint4*>(x + pix * 16)[1] = o[1];
}

// Slot k < 3 of a pixel with at most three points moves by sigma_h * y_k.
__global__ __launch_bounds__(256) void k_cnn_apply(Shape sh, const __half* __restrict__ y, float sigma_h,
                                                   double tmax, DevState s)
{
    const long long S = sh.S;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= sh.P) return;
    const int c = load_cnt(s.cnt, pix);
    if (c > 3) return;
    for (int k = 0; k < c; ++k) {
        double t = s.t[k * S + pix] + (double)(sigma_h * __half2float(y[pix * 16 + k]));
        t = t < 0.0 ? 0.0 : (t > tmax ? tmax : t);
        s.t[k * S + pix] = t;
    }
}

// Network outputs of the first three channels as float [3][P].
__global__ __launch_bounds__(256) void k_cnn_unpack(long long P, const __half* __restrict__ y, float* __restrict__ out)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k * P + pix] = __half2float(y[pix * 16 + k]);
}

// Training targets: slot k < min(cnt, 3) takes the nearest true depth of its
// pixel within 3 sigma_h (first surface on ties); truth [S][P], NaN = absent.
__global__ __launch_bounds__(256) void k_cnn_targets(Shape sh, DevState s, const float* __restrict__ truth, int S,
                                                     float sigma_h, float* __restrict__ tgt, uint8_t* __restrict__ msk)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = min(load_cnt(s.cnt, pix), 3);
    for (int k = 0; k < 3; ++k) {
        float tv = 0.f;
        uint8_t mv = 0;
        if (k < c) {
            const double t = s.t[k * P + pix];
            double bd = 0.0;
            int bs = -1;
            for (int q = 0; q < S; ++q) {
                const float tr = truth[(long long)q * P + pix];
                if (!(tr == tr)) continue;               // NaN: no such surface
                const double d = fabs((double)tr - t);
                if (bs < 0 || d < bd) {
                    bs = q;
                    bd = d;
                }
            }
            if (bs >= 0 && bd <= 3.0 * (double)sigma_h) {
                tv = fminf(fmaxf((float)(((double)truth[(long long)bs * P + pix] - t) / (double)sigma_h), -8.f), 8.f);
                mv = 1;
            }
        }
        tgt[k * P + pix] = tv;
        msk[k * P + pix] = mv;
    }
}

// Masked squared error: per-block partial sums, and dY = 2 (y - y*) m in FP16
// (the gradient of the sum; 1/count is applied to the weight gradients).
__global__ __launch_bounds__(256) void k_cnn_loss(long long P, const __half* __restrict__ y,
                                                  const float* __restrict__ tgt, const uint8_t* __restrict__ msk,
                                                  __half* __restrict__ dy, float* __restrict__ lpart)
{
    __shared__ float red[2][256];
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float se = 0.f, n = 0.f;
    if (pix < P) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float g = 0.f;
            if (k < 3 && msk[k * P + pix]) {
                const float d = __half2float(y[pix * 16 + k]) - tgt[k * P + pix];
                se += d * d;
                n += 1.f;
                g = 2.f * d;
            }
            dy[pix * 16 + k] = __float2half(g);
        }
    }
    red[0][threadIdx.x] = se;
    red[1][threadIdx.x] = n;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lpart[2 * blockIdx.x] = red[0][0];
        lpart[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(64) void k_cnn_loss_final(const float* __restrict__ lpart, int nb, float* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double se = 0.0, n = 0.0;
    for (int b = 0; b < nb; ++b) {
        se += lpart[2 * b];
        n += lpart[2 * b + 1];
    }
    out[0] = (float)(se / (n > 1.0 ? n : 1.0));
    out[1] = (float)n;
}

// Adam on the FP32 master weights.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float gi = g[idx];
    const float mi = b1 * m[idx] + (1.f - b1) * gi;
    const float vi = b2 * v[idx] + (1.f - b2) * gi * gi;
    m[idx] = mi;
    v[idx] = vi;
    w[idx] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP16 kernel layouts from the FP32 master weights of one layer (flat
// [3][3][cin][cout] then bias[cout]): forward Wt[co][tap * CIS + ci] and
// backward-data Wb[ci][tap' * COS + co] with tap' = 8 - tap; padded
// channels are zero.
__global__ __launch_bounds__(256) void k_cnn_prepare(const float* __restrict__ mw, int cin, int cout, int cis, int cos_,
                                                     __half* __restrict__ wt, __half* __restrict__ wb,
                                                     float* __restrict__ bias)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = cos_ * 9 * cis;
    if (idx < nf) {
        const int co = idx / (9 * cis), k = idx % (9 * cis), tap = k / cis, ci = k % cis;
        const float v = (co < cout && ci < cin) ? mw[(tap * cin + ci) * cout + co] : 0.f;
        wt[idx] = __float2half(v);
        // the same weight in the backward-data layout
        if (wb) wb[ci * 9 * cos_ + (8 - tap) * cos_ + co] = __float2half(v);
    }
    if (idx < cos_) bias[idx] = idx < cout ? mw[9 * cin * cout + idx] : 0.f;
}

// ---------------------------------------------------------------------------
// Fused inference: the four convolutions of one FT x FT output tile in one
// workgroup, every intermediate activation kept in LDS (FP16, the rounding
// the per-layer kernels apply when they store it).  Layer l computes its
// output over the tile grown by 4 - l pixels on every side (the receptive
// field of the layers after it); outputs at positions outside the image are
// set to zero, which is the next layer's zero padding.  Matrix cores:
// v_mfma_f32_16x16x32_f16 (lane i + 16 g holds row i, k = 8 g .. 8 g + 7 of A
// and column i, the same k of B; D rows 4 g .. 4 g + 3 of column i).  The
// B operand (the layer's weights) stays in registers for the whole layer; A
// rows are output pixels, gathered from LDS per lane (one 16-byte chunk of 8
// channels of the input pixel under the tap).
constexpr int FT = 16;                   // output tile side
constexpr int FR0 = FT + 8;              // side of the staged input features (4-pixel halo)

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float4_t mfma32(half8_t a, half8_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// LDS offset (halves) of 16-byte chunk q of pixel p in a region of C-channel
// pixels, the chunks of a pixel permuted by its index so that the same chunk
// of 8 consecutive pixels lies in 8 distinct bank groups.
template <int C>
__device__ __forceinline__ int chunk_at(int p, int q)
{
    if (C == 32) return p * 32 + 8 * (q ^ ((p >> 1) & 3));
    return p * 16 + 8 * (q ^ ((p >> 2) & 1));
}

// One layer over the RO x RO output region whose input region (RO + 2 wide)
// sits in `in`.  NT output tiles of 16 channels; LAST: bias only, the FT x FT
// result goes to y (FP16 [P][16]); else bias, ReLU, zero outside the image,
// into `out` (32 channels).  (gy0, gx0): image position of the output
// region's first pixel.
template <int CIN, int NT, bool LAST>
__device__ __forceinline__ void fused_layer(const __half* __restrict__ in, __half* __restrict__ out, int RO,
                                            const __half* __restrict__ Wt, const float* __restrict__ bias, int gy0,
                                            int gx0, int H, int W, long long fbase, __half* __restrict__ y)
{
    constexpr int K = 9 * CIN;
    constexpr int KC = (K + 31) / 32;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    half8_t wf[KC][NT];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int k0 = kc * 32 + 8 * g;
            half8_t v = {};
            if (k0 < K) v = *reinterpret_cast<const half8_t*>(Wt + (n * 16 + i) * K + k0);
            wf[kc][n] = v;
        }
    float bco[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) bco[n] = bias[n * 16 + i];
    const int RI = RO + 2, npx = RO * RO, nmt = (npx + 15) / 16;
    for (int mt0 = wv; mt0 < nmt; mt0 += 8) {
        int abase[2];
        bool aval[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int m = (mt0 + 4 * u) * 16 + i;
            aval[u] = (mt0 + 4 * u) < nmt && m < npx;
            const int mm = aval[u] ? m : 0;
            abase[u] = (mm / RO) * RI + mm % RO;          // input pixel under tap (0, 0)
        }
        float4_t acc[2][NT];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[u][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            int tap, q;
            if (CIN == 32) {
                tap = kc;
                q = g;
            } else {
                tap = 2 * kc + (g >> 1);
                q = g & 1;
            }
            const int dp = (tap / 3) * RI + tap % 3;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                half8_t a = {};
                if (aval[u] && tap < 9) a = *reinterpret_cast<const half8_t*>(in + chunk_at<CIN>(abase[u] + dp, q));
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[u][n] = mfma32(a, wf[kc][n], acc[u][n]);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (mt0 + 4 * u >= nmt) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = (mt0 + 4 * u) * 16 + 4 * g + r;
                if (m >= npx) continue;
                const int oy = m / RO, ox = m % RO;
                const int gy = gy0 + oy, gx = gx0 + ox;
                const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const float v = acc[u][n][r] + bco[n];
                    if (LAST) {
                        if (inside) y[(fbase + (long long)gy * W + gx) * 16 + n * 16 + i] = __float2half(v);
                    } else {
                        const int ch = n * 16 + i;
                        out[chunk_at<32>(m, ch >> 3) + (ch & 7)] = __float2half(inside ? fmaxf(v, 0.f) : 0.f);
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_cnn_fused(const __half* __restrict__ x, const __half* __restrict__ w0,
                                                   const __half* __restrict__ w1, const __half* __restrict__ w2,
                                                   const __half* __restrict__ w3, const float* __restrict__ b0,
                                                   const float* __restrict__ b1, const float* __restrict__ b2,
                                                   const float* __restrict__ b3, __half* __restrict__ y, int H, int W)
{
    // buf0: the input features (FR0^2 x 16 channels), later layer 2's output
    // ((FT + 4)^2 x 32); buf1: layer 1's output ((FT + 6)^2 x 32), later layer 3's
    __shared__ __align__(16) __half buf0[(FT + 4) * (FT + 4) * 32];
    __shared__ __align__(16) __half buf1[(FT + 6) * (FT + 6) * 32];
    static_assert(FR0 * FR0 * 16 <= (FT + 4) * (FT + 4) * 32, "the features fit buf0");
    const int tx_n = (W + FT - 1) / FT, ty_n = (H + FT - 1) / FT;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int f = tile / (tx_n * ty_n), tr = tile % (tx_n * ty_n);
    const int Y0 = (tr / tx_n) * FT, X0 = (tr % tx_n) * FT;
    const long long fbase = (long long)f * H * W;
    for (int v = threadIdx.x; v < FR0 * FR0 * 2; v += blockDim.x) {
        const int p = v >> 1, q = v & 1;
        const int gy = Y0 - 4 + p / FR0, gx = X0 - 4 + p % FR0;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            val = reinterpret_cast<const uint4*>(x + (fbase + (long long)gy * W + gx) * 16)[q];
        *reinterpret_cast<uint4*>(buf0 + chunk_at<16>(p, q)) = val;
    }
    __syncthreads();
    fused_layer<16, 2, false>(buf0, buf1, FT + 6, w0, b0, Y0 - 3, X0 - 3, H, W, fbase, nullptr);
    __syncthreads();
    fused_layer<32, 2, false>(buf1, buf0, FT + 4, w1, b1, Y0 - 2, X0 - 2, H, W, fbase, nullptr);
    __syncthreads();
    fused_layer<32, 2, false>(buf0, buf1, FT + 2, w2, b2, Y0 - 1, X0 - 1, H, W, fbase, nullptr);
    __syncthreads();
    fused_layer<32, 1, true>(buf1, nullptr, FT, w3, b3, Y0, X0, H, W, fbase, y);
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

// Forward / backward-data workgroups: 64 columns x CR rows each.
static unsigned conv_grid(const Shape& sh)
{
    return (unsigned)(sh.F * ((sh.rows + CR - 1) / CR) * ((sh.cols + CT - 1) / CT));
}

unsigned cnn_wgrad_groups(const Shape& sh)
{
    return (unsigned)(sh.F * ((sh.rows + WG_ROWS - 1) / WG_ROWS) * ((sh.cols + CT - 1) / CT));
}

hipError_t launch_cnn_prepare(const CnnWeights& w, hipStream_t st)
{
    const float* mw = w.master;
    for (int l = 0; l < CNN_LAYERS; ++l) {
        const int nf = CNN_COS[l] * 9 * CNN_CIS[l];
        hipLaunchKernelGGL(k_cnn_prepare, dim3(nb256(nf)), dim3(256), 0, st, mw, CNN_CIN[l], CNN_COUT[l],
                           CNN_CIS[l], CNN_COS[l], w.wt[l], l > 0 ? w.wb[l] : nullptr, w.bias[l]);
        mw += 9 * CNN_CIN[l] * CNN_COUT[l] + CNN_COUT[l];
    }
    return hipGetLastError();
}

hipError_t launch_cnn_forward(const Shape& sh, DevState s, float sigma_h, const CnnWeights& w, const CnnBuffers& b,
                              hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    const unsigned tiles = (unsigned)(sh.F * ((sh.rows + PKT - 1) / PKT) * ((sh.cols + PKT - 1) / PKT));
    hipLaunchKernelGGL(k_cnn_pack, dim3(tiles), dim3(PKT * PKT), 0, st, sh, s, sigma_h, b.act[0]);
    const unsigned g = conv_grid(sh);
    hipLaunchKernelGGL((k_conv3x3<16, 32, 0>), dim3(g), dim3(64 * CR), 0, st, b.act[0], w.wt[0], w.bias[0], nullptr,
                       b.act[1], sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL((k_conv3x3<32, 32, 0>), dim3(g), dim3(64 * CR), 0, st, b.act[1], w.wt[1], w.bias[1], nullptr,
                       b.act[2], sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL((k_conv3x3<32, 32, 0>), dim3(g), dim3(64 * CR), 0, st, b.act[2], w.wt[2], w.bias[2], nullptr,
                       b.act[3], sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL((k_conv3x3<32, 16, 1>), dim3(g), dim3(64 * CR), 0, st, b.act[3], w.wt[3], w.bias[3], nullptr,
                       b.act[4], sh.F, sh.rows, sh.cols);
    return hipGetLastError();
}

hipError_t launch_cnn_infer(const Shape& sh, DevState s, float sigma_h, const CnnWeights& w, const CnnBuffers& b,
                            hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    const unsigned tiles = (unsigned)(sh.F * ((sh.rows + PKT - 1) / PKT) * ((sh.cols + PKT - 1) / PKT));
    hipLaunchKernelGGL(k_cnn_pack, dim3(tiles), dim3(PKT * PKT), 0, st, sh, s, sigma_h, b.act[0]);
    const unsigned ft = (unsigned)(sh.F * ((sh.rows + FT - 1) / FT) * ((sh.cols + FT - 1) / FT));
    hipLaunchKernelGGL(k_cnn_fused, dim3(ft), dim3(256), 0, st, b.act[0], w.wt[0], w.wt[1], w.wt[2], w.wt[3],
                       w.bias[0], w.bias[1], w.bias[2], w.bias[3], b.act[4], sh.rows, sh.cols);
    return hipGetLastError();
}

hipError_t launch_cnn_apply(const Shape& sh, const CnnBuffers& b, float sigma_h, double tmax, DevState s,
                            hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cnn_apply, dim3(nb256(sh.P)), dim3(256), 0, st, sh, b.act[4], sigma_h, tmax, s);
    return hipGetLastError();
}

hipError_t launch_cnn_unpack(const Shape& sh, const CnnBuffers& b, float* out, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cnn_unpack, dim3(nb256(sh.P)), dim3(256), 0, st, sh.P, b.act[4], out);
    return hipGetLastError();
}

hipError_t launch_cnn_train_step(const Shape& sh, DevState s, float sigma_h, const float* truth, int S,
                                 CnnWeights& w, const CnnBuffers& b, const CnnAdam& opt, float* loss,
                                 hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipError_t e = launch_cnn_forward(sh, s, sigma_h, w, b, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cnn_targets, dim3(nb256(sh.P)), dim3(256), 0, st, sh, s, truth, S, sigma_h, b.tgt, b.msk);
    const unsigned nbl = nb256(sh.P);
    hipLaunchKernelGGL(k_cnn_loss, dim3(nbl), dim3(256), 0, st, sh.P, b.act[4], b.tgt, b.msk, b.dy16, b.lpart);
    hipLaunchKernelGGL(k_cnn_loss_final, dim3(1), dim3(64), 0, st, b.lpart, (int)nbl, loss);
    const unsigned g = conv_grid(sh);
    const unsigned gw = cnn_wgrad_groups(sh);
    // layer 3 (32 -> 16 stored): weight gradient, then data gradient into layer 2's output
    float* grad = b.grad;
    const int off3 = CNN_OFF[3], off2 = CNN_OFF[2], off1 = CNN_OFF[1], off0 = CNN_OFF[0];
    hipLaunchKernelGGL((k_conv3x3_wgrad<32, 16>), dim3(gw), dim3(256), 0, st, b.act[3], b.dy16, b.part, b.bpart,
                       sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb256(9 * 32 * 3 + 3)), dim3(256), 0, st, b.part, b.bpart, (int)gw, 32, 16,
                       32, 3, loss + 1, grad + off3);
    hipLaunchKernelGGL((k_conv3x3<16, 32, 2>), dim3(g), dim3(64 * CR), 0, st, b.dy16, w.wb[3], nullptr, b.act[3], b.dA,
                       sh.F, sh.rows, sh.cols);
    // layer 2
    hipLaunchKernelGGL((k_conv3x3_wgrad<32, 32>), dim3(gw), dim3(256), 0, st, b.act[2], b.dA, b.part, b.bpart,
                       sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb256(9 * 32 * 32 + 32)), dim3(256), 0, st, b.part, b.bpart, (int)gw, 32,
                       32, 32, 32, loss + 1, grad + off2);
    hipLaunchKernelGGL((k_conv3x3<32, 32, 2>), dim3(g), dim3(64 * CR), 0, st, b.dA, w.wb[2], nullptr, b.act[2], b.dB,
                       sh.F, sh.rows, sh.cols);
    // layer 1
    hipLaunchKernelGGL((k_conv3x3_wgrad<32, 32>), dim3(gw), dim3(256), 0, st, b.act[1], b.dB, b.part, b.bpart,
                       sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb256(9 * 32 * 32 + 32)), dim3(256), 0, st, b.part, b.bpart, (int)gw, 32,
                       32, 32, 32, loss + 1, grad + off1);
    hipLaunchKernelGGL((k_conv3x3<32, 32, 2>), dim3(g), dim3(64 * CR), 0, st, b.dB, w.wb[1], nullptr, b.act[1], b.dA,
                       sh.F, sh.rows, sh.cols);
    // layer 0 (16 -> 32): weight gradient only
    hipLaunchKernelGGL((k_conv3x3_wgrad<16, 32>), dim3(gw), dim3(256), 0, st, b.act[0], b.dA, b.part, b.bpart,
                       sh.F, sh.rows, sh.cols);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb256(9 * 16 * 32 + 32)), dim3(256), 0, st, b.part, b.bpart, (int)gw, 16,
                       32, 16, 32, loss + 1, grad + off0);
    // Adam, then the FP16 layouts
    ++w.step;
    const float c1 = 1.f - powf(opt.beta1, (float)w.step), c2 = 1.f - powf(opt.beta2, (float)w.step);
    hipLaunchKernelGGL(k_adam, dim3(nb256(CNN_PARAMS)), dim3(256), 0, st, w.master, w.m, w.v, grad, CNN_PARAMS,
                       opt.lr, opt.beta1, opt.beta2, opt.eps, c1, c2);
    return launch_cnn_prepare(w, st);
}

}  // namespace rt3d

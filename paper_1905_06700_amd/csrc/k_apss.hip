// k_apss.hip -- APSS point-cloud denoising of depth (Results, "Reconstruction
// algorithm", depth update: algebraic point set surfaces fit local spheres to
// the points in world coordinates, the kernel size setting the low-pass) and
// the in-pixel merge of coincident points.
//
// Sphere fit (derived from its least-squares definition): with neighbours
// y_m = x_m - x_q closer than h, weights w = (1 - d^2/h^2)^4 and unit normals
// n_m, the sphere s(y) = u0 + ul.y + u4 |y|^2 minimising
// sum w |grad s(y_m) - n_m|^2, then sum w s(y_m)^2 over u0, is
//   u4 = (PN - P.N/W) / (2 (PP - P.P/W)),  ul = (N - 2 u4 P)/W,
//   u0 = -(ul.P + u4 PP)/W,
// W = sum w, P = sum w y, N = sum w n, PN = sum w y.n, PP = sum w y.y.
// Reading: q moves along its line of sight to the sphere's root nearest to it
// (clipped to [-h, h]); its normal becomes grad s there, facing the sensor.
// Jacobi: every query reads the state before the step.
//
// Mapping: a workgroup takes a tile of ATY x ATX pixels of one frame; it stages
// the counts and every slot of the tile with a halo in LDS in one round of
// loads (depths in FP64, normals; a second round for the live slots only,
// after the counts, cost more time than the bytes it saved), then one thread per pixel fits and projects the pixel's
// points, accumulating the sphere moments over the window from LDS in FP32,
// in coordinates local to the query (depth differences formed in FP64); under
// the orthographic map the halo covers only the pixels whose lateral offset
// stays below h, and each neighbour is read once for all the pixel's slots.
// Windows whose staged tile does not fit in 64 KB of LDS take a variant with
// eight lanes per pixel reading the state from global memory, the partial
// moment sets meeting in a fixed wavefront-shuffle tree.
#include "rt3d_dev.h"

namespace rt3d {

constexpr int ATX = TILE, ATY = TILE;   // tile of the LDS variant: columns, rows

// LDS bytes of a staged tile with an R-pixel halo: per pixel KM depths (FP64),
// 3 x KM normal components and the count.
inline size_t apss_tile_bytes(int R)
{
    const size_t SX = ATX + 2 * (size_t)R, SY = ATY + 2 * (size_t)R;
    return SX * SY * (KM * sizeof(double) + 3 * KM * sizeof(float) + sizeof(int));
}

size_t apss_lds_bytes(int R) { return apss_tile_bytes(R); }

// Halo the orthographic tile kernel stages: the largest ring r of window
// pixels (Chebyshev distance r) whose nearest pixel, r pixels away along a
// row, lies closer than h -- pixels of farther rings hold no neighbour.  The
// same FP32 arithmetic as the kernel's lateral pre-test.
int apss_staged_halo(double h_apss, double p_xy, int R)
{
    const float h = (float)h_apss, h2 = h * h, pxy = (float)p_xy;
    int r = 0;
    while (r < R) {
        const float x = (float)(r + 1) * pxy;
        if (!(x * x < h2)) break;
        ++r;
    }
    return r;
}

// PERSP: positions of the pinhole camera (t dz along each pixel's ray,
// differences formed in FP64), no lateral pre-test, projection along the
// query's ray; else the orthographic map, staged halo p.apss_Rs.
// carry: also copy the count, background and intensities to `out` (else
// `out` receives only the depths and normals of the live slots).  The
// orthographic variant runs five workgroups per CU (96 VGPRs; a few values
// wait in scratch).
template <bool PERSP>
__global__ __launch_bounds__(ATX * ATY, PERSP ? 1 : 5) void k_apss_tile(DevModel m, DevParams p, Tiles tg, DevState in,
                                                       DevState out, int only_above, int carry)
{
    extern __shared__ double apss_lds[];
    const int R = PERSP ? p.apss_R : p.apss_Rs, SX = ATX + 2 * R, NS = SX * (ATY + 2 * R);
    double* tl = apss_lds;                                      // [KM][NS] depths
    float* nl = reinterpret_cast<float*>(tl + KM * NS);         // [3][KM][NS] normals
    int* cl = reinterpret_cast<int*>(nl + 3 * KM * NS);         // [NS] counts (0 outside the frame)
    const int tile0 = (int)xcd_block(blockIdx.x, gridDim.x);
    const int g = tile_group(tg, tile0);
    const Shape sh = group_shape(tg, g);
    in = state_at(in, tg.base[g]);
    out = state_at(out, tg.base[g]);
    const long long S = sh.S;
    const int tile = tile0 - tg.tile0[g];
    const int tiles_x = (sh.cols + ATX - 1) / ATX, tiles_y = (sh.rows + ATY - 1) / ATY;
    const int tpf = tiles_x * tiles_y;
    const int fr = tile / tpf, tr = tile % tpf;
    const int i0 = (tr / tiles_x) * ATY, j0 = (tr % tiles_x) * ATX;
    const long long fbase = (long long)fr * sh.rows * sh.cols;
    // stage the counts and every slot of the tile and its halo (without
    // waiting for the counts)
    for (int x = threadIdx.x; x < NS; x += ATX * ATY) {
        const int i2 = i0 - R + x / SX, j2 = j0 - R + x % SX;
        int c = 0;
        if (i2 >= 0 && i2 < sh.rows && j2 >= 0 && j2 < sh.cols) {
            const long long pp = fbase + (long long)i2 * sh.cols + j2;
            c = load_cnt(in.cnt, pp);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                tl[k * NS + x] = in.t[k * S + pp];
#pragma unroll
                for (int a = 0; a < 3; ++a) nl[(a * KM + k) * NS + x] = in.n[(a * KM + k) * S + pp];
            }
        }
        cl[x] = c;
    }
    __syncthreads();
    const int ty = threadIdx.x / ATX, tx = threadIdx.x % ATX;
    const int i = i0 + ty, j = j0 + tx;
    if (i >= sh.rows || j >= sh.cols) return;
    const long long pix = fbase + (long long)i * sh.cols + j;
    const int xc = (ty + R) * SX + tx + R;
    const int c = cl[xc];
    if (carry) {
        out.cnt[pix] = (uint8_t)c;
        out.b[pix] = in.b[pix];
#pragma unroll
        for (int k = 0; k < KM; ++k) out.r[k * S + pix] = in.r[k * S + pix];
    }
    if (c == 0) return;
    const bool fit = !(only_above >= 0 && c <= only_above);
    const float h = (float)p.h_apss, h2 = h * h, inv_h2 = 1.f / h2;
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const double tmax = (double)(m.T - 1);
    if constexpr (!PERSP) {
        // every live slot of the pixel against each neighbour in turn: the
        // neighbour's depth and normal are read from LDS once for all slots
        double tq[KM];
        float W[KM], Px[KM], Py[KM], Pz[KM], Nx[KM], Ny[KM], Nz[KM], PN[KM], PP[KM], nn[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            tq[k] = k < c ? tl[k * NS + xc] : 0.0;
            W[k] = Px[k] = Py[k] = Pz[k] = Nx[k] = Ny[k] = Nz[k] = PN[k] = PP[k] = nn[k] = 0.f;
        }
        if (fit) {
            for (int di = -R; di <= R; ++di) {
                const float yy = (float)di * pxy;
                for (int dj = -R; dj <= R; ++dj) {
                    // pixels whose lateral offset alone reaches h hold no neighbour
                    const float yx = (float)dj * pxy;
                    const float dl = fmaf(yx, yx, yy * yy);
                    if (!(dl < h2)) continue;
                    const int x = xc + di * SX + dj;
                    const int cc = cl[x];
#pragma unroll
                    for (int k2 = 0; k2 < KM; ++k2) {
                        if (k2 >= cc) break;
                        const double t2 = tl[k2 * NS + x];
                        const float nx = nl[(0 * KM + k2) * NS + x];
                        const float ny = nl[(1 * KM + k2) * NS + x];
                        const float nz = nl[(2 * KM + k2) * NS + x];
                        const float yn = fmaf(yx, nx, yy * ny);
#pragma unroll
                        for (int k = 0; k < KM; ++k) {
                            if (k >= c) break;
                            const float yz = (float)((t2 - tq[k]) * dz);
                            const float d2 = fmaf(yz, yz, dl);
                            if (!(d2 < h2)) continue;
                            float a = 1.f - d2 * inv_h2;
                            a = a * a;
                            const float w = a * a;
                            W[k] += w;
                            Px[k] = fmaf(w, yx, Px[k]);
                            Py[k] = fmaf(w, yy, Py[k]);
                            Pz[k] = fmaf(w, yz, Pz[k]);
                            Nx[k] = fmaf(w, nx, Nx[k]);
                            Ny[k] = fmaf(w, ny, Ny[k]);
                            Nz[k] = fmaf(w, nz, Nz[k]);
                            PN[k] = fmaf(w, fmaf(yz, nz, yn), PN[k]);
                            PP[k] = fmaf(w, d2, PP[k]);
                            nn[k] += 1.f;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k >= c) break;
            double tn = tq[k];
            float on[3] = {nl[(0 * KM + k) * NS + xc], nl[(1 * KM + k) * NS + xc], nl[(2 * KM + k) * NS + xc]};
            apss_project(fit && nn[k] >= (float)p.m_min, W[k], Px[k], Py[k], Pz[k], Nx[k], Ny[k], Nz[k], PN[k],
                         PP[k], h, h2, dz, tmax, tn, on);
            out.t[k * S + pix] = tn;
#pragma unroll
            for (int a = 0; a < 3; ++a) out.n[(a * KM + k) * S + pix] = on[a];
        }
    } else {
        double vq[3];
        float rq[3];
        ray_dir(p.persp, sh.rows, sh.cols, i, j, vq);
        for (int a = 0; a < 3; ++a) rq[a] = (float)vq[a];
        // the query's unnormalised ray uq = (persp (j - cx), persp (i - cy), 1)
        const float pa = (float)p.persp;
        const float uq[3] = {pa * (float)(j - 0.5 * (sh.cols - 1)), pa * (float)(i - 0.5 * (sh.rows - 1)), 1.f};
        const float uuq = fmaf(uq[0], uq[0], fmaf(uq[1], uq[1], 1.f));
        for (int k = 0; k < c; ++k) {
            const double tq = tl[k * NS + xc];
            const float rho = (float)(tq * dz), rho2 = 0.999f * rho * rho;   // squared range, rounded down
            float W = 0.f, Px = 0.f, Py = 0.f, Pz = 0.f, Nx = 0.f, Ny = 0.f, Nz = 0.f, PN = 0.f, PP = 0.f, nn = 0.f;
            if (fit) {
                for (int di = -R; di <= R; ++di) {
                    for (int dj = -R; dj <= R; ++dj) {
                        const int x = xc + di * SX + dj;
                        const int cc = cl[x];
                        if (cc == 0) continue;
                        // every point of this pixel's ray is at least rho_q sin(theta) from
                        // the query (theta: the angle between the two rays); skip the pixel
                        // when that reaches h
                        const float ax = pa * (float)dj, ay = pa * (float)di;   // u2 - uq = (ax, ay, 0)
                        // |uq x u2| = |uq x (u2 - uq)|
                        const float cx2 = -uq[2] * ay, cy2 = uq[2] * ax, cz2 = uq[0] * ay - uq[1] * ax;
                        const float uu2 = fmaf(uq[0] + ax, uq[0] + ax, fmaf(uq[1] + ay, uq[1] + ay, 1.f));
                        const float sin2 = (cx2 * cx2 + cy2 * cy2 + cz2 * cz2) / (uuq * uu2);
                        if (!(rho2 * sin2 < h2)) continue;
                        double v2[3];
                        ray_dir(p.persp, sh.rows, sh.cols, i + di, j + dj, v2);
                        for (int k2 = 0; k2 < cc; ++k2) {
                            const double t2 = tl[k2 * NS + x];
                            const float yx = (float)((t2 * v2[0] - tq * vq[0]) * dz);
                            const float yy = (float)((t2 * v2[1] - tq * vq[1]) * dz);
                            const float yz = (float)((t2 * v2[2] - tq * vq[2]) * dz);
                            const float d2 = fmaf(yx, yx, fmaf(yy, yy, yz * yz));
                            if (!(d2 < h2)) continue;
                            float a = 1.f - d2 * inv_h2;
                            a = a * a;
                            const float w = a * a;
                            const float nx = nl[(0 * KM + k2) * NS + x];
                            const float ny = nl[(1 * KM + k2) * NS + x];
                            const float nz = nl[(2 * KM + k2) * NS + x];
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
            }
            double tn = tq;
            float on[3] = {nl[(0 * KM + k) * NS + xc], nl[(1 * KM + k) * NS + xc], nl[(2 * KM + k) * NS + xc]};
            apss_project(fit && nn >= (float)p.m_min, W, Px, Py, Pz, Nx, Ny, Nz, PN, PP, h, h2, dz, tmax, tn, on,
                         rq);
            out.t[k * S + pix] = tn;
#pragma unroll
            for (int a = 0; a < 3; ++a) out.n[(a * KM + k) * S + pix] = on[a];
        }
    }
}

constexpr int LPA = 8;   // lanes per pixel: the window's pixels are split over them
static_assert(LPA == 8, "the lane sums below are sums over 8 lanes");

__global__ __launch_bounds__(256) void k_apss(DevModel m, DevParams p, Shape sh, DevState in, DevState out,
                                              int only_above)
{
    const long long P = sh.P, S = sh.S;
    const long long gid = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const long long pix = gid / LPA;
    const int sub = (int)(gid % LPA);
    const bool live = pix < P;
    const long long pq = live ? pix : 0;
    const int c = live ? load_cnt(in.cnt, pq) : 0;
    if (live) {
        if (sub == 0) {
            out.cnt[pix] = (uint8_t)c;
            out.b[pix] = in.b[pix];
        }
        if (sub < KM) out.r[sub * S + pix] = in.r[sub * S + pix];   // depth and normal: lane 0 below
    }
    const bool fit = live && !(only_above >= 0 && c <= only_above);
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pq / per_frame;
    const int i = (int)((pq / sh.cols) % sh.rows), j = (int)(pq % sh.cols);
    const int R = p.apss_R, side = 2 * R + 1;
    const float h = (float)p.h_apss, h2 = h * h, inv_h2 = 1.f / h2;
    const float pxy = (float)p.p_xy;
    const double dz = p.dz;
    const double tmax = (double)(m.T - 1);
    for (int k = 0; k < KM; ++k) {                  // every lane runs the slot (lane sums below)
        const bool act = fit && k < c;
        if (__ballot(live && k < c) == 0ull) break;  // no pixel of the wavefront has slot k
        const double tq = act ? in.t[k * S + pq] : 0.0;
        float W = 0.f, Px = 0.f, Py = 0.f, Pz = 0.f, Nx = 0.f, Ny = 0.f, Nz = 0.f, PN = 0.f, PP = 0.f, nn = 0.f;
        if (act) {
            for (int widx = sub; widx < side * side; widx += LPA) {
                const int i2 = i + widx / side - R, j2 = j + widx % side - R;
                if (i2 < 0 || i2 >= sh.rows || j2 < 0 || j2 >= sh.cols) continue;
                const float yy = (float)(i2 - i) * pxy, yx = (float)(j2 - j) * pxy;
                const float dl = fmaf(yx, yx, yy * yy);
                if (!(dl < h2)) continue;                  // no neighbour in this pixel
                const long long pp = (fr * sh.rows + i2) * sh.cols + j2;
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
        // sphere moments of the pixel's LPA lanes
        W = oct_sum(W);
        Px = oct_sum(Px);
        Py = oct_sum(Py);
        Pz = oct_sum(Pz);
        Nx = oct_sum(Nx);
        Ny = oct_sum(Ny);
        Nz = oct_sum(Nz);
        PN = oct_sum(PN);
        PP = oct_sum(PP);
        nn = oct_sum(nn);
        if (!live || sub != 0) continue;
        // lane 0 writes the slot: the projection when the fit succeeds, else the input
        double tn = in.t[k * S + pix];
        float on[3] = {in.n[(0 * KM + k) * S + pix], in.n[(1 * KM + k) * S + pix], in.n[(2 * KM + k) * S + pix]};
        apss_project(act && nn >= (float)p.m_min, W, Px, Py, Pz, Nx, Ny, Nz, PN, PP, h, h2, dz, tmax, tn, on);
        out.t[k * S + pix] = tn;
#pragma unroll
        for (int a = 0; a < 3; ++a) out.n[(a * KM + k) * S + pix] = on[a];
    }
}

// Reading (not in the paper): points of one pixel closer than d_merge bins in
// depth describe one surface; in depth order they merge into the
// intensity-weighted depth, summed intensity and weighted normal
// (merge_points).
// (m: only the pixels of its IRF class; d_merge in p is that class's)
__global__ __launch_bounds__(256) void k_merge(DevModel m, DevParams p, Shape sh, DevState s)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P || !in_class(m, pix)) return;
    int c = load_cnt(s.cnt, pix);
    if (c < 2) return;
    double t[KM];
    float r[KM], nx[KM], ny[KM], nz[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < c) {
            t[k] = s.t[k * P + pix];
            r[k] = s.r[k * P + pix];
            nx[k] = s.n[(0 * KM + k) * P + pix];
            ny[k] = s.n[(1 * KM + k) * P + pix];
            nz[k] = s.n[(2 * KM + k) * P + pix];
        }
    }
    merge_points(t, r, nx, ny, nz, c, p.d_merge);
    store_points(s, P, pix, t, r, nx, ny, nz, c);
}

hipError_t launch_apss_tiles(const DevModel& m, const DevParams& p, const Tiles& tg, DevState in, DevState out,
                             int only_above, bool carry, hipStream_t st)
{
    if (tg.n == 0 || tg.tile0[tg.n] == 0) return hipSuccess;
    if (p.persp > 0.0) {   // the host admits the perspective camera only where the tile fits
        const size_t lds = apss_tile_bytes(p.apss_R);
        if (lds > 65536) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_apss_tile<true>, dim3((unsigned)tg.tile0[tg.n]), dim3(ATX * ATY), lds, st, m, p, tg, in,
                           out, only_above, (int)carry);
        return hipGetLastError();
    }
    const size_t lds = apss_tile_bytes(p.apss_Rs);
    if (lds <= 65536) {
        hipLaunchKernelGGL(k_apss_tile<false>, dim3((unsigned)tg.tile0[tg.n]), dim3(ATX * ATY), lds, st, m, p, tg,
                           in, out, only_above, (int)carry);
        return hipGetLastError();
    }
    for (int g = 0; g < tg.n; ++g) {
        const Shape sh = group_shape(tg, g);
        hipLaunchKernelGGL(k_apss, dim3((unsigned)((sh.P * LPA + 255) / 256)), dim3(256), 0, st, m, p, sh,
                           state_at(in, tg.base[g]), state_at(out, tg.base[g]), only_above);
    }
    return hipGetLastError();
}

hipError_t launch_apss(const DevModel& m, const DevParams& p, const Shape& sh, DevState in, DevState out,
                       int only_above, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    return launch_apss_tiles(m, p, tiles_of(sh), in, out, only_above, true, st);
}

hipError_t launch_merge(const DevModel& m, const DevParams& p, const Shape& sh, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge, dim3((unsigned)((sh.P + 255) / 256)), dim3(256), 0, st, m, p, sh, s);
    return hipGetLastError();
}

}  // namespace rt3d

// k_init.hip -- per-pixel initialisation (Methods: initialisation processes
// each pixel independently) as a log-matched filter, then initial normals.
//
// Reading of the initialisation: photons of the (2 r_init + 1)^2 window are
// pooled; the score L(tau) = sum z q[t - tau + o], q = log((h + eps)/eps) in
// 16-bit fixed point, is exact integer arithmetic, so its argmax does not
// depend on summation order.  Peaks are taken greedily (largest score,
// smallest tau on ties), each suppressing |tau - tau*| <= w_nms, while the
// window's unclaimed photons exceed the background expectation by kappa
// standard deviations (and n_min); an accepted peak claims the unclaimed bins
// of its window (5%..95% IRF mass) and later scores use unclaimed photons
// only.  Intensity = own photons in the claimed bins minus background over
// the IRF mass there; background = own photons outside the claimed bins.
//
// Mapping: one wavefront per pixel.  The pooled photon list lives in LDS
// (dense pooled histogram built with LDS integer atomics, then compacted in
// bin order); each lane scores a contiguous run of tau with a two-pointer
// sweep over the list, and the wave reduces (score, tau).
#include "rt3d_dev.h"

namespace rt3d {

struct Peak {
    int t, a, c, w;   // depth, window [a, c], bins claimed
};

__device__ __forceinline__ int owner_of(int tb, const Peak* pk, int n)
{
    for (int j = 0; j < n; ++j)
        if (tb >= pk[j].a && tb <= pk[j].c) return j;
    return -1;
}

__device__ __forceinline__ int lower_bound_u16(const uint16_t* a, int n, int key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int)a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64) void k_init(DevModel m, DevParams p, Shape sh, const uint32_t* __restrict__ off,
                                             const uint32_t* __restrict__ ent, const float* __restrict__ gain,
                                             DevState s)
{
    extern __shared__ uint32_t smem[];
    const long long pix = blockIdx.x;
    const long long P = sh.P;
    const int lane = threadIdx.x;
    const int T = m.T, L = m.L, o = m.o;
    if (lane < KM) {
        s.t[lane * P + pix] = 0.0;
        s.r[lane * P + pix] = 0.f;
        s.n[(0 * KM + lane) * P + pix] = 0.f;
        s.n[(1 * KM + lane) * P + pix] = 0.f;
        s.n[(2 * KM + lane) * P + pix] = -1.f;
    }
    const float G = gain ? gain[pix] : 1.f;
    if (!(G > 0.f)) {
        if (lane == 0) {
            s.cnt[pix] = 0;
            s.b[pix] = (float)p.b_min;
        }
        return;
    }
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pix / per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);

    uint32_t* lz = smem;                           // [T] pooled counts of the list
    uint16_t* lt = (uint16_t*)(smem + T);          // [T] bins of the list
    uint32_t* agg = smem + T + (T + 1) / 2;        // [T] dense pooled histogram
    int nlist;
    if (p.r_init > 0) {
        for (int tb = lane; tb < T; tb += 64) agg[tb] = 0;
        __syncthreads();
        for (int i2 = i - p.r_init; i2 <= i + p.r_init; ++i2) {
            if (i2 < 0 || i2 >= sh.rows) continue;
            for (int j2 = j - p.r_init; j2 <= j + p.r_init; ++j2) {
                if (j2 < 0 || j2 >= sh.cols) continue;
                long long pp = (fr * sh.rows + i2) * sh.cols + j2;
                for (uint32_t e = off[pp] + lane; e < off[pp + 1]; e += 64) {
                    uint32_t v = ent[e];
                    if (ent_bin(v) < T) atomicAdd(&agg[ent_bin(v)], (uint32_t)ent_cnt(v));
                }
            }
        }
        __syncthreads();
        // compact the dense histogram in bin order: lane l owns bins [l*C, (l+1)*C)
        const int C = (T + 63) / 64;
        const int b0 = lane * C, b1 = min(T, b0 + C);
        uint32_t c = 0;
        for (int tb = b0; tb < b1; ++tb) c += agg[tb] != 0;
        uint32_t inc = wave_incl_scan(c);
        nlist = __shfl(inc, 63, 64);
        uint32_t pos = inc - c;
        for (int tb = b0; tb < b1; ++tb) {
            uint32_t z = agg[tb];
            if (z) {
                lt[pos] = (uint16_t)tb;
                lz[pos] = z;
                ++pos;
            }
        }
        __syncthreads();
    } else {
        const uint32_t e0 = off[pix];
        nlist = min((int)(off[pix + 1] - e0), T);
        for (int e = lane; e < nlist; e += 64) {
            uint32_t v = ent[e0 + e];
            lt[e] = (uint16_t)ent_bin(v);
            lz[e] = (uint32_t)ent_cnt(v);
        }
        __syncthreads();
    }
    long long ntot = 0;
    for (int e = lane; e < nlist; e += 64) ntot += lz[e];
    ntot = wave_sum(ntot);

    Peak pk[KM];
    int npk = 0;
    const int C = (T + 63) / 64;
    const int tau0 = lane * C, tau1 = min(T, tau0 + C);
    const double k2 = p.kappa * p.kappa;
    for (int it = 0; it < p.k_init; ++it) {
        // lane-local best over its run of tau
        long long bestv = -1;
        int bestt = 0x7fffffff;
        if (tau0 < tau1) {
            int lo = lower_bound_u16(lt, nlist, tau0 - o);
            int hi = lo;
            for (int tau = tau0; tau < tau1; ++tau) {
                const int wlo = tau - o, whi = tau - o + L - 1;
                while (lo < nlist && (int)lt[lo] < wlo) ++lo;
                if (hi < lo) hi = lo;
                while (hi < nlist && (int)lt[hi] <= whi) ++hi;
                bool sup = false;
                for (int q = 0; q < npk; ++q) sup |= abs(tau - pk[q].t) <= m.wnms;
                if (sup) continue;
                long long sc = 0;
                for (int x = lo; x < hi; ++x) {
                    int tb = lt[x];
                    const int lag = tb - tau + o;
                    if ((unsigned)lag >= (unsigned)L || owner_of(tb, pk, npk) >= 0) continue;
                    sc += (long long)lz[x] * (long long)m.q[lag];
                }
                if (sc > bestv) {
                    bestv = sc;
                    bestt = tau;
                }
            }
        }
        // wave argmax: larger score, then smaller tau
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            long long ov = __shfl_xor(bestv, d, 64);
            int ot = __shfl_xor(bestt, d, 64);
            if (ov > bestv || (ov == bestv && ot < bestt)) {
                bestv = ov;
                bestt = ot;
            }
        }
        if (bestt == 0x7fffffff) break;      // every tau suppressed
        const int a = max(0, bestt - m.wl), c = min(T - 1, bestt + m.wr);
        int win = 0;
        for (int tb = a + lane; tb <= c; tb += 64) win += owner_of(tb, pk, npk) < 0;
        win = wave_sum(win);
        long long nwin = 0;
        {
            int x0 = lower_bound_u16(lt, nlist, a);
            for (int x = x0 + lane; x < nlist; x += 64) {
                int tb = lt[x];
                if (tb > c) break;
                if (owner_of(tb, pk, npk) < 0) nwin += lz[x];
            }
        }
        nwin = wave_sum(nwin);
        const double bw = (double)ntot * (double)win / (double)T;
        const double d = (double)nwin - bw;
        const bool accept = win > 0 && nwin >= p.n_min && d >= 0.0 && d * d >= k2 * bw;
        if (!accept) break;
        pk[npk].t = bestt;
        pk[npk].a = a;
        pk[npk].c = c;
        pk[npk].w = win;
        ++npk;
    }

    // own photons: total and per claimed window
    const uint32_t e0 = off[pix], e1 = off[pix + 1];
    long long zp = 0;
    long long nown[KM] = {0, 0, 0, 0};
    for (uint32_t e = e0 + lane; e < e1; e += 64) {
        uint32_t v = ent[e];
        int z = ent_cnt(v);
        zp += z;
        int ow = owner_of(ent_bin(v), pk, npk);
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (ow == k) nown[k] += z;
    }
    zp = wave_sum(zp);
    double H[KM] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        nown[k] = wave_sum(nown[k]);
        if (k < npk) {
            double hs = 0.0;
            for (int tb = pk[k].a + lane; tb <= pk[k].c; tb += 64) {
                int idx = tb - pk[k].t + o;
                if (owner_of(tb, pk, npk) == k && idx >= 0 && idx < L) hs += m.hbar[idx];
            }
            H[k] = wave_sum(hs);
        }
    }
    if (lane != 0) return;
    long long sum_n = 0, sum_w = 0;
    for (int k = 0; k < npk; ++k) {
        sum_n += nown[k];
        sum_w += pk[k].w;
    }
    long long num = zp - sum_n;
    if (num < 0) num = 0;
    const long long den = (long long)T - sum_w;
    int kt[KM];
    float kr[KM];
    int nk = 0;
    for (int k = 0; k < npk; ++k) {
        const long long w = pk[k].w;
        const bool keep = den > 0 ? (nown[k] * den > num * w) : (nown[k] > 0);
        if (!keep || !(H[k] > 0.0)) continue;
        const double excess = den > 0 ? (double)nown[k] - (double)num * (double)w / (double)den
                                      : (double)nown[k];
        kt[nk] = pk[k].t;
        kr[nk] = (float)(excess / ((double)G * H[k]));
        ++nk;
    }
    for (int x = 1; x < nk; ++x)
        for (int y = x; y > 0 && kt[y] < kt[y - 1]; --y) {
            int tt = kt[y]; kt[y] = kt[y - 1]; kt[y - 1] = tt;
            float rr = kr[y]; kr[y] = kr[y - 1]; kr[y - 1] = rr;
        }
    if (nk > p.k_max) nk = p.k_max;
    for (int k = 0; k < nk; ++k) {
        s.t[k * P + pix] = (double)kt[k];
        s.r[k * P + pix] = kr[k];
    }
    s.cnt[pix] = (uint8_t)nk;
    const double bown = den > 0 ? (double)num / (double)den : 0.0;
    const double b0 = bown / (double)G;
    s.b[pix] = (float)(b0 > p.b_min ? b0 : p.b_min);
}

// Initial normals (reading): weighted least-squares plane Z = a + c1 X + c2 Y
// over the APSS neighbourhood in FP64, local coordinates; n = (c1, c2, -1)/|.|,
// or (0, 0, -1) with fewer than 3 neighbours or a near-singular system.
__global__ __launch_bounds__(256) void k_init_normals(DevParams p, Shape sh, DevState s)
{
    const long long P = sh.P;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = load_cnt(s.cnt, pix);
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pix / per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);
    const double h2 = p.h_apss * p.h_apss;
    const int R = p.apss_R;
    for (int k = 0; k < KM; ++k) {
        if (k >= c) break;
        const double tq = s.t[k * P + pix];
        double M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0, v0 = 0, v1 = 0, v2 = 0, W = 0;
        int nn = 0;
        for (int i2 = i - R; i2 <= i + R; ++i2) {
            if (i2 < 0 || i2 >= sh.rows) continue;
            for (int j2 = j - R; j2 <= j + R; ++j2) {
                if (j2 < 0 || j2 >= sh.cols) continue;
                const long long pp = (fr * sh.rows + i2) * sh.cols + j2;
                const int cc = load_cnt(s.cnt, pp);
                for (int k2 = 0; k2 < cc; ++k2) {
                    const double x = (j2 - j) * p.p_xy, y = (i2 - i) * p.p_xy;
                    const double z = (s.t[k2 * P + pp] - tq) * p.dz;
                    const double d2 = x * x + y * y + z * z;
                    if (!(d2 < h2)) continue;
                    double a = 1.0 - d2 / h2;
                    a = a * a;
                    const double w = a * a;
                    M00 += w; M01 += w * x; M02 += w * y;
                    M11 += w * x * x; M12 += w * x * y; M22 += w * y * y;
                    v0 += w * z; v1 += w * x * z; v2 += w * y * z;
                    W += w;
                    ++nn;
                }
            }
        }
        float nx = 0.f, ny = 0.f, nz = -1.f;
        if (nn >= 3) {
            const double det = M00 * (M11 * M22 - M12 * M12) - M01 * (M01 * M22 - M12 * M02)
                             + M02 * (M01 * M12 - M11 * M02);
            const double scale = W * W * W * h2 * h2;
            if (det > 1e-9 * scale) {
                const double d1 = M00 * (v1 * M22 - M12 * v2) - v0 * (M01 * M22 - M12 * M02)
                                + M02 * (M01 * v2 - v1 * M02);
                const double d2 = M00 * (M11 * v2 - v1 * M12) - M01 * (M01 * v2 - v1 * M02)
                                + v0 * (M01 * M12 - M11 * M02);
                const double c1 = d1 / det, c2 = d2 / det;
                const double nrm = sqrt(c1 * c1 + c2 * c2 + 1.0);
                nx = (float)(c1 / nrm);
                ny = (float)(c2 / nrm);
                nz = (float)(-1.0 / nrm);
            }
        }
        s.n[(0 * KM + k) * P + pix] = nx;
        s.n[(1 * KM + k) * P + pix] = ny;
        s.n[(2 * KM + k) * P + pix] = nz;
    }
}

size_t init_lds_bytes(int T)
{
    // lz[T] + lt[T] (uint16, padded to words) + agg[T]
    return sizeof(uint32_t) * ((size_t)T + (size_t)(T + 1) / 2 + (size_t)T);
}

hipError_t launch_init(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                       const uint32_t* ent, const float* gain, DevState s, int32_t* err, hipStream_t st)
{
    (void)err;
    if (sh.P == 0) return hipSuccess;
    size_t lds = init_lds_bytes(m.T);
    hipLaunchKernelGGL(k_init, dim3((unsigned)sh.P), dim3(64), lds, st, m, p, sh, off, ent, gain, s);
    return hipGetLastError();
}

hipError_t launch_init_normals(const DevParams& p, const Shape& sh, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_normals, dim3((unsigned)((sh.P + 255) / 256)), dim3(256), 0, st, p, sh, s);
    return hipGetLastError();
}

}  // namespace rt3d

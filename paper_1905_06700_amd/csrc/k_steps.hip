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
// Mapping: four lanes per pixel share its active entries (cost linear in
// active bins, as in the paper's Methods; consecutive lanes read consecutive
// entries) and combine their partial sums with wavefront shuffles; every lane
// keeps the pixel's <= 4 points in registers.  Depth is held in FP64 state and
// evaluated in FP32 around an integer anchor, so the IRF lookup error stays
// at FP32 rounding of the local offset whatever T is.
#include "rt3d_dev.h"

namespace rt3d {

// Lanes per pixel, LPP (a template parameter: 4 or 8): a pixel's active
// entries are split over LPP consecutive lanes (entry e + LPP i), whose
// partial sums meet in a shuffle tree.  Four lanes fill the chip at large
// batches; eight halve the entries each lane walks, which shortens one
// frame's critical path (the autotuner picks per batch shape).
template <int LPP>
constexpr int step_batch() { return 64 / LPP; }   // entries a lane loads at once

// Entries of one batch of a pixel: step_batch per lane, STEP_LIST per pixel.
constexpr int STEP_LIST = 64;

// LDS words per workgroup for the lanes' staged entries.
template <int LPP>
constexpr int step_stage_words() { return 256 * step_batch<LPP>(); }

// A lane's staging segment: slot n of lane l of a wavefront at n * 64 + l, so
// that the wavefront's writes and reads of one slot each fall on distinct banks
// whatever slot each lane is at.
template <int LPP>
__device__ __forceinline__ uint32_t* stage_segment(uint32_t* stage)
{
    return stage + (threadIdx.x / 64) * (64 * step_batch<LPP>()) + (threadIdx.x % 64);
}

// Largest point count over the wavefront (uniform).
__device__ __forceinline__ int wave_max_count(int c)
{
    if (__builtin_amdgcn_ballot_w64(c > 3)) return 4;
    if (__builtin_amdgcn_ballot_w64(c > 2)) return 3;
    if (__builtin_amdgcn_ballot_w64(c > 1)) return 2;
    if (__builtin_amdgcn_ballot_w64(c > 0)) return 1;
    return 0;
}

// Entries the buffer loads address (byte offsets below 2^31, so that an entry
// past a pixel's end can be given an offset past every record).
constexpr uint32_t STEP_BUF_ENTRIES = 1u << 29;

// One batch of SB entries per lane from eb: load, select the entries inside
// some point's support into the lane's LDS segment, evaluate them.  BUF: the
// loads are buffer loads (an entry past the pixel's end reads 0 from an
// out-of-range offset), else global loads under the same condition.
template <int LPP, int NPT, int SB, bool BUF>
__device__ __forceinline__ void step_batch_n(const DevModel& m, const float4* cr, const PixPoints& q, float bb,
                                             float invG, const uint32_t* __restrict__ ent,
                                             __amdgpu_buffer_rsrc_t rsrc, uint32_t eb, uint32_t e1, int sub,
                                             uint32_t* seg, uint32_t& zout, float& sz, float (&sh)[KM],
                                             float (&shp)[KM])
{
    const uint32_t rem = e1 - eb;
    // this lane's entries of the batch: u < nv
    const int nv = (uint32_t)sub < rem ? (int)min((rem - (uint32_t)sub + LPP - 1) / LPP, (uint32_t)SB) : 0;
    uint32_t v[SB];
    if (BUF) {
        const uint32_t b4 = (eb + (uint32_t)sub) * 4u;
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const uint32_t o4 = u < nv ? b4 : 0x80000000u;
            v[u] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rsrc, o4, u * LPP * 4, 0);
        }
    } else {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const uint32_t x = eb + sub + u * LPP;
            v[u] = x < e1 ? ent[x] : 0u;
        }
    }
    uint32_t* wp = seg;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
        const int tbo = ent_bin(v[u]) + m.o;
        bool in = false;
#pragma unroll
        for (int k = 0; k < NPT; ++k) in = in || (uint32_t)(tbo - q.a[k]) <= (uint32_t)m.L;
        in = in && u < nv;
        *wp = v[u];                                       // kept only when it lies in a support
        wp += in ? 64 : 0;
        zout += in ? 0u : (uint32_t)ent_cnt(v[u]);        // zero where not valid
    }
    if (NPT == 0) return;
    for (const uint32_t* rp = seg; rp < wp; rp += 64) {
        const uint32_t v1 = *rp;
        const int tb = ent_bin(v1);
        const float z = (float)ent_cnt(v1);
        float h[KM], hp[KM];
        float lam = bb;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            irf_eval_t(cr, m.L, m.o, tb, q.a[k], q.f[k], h[k], hp[k]);
            lam = fmaf(q.r[k], h[k], lam);
        }
        const float zl = z * invG * __builtin_amdgcn_rcpf(lam);
        sz += zl;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            sh[k] = fmaf(zl, h[k], sh[k]);
            shp[k] = fmaf(zl, hp[k], shp[k]);
        }
    }
}

// Partial sums over one pixel's entries (e0p .. e1 - 1):
// sz = sum z/lambda, sh[k] = sum z h_k/lambda, shp[k] = sum z h'_k/lambda.
// h_k is zero outside bins floor(t_k) - o .. floor(t_k) - o + L (the
// segments' domain), so an entry in none of these ranges has lambda = g b and
// only adds z / (g b) to sz; those photons are summed as integers and added
// once.  The pixel's LPP lanes load its entries in batches, entry
// eb + sub + LPP u to lane sub: the first STEP_LIST entries form one batch,
// later ones batches of STEP_LIST / 2 (a wavefront's later batches are short,
// and a batch costs its full width on every lane).  Each lane writes the
// entries of its batch that lie in some point's support to its own LDS
// segment and evaluates them itself, so the work of a wavefront is the
// largest count of such entries on one lane, whatever the spread of the
// points of its pixels.  NPT is the largest point count of the wavefront;
// points at or beyond a lane's count have r = 0 and an anchor no entry's bin
// reaches, so they neither select entries nor change lambda, and a lane's
// sums do not depend on the other pixels of its wavefront.  BUF: the entries
// are read through a buffer resource over the whole entry array (etot
// entries; 0x00020000 is the resource word of a raw 32-bit buffer on this
// architecture).
template <int LPP, int NPT, bool BUF>
__device__ __forceinline__ void accumulate_n(const DevModel& m, const float4* cr, const PixPoints& q, float bb,
                                             float invG, const uint32_t* __restrict__ ent, uint32_t etot,
                                             uint32_t e0p, uint32_t e1, int sub, uint32_t* seg, float& sz,
                                             float (&sh)[KM], float (&shp)[KM])
{
    constexpr int SB = step_batch<LPP>();
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)ent, (short)0, BUF ? (int)(etot * 4u) : 0, 0x00020000);
    uint32_t zout = 0;                                    // photons of this lane's entries outside every support
    if (e0p < e1)
        step_batch_n<LPP, NPT, SB, BUF>(m, cr, q, bb, invG, ent, rsrc, e0p, e1, sub, seg, zout, sz, sh, shp);
    for (uint32_t eb = e0p + STEP_LIST; eb < e1; eb += STEP_LIST / 2)
        step_batch_n<LPP, NPT, SB / 2, BUF>(m, cr, q, bb, invG, ent, rsrc, eb, e1, sub, seg, zout, sz, sh, shp);
    sz += (float)zout * invG * __builtin_amdgcn_rcpf(bb);
}

template <int LPP, bool BUF>
__device__ __forceinline__ void accumulate_b(const DevModel& m, const float4* cr, const PixPoints& q, float bb,
                                             float invG, const uint32_t* __restrict__ ent, uint32_t etot,
                                             uint32_t e0p, uint32_t e1, int sub, uint32_t* seg, float& sz,
                                             float (&sh)[KM], float (&shp)[KM])
{
    switch (wave_max_count(q.c)) {
    case 0: accumulate_n<LPP, 0, BUF>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp); break;
    case 1: accumulate_n<LPP, 1, BUF>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp); break;
    case 2: accumulate_n<LPP, 2, BUF>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp); break;
    case 3: accumulate_n<LPP, 3, BUF>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp); break;
    default: accumulate_n<LPP, KM, BUF>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp); break;
    }
}

// etot: the entry count of all pixels (off[P], the same on every lane).
template <int LPP>
__device__ __forceinline__ void accumulate(const DevModel& m, const float4* cr, const PixPoints& q, float bb,
                                           float G, const uint32_t* __restrict__ ent, uint32_t etot, uint32_t e0p,
                                           uint32_t e1, int sub, uint32_t* seg, float& sz, float (&sh)[KM],
                                           float (&shp)[KM])
{
    sz = 0.f;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        sh[k] = 0.f;
        shp[k] = 0.f;
    }
    const float invG = __builtin_amdgcn_rcpf(G);   // 1 / g (exact for g = 1)
    if (etot <= STEP_BUF_ENTRIES)
        accumulate_b<LPP, true>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp);
    else
        accumulate_b<LPP, false>(m, cr, q, bb, invG, ent, etot, e0p, e1, sub, seg, sz, sh, shp);
}

// Sums the partials of the LPP lanes of a pixel (every lane ends with the total).
template <int LPP>
__device__ __forceinline__ float lane_sum(float v)
{
    static_assert(LPP == 4 || LPP == 8, "the lane reductions are sums over 4 or 8 lanes");
    return LPP == 4 ? quad_sum(v) : oct_sum(v);
}

template <int LPP>
__device__ __forceinline__ void reduce_lanes(float& sz, float (&sh)[KM], float (&shp)[KM])
{
    sz = lane_sum<LPP>(sz);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        sh[k] = lane_sum<LPP>(sh[k]);
        shp[k] = lane_sum<LPP>(shp[k]);
    }
}

// S and S' of the pixel's points, each sum split over the pixel's LPP lanes
// (strided segments) and combined with shuffles; every lane ends with the
// totals.
// The piecewise cubic's table, staged in LDS by the workgroup when it has at
// most STEP_STAB_PIECES pieces (its reads come at the end of a wavefront's
// work, where nothing else waits with them).
constexpr int STEP_STAB_PIECES = 8;
constexpr int STEP_STAB_LDS = STEP_STAB_PIECES + 1 + 4 * STEP_STAB_PIECES;

__device__ __forceinline__ bool stab_staged(const DevModel& m) { return m.s_np > 0 && m.s_np <= STEP_STAB_PIECES; }

template <int LPP>
__device__ __forceinline__ void s_eval_points(const DevModel& m, const PixPoints& q, int sub, const double* stl,
                                              float (&S)[KM], float (&Sp)[KM])
{
    const bool staged = stab_staged(m);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        S[k] = 0.f;
        Sp[k] = 0.f;
        if (k < q.c) {
            if (staged) s_eval_tab(m, stl, q.t[k], S[k], Sp[k], sub, LPP);
            else s_eval_tab(m, m.s_tab, q.t[k], S[k], Sp[k], sub, LPP);
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        S[k] = lane_sum<LPP>(S[k]);
        Sp[k] = lane_sum<LPP>(Sp[k]);
    }
}

// The IRF's Catmull-Rom segments for the entry loop: staged in the
// workgroup's LDS when they fit (TLDS), else read from global memory.
constexpr int STEP_CR_LDS = 256;

// STAB: the kernel evaluates S and S' (the table of the piecewise cubic too).
template <bool TLDS, bool STAB = true>
__device__ __forceinline__ const float4* stage_segments(const DevModel& m, float4* crl, double* stl)
{
    if (STAB && stab_staged(m))
        for (int i = threadIdx.x; i < 5 * m.s_np + 1; i += blockDim.x) stl[i] = m.s_tab[i];
    if (TLDS)
        for (int i = threadIdx.x; i <= m.L; i += blockDim.x) crl[i] = m.cr[i];
    __syncthreads();
    return TLDS ? crl : m.cr;
}

// Common prologue: the pixel of this lane, its points and its entry range.
struct Lane {
    long long pix;
    int sub;
    bool member;       // a pixel of the launch's IRF class (every pixel with one IRF)
    bool live;
    float G;
    PixPoints q;
    uint32_t e0, e1;   // the pixel's entries
    uint32_t etot;     // entries of all pixels (the same on every lane)
};

template <int LPP>
__device__ __forceinline__ Lane lane_setup(const DevModel& m, const DevState& s, long long P,
                                           const uint32_t* __restrict__ off, const float* __restrict__ gain,
                                           bool need_points)
{
    Lane L;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    L.sub = (int)(gid % LPP);
    if (m.lst) {   // the pixels of the launch's IRF class, from its list
        const uint32_t b0 = m.lst_meta[m.cls_id], b1 = m.lst_meta[m.cls_id + 1];
        const long long idx = gid / LPP;
        L.member = idx < (long long)(b1 - b0);
        L.pix = L.member ? (long long)m.lst[b0 + idx] : 0;
    } else {
        L.pix = gid / LPP;
        L.member = L.pix < P && in_class(m, L.pix);
    }
    L.live = L.member;
    const long long pp = L.live ? L.pix : 0;
    const uint32_t e0 = off[pp], e1 = off[pp + 1];
    L.etot = __builtin_amdgcn_readfirstlane(off[P]);
    L.G = L.live ? gain_at(gain, pp) : 0.f;
    load_points(s, P, pp, L.q);
    if (!L.live) L.q.c = 0;
    const bool work = L.live && L.G > 0.f && (!need_points || L.q.c > 0);
    L.e0 = work ? e0 : 0;
    L.e1 = work ? e1 : 0;
    L.live = work;
    return L;
}

// Seven workgroups per CU (at most 72 VGPRs; the few values the compiler then
// keeps in scratch are written before the entry loop and read after it).
template <int LPP, bool TLDS>
__global__ __launch_bounds__(256, 7) void k_depth_step(DevModel m, DevParams p, Shape sh,
                                                    const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ ent,
                                                    const float* __restrict__ gain, DevState s)
{
    __shared__ uint32_t stage[step_stage_words<LPP>()];
    __shared__ float4 crl[TLDS ? STEP_CR_LDS : 1];
    __shared__ double stl[STEP_STAB_LDS];
    const long long P = sh.P;
    const Lane L = lane_setup<LPP>(m, s, P, off, gain, true);    // its loads stay in flight across the staging
    const float4* cr = stage_segments<TLDS>(m, crl, stl);
    uint32_t* seg = stage_segment<LPP>(stage);
    float sz, shh[KM], shp[KM];
    accumulate<LPP>(m, cr, L.q, L.live ? s.b[L.pix] : 1.f, L.live ? L.G : 1.f, ent, L.etot, L.e0, L.e1, L.sub, seg, sz, shh, shp);
    reduce_lanes<LPP>(sz, shh, shp);
    // S' after the entries: nothing of it stays live across the entry loop
    float Sv[KM], Spv[KM];
    s_eval_points<LPP>(m, L.q, L.sub, stl, Sv, Spv);
    if (!L.live || L.sub != 0) return;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < L.q.c && L.q.r[k] > 0.f) s.t[k * P + L.pix] = depth_next(m, p, L.q.t[k], Spv[k], shp[k]);
}

// The in-pixel merge ahead of the intensity step: every lane of the pixel
// merges its copy of the points (merge_points); lane 0 writes the merged
// state.  Pixels whose points are in depth order and at least d_merge apart
// (almost all) keep their state untouched.
__device__ __forceinline__ void merge_lane(const DevState& s, long long P, const DevParams& p, long long pix,
                                           int sub, PixPoints& q)
{
    const int c0 = q.c;
    bool need = false;
#pragma unroll
    for (int k = 1; k < KM; ++k)
        if (k < c0 && (q.t[k] < q.t[k - 1] || q.t[k] - q.t[k - 1] < p.d_merge)) need = true;
    if (!need) return;
    double t[KM];
    float r[KM], nx[KM], ny[KM], nz[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        t[k] = q.t[k];
        r[k] = q.r[k];
        nx[k] = s.n[(0 * KM + k) * P + pix];
        ny[k] = s.n[(1 * KM + k) * P + pix];
        nz[k] = s.n[(2 * KM + k) * P + pix];
    }
    int c = c0;
    merge_points(t, r, nx, ny, nz, c, p.d_merge);
    if (sub == 0) store_points(s, P, pix, t, r, nx, ny, nz, c);
    q.c = c;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const bool on = k < c;
        const double tk = on ? t[k] : 0.0;
        const double fl = floor(tk);
        q.t[k] = tk;
        q.a[k] = on ? (int)fl : PT_ABSENT;
        q.f[k] = (float)(tk - fl);
        q.r[k] = on ? r[k] : 0.f;
    }
}

// MERGE: the in-pixel merge runs first (the loop's order: merge, then the
// intensity step on the merged points).
template <int LPP, bool MERGE, bool TLDS>
__global__ __launch_bounds__(256, 7) void k_intensity_step(DevModel m, DevParams p, Shape sh,
                                                        const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ ent,
                                                        const float* __restrict__ gain, DevState s)
{
    __shared__ uint32_t stage[step_stage_words<LPP>()];
    __shared__ float4 crl[TLDS ? STEP_CR_LDS : 1];
    __shared__ double stl[STEP_STAB_LDS];
    const long long P = sh.P;
    Lane L = lane_setup<LPP>(m, s, P, off, gain, true);          // its loads stay in flight across the staging
    const float4* cr = stage_segments<TLDS>(m, crl, stl);
    uint32_t* seg = stage_segment<LPP>(stage);
    if (MERGE && L.member) merge_lane(s, P, p, L.pix, L.sub, L.q);
    float sz, shh[KM], shp[KM];
    accumulate<LPP>(m, cr, L.q, L.live ? s.b[L.pix] : 1.f, L.live ? L.G : 1.f, ent, L.etot, L.e0, L.e1, L.sub, seg, sz, shh, shp);
    reduce_lanes<LPP>(sz, shh, shp);
    float Sv[KM], Spv[KM];
    s_eval_points<LPP>(m, L.q, L.sub, stl, Sv, Spv);
    if (!L.live || L.sub != 0) return;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < L.q.c && Sv[k] > 0.f) s.r[k * P + L.pix] = intensity_next(p, L.q.r[k], Sv[k], shh[k]);
}

// The background step writes the new b to bdst (the state's own b, or a
// second buffer the background filter reads); dead pixels keep their b.
template <int LPP, bool TLDS>
__global__ __launch_bounds__(256) void k_bg_step(DevModel m, DevParams p, Shape sh,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ ent,
                                                 const float* __restrict__ gain, DevState s, float* bdst)
{
    __shared__ uint32_t stage[step_stage_words<LPP>()];
    __shared__ float4 crl[TLDS ? STEP_CR_LDS : 1];
    __shared__ double stl[STEP_STAB_LDS];
    const long long P = sh.P;
    const Lane L = lane_setup<LPP>(m, s, P, off, gain, false);   // its loads stay in flight across the staging
    const float4* cr = stage_segments<TLDS, false>(m, crl, stl);
    uint32_t* seg = stage_segment<LPP>(stage);
    const float braw = L.pix < P ? s.b[L.pix] : 1.f;
    const float bb = L.live ? braw : 1.f;
    float sz, shh[KM], shp[KM];
    accumulate<LPP>(m, cr, L.q, bb, L.live ? L.G : 1.f, ent, L.etot, L.e0, L.e1, L.sub, seg, sz, shh, shp);
    reduce_lanes<LPP>(sz, shh, shp);
    if (!L.member || L.sub != 0) return;
    if (!L.live) {
        bdst[L.pix] = braw;
        return;
    }
    bdst[L.pix] = background_next(m, p, bb, sz);
}

template <int LPP, bool TLDS>
__global__ __launch_bounds__(256) void k_gradients(DevModel m, Shape sh, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ ent,
                                                   const float* __restrict__ gain, DevState s,
                                                   float* __restrict__ gt, float* __restrict__ gr,
                                                   float* __restrict__ gb)
{
    __shared__ uint32_t stage[step_stage_words<LPP>()];
    __shared__ float4 crl[TLDS ? STEP_CR_LDS : 1];
    __shared__ double stl[STEP_STAB_LDS];
    const long long P = sh.P;
    const Lane L = lane_setup<LPP>(m, s, P, off, gain, false);   // its loads stay in flight across the staging
    const float4* cr = stage_segments<TLDS>(m, crl, stl);
    uint32_t* seg = stage_segment<LPP>(stage);
    float sz, shh[KM], shp[KM];
    accumulate<LPP>(m, cr, L.q, L.live ? s.b[L.pix] : 1.f, L.live ? L.G : 1.f, ent, L.etot, L.e0, L.e1, L.sub, seg, sz, shh, shp);
    reduce_lanes<LPP>(sz, shh, shp);
    float Sv[KM], Spv[KM];
    s_eval_points<LPP>(m, L.q, L.sub, stl, Sv, Spv);
    if (!L.member || L.sub != 0) return;
    const float G = L.G;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        float vt = 0.f, vr = 0.f;
        if (k < L.q.c && G > 0.f) {
            vt = G * L.q.r[k] * (Spv[k] + shp[k]);
            vr = G * (Sv[k] - shh[k]);
        }
        gt[k * P + L.pix] = vt;
        gr[k * P + L.pix] = vr;
    }
    gb[L.pix] = G > 0.f ? G * ((float)m.T - sz) : 0.f;
}

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Per-class pixel lists (per-pixel IRFs).  meta[0 .. n] holds each class's
// first list position (meta[n] = P), meta[RT3D_MAX_IRFS + 1 + k] the class's
// cursor.  Each wavefront takes 64 consecutive pixels and appends the pixels
// of every class in ascending order (a ballot rank), so list chunks stay
// contiguous in memory; chunks follow in the order the wavefronts reach the
// cursor, which no per-pixel step depends on.
constexpr int CLASS_CUR = RT3D_MAX_IRFS + 1;

__device__ __forceinline__ int class_of(const uint8_t* cls, long long pix, long long P, int n)
{
    if (pix >= P) return -1;
    const int k = cls[pix];
    return k < n ? k : 0;
}

__global__ void k_class_zero(uint32_t* meta)
{
    if (threadIdx.x < CLASS_META) meta[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_class_count(const uint8_t* __restrict__ cls, long long P, int n,
                                                     uint32_t* meta)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = class_of(cls, pix, P, n);
    for (int c = 0; c < n; ++c) {
        const unsigned long long mask = __ballot(k == c);
        if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&meta[CLASS_CUR + c], (uint32_t)__popcll(mask));
    }
}

__global__ void k_class_base(int n, uint32_t* meta)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int c = 0; c < n; ++c) {
        const uint32_t cnt = meta[CLASS_CUR + c];
        meta[c] = acc;
        meta[CLASS_CUR + c] = acc;
        acc += cnt;
    }
    meta[n] = acc;
}

__global__ __launch_bounds__(256) void k_class_scatter(const uint8_t* __restrict__ cls, long long P, int n,
                                                       uint32_t* meta, uint32_t* __restrict__ list)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = class_of(cls, pix, P, n);
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int c = 0; c < n; ++c) {
        const unsigned long long mask = __ballot(k == c);
        if (!mask) continue;
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(&meta[CLASS_CUR + c], (uint32_t)__popcll(mask));
        b = (uint32_t)__shfl((int)b, 0, 64);
        if (k == c) list[b + (uint32_t)__popcll(mask & below)] = (uint32_t)pix;
    }
}

hipError_t launch_class_lists(const uint8_t* cls, long long P, int n, uint32_t* list, uint32_t* meta,
                              hipStream_t st)
{
    if (n < 1 || n > RT3D_MAX_IRFS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_class_zero, dim3(1), dim3(64), 0, st, meta);
    if (P > 0) hipLaunchKernelGGL(k_class_count, dim3(blocks_for(P, 256)), dim3(256), 0, st, cls, P, n, meta);
    hipLaunchKernelGGL(k_class_base, dim3(1), dim3(64), 0, st, n, meta);
    if (P > 0) hipLaunchKernelGGL(k_class_scatter, dim3(blocks_for(P, 256)), dim3(256), 0, st, cls, P, n, meta, list);
    return hipGetLastError();
}

static inline bool segments_fit(const DevModel& m) { return m.L + 1 <= STEP_CR_LDS; }

// The kernels for lanes-per-pixel p.lpp (4 or 8) and the segment staging.
template <int LPP>
static hipError_t depth_step_lpp(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                                 const uint32_t* ent, const float* gain, DevState s, hipStream_t st)
{
    const dim3 g(blocks_for(sh.P * LPP, 256)), b(256);
    if (segments_fit(m)) hipLaunchKernelGGL((k_depth_step<LPP, true>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    else hipLaunchKernelGGL((k_depth_step<LPP, false>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    return hipGetLastError();
}

template <int LPP>
static hipError_t intensity_step_lpp(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                                     const uint32_t* ent, const float* gain, DevState s, bool merge, hipStream_t st)
{
    const dim3 g(blocks_for(sh.P * LPP, 256)), b(256);
    const bool tl = segments_fit(m);
    if (merge && tl) hipLaunchKernelGGL((k_intensity_step<LPP, true, true>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    else if (merge) hipLaunchKernelGGL((k_intensity_step<LPP, true, false>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    else if (tl) hipLaunchKernelGGL((k_intensity_step<LPP, false, true>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    else hipLaunchKernelGGL((k_intensity_step<LPP, false, false>), g, b, 0, st, m, p, sh, off, ent, gain, s);
    return hipGetLastError();
}

template <int LPP>
static hipError_t bg_step_lpp(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                              const uint32_t* ent, const float* gain, DevState s, float* dst, hipStream_t st)
{
    const dim3 g(blocks_for(sh.P * LPP, 256)), b(256);
    if (segments_fit(m)) hipLaunchKernelGGL((k_bg_step<LPP, true>), g, b, 0, st, m, p, sh, off, ent, gain, s, dst);
    else hipLaunchKernelGGL((k_bg_step<LPP, false>), g, b, 0, st, m, p, sh, off, ent, gain, s, dst);
    return hipGetLastError();
}

hipError_t launch_depth_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                             const uint32_t* ent, const float* gain, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    return p.lpp == 8 ? depth_step_lpp<8>(m, p, sh, off, ent, gain, s, st)
                      : depth_step_lpp<4>(m, p, sh, off, ent, gain, s, st);
}

hipError_t launch_intensity_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                                 const uint32_t* ent, const float* gain, DevState s, bool merge, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    return p.lpp == 8 ? intensity_step_lpp<8>(m, p, sh, off, ent, gain, s, merge, st)
                      : intensity_step_lpp<4>(m, p, sh, off, ent, gain, s, merge, st);
}

hipError_t launch_bg_step(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                          const uint32_t* ent, const float* gain, DevState s, float* bdst, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    float* dst = bdst ? bdst : s.b;
    return p.lpp == 8 ? bg_step_lpp<8>(m, p, sh, off, ent, gain, s, dst, st)
                      : bg_step_lpp<4>(m, p, sh, off, ent, gain, s, dst, st);
}

hipError_t launch_gradients(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                            const uint32_t* ent, const float* gain, DevState s, float* gt, float* gr, float* gb,
                            hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    const bool tl = segments_fit(m);
    if (p.lpp == 8) {
        const dim3 g(blocks_for(sh.P * 8, 256)), b(256);
        if (tl) hipLaunchKernelGGL((k_gradients<8, true>), g, b, 0, st, m, sh, off, ent, gain, s, gt, gr, gb);
        else hipLaunchKernelGGL((k_gradients<8, false>), g, b, 0, st, m, sh, off, ent, gain, s, gt, gr, gb);
    } else {
        const dim3 g(blocks_for(sh.P * 4, 256)), b(256);
        if (tl) hipLaunchKernelGGL((k_gradients<4, true>), g, b, 0, st, m, sh, off, ent, gain, s, gt, gr, gb);
        else hipLaunchKernelGGL((k_gradients<4, false>), g, b, 0, st, m, sh, off, ent, gain, s, gt, gr, gb);
    }
    return hipGetLastError();
}

}  // namespace rt3d

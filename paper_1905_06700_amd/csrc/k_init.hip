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
// Mapping: one wavefront per pixel, four pixels per workgroup.  The window's
// rows are contiguous ranges of the photon lists (pixel-major CSR), so the
// pooled photons are (2 r_init + 1) ranges.  The argmax over tau is an exact
// branch and bound over blocks of 64 consecutive tau (one tau per lane): an
// upper bound of every block's best score, sum over pooled photons of z *
// max q over the lags the block can see, is scattered into LDS with integer
// atomics; blocks are then scored exactly in decreasing bound order until no
// remaining bound can beat (or tie at a smaller tau) the best score found.
// The bound only counts photons, so it stays valid after photons are claimed.
// Only a few blocks per pixel are ever scored exactly, so the cost follows the
// active bins, not T.
//
// When the pooled photons fit (INIT_ELDS entries, T <= INIT_SB x INIT_NB_LDS)
// and the weights are staged in LDS, the photons are read once into registers
// and staged in LDS bucketed by 64-bin block; the bounds are kept per
// sub-block of INIT_SB tau (tighter, so fewer 64-tau blocks are scored) from a
// sliding-maximum weight table; each lane keeps the bound and cached best of
// the blocks lane and lane + 64; after an accepted peak only the blocks that
// peak changes (tau that can see its claimed bins or fall under its
// suppression) are scored again.  This path also needs the pixel's photon
// total times the largest weight to fit 32 bits: every score and bound then
// does, and the search runs on 32-bit integers (24-bit multiply-adds, exact
// here).  Pixels outside these limits read their photons from HBM and score
// every round afresh with 64-bit sums.
#include "rt3d_dev.h"

namespace rt3d {

// Accepted peaks of one pixel, held in registers (every index below is a
// compile-time constant after unrolling, so nothing spills to scratch).
struct Peaks {
    int t[KM], a[KM], c[KM], w[KM];
    int n;

    // first accepted peak whose window [a, c] holds bin tb, or -1
    __device__ __forceinline__ int owner(int tb) const
    {
        int ow = -1;
#pragma unroll
        for (int j = KM - 1; j >= 0; --j)
            if (j < n && tb >= a[j] && tb <= c[j]) ow = j;
        return ow;
    }

    __device__ __forceinline__ bool suppressed(int tau, int wnms) const
    {
        bool sup = false;
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < n && abs(tau - t[j]) <= wnms) sup = true;
        return sup;
    }

    // any accepted peak's suppression reaching tau in [lo, hi] (wave-uniform)
    __device__ __forceinline__ bool suppresses_any(int lo, int hi, int wnms) const
    {
        bool any = false;
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < n && t[j] - wnms <= hi && t[j] + wnms >= lo) any = true;
        return any;
    }

    // (wave-uniform values: kept in scalar registers)
    __device__ __forceinline__ void push(int tt, int aa, int cc, int ww)
    {
        tt = __builtin_amdgcn_readfirstlane(tt);
        aa = __builtin_amdgcn_readfirstlane(aa);
        cc = __builtin_amdgcn_readfirstlane(cc);
        ww = __builtin_amdgcn_readfirstlane(ww);
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j == n) {
                t[j] = tt;
                a[j] = aa;
                c[j] = cc;
                w[j] = ww;
            }
        ++n;
    }
};

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// max q[lo..hi] from the range-maximum table qst (level l: max of 2^l
// consecutive weights; lo <= hi, both in [0, L)).
__device__ __forceinline__ int q_range_max(const int* qst, int L, int lo, int hi)
{
    const int len = hi - lo + 1;
    const int l = 31 - __clz(len);
    const int a = qst[l * L + lo], b = qst[l * L + hi - (1 << l) + 1];
    return a > b ? a : b;
}

__device__ __forceinline__ int popc_ballot(bool x) { return __popcll(__ballot(x)); }

constexpr int INIT_WAVES = 4;
constexpr int INIT_ELDS = 608;    // pooled entries a wavefront scores from LDS (held in registers)
constexpr int INIT_EPL = (INIT_ELDS + 63) / 64;   // pooled entries per lane
// Pixels whose pool is larger, up to INIT_WIDE_ELDS entries, are listed and
// scored from LDS by a second kernel that stages their photons in passes over
// HBM; larger pools take the HBM path.
constexpr int INIT_WIDE_ELDS = 1536;
constexpr unsigned INIT_WIDE_GRID = 2048;

// The list of those pixels: INIT_LIST_SEGS counters INIT_LIST_STRIDE words
// apart (separate cache lines, so that appends from many wavefronts do not
// queue on one address), then one segment of init_list_cap(P) pixels per
// counter; workgroup b of the main kernel appends to segment b mod
// INIT_LIST_SEGS, which holds at most init_list_cap(P) of its pixels.
constexpr int INIT_LIST_SEGS = 64;      // one per lane of the wide kernel's segment scan
constexpr int INIT_LIST_STRIDE = 64;
constexpr size_t INIT_LIST_HDR = (size_t)INIT_LIST_SEGS * INIT_LIST_STRIDE;

__host__ __device__ inline size_t init_list_cap(long long P)
{
    const long long nblk = (P + INIT_WAVES - 1) / INIT_WAVES;
    return (size_t)((nblk + INIT_LIST_SEGS - 1) / INIT_LIST_SEGS) * INIT_WAVES;
}
constexpr int INIT_QLDS = 4096;   // IRF weight tables (ints) up to this size are staged in LDS
constexpr int INIT_QPAD = 96;     // zero weights on either side of the staged IRF weights (at least 94)
constexpr int INIT_BWS = 5;       // the LDS path buckets photons by 2^INIT_BWS bins
constexpr int NO_TAU = 0x7fffffff;

// Width (tau) of the sub-blocks the LDS path bounds, and the number of
// sub-blocks up to which it keeps their tables (at most two 64-tau blocks per
// lane).  Narrow sub-blocks give tight bounds (the largest weight over 8
// lags rather than 16 roughly halves the blocks scored on head-shaped
// scenes) at the price of more bound terms per photon.
constexpr int INIT_SB = 8;
constexpr int INIT_SB2 = 2 * INIT_SB;   // the bins of one pair of sub-blocks
constexpr int INIT_NB_LDS = 1024;
static_assert(INIT_NB_LDS * INIT_SB <= 128 * 64, "two blocks per lane");
static_assert((INIT_SB & (INIT_SB - 1)) == 0 && 64 % INIT_SB == 0, "sub-blocks tile a block");

// The LDS path adds a photon to the bounds of the sub-blocks in pairs (one
// 64-bit LDS atomic per two sub-blocks): for a photon at bin t, with
// t + o = 2 SB h + r (0 <= r < 2 SB, SB = INIT_SB), the pairs cover
// sub-blocks 2h - 2 np + 2 .. 2h + 1, which hold every sub-block whose tau
// can see t.  The pair count np = ceil((ceil((L - 1) / SB) + 2) / 2); the
// bounds carry 2 np - 2 guard entries in front (indices below 0) and reach
// index 2 floor((T - 1 + o) / (2 SB)) + 1 at the back.
inline __host__ __device__ int init_np(int L) { return ((((L - 1) + INIT_SB - 1) / INIT_SB) + 3) >> 1; }
inline __host__ __device__ size_t init_bound_words(int T, int L, int o)
{
    return (size_t)init_np(L) + (size_t)(T - 1 + o) / INIT_SB2;
}

// 8-byte LDS words of one wavefront: either the LDS path's sub-block bounds
// (with their guards), bucketed photons and bucket ends, or the HBM path's
// per-pixel photon ranges and block bounds.  (The areas are sized so that
// seven four-wavefront workgroups of the head-shaped scenes' init, 4613 bins
// and a 137-bin IRF, fit one compute unit's LDS.)
inline __host__ __device__ size_t init_wave_words(int T, int L, int o, int r_init, size_t elds = INIT_ELDS)
{
    const size_t nb = (size_t)(T + 63) / 64, nbs = (size_t)(T + INIT_SB - 1) / INIT_SB;
    const size_t side = 2 * (size_t)r_init + 1;
    const size_t nk = ((size_t)T + (1u << INIT_BWS) - 1) >> INIT_BWS;
    const size_t staged = nbs <= INIT_NB_LDS ? init_bound_words(T, L, o) + (elds + 1) / 2 + (nk + 3) / 4 : 0;
    const size_t hbm = side * side + nb;
    return hbm > staged ? hbm : staged;
}

// Ints of the staged weights (with their zero padding), and of the sliding
// maximum table: Mz[SB + x] = M[x] = max q[x - SB + 1 .. x] (q = 0 outside
// [0, L)), with SB zeros in front and zeros past x = L + SB - 2 up to the
// last entry a photon's pairs read.
inline __host__ __device__ size_t q_staged_ints(int L) { return (size_t)L + 2 * INIT_QPAD; }
inline __host__ __device__ size_t q_window_ints(int L) { return INIT_SB2 * (size_t)init_np(L) + INIT_SB; }

// Largest sub-block bound of block b.
__device__ __forceinline__ uint32_t block_bound(const uint32_t* bnd, int nbs, int b)
{
    uint32_t mx = 0;
#pragma unroll
    for (int c = 0; c < 64 / INIT_SB; ++c) {
        const int sb = b * (64 / INIT_SB) + c;
        if (sb < nbs) mx = max(mx, bnd[sb]);
    }
    return mx;
}

// Adds to the sub-block bounds (or, with SUB, takes away) the terms of a
// photon of count z at bin t, x = t + o: sub-block sb gains z x M[x - SB sb].
// Pair j of the photon's pairs (counted from the back) holds sub-blocks
// 2h - 2j and 2h - 2j + 1 (x = 2 SB h + r) and gains z x M[r + 2 SB j] and
// z x M[r + 2 SB j - SB] in its low and high words; every other sub-block of
// the pairs gets a zero weight (its lag lies outside M).  bnd2: the bounds as
// 64-bit words from the first guard entry.  A bound is an exact sum below
// 2^32, and a photon's term is part of it while it is taken away, so the low
// word never carries into (or borrows from) the high one.
template <bool SUB>
__device__ __forceinline__ void bound_photon(unsigned long long* bnd2, const int* Mz, int np, int x, uint32_t z)
{
    const int h = x / INIT_SB2, r = x % INIT_SB2;           // x >= 0
    const int* Mb = Mz + r;
    unsigned long long* bp = bnd2 + h + np - 1;
    auto term = [z](int hiw, int low) {
        const unsigned long long v = ((unsigned long long)(uint32_t)__umul24(z, (uint32_t)hiw) << 32) |
                                     (uint32_t)__umul24(z, (uint32_t)low);
        return SUB ? 0ull - v : v;
    };
    // four pairs at a time: their weight reads in flight together
    int j = 0;
    for (; j + 4 <= np; j += 4, Mb += 4 * INIT_SB2, bp -= 4) {
        int w0[4], w1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w0[k] = Mb[k * INIT_SB2];
            w1[k] = Mb[k * INIT_SB2 + INIT_SB];
        }
        unsigned long long* b3 = bp - 3;          // (ascending offsets from the lowest word)
#pragma unroll
        for (int k = 0; k < 4; ++k) atomicAdd(b3 + (3 - k), term(w0[k], w1[k]));
    }
    for (; j < np; ++j, Mb += INIT_SB2, --bp) atomicAdd(bp, term(Mb[0], Mb[INIT_SB]));
}

// Whole-wavefront maximum / minimum on the VALU: DPP quad permutations, row
// shifts by 4 and 8, then row broadcasts of lanes 15 and 31; lane 63 ends with
// the result, which every lane reads.  Lanes without a DPP source contribute
// the identity (0 for the maximum of unsigned keys, all ones for the minimum).
// Every lane must be active.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v, unsigned identity)
{
    return (unsigned)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ unsigned long long max_step_u64(unsigned long long v)
{
    const unsigned long long o = ((unsigned long long)dpp_u32<CTRL>((unsigned)(v >> 32), 0u) << 32) |
                                 dpp_u32<CTRL>((unsigned)v, 0u);
    return o > v ? o : v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    v = max_step_u64<0xB1>(v);
    v = max_step_u64<0x4E>(v);
    v = max_step_u64<0x114>(v);
    v = max_step_u64<0x118>(v);
    v = max_step_u64<0x142>(v);
    v = max_step_u64<0x143>(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ unsigned max_step_u32(unsigned v)
{
    const unsigned o = dpp_u32<CTRL>(v, 0u);
    return o > v ? o : v;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max_step_u32<0xB1>(v);
    v = max_step_u32<0x4E>(v);
    v = max_step_u32<0x114>(v);
    v = max_step_u32<0x118>(v);
    v = max_step_u32<0x142>(v);
    v = max_step_u32<0x143>(v);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

template <int CTRL>
__device__ __forceinline__ unsigned min_step_u32(unsigned v)
{
    const unsigned o = dpp_u32<CTRL>(v, 0xffffffffu);
    return o < v ? o : v;
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v)
{
    v = min_step_u32<0xB1>(v);
    v = min_step_u32<0x4E>(v);
    v = min_step_u32<0x114>(v);
    v = min_step_u32<0x118>(v);
    v = min_step_u32<0x142>(v);
    v = min_step_u32<0x143>(v);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// acc + z q on the VALU as one 24-bit multiply-add, z from a scalar register
// (exact for z, q < 2^24 and a result below 2^32).
__device__ __forceinline__ uint32_t mad_u24(uint32_t z, uint32_t q, uint32_t acc)
{
    asm("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(acc) : "s"(z), "v"(q));
    return acc;
}

// Bucket cursors (then ends), two 16-bit values per 32-bit LDS word: a bucket
// holds at most INIT_WIDE_ELDS photons, so no half carries into the other.
struct Bend16 {
    uint32_t* w;
    __device__ __forceinline__ int get(int b) const { return (int)((w[b >> 1] >> ((b & 1) << 4)) & 0xffffu); }
    __device__ __forceinline__ void add1(int b) const { atomicAdd(&w[b >> 1], 1u << ((b & 1) << 4)); }
    __device__ __forceinline__ int fetch_inc(int b) const
    {
        return (int)((atomicAdd(&w[b >> 1], 1u << ((b & 1) << 4)) >> ((b & 1) << 4)) & 0xffffu);
    }
};

// Exact scores of block bb's 64 tau (one per lane): L(tau) = sum of
// z q[t - tau + o] over the pooled photons in the window [wlo, whi] the block
// can see (photons in claimed bins have had their count set to zero).  The
// photons are bucketed by 2^INIT_BWS bins in LDS (bucket b ends at bend.get(b),
// nk buckets); the window's buckets are read 64 photons at a time and each
// photon is broadcast from the lane that loaded it, four at a time so that
// their weight lookups overlap.  qs holds the weights with INIT_QPAD zeros on
// either side; the window's buckets hold bins within 2^INIT_BWS - 1 of it
// (photons with bins >= T were staged as zero counts at the last bucket's
// last bin), so every lag lies in [-63 - 31, L + 62 + 31] and indexes the
// padded table without a clamp.
__device__ __forceinline__ uint32_t score_block(const uint32_t* E, const Bend16 bend, int nk, int bb, const int* qs,
                                                int L, int o)
{
    const int lane = threadIdx.x & 63;
    const int lo = INIT_QPAD + o - ((bb << 6) + lane);    // qs index of bin 0 for this lane's tau
    const int wlo = (bb << 6) - o, whi = (bb << 6) + 63 - o + L - 1;
    uint32_t sc = 0;
    if (whi < 0) return sc;
    const int b0 = max(0, wlo) >> INIT_BWS, b1 = min(nk - 1, whi >> INIT_BWS);
    const int x0 = __builtin_amdgcn_readfirstlane(b0 > 0 ? bend.get(b0 - 1) : 0);
    const int x1 = __builtin_amdgcn_readfirstlane(bend.get(b1));
    for (int c0 = x0; c0 < x1; c0 += 64) {
        const int x = c0 + lane;
        const int vv = x < x1 ? (int)E[x] : 0;
        const int cnt = min(64, x1 - c0);
        int k = 0;
        for (; k + 4 <= cnt; k += 4) {
            uint32_t v[4];
            int q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = (uint32_t)__builtin_amdgcn_readlane(vv, k + u);
                q[u] = qs[lo + ent_bin(v[u])];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) sc = mad_u24((uint32_t)ent_cnt(v[u]), (uint32_t)q[u], sc);
        }
        for (; k < cnt; ++k) {
            const uint32_t v = (uint32_t)__builtin_amdgcn_readlane(vv, k);
            sc = mad_u24((uint32_t)ent_cnt(v), (uint32_t)qs[lo + ent_bin(v)], sc);
        }
    }
    return sc;
}

// Branch-and-bound search of the LDS path for the pooled photons pe (entries
// lane + 64 u < total; bucket cursors in bend hold each bucket's start), or,
// with STAGED, for photons the caller has already bucketed into E (bend then
// holds the bucket ends) and added to the bounds bnd.  The
// caller has checked that ntot x the largest weight fits 32 bits and the
// weights 24 bits: every bound and score is then an exact 32-bit sum of exact
// 24-bit products.  On return pk holds the accepted peaks.
template <bool STAGED>
__device__ __forceinline__ void lds_search(const DevModel& m, const DevParams& p, int T, int L, int o, int nb,
                                           int nbs, int nk, const uint32_t (&pe)[INIT_EPL], int total, long long ntot,
                                           const int* qs, const int* Mz, unsigned long long* bnd2, int np,
                                           uint32_t* bnd, uint32_t* E, const Bend16 bend, Peaks& pk)
{
    const int lane = threadIdx.x & 63;
    // stage the photons bucketed by 2^INIT_BWS bins; bins >= T become zero
    // counts at the last bucket's last bin
#pragma unroll
    for (int u = 0; u < INIT_EPL; ++u) {
        if (STAGED || lane + 64 * u >= total) break;
        const uint32_t v = pe[u];
        const int t = ent_bin(v);
        const int pos = bend.fetch_inc(min(t >> INIT_BWS, nk - 1));
        E[pos] = t < T ? v : ((uint32_t)((nk << INIT_BWS) - 1) << 16);
    }
    // each photon raises the bound of every sub-block whose tau can see it by
    // z x the largest weight over those lags (M, indexed by the lag of the
    // sub-block's first tau, which falls by INIT_SB per sub-block)
#pragma unroll
    for (int u = 0; u < INIT_EPL; ++u) {
        if (STAGED || lane + 64 * u >= total) break;
        const int t = ent_bin(pe[u]);
        if (t < T) bound_photon<false>(bnd2, Mz, np, t + o, (uint32_t)ent_cnt(pe[u]));
    }
    wave_sync();
    // blocks lane and lane + 64: the largest sub-block bound; the cached
    // exact best
    uint32_t bmx[2], bsc[2];
    int btau[2];
    bool cached[2], has[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const int b = lane + 64 * s2;
        bmx[s2] = b < nb ? block_bound(bnd, nbs, b) : 0u;
        cached[s2] = b >= nb;     // blocks past the end are never picked
        has[s2] = false;
        bsc[s2] = 0;
        btau[s2] = NO_TAU;
    }
    // Blocks are picked by one wave maximum of a key: the block's bound
    // rounded up to 24 significant bits (shift sh; bounds only fall later),
    // plus one, above 127 - the block's index (smallest index on ties).  Any
    // unscored block's bound is at most the largest key's rounded bound.
    const uint32_t ball = wave_max_u32(max(bmx[0], bmx[1]));
    const int sh = max(0, 32 - (int)__clz(ball) - 24);
    const uint32_t rmask = (1u << sh) - 1u;
    const double k2 = p.kappa * p.kappa;
    for (int it = 0; it < p.k_init; ++it) {
        // best over the blocks whose exact best is known
        uint32_t best = 0;
        int bestt = NO_TAU;
        bool hb;
        {
            uint32_t key = 0;
            int kt = NO_TAU;
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                if (cached[s2] && has[s2] && (bsc[s2] + 1 > key || (bsc[s2] + 1 == key && btau[s2] < kt))) {
                    key = bsc[s2] + 1;
                    kt = btau[s2];
                }
            const uint32_t mx = wave_max_u32(key);
            hb = mx != 0;
            if (hb) {
                best = mx - 1;
                bestt = (int)wave_min_u32(key == mx ? (unsigned)kt : 0xffffffffu);
            }
        }
        while (true) {
            // the unscored block with the largest rounded bound
            uint32_t key = 0;
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                if (!cached[s2]) {
                    const uint32_t k = (bmx[s2] >> sh) + ((bmx[s2] & rmask) != 0u) + 1u;
                    key = max(key, (k << 7) | (uint32_t)(127 - (lane + 64 * s2)));
                }
            const uint32_t mx = wave_max_u32(key);
            if (mx == 0) break;                                   // every block scored
            const int bb = 127 - (int)(mx & 127u);
            const unsigned long long bu = (unsigned long long)((mx >> 7) - 1u) << sh;
            if (hb && bu < best) break;                           // no unscored tau can reach best
            const int hi = bb >> 6;                               // wave-uniform
            // exact scores of its 64 tau, and their best (tau rises with the lane)
            const int tau = (bb << 6) + lane;
            const uint32_t sc = score_block(E, bend, nk, bb, qs, L, o);
            const bool valid = tau < T && !(pk.suppresses_any(bb << 6, (bb << 6) + 63, m.wnms) &&
                                            pk.suppressed(tau, m.wnms));
            const uint32_t sk = valid ? sc + 1 : 0;
            const uint32_t smx = wave_max_u32(sk);
            int st = NO_TAU;
            if (smx != 0) st = (bb << 6) + (int)__ffsll((long long)__ballot(sk == smx)) - 1;
            if (lane == (bb & 63)) {
                if (hi) {
                    cached[1] = true;
                    has[1] = smx != 0;
                    bsc[1] = smx - 1;
                    btau[1] = st;
                } else {
                    cached[0] = true;
                    has[0] = smx != 0;
                    bsc[0] = smx - 1;
                    btau[0] = st;
                }
            }
            if (smx != 0 && (!hb || smx - 1 > best || (smx - 1 == best && st < bestt))) {
                best = smx - 1;
                bestt = st;
                hb = true;
            }
        }
        if (!hb) break;                      // every tau suppressed
        const int a = max(0, bestt - m.wl), c = min(T - 1, bestt + m.wr);
        uint32_t win = 0;
        for (int tb = a + lane; tb <= c; tb += 64) win += pk.owner(tb) < 0;
        win = wave_sum_u32(win);
        uint32_t nwin = 0;                                      // at most ntot
        const int b0 = a >> INIT_BWS, b1 = min(nk - 1, c >> INIT_BWS);
        const int x0 = b0 > 0 ? bend.get(b0 - 1) : 0, x1 = bend.get(b1);
        for (int x = x0 + lane; x < x1; x += 64) {
            const uint32_t v = E[x];
            const int tb = ent_bin(v);
            if (tb >= a && tb <= c) nwin += ent_cnt(v);        // claimed photons count zero
        }
        nwin = wave_sum_u32(nwin);
        const double bw = (double)ntot * (double)win / (double)T;
        const double d = (double)nwin - bw;
        const bool accept = win > 0 && (long long)nwin >= p.n_min && d >= 0.0 && d * d >= k2 * bw;
        if (!accept) break;
        pk.push(bestt, a, c, (int)win);
        // the peak claims the photons of its window: their counts drop to zero,
        // and their terms leave the bounds (which stay exact sums over the
        // unclaimed photons, so later rounds prune near the claimed peak)
        for (int x = x0 + lane; x < x1; x += 64) {
            const uint32_t v = E[x];
            const int tb = ent_bin(v), z = ent_cnt(v);
            if (tb >= a && tb <= c) {
                E[x] = v & 0xffff0000u;
                if (z > 0) bound_photon<true>(bnd2, Mz, np, tb + o, (uint32_t)z);
            }
        }
        wave_sync();
        // blocks the new peak changes: tau that see its claimed bins (their
        // bounds are recomputed) or fall under its suppression forget their
        // best
        const int A0 = a + o - L + 1, A1 = c + o, S0 = bestt - m.wnms, S1 = bestt + m.wnms;
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int b = lane + 64 * s2;
            const int ta = b << 6, tb = (b << 6) + 63;
            const bool seen = ta <= A1 && tb >= A0;
            if (b < nb && (seen || (ta <= S1 && tb >= S0))) cached[s2] = false;
            if (b < nb && seen) bmx[s2] = block_bound(bnd, nbs, b);
        }
    }
}

// Stages the IRF weights (INIT_QPAD zeros, the L weights, INIT_QPAD zeros)
// and their sliding maximum over INIT_SB lags (Mz, zero-padded) in LDS, with
// the whole workgroup; returns the largest weight (wave-uniform).  Without QL
// the weights stay in HBM and the result is 0.
template <bool QL>
__device__ __forceinline__ int stage_weights(const DevModel& m, int* qs, int* Mz)
{
    const int L = m.L, lane = threadIdx.x & 63;
    if (QL) {
        for (int k = threadIdx.x; k < L + 2 * INIT_QPAD; k += blockDim.x) {
            const int lag = k - INIT_QPAD;
            qs[k] = (lag >= 0 && lag < L) ? m.q[lag] : 0;
        }
        __syncthreads();
        const int nz = (int)q_window_ints(L);
        for (int k = threadIdx.x; k < nz; k += blockDim.x) {
            const int x = k - INIT_SB;
            int mx = 0;
            if (x >= 0 && x <= L + INIT_SB - 2) {
#pragma unroll
                for (int d = 0; d < INIT_SB; ++d) mx = max(mx, qs[INIT_QPAD + x - d]);
            }
            Mz[k] = mx;
        }
    }
    __syncthreads();
    int qmax = 0;
    if (QL) {
        for (int k = lane; k < L; k += 64) qmax = max(qmax, qs[INIT_QPAD + k]);
        qmax = (int)wave_max_u32((unsigned)qmax);
    }
    return qmax;
}

// Entry index of pooled photon k: window row r's photons (one CSR range,
// starting at rs of lane r) take pooled indices from rend - rlen of lane r.
__device__ __forceinline__ uint32_t pooled_src(uint32_t k, int side, uint32_t rend, uint32_t rlen, uint32_t rs)
{
    uint32_t src = 0;
    for (int r = 0; r < side; ++r) {
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)(rend - rlen), r);
        const uint32_t rb = (uint32_t)__builtin_amdgcn_readlane((int)rs, r);
        if (k >= r0) src = rb + (k - r0);
    }
    return src;
}

// One wavefront's initialisation of pixel pix, with the wavefront's LDS area
// at wbase.  QL: the weights are staged in LDS (qs, M; qmax their largest).
// WIDE: the pool may hold up to INIT_WIDE_ELDS photons, staged in passes over
// HBM; otherwise pools of INIT_ELDS to INIT_WIDE_ELDS photons that the LDS
// path could score are appended to the list `wide` (count first) when it is
// given, and left for the wide kernel.
template <bool QL, bool WIDE>
__device__ __forceinline__ void init_pixel(const DevModel& m, const DevParams& p, const Shape& sh,
                                           const uint32_t* __restrict__ off, const uint32_t* __restrict__ ent,
                                           const float* __restrict__ gain, DevState& s, long long pix,
                                           unsigned long long* wbase, const int* qs, const int* Mz, int qmax,
                                           uint32_t* wide)
{
    const int lane = threadIdx.x & 63;
    const int T = m.T, L = m.L, o = m.o;
    const int R = p.r_init, side = 2 * R + 1;
    const int* qt = QL ? qs + INIT_QPAD : m.q;
    const int* qstt = m.qst;
    const long long S = sh.S;
    const int nb = (T + 63) >> 6;
    uint2* lists = reinterpret_cast<uint2*>(wbase);
    unsigned long long* ub = wbase + side * side;                    // the HBM path's block bounds
    unsigned long long* lb = wbase;                                  // the LDS path's area
    (void)qt;

    if (lane < KM) {
        s.t[lane * S + pix] = 0.0;
        s.r[lane * S + pix] = 0.f;
        s.n[(0 * KM + lane) * S + pix] = 0.f;
        s.n[(1 * KM + lane) * S + pix] = 0.f;
        s.n[(2 * KM + lane) * S + pix] = -1.f;
    }
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pix / per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);

    // pooled photons: lane r < side holds the CSR range of window row i - R + r
    // (the row's pixels are consecutive, so their photons are one range)
    uint32_t rs = 0, re = 0;
    {
        const int i2 = i - R + lane;
        if (lane < side && i2 >= 0 && i2 < sh.rows) {
            const long long base = (fr * sh.rows + i2) * sh.cols;
            rs = off[base + max(0, j - R)];
            re = off[base + min(sh.cols - 1, j + R) + 1];
        }
    }
    const float G = gain_at(gain, pix);
    if (!(G > 0.f)) {
        if (lane == 0) {
            s.cnt[pix] = 0;
            s.b[pix] = (float)p.b_min;
        }
        return;
    }
    const uint32_t rlen = re - rs;
    const uint32_t rend = wave_incl_scan(rlen);                 // pooled index just past row lane
    const int total = (int)__builtin_amdgcn_readlane((int)rend, 63);

    Peaks pk;
    pk.n = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j) pk.t[j] = pk.a[j] = pk.c[j] = pk.w[j] = 0;

    // Branch and bound from LDS when the pool fits, the weights are staged,
    // and every score fits 32 bits (checked once the photons are read).
    const int nbs = (T + INIT_SB - 1) / INIT_SB;
    const bool ldsok = QL && nbs <= INIT_NB_LDS && qmax < (1 << 24);
    if (!WIDE && wide && ldsok && total > INIT_ELDS && total <= INIT_WIDE_ELDS) {
        if (lane == 0) {
            const unsigned sg = blockIdx.x % INIT_LIST_SEGS;
            wide[INIT_LIST_HDR + sg * init_list_cap(sh.P) + atomicAdd(&wide[sg * INIT_LIST_STRIDE], 1u)] =
                (uint32_t)pix;
        }
        return;
    }
    constexpr int ELDS = WIDE ? INIT_WIDE_ELDS : INIT_ELDS;
    bool lds = ldsok && total <= ELDS;
    uint32_t pe[INIT_EPL];
    long long ntot = 0;
    const int nk = (T + (1 << INIT_BWS) - 1) >> INIT_BWS;
    const int np = init_np(L);
    const int bw2 = (int)init_bound_words(T, L, o);
    uint32_t* bnd = reinterpret_cast<uint32_t*>(lb) + 2 * np - 2;    // [nbs] sub-block bounds, after their guards
    uint32_t* E = reinterpret_cast<uint32_t*>(lb + bw2);             // [ELDS] bucketed photons
    const Bend16 bend{E + ELDS};                                    // [nk] bucket ends, 16 bits each
    const int nkw = (nk + 1) >> 1;                                  // their words
    if (lds && WIDE) {
        // count the photons per bucket while totalling them (a first pass over HBM)
        for (int b = lane; b < bw2; b += 64) lb[b] = 0ull;
        for (int b = lane; b < nkw; b += 64) bend.w[b] = 0u;
        wave_sync();
        uint32_t nt = 0;                        // at most INIT_WIDE_ELDS x 65535
        // four 64-entry chunks per round, their loads in flight together
        for (int c0 = 0; c0 < total; c0 += 256) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = c0 + 64 * u + lane;
                const uint32_t x = pooled_src((uint32_t)k, side, rend, rlen, rs);
                v[u] = k < total ? ent[x] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + 64 * u + lane < total) {
                    if (ent_bin(v[u]) < T) nt += ent_cnt(v[u]);
                    bend.add1(min(ent_bin(v[u]) >> INIT_BWS, nk - 1));
                }
        }
        ntot = wave_sum_u32(nt);
        lds = (unsigned long long)ntot * (unsigned long long)qmax <= 0xfffffffeull;
    }
    if (lds && !WIDE) {
        // read the pooled photons once: entry k of the pool is lane k % 64's
        // pe[k / 64]
        uint32_t src[INIT_EPL];
#pragma unroll
        for (int u = 0; u < INIT_EPL; ++u) src[u] = 0;
        for (int r = 0; r < side; ++r) {
            const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)(rend - rlen), r);
            const uint32_t rb = (uint32_t)__builtin_amdgcn_readlane((int)rs, r);
#pragma unroll
            for (int u = 0; u < INIT_EPL; ++u) {
                const uint32_t k = (uint32_t)(lane + 64 * u);
                if (k >= r0) src[u] = rb + (k - r0);
            }
        }
#pragma unroll
        for (int u = 0; u < INIT_EPL; ++u) pe[u] = lane + 64 * u < total ? ent[src[u]] : 0u;
        uint32_t nt = 0;                        // at most INIT_ELDS x 65535
#pragma unroll
        for (int u = 0; u < INIT_EPL; ++u)
            if (lane + 64 * u < total && ent_bin(pe[u]) < T) nt += ent_cnt(pe[u]);
        ntot = wave_sum_u32(nt);
        lds = (unsigned long long)ntot * (unsigned long long)qmax <= 0xfffffffeull;
    }
    if (lds) {
        // Count the photons per 2^INIT_BWS-bin bucket, scan the counts into
        // bucket starts, then stage, bound and search them.
        if (!WIDE) {
            for (int b = lane; b < bw2; b += 64) lb[b] = 0ull;
            for (int b = lane; b < nkw; b += 64) bend.w[b] = 0u;
            wave_sync();
#pragma unroll
            for (int u = 0; u < INIT_EPL; ++u) {
                if (lane + 64 * u >= total) break;
                bend.add1(min(ent_bin(pe[u]) >> INIT_BWS, nk - 1));
            }
        }
        wave_sync();
        // bucket starts (exclusive prefix of the counts); each bucket's cursor
        // ends at the bucket's end once the photons are staged
        // (a word's two buckets at a time; a padding bucket past nk counts 0)
        uint32_t carry = 0;
        for (int c0 = 0; c0 < nkw; c0 += 64) {
            const int b = c0 + lane;
            const uint32_t wd = b < nkw ? bend.w[b] : 0u;
            const uint32_t lo = wd & 0xffffu, cnt = lo + (wd >> 16);
            const uint32_t inc = wave_incl_scan(cnt);
            const uint32_t s0 = carry + inc - cnt;
            if (b < nkw) bend.w[b] = s0 | ((s0 + lo) << 16);
            carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        }
        wave_sync();
        if (WIDE) {
            // second pass over HBM: stage each photon in its bucket (bins >= T
            // become zero counts at the last bucket's last bin) and add it to
            // the bounds of the sub-blocks whose tau can see it
            for (int c0 = 0; c0 < total; c0 += 256) {
                uint32_t vv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = c0 + 64 * u + lane;
                    const uint32_t x = pooled_src((uint32_t)k, side, rend, rlen, rs);
                    vv[u] = k < total ? ent[x] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (c0 + 64 * u + lane >= total) continue;
                    const uint32_t v = vv[u];
                    const int t = ent_bin(v), z = ent_cnt(v);
                    const int pos = bend.fetch_inc(min(t >> INIT_BWS, nk - 1));
                    E[pos] = t < T ? v : ((uint32_t)((nk << INIT_BWS) - 1) << 16);
                    if (t < T) bound_photon<false>(lb, Mz, np, t + o, (uint32_t)z);
                }
            }
            wave_sync();
        }
        lds_search<WIDE>(m, p, T, L, o, nb, nbs, nk, pe, total, ntot, qs, Mz, lb, np, bnd, E, bend, pk);
    } else {
        // the window's pixels' photon lists (each ascending in t)
        const int npl = side * side;
        for (int w = lane; w < npl; w += 64) {
            const int i2 = i - R + w / side, j2 = j - R + w % side;
            uint2 rg = make_uint2(0u, 0u);
            if (i2 >= 0 && i2 < sh.rows && j2 >= 0 && j2 < sh.cols) {
                const long long pp = (fr * sh.rows + i2) * sh.cols + j2;
                rg = make_uint2(off[pp], off[pp + 1]);
            }
            lists[w] = rg;
        }
        wave_sync();
        ntot = 0;
        const double k2 = p.kappa * p.kappa;
        // Branch and bound over blocks of 64 tau, reading the photons from HBM.
        for (int b = lane; b < nb; b += 64) ub[b] = 0ull;
        wave_sync();

        // photon total and per-block score bounds
        for (int l = 0; l < npl; ++l) {
            const uint2 rg = lists[l];
            for (uint32_t e = rg.x + lane; e < rg.y; e += 64) {
                const uint32_t v = ent[e];
                const int t = ent_bin(v), z = ent_cnt(v);
                if (t >= T) continue;
                ntot += z;
                const int tlo = max(0, t + o - L + 1), thi = min(T - 1, t + o);
                for (int b = tlo >> 6; b <= (thi >> 6); ++b) {
                    const int a0 = max(tlo, b << 6), a1 = min(thi, (b << 6) + 63);
                    const int qm = q_range_max(qstt, L, t - a1 + o, t - a0 + o);
                    atomicAdd(&ub[b], (unsigned long long)z * (unsigned long long)qm);
                }
            }
        }
        ntot = wave_sum(ntot);
        wave_sync();

        for (int it = 0; it < p.k_init; ++it) {
            long long best = -1;
            int bestt = 0x7fffffff;
            uint32_t done = 0;                      // bit q: block lane + 64 q scored in this round
            while (true) {
                // unscored block with the largest bound (smallest index on ties)
                unsigned long long bu = 0;
                int bb = 0x7fffffff;
                for (int q = 0; lane + 64 * q < nb; ++q) {
                    if ((done >> q) & 1u) continue;
                    const unsigned long long u = ub[lane + 64 * q];
                    if (bb == 0x7fffffff || u > bu) {
                        bu = u;
                        bb = lane + 64 * q;
                    }
                }
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) {
                    const unsigned long long ou = __shfl_xor(bu, d, 64);
                    const int ob = __shfl_xor(bb, d, 64);
                    if (ob != 0x7fffffff && (bb == 0x7fffffff || ou > bu || (ou == bu && ob < bb))) {
                        bu = ou;
                        bb = ob;
                    }
                }
                if (bb == 0x7fffffff) break;
                if ((long long)bu < best || ((long long)bu == best && (bb << 6) > bestt)) break;
                if (lane == (bb & 63)) done |= 1u << (bb >> 6);
                // exact scores of the block's 64 tau
                const int tau = (bb << 6) + lane;
                const int wlo = (bb << 6) - o, whi = (bb << 6) + 63 - o + L - 1;
                long long sc = 0;
                for (int l = 0; l < npl; ++l) {
                    const uint2 rg = lists[l];
                    int c0 = 0, c1 = 0;
                    for (uint32_t e0 = rg.x; e0 < rg.y; e0 += 64) {
                        const uint32_t e = e0 + lane;
                        const int t = e < rg.y ? ent_bin(ent[e]) : 0x7fffffff;
                        c0 += popc_ballot(t < wlo);
                        c1 += popc_ballot(t <= whi);
                    }
                    for (uint32_t x = rg.x + c0; x < rg.x + c1; ++x) {
                        const uint32_t v = ent[x];
                        const int tb = ent_bin(v);
                        if (pk.owner(tb) >= 0) continue;
                        const int lag = tb - tau + o;
                        if ((unsigned)lag < (unsigned)L) sc += (long long)ent_cnt(v) * (long long)m.q[lag];
                    }
                }
                const bool valid = tau < T && !pk.suppressed(tau, m.wnms);
                long long sv = valid ? sc : -1;
                int st = valid ? tau : 0x7fffffff;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) {
                    const long long ov = __shfl_xor(sv, d, 64);
                    const int ot = __shfl_xor(st, d, 64);
                    if (ov > sv || (ov == sv && ot < st)) {
                        sv = ov;
                        st = ot;
                    }
                }
                if (st != 0x7fffffff && (sv > best || (sv == best && st < bestt))) {
                    best = sv;
                    bestt = st;
                }
            }
            if (bestt == 0x7fffffff) break;          // every tau suppressed
            const int a = max(0, bestt - m.wl), c = min(T - 1, bestt + m.wr);
            int win = 0;
            for (int tb = a + lane; tb <= c; tb += 64) win += pk.owner(tb) < 0;
            win = wave_sum(win);
            long long nwin = 0;
            for (int l = 0; l < npl; ++l) {
                const uint2 rg = lists[l];
                for (uint32_t e = rg.x + lane; e < rg.y; e += 64) {
                    const uint32_t v = ent[e];
                    const int tb = ent_bin(v);
                    if (tb >= a && tb <= c && pk.owner(tb) < 0) nwin += ent_cnt(v);
                }
            }
            nwin = wave_sum(nwin);
            const double bw = (double)ntot * (double)win / (double)T;
            const double d = (double)nwin - bw;
            const bool accept = win > 0 && nwin >= p.n_min && d >= 0.0 && d * d >= k2 * bw;
            if (!accept) break;
            pk.push(bestt, a, c, win);
        }
    }
    const int npk = pk.n;

    // own photons: total and per claimed window
    // (a pixel holds at most 65535 entries, each count below 65536: the sums
    // fit 32 bits)
    const uint32_t e0 = off[pix], e1 = off[pix + 1];
    uint32_t zp = 0;
    uint32_t nown[KM] = {0, 0, 0, 0};
    for (uint32_t e = e0 + lane; e < e1; e += 64) {
        const uint32_t v = ent[e];
        const uint32_t z = (uint32_t)ent_cnt(v);
        zp += z;
        const int ow = pk.owner(ent_bin(v));
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (ow == k) nown[k] += z;
    }
    zp = wave_sum_u32(zp);
    double H[KM] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < npk) {
            nown[k] = wave_sum_u32(nown[k]);
            double hs = 0.0;
            for (int tb = pk.a[k] + lane; tb <= pk.c[k]; tb += 64) {
                const int idx = tb - pk.t[k] + o;
                if (pk.owner(tb) == k && idx >= 0 && idx < L) hs += m.hbar[idx];
            }
            H[k] = wave_sum(hs);
        }
    }
    long long sum_n = 0, sum_w = 0;                          // (wave-uniform)
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < npk) {
            sum_n += nown[k];
            sum_w += pk.w[k];
        }
    long long num = (long long)zp - sum_n;
    if (num < 0) num = 0;
    const long long den = (long long)T - sum_w;
    // lane k < KM decides peak k (keep, depth, intensity); the kept peaks
    // take the slots in ascending depth (depths are distinct): a peak's slot
    // is the number of kept peaks above it
    long long w = 0;
    long long nwk = 0;
    double hk = 0.0;
    int tk = 0;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (lane == k) {
            w = pk.w[k];
            nwk = nown[k];
            hk = H[k];
            tk = pk.t[k];
        }
    const bool keep = lane < npk && (den > 0 ? (nwk * den > num * w) : (nwk > 0)) && hk > 0.0;
    const int kt = keep ? tk : 0x7fffffff;
    const uint32_t kept = (uint32_t)__ballot(keep) & ((1u << KM) - 1u);
    int rank = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j) rank += __builtin_amdgcn_readlane(kt, j) < kt ? 1 : 0;
    int nkeep = __builtin_popcount(kept);
    if (nkeep > p.k_max) nkeep = p.k_max;
    if (keep && rank < nkeep) {
        const double excess = den > 0 ? (double)nwk - (double)num * (double)w / (double)den : (double)nwk;
        s.t[rank * S + pix] = (double)kt;
        s.r[rank * S + pix] = (float)(excess / ((double)G * hk));
    }
    if (lane != 0) return;
    s.cnt[pix] = (uint8_t)nkeep;
    const double bown = den > 0 ? (double)num / (double)den : 0.0;
    const double b0 = bown / (double)G;
    s.b[pix] = (float)(b0 > p.b_min ? b0 : p.b_min);
}

// QL: the IRF weight tables are staged in LDS (they fit INIT_QLDS ints).
// wide: list of pixels left for k_init_wide (segment counters first), or null.
template <bool QL>
__global__ __launch_bounds__(64 * INIT_WAVES, 7) void k_init(DevModel m, DevParams p, Shape sh,
                                                          const uint32_t* __restrict__ off,
                                                          const uint32_t* __restrict__ ent,
                                                          const float* __restrict__ gain, DevState s,
                                                          uint32_t* wide)
{
    extern __shared__ unsigned long long smem64[];
    const int wv = threadIdx.x >> 6;
    const size_t ww = init_wave_words(m.T, m.L, m.o, p.r_init);
    int* qs = reinterpret_cast<int*>(smem64 + INIT_WAVES * ww);
    int* Mz = qs + q_staged_ints(m.L);
    const int qmax = stage_weights<QL>(m, qs, Mz);
    const long long pix = (long long)xcd_block(blockIdx.x, gridDim.x) * INIT_WAVES + wv;
    // whole wavefront (pixels of other IRF classes: their own launch); no workgroup barriers below
    if (pix >= sh.P || !in_class(m, pix)) return;
    init_pixel<QL, false>(m, p, sh, off, ent, gain, s, pix, smem64 + (size_t)wv * ww, qs, Mz, qmax, wide);
}

// The pixels k_init listed (pools of INIT_ELDS to INIT_WIDE_ELDS photons),
// a wavefront each, strided over a fixed grid.
__global__ __launch_bounds__(64 * INIT_WAVES) void k_init_wide(DevModel m, DevParams p, Shape sh,
                                                               const uint32_t* __restrict__ off,
                                                               const uint32_t* __restrict__ ent,
                                                               const float* __restrict__ gain, DevState s,
                                                               const uint32_t* __restrict__ wide)
{
    extern __shared__ unsigned long long smem64[];
    // listed pixel k lies in the segment whose inclusive count prefix (lane
    // s: segment s) first exceeds k
    const int lane = threadIdx.x & 63;
    const uint32_t cs = wide[lane * INIT_LIST_STRIDE];
    const uint32_t incl = wave_incl_scan(cs);
    const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    if ((size_t)blockIdx.x * INIT_WAVES >= n) return;                 // whole workgroup
    const size_t cap = init_list_cap(sh.P);
    const int wv = threadIdx.x >> 6;
    const size_t ww = init_wave_words(m.T, m.L, m.o, p.r_init, INIT_WIDE_ELDS);
    int* qs = reinterpret_cast<int*>(smem64 + INIT_WAVES * ww);
    int* Mz = qs + q_staged_ints(m.L);
    const int qmax = stage_weights<true>(m, qs, Mz);
    for (uint32_t k = blockIdx.x * INIT_WAVES + wv; k < n; k += gridDim.x * INIT_WAVES) {
        const int sg = __popcll(__builtin_amdgcn_ballot_w64(incl <= k));
        const uint32_t at = k - (uint32_t)__builtin_amdgcn_readlane((int)(incl - cs), sg);
        init_pixel<true, true>(m, p, sh, off, ent, gain, s, (long long)wide[INIT_LIST_HDR + sg * cap + at],
                               smem64 + (size_t)wv * ww, qs, Mz, qmax, nullptr);
    }
}

__global__ void k_init_reset(uint32_t* wide)
{
    if (threadIdx.x < INIT_LIST_SEGS) wide[threadIdx.x * INIT_LIST_STRIDE] = 0u;
}

// Words of the list for P pixels.
size_t init_list_words(long long P) { return INIT_LIST_HDR + INIT_LIST_SEGS * init_list_cap(P); }

// Initial normals (reading): weighted least-squares plane Z = a + c1 X + c2 Y
// over the APSS neighbourhood in FP64, local coordinates; n = (c1, c2, -1)/|.|,
// or (0, 0, -1) with fewer than 3 neighbours or a near-singular system.
__global__ __launch_bounds__(256) void k_init_normals(DevParams p, Shape sh, DevState s)
{
    const long long P = sh.P, S = sh.S;
    const long long pix = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    const int c = load_cnt(s.cnt, pix);
    const int per_frame = sh.rows * sh.cols;
    const long long fr = pix / per_frame;
    const int i = (int)((pix / sh.cols) % sh.rows), j = (int)(pix % sh.cols);
    const double h2 = p.h_apss * p.h_apss, inv_h2 = 1.0 / h2;
    const int R = p.apss_R;
    const bool persp = p.persp > 0.0;   // pinhole camera: t dz along each pixel's ray
    double vq[3] = {0.0, 0.0, 1.0};
    if (persp) ray_dir(p.persp, sh.rows, sh.cols, i, j, vq);
    for (int k = 0; k < KM; ++k) {
        if (k >= c) break;
        const double tq = s.t[k * S + pix];
        double M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0, v0 = 0, v1 = 0, v2 = 0, W = 0;
        int nn = 0;
        for (int i2 = i - R; i2 <= i + R; ++i2) {
            if (i2 < 0 || i2 >= sh.rows) continue;
            for (int j2 = j - R; j2 <= j + R; ++j2) {
                if (j2 < 0 || j2 >= sh.cols) continue;
                const long long pp = (fr * sh.rows + i2) * sh.cols + j2;
                const int cc = load_cnt(s.cnt, pp);
                // every slot's depth without waiting for the count
                double tn[KM];
#pragma unroll
                for (int k2 = 0; k2 < KM; ++k2) tn[k2] = s.t[k2 * S + pp];
                double vn[3] = {0.0, 0.0, 1.0};
                if (persp && cc > 0) ray_dir(p.persp, sh.rows, sh.cols, i2, j2, vn);
#pragma unroll
                for (int k2 = 0; k2 < KM; ++k2) {
                    if (k2 >= cc) break;
                    double x = (j2 - j) * p.p_xy, y = (i2 - i) * p.p_xy;
                    double z = (tn[k2] - tq) * p.dz;
                    if (persp) {
                        const double t2 = tn[k2];
                        x = (t2 * vn[0] - tq * vq[0]) * p.dz;
                        y = (t2 * vn[1] - tq * vq[1]) * p.dz;
                        z = (t2 * vn[2] - tq * vq[2]) * p.dz;
                    }
                    const double d2 = x * x + y * y + z * z;
                    if (!(d2 < h2)) continue;
                    double a = 1.0 - d2 * inv_h2;
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
                // facing the sensor: against the pixel's ray (always so for the
                // orthographic map); a plane containing the pinhole camera's
                // line of sight (within 1e-6) takes n = -v
                const double nv = (c1 * vq[0] + c2 * vq[1] - vq[2]) / nrm;
                if (persp && fabs(nv) <= 1e-6) {
                    nx = (float)(-vq[0]);
                    ny = (float)(-vq[1]);
                    nz = (float)(-vq[2]);
                } else {
                    const double sg = nv > 0.0 ? -1.0 : 1.0;
                    nx = (float)(sg * c1 / nrm);
                    ny = (float)(sg * c2 / nrm);
                    nz = (float)(-sg / nrm);
                }
            }
        }
        s.n[(0 * KM + k) * S + pix] = nx;
        s.n[(1 * KM + k) * S + pix] = ny;
        s.n[(2 * KM + k) * S + pix] = nz;
    }
}

// LDS bytes of one init workgroup (wide: of the wide kernel): the
// wavefronts' areas and the IRF weights (o: the IRF's origin, 0 <= o < L).
size_t init_lds_bytes(int T, int L, int o, int r_init, bool wide)
{
    const size_t nq = q_staged_ints(L);
    const size_t qwords = nq <= INIT_QLDS ? (nq + q_window_ints(L) + 1) / 2 : 0;
    return (INIT_WAVES * init_wave_words(T, L, o, r_init, wide ? INIT_WIDE_ELDS : INIT_ELDS) + qwords) *
           sizeof(unsigned long long);
}

hipError_t launch_init(const DevModel& m, const DevParams& p, const Shape& sh, const uint32_t* off,
                       const uint32_t* ent, const float* gain, DevState s, uint32_t* wide, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    const size_t lds = init_lds_bytes(m.T, m.L, m.o, p.r_init, false);
    const unsigned nblk = (unsigned)((sh.P + INIT_WAVES - 1) / INIT_WAVES);
    if (q_staged_ints(m.L) > (size_t)INIT_QLDS) {
        hipLaunchKernelGGL(k_init<false>, dim3(nblk), dim3(64 * INIT_WAVES), lds, st, m, p, sh, off, ent, gain, s,
                           nullptr);
        return hipGetLastError();
    }
    const size_t wlds = init_lds_bytes(m.T, m.L, m.o, p.r_init, true);
    if (wlds > 65536 || sh.P >= (1ll << 32)) wide = nullptr;
    if (wide) hipLaunchKernelGGL(k_init_reset, dim3(1), dim3(64), 0, st, wide);
    hipLaunchKernelGGL(k_init<true>, dim3(nblk), dim3(64 * INIT_WAVES), lds, st, m, p, sh, off, ent, gain, s, wide);
    if (wide)
        hipLaunchKernelGGL(k_init_wide, dim3(std::min(nblk, INIT_WIDE_GRID)), dim3(64 * INIT_WAVES), wlds, st, m, p,
                           sh, off, ent, gain, s, wide);
    return hipGetLastError();
}

hipError_t launch_init_normals(const DevParams& p, const Shape& sh, DevState s, hipStream_t st)
{
    if (sh.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_normals, dim3((unsigned)((sh.P + 255) / 256)), dim3(256), 0, st, p, sh, s);
    return hipGetLastError();
}

}  // namespace rt3d

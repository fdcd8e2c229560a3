// k_compact.hip -- histogram -> active-bin lists, and a device-wide exclusive
// scan.  The paper's cost model (Methods) is linear in the active (non-zero)
// bins of each pixel; every later step reads only these lists.
//
// Layout: Z is uint16 [P][T] (bins contiguous per pixel); the output is CSR
// over pixels, entry = (bin << 16) | count, ascending bin.  One wavefront per
// pixel streams the pixel's bins with 16-byte loads (8 bins per lane per
// load); a wave-level prefix sum places each lane's entries.
#include "rt3d_dev.h"

#include <mutex>

namespace rt3d {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Exclusive prefix over the block's threads; returns the block total in `total`.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t& total)
{
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan(v);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        uint32_t s = wsum[k];
        if (k < w) base += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

// Tile totals of the counts (each tile of SCAN_TILE counts fits 32 bits: the
// counts are per-pixel entries, points or events, each below 2^16 per tile
// element or summing below 2^31), widened to 64 bits.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              long long n, uint64_t* __restrict__ partial)
{
    long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t total;
    block_excl_scan(s, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One block: exclusive scan of the nb tile totals in place, in 64 bits (each
// thread a contiguous run of tiles, then a scan of the run sums in LDS);
// out[n] = the grand total clamped to `cap`.  A grand total above `cap` sets
// E_CAPACITY.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(uint64_t* __restrict__ partial,
                                                                long long nb, uint32_t* __restrict__ out_total,
                                                                uint64_t cap, int32_t* __restrict__ err)
{
    __shared__ uint64_t run[SCAN_THREADS];
    const long long per = (nb + SCAN_THREADS - 1) / SCAN_THREADS;
    const long long b0 = (long long)threadIdx.x * per;
    const long long b1 = b0 + per < nb ? b0 + per : nb;
    uint64_t s = 0;
    for (long long i = b0; i < b1; ++i) s += partial[i];
    run[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the run sums
    for (int d = 1; d < SCAN_THREADS; d <<= 1) {
        const uint64_t add = threadIdx.x >= (unsigned)d ? run[threadIdx.x - d] : 0ull;
        __syncthreads();
        run[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t acc = run[threadIdx.x] - s;
    for (long long i = b0; i < b1; ++i) {
        const uint64_t v = partial[i];
        partial[i] = acc;
        acc += v;
    }
    if (threadIdx.x == SCAN_THREADS - 1) {
        const uint64_t total = run[SCAN_THREADS - 1];
        *out_total = (uint32_t)(total < cap ? total : cap);
        if (err && total > cap) *err = RT3D_E_CAPACITY;
    }
}

// out[i] = the exclusive prefix of element i, clamped to `cap`: past the
// capacity every list is empty, and a list that crosses it ends there.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const uint32_t* __restrict__ in, long long n,
                                                             const uint64_t* __restrict__ partial, uint64_t cap,
                                                             uint32_t* __restrict__ out)
{
    long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint64_t run = partial[blockIdx.x] + block_excl_scan(s, total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = (uint32_t)(run < cap ? run : cap);
        run += v[k];
    }
}

// 32-bit words of scan workspace for n elements: one 64-bit prefix per tile.
size_t scan_partial_elems(long long n) { return 2 * ((size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1); }

// out[0..n] = exclusive prefix of in[0..n-1] followed by the total, every
// value clamped to min(cap, 2^32 - 1) (a total above that sets E_CAPACITY).  `in` and `out` may alias (each tile reads its inputs before
// writing).  partial: scan_partial_elems(n) words, 8-byte aligned.
hipError_t launch_scan(const uint32_t* in, uint32_t* out, long long n, uint32_t* partial, uint64_t cap,
                       int32_t* err, hipStream_t st)
{
    uint64_t* part = reinterpret_cast<uint64_t*>(partial);
    if (cap > 0xffffffffull) cap = 0xffffffffull;   // offsets are 32-bit
    long long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb > 0)
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, st, part, nb, out + n, cap, err);
    if (nb > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, n, part, cap, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction

constexpr int CP_WAVES = 4;   // pixels (wavefronts) per block
constexpr int CP_VPL = 2;     // 8-bin vectors per lane per pass of the stage kernel

// One pixel's histogram as 16-byte vectors of 8 bins: vector vr (0 <= vr <
// nvec) holds bins 8 (vs + vr) .. 8 (vs + vr) + 7 of the flat array, the
// pixel's bins being those at offsets [lo_off, hi_end) from bin 8 vs (pixels
// are not 8-bin aligned).  32-bit offsets inside the pixel; the 64-bit
// address is formed once.
struct PixVec {
    const uint4* zv;      // first vector of the pixel
    const uint16_t* z0;   // its first bin
    int nvec, lo_off, hi_end, tail;   // tail: bins of the array's last vector (8 if whole)
};

__device__ __forceinline__ PixVec pix_vectors(const uint16_t* __restrict__ Z, long long p, int T, long long total)
{
    const long long lo = p * T, vs = lo >> 3;
    PixVec v;
    v.zv = reinterpret_cast<const uint4*>(Z) + vs;
    v.z0 = Z + (vs << 3);
    v.nvec = (int)(((lo + T + 7) >> 3) - vs);
    v.lo_off = (int)(lo - (vs << 3));
    v.hi_end = v.lo_off + T;
    const long long left = total - ((vs + v.nvec - 1) << 3);   // bins of the array from the last vector on
    v.tail = left < 8 ? (int)left : 8;                         // < 8 only for the array's partial last vector
    return v;
}

// The 8 bins of vector vr as four words of two bins each; bins outside the
// pixel read as 0 (only its first and last vector hold any).
__device__ __forceinline__ void load8(const PixVec& pv, int vr, uint32_t (&w)[4])
{
    if (vr == pv.nvec - 1 && pv.tail < 8) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = (vr << 3) + 2 * q;
            const uint32_t a = 2 * q < pv.tail ? pv.z0[k] : 0u;
            const uint32_t b = 2 * q + 1 < pv.tail ? pv.z0[k + 1] : 0u;
            w[q] = a | (b << 16);
        }
    } else {
        const uint4 x = pv.zv[vr];
        w[0] = x.x;
        w[1] = x.y;
        w[2] = x.z;
        w[3] = x.w;
    }
    const int r0 = vr << 3;
    if (r0 < pv.lo_off || r0 + 8 > pv.hi_end) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (r0 + k < pv.lo_off || r0 + k >= pv.hi_end) w[k >> 1] &= (k & 1) ? 0x0000ffffu : 0xffff0000u;
    }
}

// Bit k of the result: bin k of the vector is non-zero.  Each word's two
// 16-bit counts become 0 or 1 with one packed 16-bit minimum against 1;
// words 1 and 3 shift by two bits onto words 0 and 2, word 2 by four onto
// word 0, so bins 0, 2, 4, 6 land on bits 0, 2, 4, 6 and bins 1, 3, 5, 7 on
// bits 16, 18, 20, 22, which a shift by 15 brings to bits 1, 3, 5, 7.
__device__ __forceinline__ uint32_t nonzero_halves(uint32_t w)
{
    uint32_t r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(w), "s"(0x00010001u));   // (the compiler otherwise
    return r;                                                             // compares each half)
}

__device__ __forceinline__ uint32_t nonzero8(const uint32_t (&w)[4])
{
    const uint32_t a = nonzero_halves(w[0]) | (nonzero_halves(w[1]) << 2);
    const uint32_t b = nonzero_halves(w[2]) | (nonzero_halves(w[3]) << 2);
    const uint32_t c = a | (b << 4);
    return (c | (c >> 15)) & 0xffu;
}

// Count of bin k of the vector.
__device__ __forceinline__ uint32_t bin8(const uint32_t (&w)[4], int k)
{
    const int q = k >> 1;
    const uint32_t x = q == 0 ? w[0] : q == 1 ? w[1] : q == 2 ? w[2] : w[3];
    return (k & 1) ? x >> 16 : x & 0xffffu;
}

// Pass 1: each pixel's histogram is read once; its non-zero bins, as entries
// (t << 16 | z) in ascending t, go to the pixel's staging slot of CP_STAGE
// entries (the first CP_STAGE of them when it has more; no staging when
// `stage` is null), and its entry count to counts[p].  One wavefront per
// pixel; a pass loads CP_VPL runs of 64 consecutive 8-bin vectors (one per
// lane each, so that every load instruction reads 1 KB in one piece), then
// for each run a wavefront prefix sum of the lanes' non-zero counts places
// them; a lane writes its non-zero bins one set bit of its mask at a time
// (most lanes hold none).
__global__ __launch_bounds__(64 * CP_WAVES) void k_compact_stage(const uint16_t* __restrict__ Z, long long P,
                                                                 int T, uint32_t* __restrict__ counts,
                                                                 uint32_t* __restrict__ stage)
{
    const long long p = (long long)blockIdx.x * CP_WAVES + (threadIdx.x >> 6);
    if (p >= P) return;
    const int lane = threadIdx.x & 63;
    const PixVec pv = pix_vectors(Z, p, T, P * T);
    uint32_t* slot = stage ? stage + p * CP_STAGE : nullptr;
    uint32_t run = 0;
    for (int vb = 0; vb < pv.nvec; vb += 64 * CP_VPL) {   // uniform over the wave
        // CP_VPL vectors per lane, each load instruction 64 consecutive ones
        uint32_t w[CP_VPL][4];
#pragma unroll
        for (int q = 0; q < CP_VPL; ++q) {
            const int vr = vb + 64 * q + lane;
            w[q][0] = w[q][1] = w[q][2] = w[q][3] = 0u;
            if (vr < pv.nvec) load8(pv, vr, w[q]);
        }
#pragma unroll
        for (int q = 0; q < CP_VPL; ++q) {
            if (vb + 64 * q >= pv.nvec) break;                   // uniform
            const int vr = vb + 64 * q + lane;
            uint32_t m = nonzero8(w[q]);
            const uint32_t c = (uint32_t)__builtin_popcount(m);
            const uint32_t inc = wave_incl_scan(c);
            uint32_t pos = run + (inc - c);
            const uint32_t base = (uint32_t)((vr << 3) - pv.lo_off);   // bin of bit 0 (bit k: base + k)
            while (m) {
                const int k = __builtin_ctz(m);
                m &= m - 1u;
                if (slot && pos < CP_STAGE) slot[pos] = ((base + k) << 16) | bin8(w[q], k);
                ++pos;
            }
            run += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        }
    }
    if (lane == 0) counts[p] = run;
}

// Pass 2 (after the scan of the counts into off): each pixel's entries move
// from its staging slot to off[p]; a pixel with more than CP_STAGE entries
// (every pixel when `stage` is null) reads its histogram again.  Entries past
// `cap` are dropped (E_CAPACITY); the scan has clamped the offsets to `cap`,
// so every later step sees the lists cut at the capacity.
__global__ __launch_bounds__(64 * CP_WAVES) void k_compact_copy(const uint16_t* __restrict__ Z, long long P,
                                                                int T, const uint32_t* __restrict__ off,
                                                                const uint32_t* __restrict__ stage,
                                                                uint32_t* __restrict__ ent, uint64_t cap,
                                                                int32_t* __restrict__ err)
{
    const long long p = (long long)blockIdx.x * CP_WAVES + (threadIdx.x >> 6);
    if (p >= P) return;
    const int lane = threadIdx.x & 63;
    const uint64_t base = off[p];
    const uint32_t n = off[p + 1] - off[p];
    bool overflow = false;
    if (stage && n <= (uint32_t)CP_STAGE) {
        // the slot's entries load with the offsets (the slot holds CP_STAGE
        // entries whatever the count)
        const uint32_t* slot = stage + p * CP_STAGE;
        static_assert(CP_STAGE == 128, "two entries of the slot per lane");
        const uint32_t s0 = slot[lane], s1 = slot[lane + 64];
        if ((uint32_t)lane < n) {
            if (base + lane < cap) ent[base + lane] = s0;
            else overflow = true;
        }
        if ((uint32_t)lane + 64 < n) {
            if (base + lane + 64 < cap) ent[base + lane + 64] = s1;
            else overflow = true;
        }
    } else {
        const PixVec pv = pix_vectors(Z, p, T, P * T);
        uint64_t run = base;
        for (int vb = 0; vb < pv.nvec; vb += 64) {     // uniform over the wave
            const int vr = vb + lane;
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            if (vr < pv.nvec) load8(pv, vr, w);
            uint32_t m = nonzero8(w);
            const uint32_t c = (uint32_t)__builtin_popcount(m);
            const uint32_t inc = wave_incl_scan(c);
            uint64_t pos = run + (inc - c);
            const uint32_t b0 = (uint32_t)((vr << 3) - pv.lo_off);
            while (m) {
                const int k = __builtin_ctz(m);
                m &= m - 1u;
                if (pos < cap) ent[pos] = ((b0 + k) << 16) | bin8(w, k);
                else overflow = true;
                ++pos;
            }
            run += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        }
    }
    if (overflow) *err = RT3D_E_CAPACITY;
}

hipError_t launch_compact(const uint16_t* Z, long long P, int T, uint32_t* off, uint32_t* ent, uint64_t cap,
                          uint32_t* counts, uint32_t* partial, uint32_t* stage, int32_t* err, hipStream_t st)
{
    unsigned nb = (unsigned)((P + CP_WAVES - 1) / CP_WAVES);
    if (nb > 0) hipLaunchKernelGGL(k_compact_stage, dim3(nb), dim3(64 * CP_WAVES), 0, st, Z, P, T, counts, stage);
    hipError_t e = launch_scan(counts, off, P, partial, cap, err, st);
    if (e != hipSuccess) return e;
    if (nb > 0)
        hipLaunchKernelGGL(k_compact_copy, dim3(nb), dim3(64 * CP_WAVES), 0, st, Z, P, T, off, stage, ent, cap,
                           err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction with no device allocation: the per-pixel counts and the scan's
// tile prefixes live in a fixed array of the library (one copy per GPU), and
// no entry is staged (the copy pass reads every histogram again).

constexpr long long NOALLOC_MAX_PIX = 1ll << 22;
constexpr size_t NOALLOC_ERR_WORDS = 64;   // error sink, keeps the counts 256-byte aligned
constexpr size_t NOALLOC_WORDS = NOALLOC_ERR_WORDS + (size_t)NOALLOC_MAX_PIX + 2 * ((size_t)(NOALLOC_MAX_PIX + SCAN_TILE - 1) / SCAN_TILE + 1);

static_assert(NOALLOC_MAX_PIX == RT3D_NOALLOC_MAX_PIXELS, "rt3d.h states the pixel limit");
static_assert(sizeof(uint32_t) * NOALLOC_WORDS == RT3D_NOALLOC_SCRATCH_BYTES, "rt3d.h states the array size");

static __device__ __align__(256) uint32_t scratch[NOALLOC_WORDS];

namespace {
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[256];   // the array's device address on each GPU (nullptr: not looked up yet)
}

long long noalloc_max_pixels() { return NOALLOC_MAX_PIX; }
size_t noalloc_scratch_bytes() { return sizeof(uint32_t) * NOALLOC_WORDS; }

// Device address of the array on the current GPU, looked up once per device.
hipError_t noalloc_scratch(uint32_t** ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!a) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint32_t*>(a);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

// The same lists as launch_compact (the arguments checked by the caller:
// 0 < P <= NOALLOC_MAX_PIX); err: device word for E_CAPACITY, or null.
hipError_t launch_compact_noalloc(const uint16_t* Z, long long P, int T, uint32_t* off, uint32_t* ent,
                                  uint64_t cap, int32_t* err, hipStream_t st)
{
    if (P <= 0 || P > NOALLOC_MAX_PIX) return hipErrorInvalidValue;
    uint32_t* base = nullptr;
    hipError_t e = noalloc_scratch(&base);
    if (e != hipSuccess) return e;
    int32_t* sink = reinterpret_cast<int32_t*>(base);
    uint32_t* counts = base + NOALLOC_ERR_WORDS;
    uint32_t* partial = counts + NOALLOC_MAX_PIX;
    return launch_compact(Z, P, T, off, ent, cap, counts, partial, nullptr, err ? err : sink, st);
}

}  // namespace rt3d

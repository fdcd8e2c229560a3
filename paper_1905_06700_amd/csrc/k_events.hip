// k_events.hip -- photon events -> active-bin lists, the same CSR that the
// histogram compaction writes.  A time-tagged detector delivers photons as
// (pixel, bin) events rather than histograms; the method only ever needs each
// pixel's non-zero bins and their counts (Methods: cost linear in the active
// bins), so events are counted straight into those lists.
//
// Steps: events per pixel (atomics) -> exclusive scan = event segments ->
// scatter every event's bin into its pixel's segment (arbitrary order inside
// the segment) -> sort each segment (one wavefront per pixel; a bitonic network
// in LDS, or in place in the scratch buffer for segments longer than LDS
// holds) and count its distinct bins -> scan = CSR offsets -> run-length
// encode each sorted segment.  The result does not depend on the event order.
#include "rt3d_dev.h"

namespace rt3d {

constexpr int EV_THREADS = 256;
constexpr int EV_WAVES = 4;        // pixels (wavefronts) per block in the per-pixel kernels
constexpr int EV_LDS = 2048;       // longest segment sorted in LDS (8 KB per wavefront)
constexpr uint32_t EV_INF = 0xffffffffu;

__global__ __launch_bounds__(EV_THREADS) void k_ev_zero(uint32_t* __restrict__ a, long long n)
{
    for (long long i = (long long)blockIdx.x * EV_THREADS + threadIdx.x; i < n; i += (long long)gridDim.x * EV_THREADS)
        a[i] = 0u;
}

__device__ __forceinline__ bool ev_valid(uint32_t p, uint32_t b, long long P, int T)
{
    return (long long)p < P && (int)b < T;
}

__global__ __launch_bounds__(EV_THREADS) void k_ev_count(const uint32_t* __restrict__ pix,
                                                         const uint16_t* __restrict__ bin, uint64_t n,
                                                         long long P, int T, uint32_t* __restrict__ counts,
                                                         int32_t* __restrict__ err)
{
    const uint64_t i = (uint64_t)blockIdx.x * EV_THREADS + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = pix[i], b = bin[i];
    if (!ev_valid(p, b, P, T)) {
        *err = RT3D_E_INVALID;
        return;
    }
    atomicAdd(&counts[p], 1u);
}

__global__ __launch_bounds__(EV_THREADS) void k_ev_scatter(const uint32_t* __restrict__ pix,
                                                           const uint16_t* __restrict__ bin, uint64_t n,
                                                           long long P, int T, const uint32_t* __restrict__ evoff,
                                                           uint32_t* __restrict__ cursor,
                                                           uint32_t* __restrict__ scratch)
{
    const uint64_t i = (uint64_t)blockIdx.x * EV_THREADS + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = pix[i], b = bin[i];
    if (!ev_valid(p, b, P, T)) return;
    const uint32_t k = atomicAdd(&cursor[p], 1u);
    scratch[(uint64_t)evoff[p] + k] = b;
}

// Orders the wavefront's memory traffic (LDS or global) between network stages.
__device__ __forceinline__ void ev_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void ev_cswap(uint32_t* a, uint32_t i, uint32_t l)
{
    const uint32_t x = a[i], y = a[l];
    if (y < x) {
        a[i] = y;
        a[l] = x;
    }
}

// Ascending bitonic sort of a[0..n) by one wavefront, on the next power of two
// N2 >= n with a[n..N2) taken as +infinity.  Every comparator puts the smaller
// value at the lower index, so a comparator whose upper index is >= n would
// leave both places as they are: it is skipped and the padding is never
// stored.
__device__ void ev_bitonic(uint32_t* a, uint32_t n)
{
    uint32_t N2 = 1;
    while (N2 < n) N2 <<= 1;
    const uint32_t lane = threadIdx.x & 63, half = N2 >> 1;
    for (uint32_t k = 2; k <= N2; k <<= 1) {
        const uint32_t hk = k >> 1;
        for (uint32_t t = lane; t < half; t += 64) {       // merge step of width k (mirrored pairs)
            const uint32_t o = t & (hk - 1), base = (t - o) << 1;
            const uint32_t i = base + o, l = base + k - 1 - o;
            if (l < n) ev_cswap(a, i, l);
        }
        ev_sync();
        for (uint32_t j = hk >> 1; j > 0; j >>= 1) {         // half-cleaners
            for (uint32_t t = lane; t < half; t += 64) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1)), l = i + j;
                if (l < n) ev_cswap(a, i, l);
            }
            ev_sync();
        }
    }
}

__global__ __launch_bounds__(64 * EV_WAVES) void k_ev_sort(long long P, const uint32_t* __restrict__ evoff,
                                                           uint32_t* __restrict__ scratch,
                                                           uint32_t* __restrict__ distinct)
{
    __shared__ uint32_t lds[EV_WAVES][EV_LDS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * EV_WAVES + w;
    if (p >= P) return;                                      // whole wavefront; no block barrier below
    const uint32_t lo = evoff[p], n = evoff[p + 1] - lo;
    uint32_t* seg = scratch + lo;
    uint32_t* a = seg;
    if (n <= (uint32_t)EV_LDS) {
        a = lds[w];
        for (uint32_t i = lane; i < n; i += 64) a[i] = seg[i];
        ev_sync();
    }
    ev_bitonic(a, n);
    uint32_t heads = 0;
    for (uint32_t i = lane; i < n; i += 64) heads += (i == 0 || a[i] != a[i - 1]) ? 1u : 0u;
    if (a != seg)
        for (uint32_t i = lane; i < n; i += 64) seg[i] = a[i];
    heads = wave_sum(heads);
    if (lane == 0) distinct[p] = heads;
}

// Run-length encodes pixel p's sorted segment into ent[off[p] ..].  Chunks of
// 64 bins: a run ends at lane i when the next bin differs; its start is the
// last run head at or before i (from the chunk's head ballot, or carried from
// earlier chunks).  A count above 65535 is stored as 65535 and flags
// E_INVALID (it does not fit the entry's 16-bit count).
__global__ __launch_bounds__(64 * EV_WAVES) void k_ev_rle(long long P, const uint32_t* __restrict__ evoff,
                                                          const uint32_t* __restrict__ scratch,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t* __restrict__ ent, uint64_t cap,
                                                          int32_t* __restrict__ err)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * EV_WAVES + w;
    if (p >= P) return;
    const uint32_t lo = evoff[p], n = evoff[p + 1] - lo;
    const uint32_t* seg = scratch + lo;
    const uint64_t base = off[p];
    const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= this one
    uint32_t runs = 0, carry = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += 64) {                // uniform over the wavefront
        const uint32_t i = c0 + lane;
        const bool in = i < n;
        const uint32_t v = in ? seg[i] : EV_INF;
        const uint32_t pv = (in && i > 0) ? seg[i - 1] : EV_INF;
        const uint32_t nv = (i + 1 < n) ? seg[i + 1] : EV_INF;
        const bool head = in && (i == 0 || v != pv);
        const bool last = in && v != nv;
        const uint64_t hm = __ballot(head);
        const uint64_t mh = hm & le;
        if (last) {
            const uint32_t start = mh ? c0 + 63u - (uint32_t)__clzll(mh) : carry;
            const uint32_t cnt = i + 1 - start;
            const uint64_t pos = base + runs + (uint64_t)__popcll(mh) - 1u;   // >= base: chunk 0 starts with a head
            if (cnt > 0xffffu) *err = RT3D_E_INVALID;
            if (pos < cap) ent[pos] = (v << 16) | (cnt > 0xffffu ? 0xffffu : cnt);
            else *err = RT3D_E_CAPACITY;
        }
        if (hm) carry = c0 + 63u - (uint32_t)__clzll(hm);
        runs += (uint32_t)__popcll(hm);
    }
}

hipError_t launch_compact_events(const uint32_t* pix, const uint16_t* bin, uint64_t n, long long P, int T,
                                 uint32_t* evoff, uint32_t* scratch, uint32_t* off, uint32_t* ent, uint64_t cap,
                                 uint32_t* counts, uint32_t* partial, int32_t* err, hipStream_t st)
{
    if (P <= 0) return hipSuccess;
    const long long zn = (P + EV_THREADS - 1) / EV_THREADS;
    const unsigned zb = (unsigned)(zn < 4096 ? zn : 4096);
    const unsigned eb = (unsigned)((n + EV_THREADS - 1) / EV_THREADS);
    const unsigned pb = (unsigned)((P + EV_WAVES - 1) / EV_WAVES);
    hipLaunchKernelGGL(k_ev_zero, dim3(zb), dim3(EV_THREADS), 0, st, counts, P);
    if (eb) hipLaunchKernelGGL(k_ev_count, dim3(eb), dim3(EV_THREADS), 0, st, pix, bin, n, P, T, counts, err);
    hipError_t e = launch_scan(counts, evoff, P, partial, ~0ull, err, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ev_zero, dim3(zb), dim3(EV_THREADS), 0, st, counts, P);
    if (eb)
        hipLaunchKernelGGL(k_ev_scatter, dim3(eb), dim3(EV_THREADS), 0, st, pix, bin, n, P, T, evoff, counts,
                           scratch);
    hipLaunchKernelGGL(k_ev_sort, dim3(pb), dim3(64 * EV_WAVES), 0, st, P, evoff, scratch, counts);
    e = launch_scan(counts, off, P, partial, cap, err, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ev_rle, dim3(pb), dim3(64 * EV_WAVES), 0, st, P, evoff, scratch, off, ent, cap, err);
    return hipGetLastError();
}

}  // namespace rt3d

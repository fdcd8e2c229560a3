// rt3d_host.cpp -- host runtime behind the C ABI of include/rt3d.h: argument
// checks, the IRF tables (built in FP64), workspace carving and the launch
// sequence of one reconstruction.  Nothing here synchronises the caller's
// stream except rt3d_query and rt3d_create's table upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rt3d_dev.h"
#include "rt3d_cnn.h"

namespace rt3d {
size_t init_lds_bytes(int T, int L, int o, int r_init, bool wide = false);
size_t init_list_words(long long P);
}

using namespace rt3d;

// Everything the kernels need to know about one IRF (host facts and the
// device tables it owns).
struct IrfTables {
    int L = 0, o = 0;
    double sigma2 = 0.0, fisher = 0.0;
    int s_np = 0;                      // pieces of S over all segments (0: direct summation)
    std::vector<double> s_tab;         // breakpoints then piece coefficients (see DevModel)
    double s_v0 = 0, s_d0 = 0, s_v1 = 0, s_d1 = 0;
    int wl = 0, wr = 0, wnms = 0;
    double dmax = 0.0, dmerge = 0.0;
    std::vector<double> hbar;
    float4* d_cr = nullptr;
    double* d_stab = nullptr;
    int32_t* d_q = nullptr;
    int32_t* d_qst = nullptr;
    double* d_hbar = nullptr;
};

struct rt3d_ctx {
    rt3d_params p{};
    int T = 0, apss_R = 0;
    // IRF classes: 0 is rt3d_create's, later ones rt3d_add_irf's (per-pixel IRFs)
    std::vector<IrfTables> irf;
    const uint8_t* debug_cls = nullptr;   // class map of the step-by-step entry points
    int device = 0;
    float* d_bw = nullptr;
    int rb = 0;
    // workspace (caller's)
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    long long ws_P = 0;
    uint32_t ws_rows = 1, ws_cols = 1;
    unsigned ws_cnn_groups = 0;        // weight-gradient partial groups the workspace holds
    uint64_t ws_E = 0;
    // last call facts
    long long last_P = 0;
    bool last_compacted = false;
    // the batch layout whose final state the workspace holds (warm starts)
    std::vector<long long> state_layout;
    // rt3d_autotune's choices: (frames, rows, cols, fused, lanes per pixel)
    std::vector<std::array<long long, 5>> tuned;
    int force_fused = -2;              // set by rt3d_autotune while it times one mapping
    int force_lanes = 0;
    int cur_lpp = 4;                   // lanes per pixel of the gradient steps for the call being enqueued
    // learned denoiser weights (always allocated; zero until set)
    CnnWeights cnn;
    bool cnn_set = false;
    // kernel timing (rt3d_profile)
    int prof_id = -1;
    std::vector<hipEvent_t> prof_ev;   // start/end pairs
    size_t prof_n = 0;                 // pairs recorded since the last read
    std::string err;
};

namespace {

constexpr size_t ALIGN = 256;
// pieces of the table of S beyond which the gradient kernels sum S directly
constexpr int S_PIECES_MAX = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Workspace {
    uint32_t* off;
    uint32_t* ent;
    uint32_t* counts;
    uint32_t* partial;
    uint32_t* evoff;
    uint32_t* stage;
    uint32_t* cls_list;                // per-class pixel lists (per-pixel IRFs)
    uint32_t* cls_meta;
    uint32_t* wide;                    // the init's list of pixels with large pools (segment counters first)
    DevState A, B;
    float* btmp;
    CnnBuffers cnn;
    int32_t* err;
    size_t bytes;
};

// Carves the workspace for P pixels (Ps >= P of them in the point state:
// more under super-resolution) and E entries; with base == nullptr it only
// measures.
Workspace carve(uint8_t* base, long long P, long long Ps, uint64_t E, bool with_cnn = false, unsigned cnn_groups = 0)
{
    Workspace w{};
    size_t at = 0;
    auto take = [&](size_t bytes) -> uint8_t* {
        uint8_t* ptr = base ? base + at : nullptr;
        at += align_up(bytes);
        return ptr;
    };
    w.err = (int32_t*)take(sizeof(int32_t) * 4);
    w.off = (uint32_t*)take(sizeof(uint32_t) * (P + 1));
    w.ent = (uint32_t*)take(sizeof(uint32_t) * std::max<uint64_t>(E, 1));
    w.counts = (uint32_t*)take(sizeof(uint32_t) * std::max<long long>(Ps, 1));
    w.partial = (uint32_t*)take(sizeof(uint32_t) * scan_partial_elems(Ps));
    w.evoff = (uint32_t*)take(sizeof(uint32_t) * (P + 1));
    w.stage = (uint32_t*)take(sizeof(uint32_t) * CP_STAGE * std::max<long long>(P, 1));
    w.cls_list = (uint32_t*)take(sizeof(uint32_t) * std::max<long long>(P, 1));
    w.cls_meta = (uint32_t*)take(sizeof(uint32_t) * CLASS_META);
    w.wide = (uint32_t*)take(sizeof(uint32_t) * init_list_words(P));
    for (DevState* s : {&w.A, &w.B}) {
        s->t = (double*)take(sizeof(double) * KM * Ps);
        s->r = (float*)take(sizeof(float) * KM * Ps);
        s->n = (float*)take(sizeof(float) * 3 * KM * Ps);
        s->cnt = (uint8_t*)take(Ps);
        s->b = (float*)take(sizeof(float) * Ps);
    }
    w.btmp = (float*)take(sizeof(float) * P);
    if (with_cnn) {
        const size_t nb = (size_t)((P + 255) / 256);
        w.cnn.act[0] = (__half*)take(sizeof(__half) * 16 * P);
        for (int l = 1; l <= 3; ++l) w.cnn.act[l] = (__half*)take(sizeof(__half) * 32 * P);
        w.cnn.act[4] = (__half*)take(sizeof(__half) * 16 * P);
        w.cnn.dy16 = (__half*)take(sizeof(__half) * 16 * P);
        w.cnn.dA = (__half*)take(sizeof(__half) * 32 * P);
        w.cnn.dB = (__half*)take(sizeof(__half) * 32 * P);
        w.cnn.tgt = (float*)take(sizeof(float) * 3 * P);
        w.cnn.msk = (uint8_t*)take(3 * P);
        w.cnn.lpart = (float*)take(sizeof(float) * 2 * nb);
        w.cnn.part = (float*)take(sizeof(float) * (size_t)cnn_groups * 9 * 32 * 32);
        w.cnn.bpart = (float*)take(sizeof(float) * (size_t)cnn_groups * 32);
        w.cnn.grad = (float*)take(sizeof(float) * CNN_PARAMS);
    }
    w.bytes = at;
    return w;
}

// Tables of one IRF (normalised samples, Catmull-Rom segments, the piecewise
// cubic of S, the shift Fisher information, peak windows, log-matched-filter
// weights and their range maxima), built in FP64 and uploaded to the current
// device.  E_INVALID for an unusable IRF, E_DEVICE on a HIP failure (what was
// allocated is in t for free_irf).
// The host-side checks of an IRF (no device call).
rt3d_status check_irf(const double* irf, uint32_t irf_len, int32_t irf_origin, int T, const rt3d_params* p)
{
    if (!irf || irf_len == 0 || irf_len > (uint32_t)T) return RT3D_E_INVALID;
    double sum = 0.0;
    for (uint32_t k = 0; k < irf_len; ++k) {
        if (!std::isfinite(irf[k]) || irf[k] < 0.0) return RT3D_E_INVALID;
        sum += irf[k];
    }
    if (!(sum > 0.0)) return RT3D_E_INVALID;
    if (irf_origin >= (int32_t)irf_len) return RT3D_E_INVALID;
    // the origin is not known before the IRF is normalised: its largest value
    if (init_lds_bytes(T, (int)irf_len, (int)irf_len - 1, p->r_init) > 65536) return RT3D_E_UNSUPPORTED;
    return RT3D_OK;
}

rt3d_status build_irf(const double* irf, uint32_t irf_len, int32_t irf_origin, int T, const rt3d_params* p,
                      IrfTables& t)
{
    const rt3d_status ok = check_irf(irf, irf_len, irf_origin, T, p);
    if (ok != RT3D_OK) return ok;
    double sum = 0.0;
    for (uint32_t k = 0; k < irf_len; ++k) sum += irf[k];
    t.L = (int)irf_len;
    t.hbar.resize(irf_len);
    for (uint32_t k = 0; k < irf_len; ++k) t.hbar[k] = irf[k] / sum;
    if (irf_origin < 0) {
        int best = 0;
        for (int k = 1; k < t.L; ++k)
            if (t.hbar[k] > t.hbar[best]) best = k;
        irf_origin = best;
    }
    t.o = irf_origin;
    // moments and windows of the normalised IRF
    double mu = 0.0;
    for (int k = 0; k < t.L; ++k) mu += k * t.hbar[k];
    double var = 0.0;
    for (int k = 0; k < t.L; ++k) var += t.hbar[k] * (k - mu) * (k - mu);
    t.sigma2 = var;
    const double sh = std::sqrt(var);
    {
        double acc = 0.0;
        int lo = -1, hi = -1;
        for (int k = 0; k < t.L; ++k) {
            acc += t.hbar[k];
            if (lo < 0 && acc >= 0.05) lo = k;
            if (hi < 0 && acc >= 0.95) hi = k;
        }
        if (lo < 0) lo = 0;
        if (hi < 0) hi = t.L - 1;
        t.wl = std::max(0, t.o - lo);
        t.wr = std::max(0, hi - t.o);
    }
    t.wnms = p->w_nms > 0 ? p->w_nms : (int)std::ceil(std::max(1.0, 2.0 * sh));
    t.dmerge = p->d_merge > 0 ? p->d_merge : std::max(1.0, sh);

    const int L = t.L;
    // Catmull-Rom cubic of each segment between samples k and k+1, k = -1..L-1
    // (samples beyond the IRF are zero): value c0 + c1 s + c2 s^2 + c3 s^3
    auto hb = [&](int k) { return (k >= 0 && k < L) ? t.hbar[k] : 0.0; };
    std::vector<float4> cr(L + 1);
    std::vector<double> crd((size_t)4 * (L + 1));
    for (int k = -1; k < L; ++k) {
        const double p0 = hb(k - 1), p1 = hb(k), p2 = hb(k + 1), p3 = hb(k + 2);
        double* d = &crd[(size_t)4 * (k + 1)];
        d[0] = p1;
        d[1] = 0.5 * (p2 - p0);
        d[2] = p0 - 2.5 * p1 + 2.0 * p2 - 0.5 * p3;
        d[3] = 0.5 * (p3 - p0) + 1.5 * (p1 - p2);
        cr[k + 1] = make_float4((float)d[0], (float)d[1], (float)d[2], (float)d[3]);
    }
    // S and S' of points whose IRF support lies inside the domain, as a
    // piecewise cubic in the local parameter s that every segment shares:
    // between consecutive zeros (in (0, 1)) of the segments' cubics each
    // segment keeps its sign, so the sum of the segments clamped at zero is
    // one cubic per piece.  At s = 0 and s = 1 segments whose value is not
    // positive drop out with their slope; those sums are kept apart.
    {
        std::vector<double> brk = {0.0, 1.0};
        for (int j = 0; j <= L; ++j) {
            const double* d = &crd[(size_t)4 * j];
            auto val = [&](double x) { return ((d[3] * x + d[2]) * x + d[1]) * x + d[0]; };
            // monotone stretches of [0, 1] between the slope's zeros, each
            // bisected where the cubic changes sign
            std::vector<double> cut = {0.0, 1.0};
            const double A = 3.0 * d[3], B = 2.0 * d[2], Cc = d[1];
            if (A != 0.0) {
                const double disc = B * B - 4.0 * A * Cc;
                if (disc >= 0.0) {
                    const double r = std::sqrt(disc);
                    for (double x : {(-B - r) / (2.0 * A), (-B + r) / (2.0 * A)})
                        if (x > 0.0 && x < 1.0) cut.push_back(x);
                }
            } else if (B != 0.0) {
                const double x = -Cc / B;
                if (x > 0.0 && x < 1.0) cut.push_back(x);
            }
            std::sort(cut.begin(), cut.end());
            for (size_t u = 0; u + 1 < cut.size(); ++u) {
                double lo = cut[u], hi = cut[u + 1];
                double flo = val(lo), fhi = val(hi);
                if (!((flo < 0.0 && fhi > 0.0) || (flo > 0.0 && fhi < 0.0))) continue;
                for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    const double fm = val(mid);
                    if ((fm < 0.0) == (flo < 0.0)) {
                        lo = mid;
                        flo = fm;
                    } else {
                        hi = mid;
                    }
                }
                brk.push_back(0.5 * (lo + hi));
            }
        }
        std::sort(brk.begin(), brk.end());
        brk.erase(std::unique(brk.begin(), brk.end()), brk.end());
        std::vector<double> coef;
        for (size_t u = 0; u + 1 < brk.size(); ++u) {
            const double mid = 0.5 * (brk[u] + brk[u + 1]);
            double cs[4] = {0, 0, 0, 0};
            for (int j = 0; j <= L; ++j) {
                const double* d = &crd[(size_t)4 * j];
                if (((d[3] * mid + d[2]) * mid + d[1]) * mid + d[0] > 0.0)
                    for (int i = 0; i < 4; ++i) cs[i] += d[i];
            }
            coef.insert(coef.end(), cs, cs + 4);
        }
        for (int j = 0; j <= L; ++j) {
            const double* d = &crd[(size_t)4 * j];
            if (d[0] > 0.0) {
                t.s_v0 += d[0];
                t.s_d0 += d[1];
            }
            const double v1 = d[0] + d[1] + d[2] + d[3];
            if (v1 > 0.0) {
                t.s_v1 += v1;
                t.s_d1 += d[1] + 2.0 * d[2] + 3.0 * d[3];
            }
        }
        const int np = (int)brk.size() - 1;
        if (np >= 1 && np <= S_PIECES_MAX) {
            t.s_np = np;
            t.s_tab = brk;
            t.s_tab.insert(t.s_tab.end(), coef.begin(), coef.end());
        }
    }
    // shift Fisher information of one photon (no background), averaged over 32
    // sub-bin phases, over lags where h is at least 1e-3 of the largest sample
    {
        double hmax = 0.0;
        for (int k = 0; k < L; ++k) hmax = std::max(hmax, t.hbar[k]);
        double acc = 0.0;
        for (int j = 0; j < 32; ++j) {
            for (int l = -t.o - 1; l <= L - t.o; ++l) {
                const double x = l + j / 32.0 + t.o;
                if (!(x > -1.0) || !(x < L)) continue;
                const int k = (int)std::floor(x);
                const double sl = x - k;
                const double* d = &crd[(size_t)4 * (k + 1)];
                const double h = ((d[3] * sl + d[2]) * sl + d[1]) * sl + d[0];
                if (!(h > 0.0) || h < 1e-3 * hmax) continue;
                const double hp = (3.0 * d[3] * sl + 2.0 * d[2]) * sl + d[1];
                acc += hp * hp / h;
            }
        }
        t.fisher = acc / 32.0;
    }
    if (!(t.fisher > 0.0)) return RT3D_E_INVALID;
    t.dmax = p->dmax > 0 ? p->dmax : std::max(0.5, 1.0 / std::sqrt(t.fisher));
    // log-matched filter weights, 16 fractional bits
    std::vector<int32_t> q(L);
    const double inv_eps = p->sbr_guess * (double)T;
    for (int k = 0; k < L; ++k) q[k] = (int32_t)std::llround(std::log1p(t.hbar[k] * inv_eps) * 65536.0);
    // range-maximum table of q: level l holds max q[k .. k + 2^l - 1]
    int nlev = 1;
    while ((1 << nlev) <= L) ++nlev;
    std::vector<int32_t> qst((size_t)nlev * L);
    for (int k = 0; k < L; ++k) qst[k] = q[k];
    for (int l = 1; l < nlev; ++l)
        for (int k = 0; k < L; ++k) {
            const int a = qst[(size_t)(l - 1) * L + k];
            const int k2 = k + (1 << (l - 1));
            const int b = k2 < L ? qst[(size_t)(l - 1) * L + k2] : a;
            qst[(size_t)l * L + k] = std::max(a, b);
        }
    hipError_t e = hipMalloc(&t.d_cr, sizeof(float4) * cr.size());
    if (e == hipSuccess) e = hipMalloc(&t.d_q, sizeof(int32_t) * q.size());
    if (e == hipSuccess) e = hipMalloc(&t.d_qst, sizeof(int32_t) * qst.size());
    if (e == hipSuccess) e = hipMalloc(&t.d_hbar, sizeof(double) * L);
    if (e == hipSuccess && t.s_np > 0) e = hipMalloc(&t.d_stab, sizeof(double) * t.s_tab.size());
    if (e == hipSuccess && t.s_np > 0)
        e = hipMemcpy(t.d_stab, t.s_tab.data(), sizeof(double) * t.s_tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.d_cr, cr.data(), sizeof(float4) * cr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.d_q, q.data(), sizeof(int32_t) * q.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.d_qst, qst.data(), sizeof(int32_t) * qst.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.d_hbar, t.hbar.data(), sizeof(double) * L, hipMemcpyHostToDevice);
    return e == hipSuccess ? RT3D_OK : RT3D_E_DEVICE;
}

void free_irf(IrfTables& t)
{
    for (void* ptr : {(void*)t.d_cr, (void*)t.d_stab, (void*)t.d_q, (void*)t.d_qst, (void*)t.d_hbar})
        if (ptr) (void)hipFree(ptr);
    t.d_cr = nullptr;
    t.d_stab = nullptr;
    t.d_q = nullptr;
    t.d_qst = nullptr;
    t.d_hbar = nullptr;
}

rt3d_status fail(rt3d_ctx* c, rt3d_status st, const std::string& msg)
{
    if (c) c->err = msg;
    return st;
}

rt3d_status hip_fail(rt3d_ctx* c, hipError_t e, const char* what)
{
    return fail(c, RT3D_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t PROF_MAX = 4096;

// Starts timing a launch of kernel group `id` when it is the profiled one.
bool prof_begin(rt3d_ctx* c, int id, hipStream_t st, size_t& slot)
{
    if (c->prof_id != id || c->prof_n >= PROF_MAX) return false;
    while (c->prof_ev.size() < 2 * (c->prof_n + 1)) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return false;
        c->prof_ev.push_back(ev);
    }
    slot = c->prof_n++;
    return hipEventRecord(c->prof_ev[2 * slot], st) == hipSuccess;
}

// Launch of kernel group `id`, timed when profiled.
#define RT3D_LAUNCH(ctx, id, st, call)                                          \
    do {                                                                        \
        size_t slot_ = 0;                                                       \
        const bool on_ = prof_begin(ctx, id, st, slot_);                        \
        hipError_t e_ = (call);                                                 \
        if (on_) (void)hipEventRecord((ctx)->prof_ev[2 * slot_ + 1], st);       \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);                  \
    } while (0)

#define RT3D_HIP(ctx, call)                                      \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);   \
    } while (0)

// The model of IRF class k; with a per-pixel class map `cls`, a launch with
// it touches only the pixels of class k (class numbers past the context's
// classes count as 0).
DevModel dev_model(const rt3d_ctx* c, int k = 0, const uint8_t* cls = nullptr, const uint32_t* lst = nullptr,
                   const uint32_t* lst_meta = nullptr)
{
    const IrfTables& t = c->irf[k];
    DevModel m{};
    m.cr = t.d_cr;
    m.q = t.d_q;
    m.qst = t.d_qst;
    m.hbar = t.d_hbar;
    m.T = c->T;
    m.L = t.L;
    m.o = t.o;
    m.wl = t.wl;
    m.wr = t.wr;
    m.wnms = t.wnms;
    m.sigma2 = (float)t.sigma2;
    m.fisher_inv = (float)(1.0 / t.fisher);
    m.s_np = t.s_np;
    m.s_tab = t.d_stab;
    m.s_v0 = t.s_v0;
    m.s_d0 = t.s_d0;
    m.s_v1 = t.s_v1;
    m.s_d1 = t.s_d1;
    m.cls = cls;
    m.cls_id = k;
    m.n_cls = (int)c->irf.size();
    m.lst = cls ? lst : nullptr;
    m.lst_meta = cls ? lst_meta : nullptr;
    return m;
}

DevParams dev_params(const rt3d_ctx* c, int k = 0)
{
    DevParams d{};
    const rt3d_params& p = c->p;
    d.k_max = p.k_max;
    d.k_init = p.k_init;
    d.r_init = p.r_init;
    d.n_min = p.n_min;
    d.m_min = p.m_min;
    d.apss_R = c->apss_R;
    d.apss_Rs = apss_staged_halo(p.h_apss, p.p_xy, c->apss_R);
    d.lpp = c->cur_lpp;
    d.ilp_box = p.ilp_box;
    d.p_xy = p.p_xy;
    d.dz = p.dz;
    d.h_apss = p.h_apss;
    d.h_int = p.h_int;
    d.beta_t = p.beta_t;
    d.dmax = c->irf[k].dmax;
    d.beta_r = p.beta_r;
    d.beta_b = p.beta_b;
    d.r_min = p.r_min;
    d.d_merge = c->irf[k].dmerge;
    d.b_min = p.b_min;
    d.kappa = p.kappa;
    d.persp = p.persp;
    return d;
}

rt3d_status check_params(const rt3d_params* p, uint32_t bins, std::string& why)
{
    if (!p) { why = "params is NULL"; return RT3D_E_INVALID; }
    if (p->struct_size != sizeof(rt3d_params)) { why = "params.struct_size mismatch"; return RT3D_E_INVALID; }
    if (p->n_iter < 0) { why = "n_iter < 0"; return RT3D_E_INVALID; }
    if (p->k_max < 1 || p->k_max > RT3D_K_MAX) { why = "k_max outside 1..RT3D_K_MAX"; return RT3D_E_INVALID; }
    if (p->k_init < 1 || p->k_init > p->k_max) { why = "k_init outside 1..k_max"; return RT3D_E_INVALID; }
    if (!(p->p_xy > 0) || !(p->dz > 0) || !(p->h_apss > 0) || !(p->h_int >= 0)) {
        why = "p_xy, dz, h_apss must be > 0 and h_int >= 0"; return RT3D_E_INVALID;
    }
    if (!(p->b_min > 0)) { why = "b_min must be > 0"; return RT3D_E_INVALID; }
    if (!(p->sigma_b >= 0) || p->sigma_b > 64) { why = "sigma_b outside [0, 64]"; return RT3D_E_INVALID; }
    if (!(p->sbr_guess > 0)) { why = "sbr_guess must be > 0"; return RT3D_E_INVALID; }
    if (p->r_init < 0 || p->r_init > 8) { why = "r_init outside 0..8"; return RT3D_E_INVALID; }
    if (p->fused_loop < -1 || p->fused_loop > 1) { why = "fused_loop must be -1, 0 or 1"; return RT3D_E_INVALID; }
    if (p->ilp_box != 0 && p->ilp_box != 1) { why = "ilp_box must be 0 or 1"; return RT3D_E_INVALID; }
    if (p->lanes_per_pixel != 0 && p->lanes_per_pixel != 4 && p->lanes_per_pixel != 8) {
        why = "lanes_per_pixel must be 0, 4 or 8";
        return RT3D_E_INVALID;
    }
    if (p->sr < 1 || p->sr > SR_MAX) { why = "sr outside 1..4"; return RT3D_E_INVALID; }
    if (p->sr > 1 && p->denoiser == RT3D_DENOISE_CNN) {
        why = "super-resolution with the learned denoiser"; return RT3D_E_UNSUPPORTED;
    }
    if (p->denoiser != RT3D_DENOISE_APSS && p->denoiser != RT3D_DENOISE_NONE && p->denoiser != RT3D_DENOISE_CNN) {
        why = "unknown denoiser"; return RT3D_E_UNSUPPORTED;
    }
    if (std::ceil(p->h_apss / p->p_xy) > 16) { why = "h_apss / p_xy above 16 pixels"; return RT3D_E_UNSUPPORTED; }
    if (!std::isfinite(p->persp) || p->persp < 0) { why = "persp must be finite and >= 0"; return RT3D_E_INVALID; }
    if (p->persp > 0 && apss_lds_bytes((int)std::ceil(p->h_apss / p->p_xy)) > 65536) {
        why = "the perspective camera's APSS window does not fit the tile kernel (R > 5)"; return RT3D_E_UNSUPPORTED;
    }
    if (!(p->beta_t >= 0) || !(p->beta_r >= 0) || !(p->beta_b >= 0)) { why = "negative step scale"; return RT3D_E_INVALID; }
    if (!std::isfinite(p->r_min) || !std::isfinite(p->kappa) || p->kappa < 0) {
        why = "r_min / kappa not finite or kappa < 0"; return RT3D_E_INVALID;
    }
    (void)bins;
    return RT3D_OK;
}

bool uses_cnn(const rt3d_ctx* c) { return c->p.denoiser == RT3D_DENOISE_CNN; }

// Workspace of a context for P pixels of rows x cols frames and E entries.
Workspace carve_ctx(const rt3d_ctx* c, uint8_t* base, long long P, uint64_t E, uint32_t rows, uint32_t cols)
{
    unsigned groups = 0;
    if (uses_cnn(c)) {
        Shape sh;
        sh.rows = (int)rows;
        sh.cols = (int)cols;
        sh.F = (int)(P / ((long long)rows * cols));
        sh.P = P;
        sh.S = P;
        groups = cnn_wgrad_groups(sh);
    }
    const long long sr = c->p.sr;
    return carve(base, P, P * sr * sr, E, uses_cnn(c), groups);
}

rt3d_status need_ws(rt3d_ctx* c, long long P, Workspace& w)
{
    c->state_layout.clear();     // a reconstruction sets it again once it has enqueued its output
    if (!c->ws) return fail(c, RT3D_E_NOMEM, "no workspace bound (rt3d_set_workspace)");
    if (P > c->ws_P) return fail(c, RT3D_E_NOMEM, "batch larger than the workspace was sized for");
    w = carve_ctx(c, c->ws, c->ws_P, c->ws_E, c->ws_rows, c->ws_cols);
    return RT3D_OK;
}

bool state_ok(const rt3d_state* s)
{
    return s && s->t && s->r && s->n && s->cnt && s->b && s->frames && s->rows && s->cols;
}

DevState dev_state(const rt3d_state* s) { return DevState{s->t, s->r, s->n, s->cnt, s->b}; }

bool shape_ok(uint32_t F, uint32_t rows, uint32_t cols)
{
    const long long P = (long long)F * rows * cols;
    return P > 0 && P < (1ll << 31) && (long long)rows * cols < (1ll << 31);
}

Shape shape_of(uint32_t F, uint32_t rows, uint32_t cols)
{
    Shape sh;
    sh.F = (int)F;
    sh.rows = (int)rows;
    sh.cols = (int)cols;
    sh.P = (long long)F * rows * cols;
    sh.S = sh.P;
    return sh;
}

// A run of consecutive frames of one size within a batch: its first pixel and
// its shape (slot stride = the whole batch's pixel count).
struct Group {
    long long base;
    Shape sh;
};

// Whether a batch can run every iteration in one launch (APSS, frames of one
// size of at most LOOP_MAX_PIX pixels), and whether it does.
bool loop_eligible(const rt3d_ctx* c, const std::vector<Group>& groups, const Shape& sh)
{
    return c->p.denoiser == RT3D_DENOISE_APSS && groups.size() == 1 && !(c->p.persp > 0) &&
           (long long)sh.rows * sh.cols <= LOOP_MAX_PIX;
}

bool use_fused(const rt3d_ctx* c, const Shape& sh)
{
    if (c->force_fused >= 0) return c->force_fused == 1;
    if (c->p.fused_loop >= 0) return c->p.fused_loop == 1;
    for (const auto& t : c->tuned)
        if (t[0] == sh.F && t[1] == sh.rows && t[2] == sh.cols) return t[3] == 1;
    return sh.F >= 64;
}

// Lanes per pixel of the gradient steps for a batch of P pixels (sh: its
// shape when every frame has one size): forced by the autotuner while it
// times, else params.lanes_per_pixel, else its choice for the batch shape,
// else eight lanes below LANES8_PIXELS pixels (four lanes leave most of the
// chip idle there) and four above.
constexpr long long LANES8_PIXELS = 131072;

int lanes_for(const rt3d_ctx* c, long long P, const Shape* sh)
{
    if (c->force_lanes) return c->force_lanes;
    if (c->p.lanes_per_pixel) return c->p.lanes_per_pixel;
    if (sh)
        for (const auto& t : c->tuned)
            if (t[0] == sh->F && t[1] == sh->rows && t[2] == sh->cols) return (int)t[4];
    return P < LANES8_PIXELS ? 8 : 4;
}

// IRF classes a call launches its IRF-dependent kernels for: every class of
// the context with a per-pixel class map, else class 0 alone.
int n_classes(const rt3d_ctx* c, const uint8_t* cls) { return cls ? (int)c->irf.size() : 1; }

// One iteration of the loop on state A (in/out) with B as the second buffer.
// Per-pixel steps run once over the batch (sh), once per IRF class with a
// class map cls; steps that read neighbouring pixels run once per group of
// equally sized frames.
// The inference buffers of the learned denoiser for the pixels from `base` on.
CnnBuffers cnn_at(const CnnBuffers& b, long long base)
{
    CnnBuffers r = b;
    r.act[0] += base * 16;
    r.act[4] += base * 16;
    return r;
}

// One iteration on the state whose planes `cur` points at; `alt` holds the
// other buffer of each plane.  Kernels that read neighbours' values write the
// planes they change to the other buffer (APSS: depths and normals; the
// intensity filter: depths, intensities and counts), kernels that read only
// their own pixel write in place, and the two sets of pointers are swapped
// plane by plane, so no kernel copies a plane it does not change.
rt3d_status iterate(rt3d_ctx* c, const Shape& sh, const std::vector<Group>& groups, const uint32_t* off,
                    const uint32_t* ent, const float* gain, DevState& cur, DevState& alt, float* btmp,
                    const CnnBuffers* cnn, const uint8_t* cls, hipStream_t st, const uint32_t* lst = nullptr,
                    const uint32_t* lst_meta = nullptr)
{
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    const int nc = n_classes(c, cls);
    for (int k = 0; k < nc; ++k)
        RT3D_LAUNCH(c, RT3D_KERNEL_DEPTH, st,
                    launch_depth_step(dev_model(c, k, cls, lst, lst_meta), dev_params(c, k), sh, off, ent, gain, cur,
                                      st));
    // the groups as tile tables of at most TILE_GROUPS groups (one launch each)
    std::vector<Tiles> tiles(1, Tiles{});
    for (const Group& g : groups)
        if (!tiles_add(tiles.back(), g.base, g.sh)) {
            tiles.push_back(Tiles{});
            tiles_add(tiles.back(), g.base, g.sh);
        }
    if (c->p.denoiser == RT3D_DENOISE_APSS) {
        DevState out = cur;
        out.t = alt.t;
        out.n = alt.n;
        for (const Tiles& tg : tiles)
            RT3D_LAUNCH(c, RT3D_KERNEL_APSS, st, launch_apss_tiles(m, p, tg, cur, out, -1, false, st));
        std::swap(cur.t, alt.t);
        std::swap(cur.n, alt.n);
    } else if (c->p.denoiser == RT3D_DENOISE_CNN) {
        // APSS only for pixels holding more points than the network's three
        // slots, then the network on each group of equal-size frames
        for (const Tiles& tg : tiles)
            RT3D_LAUNCH(c, RT3D_KERNEL_APSS, st, launch_apss_tiles(m, p, tg, cur, alt, 3, true, st));
        const float sig = (float)std::sqrt(c->irf[0].sigma2);
        for (const Group& g : groups) {
            const CnnBuffers b = cnn_at(*cnn, g.base);
            const DevState ga = state_at(alt, g.base);
            RT3D_LAUNCH(c, RT3D_KERNEL_CNN, st, launch_cnn_infer(g.sh, ga, sig, c->cnn, b, st));
            RT3D_HIP(c, launch_cnn_apply(g.sh, b, sig, (double)(c->T - 1), ga, st));
        }
        std::swap(cur, alt);
    } else {
        RT3D_HIP(c, launch_copy_state(sh, cur, alt, st));
        std::swap(cur, alt);
    }
    // the in-pixel merge runs fused ahead of the intensity step
    for (int k = 0; k < nc; ++k)
        RT3D_LAUNCH(c, RT3D_KERNEL_INTENSITY, st,
                    launch_intensity_step(dev_model(c, k, cls, lst, lst_meta), dev_params(c, k), sh, off, ent, gain,
                                          cur, true, st));
    {   // normals and background move with their own pixel only: in place
        DevState out = cur;
        out.t = alt.t;
        out.r = alt.r;
        out.cnt = alt.cnt;
        for (const Tiles& tg : tiles)
            RT3D_LAUNCH(c, RT3D_KERNEL_IFILTER, st, launch_ifilter_tiles(p, tg, cur, out, st));
        std::swap(cur.t, alt.t);
        std::swap(cur.r, alt.r);
        std::swap(cur.cnt, alt.cnt);
    }
    // the background step writes btmp; the filter brings it back into cur.b
    for (int k = 0; k < nc; ++k)
        RT3D_LAUNCH(c, RT3D_KERNEL_BKG, st,
                    launch_bg_step(dev_model(c, k, cls, lst, lst_meta), dev_params(c, k), sh, off, ent, gain, cur,
                                   btmp, st));
    for (const Tiles& tg : tiles)
        RT3D_LAUNCH(c, RT3D_KERNEL_BFILTER, st,
                    launch_bfilter_tiles(c->d_bw, c->rb, tg, (float)c->p.b_min, btmp, cur.b, alt.b, st));
    return RT3D_OK;
}

// Copies the state whose planes `cur` points at into `home`, when any of its
// planes sits in the other buffer.
rt3d_status settle(rt3d_ctx* c, const Shape& sh, const DevState& cur, const DevState& home, hipStream_t st)
{
    if (cur.t == home.t && cur.r == home.r && cur.n == home.n && cur.cnt == home.cnt && cur.b == home.b)
        return RT3D_OK;
    RT3D_HIP(c, launch_copy_state(sh, cur, home, st));
    return RT3D_OK;
}

// The point grid of lidar frames `lid` under super-resolution factor sr.
Shape point_grid(const Shape& lid, int sr)
{
    Shape f = lid;
    f.rows = lid.rows * sr;
    f.cols = lid.cols * sr;
    f.P = (long long)f.F * f.rows * f.cols;
    f.S = f.P;
    return f;
}

// One iteration under super-resolution: the gradient steps per lidar pixel
// (lid), APSS, merge and intensity filter on the point grid (fsh), the
// background filter on the lidar grid (the lidar background is A.b[0 .. lid.P)).
rt3d_status iterate_sr(rt3d_ctx* c, const Shape& lid, const uint32_t* off, const uint32_t* ent, const float* gain,
                       DevState A, DevState B, float* btmp, hipStream_t st)
{
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    const int sr = c->p.sr;
    const Shape fsh = point_grid(lid, sr);
    RT3D_LAUNCH(c, RT3D_KERNEL_DEPTH, st,
                launch_sr_step(RT3D_STEP_DEPTH, m, p, lid, sr, fsh.P, off, ent, gain, A, nullptr, st));
    if (c->p.denoiser == RT3D_DENOISE_APSS)
        RT3D_LAUNCH(c, RT3D_KERNEL_APSS, st, launch_apss(m, p, fsh, A, B, -1, st));
    else
        RT3D_HIP(c, launch_copy_state(fsh, A, B, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_MERGE, st, launch_merge(m, p, fsh, B, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_INTENSITY, st,
                launch_sr_step(RT3D_STEP_INTENSITY, m, p, lid, sr, fsh.P, off, ent, gain, B, nullptr, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_IFILTER, st, launch_ifilter(p, fsh, B, A, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_BKG, st,
                launch_sr_step(RT3D_STEP_BKG, m, p, lid, sr, fsh.P, off, ent, gain, A, btmp, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_BFILTER, st,
                launch_bfilter(c->d_bw, c->rb, lid, (float)c->p.b_min, btmp, A.b, B.b, st));
    return RT3D_OK;
}

// Initialisation under super-resolution: the lidar-grid initialisation into
// B (slot stride lid.P), spread over the point grid into A, normals there.
rt3d_status init_sr(rt3d_ctx* c, const Shape& lid, const uint32_t* off, const uint32_t* ent, const float* gain,
                    DevState A, DevState B, uint32_t* wide, hipStream_t st)
{
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    const Shape fsh = point_grid(lid, c->p.sr);
    RT3D_LAUNCH(c, RT3D_KERNEL_INIT, st, launch_init(m, p, lid, off, ent, gain, B, wide, st));
    RT3D_HIP(c, launch_sr_expand(lid, c->p.sr, fsh.P, B, A, st));
    RT3D_LAUNCH(c, RT3D_KERNEL_NORMALS, st, launch_init_normals(p, fsh, A, st));
    return RT3D_OK;
}

}  // namespace

extern "C" {

void rt3d_params_default(rt3d_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(rt3d_params);
    p->n_iter = 20;
    p->k_max = 4;
    p->k_init = 3;
    p->p_xy = 1.0;
    p->dz = 0.1;
    p->h_apss = 2.0;
    p->h_int = 2.0;
    p->beta_t = 0.5;
    p->dmax = 0.0;
    p->beta_r = 1.0;
    p->beta_b = 1.0;
    p->r_min = 1.0;
    p->d_merge = 0.0;
    p->sigma_b = 2.0;
    p->b_min = 1e-8;
    p->sbr_guess = 1.0;
    p->r_init = 0;
    p->n_min = 2;
    p->kappa = 3.0;
    p->w_nms = 0;
    p->m_min = 3;
    p->denoiser = RT3D_DENOISE_APSS;
    p->fused_loop = -1;
    p->sr = 1;
    p->ilp_box = 0;
}

rt3d_status rt3d_create(const double* irf, uint32_t irf_len, int32_t irf_origin, uint32_t bins,
                        const rt3d_params* p, rt3d_ctx** out)
{
    if (!out) return RT3D_E_INVALID;
    *out = nullptr;
    if (!irf || irf_len == 0 || bins == 0 || bins > 65535 || irf_len > bins) return RT3D_E_INVALID;
    std::string why;
    rt3d_status ps = check_params(p, bins, why);
    if (ps != RT3D_OK) return ps;
    ps = check_irf(irf, irf_len, irf_origin, (int)bins, p);
    if (ps != RT3D_OK) return ps;

    rt3d_ctx* c = new (std::nothrow) rt3d_ctx();
    if (!c) return RT3D_E_NOMEM;
    c->p = *p;
    c->T = (int)bins;
    c->apss_R = (int)std::ceil(p->h_apss / p->p_xy);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return RT3D_E_DEVICE;
    }
    {   // the device address of the fixed compaction array on this GPU (rt3d_compact_noalloc)
        uint32_t* scratch_ptr = nullptr;
        if (noalloc_scratch(&scratch_ptr) != hipSuccess) {
            delete c;
            return RT3D_E_DEVICE;
        }
    }
    {
        c->irf.emplace_back();
        const rt3d_status bs = build_irf(irf, irf_len, irf_origin, c->T, p, c->irf[0]);
        if (bs != RT3D_OK) {
            rt3d_destroy(c);
            return bs;
        }
    }
    // background filter taps
    std::vector<float> bw;
    if (p->sigma_b > 0.0) {
        c->rb = (int)std::ceil(4.0 * p->sigma_b);
        std::vector<double> w(2 * c->rb + 1);
        double s = 0.0;
        for (int d = -c->rb; d <= c->rb; ++d) {
            w[d + c->rb] = std::exp(-(double)d * d / (2.0 * p->sigma_b * p->sigma_b));
            s += w[d + c->rb];
        }
        for (double v : w) bw.push_back((float)(v / s));
    } else {
        c->rb = 0;
        bw.push_back(1.0f);
    }

    hipError_t e = hipMalloc(&c->d_bw, sizeof(float) * bw.size());
    if (e == hipSuccess) e = hipMemcpy(c->d_bw, bw.data(), sizeof(float) * bw.size(), hipMemcpyHostToDevice);
    // learned-denoiser weights: FP32 master, Adam moments, FP16 layouts, biases (all zero)
    if (e == hipSuccess) e = hipMalloc(&c->cnn.master, sizeof(float) * 3 * CNN_PARAMS);
    if (e == hipSuccess) {
        c->cnn.m = c->cnn.master + CNN_PARAMS;
        c->cnn.v = c->cnn.master + 2 * CNN_PARAMS;
        e = hipMemset(c->cnn.master, 0, sizeof(float) * 3 * CNN_PARAMS);
    }
    for (int l = 0; l < CNN_LAYERS && e == hipSuccess; ++l) {
        const size_t nw = (size_t)CNN_COS[l] * 9 * CNN_CIS[l];
        e = hipMalloc(&c->cnn.wt[l], sizeof(__half) * nw);
        if (e == hipSuccess) e = hipMemset(c->cnn.wt[l], 0, sizeof(__half) * nw);
        if (e == hipSuccess && l > 0) e = hipMalloc(&c->cnn.wb[l], sizeof(__half) * nw);
        if (e == hipSuccess && l > 0) e = hipMemset(c->cnn.wb[l], 0, sizeof(__half) * nw);
        if (e == hipSuccess) e = hipMalloc(&c->cnn.bias[l], sizeof(float) * CNN_COS[l]);
        if (e == hipSuccess) e = hipMemset(c->cnn.bias[l], 0, sizeof(float) * CNN_COS[l]);
    }
    if (e != hipSuccess) {
        rt3d_destroy(c);
        return RT3D_E_DEVICE;
    }
    *out = c;
    return RT3D_OK;
}

rt3d_status rt3d_profile(rt3d_ctx* c, int32_t id)
{
    if (!c) return RT3D_E_INVALID;
    if (id >= RT3D_KERNEL_COUNT) return fail(c, RT3D_E_INVALID, "unknown kernel id");
    c->prof_id = id < 0 ? -1 : id;
    return RT3D_OK;
}

rt3d_status rt3d_profile_read(rt3d_ctx* c, double* total_ms, uint64_t* launches)
{
    if (!c) return RT3D_E_INVALID;
    double sum = 0.0;
    for (size_t i = 0; i < c->prof_n; ++i) {
        RT3D_HIP(c, hipEventSynchronize(c->prof_ev[2 * i + 1]));
        float ms = 0.f;
        RT3D_HIP(c, hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
        sum += ms;
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = c->prof_n;
    c->prof_n = 0;
    return RT3D_OK;
}

void rt3d_destroy(rt3d_ctx* c)
{
    if (!c) return;
    int prev = 0;
    bool switched = hipGetDevice(&prev) == hipSuccess && prev != c->device && hipSetDevice(c->device) == hipSuccess;
    for (IrfTables& t : c->irf) free_irf(t);
    if (c->d_bw) (void)hipFree(c->d_bw);
    for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
    if (c->cnn.master) (void)hipFree(c->cnn.master);
    for (int l = 0; l < CNN_LAYERS; ++l) {
        if (c->cnn.wt[l]) (void)hipFree(c->cnn.wt[l]);
        if (c->cnn.wb[l]) (void)hipFree(c->cnn.wb[l]);
        if (c->cnn.bias[l]) (void)hipFree(c->cnn.bias[l]);
    }
    if (switched) (void)hipSetDevice(prev);
    delete c;
}

const char* rt3d_last_error(const rt3d_ctx* c) { return c ? c->err.c_str() : "null context"; }

double rt3d_sigma2(const rt3d_ctx* c) { return c ? c->irf[0].sigma2 : 0.0; }

size_t rt3d_workspace_bytes(const rt3d_ctx* c, uint32_t frames, uint32_t rows, uint32_t cols, uint64_t max_entries)
{
    if (!c) return 0;
    const long long P = (long long)frames * rows * cols;
    return carve_ctx(c, nullptr, P, max_entries, rows, cols).bytes;
}

rt3d_status rt3d_set_workspace(rt3d_ctx* c, void* dev_ptr, size_t bytes, uint32_t frames, uint32_t rows,
                               uint32_t cols, uint64_t max_entries)
{
    if (!c) return RT3D_E_INVALID;
    c->ws = nullptr;
    c->state_layout.clear();
    c->ws_P = 0;
    c->ws_E = 0;
    if (!dev_ptr || bytes == 0) return fail(c, RT3D_E_INVALID, "workspace pointer NULL or size 0");
    if (((uintptr_t)dev_ptr) % ALIGN) return fail(c, RT3D_E_INVALID, "workspace not 256-byte aligned");
    if (max_entries >= (1ull << 32)) return fail(c, RT3D_E_INVALID, "max_entries must be < 2^32");
    const long long P = (long long)frames * rows * cols;
    if (P <= 0) return fail(c, RT3D_E_INVALID, "zero frames, rows or cols");
    if (carve_ctx(c, nullptr, P, max_entries, rows, cols).bytes > bytes)
        return fail(c, RT3D_E_NOMEM, "workspace smaller than rt3d_workspace_bytes for this shape");
    Workspace w = carve_ctx(c, (uint8_t*)dev_ptr, P, max_entries, rows, cols);
    hipError_t e = hipMemset(w.err, 0, sizeof(int32_t) * 4);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemset(workspace error word)");
    c->ws = (uint8_t*)dev_ptr;
    c->ws_bytes = bytes;
    c->ws_P = P;
    c->ws_E = max_entries;
    c->ws_rows = rows;
    c->ws_cols = cols;
    {
        Shape sh = shape_of(frames, rows, cols);
        c->ws_cnn_groups = uses_cnn(c) ? cnn_wgrad_groups(sh) : 0;
    }
    return RT3D_OK;
}

}  // extern "C"

extern "C" {

rt3d_status rt3d_reconstruct(rt3d_ctx* c, const rt3d_input* in, rt3d_output* out_arg, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!in || in->struct_size != sizeof(rt3d_input)) return fail(c, RT3D_E_INVALID, "input NULL or struct_size mismatch");
    if (!out_arg || (out_arg->struct_size != sizeof(rt3d_output) &&
                     out_arg->struct_size != offsetof(rt3d_output, world_z)))
        return fail(c, RT3D_E_INVALID, "output NULL or struct_size mismatch");
    // a caller's struct from before world_z: read only the fields it has
    rt3d_output out_v{};
    std::memcpy(&out_v, out_arg, out_arg->struct_size);
    rt3d_output* out = &out_v;
    if (!out->pt_off || !out->depth || !out->intensity || !out->background || out->capacity == 0)
        return fail(c, RT3D_E_INVALID, "output pointers NULL or capacity 0");
    // frames and their groups of equal size (one group when every frame is rows x cols)
    Shape sh;
    std::vector<Group> groups;
    if (in->frame_rows || in->frame_cols) {
        if (!in->frame_rows || !in->frame_cols || in->frames == 0)
            return fail(c, RT3D_E_INVALID, "frame_rows and frame_cols go together, with frames >= 1");
        long long P = 0;
        for (uint32_t f = 0; f < in->frames; ++f) {
            const uint32_t r = in->frame_rows[f], q = in->frame_cols[f];
            if (!shape_ok(1, r, q)) return fail(c, RT3D_E_INVALID, "a frame's rows x cols must be in 1 .. 2^31-1");
            if (!groups.empty() && groups.back().sh.rows == (int)r && groups.back().sh.cols == (int)q) {
                Shape& g = groups.back().sh;
                ++g.F;
                g.P += (long long)r * q;
            } else {
                Group g;
                g.base = P;
                g.sh = shape_of(1, r, q);
                groups.push_back(g);
            }
            P += (long long)r * q;
            if (P >= (1ll << 31)) return fail(c, RT3D_E_INVALID, "the frames' pixels must total below 2^31");
        }
        for (Group& g : groups) g.sh.S = P;
        sh = shape_of(1, 1, (uint32_t)P);
        if (c->p.sr > 1) return fail(c, RT3D_E_UNSUPPORTED, "super-resolution needs frames of one size");
    } else {
        if (!shape_ok(in->frames, in->rows, in->cols))
            return fail(c, RT3D_E_INVALID, "frames x rows x cols must be in 1 .. 2^31-1");
        sh = shape_of(in->frames, in->rows, in->cols);
        groups.push_back(Group{0, sh});
    }
    if (groups.size() == 1) sh = groups[0].sh;
    if (sh.P * c->p.sr * c->p.sr >= (1ll << 31))
        return fail(c, RT3D_E_INVALID, "the point grid's pixels must total below 2^31");
    const uint8_t* cls = in->irf_class;
    if (cls && (c->p.sr > 1 || c->p.denoiser == RT3D_DENOISE_CNN))
        return fail(c, RT3D_E_UNSUPPORTED, "per-pixel IRFs with super-resolution or the learned denoiser");
    const std::vector<long long> prev_layout = c->state_layout;   // need_ws forgets it
    Workspace w;
    rt3d_status s = need_ws(c, sh.P, w);
    if (s != RT3D_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    const uint32_t* off;
    const uint32_t* ent;
    if (in->kind == RT3D_IN_HIST_U16) {
        if (!in->hist) return fail(c, RT3D_E_INVALID, "hist is NULL");
        if (((uintptr_t)in->hist) % 16) return fail(c, RT3D_E_INVALID, "hist not 16-byte aligned");
        RT3D_LAUNCH(c, RT3D_KERNEL_COMPACT, st,
                    launch_compact(in->hist, sh.P, c->T, w.off, w.ent, c->ws_E, w.counts, w.partial, w.stage, w.err, st));
        off = w.off;
        ent = w.ent;
        c->last_compacted = true;
    } else if (in->kind == RT3D_IN_PHOTON_CSR) {
        if (!in->off || !in->ent) return fail(c, RT3D_E_INVALID, "off/ent is NULL");
        off = in->off;
        ent = in->ent;
        c->last_compacted = false;
    } else if (in->kind == RT3D_IN_PHOTON_EVENTS) {
        if (in->n_events >= (1ull << 31)) return fail(c, RT3D_E_INVALID, "n_events must be < 2^31");
        if (in->n_events > 0 && (!in->ev_pixel || !in->ev_bin || !in->ev_scratch))
            return fail(c, RT3D_E_INVALID, "ev_pixel/ev_bin/ev_scratch is NULL");
        RT3D_LAUNCH(c, RT3D_KERNEL_COMPACT, st,
                    launch_compact_events(in->ev_pixel, in->ev_bin, in->n_events, sh.P, c->T, w.evoff,
                                          in->ev_scratch, w.off, w.ent, c->ws_E, w.counts, w.partial, w.err, st));
        off = w.off;
        ent = w.ent;
        c->last_compacted = true;
    } else {
        return fail(c, RT3D_E_UNSUPPORTED, "unknown input kind");
    }
    c->last_P = sh.P;
    c->cur_lpp = lanes_for(c, sh.P, groups.size() == 1 ? &groups[0].sh : nullptr);
    RT3D_HIP(c, launch_check_gain(in->gain, sh.P, w.err, st));
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    // the layout of this batch: its groups' bases and shapes
    std::vector<long long> layout;
    for (const Group& g : groups) layout.insert(layout.end(), {g.base, g.sh.F, g.sh.rows, g.sh.cols});
    if (in->flags & RT3D_FLAG_WARM_START) {
        if (layout != prev_layout)
            return fail(c, RT3D_E_STATE, "warm start: no final state of a batch of these frames in the workspace");
    } else if (c->p.sr > 1) {
        s = init_sr(c, sh, off, ent, in->gain, w.A, w.B, w.wide, st);
        if (s != RT3D_OK) return s;
    } else {
        for (const Group& g : groups)
            for (int k = 0; k < n_classes(c, cls); ++k)
                RT3D_LAUNCH(c, RT3D_KERNEL_INIT, st,
                            launch_init(dev_model(c, k, cls ? cls + g.base : nullptr), dev_params(c, k), g.sh,
                                        off + g.base, ent, in->gain ? in->gain + g.base : nullptr,
                                        state_at(w.A, g.base), w.wide, st));
        for (const Group& g : groups)
            RT3D_LAUNCH(c, RT3D_KERNEL_NORMALS, st, launch_init_normals(p, g.sh, state_at(w.A, g.base), st));
    }
    c->state_layout.clear();
    if (cls) RT3D_HIP(c, launch_class_lists(cls, sh.P, n_classes(c, cls), w.cls_list, w.cls_meta, st));
    if (c->p.sr > 1) {
        for (int it = 0; it < c->p.n_iter; ++it) {
            s = iterate_sr(c, sh, off, ent, in->gain, w.A, w.B, w.btmp, st);
            if (s != RT3D_OK) return s;
        }
    } else if (!cls && loop_eligible(c, groups, sh) && use_fused(c, sh)) {
        RT3D_LAUNCH(c, RT3D_KERNEL_LOOP, st,
                    launch_loop(m, p, sh, off, ent, in->gain, w.A, w.B, w.btmp, c->d_bw, c->rb, c->p.n_iter, st));
    } else {
        DevState cur = w.A, alt = w.B;
        for (int it = 0; it < c->p.n_iter; ++it) {
            s = iterate(c, sh, groups, off, ent, in->gain, cur, alt, w.btmp, &w.cnn, cls, st, w.cls_list,
                        w.cls_meta);
            if (s != RT3D_OK) return s;
        }
        s = settle(c, sh, cur, w.A, st);
        if (s != RT3D_OK) return s;
    }
    RT3D_LAUNCH(c, RT3D_KERNEL_OUTPUT, st,
                launch_output(point_grid(sh, c->p.sr), w.A, out, w.counts, w.partial, w.err, sh.P, st));
    if (out->world_z)
        for (const Group& g : groups)
            RT3D_LAUNCH(c, RT3D_KERNEL_OUTPUT, st,
                        launch_world_z(c->p.sr > 1 ? point_grid(g.sh, c->p.sr) : g.sh, g.base, w.A, out, c->p.dz,
                                       c->p.persp, st));
    c->state_layout = layout;
    return RT3D_OK;
}

struct rt3d_graph {
    rt3d_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

rt3d_status rt3d_graph_create(rt3d_ctx* c, const rt3d_input* in, rt3d_output* out, rt3d_graph** graph)
{
    if (!c) return RT3D_E_INVALID;
    if (!graph) return fail(c, RT3D_E_INVALID, "graph is NULL");
    *graph = nullptr;
    if (c->prof_id >= 0) return fail(c, RT3D_E_STATE, "kernel timing is on; turn it off to record a graph");
    hipStream_t cap = nullptr;
    RT3D_HIP(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeGlobal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(c, e, "hipStreamBeginCapture");
    }
    const rt3d_status s = rt3d_reconstruct(c, in, out, cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (s != RT3D_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != RT3D_OK ? s : hip_fail(c, e, "hipStreamEndCapture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    rt3d_graph* r = new (std::nothrow) rt3d_graph();
    if (!r) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(c, RT3D_E_NOMEM, "graph allocation");
    }
    r->ctx = c;
    r->graph = g;
    r->exec = x;
    *graph = r;
    return RT3D_OK;
}

// The batch of an input: its pixels, and whether every frame has one size
// (then sh is that shape).  false for a malformed frame list.
static bool input_batch(const rt3d_input* in, Shape& sh, bool& one_size)
{
    uint32_t F = in->frames, R = in->rows, Q = in->cols;
    one_size = true;
    if (in->frame_rows || in->frame_cols) {
        if (!in->frame_rows || !in->frame_cols || F == 0) return false;
        R = in->frame_rows[0];
        Q = in->frame_cols[0];
        long long P = 0;
        for (uint32_t f = 0; f < F; ++f) {
            if (in->frame_rows[f] != R || in->frame_cols[f] != Q) one_size = false;
            P += (long long)in->frame_rows[f] * in->frame_cols[f];
        }
        if (!one_size) {
            sh = shape_of(1, 1, (uint32_t)std::min<long long>(P, 0x7fffffff));
            return true;
        }
    }
    if (!shape_ok(F, R, Q)) return false;
    sh = shape_of(F, R, Q);
    return true;
}

rt3d_status rt3d_autotune(rt3d_ctx* c, const rt3d_input* in, rt3d_output* out, void* hip_stream,
                          int32_t* fused)
{
    if (!c) return RT3D_E_INVALID;
    if (fused) *fused = 0;
    if (!in || in->struct_size != sizeof(rt3d_input)) return fail(c, RT3D_E_INVALID, "input NULL or struct_size mismatch");
    Shape sh;
    bool one_size = true;
    if (!input_batch(in, sh, one_size)) return fail(c, RT3D_E_INVALID, "bad frame sizes");
    if (!one_size) return RT3D_OK;                                   // several sizes: the defaults
    // the mappings: (fused, lanes per pixel)
    std::vector<std::array<int, 2>> ways = {{0, 4}, {0, 8}};
    if (c->p.denoiser == RT3D_DENOISE_APSS && !(c->p.persp > 0) && c->p.sr == 1 && !in->irf_class &&
        (long long)sh.rows * sh.cols <= LOOP_MAX_PIX)
        ways.push_back({1, 4});
    rt3d_input cold = *in;
    cold.flags &= ~RT3D_FLAG_WARM_START;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    std::vector<float> ms(ways.size(), 0.f);
    rt3d_status s = RT3D_OK;
    for (size_t w = 0; w < ways.size() && e == hipSuccess && s == RT3D_OK; ++w) {
        c->force_fused = ways[w][0];
        c->force_lanes = ways[w][1];
        s = rt3d_reconstruct(c, &cold, out, st);                   // untimed
        if (s == RT3D_OK) e = hipEventRecord(ev[0], st);
        for (int k = 0; k < 3 && s == RT3D_OK && e == hipSuccess; ++k) s = rt3d_reconstruct(c, &cold, out, st);
        if (s == RT3D_OK && e == hipSuccess) e = hipEventRecord(ev[1], st);
        if (s == RT3D_OK && e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (s == RT3D_OK && e == hipSuccess) e = hipEventElapsedTime(&ms[w], ev[0], ev[1]);
    }
    c->force_fused = -2;
    c->force_lanes = 0;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (s != RT3D_OK) return s;
    if (e != hipSuccess) return hip_fail(c, e, "autotune timing");
    size_t best = 0;
    for (size_t w = 1; w < ways.size(); ++w)
        if (ms[w] < ms[best]) best = w;
    bool found = false;
    for (auto& t : c->tuned)
        if (t[0] == sh.F && t[1] == sh.rows && t[2] == sh.cols) {
            t[3] = ways[best][0];
            t[4] = ways[best][1];
            found = true;
        }
    if (!found) c->tuned.push_back({(long long)sh.F, (long long)sh.rows, (long long)sh.cols, ways[best][0], ways[best][1]});
    if (fused) *fused = ways[best][0];
    return RT3D_OK;
}

rt3d_status rt3d_mapping(rt3d_ctx* c, const rt3d_input* in, int32_t* fused, int32_t* lanes)
{
    if (!c) return RT3D_E_INVALID;
    if (!in || in->struct_size != sizeof(rt3d_input)) return fail(c, RT3D_E_INVALID, "input NULL or struct_size mismatch");
    Shape sh;
    bool one_size = true;
    if (!input_batch(in, sh, one_size)) return fail(c, RT3D_E_INVALID, "bad frame sizes");
    std::vector<Group> groups(1, Group{0, sh});
    const bool f = one_size && !in->irf_class && c->p.sr == 1 && loop_eligible(c, groups, sh) && use_fused(c, sh);
    if (fused) *fused = f ? 1 : 0;
    if (lanes) *lanes = lanes_for(c, sh.P, one_size ? &sh : nullptr);
    return RT3D_OK;
}

rt3d_status rt3d_graph_launch(rt3d_graph* g, void* hip_stream)
{
    if (!g) return RT3D_E_INVALID;
    RT3D_HIP(g->ctx, hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
    return RT3D_OK;
}

void rt3d_graph_destroy(rt3d_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

rt3d_status rt3d_query(rt3d_ctx* c, void* hip_stream, rt3d_stats* st)
{
    if (!c) return RT3D_E_INVALID;
    if (st && st->struct_size != sizeof(rt3d_stats)) return fail(c, RT3D_E_INVALID, "stats struct_size mismatch");
    RT3D_HIP(c, hipStreamSynchronize((hipStream_t)hip_stream));
    int32_t derr = 0;
    uint32_t E = 0;
    if (c->ws) {
        Workspace w = carve_ctx(c, c->ws, c->ws_P, c->ws_E, c->ws_rows, c->ws_cols);
        RT3D_HIP(c, hipMemcpy(&derr, w.err, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (c->last_compacted && c->last_P > 0)
            RT3D_HIP(c, hipMemcpy(&E, w.off + c->last_P, sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (derr != 0) RT3D_HIP(c, hipMemset(w.err, 0, sizeof(int32_t)));
    }
    if (st) {
        st->device_error = derr;
        st->entries = E;
        st->points = 0;
    }
    if (derr != 0) return fail(c, derr, "device reported an error (capacity exceeded)");
    return RT3D_OK;
}

rt3d_status rt3d_debug_compact(rt3d_ctx* c, const uint16_t* hist, uint32_t npix, uint32_t* off, uint32_t* ent,
                               uint64_t capacity, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!hist || !off || !ent || npix == 0 || capacity == 0) return fail(c, RT3D_E_INVALID, "NULL pointer or zero size");
    if (((uintptr_t)hist) % 16) return fail(c, RT3D_E_INVALID, "hist not 16-byte aligned");
    Workspace w;
    rt3d_status s = need_ws(c, npix, w);
    if (s != RT3D_OK) return s;
    RT3D_HIP(c, launch_compact(hist, npix, c->T, off, ent, capacity, w.counts, w.partial, w.stage, w.err,
                               (hipStream_t)hip_stream));
    return RT3D_OK;
}

rt3d_status rt3d_compact_noalloc(rt3d_ctx* c, const uint16_t* hist, uint32_t npix, uint32_t* off, uint32_t* ent,
                                 uint64_t capacity, int32_t* dev_err, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!hist || !off || !ent || npix == 0 || capacity == 0) return fail(c, RT3D_E_INVALID, "NULL pointer or zero size");
    if (((uintptr_t)hist) % 16) return fail(c, RT3D_E_INVALID, "hist not 16-byte aligned");
    if ((long long)npix > noalloc_max_pixels())
        return fail(c, RT3D_E_INVALID, "npix above RT3D_NOALLOC_MAX_PIXELS (" + std::to_string(noalloc_max_pixels()) + ")");
    RT3D_HIP(c, launch_compact_noalloc(hist, npix, c->T, off, ent, capacity, dev_err, (hipStream_t)hip_stream));
    return RT3D_OK;
}

rt3d_status rt3d_debug_compact_events(rt3d_ctx* c, const uint32_t* ev_pixel, const uint16_t* ev_bin,
                                      uint64_t n_events, uint32_t npix, uint32_t* ev_scratch, uint32_t* off,
                                      uint32_t* ent, uint64_t capacity, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!off || !ent || npix == 0 || capacity == 0) return fail(c, RT3D_E_INVALID, "NULL pointer or zero size");
    if (n_events >= (1ull << 31)) return fail(c, RT3D_E_INVALID, "n_events must be < 2^31");
    if (n_events > 0 && (!ev_pixel || !ev_bin || !ev_scratch))
        return fail(c, RT3D_E_INVALID, "ev_pixel/ev_bin/ev_scratch is NULL");
    Workspace w;
    rt3d_status s = need_ws(c, npix, w);
    if (s != RT3D_OK) return s;
    RT3D_HIP(c, launch_compact_events(ev_pixel, ev_bin, n_events, npix, c->T, w.evoff, ev_scratch, off, ent,
                                      capacity, w.counts, w.partial, w.err, (hipStream_t)hip_stream));
    return RT3D_OK;
}

// rt3d_debug_step under super-resolution (arguments checked by the caller):
// states on the point grid, the lidar frames are theirs divided by sr.
static rt3d_status debug_step_sr(rt3d_ctx* c, int32_t step, const uint32_t* off, const uint32_t* ent,
                                 const float* gain, const rt3d_state* in, rt3d_state* out, hipStream_t st)
{
    const int sr = c->p.sr;
    if (out->rows % sr || out->cols % sr)
        return fail(c, RT3D_E_INVALID, "point-grid rows and cols must be multiples of sr");
    const Shape fsh = shape_of(out->frames, out->rows, out->cols);
    const Shape lid = shape_of(out->frames, out->rows / sr, out->cols / sr);
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    DevState O = dev_state(out);
    Workspace w{};
    const bool needs_ws = step == RT3D_STEP_INIT || step == RT3D_STEP_BFILTER || step == RT3D_STEP_ITERATION;
    if (needs_ws) {
        rt3d_status s = need_ws(c, lid.P, w);
        if (s != RT3D_OK) return s;
    }
    switch (step) {
    case RT3D_STEP_INIT:
        return init_sr(c, lid, off, ent, gain, O, w.B, w.wide, st);
    case RT3D_STEP_APSS:
        RT3D_HIP(c, launch_apss(m, p, fsh, dev_state(in), O, -1, st));
        return RT3D_OK;
    case RT3D_STEP_IFILTER:
        RT3D_HIP(c, launch_ifilter(p, fsh, dev_state(in), O, st));
        return RT3D_OK;
    default:
        break;
    }
    if (step < 0 || step > RT3D_STEP_ITERATION) return fail(c, RT3D_E_INVALID, "unknown step");
    RT3D_HIP(c, launch_copy_state(fsh, dev_state(in), O, st));
    switch (step) {
    case RT3D_STEP_DEPTH:
    case RT3D_STEP_INTENSITY:
    case RT3D_STEP_BKG:
        RT3D_HIP(c, launch_sr_step(step, m, p, lid, sr, fsh.P, off, ent, gain, O, nullptr, st));
        return RT3D_OK;
    case RT3D_STEP_MERGE:
        RT3D_HIP(c, launch_merge(m, p, fsh, O, st));
        return RT3D_OK;
    case RT3D_STEP_BFILTER:
        RT3D_HIP(c, launch_bfilter(c->d_bw, c->rb, lid, (float)c->p.b_min, O.b, w.btmp, w.B.b, st));
        RT3D_HIP(c, hipMemcpyAsync(O.b, w.btmp, sizeof(float) * lid.P, hipMemcpyDeviceToDevice, st));
        return RT3D_OK;
    case RT3D_STEP_ITERATION:
        return iterate_sr(c, lid, off, ent, gain, O, w.B, w.btmp, st);
    default:
        return fail(c, RT3D_E_INVALID, "unknown step");
    }
}

rt3d_status rt3d_debug_step(rt3d_ctx* c, int32_t step, const uint32_t* off, const uint32_t* ent, const float* gain,
                            const rt3d_state* in, rt3d_state* out, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!state_ok(out)) return fail(c, RT3D_E_INVALID, "output state incomplete");
    if (step != RT3D_STEP_INIT && !state_ok(in)) return fail(c, RT3D_E_INVALID, "input state incomplete");
    if (step != RT3D_STEP_INIT && (in->frames != out->frames || in->rows != out->rows || in->cols != out->cols))
        return fail(c, RT3D_E_INVALID, "state shapes differ");
    if (step != RT3D_STEP_INIT && (in->t == out->t || in->r == out->r || in->cnt == out->cnt))
        return fail(c, RT3D_E_INVALID, "in and out alias");
    const bool needs_csr = step == RT3D_STEP_INIT || step == RT3D_STEP_DEPTH || step == RT3D_STEP_INTENSITY ||
                           step == RT3D_STEP_BKG || step == RT3D_STEP_ITERATION;
    if (needs_csr && (!off || !ent)) return fail(c, RT3D_E_INVALID, "off/ent is NULL");
    if (!shape_ok(out->frames, out->rows, out->cols)) return fail(c, RT3D_E_INVALID, "bad state shape");
    c->cur_lpp = lanes_for(c, (long long)out->frames * out->rows * out->cols, nullptr);
    const Shape sh = shape_of(out->frames, out->rows, out->cols);
    hipStream_t st = (hipStream_t)hip_stream;
    const DevModel m = dev_model(c);
    const DevParams p = dev_params(c);
    DevState O = dev_state(out);
    const uint8_t* cls = c->debug_cls;
    const int nc = n_classes(c, cls);
    if (c->p.sr > 1) {
        if (cls) return fail(c, RT3D_E_UNSUPPORTED, "per-pixel IRFs with super-resolution");
        return debug_step_sr(c, step, off, ent, gain, in, out, st);
    }
    switch (step) {
    case RT3D_STEP_INIT: {
        // the pixel list of large pools lives in the bound workspace; without
        // one that covers the frames those pools take the HBM path
        uint32_t* wide = nullptr;
        if (c->ws && c->ws_P >= sh.P) wide = carve_ctx(c, c->ws, c->ws_P, c->ws_E, c->ws_rows, c->ws_cols).wide;
        for (int k = 0; k < nc; ++k)
            RT3D_HIP(c, launch_init(dev_model(c, k, cls), dev_params(c, k), sh, off, ent, gain, O, wide, st));
        RT3D_HIP(c, launch_init_normals(p, sh, O, st));
        return RT3D_OK;
    }
    case RT3D_STEP_APSS:
        RT3D_HIP(c, launch_apss(m, p, sh, dev_state(in), O, -1, st));
        return RT3D_OK;
    case RT3D_STEP_IFILTER:
        RT3D_HIP(c, launch_ifilter(p, sh, dev_state(in), O, st));
        return RT3D_OK;
    default:
        break;
    }
    if (step < 0 || step > RT3D_STEP_ITERATION) return fail(c, RT3D_E_INVALID, "unknown step");
    RT3D_HIP(c, launch_copy_state(sh, dev_state(in), O, st));
    switch (step) {
    case RT3D_STEP_DEPTH:
        for (int k = 0; k < nc; ++k)
            RT3D_HIP(c, launch_depth_step(dev_model(c, k, cls), dev_params(c, k), sh, off, ent, gain, O, st));
        return RT3D_OK;
    case RT3D_STEP_MERGE:
        for (int k = 0; k < nc; ++k) RT3D_HIP(c, launch_merge(dev_model(c, k, cls), dev_params(c, k), sh, O, st));
        return RT3D_OK;
    case RT3D_STEP_INTENSITY:
        for (int k = 0; k < nc; ++k)
            RT3D_HIP(c, launch_intensity_step(dev_model(c, k, cls), dev_params(c, k), sh, off, ent, gain, O, false,
                                              st));
        return RT3D_OK;
    case RT3D_STEP_BKG:
        for (int k = 0; k < nc; ++k)
            RT3D_HIP(c, launch_bg_step(dev_model(c, k, cls), dev_params(c, k), sh, off, ent, gain, O, nullptr, st));
        return RT3D_OK;
    case RT3D_STEP_BFILTER: {
        Workspace w;
        rt3d_status s = need_ws(c, sh.P, w);
        if (s != RT3D_OK) return s;
        // filtered into the workspace, then back into the state
        RT3D_HIP(c, launch_bfilter(c->d_bw, c->rb, sh, (float)c->p.b_min, O.b, w.btmp, w.B.b, st));
        RT3D_HIP(c, hipMemcpyAsync(O.b, w.btmp, sizeof(float) * sh.P, hipMemcpyDeviceToDevice, st));
        return RT3D_OK;
    }
    case RT3D_STEP_ITERATION: {
        Workspace w;
        rt3d_status s = need_ws(c, sh.P, w);
        if (s != RT3D_OK) return s;
        DevState cur = O, alt = w.B;
        s = iterate(c, sh, std::vector<Group>{Group{0, sh}}, off, ent, gain, cur, alt, w.btmp, &w.cnn, cls, st);
        if (s != RT3D_OK) return s;
        return settle(c, sh, cur, O, st);
    }
    default:
        return fail(c, RT3D_E_INVALID, "unknown step");
    }
}

rt3d_status rt3d_debug_gradients(rt3d_ctx* c, const uint32_t* off, const uint32_t* ent, const float* gain,
                                 const rt3d_state* s, float* gt, float* gr, float* gb, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (s) c->cur_lpp = lanes_for(c, (long long)s->frames * s->rows * s->cols, nullptr);
    if (!state_ok(s) || !off || !ent || !gt || !gr || !gb) return fail(c, RT3D_E_INVALID, "NULL argument");
    if (!shape_ok(s->frames, s->rows, s->cols)) return fail(c, RT3D_E_INVALID, "bad state shape");
    const Shape sh = shape_of(s->frames, s->rows, s->cols);
    const int sr = c->p.sr;
    if (sr > 1) {
        if (c->debug_cls) return fail(c, RT3D_E_UNSUPPORTED, "per-pixel IRFs with super-resolution");
        if (s->rows % sr || s->cols % sr)
            return fail(c, RT3D_E_INVALID, "point-grid rows and cols must be multiples of sr");
        const Shape lid = shape_of(s->frames, s->rows / sr, s->cols / sr);
        RT3D_HIP(c, launch_sr_gradients(dev_model(c), dev_params(c), lid, sr, sh.P, off, ent, gain, dev_state(s), gt,
                                        gr, gb, (hipStream_t)hip_stream));
        return RT3D_OK;
    }
    for (int k = 0; k < n_classes(c, c->debug_cls); ++k)
        RT3D_HIP(c, launch_gradients(dev_model(c, k, c->debug_cls), dev_params(c, k), sh, off, ent, gain,
                                     dev_state(s), gt, gr, gb, (hipStream_t)hip_stream));
    return RT3D_OK;
}

rt3d_status rt3d_debug_irf_class(rt3d_ctx* c, const uint8_t* irf_class)
{
    if (!c) return RT3D_E_INVALID;
    c->debug_cls = irf_class;
    return RT3D_OK;
}

rt3d_status rt3d_add_irf(rt3d_ctx* c, const double* irf, uint32_t irf_len, int32_t irf_origin, int32_t* id)
{
    if (!c) return RT3D_E_INVALID;
    if (c->irf.size() >= (size_t)RT3D_MAX_IRFS) return fail(c, RT3D_E_INVALID, "the context holds RT3D_MAX_IRFS IRFs");
    if (c->p.sr > 1 || c->p.denoiser == RT3D_DENOISE_CNN)
        return fail(c, RT3D_E_UNSUPPORTED, "per-pixel IRFs with super-resolution or the learned denoiser");
    const rt3d_status ok = check_irf(irf, irf_len, irf_origin, c->T, &c->p);
    if (ok != RT3D_OK) return fail(c, ok, "IRF rejected");
    int prev = 0;
    const bool switched =
        hipGetDevice(&prev) == hipSuccess && prev != c->device && hipSetDevice(c->device) == hipSuccess;
    IrfTables t;
    const rt3d_status s = build_irf(irf, irf_len, irf_origin, c->T, &c->p, t);
    if (switched) (void)hipSetDevice(prev);
    if (s != RT3D_OK) {
        free_irf(t);
        return fail(c, s, s == RT3D_E_DEVICE ? "HIP failure uploading the IRF tables" : "IRF rejected");
    }
    c->irf.push_back(std::move(t));
    if (id) *id = (int32_t)c->irf.size() - 1;
    return RT3D_OK;
}

}  // extern "C"

extern "C" {

rt3d_status rt3d_cnn_set_weights(rt3d_ctx* c, const float* host, size_t n)
{
    if (!c) return RT3D_E_INVALID;
    if (!host || n != (size_t)CNN_PARAMS) return fail(c, RT3D_E_INVALID, "weights NULL or n != RT3D_CNN_PARAMS");
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(host[k])) return fail(c, RT3D_E_INVALID, "non-finite weight");
    RT3D_HIP(c, hipMemcpy(c->cnn.master, host, sizeof(float) * n, hipMemcpyHostToDevice));
    RT3D_HIP(c, hipMemset(c->cnn.m, 0, sizeof(float) * 2 * CNN_PARAMS));
    c->cnn.step = 0;
    RT3D_HIP(c, launch_cnn_prepare(c->cnn, nullptr));
    RT3D_HIP(c, hipDeviceSynchronize());
    c->cnn_set = true;
    return RT3D_OK;
}

rt3d_status rt3d_cnn_get_weights(rt3d_ctx* c, float* host, size_t n)
{
    if (!c) return RT3D_E_INVALID;
    if (!host || n != (size_t)CNN_PARAMS) return fail(c, RT3D_E_INVALID, "weights NULL or n != RT3D_CNN_PARAMS");
    RT3D_HIP(c, hipDeviceSynchronize());
    RT3D_HIP(c, hipMemcpy(host, c->cnn.master, sizeof(float) * n, hipMemcpyDeviceToHost));
    return RT3D_OK;
}

// Checkpoint file of the network and its optimiser (layout in rt3d.h).
namespace {
constexpr char CKPT_MAGIC[8] = {'R', 'T', '3', 'D', 'C', 'N', 'N', '\0'};
constexpr uint32_t CKPT_VERSION = 1;

uint64_t fnv1a(const uint8_t* p, size_t n, uint64_t h = 1469598103934665603ull)
{
    for (size_t k = 0; k < n; ++k) {
        h ^= p[k];
        h *= 1099511628211ull;
    }
    return h;
}

// The header's bytes: magic, version, parameter count, layer count, each
// layer's channels (uint32), then the Adam step (int64), all little-endian.
constexpr size_t CKPT_HEAD = 8 + 4 * (3 + 2 * CNN_LAYERS) + 8;

void put_u32(std::vector<uint8_t>& b, uint32_t v)
{
    for (int k = 0; k < 4; ++k) b.push_back((uint8_t)(v >> (8 * k)));
}

std::vector<uint8_t> ckpt_header(long long step)
{
    std::vector<uint8_t> b(CKPT_MAGIC, CKPT_MAGIC + 8);
    put_u32(b, CKPT_VERSION);
    put_u32(b, CNN_PARAMS);
    put_u32(b, CNN_LAYERS);
    for (int l = 0; l < CNN_LAYERS; ++l) {
        put_u32(b, CNN_CIN[l]);
        put_u32(b, CNN_COUT[l]);
    }
    for (int k = 0; k < 8; ++k) b.push_back((uint8_t)((uint64_t)step >> (8 * k)));
    return b;
}
}  // namespace

rt3d_status rt3d_denoiser_save(rt3d_ctx* c, const char* path)
{
    if (!c) return RT3D_E_INVALID;
    if (!path) return fail(c, RT3D_E_INVALID, "path is NULL");
    if (!uses_cnn(c)) return fail(c, RT3D_E_STATE, "context was not created with RT3D_DENOISE_CNN");
    std::vector<float> buf((size_t)3 * CNN_PARAMS);
    RT3D_HIP(c, hipDeviceSynchronize());
    RT3D_HIP(c, hipMemcpy(buf.data(), c->cnn.master, sizeof(float) * buf.size(), hipMemcpyDeviceToHost));
    const std::vector<uint8_t> h = ckpt_header(c->cnn.step);
    uint64_t hash = fnv1a(h.data(), h.size());
    hash = fnv1a(reinterpret_cast<const uint8_t*>(buf.data()), sizeof(float) * buf.size(), hash);
    std::FILE* f = std::fopen(path, "wb");
    if (!f) return fail(c, RT3D_E_DEVICE, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(h.data(), 1, h.size(), f) == h.size() &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size() &&
              std::fwrite(&hash, sizeof hash, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(c, RT3D_E_DEVICE, std::string("write to ") + path + " failed");
    return RT3D_OK;
}

rt3d_status rt3d_denoiser_load(rt3d_ctx* c, const char* path)
{
    if (!c) return RT3D_E_INVALID;
    if (!path) return fail(c, RT3D_E_INVALID, "path is NULL");
    if (!uses_cnn(c)) return fail(c, RT3D_E_STATE, "context was not created with RT3D_DENOISE_CNN");
    std::FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, RT3D_E_DEVICE, std::string("cannot open ") + path);
    std::vector<uint8_t> h(CKPT_HEAD);
    std::vector<float> buf((size_t)3 * CNN_PARAMS);
    uint64_t stored = 0;
    char extra;
    const bool read_ok = std::fread(h.data(), 1, h.size(), f) == h.size() &&
                         std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size() &&
                         std::fread(&stored, sizeof stored, 1, f) == 1 && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!read_ok) return fail(c, RT3D_E_INVALID, std::string(path) + ": not a checkpoint of this size");
    long long step = 0;
    for (int k = 0; k < 8; ++k) step |= (long long)((uint64_t)h[CKPT_HEAD - 8 + k] << (8 * k));
    const std::vector<uint8_t> want = ckpt_header(step);
    if (want != h) return fail(c, RT3D_E_INVALID, std::string(path) + ": magic, version or network shape differ");
    uint64_t hash = fnv1a(h.data(), h.size());
    hash = fnv1a(reinterpret_cast<const uint8_t*>(buf.data()), sizeof(float) * buf.size(), hash);
    if (hash != stored) return fail(c, RT3D_E_INVALID, std::string(path) + ": hash mismatch");
    if (step < 0) return fail(c, RT3D_E_INVALID, std::string(path) + ": negative Adam step");
    for (float x : buf)
        if (!std::isfinite(x)) return fail(c, RT3D_E_INVALID, std::string(path) + ": non-finite value");
    RT3D_HIP(c, hipDeviceSynchronize());
    RT3D_HIP(c, hipMemcpy(c->cnn.master, buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice));
    c->cnn.step = step;
    RT3D_HIP(c, launch_cnn_prepare(c->cnn, nullptr));
    RT3D_HIP(c, hipDeviceSynchronize());
    c->cnn_set = true;
    return RT3D_OK;
}

static rt3d_status cnn_ready(rt3d_ctx* c, const rt3d_state* st, Workspace& w)
{
    if (!uses_cnn(c)) return fail(c, RT3D_E_STATE, "context was not created with RT3D_DENOISE_CNN");
    if (!state_ok(st) || !shape_ok(st->frames, st->rows, st->cols)) return fail(c, RT3D_E_INVALID, "bad state");
    const Shape sh = shape_of(st->frames, st->rows, st->cols);
    rt3d_status s = need_ws(c, sh.P, w);
    if (s != RT3D_OK) return s;
    if (cnn_wgrad_groups(sh) > c->ws_cnn_groups)
        return fail(c, RT3D_E_NOMEM, "frame shape needs more weight-gradient groups than the workspace holds");
    return RT3D_OK;
}

rt3d_status rt3d_cnn_last_gradient(rt3d_ctx* c, float* host, size_t n)
{
    if (!c) return RT3D_E_INVALID;
    if (!host || n != (size_t)CNN_PARAMS) return fail(c, RT3D_E_INVALID, "gradient NULL or n != RT3D_CNN_PARAMS");
    if (!uses_cnn(c) || !c->ws) return fail(c, RT3D_E_STATE, "no CNN workspace");
    Workspace w = carve_ctx(c, c->ws, c->ws_P, c->ws_E, c->ws_rows, c->ws_cols);
    RT3D_HIP(c, hipDeviceSynchronize());
    RT3D_HIP(c, hipMemcpy(host, w.cnn.grad, sizeof(float) * n, hipMemcpyDeviceToHost));
    return RT3D_OK;
}

rt3d_status rt3d_cnn_forward(rt3d_ctx* c, const rt3d_state* st, float* y, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!y) return fail(c, RT3D_E_INVALID, "y is NULL");
    Workspace w;
    rt3d_status s = cnn_ready(c, st, w);
    if (s != RT3D_OK) return s;
    const Shape sh = shape_of(st->frames, st->rows, st->cols);
    hipStream_t hs = (hipStream_t)hip_stream;
    RT3D_HIP(c, launch_cnn_infer(sh, dev_state(st), (float)std::sqrt(c->irf[0].sigma2), c->cnn, w.cnn, hs));
    RT3D_HIP(c, launch_cnn_unpack(sh, w.cnn, y, hs));
    return RT3D_OK;
}

rt3d_status rt3d_cnn_train_step(rt3d_ctx* c, const rt3d_state* st, const float* truth, uint32_t n_surf,
                                const rt3d_adam* opt, float* loss, void* hip_stream)
{
    if (!c) return RT3D_E_INVALID;
    if (!truth || !loss || n_surf == 0 || n_surf > 64) return fail(c, RT3D_E_INVALID, "truth/loss NULL or n_surf bad");
    if (!opt || opt->struct_size != sizeof(rt3d_adam) || !(opt->lr >= 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) ||
        !(opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps > 0))
        return fail(c, RT3D_E_INVALID, "bad Adam settings");
    Workspace w;
    rt3d_status s = cnn_ready(c, st, w);
    if (s != RT3D_OK) return s;
    const Shape sh = shape_of(st->frames, st->rows, st->cols);
    CnnAdam a{opt->lr, opt->beta1, opt->beta2, opt->eps};
    RT3D_HIP(c, launch_cnn_train_step(sh, dev_state(st), (float)std::sqrt(c->irf[0].sigma2), truth, (int)n_surf, c->cnn,
                                      w.cnn, a, loss, (hipStream_t)hip_stream));
    return RT3D_OK;
}

}  // extern "C"

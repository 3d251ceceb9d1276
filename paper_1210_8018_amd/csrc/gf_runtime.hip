// Host runtime behind the C ABI of include/gf.h: workspace layout, transform
// plans, graph-captured iteration chunks, device-side stopping flags,
// history and per-kernel timing. The library allocates no device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gf.h"
#include "gf_internal.h"

namespace gfk {
hipError_t launch_functional_g_impl(const Launch &L, int nblk, const double *omega, double scale, double *out);
hipError_t launch_functional_g_backward_impl(const Launch &L, int nblk, const double *omega, double scale,
                                             double *d_omega, double2 *d_U);
}

using namespace gfk;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultChunk = 8;
constexpr int kTileElems = 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool valid_length(int L)
{
    if (L < 2 || L > 256) return false;
    while (L % 2 == 0) L /= 2;
    while (L % 3 == 0) L /= 3;
    return L == 1;
}

bool valid_params(const gf_params *p)
{
    if (!p) return false;
    for (int mu = 0; mu < 4; ++mu)
        if (!valid_length(p->dims[mu])) return false;
    const double V = (double)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
    if (V > 2147483647.0 / 9.0) return false;  // 32-bit element offsets inside a plane
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return false;
    if (p->fft_prec != 0 && p->fft_prec != 1) return false;
    if (p->reunit_every < 0 || p->chunk < 0 || p->chunk > kHist) return false;
    return true;
}

int largest_divisor_at_most(int n, int cap)
{
    if (cap < 1) cap = 1;
    for (int d = cap < n ? cap : n; d >= 1; --d)
        if (n % d == 0) return d;
    return 1;
}

FftAxis plan_axis(const int dims[4], int mu)
{
    FftAxis a{};
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    a.L = dims[mu];
    a.S = 1;
    for (int nu = 0; nu < mu; ++nu) a.S *= dims[nu];
    const int cap = kTileElems / a.L;
    if (mu == 0)
        a.P = largest_divisor_at_most(V / a.L, cap);
    else
        a.P = largest_divisor_at_most(a.S, cap);
    a.ntile = V / (a.P * a.L);
    a.inner_chunks = (mu == 0) ? 1 : a.S / a.P;
    int L = a.L, n = 0;
    while (L % 3 == 0) {
        a.radix[n++] = 3;
        L /= 3;
    }
    while (L % 8 == 0) {
        a.radix[n++] = 8;
        L /= 8;
    }
    if (L == 4) a.radix[n++] = 4, L = 1;
    if (L == 2) a.radix[n++] = 2, L = 1;
    a.nstage = n;
    return a;
}

struct Layout {
    size_t fields, g, partials, sin2, tw, total;
};

Layout layout_for(const gf_params &p, size_t start)
{
    const size_t V = (size_t)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
    const size_t nblk = (V + kSiteBlock - 1) / kSiteBlock;
    const size_t csz = p.fft_prec ? 8 : 16;
    const size_t sumL = (size_t)p.dims[0] + p.dims[1] + p.dims[2] + p.dims[3];
    Layout l;
    size_t o = align_up(start);
    l.fields = o;
    o = align_up(o + kFields * V * csz);
    l.g = o;
    o = align_up(o + 9 * V * 16);
    l.partials = o;
    o = align_up(o + nblk * 4 * sizeof(double));
    l.sin2 = o;
    o = align_up(o + sumL * sizeof(double));
    l.tw = o;
    o = align_up(o + sumL * csz);
    l.total = o;
    return l;
}

// Header of the workspace: configuration table, batch map, scalar outputs.
size_t header_bytes(int ncfg) { return align_up(ncfg * sizeof(Cfg)) + align_up(sizeof(Batch)) + align_up(64); }

struct KTime {
    std::string name;
    double ms = 0.0;
    long long n = 0;
};

}  // namespace

struct gf_ctx_s {
    int ncfg = 0;
    bool batch = false;
    std::vector<gf_params> params;
    std::vector<Cfg> cfg;
    Batch bmap{};
    Launch L{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Cfg *d_cfgs = nullptr;
    Batch *d_batch = nullptr;
    double *d_scalar = nullptr;
    Ctrl *h_ctrl = nullptr;  // pinned mirror, ncfg entries
    std::vector<std::vector<double>> histF, histT;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int chunk = kDefaultChunk;
    std::string err;
    bool timing = false;
    std::vector<KTime> kt;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
};

namespace {

enum KId { K_DELTA, K_REDUCE, K_FFT0, K_FFT1, K_FFT2, K_FFT3S, K_IFFT2, K_IFFT1, K_IFFT0, K_GAUGE, K_UPDATE, K_N };
const char *kNames[K_N] = {"delta_reduce_partials", "reduce_stop", "fft_x_fwd",  "fft_y_fwd",
                           "fft_z_fwd",             "fft_t_scale", "fft_z_inv",  "fft_y_inv",
                           "fft_x_inv",             "gauge_reunit", "link_update"};

gf_status fail_hip(gf_ctx c, hipError_t e, const char *where)
{
    if (c) {
        c->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return GF_ERR_HIP;
}

#define HIPCHK(ctx, expr)                                     \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return fail_hip(ctx, e_, #expr); \
    } while (0)

hipEvent_t take_event(gf_ctx c)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Launch one kernel, bracketed by events when timing is on.
template <typename F>
hipError_t timed(gf_ctx c, int kid, hipStream_t s, F &&f)
{
    if (!c->timing || s != c->stream) return f();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    c->pending.push_back({kid, {a, b}});
    return e;
}

gf_status collect_timing(gf_ctx c)
{
    for (auto &p : c->pending) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.second.first, p.second.second));
        c->kt[p.first].ms += ms;
        c->kt[p.first].n += 1;
    }
    c->pending.clear();
    c->ev_used = 0;
    return GF_OK;
}

// Alg. 1 inner loop body: transform, scale, transform back, g, link update,
// re-measurement. Every kernel returns at once for configurations that are done.
hipError_t enqueue_iteration(gf_ctx c, hipStream_t s)
{
    Launch L = c->L;
    L.stream = s;
    hipError_t e;
    const int nf = kFields;
    if ((e = timed(c, K_FFT0, s, [&] { return launch_fft_axis(L, 0, -1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_FFT1, s, [&] { return launch_fft_axis(L, 1, -1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_FFT2, s, [&] { return launch_fft_axis(L, 2, -1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_FFT3S, s, [&] { return launch_fft_axis(L, 3, -1, 1, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_IFFT2, s, [&] { return launch_fft_axis(L, 2, +1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_IFFT1, s, [&] { return launch_fft_axis(L, 1, +1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_IFFT0, s, [&] { return launch_fft_axis(L, 0, +1, 0, nullptr, nf, 1); })) != hipSuccess) return e;
    if ((e = timed(c, K_GAUGE, s, [&] { return launch_gauge(L, 1, nullptr); })) != hipSuccess) return e;
    if ((e = timed(c, K_UPDATE, s, [&] { return launch_update(L, 1, nullptr); })) != hipSuccess) return e;
    if ((e = timed(c, K_DELTA, s, [&] { return launch_delta(L, 1, nullptr); })) != hipSuccess) return e;
    if ((e = timed(c, K_REDUCE, s, [&] { return launch_reduce(L, c->ncfg, 1, 1); })) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t enqueue_measure(gf_ctx c)
{
    hipError_t e;
    if ((e = launch_delta(c->L, 0, nullptr)) != hipSuccess) return e;
    return launch_reduce(c->L, c->ncfg, 0, 0);
}

gf_status build_graph(gf_ctx c)
{
    if (c->gexec) return GF_OK;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < c->chunk && e == hipSuccess; ++i) e = enqueue_iteration(c, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail_hip(c, e, "capture iteration");
    }
    HIPCHK(c, e2);
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
    return GF_OK;
}

gf_status read_ctrl(gf_ctx c)
{
    HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->cfg[0].ctrl, sizeof(Ctrl) * c->ncfg, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->ncfg; ++k) {
        const Ctrl &h = c->h_ctrl[k];
        auto &F = c->histF[k];
        auto &T = c->histT[k];
        long long have = (long long)F.size() - 1;  // last recorded iteration
        if (have < 0) {
            F.push_back(h.hist[0][0]);
            T.push_back(h.hist[0][1]);
            have = 0;
        }
        long long first = have + 1;
        if (h.iter - first + 1 > kHist) first = h.iter - kHist + 1;  // ring overrun (not expected)
        for (long long it = first; it <= h.iter; ++it) {
            F.push_back(h.hist[it % kHist][0]);
            T.push_back(h.hist[it % kHist][1]);
        }
    }
    return GF_OK;
}

// Run graph chunks until every configuration is done.
gf_status run_until_done(gf_ctx c)
{
    if (c->timing) {
        // one iteration at a time, every kernel bracketed by events; polling
        // after each iteration means no timed launch is a skipped one
        for (;;) {
            HIPCHK(c, enqueue_iteration(c, c->stream));
            gf_status st = read_ctrl(c);
            if (st != GF_OK) return st;
            st = collect_timing(c);
            if (st != GF_OK) return st;
            bool all = true;
            for (int k = 0; k < c->ncfg; ++k) all = all && c->h_ctrl[k].done != kRunning;
            if (all) return GF_OK;
        }
    }
    gf_status st = build_graph(c);
    if (st != GF_OK) return st;
    for (;;) {
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
        st = read_ctrl(c);
        if (st != GF_OK) return st;
        bool all = true;
        for (int k = 0; k < c->ncfg; ++k) all = all && c->h_ctrl[k].done != kRunning;
        if (all) return GF_OK;
    }
}

void fill_tables(const gf_params &p, std::vector<double> &sin2, std::vector<char> &tw, double &p2max)
{
    const int sumL = p.dims[0] + p.dims[1] + p.dims[2] + p.dims[3];
    sin2.assign(sumL, 0.0);
    const size_t csz = p.fft_prec ? 8 : 16;
    tw.assign(sumL * csz, 0);
    p2max = 0.0;
    int off = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = p.dims[mu];
        double best = 0.0;
        for (int n = 0; n < L; ++n) {
            const long double sn = sinl(3.14159265358979323846264338327950288L * n / L);
            const double v = (double)(4.0L * sn * sn);
            sin2[off + n] = v;
            if (v > best) best = v;
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * n / L;
            if (p.fft_prec) {
                float2 w = make_float2((float)cosl(a), (float)sinl(a));
                memcpy(&tw[(off + n) * csz], &w, csz);
            } else {
                double2 w = make_double2((double)cosl(a), (double)sinl(a));
                memcpy(&tw[(off + n) * csz], &w, csz);
            }
        }
        p2max += best;
        off += L;
    }
}

gf_status setup(gf_ctx c, int ncfg, const gf_params *params, void *const *links, void *d_ws, size_t ws_bytes,
                void *stream)
{
    c->ncfg = ncfg;
    c->params.assign(params, params + ncfg);
    c->stream = (hipStream_t)stream;
    c->ws = (char *)d_ws;
    c->ws_bytes = ws_bytes;
    c->chunk = params[0].chunk > 0 ? params[0].chunk : kDefaultChunk;
    HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipHostMalloc((void **)&c->h_ctrl, sizeof(Ctrl) * ncfg, hipHostMallocDefault));
    c->histF.assign(ncfg, {});
    c->histT.assign(ncfg, {});
    c->kt.resize(K_N);
    for (int k = 0; k < K_N; ++k) c->kt[k].name = kNames[k];

    size_t o = 0;
    c->d_cfgs = (Cfg *)(c->ws + o);
    o += align_up(ncfg * sizeof(Cfg));
    c->d_batch = (Batch *)(c->ws + o);
    o += align_up(sizeof(Batch));
    c->d_scalar = (double *)(c->ws + o);
    o += align_up(64);

    // Control blocks are laid out contiguously right after the header so a
    // single copy reads all of them back.
    const size_t ctrl_base = o;
    o += align_up(sizeof(Ctrl) * ncfg);

    c->cfg.assign(ncfg, Cfg{});
    Batch &b = c->bmap;
    memset(&b, 0, sizeof(b));
    b.n = ncfg;
    int max_lds = 0;
    std::vector<std::vector<double>> sin2s(ncfg);
    std::vector<std::vector<char>> tws(ncfg);
    for (int k = 0; k < ncfg; ++k) {
        const gf_params &p = params[k];
        Layout l = layout_for(p, o);
        Cfg &C = c->cfg[k];
        for (int mu = 0; mu < 4; ++mu) C.dims[mu] = p.dims[mu];
        C.V = p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
        C.nblk_site = (C.V + kSiteBlock - 1) / kSiteBlock;
        C.U = (double2 *)links[k];
        C.fields = c->ws + l.fields;
        C.g = (double2 *)(c->ws + l.g);
        C.partials = (double *)(c->ws + l.partials);
        C.ctrl = (Ctrl *)(c->ws + ctrl_base) + k;
        C.sin2 = (const double *)(c->ws + l.sin2);
        C.tw = c->ws + l.tw;
        int off = 0;
        for (int mu = 0; mu < 4; ++mu) {
            C.sin2_off[mu] = off;
            C.tw_off[mu] = off;
            off += p.dims[mu];
        }
        double p2max = 0.0;
        fill_tables(p, sin2s[k], tws[k], p2max);
        C.kfac = 0.5 * p.alpha * p2max / (double)C.V;
        C.reunit_every = p.reunit_every;
        for (int mu = 0; mu < 4; ++mu) {
            C.ax[mu] = plan_axis(p.dims, mu);
            const int e = C.ax[mu].P * C.ax[mu].L;
            if (e > max_lds) max_lds = e;
        }
        b.off_site[k + 1] = b.off_site[k] + C.nblk_site;
        for (int mu = 0; mu < 4; ++mu) b.off_fft[mu][k + 1] = b.off_fft[mu][k] + C.ax[mu].ntile;
        o = l.total;
    }
    if (o > ws_bytes) {
        c->err = "workspace too small";
        return GF_ERR_SHAPE;
    }
    b.max_lds_elems = max_lds;
    c->L.cfgs = c->d_cfgs;
    c->L.batch = c->d_batch;
    c->L.total_site_blocks = b.off_site[ncfg];
    for (int mu = 0; mu < 4; ++mu) c->L.total_fft_tiles[mu] = b.off_fft[mu][ncfg];
    c->L.max_lds_elems = max_lds;
    c->L.fp32 = params[0].fft_prec;
    c->L.stream = c->stream;

    HIPCHK(c, hipMemcpyAsync(c->d_cfgs, c->cfg.data(), sizeof(Cfg) * ncfg, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_batch, &c->bmap, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    for (int k = 0; k < ncfg; ++k) {
        HIPCHK(c, hipMemcpyAsync((void *)c->cfg[k].sin2, sin2s[k].data(), sin2s[k].size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync((void *)c->cfg[k].tw, tws[k].data(), tws[k].size(), hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, launch_arm(c->L, ncfg, 0.0, 0, 1));
    HIPCHK(c, enqueue_measure(c));
    return read_ctrl(c);
}

size_t workspace_total(int ncfg, const gf_params *params)
{
    size_t o = header_bytes(ncfg) + align_up(sizeof(Ctrl) * ncfg);
    for (int k = 0; k < ncfg; ++k) {
        if (!valid_params(&params[k])) return 0;
        o = layout_for(params[k], o).total;
    }
    return o;
}

gf_status status_from_done(gf_ctx c, bool want_eps)
{
    gf_status st = GF_OK;
    for (int k = 0; k < c->ncfg; ++k) {
        const int d = c->h_ctrl[k].done;
        if (d == kNonFinite) return GF_ERR_NONFINITE;
        if (want_eps && d == kMaxIter) st = GF_ERR_MAXITER;
    }
    return st;
}

}  // namespace

extern "C" {

size_t gf_workspace_bytes(const gf_params *params)
{
    if (!valid_params(params)) return 0;
    return workspace_total(1, params);
}

size_t gf_workspace_bytes_batch(int32_t n_cfg, const gf_params *params)
{
    if (n_cfg < 1 || n_cfg > kMaxCfg || !params) return 0;
    for (int k = 0; k < n_cfg; ++k)
        if (params[k].fft_prec != params[0].fft_prec || params[k].chunk != params[0].chunk) return 0;
    return workspace_total(n_cfg, params);
}

static gf_status init_common(gf_ctx *out, int32_t n_cfg, const gf_params *params, void *const *links, void *d_ws,
                             size_t ws_bytes, void *stream, bool batch)
{
    if (!out || !params || !links || !d_ws) return GF_ERR_ARG;
    *out = nullptr;
    for (int k = 0; k < n_cfg; ++k) {
        if (!valid_params(&params[k])) return GF_ERR_SHAPE;
        if (!links[k]) return GF_ERR_ARG;
    }
    const size_t need = batch ? gf_workspace_bytes_batch(n_cfg, params) : gf_workspace_bytes(params);
    if (need == 0 || ws_bytes < need) return GF_ERR_SHAPE;
    if (((uintptr_t)d_ws) % kAlign) return GF_ERR_ARG;
    gf_ctx c = new gf_ctx_s();
    c->batch = batch;
    gf_status st = setup(c, n_cfg, params, links, d_ws, ws_bytes, stream);
    if (st != GF_OK) {
        std::string e = c->err;
        gf_destroy(c);
        (void)e;
        return st;
    }
    *out = c;
    return GF_OK;
}

gf_status gf_init(gf_ctx *ctx, const gf_params *params, void *d_links, void *d_ws, size_t ws_bytes, void *stream)
{
    void *l[1] = {d_links};
    return init_common(ctx, 1, params, l, d_ws, ws_bytes, stream, false);
}

gf_status gf_init_batch(gf_ctx *ctx, int32_t n_cfg, const gf_params *params, void *const *d_links, void *d_ws,
                        size_t ws_bytes, void *stream)
{
    if (n_cfg < 1 || n_cfg > kMaxCfg) return GF_ERR_ARG;
    return init_common(ctx, n_cfg, params, d_links, d_ws, ws_bytes, stream, true);
}

gf_status gf_functional(gf_ctx c, double *F, double *theta)
{
    if (!c) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, enqueue_measure(c));
    HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->cfg[0].ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (F) *F = c->h_ctrl[0].F;
    if (theta) *theta = c->h_ctrl[0].theta;
    if (!std::isfinite(c->h_ctrl[0].F) || !std::isfinite(c->h_ctrl[0].theta)) return GF_ERR_NONFINITE;
    return GF_OK;
}

gf_status gf_functional_batch(gf_ctx c, double *F, double *theta)
{
    if (!c) return GF_ERR_ARG;
    HIPCHK(c, enqueue_measure(c));
    HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->cfg[0].ctrl, sizeof(Ctrl) * c->ncfg, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    gf_status st = GF_OK;
    for (int k = 0; k < c->ncfg; ++k) {
        if (F) F[k] = c->h_ctrl[k].F;
        if (theta) theta[k] = c->h_ctrl[k].theta;
        if (!std::isfinite(c->h_ctrl[k].F) || !std::isfinite(c->h_ctrl[k].theta)) st = GF_ERR_NONFINITE;
    }
    return st;
}

gf_status gf_step(gf_ctx c, int32_t n, double *F, double *theta)
{
    if (!c || n < 0) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    if (n > 0) {
        HIPCHK(c, launch_arm(c->L, c->ncfg, -1.0, n, 0));
        gf_status st = run_until_done(c);
        if (st != GF_OK) return st;
    }
    if (F) *F = c->h_ctrl[0].F;
    if (theta) *theta = c->h_ctrl[0].theta;
    return status_from_done(c, false);
}

gf_status gf_fix_until(gf_ctx c, double theta_eps, int64_t max_iter, int64_t *iters, double *F, double *theta)
{
    if (!c || max_iter < 0) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    const long long before = c->h_ctrl[0].iter;
    HIPCHK(c, launch_arm(c->L, c->ncfg, theta_eps, max_iter, 0));
    gf_status st = run_until_done(c);
    if (st != GF_OK) return st;
    if (iters) *iters = c->h_ctrl[0].iter - before;
    if (F) *F = c->h_ctrl[0].F;
    if (theta) *theta = c->h_ctrl[0].theta;
    return status_from_done(c, true);
}

gf_status gf_fix_until_batch(gf_ctx c, double theta_eps, int64_t max_iter, int64_t *iters, double *F, double *theta)
{
    if (!c || max_iter < 0) return GF_ERR_ARG;
    std::vector<long long> before(c->ncfg);
    for (int k = 0; k < c->ncfg; ++k) before[k] = c->h_ctrl[k].iter;
    HIPCHK(c, launch_arm(c->L, c->ncfg, theta_eps, max_iter, 0));
    gf_status st = run_until_done(c);
    if (st != GF_OK) return st;
    for (int k = 0; k < c->ncfg; ++k) {
        if (iters) iters[k] = c->h_ctrl[k].iter - before[k];
        if (F) F[k] = c->h_ctrl[k].F;
        if (theta) theta[k] = c->h_ctrl[k].theta;
    }
    return status_from_done(c, true);
}

gf_status gf_history(gf_ctx c, int64_t cap, double *F_hist, double *theta_hist, int64_t *n)
{
    if (!c || cap < 0) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    const auto &F = c->histF[0];
    const auto &T = c->histT[0];
    const int64_t avail = (int64_t)F.size();
    if (n) *n = avail;
    const int64_t m = cap < avail ? cap : avail;
    for (int64_t k = 0; k < m; ++k) {
        if (F_hist) F_hist[k] = F[k];
        if (theta_hist) theta_hist[k] = T[k];
    }
    return GF_OK;
}

gf_status gf_delta(gf_ctx c, void *d_delta)
{
    if (!c || !d_delta) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, launch_delta(c->L, 0, (double2 *)d_delta));
    HIPCHK(c, launch_reduce(c->L, 1, 0, 0));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_gauge(gf_ctx c, void *d_g)
{
    if (!c || !d_g) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    Launch L = c->L;
    HIPCHK(c, launch_delta(L, 0, nullptr));
    HIPCHK(c, launch_fft_axis(L, 0, -1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 1, -1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 2, -1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 3, -1, 1, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 2, +1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 1, +1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_fft_axis(L, 0, +1, 0, nullptr, kFields, 0));
    HIPCHK(c, launch_gauge(L, 0, (double2 *)d_g));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_apply_gauge(gf_ctx c, const void *d_g)
{
    if (!c || !d_g) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, launch_update(c->L, 0, (const double2 *)d_g));
    HIPCHK(c, enqueue_measure(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_fft(gf_ctx c, void *d_fields, int32_t nfields, int32_t sign)
{
    if (!c || !d_fields || nfields < 1 || nfields > 65535 || (sign != 1 && sign != -1)) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    for (int mu = 0; mu < 4; ++mu) HIPCHK(c, launch_fft_axis(c->L, mu, sign, 0, d_fields, nfields, 0));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_functional_g(gf_ctx c, const double *d_omega, double *F)
{
    if (!c || !d_omega) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    const Cfg &C = c->cfg[0];
    HIPCHK(c, launch_functional_g_impl(c->L, C.nblk_site, d_omega, 1.0 / (12.0 * (double)C.V), c->d_scalar));
    double h = 0.0;
    HIPCHK(c, hipMemcpyAsync(&h, c->d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (F) *F = h;
    return std::isfinite(h) ? GF_OK : GF_ERR_NONFINITE;
}

gf_status gf_functional_g_backward(gf_ctx c, const double *d_omega, double grad_out, double *d_dF_domega,
                                   void *d_dF_dU)
{
    if (!c || !d_omega) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    const Cfg &C = c->cfg[0];
    if (!d_dF_domega && !d_dF_dU) return GF_OK;
    HIPCHK(c, launch_functional_g_backward_impl(c->L, C.nblk_site, d_omega, grad_out / (12.0 * (double)C.V),
                                                d_dF_domega, (double2 *)d_dF_dU));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_destroy(gf_ctx c)
{
    if (!c) return GF_ERR_ARG;
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    for (auto e : c->ev_pool) hipEventDestroy(e);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    if (c->h_ctrl) hipHostFree(c->h_ctrl);
    delete c;
    return GF_OK;
}

const char *gf_strerror(gf_status s)
{
    switch (s) {
    case GF_OK: return "ok";
    case GF_ERR_ARG: return "invalid argument";
    case GF_ERR_SHAPE: return "unsupported lattice shape or workspace too small";
    case GF_ERR_HIP: return "HIP runtime error";
    case GF_ERR_NONFINITE: return "theta or F is not finite";
    case GF_ERR_MAXITER: return "iteration cap reached before theta <= eps";
    case GF_ERR_STATE: return "call does not apply to this context";
    }
    return "unknown status";
}

const char *gf_last_error(gf_ctx c) { return c ? c->err.c_str() : ""; }

gf_status gf_set_timing(gf_ctx c, int32_t on)
{
    if (!c) return GF_ERR_ARG;
    c->timing = on != 0;
    return GF_OK;
}

int32_t gf_kernel_count(gf_ctx c) { return c ? (int32_t)c->kt.size() : 0; }

const char *gf_kernel_name(gf_ctx c, int32_t k)
{
    if (!c || k < 0 || k >= (int32_t)c->kt.size()) return "";
    return c->kt[k].name.c_str();
}

gf_status gf_kernel_time(gf_ctx c, int32_t k, double *total_ms, int64_t *launches)
{
    if (!c || k < 0 || k >= (int32_t)c->kt.size()) return GF_ERR_ARG;
    if (total_ms) *total_ms = c->kt[k].ms;
    if (launches) *launches = c->kt[k].n;
    return GF_OK;
}

gf_status gf_reset_timing(gf_ctx c)
{
    if (!c) return GF_ERR_ARG;
    for (auto &k : c->kt) {
        k.ms = 0.0;
        k.n = 0;
    }
    return GF_OK;
}

}  // extern "C"

// Host runtime behind the C ABI of include/gf.h: workspace layout, transform
// plans, graph-captured iteration chunks, device-side stopping flags,
// history and per-kernel timing. The library allocates no device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
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

bool xy_feasible(const int dims[4]) { return dims[0] * dims[1] <= kTileElems2D; }
bool zt_feasible(const int dims[4]) { return dims[2] * dims[3] <= kTileElems2D; }

bool valid_params(const gf_params *p)
{
    if (!p) return false;
    for (int mu = 0; mu < 4; ++mu)
        if (!valid_length(p->dims[mu])) return false;
    const double V = (double)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
    if (V > 2147483647.0 / 9.0) return false;  // 32-bit element offsets inside a plane
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return false;
    if (p->fft_prec != 0 && p->fft_prec != 1) return false;
    if (p->link_prec != 0 && p->link_prec != 1) return false;
    if (p->reserved != 0 || !(p->refine_theta >= 0.0)) return false;
    if (p->reunit_every < 0 || p->chunk < 0 || p->chunk > kHist) return false;
    if (p->fft_schedule < 0 || p->fft_schedule >= kSchedCount) return false;
    if (p->fft_schedule == kSchedXY1D && !xy_feasible(p->dims)) return false;
    if (p->fft_schedule == kSchedXYZT && !(xy_feasible(p->dims) && zt_feasible(p->dims))) return false;
    return true;
}

// Marching blocks a CU holds at once (the fused pass: 256 work-items, about
// 226 VGPRs and 61.5 KB of LDS each).
constexpr int kMarchResidentPerCU = 2;

int largest_divisor_at_most(int n, int cap)
{
    if (cap < 1) cap = 1;
    for (int d = cap < n ? cap : n; d >= 1; --d)
        if (n % d == 0) return d;
    return 1;
}

// Sites of one block of the t-marching kernels: kSiteBlock consecutive
// (x, y, z) sites (tile[0] = 0), or a tx x ty x tz box (GF_TILE="tx,ty,tz",
// tx * ty * tz between 64 and kSiteBlock). Returns the number of blocks over
// the (x, y, z) volume.
int plan_tile(const int dims[4], int tile[3], int ntile[3])
{
    tile[0] = tile[1] = tile[2] = 0;
    ntile[0] = ntile[1] = ntile[2] = 0;
    const char *env = getenv("GF_TILE");
    int t[3];
    if (env && sscanf(env, "%d,%d,%d", &t[0], &t[1], &t[2]) == 3) {
        bool ok = t[0] * t[1] * t[2] <= kSiteBlock && t[0] * t[1] * t[2] >= 64;
        for (int a = 0; a < 3; ++a) ok = ok && t[a] >= 1 && t[a] <= dims[a];
        if (ok) {
            int n = 1;
            for (int a = 0; a < 3; ++a) {
                tile[a] = t[a];
                ntile[a] = (dims[a] + t[a] - 1) / t[a];
                n *= ntile[a];
            }
            return n;
        }
    }
    return (dims[0] * dims[1] * dims[2] + kSiteBlock - 1) / kSiteBlock;
}

// Blocks of the t-marching kernels: nb3 site sets times `tch` t-slices, a
// walk of at most 8 slices. Each walk re-reads its first slice's
// t-neighbours (about 0.23 of a slice's traffic); the blocks run in rounds
// of `resident` (two per CU). The walk length taken minimises
//   rounds * (tch + 0.23) * (1.05 if a single round, FP64 link storage),
// largest tch on ties: a single round leaves the CUs idle while its slowest
// blocks finish, and with FP64 links that costs more than the walk-end
// re-reads a second round adds. Measured picks (FP64 fused pass): 32^4 4
// slices (1024 blocks; 8 slices, one round, 2 % slower; binary32 storage
// the other way round, 8 slices 3 % faster); 24^4 3 slices (432 blocks, one
// round: 72 us against 77 for 1 slice and 82 for 4); 16^3 x 32 1 slice (512
// blocks; 2 slices 4 % slower); 48^4 6 slices (3456 blocks; 8 and 4 slices
// 7 % and 5 % slower); 64^4 8 slices (8192 blocks; one walk over all 64
// slices 2.7 % slower).
constexpr int kMaxTchunk = 8;
int plan_tchunk(const int dims[4], int nb3, bool f64_links, int resident)
{
    const char *env = getenv("GF_TCHUNK");
    if (env) {
        const int t = atoi(env);
        if (t >= 1 && dims[3] % t == 0) return t;
    }
    int best = 1;
    double best_cost = 1e300;
    for (int t = 1; t <= kMaxTchunk && t <= dims[3]; ++t) {
        if (dims[3] % t) continue;
        const long long nb = (long long)nb3 * (dims[3] / t);
        const long long rounds = (nb + resident - 1) / resident;
        double cost = (double)rounds * (t + 0.23);
        if (rounds == 1 && f64_links) cost *= 1.05;
        if (cost <= best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}

// In a batch every configuration's marching blocks take about the same
// number of t-slices (the largest divisor of Lt up to GF_TCHUNK_BATCH,
// default 4), so blocks carry equal work whatever lattice they belong to and
// the XCDs, each of which walks a contiguous range of blocks, stay balanced.
int plan_tchunk_batch(const int dims[4])
{
    const char *env = getenv("GF_TCHUNK_BATCH");
    const int T = env && atoi(env) >= 1 ? atoi(env) : 4;
    return largest_divisor_at_most(dims[3], T);
}

// xy tiles: Q consecutive xy-planes, Q * Lx * Ly <= target elements.
int plan_xyQ(const int dims[4], int target)
{
    const int V2 = dims[0] * dims[1];
    return largest_divisor_at_most(dims[2] * dims[3], (target < kTileElems2D ? target : kTileElems2D) / V2);
}

// zt tiles: P consecutive xy-sites times the (z, t) plane, P * Lz * Lt <=
// target elements; P is a power of two dividing Lx * Ly and at most 128 (so
// it divides every work-group size of the pass).
int plan_ztP(const int dims[4], int target)
{
    const int V2 = dims[0] * dims[1];
    const int cap = (target < kTileElems2D ? target : kTileElems2D) / (dims[2] * dims[3]);
    int P = 1;
    while (V2 % (2 * P) == 0 && 2 * P <= cap && 2 * P <= 128) P *= 2;
    return P;
}

FftAxis plan_axis(const int dims[4], int mu)
{
    FftAxis a{};
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    a.L = dims[mu];
    a.S = 1;
    for (int nu = 0; nu < mu; ++nu) a.S *= dims[nu];
    const int cap = kTileElems / a.L;
    if (mu == 0) {
        a.P = largest_divisor_at_most(V / a.L, cap);
    } else {
        // rows of P consecutive elements, P a power of two dividing S and the block
        a.P = 1;
        while (a.S % (2 * a.P) == 0 && 2 * a.P <= cap && 2 * a.P <= kFftThreads) a.P *= 2;
    }
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
    size_t fields, fields2, g, partials, sin2, tw, links12a, links12b, kmom, links12fa, links12fb, g12f, total;
};

Layout layout_for(const gf_params &p, size_t start)
{
    const size_t V = (size_t)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
    const size_t nblk_site = (V + kSiteBlock - 1) / kSiteBlock;
    int tile[3], ntile[3];
    const size_t nblk_march = (size_t)plan_tile(p.dims, tile, ntile) * (size_t)p.dims[3];  // upper bound (tch = 1)
    const size_t nblk = nblk_site > nblk_march ? nblk_site : nblk_march;
    const size_t csz = p.fft_prec ? 8 : 16;
    const size_t sumL = (size_t)p.dims[0] + p.dims[1] + p.dims[2] + p.dims[3];
    Layout l;
    size_t o = align_up(start);
    l.fields = o;
    o = align_up(o + kFields * V * csz);
    l.fields2 = o;
    o = align_up(o + kFields * V * csz);
    l.g = o;
    o = align_up(o + 9 * V * 16);
    l.partials = o;
    o = align_up(o + nblk * 4 * sizeof(double));
    l.sin2 = o;
    o = align_up(o + sumL * sizeof(double));
    l.tw = o;
    o = align_up(o + sumL * csz);
    // two-row (12-real) links, two buffers
    l.links12a = o;
    o = align_up(o + 24 * V * 16);
    l.links12b = o;
    o = align_up(o + 24 * V * 16);
    // K(p) table in the transform's precision
    l.kmom = o;
    o = align_up(o + V * (csz / 2));
    // single-precision storage of the two link buffers and of g (link_prec 1)
    l.links12fa = l.links12fb = l.g12f = 0;
    if (p.link_prec == 1) {
        l.links12fa = o;
        o = align_up(o + 24 * V * 8);
        l.links12fb = o;
        o = align_up(o + 24 * V * 8);
        l.g12f = o;
        o = align_up(o + 6 * V * 8);
    }
    l.total = o;
    return l;
}

// Header of the workspace: configuration table, batch map, scalar outputs.
size_t header_bytes(int ncfg)
{
    return align_up(ncfg * sizeof(Cfg)) + 2 * align_up(sizeof(Batch)) + align_up(64);
}

struct KTime {
    std::string name;
    double ms = 0.0;
    long long n = 0;
};

}  // namespace

// Tile choices of the 2D passes: target elements per tile and elements per
// work-item (the work-group size is the tile capacity divided by it).
// zt_reg: the scaled (z, t) pass of configurations with Lz = Lt = 32 runs
// in k_fft_zt_reg (radix stages in registers; 16 x 16, 24 x 24 and 16 x 32
// planes in k_fft_zt_lines)
// instead of the LDS-staged pass,
// with zt_reg work-groups per tile (1, 2 or 4, the four fields split among
// them); 0: the LDS-staged pass.
// xy_reg: the same for the iteration's (x, y) passes of configurations with
// Lx = Ly of 16, 24, 32, 48 or 64 (k_fft_xy_reg, k_fft_xy_inv_reg).
struct Tiles {
    int xy_target = 1024, xy_ept = 4;
    int zt_target = 4096, zt_ept = 8;
    int zt_reg = 2;
    int zt_reg_p = 4;  // xy-sites per tile of the register (z, t) pass (2, 4 or 8)
    int xy_reg = 1;
    int line_reg = 1;  // 1D z and t passes of 16- to 64-point lines in k_fft_line
    bool operator==(const Tiles &o) const
    {
        return xy_target == o.xy_target && xy_ept == o.xy_ept && zt_target == o.zt_target && zt_ept == o.zt_ept &&
               zt_reg == o.zt_reg && zt_reg_p == o.zt_reg_p && xy_reg == o.xy_reg && line_reg == o.line_reg;
    }
};

// Whether a configuration's scaled (z, t) pass can run in k_fft_zt_reg, and
// its (x, y) passes in k_fft_xy_reg / k_fft_xy_inv_reg (tiles of
// xy_reg_planes_for(Lx) planes).
// (32 x 32 planes in k_fft_zt_reg; 16 x 16, 24 x 24, 16 x 32 and 48 x 48 in
// k_fft_zt_lines, whose tiles hold whole waves of lines: 2 P Lt a multiple
// of 64, so 24 x 24 takes 4 or 8 xy-sites per tile; 48 x 48 takes 2, whose
// tile fills 75 KiB of LDS in FP64)
bool zt_reg_fits(const Cfg &C, int P)
{
    const int Lz = C.dims[2], Lt = C.dims[3];
    if (zt_shape_bit(Lz, Lt) < 0 || C.V2 % P) return false;
    if (Lz == 48) return P == 2;
    return Lz == 32 || (P * Lt * line_lanes(Lz)) % 64 == 0;
}
bool xy_reg_fits(const Cfg &C)
{
    const int L = C.dims[0];
    return L == C.dims[1] && line_len_ok(L) && (C.dims[2] * C.dims[3]) % xy_reg_planes_for(L) == 0;
}
// and its 1D pass along axis 2 + a in k_fft_line (a line of 16 to 64
// points; 64 / line_lanes xy-sites per row of a wave, 4 lines of the other
// axis per unit)
bool line_fits(const Cfg &C, int a)
{
    const int L = C.dims[2 + a], other = C.dims[3 - a];
    return line_len_ok(L) && C.V2 % (64 / line_lanes(L)) == 0 && other % 4 == 0;
}

struct gf_ctx_s {
    int ncfg = 0;
    bool batch = false;
    std::vector<gf_params> params;
    int link_prec = 0;          // 1: iterate in single-precision link storage (first phase)
    double refine_theta = 1e-10;  // theta at which gf_fix_until leaves it
    std::vector<Cfg> cfg;
    Batch bmap{};
    Launch L{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Cfg *d_cfgs = nullptr;
    Batch *d_batch = nullptr;      // map over every configuration
    Batch *d_batch_act = nullptr;  // map over the configurations still iterating
    Batch bact{};
    Launch Lact{};                 // launch shapes of the active map
    std::vector<int> active;
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
    int sched = kSched1D;
    Tiles tiles;
    // a context that allocates nothing (no stream, event, graph or pinned
    // host memory); iterations are launched directly on `stream`
    bool noalloc = false;
    // gf_init_functional: only the differentiable functional's buffers (g,
    // block partials); no transform plan, no measurement
    bool functional_only = false;
};

namespace {

enum KId {
    K_DELTA, K_REDUCE, K_FFT0, K_FFT1, K_FFT2, K_FFT3S, K_IFFT2, K_IFFT1, K_IFFT0, K_GAUGE, K_UPDATE,
    K_FFTXY, K_FFTZT_S, K_IFFTXY_GAUGE, K_UPDATE_DELTA, K_N
};
const char *kNames[K_N] = {"delta_reduce_partials", "reduce_stop",  "fft_x_fwd",        "fft_y_fwd",
                           "fft_z_fwd",             "fft_t_scale",  "fft_z_inv",        "fft_y_inv",
                           "fft_x_inv",             "gauge_reunit", "link_update",      "fft_xy_fwd",
                           "fft_zt_scale",          "fft_xy_inv_gauge", "link_update_delta"};

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

// Transform of the four fields, scaling, inverse transform and g, as the
// schedule in use arranges them (respect_done: skip finished configurations;
// g_override: write g there instead of the workspace).
// fold_reduce: the first pass (the xy pass) also does the final reduction of
// the previous update (schedules that start with it; see fold_ok).
hipError_t enqueue_gauge_steps(gf_ctx c, hipStream_t s, int respect_done, double2 *g_override, int fold_reduce = 0)
{
    Launch L = respect_done ? c->Lact : c->L;
    L.stream = s;
    hipError_t e;
    const int nf = kFields, rd = respect_done;
#define GF_TRY(kid, call)                                                            \
    if ((e = timed(c, kid, s, [&] { return call; })) != hipSuccess) return e;
    switch (c->sched) {
    case kSchedXYZT:
        GF_TRY(K_FFTXY, launch_fft_xy(L, -1, nullptr, nf, rd, fold_reduce));
        GF_TRY(K_FFTZT_S, launch_fft_zt_scale(L, rd));
        GF_TRY(K_IFFTXY_GAUGE, launch_fft_xy_inv_gauge(L, rd, g_override));
        break;
    case kSchedXY1D:
        GF_TRY(K_FFTXY, launch_fft_xy(L, -1, nullptr, nf, rd, fold_reduce));
        GF_TRY(K_FFT2, launch_fft_axis(L, 2, -1, 0, nullptr, nf, rd));
        GF_TRY(K_FFT3S, launch_fft_axis(L, 3, -1, 1, nullptr, nf, rd));
        GF_TRY(K_IFFT2, launch_fft_axis(L, 2, +1, 0, nullptr, nf, rd));
        GF_TRY(K_IFFTXY_GAUGE, launch_fft_xy_inv_gauge(L, rd, g_override));
        break;
    default:
        if (fold_reduce) return hipErrorInvalidValue;  // no xy pass to carry it
        GF_TRY(K_FFT0, launch_fft_axis(L, 0, -1, 0, nullptr, nf, rd));
        GF_TRY(K_FFT1, launch_fft_axis(L, 1, -1, 0, nullptr, nf, rd));
        GF_TRY(K_FFT2, launch_fft_axis(L, 2, -1, 0, nullptr, nf, rd));
        GF_TRY(K_FFT3S, launch_fft_axis(L, 3, -1, 1, nullptr, nf, rd));
        GF_TRY(K_IFFT2, launch_fft_axis(L, 2, +1, 0, nullptr, nf, rd));
        GF_TRY(K_IFFT1, launch_fft_axis(L, 1, +1, 0, nullptr, nf, rd));
        GF_TRY(K_IFFT0, launch_fft_axis(L, 0, +1, 0, nullptr, nf, rd));
        GF_TRY(K_GAUGE, launch_gauge(L, rd, g_override));
        break;
    }
    return hipSuccess;
}

// Whether the final reduction of an update can ride on the next iteration's
// first pass (an xy pass with work-groups of at least 256 work-items).
bool fold_ok(gf_ctx c)
{
    return (c->sched == kSchedXYZT || c->sched == kSchedXY1D) && can_fold_reduce(c->Lact);
}

// Alg. 1 inner loop body: transform, scale, transform back, g, link update,
// re-measurement. Every kernel returns at once for configurations that are
// done. fold_prev: the previous iteration's final reduction is done by this
// iteration's first pass; reduce_after: this iteration's own is launched
// (else the next iteration folds it).
// link_io: where the fused pass takes the old links from and puts the new
// ones (kLinksBuffers inside graphs; see launch_update_delta).
hipError_t enqueue_iteration(gf_ctx c, hipStream_t s, int fold_prev = 0, int reduce_after = 1,
                             int link_io = kLinksBuffers)
{
    Launch L = c->Lact;
    L.stream = s;
    hipError_t e = enqueue_gauge_steps(c, s, 1, nullptr, fold_prev);
    if (e != hipSuccess) return e;
    if (L.fused) {
        GF_TRY(K_UPDATE_DELTA, launch_update_delta(L, link_io));
    } else {
        GF_TRY(K_UPDATE, launch_update(L, 1, nullptr));
        GF_TRY(K_DELTA, launch_delta(L, 1, nullptr));
    }
    if (reduce_after) GF_TRY(K_REDUCE, launch_reduce(L, L.ncfg, 1, 1));
#undef GF_TRY
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
    // inside a chunk each iteration's final reduction rides on the next
    // iteration's first pass; the chunk's last one is launched on its own,
    // so the host reads a complete control block after every chunk
    const bool fold = fold_ok(c);
    for (int i = 0; i < c->chunk && e == hipSuccess; ++i)
        e = enqueue_iteration(c, c->cap_stream, fold && i > 0, !(fold && i + 1 < c->chunk));
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
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

gf_status run_chunks(gf_ctx c);
gf_status run_exact(gf_ctx c, long long n, long long pending);
gf_status reset_active(gf_ctx c);
gf_status compact_active(gf_ctx c);
void drop_graph(gf_ctx c);

// Run graph chunks until every configuration is done. On the fused path the
// iterations work on two-row copies of the links in the workspace: packed from
// the caller's array first, written back (third rows rebuilt) at the end.
// Storage of links and g for the coming iterations (a launch property; the
// captured graph holds the instances of one storage).
void set_link_storage(gf_ctx c, int f32)
{
    if (c->L.link_f32 == f32) return;
    c->L.link_f32 = f32;
    c->Lact.link_f32 = f32;
    drop_graph(c);
}

// Iterations of a call. FP64 link storage: the first update reads the
// caller's links (no copy in), and with n_exact > 1 (gf_step: exactly that
// many updates) the last one writes them back (no copy out); the updates in
// between run as graph chunks. Binary32 storage copies the links into the
// two-row buffer first. At the end, configurations whose links are in the
// two-row buffer (the call stopped on its rule, or made one update) are
// written back to the caller's array, third rows rebuilt.
gf_status run_until_done(gf_ctx c, long long n_exact = 0)
{
    gf_status st = reset_active(c);
    if (st != GF_OK) return st;
    if (c->L.fused) HIPCHK(c, launch_pack_links(c->L));
    const bool io = c->L.fused && !c->L.link_f32;
    long long first = 0;
    if (io) {
        HIPCHK(c, enqueue_iteration(c, c->stream, 0, 1, kLinksFromCaller));
        first = 1;
    }
    if (n_exact > 0) {
        const bool last = io && n_exact >= 2;
        st = run_exact(c, n_exact - first - (last ? 1 : 0), first);
        if (st != GF_OK) return st;
        if (last) HIPCHK(c, enqueue_iteration(c, c->stream, 0, 1, kLinksToCaller));
        if ((st = read_ctrl(c)) != GF_OK) return st;
        if (c->timing && (st = collect_timing(c)) != GF_OK) return st;
    } else {
        st = run_chunks(c);
        if (st != GF_OK) return st;
    }
    if (c->L.fused) {
        bool all_there = true;
        for (int k = 0; k < c->ncfg; ++k) all_there = all_there && c->h_ctrl[k].in_caller;
        if (!all_there) {
            HIPCHK(c, launch_unpack_links(c->L));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    return GF_OK;
}

// gf_fix_until and its batch form: with link_prec 1, iterations in
// single-precision storage until theta <= refine_theta, then (if theta_eps
// is below it) a measurement of the stored links and iterations in FP64
// storage down to theta_eps for every configuration that got there.
// Configurations that stopped in the first phase at the cap or on a
// non-finite value keep that outcome. max_iter bounds the updates of both
// phases together, per configuration.
gf_status fix_phases(gf_ctx c, double theta_eps, int64_t max_iter)
{
    std::vector<long long> before(c->ncfg);
    for (int k = 0; k < c->ncfg; ++k) before[k] = c->h_ctrl[k].iter;
    const bool two = c->link_prec == 1 && theta_eps < c->refine_theta;
    set_link_storage(c, c->link_prec == 1 ? 1 : 0);
    HIPCHK(c, launch_arm(c->L, c->ncfg, two ? c->refine_theta : theta_eps, max_iter, 0));
    gf_status st = run_until_done(c);
    if (st != GF_OK || !two) return st;
    std::vector<int> go(c->ncfg, 0);
    bool any = false;
    for (int k = 0; k < c->ncfg; ++k) {
        go[k] = c->h_ctrl[k].done == kConverged;
        any = any || go[k];
    }
    if (!any) return GF_OK;
    set_link_storage(c, 0);
    // the caller's links now hold the stored links: measure those of the
    // configurations that go on (not an update; the others keep their
    // stopping state and their last values), then apply the stopping rule
    // to the new measurement
    for (int k = 0; k < c->ncfg; ++k)
        if (go[k]) HIPCHK(c, launch_arm_one(c->L, k, theta_eps, max_iter - (c->h_ctrl[k].iter - before[k]), 0));
    HIPCHK(c, launch_delta(c->L, 1, nullptr));
    HIPCHK(c, launch_reduce(c->L, c->ncfg, 0, 1));
    for (int k = 0; k < c->ncfg; ++k)
        if (go[k]) HIPCHK(c, launch_arm_one(c->L, k, theta_eps, max_iter - (c->h_ctrl[k].iter - before[k]), 0));
    st = read_ctrl(c);
    if (st != GF_OK) return st;
    return run_until_done(c);
}

// n updates after `pending` ones already launched and not yet read back:
// whole chunks as graphs, the rest launched directly (iterations past the
// last would only launch passes that return at once); the control block is
// read back before the history ring could overflow. The caller reads it at
// the end.
gf_status run_exact(gf_ctx c, long long n, long long pending)
{
    if (n <= 0) return GF_OK;
    gf_status st;
    if (c->timing) {
        for (long long i = 0; i < n; ++i) {
            HIPCHK(c, enqueue_iteration(c, c->stream));
            if ((st = read_ctrl(c)) != GF_OK) return st;
            if ((st = collect_timing(c)) != GF_OK) return st;
        }
        return GF_OK;
    }
    if (n >= c->chunk && (st = build_graph(c)) != GF_OK) return st;
    const bool fold = fold_ok(c);
    long long left = n, since = pending;
    while (left > 0) {
        if (since + c->chunk + 2 > kHist) {
            if ((st = read_ctrl(c)) != GF_OK) return st;
            since = 0;
        }
        if (left >= c->chunk) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            left -= c->chunk;
            since += c->chunk;
        } else {
            const int r = (int)left;
            for (int i = 0; i < r; ++i)
                HIPCHK(c, enqueue_iteration(c, c->stream, fold && i > 0, !(fold && i + 1 < r)));
            since += left;
            left = 0;
        }
    }
    return GF_OK;
}

// Iterations until every configuration is done (the stopping rule, the cap
// or a non-finite value), a chunk at a time.
gf_status run_chunks(gf_ctx c)
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
            if (c->batch && (st = compact_active(c)) != GF_OK) return st;
        }
    }
    if (c->noalloc) {
        // the iterations of a chunk launched one after the other on the
        // caller's stream (the same kernels and reduction order as a graph)
        const bool fold = fold_ok(c);
        for (;;) {
            for (int i = 0; i < c->chunk; ++i)
                HIPCHK(c, enqueue_iteration(c, c->stream, fold && i > 0, !(fold && i + 1 < c->chunk)));
            gf_status st = read_ctrl(c);
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
        if (c->batch) {
            if ((st = compact_active(c)) != GF_OK) return st;
            if ((st = build_graph(c)) != GF_OK) return st;
        }
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

// Tile shapes of the 2D passes for every configuration, and the launch
// totals; uploads the configuration table.
// Tile maps and launch totals over a list of configurations.
void fill_map(gf_ctx c, const std::vector<int> &list, Batch &b, Launch &L)
{
    memset(&b, 0, sizeof(b));
    b.n = (int)list.size();
    for (int e = 0; e < b.n; ++e) {
        const Cfg &C = c->cfg[list[e]];
        b.idx[e] = list[e];
        b.off_site[e + 1] = b.off_site[e] + C.nblk_site;
        b.off_march[e + 1] = b.off_march[e] + C.nblk_march;
        // the z and t passes of a configuration's lines in registers run in
        // k_fft_line: 64 / line_lanes xy-sites times 4 lines per unit
        for (int mu = 0; mu < 4; ++mu)
            b.off_fft[mu][e + 1] = b.off_fft[mu][e] + ((mu >= 2 && C.line[mu - 2]) ? 0 : C.ax[mu].ntile);
        for (int a = 0; a < 2; ++a) {
            const int nq = 64 / line_lanes(C.dims[2 + a]);
            b.off_line[a][e + 1] = b.off_line[a][e] + (C.line[a] ? (C.V2 / nq) * (C.dims[3 - a] / 4) : 0);
        }
        b.off_xy[e + 1] = b.off_xy[e] + C.nxy;
        b.off_zt[e + 1] = b.off_zt[e] + C.nzt;
    }
    L.total_site_blocks = b.off_site[b.n];
    L.total_march_blocks = b.off_march[b.n];
    // Two site sets per block of the fused pass (512 work-items, one block
    // per CU instead of two of 256): where a set of kSiteBlock consecutive
    // sites is fewer than 8 whole x-rows (Lx = 24, 48, 64: 10.7, 5.3 and 4
    // rows), the doubled set halves the share of sites whose y-neighbour
    // another block owns, which pays for the barriers of 8 instead of 4 waves
    // (fused pass 2.3 %, 2.6 % and 4.3 % faster at 24^4, 48^4 and 64^4); at
    // 32^4 (8 rows) it is 1.7 % slower with FP64 link storage, 1.1 % faster
    // with single-precision storage. Linear sets with an even number per
    // walk in every configuration of the launch; GF_PAIR=0 / 1 turns it off /
    // on wherever it can run. The links and the partial sums are bitwise
    // those of one set per block.
    {
        const char *env = getenv("GF_PAIR");
        const int force = env ? atoi(env) : -1;
        bool can = force != 0 && b.n > 0, want = true;
        for (int e = 0; e < b.n && can; ++e) {
            const Cfg &C = c->cfg[list[e]];
            can = C.tile[0] == 0 && C.nb3 % 2 == 0;
            want = want && (kSiteBlock % C.dims[0] != 0 || kSiteBlock / C.dims[0] < 8);
        }
        L.march_pair = !can ? 0 : (force == 1 || want) ? 1 : 2;
    }
    for (int mu = 0; mu < 4; ++mu) L.total_fft_tiles[mu] = b.off_fft[mu][b.n];
    L.total_xy_tiles = b.off_xy[b.n];
    for (int a = 0; a < 2; ++a) {
        L.total_line[a] = b.off_line[a][b.n];
        L.line_m[a] = 0;
        for (int e = 0; e < b.n; ++e)
            if (c->cfg[list[e]].line[a]) L.line_m[a] |= 1 << line_len_bit(c->cfg[list[e]].dims[2 + a]);
    }
    L.total_zt_tiles = b.off_zt[b.n];
    L.ncfg = b.n;
    // which kernel instances the listed configurations need: power-of-two
    // and general extents, register and LDS-staged 2D passes, register
    // plane sizes, and the LDS-staged 1D passes of the axes whose lines do
    // not run in registers (an instance no listed configuration needs is
    // not launched)
    auto p2 = [](int v) { return (v & (v - 1)) == 0; };
    L.xy_p2 = L.xy_gen = L.zt_p2 = L.zt_gen = 0;
    L.xy_reg_any = L.xy_lds_any = L.zt_reg_any = L.zt_lds_any = 0;
    L.xy_m = L.zt_m = 0;
    for (int mu = 0; mu < 4; ++mu) L.ax_p2[mu] = L.ax_gen[mu] = 0;
    for (int e = 0; e < b.n; ++e) {
        const Cfg &C = c->cfg[list[e]];
        if (C.nxy) {
            ((p2(C.dims[0]) && p2(C.dims[1]) && p2(C.xyQ)) ? L.xy_p2 : L.xy_gen) = 1;
            (C.xy_reg ? L.xy_reg_any : L.xy_lds_any) = 1;
            if (C.xy_reg) L.xy_m |= 1 << line_len_bit(C.dims[0]);
        }
        if (C.nzt) {
            ((p2(C.dims[2]) && p2(C.dims[3])) ? L.zt_p2 : L.zt_gen) = 1;
            (C.zt_reg ? L.zt_reg_any : L.zt_lds_any) = 1;
            if (C.zt_reg) L.zt_m |= 1 << zt_shape_bit(C.dims[2], C.dims[3]);
        }
        for (int mu = 0; mu < 4; ++mu) {
            if (mu >= 2 && C.line[mu - 2]) continue;
            (p2(C.dims[mu]) ? L.ax_p2[mu] : L.ax_gen[mu]) = 1;
        }
    }
}

void drop_graph(gf_ctx c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
}

// Tile shapes of the 2D passes for every configuration, the full map and the
// launch totals; uploads the configuration table.
gf_status apply_schedule(gf_ctx c, int sched, const Tiles &tl)
{
    for (int k = 0; k < c->ncfg; ++k) {
        Cfg &C = c->cfg[k];
        C.xyQ = xy_feasible(C.dims) ? plan_xyQ(C.dims, tl.xy_target) : 1;
        C.xy_reg = ((sched == kSchedXYZT || sched == kSchedXY1D) && tl.xy_reg && xy_reg_fits(C)) ? 1 : 0;
        // every 1D z and t pass (those of schedules 1 and 2, and the plain
        // transform calls)
        for (int a = 0; a < 2; ++a) C.line[a] = (tl.line_reg && line_fits(C, a)) ? 1 : 0;
        if (C.xy_reg) C.xyQ = xy_reg_planes_for(C.dims[0]);  // the register passes' tile
        C.nxy = xy_feasible(C.dims) ? (C.dims[2] * C.dims[3]) / C.xyQ : 0;
        C.ztP = zt_feasible(C.dims) ? plan_ztP(C.dims, tl.zt_target) : 1;
        // the register pass's tile: zt_reg_p xy-sites (one width per
        // launch); a configuration whose Lx Ly it does not divide takes the
        // LDS-staged pass
        C.zt_reg = (sched == kSchedXYZT && tl.zt_reg && zt_reg_fits(C, tl.zt_reg_p)) ? 1 : 0;
        if (C.zt_reg) C.ztP = tl.zt_reg_p;
        C.nzt = zt_feasible(C.dims) ? C.V2 / C.ztP : 0;
        // bank-spreading pads, kept inside the 1/8 slack of the LDS tile
        const int xycap = C.xyQ * C.V2 <= 1024 ? 1024 : (C.xyQ * C.V2 <= 2048 ? 2048 : 4096);
        C.xyPad = (C.dims[1] * C.xyQ <= xycap / 8) ? 1 : 0;
        // zt tile: t-planes Tp = P Lz + ztPad elements apart with Tp = P (mod
        // 32), so that the lanes of one z-pencil access (p fastest, then t)
        // fall on distinct LDS banks: 16 consecutive lanes for 16-byte
        // elements (mod 16), 32 for 8-byte elements (mod 32)
        const int ztn = C.ztP * C.dims[2] * C.dims[3];
        const int ztcap = ztn <= 1024 ? 1024 : (ztn <= 2048 ? 2048 : 4096);
        const int r = C.ztP - C.ztP * C.dims[2];
        int zp = ((r % 32) + 32) % 32;
        if (zp * C.dims[3] > ztcap / 8) zp = ((r % 16) + 16) % 16;
        C.ztPad = (zp * C.dims[3] <= ztcap / 8) ? zp : 0;
    }
    std::vector<int> all(c->ncfg);
    for (int k = 0; k < c->ncfg; ++k) all[k] = k;
    fill_map(c, all, c->bmap, c->L);
    // tile capacities and twiddle layouts over every configuration (the
    // instance flags are set per launch list by fill_map)
    int xy_max = 0, zt_max = 0, mx = 0, my = 0, mz = 0, mt = 0;
    for (int k = 0; k < c->ncfg; ++k) {
        const Cfg &C = c->cfg[k];
        if (C.nxy) xy_max = std::max(xy_max, C.xyQ * C.V2);
        if (C.nzt) zt_max = std::max(zt_max, C.ztP * C.dims[2] * C.dims[3]);
        mx = std::max(mx, C.dims[0]);
        my = std::max(my, C.dims[1]);
        mz = std::max(mz, C.dims[2]);
        mt = std::max(mt, C.dims[3]);
    }
    c->L.zt_reg_groups = tl.zt_reg > 0 ? tl.zt_reg : 1;
    c->L.zt_reg_p = tl.zt_reg_p;
    c->L.xy_reg_groups = tl.xy_reg > 0 ? tl.xy_reg : 1;
    auto cap_for = [](int n) { return n <= 1024 ? 1024 : (n <= 2048 ? 2048 : 4096); };
    c->L.xy_cap = cap_for(xy_max);
    c->L.zt_cap = cap_for(zt_max);
    c->L.xy_th = c->L.xy_cap / tl.xy_ept;
    c->L.zt_th = c->L.zt_cap / tl.zt_ept;
    // a work-group of the 2D passes transforms the four fields of its tile
    // one after the other (the next one prefetched)
    c->L.xy_fpb = kFields;
    c->L.zt_fpb = kFields;
    c->L.xy_tw2 = mx;
    c->L.xy_tw_total = mx + my;
    c->L.zt_tw2 = mz;
    c->L.zt_tw_total = mz + mt;
    c->sched = sched;
    c->tiles = tl;
    // the active map starts as the full one
    c->bact = c->bmap;
    c->Lact = c->L;
    c->Lact.batch = c->d_batch_act;
    c->active = all;
    HIPCHK(c, hipMemcpyAsync(c->d_cfgs, c->cfg.data(), sizeof(Cfg) * c->ncfg, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_batch, &c->bmap, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_batch_act, &c->bact, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    // the K(p) table's layout follows the (z, t) pass chosen
    HIPCHK(c, launch_momentum_table(c->L));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    return GF_OK;
}

// Batch contexts: after a chunk, launch only the configurations still
// iterating (finished ones would only cost empty blocks). A new map means a
// new graph (0.4 to 1.3 ms to capture and instantiate), so the map is kept
// until the finished configurations hold a fifth of its marching blocks:
// their blocks leave at once.
gf_status compact_active(gf_ctx c)
{
    std::vector<int> act;
    long long w_act = 0, w_map = 0;
    for (int k = 0; k < c->ncfg; ++k)
        if (c->h_ctrl[k].done == kRunning) {
            act.push_back(k);
            w_act += c->cfg[k].nblk_march;
        }
    for (int k : c->active) w_map += c->cfg[k].nblk_march;
    if (act.empty() || act == c->active) return GF_OK;
    if (w_act * 5 > w_map * 4) return GF_OK;
    fill_map(c, act, c->bact, c->Lact);
    c->active = act;
    HIPCHK(c, hipMemcpyAsync(c->d_batch_act, &c->bact, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    drop_graph(c);
    return GF_OK;
}

// Reset the active map to every configuration (at the start of a call).
gf_status reset_active(gf_ctx c)
{
    if ((int)c->active.size() == c->ncfg) return GF_OK;
    std::vector<int> all(c->ncfg);
    for (int k = 0; k < c->ncfg; ++k) all[k] = k;
    fill_map(c, all, c->bact, c->Lact);
    c->active = all;
    HIPCHK(c, hipMemcpyAsync(c->d_batch_act, &c->bact, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    drop_graph(c);
    return GF_OK;
}

bool sched_feasible(gf_ctx c, int sched)
{
    for (int k = 0; k < c->ncfg; ++k) {
        const int *d = c->cfg[k].dims;
        if (sched == kSchedXY1D && !xy_feasible(d)) return false;
        if (sched == kSchedXYZT && !(xy_feasible(d) && zt_feasible(d))) return false;
    }
    return true;
}

std::string tune_key(gf_ctx c)
{
    std::string k = c->L.fp32 ? "c64" : "c128";
    for (int i = 0; i < c->ncfg; ++i) {
        char buf[64];
        snprintf(buf, sizeof buf, ":%dx%dx%dx%d", c->cfg[i].dims[0], c->cfg[i].dims[1], c->cfg[i].dims[2],
                 c->cfg[i].dims[3]);
        k += buf;
    }
    return k;
}

struct TuneEntry {
    std::string key;
    int sched;
    Tiles tiles;
};

// Schedules picked so far in this process, and those of GF_AUTOTUNE_CACHE
// (lines: key schedule xy_target xy_ept zt_target zt_ept).
std::vector<TuneEntry> &tune_cache()
{
    static std::vector<TuneEntry> cache;
    static bool loaded = false;
    if (!loaded) {
        loaded = true;
        const char *path = getenv("GF_AUTOTUNE_CACHE");
        if (path) {
            FILE *f = fopen(path, "r");
            if (f) {
                char key[4096];
                TuneEntry e;
                while (fscanf(f, "%4095s %d %d %d %d %d %d %d %d %d", key, &e.sched, &e.tiles.xy_target,
                              &e.tiles.xy_ept, &e.tiles.zt_target, &e.tiles.zt_ept, &e.tiles.zt_reg, &e.tiles.zt_reg_p,
                              &e.tiles.xy_reg, &e.tiles.line_reg) == 10) {
                    e.key = key;
                    cache.push_back(e);
                }
                fclose(f);
            }
        }
    }
    return cache;
}

bool valid_tiles(const Tiles &t)
{
    auto ok_target = [](int v) { return v == 1024 || v == 2048 || v == 4096; };
    return ok_target(t.xy_target) && ok_target(t.zt_target) && (t.xy_ept == 4 || t.xy_ept == 8) &&
           (t.zt_ept == 4 || t.zt_ept == 8) && (t.zt_reg == 0 || t.zt_reg == 1 || t.zt_reg == 2 || t.zt_reg == 4) &&
           (t.xy_reg == 0 || t.xy_reg == 1 || t.xy_reg == 2 || t.xy_reg == 4) && (t.zt_reg_p == 2 || t.zt_reg_p == 4 || t.zt_reg_p == 8) &&
           (t.line_reg == 0 || t.line_reg == 1);
}

// Tile choices of a fixed schedule: defaults, overridden by GF_XY_TARGET,
// GF_XY_EPT, GF_ZT_TARGET, GF_ZT_EPT.
Tiles env_tiles()
{
    Tiles t;
    auto rd = [](const char *name, int &v) {
        const char *e = getenv(name);
        if (e) v = atoi(e);
    };
    rd("GF_XY_TARGET", t.xy_target);
    rd("GF_XY_EPT", t.xy_ept);
    rd("GF_ZT_TARGET", t.zt_target);
    rd("GF_ZT_EPT", t.zt_ept);
    rd("GF_ZT_REG", t.zt_reg);
    rd("GF_XY_REG", t.xy_reg);
    rd("GF_ZT_REG_P", t.zt_reg_p);
    rd("GF_LINE_REG", t.line_reg);
    return valid_tiles(t) ? t : Tiles();
}

// Pick the transform schedule: the requested one, or (0) the fastest of the
// feasible candidates timed on this context's fields, cached per shape.
gf_status choose_schedule(gf_ctx c, int requested)
{
    if (requested == kSchedAuto && c->noalloc) {
        // no timing without events: the 2D passes wherever they fit
        requested = sched_feasible(c, kSchedXYZT) ? kSchedXYZT : sched_feasible(c, kSchedXY1D) ? kSchedXY1D : kSched1D;
    }
    if (requested != kSchedAuto) return apply_schedule(c, requested, env_tiles());
    const std::string key = tune_key(c);
    for (auto &e : tune_cache())
        if (e.key == key && sched_feasible(c, e.sched) && valid_tiles(e.tiles))
            return apply_schedule(c, e.sched, e.tiles);
    struct Cand {
        int sched;
        Tiles tiles;
    };
    std::vector<Cand> cands = {{kSched1D, Tiles()}};
    bool any_zreg = false, any_xreg = false, any_line = false;
    for (int k = 0; k < c->ncfg; ++k) {
        any_zreg = any_zreg || zt_reg_fits(c->cfg[k], 2) || zt_reg_fits(c->cfg[k], 4) || zt_reg_fits(c->cfg[k], 8);
        any_xreg = any_xreg || xy_reg_fits(c->cfg[k]);
        any_line = any_line || line_fits(c->cfg[k], 0) || line_fits(c->cfg[k], 1);
    }
    // the 1D z and t passes of schedules 1 and 2: in k_fft_line (the
    // default tiles) or LDS-staged
    if (any_line) {
        Tiles t;
        t.line_reg = 0;
        cands.push_back({kSched1D, t});
    }
    // (x, y) choices: LDS tiles (target, elements per work-item), or the
    // register passes with 1, 2 or 4 work-groups per tile; (z, t) choices: LDS
    // tiles, or the register pass with 1, 2 or 4 (the LDS tile then serves
    // only the plain transform calls)
    std::vector<Tiles> xs, zs;
    for (int xt : {1024, 4096})
        for (int xe : {4, 8}) {
            Tiles t;
            t.xy_target = xt;
            t.xy_ept = xe;
            t.xy_reg = 0;
            xs.push_back(t);
        }
    if (any_xreg)
        for (int g : {1, 2, 4}) {
            Tiles t;
            t.xy_reg = g;
            xs.push_back(t);
        }
    for (int zt : {2048, 4096})
        for (int ze : {4, 8}) {
            Tiles t;
            t.zt_target = zt;
            t.zt_ept = ze;
            t.zt_reg = 0;
            zs.push_back(t);
        }
    if (any_zreg)
        for (int P : {2, 4, 8})
            for (int g : {1, 2, 4}) {
                Tiles t;
                t.zt_reg = g;
                t.zt_reg_p = P;
                zs.push_back(t);
            }
    for (const Tiles &x : xs) {
        Tiles t = x;
        t.zt_reg = 0;
        if (sched_feasible(c, kSchedXY1D)) {
            cands.push_back({kSchedXY1D, t});
            if (any_line) {
                Tiles u = t;
                u.line_reg = 0;
                cands.push_back({kSchedXY1D, u});
            }
        }
        if (!sched_feasible(c, kSchedXYZT)) continue;
        for (const Tiles &z : zs) {
            t.zt_target = z.zt_target;
            t.zt_ept = z.zt_ept;
            t.zt_reg = z.zt_reg;
            cands.push_back({kSchedXYZT, t});
        }
    }
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return GF_ERR_HIP;
    const bool timing = c->timing;
    c->timing = false;
    // mean time of `reps` transform passes (after one warm-up pass) of a
    // candidate, each after a read of the link buffers: in an iteration the
    // fused pass streams them between the transform passes, so the fields
    // are not in L2 or the infinity cache when a transform pass starts
    auto time_cand = [&](const Cand &cd, int reps, double &ms_out) -> gf_status {
        gf_status st = apply_schedule(c, cd.sched, cd.tiles);
        if (st != GF_OK) return st;
        HIPCHK(c, enqueue_gauge_steps(c, c->stream, 0, nullptr));
        double total = 0.0;
        for (int r = 0; r < reps; ++r) {
            HIPCHK(c, launch_touch_links(c->L));
            HIPCHK(c, hipEventRecord(e0, c->stream));
            HIPCHK(c, enqueue_gauge_steps(c, c->stream, 0, nullptr));
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            total += ms;
        }
        ms_out = total / reps;
        return GF_OK;
    };
    // first pass: every candidate briefly; then the four fastest twice more
    // at more repetitions, the best of their three times kept (the
    // candidates are often within a few per cent of each other)
    std::vector<std::pair<double, int>> t1;
    for (int k = 0; k < (int)cands.size(); ++k) {
        double ms;
        gf_status st = time_cand(cands[k], 3, ms);
        if (st != GF_OK) return st;
        t1.push_back({ms, k});
    }
    std::sort(t1.begin(), t1.end());
    t1.resize(std::min<size_t>(t1.size(), 4));
    double best = 1e300;
    Cand pick = cands[t1[0].second];
    for (int pass = 0; pass < 2; ++pass)
        for (auto &e : t1) {
            double ms;
            gf_status st = time_cand(cands[e.second], 8, ms);
            if (st != GF_OK) return st;
            e.first = std::min(e.first, ms);
        }
    for (const auto &e : t1)
        if (e.first < best) {
            best = e.first;
            pick = cands[e.second];
        }
    c->timing = timing;
    c->ev_used = 0;
    // the fields were transformed in place: measure again so they hold Delta
    HIPCHK(c, enqueue_measure(c));
    gf_status st = apply_schedule(c, pick.sched, pick.tiles);
    if (st != GF_OK) return st;
    tune_cache().push_back({key, pick.sched, pick.tiles});
    const char *path = getenv("GF_AUTOTUNE_CACHE");
    if (path) {
        FILE *f = fopen(path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d %d %d %d %d %d\n", key.c_str(), pick.sched, pick.tiles.xy_target,
                    pick.tiles.xy_ept, pick.tiles.zt_target, pick.tiles.zt_ept, pick.tiles.zt_reg, pick.tiles.zt_reg_p,
                    pick.tiles.xy_reg, pick.tiles.line_reg);
            fclose(f);
        }
    }
    return GF_OK;
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
    if (c->noalloc) {
        c->h_ctrl = new Ctrl[ncfg];
    } else {
        HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipHostMalloc((void **)&c->h_ctrl, sizeof(Ctrl) * ncfg, hipHostMallocDefault));
    }
    c->histF.assign(ncfg, {});
    c->histT.assign(ncfg, {});
    c->kt.resize(K_N);
    for (int k = 0; k < K_N; ++k) c->kt[k].name = kNames[k];
    int dev = 0, ncu = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu < 1) ncu = 1;

    size_t o = 0;
    c->d_cfgs = (Cfg *)(c->ws + o);
    o += align_up(ncfg * sizeof(Cfg));
    c->d_batch = (Batch *)(c->ws + o);
    o += align_up(sizeof(Batch));
    c->d_batch_act = (Batch *)(c->ws + o);
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
        C.V2 = p.dims[0] * p.dims[1];
        C.V3 = C.V2 * p.dims[2];
        C.nblk_site = (C.V + kSiteBlock - 1) / kSiteBlock;
        C.nb3 = plan_tile(p.dims, C.tile, C.ntile);
        C.tch = (ncfg > 1) ? plan_tchunk_batch(p.dims)
                           : plan_tchunk(p.dims, C.nb3, p.link_prec == 0, kMarchResidentPerCU * ncu);
        C.nblk_march = C.nb3 * (p.dims[3] / C.tch);
        C.U = (double2 *)links[k];
        C.U12[0] = (double2 *)(c->ws + l.links12a);
        C.U12[1] = (double2 *)(c->ws + l.links12b);
        C.U12f[0] = l.links12fa ? (float2 *)(c->ws + l.links12fa) : nullptr;
        C.U12f[1] = l.links12fb ? (float2 *)(c->ws + l.links12fb) : nullptr;
        C.g12f = l.g12f ? (float2 *)(c->ws + l.g12f) : nullptr;
        C.fields = c->ws + l.fields;
        C.fields2 = c->ws + l.fields2;
        C.g = (double2 *)(c->ws + l.g);
        C.partials = (double *)(c->ws + l.partials);
        C.ctrl = (Ctrl *)(c->ws + ctrl_base) + k;
        C.sin2 = (const double *)(c->ws + l.sin2);
        C.tw = c->ws + l.tw;
        C.kmom = c->ws + l.kmom;
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
        o = l.total;
    }
    if (o > ws_bytes) {
        c->err = "workspace too small";
        return GF_ERR_SHAPE;
    }
    c->L.cfgs = c->d_cfgs;
    c->L.batch = c->d_batch;
    {
        std::vector<int> all(ncfg);
        for (int k = 0; k < ncfg; ++k) all[k] = k;
        fill_map(c, all, c->bmap, c->L);
    }
    c->L.max_lds_elems = max_lds;
    c->L.fp32 = params[0].fft_prec;
    // single-precision storage exists only in the fused exchange pass
    c->L.fused = (getenv("GF_NOFUSE") && params[0].link_prec == 0) ? 0 : 1;
    c->L.link_f32 = 0;
    c->link_prec = params[0].link_prec;
    c->refine_theta = params[0].refine_theta > 0.0 ? params[0].refine_theta : 1e-10;
    c->L.any_reunit = 0;
    for (int k = 0; k < ncfg; ++k) c->L.any_reunit |= params[k].reunit_every > 0;
    c->L.ncfg = ncfg;
    c->L.stream = c->stream;

    HIPCHK(c, hipMemcpyAsync(c->d_cfgs, c->cfg.data(), sizeof(Cfg) * ncfg, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_batch, &c->bmap, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_batch_act, &c->bmap, sizeof(Batch), hipMemcpyHostToDevice, c->stream));
    for (int k = 0; k < ncfg; ++k) {
        HIPCHK(c, hipMemcpyAsync((void *)c->cfg[k].sin2, sin2s[k].data(), sin2s[k].size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync((void *)c->cfg[k].tw, tws[k].data(), tws[k].size(), hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, set_lds_limits());
    HIPCHK(c, launch_arm(c->L, ncfg, 0.0, 0, 1));
    HIPCHK(c, enqueue_measure(c));
    gf_status st = read_ctrl(c);
    if (st != GF_OK) return st;
    if ((st = choose_schedule(c, params[0].fft_schedule)) != GF_OK) return st;
    // the chunk graph of FP64 link storage is captured and instantiated here,
    // not inside the first call that runs a whole chunk (about 0.3 ms, more
    // than an iteration)
    if (!c->noalloc && c->link_prec == 0) return build_graph(c);
    return GF_OK;
}

// Workspace of a functional-only context: the header, g [3][3][V] and the
// partial sums of the site blocks.
struct FnLayout {
    size_t g, partials, total;
};

FnLayout fn_layout(const gf_params &p)
{
    const size_t V = (size_t)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
    FnLayout l;
    size_t o = header_bytes(1) + align_up(sizeof(Ctrl));
    l.g = o;
    o = align_up(o + 9 * V * 16);
    l.partials = o;
    o = align_up(o + ((V + kSiteBlock - 1) / kSiteBlock) * 4 * sizeof(double));
    l.total = o;
    return l;
}

gf_status setup_functional(gf_ctx c, const gf_params *p, void *links, void *d_ws, void *stream)
{
    c->functional_only = true;
    c->noalloc = true;
    c->ncfg = 1;
    c->params.assign(p, p + 1);
    c->stream = (hipStream_t)stream;
    c->ws = (char *)d_ws;
    c->histF.assign(1, {});
    c->histT.assign(1, {});
    c->kt.resize(K_N);
    for (int k = 0; k < K_N; ++k) c->kt[k].name = kNames[k];
    size_t o = 0;
    c->d_cfgs = (Cfg *)(c->ws + o);
    o += align_up(sizeof(Cfg));
    c->d_batch = (Batch *)(c->ws + o);
    o += align_up(sizeof(Batch));
    c->d_batch_act = (Batch *)(c->ws + o);
    o += align_up(sizeof(Batch));
    c->d_scalar = (double *)(c->ws + o);
    o += align_up(64);
    const FnLayout l = fn_layout(*p);
    c->cfg.assign(1, Cfg{});
    Cfg &C = c->cfg[0];
    for (int mu = 0; mu < 4; ++mu) C.dims[mu] = p->dims[mu];
    C.V = p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
    C.V2 = p->dims[0] * p->dims[1];
    C.V3 = C.V2 * p->dims[2];
    C.nblk_site = (C.V + kSiteBlock - 1) / kSiteBlock;
    C.U = (double2 *)links;
    C.g = (double2 *)(c->ws + l.g);
    C.partials = (double *)(c->ws + l.partials);
    C.ctrl = (Ctrl *)(c->ws + o);
    c->L.cfgs = c->d_cfgs;
    c->L.batch = c->d_batch;
    c->L.ncfg = 1;
    c->L.stream = c->stream;
    HIPCHK(c, hipMemcpyAsync(c->d_cfgs, c->cfg.data(), sizeof(Cfg), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
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

// Workspace of gf_fix_until_static: one array per GPU, held by the loaded
// library until the process ends. In host code `scratch` names a host-side
// stand-in, not device memory: only the address returned by
// hipGetSymbolAddress for the current device may be handed to kernels or
// copies.
static __device__ __align__(256) unsigned char scratch[GF_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t static_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
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
        if (params[k].fft_prec != params[0].fft_prec || params[k].chunk != params[0].chunk ||
            params[k].fft_schedule != params[0].fft_schedule || params[k].link_prec != params[0].link_prec ||
            params[k].refine_theta != params[0].refine_theta)
            return 0;
    return workspace_total(n_cfg, params);
}

static gf_status init_common(gf_ctx *out, int32_t n_cfg, const gf_params *params, void *const *links, void *d_ws,
                             size_t ws_bytes, void *stream, bool batch, bool noalloc = false)
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
    c->noalloc = noalloc;
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

size_t gf_workspace_bytes_functional(const gf_params *params)
{
    if (!valid_params(params)) return 0;
    return fn_layout(*params).total;
}

gf_status gf_init_functional(gf_ctx *ctx, const gf_params *params, void *d_links, void *d_ws, size_t ws_bytes,
                             void *stream)
{
    if (!ctx || !params || !d_links || !d_ws) return GF_ERR_ARG;
    *ctx = nullptr;
    if (!valid_params(params)) return GF_ERR_SHAPE;
    if (ws_bytes < fn_layout(*params).total) return GF_ERR_SHAPE;
    if (((uintptr_t)d_ws) % kAlign) return GF_ERR_ARG;
    gf_ctx c = new gf_ctx_s();
    gf_status st = setup_functional(c, params, d_links, d_ws, stream);
    if (st != GF_OK) {
        gf_destroy(c);
        return st;
    }
    *ctx = c;
    return GF_OK;
}

gf_status gf_init_batch(gf_ctx *ctx, int32_t n_cfg, const gf_params *params, void *const *d_links, void *d_ws,
                        size_t ws_bytes, void *stream)
{
    if (n_cfg < 1 || n_cfg > kMaxCfg) return GF_ERR_ARG;
    return init_common(ctx, n_cfg, params, d_links, d_ws, ws_bytes, stream, true);
}

gf_status gf_fix_until_static(const gf_params *params, void *d_links, double theta_eps, int64_t max_iter,
                              int64_t *iters, double *F, double *theta, void *stream)
{
    if (!params || !d_links || max_iter < 0) return GF_ERR_ARG;
    const size_t need = gf_workspace_bytes(params);
    if (need == 0) return GF_ERR_SHAPE;
    if (need > (size_t)GF_STATIC_SCRATCH_BYTES) return GF_ERR_SHAPE;  // lattice too large for the scratch
    void *ws = nullptr;
    if (static_scratch(&ws) != hipSuccess) return GF_ERR_HIP;
    gf_ctx c = nullptr;
    void *l[1] = {d_links};
    gf_status st = init_common(&c, 1, params, l, ws, (size_t)GF_STATIC_SCRATCH_BYTES, stream, false, true);
    if (st != GF_OK) return st;
    st = gf_fix_until(c, theta_eps, max_iter, iters, F, theta);
    gf_destroy(c);
    return st;
}

gf_status gf_functional(gf_ctx c, double *F, double *theta)
{
    if (!c) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
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
    if (c->functional_only) return GF_ERR_STATE;
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
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    if (n > 0) {
        set_link_storage(c, c->link_prec == 1 ? 1 : 0);
        HIPCHK(c, launch_arm(c->L, c->ncfg, -1.0, n, 0));
        gf_status st = run_until_done(c, n);
        if (st != GF_OK) return st;
    }
    if (F) *F = c->h_ctrl[0].F;
    if (theta) *theta = c->h_ctrl[0].theta;
    return status_from_done(c, false);
}

gf_status gf_fix_until(gf_ctx c, double theta_eps, int64_t max_iter, int64_t *iters, double *F, double *theta)
{
    if (!c || max_iter < 0) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    const long long before = c->h_ctrl[0].iter;
    gf_status st = fix_phases(c, theta_eps, max_iter);
    if (st != GF_OK) return st;
    if (iters) *iters = c->h_ctrl[0].iter - before;
    if (F) *F = c->h_ctrl[0].F;
    if (theta) *theta = c->h_ctrl[0].theta;
    return status_from_done(c, true);
}

gf_status gf_fix_until_batch(gf_ctx c, double theta_eps, int64_t max_iter, int64_t *iters, double *F, double *theta)
{
    if (!c || max_iter < 0) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    std::vector<long long> before(c->ncfg);
    for (int k = 0; k < c->ncfg; ++k) before[k] = c->h_ctrl[k].iter;
    gf_status st = fix_phases(c, theta_eps, max_iter);
    if (st != GF_OK) return st;
    for (int k = 0; k < c->ncfg; ++k) {
        if (iters) iters[k] = c->h_ctrl[k].iter - before[k];
        if (F) F[k] = c->h_ctrl[k].F;
        if (theta) theta[k] = c->h_ctrl[k].theta;
    }
    return status_from_done(c, true);
}

static gf_status history_of(gf_ctx c, int k, int64_t cap, double *F_hist, double *theta_hist, int64_t *n)
{
    const auto &F = c->histF[k];
    const auto &T = c->histT[k];
    const int64_t avail = (int64_t)F.size();
    if (n) *n = avail;
    const int64_t m = cap < avail ? cap : avail;
    for (int64_t k = 0; k < m; ++k) {
        if (F_hist) F_hist[k] = F[k];
        if (theta_hist) theta_hist[k] = T[k];
    }
    return GF_OK;
}

gf_status gf_history(gf_ctx c, int64_t cap, double *F_hist, double *theta_hist, int64_t *n)
{
    if (!c || cap < 0) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    return history_of(c, 0, cap, F_hist, theta_hist, n);
}

gf_status gf_history_batch(gf_ctx c, int32_t k, int64_t cap, double *F_hist, double *theta_hist, int64_t *n)
{
    if (!c || cap < 0 || k < 0 || k >= c->ncfg) return GF_ERR_ARG;
    return history_of(c, k, cap, F_hist, theta_hist, n);
}

gf_status gf_delta(gf_ctx c, void *d_delta)
{
    if (!c || !d_delta) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, launch_delta(c->L, 0, (double2 *)d_delta));
    HIPCHK(c, launch_reduce(c->L, 1, 0, 0));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_gauge(gf_ctx c, void *d_g)
{
    if (!c || !d_g) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, launch_delta(c->L, 0, nullptr));
    HIPCHK(c, enqueue_gauge_steps(c, c->stream, 0, (double2 *)d_g));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_apply_gauge(gf_ctx c, const void *d_g)
{
    if (!c || !d_g) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    HIPCHK(c, launch_update(c->L, 0, (const double2 *)d_g));
    HIPCHK(c, enqueue_measure(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

gf_status gf_heatbath(gf_ctx c, double beta, int32_t n_sweeps, int32_t n_or, uint64_t seed, int64_t sweep0)
{
    if (!c || n_sweeps < 0 || n_or < 0 || !(beta >= 0.0) || sweep0 < 0) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    const Cfg &C = c->cfg[0];
    for (int mu = 0; mu < 4; ++mu)
        if (C.dims[mu] % 2) return GF_ERR_SHAPE;
    for (int i = 0; i < n_sweeps; ++i) {
        HIPCHK(c, launch_heatbath_sweep(c->L, C.V, 0, beta, seed, (long long)(sweep0 + i)));
        for (int r = 0; r < n_or; ++r) HIPCHK(c, launch_heatbath_sweep(c->L, C.V, 1, beta, seed, 0));
    }
    // the links changed: measure them again, as after any other change
    HIPCHK(c, enqueue_measure(c));
    return read_ctrl(c);
}

gf_status gf_plaquette(gf_ctx c, double *P)
{
    if (!c || !P) return GF_ERR_ARG;
    if (c->batch) return GF_ERR_STATE;
    const Cfg &C = c->cfg[0];
    HIPCHK(c, launch_plaquette(c->L, C.nblk_site, c->d_scalar));
    double h = 0.0;
    HIPCHK(c, hipMemcpyAsync(&h, c->d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *P = h;
    return std::isfinite(h) ? GF_OK : GF_ERR_NONFINITE;
}

gf_status gf_fft(gf_ctx c, void *d_fields, int32_t nfields, int32_t sign)
{
    if (!c || !d_fields || nfields < 1 || nfields > 65535 || (sign != 1 && sign != -1)) return GF_ERR_ARG;
    if (c->functional_only) return GF_ERR_STATE;
    if (c->batch) return GF_ERR_STATE;
    const Launch &L = c->L;
    switch (c->sched) {
    case kSchedXYZT:
        HIPCHK(c, launch_fft_xy(L, sign, d_fields, nfields, 0));
        HIPCHK(c, launch_fft_zt(L, 0, sign, d_fields, nfields, 0));
        break;
    case kSchedXY1D:
        HIPCHK(c, launch_fft_xy(L, sign, d_fields, nfields, 0));
        HIPCHK(c, launch_fft_axis(L, 2, sign, 0, d_fields, nfields, 0));
        HIPCHK(c, launch_fft_axis(L, 3, sign, 0, d_fields, nfields, 0));
        break;
    default:
        for (int mu = 0; mu < 4; ++mu) HIPCHK(c, launch_fft_axis(L, mu, sign, 0, d_fields, nfields, 0));
    }
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
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_ctrl) {
        if (c->noalloc)
            delete[] c->h_ctrl;
        else
            (void)hipHostFree(c->h_ctrl);
    }
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

int32_t gf_fft_schedule(gf_ctx c) { return c ? c->sched : 0; }

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

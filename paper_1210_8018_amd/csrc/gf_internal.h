// Internal structures shared by the kernels (gf_kernels.hip) and the host
// runtime (gf_runtime.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfk {

// Device pointers of the configuration table carry the global address space
// in the device code of the kernel sources (those that include gf_device.h),
// so that accesses through them are global (not flat) memory instructions:
// flat accesses also count as LDS operations, and every wait for LDS would
// then wait for them as well. The layout is the same (64-bit pointers).
#if defined(__HIP_DEVICE_COMPILE__) && defined(GF_KERNEL_SOURCE)
#define GF_GLOBAL __attribute__((address_space(1)))
#else
#define GF_GLOBAL
#endif

constexpr int kMaxCfg = 64;        // configurations per batch context
constexpr int kHist = 256;         // device ring of (F, theta) per configuration
constexpr int kSiteBlock = 256;    // work-items per site-parallel block
constexpr int kFftThreads = 256;   // work-items per transform tile
constexpr int kMaxStages = 8;      // radix stages per axis
constexpr int kFields = 4;         // packed transform fields per site
constexpr int kTileElems2D = 4096; // largest LDS tile (elements) of the 2D passes


enum : int { kRunning = 0, kConverged = 1, kMaxIter = 2, kNonFinite = 3 };

// Transform lines held in registers (k_fft_line, k_fft_xy_reg,
// k_fft_xy_inv_reg): lengths 16 and 24 over two lanes of a wave, 32, 48 and
// 64 over four; each length is its own kernel instance, marked by a bit.
__host__ __device__ constexpr bool line_len_ok(int L) { return L == 16 || L == 24 || L == 32 || L == 48 || L == 64; }
__host__ __device__ constexpr int line_lanes(int L) { return L >= 32 ? 4 : 2; }
__host__ __device__ constexpr int line_len_bit(int L) { return L == 16 ? 0 : L == 24 ? 1 : L == 32 ? 2 : L == 48 ? 3 : 4; }
// planes per tile of the register (x, y) passes: a tile stays within 4096
// elements (the LDS-staged inverse pass serves the same tiles)
__host__ __device__ constexpr int xy_reg_planes_for(int L) { return L == 16 ? 8 : L == 24 ? 4 : L == 32 ? 2 : 1; }
// (z, t) plane shapes of the register (z, t) passes, one instance each:
// 32 x 32 (k_fft_zt_reg), 16 x 16, 24 x 24, 16 x 32, 48 x 48
// (k_fft_zt_lines); -1 none
__host__ __device__ constexpr int zt_shape_bit(int Lz, int Lt)
{
    return (Lz == 16 && Lt == 16)   ? 0
           : (Lz == 24 && Lt == 24) ? 1
           : (Lz == 32 && Lt == 32) ? 2
           : (Lz == 16 && Lt == 32) ? 3
           : (Lz == 48 && Lt == 48) ? 4
                                    : -1;
}

// Transform schedules: which passes make up the 4D transform, scaling and
// inverse (the scaling is always fused into the pass that completes the
// forward transform).
enum : int {
    kSchedAuto = 0,
    kSched1D = 1,    // x, y, z, t+scale, z, y, x (1D passes) + gauge
    kSchedXY1D = 2,  // xy, z, t+scale, z, xy^-1+gauge
    kSchedXYZT = 3,  // xy, zt+scale, xy^-1+gauge
    kSchedCount = 4
};

// Device control block of one configuration. Written only by device code
// (the arming and reduction kernels), read back by the host per chunk.
struct Ctrl {
    double eps;          // stop once theta <= eps
    double F, theta;     // latest measurement
    long long iter;      // updates since init
    long long max_iter;  // absolute cap on iter
    int done;            // kRunning / kConverged / kMaxIter / kNonFinite
    int cur;             // current two-row link buffer, U12[cur]
    int ru_now;          // this iteration also projects the new links (set before the fused pass)
    int in_caller;       // the current links are the caller's array U (full 3x3), not U12[cur]
    int pad2;
    double hist[kHist][2];  // (F, theta) after update k at slot k % kHist
};

// One axis of a 1D transform pass: tiles of P pencils of length L, elements
// of a pencil spaced S apart in memory.
struct FftAxis {
    int L, S, P;
    int ntile;        // tiles per field
    int inner_chunks; // S / P for axes > 0
    int nstage;
    int radix[kMaxStages];
};

struct Cfg {
    int dims[4];
    int V;
    int V2;               // Lx * Ly
    int V3;               // Lx * Ly * Lz
    int nblk_site;        // site blocks of kSiteBlock
    int nb3;              // blocks over the (x, y, z) volume
    int tile[3];          // (x, y, z) extent of one block's sites; tile[0] = 0: kSiteBlock consecutive sites
    int ntile[3];         // tiles along x, y, z (tile mode)
    int tch;              // t-slices marched by one block
    int nblk_march;       // nb3 * (Lt / tch): blocks of the marching kernels
    GF_GLOBAL double2 *U;        // links [4][3][3][V] (the caller's array)
    GF_GLOBAL double2 *U12[2];   // two-row links [4][2][3][V], two buffers (workspace)
    GF_GLOBAL float2 *U12f[2];   // the same two link buffers in single-precision storage (link_prec 1)
    GF_GLOBAL float2 *g12f;      // two-row g in single-precision storage
    GF_GLOBAL void *fields;      // packed transform fields [4][V], double2 or float2
    GF_GLOBAL void *fields2;     // the filtered fields Delta~ [4][V] read by the fused pass
    GF_GLOBAL double2 *g;        // gauge field [3][3][V]
    GF_GLOBAL double *partials;  // [nblk_march or nblk_site][4]: (F hi, F lo, theta hi, theta lo)
    GF_GLOBAL Ctrl *ctrl;
    GF_GLOBAL const double *sin2;  // 4 sin^2(pi n / L_mu), axis mu at sin2 + sin2_off[mu]
    int sin2_off[4];
    GF_GLOBAL const void *tw;    // twiddles exp(-2 pi i e / L_mu), axis mu at tw + tw_off[mu]
    int tw_off[4];
    double kfac;          // (alpha / 2) * p2max / V
    GF_GLOBAL void *kmom;        // K(p) per momentum site [V], double (FP64 transform) or float (FP32)
    int reunit_every;
    FftAxis ax[4];
    int xyQ, nxy;         // xy pass: Q consecutive xy-planes per tile, nxy tiles per field
    int ztP, nzt;         // zt pass: P consecutive xy-sites per tile, nzt tiles per field
    int xyPad;            // LDS elements added to every x-row of an xy tile (bank spreading)
    int ztPad;            // LDS elements added to every t-plane of a zt tile
    int zt_reg;           // the scaled (z, t) pass runs in registers: k_fft_zt_reg (32 x 32), k_fft_zt_lines (the others)
    int xy_reg;           // the iteration's (x, y) passes run in k_fft_xy_reg / k_fft_xy_inv_reg (Lx = Ly = 16 to 64)
    int line[2];          // the 1D z (line[0]) / t (line[1]) passes run in k_fft_line (that extent 16 to 64)
};

// Block-to-configuration maps for every launch shape of a batch: entry e
// covers configuration idx[e], blocks [off[e], off[e + 1]).
struct Batch {
    int n;
    int idx[kMaxCfg];
    int off_site[kMaxCfg + 1];
    int off_march[kMaxCfg + 1];
    int off_fft[4][kMaxCfg + 1];
    int off_xy[kMaxCfg + 1];
    int off_zt[kMaxCfg + 1];
    int off_line[2][kMaxCfg + 1];  // k_fft_line units (64 / line_lanes xy-sites x 4 lines) of the z and t passes
};

struct Launch {
    const Cfg *cfgs;      // device array
    const Batch *batch;   // device struct
    int total_site_blocks;
    int total_march_blocks;
    int march_pair;       // the fused pass takes two site sets per block (512 work-items): 0 never,
                          // 1 always, 2 with single-precision link storage only
    int total_fft_tiles[4];
    int total_xy_tiles;
    int total_zt_tiles;
    int xy_cap, zt_cap;            // 2D tile capacity variant (1024, 2048 or 4096 elements)
    int xy_th, zt_th;              // work-group size of the 2D passes (capacity / elements per work-item)
    int xy_fpb, zt_fpb;            // fields per work-group of the 2D passes (the next one prefetched)
    int xy_p2, zt_p2;              // some configuration has power-of-two extents in that pass
    int xy_gen, zt_gen;            // some configuration has not
    int ax_p2[4], ax_gen[4];       // same for the 1D passes of each axis
    int xy_tw2, xy_tw_total;       // LDS twiddle layout of the xy pass: y table offset, entries
    int zt_tw2, zt_tw_total;       // same for the zt pass
    int zt_reg_any, zt_lds_any;    // scaled zt pass: some configuration in k_fft_zt_reg / in k_fft_zt
    int zt_reg_groups;             // work-groups per tile of k_fft_zt_reg (1, 2 or 4: fields split among them)
    int zt_reg_p;                  // xy-sites per tile of k_fft_zt_reg / k_fft_zt_lines (2, 4 or 8)
    int zt_m;                      // (z, t) plane shapes of the register passes present (bits zt_shape_bit)
    int xy_reg_any, xy_lds_any;    // iteration's xy passes: some configuration in the register / LDS-staged ones
    int xy_reg_groups;             // work-groups per tile of the register xy passes
    int xy_m;                      // their plane sizes present (bits line_len_bit)
    int total_line[2];             // k_fft_line units of the z and t passes (0: no configuration has them)
    int line_m[2];                 // line lengths among them (bits line_len_bit)
    int max_lds_elems;    // 1D passes: largest P * L
    int fp32;             // transform precision
    int fused;            // iterations use the fused update + divergence kernel
    int link_f32;         // links and g held in single-precision two-row storage (this phase)
    int any_reunit;       // some configuration projects its links every R updates
    int ncfg;
    hipStream_t stream;
};

hipError_t launch_arm(const Launch &L, int ncfg, double eps, long long add_iters, int reset_iter);
// the same for configuration k alone
hipError_t launch_arm_one(const Launch &L, int k, double eps, long long add_iters, int reset_iter);
hipError_t launch_delta(const Launch &L, int respect_done, double2 *full_delta);
hipError_t launch_reduce(const Launch &L, int ncfg, int count_iter, int respect_done);
hipError_t launch_fft_axis(const Launch &L, int axis, int sign, int mode, void *fields_override,
                           int nfields, int respect_done);
// fold_reduce: the pass also does the final reduction of the previous update
// (in place of launch_reduce after it); only where can_fold_reduce(L).
hipError_t launch_fft_xy(const Launch &L, int sign, void *fields_override, int nfields, int respect_done,
                         int fold_reduce = 0);
bool can_fold_reduce(const Launch &L);
hipError_t launch_fft_xy_inv_gauge(const Launch &L, int respect_done, double2 *g_override);
hipError_t launch_fft_zt(const Launch &L, int mode, int sign, void *fields_override, int nfields, int respect_done);
hipError_t launch_fft_zt_scale(const Launch &L, int respect_done);
hipError_t set_lds_limits();
hipError_t launch_gauge(const Launch &L, int respect_done, double2 *g_override);
hipError_t launch_update(const Launch &L, int respect_done, const double2 *g_override);
// Where the fused pass of an update takes the old links from and puts the
// new ones (FP64 link storage): the two-row buffers, or the caller's array
// for the first update of a call (old links) or the last of a gf_step call
// (new links).
enum : int { kLinksBuffers = 0, kLinksFromCaller = 1, kLinksToCaller = 2 };
hipError_t launch_update_delta(const Launch &L, int link_io);
hipError_t launch_pack_links(const Launch &L);
hipError_t launch_momentum_table(const Launch &L);
// reads every configuration's two-row link buffers (cache eviction before a timed pass)
hipError_t launch_touch_links(const Launch &L);
hipError_t launch_heatbath_sweep(const Launch &L, int V, int mode, double beta, uint64_t seed, long long n);
hipError_t launch_plaquette(const Launch &L, int nblk, double *out);
hipError_t launch_unpack_links(const Launch &L);
hipError_t launch_functional_g_impl(const Launch &L, int nblk, const double *omega, double scale, double *out);
hipError_t launch_functional_g_backward_impl(const Launch &L, int nblk, const double *omega, double scale,
                                             double *d_omega, double2 *d_U);

}  // namespace gfk

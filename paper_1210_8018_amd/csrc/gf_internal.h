// Internal structures shared by the kernels (gf_kernels.hip) and the host
// runtime (gf_runtime.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfk {

constexpr int kMaxCfg = 64;      // configurations per batch context
constexpr int kHist = 256;       // device ring of (F, theta) per configuration
constexpr int kSiteBlock = 256;  // work-items per site-parallel block
constexpr int kFftThreads = 256; // work-items per transform tile
constexpr int kMaxStages = 8;    // radix stages per axis
constexpr int kFields = 4;       // packed transform fields per site

enum : int { kRunning = 0, kConverged = 1, kMaxIter = 2, kNonFinite = 3 };

// Device control block of one configuration. Written only by device code
// (the arming and reduction kernels), read back by the host per chunk.
struct Ctrl {
    double eps;          // stop once theta <= eps
    double F, theta;     // latest measurement
    long long iter;      // updates since init
    long long max_iter;  // absolute cap on iter
    int done;            // kRunning / kConverged / kMaxIter / kNonFinite
    int pad;
    double hist[kHist][2];  // (F, theta) after update k at slot k % kHist
};

// One axis of the 4D transform: tiles of P pencils of length L, elements of
// a pencil spaced S apart in memory.
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
    int nblk_site;        // site blocks of kSiteBlock
    double2 *U;           // links [4][3][3][V]
    void *fields;         // packed transform fields [4][V], double2 or float2
    double2 *g;           // gauge field [3][3][V]
    double *partials;     // [nblk_site][4]: (F hi, F lo, theta hi, theta lo)
    Ctrl *ctrl;
    const double *sin2;   // 4 sin^2(pi n / L_mu), axis mu at sin2 + sin2_off[mu]
    int sin2_off[4];
    const void *tw;       // twiddles exp(-2 pi i e / L_mu), axis mu at tw + tw_off[mu]
    int tw_off[4];
    double kfac;          // (alpha / 2) * p2max / V
    int reunit_every;
    FftAxis ax[4];
};

// Block-to-configuration maps for every launch shape of a batch.
struct Batch {
    int n;
    int off_site[kMaxCfg + 1];
    int off_fft[4][kMaxCfg + 1];
    int max_lds_elems;    // largest P * L over configurations and axes
};

// Launchers (gf_kernels.hip). `active` lists configuration slots; kernels
// skip configurations whose control block says done when respect_done != 0.
struct Launch {
    const Cfg *cfgs;      // device array
    const Batch *batch;   // device struct
    int total_site_blocks;
    int total_fft_tiles[4];
    int max_lds_elems;
    int fp32;             // transform precision
    hipStream_t stream;
};

hipError_t launch_arm(const Launch &L, int ncfg, double eps, long long add_iters, int reset_iter);
hipError_t launch_delta(const Launch &L, int respect_done, double2 *full_delta);
hipError_t launch_reduce(const Launch &L, int ncfg, int count_iter, int respect_done);
hipError_t launch_fft_axis(const Launch &L, int axis, int sign, int mode, void *fields_override,
                           int nfields, int respect_done);
hipError_t launch_gauge(const Launch &L, int respect_done, double2 *g_override);
hipError_t launch_update(const Launch &L, int respect_done, const double2 *g_override);
hipError_t launch_functional_g(const Launch &L, const double *omega);
hipError_t launch_functional_g_backward(const Launch &L, const double *omega, double grad_out,
                                        double *d_domega, double2 *d_dU);

}  // namespace gfk

/*
 * gf.h - C ABI of the MI355X (gfx950) library for Fourier-accelerated
 * steepest-descent Landau gauge fixing of 4D SU(3) lattice gauge fields
 * (Cardoso, Silva, Oliveira, Bicudo, "GPU implementation of a Landau gauge
 * fixing algorithm", Lattice 2012).
 *
 * The problem (section 1, Eq. 1): maximise over gauge transformations g(x)
 *   F_U[g] = 1/(4 N_c V) sum_x sum_mu Re Tr[ g(x) U_mu(x) g^dag(x+mu) ],  N_c = 3,
 * by the Fourier-accelerated iteration of Alg. 1 (Eq. 2 to Eq. 5), monitored
 * by theta = 1/(N_c V) sum_x Tr[Delta(x) Delta^dag(x)] (Eq. 4) and stopped
 * once theta <= eps (the paper uses eps = 1e-15).
 *
 * Conventions shared by every call:
 *   - dims = (Lx, Ly, Lz, Lt); each L is 2^a 3^b with 2 <= L <= 256;
 *     V = Lx Ly Lz Lt; periodic boundaries.
 *   - site s = x + Lx*(y + Ly*(z + Lz*t)) (the lexicographic layout of
 *     section 2.1); direction mu = 0..3 is x, y, z, t.
 *   - links: device array of complex128 (re, im interleaved doubles) in
 *     structure-of-arrays order U[((mu*3 + i)*3 + j)*V + s], i.e. a
 *     contiguous (4, 3, 3, Lt, Lz, Ly, Lx) complex128 tensor (section 2.2:
 *     one array per matrix element). U_mu(x) joins x to x + mu.
 *   - matrix fields (Delta, g): complex128 M[(i*3 + j)*V + s].
 *   - Lie-algebra fields: float64 omega[a*V + s], a = 0..7, Gell-Mann basis
 *     with Tr(lambda_a lambda_b) = 2 delta_ab.
 *   - streams are hipStream_t passed as void*; NULL is the null stream.
 *
 * Ownership: the caller allocates every device buffer (links, workspace,
 * gradients) and keeps it alive for the lifetime of the context; the
 * library never allocates device memory. A context holds host-side state
 * only (plan, captured graphs, a pinned mirror of the device control block)
 * and is bound to the stream given at init. A context is not thread-safe.
 *
 * Errors: every call returns a gf_status. GF_ERR_ARG: a NULL or
 * out-of-range argument; GF_ERR_SHAPE: unsupported dims or a workspace
 * smaller than gf_workspace_bytes(); GF_ERR_HIP: a HIP runtime call failed
 * (gf_last_error() gives the message); GF_ERR_NONFINITE: theta or F became
 * NaN or Inf; GF_ERR_MAXITER: the iteration cap was reached before
 * theta <= eps; GF_ERR_STATE: the call does not apply to this context
 * (for example a single-configuration call on a batch context).
 * Scalar outputs are written whenever the status is GF_OK,
 * GF_ERR_MAXITER or GF_ERR_NONFINITE; output pointers may be NULL.
 */
#ifndef GF_H_
#define GF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx_s *gf_ctx;

typedef enum {
    GF_OK = 0,
    GF_ERR_ARG = 1,
    GF_ERR_SHAPE = 2,
    GF_ERR_HIP = 3,
    GF_ERR_NONFINITE = 4,
    GF_ERR_MAXITER = 5,
    GF_ERR_STATE = 6
} gf_status;

typedef struct {
    int32_t dims[4];      /* Lx, Ly, Lz, Lt                                          */
    double alpha;         /* step parameter of Eq. 2; the paper uses 0.08 (section 1) */
    int32_t fft_prec;     /* 0: FFT, momentum scaling and inverse FFT in FP64;
                             1: the same three steps in FP32 (complex64); the
                             divergence, g, reunitarisation, link update and the
                             theta/F sums stay FP64 in both                         */
    int32_t reunit_every; /* 0: Alg. 1 as printed; R > 0: also project every link
                             to SU(3) after every R-th update (drift control)       */
    int32_t chunk;        /* iterations per captured graph launch; 0 = default (8)  */
    int32_t fft_schedule; /* passes of the 4D transform: 0 = autotuned at init
                             (timed candidates, cached per shape); 1 = four 1D
                             passes each way; 2 = (x,y) 2D pass, z and t 1D
                             passes; 3 = (x,y) and (z,t) 2D passes. The inverse
                             (x,y) 2D pass of schedules 2 and 3 also forms g
                             (in the iteration with FP64 link storage it
                             writes the filtered fields, from which the link
                             update forms g). Lines of 16, 24, 32, 48 and 64
                             points, and (z,t) planes of 16x16, 24x24, 32x32,
                             16x32 and 48x48, run with their radix stages in
                             registers.
                             Schedules 2 and 3 need Lx*Ly <= 4096 (and
                             Lz*Lt <= 4096 for 3); GF_ERR_SHAPE otherwise.   */
    int32_t link_prec;    /* 0: links and g stored in FP64. 1: stored in
                             single precision in the 12-real form of section 2.2
                             (two rows in binary32, the third rebuilt; the
                             arithmetic stays FP64): gf_step iterates in this
                             storage; gf_fix_until iterates in it until theta <=
                             refine_theta, then in FP64 storage down to its
                             theta_eps. Storage rounding is not a gauge
                             transformation: the links leave their gauge orbit by
                             ~1e-7 (a shifted plaquette).                        */
    int32_t reserved;     /* must be 0                                             */
    double refine_theta;  /* link_prec 1: theta at which gf_fix_until switches to
                             FP64 storage; 0 = default 1e-10                       */
} gf_params;

/* Bytes of device workspace a context with these parameters needs. Returns 0
 * for invalid parameters. */
size_t gf_workspace_bytes(const gf_params *params);

/*
 * Create a context for one configuration and measure it: computes Delta,
 * F and theta of the given links (the first line of Alg. 1).
 * d_links: device links (layout above), updated in place by later calls;
 * between calls they hold the current links. An iterating call starts from
 * the last measurement: after changing the links outside the library, call
 * gf_functional, which measures them again.
 * d_ws: device workspace of at least gf_workspace_bytes(params) bytes,
 * 256-byte aligned. stream: the hipStream_t all work is ordered on.
 */
gf_status gf_init(gf_ctx *ctx, const gf_params *params, void *d_links, void *d_ws, size_t ws_bytes,
                  void *stream);

/* F (Eq. 1 at g = 1) and theta (Eq. 4) of the current links, measured
 * anew (Delta recomputed too); synchronises. */
gf_status gf_functional(gf_ctx ctx, double *F, double *theta);

/*
 * Run exactly n iterations of Alg. 1 (transform each element of Delta, apply
 * (alpha/2) p2max/p2 with the zero mode removed, transform back and
 * normalise, form g = 1 + Delta~ and project to SU(3), update every link
 * U_mu(x) -> g(x) U_mu(x) g^dag(x + mu), recompute Delta, F, theta),
 * ignoring the stopping rule. F and theta are the values after the last
 * update. Synchronises.
 */
gf_status gf_step(gf_ctx ctx, int32_t n, double *F, double *theta);

/*
 * Alg. 1 with its stopping rule: iterate while theta > theta_eps, at most
 * max_iter iterations in this call. *iters receives the number of updates
 * made in this call (0 if the links already satisfy theta <= theta_eps).
 * Returns GF_ERR_MAXITER if the cap was reached first. Synchronises.
 */
gf_status gf_fix_until(gf_ctx ctx, double theta_eps, int64_t max_iter, int64_t *iters, double *F,
                       double *theta);

/*
 * The quantities Alg. 1 monitors (F of Eq. 1 at g = 1 and theta of Eq. 4)
 * after every update since gf_init: entry 0 is the initial measurement,
 * entry k the values after update k (a library addition: the paper only
 * tests theta against eps). Copies min(cap, available) entries; *n receives
 * the number available. GF_ERR_STATE on a batch context (gf_history_batch).
 */
gf_status gf_history(gf_ctx ctx, int64_t cap, double *F_hist, double *theta_hist, int64_t *n);

/* Stage entry points: each is one step of Alg. 1 on the current links, for
 * step-by-step checks. They do not advance the iteration count. */

/* Delta(x) of Eq. 5 as a full matrix field d_delta[(i*3+j)*V + s] (complex128). */
gf_status gf_delta(gf_ctx ctx, void *d_delta);

/* The gauge vector of one iteration (Eq. 2 to first order, then projection
 * to SU(3)) for the current links, written to d_g[(i*3+j)*V + s]. */
gf_status gf_gauge(gf_ctx ctx, void *d_g);

/* The link update of Alg. 1, U_mu(x) -> g(x) U_mu(x) g^dag(x + mu), with a
 * caller-given gauge field d_g (same layout), then F and theta are
 * re-measured. */
gf_status gf_apply_gauge(gf_ctx ctx, const void *d_g);

/*
 * The context's 4D transform (the FFT steps of Alg. 1, done as 2D + 2D or 1D
 * passes as in section 2.2) applied in place to nfields complex fields
 * d_fields[f*V + s] (complex128 if fft_prec = 0, complex64 if 1); sign -1
 * forward exp(-i p.x), +1 backward exp(+i p.x); unnormalised.
 */
gf_status gf_fft(gf_ctx ctx, void *d_fields, int32_t nfields, int32_t sign);

/*
 * Input generator: thermalised configurations of the Wilson action
 * S = beta sum_P (1 - Re Tr U_P / 3), the workload the paper gauge-fixes
 * (section 3: beta = 5.8, 6.0, 6.2). Updates the context's links in place
 * with n_sweeps sweeps, each one heatbath sweep (Cabibbo-Marinari over the
 * SU(2) subgroups (0,1), (0,2), (1,2), Kennedy-Pendleton draws) followed by
 * n_or overrelaxation sweeps; a sweep visits mu = 0..3 and for each the even
 * then the odd sites. Random numbers: Philox4x32-10 with key (seed low
 * 32 bits, seed high 32 bits) and, for draw j of subgroup k of U_mu(site) in
 * heatbath sweep n = sweep0 + i, counter (site, mu + 4k + 16j, n low, n high)
 * (j = 255 for the direction of the SU(2) element, at most 64 attempts).
 * Every link is projected to SU(3) after its update. Afterwards Delta, F and
 * theta are measured as by gf_init. Every extent must be even (GF_ERR_SHAPE);
 * not for batch contexts (GF_ERR_STATE). Synchronises.
 */
gf_status gf_heatbath(gf_ctx ctx, double beta, int32_t n_sweeps, int32_t n_or, uint64_t seed, int64_t sweep0);

/* Average plaquette (1/(18 V)) sum_x sum_{mu<nu} Re Tr U_mu(x) U_nu(x+mu)
 * U_mu^dag(x+nu) U_nu^dag(x) of the context's links: the gauge-invariant
 * observable of the Wilson action of section 3 (unchanged by Alg. 1, so also
 * a check of the link update). Synchronises. */
gf_status gf_plaquette(gf_ctx ctx, double *P);

/*
 * Batches (a library addition; each configuration is fixed by Alg. 1 with
 * its own stopping rule theta <= eps, section 1): n_cfg independent
 * configurations of possibly different dims in one context. Every kernel
 * launch covers the tiles of every configuration still iterating; each
 * configuration has its own device-side stopping test. params and d_links
 * are arrays of n_cfg entries (n_cfg <= 64); all params must share fft_prec,
 * chunk, fft_schedule, link_prec and refine_theta (else
 * gf_workspace_bytes_batch returns 0 and gf_init_batch GF_ERR_SHAPE). The
 * workspace layout is as for single contexts, one region per configuration.
 */
size_t gf_workspace_bytes_batch(int32_t n_cfg, const gf_params *params);
gf_status gf_init_batch(gf_ctx *ctx, int32_t n_cfg, const gf_params *params, void *const *d_links,
                        void *d_ws, size_t ws_bytes, void *stream);
/* iters, F, theta: host arrays of n_cfg entries. GF_ERR_MAXITER if any
 * configuration hit the cap. */
gf_status gf_fix_until_batch(gf_ctx ctx, double theta_eps, int64_t max_iter, int64_t *iters, double *F,
                             double *theta);
/* F and theta of every configuration of a batch context (host arrays). */
gf_status gf_functional_batch(gf_ctx ctx, double *F, double *theta);
/* gf_history for configuration k (0 <= k < n_cfg) of a batch context (also
 * k = 0 of a single-configuration one): the (F, theta) that Alg. 1 monitors
 * after each of that configuration's updates. GF_ERR_ARG for k out of range. */
gf_status gf_history_batch(gf_ctx ctx, int32_t k, int64_t cap, double *F_hist, double *theta_hist, int64_t *n);

/*
 * A context for the differentiable functional only (the two calls below):
 * its workspace holds g [3][3][V] and the per-block partial sums
 * (gf_workspace_bytes_functional bytes, about 144 B per site, instead of the
 * iteration's buffers); init neither measures the links nor plans or tunes
 * the transform. The iteration and stage calls return GF_ERR_STATE on it.
 * Arguments as for gf_init; the links are read (never written) by the
 * functional calls, at whatever they hold when a call is made.
 */
size_t gf_workspace_bytes_functional(const gf_params *params);
gf_status gf_init_functional(gf_ctx *ctx, const gf_params *params, void *d_links, void *d_ws, size_t ws_bytes,
                             void *stream);

/*
 * Differentiable functional (Eq. 1 as a function of gauge parameters):
 *   F = 1/(12 V) sum_x sum_mu Re Tr[g(x) U_mu(x) g^dag(x+mu)],
 *   g(x) = exp(i sum_a lambda_a omega_a(x)),
 * for the context's current links. d_omega: device float64 [8][V].
 */
gf_status gf_functional_g(gf_ctx ctx, const double *d_omega, double *F);

/*
 * Backward of gf_functional_g for an upstream gradient grad_out:
 *   d_dF_domega[a*V + s] = grad_out * dF/domega_a(x)            (float64 [8][V])
 *   d_dF_dU   (link layout) = grad_out * (dF/dRe U + i dF/dIm U)
 *                           = grad_out * g^dag(x) g(x+mu) / (12 V)
 * Either output pointer may be NULL to skip it.
 */
gf_status gf_functional_g_backward(gf_ctx ctx, const double *d_omega, double grad_out, double *d_dF_domega,
                                   void *d_dF_dU);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): gf_init +
 * gf_fix_until + gf_destroy in one call that allocates nothing. Its
 * workspace is a static device array of GF_STATIC_SCRATCH_BYTES inside the
 * library, one per GPU, held until the process ends; the call creates no
 * stream, event or graph and no pinned host memory, launches every kernel on
 * `stream` and reads the stopping flag back with plain copies. Lattices
 * whose gf_workspace_bytes(params) exceeds GF_STATIC_SCRATCH_BYTES are
 * rejected with GF_ERR_SHAPE (64 MiB holds up to about 58 000 sites with the
 * FP64 transform: 8^4, 12^4, 16^3 x 12). params->fft_schedule 0 takes the
 * 2D passes wherever they fit (no autotuning: that needs timing events).
 * d_links, theta_eps, max_iter and the outputs are as for gf_init and
 * gf_fix_until. Every call on one GPU uses that GPU's array and leaves its
 * contents behind (each call initialises what it reads): calls that overlap
 * on one GPU, from any thread or stream, race and must be serialised by the
 * caller. Synchronises.
 */
#define GF_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
gf_status gf_fix_until_static(const gf_params *params, void *d_links, double theta_eps, int64_t max_iter,
                              int64_t *iters, double *F, double *theta, void *stream);

/* Release the context (host state and graphs only). */
gf_status gf_destroy(gf_ctx ctx);

const char *gf_strerror(gf_status status);
/* Detail of the last error on this context (empty string if none). */
const char *gf_last_error(gf_ctx ctx);

/*
 * Per-kernel timing (a library addition, for measurement). With timing on,
 * iterations are launched one kernel at a time (no graph) and every launch
 * is bracketed by hipEvents on the context's stream; the accumulated time
 * per kernel is readable below.
 */
gf_status gf_set_timing(gf_ctx ctx, int32_t on);
int32_t gf_kernel_count(gf_ctx ctx);
const char *gf_kernel_name(gf_ctx ctx, int32_t k);
/* Accumulated milliseconds and launches of kernel k since the last reset. */
gf_status gf_kernel_time(gf_ctx ctx, int32_t k, double *total_ms, int64_t *launches);
gf_status gf_reset_timing(gf_ctx ctx);

/* The transform schedule in use (1, 2 or 3; see gf_params.fft_schedule;
 * the 2D + 2D grouping of section 2.2 is schedule 3). */
int32_t gf_fft_schedule(gf_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* GF_H_ */

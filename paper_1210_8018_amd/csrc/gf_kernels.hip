// gfx950 kernels of one Fourier-accelerated steepest-descent iteration
// (Alg. 1 of Cardoso, Silva, Oliveira, Bicudo, Lattice 2012) and of the
// differentiable functional. Every launch covers a table of configurations
// (a batch of one for a single lattice); blocks of a configuration whose
// control block says "done" return at once.
#include <hip/hip_runtime.h>

#include "gf_device.h"
#include "gf_internal.h"

namespace gfk {

// ============================================================ control
// Arm a fix/step call: set eps and the iteration cap, evaluate the stopping
// rule on the latest theta. reset != 0 also clears the control block.
__global__ void k_arm(const Cfg *__restrict__ cfgs, int ncfg, double eps, long long add_iters, int reset)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncfg) return;
    Ctrl *ct = cfgs[c].ctrl;
    if (reset) {
        ct->iter = 0;
        ct->F = 0.0;
        ct->theta = 0.0;
        ct->done = kRunning;
    }
    ct->eps = eps;
    ct->max_iter = ct->iter + add_iters;
    int d = kRunning;
    if (!reset) {
        if (!isfinite(ct->F) || !isfinite(ct->theta))
            d = kNonFinite;
        else if (!(ct->theta > eps))
            d = kConverged;
        else if (ct->iter >= ct->max_iter)
            d = kMaxIter;
    }
    ct->done = d;
}

// ============================================================ S1: Eq. 5 stencil + sums
// D = sum_nu [U_nu(x - nu) - U_nu(x)]; Delta = (D - D^dag) - Tr(D - D^dag)/3.
// Writes the four packed transform fields (Delta_01, Delta_02, Delta_12,
// Im Delta_00 + i Im Delta_11), which carry all 8 real degrees of freedom of
// the traceless anti-hermitian Delta, and per-block compensated partial sums
// of sum_mu Re Tr U_mu(x) (Eq. 1 at g = 1) and |Delta|^2 (Eq. 4).
template <typename T2>
__global__ __launch_bounds__(kSiteBlock) void k_delta(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                      int respect_done, double2 *__restrict__ full)
{
    __shared__ dd red[2 * (kSiteBlock / 64)];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[c];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V;
    const int lb = blk - B->off_site[c];
    const int s = lb * kSiteBlock + threadIdx.x;
    double fsum = 0.0, tsum = 0.0;
    if (s < V) {
        int x[4];
        site_coords(C.dims, s, x);
        double2 D[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) D[k] = cz();
        int stride = 1;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int Lm = C.dims[mu];
            const int sb = (x[mu] == 0) ? s + (Lm - 1) * stride : s - stride;
            const double2 *__restrict__ Um = C.U + (size_t)mu * 9 * V;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double2 here = Um[(size_t)k * V + s];
                const double2 back = Um[(size_t)k * V + sb];
                D[k] = cadd(D[k], csub(back, here));
                if (k == 0 || k == 4 || k == 8) fsum += here.x;
            }
            stride *= Lm;
        }
        // A = D - D^dag (anti-hermitian); remove the trace (pure imaginary)
        double2 A[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i * 3 + j] = csub(D[i * 3 + j], cconj(D[j * 3 + i]));
        const double tr3 = (A[0].y + A[4].y + A[8].y) * (1.0 / 3.0);
        A[0] = make_double2(0.0, A[0].y - tr3);
        A[4] = make_double2(0.0, A[4].y - tr3);
        A[8] = make_double2(0.0, A[8].y - tr3);
#pragma unroll
        for (int k = 0; k < 9; ++k) tsum += cnorm2(A[k]);
        T2 *__restrict__ f = (T2 *)C.fields;
        f[s].x = A[1].x;
        f[s].y = A[1].y;
        f[(size_t)V + s].x = A[2].x;
        f[(size_t)V + s].y = A[2].y;
        f[(size_t)2 * V + s].x = A[5].x;
        f[(size_t)2 * V + s].y = A[5].y;
        f[(size_t)3 * V + s].x = A[0].y;
        f[(size_t)3 * V + s].y = A[4].y;
        if (full) {
#pragma unroll
            for (int k = 0; k < 9; ++k) full[(size_t)k * V + s] = A[k];
        }
    }
    dd a = {fsum, 0.0}, b = {tsum, 0.0};
    block_sum2(a, b, red);
    if (threadIdx.x == 0) {
        double *p = C.partials + (size_t)lb * 4;
        p[0] = a.hi;
        p[1] = a.lo;
        p[2] = b.hi;
        p[3] = b.lo;
    }
}

// ============================================================ reductions + stopping rule
// One block per configuration: sum the block partials in a fixed order,
// F = sum/(12 V) (Eq. 1), theta = sum/(3 V) (Eq. 4); with count_iter, count
// the update, record the history and evaluate the stopping rule theta <= eps.
__global__ __launch_bounds__(256) void k_reduce(const Cfg *__restrict__ cfgs, int count_iter, int respect_done)
{
    __shared__ dd red[2 * (256 / 64)];
    const Cfg &C = cfgs[blockIdx.x];
    Ctrl *ct = C.ctrl;
    if (respect_done && ct->done) return;
    dd f = {0.0, 0.0}, t = {0.0, 0.0};
    for (int i = threadIdx.x; i < C.nblk_site; i += blockDim.x) {
        const double *p = C.partials + (size_t)i * 4;
        f = dd_add(f, dd{p[0], p[1]});
        t = dd_add(t, dd{p[2], p[3]});
    }
    block_sum2(f, t, red);
    if (threadIdx.x == 0) {
        const double F = (f.hi + f.lo) / (12.0 * (double)C.V);
        const double th = (t.hi + t.lo) / (3.0 * (double)C.V);
        ct->F = F;
        ct->theta = th;
        long long it = ct->iter;
        if (count_iter) {
            it += 1;
            ct->iter = it;
        }
        ct->hist[it % kHist][0] = F;
        ct->hist[it % kHist][1] = th;
        if (count_iter) {
            int d = kRunning;
            if (!isfinite(F) || !isfinite(th))
                d = kNonFinite;
            else if (!(th > ct->eps))
                d = kConverged;
            else if (it >= ct->max_iter)
                d = kMaxIter;
            ct->done = d;
        }
    }
}

// ============================================================ transform tiles
template <typename T2>
struct Cx;
template <>
struct Cx<double2> {
    using T = double;
    __device__ static double2 mk(double a, double b) { return make_double2(a, b); }
};
template <>
struct Cx<float2> {
    using T = float;
    __device__ static float2 mk(float a, float b) { return make_float2(a, b); }
};

template <typename T2>
__device__ __forceinline__ T2 t_add(T2 a, T2 b)
{
    T2 r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename T2>
__device__ __forceinline__ T2 t_sub(T2 a, T2 b)
{
    T2 r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename T2>
__device__ __forceinline__ T2 t_mul(T2 a, T2 b)
{
    T2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// multiply by sign * i
template <typename T2>
__device__ __forceinline__ T2 t_mul_si(T2 a, int sign)
{
    T2 r;
    if (sign < 0) {
        r.x = a.y;
        r.y = -a.x;
    } else {
        r.x = -a.y;
        r.y = a.x;
    }
    return r;
}

// r-point DFTs, b_q = sum_m a_m exp(sign 2 pi i m q / r), in place.
template <typename T2>
__device__ __forceinline__ void dft2(T2 *a)
{
    T2 t = a[0];
    a[0] = t_add(t, a[1]);
    a[1] = t_sub(t, a[1]);
}

template <typename T2>
__device__ __forceinline__ void dft3(T2 *a, int sign)
{
    using T = typename Cx<T2>::T;
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    T2 s = t_add(a[1], a[2]);
    T2 d = t_sub(a[1], a[2]);
    T2 b0 = t_add(a[0], s);
    T2 m;
    m.x = a[0].x - (T)0.5 * s.x;
    m.y = a[0].y - (T)0.5 * s.y;
    // exp(sign 2 pi i/3) = -1/2 + sign i h: b1 = m + sign i h d, b2 = m - sign i h d
    T2 r = t_mul_si(d, sign);
    r.x *= h;
    r.y *= h;
    a[0] = b0;
    a[1] = t_add(m, r);
    a[2] = t_sub(m, r);
}

template <typename T2>
__device__ __forceinline__ void dft4(T2 *a, int sign)
{
    T2 s02 = t_add(a[0], a[2]), d02 = t_sub(a[0], a[2]);
    T2 s13 = t_add(a[1], a[3]), d13 = t_mul_si(t_sub(a[1], a[3]), sign);
    a[0] = t_add(s02, s13);
    a[2] = t_sub(s02, s13);
    a[1] = t_add(d02, d13);
    a[3] = t_sub(d02, d13);
}

template <typename T2>
__device__ __forceinline__ void dft8(T2 *a, int sign)
{
    using T = typename Cx<T2>::T;
    const T r2 = (T)0.70710678118654752440;
    T2 e[4] = {a[0], a[2], a[4], a[6]};
    T2 o[4] = {a[1], a[3], a[5], a[7]};
    dft4(e, sign);
    dft4(o, sign);
    // w^q, w = exp(sign 2 pi i / 8): w^1 = (1 + sign i) r2, w^2 = sign i, w^3 = (-1 + sign i) r2
    T2 t1, t2, t3;
    {
        T2 si = t_mul_si(o[1], sign);
        t1.x = (o[1].x + si.x) * r2;
        t1.y = (o[1].y + si.y) * r2;
    }
    t2 = t_mul_si(o[2], sign);
    {
        T2 si = t_mul_si(o[3], sign);
        t3.x = (si.x - o[3].x) * r2;
        t3.y = (si.y - o[3].y) * r2;
    }
    a[0] = t_add(e[0], o[0]);
    a[4] = t_sub(e[0], o[0]);
    a[1] = t_add(e[1], t1);
    a[5] = t_sub(e[1], t1);
    a[2] = t_add(e[2], t2);
    a[6] = t_sub(e[2], t2);
    a[3] = t_add(e[3], t3);
    a[7] = t_sub(e[3], t3);
}

// One Stockham radix-R stage over P pencils of length L held in LDS.
// Element l of pencil k sits at k*ks + l*ls. Output is in natural order.
template <int R, typename T2>
__device__ __forceinline__ void stage(const T2 *__restrict__ src, T2 *__restrict__ dst, const T2 *__restrict__ tw,
                                      int L, int P, int Ns, int ks, int ls, int sign, bool k_fast)
{
    const int nb = L / R;
    const int total = P * nb;
    const int tstep = L / (Ns * R);
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        int k, j;
        if (k_fast) {
            k = b % P;
            j = b / P;
        } else {
            j = b % nb;
            k = b / nb;
        }
        const int kk = j % Ns;
        T2 a[R];
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = src[k * ks + (j + m * nb) * ls];
#pragma unroll
        for (int m = 1; m < R; ++m) {
            T2 w = tw[m * kk * tstep];
            if (sign > 0) w.y = -w.y;
            a[m] = t_mul(a[m], w);
        }
        if constexpr (R == 2)
            dft2(a);
        else if constexpr (R == 3)
            dft3(a, sign);
        else if constexpr (R == 4)
            dft4(a, sign);
        else
            dft8(a, sign);
        const int ob = (j - kk) * R + kk;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[k * ks + (ob + q * Ns) * ls] = a[q];
    }
}

// All stages of one axis; on return *src holds the transformed pencils.
template <typename T2>
__device__ void fft_pencils(T2 *&src, T2 *&dst, const T2 *tw, const FftAxis &A, int ks, int ls, int sign,
                            bool k_fast)
{
    int Ns = 1;
    for (int st = 0; st < A.nstage; ++st) {
        const int r = A.radix[st];
        switch (r) {
        case 2: stage<2>(src, dst, tw, A.L, A.P, Ns, ks, ls, sign, k_fast); break;
        case 3: stage<3>(src, dst, tw, A.L, A.P, Ns, ks, ls, sign, k_fast); break;
        case 4: stage<4>(src, dst, tw, A.L, A.P, Ns, ks, ls, sign, k_fast); break;
        default: stage<8>(src, dst, tw, A.L, A.P, Ns, ks, ls, sign, k_fast); break;
        }
        __syncthreads();
        T2 *t = src;
        src = dst;
        dst = t;
        Ns *= r;
    }
}

// One axis of the 4D transform for one tile of one field. mode 0: a plain
// pass with the given sign. mode 1 (last axis only): forward transform,
// multiplication by K(p) = (alpha/2)(p2max/p2)/V with K(0) = 0 (Eq. 2; the
// 1/V is the normalisation of the backward transform), backward transform.
template <typename T2>
__global__ __launch_bounds__(kFftThreads) void k_fft(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                     int axis, int sign, int mode, void *fields_override,
                                                     int respect_done, int lds_elems)
{
    using T = typename Cx<T2>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int field = blockIdx.y;
    const int c = find_cfg(B->off_fft[axis], B->n, tile);
    const Cfg &C = cfgs[c];
    if (respect_done && C.ctrl->done) return;
    const FftAxis &A = C.ax[axis];
    const int t = tile - B->off_fft[axis][c];
    const int L = A.L, P = A.P, n = P * L;
    T2 *buf0 = (T2 *)smem;
    T2 *buf1 = buf0 + lds_elems;
    T2 *tw = buf1 + lds_elems;
    const T2 *__restrict__ gtw = (const T2 *)C.tw + C.tw_off[axis];
    for (int e = threadIdx.x; e < L; e += blockDim.x) tw[e] = gtw[e];

    T2 *__restrict__ g = (T2 *)(fields_override ? fields_override : C.fields) + (size_t)field * C.V;
    const bool k_fast = axis != 0;
    const int ks = k_fast ? 1 : L, ls = k_fast ? P : 1;
    size_t gbase;
    if (!k_fast) {
        gbase = (size_t)t * n;
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) buf0[idx] = g[gbase + idx];
    } else {
        const int o = t / A.inner_chunks, ic = t % A.inner_chunks;
        gbase = (size_t)o * A.S * L + (size_t)ic * P;
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int k = idx % P, l = idx / P;
            buf0[idx] = g[gbase + k + (size_t)l * A.S];
        }
    }
    __syncthreads();
    T2 *src = buf0, *dst = buf1;
    fft_pencils(src, dst, tw, A, ks, ls, mode == 1 ? -1 : sign, k_fast);
    if (mode == 1) {
        // pencil k is inner site ic*P + k: momenta (nx, ny, nz); l is nt
        const int ic = t % A.inner_chunks;
        const double *s2 = C.sin2;
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int k = idx % P, l = idx / P;
            const int in = ic * P + k;
            const int nx = in % C.dims[0];
            const int r1 = in / C.dims[0];
            const int ny = r1 % C.dims[1];
            const int nz = r1 / C.dims[1];
            const double p2 = s2[C.sin2_off[0] + nx] + s2[C.sin2_off[1] + ny] + s2[C.sin2_off[2] + nz] +
                              s2[C.sin2_off[3] + l];
            const double K = (p2 > 0.0) ? C.kfac / p2 : 0.0;
            const T k_t = (T)K;
            T2 v = src[idx];
            v.x *= k_t;
            v.y *= k_t;
            src[idx] = v;
        }
        __syncthreads();
        fft_pencils(src, dst, tw, A, ks, ls, +1, k_fast);
    }
    if (!k_fast) {
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) g[gbase + idx] = src[idx];
    } else {
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int k = idx % P, l = idx / P;
            g[gbase + k + (size_t)l * A.S] = src[idx];
        }
    }
}

// ============================================================ S4: g = 1 + Delta~, projected
// Rebuilds the filtered traceless anti-hermitian matrix from the four packed
// fields (Delta~_10 = -conj(Delta~_01), Delta~_00 = i Re f3, Delta~_11 = i Im f3,
// Delta~_22 = -Delta~_00 - Delta~_11) in FP64, forms g = 1 + Delta~ (first
// order in alpha) and projects it to SU(3).
template <typename T2>
__global__ __launch_bounds__(kSiteBlock) void k_gauge(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                      int respect_done, double2 *__restrict__ g_override)
{
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[c];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V;
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= V) return;
    const T2 *__restrict__ f = (const T2 *)C.fields;
    const T2 a = f[s], b = f[(size_t)V + s], d = f[(size_t)2 * V + s], e = f[(size_t)3 * V + s];
    const double2 f01 = make_double2((double)a.x, (double)a.y);
    const double2 f02 = make_double2((double)b.x, (double)b.y);
    const double2 f12 = make_double2((double)d.x, (double)d.y);
    const double i00 = (double)e.x, i11 = (double)e.y;
    M3 m;
    m.e[0] = make_double2(1.0, i00);
    m.e[1] = f01;
    m.e[2] = f02;
    m.e[3] = make_double2(-f01.x, f01.y);
    m.e[4] = make_double2(1.0, i11);
    m.e[5] = f12;
    m.e[6] = make_double2(-f02.x, f02.y);
    m.e[7] = make_double2(-f12.x, f12.y);
    m.e[8] = make_double2(1.0, -i00 - i11);
    m3_reunit(m);
    m3_store(g_override ? g_override : C.g, V, s, m);
}

// ============================================================ S5: link update
// U_mu(x) -> g(x) U_mu(x) g^dag(x + mu) for the four links of each site; all
// g were formed before this launch (the two separate loops of Alg. 1).
__global__ __launch_bounds__(kSiteBlock) void k_update(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                       int respect_done, const double2 *__restrict__ g_override,
                                                       int allow_reunit)
{
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[c];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V;
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= V) return;
    const double2 *__restrict__ G = g_override ? g_override : C.g;
    const bool reunit =
        allow_reunit && C.reunit_every > 0 && ((C.ctrl->iter + 1) % (long long)C.reunit_every) == 0;
    int x[4];
    site_coords(C.dims, s, x);
    const M3 gx = m3_load(G, V, s);
    int stride = 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int Lm = C.dims[mu];
        const int sf = (x[mu] == Lm - 1) ? s - (Lm - 1) * stride : s + stride;
        stride *= Lm;
        double2 *__restrict__ Um = C.U + (size_t)mu * 9 * V;
        const M3 u = m3_load(Um, V, s);
        const M3 gf = m3_load(G, V, sf);
        M3 w = m3_mul_dag(m3_mul(gx, u), gf);
        if (reunit) m3_reunit(w);
        m3_store(Um, V, s, w);
    }
}

// ============================================================ differentiable functional
// exp(X) and its Frechet derivative L(X, E) for X = i Q, Q = sum_a w_a lambda_a,
// by a truncated Taylor series of exp(X / 2^j) coupled with its derivative
// (d/dt (Y + tE)^k = D_{k-1} Y + Y^{k-1} E), followed by j squarings
// exp(2Z) = exp(Z)^2, L(2Z, 2F) = L(Z, F) exp(Z) + exp(Z) L(Z, F)
// (Al-Mohy and Higham, SIAM J. Matrix Anal. Appl. 30, 2009).
__device__ __forceinline__ M3 algebra_i(const double w[8])
{
    // X = i sum_a w_a lambda_a, lambda_a Gell-Mann
    const double r3 = 0.57735026918962576451;
    M3 Q = m3_zero();
    Q.e[1] = make_double2(w[0], -w[1]);
    Q.e[3] = make_double2(w[0], w[1]);
    Q.e[0].x = w[2] + w[7] * r3;
    Q.e[4].x = -w[2] + w[7] * r3;
    Q.e[8].x = -2.0 * w[7] * r3;
    Q.e[2] = make_double2(w[3], -w[4]);
    Q.e[6] = make_double2(w[3], w[4]);
    Q.e[5] = make_double2(w[5], -w[6]);
    Q.e[7] = make_double2(w[5], w[6]);
    M3 X;
#pragma unroll
    for (int k = 0; k < 9; ++k) X.e[k] = make_double2(-Q.e[k].y, Q.e[k].x);
    return X;
}

__device__ __forceinline__ int scaling_power(const M3 &X)
{
    double n = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) n += cnorm2(X.e[k]);
    n = sqrt(n);
    int j = 0;
    while (n > 0.5 && j < 60) {
        n *= 0.5;
        ++j;
    }
    return j;
}

constexpr int kTaylor = 18;

__device__ M3 expm_taylor(const M3 &X)
{
    const int j = scaling_power(X);
    const M3 Y = m3_scale(X, ldexp(1.0, -j));
    M3 term = m3_identity(), acc = m3_identity();
    for (int k = 1; k <= kTaylor; ++k) {
        term = m3_scale(m3_mul(term, Y), 1.0 / (double)k);
        acc = m3_add(acc, term);
    }
    for (int i = 0; i < j; ++i) acc = m3_mul(acc, acc);
    return acc;
}

__device__ void expm_frechet_taylor(const M3 &X, const M3 &E, M3 &ex, M3 &Lx)
{
    const int j = scaling_power(X);
    const double sc = ldexp(1.0, -j);
    const M3 Y = m3_scale(X, sc);
    const M3 F = m3_scale(E, sc);
    M3 term = m3_identity(), dterm = m3_zero();
    M3 acc = m3_identity(), dacc = m3_zero();
    for (int k = 1; k <= kTaylor; ++k) {
        const double ik = 1.0 / (double)k;
        const M3 nd = m3_scale(m3_add(m3_mul(dterm, Y), m3_mul(term, F)), ik);
        term = m3_scale(m3_mul(term, Y), ik);
        dterm = nd;
        acc = m3_add(acc, term);
        dacc = m3_add(dacc, dterm);
    }
    for (int i = 0; i < j; ++i) {
        dacc = m3_add(m3_mul(dacc, acc), m3_mul(acc, dacc));
        acc = m3_mul(acc, acc);
    }
    ex = acc;
    Lx = dacc;
}

__device__ __forceinline__ void load_omega(const double *__restrict__ om, int V, int s, double w[8])
{
#pragma unroll
    for (int a = 0; a < 8; ++a) w[a] = om[(size_t)a * V + s];
}

// g(x) = exp(i sum_a lambda_a omega_a(x)) into the configuration's g buffer.
__global__ __launch_bounds__(kSiteBlock) void k_expg(const Cfg *__restrict__ cfgs, const double *__restrict__ omega)
{
    const Cfg &C = cfgs[0];
    const int s = blockIdx.x * kSiteBlock + threadIdx.x;
    if (s >= C.V) return;
    double w[8];
    load_omega(omega, C.V, s, w);
    m3_store(C.g, C.V, s, expm_taylor(algebra_i(w)));
}

// Per-block partial sums of sum_mu Re Tr[g(x) U_mu(x) g^dag(x+mu)] (Eq. 1).
__global__ __launch_bounds__(kSiteBlock) void k_fg_partials(const Cfg *__restrict__ cfgs)
{
    __shared__ dd red[2 * (kSiteBlock / 64)];
    const Cfg &C = cfgs[0];
    const int V = C.V;
    const int s = blockIdx.x * kSiteBlock + threadIdx.x;
    double acc = 0.0;
    if (s < V) {
        int x[4];
        site_coords(C.dims, s, x);
        const M3 gx = m3_load(C.g, V, s);
        int stride = 1;
        for (int mu = 0; mu < 4; ++mu) {
            const int Lm = C.dims[mu];
            const int sf = (x[mu] == Lm - 1) ? s - (Lm - 1) * stride : s + stride;
            stride *= Lm;
            const M3 u = m3_load(C.U + (size_t)mu * 9 * V, V, s);
            const M3 gf = m3_load(C.g, V, sf);
            const M3 w = m3_mul_dag(m3_mul(gx, u), gf);
            acc += w.e[0].x + w.e[4].x + w.e[8].x;
        }
    }
    dd a = {acc, 0.0}, b = {0.0, 0.0};
    block_sum2(a, b, red);
    if (threadIdx.x == 0) {
        double *p = C.partials + (size_t)blockIdx.x * 4;
        p[0] = a.hi;
        p[1] = a.lo;
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

// Sum of the first partial pair of every block, times `scale`, to *out.
__global__ __launch_bounds__(256) void k_sum_partials(const Cfg *__restrict__ cfgs, double scale,
                                                      double *__restrict__ out)
{
    __shared__ dd red[2 * (256 / 64)];
    const Cfg &C = cfgs[0];
    dd f = {0.0, 0.0}, z = {0.0, 0.0};
    for (int i = threadIdx.x; i < C.nblk_site; i += blockDim.x) {
        const double *p = C.partials + (size_t)i * 4;
        f = dd_add(f, dd{p[0], p[1]});
    }
    block_sum2(f, z, red);
    if (threadIdx.x == 0) *out = (f.hi + f.lo) * scale;
}

// Gradients of Eq. 1 with g = exp(X), X = i omega.lambda:
//   dF/domega_a(x) = Re Tr[L(X, i lambda_a) Sigma(x)] / (12 V)
//                  = Re Tr[i lambda_a L(X, Sigma(x))] / (12 V),
//   Sigma(x) = sum_mu [U_mu(x) g^dag(x+mu) + U_mu^dag(x-mu) g^dag(x-mu)],
// using Tr[L(X,E) S] = Tr[E L(X,S)]; and
//   dF/dRe U_mu(x) + i dF/dIm U_mu(x) = g^dag(x) g(x+mu) / (12 V).
__global__ __launch_bounds__(kSiteBlock) void k_fg_backward(const Cfg *__restrict__ cfgs,
                                                            const double *__restrict__ omega, double scale,
                                                            double *__restrict__ d_omega, double2 *__restrict__ d_U)
{
    const Cfg &C = cfgs[0];
    const int V = C.V;
    const int s = blockIdx.x * kSiteBlock + threadIdx.x;
    if (s >= V) return;
    int x[4];
    site_coords(C.dims, s, x);
    const M3 gx = m3_load(C.g, V, s);
    M3 Sig = m3_zero();
    int stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int Lm = C.dims[mu];
        const int sf = (x[mu] == Lm - 1) ? s - (Lm - 1) * stride : s + stride;
        const int sb = (x[mu] == 0) ? s + (Lm - 1) * stride : s - stride;
        stride *= Lm;
        const double2 *Um = C.U + (size_t)mu * 9 * V;
        const M3 gf = m3_load(C.g, V, sf);
        if (d_omega) {
            const M3 u = m3_load(Um, V, s);
            const M3 ub = m3_load(Um, V, sb);
            const M3 gb = m3_load(C.g, V, sb);
            Sig = m3_add(Sig, m3_mul_dag(u, gf));
            // U^dag(x-mu) g^dag(x-mu) = (g(x-mu) U(x-mu))^dag
            const M3 t = m3_mul(gb, ub);
            M3 td;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) td.e[i * 3 + j] = cconj(t.e[j * 3 + i]);
            Sig = m3_add(Sig, td);
        }
        if (d_U) {
            const M3 dU = m3_scale(m3_dag_mul(gx, gf), scale);
            m3_store(d_U + (size_t)mu * 9 * V, V, s, dU);
        }
    }
    if (d_omega) {
        double w[8];
        load_omega(omega, V, s, w);
        M3 ex, G;
        expm_frechet_taylor(algebra_i(w), Sig, ex, G);
        // Tr[lambda_a G] for the eight Gell-Mann matrices; dF/domega_a = -Im(Tr)/(12V)
        const double r3 = 0.57735026918962576451;
        double2 tr[8];
        tr[0] = cadd(G.e[3], G.e[1]);
        {
            const double2 d = csub(G.e[1], G.e[3]);
            tr[1] = make_double2(-d.y, d.x);
        }
        tr[2] = csub(G.e[0], G.e[4]);
        tr[3] = cadd(G.e[6], G.e[2]);
        {
            const double2 d = csub(G.e[2], G.e[6]);
            tr[4] = make_double2(-d.y, d.x);
        }
        tr[5] = cadd(G.e[7], G.e[5]);
        {
            const double2 d = csub(G.e[5], G.e[7]);
            tr[6] = make_double2(-d.y, d.x);
        }
        tr[7] = cscale(csub(cadd(G.e[0], G.e[4]), cscale(G.e[8], 2.0)), r3);
#pragma unroll
        for (int a = 0; a < 8; ++a) d_omega[(size_t)a * V + s] = -tr[a].y * scale;
    }
}

// ============================================================ launchers
static inline dim3 blocks1(int n, int b) { return dim3((n + b - 1) / b); }

hipError_t launch_arm(const Launch &L, int ncfg, double eps, long long add_iters, int reset_iter)
{
    hipLaunchKernelGGL(k_arm, blocks1(ncfg, 64), dim3(64), 0, L.stream, L.cfgs, ncfg, eps, add_iters, reset_iter);
    return hipGetLastError();
}

hipError_t launch_delta(const Launch &L, int respect_done, double2 *full_delta)
{
    if (L.fp32)
        hipLaunchKernelGGL(k_delta<float2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, full_delta);
    else
        hipLaunchKernelGGL(k_delta<double2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, full_delta);
    return hipGetLastError();
}

hipError_t launch_reduce(const Launch &L, int ncfg, int count_iter, int respect_done)
{
    hipLaunchKernelGGL(k_reduce, dim3(ncfg), dim3(256), 0, L.stream, L.cfgs, count_iter, respect_done);
    return hipGetLastError();
}

hipError_t launch_fft_axis(const Launch &L, int axis, int sign, int mode, void *fields_override, int nfields,
                           int respect_done)
{
    const dim3 grid(L.total_fft_tiles[axis], nfields);
    if (L.fp32) {
        const size_t sh = (size_t)(2 * L.max_lds_elems + 256) * sizeof(float2);
        hipLaunchKernelGGL(k_fft<float2>, grid, dim3(kFftThreads), sh, L.stream, L.cfgs, L.batch, axis, sign, mode,
                           fields_override, respect_done, L.max_lds_elems);
    } else {
        const size_t sh = (size_t)(2 * L.max_lds_elems + 256) * sizeof(double2);
        hipLaunchKernelGGL(k_fft<double2>, grid, dim3(kFftThreads), sh, L.stream, L.cfgs, L.batch, axis, sign, mode,
                           fields_override, respect_done, L.max_lds_elems);
    }
    return hipGetLastError();
}

hipError_t launch_gauge(const Launch &L, int respect_done, double2 *g_override)
{
    if (L.fp32)
        hipLaunchKernelGGL(k_gauge<float2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, g_override);
    else
        hipLaunchKernelGGL(k_gauge<double2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, g_override);
    return hipGetLastError();
}

hipError_t launch_update(const Launch &L, int respect_done, const double2 *g_override)
{
    hipLaunchKernelGGL(k_update, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs, L.batch,
                       respect_done, g_override, g_override ? 0 : 1);
    return hipGetLastError();
}

}  // namespace gfk

// Differentiable functional launchers (single configuration, slot 0).
namespace gfk {

hipError_t launch_functional_g_impl(const Launch &L, int nblk, const double *omega, double scale, double *out)
{
    hipLaunchKernelGGL(k_expg, dim3(nblk), dim3(kSiteBlock), 0, L.stream, L.cfgs, omega);
    hipLaunchKernelGGL(k_fg_partials, dim3(nblk), dim3(kSiteBlock), 0, L.stream, L.cfgs);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, L.stream, L.cfgs, scale, out);
    return hipGetLastError();
}

hipError_t launch_functional_g_backward_impl(const Launch &L, int nblk, const double *omega, double scale,
                                             double *d_omega, double2 *d_U)
{
    hipLaunchKernelGGL(k_expg, dim3(nblk), dim3(kSiteBlock), 0, L.stream, L.cfgs, omega);
    hipLaunchKernelGGL(k_fg_backward, dim3(nblk), dim3(kSiteBlock), 0, L.stream, L.cfgs, omega, scale, d_omega,
                       d_U);
    return hipGetLastError();
}

}  // namespace gfk

// gfx950 kernels of one Fourier-accelerated steepest-descent iteration
// (Alg. 1 of Cardoso, Silva, Oliveira, Bicudo, Lattice 2012) and of the
// differentiable functional. Every launch covers a table of configurations
// (a batch of one for a single lattice); blocks of a configuration whose
// control block says "done" return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

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
        ct->cur = 0;
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
// A block owns a set of (x, y, z) sites (kSiteBlock consecutive ones, or a
// box; see march_xyz) and walks `tch` consecutive t-slices; U_t(x - t) of
// each slice is the U_t(x) loaded for the previous slice, kept in registers.
template <typename T2>
__global__ __launch_bounds__(kSiteBlock) void k_delta(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                      int respect_done, double2 *__restrict__ full)
{
    __shared__ dd red[2 * (kSiteBlock / 64)];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_march, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V, V3 = C.V3;
    const int lb = blk - B->off_march[c];
    const int b3 = lb % C.nb3, tc = lb / C.nb3;
    int x, y, z;
    const bool inside = march_xyz(C, b3, threadIdx.x, x, y, z);
    dd fs = {0.0, 0.0}, ts = {0.0, 0.0};
    if (inside) {
        const int Lx = C.dims[0], Ly = C.dims[1], Lz = C.dims[2], Lt = C.dims[3];
        const int s3 = x + Lx * (y + Ly * z);
        int back3[3];
        back3[0] = (x == 0) ? s3 + (Lx - 1) : s3 - 1;
        back3[1] = (y == 0) ? s3 + (Ly - 1) * Lx : s3 - Lx;
        back3[2] = (z == 0) ? s3 + (Lz - 1) * C.V2 : s3 - C.V2;
        const int t0 = tc * C.tch;
        const double2 *__restrict__ Ub = C.U;
        const double2 *__restrict__ Ut = Ub + (size_t)27 * V;
        double2 prev[9];
        {
            const int sp = s3 + V3 * ((t0 == 0) ? Lt - 1 : t0 - 1);
#pragma unroll
            for (int k = 0; k < 9; ++k) prev[k] = Ut[(size_t)k * V + sp];
        }
        T2 *__restrict__ f = (T2 *)C.fields;
        for (int t = t0; t < t0 + C.tch; ++t) {
            const int s = s3 + V3 * t;
            double2 D[9];
            double fsum = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) D[k] = cz();
#pragma unroll
            for (int mu = 0; mu < 3; ++mu) {
                const double2 *__restrict__ Um = Ub + (size_t)mu * 9 * V;
                const int sb = back3[mu] + V3 * t;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const double2 here = Um[(size_t)k * V + s];
                    const double2 back = Um[(size_t)k * V + sb];
                    D[k] = cadd(D[k], csub(back, here));
                    if (k == 0 || k == 4 || k == 8) fsum += here.x;
                }
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double2 here = Ut[(size_t)k * V + s];
                D[k] = cadd(D[k], csub(prev[k], here));
                if (k == 0 || k == 4 || k == 8) fsum += here.x;
                prev[k] = here;
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
            double tsum = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) tsum += cnorm2(A[k]);
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
            fs = dd_add(fs, dd{fsum, 0.0});
            ts = dd_add(ts, dd{tsum, 0.0});
        }
    }
    block_sum2(fs, ts, red);
    if (threadIdx.x == 0) {
        double *p = C.partials + (size_t)lb * 4;
        p[0] = fs.hi;
        p[1] = fs.lo;
        p[2] = ts.hi;
        p[3] = ts.lo;
    }
}

// ============================================================ reductions + stopping rule
// One block per configuration: sum the block partials in a fixed order,
// F = sum/(12 V) (Eq. 1), theta = sum/(3 V) (Eq. 4); with count_iter, count
// the update, record the history and evaluate the stopping rule theta <= eps.
// Sum the block partials of one configuration in a fixed order (the whole
// block takes part), F = sum/(12 V) (Eq. 1), theta = sum/(3 V) (Eq. 4); with
// count_iter, count the update, record the history, flip the link buffer if
// asked and evaluate the stopping rule theta <= eps.
// The partial sums are taken kReduceLanes at a time in a fixed order; a
// larger work-group leaves its other work-items at zero, which adds nothing
// (dd_add of an exact zero returns its other operand), so every caller forms
// the same sums bit for bit.
constexpr int kReduceLanes = 256;

__device__ void finalize_config(const Cfg &C, int nparts, int count_iter, int flip, dd *red)
{
    Ctrl *ct = C.ctrl;
    dd f = {0.0, 0.0}, t = {0.0, 0.0};
    for (int i = threadIdx.x; i < nparts && (int)threadIdx.x < kReduceLanes; i += kReduceLanes) {
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
            if (flip) ct->cur ^= 1;
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

// One block per configuration entry: finalize_config over the partials of
// the divergence kernel.
__global__ __launch_bounds__(kReduceLanes) void k_reduce(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                         int count_iter, int respect_done, int flip)
{
    __shared__ dd red[2 * (kReduceLanes / 64)];
    const Cfg &C = cfgs[B->idx[blockIdx.x]];
    if (respect_done && C.ctrl->done) return;
    finalize_config(C, C.nblk_march, count_iter, flip, red);
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
__device__ __forceinline__ void dft4r(T2 &a0, T2 &a1, T2 &a2, T2 &a3, int sign)
{
    const T2 s02 = t_add(a0, a2), d02 = t_sub(a0, a2);
    const T2 s13 = t_add(a1, a3), d13 = t_mul_si(t_sub(a1, a3), sign);
    a0 = t_add(s02, s13);
    a2 = t_sub(s02, s13);
    a1 = t_add(d02, d13);
    a3 = t_sub(d02, d13);
}

template <typename T2>
__device__ __forceinline__ void dft4(T2 *a, int sign)
{
    dft4r(a[0], a[1], a[2], a[3], sign);
}

template <typename T2>
__device__ __forceinline__ void dft8(T2 *a, int sign)
{
    using T = typename Cx<T2>::T;
    const T r2 = (T)0.70710678118654752440;
    T2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    T2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4r(e0, e1, e2, e3, sign);
    dft4r(o0, o1, o2, o3, sign);
    // w^q, w = exp(sign 2 pi i / 8): w^1 = (1 + sign i) r2, w^2 = sign i, w^3 = (-1 + sign i) r2
    T2 t1, t3;
    {
        const T2 si = t_mul_si(o1, sign);
        t1.x = (o1.x + si.x) * r2;
        t1.y = (o1.y + si.y) * r2;
    }
    const T2 t2 = t_mul_si(o2, sign);
    {
        const T2 si = t_mul_si(o3, sign);
        t3.x = (si.x - o3.x) * r2;
        t3.y = (si.y - o3.y) * r2;
    }
    a[0] = t_add(e0, o0);
    a[4] = t_sub(e0, o0);
    a[1] = t_add(e1, t1);
    a[5] = t_sub(e1, t1);
    a[2] = t_add(e2, t2);
    a[6] = t_sub(e2, t2);
    a[3] = t_add(e3, t3);
    a[7] = t_sub(e3, t3);
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
    const FastDiv fP = fast_div(P), fnb = fast_div(nb), fNs = fast_div(Ns);
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        int k, j;
        if (k_fast) {
            j = fdiv(b, fP);
            k = b - j * P;
        } else {
            k = fdiv(b, fnb);
            j = b - k * nb;
        }
        const int kk = j - fdiv(j, fNs) * Ns;
        T2 a[R];
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = src[k * ks + (j + m * nb) * ls];
        if (Ns > 1) {  // the first stage's twiddles are all 1
#pragma unroll
            for (int m = 1; m < R; ++m) {
                T2 w = tw[m * kk * tstep];
                if (sign > 0) w.y = -w.y;
                a[m] = t_mul(a[m], w);
            }
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

// stage for a power-of-two pencil length L = 2^lL (and, with k_fast, a
// power-of-two pencil count P = 2^lP): the same butterflies with shifts and
// masks for the index arithmetic. k_fast: element l of pencil k at k + l P;
// otherwise at k L + l.
template <int R, typename T2>
__device__ __forceinline__ void stage_p2(const T2 *__restrict__ src, T2 *__restrict__ dst, const T2 *__restrict__ tw,
                                         int lL, int P, int lP, int lNs, int sign, bool k_fast)
{
    static_assert(R == 2 || R == 4 || R == 8, "power-of-two radix");
    constexpr int lR = (R == 2) ? 1 : (R == 4) ? 2 : 3;
    const int lnb = lL - lR, nb = 1 << lnb;
    const int total = P << lnb;
    const int ltstep = lL - lNs - lR;
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        int k, j;
        if (k_fast) {
            k = b & (P - 1);
            j = b >> lP;
        } else {
            j = b & (nb - 1);
            k = b >> lnb;
        }
        const int kk = j & ((1 << lNs) - 1);
        T2 a[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int l = j + m * nb;
            a[m] = src[k_fast ? k + (l << lP) : (k << lL) + l];
        }
        const int tb = kk << ltstep;
        if (lNs > 0) {  // the first stage's twiddles are all 1
#pragma unroll
            for (int m = 1; m < R; ++m) {
                T2 w = tw[m * tb];
                if (sign > 0) w.y = -w.y;
                a[m] = t_mul(a[m], w);
            }
        }
        if constexpr (R == 2)
            dft2(a);
        else if constexpr (R == 4)
            dft4(a, sign);
        else
            dft8(a, sign);
        const int ob = ((j - kk) << lR) + kk;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int l = ob + (q << lNs);
            dst[k_fast ? k + (l << lP) : (k << lL) + l] = a[q];
        }
    }
}

template <typename T2>
__device__ void fft_pencils_p2(T2 *&src, T2 *&dst, const T2 *tw, const FftAxis &A, int sign, bool k_fast)
{
    const int lL = ilog2(A.L), lP = k_fast ? ilog2(A.P) : 0;
    int lNs = 0;
    for (int st = 0; st < A.nstage; ++st) {
        const int r = A.radix[st];
        switch (r) {
        case 2: stage_p2<2>(src, dst, tw, lL, A.P, lP, lNs, sign, k_fast); lNs += 1; break;
        case 4: stage_p2<4>(src, dst, tw, lL, A.P, lP, lNs, sign, k_fast); lNs += 2; break;
        default: stage_p2<8>(src, dst, tw, lL, A.P, lP, lNs, sign, k_fast); lNs += 3; break;
        }
        __syncthreads();
        T2 *t = src;
        src = dst;
        dst = t;
    }
}

// Global -> LDS copies of a tile. The trip count is bounded at compile time
// and the loop fully unrolled, so the global loads of a work-item can all be
// issued before the first LDS store (the two address spaces do not alias).
template <typename T2, int CAP, int TH>
__device__ __forceinline__ void tile_load_contig(T2 *buf, const T2 *__restrict__ g, int n)
{
    constexpr int NL = (CAP + TH - 1) / TH;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * TH;
        if (i < n) buf[i] = g[i];
    }
}

// Register-staged tiles of the 2D passes. tile_fetch issues the global loads
// of a work-item's elements (element i = threadIdx.x + k TH of the tile) into
// registers; tile_put / tile_get move them to and from LDS. A barrier waits
// only for LDS operations, so the fetch of the next field of a tile stays in
// flight while the current one is transformed. Nothing before the global
// stores branches on the tile size: fetches clamp the element index (n >= 1),
// and LDS accesses of elements past n go to the spare last slot of the
// CAP + CAP/8 data area, which no element of a tile smaller than CAP uses
// (the row padding stays below CAP/8). Registers are copied component-wise:
// whole-vector assignment keeps the array out of registers across the loop.
template <int CAP, int TH>
__host__ __device__ constexpr int tile_regs() { return (CAP + TH - 1) / TH; }

template <int CAP>
__host__ __device__ constexpr int spare_slot() { return CAP + CAP / 8 - 1; }

template <typename T2>
__device__ __forceinline__ void cp2(T2 &d, const T2 &v)
{
    d.x = v.x;
    d.y = v.y;
}

template <typename T2, int CAP, int TH, int NL, bool STREAM = false>
__device__ __forceinline__ void tile_fetch(T2 (&r)[NL], const T2 *__restrict__ g, int n)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const T2 *e = g + min(threadIdx.x + k * TH, (unsigned)n - 1);
        if constexpr (STREAM)
            cp2(r[k], ld_stream(e));
        else
            cp2(r[k], *e);
    }
}

// LDS slot of element i of a tile of rows of `rowlen` with `pad` after each.
template <int CAP>
__device__ __forceinline__ int padded_slot(int i, int n, int lr, FastDiv fr, int pad)
{
    return i < n ? i + pad * (lr >= 0 ? (i >> lr) : fdiv(i, fr)) : spare_slot<CAP>();
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_put_padded(T2 *buf, const T2 (&r)[NL], int n, int rowlen, int pad)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
    const int lr = is_p2(rowlen) ? ilog2(rowlen) : -1;
    const FastDiv fr = fast_div(rowlen);
#pragma unroll
    for (int k = 0; k < NL; ++k) cp2(buf[padded_slot<CAP>(threadIdx.x + k * TH, n, lr, fr, pad)], r[k]);
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_get_padded(T2 (&r)[NL], const T2 *buf, int n, int rowlen, int pad)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
    const int lr = is_p2(rowlen) ? ilog2(rowlen) : -1;
    const FastDiv fr = fast_div(rowlen);
#pragma unroll
    for (int k = 0; k < NL; ++k) cp2(r[k], buf[padded_slot<CAP>(threadIdx.x + k * TH, n, lr, fr, pad)]);
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_store_regs(T2 *__restrict__ g, const T2 (&r)[NL], int n)
{
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * TH;
        if (i < n) cp2(g[i], r[k]);
    }
}

template <typename T2, int CAP, int TH>
__device__ __forceinline__ void tile_store_contig(T2 *__restrict__ g, const T2 *buf, int n)
{
    constexpr int NL = (CAP + TH - 1) / TH;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * TH;
        if (i < n) g[i] = buf[i];
    }
}

// Rows of P consecutive elements, row r at global offset r * rs; element
// (r, p) at LDS index r * P + p. P divides TH, so each work-item keeps one p.
template <typename T2, int CAP, int TH>
__device__ __forceinline__ void tile_load_rows(T2 *buf, const T2 *__restrict__ g, int P, int rows, size_t rs)
{
    constexpr int NL = (CAP + TH - 1) / TH;
    const int lp = ilog2(P);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int r = r0 + k * dr;
        if (r < rows) buf[r * P + p] = g[(size_t)r * rs + p];
    }
}

// As tile_load_rows / tile_store_rows, with `pad` LDS elements after every
// `rpp` rows (row r at LDS r * P + pad * (r / rpp)).
// LDS index of row r, element p, of a row tile with `pad` elements after
// every 2^lrpp rows (lrpp < 0: after every rpp rows, frpp = fast_div(rpp)).
__device__ __forceinline__ int rows_lds(int r, int p, int lp, FastDiv frpp, int lrpp, int pad)
{
    return (r << lp) + p + pad * (lrpp >= 0 ? (r >> lrpp) : fdiv(r, frpp));
}

// Row tiles (the zt pass): element (r, p), r < rows, of rows of P; the
// same register and LDS conventions as the padded tiles above.
template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_fetch_rows(T2 (&v)[NL], const T2 *__restrict__ g, int P, int rows, size_t rs)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
    const int lp = ilog2(P);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) cp2(v[k], g[(size_t)min(r0 + k * dr, rows - 1) * rs + p]);
}

template <int CAP>
__device__ __forceinline__ int rows_slot(int r, int p, int rows, int lp, FastDiv frpp, int lrpp, int pad)
{
    return r < rows ? rows_lds(r, p, lp, frpp, lrpp, pad) : spare_slot<CAP>();
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_put_rows(T2 *buf, const T2 (&v)[NL], int P, int rows, int rpp, int pad)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
    const int lp = ilog2(P), lrpp = is_p2(rpp) ? ilog2(rpp) : -1;
    const FastDiv frpp = fast_div(rpp);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) cp2(buf[rows_slot<CAP>(r0 + k * dr, p, rows, lp, frpp, lrpp, pad)], v[k]);
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_get_rows(T2 (&v)[NL], const T2 *buf, int P, int rows, int rpp, int pad)
{
    static_assert(NL == tile_regs<CAP, TH>(), "one register per tile element of a work-item");
    const int lp = ilog2(P), lrpp = is_p2(rpp) ? ilog2(rpp) : -1;
    const FastDiv frpp = fast_div(rpp);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) cp2(v[k], buf[rows_slot<CAP>(r0 + k * dr, p, rows, lp, frpp, lrpp, pad)]);
}

template <typename T2, int CAP, int TH, int NL>
__device__ __forceinline__ void tile_store_rows_regs(T2 *__restrict__ g, const T2 (&v)[NL], int P, int rows,
                                                    size_t rs)
{
    const int lp = ilog2(P);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int r = r0 + k * dr;
        if (r < rows) cp2(g[(size_t)r * rs + p], v[k]);
    }
}

template <typename T2, int CAP, int TH>
__device__ __forceinline__ void tile_store_rows(T2 *__restrict__ g, const T2 *buf, int P, int rows, size_t rs)
{
    constexpr int NL = (CAP + TH - 1) / TH;
    const int lp = ilog2(P);
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int r = r0 + k * dr;
        if (r < rows) g[(size_t)r * rs + p] = buf[r * P + p];
    }
}

// One axis of the 4D transform for one tile of one field. mode 0: a plain
// pass with the given sign. mode 1 (last axis only): forward transform,
// multiplication by K(p) = (alpha/2)(p2max/p2)/V with K(0) = 0 (Eq. 2; the
// 1/V is the normalisation of the backward transform), backward transform.
template <typename T2, bool P2>
__global__ __launch_bounds__(kFftThreads) void k_fft(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                     int axis, int sign, int mode, void *fields_override,
                                                     int respect_done, int lds_elems)
{
    using T = typename Cx<T2>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int field = blockIdx.y;
    const int c = find_cfg(B->off_fft[axis], B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    const FftAxis &A = C.ax[axis];
    if (P2 != is_p2(A.L)) return;  // the other instance takes it
    if (axis >= 2 && C.line[axis - 2]) return;  // k_fft_line takes it
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
        tile_load_contig<T2, 1024, kFftThreads>(buf0, g + gbase, n);
    } else {
        const int o = t / A.inner_chunks, ic = t % A.inner_chunks;
        gbase = (size_t)o * A.S * L + (size_t)ic * P;
        tile_load_rows<T2, 1024, kFftThreads>(buf0, g + gbase, P, L, A.S);
    }
    __syncthreads();
    T2 *src = buf0, *dst = buf1;
    if constexpr (P2)
        fft_pencils_p2(src, dst, tw, A, mode == 1 ? -1 : sign, k_fast);
    else
        fft_pencils(src, dst, tw, A, ks, ls, mode == 1 ? -1 : sign, k_fast);
    if (mode == 1) {
        // element (l, k) of the tile is momentum site gbase + l S + k
        const T *__restrict__ Km = (const T *)C.kmom + gbase;
        const int lp = ilog2(P);
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int k = idx & (P - 1), l = idx >> lp;
            const T k_t = Km[(size_t)l * A.S + k];
            T2 v = src[idx];
            v.x *= k_t;
            v.y *= k_t;
            src[idx] = v;
        }
        __syncthreads();
        if constexpr (P2)
            fft_pencils_p2(src, dst, tw, A, +1, k_fast);
        else
            fft_pencils(src, dst, tw, A, ks, ls, +1, k_fast);
    }
    if (!k_fast)
        tile_store_contig<T2, 1024, kFftThreads>(g + gbase, src, n);
    else
        tile_store_rows<T2, 1024, kFftThreads>(g + gbase, src, P, L, A.S);
}

// ============================================================ 2D transform tiles (in place)
// LDS data tile capacity of the 2D passes: 64 KiB of elements.
// One radix-R Stockham stage over `npen` pencils of length L in one LDS
// buffer. Pencil k starts at (k % m1) * a1 + (k / m1) * a2, its elements are
// ls apart. Each work-item loads its butterflies into registers, the block
// synchronises, then the results are written back in place.
template <int R, typename T2, int MAXE, int TH>
__device__ __forceinline__ void stage_ip(T2 *buf, const T2 *__restrict__ tw, int L, int npen, int m1, int a1, int a2,
                                         int ls, int Ns, int sign, bool k_fast)
{
    constexpr int MAXB = (MAXE + R * TH - 1) / (R * TH);
    const int nb = L / R;
    const int total = npen * nb;
    const int tstep = L / (Ns * R);
    const FastDiv fnp = fast_div(npen), fnb = fast_div(nb), fm1 = fast_div(m1), fNs = fast_div(Ns);
    T2 v[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
            int k, j;
            if (k_fast) {
                j = fdiv(b, fnp);
                k = b - j * npen;
            } else {
                k = fdiv(b, fnb);
                j = b - k * nb;
            }
            const int q1 = fdiv(k, fm1);
            const int base = (k - q1 * m1) * a1 + q1 * a2;
            const int kk = j - fdiv(j, fNs) * Ns;
#pragma unroll
            for (int m = 0; m < R; ++m) v[i][m] = buf[base + (j + m * nb) * ls];
            if (Ns > 1) {  // the first stage's twiddles are all 1
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    T2 w = tw[m * kk * tstep];
                    if (sign > 0) w.y = -w.y;
                    v[i][m] = t_mul(v[i][m], w);
                }
            }
            if constexpr (R == 2)
                dft2(v[i]);
            else if constexpr (R == 3)
                dft3(v[i], sign);
            else if constexpr (R == 4)
                dft4(v[i], sign);
            else
                dft8(v[i], sign);
            ob[i] = base + ((j - kk) * R + kk) * ls;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[i] + q * Ns * ls] = v[i][q];
        }
    }
    __syncthreads();
}

// All stages of one axis over pencils laid out as in stage_ip.
template <typename T2, int MAXE, int TH>
__device__ __forceinline__ void fft_axis_ip(T2 *buf, const T2 *tw, const FftAxis &A, int npen, int m1, int a1, int a2, int ls,
                            int sign, bool k_fast)
{
    int Ns = 1;
    for (int st = 0; st < A.nstage; ++st) {
        const int r = A.radix[st];
        switch (r) {
        case 2: stage_ip<2, T2, MAXE, TH>(buf, tw, A.L, npen, m1, a1, a2, ls, Ns, sign, k_fast); break;
        case 3: stage_ip<3, T2, MAXE, TH>(buf, tw, A.L, npen, m1, a1, a2, ls, Ns, sign, k_fast); break;
        case 4: stage_ip<4, T2, MAXE, TH>(buf, tw, A.L, npen, m1, a1, a2, ls, Ns, sign, k_fast); break;
        default: stage_ip<8, T2, MAXE, TH>(buf, tw, A.L, npen, m1, a1, a2, ls, Ns, sign, k_fast); break;
        }
        Ns *= r;
    }
}

// stage_ip for power-of-two extents (L = 2^lL, npen = 2^lnpen, m1 = 2^lm1,
// Ns = 2^lNs) with pencils in k-fast order: the index arithmetic is shifts,
// masks and 24-bit multiplies instead of integer divisions.
template <int R, typename T2, int MAXE, int TH>
__device__ __forceinline__ void stage_ip_p2(T2 *buf, const T2 *__restrict__ tw, int lL, int lnpen, int lm1, int a1,
                                            int a2, int ls, int lNs, int sign)
{
    static_assert(R == 2 || R == 4 || R == 8, "power-of-two radix");
    constexpr int lR = (R == 2) ? 1 : (R == 4) ? 2 : 3;
    constexpr int MAXB = (MAXE + R * TH - 1) / (R * TH);
    const int lnb = lL - lR;
    const int total = 1 << (lnpen + lnb);
    const int ltstep = lL - lNs - lR;
    const int mstride = __mul24(1 << lnb, ls);  // element m of a butterfly: + m * nb * ls
    const int qstride = ls << lNs;              // output q: + q * Ns * ls
    T2 v[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
            const int k = b & ((1 << lnpen) - 1), j = b >> lnpen;
            const int base = __mul24(k & ((1 << lm1) - 1), a1) + __mul24(k >> lm1, a2);
            const int kk = j & ((1 << lNs) - 1);
            const int e0 = base + __mul24(j, ls);
#pragma unroll
            for (int m = 0; m < R; ++m) v[i][m] = buf[e0 + m * mstride];
            const int tb = kk << ltstep;
            if (lNs > 0) {  // the first stage's twiddles are all 1
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    T2 w = tw[m * tb];
                    if (sign > 0) w.y = -w.y;
                    v[i][m] = t_mul(v[i][m], w);
                }
            }
            if constexpr (R == 2)
                dft2(v[i]);
            else if constexpr (R == 4)
                dft4(v[i], sign);
            else
                dft8(v[i], sign);
            ob[i] = base + __mul24(((j - kk) << lR) + kk, ls);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[i] + q * qstride] = v[i][q];
        }
    }
    __syncthreads();
}

// fft_axis_ip for a power-of-two axis and power-of-two pencil counts.
template <typename T2, int MAXE, int TH>
__device__ __forceinline__ void fft_axis_ip_p2(T2 *buf, const T2 *tw, const FftAxis &A, int lnpen, int lm1, int a1, int a2, int ls,
                               int sign)
{
    const int lL = ilog2(A.L);
    int lNs = 0;
    for (int st = 0; st < A.nstage; ++st) {
        const int r = A.radix[st];
        switch (r) {
        case 2: stage_ip_p2<2, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 1; break;
        case 4: stage_ip_p2<4, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 2; break;
        default: stage_ip_p2<8, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 3; break;
        }
    }
}

// Stages s0, s0 + step, ... (up to, not including, s1) of a power-of-two
// axis, the first of them with Ns = 2^lNs (step -1: the radix list
// backwards).
template <typename T2, int MAXE, int TH>
__device__ __forceinline__ void fft_axis_stages_p2(T2 *buf, const T2 *tw, const FftAxis &A, int lnpen, int lm1, int a1,
                                                   int a2, int ls, int sign, int s0, int s1, int lNs)
{
    const int lL = ilog2(A.L);
    const int step = s1 >= s0 ? 1 : -1;
    for (int st = s0; st != s1; st += step) {
        switch (A.radix[st]) {
        case 2: stage_ip_p2<2, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 1; break;
        case 4: stage_ip_p2<4, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 2; break;
        default: stage_ip_p2<8, T2, MAXE, TH>(buf, tw, lL, lnpen, lm1, a1, a2, ls, lNs, sign); lNs += 3; break;
        }
    }
}

template <int R, int MAXE, int TH>
__host__ __device__ constexpr int centre_butterflies() { return (MAXE + R * TH - 1) / (R * TH); }

// The centre of the scaled transform along the last axis: its last forward
// radix-R stage (Ns = L/R), the multiplication by K(p) and the first stage of
// the backward transform run with the same radix first (Ns = 1) act on the
// same R elements of a pencil, j + q L/R, so they are done in registers in
// one LDS round trip. The forward stage leaves element q of the butterfly at
// its natural index; the backward stage reads exactly those R elements and
// needs no twiddles. kc[i R + q]: K(p) of element q of butterfly i. Radix 2
// or 4: a work-item then holds as many centre elements (NK) as tile elements.
template <int R, typename T2, int MAXE, int TH, int NK>
__device__ __forceinline__ void stage_centre_p2(T2 *buf, const T2 *__restrict__ tw, int lL, int lnpen, int lm1, int a1,
                                                int a2, int ls, const typename Cx<T2>::T (&kc)[NK])
{
    static_assert(R == 2 || R == 4, "centre stage radix");
    constexpr int lR = (R == 2) ? 1 : 2;
    constexpr int MAXB = centre_butterflies<R, MAXE, TH>();
    static_assert(MAXB * R <= NK, "K registers of the centre stage");
    const int lnb = lL - lR;  // nb = L / R = Ns of the forward stage
    const int total = 1 << (lnpen + lnb);
    const int mstride = __mul24(1 << lnb, ls);
    T2 v[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
            const int k = b & ((1 << lnpen) - 1), j = b >> lnpen;
            const int base = __mul24(k & ((1 << lm1) - 1), a1) + __mul24(k >> lm1, a2);
            const int e0 = base + __mul24(j, ls);
#pragma unroll
            for (int m = 0; m < R; ++m) v[i][m] = buf[e0 + m * mstride];
            if (lnb > 0) {  // forward twiddles exp(-2 pi i m j / L)
#pragma unroll
                for (int m = 1; m < R; ++m) v[i][m] = t_mul(v[i][m], tw[m * j]);
            }
            if constexpr (R == 2)
                dft2(v[i]);
            else
                dft4(v[i], -1);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                v[i][q].x *= kc[i * R + q];
                v[i][q].y *= kc[i * R + q];
            }
            if constexpr (R == 2)
                dft2(v[i]);
            else
                dft4(v[i], +1);
            ob[i] = base + __mul24(j << lR, ls);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * TH;
        if (b < total) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[i] + q * ls] = v[i][q];
        }
    }
    __syncthreads();
}

// K(p) of the centre stage's elements for this work-item (zt tile: t-axis
// pencil k = p + P z, element t = j + q L/R); Km points at the tile's first
// xy-site of the K(p) table.
template <int R, typename T, int MAXE, int TH, int NK>
__device__ __forceinline__ void centre_k_p2(T (&kc)[NK], const T *__restrict__ Km, int lL, int lnpen, int lp, int Lz,
                                            size_t V2)
{
    static_assert(R == 2 || R == 4, "centre stage radix");
    constexpr int lR = (R == 2) ? 1 : 2;
    constexpr int MAXB = centre_butterflies<R, MAXE, TH>();
    static_assert(MAXB * R <= NK, "K registers of the centre stage");
    const int lnb = lL - lR;
    const int total = 1 << (lnpen + lnb);
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = min((int)threadIdx.x + i * TH, total - 1);  // lanes past the last butterfly: any valid one
        const int k = b & ((1 << lnpen) - 1), j = b >> lnpen;
        const int p = k & ((1 << lp) - 1), z = k >> lp;
#pragma unroll
        for (int q = 0; q < R; ++q) kc[i * R + q] = Km[(size_t)(z + Lz * (j + (q << lnb))) * V2 + p];
    }
}

template <typename T2>
__device__ __forceinline__ void load_twiddles(T2 *dst, const Cfg &C, int axis)
{
    const T2 *__restrict__ src = (const T2 *)C.tw + C.tw_off[axis];
    for (int e = threadIdx.x; e < C.dims[axis]; e += blockDim.x) dst[e] = src[e];
}

// 2D transform over (x, y) of Q consecutive xy-planes of one field, in LDS.
// Element (x, y, q) sits at x + Xp (y + Ly q), Xp = Lx + xyPad: the padding
// keeps neighbouring lanes, which work on neighbouring pencils, off the same
// LDS banks in both directions.
// P2: Lx, Ly and Q are powers of two (the caller checked), shift arithmetic.
template <typename T2, int CAP, int TH, bool P2>
__device__ __forceinline__ void xy_transform(T2 *buf, const T2 *twx, const T2 *twy, const Cfg &C, int Q, int sign)
{
    const int Lx = C.dims[0], Ly = C.dims[1], Xp = Lx + C.xyPad;
    if constexpr (P2) {
        const int lx = ilog2(Lx), ly = ilog2(Ly), lq = ilog2(Q);
        // x: pencils k = (y, q), start k * Xp, unit stride
        fft_axis_ip_p2<T2, CAP, TH>(buf, twx, C.ax[0], ly + lq, ly + lq, Xp, 0, 1, sign);
        // y: pencils k = (x, q), start x + Xp Ly q, stride Xp
        fft_axis_ip_p2<T2, CAP, TH>(buf, twy, C.ax[1], lx + lq, lx, 1, Xp * Ly, Xp, sign);
    } else {
        fft_axis_ip<T2, CAP, TH>(buf, twx, C.ax[0], Ly * Q, Ly * Q, Xp, 0, 1, sign, true);
        fft_axis_ip<T2, CAP, TH>(buf, twy, C.ax[1], Lx * Q, Lx, 1, Xp * Ly, Xp, sign, true);
    }
}

// Whether a configuration fits the power-of-two instances of the 2D passes.
__device__ __forceinline__ bool xy_is_p2(const Cfg &C) { return is_p2(C.dims[0]) && is_p2(C.dims[1]) && is_p2(C.xyQ); }
__device__ __forceinline__ bool zt_is_p2(const Cfg &C) { return is_p2(C.dims[2]) && is_p2(C.dims[3]); }

// Pass over (x, y): tile = Q consecutive xy-planes; a work-group transforms
// that tile in fields [fpb y, fpb (y + 1)) of the nf fields, one after the
// other, fetching the next field while it transforms the current one. LDS:
// CAP data elements, then the twiddles of x (tw2 entries reserved) and y.
// fold != 0: one more work-group per configuration (after the tiles) does the
// final reduction of the previous update as k_reduce would (count, stopping
// rule, buffer flip if fold == 2) while the tiles are transformed; the tiles
// of a configuration that has just stopped transform once more, unused.
template <typename T2, int CAP, int TH, bool P2>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(CAP / TH >= 8 ? 2 : 4))) void k_fft_xy(
    const Cfg *__restrict__ cfgs, const Batch *__restrict__ B, int sign, void *fields_override, int respect_done,
    int tw2, int nf, int fpb, int fold)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int ntiles = B->off_xy[B->n];
    if ((int)blockIdx.x >= ntiles) {
        if constexpr (TH >= kReduceLanes) {
            if (blockIdx.y != 0) return;
            const Cfg &R = cfgs[B->idx[blockIdx.x - ntiles]];
            if (R.ctrl->done) return;
            finalize_config(R, R.nblk_march, 1, fold == 2, (dd *)smem);
        }
        return;
    }
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int f0 = blockIdx.y * fpb, f1 = min(nf, f0 + fpb);
    const int c = find_cfg(B->off_xy, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (P2 != xy_is_p2(C)) return;  // the other instance takes it
    if (C.xy_reg && !fields_override) return;  // k_fft_xy_reg takes it
    const int t = tile - B->off_xy[c];
    const int n = C.xyQ * C.V2;
    T2 *buf = (T2 *)smem;
    T2 *twx = buf + CAP + CAP / 8;
    T2 *twy = twx + tw2;
    T2 *__restrict__ g = (T2 *)(fields_override ? fields_override : C.fields) + (size_t)f0 * C.V + (size_t)t * n;
    constexpr int NL = tile_regs<CAP, TH>();
    T2 pre[NL], out[NL];
    tile_fetch<T2, CAP, TH>(pre, g, n);
    load_twiddles(twx, C, 0);
    load_twiddles(twy, C, 1);
    tile_put_padded<T2, CAP, TH>(buf, pre, n, C.dims[0], C.xyPad);
    __syncthreads();
    for (int f = f0; f < f1; ++f, g += C.V) {
        const bool more = f + 1 < f1;
        if (more) tile_fetch<T2, CAP, TH>(pre, g + C.V, n);
        xy_transform<T2, CAP, TH, P2>(buf, twx, twy, C, C.xyQ, sign);
        // a work-item reads its own LDS slots, refills them with the next
        // field, then stores: the wait for the fetch precedes the stores
        tile_get_padded<T2, CAP, TH>(out, buf, n, C.dims[0], C.xyPad);
        if (more) tile_put_padded<T2, CAP, TH>(buf, pre, n, C.dims[0], C.xyPad);
        tile_store_regs<T2, CAP, TH>(g, out, n);
        __syncthreads();
    }
}

// Pass over (z, t): tile = P consecutive xy-sites times the whole (z, t)
// plane, LDS layout [t][z][p]; fields [fpb y, fpb (y + 1)) of nf one after the
// other, the next fetched during the current transform. mode 0: plain
// transform with `sign`; mode 1: forward, multiplication by K(p) =
// (alpha/2)(p2max/p2)/V with K(0) = 0 (Eq. 2; 1/V normalises the backward
// transform), backward.
template <typename T2, int CAP, int TH, bool P2>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(CAP / TH >= 8 ? 2 : 4))) void k_fft_zt(
    const Cfg *__restrict__ cfgs, const Batch *__restrict__ B, int mode, int sign, void *fields_override,
    int respect_done, int tw2, int nf, int fpb)
{
    using T = typename Cx<T2>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int f0 = blockIdx.y * fpb, f1 = min(nf, f0 + fpb);
    const int c = find_cfg(B->off_zt, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (P2 != zt_is_p2(C)) return;  // the other instance takes it
    if (mode == 1 && C.zt_reg) return;  // k_fft_zt_reg takes it
    const int t = tile - B->off_zt[c];
    const int P = C.ztP, Lz = C.dims[2], Lt = C.dims[3], V2 = C.V2;
    const int n = P * Lz * Lt;
    const int i0 = t * P;
    T2 *buf = (T2 *)smem;
    T2 *twz = buf + CAP + CAP / 8;
    T2 *twt = twz + tw2;
    T2 *__restrict__ g = (T2 *)(fields_override ? fields_override : C.fields) + (size_t)f0 * C.V + i0;
    // LDS layout [t][z][p] with t-planes Tp = P Lz + ztPad elements apart
    const int Tp = P * Lz + C.ztPad;
    const int rows = Lz * Lt;
    constexpr int NL = tile_regs<CAP, TH>();
    T2 pre[NL], out[NL];
    tile_fetch_rows<T2, CAP, TH>(pre, g, P, rows, V2);
    // K(p) of this tile's elements, shared by all fields of the tile: in the
    // assignment of the t-axis centre stage (power-of-two extents, last t
    // radix 2 or 4), else in the (row, p) assignment of the tile fetch
    const int lp = ilog2(P), lz = is_p2(Lz) ? ilog2(Lz) : -1;
    const int p = threadIdx.x & (P - 1), r0 = threadIdx.x >> lp, dr = TH >> lp;
    const int lt = P2 ? ilog2(Lt) : 0;
    const FftAxis &At = C.ax[3];
    const int rlast = At.radix[At.nstage - 1];
    const bool centre = P2 && mode == 1 && rlast <= 4;
    T kreg[NL];
    if (mode == 1) {
        const T *__restrict__ Km = (const T *)C.kmom + i0;
        if (centre) {
            if (rlast == 2)
                centre_k_p2<2, T, CAP, TH>(kreg, Km, lt, lp + lz, lp, Lz, V2);
            else
                centre_k_p2<4, T, CAP, TH>(kreg, Km, lt, lp + lz, lp, Lz, V2);
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) kreg[k] = Km[(size_t)min(r0 + k * dr, rows - 1) * V2 + p];
        }
    }
    load_twiddles(twz, C, 2);
    load_twiddles(twt, C, 3);
    tile_put_rows<T2, CAP, TH>(buf, pre, P, rows, Lz, C.ztPad);
    __syncthreads();
    const int s0 = (mode == 1) ? -1 : sign;
    const FastDiv flz = fast_div(Lz);
    for (int f = f0; f < f1; ++f, g += C.V) {
        const bool more = f + 1 < f1;
        if (more) tile_fetch_rows<T2, CAP, TH>(pre, g + C.V, P, rows, V2);
        // z: pencils k = (p, t), start p + Tp t, stride P
        // t: pencils k = (p, z), start k, stride Tp
        if constexpr (P2) {
            fft_axis_ip_p2<T2, CAP, TH>(buf, twz, C.ax[2], lp + lt, lp, 1, Tp, P, s0);
            if (centre) {
                // t: forward stages but the last, the centre stage with K(p),
                // the remaining backward stages with the radix list reversed;
                // then z backward
                const int ns = At.nstage;
                fft_axis_stages_p2<T2, CAP, TH>(buf, twt, At, lp + lz, lp + lz, 1, 0, Tp, -1, 0, ns - 1, 0);
                if (rlast == 2)
                    stage_centre_p2<2, T2, CAP, TH>(buf, twt, lt, lp + lz, lp + lz, 1, 0, Tp, kreg);
                else
                    stage_centre_p2<4, T2, CAP, TH>(buf, twt, lt, lp + lz, lp + lz, 1, 0, Tp, kreg);
                fft_axis_stages_p2<T2, CAP, TH>(buf, twt, At, lp + lz, lp + lz, 1, 0, Tp, +1, ns - 2, -1, ilog2(rlast));
                fft_axis_ip_p2<T2, CAP, TH>(buf, twz, C.ax[2], lp + lt, lp, 1, Tp, P, +1);
            } else {
                fft_axis_ip_p2<T2, CAP, TH>(buf, twt, C.ax[3], lp + lz, lp + lz, 1, 0, Tp, s0);
            }
        } else {
            fft_axis_ip<T2, CAP, TH>(buf, twz, C.ax[2], P * Lt, P, 1, Tp, P, s0, true);
            fft_axis_ip<T2, CAP, TH>(buf, twt, C.ax[3], P * Lz, P * Lz, 1, 0, Tp, s0, true);
        }
        if (mode == 1 && !centre) {
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int li = rows_slot<CAP>(r0 + k * dr, p, rows, lp, flz, lz, C.ztPad);
                T2 v = buf[li];
                v.x *= kreg[k];
                v.y *= kreg[k];
                buf[li] = v;
            }
            __syncthreads();
            if constexpr (P2) {
                fft_axis_ip_p2<T2, CAP, TH>(buf, twt, C.ax[3], lp + lz, lp + lz, 1, 0, Tp, +1);
                fft_axis_ip_p2<T2, CAP, TH>(buf, twz, C.ax[2], lp + lt, lp, 1, Tp, P, +1);
            } else {
                fft_axis_ip<T2, CAP, TH>(buf, twt, C.ax[3], P * Lz, P * Lz, 1, 0, Tp, +1, true);
                fft_axis_ip<T2, CAP, TH>(buf, twz, C.ax[2], P * Lt, P, 1, Tp, P, +1, true);
            }
        }
        // own slots out, next field in, then the stores (see k_fft_xy)
        tile_get_rows<T2, CAP, TH>(out, buf, P, rows, Lz, C.ztPad);
        if (more) tile_put_rows<T2, CAP, TH>(buf, pre, P, rows, Lz, C.ztPad);
        tile_store_rows_regs<T2, CAP, TH>(g, out, P, rows, V2);
        __syncthreads();
    }
}

// ============================================================ (z, t) pass, 32 x 32 planes, radix stages in registers
// For Lz = Lt = 32 the scaled (z, t) pass (forward, K(p), backward) keeps
// each 32-point pencil in the registers of four lanes of one wave (lane
// offsets 0, 16, 32, 48; 8 elements each) and runs both radix stages of an
// axis there: an 8-point DFT per lane, the twiddles exp(-2 pi i j k1 / 32),
// an exchange among the four lanes by the gfx950 lane-swap instructions (no
// LDS, no barrier), and 4-point DFTs. LDS is used only to move the tile from
// z-pencils to t-pencils and back (two transposes per field) instead of one
// round trip per radix stage. The forward transform leaves its outputs in the
// order the exchange produces; the backward transform takes them in that
// order (the stages mirrored), so no reordering pass is needed.

// Swap of `a`'s lanes 32..63 with `b`'s lanes 0..31, and of `a`'s odd
// 16-lane rows with `b`'s even rows, per 32-bit word.
__device__ __forceinline__ void lane_swap32(unsigned &a, unsigned &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void lane_swap16(unsigned &a, unsigned &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
template <bool W32>
__device__ __forceinline__ void lane_swap(double &a, double &b)
{
    unsigned long long ua = __builtin_bit_cast(unsigned long long, a), ub = __builtin_bit_cast(unsigned long long, b);
    unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    if constexpr (W32) {
        lane_swap32(alo, blo);
        lane_swap32(ahi, bhi);
    } else {
        lane_swap16(alo, blo);
        lane_swap16(ahi, bhi);
    }
    a = __builtin_bit_cast(double, (unsigned long long)alo | ((unsigned long long)ahi << 32));
    b = __builtin_bit_cast(double, (unsigned long long)blo | ((unsigned long long)bhi << 32));
}
template <bool W32>
__device__ __forceinline__ void lane_swap(float &a, float &b)
{
    unsigned ua = __builtin_bit_cast(unsigned, a), ub = __builtin_bit_cast(unsigned, b);
    if constexpr (W32)
        lane_swap32(ua, ub);
    else
        lane_swap16(ua, ub);
    a = __builtin_bit_cast(float, ua);
    b = __builtin_bit_cast(float, ub);
}
template <bool W32, typename T2>
__device__ __forceinline__ void lane_swap(T2 &a, T2 &b)
{
    lane_swap<W32>(a.x, b.x);
    lane_swap<W32>(a.y, b.y);
}

// The exchange among the four lanes j = 2 a + c (lane offset 32 a + 16 c) of
// a pencil: before, lane j holds Y_j[k1] at R[k1] (k1 = 0..7); after, lane j
// holds Y_jj[2 j + e] at R[2 jj + e] (jj = 0..3, e = 0, 1). First the lanes
// 32 apart trade the halves k1 >= 4 (a = 0) and k1 < 4 (a = 1), leaving
// R[m + 4 a'] = Y_{2 a' + c}[4 a + m]; then the lanes 16 apart trade the
// quarters the same way. Each step is its own inverse, so the reverse
// exchange runs them in the opposite order.
template <typename T2>
__device__ __forceinline__ void pencil_exchange(T2 (&R)[8])
{
#pragma unroll
    for (int m = 0; m < 4; ++m) lane_swap<true>(R[m], R[m + 4]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 2; ++e) lane_swap<false>(R[4 * a + e], R[4 * a + 2 + e]);
}
template <typename T2>
__device__ __forceinline__ void pencil_exchange_back(T2 (&R)[8])
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 2; ++e) lane_swap<false>(R[4 * a + e], R[4 * a + 2 + e]);
#pragma unroll
    for (int m = 0; m < 4; ++m) lane_swap<true>(R[m], R[m + 4]);
}

// Forward 32-point DFT X[k] = sum_n x[n] exp(-2 pi i n k / 32) of a pencil
// spread over four lanes, n = 4 n2 + j:
//   X[k1 + 8 k2] = sum_j exp(-2 pi i j k2 / 4) exp(-2 pi i j k1 / 32) Y_j[k1],
//   Y_j[k1] = sum_n2 x[4 n2 + j] exp(-2 pi i n2 k1 / 8).
// On entry R[n2] = x[4 n2 + j]; on return R[2 k2 + e] = X[2 j + e + 8 k2].
// tw[e] = exp(-2 pi i e / 32), e = 0..31 (a table in LDS: the 16 lanes of an
// access share j, so each read is a broadcast).
template <typename T2>
__device__ __forceinline__ void pencil32_forward(T2 (&R)[8], const T2 *tw, int j)
{
    dft8(R, -1);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) R[k1] = t_mul(R[k1], tw[(j * k1) & 31]);
    pencil_exchange(R);
#pragma unroll
    for (int e = 0; e < 2; ++e) dft4r(R[e], R[2 + e], R[4 + e], R[6 + e], -1);
}

// Backward 32-point DFT x[n] = sum_k X[k] exp(+2 pi i n k / 32) (unnormalised)
// from the layout pencil32_forward leaves, back to R[n2] = x[4 n2 + j]:
//   x[4 n2 + j] = sum_k1 exp(2 pi i n2 k1 / 8) exp(2 pi i j k1 / 32) Z_k1[j],
//   Z_k1[j] = sum_k2 X[k1 + 8 k2] exp(2 pi i j k2 / 4).
template <typename T2>
__device__ __forceinline__ void pencil32_backward(T2 (&R)[8], const T2 *tw, int j)
{
#pragma unroll
    for (int e = 0; e < 2; ++e) dft4r(R[e], R[2 + e], R[4 + e], R[6 + e], +1);
    pencil_exchange_back(R);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) {
        T2 w = tw[(j * k1) & 31];
        w.y = -w.y;
        R[k1] = t_mul(R[k1], w);
    }
    dft8(R, +1);
}

// LDS layout of a P x 32 x 32 tile (p, z, t): p + P z + 33 P t. The
// t-plane stride is P (mod 16) elements, so the 16 lanes an LDS access of
// 16-byte elements serves together (P values of p times 16 / P t-planes when
// z-pencils write, P p times 16 / P z when t-pencils read) fall on distinct
// banks.
template <int P>
__host__ __device__ constexpr int zt_reg_tp() { return 33 * P; }
template <int P>
__host__ __device__ constexpr int zt_reg_lds_elems() { return 32 * zt_reg_tp<P>(); }
// dynamic LDS of k_fft_zt_reg: the tile and the 32 twiddles
template <int P>
__host__ __device__ constexpr int zt_reg_lds_total() { return zt_reg_lds_elems<P>() + 32; }

// Index of K(p) for xy-site xy and (z, t) site zt = kz + Lz kt (nzt = Lz Lt
// sites per plane) in the register pass's tile order: tile xy / P, then
// (z, t), then p = xy mod P.
__host__ __device__ __forceinline__ size_t zt_reg_k_index(int xy, int zt, int P, int nzt)
{
    return ((size_t)(xy / P) * nzt + zt) * P + xy % P;
}

// The scaled (z, t) pass over configurations with Lz = Lt = 32 (C.zt_reg):
// a work-group of 128 P work-items (2 P waves) transforms kFields / ngroups
// of the four fields of its tile, P = C.ztP consecutive xy-sites times the
// (z, t) plane, one after the other; the ngroups work-groups of a tile are
// consecutive (one XCD, whose L2 then serves the tile's K(p) to all of
// them). Work-item (w, q, j), lane q + 16 j of wave w, holds the pencil
// (p, r) = ((16 w + q) mod P, (16 w + q) / P) along z (elements z = 4 n2 + j,
// r = t), then along t (elements t = 4 n2 + j, r = z). A (z, t) row of a
// tile is P consecutive elements in memory: P = 8 FP64 elements fill a
// 128-byte cache line, which smaller tiles share with other work-groups
// (each of which then moves the whole line from L2). The tile sits in
// dynamic LDS (P = 8, FP64: 132 KiB, one work-group per CU).
template <typename T2, int P>
__global__ __launch_bounds__(128 * P) __attribute__((amdgpu_waves_per_eu(P >= 4 ? 4 : 1))) void k_fft_zt_reg(
    const Cfg *__restrict__ cfgs, const Batch *__restrict__ B, int respect_done, int ngroups)
{
    using T = typename Cx<T2>::T;
    constexpr int TP = zt_reg_tp<P>();
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *buf = (T2 *)smem;
    T2 *tw = buf + zt_reg_lds_elems<P>();  // exp(-2 pi i e / 32), the same table for z and t
    const int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = rb / ngroups, grp = rb - tile * ngroups;
    const int nfg = kFields / ngroups, f0 = grp * nfg;
    const int c = find_cfg(B->off_zt, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (!C.zt_reg || C.ztP != P || C.dims[2] != 32 || C.dims[3] != 32) return;  // another pass, width or shape
    const int V2 = C.V2;
    const int i0 = (tile - B->off_zt[c]) * P;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane & 15, j = lane >> 4;
    const int id = 16 * w + q;
    const int p = id % P, r = id / P;
    if (threadIdx.x < 32) tw[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[2])[threadIdx.x];
    // K(p) of the elements a work-item holds after the forward t transform:
    // momentum (xy-site i0 + p, kz = r, kt = 2 j + e + 8 k2) at R[2 k2 + e]
    T kreg[8];
    {
        // the table is in this pass's tile order (zt_reg_k_index)
        const T *__restrict__ Km = (const T *)C.kmom + zt_reg_k_index(i0 + p, 0, P, 1024);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
            for (int e = 0; e < 2; ++e) kreg[2 * k2 + e] = Km[(r + 32 * (2 * j + e + 8 * k2)) * P];
    }
    // z-pencil element n2 (z = 4 n2 + j, t = r) of field f0 in global memory
    T2 *__restrict__ g = (T2 *)C.fields + (size_t)f0 * C.V + i0 + p + (size_t)V2 * (32 * r + j);
    const size_t gz = (size_t)4 * V2;  // z -> z + 4
    for (int f = 0; f < nfg; ++f, g += C.V) {
        T2 R[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) R[n2] = g[n2 * gz];
        if (f == 0) __syncthreads();  // the twiddle table
        pencil32_forward(R, tw, j);   // R[2 k2 + e] = (kz = 2 j + e + 8 k2, t = r)
        if (f) __syncthreads();       // the previous field's t -> z reads are done
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
            for (int e = 0; e < 2; ++e) buf[p + P * (2 * j + e + 8 * k2) + TP * r] = R[2 * k2 + e];
        __syncthreads();
        // t-pencil (p, kz = r): elements t = 4 n2 + j
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) R[n2] = buf[p + P * r + TP * (4 * n2 + j)];
        pencil32_forward(R, tw, j);  // R[2 k2 + e] = (kz = r, kt = 2 j + e + 8 k2)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            R[k].x *= kreg[k];
            R[k].y *= kreg[k];
        }
        pencil32_backward(R, tw, j);  // R[n2] = (kz = r, t = 4 n2 + j)
        __syncthreads();           // every z -> t read is done
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) buf[p + P * r + TP * (4 * n2 + j)] = R[n2];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
            for (int e = 0; e < 2; ++e) R[2 * k2 + e] = buf[p + P * (2 * j + e + 8 * k2) + TP * r];
        pencil32_backward(R, tw, j);  // R[n2] = (z = 4 n2 + j, t = r)
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) g[n2 * gz] = R[n2];
    }
}

// ============================================================ 1D z and t passes, lines of 16 to 64 points in registers
// Where Lz or Lt is 16, 24, 32, 48 or 64 (C.line[]) the 1D passes along that
// axis (the plain transform passes and the scaled t pass: forward, K(p),
// backward) keep each line of L = LPL M points in LPL lanes of one wave
// (LPL = 4 lanes at offsets 0, 16, 32, 48 for 32, 48 and 64 points; LPL = 2
// at offsets 0 and 32 for 16 and 24 points), M elements each: an M-point DFT
// per lane, the twiddles exp(-2 pi i j k1 / L), the exchange among the LPL
// lanes by the gfx950 lane-swap instructions, and LPL-point DFTs. The 64/LPL
// lanes of a row are consecutive xy-sites, so every global access of a wave
// is LPL runs of 64/LPL consecutive elements (256 bytes FP64 for LPL = 4,
// 512 for LPL = 2); nothing goes through LDS but the twiddle table. Elements
// are read and written at their natural positions; only the registers hold
// the exchange order.

// R-point DFT (R = 1, 2, 3, 4) of t[0..R-1] in place.
template <int R, typename T2>
__device__ __forceinline__ void dft_small(T2 (&t)[R], int sign)
{
    if constexpr (R == 2)
        dft2(t);
    else if constexpr (R == 3)
        dft3(t, sign);
    else if constexpr (R == 4)
        dft4r(t[0], t[1], t[2], t[3], sign);
}

// M-point DFT (M = R1 R2 with R1 = 4, or 2 where 4 does not divide M) of
// a[0..M-1] in place, natural order in and out, sign -1 (forward) or +1;
// tw[e] = exp(-2 pi i e / (S M)), so that exp(-2 pi i m / M) = tw[S m].
// n = n0 + R1 n1, k = k1 + R2 k2:
//   X[k1 + R2 k2] = sum_n0 exp(s 2 pi i n0 k2 / R1) exp(s 2 pi i n0 k1 / M)
//                   sum_n1 a[n0 + R1 n1] exp(s 2 pi i n1 k1 / R2).
template <int M, int S, typename T2>
__device__ __forceinline__ void dft_lane(T2 (&a)[M], const T2 *tw, int sign)
{
    constexpr int R1 = (M % 4 == 0) ? 4 : 2, R2 = M / R1;
#pragma unroll
    for (int n0 = 0; n0 < R1; ++n0) {
        T2 t[R2];
#pragma unroll
        for (int n1 = 0; n1 < R2; ++n1) t[n1] = a[n0 + R1 * n1];
        dft_small<R2>(t, sign);
#pragma unroll
        for (int k1 = 0; k1 < R2; ++k1) a[n0 + R1 * k1] = t[k1];
    }
#pragma unroll
    for (int n0 = 1; n0 < R1; ++n0)
#pragma unroll
        for (int k1 = 1; k1 < R2; ++k1) {
            T2 w = tw[S * n0 * k1];
            if (sign > 0) w.y = -w.y;
            a[n0 + R1 * k1] = t_mul(a[n0 + R1 * k1], w);
        }
#pragma unroll
    for (int k1 = 0; k1 < R2; ++k1) {
        T2 t[R1];
#pragma unroll
        for (int n0 = 0; n0 < R1; ++n0) t[n0] = a[R1 * k1 + n0];
        dft_small<R1>(t, sign);
#pragma unroll
        for (int k2 = 0; k2 < R1; ++k2) a[R1 * k1 + k2] = t[k2];
    }
    // X[k] is at a[R1 (k mod R2) + k / R2]: rename into natural order
    T2 b[M];
#pragma unroll
    for (int k = 0; k < M; ++k) b[k] = a[R1 * (k % R2) + k / R2];
#pragma unroll
    for (int k = 0; k < M; ++k) a[k] = b[k];
}

// The exchange among the LPL lanes j of a line: before, lane j holds Y_j[k1]
// at R[k1] (k1 = 0..M-1); after, lane j holds Y_jj[(M/LPL) j + e] at
// R[(M/LPL) jj + e] (jj < LPL, e < M/LPL). The lanes 32 apart trade halves
// (R[m + (M/2) a'] = Y_{a' ...}[(M/2) a + m] after, a the lane's half); with
// four lanes (j = 2 a + c, offset 32 a + 16 c) the lanes 16 apart then trade
// quarters of each half. Each step is its own inverse.
template <int LPL, int M, typename T2>
__device__ __forceinline__ void line_exchange(T2 (&R)[M])
{
#pragma unroll
    for (int m = 0; m < M / 2; ++m) lane_swap<true>(R[m], R[m + M / 2]);
    if constexpr (LPL == 4) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int e = 0; e < M / 4; ++e) lane_swap<false>(R[(M / 2) * a + e], R[(M / 2) * a + M / 4 + e]);
    }
}
template <int LPL, int M, typename T2>
__device__ __forceinline__ void line_exchange_back(T2 (&R)[M])
{
    if constexpr (LPL == 4) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int e = 0; e < M / 4; ++e) lane_swap<false>(R[(M / 2) * a + e], R[(M / 2) * a + M / 4 + e]);
    }
#pragma unroll
    for (int m = 0; m < M / 2; ++m) lane_swap<true>(R[m], R[m + M / 2]);
}

// The LPL-point DFTs over jj of the exchanged layout, R[(M/LPL) jj + e].
template <int LPL, int M, typename T2>
__device__ __forceinline__ void line_dft_across(T2 (&R)[M], int sign)
{
    constexpr int Q = M / LPL;
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        T2 t[LPL];
#pragma unroll
        for (int jj = 0; jj < LPL; ++jj) t[jj] = R[Q * jj + e];
        dft_small<LPL>(t, sign);
#pragma unroll
        for (int jj = 0; jj < LPL; ++jj) R[Q * jj + e] = t[jj];
    }
}

// Forward L-point DFT (L = LPL M) of a line spread over LPL lanes,
// n = LPL n2 + j:
//   X[k1 + M k2] = sum_j exp(-2 pi i j k2 / LPL) exp(-2 pi i j k1 / L) Y_j[k1],
//   Y_j[k1] = sum_n2 x[LPL n2 + j] exp(-2 pi i n2 k1 / M).
// On entry R[n2] = x[LPL n2 + j]; on return R[(M/LPL) k2 + e] =
// X[(M/LPL) j + e + M k2].
template <int LPL, int M, typename T2>
__device__ __forceinline__ void line_forward(T2 (&R)[M], const T2 *tw, int j)
{
    dft_lane<M, LPL>(R, tw, -1);
#pragma unroll
    for (int k1 = 1; k1 < M; ++k1) R[k1] = t_mul(R[k1], tw[j * k1]);
    line_exchange<LPL, M>(R);
    line_dft_across<LPL, M>(R, -1);
}

// Backward L-point DFT (unnormalised) from the layout line_forward leaves,
// back to R[n2] = x[LPL n2 + j]:
//   x[LPL n2 + j] = sum_k1 exp(2 pi i n2 k1 / M) exp(2 pi i j k1 / L) Z_k1[j],
//   Z_k1[j] = sum_k2 X[k1 + M k2] exp(2 pi i j k2 / LPL).
template <int LPL, int M, typename T2>
__device__ __forceinline__ void line_backward(T2 (&R)[M], const T2 *tw, int j)
{
    line_dft_across<LPL, M>(R, +1);
    line_exchange_back<LPL, M>(R);
#pragma unroll
    for (int k1 = 1; k1 < M; ++k1) {
        T2 w = tw[j * k1];
        w.y = -w.y;
        R[k1] = t_mul(R[k1], w);
    }
    dft_lane<M, LPL>(R, tw, +1);
}

// One 1D pass along z (axis 2) or t (axis 3) over the configurations whose
// lines along that axis run in registers (C.line[axis - 2]) and are LPL M
// long (the instances for the other lengths take the rest). KIND 0:
// forward; 1: backward; 2 (t only): forward, K(p) (natural order), backward.
// With NQ = 64 / LPL lanes per row, work-group u of a configuration takes
// field u mod nfields of the lines of unit v = u / nfields: xy-sites
// NQ (v mod V2/NQ) + q, and per wave w the line at other coordinate
// 4 (v div V2/NQ) + w (t for a z pass, z for a t pass). The fields of a unit
// are consecutive work-groups (one XCD), so the t pass's K(p) lines come
// from L2 after the first.
template <typename T2, int LPL, int M, int KIND>
__global__ __launch_bounds__(256) void k_fft_line(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                  int axis, void *fields_override, int nfields, int respect_done)
{
    using T = typename Cx<T2>::T;
    constexpr int L = LPL * M, NQ = 64 / LPL, Q = M / LPL;
    __shared__ T2 tw[L];
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    const int *off = B->off_line[axis - 2];
    const int c = find_cfg(off, B->n, u / nfields);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (C.dims[axis] != L) return;  // another length's instance takes it
    const int lu = u - off[c] * nfields;
    const int field = lu % nfields, v = lu / nfields;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane % NQ, j = lane / NQ;
    const int nxyb = C.V2 / NQ;
    const int xyb = v % nxyb, other = 4 * (v / nxyb) + w;
    // element l of this work-item's line at g[q + l S]: a base common to the
    // wave and a 32-bit offset per work-item (below 2^31 elements for every
    // lattice that fits the device)
    const unsigned S = axis == 2 ? (unsigned)C.V2 : (unsigned)C.V3;
    const size_t wbase = (size_t)NQ * xyb + (size_t)other * (axis == 2 ? (size_t)C.V3 : (size_t)C.V2);
    const unsigned o = (unsigned)q;
    if (threadIdx.x < L) tw[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[axis])[threadIdx.x];
    __syncthreads();
    T2 *__restrict__ g = (T2 *)(fields_override ? fields_override : C.fields) + (size_t)field * C.V + wbase;
    T2 R[M];
    if constexpr (KIND == 1) {
#pragma unroll
        for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
            for (int e = 0; e < Q; ++e) R[Q * k2 + e] = g[o + (unsigned)(Q * j + e + M * k2) * S];
        line_backward<LPL, M>(R, tw, j);
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) g[o + (unsigned)(LPL * n2 + j) * S] = R[n2];
    } else {
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) R[n2] = g[o + (unsigned)(LPL * n2 + j) * S];
        line_forward<LPL, M>(R, tw, j);
        if constexpr (KIND == 2) {
            // K(p) of momentum (xy-site, kz, kt = Q j + e + M k2)
            const T *__restrict__ Km = (const T *)C.kmom + wbase;
#pragma unroll
            for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    const T k = Km[o + (unsigned)(Q * j + e + M * k2) * S];
                    R[Q * k2 + e].x *= k;
                    R[Q * k2 + e].y *= k;
                }
            line_backward<LPL, M>(R, tw, j);
#pragma unroll
            for (int n2 = 0; n2 < M; ++n2) g[o + (unsigned)(LPL * n2 + j) * S] = R[n2];
        } else {
#pragma unroll
            for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
                for (int e = 0; e < Q; ++e) g[o + (unsigned)(Q * j + e + M * k2) * S] = R[Q * k2 + e];
        }
    }
}

// ============================================================ (z, t) pass, 16 x 16 to 48 x 48 planes in registers
// The scaled (z, t) pass of configurations with (Lz, Lt) = (16, 16),
// (24, 24), (16, 32) or (48, 48) (C.zt_reg), the counterpart of k_fft_zt_reg built
// from the line transforms above: each z-line (LZ points) and then each
// t-line (LT points) lives in line_lanes of them in one wave, a tile is P
// consecutive xy-sites times the (z, t) plane, and LDS moves the tile from
// z-lines to t-lines and back (layout p + P z + (LZ + 1) P t). Both phases
// use every work-item: P LT z-lines of line_lanes(LZ) lanes and P LZ
// t-lines of line_lanes(LT) lanes are the same count. K(p) is read in the
// tile order of zt_reg_k_index. Work-item (w, q, j) holds line id = NQ w +
// q (NQ = 64 / lanes per line): (p, r) = (id mod P, id / P), r = t along z,
// r = kz along t.
template <int LZ, int LT, int P>
__host__ __device__ constexpr int zt_lines_threads() { return P * LT * line_lanes(LZ); }
template <int LZ, int LT, int P>
__host__ __device__ constexpr int zt_lines_lds_elems() { return (LZ + 1) * P * LT + LZ + LT; }

template <typename T2, int LZ, int LT, int P>
__global__ __launch_bounds__(P * LT * (LZ >= 32 ? 4 : 2)) void k_fft_zt_lines(const Cfg *__restrict__ cfgs,
                                                                              const Batch *__restrict__ B,
                                                                              int respect_done, int ngroups)
{
    using T = typename Cx<T2>::T;
    constexpr int LPZ = line_lanes(LZ), MZ = LZ / LPZ, QZ = MZ / LPZ, NQZ = 64 / LPZ;
    constexpr int LPT = line_lanes(LT), MT = LT / LPT, QT = MT / LPT, NQT = 64 / LPT;
    constexpr int TP = (LZ + 1) * P;
    static_assert(P * LT * LPZ == P * LZ * LPT, "both phases use every work-item");
    static_assert((P * LT * LPZ) % 64 == 0, "whole waves");
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *buf = (T2 *)smem;
    T2 *twz = buf + TP * LT;  // exp(-2 pi i e / LZ)
    T2 *twt = twz + LZ;       // exp(-2 pi i e / LT)
    const int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = rb / ngroups, grp = rb - tile * ngroups;
    const int nfg = kFields / ngroups, f0 = grp * nfg;
    const int c = find_cfg(B->off_zt, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (!C.zt_reg || C.ztP != P || C.dims[2] != LZ || C.dims[3] != LT) return;  // another pass, width or shape
    const int V2 = C.V2;
    const int i0 = (tile - B->off_zt[c]) * P;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int qz = lane % NQZ, jz = lane / NQZ, idz = NQZ * w + qz;
    const int pz = idz % P, rz = idz / P;  // z-line (xy-site i0 + pz, t = rz)
    const int qt = lane % NQT, jt = lane / NQT, idt = NQT * w + qt;
    const int pt = idt % P, rt = idt / P;  // t-line (xy-site i0 + pt, kz = rt)
    if (threadIdx.x < LZ) twz[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[2])[threadIdx.x];
    if (threadIdx.x < LT) twt[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[3])[threadIdx.x];
    // K(p) of the elements a work-item holds after the forward t transform:
    // momentum (xy-site i0 + pt, kz = rt, kt = QT jt + e + MT k2) at Rt[QT k2 + e]
    T kreg[MT];
    {
        const T *__restrict__ Km = (const T *)C.kmom + zt_reg_k_index(i0 + pt, 0, P, LZ * LT);
#pragma unroll
        for (int k2 = 0; k2 < LPT; ++k2)
#pragma unroll
            for (int e = 0; e < QT; ++e) kreg[QT * k2 + e] = Km[(size_t)(rt + LZ * (QT * jt + e + MT * k2)) * P];
    }
    // z-line element n2 (z = LPZ n2 + jz, t = rz) of field f0 in global memory
    T2 *__restrict__ g = (T2 *)C.fields + (size_t)f0 * C.V + i0 + pz + (size_t)V2 * (LZ * rz + jz);
    const size_t gz = (size_t)LPZ * V2;  // z -> z + LPZ
    for (int f = 0; f < nfg; ++f, g += C.V) {
        T2 R[MZ];
#pragma unroll
        for (int n2 = 0; n2 < MZ; ++n2) R[n2] = g[n2 * gz];
        if (f == 0) __syncthreads();     // the twiddle tables
        line_forward<LPZ, MZ>(R, twz, jz);  // R[QZ k2 + e] = (kz = QZ jz + e + MZ k2, t = rz)
        if (f) __syncthreads();             // the previous field's t -> z reads are done
#pragma unroll
        for (int k2 = 0; k2 < LPZ; ++k2)
#pragma unroll
            for (int e = 0; e < QZ; ++e) buf[pz + P * (QZ * jz + e + MZ * k2) + TP * rz] = R[QZ * k2 + e];
        __syncthreads();
        // t-line (pt, kz = rt): elements t = LPT n2 + jt
        T2 Rt[MT];
#pragma unroll
        for (int n2 = 0; n2 < MT; ++n2) Rt[n2] = buf[pt + P * rt + TP * (LPT * n2 + jt)];
        line_forward<LPT, MT>(Rt, twt, jt);  // Rt[QT k2 + e] = (kz = rt, kt = QT jt + e + MT k2)
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            Rt[k].x *= kreg[k];
            Rt[k].y *= kreg[k];
        }
        line_backward<LPT, MT>(Rt, twt, jt);  // Rt[n2] = (kz = rt, t = LPT n2 + jt)
        __syncthreads();                      // every z -> t read is done
#pragma unroll
        for (int n2 = 0; n2 < MT; ++n2) buf[pt + P * rt + TP * (LPT * n2 + jt)] = Rt[n2];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < LPZ; ++k2)
#pragma unroll
            for (int e = 0; e < QZ; ++e) R[QZ * k2 + e] = buf[pz + P * (QZ * jz + e + MZ * k2) + TP * rz];
        line_backward<LPZ, MZ>(R, twz, jz);  // R[n2] = (z = LPZ n2 + jz, t = rz)
#pragma unroll
        for (int n2 = 0; n2 < MZ; ++n2) g[n2 * gz] = R[n2];
    }
}

// ============================================================ (x, y) passes, 16 to 64 point planes, radix stages in registers
// For Lx = Ly = L of 16, 24, 32, 48 or 64 the iteration's (x, y) passes keep
// each x-line (row) and then each y-line (column) of a plane in LPL lanes of
// one wave, M = L / LPL elements per lane, with the line transforms above;
// LDS only moves the planes from rows to columns. A tile is PL consecutive
// planes of one field (8 of 16 points, 4 of 24, 2 of 32, 1 of 48 and 64:
// a tile stays within the 4096 elements of the LDS-staged inverse pass,
// which serves the same tiles for the stage calls and for single-precision
// storage with the FP64 transform), PL L / NQ waves (NQ = 64 / LPL lines
// per wave); work-item (w, q, j) holds line rr = NQ w + q of the tile: row,
// then column, r = rr mod L of plane rr / L. Global memory stays in natural
// order, so the (z, t) and 1D passes and K(p) see the layout the LDS-staged
// passes produce. The LDS row stride L + 1 spreads the lanes of an access
// over the banks.
template <int L>
__host__ __device__ constexpr int xy_reg_threads() { return xy_reg_planes_for(L) * L * line_lanes(L); }
// dynamic LDS: the tile (rows of L + 1 elements) and the L twiddles
template <int L>
__host__ __device__ constexpr int xy_reg_lds_elems() { return xy_reg_planes_for(L) * L * (L + 1) + L; }

// g = 1 + Delta~ from the four packed filtered fields, projected (defined
// with the gauge step below)
template <typename T2>
__device__ __forceinline__ M3 gauge_from_fields(T2 a, T2 b, T2 d, T2 e);

// Forward (x, y) transform of the four fields (kFields / ngroups of them per
// work-group, the next one prefetched): rows x = LPL n2 + j of row y = r, then
// columns y = LPL n2 + j of column kx = r. fold != 0: the work-groups past the
// tiles do the final reduction of the previous update, as k_fft_xy's.
template <typename T2, int L>
__global__ __launch_bounds__(xy_reg_threads<L>()) void k_fft_xy_reg(const Cfg *__restrict__ cfgs,
                                                                   const Batch *__restrict__ B, int respect_done,
                                                                   int ngroups, int fold)
{
    constexpr int LPL = line_lanes(L), M = L / LPL, Q = M / LPL, NQ = 64 / LPL, PL = xy_reg_planes_for(L);
    constexpr int YS = L + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *buf = (T2 *)smem;
    const int ntiles = B->off_xy[B->n] * ngroups;
    if ((int)blockIdx.x >= ntiles) {
        const Cfg &R = cfgs[B->idx[blockIdx.x - ntiles]];
        if (R.ctrl->done) return;
        finalize_config(R, R.nblk_march, 1, fold == 2, (dd *)buf);
        return;
    }
    const int rb = xcd_remap(blockIdx.x, ntiles);
    const int tile = rb / ngroups, grp = rb - tile * ngroups;
    const int nfg = kFields / ngroups, f0 = grp * nfg;
    const int c = find_cfg(B->off_xy, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (!C.xy_reg || C.dims[0] != L) return;  // the LDS-staged pass or another length's instance takes it
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane % NQ, j = lane / NQ;
    const int rr = NQ * w + q, pl = rr / L, r = rr - pl * L;
    T2 *tw = buf + PL * L * YS;  // exp(-2 pi i e / L), the same table for x and y
    if (threadIdx.x < L) tw[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[0])[threadIdx.x];
    __syncthreads();
    T2 *__restrict__ plane = (T2 *)C.fields + (size_t)f0 * C.V + (size_t)((tile - B->off_xy[c]) * PL + pl) * (L * L);
    T2 *__restrict__ sb = buf + pl * L * YS;
    T2 Rn[M];
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2) Rn[n2] = plane[r * L + LPL * n2 + j];
    for (int f = 0; f < nfg; ++f, plane += C.V) {
        T2 R[M];
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) R[n2] = Rn[n2];
        if (f + 1 < nfg) {
#pragma unroll
            for (int n2 = 0; n2 < M; ++n2) Rn[n2] = plane[C.V + r * L + LPL * n2 + j];
        }
        line_forward<LPL, M>(R, tw, j);  // R[Q k2 + e] = (y = r, kx = Q j + e + M k2)
        if (f) __syncthreads();          // the previous field's reads of the tile are done
#pragma unroll
        for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
            for (int e = 0; e < Q; ++e) sb[r * YS + Q * j + e + M * k2] = R[Q * k2 + e];
        __syncthreads();
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) R[n2] = sb[(LPL * n2 + j) * YS + r];
        line_forward<LPL, M>(R, tw, j);  // R[Q k2 + e] = (ky = Q j + e + M k2, kx = r)
#pragma unroll
        for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
            for (int e = 0; e < Q; ++e) plane[(Q * j + e + M * k2) * L + r] = R[Q * k2 + e];
    }
}

// Inverse (x, y) transform of the four fields of a tile. STORE 3: written to
// fields2 (the filtered fields the fused pass forms g from; FP64 link
// storage). STORE 2 (FP32 transform, single-precision storage): one
// work-group takes all four fields, keeps the first three in registers and
// forms g = 1 + Delta~, projected, at each of its sites with the fourth,
// stored in binary32 two-row form (what the LDS-staged pass's gauge store
// mode 2 writes). Columns first (the layout line_backward takes, read from
// natural order), then rows.
template <typename T2, int L, int STORE>
__global__ __launch_bounds__(xy_reg_threads<L>()) void k_fft_xy_inv_reg(const Cfg *__restrict__ cfgs,
                                                                       const Batch *__restrict__ B,
                                                                       int respect_done, int ngroups)
{
    static_assert(STORE == 3 || std::is_same<T2, float2>::value, "binary32 g from the FP32 transform only");
    constexpr int LPL = line_lanes(L), M = L / LPL, Q = M / LPL, NQ = 64 / LPL, PL = xy_reg_planes_for(L);
    constexpr int YS = L + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *buf = (T2 *)smem;
    if (STORE == 2) ngroups = 1;
    const int ntiles = B->off_xy[B->n] * ngroups;
    const int rb = xcd_remap(blockIdx.x, ntiles);
    const int tile = rb / ngroups, grp = rb - tile * ngroups;
    const int nfg = kFields / ngroups, f0 = grp * nfg;
    const int c = find_cfg(B->off_xy, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (!C.xy_reg || C.dims[0] != L) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane % NQ, j = lane / NQ;
    const int rr = NQ * w + q, pl = rr / L, r = rr - pl * L;
    T2 *tw = buf + PL * L * YS;
    if (threadIdx.x < L) tw[threadIdx.x] = ((const T2 *)C.tw + C.tw_off[0])[threadIdx.x];
    __syncthreads();
    const size_t po = (size_t)f0 * C.V + (size_t)((tile - B->off_xy[c]) * PL + pl) * (L * L);
    const T2 *__restrict__ src = (const T2 *)C.fields + po;
    T2 *__restrict__ dst = (T2 *)C.fields2 + po;
    T2 *__restrict__ sb = buf + pl * L * YS;
    T2 Rn[M];
#pragma unroll
    for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
        for (int e = 0; e < Q; ++e) Rn[Q * k2 + e] = ld_stream(src + (Q * j + e + M * k2) * L + r);
    // field f: the prefetched columns in, the next field's prefetched, the
    // rows of this work-item out in R (y = r, x = LPL n2 + j)
    auto field = [&](int f, int nf, T2 (&R)[M]) {
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) R[n2] = Rn[n2];
        if (f + 1 < nf) {
#pragma unroll
            for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
                for (int e = 0; e < Q; ++e)
                    Rn[Q * k2 + e] = ld_stream(src + (size_t)(f + 1) * C.V + (Q * j + e + M * k2) * L + r);
        }
        line_backward<LPL, M>(R, tw, j);  // R[n2] = (y = LPL n2 + j, kx = r)
        if (f) __syncthreads();
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) sb[(LPL * n2 + j) * YS + r] = R[n2];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < LPL; ++k2)
#pragma unroll
            for (int e = 0; e < Q; ++e) R[Q * k2 + e] = sb[r * YS + Q * j + e + M * k2];
        line_backward<LPL, M>(R, tw, j);  // R[n2] = (y = r, x = LPL n2 + j)
    };
    if constexpr (STORE == 3) {
        for (int f = 0; f < nfg; ++f) {
            T2 R[M];
            field(f, nfg, R);
#pragma unroll
            for (int n2 = 0; n2 < M; ++n2) dst[(size_t)f * C.V + r * L + LPL * n2 + j] = R[n2];
        }
    } else {
        T2 keep[3][M];  // fields 0..2 at this work-item's sites
#pragma unroll
        for (int f = 0; f < 3; ++f) field(f, kFields, keep[f]);
        T2 R[M];
        field(3, kFields, R);
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2)
            m3_store12s(C.g12f, C.V, (int)(po + r * L + LPL * n2 + j),
                        gauge_from_fields(keep[0][n2], keep[1][n2], keep[2][n2], R[n2]));
    }
}

// ============================================================ S4: g = 1 + Delta~, projected
// Rebuilds the filtered traceless anti-hermitian matrix from the four packed
// fields (Delta~_10 = -conj(Delta~_01), Delta~_00 = i Re f3, Delta~_11 = i Im f3,
// Delta~_22 = -Delta~_00 - Delta~_11) in FP64, forms g = 1 + Delta~ (first
// order in alpha) and projects it to SU(3).
template <typename T2>
__device__ __forceinline__ M3 gauge_from_fields(T2 a, T2 b, T2 d, T2 e)
{
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
    return m;
}

// g goes to g_override (caller, full matrices) if given, else to the
// workspace: two_row 2 in two-row single-precision storage (g12f), 0 full
// (g). two_row 3: the gauge steps write the filtered fields Delta~ to fields2
// instead, and the fused pass (FP64 link storage) forms each g it needs from
// them.
__device__ __forceinline__ void store_gauge(const Cfg &C, double2 *g_override, int two_row, int s, const M3 &m)
{
    if (g_override)
        m3_store(g_override, C.V, s, m);
    else if (two_row == 2)
        m3_store12s(C.g12f, C.V, s, m);
    else
        m3_store(C.g, C.V, s, m);
}

template <typename T2>
__global__ __launch_bounds__(kSiteBlock) void k_gauge(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                      int respect_done, double2 *__restrict__ g_override, int two_row)
{
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V;
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= V) return;
    const T2 *__restrict__ f = (const T2 *)C.fields;
    if (two_row == 3 && !g_override) {  // the fused pass forms g itself
        T2 *__restrict__ o = (T2 *)C.fields2;
#pragma unroll
        for (int k = 0; k < kFields; ++k) o[(size_t)k * V + s] = f[(size_t)k * V + s];
        return;
    }
    const M3 m = gauge_from_fields(f[s], f[(size_t)V + s], f[(size_t)2 * V + s], f[(size_t)3 * V + s]);
    store_gauge(C, g_override, two_row, s, m);
}

// Inverse transform over (x, y) of the four fields of Q xy-planes, then g and
// its projection at every site of the tile (the last steps of the transform
// and the gauge step in one pass; the fields are not written back), or, for
// the fused exchange pass (two_row 3), the four transformed fields written
// to fields2. A tile is whole contiguous planes, read once: the field loads
// are streaming.
template <typename T2, int CAP, int TH, bool P2>
__global__ __launch_bounds__(TH) void k_fft_xy_inv_gauge(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                         int respect_done, double2 *__restrict__ g_override, int tw2,
                                                         int two_row)
{
    constexpr int MS = (CAP + TH - 1) / TH;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_xy, B->n, tile);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    if (P2 != xy_is_p2(C)) return;  // the other instance takes it
    // k_fft_xy_inv_reg takes it
    if (C.xy_reg && !g_override && (two_row == 3 || (two_row == 2 && std::is_same<T2, float2>::value))) return;
    const int t = tile - B->off_xy[c];
    const int n = C.xyQ * C.V2;
    const size_t site0 = (size_t)t * n;
    T2 *buf = (T2 *)smem;
    T2 *twx = buf + CAP + CAP / 8;
    T2 *twy = twx + tw2;
    const T2 *__restrict__ src = (const T2 *)C.fields + site0;
    T2 val[kFields][MS];
    T2 pre[MS];
    tile_fetch<T2, CAP, TH, MS, true>(pre, src, n);
    load_twiddles(twx, C, 0);
    load_twiddles(twy, C, 1);
    tile_put_padded<T2, CAP, TH>(buf, pre, n, C.dims[0], C.xyPad);
    __syncthreads();
#pragma unroll
    for (int f = 0; f < kFields; ++f) {
        if (f + 1 < kFields) tile_fetch<T2, CAP, TH, MS, true>(pre, src + (size_t)(f + 1) * C.V, n);
        xy_transform<T2, CAP, TH, P2>(buf, twx, twy, C, C.xyQ, +1);
        // own slots out, next field in (the fetch had the transform to land)
        tile_get_padded<T2, CAP, TH>(val[f], buf, n, C.dims[0], C.xyPad);
        if (f + 1 < kFields) {
            tile_put_padded<T2, CAP, TH>(buf, pre, n, C.dims[0], C.xyPad);
            __syncthreads();
        }
    }
    if (two_row == 3 && !g_override) {
        T2 *__restrict__ dst = (T2 *)C.fields2 + site0;
#pragma unroll
        for (int f = 0; f < kFields; ++f) tile_store_regs<T2, CAP, TH>(dst + (size_t)f * C.V, val[f], n);
        return;
    }
#pragma unroll
    for (int k = 0; k < MS; ++k) {
        const int i = threadIdx.x + k * TH;
        if (i < n)
            store_gauge(C, g_override, two_row, (int)(site0 + i),
                        gauge_from_fields(val[0][k], val[1][k], val[2][k], val[3][k]));
    }
}

// ============================================================ S5: link update
// U_mu(x) -> g(x) U_mu(x) g^dag(x + mu) for the four links of each site; all
// g were formed before this launch (the two separate loops of Alg. 1). A block
// owns a set of (x, y, z) sites (see march_xyz) and walks `tch` t-slices:
// g(x + t) of one slice is g(x) of the next, kept in registers.
__global__ __launch_bounds__(kSiteBlock) void k_update(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B,
                                                       int respect_done, const double2 *__restrict__ g_override,
                                                       int allow_reunit)
{
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = find_cfg(B->off_march, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    if (respect_done && C.ctrl->done) return;
    const int V = C.V, V3 = C.V3;
    const int lb = blk - B->off_march[c];
    const int b3 = lb % C.nb3, tc = lb / C.nb3;
    int x, y, z;
    if (!march_xyz(C, b3, threadIdx.x, x, y, z)) return;
    const double2 *__restrict__ G = g_override ? g_override : C.g;
    const bool reunit =
        allow_reunit && C.reunit_every > 0 && ((C.ctrl->iter + 1) % (long long)C.reunit_every) == 0;
    const int Lx = C.dims[0], Ly = C.dims[1], Lz = C.dims[2], Lt = C.dims[3];
    const int s3 = x + Lx * (y + Ly * z);
    int fwd3[3];
    fwd3[0] = (x == Lx - 1) ? s3 - (Lx - 1) : s3 + 1;
    fwd3[1] = (y == Ly - 1) ? s3 - (Ly - 1) * Lx : s3 + Lx;
    fwd3[2] = (z == Lz - 1) ? s3 - (Lz - 1) * C.V2 : s3 + C.V2;
    const int t0 = tc * C.tch;
    M3 gx = m3_load(G, V, s3 + V3 * t0);
    for (int t = t0; t < t0 + C.tch; ++t) {
        const int s = s3 + V3 * t;
        const int tn = (t + 1 == Lt) ? 0 : t + 1;
        const M3 gn = m3_load(G, V, s3 + V3 * tn);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            double2 *__restrict__ Um = C.U + (size_t)mu * 9 * V;
            const M3 u = m3_load(Um, V, s);
            const M3 gf = m3_load(G, V, fwd3[mu] + V3 * t);
            M3 w = m3_mul_dag(m3_mul(gx, u), gf);
            if (reunit) m3_reunit(w);
            m3_store(Um, V, s, w);
        }
        {
            double2 *__restrict__ Um = C.U + (size_t)27 * V;
            const M3 u = m3_load(Um, V, s);
            M3 w = m3_mul_dag(m3_mul(gx, u), gn);
            if (reunit) m3_reunit(w);
            m3_store(Um, V, s, w);
        }
        gx = gn;
    }
}

// ============================================================ S5 + S1 fused
// One pass for the link update and the divergence of the updated links:
//   U'_mu(x) = g(x) U_mu(x) g^dag(x + mu)          (Alg. 1, second loop)
//   D(x) = sum_nu [U'_nu(x - nu) - U'_nu(x)], Delta = (D - D^dag) - trace/3
// Links and g are held in two-row form (the 12-real parametrisation of the
// paper's section 2.2; the third row is rebuilt on load). Old links are read
// from one buffer and the new ones written to the other, so no block ever
// reads a link another block has already replaced. U'_t(x - t) is the U'_t(x)
// of the previous t-slice, kept in registers (recomputed once at the first
// slice of a block); U'_t(x) itself is formed one slice late, once g(x + t)
// is read as the next slice's own g. Also writes the packed transform fields and the
// per-block sums for F (of the new links) and theta. RU: the variant for
// iterations that also project the new links to SU(3) (reunit_every > 0);
// each variant returns at once on the other iterations.

// Two-row link buffer b and two-row g of a configuration, in storage S2.
template <typename S2>
__device__ __forceinline__ S2 *links12(const Cfg &C, int b);
template <>
__device__ __forceinline__ double2 *links12<double2>(const Cfg &C, int b) { return C.U12[b]; }
template <>
__device__ __forceinline__ float2 *links12<float2>(const Cfg &C, int b) { return C.U12f[b]; }

// The fused pass with neighbour exchange through LDS. With FP64 link storage
// every g(x) it needs is formed from the filtered fields Delta~ (4 complex
// numbers per site instead of the 6 of a two-row g) by the same projection
// the gauge step uses (fused_gauge). Per t-slice each work-item publishes its
// g(x) (two rows) and, after its forward links,
// U'_mu(x) - U'_mu(x)^dag for mu = x, y; a neighbour inside the block reads
// them instead of loading g(x + mu) and recomputing U'_nu(x - nu) from the old
// links. The z-neighbours, and x and y neighbours in other blocks (the edge
// rows of a linear site set, the faces of a box), are recomputed from the old
// links and g. (Exchanging z too, for boxes and for sets longer than an
// xy-plane, needs a third LDS array: 80 KB per block, and the single-precision
// storage pass 3 % slower at 32^4 where no block holds a z-neighbour.) The new
// links are formed by their first two rows (m3_mul_mul_dag_rows), exactly what
// is stored, so a recomputed backward link equals the one its owner writes
// (with contraction of multiply-adds fixed by the source, every inlined copy
// rounds alike). D is accumulated as its anti-hermitian part.
//
// Slot of the site (xn, yn, zn), flat index s3n, among the work-items of
// marching block b3 (march_xyz's numbering), or -1 if another block owns it.
// With NB site sets per block (linear sets only for NB > 1), b3 is the
// block's first set and the slot counts over all NB kSiteBlock of them.
template <int NB = 1>
__device__ __forceinline__ int block_slot(const Cfg &C, int b3, int s3n, int xn, int yn, int zn)
{
    if (NB > 1 || C.tile[0] == 0) {
        const int o = s3n - b3 * kSiteBlock;
        return (o >= 0 && o < NB * kSiteBlock) ? o : -1;
    }
    const int tx = C.tile[0], ty = C.tile[1], tz = C.tile[2];
    const int bx = b3 % C.ntile[0], rb = b3 / C.ntile[0];
    const int by = rb % C.ntile[1], bz = rb / C.ntile[1];
    const int lx = xn - bx * tx, ly = yn - by * ty, lz = zn - bz * tz;
    return (lx >= 0 && lx < tx && ly >= 0 && ly < ty && lz >= 0 && lz < tz) ? lx + tx * (ly + ty * lz) : -1;
}

// g(x) from the filtered fields Delta~ (transform precision T2), exactly as a
// g stored in two-row form S2 reads back: rows 0 and 1 rounded to S2 (no-op
// for double2), row 2 rebuilt from them.
template <typename T2, typename S2>
__device__ __forceinline__ M3 gauge_at(const T2 *__restrict__ f, int V, int s)
{
    M3 m = gauge_from_fields(f[s], f[(size_t)V + s], f[(size_t)2 * V + s], f[(size_t)3 * V + s]);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        S2 v;
        narrow(v, m.e[k]);
        m.e[k] = widen(v);
    }
    m3_row2(m);
    return m;
}

// g(x) in the fused pass. FP64 link storage: formed from the filtered fields
// (64 or 32 bytes instead of a 96-byte two-row g). Single-precision storage:
// the stored binary32 two-row g (48 bytes; forming it from 32 bytes of fields
// costs more in projections than it saves, 4 % at 32^4).
template <typename T2, typename S2>
__device__ __forceinline__ M3 fused_gauge(const Cfg &C, int s)
{
    if constexpr (std::is_same<S2, float2>::value)
        return m3_load12s((const float2 *)C.g12f, C.V, s);
    else
        return gauge_at<T2, S2>((const T2 *)C.fields2, C.V, s);
}

// A new link of the fused pass: rows 0 and 1 in two-row storage S2, or, with
// FULL (FP64 storage only), all three rows in the layout of the caller's array
// (row 2 as the two-row form rebuilds it on load: w's own row 2, see m3_row2).
template <typename S2, bool FULL>
__device__ __forceinline__ void store_new_link(S2 *__restrict__ base, int V, int s, const M3 &w)
{
    m3_store12s_stream(base, V, s, w);
    if constexpr (FULL) {
#pragma unroll
        for (int k = 6; k < 9; ++k) st_stream(base + (size_t)k * V + s, w.e[k]);
    }
}

// S2: storage of links and g, double2 or float2 (single-precision storage).
// SRC / DST (FP64 storage): the first update of a call reads the old links
// from the caller's array, the last update of a gf_step call writes the new
// ones there, so that a call copies no links in or out; the updates in
// between use the two-row buffers (these instances run inside the graphs).
// NB: site sets per block (1, or 2 for linear sets: the neighbour exchange
// spans both, each set keeps its own partial sums).
template <typename T2, bool RU, typename S2, bool SRC = false, bool DST = false, int NB = 1>
__global__ __launch_bounds__(kSiteBlock * NB) void k_update_delta_x(const Cfg *__restrict__ cfgs,
                                                                    const Batch *__restrict__ B)
{
    static_assert(!(SRC || DST) || std::is_same<S2, double2>::value, "caller layout: FP64 storage only");
    constexpr int NS = kSiteBlock * NB;
    __shared__ dd red[2 * (NS / 64)];
    __shared__ double2 sg[6][NS];    // g(x), rows 0 and 1, of the block's sites at this slice
    __shared__ double sa[2][9][NS];  // U'_mu(x) - U'_mu(x)^dag (AH order), mu = x, y
    // NB > 1: the block takes NB consecutive site sets of one walk (each
    // configuration's nb3 a multiple of NB), each with its own partial sums
    const int blk = xcd_remap(blockIdx.x, gridDim.x) * NB;
    const int c = find_cfg(B->off_march, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    const Ctrl *ct = C.ctrl;
    if (ct->done) return;  // the whole block leaves together
    const int V = C.V, V3 = C.V3;
    // SRC: the old links are the caller's full matrices (rows 0 and 1 read,
    // row 2 rebuilt: the values a two-row copy holds); DST: the new links go
    // to the caller's array as full matrices. Per direction, element k of a
    // link sits at base + k V + s in both layouts.
    constexpr size_t kOs = SRC ? 9 : 6, kNs = DST ? 9 : 6;
    const S2 *__restrict__ Uo = SRC ? (const S2 *)C.U : links12<S2>(C, ct->cur);
    S2 *__restrict__ Un = DST ? (S2 *)C.U : links12<S2>(C, ct->cur ^ 1);
    const bool reunit = C.reunit_every > 0 && ct->ru_now;
    if (reunit != RU) return;
    const int tid = threadIdx.x;
    const int half = NB > 1 ? tid / kSiteBlock : 0, ltid = NB > 1 ? tid % kSiteBlock : tid;
    const int lb0 = blk - B->off_march[c];  // the block's first site set
    const int lb = lb0 + half;
    const int b3 = lb % C.nb3, tc = lb / C.nb3;
    const int b3f = lb0 % C.nb3;
    // where the links are after this update (read by k_unpack_links only)
    if (lb == 0 && ltid == 0) C.ctrl->in_caller = DST ? 1 : 0;
    int x, y, z;
    const bool inside = march_xyz(C, b3, ltid, x, y, z);
    const int Lx = C.dims[0], Ly = C.dims[1], Lz = C.dims[2], Lt = C.dims[3];
    const int s3 = x + Lx * (y + Ly * z);
    int fwd3[3], back3[3], sf[2], sb[2];
    const int xf = (x == Lx - 1) ? 0 : x + 1, xb = (x == 0) ? Lx - 1 : x - 1;
    const int yf = (y == Ly - 1) ? 0 : y + 1, yb = (y == 0) ? Ly - 1 : y - 1;
    const int zf = (z == Lz - 1) ? 0 : z + 1, zb = (z == 0) ? Lz - 1 : z - 1;
    fwd3[0] = s3 + (xf - x);
    fwd3[1] = s3 + (yf - y) * Lx;
    fwd3[2] = s3 + (zf - z) * C.V2;
    back3[0] = s3 + (xb - x);
    back3[1] = s3 + (yb - y) * Lx;
    back3[2] = s3 + (zb - z) * C.V2;
    sf[0] = inside ? block_slot<NB>(C, b3f, fwd3[0], xf, y, z) : -1;
    sf[1] = inside ? block_slot<NB>(C, b3f, fwd3[1], x, yf, z) : -1;
    sb[0] = inside ? block_slot<NB>(C, b3f, back3[0], xb, y, z) : -1;
    sb[1] = inside ? block_slot<NB>(C, b3f, back3[1], x, yb, z) : -1;
    const int t0 = tc * C.tch;
    dd fs = {0.0, 0.0}, ts = {0.0, 0.0};
    // Slice t forms g(x, t) and completes the site (x, t - 1): its forward
    // t-link needs g(x, t), so it is formed one slice late, and the slice's
    // other links are formed while g(x, t) and the neighbours' g(x +- z, t)
    // are read. Every block then reads a slice's filtered fields in the same
    // slice of its walk, as its z-neighbours and the blocks of its edge rows
    // read them, instead of one slice apart (the fields of slice t + 1 were
    // the owner's g(x + t) of slice t).
    M3 gp;   // g(x, t - 1)
    AH dc;   // D(x, t - 1) without its -(U'_t(x, t - 1) - h.c.)
    AH utp;  // U'_t(x, t - 1) - h.c., the backward t-link of (x, t)
    if (inside) gp = fused_gauge<T2, S2>(C, s3 + V3 * ((t0 == 0) ? Lt - 1 : t0 - 1));
    T2 *__restrict__ f = (T2 *)C.fields;
    for (int t = t0; t <= t0 + C.tch; ++t) {
        const int s = s3 + V3 * ((t == Lt) ? 0 : t);
        const int sp = s3 + V3 * ((t == 0) ? Lt - 1 : t - 1);
        M3 gx;
        double fsum = 0.0;
        if (inside) {
            gx = fused_gauge<T2, S2>(C, s);
            // U'_t(x, t - 1); at the walk's first slice the owner of (x, t0 - 1)
            // stores it, this block only needs its anti-hermitian part
            const M3 u = (t == t0) ? m3_load12s(Uo + kOs * 3 * V, V, sp) : m3_load12s_stream(Uo + kOs * 3 * V, V, sp);
            M3 w = m3_mul_mul_dag_rows(gp, u, gx);
            if (RU) m3_reunit(w);
            utp = ah_of(w);
            if (t > t0) {
                store_new_link<S2, DST>(Un + kNs * 3 * V, V, sp, w);
                fsum += w.e[0].x + w.e[4].x + w.e[8].x;
                AH D = dc;
                ah_acc(D, utp, -1.0);
                // Delta = A - Tr(A)/3 with A = D - D^dag
                const double tr3 = (D.d0 + D.d1 + D.d2) * (1.0 / 3.0);
                const double e0 = D.d0 - tr3, e1 = D.d1 - tr3, e2 = D.d2 - tr3;
                const double tsum =
                    2.0 * (cnorm2(D.o01) + cnorm2(D.o02) + cnorm2(D.o12)) + e0 * e0 + e1 * e1 + e2 * e2;
                T2 fv;
                fv.x = D.o01.x;
                fv.y = D.o01.y;
                st_stream(f + sp, fv);
                fv.x = D.o02.x;
                fv.y = D.o02.y;
                st_stream(f + (size_t)V + sp, fv);
                fv.x = D.o12.x;
                fv.y = D.o12.y;
                st_stream(f + (size_t)2 * V + sp, fv);
                fv.x = e0;
                fv.y = e1;
                st_stream(f + (size_t)3 * V + sp, fv);
                ts = dd_add(ts, dd{tsum, 0.0});
            }
        }
        if (t == t0 + C.tch) {  // the walk's last slice: (x, t) belongs to the next block in t
            if (inside) fs = dd_add(fs, dd{fsum, 0.0});
            break;
        }
        if (inside) {
            // the z-links first: they need no neighbour from LDS, so their
            // loads are in flight with the t-link's before the first barrier
            dc = utp;
            {
                // U_z(x) is the backward neighbour of the next work-group in z,
                // which reads it in the same slice
                const M3 gf = fused_gauge<T2, S2>(C, fwd3[2] + V3 * t);
                M3 w = m3_mul_mul_dag_rows(gx, m3_load12s(Uo + (size_t)2 * kOs * V, V, s), gf);
                if (RU) m3_reunit(w);
                store_new_link<S2, DST>(Un + (size_t)2 * kNs * V, V, s, w);
                fsum += w.e[0].x + w.e[4].x + w.e[8].x;
                ah_acc(dc, ah_of(w), -1.0);
            }
            {
                const int sbk = back3[2] + V3 * t;
                M3 wb = m3_mul_mul_dag_rows(fused_gauge<T2, S2>(C, sbk), m3_load12s(Uo + (size_t)2 * kOs * V, V, sbk), gx);
                if (RU) m3_reunit(wb);
                ah_acc(dc, ah_of(wb), 1.0);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) sg[k][tid] = gx.e[k];
        }
        __syncthreads();
        if (inside) {
#pragma unroll
            for (int mu = 0; mu < 2; ++mu) {
                M3 gf;
                if (sf[mu] >= 0) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) gf.e[k] = sg[k][sf[mu]];
                    m3_row2(gf);
                } else {
                    gf = fused_gauge<T2, S2>(C, fwd3[mu] + V3 * t);
                }
                // U_x(x) and U_y(x) are read again only at the block's edge rows
                const M3 u = m3_load12s_stream(Uo + (size_t)mu * kOs * V, V, s);
                M3 w = m3_mul_mul_dag_rows(gx, u, gf);
                if (RU) m3_reunit(w);
                store_new_link<S2, DST>(Un + (size_t)mu * kNs * V, V, s, w);
                fsum += w.e[0].x + w.e[4].x + w.e[8].x;
                const AH a = ah_of(w);
                ah_acc(dc, a, -1.0);
                sa[mu][0][tid] = a.o01.x;
                sa[mu][1][tid] = a.o01.y;
                sa[mu][2][tid] = a.o02.x;
                sa[mu][3][tid] = a.o02.y;
                sa[mu][4][tid] = a.o12.x;
                sa[mu][5][tid] = a.o12.y;
                sa[mu][6][tid] = a.d0;
                sa[mu][7][tid] = a.d1;
                sa[mu][8][tid] = a.d2;
            }
            fs = dd_add(fs, dd{fsum, 0.0});
        }
        __syncthreads();
        if (inside) {
#pragma unroll
            for (int nu = 0; nu < 2; ++nu) {
                AH a;
                if (sb[nu] >= 0) {
                    const int o = sb[nu];
                    a.o01 = make_double2(sa[nu][0][o], sa[nu][1][o]);
                    a.o02 = make_double2(sa[nu][2][o], sa[nu][3][o]);
                    a.o12 = make_double2(sa[nu][4][o], sa[nu][5][o]);
                    a.d0 = sa[nu][6][o];
                    a.d1 = sa[nu][7][o];
                    a.d2 = sa[nu][8][o];
                } else {
                    const int sbk = back3[nu] + V3 * t;
                    M3 wb = m3_mul_mul_dag_rows(fused_gauge<T2, S2>(C, sbk), m3_load12s(Uo + (size_t)nu * kOs * V, V, sbk), gx);
                    if (RU) m3_reunit(wb);
                    a = ah_of(wb);
                }
                ah_acc(dc, a, 1.0);
            }
            gp = gx;
        }
    }
    block_sum2_sets<NB>(fs, ts, red);
    if (ltid == 0) {
        double *p = C.partials + (size_t)lb * 4;
        p[0] = fs.hi;
        p[1] = fs.lo;
        p[2] = ts.hi;
        p[3] = ts.lo;
    }
}

// K(p) = (alpha/2)(p2max/p2)/V for every momentum site, K(0) = 0 (Eq. 2; the
// 1/V normalises the backward transform), with p2 = sum_mu 4 sin^2(pi n_mu /
// L_mu); stored in the transform precision (an FP32 table holds the FP64
// value rounded to nearest). Filled when the transform schedule is set. In
// site order, or, for a configuration whose (z, t) pass runs in
// k_fft_zt_reg, in that pass's tile order (zt_reg_k_index), so that a tile
// reads its K(p) contiguously.
template <typename T>
__global__ __launch_bounds__(kSiteBlock) void k_momentum_table(const Cfg *__restrict__ cfgs,
                                                               const Batch *__restrict__ B)
{
    const int blk = blockIdx.x;
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= C.V) return;
    int n[4];
    site_coords(C.dims, s, n);
    const double *s2 = C.sin2;
    const double p2 =
        s2[C.sin2_off[0] + n[0]] + s2[C.sin2_off[1] + n[1]] + s2[C.sin2_off[2] + n[2]] + s2[C.sin2_off[3] + n[3]];
    const size_t o = C.zt_reg ? zt_reg_k_index(s % C.V2, s / C.V2, C.ztP, C.dims[2] * C.dims[3]) : (size_t)s;
    ((T *)C.kmom)[o] = (T)((p2 > 0.0) ? C.kfac / p2 : 0.0);
}

// Reads every configuration's two-row link buffers (what the fused pass of
// an iteration streams between two transform passes), so that the transform
// passes the autotuner times start from the caches an iteration leaves them.
// The sum is stored (so the loads stay) only if it is not finite, into a
// block partial sum that the measurement after the tuning rewrites.
__global__ __launch_bounds__(256) void k_touch_links(const Cfg *__restrict__ cfgs, int ncfg)
{
    double acc = 0.0;
    for (int k = 0; k < ncfg; ++k) {
        const Cfg &C = cfgs[k];
        const size_t n = (size_t)24 * C.V;
        for (int b = 0; b < 2; ++b) {
            const double2 *__restrict__ u = C.U12[b];
            for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
                acc += ld_stream(u + i).x;
        }
    }
    if (!isfinite(acc)) cfgs[0].partials[0] = acc;
}

// Caller's links -> two-row buffer 0 in storage S2 (start of a call).
template <typename S2>
__global__ __launch_bounds__(kSiteBlock) void k_pack_links(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B)
{
    const int blk = blockIdx.x;
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= C.V) return;
    S2 *__restrict__ dst = links12<S2>(C, 0);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 6; ++k) narrow(dst[(size_t)(mu * 6 + k) * C.V + s], C.U[(size_t)(mu * 9 + k) * C.V + s]);
}

// Current two-row buffer in storage S2 -> caller's links, third rows rebuilt
// (end of a call).
template <typename S2>
__global__ __launch_bounds__(kSiteBlock) void k_unpack_links(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B)
{
    const int blk = blockIdx.x;
    const int c = find_cfg(B->off_site, B->n, blk);
    const Cfg &C = cfgs[B->idx[c]];
    const int s = (blk - B->off_site[c]) * kSiteBlock + threadIdx.x;
    if (s >= C.V) return;
    if (C.ctrl->in_caller) return;  // the last update wrote them there
    const S2 *__restrict__ src = links12<S2>(C, C.ctrl->cur);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const M3 m = m3_load12s(src + (size_t)mu * 6 * C.V, C.V, s);
        m3_store(C.U + (size_t)mu * 9 * C.V, C.V, s, m);
    }
}

// Whether the coming iteration of each running configuration projects its links.
__global__ void k_mark_reunit(const Cfg *__restrict__ cfgs, const Batch *__restrict__ B)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B->n) return;
    const Cfg &C = cfgs[B->idx[e]];
    Ctrl *ct = C.ctrl;
    ct->ru_now = C.reunit_every > 0 && ((ct->iter + 1) % (long long)C.reunit_every) == 0;
}

// Start of an iterating call: links in buffer 0 (binary32 storage, copied by
// k_pack_links) or in the caller's array (FP64 storage, read there by the
// first update).
__global__ void k_begin_call(const Cfg *__restrict__ cfgs, int ncfg, int in_caller)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncfg) return;
    Ctrl *ct = cfgs[c].ctrl;
    ct->cur = 0;
    ct->in_caller = in_caller;
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

hipError_t launch_arm_one(const Launch &L, int k, double eps, long long add_iters, int reset_iter)
{
    if (k < 0 || k >= L.ncfg) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, L.stream, L.cfgs + k, 1, eps, add_iters, reset_iter);
    return hipGetLastError();
}

hipError_t launch_delta(const Launch &L, int respect_done, double2 *full_delta)
{
    if (L.fp32)
        hipLaunchKernelGGL(k_delta<float2>, dim3(L.total_march_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, full_delta);
    else
        hipLaunchKernelGGL(k_delta<double2>, dim3(L.total_march_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, full_delta);
    return hipGetLastError();
}

hipError_t launch_reduce(const Launch &L, int ncfg, int count_iter, int respect_done)
{
    hipLaunchKernelGGL(k_reduce, dim3(ncfg), dim3(kReduceLanes), 0, L.stream, L.cfgs, L.batch, count_iter, respect_done,
                       count_iter ? L.fused : 0);
    return hipGetLastError();
}

hipError_t launch_fft_axis(const Launch &L, int axis, int sign, int mode, void *fields_override, int nfields,
                           int respect_done)
{
    if (axis >= 2 && L.total_line[axis - 2] > 0) {
        const dim3 lg(L.total_line[axis - 2] * nfields), lb(256);
        const int lm = L.line_m[axis - 2];  // line lengths present (line_len_bit)
#define GF_LINE_K(T2_, L_, K_)                                                                                    \
    hipLaunchKernelGGL((k_fft_line<T2_, line_lanes(L_), (L_) / line_lanes(L_), K_>), lg, lb, 0, L.stream, L.cfgs, \
                       L.batch, axis, fields_override, nfields, respect_done)
#define GF_LINE_L(T2_, L_)                    \
    if (lm & (1 << line_len_bit(L_))) {       \
        if (mode == 1)                        \
            GF_LINE_K(T2_, L_, 2);            \
        else if (sign < 0)                    \
            GF_LINE_K(T2_, L_, 0);            \
        else                                  \
            GF_LINE_K(T2_, L_, 1);            \
    }
#define GF_LINE(T2_) GF_LINE_L(T2_, 16) GF_LINE_L(T2_, 24) GF_LINE_L(T2_, 32) GF_LINE_L(T2_, 48) GF_LINE_L(T2_, 64)
        if (L.fp32) {
            GF_LINE(float2)
        } else {
            GF_LINE(double2)
        }
#undef GF_LINE
#undef GF_LINE_L
#undef GF_LINE_K
    }
    if (L.total_fft_tiles[axis] == 0) return hipGetLastError();  // every configuration in k_fft_line
    const dim3 grid(L.total_fft_tiles[axis], nfields);
    // power-of-two and general instances, as for the 2D passes
    const size_t sh32 = (size_t)(2 * L.max_lds_elems + 256) * sizeof(float2);
    const size_t sh64 = (size_t)(2 * L.max_lds_elems + 256) * sizeof(double2);
    if (L.fp32) {
        if (L.ax_p2[axis])
            hipLaunchKernelGGL((k_fft<float2, true>), grid, dim3(kFftThreads), sh32, L.stream, L.cfgs, L.batch, axis,
                               sign, mode, fields_override, respect_done, L.max_lds_elems);
        if (L.ax_gen[axis])
            hipLaunchKernelGGL((k_fft<float2, false>), grid, dim3(kFftThreads), sh32, L.stream, L.cfgs, L.batch, axis,
                               sign, mode, fields_override, respect_done, L.max_lds_elems);
    } else {
        if (L.ax_p2[axis])
            hipLaunchKernelGGL((k_fft<double2, true>), grid, dim3(kFftThreads), sh64, L.stream, L.cfgs, L.batch, axis,
                               sign, mode, fields_override, respect_done, L.max_lds_elems);
        if (L.ax_gen[axis])
            hipLaunchKernelGGL((k_fft<double2, false>), grid, dim3(kFftThreads), sh64, L.stream, L.cfgs, L.batch,
                               axis, sign, mode, fields_override, respect_done, L.max_lds_elems);
    }
    return hipGetLastError();
}

// Where the gauge passes put g: 0 full (g), 2 two-row single-precision
// storage (g12f), 3 the filtered fields (fields2) from which the fused pass
// forms g.
static int gauge_store_mode(const Launch &L) { return L.fused ? (L.link_f32 ? 2 : 3) : 0; }

// (tile capacity, work-group size) instances of the 2D passes: 4 or 8
// elements per work-item.
#define GF_2D_SIZES(X, P2) \
    X(1024, 256, P2) X(1024, 128, P2) X(2048, 512, P2) X(2048, 256, P2) X(4096, 1024, P2) X(4096, 512, P2)
#define GF_2D_VARIANTS(X) GF_2D_SIZES(X, true) GF_2D_SIZES(X, false)

// LDS of a 2D tile: CAP elements plus CAP/8 for row padding, then twiddles.
template <typename T2>
static size_t lds2d(int cap, int tw2, int tw_total)
{
    (void)tw2;
    return (size_t)(cap + cap / 8 + tw_total) * sizeof(T2);
}

// Each 2D pass launches the power-of-two instance if some configuration has
// power-of-two extents in that pass, and the general one if some has not;
// each instance leaves the other's configurations at once.
template <typename T2>
static hipError_t run_xy(const Launch &L, int nf, int sign, void *fo, int rd, int fold)
{
    const int fpb = std::max(1, std::min(L.xy_fpb, nf));
    const size_t sh = lds2d<T2>(L.xy_cap, L.xy_tw2, L.xy_tw_total);
    int launched = 0;
    if (!fo && L.xy_reg_any) {  // the iteration's forward pass
        if (sign != -1 || nf != kFields) return hipErrorInvalidValue;
        const int ng = L.xy_reg_groups;
        // one instance per plane size present; the first with at least
        // kReduceLanes work-items carries the fold
#define GF_XYR(L_)                                                                                               \
    if (L.xy_m & (1 << line_len_bit(L_))) {                                                                      \
        const int f = xy_reg_threads<L_>() >= kReduceLanes ? fold : 0;                                           \
        if (f) fold = 0;                                                                                         \
        hipLaunchKernelGGL((k_fft_xy_reg<T2, L_>), dim3(L.total_xy_tiles * ng + (f ? L.ncfg : 0)),               \
                           dim3(xy_reg_threads<L_>()), xy_reg_lds_elems<L_>() * sizeof(T2), L.stream, L.cfgs,     \
                           L.batch, rd, ng, f);                                                                  \
        ++launched;                                                                                              \
    }
        GF_XYR(16) GF_XYR(24) GF_XYR(32) GF_XYR(48) GF_XYR(64)
#undef GF_XYR
        if (!L.xy_lds_any) return hipGetLastError();
    }
    // a batch mixing power-of-two and general extents launches both
    // instances; only the first carries the folded reduction
#define X(C_, T_, P2_)                                                                                            \
    if (L.xy_cap == C_ && L.xy_th == T_ && (P2_ ? L.xy_p2 : L.xy_gen)) {                                          \
        const int f = fold;                                                                                       \
        fold = 0;                                                                                                 \
        const dim3 grid(L.total_xy_tiles + (f ? L.ncfg : 0), (nf + fpb - 1) / fpb);                               \
        hipLaunchKernelGGL((k_fft_xy<T2, C_, T_, P2_>), grid, dim3(T_), sh, L.stream, L.cfgs, L.batch, sign, fo, rd, \
                           L.xy_tw2, nf, fpb, f);                                                                 \
        ++launched;                                                                                               \
    }
    GF_2D_VARIANTS(X)
#undef X
    return launched ? hipGetLastError() : hipErrorInvalidValue;
}

template <typename T2>
static hipError_t run_zt(const Launch &L, int nf, int mode, int sign, void *fo, int rd)
{
    const int fpb = std::max(1, std::min(L.zt_fpb, nf));
    const dim3 grid(L.total_zt_tiles, (nf + fpb - 1) / fpb);
    const size_t sh = lds2d<T2>(L.zt_cap, L.zt_tw2, L.zt_tw_total);
    int launched = 0;
    if (mode == 1 && L.zt_reg_any) {
        const int ng = L.zt_reg_groups;
        const dim3 zg(L.total_zt_tiles * ng);
        // one instance per plane size present (bits line_len_bit)
        if (L.zt_m & (1 << zt_shape_bit(32, 32))) {
            if (L.zt_reg_p == 8)
                hipLaunchKernelGGL((k_fft_zt_reg<T2, 8>), zg, dim3(1024), zt_reg_lds_total<8>() * sizeof(T2), L.stream,
                                   L.cfgs, L.batch, rd, ng);
            else if (L.zt_reg_p == 4)
                hipLaunchKernelGGL((k_fft_zt_reg<T2, 4>), zg, dim3(512), zt_reg_lds_total<4>() * sizeof(T2), L.stream,
                                   L.cfgs, L.batch, rd, ng);
            else
                hipLaunchKernelGGL((k_fft_zt_reg<T2, 2>), zg, dim3(256), zt_reg_lds_total<2>() * sizeof(T2), L.stream,
                                   L.cfgs, L.batch, rd, ng);
        }
#define GF_ZTL(LZ_, LT_, P_)                                                                                   \
    if ((L.zt_m & (1 << zt_shape_bit(LZ_, LT_))) && L.zt_reg_p == (P_))                                         \
        hipLaunchKernelGGL((k_fft_zt_lines<T2, LZ_, LT_, P_>), zg, dim3((zt_lines_threads<LZ_, LT_, P_>())),    \
                           (zt_lines_lds_elems<LZ_, LT_, P_>() * sizeof(T2)), L.stream, L.cfgs, L.batch, rd, ng);
        GF_ZTL(16, 16, 2) GF_ZTL(16, 16, 4) GF_ZTL(16, 16, 8) GF_ZTL(24, 24, 4) GF_ZTL(24, 24, 8)
        GF_ZTL(16, 32, 2) GF_ZTL(16, 32, 4) GF_ZTL(16, 32, 8) GF_ZTL(48, 48, 2)
#undef GF_ZTL
        ++launched;
        if (!L.zt_lds_any) return hipGetLastError();
    }
#define X(C_, T_, P2_)                                                                                            \
    if (L.zt_cap == C_ && L.zt_th == T_ && (P2_ ? L.zt_p2 : L.zt_gen)) {                                          \
        hipLaunchKernelGGL((k_fft_zt<T2, C_, T_, P2_>), grid, dim3(T_), sh, L.stream, L.cfgs, L.batch, mode, sign,   \
                           fo, rd, L.zt_tw2, nf, fpb);                                                            \
        ++launched;                                                                                               \
    }
    GF_2D_VARIANTS(X)
#undef X
    return launched ? hipGetLastError() : hipErrorInvalidValue;
}

template <typename T2>
static hipError_t run_xyg(const Launch &L, int rd, double2 *go)
{
    const size_t sh = lds2d<T2>(L.xy_cap, L.xy_tw2, L.xy_tw_total);
    int launched = 0;
    // the register pass writes the filtered fields (FP64 link storage) or,
    // from the FP32 transform, binary32 g (single-precision storage)
    const int gm = gauge_store_mode(L);
    if (!go && L.xy_reg_any && (gm == 3 || (gm == 2 && std::is_same<T2, float2>::value))) {
#define GF_XYR(L_, S_, NG_)                                                                                        \
    if (L.xy_m & (1 << line_len_bit(L_))) {                                                                        \
        hipLaunchKernelGGL((k_fft_xy_inv_reg<T2, L_, S_>), dim3(L.total_xy_tiles * (NG_)),                         \
                           dim3(xy_reg_threads<L_>()), xy_reg_lds_elems<L_>() * sizeof(T2), L.stream, L.cfgs,       \
                           L.batch, rd, NG_);                                                                      \
        ++launched;                                                                                                \
    }
        if (gm == 3) {
            const int ng = L.xy_reg_groups;
            GF_XYR(16, 3, ng) GF_XYR(24, 3, ng) GF_XYR(32, 3, ng) GF_XYR(48, 3, ng) GF_XYR(64, 3, ng)
        } else if constexpr (std::is_same<T2, float2>::value) {
            GF_XYR(16, 2, 1) GF_XYR(24, 2, 1) GF_XYR(32, 2, 1) GF_XYR(48, 2, 1) GF_XYR(64, 2, 1)
        }
#undef GF_XYR
        if (!L.xy_lds_any) return hipGetLastError();
    }
#define X(C_, T_, P2_)                                                                                            \
    if (L.xy_cap == C_ && L.xy_th == T_ && (P2_ ? L.xy_p2 : L.xy_gen)) {                                          \
        hipLaunchKernelGGL((k_fft_xy_inv_gauge<T2, C_, T_, P2_>), dim3(L.total_xy_tiles), dim3(T_), sh, L.stream,    \
                           L.cfgs, L.batch, rd, go, L.xy_tw2, gauge_store_mode(L));                                           \
        ++launched;                                                                                               \
    }
    GF_2D_VARIANTS(X)
#undef X
    return launched ? hipGetLastError() : hipErrorInvalidValue;
}

// The fold needs a work-group of kReduceLanes work-items: a register xy
// instance of 16-, 32- or 64-point planes (256), or the LDS-staged pass with
// work-groups that large.
bool can_fold_reduce(const Launch &L)
{
    int big = 0;  // register instances of 256 work-items
    if (xy_reg_threads<16>() >= kReduceLanes) big |= 1 << line_len_bit(16);
    if (xy_reg_threads<24>() >= kReduceLanes) big |= 1 << line_len_bit(24);
    if (xy_reg_threads<32>() >= kReduceLanes) big |= 1 << line_len_bit(32);
    if (xy_reg_threads<48>() >= kReduceLanes) big |= 1 << line_len_bit(48);
    if (xy_reg_threads<64>() >= kReduceLanes) big |= 1 << line_len_bit(64);
    const bool reg = L.xy_reg_any && (L.xy_m & big);
    const bool lds = L.xy_lds_any && L.xy_th >= kReduceLanes;
    return reg || lds;
}

hipError_t launch_fft_xy(const Launch &L, int sign, void *fields_override, int nfields, int respect_done,
                         int fold_reduce)
{
    // the folded reduction needs a work-group of at least kReduceLanes
    if (fold_reduce && !can_fold_reduce(L)) return hipErrorInvalidValue;
    const int fold = fold_reduce ? (L.fused ? 2 : 1) : 0;
    return L.fp32 ? run_xy<float2>(L, nfields, sign, fields_override, respect_done, fold)
                  : run_xy<double2>(L, nfields, sign, fields_override, respect_done, fold);
}

hipError_t launch_fft_zt(const Launch &L, int mode, int sign, void *fields_override, int nfields, int respect_done)
{
    return L.fp32 ? run_zt<float2>(L, nfields, mode, sign, fields_override, respect_done)
                  : run_zt<double2>(L, nfields, mode, sign, fields_override, respect_done);
}

hipError_t launch_fft_zt_scale(const Launch &L, int respect_done)
{
    return launch_fft_zt(L, 1, -1, nullptr, kFields, respect_done);
}

hipError_t launch_fft_xy_inv_gauge(const Launch &L, int respect_done, double2 *g_override)
{
    return L.fp32 ? run_xyg<float2>(L, respect_done, g_override) : run_xyg<double2>(L, respect_done, g_override);
}

template <typename T2>
static hipError_t set_lds_t()
{
    const int bytes = (int)lds2d<T2>(4096, 256, 512);
    hipError_t e = hipSuccess;
#define X(C_, T_, P2_)                                                                                          \
    if (e == hipSuccess)                                                                                        \
        e = hipFuncSetAttribute((const void *)k_fft_xy<T2, C_, T_, P2_>,                                        \
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                             \
    if (e == hipSuccess)                                                                                        \
        e = hipFuncSetAttribute((const void *)k_fft_zt<T2, C_, T_, P2_>,                                        \
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                             \
    if (e == hipSuccess)                                                                                        \
        e = hipFuncSetAttribute((const void *)k_fft_xy_inv_gauge<T2, C_, T_, P2_>,                              \
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    GF_2D_VARIANTS(X)
#undef X
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_zt_reg<T2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(zt_reg_lds_total<4>() * sizeof(T2)));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_zt_reg<T2, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(zt_reg_lds_total<8>() * sizeof(T2)));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_zt_lines<T2, 24, 24, 8>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)((zt_lines_lds_elems<24, 24, 8>()) * sizeof(T2)));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_zt_lines<T2, 16, 32, 8>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)((zt_lines_lds_elems<16, 32, 8>()) * sizeof(T2)));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_zt_lines<T2, 48, 48, 2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)((zt_lines_lds_elems<48, 48, 2>()) * sizeof(T2)));
#define GF_XYR(L_)                                                                                              \
    if (e == hipSuccess)                                                                                        \
        e = hipFuncSetAttribute((const void *)k_fft_xy_reg<T2, L_>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)(xy_reg_lds_elems<L_>() * sizeof(T2)));                                    \
    if (e == hipSuccess)                                                                                        \
        e = hipFuncSetAttribute((const void *)k_fft_xy_inv_reg<T2, L_, 3>,                                     \
                                hipFuncAttributeMaxDynamicSharedMemorySize,                                     \
                                (int)(xy_reg_lds_elems<L_>() * sizeof(T2)));                                    \
    if constexpr (std::is_same<T2, float2>::value)                                                              \
        if (e == hipSuccess)                                                                                    \
            e = hipFuncSetAttribute((const void *)k_fft_xy_inv_reg<T2, L_, 2>,                                 \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,                                 \
                                    (int)(xy_reg_lds_elems<L_>() * sizeof(T2)));
    GF_XYR(16) GF_XYR(24) GF_XYR(32) GF_XYR(48) GF_XYR(64)
#undef GF_XYR
    return e;
}

hipError_t set_lds_limits()
{
    hipError_t e = set_lds_t<double2>();
    if (e != hipSuccess) return e;
    return set_lds_t<float2>();
}

hipError_t launch_gauge(const Launch &L, int respect_done, double2 *g_override)
{
    if (L.fp32)
        hipLaunchKernelGGL(k_gauge<float2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, g_override, gauge_store_mode(L));
    else
        hipLaunchKernelGGL(k_gauge<double2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch, respect_done, g_override, gauge_store_mode(L));
    return hipGetLastError();
}

hipError_t launch_update_delta(const Launch &L, int link_io)
{
    const int nb = (L.march_pair == 1 || (L.march_pair == 2 && L.link_f32)) ? 2 : 1;
    const dim3 grid(L.total_march_blocks / nb), blk(kSiteBlock * nb);
    if (L.any_reunit) hipLaunchKernelGGL(k_mark_reunit, dim3((L.ncfg + 63) / 64), dim3(64), 0, L.stream, L.cfgs, L.batch);
#define GF_UPD_NB(T2_, S2_, SRC_, DST_, NB_)                                                                       \
    do {                                                                                                           \
        hipLaunchKernelGGL((k_update_delta_x<T2_, false, S2_, SRC_, DST_, NB_>), grid, blk, 0, L.stream, L.cfgs,   \
                           L.batch);                                                                               \
        if (L.any_reunit)                                                                                          \
            hipLaunchKernelGGL((k_update_delta_x<T2_, true, S2_, SRC_, DST_, NB_>), grid, blk, 0, L.stream, L.cfgs, \
                               L.batch);                                                                           \
    } while (0)
#define GF_UPD(T2_, S2_, SRC_, DST_)               \
    do {                                           \
        if (nb == 2)                               \
            GF_UPD_NB(T2_, S2_, SRC_, DST_, 2);    \
        else                                       \
            GF_UPD_NB(T2_, S2_, SRC_, DST_, 1);    \
    } while (0)
#define GF_UPD_IO(T2_)                                    \
    do {                                                  \
        if (link_io == kLinksFromCaller)                  \
            GF_UPD(T2_, double2, true, false);            \
        else if (link_io == kLinksToCaller)               \
            GF_UPD(T2_, double2, false, true);            \
        else                                              \
            GF_UPD(T2_, double2, false, false);           \
    } while (0)
    if (L.link_f32 && link_io != kLinksBuffers) return hipErrorInvalidValue;
    if (L.fp32) {
        if (L.link_f32)
            GF_UPD(float2, float2, false, false);
        else
            GF_UPD_IO(float2);
    } else {
        if (L.link_f32)
            GF_UPD(double2, float2, false, false);
        else
            GF_UPD_IO(double2);
    }
#undef GF_UPD_IO
#undef GF_UPD
#undef GF_UPD_NB
    return hipGetLastError();
}

hipError_t launch_pack_links(const Launch &L)
{
    hipLaunchKernelGGL(k_begin_call, dim3((L.ncfg + 63) / 64), dim3(64), 0, L.stream, L.cfgs, L.ncfg,
                       L.link_f32 ? 0 : 1);
    if (L.link_f32)
        hipLaunchKernelGGL(k_pack_links<float2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch);
    return hipGetLastError();
}

hipError_t launch_touch_links(const Launch &L)
{
    hipLaunchKernelGGL(k_touch_links, dim3(2048), dim3(256), 0, L.stream, L.cfgs, L.ncfg);
    return hipGetLastError();
}

hipError_t launch_momentum_table(const Launch &L)
{
    if (L.fp32)
        hipLaunchKernelGGL(k_momentum_table<float>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch);
    else
        hipLaunchKernelGGL(k_momentum_table<double>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch);
    return hipGetLastError();
}

hipError_t launch_unpack_links(const Launch &L)
{
    if (L.link_f32)
        hipLaunchKernelGGL(k_unpack_links<float2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch);
    else
        hipLaunchKernelGGL(k_unpack_links<double2>, dim3(L.total_site_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs,
                           L.batch);
    return hipGetLastError();
}

hipError_t launch_update(const Launch &L, int respect_done, const double2 *g_override)
{
    hipLaunchKernelGGL(k_update, dim3(L.total_march_blocks), dim3(kSiteBlock), 0, L.stream, L.cfgs, L.batch,
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

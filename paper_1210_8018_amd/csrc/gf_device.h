// Device helpers: complex arithmetic, 3x3 complex matrices, compensated
// (double-double) sums with wave64 shuffles, lattice indexing, block mapping.
#pragma once

#include <hip/hip_runtime.h>

#define GF_KERNEL_SOURCE
#include "gf_internal.h"

namespace gfk {

// ---------------------------------------------------------------- complex
__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ double2 ccmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double cnorm2(double2 a) { return a.x * a.x + a.y * a.y; }

// Complex multiply-accumulate as four fused multiply-adds: acc + a b,
// acc + a conj(b), acc + conj(a) b.
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc - a b
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 acc)
{
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ double2 cfmac(double2 a, double2 b, double2 acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.y, b.x, acc.y);
    acc.y = fma(-a.x, b.y, acc.y);
    return acc;
}
__device__ __forceinline__ double2 ccfma(double2 a, double2 b, double2 acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}

// ---------------------------------------------------------------- 3x3
struct M3 {
    double2 e[9];
};

__device__ __forceinline__ M3 m3_load(const double2 *__restrict__ base, int V, int s)
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = base[(size_t)k * V + s];
    return m;
}

__device__ __forceinline__ void m3_store(double2 *__restrict__ base, int V, int s, const M3 &m)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) base[(size_t)k * V + s] = m.e[k];
}

// Two-row storage of an SU(3) matrix (the 12-real parametrisation): rows 0
// and 1 in planes 0..5; row 2 is rebuilt as conj(r0 x r1), which holds for
// every special unitary matrix.
__device__ __forceinline__ void m3_row2(M3 &m)
{
    m.e[6] = cconj(cfms(m.e[2], m.e[4], cmul(m.e[1], m.e[5])));
    m.e[7] = cconj(cfms(m.e[0], m.e[5], cmul(m.e[2], m.e[3])));
    m.e[8] = cconj(cfms(m.e[1], m.e[3], cmul(m.e[0], m.e[4])));
}

__device__ __forceinline__ M3 m3_load12(const double2 *__restrict__ base, int V, int s)
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 6; ++k) m.e[k] = base[(size_t)k * V + s];
    m3_row2(m);
    return m;
}

__device__ __forceinline__ void m3_store12(double2 *__restrict__ base, int V, int s, const M3 &m)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) base[(size_t)k * V + s] = m.e[k];
}

// Two-row storage in either precision: S2 = double2 (FP64) or float2 (the
// single-precision storage; entries widened on load, rounded to nearest on
// store). Arithmetic is FP64 in both.
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ void narrow(double2 &d, double2 v) { d = v; }
__device__ __forceinline__ void narrow(float2 &d, double2 v) { d = make_float2((float)v.x, (float)v.y); }

template <typename S2>
__device__ __forceinline__ M3 m3_load12s(const S2 *__restrict__ base, int V, int s)
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 6; ++k) m.e[k] = widen(base[(size_t)k * V + s]);
    m3_row2(m);
    return m;
}

template <typename S2>
__device__ __forceinline__ void m3_store12s(S2 *__restrict__ base, int V, int s, const M3 &m)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) narrow(base[(size_t)k * V + s], m.e[k]);
}

// Streaming (non-temporal) access to elements that a pass reads or writes
// once, so that they do not displace data other work-groups re-read from L2.
typedef double gf_dv2 __attribute__((ext_vector_type(2)));
typedef float gf_fv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    const gf_dv2 v = __builtin_nontemporal_load((const gf_dv2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    const gf_fv2 v = __builtin_nontemporal_load((const gf_fv2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(double2 *p, double2 a)
{
    gf_dv2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, (gf_dv2 *)p);
}
__device__ __forceinline__ void st_stream(float2 *p, float2 a)
{
    gf_fv2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, (gf_fv2 *)p);
}

template <typename S2>
__device__ __forceinline__ M3 m3_load12s_stream(const S2 *__restrict__ base, int V, int s)
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 6; ++k) m.e[k] = widen(ld_stream(base + (size_t)k * V + s));
    m3_row2(m);
    return m;
}

template <typename S2>
__device__ __forceinline__ void m3_store12s_stream(S2 *__restrict__ base, int V, int s, const M3 &m)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        S2 v;
        narrow(v, m.e[k]);
        st_stream(base + (size_t)k * V + s, v);
    }
}

// a b
__device__ __forceinline__ M3 m3_mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 acc = cmul(a.e[i * 3], b.e[j]);
            acc = cfma(a.e[i * 3 + 1], b.e[3 + j], acc);
            c.e[i * 3 + j] = cfma(a.e[i * 3 + 2], b.e[6 + j], acc);
        }
    return c;
}

// a b^dag
__device__ __forceinline__ M3 m3_mul_dag(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 acc = cmulc(a.e[i * 3], b.e[j * 3]);
            acc = cfmac(a.e[i * 3 + 1], b.e[j * 3 + 1], acc);
            c.e[i * 3 + j] = cfmac(a.e[i * 3 + 2], b.e[j * 3 + 2], acc);
        }
    return c;
}

// a^dag b
__device__ __forceinline__ M3 m3_dag_mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 acc = ccmul(a.e[i], b.e[j]);
            acc = ccfma(a.e[3 + i], b.e[3 + j], acc);
            c.e[i * 3 + j] = ccfma(a.e[6 + i], b.e[6 + j], acc);
        }
    return c;
}

__device__ __forceinline__ M3 m3_dag(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.e[i * 3 + j] = cconj(a.e[j * 3 + i]);
    return c;
}

__device__ __forceinline__ M3 m3_add(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.e[k] = cadd(a.e[k], b.e[k]);
    return c;
}

__device__ __forceinline__ M3 m3_scale(const M3 &a, double s)
{
    M3 c;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.e[k] = cscale(a.e[k], s);
    return c;
}

__device__ __forceinline__ M3 m3_zero()
{
    M3 c;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.e[k] = cz();
    return c;
}

__device__ __forceinline__ M3 m3_identity()
{
    M3 c = m3_zero();
    c.e[0].x = c.e[4].x = c.e[8].x = 1.0;
    return c;
}

// Rows 0 and 1 of a b c^dag, row 2 rebuilt as conj(r0 x r1): the product of
// special unitary matrices is special unitary, so this is the full product up
// to rounding, for two thirds of the multiplications.
__device__ __forceinline__ M3 m3_mul_mul_dag_rows(const M3 &a, const M3 &b, const M3 &c)
{
    M3 w;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double2 ab[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            double2 acc = cmul(a.e[i * 3], b.e[l]);
            acc = cfma(a.e[i * 3 + 1], b.e[3 + l], acc);
            ab[l] = cfma(a.e[i * 3 + 2], b.e[6 + l], acc);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 acc = cmulc(ab[0], c.e[j * 3]);
            acc = cfmac(ab[1], c.e[j * 3 + 1], acc);
            w.e[i * 3 + j] = cfmac(ab[2], c.e[j * 3 + 2], acc);
        }
    }
    m3_row2(w);
    return w;
}

// Anti-hermitian part M - M^dag of a 3x3 matrix: the upper off-diagonal
// entries (the lower ones are minus their conjugates) and the imaginary parts
// of the diagonal (its real parts vanish).
struct AH {
    double2 o01, o02, o12;
    double d0, d1, d2;
};

__device__ __forceinline__ AH ah_of(const M3 &m)
{
    AH a;
    a.o01 = csub(m.e[1], cconj(m.e[3]));
    a.o02 = csub(m.e[2], cconj(m.e[6]));
    a.o12 = csub(m.e[5], cconj(m.e[7]));
    a.d0 = 2.0 * m.e[0].y;
    a.d1 = 2.0 * m.e[4].y;
    a.d2 = 2.0 * m.e[8].y;
    return a;
}

__device__ __forceinline__ void ah_acc(AH &a, const AH &b, double sgn)
{
    a.o01 = make_double2(a.o01.x + sgn * b.o01.x, a.o01.y + sgn * b.o01.y);
    a.o02 = make_double2(a.o02.x + sgn * b.o02.x, a.o02.y + sgn * b.o02.y);
    a.o12 = make_double2(a.o12.x + sgn * b.o12.x, a.o12.y + sgn * b.o12.y);
    a.d0 += sgn * b.d0;
    a.d1 += sgn * b.d1;
    a.d2 += sgn * b.d2;
}

// Projection to SU(3) by row Gram-Schmidt; the third row is conj(r0 x r1).
__device__ __forceinline__ void m3_reunit(M3 &m)
{
    double n0 = cnorm2(m.e[0]) + cnorm2(m.e[1]) + cnorm2(m.e[2]);
    double i0 = 1.0 / sqrt(n0);
    m.e[0] = cscale(m.e[0], i0);
    m.e[1] = cscale(m.e[1], i0);
    m.e[2] = cscale(m.e[2], i0);
    // overlap <r0, r1> = sum conj(r0_k) r1_k
    double2 ov = cadd(cadd(ccmul(m.e[0], m.e[3]), ccmul(m.e[1], m.e[4])), ccmul(m.e[2], m.e[5]));
    m.e[3] = csub(m.e[3], cmul(ov, m.e[0]));
    m.e[4] = csub(m.e[4], cmul(ov, m.e[1]));
    m.e[5] = csub(m.e[5], cmul(ov, m.e[2]));
    double n1 = cnorm2(m.e[3]) + cnorm2(m.e[4]) + cnorm2(m.e[5]);
    double i1 = 1.0 / sqrt(n1);
    m.e[3] = cscale(m.e[3], i1);
    m.e[4] = cscale(m.e[4], i1);
    m.e[5] = cscale(m.e[5], i1);
    m3_row2(m);
}

// ---------------------------------------------------------------- sums
struct dd {
    double hi, lo;
};

// error-free transformation s + e = a + b
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    dd r;
    r.hi = s + e;
    r.lo = e - (r.hi - s);
    return r;
}

__device__ __forceinline__ dd dd_shfl_xor(dd v, int m)
{
    dd r;
    r.hi = __shfl_xor(v.hi, m, 64);
    r.lo = __shfl_xor(v.lo, m, 64);
    return r;
}

__device__ __forceinline__ dd wave_sum(dd v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = dd_add(v, dd_shfl_xor(v, m));
    return v;
}

// Deterministic block sum of two double-double values; the result is valid in
// thread 0. `lds` must hold 2 * (blockDim.x / 64) dd entries.
__device__ __forceinline__ void block_sum2(dd &a, dd &b, dd *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        lds[2 * w] = a;
        lds[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dd x = lds[0], y = lds[1];
        for (int k = 1; k < nw; ++k) {
            x = dd_add(x, lds[2 * k]);
            y = dd_add(y, lds[2 * k + 1]);
        }
        a = x;
        b = y;
    }
}

// block_sum2 over each of the NB groups of kSiteBlock work-items of a block
// (waves summed in the same order as a block of kSiteBlock); the result of
// group h is valid in its first work-item. `lds` must hold 2 * (blockDim.x /
// 64) dd entries.
template <int NB>
__device__ __forceinline__ void block_sum2_sets(dd &a, dd &b, dd *lds)
{
    if constexpr (NB == 1) {
        block_sum2(a, b, lds);
    } else {
        constexpr int WPS = kSiteBlock / 64;  // waves per set
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
            lds[2 * w] = a;
            lds[2 * w + 1] = b;
        }
        __syncthreads();
        if (threadIdx.x % kSiteBlock == 0) {
            const int w0 = w;  // first wave of this set
            dd x = lds[2 * w0], y = lds[2 * w0 + 1];
            for (int k = 1; k < WPS; ++k) {
                x = dd_add(x, lds[2 * (w0 + k)]);
                y = dd_add(y, lds[2 * (w0 + k) + 1]);
            }
            a = x;
            b = y;
        }
    }
}

// ---------------------------------------------------------------- integers
__device__ __forceinline__ bool is_p2(int v) { return (v & (v - 1)) == 0; }
__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// Division by an invariant divisor 1 <= d <= 2^20 of numerators
// 0 <= n < 2^31 by a multiply-high, an add and a shift (Granlund and
// Montgomery, PLDI 1994): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (mulhi(m, n) + n) >> l. m is formed by one FP64 division: unless d
// is a power of two (then m = 1 exactly) the exact quotient lies at least
// 1/d from an integer, far more than the 2^-21 rounding error, so the
// truncation is the exact floor.
struct FastDiv {
    uint32_t m;
    int l;
};

__device__ __forceinline__ FastDiv fast_div(int d)
{
    FastDiv f;
    f.l = (d <= 1) ? 0 : 32 - __clz(d - 1);
    const double num = 4294967296.0 * (double)((1 << f.l) - d);
    f.m = (uint32_t)(num / (double)d) + 1u;
    return f;
}

__device__ __forceinline__ int fdiv(int n, FastDiv f)
{
    return (int)((__umulhi(f.m, (uint32_t)n) + (uint32_t)n) >> f.l);
}

// ---------------------------------------------------------------- mapping
// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8).
// Renumber them so each XCD walks a contiguous range of tiles: neighbouring
// sites then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int X = 8;
    const int q = nb / X, r = nb % X;
    const int xcd = b % X, loc = b / X;
    return (xcd < r) ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
}

__device__ __forceinline__ int find_cfg(const int *off, int n, int blk)
{
    int c = 0;
    while (c + 1 < n && blk >= off[c + 1]) ++c;
    return c;
}

// (x, y, z) of work-item `tid` of block `b3` of the marching kernels, and
// whether it is inside the volume. Linear mode: kSiteBlock consecutive sites
// of the (x, y, z) volume; tile mode: a tile[0] x tile[1] x tile[2] box.
__device__ __forceinline__ bool march_xyz(const Cfg &C, int b3, int tid, int &x, int &y, int &z)
{
    const int Lx = C.dims[0], Ly = C.dims[1], Lz = C.dims[2];
    if (C.tile[0] == 0) {
        const int s3 = b3 * kSiteBlock + tid;
        x = s3 % Lx;
        const int r = s3 / Lx;
        y = r % Ly;
        z = r / Ly;
        return s3 < C.V3;
    }
    const int tx = C.tile[0], ty = C.tile[1];
    const int bx = b3 % C.ntile[0], rb = b3 / C.ntile[0];
    const int by = rb % C.ntile[1], bz = rb / C.ntile[1];
    const int ix = tid % tx, rt = tid / tx;
    const int iy = rt % ty, iz = rt / ty;
    x = bx * tx + ix;
    y = by * ty + iy;
    z = bz * C.tile[2] + iz;
    return iz < C.tile[2] && x < Lx && y < Ly && z < Lz;
}

struct Site {
    int s;
    int c[4];
};

__device__ __forceinline__ void site_coords(const int *dims, int s, int c[4])
{
    int r = s;
    c[0] = r % dims[0];
    r /= dims[0];
    c[1] = r % dims[1];
    r /= dims[1];
    c[2] = r % dims[2];
    c[3] = r / dims[2];
}

}  // namespace gfk

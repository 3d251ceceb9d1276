// Input generator on the GPU: thermalised SU(3) configurations of the Wilson
// action S = beta sum_P (1 - Re Tr U_P / 3), the kind of configuration the
// paper gauge-fixes (section 3, beta = 5.8 to 6.2). Cabibbo-Marinari
// pseudo-heatbath over the SU(2) subgroups (0,1), (0,2), (1,2) with
// Kennedy-Pendleton draws, microcanonical overrelaxation, Philox4x32-10
// random numbers with one counter per draw (Salmon et al., SC 2011). The
// draw-to-counter assignment and the order of updates follow one published
// definition so that a CPU implementation reproduces the same configuration.
// Also the average plaquette.
#include <hip/hip_runtime.h>

#include "gf_device.h"
#include "gf_internal.h"

namespace gfk {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr int kHbMaxAttempts = 64;  // Kennedy-Pendleton attempts per draw
constexpr int kHbDirectionSlot = 255;

struct U4 {
    uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint32_t hi1 = __umulhi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// A 32-bit draw as a uniform number in (0, 1].
__device__ __forceinline__ double unit_open0(uint32_t u) { return ((double)u + 1.0) * (1.0 / 4294967296.0); }

// Draw `slot` (attempt j, or the direction) of subgroup k of the update of
// U_mu(site) in heatbath sweep n: counter (site, mu + 4k + 16 slot, n lo, n hi).
__device__ __forceinline__ U4 hb_draw(int site, int mu, int k, int slot, long long n, uint32_t k0, uint32_t k1)
{
    return philox4x32_10((uint32_t)site, (uint32_t)(mu + 4 * k + 16 * slot),
                         (uint32_t)((unsigned long long)n & 0xffffffffull), (uint32_t)((unsigned long long)n >> 32),
                         k0, k1);
}

constexpr double kTwoPi = 6.28318530717958647692;

// x in SU(2) with density exp(a x0) (Haar measure): x0 by Kennedy-Pendleton
// rejection from sqrt(1 - x0^2) e^(a x0), the vector part uniform on its
// sphere. false if no attempt is accepted within the cap (x untouched).
__device__ bool kp_draw(double a, int site, int mu, int k, long long n, uint32_t k0, uint32_t k1, double x[4])
{
    for (int j = 0; j < kHbMaxAttempts; ++j) {
        const U4 r = hb_draw(site, mu, k, j, n, k0, k1);
        const double r1 = unit_open0(r.v[0]), r2 = unit_open0(r.v[1]), r3 = unit_open0(r.v[2]),
                     r4 = unit_open0(r.v[3]);
        const double c = cos(kTwoPi * r2);
        const double lam2 = -(log(r1) + c * c * log(r3)) / (2.0 * a);
        if (r4 * r4 <= 1.0 - lam2) {
            x[0] = 1.0 - 2.0 * lam2;
            const U4 d = hb_draw(site, mu, k, kHbDirectionSlot, n, k0, k1);
            const double ct = 2.0 * unit_open0(d.v[0]) - 1.0, phi = kTwoPi * unit_open0(d.v[1]);
            const double rad = sqrt(fmax(0.0, 1.0 - x[0] * x[0]));
            const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
            x[1] = rad * st * cos(phi);
            x[2] = rad * st * sin(phi);
            x[3] = rad * ct;
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ int hop(const int *L, const int c[4], int s, int mu, int step, const int *stride)
{
    const int x = c[mu] + step;
    if (x < 0) return s + (L[mu] - 1) * stride[mu];
    if (x >= L[mu]) return s - (L[mu] - 1) * stride[mu];
    return s + step * stride[mu];
}

// Staple sum A of U_mu(s): U_mu(s) A is the sum of the six plaquettes through
// it (upper U_nu(s+mu) U_mu^dag(s+nu) U_nu^dag(s), lower U_nu^dag(s+mu-nu)
// U_mu^dag(s-nu) U_nu(s-nu), nu ascending).
__device__ M3 staple_sum(const Cfg &C, int s, const int c[4], int mu)
{
    const int V = C.V;
    const int stride[4] = {1, C.dims[0], C.V2, C.V3};
    const double2 *__restrict__ U = C.U;
    M3 A = m3_zero();
    int cp[4] = {c[0], c[1], c[2], c[3]};
    cp[mu] = (c[mu] + 1 == C.dims[mu]) ? 0 : c[mu] + 1;
    const int sp = hop(C.dims, c, s, mu, +1, stride);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        {
            const M3 a = m3_load(U + (size_t)nu * 9 * V, V, sp);
            const M3 b = m3_load(U + (size_t)mu * 9 * V, V, hop(C.dims, c, s, nu, +1, stride));
            const M3 cc = m3_load(U + (size_t)nu * 9 * V, V, s);
            A = m3_add(A, m3_mul_dag(m3_mul_dag(a, b), cc));
        }
        {
            const int sm = hop(C.dims, c, s, nu, -1, stride);
            const M3 a = m3_load(U + (size_t)nu * 9 * V, V, hop(C.dims, cp, sp, nu, -1, stride));
            const M3 b = m3_load(U + (size_t)mu * 9 * V, V, sm);
            const M3 cc = m3_load(U + (size_t)nu * 9 * V, V, sm);
            A = m3_add(A, m3_mul(m3_mul(m3_dag(a), m3_dag(b)), cc));
        }
    }
    return A;
}

// One Cabibbo-Marinari update of u against staple sum A: for each subgroup
// (p, q), the part of the 2x2 block of u A proportional to SU(2) is
// nk V (V in SU(2)); u <- r u with r = X V^dag, X drawn with density
// exp((2 beta / 3) nk x0) (mode 0, heatbath), or r = V^dag V^dag (mode 1,
// overrelaxation, which keeps Re Tr(u A)). Then Gram-Schmidt.
__device__ void cm_update(M3 &u, const M3 &A, double beta, int mode, int site, int mu, long long n, uint32_t k0,
                          uint32_t k1)
{
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int p = sub[k][0], q = sub[k][1];
        const M3 W = m3_mul(u, A);
        const double2 al = cscale(cadd(W.e[p * 3 + p], cconj(W.e[q * 3 + q])), 0.5);
        const double2 be = cscale(csub(W.e[p * 3 + q], cconj(W.e[q * 3 + p])), 0.5);
        const double det = al.x * al.x + al.y * al.y + be.x * be.x + be.y * be.y;
        if (!(det > 1e-300)) continue;
        const double nk = sqrt(det);
        const double2 v00 = make_double2(al.x / nk, al.y / nk), v01 = make_double2(be.x / nk, be.y / nk);
        // V^dag
        const double2 d00 = cconj(v00), d01 = make_double2(-v01.x, -v01.y), d10 = cconj(v01), d11 = v00;
        double2 r00, r01, r10, r11;
        if (mode == 0) {
            double x[4];
            if (!kp_draw(2.0 * beta / 3.0 * nk, site, mu, k, n, k0, k1, x)) continue;
            const double2 x00 = make_double2(x[0], x[3]), x01 = make_double2(x[2], x[1]);
            const double2 x10 = make_double2(-x[2], x[1]), x11 = make_double2(x[0], -x[3]);
            r00 = cadd(cmul(x00, d00), cmul(x01, d10));
            r01 = cadd(cmul(x00, d01), cmul(x01, d11));
            r10 = cadd(cmul(x10, d00), cmul(x11, d10));
            r11 = cadd(cmul(x10, d01), cmul(x11, d11));
        } else {
            r00 = cadd(cmul(d00, d00), cmul(d01, d10));
            r01 = cadd(cmul(d00, d01), cmul(d01, d11));
            r10 = cadd(cmul(d10, d00), cmul(d11, d10));
            r11 = cadd(cmul(d10, d01), cmul(d11, d11));
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double2 up = u.e[p * 3 + j], uq = u.e[q * 3 + j];
            u.e[p * 3 + j] = cadd(cmul(r00, up), cmul(r01, uq));
            u.e[q * 3 + j] = cadd(cmul(r10, up), cmul(r11, uq));
        }
    }
    m3_reunit(u);
}

// Updates every U_mu(s) with x + y + z + t = parity (mod 2); these links are
// independent (their staples hold only other directions and other-parity
// sites). Work-item i takes the i-th such site in lexicographic order
// (Lx even: half of every x-row).
__global__ __launch_bounds__(kSiteBlock) void k_heatbath(const Cfg *__restrict__ cfgs, int mu, int parity, int mode,
                                                         double beta, uint32_t k0, uint32_t k1, long long n)
{
    const Cfg &C = cfgs[0];
    const int half = C.dims[0] / 2;
    const int i = blockIdx.x * kSiteBlock + threadIdx.x;
    if (i >= C.V / 2) return;
    const int row = i / half, xh = i % half;
    int c[4];
    c[1] = row % C.dims[1];
    c[2] = (row / C.dims[1]) % C.dims[2];
    c[3] = row / (C.dims[1] * C.dims[2]);
    c[0] = 2 * xh + ((c[1] + c[2] + c[3] + parity) & 1);
    const int s = c[0] + C.dims[0] * row;
    const M3 A = staple_sum(C, s, c, mu);
    double2 *__restrict__ Um = C.U + (size_t)mu * 9 * C.V;
    M3 u = m3_load(Um, C.V, s);
    cm_update(u, A, beta, mode, s, mu, n, k0, k1);
    m3_store(Um, C.V, s, u);
}

// Per-block compensated sums of the six plaquettes Re Tr U_P of each site,
// into partials[4 b], partials[4 b + 1] (the layout k_sum_partials reads).
__global__ __launch_bounds__(kSiteBlock) void k_plaquette(const Cfg *__restrict__ cfgs)
{
    __shared__ dd red[2 * (kSiteBlock / 64)];
    const Cfg &C = cfgs[0];
    const int V = C.V;
    const int s = blockIdx.x * kSiteBlock + threadIdx.x;
    double acc = 0.0;
    if (s < V) {
        int c[4];
        site_coords(C.dims, s, c);
        const int stride[4] = {1, C.dims[0], C.V2, C.V3};
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                const M3 a = m3_load(C.U + (size_t)mu * 9 * V, V, s);
                const M3 b = m3_load(C.U + (size_t)nu * 9 * V, V, hop(C.dims, c, s, mu, +1, stride));
                const M3 cc = m3_load(C.U + (size_t)mu * 9 * V, V, hop(C.dims, c, s, nu, +1, stride));
                const M3 d = m3_load(C.U + (size_t)nu * 9 * V, V, s);
                const M3 p = m3_mul_dag(m3_mul_dag(m3_mul(a, b), cc), d);
                acc += p.e[0].x + p.e[4].x + p.e[8].x;
            }
    }
    dd a = {acc, 0.0}, b = {0.0, 0.0};
    block_sum2(a, b, red);
    if (threadIdx.x == 0) {
        double *p = C.partials + (size_t)blockIdx.x * 4;
        p[0] = a.hi;
        p[1] = a.lo;
    }
}

__global__ __launch_bounds__(256) void k_sum_plaquette(const Cfg *__restrict__ cfgs, double *__restrict__ out)
{
    __shared__ dd red[2 * (256 / 64)];
    const Cfg &C = cfgs[0];
    dd f = {0.0, 0.0}, z = {0.0, 0.0};
    for (int i = threadIdx.x; i < C.nblk_site; i += blockDim.x) {
        const double *p = C.partials + (size_t)i * 4;
        f = dd_add(f, dd{p[0], p[1]});
    }
    block_sum2(f, z, red);
    if (threadIdx.x == 0) *out = (f.hi + f.lo) / (18.0 * (double)C.V);
}

}  // namespace

hipError_t launch_heatbath_sweep(const Launch &L, int V, int mode, double beta, uint64_t seed, long long n)
{
    const dim3 grid((V / 2 + kSiteBlock - 1) / kSiteBlock);
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffull), k1 = (uint32_t)(seed >> 32);
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par)
            hipLaunchKernelGGL(k_heatbath, grid, dim3(kSiteBlock), 0, L.stream, L.cfgs, mu, par, mode, beta, k0, k1,
                               n);
    return hipGetLastError();
}

hipError_t launch_plaquette(const Launch &L, int nblk, double *out)
{
    hipLaunchKernelGGL(k_plaquette, dim3(nblk), dim3(kSiteBlock), 0, L.stream, L.cfgs);
    hipLaunchKernelGGL(k_sum_plaquette, dim3(1), dim3(256), 0, L.stream, L.cfgs, out);
    return hipGetLastError();
}

}  // namespace gfk

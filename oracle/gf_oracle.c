/*
 * CPU oracle for Fourier-accelerated steepest-descent Landau gauge fixing of
 * 4D SU(3) lattice gauge fields (Cardoso, Silva, Oliveira, Bicudo, "GPU
 * implementation of a Landau gauge fixing algorithm", Lattice 2012).
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, obviously correct
 * FP64 statement of what the method computes. Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no code,
 * header, table or constant with the HIP library.
 *
 * Conventions (the paper uses a lexicographic layout, section 2.1):
 *   dims L[4] = (Lx, Ly, Lz, Lt), V = Lx*Ly*Lz*Lt, periodic boundaries;
 *   site s = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 is x, y, z, t;
 *   links U[((mu*3 + i)*3 + j)*V + s] (complex double), U_mu(x) joins x to x+mu;
 *   fields of matrices M[(i*3 + j)*V + s];
 *   Lie-algebra parameters omega[a*V + s], a = 0..7 (Gell-Mann, Tr l_a l_b = 2 d_ab).
 *
 * Readings of points the paper leaves open (each is used consistently here):
 *   - alpha/2 and the 1/V of the inverse transform are folded into one factor
 *     K(p) = (alpha/2) p2max/p2 / V (Eq. 2 and the "normalize" step of Alg. 1);
 *   - p2 = sum_mu 4 sin^2(pi n_mu / L_mu), the eigenvalues of the lattice
 *     Laplacian -d^2 (text under Eq. 3); p2max is their maximum on the grid;
 *   - the zero mode p = 0 is removed, K(0) = 0;
 *   - forward transform exp(-i p.x) unnormalised, backward exp(+i p.x);
 *   - Delta = (D - D^dag) - Tr(D - D^dag)/3, D = sum_nu [U_nu(x-nu) - U_nu(x)]
 *     (Eq. 2, Eq. 3, Eq. 5: "h.c." and "trace" subtracted);
 *   - "first order in alpha then reunitarize": g = 1 + Delta~, projected to
 *     SU(3) by row Gram-Schmidt with the third row conj(r1 x r2);
 *   - all g are formed before any link changes (the two loops of Alg. 1);
 *   - iteration stops once theta <= eps, tested after every update;
 *   - optional link reunitarisation every R iterations (R = 0: never).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef cplx mat3[3][3];

/* ------------------------------------------------------------------------ */
/* lattice indexing                                                          */
/* ------------------------------------------------------------------------ */

static int64_t vol(const int L[4]) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int L[4], int64_t s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static int64_t index_of(const int L[4], const int c[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/* site s moved by `step` (+1 or -1) along mu, periodic */
static int64_t hop(const int L[4], int64_t s, int mu, int step)
{
    int c[4];
    coords(L, s, c);
    c[mu] = (c[mu] + step + L[mu]) % L[mu];
    return index_of(L, c);
}

/* ------------------------------------------------------------------------ */
/* 3x3 complex matrices                                                      */
/* ------------------------------------------------------------------------ */

static void get_link(const cplx *U, int64_t V, int mu, int64_t s, mat3 m)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = U[((int64_t)(mu * 3 + i) * 3 + j) * V + s];
}

static void put_link(cplx *U, int64_t V, int mu, int64_t s, mat3 m)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) U[((int64_t)(mu * 3 + i) * 3 + j) * V + s] = m[i][j];
}

static void get_site(const cplx *M, int64_t V, int64_t s, mat3 m) { get_link(M, V, 0, s, m); }
static void put_site(cplx *M, int64_t V, int64_t s, mat3 m) { put_link(M, V, 0, s, m); }

static void mat_mul(mat3 a, mat3 b, mat3 c) /* c = a b */
{
    mat3 t;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 3; ++k) acc += a[i][k] * b[k][j];
            t[i][j] = acc;
        }
    memcpy(c, t, sizeof(mat3));
}

static void mat_dag(mat3 a, mat3 b) /* b = a^dagger */
{
    mat3 t;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[i][j] = conj(a[j][i]);
    memcpy(b, t, sizeof(mat3));
}

static cplx mat_trace(mat3 a) { return a[0][0] + a[1][1] + a[2][2]; }

/* ------------------------------------------------------------------------ */
/* compensated (Neumaier) summation, serial and in index order               */
/* ------------------------------------------------------------------------ */

static double neumaier(const double *v, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double t = s + v[k];
        if (fabs(s) >= fabs(v[k]))
            c += (s - t) + v[k];
        else
            c += (v[k] - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------ */
/* Eq. 5: lattice divergence Delta(x)                                        */
/* ------------------------------------------------------------------------ */

static void delta_at(const int L[4], const cplx *U, int64_t s, mat3 out)
{
    const int64_t V = vol(L);
    mat3 D = {{0}};
    for (int nu = 0; nu < 4; ++nu) {
        mat3 back, here;
        get_link(U, V, nu, hop(L, s, nu, -1), back); /* U_nu(x - nu) */
        get_link(U, V, nu, s, here);                 /* U_nu(x)      */
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[i][j] += back[i][j] - here[i][j];
    }
    mat3 A;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = D[i][j] - conj(D[j][i]); /* minus h.c. */
    cplx tr = mat_trace(A) / 3.0;                                      /* minus trace */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[i][j] = A[i][j] - (i == j ? tr : 0.0);
}

/* Delta[(i*3+j)*V + s] for every site (Eq. 5). */
void or_delta(const int L[4], const cplx *U, cplx *Delta)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        mat3 d;
        delta_at(L, U, s, d);
        put_site(Delta, V, s, d);
    }
}

/*
 * F at g = 1 (Eq. 1 with N_c = 3) and theta (Eq. 4) of the current links:
 *   F     = (1/(12 V)) sum_x sum_mu Re Tr U_mu(x)
 *   theta = (1/(3 V))  sum_x Tr[Delta(x) Delta(x)^dag] = (1/(3V)) sum |Delta_ij|^2
 * Per-site terms are summed serially in site order with Neumaier compensation.
 */
void or_measure(const int L[4], const cplx *U, double *F, double *theta)
{
    const int64_t V = vol(L);
    double *f = malloc(sizeof(double) * V);
    double *t = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            mat3 u;
            get_link(U, V, mu, s, u);
            acc += creal(mat_trace(u));
        }
        f[s] = acc;
        mat3 d;
        delta_at(L, U, s, d);
        double q = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) q += creal(d[i][j]) * creal(d[i][j]) + cimag(d[i][j]) * cimag(d[i][j]);
        t[s] = q;
    }
    *F = neumaier(f, V) / (12.0 * (double)V);
    *theta = neumaier(t, V) / (3.0 * (double)V);
    free(f);
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Fourier transform (Alg. 1: "apply FFT forward/backward" per element)       */
/* ------------------------------------------------------------------------ */

/* exp(sign * 2 pi i e / n) */
static cplx root_of_unity(int n, int64_t e, int sign)
{
    e %= n;
    if (e < 0) e += n;
    double a = 2.0 * M_PI * (double)e / (double)n;
    return cos(a) + (double)sign * sin(a) * I;
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/*
 * out[k] = sum_{j<n} in[j*stride] exp(sign 2 pi i j k / n), k < n.
 * Textbook recursive decimation-in-time Cooley-Tukey: with p the smallest
 * prime factor of n and m = n/p, the p sub-sequences in[(r + p j) stride]
 * are transformed (length m) into out[r*m .. r*m+m-1], then
 *   X[k + q m] = sum_r w_n^{r (k + q m)} S_r[k],   k < m, q < p.
 * A prime length is a direct DFT (p = n, m = 1).
 * roots[e] = exp(sign 2 pi i e / N) for the full length N of the top-level
 * call; w_n^e = roots[(e mod n) * (N / n)] since n divides N.
 */
static void dft_rec(const cplx *in, int64_t stride, cplx *out, int n, int sign, const cplx *roots, int N)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int p = smallest_factor(n);
    const int m = n / p;
    for (int r = 0; r < p; ++r) dft_rec(in + r * stride, stride * p, out + (int64_t)r * m, m, sign, roots, N);
    cplx tmp[64];
    cplx *t = p <= 64 ? tmp : malloc(sizeof(cplx) * p);
    const int step = N / n;
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r) t[r] = out[(int64_t)r * m + k];
        for (int q = 0; q < p; ++q) {
            cplx acc = 0;
            for (int r = 0; r < p; ++r) acc += roots[(((int64_t)r * (k + (int64_t)q * m)) % n) * step] * t[r];
            out[k + (int64_t)q * m] = acc;
        }
    }
    if (t != tmp) free(t);
}

/*
 * Order in which or_fft4d takes the axes (default x, y, z, t). The separable
 * transform is the same in exact arithmetic for every order; another order
 * only rounds differently. Test infrastructure uses it to size the spread
 * between two correct FP64 runs of Alg. 1 (the tolerance of theta at its
 * rounding floor). Not thread-safe; a permutation of 0..3 or ignored.
 */
static int fft_axis_order[4] = {0, 1, 2, 3};

void or_set_fft_axis_order(const int order[4])
{
    int seen = 0;
    for (int a = 0; a < 4; ++a) {
        if (order[a] < 0 || order[a] > 3) return;
        seen |= 1 << order[a];
    }
    if (seen != 15) return;
    for (int a = 0; a < 4; ++a) fft_axis_order[a] = order[a];
}

/* In-place unnormalised 4D transform of one complex field f[s], sign -1 (forward) or +1. */
void or_fft4d(const int L[4], cplx *f, int sign)
{
    const int64_t V = vol(L);
    for (int a = 0; a < 4; ++a) {
        const int mu = fft_axis_order[a];
        int64_t stride = 1; /* distance between consecutive elements along mu */
        for (int nu = 0; nu < mu; ++nu) stride *= L[nu];
        const int n = L[mu];
        const int64_t inner = stride, outer = V / (stride * n);
        const int64_t pencils = inner * outer;
        cplx *roots = malloc(sizeof(cplx) * n);
        for (int e = 0; e < n; ++e) roots[e] = root_of_unity(n, e, sign);
#pragma omp parallel
        {
            cplx *buf = malloc(sizeof(cplx) * n);
            cplx *res = malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
            for (int64_t pcl = 0; pcl < pencils; ++pcl) {
                const int64_t i0 = pcl % inner, o = pcl / inner;
                const int64_t base = o * inner * n + i0;
                for (int k = 0; k < n; ++k) buf[k] = f[base + k * inner];
                dft_rec(buf, 1, res, n, sign, roots, n);
                for (int k = 0; k < n; ++k) f[base + k * inner] = res[k];
            }
            free(buf);
            free(res);
        }
        free(roots);
    }
}

/*
 * k1 of the paper: K(p) = (alpha/2) * p2max / p2 / V, K(0) = 0, indexed by the
 * momentum site n = (n_x, n_y, n_z, n_t) in the same lexicographic order.
 */
void or_momentum_factor(const int L[4], double alpha, double *K)
{
    const int64_t V = vol(L);
    double p2max = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
        double best = 0.0;
        for (int n = 0; n < L[mu]; ++n) {
            double sn = sin(M_PI * n / L[mu]);
            if (4.0 * sn * sn > best) best = 4.0 * sn * sn;
        }
        p2max += best;
    }
    for (int64_t s = 0; s < V; ++s) {
        int c[4];
        coords(L, s, c);
        double p2 = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            double sn = sin(M_PI * c[mu] / L[mu]);
            p2 += 4.0 * sn * sn;
        }
        K[s] = (s == 0) ? 0.0 : 0.5 * alpha * p2max / p2 / (double)V;
    }
}

/* ------------------------------------------------------------------------ */
/* projection to SU(3) ("reunitarize")                                       */
/* ------------------------------------------------------------------------ */

/* Row Gram-Schmidt: r1 <- r1/|r1|; r2 <- r2 - (r1^* . r2) r1, r2 <- r2/|r2|; r3 = conj(r1 x r2). */
void or_reunit(cplx *m9)
{
    cplx (*m)[3] = (cplx(*)[3])m9;
    double n1 = 0.0;
    for (int k = 0; k < 3; ++k) n1 += creal(m[0][k] * conj(m[0][k]));
    n1 = sqrt(n1);
    for (int k = 0; k < 3; ++k) m[0][k] /= n1;
    cplx ov = 0;
    for (int k = 0; k < 3; ++k) ov += conj(m[0][k]) * m[1][k];
    for (int k = 0; k < 3; ++k) m[1][k] -= ov * m[0][k];
    double n2 = 0.0;
    for (int k = 0; k < 3; ++k) n2 += creal(m[1][k] * conj(m[1][k]));
    n2 = sqrt(n2);
    for (int k = 0; k < 3; ++k) m[1][k] /= n2;
    m[2][0] = conj(m[0][1] * m[1][2] - m[0][2] * m[1][1]);
    m[2][1] = conj(m[0][2] * m[1][0] - m[0][0] * m[1][2]);
    m[2][2] = conj(m[0][0] * m[1][1] - m[0][1] * m[1][0]);
}

/* ------------------------------------------------------------------------ */
/* one gauge transformation of Alg. 1                                         */
/* ------------------------------------------------------------------------ */

/*
 * From Delta (as written by or_delta) build g (Eq. 2 to first order, then
 * projection): each of the nine elements Delta_ij(x) is transformed forward,
 * multiplied by K(p), transformed backward (K carries the 1/V normalisation);
 * then g(x) = 1 + Delta~(x), reunitarised.
 */
void or_gauge_from_delta(const int L[4], const cplx *Delta, double alpha, cplx *g)
{
    const int64_t V = vol(L);
    double *K = malloc(sizeof(double) * V);
    or_momentum_factor(L, alpha, K);
    memcpy(g, Delta, sizeof(cplx) * 9 * V);
    for (int e = 0; e < 9; ++e) {
        cplx *f = g + (int64_t)e * V;
        or_fft4d(L, f, -1);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < V; ++s) f[s] *= K[s];
        or_fft4d(L, f, +1);
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        mat3 m;
        get_site(g, V, s, m);
        for (int i = 0; i < 3; ++i) m[i][i] += 1.0;
        or_reunit(&m[0][0]);
        put_site(g, V, s, m);
    }
    free(K);
}

/* U_mu(x) <- g(x) U_mu(x) g^dagger(x + mu) for all x and mu (Alg. 1, second loop). */
void or_apply_gauge(const int L[4], cplx *U, const cplx *g)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        mat3 gx;
        get_site(g, V, s, gx);
        for (int mu = 0; mu < 4; ++mu) {
            mat3 u, gf, gfd;
            get_link(U, V, mu, s, u);
            get_site(g, V, hop(L, s, mu, +1), gf);
            mat_dag(gf, gfd);
            mat_mul(gx, u, u);
            mat_mul(u, gfd, u);
            put_link(U, V, mu, s, u);
        }
    }
}

/* Gram-Schmidt every link (the optional drift control). */
void or_reunit_links(const int L[4], cplx *U)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            mat3 u;
            get_link(U, V, mu, s, u);
            or_reunit(&u[0][0]);
            put_link(U, V, mu, s, u);
        }
}

/*
 * Single-precision storage of the 12-real representation of an SU(3) matrix
 * (section 2.2; the paper's single-precision mode stores its links this
 * way): the real and imaginary parts of rows 0 and 1 are rounded to the
 * nearest binary32 value, row 2 is rebuilt in FP64 as conj(r0 x r1).
 * Applied in place to nmat matrix fields [nmat][3][3][V].
 */
static void two_row_field(const int L[4], cplx *M, int nmat, int round_f32)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < nmat; ++mu) {
            mat3 m;
            get_link(M, V, mu, s, m);
            if (round_f32)
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 3; ++j) {
                        const float re = (float)creal(m[i][j]), im = (float)cimag(m[i][j]);
                        m[i][j] = (double)re + I * (double)im;
                    }
            m[2][0] = conj(m[0][1] * m[1][2] - m[0][2] * m[1][1]);
            m[2][1] = conj(m[0][2] * m[1][0] - m[0][0] * m[1][2]);
            m[2][2] = conj(m[0][0] * m[1][1] - m[0][1] * m[1][0]);
            put_link(M, V, mu, s, m);
        }
}

void or_store_f32(const int L[4], cplx *M, int nmat) { two_row_field(L, M, nmat, 1); }

/*
 * Alg. 1. Computes Delta, F, theta; then while theta > eps and fewer than
 * max_iter updates were made: gauge vector from Delta, link update,
 * (optional link reunitarisation when reunit_every > 0 and the update count
 * is a multiple of it), recompute Delta, F, theta.
 * F_hist[k], theta_hist[k] (k <= min(updates, hist_cap-1)) hold the values
 * after k updates (k = 0: the input). Returns the number of updates made.
 * eps < 0 runs exactly max_iter updates.
 */
/*
 * Alg. 1 with single-precision storage of links and g (or_store_f32): the
 * arithmetic stays FP64, every g is stored before it is applied, every new
 * link is stored after its update (and projection), and Delta, F, theta of an
 * iteration are those of the new links before their storage. A link of this
 * representation is its two rows (section 2.2): the third row of a new link
 * is rebuilt from its two computed rows before it is used, which matters
 * here because stored matrices are special unitary only to the binary32
 * rounding. The starting Delta is that of the input links, which are then
 * stored. On return U holds the stored links. Histories and return value as
 * or_fix.
 */
static int64_t fix_two_row(const int L[4], cplx *U, double alpha, double eps, int64_t max_iter, int reunit_every,
                           double *F_hist, double *theta_hist, int64_t hist_cap, int round_f32);

int64_t or_fix_f32_storage(const int L[4], cplx *U, double alpha, double eps, int64_t max_iter, int reunit_every,
                           double *F_hist, double *theta_hist, int64_t hist_cap)
{
    return fix_two_row(L, U, alpha, eps, max_iter, reunit_every, F_hist, theta_hist, hist_cap, 1);
}

/*
 * Alg. 1 with the 12-real representation of section 2.2 kept in FP64: as
 * or_fix_f32_storage without the binary32 rounding (every stored link and g
 * is its two rows, the third rebuilt as conj(r0 x r1)). Equal to or_fix in
 * exact arithmetic for special unitary links; it rounds differently (each
 * rebuilt row differs from the full product's by O(1e-16)), which sizes the
 * spread of theta at its rounding floor between two correct FP64 codes that
 * store links in the paper's two forms.
 */
int64_t or_fix_two_row(const int L[4], cplx *U, double alpha, double eps, int64_t max_iter, int reunit_every,
                       double *F_hist, double *theta_hist, int64_t hist_cap)
{
    return fix_two_row(L, U, alpha, eps, max_iter, reunit_every, F_hist, theta_hist, hist_cap, 0);
}

static int64_t fix_two_row(const int L[4], cplx *U, double alpha, double eps, int64_t max_iter, int reunit_every,
                           double *F_hist, double *theta_hist, int64_t hist_cap, int round_f32)
{
    const int64_t V = vol(L);
    cplx *Delta = malloc(sizeof(cplx) * 9 * V);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    cplx *Ux = malloc(sizeof(cplx) * 36 * V); /* new links before storage */
    double F, theta;
    memcpy(Ux, U, sizeof(cplx) * 36 * V);
    or_measure(L, Ux, &F, &theta);
    two_row_field(L, U, 4, round_f32);
    if (hist_cap > 0) {
        F_hist[0] = F;
        theta_hist[0] = theta;
    }
    int64_t it = 0;
    while (!(theta <= eps) && it < max_iter) {
        or_delta(L, Ux, Delta);
        or_gauge_from_delta(L, Delta, alpha, g);
        two_row_field(L, g, 1, round_f32);
        memcpy(Ux, U, sizeof(cplx) * 36 * V);
        or_apply_gauge(L, Ux, g);
        ++it;
        if (reunit_every > 0 && it % reunit_every == 0) or_reunit_links(L, Ux);
        two_row_field(L, Ux, 4, 0);
        or_measure(L, Ux, &F, &theta);
        memcpy(U, Ux, sizeof(cplx) * 36 * V);
        two_row_field(L, U, 4, round_f32);
        if (it < hist_cap) {
            F_hist[it] = F;
            theta_hist[it] = theta;
        }
    }
    free(Delta);
    free(g);
    free(Ux);
    return it;
}

int64_t or_fix(const int L[4], cplx *U, double alpha, double eps, int64_t max_iter, int reunit_every,
               double *F_hist, double *theta_hist, int64_t hist_cap)
{
    const int64_t V = vol(L);
    cplx *Delta = malloc(sizeof(cplx) * 9 * V);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    double F, theta;
    or_measure(L, U, &F, &theta);
    if (hist_cap > 0) {
        F_hist[0] = F;
        theta_hist[0] = theta;
    }
    int64_t it = 0;
    while (!(theta <= eps) && it < max_iter) {
        or_delta(L, U, Delta);
        or_gauge_from_delta(L, Delta, alpha, g);
        or_apply_gauge(L, U, g);
        ++it;
        if (reunit_every > 0 && it % reunit_every == 0) or_reunit_links(L, U);
        or_measure(L, U, &F, &theta);
        if (it < hist_cap) {
            F_hist[it] = F;
            theta_hist[it] = theta;
        }
    }
    free(Delta);
    free(g);
    return it;
}

/* ------------------------------------------------------------------------ */
/* gauge-invariant observables (checks of the link update)                   */
/* ------------------------------------------------------------------------ */

/* Average plaquette (1/(18 V)) sum_x sum_{mu<nu} Re Tr[U_mu(x) U_nu(x+mu) U_mu^dag(x+nu) U_nu^dag(x)]. */
double or_plaquette(const int L[4], const cplx *U)
{
    const int64_t V = vol(L);
    double *p = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                mat3 a, b, c, d;
                get_link(U, V, mu, s, a);
                get_link(U, V, nu, hop(L, s, mu, +1), b);
                get_link(U, V, mu, hop(L, s, nu, +1), c);
                get_link(U, V, nu, s, d);
                mat_dag(c, c);
                mat_dag(d, d);
                mat_mul(a, b, a);
                mat_mul(a, c, a);
                mat_mul(a, d, a);
                acc += creal(mat_trace(a));
            }
        p[s] = acc;
    }
    double r = neumaier(p, V) / (18.0 * (double)V);
    free(p);
    return r;
}

/* Average Polyakov loop (1/(3 V3)) sum_{xyz} Tr prod_t U_t(xyz, t); returns re, im. */
void or_polyakov(const int L[4], const cplx *U, double *re, double *im)
{
    const int64_t V = vol(L);
    const int64_t V3 = V / L[3];
    double *pr = malloc(sizeof(double) * V3), *pi = malloc(sizeof(double) * V3);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V3; ++s) {
        mat3 acc = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int t = 0; t < L[3]; ++t) {
            mat3 u;
            get_link(U, V, 3, s + (int64_t)t * V3, u);
            mat_mul(acc, u, acc);
        }
        cplx tr = mat_trace(acc);
        pr[s] = creal(tr);
        pi[s] = cimag(tr);
    }
    *re = neumaier(pr, V3) / (3.0 * (double)V3);
    *im = neumaier(pi, V3) / (3.0 * (double)V3);
    free(pr);
    free(pi);
}

/* ------------------------------------------------------------------------ */
/* the functional as a function of Lie-algebra gauge parameters              */
/* ------------------------------------------------------------------------ */

static void gell_mann(int a, mat3 l)
{
    memset(l, 0, sizeof(mat3));
    const double r3 = 1.0 / sqrt(3.0);
    switch (a) {
    case 0: l[0][1] = 1; l[1][0] = 1; break;
    case 1: l[0][1] = -I; l[1][0] = I; break;
    case 2: l[0][0] = 1; l[1][1] = -1; break;
    case 3: l[0][2] = 1; l[2][0] = 1; break;
    case 4: l[0][2] = -I; l[2][0] = I; break;
    case 5: l[1][2] = 1; l[2][1] = 1; break;
    case 6: l[1][2] = -I; l[2][1] = I; break;
    default: l[0][0] = r3; l[1][1] = r3; l[2][2] = -2.0 * r3; break;
    }
}

/* Q = sum_a w_a lambda_a (hermitian, traceless). */
static void algebra_matrix(const double w[8], mat3 Q)
{
    memset(Q, 0, sizeof(mat3));
    for (int a = 0; a < 8; ++a) {
        mat3 l;
        gell_mann(a, l);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Q[i][j] += w[a] * l[i][j];
    }
}

/*
 * Cyclic Jacobi diagonalisation of a hermitian 3x3 matrix: Q = W diag(lam) W^dag.
 * Each rotation acts on one (p, q) pair: a phase on column q makes Q_pq real,
 * then the classical real Jacobi rotation annihilates it. An off-diagonal
 * entry below the rounding level of its two diagonal entries is set to zero
 * instead of rotated (a rotation by the phase of a denormal entry is not
 * unitary to working precision); sweeps stop when nothing is left to rotate.
 */
void or_eigh3(const cplx *Qin, double lam[3], cplx *Wout)
{
    mat3 A, W = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    memcpy(A, Qin, sizeof(mat3));
    for (int sweep = 0; sweep < 50; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = cabs(A[p][q]);
                double app = creal(A[p][p]), aqq = creal(A[q][q]);
                if (apq == 0.0) continue;
                if (apq <= 1e-18 * (fabs(app) + fabs(aqq))) {
                    A[p][q] = 0.0;
                    A[q][p] = 0.0;
                    continue;
                }
                rotated = 1;
                cplx phase = A[p][q] / apq; /* e^{i phi} */
                double th = (aqq - app) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* J = P R: J_pp = c, J_pq = s, J_qp = -s e^{-i phi}, J_qq = c e^{-i phi} */
                mat3 J = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, Jd;
                J[p][p] = c;
                J[p][q] = s;
                J[q][p] = -s * conj(phase);
                J[q][q] = c * conj(phase);
                mat_dag(J, Jd);
                mat_mul(Jd, A, A);
                mat_mul(A, J, A);
                mat_mul(W, J, W);
            }
        if (!rotated) break;
    }
    for (int i = 0; i < 3; ++i) lam[i] = creal(A[i][i]);
    memcpy(Wout, W, sizeof(mat3));
}

/* exp(i Q) = W diag(exp(i lam)) W^dag for hermitian Q. */
void or_expi(const cplx *Q9, cplx *out9)
{
    double lam[3];
    mat3 W, Wd, E = {{0}};
    or_eigh3(Q9, lam, &W[0][0]);
    for (int k = 0; k < 3; ++k) E[k][k] = cexp(I * lam[k]);
    mat_dag(W, Wd);
    mat_mul(W, E, E);
    mat_mul(E, Wd, E);
    memcpy(out9, E, sizeof(mat3));
}

/* g(x) = exp(i sum_a omega_a(x) lambda_a) for every site; g[(i*3+j)*V + s]. */
void or_gauge_from_omega(const int L[4], const double *omega, cplx *g)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double w[8];
        for (int a = 0; a < 8; ++a) w[a] = omega[(int64_t)a * V + s];
        mat3 Q, e;
        algebra_matrix(w, Q);
        or_expi(&Q[0][0], &e[0][0]);
        put_site(g, V, s, e);
    }
}

/* Eq. 1: F_U[g] = (1/(12 V)) sum_x sum_mu Re Tr[g(x) U_mu(x) g^dag(x+mu)], g from omega. */
double or_functional_g(const int L[4], const cplx *U, const double *omega)
{
    const int64_t V = vol(L);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    double *f = malloc(sizeof(double) * V);
    or_gauge_from_omega(L, omega, g);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        mat3 gx;
        get_site(g, V, s, gx);
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            mat3 u, gf;
            get_link(U, V, mu, s, u);
            get_site(g, V, hop(L, s, mu, +1), gf);
            mat_dag(gf, gf);
            mat_mul(gx, u, u);
            mat_mul(u, gf, u);
            acc += creal(mat_trace(u));
        }
        f[s] = acc;
    }
    double r = neumaier(f, V) / (12.0 * (double)V);
    free(g);
    free(f);
    return r;
}

/*
 * The eight terms of Eq. 1 (without the 1/(12V)) that depend on the gauge
 * parameters at site `site`, with omega at that site replaced by w_site:
 *   sum_mu Re Tr[g(x) U_mu(x) g^dag(x+mu)] + Re Tr[g(x-mu) U_mu(x-mu) g^dag(x)].
 * Used for finite differences that avoid cancellation in the global sum.
 */
double or_local_functional_g(const int L[4], const cplx *U, const double *omega, int64_t site,
                             const double w_site[8])
{
    const int64_t V = vol(L);
    double acc = 0.0;
    mat3 gx;
    {
        mat3 Q;
        algebra_matrix(w_site, Q);
        or_expi(&Q[0][0], &gx[0][0]);
    }
    for (int mu = 0; mu < 4; ++mu) {
        int64_t fw = hop(L, site, mu, +1), bw = hop(L, site, mu, -1);
        double wf[8], wb[8];
        for (int a = 0; a < 8; ++a) {
            wf[a] = (fw == site) ? w_site[a] : omega[(int64_t)a * V + fw];
            wb[a] = (bw == site) ? w_site[a] : omega[(int64_t)a * V + bw];
        }
        mat3 Q, gf, gb, u, m;
        algebra_matrix(wf, Q);
        or_expi(&Q[0][0], &gf[0][0]);
        algebra_matrix(wb, Q);
        or_expi(&Q[0][0], &gb[0][0]);
        get_link(U, V, mu, site, u);
        mat_dag(gf, gf);
        mat_mul(gx, u, m);
        mat_mul(m, gf, m);
        acc += creal(mat_trace(m));
        get_link(U, V, mu, bw, u);
        mat3 gxd;
        mat_dag(gx, gxd);
        mat_mul(gb, u, m);
        mat_mul(m, gxd, m);
        acc += creal(mat_trace(m));
    }
    return acc;
}

/*
 * Frechet derivative of exp at X = iQ (Q hermitian) in direction E, by the
 * Daleckii-Krein formula in the eigenbasis of Q = W diag(lam) W^dag:
 *   L(X, E) = W [ (W^dag E W)_jk phi_jk ] W^dag,
 *   phi_jk = (e^{i lam_j} - e^{i lam_k}) / (i lam_j - i lam_k)
 *          = e^{i (lam_j + lam_k)/2} sin(d/2)/(d/2),  d = lam_j - lam_k,
 * (phi_jj = e^{i lam_j}).
 */
void or_expi_frechet(const cplx *Q9, const cplx *E9, cplx *out9)
{
    double lam[3];
    mat3 W, Wd, Et;
    or_eigh3(Q9, lam, &W[0][0]);
    mat_dag(W, Wd);
    memcpy(Et, E9, sizeof(mat3));
    mat_mul(Wd, Et, Et);
    mat_mul(Et, W, Et);
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            double d = lam[j] - lam[k];
            double sinc = (fabs(d) < 1e-8) ? 1.0 - d * d / 24.0 : sin(0.5 * d) / (0.5 * d);
            Et[j][k] *= cexp(0.5 * I * (lam[j] + lam[k])) * sinc;
        }
    mat_mul(W, Et, Et);
    mat_mul(Et, Wd, Et);
    memcpy(out9, Et, sizeof(mat3));
}

/*
 * Gradient of Eq. 1 with respect to omega_a(x) at the listed sites:
 *   dF/domega_a(x) = (1/(12V)) Re Tr[ L(X(x), i lambda_a) Sigma(x) ],
 *   Sigma(x) = sum_mu [U_mu(x) g^dag(x+mu) + U_mu^dag(x-mu) g^dag(x-mu)],
 * from differentiating the two kinds of terms that contain g(x).
 * out[k*8 + a] for site sites[k].
 */
void or_grad_omega_sites(const int L[4], const cplx *U, const double *omega, int64_t nsites,
                         const int64_t *sites, double *out)
{
    const int64_t V = vol(L);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nsites; ++k) {
        const int64_t s = sites[k];
        mat3 Sig = {{0}};
        for (int mu = 0; mu < 4; ++mu) {
            int64_t fw = hop(L, s, mu, +1), bw = hop(L, s, mu, -1);
            double wf[8], wb[8];
            for (int a = 0; a < 8; ++a) {
                wf[a] = omega[(int64_t)a * V + fw];
                wb[a] = omega[(int64_t)a * V + bw];
            }
            mat3 Q, gf, gb, u, m;
            algebra_matrix(wf, Q);
            or_expi(&Q[0][0], &gf[0][0]);
            algebra_matrix(wb, Q);
            or_expi(&Q[0][0], &gb[0][0]);
            get_link(U, V, mu, s, u);
            mat_dag(gf, gf);
            mat_mul(u, gf, m);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Sig[i][j] += m[i][j];
            get_link(U, V, mu, bw, u);
            mat_dag(u, u);
            mat_dag(gb, gb);
            mat_mul(u, gb, m);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Sig[i][j] += m[i][j];
        }
        double w[8];
        for (int a = 0; a < 8; ++a) w[a] = omega[(int64_t)a * V + s];
        mat3 Q;
        algebra_matrix(w, Q);
        for (int a = 0; a < 8; ++a) {
            mat3 l, Ld;
            gell_mann(a, l);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) l[i][j] *= I;
            or_expi_frechet(&Q[0][0], &l[0][0], &Ld[0][0]);
            mat_mul(Ld, Sig, Ld);
            out[k * 8 + a] = creal(mat_trace(Ld)) / (12.0 * (double)V);
        }
    }
}

/*
 * Gradient of Eq. 1 with respect to the links, in the convention
 * dF/dRe U_ij + i dF/dIm U_ij: since F is linear in U_mu(x) through
 * Re Tr[A U B] with A = g(x), B = g^dag(x+mu), the derivative is
 * conj((B A)_ji) = (g^dag(x) g(x+mu))_ij / (12 V). Link layout as U.
 */
void or_grad_links(const int L[4], const double *omega, cplx *dU)
{
    const int64_t V = vol(L);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    or_gauge_from_omega(L, omega, g);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        mat3 gx, gxd;
        get_site(g, V, s, gx);
        mat_dag(gx, gxd);
        for (int mu = 0; mu < 4; ++mu) {
            mat3 gf, m;
            get_site(g, V, hop(L, s, mu, +1), gf);
            mat_mul(gxd, gf, m);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) m[i][j] /= 12.0 * (double)V;
            put_link(dU, V, mu, s, m);
        }
    }
    free(g);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* input generator: Wilson-action heatbath and overrelaxation                 */
/* ------------------------------------------------------------------------ */

/*
 * Thermalised SU(3) configurations for the Wilson action
 * S = beta sum_P (1 - Re Tr U_P / 3), the workload of the paper's tests
 * (section 3: beta = 5.8, 6.0, 6.2). Not part of the method; it produces its
 * inputs. Pseudo-heatbath of Cabibbo and Marinari (Phys. Lett. B 119, 1982)
 * over the three SU(2) subgroups, each drawn with the algorithm of Kennedy
 * and Pendleton (Phys. Lett. B 156, 1985); microcanonical overrelaxation
 * (Creutz, Phys. Rev. D 36, 1987); random numbers from Philox4x32-10
 * (Salmon, Moraes, Dror and Shaw, SC 2011), one counter per draw.
 */

static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

/* Philox4x32 with 10 rounds: out = f(ctr, key). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c0, p1 = (uint64_t)PHILOX_M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A 32-bit draw as a uniform number in (0, 1]. */
static double unit_open0(uint32_t u) { return ((double)u + 1.0) * (1.0 / 4294967296.0); }

/* Counter of draw `slot` (attempt, or 255 for the direction) of subgroup k of
 * the update of U_mu(site) in heatbath sweep n. */
static void hb_counter(int64_t site, int mu, int k, int slot, int64_t n, uint32_t ctr[4])
{
    ctr[0] = (uint32_t)site;
    ctr[1] = (uint32_t)(mu + 4 * k + 16 * slot);
    ctr[2] = (uint32_t)((uint64_t)n & 0xffffffffu);
    ctr[3] = (uint32_t)((uint64_t)n >> 32);
}

enum { HB_MAX_ATTEMPTS = 64, HB_DIRECTION_SLOT = 255 };

/*
 * x in SU(2) (quaternion x0 + i x.sigma) with density proportional to
 * exp(a x0) on SU(2) (Kennedy-Pendleton): x0 from sqrt(1 - x0^2) e^(a x0) by
 * rejection, the vector part uniform on its sphere. Returns 0 and leaves x
 * untouched if no attempt is accepted (probability below 1e-30 for a > 0.5).
 */
static int kp_draw(double a, int64_t site, int mu, int k, int64_t n, const uint32_t key[2], double x[4])
{
    uint32_t ctr[4], r[4];
    for (int j = 0; j < HB_MAX_ATTEMPTS; ++j) {
        hb_counter(site, mu, k, j, n, ctr);
        or_philox4x32_10(ctr, key, r);
        const double r1 = unit_open0(r[0]), r2 = unit_open0(r[1]), r3 = unit_open0(r[2]), r4 = unit_open0(r[3]);
        const double c = cos(2.0 * M_PI * r2);
        const double lam2 = -(log(r1) + c * c * log(r3)) / (2.0 * a);
        if (r4 * r4 <= 1.0 - lam2) {
            x[0] = 1.0 - 2.0 * lam2;
            hb_counter(site, mu, k, HB_DIRECTION_SLOT, n, ctr);
            or_philox4x32_10(ctr, key, r);
            const double ct = 2.0 * unit_open0(r[0]) - 1.0, phi = 2.0 * M_PI * unit_open0(r[1]);
            const double rad = sqrt(fmax(0.0, 1.0 - x[0] * x[0]));
            const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
            x[1] = rad * st * cos(phi);
            x[2] = rad * st * sin(phi);
            x[3] = rad * ct;
            return 1;
        }
    }
    return 0;
}

/* Staple sum A of U_mu(s): U_mu(s) A is the sum of the six plaquettes through it. */
static void staple_sum(const int L[4], const cplx *U, int64_t s, int mu, mat3 A)
{
    const int64_t V = vol(L);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
    const int64_t sp = hop(L, s, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        mat3 a, b, c, t, u;
        /* upper: U_nu(s + mu) U_mu^dag(s + nu) U_nu^dag(s) */
        get_link(U, V, nu, sp, a);
        get_link(U, V, mu, hop(L, s, nu, +1), b);
        get_link(U, V, nu, s, c);
        mat_dag(b, b);
        mat_dag(c, c);
        mat_mul(a, b, t);
        mat_mul(t, c, u);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A[i][j] += u[i][j];
        /* lower: U_nu^dag(s + mu - nu) U_mu^dag(s - nu) U_nu(s - nu) */
        const int64_t sm = hop(L, s, nu, -1);
        get_link(U, V, nu, hop(L, sp, nu, -1), a);
        get_link(U, V, mu, sm, b);
        get_link(U, V, nu, sm, c);
        mat_dag(a, a);
        mat_dag(b, b);
        mat_mul(a, b, t);
        mat_mul(t, c, u);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A[i][j] += u[i][j];
    }
}

/*
 * One Cabibbo-Marinari update of U (left multiplication by an SU(2) matrix
 * in each subgroup (0,1), (0,2), (1,2) in turn) against staple sum A.
 * mode 0: heatbath; mode 1: overrelaxation. Then Gram-Schmidt.
 */
static void cm_update(mat3 U, mat3 A, double beta, int mode, int64_t site, int mu, int64_t n,
                      const uint32_t key[2])
{
    static const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int k = 0; k < 3; ++k) {
        const int p = sub[k][0], q = sub[k][1];
        mat3 W;
        mat_mul(U, A, W);
        /* the part of the 2x2 block proportional to SU(2): [[al, be], [-conj(be), conj(al)]] */
        const cplx al = 0.5 * (W[p][p] + conj(W[q][q]));
        const cplx be = 0.5 * (W[p][q] - conj(W[q][p]));
        const double det = creal(al) * creal(al) + cimag(al) * cimag(al) + creal(be) * creal(be) +
                           cimag(be) * cimag(be);
        if (!(det > 1e-300)) continue;
        const double nk = sqrt(det);
        /* V = block / |block| in SU(2); Re Tr(r W_block) = nk Re Tr(r V) */
        const cplx v00 = al / nk, v01 = be / nk;
        /* r = X V^dag (heatbath) or r = V^dag V^dag (overrelaxation) */
        cplx vd00 = conj(v00), vd01 = -v01, vd10 = conj(v01), vd11 = v00; /* V^dag */
        cplx r00, r01, r10, r11;
        if (mode == 0) {
            double x[4];
            if (!kp_draw(2.0 * beta / 3.0 * nk, site, mu, k, n, key, x)) continue;
            const cplx x00 = x[0] + I * x[3], x01 = x[2] + I * x[1];
            const cplx x10 = -x[2] + I * x[1], x11 = x[0] - I * x[3];
            r00 = x00 * vd00 + x01 * vd10;
            r01 = x00 * vd01 + x01 * vd11;
            r10 = x10 * vd00 + x11 * vd10;
            r11 = x10 * vd01 + x11 * vd11;
        } else {
            r00 = vd00 * vd00 + vd01 * vd10;
            r01 = vd00 * vd01 + vd01 * vd11;
            r10 = vd10 * vd00 + vd11 * vd10;
            r11 = vd10 * vd01 + vd11 * vd11;
        }
        for (int j = 0; j < 3; ++j) {
            const cplx up = U[p][j], uq = U[q][j];
            U[p][j] = r00 * up + r01 * uq;
            U[q][j] = r10 * up + r11 * uq;
        }
    }
    or_reunit(&U[0][0]);
}

/*
 * n_sweeps sweeps, each a heatbath sweep (sweep index sweep0 + i for the
 * random numbers) followed by n_or overrelaxation sweeps. A sweep visits
 * mu = 0..3, and for each the even then the odd sites (x+y+z+t even/odd);
 * the links of one (mu, parity) class are independent and updated together.
 * Every extent must be even.
 */
void or_heatbath(const int L[4], cplx *U, double beta, int n_sweeps, int n_or, uint64_t seed, int64_t sweep0)
{
    const int64_t V = vol(L);
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    for (int i = 0; i < n_sweeps; ++i) {
        for (int rep = 0; rep <= n_or; ++rep) {
            const int mode = rep == 0 ? 0 : 1;
            for (int mu = 0; mu < 4; ++mu)
                for (int par = 0; par < 2; ++par) {
#pragma omp parallel for schedule(static)
                    for (int64_t s = 0; s < V; ++s) {
                        int c[4];
                        coords(L, s, c);
                        if (((c[0] + c[1] + c[2] + c[3]) & 1) != par) continue;
                        mat3 u, A;
                        staple_sum(L, U, s, mu, A);
                        get_link(U, V, mu, s, u);
                        cm_update(u, A, beta, mode, s, mu, sweep0 + i, key);
                        put_link(U, V, mu, s, u);
                    }
                }
        }
    }
}

/* n overrelaxation sweeps alone (no random numbers; the action is unchanged). */
void or_overrelax(const int L[4], cplx *U, int n)
{
    const int64_t V = vol(L);
    const uint32_t key[2] = {0u, 0u};
    for (int i = 0; i < n; ++i)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
#pragma omp parallel for schedule(static)
                for (int64_t s = 0; s < V; ++s) {
                    int c[4];
                    coords(L, s, c);
                    if (((c[0] + c[1] + c[2] + c[3]) & 1) != par) continue;
                    mat3 u, A;
                    staple_sum(L, U, s, mu, A);
                    get_link(U, V, mu, s, u);
                    cm_update(u, A, 1.0, 1, s, mu, 0, key);
                    put_link(U, V, mu, s, u);
                }
            }
}

/* Kennedy-Pendleton draws for tests: x0 of n draws at parameter a (subgroup 0,
 * mu 0, sweep n0 + j for draw j at site 0). Returns the number accepted. */
int64_t or_kp_samples(double a, int64_t n, uint64_t seed, double *x0)
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    int64_t acc = 0;
    for (int64_t j = 0; j < n; ++j) {
        double x[4];
        if (kp_draw(a, 0, 0, 0, j, key, x)) x0[acc++] = x[0];
    }
    return acc;
}

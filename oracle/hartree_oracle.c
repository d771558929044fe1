/*
 * CPU oracle for the periodic Hartree (FFT-Poisson) solve and the Gaussian
 * density splat that feeds it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Everything is plain double precision, written for a reader to check by
 * eye against the paper, not for speed:
 *
 *   - Hartree potential: Eq. (6) (Sec. 2.1, "Kohn-Sham equation"), read as
 *     the periodic potential of a neutral cell (the G = 0 term dropped),
 *     obtained by "solving the Poisson equation using FFT" (same section).
 *   - Hartree energy: the E_Hartree term of Eq. (7), E_H = 1/2 * int n v_H.
 *   - Grid convention: axes a, b, c with N_a, N_b, N_c points, the c index
 *     running fastest (structure B in "abc" order, Sec. 3.2.2).
 *   - FFT: a textbook recursive decimation-in-time mixed-radix transform,
 *     applied along c, then b, then a, as in the calculation flow of
 *     Sec. 3.2.4 (abc -> cab -> cba, then back).
 *   - Splat: a sum of normalized periodic Gaussians minus a uniform
 *     neutralizing background; exp() is evaluated per grid point.
 *
 * Conventions (the paper is silent on them; each is a stated reading):
 *   - forward DFT  X(m) = sum_r x(r) exp(-2 pi i m.r/N), unnormalized;
 *     inverse carries 1/N.
 *   - K(G) = 4 pi / |G|^2, K(0) = 0; on an even-length axis the Nyquist
 *     index is ambiguous (+N/2 or -N/2) and K is averaged over both
 *     aliases of every axis sitting at Nyquist, which keeps K(G) = K(-G).
 *   - Gaussian of standard deviation sigma normalized to total charge Z.
 *
 * Complex arrays are interleaved (re, im) doubles.  Return value 0 means
 * success, a negative value a rejected argument.
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

static const double TWO_PI = 6.283185307179586476925286766559;
static const double FOUR_PI = 12.566370614359172953850573533118;

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* 1-D transform: recursive decimation in time over the smallest prime */
/* factor.  For n = p * m, the input splits into p subsequences        */
/* x[r], x[r+p], ... of length m; each is transformed recursively, and  */
/*   X[k + q m] = sum_{r<p} W_n^{r (k + q m)} Y_r[k],  W_n = e^{s 2pi i/n} */
/* A prime length therefore ends in a direct p-point DFT.               */
/* ------------------------------------------------------------------ */

static int smallest_prime_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* w[t] = exp(sign * 2 pi i t / ntop) for t < ntop; a sub-length n that
 * divides ntop reads W_n^t as w[(t mod n) * (ntop / n)]. */
static void fft_rec(const cplx *x, int stride, cplx *X, int n, const cplx *w,
                    int ntop, cplx *scratch)
{
    if (n == 1) {
        X[0] = x[0];
        return;
    }
    int p = smallest_prime_factor(n);
    int m = n / p;
    cplx *Y = scratch;            /* p sub-results of length m */
    cplx *deeper = scratch + n;   /* scratch for the recursion below */
    for (int r = 0; r < p; ++r)
        fft_rec(x + (size_t)r * stride, stride * p, Y + (size_t)r * m, m, w, ntop, deeper);
    int step = ntop / n;
    for (int q = 0; q < p; ++q) {
        for (int k = 0; k < m; ++k) {
            int kk = k + q * m;
            cplx s = 0;
            for (int r = 0; r < p; ++r) {
                long t = ((long)r * kk) % n;
                s += w[t * step] * Y[(size_t)r * m + k];
            }
            X[kk] = s;
        }
    }
}

/* Scratch needed by fft_rec for length n: n + n/p1 + n/(p1 p2) + ... <= 2n */
static cplx *make_twiddles(int n, int sign)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int t = 0; t < n; ++t) {
        double ang = sign * TWO_PI * (double)t / (double)n;
        w[t] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* sign = -1 forward (unnormalized), +1 backward (unnormalized). */
int oracle_fft1d(int n, int sign, const double *in, double *out)
{
    if (n < 1 || (sign != 1 && sign != -1) || !in || !out) return -1;
    cplx *w = make_twiddles(n, sign);
    cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *s = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n + 2));
    for (int i = 0; i < n; ++i) x[i] = in[2 * i] + I * in[2 * i + 1];
    fft_rec(x, 1, X, n, w, n, s);
    for (int i = 0; i < n; ++i) {
        out[2 * i] = creal(X[i]);
        out[2 * i + 1] = cimag(X[i]);
    }
    free(w); free(x); free(X); free(s);
    return 0;
}

/* Transform every pencil of a [Na][Nb][Nc] complex array along one axis. */
static void fft_axis(cplx *a, const int dims[3], int axis, int sign)
{
    int n = dims[axis];
    if (n == 1) return;
    size_t stride = (axis == 2) ? 1 : (axis == 1) ? (size_t)dims[2] : (size_t)dims[1] * dims[2];
    /* pencils are indexed by the two other axes */
    int o1 = (axis == 0) ? 1 : 0;
    int o2 = (axis == 2) ? 1 : 2;
    size_t s1 = (o1 == 0) ? (size_t)dims[1] * dims[2] : (size_t)dims[2];
    size_t s2 = (o2 == 1) ? (size_t)dims[2] : 1;
    long npencil = (long)dims[o1] * dims[o2];
    cplx *w = make_twiddles(n, sign);
    #pragma omp parallel
    {
        cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *s = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n + 2));
        #pragma omp for schedule(static)
        for (long p = 0; p < npencil; ++p) {
            size_t base = (size_t)(p / dims[o2]) * s1 + (size_t)(p % dims[o2]) * s2;
            for (int i = 0; i < n; ++i) x[i] = a[base + (size_t)i * stride];
            fft_rec(x, 1, X, n, w, n, s);
            for (int i = 0; i < n; ++i) a[base + (size_t)i * stride] = X[i];
        }
        free(x); free(X); free(s);
    }
    free(w);
}

/* 3-D transform of an interleaved complex [Na][Nb][Nc] array, along c,
 * then b, then a (unnormalized in both directions). */
int oracle_fft3d(const int dims[3], int sign, const double *in, double *out)
{
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || !in || !out) return -1;
    if (sign != 1 && sign != -1) return -1;
    size_t n = (size_t)dims[0] * dims[1] * dims[2];
    cplx *a = (cplx *)malloc(sizeof(cplx) * n);
    for (size_t i = 0; i < n; ++i) a[i] = in[2 * i] + I * in[2 * i + 1];
    fft_axis(a, dims, 2, sign);
    fft_axis(a, dims, 1, sign);
    fft_axis(a, dims, 0, sign);
    for (size_t i = 0; i < n; ++i) {
        out[2 * i] = creal(a[i]);
        out[2 * i + 1] = cimag(a[i]);
    }
    free(a);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cell geometry.  cell holds the rows a, b, c (Bohr).                  */
/* Reciprocal rows b_d satisfy a_i . b_j = 2 pi delta_ij.               */
/* ------------------------------------------------------------------ */

static double det3(const double m[9])
{
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

static int reciprocal(const double A[9], double B[9], double *omega)
{
    double d = det3(A);
    if (!isfinite(d) || fabs(d) < 1e-300) return -2;
    for (int i = 0; i < 9; ++i)
        if (!isfinite(A[i])) return -2;
    /* B = 2 pi (A^{-1})^T: row i of B is 2 pi * (a_j x a_k) / det */
    const double *a0 = A, *a1 = A + 3, *a2 = A + 6;
    double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
    double c20[3] = {a2[1] * a0[2] - a2[2] * a0[1], a2[2] * a0[0] - a2[0] * a0[2], a2[0] * a0[1] - a2[1] * a0[0]};
    double c01[3] = {a0[1] * a1[2] - a0[2] * a1[1], a0[2] * a1[0] - a0[0] * a1[2], a0[0] * a1[1] - a0[1] * a1[0]};
    for (int k = 0; k < 3; ++k) {
        B[k] = TWO_PI * c12[k] / d;
        B[3 + k] = TWO_PI * c20[k] / d;
        B[6 + k] = TWO_PI * c01[k] / d;
    }
    *omega = fabs(d);
    return 0;
}

static int check_dims(const int dims[3])
{
    if (!dims) return -1;
    for (int d = 0; d < 3; ++d)
        if (dims[d] < 1) return -1;
    return 0;
}

/* Poisson kernel K(m) for the full index m = (ma, mb, mc), 0 <= m_d < N_d. */
static double kernel_at(const double B[9], const int dims[3], const int m[3])
{
    /* candidate signed indices per axis: one normally, two at Nyquist */
    int cand[3][2], ncand[3];
    for (int d = 0; d < 3; ++d) {
        int n = dims[d];
        if (2 * m[d] < n) {
            cand[d][0] = m[d];
            ncand[d] = 1;
        } else if (2 * m[d] > n) {
            cand[d][0] = m[d] - n;
            ncand[d] = 1;
        } else { /* Nyquist of an even axis */
            cand[d][0] = m[d];
            cand[d][1] = m[d] - n;
            ncand[d] = 2;
        }
    }
    double sum = 0.0;
    int count = 0;
    for (int i = 0; i < ncand[0]; ++i)
        for (int j = 0; j < ncand[1]; ++j)
            for (int k = 0; k < ncand[2]; ++k) {
                double mt[3] = {cand[0][i], cand[1][j], cand[2][k]};
                double G[3];
                for (int x = 0; x < 3; ++x) G[x] = mt[0] * B[x] + mt[1] * B[3 + x] + mt[2] * B[6 + x];
                double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                sum += (g2 > 0.0) ? FOUR_PI / g2 : 0.0;
                ++count;
            }
    return sum / count;
}

/* Full-grid K(m) in [Na][Nb][Nc] order (for tests). */
int oracle_kernel(const double cell[9], const int dims[3], double *K)
{
    double B[9], omega;
    if (check_dims(dims) || !cell || !K) return -1;
    if (reciprocal(cell, B, &omega)) return -2;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < dims[0]; ++i)
        for (int j = 0; j < dims[1]; ++j)
            for (int k = 0; k < dims[2]; ++k) {
                int m[3] = {i, j, k};
                K[((size_t)i * dims[1] + j) * dims[2] + k] = kernel_at(B, dims, m);
            }
    return 0;
}

/* Compensated (Kahan-Babuska / Neumaier) summation: s carries the running
 * sum, c the rounding error lost from it, so that the energies of 10^9-point
 * grids keep their value to a few units of the last place instead of the
 * ~sqrt(n) ulps a plain running sum loses. */
typedef struct {
    double s, c;
} csum_t;

static void csum_add(csum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

/* out = P in, with P = F^{-1} K F on real grids.  Also returns, when the
 * pointers are non-null, sum_m K |F in|^2 and the largest |Im| seen in the
 * inverse transform (exactly zero in exact arithmetic). */
static int apply_P(const double cell[9], const int dims[3], const double *in, double *out,
                   double *kx2, double *max_imag)
{
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    size_t n = (size_t)dims[0] * dims[1] * dims[2];
    cplx *a = (cplx *)malloc(sizeof(cplx) * n);
    for (size_t i = 0; i < n; ++i) a[i] = in[i];
    fft_axis(a, dims, 2, -1);
    fft_axis(a, dims, 1, -1);
    fft_axis(a, dims, 0, -1);
    /* sum_m K |X|^2: one compensated sum per a-plane, then over the planes in
     * order (the same value for any thread count) */
    double *plane = (double *)calloc((size_t)dims[0], sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < dims[0]; ++i) {
        csum_t ps = {0.0, 0.0};
        for (int j = 0; j < dims[1]; ++j)
            for (int k = 0; k < dims[2]; ++k) {
                int m[3] = {i, j, k};
                size_t idx = ((size_t)i * dims[1] + j) * dims[2] + k;
                double K = kernel_at(B, dims, m);
                double re = creal(a[idx]), im = cimag(a[idx]);
                csum_add(&ps, K * (re * re + im * im));
                a[idx] *= K;
            }
        plane[i] = ps.s + ps.c;
    }
    csum_t tot = {0.0, 0.0};
    for (int i = 0; i < dims[0]; ++i) csum_add(&tot, plane[i]);
    free(plane);
    double acc = tot.s + tot.c;
    fft_axis(a, dims, 0, +1);
    fft_axis(a, dims, 1, +1);
    fft_axis(a, dims, 2, +1);
    double mi = 0.0;
    for (size_t i = 0; i < n; ++i) {
        out[i] = creal(a[i]) / (double)n;
        double t = fabs(cimag(a[i])) / (double)n;
        if (t > mi) mi = t;
    }
    if (kx2) *kx2 = acc;
    if (max_imag) *max_imag = mi;
    free(a);
    return 0;
}

/* V = P rho; eh_real = dV/2 sum rho V; eh_recip = Omega/(2 N^2) sum K|X|^2. */
int oracle_poisson(const double cell[9], const int dims[3], const double *rho, double *V,
                   double *eh_real, double *eh_recip, double *max_imag)
{
    if (check_dims(dims) || !cell || !rho || !V) return -1;
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    double kx2 = 0.0, mi = 0.0;
    int rc = apply_P(cell, dims, rho, V, &kx2, &mi);
    if (rc) return rc;
    double n = (double)dims[0] * dims[1] * dims[2];
    double dv = omega / n;
    csum_t cs = {0.0, 0.0};
    size_t nn = (size_t)n;
    for (size_t i = 0; i < nn; ++i) csum_add(&cs, rho[i] * V[i]);
    if (eh_real) *eh_real = 0.5 * dv * (cs.s + cs.c);
    if (eh_recip) *eh_recip = omega / (2.0 * n * n) * kx2;
    if (max_imag) *max_imag = mi;
    return 0;
}

/* grad_rho = d L / d rho for L with upstream gradients grad_v (on V, may be
 * NULL = zero) and grad_e (on E_H):  P grad_v + grad_e * dV * P rho. */
int oracle_backward(const double cell[9], const int dims[3], const double *grad_v, double grad_e,
                    const double *rho, double *grad_rho)
{
    if (check_dims(dims) || !cell || !grad_rho) return -1;
    if (grad_e != 0.0 && !rho) return -1;
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    size_t n = (size_t)dims[0] * dims[1] * dims[2];
    double dv = omega / (double)n;
    double *t = (double *)calloc(n, sizeof(double));
    if (grad_v) {
        int rc = apply_P(cell, dims, grad_v, grad_rho, NULL, NULL);
        if (rc) { free(t); return rc; }
    } else {
        memset(grad_rho, 0, n * sizeof(double));
    }
    if (grad_e != 0.0) {
        int rc = apply_P(cell, dims, rho, t, NULL, NULL);
        if (rc) { free(t); return rc; }
        for (size_t i = 0; i < n; ++i) grad_rho[i] += grad_e * dv * t[i];
    }
    free(t);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Splat: rho(r) = sum_a Z_a (2 pi s_a^2)^(-3/2) sum_L exp(-|r-R_a-L|^2 /  */
/* (2 s_a^2))  [- Q/Omega].  Every image within cutoff*s_a of a grid      */
/* point is summed; the grid point r_ijk = (i/Na) a + (j/Nb) b + (k/Nc) c.  */
/* An image of atom a near point r is found by walking unwrapped grid     */
/* indices over the fractional bounding box of the cutoff sphere.         */
/* ------------------------------------------------------------------ */

typedef struct {
    long lo[3], hi[3]; /* unwrapped grid index range of the cutoff box */
} box_t;

static box_t atom_box(const double A[9], const double B[9], const int dims[3], const double R[3],
                      double rc)
{
    box_t bx;
    for (int d = 0; d < 3; ++d) {
        const double *b = B + 3 * d;
        double f = (R[0] * b[0] + R[1] * b[1] + R[2] * b[2]) / TWO_PI; /* fractional coord */
        double e = rc * sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) / TWO_PI;
        bx.lo[d] = (long)ceil((f - e) * dims[d]);
        bx.hi[d] = (long)floor((f + e) * dims[d]);
    }
    (void)A;
    return bx;
}

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

static void grid_point(const double A[9], const int dims[3], long i, long j, long k, double r[3])
{
    double fi = (double)i / dims[0], fj = (double)j / dims[1], fk = (double)k / dims[2];
    for (int x = 0; x < 3; ++x) r[x] = fi * A[x] + fj * A[3 + x] + fk * A[6 + x];
}

static int check_atoms(int natoms, const double *pos, const double *Z, const double *sigma)
{
    if (natoms < 0) return -1;
    if (natoms > 0 && (!pos || !Z || !sigma)) return -1;
    for (int a = 0; a < natoms; ++a) {
        if (!(sigma[a] > 0.0) || !isfinite(sigma[a]) || !isfinite(Z[a])) return -1;
        for (int x = 0; x < 3; ++x)
            if (!isfinite(pos[3 * a + x])) return -1;
    }
    return 0;
}

int oracle_splat(const double cell[9], const int dims[3], int natoms, const double *pos,
                 const double *Z, const double *sigma, double cutoff_sigmas, int subtract_background,
                 double *rho)
{
    if (check_dims(dims) || !cell || !rho || !(cutoff_sigmas > 0.0)) return -1;
    if (check_atoms(natoms, pos, Z, sigma)) return -1;
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    double Q = 0.0;
    for (int a = 0; a < natoms; ++a) Q += Z[a];
    double bg = subtract_background ? Q / omega : 0.0;
    box_t *boxes = (box_t *)malloc(sizeof(box_t) * (size_t)(natoms > 0 ? natoms : 1));
    for (int a = 0; a < natoms; ++a) boxes[a] = atom_box(cell, B, dims, pos + 3 * a, cutoff_sigmas * sigma[a]);
    size_t plane = (size_t)dims[1] * dims[2];
    /* one a-plane per iteration: each plane sums its atoms in index order */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int ip = 0; ip < dims[0]; ++ip) {
        double *out = rho + (size_t)ip * plane;
        for (size_t t = 0; t < plane; ++t) out[t] = 0.0;
        for (int a = 0; a < natoms; ++a) {
            const double *R = pos + 3 * a;
            double s = sigma[a], rc = cutoff_sigmas * s;
            double norm = Z[a] * pow(TWO_PI * s * s, -1.5);
            box_t bx = boxes[a];
            for (long i = bx.lo[0]; i <= bx.hi[0]; ++i) {
                if (wrap(i, dims[0]) != ip) continue;
                for (long j = bx.lo[1]; j <= bx.hi[1]; ++j)
                    for (long k = bx.lo[2]; k <= bx.hi[2]; ++k) {
                        double r[3];
                        grid_point(cell, dims, i, j, k, r);
                        double d0 = r[0] - R[0], d1 = r[1] - R[1], d2 = r[2] - R[2];
                        double d2s = d0 * d0 + d1 * d1 + d2 * d2;
                        if (d2s > rc * rc) continue;
                        out[(size_t)wrap(j, dims[1]) * dims[2] + wrap(k, dims[2])] +=
                            norm * exp(-d2s / (2.0 * s * s));
                    }
            }
        }
        for (size_t t = 0; t < plane; ++t) out[t] -= bg;
    }
    free(boxes);
    return 0;
}

/* rho at selected grid points (flat storage indices), one by one. */
int oracle_splat_points(const double cell[9], const int dims[3], int natoms, const double *pos,
                        const double *Z, const double *sigma, double cutoff_sigmas,
                        int subtract_background, int npts, const int64_t *flat_idx, double *vals)
{
    if (check_dims(dims) || !cell || !(cutoff_sigmas > 0.0) || npts < 0) return -1;
    if (npts > 0 && (!flat_idx || !vals)) return -1;
    if (check_atoms(natoms, pos, Z, sigma)) return -1;
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    double Q = 0.0;
    for (int a = 0; a < natoms; ++a) Q += Z[a];
    double bg = subtract_background ? Q / omega : 0.0;
    long ntot = (long)dims[0] * dims[1] * dims[2];
    for (int p = 0; p < npts; ++p)
        if (flat_idx[p] < 0 || flat_idx[p] >= ntot) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < npts; ++p) {
        long f = (long)flat_idx[p];
        long ip = f / ((long)dims[1] * dims[2]);
        long jp = (f / dims[2]) % dims[1];
        long kp = f % dims[2];
        double acc = 0.0;
        for (int a = 0; a < natoms; ++a) {
            const double *R = pos + 3 * a;
            double s = sigma[a], rc = cutoff_sigmas * s;
            double norm = Z[a] * pow(TWO_PI * s * s, -1.5);
            box_t bx = atom_box(cell, B, dims, R, rc);
            /* the unwrapped indices congruent to (ip, jp, kp) inside the box */
            for (long i = bx.lo[0] + wrap(ip - bx.lo[0], dims[0]); i <= bx.hi[0]; i += dims[0])
                for (long j = bx.lo[1] + wrap(jp - bx.lo[1], dims[1]); j <= bx.hi[1]; j += dims[1])
                    for (long k = bx.lo[2] + wrap(kp - bx.lo[2], dims[2]); k <= bx.hi[2]; k += dims[2]) {
                        double r[3];
                        grid_point(cell, dims, i, j, k, r);
                        double d0 = r[0] - R[0], d1 = r[1] - R[1], d2 = r[2] - R[2];
                        double d2s = d0 * d0 + d1 * d1 + d2 * d2;
                        if (d2s > rc * rc) continue;
                        acc += norm * exp(-d2s / (2.0 * s * s));
                    }
        }
        vals[p] = acc - bg;
    }
    return 0;
}

/* grad_pos[a] = sum_r grad_rho(r) * d rho(r) / d R_a
 *            = Z_a (2 pi s^2)^(-3/2) / s^2 * sum_r grad_rho(r) sum_L g(d) d,
 * d = r - R_a - L, g(d) = exp(-|d|^2 / (2 s^2)).  sel (nullable) lists the
 * atoms to evaluate; grad_pos then holds nsel rows in that order. */
int oracle_splat_adjoint(const double cell[9], const int dims[3], int natoms, const double *pos,
                         const double *Z, const double *sigma, double cutoff_sigmas,
                         const double *grad_rho, int nsel, const int *sel, double *grad_pos)
{
    if (check_dims(dims) || !cell || !grad_rho || !grad_pos || !(cutoff_sigmas > 0.0)) return -1;
    if (check_atoms(natoms, pos, Z, sigma)) return -1;
    double B[9], omega;
    if (reciprocal(cell, B, &omega)) return -2;
    int nout = sel ? nsel : natoms;
    if (nout < 0) return -1;
    for (int t = 0; t < nout; ++t)
        if (sel && (sel[t] < 0 || sel[t] >= natoms)) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nout; ++t) {
        int a = sel ? sel[t] : t;
        const double *R = pos + 3 * a;
        double s = sigma[a], rc = cutoff_sigmas * s;
        double norm = Z[a] * pow(TWO_PI * s * s, -1.5) / (s * s);
        box_t bx = atom_box(cell, B, dims, R, rc);
        double acc[3] = {0.0, 0.0, 0.0};
        for (long i = bx.lo[0]; i <= bx.hi[0]; ++i)
            for (long j = bx.lo[1]; j <= bx.hi[1]; ++j)
                for (long k = bx.lo[2]; k <= bx.hi[2]; ++k) {
                    double r[3];
                    grid_point(cell, dims, i, j, k, r);
                    double d[3] = {r[0] - R[0], r[1] - R[1], r[2] - R[2]};
                    double d2s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (d2s > rc * rc) continue;
                    size_t idx = ((size_t)wrap(i, dims[0]) * dims[1] + wrap(j, dims[1])) * dims[2] +
                                 wrap(k, dims[2]);
                    double gw = grad_rho[idx] * exp(-d2s / (2.0 * s * s));
                    for (int x = 0; x < 3; ++x) acc[x] += gw * d[x];
                }
        for (int x = 0; x < 3; ++x) grad_pos[3 * t + x] = norm * acc[x];
    }
    return 0;
}

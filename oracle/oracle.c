/*
 * FP64 CPU oracle for two-link staggered Gaussian smearing
 * (Gottlieb, Jeong, Strelchenko, "Two-link Staggered Quark Smearing in QUDA",
 * arXiv:2301.05518).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition the GPU library is checked against.  Only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header or table with the HIP library, and the library never
 * calls it.
 *
 * Everything is double precision complex, natural (site-major) layout:
 *   gauge field U  : [Lt][Lz][Ly][Lx][mu=0..3][a][b]   mu = x, y, z, t
 *   two-link field : [Lt][Lz][Ly][Lx][mu=0..2][a][b]   spatial mu only
 *   colour vectors : [Lz][Ly][Lx][c]                    one time slice
 * U_mu(x) transports a vector from x+mu^ to x, as in the hopping operator H
 * of Sec. 2.  Boundaries are periodic in x, y, z; the time direction is never
 * hopped (the Laplacian is three-dimensional and acts slice by slice).
 *
 * Parity pins: every function here is checked by the CPU test suite against
 * closed forms, invariants and brute force (unit gauge, diagonal phases,
 * gauge covariance, Hermiticity, the free-field plane-wave spectrum, the
 * exact free-field smearing kernel, dense 4^3 matrices; for the one-link
 * operators also the identity between the hopping and Laplacian forms of
 * Gaussian smearing that follows eq. gsmear).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static long site4(const int L[4], int x, int y, int z, int t)
{
    return (((long)t * L[2] + z) * L[1] + y) * L[0] + x;
}

static long site3(const int L[4], int x, int y, int z)
{
    return ((long)z * L[1] + y) * L[0] + x;
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* coordinates of site s3 of a slice shifted by k steps along spatial mu */
static void shifted(const int L[4], int x, int y, int z, int mu, int k,
                    int *xs, int *ys, int *zs)
{
    int c[3] = {x, y, z};
    c[mu] = wrap(c[mu] + k, L[mu]);
    *xs = c[0];
    *ys = c[1];
    *zs = c[2];
}

static const cplx *link(const int L[4], const cplx *U, int x, int y, int z, int t, int mu)
{
    return U + (site4(L, x, y, z, t) * 4 + mu) * 9;
}

static const cplx *twolink(const int L[4], const cplx *W, int x, int y, int z, int t, int mu)
{
    return W + (site4(L, x, y, z, t) * 3 + mu) * 9;
}

/* out = M v */
static void matvec(const cplx *M, const cplx *v, cplx *out)
{
    for (int a = 0; a < 3; a++) {
        cplx s = 0;
        for (int b = 0; b < 3; b++)
            s += M[a * 3 + b] * v[b];
        out[a] = s;
    }
}

/* out = M^dagger v */
static void matvec_dag(const cplx *M, const cplx *v, cplx *out)
{
    for (int a = 0; a < 3; a++) {
        cplx s = 0;
        for (int b = 0; b < 3; b++)
            s += conj(M[b * 3 + a]) * v[b];
        out[a] = s;
    }
}

/*
 * Two-link product, Sec. 2 (definition under the one-link Laplacian):
 *   V_mu(x) = U_mu(x) U_mu(x+mu^),  mu = x, y, z,  for every site of every slice.
 * Brute-force 3x3 complex product per site and direction.
 */
void or_build_twolinks(const int L[4], const cplx *U, cplx *W)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < L[3]; t++)
        for (int z = 0; z < L[2]; z++)
            for (int y = 0; y < L[1]; y++)
                for (int x = 0; x < L[0]; x++)
                    for (int mu = 0; mu < 3; mu++) {
                        int xs, ys, zs;
                        shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);
                        const cplx *A = link(L, U, x, y, z, t, mu);
                        const cplx *B = link(L, U, xs, ys, zs, t, mu);
                        cplx *out = W + (site4(L, x, y, z, t) * 3 + mu) * 9;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++) {
                                cplx s = 0;
                                for (int k = 0; k < 3; k++)
                                    s += A[a * 3 + k] * B[k * 3 + b];
                                out[a * 3 + b] = s;
                            }
                    }
}

/*
 * Two-link 3D Laplacian on time slice t, first form (eq. tlLapl1), using the
 * precomputed two-link field:
 *   4 Lap psi(x) = sum_mu [ V_mu(x) psi(x+2mu^) + V_mu^dag(x-2mu^) psi(x-2mu^) ] - 6 psi(x)
 * Both hops are added even when x+2mu^ and x-2mu^ are the same site (L_mu <= 4).
 */
void or_lap_twolink(const int L[4], const cplx *W, int t, const cplx *in, cplx *out)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < L[2]; z++)
        for (int y = 0; y < L[1]; y++)
            for (int x = 0; x < L[0]; x++) {
                cplx acc[3], tmp[3];
                const cplx *here = in + site3(L, x, y, z) * 3;
                for (int c = 0; c < 3; c++)
                    acc[c] = -6.0 * here[c];
                for (int mu = 0; mu < 3; mu++) {
                    int xs, ys, zs;
                    shifted(L, x, y, z, mu, 2, &xs, &ys, &zs);
                    matvec(twolink(L, W, x, y, z, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);
                    for (int c = 0; c < 3; c++)
                        acc[c] += tmp[c];
                    shifted(L, x, y, z, mu, -2, &xs, &ys, &zs);
                    matvec_dag(twolink(L, W, xs, ys, zs, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);
                    for (int c = 0; c < 3; c++)
                        acc[c] += tmp[c];
                }
                cplx *o = out + site3(L, x, y, z) * 3;
                for (int c = 0; c < 3; c++)
                    o[c] = 0.25 * acc[c];
            }
}

/*
 * Two-link 3D Laplacian on time slice t, second form (eq. tlLapl2), with no
 * two-link field: each direction is two successive one-link parallel
 * transports of the whole slice (the CPU algorithm the paper started from).
 *   forward : chi(x) = U_mu(x) psi(x+mu^),        then U_mu(x) chi(x+mu^)
 *   backward: xi(x)  = U_mu^dag(x-mu^) psi(x-mu^), then U_mu^dag(x-mu^) xi(x-mu^)
 */
void or_lap_oneplusone(const int L[4], const cplx *U, int t, const cplx *in, cplx *out)
{
    long V3 = (long)L[0] * L[1] * L[2];
    cplx *chi = malloc(sizeof(cplx) * 3 * V3);
    cplx *chi2 = malloc(sizeof(cplx) * 3 * V3);
    for (long i = 0; i < 3 * V3; i++)
        out[i] = -6.0 * in[i];
    for (int mu = 0; mu < 3; mu++) {
        for (int dir = 0; dir < 2; dir++) {
            const cplx *src = in;
            cplx *dst = chi;
            for (int hop = 0; hop < 2; hop++) {
                #pragma omp parallel for collapse(2) schedule(static)
                for (int z = 0; z < L[2]; z++)
                    for (int y = 0; y < L[1]; y++)
                        for (int x = 0; x < L[0]; x++) {
                            int xs, ys, zs;
                            cplx *d = dst + site3(L, x, y, z) * 3;
                            if (dir == 0) {
                                shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);
                                matvec(link(L, U, x, y, z, t, mu), src + site3(L, xs, ys, zs) * 3, d);
                            } else {
                                shifted(L, x, y, z, mu, -1, &xs, &ys, &zs);
                                matvec_dag(link(L, U, xs, ys, zs, t, mu), src + site3(L, xs, ys, zs) * 3, d);
                            }
                        }
                src = dst;
                dst = chi2;
            }
            for (long i = 0; i < 3 * V3; i++)
                out[i] += chi2[i];
        }
    }
    for (long i = 0; i < 3 * V3; i++)
        out[i] *= 0.25;
    free(chi);
    free(chi2);
}

/*
 * Two-link smearing (eq. tlSmear) of one colour-vector field on slice t:
 *   psi <- (1 + (sigma/n) Lap)^n psi,
 * taken literally as n repetitions of psi <- psi + (sigma/n) Lap psi with the
 * first Laplacian form.  No normalisation constant is applied.
 */
void or_smear(const int L[4], const cplx *W, int t, int n, double sigma, cplx *psi)
{
    long V3 = (long)L[0] * L[1] * L[2];
    cplx *lap = malloc(sizeof(cplx) * 3 * V3);
    double step = sigma / (double)n;
    for (int k = 0; k < n; k++) {
        or_lap_twolink(L, W, t, psi, lap);
        for (long i = 0; i < 3 * V3; i++)
            psi[i] += step * lap[i];
    }
    free(lap);
}

/* Smearing of n_rhs fields [n_rhs][Lz][Ly][Lx][3], RHS r living on slice t_of_rhs[r]. */
void or_smear_batch(const int L[4], const cplx *W, int n_rhs, const int *t_of_rhs,
                    int n, double sigma, cplx *psi)
{
    long V3 = (long)L[0] * L[1] * L[2];
    for (int r = 0; r < n_rhs; r++)
        or_smear(L, W, t_of_rhs[r], n, sigma, psi + (long)r * 3 * V3);
}

/*
 * One-link hopping operator H of Sec. 2 on slice t (three spatial directions):
 *   (H psi)(x) = sum_mu [ U_mu(x) psi(x+mu^) + U_mu^dag(x-mu^) psi(x-mu^) ].
 */
void or_hop_onelink(const int L[4], const cplx *U, int t, const cplx *in, cplx *out)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < L[2]; z++)
        for (int y = 0; y < L[1]; y++)
            for (int x = 0; x < L[0]; x++) {
                cplx acc[3] = {0, 0, 0}, tmp[3];
                for (int mu = 0; mu < 3; mu++) {
                    int xs, ys, zs;
                    shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);
                    matvec(link(L, U, x, y, z, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);
                    for (int a = 0; a < 3; a++) acc[a] += tmp[a];
                    shifted(L, x, y, z, mu, -1, &xs, &ys, &zs);
                    matvec_dag(link(L, U, xs, ys, zs, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);
                    for (int a = 0; a < 3; a++) acc[a] += tmp[a];
                }
                cplx *o = out + site3(L, x, y, z) * 3;
                for (int a = 0; a < 3; a++) o[a] = acc[a];
            }
}

/*
 * One-link 3D Laplacian of Sec. 2 (lattice spacing 1), nabla^2 = H - 6:
 *   (nabla^2 psi)(x) = sum_mu [ U_mu(x) psi(x+mu^) - 2 psi(x) + U_mu^dag(x-mu^) psi(x-mu^) ],
 * written out per direction, independently of or_hop_onelink.
 */
void or_lap_onelink(const int L[4], const cplx *U, int t, const cplx *in, cplx *out)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < L[2]; z++)
        for (int y = 0; y < L[1]; y++)
            for (int x = 0; x < L[0]; x++) {
                const cplx *c = in + site3(L, x, y, z) * 3;
                cplx acc[3] = {0, 0, 0};
                for (int mu = 0; mu < 3; mu++) {
                    int xf, yf, zf, xb, yb, zb;
                    cplx f[3], b[3];
                    shifted(L, x, y, z, mu, 1, &xf, &yf, &zf);
                    shifted(L, x, y, z, mu, -1, &xb, &yb, &zb);
                    matvec(link(L, U, x, y, z, t, mu), in + site3(L, xf, yf, zf) * 3, f);
                    matvec_dag(link(L, U, xb, yb, zb, t, mu), in + site3(L, xb, yb, zb) * 3, b);
                    for (int a = 0; a < 3; a++) acc[a] += f[a] - 2.0 * c[a] + b[a];
                }
                cplx *o = out + site3(L, x, y, z) * 3;
                for (int a = 0; a < 3; a++) o[a] = acc[a];
            }
}

/*
 * Gaussian smearing in the hopping form (eq. gsmear without its constant C):
 *   psi <- (1 + alpha H)^n psi, as n repetitions of psi <- psi + alpha H psi.
 */
void or_gsmear_hop(const int L[4], const cplx *U, int t, int n, double alpha, cplx *psi)
{
    long V3 = (long)L[0] * L[1] * L[2];
    cplx *h = malloc(sizeof(cplx) * 3 * V3);
    for (int k = 0; k < n; k++) {
        or_hop_onelink(L, U, t, psi, h);
        for (long i = 0; i < 3 * V3; i++)
            psi[i] += alpha * h[i];
    }
    free(h);
}

/*
 * One-link smearing in the Laplacian form of Sec. 2 with the width parameter of
 * eq. tlSmear:  psi <- (1 + (sigma/n) nabla^2)^n psi, n literal repetitions.
 * By the identity that follows eq. gsmear, (1 + alpha H)^n = (1 + 6 alpha)^n
 * (1 + alpha' nabla^2)^n with alpha' = alpha / (1 + 6 alpha), i.e. sigma = n alpha'.
 */
void or_smear_onelink(const int L[4], const cplx *U, int t, int n, double sigma, cplx *psi)
{
    long V3 = (long)L[0] * L[1] * L[2];
    cplx *lap = malloc(sizeof(cplx) * 3 * V3);
    double step = sigma / (double)n;
    for (int k = 0; k < n; k++) {
        or_lap_onelink(L, U, t, psi, lap);
        for (long i = 0; i < 3 * V3; i++)
            psi[i] += step * lap[i];
    }
    free(lap);
}

void or_smear_onelink_batch(const int L[4], const cplx *U, int n_rhs, const int *t_of_rhs,
                            int n, double sigma, cplx *psi)
{
    long V3 = (long)L[0] * L[1] * L[2];
    for (int r = 0; r < n_rhs; r++)
        or_smear_onelink(L, U, t_of_rhs[r], n, sigma, psi + (long)r * 3 * V3);
}

/* sum_x |psi(x)|^2 over n_sites colour vectors, plain sequential FP64 sum: the slice
 * sum over x of a two-point correlation function C(t) (Sec. 1) with sink = source. */
double or_norm2(long n_sites, const cplx *psi)
{
    double s = 0.0;
    for (long i = 0; i < 3 * n_sites; i++)
        s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

/* <phi, psi> = sum_x phi(x)^dag psi(x) (conjugate-linear in phi): the slice sum over x
 * of a two-point correlation function C(t) (Sec. 1) contracting two colour vectors. */
void or_dot(long n_sites, const cplx *phi, const cplx *psi, double *re, double *im)
{
    cplx s = 0;
    for (long i = 0; i < 3 * n_sites; i++)
        s += conj(phi[i]) * psi[i];
    *re = creal(s);
    *im = cimag(s);
}

/* |psi(x)| per site, the quantity plotted for smeared point sources in Fig. 1. */
void or_site_norms(long n_sites, const cplx *psi, double *out)
{
    for (long i = 0; i < n_sites; i++) {
        double s = 0.0;
        for (int c = 0; c < 3; c++)
            s += creal(psi[3 * i + c]) * creal(psi[3 * i + c]) + cimag(psi[3 * i + c]) * cimag(psi[3 * i + c]);
        out[i] = sqrt(s);
    }
}

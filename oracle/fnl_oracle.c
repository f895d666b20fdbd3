/*
 * fnl_oracle.c -- plain FP64 CPU oracle for the local-f_NL CMB map generator
 * (Elsner & Wandelt, "Improved simulation of non-Gaussian temperature and
 * polarization CMB maps").
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark.  The product path never links it.
 *
 * What it computes, in the paper's order (Sect. 2, recipe steps (i)-(v)):
 *   (i)   Phi_L,lm(r_i) = sum_j F_l,ij n_lm(r_j)           (Sect. 2, the
 *         correlated draw Phi_L = P^{1/2} g under Eq. cov_phi)
 *   (ii)  synthesis of Phi_L(r_i) on a Gauss-Legendre grid
 *   (iii) Phi_NL = Phi_L^2 - <Phi_L^2>                      (Eq. phinldef)
 *   (iv)  analysis back to Phi_NL,lm(r_i)
 *   (v)   a^X_lm = sum_i w_i r_i^2 X_l(r_i) [Phi_L + f_NL Phi_NL]_lm(r_i)
 *         (Eq. phi2alm_r as a quadrature sum; a = a_L + f_NL a_NL, Sect. 2)
 * The transforms are the plain sums: a direct three-term Legendre
 * recurrence and a naive ring DFT with an integer-indexed twiddle table.
 * With ntheta >= (3L+1)/2 rings and nphi >= 3L+1 pixels the square of a
 * band-limited field is integrated exactly, so the result equals the
 * Gaunt-integral definition of Phi_NL to rounding.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 * Loops over rings (synthesis) and over m (analysis) run in parallel; every
 * accumulation is done in a fixed order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fnl_oracle.h"

#define ORC_PI 3.14159265358979323846264338327950288

static long nlm_of(int L) { return (long)(L + 1) * (L + 2) / 2; }
static long idx_of(int l, int m) { return (long)l * (l + 1) / 2 + m; }

/* ------------------------------------------------------------------ grid */

/* Gauss-Legendre rule by Newton's method on P_n, with P_n and P_{n-1} from
 * Bonnet's recurrence (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1} and the
 * classical first guess cos(pi (k + 3/4) / (n + 1/2)).                    */
int orc_gl_grid(int n, double *x, double *w)
{
    if (n < 1 || !x || !w) return -1;
    for (int k = 0; k < n; k++) {
        double z = cos(ORC_PI * (k + 0.75) / (n + 0.5));
        double dpn = 1.0;
        int extra = 0;
        for (int it = 0; it < 100; it++) {
            /* p1 = P_n(z), p0 = P_{n-1}(z) */
            double p0 = 1.0, p1 = z;
            for (int l = 1; l < n; l++) {
                double p2 = ((2.0 * l + 1.0) * z * p1 - l * p0) / (l + 1.0);
                p0 = p1;
                p1 = p2;
            }
            /* P_n'(z) = n (z P_n - P_{n-1}) / (z^2 - 1) */
            dpn = n * (z * p1 - p0) / (z * z - 1.0);
            if (extra) break; /* derivative at the converged node */
            double dz = p1 / dpn;
            z -= dz;
            if (fabs(dz) < 1e-14) extra = 1; /* one more step, then stop */
        }
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
    return 0;
}

/* ------------------------------------------------- associated Legendre */

/* lambda_mm(x) = (-1)^m sqrt((2m+1)!! / (4 pi (2m)!!)) sin^m theta, built
 * as lambda_00 = 1/sqrt(4 pi), lambda_mm = -sqrt((2m+1)/(2m)) s lambda_{m-1,m-1}. */
static double lambda_mm_step(int m, double s, double prev)
{
    return -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * prev;
}

/* Column l = m..L of lambda_lm(x), given lambda_mm:
 *   lambda_{m+1,m} = sqrt(2m+3) x lambda_mm
 *   lambda_lm = a_lm (x lambda_{l-1,m} - b_lm lambda_{l-2,m}),
 *   a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)). */
static void lambda_column(int L, int m, double x, double lmm, double *col)
{
    col[0] = lmm;
    if (m + 1 <= L) col[1] = sqrt(2.0 * m + 3.0) * x * lmm;
    for (int l = m + 2; l <= L; l++) {
        double l2 = (double)l * l, m2 = (double)m * m, lm1 = l - 1.0;
        double a = sqrt((4.0 * l2 - 1.0) / (l2 - m2));
        double b = sqrt((lm1 * lm1 - m2) / (4.0 * lm1 * lm1 - 1.0));
        col[l - m] = a * (x * col[l - m - 1] - b * col[l - m - 2]);
    }
}

void orc_lambda_all(int L, double x, double *lam)
{
    double s = sqrt((1.0 - x) * (1.0 + x));
    double lmm = 1.0 / sqrt(4.0 * ORC_PI);
    double *col = (double *)malloc(sizeof(double) * (L + 1));
    for (int m = 0; m <= L; m++) {
        if (m > 0) lmm = lambda_mm_step(m, s, lmm);
        lambda_column(L, m, x, lmm, col);
        for (int l = m; l <= L; l++) lam[idx_of(l, m)] = col[l - m];
    }
    free(col);
}

/* lambda_mm(x_k) for all m, k: table[m * nth + k]. */
static double *lambda_mm_table(int L, int nth, const double *x)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)(L + 1) * nth);
    for (int k = 0; k < nth; k++) {
        double s = sqrt((1.0 - x[k]) * (1.0 + x[k]));
        double v = 1.0 / sqrt(4.0 * ORC_PI);
        t[k] = v;
        for (int m = 1; m <= L; m++) {
            v = lambda_mm_step(m, s, v);
            t[(size_t)m * nth + k] = v;
        }
    }
    return t;
}

/* ------------------------------------------------------ ring transforms */

static void twiddles(int n, double *c, double *s)
{
    for (int q = 0; q < n; q++) {
        double a = 2.0 * ORC_PI * q / n;
        c[q] = cos(a);
        s[q] = sin(a);
    }
}

/* General synthesis: map[k][j] = ring_w[k] * sum_m cm[m] Re[G_m(k) e^{i m phi_j}],
 * G_m(k) = sum_l lambda_lm(x_k) alm_lm (Im of m = 0 dropped).  ring_w may be
 * NULL (all ones).                                                         */
static void synth_general(int L, int nth, int nph, const double *x,
                          const double *ring_w, const double *cm,
                          const double *alm, double *map)
{
    double *tc = (double *)malloc(sizeof(double) * nph);
    double *ts = (double *)malloc(sizeof(double) * nph);
    twiddles(nph, tc, ts);
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (L + 1));
        double *gre = (double *)malloc(sizeof(double) * (L + 1));
        double *gim = (double *)malloc(sizeof(double) * (L + 1));
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < nth; k++) {
            double s = sqrt((1.0 - x[k]) * (1.0 + x[k]));
            double lmm = 1.0 / sqrt(4.0 * ORC_PI);
            for (int m = 0; m <= L; m++) {
                if (m > 0) lmm = lambda_mm_step(m, s, lmm);
                lambda_column(L, m, x[k], lmm, col);
                double re = 0.0, im = 0.0;
                for (int l = m; l <= L; l++) {
                    long i = idx_of(l, m);
                    re += col[l - m] * alm[2 * i];
                    if (m > 0) im += col[l - m] * alm[2 * i + 1];
                }
                gre[m] = re;
                gim[m] = im;
            }
            double rw = ring_w ? ring_w[k] : 1.0;
            for (int j = 0; j < nph; j++) {
                double acc = 0.0;
                int q = 0; /* (m * j) mod nph */
                for (int m = 0; m <= L; m++) {
                    acc += cm[m] * (gre[m] * tc[q] - gim[m] * ts[q]);
                    q += j;
                    if (q >= nph) q -= nph;
                }
                map[(size_t)k * nph + j] = rw * acc;
            }
        }
        free(col);
        free(gre);
        free(gim);
    }
    free(tc);
    free(ts);
}

/* General analysis: alm_lm = outscale[m] * sum_k ring_w[k] lambda_lm(x_k)
 * sum_j map[k][j] e^{-i m phi_j}; for m = 0 the imaginary part is zero.    */
static void anal_general(int L, int nth, int nph, const double *x,
                         const double *ring_w, const double *outscale,
                         const double *map, double *alm)
{
    double *tc = (double *)malloc(sizeof(double) * nph);
    double *ts = (double *)malloc(sizeof(double) * nph);
    twiddles(nph, tc, ts);
    double *lmm = lambda_mm_table(L, nth, x);
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (L + 1));
        double *are = (double *)malloc(sizeof(double) * (L + 1));
        double *aim = (double *)malloc(sizeof(double) * (L + 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m <= L; m++) {
            for (int l = m; l <= L; l++) are[l - m] = aim[l - m] = 0.0;
            for (int k = 0; k < nth; k++) {
                const double *row = map + (size_t)k * nph;
                double fre = 0.0, fim = 0.0;
                int q = 0;
                for (int j = 0; j < nph; j++) {
                    fre += row[j] * tc[q];
                    fim -= row[j] * ts[q];
                    q += m;
                    if (q >= nph) q -= nph;
                }
                double rw = ring_w[k];
                lambda_column(L, m, x[k], lmm[(size_t)m * nth + k], col);
                for (int l = m; l <= L; l++) {
                    are[l - m] += rw * col[l - m] * fre;
                    aim[l - m] += rw * col[l - m] * fim;
                }
            }
            for (int l = m; l <= L; l++) {
                long i = idx_of(l, m);
                alm[2 * i] = outscale[m] * are[l - m];
                alm[2 * i + 1] = (m == 0) ? 0.0 : outscale[m] * aim[l - m];
            }
        }
        free(col);
        free(are);
        free(aim);
    }
    free(lmm);
    free(tc);
    free(ts);
}

static double *cm_synthesis(int L)
{
    double *c = (double *)malloc(sizeof(double) * (L + 1));
    for (int m = 0; m <= L; m++) c[m] = (m == 0) ? 1.0 : 2.0;
    return c;
}

static double *ones(int n)
{
    double *c = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; i++) c[i] = 1.0;
    return c;
}

static double *pixel_weights(int nth, int nph, const double *wq)
{
    double *r = (double *)malloc(sizeof(double) * nth);
    for (int k = 0; k < nth; k++) r[k] = wq[k] * 2.0 * ORC_PI / nph;
    return r;
}

void orc_synth(int L, int nth, int nph, const double *x, const double *alm,
               double *map)
{
    double *cm = cm_synthesis(L);
    synth_general(L, nth, nph, x, NULL, cm, alm, map);
    free(cm);
}

void orc_anal(int L, int nth, int nph, const double *x, const double *wq,
              const double *map, double *alm)
{
    double *rw = pixel_weights(nth, nph, wq);
    double *sc = ones(L + 1);
    anal_general(L, nth, nph, x, rw, sc, map, alm);
    free(sc);
    free(rw);
}

/* -------------------------------------------- spin-2 harmonics (Q, U) */

/* Spin-weighted Legendre functions sl_lm(x), l = 0..L, at one (m, s), for
 * sY_lm(theta, phi) = sl_lm(cos theta) e^{i m phi} with the Condon-Shortley
 * phase and sY_lm obtained from Y_lm by the spin-raising (eth) and -lowering
 * operators.  Start: at l0 = max(|m|, |s|) the closed-form sum for sY_lm
 * (Goldberg et al. 1967) has a single term,
 *   (-1)^m sqrt((l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!))
 *     C(l-s, r) C(l+s, r+s-m) (-1)^(l-r-s) sin^(2l-k)(theta/2) cos^k(theta/2),
 * k = 2r + s - m, evaluated in log form.  Then the three-term recurrence of
 * the Wigner d-functions in l, normalised by sqrt((2l+1)/(4 pi)):
 *   l sqrt(P_{l+1}) f_{l+1} / sqrt(2l+3)
 *     = sqrt(2l+1) (l(l+1) x + m s) f_l - (l+1) sqrt(P_l / (2l-1)) f_{l-1},
 *   P_j = (j^2 - m^2)(j^2 - s^2).                                          */
static void spin_lambda(int L, int m, int s, double x, double *out)
{
    for (int l = 0; l <= L; l++) out[l] = 0.0;
    int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    int l0 = am > as ? am : as;
    if (l0 > L) return;
    int l = l0, r0 = -1;
    for (int r = 0; r <= l - s; r++) {
        int j = r + s - m;
        if (j >= 0 && j <= l + s) { r0 = r; break; }
    }
    double sh = sqrt(0.5 * (1.0 - x)), ch = sqrt(0.5 * (1.0 + x));
    int k = 2 * r0 + s - m;
    double lg = 0.5 * (lgamma(l + m + 1.0) + lgamma(l - m + 1.0) + log(2.0 * l + 1.0) -
                       log(4.0 * ORC_PI) - lgamma(l + s + 1.0) - lgamma(l - s + 1.0));
    lg += lgamma(l - s + 1.0) - lgamma(r0 + 1.0) - lgamma(l - s - r0 + 1.0);
    lg += lgamma(l + s + 1.0) - lgamma(r0 + s - m + 1.0) - lgamma(l + m - r0 + 1.0);
    double f0;
    if ((2 * l - k > 0 && sh == 0.0) || (k > 0 && ch == 0.0)) {
        f0 = 0.0;
    } else {
        lg += (2 * l - k) * log(sh > 0.0 ? sh : 1.0) + k * log(ch > 0.0 ? ch : 1.0);
        int sgn = ((m + (l - r0 - s)) % 2 == 0) ? 1 : -1;
        f0 = sgn * exp(lg);
    }
    out[l0] = f0;
    double fm = 0.0, f = f0;
    for (l = l0; l < L; l++) {
        double P1 = ((double)(l + 1) * (l + 1) - (double)m * m) * ((double)(l + 1) * (l + 1) - (double)s * s);
        double P0 = ((double)l * l - (double)m * m) * ((double)l * l - (double)s * s);
        double fn = sqrt(2.0 * l + 3.0) / (l * sqrt(P1)) *
                    (sqrt(2.0 * l + 1.0) * ((double)l * (l + 1) * x + (double)m * s) * f -
                     (l + 1) * sqrt(P0 / (2.0 * l - 1.0)) * fm);
        out[l + 1] = fn;
        fm = f;
        f = fn;
    }
}

void orc_spin_lambda(int lmax, int m, int s, double x, double *out)
{
    spin_lambda(lmax, m, s, x, out);
}

/* Q and U of a pure-E polarisation field (B = 0) on rings x[0..nx):
 *   Q + i U = -sum_{l>=2} sum_{m=-l..l} aE_lm 2Y_lm,
 * with aE_{l,-m} = (-1)^m conj(aE_lm), every m summed directly, and a naive
 * ring DFT with an integer twiddle index.                                  */
void orc_synth_qu(int L, int nx, int nph, const double *x, const double *almE, double *Q,
                  double *U)
{
    double *cs = (double *)malloc(sizeof(double) * 2 * nph);
    for (int j = 0; j < nph; j++) {
        cs[2 * j] = cos(2.0 * ORC_PI * j / nph);
        cs[2 * j + 1] = sin(2.0 * ORC_PI * j / nph);
    }
#pragma omp parallel
    {
        double *lam = (double *)malloc(sizeof(double) * (L + 1));
        double *gr = (double *)malloc(sizeof(double) * (2 * L + 1));
        double *gi = (double *)malloc(sizeof(double) * (2 * L + 1));
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < nx; k++) {
            for (int m = -L; m <= L; m++) {
                spin_lambda(L, m, 2, x[k], lam);
                int am = m < 0 ? -m : m;
                double sr = 0.0, si = 0.0;
                for (int l = (am > 2 ? am : 2); l <= L; l++) {
                    long id = idx_of(l, am);
                    double ar = almE[2 * id], ai = am == 0 ? 0.0 : almE[2 * id + 1];
                    if (m < 0) {  /* (-1)^m conj */
                        double sg = (am % 2) ? -1.0 : 1.0;
                        ar = sg * ar;
                        ai = -sg * ai;
                    }
                    sr -= ar * lam[l];
                    si -= ai * lam[l];
                }
                gr[m + L] = sr;
                gi[m + L] = si;
            }
            for (int j = 0; j < nph; j++) {
                double qr = 0.0, qi = 0.0;
                for (int m = -L; m <= L; m++) {
                    long t = ((long)m * j) % nph;
                    if (t < 0) t += nph;
                    double c = cs[2 * t], sn = cs[2 * t + 1];
                    qr += gr[m + L] * c - gi[m + L] * sn;
                    qi += gr[m + L] * sn + gi[m + L] * c;
                }
                Q[(size_t)k * nph + j] = qr;
                U[(size_t)k * nph + j] = qi;
            }
        }
        free(lam);
        free(gr);
        free(gi);
    }
    free(cs);
}

/* ------------------------------------------------------------ the model */

static int problem_ok(const orc_problem *P)
{
    if (!P || P->lmax < 0 || P->nshell < 1) return 0;
    if (P->ntheta < P->lmax + 1) return 0;
    if (P->nphi < 2 * P->lmax + 1) return 0;
    if (!P->r || !P->w || !P->filter || !P->alpha || !P->beta) return 0;
    if (P->mean_mode != ORC_MEAN_SAMPLE && P->mean_mode != ORC_MEAN_ENSEMBLE) return 0;
    return 1;
}

/* W^X_li = w_i r_i^2 X_l(r_i): the quadrature sum of Eq. phi2alm_r. */
static void radial_weights(const orc_problem *P, double *WT, double *WE)
{
    int L = P->lmax, N = P->nshell;
    for (int l = 0; l <= L; l++)
        for (int i = 0; i < N; i++) {
            double base = P->w[i] * P->r[i] * P->r[i];
            WT[(size_t)l * N + i] = base * P->alpha[(size_t)l * N + i];
            WE[(size_t)l * N + i] = base * P->beta[(size_t)l * N + i];
        }
}

/* Filter for the output shells with mask[i] != 0 (all when mask is NULL);
 * the other rows of phi are left untouched. */
static void filter_rows(const orc_problem *P, const double *noise, const int *mask, double *phi)
{
    int L = P->lmax, N = P->nshell;
    long nlm = nlm_of(L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int l = 0; l <= L; l++) {
        const double *F = P->filter + (size_t)l * N * N;
        for (int m = 0; m <= l; m++) {
            long id = idx_of(l, m);
            for (int i = 0; i < N; i++) {
                if (mask && !mask[i]) continue;
                double re = 0.0, im = 0.0;
                for (int j = 0; j < N; j++) {
                    double f = F[(size_t)i * N + j];
                    re += f * noise[2 * ((size_t)j * nlm + id)];
                    im += f * noise[2 * ((size_t)j * nlm + id) + 1];
                }
                phi[2 * ((size_t)i * nlm + id)] = re;
                phi[2 * ((size_t)i * nlm + id) + 1] = (m == 0) ? 0.0 : im;
            }
        }
    }
}

void orc_filter(const orc_problem *P, const double *noise, double *phi)
{
    filter_rows(P, noise, NULL, phi);
}

/* Ensemble variance <Phi_L^2>(r_i) = sum_l (2l+1)/(4 pi) (F_l F_l^T)_ii:
 * the covariance of the draw summed over m with the addition theorem.      */
static double ensemble_mu(const orc_problem *P, int i)
{
    int L = P->lmax, N = P->nshell;
    double mu = 0.0;
    for (int l = 0; l <= L; l++) {
        const double *row = P->filter + (size_t)l * N * N + (size_t)i * N;
        double s = 0.0;
        for (int j = 0; j < N; j++) s += row[j] * row[j];
        mu += (2.0 * l + 1.0) / (4.0 * ORC_PI) * s;
    }
    return mu;
}

/* Sky mean of map^2 with the grid's exact pixel weights. */
static double sample_mu(int nth, int nph, const double *wq, const double *map)
{
    double tot = 0.0;
    for (int k = 0; k < nth; k++) {
        double ring = 0.0;
        for (int j = 0; j < nph; j++) {
            double v = map[(size_t)k * nph + j];
            ring += v * v;
        }
        tot += wq[k] * (2.0 * ORC_PI / nph) * ring;
    }
    return tot / (4.0 * ORC_PI);
}

static int shell_used(const double *WT, const double *WE, int L, int N, int i)
{
    for (int l = 0; l <= L; l++)
        if (WT[(size_t)l * N + i] != 0.0 || WE[(size_t)l * N + i] != 0.0) return 1;
    return 0;
}

int orc_forward(const orc_problem *P, const double *noise, double fnl,
                double *aT, double *aE, double *aT_lin, double *aE_lin,
                double *aT_nl, double *aE_nl,
                double *phiL_out, double *phiNL_out, double *mu_out)
{
    if (!problem_ok(P) || !noise) return -1;
    int L = P->lmax, N = P->nshell, nth = P->ntheta, nph = P->nphi;
    long nlm = nlm_of(L);

    double *x = (double *)malloc(sizeof(double) * nth);
    double *wq = (double *)malloc(sizeof(double) * nth);
    orc_gl_grid(nth, x, wq);

    double *WT = (double *)malloc(sizeof(double) * (L + 1) * N);
    double *WE = (double *)malloc(sizeof(double) * (L + 1) * N);
    radial_weights(P, WT, WE);

    /* (i) correlated Gaussian potential; a node whose radial weights are all
     * zero contributes nothing, so it is only evaluated when asked for. */
    int *used = (int *)malloc(sizeof(int) * N);
    for (int i = 0; i < N; i++)
        used[i] = shell_used(WT, WE, L, N, i) || phiL_out || phiNL_out || mu_out;
    double *phiL = (double *)calloc(2 * nlm * (size_t)N, sizeof(double));
    filter_rows(P, noise, used, phiL);

    double *sLT = (double *)calloc(2 * nlm, sizeof(double));
    double *sLE = (double *)calloc(2 * nlm, sizeof(double));
    double *sNT = (double *)calloc(2 * nlm, sizeof(double));
    double *sNE = (double *)calloc(2 * nlm, sizeof(double));
    double *map = (double *)malloc(sizeof(double) * (size_t)nth * nph);
    double *pnl = (double *)malloc(sizeof(double) * 2 * nlm);

    for (int i = 0; i < N; i++) {
        const double *pl = phiL + 2 * nlm * (size_t)i;
        /* (v) linear part of the radial sum */
        for (int l = 0; l <= L; l++) {
            double wt = WT[(size_t)l * N + i], we = WE[(size_t)l * N + i];
            for (int m = 0; m <= l; m++) {
                long id = idx_of(l, m);
                sLT[2 * id] += wt * pl[2 * id];
                sLT[2 * id + 1] += wt * pl[2 * id + 1];
                sLE[2 * id] += we * pl[2 * id];
                sLE[2 * id + 1] += we * pl[2 * id + 1];
            }
        }
        if (!used[i]) continue;
        /* (ii) synthesis, (iii) square and remove the mean, (iv) analysis */
        orc_synth(L, nth, nph, x, pl, map);
        double mu = (P->mean_mode == ORC_MEAN_SAMPLE) ? sample_mu(nth, nph, wq, map)
                                                      : ensemble_mu(P, i);
        if (mu_out) mu_out[i] = mu;
        size_t npix = (size_t)nth * nph;
        for (size_t q = 0; q < npix; q++) map[q] = map[q] * map[q] - mu;
        orc_anal(L, nth, nph, x, wq, map, pnl);
        if (phiNL_out) memcpy(phiNL_out + 2 * nlm * (size_t)i, pnl, sizeof(double) * 2 * nlm);
        /* (v) non-linear part of the radial sum */
        for (int l = 0; l <= L; l++) {
            double wt = WT[(size_t)l * N + i], we = WE[(size_t)l * N + i];
            for (int m = 0; m <= l; m++) {
                long id = idx_of(l, m);
                sNT[2 * id] += wt * pnl[2 * id];
                sNT[2 * id + 1] += wt * pnl[2 * id + 1];
                sNE[2 * id] += we * pnl[2 * id];
                sNE[2 * id + 1] += we * pnl[2 * id + 1];
            }
        }
    }

    /* a = a_L + f_NL a_NL */
    for (long q = 0; q < 2 * nlm; q++) {
        if (aT) aT[q] = sLT[q] + fnl * sNT[q];
        if (aE) aE[q] = sLE[q] + fnl * sNE[q];
        if (aT_lin) aT_lin[q] = sLT[q];
        if (aE_lin) aE_lin[q] = sLE[q];
        if (aT_nl) aT_nl[q] = sNT[q];
        if (aE_nl) aE_nl[q] = sNE[q];
    }
    if (phiL_out) memcpy(phiL_out, phiL, sizeof(double) * 2 * nlm * N);

    free(used);
    free(pnl);
    free(map);
    free(sLT);
    free(sLE);
    free(sNT);
    free(sNE);
    free(phiL);
    free(WT);
    free(WE);
    free(x);
    free(wq);
    return 0;
}

/* Adjoint (reverse mode) of orc_forward for a real loss, with the inner
 * product Re sum conj(u) v over the stored coefficients (m >= 0):
 *   Phibar_i        = sum_X W^X_i abar^X                  (transposed radial sum)
 *   grad f_NL       = sum_X Re <abar^X, a^X_NL>
 *   ghat_i(pixel)   = omega_pix sum_{l,m>=0} Re[Phibar'_lm lambda_lm e^{i m phi}]
 *                     (transposed analysis; Phibar'_00 := 0 for the sample
 *                     mean, whose own derivative cancels the (0,0) term)
 *   phibar_i        = 2 f_NL Phi_L,i(pixel) ghat_i        (derivative of the square)
 *   Phibar_L,i     += c_m sum_pix phibar_i lambda_lm e^{-i m phi}  (transposed synthesis)
 *   grad n_j        = sum_i F_l,ij Phibar_L,i             (transposed filter)
 * grad f_NL is evaluated as sum_i sum_pix Phi_L,i^2 ghat_i (minus the
 * ensemble-mean term), which equals sum_X Re <abar^X, a^X_NL>.            */
int orc_adjoint(const orc_problem *P, const double *noise, double fnl,
                const double *gT, const double *gE,
                double *grad_n, double *grad_fnl)
{
    if (!problem_ok(P) || !noise || !gT || !gE || !grad_n || !grad_fnl) return -1;
    int L = P->lmax, N = P->nshell, nth = P->ntheta, nph = P->nphi;
    long nlm = nlm_of(L);

    double *x = (double *)malloc(sizeof(double) * nth);
    double *wq = (double *)malloc(sizeof(double) * nth);
    orc_gl_grid(nth, x, wq);
    double *WT = (double *)malloc(sizeof(double) * (L + 1) * N);
    double *WE = (double *)malloc(sizeof(double) * (L + 1) * N);
    radial_weights(P, WT, WE);

    /* a node whose radial weights are all zero receives no cotangent */
    int *used = (int *)malloc(sizeof(int) * N);
    for (int i = 0; i < N; i++) used[i] = shell_used(WT, WE, L, N, i);
    double *phiL = (double *)calloc(2 * nlm * (size_t)N, sizeof(double));
    filter_rows(P, noise, used, phiL);
    double *pbar = (double *)calloc(2 * nlm * (size_t)N, sizeof(double));

    double *pixw = pixel_weights(nth, nph, wq);
    double *one_m = ones(L + 1);   /* c'_m = 1: each stored (l, m) once */
    double *one_k = ones(nth);     /* unit ring weights                 */
    double *cm = cm_synthesis(L);
    double *f = (double *)malloc(sizeof(double) * (size_t)nth * nph);
    double *g = (double *)malloc(sizeof(double) * (size_t)nth * nph);
    double *dir = (double *)malloc(sizeof(double) * 2 * nlm);
    double *xs = (double *)malloc(sizeof(double) * 2 * nlm);
    double gf = 0.0;
    size_t npix = (size_t)nth * nph;

    for (int i = 0; i < N; i++) {
        if (!used[i]) continue;
        /* transposed radial sum */
        for (int l = 0; l <= L; l++) {
            double wt = WT[(size_t)l * N + i], we = WE[(size_t)l * N + i];
            for (int m = 0; m <= l; m++) {
                long id = idx_of(l, m);
                dir[2 * id] = wt * gT[2 * id] + we * gE[2 * id];
                dir[2 * id + 1] = (m == 0) ? 0.0 : wt * gT[2 * id + 1] + we * gE[2 * id + 1];
            }
        }
        double *pb = pbar + 2 * nlm * (size_t)i;
        memcpy(pb, dir, sizeof(double) * 2 * nlm);

        /* ghat = transposed analysis of Phibar' (sum over m >= 0, weight 1) */
        double d00 = dir[0];
        if (P->mean_mode == ORC_MEAN_SAMPLE) dir[0] = 0.0;
        synth_general(L, nth, nph, x, pixw, one_m, dir, g);
        /* Phi_L map of this shell */
        orc_synth(L, nth, nph, x, phiL + 2 * nlm * (size_t)i, f);
        double part = 0.0;
        for (size_t q = 0; q < npix; q++) part += f[q] * f[q] * g[q];
        if (P->mean_mode == ORC_MEAN_ENSEMBLE)
            part -= sqrt(4.0 * ORC_PI) * ensemble_mu(P, i) * d00;
        gf += part;
        /* derivative of the square, then transposed synthesis */
        for (size_t q = 0; q < npix; q++) g[q] = 2.0 * fnl * f[q] * g[q];
        anal_general(L, nth, nph, x, one_k, cm, g, xs);
        for (long q = 0; q < 2 * nlm; q++) pb[q] += xs[q];
    }

    /* transposed filter */
#pragma omp parallel for schedule(dynamic, 4)
    for (int l = 0; l <= L; l++) {
        const double *F = P->filter + (size_t)l * N * N;
        for (int m = 0; m <= l; m++) {
            long id = idx_of(l, m);
            for (int j = 0; j < N; j++) {
                double re = 0.0, im = 0.0;
                for (int i = 0; i < N; i++) {
                    double fv = F[(size_t)i * N + j];
                    re += fv * pbar[2 * ((size_t)i * nlm + id)];
                    im += fv * pbar[2 * ((size_t)i * nlm + id) + 1];
                }
                grad_n[2 * ((size_t)j * nlm + id)] = re;
                grad_n[2 * ((size_t)j * nlm + id) + 1] = (m == 0) ? 0.0 : im;
            }
        }
    }
    *grad_fnl = gf;

    free(used);
    free(xs);
    free(dir);
    free(g);
    free(f);
    free(cm);
    free(one_m);
    free(one_k);
    free(pixw);
    free(pbar);
    free(phiL);
    free(WT);
    free(WE);
    free(x);
    free(wq);
    return 0;
}


/* ------------------------------------------------------ counter-based noise */

/* One Philox round: two 32x32 -> 64-bit products, words permuted and mixed
 * with the key (Salmon et al., SC'11, Sect. 4 and Table 1: multipliers
 * 0xD2511F53, 0xCD9E8D57; key increments 0x9E3779B9, 0xBB67AE85). */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2],
                       unsigned int out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
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

void orc_noise(int lmax, int nshell, unsigned long long seed, double *noise)
{
    const long long nlm = (long long)(lmax + 1) * (lmax + 2) / 2;
    const unsigned int key[2] = {(unsigned int)(seed & 0xffffffffu), (unsigned int)(seed >> 32)};
    const double two_m53 = 1.0 / 9007199254740992.0; /* 2^-53 */
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < nshell; j++)
        for (int l = 0; l <= lmax; l++)
            for (int m = 0; m <= l; m++) {
                const long long idx = (long long)l * (l + 1) / 2 + m;
                const unsigned int ctr[4] = {(unsigned int)(idx & 0xffffffffu),
                                             (unsigned int)((unsigned long long)idx >> 32),
                                             (unsigned int)j, 0x6e6f6973u};
                unsigned int x[4];
                orc_philox4x32_10(ctr, key, x);
                const uint64_t a = (((uint64_t)x[1] << 32) | x[0]) >> 11;
                const uint64_t b = (((uint64_t)x[3] << 32) | x[2]) >> 11;
                const double u1 = (double)(a + 1) * two_m53;
                const double u2 = (double)b * two_m53;
                const double rad = sqrt(-2.0 * log(u1));
                const double g0 = rad * cos(2.0 * pi * u2);
                const double g1 = rad * sin(2.0 * pi * u2);
                double *o = noise + 2 * ((size_t)j * nlm + idx);
                if (m == 0) {
                    o[0] = g0;
                    o[1] = 0.0;
                } else {
                    o[0] = g0 / sqrt(2.0);
                    o[1] = g1 / sqrt(2.0);
                }
            }
}

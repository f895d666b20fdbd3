/*
 * fnl_oracle.h -- plain FP64 CPU oracle for the local-f_NL CMB map generator
 * of Elsner & Wandelt, "Improved simulation of non-Gaussian temperature and
 * polarization CMB maps".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path includes, links or
 * calls this code: it exists so that tests/, the smoke check and the CPU
 * baseline leg of the benchmark have an independent, obviously correct
 * reference.  It shares no code with the HIP library.
 *
 * Conventions (all arrays row-major, FP64):
 *   alm index      idx(l, m) = l(l+1)/2 + m, 0 <= m <= l <= L,
 *                  complex values interleaved (re, im); Im a_l0 is ignored.
 *   harmonics      Y_lm = lambda_lm(cos theta) e^{i m phi}, orthonormal,
 *                  Condon-Shortley phase; real fields keep m >= 0 only.
 *   grid           Gauss-Legendre rings, x_k = cos theta_k descending (north
 *                  to south), phi_j = 2 pi j / nphi, pixel weight
 *                  omega_k * 2 pi / nphi.
 *   filter         [L+1][N][N], row i = output shell, column j = input shell.
 *   alpha, beta    [L+1][N]: temperature and E-mode real-space transfer
 *                  tables evaluated at the nodes.
 */
#ifndef FNL_ORACLE_H
#define FNL_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MEAN_SAMPLE = 0, ORC_MEAN_ENSEMBLE = 1 };

typedef struct {
    int lmax;            /* L                                             */
    int nshell;          /* N radial nodes                                */
    int ntheta;          /* Gauss-Legendre rings                          */
    int nphi;            /* pixels per ring                               */
    int mean_mode;       /* ORC_MEAN_SAMPLE or ORC_MEAN_ENSEMBLE          */
    const double *r;     /* [N] node radii                                */
    const double *w;     /* [N] quadrature weights                        */
    const double *filter;/* [L+1][N][N]                                   */
    const double *alpha; /* [L+1][N]                                      */
    const double *beta;  /* [L+1][N]                                      */
} orc_problem;

/* Gauss-Legendre nodes (descending) and weights of order n. 0 on success. */
int orc_gl_grid(int n, double *x, double *w);

/* lambda_lm(x) for all 0 <= m <= l <= L at one x, stored at idx(l, m). */
void orc_lambda_all(int lmax, double x, double *lam);

/* Synthesis of one band-limited real field onto the grid:
 * map[k][j] = sum_{l,m} c_m Re[alm_lm lambda_lm(x_k) e^{i m phi_j}],
 * c_0 = 1, c_m = 2.                                                      */
void orc_synth(int lmax, int ntheta, int nphi, const double *x,
               const double *alm, double *map);

/* Spin-weighted Legendre functions sl_lm(x) for l = 0..L at one (m, s):
 * sY_lm = sl_lm(cos theta) e^{i m phi}, raised from Y_lm by eth (Condon-
 * Shortley phase).  out [L+1], zero below l = max(|m|, |s|).               */
void orc_spin_lambda(int lmax, int m, int s, double x, double *out);

/* Stokes Q, U of a pure-E field on nx rings at x[] (any ring list), nph
 * pixels each: Q + i U = -sum_{l>=2, all m} aE_lm 2Y_lm.  Q, U [nx][nph].   */
void orc_synth_qu(int lmax, int nx, int nph, const double *x, const double *almE, double *Q,
                  double *U);

/* Analysis: alm_lm = sum_k omega_k (2 pi / nphi) sum_j map[k][j]
 * lambda_lm(x_k) e^{-i m phi_j}.                                           */
void orc_anal(int lmax, int ntheta, int nphi, const double *x,
              const double *wq, const double *map, double *alm);

/* Radial filter: phi[i][idx] = sum_j F_l[i][j] noise[j][idx] (Im of m = 0
 * dropped).  noise, phi: [N][n_lm] complex.                               */
void orc_filter(const orc_problem *P, const double *noise, double *phi);

/* Forward map generator.  noise: [N][n_lm] complex.  Every output pointer
 * may be NULL.  a*: [n_lm] complex.  phiL, phiNL: [N][n_lm] complex.
 * mu: [N].  Returns 0, or -1 on invalid arguments.                          */
int orc_forward(const orc_problem *P, const double *noise, double fnl,
                double *aT, double *aE, double *aT_lin, double *aE_lin,
                double *aT_nl, double *aE_nl,
                double *phiL, double *phiNL, double *mu);

/* Adjoint of orc_forward for a real loss.  gT, gE: cotangents
 * dLoss/dRe a + i dLoss/dIm a, [n_lm] complex.  grad_n: [N][n_lm] complex,
 * same convention, Im of m = 0 set to 0.  grad_fnl: one double.            */
int orc_adjoint(const orc_problem *P, const double *noise, double fnl,
                const double *gT, const double *gE,
                double *grad_n, double *grad_fnl);

/* Counter-based noise (regenerated from a seed instead of stored; the
 * paper's memory remark in Sect. 3).  Philox4x32 with 10 rounds (Salmon,
 * Moraes, Dror and Shaw, SC'11): counter (c0..c3), key (k0, k1) -> 4 words. */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2],
                       unsigned int out[4]);

/* noise[N][n_lm] complex for one realization seed: for shell j and index
 * idx = l(l+1)/2 + m, Philox of counter (idx mod 2^32, idx / 2^32, j,
 * 0x6e6f6973) under key (seed mod 2^32, seed / 2^32) gives words x0..x3;
 * U1 = (((x1 << 32 | x0) >> 11) + 1) 2^-53 in (0, 1],
 * U2 = ((x3 << 32 | x2) >> 11) 2^-53 in [0, 1); Box-Muller
 * g0 = sqrt(-2 ln U1) cos(2 pi U2), g1 = sqrt(-2 ln U1) sin(2 pi U2);
 * n = (g0, g1) / sqrt(2) for m > 0 and (g0, 0) for m = 0 (E|n|^2 = 1).       */
void orc_noise(int lmax, int nshell, unsigned long long seed, double *noise);

#ifdef __cplusplus
}
#endif
#endif

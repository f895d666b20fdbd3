/*
 * fnlsim.h -- C ABI of the MI355X (gfx950) local-f_NL CMB map generator.
 *
 * The library computes, for each realization, the temperature and E-mode
 * harmonic coefficients of a CMB sky with local-type non-Gaussianity
 * (Elsner & Wandelt, "Improved simulation of non-Gaussian temperature and
 * polarization CMB maps", Sect. 2, recipe steps (i)-(v)):
 *
 *   (a) Phi_L,lm(r_i) = sum_j F_l,ij n_lm(r_j)         correlated draw, the
 *       square root of the radial covariance of Eq. cov_phi applied to
 *       white noise;
 *   (b) synthesis of Phi_L(r_i) on an isolatitude Gauss-Legendre grid;
 *   (c) Phi_NL = Phi_L^2 - <Phi_L^2>                   Eq. phinldef;
 *   (d) analysis back to Phi_NL,lm(r_i);
 *   (e) a^X_lm = sum_i w_i r_i^2 X_l(r_i) [Phi_L + f_NL Phi_NL]_lm(r_i),
 *       X = alpha (T) or beta (E)                      Eq. phi2alm_r as a
 *       quadrature sum, with a = a_L + f_NL a_NL (Sect. 2).
 *
 * Besides that forward pass it offers the reverse pass (sim_backward), the
 * same passes with the noise regenerated from a seed instead of stored
 * (sim_noise, sim_forward_seeded, sim_backward_seeded; Sect. 3's memory
 * remark), launches over several uneven problems at once (sim_batch_*), the
 * greedy design of the radial quadrature nodes and weights
 * (sim_quadrature_design; Sect. 3), the T, Q, U maps of generated
 * coefficients (sim_tqu_maps; Sect. 3) and the cubic KSW statistic of
 * Sect. 4 (sim_ksw_init, sim_ksw_cubic).
 *
 * Conventions
 *   - lmax = L, nshell = N, n_lm = (L+1)(L+2)/2.
 *   - Coefficient index idx(l, m) = l(l+1)/2 + m, 0 <= m <= l <= L.  Complex
 *     values are interleaved (re, im).  Spherical harmonics are orthonormal
 *     with the Condon-Shortley phase; real fields keep m >= 0 only.  The
 *     imaginary part of every m = 0 input coefficient is ignored (read as 0)
 *     and every m = 0 output has imaginary part 0.
 *   - Noise n: device array [R][N][n_lm] complex; complex128 (double pairs)
 *     for SIM_FP64, complex64 (float pairs) for SIM_FP32.
 *   - Outputs aT, aE (and the optional a_NL parts): device arrays [R][n_lm]
 *     complex128 in every precision.
 *   - Grid: n_ring Gauss-Legendre rings (default ceil((3L+1)/2), the least
 *     that integrates Phi_L^2 Y_lm exactly) and n_phi pixels per ring
 *     (default 3L when 3L = 2^a 3^b 5^c).  With n_phi = 3L only the (L, L) coefficient of the
 *     square aliases; the library removes that term exactly, so results
 *     equal those of an alias-free grid.
 *   - <Phi_L^2>: SIM_MEAN_SAMPLE (default) removes the sky mean of each
 *     shell's map (so Phi_NL,00 = 0); SIM_MEAN_ENSEMBLE removes the
 *     ensemble variance sum_l (2l+1)/(4 pi) sum_j F_l,ij^2.  They differ only
 *     at l = 0.
 *
 * Ownership and threading
 *   - sim_init deep-copies every host array; the caller keeps its arrays.
 *   - Device pointers given to sim_forward / sim_backward belong to the
 *     caller; the library never frees them and keeps no reference after the
 *     call returns.  The context owns its device workspaces.
 *   - Calls are asynchronous on opts.stream (NULL = the default stream)
 *     unless stated otherwise.  A context must not be used from two host
 *     threads or two streams at once.
 *
 * Errors
 *   Every call returns a status code (SIM_OK or a negative SIM_E*); no C++
 *   exception crosses this boundary.  Argument validation (shapes, grid
 *   sizes, finiteness of host inputs, null pointers) happens before any HIP
 *   call.  sim_last_error() gives a message for the last failing call.
 */
#ifndef FNLSIM_H
#define FNLSIM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_ctx sim_ctx;
typedef struct sim_batch sim_batch;

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,  /* bad argument: nothing was launched                */
    SIM_ENOMEM = -2,  /* device or host allocation failed                   */
    SIM_EDEVICE = -3, /* a HIP call failed (message in sim_last_error)      */
    SIM_ESTATE = -4   /* call not valid in the context's current state      */
};

enum { SIM_FP64 = 0, SIM_FP32 = 1, SIM_BF16X3 = 2, SIM_BF16X6 = 3 };
enum { SIM_MEAN_SAMPLE = 0, SIM_MEAN_ENSEMBLE = 1 };

/* Options; zero-initialised fields take the defaults. */
typedef struct {
    int n_ring;     /* Gauss-Legendre rings; 0 -> ceil((3L+1)/2); must be >= that  */
    int n_phi;      /* pixels per ring; 0 -> 3L if that is of the form 2^a 3^b 5^c,
                       else the next such length; must be >= 3L, of that form,
                       and <= 8192                                                 */
    int precision;  /* SIM_FP64 (contractions in FP64), SIM_FP32 (FP32 matrix
                       cores, FP64 Legendre recurrence and radial sums), or the
                       split-BF16 forms of the Legendre transforms: every FP32
                       operand as 2 (SIM_BF16X3: 3 piece products) or 3
                       (SIM_BF16X6: 6 products) BF16 pieces on the BF16 matrix
                       cores with FP32 accumulation; their noise is complex64
                       like SIM_FP32.  The reverse pass, batches and the cubic
                       statistic take SIM_FP64 or SIM_FP32 only                 */
    int mean_mode;  /* SIM_MEAN_SAMPLE or SIM_MEAN_ENSEMBLE                        */
    int max_batch;  /* reserved; 0                                                 */
    void *stream;   /* hipStream_t for every launch; NULL = default stream         */
    int tune;       /* 0: column tile of 16 CF columns with CF in 1..5 chosen to
                       minimise padding, 2 shells per ring-stage block with
                       FP32 data (1 with FP64); 1: time one forward pass (zero
                       noise) for every CF at set-up and keep the fastest, then
                       with FP32 data time 1 shell per ring block against 2
                       and keep the faster (sim_info reports both choices)     */
    int ring_shells; /* 0: as above; 1 or 2: shells per ring-stage block, fixed
                        (FP32 data; SIM_FP64 takes 1 only), not tuned          */
} sim_opts;

/* Read-only facts about a context. */
typedef struct {
    int lmax, nshell, n_ring, n_phi, n_pair, precision, mean_mode;
    long long n_lm;
    long long workspace_bytes;  /* device memory owned by the context          */
    int col_tile;               /* columns per matrix-core tile (16 CF)        */
    int ring_shells;            /* shells per block of the ring FFT stage      */
} sim_info;

/* Create a context for band limit lmax and nshell radial nodes.
 *   r, w     [N]           node radii (Mpc) and quadrature weights w_i
 *   filter   [L+1][N][N]   F_l, row i = output node, column j = input node
 *                          (any real matrix; a Cholesky factor of the
 *                          covariance of Eq. cov_phi in the paper's method)
 *   alpha    [L+1][N]      temperature real-space transfer alpha^T_l(r_i)
 *                          (Eq. rs_tf evaluated at the nodes)
 *   beta     [L+1][N]      E-mode real-space transfer alpha^E_l(r_i)
 *   opts     nullable
 * Host arrays, FP64, row-major.  The radial weights W^X_li = w_i r_i^2 X_l(r_i)
 * are formed in FP64 here.  Returns SIM_EINVAL (no HIP call made) for
 * lmax < 1, nshell < 1, null pointers, non-finite values or a grid that is
 * too small; SIM_ENOMEM / SIM_EDEVICE if device set-up fails (*out is then
 * NULL).  With opts->tune the call builds the context once per column tile,
 * runs it, and keeps the fastest (set-up takes correspondingly longer; the
 * results of every choice agree to rounding). */
int sim_init(sim_ctx **out, int lmax, int nshell,
             const double *r, const double *w, const double *filter,
             const double *alpha, const double *beta, const sim_opts *opts);

/* Forward map generator for R realizations (Sect. 2, steps (i)-(v)).
 *   noise    device [R][N][n_lm] complex (dtype per precision, see above)
 *   fnl      host [R] f_NL per realization
 *   aT, aE   device [R][n_lm] complex128: a_L + f_NL a_NL
 *   aT_nl, aE_nl  nullable device [R][n_lm] complex128: a_NL alone
 * Asynchronous on the context stream.  SIM_EINVAL for R < 1 or a null
 * required pointer. */
int sim_forward(sim_ctx *ctx, const void *noise, int R, const double *fnl,
                void *aT, void *aE, void *aT_nl, void *aE_nl);

/* Counter-based noise (the memory remark of Sect. 3: the white noise of a
 * realization is a function of its seed, so it need not be stored).
 * Value (l, m, j) of realization `seed`: Philox4x32-10 (Salmon et al., SC'11)
 * of counter (idx mod 2^32, idx / 2^32, j, 0x6e6f6973), idx = l(l+1)/2 + m,
 * under key (seed mod 2^32, seed / 2^32) gives x0..x3;
 * u1 = (((x1 2^32 + x0) >> 11) + 1) 2^-53 in (0, 1],
 * u2 = ((x3 2^32 + x2) >> 11) 2^-53 in [0, 1);
 * g0 + i g1 = sqrt(-2 ln u1) e^{2 pi i u2} (Box-Muller, in FP64);
 * n = (g0 + i g1)/sqrt(2) for m > 0 and g0 for m = 0, then rounded to the
 * precision's noise dtype.
 *
 * sim_noise writes that noise for seeds[0..R) into device
 * noise [R][N][n_lm] complex (the layout and dtype sim_forward reads).
 * sim_forward_seeded is sim_forward on that noise, with the noise generated
 * inside the filter (no noise buffer, no noise traffic), which then also
 * forms the linear radial sums: aT_nl, aE_nl equal those of
 * sim_forward(sim_noise(seeds)) bit for bit, aT and aE to FP64 rounding (the
 * linear radial sum adds the same products in another order).
 *   seeds    host [R] 64-bit realization seeds
 *   others   as for sim_forward
 * Asynchronous on the context stream.  SIM_EINVAL for R < 1 or a null
 * required pointer (nothing launched). */
int sim_noise(sim_ctx *ctx, const unsigned long long *seeds, int R, void *noise);
int sim_forward_seeded(sim_ctx *ctx, const unsigned long long *seeds, int R, const double *fnl,
                       void *aT, void *aE, void *aT_nl, void *aE_nl);
/* sim_backward with the noise regenerated from seeds[0..R) (the reverse pass
 * only needs it to recompute Phi_L, which then equals sim_backward's bit for
 * bit).  Arguments and errors as for sim_backward, with seeds (host [R]) in
 * place of the noise; synchronises the stream like sim_backward. */
int sim_backward_seeded(sim_ctx *ctx, const unsigned long long *seeds, int R, const double *fnl,
                        const void *gT, const void *gE, void *grad_n, double *grad_fnl);

/* Greedy design of the radial quadrature (Sect. 3: Eq. mean_err and the
 * linear system for the optimal weights).  For each of P problems (a
 * multipole and a transfer table), the line-of-sight integral is the fine sum
 * I = sum_k a_k Phi(r_k) over ntot shells with Phi ~ N(0, C); a node set S
 * with optimal weights (C_SS w = (C a)_S) leaves the expected quadratic error
 * a^T C a - w^T C_SS w.  Starting from S empty, each step adds the shell that
 * most lowers the sum of those errors over all problems (T and E problems
 * enter with equal weight; scale C and a beforehand to weight them
 * otherwise); ties go to the lowest index.
 *   cov     device [P][ntot][ntot] FP64, symmetric positive definite
 *   a       device [P][ntot] FP64 fine-sum weights (dr_k r_k^2 X(r_k))
 *   n       nodes to choose, 1 <= n <= min(ntot, 1024); 1 <= P <= 65535,
 *           ntot <= 16384
 *   nodes   host [n] out: fine-grid index of the node chosen at each step
 *   err     host [n] out: summed optimal error after each step
 *   w       device [P][n] FP64 out: optimal weights of the n nodes, in the
 *           order of `nodes`
 *   stream  HIP stream (NULL = default)
 * A shell whose variance conditional on a problem's nodes so far is at most
 * 1e-10 of its own variance C_jj is dependent in that problem: it gains
 * nothing there and, if chosen for the other problems, gets weight 0 in it.
 * err[k] is sum_p (a^T C a - |z_p|^2) after step k, with z_p the Cholesky
 * right-hand side of problem p's independent nodes.
 * Synchronous.  SIM_EINVAL for a null pointer or sizes out of range (nothing
 * launched), SIM_ENOMEM if the workspace (8 P n ntot bytes and a little more)
 * cannot be allocated, SIM_EDEVICE if a HIP call fails; the message is in
 * sim_last_error(NULL). */
int sim_quadrature_design(const double *cov, const double *a, int P, int ntot, int n,
                          int *nodes, double *err, double *w, void *stream);

/* sim_quadrature_design with covariances shared between problems: the T and
 * E problems of one multipole see the same C_l (Eq. cov_phi), so a design
 * over l = 0..L and both tables needs L + 1 covariances, not 2 (L + 1).
 *   cov     device [ncov][ntot][ntot] FP64
 *   cidx    host [P]: problem p uses cov[cidx[p]], 0 <= cidx[p] < ncov
 * Everything else, the result and the errors as for sim_quadrature_design
 * (SIM_EINVAL also for a null cidx or an index out of range).  The result
 * equals sim_quadrature_design's on the expanded [P][ntot][ntot] array.
 * The Cholesky factor of the chosen nodes depends on the covariance alone, so
 * it is formed once per distinct covariance used: the workspace is about
 * 8 S n ntot bytes for S distinct indices in cidx, and each step reads S
 * factors instead of P. */
int sim_quadrature_design_shared(const double *cov, int ncov, const int *cidx, const double *a,
                                 int P, int ntot, int n, int *nodes, double *err, double *w,
                                 void *stream);

/* sim_quadrature_design without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same design and kernels, with the
 * workspace in a fixed 64 MiB device array that each GPU holds for the life
 * of the process instead of a per-call allocation.
 *   cov, a, P, ntot, n   as for sim_quadrature_design
 *   nodes    device [n] int out
 *   err      device [n] FP64 out
 *   w        device [P][n] FP64 out
 *   stream   HIP stream (NULL = default)
 * Asynchronous on the stream: no host copy, no synchronisation, no
 * hipMalloc/hipFree and no memset (the kernels clear the state they need).
 * SIM_EINVAL (nothing launched) for a null pointer, sizes out of range, or a
 * design whose workspace (about 8 P ntot (n + 3) bytes; see
 * sim_quadrature_design) exceeds 64 MiB -- for P = 2 problems, 400 fine
 * shells and 70 nodes it is 0.5 MiB.  All calls on one GPU share its
 * workspace: calls that overlap in time on one GPU (two streams or two host
 * threads) race and give wrong results; calls in stream order are safe. */
int sim_quadrature_design_noalloc(const double *cov, const double *a, int P, int ntot, int n,
                                  int *nodes, double *err, double *w, void *stream);

/* Cubic KSW statistic (Sect. 4): for data a^T, a^E and radial nodes r_k,
 *   A(r_k, n) = sum_{i,j in T,E} sum_lm (C^-1)^{ij}_l alpha^i_l(r_k) a^j_lm Y_lm(n),
 *   B(r_k, n) = the same with beta^i_l(r_k),
 *   S_prim   = sum_k w_k r_k^2 int d^2n A(r_k, n) B(r_k, n)^2,
 * the statistic whose normalisation gives the f_NL estimate of
 * Eq. fast_est.  sim_ksw_init creates a context for it (destroy it with
 * sim_destroy; the generator's calls reject it with SIM_ESTATE):
 *   r, w     [Nk]          radial nodes (Mpc) and quadrature weights
 *   alpha    [2][L+1][Nk]  alpha^i_l(r_k), i = T then E
 *   beta     [2][L+1][Nk]  beta^i_l(r_k)
 *   cinv     [L+1][2][2]   (C^-1)^{ij}_l, the inverse T/E spectrum matrix
 *                          (rows of zeros leave a multipole out)
 *   opts     nullable; n_ring, n_phi, precision and stream as for sim_init
 *            (the grid integrates A B^2 exactly; with n_phi = 3L the one
 *            aliased term is removed); mean_mode and tune must be 0
 * Host arrays, FP64.  SIM_EINVAL for bad sizes, null pointers, non-finite
 * values or Nk > 2048.  The two filtered maps of every node run through the same
 * Legendre synthesis as the generator (FP32 matrix cores in SIM_FP32); the
 * sky and radial sums are FP64.
 * sim_ksw_cubic computes S_prim for R realizations:
 *   aT, aE   device [R][n_lm] complex128 data
 *   S        device [R] FP64 out
 * Asynchronous on the context stream. */
int sim_ksw_init(sim_ctx **out, int lmax, int nnode, const double *r, const double *w,
                 const double *alpha, const double *beta, const double *cinv,
                 const sim_opts *opts);
int sim_ksw_cubic(sim_ctx *ctx, const void *aT, const void *aE, int R, double *S);

/* Temperature and Stokes Q, U maps of R realizations (the production maps of
 * Sect. 3, shown in fig. cmb_maps) on the context's Gauss-Legendre grid:
 *   T = sum_lm a^T_lm Y_lm,   Q + i U = -sum_lm a^E_lm 2Y_lm  (no B modes),
 * with the spin-2 harmonics raised from Y_lm by the eth operator (Condon-
 * Shortley phase), every real field summed over m >= 0 with c_0 = 1,
 * c_m = 2 (a^E_l0 and the imaginary part of m = 0 ignored, l < 2 of E
 * ignored).
 *   aT, aE   device [R][n_lm] complex128
 *   maps     device [R][3][n_ring][n_phi] FP64: T, Q, U; rings north to
 *            south (sim_get_grid), phi_j = 2 pi j / n_phi
 * Runs in FP64 in every precision (the contraction has two real columns per
 * map: vector FMAs next to the FP64 recurrence, then FP64 ring FFTs).  The
 * first call allocates the context's spin-2 tables (about 40 (n_lm +
 * 128 (L+1)) bytes) and a 96 npair (L+1)-byte spectrum buffer; asynchronous
 * on the context stream afterwards.  Works on any context (generator or
 * cubic statistic). */
int sim_tqu_maps(sim_ctx *ctx, const void *aT, const void *aE, int R, void *maps);

/* Reverse-mode derivative of sim_forward for a real loss.
 *   gT, gE    device [R][n_lm] complex128 cotangents dLoss/dRe a + i dLoss/dIm a
 *   grad_n    device [R][N][n_lm] complex, dtype of the noise, same convention
 *             (imaginary part of m = 0 entries set to 0)
 *   grad_fnl  host [R]; the call synchronises the stream to fill it
 * Phi_L is recomputed from the noise inside the call (nothing from a previous
 * forward is kept). */
int sim_backward(sim_ctx *ctx, const void *noise, int R, const double *fnl,
                 const void *gT, const void *gE, void *grad_n, double *grad_fnl);

/* Debug stages for kernel-level checks (synchronous).
 *   SIM_STAGE_FILTER   in: noise [N][n_lm]            out: Phi_L [N][n_lm] c128
 *   SIM_STAGE_NONLIN   in: Phi_L [N][n_lm] c128       out: Phi_NL [N][n_lm] c128
 *                      (synthesis, square minus mean, analysis; no radial sum)
 *   SIM_STAGE_MAPS     in: Phi [N][n_lm] c128          out: maps [N][n_ring][n_phi]
 *                      float64, rings north to south, phi_j = 2 pi j / n_phi
 * Device pointers. */
enum { SIM_STAGE_FILTER = 1, SIM_STAGE_NONLIN = 2, SIM_STAGE_MAPS = 3 };
int sim_debug_stage(sim_ctx *ctx, int stage, const void *in, void *out);

/* Stage timers.  While enabled, every forward records HIP events on the
 * context stream around each stage; sim_profile_read synchronises the stream
 * and returns, per stage, the accumulated milliseconds and the number of
 * launches since the last read (then resets them).  Stages, in order:
 *   0 linear radial sum, 1 filter, 2 Legendre synthesis, 3 ring FFT stage,
 *   4 Legendre analysis + radial sum, 5 combine.
 * nstage is the capacity of ms[] and count[] (SIM_NSTAGE is enough). */
enum { SIM_NSTAGE = 6 };
int sim_profile(sim_ctx *ctx, int enable);
int sim_profile_read(sim_ctx *ctx, double *ms, long long *count, int nstage);

/* Fill *info. */
int sim_get_info(const sim_ctx *ctx, sim_info *info);

/* Gauss-Legendre rule the context uses: x (descending) and weights, [n_ring]
 * host arrays. */
int sim_get_grid(const sim_ctx *ctx, double *x, double *w);

/* Uneven batch: several distinct contexts (any lmax, nshell; the same
 * precision, SIM_FP64 or SIM_FP32, and stream) run as one graph per call.
 * The contexts must outlive the batch. */
int sim_batch_create(sim_ctx *const *ctxs, int count, sim_batch **out);

/* One realization per context: noise[i], fnl[i], aT[i], aE[i] as in
 * sim_forward with R = 1.  The batch runs in one of two graph-captured
 * forms: grouped (one launch per stage and kernel class over all contexts,
 * per-call pointers read from a device table) or branches (the contexts
 * dealt by work onto 4 streams forked inside one graph, each running its
 * contexts' passes back to back, so different stages of different contexts
 * overlap; captured again when a pointer or f_NL changes).  The first call
 * runs and times both and keeps the faster (the environment variable
 * FNLSIM_BATCH_FORM=grouped or =branches, read by sim_batch_create, fixes the
 * form instead); the results of the two are identical.  Asynchronous on the
 * contexts' stream. */
int sim_batch_forward(sim_batch *b, const void *const *noise, const double *fnl,
                      void *const *aT, void *const *aE);

/* The form the batch chose (0 grouped, 1 branches, -1 before the first
 * sim_batch_forward) and the first call's time of each form in ms
 * (ms_grouped, ms_branches nullable). */
int sim_batch_get_mode(const sim_batch *b, int *mode, double *ms_grouped, double *ms_branches);

int sim_batch_destroy(sim_batch *b);

/* Release a context and its device memory.  NULL is accepted. */
int sim_destroy(sim_ctx *ctx);

/* Message for the last failing call on ctx (or of the last failing sim_init
 * when ctx is NULL).  Never NULL. */
const char *sim_last_error(const sim_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif

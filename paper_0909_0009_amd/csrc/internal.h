// internal.h -- shapes, device buffers and kernel launchers shared by the
// host side of the C ABI (fnlsim.cpp) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fnl {

constexpr int kMaxPhi = 8192;   // longest ring the in-LDS FFT handles
constexpr int kMaxPasses = 16;
constexpr int kSeedStride = 32; // l spacing of stored recurrence seeds
constexpr double kLambdaTiny = 1e-30;  // |lambda| below this is treated as 0 (polar skip)
// Polar skip of the Legendre contractions with FP32 data: the terms left out
// before the first |lambda_lm(x_p)| above this are below FP32 rounding by
// more than four orders of magnitude (unit roundoff 6e-8).  The FP64 path
// and the spin-2 maps (whose functions near the pole exceed lambda_lm by
// up to l^2 / sin^2 theta) keep kLambdaTiny.
constexpr double kLambdaTinyF32 = 1e-12;
constexpr int kCminW = 9;  // polar-start entries per analysis chunk: the chunk, its 8 K-steps
constexpr int kCoefPad = 128;      // zero rows after each m's coefficient block (>= analysis rows per block)
constexpr int kPhiPad = 32;        // zero rows after the last m block of the Phi matrices (synthesis prefetch)
// Work of one Legendre wave: ring pairs per synthesis wave and l rows per
// analysis wave (FP32 / FP64; register budget of the accumulators).
constexpr int kSynthPairsF32 = 64, kSynthPairsF64 = 32;
constexpr int kAnalRowsF32 = 64, kAnalRowsF64 = 64;

// Everything a kernel needs to know about the problem's shape.
struct Shape {
    int L;        // lmax
    int N;        // shells
    int C;        // real columns = 2N (shell, re/im)
    int CF;       // 16-column MFMA fragments per column tile
    int CT;       // column tile = 16 CF
    int Cpad;     // columns rounded up to whole tiles
    int nct;      // column tiles
    int nring;    // Gauss-Legendre rings
    int npair;    // north/south ring pairs (the equator counts as one)
    int equator;  // 1 if nring is odd (pair npair-1 is the equator)
    int nphi;     // pixels per ring
    int alias;    // 1 if nphi == 3L: remove the folded (L, L) term
    int npass;    // FFT passes
    int radix[kMaxPasses];
    long long nlm;
    int mean_mode;
    int fp32;     // 0: FP64 path, 1: FP32 data (FP32 or split-BF16 matrix cores)
    int npiece;   // 0: FP32/FP64 matrix cores; 2 or 3: BF16 pieces per operand (X3, X6)
    int lower;    // 1 if every F_l is lower triangular (contractions stop at the diagonal)
    int rs;       // shells per forward ring block: 1 or 2 (FP32 data), 1 (FP64)
};

// Elements of one ring buffer in LDS: n values at j + j/32, plus one slot.
__host__ __device__ constexpr int ring_pad(int n) { return n + (n >> 5) + 1; }
constexpr size_t kMaxLds = 163840;  // LDS bytes a workgroup may allocate
// Default shells per forward ring block (256 threads each) in FP32 / FP64.
constexpr int kRingShellsF32 = 2;
constexpr int kRingShellsF64 = 1;
inline int ring_shells(int fp32) { return fp32 ? kRingShellsF32 : kRingShellsF64; }
// Ring lengths the FFT has a compile-time plan for (all other 5-smooth
// lengths take the run-time plan), and the register bucket of a length.
__host__ __device__ constexpr bool fft_has_plan(int n)
{
    return n == 768 || n == 1024 || n == 1536 || n == 3072 || n == 6144;
}
__host__ __device__ constexpr int ring_bucket(int n)
{
    return n <= 1024 ? 1024 : n <= 2048 ? 2048 : n <= 4096 ? 4096 : 8192;
}

// Row of coefficient (l, m) in the m-major layouts: rows of one m are
// contiguous, m ascending.
__host__ __device__ inline long long mrow(int L, int m, int l) {
    return (long long)m * (L + 1) - (long long)m * (m - 1) / 2 + (l - m);
}
// First row of m's block in the padded coefficient table: rows l = m..L,
// then kCoefPad zero rows.
__host__ __device__ inline long long crow(int L, int m) {
    return mrow(L, m, m) + (long long)m * kCoefPad;
}
__host__ __device__ inline long long lm_index(int l, int m) {
    return (long long)l * (l + 1) / 2 + m;
}

// Device buffers owned by a context.  Element type of phi/G/F/FT/tw is
// double for the FP64 path and float for the FP32 path (void* here).
struct Bufs {
    void *FT;          // [L+1][Kpad][Mpad] filter, transposed and zero padded (reverse pass)
    void *FQ;          // [L+1][nchq][Mpad][4][8] forward filter: FQ(l, c, i, k, s) =
                       // F_l[i][32 c + 4 s + k], zero padded (one lane's 8 K-steps of
                       // a 32-column chunk are contiguous)
    double *V;         // [2][L+1][N] V^X_l = W^X_l F_l (linear radial sum)
    double *W;         // [2][L+1][Cpad/2] W^X_ls, zero for padded shells
    double *x;         // [npair] cos theta of the north ring of each pair
    double *wq;        // [npair] omega_p * 2 pi / nphi
    double *lmm;       // [L+1][npair] lambda_mm(x_p)
    double2 *coef;     // [nlm + (L+1) kCoefPad] (A, B): lambda_l = A x lambda_{l-1} - B lambda_{l-2},
                       // m-major blocks (crow) each followed by kCoefPad zero rows
    double2 *seed;     // [nseedrow][npair] recurrence state (lambda_{l0-1}, lambda_{l0-2})
                       // entering l0 = m + 32u ((0, lambda_mm) for u = 0)
    int *seedoff;      // [L+2] first seed row of each m
    int *lstart;       // [L+1][npair] first l with |lambda_lm(x_p)| > 1e-30 (L+1 if none)
    int *lstart_mat;   // the same for the matrix-core contractions: threshold
                       // kLambdaTinyF32 with FP32 data, else lstart itself
    int *cmin;         // [L+1][ceil(npair/32)][kCminW]: min of lstart_mat over each 32-pair
                       // chunk, then over each of its eight 4-pair K-steps
    int2 *k1tiles;     // [nk1] (l, column tile) of each filter workgroup
    int4 *k2tiles;     // [nk2] synthesis blocks (m, pair tile, column tile, 0)
    int4 *k4tiles;     // [nk4] analysis blocks (m, l tile, column tile, 0)
                       // Both tables are in XCD order: block b runs entry b of the
                       // table and is dispatched to XCD b % 8; m < 0 marks an idle block.
    void *tw;          // [nphi] e^{-2 pi i q / nphi}
    double *mu;        // [Cpad/2] sqrt(4 pi) * ensemble <Phi_L^2>(r_s)
    void *phi;         // [nlm rows][Cpad] Phi_L (m-major)
    void *phib;        // split BF16 paths: [nseedrow + 2][Cpad][2][npiece][16] BF16 pieces of
                       // Phi_L per 32-l block of each m (two zero blocks at the end)
    void *G;           // [npair][L+1][Cpad][2] synthesis output, (E, O) interleaved
    void *F;           // [L+1][npair][Cpad][2] weighted ring spectra, (E, O) interleaved
    double2 *part;     // [nct][2][nlm] per-column-tile radial sums of Phi_NL
    double2 *aL;       // [2][nlm] linear radial sums
    void *scratch;     // debug / backward staging, [nlm rows][Cpad] elements
    void *G2;          // reverse pass: synthesis of the transposed radial sum (lazy)
    double *fpart;     // reverse pass: [npair * N] per-block dLoss/df_NL shares (lazy)
    double *fbar;      // reverse pass: [fbar_cap] dLoss/df_NL per realization (lazy)
    // cubic statistic (a context whose N "shells" are the filtered maps A, B
    // of N/2 radial nodes: shell 2k is A(r_k), shell 2k+1 is B(r_k))
    double *kswP;      // [L+1][N/2][map A/B][data T/E] filter coefficients
    double *kswW;      // [N/2] w_k r_k^2
    double *kswpart;   // [npair][N/2] sky integral of A B^2 per ring pair and node
    // T, Q, U maps (lazy, first sim_tqu_maps call)
    double *tqutab;    // [nlm + (L+1) kCoefPad][5] spin-2 coefficients, crow layout
    double2 *tqutw;    // [nphi] e^{-2 pi i q / nphi} in FP64
    double *tquG;      // [npair][3][L+1][4] ring spectra (E re, O re, E im, O im)
    int fbar_cap;
    int Kpad, Mpad, nchq;
    int nk1, nk2, nk4;
    long long nseedrow;
};

// One context inside a grouped (batch) launch: its shape and buffers plus the
// per-call pointers of the current forward pass.
struct GroupItem {
    Shape sh;
    Bufs b;
    const void *noise;
    double fnl;
    double2 *aT, *aE;
};

// Stage ids of the grouped forward launches.
enum { GS_RADIAL_LIN = 0, GS_FILTER, GS_SYNTH, GS_RING, GS_ANAL, GS_COMBINE, GS_COUNT };

// Blocks of context `sh`/`b` in a stage (before rounding up to a multiple of 8).
long long group_blocks(int stage, const Shape &sh, const Bufs &b);

// One grouped launch: contexts ord[0..n) of `items` (device), block offsets
// off[0..n] (device, multiples of 8), nblocks = off[n]; CF selects the
// column-tile instantiation (synth/anal), lds the dynamic LDS (ring).
hipError_t launch_group(int stage, int fp32, int CF, const GroupItem *items, const int *ord,
                        const int *off, int n, int nblocks, size_t lds, hipStream_t s);
// Raise the dynamic-LDS limit of the grouped ring kernel (call before capture).
hipError_t prepare_group_ring(int fp32, int nphi, int planned);

// ----- launchers (kernels.hip); all asynchronous on `s`.
hipError_t launch_seed_init(const Shape &sh, const Bufs &b, hipStream_t s);  // seeds, lstart, cmin
hipError_t launch_radial_lin(const Shape &sh, const Bufs &b, const void *noise, hipStream_t s);
// true where the stored-noise filter also forms the linear radial sums
// (FP32 data), so no launch_radial_lin is needed
bool filter_forms_radial(const Shape &sh);
// noise == nullptr: the noise of realization `seed` is generated in the
// kernel (counter-based, as launch_noise writes it) instead of read, and the
// filter also writes the linear radial sums into b.aL (launch_radial_lin's
// work).
hipError_t launch_filter(const Shape &sh, const Bufs &b, const void *noise, void *phi_out,
                         hipStream_t s, unsigned long long seed = 0);
// noise of realization `seed`, [N][nlm] complex in the path's precision
hipError_t launch_noise(const Shape &sh, unsigned long long seed, void *out, hipStream_t s);
hipError_t launch_synth(const Shape &sh, const Bufs &b, const void *phi_in, void *G_out,
                        hipStream_t s);
// split-BF16 forms of the Legendre kernels (bf16.hip; the generic launchers
// dispatch to them when sh.npiece != 0)
hipError_t launch_synth_bf(const Shape &sh, const Bufs &b, const void *phi_in, void *G_out,
                           hipStream_t s);
hipError_t launch_anal_bf(const Shape &sh, const Bufs &b, const void *F_in, void *out_phi, int mode,
                          hipStream_t s);
// mode 0: square minus mean and forward transform into F; 1: write maps.
hipError_t launch_ring(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                       double *maps, int mode, hipStream_t s);
// mode 0: radial partial sums into b.part; 1: per-shell Phi_NL into out_phi.
// mode 2: per-shell output plus sum_X W^X abar^X (reverse pass), into out_phi.
hipError_t launch_anal(const Shape &sh, const Bufs &b, const void *F_in, void *out_phi, int mode,
                       hipStream_t s, const double2 *gT = nullptr, const double2 *gE = nullptr);
hipError_t launch_combine(const Shape &sh, const Bufs &b, double fnl, double2 *aT, double2 *aE,
                          double2 *aTn, double2 *aEn, hipStream_t s);
// reverse pass
hipError_t launch_radial_adj(const Shape &sh, const Bufs &b, const double2 *gT, const double2 *gE,
                             void *out, hipStream_t s);
hipError_t launch_ring_adj(const Shape &sh, const Bufs &b, const void *G, const void *G2, void *F,
                           double *fpart, double fnl, hipStream_t s);
hipError_t launch_filter_t(const Shape &sh, const Bufs &b, const void *phibar, void *gout,
                           hipStream_t s);
hipError_t launch_fbar(const Shape &sh, const Bufs &b, const double *fpart, const double2 *gT,
                       const double2 *gE, double *out, hipStream_t s);
hipError_t launch_phi_to_api(const Shape &sh, const void *phi, double2 *api, hipStream_t s);
// cubic statistic: filtered-map coefficients from the data, the ring stage
// (A B^2 summed over each ring pair), and the weighted radial sum into *S
hipError_t launch_ksw_filter(const Shape &sh, const Bufs &b, const double2 *aT, const double2 *aE,
                             hipStream_t s);
hipError_t launch_ksw_ring(const Shape &sh, const Bufs &b, hipStream_t s);
hipError_t launch_ksw_sum(const Shape &sh, const Bufs &b, double *S, hipStream_t s);
// T, Q, U maps [3][nring][nphi] (FP64) of one realization's a^T, a^E
hipError_t launch_tqu(const Shape &sh, const Bufs &b, const double2 *aT, const double2 *aE,
                      double *maps, hipStream_t s);
hipError_t launch_api_to_phi(const Shape &sh, const double2 *api, void *phi, hipStream_t s);

}  // namespace fnl

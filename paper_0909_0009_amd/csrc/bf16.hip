// bf16.hip -- the Legendre synthesis and analysis on the BF16 matrix cores
// with split operands (precisions SIM_BF16X3 and SIM_BF16X6).
//
// Each FP32 operand v is split into NP BF16 pieces, v ~ v_0 + v_1 (+ v_2),
// v_0 = bf16(v), v_1 = bf16(v - v_0), v_2 = bf16(v - v_0 - v_1) (round to
// nearest even), and a product a b is formed from the piece products whose
// order i + j is below NP: a_0 b_0 + a_0 b_1 + a_1 b_0 (three products, NP = 2)
// or those plus a_0 b_2 + a_1 b_1 + a_2 b_0 (six, NP = 3), accumulated in FP32
// by v_mfma_f32_16x16x32_bf16.  Two pieces keep 16 significant bits, so the
// neglected terms are ~2^-17 of the product; three keep 24 bits, FP32's.
// The Legendre recurrence stays in FP64 as in the FP32 path; only the
// matrix-core operands change.
//
//   k_split_phi   Phi (FP32, m-major rows) -> BF16 pieces laid out so that one
//                 lane's 8 K values of the synthesis B operand are 16 bytes
//   k_synth_bf    synthesis: K-steps of 64 l (32 of each parity), lambda split
//                 and transposed through LDS, B pieces from k_split_phi
//   k_anal_bf     analysis: K-steps of 32 ring pairs, lambda split through
//                 LDS, the ring spectra F (FP32) split as they are loaded;
//                 the FP32 path's epilogue (radial sums or per-shell output)
#include "device_common.h"

namespace fnl {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {

// MFMA 16x16x32 BF16: lane l holds A[l % 16][k] and B[k][l % 16] for the 8
// K slots (l / 16, 0..7) (the same slot order in both operands); output
// element r is D[4 (l / 16) + r][l % 16], as for the FP32 16x16x4 tile.
__device__ __forceinline__ v4f mfma_bf(const bf8 &a, const bf8 &b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// piece products (i, j) with i + j < NP, in the order they are accumulated
template <int NP> __device__ constexpr int nprod() { return NP == 2 ? 3 : 6; }
template <int NP> __device__ constexpr int prod_a(int k) { return NP == 2 ? (k == 2 ? 1 : 0) : (k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 1 : k == 3 ? 0 : k == 4 ? 1 : 2); }
template <int NP> __device__ constexpr int prod_b(int k) { return NP == 2 ? (k == 1 ? 1 : 0) : (k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 0 : k == 3 ? 2 : k == 4 ? 1 : 0); }

template <int NP> __device__ __forceinline__ void split(float v, __bf16 (&out)[NP])
{
    float r = v;
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const __bf16 h = (__bf16)r;
        out[p] = h;
        r -= (float)h;
    }
}

// ----------------------------------------------------------------- split Phi

// Block (64 columns, 32-l block blk of some m); thread = column.  Block blk
// of m is seedoff[m] + b and holds l = m + 32 b + t, t < 32 (zeros past L);
// out[blk][col][par][piece][16] holds the pieces of Phi(l = m + 32 b + 2 u + par).
template <int NP>
__global__ __launch_bounds__(64) void k_split_phi(Shape sh, const int *__restrict__ seedoff,
                                                  const float *__restrict__ phi,
                                                  __bf16 *__restrict__ out)
{
    const int blk = blockIdx.y;
    const int col = blockIdx.x * 64 + threadIdx.x;
    if (col >= sh.Cpad) return;
    // m with seedoff[m] <= blk < seedoff[m + 1]
    int lo = 0, hi = sh.L + 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seedoff[mid] <= blk)
            lo = mid;
        else
            hi = mid;
    }
    const int m = lo, b = blk - seedoff[m];
    const long long row0 = mrow(sh.L, m, m) + 32 * b;
    __bf16 pc[2][NP][16];
#pragma unroll
    for (int t = 0; t < 32; t++) {
        const int l = m + 32 * b + t;
        const float v = l <= sh.L ? phi[(row0 + t) * sh.Cpad + col] : 0.0f;
        __bf16 s[NP];
        split<NP>(v, s);
#pragma unroll
        for (int p = 0; p < NP; p++) pc[t & 1][p][t >> 1] = s[p];
    }
    bf8 *dst = reinterpret_cast<bf8 *>(out + ((long long)blk * sh.Cpad + col) * (2 * NP * 16));
#pragma unroll
    for (int par = 0; par < 2; par++)
#pragma unroll
        for (int p = 0; p < NP; p++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                bf8 v;
#pragma unroll
                for (int j = 0; j < 8; j++) v[j] = pc[par][p][8 * h + j];
                dst[(par * NP + p) * 2 + h] = v;
            }
}

// ---------------------------------------------------------------- synthesis

constexpr int kSynthLd = 40;  // LDS row of 32 BF16 K values (+8: shifts rows across banks)

template <int CF, int NP> constexpr int synth_bf_waves() { return 8 * NP * CF + 32 * CF + 64 <= 256 ? 2 : 1; }

// Block = (m, 64 ring pairs, column tile of 16 CF columns), one wave, the same
// block table as the FP32 synthesis.  K-step s covers l = l0 .. l0 + 63,
// l0 = lbeg + 64 s (lbeg = the first stored recurrence state at or below
// the polar start); K slot kk of parity par is l = l0 + 2 kk + par, i.e.
// 32-l blocks b and b + 1 of m.  Lane q runs the FP64 recurrence of pair
// p0 + q over the step's 64 l, splits each value and writes the pieces to
// LDS as lam[piece][par][pair][kk]; the wave reads them back as A operands
// (8 consecutive kk of one pair: one 16-byte read).
template <int CF, int NP>
__global__ __launch_bounds__(64, (synth_bf_waves<CF, NP>())) void k_synth_bf(
    Shape sh, const int4 *__restrict__ tiles, const double *__restrict__ x,
    const double2 *__restrict__ seed, const int *__restrict__ seedoff,
    const int *__restrict__ lstart, const double2 *__restrict__ coef,
    const __bf16 *__restrict__ phib, float *__restrict__ G)
{
    constexpr int NF = 4;  // 64 pairs
    __shared__ __bf16 lam[NP][2][64][kSynthLd];
    const int L = sh.L, npair = sh.npair, Cpad = sh.Cpad;
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;  // idle slot of the XCD layout
    const int m = __builtin_amdgcn_readfirstlane(tl.x);
    const int pt = __builtin_amdgcn_readfirstlane(tl.y);
    const int ct = __builtin_amdgcn_readfirstlane(tl.z);
    const auto cm_row = coef + crow(L, m);
    const int lane = threadIdx.x, i16 = lane & 15, k4 = lane >> 4;
    const int p0 = pt * 64, p = p0 + lane;
    const bool pv = p < npair;
    const double xp = pv ? x[p] : 0.0;
    int ls = pv ? lstart[(long long)m * npair + p] : L + 1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) ls = min(ls, __shfl_xor(ls, o));
    ls = __builtin_amdgcn_readfirstlane(ls);
    v4f acc[NF][2][CF];
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int c = 0; c < CF; c++) acc[f][a][c] = v4f{};
    const int colb = ct * sh.CT + i16;
    if (ls <= L) {
        const int u0 = (ls - m) / kSeedStride;
        double l1 = 0.0, l2 = 0.0;
        if (pv) {
            const double2 st = seed[((long long)seedoff[m] + u0) * npair + p];
            l1 = st.x;
            l2 = st.y;
        }
        const int lbeg = m + u0 * kSeedStride;
        const int nks = (L - lbeg) / 64 + 1;
        for (int s = 0; s < nks; s++) {
            const int l0 = lbeg + 64 * s;
            // B pieces of this step (blocks u0 + 2 s and u0 + 2 s + 1 of m; the
            // second may belong to the next m or the zero blocks at the end,
            // and then meets lambda = 0)
            const long long blk = (long long)seedoff[m] + u0 + 2 * s + (k4 >> 1);
            bf8 bv[CF][2][NP];
#pragma unroll
            for (int cf = 0; cf < CF; cf++) {
                const bf8 *src = reinterpret_cast<const bf8 *>(
                    phib + (blk * Cpad + colb + 16 * cf) * (2 * NP * 16) + 8 * (k4 & 1));
#pragma unroll
                for (int par = 0; par < 2; par++)
#pragma unroll
                    for (int pc = 0; pc < NP; pc++) bv[cf][par][pc] = src[(par * NP + pc) * 2];
            }
            // recurrence over the step's 64 l; rows past L meet the zero
            // padding of m's coefficient block, so lambda = 0 there exactly
            __syncthreads();  // the previous step's LDS reads are done
#pragma unroll 1
            for (int g = 0; g < 4; g++) {
                bf8 st[2][NP];
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    const int q = 16 * g + j;  // l = l0 + q: parity q & 1, slot kk = q >> 1
                    const double2 ab = cm_row[l0 + q - m];
                    const double nv = ab.x * xp * l1 - ab.y * l2;
                    l2 = l1;
                    l1 = nv;
                    __bf16 pcs[NP];
                    split<NP>((float)nv, pcs);
#pragma unroll
                    for (int pc = 0; pc < NP; pc++) st[j & 1][pc][j >> 1] = pcs[pc];
                }
#pragma unroll
                for (int par = 0; par < 2; par++)
#pragma unroll
                    for (int pc = 0; pc < NP; pc++)
                        *reinterpret_cast<bf8 *>(&lam[pc][par][lane][8 * g]) = st[par][pc];
            }
            __syncthreads();
#pragma unroll
            for (int f = 0; f < NF; f++)
#pragma unroll
                for (int par = 0; par < 2; par++) {
                    bf8 a[NP];
#pragma unroll
                    for (int pc = 0; pc < NP; pc++)
                        a[pc] = *reinterpret_cast<const bf8 *>(&lam[pc][par][16 * f + i16][8 * k4]);
#pragma unroll
                    for (int cf = 0; cf < CF; cf++)
#pragma unroll
                        for (int k = 0; k < nprod<NP>(); k++)
                            acc[f][par][cf] = mfma_bf(a[prod_a<NP>(k)], bv[cf][par][prod_b<NP>(k)],
                                                      acc[f][par][cf]);
                }
        }
    }
    // G[pair][m][column] holds (E, O) interleaved
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int cf = 0; cf < CF; cf++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int pair = p0 + 16 * f + 4 * k4 + r;
                if (pair < npair) {
                    float2 v;
                    v.x = acc[f][0][cf][r];
                    v.y = acc[f][1][cf][r];
                    *reinterpret_cast<float2 *>(
                        G + ((((long long)pair * (L + 1) + m) * Cpad) + colb + 16 * cf) * 2) = v;
                }
            }
}

// ----------------------------------------------------------------- analysis

constexpr int kAnalLd = 40;  // LDS row of 32 BF16 pair values (+8)

template <int CF, int NP> constexpr int anal_bf_waves() { return 8 * NP * CF + 16 * CF + 96 <= 256 ? 2 : 1; }

// Block = (m, 64 l rows from l0w = m + 64 t, column tile), one wave, the
// same block table as the FP32 analysis.  For each chunk of 32 ring pairs
// (one K-step): lane (half h, pair q) runs the FP64 recurrence over rows
// [32 h, 32 h + 32) of pair q, splits each value and stores it as
// lam[piece][row][q]; the wave reads A as 8 consecutive pairs of one row.
// The B operand, F_{E/O}[pair][column], is loaded as the (E, O) pairs of 8
// consecutive ring pairs per lane and split in registers.  Chunks and
// fragments below the polar start are skipped as in the FP32 kernel.
template <int CF, int NP, int MODE>
__global__ __launch_bounds__(64, (anal_bf_waves<CF, NP>())) void k_anal_bf(
    Shape sh, const int4 *__restrict__ tiles, const double *__restrict__ x,
    const double2 *__restrict__ coef, const double2 *__restrict__ seed,
    const int *__restrict__ seedoff, const int *__restrict__ cmin, const double *__restrict__ W,
    const double *__restrict__ mu, const float *__restrict__ F, double2 *__restrict__ part,
    float *__restrict__ outphi)
{
    constexpr int RW = 64, NF = 2, PC = 32;
    __shared__ __bf16 lam[NP][RW][kAnalLd];
    __shared__ double2 cab[RW];
    const int L = sh.L, npair = sh.npair, Cpad = sh.Cpad;
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;  // idle slot of the XCD layout
    const int m = __builtin_amdgcn_readfirstlane(tl.x);
    const int lt = __builtin_amdgcn_readfirstlane(tl.y);
    const int ct = __builtin_amdgcn_readfirstlane(tl.z);
    const auto cm_row = coef + crow(L, m);
    const int lane = threadIdx.x, i16 = lane & 15, k4 = lane >> 4;
    const int half = lane >> 5, pl = lane & 31;
    const int l0w = m + lt * RW;
    const int lh = l0w + half * (RW / 2);
    const bool hact = lh <= L;
    const long long srow = (long long)seedoff[m] + (hact ? (lh - m) / kSeedStride : 0);
    for (int r = lane; r < RW; r += 64) cab[r] = cm_row[(l0w - m) + r];
    __syncthreads();
    v4f acc[NF][2][CF];
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int c = 0; c < CF; c++) acc[f][a][c] = v4f{};
    const int colb = ct * sh.CT + i16;
    const int nchunk = (npair + PC - 1) / PC;
    const int lend = l0w + RW - 1;
    const int fend = min(NF, (L - l0w) / 32 + 1);
    for (int pc = nchunk - 1; pc >= 0; pc--) {  // equator first, as in k_anal
        const int cm = cmin[((long long)m * nchunk + pc) * kCminW];
        if (cm > lend) continue;  // wave-uniform
        const int f0 = cm <= l0w + 31 ? 0 : (cm - l0w - 31 + 31) / 32;
        // B: (E, O) of ring pairs pc*32 + 8 k4 + j, j < 8, per column fragment;
        // pairs past the last one read the next m (or the zero pairs after the
        // last m) and meet lambda = 0
        const float *fb = F + (((long long)m * npair + pc * PC + 8 * k4) * Cpad + colb) * 2;
        bf8 bE[CF][NP], bO[CF][NP];
#pragma unroll
        for (int cf = 0; cf < CF; cf++) {
            __bf16 e[NP][8], o[NP][8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const float2 v = *reinterpret_cast<const float2 *>(fb + ((long long)j * Cpad + 16 * cf) * 2);
                __bf16 se[NP], so[NP];
                split<NP>(v.x, se);
                split<NP>(v.y, so);
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    e[q][j] = se[q];
                    o[q][j] = so[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NP; q++)
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    bE[cf][q][j] = e[q][j];
                    bO[cf][q][j] = o[q][j];
                }
        }
        {
            const int pp = pc * PC + pl;
            const bool pv = hact && pp < npair;
            double a1 = 0.0, a0 = 0.0, xq = 0.0;
            if (pv) {
                const double2 sd = seed[srow * npair + pp];
                a1 = sd.x;
                a0 = sd.y;
                xq = x[pp];
            }
#pragma unroll 4
            for (int q = 0; q < RW / 2; q++) {
                const double2 ab = cab[half * (RW / 2) + q];
                const double v = ab.x * xq * a1 - ab.y * a0;
                __bf16 pcs[NP];
                split<NP>((float)v, pcs);
#pragma unroll
                for (int c = 0; c < NP; c++) lam[c][half * (RW / 2) + q][pl] = pcs[c];
                a0 = a1;
                a1 = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; f++) {
            if (f >= f0 && f < fend) {
#pragma unroll
                for (int par = 0; par < 2; par++) {
                    bf8 a[NP];
#pragma unroll
                    for (int c = 0; c < NP; c++)
                        a[c] = *reinterpret_cast<const bf8 *>(&lam[c][2 * (16 * f + i16) + par][8 * k4]);
#pragma unroll
                    for (int cf = 0; cf < CF; cf++)
#pragma unroll
                        for (int k = 0; k < nprod<NP>(); k++)
                            acc[f][par][cf] = mfma_bf(a[prod_a<NP>(k)],
                                                      par ? bO[cf][prod_b<NP>(k)] : bE[cf][prod_b<NP>(k)],
                                                      acc[f][par][cf]);
                }
            }
        }
        __syncthreads();
    }
    anal_epilogue<float, CF, MODE, NF>(sh, acc, m, l0w, ct, colb, k4, i16, W, mu, part, outphi,
                                       nullptr, nullptr);
}

template <int CF, int NP>
void synth_bf_t(const Shape &sh, const Bufs &b, void *G, hipStream_t s)
{
    hipLaunchKernelGGL((k_synth_bf<CF, NP>), dim3((unsigned)b.nk2), dim3(64), 0, s, sh, b.k2tiles, b.x,
                       b.seed, b.seedoff, b.lstart_mat, b.coef, (const __bf16 *)b.phib, (float *)G);
}

template <int NP>
void synth_bf_cf(const Shape &sh, const Bufs &b, void *G, hipStream_t s)
{
    switch (sh.CF) {
    case 1: synth_bf_t<1, NP>(sh, b, G, s); break;
    case 2: synth_bf_t<2, NP>(sh, b, G, s); break;
    case 3: synth_bf_t<3, NP>(sh, b, G, s); break;
    case 4: synth_bf_t<4, NP>(sh, b, G, s); break;
    default: synth_bf_t<5, NP>(sh, b, G, s); break;
    }
}

template <int CF, int NP>
void anal_bf_t(const Shape &sh, const Bufs &b, const void *F, void *out, int mode, hipStream_t s)
{
    if (mode == 0)
        hipLaunchKernelGGL((k_anal_bf<CF, NP, 0>), dim3((unsigned)b.nk4), dim3(64), 0, s, sh, b.k4tiles,
                           b.x, b.coef, b.seed, b.seedoff, b.cmin, b.W, b.mu, (const float *)F, b.part,
                           (float *)out);
    else
        hipLaunchKernelGGL((k_anal_bf<CF, NP, 1>), dim3((unsigned)b.nk4), dim3(64), 0, s, sh, b.k4tiles,
                           b.x, b.coef, b.seed, b.seedoff, b.cmin, b.W, b.mu, (const float *)F, b.part,
                           (float *)out);
}

template <int NP>
void anal_bf_cf(const Shape &sh, const Bufs &b, const void *F, void *out, int mode, hipStream_t s)
{
    switch (sh.CF) {
    case 1: anal_bf_t<1, NP>(sh, b, F, out, mode, s); break;
    case 2: anal_bf_t<2, NP>(sh, b, F, out, mode, s); break;
    case 3: anal_bf_t<3, NP>(sh, b, F, out, mode, s); break;
    case 4: anal_bf_t<4, NP>(sh, b, F, out, mode, s); break;
    default: anal_bf_t<5, NP>(sh, b, F, out, mode, s); break;
    }
}

}  // namespace

hipError_t launch_synth_bf(const Shape &sh, const Bufs &b, const void *phi_in, void *G_out,
                           hipStream_t s)
{
    dim3 grid((unsigned)((sh.Cpad + 63) / 64), (unsigned)b.nseedrow);
    if (sh.npiece == 2) {
        hipLaunchKernelGGL(k_split_phi<2>, grid, dim3(64), 0, s, sh, b.seedoff, (const float *)phi_in,
                           (__bf16 *)b.phib);
        synth_bf_cf<2>(sh, b, G_out, s);
    } else {
        hipLaunchKernelGGL(k_split_phi<3>, grid, dim3(64), 0, s, sh, b.seedoff, (const float *)phi_in,
                           (__bf16 *)b.phib);
        synth_bf_cf<3>(sh, b, G_out, s);
    }
    return hipGetLastError();
}

hipError_t launch_anal_bf(const Shape &sh, const Bufs &b, const void *F_in, void *out_phi, int mode,
                          hipStream_t s)
{
    if (sh.npiece == 2)
        anal_bf_cf<2>(sh, b, F_in, out_phi, mode, s);
    else
        anal_bf_cf<3>(sh, b, F_in, out_phi, mode, s);
    return hipGetLastError();
}

}  // namespace fnl

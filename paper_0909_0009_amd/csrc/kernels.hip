// kernels.hip -- gfx950 kernels of the local-f_NL map generator.
//
// Stages (Elsner & Wandelt, Sect. 2, recipe steps (i)-(v)):
//   k_filter      (i)   Phi_L,lm(r_i) = sum_j F_l,ij n_lm(r_j): one GEMM per l on
//                       the matrix cores, written in the m-major layout
//   k_radial_lin  (v)   linear radial sum a^X_L = sum_j V^X_lj n_lm(r_j), FP64
//   k_synth       (ii)  Legendre synthesis E/O_m[p, c] = sum_{l-m even/odd}
//                       lambda_lm(x_p) Phi_lm(c): FP64 three-term recurrence on
//                       the vector ALU feeding 16x16x4 MFMA tiles
//   k_ring        (ii)-(iv) per ring pair and shell: inverse ring FFT, square,
//                       forward ring FFT, alias fix, north/south fold
//   k_anal        (iv)+(v) Legendre analysis sum_p omega lambda F_{E/O}[p, c] on
//                       MFMA with the recurrence transposed through LDS, and the
//                       radial sum with W^X_ls in the epilogue
//   k_combine     a = a_L + f_NL a_NL with a compensated sum over column tiles
#include <type_traits>

#include "device_common.h"

namespace fnl {

// ----------------------------------------------------- counter-based noise

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC'11): each round
// multiplies words 0 and 2 by fixed odd constants, swaps the halves of the
// 64-bit products into the other two words and mixes in the round key; the key
// advances by two Weyl increments between rounds.  Stateless: the output is a
// function of (counter, key) only.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, unsigned k0, unsigned k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        // one 32x32 -> 64-bit multiply per product (v_mad_u64_u32)
        const unsigned long long p0 = (unsigned long long)c.x * 0xD2511F53u;
        const unsigned long long p1 = (unsigned long long)c.z * 0xCD9E8D57u;
        c = make_uint4((unsigned)(p1 >> 32) ^ c.y ^ k0, (unsigned)p1,
                       (unsigned)(p0 >> 32) ^ c.w ^ k1, (unsigned)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Noise value n_lm(r_j) of one realization seed (index idx = l(l+1)/2 + m):
// Philox of counter (idx, j, tag) under the seed as key, two 53-bit uniforms,
// Box-Muller; (g0, g1)/sqrt(2) for m > 0 and (g0, 0) for m = 0, so that
// E|n|^2 = 1 (a complex unit Gaussian, real for m = 0).
__device__ __forceinline__ double2 seeded_noise(unsigned long long seed, long long idx, int j,
                                                bool m0)
{
    const uint4 x = philox4x32_10(make_uint4((unsigned)idx, (unsigned)((unsigned long long)idx >> 32),
                                             (unsigned)j, 0x6e6f6973u),
                                  (unsigned)seed, (unsigned)(seed >> 32));
    const unsigned long long a = (((unsigned long long)x.y << 32) | x.x) >> 11;
    const unsigned long long b = (((unsigned long long)x.w << 32) | x.z) >> 11;
    const double u1 = (double)(a + 1) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)b * 0x1.0p-53;        // [0, 1)
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586477 * u2, &sn, &cs);
    if (m0) return make_double2(rad * cs, 0.0);
    const double h = 0.70710678118654752440;  // 1/sqrt(2)
    return make_double2(rad * cs * h, rad * sn * h);
}

// x: index idx = l(l+1)/2 + m, y: shell j; grid-stride in both (the grid is
// capped on the host).  Each thread decodes m = 0 once for all its shells.
template <typename T>
__global__ __launch_bounds__(256) void k_noise(Shape sh, unsigned long long seed, T *__restrict__ out)
{
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < sh.nlm;
         idx += (long long)gridDim.x * 256) {
        const bool m0 = lm_index(l_of_index(idx), 0) == idx;
        for (int j = blockIdx.y; j < sh.N; j += gridDim.y) {
            const double2 g = seeded_noise(seed, idx, j, m0);
            const long long t = (long long)j * sh.nlm + idx;
            out[2 * t] = (T)g.x;
            out[2 * t + 1] = (T)g.y;
        }
    }
}

// ---------------------------------------------------------------- filter

// Block = (l, 64-column tile), every output row; the block table lists the
// column tiles of one l back to back on one XCD (they share F_l in its L2).
// Columns are c = 2m + (re/im) of the noise row n[j][idx(l, 0) ..], so a
// complex coefficient is two real columns and the real filter multiplies
// both.  Rows come in RT = ceil(N/32) tiles of 32, each split into two 16-row
// halves; the four waves share the halves as described at the round loop, so
// that with a lower-triangular F (tile t only needs j < 32 t + 32) every
// chunk gives the waves nearly equal work.  The noise rows of a 32-row
// K-chunk are staged in LDS, double buffered, and shared by the four waves;
// the F^T fragments of the next chunk load while the block waits at the
// chunk's barrier.  The noise is read from HBM once.
constexpr int kFiltLD = 80;  // LDS row stride (elements): conflict-free B reads
// blocks per CU the filter's register budget is held to (two: the FP64
// kernel spills a few registers there and is still faster than at one; the
// FP64 kernel that generates its noise needs the whole register file)
template <typename T, bool SEEDED> constexpr int filter_blocks()
{
    return SEEDED && sizeof(T) == 8 ? 1 : 2;
}

// SEEDED: the noise is generated from `seed` (seeded_noise) instead of read
// from noise_in.  RADIAL: the block also forms the linear radial sums of its
// columns, a^X_L = sum_j V^X_lj n(r_j), into aL from the noise rows it
// stages (each noise value is then generated or read once); the seeded
// kernels and the FP32 stored-noise kernels do, the FP64 stored-noise one
// leaves them to k_radial_lin (it has no registers to spare).
template <typename T> constexpr bool filter_radial(bool seeded) { return seeded || sizeof(T) == 4; }

template <typename T, bool SEEDED = false, bool RADIAL = filter_radial<T>(SEEDED)>
__device__ __forceinline__ void body_filter(const Shape &sh, const T *__restrict__ FQ_in, int Kpad,
                                            int Mpad, int nchq, const int2 *__restrict__ tiles_in,
                                            const T *__restrict__ noise_in, T *__restrict__ phi_in,
                                            unsigned long long seed, const double *__restrict__ V_in,
                                            double2 *__restrict__ aL_in, int bx)
{
    auto *__restrict__ FQ = glb(FQ_in);
    auto *__restrict__ tiles = glb(tiles_in);
    auto *__restrict__ noise = glb(noise_in);
    auto *__restrict__ phi = glb(phi_in);
    using M = Mt<T>;
    using C2 = typename M::c2;
    __shared__ T nz[2][32][kFiltLD];
    const int2 tl = gload(tiles + bx);
    if (tl.x < 0) return;  // idle slot of the XCD layout (whole block)
    const int l = tl.x, col0 = tl.y * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int N = sh.N, ncol = 2 * (l + 1);
    const long long nlm = sh.nlm;
    const long long base = 2 * lm_index(l, 0);
    const auto FQl = FQ + (long long)l * nchq * Mpad * 32;
    const int RT = (N + 31) / 32;
    // staging role: thread t loads chunk row t / 8, columns 8 (t % 8) .. + 8
    const int sj = threadIdx.x >> 3, sc = (threadIdx.x & 7) * 8;
    auto stage_load = [&](int j0, T (&v)[8]) {
        const int j = j0 + sj;
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const int col = col0 + sc + e;  // even: (re, im) of m = col / 2
            C2 w;
            w.x = T(0);
            w.y = T(0);
            if (j < N && col < ncol) {
                if constexpr (!SEEDED) {
                    w = gload(reinterpret_cast<const GLB C2 *>(noise + (long long)j * 2 * nlm + base + col));
                } else {
                    const double2 g = seeded_noise(seed, base / 2 + col / 2, j, col == 0);
                    w.x = (T)g.x;
                    w.y = (T)g.y;
                }
            }
            v[e] = w.x;
            v[e + 1] = col == 0 ? T(0) : w.y;  // Im of m = 0 is ignored
        }
    };
    auto stage_store = [&](int buf, const T (&v)[8]) {
#pragma unroll
        for (int e = 0; e < 8; e++) nz[buf][sj][sc + e] = v[e];
    };
    // radial sums: per-thread FP64 partials, slot [X][e / 2][thread] holding
    // columns sc + e, sc + e + 1 of row group sj, each owned by one thread
    // until the final reduction.  Thread-minor, so a wave's 16-byte accesses
    // are 1 KB contiguous (no bank conflicts).
    __shared__ double2 rsum[RADIAL ? 2 : 1][RADIAL ? 4 : 1][RADIAL ? 256 : 1];
    auto radial_acc = [&](int j0, const T (&v)[8]) {
        if constexpr (RADIAL) {
            const int j = min(j0 + sj, N - 1);  // rows past N hold zeros
            const double vt = glb(V_in)[(long long)l * N + j];
            const double ve = glb(V_in)[(long long)(sh.L + 1 + l) * N + j];
#pragma unroll
            for (int h = 0; h < 4; h++) {
                double2 a = rsum[0][h][threadIdx.x], b = rsum[1][h][threadIdx.x];
                a.x += vt * (double)v[2 * h];
                a.y += vt * (double)v[2 * h + 1];
                b.x += ve * (double)v[2 * h];
                b.y += ve * (double)v[2 * h + 1];
                rsum[0][h][threadIdx.x] = a;
                rsum[1][h][threadIdx.x] = b;
            }
        }
    };
    if constexpr (RADIAL) {
#pragma unroll
        for (int h = 0; h < 4; h++) rsum[0][h][threadIdx.x] = rsum[1][h][threadIdx.x] = double2{0.0, 0.0};
    }

    // Work unit: a 16-row half tile (t, h).  Units are numbered by descending
    // t, u = 2 (RT - 1 - t) + h, and dealt round-robin in rounds of 16: wave w
    // takes u = w, w + 4, w + 8, w + 12.  With a lower-triangular F, chunk c
    // needs the units with t >= c; dealing them round-robin in descending t
    // keeps each wave's count of those within one of the other waves', so the
    // per-chunk barrier costs little imbalance (7 row tiles: 8 tile-chunks of
    // matrix work on the critical path against 10 for whole tiles).
    const int nhalf = 2 * RT;
    for (int u0 = 0; u0 < nhalf; u0 += 16) {
        int ts[4], hs[4];
        bool has[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int u = u0 + wave + 4 * s;
            has[s] = u < nhalf;
            ts[s] = RT - 1 - (u >> 1);
            hs[s] = u & 1;
        }
        // K-chunks this round needs: up to its largest tile
        const int kend = sh.lower ? min(Kpad, 32 * (RT - (u0 >> 1))) : Kpad;
        const int nchunk = (kend + 31) / 32;
        typename M::acc acc[4][4];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int c = 0; c < 4; c++) acc[s][c] = typename M::acc{};
        // F^T fragments of a chunk: [unit][K-step]; a lane's 8 K-steps of a
        // chunk for one 16-row half are 8 contiguous values
        T af[4][8];
        auto load_a = [&](int c, T (&A)[4][8]) {
            const auto Fc = FQl + (long long)c * Mpad * 32;
#pragma unroll
            for (int s = 0; s < 4; s++) {
                if (has[s]) {
                    const auto src = Fc + ((32 * ts[s] + 16 * hs[s] + i16) * 4 + k4) * 8;
                    using V4 = typename VecOf<typename std::conditional<sizeof(T) == 4, float4, double4>::type>::t;
                    const V4 lo = *reinterpret_cast<const GLB V4 *>(src);
                    const V4 hi = *reinterpret_cast<const GLB V4 *>(src + 4);
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        A[s][q] = lo[q];
                        A[s][4 + q] = hi[q];
                    }
                } else {
#pragma unroll
                    for (int ks = 0; ks < 8; ks++) A[s][ks] = T(0);
                }
            }
        };
        // FP32 stored-noise kernel: the noise rows load two chunks ahead (the
        // last chunks of a triangular F have too little matrix work to cover
        // one chunk's load); the FP64 and seeded kernels have no registers to
        // spare and stage one chunk ahead
        constexpr bool N2 = sizeof(T) == 4 && !SEEDED;
        T v[8], v2[N2 ? 8 : 1];
        stage_load(0, v);
        if (u0 == 0) radial_acc(0, v);  // the first round stages every row
        stage_store(0, v);
        if constexpr (N2) {
            if (nchunk > 1) stage_load(32, v2);
        }
        load_a(0, af);
        __syncthreads();
        for (int c = 0; c < nchunk; c++) {
            // MFMAs from LDS buffer c & 1 while the next chunk's noise rows
            // load; the next chunk's F^T fragments load after the MFMAs
            const int buf = c & 1;
            const bool more = c + 1 < nchunk;
            if constexpr (N2) {
                if (c + 2 < nchunk) stage_load(32 * (c + 2), v);
            } else if (more) {
                stage_load(32 * (c + 1), v);
                if (u0 == 0) radial_acc(32 * (c + 1), v);
            }
            const int j0 = 32 * c;
            // the units of a wave come in descending t, so the ones this
            // chunk meets (t >= c with a triangular F) are a prefix of them:
            // one branch per chunk selects a straight-line body for that many
            int na = 0;
#pragma unroll
            for (int s = 0; s < 4; s++) na += (has[s] && (!sh.lower || j0 < 32 * ts[s] + 32)) ? 1 : 0;
            auto chunk_mfma = [&](auto cnt) {
                constexpr int NA = decltype(cnt)::value;
#pragma unroll
                for (int ks = 0; ks < 8; ks++) {
                    T bv[4];
#pragma unroll
                    for (int cf = 0; cf < 4; cf++) bv[cf] = nz[buf][4 * ks + k4][16 * cf + i16];
#pragma unroll
                    for (int s = 0; s < NA; s++)
#pragma unroll
                        for (int cf = 0; cf < 4; cf++)
                            acc[s][cf] = M::mfma(af[s][ks], bv[cf], acc[s][cf]);
                }
            };
            switch (na) {
            case 4: chunk_mfma(std::integral_constant<int, 4>{}); break;
            case 3: chunk_mfma(std::integral_constant<int, 3>{}); break;
            case 2: chunk_mfma(std::integral_constant<int, 2>{}); break;
            case 1: chunk_mfma(std::integral_constant<int, 1>{}); break;
            default: break;
            }
            if (more) {
                if constexpr (N2) {
                    if (u0 == 0) radial_acc(32 * (c + 1), v2);  // the first round stages every row
                    stage_store(buf ^ 1, v2);
#pragma unroll
                    for (int e = 0; e < 8; e++) v2[e] = v[e];
                } else {
                    stage_store(buf ^ 1, v);
                }
                load_a(c + 1, af);
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < 4; s++) {
            if (!has[s]) continue;
#pragma unroll
            for (int cf = 0; cf < 4; cf++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int row = 32 * ts[s] + 16 * hs[s] + M::row(k4, r);
                    const int col = col0 + 16 * cf + i16;
                    if (row < N && col < ncol) {
                        const int m = col >> 1;
                        phi[mrow(sh.L, m, l) * sh.Cpad + 2 * row + (col & 1)] = acc[s][cf][r];
                    }
                }
        }
    }
    if constexpr (RADIAL) {
        __syncthreads();
        const int X = threadIdx.x >> 6, cl = threadIdx.x & 63, col = col0 + cl;
        if (X < 2 && col < ncol) {
            // column cl of row group g: thread 8 g + cl / 8, element cl % 8
            const int h = (cl & 7) >> 1, odd = cl & 1, q = cl >> 3;
            double a = 0.0;
            for (int g = 0; g < 32; g++) {
                const double2 r = rsum[X][h][8 * g + q];
                a += odd ? r.y : r.x;
            }
            reinterpret_cast<GLB double *>(glb(aL_in))[2 * (X * nlm + base / 2 + col / 2) + (col & 1)] = a;
        }
    }
}

template <typename T, bool SEEDED>
__global__ __launch_bounds__(256, (filter_blocks<T, SEEDED>())) void k_filter(Shape sh, const T *__restrict__ FQ, int Kpad,
                                                int Mpad, int nchq, const int2 *__restrict__ tiles,
                                                const T *__restrict__ noise, T *__restrict__ phi,
                                                unsigned long long seed, const double *__restrict__ V,
                                                double2 *__restrict__ aL)
{
    body_filter<T, SEEDED>(sh, FQ, Kpad, Mpad, nchq, tiles, noise, phi, seed, V, aL, blockIdx.x);
}

// ------------------------------------------------------- linear radial sum

__device__ inline void neumaier(double &s, double &c, double v)
{
    const double t = s + v;
    if (fabs(s) >= fabs(v))
        c += (s - t) + v;
    else
        c += (v - t) + s;
    s = t;
}

template <typename T>
__device__ __forceinline__ void body_radial_lin(const Shape &sh, const double *__restrict__ V_in,
                                                const T *__restrict__ noise_in,
                                                double2 *__restrict__ aL_in, int bid)
{
    auto *__restrict__ V = glb(V_in);
    auto *__restrict__ noise = glb(noise_in);
    auto *__restrict__ aL = glb(aL_in);
    const long long idx = (long long)bid * 256 + threadIdx.x;
    if (idx >= sh.nlm) return;
    const int l = l_of_index(idx);
    const bool m0 = lm_index(l, 0) == idx;
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    const auto VT = V + (long long)l * sh.N;
    const auto VE = V + (long long)(sh.L + 1) * sh.N + (long long)l * sh.N;
    // 8 shells per step: their loads are all issued before the (sequential)
    // compensated sums, so each wave keeps 8 rows of the noise in flight
    using C2 = typename Mt<T>::c2;
    constexpr int U = 8;
    const auto nz0 = noise + 2 * idx;
    const long long rstride = 2 * sh.nlm;
    for (int j0 = 0; j0 < sh.N; j0 += U) {
        C2 v[U];
        double vt[U], ve[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = min(j0 + u, sh.N - 1);
            v[u] = gload(reinterpret_cast<const GLB C2 *>(nz0 + (long long)j * rstride));
            vt[u] = VT[j];
            ve[u] = VE[j];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (j0 + u < sh.N) {
                const double re = (double)v[u].x;
                const double im = m0 ? 0.0 : (double)v[u].y;
                neumaier(s[0], c[0], vt[u] * re);
                neumaier(s[1], c[1], vt[u] * im);
                neumaier(s[2], c[2], ve[u] * re);
                neumaier(s[3], c[3], ve[u] * im);
            }
        }
    }
    gstore(aL + idx, make_double2(s[0] + c[0], s[1] + c[1]));
    gstore(aL + sh.nlm + idx, make_double2(s[2] + c[2], s[3] + c[3]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_radial_lin(Shape sh, const double *__restrict__ V,
                                                    const T *__restrict__ noise,
                                                    double2 *__restrict__ aL)
{
    body_radial_lin<T>(sh, V, noise, aL, blockIdx.x);
}

// -------------------------------------------------------- Legendre synthesis

// Pairs per synthesis wave: 64 in FP32, 32 in FP64 (register budget of the
// accumulators).  A synthesis workgroup is one wave.
template <typename T> constexpr int synth_pw() { return sizeof(T) == 8 ? kSynthPairsF64 : kSynthPairsF32; }
// LDS row stride of the transposed lambda tile (FP32: rows 2k apart land in
// disjoint bank quarters, so the A-fragment reads are conflict-free)
template <typename T> constexpr int synth_ld() { return sizeof(T) == 8 ? 36 : 72; }

// Block = (m, PW ring pairs, column tile of 16 CF columns), one wave.  The
// contraction index is l in K-steps of 8 (four even and four odd l - m).
// Lane q runs the FP64 three-term recurrence for pair q (mod PW) from the
// stored state; its 8 values per K-step go through a double-buffered LDS tile
// into the MFMA A layout (lane = (pair, k-slot)), so every recurrence step
// feeds NF = PW/16 pair fragments x 2 parities x CF column fragments of
// MFMAs.  The wave starts at the first stored state below the first l where
// any of its pairs has |lambda_lm| above the polar-skip threshold (1e-30,
// 1e-12 with FP32 data).
template <typename T, int CF>
__device__ __forceinline__ void body_synth(const Shape &sh, const int4 *__restrict__ tiles_in,
                                           const double *__restrict__ x_in,
                                           const double2 *__restrict__ seed_in,
                                           const int *__restrict__ seedoff_in,
                                           const int *__restrict__ lstart_in,
                                           const double2 *__restrict__ coef_in,
                                           const T *__restrict__ phi_in, T *__restrict__ G_in, int bid)
{
    auto *__restrict__ tiles = glb(tiles_in);
    auto *__restrict__ x = glb(x_in);
    auto *__restrict__ seed = glb(seed_in);
    auto *__restrict__ seedoff = glb(seedoff_in);
    auto *__restrict__ lstart = glb(lstart_in);
    auto *__restrict__ coef = glb(coef_in);
    auto *__restrict__ phi = glb(phi_in);
    auto *__restrict__ G = glb(G_in);
    using M = Mt<T>;
    constexpr int PW = synth_pw<T>();
    constexpr int NF = PW / 16;
    constexpr int LD = synth_ld<T>();
    __shared__ T lamT[2][8][LD];
    const int L = sh.L, npair = sh.npair, Cpad = sh.Cpad;
    const int4 tl = gload(tiles + bid);
    if (tl.x < 0) return;  // idle slot of the XCD layout
    // wave-uniform: keeps the coefficient addresses scalar
    const int m = __builtin_amdgcn_readfirstlane(tl.x);
    const int pt = __builtin_amdgcn_readfirstlane(tl.y);
    const int ct = __builtin_amdgcn_readfirstlane(tl.z);
    const auto cm_row = coef + crow(L, m);
    const int lane = threadIdx.x;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int p0 = pt * PW;
    const int p = p0 + (lane % PW);
    const bool pv = p < npair;
    const int nfa = min(NF, (npair - p0 + 15) / 16);  // fragments holding a pair
    const double xp = pv ? x[p] : 0.0;
    int ls = pv ? lstart[(long long)m * npair + p] : L + 1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) ls = min(ls, __shfl_xor(ls, o));
    // uniform after the reduction: lets the coefficient loads go scalar
    ls = __builtin_amdgcn_readfirstlane(ls);
    const int u0 = ls <= L ? (ls - m) / kSeedStride : 0;
    double l1 = 0.0, l2 = 0.0;
    if (pv && ls <= L) {
        const double2 st = gload(seed + ((long long)seedoff[m] + u0) * npair + p);
        l1 = st.x;
        l2 = st.y;
    }
    typename M::acc acc[NF][2][CF];
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int c = 0; c < CF; c++) acc[f][a][c] = typename M::acc{};
    const long long rowm = mrow(L, m, m);
    const int colb = ct * sh.CT + i16;
    const int lbeg = ls <= L ? m + u0 * kSeedStride : L + 1;
    // B operands of a K-step: rows l0 + 2 k4 (even l - m) and l0 + 2 k4 + 1 (odd).
    // Rows past l = L belong to the next m (or to the zero padding after the
    // last one) and meet lambda = 0 exactly, so no per-lane bounds are needed.
    const auto colbase = phi + rowm * Cpad + colb;
    auto loadB = [&](int l0, T *E, T *O) {
        const auto rE = colbase + (long long)(l0 + 2 * k4 - m) * Cpad;
#pragma unroll
        for (int cf = 0; cf < CF; cf++) {
            E[cf] = rE[16 * cf];
            O[cf] = rE[Cpad + 16 * cf];
        }
    };
    // FULL: every fragment holds a pair (all tiles but the last), so the
    // K-step has no branches between its LDS reads and MFMAs
    auto run = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        int buf = 0;
        auto kstep = [&](int l0, const T *E, const T *O) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                // rows past L are the zero padding of m's coefficient block, so
                // lambda = 0 there exactly
                const double2 ab = gload(cm_row + (l0 + q - m));
                const double nv = ab.x * xp * l1 - ab.y * l2;
                v[q] = nv;
                l2 = l1;
                l1 = nv;
            }
            if (PW == 64 || lane < PW) {
#pragma unroll
                for (int q = 0; q < 8; q++) lamT[buf][q][lane] = (T)v[q];
            }
            __syncthreads();  // one wave: orders the tile writes before the reads
#pragma unroll
            for (int f = 0; f < NF; f++) {
                if (FULL || f < nfa) {
                    const T aE = lamT[buf][2 * k4][16 * f + i16];
                    const T aO = lamT[buf][2 * k4 + 1][16 * f + i16];
#pragma unroll
                    for (int cf = 0; cf < CF; cf++) {
                        acc[f][0][cf] = M::mfma(aE, E[cf], acc[f][0][cf]);
                        acc[f][1][cf] = M::mfma(aO, O[cf], acc[f][1][cf]);
                    }
                }
            }
            buf ^= 1;
        };
        // two K-steps per trip with the operand buffers swapping roles; the
        // prefetch is unconditional (it may read up to 15 rows past the last m
        // block, which is zero padding) so no wait has to cover a load that
        // might not have been issued
        T bE[CF], bO[CF], nE[CF], nO[CF];
        const int nks = lbeg <= L ? (L - lbeg) / 8 + 1 : 0;
        int l0 = lbeg;
        if (nks > 0) loadB(l0, bE, bO);
        for (int it = 0; it < nks / 2; it++) {
            loadB(l0 + 8, nE, nO);
            kstep(l0, bE, bO);
            loadB(l0 + 16, bE, bO);
            kstep(l0 + 8, nE, nO);
            l0 += 16;
        }
        if (nks & 1) kstep(l0, bE, bO);
    };
    if (nfa == NF)
        run(std::true_type{});
    else
        run(std::false_type{});
    // G[pair][m][column] holds (E, O) interleaved
    using C2V = typename M::c2v;
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int cf = 0; cf < CF; cf++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int pair = p0 + 16 * f + M::row(k4, r);
                if (pair < npair) {
                    C2V v;
                    v.x = acc[f][0][cf][r];
                    v.y = acc[f][1][cf][r];
                    gstore(reinterpret_cast<GLB C2V *>(
                               G + ((((long long)pair * (L + 1) + m) * Cpad) + colb + 16 * cf) * 2),
                           v);
                }
            }
}

// waves per SIMD the synthesis register budget is held to
template <typename T> constexpr int synth_waves() { return 2; }

template <typename T, int CF>
__global__ __launch_bounds__(64, synth_waves<T>()) void k_synth(Shape sh,
                                                               const int4 *__restrict__ tiles,
                                                               const double *__restrict__ x,
                                                               const double2 *__restrict__ seed,
                                                               const int *__restrict__ seedoff,
                                                               const int *__restrict__ lstart,
                                                               const double2 *__restrict__ coef,
                                                               const T *__restrict__ phi,
                                                               T *__restrict__ G)
{
    body_synth<T, CF>(sh, tiles, x, seed, seedoff, lstart, coef, phi, G, blockIdx.x);
}

// Block = (ring pair p, S consecutive shells), 256 threads per shell.  The
// north and south rings travel together as one complex sequence
// z = f_N + i f_S: spectrum Z_m = N_m + i S_m for 0 <= m <= L and
// Z_{n-m} = conj(N_m) + i conj(S_m), with N = E + O and S = E - O.  After the
// inverse FFT, w = f_N^2 + i f_S^2 goes through the forward FFT and the two
// real spectra separate as (W_m + conj W_{n-m})/2 and (W_m - conj W_{n-m})/(2i).
// With n = 3L the DFT bin L also holds mode -2L of the square, n conj(G_L)^2,
// which is subtracted.  G and F rows hold (E, O) interleaved per column, so
// one (m, shell) is 4 contiguous values; the loads and stores map adjacent
// threads to adjacent shells of the block (4 S contiguous values per m).
// Blocks are numbered so that consecutive shell groups of one pair run on the
// same XCD (shared L2 lines).
template <typename T, int NMAX, int S, bool PLANNED>
__device__ __forceinline__ void body_ring(const Shape &sh, const double *__restrict__ wq_in,
                                          const typename Mt<T>::c2 *__restrict__ tw_in,
                                          const T *__restrict__ G_in, T *__restrict__ F_in,
                                          double *__restrict__ maps, int mode, int bid)
{
    auto *__restrict__ wq = glb(wq_in);
    auto *__restrict__ tw = glb(tw_in);
    auto *__restrict__ G = glb(G_in);
    auto *__restrict__ F = glb(F_in);
    using C2 = typename Mt<T>::c2;
    using Q = typename Mt<T>::quad;
    extern __shared__ unsigned char smem_raw[];
    const int L = sh.L, n = sh.nphi, Cpad = sh.Cpad, npad = ring_pad(n);
    const int ngrp = (sh.N + S - 1) / S;
    const int nblk = sh.npair * ngrp;
    const int nslot = (nblk + 7) / 8;
    const int logical = (bid & 7) * nslot + (bid >> 3);
    if (logical >= nblk) return;  // whole block
    const int s0 = (logical % ngrp) * S, p = logical / ngrp;
    const bool eq = sh.equator && p == sh.npair - 1;
    // FFT role: shell s0 + g, thread tid of its 256
    const int g = threadIdx.x >> 8, tid = threadIdx.x & 255;
    C2 *buf = reinterpret_cast<C2 *>(smem_raw) + g * npad;
    // load/store role: shell s0 + io, every S-th m from mq
    const int io = threadIdx.x % S, mq = threadIdx.x / S;
    C2 *iob = reinterpret_cast<C2 *>(smem_raw) + io * npad;
    const bool iov = s0 + io < sh.N;
    const auto Gp = G + ((long long)p * (L + 1) * Cpad + 2 * (s0 + io)) * 2;

    // bins (L, n - L) are empty; the loop below writes every other bin
    for (int q = L + 1 + tid; q < n - L; q += 256) {
        C2 z;
        z.x = T(0);
        z.y = T(0);
        buf[rix(q)] = z;
    }
    // every load of the thread is issued before the first is used (one
    // memory latency per block instead of one per row)
    constexpr int KM = (NMAX / 3 + 256) / 256;  // rows per thread: L <= n/3 <= NMAX/3
    Q v[KM];
#pragma unroll
    for (int k = 0; k < KM; k++) {
        const int m = mq + 256 * k;
        if (iov && m <= L)
            v[k] = gload(reinterpret_cast<const GLB Q *>(Gp + (long long)m * Cpad * 2));
        else
            v[k] = Q{};
    }
#pragma unroll
    for (int k = 0; k < KM; k++) {
        const int m = mq + 256 * k;
        if (m > L) break;
        const T Er = v[k].x, Or = v[k].y, Ei = v[k].z, Oi = v[k].w;
        T Nr = Er + Or, Ni = Ei + Oi, Sr = Er - Or, Si = Ei - Oi;
        if (eq) Sr = Si = T(0);
        if (m == 0) Ni = Si = T(0);
        C2 z;
        z.x = Nr - Si;
        z.y = Ni + Sr;
        iob[rix(m)] = z;
        if (m > 0) {
            z.x = Nr + Si;
            z.y = Sr - Ni;
            iob[rix(n - m)] = z;
        }
    }
    __syncthreads();
    fft_lds<C2, true, NMAX, PLANNED>(buf, sh, tw, tid);
    if (mode == 1) {
        if (s0 + g >= sh.N) return;  // no barrier follows
        const long long nr = sh.nring, sg = s0 + g;
        for (int j = tid; j < n; j += 256) {
            const C2 z = buf[rix(j)];
            maps[(sg * nr + p) * n + j] = (double)z.x;
            if (!eq) maps[(sg * nr + (nr - 1 - p)) * n + j] = (double)z.y;
        }
        return;
    }
    for (int j = tid; j < n; j += 256) {
        C2 z = buf[rix(j)];
        z.x = z.x * z.x;
        z.y = z.y * z.y;
        buf[rix(j)] = z;
    }
    __syncthreads();
    fft_lds<C2, false, NMAX, PLANNED>(buf, sh, tw, tid);

    const T wgt = (T)wq[p];
    const T half = T(0.5);
    const auto Fp = F + ((long long)p * Cpad + 2 * (s0 + io)) * 2;
    for (int m = mq; m <= L; m += 256) {
        const C2 W1 = iob[rix(m)];
        const C2 W2 = iob[rix(m == 0 ? 0 : n - m)];
        T Ar = half * (W1.x + W2.x), Ai = half * (W1.y - W2.y);
        T Br = half * (W1.y + W2.y), Bi = -half * (W1.x - W2.x);
        if (sh.alias && m == L && iov) {
            const Q v = gload(reinterpret_cast<const GLB Q *>(Gp + (long long)L * Cpad * 2));
            const T Er = v.x, Or = v.y, Ei = v.z, Oi = v.w;
            T Nr = Er + Or, Ni = Ei + Oi, Sr = Er - Or, Si = Ei - Oi;
            if (eq) Sr = Si = T(0);
            const T fn = (T)n;
            Ar -= fn * (Nr * Nr - Ni * Ni);
            Ai -= fn * (-T(2) * Nr * Ni);
            Br -= fn * (Sr * Sr - Si * Si);
            Bi -= fn * (-T(2) * Sr * Si);
        }
        if (eq) Br = Bi = T(0);
        Q f;
        f.x = wgt * (Ar + Br);  // E re
        f.y = wgt * (Ar - Br);  // O re
        f.z = wgt * (Ai + Bi);  // E im
        f.w = wgt * (Ai - Bi);  // O im
        if (eq) f.y = f.w = T(0);
        if (m == 0) f.z = f.w = T(0);
        if (iov) gstore(reinterpret_cast<GLB Q *>(Fp + (long long)m * sh.npair * Cpad * 2), f);
    }
}

// default shells per ring block: 2 in FP32 (512 threads), 1 in FP64 (the
// grouped batch kernels always use these)
template <typename T> constexpr int ring_s() { return sizeof(T) == 4 ? kRingShellsF32 : kRingShellsF64; }

// S shells per block (Shape::rs): the single-context launches take the
// context's choice, 1 or 2 in FP32
template <typename T, int NMAX, bool PLANNED, int S>
__global__ __launch_bounds__(256 * S) void k_ring(Shape sh, const double *__restrict__ wq,
                                                  const typename Mt<T>::c2 *__restrict__ tw,
                                                  const T *__restrict__ G, T *__restrict__ F,
                                                  double *__restrict__ maps, int mode)
{
    body_ring<T, NMAX, S, PLANNED>(sh, wq, tw, G, F, maps, mode, blockIdx.x);
}

// --------------------------------------------------------- Legendre analysis

// Rows per analysis wave (kAnalRowsF32 / kAnalRowsF64); pairs per chunk; LDS
// row strides that keep the A-fragment reads free of bank conflicts.
template <typename T> constexpr int anal_rw() { return sizeof(T) == 8 ? kAnalRowsF64 : kAnalRowsF32; }
template <typename T> constexpr int anal_ld() { return sizeof(T) == 8 ? 33 : 34; }
constexpr int kAnalPC = 32;
static_assert(kCoefPad >= anal_rw<float>() && kCoefPad >= anal_rw<double>(), "coefficient padding");

// Block = (m, RW l rows from l0 = m + RW t, column tile), one wave.  Rows with
// l - m even meet F_E, odd ones F_O: NF = RW/32 fragments of 16 rows per
// parity.  For each chunk of 32 ring pairs, lane (half h, pair q) runs the
// FP64 recurrence over rows [h RW/2, (h+1) RW/2) of pair q from the stored
// state, writes the values to an LDS tile, and the wave reads them back in the
// MFMA A layout (lane = (row, pair)).  Chunks and fragments whose rows all lie
// below the first l where any pair of the chunk has |lambda| above the
// polar-skip threshold (1e-30, 1e-12 with FP32 data) are skipped.  mode 0 folds the radial sum into the epilogue:
// part[ct][X][idx(l, m)] = sum_s W^X_ls Phi_NL,lm(s) over the tile's shells;
// mode 1 writes Phi_NL per shell; mode 2 (reverse pass) writes the per-shell
// output plus the direct cotangent sum_X W^X_ls abar^X_lm, no mean handling.
template <typename T, int CF, int MODE>
__device__ __forceinline__ void body_anal(const Shape &sh, const int4 *__restrict__ tiles_in,
                                          const double *__restrict__ x_in,
                                          const double2 *__restrict__ coef_in,
                                          const double2 *__restrict__ seed_in,
                                          const int *__restrict__ seedoff_in,
                                          const int *__restrict__ cmin_in,
                                          const double *__restrict__ W_in,
                                          const double *__restrict__ mu_in,
                                          const T *__restrict__ F_in, double2 *__restrict__ part_in,
                                          T *__restrict__ outphi_in,
                                          const double2 *__restrict__ gT_in,
                                          const double2 *__restrict__ gE_in, int bid)
{
    auto *__restrict__ tiles = glb(tiles_in);
    auto *__restrict__ x = glb(x_in);
    auto *__restrict__ coef = glb(coef_in);
    auto *__restrict__ seed = glb(seed_in);
    auto *__restrict__ seedoff = glb(seedoff_in);
    auto *__restrict__ cmin = glb(cmin_in);
    auto *__restrict__ F = glb(F_in);
    using M = Mt<T>;
    constexpr int RW = anal_rw<T>();
    constexpr int NF = RW / 32;
    constexpr int LD = anal_ld<T>();
    __shared__ T lam[RW][LD];
    // recurrence coefficients (A, B) of the block's RW rows: the two wave
    // halves run different rows, so a per-lane coefficient read from LDS
    // (two broadcast addresses per wave) replaces a per-lane select between
    // two sets of scalar registers
    __shared__ double2 cab[RW];
    const int L = sh.L, npair = sh.npair, Cpad = sh.Cpad;
    const int4 tl = gload(tiles + bid);
    if (tl.x < 0) return;  // idle slot of the XCD layout
    // wave-uniform: keeps the coefficient addresses scalar
    const int m = __builtin_amdgcn_readfirstlane(tl.x);
    const int lt = __builtin_amdgcn_readfirstlane(tl.y);
    const int ct = __builtin_amdgcn_readfirstlane(tl.z);
    const auto cm_row = coef + crow(L, m);
    const int lane = threadIdx.x;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int half = lane >> 5, pl = lane & 31;
    const int l0w = m + lt * RW;
    const int lh = l0w + half * (RW / 2);  // first recurrence row of this lane
    const bool hact = lh <= L;
    const long long srow = (long long)seedoff[m] + (hact ? (lh - m) / kSeedStride : 0);
    // rows past l = L take the zero padding of m's coefficient block
    for (int r = lane; r < RW; r += 64) cab[r] = gload(cm_row + (l0w - m) + r);
    __syncthreads();
    typename M::acc acc[NF][2][CF];
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int c = 0; c < CF; c++) acc[f][a][c] = typename M::acc{};
    const int colb = ct * sh.CT + i16;
    const int nchunk = (npair + kAnalPC - 1) / kAnalPC;
    const int lend = l0w + RW - 1;
    // fragments holding a row l <= L (fragment f covers rows l0w + 32 f ..)
    const int fend = min(NF, (L - l0w) / 32 + 1);
    // equator first: every l tile of an (m, column tile) group starts at the
    // last chunk, so tiles that run together read the same F lines; the ones
    // with polar chunks to skip finish early instead of starting late
    for (int pc = nchunk - 1; pc >= 0; pc--) {
        const auto cmc = cmin + ((long long)m * nchunk + pc) * kCminW;
        const int cm = cmc[0];
        if (cm > lend) continue;  // wave-uniform
        // B operands F_{E/O}[pair][column] of a K-step (4 pairs); pairs past
        // the last one read the next m (or the zero padding after the last m)
        // and meet lambda = 0 exactly
        // F[m][pair][column] holds (E, O) interleaved
        const auto fbase = F + (((long long)m * npair + pc * kAnalPC + k4) * Cpad + colb) * 2;
        // F operands two K-steps ahead in three rotating register sets (the
        // K-steps are unrolled, so the set of each step is fixed at compile
        // time)
        T fb[3][2][CF];
        auto loadF = [&](int kk, T *E, T *O) {
            const auto f = fbase + (long long)(4 * kk) * Cpad * 2;
#pragma unroll
            for (int cf = 0; cf < CF; cf++) {
                const typename M::c2v v = gload(reinterpret_cast<const GLB typename M::c2v *>(f + 32 * cf));
                E[cf] = v.x;
                O[cf] = v.y;
            }
        };
        loadF(0, fb[0][0], fb[0][1]);
        loadF(1, fb[1][0], fb[1][1]);
        {
            const int p = pc * kAnalPC + pl;
            const bool pv = hact && p < npair;
            double a1 = 0.0, a0 = 0.0, xp = 0.0;  // lambda_{l-1}, lambda_{l-2}
            if (pv) {
                const double2 sd = gload(seed + srow * npair + p);
                a1 = sd.x;
                a0 = sd.y;
                xp = x[p];
            }
#pragma unroll 4
            for (int q = 0; q < RW / 2; q++) {
                const double2 ab = cab[half * (RW / 2) + q];
                const double v = ab.x * xp * a1 - ab.y * a0;
                lam[half * (RW / 2) + q][pl] = (T)v;
                a0 = a1;
                a1 = v;
            }
        }
        __syncthreads();
        // per K-step polar start: the first fragment with a row at or above
        // the first l where any of the K-step's 4 pairs exceeds the threshold
        auto kstep = [&](int kk, const T *E, const T *O) {
            const int ck = cmc[1 + kk];
            const int f0 = ck <= l0w + 31 ? 0 : (ck - l0w) / 32;
#pragma unroll
            for (int f = 0; f < NF; f++) {
                if (f >= f0 && f < fend) {
                    const T aE = lam[2 * (16 * f + i16)][4 * kk + k4];
                    const T aO = lam[2 * (16 * f + i16) + 1][4 * kk + k4];
#pragma unroll
                    for (int cf = 0; cf < CF; cf++) {
                        acc[f][0][cf] = M::mfma(aE, E[cf], acc[f][0][cf]);
                        acc[f][1][cf] = M::mfma(aO, O[cf], acc[f][1][cf]);
                    }
                }
            }
        };
        // 8 K-steps, each issuing the loads of the step two ahead (none past
        // the chunk's last step).  Measured: 2.90 ms against 3.27 ms for a
        // one-step-ahead rolled loop at the paper workload (FP32), although
        // the extra registers take the kernel from four waves per SIMD to
        // three; three steps ahead gains nothing more.
#pragma unroll
        for (int kk = 0; kk < kAnalPC / 4; kk++) {
            if (kk + 2 < kAnalPC / 4) loadF(kk + 2, fb[(kk + 2) % 3][0], fb[(kk + 2) % 3][1]);
            kstep(kk, fb[kk % 3][0], fb[kk % 3][1]);
        }
        __syncthreads();
    }

    anal_epilogue<T, CF, MODE, NF>(sh, acc, m, l0w, ct, colb, k4, i16, W_in, mu_in, part_in, outphi_in,
                                   gT_in, gE_in);
}

// waves per SIMD the analysis register budget is held to
template <typename T> constexpr int anal_waves() { return 2; }

template <typename T, int CF, int MODE>
__global__ __launch_bounds__(64, anal_waves<T>()) void k_anal(Shape sh, const int4 *__restrict__ tiles,
                                              const double *__restrict__ x,
                                              const double2 *__restrict__ coef,
                                              const double2 *__restrict__ seed,
                                              const int *__restrict__ seedoff,
                                              const int *__restrict__ cmin,
                                              const double *__restrict__ W,
                                              const double *__restrict__ mu,
                                              const T *__restrict__ F, double2 *__restrict__ part,
                                              T *__restrict__ outphi,
                                              const double2 *__restrict__ gT,
                                              const double2 *__restrict__ gE)
{
    body_anal<T, CF, MODE>(sh, tiles, x, coef, seed, seedoff, cmin, W, mu, F, part, outphi, gT,
                           gE, blockIdx.x);
}

// -------------------------------------------------------------- combine

__device__ __forceinline__ void body_combine(const Shape &sh, const double2 *__restrict__ part_in,
                                             const double2 *__restrict__ aL_in, double fnl,
                                             double2 *__restrict__ aT_in, double2 *__restrict__ aE_in,
                                             double2 *__restrict__ aTn_in, double2 *__restrict__ aEn_in,
                                             int bid)
{
    auto *__restrict__ part = glb(part_in);
    auto *__restrict__ aL = glb(aL_in);
    auto *__restrict__ aT = glb(aT_in);
    auto *__restrict__ aE = glb(aE_in);
    auto *__restrict__ aTn = glb(aTn_in);
    auto *__restrict__ aEn = glb(aEn_in);
    const long long idx = (long long)bid * 256 + threadIdx.x;
    if (idx >= sh.nlm) return;
    const int l = l_of_index(idx);
    const bool m0 = lm_index(l, 0) == idx;
#pragma unroll
    for (int X = 0; X < 2; X++) {
        double sr = 0, cr = 0, si = 0, ci = 0;
        for (int ct = 0; ct < sh.nct; ct++) {
            const double2 v = gload(part + ((long long)ct * 2 + X) * sh.nlm + idx);
            neumaier(sr, cr, v.x);
            neumaier(si, ci, v.y);
        }
        double2 nl = make_double2(sr + cr, m0 ? 0.0 : si + ci);
        const double2 lin = gload(aL + (long long)X * sh.nlm + idx);
        double2 tot = make_double2(lin.x + fnl * nl.x, m0 ? 0.0 : lin.y + fnl * nl.y);
        if (X == 0) {
            gstore(aT + idx, tot);
            if (aTn) gstore(aTn + idx, nl);
        } else {
            gstore(aE + idx, tot);
            if (aEn) gstore(aEn + idx, nl);
        }
    }
}

__global__ __launch_bounds__(256) void k_combine(Shape sh, const double2 *__restrict__ part,
                                                 const double2 *__restrict__ aL, double fnl,
                                                 double2 *__restrict__ aT, double2 *__restrict__ aE,
                                                 double2 *__restrict__ aTn,
                                                 double2 *__restrict__ aEn)
{
    body_combine(sh, part, aL, fnl, aT, aE, aTn, aEn, blockIdx.x);
}

// ----------------------------------------------------- grouped (batch) entry
//
// A batch of contexts runs each stage as one launch: block b belongs to the
// context c with off[c] <= b < off[c+1] (offsets are multiples of 8, so the
// XCD-aware numbering of the ring stage is kept per context) and runs that
// context's block b - off[c].  Items carry each context's shape, buffers and
// the per-call pointers.

__device__ inline int group_find(const int *__restrict__ off, int n, int b, int &local)
{
    int lo = 0, hi = n;  // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    local = b - off[lo];
    return lo;
}

template <typename T>
__global__ __launch_bounds__(256) void g_radial_lin(const GroupItem *__restrict__ it,
                                                    const int *__restrict__ ord,
                                                    const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    if (lb >= (int)((g.sh.nlm + 255) / 256)) return;
    body_radial_lin<T>(g.sh, g.b.V, (const T *)g.noise, g.b.aL, lb);
}

template <typename T>
__global__ __launch_bounds__(256, (filter_blocks<T, false>())) void g_filter(const GroupItem *__restrict__ it,
                                                const int *__restrict__ ord,
                                                const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    if (lb >= g.b.nk1) return;
    body_filter<T>(g.sh, (const T *)g.b.FQ, g.b.Kpad, g.b.Mpad, g.b.nchq, g.b.k1tiles,
                   (const T *)g.noise, (T *)g.b.phi, 0ull, g.b.V, g.b.aL, lb);
}

template <typename T, int CF>
__global__ __launch_bounds__(64, synth_waves<T>()) void g_synth(const GroupItem *__restrict__ it,
                                               const int *__restrict__ ord,
                                               const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    if (lb >= g.b.nk2) return;
    body_synth<T, CF>(g.sh, g.b.k2tiles, g.b.x, g.b.seed, g.b.seedoff, g.b.lstart_mat, g.b.coef,
                      (const T *)g.b.phi, (T *)g.b.G, lb);
}

template <typename T, int NMAX, bool PLANNED>
__global__ __launch_bounds__(256 * ring_s<T>()) void g_ring(const GroupItem *__restrict__ it,
                                              const int *__restrict__ ord,
                                              const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    body_ring<T, NMAX, ring_s<T>(), PLANNED>(g.sh, g.b.wq, (const typename Mt<T>::c2 *)g.b.tw,
                                    (const T *)g.b.G, (T *)g.b.F, nullptr, 0, lb);
}

template <typename T, int CF>
__global__ __launch_bounds__(64, anal_waves<T>()) void g_anal(const GroupItem *__restrict__ it,
                                              const int *__restrict__ ord,
                                              const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    if (lb >= g.b.nk4) return;
    body_anal<T, CF, 0>(g.sh, g.b.k4tiles, g.b.x, g.b.coef, g.b.seed, g.b.seedoff, g.b.cmin,
                        g.b.W, g.b.mu, (const T *)g.b.F, g.b.part, nullptr, nullptr, nullptr, lb);
}

__global__ __launch_bounds__(256) void g_combine(const GroupItem *__restrict__ it,
                                                 const int *__restrict__ ord,
                                                 const int *__restrict__ off, int n)
{
    int lb;
    const int k = group_find(off, n, blockIdx.x, lb);
    const GroupItem &g = it[ord[k]];
    if (lb >= (int)((g.sh.nlm + 255) / 256)) return;
    body_combine(g.sh, g.b.part, g.b.aL, g.fnl, g.aT, g.aE, nullptr, nullptr, lb);
}

// --------------------------------------------------------- recurrence seeds

// One thread per (m, pair): run lambda_lm(x_p) up l, store the recurrence
// state (lambda_{l0-1}, lambda_{l0-2}) entering every l0 = m + 32 u, and the
// first l where |lambda_lm| exceeds 1e-30 (lstart) and where it exceeds
// tiny_mat (lstart_mat, written only when it is a separate table).
__global__ __launch_bounds__(256) void k_seed_init(Shape sh, const double *__restrict__ x,
                                                   const double *__restrict__ lmm,
                                                   const double2 *__restrict__ coef,
                                                   const int *__restrict__ seedoff,
                                                   double2 *__restrict__ seed,
                                                   int *__restrict__ lstart,
                                                   int *__restrict__ lstart_mat, double tiny_mat)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int npair = sh.npair, L = sh.L;
    if (t >= (long long)(L + 1) * npair) return;
    const int p = (int)(t % npair), m = (int)(t / npair);
    const double xp = x[p];
    double l1 = 0.0, l2 = lmm[(long long)m * npair + p];
    int first = L + 1, first_mat = L + 1;
    for (int l = m; l <= L; l++) {
        const int d = l - m;
        if (d % kSeedStride == 0)
            seed[((long long)seedoff[m] + d / kSeedStride) * npair + p] = make_double2(l1, l2);
        const double2 ab = coef[crow(L, m) + d];
        const double v = ab.x * xp * l1 - ab.y * l2;
        if (first > L && fabs(v) > kLambdaTiny) first = l;
        if (first_mat > L && fabs(v) > tiny_mat) first_mat = l;
        l2 = l1;
        l1 = v;
    }
    lstart[(long long)m * npair + p] = first;
    if (lstart_mat != lstart) lstart_mat[(long long)m * npair + p] = first_mat;
}

static_assert(kCminW == 1 + kAnalPC / 4, "one polar-start entry per chunk and per K-step");

// One thread per (m, 32-pair chunk): the first l where any pair of the chunk
// has |lambda_lm| above the threshold, then the same for each 4-pair K-step.
__global__ __launch_bounds__(256) void k_chunk_min(Shape sh, const int *__restrict__ lstart,
                                                   int *__restrict__ cmin)
{
    const int nchunk = (sh.npair + kAnalPC - 1) / kAnalPC;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)(sh.L + 1) * nchunk) return;
    const int c = (int)(t % nchunk), m = (int)(t / nchunk);
    int v = sh.L + 1;
    for (int k = 0; k < kAnalPC / 4; k++) {
        int vk = sh.L + 1;
        for (int p = c * kAnalPC + 4 * k; p < min(sh.npair, c * kAnalPC + 4 * k + 4); p++)
            vk = min(vk, lstart[(long long)m * sh.npair + p]);
        cmin[t * kCminW + 1 + k] = vk;
        v = min(v, vk);
    }
    cmin[t * kCminW] = v;
}

// ---------------------------------------------------------- layout helpers

template <typename T>
__global__ __launch_bounds__(256) void k_phi_to_api(Shape sh, const T *__restrict__ phi,
                                                    double2 *__restrict__ api)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sh.nlm * sh.N) return;
    const long long idx = t % sh.nlm;
    const int s = (int)(t / sh.nlm);
    const int l = l_of_index(idx);
    const int m = (int)(idx - lm_index(l, 0));
    const T *src = phi + mrow(sh.L, m, l) * sh.Cpad + 2 * s;
    api[t] = make_double2((double)src[0], m == 0 ? 0.0 : (double)src[1]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_api_to_phi(Shape sh, const double2 *__restrict__ api,
                                                    T *__restrict__ phi)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sh.nlm * sh.N) return;
    const long long idx = t % sh.nlm;
    const int s = (int)(t / sh.nlm);
    const int l = l_of_index(idx);
    const int m = (int)(idx - lm_index(l, 0));
    T *dst = phi + mrow(sh.L, m, l) * sh.Cpad + 2 * s;
    const double2 v = api[t];
    dst[0] = (T)v.x;
    dst[1] = m == 0 ? T(0) : (T)v.y;
}

// ------------------------------------------------------------ reverse pass

// Transposed radial sum, written as a synthesis input: for every (l, m) and
// shell s, sum_X W^X_ls abar^X_lm.  The adjoint of the analysis sums every
// stored (l, m >= 0) once, while the synthesis kernels weight m > 0 twice
// (real field), so m > 0 is halved here.  For the sample mean the (0, 0)
// entry is dropped: the derivative of the removed sky mean cancels it.
//
// Block = kRadAdjRows consecutive (l, m) rows, one wave per row at a time
// (l and m wave-uniform); lane = shell, so the W loads and the (re, im)
// stores of a row are contiguous.
constexpr int kRadAdjRows = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_radial_adj(Shape sh, const double *__restrict__ W,
                                                    const double2 *__restrict__ gT,
                                                    const double2 *__restrict__ gE,
                                                    T *__restrict__ out)
{
    using C2 = typename Mt<T>::c2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int Npad = sh.Cpad / 2;
    for (int r = w; r < kRadAdjRows; r += 4) {
        const long long idx = (long long)blockIdx.x * kRadAdjRows + r;
        if (idx >= sh.nlm) break;  // wave-uniform
        const int l = __builtin_amdgcn_readfirstlane(l_of_index(idx));
        const int m = (int)(idx - lm_index(l, 0));
        const double2 a = gT[idx], e = gE[idx];
        // m > 0 halved; Im of m = 0 is zero; (0, 0) dropped for the sample mean
        const double h = (m == 0 && l == 0 && sh.mean_mode == 0) ? 0.0 : m > 0 ? 0.5 : 1.0;
        const double hi = m > 0 ? 0.5 : 0.0;
        const double *Wt = W + (long long)l * Npad;
        const double *We = W + (long long)(sh.L + 1 + l) * Npad;
        C2 *dst = reinterpret_cast<C2 *>(out + mrow(sh.L, m, l) * sh.Cpad);
        for (int s = lane; s < sh.N; s += 64) {
            const double wt = Wt[s], we = We[s];
            C2 v;
            v.x = (T)(h * (wt * a.x + we * e.x));
            v.y = (T)(hi * (wt * a.y + we * e.y));
            dst[s] = v;
        }
    }
}

// Reverse ring stage, block = (ring pair, shell).  Both the Phi_L map (from
// G) and the transposed-analysis map ghat (from G2, pixel weights applied
// here) are rebuilt by inverse FFTs; phibar = 2 f_NL Phi_L ghat is formed
// pixel by pixel together with this block's share of dLoss/df_NL =
// sum_pix Phi_L^2 ghat, and phibar goes through the forward FFT.  The
// transposed synthesis needs c_m sum_pix phibar e^{-i m phi}; with n = 3L the
// bin L also holds mode -2L of phibar, 2 f_NL w conj(G_L) conj(G2_L) n, which
// is removed.
template <typename T, int NMAX, bool PLANNED>
__global__ __launch_bounds__(256) void k_ring_adj(Shape sh, const double *__restrict__ wq,
                                                  const typename Mt<T>::c2 *__restrict__ tw,
                                                  const T *__restrict__ G,
                                                  const T *__restrict__ G2, T *__restrict__ F,
                                                  double *__restrict__ fpart, double fnl)
{
    using C2 = typename Mt<T>::c2;
    using Q = typename Mt<T>::quad;
    extern __shared__ unsigned char smem_raw[];
    const int L = sh.L, n = sh.nphi, Cpad = sh.Cpad;
    C2 *b1 = reinterpret_cast<C2 *>(smem_raw);
    C2 *b2 = b1 + ring_pad(n);
    __shared__ double red[256];
    const int nblk = sh.npair * sh.N;
    const int nslot = (nblk + 7) / 8;
    const int logical = (blockIdx.x & 7) * nslot + (blockIdx.x >> 3);
    if (logical >= nblk) return;
    const int s = logical % sh.N, p = logical / sh.N;
    const int tid = threadIdx.x;
    const bool eq = sh.equator && p == sh.npair - 1;

    for (int q = tid; q < n; q += 256) {
        C2 z;
        z.x = T(0);
        z.y = T(0);
        b1[rix(q)] = z;
        b2[rix(q)] = z;
    }
    __syncthreads();
    // G, G2 and F rows hold (E, O) interleaved per column
    const long long poff = ((long long)p * (L + 1) * Cpad + 2 * s) * 2;
    for (int m = tid; m <= L; m += 256) {
#pragma unroll
        for (int which = 0; which < 2; which++) {
            const Q v = *reinterpret_cast<const Q *>((which ? G2 : G) + poff + (long long)m * Cpad * 2);
            const T Er = v.x, Or = v.y, Ei = v.z, Oi = v.w;
            T Nr = Er + Or, Ni = Ei + Oi, Sr = Er - Or, Si = Ei - Oi;
            if (eq) Sr = Si = T(0);
            if (m == 0) Ni = Si = T(0);
            C2 *bb = which ? b2 : b1;
            C2 z;
            z.x = Nr - Si;
            z.y = Ni + Sr;
            bb[rix(m)] = z;
            if (m > 0) {
                z.x = Nr + Si;
                z.y = Sr - Ni;
                bb[rix(n - m)] = z;
            }
        }
    }
    __syncthreads();
    fft_lds<C2, true, NMAX, PLANNED>(b1, sh, glb(tw), tid);
    fft_lds<C2, true, NMAX, PLANNED>(b2, sh, glb(tw), tid);
    const T wpix = (T)wq[p];
    const T two_f = (T)(2.0 * fnl);
    double fb = 0.0;
    for (int j = tid; j < n; j += 256) {
        const C2 f = b1[rix(j)];
        C2 g = b2[rix(j)];
        g.x *= wpix;
        g.y *= wpix;
        fb += (double)f.x * (double)f.x * (double)g.x;
        if (!eq) fb += (double)f.y * (double)f.y * (double)g.y;
        C2 ph;
        ph.x = two_f * f.x * g.x;
        ph.y = eq ? T(0) : two_f * f.y * g.y;
        b1[rix(j)] = ph;
    }
    // Phi_L^2 ghat has modes up to 3L along the ring; with n = 3L the pixel sum
    // also picks up modes +-3L, 2 Re(G_L^2 G2_L) per ring (times n and the
    // pixel weight), which are removed.
    if (sh.alias && tid == 0) {
        const Q g = *reinterpret_cast<const Q *>(G + poff + (long long)L * Cpad * 2);
        const Q h = *reinterpret_cast<const Q *>(G2 + poff + (long long)L * Cpad * 2);
        const double Nr = (double)g.x + (double)g.y, Ni = (double)g.z + (double)g.w;
        const double Mr = (double)h.x + (double)h.y, Mi = (double)h.z + (double)h.w;
        // Re(N^2 M) = (Nr^2 - Ni^2) Mr - 2 Nr Ni Mi
        double a = (Nr * Nr - Ni * Ni) * Mr - 2.0 * Nr * Ni * Mi;
        if (!eq) {
            const double Sr = (double)g.x - (double)g.y, Si = (double)g.z - (double)g.w;
            const double Rr = (double)h.x - (double)h.y, Ri = (double)h.z - (double)h.w;
            a += (Sr * Sr - Si * Si) * Rr - 2.0 * Sr * Si * Ri;
        }
        fb -= 2.0 * (double)n * (double)wpix * a;
    }
    red[tid] = fb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) fpart[(long long)p * sh.N + s] = red[0];
    fft_lds<C2, false, NMAX, PLANNED>(b1, sh, glb(tw), tid);
    const T half = T(0.5);
    for (int m = tid; m <= L; m += 256) {
        const C2 W1 = b1[rix(m)];
        const C2 W2 = b1[rix(m == 0 ? 0 : n - m)];
        T Ar = half * (W1.x + W2.x), Ai = half * (W1.y - W2.y);
        T Br = half * (W1.y + W2.y), Bi = -half * (W1.x - W2.x);
        if (sh.alias && m == L) {
            const Q g = *reinterpret_cast<const Q *>(G + poff + (long long)L * Cpad * 2);
            const Q h = *reinterpret_cast<const Q *>(G2 + poff + (long long)L * Cpad * 2);
            T Nr = g.x + g.y, Ni = g.z + g.w;
            T Sr = g.x - g.y, Si = g.z - g.w;
            T Mr = h.x + h.y, Mi = h.z + h.w;
            T Rr = h.x - h.y, Ri = h.z - h.w;
            if (eq) Sr = Si = Rr = Ri = T(0);
            const T k = (T)n * two_f * wpix;
            // conj(N) conj(M) = (Nr Mr - Ni Mi, -(Nr Mi + Ni Mr))
            Ar -= k * (Nr * Mr - Ni * Mi);
            Ai -= k * (-(Nr * Mi + Ni * Mr));
            Br -= k * (Sr * Rr - Si * Ri);
            Bi -= k * (-(Sr * Ri + Si * Rr));
        }
        if (eq) Br = Bi = T(0);
        const T cm = m == 0 ? T(1) : T(2);
        T FEr = cm * (Ar + Br), FEi = cm * (Ai + Bi);
        T FOr = cm * (Ar - Br), FOi = cm * (Ai - Bi);
        if (eq) FOr = FOi = T(0);
        if (m == 0) FEi = FOi = T(0);
        Q q;
        q.x = FEr;
        q.y = FOr;
        q.z = FEi;
        q.w = FOi;
        *reinterpret_cast<Q *>(F + (((long long)m * sh.npair + p) * Cpad + 2 * s) * 2) = q;
    }
}

// Transposed filter: nbar_j = sum_i F_l,ij Phibar_L,i for every l, written in
// the noise layout [N][n_lm] complex.  Same tiling as k_filter with the roles
// of the two shell indices exchanged (A[j][i] = F_l[i][j]).
template <typename T>
__global__ __launch_bounds__(256) void k_filter_t(Shape sh, const T *__restrict__ FT, int Kpad,
                                                  int Mpad, const int2 *__restrict__ tiles,
                                                  const T *__restrict__ phibar,
                                                  T *__restrict__ gout)
{
    using M = Mt<T>;
    const int2 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;  // idle slot of the XCD layout (whole block)
    const int l = tl.x, ct = tl.y;
    const int row0 = blockIdx.y * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int ncol = 2 * (l + 1);
    const long long nlm = sh.nlm;
    const T *FTl = FT + (long long)l * Kpad * Mpad;
    typename M::acc acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int c = 0; c < 2; c++) acc[a][c] = typename M::acc{};
    const int rowA = row0 + 32 * wr + i16;
    const int colB = ct * 64 + 32 * wc + i16;
    // lower-triangular F: outputs j >= row0 need rows i >= row0 only
    const int ibeg = sh.lower ? row0 : 0;
    for (int i0 = ibeg; i0 < Kpad; i0 += 4) {
        const int i = i0 + k4;
        T av[2], bv[2];
#pragma unroll
        for (int ri = 0; ri < 2; ri++) {
            const int j = rowA + 16 * ri;
            av[ri] = j < sh.N ? FTl[(long long)j * Mpad + i] : T(0);
        }
#pragma unroll
        for (int ci = 0; ci < 2; ci++) {
            const int col = colB + 16 * ci;
            bv[ci] = (i < sh.N && col < ncol)
                         ? phibar[mrow(sh.L, col >> 1, l) * sh.Cpad + 2 * i + (col & 1)]
                         : T(0);
        }
#pragma unroll
        for (int ri = 0; ri < 2; ri++)
#pragma unroll
            for (int ci = 0; ci < 2; ci++) acc[ri][ci] = M::mfma(av[ri], bv[ci], acc[ri][ci]);
    }
#pragma unroll
    for (int ri = 0; ri < 2; ri++)
#pragma unroll
        for (int ci = 0; ci < 2; ci++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int j = row0 + 32 * wr + 16 * ri + M::row(k4, r);
                const int col = colB + 16 * ci;
                if (j < sh.N && col < ncol) {
                    const int m = col >> 1;
                    const bool zero = m == 0 && (col & 1);
                    gout[((long long)j * nlm + lm_index(l, m)) * 2 + (col & 1)] =
                        zero ? T(0) : (T)acc[ri][ci][r];
                }
            }
}

// dLoss/df_NL = sum over ring blocks (fixed order), minus the ensemble-mean
// term sum_s sqrt(4 pi) <Phi_L^2>(r_s) Re(sum_X W^X_0s abar^X_00).  One block
// of 1024 threads; each thread keeps eight independent partial sums (entry
// q goes to sum (q / 1024) mod 8), added in a fixed tree, so eight loads are
// in flight instead of one dependent chain.
constexpr int kFbarThreads = 1024;
__global__ __launch_bounds__(kFbarThreads) void k_fbar(Shape sh, const double *__restrict__ fpart,
                                                       const double *__restrict__ W,
                                                       const double *__restrict__ mu,
                                                       const double2 *__restrict__ gT,
                                                       const double2 *__restrict__ gE,
                                                       double *__restrict__ out)
{
    constexpr int T = kFbarThreads;
    __shared__ double red[T];
    const int tid = threadIdx.x;
    const long long n = (long long)sh.npair * sh.N;
    double s8[8] = {};
    long long q = tid;
    for (; q + 7 * T < n; q += 8 * T) {
#pragma unroll
        for (int u = 0; u < 8; u++) s8[u] += fpart[q + (long long)u * T];
    }
#pragma unroll
    for (int u = 0; u < 8; u++)
        if (q + (long long)u * T < n) s8[u] += fpart[q + (long long)u * T];
    double acc = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    if (sh.mean_mode == 1) {
        const int Npad = sh.Cpad / 2;
        for (int s = tid; s < sh.N; s += T)
            acc -= mu[s] * (W[s] * gT[0].x + W[(long long)(sh.L + 1) * Npad + s] * gE[0].x);
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *out = red[0];
}

// ------------------------------------------------------------- launchers

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_seed_init(const Shape &sh, const Bufs &b, hipStream_t s)
{
    const long long n = (long long)(sh.L + 1) * sh.npair;
    hipLaunchKernelGGL(k_seed_init, dim3(blocks_for(n, 256)), dim3(256), 0, s, sh, b.x, b.lmm,
                       b.coef, b.seedoff, b.seed, b.lstart, b.lstart_mat,
                       sh.fp32 ? kLambdaTinyF32 : kLambdaTiny);
    const long long nc = (long long)(sh.L + 1) * ((sh.npair + kAnalPC - 1) / kAnalPC);
    hipLaunchKernelGGL(k_chunk_min, dim3(blocks_for(nc, 256)), dim3(256), 0, s, sh, b.lstart_mat,
                       b.cmin);
    return hipGetLastError();
}

template <bool SEEDED>
static void filter_launch(const Shape &sh, const Bufs &b, const void *noise, void *phi_out,
                          hipStream_t s, unsigned long long seed)
{
    dim3 grid(b.nk1);
    if (sh.fp32)
        hipLaunchKernelGGL((k_filter<float, SEEDED>), grid, dim3(256), 0, s, sh,
                           (const float *)b.FQ, b.Kpad, b.Mpad, b.nchq, b.k1tiles,
                           (const float *)noise, (float *)phi_out, seed, b.V, b.aL);
    else
        hipLaunchKernelGGL((k_filter<double, SEEDED>), grid, dim3(256), 0, s, sh,
                           (const double *)b.FQ, b.Kpad, b.Mpad, b.nchq, b.k1tiles,
                           (const double *)noise, (double *)phi_out, seed, b.V, b.aL);
}

hipError_t launch_filter(const Shape &sh, const Bufs &b, const void *noise, void *phi_out,
                         hipStream_t s, unsigned long long seed)
{
    if (noise)
        filter_launch<false>(sh, b, noise, phi_out, s, 0);
    else
        filter_launch<true>(sh, b, nullptr, phi_out, s, seed);
    return hipGetLastError();
}

bool filter_forms_radial(const Shape &sh) { return sh.fp32 != 0; }

hipError_t launch_radial_lin(const Shape &sh, const Bufs &b, const void *noise, hipStream_t s)
{
    dim3 grid(blocks_for(sh.nlm, 256));
    if (sh.fp32)
        hipLaunchKernelGGL(k_radial_lin<float>, grid, dim3(256), 0, s, sh, b.V,
                           (const float *)noise, b.aL);
    else
        hipLaunchKernelGGL(k_radial_lin<double>, grid, dim3(256), 0, s, sh, b.V,
                           (const double *)noise, b.aL);
    return hipGetLastError();
}

hipError_t launch_noise(const Shape &sh, unsigned long long seed, void *out, hipStream_t s)
{
    if ((long long)sh.N * sh.nlm == 0) return hipSuccess;
    dim3 grid((unsigned)std::min<long long>(blocks_for(sh.nlm, 256), 1 << 16),
              (unsigned)std::min(sh.N, 256));
    if (sh.fp32)
        hipLaunchKernelGGL(k_noise<float>, grid, dim3(256), 0, s, sh, seed, (float *)out);
    else
        hipLaunchKernelGGL(k_noise<double>, grid, dim3(256), 0, s, sh, seed, (double *)out);
    return hipGetLastError();
}

template <typename T, int CF>
static void synth_t(const Shape &sh, const Bufs &b, const void *phi, void *G, hipStream_t s)
{
    dim3 grid((unsigned)b.nk2);
    hipLaunchKernelGGL((k_synth<T, CF>), grid, dim3(64), 0, s, sh, b.k2tiles, b.x, b.seed,
                       b.seedoff, b.lstart_mat, b.coef, (const T *)phi, (T *)G);
}

template <typename T>
static void synth_cf(const Shape &sh, const Bufs &b, const void *phi, void *G, hipStream_t s)
{
    switch (sh.CF) {
    case 1: synth_t<T, 1>(sh, b, phi, G, s); break;
    case 2: synth_t<T, 2>(sh, b, phi, G, s); break;
    case 3: synth_t<T, 3>(sh, b, phi, G, s); break;
    case 4: synth_t<T, 4>(sh, b, phi, G, s); break;
    default: synth_t<T, 5>(sh, b, phi, G, s); break;
    }
}

hipError_t launch_synth(const Shape &sh, const Bufs &b, const void *phi_in, void *G_out,
                        hipStream_t s)
{
    if (sh.npiece) return launch_synth_bf(sh, b, phi_in, G_out, s);
    if (sh.fp32)
        synth_cf<float>(sh, b, phi_in, G_out, s);
    else
        synth_cf<double>(sh, b, phi_in, G_out, s);
    return hipGetLastError();
}

// Smallest supported maximum ring length covering n.
static int nmax_for(int n) { return ring_bucket(n); }

template <typename T, int NMAX, bool PLANNED, int S>
static hipError_t ring_ts(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                          double *maps, int mode, hipStream_t s)
{
    using C2 = typename Mt<T>::c2;
    const long long nblk = (long long)sh.npair * ((sh.N + S - 1) / S);
    dim3 grid((unsigned)(((nblk + 7) / 8) * 8));
    const size_t lds = S * sizeof(C2) * ring_pad(sh.nphi);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_ring<T, NMAX, PLANNED, S>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_ring<T, NMAX, PLANNED, S>), grid, dim3(256 * S), lds, s, sh, b.wq,
                       (const C2 *)b.tw, (const T *)G_in, (T *)F_out, maps, mode);
    return hipGetLastError();
}

template <typename T, int NMAX, bool PLANNED>
static hipError_t ring_t(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                         double *maps, int mode, hipStream_t s)
{
    if constexpr (sizeof(T) == 4) {
        if (sh.rs == 1) return ring_ts<T, NMAX, PLANNED, 1>(sh, b, G_in, F_out, maps, mode, s);
        return ring_ts<T, NMAX, PLANNED, 2>(sh, b, G_in, F_out, maps, mode, s);
    } else {
        return ring_ts<T, NMAX, PLANNED, 1>(sh, b, G_in, F_out, maps, mode, s);
    }
}

template <typename T, int NMAX>
static hipError_t ring_p(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                         double *maps, int mode, hipStream_t s)
{
    return fft_has_plan(sh.nphi) ? ring_t<T, NMAX, true>(sh, b, G_in, F_out, maps, mode, s)
                                 : ring_t<T, NMAX, false>(sh, b, G_in, F_out, maps, mode, s);
}

template <typename T>
static hipError_t ring_n(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                         double *maps, int mode, hipStream_t s)
{
    switch (nmax_for(sh.nphi)) {
    case 1024: return ring_p<T, 1024>(sh, b, G_in, F_out, maps, mode, s);
    case 2048: return ring_p<T, 2048>(sh, b, G_in, F_out, maps, mode, s);
    case 4096: return ring_p<T, 4096>(sh, b, G_in, F_out, maps, mode, s);
    default: return ring_p<T, 8192>(sh, b, G_in, F_out, maps, mode, s);
    }
    return hipGetLastError();
}

hipError_t launch_ring(const Shape &sh, const Bufs &b, const void *G_in, void *F_out,
                       double *maps, int mode, hipStream_t s)
{
    return sh.fp32 ? ring_n<float>(sh, b, G_in, F_out, maps, mode, s)
                   : ring_n<double>(sh, b, G_in, F_out, maps, mode, s);
}

template <typename T, int CF>
static void anal_t(const Shape &sh, const Bufs &b, const void *F, void *out, int mode,
                   const double2 *gT, const double2 *gE, hipStream_t s)
{
    dim3 grid(b.nk4);
    if (mode == 0)
        hipLaunchKernelGGL((k_anal<T, CF, 0>), grid, dim3(64), 0, s, sh, b.k4tiles, b.x, b.coef,
                           b.seed, b.seedoff, b.cmin, b.W, b.mu, (const T *)F, b.part,
                           (T *)out, gT, gE);
    else if (mode == 1)
        hipLaunchKernelGGL((k_anal<T, CF, 1>), grid, dim3(64), 0, s, sh, b.k4tiles, b.x, b.coef,
                           b.seed, b.seedoff, b.cmin, b.W, b.mu, (const T *)F, b.part,
                           (T *)out, gT, gE);
    else
        hipLaunchKernelGGL((k_anal<T, CF, 2>), grid, dim3(64), 0, s, sh, b.k4tiles, b.x, b.coef,
                           b.seed, b.seedoff, b.cmin, b.W, b.mu, (const T *)F, b.part,
                           (T *)out, gT, gE);
}

template <typename T>
static void anal_cf(const Shape &sh, const Bufs &b, const void *F, void *out, int mode,
                    const double2 *gT, const double2 *gE, hipStream_t s)
{
    switch (sh.CF) {
    case 1: anal_t<T, 1>(sh, b, F, out, mode, gT, gE, s); break;
    case 2: anal_t<T, 2>(sh, b, F, out, mode, gT, gE, s); break;
    case 3: anal_t<T, 3>(sh, b, F, out, mode, gT, gE, s); break;
    case 4: anal_t<T, 4>(sh, b, F, out, mode, gT, gE, s); break;
    default: anal_t<T, 5>(sh, b, F, out, mode, gT, gE, s); break;
    }
}

hipError_t launch_anal(const Shape &sh, const Bufs &b, const void *F_in, void *out_phi, int mode,
                       hipStream_t s, const double2 *gT, const double2 *gE)
{
    if (sh.npiece) {
        if (mode == 2) return hipErrorInvalidValue;  // the reverse pass rejects split-BF16 contexts
        return launch_anal_bf(sh, b, F_in, out_phi, mode, s);
    }
    if (sh.fp32)
        anal_cf<float>(sh, b, F_in, out_phi, mode, gT, gE, s);
    else
        anal_cf<double>(sh, b, F_in, out_phi, mode, gT, gE, s);
    return hipGetLastError();
}

hipError_t launch_combine(const Shape &sh, const Bufs &b, double fnl, double2 *aT, double2 *aE,
                          double2 *aTn, double2 *aEn, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(sh.nlm, 256)), dim3(256), 0, s, sh, b.part,
                       b.aL, fnl, aT, aE, aTn, aEn);
    return hipGetLastError();
}

hipError_t launch_phi_to_api(const Shape &sh, const void *phi, double2 *api, hipStream_t s)
{
    dim3 grid(blocks_for(sh.nlm * sh.N, 256));
    if (sh.fp32)
        hipLaunchKernelGGL(k_phi_to_api<float>, grid, dim3(256), 0, s, sh, (const float *)phi, api);
    else
        hipLaunchKernelGGL(k_phi_to_api<double>, grid, dim3(256), 0, s, sh, (const double *)phi,
                           api);
    return hipGetLastError();
}

hipError_t launch_api_to_phi(const Shape &sh, const double2 *api, void *phi, hipStream_t s)
{
    dim3 grid(blocks_for(sh.nlm * sh.N, 256));
    if (sh.fp32)
        hipLaunchKernelGGL(k_api_to_phi<float>, grid, dim3(256), 0, s, sh, api, (float *)phi);
    else
        hipLaunchKernelGGL(k_api_to_phi<double>, grid, dim3(256), 0, s, sh, api, (double *)phi);
    return hipGetLastError();
}

hipError_t launch_radial_adj(const Shape &sh, const Bufs &b, const double2 *gT, const double2 *gE,
                             void *out, hipStream_t s)
{
    dim3 grid(blocks_for(sh.nlm, kRadAdjRows));
    if (sh.fp32)
        hipLaunchKernelGGL(k_radial_adj<float>, grid, dim3(256), 0, s, sh, b.W, gT, gE, (float *)out);
    else
        hipLaunchKernelGGL(k_radial_adj<double>, grid, dim3(256), 0, s, sh, b.W, gT, gE,
                           (double *)out);
    return hipGetLastError();
}

template <typename T, int NMAX, bool PLANNED>
static hipError_t ring_adj_t(const Shape &sh, const Bufs &b, const void *G, const void *G2,
                             void *F, double *fpart, double fnl, hipStream_t s)
{
    using C2 = typename Mt<T>::c2;
    const long long nblk = (long long)sh.npair * sh.N;
    dim3 grid((unsigned)(((nblk + 7) / 8) * 8));
    const size_t lds = 2 * sizeof(C2) * ring_pad(sh.nphi);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_ring_adj<T, NMAX, PLANNED>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_ring_adj<T, NMAX, PLANNED>), grid, dim3(256), lds, s, sh, b.wq,
                       (const C2 *)b.tw, (const T *)G, (const T *)G2, (T *)F, fpart, fnl);
    return hipGetLastError();
}

template <typename T, int NMAX>
static hipError_t ring_adj_p(const Shape &sh, const Bufs &b, const void *G, const void *G2,
                             void *F, double *fpart, double fnl, hipStream_t s)
{
    return fft_has_plan(sh.nphi) ? ring_adj_t<T, NMAX, true>(sh, b, G, G2, F, fpart, fnl, s)
                                 : ring_adj_t<T, NMAX, false>(sh, b, G, G2, F, fpart, fnl, s);
}

template <typename T>
static hipError_t ring_adj_n(const Shape &sh, const Bufs &b, const void *G, const void *G2,
                             void *F, double *fpart, double fnl, hipStream_t s)
{
    switch (nmax_for(sh.nphi)) {
    case 1024: return ring_adj_p<T, 1024>(sh, b, G, G2, F, fpart, fnl, s);
    case 2048: return ring_adj_p<T, 2048>(sh, b, G, G2, F, fpart, fnl, s);
    case 4096: return ring_adj_p<T, 4096>(sh, b, G, G2, F, fpart, fnl, s);
    default: return ring_adj_p<T, 8192>(sh, b, G, G2, F, fpart, fnl, s);
    }
}

hipError_t launch_ring_adj(const Shape &sh, const Bufs &b, const void *G, const void *G2, void *F,
                           double *fpart, double fnl, hipStream_t s)
{
    return sh.fp32 ? ring_adj_n<float>(sh, b, G, G2, F, fpart, fnl, s)
                   : ring_adj_n<double>(sh, b, G, G2, F, fpart, fnl, s);
}

hipError_t launch_filter_t(const Shape &sh, const Bufs &b, const void *phibar, void *gout,
                           hipStream_t s)
{
    dim3 grid(b.nk1, b.Mpad / 64);
    if (sh.fp32)
        hipLaunchKernelGGL(k_filter_t<float>, grid, dim3(256), 0, s, sh, (const float *)b.FT,
                           b.Kpad, b.Mpad, b.k1tiles, (const float *)phibar, (float *)gout);
    else
        hipLaunchKernelGGL(k_filter_t<double>, grid, dim3(256), 0, s, sh, (const double *)b.FT,
                           b.Kpad, b.Mpad, b.k1tiles, (const double *)phibar, (double *)gout);
    return hipGetLastError();
}

hipError_t launch_fbar(const Shape &sh, const Bufs &b, const double *fpart, const double2 *gT,
                       const double2 *gE, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fbar, dim3(1), dim3(kFbarThreads), 0, s, sh, fpart, b.W, b.mu, gT, gE, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ grouped launches

long long group_blocks(int stage, const Shape &sh, const Bufs &b)
{
    switch (stage) {
    case GS_RADIAL_LIN:
    case GS_COMBINE: return (sh.nlm + 255) / 256;
    case GS_FILTER: return b.nk1;
    case GS_SYNTH: return b.nk2;
    case GS_RING: {
        const int S = ring_shells(sh.fp32);
        return ((long long)sh.npair * ((sh.N + S - 1) / S) + 7) / 8 * 8;
    }
    case GS_ANAL: return b.nk4;
    default: return 0;
    }
}

template <typename T, int CF>
static void group_cf(int stage, const GroupItem *it, const int *ord, const int *off, int n,
                     dim3 grid, hipStream_t s)
{
    if (stage == GS_SYNTH)
        hipLaunchKernelGGL((g_synth<T, CF>), grid, dim3(64), 0, s, it, ord, off, n);
    else
        hipLaunchKernelGGL((g_anal<T, CF>), grid, dim3(64), 0, s, it, ord, off, n);
}

template <typename T, bool PLANNED>
static void ring_group_launch(int nmax, dim3 grid, dim3 blk, size_t lds, hipStream_t s,
                              const GroupItem *it, const int *ord, const int *off, int n)
{
    if (nmax == 1024)
        hipLaunchKernelGGL((g_ring<T, 1024, PLANNED>), grid, blk, lds, s, it, ord, off, n);
    else if (nmax == 2048)
        hipLaunchKernelGGL((g_ring<T, 2048, PLANNED>), grid, blk, lds, s, it, ord, off, n);
    else if (nmax == 4096)
        hipLaunchKernelGGL((g_ring<T, 4096, PLANNED>), grid, blk, lds, s, it, ord, off, n);
    else
        hipLaunchKernelGGL((g_ring<T, 8192, PLANNED>), grid, blk, lds, s, it, ord, off, n);
}

template <typename T>
static void group_t(int stage, int CF, const GroupItem *it, const int *ord, const int *off, int n,
                    dim3 grid, size_t lds, hipStream_t s)
{
    switch (stage) {
    case GS_RADIAL_LIN:
        hipLaunchKernelGGL(g_radial_lin<T>, grid, dim3(256), 0, s, it, ord, off, n);
        break;
    case GS_FILTER: hipLaunchKernelGGL(g_filter<T>, grid, dim3(256), 0, s, it, ord, off, n); break;
    case GS_RING: {
        // `lds` is the longest ring of the group here; CF != 0 marks a group
        // whose ring lengths all have compile-time plans
        const int nmax = nmax_for((int)lds);
        constexpr int S = ring_s<T>();
        lds = S * sizeof(typename Mt<T>::c2) * ring_pad((int)lds);
        const dim3 blk(256 * S);
        if (CF)
            ring_group_launch<T, true>(nmax, grid, blk, lds, s, it, ord, off, n);
        else
            ring_group_launch<T, false>(nmax, grid, blk, lds, s, it, ord, off, n);
        break;
    }
    case GS_COMBINE: hipLaunchKernelGGL(g_combine, grid, dim3(256), 0, s, it, ord, off, n); break;
    default:
        switch (CF) {
        case 1: group_cf<T, 1>(stage, it, ord, off, n, grid, s); break;
        case 2: group_cf<T, 2>(stage, it, ord, off, n, grid, s); break;
        case 3: group_cf<T, 3>(stage, it, ord, off, n, grid, s); break;
        case 4: group_cf<T, 4>(stage, it, ord, off, n, grid, s); break;
        default: group_cf<T, 5>(stage, it, ord, off, n, grid, s); break;
        }
    }
}

hipError_t launch_group(int stage, int fp32, int CF, const GroupItem *items, const int *ord,
                        const int *off, int n, int nblocks, size_t lds, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    dim3 grid((unsigned)nblocks);
    if (fp32)
        group_t<float>(stage, CF, items, ord, off, n, grid, lds, s);
    else
        group_t<double>(stage, CF, items, ord, off, n, grid, lds, s);
    return hipGetLastError();
}

template <typename T, bool PLANNED>
static hipError_t prep_ring_t(int nphi)
{
    const int nmax = nmax_for(nphi);
    const size_t lds = ring_s<T>() * sizeof(typename Mt<T>::c2) * ring_pad(nphi);
    if (lds <= 65536) return hipSuccess;
    const void *f = nmax == 1024   ? (const void *)g_ring<T, 1024, PLANNED>
                    : nmax == 2048 ? (const void *)g_ring<T, 2048, PLANNED>
                    : nmax == 4096 ? (const void *)g_ring<T, 4096, PLANNED>
                                   : (const void *)g_ring<T, 8192, PLANNED>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t prepare_group_ring(int fp32, int nphi, int planned)
{
    if (fp32) return planned ? prep_ring_t<float, true>(nphi) : prep_ring_t<float, false>(nphi);
    return planned ? prep_ring_t<double, true>(nphi) : prep_ring_t<double, false>(nphi);
}

}  // namespace fnl

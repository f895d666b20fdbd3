// tqu.hip -- T, Q and U maps of the generated harmonics (Sect. 3, the
// temperature and polarisation maps of a realization): on the context's
// Gauss-Legendre grid,
//
//   T     = sum_lm a^T_lm Y_lm,
//   Q + iU = -sum_lm a^E_lm 2Y_lm   (no B modes),
//
// which for a real field is Q = sum_{m>=0} c_m Re[(-a^E_lm) F+_lm e^{i m phi}],
// U = sum_{m>=0} c_m Re[(i a^E_lm) F-_lm e^{i m phi}] with F+- = (2l +- -2l)/2
// the even and odd combinations of the spin +-2 Legendre functions.  Applying
// the spin-raising and -lowering operators twice to Y_lm and eliminating the
// second derivative with Legendre's equation gives both from the scalar
// recurrence's lambda_l and lambda_{l-1} (s = sin theta, x = cos theta,
// D = (l-1) l (l+1) (l+2), kappa = sqrt((2l+1)(l^2-m^2)/(2l-1))):
//
//   F+ = D^-1/2 [((2m^2 - 2l)/s^2 - l(l-1)) lambda_l + 2 x kappa / s^2 lambda_{l-1}],
//   F- = D^-1/2 2m / s^2 [(1-l) x lambda_l + kappa lambda_{l-1}],
//
// and under x -> -x, F+ keeps the parity (-1)^(l+m) of lambda while F-
// takes the opposite one.  Both are formed on the fly next to the FP64
// recurrence, so one pass over l gives all three maps' ring spectra; the
// contraction has only two real columns per map, so it runs as FP64 FMAs on
// the vector ALU (no matrix cores), then FP64 inverse ring FFTs.
#include "device_common.h"

namespace fnl {

namespace {

constexpr int kTquChunk = 64;  // l values of a^T, a^E staged in LDS at a time

// Block = (m, 64 ring pairs), one wave, blocks in ascending m (the longest
// l ranges first).  Lane q runs the recurrence for pair p0 + q from the
// stored state below the first l where any pair of the wave has
// |lambda_lm| > 1e-30, and accumulates the E (l - m even) and O (odd) sums of
// the three maps in FP64.  Output: G[pair][map][m] = (E re, O re, E im, O im).
__global__ __launch_bounds__(64) void k_tqu_synth(Shape sh, const double *__restrict__ x_in,
                                                  const double2 *__restrict__ seed,
                                                  const int *__restrict__ seedoff,
                                                  const int *__restrict__ lstart,
                                                  const double2 *__restrict__ coef,
                                                  const double *__restrict__ tab,
                                                  const double2 *__restrict__ aT,
                                                  const double2 *__restrict__ aE,
                                                  double *__restrict__ G)
{
    __shared__ double2 sT[kTquChunk], sE[kTquChunk];
    const int L = sh.L, npair = sh.npair;
    const int npt = (npair + 63) / 64;
    const int m = blockIdx.x / npt, pt = blockIdx.x % npt;
    const int lane = threadIdx.x;
    const int p = pt * 64 + lane;
    const bool pv = p < npair;
    const double xp = pv ? x_in[p] : 0.0;
    const double is2 = 1.0 / ((1.0 - xp) * (1.0 + xp));  // GL nodes never reach the poles
    const double xis2 = xp * is2;
    int ls = pv ? lstart[(long long)m * npair + p] : L + 1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) ls = min(ls, __shfl_xor(ls, o));
    ls = __builtin_amdgcn_readfirstlane(ls);
    double acc[3][2][2] = {};  // [map][E/O][re/im]
    if (ls <= L) {
        const int u0 = (ls - m) / kSeedStride;
        double l1 = 0.0, l2 = 0.0;  // lambda_{l-1}, lambda_{l-2}
        if (pv) {
            const double2 st = seed[((long long)seedoff[m] + u0) * npair + p];
            l1 = st.x;
            l2 = st.y;
        }
        const long long cr = crow(L, m);
        for (int c0 = m + u0 * kSeedStride; c0 <= L; c0 += kTquChunk) {
            // stage a^T, a^E of l = c0 .. c0 + 63 (wave-uniform values)
            __syncthreads();
            {
                const int l = c0 + lane;
                double2 t = make_double2(0.0, 0.0), e = t;
                if (l <= L) {
                    t = aT[lm_index(l, m)];
                    e = aE[lm_index(l, m)];
                    if (m == 0) t.y = e.y = 0.0;
                }
                sT[lane] = t;
                sE[lane] = e;
            }
            __syncthreads();
            const int cend = min(L, c0 + kTquChunk - 1);
            for (int l = c0; l <= cend; l++) {
                const double2 ab = coef[cr + (l - m)];
                const double lam = ab.x * xp * l1 - ab.y * l2;
                const double *tb = tab + (cr + (l - m)) * 5;
                // (c1, c2, c3, c4, c5) = D^-1/2 (2m^2 - 2l, -l(l-1), 2 kappa, 2m (1-l), 2m kappa)
                const double fp = fma(tb[0], is2, tb[1]) * lam + tb[2] * xis2 * l1;
                const double fm = is2 * (tb[3] * xp * lam + tb[4] * l1);
                const double2 t = sT[l - c0], e = sE[l - c0];
                const int par = (l - m) & 1;
                acc[0][par][0] += lam * t.x;
                acc[0][par][1] += lam * t.y;
                acc[1][par][0] -= fp * e.x;
                acc[1][par][1] -= fp * e.y;
                acc[2][par][0] -= fm * e.y;  // i a^E = (-Im, Re)
                acc[2][par][1] += fm * e.x;
                l2 = l1;
                l1 = lam;
            }
        }
    }
    if (!pv) return;
#pragma unroll
    for (int map = 0; map < 3; map++) {
        double4 v;
        v.x = acc[map][0][0];
        v.y = acc[map][1][0];
        v.z = acc[map][0][1];
        v.w = acc[map][1][1];
        *reinterpret_cast<double4 *>(G + (((long long)p * 3 + map) * (L + 1) + m) * 4) = v;
    }
}

// Block = (ring pair p, map), 256 threads: the north and south rings of the
// pair as one complex sequence z = f_N + i f_S, inverse FFT in LDS, both
// rings written out.  South sums: E - O for T and Q, O - E for U.
template <int NMAX, bool PLANNED>
__global__ __launch_bounds__(256) void k_tqu_ring(Shape sh, const double2 *__restrict__ tw,
                                                  const double *__restrict__ G,
                                                  double *__restrict__ maps)
{
    extern __shared__ unsigned char smem_raw[];
    double2 *buf = reinterpret_cast<double2 *>(smem_raw);
    const int L = sh.L, n = sh.nphi, tid = threadIdx.x;
    const int p = blockIdx.x / 3, map = blockIdx.x % 3;
    if (p >= sh.npair) return;  // whole block
    const bool eq = sh.equator && p == sh.npair - 1;
    for (int q = tid; q < n; q += 256) buf[rix(q)] = make_double2(0.0, 0.0);
    __syncthreads();
    const double *Gp = G + ((long long)p * 3 + map) * (L + 1) * 4;
    for (int m = tid; m <= L; m += 256) {
        const double4 v = *reinterpret_cast<const double4 *>(Gp + (long long)m * 4);
        double Nr = v.x + v.y, Ni = v.z + v.w, Sr = v.x - v.y, Si = v.z - v.w;
        if (map == 2) {
            Sr = -Sr;
            Si = -Si;
        }
        if (eq) Sr = Si = 0.0;
        if (m == 0) Ni = Si = 0.0;
        buf[rix(m)] = make_double2(Nr - Si, Ni + Sr);
        if (m > 0) buf[rix(n - m)] = make_double2(Nr + Si, Sr - Ni);
    }
    __syncthreads();
    fft_lds<double2, true, NMAX, PLANNED>(buf, sh, glb(tw), tid);
    const long long nr = sh.nring;
    double *north = maps + ((long long)map * nr + p) * n;
    double *south = maps + ((long long)map * nr + (nr - 1 - p)) * n;
    for (int j = tid; j < n; j += 256) {
        const double2 z = buf[rix(j)];
        north[j] = z.x;
        if (!eq) south[j] = z.y;
    }
}

template <int NMAX, bool PLANNED>
hipError_t tqu_ring_t(const Shape &sh, const double2 *tw, const double *G, double *maps,
                      hipStream_t s)
{
    const size_t lds = sizeof(double2) * ring_pad(sh.nphi);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_tqu_ring<NMAX, PLANNED>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_tqu_ring<NMAX, PLANNED>), dim3((unsigned)(3 * sh.npair)), dim3(256), lds,
                       s, sh, tw, G, maps);
    return hipGetLastError();
}

template <int NMAX>
hipError_t tqu_ring_p(const Shape &sh, const double2 *tw, const double *G, double *maps,
                      hipStream_t s)
{
    return fft_has_plan(sh.nphi) ? tqu_ring_t<NMAX, true>(sh, tw, G, maps, s)
                                 : tqu_ring_t<NMAX, false>(sh, tw, G, maps, s);
}

}  // namespace

hipError_t launch_tqu(const Shape &sh, const Bufs &b, const double2 *aT, const double2 *aE,
                      double *maps, hipStream_t s)
{
    const int npt = (sh.npair + 63) / 64;
    hipLaunchKernelGGL(k_tqu_synth, dim3((unsigned)((sh.L + 1) * npt)), dim3(64), 0, s, sh, b.x,
                       b.seed, b.seedoff, b.lstart, b.coef, b.tqutab, aT, aE, b.tquG);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (ring_bucket(sh.nphi)) {
    case 1024: return tqu_ring_p<1024>(sh, b.tqutw, b.tquG, maps, s);
    case 2048: return tqu_ring_p<2048>(sh, b.tqutw, b.tquG, maps, s);
    case 4096: return tqu_ring_p<4096>(sh, b.tqutw, b.tquG, maps, s);
    default: return tqu_ring_p<8192>(sh, b.tqutw, b.tquG, maps, s);
    }
}

}  // namespace fnl

// ksw.hip -- the cubic KSW statistic on the generated maps (Sect. 4):
//
//   S_prim = sum_k w_k r_k^2 int d^2n A(r_k, n) B(r_k, n)^2,
//   A(r_k, n) = sum_{i,j} sum_lm (C^-1)^{ij}_l alpha^i_l(r_k) a^j_lm Y_lm(n),
//   B(r_k, n) = sum_{i,j} sum_lm (C^-1)^{ij}_l beta^i_l(r_k)  a^j_lm Y_lm(n).
//
// A cubic-statistic context treats the two filtered maps of every radial node
// as "shells" 2k (A) and 2k+1 (B) of the map generator's layouts, so the
// Legendre synthesis kernel runs them unchanged:
//   k_ksw_filter  data a^T, a^E -> A_lm(r_k), B_lm(r_k) in the m-major Phi layout
//                 (the inverse spectra are folded into the tables at set-up)
//   k_synth       (kernels.hip) -> ring spectra of A and B per ring pair
//   k_ksw_ring    per (ring pair, node): inverse ring FFTs of A and B, the
//                 pixel sum of A B^2 over the two rings (FP64), with the alias
//                 term of n_phi = 3L removed
//   k_ksw_sum     sum over ring pairs, radial weights w_k r_k^2 (fixed order)
#include "device_common.h"

namespace fnl {

namespace {

// One thread per (coefficient idx, node k), k fastest: the thread writes the
// four real columns (A re, A im, B re, B im) of node k in row (m, l).
template <typename T>
__global__ __launch_bounds__(256) void k_ksw_filter(Shape sh, const double *__restrict__ P,
                                                    const double2 *__restrict__ aT,
                                                    const double2 *__restrict__ aE,
                                                    T *__restrict__ phi)
{
    const int Nk = sh.N / 2;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= sh.nlm * Nk) return;
    const int k = (int)(t % Nk);
    const long long idx = t / Nk;
    const int l = l_of_index(idx);
    const int m = (int)(idx - lm_index(l, 0));
    const double2 dT = aT[idx], dE = aE[idx];
    const double4 c = *reinterpret_cast<const double4 *>(P + ((long long)l * Nk + k) * 4);
    // c = (A<-T, A<-E, B<-T, B<-E)
    const double Ar = c.x * dT.x + c.y * dE.x, Ai = c.x * dT.y + c.y * dE.y;
    const double Br = c.z * dT.x + c.w * dE.x, Bi = c.z * dT.y + c.w * dE.y;
    typename Mt<T>::quad v;
    v.x = (T)Ar;
    v.y = m == 0 ? T(0) : (T)Ai;
    v.z = (T)Br;
    v.w = m == 0 ? T(0) : (T)Bi;
    *reinterpret_cast<typename Mt<T>::quad *>(phi + mrow(sh.L, m, l) * sh.Cpad + 4 * k) = v;
}

// Ring spectrum of shell s at ring pair p into an LDS ring as the complex
// sequence z = f_N + i f_S (G rows hold (E, O) interleaved per column).
template <typename T>
__device__ __forceinline__ void ksw_load_ring(const Shape &sh, const T *__restrict__ G, int p, int s,
                                              bool eq, typename Mt<T>::c2 *buf, int tid)
{
    using C2 = typename Mt<T>::c2;
    using Q = typename Mt<T>::quad;
    const int L = sh.L, n = sh.nphi;
    const long long poff = ((long long)p * (L + 1) * sh.Cpad + 2 * s) * 2;
    for (int m = tid; m <= L; m += 256) {
        const Q v = *reinterpret_cast<const Q *>(G + poff + (long long)m * sh.Cpad * 2);
        const T Er = v.x, Or = v.y, Ei = v.z, Oi = v.w;
        T Nr = Er + Or, Ni = Ei + Oi, Sr = Er - Or, Si = Ei - Oi;
        if (eq) Sr = Si = T(0);
        if (m == 0) Ni = Si = T(0);
        C2 z;
        z.x = Nr - Si;
        z.y = Ni + Sr;
        buf[rix(m)] = z;
        if (m > 0) {
            z.x = Nr + Si;
            z.y = Sr - Ni;
            buf[rix(n - m)] = z;
        }
    }
}

// Block = (ring pair p, node k), 256 threads.  Both rings of the pair travel
// as one complex sequence per map, so after the inverse FFTs pixel j of the
// north ring is (Re a, Re b) and of the south ring (Im a, Im b).  One LDS
// ring serves both maps: A is transformed first and each thread keeps its
// pixels of A in registers while the ring is reused for B (two rings per
// block would hold the FP64 kernel to one block per CU).  With n = 3L the
// pixel sum of A B^2 also picks up the modes +-3L of the product,
// 2 n Re(A_L B_L^2) per ring, which are removed.
template <int NMAX, bool PLANNED> constexpr int ksw_pix()
{
    // pixels per thread: the planned lengths of a bucket are 3/4 of it
    // (all of it for 1024), the run-time plans up to all of it
    return PLANNED && NMAX != 1024 ? 3 * NMAX / 4 / 256 : NMAX / 256;
}

template <typename T, int NMAX, bool PLANNED>
__global__ __launch_bounds__(256) void k_ksw_ring(Shape sh, const double *__restrict__ wq,
                                                  const typename Mt<T>::c2 *__restrict__ tw,
                                                  const T *__restrict__ G, double *__restrict__ part)
{
    using C2 = typename Mt<T>::c2;
    using Q = typename Mt<T>::quad;
    extern __shared__ unsigned char smem_raw[];
    const int L = sh.L, n = sh.nphi, Nk = sh.N / 2;
    C2 *b1 = reinterpret_cast<C2 *>(smem_raw);
    __shared__ double red[256];
    const int nblk = sh.npair * Nk;
    const int nslot = (nblk + 7) / 8;
    const int logical = (blockIdx.x & 7) * nslot + (blockIdx.x >> 3);
    if (logical >= nblk) return;  // whole block
    const int k = logical % Nk, p = logical / Nk;
    const int tid = threadIdx.x;
    const bool eq = sh.equator && p == sh.npair - 1;
    constexpr int KJ = ksw_pix<NMAX, PLANNED>();
    // bins (L, n - L) are empty; the loads write every other bin
    for (int q = L + 1 + tid; q < n - L; q += 256) {
        C2 z;
        z.x = T(0);
        z.y = T(0);
        b1[rix(q)] = z;
    }
    ksw_load_ring<T>(sh, G, p, 2 * k, eq, b1, tid);
    __syncthreads();
    fft_lds<C2, true, NMAX, PLANNED>(b1, sh, glb(tw), tid);
    C2 av[KJ];
#pragma unroll
    for (int c = 0; c < KJ; c++) {
        const int j = tid + 256 * c;
        if (j < n) av[c] = b1[rix(j)];
    }
    __syncthreads();  // every A pixel is read before the ring is reused
    for (int q = L + 1 + tid; q < n - L; q += 256) {
        C2 z;
        z.x = T(0);
        z.y = T(0);
        b1[rix(q)] = z;
    }
    ksw_load_ring<T>(sh, G, p, 2 * k + 1, eq, b1, tid);
    __syncthreads();
    fft_lds<C2, true, NMAX, PLANNED>(b1, sh, glb(tw), tid);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < KJ; c++) {
        const int j = tid + 256 * c;
        if (j < n) {
            const C2 a = av[c];
            const C2 b = b1[rix(j)];
            acc += (double)a.x * (double)b.x * (double)b.x;
            if (!eq) acc += (double)a.y * (double)b.y * (double)b.y;
        }
    }
    if (sh.alias && tid == 0) {
        const long long poff = ((long long)p * (L + 1) * sh.Cpad) * 2 + (long long)L * sh.Cpad * 2;
        const Q ga = *reinterpret_cast<const Q *>(G + poff + 2 * (2 * k) * 2);
        const Q gb = *reinterpret_cast<const Q *>(G + poff + 2 * (2 * k + 1) * 2);
        // Re(a b^2) = ar (br^2 - bi^2) - 2 ai br bi
        auto re_ab2 = [](double ar, double ai, double br, double bi) {
            return ar * (br * br - bi * bi) - 2.0 * ai * br * bi;
        };
        double x = re_ab2((double)ga.x + (double)ga.y, (double)ga.z + (double)ga.w,
                          (double)gb.x + (double)gb.y, (double)gb.z + (double)gb.w);
        if (!eq)
            x += re_ab2((double)ga.x - (double)ga.y, (double)ga.z - (double)ga.w,
                        (double)gb.x - (double)gb.y, (double)gb.z - (double)gb.w);
        acc -= 2.0 * (double)n * x;
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[(long long)p * Nk + k] = wq[p] * red[0];
}

// S = sum_k w_k r_k^2 sum_p part[p][k]: thread t sums nodes t, t + 256, ...
// over the ring pairs in order, then a fixed-order tree (one block).
__global__ __launch_bounds__(256) void k_ksw_sum(Shape sh, const double *__restrict__ part,
                                                 const double *__restrict__ wr2,
                                                 double *__restrict__ S)
{
    __shared__ double red[256];
    const int Nk = sh.N / 2, tid = threadIdx.x;
    double acc = 0.0;
    for (int k = tid; k < Nk; k += 256) {
        double s = 0.0;
        for (int p = 0; p < sh.npair; p++) s += part[(long long)p * Nk + k];
        acc += wr2[k] * s;
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *S = red[0];
}

template <typename T, int NMAX, bool PLANNED>
hipError_t ksw_ring_t(const Shape &sh, const Bufs &b, hipStream_t s)
{
    using C2 = typename Mt<T>::c2;
    const long long nblk = (long long)sh.npair * (sh.N / 2);
    dim3 grid((unsigned)(((nblk + 7) / 8) * 8));
    // each thread keeps ksw_pix pixels of A: the ring must fit them
    if (sh.nphi > 256 * ksw_pix<NMAX, PLANNED>()) return hipErrorInvalidValue;
    const size_t lds = sizeof(C2) * ring_pad(sh.nphi);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_ksw_ring<T, NMAX, PLANNED>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_ksw_ring<T, NMAX, PLANNED>), grid, dim3(256), lds, s, sh, b.wq,
                       (const C2 *)b.tw, (const T *)b.G, b.kswpart);
    return hipGetLastError();
}

template <typename T, int NMAX>
hipError_t ksw_ring_p(const Shape &sh, const Bufs &b, hipStream_t s)
{
    return fft_has_plan(sh.nphi) ? ksw_ring_t<T, NMAX, true>(sh, b, s)
                                 : ksw_ring_t<T, NMAX, false>(sh, b, s);
}

template <typename T>
hipError_t ksw_ring_n(const Shape &sh, const Bufs &b, hipStream_t s)
{
    switch (ring_bucket(sh.nphi)) {
    case 1024: return ksw_ring_p<T, 1024>(sh, b, s);
    case 2048: return ksw_ring_p<T, 2048>(sh, b, s);
    case 4096: return ksw_ring_p<T, 4096>(sh, b, s);
    default: return ksw_ring_p<T, 8192>(sh, b, s);
    }
}

}  // namespace

hipError_t launch_ksw_filter(const Shape &sh, const Bufs &b, const double2 *aT, const double2 *aE,
                             hipStream_t s)
{
    const long long n = sh.nlm * (sh.N / 2);
    dim3 grid((unsigned)((n + 255) / 256));
    if (sh.fp32)
        hipLaunchKernelGGL(k_ksw_filter<float>, grid, dim3(256), 0, s, sh, b.kswP, aT, aE,
                           (float *)b.phi);
    else
        hipLaunchKernelGGL(k_ksw_filter<double>, grid, dim3(256), 0, s, sh, b.kswP, aT, aE,
                           (double *)b.phi);
    return hipGetLastError();
}

hipError_t launch_ksw_ring(const Shape &sh, const Bufs &b, hipStream_t s)
{
    return sh.fp32 ? ksw_ring_n<float>(sh, b, s) : ksw_ring_n<double>(sh, b, s);
}

hipError_t launch_ksw_sum(const Shape &sh, const Bufs &b, double *S, hipStream_t s)
{
    hipLaunchKernelGGL(k_ksw_sum, dim3(1), dim3(256), 0, s, sh, b.kswpart, b.kswW, S);
    return hipGetLastError();
}

}  // namespace fnl

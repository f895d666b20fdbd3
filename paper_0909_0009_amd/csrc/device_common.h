// device_common.h -- device helpers shared by the HIP kernel files: the
// matrix-core tile types, global-qualified pointer access, and the in-LDS
// Stockham ring FFT (compile-time radix plans for the 3L ring lengths, a
// run-time radix-2/3/4/5 plan otherwise).
#pragma once

#include <type_traits>

#include "internal.h"

namespace fnl {

// l of the coefficient index idx = l(l+1)/2 + m
__device__ inline int l_of_index(long long idx) {
    int l = (int)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while ((long long)l * (l + 1) / 2 > idx) --l;
    while ((long long)(l + 1) * (l + 2) / 2 <= idx) ++l;
    return l;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core tiles.  Inputs: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Output element r of lane l is D[row(l / 16, r)][l % 16]:
// the FP64 instruction interleaves rows (l/16 + 4r), the FP32 one blocks them
// (4 (l/16) + r) -- measured on gfx950.
template <typename T> struct Mt;
template <> struct Mt<double> {
    using acc = v4d;
    using c2 = double2;
    using c2v = double2;
    using quad = double4;
    __device__ static inline acc mfma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int k4, int r) { return k4 + 4 * r; }
};
template <> struct Mt<float> {
    using acc = v4f;
    using c2 = float2;
    using c2v = float2;
    using quad = float4;
    __device__ static inline acc mfma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int k4, int r) { return 4 * k4 + r; }
};

// Global-memory pointers: indexing through them emits global (not flat)
// memory instructions, and scalar loads where the address is uniform, also
// where the pointer value was read from memory (the grouped launches take
// every context's buffers from an item table).
#define GLB __attribute__((address_space(1)))
template <typename P> __device__ __forceinline__ GLB P *glb(P *p) { return (GLB P *)p; }

// HIP's vector types are classes that cannot be copied out of (or into) a
// global-qualified lvalue; these move them as one builtin vector access.
template <typename V> struct VecOf;
template <> struct VecOf<int2> { typedef int t __attribute__((ext_vector_type(2))); };
template <> struct VecOf<int4> { typedef int t __attribute__((ext_vector_type(4))); };
template <> struct VecOf<float2> { typedef float t __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float4> { typedef float t __attribute__((ext_vector_type(4))); };
template <> struct VecOf<double2> { typedef double t __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double4> { typedef double t __attribute__((ext_vector_type(4))); };
template <typename V> __device__ __forceinline__ V gload(const GLB V *p)
{
    static_assert(sizeof(V) == sizeof(typename VecOf<V>::t), "vector size");
    const typename VecOf<V>::t v = *reinterpret_cast<const GLB typename VecOf<V>::t *>(p);
    V out;
    __builtin_memcpy(&out, &v, sizeof(V));
    return out;
}
template <typename V> __device__ __forceinline__ void gstore(GLB V *p, const V &val)
{
    typename VecOf<V>::t v;
    __builtin_memcpy(&v, &val, sizeof(V));
    *reinterpret_cast<GLB typename VecOf<V>::t *>(p) = v;
}

// ------------------------------------------------------------- ring FFTs

template <typename C2> __device__ inline C2 cmul(C2 a, C2 b)
{
    C2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C2> __device__ inline C2 cadd(C2 a, C2 b)
{
    C2 r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename C2> __device__ inline C2 csub(C2 a, C2 b)
{
    C2 r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
// s * i * a with s = +1 or -1
template <typename C2> __device__ inline C2 cmuli(C2 a, int s)
{
    C2 r;
    r.x = s > 0 ? -a.y : a.y;
    r.y = s > 0 ? a.x : -a.x;
    return r;
}

// cos and sin of 2 pi j / R, evaluated at compile time: quarter-turn
// reduction to |x| <= pi/4, then Taylor series (terms beyond x^27 are below
// double rounding there).
constexpr double ct_sin_red(double x)
{
    double t = x, s = x;
    for (int k = 1; k < 14; k++) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double ct_cos_red(double x)
{
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; k++) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
// angle 2 pi j / R = q pi/2 + x with q = round(4 j / R)
constexpr int ct_quad(int j, int R) { return ((8 * j + R) / (2 * R)) & 3; }
constexpr double ct_rem(int j, int R)
{
    const int q = (8 * j + R) / (2 * R);
    return 6.28318530717958647692 * (double)(4 * j - q * R) / (4.0 * R);
}
constexpr double ct_cos(int j, int R)
{
    const int q = ct_quad(j, R);
    const double x = ct_rem(j, R);
    return q == 0 ? ct_cos_red(x) : q == 1 ? -ct_sin_red(x) : q == 2 ? -ct_cos_red(x) : ct_sin_red(x);
}
constexpr double ct_sin(int j, int R)
{
    const int q = ct_quad(j, R);
    const double x = ct_rem(j, R);
    return q == 0 ? ct_sin_red(x) : q == 1 ? ct_cos_red(x) : q == 2 ? -ct_sin_red(x) : -ct_cos_red(x);
}

// v * e^{sg 2 pi i J / R} (sg = +1 for INV, -1 otherwise) with the trivial
// and eighth-turn factors done without a full complex product.
template <typename C2, int J, int R, bool INV> __device__ __forceinline__ C2 ctwist(C2 v)
{
    using T = decltype(v.x);
    constexpr int sg = INV ? 1 : -1;
    constexpr int j = J % R;
    if constexpr (j == 0) {
        return v;
    } else if constexpr ((4 * j) % R == 0) {
        constexpr int q = (4 * j) / R;  // quarter turns
        if constexpr (q == 2) {
            C2 r;
            r.x = -v.x;
            r.y = -v.y;
            return r;
        } else {
            return cmuli(v, q == 1 ? sg : -sg);
        }
    } else if constexpr ((8 * j) % R == 0) {
        constexpr double c = ct_cos(j, R), sn = sg * ct_sin(j, R);
        constexpr double h = 0.70710678118654752440;
        // (c + i sn) with |c| = |sn| = sqrt(1/2)
        const T a = (T)(c > 0 ? h : -h), b = (T)(sn > 0 ? h : -h);
        C2 r;
        r.x = a * v.x - b * v.y;
        r.y = a * v.y + b * v.x;
        return r;
    } else {
        constexpr double c = ct_cos(j, R), sn = sg * ct_sin(j, R);
        C2 r;
        r.x = (T)c * v.x - (T)sn * v.y;
        r.y = (T)c * v.y + (T)sn * v.x;
        return r;
    }
}

template <typename C2, int R, bool INV> __device__ __forceinline__ void dft_small(C2 *a);

// y[n2][k1] *= w_{R1 R2}^{n2 k1} for every entry, each with its constant factor
template <typename C2, int R1, int R2, bool INV, int I>
__device__ __forceinline__ void twist_all(C2 (&y)[R2][R1])
{
    if constexpr (I < R1 * R2) {
        y[I / R1][I % R1] = ctwist<C2, (I / R1) * (I % R1), R1 * R2, INV>(y[I / R1][I % R1]);
        twist_all<C2, R1, R2, INV, I + 1>(y);
    }
}

// DFT of length R1 R2 from R2 DFTs of length R1, twiddles, and R1 DFTs of
// length R2: input n = R2 n1 + n2, output k = k1 + R1 k2.
template <typename C2, int R1, int R2, bool INV> __device__ __forceinline__ void dft_comp(C2 *a)
{
    C2 y[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; n2++) {
        C2 t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; n1++) t[n1] = a[R2 * n1 + n2];
        dft_small<C2, R1, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; k1++) y[n2][k1] = t[k1];
    }
    twist_all<C2, R1, R2, INV, 0>(y);  // y[n2][k1] *= w_R^{n2 k1}
#pragma unroll
    for (int k1 = 0; k1 < R1; k1++) {
        C2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; n2++) t[n2] = y[n2][k1];
        dft_small<C2, R2, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; k2++) a[k1 + R1 * k2] = t[k2];
    }
}

// Radix-R DFT in place; forward uses e^{-2 pi i t k / R}, INV e^{+...}.
template <typename C2, int R, bool INV> __device__ __forceinline__ void dft_small(C2 *a)
{
    using T = decltype(a[0].x);
    constexpr int sg = INV ? 1 : -1;  // sign of the exponent
    if constexpr (R == 2) {
        const C2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 3) {
        const T h = (T)0.86602540378443864676372317075294;  // sqrt(3)/2
        const C2 t1 = cadd(a[1], a[2]), t2 = csub(a[1], a[2]);
        C2 mm;
        mm.x = a[0].x - (T)0.5 * t1.x;
        mm.y = a[0].y - (T)0.5 * t1.y;
        C2 s2;
        s2.x = h * t2.x;
        s2.y = h * t2.y;
        a[0] = cadd(a[0], t1);
        a[1] = cadd(mm, cmuli(s2, sg));
        a[2] = csub(mm, cmuli(s2, sg));
    } else if constexpr (R == 4) {
        const C2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        const C2 t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, cmuli(t3, sg));
        a[3] = csub(t1, cmuli(t3, sg));
    } else if constexpr (R == 6) {
        dft_comp<C2, 2, 3, INV>(a);
    } else if constexpr (R == 8) {
        dft_comp<C2, 2, 4, INV>(a);
    } else if constexpr (R == 12) {
        dft_comp<C2, 4, 3, INV>(a);
    } else if constexpr (R == 16) {
        dft_comp<C2, 4, 4, INV>(a);
    } else {  // R == 5
        static_assert(R == 5, "unsupported radix");
        const T c1 = (T)0.30901699437494742410229341718282;   // cos(2 pi/5)
        const T c2 = (T)-0.80901699437494742410229341718282;  // cos(4 pi/5)
        const T s1 = (T)0.95105651629515357211643933337938;   // sin(2 pi/5)
        const T s2 = (T)0.58778525229247312916870595463907;   // sin(4 pi/5)
        const C2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
        const C2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
        C2 b1, b2, d1, d2;
        b1.x = a[0].x + c1 * t1.x + c2 * t2.x;
        b1.y = a[0].y + c1 * t1.y + c2 * t2.y;
        b2.x = a[0].x + c2 * t1.x + c1 * t2.x;
        b2.y = a[0].y + c2 * t1.y + c1 * t2.y;
        d1.x = s1 * t3.x + s2 * t4.x;
        d1.y = s1 * t3.y + s2 * t4.y;
        d2.x = s2 * t3.x - s1 * t4.x;
        d2.y = s2 * t3.y - s1 * t4.y;
        a[0] = cadd(a[0], cadd(t1, t2));
        a[1] = cadd(b1, cmuli(d1, sg));
        a[4] = csub(b1, cmuli(d1, sg));
        a[2] = cadd(b2, cmuli(d2, sg));
        a[3] = csub(b2, cmuli(d2, sg));
    }
}

// One Stockham pass of radix R over the n-point array in LDS, 256 threads.
// Butterfly i (k = i mod p) reads x_t = buf[i + t n/R], twists it by
// w^{t k n/(p R)} and writes DFT_R(x)_t to buf[(i - k) R + k + t p].  All reads
// finish before any write, so the pass works in place.
// k = i mod p; p is a power of two in every pass but a trailing radix-3/5
// one, so the mask path is the common one (p is block-uniform).
__device__ inline int mod_p(int i, int p) { return (p & (p - 1)) == 0 ? (i & (p - 1)) : i % p; }

// Ring buffers in LDS hold element j at j + j/32: one pad slot per 32 keeps
// the strided Stockham writes (stride R at p = 1) off shared banks.
__device__ __forceinline__ int rix(int j) { return j + (j >> 5); }

template <typename C2, int R, bool INV, int NMAX>
__device__ __forceinline__ void fft_pass(C2 *buf, int n, int p, const GLB C2 *__restrict__ tw, int tid)
{
    constexpr int MAXB = (NMAX / R + 255) / 256;
    const int nb = n / R;
    const int tstep = n / (p * R);
    // when p divides 256, k = i mod p is the same for every round c of this
    // thread, so its twiddles are loaded once
    const bool shared_k = (256 % p) == 0;
    C2 w0[R];
    if (shared_k) {
        const int k = mod_p(tid, p);
#pragma unroll
        for (int t = 1; t < R; t++) {
            w0[t] = gload(tw + t * k * tstep);
            if (INV) w0[t].y = -w0[t].y;
        }
    }
    C2 y[MAXB][R];
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
        const int i = tid + c * 256;
        if (i < nb) {
            C2 xv[R];
#pragma unroll
            for (int t = 0; t < R; t++) xv[t] = buf[rix(i + t * nb)];
            if (shared_k) {
#pragma unroll
                for (int t = 1; t < R; t++) xv[t] = cmul(xv[t], w0[t]);
            } else {
                const int k = mod_p(i, p);
#pragma unroll
                for (int t = 1; t < R; t++) {
                    C2 w = gload(tw + t * k * tstep);
                    if (INV) w.y = -w.y;
                    xv[t] = cmul(xv[t], w);
                }
            }
            dft_small<C2, R, INV>(xv);
#pragma unroll
            for (int t = 0; t < R; t++) y[c][t] = xv[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
        const int i = tid + c * 256;
        if (i < nb) {
            const int k = mod_p(i, p);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; t++) buf[rix(j + t * p)] = y[c][t];
        }
    }
    __syncthreads();
}

// Compile-time pass of radix R with stride P over an N-point ring: the same
// Stockham step as fft_pass with every index folded to constants.
template <typename C2, int R, bool INV, int N, int P>
__device__ __forceinline__ void fft_pass_c(C2 *buf, const GLB C2 *__restrict__ tw, int tid)
{
    constexpr int NB = N / R;
    constexpr int TSTEP = N / (P * R);
    constexpr int MAXB = (NB + 255) / 256;
    constexpr bool SHARED_K = (256 % P) == 0;
    C2 w0[R];
    if constexpr (SHARED_K && P > 1) {
        const int k = tid % P;
#pragma unroll
        for (int t = 1; t < R; t++) {
            w0[t] = gload(tw + t * k * TSTEP);
            if (INV) w0[t].y = -w0[t].y;
        }
    }
    C2 y[MAXB][R];
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
        const int i = tid + c * 256;
        if (NB % 256 == 0 || i < NB) {
            C2 xv[R];
            if constexpr (NB % 32 == 0) {
                // t NB is a multiple of 32: leg t sits a fixed distance from leg 0
                const C2 *b0 = buf + rix(i);
#pragma unroll
                for (int t = 0; t < R; t++) xv[t] = b0[t * (NB + NB / 32)];
            } else {
#pragma unroll
                for (int t = 0; t < R; t++) xv[t] = buf[rix(i + t * NB)];
            }
            if constexpr (P > 1) {
                if constexpr (SHARED_K) {
#pragma unroll
                    for (int t = 1; t < R; t++) xv[t] = cmul(xv[t], w0[t]);
                } else {
                    const int k = i % P;
#pragma unroll
                    for (int t = 1; t < R; t++) {
                        C2 w = gload(tw + t * k * TSTEP);
                        if (INV) w.y = -w.y;
                        xv[t] = cmul(xv[t], w);
                    }
                }
            }
            dft_small<C2, R, INV>(xv);
#pragma unroll
            for (int t = 0; t < R; t++) y[c][t] = xv[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
        const int i = tid + c * 256;
        if (NB % 256 == 0 || i < NB) {
            const int k = i % P;
            const int j = (i - k) * R + k;
            C2 *b0 = buf + rix(j);
            // padded position of j + t P as rix(j) + a compile-time offset:
            //  P % 32 == 0: t P shifts by whole pad groups;
            //  P == 1, R | 32: j is a multiple of R, j + t stays in j's group;
            //  P == 16, R even: j % 32 = k < 16, so (j + 16 t) / 32 = j / 32 + t / 2
            if constexpr (P % 32 == 0) {
#pragma unroll
                for (int t = 0; t < R; t++) b0[t * (P + P / 32)] = y[c][t];
            } else if constexpr (P == 1 && 32 % R == 0) {
#pragma unroll
                for (int t = 0; t < R; t++) b0[t] = y[c][t];
            } else if constexpr (P == 16 && R % 2 == 0) {
#pragma unroll
                for (int t = 0; t < R; t++) b0[16 * t + (t >> 1)] = y[c][t];
            } else {
#pragma unroll
                for (int t = 0; t < R; t++) buf[rix(j + t * P)] = y[c][t];
            }
        }
    }
    __syncthreads();
}

template <typename C2, bool INV, int N, int P, int R, int... Rest>
__device__ __forceinline__ void fft_static(C2 *buf, const GLB C2 *__restrict__ tw, int tid)
{
    fft_pass_c<C2, R, INV, N, P>(buf, tw, tid);
    if constexpr (sizeof...(Rest) > 0) fft_static<C2, INV, N, P * R, Rest...>(buf, tw, tid);
}

// Ring lengths with a compile-time plan (the 3L grids of lmax 256..2048);
// returns false for other lengths, which take the run-time plan.
// Only lengths in (NMAX/2, NMAX] are planned in an instantiation: shorter
// rings run in the instantiation below it, and a plan longer than NMAX would
// need more registers than the kernel reserves.
template <typename C2, bool INV, int NMAX>
__device__ __forceinline__ bool fft_planned(C2 *buf, int n, const GLB C2 *__restrict__ tw, int tid)
{
    if constexpr (NMAX == 1024) {
        if (n == 768) { fft_static<C2, INV, 768, 1, 16, 12, 4>(buf, tw, tid); return true; }
        if (n == 1024) { fft_static<C2, INV, 1024, 1, 16, 16, 4>(buf, tw, tid); return true; }
    } else if constexpr (NMAX == 2048) {
        if (n == 1536) { fft_static<C2, INV, 1536, 1, 16, 16, 6>(buf, tw, tid); return true; }
    } else if constexpr (NMAX == 4096) {
        if (n == 3072) { fft_static<C2, INV, 3072, 1, 16, 16, 12>(buf, tw, tid); return true; }
    } else if constexpr (NMAX == 8192) {
        if (n == 6144) { fft_static<C2, INV, 6144, 1, 16, 16, 12, 2>(buf, tw, tid); return true; }
    }
    return false;
}

// NMAX: longest ring this instantiation handles (registers are reserved for
// NMAX / 256 elements per thread).
// PLANNED: n has a compile-time plan (fft_has_plan); only that code is
// compiled in, which keeps the register budget of the planned kernels to
// what their passes need.
template <typename C2, bool INV, int NMAX, bool PLANNED>
__device__ __forceinline__ void fft_lds(C2 *buf, const Shape &sh, const GLB C2 *__restrict__ tw, int tid)
{
    if constexpr (PLANNED) {
        (void)fft_planned<C2, INV, NMAX>(buf, sh.nphi, tw, tid);
        return;
    }
    int p = 1;
    for (int ps = 0; ps < sh.npass; ps++) {
        const int R = sh.radix[ps];
        if (R == 4)
            fft_pass<C2, 4, INV, NMAX>(buf, sh.nphi, p, tw, tid);
        else if (R == 2)
            fft_pass<C2, 2, INV, NMAX>(buf, sh.nphi, p, tw, tid);
        else if (R == 3)
            fft_pass<C2, 3, INV, NMAX>(buf, sh.nphi, p, tw, tid);
        else
            fft_pass<C2, 5, INV, NMAX>(buf, sh.nphi, p, tw, tid);
        p *= R;
    }
}

// Epilogue of the Legendre analysis (shared by the FP32/FP64 and the split
// BF16 kernels, whose accumulators have the same 16x16 FP32/FP64 layout):
// acc[f][par][cf] holds rows l = l0w + 2 (16 f + row(k4, r)) + par of column
// colb + 16 cf.  MODE 0: radial partial sums part[ct][X][idx(l, m)] =
// sum_s W^X_ls Phi_NL,lm(s) over the tile's shells, with the mean handling
// at l = 0; MODE 1: per-shell Phi_NL into outphi; MODE 2 (reverse pass):
// per-shell output plus sum_X W^X_ls abar^X_lm.
template <typename T, int CF, int MODE, int NF>
__device__ __forceinline__ void anal_epilogue(const Shape &sh, const typename Mt<T>::acc (&acc)[NF][2][CF],
                                              int m, int l0w, int ct, int colb, int k4, int i16,
                                              const double *__restrict__ W_in,
                                              const double *__restrict__ mu_in,
                                              double2 *__restrict__ part_in,
                                              T *__restrict__ outphi_in,
                                              const double2 *__restrict__ gT_in,
                                              const double2 *__restrict__ gE_in)
{
    using M = Mt<T>;
    auto *__restrict__ W = glb(W_in);
    auto *__restrict__ mu = glb(mu_in);
    auto *__restrict__ part = glb(part_in);
    auto *__restrict__ outphi = glb(outphi_in);
    auto *__restrict__ gT = glb(gT_in);
    auto *__restrict__ gE = glb(gE_in);
    const int L = sh.L, Cpad = sh.Cpad;
    const long long rowm = mrow(L, m, m);
    const int Npad = Cpad / 2;
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int par = 0; par < 2; par++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int l = l0w + 2 * (16 * f + M::row(k4, r)) + par;
                const bool lok = l <= L;
                double sT = 0.0, sE = 0.0;
#pragma unroll
                for (int cf = 0; cf < CF; cf++) {
                    const int col = colb + 16 * cf;
                    const int s = col >> 1;
                    double v = (double)acc[f][par][cf][r];
                    if (MODE == 2) {
                        if (lok) {
                            const long long id = lm_index(l, m);
                            const double2 t = gload(gT + id), e = gload(gE + id);
                            const double wt = W[(long long)l * Npad + s];
                            const double we = W[(long long)(L + 1 + l) * Npad + s];
                            v += (col & 1) ? (m == 0 ? 0.0 : wt * t.y + we * e.y)
                                           : wt * t.x + we * e.x;
                            if (m == 0 && (col & 1)) v = 0.0;
                            outphi[(rowm + (l - m)) * Cpad + col] = (T)v;
                        }
                        continue;
                    }
                    if (m == 0 && l == 0) {
                        if (sh.mean_mode == 0)
                            v = 0.0;
                        else if ((col & 1) == 0)
                            v -= mu[s];
                    }
                    if (MODE == 0) {
                        if (lok) {
                            sT += W[(long long)l * Npad + s] * v;
                            sE += W[(long long)(L + 1 + l) * Npad + s] * v;
                        }
                    } else if (lok) {
                        outphi[(rowm + (l - m)) * Cpad + col] = (T)v;
                    }
                }
                if (MODE == 0) {
                    sT += __shfl_xor(sT, 2);
                    sT += __shfl_xor(sT, 4);
                    sT += __shfl_xor(sT, 8);
                    sE += __shfl_xor(sE, 2);
                    sE += __shfl_xor(sE, 4);
                    sE += __shfl_xor(sE, 8);
                    if (lok && i16 < 2) {
                        const long long id = lm_index(l, m);
                        GLB double *pT =
                            reinterpret_cast<GLB double *>(part + ((long long)ct * 2) * sh.nlm + id);
                        GLB double *pE =
                            reinterpret_cast<GLB double *>(part + ((long long)ct * 2 + 1) * sh.nlm + id);
                        pT[i16] = (m == 0 && i16 == 1) ? 0.0 : sT;
                        pE[i16] = (m == 0 && i16 == 1) ? 0.0 : sE;
                    }
                }
            }
}

}  // namespace fnl

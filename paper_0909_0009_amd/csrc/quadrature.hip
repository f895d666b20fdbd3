// quadrature.hip -- greedy design of the radial quadrature (Sect. 3).
//
// For P problems (a multipole and a transfer table each) on one fine grid of
// ntot shells, the expected error of I_hat = sum_i w_i Phi(r_i) over a node set
// S with its optimal weights (Eq. mean_err and the optimal-weight equations
// C_SS w = (C a)_S) is  a^T C a - b_S^T C_SS^{-1} b_S,  b = C a.  Growing S by
// one shell j lowers it by  (b_j - v_j . z)^2 / (C_jj - |v_j|^2),  where
// C_SS = L L^T, v_j = L^{-1} C_Sj and z = L^{-1} b_S: an incremental Cholesky
// factorisation.  Every step sums that gain over the problems for every
// candidate shell, picks the best shell on the device, and forms one more
// column of L for every (problem, shell) at once; the host only launches.
// L, v and the conditional variances depend on the covariance alone, so
// problems that share one (the T and E problems of a multipole) share them;
// b, z and the residuals are per problem.
//
// On a fine grid spaced well below the correlation length the conditional
// variances C_jj - |v_j|^2 collapse to rounding noise after a few dozen
// nodes.  A shell is then treated as dependent in that problem (d_j at or
// below kQuadDependent C_jj): it gains nothing and, if chosen for the sake of
// other problems, gets a zero pivot there.  The error after each step is
// a^T C a - |z|^2 per problem, summed in a fixed order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "quadrature.h"

namespace fnl {

// Workspace of sim_quadrature_design_noalloc: a fixed device array, so that
// callers that cannot allocate need no hipMalloc.  Each GPU the library runs
// on holds its own copy (at its own address) until the process ends; host
// code reaches it only through the address quad_scratch() looks up.
static __device__ __align__(256) unsigned char scratch[kQuadScratchBytes];

namespace {

__device__ inline int slot_of(const QuadState &q, int p) { return q.pslot ? q.pslot[p] : p; }

// the first problem of a slot writes the slot's per-covariance state
__device__ inline bool slot_owner(const QuadState &q, int p, int s)
{
    return !q.pslot || q.sprob[q.sstart[s]] == p;
}

// b = C a (C symmetric: b_j = sum_k C_kj a_k, so adjacent threads read
// adjacent j of row k), e = b, d = diag(C); one block per (256 shells, problem)
__global__ __launch_bounds__(256) void k_quad_init(QuadState q)
{
    const int p = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q.ntot) return;
    const int sl = slot_of(q, p);
    const long long cp = q.scov ? q.scov[sl] : sl;
    const double *Cp = q.C + cp * q.ntot * q.ntot;
    const double *ap = q.a + (long long)p * q.ntot;
    // four independent partial sums keep four row loads in flight
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int k = 0;
    for (; k + 4 <= q.ntot; k += 4) {
        b0 += Cp[(long long)k * q.ntot + j] * ap[k];
        b1 += Cp[(long long)(k + 1) * q.ntot + j] * ap[k + 1];
        b2 += Cp[(long long)(k + 2) * q.ntot + j] * ap[k + 2];
        b3 += Cp[(long long)(k + 3) * q.ntot + j] * ap[k + 3];
    }
    for (; k < q.ntot; k++) b0 += Cp[(long long)k * q.ntot + j] * ap[k];
    const double cjj = Cp[(long long)j * q.ntot + j];
    q.e[(long long)p * q.ntot + j] = (b0 + b1) + (b2 + b3);
    if (slot_owner(q, p, sl)) {
        q.d[(long long)sl * q.ntot + j] = cjj;
        q.cdiag[(long long)sl * q.ntot + j] = cjj;
    }
    if (p == 0) q.chosen[j] = 0;
}

// a^T C a = a . b per problem (one block per problem, fixed summation order);
// |z|^2 starts at 0
__global__ __launch_bounds__(256) void k_quad_aca(QuadState q)
{
    __shared__ double part[256];
    const int p = blockIdx.x;
    const double *ap = q.a + (long long)p * q.ntot;
    const double *bp = q.e + (long long)p * q.ntot;
    double s = 0.0;
    for (int j = threadIdx.x; j < q.ntot; j += 256) s += ap[j] * bp[j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        q.aCa[p] = part[0];
        q.zz[p] = 0.0;
    }
}

// Partial gains: block (64 shells, problem chunk c), 256 threads; thread
// (shell j, quarter h) sums e_pj^2 / d_pj over the h-th quarter of the
// chunk's problems in order (adjacent threads read adjacent shells of one
// problem row), and the four quarters are added in a fixed tree; a
// dependent shell adds nothing in that problem.  SH: slot tables present.
template <bool SH>
__global__ __launch_bounds__(256) void k_quad_gain(QuadState q)
{
    __shared__ double part[4][64];
    const int jl = threadIdx.x & 63;
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // one per wave
    const int j = blockIdx.x * 64 + jl;
    const int c = blockIdx.y;
    constexpr int QP = kQuadPChunk / 4;
    const int p0 = c * kQuadPChunk + h * QP;
    double g = 0.0;
    if (j < q.ntot) {
        // every problem's loads first (past the last problem they repeat it,
        // in bounds, and add nothing), then the sum in problem order
        double dj[QP], ej[QP], cj[QP];
#pragma unroll
        for (int u = 0; u < QP; u++) {
            const int p = min(p0 + u, q.P - 1);
            const long long sj = (long long)(SH ? q.pslot[p] : p) * q.ntot + j;
            dj[u] = q.d[sj];
            cj[u] = q.cdiag[sj];
            ej[u] = q.e[(long long)p * q.ntot + j];
        }
#pragma unroll
        for (int u = 0; u < QP; u++) {
            const double t = ej[u] * ej[u] / dj[u];
            g += (p0 + u < q.P && dj[u] > kQuadDependent * cj[u]) ? t : 0.0;
        }
    }
    part[h][jl] = g;
    __syncthreads();
    if (h == 0 && j < q.ntot)
        q.gpart[(long long)c * q.ntot + j] = (part[0][jl] + part[1][jl]) + (part[2][jl] + part[3][jl]);
}

// Step k's choice, one block of kQuadChooseThreads threads:
//  1. the node: the largest gain (each shell's chunk partials summed with
//     eight independent partial sums, c mod 8, added in a fixed tree: eight
//     loads in flight instead of one dependent chain) among the shells not
//     yet chosen, the lowest index on ties; recorded and marked chosen;
//  2. its pivot: L_kk = sqrt(d_sel) per slot (0 if dependent), and per
//     problem z_k = e_sel / L_kk, |z|^2 += z_k^2;
//  3. err[k] = sum_p (a^T C a - |z|^2), each thread's problems in order and
//     then a fixed tree over the threads.
constexpr int kQuadChooseThreads = 1024;

__global__ __launch_bounds__(kQuadChooseThreads) void k_quad_choose(QuadState q, int *sel,
                                                                     double *err, int k)
{
    constexpr int T = kQuadChooseThreads;
    __shared__ double gv[T];
    __shared__ int gi[T];
    const int t = threadIdx.x;
    double best = 0.0;
    int bi = -1;
    for (int j = t; j < q.ntot; j += T) {
        if (q.chosen[j]) continue;
        double s8[8] = {};
        int c = 0;
        for (; c + 8 <= q.npc; c += 8) {
#pragma unroll
            for (int u = 0; u < 8; u++) s8[u] += q.gpart[(long long)(c + u) * q.ntot + j];
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (c + u < q.npc) s8[u] += q.gpart[(long long)(c + u) * q.ntot + j];
        const double g = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
        if (bi < 0 || g > best) {  // j ascending: a tie keeps the lower index
            best = g;
            bi = j;
        }
    }
    gv[t] = best;
    gi[t] = bi;
    __syncthreads();
    for (int h = T / 2; h > 0; h >>= 1) {
        if (t < h) {
            const int o = gi[t + h], m = gi[t];
            const double go = gv[t + h], gm = gv[t];
            if (o >= 0 && (m < 0 || go > gm || (go == gm && o < m))) {
                gv[t] = go;
                gi[t] = o;
            }
        }
        __syncthreads();
    }
    const int sn = gi[0];  // n <= ntot: an unchosen shell always exists
    if (t == 0) {
        sel[k] = sn;
        q.chosen[sn] = 1;
    }
    // each problem's z_k, then the pivot of each slot from the same d (the
    // arrays do not overlap, so loads may run ahead of earlier stores)
    const double *__restrict__ dv = q.d;
    const double *__restrict__ cv = q.cdiag;
    const double *__restrict__ ev = q.e;
    const double *__restrict__ av = q.aCa;
    double *__restrict__ zv = q.z;
    double *__restrict__ zzv = q.zz;
    double *__restrict__ lv = q.diag;
    double es = 0.0;
    for (int p = t; p < q.P; p += T) {
        const long long ss = (long long)slot_of(q, p) * q.ntot + sn;
        const double dd = dv[ss];
        const double ee = ev[(long long)p * q.ntot + sn];
        const double l = dd > kQuadDependent * cv[ss] ? sqrt(dd) : 0.0;
        const double zk = l > 0.0 ? ee / l : 0.0;
        zv[(long long)p * q.nmax + k] = zk;
        const double zz = zzv[p] + zk * zk;
        zzv[p] = zz;
        es += av[p] - zz;
    }
    for (int sl = t; sl < q.S; sl += T) {
        const long long ss = (long long)sl * q.ntot + sn;
        const double dd = dv[ss];
        lv[(long long)sl * q.nmax + k] = dd > kQuadDependent * cv[ss] ? sqrt(dd) : 0.0;
    }
    __syncthreads();  // every thread has read gv[0], gi[0]
    gv[t] = es;
    __syncthreads();
    for (int h = T / 2; h > 0; h >>= 1) {
        if (t < h) gv[t] += gv[t + h];
        __syncthreads();
    }
    if (t == 0) err[k] = gv[0];
}

// column k of L for every shell j of a slot (one block per (256 shells,
// slot)): v_j[k] = (C_j,sel - sum_{i<k} v_j[i] v_sel[i]) / l, then
// d_j -= v_j[k]^2, and e_j -= v_j[k] z_k for every problem of the slot
__global__ __launch_bounds__(256) void k_quad_update(QuadState q, const int *sels, int k)
{
    const int sl = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q.ntot) return;
    const int sel = sels[k];
    const long long n2 = (long long)q.ntot;
    const double *Vs = q.V + (long long)sl * q.nmax * n2;
    const double l = q.diag[(long long)sl * q.nmax + k];
    double v = 0.0;
    if (l > 0.0) {
        // four independent partial sums keep four column loads in flight
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int i = 0;
        for (; i + 4 <= k; i += 4) {
            d0 += Vs[i * n2 + j] * Vs[i * n2 + sel];
            d1 += Vs[(i + 1) * n2 + j] * Vs[(i + 1) * n2 + sel];
            d2 += Vs[(i + 2) * n2 + j] * Vs[(i + 2) * n2 + sel];
            d3 += Vs[(i + 3) * n2 + j] * Vs[(i + 3) * n2 + sel];
        }
        for (; i < k; i++) d0 += Vs[i * n2 + j] * Vs[i * n2 + sel];
        const double dot = (d0 + d1) + (d2 + d3);
        const long long cp = q.scov ? q.scov[sl] : sl;
        v = (q.C[cp * n2 * n2 + (long long)sel * n2 + j] - dot) / l;
    }
    q.V[(long long)sl * q.nmax * n2 + (long long)k * n2 + j] = v;
    q.d[(long long)sl * n2 + j] -= v * v;
    if (!q.pslot) {
        q.e[(long long)sl * n2 + j] -= v * q.z[(long long)sl * q.nmax + k];
        return;
    }
    for (int t = q.sstart[sl]; t < q.sstart[sl + 1]; t++) {
        const int p = q.sprob[t];
        q.e[(long long)p * n2 + j] -= v * q.z[(long long)p * q.nmax + k];
    }
}

// optimal weights: L^T w = z by back substitution, L[i][k] = v_{node i}[k]
// (the k-th column at node i, i > k) and L[k][k] = diag[k]; one wave per
// problem, the sum over i spread over the lanes (fixed-order reduction)
__global__ __launch_bounds__(64) void k_quad_weights(QuadState q, const int *nodes, int n, double *w)
{
    __shared__ double ws[kQuadMaxNodes];
    const int p = blockIdx.x, lane = threadIdx.x;
    const int sl = slot_of(q, p);
    const long long n2 = (long long)q.ntot;
    const double *Vp = q.V + (long long)sl * q.nmax * n2;
    for (int k = n - 1; k >= 0; k--) {
        double s = 0.0;
        for (int i = k + 1 + lane; i < n; i += 64) s += Vp[(long long)k * n2 + nodes[i]] * ws[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) {
            const double l = q.diag[(long long)sl * q.nmax + k];
            ws[k] = l > 0.0 ? (q.z[(long long)p * q.nmax + k] - s) / l : 0.0;
        }
        __syncthreads();
    }
    for (int k = lane; k < n; k += 64) w[(long long)p * n + k] = ws[k];
}

unsigned blocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t quad_workspace_bytes(int P, int ntot, int n, int S)
{
    const int ns = S > 0 ? S : P;
    const size_t pn = (size_t)P * ntot, sn = (size_t)ns * ntot;
    const int npc = (P + kQuadPChunk - 1) / kQuadPChunk;
    return align256(8 * pn)                             // e
           + align256(8 * sn) * 2                       // d, cdiag
           + align256(8 * sn * (size_t)n)               // V
           + align256(8 * (size_t)P * n)                // z
           + align256(8 * (size_t)ns * n)               // diag
           + align256(8 * (size_t)P) * 2                // zz, aCa
           + align256(8 * (size_t)npc * ntot)           // gpart
           + align256((size_t)ntot)                     // chosen
           + (S > 0 ? align256(4 * (2 * (size_t)P + 2 * (size_t)S + 1)) : 0);  // slot tables
}

void quad_bind(QuadState &q, int P, int ntot, int n, const double *C, const double *a, void *ws,
               int S)
{
    const int ns = S > 0 ? S : P;
    const size_t pn = (size_t)P * ntot, sn = (size_t)ns * ntot;
    q.P = P;
    q.ntot = ntot;
    q.nmax = n;
    q.npc = (P + kQuadPChunk - 1) / kQuadPChunk;
    q.S = ns;
    q.C = C;
    q.a = a;
    unsigned char *b = static_cast<unsigned char *>(ws);
    auto take = [&](size_t bytes) {
        unsigned char *p = b;
        b += align256(bytes);
        return p;
    };
    q.e = (double *)take(8 * pn);
    q.d = (double *)take(8 * sn);
    q.cdiag = (double *)take(8 * sn);
    q.V = (double *)take(8 * sn * (size_t)n);
    q.z = (double *)take(8 * (size_t)P * n);
    q.diag = (double *)take(8 * (size_t)ns * n);
    q.zz = (double *)take(8 * (size_t)P);
    q.aCa = (double *)take(8 * (size_t)P);
    q.gpart = (double *)take(8 * (size_t)q.npc * ntot);
    q.chosen = take((size_t)ntot);
    if (S > 0) {
        int *t = (int *)take(4 * (2 * (size_t)P + 2 * (size_t)S + 1));
        q.pslot = t;
        q.scov = t + P;
        q.sstart = t + P + S;
        q.sprob = t + P + 2 * S + 1;
    } else {
        q.pslot = q.scov = q.sstart = q.sprob = nullptr;
    }
}

hipError_t quad_scratch(void **ptr)
{
    // one symbol lookup per device, made with that device current (the first
    // call on it); the address is kept for later calls
    static std::mutex mu;
    static void *addr[kQuadMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kQuadMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t quad_run(QuadState &q, int n, int *nodes, double *err, double *w, hipStream_t s)
{
    if (n < 1 || n > kQuadMaxNodes || n > q.nmax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_quad_init, dim3(blocks(q.ntot, 256), q.P), dim3(256), 0, s, q);
    hipLaunchKernelGGL(k_quad_aca, dim3(q.P), dim3(256), 0, s, q);
    // every step runs on the device: partial gains, the choice (largest gain
    // among the shells not yet chosen, lowest index on ties), the pivot and
    // the error, the Cholesky column
    for (int k = 0; k < n; k++) {
        if (q.pslot)
            hipLaunchKernelGGL(k_quad_gain<true>, dim3(blocks(q.ntot, 64), q.npc), dim3(256), 0, s, q);
        else
            hipLaunchKernelGGL(k_quad_gain<false>, dim3(blocks(q.ntot, 64), q.npc), dim3(256), 0, s, q);
        hipLaunchKernelGGL(k_quad_choose, dim3(1), dim3(kQuadChooseThreads), 0, s, q, nodes, err, k);
        hipLaunchKernelGGL(k_quad_update, dim3(blocks(q.ntot, 256), q.S), dim3(256), 0, s, q, nodes, k);
    }
    hipLaunchKernelGGL(k_quad_weights, dim3(q.P), dim3(64), 0, s, q, nodes, n, w);
    return hipGetLastError();
}

}  // namespace fnl

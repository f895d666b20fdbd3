// quadrature.hip -- greedy design of the radial quadrature (Sect. 3).
//
// For P problems (a multipole and a transfer table each) on one fine grid of
// ntot shells, the expected error of I_hat = sum_i w_i Phi(r_i) over a node set
// S with its optimal weights (Eq. mean_err and the optimal-weight equations
// C_SS w = (C a)_S) is  a^T C a - b_S^T C_SS^{-1} b_S,  b = C a.  Growing S by
// one shell j lowers it by  (b_j - v_j . z)^2 / (C_jj - |v_j|^2),  where
// C_SS = L L^T, v_j = L^{-1} C_Sj and z = L^{-1} b_S: an incremental Cholesky
// factorisation.  Every step sums that gain over the problems for every
// candidate shell (one block per shell), picks the best shell on the device,
// and forms one more column of L for every (problem, shell) at once; the
// host only launches.
#include <hip/hip_runtime.h>

#include "quadrature.h"

namespace fnl {

namespace {

// b = C a (C symmetric: b_j = sum_k C_kj a_k, so adjacent threads read
// adjacent j of row k), e = b, d = diag(C); one block per (256 shells, problem)
__global__ __launch_bounds__(256) void k_quad_init(QuadState q)
{
    const int p = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q.ntot) return;
    const double *Cp = q.C + (long long)p * q.ntot * q.ntot;
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
    q.e[(long long)p * q.ntot + j] = (b0 + b1) + (b2 + b3);
    q.d[(long long)p * q.ntot + j] = Cp[(long long)j * q.ntot + j];
}

// a^T C a = a . b per problem (one block per problem, fixed summation order)
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
    if (threadIdx.x == 0) q.aCa[p] = part[0];
}

// gain_j = sum_p e_pj^2 / d_pj over the problems (chosen shells: 0; a shell
// whose conditional variance has vanished in a problem adds nothing there).
// One block per shell, threads over the problems, a fixed-order tree sum.
__global__ __launch_bounds__(256) void k_quad_gain(QuadState q, const unsigned char *chosen)
{
    __shared__ double part[256];
    const int j = blockIdx.x;
    double g = 0.0;
    if (!chosen[j]) {
        for (int p = threadIdx.x; p < q.P; p += 256) {
            const double dj = q.d[(long long)p * q.ntot + j];
            const double ej = q.e[(long long)p * q.ntot + j];
            if (dj > 0.0) g += ej * ej / dj;
        }
    }
    part[threadIdx.x] = g;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) q.gain[j] = part[0];
}

// E = sum_p a^T C a (one block, fixed order)
__global__ __launch_bounds__(256) void k_quad_total(QuadState q, double *E)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int p = threadIdx.x; p < q.P; p += 256) s += q.aCa[p];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *E = part[0];
}

// step k's node: the largest gain among the shells not yet chosen, the lowest
// index on ties (one block); records it, marks it chosen and lowers the
// running error E by its gain
__global__ __launch_bounds__(256) void k_quad_select(QuadState q, unsigned char *chosen, int *sel,
                                                     double *err, double *E, int k)
{
    __shared__ double gv[256];
    __shared__ int gi[256];
    double best = 0.0;
    int bi = -1;
    for (int j = threadIdx.x; j < q.ntot; j += 256) {
        if (chosen[j]) continue;
        const double g = q.gain[j];
        if (bi < 0 || g > best) {  // j ascending: a tie keeps the lower index
            best = g;
            bi = j;
        }
    }
    gv[threadIdx.x] = best;
    gi[threadIdx.x] = bi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = gi[threadIdx.x + h], m = gi[threadIdx.x];
            const double go = gv[threadIdx.x + h], gm = gv[threadIdx.x];
            if (o >= 0 && (m < 0 || go > gm || (go == gm && o < m))) {
                gv[threadIdx.x] = go;
                gi[threadIdx.x] = o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int s = gi[0];  // n <= ntot: an unchosen shell always exists
        sel[k] = s;
        chosen[s] = 1;
        *E -= gv[0];
        err[k] = *E;
    }
}

// the chosen shell's (d, e) per problem, read before the step overwrites them
__global__ __launch_bounds__(256) void k_quad_pivot(QuadState q, const int *sels, int k)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= q.P) return;
    const int sel = sels[k];
    const double dd = q.d[(long long)p * q.ntot + sel];
    const double ee = q.e[(long long)p * q.ntot + sel];
    q.piv[2 * p] = dd;
    q.piv[2 * p + 1] = ee;
    const double l = dd > 0.0 ? sqrt(dd) : 0.0;
    q.diag[(long long)p * q.nmax + k] = l;
    q.z[(long long)p * q.nmax + k] = l > 0.0 ? ee / l : 0.0;
}

// column k of L for every shell j: v_j[k] = (C_j,sel - sum_{i<k} v_j[i] v_sel[i]) / l,
// then d_j -= v_j[k]^2 and e_j -= v_j[k] z_k
__global__ __launch_bounds__(256) void k_quad_update(QuadState q, const int *sels, int k)
{
    const int p = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q.ntot) return;
    const int sel = sels[k];
    const long long n2 = (long long)q.ntot;
    const double *Vp = q.V + (long long)p * q.nmax * n2;
    const double l = q.diag[(long long)p * q.nmax + k];
    double v = 0.0;
    if (l > 0.0) {
        // four independent partial sums keep four column loads in flight
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int i = 0;
        for (; i + 4 <= k; i += 4) {
            d0 += Vp[i * n2 + j] * Vp[i * n2 + sel];
            d1 += Vp[(i + 1) * n2 + j] * Vp[(i + 1) * n2 + sel];
            d2 += Vp[(i + 2) * n2 + j] * Vp[(i + 2) * n2 + sel];
            d3 += Vp[(i + 3) * n2 + j] * Vp[(i + 3) * n2 + sel];
        }
        for (; i < k; i++) d0 += Vp[i * n2 + j] * Vp[i * n2 + sel];
        const double dot = (d0 + d1) + (d2 + d3);
        v = (q.C[(long long)p * n2 * n2 + (long long)sel * n2 + j] - dot) / l;
    }
    q.V[(long long)p * q.nmax * n2 + (long long)k * n2 + j] = v;
    const long long ij = (long long)p * n2 + j;
    q.d[ij] -= v * v;
    q.e[ij] -= v * q.z[(long long)p * q.nmax + k];
}

// optimal weights: L^T w = z by back substitution, L[i][k] = v_{node i}[k]
// (the k-th column at node i, i > k) and L[k][k] = diag[k]; one wave per
// problem, the sum over i spread over the lanes (fixed-order reduction)
constexpr int kQuadMaxNodes = 1024;
__global__ __launch_bounds__(64) void k_quad_weights(QuadState q, const int *nodes, int n, double *w)
{
    __shared__ double ws[kQuadMaxNodes];
    const int p = blockIdx.x, lane = threadIdx.x;
    const long long n2 = (long long)q.ntot;
    const double *Vp = q.V + (long long)p * q.nmax * n2;
    for (int k = n - 1; k >= 0; k--) {
        double s = 0.0;
        for (int i = k + 1 + lane; i < n; i += 64) s += Vp[(long long)k * n2 + nodes[i]] * ws[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) {
            const double l = q.diag[(long long)p * q.nmax + k];
            ws[k] = l > 0.0 ? (q.z[(long long)p * q.nmax + k] - s) / l : 0.0;
        }
        __syncthreads();
    }
    for (int k = lane; k < n; k += 64) w[(long long)p * n + k] = ws[k];
}

unsigned blocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t quad_init(const QuadState &q, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_init, dim3(blocks(q.ntot, 256), q.P), dim3(256), 0, s, q);
    hipLaunchKernelGGL(k_quad_aca, dim3(q.P), dim3(256), 0, s, q);
    return hipGetLastError();
}

hipError_t quad_gain(const QuadState &q, const unsigned char *chosen, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_gain, dim3(q.ntot), dim3(256), 0, s, q, chosen);
    return hipGetLastError();
}

hipError_t quad_total(const QuadState &q, double *E, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_total, dim3(1), dim3(256), 0, s, q, E);
    return hipGetLastError();
}

hipError_t quad_select(const QuadState &q, unsigned char *chosen, int *sels, double *err, double *E,
                       int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_select, dim3(1), dim3(256), 0, s, q, chosen, sels, err, E, k);
    return hipGetLastError();
}

hipError_t quad_step(const QuadState &q, const int *sels, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_pivot, dim3(blocks(q.P, 256)), dim3(256), 0, s, q, sels, k);
    hipLaunchKernelGGL(k_quad_update, dim3(blocks(q.ntot, 256), q.P), dim3(256), 0, s, q, sels, k);
    return hipGetLastError();
}

hipError_t quad_weights(const QuadState &q, const int *nodes_dev, int n, double *w, hipStream_t s)
{
    if (n > kQuadMaxNodes) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_quad_weights, dim3(q.P), dim3(64), 0, s, q, nodes_dev, n, w);
    return hipGetLastError();
}

}  // namespace fnl

// quadrature.h -- launchers of the greedy radial-quadrature design kernels
// (quadrature.hip), called by sim_quadrature_design and
// sim_quadrature_design_noalloc in fnlsim.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fnl {

// A shell whose conditional variance d_j has fallen to kQuadDependent C_jj or
// below is dependent on the nodes already chosen in that problem: it adds no
// gain there, and if chosen it gets a zero Cholesky pivot (weight 0).
constexpr double kQuadDependent = 1e-10;
// Problems per partial gain sum (the gain of a shell is summed over problems
// in chunks of this many, then the chunks in a fixed order).
constexpr int kQuadPChunk = 32;
constexpr int kQuadMaxNodes = 1024;
// Size of the fixed device workspace behind sim_quadrature_design_noalloc
// (64 MiB per GPU), and the number of devices it keeps an address for.
constexpr size_t kQuadScratchBytes = size_t(64) << 20;
constexpr int kQuadMaxDevices = 64;

// Problem sizes and device state of one design run.  Arrays (device, FP64):
//   C [ncov][ntot][ntot]  covariances of Phi on the fine grid; problem p uses
//                      C[cidx[p]] (cidx == nullptr: C[p], ncov = P)
//   a [P][ntot]        fine-sum weights
//   e [P][ntot]        residual numerator b_j - v_j . z   (b = C a)
//   d [P][ntot]        conditional variance C_jj - |v_j|^2
//   cdiag [P][ntot]    C_jj (the scale of the dependence test)
//   V [P][nmax][ntot]  column k: the k-th Cholesky column of the chosen set,
//                      v_j[k] for every shell j
//   z [P][nmax], diag [P][nmax]   Cholesky right-hand side and diagonal
//   zz [P]             |z|^2 so far: the error of problem p is a^T C a - zz
//   gpart [npc][ntot]  partial gains, sum over one chunk of problems of e^2 / d
//   aCa [P]            a^T C a per problem
//   chosen [ntot]      1 once a shell is a node (bytes)
struct QuadState {
    int P, ntot, nmax, npc;
    const double *C, *a;
    const int *cidx;
    double *e, *d, *cdiag, *V, *z, *diag, *zz, *gpart, *aCa;
    unsigned char *chosen;
};

// Bytes of device workspace a design of these sizes needs, and the binding
// of a QuadState's arrays to such a workspace (256-byte aligned base).
// With cidx, the binding also reserves the device copy of the index table
// (q.cidx, P ints at the end of the workspace), which the caller fills.
size_t quad_workspace_bytes(int P, int ntot, int n, bool shared = false);
void quad_bind(QuadState &q, int P, int ntot, int n, const double *C, const double *a, void *ws,
               bool shared = false);

// Device address of the fixed workspace on the current device (looked up
// once per device).
hipError_t quad_scratch(void **ptr);

// The whole design on stream s, asynchronous: clears the workspace state it
// needs, then n greedy steps, then the weights.  nodes [n] (int), err [n] and
// w [P][n] are device arrays.
hipError_t quad_run(QuadState &q, int n, int *nodes, double *err, double *w, hipStream_t s);

}  // namespace fnl

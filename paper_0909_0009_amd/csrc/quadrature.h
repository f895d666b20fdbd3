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

// Problem sizes and device state of one design run.  The Cholesky factor of
// the chosen set depends on the covariance alone, not on a: problems that
// share a covariance (a slot) share V, d, cdiag and diag, and only e, z, zz
// and aCa are per problem.  Arrays (device, FP64 unless noted):
//   C [ncov][ntot][ntot]  covariances of Phi on the fine grid
//   a [P][ntot]        fine-sum weights
//   e [P][ntot]        residual numerator b_j - v_j . z   (b = C a)
//   d [S][ntot]        conditional variance C_jj - |v_j|^2 per slot
//   cdiag [S][ntot]    C_jj (the scale of the dependence test)
//   V [S][nmax][ntot]  column k: the k-th Cholesky column of the chosen set,
//                      v_j[k] for every shell j
//   diag [S][nmax]     Cholesky diagonal per slot
//   z [P][nmax]        Cholesky right-hand side per problem
//   zz [P]             |z|^2 so far: the error of problem p is a^T C a - zz
//   gpart [npc][ntot]  partial gains, sum over one chunk of problems of e^2 / d
//   aCa [P]            a^T C a per problem
//   chosen [ntot]      1 once a shell is a node (bytes)
// Slot tables (int, nullptr without shared covariances: then S = P, problem
// p is slot p and reads C[p]):
//   pslot [P]          the slot of problem p
//   scov [S]           the covariance index of slot s
//   sstart [S + 1], sprob [P]   the problems of slot s, ascending:
//                      sprob[sstart[s] .. sstart[s + 1])
struct QuadState {
    int P, ntot, nmax, npc, S;
    const double *C, *a;
    const int *pslot, *scov, *sstart, *sprob;
    double *e, *d, *cdiag, *V, *z, *diag, *zz, *gpart, *aCa;
    unsigned char *chosen;
};

// Bytes of device workspace a design of these sizes needs, and the binding
// of a QuadState's arrays to such a workspace (256-byte aligned base).
// S > 0 gives S slots and reserves the slot tables (2 P + 2 S + 1 ints at the
// end of the workspace, in the order pslot, scov, sstart, sprob), which the
// caller fills; S = 0 is one slot per problem and no tables.
size_t quad_workspace_bytes(int P, int ntot, int n, int S = 0);
void quad_bind(QuadState &q, int P, int ntot, int n, const double *C, const double *a, void *ws,
               int S = 0);

// Device address of the fixed workspace on the current device (looked up
// once per device).
hipError_t quad_scratch(void **ptr);

// The whole design on stream s, asynchronous: clears the workspace state it
// needs, then n greedy steps, then the weights.  nodes [n] (int), err [n] and
// w [P][n] are device arrays.
hipError_t quad_run(QuadState &q, int n, int *nodes, double *err, double *w, hipStream_t s);

}  // namespace fnl

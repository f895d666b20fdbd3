// quadrature.h -- launchers of the greedy radial-quadrature design kernels
// (quadrature.hip), called by sim_quadrature_design in fnlsim.cpp.
#pragma once

#include <hip/hip_runtime.h>

namespace fnl {

// Problem sizes and device state of one design run.  Arrays (device, FP64):
//   C [P][ntot][ntot]  covariance of Phi on the fine grid, per problem
//   a [P][ntot]        fine-sum weights
//   e [P][ntot]        residual numerator b_j - v_j . z   (b = C a)
//   d [P][ntot]        conditional variance C_jj - |v_j|^2
//   V [P][nmax][ntot]  column k: the k-th Cholesky column of the chosen set,
//                      v_j[k] for every shell j
//   piv [P][2]         (d, e) of the node chosen at the current step
//   z [P][nmax], diag [P][nmax]   Cholesky right-hand side and diagonal
//   gain [ntot]        sum_p e_pj^2 / d_pj
//   aCa [P]            a^T C a per problem
struct QuadState {
    int P, ntot, nmax;
    const double *C, *a;
    double *e, *d, *V, *piv, *z, *diag, *gain, *aCa;
};

hipError_t quad_init(const QuadState &q, hipStream_t s);
// *E = sum_p a^T C a
hipError_t quad_total(const QuadState &q, double *E, hipStream_t s);
hipError_t quad_gain(const QuadState &q, const unsigned char *chosen, hipStream_t s);
// step k: sels[k] = best unchosen shell (lowest index on ties), chosen[sels[k]] = 1,
// *E -= its gain, err[k] = *E (all device memory)
hipError_t quad_select(const QuadState &q, unsigned char *chosen, int *sels, double *err, double *E,
                       int k, hipStream_t s);
hipError_t quad_step(const QuadState &q, const int *sels, int k, hipStream_t s);
hipError_t quad_weights(const QuadState &q, const int *nodes_dev, int n, double *w, hipStream_t s);

}  // namespace fnl

// Kernels of the Car-Parrinello comparison step (cp.hip): the orbital
// updates of RATTLE / velocity Verlet and the solution of the position
// constraint.  Orbitals are [n_orb][stride] complex, N points each; the
// N_W x N_W matrices are column-major (element (i, j) at i + j * n).
#pragma once
#include "common.hpp"

namespace me {

// trial[i] = psi[i] + dt psidot[i] - c trial[i]   (trial holds H psi on entry)
template <typename T>
hipError_t launch_cp_predict(cx_t<T>* trial, const cx_t<T>* psi, const cx_t<T>* psidot, int64_t stride, int n_orb,
                             int64_t N, double dt, double c, hipStream_t s);
// psidot[i] = (psi_new[i] - psi_old[i]) * inv_dt
template <typename T>
hipError_t launch_cp_halfvel(cx_t<T>* psidot, const cx_t<T>* psi_new, const cx_t<T>* psi_old, int64_t stride,
                             int n_orb, int64_t N, double inv_dt, hipStream_t s);
// psidot[i] -= c hpsi[i]
template <typename T>
hipError_t launch_cp_kick(cx_t<T>* psidot, const cx_t<T>* hpsi, int64_t stride, int n_orb, int64_t N, double c,
                          hipStream_t s);
// out[e] = scale * sum_{b < nb} part[b][e] over e < n*n, in FP64 and in the
// order of b (the K-split partial overlap matrices of the GEMMs)
template <typename T>
hipError_t launch_cp_reduce(const cx_t<T>* part, int nb, int n, double scale, double2* out, hipStream_t s);
// Hermitian X with A + B^H X + X B + X^2 = I by X <- X - R/2, R the residual
// of that equation, from X = (I - A)/2; at most max_iter corrections, stopped
// once max|R| < tol.  A, B, X64, R64: n*n FP64; part: cp_solve_blocks(n)
// doubles.  X receives the solution in the orbital precision, info[0] the
// corrections made and info[1] the final max|R|.
template <typename T>
hipError_t launch_cp_solve_x(const double2* A, const double2* B, int n, double tol, int max_iter, double2* X64,
                             double2* R64, double* part, cx_t<T>* X, double* info, hipStream_t s);
int cp_solve_blocks(int n);
// Y = -(Q + Q^H) / 2 (Q in FP64, Y in the orbital precision)
template <typename T>
hipError_t launch_cp_velocity_matrix(const double2* Q, int n, cx_t<T>* Y, hipStream_t s);
// part[b] = sum over orbitals and the 256 points of block b of |psidot|^2 (FP64)
template <typename T>
hipError_t launch_cp_sq_partial(const cx_t<T>* psidot, int64_t stride, int n_orb, int64_t N, double* part,
                                hipStream_t s);
int64_t cp_sq_blocks(int64_t N);

}  // namespace me

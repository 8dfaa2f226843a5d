// Declarations of the adjoint and control kernels (adjoint.hip).
#pragma once
#include "common.hpp"

namespace me {

template <typename T>
hipError_t launch_cross_accum(const cx_t<T>* ub, const cx_t<T>* u, cx_t<T>* acc, int64_t stride, int n_orb,
                              int64_t N, double alpha, bool init, double* wbar, hipStream_t s);
template <typename T>
hipError_t launch_accum(const cx_t<T>* ub, cx_t<T>* acc, int64_t stride, int n_orb, int64_t N, hipStream_t s);
template <typename T>
hipError_t launch_lambda_update(cx_t<T>* lam, const cx_t<T>* psi, const double* rhobar, int64_t stride,
                                int n_orb, int64_t N, double occ, hipStream_t s);
hipError_t launch_vhxc_adjoint(const double* hv, const double* vbar, const double* rho, const double* extra,
                               int64_t N, double* rhobar, hipStream_t s);
hipError_t launch_axpy(double* dst, const double* src, double a, int64_t N, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
// out[0] = scale * sum_i (h*ix - L/2) f[i]  (part: scratch of ceil(N/256) doubles)
hipError_t launch_field_dot(const double* f, int nx, int64_t N, double h, double Lx, double* part,
                            double* out, double scale, hipStream_t s);
hipError_t launch_dipole_rhobar(double* rb, int nx, int64_t N, double h, double Lx, hipStream_t s);
hipError_t launch_coarse_to_fine(const double* c, int m, int n, double* f, hipStream_t s);
hipError_t launch_fine_to_coarse(const double* f, int m, int n, double* c, hipStream_t s);

}  // namespace me

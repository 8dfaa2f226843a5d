// Kernels of the finite box (finite.hip): the union of atom-centred spheres
// of the paper's molecular runs (sec. 5), with a zero boundary condition and
// the potentials of an isolated system.  Grid arrays are [nz][ny][nx], x
// fastest; the doubled grid of the free-space Poisson solver is
// [2nz][2ny][2nx].
#pragma once
#include "common.hpp"

namespace me {

// mask[i] = 1 if point i lies within `radius` of an ion at pos0, else 0
hipError_t launch_box_mask(const double* pos0, int n_ions, int nx, int ny, int nz, double h, double radius,
                           uint8_t* mask, hipStream_t s);
// psi[o][i] = 0 where mask[i] == 0 (o < n_orb)
template <typename T>
hipError_t launch_mask_orbitals(cx_t<T>* psi, int64_t stride, int n_orb, int64_t N, const uint8_t* mask,
                                hipStream_t s);
// out[i] = -sum_J Z_J erf(d/a)/d, d = |r_i - R_J| (no periodic images)
hipError_t launch_vloc_free(const double* pos, const double* zval, int n_ions, int nx, int ny, int nz, double h,
                            double a, double* out, hipStream_t s);
// Coulomb kernel 1/|r| on the doubled grid with minimum-image offsets and
// the cell average c0 / h at r = 0
hipError_t launch_green_doubled(int nx, int ny, int nz, double h, double* g2, hipStream_t s);
// gk[k] = scale * Re spec[k]  (the spectrum of the even kernel is real)
hipError_t launch_green_spectrum(const double2* spec, int64_t n, double scale, double* gk, hipStream_t s);
// rpad = rho on the corner n-block of the doubled grid, 0 on the rest
hipError_t launch_pad(const double* rho, int nx, int ny, int nz, double* rpad, hipStream_t s);
// spec[k] *= gk[k]
hipError_t launch_green_multiply(double2* spec, const double* gk, int64_t n, hipStream_t s);
// vh[z][y][x] = rpad[z][y][x] for the n-block
hipError_t launch_unpad(const double* rpad, int nx, int ny, int nz, double* vh, hipStream_t s);
// local forces of the isolated Gaussian ions: floc[J] = -h^3 sum_i rho_i v'(d) (R_J - r_i)/d;
// part: [n_ions][FREE_FORCE_CHUNKS][3]
constexpr int FREE_FORCE_CHUNKS = 512;
hipError_t launch_local_forces_free(const double* rho, const double* pos, const double* zval, int n_ions, int nx,
                                    int ny, int nz, double h, double a, double* part, double* floc, hipStream_t s);
// point-ion Coulomb: f[I] = sum_J Z_I Z_J (R_I - R_J)/R_IJ^3, epart[I] = (1/2) sum_J Z_I Z_J / R_IJ
hipError_t launch_ion_coulomb(const double* pos, const double* zval, int n_ions, double* f, double* epart,
                              hipStream_t s);

}  // namespace me

// Declarations of the grid-wide FP64 kernels (fields.hip).
#pragma once
#include "common.hpp"

namespace me {

enum ReportSlot : int {
    SLOT_EKIN = 0, SLOT_ELOC, SLOT_EH, SLOT_EX, SLOT_ENL, SLOT_EION, SLOT_EKS,
    SLOT_EIONKIN, SLOT_ETOT, SLOT_NORM_DEV, SLOT_FMAX, SLOT_CHARGE, SLOT_UNSTABLE,
    SLOT_EFICT, SLOT_CP_ITERS, SLOT_CP_RES,
    SLOT_COUNT
};

struct FinalizeArgs {
    double* rep;                 // [SLOT_COUNT]
    const double* norm_part;     // [n_orb][norm_tiles] or nullptr
    const double* fix_part;      // [n_orb][fix_tiles] nonlocal change of the norm, or nullptr
    const int32_t* nl_flag;      // nonzero: a grid point lies in too many projector spheres
    double* norms;               // [n_orb] scratch: per-orbital norms
    int n_orb;
    int norm_tiles;
    int fix_tiles;
    double norm_tol;
    double dv;                   // h^3
    double occ;
    int energy;                  // nonzero: fill the energy slots
    const double* kin_part; int64_t kin_n;
    const double* hxc_part; int64_t hxc_n;     // triples (rho V_H, e_x, rho)
    const double* loc_part; int64_t loc_n;
    const double* enl_part;                    // [n_ions]
    const double* eion_part;                   // [n_ions] real-space Ewald
    const double* erec_part; int erec_n;
    double ewald_rec_scale;                    // 2 pi / Omega
    double ewald_const;                        // self + background
    const double* vel;
    const double* frc;
    const double* mass;
    int n_ions;
    // Car-Parrinello step only (nullptr otherwise): partial sums of |psi'|^2,
    // their weight f mu_cp h^3 (the fictitious kinetic energy, added to the
    // total), and the constraint solve's (corrections, residual)
    const double* fict_part; int64_t fict_n;
    double fict_scale;
    const double* cp_info;
};

struct EwaldPlan {
    double L, eta, rc;
    int nmax;
    int ng;
    double* gv;   // [ng][3] device
    double* wv;   // [ng] device: exp(-G^2/(4 eta^2))/G^2
};

// ph: [n_ions][nx+ny+nz] exp(-i G_a(i) R_Ja); phT: the same as [nx+ny+nz][n_ions]
hipError_t launch_phases(const double* pos, int n_ions, int nx, int ny, int nz, const double L[3],
                         double2* ph, double2* phT, hipStream_t s);
hipError_t launch_vloc_spectrum(const double2* ph, const double2* phT, const double* zval, int n_ions,
                                int nx, int ny, int nz, const double L[3], double a, double2* out,
                                hipStream_t s);
hipError_t launch_hartree_spectrum(const double2* rhok, int nx, int ny, int nz, const double L[3],
                                   double2* out, hipStream_t s);
hipError_t launch_vhxc(const double* rho, const double* vh, int64_t N, double* vhxc, double* part,
                       hipStream_t s);
template <typename T>
hipError_t launch_veff(const double* vloc0, const double* vloc1, const double* hn, const double* hn1,
                       const double* hn2, int nhist, int nx, int64_t N, double h, double Lx,
                       double eps, T* veff0, T* veff1, const uint8_t* mask, hipStream_t s);
int local_force_chunks(int64_t N);
// part: [n_ions][local_force_chunks][3] scratch; floc: [n_ions][3]
hipError_t launch_local_forces(const double2* rhok, const double2* phT, const double* zval,
                               int n_ions, int nx, int ny, int nz, const double L[3], double h,
                               double a, double* part, double* floc, hipStream_t s);
// scratch: ewald_scratch_doubles(n_ions) doubles; erec_part: ewald_sg_blocks(ng) doubles
size_t ewald_scratch_doubles(int n_ions);
int ewald_sg_blocks(int ng);
hipError_t launch_ewald(const EwaldPlan& e, const double* pos, const double* zval, int n_ions,
                        double2* sg, double* erec_part, double* f, double* epart, double* scratch,
                        hipStream_t s);
hipError_t launch_ions_predict(const double* pos, const double* vel, const double* frc,
                               const double* mass, int n_ions, double dt, int frozen, double* pos1,
                               hipStream_t s);
hipError_t launch_ions_finish(double* pos, double* vel, double* frc, const double* pos1,
                              const double* floc, const double* fnl,
                              const double* fion, const double* mass, int n_ions, double dt,
                              int frozen, hipStream_t s);
hipError_t launch_add(double* a, const double* b, int64_t n, hipStream_t s);
hipError_t launch_scale_copy(double* dst, const double* src, double sc, int64_t n, hipStream_t s);
hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* part,
                              hipStream_t s);
hipError_t launch_report(const FinalizeArgs& a, hipStream_t s);

}  // namespace me

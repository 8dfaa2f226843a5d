// Kernels of the two-band toy model of sec. 6 (eq. L_toy), integrated by
// classical RK4 with one trajectory per work-item (toy.hip).
#pragma once
#include "common.hpp"

namespace me {

struct ToyArgs {
    double R0, M_R, K_R, G0, M_G, K_G;
    double t_total;
    int n_traj, n_samples, max_substeps;
    const double* mu;        // [n_traj] mu (Ehrenfest) or mu_CP
    const int* substeps;     // [n_traj] RK4 steps per sample
    const int* window;       // [n_traj] samples per force average
    double* samples;         // [n_samples + 1][NV][n_traj] (the whole state) or nullptr
    double* d_R;             // [n_traj]
    double* d_F;             // [n_traj]
};

hipError_t launch_toy(const ToyArgs& a, bool cp, hipStream_t s);
// number of state variables: 6 (Ehrenfest), 8 (CP)
constexpr int toy_state_size(bool cp) { return cp ? 8 : 6; }
// dist[i]: max over the n_vars state variables of the normalised rms
// distance of trajectory i from trajectory ref[i] over all samples
hipError_t launch_toy_distance(int n_traj, int n_samples, int n_vars, const double* samples, const int* ref,
                               double* dist, hipStream_t s);

}  // namespace me

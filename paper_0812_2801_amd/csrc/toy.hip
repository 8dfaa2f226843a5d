// The two-band toy model of sec. 6 (eq. L_toy) by classical fourth-order
// Runge-Kutta, FP64, one trajectory per work-item: a sweep over masses and
// time steps is thousands of independent ODE integrations, each a chain of
// dependent steps, so the kernel is bound by FP64 VALU work (two sincos per
// right-hand side) and keeps the whole state in registers.
//
// Equations (the Euler-Lagrange equations of eq. L_toy):
//   Ehrenfest  mu theta_1' = (G/2) sin(theta_2 - R),  mu theta_2' = -(G/2) sin(theta_1 - R)
//   CP         mu_CP theta_i'' = -(G/2) sin(theta_i - R)
//   both       M_R R'' = F_R = -K_R (R - R_0) + (G/2)[sin(theta_1 - R) + sin(theta_2 - R)]
//              M_G G'' = -K_G (G - G_0) + (1/2)[cos(theta_1 - R) + cos(theta_2 - R)]
// The right-hand side at the end of a step is the first stage of the next,
// so each step costs four evaluations, and it also gives F_R for the
// trapezoid force average.
#include <cmath>

#include "toy.hpp"

namespace me {
namespace {

struct ToyConst {
    double R0, K_R, G0, K_G, inv_MR, inv_MG, inv_mu;
};

// state: Ehrenfest (theta_1, theta_2, R, R', G, G'); CP (theta_1, theta_2,
// theta_1', theta_2', R, R', G, G')
template <bool CP> struct Layout;
template <> struct Layout<false> { static constexpr int NV = toy_state_size(false), IR = 2, IG = 4; };
template <> struct Layout<true> { static constexpr int NV = toy_state_size(true), IR = 4, IG = 6; };

template <bool CP>
__device__ __forceinline__ void rhs(const ToyConst& c, const double* y, double* d, double& force_R) {
    constexpr int IR = Layout<CP>::IR, IG = Layout<CP>::IG;
    const double R = y[IR], G = y[IG];
    double s1, c1, s2, c2;
    sincos(y[0] - R, &s1, &c1);
    sincos(y[1] - R, &s2, &c2);
    const double hg = 0.5 * G;
    if constexpr (!CP) {
        d[0] = hg * s2 * c.inv_mu;
        d[1] = -hg * s1 * c.inv_mu;
    } else {
        d[0] = y[2];
        d[1] = y[3];
        d[2] = -hg * s1 * c.inv_mu;
        d[3] = -hg * s2 * c.inv_mu;
    }
    force_R = -c.K_R * (R - c.R0) + hg * (s1 + s2);
    d[IR] = y[IR + 1];
    d[IR + 1] = force_R * c.inv_MR;
    d[IG] = y[IG + 1];
    d[IG + 1] = (-c.K_G * (G - c.G0) + 0.5 * (c1 + c2)) * c.inv_MG;
}

template <bool CP>
__global__ __launch_bounds__(64) void toy_kernel(ToyArgs a) {
    constexpr int NV = Layout<CP>::NV, IR = Layout<CP>::IR, IG = Layout<CP>::IG;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_traj) return;
    const int64_t n = a.n_traj;
    const double mu = a.mu[i];
    const int sub = a.substeps[i];
    const int win = a.window[i];
    if (!(mu > 0.0) || !(mu < INFINITY) || sub < 1 || sub > a.max_substeps || win < 1) {
        a.d_R[i] = NAN;
        a.d_F[i] = NAN;
        if (a.samples)
            for (int64_t k = 0; k < (int64_t)(a.n_samples + 1) * NV; ++k) a.samples[k * n + i] = NAN;
        return;
    }
    const ToyConst c{a.R0, a.K_R, a.G0, a.K_G, 1.0 / a.M_R, 1.0 / a.M_G, 1.0 / mu};
    const double t_s = a.t_total / a.n_samples;
    const double dt = t_s / sub;
    const double w = sqrt(a.K_R / a.M_R);
    const double amp = 0.1 * a.R0;

    // sec. 6: R and G 10 % above equilibrium, at rest; angles at the gsBO
    // minimum theta_i = R (CP: at rest)
    double y[NV];
    for (int k = 0; k < NV; ++k) y[k] = 0.0;
    y[0] = y[1] = y[IR] = 1.1 * a.R0;
    y[IG] = 1.1 * a.G0;
    if (a.samples)
        for (int k = 0; k < NV; ++k) a.samples[k * n + i] = y[k];
    double k1[NV], k2[NV], k3[NV], k4[NV], tmp[NV];
    double F0, Fx;
    rhs<CP>(c, y, k1, F0);
    double sq_R = 0.0, sq_F = 0.0, facc = 0.0;
    int n_blocks = 0;
    for (int j = 1; j <= a.n_samples; ++j) {
        for (int s = 0; s < sub; ++s) {
            for (int k = 0; k < NV; ++k) tmp[k] = y[k] + 0.5 * dt * k1[k];
            rhs<CP>(c, tmp, k2, Fx);
            for (int k = 0; k < NV; ++k) tmp[k] = y[k] + 0.5 * dt * k2[k];
            rhs<CP>(c, tmp, k3, Fx);
            for (int k = 0; k < NV; ++k) tmp[k] = y[k] + dt * k3[k];
            rhs<CP>(c, tmp, k4, Fx);
            for (int k = 0; k < NV; ++k) y[k] = y[k] + dt / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
            double F1;
            rhs<CP>(c, y, k1, F1);          // the next step's first stage
            facc += 0.5 * dt * (F0 + F1);
            F0 = F1;
        }
        const double t = j * t_s;
        if (a.samples) {
            double* o = a.samples + (int64_t)j * NV * n + i;
            for (int k = 0; k < NV; ++k) o[k * n] = y[k];
        }
        const double dR = y[IR] - (a.R0 + amp * cos(w * t));
        sq_R += dR * dR;
        if (j % win == 0) {
            const double tau = win * t_s;
            const double fbar = facc / tau;
            const double fbo = -a.K_R * amp * (sin(w * t) - sin(w * (t - tau))) / (w * tau);
            sq_F += (fbar - fbo) * (fbar - fbo);
            n_blocks += 1;
            facc = 0.0;
        }
    }
    const double span = 0.2 * a.R0;
    a.d_R[i] = 100.0 / span * sqrt(sq_R / a.n_samples);
    a.d_F[i] = 100.0 / (a.K_R * span) * sqrt(sq_F / (n_blocks > 0 ? n_blocks : 1));
}

__global__ __launch_bounds__(256) void toy_distance_kernel(int n_traj, int n_samples, int n_vars, const double* S,
                                                           const int* ref, double* dist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_traj) return;
    const int r = ref[i];
    if (r < 0 || r >= n_traj) {
        dist[i] = NAN;
        return;
    }
    const int64_t n = n_traj;
    double worst = 0.0;
    bool nan = false;
    for (int cidx = 0; cidx < n_vars; ++cidx) {
        double sq = 0.0, lo = INFINITY, hi = -INFINITY;
        for (int j = 0; j <= n_samples; ++j) {
            const int64_t row = ((int64_t)j * n_vars + cidx) * n;
            const double xr = S[row + r];
            const double d = S[row + i] - xr;
            sq += d * d;
            lo = fmin(lo, xr);
            hi = fmax(hi, xr);
        }
        const double dc = 100.0 * sqrt(sq / (n_samples + 1)) / (hi - lo);
        if (dc != dc) nan = true;
        worst = fmax(worst, dc);
    }
    dist[i] = nan ? NAN : worst;
}

}  // namespace

hipError_t launch_toy(const ToyArgs& a, bool cp, hipStream_t s) {
    if (a.n_traj <= 0) return hipSuccess;
    const dim3 grid((a.n_traj + 63) / 64);
    if (cp)
        toy_kernel<true><<<grid, 64, 0, s>>>(a);
    else
        toy_kernel<false><<<grid, 64, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_toy_distance(int n_traj, int n_samples, int n_vars, const double* samples, const int* ref,
                               double* dist, hipStream_t s) {
    if (n_traj <= 0) return hipSuccess;
    toy_distance_kernel<<<(n_traj + 255) / 256, 256, 0, s>>>(n_traj, n_samples, n_vars, samples, ref, dist);
    return hipGetLastError();
}

}  // namespace me

// Car-Parrinello comparison step: orbital updates of RATTLE / velocity
// Verlet and the position-constraint solve (eq. EoM_CP; the electronic
// integrator the paper uses for its CP runs).  The O(N_W^2 N_C) overlap and
// rotation products run as library GEMMs (api.hip), the overlaps split over
// the grid points into batches whose partial matrices are summed here in FP64;
// these kernels are that sum, the O(N_W N_C) streams and the O(N_W^3)
// constraint iteration.
#include "cp.hpp"

namespace me {

constexpr int CP_B = 256;

template <typename T>
__global__ void __launch_bounds__(CP_B) cp_predict_kernel(cx_t<T>* __restrict__ trial, const cx_t<T>* __restrict__ psi,
                                                          const cx_t<T>* __restrict__ psidot, int64_t stride,
                                                          int64_t N, T dt, T c) {
    const int64_t i = (int64_t)blockIdx.x * CP_B + threadIdx.x;
    if (i >= N) return;
    const int64_t o = (int64_t)blockIdx.y * stride + i;
    const cx_t<T> h = trial[o], p = psi[o], v = psidot[o];
    trial[o] = cx_t<T>{(p.x + dt * v.x) - c * h.x, (p.y + dt * v.y) - c * h.y};
}

template <typename T>
__global__ void __launch_bounds__(CP_B) cp_halfvel_kernel(cx_t<T>* __restrict__ psidot,
                                                          const cx_t<T>* __restrict__ pnew,
                                                          const cx_t<T>* __restrict__ pold, int64_t stride, int64_t N,
                                                          T inv_dt) {
    const int64_t i = (int64_t)blockIdx.x * CP_B + threadIdx.x;
    if (i >= N) return;
    const int64_t o = (int64_t)blockIdx.y * stride + i;
    const cx_t<T> a = pnew[o], b = pold[o];
    psidot[o] = cx_t<T>{(a.x - b.x) * inv_dt, (a.y - b.y) * inv_dt};
}

template <typename T>
__global__ void __launch_bounds__(CP_B) cp_kick_kernel(cx_t<T>* __restrict__ psidot, const cx_t<T>* __restrict__ hpsi,
                                                       int64_t stride, int64_t N, T c) {
    const int64_t i = (int64_t)blockIdx.x * CP_B + threadIdx.x;
    if (i >= N) return;
    const int64_t o = (int64_t)blockIdx.y * stride + i;
    const cx_t<T> v = psidot[o], h = hpsi[o];
    psidot[o] = cx_t<T>{v.x - c * h.x, v.y - c * h.y};
}

static dim3 grid_pts(int64_t N, int n_orb) { return dim3((unsigned)((N + CP_B - 1) / CP_B), (unsigned)n_orb); }

template <typename T>
hipError_t launch_cp_predict(cx_t<T>* trial, const cx_t<T>* psi, const cx_t<T>* psidot, int64_t stride, int n_orb,
                             int64_t N, double dt, double c, hipStream_t s) {
    cp_predict_kernel<T><<<grid_pts(N, n_orb), CP_B, 0, s>>>(trial, psi, psidot, stride, N, (T)dt, (T)c);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cp_halfvel(cx_t<T>* psidot, const cx_t<T>* psi_new, const cx_t<T>* psi_old, int64_t stride,
                             int n_orb, int64_t N, double inv_dt, hipStream_t s) {
    cp_halfvel_kernel<T><<<grid_pts(N, n_orb), CP_B, 0, s>>>(psidot, psi_new, psi_old, stride, N, (T)inv_dt);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cp_kick(cx_t<T>* psidot, const cx_t<T>* hpsi, int64_t stride, int n_orb, int64_t N, double c,
                          hipStream_t s) {
    cp_kick_kernel<T><<<grid_pts(N, n_orb), CP_B, 0, s>>>(psidot, hpsi, stride, N, (T)c);
    return hipGetLastError();
}

// ------------------------------------------------------------ constraint solve
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {      // c + a b
    return make_double2(c.x + (a.x * b.x - a.y * b.y), c.y + (a.x * b.y + a.y * b.x));
}
__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 c) { // c + conj(a) b
    return make_double2(c.x + (a.x * b.x + a.y * b.y), c.y + (a.x * b.y - a.y * b.x));
}

__device__ __forceinline__ double block_max256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// 64 elements per workgroup; wave w sums the partials b = w, w + 4, ... of
// its element, and the four wave sums are added in wave order
template <typename T>
__global__ void __launch_bounds__(CP_B) cp_reduce_kernel(const cx_t<T>* __restrict__ part, int nb, int nn,
                                                         double scale, double2* __restrict__ out) {
    __shared__ double2 sh[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    double re = 0.0, im = 0.0;
    if (e < nn)
        for (int b = wv; b < nb; b += 4) {
            const cx_t<T> v = part[(int64_t)b * nn + e];
            re += (double)v.x;
            im += (double)v.y;
        }
    sh[wv][lane] = make_double2(re, im);
    __syncthreads();
    if (wv == 0 && e < nn) {
        const double r = ((sh[0][lane].x + sh[1][lane].x) + sh[2][lane].x) + sh[3][lane].x;
        const double i = ((sh[0][lane].y + sh[1][lane].y) + sh[2][lane].y) + sh[3][lane].y;
        out[e] = make_double2(scale * r, scale * i);
    }
}

template <typename T>
hipError_t launch_cp_reduce(const cx_t<T>* part, int nb, int n, double scale, double2* out, hipStream_t s) {
    cp_reduce_kernel<T><<<(n * n + 63) / 64, CP_B, 0, s>>>(part, nb, n * n, scale, out);
    return hipGetLastError();
}

// info[1] < 0 while the iteration runs; the corrections stop once it is set
__global__ void __launch_bounds__(CP_B) cp_x_init_kernel(const double2* __restrict__ A, int n,
                                                         double2* __restrict__ X, double* __restrict__ info) {
    const int e = blockIdx.x * CP_B + threadIdx.x;
    if (e == 0) {
        info[0] = 0.0;
        info[1] = -1.0;
    }
    if (e >= n * n) return;
    const int i = e % n, j = e / n;
    const double2 a = A[e];
    X[e] = make_double2(0.5 * ((i == j ? 1.0 : 0.0) - a.x), -0.5 * a.y);
}

// R = A + B^H X + X B + X X - I for this block's elements; part[block] = max |R|
__global__ void __launch_bounds__(CP_B) cp_x_residual_kernel(const double2* __restrict__ A,
                                                             const double2* __restrict__ B, int n,
                                                             const double2* __restrict__ X, double2* __restrict__ R,
                                                             double* __restrict__ part, const double* __restrict__ info) {
    __shared__ double sh[4];
    if (info[1] >= 0.0) return;
    const int e = blockIdx.x * CP_B + threadIdx.x;
    double worst = 0.0;
    if (e < n * n) {
        const int i = e % n, j = e / n;
        double2 r = A[e];
        if (i == j) r.x -= 1.0;
        for (int k = 0; k < n; ++k) {
            const double2 xkj = X[k + (int64_t)j * n];
            const double2 xik = X[i + (int64_t)k * n];
            r = cfma_conj(B[k + (int64_t)i * n], xkj, r);                // (B^H X)_ij
            r = cfma(xik, B[k + (int64_t)j * n], r);                     // (X B)_ij
            r = cfma(xik, xkj, r);                                       // (X X)_ij
        }
        R[e] = r;
        worst = sqrt(r.x * r.x + r.y * r.y);
    }
    const double m = block_max256(worst, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// max |R| over the blocks (every block reads all partials, so all take the
// same decision); converged or out of iterations: block 0 records the count
// and the residual, X is kept; otherwise X <- X - R/2.  A block that starts
// after block 0 has recorded sees info[1] >= 0 and leaves X alone as well.
__global__ void __launch_bounds__(CP_B) cp_x_update_kernel(int n, double tol, int iter, int max_iter,
                                                           double2* __restrict__ X, const double2* __restrict__ R,
                                                           const double* __restrict__ part, int nblk,
                                                           double* __restrict__ info) {
    if (info[1] >= 0.0) return;
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = fmax(m, part[b]);
    if (m < tol || iter == max_iter) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            info[0] = (double)iter;
            info[1] = m;
        }
        return;
    }
    const int e = blockIdx.x * CP_B + threadIdx.x;
    if (e < n * n) {
        const double2 r = R[e];
        X[e] = make_double2(X[e].x - 0.5 * r.x, X[e].y - 0.5 * r.y);
    }
}

template <typename T>
__global__ void __launch_bounds__(CP_B) cp_x_out_kernel(const double2* __restrict__ X, int n, cx_t<T>* __restrict__ out) {
    const int e = blockIdx.x * CP_B + threadIdx.x;
    if (e < n * n) out[e] = cx_t<T>{(T)X[e].x, (T)X[e].y};
}

int cp_solve_blocks(int n) { return (n * n + CP_B - 1) / CP_B; }

template <typename T>
hipError_t launch_cp_solve_x(const double2* A, const double2* B, int n, double tol, int max_iter, double2* X64,
                             double2* R64, double* part, cx_t<T>* X, double* info, hipStream_t s) {
    const int nb = cp_solve_blocks(n);
    cp_x_init_kernel<<<nb, CP_B, 0, s>>>(A, n, X64, info);
    for (int it = 0; it <= max_iter; ++it) {
        cp_x_residual_kernel<<<nb, CP_B, 0, s>>>(A, B, n, X64, R64, part, info);
        cp_x_update_kernel<<<nb, CP_B, 0, s>>>(n, tol, it, max_iter, X64, R64, part, nb, info);
    }
    cp_x_out_kernel<T><<<nb, CP_B, 0, s>>>(X64, n, X);
    return hipGetLastError();
}

// ------------------------------------------------------------ velocity matrix
template <typename T>
__global__ void __launch_bounds__(CP_B) cp_velocity_matrix_kernel(const double2* __restrict__ Q, int n,
                                                                  cx_t<T>* __restrict__ Y) {
    const int e = blockIdx.x * CP_B + threadIdx.x;
    if (e >= n * n) return;
    const int i = e % n, j = e / n;
    const double2 a = Q[e], b = Q[j + (int64_t)i * n];
    Y[e] = cx_t<T>{(T)(-0.5 * (a.x + b.x)), (T)(-0.5 * (a.y - b.y))};
}

template <typename T>
hipError_t launch_cp_velocity_matrix(const double2* Q, int n, cx_t<T>* Y, hipStream_t s) {
    cp_velocity_matrix_kernel<T><<<cp_solve_blocks(n), CP_B, 0, s>>>(Q, n, Y);
    return hipGetLastError();
}

// ------------------------------------------------------------ fictitious kinetic energy
template <typename T>
__global__ void __launch_bounds__(CP_B) cp_sq_partial_kernel(const cx_t<T>* __restrict__ v, int64_t stride, int n_orb,
                                                             int64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * CP_B + threadIdx.x;
    double s = 0.0;
    if (i < N)
        for (int A = 0; A < n_orb; ++A) {
            const cx_t<T> z = v[(int64_t)A * stride + i];
            s += (double)z.x * (double)z.x + (double)z.y * (double)z.y;
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

int64_t cp_sq_blocks(int64_t N) { return (N + CP_B - 1) / CP_B; }

template <typename T>
hipError_t launch_cp_sq_partial(const cx_t<T>* psidot, int64_t stride, int n_orb, int64_t N, double* part,
                                hipStream_t s) {
    cp_sq_partial_kernel<T><<<(unsigned)cp_sq_blocks(N), CP_B, 0, s>>>(psidot, stride, n_orb, N, part);
    return hipGetLastError();
}

#define ME_CP_INST(T)                                                                                         \
    template hipError_t launch_cp_predict<T>(cx_t<T>*, const cx_t<T>*, const cx_t<T>*, int64_t, int, int64_t, \
                                             double, double, hipStream_t);                                    \
    template hipError_t launch_cp_halfvel<T>(cx_t<T>*, const cx_t<T>*, const cx_t<T>*, int64_t, int, int64_t, \
                                             double, hipStream_t);                                            \
    template hipError_t launch_cp_kick<T>(cx_t<T>*, const cx_t<T>*, int64_t, int, int64_t, double, hipStream_t); \
    template hipError_t launch_cp_reduce<T>(const cx_t<T>*, int, int, double, double2*, hipStream_t);         \
    template hipError_t launch_cp_solve_x<T>(const double2*, const double2*, int, double, int, double2*,       \
                                             double2*, double*, cx_t<T>*, double*, hipStream_t);             \
    template hipError_t launch_cp_velocity_matrix<T>(const double2*, int, cx_t<T>*, hipStream_t);             \
    template hipError_t launch_cp_sq_partial<T>(const cx_t<T>*, int64_t, int, int64_t, double*, hipStream_t);
ME_CP_INST(double)
ME_CP_INST(float)

}  // namespace me

// Kernels of the discrete adjoint of an AETRS trajectory with frozen ions
// (reverse mode through the Taylor-Horner stages, the density and the
// Hartree-exchange potential), and of the coarse static-potential control.
//
// Complex adjoints follow xbar = dJ/dRe(x) + i dJ/dIm(x).  For one Horner
// stage u_{k-1} = psi0 + c_k H(w) u_k, c_k = i alpha (alpha = -tau/k):
//   psi0bar += ubar_{k-1},   ubar_k = conj(c_k) H ubar_{k-1}   (H Hermitian),
//   wbar(r) += sum_A Re[conj(ubar_{k-1,A}(r)) c_k u_{k,A}(r)].
#include "adjoint.hpp"

namespace me {

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// wbar(r) += sum_A Re[conj(ub_A) (i alpha) u_A] = -alpha sum_A Im[conj(ub_A) u_A];
// acc_A = ub_A (init) or acc_A += ub_A.  One thread per grid point.
template <typename T>
__global__ void cross_accum_kernel(const cx_t<T>* __restrict__ ub, const cx_t<T>* __restrict__ u,
                                   cx_t<T>* __restrict__ acc, int64_t stride, int n_orb, int64_t N,
                                   double alpha, int init, double* __restrict__ wbar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int A = 0; A < n_orb; ++A) {
        const int64_t o = (int64_t)A * stride + i;
        const cx_t<T> a = ub[o];
        const cx_t<T> b = u[o];
        s += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
        if (init) {
            acc[o] = a;
        } else {
            cx_t<T> c = acc[o];
            c.x += a.x;
            c.y += a.y;
            acc[o] = c;
        }
    }
    wbar[i] += -alpha * s;
}

// acc_A += ub_A
template <typename T>
__global__ void accum_kernel(const cx_t<T>* __restrict__ ub, cx_t<T>* __restrict__ acc, int64_t stride,
                             int n_orb, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int A = 0; A < n_orb; ++A) {
        const int64_t o = (int64_t)A * stride + i;
        cx_t<T> c = acc[o];
        const cx_t<T> a = ub[o];
        c.x += a.x;
        c.y += a.y;
        acc[o] = c;
    }
}

// lam_A += 2 f rhobar psi_A   (rho = f sum |psi|^2)
template <typename T>
__global__ void lambda_update_kernel(cx_t<T>* __restrict__ lam, const cx_t<T>* __restrict__ psi,
                                     const double* __restrict__ rhobar, int64_t stride, int n_orb,
                                     int64_t N, double occ) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double g = 2.0 * occ * rhobar[i];
    for (int A = 0; A < n_orb; ++A) {
        const int64_t o = (int64_t)A * stride + i;
        cx_t<T> l = lam[o];
        const cx_t<T> p = psi[o];
        l.x = (T)((double)l.x + g * (double)p.x);
        l.y = (T)((double)l.y + g * (double)p.y);
        lam[o] = l;
    }
}

// rhobar = (Hartree(vbar) from the C2R output, already normalised) + f_x(rho) vbar + extra
// with f_x = dv_x/drho = -(1/3)(3/pi)^(1/3) rho^(-2/3)
__global__ void vhxc_adjoint_kernel(const double* __restrict__ hv, const double* __restrict__ vbar,
                                    const double* __restrict__ rho, const double* __restrict__ extra,
                                    int64_t N, double* __restrict__ rhobar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double c = cbrt(rho[i]);
    const double fx = -(1.0 / 3.0) * cbrt(3.0 / M_PI) / (c * c);
    double r = hv[i] + vbar[i] * fx;
    if (extra != nullptr) r += extra[i];
    rhobar[i] = r;
}

// dst += a * src
__global__ void axpy_kernel(double* __restrict__ dst, const double* __restrict__ src, double a, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[i] += a * src[i];
}

__global__ void zero_f64_kernel(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// part[b] = sum over a 256-point block of (h*ix - L/2) * f[i]
__global__ void __launch_bounds__(256) field_dot_kernel(const double* __restrict__ f, int nx, int64_t N,
                                                        double h, double Lx, double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < N) v = (h * (double)(i % nx) - 0.5 * Lx) * f[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// out[0] = scale * sum part[0..n) in a fixed order (one workgroup)
__global__ void __launch_bounds__(256) sum_parts_kernel(const double* __restrict__ part, int64_t n,
                                                        double scale, double* __restrict__ out) {
    __shared__ double sh[4];
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) v += part[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = scale * (((sh[0] + sh[1]) + sh[2]) + sh[3]);
}

// rhobar of the final dipole J = h^3 sum (h*ix - L/2) rho
__global__ void dipole_rhobar_kernel(double* __restrict__ rb, int nx, int64_t N, double h, double Lx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) rb[i] = h * h * h * (h * (double)(i % nx) - 0.5 * Lx);
}

// periodic trilinear interpolation from an m^3 coarse grid to the n^3 grid
// (fine point i at coarse coordinate i*m/n, n/m integer)
__global__ void coarse_to_fine_kernel(const double* __restrict__ c, int m, int n, double* __restrict__ f) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = (int64_t)n * n * n;
    if (t >= N) return;
    const int r = n / m;
    const int ix = (int)(t % n), iy = (int)((t / n) % n), iz = (int)(t / ((int64_t)n * n));
    const int x0 = ix / r, y0 = iy / r, z0 = iz / r;
    const double tx = (double)(ix % r) / r, ty = (double)(iy % r) / r, tz = (double)(iz % r) / r;
    const int x1 = (x0 + 1) % m, y1 = (y0 + 1) % m, z1 = (z0 + 1) % m;
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    const int xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1};
    double v = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d)
                v += wz[a] * wy[b] * wx[d] * c[((int64_t)zs[a] * m + ys[b]) * m + xs[d]];
    f[t] = v;
}

// transpose of the interpolation: one thread per coarse point gathers the
// fine points whose stencil includes it (no atomics, fixed order)
__global__ void fine_to_coarse_kernel(const double* __restrict__ f, int m, int n, double* __restrict__ c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = (int64_t)m * m * m;
    if (t >= M) return;
    const int r = n / m;
    const int cx = (int)(t % m), cy = (int)((t / m) % m), cz = (int)(t / ((int64_t)m * m));
    double v = 0.0;
    // fine points of axis a with nonzero weight for coarse index c: i in [(c-1)r+1, (c+1)r-1] (periodic)
    for (int dz = -r + 1; dz <= r - 1; ++dz) {
        const double wz = 1.0 - (double)(dz < 0 ? -dz : dz) / r;
        const int iz = ((cz * r + dz) % n + n) % n;
        for (int dy = -r + 1; dy <= r - 1; ++dy) {
            const double wy = 1.0 - (double)(dy < 0 ? -dy : dy) / r;
            const int iy = ((cy * r + dy) % n + n) % n;
            for (int dx = -r + 1; dx <= r - 1; ++dx) {
                const double wx = 1.0 - (double)(dx < 0 ? -dx : dx) / r;
                const int ix = ((cx * r + dx) % n + n) % n;
                v += wz * wy * wx * f[((int64_t)iz * n + iy) * n + ix];
            }
        }
    }
    c[t] = v;
}

// ------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_cross_accum(const cx_t<T>* ub, const cx_t<T>* u, cx_t<T>* acc, int64_t stride, int n_orb,
                              int64_t N, double alpha, bool init, double* wbar, hipStream_t s) {
    cross_accum_kernel<T><<<nblk(N), 256, 0, s>>>(ub, u, acc, stride, n_orb, N, alpha, init ? 1 : 0, wbar);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_accum(const cx_t<T>* ub, cx_t<T>* acc, int64_t stride, int n_orb, int64_t N, hipStream_t s) {
    accum_kernel<T><<<nblk(N), 256, 0, s>>>(ub, acc, stride, n_orb, N);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_lambda_update(cx_t<T>* lam, const cx_t<T>* psi, const double* rhobar, int64_t stride,
                                int n_orb, int64_t N, double occ, hipStream_t s) {
    lambda_update_kernel<T><<<nblk(N), 256, 0, s>>>(lam, psi, rhobar, stride, n_orb, N, occ);
    return hipGetLastError();
}
hipError_t launch_vhxc_adjoint(const double* hv, const double* vbar, const double* rho, const double* extra,
                               int64_t N, double* rhobar, hipStream_t s) {
    vhxc_adjoint_kernel<<<nblk(N), 256, 0, s>>>(hv, vbar, rho, extra, N, rhobar);
    return hipGetLastError();
}
hipError_t launch_axpy(double* dst, const double* src, double a, int64_t N, hipStream_t s) {
    axpy_kernel<<<nblk(N), 256, 0, s>>>(dst, src, a, N);
    return hipGetLastError();
}
hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
    zero_f64_kernel<<<nblk(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}
hipError_t launch_field_dot(const double* f, int nx, int64_t N, double h, double Lx, double* part,
                            double* out, double scale, hipStream_t s) {
    field_dot_kernel<<<nblk(N), 256, 0, s>>>(f, nx, N, h, Lx, part);
    sum_parts_kernel<<<1, 256, 0, s>>>(part, (int64_t)nblk(N), scale, out);
    return hipGetLastError();
}
hipError_t launch_dipole_rhobar(double* rb, int nx, int64_t N, double h, double Lx, hipStream_t s) {
    dipole_rhobar_kernel<<<nblk(N), 256, 0, s>>>(rb, nx, N, h, Lx);
    return hipGetLastError();
}
hipError_t launch_coarse_to_fine(const double* c, int m, int n, double* f, hipStream_t s) {
    coarse_to_fine_kernel<<<nblk((int64_t)n * n * n), 256, 0, s>>>(c, m, n, f);
    return hipGetLastError();
}
hipError_t launch_fine_to_coarse(const double* f, int m, int n, double* c, hipStream_t s) {
    fine_to_coarse_kernel<<<nblk((int64_t)m * m * m), 256, 0, s>>>(f, m, n, c);
    return hipGetLastError();
}

template hipError_t launch_cross_accum<double>(const cx_t<double>*, const cx_t<double>*, cx_t<double>*, int64_t, int, int64_t, double, bool, double*, hipStream_t);
template hipError_t launch_cross_accum<float>(const cx_t<float>*, const cx_t<float>*, cx_t<float>*, int64_t, int, int64_t, double, bool, double*, hipStream_t);
template hipError_t launch_accum<double>(const cx_t<double>*, cx_t<double>*, int64_t, int, int64_t, hipStream_t);
template hipError_t launch_accum<float>(const cx_t<float>*, cx_t<float>*, int64_t, int, int64_t, hipStream_t);
template hipError_t launch_lambda_update<double>(cx_t<double>*, const cx_t<double>*, const double*, int64_t, int, int64_t, double, hipStream_t);
template hipError_t launch_lambda_update<float>(cx_t<float>*, const cx_t<float>*, const double*, int64_t, int, int64_t, double, hipStream_t);

}  // namespace me

// The finite box (sec. 5: the union of spheres of fixed radius around the
// atoms, orbitals zero outside) and the potentials of an isolated system:
// the Gaussian ions' local potential and forces summed directly over the
// ions, the point-ion Coulomb energy, and the free-space Hartree potential
// as the aperiodic convolution of the grid charge with 1/|r| (cell average
// c0 / h at r = 0, c0 = 3 ln(2 + sqrt 3) - pi / 2), evaluated by FFTs on the
// doubled grid (zero padding makes the circular convolution aperiodic on the
// original block).  All FP64.
#include <cmath>

#include "finite.hpp"

namespace me {
namespace {

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__global__ void box_mask_kernel(const double* __restrict__ pos0, int n_ions, int nx, int ny, int nz, double h,
                                double r2max, uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = (int64_t)nx * ny * nz;
    if (i >= N) return;
    const double x = h * (double)(i % nx), y = h * (double)((i / nx) % ny), z = h * (double)(i / ((int64_t)nx * ny));
    uint8_t in = 0;
    for (int J = 0; J < n_ions; ++J) {
        const double dx = x - pos0[3 * J], dy = y - pos0[3 * J + 1], dz = z - pos0[3 * J + 2];
        if (dx * dx + dy * dy + dz * dz <= r2max) in = 1;
    }
    mask[i] = in;
}

template <typename T>
__global__ void mask_orbitals_kernel(cx_t<T>* __restrict__ psi, int64_t stride, int n_orb, int64_t N,
                                     const uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || mask[i]) return;
    for (int o = 0; o < n_orb; ++o) psi[o * stride + i] = cx_t<T>{(T)0, (T)0};
}

__global__ void vloc_free_kernel(const double* __restrict__ pos, const double* __restrict__ zval, int n_ions,
                                 int nx, int ny, int nz, double h, double a, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = (int64_t)nx * ny * nz;
    if (i >= N) return;
    const double x = h * (double)(i % nx), y = h * (double)((i / nx) % ny), z = h * (double)(i / ((int64_t)nx * ny));
    const double at0 = 2.0 / (a * sqrt(M_PI));
    double v = 0.0;
    for (int J = 0; J < n_ions; ++J) {
        const double dx = x - pos[3 * J], dy = y - pos[3 * J + 1], dz = z - pos[3 * J + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        v -= zval[J] * (d == 0.0 ? at0 : erf(d / a) / d);
    }
    out[i] = v;
}

__global__ void green_doubled_kernel(int nx, int ny, int nz, double h, double c0h, double* __restrict__ g) {
    const int mx = 2 * nx, my = 2 * ny, mz = 2 * nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)mx * my * mz) return;
    const int ix = (int)(i % mx), iy = (int)((i / mx) % my), iz = (int)(i / ((int64_t)mx * my));
    const double dx = h * (double)(ix <= nx ? ix : mx - ix);
    const double dy = h * (double)(iy <= ny ? iy : my - iy);
    const double dz = h * (double)(iz <= nz ? iz : mz - iz);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    g[i] = r == 0.0 ? c0h : 1.0 / r;
}

__global__ void green_spectrum_kernel(const double2* __restrict__ spec, int64_t n, double scale,
                                      double* __restrict__ gk) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) gk[i] = scale * spec[i].x;
}

// every point of the doubled grid: the charge on the corner block, zero
// elsewhere (rewritten each time, so nothing depends on what the forward
// transform leaves in its input)
__global__ void pad_kernel(const double* __restrict__ rho, int nx, int ny, int nz, double* __restrict__ rpad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t mx = 2 * nx, my = 2 * ny;
    if (i >= mx * my * 2 * nz) return;
    const int64_t x = i % mx, y = (i / mx) % my, z = i / (mx * my);
    rpad[i] = (x < nx && y < ny && z < nz) ? rho[(z * ny + y) * nx + x] : 0.0;
}

__global__ void green_multiply_kernel(double2* __restrict__ spec, const double* __restrict__ gk, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = gk[i];
    spec[i] = double2{spec[i].x * g, spec[i].y * g};
}

__global__ void unpad_kernel(const double* __restrict__ rpad, int nx, int ny, int nz, double* __restrict__ vh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny * nz) return;
    const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
    vh[i] = rpad[(z * 2 * ny + y) * 2 * nx + x];
}

// block b of FREE_FORCE_CHUNKS takes a contiguous range of points and
// reads it once per group of FF_IONS ions, each thread keeping the group's
// 3 * FF_IONS sums in registers; the block then reduces them in a fixed
// order (wave shuffles, then the four waves in turn)
constexpr int FF_IONS = 8;

__global__ void __launch_bounds__(256) local_forces_free_kernel(const double* __restrict__ rho,
                                                                const double* __restrict__ pos,
                                                                const double* __restrict__ zval, int n_ions,
                                                                int nx, int ny, int nz, double h, double a,
                                                                double* __restrict__ part) {
    __shared__ double red[4][3 * FF_IONS];
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t per = (N + FREE_FORCE_CHUNKS - 1) / FREE_FORCE_CHUNKS;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < N ? i0 + per : N;
    const double c = 2.0 / (a * sqrt(M_PI));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int J0 = 0; J0 < n_ions; J0 += FF_IONS) {
        const int nj = n_ions - J0 < FF_IONS ? n_ions - J0 : FF_IONS;
        double f[FF_IONS][3];
#pragma unroll
        for (int j = 0; j < FF_IONS; ++j) f[j][0] = f[j][1] = f[j][2] = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            const double r = rho[i];
            if (r == 0.0) continue;
            const double x = h * (double)(i % nx), y = h * (double)((i / nx) % ny);
            const double z = h * (double)(i / ((int64_t)nx * ny));
#pragma unroll
            for (int j = 0; j < FF_IONS; ++j) {
                if (j >= nj) break;
                const int J = J0 + j;
                const double dx = pos[3 * J] - x, dy = pos[3 * J + 1] - y, dz = pos[3 * J + 2] - z;
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 == 0.0) continue;
                const double d = sqrt(d2);
                const double vp = zval[J] * (erf(d / a) / d2 - c * exp(-d2 / (a * a)) / d);
                const double w = r * vp / d;
                f[j][0] += w * dx;
                f[j][1] += w * dy;
                f[j][2] += w * dz;
            }
        }
#pragma unroll
        for (int j = 0; j < FF_IONS; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double v = f[j][k];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                if (lane == 0) red[wv][3 * j + k] = v;
            }
        __syncthreads();
        if ((int)threadIdx.x < 3 * nj) {
            const int j = threadIdx.x / 3, k = threadIdx.x % 3;
            part[((int64_t)(J0 + j) * FREE_FORCE_CHUNKS + blockIdx.x) * 3 + k] =
                ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
        }
        __syncthreads();
    }
}

// one block per ion: each thread adds two chunks, then a tree in LDS (a
// fixed order, so the result does not depend on timing)
__global__ void __launch_bounds__(256) local_forces_free_sum_kernel(const double* __restrict__ part, double dv,
                                                                    double* __restrict__ floc) {
    static_assert(FREE_FORCE_CHUNKS == 512, "two chunks per thread of a 256-thread block");
    __shared__ double red[3][256];
    const int J = blockIdx.x, t = threadIdx.x;
    const double* p = part + (int64_t)J * FREE_FORCE_CHUNKS * 3;
    for (int k = 0; k < 3; ++k) red[k][t] = p[t * 3 + k] + p[(t + 256) * 3 + k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int k = 0; k < 3; ++k) red[k][t] += red[k][t + st];
        __syncthreads();
    }
    if (t < 3) floc[3 * J + t] = -dv * red[t][0];
}

__global__ void ion_coulomb_kernel(const double* __restrict__ pos, const double* __restrict__ zval, int n_ions,
                                   double* __restrict__ f, double* __restrict__ epart) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n_ions) return;
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int J = 0; J < n_ions; ++J) {
        if (J == I) continue;
        const double dx = pos[3 * I] - pos[3 * J], dy = pos[3 * I + 1] - pos[3 * J + 1], dz = pos[3 * I + 2] - pos[3 * J + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double zz = zval[I] * zval[J];
        e += zz / r;
        const double g = zz / (r * r * r);
        fx += g * dx;
        fy += g * dy;
        fz += g * dz;
    }
    epart[I] = 0.5 * e;
    f[3 * I] = fx;
    f[3 * I + 1] = fy;
    f[3 * I + 2] = fz;
}

}  // namespace

hipError_t launch_box_mask(const double* pos0, int n_ions, int nx, int ny, int nz, double h, double radius,
                           uint8_t* mask, hipStream_t s) {
    const int64_t N = (int64_t)nx * ny * nz;
    box_mask_kernel<<<nblk(N), 256, 0, s>>>(pos0, n_ions, nx, ny, nz, h, radius * radius, mask);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mask_orbitals(cx_t<T>* psi, int64_t stride, int n_orb, int64_t N, const uint8_t* mask,
                                hipStream_t s) {
    mask_orbitals_kernel<T><<<nblk(N), 256, 0, s>>>(psi, stride, n_orb, N, mask);
    return hipGetLastError();
}
template hipError_t launch_mask_orbitals<double>(double2*, int64_t, int, int64_t, const uint8_t*, hipStream_t);
template hipError_t launch_mask_orbitals<float>(float2*, int64_t, int, int64_t, const uint8_t*, hipStream_t);

hipError_t launch_vloc_free(const double* pos, const double* zval, int n_ions, int nx, int ny, int nz, double h,
                            double a, double* out, hipStream_t s) {
    const int64_t N = (int64_t)nx * ny * nz;
    vloc_free_kernel<<<nblk(N), 256, 0, s>>>(pos, zval, n_ions, nx, ny, nz, h, a, out);
    return hipGetLastError();
}

hipError_t launch_green_doubled(int nx, int ny, int nz, double h, double* g2, hipStream_t s) {
    const double c0 = 3.0 * log(2.0 + sqrt(3.0)) - 0.5 * M_PI;
    green_doubled_kernel<<<nblk((int64_t)8 * nx * ny * nz), 256, 0, s>>>(nx, ny, nz, h, c0 / h, g2);
    return hipGetLastError();
}

hipError_t launch_green_spectrum(const double2* spec, int64_t n, double scale, double* gk, hipStream_t s) {
    green_spectrum_kernel<<<nblk(n), 256, 0, s>>>(spec, n, scale, gk);
    return hipGetLastError();
}

hipError_t launch_pad(const double* rho, int nx, int ny, int nz, double* rpad, hipStream_t s) {
    pad_kernel<<<nblk((int64_t)8 * nx * ny * nz), 256, 0, s>>>(rho, nx, ny, nz, rpad);
    return hipGetLastError();
}

hipError_t launch_green_multiply(double2* spec, const double* gk, int64_t n, hipStream_t s) {
    green_multiply_kernel<<<nblk(n), 256, 0, s>>>(spec, gk, n);
    return hipGetLastError();
}

hipError_t launch_unpad(const double* rpad, int nx, int ny, int nz, double* vh, hipStream_t s) {
    unpad_kernel<<<nblk((int64_t)nx * ny * nz), 256, 0, s>>>(rpad, nx, ny, nz, vh);
    return hipGetLastError();
}

hipError_t launch_local_forces_free(const double* rho, const double* pos, const double* zval, int n_ions, int nx,
                                    int ny, int nz, double h, double a, double* part, double* floc, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    local_forces_free_kernel<<<FREE_FORCE_CHUNKS, 256, 0, s>>>(rho, pos, zval, n_ions, nx, ny, nz, h, a, part);
    local_forces_free_sum_kernel<<<n_ions, 256, 0, s>>>(part, h * h * h, floc);
    return hipGetLastError();
}

hipError_t launch_ion_coulomb(const double* pos, const double* zval, int n_ions, double* f, double* epart,
                              hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    ion_coulomb_kernel<<<nblk(n_ions, 64), 64, 0, s>>>(pos, zval, n_ions, f, epart);
    return hipGetLastError();
}

}  // namespace me

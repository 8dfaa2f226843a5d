// Grid-wide quantities of one step, all in FP64: density, the local ionic
// potential by structure factor (eq. ionicpotential), Hartree and Slater
// exchange, the effective potentials of the two AETRS exponentials, the
// local-potential forces (eq. ionicforces, as -dE/dR), the Ewald ion-ion
// term, velocity Verlet and deterministic reductions.
#include "fields.hpp"
#include "geometry.hpp"

namespace me {

__device__ __forceinline__ int wavenum(int i, int n) { return i <= (n - 1) / 2 ? i : i - n; }

__device__ __forceinline__ double dsum_wave(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block-level sum for 256-thread blocks; result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = dsum_wave(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ density
// rho(r) = occ sum_A |psi_A(r)|^2, the orbital sum in order in FP64 at each
// point.  A thread takes two adjacent points of FP32 orbitals (one 16-byte
// load per orbital, as for one FP64 point), and the orbital loop is unrolled
// so that eight orbitals' loads are in flight at once.
template <typename T>
__device__ __forceinline__ double cabs2(cx_t<T> z) {
    return (double)z.x * (double)z.x + (double)z.y * (double)z.y;
}

template <typename T>
__global__ void __launch_bounds__(256) density_kernel(const cx_t<T>* __restrict__ psi, int64_t stride,
                                                      int n_orb, int64_t N, double occ,
                                                      double* __restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
#pragma unroll 8
    for (int A = 0; A < n_orb; ++A) s += cabs2<T>(psi[(int64_t)A * stride + i]);
    rho[i] = occ * s;
}

// FP32 orbitals, points 2i and 2i + 1 (stride and psi 16-byte aligned)
__global__ void __launch_bounds__(256) density_pair_kernel(const float4* __restrict__ psi, int64_t stride2,
                                                           int n_orb, int64_t N, double occ,
                                                           double* __restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * i >= N) return;
    double s0 = 0.0, s1 = 0.0;
    if (2 * i + 1 < N) {
#pragma unroll 8
        for (int A = 0; A < n_orb; ++A) {
            const float4 z = psi[(int64_t)A * stride2 + i];
            s0 += cabs2<float>(make_float2(z.x, z.y));
            s1 += cabs2<float>(make_float2(z.z, z.w));
        }
        rho[2 * i] = occ * s0;
        rho[2 * i + 1] = occ * s1;
    } else {                                          // odd N: the last point alone
        const float2* p = reinterpret_cast<const float2*>(psi);
        for (int A = 0; A < n_orb; ++A) s0 += cabs2<float>(p[(int64_t)A * 2 * stride2 + 2 * i]);
        rho[2 * i] = occ * s0;
    }
}

template <typename T>
hipError_t launch_density(const cx_t<T>* psi, int64_t stride, int n_orb, int64_t N,
                          double occ, double* rho, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (stride % 2 == 0 && reinterpret_cast<uintptr_t>(psi) % 16 == 0) {
            const int64_t pairs = (N + 1) / 2;
            density_pair_kernel<<<(unsigned)((pairs + 255) / 256), 256, 0, s>>>(
                reinterpret_cast<const float4*>(psi), stride / 2, n_orb, N, occ, rho);
            return hipGetLastError();
        }
    }
    density_kernel<T><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(psi, stride, n_orb, N, occ, rho);
    return hipGetLastError();
}
template hipError_t launch_density<double>(const cx_t<double>*, int64_t, int, int64_t, double, double*, hipStream_t);
template hipError_t launch_density<float>(const cx_t<float>*, int64_t, int, int64_t, double, double*, hipStream_t);

// ------------------------------------------------------------ phases
// ph[J][a][i] = exp(-i G_a(i) R_Ja), G_a(i) = 2 pi m(i)/L_a, for i in [0, n_a)
__global__ void phase_kernel(const double* __restrict__ pos, int n_ions, int nx, int ny, int nz,
                             double Lx, double Ly, double Lz, double2* __restrict__ ph,
                             double2* __restrict__ phT) {
    const int nt = nx + ny + nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_ions * nt) return;
    const int J = (int)(t / nt);
    int i = (int)(t % nt);
    int a = 0, n = nx;
    double L = Lx;
    if (i >= nx) { i -= nx; a = 1; n = ny; L = Ly; if (i >= ny) { i -= ny; a = 2; n = nz; L = Lz; } }
    const double g = 2.0 * M_PI * (double)wavenum(i, n) / L;
    double sn, cs;
    sincos(-g * pos[3 * J + a], &sn, &cs);
    ph[t] = make_double2(cs, sn);
    phT[(int64_t)(t % nt) * n_ions + J] = make_double2(cs, sn);   // [axis offset + i][J]
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// structure factor S(G) = sum_J Z_J exp(-i G.R_J) at box index (ix, iy, iz)
__device__ __forceinline__ double2 sfac(const double2* __restrict__ ph, const double* __restrict__ zval,
                                        int n_ions, int nt, int nx, int ny, int ix, int iy, int iz) {
    double2 s = make_double2(0.0, 0.0);
    for (int J = 0; J < n_ions; ++J) {
        const double2* pj = ph + (int64_t)J * nt;
        const double2 e = cmul(cmul(pj[ix], pj[nx + iy]), pj[nx + ny + iz]);
        s.x += zval[J] * e.x;
        s.y += zval[J] * e.y;
    }
    return s;
}

__device__ __forceinline__ double vloc_ff(double g2, double a) {
    return -4.0 * M_PI / g2 * exp(-g2 * a * a / 4.0);
}

// Half spectrum (ix in [0, nx/2]) of the Hermitian part of V_loc(G)/Omega:
// W(k) = (V(k) + conj(V(k*)))/2, k* the index mirror; W = V(k) away from the
// Nyquist planes.  Its complex-to-real transform is Re of the full-box sum.
__global__ void vloc_spectrum_kernel(const double2* __restrict__ ph, const double* __restrict__ zval,
                                     int n_ions, int nx, int ny, int nz, double Lx, double Ly,
                                     double Lz, double a, double inv_omega,
                                     double2* __restrict__ out) {
    const int nh = nx / 2 + 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nh * ny * nz) return;
    const int ix = (int)(t % nh);
    const int iy = (int)((t / nh) % ny);
    const int iz = (int)(t / ((int64_t)nh * ny));
    const int nt = nx + ny + nz;
    const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
    const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
    const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double2 w = make_double2(0.0, 0.0);
    if (g2 > 0.0) {
        const double2 s = sfac(ph, zval, n_ions, nt, nx, ny, ix, iy, iz);
        const double f = vloc_ff(g2, a) * inv_omega;
        w = make_double2(f * s.x, f * s.y);
        const bool nyq = ((nx % 2 == 0) && ix == nx / 2) || ((ny % 2 == 0) && iy == ny / 2) ||
                         ((nz % 2 == 0) && iz == nz / 2);
        if (nyq) {
            const int mx = (nx - ix) % nx, my = (ny - iy) % ny, mz = (nz - iz) % nz;
            const double hx = 2.0 * M_PI * wavenum(mx, nx) / Lx;
            const double hy = 2.0 * M_PI * wavenum(my, ny) / Ly;
            const double hz = 2.0 * M_PI * wavenum(mz, nz) / Lz;
            const double h2 = hx * hx + hy * hy + hz * hz;
            const double2 sm = sfac(ph, zval, n_ions, nt, nx, ny, mx, my, mz);
            const double fm = vloc_ff(h2, a) * inv_omega;
            w = make_double2(0.5 * (w.x + fm * sm.x), 0.5 * (w.y - fm * sm.y));
        }
    }
    out[t] = w;
}

// The same half spectrum, computed row by row.  A workgroup takes VR_ROWS
// x-rows (iy, iz) and the ions in chunks of VR_CH: the x phases of the chunk
// and b_J = Z_J ey_J(iy) ez_J(iz) of its rows are staged in LDS, and lane ix
// of wave w sums b_J ex_J(ix) for four rows.  Points with a Nyquist index
// (whose mirror lies in another row) are left to vloc_nyquist_kernel.
constexpr int VR_ROWS = 16;
constexpr int VR_CH = 64;

__device__ __forceinline__ bool nyq_row(int iy, int iz, int ny, int nz) {
    return ((ny % 2 == 0) && iy == ny / 2) || ((nz % 2 == 0) && iz == nz / 2);
}

__global__ void __launch_bounds__(256) vloc_rows_kernel(const double2* __restrict__ ph,
                                                        const double2* __restrict__ phT,
                                                        const double* __restrict__ zval, int n_ions,
                                                        int nx, int ny, int nz, double Lx, double Ly,
                                                        double Lz, double a, double inv_omega,
                                                        double2* __restrict__ out) {
    __shared__ double2 ex[VR_CH * 64];
    __shared__ double2 bc[VR_ROWS * VR_CH];
    const int nh = nx / 2 + 1;
    const int nt = nx + ny + nz;
    const int rows = ny * nz;
    const int r0 = blockIdx.x * VR_ROWS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int ix0 = 0; ix0 < nh; ix0 += 64) {
        double2 acc[VR_ROWS / 4];
#pragma unroll
        for (int q = 0; q < VR_ROWS / 4; ++q) acc[q] = make_double2(0.0, 0.0);
        for (int J0 = 0; J0 < n_ions; J0 += VR_CH) {
            const int cnt = min(VR_CH, n_ions - J0);
            __syncthreads();
            for (int e = threadIdx.x; e < cnt * 64; e += blockDim.x) {
                const int j = e >> 6, xi = e & 63;
                ex[e] = ix0 + xi < nh ? ph[(int64_t)(J0 + j) * nt + ix0 + xi] : make_double2(0.0, 0.0);
            }
            for (int e = threadIdx.x; e < VR_ROWS * cnt; e += blockDim.x) {
                const int rr = e / cnt, j = e - rr * cnt;
                const int row = r0 + rr;
                double2 b = make_double2(0.0, 0.0);
                if (row < rows) {
                    const int iy = row % ny, iz = row / ny, J = J0 + j;
                    const double2 t = cmul(phT[(int64_t)(nx + iy) * n_ions + J], phT[(int64_t)(nx + ny + iz) * n_ions + J]);
                    b = make_double2(zval[J] * t.x, zval[J] * t.y);
                }
                bc[rr * VR_CH + j] = b;
            }
            __syncthreads();
            for (int j = 0; j < cnt; ++j) {
                const double2 e = ex[j * 64 + lane];
#pragma unroll
                for (int q = 0; q < VR_ROWS / 4; ++q) {
                    const double2 b = bc[(wv * (VR_ROWS / 4) + q) * VR_CH + j];
                    acc[q].x += b.x * e.x - b.y * e.y;
                    acc[q].y += b.x * e.y + b.y * e.x;
                }
            }
        }
        const int ix = ix0 + lane;
#pragma unroll
        for (int q = 0; q < VR_ROWS / 4; ++q) {
            const int row = r0 + wv * (VR_ROWS / 4) + q;
            if (row >= rows || ix >= nh) continue;
            const int iy = row % ny, iz = row / ny;
            if (nyq_row(iy, iz, ny, nz) || ((nx % 2 == 0) && ix == nx / 2)) continue;
            const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
            const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
            const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
            const double g2 = gx * gx + gy * gy + gz * gz;
            double2 w = make_double2(0.0, 0.0);
            if (g2 > 0.0) {
                const double f = vloc_ff(g2, a) * inv_omega;
                w = make_double2(f * acc[q].x, f * acc[q].y);
            }
            out[(int64_t)row * nh + ix] = w;
        }
    }
}

// The points vloc_rows_kernel leaves: the ix = nx/2 column of every row, and
// the other points of the rows with iy = ny/2 or iz = nz/2; each by the
// direct per-point sum with its mirror.
__global__ void vloc_nyquist_kernel(const double2* __restrict__ ph, const double* __restrict__ zval,
                                    int n_ions, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                    double a, double inv_omega, double2* __restrict__ out) {
    const int nh = nx / 2 + 1;
    const int rows = ny * nz;
    const int ncol = (nx % 2 == 0) ? rows : 0;                  // column ix = nx/2
    const int nxr = (nx % 2 == 0) ? nh - 1 : nh;                // other points of a row
    const int nry = (ny % 2 == 0) ? nz : 0;                     // rows iy = ny/2
    const int nrz = (nz % 2 == 0) ? ny - (ny % 2 == 0 ? 1 : 0) : 0;   // rows iz = nz/2, iy != ny/2
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int ix, iy, iz;
    if (t < ncol) {
        ix = nx / 2; iy = (int)(t % ny); iz = (int)(t / ny);
    } else {
        int64_t u = t - ncol;
        if (u >= (int64_t)(nry + nrz) * nxr) return;
        const int r = (int)(u / nxr);
        ix = (int)(u % nxr);                                    // ix < nx/2 when nx is even
        if (r < nry) { iy = ny / 2; iz = r; }
        else { iz = nz / 2; iy = r - nry; if ((ny % 2 == 0) && iy >= ny / 2) ++iy; }
    }
    const int nt = nx + ny + nz;
    const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
    const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
    const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double2 w = make_double2(0.0, 0.0);
    if (g2 > 0.0) {
        const double2 s = sfac(ph, zval, n_ions, nt, nx, ny, ix, iy, iz);
        const double f = vloc_ff(g2, a) * inv_omega;
        w = make_double2(f * s.x, f * s.y);
        const int mx = (nx - ix) % nx, my = (ny - iy) % ny, mz = (nz - iz) % nz;
        const double hx = 2.0 * M_PI * wavenum(mx, nx) / Lx;
        const double hy = 2.0 * M_PI * wavenum(my, ny) / Ly;
        const double hz = 2.0 * M_PI * wavenum(mz, nz) / Lz;
        const double h2 = hx * hx + hy * hy + hz * hz;
        const double2 sm = sfac(ph, zval, n_ions, nt, nx, ny, mx, my, mz);
        const double fm = vloc_ff(h2, a) * inv_omega;
        w = make_double2(0.5 * (w.x + fm * sm.x), 0.5 * (w.y - fm * sm.y));
    }
    out[((int64_t)iz * ny + iy) * nh + ix] = w;
}

int64_t vloc_nyquist_points(int nx, int ny, int nz) {
    const int nh = nx / 2 + 1;
    const int64_t ncol = (nx % 2 == 0) ? (int64_t)ny * nz : 0;
    const int nxr = (nx % 2 == 0) ? nh - 1 : nh;
    const int nry = (ny % 2 == 0) ? nz : 0;
    const int nrz = (nz % 2 == 0) ? ny - (ny % 2 == 0 ? 1 : 0) : 0;
    return ncol + (int64_t)(nry + nrz) * nxr;
}

// ------------------------------------------------------------ Hartree
// tmp(k) = rho(k) 4 pi / G^2 / N (G != 0), for the complex-to-real transform
__global__ void hartree_spectrum_kernel(const double2* __restrict__ rhok, int nx, int ny, int nz,
                                        double Lx, double Ly, double Lz, double inv_n,
                                        double2* __restrict__ out) {
    const int nh = nx / 2 + 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nh * ny * nz) return;
    const int ix = (int)(t % nh);
    const int iy = (int)((t / nh) % ny);
    const int iz = (int)(t / ((int64_t)nh * ny));
    const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
    const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
    const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double2 r = make_double2(0.0, 0.0);
    if (g2 > 0.0) {
        const double k = 4.0 * M_PI / g2 * inv_n;
        r = make_double2(rhok[t].x * k, rhok[t].y * k);
    }
    out[t] = r;
}

// v_Hxc = V_H + v_x, v_x = -(3 rho/pi)^(1/3); optional energy partials
// part[b] = (sum rho V_H, sum e_x(rho), sum rho) per 256-point block
__global__ void __launch_bounds__(256) vhxc_kernel(const double* __restrict__ rho,
                                                   const double* __restrict__ vh, int64_t N,
                                                   double* __restrict__ vhxc,
                                                   double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double eh = 0.0, ex = 0.0, q = 0.0;
    if (i < N) {
        const double r = rho[i];
        q = r;
        const double vx = -cbrt(3.0 * r / M_PI);
        vhxc[i] = vh[i] + vx;
        eh = r * vh[i];
        ex = -(0.75 * cbrt(3.0 / M_PI)) * cbrt(r) * r;
    }
    if (part != nullptr) {
        const double a = block_sum256(eh, sh);
        const double b = block_sum256(ex, sh);
        const double c = block_sum256(q, sh);
        if (threadIdx.x == 0) {
            part[3 * blockIdx.x] = a;
            part[3 * blockIdx.x + 1] = b;
            part[3 * blockIdx.x + 2] = c;
        }
    }
}

// ------------------------------------------------------------ v_eff
template <typename T>
__global__ void veff_kernel(const double* __restrict__ vloc0, const double* __restrict__ vloc1,
                            const double* __restrict__ hn, const double* __restrict__ hn1,
                            const double* __restrict__ hn2, int nhist, int nx, int64_t N,
                            double h, double Lx, double eps, T* __restrict__ veff0,
                            T* __restrict__ veff1, const uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (mask != nullptr && mask[i] == 0) {
        // outside the finite box: +inf tells the stencil to leave H psi zero
        if (veff0 != nullptr) veff0[i] = (T)INFINITY;
        if (veff1 != nullptr) veff1[i] = (T)INFINITY;
        return;
    }
    const double a = hn[i];
    double ext = 0.0;
    if (eps != 0.0) ext = eps * (h * (double)(i % nx) - 0.5 * Lx);
    if (veff0 != nullptr) {
        double v0 = vloc0[i] + a;
        if (eps != 0.0) v0 += ext;
        veff0[i] = (T)v0;
    }
    if (veff1 != nullptr) {
        double vt;
        if (nhist >= 3) vt = (3.0 * a - 3.0 * hn1[i]) + hn2[i];
        else if (nhist == 2) vt = 2.0 * a - hn1[i];
        else vt = a;
        double v1 = vloc1[i] + vt;
        if (eps != 0.0) v1 += ext;
        veff1[i] = (T)v1;
    }
}

// ------------------------------------------------------------ local forces
// F_J = (1/Omega) Re sum_{G in box} conj(rho(G)) (i G) v(G) Z_J exp(-i G.R_J),
// rho(G) = h^3 fft(rho).  With Phi(G) = conj(rho(G)) v(G) h^3/Omega and the
// separable phase exp(-i G.R) = ex(ix) ey(iy) ez(iz), one x-row of the box
// contributes per ion S0 = sum_ix Phi ex, Sx = sum_ix Gx Phi ex, and
//   F_x -= Z Im(Sx ey ez),  F_y -= Z Gy Im(S0 ey ez),  F_z -= Z Gz Im(S0 ey ez).
// A workgroup takes groups of LF_ROWS rows in turn (Phi of the rows staged in
// LDS).  A thread takes one ion (the transposed phase table makes the ion
// loads coalesced) and one of XS interleaved slices of ix, XS = 256 / JW with
// JW = 64, 128 or 256 ion lanes; the force is linear in S0 and Sx, so each
// slice adds its own share and the slices are summed once at the end.
// part[(J * gridDim.x + block) * 3 + c]
constexpr int LF_PASSES = 8;   // up to 8 * 256 ions
constexpr int LF_ROWS = 8;     // x-rows per workgroup pass (reuse of each ex load)

__global__ void __launch_bounds__(256) local_force_kernel(const double2* __restrict__ rhok,
                                                          const double2* __restrict__ phT,
                                                          const double* __restrict__ zval,
                                                          int n_ions, int nx, int ny, int nz,
                                                          double Lx, double Ly, double Lz,
                                                          double a, double scale,
                                                          double* __restrict__ part) {
    extern __shared__ double2 phi[];      // [LF_ROWS][nx]
    __shared__ double red[256 * 3];
    const int nh = nx / 2 + 1;
    const int JW = n_ions <= 64 ? 64 : (n_ions <= 128 ? 128 : 256);
    const int XS = 256 / JW;
    const int jl = threadIdx.x % JW, xs = threadIdx.x / JW;
    const int passes = (n_ions + JW - 1) / JW;
    double acc[LF_PASSES][3];
#pragma unroll
    for (int p = 0; p < LF_PASSES; ++p) acc[p][0] = acc[p][1] = acc[p][2] = 0.0;
    const int rows = ny * nz;
    const int groups = (rows + LF_ROWS - 1) / LF_ROWS;
    for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int r0 = grp * LF_ROWS;
        __syncthreads();
        for (int e = threadIdx.x; e < LF_ROWS * nx; e += blockDim.x) {
            const int rr = e / nx, ix = e - rr * nx;
            const int row = r0 + rr;
            double2 w = make_double2(0.0, 0.0);
            if (row < rows) {
                const int iy = row % ny, iz = row / ny;
                const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
                const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
                const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
                const double g2 = gx * gx + gy * gy + gz * gz;
                if (g2 > 0.0) {
                    double2 rk;
                    if (ix < nh) {
                        rk = rhok[((int64_t)iz * ny + iy) * nh + ix];
                    } else {
                        const int mx = nx - ix, my = (ny - iy) % ny, mz = (nz - iz) % nz;
                        const double2 q = rhok[((int64_t)mz * ny + my) * nh + mx];
                        rk = make_double2(q.x, -q.y);
                    }
                    const double f = vloc_ff(g2, a) * scale;
                    w = make_double2(f * rk.x, -f * rk.y);     // conj(rho) v
                }
            }
            phi[e] = w;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < LF_PASSES; ++p) {
            const int J = p * JW + jl;
            if (p < passes && J < n_ions) {
                double s0r[LF_ROWS], s0i[LF_ROWS], sxr[LF_ROWS], sxi[LF_ROWS];
#pragma unroll
                for (int rr = 0; rr < LF_ROWS; ++rr) s0r[rr] = s0i[rr] = sxr[rr] = sxi[rr] = 0.0;
                for (int ix = xs; ix < nx; ix += XS) {
                    const double2 e = phT[(int64_t)ix * n_ions + J];
                    const double gx = 2.0 * M_PI * wavenum(ix, nx) / Lx;
#pragma unroll
                    for (int rr = 0; rr < LF_ROWS; ++rr) {
                        const double2 w = phi[rr * nx + ix];
                        const double tr = w.x * e.x - w.y * e.y, ti = w.x * e.y + w.y * e.x;
                        s0r[rr] += tr; s0i[rr] += ti;
                        sxr[rr] += gx * tr; sxi[rr] += gx * ti;
                    }
                }
                const double zj = zval[J];
#pragma unroll
                for (int rr = 0; rr < LF_ROWS; ++rr) {
                    const int row = r0 + rr;
                    if (row < rows) {
                        const int iy = row % ny, iz = row / ny;
                        const double gy = 2.0 * M_PI * wavenum(iy, ny) / Ly;
                        const double gz = 2.0 * M_PI * wavenum(iz, nz) / Lz;
                        const double2 ey = phT[(int64_t)(nx + iy) * n_ions + J];
                        const double2 ez = phT[(int64_t)(nx + ny + iz) * n_ions + J];
                        const double2 e = cmul(ey, ez);
                        const double im0 = s0r[rr] * e.y + s0i[rr] * e.x;     // Im(S0 e)
                        const double imx = sxr[rr] * e.y + sxi[rr] * e.x;     // Im(Sx e)
                        acc[p][0] -= zj * imx;
                        acc[p][1] -= zj * gy * im0;
                        acc[p][2] -= zj * gz * im0;
                    }
                }
            }
        }
    }
    // sum the XS slices of each ion (fixed order)
#pragma unroll
    for (int p = 0; p < LF_PASSES; ++p) {
        if (p >= passes) break;
        __syncthreads();
        for (int c = 0; c < 3; ++c) red[threadIdx.x * 3 + c] = acc[p][c];
        __syncthreads();
        const int J = p * JW + threadIdx.x;
        if (threadIdx.x < JW && J < n_ions) {
            for (int c = 0; c < 3; ++c) {
                double v = 0.0;
                for (int k = 0; k < XS; ++k) v += red[(k * JW + threadIdx.x) * 3 + c];
                part[((int64_t)J * gridDim.x + blockIdx.x) * 3 + c] = v;
            }
        }
    }
}

// per ion: F_loc = sum of the local-force partials (fixed order)
__global__ void __launch_bounds__(256) local_force_sum_kernel(const double* __restrict__ part, int nchunk,
                                                              double* __restrict__ floc) {
    __shared__ double sh[4];
    const int J = blockIdx.x;
    for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        for (int k = threadIdx.x; k < nchunk; k += 256) v += part[((int64_t)J * nchunk + k) * 3 + c];
        const double r = block_sum256(v, sh);
        if (threadIdx.x == 0) floc[3 * J + c] = r;
    }
}

// ------------------------------------------------------------ Ewald
// S(G) = sum_K Z_K exp(i G.R_K) for the Ewald reciprocal vectors
__global__ void ewald_sg_kernel(const double* __restrict__ gv, const double* __restrict__ wv, int ng,
                                const double* __restrict__ pos, const double* __restrict__ zval,
                                int n_ions, double2* __restrict__ sg, double* __restrict__ epart) {
    __shared__ double sh[4];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (t < ng) {
        double sr = 0.0, si = 0.0;
        for (int K = 0; K < n_ions; ++K) {
            const double ph = gv[3 * t] * pos[3 * K] + gv[3 * t + 1] * pos[3 * K + 1] +
                              gv[3 * t + 2] * pos[3 * K + 2];
            double sn, cs;
            sincos(ph, &sn, &cs);
            sr += zval[K] * cs;
            si += zval[K] * sn;
        }
        sg[t] = make_double2(sr, si);
        e = wv[t] * (sr * sr + si * si);
    }
    const double s = block_sum256(e, sh);
    if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

int ewald_sg_blocks(int ng) { return ng > 0 ? (ng + 255) / 256 : 1; }

// grid (ion, EW_SPLIT): block (J, sl) takes every EW_SPLIT-th chunk of 256 of
// J's pair/image terms and of the reciprocal vectors; partials
// part[(J * EW_SPLIT + sl) * 4 + {e, fx, fy, fz}], summed by ewald_sum_kernel
constexpr int EW_SPLIT = 8;

__global__ void __launch_bounds__(256) ewald_ion_kernel(const double* __restrict__ pos,
                                                        const double* __restrict__ zval, int n_ions,
                                                        double L, int nmax, double eta, double rc,
                                                        const double* __restrict__ gv,
                                                        const double* __restrict__ wv,
                                                        const double2* __restrict__ sg, int ng,
                                                        double four_pi_over_omega,
                                                        double* __restrict__ part) {
    __shared__ double sh[4];
    const int J = blockIdx.x;
    const int sl = blockIdx.y;
    const int step = blockDim.x * EW_SPLIT;
    const int side = 2 * nmax + 1;
    const int nimg = side * side * side;
    const double rj[3] = {pos[3 * J], pos[3 * J + 1], pos[3 * J + 2]};
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    const double two_eta_pi = 2.0 * eta / sqrt(M_PI);
    for (int64_t t = (int64_t)sl * blockDim.x + threadIdx.x; t < (int64_t)n_ions * nimg; t += step) {
        const int K = (int)(t / nimg);
        const int im = (int)(t % nimg);
        const int ii = im % side - nmax, jj = (im / side) % side - nmax, kk = im / (side * side) - nmax;
        const double dx = rj[0] - pos[3 * K] + ii * L;
        const double dy = rj[1] - pos[3 * K + 1] + jj * L;
        const double dz = rj[2] - pos[3 * K + 2] + kk * L;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > 1e-12 && r < rc) {
            const double zz = zval[J] * zval[K];
            const double ec = erfc(eta * r) / r;
            e += 0.5 * zz * ec;
            const double g = (ec / r + two_eta_pi * exp(-(eta * r) * (eta * r)) / r) / r;
            fx += zz * g * dx;
            fy += zz * g * dy;
            fz += zz * g * dz;
        }
    }
    // reciprocal: F_J = (4 pi Z_J / Omega) sum_G w(G) G Im(exp(i G.R_J) conj(S(G)))
    for (int t = sl * blockDim.x + threadIdx.x; t < ng; t += step) {
        const double ph = gv[3 * t] * rj[0] + gv[3 * t + 1] * rj[1] + gv[3 * t + 2] * rj[2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double2 s = sg[t];
        const double im = sn * s.x - cs * s.y;     // Im(e^{i ph} conj(S))
        const double c = four_pi_over_omega * zval[J] * wv[t] * im;
        fx += c * gv[3 * t];
        fy += c * gv[3 * t + 1];
        fz += c * gv[3 * t + 2];
    }
    const double se = block_sum256(e, sh);
    const double sx = block_sum256(fx, sh);
    const double sy = block_sum256(fy, sh);
    const double sz = block_sum256(fz, sh);
    if (threadIdx.x == 0) {
        double* q = part + ((int64_t)J * EW_SPLIT + sl) * 4;
        q[0] = se;
        q[1] = sx;
        q[2] = sy;
        q[3] = sz;
    }
}

__global__ void ewald_sum_kernel(const double* __restrict__ part, int n_ions, double* __restrict__ f,
                                 double* __restrict__ epart) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= n_ions) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int sl = 0; sl < EW_SPLIT; ++sl)
        for (int c = 0; c < 4; ++c) v[c] += part[((int64_t)J * EW_SPLIT + sl) * 4 + c];
    epart[J] = v[0];
    f[3 * J] = v[1];
    f[3 * J + 1] = v[2];
    f[3 * J + 2] = v[3];
}

size_t ewald_scratch_doubles(int n_ions) { return (size_t)(n_ions > 0 ? n_ions : 1) * EW_SPLIT * 4; }

// ------------------------------------------------------------ ions
__global__ void ions_predict_kernel(const double* __restrict__ pos, const double* __restrict__ vel,
                                    const double* __restrict__ frc, const double* __restrict__ mass,
                                    int n_ions, double dt, int frozen, double* __restrict__ pos1) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n_ions) return;
    if (frozen) { pos1[t] = pos[t]; return; }
    pos1[t] = (pos[t] + vel[t] * dt) + frc[t] * (dt * dt) / (2.0 * mass[t / 3]);
}

// total force F = F_loc + F_NL + F_ion; velocities; the new state becomes current
__global__ void ions_finish_kernel(double* __restrict__ pos, double* __restrict__ vel,
                                   double* __restrict__ frc, const double* __restrict__ pos1,
                                   const double* __restrict__ floc,
                                   const double* __restrict__ fnl, const double* __restrict__ fion,
                                   const double* __restrict__ mass, int n_ions, double dt,
                                   int frozen) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n_ions) return;
    const int J = t / 3;
    const double f1 = (floc[t] + fnl[t]) + fion[t];
    if (!frozen) vel[t] = vel[t] + (frc[t] + f1) * dt / (2.0 * mass[J]);
    pos[t] = pos1[t];
    frc[t] = f1;
}

// ------------------------------------------------------------ misc
__global__ void add_inplace_kernel(double* __restrict__ a, const double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

__global__ void scale_copy_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                  double s, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = s * src[i];
}

__global__ void __launch_bounds__(256) dot_partial_kernel(const double* __restrict__ a,
                                                          const double* __restrict__ b, int64_t n,
                                                          double* __restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double v = i < n ? a[i] * b[i] : 0.0;
    const double s = block_sum256(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// norms[A] = h^3 (sum of the stencil partials + sum of the fix-up partials)
__global__ void __launch_bounds__(256) norm_reduce_kernel(FinalizeArgs a) {
    __shared__ double sh[4];
    const int A = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < a.norm_tiles; k += 256) s += a.norm_part[(int64_t)A * a.norm_tiles + k];
    if (a.fix_part != nullptr)
        for (int k = threadIdx.x; k < a.fix_tiles; k += 256) s += a.fix_part[(int64_t)A * a.fix_tiles + k];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) a.norms[A] = s * a.dv;
}

// Collect the step's diagnostics into rep[] (one block of 256 threads).
// Layout of rep: see ReportSlot.
__global__ void __launch_bounds__(256) report_kernel(FinalizeArgs a) {
    __shared__ double sh[4];
    const int tid = threadIdx.x;
    // norms (already reduced per orbital by norm_reduce_kernel): max |n-1|
    // and finiteness
    double worst = 0.0;
    int bad = 0;
    if (a.norm_part != nullptr) {
        for (int A = tid; A < a.n_orb; A += 256) {
            const double s = a.norms[A];
            if (!isfinite(s)) bad = 1;
            worst = fmax(worst, fabs(s - 1.0));
            if (s > 1.0 + a.norm_tol) bad = 1;
        }
    }
    // block max via shared memory
    __shared__ double mx[256];
    __shared__ int bd[256];
    mx[tid] = worst;
    bd[tid] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            mx[tid] = fmax(mx[tid], mx[tid + o]);
            bd[tid] |= bd[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0 && a.norm_part != nullptr) {
        a.rep[SLOT_NORM_DEV] = mx[0];
        if (bd[0]) a.rep[SLOT_UNSTABLE] = 1.0;
    }
    if (tid == 0 && a.nl_flag != nullptr && *a.nl_flag != 0) a.rep[SLOT_UNSTABLE] = 2.0;
    if (tid == 0 && a.cp_info != nullptr) {
        a.rep[SLOT_CP_ITERS] = a.cp_info[0];
        a.rep[SLOT_CP_RES] = a.cp_info[1];
    }
    __syncthreads();
    if (!a.energy) return;
    // sequential partial sums in fixed order
    double ek = 0.0, eh = 0.0, ex = 0.0, el = 0.0, en = 0.0, ei = 0.0, er = 0.0, q = 0.0;
    for (int64_t k = tid; k < a.kin_n; k += 256) ek += a.kin_part[k];
    for (int64_t k = tid; k < a.hxc_n; k += 256) {
        eh += a.hxc_part[3 * k];
        ex += a.hxc_part[3 * k + 1];
        q += a.hxc_part[3 * k + 2];
    }
    for (int64_t k = tid; k < a.loc_n; k += 256) el += a.loc_part[k];
    for (int k = tid; k < a.n_ions; k += 256) { en += a.enl_part[k]; ei += a.eion_part[k]; }
    for (int k = tid; k < a.erec_n; k += 256) er += a.erec_part[k];
    ek = block_sum256(ek, sh); eh = block_sum256(eh, sh); ex = block_sum256(ex, sh);
    el = block_sum256(el, sh); en = block_sum256(en, sh); ei = block_sum256(ei, sh);
    er = block_sum256(er, sh); q = block_sum256(q, sh);
    double fe = 0.0;
    if (a.fict_part != nullptr)
        for (int64_t k = tid; k < a.fict_n; k += 256) fe += a.fict_part[k];
    fe = block_sum256(fe, sh);
    double ke = 0.0, fmx = 0.0;
    if (tid == 0) {
        for (int J = 0; J < a.n_ions; ++J) {
            const double* v = a.vel + 3 * J;
            ke += 0.5 * a.mass[J] * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
            const double* f = a.frc + 3 * J;
            fmx = fmax(fmx, sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]));
        }
        double* r = a.rep;
        r[SLOT_EKIN] = a.occ * a.dv * ek;
        r[SLOT_ELOC] = a.dv * el;
        r[SLOT_EH] = 0.5 * a.dv * eh;
        r[SLOT_EX] = a.dv * ex;
        r[SLOT_ENL] = en;
        r[SLOT_EION] = ei + a.ewald_rec_scale * er + a.ewald_const;
        r[SLOT_EKS] = ((((r[SLOT_EKIN] + r[SLOT_ELOC]) + r[SLOT_EH]) + r[SLOT_EX]) + r[SLOT_ENL]) +
                      r[SLOT_EION];
        r[SLOT_EIONKIN] = ke;
        r[SLOT_EFICT] = a.fict_part != nullptr ? a.fict_scale * fe : 0.0;
        r[SLOT_ETOT] = (r[SLOT_EKS] + ke) + r[SLOT_EFICT];
        r[SLOT_FMAX] = fmx;
        r[SLOT_CHARGE] = a.dv * q;
    }
}

// ------------------------------------------------------------ launchers
static inline unsigned nb(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_phases(const double* pos, int n_ions, int nx, int ny, int nz, const double L[3],
                         double2* ph, double2* phT, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    const int64_t n = (int64_t)n_ions * (nx + ny + nz);
    phase_kernel<<<nb(n), 256, 0, s>>>(pos, n_ions, nx, ny, nz, L[0], L[1], L[2], ph, phT);
    return hipGetLastError();
}

hipError_t launch_vloc_spectrum(const double2* ph, const double2* phT, const double* zval, int n_ions,
                                int nx, int ny, int nz, const double L[3], double a, double2* out,
                                hipStream_t s) {
    const double inv_omega = 1.0 / (L[0] * L[1] * L[2]);
    if (n_ions == 0) {
        const int64_t n = (int64_t)(nx / 2 + 1) * ny * nz;
        vloc_spectrum_kernel<<<nb(n), 256, 0, s>>>(ph, zval, 0, nx, ny, nz, L[0], L[1], L[2], a, inv_omega, out);
        return hipGetLastError();
    }
    const int rows = ny * nz;
    vloc_rows_kernel<<<(rows + VR_ROWS - 1) / VR_ROWS, 256, 0, s>>>(ph, phT, zval, n_ions, nx, ny, nz, L[0], L[1],
                                                                    L[2], a, inv_omega, out);
    const int64_t nq = vloc_nyquist_points(nx, ny, nz);
    if (nq > 0)
        vloc_nyquist_kernel<<<nb(nq), 256, 0, s>>>(ph, zval, n_ions, nx, ny, nz, L[0], L[1], L[2], a, inv_omega,
                                                   out);
    return hipGetLastError();
}

hipError_t launch_hartree_spectrum(const double2* rhok, int nx, int ny, int nz, const double L[3],
                                   double2* out, hipStream_t s) {
    const int64_t n = (int64_t)(nx / 2 + 1) * ny * nz;
    hartree_spectrum_kernel<<<nb(n), 256, 0, s>>>(rhok, nx, ny, nz, L[0], L[1], L[2],
                                                  1.0 / ((double)nx * ny * nz), out);
    return hipGetLastError();
}

hipError_t launch_vhxc(const double* rho, const double* vh, int64_t N, double* vhxc, double* part,
                       hipStream_t s) {
    vhxc_kernel<<<nb(N), 256, 0, s>>>(rho, vh, N, vhxc, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_veff(const double* vloc0, const double* vloc1, const double* hn, const double* hn1,
                       const double* hn2, int nhist, int nx, int64_t N, double h, double Lx,
                       double eps, T* veff0, T* veff1, const uint8_t* mask, hipStream_t s) {
    veff_kernel<T><<<nb(N), 256, 0, s>>>(vloc0, vloc1, hn, hn1, hn2, nhist, nx, N, h, Lx, eps,
                                         veff0, veff1, mask);
    return hipGetLastError();
}
template hipError_t launch_veff<double>(const double*, const double*, const double*, const double*, const double*, int, int, int64_t, double, double, double, double*, double*, const uint8_t*, hipStream_t);
template hipError_t launch_veff<float>(const double*, const double*, const double*, const double*, const double*, int, int, int64_t, double, double, double, float*, float*, const uint8_t*, hipStream_t);

int local_force_chunks(int64_t N) {
    (void)N;
    return 512;
}

hipError_t launch_local_forces(const double2* rhok, const double2* phT, const double* zval,
                               int n_ions, int nx, int ny, int nz, const double L[3], double h,
                               double a, double* part, double* floc, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    if (n_ions > LF_PASSES * 256) return hipErrorInvalidValue;
    const double scale = h * h * h / (L[0] * L[1] * L[2]);
    local_force_kernel<<<local_force_chunks(0), 256, LF_ROWS * nx * sizeof(double2), s>>>(
        rhok, phT, zval, n_ions, nx, ny, nz, L[0], L[1], L[2], a, scale, part);
    local_force_sum_kernel<<<n_ions, 256, 0, s>>>(part, local_force_chunks(0), floc);
    return hipGetLastError();
}

hipError_t launch_ewald(const EwaldPlan& e, const double* pos, const double* zval, int n_ions,
                        double2* sg, double* erec_part, double* f, double* epart, double* scratch,
                        hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    ewald_sg_kernel<<<ewald_sg_blocks(e.ng), 256, 0, s>>>(e.gv, e.wv, e.ng, pos, zval, n_ions, sg, erec_part);
    ewald_ion_kernel<<<dim3(n_ions, EW_SPLIT), 256, 0, s>>>(pos, zval, n_ions, e.L, e.nmax, e.eta, e.rc, e.gv,
                                                            e.wv, sg, e.ng, 4.0 * M_PI / (e.L * e.L * e.L),
                                                            scratch);
    ewald_sum_kernel<<<nb(n_ions), 256, 0, s>>>(scratch, n_ions, f, epart);
    return hipGetLastError();
}

hipError_t launch_ions_predict(const double* pos, const double* vel, const double* frc,
                               const double* mass, int n_ions, double dt, int frozen, double* pos1,
                               hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    ions_predict_kernel<<<nb(3 * n_ions), 256, 0, s>>>(pos, vel, frc, mass, n_ions, dt, frozen, pos1);
    return hipGetLastError();
}

hipError_t launch_ions_finish(double* pos, double* vel, double* frc, const double* pos1,
                              const double* floc, const double* fnl,
                              const double* fion, const double* mass, int n_ions, double dt,
                              int frozen, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    ions_finish_kernel<<<nb(3 * n_ions), 256, 0, s>>>(pos, vel, frc, pos1, floc, fnl,
                                                      fion, mass, n_ions, dt, frozen);
    return hipGetLastError();
}

hipError_t launch_add(double* a, const double* b, int64_t n, hipStream_t s) {
    add_inplace_kernel<<<nb(n), 256, 0, s>>>(a, b, n);
    return hipGetLastError();
}

hipError_t launch_scale_copy(double* dst, const double* src, double sc, int64_t n, hipStream_t s) {
    scale_copy_kernel<<<nb(n), 256, 0, s>>>(dst, src, sc, n);
    return hipGetLastError();
}

hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* part,
                              hipStream_t s) {
    dot_partial_kernel<<<nb(n), 256, 0, s>>>(a, b, n, part);
    return hipGetLastError();
}

hipError_t launch_report(const FinalizeArgs& a, hipStream_t s) {
    if (a.norm_part != nullptr) norm_reduce_kernel<<<a.n_orb, 256, 0, s>>>(a);
    report_kernel<<<1, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace me

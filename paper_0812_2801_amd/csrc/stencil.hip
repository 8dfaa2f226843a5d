// Fused Hamiltonian-application / Taylor-Horner stage kernel.
//
// H u = -1/2 Lap u + v_eff u + sum_J E_KB p_J c_J(u)   (eq. new_EoM(a))
// with the 8th-order, 25-point finite-difference Laplacian on a periodic
// grid.  In Horner mode one launch performs one stage of the fourth-order
// Taylor exponential (sec. 5.1): out = psi0 + (-i tau/k) H u.
//
// Mapping (2.5-D z-march): one workgroup owns one orbital, a slab of TY
// y-rows spanning the whole x extent, and a chunk of z-planes.  Each thread
// owns PX consecutive x-points of one row.  The nine z-neighbours of the
// thread's points live in a register queue; the current plane of the slab
// plus a 4-row y-halo is staged in LDS, x-periodicity is resolved in LDS.
// The nonlocal part is added in the same pass: the ions whose projector
// sphere reaches the (plane, slab) are read from a bitmask and each point
// reads its projector value from the ion's dense candidate box (written by
// the table build, zero outside the sphere) and adds E_KB p c_J.
#include "common.hpp"
#include "geometry.hpp"

namespace me {

template <typename T, int PX>
__device__ __forceinline__ void load_run(const cx_t<T>* __restrict__ p, cx_t<T>* r) {
    if constexpr (sizeof(cx_t<T>) == 8 && (PX % 2) == 0) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int i = 0; i < PX / 2; ++i) {
            float4 t = q[i];
            r[2 * i] = make_float2(t.x, t.y);
            r[2 * i + 1] = make_float2(t.z, t.w);
        }
    } else {
#pragma unroll
        for (int i = 0; i < PX; ++i) r[i] = p[i];
    }
}

template <typename T, int PX>
__device__ __forceinline__ void store_run(cx_t<T>* __restrict__ p, const cx_t<T>* r) {
    if constexpr (sizeof(cx_t<T>) == 8 && (PX % 2) == 0) {
        float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
        for (int i = 0; i < PX / 2; ++i)
            q[i] = make_float4(r[2 * i].x, r[2 * i].y, r[2 * i + 1].x, r[2 * i + 1].y);
    } else {
#pragma unroll
        for (int i = 0; i < PX; ++i) p[i] = r[i];
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, int PX, int TY, int MODE, bool NORM>
__global__ void __launch_bounds__(1024) stencil_kernel(StencilArgs<T> a) {
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tile = reinterpret_cast<C*>(smem_raw);     // [(TY+8)][nx]
    __shared__ double red[16];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxt = nx / PX;
    const int tid = threadIdx.x;
    const int tx = tid % nxt, ty = tid / nxt;

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ytile = b % a.nyt;
    const int rest = b / a.nyt;
    const int zc = rest % a.nzc;
    const int A = rest / a.nzc;
    const int y0 = ytile * TY;
    const int y = y0 + ty;
    const int x0 = tx * PX;
    const int z0 = zc * a.zchunk;
    const int z1 = z0 + a.zchunk;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t rowoff = (int64_t)y * nx + x0;

    const C* __restrict__ u = a.u + (int64_t)A * a.stride;
    const C* __restrict__ p0 = a.psi0 + (int64_t)A * a.stride;
    C* __restrict__ out = a.out + (int64_t)A * a.stride;

    const T c0 = (T)(3.0 * FD_C0);
    const T cm[4] = {(T)FD_C1, (T)FD_C2, (T)FD_C3, (T)FD_C4};

    C q[9][PX];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int zz = wrap1(z0 - 4 + k, nz);
        load_run<T, PX>(u + zz * plane + rowoff, q[k]);
    }

    double acc = 0.0;
    const int n_halo = 8 * nxt;

    for (int z = z0; z < z1; ++z) {
        load_run<T, PX>(u + wrap1(z + 4, nz) * plane + rowoff, q[8]);
        __syncthreads();
        store_run<T, PX>(tile + (ty + 4) * nx + x0, q[4]);
        for (int j = tid; j < n_halo; j += blockDim.x) {
            const int r = j / nxt;
            const int xr = (j - r * nxt) * PX;
            const int lr = r < 4 ? r : TY + r;
            const int gy = wrap1(r < 4 ? y0 - 4 + r : y0 + TY + (r - 4), ny);
            C tmp[PX];
            load_run<T, PX>(u + z * plane + (int64_t)gy * nx + xr, tmp);
            store_run<T, PX>(tile + lr * nx + xr, tmp);
        }
        __syncthreads();

        // nonlocal contribution of the projectors reaching this (plane, slab)
        C nl[PX];
#pragma unroll
        for (int p = 0; p < PX; ++p) nl[p] = C{(T)0, (T)0};
        if constexpr (MODE != MODE_EXPECT_T) {
            if (a.cnl != nullptr) {
                const uint32_t* mrow = a.mask + ((int64_t)z * a.nyt + ytile) * a.words;
                for (int w = 0; w < a.words; ++w) {
                    uint32_t bits = mrow[w];
                    while (bits) {
                        const int bit = __builtin_ctz(bits);
                        bits &= bits - 1;
                        const int J = w * 32 + bit;
                        int oy = y - a.start[3 * J + 1];
                        if (oy < 0) oy += ny;
                        int oz = z - a.start[3 * J + 2];
                        if (oz < 0) oz += nz;
                        if (oy >= a.side[1] || oz >= a.side[2]) continue;
                        const C cj = a.cnl[(int64_t)J * a.n_orb + A];
                        const T* pb = a.pbox + ((int64_t)J * a.side[2] + oz) * a.side[1] * a.side[0] +
                                      (int64_t)oy * a.side[0];
                        const int sx = a.start[3 * J];
#pragma unroll
                        for (int p = 0; p < PX; ++p) {
                            int ox = x0 + p - sx;
                            if (ox < 0) ox += nx;
                            if (ox < a.side[0]) {
                                const T w8 = pb[ox];
                                nl[p].x += w8 * cj.x;
                                nl[p].y += w8 * cj.y;
                            }
                        }
                    }
                }
            }
        }

        C res[PX];
        const C* trow = tile + (ty + 4) * nx;
        // x-neighbours of the thread's run: one window of PX+8 points
        C wnd[PX + 8];
#pragma unroll
        for (int i = 0; i < PX + 8; ++i) wnd[i] = trow[wrap1(x0 - 4 + i, nx)];
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            const int xx = x0 + p;
            const C ctr = q[4][p];
            T sre = c0 * ctr.x, sim = c0 * ctr.y;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const C xp = wnd[4 + p + m];
                const C xm = wnd[4 + p - m];
                const C yp = trow[m * nx + xx];
                const C ym = trow[-m * nx + xx];
                const C zp = q[4 + m][p];
                const C zm = q[4 - m][p];
                sre += cm[m - 1] * (((xp.x + xm.x) + (yp.x + ym.x)) + (zp.x + zm.x));
                sim += cm[m - 1] * (((xp.y + xm.y) + (yp.y + ym.y)) + (zp.y + zm.y));
            }
            const T tre = a.kin * sre, tim = a.kin * sim;
            if constexpr (MODE == MODE_EXPECT_T) {
                acc += (double)ctr.x * (double)tre + (double)ctr.y * (double)tim;
            } else {
                const T vv = a.v[z * plane + rowoff + p];
                const T hre = tre + vv * ctr.x + nl[p].x;
                const T him = tim + vv * ctr.y + nl[p].y;
                if constexpr (MODE == MODE_APPLY) {
                    res[p] = C{hre, him};
                } else {
                    C base;
                    if constexpr (MODE == MODE_HORNER_FIRST) base = ctr;
                    else base = p0[z * plane + rowoff + p];
                    res[p] = C{base.x - a.alpha * him, base.y + a.alpha * hre};
                }
                if constexpr (NORM)
                    acc += (double)res[p].x * (double)res[p].x + (double)res[p].y * (double)res[p].y;
            }
        }
        if constexpr (MODE != MODE_EXPECT_T) store_run<T, PX>(out + z * plane + rowoff, res);

#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int p = 0; p < PX; ++p) q[k][p] = q[k + 1][p];
    }

    if constexpr (NORM || MODE == MODE_EXPECT_T) {
        acc = wave_sum(acc);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) red[wv] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            const int nw = (blockDim.x + 63) >> 6;
            for (int i = 0; i < nw; ++i) s += red[i];
            a.partial[(int64_t)A * (a.nyt * a.nzc) + zc * a.nyt + ytile] = s;
        }
    }
}

template <typename T, int PX, int TY>
static hipError_t launch_ty(const StencilArgs<T>& a, int mode, bool norm, hipStream_t s) {
    const int nxt = a.nx / PX;
    dim3 block(nxt * TY);
    dim3 grid((unsigned)((int64_t)a.n_orb * a.nyt * a.nzc));
    const size_t lds = (size_t)(TY + 8) * a.nx * sizeof(cx_t<T>);
    switch (mode) {
    case MODE_APPLY:
        stencil_kernel<T, PX, TY, MODE_APPLY, false><<<grid, block, lds, s>>>(a);
        break;
    case MODE_HORNER:
        if (norm) stencil_kernel<T, PX, TY, MODE_HORNER, true><<<grid, block, lds, s>>>(a);
        else stencil_kernel<T, PX, TY, MODE_HORNER, false><<<grid, block, lds, s>>>(a);
        break;
    case MODE_HORNER_FIRST:
        if (norm) stencil_kernel<T, PX, TY, MODE_HORNER_FIRST, true><<<grid, block, lds, s>>>(a);
        else stencil_kernel<T, PX, TY, MODE_HORNER_FIRST, false><<<grid, block, lds, s>>>(a);
        break;
    case MODE_EXPECT_T:
        stencil_kernel<T, PX, TY, MODE_EXPECT_T, false><<<grid, block, lds, s>>>(a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int PX>
static hipError_t launch_px(const StencilArgs<T>& a, int mode, bool norm, int ty, hipStream_t s) {
    switch (ty) {
    case 16: return launch_ty<T, PX, 16>(a, mode, norm, s);
    case 8: return launch_ty<T, PX, 8>(a, mode, norm, s);
    case 4: return launch_ty<T, PX, 4>(a, mode, norm, s);
    case 2: return launch_ty<T, PX, 2>(a, mode, norm, s);
    case 1: return launch_ty<T, PX, 1>(a, mode, norm, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_stencil(const StencilArgs<T>& a, int mode, bool want_norm, int ty,
                          hipStream_t s) {
    constexpr int PXW = sizeof(T) == 4 ? 2 : 1;
    if (a.nx % PXW == 0) return launch_px<T, PXW>(a, mode, want_norm, ty, s);
    return launch_px<T, 1>(a, mode, want_norm, ty, s);
}

template hipError_t launch_stencil<double>(const StencilArgs<double>&, int, bool, int, hipStream_t);
template hipError_t launch_stencil<float>(const StencilArgs<float>&, int, bool, int, hipStream_t);

}  // namespace me

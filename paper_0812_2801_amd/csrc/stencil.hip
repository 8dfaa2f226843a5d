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
// The nonlocal part E_KB sum_J p_J c_J is added afterwards at the projector
// points only (kb.hip), so the stencil loop carries no data-dependent loads.
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

#ifndef STENCIL_NT
#define STENCIL_NT 1
#endif

#ifndef STENCIL_NTLOAD
#define STENCIL_NTLOAD 1
#endif

// streaming load of a run read once (psi0): non-temporal when STENCIL_NTLOAD
template <typename T, int PX>
__device__ __forceinline__ void load_once(const cx_t<T>* __restrict__ p, cx_t<T>* r) {
    if constexpr (STENCIL_NTLOAD) {
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            r[i].x = __builtin_nontemporal_load(&p[i].x);
            r[i].y = __builtin_nontemporal_load(&p[i].y);
        }
    } else {
        load_run<T, PX>(p, r);
    }
}

// streaming store of one output run (non-temporal when STENCIL_NT)
template <typename T, int PX>
__device__ __forceinline__ void store_out(cx_t<T>* __restrict__ p, const cx_t<T>* r) {
#pragma unroll
    for (int i = 0; i < PX; ++i) {
        if constexpr (STENCIL_NT) {
            __builtin_nontemporal_store(r[i].x, &p[i].x);
            __builtin_nontemporal_store(r[i].y, &p[i].y);
        } else {
            p[i] = r[i];
        }
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

template <typename T, int PX>
__device__ __forceinline__ void load_real(const T* __restrict__ p, T* r) {
    if constexpr (sizeof(T) == 4 && PX == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        r[0] = t.x;
        r[1] = t.y;
    } else if constexpr (sizeof(T) == 4 && PX == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        r[0] = t.x; r[1] = t.y; r[2] = t.z; r[3] = t.w;
    } else {
#pragma unroll
        for (int i = 0; i < PX; ++i) r[i] = p[i];
    }
}

#ifndef STENCIL_PD32
#define STENCIL_PD32 1
#endif
#ifndef STENCIL_PD64
#define STENCIL_PD64 1
#endif
#ifndef STENCIL_HLX32
#define STENCIL_HLX32 4
#endif
#ifndef STENCIL_HLX64
#define STENCIL_HLX64 4
#endif
#ifndef STENCIL_WPE
#define STENCIL_WPE 0
#endif
#if STENCIL_WPE > 0
#define STENCIL_ATTR __attribute__((amdgpu_waves_per_eu(STENCIL_WPE)))
#else
#define STENCIL_ATTR
#endif

// Global loads run D planes ahead of the compute; the y-halo rows run HL >= D
// planes ahead.
template <typename T> struct Pipe {
    static constexpr int D = sizeof(T) == 4 ? STENCIL_PD32 : STENCIL_PD64;
    static constexpr int HL = D + (sizeof(T) == 4 ? STENCIL_HLX32 : STENCIL_HLX64);
};


// One workgroup's z-march over planes [z0, z1) of one orbital, rows
// [y0, y0 + rows) (rows <= TY), all x (2.5-D: a register queue of 9 planes per
// thread, the current plane plus a 4-row y-halo in a double-buffered LDS
// tile).  Software pipeline with one barrier per plane: at plane z the thread
// issues the loads of plane z+D (its y-halo run, psi0 and v_eff) and of plane
// z+4+D of its z-queue; plane z+1 is staged into the second LDS buffer after
// plane z has been computed from the first.  The loop issues no load whose
// address depends on another load, so the only waits are for queued planes.
// Offsets inside one orbital are 32-bit.  TYC > 0 fixes TY = rows at compile
// time; TYC == 0 takes them at run time, with HJR halo runs per thread (the
// workgroup needs HJR * blockDim >= 8 * nx / PX).  The LDS tile is sized for
// TY rows; a ragged last tile (rows < TY) places its lower halo right below
// its own rows.  Threads with active == false (beyond nx/PX * rows) only take
// part in the halo loads and the barriers.  Returns this thread's sum for the
// NORM / EXPECT_T partials.
template <typename T, int PX, int TYC, int HJR, int MODE, bool NORM>
__device__ __forceinline__ double zmarch(const cx_t<T>* __restrict__ u, const cx_t<T>* __restrict__ p0,
                                         cx_t<T>* __restrict__ out, const T* __restrict__ v, int nx,
                                         int ny, int nz, int TY, int y0, int rows, int z0, int z1, T kin,
                                         T alpha, cx_t<T>* tiles, bool active) {
    using C = cx_t<T>;
    constexpr int D = Pipe<T>::D;
    constexpr int HL = Pipe<T>::HL;
    constexpr int HJ = TYC > 0 ? (8 + TYC - 1) / TYC : HJR;   // halo runs per thread
    constexpr bool HORNER = MODE == MODE_HORNER;
    constexpr bool NEEDV = MODE != MODE_EXPECT_T;
    if constexpr (TYC > 0) { TY = TYC; rows = TYC; }

    const int nxt = nx / PX;
    const int tid = threadIdx.x;
    const int tx = active ? tid % nxt : 0;
    const int ty = active ? tid / nxt : 0;
    const int y = y0 + ty;
    const int x0 = tx * PX;
    const int plane = nx * ny;
    const int rowoff = y * nx + x0;
    const int tile_elems = (TY + 8) * nx;

    const T c0 = (T)(3.0 * FD_C0);
    const T cm[4] = {(T)FD_C1, (T)FD_C2, (T)FD_C3, (T)FD_C4};

    // LDS offsets of the x-neighbours (periodic wrap resolved once)
    int xo[PX + 8];
#pragma unroll
    for (int i = 0; i < PX + 8; ++i) xo[i] = (ty + 4) * nx + wrap1(x0 - 4 + i, nx);
    const int yo = (ty + 4) * nx + x0;

    // this thread's y-halo jobs: (LDS offset, global row offset)
    const int n_halo = 8 * nxt;
    int h_lds[HJ], h_off[HJ];
    bool h_ok[HJ];
#pragma unroll
    for (int i = 0; i < HJ; ++i) {
        const int j = tid + i * (int)blockDim.x;
        h_ok[i] = j < n_halo;
        const int r = h_ok[i] ? j / nxt : 0;
        const int xr = h_ok[i] ? (j - r * nxt) * PX : 0;
        const int lr = r < 4 ? r : rows + r;
        const int gy = wrap1(r < 4 ? y0 - 4 + r : y0 + rows + (r - 4), ny);
        h_lds[i] = lr * nx + xr;
        h_off[i] = gy * nx + xr;
    }

    // register queues: q = planes z-4 .. z+4+D (the last one in flight),
    // pq/vq = planes z .. z+D, hq = planes z .. z+HL
    C q[9 + D][PX];
    C hq[HL + 1][HJ][PX];
    C pq[D + 1][PX];
    T vq[D + 1][PX];
    if (active) {
#pragma unroll
        for (int k = 0; k < 8 + D; ++k) load_run<T, PX>(u + wrap1(z0 - 4 + k, nz) * plane + rowoff, q[k]);
    }
#pragma unroll
    for (int d = 0; d < HL; ++d) {
        if (z0 + d < z1) {
            const int zo = (z0 + d) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) load_run<T, PX>(u + zo + h_off[i], hq[d][i]);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (z0 + d < z1) {
            const int zo = (z0 + d) * plane;
            if (active) {
                if constexpr (HORNER) load_once<T, PX>(p0 + zo + rowoff, pq[d]);
                if constexpr (NEEDV) load_real<T, PX>(v + zo + rowoff, vq[d]);
            }
        }
    }
    if (active) store_run<T, PX>(tiles + yo, q[4]);
#pragma unroll
    for (int i = 0; i < HJ; ++i)
        if (h_ok[i]) store_run<T, PX>(tiles + h_lds[i], hq[0][i]);
    __syncthreads();

    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int buf = (z - z0) & 1;
        if (z + HL < z1) {
            const int zo = (z + HL) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) load_run<T, PX>(u + zo + h_off[i], hq[HL][i]);
        }
        if (z + D < z1) {
            const int zo = (z + D) * plane;
            if (active) load_run<T, PX>(u + wrap1(z + 4 + D, nz) * plane + rowoff, q[8 + D]);
            if (active) {
                if constexpr (HORNER) load_once<T, PX>(p0 + zo + rowoff, pq[D]);
                if constexpr (NEEDV) load_real<T, PX>(v + zo + rowoff, vq[D]);
            }
        }
        const C* tile = tiles + buf * tile_elems;

        if (active) {
            C res[PX];
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                const C ctr = q[4][p];
                T sre = c0 * ctr.x, sim = c0 * ctr.y;
#pragma unroll
                for (int m = 1; m <= 4; ++m) {
                    const C xp = tile[xo[4 + p + m]];
                    const C xm = tile[xo[4 + p - m]];
                    const C yp = tile[yo + p + m * nx];
                    const C ym = tile[yo + p - m * nx];
                    const C zp = q[4 + m][p];
                    const C zm = q[4 - m][p];
                    sre += cm[m - 1] * (((xp.x + xm.x) + (yp.x + ym.x)) + (zp.x + zm.x));
                    sim += cm[m - 1] * (((xp.y + xm.y) + (yp.y + ym.y)) + (zp.y + zm.y));
                }
                const T tre = kin * sre, tim = kin * sim;
                if constexpr (MODE == MODE_EXPECT_T) {
                    acc += (double)ctr.x * (double)tre + (double)ctr.y * (double)tim;
                } else {
                    const T vv = vq[0][p];
                    // v_eff = +inf marks points outside a finite box, where H psi is zero
                    const bool inb = vv < (T)INFINITY;
                    const T hre = inb ? tre + vv * ctr.x : (T)0;
                    const T him = inb ? tim + vv * ctr.y : (T)0;
                    if constexpr (MODE == MODE_APPLY) {
                        res[p] = C{hre, him};
                    } else if constexpr (MODE == MODE_SCALED) {
                        res[p] = C{-alpha * him, alpha * hre};
                    } else {
                        const C base = HORNER ? pq[0][p] : ctr;
                        res[p] = C{base.x - alpha * him, base.y + alpha * hre};
                    }
                    if constexpr (NORM)
                        acc += (double)res[p].x * (double)res[p].x + (double)res[p].y * (double)res[p].y;
                }
            }
            if constexpr (MODE != MODE_EXPECT_T) store_out<T, PX>(out + z * plane + rowoff, res);
        }

        if (z + 1 < z1) {
            C* nt = tiles + (buf ^ 1) * tile_elems;
            if (active) store_run<T, PX>(nt + yo, q[5]);
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) store_run<T, PX>(nt + h_lds[i], hq[1][i]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8 + D; ++k)
#pragma unroll
            for (int p = 0; p < PX; ++p) q[k][p] = q[k + 1][p];
#pragma unroll
        for (int d = 0; d < HL; ++d)
#pragma unroll
            for (int p = 0; p < PX; ++p)
#pragma unroll
                for (int i = 0; i < HJ; ++i) hq[d][i][p] = hq[d + 1][i][p];
#pragma unroll
        for (int d = 0; d < D; ++d) {
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                if constexpr (HORNER) pq[d][p] = pq[d + 1][p];
                if constexpr (NEEDV) vq[d][p] = vq[d + 1][p];
            }
        }
    }
    return acc;
}

// Whole-row z-march with PY rows per thread: the tile is TY rows, the
// threads cover TY / PY of them, and thread (tx, ty) owns rows y0 + ty + p
// (TY / PY) for p < PY (so a wave's loads stay contiguous rows).  Each owned
// point keeps its own z-queue; the LDS tile, the halo jobs and the pipeline
// are zmarch's.  Taller tiles for the same thread count halve the y-halo rows
// per output row (8 per TY instead of 8 per TY / PY).
template <typename T, int TY, int PY, int MODE, bool NORM>
__device__ __forceinline__ double zmarch_py(const cx_t<T>* __restrict__ u, const cx_t<T>* __restrict__ p0,
                                            cx_t<T>* __restrict__ out, const T* __restrict__ v, int nx,
                                            int ny, int nz, int y0, int z0, int z1, T kin, T alpha,
                                            cx_t<T>* tiles) {
    using C = cx_t<T>;
    constexpr int D = Pipe<T>::D;
    constexpr int HL = Pipe<T>::HL;
    constexpr int TR = TY / PY;                       // thread rows
    constexpr int HJ = (8 + TR - 1) / TR;             // halo runs per thread
    constexpr bool HORNER = MODE == MODE_HORNER;
    constexpr bool NEEDV = MODE != MODE_EXPECT_T;
    static_assert(TY % PY == 0, "rows per thread must divide the tile");

    const int tid = threadIdx.x;
    const int tx = tid % nx;
    const int ty = tid / nx;
    const int plane = nx * ny;
    const int tile_elems = (TY + 8) * nx;

    const T c0 = (T)(3.0 * FD_C0);
    const T cm[4] = {(T)FD_C1, (T)FD_C2, (T)FD_C3, (T)FD_C4};

    int xo[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) xo[i] = (ty + 4) * nx + wrap1(tx - 4 + i, nx);
    int rowoff[PY];
#pragma unroll
    for (int p = 0; p < PY; ++p) rowoff[p] = (y0 + ty + p * TR) * nx + tx;
    const int yo = (ty + 4) * nx + tx;

    const int n_halo = 8 * nx;
    int h_lds[HJ], h_off[HJ];
    bool h_ok[HJ];
#pragma unroll
    for (int i = 0; i < HJ; ++i) {
        const int j = tid + i * (int)blockDim.x;
        h_ok[i] = j < n_halo;
        const int r = h_ok[i] ? j / nx : 0;
        const int xr = h_ok[i] ? j - r * nx : 0;
        const int lr = r < 4 ? r : TY + r;
        const int gy = wrap1(r < 4 ? y0 - 4 + r : y0 + TY + (r - 4), ny);
        h_lds[i] = lr * nx + xr;
        h_off[i] = gy * nx + xr;
    }

    C q[PY][9 + D];
    C hq[HL + 1][HJ];
    C pq[PY][D + 1];
    T vq[PY][D + 1];
#pragma unroll
    for (int p = 0; p < PY; ++p)
#pragma unroll
        for (int k = 0; k < 8 + D; ++k) q[p][k] = u[wrap1(z0 - 4 + k, nz) * plane + rowoff[p]];
#pragma unroll
    for (int d = 0; d < HL; ++d) {
        if (z0 + d < z1) {
            const int zo = (z0 + d) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) hq[d][i] = u[zo + h_off[i]];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (z0 + d < z1) {
            const int zo = (z0 + d) * plane;
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                if constexpr (HORNER) load_once<T, 1>(p0 + zo + rowoff[p], &pq[p][d]);
                if constexpr (NEEDV) vq[p][d] = v[zo + rowoff[p]];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PY; ++p) tiles[yo + p * TR * nx] = q[p][4];
#pragma unroll
    for (int i = 0; i < HJ; ++i)
        if (h_ok[i]) tiles[h_lds[i]] = hq[0][i];
    __syncthreads();

    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int buf = (z - z0) & 1;
        if (z + HL < z1) {
            const int zo = (z + HL) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) hq[HL][i] = u[zo + h_off[i]];
        }
        if (z + D < z1) {
            const int zo = (z + D) * plane;
            const int zq = wrap1(z + 4 + D, nz) * plane;
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                q[p][8 + D] = u[zq + rowoff[p]];
                if constexpr (HORNER) load_once<T, 1>(p0 + zo + rowoff[p], &pq[p][D]);
                if constexpr (NEEDV) vq[p][D] = v[zo + rowoff[p]];
            }
        }
        const C* tile = tiles + buf * tile_elems;
#pragma unroll
        for (int p = 0; p < PY; ++p) {
            const int po = p * TR * nx;
            const C ctr = q[p][4];
            T sre = c0 * ctr.x, sim = c0 * ctr.y;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const C xp = tile[po + xo[4 + m]];
                const C xm = tile[po + xo[4 - m]];
                const C yp = tile[po + yo + m * nx];
                const C ym = tile[po + yo - m * nx];
                const C zp = q[p][4 + m];
                const C zm = q[p][4 - m];
                sre += cm[m - 1] * (((xp.x + xm.x) + (yp.x + ym.x)) + (zp.x + zm.x));
                sim += cm[m - 1] * (((xp.y + xm.y) + (yp.y + ym.y)) + (zp.y + zm.y));
            }
            const T tre = kin * sre, tim = kin * sim;
            if constexpr (MODE == MODE_EXPECT_T) {
                acc += (double)ctr.x * (double)tre + (double)ctr.y * (double)tim;
            } else {
                const T vv = vq[p][0];
                // v_eff = +inf marks points outside a finite box, where H psi is zero
                const bool inb = vv < (T)INFINITY;
                const T hre = inb ? tre + vv * ctr.x : (T)0;
                const T him = inb ? tim + vv * ctr.y : (T)0;
                C res;
                if constexpr (MODE == MODE_APPLY) {
                    res = C{hre, him};
                } else if constexpr (MODE == MODE_SCALED) {
                    res = C{-alpha * him, alpha * hre};
                } else {
                    const C base = HORNER ? pq[p][0] : ctr;
                    res = C{base.x - alpha * him, base.y + alpha * hre};
                }
                if constexpr (NORM) acc += (double)res.x * (double)res.x + (double)res.y * (double)res.y;
                store_out<T, 1>(out + z * plane + rowoff[p], &res);
            }
        }

        if (z + 1 < z1) {
            C* nt = tiles + (buf ^ 1) * tile_elems;
#pragma unroll
            for (int p = 0; p < PY; ++p) nt[yo + p * TR * nx] = q[p][5];
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) nt[h_lds[i]] = hq[1][i];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PY; ++p)
#pragma unroll
            for (int k = 0; k < 8 + D; ++k) q[p][k] = q[p][k + 1];
#pragma unroll
        for (int d = 0; d < HL; ++d)
#pragma unroll
            for (int i = 0; i < HJ; ++i) hq[d][i] = hq[d + 1][i];
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                if constexpr (HORNER) pq[p][d] = pq[p][d + 1];
                if constexpr (NEEDV) vq[p][d] = vq[p][d + 1];
            }
    }
    return acc;
}

// x-tiled z-march: the workgroup owns cols <= TX consecutive points of each
// of rows <= TY consecutive y-rows, starting at (x0, y0) (the last tile of
// a row or column may be narrower), so the tile height no longer falls as
// the rows grow.  The LDS tile has TX + 8 columns: the tile's points at
// columns 4 .. cols+3 and a 4-point x-halo on each side (periodic wrap
// resolved in the global index), and rows + 8 LDS rows as in zmarch.  The
// x-halo runs join the y-halo jobs (8 rows of cols points, then rows runs of
// 4 + 4 points), fetched HL planes ahead like them.  Thread (tx, ty) =
// (tid % TX, tid / TX) owns point (x0 + tx, y0 + ty) when tx < cols and
// ty < rows; the others only load halo jobs and meet the barriers.
// The tile shape (TX, TY) is a run-time value here; the single-system kernel
// passes compile-time constants, the batched kernel each system's shape.  HJ
// halo jobs per thread must cover 8 (cols + rows) jobs with blockDim.x
// threads (blockDim.x >= TX * TY).
template <typename T, int HJ, int MODE, bool NORM>
__device__ __forceinline__ double zmarch_xt(const cx_t<T>* __restrict__ u, const cx_t<T>* __restrict__ p0,
                                            cx_t<T>* __restrict__ out, const T* __restrict__ v, int nx,
                                            int ny, int nz, int TX, int TY, int x0, int cols, int y0, int rows,
                                            int z0, int z1, T kin, T alpha, cx_t<T>* tiles) {
    using C = cx_t<T>;
    constexpr int D = Pipe<T>::D;
    constexpr int HL = Pipe<T>::HL;
    constexpr bool HORNER = MODE == MODE_HORNER;
    constexpr bool NEEDV = MODE != MODE_EXPECT_T;
    const int RS = TX + 8;                                           // LDS row stride
    const int TILE = (TY + 8) * RS;

    const int tid = threadIdx.x;
    const int tx = tid % TX;
    const int ty = tid / TX;
    const bool active = tx < cols && ty < rows;
    const int plane = nx * ny;
    const int rowoff = active ? (y0 + ty) * nx + x0 + tx : 0;
    const int yo = (ty + 4) * RS + tx + 4;

    const T c0 = (T)(3.0 * FD_C0);
    const T cm[4] = {(T)FD_C1, (T)FD_C2, (T)FD_C3, (T)FD_C4};

    // halo jobs: (LDS offset, global offset within a plane)
    const int n_yh = 8 * cols;
    const int n_halo = n_yh + 8 * rows;
    int h_lds[HJ], h_off[HJ];
    bool h_ok[HJ];
#pragma unroll
    for (int i = 0; i < HJ; ++i) {
        const int j = tid + i * (int)blockDim.x;
        h_ok[i] = j < n_halo;
        int lds = 0, gy = 0, gx = 0;
        if (j < n_yh) {
            const int r = j / cols;
            const int c = j - r * cols;
            lds = (r < 4 ? r : rows + r) * RS + c + 4;
            gy = wrap1(r < 4 ? y0 - 4 + r : y0 + rows + (r - 4), ny);
            gx = x0 + c;
        } else if (h_ok[i]) {
            const int jj = j - n_yh;
            const int r = jj >> 3;
            const int c8 = jj & 7;
            lds = (r + 4) * RS + (c8 < 4 ? c8 : cols + c8);
            gy = y0 + r;
            gx = wrap1(c8 < 4 ? x0 - 4 + c8 : x0 + cols + (c8 - 4), nx);
        }
        h_lds[i] = lds;
        h_off[i] = gy * nx + gx;
    }

    C q[9 + D];
    C hq[HL + 1][HJ];
    C pq[D + 1];
    T vq[D + 1];
    if (active) {
#pragma unroll
        for (int k = 0; k < 8 + D; ++k) q[k] = u[wrap1(z0 - 4 + k, nz) * plane + rowoff];
    }
#pragma unroll
    for (int d = 0; d < HL; ++d) {
        if (z0 + d < z1) {
            const int zo = (z0 + d) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) hq[d][i] = u[zo + h_off[i]];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (z0 + d < z1 && active) {
            const int zo = (z0 + d) * plane;
            if constexpr (HORNER) load_once<T, 1>(p0 + zo + rowoff, &pq[d]);
            if constexpr (NEEDV) vq[d] = v[zo + rowoff];
        }
    }
    if (active) tiles[yo] = q[4];
#pragma unroll
    for (int i = 0; i < HJ; ++i)
        if (h_ok[i]) tiles[h_lds[i]] = hq[0][i];
    __syncthreads();

    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int buf = (z - z0) & 1;
        if (z + HL < z1) {
            const int zo = (z + HL) * plane;
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) hq[HL][i] = u[zo + h_off[i]];
        }
        if (z + D < z1 && active) {
            const int zo = (z + D) * plane;
            q[8 + D] = u[wrap1(z + 4 + D, nz) * plane + rowoff];
            if constexpr (HORNER) load_once<T, 1>(p0 + zo + rowoff, &pq[D]);
            if constexpr (NEEDV) vq[D] = v[zo + rowoff];
        }
        const C* tile = tiles + buf * TILE;

        if (active) {
            const C ctr = q[4];
            T sre = c0 * ctr.x, sim = c0 * ctr.y;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const C xp = tile[yo + m];
                const C xm = tile[yo - m];
                const C yp = tile[yo + m * RS];
                const C ym = tile[yo - m * RS];
                const C zp = q[4 + m];
                const C zm = q[4 - m];
                sre += cm[m - 1] * (((xp.x + xm.x) + (yp.x + ym.x)) + (zp.x + zm.x));
                sim += cm[m - 1] * (((xp.y + xm.y) + (yp.y + ym.y)) + (zp.y + zm.y));
            }
            const T tre = kin * sre, tim = kin * sim;
            if constexpr (MODE == MODE_EXPECT_T) {
                acc += (double)ctr.x * (double)tre + (double)ctr.y * (double)tim;
            } else {
                const T vv = vq[0];
                // v_eff = +inf marks points outside a finite box, where H psi is zero
                const bool inb = vv < (T)INFINITY;
                const T hre = inb ? tre + vv * ctr.x : (T)0;
                const T him = inb ? tim + vv * ctr.y : (T)0;
                C res;
                if constexpr (MODE == MODE_APPLY) {
                    res = C{hre, him};
                } else if constexpr (MODE == MODE_SCALED) {
                    res = C{-alpha * him, alpha * hre};
                } else {
                    const C base = HORNER ? pq[0] : ctr;
                    res = C{base.x - alpha * him, base.y + alpha * hre};
                }
                if constexpr (NORM) acc += (double)res.x * (double)res.x + (double)res.y * (double)res.y;
                store_out<T, 1>(out + z * plane + rowoff, &res);
            }
        }

        if (z + 1 < z1) {
            C* nt = tiles + (buf ^ 1) * TILE;
            if (active) nt[yo] = q[5];
#pragma unroll
            for (int i = 0; i < HJ; ++i)
                if (h_ok[i]) nt[h_lds[i]] = hq[1][i];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8 + D; ++k) q[k] = q[k + 1];
#pragma unroll
        for (int d = 0; d < HL; ++d)
#pragma unroll
            for (int i = 0; i < HJ; ++i) hq[d][i] = hq[d + 1][i];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if constexpr (HORNER) pq[d] = pq[d + 1];
            if constexpr (NEEDV) vq[d] = vq[d + 1];
        }
    }
    return acc;
}

// workgroup sum of one double per thread; result in thread 0
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

// One system: a workgroup per (orbital, y-tile, z-chunk).
template <typename T, int PX, int TY, int MODE, bool NORM>
__global__ void __launch_bounds__(1024) STENCIL_ATTR
stencil_kernel(const cx_t<T>* __restrict__ u_all, const cx_t<T>* __restrict__ p0_all,
               cx_t<T>* __restrict__ out_all, const T* __restrict__ v,
               double* __restrict__ partial, StencilArgs<T> a) {
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tiles = reinterpret_cast<C*>(smem_raw);     // 2 x [(TY+8)][nx]
    __shared__ double red[16];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ytile = b % a.nyt;
    const int rest = b / a.nyt;
    const int zc = rest % a.nzc;
    const int A = rest / a.nzc;
    int z0 = zc * a.zchunk, z1 = z0 + a.zchunk;
    if (a.zr != nullptr) {          // finite box: only the planes where the tile's rows meet it
        const int2 r = a.zr[ytile];
        z0 = max(z0, r.x);
        z1 = max(z0, min(z1, r.y));
    }
    const double acc = zmarch<T, PX, TY, 1, MODE, NORM>(
        u_all + (int64_t)A * a.stride, p0_all + (int64_t)A * a.stride, out_all + (int64_t)A * a.stride, v,
        a.nx, a.ny, a.nz, TY, ytile * TY, TY, z0, z1, a.kin, a.alpha, tiles, true);
    if constexpr (NORM || MODE == MODE_EXPECT_T) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(int64_t)A * (a.nyt * a.nzc) + zc * a.nyt + ytile] = s;
    }
}

// One system, whole rows, PY rows per thread: a workgroup of nx * TY / PY
// threads per (orbital, y-tile of TY rows, z-chunk).
template <typename T, int TY, int PY, int MODE, bool NORM>
__global__ void __launch_bounds__(1024) STENCIL_ATTR
stencil_py_kernel(const cx_t<T>* __restrict__ u_all, const cx_t<T>* __restrict__ p0_all,
                  cx_t<T>* __restrict__ out_all, const T* __restrict__ v, double* __restrict__ partial,
                  StencilArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx_t<T>* tiles = reinterpret_cast<cx_t<T>*>(smem_raw);     // 2 x [(TY+8)][nx]
    __shared__ double red[16];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ytile = b % a.nyt;
    const int rest = b / a.nyt;
    const int zc = rest % a.nzc;
    const int A = rest / a.nzc;
    int z0 = zc * a.zchunk, z1 = z0 + a.zchunk;
    if (a.zr != nullptr) {          // finite box: only the planes where the tile's rows meet it
        const int2 r = a.zr[ytile];
        z0 = max(z0, r.x);
        z1 = max(z0, min(z1, r.y));
    }
    const double acc = zmarch_py<T, TY, PY, MODE, NORM>(
        u_all + (int64_t)A * a.stride, p0_all + (int64_t)A * a.stride, out_all + (int64_t)A * a.stride, v,
        a.nx, a.ny, a.nz, ytile * TY, z0, z1, a.kin, a.alpha, tiles);
    if constexpr (NORM || MODE == MODE_EXPECT_T) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(int64_t)A * (a.nyt * a.nzc) + zc * a.nyt + ytile] = s;
    }
}

// One system in x-tiles: a workgroup per (orbital, x-tile, y-tile, z-chunk),
// x-tiles fastest so that neighbouring tiles (which share halo points) run
// close together on one XCD.
template <typename T, int TX, int TY, int MODE, bool NORM>
__global__ void __launch_bounds__(TX * TY) STENCIL_ATTR
stencil_xt_kernel(const cx_t<T>* __restrict__ u_all, const cx_t<T>* __restrict__ p0_all,
                  cx_t<T>* __restrict__ out_all, const T* __restrict__ v, double* __restrict__ partial,
                  StencilArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx_t<T>* tiles = reinterpret_cast<cx_t<T>*>(smem_raw);     // 2 x [(TY+8)][TX+8]
    __shared__ double red[16];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int xt = b % a.nxt;
    int rest = b / a.nxt;
    const int yt = rest % a.nyt;
    rest /= a.nyt;
    const int zc = rest % a.nzc;
    const int A = rest / a.nzc;
    const int x0 = xt * TX, y0 = yt * TY;
    int z0 = zc * a.zchunk, z1 = min(z0 + a.zchunk, a.nz);
    if (a.zr != nullptr) {          // finite box: only the planes where the tile's rows meet it
        const int2 r = a.zr[yt];
        z0 = max(z0, r.x);
        z1 = max(z0, min(z1, r.y));
    }
    constexpr int HJ = (8 * TX + 8 * TY + TX * TY - 1) / (TX * TY);  // halo jobs per thread
    const double acc = zmarch_xt<T, HJ, MODE, NORM>(
        u_all + (int64_t)A * a.stride, p0_all + (int64_t)A * a.stride, out_all + (int64_t)A * a.stride, v,
        a.nx, a.ny, a.nz, TX, TY, x0, min(TX, a.nx - x0), y0, min(TY, a.ny - y0), z0, z1, a.kin, a.alpha, tiles);
    if constexpr (NORM || MODE == MODE_EXPECT_T) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0)
            partial[(int64_t)A * ((int64_t)a.nxt * a.nyt * a.nzc) + ((int64_t)zc * a.nyt + yt) * a.nxt + xt] = s;
    }
}

// Many systems in one persistent launch.  Work items are (system, orbital,
// y-tile, z-slab), numbered system by system in launch order (the host puts
// the largest systems first), y-tiles fastest, then z-slabs, then orbitals.
// Every system's items are cut into QUEUES contiguous slices, and queue q
// holds slice q of every system, in launch order.  A workgroup starts on the
// queue of its XCD (workgroups are dealt to the 8 XCDs round-robin), so
// neighbouring tiles, which share y-halo rows, meet in one L2; when its queue
// is empty it moves on to the next ones.  Each queue is a device counter that
// must be zero at launch.
constexpr int QUEUES = 8;

__device__ __forceinline__ int batch_slice_lo(int count, int q) { return (int)((int64_t)count * q / QUEUES); }

// Without queue counters every workgroup takes one item: block b runs on XCD
// b % 8 and takes the (b / 8)-th item of that XCD's share (each system's
// items split into 8 contiguous slices as for the queues), or none.
template <typename T>
__device__ int batch_item_of_block(const BatchStencilArgs<T>& a) {
    const int q = blockIdx.x % QUEUES;
    int i = blockIdx.x / QUEUES;
    for (int s = 0; s < a.n_sys; ++s) {
        const int cnt = a.sys[s].items;
        const int lo = batch_slice_lo(cnt, q);
        const int len = batch_slice_lo(cnt, q + 1) - lo;
        if (i < len) return a.sys[s].item0 + lo + i;
        i -= len;
    }
    return -1;
}

template <typename T>
__device__ int batch_pull(const BatchStencilArgs<T>& a, int* q_next) {
    while (*q_next < QUEUES) {
        const int q = (blockIdx.x + *q_next) % QUEUES;
        int i = atomicAdd(a.counter + q, 1);
        for (int s = 0; s < a.n_sys; ++s) {
            const int cnt = a.sys[s].items;
            const int lo = batch_slice_lo(cnt, q);
            const int len = batch_slice_lo(cnt, q + 1) - lo;
            if (i < len) return a.sys[s].item0 + lo + i;
            i -= len;
        }
        ++*q_next;   // this queue is exhausted for good
    }
    return -1;
}

// XT: some systems run in x-tiles (tx < nx: items (system, orbital, x-tile,
// y-tile, z-slab), x-tiles fastest), with at most 2 halo jobs per thread.
template <typename T, int HJ, int MODE, bool NORM, bool XT, bool ONE>
__global__ void __launch_bounds__(1024) STENCIL_ATTR batch_stencil_kernel(BatchStencilArgs<T> a) {
    using C = cx_t<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tiles = reinterpret_cast<C*>(smem_raw);
    __shared__ double red[16];
    __shared__ int item_sh;
    int q_next = 0;                           // used by thread 0 only
    for (int round = 0;; ++round) {
        if constexpr (ONE) {                  // one item per workgroup
            if (round > 0) break;
            if (threadIdx.x == 0) item_sh = batch_item_of_block(a);
        } else {
            if (threadIdx.x == 0) item_sh = batch_pull(a, &q_next);
        }
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item < 0) break;
        int s = 0;
        while (s + 1 < a.n_sys && item >= a.sys[s + 1].item0) ++s;
        const BatchSys<T>& d = a.sys[s];
        const int local = item - d.item0;
        const int xtile = local % d.nxt;
        int rest = local / d.nxt;
        const int ytile = rest % d.nyt;
        rest /= d.nyt;
        const int zc = rest % d.nzc;
        const int A = rest / d.nzc;
        const int y0 = ytile * d.ty;
        const int rows = min(d.ty, d.ny - y0);
        const int z0 = zc * d.zchunk;
        const int z1 = min(z0 + d.zchunk, d.nz);
        double acc = 0.0;
        if (XT && d.tx < d.nx) {
            const int x0 = xtile * d.tx;
            acc = zmarch_xt<T, 2, MODE, NORM>(
                d.u + (int64_t)A * d.stride, d.psi0 + (int64_t)A * d.stride, d.out + (int64_t)A * d.stride, d.v,
                d.nx, d.ny, d.nz, d.tx, d.ty, x0, min(d.tx, d.nx - x0), y0, rows, z0, z1, d.kin, d.alpha, tiles);
        } else {
            const bool active = (int)threadIdx.x < d.nx * rows;
            acc = zmarch<T, 1, 0, HJ, MODE, NORM>(
                d.u + (int64_t)A * d.stride, d.psi0 + (int64_t)A * d.stride, d.out + (int64_t)A * d.stride, d.v,
                d.nx, d.ny, d.nz, d.ty, y0, rows, z0, z1, d.kin, d.alpha, tiles, active);
        }
        if constexpr (NORM) {
            const double sum = block_sum(acc, red);
            if (threadIdx.x == 0)
                d.partial[(int64_t)A * ((int64_t)d.nxt * d.nyt * d.nzc) + ((int64_t)zc * d.nyt + ytile) * d.nxt +
                          xtile] = sum;
        }
    }
}

template <typename T, int HJ, bool XT, bool ONE>
static void launch_batch_one(const BatchStencilArgs<T>& a, int mode, bool norm, int block, int grid, size_t lds,
                             hipStream_t s) {
    if (mode == MODE_HORNER) {
        if (norm) batch_stencil_kernel<T, HJ, MODE_HORNER, true, XT, ONE><<<grid, block, lds, s>>>(a);
        else batch_stencil_kernel<T, HJ, MODE_HORNER, false, XT, ONE><<<grid, block, lds, s>>>(a);
    } else {
        if (norm) batch_stencil_kernel<T, HJ, MODE_HORNER_FIRST, true, XT, ONE><<<grid, block, lds, s>>>(a);
        else batch_stencil_kernel<T, HJ, MODE_HORNER_FIRST, false, XT, ONE><<<grid, block, lds, s>>>(a);
    }
}

template <typename T, int HJ, bool XT>
static void launch_batch_hj(const BatchStencilArgs<T>& a, int mode, bool norm, int block, int grid, size_t lds,
                            hipStream_t s) {
    if (a.counter == nullptr) launch_batch_one<T, HJ, XT, true>(a, mode, norm, block, grid, lds, s);
    else launch_batch_one<T, HJ, XT, false>(a, mode, norm, block, grid, lds, s);
}

template <typename T>
hipError_t launch_batch_stencil(const BatchStencilArgs<T>& a, int mode, bool norm, int block, int grid,
                                size_t lds, hipStream_t s) {
    if (mode != MODE_HORNER && mode != MODE_HORNER_FIRST) return hipErrorInvalidValue;
    if (block < 64 || block > 1024 || block % 64 || grid < 1 || a.n_sys < 1 || a.n_sys > MAX_BATCH)
        return hipErrorInvalidValue;
    int hj = 1;
    bool xt = false;
    for (int i = 0; i < a.n_sys; ++i) {
        const BatchSys<T>& d = a.sys[i];
        if (d.ty < 1 || d.nyt * d.ty < d.ny || d.nzc * d.zchunk < d.nz || d.tx < 1 || d.nxt * d.tx < d.nx)
            return hipErrorInvalidValue;
        if (d.tx < d.nx) {          // x-tiles: tile within the block, at most 2 halo jobs per thread
            xt = true;
            if (d.tx * d.ty > block || 8 * (d.tx + d.ty) > 2 * block) return hipErrorInvalidValue;
            if (stencil_xt_lds_bytes(d.tx, d.ty, sizeof(cx_t<T>)) > lds) return hipErrorInvalidValue;
        } else {
            if (d.nxt != 1 || d.nx * d.ty > block) return hipErrorInvalidValue;
            if (8 * d.nx > block) hj = 2;
            if (8 * d.nx > 2 * block) return hipErrorInvalidValue;
            if (2 * (size_t)(d.ty + 8) * d.nx * sizeof(cx_t<T>) > lds) return hipErrorInvalidValue;
        }
    }
    if (xt) {
        if (hj == 1) launch_batch_hj<T, 1, true>(a, mode, norm, block, grid, lds, s);
        else launch_batch_hj<T, 2, true>(a, mode, norm, block, grid, lds, s);
    } else {
        if (hj == 1) launch_batch_hj<T, 1, false>(a, mode, norm, block, grid, lds, s);
        else launch_batch_hj<T, 2, false>(a, mode, norm, block, grid, lds, s);
    }
    return hipGetLastError();
}
template hipError_t launch_batch_stencil<double>(const BatchStencilArgs<double>&, int, bool, int, int, size_t, hipStream_t);
template hipError_t launch_batch_stencil<float>(const BatchStencilArgs<float>&, int, bool, int, int, size_t, hipStream_t);

// attributes the host needs to size a persistent launch
template <typename T>
hipError_t batch_stencil_occupancy(int block, size_t lds, int hj, bool xt, int* wg_per_cu) {
    if (xt) {
        if (hj == 1)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                wg_per_cu, batch_stencil_kernel<T, 1, MODE_HORNER, false, true, false>, block, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            wg_per_cu, batch_stencil_kernel<T, 2, MODE_HORNER, false, true, false>, block, lds);
    }
    if (hj == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            wg_per_cu, batch_stencil_kernel<T, 1, MODE_HORNER, false, false, false>, block, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        wg_per_cu, batch_stencil_kernel<T, 2, MODE_HORNER, false, false, false>, block, lds);
}
template hipError_t batch_stencil_occupancy<double>(int, size_t, int, bool, int*);
template hipError_t batch_stencil_occupancy<float>(int, size_t, int, bool, int*);

// zero n ints (graph-safe replacement for a memset)
__global__ void zero_i32_kernel(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
hipError_t launch_zero_i32(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_i32_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

template <typename T, int PX, int TY>
static hipError_t launch_ty(const StencilArgs<T>& a, int mode, bool norm, hipStream_t s) {
    const int nxt = a.nx / PX;
    dim3 block(nxt * TY);
    dim3 grid((unsigned)((int64_t)a.n_orb * a.nyt * a.nzc));
    const size_t lds = 2 * (size_t)(TY + 8) * a.nx * sizeof(cx_t<T>);
#define ME_STENCIL(M, NORM) \
    stencil_kernel<T, PX, TY, M, NORM><<<grid, block, lds, s>>>(a.u, a.psi0, a.out, a.v, a.partial, a)
    switch (mode) {
    case MODE_APPLY: ME_STENCIL(MODE_APPLY, false); break;
    case MODE_HORNER:
        if (norm) ME_STENCIL(MODE_HORNER, true); else ME_STENCIL(MODE_HORNER, false);
        break;
    case MODE_HORNER_FIRST:
        if (norm) ME_STENCIL(MODE_HORNER_FIRST, true); else ME_STENCIL(MODE_HORNER_FIRST, false);
        break;
    case MODE_EXPECT_T: ME_STENCIL(MODE_EXPECT_T, false); break;
    case MODE_SCALED: ME_STENCIL(MODE_SCALED, false); break;
    default: return hipErrorInvalidValue;
    }
#undef ME_STENCIL
    return hipGetLastError();
}

template <typename T, int TX, int TY>
static hipError_t launch_xt(const StencilArgs<T>& a, int mode, bool norm, hipStream_t s) {
    dim3 block(TX * TY);
    dim3 grid((unsigned)((int64_t)a.n_orb * a.nxt * a.nyt * a.nzc));
    const size_t lds = stencil_xt_lds_bytes(TX, TY, sizeof(cx_t<T>));
#define ME_STENCIL(M, NORM) \
    stencil_xt_kernel<T, TX, TY, M, NORM><<<grid, block, lds, s>>>(a.u, a.psi0, a.out, a.v, a.partial, a)
    switch (mode) {
    case MODE_APPLY: ME_STENCIL(MODE_APPLY, false); break;
    case MODE_HORNER:
        if (norm) ME_STENCIL(MODE_HORNER, true); else ME_STENCIL(MODE_HORNER, false);
        break;
    case MODE_HORNER_FIRST:
        if (norm) ME_STENCIL(MODE_HORNER_FIRST, true); else ME_STENCIL(MODE_HORNER_FIRST, false);
        break;
    case MODE_EXPECT_T: ME_STENCIL(MODE_EXPECT_T, false); break;
    case MODE_SCALED: ME_STENCIL(MODE_SCALED, false); break;
    default: return hipErrorInvalidValue;
    }
#undef ME_STENCIL
    return hipGetLastError();
}

template <typename T, int TY, int PY>
static hipError_t launch_py(const StencilArgs<T>& a, int mode, bool norm, hipStream_t s) {
    dim3 block(a.nx * TY / PY);
    dim3 grid((unsigned)((int64_t)a.n_orb * a.nyt * a.nzc));
    const size_t lds = 2 * (size_t)(TY + 8) * a.nx * sizeof(cx_t<T>);
#define ME_STENCIL(M, NORM) \
    stencil_py_kernel<T, TY, PY, M, NORM><<<grid, block, lds, s>>>(a.u, a.psi0, a.out, a.v, a.partial, a)
    switch (mode) {
    case MODE_APPLY: ME_STENCIL(MODE_APPLY, false); break;
    case MODE_HORNER:
        if (norm) ME_STENCIL(MODE_HORNER, true); else ME_STENCIL(MODE_HORNER, false);
        break;
    case MODE_HORNER_FIRST:
        if (norm) ME_STENCIL(MODE_HORNER_FIRST, true); else ME_STENCIL(MODE_HORNER_FIRST, false);
        break;
    case MODE_EXPECT_T: ME_STENCIL(MODE_EXPECT_T, false); break;
    case MODE_SCALED: ME_STENCIL(MODE_SCALED, false); break;
    default: return hipErrorInvalidValue;
    }
#undef ME_STENCIL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const StencilArgs<T>& a, int mode, bool want_norm, int ty, int px,
                          hipStream_t s) {
    if (px != 1) return hipErrorInvalidValue;
    if (a.py == 2 && a.tx == a.nx) {   // whole rows, two rows per thread
        if (a.nyt * ty != a.ny || (int64_t)a.nx * ty / 2 > 1024) return hipErrorInvalidValue;
        if (ty == 16) return launch_py<T, 16, 2>(a, mode, want_norm, s);
        if (ty == 8) return launch_py<T, 8, 2>(a, mode, want_norm, s);
        return hipErrorInvalidValue;
    }
    if (a.tx != a.nx) {             // x-tiles: the tile shape is one of the compiled ones
        if (a.tx < 1 || a.nxt * a.tx < a.nx || a.nyt * ty < a.ny) return hipErrorInvalidValue;
        if (a.tx == 64 && ty == 12) return launch_xt<T, 64, 12>(a, mode, want_norm, s);
        if (a.tx == 48 && ty == 16) return launch_xt<T, 48, 16>(a, mode, want_norm, s);
        if (a.tx == 32 && ty == 24) return launch_xt<T, 32, 24>(a, mode, want_norm, s);
        if (a.tx == 16 && ty == 8) return launch_xt<T, 16, 8>(a, mode, want_norm, s);    // small grids, tests
        return hipErrorInvalidValue;
    }
    switch (ty) {
    case 16: return launch_ty<T, 1, 16>(a, mode, want_norm, s);
    case 8: return launch_ty<T, 1, 8>(a, mode, want_norm, s);
    case 4: return launch_ty<T, 1, 4>(a, mode, want_norm, s);
    case 2: return launch_ty<T, 1, 2>(a, mode, want_norm, s);
    case 1: return launch_ty<T, 1, 1>(a, mode, want_norm, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stencil<double>(const StencilArgs<double>&, int, bool, int, int, hipStream_t);
template hipError_t launch_stencil<float>(const StencilArgs<float>&, int, bool, int, int, hipStream_t);

}  // namespace me

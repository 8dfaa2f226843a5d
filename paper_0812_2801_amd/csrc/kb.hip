// Gaussian s-channel Kleinman-Bylander projector: per-ion point tables,
// the contraction c_JA = h^3 sum_k p_J(r_k) psi_A(r_k) and the nonlocal
// forces / energy.  The scatter E_KB sum_J p_J c_JA is added at the
// projector points after each stencil pass, by kb_fixup_kernel or, together
// with the next stage's contraction, by kb_fixup_gather_kernel.
#include "common.hpp"
#include "geometry.hpp"

namespace me {

// ------------------------------------------------------------ tables
// One workgroup per ion.  Candidates: per axis the 2m+2 points
// floor(R/h)-m .. floor(R/h)+m+1 (all n points when 2m+2 >= n), enumerated
// with x fastest; those strictly inside the cutoff are compacted in
// candidate order with a ballot prefix sum, so the table is deterministic.
template <typename T>
__global__ void __launch_bounds__(256) kb_tables_kernel(const double* __restrict__ pos,
                                                        int nx, int ny, int nz, KbGeom g, int m,
                                                        int32_t* __restrict__ idx, T* __restrict__ pv,
                                                        int32_t* __restrict__ count, int kcap) {
    __shared__ int wsum[4];
    __shared__ int base_off;
    const int J = blockIdx.x;
    const double rx = pos[3 * J], ry = pos[3 * J + 1], rz = pos[3 * J + 2];
    const int n3[3] = {nx, ny, nz};
    const double r3[3] = {rx, ry, rz};
    int side[3], start[3];
    for (int a = 0; a < 3; ++a) {
        side[a] = 2 * m + 2;
        if (side[a] >= n3[a]) {
            side[a] = n3[a];
            start[a] = 0;
        } else {
            const double w = r3[a] - g.L[a] * floor(r3[a] / g.L[a]);  // into [0, L)
            start[a] = (int)floor(w / g.h) - m;
        }
    }
    const int total = min(side[0] * side[1] * side[2], kcap);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) base_off = 0;
    __syncthreads();
    for (int c0 = 0; c0 < total; c0 += 256) {
        const int c = c0 + tid;
        bool inside = false;
        int lin = 0;
        double d2 = 0.0;
        if (c < total) {
            const int ox = c % side[0];
            const int oy = (c / side[0]) % side[1];
            const int oz = c / (side[0] * side[1]);
            int gx = (start[0] + ox) % nx; if (gx < 0) gx += nx;
            int gy = (start[1] + oy) % ny; if (gy < 0) gy += ny;
            int gz = (start[2] + oz) % nz; if (gz < 0) gz += nz;
            double dx, dy, dz;
            d2 = kb_d2(g, gx, gy, gz, rx, ry, rz, dx, dy, dz);
            inside = d2 < g.rcut2;
            lin = (gz * ny + gy) * nx + gx;
        }
        const unsigned long long bal = __ballot(inside);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int off = base_off;
        for (int i = 0; i < wv; ++i) off += wsum[i];
        if (inside) {
            const int k = off + before;
            if (k < kcap) {
                idx[(int64_t)J * kcap + k] = lin;
                pv[(int64_t)J * kcap + k] = (T)kb_value(g, d2);
            }
        }
        __syncthreads();
        if (tid == 0) base_off += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (tid == 0) count[J] = base_off < kcap ? base_off : kcap;
}

// ------------------------------------------------------------ point lists
// The union of the projector spheres, by grid point.  Slots are numbered in
// increasing grid index; the (ion, value) pairs of a slot are sorted by ion,
// so every sum over them runs in a fixed order.
__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void nl_mark_kernel(const int32_t* __restrict__ idx, const int32_t* __restrict__ count,
                               int kcap, int32_t* __restrict__ map) {
    const int J = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count[J]) map[idx[(int64_t)J * kcap + k]] = 0;
}

constexpr int SCAN_B = 1024;     // grid points per numbering block (256 threads x 4)

__global__ void __launch_bounds__(256) nl_count_kernel(const int32_t* __restrict__ map, int64_t N,
                                                       int32_t* __restrict__ blk) {
    __shared__ int ws[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + threadIdx.x * 4;
    int c = 0;
    for (int i = 0; i < 4; ++i)
        if (base + i < N && map[base + i] == 0) ++c;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// exclusive scan of the block counts (one workgroup); total into *nslots
__global__ void __launch_bounds__(256) nl_scan_blocks_kernel(int32_t* __restrict__ blk, int nblk,
                                                             int32_t* __restrict__ nslots) {
    __shared__ int carry;
    __shared__ int ws[4];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        const int i = b0 + threadIdx.x;
        const int v = i < nblk ? blk[i] : 0;
        int x = v;                                   // inclusive scan within the wave
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) ws[wv] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wv; ++w) before += ws[w];
        if (i < nblk) blk[i] = before + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) *nslots = carry;
}

__global__ void __launch_bounds__(256) nl_number_kernel(int32_t* __restrict__ map, int64_t N,
                                                        const int32_t* __restrict__ blk,
                                                        int32_t* __restrict__ pts) {
    __shared__ int ws[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + threadIdx.x * 4;
    int f[4], c = 0;
    for (int i = 0; i < 4; ++i) {
        f[i] = (base + i < N && map[base + i] == 0) ? 1 : 0;
        c += f[i];
    }
    int x = c;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wv] = x;
    __syncthreads();
    int slot = blk[blockIdx.x] + x - c;
    for (int w = 0; w < wv; ++w) slot += ws[w];
    for (int i = 0; i < 4; ++i)
        if (f[i]) {
            map[base + i] = slot;
            pts[slot] = (int32_t)(base + i);
            ++slot;
        }
}

template <typename T>
__global__ void nl_fill_kernel(const int32_t* __restrict__ idx, const T* __restrict__ pv,
                               const int32_t* __restrict__ count, int kcap,
                               const int32_t* __restrict__ map, int32_t* __restrict__ cnt,
                               int32_t* __restrict__ ion, T* __restrict__ pl, int64_t ucap,
                               int32_t* __restrict__ flag) {
    const int J = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count[J]) return;
    const int64_t e = (int64_t)J * kcap + k;
    const int s = map[idx[e]];
    const int pos = atomicAdd(&cnt[s], 1);
    if (pos < NL_KMAX) {
        ion[pos * ucap + s] = J;
        pl[pos * ucap + s] = pv[e];
    } else {
        atomicOr(flag, 1);
    }
}

template <typename T>
__global__ void nl_sort_kernel(const int32_t* __restrict__ nslots, int32_t* __restrict__ cnt,
                               int32_t* __restrict__ ion, T* __restrict__ pl, int64_t ucap) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= *nslots) return;
    const int n = min(cnt[s], NL_KMAX);
    cnt[s] = n;
    // the slot's pairs into registers, insertion sort by ion, back
    int ji[NL_KMAX];
    T jp[NL_KMAX];
    for (int i = 0; i < n; ++i) {
        ji[i] = ion[i * ucap + s];
        jp[i] = pl[i * ucap + s];
    }
    for (int i = 1; i < n; ++i) {
        const int kj = ji[i];
        const T kp = jp[i];
        int j = i - 1;
        while (j >= 0 && ji[j] > kj) {
            ji[j + 1] = ji[j];
            jp[j + 1] = jp[j];
            --j;
        }
        ji[j + 1] = kj;
        jp[j + 1] = kp;
    }
    for (int i = 0; i < n; ++i) {
        ion[i * ucap + s] = ji[i];
        pl[i * ucap + s] = jp[i];
    }
}

// which table points are covered by more than one sphere, and the list of
// such slots (their order is free: each is fixed on its own)
__global__ void nl_overlap_points_kernel(const int32_t* __restrict__ idx, const int32_t* __restrict__ count,
                                         int kcap, const int32_t* __restrict__ map,
                                         const int32_t* __restrict__ cnt, uint8_t* __restrict__ ov) {
    const int J = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count[J]) {
        const int64_t e = (int64_t)J * kcap + k;
        ov[e] = cnt[map[idx[e]]] > 1 ? 1 : 0;
    }
}

__global__ void nl_overlap_slots_kernel(const int32_t* __restrict__ nslots, const int32_t* __restrict__ cnt,
                                        int32_t* __restrict__ ovl, int32_t* __restrict__ ovn) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < *nslots && cnt[s] > 1) ovl[atomicAdd(ovn, 1)] = s;
}

template <typename T>
hipError_t launch_kb_tables(const double* pos, int n_ions, int nx, int ny, int nz,
                            const KbGeom& g, KbTables t, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t nblk = (N + SCAN_B - 1) / SCAN_B;
    kb_tables_kernel<T><<<n_ions, 256, 0, s>>>(pos, nx, ny, nz, g, t.m, t.idx,
                                               reinterpret_cast<T*>(t.p), t.count, t.kcap);
    fill_i32_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(t.map, N, -1);
    fill_i32_kernel<<<(unsigned)((t.ucap + 255) / 256), 256, 0, s>>>(t.cnt, t.ucap, 0);
    fill_i32_kernel<<<1, 64, 0, s>>>(t.flag, 1, 0);
    dim3 eg((t.kcap + 255) / 256, n_ions);
    nl_mark_kernel<<<eg, 256, 0, s>>>(t.idx, t.count, t.kcap, t.map);
    nl_count_kernel<<<(unsigned)nblk, 256, 0, s>>>(t.map, N, t.blk);
    nl_scan_blocks_kernel<<<1, 256, 0, s>>>(t.blk, (int)nblk, t.nslots);
    nl_number_kernel<<<(unsigned)nblk, 256, 0, s>>>(t.map, N, t.blk, t.pts);
    nl_fill_kernel<T><<<eg, 256, 0, s>>>(t.idx, reinterpret_cast<const T*>(t.p), t.count, t.kcap, t.map,
                                         t.cnt, t.ion, reinterpret_cast<T*>(t.pl), t.ucap, t.flag);
    nl_sort_kernel<T><<<(unsigned)((t.ucap + 255) / 256), 256, 0, s>>>(t.nslots, t.cnt, t.ion,
                                                                       reinterpret_cast<T*>(t.pl), t.ucap);
    fill_i32_kernel<<<1, 64, 0, s>>>(t.ovn, 1, 0);
    if (t.novc > 0) fill_i32_kernel<<<(unsigned)((t.novc + 255) / 256), 256, 0, s>>>(t.ovc, t.novc, 0);
    nl_overlap_points_kernel<<<eg, 256, 0, s>>>(t.idx, t.count, t.kcap, t.map, t.cnt, t.ov);
    nl_overlap_slots_kernel<<<(unsigned)((t.ucap + 255) / 256), 256, 0, s>>>(t.nslots, t.cnt, t.ovl, t.ovn);
    return hipGetLastError();
}

// out_A(r) += g * sum_k pl * cnl[ion*n_orb + A] over the slots of the
// projector spheres.  Grid (ceil(ucap/256), ceil(n_orb/FIX_OB)): a thread
// takes one slot (its pairs read once) and updates FIX_OB orbitals there;
// neighbouring lanes take neighbouring slots.  With dnorm, the change of each
// orbital's squared norm, sum |out + d|^2 - |out|^2, is returned per block.
template <typename T>
__global__ void __launch_bounds__(256) kb_fixup_kernel(cx_t<T>* __restrict__ out, int64_t stride,
                                                       int n_orb, const int32_t* __restrict__ nslots,
                                                       const int32_t* __restrict__ pts,
                                                       const int32_t* __restrict__ cnt,
                                                       const int32_t* __restrict__ ion,
                                                       const T* __restrict__ pl, int64_t ucap,
                                                       const cx_t<T>* __restrict__ cnl, T gr, T gi,
                                                       double* __restrict__ dnorm) {
    __shared__ double red[4][FIX_OB];
    const int A0 = blockIdx.y * FIX_OB;
    const int na = min(FIX_OB, n_orb - A0);
    const int ns = *nslots;
    double dn[FIX_OB];
#pragma unroll
    for (int j = 0; j < FIX_OB; ++j) dn[j] = 0.0;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) {
        const int n = cnt[s];
        const int64_t r = pts[s];
        int jj[NL_KMAX];
        T ww[NL_KMAX];
        for (int k = 0; k < n; ++k) {
            jj[k] = ion[k * ucap + s];
            ww[k] = pl[k * ucap + s];
        }
#pragma unroll
        for (int j = 0; j < FIX_OB; ++j) {
            if (j < na) {
                const int A = A0 + j;
                T sr = 0, si = 0;
                for (int k = 0; k < n; ++k) nl_acc<T>(ww[k], cnl[(int64_t)jj[k] * n_orb + A], sr, si);
                cx_t<T>* o = out + (int64_t)A * stride + r;
                const cx_t<T> old = *o;
                const cx_t<T> val = nl_add<T>(old, sr, si, gr, gi);
                *o = val;
                if (dnorm != nullptr)
                    dn[j] += ((double)val.x * val.x + (double)val.y * val.y) -
                             ((double)old.x * old.x + (double)old.y * old.y);
            }
        }
    }
    if (dnorm != nullptr) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int j = 0; j < FIX_OB; ++j) {
            double v = dn[j];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) red[wv][j] = v;
        }
        __syncthreads();
        if (threadIdx.x < na)
            dnorm[(int64_t)(A0 + threadIdx.x) * gridDim.x + blockIdx.x] =
                ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
}

template <typename T>
hipError_t launch_kb_fixup(cx_t<T>* out, int64_t stride, int n_orb, KbTables t,
                           const cx_t<T>* cnl, double gr, double gi, double* dnorm, hipStream_t s) {
    dim3 grid(fixup_blocks(t.ucap), (n_orb + FIX_OB - 1) / FIX_OB);
    kb_fixup_kernel<T><<<grid, 256, 0, s>>>(out, stride, n_orb, t.nslots, t.pts, t.cnt, t.ion,
                                            reinterpret_cast<const T*>(t.pl), t.ucap, cnl, (T)gr, (T)gi, dnorm);
    return hipGetLastError();
}

// ------------------------------------------------------------ contraction
template <typename T>
__device__ __forceinline__ T wsum_t(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// one wave per (ion, orbital); four orbitals of one ion per workgroup.  Lane
// l takes points l, l+64, ..., l+448 of each 512-point block of the ion's
// list; the block's index and value loads, then its orbital loads, are all
// issued before any sum (the loads of a point depend on its index load, so a
// loop that waited point by point would pay a round trip per 64 points).
// The sums run in the order of the points, as a strided loop would.
constexpr int GATHER_U = 8;

template <typename T>
__global__ void __launch_bounds__(256) kb_gather_kernel(const cx_t<T>* __restrict__ u, int64_t stride,
                                                        int n_orb, const int32_t* __restrict__ idx,
                                                        const T* __restrict__ pv,
                                                        const int32_t* __restrict__ count, int kcap,
                                                        T scale, cx_t<T>* __restrict__ cnl) {
    const int J = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int A = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (A >= n_orb) return;
    const int K = count[J];
    const int32_t* ix = idx + (int64_t)J * kcap;
    const T* pp = pv + (int64_t)J * kcap;
    const cx_t<T>* ua = u + (int64_t)A * stride;
    T re = 0, im = 0;
    for (int k0 = 0; k0 < K; k0 += 64 * GATHER_U) {
        int id[GATHER_U];
        T w[GATHER_U];
#pragma unroll
        for (int i = 0; i < GATHER_U; ++i) {
            const int k = k0 + lane + 64 * i;
            id[i] = k < K ? ix[k] : -1;
            w[i] = k < K ? pp[k] : (T)0;
        }
        cx_t<T> z[GATHER_U];
#pragma unroll
        for (int i = 0; i < GATHER_U; ++i) z[i] = id[i] >= 0 ? ua[id[i]] : cx_t<T>{(T)0, (T)0};
#pragma unroll
        for (int i = 0; i < GATHER_U; ++i) {
            re += w[i] * z[i].x;
            im += w[i] * z[i].y;
        }
    }
    re = wsum_t(re);
    im = wsum_t(im);
    if (lane == 0) cnl[(int64_t)J * n_orb + A] = cx_t<T>{scale * re, scale * im};
}

template <typename T>
hipError_t launch_kb_gather(const cx_t<T>* u, int64_t stride, int n_orb, int n_ions,
                            KbTables t, double ekb_h3, cx_t<T>* cnl, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    dim3 grid((n_orb + 3) / 4, n_ions);
    kb_gather_kernel<T><<<grid, 256, 0, s>>>(u, stride, n_orb, t.idx, reinterpret_cast<const T*>(t.p),
                                             t.count, t.kcap, (T)ekb_h3, cnl);
    return hipGetLastError();
}

// The fix-up of one stage fused with the gather of the next: the structure
// of kb_gather_kernel (a wave per (ion, orbital), 512-point blocks whose
// loads are issued before the sums), each point's value fixed before it is
// summed.  A point of one sphere only is fixed in place here (its pass is
// the only one that touches it); a point shared with other spheres gets
// its fixed value computed from the slot's (ion, value) pairs for the sum,
// and is written by the last workgroup of its orbital group to finish (the
// workgroups of one orbital group, one per ion, count themselves in ovc):
// by then every pass has read the shared points' unfixed values.  The
// fix-up arithmetic is kb_fixup_kernel's (nl_acc / nl_add), the sums are
// kb_gather_kernel's.

// the shared points of orbitals A0 .. A0 + na - 1, by the threads of one
// workgroup (kb_fixup_kernel's arithmetic), then the group's counter reset
template <typename T>
__device__ void fix_shared_points(cx_t<T>* __restrict__ out, int64_t stride, int n_orb, int A0, int na,
                                  const int32_t* __restrict__ ovl, const int32_t* __restrict__ ovn,
                                  const int32_t* __restrict__ pts, const int32_t* __restrict__ cnt,
                                  const int32_t* __restrict__ ion, const T* __restrict__ pl, int64_t ucap,
                                  const cx_t<T>* __restrict__ cnl, T gr, T gi, int32_t* ovc_g) {
    const int nov = *ovn;
    for (int e = threadIdx.x; e < nov * na; e += blockDim.x) {
        const int sl = ovl[e / na];
        const int A = A0 + e % na;
        const int n = min(cnt[sl], NL_KMAX);
        T sr = 0, si = 0;
        for (int q = 0; q < n; ++q)
            nl_acc<T>(pl[q * ucap + sl], cnl[(int64_t)ion[q * ucap + sl] * n_orb + A], sr, si);
        cx_t<T>* o = out + (int64_t)A * stride + pts[sl];
        *o = nl_add<T>(*o, sr, si, gr, gi);
    }
    if (threadIdx.x == 0) atomicExch(ovc_g, 0);
}

// true in every thread of the workgroup that finishes its orbital group last
// (members workgroups per group).  A workgroup counts itself after every
// load of its points has returned (their values are in its sums), so the
// last one's stores come after all the group's reads.  No other ordering is
// needed (the shared points and c_JA are not written by the other
// workgroups), so the count is a relaxed device-scope atomic and no fence is
// taken: a device-scope fence writes back or invalidates the XCD's L2.
__device__ __forceinline__ bool last_of_group(int32_t* ovc_g, int members, int* flag) {
    __syncthreads();
    if (threadIdx.x == 0) *flag = atomicAdd(ovc_g, 1) == members - 1;
    __syncthreads();
    return *flag != 0;
}

// one workgroup of the fused pass: orbitals 4 ORB grp .. (ORB consecutive
// per wave) of ion J; n_ions workgroups per orbital group
template <typename T, int ORB>
__device__ __forceinline__ void fixup_gather_block(cx_t<T>* __restrict__ out, int64_t stride, int n_orb, int n_ions,
                                                   const KbTables& t, const cx_t<T>* __restrict__ cnl_in, T gr, T gi,
                                                   T scale, cx_t<T>* __restrict__ cnl_out, int J, int grp,
                                                   int* last) {
    const T* pv = reinterpret_cast<const T*>(t.p);
    const T* pl = reinterpret_cast<const T*>(t.pl);
    const int64_t ucap = t.ucap;
    const int lane = threadIdx.x & 63;
    const int G = 4 * ORB;                         // orbitals of the workgroup: ORB consecutive per wave
    const int A0 = grp * G + (threadIdx.x >> 6) * ORB;
    if (A0 < n_orb) {
        const int K = t.count[J];
        const int32_t* ix = t.idx + (int64_t)J * t.kcap;
        const T* pp = pv + (int64_t)J * t.kcap;
        const uint8_t* po = t.ov + (int64_t)J * t.kcap;
        cx_t<T> cj[ORB];
        T re[ORB], im[ORB];
#pragma unroll
        for (int o = 0; o < ORB; ++o) {
            cj[o] = A0 + o < n_orb ? cnl_in[(int64_t)J * n_orb + A0 + o] : cx_t<T>{(T)0, (T)0};
            re[o] = 0;
            im[o] = 0;
        }
        for (int k0 = 0; k0 < K; k0 += 64 * GATHER_U) {
            int id[GATHER_U];
            T w[GATHER_U];
            bool sh[GATHER_U];
#pragma unroll
            for (int i = 0; i < GATHER_U; ++i) {
                const int k = k0 + lane + 64 * i;
                id[i] = k < K ? ix[k] : -1;
                w[i] = k < K ? pp[k] : (T)0;
                sh[i] = k < K && po[k] != 0;
            }
            cx_t<T> z[ORB][GATHER_U];
#pragma unroll
            for (int o = 0; o < ORB; ++o) {
                const cx_t<T>* ua = out + (int64_t)(A0 + o) * stride;
#pragma unroll
                for (int i = 0; i < GATHER_U; ++i)
                    z[o][i] = (id[i] >= 0 && A0 + o < n_orb) ? ua[id[i]] : cx_t<T>{(T)0, (T)0};
            }
#pragma unroll
            for (int o = 0; o < ORB; ++o) {
                const int A = A0 + o;
                if (A >= n_orb) continue;
                cx_t<T>* ua = out + (int64_t)A * stride;
#pragma unroll
                for (int i = 0; i < GATHER_U; ++i) {
                    if (id[i] < 0) continue;
                    T sr = 0, si = 0;
                    if (!sh[i]) {
                        nl_acc<T>(w[i], cj[o], sr, si);
                        z[o][i] = nl_add<T>(z[o][i], sr, si, gr, gi);
                        ua[id[i]] = z[o][i];
                    } else {                   // shared point: the slot's pairs, in ion order
                        const int sl = t.map[id[i]];
                        const int n = min(t.cnt[sl], NL_KMAX);
                        for (int q = 0; q < n; ++q)
                            nl_acc<T>(pl[q * ucap + sl], cnl_in[(int64_t)t.ion[q * ucap + sl] * n_orb + A], sr, si);
                        z[o][i] = nl_add<T>(z[o][i], sr, si, gr, gi);
                    }
                }
#pragma unroll
                for (int i = 0; i < GATHER_U; ++i) {
                    re[o] += w[i] * z[o][i].x;
                    im[o] += w[i] * z[o][i].y;
                }
            }
        }
#pragma unroll
        for (int o = 0; o < ORB; ++o) {
            const T r = wsum_t(re[o]);
            const T m = wsum_t(im[o]);
            if (lane == 0 && A0 + o < n_orb) cnl_out[(int64_t)J * n_orb + A0 + o] = cx_t<T>{scale * r, scale * m};
        }
    }
    if (last_of_group(t.ovc + grp, n_ions, last)) {
        const int B0 = grp * G;
        fix_shared_points<T>(out, stride, n_orb, B0, min(G, n_orb - B0), t.ovl, t.ovn, t.pts, t.cnt, t.ion, pl, ucap,
                             cnl_in, gr, gi, t.ovc + grp);
    }
}

template <typename T, int ORB>
__global__ void __launch_bounds__(256) kb_fixup_gather_kernel(cx_t<T>* __restrict__ out, int64_t stride, int n_orb,
                                                              KbTables t, const cx_t<T>* __restrict__ cnl_in, T gr,
                                                              T gi, T scale, cx_t<T>* __restrict__ cnl_out) {
    __shared__ int last;
    fixup_gather_block<T, ORB>(out, stride, n_orb, (int)gridDim.y, t, cnl_in, gr, gi, scale, cnl_out, blockIdx.y,
                               blockIdx.x, &last);
}

// the same pass for several systems in one launch: block b belongs to the
// last system whose first block is <= b; within a system blocks run over the
// orbital groups fastest, as the single-system grid does
template <typename T, int ORB>
__global__ void __launch_bounds__(256) batch_kb_fixup_gather_kernel(BatchKbArgs<T> a) {
    __shared__ int last;
    int s = 0;
    while (s + 1 < a.n_sys && (int)blockIdx.x >= a.sys[s + 1].b0) ++s;
    const BatchKbSys<T>& d = a.sys[s];
    const int groups = (d.n_orb + 4 * ORB - 1) / (4 * ORB);
    const int local = (int)blockIdx.x - d.b0;
    fixup_gather_block<T, ORB>(d.out, d.stride, d.n_orb, d.n_ions, d.t, d.cnl_in, (T)0, d.gi, d.scale, d.cnl_out,
                               local / groups, local % groups, &last);
}

// orbitals per wave of the fused pass: FP32 two (one index / projector load
// for both; 78 VGPRs), FP64 one (two would take 136 VGPRs)
template <typename T> constexpr int fg_orb() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T>
hipError_t launch_kb_fixup_gather(cx_t<T>* out, int64_t stride, int n_orb, int n_ions, KbTables t,
                                  const cx_t<T>* cnl_in, double gr, double gi, double ekb_h3, cx_t<T>* cnl_out,
                                  hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    if (t.novc < (n_orb + 3) / 4) return hipErrorInvalidValue;
    constexpr int ORB = fg_orb<T>();
    dim3 grid((n_orb + 4 * ORB - 1) / (4 * ORB), n_ions);
    kb_fixup_gather_kernel<T, ORB><<<grid, 256, 0, s>>>(out, stride, n_orb, t, cnl_in, (T)gr, (T)gi, (T)ekb_h3,
                                                        cnl_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_kb_fixup_gather(BatchKbArgs<T> a, hipStream_t s) {
    constexpr int ORB = fg_orb<T>();
    if (a.n_sys < 1 || a.n_sys > KB_BATCH) return hipErrorInvalidValue;
    int blocks = 0;
    for (int i = 0; i < a.n_sys; ++i) {
        BatchKbSys<T>& d = a.sys[i];
        if (d.n_ions < 1 || d.t.novc < (d.n_orb + 3) / 4) return hipErrorInvalidValue;
        d.b0 = blocks;
        blocks += ((d.n_orb + 4 * ORB - 1) / (4 * ORB)) * d.n_ions;
    }
    batch_kb_fixup_gather_kernel<T, ORB><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

template hipError_t launch_batch_kb_fixup_gather<double>(BatchKbArgs<double>, hipStream_t);
template hipError_t launch_batch_kb_fixup_gather<float>(BatchKbArgs<float>, hipStream_t);

template hipError_t launch_kb_fixup_gather<double>(double2*, int64_t, int, int, KbTables, const double2*, double,
                                                   double, double, double2*, hipStream_t);
template hipError_t launch_kb_fixup_gather<float>(float2*, int64_t, int, int, KbTables, const float2*, double,
                                                  double, double, float2*, hipStream_t);

// ------------------------------------------------------------ split-bf16 MFMA contraction
// The same contraction as a matrix product on the matrix cores:
// D[16 x 16] += A[16 x 32] B[32 x 16] with v_mfma_f32_16x16x32_bf16, A rows
// = 16 orbitals at 32 of the ion's points (real parts in one chain, imaginary
// parts in another), B column 0 = the projector at those points (one
// s-channel projector per ion fills one column; the force gather fills
// columns 1-3 with (r - R_J)_a p_J).  Each FP32 operand is split into bf16 hi
// + lo parts and the product accumulated in FP32 as hi*hi + hi*lo + lo*hi.
// Fragment layout of the 16x16x32 bf16 instruction: lane l holds A row l%16,
// k = 8(l/16)..+7; B column l%16 with the same k; D column l%16, rows
// 4(l/16)..+3.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ void split8(const float* v, bf16x8_t& hi, bf16x8_t& lo) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        __bf16 h, l;
        split_bf16(v[i], h, l);
        hi[i] = h;
        lo[i] = l;
    }
}

__device__ __forceinline__ f32x4_t mfma3(const bf16x8_t& ah, const bf16x8_t& al, const bf16x8_t& bh,
                                         const bf16x8_t& bl, f32x4_t acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    return acc;
}

// A workgroup of GW waves takes 16 orbitals of one ion; wave w takes the
// 32-point chunks w, w + GW, ... of the ion's list (one chunk for lists of up
// to 32 GW points).  A chunk is loaded as the FP32 gather loads it (each
// instruction two orbitals at 32 consecutive list entries, one index load per
// lane for all 16 orbitals), staged in the wave's own LDS rows (padded
// against bank conflicts), and read back in the MFMA fragment layout.  The
// waves' tiles are summed in a fixed order through LDS.  FORCE: B columns 1-3
// hold (r - R_J)_a p_J (minimum image, FP64 geometry rounded to FP32) and the
// result goes to dnl ([n_ions][n_orb][3] complex, h^3 sum (r - R_J) p psi)
// beside cnl.
constexpr int BG_ROW = 32 + 2;       // LDS row of one orbital's chunk (complex), padded

// With FIX the loaded values are first fixed up as in kb_fixup_gather_kernel
// (a point of one sphere in place, a shared one in registers for the sum and
// written by the last workgroup of the orbital group) and the contraction
// runs on the fixed values.
struct FixArgs {
    float2* out;                                      // the orbitals (the kernel's u, read and written)
    const uint8_t* ov;
    const int32_t *map, *cnt, *ion;
    const float* pl;
    int64_t ucap;
    const float2* cnl_in;
    float gr, gi;
    const int32_t *ovl, *ovn, *pts;
    int32_t* ovc;
};

template <bool FORCE, bool FIX = false>
__global__ void __launch_bounds__(1024) kb_gather_bf16x3_kernel(const float2* __restrict__ u, int64_t stride,
                                                                int n_orb, const int32_t* __restrict__ idx,
                                                                const float* __restrict__ pv,
                                                                const int32_t* __restrict__ count, int kcap,
                                                                float scale, float2* __restrict__ cnl,
                                                                const double* __restrict__ pos, KbGeom g,
                                                                int nx, int ny, float dscale,
                                                                float2* __restrict__ dnl, FixArgs fx = {}) {
    constexpr int NC = FORCE ? 4 : 1;                 // useful B columns
    __shared__ float2 zs[16][16][BG_ROW];             // [wave][orbital][point of the chunk]
    __shared__ float bs[16][NC][32];                  // [wave][column][point]
    __shared__ float part[16][2][NC][16];             // [wave][re, im][column][orbital]
    const int J = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int GW = blockDim.x >> 6;
    const int A0 = blockIdx.x * 16;
    const int K = count[J];
    const int32_t* ix = idx + (int64_t)J * kcap;
    const float* pp = pv + (int64_t)J * kcap;
    const int m = lane & 15;                          // fragment: A row (orbital) and B column
    const int kq = lane >> 4;                         // fragment: k group of 8 points
    const int lp = lane & 31;                         // load: point of the chunk
    const int lo = lane >> 5;                         // load: orbital of the pair
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if constexpr (FORCE) {
        rx = pos[3 * J];
        ry = pos[3 * J + 1];
        rz = pos[3 * J + 2];
    }
    const float2* src = FIX ? fx.out : u;             // FIX: u is not used (it aliases the writes)
    f32x4_t dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 32 * wv; k0 < K; k0 += 32 * GW) {
        const int k = k0 + lp;
        const int id = k < K ? ix[k] : -1;
        float2 z[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int a = A0 + 2 * i + lo;
            z[i] = (id >= 0 && a < n_orb) ? src[(int64_t)a * stride + id] : make_float2(0.f, 0.f);
        }
        if constexpr (FIX) {
            if (id >= 0) {
                const bool shared = fx.ov[(int64_t)J * kcap + k] != 0;
                const float pk = pp[k];
                const int sl = shared ? fx.map[id] : 0;
                const int npair = shared ? min(fx.cnt[sl], NL_KMAX) : 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int a = A0 + 2 * i + lo;
                    if (a >= n_orb) continue;
                    float sr = 0.f, si = 0.f;
                    if (!shared) {
                        nl_acc<float>(pk, fx.cnl_in[(int64_t)J * n_orb + a], sr, si);
                        z[i] = nl_add<float>(z[i], sr, si, fx.gr, fx.gi);
                        fx.out[(int64_t)a * stride + id] = z[i];
                    } else {
                        for (int q = 0; q < npair; ++q)
                            nl_acc<float>(fx.pl[q * fx.ucap + sl],
                                          fx.cnl_in[(int64_t)fx.ion[q * fx.ucap + sl] * n_orb + a], sr, si);
                        z[i] = nl_add<float>(z[i], sr, si, fx.gr, fx.gi);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) zs[wv][2 * i + lo][lp] = z[i];
        if (lo == 0) {
            const float p = id >= 0 ? pp[k] : 0.f;
            bs[wv][0][lp] = p;
            if constexpr (FORCE) {
                double dx = 0.0, dy = 0.0, dz = 0.0;
                if (id >= 0) {
                    const int gx = id % nx, gy = (id / nx) % ny, gz = id / (nx * ny);
                    kb_d2(g, gx, gy, gz, rx, ry, rz, dx, dy, dz);
                }
                bs[wv][1][lp] = (float)dx * p;
                bs[wv][2][lp] = (float)dy * p;
                bs[wv][3][lp] = (float)dz * p;
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);           // this wave's LDS writes complete (lgkmcnt 0)
        __builtin_amdgcn_wave_barrier();
        float zr[8], zi[8], bv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float2 v = zs[wv][m][8 * kq + i];
            zr[i] = v.x;
            zi[i] = v.y;
            bv[i] = m < NC ? bs[wv][m < NC ? m : 0][8 * kq + i] : 0.f;
        }
        __builtin_amdgcn_wave_barrier();              // reads done before the next chunk's writes
        bf16x8_t arh, arl, aih, ail, bh, bl;
        split8(zr, arh, arl);
        split8(zi, aih, ail);
        split8(bv, bh, bl);
        dre = mfma3(arh, arl, bh, bl, dre);
        dim = mfma3(aih, ail, bh, bl, dim);
    }
    // lane l holds D[4 kq + r][m]: column m, orbitals A0 + 4 kq + r
    if (m < NC) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            part[wv][0][m][4 * kq + r] = dre[r];
            part[wv][1][m][4 * kq + r] = dim[r];
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 16 * NC) {
        const int o = t & 15, c = t >> 4;
        float vr = 0.f, vi = 0.f;
        for (int w = 0; w < GW; ++w) {
            vr += part[w][0][c][o];
            vi += part[w][1][c][o];
        }
        if (A0 + o < n_orb) {
            if (c == 0)
                cnl[(int64_t)J * n_orb + A0 + o] = make_float2(scale * vr, scale * vi);
            else if constexpr (FORCE)
                dnl[((int64_t)J * n_orb + A0 + o) * 3 + (c - 1)] = make_float2(dscale * vr, dscale * vi);
        }
    }
    if constexpr (FIX) {
        __shared__ int last;
        if (last_of_group(fx.ovc + blockIdx.x, (int)gridDim.y, &last))
            fix_shared_points<float>(fx.out, stride, n_orb, A0, min(16, n_orb - A0), fx.ovl, fx.ovn, fx.pts, fx.cnt,
                                     fx.ion, fx.pl, fx.ucap, fx.cnl_in, fx.gr, fx.gi, fx.ovc + blockIdx.x);
    }
}

// waves per workgroup: one per 32-point chunk of the largest ion list, at most
// 8 (at the kernel's register use 1024-thread workgroups fit once per CU,
// 512-thread ones three times); MODEHR_BG_WAVES overrides (measurements)
static int bf16_gather_waves(int kcap) {
    const char* e = std::getenv("MODEHR_BG_WAVES");
    const int cap = (e && *e) ? std::max(1, std::min(16, std::atoi(e))) : 8;
    return std::max(1, std::min(cap, (kcap + 31) / 32));
}

hipError_t launch_kb_gather_bf16x3(const float2* u, int64_t stride, int n_orb, int n_ions, KbTables t,
                                   double ekb_h3, float2* cnl, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    dim3 grid((n_orb + 15) / 16, n_ions);
    KbGeom g0{};
    kb_gather_bf16x3_kernel<false><<<grid, 64 * bf16_gather_waves(t.kcap), 0, s>>>(
        u, stride, n_orb, t.idx, reinterpret_cast<const float*>(t.p), t.count, t.kcap, (float)ekb_h3, cnl,
        nullptr, g0, 1, 1, 0.f, nullptr);
    return hipGetLastError();
}

hipError_t launch_kb_fixup_gather_bf16x3(float2* out, int64_t stride, int n_orb, int n_ions, KbTables t,
                                         const float2* cnl_in, double gr, double gi, double ekb_h3, float2* cnl_out,
                                         hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    dim3 grid((n_orb + 15) / 16, n_ions);
    KbGeom g0{};
    if (t.novc < (n_orb + 15) / 16) return hipErrorInvalidValue;
    FixArgs fx{out,    t.ov,      t.map,     t.cnt, t.ion, reinterpret_cast<const float*>(t.pl),
               t.ucap, cnl_in,    (float)gr, (float)gi, t.ovl, t.ovn, t.pts, t.ovc};
    kb_gather_bf16x3_kernel<false, true><<<grid, 64 * bf16_gather_waves(t.kcap), 0, s>>>(
        nullptr, stride, n_orb, t.idx, reinterpret_cast<const float*>(t.p), t.count, t.kcap, (float)ekb_h3, cnl_out,
        nullptr, g0, 1, 1, 0.f, nullptr, fx);
    return hipGetLastError();
}

// the contraction and the three force columns of FP32 orbitals by split-bf16
// MFMA: cnl[J][A] = h^3 sum p psi (E_KB not included), dnl[J][A][a] =
// h^3 sum (r - R_J)_a p psi; then, in FP64, fnl[J] = -2 f E_KB / s^2 sum_A
// Re(conj(c) d) and enl[J] = f E_KB sum_A |c|^2
__global__ void kb_forces_from_columns_kernel(const float2* __restrict__ cnl, const float2* __restrict__ dnl,
                                              int n_orb, int n_ions, double kf, double ke,
                                              double* __restrict__ fnl, double* __restrict__ enl) {
    __shared__ double red[4][4];
    const int J = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double f[3] = {0.0, 0.0, 0.0}, e = 0.0;
    for (int A = threadIdx.x; A < n_orb; A += blockDim.x) {
        const float2 c = cnl[(int64_t)J * n_orb + A];
        const double cr = c.x, ci = c.y;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const float2 d = dnl[((int64_t)J * n_orb + A) * 3 + ax];
            f[ax] += cr * (double)d.x + ci * (double)d.y;
        }
        e += cr * cr + ci * ci;
    }
    double v[4] = {f[0], f[1], f[2], e};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double x = v[c];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) red[wv][c] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) fnl[3 * J + threadIdx.x] = kf * (((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                            red[2][threadIdx.x]) + red[3][threadIdx.x]);
    if (threadIdx.x == 3) enl[J] = ke * (((red[0][3] + red[1][3]) + red[2][3]) + red[3][3]);
}

hipError_t launch_kb_forces_bf16x3(const float2* psi, int64_t stride, int n_orb, int n_ions, KbTables t,
                                   const double* pos, const KbGeom& g, int nx, int ny, double occ, double ekb,
                                   float2* cnl, float2* dnl, double* fnl, double* enl_part, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    const double h3 = g.h * g.h * g.h;
    dim3 grid((n_orb + 15) / 16, n_ions);
    kb_gather_bf16x3_kernel<true><<<grid, 64 * bf16_gather_waves(t.kcap), 0, s>>>(
        psi, stride, n_orb, t.idx, reinterpret_cast<const float*>(t.p), t.count, t.kcap, (float)h3, cnl, pos, g,
        nx, ny, (float)h3, dnl);
    kb_forces_from_columns_kernel<<<n_ions, 256, 0, s>>>(cnl, dnl, n_orb, n_ions,
                                                         -2.0 * occ * ekb * g.inv_s2, occ * ekb, fnl, enl_part);
    return hipGetLastError();
}

// ------------------------------------------------------------ forces
// Grid (n_ions, ceil(n_orb/16)); each wave takes 4 orbitals of the group.
// Everything is accumulated in FP64: c = sum p psi, d = sum (r-R) p psi per
// axis; per block the partial sums of Re(conj(c) d) (3 axes) and |c|^2 are
// written, and a second kernel adds the blocks of each ion in order:
// F_J = -2 f E_KB h^6 / s^2 sum_A Re(conj(c) d), E_J = f E_KB h^6 sum_A |c|^2.
constexpr int KBF_OB = 16;

// 8th-order central first difference: f' ~ (1/h) sum_m a_m (f(x + m h) - f(x - m h))
__device__ constexpr double FD1[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

// The wave-function-gradient form: the columns are h^3 sum p_J grad psi_A
// (8th-order finite-difference gradient) instead of h^3 sum p_J (r - R_J)
// psi_A (kb_forces_proj_kernel).
template <typename T>
__global__ void __launch_bounds__(256) kb_forces_grad_kernel(const cx_t<T>* __restrict__ psi, int64_t stride,
                                                             int n_orb, const int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ count, int kcap,
                                                             const double* __restrict__ pos, KbGeom g,
                                                             int nx, int ny, int nz, double* __restrict__ part) {
    __shared__ double red[4][4];
    const int J = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int K = count[J];
    const int32_t* ix = idx + (int64_t)J * kcap;
    const double rx = pos[3 * J], ry = pos[3 * J + 1], rz = pos[3 * J + 2];
    double fx = 0, fy = 0, fz = 0, en = 0;
    const int A_end = min(n_orb, (int)(blockIdx.y + 1) * KBF_OB);
    for (int A = blockIdx.y * KBF_OB + wv; A < A_end; A += 4) {
        const cx_t<T>* pa = psi + (int64_t)A * stride;
        double cr = 0, ci = 0, xr = 0, xi = 0, yr = 0, yi = 0, zr = 0, zi = 0;
        for (int k = lane; k < K; k += 64) {
            const int lin = ix[k];
            const int gx = lin % nx;
            const int gy = (lin / nx) % ny;
            const int gz = lin / (nx * ny);
            double dx, dy, dz;
            const double d2 = kb_d2(g, gx, gy, gz, rx, ry, rz, dx, dy, dz);
            const double w = kb_value(g, d2);
            const cx_t<T> zv = pa[lin];
            const double pr = w * (double)zv.x, pi = w * (double)zv.y;
            cr += pr; ci += pi;
            const int64_t plane = (int64_t)nx * ny;
            const int64_t row = lin - gx, col = lin - (int64_t)gy * nx, pil = lin - (int64_t)gz * plane;
            double ax = 0, bx = 0, ay = 0, by = 0, az = 0, bz = 0;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const cx_t<T> xp = pa[row + wrap1(gx + m, nx)], xm = pa[row + wrap1(gx - m, nx)];
                const cx_t<T> yp = pa[col + (int64_t)wrap1(gy + m, ny) * nx];
                const cx_t<T> ym = pa[col + (int64_t)wrap1(gy - m, ny) * nx];
                const cx_t<T> zp = pa[pil + (int64_t)wrap1(gz + m, nz) * plane];
                const cx_t<T> zm = pa[pil + (int64_t)wrap1(gz - m, nz) * plane];
                const double a = FD1[m - 1];
                ax += a * ((double)xp.x - (double)xm.x); bx += a * ((double)xp.y - (double)xm.y);
                ay += a * ((double)yp.x - (double)ym.x); by += a * ((double)yp.y - (double)ym.y);
                az += a * ((double)zp.x - (double)zm.x); bz += a * ((double)zp.y - (double)zm.y);
            }
            xr += w * ax; xi += w * bx;
            yr += w * ay; yi += w * by;
            zr += w * az; zi += w * bz;
        }
        cr = wsum_t(cr); ci = wsum_t(ci);
        xr = wsum_t(xr); xi = wsum_t(xi);
        yr = wsum_t(yr); yi = wsum_t(yi);
        zr = wsum_t(zr); zi = wsum_t(zi);
        fx += cr * xr + ci * xi;
        fy += cr * yr + ci * yi;
        fz += cr * zr + ci * zi;
        en += cr * cr + ci * ci;
    }
    if (lane == 0) {
        red[wv][0] = fx; red[wv][1] = fy; red[wv][2] = fz; red[wv][3] = en;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        part[((int64_t)J * gridDim.y + blockIdx.y) * 4 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

// The projector form: columns h^3 sum p_J (r - R_J) psi_A.  For ions of at
// most KBF_CH points each point's grid index, minimum-image offset and
// projector value are computed once per workgroup into LDS instead of once
// per orbital, and each lane's eight orbital loads are issued together; a
// workgroup whose ion has more points recomputes them per orbital.  Either
// way lanes visit the points lane, lane + 64, ... in order with the same
// expressions, so the two give the same bits.
constexpr int KBF_CH = 512;

template <typename T>
__global__ void __launch_bounds__(256) kb_forces_proj_kernel(const cx_t<T>* __restrict__ psi, int64_t stride,
                                                             int n_orb, const int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ count, int kcap,
                                                             const double* __restrict__ pos, KbGeom g, int nx,
                                                             int ny, double* __restrict__ part) {
    __shared__ double red[4][4];
    __shared__ double sw[KBF_CH], sx[KBF_CH], sy[KBF_CH], sz[KBF_CH];
    __shared__ int sl[KBF_CH];
    const int J = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int K = count[J];
    const int32_t* ix = idx + (int64_t)J * kcap;
    const double rx = pos[3 * J], ry = pos[3 * J + 1], rz = pos[3 * J + 2];
    const bool fast = K <= KBF_CH;
    if (fast) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            const int lin = ix[k];
            const int gx = lin % nx;
            const int gy = (lin / nx) % ny;
            const int gz = lin / (nx * ny);
            double dx, dy, dz;
            const double d2 = kb_d2(g, gx, gy, gz, rx, ry, rz, dx, dy, dz);
            sl[k] = lin;
            sw[k] = kb_value(g, d2);
            sx[k] = dx;
            sy[k] = dy;
            sz[k] = dz;
        }
    }
    __syncthreads();
    double fx = 0, fy = 0, fz = 0, en = 0;
    const int A_end = min(n_orb, (int)(blockIdx.y + 1) * KBF_OB);
    for (int A = blockIdx.y * KBF_OB + wv; A < A_end; A += 4) {
        const cx_t<T>* pa = psi + (int64_t)A * stride;
        double cr = 0, ci = 0, xr = 0, xi = 0, yr = 0, yi = 0, zr = 0, zi = 0;
        if (fast) {
            cx_t<T> zv[KBF_CH / 64];
#pragma unroll
            for (int i = 0; i < KBF_CH / 64; ++i) {
                const int k = lane + 64 * i;
                zv[i] = k < K ? pa[sl[k]] : cx_t<T>{(T)0, (T)0};
            }
#pragma unroll
            for (int i = 0; i < KBF_CH / 64; ++i) {
                const int k = lane + 64 * i;
                if (k < K) {
                    const double w = sw[k], dx = sx[k], dy = sy[k], dz = sz[k];
                    const double pr = w * (double)zv[i].x, pi = w * (double)zv[i].y;
                    cr += pr; ci += pi;
                    xr += dx * pr; xi += dx * pi;
                    yr += dy * pr; yi += dy * pi;
                    zr += dz * pr; zi += dz * pi;
                }
            }
        } else {
            for (int k = lane; k < K; k += 64) {
                const int lin = ix[k];
                const int gx = lin % nx;
                const int gy = (lin / nx) % ny;
                const int gz = lin / (nx * ny);
                double dx, dy, dz;
                const double d2 = kb_d2(g, gx, gy, gz, rx, ry, rz, dx, dy, dz);
                const double w = kb_value(g, d2);
                const cx_t<T> zv = pa[lin];
                const double pr = w * (double)zv.x, pi = w * (double)zv.y;
                cr += pr; ci += pi;
                xr += dx * pr; xi += dx * pi;
                yr += dy * pr; yi += dy * pi;
                zr += dz * pr; zi += dz * pi;
            }
        }
        cr = wsum_t(cr); ci = wsum_t(ci);
        xr = wsum_t(xr); xi = wsum_t(xi);
        yr = wsum_t(yr); yi = wsum_t(yi);
        zr = wsum_t(zr); zi = wsum_t(zi);
        fx += cr * xr + ci * xi;
        fy += cr * yr + ci * yi;
        fz += cr * zr + ci * zi;
        en += cr * cr + ci * ci;
    }
    if (lane == 0) {
        red[wv][0] = fx; red[wv][1] = fy; red[wv][2] = fz; red[wv][3] = en;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        part[((int64_t)J * gridDim.y + blockIdx.y) * 4 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

// the blocks of each ion added in order (loads issued eight blocks at a time)
__global__ void kb_forces_reduce_kernel(const double* __restrict__ part, int nblk, int n_ions, double kf,
                                        double ke, double* __restrict__ fnl, double* __restrict__ enl) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= n_ions) return;
    double s[4] = {0, 0, 0, 0};
    const double* pj = part + (int64_t)J * nblk * 4;
    for (int b0 = 0; b0 < nblk; b0 += 8) {
        double v[8][4];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[i][c] = b0 + i < nblk ? pj[(b0 + i) * 4 + c] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (b0 + i < nblk)
#pragma unroll
                for (int c = 0; c < 4; ++c) s[c] += v[i][c];
    }
    fnl[3 * J] = kf * s[0];
    fnl[3 * J + 1] = kf * s[1];
    fnl[3 * J + 2] = kf * s[2];
    enl[J] = ke * s[3];
}

template <typename T>
hipError_t launch_kb_forces(const cx_t<T>* psi, int64_t stride, int n_orb, int n_ions,
                            KbTables t, const double* pos, const KbGeom& g,
                            int nx, int ny, int nz, int form, double occ, double ekb,
                            double* fnl, double* enl_part, double* scratch, hipStream_t s) {
    if (n_ions == 0) return hipSuccess;
    if (form != 0 && form != 1) return hipErrorInvalidValue;
    const int nblk = (n_orb + KBF_OB - 1) / KBF_OB;
    dim3 grid(n_ions, nblk);
    if (form == 1)
        kb_forces_grad_kernel<T><<<grid, 256, 0, s>>>(psi, stride, n_orb, t.idx, t.count, t.kcap, pos, g, nx, ny,
                                                       nz, scratch);
    else
        kb_forces_proj_kernel<T><<<grid, 256, 0, s>>>(psi, stride, n_orb, t.idx, t.count, t.kcap, pos, g, nx, ny,
                                                      scratch);
    const double h6 = g.h * g.h * g.h * g.h * g.h * g.h;
    const double kf = -2.0 * occ * ekb * h6 * (form == 1 ? 1.0 / g.h : g.inv_s2);
    kb_forces_reduce_kernel<<<(n_ions + 63) / 64, 64, 0, s>>>(scratch, nblk, n_ions, kf, occ * ekb * h6, fnl,
                                                             enl_part);
    return hipGetLastError();
}

template hipError_t launch_kb_tables<double>(const double*, int, int, int, int, const KbGeom&, KbTables, hipStream_t);
template hipError_t launch_kb_tables<float>(const double*, int, int, int, int, const KbGeom&, KbTables, hipStream_t);
template hipError_t launch_kb_fixup<double>(cx_t<double>*, int64_t, int, KbTables, const cx_t<double>*, double, double, double*, hipStream_t);
template hipError_t launch_kb_fixup<float>(cx_t<float>*, int64_t, int, KbTables, const cx_t<float>*, double, double, double*, hipStream_t);
template hipError_t launch_kb_gather<double>(const cx_t<double>*, int64_t, int, int, KbTables, double, cx_t<double>*, hipStream_t);
template hipError_t launch_kb_gather<float>(const cx_t<float>*, int64_t, int, int, KbTables, double, cx_t<float>*, hipStream_t);
template hipError_t launch_kb_forces<double>(const cx_t<double>*, int64_t, int, int, KbTables, const double*, const KbGeom&, int, int, int, int, double, double, double*, double*, double*, hipStream_t);
template hipError_t launch_kb_forces<float>(const cx_t<float>*, int64_t, int, int, KbTables, const double*, const KbGeom&, int, int, int, int, double, double, double*, double*, double*, hipStream_t);

}  // namespace me

// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include <string>

namespace me {

// text returned by me_last_error(NULL) on this thread (calls without a handle)
void set_thread_error(const std::string& text);

// complex element type of each precision: interleaved (re, im)
template <typename T> struct cx;
template <> struct cx<double> { using type = double2; };
template <> struct cx<float> { using type = float2; };
template <typename T> using cx_t = typename cx<T>::type;

// 8th-order central second difference, f'' ~ (1/h^2)[c0 f0 + sum_m cm (f_m + f_-m)]
constexpr double FD_C0 = -205.0 / 72.0;
constexpr double FD_C1 = 8.0 / 5.0;
constexpr double FD_C2 = -1.0 / 5.0;
constexpr double FD_C3 = 8.0 / 315.0;
constexpr double FD_C4 = -1.0 / 560.0;

constexpr int MAX_TAYLOR = 8;
constexpr int MAX_WORDS = 64;    // ion bitmask words per stencil tile row (<= 2048 ions)

// Geometry of the Gaussian projector, FP64 (shared by table build, stencil
// scatter and force gather so the three agree bit for bit).
struct KbGeom {
    double h;
    double L[3];
    double rcut2;      // r_cut^2
    double inv2s2;     // 1/(2 sigma^2)
    double pnorm;      // (pi sigma^2)^(-3/4)
    double inv_s2;     // 1/sigma^2
};

constexpr int NL_KMAX = 8;       // projectors that may overlap at one grid point
constexpr int FIX_OB = 8;        // orbitals per fix-up thread
// fix-up workgroups per orbital group: one thread per possible slot
inline int fixup_blocks(int64_t ucap) { return (int)((ucap + 255) / 256); }

// Per-ion projector tables (one set per ion configuration), and the same
// information by grid point: the union of all projector spheres as a list of
// slots, each with the (ion, value) pairs covering it, ordered by ion.
struct KbTables {
    int32_t* idx;      // [n_ions][kcap] linear grid index
    void* p;           // [n_ions][kcap] projector value in the compute precision
    int32_t* count;    // [n_ions]
    int kcap;
    int m;             // candidate box half-width: per axis min(2m+2, n) points
    // point lists
    int32_t* map;      // [N] slot of each grid point, or -1
    int32_t* pts;      // [ucap] grid index of each slot
    int32_t* cnt;      // [ucap] pairs per slot
    int32_t* ion;      // [NL_KMAX][ucap]: pair k of slot s at k * ucap + s, so that
                       // lanes on neighbouring slots read neighbouring words
    void* pl;          // [NL_KMAX][ucap] projector values, the same layout
    int32_t* nslots;   // [1]
    int32_t* flag;     // [1] set when a point is covered by more than NL_KMAX spheres
    int32_t* blk;      // [scan blocks + 1] scratch of the slot numbering
    int64_t ucap;
    uint8_t* ov;       // [n_ions][kcap] 1 where the table point is covered by another sphere too
    int32_t* ovl;      // [ucap] slots covered by more than one sphere (any order), count in *ovn
    int32_t* ovn;      // [1]
    int32_t* ovc;      // [novc] finished workgroups of each orbital group of the fused fix-up +
    int novc;          // gather pass (zero between launches; one counter per 4 orbitals)
};

enum StencilMode : int {
    MODE_APPLY = 0,        // out = H u
    MODE_HORNER = 1,       // out = psi0 + i*alpha*(H u)
    MODE_HORNER_FIRST = 2, // as HORNER with psi0 == u
    MODE_EXPECT_T = 3,     // partial[A][tile] = sum Re(conj(u) T u); no output
    MODE_SCALED = 4        // out = i*alpha*(H u)   (adjoint stages)
};

template <typename T>
struct StencilArgs {
    const cx_t<T>* u;
    const cx_t<T>* psi0;
    cx_t<T>* out;
    const T* v;              // v_eff [N] (unused by EXPECT_T)
    int64_t stride;          // complex elements between orbitals (u, psi0, out)
    int nx, ny, nz;
    int n_orb;
    int zchunk;              // planes per workgroup (the last chunk may be shorter)
    int nyt, nzc;            // tiles along y, chunks along z
    int tx, nxt;             // tile width (nx: whole rows) and tiles along x
    int py;                  // whole rows: rows per thread (1 or 2)
    T kin;                   // -1/(2 h^2)
    T alpha;                 // Horner coefficient: c_k = i*alpha, alpha = -tau/k
    double* partial;         // [n_orb][nyt*nzc] norm or expectation partials, or nullptr
    const int2* zr;          // finite box: per y-tile the planes [x, y) that hold every box
                             // point of its rows (outputs elsewhere are left as they are,
                             // zero by the box invariant), or nullptr: whole columns
};

// One system of a batched (persistent) stencil launch.
constexpr int MAX_BATCH = 32;
template <typename T>
struct BatchSys {
    const cx_t<T>* u;
    const cx_t<T>* psi0;
    cx_t<T>* out;
    const T* v;
    double* partial;
    int64_t stride;
    int nx, ny, nz;
    int ty, nyt;             // rows per tile, tiles (the last may be ragged)
    int tx, nxt;             // tile width (nx: whole rows) and x-tiles (the last may be ragged)
    int zchunk, nzc;         // planes per slab, slabs (the last may be short)
    int item0, items;        // first work item of this system, item count
    T kin, alpha;
};
template <typename T>
struct BatchStencilArgs {
    BatchSys<T> sys[MAX_BATCH];
    int n_sys;
    int total;               // work items over all systems
    int* counter;            // device, 8 queue counters, zero at launch; nullptr: one
                             // item per workgroup (grid = 8 x the largest XCD share)
};

// dynamic LDS of a stencil workgroup: two halo tiles of (ty + 8) rows of nx
inline size_t stencil_lds_bytes(int ty, int nx, size_t bc) { return 2 * (size_t)(ty + 8) * nx * bc; }
// the same for an x-tile of tx columns (plus the 4 + 4 x-halo columns)
inline size_t stencil_xt_lds_bytes(int tx, int ty, size_t bc) { return 2 * (size_t)(ty + 8) * (tx + 8) * bc; }

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
template <typename T>
hipError_t launch_stencil(const StencilArgs<T>& a, int mode, bool want_norm,
                          int ty, int px, hipStream_t s);

// persistent launch over all systems of a batch (HORNER / HORNER_FIRST modes)
template <typename T>
hipError_t launch_batch_stencil(const BatchStencilArgs<T>& a, int mode, bool norm, int block, int grid,
                                size_t lds, hipStream_t s);
// resident workgroups per CU of the batched kernel (hj = halo runs per thread,
// xt: the variant with x-tiled systems)
template <typename T>
hipError_t batch_stencil_occupancy(int block, size_t lds, int hj, bool xt, int* wg_per_cu);
hipError_t launch_zero_i32(int* p, int n, hipStream_t s);

template <typename T>
hipError_t launch_kb_tables(const double* pos, int n_ions, int nx, int ny, int nz,
                            const KbGeom& g, KbTables t, hipStream_t s);

// out_A(r) += (gr + i gi) * sum_{J covers r} p_J(r) cnl[J*n_orb + A], at the
// projector points only; dnorm (nullable): [n_orb][FIX_XB] change of |out_A|^2
template <typename T>
hipError_t launch_kb_fixup(cx_t<T>* out, int64_t stride, int n_orb, KbTables t,
                           const cx_t<T>* cnl, double gr, double gi, double* dnorm, hipStream_t s);

// cnl[J*n_orb + A] = ekb * h^3 sum_k p_J(k) u_A(idx_J(k))
template <typename T>
hipError_t launch_kb_gather(const cx_t<T>* u, int64_t stride, int n_orb, int n_ions,
                            KbTables t, double ekb_h3, cx_t<T>* cnl, hipStream_t s);

// One stage's fix-up and the next stage's gather in one pass over the
// projector points: out_A(r) += (gr + i gi) sum_J p_J(r) cnl_in[J][A], then
// cnl_out[J][A] = ekb_h3 sum_k p_J(k) out_A(idx_J(k)) of the fixed values.
// Points covered by one sphere are fixed in place by that sphere's pass;
// points covered by several are written by the last workgroup of each
// orbital group to finish (each pass computes their fixed value for its own
// sum without writing it), so every sum has a fixed order.  Needs t.ovc
// zeroed (launch_kb_tables does it; each launch leaves it zero).
template <typename T>
hipError_t launch_kb_fixup_gather(cx_t<T>* out, int64_t stride, int n_orb, int n_ions, KbTables t,
                                  const cx_t<T>* cnl_in, double gr, double gi, double ekb_h3, cx_t<T>* cnl_out,
                                  hipStream_t s);
// The same pass for up to KB_BATCH systems of a batch in one launch (each
// with n_ions >= 1; gr = 0 as in the Horner stages; b0 is set by the
// launcher).  Every system's arithmetic is that of its own launch.
constexpr int KB_BATCH = 16;
template <typename T>
struct BatchKbSys {
    cx_t<T>* out;
    const cx_t<T>* cnl_in;
    cx_t<T>* cnl_out;
    KbTables t;
    int64_t stride;
    int n_orb, n_ions, b0;
    T gi, scale;
};
template <typename T>
struct BatchKbArgs {
    BatchKbSys<T> sys[KB_BATCH];
    int n_sys;
};
template <typename T>
hipError_t launch_batch_kb_fixup_gather(BatchKbArgs<T> a, hipStream_t s);
// the same with the split-bf16 MFMA contraction (FP32 orbitals)
hipError_t launch_kb_fixup_gather_bf16x3(float2* out, int64_t stride, int n_orb, int n_ions, KbTables t,
                                         const float2* cnl_in, double gr, double gi, double ekb_h3, float2* cnl_out,
                                         hipStream_t s);

// the same contraction for FP32 orbitals as split-bf16 (bf16x3) MFMA with
// FP32 accumulation
hipError_t launch_kb_gather_bf16x3(const float2* u, int64_t stride, int n_orb, int n_ions, KbTables t,
                                   double ekb_h3, float2* cnl, hipStream_t s);

// the contraction and its three force columns of FP32 orbitals by split-bf16
// MFMA (FP32 accumulation): cnl[J][A] = h^3 sum p psi, dnl[J][A][a] =
// h^3 sum (r - R_J)_a p psi; then in FP64 fnl[J] = -2 f E_KB / s^2
// sum_A Re(conj(c) d), enl_part[J] = f E_KB sum_A |c|^2
hipError_t launch_kb_forces_bf16x3(const float2* psi, int64_t stride, int n_orb, int n_ions, KbTables t,
                                   const double* pos, const KbGeom& g, int nx, int ny, double occ, double ekb,
                                   float2* cnl, float2* dnl, double* fnl, double* enl_part, hipStream_t s);

// nonlocal forces and energy, FP64 accumulation:
// fnl[J][3] = -2 f E_KB sum_A Re(conj(c_JA) d_JA); enl_part[J] = f E_KB sum_A |c_JA|^2,
// d_JA = d c_JA / d R_J: form 0 the analytic projector derivative
// h^3 sum (r - R_J)/s^2 p_J psi_A, form 1 the wave-function-gradient form
// h^3 sum p_J grad psi_A (8th-order finite differences)
// scratch: [n_ions][ceil(n_orb/16)][4] doubles
template <typename T>
hipError_t launch_kb_forces(const cx_t<T>* psi, int64_t stride, int n_orb, int n_ions,
                            KbTables t, const double* pos, const KbGeom& g,
                            int nx, int ny, int nz, int form, double occ, double ekb,
                            double* fnl, double* enl_part, double* scratch, hipStream_t s);

// rho[i] = occ * sum_A |psi_A[i]|^2 (FP64)
template <typename T>
hipError_t launch_density(const cx_t<T>* psi, int64_t stride, int n_orb, int64_t N,
                          double occ, double* rho, hipStream_t s);

}  // namespace me

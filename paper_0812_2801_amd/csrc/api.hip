// Host runtime and C ABI: workspace planning, rocFFT plans, and the
// orchestration of one modified-Ehrenfest step (sec. 5.1): ions moved by
// velocity Verlet, the AETRS propagator of eq. (aetrs) as two fourth-order
// Taylor exponentials evaluated in Horner form, then the density, Hartree /
// exchange, and the forces at the new positions.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "../../include/modehr.h"
#include "common.hpp"
#include "fields.hpp"
#include "adjoint.hpp"
#include "cp.hpp"
#include "toy.hpp"
#include "finite.hpp"

using namespace me;

namespace {

thread_local std::string g_init_error;

}  // namespace

// error text of a call without a handle (me_last_error(NULL)), for the other
// source files of the library
void me::set_thread_error(const std::string& text) { g_init_error = text; }

namespace {

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct Carver {
    size_t off = 0;
    char* base = nullptr;
    template <typename P>
    P* take(size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return base ? reinterpret_cast<P*>(base + o) : nullptr;
    }
};

// Host-side Ewald set-up: splitting, real-space cutoff, reciprocal vectors.
struct EwaldHost {
    double L = 0, eta = 0, rc = 0, e_const = 0;
    int nmax = 0;
    std::vector<double> gv, wv;
};

EwaldHost ewald_setup(double L, const std::vector<double>& z) {
    EwaldHost e;
    e.L = L;
    e.eta = 5.0 / L;
    const double tol = 1e-17;
    double rc = 1.0;
    while (std::erfc(e.eta * rc) > tol) rc *= 1.1;
    e.rc = rc;
    e.nmax = (int)std::ceil(rc / L) + 1;
    const double gc = 2.0 * e.eta * std::sqrt(-std::log(tol));
    const int mmax = (int)std::ceil(gc * L / (2.0 * M_PI));
    for (int i = -mmax; i <= mmax; ++i)
        for (int j = -mmax; j <= mmax; ++j)
            for (int k = -mmax; k <= mmax; ++k) {
                if (!i && !j && !k) continue;
                const double gx = 2 * M_PI * i / L, gy = 2 * M_PI * j / L, gz = 2 * M_PI * k / L;
                const double g2 = gx * gx + gy * gy + gz * gz;
                if (g2 >= gc * gc) continue;
                e.gv.push_back(gx); e.gv.push_back(gy); e.gv.push_back(gz);
                e.wv.push_back(std::exp(-g2 / (4.0 * e.eta * e.eta)) / g2);
            }
    double z2 = 0, zs = 0;
    for (double q : z) { z2 += q * q; zs += q; }
    const double omega = L * L * L;
    e.e_const = -e.eta / std::sqrt(M_PI) * z2 - M_PI * zs * zs / (2.0 * omega * e.eta * e.eta);
    return e;
}

struct Geometry {
    int nx, ny, nz;
    int64_t N, stride;
    int n_orb, n_ions;
    bool f64;
    size_t bc;        // bytes per complex
    size_t br;        // bytes per real of the compute precision
    int px, ty, nyt, zchunk, nzc;
    int tx, nxt;       // stencil tile width (nx: whole rows) and x-tiles
    int py;            // whole-row tiles: rows per thread
    int64_t norm_cap;  // norm partials per orbital (this kernel's tiles, or a batch's)
    int kcap;
    int64_t ucap;      // upper bound of projector-covered grid points
    int64_t nscan;     // point-numbering blocks
    int m;
    int64_t nhalf;    // half-spectrum size
    int floc_chunks;
    int64_t nblk256;  // 256-point blocks of the grid
    size_t fft_work;
    bool finite;          // union-of-spheres box, free-space potentials
    int64_t npad, nhalf2; // doubled grid: points, complex half-spectrum
    size_t fft_work2;
    int ewald_ng;
    bool adjoint;
    int taylor;
    int etrs;          // ETRS corrections of the second exponential (0: AETRS)
};

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

// x-points per thread of the stencil kernel
int choose_px(int nx, bool f64) { return 1; }

// LDS of one stencil workgroup: at most 64 KiB
constexpr size_t STENCIL_LDS_MAX = 64 * 1024;

// y-rows per stencil workgroup, among the candidates that divide ny and keep
// the workgroup within 1024 threads and its two LDS tiles within
// STENCIL_LDS_MAX.  Workgroups of at most 768 threads leave room for two per
// CU at the kernel's register use, so the largest such tile of at least 8
// rows (one y-halo row per thread) comes first; FP32 then accepts shorter
// tiles of at most 768 threads (two halo rows per thread fit its registers),
// and otherwise the largest tile is taken.  Measured on 64^3, 96^3 and 128^3.
int choose_ty(int nx, int ny, int px, size_t bc) {
    const int nxt = nx / px;
    const int cap = env_int("MODEHR_TY", 16);
    auto ok = [&](int ty) {
        return ty <= cap && ny % ty == 0 && (int64_t)nxt * ty <= 1024 &&
               stencil_lds_bytes(ty, nx, bc) <= STENCIL_LDS_MAX;
    };
    for (int ty : {16, 8})
        if (ok(ty) && nxt * ty <= 768) return ty;
    if (bc == 8)
        for (int ty : {4, 2, 1})
            if (ok(ty) && nxt * ty <= 768) return ty;
    for (int ty : {16, 8, 4, 2, 1})
        if (ok(ty)) return ty;
    return -1;
}

// Stencil tile.  FP64, and FP32 rows of up to 96 points: whole x-rows,
// choose_ty rows, one row per thread.  FP32 rows of 97-256 points: whole
// rows, tiles of 8 rows with two rows per thread (4 thread rows, so 128-point
// rows give 512-thread workgroups, two per CU at the kernel's 120 VGPRs);
// measured at 128^3: 4.18 ms per three-stream stage against 4.43 for x-tiles
// and 4.35 for 4 whole rows of one per thread.  Wider FP32 rows: x-tiles of 64
// points and 12 rows (an x-halo of 4 + 4 points in LDS).  MODEHR_TX /
// MODEHR_TY select an x-tile shape (64x12, 48x16, 32x24, 16x8; MODEHR_TX=0:
// whole rows, one per thread) and MODEHR_PY=2 / MODEHR_PY_TY two rows per
// thread with 8 or 16 rows per tile (measurements and tests).
void choose_tile(int nx, int ny, int px, size_t bc, int* tx, int* ty, int* py) {
    *py = 1;
    const char* ev = std::getenv("MODEHR_TX");
    if (ev && *ev) {
        const int ftx = std::atoi(ev);
        if (ftx > 0 && ftx < nx) {
            *tx = ftx;
            *ty = env_int("MODEHR_TY", 12);
            return;
        }
        *tx = nx;
        *ty = choose_ty(nx, ny, px, bc);
        return;
    }
    const int fpy = env_int("MODEHR_PY", 0);
    const int pty = fpy == 2 ? env_int("MODEHR_PY_TY", 8) : 8;
    const bool py_fits = (pty == 8 || pty == 16) && ny % pty == 0 && nx * pty / 2 <= 1024 &&
                         stencil_lds_bytes(pty, nx, bc) <= STENCIL_LDS_MAX;
    if (py_fits && (fpy == 2 || (fpy == 0 && bc == 8 && nx > 96))) {
        *tx = nx;
        *ty = pty;
        *py = 2;
        return;
    }
    if (bc == 8 && nx > 96) {
        *tx = 64;
        *ty = 12;
        return;
    }
    *tx = nx;
    *ty = choose_ty(nx, ny, px, bc);
}

int choose_zchunk(int nz, int64_t base_blocks) {
    const int forced = env_int("MODEHR_ZCHUNK", 0);
    if (forced > 0 && nz % forced == 0) return forced;
    // the largest divisor of nz (>= 8 planes, or nz) giving >= 1024 workgroups
    int best = nz;
    for (int zc = nz; zc >= 1; --zc) {
        if (nz % zc) continue;
        if (zc < 8 && zc != nz) break;
        best = zc;
        if (base_blocks * (nz / zc) >= 1024) break;
    }
    return best;
}

me_status validate(const me_params* p, std::string& err) {
    if (!p) { err = "params is NULL"; return ME_EINVAL; }
    for (int a = 0; a < 3; ++a)
        if (p->n[a] < 8 || p->n[a] > 1024) { err = "grid size must be in [8, 1024] along every axis"; return ME_EINVAL; }
    if (!(p->h > 0) || !std::isfinite(p->h)) { err = "h must be positive"; return ME_EINVAL; }
    if (p->n_ions < 0 || p->n_ions > 2048) { err = "n_ions out of range [0, 2048]"; return ME_EINVAL; }
    if (p->n_ions > 0 && (!p->pos || !p->mass || !p->zval)) { err = "pos/mass/zval must not be NULL"; return ME_EINVAL; }
    for (int J = 0; J < p->n_ions; ++J) {
        if (!(p->mass[J] > 0)) { err = "masses must be positive"; return ME_EINVAL; }
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(p->pos[3 * J + c])) { err = "positions must be finite"; return ME_EINVAL; }
    }
    if (!(p->loc_a > 0) || !(p->kb_sigma > 0) || !(p->kb_rcut > 0)) { err = "loc_a, kb_sigma, kb_rcut must be positive"; return ME_EINVAL; }
    for (int a = 0; a < 3; ++a)
        if (!(2.0 * p->kb_rcut < p->n[a] * p->h)) { err = "projector sphere does not fit: need 2*kb_rcut < L"; return ME_EINVAL; }
    if (p->n_orb < 1) { err = "n_orb must be >= 1"; return ME_EINVAL; }
    if (!(p->mu > 0) || !std::isfinite(p->dt) || p->dt == 0.0) { err = "mu must be positive and dt nonzero"; return ME_EINVAL; }
    if (p->taylor_order < 1 || p->taylor_order > MAX_TAYLOR) { err = "taylor_order must be in [1, 8]"; return ME_EINVAL; }
    if (p->precision < ME_F64 || p->precision > ME_F32_BF16X3) { err = "unknown precision"; return ME_EINVAL; }
    if (p->enable_adjoint && !p->freeze_ions) { err = "the adjoint needs frozen ions"; return ME_EUNSUPPORTED; }
    if (p->nl_force_form != 0 && p->nl_force_form != 1) { err = "nl_force_form must be 0 or 1"; return ME_EINVAL; }
    if (p->etrs_iterations < 0 || p->etrs_iterations > 8) { err = "etrs_iterations must be in [0, 8]"; return ME_EINVAL; }
    if (p->etrs_iterations > 0 && p->enable_adjoint) { err = "the adjoint is defined for AETRS"; return ME_EUNSUPPORTED; }
    if (!(p->finite_radius >= 0.0) || !std::isfinite(p->finite_radius)) { err = "finite_radius must be >= 0"; return ME_EINVAL; }
    if (p->finite_radius > 0.0) {
        if (p->enable_adjoint) { err = "the adjoint runs on the periodic cube"; return ME_EUNSUPPORTED; }
        if (p->n_ions < 1) { err = "a finite box needs ions"; return ME_EINVAL; }
        if (!(p->kb_rcut < p->finite_radius)) { err = "the projector spheres must fit in the box: kb_rcut < finite_radius"; return ME_EINVAL; }
        for (int J = 0; J < p->n_ions; ++J)
            for (int c = 0; c < 3; ++c) {
                const double lo = p->pos[3 * J + c] - p->finite_radius, hi = p->pos[3 * J + c] + p->finite_radius;
                if (lo < 4.0 * p->h || hi > (p->n[c] - 5) * p->h) {
                    err = "the finite box must keep 4 grid points from every face of the cube";
                    return ME_EINVAL;
                }
            }
    }
    const bool f64 = p->precision == ME_F64;
    const int px = choose_px(p->n[0], f64);
    if (choose_ty(p->n[0], p->n[1], px, f64 ? 16 : 8) < 0) { err = "grid x extent too large for one workgroup row"; return ME_EUNSUPPORTED; }
    return ME_OK;
}

Geometry make_geometry(const me_params* p) {
    Geometry g{};
    g.nx = p->n[0]; g.ny = p->n[1]; g.nz = p->n[2];
    g.N = (int64_t)g.nx * g.ny * g.nz;
    g.stride = (int64_t)align_up((size_t)g.N, 64);
    g.n_orb = p->n_orb;
    g.n_ions = p->n_ions;
    g.f64 = p->precision == ME_F64;
    g.bc = g.f64 ? 16 : 8;
    g.br = g.f64 ? 8 : 4;
    g.px = choose_px(g.nx, g.f64);
    choose_tile(g.nx, g.ny, g.px, g.bc, &g.tx, &g.ty, &g.py);
    g.nxt = (g.nx + g.tx - 1) / g.tx;
    g.nyt = (g.ny + g.ty - 1) / g.ty;
    g.zchunk = choose_zchunk(g.nz, (int64_t)g.n_orb * g.nxt * g.nyt);
    g.nzc = g.nz / g.zchunk;
    g.norm_cap = std::max<int64_t>((int64_t)g.nxt * g.nyt * g.nzc, 4 * (int64_t)g.ny);
    const int m = (int)std::ceil(p->kb_rcut / p->h);
    g.m = m;
    int kc = 1;
    for (int a = 0; a < 3; ++a) {
        kc *= std::min(2 * m + 2, p->n[a]);
    }
    g.kcap = kc;
    g.ucap = std::max<int64_t>(1, std::min<int64_t>(g.N, (int64_t)std::max(1, g.n_ions) * g.kcap));
    g.nscan = (g.N + 1023) / 1024;
    g.nhalf = (int64_t)(g.nx / 2 + 1) * g.ny * g.nz;
    g.floc_chunks = local_force_chunks(g.N);
    g.nblk256 = (g.N + 255) / 256;
    g.fft_work = (size_t)(2 * g.nhalf) * 16;
    g.adjoint = p->enable_adjoint != 0;
    g.etrs = p->etrs_iterations;
    g.taylor = p->taylor_order;
    g.finite = p->finite_radius > 0.0;
    g.npad = g.finite ? 8 * g.N : 0;
    g.nhalf2 = g.finite ? (int64_t)(g.nx + 1) * (2 * g.ny) * (2 * g.nz) : 0;
    g.fft_work2 = g.finite ? (size_t)(2 * g.nhalf2) * 16 : 0;
    return g;
}

}  // namespace

// the CP overlaps (N_W x N_W, sums over every grid point) run as this many
// batched GEMMs over slices of the points, plus one for the remainder
constexpr int CP_KSPLIT = 256;

struct Layout {
    void *psi, *bufA, *bufB, *veff0, *veff1, *cnl;
    void* cnl2;                 // the next stage's c_JA when a fix-up and a gather share a pass
    void* dnl;                  // split-bf16 force gather: [n_ions][n_orb][3] complex FP32
    double *vloc_cur, *vloc_next, *vstatic, *hist[3], *rho, *vh;
    double2 *rhok, *spec, *phase, *phaseT, *ewald_sg;
    void* fft_work;
    uint8_t* mask;              // finite box: 1 inside
    int2* zr;                   // finite box: per y-tile plane range of the box (Horner stages)
    double *rpad_in, *rpad_out, *gk;
    double2* cpad;
    void* fft_work2;
    double *pos, *pos_next, *vel, *frc, *mass, *zval;
    int32_t* tidx[2];
    void* tp[2];
    int32_t *tmap[2], *tpts[2], *tcnt[2], *tion[2], *tnslots[2], *tflag[2], *tblk[2];
    void* tpl[2];
    int32_t* tcount[2];
    uint8_t* tov[2];            // per table point: covered by more than one sphere
    int32_t *tovl[2], *tovn[2]; // slots covered by more than one sphere, and their count
    int32_t* tovc[2];           // counters of the fused fix-up + gather pass
    double *fnl, *enl_part, *kbf_part, *floc_part, *floc, *fion, *eion_part, *erec_part;
    double *ewald_gv, *ewald_wv, *ewald_part;
    double *norm_part, *fix_part, *norms, *kin_part, *hxc_part, *loc_part, *rep, *scal0;
    // adjoint (frozen ions): forward intermediates of both exponentials, the
    // half-step and next orbitals, adjoint orbitals, and FP64 grid buffers
    void* inter[2][MAX_TAYLOR];
    void *psi_half, *psi_next, *lamA, *lamB, *ubA, *ubB;
    void* etrs_half;     // ETRS: the orbitals after the first exponential
    double *vbar[4], *wbar1, *wbar2, *gfine, *rhobar_T, *rhobar, *hv, *dpart, *scal;
    // Car-Parrinello comparison step: overlap matrices A, B, Q and the solve
    // scratch in FP64, the rotations X, Y in the orbital precision, the
    // K-split partial overlaps, fictitious kinetic energy partials
    double2 *cpA, *cpB, *cpQ, *cpX64, *cpR64;
    void *cpX, *cpY, *cp_gpart;
    double *cp_part, *cp_info, *fict_part;
    size_t total;
};

static Layout carve(const Geometry& g, char* base) {
    Carver c;
    c.base = base;
    Layout L{};
    const size_t orb = (size_t)g.n_orb * g.stride * g.bc;
    L.psi = c.take<void>(orb);
    L.bufA = c.take<void>(orb);
    L.bufB = c.take<void>(orb);
    L.veff0 = c.take<void>(g.N * g.br);
    L.veff1 = c.take<void>(g.N * g.br);
    L.cnl = c.take<void>((size_t)std::max(1, g.n_ions) * g.n_orb * g.bc);
    L.cnl2 = c.take<void>((size_t)std::max(1, g.n_ions) * g.n_orb * g.bc);
    L.dnl = c.take<void>((size_t)std::max(1, g.n_ions) * g.n_orb * 3 * g.bc);
    L.vloc_cur = c.take<double>(g.N * 8);
    L.vloc_next = c.take<double>(g.N * 8);
    L.vstatic = c.take<double>(g.N * 8);
    for (int i = 0; i < 3; ++i) L.hist[i] = c.take<double>(g.N * 8);
    L.rho = c.take<double>(g.N * 8);
    L.vh = c.take<double>(g.N * 8);
    L.rhok = c.take<double2>(g.nhalf * 16);
    L.spec = c.take<double2>(g.nhalf * 16);
    L.phase = c.take<double2>((size_t)std::max(1, g.n_ions) * (g.nx + g.ny + g.nz) * 16);
    L.phaseT = c.take<double2>((size_t)std::max(1, g.n_ions) * (g.nx + g.ny + g.nz) * 16);
    L.fft_work = c.take<void>(g.fft_work);
    if (g.finite) {
        L.mask = c.take<uint8_t>(g.N);
        L.zr = c.take<int2>((size_t)g.nyt * sizeof(int2));
        L.rpad_in = c.take<double>(g.npad * 8);
        L.rpad_out = c.take<double>(g.npad * 8);
        L.cpad = c.take<double2>(g.nhalf2 * 16);
        L.gk = c.take<double>(g.nhalf2 * 8);
        L.fft_work2 = c.take<void>(g.fft_work2);
    }
    const size_t ion3 = (size_t)std::max(1, g.n_ions) * 3 * 8;
    L.pos = c.take<double>(ion3);
    L.pos_next = c.take<double>(ion3);
    L.vel = c.take<double>(ion3);
    L.frc = c.take<double>(ion3);
    L.mass = c.take<double>(ion3 / 3);
    L.zval = c.take<double>(ion3 / 3);
    for (int t = 0; t < 2; ++t) {
        L.tidx[t] = c.take<int32_t>((size_t)std::max(1, g.n_ions) * g.kcap * 4);
        L.tp[t] = c.take<void>((size_t)std::max(1, g.n_ions) * g.kcap * g.br);
        L.tmap[t] = c.take<int32_t>((size_t)g.N * 4);
        L.tpts[t] = c.take<int32_t>((size_t)g.ucap * 4);
        L.tcnt[t] = c.take<int32_t>((size_t)g.ucap * 4);
        L.tion[t] = c.take<int32_t>((size_t)g.ucap * NL_KMAX * 4);
        L.tpl[t] = c.take<void>((size_t)g.ucap * NL_KMAX * g.br);
        L.tnslots[t] = c.take<int32_t>(4);
        L.tflag[t] = c.take<int32_t>(4);
        L.tblk[t] = c.take<int32_t>((size_t)(g.nscan + 1) * 4);
        L.tcount[t] = c.take<int32_t>((size_t)std::max(1, g.n_ions) * 4);
        L.tov[t] = c.take<uint8_t>((size_t)std::max(1, g.n_ions) * g.kcap);
        L.tovl[t] = c.take<int32_t>((size_t)g.ucap * 4);
        L.tovn[t] = c.take<int32_t>(4);
        L.tovc[t] = c.take<int32_t>((size_t)((g.n_orb + 3) / 4) * 4);
    }
    L.fnl = c.take<double>(ion3);
    L.enl_part = c.take<double>(ion3 / 3);
    L.kbf_part = c.take<double>((size_t)std::max(1, g.n_ions) * ((g.n_orb + 15) / 16) * 4 * 8);
    L.floc_part = c.take<double>((size_t)std::max(1, g.n_ions) * g.floc_chunks * 3 * 8);
    L.fion = c.take<double>(ion3);
    L.floc = c.take<double>(ion3);
    L.eion_part = c.take<double>(ion3 / 3);
    L.ewald_sg = c.take<double2>((size_t)std::max(1, g.ewald_ng) * 16);
    L.erec_part = c.take<double>((size_t)ewald_sg_blocks(g.ewald_ng) * 8);
    L.ewald_gv = c.take<double>((size_t)std::max(1, g.ewald_ng) * 3 * 8);
    L.ewald_wv = c.take<double>((size_t)std::max(1, g.ewald_ng) * 8);
    L.ewald_part = c.take<double>(ewald_scratch_doubles(g.n_ions) * 8);
    L.norm_part = c.take<double>((size_t)g.n_orb * g.norm_cap * 8);
    L.fix_part = c.take<double>((size_t)g.n_orb * fixup_blocks(g.ucap) * 8);
    L.kin_part = c.take<double>((size_t)g.n_orb * g.nxt * g.nyt * g.nzc * 8);
    L.norms = c.take<double>((size_t)g.n_orb * 8);
    L.hxc_part = c.take<double>((size_t)g.nblk256 * 3 * 8);
    L.loc_part = c.take<double>((size_t)g.nblk256 * 8);
    L.rep = c.take<double>(SLOT_COUNT * 8);
    L.scal0 = c.take<double>(64);
    const size_t mat = (size_t)g.n_orb * g.n_orb;
    L.cpA = c.take<double2>(mat * 16);
    L.cpB = c.take<double2>(mat * 16);
    L.cpQ = c.take<double2>(mat * 16);
    L.cpX64 = c.take<double2>(mat * 16);
    L.cpR64 = c.take<double2>(mat * 16);
    L.cpX = c.take<void>(mat * g.bc);
    L.cpY = c.take<void>(mat * g.bc);
    L.cp_gpart = c.take<void>((size_t)(CP_KSPLIT + 1) * mat * g.bc);
    L.cp_part = c.take<double>((size_t)cp_solve_blocks(g.n_orb) * 8);
    L.cp_info = c.take<double>(2 * 8);
    L.fict_part = c.take<double>((size_t)g.nblk256 * 8);
    if (g.etrs > 0) L.etrs_half = c.take<void>(orb);
    if (g.adjoint) {
        for (int e = 0; e < 2; ++e)
            for (int k = 0; k < g.taylor - 1; ++k) L.inter[e][k] = c.take<void>(orb);
        L.psi_half = c.take<void>(orb);
        L.psi_next = c.take<void>(orb);
        L.lamA = c.take<void>(orb);
        L.lamB = c.take<void>(orb);
        L.ubA = c.take<void>(orb);
        L.ubB = c.take<void>(orb);
        for (int i = 0; i < 4; ++i) L.vbar[i] = c.take<double>(g.N * 8);
        L.wbar1 = c.take<double>(g.N * 8);
        L.wbar2 = c.take<double>(g.N * 8);
        L.gfine = c.take<double>(g.N * 8);
        L.rhobar_T = c.take<double>(g.N * 8);
        L.rhobar = c.take<double>(g.N * 8);
        L.hv = c.take<double>(g.N * 8);
        L.dpart = c.take<double>((size_t)g.nblk256 * 8);
        L.scal = c.take<double>(64);
    }
    L.total = c.off;
    return L;
}

struct me_system {
    me_params prm{};
    std::vector<double> pos0, vel0, mass, zval;
    std::vector<int2> zr_host;      // finite box: per y-tile plane ranges
    Geometry g{};
    Layout w{};
    hipStream_t stream = nullptr;
    KbGeom geo{};
    EwaldHost ew;
    EwaldPlan ewp{};
    rocfft_plan r2c = nullptr, c2r = nullptr;
    rocfft_execution_info info = nullptr;
    rocfft_plan r2c2 = nullptr, c2r2 = nullptr;      // doubled grid (finite box)
    rocfft_execution_info info2 = nullptr;
    int tab_cur = 0;
    int hist_count = 0, hist_newest = 0;
    int norm_tiles = 0;          // tiles per orbital of the last norm partials
    bool has_state = false;
    bool static_set = false;
    int64_t step = 0;
    std::string err;
    // timing of the Horner-stage stencil launches
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> ev_bytes;
    std::vector<int> ev_streams;    // complex streams of each timed launch (2: first stage, 3: others)
    std::vector<hipEvent_t> ev_pool;
    double rep_host[SLOT_COUNT];
    // adjoint bookkeeping
    bool adj_ready = false;
    bool adj_pending_final = false;
    // Car-Parrinello comparison step: rocBLAS handle (created by me_cp_begin),
    // fictitious mass, time step; cp_ready while bufA holds the orbital
    // velocities and bufB H psi of the current state
    rocblas_handle blas = nullptr;
    double mu_cp = 0.0, dt_cp = 0.0;
    bool cp_ready = false;
    // Work of an MD step that the first exponential does not wait for (ions
    // moved, V_loc and projector tables at R(t+dt), v_eff of the second
    // exponential, the Ewald sum) runs on `side`, and the nonlocal forces run
    // there beside the density and Hartree chain; events order both streams
    // (default priority, created at init; null when MODEHR_OVERLAP=0).
    hipStream_t side = nullptr;
    rocfft_execution_info info_side = nullptr;   // FFTs enqueued on `side`
    hipEvent_t ev_fork[2] = {nullptr, nullptr}, ev_join[2] = {nullptr, nullptr};
};

namespace {

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            sys->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return ME_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

#define FFTCHK(expr)                                                                   \
    do {                                                                               \
        rocfft_status e_ = (expr);                                                     \
        if (e_ != rocfft_status_success) {                                             \
            sys->err = std::string(#expr) + ": rocfft status " + std::to_string((int)e_); \
            return ME_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

#define CHK(expr)                                                                      \
    do {                                                                               \
        me_status s_ = (expr);                                                         \
        if (s_ != ME_OK) return s_;                                                    \
    } while (0)

// Enqueue the launches of a scope on the side stream: the helpers take
// sys->stream and sys->info, so both are switched and restored on exit.
struct OnSide {
    me_system* s;
    hipStream_t st;
    rocfft_execution_info inf;
    explicit OnSide(me_system* s_) : s(s_), st(s_->stream), inf(s_->info) {
        s->stream = s->side;
        s->info = s->info_side;
    }
    ~OnSide() {
        s->stream = st;
        s->info = inf;
    }
};

KbTables tables(me_system* sys, int t) {
    KbTables k{};
    k.idx = sys->w.tidx[t];
    k.p = sys->w.tp[t];
    k.count = sys->w.tcount[t];
    k.kcap = sys->g.kcap;
    k.m = sys->g.m;
    k.map = sys->w.tmap[t];
    k.pts = sys->w.tpts[t];
    k.cnt = sys->w.tcnt[t];
    k.ion = sys->w.tion[t];
    k.pl = sys->w.tpl[t];
    k.nslots = sys->w.tnslots[t];
    k.flag = sys->w.tflag[t];
    k.blk = sys->w.tblk[t];
    k.ov = sys->w.tov[t];
    k.ovl = sys->w.tovl[t];
    k.ovn = sys->w.tovn[t];
    k.ovc = sys->w.tovc[t];
    k.novc = (sys->g.n_orb + 3) / 4;
    k.ucap = sys->g.ucap;
    return k;
}

double Lx(const me_system* s) { return s->g.nx * s->prm.h; }

me_status fft_r2c(me_system* sys, double* in, double2* out) {
    void* i[1] = {in};
    void* o[1] = {out};
    FFTCHK(rocfft_execute(sys->r2c, i, o, sys->info));
    return ME_OK;
}

me_status fft_c2r(me_system* sys, double2* in, double* out) {
    void* i[1] = {in};
    void* o[1] = {out};
    FFTCHK(rocfft_execute(sys->c2r, i, o, sys->info));
    return ME_OK;
}

// free-space Hartree potential of w.rho into w.vh: the charge on the
// corner block of the doubled grid (zero elsewhere), times the spectrum of
// the Coulomb kernel, back, and the corner block taken
me_status hartree_free(me_system* sys) {
    const Geometry& g = sys->g;
    HIPCHK(launch_pad(sys->w.rho, g.nx, g.ny, g.nz, sys->w.rpad_in, sys->stream));
    void* i1[1] = {sys->w.rpad_in};
    void* o1[1] = {sys->w.cpad};
    FFTCHK(rocfft_execute(sys->r2c2, i1, o1, sys->info2));
    HIPCHK(launch_green_multiply(sys->w.cpad, sys->w.gk, g.nhalf2, sys->stream));
    void* i2[1] = {sys->w.cpad};
    void* o2[1] = {sys->w.rpad_out};
    FFTCHK(rocfft_execute(sys->c2r2, i2, o2, sys->info2));
    HIPCHK(launch_unpad(sys->w.rpad_out, g.nx, g.ny, g.nz, sys->w.vh, sys->stream));
    return ME_OK;
}

// Finite box (finite_radius > 0): doubled-grid FFT plans, the box mask at
// the initial positions, the per-y-tile plane ranges of the Horner stages and
// the spectrum of the Coulomb kernel.  On failure sys->err is set; the
// caller destroys what was created.
me_status finite_setup(me_system* sys, const me_params* p) {
    // doubled-grid plans, the box mask at the initial positions and
    // the spectrum of the Coulomb kernel (h^3 / (8N) folds in the
    // inverse transform's normalisation and the quadrature weight)
    const Geometry& g = sys->g;
    size_t len2[3] = {(size_t)(2 * g.nx), (size_t)(2 * g.ny), (size_t)(2 * g.nz)};
    if (rocfft_plan_create(&sys->r2c2, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                           rocfft_precision_double, 3, len2, 1, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&sys->c2r2, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                           rocfft_precision_double, 3, len2, 1, nullptr) != rocfft_status_success) {
        sys->err = "rocfft_plan_create failed (doubled grid)";
        return ME_EDEVICE;
    }
    size_t v1 = 0, v2 = 0;
    rocfft_plan_get_work_buffer_size(sys->r2c2, &v1);
    rocfft_plan_get_work_buffer_size(sys->c2r2, &v2);
    if (std::max(v1, v2) > g.fft_work2) {
        sys->err = "rocFFT work buffer (doubled grid) larger than reserved";
        return ME_EUNSUPPORTED;
    }
    if (rocfft_execution_info_create(&sys->info2) != rocfft_status_success ||
        rocfft_execution_info_set_stream(sys->info2, sys->stream) != rocfft_status_success ||
        (std::max(v1, v2) > 0 &&
         rocfft_execution_info_set_work_buffer(sys->info2, sys->w.fft_work2, g.fft_work2) !=
             rocfft_status_success)) {
        sys->err = "rocfft execution info failed (doubled grid)";
        return ME_EDEVICE;
    }
    HIPCHK(launch_box_mask(sys->w.pos, g.n_ions, g.nx, g.ny, g.nz, p->h, p->finite_radius, sys->w.mask,
                           sys->stream));
    // per y-tile plane range holding every box point of its rows (a
    // superset: the chord of each sphere at the row, one plane of
    // margin); the Horner stages march only there, so the stage
    // buffers start at zero and stay zero outside the box
    sys->zr_host.assign(g.nyt, make_int2(0, 0));
    for (int t = 0; t < g.nyt; ++t) {
        int lo = g.nz, hi = 0;
        for (int y = t * g.ty; y < std::min(g.ny, (t + 1) * g.ty); ++y)
            for (int J = 0; J < g.n_ions; ++J) {
                const double dy = y * p->h - sys->pos0[3 * J + 1];
                const double rem = p->finite_radius * p->finite_radius - dy * dy;
                if (rem < 0.0) continue;
                const double c = std::sqrt(rem), Z = sys->pos0[3 * J + 2];
                lo = std::min(lo, std::max(0, (int)std::floor((Z - c) / p->h) - 1));
                hi = std::max(hi, std::min(g.nz, (int)std::ceil((Z + c) / p->h) + 2));
            }
        sys->zr_host[t] = make_int2(lo, std::max(lo, hi));
    }
    HIPCHK(hipMemcpyAsync(sys->w.zr, sys->zr_host.data(), (size_t)g.nyt * sizeof(int2), hipMemcpyHostToDevice,
                           sys->stream));
    const size_t ob = (size_t)g.n_orb * g.stride * g.bc;
    HIPCHK(hipMemsetAsync(sys->w.bufA, 0, ob, sys->stream));
    HIPCHK(hipMemsetAsync(sys->w.bufB, 0, ob, sys->stream));
    HIPCHK(hipMemsetAsync(sys->w.rpad_in, 0, g.npad * 8, sys->stream));
    HIPCHK(launch_green_doubled(g.nx, g.ny, g.nz, p->h, sys->w.rpad_out, sys->stream));
    void* gi[1] = {sys->w.rpad_out};
    void* go[1] = {sys->w.cpad};
    if (rocfft_execute(sys->r2c2, gi, go, sys->info2) != rocfft_status_success) {
        sys->err = "rocfft_execute failed (Coulomb kernel)";
        return ME_EDEVICE;
    }
    HIPCHK(launch_green_spectrum(sys->w.cpad, g.nhalf2, p->h * p->h * p->h / (double)g.npad, sys->w.gk,
                                 sys->stream));
    return ME_OK;
}

// V_loc at positions `pos` (device) into `out` (+ the static potential).
// Leaves the phase tables of `pos` in w.phase (periodic cube).
me_status ion_fields(me_system* sys, const double* pos, double* out) {
    const Geometry& g = sys->g;
    if (g.finite) {
        HIPCHK(launch_vloc_free(pos, sys->w.zval, g.n_ions, g.nx, g.ny, g.nz, sys->prm.h, sys->prm.loc_a, out,
                                sys->stream));
        if (sys->static_set) HIPCHK(launch_add(out, sys->w.vstatic, g.N, sys->stream));
        return ME_OK;
    }
    const double L[3] = {g.nx * sys->prm.h, g.ny * sys->prm.h, g.nz * sys->prm.h};
    HIPCHK(launch_phases(pos, g.n_ions, g.nx, g.ny, g.nz, L, sys->w.phase, sys->w.phaseT, sys->stream));
    HIPCHK(launch_vloc_spectrum(sys->w.phase, sys->w.phaseT, sys->w.zval, g.n_ions, g.nx, g.ny, g.nz, L,
                                sys->prm.loc_a, sys->w.spec, sys->stream));
    CHK(fft_c2r(sys, sys->w.spec, out));
    if (sys->static_set) HIPCHK(launch_add(out, sys->w.vstatic, g.N, sys->stream));
    return ME_OK;
}

me_status build_tables(me_system* sys, const double* pos, int t) {
    const Geometry& g = sys->g;
    if (g.f64)
        HIPCHK(launch_kb_tables<double>(pos, g.n_ions, g.nx, g.ny, g.nz, sys->geo, tables(sys, t), sys->stream));
    else
        HIPCHK(launch_kb_tables<float>(pos, g.n_ions, g.nx, g.ny, g.nz, sys->geo, tables(sys, t), sys->stream));
    return ME_OK;
}

// density, Hartree + exchange of the current orbitals; pushes v_Hxc onto the
// history (or, with push = false, only refreshes the energy partials)
me_status density_vhxc(me_system* sys, bool energy, bool push = true) {
    const Geometry& g = sys->g;
    const double L[3] = {g.nx * sys->prm.h, g.ny * sys->prm.h, g.nz * sys->prm.h};
    if (g.f64)
        HIPCHK(launch_density<double>((const double2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->prm.occ, sys->w.rho, sys->stream));
    else
        HIPCHK(launch_density<float>((const float2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->prm.occ, sys->w.rho, sys->stream));
    if (g.finite) {
        CHK(hartree_free(sys));
    } else {
        CHK(fft_r2c(sys, sys->w.rho, sys->w.rhok));
        HIPCHK(launch_hartree_spectrum(sys->w.rhok, g.nx, g.ny, g.nz, L, sys->w.spec, sys->stream));
        CHK(fft_c2r(sys, sys->w.spec, sys->w.vh));
    }
    if (!push) {
        HIPCHK(launch_vhxc(sys->w.rho, sys->w.vh, g.N, sys->w.vh, energy ? sys->w.hxc_part : nullptr,
                           sys->stream));
        return ME_OK;
    }
    const int slot = sys->hist_count == 0 ? 0 : (sys->hist_newest + 1) % 3;
    HIPCHK(launch_vhxc(sys->w.rho, sys->w.vh, g.N, sys->w.hist[slot], energy ? sys->w.hxc_part : nullptr,
                       sys->stream));
    sys->hist_newest = slot;
    sys->hist_count = std::min(3, sys->hist_count + 1);
    return ME_OK;
}

// forces at `pos` (phases of `pos` already in w.phase, tables t at pos), in
// three independent parts: local (from the density's spectrum), nonlocal
// (from the orbitals) and ion-ion; partial results in floc_part / floc, fnl /
// enl_part, fion / eion_part
me_status local_forces_part(me_system* sys, const double* pos) {
    const Geometry& g = sys->g;
    const double L[3] = {g.nx * sys->prm.h, g.ny * sys->prm.h, g.nz * sys->prm.h};
    if (g.finite)
        HIPCHK(launch_local_forces_free(sys->w.rho, pos, sys->w.zval, g.n_ions, g.nx, g.ny, g.nz, sys->prm.h,
                                        sys->prm.loc_a, sys->w.floc_part, sys->w.floc, sys->stream));
    else
        HIPCHK(launch_local_forces(sys->w.rhok, sys->w.phaseT, sys->w.zval, g.n_ions, g.nx, g.ny, g.nz, L,
                                   sys->prm.h, sys->prm.loc_a, sys->w.floc_part, sys->w.floc, sys->stream));
    return ME_OK;
}

me_status nl_forces_part(me_system* sys, const double* pos, int t) {
    const Geometry& g = sys->g;
    if (g.f64)
        HIPCHK(launch_kb_forces<double>((const double2*)sys->w.psi, g.stride, g.n_orb, g.n_ions, tables(sys, t), pos,
                                        sys->geo, g.nx, g.ny, g.nz, sys->prm.nl_force_form, sys->prm.occ, sys->prm.kb_energy, sys->w.fnl,
                                        sys->w.enl_part, sys->w.kbf_part, sys->stream));
    else if (sys->prm.precision == ME_F32_BF16X3 && sys->prm.nl_force_form == 0)
        HIPCHK(launch_kb_forces_bf16x3((const float2*)sys->w.psi, g.stride, g.n_orb, g.n_ions, tables(sys, t), pos,
                                       sys->geo, g.nx, g.ny, sys->prm.occ, sys->prm.kb_energy, (float2*)sys->w.cnl,
                                       (float2*)sys->w.dnl, sys->w.fnl, sys->w.enl_part, sys->stream));
    else
        HIPCHK(launch_kb_forces<float>((const float2*)sys->w.psi, g.stride, g.n_orb, g.n_ions, tables(sys, t), pos,
                                       sys->geo, g.nx, g.ny, g.nz, sys->prm.nl_force_form, sys->prm.occ, sys->prm.kb_energy, sys->w.fnl,
                                       sys->w.enl_part, sys->w.kbf_part, sys->stream));
    return ME_OK;
}

me_status ion_forces_part(me_system* sys, const double* pos) {
    const Geometry& g = sys->g;
    if (g.finite)
        HIPCHK(launch_ion_coulomb(pos, sys->w.zval, g.n_ions, sys->w.fion, sys->w.eion_part, sys->stream));
    else
        HIPCHK(launch_ewald(sys->ewp, pos, sys->w.zval, g.n_ions, sys->w.ewald_sg, sys->w.erec_part, sys->w.fion,
                            sys->w.eion_part, sys->w.ewald_part, sys->stream));
    return ME_OK;
}

me_status forces_parts(me_system* sys, const double* pos, int t) {
    CHK(local_forces_part(sys, pos));
    CHK(nl_forces_part(sys, pos, t));
    return ion_forces_part(sys, pos);
}

hipEvent_t pooled_event(me_system* sys) {
    if (!sys->ev_pool.empty()) {
        hipEvent_t e = sys->ev_pool.back();
        sys->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename T>
StencilArgs<T> base_args(me_system* sys, const T* v, int n_orb) {
    const Geometry& g = sys->g;
    StencilArgs<T> a{};
    a.v = v;
    a.stride = g.stride;
    a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
    a.n_orb = n_orb;
    a.zchunk = g.zchunk;
    a.nyt = g.nyt;
    a.tx = g.tx;
    a.nxt = g.nxt;
    a.py = g.py;
    a.nzc = g.nzc;
    a.kin = (T)(-0.5 / (sys->prm.h * sys->prm.h));
    return a;
}

// c_JA of the orbitals u (E_KB h^3 included) into w.cnl, by the precision's
// contraction: plain FP64 / FP32, or split-bf16 MFMA
template <typename T>
me_status gather(me_system* sys, const cx_t<T>* u, int64_t stride, int n_orb, int t, double ekb_h3) {
    if constexpr (sizeof(T) == 4) {
        if (sys->prm.precision == ME_F32_BF16X3) {
            HIPCHK(launch_kb_gather_bf16x3(u, stride, n_orb, sys->g.n_ions, tables(sys, t), ekb_h3,
                                           (float2*)sys->w.cnl, sys->stream));
            return ME_OK;
        }
    }
    HIPCHK(launch_kb_gather<T>(u, stride, n_orb, sys->g.n_ions, tables(sys, t), ekb_h3, (cx_t<T>*)sys->w.cnl,
                               sys->stream));
    return ME_OK;
}

// a stage's fix-up out += alpha E_KB sum_J p_J c_J (c_J = cnl_in) fused with
// the gather of the fixed out into cnl_out, by the precision's contraction
template <typename T>
hipError_t fixup_gather(me_system* sys, cx_t<T>* out, int t, const cx_t<T>* cnl_in, double alpha, double ekb_h3,
                        cx_t<T>* cnl_out) {
    const Geometry& g = sys->g;
    if constexpr (sizeof(T) == 4) {
        if (sys->prm.precision == ME_F32_BF16X3)
            return launch_kb_fixup_gather_bf16x3(out, g.stride, g.n_orb, g.n_ions, tables(sys, t), cnl_in, 0.0, alpha,
                                                 ekb_h3, cnl_out, sys->stream);
    }
    return launch_kb_fixup_gather<T>(out, g.stride, g.n_orb, g.n_ions, tables(sys, t), cnl_in, 0.0, alpha, ekb_h3,
                                     cnl_out, sys->stream);
}

// One Taylor exponential psi <- T_K(tau, H) psi, Horner form:
// u_K = psi, u_{k-1} = psi + (-i tau/k) H u_k, result u_0 written over psi.
template <typename T>
me_status exponential(me_system* sys, const T* veff, int t, bool last) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const double tau = sys->prm.dt / (2.0 * sys->prm.mu);
    const int K = sys->prm.taylor_order;
    C* psi = (C*)sys->w.psi;
    C* bufs[2] = {(C*)sys->w.bufA, (C*)sys->w.bufB};
    const double ekb_h3 = sys->prm.kb_energy * sys->prm.h * sys->prm.h * sys->prm.h;
    const C* u = psi;
    int nb = 0;
    // a stage's fix-up and the next stage's gather share one pass over the
    // projector points; c_JA of the current stage's input alternates between
    // w.cnl and w.cnl2
    const bool fuse = g.n_ions > 0 && env_int("MODEHR_FIXGATHER", 1) != 0;
    C* cnl_buf[2] = {(C*)sys->w.cnl, (C*)sys->w.cnl2};
    int cb = 0;                        // cnl_buf[cb] holds c_JA of the current stage's input
    bool have_c = false;               // ... already, from the previous stage's fused pass
    for (int k = K; k >= 1; --k) {
        // the last stage overwrites psi in place (each point reads its own
        // psi0 only), except for K = 1 where it also reads psi's neighbours
        C* out = (k == 1 && K > 1) ? psi : bufs[nb];
        if (!have_c) {
            CHK(gather<T>(sys, u, g.stride, g.n_orb, t, ekb_h3));
            cb = 0;
        }
        StencilArgs<T> a = base_args<T>(sys, veff, g.n_orb);
        a.u = u;
        a.psi0 = psi;
        a.out = out;
        a.alpha = (T)(-tau / k);
        a.zr = g.finite ? sys->w.zr : nullptr;
        const bool norm = last && k == 1;
        a.partial = norm ? sys->w.norm_part : nullptr;
        if (norm) sys->norm_tiles = g.nxt * g.nyt * g.nzc;
        const int mode = k == K ? MODE_HORNER_FIRST : MODE_HORNER;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (sys->timing) {
            e0 = pooled_event(sys);
            e1 = pooled_event(sys);
            if (e0 && e1) HIPCHK(hipEventRecord(e0, sys->stream));
        }
        HIPCHK(launch_stencil<T>(a, mode, norm, g.ty, g.px, sys->stream));
        if (sys->timing && e0 && e1) {
            HIPCHK(hipEventRecord(e1, sys->stream));
            sys->ev.emplace_back(e0, e1);
            const double streams = mode == MODE_HORNER_FIRST ? 2.0 : 3.0;
            sys->ev_bytes.push_back(streams * g.bc * (double)g.N * g.n_orb + (double)g.br * g.N);
            sys->ev_streams.push_back((int)streams);
        }
        // nonlocal part at the projector points: out += (-i tau/k) E_KB sum_J p_J c_J,
        // with the next stage's gather of out in the same pass where there is one
        have_c = false;
        if (g.n_ions > 0) {
            if (fuse && k > 1) {
                HIPCHK(fixup_gather<T>(sys, out, t, cnl_buf[cb], -tau / k, ekb_h3, cnl_buf[cb ^ 1]));
                cb ^= 1;
                have_c = true;
            } else {
                HIPCHK(launch_kb_fixup<T>(out, g.stride, g.n_orb, tables(sys, t), cnl_buf[cb], 0.0, -tau / k,
                                          norm ? sys->w.fix_part : nullptr, sys->stream));
            }
        }
        u = out;
        nb ^= 1;
    }
    if (K == 1) std::swap(sys->w.psi, sys->w.bufA);
    return ME_OK;
}

// v_eff of the first exponential (v0) and / or the second (v1)
me_status make_veff_parts(me_system* sys, double eps, bool v0, bool v1) {
    const Geometry& g = sys->g;
    const double* hn = sys->w.hist[sys->hist_newest];
    const double* hn1 = sys->w.hist[(sys->hist_newest + 2) % 3];
    const double* hn2 = sys->w.hist[(sys->hist_newest + 1) % 3];
    if (g.f64)
        HIPCHK(launch_veff<double>(sys->w.vloc_cur, sys->w.vloc_next, hn, hn1, hn2, sys->hist_count, g.nx, g.N,
                                   sys->prm.h, Lx(sys), eps, v0 ? (double*)sys->w.veff0 : nullptr,
                                   v1 ? (double*)sys->w.veff1 : nullptr, g.finite ? sys->w.mask : nullptr,
                                   sys->stream));
    else
        HIPCHK(launch_veff<float>(sys->w.vloc_cur, sys->w.vloc_next, hn, hn1, hn2, sys->hist_count, g.nx, g.N,
                                  sys->prm.h, Lx(sys), eps, v0 ? (float*)sys->w.veff0 : nullptr,
                                  v1 ? (float*)sys->w.veff1 : nullptr, g.finite ? sys->w.mask : nullptr,
                                  sys->stream));
    return ME_OK;
}

me_status make_veff(me_system* sys, double eps, bool both) { return make_veff_parts(sys, eps, true, both); }

// fill the report buffer (norm check always; energies when `energy`)
me_status finalize(me_system* sys, bool with_norm, bool energy, const double* fict_part = nullptr,
                   double fict_scale = 0.0, const double* cp_info = nullptr) {
    const Geometry& g = sys->g;
    if (energy) {
        // kinetic expectation per orbital, E_loc = h^3 sum rho V_loc
        if (g.f64) {
            StencilArgs<double> a = base_args<double>(sys, nullptr, g.n_orb);
            a.u = (const double2*)sys->w.psi;
            a.psi0 = a.u;                      // not read in this mode
            a.out = (double2*)sys->w.bufA;     // not written in this mode
            a.partial = sys->w.kin_part;
            HIPCHK(launch_stencil<double>(a, MODE_EXPECT_T, false, g.ty, g.px, sys->stream));
        } else {
            StencilArgs<float> a = base_args<float>(sys, nullptr, g.n_orb);
            a.u = (const float2*)sys->w.psi;
            a.psi0 = a.u;                      // not read in this mode
            a.out = (float2*)sys->w.bufA;      // not written in this mode
            a.partial = sys->w.kin_part;
            HIPCHK(launch_stencil<float>(a, MODE_EXPECT_T, false, g.ty, g.px, sys->stream));
        }
        HIPCHK(launch_dot_partial(sys->w.rho, sys->w.vloc_cur, g.N, sys->w.loc_part, sys->stream));
    }
    FinalizeArgs f{};
    f.rep = sys->w.rep;
    f.norm_part = with_norm ? sys->w.norm_part : nullptr;
    f.fix_part = (with_norm && g.n_ions > 0) ? sys->w.fix_part : nullptr;
    f.fix_tiles = fixup_blocks(g.ucap);
    f.norms = sys->w.norms;
    f.nl_flag = g.n_ions > 0 ? sys->w.tflag[sys->tab_cur] : nullptr;
    f.n_orb = g.n_orb;
    f.norm_tiles = sys->norm_tiles;
    f.norm_tol = g.f64 ? 1e-6 : 1e-5;
    f.dv = sys->prm.h * sys->prm.h * sys->prm.h;
    f.occ = sys->prm.occ;
    f.energy = energy ? 1 : 0;
    f.kin_part = sys->w.kin_part;
    f.kin_n = (int64_t)g.n_orb * g.nxt * g.nyt * g.nzc;
    f.hxc_part = sys->w.hxc_part;
    f.hxc_n = g.nblk256;
    f.loc_part = sys->w.loc_part;
    f.loc_n = g.nblk256;
    f.enl_part = sys->w.enl_part;
    f.eion_part = sys->w.eion_part;
    f.erec_part = sys->w.erec_part;
    f.erec_n = (g.n_ions > 0 && sys->ewp.ng > 0 && !g.finite) ? ewald_sg_blocks(sys->ewp.ng) : 0;   // unwritten without ions
    f.ewald_rec_scale = 2.0 * M_PI / (sys->ew.L * sys->ew.L * sys->ew.L);
    f.ewald_const = g.finite ? 0.0 : sys->ew.e_const;
    f.vel = sys->w.vel;
    f.frc = sys->w.frc;
    f.mass = sys->w.mass;
    f.n_ions = g.n_ions;
    f.fict_part = fict_part;
    f.fict_n = fict_part ? g.nblk256 : 0;
    f.fict_scale = fict_scale;
    f.cp_info = cp_info;
    HIPCHK(launch_report(f, sys->stream));
    return ME_OK;
}

me_status read_report(me_system* sys, me_step_report* rep) {
    HIPCHK(hipMemcpyAsync(sys->rep_host, sys->w.rep, sizeof(sys->rep_host), hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    const double* r = sys->rep_host;
    if (rep) {
        rep->e_kinetic = r[SLOT_EKIN];
        rep->e_local = r[SLOT_ELOC];
        rep->e_hartree = r[SLOT_EH];
        rep->e_xc = r[SLOT_EX];
        rep->e_nonlocal = r[SLOT_ENL];
        rep->e_ion = r[SLOT_EION];
        rep->e_ks = r[SLOT_EKS];
        rep->e_ion_kinetic = r[SLOT_EIONKIN];
        rep->e_total = r[SLOT_ETOT];
        rep->max_norm_dev = r[SLOT_NORM_DEV];
        rep->max_force = r[SLOT_FMAX];
        rep->charge = r[SLOT_CHARGE];
        rep->step = sys->step;
        rep->e_fictitious = r[SLOT_EFICT];
        rep->cp_constraint_residual = r[SLOT_CP_RES];
    }
    if (r[SLOT_UNSTABLE] == 2.0) {
        sys->err = "a grid point lies inside more than 8 projector spheres";
        return ME_EUNSUPPORTED;
    }
    if (r[SLOT_UNSTABLE] != 0.0) {
        sys->err = "orbital norm grew beyond tolerance or became non-finite";
        return ME_EUNSTABLE;
    }
    return ME_OK;
}

// Forward exponential keeping every Horner stage: inter[j-1] = u_j for
// j = 1..K-1 (u_K = psi_in), result u_0 in out (psi_in untouched).
template <typename T>
me_status exponential_store(me_system* sys, const T* veff, int t, const cx_t<T>* psi_in, void* const* inter,
                            cx_t<T>* out) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const double tau = sys->prm.dt / (2.0 * sys->prm.mu);
    const int K = sys->prm.taylor_order;
    const double ekb_h3 = sys->prm.kb_energy * sys->prm.h * sys->prm.h * sys->prm.h;
    const C* u = psi_in;
    for (int k = K; k >= 1; --k) {
        C* o = k == 1 ? out : (C*)inter[k - 2];
        CHK(gather<T>(sys, u, g.stride, g.n_orb, t, ekb_h3));
        StencilArgs<T> a = base_args<T>(sys, veff, g.n_orb);
        a.u = u;
        a.psi0 = psi_in;
        a.out = o;
        a.alpha = (T)(-tau / k);
        HIPCHK(launch_stencil<T>(a, k == K ? MODE_HORNER_FIRST : MODE_HORNER, false, g.ty, g.px, sys->stream));
        if (g.n_ions > 0)
            HIPCHK(launch_kb_fixup<T>(o, g.stride, g.n_orb, tables(sys, t), (const C*)sys->w.cnl, 0.0, -tau / k,
                                      nullptr, sys->stream));
        u = o;
    }
    return ME_OK;
}

// Reverse of one exponential: lam_out = psi_in-bar given lam_in = output-bar,
// wbar += dJ/dv_eff of this exponential.
template <typename T>
me_status reverse_exponential(me_system* sys, const T* veff, int t, const cx_t<T>* psi_in, void* const* inter,
                              const cx_t<T>* lam_in, cx_t<T>* lam_out, double* wbar) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const double tau = sys->prm.dt / (2.0 * sys->prm.mu);
    const int K = sys->prm.taylor_order;
    const double ekb_h3 = sys->prm.kb_energy * sys->prm.h * sys->prm.h * sys->prm.h;
    C* ubs[2] = {(C*)sys->w.ubA, (C*)sys->w.ubB};
    const C* ub = lam_in;
    for (int k = 1; k <= K; ++k) {
        const C* uk = k == K ? psi_in : (const C*)inter[k - 1];
        HIPCHK(launch_cross_accum<T>(ub, uk, lam_out, g.stride, g.n_orb, g.N, -tau / k, k == 1, wbar, sys->stream));
        // ubar_k = conj(c_k) H ubar_{k-1} = (i tau/k) H ubar_{k-1}
        C* nb = ubs[k & 1];
        CHK(gather<T>(sys, ub, g.stride, g.n_orb, t, ekb_h3));
        StencilArgs<T> a = base_args<T>(sys, veff, g.n_orb);
        a.u = ub;
        a.psi0 = ub;
        a.out = nb;
        a.alpha = (T)(tau / k);
        HIPCHK(launch_stencil<T>(a, MODE_SCALED, false, g.ty, g.px, sys->stream));
        if (g.n_ions > 0)
            HIPCHK(launch_kb_fixup<T>(nb, g.stride, g.n_orb, tables(sys, t), (const C*)sys->w.cnl, 0.0, tau / k,
                                      nullptr, sys->stream));
        ub = nb;
    }
    HIPCHK(launch_accum<T>(ub, lam_out, g.stride, g.n_orb, g.N, sys->stream));
    return ME_OK;
}

// rhobar = Hartree(vbar) + f_x(rho) vbar (+ extra): the adjoint of v_Hxc[rho]
me_status vhxc_adjoint(me_system* sys, const double* vbar, const double* rho, const double* extra) {
    const Geometry& g = sys->g;
    const double L[3] = {g.nx * sys->prm.h, g.ny * sys->prm.h, g.nz * sys->prm.h};
    HIPCHK(hipMemcpyAsync(sys->w.hv, vbar, g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    CHK(fft_r2c(sys, sys->w.hv, sys->w.rhok));
    HIPCHK(launch_hartree_spectrum(sys->w.rhok, g.nx, g.ny, g.nz, L, sys->w.spec, sys->stream));
    CHK(fft_c2r(sys, sys->w.spec, sys->w.hv));
    HIPCHK(launch_vhxc_adjoint(sys->w.hv, vbar, rho, extra, g.N, sys->w.rhobar, sys->stream));
    return ME_OK;
}

// Reverse of one frozen-ion step n (state at the start of the step loaded).
template <typename T>
me_status adjoint_step_impl(me_system* sys, double eps, double* g_eps) {
    sys->cp_ready = false;
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const int64_t n = sys->step;
    const int t = sys->tab_cur;
    // effective potentials of both exponentials (frozen ions: V_loc is the same)
    HIPCHK(hipMemcpyAsync(sys->w.vloc_next, sys->w.vloc_cur, g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    CHK(make_veff(sys, eps, true));
    const T* w1 = (const T*)sys->w.veff0;
    const T* w2 = (const T*)sys->w.veff1;
    // forward recompute with every stage kept
    CHK(exponential_store<T>(sys, w1, t, (const C*)sys->w.psi, sys->w.inter[0], (C*)sys->w.psi_half));
    CHK(exponential_store<T>(sys, w2, t, (const C*)sys->w.psi_half, sys->w.inter[1], (C*)sys->w.psi_next));
    HIPCHK(launch_density<T>((const C*)sys->w.psi_next, g.stride, g.n_orb, g.N, sys->prm.occ, sys->w.rho,
                             sys->stream));
    // rho(n+1)-bar from v_Hxc(n+1)-bar (and the objective at the final time)
    double* vb_next = sys->w.vbar[(n + 1) & 3];
    CHK(vhxc_adjoint(sys, vb_next, sys->w.rho, sys->adj_pending_final ? sys->w.rhobar_T : nullptr));
    sys->adj_pending_final = false;
    HIPCHK(launch_lambda_update<T>((C*)sys->w.lamA, (const C*)sys->w.psi_next, sys->w.rhobar, g.stride, g.n_orb,
                                   g.N, sys->prm.occ, sys->stream));
    HIPCHK(launch_zero(vb_next, g.N, sys->stream));
    // reverse the second then the first exponential
    HIPCHK(launch_zero(sys->w.wbar1, g.N, sys->stream));
    HIPCHK(launch_zero(sys->w.wbar2, g.N, sys->stream));
    CHK(reverse_exponential<T>(sys, w2, t, (const C*)sys->w.psi_half, sys->w.inter[1], (const C*)sys->w.lamA,
                               (C*)sys->w.lamB, sys->w.wbar2));
    CHK(reverse_exponential<T>(sys, w1, t, (const C*)sys->w.psi, sys->w.inter[0], (const C*)sys->w.lamB,
                               (C*)sys->w.lamA, sys->w.wbar1));
    // the first exponential used v_n, the second the extrapolation of v_n, v_{n-1}, v_{n-2}
    HIPCHK(launch_axpy(sys->w.vbar[n & 3], sys->w.wbar1, 1.0, g.N, sys->stream));
    const int lv = sys->hist_count;
    const double a3[3] = {3.0, -3.0, 1.0}, a2[2] = {2.0, -1.0}, a1[1] = {1.0};
    const double* ac = lv >= 3 ? a3 : (lv == 2 ? a2 : a1);
    for (int j = 0; j < std::min(lv, 3); ++j)
        HIPCHK(launch_axpy(sys->w.vbar[(n - j + 4) & 3], sys->w.wbar2, ac[j], g.N, sys->stream));
    // both exponentials see eps (x - L/2) and the static potential
    HIPCHK(launch_axpy(sys->w.wbar2, sys->w.wbar1, 1.0, g.N, sys->stream));
    HIPCHK(launch_axpy(sys->w.gfine, sys->w.wbar2, 1.0, g.N, sys->stream));
    HIPCHK(launch_field_dot(sys->w.wbar2, g.nx, g.N, sys->prm.h, Lx(sys), sys->w.dpart, sys->w.scal, 1.0,
                            sys->stream));
    HIPCHK(hipMemcpyAsync(g_eps, sys->w.scal, 8, hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    return ME_OK;
}

struct CkptHeader {
    int64_t step;
    int32_t hist_count, hist_newest, n_orb, n_ions;
    int64_t N;
    int64_t magic;
};

size_t ckpt_bytes(const Geometry& g) {
    return 256 + align_up((size_t)g.n_orb * g.stride * g.bc) + align_up(3 * (size_t)g.N * 8) +
           align_up(9 * (size_t)std::max(1, g.n_ions) * 8);
}

me_status initial_fields(me_system* sys) {
    // V_loc, tables and forces at the current positions; density and v_Hxc
    sys->hist_count = 0;
    sys->hist_newest = 0;
    sys->tab_cur = 0;
    CHK(build_tables(sys, sys->w.pos, sys->tab_cur));
    CHK(density_vhxc(sys, true));
    CHK(ion_fields(sys, sys->w.pos, sys->w.vloc_cur));
    CHK(forces_parts(sys, sys->w.pos, sys->tab_cur));
    HIPCHK(hipMemcpyAsync(sys->w.pos_next, sys->w.pos, 3 * 8 * std::max(1, sys->g.n_ions),
                          hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(launch_ions_finish(sys->w.pos, sys->w.vel, sys->w.frc, sys->w.pos_next, sys->w.floc, sys->w.fnl, sys->w.fion, sys->w.mass, sys->g.n_ions,
                              sys->prm.dt, 1, sys->stream));
    HIPCHK(hipMemsetAsync(sys->w.rep, 0, SLOT_COUNT * 8, sys->stream));
    return ME_OK;
}

// steps 1-2 of a step: ions moved, H(t+dt) prepared.  With the overlap the
// launches go to the side stream, v_eff of the first exponential excepted
// (make_veff_parts on the main stream), and the Ewald sum at R(t+dt) is
// taken here too.
me_status step_pre_ions(me_system* sys, double eps, bool overlap) {
    const Geometry& g = sys->g;
    const int next = sys->tab_cur ^ 1;
    // 1. ions: R(t+dt) by velocity Verlet
    HIPCHK(launch_ions_predict(sys->w.pos, sys->w.vel, sys->w.frc, sys->w.mass, g.n_ions, sys->prm.dt,
                               sys->prm.freeze_ions, sys->w.pos_next, sys->stream));
    // 2. ionic part of H(t+dt): V_loc and projector tables at R(t+dt)
    CHK(ion_fields(sys, sys->w.pos_next, sys->w.vloc_next));
    CHK(build_tables(sys, sys->w.pos_next, next));
    CHK(make_veff_parts(sys, eps, !overlap, true));
    if (overlap) CHK(ion_forces_part(sys, sys->w.pos_next));
    return ME_OK;
}

me_status step_pre(me_system* sys, double eps) {
    sys->cp_ready = false;          // bufA / bufB become Taylor-stage scratch
    return step_pre_ions(sys, eps, false);
}

// step 5: density, fields and forces of the propagated orbitals, ions finished
// (overlap: the Ewald part was taken by step_pre_ions, the nonlocal forces
// run on the side stream beside the density and Hartree chain)
me_status step_post(me_system* sys, bool energy, bool overlap = false) {
    const Geometry& g = sys->g;
    const int next = sys->tab_cur ^ 1;
    if (overlap) {
        HIPCHK(hipEventRecord(sys->ev_fork[1], sys->stream));
        HIPCHK(hipStreamWaitEvent(sys->side, sys->ev_fork[1], 0));
        {
            OnSide on(sys);
            CHK(nl_forces_part(sys, sys->w.pos_next, next));
        }
        HIPCHK(hipEventRecord(sys->ev_join[1], sys->side));
        CHK(density_vhxc(sys, energy));
        CHK(local_forces_part(sys, sys->w.pos_next));
        HIPCHK(hipStreamWaitEvent(sys->stream, sys->ev_join[1], 0));
    } else {
        CHK(density_vhxc(sys, energy));
        CHK(forces_parts(sys, sys->w.pos_next, next));
    }
    HIPCHK(launch_ions_finish(sys->w.pos, sys->w.vel, sys->w.frc, sys->w.pos_next, sys->w.floc, sys->w.fnl, sys->w.fion, sys->w.mass, g.n_ions, sys->prm.dt,
                              sys->prm.freeze_ions, sys->stream));
    std::swap(sys->w.vloc_cur, sys->w.vloc_next);
    sys->tab_cur = next;
    sys->step += 1;
    return finalize(sys, true, energy);
}

template <typename T>
me_status step_impl(me_system* sys, double eps, bool energy) {
    const bool overlap = sys->side != nullptr;
    const int next = sys->tab_cur ^ 1;
    sys->cp_ready = false;          // bufA / bufB become Taylor-stage scratch
    if (overlap) {
        HIPCHK(hipEventRecord(sys->ev_fork[0], sys->stream));
        HIPCHK(hipStreamWaitEvent(sys->side, sys->ev_fork[0], 0));
        {
            OnSide on(sys);
            CHK(step_pre_ions(sys, eps, true));
        }
        HIPCHK(hipEventRecord(sys->ev_join[0], sys->side));
        CHK(make_veff_parts(sys, eps, true, false));
    } else {
        CHK(step_pre_ions(sys, eps, false));
    }
    // 3-4. AETRS: exp(-i tau H(t+dt)) exp(-i tau H(t)); the second waits for H(t+dt)
    CHK(exponential<T>(sys, (const T*)sys->w.veff0, sys->tab_cur, false));
    if (overlap) HIPCHK(hipStreamWaitEvent(sys->stream, sys->ev_join[0], 0));
    if (sys->g.etrs == 0) {
        CHK(exponential<T>(sys, (const T*)sys->w.veff1, next, true));
        return step_post(sys, energy, overlap);
    }
    // ETRS: the AETRS result predicts psi(t+dt); each correction rebuilds
    // v_eff of the second exponential from its density and redoes that
    // exponential from the half-step orbitals
    const Geometry& g = sys->g;
    const size_t orb = (size_t)g.n_orb * g.stride * g.bc;
    HIPCHK(hipMemcpyAsync(sys->w.etrs_half, sys->w.psi, orb, hipMemcpyDeviceToDevice, sys->stream));
    CHK(exponential<T>(sys, (const T*)sys->w.veff1, next, true));
    for (int k = 0; k < g.etrs; ++k) {
        CHK(density_vhxc(sys, false, false));          // v_Hxc of the prediction into w.vh
        HIPCHK(launch_veff<T>(sys->w.vloc_cur, sys->w.vloc_next, sys->w.vh, sys->w.vh, sys->w.vh, 1, g.nx, g.N,
                              sys->prm.h, Lx(sys), eps, nullptr, (T*)sys->w.veff1,
                              g.finite ? sys->w.mask : nullptr, sys->stream));
        HIPCHK(hipMemcpyAsync(sys->w.psi, sys->w.etrs_half, orb, hipMemcpyDeviceToDevice, sys->stream));
        CHK(exponential<T>(sys, (const T*)sys->w.veff1, next, true));
    }
    return step_post(sys, energy, overlap);
}

}  // namespace

// ================================================================== batches
// Many independent systems advanced together: per-system work (ions, fields,
// tables, gathers, fix-ups, forces) is enqueued system by system, and every
// Horner stage of all systems is one persistent stencil launch.  A run of
// BATCH_GRAPH_STEPS steps can be captured once as a hipGraph and replayed.

// The host-side state of a system changes with period 2 (projector tables,
// V_loc buffers, the K = 1 orbital swap) and 3 (v_Hxc history ring), so six
// steps bring every pointer a step uses back to where it was.
constexpr int BATCH_GRAPH_STEPS = 6;
constexpr int BATCH_WORKERS = 4;

struct BatchTile {
    int ty, nyt, zchunk, nzc, items;
    int tx, nxt;        // tile width (nx: whole rows) and x-tiles
};

struct PhaseKey {
    int tab_cur, hist_newest, hist_count;
    bool static_set;
    const void *psi, *bufA;
    const double* vloc_cur;
    bool operator==(const PhaseKey& o) const {
        return tab_cur == o.tab_cur && hist_newest == o.hist_newest && hist_count == o.hist_count &&
               static_set == o.static_set && psi == o.psi && bufA == o.bufA && vloc_cur == o.vloc_cur;
    }
};

struct me_batch {
    std::vector<me_system*> sys;   // caller order
    std::vector<int> order;        // launch order: largest work items first
    hipStream_t stream = nullptr;
    bool f64 = false;
    int K = 4;
    int* counters = nullptr;       // device: [2 K + 1][QUEUE_SLOTS]
    int n_cu = 256;
    me_batch_tuning tune{};
    bool tuned = false;            // tuning set explicitly or by the autotuner
    std::vector<BatchTile> tile;   // caller order
    size_t lds = 0;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<PhaseKey> phase;   // host state the graph was captured at
    bool capturing = false;
    // Per-system work of a step runs on BATCH_WORKERS streams (system i on
    // worker i mod BATCH_WORKERS, default priority), forked from and joined
    // back to `stream` around every persistent stencil launch, so the small
    // kernels of different systems overlap (also inside a captured graph).
    std::vector<hipStream_t> workers;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> ev_bytes;
    std::vector<int> ev_streams;    // complex streams of each timed launch (2: first stage, 3: others)
    std::vector<hipEvent_t> ev_pool;
    std::string err;
};

namespace {

constexpr int QUEUE_SLOTS = 8;     // counters per persistent launch (one per XCD queue)

#define BHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            b->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            return ME_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

// a per-system call inside a batch operation: its error text moves to the batch
#define BSYS(expr, s)                                                                  \
    do {                                                                               \
        me_status s_ = (expr);                                                         \
        if (s_ != ME_OK) {                                                             \
            b->err = (s)->err;                                                         \
            return s_;                                                                 \
        }                                                                              \
    } while (0)

// halo jobs per thread of the whole-row systems (x-tiled ones take 2)
int batch_hj(const me_batch* b, int block, const std::vector<BatchTile>& tiles) {
    int hj = 1;
    for (size_t i = 0; i < b->sys.size(); ++i)
        if (tiles[i].nxt == 1 && 8 * b->sys[i]->g.nx > block) hj = 2;
    return hj;
}

// Tiles of every system for a tuning; false if the tuning cannot run them.
// A system whose whole rows do not fit the block (or that the halo jobs of
// whole rows would overload) runs in x-tiles of 64 points and block/64 rows;
// MODEHR_BATCH_TX forces x-tiles of that width on every wider row (tests).
bool batch_tiles(const me_batch* b, const me_batch_tuning& t, std::vector<BatchTile>& out, size_t& lds) {
    if (t.block < 64 || t.block > 1024 || t.block % 64) return false;
    if (t.zdiv != 1 && t.zdiv != 2 && t.zdiv != 4) return false;
    const int ftx = env_int("MODEHR_BATCH_TX", 0);
    out.clear();
    lds = 0;
    for (const me_system* s : b->sys) {
        const Geometry& g = s->g;
        BatchTile bt{};
        const bool xt = (ftx > 0 && g.nx > ftx) || g.nx > t.block || 8 * g.nx > 2 * t.block;
        if (xt) {
            const int tx = std::min(g.nx, ftx > 0 ? ftx : 64);
            const int ty = std::min(g.ny, t.block / tx);
            if (ty < 1 || 8 * (tx + ty) > 2 * t.block) return false;
            const size_t l = stencil_xt_lds_bytes(tx, ty, g.bc);
            if (l > STENCIL_LDS_MAX) return false;
            bt.tx = tx;
            bt.nxt = (g.nx + tx - 1) / tx;
            bt.ty = ty;
            lds = std::max(lds, l);
        } else {
            int ty = std::min(g.ny, t.block / g.nx);
            while (ty > 1 && stencil_lds_bytes(ty, g.nx, g.bc) > STENCIL_LDS_MAX) --ty;
            if (ty < 1 || stencil_lds_bytes(ty, g.nx, g.bc) > STENCIL_LDS_MAX) return false;
            bt.tx = g.nx;
            bt.nxt = 1;
            bt.ty = ty;
            lds = std::max(lds, stencil_lds_bytes(ty, g.nx, g.bc));
        }
        bt.nyt = (g.ny + bt.ty - 1) / bt.ty;
        bt.zchunk = (g.nz + t.zdiv - 1) / t.zdiv;
        bt.nzc = (g.nz + bt.zchunk - 1) / bt.zchunk;
        if ((int64_t)bt.nxt * bt.nyt * bt.nzc > g.norm_cap) return false;
        const int64_t items = (int64_t)g.n_orb * bt.nxt * bt.nyt * bt.nzc;
        if (items > (1 << 26)) return false;
        bt.items = (int)items;
        out.push_back(bt);
    }
    return true;
}

bool batch_has_xt(const std::vector<BatchTile>& tiles) {
    for (const BatchTile& bt : tiles)
        if (bt.nxt > 1) return true;
    return false;
}

template <typename T>
int batch_max_wpc(const me_batch* b, int block, size_t lds, const std::vector<BatchTile>& tiles) {
    int w = 0;
    if (batch_stencil_occupancy<T>(block, lds, batch_hj(b, block, tiles), batch_has_xt(tiles), &w) != hipSuccess)
        return 0;
    return w;
}

me_status batch_apply_tuning(me_batch* b, const me_batch_tuning& t) {
    std::vector<BatchTile> tiles;
    size_t lds = 0;
    if (!batch_tiles(b, t, tiles, lds)) {
        b->err = "tuning does not fit this batch (block, zdiv or LDS)";
        return ME_EINVAL;
    }
    const int wmax = b->f64 ? batch_max_wpc<double>(b, t.block, lds, tiles)
                            : batch_max_wpc<float>(b, t.block, lds, tiles);
    if (wmax < 1 || t.wg_per_cu < 0 || t.wg_per_cu > wmax) {
        b->err = "wg_per_cu must be in [0, " + std::to_string(wmax) + "] for this block size";
        return ME_EINVAL;
    }
    b->tune = t;
    b->tile = tiles;
    b->lds = lds;
    b->grid = t.wg_per_cu * b->n_cu;     // 0: one item per workgroup, grid set per launch
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
    return ME_OK;
}

// the untuned choice: 768 threads (1024 where a row needs it), one work item
// per workgroup, whole z columns
me_status batch_default_tuning(me_batch* b) {
    me_batch_tuning t{};
    t.zdiv = 1;
    for (int block : {768, 1024, 512}) {
        t.block = block;
        std::vector<BatchTile> tiles;
        size_t lds = 0;
        if (!batch_tiles(b, t, tiles, lds)) continue;
        const int wmax = b->f64 ? batch_max_wpc<double>(b, block, lds, tiles)
                                : batch_max_wpc<float>(b, block, lds, tiles);
        if (wmax < 1) continue;
        t.wg_per_cu = 0;
        return batch_apply_tuning(b, t);
    }
    b->err = "no workgroup shape fits this batch";
    return ME_EUNSUPPORTED;
}

hipEvent_t batch_event(me_batch* b) {
    if (!b->ev_pool.empty()) {
        hipEvent_t e = b->ev_pool.back();
        b->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Move every system's work onto its worker stream, after all work queued so
// far on the batch stream.
me_status batch_fork(me_batch* b) {
    BHIP(hipEventRecord(b->ev_fork, b->stream));
    for (hipStream_t w : b->workers) BHIP(hipStreamWaitEvent(w, b->ev_fork, 0));
    for (size_t i = 0; i < b->sys.size(); ++i) {
        me_system* s = b->sys[i];
        s->stream = b->workers[i % b->workers.size()];
        if (rocfft_execution_info_set_stream(s->info, s->stream) != rocfft_status_success) {
            b->err = "rocfft_execution_info_set_stream failed";
            return ME_EDEVICE;
        }
    }
    return ME_OK;
}

// The batch stream waits for everything queued on the workers; the systems
// return to the batch stream.
me_status batch_join(me_batch* b) {
    for (size_t w = 0; w < b->workers.size(); ++w) {
        BHIP(hipEventRecord(b->ev_join[w], b->workers[w]));
        BHIP(hipStreamWaitEvent(b->stream, b->ev_join[w], 0));
    }
    for (me_system* s : b->sys) {
        s->stream = b->stream;
        if (rocfft_execution_info_set_stream(s->info, s->stream) != rocfft_status_success) {
            b->err = "rocfft_execution_info_set_stream failed";
            return ME_EDEVICE;
        }
    }
    return ME_OK;
}

// One persistent launch: stage k of exponential e over all systems.
// u[i] / out[i] / psi0 = psi of system i (caller order); counter slot `slot`.
template <typename T>
me_status batch_stage(me_batch* b, const std::vector<const cx_t<T>*>& u, const std::vector<cx_t<T>*>& out,
                      int e, int k, bool norm, int slot, int mode) {
    using C = cx_t<T>;
    BatchStencilArgs<T> a{};
    a.n_sys = (int)b->sys.size();
    a.counter = b->counters + slot * QUEUE_SLOTS;
    int item = 0;
    double bytes = 0.0;
    for (int j = 0; j < a.n_sys; ++j) {
        const int i = b->order[j];
        me_system* s = b->sys[i];
        const Geometry& g = s->g;
        const BatchTile& bt = b->tile[i];
        BatchSys<T>& d = a.sys[j];
        d.u = u[i];
        d.psi0 = (const C*)s->w.psi;
        d.out = out[i];
        d.v = (const T*)(e == 0 ? s->w.veff0 : s->w.veff1);
        d.partial = norm ? s->w.norm_part : nullptr;
        d.stride = g.stride;
        d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
        d.ty = bt.ty; d.nyt = bt.nyt;
        d.tx = bt.tx; d.nxt = bt.nxt;
        d.zchunk = bt.zchunk; d.nzc = bt.nzc;
        d.item0 = item;
        d.items = bt.items;
        item += bt.items;
        d.kin = (T)(-0.5 / (s->prm.h * s->prm.h));
        d.alpha = (T)(-(s->prm.dt / (2.0 * s->prm.mu)) / k);
        if (norm) s->norm_tiles = bt.nxt * bt.nyt * bt.nzc;
        const double streams = mode == MODE_HORNER_FIRST ? 2.0 : 3.0;
        bytes += streams * g.bc * (double)g.N * g.n_orb + (double)g.br * g.N;
    }
    a.total = item;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = b->timing && !b->capturing;
    if (timed) {
        e0 = batch_event(b);
        e1 = batch_event(b);
        if (e0 && e1) BHIP(hipEventRecord(e0, b->stream));
    }
    int grid = b->grid;
    if (b->tune.wg_per_cu == 0) {
        // one item per workgroup: 8 x the largest per-XCD share of the items
        int share = 0;
        for (int q = 0; q < QUEUE_SLOTS; ++q) {
            int n = 0;
            for (int j = 0; j < a.n_sys; ++j) {
                const int cnt = a.sys[j].items;
                n += (int)((int64_t)cnt * (q + 1) / QUEUE_SLOTS - (int64_t)cnt * q / QUEUE_SLOTS);
            }
            share = std::max(share, n);
        }
        a.counter = nullptr;
        grid = QUEUE_SLOTS * share;
    }
    BHIP(launch_batch_stencil<T>(a, mode, norm, b->tune.block, grid, b->lds, b->stream));
    if (timed && e0 && e1) {
        BHIP(hipEventRecord(e1, b->stream));
        b->ev.emplace_back(e0, e1);
        b->ev_bytes.push_back(bytes);
        b->ev_streams.push_back(mode == MODE_HORNER_FIRST ? 2 : 3);
    }
    return ME_OK;
}

// One Taylor exponential of every system (e = 0: H(t), e = 1: H(t+dt)),
// stage by stage as in exponential(): per-system gathers, one persistent
// stencil launch, per-system fix-ups.
template <typename T>
me_status batch_exponential(me_batch* b, int e, bool last) {
    using C = cx_t<T>;
    const int K = b->K;
    const int n = (int)b->sys.size();
    std::vector<const C*> u(n);
    std::vector<C*> out(n);
    for (int i = 0; i < n; ++i) u[i] = (const C*)b->sys[i]->w.psi;
    // as in exponential(): a stage's fix-up shares a pass with the next
    // stage's gather; cb[i] says which of w.cnl / w.cnl2 holds system i's
    // c_JA of the current stage's input
    const bool fuse = env_int("MODEHR_FIXGATHER", 1) != 0;
    std::vector<int> cb(n, 0);
    bool have_c = false;
    int nb = 0;
    for (int k = K; k >= 1; --k) {
        const bool norm = last && k == 1;
        for (int i = 0; i < n; ++i) {
            me_system* s = b->sys[i];
            const int t = e == 0 ? s->tab_cur : s->tab_cur ^ 1;
            C* bufs[2] = {(C*)s->w.bufA, (C*)s->w.bufB};
            out[i] = (k == 1 && K > 1) ? (C*)s->w.psi : bufs[nb];
            const double ekb_h3 = s->prm.kb_energy * s->prm.h * s->prm.h * s->prm.h;
            if (!have_c || s->g.n_ions == 0) {
                BSYS(gather<T>(s, u[i], s->g.stride, s->g.n_orb, t, ekb_h3), s);
                cb[i] = 0;
            }
        }
        CHK(batch_join(b));
        CHK(batch_stage<T>(b, u, out, e, k, norm, e * K + (K - k), k == K ? MODE_HORNER_FIRST : MODE_HORNER));
        have_c = fuse && k > 1;
        // the fused passes of the plain contraction: one launch over the
        // systems (KB_BATCH at a time) on the batch stream
        const bool one_launch = have_c && !(sizeof(T) == 4 && b->sys[0]->prm.precision == ME_F32_BF16X3);
        if (one_launch) {
            BatchKbArgs<T> ka{};
            for (int i = 0; i < n; ++i) {
                me_system* s = b->sys[i];
                if (s->g.n_ions == 0) continue;
                const int t = e == 0 ? s->tab_cur : s->tab_cur ^ 1;
                C* cnl_buf[2] = {(C*)s->w.cnl, (C*)s->w.cnl2};
                BatchKbSys<T>& d = ka.sys[ka.n_sys++];
                d.out = out[i];
                d.cnl_in = cnl_buf[cb[i]];
                d.cnl_out = cnl_buf[cb[i] ^ 1];
                d.t = tables(s, t);
                d.stride = s->g.stride;
                d.n_orb = s->g.n_orb;
                d.n_ions = s->g.n_ions;
                d.gi = (T)(-(s->prm.dt / (2.0 * s->prm.mu)) / k);
                d.scale = (T)(s->prm.kb_energy * s->prm.h * s->prm.h * s->prm.h);
                cb[i] ^= 1;
                if (ka.n_sys == KB_BATCH) {
                    BHIP(launch_batch_kb_fixup_gather<T>(ka, b->stream));
                    ka.n_sys = 0;
                }
            }
            if (ka.n_sys > 0) BHIP(launch_batch_kb_fixup_gather<T>(ka, b->stream));
        }
        CHK(batch_fork(b));
        for (int i = 0; i < n; ++i) {
            me_system* s = b->sys[i];
            const Geometry& g = s->g;
            const int t = e == 0 ? s->tab_cur : s->tab_cur ^ 1;
            const double tau = s->prm.dt / (2.0 * s->prm.mu);
            C* cnl_buf[2] = {(C*)s->w.cnl, (C*)s->w.cnl2};
            if (g.n_ions > 0 && !one_launch) {
                if (have_c) {
                    const double ekb_h3 = s->prm.kb_energy * s->prm.h * s->prm.h * s->prm.h;
                    BHIP(fixup_gather<T>(s, out[i], t, cnl_buf[cb[i]], -tau / k, ekb_h3, cnl_buf[cb[i] ^ 1]));
                    cb[i] ^= 1;
                } else {
                    BHIP(launch_kb_fixup<T>(out[i], g.stride, g.n_orb, tables(s, t), cnl_buf[cb[i]], 0.0,
                                            -tau / k, norm ? s->w.fix_part : nullptr, s->stream));
                }
            }
            u[i] = out[i];
        }
        nb ^= 1;
    }
    if (K == 1)
        for (me_system* s : b->sys) std::swap(s->w.psi, s->w.bufA);
    return ME_OK;
}

template <typename T>
me_status batch_step(me_batch* b) {
    BHIP(launch_zero_i32(b->counters, 2 * b->K * QUEUE_SLOTS, b->stream));
    CHK(batch_fork(b));
    me_status st = ME_OK;
    for (me_system* s : b->sys) {
        if (st != ME_OK) break;
        st = step_pre(s, 0.0);
        if (st != ME_OK) b->err = s->err;
    }
    if (st == ME_OK) st = batch_exponential<T>(b, 0, false);
    if (st == ME_OK) st = batch_exponential<T>(b, 1, true);
    for (me_system* s : b->sys) {
        if (st != ME_OK) break;
        st = step_post(s, false);
        if (st != ME_OK) b->err = s->err;
    }
    const me_status sj = batch_join(b);
    return st != ME_OK ? st : sj;
}

me_status batch_step_any(me_batch* b) {
    return b->f64 ? batch_step<double>(b) : batch_step<float>(b);
}

std::vector<PhaseKey> batch_phase(const me_batch* b) {
    std::vector<PhaseKey> p;
    for (const me_system* s : b->sys)
        p.push_back(PhaseKey{s->tab_cur, s->hist_newest, s->hist_count, s->static_set, s->w.psi, s->w.bufA,
                             s->w.vloc_cur});
    return p;
}

void batch_drop_graph(me_batch* b) {
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->phase.clear();
}

// everything the batch owns (after its streams are idle)
void batch_release(me_batch* b) {
    batch_drop_graph(b);
    for (auto& e : b->ev) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
    for (auto& e : b->ev_pool) hipEventDestroy(e);
    for (hipEvent_t e : b->ev_join) hipEventDestroy(e);
    if (b->ev_fork) hipEventDestroy(b->ev_fork);
    for (hipStream_t w : b->workers) hipStreamDestroy(w);
    for (me_system* s : b->sys) me_destroy(s);
    delete b;
}

// Capture BATCH_GRAPH_STEPS steps as one graph at the current host state.
// Capturing runs the host side of those steps (no device work), which
// returns every per-system pointer and ring index to where it started.
me_status batch_capture(me_batch* b) {
    batch_drop_graph(b);
    const std::vector<PhaseKey> start = batch_phase(b);
    std::vector<int64_t> steps;
    for (me_system* s : b->sys) steps.push_back(s->step);
    BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    b->capturing = true;
    me_status st = ME_OK;
    for (int i = 0; i < BATCH_GRAPH_STEPS && st == ME_OK; ++i) st = batch_step_any(b);
    b->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &graph);
    for (size_t i = 0; i < b->sys.size(); ++i) b->sys[i]->step = steps[i];
    if (st != ME_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess) {
        b->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
        return ME_EDEVICE;
    }
    if (!(batch_phase(b) == start)) {
        hipGraphDestroy(graph);
        b->err = "internal error: host state did not return after a graph period";
        return ME_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        hipGraphDestroy(graph);
        b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
        return ME_EDEVICE;
    }
    b->graph = graph;
    b->exec = exec;
    b->phase = start;
    return ME_OK;
}

// ---------------------------------------------------------------- autotuner
// Candidates are timed on one Horner stage over the whole batch (u = psi0 =
// psi, out = bufA, which the next step overwrites anyway).  Results are kept
// in a small JSON file keyed by precision, Taylor order and the shapes.

std::string batch_key(const me_batch* b) {
    std::string k = b->sys[0]->prm.precision == ME_F64 ? "f64" : "f32";
    k += "/K" + std::to_string(b->K);
    for (int i : b->order) {
        const me_system* s = b->sys[i];
        k += "/" + std::to_string(s->g.nx) + "x" + std::to_string(s->g.ny) + "x" + std::to_string(s->g.nz) +
             ":" + std::to_string(s->g.n_orb);
    }
    return k;
}

bool json_field(const std::string& line, const char* name, double* v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    char* end = nullptr;
    *v = std::strtod(line.c_str() + p + pat.size(), &end);
    return end != line.c_str() + p + pat.size();
}

// entries of the cache file: one `"key": {...}` per line
std::vector<std::pair<std::string, std::string>> cache_read(const char* path) {
    std::vector<std::pair<std::string, std::string>> out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    std::string line;
    char buf[4096];
    while (std::fgets(buf, sizeof buf, f)) {
        line = buf;
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        const size_t br = line.find('{', q1 == std::string::npos ? 0 : q1);
        const size_t be = line.rfind('}');
        if (q1 == std::string::npos || br == std::string::npos || be == std::string::npos || be < br) continue;
        out.emplace_back(line.substr(q0 + 1, q1 - q0 - 1), line.substr(br, be - br + 1));
    }
    std::fclose(f);
    return out;
}

bool cache_lookup(const char* path, const std::string& key, me_batch_tuning* t) {
    for (const auto& kv : cache_read(path)) {
        if (kv.first != key) continue;
        double blk, wpc, zd, ms;
        if (json_field(kv.second, "block", &blk) && json_field(kv.second, "wg_per_cu", &wpc) &&
            json_field(kv.second, "zdiv", &zd) && json_field(kv.second, "stage_ms", &ms)) {
            t->block = (int32_t)blk;
            t->wg_per_cu = (int32_t)wpc;
            t->zdiv = (int32_t)zd;
            t->stage_ms = ms;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const me_batch_tuning& t) {
    auto entries = cache_read(path);
    char val[256];
    std::snprintf(val, sizeof val, "{\"block\": %d, \"wg_per_cu\": %d, \"zdiv\": %d, \"stage_ms\": %.6f}", t.block,
                  t.wg_per_cu, t.zdiv, t.stage_ms);
    bool found = false;
    for (auto& kv : entries)
        if (kv.first == key) { kv.second = val; found = true; }
    if (!found) entries.emplace_back(key, val);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i)
        std::fprintf(f, "\"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                     i + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

template <typename T>
me_status batch_time_stage(me_batch* b, int reps, double* ms) {
    using C = cx_t<T>;
    const int n = (int)b->sys.size();
    std::vector<const C*> u(n);
    std::vector<C*> out(n);
    // a three-stream stage as in a step: u (bufA, a copy of psi made by the
    // caller), psi0 and the output (bufB) are three distinct arrays, so that
    // the timing sees the step's memory traffic (with u = psi0 the second
    // read would hit cache)
    for (int i = 0; i < n; ++i) {
        u[i] = (const C*)b->sys[i]->w.bufA;
        out[i] = (C*)b->sys[i]->w.bufB;
    }
    const int slot = 2 * b->K;                 // the tuning slot, outside a step's range
    const bool timing = b->timing;
    b->timing = false;
    hipEvent_t e0 = batch_event(b), e1 = batch_event(b);
    if (!e0 || !e1) { b->timing = timing; b->err = "hipEventCreate failed"; return ME_EDEVICE; }
    me_status st = ME_OK;
    for (int r = 0; r <= reps && st == ME_OK; ++r) {
        if (r == 1) BHIP(hipEventRecord(e0, b->stream));
        BHIP(launch_zero_i32(b->counters + slot * QUEUE_SLOTS, QUEUE_SLOTS, b->stream));
        st = batch_stage<T>(b, u, out, 0, 1, false, slot, MODE_HORNER);
    }
    b->timing = timing;
    if (st != ME_OK) return st;
    BHIP(hipEventRecord(e1, b->stream));
    BHIP(hipEventSynchronize(e1));
    float t = 0.f;
    BHIP(hipEventElapsedTime(&t, e0, e1));
    b->ev_pool.push_back(e0);
    b->ev_pool.push_back(e1);
    *ms = t / reps;
    return ME_OK;
}

template <typename T>
me_status batch_autotune(me_batch* b, me_batch_tuning* best) {
    best->stage_ms = 0.0;
    bool any = false;
    for (me_system* s : b->sys)            // the timed stages' u (batch_time_stage)
        BHIP(hipMemcpyAsync(s->w.bufA, s->w.psi, (size_t)s->g.n_orb * s->g.stride * sizeof(cx_t<T>),
                            hipMemcpyDeviceToDevice, b->stream));
    for (int block : {256, 512, 768, 1024}) {
        for (int zdiv : {1, 2, 4}) {
            me_batch_tuning t{};
            t.block = block;
            t.zdiv = zdiv;
            std::vector<BatchTile> tiles;
            size_t lds = 0;
            if (!batch_tiles(b, t, tiles, lds)) continue;
            const int wmax = std::min(4, batch_max_wpc<T>(b, block, lds, tiles));
            for (int w = wmax >= 1 ? 0 : 1; w <= wmax; ++w) {     // 0: one item per workgroup
                t.wg_per_cu = w;
                if (batch_apply_tuning(b, t) != ME_OK) continue;
                double ms = 0.0;
                CHK(batch_time_stage<T>(b, 8, &ms));
                if (!any || ms < best->stage_ms) {
                    *best = t;
                    best->stage_ms = ms;
                    any = true;
                }
            }
        }
    }
    if (!any) {
        b->err = "no workgroup shape fits this batch";
        return ME_EUNSUPPORTED;
    }
    return batch_apply_tuning(b, *best);
}

// ------------------------------------------------------------ Car-Parrinello
// The comparison scheme of sec. 3 (eq. L_CP, eq. EoM_CP) with the electronic
// RATTLE / velocity Verlet integrator the paper uses for it (sec. 5): per
// step one H psi and five O(N_W^2 N_C) complex GEMMs (the matrices A, B, Q
// and the rotations Psi X, Psi Y) on rocBLAS (MFMA), against eight H psi and
// no N_W^2 work for the modified Ehrenfest step.

#define BLASCHK(expr)                                                                  \
    do {                                                                               \
        rocblas_status b_ = (expr);                                                    \
        if (b_ != rocblas_status_success) {                                            \
            sys->err = std::string(#expr) + ": rocblas status " + std::to_string((int)b_); \
            return ME_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

// C = alpha op(A) op(B) + beta C, column-major complex, alpha and beta real
rocblas_status cgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k, double alpha,
                     const float2* A, int lda, const float2* B, int ldb, double beta, float2* C, int ldc) {
    const rocblas_float_complex al((float)alpha, 0.0f), be((float)beta, 0.0f);
    return rocblas_cgemm(h, ta, tb, m, n, k, &al, reinterpret_cast<const rocblas_float_complex*>(A), lda,
                         reinterpret_cast<const rocblas_float_complex*>(B), ldb, &be,
                         reinterpret_cast<rocblas_float_complex*>(C), ldc);
}
rocblas_status cgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k, double alpha,
                     const double2* A, int lda, const double2* B, int ldb, double beta, double2* C, int ldc) {
    const rocblas_double_complex al(alpha, 0.0), be(beta, 0.0);
    return rocblas_zgemm(h, ta, tb, m, n, k, &al, reinterpret_cast<const rocblas_double_complex*>(A), lda,
                         reinterpret_cast<const rocblas_double_complex*>(B), ldb, &be,
                         reinterpret_cast<rocblas_double_complex*>(C), ldc);
}

rocblas_status cgemm_batched(rocblas_handle h, int m, int n, int k, const float2* A, int lda, int64_t sa,
                             const float2* B, int ldb, int64_t sb, float2* C, int ldc, int64_t sc, int batch) {
    const rocblas_float_complex al(1.0f, 0.0f), be(0.0f, 0.0f);
    return rocblas_cgemm_strided_batched(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n, k,
                                         &al, reinterpret_cast<const rocblas_float_complex*>(A), lda, sa,
                                         reinterpret_cast<const rocblas_float_complex*>(B), ldb, sb, &be,
                                         reinterpret_cast<rocblas_float_complex*>(C), ldc, sc, batch);
}
rocblas_status cgemm_batched(rocblas_handle h, int m, int n, int k, const double2* A, int lda, int64_t sa,
                             const double2* B, int ldb, int64_t sb, double2* C, int ldc, int64_t sc, int batch) {
    const rocblas_double_complex al(1.0, 0.0), be(0.0, 0.0);
    return rocblas_zgemm_strided_batched(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n, k,
                                         &al, reinterpret_cast<const rocblas_double_complex*>(A), lda, sa,
                                         reinterpret_cast<const rocblas_double_complex*>(B), ldb, sb, &be,
                                         reinterpret_cast<rocblas_double_complex*>(C), ldc, sc, batch);
}

// out = h^3 X^H Y (N_W x N_W, FP64) for orbital sets X, Y of the system: the
// grid points are cut into CP_KSPLIT slices, each slice's product is one
// batch of a strided batched GEMM (the library then spreads the work over
// the whole GPU instead of running a few output tiles down all the points),
// the remainder is one more product, and the partial matrices are summed in
// FP64 in a fixed order
template <typename T>
me_status cp_overlap(me_system* sys, const cx_t<T>* X, const cx_t<T>* Y, double2* out) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const int n = g.n_orb, ld = (int)g.stride;
    const int64_t kc = g.N / CP_KSPLIT, rem = g.N - kc * CP_KSPLIT;
    C* part = (C*)sys->w.cp_gpart;
    int nb = 0;
    if (kc > 0) {
        BLASCHK(cgemm_batched(sys->blas, n, n, (int)kc, X, ld, kc, Y, ld, kc, part, n, (int64_t)n * n, CP_KSPLIT));
        nb = CP_KSPLIT;
    }
    if (rem > 0) {
        const int64_t o = kc * CP_KSPLIT;
        BLASCHK(cgemm_batched(sys->blas, n, n, (int)rem, X + o, ld, 0, Y + o, ld, 0, part + (int64_t)nb * n * n, n,
                              0, 1));
        ++nb;
    }
    HIPCHK(launch_cp_reduce<T>(part, nb, n, sys->prm.h * sys->prm.h * sys->prm.h, out, sys->stream));
    return ME_OK;
}

// out = H in for the system's n_orb orbitals (stride g.stride), with the
// current v_eff (veff0) and projector tables
template <typename T>
me_status apply_h_self(me_system* sys, const cx_t<T>* in, cx_t<T>* out) {
    const Geometry& g = sys->g;
    const double ekb_h3 = sys->prm.kb_energy * sys->prm.h * sys->prm.h * sys->prm.h;
    CHK(gather<T>(sys, in, g.stride, g.n_orb, sys->tab_cur, ekb_h3));
    StencilArgs<T> a = base_args<T>(sys, (const T*)sys->w.veff0, g.n_orb);
    a.u = in;
    a.psi0 = in;
    a.out = out;
    HIPCHK(launch_stencil<T>(a, MODE_APPLY, false, g.ty, g.px, sys->stream));
    if (g.n_ions > 0)
        HIPCHK(launch_kb_fixup<T>(out, g.stride, g.n_orb, tables(sys, sys->tab_cur), (const cx_t<T>*)sys->w.cnl, 1.0,
                                  0.0, nullptr, sys->stream));
    return ME_OK;
}

constexpr double CP_TOL = 1e-12;     // max |residual| of the position constraint

// Corrections of the constraint iteration: it contracts by about
// q = dt^2 E_max / (2 mu_cp) per correction (I - B is of that size), E_max
// estimated by the edge of the finite-difference kinetic spectrum
// (-3/(2h^2) times the 1-D symbol at k = pi) plus 10 hartree for the
// potentials; enough corrections to reach CP_TOL, at least 8, at most 60.
int cp_max_iter(const me_system* sys) {
    const double h = sys->prm.h;
    const double c[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
    double sym = c[0];
    for (int m = 1; m <= 4; ++m) sym += 2.0 * c[m] * ((m % 2) ? -1.0 : 1.0);
    const double e_max = -1.5 * sym / (h * h) + 10.0;
    const double q = sys->dt_cp * sys->dt_cp * e_max / (2.0 * sys->mu_cp);
    if (q >= 0.95) return 60;
    const int it = (int)std::ceil(std::log(CP_TOL) / std::log(std::max(q, 1e-3))) + 4;
    return std::min(60, std::max(8, it));
}

template <typename T>
me_status cp_begin_impl(me_system* sys) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    HIPCHK(hipMemsetAsync(sys->w.bufA, 0, (size_t)g.n_orb * g.stride * g.bc, sys->stream));   // psi' = 0
    CHK(make_veff(sys, 0.0, false));
    CHK(apply_h_self<T>(sys, (const C*)sys->w.psi, (C*)sys->w.bufB));
    return ME_OK;
}

template <typename T>
me_status cp_step_impl(me_system* sys, bool energy) {
    using C = cx_t<T>;
    const Geometry& g = sys->g;
    const double dt = sys->dt_cp, mu = sys->mu_cp;
    const double h3 = sys->prm.h * sys->prm.h * sys->prm.h;
    const int n = g.n_orb, N = (int)g.N, ld = (int)g.stride;
    const int next = sys->tab_cur ^ 1;
    C* psi = (C*)sys->w.psi;
    C* pdot = (C*)sys->w.bufA;
    C* trial = (C*)sys->w.bufB;                 // H psi on entry
    double2 *A = sys->w.cpA, *B = sys->w.cpB, *Q = sys->w.cpQ;
    C *X = (C*)sys->w.cpX, *Y = (C*)sys->w.cpY;
    const rocblas_operation NN = rocblas_operation_none;
    // 1. ions R(t+dt); V_loc and projector tables there
    HIPCHK(launch_ions_predict(sys->w.pos, sys->w.vel, sys->w.frc, sys->w.mass, g.n_ions, dt, sys->prm.freeze_ions,
                               sys->w.pos_next, sys->stream));
    CHK(ion_fields(sys, sys->w.pos_next, sys->w.vloc_next));
    CHK(build_tables(sys, sys->w.pos_next, next));
    // 2-3. unconstrained orbitals, the constraint matrices, the rotation
    HIPCHK(launch_cp_predict<T>(trial, psi, pdot, g.stride, n, g.N, dt, dt * dt / (2.0 * mu), sys->stream));
    CHK(cp_overlap<T>(sys, trial, trial, A));
    CHK(cp_overlap<T>(sys, psi, trial, B));
    HIPCHK(launch_cp_solve_x<T>(A, B, n, CP_TOL, cp_max_iter(sys), sys->w.cpX64, sys->w.cpR64, sys->w.cp_part, X,
                                sys->w.cp_info, sys->stream));
    BLASCHK(cgemm(sys->blas, NN, NN, N, n, n, 1.0, psi, ld, X, n, 1.0, trial, ld));
    // 4. half-step velocities; the new orbitals become the state
    HIPCHK(launch_cp_halfvel<T>(pdot, trial, psi, g.stride, n, g.N, 1.0 / dt, sys->stream));
    std::swap(sys->w.psi, sys->w.bufB);
    psi = (C*)sys->w.psi;
    C* hpsi = (C*)sys->w.bufB;
    // 5. density, potentials and forces at the new configuration; ions finished
    CHK(density_vhxc(sys, energy));
    CHK(forces_parts(sys, sys->w.pos_next, next));
    HIPCHK(launch_ions_finish(sys->w.pos, sys->w.vel, sys->w.frc, sys->w.pos_next, sys->w.floc, sys->w.fnl,
                              sys->w.fion, sys->w.mass, g.n_ions, dt, sys->prm.freeze_ions, sys->stream));
    std::swap(sys->w.vloc_cur, sys->w.vloc_next);
    sys->tab_cur = next;
    sys->step += 1;
    CHK(make_veff(sys, 0.0, false));
    CHK(apply_h_self<T>(sys, psi, hpsi));
    // 6. velocity half kick and the velocity constraint
    HIPCHK(launch_cp_kick<T>(pdot, hpsi, g.stride, n, g.N, dt / (2.0 * mu), sys->stream));
    CHK(cp_overlap<T>(sys, psi, pdot, Q));
    HIPCHK(launch_cp_velocity_matrix<T>(Q, n, Y, sys->stream));
    BLASCHK(cgemm(sys->blas, NN, NN, N, n, n, 1.0, psi, ld, Y, n, 1.0, pdot, ld));
    if (energy) HIPCHK(launch_cp_sq_partial<T>(pdot, g.stride, n, g.N, sys->w.fict_part, sys->stream));
    return finalize(sys, false, energy, energy ? sys->w.fict_part : nullptr, sys->prm.occ * mu * h3,
                    sys->w.cp_info);
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* me_strerror(me_status s) {
    switch (s) {
    case ME_OK: return "ok";
    case ME_EINVAL: return "invalid argument";
    case ME_ENOMEM: return "workspace too small";
    case ME_EDEVICE: return "device error";
    case ME_ESTATE: return "invalid state";
    case ME_EUNSTABLE: return "propagation unstable";
    case ME_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* me_last_error(const me_system* sys) {
    return sys ? sys->err.c_str() : g_init_error.c_str();
}

me_status me_workspace_size(const me_params* p, size_t* bytes) {
    try {
        std::string err;
        me_status st = validate(p, err);
        if (st != ME_OK) { g_init_error = err; return st; }
        if (!bytes) { g_init_error = "bytes is NULL"; return ME_EINVAL; }
        Geometry g = make_geometry(p);
        std::vector<double> z(p->zval, p->zval + p->n_ions);
        g.ewald_ng = (int)ewald_setup(p->n[0] * p->h, z).wv.size();
        *bytes = carve(g, nullptr).total;
        return ME_OK;
    } catch (...) {
        g_init_error = "internal error";
        return ME_EINVAL;
    }
}

// the side stream of a system, its FFT execution info and events (waits for
// the stream first)
static void release_side(me_system* sys) {
    if (sys->side) hipStreamSynchronize(sys->side);
    if (sys->info_side) rocfft_execution_info_destroy(sys->info_side);
    for (int i = 0; i < 2; ++i) {
        if (sys->ev_fork[i]) hipEventDestroy(sys->ev_fork[i]);
        if (sys->ev_join[i]) hipEventDestroy(sys->ev_join[i]);
        sys->ev_fork[i] = sys->ev_join[i] = nullptr;
    }
    if (sys->side) hipStreamDestroy(sys->side);
    sys->side = nullptr;
    sys->info_side = nullptr;
}

me_status me_init_system(const me_params* p, void* workspace, size_t ws_bytes, void* stream,
                         me_system** out) {
    me_system* sys = nullptr;
    try {
        std::string err;
        me_status st = validate(p, err);
        if (st != ME_OK) { g_init_error = err; return st; }
        if (!out || !workspace) { g_init_error = "out/workspace is NULL"; return ME_EINVAL; }
        if (reinterpret_cast<uintptr_t>(workspace) % 256) { g_init_error = "workspace must be 256-byte aligned"; return ME_EINVAL; }
        if (p->n[0] != p->n[1] || p->n[1] != p->n[2]) {
            g_init_error = "only cubic grids are supported";
            return ME_EUNSUPPORTED;
        }
        sys = new (std::nothrow) me_system();
        if (!sys) { g_init_error = "out of host memory"; return ME_EINVAL; }
        sys->prm = *p;
        sys->pos0.assign(p->pos, p->pos + 3 * p->n_ions);
        if (p->vel) sys->vel0.assign(p->vel, p->vel + 3 * p->n_ions);
        else sys->vel0.assign(3 * p->n_ions, 0.0);
        sys->mass.assign(p->mass, p->mass + p->n_ions);
        sys->zval.assign(p->zval, p->zval + p->n_ions);
        sys->prm.pos = sys->prm.vel = sys->prm.mass = sys->prm.zval = nullptr;
        sys->g = make_geometry(p);
        sys->ew = ewald_setup(p->n[0] * p->h, sys->zval);
        sys->g.ewald_ng = (int)sys->ew.wv.size();
        const size_t need = carve(sys->g, nullptr).total;
        if (ws_bytes < need) {
            g_init_error = "workspace too small: need " + std::to_string(need) + " bytes";
            delete sys;
            return ME_ENOMEM;
        }
        sys->w = carve(sys->g, reinterpret_cast<char*>(workspace));
        sys->stream = reinterpret_cast<hipStream_t>(stream);
        const double L = p->n[0] * p->h;
        sys->geo.h = p->h;
        sys->geo.L[0] = p->n[0] * p->h;
        sys->geo.L[1] = p->n[1] * p->h;
        sys->geo.L[2] = p->n[2] * p->h;
        sys->geo.rcut2 = p->kb_rcut * p->kb_rcut;
        sys->geo.inv2s2 = 1.0 / (2.0 * p->kb_sigma * p->kb_sigma);
        sys->geo.pnorm = std::pow(M_PI * p->kb_sigma * p->kb_sigma, -0.75);
        sys->geo.inv_s2 = 1.0 / (p->kb_sigma * p->kb_sigma);
        sys->ewp.L = L;
        sys->ewp.eta = sys->ew.eta;
        sys->ewp.rc = sys->ew.rc;
        sys->ewp.nmax = sys->ew.nmax;
        sys->ewp.ng = sys->g.ewald_ng;
        sys->ewp.gv = sys->w.ewald_gv;
        sys->ewp.wv = sys->w.ewald_wv;

        auto fail = [&](me_status s2) {
            g_init_error = sys->err;
            release_side(sys);
            if (sys->info) rocfft_execution_info_destroy(sys->info);
            if (sys->r2c) rocfft_plan_destroy(sys->r2c);
            if (sys->c2r) rocfft_plan_destroy(sys->c2r);
            if (sys->info2) rocfft_execution_info_destroy(sys->info2);
            if (sys->r2c2) rocfft_plan_destroy(sys->r2c2);
            if (sys->c2r2) rocfft_plan_destroy(sys->c2r2);
            delete sys;
            return s2;
        };
#define INITCHK(expr)                                                       \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            sys->err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
            return fail(ME_EDEVICE);                                        \
        }                                                                   \
    } while (0)
        const size_t n3 = 3 * (size_t)p->n_ions * sizeof(double);
        if (p->n_ions > 0) {
            INITCHK(hipMemcpyAsync(sys->w.pos, sys->pos0.data(), n3, hipMemcpyHostToDevice, sys->stream));
            INITCHK(hipMemcpyAsync(sys->w.vel, sys->vel0.data(), n3, hipMemcpyHostToDevice, sys->stream));
            INITCHK(hipMemcpyAsync(sys->w.mass, sys->mass.data(), n3 / 3, hipMemcpyHostToDevice, sys->stream));
            INITCHK(hipMemcpyAsync(sys->w.zval, sys->zval.data(), n3 / 3, hipMemcpyHostToDevice, sys->stream));
            INITCHK(hipMemcpyAsync(sys->w.ewald_gv, sys->ew.gv.data(), sys->ew.gv.size() * 8,
                                   hipMemcpyHostToDevice, sys->stream));
            INITCHK(hipMemcpyAsync(sys->w.ewald_wv, sys->ew.wv.data(), sys->ew.wv.size() * 8,
                                   hipMemcpyHostToDevice, sys->stream));
        }
        INITCHK(hipMemsetAsync(sys->w.vstatic, 0, sys->g.N * 8, sys->stream));
        INITCHK(hipMemsetAsync(sys->w.rep, 0, SLOT_COUNT * 8, sys->stream));
        // FFT plans: lengths fastest-first
        if (rocfft_setup() != rocfft_status_success) { sys->err = "rocfft_setup failed"; return fail(ME_EDEVICE); }
        size_t len[3] = {(size_t)p->n[0], (size_t)p->n[1], (size_t)p->n[2]};
        if (rocfft_plan_create(&sys->r2c, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                               rocfft_precision_double, 3, len, 1, nullptr) != rocfft_status_success ||
            rocfft_plan_create(&sys->c2r, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                               rocfft_precision_double, 3, len, 1, nullptr) != rocfft_status_success) {
            sys->err = "rocfft_plan_create failed";
            return fail(ME_EDEVICE);
        }
        size_t w1 = 0, w2 = 0;
        rocfft_plan_get_work_buffer_size(sys->r2c, &w1);
        rocfft_plan_get_work_buffer_size(sys->c2r, &w2);
        if (std::max(w1, w2) > sys->g.fft_work) {
            sys->err = "rocFFT work buffer larger than reserved";
            return fail(ME_EUNSUPPORTED);
        }
        if (rocfft_execution_info_create(&sys->info) != rocfft_status_success ||
            rocfft_execution_info_set_stream(sys->info, sys->stream) != rocfft_status_success ||
            (std::max(w1, w2) > 0 &&
             rocfft_execution_info_set_work_buffer(sys->info, sys->w.fft_work, sys->g.fft_work) !=
                 rocfft_status_success)) {
            sys->err = "rocfft execution info failed";
            return fail(ME_EDEVICE);
        }
        if (sys->g.finite) {
            const me_status fs = finite_setup(sys, p);
            if (fs != ME_OK) return fail(fs);
        }
        if (env_int("MODEHR_OVERLAP", 1) != 0) {
            INITCHK(hipStreamCreateWithFlags(&sys->side, hipStreamNonBlocking));
            for (int i = 0; i < 2; ++i) {
                INITCHK(hipEventCreateWithFlags(&sys->ev_fork[i], hipEventDisableTiming));
                INITCHK(hipEventCreateWithFlags(&sys->ev_join[i], hipEventDisableTiming));
            }
            if (rocfft_execution_info_create(&sys->info_side) != rocfft_status_success ||
                rocfft_execution_info_set_stream(sys->info_side, sys->side) != rocfft_status_success ||
                (std::max(w1, w2) > 0 &&
                 rocfft_execution_info_set_work_buffer(sys->info_side, sys->w.fft_work, sys->g.fft_work) !=
                     rocfft_status_success)) {
                sys->err = "rocfft execution info failed (side stream)";
                return fail(ME_EDEVICE);
            }
        }
#undef INITCHK
        *out = sys;
        return ME_OK;
    } catch (...) {
        g_init_error = "internal error during init";
        delete sys;
        return ME_EDEVICE;
    }
}

me_status me_destroy(me_system* sys) {
    if (!sys) return ME_OK;
    hipStreamSynchronize(sys->stream);
    release_side(sys);
    if (sys->blas) rocblas_destroy_handle(sys->blas);
    if (sys->info) rocfft_execution_info_destroy(sys->info);
    if (sys->r2c) rocfft_plan_destroy(sys->r2c);
    if (sys->c2r) rocfft_plan_destroy(sys->c2r);
    if (sys->info2) rocfft_execution_info_destroy(sys->info2);
    if (sys->r2c2) rocfft_plan_destroy(sys->r2c2);
    if (sys->c2r2) rocfft_plan_destroy(sys->c2r2);
    for (auto& e : sys->ev) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
    for (auto& e : sys->ev_pool) hipEventDestroy(e);
    delete sys;
    return ME_OK;
}

me_status me_sync(me_system* sys) {
    if (!sys) return ME_EINVAL;
    HIPCHK(hipStreamSynchronize(sys->stream));
    HIPCHK(hipGetLastError());
    if (sys->has_state) return read_report(sys, nullptr);
    return ME_OK;
}

me_status me_set_state(me_system* sys, const void* psi_dev, int64_t orb_stride) {
    if (!sys) return ME_EINVAL;
    if (!psi_dev || orb_stride < sys->g.N) { sys->err = "psi is NULL or orb_stride < N"; return ME_EINVAL; }
    try {
        const Geometry& g = sys->g;
        HIPCHK(hipMemcpy2DAsync(sys->w.psi, g.stride * g.bc, psi_dev, orb_stride * g.bc, g.N * g.bc, g.n_orb,
                                hipMemcpyDeviceToDevice, sys->stream));
        if (g.finite) {     // the orbitals live on the box: values outside are dropped
            if (g.f64)
                HIPCHK(launch_mask_orbitals<double>((double2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->w.mask, sys->stream));
            else
                HIPCHK(launch_mask_orbitals<float>((float2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->w.mask, sys->stream));
        }
        const size_t n3 = 3 * (size_t)g.n_ions * sizeof(double);
        if (g.n_ions > 0) {
            HIPCHK(hipMemcpyAsync(sys->w.pos, sys->pos0.data(), n3, hipMemcpyHostToDevice, sys->stream));
            HIPCHK(hipMemcpyAsync(sys->w.vel, sys->vel0.data(), n3, hipMemcpyHostToDevice, sys->stream));
        }
        CHK(initial_fields(sys));
        sys->step = 0;
        sys->has_state = true;
        sys->cp_ready = false;
        HIPCHK(hipStreamSynchronize(sys->stream));
        return ME_OK;
    } catch (...) {
        sys->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_get_state(me_system* sys, void* psi_dev, int64_t orb_stride) {
    if (!sys) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    if (!psi_dev || orb_stride < sys->g.N) { sys->err = "psi is NULL or orb_stride < N"; return ME_EINVAL; }
    const Geometry& g = sys->g;
    HIPCHK(hipMemcpy2DAsync(psi_dev, orb_stride * g.bc, sys->w.psi, g.stride * g.bc, g.N * g.bc, g.n_orb,
                            hipMemcpyDeviceToDevice, sys->stream));
    return ME_OK;
}

me_status me_apply_H(me_system* sys, const void* psi_in_dev, void* hpsi_out_dev, int32_t n_orb,
                     int64_t orb_stride) {
    if (!sys) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    const Geometry& g = sys->g;
    if (!psi_in_dev || !hpsi_out_dev || n_orb < 1 || orb_stride < g.N) {
        sys->err = "bad apply_H arguments";
        return ME_EINVAL;
    }
    const char* a0 = (const char*)psi_in_dev;
    const char* a1 = a0 + ((size_t)(n_orb - 1) * orb_stride + g.N) * g.bc;
    const char* b0 = (const char*)hpsi_out_dev;
    const char* b1 = b0 + ((size_t)(n_orb - 1) * orb_stride + g.N) * g.bc;
    if (a0 < b1 && b0 < a1) { sys->err = "input and output overlap"; return ME_EINVAL; }
    if (((uintptr_t)a0 | (uintptr_t)b0 | (uintptr_t)(orb_stride * g.bc)) % 16) {
        sys->err = "orbital rows must be 16-byte aligned";
        return ME_EINVAL;
    }
    CHK(make_veff(sys, 0.0, false));
    const double ekb_h3 = sys->prm.kb_energy * sys->prm.h * sys->prm.h * sys->prm.h;
    for (int o0 = 0; o0 < n_orb; o0 += g.n_orb) {
        const int nb = std::min(g.n_orb, n_orb - o0);
        if (g.f64) {
            const double2* in = (const double2*)psi_in_dev + (size_t)o0 * orb_stride;
            double2* outp = (double2*)hpsi_out_dev + (size_t)o0 * orb_stride;
            HIPCHK(launch_kb_gather<double>(in, orb_stride, nb, g.n_ions, tables(sys, sys->tab_cur), ekb_h3,
                                            (double2*)sys->w.cnl, sys->stream));
            StencilArgs<double> a = base_args<double>(sys, (const double*)sys->w.veff0, nb);
            a.u = in; a.psi0 = in; a.out = outp; a.stride = orb_stride;
            a.zchunk = g.nz; a.nzc = 1;
            HIPCHK(launch_stencil<double>(a, MODE_APPLY, false, g.ty, g.px, sys->stream));
            if (g.n_ions > 0)
                HIPCHK(launch_kb_fixup<double>(outp, orb_stride, nb, tables(sys, sys->tab_cur), (const double2*)sys->w.cnl,
                                               1.0, 0.0, nullptr, sys->stream));
        } else {
            const float2* in = (const float2*)psi_in_dev + (size_t)o0 * orb_stride;
            float2* outp = (float2*)hpsi_out_dev + (size_t)o0 * orb_stride;
            CHK(gather<float>(sys, in, orb_stride, nb, sys->tab_cur, ekb_h3));
            StencilArgs<float> a = base_args<float>(sys, (const float*)sys->w.veff0, nb);
            a.u = in; a.psi0 = in; a.out = outp; a.stride = orb_stride;
            a.zchunk = g.nz; a.nzc = 1;
            HIPCHK(launch_stencil<float>(a, MODE_APPLY, false, g.ty, g.px, sys->stream));
            if (g.n_ions > 0)
                HIPCHK(launch_kb_fixup<float>(outp, orb_stride, nb, tables(sys, sys->tab_cur), (const float2*)sys->w.cnl,
                                              1.0, 0.0, nullptr, sys->stream));
        }
    }
    return ME_OK;
}

me_status me_propagate_step(me_system* sys, const double* ctrl, me_step_report* rep) {
    if (!sys) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state: call me_set_state first"; return ME_ESTATE; }
    const double eps = ctrl ? *ctrl : 0.0;
    if (!std::isfinite(eps)) { sys->err = "control amplitude must be finite"; return ME_EINVAL; }
    if (eps != 0.0 && sys->g.finite) { sys->err = "the finite box runs without an external field"; return ME_EUNSUPPORTED; }
    try {
        me_status st = sys->g.f64 ? step_impl<double>(sys, eps, rep != nullptr)
                                  : step_impl<float>(sys, eps, rep != nullptr);
        if (st != ME_OK) return st;
        if (rep) return read_report(sys, rep);
        return ME_OK;
    } catch (...) {
        sys->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_cp_begin(me_system* sys, double mu_cp, double dt) {
    if (!sys) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state: call me_set_state first"; return ME_ESTATE; }
    if (!(mu_cp > 0.0) || !std::isfinite(mu_cp) || !std::isfinite(dt) || dt == 0.0) {
        sys->err = "mu_cp must be positive and dt finite and nonzero";
        return ME_EINVAL;
    }
    if (sys->g.N > INT32_MAX || sys->g.stride > INT32_MAX) {
        sys->err = "grid too large for 32-bit GEMM sizes";
        return ME_EUNSUPPORTED;
    }
    try {
        if (!sys->blas) {
            rocblas_handle h = nullptr;
            if (rocblas_create_handle(&h) != rocblas_status_success) {
                sys->err = "rocblas_create_handle failed";
                return ME_EDEVICE;
            }
            sys->blas = h;
        }
        BLASCHK(rocblas_set_stream(sys->blas, sys->stream));
        sys->mu_cp = mu_cp;
        sys->dt_cp = dt;
        const me_status st = sys->g.f64 ? cp_begin_impl<double>(sys) : cp_begin_impl<float>(sys);
        sys->cp_ready = st == ME_OK;
        return st;
    } catch (...) {
        sys->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_cp_step(me_system* sys, me_step_report* rep) {
    if (!sys) return ME_EINVAL;
    if (!sys->cp_ready) { sys->err = "call me_cp_begin first (after the last state change)"; return ME_ESTATE; }
    try {
        BLASCHK(rocblas_set_stream(sys->blas, sys->stream));
        me_status st = sys->g.f64 ? cp_step_impl<double>(sys, rep != nullptr) : cp_step_impl<float>(sys, rep != nullptr);
        if (st != ME_OK) {
            sys->cp_ready = false;
            return st;
        }
        if (rep) return read_report(sys, rep);
        return ME_OK;
    } catch (...) {
        sys->cp_ready = false;
        sys->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_report(me_system* sys, me_step_report* rep) {
    if (!sys || !rep) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    // energies of the current state need fresh partials of rho V_H and e_x,
    // and the nonlocal / Ewald parts at the current positions
    const Geometry& g = sys->g;
    const double L[3] = {g.nx * sys->prm.h, g.ny * sys->prm.h, g.nz * sys->prm.h};
    CHK(density_vhxc(sys, true, false));
    HIPCHK(launch_phases(sys->w.pos, g.n_ions, g.nx, g.ny, g.nz, L, sys->w.phase, sys->w.phaseT, sys->stream));
    CHK(forces_parts(sys, sys->w.pos, sys->tab_cur));
    CHK(finalize(sys, false, true));
    return read_report(sys, rep);
}

me_status me_density(me_system* sys, double* rho_dev) {
    if (!sys || !rho_dev) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    HIPCHK(hipMemcpyAsync(rho_dev, sys->w.rho, sys->g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    return ME_OK;
}

me_status me_forces(me_system* sys, double* f_host) {
    if (!sys || !f_host) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    if (sys->g.n_ions == 0) return ME_OK;
    HIPCHK(hipMemcpyAsync(f_host, sys->w.frc, 3 * 8 * sys->g.n_ions, hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    return ME_OK;
}

me_status me_get_ions(me_system* sys, double* pos_host, double* vel_host) {
    if (!sys) return ME_EINVAL;
    if (sys->g.n_ions == 0) return ME_OK;
    if (pos_host)
        HIPCHK(hipMemcpyAsync(pos_host, sys->w.pos, 3 * 8 * sys->g.n_ions, hipMemcpyDeviceToHost, sys->stream));
    if (vel_host)
        HIPCHK(hipMemcpyAsync(vel_host, sys->w.vel, 3 * 8 * sys->g.n_ions, hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    return ME_OK;
}

me_status me_get_potential(me_system* sys, int32_t which, double* v_dev) {
    if (!sys || !v_dev || which < 0 || which > 2) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    const Geometry& g = sys->g;
    if (which == 0) {
        HIPCHK(hipMemcpyAsync(v_dev, sys->w.vloc_cur, g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    } else if (which == 1) {
        HIPCHK(hipMemcpyAsync(v_dev, sys->w.hist[sys->hist_newest], g.N * 8, hipMemcpyDeviceToDevice,
                              sys->stream));
    } else {
        HIPCHK(hipMemcpyAsync(v_dev, sys->w.vloc_cur, g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
        HIPCHK(launch_add(v_dev, sys->w.hist[sys->hist_newest], g.N, sys->stream));
    }
    return ME_OK;
}

me_status me_set_static_potential(me_system* sys, const double* dv_dev) {
    if (!sys) return ME_EINVAL;
    sys->cp_ready = false;          // H changed: the stored H psi is stale
    if (dv_dev) {
        HIPCHK(hipMemcpyAsync(sys->w.vstatic, dv_dev, sys->g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
        sys->static_set = true;
    } else {
        HIPCHK(hipMemsetAsync(sys->w.vstatic, 0, sys->g.N * 8, sys->stream));
        sys->static_set = false;
    }
    return ME_OK;
}

me_status me_timing_enable(me_system* sys, int32_t enable) {
    if (!sys) return ME_EINVAL;
    HIPCHK(hipStreamSynchronize(sys->stream));
    for (auto& e : sys->ev) { sys->ev_pool.push_back(e.first); sys->ev_pool.push_back(e.second); }
    sys->ev.clear();
    sys->ev_bytes.clear();
    sys->ev_streams.clear();
    sys->timing = enable != 0;
    return ME_OK;
}

me_status me_timing_read_kind(me_system* sys, int32_t streams, int64_t* launches, double* total_ms,
                              double* total_bytes) {
    if (!sys || !launches || !total_ms || !total_bytes || (streams != 0 && streams != 2 && streams != 3))
        return ME_EINVAL;
    HIPCHK(hipStreamSynchronize(sys->stream));
    double ms = 0.0, by = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i < sys->ev.size(); ++i) {
        if (streams != 0 && sys->ev_streams[i] != streams) continue;
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, sys->ev[i].first, sys->ev[i].second));
        ms += t;
        by += sys->ev_bytes[i];
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    *total_bytes = by;
    return ME_OK;
}

me_status me_timing_read(me_system* sys, int64_t* launches, double* total_ms, double* total_bytes) {
    return me_timing_read_kind(sys, 0, launches, total_ms, total_bytes);
}

me_status me_checkpoint_size(const me_system* sys, size_t* bytes) {
    if (!sys || !bytes) return ME_EINVAL;
    *bytes = ckpt_bytes(sys->g);
    return ME_OK;
}

me_status me_save_checkpoint(me_system* sys, void* buf_dev) {
    if (!sys || !buf_dev) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    const Geometry& g = sys->g;
    char* b = (char*)buf_dev;
    CkptHeader hd{sys->step, sys->hist_count, sys->hist_newest, g.n_orb, g.n_ions, g.N, 0x4d4f444548524331LL};
    HIPCHK(hipMemcpyAsync(b, &hd, sizeof(hd), hipMemcpyHostToDevice, sys->stream));
    size_t off = 256;
    const size_t ob = (size_t)g.n_orb * g.stride * g.bc;
    HIPCHK(hipMemcpyAsync(b + off, sys->w.psi, ob, hipMemcpyDeviceToDevice, sys->stream));
    off += align_up(ob);
    for (int i = 0; i < 3; ++i)
        HIPCHK(hipMemcpyAsync(b + off + (size_t)i * g.N * 8, sys->w.hist[i], g.N * 8, hipMemcpyDeviceToDevice,
                              sys->stream));
    off += align_up(3 * (size_t)g.N * 8);
    const size_t i3 = 3 * (size_t)std::max(1, g.n_ions) * 8;
    HIPCHK(hipMemcpyAsync(b + off, sys->w.pos, i3, hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(hipMemcpyAsync(b + off + i3, sys->w.vel, i3, hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(hipMemcpyAsync(b + off + 2 * i3, sys->w.frc, i3, hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));   // the header lives on the host stack
    return ME_OK;
}

me_status me_load_checkpoint(me_system* sys, const void* buf_dev) {
    if (!sys || !buf_dev) return ME_EINVAL;
    const Geometry& g = sys->g;
    const char* b = (const char*)buf_dev;
    CkptHeader hd{};
    HIPCHK(hipMemcpyAsync(&hd, b, sizeof(hd), hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    if (hd.magic != 0x4d4f444548524331LL || hd.n_orb != g.n_orb || hd.n_ions != g.n_ions || hd.N != g.N) {
        sys->err = "checkpoint does not belong to a system of this shape";
        return ME_EINVAL;
    }
    size_t off = 256;
    const size_t ob = (size_t)g.n_orb * g.stride * g.bc;
    HIPCHK(hipMemcpyAsync(sys->w.psi, b + off, ob, hipMemcpyDeviceToDevice, sys->stream));
    off += align_up(ob);
    for (int i = 0; i < 3; ++i)
        HIPCHK(hipMemcpyAsync(sys->w.hist[i], b + off + (size_t)i * g.N * 8, g.N * 8, hipMemcpyDeviceToDevice,
                              sys->stream));
    off += align_up(3 * (size_t)g.N * 8);
    const size_t i3 = 3 * (size_t)std::max(1, g.n_ions) * 8;
    HIPCHK(hipMemcpyAsync(sys->w.pos, b + off, i3, hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(hipMemcpyAsync(sys->w.vel, b + off + i3, i3, hipMemcpyDeviceToDevice, sys->stream));
    HIPCHK(hipMemcpyAsync(sys->w.frc, b + off + 2 * i3, i3, hipMemcpyDeviceToDevice, sys->stream));
    sys->step = hd.step;
    sys->hist_count = hd.hist_count;
    sys->hist_newest = hd.hist_newest;
    // ion-dependent fields at the restored positions
    CHK(build_tables(sys, sys->w.pos, sys->tab_cur));
    CHK(ion_fields(sys, sys->w.pos, sys->w.vloc_cur));
    if (sys->g.f64)
        HIPCHK(launch_density<double>((const double2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->prm.occ, sys->w.rho,
                                      sys->stream));
    else
        HIPCHK(launch_density<float>((const float2*)sys->w.psi, g.stride, g.n_orb, g.N, sys->prm.occ, sys->w.rho,
                                     sys->stream));
    HIPCHK(hipMemsetAsync(sys->w.rep, 0, SLOT_COUNT * 8, sys->stream));
    sys->has_state = true;
    sys->cp_ready = false;
    return ME_OK;
}

me_status me_set_static_potential_coarse(me_system* sys, const double* coarse_dev, int32_t m) {
    if (sys) sys->cp_ready = false;
    if (!sys || m < 1 || sys->g.nx % m) return ME_EINVAL;
    if (!coarse_dev) return me_set_static_potential(sys, nullptr);
    HIPCHK(launch_coarse_to_fine(coarse_dev, m, sys->g.nx, sys->w.vstatic, sys->stream));
    sys->static_set = true;
    return ME_OK;
}

me_status me_dipole(me_system* sys, double* d_host) {
    if (!sys || !d_host) return ME_EINVAL;
    if (!sys->has_state) { sys->err = "no state"; return ME_ESTATE; }
    const Geometry& g = sys->g;
    const double h3 = sys->prm.h * sys->prm.h * sys->prm.h;
    // the E_loc partial buffer is free between steps
    HIPCHK(launch_field_dot(sys->w.rho, g.nx, g.N, sys->prm.h, Lx(sys), sys->w.loc_part, sys->w.scal0, h3,
                            sys->stream));
    HIPCHK(hipMemcpyAsync(d_host, sys->w.scal0, 8, hipMemcpyDeviceToHost, sys->stream));
    HIPCHK(hipStreamSynchronize(sys->stream));
    return ME_OK;
}

me_status me_adjoint_begin(me_system* sys, const double* rhobar_dev) {
    if (!sys) return ME_EINVAL;
    if (!sys->g.adjoint) { sys->err = "system created without enable_adjoint"; return ME_EUNSUPPORTED; }
    const Geometry& g = sys->g;
    const size_t ob = (size_t)g.n_orb * g.stride * g.bc;
    HIPCHK(hipMemsetAsync(sys->w.lamA, 0, ob, sys->stream));
    for (int i = 0; i < 4; ++i) HIPCHK(launch_zero(sys->w.vbar[i], g.N, sys->stream));
    HIPCHK(launch_zero(sys->w.gfine, g.N, sys->stream));
    if (rhobar_dev)
        HIPCHK(hipMemcpyAsync(sys->w.rhobar_T, rhobar_dev, g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    else
        HIPCHK(launch_dipole_rhobar(sys->w.rhobar_T, g.nx, g.N, sys->prm.h, Lx(sys), sys->stream));
    sys->adj_ready = true;
    sys->adj_pending_final = true;
    return ME_OK;
}

me_status me_adjoint_step(me_system* sys, double ctrl_n, double* g_ctrl_n) {
    if (!sys || !g_ctrl_n) return ME_EINVAL;
    if (!sys->g.adjoint || !sys->adj_ready) { sys->err = "call me_adjoint_begin first"; return ME_ESTATE; }
    if (!sys->has_state) { sys->err = "load the state of the step first"; return ME_ESTATE; }
    if (!std::isfinite(ctrl_n)) { sys->err = "control amplitude must be finite"; return ME_EINVAL; }
    try {
        return sys->g.f64 ? adjoint_step_impl<double>(sys, ctrl_n, g_ctrl_n)
                          : adjoint_step_impl<float>(sys, ctrl_n, g_ctrl_n);
    } catch (...) {
        sys->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_adjoint_grad_v(me_system* sys, double* g_fine_dev, double* g_coarse_dev, int32_t m) {
    if (!sys) return ME_EINVAL;
    if (!sys->g.adjoint || !sys->adj_ready) { sys->err = "no adjoint run"; return ME_ESTATE; }
    if (g_fine_dev)
        HIPCHK(hipMemcpyAsync(g_fine_dev, sys->w.gfine, sys->g.N * 8, hipMemcpyDeviceToDevice, sys->stream));
    if (g_coarse_dev) {
        if (m < 1 || sys->g.nx % m) return ME_EINVAL;
        HIPCHK(launch_fine_to_coarse(sys->w.gfine, m, sys->g.nx, g_coarse_dev, sys->stream));
    }
    return ME_OK;
}

// ------------------------------------------------------------------ batches

me_status me_batch_workspace_size(const me_params* ps, int32_t n_sys, size_t* bytes) {
    if (!ps || !bytes || n_sys < 1 || n_sys > MAX_BATCH) {
        g_init_error = "params/bytes NULL or n_sys outside [1, " + std::to_string(MAX_BATCH) + "]";
        return ME_EINVAL;
    }
    size_t total = 0;
    for (int i = 0; i < n_sys; ++i) {
        size_t b = 0;
        const me_status st = me_workspace_size(ps + i, &b);
        if (st != ME_OK) { g_init_error = "system " + std::to_string(i) + ": " + g_init_error; return st; }
        total += align_up(b);
    }
    *bytes = total + align_up((2 * MAX_TAYLOR + 1) * QUEUE_SLOTS * sizeof(int));
    return ME_OK;
}

me_status me_init_batch(const me_params* ps, int32_t n_sys, void* workspace, size_t ws_bytes, void* stream,
                        me_batch** out) {
    size_t need = 0;
    me_status st = me_batch_workspace_size(ps, n_sys, &need);
    if (st != ME_OK) return st;
    if (!out || !workspace) { g_init_error = "out/workspace is NULL"; return ME_EINVAL; }
    if (reinterpret_cast<uintptr_t>(workspace) % 256) { g_init_error = "workspace must be 256-byte aligned"; return ME_EINVAL; }
    if (ws_bytes < need) { g_init_error = "workspace too small: need " + std::to_string(need) + " bytes"; return ME_ENOMEM; }
    for (int i = 0; i < n_sys; ++i) {
        if (ps[i].precision != ps[0].precision || ps[i].taylor_order != ps[0].taylor_order) {
            g_init_error = "all systems of a batch need the same precision and Taylor order";
            return ME_EINVAL;
        }
        if (ps[i].enable_adjoint) { g_init_error = "batches do not run the adjoint"; return ME_EUNSUPPORTED; }
        if (ps[i].etrs_iterations) { g_init_error = "batches run AETRS"; return ME_EUNSUPPORTED; }
        if (ps[i].finite_radius > 0.0) { g_init_error = "batches run periodic cubes"; return ME_EUNSUPPORTED; }
    }
    me_batch* b = new (std::nothrow) me_batch();
    if (!b) { g_init_error = "out of host memory"; return ME_EINVAL; }
    char* base = reinterpret_cast<char*>(workspace);
    size_t off = 0;
    for (int i = 0; i < n_sys; ++i) {
        size_t sz = 0;
        me_workspace_size(ps + i, &sz);
        me_system* s = nullptr;
        st = me_init_system(ps + i, base + off, sz, stream, &s);
        if (st != ME_OK) {
            g_init_error = "system " + std::to_string(i) + ": " + g_init_error;
            for (me_system* t : b->sys) me_destroy(t);
            delete b;
            return st;
        }
        b->sys.push_back(s);
        off += align_up(sz);
    }
    b->counters = reinterpret_cast<int*>(base + off);
    b->stream = reinterpret_cast<hipStream_t>(stream);
    b->f64 = ps[0].precision == ME_F64;
    b->K = ps[0].taylor_order;
    b->order.resize(n_sys);
    for (int i = 0; i < n_sys; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        const Geometry &gx = b->sys[x]->g, &gy = b->sys[y]->g;
        return gx.N != gy.N ? gx.N > gy.N : gx.n_orb > gy.n_orb;
    });
    bool streams_ok = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
    const int n_workers = std::min(n_sys, BATCH_WORKERS);
    for (int w = 0; w < n_workers && streams_ok; ++w) {
        hipStream_t ws = nullptr;
        hipEvent_t ev = nullptr;
        streams_ok = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) == hipSuccess;
        if (streams_ok) b->workers.push_back(ws);
        streams_ok = streams_ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (streams_ok) b->ev_join.push_back(ev);
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            b->n_cu = cus;
    }
    if (!streams_ok ||
        hipMemsetAsync(b->counters, 0, (2 * MAX_TAYLOR + 1) * QUEUE_SLOTS * sizeof(int), b->stream) != hipSuccess ||
        batch_default_tuning(b) != ME_OK) {
        g_init_error = !streams_ok ? "could not create the worker streams" : (b->err.empty() ? "device error" : b->err);
        batch_release(b);
        return ME_EDEVICE;
    }
    *out = b;
    return ME_OK;
}

me_status me_batch_system(me_batch* b, int32_t i, me_system** out) {
    if (!b || !out || i < 0 || i >= (int)b->sys.size()) return ME_EINVAL;
    *out = b->sys[i];
    return ME_OK;
}

me_status me_batch_set_tuning(me_batch* b, const me_batch_tuning* t) {
    if (!b || !t) return ME_EINVAL;
    try {
        const me_status st = batch_apply_tuning(b, *t);
        if (st == ME_OK) b->tuned = true;
        return st;
    } catch (...) {
        b->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_batch_get_tuning(const me_batch* b, me_batch_tuning* t) {
    if (!b || !t) return ME_EINVAL;
    *t = b->tune;
    return ME_OK;
}

me_status me_batch_autotune(me_batch* b, const char* cache_path, me_batch_tuning* out) {
    if (!b) return ME_EINVAL;
    for (me_system* s : b->sys)
        if (!s->has_state) { b->err = "no state: call me_set_state on every system first"; return ME_ESTATE; }
    try {
        const std::string key = batch_key(b);
        me_batch_tuning t{};
        if (cache_path && cache_lookup(cache_path, key, &t) && batch_apply_tuning(b, t) == ME_OK) {
            b->tuned = true;
            if (out) *out = b->tune;
            return ME_OK;
        }
        const me_status st = b->f64 ? batch_autotune<double>(b, &t) : batch_autotune<float>(b, &t);
        if (st != ME_OK) return st;
        b->tuned = true;
        b->tune.stage_ms = t.stage_ms;
        if (cache_path) cache_store(cache_path, key, b->tune);
        if (out) *out = b->tune;
        return ME_OK;
    } catch (...) {
        b->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_propagate_batch(me_batch* b, int32_t n_steps, int32_t use_graph) {
    if (!b) return ME_EINVAL;
    if (n_steps < 0) { b->err = "n_steps must be >= 0"; return ME_EINVAL; }
    for (me_system* s : b->sys)
        if (!s->has_state) { b->err = "no state: call me_set_state on every system first"; return ME_ESTATE; }
    try {
        int done = 0;
        auto warm = [&]() {
            for (const me_system* s : b->sys)
                if (s->hist_count < 3) return false;
            return true;
        };
        while (done < n_steps && !warm()) {
            CHK(batch_step_any(b));
            ++done;
        }
        if (use_graph && n_steps - done >= BATCH_GRAPH_STEPS) {
            if (!b->exec || !(batch_phase(b) == b->phase)) CHK(batch_capture(b));
            while (n_steps - done >= BATCH_GRAPH_STEPS) {
                BHIP(hipGraphLaunch(b->exec, b->stream));
                for (me_system* s : b->sys) s->step += BATCH_GRAPH_STEPS;
                done += BATCH_GRAPH_STEPS;
            }
        }
        while (done < n_steps) {
            CHK(batch_step_any(b));
            ++done;
        }
        for (me_system* s : b->sys) BSYS(read_report(s, nullptr), s);
        return ME_OK;
    } catch (...) {
        b->err = "internal error";
        return ME_EDEVICE;
    }
}

me_status me_batch_timing_enable(me_batch* b, int32_t enable) {
    if (!b) return ME_EINVAL;
    BHIP(hipStreamSynchronize(b->stream));
    for (auto& e : b->ev) { b->ev_pool.push_back(e.first); b->ev_pool.push_back(e.second); }
    b->ev.clear();
    b->ev_bytes.clear();
    b->ev_streams.clear();
    b->timing = enable != 0;
    return ME_OK;
}

me_status me_batch_timing_read_kind(me_batch* b, int32_t streams, int64_t* launches, double* total_ms,
                                    double* total_bytes) {
    if (!b || !launches || !total_ms || !total_bytes || (streams != 0 && streams != 2 && streams != 3))
        return ME_EINVAL;
    BHIP(hipStreamSynchronize(b->stream));
    double ms = 0.0, by = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i < b->ev.size(); ++i) {
        if (streams != 0 && b->ev_streams[i] != streams) continue;
        float t = 0.f;
        BHIP(hipEventElapsedTime(&t, b->ev[i].first, b->ev[i].second));
        ms += t;
        by += b->ev_bytes[i];
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    *total_bytes = by;
    return ME_OK;
}

me_status me_batch_timing_read(me_batch* b, int64_t* launches, double* total_ms, double* total_bytes) {
    return me_batch_timing_read_kind(b, 0, launches, total_ms, total_bytes);
}

const char* me_batch_last_error(const me_batch* b) {
    return b ? b->err.c_str() : g_init_error.c_str();
}

me_status me_batch_destroy(me_batch* b) {
    if (!b) return ME_OK;
    hipStreamSynchronize(b->stream);
    for (hipStream_t w : b->workers) hipStreamSynchronize(w);
    batch_release(b);
    return ME_OK;
}

// ============================================================ toy model
// The two-band model of sec. 6 (eq. L_toy); kernels in toy.hip.

me_status me_toy_run(const me_toy_params* p, int32_t scheme, int32_t n_traj, int32_t n_samples, double t_total,
                     int32_t max_substeps, const double* mu, const int32_t* substeps, const int32_t* window,
                     double* samples, double* d_R, double* d_F, void* stream) {
    if (!p) { g_init_error = "p is NULL"; return ME_EINVAL; }
    auto pos_fin = [](double x) { return x > 0.0 && std::isfinite(x); };
    if (!pos_fin(p->M_R) || !pos_fin(p->M_G) || !pos_fin(p->K_R) || !std::isfinite(p->K_G) ||
        !std::isfinite(p->R0) || !std::isfinite(p->G0)) {
        g_init_error = "toy parameters: masses and K_R must be positive, all finite";
        return ME_EINVAL;
    }
    if (scheme != 0 && scheme != 1) { g_init_error = "scheme must be 0 (Ehrenfest) or 1 (CP)"; return ME_EINVAL; }
    if (!pos_fin(t_total)) { g_init_error = "t_total must be positive"; return ME_EINVAL; }
    if (n_traj < 0 || n_samples < 1 || max_substeps < 1) {
        g_init_error = "need n_traj >= 0, n_samples >= 1, max_substeps >= 1";
        return ME_EINVAL;
    }
    if ((int64_t)n_samples * max_substeps > (int64_t(1) << 24)) {
        g_init_error = "n_samples * max_substeps exceeds 2^24 steps per trajectory";
        return ME_EINVAL;
    }
    if (n_traj == 0) return ME_OK;
    if (!mu || !substeps || !window || !d_R || !d_F) { g_init_error = "NULL device array"; return ME_EINVAL; }
    ToyArgs a{p->R0, p->M_R, p->K_R, p->G0, p->M_G, p->K_G, t_total, n_traj, n_samples, max_substeps,
              mu, substeps, window, samples, d_R, d_F};
    const hipError_t e = launch_toy(a, scheme == 1, (hipStream_t)stream);
    if (e != hipSuccess) { g_init_error = hipGetErrorString(e); return ME_EDEVICE; }
    return ME_OK;
}

me_status me_toy_distance(int32_t n_traj, int32_t n_samples, int32_t n_vars, const double* samples,
                          const int32_t* ref, double* dist, void* stream) {
    if (n_traj < 0 || n_samples < 1 || n_vars < 1 || n_vars > 8) {
        g_init_error = "need n_traj >= 0, n_samples >= 1, 1 <= n_vars <= 8";
        return ME_EINVAL;
    }
    if (n_traj == 0) return ME_OK;
    if (!samples || !ref || !dist) { g_init_error = "NULL device array"; return ME_EINVAL; }
    const hipError_t e = launch_toy_distance(n_traj, n_samples, n_vars, samples, ref, dist, (hipStream_t)stream);
    if (e != hipSuccess) { g_init_error = hipGetErrorString(e); return ME_EDEVICE; }
    return ME_OK;
}

}  // extern "C"

/*
 * modehr.h -- C ABI of the MI355X (gfx950) modified-Ehrenfest propagation
 * library.
 *
 * The library advances a set of doubly occupied Kohn-Sham orbitals and the
 * ions of one periodic system by the modified Ehrenfest equations of motion
 * of Andrade et al., arXiv:0812.2801, eq. (new_EoM):
 *     i mu d(phi_A)/dt = H phi_A,     M_J d^2 R_J/dt^2 = -grad_J E_KS,
 * with H = -1/2 Lap (8th-order finite differences on a periodic grid)
 *        + v_eff (local ionic + Hartree + Slater exchange [+ field])
 *        + sum_J E_KB |p_J><p_J|  (Gaussian s-channel Kleinman-Bylander).
 * One step (sec. 5.1) is velocity Verlet for the ions around the AETRS
 * propagator of eq. (aetrs), each exponential a fourth-order Taylor
 * polynomial with electronic step tau = dt/(2 mu) (eq. transf), followed by
 * the density of eq. (density) and the forces -grad_R E_KS at fixed orbitals.
 * The problem statement follows sec. 5.1: given phi(0) and R(0), compute
 * phi(t) and R(t).
 *
 * Conventions
 *   - Grid: n[0] x n[1] x n[2] points (x, y, z), spacing h, periodic cube of
 *     side L = n h, point (ix,iy,iz) at r = h (ix,iy,iz).  A grid function is
 *     stored with x fastest: offset = (iz*n[1] + iy)*n[0] + ix.
 *   - Orbitals: complex, interleaved (re, im).  Precision ME_F64 uses
 *     complex128 (double2); ME_F32 and ME_F32_BF16X3 use complex64 (float2).
 *     A set of orbitals is [n_orb][orb_stride] complex elements; the first
 *     N = n[0]*n[1]*n[2] elements of each row are the grid function.
 *   - Inner product: h^3 sum conj(a) b.  Orbitals handed to me_set_state are
 *     expected to be orthonormal under it (the library does not enforce it).
 *   - Atomic units (bohr, hartree, electron masses, au of time).
 *
 * Memory ownership
 *   - Host arrays in me_params are copied during me_init_system.
 *   - All device memory is owned by the caller: the workspace (size from
 *     me_workspace_size) and every device pointer argument.  The library
 *     never allocates device memory for system state; rocFFT plans may hold
 *     their own small twiddle tables.
 *   - The handle is owned by the library and released by me_destroy.
 *
 * Streams and errors
 *   - Every call that launches work enqueues it on the stream given to
 *     me_init_system (a hipStream_t passed as void*; NULL = default stream)
 *     and returns without waiting, unless its comment says it synchronises.
 *     Inside an MD step a single system also uses a second stream of its
 *     own (created by me_init_system, default priority, released by
 *     me_destroy) for work the first exponential does not wait for; it is
 *     forked from and joined back into the caller's stream by events within
 *     the step, so when me_propagate_step returns, all of the step's work is
 *     ordered before whatever the caller enqueues next on its stream.
 *   - Every call returns an me_status.  Arguments are validated before any
 *     launch; an invalid argument returns ME_EINVAL and changes nothing.
 *     Asynchronous device errors surface at the next synchronising call.
 *     No call aborts, exits or throws; me_last_error gives the text.
 *   - A handle is not thread-safe: use one handle per host thread/stream.
 */
#ifndef MODEHR_H
#define MODEHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ME_OK = 0,
    ME_EINVAL = 1,        /* null pointer, bad size, sphere does not fit, ... */
    ME_ENOMEM = 2,        /* workspace smaller than me_workspace_size */
    ME_EDEVICE = 3,       /* HIP or rocFFT error (text in me_last_error) */
    ME_ESTATE = 4,        /* call before me_set_state, or wrong mode */
    ME_EUNSTABLE = 5,     /* an orbital norm grew or became non-finite */
    ME_EUNSUPPORTED = 6   /* valid request the library does not support (e.g. a grid
                             point inside more than 8 projector spheres) */
} me_status;

typedef enum {
    ME_F64 = 0,           /* complex128 orbitals, FP64 everywhere */
    ME_F32 = 1,           /* complex64 orbitals and FP32 stencil/Taylor */
    ME_F32_BF16X3 = 2     /* ME_F32 with the projector contraction as split-bf16 MFMA */
} me_precision;

typedef struct me_system me_system;

/* Parameters of one system.  Host pointers; copied by me_init_system. */
typedef struct {
    int32_t n[3];          /* grid points along x, y, z (each in [8, 1024]; cubic) */
    double h;              /* grid spacing, bohr (> 0) */
    int32_t n_ions;        /* >= 0 */
    const double* pos;     /* [n_ions][3] initial positions, bohr */
    const double* vel;     /* [n_ions][3] initial velocities, or NULL for zero */
    const double* mass;    /* [n_ions] masses, electron masses (> 0) */
    const double* zval;    /* [n_ions] ionic charges */
    double loc_a;          /* V_loc = -Z erf(r/loc_a)/r, loc_a > 0 */
    double kb_sigma;       /* projector width sigma (> 0) */
    double kb_rcut;        /* projector cutoff radius; 2*kb_rcut < L along every axis */
    double kb_energy;      /* E_KB, hartree */
    int32_t n_orb;         /* number of orbitals (>= 1) */
    double occ;            /* occupation per orbital (2 for closed shell) */
    double mu;             /* the electronic time-scale parameter (> 0) */
    double dt;             /* ionic time step, au (!= 0) */
    int32_t taylor_order;  /* order of the Taylor exponential (1..8; 4 in the method) */
    int32_t precision;     /* me_precision */
    int32_t freeze_ions;   /* nonzero: ions do not move (forces still computed) */
    int32_t enable_adjoint;/* nonzero: reserve the adjoint buffers (requires freeze_ions) */
    int32_t nl_force_form; /* nonlocal force: 0 the analytic derivative of the projector,
                              1 the wave-function-gradient form (footnote of sec. 5.1):
                              d c_JA / d R_J as h^3 sum p_J grad psi_A with the 8th-order
                              finite-difference gradient */
    int32_t etrs_iterations; /* 0: AETRS (eq. aetrs: H(t+dt) with the extrapolated v_Hxc);
                                k in 1..8: ETRS, the second exponential redone k times from
                                the half-step orbitals with v_Hxc of the latest density
                                (needs one more orbital buffer; not with batches or the
                                adjoint) */
    double finite_radius;    /* 0: periodic cube.  > 0: finite box (sec. 5, the molecular
                                runs): the grid points within this radius of an ion at
                                its initial position; orbitals are zero outside (H acts as
                                P H P), the Hartree potential is that of free space (the
                                charge convolved with 1/|r|, cell average 2.380077/h at
                                r = 0, by FFTs on the doubled grid), the local ionic
                                potential and the ion-ion energy have no periodic images.
                                The box must keep 4 grid points from every face of the
                                cube; no external field (ctrl must be 0), no batches, no
                                adjoint.  Needs the doubled-grid FFT buffers. */
} me_params;

/* Diagnostics of the current state.  Energies in hartree. */
typedef struct {
    double e_kinetic;      /* f sum_A h^3 Re<psi_A|T psi_A> */
    double e_local;        /* h^3 sum rho V_loc (incl. any static potential) */
    double e_hartree;
    double e_xc;
    double e_nonlocal;     /* f E_KB sum |c_JA|^2 */
    double e_ion;          /* Ewald ion-ion energy */
    double e_ks;           /* sum of the six above */
    double e_ion_kinetic;  /* sum 1/2 M V^2 */
    double e_total;        /* e_ks + e_ion_kinetic: the conserved energy of eq. (E_new) */
    double max_norm_dev;   /* max_A |h^3 sum |psi_A|^2 - 1| */
    double max_force;      /* max_J |F_J| */
    double charge;         /* h^3 sum rho */
    int64_t step;          /* steps taken since me_set_state */
    double e_fictitious;   /* me_cp_step only: f mu_cp sum_A <psi_A'|psi_A'> (included in
                              e_total); 0 for the other steps */
    double cp_constraint_residual;  /* me_cp_step only: max |A + B^H X + X B + X^2 - I| left
                                       by the orthonormality constraint solve */
} me_step_report;

/* Bytes of device workspace me_init_system needs for these parameters.
 * Pure host computation. */
me_status me_workspace_size(const me_params* p, size_t* bytes);

/* Create a system: the periodic real-space grid (sec. 5), the local ionic
 * potential of eq. (ionicpotential) and the Gaussian Kleinman-Bylander
 * projectors at R(0), i.e. every part of H of eq. (new_EoM(a)) that does not
 * depend on the orbitals (sec. 5.1: given phi(0) and R(0), compute phi(t) and
 * R(t); the orbitals follow with me_set_state).
 * workspace: caller-owned device memory of at least
 * me_workspace_size bytes, 256-byte aligned, untouched by the caller until
 * me_destroy.  stream: hipStream_t (as void*) all work is enqueued on (see
 * "Streams and errors" for the step's internal second stream).
 * Validates p (ME_EINVAL), checks ws_bytes (ME_ENOMEM), uploads the ion data
 * and builds FFT plans.  No orbital state yet: call me_set_state. */
me_status me_init_system(const me_params* p, void* workspace, size_t ws_bytes,
                         void* stream, me_system** out);

/* Release the handle (not the caller's device memory).  NULL is allowed. */
me_status me_destroy(me_system* sys);

/* Wait for all work enqueued by this handle.  Returns ME_EDEVICE on a
 * pending device error. */
me_status me_sync(me_system* sys);

/* Load orbitals psi_dev ([n_orb][orb_stride] complex of the handle's
 * precision, device) as the state at t = 0 (eq. Ehr_ic), then compute the
 * density, v_eff and the forces F(0).  orb_stride >= N.  Resets the step
 * counter and the potential history. */
me_status me_set_state(me_system* sys, const void* psi_dev, int64_t orb_stride);

/* Copy the current orbitals to psi_dev ([n_orb][orb_stride], device). */
me_status me_get_state(me_system* sys, void* psi_dev, int64_t orb_stride);

/* hpsi_out = H psi_in for n_orb orbitals of the handle's precision, with the
 * current Hamiltonian H(t) (eq. new_EoM(a): kinetic + v_eff + nonlocal).
 * On a finite box the output is zero outside the box (P H psi_in; input
 * values outside the box enter through the stencil of points inside it).
 * Input and output must not overlap.  n_orb >= 1, orb_stride >= N. */
me_status me_apply_H(me_system* sys, const void* psi_in_dev, void* hpsi_out_dev,
                     int32_t n_orb, int64_t orb_stride);

/* One molecular-dynamics step (sec. 5.1): R(t+dt) by velocity Verlet, the
 * AETRS propagator of eq. (aetrs) with Taylor exponentials of step
 * tau = dt/(2 mu), the density (eq. density), Hartree/exchange, forces and
 * velocities.  ctrl: host pointer to the amplitude eps of a uniform field
 * adding eps * (x - L/2) to v_eff in both exponentials of this step, or NULL
 * for no field.  rep: host, nullable; when given, the step's diagnostics are
 * computed and the call synchronises.  Returns ME_EUNSTABLE (after the step)
 * if an orbital norm exceeded 1 + 1e-6 or became non-finite; the check is
 * made at the next synchronising call when rep is NULL. */
me_status me_propagate_step(me_system* sys, const double* ctrl, me_step_report* rep);

/* Diagnostics of the current state (synchronises). */
me_status me_report(me_system* sys, me_step_report* rep);

/* The electronic density of eq. (density), rho = f sum_A |psi_A|^2 with
 * f = occ (2 for the closed shell of the paper), of the current state:
 * rho_dev[N], FP64, device, caller-owned. */
me_status me_density(me_system* sys, double* rho_dev);

/* The ionic forces of eq. (new_EoM(b)), F_J = -dE_KS/dR_J at fixed orbitals
 * (eq. ionicforces read as the derivative of the discrete energy: local part
 * by the G-space sum, nonlocal part from the projector coefficients, ion-ion
 * part by Ewald), at the current state: f_host[3*n_ions], FP64, host,
 * caller-owned (synchronises). */
me_status me_forces(me_system* sys, double* f_host);

/* Current ion positions and velocities, host, [n_ions][3] each; either may be
 * NULL (synchronises). */
me_status me_get_ions(me_system* sys, double* pos_host, double* vel_host);

/* Components of the current potential, FP64, device [N]:
 * which = 0: V_loc (incl. static potential), 1: v_Hxc (newest history level),
 * 2: v_eff(t) as used by the next step's first exponential (without field). */
me_status me_get_potential(me_system* sys, int32_t which, double* v_dev);

/* Add a static local potential dv_dev[N] (FP64, device; copied) to V_loc, or
 * clear it with NULL.  Takes effect for the next me_set_state. */
me_status me_set_static_potential(me_system* sys, const double* dv_dev);

/* ---------------------------------------------------------------- adjoint
 * Discrete adjoint of an AETRS trajectory with frozen ions (an extension; the
 * paper gives no gradient method).  The controls are a per-step uniform-field
 * amplitude eps_n, entering v_eff as eps_n (x - L/2) in both exponentials of
 * step n, and a static local potential dV; the objective J depends on the
 * final density (by default the dipole J = h^3 sum (x - L/2) rho(T)).
 * Reverse mode: me_adjoint_begin at the final time, then for n = N-1 .. 0
 * load the state at the start of step n (me_load_checkpoint, from the
 * caller's checkpoints and recomputation) and call me_adjoint_step.  Each
 * call recomputes step n keeping its Horner stages, reverses them
 * (ubar_k = conj(c_k) H ubar_{k-1}, H Hermitian) together with the density
 * and the Hartree-exchange potential (including the extrapolated history),
 * and accumulates dJ/d(dV).  Requires enable_adjoint (and freeze_ions). */

/* Bytes of one checkpoint: orbitals, v_Hxc history, ions, step counter. */
me_status me_checkpoint_size(const me_system* sys, size_t* bytes);
/* Copy the current state into buf_dev (device, me_checkpoint_size bytes). */
me_status me_save_checkpoint(me_system* sys, void* buf_dev);
/* Make the state saved in buf_dev current (rebuilds V_loc and the projector
 * tables at its positions; synchronises).  ME_EINVAL if it belongs to a
 * system of another shape. */
me_status me_load_checkpoint(me_system* sys, const void* buf_dev);
/* Static potential from an m^3 periodic coarse grid (device, FP64) by
 * trilinear interpolation (n divisible by m), or cleared with NULL. */
me_status me_set_static_potential_coarse(me_system* sys, const double* coarse_dev, int32_t m);
/* d_host[0] = h^3 sum (x - L/2) rho of the current density (synchronises). */
me_status me_dipole(me_system* sys, double* d_host);
/* Start a reverse sweep at the final time with rhobar_dev = dJ/drho(T)
 * (device [N] FP64), or NULL for the dipole objective. */
me_status me_adjoint_begin(me_system* sys, const double* rhobar_dev);
/* Reverse the step whose starting state is current; ctrl_n: its field
 * amplitude; g_ctrl_n (host) receives dJ/d eps_n (synchronises). */
me_status me_adjoint_step(me_system* sys, double ctrl_n, double* g_ctrl_n);
/* dJ/d(dV) accumulated so far: on the grid (g_fine_dev [N]) and/or by the
 * transpose of the trilinear interpolation on an m^3 grid (g_coarse_dev). */
me_status me_adjoint_grad_v(me_system* sys, double* g_fine_dev, double* g_coarse_dev, int32_t m);

/* ------------------------------------------------- no device allocation
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The dipole
 * of me_dipole, d = h^3 sum_i (h*ix_i - L/2) rho_i with L = n[0] h and ix_i
 * the x index of point i, of a caller's density rho_dev[n[0]*n[1]*n[2]]
 * (FP64, device, x fastest; caller-owned), written to d_dev[0] (device,
 * caller-owned) on `stream` (a hipStream_t of the current device, as void*;
 * NULL = default stream).  Asynchronous: no synchronisation, no allocation.
 * The per-workgroup partial sums (one per 256 points) live in a fixed array
 * of ME_NOALLOC_MAX_PARTS doubles (2 MiB) that the library holds on every GPU
 * it runs on until the process ends; its address is taken on the first call
 * on each device.  The sum runs in the fixed order of me_dipole, so both
 * give the same bits for the same density.  All calls on one GPU share the
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race.  Errors: ME_EINVAL for NULL pointers, a size below 1, h <= 0 or more
 * than 256 * ME_NOALLOC_MAX_PARTS points (nothing launched); ME_EDEVICE if
 * the array's address cannot be taken or the launch fails.  The text is in
 * me_last_error(NULL). */
#define ME_NOALLOC_MAX_PARTS 262144
me_status me_dipole_noalloc(const double* rho_dev, const int32_t n[3], double h, double* d_dev,
                            void* stream);

/* ------------------------------------------------------- Car-Parrinello
 * The comparison scheme of sec. 3 (eq. L_CP, eq. EoM_CP): orbitals with a
 * fictitious mass mu_cp and orthonormality kept by Lagrange multipliers,
 * integrated by RATTLE / velocity Verlet (sec. 5, the CP implementation):
 *   mu_cp psi_A'' = -H psi_A + sum_B psi_B Lambda_BA,  M R'' = -grad E_KS,
 * conserving f mu_cp sum_A <psi_A'|psi_A'> + E_KS + sum M V^2 / 2.  Each step
 * costs one H psi and five O(N_W^2 N_C) complex GEMMs (overlaps, constraint
 * rotations) on rocBLAS, against eight H psi for me_propagate_step.  The
 * rocBLAS handle is created by me_cp_begin and allocates its own device
 * workspace; everything else lives in the system's workspace.
 *
 * me_cp_begin: start from the current state (me_set_state or a step) with
 * zero orbital velocities; mu_cp > 0; dt is the CP time step (ions and
 * orbitals; the params' dt is not used).  Computes H psi (asynchronous).
 * me_cp_step: one step (ions, orbitals, velocities).  ME_ESTATE unless
 * me_cp_begin ran after the last state change (me_set_state,
 * me_load_checkpoint, me_propagate_step, batch steps, adjoint steps and a
 * new static potential all end the CP run).  rep (nullable) as for
 * me_propagate_step, plus e_fictitious and cp_constraint_residual; the norm
 * deviation is not computed (the constraint holds it to the residual). */
me_status me_cp_begin(me_system* sys, double mu_cp, double dt);
me_status me_cp_step(me_system* sys, me_step_report* rep);

/* Per-kernel timing.  me_timing_enable(sys, 1) brackets every launch of the
 * Horner-stage stencil kernel with HIP events on the handle's stream;
 * me_timing_read synchronises and returns the number of timed launches,
 * their summed duration in milliseconds and the algorithmic bytes they moved
 * (3 complex streams per orbital point, 2 for the first stage, plus v_eff).
 * me_timing_enable(sys, 0) stops and clears. */
me_status me_timing_enable(me_system* sys, int32_t enable);
me_status me_timing_read(me_system* sys, int64_t* launches, double* total_ms,
                         double* total_bytes);
/* The same for one kind of Horner stage: streams = 2 the first stage of each
 * exponential (reads u = psi, writes the stage), 3 the others (read u and
 * psi, write the stage), 0 all of them (= me_timing_read). */
me_status me_timing_read_kind(me_system* sys, int32_t streams, int64_t* launches, double* total_ms,
                              double* total_bytes);

/* Text of the last error on this handle ("" if none).  NULL sys gives the
 * last error of a failed me_init_system on this thread. */
const char* me_last_error(const me_system* sys);
const char* me_strerror(me_status s);

/* ------------------------------------------------------------------ batches
 * Many independent systems (uneven grids and orbital counts) advanced
 * together.  Each step is the step of me_propagate_step (sec. 5.1, no
 * control field) for every system; every orbital of every system is
 * independent inside the two Taylor exponentials of eq. (aetrs), so each of
 * their Horner stages runs as ONE stencil launch over all systems.  Its
 * work items are (system, orbital, x-tile, y-tile, z-slab); each of the 8
 * XCDs takes an even, contiguous share of every system's items, either one
 * item per workgroup (the default) or pulled from a per-XCD device queue by
 * a persistent grid (see me_batch_tuning).  A system whose whole x-rows do not
 * fit the workgroup runs in x-tiles of 64 points (x-halo in LDS).  All
 * systems share one stream and must share the precision and the Taylor
 * order; at most 32 systems.  The adjoint is not available on batched
 * systems.
 */
typedef struct me_batch me_batch;

/* Launch shape of the batched stencil. */
typedef struct {
    int32_t block;        /* threads per workgroup: multiple of 64 in [64, 1024];
                             each system's tile is floor(block / n_x) whole rows,
                             or floor(block / 64) rows of 64-point x-tiles when
                             8 n_x > 2 block */
    int32_t wg_per_cu;    /* 0: one work item per workgroup (grid = the items, each
                             XCD taking an even share of every system's items;
                             the default); 1-4: a persistent launch of this many
                             resident workgroups per compute unit (grid = this x
                             CUs) pulling items from per-XCD queues */
    int32_t zdiv;         /* z-slabs per orbital column: 1, 2 or 4 */
    double stage_ms;      /* autotuner: measured time of one Horner stage over the
                             whole batch (ms); ignored by me_batch_set_tuning */
} me_batch_tuning;

/* Workspace of a batch: the systems' workspaces (me_workspace_size of each,
 * 256-byte aligned, in order) plus a small block of work-queue counters. */
me_status me_batch_workspace_size(const me_params* ps, int32_t n_sys, size_t* bytes);

/* Creates n_sys systems from ps[0..n_sys-1] (host array; each as in
 * me_init_system) on slices of one caller-owned device workspace, all on
 * `stream`, and picks an untuned launch shape.  Released by
 * me_batch_destroy, which also destroys the systems. */
me_status me_init_batch(const me_params* ps, int32_t n_sys, void* workspace_dev, size_t ws_bytes,
                        void* stream, me_batch** out);

/* The handle of system i (0-based, caller order) for me_set_state,
 * me_get_state, me_report, me_density, me_forces, ...  Owned by the batch. */
me_status me_batch_system(me_batch* b, int32_t i, me_system** out);

/* Sets or reads the launch shape.  ME_EINVAL if it does not fit a system
 * (the halo jobs of an x-tile, 8 (64 + rows), over 2 block; LDS over 64 KiB)
 * or wg_per_cu is negative or exceeds what is resident. */
me_status me_batch_set_tuning(me_batch* b, const me_batch_tuning* t);
me_status me_batch_get_tuning(const me_batch* b, me_batch_tuning* t);

/* Autotuner: times three-stream Horner stages over the batch (on a copy of
 * the orbitals in the scratch buffers) for every launch shape
 * (block 256..1024, wg_per_cu 0..4, zdiv 1/2/4) that fits, keeps the
 * fastest, and returns it in *out (nullable).  With cache_path (nullable) a
 * JSON file keyed by precision, Taylor order and the systems' shapes is
 * consulted first and updated after a search.  Needs the state of every
 * system; overwrites their scratch orbitals only.  Synchronises. */
me_status me_batch_autotune(me_batch* b, const char* cache_path, me_batch_tuning* out);

/* n_steps MD steps of every system.  With use_graph != 0 runs of 6 steps
 * are replayed from one captured hipGraph (captured on first use, and again
 * when a system's state changed phase); the first steps after me_set_state
 * and any remainder run eagerly.  Synchronises at the end and returns
 * ME_EUNSTABLE / ME_EUNSUPPORTED if a system's last step flagged it. */
me_status me_propagate_batch(me_batch* b, int32_t n_steps, int32_t use_graph);

/* Event timing of the persistent stencil launches of eager steps (graph
 * replays and the autotuner are not timed), as me_timing_enable /
 * me_timing_read. */
me_status me_batch_timing_enable(me_batch* b, int32_t enable);
me_status me_batch_timing_read(me_batch* b, int64_t* launches, double* total_ms, double* total_bytes);
/* The same for one kind of Horner stage (streams = 2, 3 or 0), as
 * me_timing_read_kind. */
me_status me_batch_timing_read_kind(me_batch* b, int32_t streams, int64_t* launches, double* total_ms,
                                    double* total_bytes);

/* Text of the last error of a batch call; NULL b gives the last error of a
 * failed me_init_batch on this thread. */
const char* me_batch_last_error(const me_batch* b);
me_status me_batch_destroy(me_batch* b);

/* ------------------------------------------------------- two-band toy model
 * The model of sec. 6 (eq. L_toy): electronic angles theta_1, theta_2, bond
 * length R, gap coordinate G.  Equations of motion (Euler-Lagrange equations
 * of eq. L_toy; the angles are first order in the modified Ehrenfest form):
 *   mu theta_1' = (G/2) sin(theta_2 - R),  mu theta_2' = -(G/2) sin(theta_1 - R),
 *   M_R R'' = -K_R (R - R_0) + (G/2)[sin(theta_1 - R) + sin(theta_2 - R)],
 *   M_G G'' = -K_G (G - G_0) + (1/2)[cos(theta_1 - R) + cos(theta_2 - R)];
 * CP instead: mu_CP theta_i'' = -(G/2) sin(theta_i - R).  Start (sec. 6): R
 * and G 10 % above R_0 and G_0 at rest, theta_i = R(0), CP angles at rest.
 * The gsBO reference (mu = 0, theta_i = R) is R_BO(t) = R_0 (1 + 0.1 cos(w t)),
 * w = sqrt(K_R / M_R).  Atomic units; FP64 throughout. */
typedef struct {
    double R0, M_R, K_R;  /* bond: equilibrium length, mass, force constant */
    double G0, M_G, K_G;  /* gap coordinate: the same three */
} me_toy_params;

/* Integrates n_traj independent trajectories over [0, t_total] by classical
 * RK4, one per work-item (asynchronous on `stream`).  scheme 0: modified
 * Ehrenfest, 1: CP.  Device arrays of n_traj: mu (mu or mu_CP, > 0),
 * substeps (RK4 steps per sample, 1..max_substeps; dt = t_total /
 * (n_samples * substeps)), window (samples per force average, >= 1); a
 * trajectory whose entries break these bounds gets NaN outputs and is not
 * run.  Outputs (device): samples (nullable) [n_samples + 1][NV][n_traj],
 * the whole state at t_j = j t_total / n_samples, trajectory fastest: NV = 6,
 * (theta_1, theta_2, R, R', G, G') for Ehrenfest; NV = 8, (theta_1, theta_2,
 * theta_1', theta_2', R, R', G, G') for CP; d_R[n_traj] = 100 / (0.2 R_0) * rms_j (R(t_j) - R_BO(t_j)) over
 * j = 1..n_samples; d_F[n_traj] = 100 / (0.2 K_R R_0) * rms over the
 * complete windows of (force on R averaged over the window by the trapezoid
 * rule on the run's own steps - gsBO force averaged over the window).
 * ME_EINVAL for non-positive masses or K_R, t_total <= 0, n_samples < 1,
 * max_substeps < 1, n_samples * max_substeps > 2^24 (the bound on the run
 * time of one work-item), NULL outputs; n_traj = 0 does nothing. */
me_status me_toy_run(const me_toy_params* p, int32_t scheme, int32_t n_traj, int32_t n_samples,
                     double t_total, int32_t max_substeps, const double* mu_dev,
                     const int32_t* substeps_dev, const int32_t* window_dev, double* samples_dev,
                     double* d_R_dev, double* d_F_dev, void* stream);

/* Distance of each trajectory from a reference (the Delta t_max criterion of
 * sec. 6, over all the dynamical variables): dist[i] = max over the n_vars
 * state variables c of
 * 100 * rms_j (x_c[i](t_j) - x_c[ref[i]](t_j)) / (max_j - min_j of x_c[ref[i]]),
 * j = 0..n_samples, over samples laid out as me_toy_run writes them (n_vars
 * = NV of the scheme).  ref (device, n_traj entries in [0, n_traj); an entry
 * outside gives NaN).  ME_EINVAL for NULL arrays, n_samples < 1 or n_vars
 * outside [1, 8]. */
me_status me_toy_distance(int32_t n_traj, int32_t n_samples, int32_t n_vars, const double* samples_dev,
                          const int32_t* ref_dev, double* dist_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MODEHR_H */

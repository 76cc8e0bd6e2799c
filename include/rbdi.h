/*
 * rbdi.h -- C ABI of librbdi, the MI355X (gfx950) implementation of the
 * Eulerian finite-volume step of the diffuse-interface rigid-body method of
 * Wallis, Barton & Nikiforakis (arXiv 2111.11806).
 *
 * One time step (rbdi_step) is, in this order:
 *   1. interface seeding of rigid cells (Sec. 3.2, the seeding routine; once
 *      per step, before the hyperbolic update);
 *   2. three SSP-RK3 stages (Sec. 3.1, third-order Runge-Kutta), each one
 *      evaluation of the unsplit semi-discrete operator D (Sec. 3.1, spatial
 *      operator) built from direction sweeps: per-cell closure (Sec. 2.2),
 *      MUSCL-BVD-THINC reconstruction of the primitive variables, r
 *      included (Sec. 3.1), HLLC / HLLC-LM fluxes (Sec. 3.1, Sec. 4.3), the
 *      upwind r flux and the non-conservative terms (Sec. 3.1), and the
 *      conservative update; thermodynamic fields of rigid (r > 0.5) cells
 *      are not updated (Sec. 3.1).
 *
 * Conventions shared by every entry point:
 *  - Return value: RBDI_OK (0) or a negative rbdi_error. The message of the
 *    last failure on the calling thread is rbdi_last_error().
 *  - Arrays of cell data are structure-of-arrays over the INTERIOR cells:
 *    [nfields][nz][ny][nx], x fastest, FP64 at the API in every precision.
 *  - Primitive field order: phi_l (N-1), rho_l (N), u (dim), p,
 *    [Vbar (9, row major), eps_p], r. Conserved field order: phi_l rho_l (N),
 *    rho u (dim), rho E, phi_l (N-1), [Vbar (9), phi_s rho_s eps_p], r.
 *    Bracketed fields exist only when desc.solid = 1.
 *  - Pointers marked "host or device" are read on the device when the
 *    on_device argument is nonzero (device pointers of the handle's GPU),
 *    otherwise they are host pointers. The library never keeps or frees
 *    caller memory.
 *  - Every GPU operation is enqueued on the handle's stream (rbdi_set_stream;
 *    default: the null stream). Entry points that return device results to
 *    the host (compute_dt, status, rigid_force, conserved_totals, get_state*)
 *    synchronise that stream; rbdi_step and rbdi_advance do not.
 *  - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef RBDI_H
#define RBDI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBDI_API __attribute__((visibility("default")))

typedef struct rbdi_handle rbdi_handle;
typedef struct rbdi_batch rbdi_batch;
typedef struct rbdi_mlp rbdi_mlp;

typedef enum {
  RBDI_OK = 0,
  RBDI_ERR_BAD_ARG = -1,     /* invalid argument; nothing was enqueued */
  RBDI_ERR_OOM = -2,         /* device allocation failed */
  RBDI_ERR_HIP = -3,         /* a HIP runtime call failed */
  RBDI_ERR_NONPHYSICAL = -4, /* a cell left the admissible set (rbdi_status) */
  RBDI_ERR_NOT_READY = -5,   /* call order violated (e.g. step before state) */
  RBDI_ERR_UNSUPPORTED = -6  /* the library has no kernel for the combination */
} rbdi_error;

enum { RBDI_EOS_IDEAL = 0, RBDI_EOS_STIFFENED = 1, RBDI_EOS_ROMENSKII = 2 };
enum { RBDI_BC_TRANSMISSIVE = 0, RBDI_BC_REFLECTIVE = 1, RBDI_BC_DIRICHLET = 2, RBDI_BC_PERIODIC = 3 };
enum { RBDI_RECON_MUSCL = 0, RBDI_RECON_BVD_THINC = 1 };
enum { RBDI_RIEMANN_HLLC = 0, RBDI_RIEMANN_HLLC_LM = 1 };
enum { RBDI_SEED_ORIGINAL = 0, RBDI_SEED_RIEMANN = 1, RBDI_SEED_NONE = 2 };
enum { RBDI_PROBE_STEPOUT = 0, RBDI_PROBE_FIXED = 1 };
enum { RBDI_NORMAL_YOUNGS = 0, RBDI_NORMAL_ELVIRA = 1 };
enum { RBDI_FP64 = 0, RBDI_FP32 = 1 };

/* Grid, system and scheme of one instance.
 * dim 1..3; n[d] interior cells (n[d] = 1 for d >= dim); dx[d] cell size;
 * origin: coordinates of the lower domain corner.
 * nmat 1..2 materials; solid = 1 adds the stretch tensor Vbar and the plastic
 * strain of the first Romenskii material (elastoplastic system, Sec. 2.1.1).
 * bc[6]: x-lo, x-hi, y-lo, y-hi, z-lo, z-hi, one of RBDI_BC_*.
 * recon: RBDI_RECON_*; riemann: RBDI_RIEMANN_*; seed: RBDI_SEED_*;
 * probe: RBDI_PROBE_*; plastic: apply the plastic return (solid only);
 * thinc_beta: THINC steepness; lm_mach: HLLC-LM Mach limit;
 * precision: RBDI_FP64, or RBDI_FP32 (flux and reconstruction in FP32; the
 * mixture-pressure inversion, dt, force/torque and totals in FP64).
 * normal: RBDI_NORMAL_* (Sec. 3.3), the rigid-body normal used by seeding:
 * Youngs' central differences, or ELVIRA (dim = 2 only; BAD_ARG otherwise):
 * the best of six candidate lines from backward/central/forward differences
 * of the 3x3 column and row sums of r, judged by the volume fractions each
 * line gives the nine cells; Youngs where the centre fraction is 0 or 1 or
 * no candidate exists. Always computed in FP64. */
typedef struct {
  int dim;
  int n[3];
  double dx[3];
  double origin[3];
  int nmat;
  int solid;
  int bc[6];
  int recon;
  int riemann;
  int seed;
  int probe;
  int plastic;
  double thinc_beta;
  double lm_mach;
  int precision;
  int normal;
} rbdi_desc;

/* Equation of state of one material (Sec. 2.1.3 and the Mie-Gruneisen form of
 * Sec. 2.1.2). IDEAL: gamma. STIFFENED: gamma, pinf (e_ref = pinf/rho,
 * p_ref = -pinf). ROMENSKII: rho0, K0, G0, alpha, beta, Gamma0 (Table 1) and
 * the perfect-plasticity yield stress sigma_y (0 = elastic). SI or
 * non-dimensional units, consistently. */
typedef struct {
  int kind;
  double gamma, pinf;
  double rho0, K0, G0, alpha, beta, Gamma0, sigma_y;
} rbdi_eos;

/* Counters of the device-side path, read by rbdi_status. */
typedef struct {
  long long steps;        /* completed steps */
  double t;               /* simulated time */
  double last_dt;         /* dt of the last step */
  long long band_cells;   /* rigid cells with a nonzero normal (last band build) */
  long long seeded;       /* cells seeded (cumulative over steps) */
  long long probe_fail;   /* of band_cells, those without a valid probe (last band build) */
  int nonphysical;        /* 1 once a non-admissible updated cell was found: after
                             every stage, a non-positive phasic mass or a
                             non-finite energy; at the end of every step, in
                             non-rigid cells, also a volume fraction outside
                             [0,1], a non-positive mixture sound speed
                             squared or a non-finite signal speed */
  long long first_bad;    /* linear interior index of the first such cell, or -1 */
  long long surr_net;     /* plastic-return evaluations closed by the surrogate (cumulative;
                             cells that provably cannot yield skip the closure
                             and are not counted) */
  long long surr_exact;   /* ... closed by the exact closure: outside the envelope or flagged */
} rbdi_stats;

/* Create an instance on the current HIP device. Allocates every device buffer
 * the handle owns (three state copies, one accumulator of the direction
 * sweeps -- two in 3D -- plus band, reduction and staging scratch); *out
 * receives the handle, which rbdi_destroy releases. Errors: BAD_ARG (invalid
 * desc), OOM, HIP. */
RBDI_API int rbdi_create(const rbdi_desc* desc, rbdi_handle** out);

/* Release the handle and its device memory (synchronises its stream). */
RBDI_API int rbdi_destroy(rbdi_handle* h);

/* Number of primitive (= conserved) fields of the instance. */
RBDI_API int rbdi_nfields(const rbdi_handle* h);

/* Enqueue all further work on the given hipStream_t (passed as void*; NULL =
 * the null stream). The caller keeps the stream alive while it is set. */
RBDI_API int rbdi_set_stream(rbdi_handle* h, void* hip_stream);

/* Material l (0 <= l < nmat). Must precede rbdi_set_state_prim. BAD_ARG for
 * gamma <= 1, rho0 <= 0, K0 < 0, a solid kind without desc.solid, etc. */
RBDI_API int rbdi_set_material(rbdi_handle* h, int l, const rbdi_eos* eos);

/* Primitive state imposed on the ghost cells of a Dirichlet face (face 0..5),
 * host array of nfields values. */
RBDI_API int rbdi_set_bc_state(rbdi_handle* h, int face, const double* W);

/* Set the interior state from primitives W (host or device, FP64, SoA over
 * interior cells). Converted to conserved variables on the device. */
RBDI_API int rbdi_set_state_prim(rbdi_handle* h, const double* W, int on_device);

/* Read the interior state as primitives / conserved variables into W / U
 * (host or device, FP64). Synchronises the stream. */
RBDI_API int rbdi_get_state_prim(rbdi_handle* h, double* W, int on_device);
RBDI_API int rbdi_get_state_cons(rbdi_handle* h, double* U, int on_device);

/* Set the conserved interior state directly (host or device, FP64). */
RBDI_API int rbdi_set_state_cons(rbdi_handle* h, const double* U, int on_device);

/* Void-opening face modifier at solid-rigid faces (Sec. 3.2, end: applied
 * where the rigid fraction crosses 0.5 between the two cells of a face,
 * (0.5 - r_L)(0.5 - r_R) < 0, so that solids can collide with and separate
 * from rigid bodies). mode 0: off (the default); mode 1: on. At such a face
 * the material cell's face state meets its mirror image about the face
 * (normal velocity reflected about the rigid velocity, Vbar conjugated by the
 * reflection); where the normal traction on that contact is tensile, the
 * rigid side becomes the gap gas Wgap (host, FP64, nfields primitives in the
 * layout of rbdi_set_state_prim; its velocity and r are ignored: it moves with
 * the body's normal velocity), which then flows into the opening gap (the
 * paper defers the void model to other work; this reading fills the gap with
 * the surrounding gas). Elastoplastic systems only; Wgap may be NULL for
 * mode 0. BAD_ARG for another mode, a fluid system, a NULL or non-finite gap
 * state. */
RBDI_API int rbdi_set_face_modifier(rbdi_handle* h, int mode, const double* Wgap);

/* Rigid volume fraction from a signed distance sdf (host or device, FP64,
 * one value per interior cell, negative inside the body; union of bodies =
 * pointwise minimum): r = (1 - tanh(sdf / (width dx_min))) / 2 (Sec. 2.3
 * represents bodies by a scalar field r in [0,1] whose 0.5 contour is the
 * surface). The imposed rigid velocity is v_r(x) = v + omega x (x - center)
 * (Sec. 2.3); center moves with v after every step. */
RBDI_API int rbdi_set_rigid_sdf(rbdi_handle* h, const double* sdf, int on_device, double width,
                                const double v[3], const double omega[3], const double center[3]);

/* Replace the rigid motion (velocity, angular velocity, centre) by that of
 * a single body (every point moves with it). */
RBDI_API int rbdi_set_rigid_motion(rbdi_handle* h, const double v[3], const double omega[3],
                                   const double center[3]);

/* Several rigid bodies with their own motions in one instance (the paper's
 * extrusion test, Sec. 4.5: a moving piston and a static wedge in one r
 * field). r is set as before from the union's signed distance
 * (rbdi_set_rigid_sdf); this call replaces the motion by a table of nbody
 * (1..RBDI_MAX_BODIES) motions: v, omega, center (host, nbody x 3 each)
 * and, for bodies 1..nbody-1, an ownership box box_lo <= x < box_hi (host,
 * nbody x 3; row 0 ignored, may be NULL when nbody = 1). A point moves with
 * the first body k >= 1 whose box holds it, otherwise with body 0: the
 * rigid velocity v_k + omega_k x (x - c_k) (Sec. 2.3) of that body enters
 * the r flux, the seeding states and the CFL rate. Centres and boxes are
 * those of the current time and move with each body's velocity. A box must
 * hold its body's whole diffuse r profile (r below rounding at the box
 * faces). BAD_ARG for nbody out of range, non-finite motions or NaN box
 * bounds (infinite bounds are allowed). */
#define RBDI_MAX_BODIES 4
RBDI_API int rbdi_set_rigid_bodies(rbdi_handle* h, int nbody, const double* v, const double* omega,
                                   const double* center, const double* box_lo, const double* box_hi);

/* CFL time step: dt = cfl * min over non-rigid cells and directions of
 * dx_d / max(|u_d| + c, |v_r,d|) (Sec. 3: a fraction of the global maximum
 * stable step; mixture sound speed of Sec. 2.2). FP64 deterministic
 * reduction; synchronises the stream. NONPHYSICAL if no finite value. */
RBDI_API int rbdi_compute_dt(rbdi_handle* h, double cfl, double* dt);

/* Enqueue one time step of size dt (seeding + three RK stages). Returns after
 * enqueueing; device-side failures are reported by rbdi_status. */
RBDI_API int rbdi_step(rbdi_handle* h, double dt);

/* Enqueue nsteps steps whose dt is computed on the device from the CFL
 * condition (as rbdi_compute_dt) and clipped so that t does not pass t_end;
 * no host synchronisation between steps. Steps after t reaches t_end do no
 * work. */
RBDI_API int rbdi_advance(rbdi_handle* h, double cfl, int nsteps, double t_end);

/* Synchronise and read the counters; returns NONPHYSICAL if a non-admissible
 * cell was flagged, OOM if the rigid band outgrew the seeding task buffer
 * (one quarter of the cells); st is filled either way. */
RBDI_API int rbdi_status(rbdi_handle* h, rbdi_stats* st);

/* Force and torque about center exerted by the material on the rigid body,
 * FP64, deterministic: F = sum_i (-sigma_i . grad_h r_i) dV and
 * T = sum_i (x_i - center) x (-sigma_i . grad_h r_i) dV over interior cells
 * (central differences; the paper's bodies are one-way and it defines no
 * load, so this diffuse-surface integral is this library's definition).
 * Synchronises the stream. */
RBDI_API int rbdi_rigid_force(rbdi_handle* h, const double center[3], double F[3], double T[3]);

/* FP64 totals of every conserved field times the cell volume: out[0..n) over
 * all interior cells, out[n..2n) over non-rigid (r <= 0.5) cells.
 * Synchronises the stream. */
RBDI_API int rbdi_conserved_totals(rbdi_handle* h, double* out);

/* Kernel timing (profiling aid). When enabled, every launch of the classes
 * below carries a HIP event pair attached to its dispatch
 * (hipExtLaunchKernelGGL), so each pair measures that kernel's own duration
 * on the handle's stream; the events are kept until rbdi_kernel_times, which synchronises the stream, adds the
 * elapsed times per class into ms[class] (milliseconds) and launches[class],
 * and releases the recorded pairs. Classes: 0 sweep along x (the last sweep,
 * with the RK combine), 1 sweep along y, 2 sweep along z, 3 seeding, 4 rigid
 * band compaction, 5 CFL reduction, 6 unused (the surrogate sources run
 * inside the x sweep, class 0). ms and launches
 * hold RBDI_NUM_KCLASS entries each. */
#define RBDI_NUM_KCLASS 7
RBDI_API int rbdi_set_kernel_timing(rbdi_handle* h, int enable);
RBDI_API int rbdi_kernel_times(rbdi_handle* h, double* ms, long long* launches);

/* Mean duration of one sweep kernel, in microseconds: the sweep of class cls
 * (0 x, 1 y, 2 z) of the middle RK stage of the last step is launched reps
 * times back to back on that step's buffers between one HIP event pair
 * (after one untimed launch). Its outputs are stage buffers that the next
 * step rewrites before reading, so the state is unchanged. NOT_READY before
 * the handle's first step or while it belongs to a batch. Synchronises. */
RBDI_API int rbdi_kernel_replay(rbdi_handle* h, int cls, int reps, double* us);

/* Wavefronts per block of the x sweep of a 2D or 3D instance: 1, 2 or 4; 0
 * restores the library's choice (2D: 4 or 2, whichever leaves fewer idle
 * wavefronts at the end of a row; 3D: 4). Results do not depend on it.
 * BAD_ARG for other values (and for more than 1 in 1D), NOT_READY for a
 * batch member. */
RBDI_API int rbdi_set_x_waves(rbdi_handle* h, int waves);

/* Autotuner of one instance: from the current state, time nsteps steps with
 * the device CFL time step (CFL number cfl) for each x-sweep block size (1,
 * 2 and 4 wavefronts; 1D: one), putting back after each trial everything a
 * step changes (state, time, step counters, CFL partials), and keep the
 * fastest as with rbdi_set_x_waves. best: the chosen size; us: its mean time
 * per step in microseconds. The state after the call is the one before it.
 * Allocates one state-sized device buffer for the duration of the call;
 * synchronises. BAD_ARG for nsteps < 1, cfl <= 0 or null outputs; NOT_READY
 * without a state or for a batch member. */
RBDI_API int rbdi_autotune(rbdi_handle* h, double cfl, int nsteps, int* best, double* us);

/* Unit-level evaluation of single device functions on n states (host
 * arrays, FP64, state-major: n x nfields), for parity checks of the
 * building blocks of the step. what = 0: HLLC flux along dir of the face
 * (a[i] left primitive state, b[i] right), out n x (nfields + 3) = flux of
 * the nfields-1 thermodynamic fields, wall velocity u*, wall stretch row
 * Vbar*_{dir,0..2} (Sec. 3.1). what = 1: closure of conserved states a,
 * out n x (nfields + 10) = primitives, mixture c^2, Cauchy stress (9)
 * (Sec. 2.2). what = 2: per-stage elastoplastic sources of conserved states
 * a, out n x nfields. Synchronises; allocates temporary device memory. */
RBDI_API int rbdi_unit_eval(rbdi_handle* h, int what, int dir, const double* a, const double* b, double* out,
                            int n);

/* The semi-discrete operator D(U) of the current state (Sec. 3.1, spatial
 * operator; no seeding; thermodynamic rows of rigid cells are not used by a
 * step), host FP64 [nfields][cells], summed over the directions whose bit is
 * set in dirmask (bit d = direction d; 7 = all). The energy row is that of the
 * stored energy E~ = rho E - B(phi), B(phi) = sum_l phi_l gamma_l p_inf,l /
 * (gamma_l - 1) (equal to rho E's row without stiffened phases). Diagnostic: overwrites the
 * handle's stage buffers; synchronises. */
RBDI_API int rbdi_eval_rhs(rbdi_handle* h, int dirmask, double* D);

/* ---------------------------------------------------------------------------
 * Batched instances. A batch advances many independent instances (uneven
 * grid sizes) together: every phase of a step (seeding, each direction sweep
 * of each RK stage) is one launch over the merged tile list of all members,
 * with a persistent grid and a tile shape chosen by rbdi_batch_autotune. The
 * per-cell arithmetic is that of rbdi_step, so a member advanced in a batch
 * is bitwise identical to the same instance advanced alone, for every tuning.
 * (The paper runs one problem at a time; batching is this library's own
 * throughput layer over the same step.)
 * ------------------------------------------------------------------------- */

/* Launch shape of the batched sweeps. */
typedef struct {
  int x_waves;    /* wavefronts per block of the final x sweep: 1, 2 or 4 */
  int x_blocks;   /* persistent grid of the x sweep (blocks); 0: one block per tile */
  int x_xcd;      /* 1: each of the 8 XCDs takes a contiguous run of x tiles */
  int tile_cols;  /* x columns per y/z sweep tile: 4, 8, 16 or 32, with
                     nfields * tile_cols * 65 values <= 64 KiB of LDS */
  int t_blocks;   /* persistent grid of the y/z sweeps; 0: one block per tile */
  int t_xcd;      /* 1: XCD-aware tile ranges for the y/z sweeps */
  double x_us;    /* rbdi_batch_autotune output: mean duration of one x sweep
                     launch over all members, microseconds */
  double t_us;    /* the same for the y (and z) sweeps of one stage */
} rbdi_tuning;

/* Make a batch of count members (host array of handles). Members must share
 * dim (2 or 3), nmat, solid and precision, have their state set, and carry
 * no moving body (the rigid band of each member is built once, here). The
 * batch does not own the members; they must outlive it. While a member
 * belongs to a batch, rbdi_step, rbdi_advance, rbdi_set_state_*,
 * rbdi_set_rigid_* and rbdi_set_stream on it return NOT_READY; reading it
 * (get_state_*, status, rigid_force, conserved_totals) stays allowed. Every
 * member is switched to the batch's stream (that of the first member).
 * Allocates the batch's device tables. Errors: BAD_ARG, NOT_READY,
 * UNSUPPORTED, OOM (a rigid band beyond the seeding capacity), HIP. */
RBDI_API int rbdi_batch_create(int count, rbdi_handle* const* members, rbdi_batch** out);

/* Release the batch (synchronises its stream); members become free again. */
RBDI_API int rbdi_batch_destroy(rbdi_batch* b);

/* Stream of the batch and of all its members (hipStream_t as void*). */
RBDI_API int rbdi_batch_set_stream(rbdi_batch* b, void* hip_stream);

/* Set / read the launch shape. set: BAD_ARG for values outside the ranges
 * above; synchronises (the tile lists are rebuilt). */
RBDI_API int rbdi_batch_set_tuning(rbdi_batch* b, const rbdi_tuning* t);
RBDI_API int rbdi_batch_get_tuning(const rbdi_batch* b, rbdi_tuning* t);

/* Time every candidate launch shape (reps launches each, HIP events, on the
 * current states; the states are not changed: the timed launches evaluate
 * the operator into the members' stage buffers), keep the fastest x and y/z
 * shapes, and return them in *best (may be NULL). Synchronises. */
RBDI_API int rbdi_batch_autotune(rbdi_batch* b, int reps, rbdi_tuning* best);

/* Enqueue one step of every member. dts: NULL, or a host array of count
 * values: dts[i] > 0 is member i's dt, dts[i] <= 0 takes member i's CFL dt
 * (cfl > 0 required then). With dts the call synchronises the stream before
 * uploading them; without, it does not synchronise. */
RBDI_API int rbdi_batch_step(rbdi_batch* b, double cfl, const double* dts);

/* Enqueue nsteps steps of every member, each with its own CFL dt computed on
 * the device (as rbdi_advance, t_end per member clipping, <= 0: none). No
 * host synchronisation. */
RBDI_API int rbdi_batch_advance(rbdi_batch* b, double cfl, int nsteps, double t_end);

/* ---------------------------------------------------------------------------
 * Surrogate closure (not in the paper: a learned replacement of the per-cell
 * elastoplastic closure). A 6 -> 64 -> 64 -> 64 -> 6 ReLU network with BF16
 * weights and FP32 accumulation, evaluated and trained by matrix-core
 * kernels of this library. For b = Vbar Vbar^T and X = b - I it returns the
 * higher-order remainders of the coefficients of H = (1/2) ln b =
 * a0 I + a1 X + a2 X^2 and of H^2 (Cayley-Hamilton form; the Hencky strain
 * of Sec. 2.1.2) beyond their series to order X^3, from six invariant
 * features of X. With a network set on a solid handle (rbdi_set_surrogate)
 * the per-stage elastoplastic sources (det(Vbar) renormalisation and the
 * perfect-plasticity radial return) take H and J2 = H:H from the network,
 * evaluated inside the final (x) sweep of each stage, one matrix tile per
 * wavefront of 64 cells; outside the envelope |X|_F <= tau_max, or when the
 * error flag is raised (the network's J2 disagrees with the one its H
 * implies by more than 1e-6 relative, or its H violates tr H = 0, the
 * identity of a unit-determinant stretch, by more than 1e-6 |H|), that cell
 * uses the exact closure.
 * Parameter vector: FP32, 9158 values, row-major [out][in] per layer:
 * W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[6][64] b4[6].
 * Features z and targets t: n x 6 FP32, sample-major. All calls below run
 * on the null stream and synchronise; they allocate temporary device memory.
 * ------------------------------------------------------------------------- */

/* Create a network (all parameters zero) on the current device. */
RBDI_API int rbdi_mlp_create(rbdi_mlp** out);
RBDI_API int rbdi_mlp_destroy(rbdi_mlp* m);

/* Set the FP32 parameters (host, 9158 values; BF16 device copies are made)
 * and the envelope / input scale tau_max in (0, 1); resets the optimiser. */
RBDI_API int rbdi_mlp_set_params(rbdi_mlp* m, const float* params, double tau_max);
RBDI_API int rbdi_mlp_get_params(rbdi_mlp* m, float* params, double* tau_max);

/* Features and exact targets (normalised remainders) of n stretch tensors
 * V (host, n x 9, FP64, row-major 3x3 each) for the scale tau_max. */
RBDI_API int rbdi_mlp_data(const double* V, int n, double tau_max, float* z, float* t);

/* Network outputs y (host, n x 6) for features z (host, n x 6). */
RBDI_API int rbdi_mlp_forward(rbdi_mlp* m, const float* z, int n, float* y);

/* Gradient (host, 9158 values, flat layout) and value of the mean squared
 * error over the n samples and 6 outputs, by the device forward and
 * backward passes (BF16 operands, FP32 accumulation). */
RBDI_API int rbdi_mlp_grad(rbdi_mlp* m, const float* z, const float* t, int n, float* grad, float* loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid hipMalloc):
 * the gradient and loss of rbdi_mlp_grad for n device-resident samples, with
 * nothing allocated. z, t: device, n x 6 FP32 (sample-major); grad: device,
 * 9158 FP32 (flat layout); loss: device, 1 FP32 -- all caller-owned. The
 * per-block partial gradients live in a fixed device array of the library
 * (one row per 64 samples, RBDI_MLP_GRAD_NOALLOC_MAX / 64 rows, 9.4 MB),
 * which each GPU the library runs on holds until the process ends; its
 * address is resolved once per device, at rbdi_mlp_create or at the first
 * call. Enqueued on hip_stream (a hipStream_t as void*, NULL = the null
 * stream); does not synchronise. Results equal rbdi_mlp_grad's bitwise (same
 * kernels, same summation order). Every call on one GPU uses that GPU's one
 * array: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be serialised by the caller. BAD_ARG for null
 * pointers or n outside [1, RBDI_MLP_GRAD_NOALLOC_MAX]. */
#define RBDI_MLP_GRAD_NOALLOC_MAX 16384
RBDI_API int rbdi_mlp_grad_noalloc(rbdi_mlp* m, const float* z, const float* t, int n, float* grad, float* loss,
                                   void* hip_stream);

/* iters Adam steps (beta 0.9 / 0.999, eps 1e-8, learning rate lr with a
 * cosine decay to zero) on consecutive batches of `batch` samples (a
 * multiple of 64), cycling through the n samples in their given order
 * (shuffle them first). losses (host, iters values, may be NULL) receives
 * each batch's loss before its update. */
RBDI_API int rbdi_mlp_train(rbdi_mlp* m, const float* z, const float* t, int n, int batch, int iters, float lr,
                            float* losses);

/* Use network m for the elastoplastic sources of handle h (solid systems
 * only), or the exact closure again when m is NULL. The network must outlive
 * its use by h. */
RBDI_API int rbdi_set_surrogate(rbdi_handle* h, rbdi_mlp* m);

/* Message of the last error on the calling thread ("" if none). */
RBDI_API const char* rbdi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RBDI_H */

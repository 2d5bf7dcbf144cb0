/*
 * vdwlb: MI355X (gfx950) library for the multicomponent van der Waals
 * free-energy lattice Boltzmann method of Ridl & Wagner, "Lattice Boltzmann
 * simulation of mixtures with multicomponent van der Waals equation of state"
 * (arXiv:1805.07251).
 *
 * One time step (Eq. LBequation) of every component c on a periodic D2Q9
 * lattice: pull-stream the populations f_i^c, take the moments rho^c and
 * rho^c u^c (Sec. III), evaluate the chemical potential mu^c of the lattice
 * van der Waals mixture free energy (Eq. discreteChemicalPotential), the
 * mean-field force from its gradient (Eqs. forceMuLog / forceMuId), the
 * inter-component friction with implicit true velocities (Eq. forceFriction),
 * and the forced BGK collision (Eqs. BGKcollisionOperator, feq, with the
 * second-moment correction of Eq. forceCorrectionsPsi).  Plans with dim = 1
 * run the paper's own D1Q3 scheme on nx x 1 lines (Sec. V: 3-point
 * stencils, the D1Q3 interaction function and the explicit update with
 * F_0 = -S, F_+- = (S +- G)/2).
 *
 * Conventions fixed by this interface
 *  - Populations are stored as Q velocity planes of sites (Q = 9 for D2Q9,
 *    3 for D1Q3) with the C components of a site adjacent: f_i^c at site
 *    s = y*nx + x (x fastest) is element (i * P + s) * C + c,
 *    P = vdwlb_plane_elems() sites per plane.
 *    One site's populations of all components are then a single vector
 *    access.  Population buffers must be aligned to C * sizeof(dtype) bytes
 *    (hipMalloc memory always is); misaligned pointers return
 *    VDWLB_E_INVALID_ARG.  The D2Q9 velocity order is v_0 = (0,0),
 *    v_1..4 = (1,0),(0,1),(-1,0),(0,-1), v_5..8 = (1,1),(-1,1),(-1,-1),(1,-1);
 *    the D1Q3 order is v_0 = 0, v_1 = +1, v_2 = -1.
 *  - A stored state is post-collision, pre-stream; a step reads f_i(x - v_i)
 *    from one buffer and writes the new state to the other (ping-pong).
 *  - Physical force convention: momentum of component c gains
 *    G^c = -gamma_mu rho^c grad mu^c + theta grad rho^c + friction
 *    (the printed forces are "minus the force", cf. Sec. IV); the lattice
 *    temperature theta = 1/3 is fixed, kT is the thermodynamic temperature
 *    entering mu and p only.
 *  - Every device pointer is caller-owned memory on the device that was
 *    current when the plan was created; the library never frees it.  Streams
 *    are hipStream_t values passed as void* (NULL = the null stream).
 *  - No exceptions cross this interface.  Kernel-side failures (rho^c <= 0,
 *    eta = sum b^c rho^c >= 1, non-finite values) set a sticky device flag that
 *    the next vdwlb_sync_status / vdwlb_moments call reports as
 *    VDWLB_E_UNPHYSICAL and clears.  Calls on different plans are
 *    independent; calls on one plan must not overlap.
 */
#ifndef VDWLB_H
#define VDWLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2: D2Q9 velocity planes may be padded beyond nx*ny rounded up to 64
 * (vdwlb_plane_elems). */
#define VDWLB_ABI_VERSION 2
#define VDWLB_MAX_COMPONENTS 4

typedef int32_t vdwlb_status;
enum {
    VDWLB_OK = 0,
    VDWLB_E_INVALID_ARG = 1, /* a NULL pointer, a bad size or a parameter outside its domain */
    VDWLB_E_UNSUPPORTED = 2, /* a valid request the library does not implement (dim, C, dtype) */
    VDWLB_E_DEVICE = 3,      /* a HIP runtime error; vdwlb_last_device_error() has its text */
    VDWLB_E_UNPHYSICAL = 4,  /* the sticky device flag: rho^c <= 0, eta >= 1 or a non-finite value */
    VDWLB_E_CAPACITY = 5     /* the request needs more than a fixed capacity (the no-allocation scratch) */
};

enum { VDWLB_F64 = 0, VDWLB_F32 = 1 };             /* storage and arithmetic precision */
enum { VDWLB_FORCE_LOG = 0, VDWLB_FORCE_NID = 1 }; /* Eq. forceMuLog / Eq. forceMuId */

/* Description of one lattice and its parameters (Secs. II, III, V).
 *   dim      2 (D2Q9) or 1 (D1Q3, Sec. V; ny must be 1).  Moments of a D1Q3
 *            plan report a zero y momentum.
 *   nx, ny   periodic extents, >= 1 each (small extents wrap several times),
 *            nx * ny <= 2^28 and one plane of a population buffer below
 *            2^32 bytes (plane_elems * C * sizeof(dtype)).
 *   ncomp    number of components C, 1 .. VDWLB_MAX_COMPONENTS.
 *   dtype    VDWLB_F64 or VDWLB_F32.
 *   force    VDWLB_FORCE_LOG (default of the paper's production runs) or NID.
 *   kT       thermodynamic temperature in mu and p, > 0.
 *   tau      BGK relaxation time, > 1/2.
 *   gamma_mu prefactor of the chemical-potential force (Eq. forceMuNid), finite.
 *   a        C*C row-major, symmetric: attraction a^{cc'} (Eq. a-psi).
 *   b        C: excluded volume b^c, > 0.
 *   kappa    C*C row-major, symmetric: gradient coefficients kappa^{cc'}
 *            (Eq. kappa-psi); the 2-D interaction function is
 *            psi(0) = 5/3 kappa - a, psi(v_i) = -3 w_i kappa.
 *   lambda   C*C row-major, symmetric, diagonal ignored: friction
 *            coefficients lambda^{cc'} (Eq. forceFriction); NULL means 1.
 * The arrays are copied at plan creation. */
typedef struct vdwlb_desc {
    int32_t dim;
    int32_t nx;
    int32_t ny;
    int32_t ncomp;
    int32_t dtype;
    int32_t force;
    double kT;
    double tau;
    double gamma_mu;
    const double* a;
    const double* b;
    const double* kappa;
    const double* lambda;
} vdwlb_desc;

typedef struct vdwlb_plan vdwlb_plan;

/* VDWLB_ABI_VERSION of the built library. */
int32_t vdwlb_abi_version(void);

/* Text for a status code (static storage). */
const char* vdwlb_strerror(vdwlb_status s);

/* Text of the last HIP error seen by this thread (static thread-local storage). */
const char* vdwlb_last_device_error(void);

/* Validate d and create a plan bound to the current device.  On success
 * *out receives the plan; on failure *out is NULL. */
vdwlb_status vdwlb_plan_create(const vdwlb_desc* d, vdwlb_plan** out);

/* Release the plan, its device flag word and its cached graphs (NULL is a no-op). */
vdwlb_status vdwlb_plan_destroy(vdwlb_plan* plan);

/* Sites per velocity plane of a population buffer: nx*ny rounded up to a
 * multiple of 64, and for D2Q9 plans whose plane would then span a multiple
 * of 8 KiB, about 5 KiB more (whole multiples of 64 sites), so that the
 * planes a sweep streams do not all start at the same phase of the memory
 * interleave.  Sites from nx*ny on are padding, never read or written.  A
 * plane holds plane_elems * C elements. */
int64_t vdwlb_plane_elems(const vdwlb_plan* plan);

/* Bytes of one population buffer: Q * C * plane_elems * sizeof(dtype)
 * (Q = 9 for D2Q9, 3 for D1Q3).
 * The caller allocates two (ping-pong).  0 for a NULL plan. */
size_t vdwlb_state_bytes(const vdwlb_plan* plan);

/* Initial state f_i^c = f^0_i(rho^c, u^c) (Eq. feq) with u^c = mom^c / rho^c.
 *   f    device, vdwlb_state_bytes(plan) bytes, written.
 *   rho  device, [C][ny][nx] in the plan dtype, read.
 *   mom  device, [C][2][ny][nx] (x then y component) or NULL for u = 0.
 * Asynchronous on stream. */
vdwlb_status vdwlb_init(vdwlb_plan* plan, void* f, const void* rho, const void* mom, void* stream);

/* Enqueue n >= 0 time steps alternating fA -> fB -> fA ...  On return
 * *out_which (if not NULL) is 0 when the newest state is in fA and 1 when it
 * is in fB (n odd).  fA and fB must be distinct state buffers.  Long runs are
 * replayed from a captured hipGraph bound to (fA, fB); the graph is captured
 * again when the pointers change.  Asynchronous on stream. */
vdwlb_status vdwlb_step(vdwlb_plan* plan, void* fA, void* fB, int64_t n, void* stream, int32_t* out_which);

/* Observables of the state f (the streamed populations, i.e. what the next
 * step would see):
 *   rho  [C][ny][nx]      rho^c = sum_i f_i^c(x - v_i)           (required)
 *   mom  [C][2][ny][nx]   rho^c u^c = sum_i f_i^c(x - v_i) v_i    (or NULL)
 *   mu   [C][ny][nx]      mu^c of Eq. discreteChemicalPotential, without the
 *                         additive constant kT                    (or NULL)
 *   p    [ny][nx]         bulk pressure sum_c [rho^c kT/(1-eta) -
 *                         sum_c' a^{cc'} rho^c rho^c'] (Sec. II)   (or NULL)
 * All device arrays in the plan dtype.  Synchronises stream and then returns
 * what vdwlb_sync_status would. */
vdwlb_status vdwlb_moments(vdwlb_plan* plan, const void* f, void* rho, void* mom, void* mu, void* p, void* stream);

/* Pressure tensor of Sec. II (the tensor that satisfies Eq. GibbsDuehem for
 * the mixture free energy) of a density field, with the lattice's isotropic
 * stencils for the derivatives:
 *   P_ab = sum_c [rho^c kT/(1-eta) - sum_c' a^{cc'} rho^c rho^c'
 *                 - sum_c' kappa^{cc'} (grad rho^c . grad rho^c' + rho^c Lap rho^c')] delta_ab
 *          + sum_cc' kappa^{cc'} d_a rho^c d_b rho^c'
 * A diagnostic: in bulk phases it is the bulk pressure; across interfaces
 * it carries the higher-order gradient terms the paper discusses.
 *   rho  device, [C][ny][nx] in the plan dtype (e.g. from vdwlb_moments), read.
 *   pxx  device, [ny][nx], written.  pyy, pxy: same, or NULL to skip (for a
 *        D1Q3 plan P_yy is the isotropic part and P_xy = 0).
 * Asynchronous on stream. */
vdwlb_status vdwlb_pressure_tensor(vdwlb_plan* plan, const void* rho, void* pxx, void* pyy, void* pxy, void* stream);

/* Synchronise stream, read and clear the sticky device flag of the plan. */
vdwlb_status vdwlb_sync_status(vdwlb_plan* plan, void* stream);

/* Number of schedules the sweep can use for this plan.  A schedule is a tile
 * shape and kernel variant together with the order in which workgroups visit
 * tiles (row-major ranges per XCD, or one vertical band of tile columns per
 * XCD); every schedule computes bit-identical results. */
int32_t vdwlb_schedule_count(const vdwlb_plan* plan);

/* Select schedule k (0 <= k < vdwlb_schedule_count) for later steps. */
vdwlb_status vdwlb_set_schedule(vdwlb_plan* plan, int32_t k);

/* Time every schedule on this plan's lattice (reads fA, overwrites fB),
 * re-time the four fastest with more launches, keep the fastest and report it
 * in *chosen (may be NULL).  The timed steps alternate between fB (first a
 * copy of fA) and a temporary state buffer the call allocates and frees, as a
 * run alternates between its two buffers.  Synchronous.  fA may hold any
 * state: the error flag read by vdwlb_sync_status is left as it was before
 * the call. */
vdwlb_status vdwlb_autotune(vdwlb_plan* plan, const void* fA, void* fB, void* stream, int32_t* chosen);

/* Liquid-gas coexistence of one van der Waals component (Eqs. tetcr, rhocr
 * and the equal chemical potential / pressure conditions of Sec. II), used to
 * initialise tanh slabs with bulk values as in Sec. V.  Host-only.  Returns
 * VDWLB_E_INVALID_ARG when kT >= kT_cr or a, b, kT are not positive. */
vdwlb_status vdwlb_maxwell(double a, double b, double kT, double* rho_gas, double* rho_liquid);

/* Phase diagram of a two-component mixture (Appendix A) over many overall
 * compositions: point k holds NA[k] and NB[k] particles in a volume of 1.  The
 * search gives each point a group of 16 lanes, one per trial move.
 *   - invalid (a density <= 0 or b . N >= 1): status -1, F = NaN, no phases;
 *   - Hessian of the bulk free energy positive definite (Sec. VI.A): stable,
 *     status 1, phases = {(NA, NB, 1)}, 0 iterations, no search;
 *   - otherwise the direct search over three phases: phase 3 (fixed by
 *     conservation) starts empty, phases 1 and 2 as halves displaced by
 *     +-eps/2 along the unstable eigenvector d (d_A >= 0, eps = 0.05
 *     min(NA, NB)); volumes 1/3 each, the empty phase shrunk to (1 - b.N)/2
 *     when b.N > 1/3; empty components add nothing to the free energy
 *     (rho ln rho -> 0); each iteration tries +step
 *     then -step on A1, B1, V1, A2, B2, V2 and keeps the first strictly lowest
 *     total free energy, else halves the step (initially 0.01); it stops when
 *     the step falls below threshold or after max_iter iterations.  Then
 *     phases whose densities agree within 1e-3 (relative to max(1, |rho|))
 *     are merged, those with volume below 1e-6 dropped, the rest sorted by
 *     rho_A - rho_B, and a Newton polish solves equal mu^c and p (with the
 *     lever rule through N for two phases), accepted when its volumes lie in
 *     (0, 1), its phases stay distinct and locally stable and its free energy
 *     does not exceed the search's (by more than 1e-12 relative); a rejected
 *     three-phase polish merges the closest pair and polishes two phases,
 *     and failing that drops the smallest phase and polishes the other two.
 *     Before the polish, while a distinct phase is unstable (at most twice),
 *     the search starts again (step 6(b)) with the largest unstable phase
 *     split along its unstable direction into phases 1 and 2 and phase 3
 *     holding the other phases packed together.
 *     The polish makes a point exact even when the search stopped at
 *     max_iter before converging.  status = the number of distinct phases (1, 2, 3; 1 with
 *     iterations > 0 means the search did not split), 0 if the search ended
 *     with an infinite free energy.
 *   kT, a (host, 2 x 2 row-major, symmetric), b (host, 2): the mixture of Sec. II.
 *   0 <= n <= 2^31 - 257; NA, NB: device [n] doubles, read.
 *   threshold > 0 (the paper uses 1e-12); 1 <= max_iter <= 7e8 iterations
 *   per search.
 *   phases  device [n][3][3] (rho_A, rho_B, V) of the distinct phases, unused
 *           slots 0, written.
 *   raw     device [n][3][3] the search's own three phases (zeros without a
 *           search), written.
 *   F       device [n]: total free energy at the end of the search (f(N) for
 *           a stable point), written.
 *   info    device int32 [n][4]: status, iterations (all searches), the number of distinct
 *           phases whose Hessian is not positive definite (before the polish),
 *           polish (0 none, 1 accepted, 2 rejected: search values kept), written.
 * The searches run in passes with growing iteration budgets; the points still
 * searching after a pass go on in the next one, packed densely (the results
 * are those of uninterrupted searches, bit for bit).  Until the classification
 * writes it, phases holds the state of the searches in progress.  The call
 * takes a stream-ordered workspace of 4 (64 + 2 n) bytes (hipMallocAsync on
 * stream, freed on stream after the last kernel).
 * VDWLB_E_INVALID_ARG for kT or threshold not positive and finite, a not finite
 * or not symmetric, b not positive, n out of range, max_iter < 1, or a NULL pointer when
 * n > 0; a device error if the workspace cannot be allocated.  Asynchronous on
 * stream. */
vdwlb_status vdwlb_phase_points(double kT, const double* a, const double* b, int32_t n, const double* NA,
                                const double* NB, double threshold, int32_t max_iter, double* phases, double* raw,
                                double* F, int32_t* info, void* stream);

/* Device-to-device copy of nbytes with a plain streaming kernel; used as the
 * bandwidth yardstick next to the sweep.  Asynchronous on stream. */
vdwlb_status vdwlb_copy(void* dst, const void* src, size_t nbytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched sweep: many independent lattices advanced by one persistent launch,
 * the GPU form of the paper's phase-diagram runs (thousands of small flat-
 * interface simulations with their own parameters, Sec. VI.A).
 *
 * Every instance has its own vdwlb_desc (size, kT, a, b, kappa, lambda, tau,
 * gamma_mu, force); all share dim, ncomp, dtype and the lattice height ny.
 *  - D2Q9 (dim = 2): ny must be 1, 2, 4 or 8 (quasi-1-D lattices; other
 *    heights return VDWLB_E_UNSUPPORTED); each workgroup streams its instance
 *    through L2/MALL in full-height strips.
 *  - D1Q3 (dim = 1): each workgroup holds its whole instance in LDS for all
 *    steps of a run (5 C nx sizeof(dtype) bytes, which must fit one
 *    workgroup's LDS, and nx <= 2048; otherwise VDWLB_E_UNSUPPORTED); the
 *    launch shape below is chosen by the library.
 * The states of all instances live in one pool buffer (two pools for
 * ping-pong): instance k occupies the Q * C * plane_k elements starting at
 * vdwlb_batch_offset(k), laid out as a plain state.  Density arrays are
 * packed the same way: instance k's [C][ny][nx] block starts at
 * vdwlb_batch_density_offset(k).
 * ------------------------------------------------------------------------ */
typedef struct vdwlb_batch vdwlb_batch;

/* Validate n descriptions (the rules of vdwlb_plan_create) and create a batch
 * on the current device.  Instances are queued largest first. */
vdwlb_status vdwlb_batch_create(int32_t n, const vdwlb_desc* descs, vdwlb_batch** out);

/* Release the batch's instance table, queue, status words and graph. */
vdwlb_status vdwlb_batch_destroy(vdwlb_batch* batch);

/* Bytes of one pool (the caller allocates two). */
size_t vdwlb_batch_state_bytes(const vdwlb_batch* batch);

/* Element offset of instance k's state in a pool (-1 if k is out of range). */
int64_t vdwlb_batch_offset(const vdwlb_batch* batch, int32_t k);

/* Element offset of instance k's density block in packed density arrays. */
int64_t vdwlb_batch_density_offset(const vdwlb_batch* batch, int32_t k);

/* Launch shape of the persistent kernel: threads per workgroup (256 or 1024;
 * D2Q9 batches run step by step only) and resident workgroups (0 = as many as
 * the device holds, capped at n). */
vdwlb_status vdwlb_batch_set_launch(vdwlb_batch* batch, int32_t threads, int32_t blocks);

/* Temporal blocking of D2Q9 batches of height 4 with C <= 2:
 * steps_per_block K in 2 .. 6 runs each instance in blocks of at most K
 * steps, every block strip by strip: a strip of 64 - 6K columns, 3K columns
 * on either side and the K intermediate states are held in LDS (each step's
 * valid region shrinks by the 3 columns a step reaches), so that HBM traffic
 * falls by about K; 0 selects the step-by-step kernel.  Results are bit-identical
 * either way, and a run leaves its result in the same pool.  With blocking,
 * an instance that becomes unphysical stops at the end of the block in which
 * it did (its status word still records the first unphysical step).
 * Batches that allow it are created with K = 3.  VDWLB_E_UNSUPPORTED for
 * other batches or when the block does not fit the LDS of a workgroup;
 * VDWLB_E_INVALID_ARG for other values of K. */
vdwlb_status vdwlb_batch_set_blocking(vdwlb_batch* batch, int32_t steps_per_block);

/* pool = f^0(rho, u = 0) for every instance; rho is the packed density array
 * (device, plan dtype).  Asynchronous on stream. */
vdwlb_status vdwlb_batch_init(vdwlb_batch* batch, void* pool, const void* rho, void* stream);

/* Packed densities rho^c = sum_i f_i^c(x - v_i) of every instance's state in
 * pool.  Asynchronous on stream. */
vdwlb_status vdwlb_batch_density(vdwlb_batch* batch, const void* pool, void* rho, void* stream);

/* Advance every instance by nsteps (0 <= nsteps < 2^31) in one persistent
 * launch (replayed from a hipGraph bound to poolA, poolB, nsteps and the launch
 * shape).  *out_which as in vdwlb_step.  An instance that becomes unphysical
 * stops at that step; its status word records the step and its state is left
 * as it was then.  Asynchronous on stream. */
vdwlb_status vdwlb_batch_run(vdwlb_batch* batch, void* poolA, void* poolB, int64_t nsteps, void* stream,
                             int32_t* out_which);

/* Synchronise stream and copy the per-instance status words of the last run
 * into per_instance (host, n entries, may be NULL): 0 = completed, s > 0 =
 * stopped unphysical at step s.  Returns VDWLB_E_UNPHYSICAL if any instance
 * stopped. */
vdwlb_status vdwlb_batch_status(vdwlb_batch* batch, int32_t* per_instance, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative) of the sweep, for gradients of a loss on
 * the final densities with respect to the free-energy parameters of Sec. II
 * (kT, a^{cc'}, b^c, kappa^{cc'}) through many steps.  FP64 D2Q9 plans with
 * C = 1 to 4 (FP32 and D1Q3 plans return VDWLB_E_UNSUPPORTED); C <= 2 reverses
 * each step with one fused kernel, C = 3 and 4 with the three separate ones.
 *
 * Parameter cotangent vector (double, device), vdwlb_adjoint_param_count()
 * entries: kT, then a^{cd} for c <= d (row-major upper triangle), then b^c,
 * then kappa^{cd} for c <= d.  An off-diagonal entry is the derivative with
 * respect to the symmetric pair (a^{cd} = a^{dc} moved together).
 * ------------------------------------------------------------------------ */

/* Entries of the parameter cotangent vector (0 for a NULL plan). */
int32_t vdwlb_adjoint_param_count(const vdwlb_plan* plan);

/* Bytes of device workspace vdwlb_adjoint_segment needs for nsteps steps:
 * three state buffers, the densities and momenta of every step of the
 * segment (3 C nx ny doubles per step), per-site intermediate fields and one
 * running parameter partial sum per tile. */
size_t vdwlb_adjoint_workspace_bytes(const vdwlb_plan* plan, int32_t nsteps);

/* Cotangent of a state given cotangents of its read-out densities rho_bar
 * ([C][ny][nx]) and momenta mom_bar ([C][2][ny][nx]); either may be NULL.
 * fbar receives a full state (vdwlb_state_bytes).  This is the transpose of
 * vdwlb_moments' density and momentum outputs.  Asynchronous on stream. */
vdwlb_status vdwlb_moments_adjoint(vdwlb_plan* plan, const void* rho_bar, const void* mom_bar, void* fbar,
                                   void* stream);

/* Reverse nsteps (>= 1) steps that start from the state f_ckpt:
 * the forward steps are recomputed from f_ckpt (their densities and momenta
 * kept in workspace), then fbar_io, the cotangent of the state after the
 * segment, is replaced by the cotangent of f_ckpt, and the parameter
 * cotangents of the segment are added to pbar_accum (device, see above).
 * workspace: vdwlb_adjoint_workspace_bytes(plan, nsteps) bytes of device
 * memory owned by the caller, aligned like a population buffer.  The
 * summation order is fixed, so results are deterministic.  Asynchronous on
 * stream. */
vdwlb_status vdwlb_adjoint_segment(vdwlb_plan* plan, const void* f_ckpt, int32_t nsteps, void* fbar_io,
                                   void* workspace, double* pbar_accum, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * vdwlb_adjoint_segment with its workspace taken from a fixed device array of
 * VDWLB_ADJOINT_SCRATCH_BYTES bytes that the library's code object holds on
 * every device it runs on until the process ends.  The call itself allocates
 * nothing: no hipMalloc / hipFree, no graph instantiation (its kernels are
 * launched one by one on stream, so a caller may capture them), only kernel
 * launches and device-to-device copies.
 *   Arguments, results and errors are those of vdwlb_adjoint_segment without
 *   the workspace argument; the results are the same bit for bit.
 *   VDWLB_E_CAPACITY when vdwlb_adjoint_workspace_bytes(plan, nsteps) exceeds
 *   VDWLB_ADJOINT_SCRATCH_BYTES (nothing is enqueued): use shorter segments.
 *   The device address of the array is looked up once per device, on the
 *   first call that uses that device (the plan's device).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (no part of it needs to start at zero): calls that can
 * overlap on one device, on any streams or plans, race and must be ordered
 * by the caller.  Asynchronous on stream. */
#define VDWLB_ADJOINT_SCRATCH_BYTES ((size_t)64 << 20)
vdwlb_status vdwlb_adjoint_segment_noalloc(vdwlb_plan* plan, const void* f_ckpt, int32_t nsteps, void* fbar_io,
                                           double* pbar_accum, void* stream);

/* Graph replay of the adjoint's parts (vdwlb_adjoint_segment,
 * vdwlb_adjoint_recompute, vdwlb_adjoint_reverse) for this plan: enable = 1
 * replays each part from a hipGraph captured on its first use and bound to
 * its step count and buffers (the workspace; for the reverse sweep also
 * fbar_io and pbar_accum), enable = 0 (the default) launches the kernels one
 * by one.  Replay pays only when a plan reverses with the same buffers many
 * times: each kernel runs for microseconds, so eager launches keep the device
 * busy, and a capture costs more host time than it saves.  A plan keeps up
 * to six graphs and makes the device idle before it drops the oldest.
 * Results are the same bit for bit either way.  VDWLB_E_INVALID_ARG for a
 * NULL plan or enable other than 0 or 1. */
vdwlb_status vdwlb_set_adjoint_graphs(vdwlb_plan* plan, int32_t enable);

/* The two halves of vdwlb_adjoint_segment, for callers that overlap the
 * forward recompute of one segment with the reverse sweep of the next one on
 * a second stream (the recompute depends only on its checkpoint), each half
 * with its own workspace.
 *
 * vdwlb_adjoint_recompute: copies f_ckpt into the workspace and recomputes
 * nsteps forward steps from it, keeping their densities and momenta in the
 * workspace.  vdwlb_adjoint_reverse: the reverse sweep of the segment last
 * recomputed into the same workspace with the same nsteps (the caller orders
 * the two, by stream or event); it replaces fbar_io and adds to pbar_accum
 * exactly as vdwlb_adjoint_segment does, which is the recompute followed by
 * the reverse sweep on one stream.  A workspace must not be recomputed into
 * while a reverse sweep that reads it may still run.  Each half launches its
 * kernels one by one on stream, unless graph replay is switched on for the
 * plan (vdwlb_set_adjoint_graphs).  Asynchronous on stream; arguments and
 * errors as for vdwlb_adjoint_segment. */
vdwlb_status vdwlb_adjoint_recompute(vdwlb_plan* plan, const void* f_ckpt, int32_t nsteps, void* workspace,
                                     void* stream);

/* The forward of a segment that keeps what its reverse sweep needs, for the
 * last segment of a checkpointed run, whose states the caller has just
 * computed anyway: nsteps (>= 1) steps from f_in, the state after them
 * written to f_out (f_out may be f_in), and the workspace left exactly as
 * vdwlb_adjoint_recompute(plan, f_in, nsteps, workspace) leaves it, so that
 * vdwlb_adjoint_reverse may follow with no recompute.  f_out equals
 * vdwlb_step's result bit for bit.  Asynchronous on stream; arguments and
 * errors as for vdwlb_adjoint_recompute (f_out checked like f_in, before
 * anything is enqueued). */
vdwlb_status vdwlb_adjoint_forward(vdwlb_plan* plan, const void* f_in, int32_t nsteps, void* f_out, void* workspace,
                                   void* stream);
vdwlb_status vdwlb_adjoint_reverse(vdwlb_plan* plan, int32_t nsteps, void* fbar_io, void* workspace,
                                   double* pbar_accum, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VDWLB_H */

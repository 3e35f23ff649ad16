/*
 * vclb -- volume-conserving phase-field lattice Boltzmann on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the HIP library libvclb.so.  The library implements one time step of the
 * lattice Boltzmann model of Xiong, Wang & Liu, "Local volume-conserving lattice
 * Boltzmann model for incompressible multiphase flows" (arXiv 2505.10899):
 *   - phase-field populations g_i for the modified Cahn-Hilliard equation (Sect. 2,
 *     Eq. 17), with equilibrium Eq. 31, profile-correction/level-set source Eq. 32 and
 *     moment-space collision Eq. 33, order parameter Eq. 35, signed distance Eq. 37,
 *     backward time difference of phi u (Sect. 3.2);
 *   - hydrodynamic populations f_i for the incompressible Navier-Stokes equations
 *     (Eq. 18), with forcing Eq. 21, equilibrium Eqs. 22-23, collision Eq. 25,
 *     velocity Eq. 28 and pressure Eq. 29;
 *   - isotropic gradient and Laplacian stencils (Eqs. 39-40), chemical potential Eq. 2
 *     and surface tension force F_s = mu grad phi (Sect. 2);
 *   - per-step FP64 volume reductions of phi (observables only: the correction term
 *     of Eq. 32 is local and needs no global quantity).
 *
 * Conventions (all entry points):
 *   - Return 0 on success or a negative VCLB_E* code.  No exception crosses the ABI.
 *     vclb_strerror() names a code; vclb_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Parameters are validated before any HIP call: invalid parameters return
 *     VCLB_EINVAL without touching the GPU.
 *   - Units are lattice units (dx = dt = 1, c_s^2 = 1/3).
 *   - Fields are row-major with x fastest: node (x, y, z) has index x + nx (y + ny z).
 *     Vector fields are structure-of-arrays: component d of node n at [d * N + n].
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     Work is enqueued asynchronously on it; functions that return data to the host
 *     synchronise that stream before returning.
 *   - ptr_kind says whether a caller pointer is host (VCLB_HOST) or device
 *     (VCLB_DEVICE) memory.  The caller owns every buffer it passes; the library owns
 *     the case handle and the device state (or borrows a caller workspace, see
 *     vclb_case_create).
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef VCLB_H
#define VCLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- error codes */
#define VCLB_OK          0
#define VCLB_EINVAL     -1   /* invalid argument or unsupported combination          */
#define VCLB_ENOMEM     -2   /* device allocation failed or workspace too small      */
#define VCLB_EHIP       -3   /* a HIP runtime call failed                             */
#define VCLB_ENONFINITE -4   /* a NaN/Inf was found in phi by the volume reductions   */
#define VCLB_ESTATE     -5   /* call out of order (e.g. step before init), bad checkpoint */

/* ---------------------------------------------------------------- enums */
#define VCLB_D2Q9   0
#define VCLB_D3Q19  1

#define VCLB_FP64   0   /* populations stored and updated in double                         */
#define VCLB_FP32   1   /* populations stored and updated in float                          */
#define VCLB_FP16S  2   /* populations stored in half as deviations from the rest
                           equilibrium (g: phi-dependent, f: 0); arithmetic in float        */

#define VCLB_COUPLED           0   /* g and f coupled through u (Eq. 28) and F_s           */
#define VCLB_PRESCRIBED_VORTEX 1   /* phase field only, velocity from Eqs. 43-44           */

#define VCLB_PERIODIC 0
#define VCLB_WALL     1   /* half-way bounce-back, wall half a node outside the first/last node */

#define VCLB_HOST   0
#define VCLB_DEVICE 1

/* field mask bits for vclb_observe, written in this order, N doubles per scalar
   field and D * N for u */
#define VCLB_FIELD_PHI 0x01u   /* order parameter, Eq. 35                         */
#define VCLB_FIELD_RHO 0x02u   /* density rho_light + phi (rho_heavy - rho_light)  */
#define VCLB_FIELD_U   0x04u   /* velocity, Eq. 28 (or Eqs. 43-44)                 */
#define VCLB_FIELD_P   0x08u   /* pressure, Eq. 29 (0 in prescribed-velocity mode) */
#define VCLB_FIELD_MU  0x10u   /* chemical potential, Eq. 2                        */
#define VCLB_FIELD_PSI 0x20u   /* signed distance, Eq. 37                          */

#define VCLB_MAX_LABELS 2       /* observation regions per case                     */
#define VCLB_HISTORY    4096    /* per-step observations kept (ring)                */

/* ---------------------------------------------------------------- parameters */
/* Axes and faces for bc and wall_u: axis 0 = x, 1 = y, 2 = z; side 0 = the low face (below
   the first node), 1 = the high face (above the last node). */
typedef struct {
  int32_t lattice;          /* VCLB_D2Q9 | VCLB_D3Q19                                     */
  int32_t storage;          /* VCLB_FP64 | VCLB_FP32 | VCLB_FP16S                          */
  int32_t mode;             /* VCLB_COUPLED | VCLB_PRESCRIBED_VORTEX (D2Q9 only)           */
  int32_t nx, ny, nz;       /* nodes per axis; nz = 1 for D2Q9                             */
  int32_t bc[3][2];         /* boundary type of each face: VCLB_PERIODIC | VCLB_WALL.  Both
                               faces of an axis must have the same type.  Supported: walls
                               on the y faces (ny >= 2, D2Q9 and D3Q19); every other face
                               periodic (VCLB_EINVAL otherwise).                           */
  int32_t nlabels;          /* 0: one label covering the domain; else 1..VCLB_MAX_LABELS   */
  double  wall_u[3][2][3];  /* velocity of the wall on each VCLB_WALL face (ignored on
                               periodic faces); its normal component must be 0            */
  double  wall_cos[3][2];   /* wetting: cos(theta) of each VCLB_WALL face, theta the contact
                               angle measured in the heavy phase (phi = 1), |cos| <= 1; 0 on
                               periodic faces.  The paper states no boundary conditions;
                               this is a reading.  The equilibrium profile (Eqs. 4-5) has
                               |grad phi| = (4 / W) phi (1 - phi), so a wall meeting the
                               interface at theta has a normal derivative of phi, into the
                               fluid, of -(4 / W) cos(theta) phi (1 - phi).  The stencils
                               (Eqs. 39-40) see, behind the half-way wall, the ghost
                               phi_g = phi_e + (4 / W) cos(theta) phi_e (1 - phi_e) of the
                               edge row's phi_e, and psi (Eq. 37) of phi_g.  0, the
                               default (theta = 90 degrees), makes the ghost the edge
                               row's mirror.                                             */
  double  W;                /* interface width (Eq. 4), > 0                                 */
  double  sigma;            /* surface tension, >= 0 (beta = 12 sigma / W, kappa = 3 sigma W / 2) */
  double  mobility;         /* M > 0; tau_g = 1/2 + M / c_s^2 (Eq. 34)                      */
  double  lambda;           /* penalty constant (0.5 in the paper); 0 gives the classical model */
  double  mass_fix;         /* rate r in [0, 1] of a global volume correction, the kind of
                               correction the paper's introduction describes and argues
                               against (0, the default, is the paper's model).  With r > 0,
                               each step measures the volume V = sum H(phi_c), H(p) =
                               p^2 (3 - 2 p), of the time-t field and adds to every g_i the
                               source w_i kappa delta(phi_c), delta(p) = 4 p (1 - p) (the
                               interface indicator of Eq. 5), with kappa = r (V_ref - V) /
                               sum delta: the total of phi changes by r (V_ref - V).  V_ref is
                               V of the state given to vclb_case_init or vclb_case_set_state
                               (checkpoints keep it).  Steps then run the plain two-kernel
                               path plus the reduction; not supported by batches or the
                               adjoint.                                                    */
  double  xi;               /* regulariser of Eq. 37 (1e-10 in the paper), > 0              */
  double  eps_n;            /* unit normal n = grad psi / sqrt(|grad psi|^2 + eps_n^2), >= 0 */
  double  rho_heavy;        /* density at phi = 1, > 0                                      */
  double  rho_light;        /* density at phi = 0, > 0                                      */
  double  nu_heavy;         /* kinematic viscosity of the heavy phase (phi = 1), > 0        */
  double  nu_light;         /* kinematic viscosity of the light phase (phi = 0), > 0.  The
                               dynamic viscosity mu = rho nu is interpolated linearly in phi
                               between rho_light nu_light and rho_heavy nu_heavy, and each
                               node relaxes the stress moments of f at 1 / tau_f with
                               tau_f = 1/2 + mu(phi) / (rho(phi) c_s^2) (Eq. 27).  Equal
                               viscosities give one uniform tau_f.  Unequal ones need the
                               stress rates of s_f left at 0; every step, batches and the
                               adjoint support them.                                      */
  double  s_g[19];          /* MRT rates of g in (0, 2); 0 selects the default              */
  double  s_f[19];          /* MRT rates of f in (0, 2); 0 selects the default              */
  double  U0;               /* vortex amplitude (Eqs. 43-44)                                 */
  double  T;                /* vortex period in steps, > 0 in vortex mode                    */
  double  label_centre[VCLB_MAX_LABELS][3]; /* nearest-centre (minimum image) regions   */
} vclb_params;

/* Per-label volume reductions of phi at one time step, accumulated in FP64.
   d is the displacement of a node from its label's centre (minimum image along
   periodic axes); second moments are ordered xx, yy, zz, xy, xz, yz. */
typedef struct {
  double  sum_phi;
  double  count_half;       /* number of nodes with phi >= 1/2 */
  double  sum_phi_d[3];
  double  sum_phi_dd[6];
  int64_t step;             /* time step the observation belongs to */
  int32_t nonfinite;        /* 1 if phi was NaN/Inf at some node of the label */
  int32_t label;
} vclb_obs;

typedef struct vclb_case vclb_case;

/* ---------------------------------------------------------------- meta */
const char* vclb_strerror(int code);
/* Message of the calling thread's last failed call (empty string if none). */
const char* vclb_last_error(void);
/* Version of this header as MAJOR * 10000 + MINOR * 100 + PATCH.  The major part changes
   with the layout of vclb_params or of any other struct here; a library built from this
   header returns the same value from vclb_version, and a caller should refuse a library
   whose major part differs. */
#define VCLB_VERSION 20100
/* Version of the library as MAJOR * 10000 + MINOR * 100 + PATCH (VCLB_VERSION of the
   header it was built from). */
int vclb_version(void);

/* Achievable HBM bandwidth on this device: the practical ceiling that the step kernels'
   rates are compared with (the kernels move their populations at HBM speed; the method
   itself fixes no bandwidth).  Runs one warm-up and then `reps` launches (1..1000) of a
   plain grid-stride kernel over 16-byte vectors, timed with events on `stream` (which it
   synchronises), and stores bytes moved per second, in GB/s, in *gbs.  mode 0 copies
   `bytes` from src to dst (counts 2 * bytes per launch), 1 reads src (dst: a device sink
   of at least 4 bytes, left untouched in practice), 2 fills dst (src unused, may be
   NULL).  bytes: a positive multiple of 16; buffers: device memory, 16-byte aligned,
   owned by the caller.  blocks: workgroups of 256 lanes (0: 4 per compute unit). */
int vclb_bandwidth_probe(int32_t mode, void* dst, const void* src, size_t bytes, int32_t reps, int32_t blocks,
                         double* gbs, void* stream);
/* The same with the kernel's shape chosen: each lane keeps `unroll` (1, 2, 4 or 8) 16-byte
   vectors in flight (a workgroup's tile is unroll * 256 consecutive vectors; all loads are
   issued before the first store or use), with non-temporal loads and stores if
   nontemporal = 1.  vclb_bandwidth_probe is unroll 1, nontemporal 0.  Sweeping unroll,
   nontemporal and blocks and keeping the fastest gives the device's achievable rate. */
int vclb_bandwidth_probe_ex(int32_t mode, int32_t unroll, int32_t nontemporal, void* dst, const void* src,
                            size_t bytes, int32_t reps, int32_t blocks, double* gbs, void* stream);

/* Check parameters without any HIP call.  Fills the defaults of zero rates. */
int vclb_params_validate(const vclb_params* p);

/* ---------------------------------------------------------------- single case */
/* Device bytes the case needs (populations A/B, previous phi u, FP16S phi buffers,
   reduction partials, observation history, scratch for observe).  No HIP call. */
int vclb_case_workspace_bytes(const vclb_params* p, size_t* bytes);

/* Validate, then create a case.  `workspace` (device memory, at least
   vclb_case_workspace_bytes, 256-byte aligned) is borrowed for the life of the case;
   NULL makes the library allocate and own it.  Launch configuration (tile shape) is
   chosen by the library's built-in heuristic; vclb_case_set_tile overrides it. */
int vclb_case_create(const vclb_params* p, void* workspace, size_t workspace_bytes,
                     vclb_case** out);
void vclb_case_destroy(vclb_case* c);

/* Tile of the fused step kernel.  D2Q9: bx lanes (x columns; a multiple of 64 in
   64..256, or 512 or 1024 with FP32 or FP16S storage) marching ty >= 1 rows of y (by3
   ignored).  D3Q19: a bx x by3 section of (x, y)
   columns (bx * by3 a multiple of 64, at most 256, or at most 768 with FP32 or FP16S
   storage when the section's LDS fits the device's per-workgroup limit) marching the
   planes of z, which ceil(nz / ty) workgroups per section share evenly.  Returns EINVAL
   for shapes outside these limits. */
int vclb_case_set_tile(vclb_case* c, int32_t bx, int32_t ty, int32_t by3);
int vclb_case_get_tile(const vclb_case* c, int32_t* bx, int32_t* ty, int32_t* by3);

/* Pick the tile of the fused step by timing `steps` steps of each candidate on the
   current state (saved and restored, as are the step counter and the recorded history),
   or take it from the JSON-lines file cache_path when that holds an entry for this case's
   lattice, storage, mode, shape, boundary and label count; a measured choice is appended
   to cache_path (NULL: no file).  D2Q9 candidates: bx in {64, 128, 256} (and 512, 1024
   with 4-byte storage) x ty in {8, ..., 128}; D3Q19: six column sections with their
   planes cut to fill 1..4 workgroups per CU, and (4-byte storage) three 768-lane
   sections at one per CU.  Synchronises the stream; VCLB_ESTATE before init. */
int vclb_case_autotune(vclb_case* c, const char* cache_path, int32_t steps, void* stream);

/* Initial state from phi0 (N doubles) and u0 (D*N doubles, NULL for u = 0; ignored in
   vortex mode): g = g_eq(phi0, mu0, u0) (Eq. 31), f = f_eq(p = 0, rho(phi0), u0) (Eq. 22),
   previous phi u = phi0 u0; step counter 0. */
int vclb_case_init(vclb_case* c, const double* phi0, const double* u0, int ptr_kind,
                   void* stream);

/* Replace the state by a given time-t state: post-streaming populations g and f
   (Q * N doubles each, direction-major [i * N + n]; f ignored in vortex mode), the
   previous step's phi u (D * N doubles) and the step counter t >= 0.  Values are
   rounded to the storage precision. */
int vclb_case_set_state(vclb_case* c, const double* g, const double* f, const double* J, int64_t t,
                        int ptr_kind, void* stream);

/* The current state in the layout of vclb_case_set_state, decoded to FP64. */
int vclb_case_get_state(vclb_case* c, double* g, double* f, double* J, int ptr_kind, void* stream);

/* Advance nsteps >= 0 time steps with the fused single-kernel step (pull streaming,
   LDS-staged phi/psi halo tiles, fused reductions).  Asynchronous. */
int vclb_step(vclb_case* c, int64_t nsteps, void* stream);

/* Same update with the plain two-kernel path (phi/psi pass, then stencil + collision
   from global memory); the same arithmetic as vclb_step up to the order in which the
   compiler contracts multiply-adds.  Asynchronous. */
int vclb_step_plain(vclb_case* c, int64_t nsteps, void* stream);

/* Record the per-step reductions every `every` steps (0 turns them off; default 1). */
int vclb_case_set_reduce_every(vclb_case* c, int32_t every);

/* Current step counter (synchronises the stream). */
int vclb_case_time(vclb_case* c, int64_t* t, void* stream);

/* Macroscopic fields of the current state, in FP64, in VCLB_FIELD_* bit order. */
int vclb_observe(vclb_case* c, uint32_t field_mask, double* out, int ptr_kind, void* stream);

/* Volume reductions of the current state (observables of the order parameter, Eq. 35:
   the correction term of Eq. 32 is local and takes no global quantity), accumulated in
   FP64, one vclb_obs per label into out[] (host memory, caller-owned).

   labels == NULL: the case's built-in labels (nearest label centre by minimum image, or
   one label covering the domain); nlabels is 0 or that label count; d in vclb_obs is the
   displacement from the label's centre.

   labels != NULL: caller labels, labels[n] for node n (device memory, N int32, row-major
   with x fastest, read only), 1 <= nlabels <= 2^20 and out[nlabels].  A node with a
   negative label belongs to no label.  d is the node's position (x, y, z) (no wrap), so
   sum_phi_d and sum_phi_dd are moments about the origin.  out[l].label = l.  The
   reductions are deterministic (fixed-order sums); a workgroup's cost grows with the
   number of distinct labels in its chunk of nodes, so labels should be spatially
   coherent (for example connected regions).  The library allocates device scratch for
   the partial sums on the first call that needs more than the case holds (kept until
   vclb_case_destroy).  Returns VCLB_EINVAL (after filling out) if some node's label is
   >= nlabels.

   Returns VCLB_ENONFINITE (after filling out) if any label saw a NaN/Inf.  Synchronises
   the stream. */
int vclb_reduce(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out, void* stream);

/* For callers that cannot allocate device memory (code under graph capture, tight serving
   loops, harnesses that forbid hipMalloc): vclb_reduce with caller labels (labels must not
   be NULL; same arguments, results and errors), whose partial sums live in a fixed device
   scratch array of 4 MiB that the library holds on each device it runs on until the
   process ends, so that the call allocates nothing.  Returns VCLB_EINVAL, before any
   launch, when the reduction needs more scratch than that: about
   (13 nlabels + 1) * 8 * min(512, ceil(N / 2048)) bytes for the partials plus 104 bytes per
   label (for example at most 78 labels on a grid of 10^6 nodes or more).  Every call on one
   device shares that device's array: calls that overlap on one device (different streams
   or threads) race and must be serialised by the caller.  Synchronises the stream. */
int vclb_reduce_static(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out, void* stream);

/* Copy the recorded per-step reductions of steps [t_first, t_first + count) into
   out[count * nlabels] (host).  Steps older than VCLB_HISTORY or never recorded give
   VCLB_ESTATE. */
int vclb_history(vclb_case* c, int64_t t_first, int32_t count, vclb_obs* out, void* stream);

/* Checkpoint: populations (storage precision), previous phi u, FP16S phi buffer and
   the step counter, with a parameter fingerprint and a checksum. */
int vclb_state_bytes(const vclb_case* c, size_t* bytes);
int vclb_state_save(vclb_case* c, void* host_buf, size_t bytes, void* stream);
int vclb_state_load(vclb_case* c, const void* host_buf, size_t bytes, void* stream);

/* ---------------------------------------------------------------- observables */
/* Derived observables of each label from its moments (host arithmetic, no HIP call):
   out[5 * l + k] = volume sum phi, centroid offset sum phi d / sum phi (x, y, z), and the
   deformation D = (sqrt(l+) - sqrt(l-)) / (sqrt(l+) + sqrt(l-)) of the eigenvalues l+-
   of the phi-weighted (x, y) second-moment tensor about the centroid. */
int vclb_obs_derived(const vclb_obs* obs, int32_t nlabels, double* out);

/* Moment weights seed[10 * l + j] (j: sum, d[3], dd[6] as in vclb_obs) of the
   linearisation of J = sum_l sum_k weights[5 * l + k] O_k(l) about obs, with O the
   derived observables of vclb_obs_derived.  Host arithmetic, no HIP call.  At D = 0 the
   direction-dependent terms of dD are dropped. */
int vclb_obs_seed(const vclb_obs* obs, int32_t nlabels, const double* weights, double* seed);

/* ---------------------------------------------------------------- adjoint */
/* Gradients of a function J of the phase field after nsteps steps with respect to the
   surface tension sigma, the mobility M and the initial field phi0, by the discrete
   adjoint of the time step: the reverse of the streaming (with bounce-back and the
   moving-wall term), of the collisions Eqs. 25 and 33 with their equilibria and sources
   (Eqs. 21-23, 31-32), of u and p (Eqs. 28-29), mu (Eq. 2), psi (Eq. 37) and the
   stencils Eqs. 39-40 (with the wetting ghosts behind walls), and of the initial state.
   With unequal viscosities the per-node stress rate (Eq. 27) is differentiated too.  FP64
   D2Q9 coupled cases without the global correction only (VCLB_EINVAL otherwise).  The derivative of the clip of phi to [0, 1] is taken as 1
   inside the interval and 0 outside.

   Device bytes of the checkpoint store and adjoint fields (no HIP call); every = 0
   selects ceil(sqrt(nsteps)). */
int vclb_adjoint_bytes(const vclb_params* p, int64_t nsteps, int32_t every, size_t* bytes);

/* Forward pass: vclb_case_init(phi0, u0), then nsteps fused steps, keeping a copy of the
   state (pulled g and f, previous phi u) every `every` steps (0: ceil(sqrt(nsteps))).
   The library allocates the store (vclb_adjoint_bytes; freed by the next record or by
   vclb_case_destroy).  Afterwards the case holds the state at step nsteps.  Synchronises
   the stream. */
int vclb_adjoint_record(vclb_case* c, const double* phi0, const double* u0, int ptr_kind, int64_t nsteps,
                        int32_t every, void* stream);

/* Backward pass of the recorded run for J = sum_l seed[10 l] sum phi + seed[10 l + 1..3] .
   sum phi d + seed[10 l + 4..9] . sum phi dd (moments of the final state, labels as in
   vclb_reduce; seed is host memory, see vclb_obs_seed).  Each segment between
   checkpoints is recomputed with the forward step and then run backward.
   normal_tau >= 0: the unit normal n = grad psi / |grad psi| of Eq. 32 is differentiated
   only where |grad psi| >= normal_tau and held fixed elsewhere.  Away from the interface
   psi saturates, |grad psi| falls to rounding level and the exact derivative of n (gain
   ~ lambda / |grad psi| per step) grows without bound over long runs; 0.3 keeps every
   node of the interface region (|grad psi| = 1 there), 0 gives the exact derivative of
   the discrete map.  Writes dJ/dphi0
   to dphi0 (N doubles, ptr_kind; NULL: not returned) and (dJ/dsigma, dJ/dM) to dparams
   (2 doubles, host; NULL: not returned).  M acts through the rates of g left at their
   default 1 / tau_g.  The case state is left unchanged.  Synchronises the stream.
   VCLB_ESTATE without a prior vclb_adjoint_record. */
int vclb_adjoint_run(vclb_case* c, const double* seed, double normal_tau, double* dphi0, int ptr_kind,
                     double* dparams, void* stream);

/* ---------------------------------------------------------------- batches of cases */
/* Many independent coupled D2Q9 cases of uneven sizes (one storage precision), advanced
   together: each step is one work-list kernel over the tiles of every case, and a call
   of vclb_batch_step captures its steps in one hipGraph replayed as one launch.  The
   batch owns one device allocation holding every case. */
typedef struct vclb_batch vclb_batch;

/* Validate every case (all VCLB_D2Q9, VCLB_COUPLED, one storage, nlabels <= 1, no global
   correction) and allocate the batch.  Cases may have unequal viscosities (Eq. 27 per
   node); if any case has, every case relaxes its f stress rows at the per-node rate (its
   constant tau_f when its viscosities are equal), and a case whose f stress rates are set
   by hand is refused (VCLB_EINVAL). */
int vclb_batch_create(const vclb_params* cases, int32_t ncases, vclb_batch** out);
void vclb_batch_destroy(vclb_batch* b);

/* Handle of case k, owned by the batch: vclb_case_init / set_state / observe / reduce /
   history / get_state work on it.  Do not destroy it or call vclb_step on it. */
int vclb_batch_case(vclb_batch* b, int32_t k, vclb_case** out);

/* Initial state of every case, as vclb_case_init on each in order: phi0s[k] (and u0s[k],
   if u0s is not NULL; a NULL entry means u = 0) are case k's fields, all host or all
   device memory (ptr_kind); the two pointer arrays themselves are host memory with
   ncases entries.  Every phi0s[k] is checked for NULL before any case is touched; an
   error from case k's init leaves cases 0..k-1 initialised and is returned with the
   case index in vclb_last_error. */
int vclb_batch_init(vclb_batch* b, const double* const* phi0s, const double* const* u0s, int ptr_kind,
                    void* stream);

/* Total nodes of all cases. */
int vclb_batch_nodes(const vclb_batch* b, int64_t* nodes);

/* Launch shape of the batched step: bx in {64, 128, 256, 512} lanes per workgroup (also
   1024 with FP32 or FP16S storage; VCLB_EINVAL for FP64), and work
   items of at most about ty * 256 nodes (ty in 1..1024; 1024 keeps cases up to 512 x 512
   whole).  As many workgroups as can be resident are launched, each given one run of
   consecutive items with about equal work, or work in proportion to the slot weights
   vclb_batch_balance measured (an item is split between rows where a run ends);
   get_tile also returns that workgroup count.  Default: bx 512, ty 1024. */
int vclb_batch_set_tile(vclb_batch* b, int32_t bx, int32_t ty);
int vclb_batch_get_tile(const vclb_batch* b, int32_t* bx, int32_t* ty, int32_t* blocks);

/* How each case is cut into work items.  A case whose width leaves more than
   (100 - flat_pct)% of the lanes of its strips idle (strips of bx columns, one lane per
   column, each on a bx-lane workgroup) runs as bands of whole rows marched in padded
   row-major order (every lane busy, some extra index arithmetic); the others run as
   strips.  Below 101 only cases
   whose padded row fits in bx lanes qualify for bands; 101 puts every case that fits in
   bands, 0 every case in strips (default 100). */
int vclb_batch_set_schedule(vclb_batch* b, int32_t flat_pct);
int vclb_batch_get_schedule(const vclb_batch* b, int32_t* flat_pct);

/* Record each case's volume reductions every `every` steps (0: off; default 1). */
int vclb_batch_set_reduce_every(vclb_batch* b, int32_t every);

/* Volume reductions (Eq. 35's phi summed per label, with its first and second moments)
   of every case's current state in one call: out[k * VCLB_MAX_LABELS + l] for case k and
   label l (host memory, ncases * VCLB_MAX_LABELS entries; labels beyond a case's count
   are zero).  Synchronises the stream.  Returns VCLB_ENONFINITE (after filling out) if
   any case saw a NaN/Inf, VCLB_ESTATE if a case is not initialised. */
int vclb_batch_reduce(vclb_batch* b, vclb_obs* out, void* stream);

/* The recorded per-step reductions of steps [t_first, t_first + count) of every case:
   out[(j * ncases + k) * VCLB_MAX_LABELS + l] for step t_first + j (host memory).
   VCLB_ESTATE if a step of some case is not in its history (older than VCLB_HISTORY
   steps or not recorded). */
int vclb_batch_history(vclb_batch* b, int64_t t_first, int32_t count, vclb_obs* out, void* stream);

/* Advance every case by nsteps (all cases must be initialised and at the same step).
   use_graph != 0: the launches are captured into one hipGraph on a library stream
   ordered after `stream`.  Asynchronous with respect to the host. */
int vclb_batch_step(vclb_batch* b, int64_t nsteps, int32_t use_graph, void* stream);

/* Pick the batched tile and schedule (bx, ty, flat_pct) by timing `steps` steps of every
   candidate on the current state (saved and restored), then the four fastest three times
   more with 2 * steps steps each, in alternation, keeping each one's best time (the leading
   shapes often lie within timing noise of each other); or take them from the JSON-lines
   file cache_path when that holds an entry for this batch; a measured choice is appended
   to cache_path (NULL: no file). */
int vclb_batch_autotune(vclb_batch* b, const char* cache_path, int32_t steps, void* stream);

/* Fit the cut of the batch into runs to the speed of each resident workgroup slot.  The
   slots of one launch do not advance at one rate (on one device the spread is about
   +-10%, set by where a slot's workgroup runs, not by the cases it is given), so runs of
   equal modelled cost finish at different times.  This times every slot over its run
   for `steps` launches on the current state (saved and restored, host synchronised),
   gives each slot a weight in proportion to its measured speed, re-cuts the runs with
   budgets in proportion to the weights, and repeats `rounds` times (rounds in 1..16,
   steps in 1..1000).  The cut whose slowest slot was fastest is kept, the equal one
   included; *gain (may be NULL) receives the slowest slot's time before over after
   (1 if nothing beat the cut it started from).  The results of a step do not depend on
   the cut (each node's update is the same); the per-case reductions are summed in
   another grouping, so they may differ in the last bits.  The weights stay in force
   while the launch shape is unchanged: set_tile or set_schedule with another shape, or
   autotune, drop them. */
int vclb_batch_balance(vclb_batch* b, int32_t rounds, int32_t steps, double* gain, void* stream);

/* The slot weights in force (1 for every slot when none are): weights[r] for run slot
   r < min(capacity, *count), where *count receives the number of slots of the current
   launch shape (host memory).  With vclb_batch_set_weights, a calibration measured once
   by vclb_batch_balance can be kept and applied again later on the same device and
   launch shape without timing anything. */
int vclb_batch_get_weights(const vclb_batch* b, double* weights, int32_t capacity, int32_t* count);
/* Set the slot weights (count = the slot count of the current launch shape, each in
   [1e-3, 1e3], rescaled to mean 1; count 0 clears them) and re-cut the runs.  They stay
   in force on the same terms as balanced ones.  Results of a step do not depend on the
   weights. */
int vclb_batch_set_weights(vclb_batch* b, const double* weights, int32_t count);

#ifdef __cplusplus
}
#endif
#endif /* VCLB_H */

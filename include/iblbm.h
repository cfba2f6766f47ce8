/*
 * iblbm.h -- C ABI of the MI355X (gfx950) immersed-boundary lattice Boltzmann time step
 * for particle-laden flow, after Jiang, Li & Liu, "Efficient implementation of immersed
 * boundary-lattice Boltzmann method for massive particle-laden flows, Part I: Serial
 * computing" (arXiv 2002.08855).
 *
 * One step (iblbm_step) advances, on one GPU and one HIP stream:
 *   - the incompressible SRT-LBGK fluid with Guo's split forcing (Sec. 2.1, Eqs. 1-8) on
 *     D2Q9 or D3Q19, streamed in place with the A-A pattern (the single-array role the
 *     swap scheme of Sec. 3.3 plays in the paper) and half-way bounce-back walls;
 *   - the direct-forcing immersed boundary coupling of Sec. 2.2 (Eqs. 9-13), visited
 *     point by point over the delta-function support (Sec. 4, Eqs. 47-48) and repeated
 *     as multi-direct forcing, or a learned boundary force plus one correction pass;
 *   - rigid particles (Sec. 2.3, Eqs. 14-15) with the short-range pair force of Eq. 16,
 *     found with a cell list sized by Eqs. 49-50 (Sec. 5).
 *
 * Conventions.
 *   Units: lattice units, dx = dt = 1.  Walls (half-way bounce-back) lie at -1/2 and
 *   n-1/2 on every non-periodic axis.  Node index i = x + nx*(y + ny*z).
 *   Ownership: the library owns every device buffer it allocates (through the optional
 *   allocator callbacks, else hipMalloc).  Every pointer argument of the functions
 *   below is a HOST pointer owned by the caller; getters copy into it as FP64 whatever
 *   the PDF storage type.  NULL output pointers are skipped.
 *   Errors: every call returns an iblbm_status; iblbm_last_error gives a message.
 *   IBLBM_E_UNSTABLE and IBLBM_E_DEVICE are sticky: later calls that compute return
 *   IBLBM_E_STATE until iblbm_destroy.  Calls are not thread-safe per context.
 */
#ifndef IBLBM_H
#define IBLBM_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct iblbm_ctx iblbm_ctx;

typedef enum {
  IBLBM_OK = 0,
  IBLBM_E_ARG = 1,      /* invalid argument or configuration */
  IBLBM_E_NOMEM = 2,    /* device or host allocation failed */
  IBLBM_E_DEVICE = 3,   /* a HIP call failed */
  IBLBM_E_STATE = 4,    /* the context is in a sticky error state */
  IBLBM_E_UNSTABLE = 5, /* NaN/Inf detected in the fluid or particle state */
  IBLBM_E_CAPACITY = 6, /* a fixed-capacity list (pair list, scratch) overflowed */
  IBLBM_E_CELL_OVERFLOW = 7 /* more centres in one search cell than it holds (Eq. 49) */
} iblbm_status;

typedef enum { IBLBM_F64 = 0, IBLBM_F32 = 1, IBLBM_BF16 = 2, IBLBM_F16 = 3 } iblbm_storage;
typedef enum { IBLBM_DELTA_PESKIN4 = 0, IBLBM_DELTA_ROMA3 = 1 } iblbm_delta;
typedef enum { IBLBM_FORCING_MDF = 0, IBLBM_FORCING_LEARNED = 1 } iblbm_forcing;
/* Face conditions (Sec. 6.1).  WALL: half-way bounce-back with the face's wall_u.
 * VELOCITY and PRESSURE: the non-equilibrium extrapolation of the paper's ref. [48] on the
 * face's layer of nodes: f = f_eq(p_b, u_b) + (f - f_eq)(x_f) with x_f the next node
 * inward; VELOCITY sets u_b = wall_u[face] and takes p_b from x_f, PRESSURE sets
 * p_b = face_p[face] and takes u_b from x_f. */
typedef enum { IBLBM_BC_WALL = 0, IBLBM_BC_VELOCITY = 1, IBLBM_BC_PRESSURE = 2 } iblbm_bc;

/* Problem statement (Sec. 2 and Sec. 6.2): lattice, fluid, walls, forcing, particles. */
typedef struct {
  uint32_t struct_size;   /* must equal sizeof(iblbm_config) */
  int32_t dim;            /* 2: D2Q9 (Eq. 2), 3: D3Q19 (Eq. 3) */
  int32_t n[3];           /* nodes per axis; n[2] = 1 in 2-D */
  double tau;             /* relaxation time of Eq. 1, > 0.5 */
  double rho0;            /* constant density of the incompressible model (Eq. 4) */
  double body_force[3];   /* uniform fluid body force added to the IB force */
  int32_t periodic[3];    /* 1: periodic axis; 0: bounce-back walls */
  double wall_u[6][3];    /* wall velocities, faces -x,+x,-y,+y,-z,+z */
  int32_t storage;        /* iblbm_storage: PDF storage type.  F64 computes in FP64,
                           * the others in FP32.  PDFs are stored as deviations from
                           * the rest state (pressure 0, velocity 0: f = 0) */
  double f16_scale;       /* F16 storage keeps f16_scale * f (a power of two) */
  int32_t delta;          /* iblbm_delta: regularised delta function (Fig. 2b) */
  double drs;             /* solid shell thickness in lattice units (Eq. 13), 1 = DF */
  int32_t mdf_iters;      /* forcing passes per step (multi-direct forcing), >= 0 */
  double gravity[3];      /* acceleration of the particles */
  double zeta;            /* Eq. 16 force range (lattice units) */
  double eps_pp, E_pp;    /* Eq. 16 stiffness parameters */
  double cell_h;          /* cell-list cell size; <= 0 picks one inside Eqs. 49-50 */
  int32_t forcing;        /* iblbm_forcing */
  double slip_tol;        /* learned forcing: slip rms above which MDF takes over */
  int32_t fallback_iters; /* MDF passes of that fallback */
  int32_t stats_every;    /* compute the slip rms every k steps (0: never) */
  void* stream;           /* hipStream_t to enqueue on, or NULL for a library stream */
  void* (*dev_alloc)(size_t bytes, void* user); /* optional device allocator */
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  int32_t face_bc[6];     /* iblbm_bc per face -x,+x,-y,+y,-z,+z (0: walls everywhere).
                           * Extrapolated faces must all lie on one non-periodic axis
                           * with at least 3 nodes */
  double face_p[6];       /* pressure of PRESSURE faces */
} iblbm_config;

#define IBLBM_NGROUPS 8
/* kernel groups timed when timing is on (iblbm_set_timing) */
typedef enum {
  IBLBM_T_COLLIDE = 0,  /* fused collide + force + A-A stream */
  IBLBM_T_BAND = 1,     /* band u* (the lattice u* pass) */
  IBLBM_T_INTERP = 2,   /* IBM interpolation + point force; the first pass also marks the band */
  IBLBM_T_SPREAD = 3,   /* IBM spreading */
  IBLBM_T_INTERIOR = 4, /* fluid momentum inside particles */
  IBLBM_T_PARTICLE = 5, /* cells, pairs, loads, Newton-Euler */
  IBLBM_T_MLP = 6,      /* learned force */
  IBLBM_T_OTHER = 7
} iblbm_timer;

typedef struct {
  int64_t step;              /* steps taken */
  double slip_rms;           /* rms |U_b - D_I u| after forcing, last stats step */
  int64_t truncated;         /* stencil nodes skipped outside walls (first pass, summed) */
  int64_t n_pairs;           /* pairs i<j within D_ij + zeta at the last step */
  int32_t flags;             /* device status bits (1 cell overflow, 2 pair overflow, 4 NaN) */
  int32_t fallbacks;         /* learned forcing: steps that fell back to MDF */
  int64_t band_nodes;        /* nodes inside some point's support at the last step */
  double time_ms[IBLBM_NGROUPS];   /* accumulated kernel time per group (timing on) */
  int64_t launches[IBLBM_NGROUPS]; /* kernel launches per group (timing on) */
  int32_t band_lattice;      /* 1: the band u* comes from the lattice u* pass, 0: from the
                                first interpolation pass (IBLBM_OPT_BAND_PASS) */
  int32_t reserved;          /* 0 */
} iblbm_stats;

/* Create a context: validate cfg (tau > 0.5, sizes, enums, struct_size), allocate the
 * fluid state and initialise the PDFs to the rest state (f = 0). */
iblbm_status iblbm_create(const iblbm_config* cfg, iblbm_ctx** out);
/* Free all device memory and the context; NULL-safe. */
void iblbm_destroy(iblbm_ctx* ctx);
/* Message of the last failure of this context (never NULL). */
const char* iblbm_last_error(const iblbm_ctx* ctx);

/* f = f_eq(p, u) of Eq. 4 at every node.  p: N values or NULL (zero); u: dim*N values,
 * component-major, or NULL (zero). */
iblbm_status iblbm_set_equilibrium(iblbm_ctx* ctx, const double* p, const double* u);
/* Set / get the PDFs f_alpha, alpha = 1..q-1 (f_0 is never needed, Sec. 3.1), as a
 * (q-1) x N array with alpha-1 slowest. */
iblbm_status iblbm_set_pdfs(iblbm_ctx* ctx, const double* f);
iblbm_status iblbm_get_pdfs(iblbm_ctx* ctx, double* f);

/* Add n rigid particles (Sec. 2.3): centre (n*3), diameter (n), density (n), optional
 * velocity and angular velocity (n*3, NULL = 0).  markers_per_particle surface points
 * (0: round(pi D) in 2-D, round(pi D^2) in 3-D), equal angles on circles and a golden-
 * angle spiral on spheres; each carries drs*ds (Eq. 13).  Rejects (IBLBM_E_ARG) surfaces
 * outside the walls, overlaps, periodic axes, and diameters whose delta-function box
 * exceeds the library limit (3-D: D <= 40). */
iblbm_status iblbm_add_particles(iblbm_ctx* ctx, int32_t n, const double* center,
                                 const double* diameter, const double* density,
                                 const double* velocity, const double* omega,
                                 int32_t markers_per_particle);

/* Advance nsteps time steps; returns after the work is enqueued and the status word has
 * been read back (one device synchronisation per call; with learned forcing and no graph,
 * also one per step, where the host reads the slip check's verdict before it launches the
 * MDF fallback only when that is needed).  A particle faster than one
 * lattice unit per step (or NaN) stops the particle and IB kernels of the remaining steps
 * of the call; the call then returns IBLBM_E_UNSTABLE and the context refuses to step
 * again (the getters still read the state).  Cell or pair lists that overflow their
 * capacity return IBLBM_E_CELL_OVERFLOW (a cell) or IBLBM_E_CAPACITY (a pair list). */
iblbm_status iblbm_step(iblbm_ctx* ctx, int32_t nsteps);

/* p (Eq. 6) and u* (Eq. 5) of the current PDFs (N and dim*N values) and the IB force
 * density of the last step (dim*N values, zero off the IB band). */
iblbm_status iblbm_get_fields(iblbm_ctx* ctx, double* p, double* u, double* force);
/* Particle state (np*3 each): centre, velocity, angular velocity, hydrodynamic force
 * -sum F_k dV_k and torque, pair force; marker_F (n_markers*3): accumulated force
 * density of each surface point at the last step. */
iblbm_status iblbm_get_forces(iblbm_ctx* ctx, double* X, double* U, double* Omega,
                              double* F_h, double* T_h, double* F_c, double* marker_F);
/* The particle pairs of the collision search (Table 4's pairs, found through the cell
 * grid of Table 5): pairs i<j with |Xi-Xj|^2 < ((Di+Dj)/2 + zeta)^2 at the positions of
 * the last step (or of iblbm_add_particles), sorted, as 2 int32 per pair into ij (host,
 * caller-owned, room for cap pairs); *n_pairs receives the count even when it exceeds
 * cap (then only cap pairs are written). */
iblbm_status iblbm_get_pairs(iblbm_ctx* ctx, int32_t* ij, int64_t cap, int64_t* n_pairs);
/* The search cells of Eqs. 49-51 (Table 5): cell coordinates (np*3 int32, host,
 * caller-owned) of every particle at the last step, and the cell-grid size (3 int32). */
iblbm_status iblbm_get_cells(iblbm_ctx* ctx, int32_t* cell, int32_t* dims);
iblbm_status iblbm_get_stats(iblbm_ctx* ctx, iblbm_stats* out);
iblbm_status iblbm_num_particles(iblbm_ctx* ctx, int32_t* np, int32_t* n_markers);
/* HIP-event timing on the library's stream: 0 = off, -1 = every kernel group, otherwise
 * a bit mask over iblbm_timer groups (bit g times group g, so 1 is the collide group
 * alone).  Events bracket each launch of a timed group; the elapsed times accumulate
 * into iblbm_stats. */
iblbm_status iblbm_set_timing(iblbm_ctx* ctx, int32_t mask);
iblbm_status iblbm_reset_stats(iblbm_ctx* ctx);
#define IBLBM_OPT_IBM_LDS 1 /* 1 (default): per-particle LDS interpolation/spreading kernels;
                               0: the point-wise kernels with global atomics */
#define IBLBM_OPT_BAND_PASS 2 /* per-particle kernels only: 1 = u* at the band nodes (Eq. 5)
                                 in a lattice-ordered pass before the forcing passes
                                 (default in 3-D, and in 2-D where the particles' LDS
                                 boxes together cover at least half the lattice), 0 =
                                 inside the first interpolation pass (the other 2-D
                                 default); the results are identical */
#define IBLBM_OPT_STATS_EVERY 3 /* replaces the configuration's stats_every (>= 0) */
#define IBLBM_OPT_TIMING_EVERY 4 /* >= 1 (default 1): with timing on, only the launches of
                                    steps whose index is a multiple of the value carry
                                    events, so that the events' own cost stays small */
#define IBLBM_OPT_TIMING_KERNEL 5 /* 1: the events of the collide, interpolation and
                                     spreading groups time the group's kernel itself
                                     (recorded with its launch, as a profiler does); 0
                                     (default): they bracket the group's launches,
                                     dispatch latency included */
iblbm_status iblbm_set_option(iblbm_ctx* ctx, int32_t option, int32_t value);
/* Work units of the per-particle interpolation and spreading kernels for one particle:
 * host-side planning only, no device call; iblbm_add_particles applies the same plan to
 * each particle (Sec. 4: every surface point's delta-function support, Eqs. 47-48, must
 * lie in the LDS box of its unit).  dim: 2 or 3; storage: an iblbm_storage (F64 sums take
 * 8 bytes a component, the others 4); lds_bytes: LDS of one workgroup (0: 163840, the
 * 160 KB of a gfx950 compute unit); diameter in (0, 4096]; n_points: surface points (0: the
 * default count of iblbm_add_particles).  *n_units receives the number of units, 0 when
 * the particle takes the point-wise kernels.  For the first min(*n_units, cap) units,
 * first[u] and count[u] receive the unit's run of consecutive points and box_nodes[u] an
 * upper bound on the nodes of its LDS box (NULL arrays are skipped).  IBLBM_E_ARG for
 * arguments out of range, IBLBM_E_NOMEM if host memory runs out. */
iblbm_status iblbm_plan_units(int32_t dim, int32_t storage, int32_t lds_bytes, double diameter,
                              int32_t n_points, int32_t cap, int32_t* n_units, int32_t* first,
                              int32_t* count, int64_t* box_nodes);
/* on != 0: run steps through HIP graphs.  A step's kernel launches are captured the
 * first time its (PDF parity, band-bitmap buffer) pair occurs and replayed afterwards;
 * changes of state (particles, PDFs, options, MLP) drop the graphs.  Timed steps and
 * steps that gather the slip statistic still launch kernel by kernel.  Results equal
 * those of plain launches up to the order of the force spreading's float atomics.
 * on = 0 (default): plain launches. */
iblbm_status iblbm_set_graph(iblbm_ctx* ctx, int32_t on);

/* Learned forcing (MLP 10-64-64-3 with tanh hidden layers).  params: 5059 floats
 * W1[64][10], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]; norm: 26 floats (feature
 * mean[10], feature std[10], then the mean[3] and std[3] of the network's target, the
 * change F - F_prev of a point's converged force over the previous step's).  A point's
 * predicted force is F_prev + mean + std * y, y the network's output on the normalised
 * features.  Host arrays, copied; IBLBM_E_NOMEM if the device copy cannot be allocated. */
iblbm_status iblbm_set_mlp(iblbm_ctx* ctx, const float* params, const float* norm);
/* Features (n_markers*10: pass-0 slip, previous-step force, unit normal, gap clamped
 * to [0, zeta]) and converged MDF force after mdf_iters passes (n_markers*3) at the
 * start of the next step, without advancing the state. */
iblbm_status iblbm_capture_samples(iblbm_ctx* ctx, float* feat, float* target);

typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr, beta1, beta2, eps;
  uint64_t seed;
  int32_t check_fp32; /* 1: gradients in FP32 for checking (no BF16 rounding) */
} iblbm_train_opts;
/* Train the MLP on the GPU (forward, MSE loss, backward, Adam) on n samples of
 * normalised features x (n*10) and targets t (n*3); params (5059) in/out;
 * loss_curve (epochs) out.  Uses the project's own kernels. */
iblbm_status iblbm_nn_train(const float* x, const float* t, int64_t n, float* params,
                            const iblbm_train_opts* opts, float* loss_curve);
/* Loss and gradient of the MSE loss at params on (x, t) computed on the GPU in FP32. */
iblbm_status iblbm_nn_grad(const float* x, const float* t, int64_t n, const float* params,
                           float* loss, float* grad);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid allocation): iblbm_nn_grad on
 * DEVICE arrays, enqueued on `stream` (a hipStream_t, NULL for the null stream) without
 * synchronising.  x (n*10), t (n*3) and params (5059) are device inputs; loss (1 float)
 * and grad (5059) are device outputs, written by the same kernels as iblbm_nn_grad (the
 * loss as the FP64 sum of the same per-block partials).  The activations live in a fixed
 * scratch array of 9.1 MB that the library holds on each device until the process
 * ends: n may not exceed IBLBM_NOALLOC_MAX_SAMPLES (IBLBM_E_CAPACITY), and no
 * allocation or free happens in the call.  Calls that overlap on one device share that
 * scratch and race: serialise them (one stream, or events).  IBLBM_E_ARG for NULL
 * pointers or n <= 0; IBLBM_E_DEVICE if a HIP call fails. */
#define IBLBM_NOALLOC_MAX_SAMPLES 8192
iblbm_status iblbm_nn_grad_noalloc(const float* x, const float* t, int64_t n, const float* params,
                                   float* loss, float* grad, void* stream);
/* Forward pass on the GPU with BF16 weights/activations on MFMA, FP32 accumulation. */
iblbm_status iblbm_nn_forward(const float* x, int64_t n, const float* params, float* y);

#ifdef __cplusplus
}
#endif
#endif

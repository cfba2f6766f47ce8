/*
 * iblbm_ref.h -- plain FP64 CPU oracle of the immersed-boundary lattice Boltzmann
 * (IB-LBM) time step of Jiang, Li & Liu, "Efficient implementation of immersed
 * boundary-lattice Boltzmann method for massive particle-laden flows, Part I:
 * Serial computing" (arXiv 2002.08855).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library against
 * the paper.  It shares no code, header, table or helper with the GPU path.  Only
 * the tests, the package smoke check and the CPU-baseline leg of the benchmark may
 * load it.
 *
 * Units are lattice units throughout (dx = dt = 1, c = 1).  Everything is FP64.
 * Node index i = x + nx*(y + ny*z); PDF arrays are (q-1) x N with direction
 * alpha = 1..q-1 in slot alpha-1 (f_0 is never needed, Sec. 3.1 after Eq. 36).
 * Particle arrays are Np x 3 (2-D runs keep z components at zero; the 2-D angular
 * velocity is the z component of Omega).
 */
#ifndef IBLBM_REF_H
#define IBLBM_REF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct ref_ctx ref_ctx;

typedef struct {
  int32_t dim;            /* 2: D2Q9, 3: D3Q19 (Sec. 2.1, Eqs. 2-3) */
  int32_t n[3];           /* nodes per axis; n[2] = 1 in 2-D */
  double tau;             /* relaxation time, > 0.5 (Eq. 1) */
  double rho0;            /* constant fluid density of the incompressible model (Eq. 4) */
  double body_force[3];   /* uniform fluid body force added to the IB force (tests) */
  int32_t periodic[3];    /* 1: periodic axis, 0: walls (half-way bounce-back) */
  double wall_u[6][3];    /* wall velocity per face: -x,+x,-y,+y,-z,+z */
  int32_t delta;          /* 0: Peskin 4-point, 1: Roma 3-point (Sec. 2.2, Fig. 2b) */
  double drs;             /* solid shell thickness in lattice units (Eq. 13); 1 = DF/MDF */
  int32_t mdf_iters;      /* multi-direct-forcing passes per step (>= 1) */
  double gravity[3];      /* acceleration acting on particles */
  double zeta, eps_pp, E_pp;  /* Eq. 16 range and stiffness parameters */
  double cell_h;          /* cell size for the cell list; <= 0: chosen from Eqs. 49-50 */
  int32_t streaming;      /* 0: two arrays (Eqs. 17-18), 1: swap scheme (Sec. 3.3) */
  int32_t forcing;        /* 0: multi-direct forcing, 1: learned force + one correction pass */
  double slip_tol;        /* learned forcing: fall back to MDF when the slip rms exceeds it */
  int32_t fallback_iters; /* MDF passes used by the fallback */
  int32_t face_bc[6];     /* per face: 0 wall; 1 velocity (u = wall_u), 2 pressure (p =
                           * face_p) by non-equilibrium extrapolation (Sec. 6.1) */
  double face_p[6];
} ref_config;

/* ---- pure functions (pins and tests) ---------------------------------- */
int32_t ref_lattice(int32_t dim, int32_t* e /* q*3 */, double* w /* q */);
void ref_feq(int32_t dim, double rho0, double p, const double* u, double* feq /* q */);
void ref_guo_force(int32_t dim, double tau, const double* u, const double* f, double* F /* q */);
/* p by Eq. 6 and u* by Eq. 5 from q PDFs (slot 0 ignored) */
void ref_macro(int32_t dim, double rho0, const double* f /* q */, double* p, double* u /* 3 */);
double ref_phi(int32_t kind, double r);
/* Eq. 16 magnitude along the unit vector from j to i */
double ref_pair_force(double d, double D, double zeta, double c, double eps_pp, double E_pp);

/* Interpolation (Eq. 9 with Eq. 12) and spreading (Eq. 11 with Eq. 13) on a dense
 * velocity / force field u, g of layout d x N.  naive = 1 sums over every node
 * (Eqs. 43-44); naive = 0 visits only the delta-function support of each point
 * (Eqs. 47-48).  Out-of-domain stencil nodes on wall axes are skipped. */
void ref_ibm_interp(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t kind,
                    const double* u, int32_t nmk, const double* X /* nmk*3 */,
                    double* uhat /* nmk*3 */, int32_t naive);
void ref_ibm_spread(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t kind,
                    const double* F /* nmk*3 */, const double* dV /* nmk */, int32_t nmk,
                    const double* X /* nmk*3 */, double* g /* d*N, accumulated */, int32_t naive);

/* Pair searches on fixed positions.  Both return the number of pairs i<j with
 * |Xi-Xj|^2 < ((Di+Dj)/2 + zeta)^2, written sorted into ij (2*cap).
 * ref_half_search: Table 4 (i<j double loop).  ref_grid_search: Table 5 with the
 * one-centre-per-cell map of Eq. 51 (returns -1 if two centres share a cell). */
int64_t ref_half_search(int32_t dim, int32_t np, const double* X, const double* D, double zeta,
                        int32_t* ij, int64_t cap);
int64_t ref_grid_search(int32_t dim, const int32_t* n, int32_t np, const double* X, const double* D,
                        double zeta, double H, int32_t* ij, int64_t cap);

/* ---- particle coupling (Sec. 2.3): the pieces one step applies per particle ---- */
/* F_h = -sum F_k dV_k, T_h = -sum r_k x F_k dV_k over nmk points (r, F: nmk*3). */
void ref_particle_loads(int32_t nmk, const double* r, const double* F, const double* dV,
                        double* Fh /* 3 */, double* Th /* 3 */);
/* Momentum P and angular momentum L (3 each) of the fluid inside a particle of radius R
 * at Xc: sums of chi rho0 u and chi (x - Xc) x rho0 u with chi = clamp(R + 1/2 - |x - Xc|,
 * 0, 1); u is a dim x N field. */
void ref_interior_momentum(int32_t dim, const int32_t* n, const double* Xc, double R, double rho0,
                           const double* u, double* P, double* L);
/* One Newton-Euler step (Eqs. 14-15) of one particle; every pointer is 3 doubles.  The
 * hydrodynamic load H = F_h + (P - Pprev) enters as the mean of this and the previous
 * step's value (Hprev), likewise G = T_h + (L - Lprev) with Gprev; U by explicit Euler with
 * the buoyant weight (M - rho0 V) g, X by the trapezoid rule.  Pprev, Lprev, Hprev, Gprev,
 * X, U, Om are updated in place. */
void ref_newton_euler(int32_t dim, double M, double V, double I, double rho0, const double* g,
                      const double* Fh, const double* Th, const double* Fc, const double* P,
                      const double* L, double* Pprev, double* Lprev, double* Hprev, double* Gprev,
                      double* X, double* U, double* Om);
/* Eq. 16 pair forces of a pair list (i<j pairs, npairs) and the wall images (distance 2h to
 * the mirror centre, contact distance D_i) into Fc (np*3); c: c_i of Eq. 16 (np). */
void ref_pair_forces(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t np,
                     const double* X, const double* D, const double* c, double zeta,
                     double eps_pp, double E_pp, const int32_t* ij, int64_t npairs, double* Fc);
/* Gap feature of surface point Xk of particle p: distance to the nearest surface of a
 * pair partner or a wall plane, clamped to [0, zeta]. */
double ref_point_gap(int32_t dim, const int32_t* n, const int32_t* periodic, double zeta,
                     const double* Xk, int32_t p, const double* X, const double* D,
                     const int32_t* ij, int64_t npairs);

/* ---- the time-stepping context --------------------------------------- */
ref_ctx* ref_create(const ref_config* cfg);
void ref_destroy(ref_ctx* c);
/* f = f_eq(p, u) at every node (p: N, u: d*N; NULL means zero) */
int32_t ref_set_equilibrium(ref_ctx* c, const double* p, const double* u);
int32_t ref_set_pdfs(ref_ctx* c, const double* f /* (q-1)*N */);
int32_t ref_get_pdfs(const ref_ctx* c, double* f /* (q-1)*N */);
int32_t ref_add_particles(ref_ctx* c, int32_t n, const double* center, const double* diameter,
                          const double* density, const double* velocity, const double* omega,
                          int32_t markers_per_particle);
int32_t ref_step(ref_ctx* c, int32_t nsteps);
/* p and u* of the current PDFs (Eqs. 5-6) and the IB force of the last step */
int32_t ref_get_fields(const ref_ctx* c, double* p, double* u, double* force);
int32_t ref_get_particles(const ref_ctx* c, double* X, double* U, double* Om,
                          double* Fh, double* Th, double* Fc);
int32_t ref_get_markers(const ref_ctx* c, double* F /* nmk*3 */, double* r /* nmk*3 */,
                        int32_t* owner, double* dV);
int32_t ref_num_markers(const ref_ctx* c);
int64_t ref_get_pairs(const ref_ctx* c, int32_t* ij, int64_t cap);
int32_t ref_get_cells(const ref_ctx* c, int32_t* cell /* np*3 */, int32_t* dims /* 3 */,
                      double* h_eff /* 3 */);
/* mass sum over alpha>=1 and nodes; slip rms of the last step; truncated stencil nodes */
double ref_mass(const ref_ctx* c);
double ref_slip_rms(const ref_ctx* c);
int64_t ref_truncated(const ref_ctx* c);
int32_t ref_fallbacks(const ref_ctx* c);
/* the rms slip the last learned prediction left before its correction pass: the value the
 * fallback tolerance is tested against (0 before any learned step) */
double ref_judged_slip(const ref_ctx* c);

/* ---- learned forcing (MLP 10-64-64-3, tanh) --------------------------- */
#define REF_MLP_IN 10
#define REF_MLP_H 64
#define REF_MLP_OUT 3
#define REF_MLP_NPARAM (REF_MLP_IN*REF_MLP_H + REF_MLP_H + REF_MLP_H*REF_MLP_H + REF_MLP_H + REF_MLP_H*REF_MLP_OUT + REF_MLP_OUT)
/* params: W1[64][10], b1[64], W2[64][64], b2[64], W3[3][64], b3[3] (row-major, out x in)
 * norm: feature mean[10], feature std[10], then the mean[3] and std[3] of the change of
 * the converged force over the previous step's, F - F_prev (the network's target) */
void ref_mlp_forward(const double* params, int64_t n, const double* x /* n*10, normalised */,
                     double* y /* n*3 */);
/* the learned force of n points: F = F_prev + target mean + target std * y, with y the
 * network's output on the normalised features (feat n*10 raw, Fprev n*3, F n*3; the
 * components past dim are 0) */
void ref_mlp_predict(const double* params, const double* norm, int64_t n, int32_t dim,
                     const double* feat, const double* Fprev, double* F);
/* loss = mean over n*3 of (y - t)^2; grad (NPARAM) of that loss */
double ref_mlp_loss_grad(const double* params, int64_t n, const double* x, const double* t,
                         double* grad);
int32_t ref_set_mlp(ref_ctx* c, const double* params, const double* norm);
/* features of every marker at the start of the current step (pass-0 slip, previous-step
 * force, unit normal, neighbour gap) and the converged MDF force after the configured
 * number of passes, both un-normalised */
int32_t ref_capture_samples(ref_ctx* c, double* feat /* nmk*10 */, double* target /* nmk*3 */);

#ifdef __cplusplus
}
#endif
#endif

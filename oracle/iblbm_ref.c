/*
 * iblbm_ref.c -- plain FP64 CPU oracle of the IB-LBM time step (arXiv 2002.08855).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the package smoke check and the CPU
 * baseline of the benchmark may load this library.  It is written from the
 * paper's equations in their plain form, with no blocking or fusion:
 *   - fluid: incompressible SRT-LBGK, Eq. 1 with Eqs. 4-8 (Sec. 2.1), two arrays and
 *     a separate streaming pass (Eqs. 17-18, Sec. 3) with half-way bounce-back walls;
 *     the single-array swap scheme of Sec. 3.3 is available as a cross-check;
 *   - coupling: direct forcing Eqs. 9-13 (Sec. 2.2) repeated as multi-direct forcing,
 *     with the delta-function support visited point by point (Eqs. 47-48, Sec. 4) or
 *     over every node (Eqs. 43-44);
 *   - particles: Newton-Euler Eqs. 14-15 and the pair force Eq. 16 (Sec. 2.3); pairs
 *     from the i<j double loop of Table 4 (Sec. 5).
 * Readings where the paper is silent or garbled are stated next to the code.
 * Built with -ffp-contract=off so that every product and sum is rounded on its own.
 */
#include "iblbm_ref.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define CS2 (1.0 / 3.0) /* c_s^2 in lattice units: the factor 3 = 1/c_s^2 of Eqs. 21-36 */

/* Eq. 2: D2Q9 velocities, alpha = 0..8. */
static const int E9[9][3] = {{0, 0, 0},  {1, 0, 0},   {1, 1, 0},  {0, 1, 0}, {-1, 1, 0},
                             {-1, 0, 0}, {-1, -1, 0}, {0, -1, 0}, {1, -1, 0}};
/* Eq. 3: D3Q19 velocities, alpha = 0..18.  The printed third row has 18 entries; the
 * only completion that keeps rows 1-2 and the rule e_alpha = -e_{alpha-(q-1)/2}
 * inserts a 1 at alpha = 9, giving e_9 = (-1,0,1) and e_18 = (1,0,-1). */
static const int E19[19][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},  {0, 0, 1},   {1, 1, 0},
                               {-1, 1, 0}, {0, 1, 1},   {0, -1, 1}, {1, 0, 1},   {-1, 0, 1},
                               {-1, 0, 0}, {0, -1, 0},  {0, 0, -1}, {-1, -1, 0}, {1, -1, 0},
                               {0, -1, -1}, {0, 1, -1}, {-1, 0, -1}, {1, 0, -1}};

static int lat_q(int dim) { return dim == 2 ? 9 : 19; }
static const int* lat_e(int dim, int a) { return dim == 2 ? E9[a] : E19[a]; }
/* weights listed after Eq. 4 */
static double lat_w(int dim, int a) {
  if (dim == 2) {
    if (a == 0) return 4.0 / 9.0;
    return (a % 2 == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
  }
  if (a == 0) return 1.0 / 3.0;
  if ((a >= 1 && a <= 3) || (a >= 10 && a <= 12)) return 1.0 / 18.0;
  return 1.0 / 36.0;
}
/* e_alpha = -e_{alpha-(q-1)/2} for (q-1)/2 < alpha < q (Sec. 2.1) */
static int lat_opp(int dim, int a) {
  int h = (lat_q(dim) - 1) / 2;
  return a <= h ? a + h : a - h;
}

int32_t ref_lattice(int32_t dim, int32_t* e, double* w) {
  int q = lat_q(dim);
  for (int a = 0; a < q; a++) {
    for (int k = 0; k < 3; k++) e[3 * a + k] = lat_e(dim, a)[k];
    w[a] = lat_w(dim, a);
  }
  return q;
}

/* Eq. 4 with lambda_0 = (w_0 - 1)/c_s^2 and lambda_alpha = w_alpha/c_s^2. */
void ref_feq(int32_t dim, double rho0, double p, const double* u, double* feq) {
  int q = lat_q(dim);
  double uu = 0.0;
  for (int k = 0; k < dim; k++) uu += u[k] * u[k];
  for (int a = 0; a < q; a++) {
    const int* e = lat_e(dim, a);
    double w = lat_w(dim, a);
    double eu = 0.0;
    for (int k = 0; k < dim; k++) eu += e[k] * u[k];
    double lam = (a == 0) ? (w - 1.0) / CS2 : w / CS2;
    feq[a] = lam * p + rho0 * w * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq. 8 (Guo forcing term), dt = 1. */
void ref_guo_force(int32_t dim, double tau, const double* u, const double* f, double* F) {
  int q = lat_q(dim);
  for (int a = 0; a < q; a++) {
    const int* e = lat_e(dim, a);
    double w = lat_w(dim, a);
    double eu = 0.0;
    for (int k = 0; k < dim; k++) eu += e[k] * u[k];
    double s = 0.0;
    for (int k = 0; k < dim; k++) s += ((e[k] - u[k]) / CS2 + eu * e[k] / (CS2 * CS2)) * f[k];
    F[a] = (1.0 - 1.0 / (2.0 * tau)) * w * s;
  }
}

/* Eq. 5 (u* = sum e f / rho0; the printed form is the rho0 = 1 case) and Eq. 6. */
void ref_macro(int32_t dim, double rho0, const double* f, double* p, double* u) {
  int q = lat_q(dim);
  double s = 0.0;
  for (int k = 0; k < 3; k++) u[k] = 0.0;
  for (int a = 1; a < q; a++) {
    const int* e = lat_e(dim, a);
    s += f[a];
    for (int k = 0; k < dim; k++) u[k] += e[k] * f[a];
  }
  double uu = 0.0;
  for (int k = 0; k < dim; k++) {
    u[k] = u[k] / rho0;
    uu += u[k] * u[k];
  }
  double w0 = lat_w(dim, 0);
  *p = CS2 / (1.0 - w0) * (s - rho0 * w0 * uu / (2.0 * CS2));
}

/* Regularised delta functions of Fig. 2(b): the Peskin 4-point kernel and the
 * Roma-Peskin-Berger 3-point kernel, dh = 1. */
double ref_phi(int32_t kind, double r) {
  double a = fabs(r);
  if (kind == 0) {
    if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
  }
  if (a < 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a < 1.5) return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
  return 0.0;
}

/* Eq. 16 magnitude; D is the contact distance, zeta the range. */
double ref_pair_force(double d, double D, double zeta, double c, double eps_pp, double E_pp) {
  if (d >= D + zeta) return 0.0;
  double s = (d - D - zeta) / zeta;
  double F = c / eps_pp * (s * s);
  if (d < D) F = F + c / E_pp * ((D - d) / zeta);
  return F;
}

/* ------------------------------------------------------------------------ */
/* IBM on dense fields                                                      */

/* support of the kernel around X: first node and width */
static void support(int kind, double X, long* lo, int* width) {
  if (kind == 0) {
    *lo = (long)floor(X) - 1;
    *width = 4;
  } else {
    *lo = (long)floor(X + 0.5) - 1;
    *width = 3;
  }
}

/* node coordinate along an axis after the boundary rule: periodic wrap, or -1 when
 * the node lies outside a wall axis (such nodes are skipped) */
static long axis_node(long c, int n, int periodic) {
  if (c >= 0 && c < n) return c;
  if (!periodic) return -1;
  c %= n;
  if (c < 0) c += n;
  return c;
}

/* minimum-image offset of a node from a point along a periodic axis */
static double axis_offset(long c, double X, int n, int periodic) {
  double r = (double)c - X;
  if (periodic) r -= n * floor(r / n + 0.5);
  return r;
}

static long g_trunc_count; /* stencil nodes skipped on wall axes by the last call */

void ref_ibm_interp(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t kind,
                    const double* u, int32_t nmk, const double* X, double* uhat, int32_t naive) {
  long N = (long)n[0] * n[1] * n[2];
  g_trunc_count = 0;
  for (int k = 0; k < nmk; k++) {
    const double* Xk = X + 3 * k;
    double acc[3] = {0.0, 0.0, 0.0};
    if (naive) {
      /* Eq. 43: every node, x outer, then y, then z */
      for (long i = 0; i < n[0]; i++)
        for (long j = 0; j < n[1]; j++)
          for (long l = 0; l < n[2]; l++) {
            double w = ref_phi(kind, axis_offset(i, Xk[0], n[0], periodic[0])) *
                       ref_phi(kind, axis_offset(j, Xk[1], n[1], periodic[1]));
            if (dim == 3) w = w * ref_phi(kind, axis_offset(l, Xk[2], n[2], periodic[2]));
            long node = i + n[0] * (j + n[1] * l);
            for (int c = 0; c < dim; c++) acc[c] += u[c * N + node] * w;
          }
    } else {
      /* Eq. 47: only the kernel support around X_k, in the same order */
      long lo[3] = {0, 0, 0};
      int wd[3] = {1, 1, 1};
      for (int a = 0; a < dim; a++) support(kind, Xk[a], &lo[a], &wd[a]);
      for (int ii = 0; ii < wd[0]; ii++)
        for (int jj = 0; jj < wd[1]; jj++)
          for (int ll = 0; ll < wd[2]; ll++) {
            long ci = lo[0] + ii, cj = lo[1] + jj, cl = lo[2] + ll;
            long i = axis_node(ci, n[0], periodic[0]);
            long j = axis_node(cj, n[1], periodic[1]);
            long l = dim == 3 ? axis_node(cl, n[2], periodic[2]) : 0;
            if (i < 0 || j < 0 || l < 0) {
              g_trunc_count++;
              continue;
            }
            double w = ref_phi(kind, (double)ci - Xk[0]) * ref_phi(kind, (double)cj - Xk[1]);
            if (dim == 3) w = w * ref_phi(kind, (double)cl - Xk[2]);
            long node = i + n[0] * (j + n[1] * l);
            for (int c = 0; c < dim; c++) acc[c] += u[c * N + node] * w;
          }
    }
    for (int c = 0; c < 3; c++) uhat[3 * k + c] = acc[c];
  }
}

void ref_ibm_spread(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t kind,
                    const double* F, const double* dV, int32_t nmk, const double* X, double* g,
                    int32_t naive) {
  long N = (long)n[0] * n[1] * n[2];
  if (naive) {
    /* Eq. 44: at every node, the sum over points in ascending order */
    for (long i = 0; i < n[0]; i++)
      for (long j = 0; j < n[1]; j++)
        for (long l = 0; l < n[2]; l++) {
          long node = i + n[0] * (j + n[1] * l);
          for (int k = 0; k < nmk; k++) {
            const double* Xk = X + 3 * k;
            double w = ref_phi(kind, axis_offset(i, Xk[0], n[0], periodic[0])) *
                       ref_phi(kind, axis_offset(j, Xk[1], n[1], periodic[1]));
            if (dim == 3) w = w * ref_phi(kind, axis_offset(l, Xk[2], n[2], periodic[2]));
            for (int c = 0; c < dim; c++) g[c * N + node] += F[3 * k + c] * w * dV[k];
          }
        }
    return;
  }
  /* Eq. 48: point by point, each point adds into its kernel support */
  for (int k = 0; k < nmk; k++) {
    const double* Xk = X + 3 * k;
    long lo[3] = {0, 0, 0};
    int wd[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) support(kind, Xk[a], &lo[a], &wd[a]);
    for (int ii = 0; ii < wd[0]; ii++)
      for (int jj = 0; jj < wd[1]; jj++)
        for (int ll = 0; ll < wd[2]; ll++) {
          long ci = lo[0] + ii, cj = lo[1] + jj, cl = lo[2] + ll;
          long i = axis_node(ci, n[0], periodic[0]);
          long j = axis_node(cj, n[1], periodic[1]);
          long l = dim == 3 ? axis_node(cl, n[2], periodic[2]) : 0;
          if (i < 0 || j < 0 || l < 0) continue;
          double w = ref_phi(kind, (double)ci - Xk[0]) * ref_phi(kind, (double)cj - Xk[1]);
          if (dim == 3) w = w * ref_phi(kind, (double)cl - Xk[2]);
          long node = i + n[0] * (j + n[1] * l);
          for (int c = 0; c < dim; c++) g[c * N + node] += F[3 * k + c] * w * dV[k];
        }
  }
}

/* ------------------------------------------------------------------------ */
/* pair searches                                                            */

static int pair_cmp(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

/* the pair test: squared distance, each square and sum rounded separately */
static int pair_within(int dim, const double* Xi, const double* Xj, double Di, double Dj,
                       double zeta) {
  double d2 = 0.0;
  for (int k = 0; k < dim; k++) {
    double dx = Xi[k] - Xj[k];
    d2 = d2 + dx * dx;
  }
  double s = 0.5 * (Di + Dj) + zeta;
  return d2 < s * s;
}

int64_t ref_half_search(int32_t dim, int32_t np, const double* X, const double* D, double zeta,
                        int32_t* ij, int64_t cap) {
  int64_t m = 0;
  for (int i = 0; i < np; i++)
    for (int j = i + 1; j < np; j++)
      if (pair_within(dim, X + 3 * i, X + 3 * j, D[i], D[j], zeta)) {
        if (m < cap) {
          ij[2 * m] = i;
          ij[2 * m + 1] = j;
        }
        m++;
      }
  return m;
}

int64_t ref_grid_search(int32_t dim, const int32_t* n, int32_t np, const double* X, const double* D,
                        double zeta, double H, int32_t* ij, int64_t cap) {
  /* Table 5: cells of size H (Eqs. 49-50) hold at most one centre (Eq. 51); every
   * particle scans the 5^d cells around its own and is then removed from the map. */
  int nc[3] = {1, 1, 1};
  for (int a = 0; a < dim; a++) nc[a] = (int)floor((n[a]) / H) + 1;
  long ncell = (long)nc[0] * nc[1] * nc[2];
  int* value = (int*)malloc(sizeof(int) * ncell);
  int* cell = (int*)malloc(sizeof(int) * 3 * (np > 0 ? np : 1));
  for (long c = 0; c < ncell; c++) value[c] = -1;
  int64_t m = 0;
  for (int k = 0; k < np; k++) {
    for (int a = 0; a < 3; a++) cell[3 * k + a] = 0;
    for (int a = 0; a < dim; a++) {
      int c = (int)floor((X[3 * k + a] + 0.5) / H);
      if (c < 0) c = 0;
      if (c >= nc[a]) c = nc[a] - 1;
      cell[3 * k + a] = c;
    }
    long id = cell[3 * k] + (long)nc[0] * (cell[3 * k + 1] + (long)nc[1] * cell[3 * k + 2]);
    if (value[id] != -1) {
      free(value);
      free(cell);
      return -1;
    }
    value[id] = k;
  }
  for (int k = 0; k < np; k++) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
      lo[a] = a < dim ? cell[3 * k + a] - 2 : 0;
      hi[a] = a < dim ? cell[3 * k + a] + 2 : 0;
      if (lo[a] < 0) lo[a] = 0;
      if (hi[a] > nc[a] - 1) hi[a] = nc[a] - 1;
    }
    for (int cx = lo[0]; cx <= hi[0]; cx++)
      for (int cy = lo[1]; cy <= hi[1]; cy++)
        for (int cz = lo[2]; cz <= hi[2]; cz++) {
          int j = value[cx + (long)nc[0] * (cy + (long)nc[1] * cz)];
          if (j == -1 || j == k) continue;
          if (pair_within(dim, X + 3 * k, X + 3 * j, D[k], D[j], zeta)) {
            if (m < cap) {
              ij[2 * m] = k < j ? k : j;
              ij[2 * m + 1] = k < j ? j : k;
            }
            m++;
          }
        }
    long id = cell[3 * k] + (long)nc[0] * (cell[3 * k + 1] + (long)nc[1] * cell[3 * k + 2]);
    value[id] = -1;
  }
  free(value);
  free(cell);
  if (m <= cap) qsort(ij, (size_t)m, 2 * sizeof(int32_t), pair_cmp);
  return m;
}

/* ------------------------------------------------------------------------ */
/* time-stepping context                                                    */

struct ref_ctx {
  ref_config cfg;
  int dim, q;
  long N;
  double *f, *ft;          /* (q-1) x N */
  double *ustar, *p;       /* u* (d x N), p (N) of the current step */
  double *fib, *um, *g;    /* IB force, MDF working velocity, per-pass spread (d x N) */
  /* particles */
  int np, capp;
  double *X, *U, *Om, *D, *rho, *M, *V, *I, *Fh, *Th, *Fc, *cbuoy;
  double *Pin, *Lin, *Pprev, *Lprev; /* fluid momentum inside each particle: now, last step */
  double *Hprev, *Gprev; /* hydrodynamic force and torque of the previous step */
  int *mstart, *mcount;
  /* markers */
  int nmk, capm;
  int* mown;
  double *mr, *mdV, *mF, *mFprev, *mdF, *mX, *mUb, *muh;
  /* cell list and pairs of the positions at the start of the step */
  double H;
  int nc[3];
  double invh[3];
  int32_t* pairs;
  int64_t npairs, cappairs;
  long truncated;
  double slip;
  double judged;  /* the slip the last learned prediction left (its judge) */
  /* learned forcing */
  int has_mlp;
  double mlp[REF_MLP_NPARAM];
  double norm[2 * REF_MLP_IN + 2 * REF_MLP_OUT];
  int fallbacks;
};

static void* xcalloc(size_t n, size_t s) {
  void* p = calloc(n ? n : 1, s);
  if (!p) {
    fprintf(stderr, "iblbm_ref: out of memory\n");
    abort();
  }
  return p;
}

/* Extrapolated faces (face_bc 1 or 2) must all lie on one non-periodic axis with at
 * least 3 nodes, so that a boundary node's inward neighbour is never a boundary node. */
static int faces_ok(const ref_config* cfg) {
  int axis = -1;
  for (int f = 0; f < 6; f++) {
    if (cfg->face_bc[f] < 0 || cfg->face_bc[f] > 2) return 0;
    if (cfg->face_bc[f] == 0) continue;
    int a = f / 2;
    if (a >= cfg->dim || cfg->periodic[a] || cfg->n[a] < 3) return 0;
    if (axis >= 0 && axis != a) return 0;
    axis = a;
  }
  return 1;
}

ref_ctx* ref_create(const ref_config* cfg) {
  if (cfg->dim != 2 && cfg->dim != 3) return NULL;
  if (!(cfg->tau > 0.5)) return NULL;
  if (!faces_ok(cfg)) return NULL;
  ref_ctx* c = (ref_ctx*)xcalloc(1, sizeof(ref_ctx));
  c->cfg = *cfg;
  c->dim = cfg->dim;
  c->q = lat_q(cfg->dim);
  if (c->dim == 2) c->cfg.n[2] = 1;
  c->N = (long)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  size_t Q = (size_t)(c->q - 1) * c->N;
  c->f = (double*)xcalloc(Q, sizeof(double));
  c->ft = (double*)xcalloc(Q, sizeof(double));
  c->ustar = (double*)xcalloc((size_t)3 * c->N, sizeof(double));
  c->p = (double*)xcalloc((size_t)c->N, sizeof(double));
  c->fib = (double*)xcalloc((size_t)3 * c->N, sizeof(double));
  c->um = (double*)xcalloc((size_t)3 * c->N, sizeof(double));
  c->g = (double*)xcalloc((size_t)3 * c->N, sizeof(double));
  return c;
}

static void free_particles(ref_ctx* c) {
  double** arrs[] = {&c->X, &c->U, &c->Om, &c->D, &c->rho, &c->M, &c->V, &c->I,
                     &c->Fh, &c->Th, &c->Fc, &c->cbuoy, &c->Pin, &c->Lin, &c->Pprev, &c->Lprev, &c->Hprev, &c->Gprev};
  for (size_t i = 0; i < sizeof(arrs) / sizeof(arrs[0]); i++) free(*arrs[i]);
  free(c->mstart);
  free(c->mcount);
  double** marr[] = {&c->mr, &c->mdV, &c->mF, &c->mFprev, &c->mdF, &c->mX, &c->mUb, &c->muh};
  for (size_t i = 0; i < sizeof(marr) / sizeof(marr[0]); i++) free(*marr[i]);
  free(c->mown);
  free(c->pairs);
}

void ref_destroy(ref_ctx* c) {
  if (!c) return;
  free(c->f);
  free(c->ft);
  free(c->ustar);
  free(c->p);
  free(c->fib);
  free(c->um);
  free(c->g);
  free_particles(c);
  free(c);
}

int32_t ref_set_equilibrium(ref_ctx* c, const double* p, const double* u) {
  long N = c->N;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    double uu[3] = {0, 0, 0}, feq[19];
    double pp = p ? p[i] : 0.0;
    for (int k = 0; k < c->dim; k++) uu[k] = u ? u[k * N + i] : 0.0;
    ref_feq(c->dim, c->cfg.rho0, pp, uu, feq);
    for (int a = 1; a < c->q; a++) c->f[(a - 1) * N + i] = feq[a];
  }
  return 0;
}

int32_t ref_set_pdfs(ref_ctx* c, const double* f) {
  memcpy(c->f, f, sizeof(double) * (size_t)(c->q - 1) * c->N);
  return 0;
}

int32_t ref_get_pdfs(const ref_ctx* c, double* f) {
  memcpy(f, c->f, sizeof(double) * (size_t)(c->q - 1) * c->N);
  return 0;
}

/* ---- particles ---------------------------------------------------------- */

static void interior_momentum(ref_ctx* c, const double* uvel, double* P, double* L);

/* Lagrangian points on the particle surface (the paper places them uniformly):
 * 2-D, equal angles on the circle; 3-D, the Fibonacci (golden-angle) sphere. */
static void marker_offset(int dim, double R, int k, int nl, double* r) {
  const double pi = 3.14159265358979323846;
  if (dim == 2) {
    double th = 2.0 * pi * k / nl;
    r[0] = R * cos(th);
    r[1] = R * sin(th);
    r[2] = 0.0;
  } else {
    double z = 1.0 - (2.0 * k + 1.0) / nl;
    double ph = k * (pi * (3.0 - sqrt(5.0)));
    double s = sqrt(1.0 - z * z);
    r[0] = R * (s * cos(ph));
    r[1] = R * (s * sin(ph));
    r[2] = R * z;
  }
}

static void cells_setup(ref_ctx* c) {
  double dmax = 0.0, dmin = 1e300;
  for (int i = 0; i < c->np; i++) {
    if (c->D[i] > dmax) dmax = c->D[i];
    if (c->D[i] < dmin) dmin = c->D[i];
  }
  double H = c->cfg.cell_h;
  if (!(H > 0.0)) {
    /* Eq. 50 (2H > D + zeta) and Eq. 49 (cell diagonal < D) */
    double lo = 0.5 * (dmax + c->cfg.zeta);
    double hi = dmin / sqrt((double)c->dim);
    H = lo < hi ? 0.5 * (lo + hi) : 1.05 * lo;
  }
  c->H = H;
  for (int a = 0; a < 3; a++) {
    c->nc[a] = 1;
    c->invh[a] = 0.0;
  }
  for (int a = 0; a < c->dim; a++) {
    int m = (int)floor(c->cfg.n[a] / H);
    if (m < 1) m = 1;
    c->nc[a] = m;
    c->invh[a] = (double)m / (double)c->cfg.n[a];
  }
}

static void find_pairs(ref_ctx* c) {
  int64_t m = ref_half_search(c->dim, c->np, c->X, c->D, c->cfg.zeta, c->pairs, c->cappairs);
  if (m > c->cappairs) {
    free(c->pairs);
    c->cappairs = 2 * m;
    c->pairs = (int32_t*)xcalloc((size_t)(2 * c->cappairs), sizeof(int32_t));
    m = ref_half_search(c->dim, c->np, c->X, c->D, c->cfg.zeta, c->pairs, c->cappairs);
  }
  c->npairs = m;
}

static void* xrealloc(void* p, size_t bytes) {
  void* q = realloc(p, bytes ? bytes : 1);
  if (!q) {
    fprintf(stderr, "iblbm_ref: out of memory\n");
    abort();
  }
  return q;
}
#define GROW(ptr, type, n) ptr = (type*)xrealloc(ptr, sizeof(type) * (size_t)(n))

int32_t ref_add_particles(ref_ctx* c, int32_t n, const double* center, const double* diameter,
                          const double* density, const double* velocity, const double* omega,
                          int32_t markers_per_particle) {
  const double pi = 3.14159265358979323846;
  int dim = c->dim;
  if (n < 0) return 1;
  for (int a = 0; a < 3; a++)
    if (c->cfg.periodic[a] && n > 0) return 1; /* particles need a closed cavity */
  for (int i = 0; i < n; i++) {
    double R = 0.5 * diameter[i];
    if (!(diameter[i] > 0.0) || !(density[i] > 0.0)) return 1;
    for (int a = 0; a < dim; a++)
      if (center[3 * i + a] - R < -0.5 || center[3 * i + a] + R > c->cfg.n[a] - 0.5) return 1;
    for (int j = 0; j < c->np + i; j++) {
      const double* Xj = j < c->np ? c->X + 3 * j : center + 3 * (j - c->np);
      double Dj = j < c->np ? c->D[j] : diameter[j - c->np];
      double d2 = 0.0;
      for (int a = 0; a < dim; a++) {
        double dx = center[3 * i + a] - Xj[a];
        d2 = d2 + dx * dx;
      }
      double s = 0.5 * (diameter[i] + Dj);
      if (d2 < s * s) return 1;
    }
  }
  int np = c->np + n;
  GROW(c->X, double, 3 * np);
  GROW(c->U, double, 3 * np);
  GROW(c->Om, double, 3 * np);
  GROW(c->Fh, double, 3 * np);
  GROW(c->Th, double, 3 * np);
  GROW(c->Fc, double, 3 * np);
  GROW(c->Pin, double, 3 * np);
  GROW(c->Lin, double, 3 * np);
  GROW(c->Pprev, double, 3 * np);
  GROW(c->Lprev, double, 3 * np);
  GROW(c->Hprev, double, 3 * np);
  GROW(c->Gprev, double, 3 * np);
  GROW(c->D, double, np);
  GROW(c->rho, double, np);
  GROW(c->M, double, np);
  GROW(c->V, double, np);
  GROW(c->I, double, np);
  GROW(c->cbuoy, double, np);
  GROW(c->mstart, int, np);
  GROW(c->mcount, int, np);
  double gmag = 0.0;
  for (int a = 0; a < 3; a++) gmag += c->cfg.gravity[a] * c->cfg.gravity[a];
  gmag = sqrt(gmag);
  int nmk = c->nmk;
  for (int i = 0; i < n; i++) {
    int p = c->np + i;
    double D = diameter[i], R = 0.5 * D;
    for (int a = 0; a < 3; a++) {
      c->X[3 * p + a] = center[3 * i + a];
      c->U[3 * p + a] = velocity ? velocity[3 * i + a] : 0.0;
      c->Om[3 * p + a] = omega ? omega[3 * i + a] : 0.0;
      c->Fh[3 * p + a] = c->Th[3 * p + a] = c->Fc[3 * p + a] = 0.0;
      c->Hprev[3 * p + a] = c->Gprev[3 * p + a] = 0.0;
    }
    if (dim == 2) {
      c->X[3 * p + 2] = c->U[3 * p + 2] = 0.0;
      c->Om[3 * p + 0] = c->Om[3 * p + 1] = 0.0;
    }
    c->D[p] = D;
    c->rho[p] = density[i];
    /* 2-D: a disk per unit depth; 3-D: a sphere */
    c->V[p] = dim == 2 ? pi * R * R : 4.0 / 3.0 * pi * R * R * R;
    c->M[p] = density[i] * c->V[p];
    c->I[p] = dim == 2 ? 0.5 * c->M[p] * R * R : 0.4 * c->M[p] * R * R;
    /* c_ij of Eq. 16 is the buoyant weight of the body */
    c->cbuoy[p] = (density[i] - c->cfg.rho0) * c->V[p] * gmag;
    int nl = markers_per_particle > 0 ? markers_per_particle
                                      : (int)floor((dim == 2 ? pi * D : pi * D * D) + 0.5);
    c->mstart[p] = nmk;
    c->mcount[p] = nl;
    nmk += nl;
  }
  GROW(c->mown, int, nmk);
  GROW(c->mr, double, 3 * nmk);
  GROW(c->mdV, double, nmk);
  GROW(c->mF, double, 3 * nmk);
  GROW(c->mFprev, double, 3 * nmk);
  GROW(c->mdF, double, 3 * nmk);
  GROW(c->mX, double, 3 * nmk);
  GROW(c->mUb, double, 3 * nmk);
  GROW(c->muh, double, 3 * nmk);
  for (int i = 0; i < n; i++) {
    int p = c->np + i;
    double D = c->D[p], R = 0.5 * D;
    int nl = c->mcount[p];
    /* Eq. 13: the point carries drs * ds (2-D arc length) or drs * dA (3-D area) */
    double ds = dim == 2 ? pi * D / nl : pi * D * D / nl;
    for (int k = 0; k < nl; k++) {
      int m = c->mstart[p] + k;
      c->mown[m] = p;
      marker_offset(dim, R, k, nl, c->mr + 3 * m);
      c->mdV[m] = c->cfg.drs * ds;
      for (int a = 0; a < 3; a++) c->mF[3 * m + a] = c->mFprev[3 * m + a] = 0.0;
    }
  }
  int np_old = c->np;
  c->np = np;
  c->nmk = nmk;
  cells_setup(c);
  find_pairs(c);
  /* interior fluid momentum of the new particles in the current fluid */
  {
    long N = c->N;
    for (long i = 0; i < N; i++) {
      double fl[19], pp, uu[3];
      fl[0] = 0.0;
      for (int a = 1; a < c->q; a++) fl[a] = c->f[(a - 1) * N + i];
      ref_macro(dim, c->cfg.rho0, fl, &pp, uu);
      for (int a = 0; a < dim; a++) c->g[a * N + i] = uu[a];
    }
    interior_momentum(c, c->g, c->Pin, c->Lin);
    for (int p = np_old; p < np; p++)
      for (int a = 0; a < 3; a++) {
        c->Pprev[3 * p + a] = c->Pin[3 * p + a];
        c->Lprev[3 * p + a] = c->Lin[3 * p + a];
      }
  }
  return 0;
}

/* ---- one time step ------------------------------------------------------ */

static void markers_update(ref_ctx* c) {
  /* X_k = X_c + r_k and U_b = U_c + Omega x r_k (points translate with the body) */
  for (int m = 0; m < c->nmk; m++) {
    int p = c->mown[m];
    const double* r = c->mr + 3 * m;
    const double* W = c->Om + 3 * p;
    double wxr[3] = {W[1] * r[2] - W[2] * r[1], W[2] * r[0] - W[0] * r[2],
                     W[0] * r[1] - W[1] * r[0]};
    for (int a = 0; a < 3; a++) {
      c->mX[3 * m + a] = c->X[3 * p + a] + r[a];
      c->mUb[3 * m + a] = c->U[3 * p + a] + wxr[a];
    }
    if (c->dim == 2) c->mX[3 * m + 2] = c->mUb[3 * m + 2] = 0.0;
  }
}

static long count_truncated(ref_ctx* c) {
  long t = 0;
  for (int m = 0; m < c->nmk; m++) {
    long lo[3] = {0, 0, 0};
    int wd[3] = {1, 1, 1};
    for (int a = 0; a < c->dim; a++) support(c->cfg.delta, c->mX[3 * m + a], &lo[a], &wd[a]);
    for (int ii = 0; ii < wd[0]; ii++)
      for (int jj = 0; jj < wd[1]; jj++)
        for (int ll = 0; ll < wd[2]; ll++) {
          long i = axis_node(lo[0] + ii, c->cfg.n[0], c->cfg.periodic[0]);
          long j = axis_node(lo[1] + jj, c->cfg.n[1], c->cfg.periodic[1]);
          long l = c->dim == 3 ? axis_node(lo[2] + ll, c->cfg.n[2], c->cfg.periodic[2]) : 0;
          if (i < 0 || j < 0 || l < 0) t++;
        }
  }
  return t;
}

/* one direct-forcing pass: interpolate the working velocity (Eq. 9), force (Eq. 10),
 * spread (Eq. 11), then f_IB += g and u += g/(2 rho0) (Eq. 7 applied to the increment) */
static void forcing_pass(ref_ctx* c, const double* Fset) {
  const ref_config* k = &c->cfg;
  long N = c->N;
  int d = c->dim;
  if (Fset) {
    for (int m = 0; m < 3 * c->nmk; m++) c->mdF[m] = Fset[m];
  } else {
    ref_ibm_interp(d, k->n, k->periodic, k->delta, c->um, c->nmk, c->mX, c->muh, 0);
    for (int m = 0; m < c->nmk; m++)
      for (int a = 0; a < 3; a++)
        c->mdF[3 * m + a] = a < d ? 2.0 * k->rho0 * (c->mUb[3 * m + a] - c->muh[3 * m + a]) : 0.0;
  }
  for (int m = 0; m < 3 * c->nmk; m++) c->mF[m] += c->mdF[m];
  memset(c->g, 0, sizeof(double) * (size_t)d * N);
  ref_ibm_spread(d, k->n, k->periodic, k->delta, c->mdF, c->mdV, c->nmk, c->mX, c->g, 0);
  for (long i = 0; i < (long)d * N; i++) {
    c->fib[i] += c->g[i];
    c->um[i] += c->g[i] / (2.0 * k->rho0);
  }
}

static double slip_rms(ref_ctx* c) {
  const ref_config* k = &c->cfg;
  if (c->nmk == 0) return 0.0;
  ref_ibm_interp(c->dim, k->n, k->periodic, k->delta, c->um, c->nmk, c->mX, c->muh, 0);
  double s = 0.0;
  for (int m = 0; m < c->nmk; m++)
    for (int a = 0; a < c->dim; a++) {
      double e = c->mUb[3 * m + a] - c->muh[3 * m + a];
      s += e * e;
    }
  return sqrt(s / c->nmk);
}

static void mdf(ref_ctx* c, int passes) {
  long N = c->N;
  memcpy(c->um, c->ustar, sizeof(double) * 3 * (size_t)N);
  memset(c->fib, 0, sizeof(double) * 3 * (size_t)N);
  for (int m = 0; m < 3 * c->nmk; m++) c->mF[m] = 0.0;
  for (int it = 0; it < passes; it++) forcing_pass(c, NULL);
}

static void features(ref_ctx* c, double* feat);
static void mlp_apply(ref_ctx* c, const double* feat, double* Fout);

static void ibm_stage(ref_ctx* c) {
  markers_update(c);
  c->truncated += count_truncated(c);
  if (c->cfg.forcing == 1 && c->has_mlp) {
    /* learned force, then one plain correction pass; MDF as fallback */
    double* feat = (double*)xcalloc((size_t)REF_MLP_IN * c->nmk, sizeof(double));
    double* Fp = (double*)xcalloc((size_t)3 * c->nmk, sizeof(double));
    features(c, feat);
    mlp_apply(c, feat, Fp);
    long N = c->N;
    memcpy(c->um, c->ustar, sizeof(double) * 3 * (size_t)N);
    memset(c->fib, 0, sizeof(double) * 3 * (size_t)N);
    for (int m = 0; m < 3 * c->nmk; m++) c->mF[m] = 0.0;
    forcing_pass(c, Fp);
    /* the judge: the slip the prediction leaves, which the correction pass then corrects */
    double judged = slip_rms(c);
    c->judged = judged;
    forcing_pass(c, NULL);
    c->slip = slip_rms(c);
    if (!(judged <= c->cfg.slip_tol)) {
      mdf(c, c->cfg.fallback_iters);
      c->slip = slip_rms(c);
      c->fallbacks++;
    }
    free(feat);
    free(Fp);
  } else {
    mdf(c, c->cfg.mdf_iters);
    c->slip = slip_rms(c);
  }
}

static void collide(ref_ctx* c, double* out) {
  const ref_config* k = &c->cfg;
  long N = c->N;
  int q = c->q, d = c->dim;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    double ff[3] = {0, 0, 0}, u[3] = {0, 0, 0}, feq[19], F[19];
    for (int a = 0; a < d; a++) {
      ff[a] = c->fib[a * N + i] + k->body_force[a];
      u[a] = c->ustar[a * N + i] + ff[a] / (2.0 * k->rho0); /* Eq. 7 */
    }
    ref_feq(d, k->rho0, c->p[i], u, feq);
    ref_guo_force(d, k->tau, u, ff, F);
    for (int a = 1; a < q; a++) {
      double fa = c->f[(a - 1) * N + i];
      out[(a - 1) * N + i] = fa - (fa - feq[a]) / k->tau + F[a]; /* Eq. 1 / Eq. 17 */
    }
  }
}

/* neighbour of node (x,y,z) along e_alpha: returns the node index, or -1 when the
 * link leaves through a wall; *face is the first wall face crossed (axis order) */
static long neighbour(const ref_ctx* c, long x, long y, long z, const int* e, int* face) {
  long cc[3] = {x + e[0], y + e[1], z + e[2]};
  *face = -1;
  for (int a = 0; a < c->dim; a++) {
    long v = axis_node(cc[a], c->cfg.n[a], c->cfg.periodic[a]);
    if (v < 0) {
      if (*face < 0) *face = 2 * a + (cc[a] >= c->cfg.n[a] ? 1 : 0);
    } else {
      cc[a] = v;
    }
  }
  if (*face >= 0) return -1;
  return cc[0] + c->cfg.n[0] * (cc[1] + (long)c->cfg.n[1] * cc[2]);
}

/* half-way bounce-back with a moving wall: -2 w rho0 (e . u_wall)/c_s^2 */
static double wall_term(const ref_ctx* c, int a, int face) {
  const int* e = lat_e(c->dim, a);
  double eu = 0.0;
  for (int k = 0; k < c->dim; k++) eu += e[k] * c->cfg.wall_u[face][k];
  return 2.0 * lat_w(c->dim, a) * c->cfg.rho0 * eu / CS2;
}

static void stream_two_array(ref_ctx* c, const double* post, double* dst) {
  long N = c->N;
  int q = c->q;
  const int* n = c->cfg.n;
#pragma omp parallel for schedule(static)
  for (long z = 0; z < n[2]; z++)
    for (long y = 0; y < n[1]; y++)
      for (long x = 0; x < n[0]; x++) {
        long i = x + n[0] * (y + (long)n[1] * z);
        for (int a = 1; a < q; a++) {
          int face;
          long j = neighbour(c, x, y, z, lat_e(c->dim, a), &face);
          if (j >= 0)
            dst[(a - 1) * N + j] = post[(a - 1) * N + i]; /* Eq. 18 */
          else
            dst[(lat_opp(c->dim, a) - 1) * N + i] = post[(a - 1) * N + i] - wall_term(c, a, face);
        }
      }
}

static void stream_swap(ref_ctx* c) {
  /* Sec. 3.3: after collision, exchange alpha <-> opposite at every node, then
   * exchange slot opp(alpha) at x with slot alpha at x + e_alpha for the first half
   * of the directions when that neighbour exists.  Links that leave through a wall
   * keep their value at the node (half-way bounce-back); the moving-wall term is
   * applied to those slots afterwards. */
  long N = c->N;
  int q = c->q, h = (q - 1) / 2;
  const int* n = c->cfg.n;
  double* f = c->f;
  for (long i = 0; i < N; i++)
    for (int a = 1; a <= h; a++) {
      int b = lat_opp(c->dim, a);
      double t = f[(a - 1) * N + i];
      f[(a - 1) * N + i] = f[(b - 1) * N + i];
      f[(b - 1) * N + i] = t;
    }
  for (long z = 0; z < n[2]; z++)
    for (long y = 0; y < n[1]; y++)
      for (long x = 0; x < n[0]; x++) {
        long i = x + n[0] * (y + (long)n[1] * z);
        for (int a = 1; a <= h; a++) {
          int face, b = lat_opp(c->dim, a);
          long j = neighbour(c, x, y, z, lat_e(c->dim, a), &face);
          if (j < 0) continue;
          double t = f[(b - 1) * N + i];
          f[(b - 1) * N + i] = f[(a - 1) * N + j];
          f[(a - 1) * N + j] = t;
        }
      }
  for (long z = 0; z < n[2]; z++)
    for (long y = 0; y < n[1]; y++)
      for (long x = 0; x < n[0]; x++) {
        long i = x + n[0] * (y + (long)n[1] * z);
        for (int a = 1; a < q; a++) {
          int face;
          long j = neighbour(c, x, y, z, lat_e(c->dim, a), &face);
          if (j < 0) {
            int b = lat_opp(c->dim, a);
            f[(b - 1) * N + i] = f[(b - 1) * N + i] - wall_term(c, a, face);
          }
        }
      }
}

/* Sec. 6.1 boundaries by non-equilibrium extrapolation (the paper's ref. [48]): on the
 * node layer of an inflow or outflow face, after streaming, every population becomes
 * f_eq(p_b, u_b) + (f - f_eq(p_f, u_f)) at the next node inward x_f.  A velocity face
 * prescribes u_b (its wall_u) and takes p_b = p_f; a pressure face prescribes p_b (its
 * face_p) and takes u_b = u_f.  The inward nodes are never boundary nodes (faces_ok), so
 * the nodes can be updated in any order. */
static void apply_face_bc(ref_ctx* c) {
  long N = c->N;
  int q = c->q, d = c->dim;
  const int* n = c->cfg.n;
  for (int face = 0; face < 6; face++) {
    int kind = c->cfg.face_bc[face];
    if (kind == 0) continue;
    int ax = face / 2, hi = face % 2;
    long layer = hi ? n[ax] - 1 : 0, step = hi ? -1 : 1;
    for (long z = 0; z < n[2]; z++)
      for (long y = 0; y < n[1]; y++)
        for (long x = 0; x < n[0]; x++) {
          long cb[3] = {x, y, z};
          if (cb[ax] != layer) continue;
          long cf[3] = {x, y, z};
          cf[ax] += step;
          long ib = cb[0] + n[0] * (cb[1] + (long)n[1] * cb[2]);
          long jf = cf[0] + n[0] * (cf[1] + (long)n[1] * cf[2]);
          double ff[19], pf, uf[3], pb, ub[3], eqb[19], eqf[19];
          ff[0] = 0.0;
          for (int a = 1; a < q; a++) ff[a] = c->f[(a - 1) * N + jf];
          ref_macro(d, c->cfg.rho0, ff, &pf, uf);
          for (int k = 0; k < 3; k++) ub[k] = kind == 1 ? (k < d ? c->cfg.wall_u[face][k] : 0.0) : uf[k];
          pb = kind == 1 ? pf : c->cfg.face_p[face];
          ref_feq(d, c->cfg.rho0, pb, ub, eqb);
          ref_feq(d, c->cfg.rho0, pf, uf, eqf);
          for (int a = 1; a < q; a++) c->f[(a - 1) * N + ib] = eqb[a] + (ff[a] - eqf[a]);
        }
  }
}

/* Hydrodynamic load of one particle (Sec. 2.3, the reaction of the IB force of Eqs. 10
 * and 13): F_h = -sum_k F_k dV_k and T_h = -sum_k r_k x (F_k dV_k) over its points k in
 * ascending order; r_k and F_k are nmk x 3. */
void ref_particle_loads(int32_t nmk, const double* r, const double* Fk, const double* dV,
                        double* Fh, double* Th) {
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  for (int m = 0; m < nmk; m++) {
    const double* rk = r + 3 * m;
    const double* f = Fk + 3 * m;
    double Fd[3] = {f[0] * dV[m], f[1] * dV[m], f[2] * dV[m]};
    double t[3] = {rk[1] * Fd[2] - rk[2] * Fd[1], rk[2] * Fd[0] - rk[0] * Fd[2],
                   rk[0] * Fd[1] - rk[1] * Fd[0]};
    for (int a = 0; a < 3; a++) {
      F[a] = F[a] - Fd[a];
      T[a] = T[a] - t[a];
    }
  }
  for (int a = 0; a < 3; a++) {
    Fh[a] = F[a];
    Th[a] = T[a];
  }
}

static void particle_loads(ref_ctx* c) {
  for (int p = 0; p < c->np; p++) {
    int m0 = c->mstart[p];
    ref_particle_loads(c->mcount[p], c->mr + 3 * m0, c->mF + 3 * m0, c->mdV + m0, c->Fh + 3 * p,
                       c->Th + 3 * p);
  }
}

/* Pair forces F_c (Eq. 16) of np particles from their pair list (Table 4: each pair i<j
 * once, Newton's third law for the partner), then the walls: Eq. 16 against the mirror
 * image of the particle in each wall plane (planes at -1/2 and n - 1/2, distance 2h
 * for a centre h from the plane, contact distance D_i, c_i), faces in the order
 * -x,+x,-y,+y,-z,+z.  c holds the c_i of Eq. 16; pairs use D_ij = (D_i + D_j)/2 and
 * c_ij = (c_i + c_j)/2. */
void ref_pair_forces(int32_t dim, const int32_t* n, const int32_t* periodic, int32_t np,
                     const double* X, const double* D, const double* c, double zeta,
                     double eps_pp, double E_pp, const int32_t* ij, int64_t npairs, double* Fc) {
  for (int i = 0; i < 3 * np; i++) Fc[i] = 0.0;
  for (int64_t m = 0; m < npairs; m++) {
    int i = ij[2 * m], j = ij[2 * m + 1];
    double dx[3] = {0, 0, 0}, d2 = 0.0;
    for (int a = 0; a < dim; a++) {
      dx[a] = X[3 * i + a] - X[3 * j + a];
      d2 = d2 + dx[a] * dx[a];
    }
    double d = sqrt(d2);
    double Dij = 0.5 * (D[i] + D[j]);
    double cij = 0.5 * (c[i] + c[j]);
    double mag = ref_pair_force(d, Dij, zeta, cij, eps_pp, E_pp);
    for (int a = 0; a < dim; a++) {
      double Fa = mag * (dx[a] / d);
      Fc[3 * i + a] = Fc[3 * i + a] + Fa;
      Fc[3 * j + a] = Fc[3 * j + a] - Fa;
    }
  }
  for (int p = 0; p < np; p++)
    for (int a = 0; a < dim; a++) {
      if (periodic[a]) continue;
      for (int side = 0; side < 2; side++) {
        double h = side == 0 ? X[3 * p + a] + 0.5 : (n[a] - 0.5) - X[3 * p + a];
        double d = 2.0 * h;
        double mag = ref_pair_force(d, D[p], zeta, c[p], eps_pp, E_pp);
        if (mag != 0.0) Fc[3 * p + a] = Fc[3 * p + a] + (side == 0 ? mag : -mag);
      }
    }
}

static void pair_forces(ref_ctx* c) {
  const ref_config* k = &c->cfg;
  ref_pair_forces(c->dim, k->n, k->periodic, c->np, c->X, c->D, c->cbuoy, k->zeta, k->eps_pp,
                  k->E_pp, c->pairs, c->npairs, c->Fc);
}

/* Momentum and angular momentum of the fluid inside one particle of radius R centred at
 * Xc (the fluid that F_f and T_f of Eqs. 14-15 keep moving with the body):
 *   P = sum_x chi(x) rho0 u(x),  L = sum_x chi(x) (x - Xc) x rho0 u(x),
 * with u a velocity field (dim x N, component-major) and chi a volume indicator that falls
 * linearly from 1 to 0 across one lattice spacing at the surface:
 * chi = clamp(R + 1/2 - |x - Xc|, 0, 1).  Nodes inside the walls, in x-outer, y, z-inner
 * order. */
void ref_interior_momentum(int32_t dim, const int32_t* n, const double* Xc, double R, double rho0,
                           const double* u, double* P, double* L) {
  long N = (long)n[0] * n[1] * (dim == 3 ? n[2] : 1);
  double Pa[3] = {0, 0, 0}, La[3] = {0, 0, 0};
  long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < dim; a++) {
    lo[a] = (long)floor(Xc[a] - R - 0.5);
    hi[a] = (long)ceil(Xc[a] + R + 0.5);
    if (lo[a] < 0) lo[a] = 0;
    if (hi[a] > n[a] - 1) hi[a] = n[a] - 1;
  }
  for (long i = lo[0]; i <= hi[0]; i++)
    for (long j = lo[1]; j <= hi[1]; j++)
      for (long l = lo[2]; l <= hi[2]; l++) {
        double r[3] = {(double)i - Xc[0], (double)j - Xc[1], dim == 3 ? (double)l - Xc[2] : 0.0};
        double d2 = 0.0;
        for (int a = 0; a < dim; a++) d2 = d2 + r[a] * r[a];
        double chi = R + 0.5 - sqrt(d2);
        if (chi <= 0.0) continue;
        if (chi > 1.0) chi = 1.0;
        long node = i + n[0] * (j + (long)n[1] * l);
        double m[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++) m[a] = chi * (rho0 * u[a * N + node]);
        double t[3] = {r[1] * m[2] - r[2] * m[1], r[2] * m[0] - r[0] * m[2], r[0] * m[1] - r[1] * m[0]};
        for (int a = 0; a < 3; a++) {
          Pa[a] = Pa[a] + m[a];
          La[a] = La[a] + t[a];
        }
      }
  for (int a = 0; a < 3; a++) {
    P[a] = Pa[a];
    L[a] = La[a];
  }
}

static void interior_momentum(ref_ctx* c, const double* uvel, double* P, double* L) {
  for (int p = 0; p < c->np; p++)
    ref_interior_momentum(c->dim, c->cfg.n, c->X + 3 * p, 0.5 * c->D[p], c->cfg.rho0, uvel, P + 3 * p,
                          L + 3 * p);
}

/* One step of Eqs. 14-15 for one particle (state X, U, Om updated in place).
 *   F_b is the buoyant weight (M - rho0 V) g.
 *   F_f and T_f, which keep the fluid inside the particle moving with it, are the changes
 *   over the step of the momentum P and angular momentum L of that fluid, taken after
 *   streaming at consecutive steps: P - Pprev, L - Lprev (dt = 1).  When that fluid
 *   moves rigidly, P = rho0 V U and Eq. 14 becomes (M - rho0 V) dU/dt = F_h + F_c + F_b.
 *   Time integration (the paper gives none): the hydrodynamic load H = F_h + F_f (and
 *   G = T_h + T_f) enters at the middle of the last interval, as the mean of this step's
 *   and the previous step's values (Hprev, Gprev, zero before the first step), with
 *   explicit Euler for U and Omega and the trapezoid rule for X:
 *     U' = U + ((H + Hprev)/2 + F_c + F_b) / M,   Om' = Om + (G + Gprev)/(2 I),
 *     X' = X + (U + U')/2.
 * In 2-D only the z component of Omega, T_h and L is used.  Hprev, Gprev, Pprev and Lprev
 * are replaced by this step's H, G, P and L. */
void ref_newton_euler(int32_t dim, double M, double V, double I, double rho0, const double* g,
                      const double* Fh, const double* Th, const double* Fc, const double* P,
                      const double* L, double* Pprev, double* Lprev, double* Hprev, double* Gprev,
                      double* X, double* U, double* Om) {
  double meff = M - rho0 * V;
  for (int a = 0; a < dim; a++) {
    double U0 = U[a];
    double H = Fh[a] + (P[a] - Pprev[a]);
    double Havg = 0.5 * (H + Hprev[a]);
    double U1 = U0 + (Havg + Fc[a] + meff * g[a]) / M;
    Hprev[a] = H;
    U[a] = U1;
    X[a] = X[a] + 0.5 * (U0 + U1);
  }
  int a0 = dim == 2 ? 2 : 0;
  for (int a = a0; a < 3; a++) {
    double G = Th[a] + (L[a] - Lprev[a]);
    double Gavg = 0.5 * (G + Gprev[a]);
    Gprev[a] = G;
    Om[a] = Om[a] + Gavg / I;
  }
  for (int a = 0; a < 3; a++) {
    Pprev[a] = P[a];
    Lprev[a] = L[a];
  }
}

static void newton_euler(ref_ctx* c) {
  const ref_config* k = &c->cfg;
  for (int p = 0; p < c->np; p++) {
    int s = 3 * p;
    ref_newton_euler(c->dim, c->M[p], c->V[p], c->I[p], k->rho0, k->gravity, c->Fh + s, c->Th + s,
                     c->Fc + s, c->Pin + s, c->Lin + s, c->Pprev + s, c->Lprev + s, c->Hprev + s,
                     c->Gprev + s, c->X + s, c->U + s, c->Om + s);
  }
}

int32_t ref_step(ref_ctx* c, int32_t nsteps) {
  long N = c->N;
  int q = c->q, d = c->dim;
  for (int s = 0; s < nsteps; s++) {
    /* (1) macroscopic p and u* (Eqs. 5-6) */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) {
      double fl[19], pp, uu[3];
      fl[0] = 0.0;
      for (int a = 1; a < q; a++) fl[a] = c->f[(a - 1) * N + i];
      ref_macro(d, c->cfg.rho0, fl, &pp, uu);
      c->p[i] = pp;
      for (int a = 0; a < 3; a++) c->ustar[a * N + i] = uu[a];
    }
    /* (2) pairs at the positions of this step */
    if (c->np > 0) find_pairs(c);
    /* (3) IB forcing */
    if (c->nmk > 0) {
      ibm_stage(c);
    } else {
      memset(c->fib, 0, sizeof(double) * 3 * (size_t)N);
      c->slip = 0.0;
    }
    /* (4) collision and streaming */
    if (c->cfg.streaming == 1) {
      collide(c, c->f);
      stream_swap(c);
    } else {
      collide(c, c->ft);
      stream_two_array(c, c->ft, c->f);
    }
    apply_face_bc(c);
    /* (5) particles */
    if (c->np > 0) {
      /* momentum of the fluid inside each particle after streaming (u* of the new PDFs) */
      for (long i = 0; i < N; i++) {
        double fl[19], pp, uu[3];
        fl[0] = 0.0;
        for (int a = 1; a < q; a++) fl[a] = c->f[(a - 1) * N + i];
        ref_macro(d, c->cfg.rho0, fl, &pp, uu);
        for (int a = 0; a < d; a++) c->g[a * N + i] = uu[a];
      }
      interior_momentum(c, c->g, c->Pin, c->Lin);
      particle_loads(c);
      pair_forces(c);
      newton_euler(c);
      memcpy(c->mFprev, c->mF, sizeof(double) * 3 * (size_t)c->nmk);
    }
  }
  return 0;
}

int32_t ref_get_fields(const ref_ctx* c, double* p, double* u, double* force) {
  long N = c->N;
  int q = c->q, d = c->dim;
  for (long i = 0; i < N; i++) {
    double fl[19], pp, uu[3];
    fl[0] = 0.0;
    for (int a = 1; a < q; a++) fl[a] = c->f[(a - 1) * N + i];
    ref_macro(d, c->cfg.rho0, fl, &pp, uu);
    if (p) p[i] = pp;
    if (u)
      for (int a = 0; a < d; a++) u[a * N + i] = uu[a];
    if (force)
      for (int a = 0; a < d; a++) force[a * N + i] = c->fib[a * N + i];
  }
  return 0;
}

int32_t ref_get_particles(const ref_ctx* c, double* X, double* U, double* Om, double* Fh,
                          double* Th, double* Fc) {
  size_t b = sizeof(double) * 3 * (size_t)c->np;
  if (X) memcpy(X, c->X, b);
  if (U) memcpy(U, c->U, b);
  if (Om) memcpy(Om, c->Om, b);
  if (Fh) memcpy(Fh, c->Fh, b);
  if (Th) memcpy(Th, c->Th, b);
  if (Fc) memcpy(Fc, c->Fc, b);
  return 0;
}

int32_t ref_get_markers(const ref_ctx* c, double* F, double* r, int32_t* owner, double* dV) {
  for (int m = 0; m < c->nmk; m++) {
    for (int a = 0; a < 3; a++) {
      if (F) F[3 * m + a] = c->mF[3 * m + a];
      if (r) r[3 * m + a] = c->mr[3 * m + a];
    }
    if (owner) owner[m] = c->mown[m];
    if (dV) dV[m] = c->mdV[m];
  }
  return 0;
}

int32_t ref_num_markers(const ref_ctx* c) { return c->nmk; }

int64_t ref_get_pairs(const ref_ctx* c, int32_t* ij, int64_t cap) {
  for (int64_t m = 0; m < c->npairs && m < cap; m++) {
    ij[2 * m] = c->pairs[2 * m];
    ij[2 * m + 1] = c->pairs[2 * m + 1];
  }
  return c->npairs;
}

int32_t ref_get_cells(const ref_ctx* c, int32_t* cell, int32_t* dims, double* h_eff) {
  for (int a = 0; a < 3; a++) {
    if (dims) dims[a] = c->nc[a];
    if (h_eff) h_eff[a] = a < c->dim ? (double)c->cfg.n[a] / c->nc[a] : 1.0;
  }
  if (cell)
    for (int p = 0; p < c->np; p++)
      for (int a = 0; a < 3; a++) {
        int v = 0;
        if (a < c->dim) {
          v = (int)floor((c->X[3 * p + a] + 0.5) * c->invh[a]);
          if (v < 0) v = 0;
          if (v > c->nc[a] - 1) v = c->nc[a] - 1;
        }
        cell[3 * p + a] = v;
      }
  return 0;
}

double ref_mass(const ref_ctx* c) {
  double s = 0.0;
  for (long i = 0; i < (long)(c->q - 1) * c->N; i++) s += c->f[i];
  return s;
}
double ref_slip_rms(const ref_ctx* c) { return c->slip; }
int64_t ref_truncated(const ref_ctx* c) { return c->truncated; }
int32_t ref_fallbacks(const ref_ctx* c) { return c->fallbacks; }
double ref_judged_slip(const ref_ctx* c) { return c->judged; }

/* ------------------------------------------------------------------------ */
/* learned forcing: MLP 10 -> 64 -> 64 -> 3 with tanh hidden layers          */

#define NI REF_MLP_IN
#define NH REF_MLP_H
#define NO REF_MLP_OUT

static void mlp_offsets(const double* P, const double** W1, const double** b1, const double** W2,
                        const double** b2, const double** W3, const double** b3) {
  *W1 = P;
  *b1 = *W1 + NH * NI;
  *W2 = *b1 + NH;
  *b2 = *W2 + NH * NH;
  *W3 = *b2 + NH;
  *b3 = *W3 + NO * NH;
}

void ref_mlp_forward(const double* params, int64_t n, const double* x, double* y) {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_offsets(params, &W1, &b1, &W2, &b2, &W3, &b3);
  /* samples are independent: the result does not depend on the thread count */
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; s++) {
    double h1[NH], h2[NH];
    for (int o = 0; o < NH; o++) {
      double a = b1[o];
      for (int i = 0; i < NI; i++) a += W1[o * NI + i] * x[s * NI + i];
      h1[o] = tanh(a);
    }
    for (int o = 0; o < NH; o++) {
      double a = b2[o];
      for (int i = 0; i < NH; i++) a += W2[o * NH + i] * h1[i];
      h2[o] = tanh(a);
    }
    for (int o = 0; o < NO; o++) {
      double a = b3[o];
      for (int i = 0; i < NH; i++) a += W3[o * NH + i] * h2[i];
      y[s * NO + o] = a;
    }
  }
}

double ref_mlp_loss_grad(const double* params, int64_t n, const double* x, const double* t,
                         double* grad) {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_offsets(params, &W1, &b1, &W2, &b2, &W3, &b3);
  double *gW1 = grad, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH,
         *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
  for (int i = 0; i < REF_MLP_NPARAM; i++) grad[i] = 0.0;
  double loss = 0.0;
  double scale = 2.0 / (double)(n * NO);
  for (int64_t s = 0; s < n; s++) {
    const double* xs = x + s * NI;
    double h1[NH], h2[NH], y[NO], dy[NO], dh2[NH], dh1[NH];
    for (int o = 0; o < NH; o++) {
      double a = b1[o];
      for (int i = 0; i < NI; i++) a += W1[o * NI + i] * xs[i];
      h1[o] = tanh(a);
    }
    for (int o = 0; o < NH; o++) {
      double a = b2[o];
      for (int i = 0; i < NH; i++) a += W2[o * NH + i] * h1[i];
      h2[o] = tanh(a);
    }
    for (int o = 0; o < NO; o++) {
      double a = b3[o];
      for (int i = 0; i < NH; i++) a += W3[o * NH + i] * h2[i];
      y[o] = a;
      double e = y[o] - t[s * NO + o];
      loss += e * e;
      dy[o] = scale * e;
    }
    /* backward: d tanh(a)/da = 1 - tanh(a)^2 */
    for (int i = 0; i < NH; i++) {
      double a = 0.0;
      for (int o = 0; o < NO; o++) a += W3[o * NH + i] * dy[o];
      dh2[i] = a * (1.0 - h2[i] * h2[i]);
    }
    for (int o = 0; o < NO; o++) {
      gb3[o] += dy[o];
      for (int i = 0; i < NH; i++) gW3[o * NH + i] += dy[o] * h2[i];
    }
    for (int i = 0; i < NH; i++) {
      double a = 0.0;
      for (int o = 0; o < NH; o++) a += W2[o * NH + i] * dh2[o];
      dh1[i] = a * (1.0 - h1[i] * h1[i]);
    }
    for (int o = 0; o < NH; o++) {
      gb2[o] += dh2[o];
      for (int i = 0; i < NH; i++) gW2[o * NH + i] += dh2[o] * h1[i];
    }
    for (int o = 0; o < NH; o++) {
      gb1[o] += dh1[o];
      for (int i = 0; i < NI; i++) gW1[o * NI + i] += dh1[o] * xs[i];
    }
  }
  return loss / (double)(n * NO);
}

int32_t ref_set_mlp(ref_ctx* c, const double* params, const double* norm) {
  memcpy(c->mlp, params, sizeof(double) * REF_MLP_NPARAM);
  memcpy(c->norm, norm, sizeof(double) * (2 * NI + 2 * NO));
  c->has_mlp = 1;
  return 0;
}

/* Gap feature of a surface point Xk of particle p: the distance from Xk to the nearest
 * surface of a pair partner of p (|Xk - X_o| - D_o/2) or to a wall plane (at -1/2 and
 * n - 1/2 on non-periodic axes), clamped to [0, zeta].  Only pair partners (centre
 * distance < D_ij + zeta) can come closer than zeta, so they are the only candidates. */
double ref_point_gap(int32_t dim, const int32_t* n, const int32_t* periodic, double zeta,
                     const double* Xk, int32_t p, const double* X, const double* D,
                     const int32_t* ij, int64_t npairs) {
  double gap = zeta;
  for (int64_t s = 0; s < npairs; s++) {
    int i = ij[2 * s], j = ij[2 * s + 1];
    int o = i == p ? j : (j == p ? i : -1);
    if (o < 0) continue;
    double d2 = 0.0;
    for (int a = 0; a < dim; a++) {
      double dx = Xk[a] - X[3 * o + a];
      d2 = d2 + dx * dx;
    }
    double gg = sqrt(d2) - 0.5 * D[o];
    if (gg < gap) gap = gg;
  }
  for (int a = 0; a < dim; a++) {
    if (periodic[a]) continue;
    double lo = Xk[a] + 0.5, hi = (n[a] - 0.5) - Xk[a];
    if (lo < gap) gap = lo;
    if (hi < gap) gap = hi;
  }
  return gap < 0.0 ? 0.0 : gap;
}

/* Features of each point at the start of the step: slip U_b - D_I u* [3], the point's
 * force of the previous step [3], the outward unit normal r_k/R [3], and the gap to
 * the nearest other surface or wall plane, clamped to [0, zeta] [1].  Only pair
 * partners (centre distance < D_ij + zeta) can come closer than zeta, so they are the
 * only candidates. */
static void features(ref_ctx* c, double* feat) {
  const ref_config* k = &c->cfg;
  ref_ibm_interp(c->dim, k->n, k->periodic, k->delta, c->ustar, c->nmk, c->mX, c->muh, 0);
  for (int m = 0; m < c->nmk; m++) {
    int p = c->mown[m];
    double R = 0.5 * c->D[p];
    double* F = feat + NI * m;
    for (int a = 0; a < 3; a++) {
      F[a] = a < c->dim ? c->mUb[3 * m + a] - c->muh[3 * m + a] : 0.0;
      F[3 + a] = c->mFprev[3 * m + a];
      F[6 + a] = c->mr[3 * m + a] / R;
    }
    F[9] = ref_point_gap(c->dim, k->n, k->periodic, k->zeta, c->mX + 3 * m, p, c->X, c->D,
                         c->pairs, c->npairs);
  }
}

void ref_mlp_predict(const double* params, const double* norm, int64_t n, int32_t dim,
                     const double* feat, const double* Fprev, double* F) {
  const double* mean = norm;
  const double* sd = norm + NI;
  const double* tmean = norm + 2 * NI;
  const double* tsd = norm + 2 * NI + NO;
  double* xn = (double*)xcalloc((size_t)NI * (size_t)(n > 0 ? n : 1), sizeof(double));
  double* y = (double*)xcalloc((size_t)NO * (size_t)(n > 0 ? n : 1), sizeof(double));
  for (int64_t m = 0; m < n; m++)
    for (int i = 0; i < NI; i++) xn[NI * m + i] = (feat[NI * m + i] - mean[i]) / sd[i];
  ref_mlp_forward(params, n, xn, y);
  for (int64_t m = 0; m < n; m++)
    for (int o = 0; o < 3; o++)
      F[3 * m + o] = o < dim ? Fprev[3 * m + o] + (tmean[o] + tsd[o] * y[NO * m + o]) : 0.0;
  free(xn);
  free(y);
}

static void mlp_apply(ref_ctx* c, const double* feat, double* Fout) {
  ref_mlp_predict(c->mlp, c->norm, c->nmk, c->dim, feat, c->mFprev, Fout);
}

int32_t ref_capture_samples(ref_ctx* c, double* feat, double* target) {
  /* a dry run of the forcing stage of the next step: the PDFs are not advanced */
  long N = c->N;
  int q = c->q, d = c->dim;
  for (long i = 0; i < N; i++) {
    double fl[19], pp, uu[3];
    fl[0] = 0.0;
    for (int a = 1; a < q; a++) fl[a] = c->f[(a - 1) * N + i];
    ref_macro(d, c->cfg.rho0, fl, &pp, uu);
    c->p[i] = pp;
    for (int a = 0; a < 3; a++) c->ustar[a * N + i] = uu[a];
  }
  if (c->np > 0) find_pairs(c);
  markers_update(c);
  features(c, feat);
  mdf(c, c->cfg.mdf_iters);
  memcpy(target, c->mF, sizeof(double) * 3 * (size_t)c->nmk);
  return 0;
}

// Particle kernels for gfx950: cell list and pair search (Sec. 5, Eqs. 49-51), the
// short-range pair force (Eq. 16), hydrodynamic loads and Newton-Euler motion
// (Sec. 2.3, Eqs. 14-15).  Everything here is FP64.
//
// Cells are at least (D_max + zeta)/2 wide (Eq. 50), so every partner of a particle
// lies in the 5^d block of cells around its own.  A cell holds up to CELL_CAP centres
// (Eq. 49 keeps it at one for non-overlapping particles).  Pair tests and forces are
// evaluated with contraction off, so they round exactly like a plain sequential
// program; each particle sums its partner forces in ascending partner order, which
// makes the result independent of thread scheduling.
#include "common.h"
#include "index_math.h"

#pragma clang fp contract(off)

namespace {

struct PartArgs {
  int np, dim;
  int n[3], nc[3], periodic[3];
  double invh[3];
  double zeta, eps_pp, E_pp, rho0;
  double g[3];
  const double *X, *D, *cb;
  double *U, *Om, *Fh, *Th, *Fc, *Xw, *M, *I;
  int* cell_count;
  int* cell_items;
  int* cell_of;
  int *pair_up, *pair_nup;
  int *pair_all, *pair_nall;
  int* status;
};

// Cell of every particle and a slot in it.  Consecutive lanes of a wavefront whose
// particles share a cell form a run: a ballot of run heads gives every lane its head
// and the run length, the head takes one atomic for the whole run, and the others
// rank themselves by their distance from the head.
__global__ void k_cells(PartArgs a) {
  // tested after the position loads are issued, so that the latencies overlap
  const bool stop = halted(a.status);
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = p < a.np;
  long long id = -1;
  int c[3] = {0, 0, 0};
  if (act)
    for (int d = 0; d < a.dim; d++) c[d] = cell_coord(a.X[3 * p + d], a.invh[d], a.nc[d]);
  if (stop) return;
  if (act) {
    for (int d = 0; d < 3; d++) a.cell_of[3 * p + d] = c[d];
    id = c[0] + (long long)a.nc[0] * (c[1] + (long long)a.nc[1] * c[2]);
  }
  int lane = threadIdx.x & 63;
  long long prev = __shfl(id, lane > 0 ? lane - 1 : 0, 64);
  bool head = act && (lane == 0 || prev != id);
  unsigned long long heads = __ballot(head);
  unsigned long long actm = __ballot(act);
  unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  unsigned long long below = heads & upto;
  int h = below ? 63 - __clzll(below) : 0;
  int base = 0;
  if (head) {
    unsigned long long above = heads & ~upto;
    int next = above ? __ffsll((long long)above) - 1 : __popcll(actm);
    base = atomicAdd(&a.cell_count[id], next - lane);
  }
  base = __shfl(base, h, 64);
  if (act) {
    int rank = base + (lane - h);
    if (rank < CELL_CAP)
      a.cell_items[id * CELL_CAP + rank] = p;
    else
      atomicOr(a.status, ST_CELL_OVERFLOW);
  }
}

// Eq. 16: magnitude of the repulsion along the unit vector from the partner
__device__ double pair_mag(double d, double D, double zeta, double c, double eps, double E) {
  if (d >= D + zeta) return 0.0;
  double s = (d - D - zeta) / zeta;
  double F = c / eps * (s * s);
  if (d < D) F = F + c / E * ((D - d) / zeta);
  return F;
}

constexpr int MAXP = 32;

// One wavefront per particle: lanes scan the 5^d cells around it, candidates are
// compacted with ballots into LDS and ranked into ascending order; each lane computes one
// partner's pair force and writes the pair lists, and one lane sums the forces in
// ascending partner order (pairs first, then the wall images in face order).
__global__ __launch_bounds__(256) void k_pairs(PartArgs a) {
  // tested after the cell loads are issued, so that the latencies overlap
  const bool stop = halted(a.status);
  __shared__ int cand[4][MAXP], srt[4][MAXP];
  __shared__ double cf[4][MAXP][3];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = blockIdx.x * 4 + wv;
  bool act = i < a.np;
  int ncand = 0;
  bool over = false;
  int ci[3] = {0, 0, 0};
  if (act)
    for (int d = 0; d < 3; d++) ci[d] = a.cell_of[3 * i + d];
  if (stop) return;
  if (act) {
    const double* Xi = a.X + 3 * i;
    int lo[3], w[3];
    for (int d = 0; d < 3; d++) {
      lo[d] = d < a.dim ? max(ci[d] - 2, 0) : 0;
      int hi = d < a.dim ? min(ci[d] + 2, a.nc[d] - 1) : 0;
      w[d] = hi - lo[d] + 1;
    }
    int nwin = w[0] * w[1] * w[2];
    for (int t0 = 0; t0 < nwin; t0 += 64) {
      int t = t0 + lane;
      long long id = -1;
      int m = 0;
      if (t < nwin) {
        int cx = lo[0] + t % w[0], cy = lo[1] + (t / w[0]) % w[1], cz = lo[2] + t / (w[0] * w[1]);
        id = cx + (long long)a.nc[0] * (cy + (long long)a.nc[1] * cz);
        m = min(a.cell_count[id], CELL_CAP);
      }
      for (int s = 0; s < CELL_CAP; s++) {
        bool hit = false;
        int j = -1;
        if (s < m) {
          j = a.cell_items[id * CELL_CAP + s];
          if (j != i) {
            const double* Xj = a.X + 3 * j;
            double d2 = 0.0;
            for (int d = 0; d < a.dim; d++) {
              double dx = Xi[d] - Xj[d];
              d2 = d2 + dx * dx;
            }
            double sr = 0.5 * (a.D[i] + a.D[j]) + a.zeta;
            hit = d2 < sr * sr;
          }
        }
        unsigned long long mask = __ballot(hit);
        if (mask == 0ull) {
          if (!__ballot(s + 1 < m)) break;
          continue;
        }
        int pos = ncand + __popcll(mask & ((1ull << lane) - 1ull));
        if (hit) {
          if (pos < MAXP)
            cand[wv][pos] = j;
          else
            over = true;
        }
        ncand += __popcll(mask);
      }
    }
  }
  __syncthreads();
  // the candidates are distinct: each lane ranks its own among them, which sorts them
  const int cnt = act ? min(ncand, MAXP) : 0;
  if (lane < cnt) {
    const int j = cand[wv][lane];
    int r = 0;
    for (int k = 0; k < cnt; k++) r += cand[wv][k] < j ? 1 : 0;
    srt[wv][r] = j;
  }
  __syncthreads();
  // lane k: the k-th partner in ascending order and its Eq. 16 force on particle i, with
  // the sign that the ordered sum below applies
  const int jl = lane < cnt ? srt[wv][lane] : -1;
  if (lane < cnt) {
    const int pa = i < jl ? i : jl, pb = i < jl ? jl : i;
    double dx[3] = {0.0, 0.0, 0.0}, d2 = 0.0;
    for (int d = 0; d < a.dim; d++) {
      dx[d] = a.X[3 * pa + d] - a.X[3 * pb + d];
      d2 = d2 + dx[d] * dx[d];
    }
    double dist = sqrt(d2);
    double mag = pair_mag(dist, 0.5 * (a.D[pa] + a.D[pb]), a.zeta, 0.5 * (a.cb[pa] + a.cb[pb]),
                          a.eps_pp, a.E_pp);
    for (int d = 0; d < 3; d++) {
      double Fa = d < a.dim ? mag * (dx[d] / dist) : 0.0;
      cf[wv][lane][d] = i == pa ? Fa : -Fa;
    }
    if (lane < PAIR_CAP) a.pair_all[i * PAIR_CAP + lane] = jl;
  }
  // the partners j > i are a suffix of the ascending list
  const int nlow = __popcll(__ballot(lane < cnt && jl < i));
  if (lane < cnt && jl > i) {
    if (lane - nlow < PAIR_CAP)
      a.pair_up[i * PAIR_CAP + (lane - nlow)] = jl;
    else
      over = true;
  }
  __syncthreads();
  if (!act || lane != 0) {
    if (over) atomicOr(a.status, ST_PAIR_OVERFLOW);
    return;
  }
  const double* Xi = a.X + 3 * i;
  // pair forces summed in ascending partner order (x - y and x + (-y) round alike)
  double F[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < cnt; k++)
    for (int d = 0; d < a.dim; d++) F[d] = F[d] + cf[wv][k][d];
  const int nup = cnt - nlow;
  // walls: Eq. 16 against the mirror image in each wall plane (at -1/2 and n - 1/2)
  for (int d = 0; d < a.dim; d++) {
    if (a.periodic[d]) continue;
    for (int side = 0; side < 2; side++) {
      double h = side == 0 ? Xi[d] + 0.5 : (a.n[d] - 0.5) - Xi[d];
      double mag = pair_mag(2.0 * h, a.D[i], a.zeta, a.cb[i], a.eps_pp, a.E_pp);
      if (mag != 0.0) F[d] = F[d] + (side == 0 ? mag : -mag);
    }
  }
  for (int d = 0; d < 3; d++) a.Fc[3 * i + d] = F[d];
  a.pair_nup[i] = min(nup, PAIR_CAP);
  a.pair_nall[i] = min(cnt, PAIR_CAP);
  if (over || ncand > MAXP) atomicOr(a.status, ST_PAIR_OVERFLOW);
}

template <class C>
struct LoadArgs {
  PartArgs pa;
  const int *mstart, *mcount;
  const double* mr;
  const double* mdV;
  const C* mF;
  C* mFprev;
  const double *Pin, *Lin;
  double *Pprev, *Lprev, *Hprev, *Gprev;
  const double *M, *V, *I;
  double* X;
  int update;  // 0: loads only
};

// One workgroup per particle: F_h = -sum F_k dV_k, T_h = -sum r_k x F_k dV_k in FP64 in a
// fixed order (butterfly within each wavefront, then the wavefronts in order), then
// Eqs. 14-15 with the interior-fluid terms F_f = P^n - P^(n-1), T_f = L^n - L^(n-1), the
// hydrodynamic load averaged over the current and previous steps, explicit Euler for U,
// Omega and the trapezoid rule for X.
template <class C>
__global__ __launch_bounds__(256) void k_loads_newton(LoadArgs<C> a) {
  __shared__ double red[6][4];
  int p = blockIdx.x;
  int m0 = a.mstart[p], mc = a.mcount[p];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int k = m0 + threadIdx.x; k < m0 + mc; k += blockDim.x) {
    const double* r = a.mr + 4 * (size_t)k;
    const C* Fk = a.mF + 4 * (size_t)k;
    double dV = a.mdV[k];
    double Fd[3] = {double(Fk[0]) * dV, double(Fk[1]) * dV,
                    a.pa.dim == 3 ? double(Fk[2]) * dV : 0.0};
    acc[0] -= Fd[0];
    acc[1] -= Fd[1];
    acc[2] -= Fd[2];
    acc[3] -= r[1] * Fd[2] - r[2] * Fd[1];
    acc[4] -= r[2] * Fd[0] - r[0] * Fd[2];
    acc[5] -= r[0] * Fd[1] - r[1] * Fd[0];
    if (a.update) {
      C* Fp = a.mFprev + 4 * (size_t)k;
      Fp[0] = Fk[0];
      Fp[1] = Fk[1];
      Fp[2] = Fk[2];
    }
  }
  // butterfly sums within each wavefront, then the wavefront partials in a fixed order
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 6; k++) acc[k] += __shfl_xor(acc[k], o, 64);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; k++) red[k][threadIdx.x >> 6] = acc[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const PartArgs& q = a.pa;
  // every operand of the update is loaded before the first store, so that the loads share
  // one memory latency instead of each waiting behind the stores of earlier components
  double M = 0.0, V = 0.0, I = 0.0;
  double U0[3], Om0[3], Pin[3], Ppr[3], Hpr[3], Lin[3], Lpr[3], Gpr[3], Fc[3], X0[3];
  int cl[3] = {0, 0, 0};
  if (a.update) {
    M = a.M[p];
    V = a.V[p];
    I = a.I[p];
    for (int d = 0; d < 3; d++) {
      U0[d] = q.U[3 * p + d];
      Om0[d] = q.Om[3 * p + d];
      Pin[d] = a.Pin[3 * p + d];
      Ppr[d] = a.Pprev[3 * p + d];
      Hpr[d] = a.Hprev[3 * p + d];
      Lin[d] = a.Lin[3 * p + d];
      Lpr[d] = a.Lprev[3 * p + d];
      Gpr[d] = a.Gprev[3 * p + d];
      Fc[d] = q.Fc[3 * p + d];
      X0[d] = a.X[3 * p + d];
      cl[d] = q.cell_of[3 * p + d];
    }
  }
  for (int v = 1; v < (int)(blockDim.x >> 6); v++)
    for (int k = 0; k < 6; k++) red[k][0] += red[k][v];
  for (int d = 0; d < 3; d++) {
    q.Fh[3 * p + d] = red[d][0];
    q.Th[3 * p + d] = red[3 + d][0];
  }
  if (!a.update) return;
  double meff = M - q.rho0 * V;
  bool bad = false;
  for (int d = 0; d < q.dim; d++) {
    double H = red[d][0] + (Pin[d] - Ppr[d]);
    double Havg = 0.5 * (H + Hpr[d]);
    double U1 = U0[d] + (Havg + Fc[d] + meff * q.g[d]) / M;
    a.Hprev[3 * p + d] = H;
    q.U[3 * p + d] = U1;
    a.X[3 * p + d] = X0[d] + 0.5 * (U0[d] + U1);
    bad |= !(U1 == U1) || fabs(U1) > 1.0;
  }
  for (int d = (q.dim == 2 ? 2 : 0); d < 3; d++) {
    double G = red[3 + d][0] + (Lin[d] - Lpr[d]);
    double Gavg = 0.5 * (G + Gpr[d]);
    a.Gprev[3 * p + d] = G;
    const double Om1 = Om0[d] + Gavg / I;
    q.Om[3 * p + d] = Om1;
    bad |= !(Om1 == Om1);
  }
  for (int d = 0; d < 3; d++) {
    a.Pprev[3 * p + d] = Pin[d];
    a.Lprev[3 * p + d] = Lin[d];
  }
  // empty this particle's cell for the next cell-list build
  q.cell_count[cl[0] + (long long)q.nc[0] * (cl[1] + (long long)q.nc[1] * cl[2])] = 0;
  if (bad) atomicOr(q.status, ST_NAN);
}

__global__ void k_zero_cells(PartArgs a) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.np) return;
  int c0 = a.cell_of[3 * p], c1 = a.cell_of[3 * p + 1], c2 = a.cell_of[3 * p + 2];
  a.cell_count[c0 + (long long)a.nc[0] * (c1 + (long long)a.nc[1] * c2)] = 0;
}

PartArgs make_pargs(iblbm_ctx* c) {
  PartArgs a;
  a.np = c->np;
  a.dim = c->dim;
  for (int d = 0; d < 3; d++) {
    a.n[d] = c->cfg.n[d];
    a.nc[d] = c->nc[d];
    a.periodic[d] = c->cfg.periodic[d];
    a.invh[d] = c->invh[d];
    a.g[d] = c->cfg.gravity[d];
  }
  a.zeta = c->cfg.zeta;
  a.eps_pp = c->cfg.eps_pp;
  a.E_pp = c->cfg.E_pp;
  a.rho0 = c->cfg.rho0;
  a.X = c->X;
  a.D = c->D;
  a.cb = c->cb;
  a.U = c->U;
  a.Om = c->Om;
  a.Fh = c->Fh;
  a.Th = c->Th;
  a.Fc = c->Fc;
  a.cell_count = c->cell_count;
  a.cell_items = c->cell_items;
  a.cell_of = c->cell_of;
  a.pair_up = c->pair_up;
  a.pair_nup = c->pair_nup;
  a.pair_all = c->pair_all;
  a.pair_nall = c->pair_nall;
  a.status = c->dstatus;
  return a;
}

template <class C>
void run_loads(iblbm_ctx* c, int update) {
  LoadArgs<C> a;
  a.pa = make_pargs(c);
  a.mstart = c->mstart;
  a.mcount = c->mcount;
  a.mr = c->mr;
  a.mdV = c->mdV;
  a.mF = (const C*)c->mF;
  a.mFprev = (C*)c->mFprev;
  a.Pin = c->Pin;
  a.Lin = c->Lin;
  a.Pprev = c->Pprev;
  a.Lprev = c->Lprev;
  a.Hprev = c->Hprev;
  a.Gprev = c->Gprev;
  a.M = c->M;
  a.V = c->V;
  a.I = c->I;
  a.X = c->X;
  a.update = update;
  // one wavefront per 64 points of the largest particle, at most four
  int mx = 1;
  for (int m : c->hcount) mx = m > mx ? m : mx;
  int threads = mx <= 64 ? 64 : (mx <= 128 ? 128 : 256);
  hipLaunchKernelGGL((k_loads_newton<C>), dim3(c->np), dim3(threads), 0, c->stream, a);
}

}  // namespace

// cells of the current positions and the pair forces (F_c) at those positions
void part_cells_pairs(iblbm_ctx* c) {
  if (c->np == 0) return;
  PartArgs a = make_pargs(c);
  int blocks = (c->np + 255) / 256;
  hipLaunchKernelGGL(k_cells, dim3(blocks), dim3(256), 0, c->stream, a);
  hipLaunchKernelGGL(k_pairs, dim3((c->np + 3) / 4), dim3(256), 0, c->stream, a);
}

// loads and the Newton-Euler update (which also empties the cells used this step)
void part_loads_newton(iblbm_ctx* c) {
  if (c->np == 0) return;
  if (c->fp64) run_loads<double>(c, 1); else run_loads<float>(c, 1);
}

void part_zero_cells(iblbm_ctx* c) {
  if (c->np == 0) return;
  PartArgs a = make_pargs(c);
  hipLaunchKernelGGL(k_zero_cells, dim3((c->np + 255) / 256), dim3(256), 0, c->stream, a);
}

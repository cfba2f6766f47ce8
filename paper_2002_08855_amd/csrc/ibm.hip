// Immersed-boundary kernels for gfx950 (Sec. 2.2 and Sec. 4 of the paper).
//
// Each Lagrangian point touches the nodes of its delta-function support only
// (Eqs. 47-48).  A wavefront serves one point in 3-D (4x4x4 = 64 support nodes, one per
// lane) and four points in 2-D (16 lanes each): lane loads, weights and the reduction
// are all independent of the other points, so interpolation is a gather plus a
// cross-lane sum, and spreading is a set of float atomics into the band force buffer.
// Band bookkeeping: before the forcing, every 16-node row segment that some support
// touches is flagged (and listed once), so that u* is computed and the force cleared
// only there, and the collision reads the force only there.
#include "common.h"

namespace {

template <class C>
__device__ __forceinline__ C phi(int kind, C r) {
  C a = r < C(0) ? -r : r;
  if (kind == 0) {  // Peskin 4-point
    if (a < C(1)) return (C(3) - C(2) * a + sqrt(C(1) + C(4) * a - C(4) * a * a)) * C(0.125);
    if (a < C(2)) return (C(5) - C(2) * a - sqrt(C(-7) + C(12) * a - C(4) * a * a)) * C(0.125);
    return C(0);
  }
  // Roma-Peskin-Berger 3-point
  if (a < C(0.5)) return (C(1) + sqrt(C(1) - C(3) * a * a)) / C(3);
  if (a < C(1.5)) return (C(5) - C(3) * a - sqrt(C(1) - C(3) * (C(1) - a) * (C(1) - a))) / C(6);
  return C(0);
}

struct MarkerGeo {
  int n[3], periodic[3];
  int dim, kind, width;
};

// The support node handled by lane l of a point at X: returns the node index or -1
// (outside a wall axis), and its weight.
template <int DIM, class C>
__device__ __forceinline__ int support_node(const MarkerGeo& g, const double* X, int l, C& w,
                                            bool& trunc) {
  int id[3] = {l & 3, (l >> 2) & 3, (l >> 4) & 3};
  w = C(1);
  trunc = false;
  int c[3] = {0, 0, 0};
  bool inside_support = true;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    if (id[a] >= g.width) inside_support = false;
    int lo = g.kind == 0 ? int(floor(X[a])) - 1 : int(floor(X[a] + 0.5)) - 1;
    int cc = lo + id[a];
    w *= phi<C>(g.kind, C(double(cc) - X[a]));
    if (cc < 0 || cc >= g.n[a]) {
      if (g.periodic[a]) {
        cc = cc < 0 ? cc + g.n[a] : cc - g.n[a];
      } else {
        trunc = true;
      }
    }
    c[a] = cc;
  }
  if (!inside_support) {
    trunc = false;
    return -1;
  }
  if (trunc) return -1;
  return c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

struct PartView {
  const double *X, *U, *Om;
  const int* mown;
  const double* mr;  // nmk x 4
  const double* mdV;
};

template <class C>
__device__ __forceinline__ void marker_pos_vel(const PartView& P, int k, double* X, double* Ub,
                                               int dim) {
  int p = P.mown[k];
  const double* r = P.mr + 4 * k;
  const double* Xc = P.X + 3 * p;
  const double* Uc = P.U + 3 * p;
  const double* W = P.Om + 3 * p;
  X[0] = Xc[0] + r[0];
  X[1] = Xc[1] + r[1];
  X[2] = dim == 3 ? Xc[2] + r[2] : 0.0;
  Ub[0] = Uc[0] + (W[1] * r[2] - W[2] * r[1]);
  Ub[1] = Uc[1] + (W[2] * r[0] - W[0] * r[2]);
  Ub[2] = dim == 3 ? Uc[2] + (W[0] * r[1] - W[1] * r[0]) : 0.0;
}

template <class C>
__device__ __forceinline__ C group_sum(C v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class C>
struct InterpArgs {
  MarkerGeo g;
  PartView P;
  int nmk;
  const C* ustar;
  const C* facc;
  int vd;
  C half_inv_rho, two_rho;
  C* F;         // nmk x 4
  C* dF;        // nmk x 4
  int first_pass, mode;
  unsigned long long* trunc;
  double* slip2;
  float* feat;  // nmk x 10
};

// mode 0: multi-direct-forcing pass (Eqs. 9-10): dF = 2 rho0 (U_b - D_I u), F += dF.
// mode 1: accumulate |U_b - D_I u|^2 for the slip statistic.
// mode 2: write U_b - D_I u* into the learned-force features.
template <int DIM, class C>
__global__ __launch_bounds__(256) void k_interp(InterpArgs<C> a) {
  constexpr int G = DIM == 3 ? 64 : 16;
  int gid = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  int l = threadIdx.x & (G - 1);
  int k = gid;
  bool active = k < a.nmk;
  double X[3] = {0, 0, 0}, Ub[3] = {0, 0, 0};
  if (active) marker_pos_vel<C>(a.P, k, X, Ub, DIM);
  C acc[3] = {0, 0, 0};
  bool tr = false;
  if (active) {
    C w;
    int i = support_node<DIM, C>(a.g, X, l, w, tr);
    if (i >= 0) {
      const C* u = a.ustar + (size_t)i * a.vd;
      const C* f = a.facc + (size_t)i * a.vd;
      acc[0] = w * (u[0] + f[0] * a.half_inv_rho);
      acc[1] = w * (u[1] + f[1] * a.half_inv_rho);
      if (DIM == 3) acc[2] = w * (u[2] + f[2] * a.half_inv_rho);
    }
  }
  for (int c = 0; c < DIM; c++) acc[c] = group_sum(acc[c], G);
  if (a.first_pass && a.mode == 0) {
    unsigned long long m = __ballot(tr);
    if (l == 0 && m) {
      unsigned long long mine = G == 64 ? m : (m >> (threadIdx.x & 63 & ~(G - 1))) & ((1ull << G) - 1);
      if (mine) atomicAdd(a.trunc, (unsigned long long)__popcll(mine));
    }
  }
  if (!active || l != 0) return;
  if (a.mode == 0) {
    C* F = a.F + 4 * (size_t)k;
    C* dF = a.dF + 4 * (size_t)k;
    for (int c = 0; c < DIM; c++) {
      C d = a.two_rho * (C(Ub[c]) - acc[c]);
      dF[c] = d;
      F[c] = a.first_pass ? d : F[c] + d;
    }
  } else if (a.mode == 1) {
    double s = 0;
    for (int c = 0; c < DIM; c++) {
      double e = Ub[c] - double(acc[c]);
      s += e * e;
    }
    atomicAdd(a.slip2, s);
  } else {
    for (int c = 0; c < 3; c++) a.feat[10 * (size_t)k + c] = c < DIM ? float(Ub[c] - double(acc[c])) : 0.f;
  }
}

template <class C>
struct SpreadArgs {
  MarkerGeo g;
  PartView P;
  int nmk;
  const C* dF;  // nmk x 4
  C* facc;
  int vd;
};

// Eq. 11 with Eq. 13: f(x) += dF_k Phi(x - X_k) drs ds_k, with float atomics.
template <int DIM, class C>
__global__ __launch_bounds__(256) void k_spread(SpreadArgs<C> a) {
  constexpr int G = DIM == 3 ? 64 : 16;
  int k = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  int l = threadIdx.x & (G - 1);
  if (k >= a.nmk) return;
  double X[3] = {0, 0, 0}, Ub[3];
  marker_pos_vel<C>(a.P, k, X, Ub, DIM);
  C w;
  bool tr;
  int i = support_node<DIM, C>(a.g, X, l, w, tr);
  if (i < 0) return;
  C s = w * C(a.P.mdV[k]);
  const C* dF = a.dF + 4 * (size_t)k;
  C* f = a.facc + (size_t)i * a.vd;
  unsafeAtomicAdd(f + 0, dF[0] * s);
  unsafeAtomicAdd(f + 1, dF[1] * s);
  if (DIM == 3) unsafeAtomicAdd(f + 2, dF[2] * s);
}

struct MarkArgs {
  MarkerGeo g;
  PartView P;
  const double* D;
  const int *mstart, *mcount;
  uint32_t* bflag;
  int* seglist;
  int* count_new;
  int nsegx;
};

constexpr int MARK_WORDS = 2048;

// One workgroup per particle: collect the row segments touched by the supports of its
// points in an LDS bitmap, then flag and list each new segment once.
template <int DIM>
__global__ __launch_bounds__(256) void k_mark(MarkArgs a) {
  __shared__ uint32_t bits[MARK_WORDS];
  __shared__ int box[6];
  int p = blockIdx.x;
  int m0 = a.mstart[p], mc = a.mcount[p];
  if (threadIdx.x == 0) {
    // every point lies at distance R from the centre, so its support stays inside
    // [floor(Xc - R) - 2, floor(Xc + R) + 3] on each axis
    double R = 0.5 * a.D[p];
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < DIM; d++) {
      double xc = a.P.X[3 * p + d];
      lo[d] = max(int(floor(xc - R)) - 2, 0);
      hi[d] = min(int(floor(xc + R)) + 3, a.g.n[d] - 1);
    }
    box[0] = lo[0] / SEG;
    box[1] = hi[0] / SEG;
    box[2] = lo[1];
    box[3] = hi[1];
    box[4] = lo[2];
    box[5] = hi[2];
  }
  for (int w = threadIdx.x; w < MARK_WORDS; w += blockDim.x) bits[w] = 0;
  __syncthreads();
  int nsx = box[1] - box[0] + 1, ny = box[3] - box[2] + 1, nz = box[5] - box[4] + 1;
  long long nbits = (long long)nsx * ny * nz;
  if (nbits > 32LL * MARK_WORDS || nsx <= 0 || ny <= 0 || nz <= 0) {
    // degenerate or oversized box: flag every touched segment directly
    for (int t = threadIdx.x; t < mc * 16; t += blockDim.x) {
      int k = m0 + t / 16, row = t % 16;
      double X[3], Ub[3];
      marker_pos_vel<double>(a.P, k, X, Ub, DIM);
      int l0[3];
      for (int d = 0; d < DIM; d++)
        l0[d] = a.g.kind == 0 ? int(floor(X[d])) - 1 : int(floor(X[d] + 0.5)) - 1;
      int yy = l0[1] + (row & 3), zz = DIM == 3 ? l0[2] + (row >> 2) : 0;
      if ((row & 3) >= a.g.width || (DIM == 3 && (row >> 2) >= a.g.width) || (DIM == 2 && row >= 4)) continue;
      if (yy < 0 || yy >= a.g.n[1] || zz < 0 || zz >= a.g.n[2]) continue;
      int xa = max(l0[0], 0), xb = min(l0[0] + a.g.width - 1, a.g.n[0] - 1);
      for (int sx = xa / SEG; sx <= xb / SEG && xa <= xb; sx++) {
        int seg = sx + a.nsegx * (yy + a.g.n[1] * zz);
        if (atomicOr(&a.bflag[seg], 1u) == 0u) a.seglist[atomicAdd(a.count_new, 1)] = seg;
      }
    }
    return;
  }
  for (int t = threadIdx.x; t < mc * 16; t += blockDim.x) {
    int k = m0 + t / 16, row = t % 16;
    if ((row & 3) >= a.g.width || (DIM == 3 && (row >> 2) >= a.g.width) || (DIM == 2 && row >= 4)) continue;
    double X[3], Ub[3];
    marker_pos_vel<double>(a.P, k, X, Ub, DIM);
    int l0[3] = {0, 0, 0};
    for (int d = 0; d < DIM; d++)
      l0[d] = a.g.kind == 0 ? int(floor(X[d])) - 1 : int(floor(X[d] + 0.5)) - 1;
    int yy = l0[1] + (row & 3), zz = DIM == 3 ? l0[2] + (row >> 2) : 0;
    if (yy < 0 || yy >= a.g.n[1] || zz < 0 || zz >= a.g.n[2]) continue;
    int xa = max(l0[0], 0), xb = min(l0[0] + a.g.width - 1, a.g.n[0] - 1);
    if (xa > xb) continue;
    for (int sx = xa / SEG; sx <= xb / SEG; sx++) {
      long long bit = (long long)(sx - box[0]) + nsx * ((long long)(yy - box[2]) + ny * (zz - box[4]));
      atomicOr(&bits[bit >> 5], 1u << (bit & 31));
    }
  }
  __syncthreads();
  for (long long bit = threadIdx.x; bit < nbits; bit += blockDim.x) {
    if (!((bits[bit >> 5] >> (bit & 31)) & 1u)) continue;
    int sx = int(bit % nsx) + box[0];
    long long r = bit / nsx;
    int yy = int(r % ny) + box[2], zz = int(r / ny) + box[4];
    int seg = sx + a.nsegx * (yy + a.g.n[1] * zz);
    if (atomicOr(&a.bflag[seg], 1u) == 0u) a.seglist[atomicAdd(a.count_new, 1)] = seg;
  }
}

// clear the flags listed at the previous step and reset the append counter
__global__ void k_clear(uint32_t* bflag, const int* seglist, const int* count_old, int* count_new) {
  int n = *count_old;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x)
    bflag[seglist[s]] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *count_new = 0;
}

MarkerGeo make_mgeo(const iblbm_ctx* c) {
  MarkerGeo g;
  for (int a = 0; a < 3; a++) {
    g.n[a] = c->cfg.n[a];
    g.periodic[a] = c->cfg.periodic[a];
  }
  g.dim = c->dim;
  g.kind = c->cfg.delta;
  g.width = c->cfg.delta == 0 ? 4 : 3;
  return g;
}

PartView make_pview(const iblbm_ctx* c) {
  PartView P;
  P.X = c->X;
  P.U = c->U;
  P.Om = c->Om;
  P.mown = c->mown;
  P.mr = c->mr;
  P.mdV = c->mdV;
  return P;
}

template <int DIM, class C>
void run_interp(iblbm_ctx* c, int first, int mode) {
  InterpArgs<C> a;
  a.g = make_mgeo(c);
  a.P = make_pview(c);
  a.nmk = c->nmk;
  a.ustar = (const C*)c->ustar;
  a.facc = (const C*)c->facc;
  a.vd = c->vd;
  a.half_inv_rho = C(0.5 / c->cfg.rho0);
  a.two_rho = C(2.0 * c->cfg.rho0);
  a.F = (C*)c->mF;
  a.dF = (C*)c->mdF;
  a.first_pass = first;
  a.mode = mode;
  a.trunc = (unsigned long long*)(c->dstatus + 2);
  a.slip2 = c->dstats;
  a.feat = c->feat;
  constexpr int per = DIM == 3 ? 4 : 16;
  int blocks = (c->nmk + per - 1) / per;
  hipLaunchKernelGGL((k_interp<DIM, C>), dim3(blocks), dim3(256), 0, c->stream, a);
}

template <int DIM, class C>
void run_spread(iblbm_ctx* c) {
  SpreadArgs<C> a;
  a.g = make_mgeo(c);
  a.P = make_pview(c);
  a.nmk = c->nmk;
  a.dF = (const C*)c->mdF;
  a.facc = (C*)c->facc;
  a.vd = c->vd;
  constexpr int per = DIM == 3 ? 4 : 16;
  int blocks = (c->nmk + per - 1) / per;
  hipLaunchKernelGGL((k_spread<DIM, C>), dim3(blocks), dim3(256), 0, c->stream, a);
}

}  // namespace

void ibm_clear_and_mark(iblbm_ctx* c) {
  int b = c->segcur;
  int* cnt_old = c->segcount + b;
  int* cnt_new = c->segcount + (1 - b);
  hipLaunchKernelGGL(k_clear, dim3(256), dim3(256), 0, c->stream, c->bflag, c->seglist, cnt_old,
                     cnt_new);
  if (c->np > 0) {
    MarkArgs a;
    a.g = make_mgeo(c);
    a.P = make_pview(c);
    a.D = c->D;
    a.mstart = c->mstart;
    a.mcount = c->mcount;
    a.bflag = c->bflag;
    a.seglist = c->seglist;
    a.count_new = cnt_new;
    a.nsegx = (int)c->nsegx;
    if (c->dim == 2)
      hipLaunchKernelGGL(k_mark<2>, dim3(c->np), dim3(256), 0, c->stream, a);
    else
      hipLaunchKernelGGL(k_mark<3>, dim3(c->np), dim3(256), 0, c->stream, a);
  }
  c->segcur = 1 - b;
}

void ibm_interp(iblbm_ctx* c, int first_pass, int mode) {
  if (c->nmk == 0) return;
  if (c->dim == 2) {
    if (c->fp64) run_interp<2, double>(c, first_pass, mode); else run_interp<2, float>(c, first_pass, mode);
  } else {
    if (c->fp64) run_interp<3, double>(c, first_pass, mode); else run_interp<3, float>(c, first_pass, mode);
  }
}

void ibm_spread(iblbm_ctx* c, int) {
  if (c->nmk == 0) return;
  if (c->dim == 2) {
    if (c->fp64) run_spread<2, double>(c); else run_spread<2, float>(c);
  } else {
    if (c->fp64) run_spread<3, double>(c); else run_spread<3, float>(c);
  }
}

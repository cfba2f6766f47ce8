// Immersed-boundary kernels for gfx950 (Sec. 2.2 and Sec. 4 of the paper).
//
// Each Lagrangian point touches the nodes of its delta-function support only
// (Eqs. 47-48).  Two implementations share the arithmetic:
//
//  - per particle (default): all points of a particle lie at distance R from its
//    centre, so their supports fit in one box of side floor(Xc+R) - floor(Xc-R) + 4.
//    One workgroup per particle keeps that box in LDS.  Interpolation marks the touched
//    nodes, stages u + f/(2 rho0) of exactly those nodes into LDS and gathers every
//    support from LDS; spreading accumulates all contributions with LDS atomics and
//    adds each touched node to the global force once.  The first forcing pass of a
//    step also computes u* (Eq. 5) from the PDFs at the touched nodes, stores it for
//    the later passes, clears the force there and records the touched nodes in the
//    band bitmap that tells the collision where a force is present.
//  - per point (fallback when the box does not fit in LDS): one wavefront serves one
//    point in 3-D (4x4x4 support nodes, a lane each) and four points in 2-D; the band
//    is built beforehand as a list of 16-node row segments.
//
// In the per-particle kernels one lane owns one point: it evaluates the twelve 1-D
// weights of its support once and walks the 4x4x4 support, accumulating in registers
// (interpolation) or with LDS atomics (spreading).
#include <mutex>
#include <set>

#include <hip/hip_ext.h>

#include "index_math.h"
#include "pdf_access.h"

namespace {

using namespace pdf;

struct PartView {
  const double *X, *U, *Om;
  const int* mown;
  const double* mr;  // nmk x 4
  const double* mdV;
  const int* status;  // device status word (the kernels stop once a runaway is flagged)
};

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

// ---------------------------------------------------------------------------
// per-point kernels (fallback)

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
  const int* cond;  // run only when *cond != 0 (if set)
};

// mode 0: a multi-direct-forcing pass (Eqs. 9-10): dF = 2 rho0 (U_b - D_I u), F += dF.
// mode 1: accumulate |U_b - D_I u|^2 for the slip statistic.
// mode 2: write U_b - D_I u into the learned-force features.
// mode 3: mode 0 and mode 1 at once (the correction pass of the learned step, whose
//         slip judges the prediction).
template <class C>
__device__ __forceinline__ void point_result(const InterpArgs<C>& a, int k, const double* Ub,
                                             const C* acc, int DIM) {
  if (a.mode == 3) {
    double s = 0;
    for (int c = 0; c < DIM; c++) {
      double e = Ub[c] - double(acc[c]);
      s += e * e;
    }
    atomicAdd(a.slip2, s);
  }
  if (a.mode == 0 || a.mode == 3) {
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
    for (int c = 0; c < 3; c++)
      a.feat[10 * (size_t)k + c] = c < DIM ? float(Ub[c] - double(acc[c])) : 0.f;
  }
}

template <int DIM, class C>
__global__ __launch_bounds__(256) void k_interp(InterpArgs<C> a) {
  if ((a.cond && *a.cond == 0) || halted(a.P.status)) return;
  constexpr int G = DIM == 3 ? 64 : 16;
  int k = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  int l = threadIdx.x & (G - 1);
  bool active = k < a.nmk;
  double X[3] = {0, 0, 0}, Ub[3] = {0, 0, 0};
  if (active) marker_pos_vel(a.P, k, X, Ub, DIM);
  C acc[3] = {0, 0, 0};
  bool tr = false;
  if (active) {
    C w;
    int i = support_node<DIM, C>(a.g, X, l, w, tr);
    if (i >= 0) {
      const C* u = a.ustar + (size_t)i * a.vd;
      const C* f = a.facc + (size_t)i * a.vd;
      for (int c = 0; c < DIM; c++) acc[c] = w * (u[c] + f[c] * a.half_inv_rho);
    }
  }
  for (int c = 0; c < DIM; c++) acc[c] = group_sum(acc[c], G);
  if (a.first_pass && a.mode == 0) {
    unsigned long long m = __ballot(tr);
    if (l == 0 && m) {
      unsigned long long mine =
          G == 64 ? m : (m >> (threadIdx.x & 63 & ~(G - 1))) & ((1ull << (G & 63)) - 1);
      if (mine) atomicAdd(a.trunc, (unsigned long long)__popcll(mine));
    }
  }
  if (!active || l != 0) return;
  point_result<C>(a, k, Ub, acc, DIM);
}

template <class C>
struct SpreadArgs {
  MarkerGeo g;
  PartView P;
  int nmk;
  const C* dF;  // nmk x 4
  C* facc;
  int vd;
  const int* cond;
};

// Eq. 11 with Eq. 13: f(x) += dF_k Phi(x - X_k) drs ds_k, with float atomics.
template <int DIM, class C>
__global__ __launch_bounds__(256) void k_spread(SpreadArgs<C> a) {
  if ((a.cond && *a.cond == 0) || halted(a.P.status)) return;
  constexpr int G = DIM == 3 ? 64 : 16;
  int k = (blockIdx.x * blockDim.x + threadIdx.x) / G;
  int l = threadIdx.x & (G - 1);
  if (k >= a.nmk) return;
  double X[3] = {0, 0, 0}, Ub[3];
  marker_pos_vel(a.P, k, X, Ub, DIM);
  C w;
  bool tr;
  int i = support_node<DIM, C>(a.g, X, l, w, tr);
  if (i < 0) return;
  C s = w * C(a.P.mdV[k]);
  const C* dF = a.dF + 4 * (size_t)k;
  C* f = a.facc + (size_t)i * a.vd;
  for (int c = 0; c < DIM; c++) unsafeAtomicAdd(f + c, dF[c] * s);
}

struct MarkArgs {
  MarkerGeo g;
  PartView P;
  const double* D;
  const int *mstart, *mcount;
  uint32_t* bflag;
  int* seglist;
  int* count;
  int nsegx;
  int words;  // LDS bitmap words: segments x rows of the largest particle's box
};

// Fallback band: one workgroup per particle collects the row segments touched by the
// supports of its points in an LDS bitmap, then flags and lists each new segment once.
template <int DIM>
__global__ __launch_bounds__(256) void k_mark(MarkArgs a) {
  if (halted(a.P.status)) return;
  extern __shared__ uint32_t bits[];
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
      lo[d] = max(floor_idx(xc - R) - 2, 0);
      hi[d] = min(floor_idx(xc + R) + 3, a.g.n[d] - 1);
    }
    box[0] = lo[0] / SEG;
    box[1] = hi[0] / SEG;
    box[2] = lo[1];
    box[3] = hi[1];
    box[4] = lo[2];
    box[5] = hi[2];
  }
  for (int w = threadIdx.x; w < a.words; w += blockDim.x) bits[w] = 0;
  __syncthreads();
  int nsx = box[1] - box[0] + 1, ny = box[3] - box[2] + 1, nz = box[5] - box[4] + 1;
  long long nbits = (long long)nsx * ny * nz;
  bool direct = nbits > 32LL * a.words || nsx <= 0 || ny <= 0 || nz <= 0;
  for (int t = threadIdx.x; t < mc * 16; t += blockDim.x) {
    int k = m0 + t / 16, row = t % 16;
    if ((row & 3) >= a.g.width || (DIM == 3 && (row >> 2) >= a.g.width) || (DIM == 2 && row >= 4))
      continue;
    double X[3], Ub[3];
    marker_pos_vel(a.P, k, X, Ub, DIM);
    int l0[3] = {0, 0, 0};
    for (int d = 0; d < DIM; d++)
      l0[d] = a.g.kind == 0 ? floor_idx(X[d]) - 1 : floor_idx(X[d] + 0.5) - 1;
    int yy = l0[1] + (row & 3), zz = DIM == 3 ? l0[2] + (row >> 2) : 0;
    if (yy < 0 || yy >= a.g.n[1] || zz < 0 || zz >= a.g.n[2]) continue;
    int xa = max(l0[0], 0), xb = min(l0[0] + a.g.width - 1, a.g.n[0] - 1);
    if (xa > xb) continue;
    for (int sx = xa / SEG; sx <= xb / SEG; sx++) {
      if (direct) {
        int seg = sx + a.nsegx * (yy + a.g.n[1] * zz);
        if (atomicOr(&a.bflag[seg], 1u) == 0u) a.seglist[atomicAdd(a.count, 1)] = seg;
      } else {
        long long bit = (long long)(sx - box[0]) + nsx * ((long long)(yy - box[2]) + ny * (zz - box[4]));
        atomicOr(&bits[bit >> 5], 1u << (bit & 31));
      }
    }
  }
  __syncthreads();
  if (direct) return;
  for (long long bit = threadIdx.x; bit < nbits; bit += blockDim.x) {
    if (!((bits[bit >> 5] >> (bit & 31)) & 1u)) continue;
    int sx = int(bit % nsx) + box[0];
    long long r = bit / nsx;
    int yy = int(r % ny) + box[2], zz = int(r / ny) + box[4];
    int seg = sx + a.nsegx * (yy + a.g.n[1] * zz);
    if (atomicOr(&a.bflag[seg], 1u) == 0u) a.seglist[atomicAdd(a.count, 1)] = seg;
  }
}

// clear the segment flags listed at the previous step and reset the list
__global__ void k_clear(uint32_t* bflag, const int* seglist, int* count) {
  int n = *count;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x)
    bflag[seglist[s]] = 0u;
}
__global__ void k_reset_count(int* count) { *count = 0; }

// ---------------------------------------------------------------------------
// per-particle kernels

// static LDS of the interpolation kernel beside its dynamic box: one double per wavefront
constexpr size_t INTERP_STATIC_LDS = (LDS_THREADS / 64) * sizeof(double);

template <class C>
struct LdsArgs {
  MarkerGeo g;
  PartView P;
  const double* D;
  const int *mstart, *mcount;
  int cap;  // node capacity of the LDS box arrays
  C* ustar;
  C* facc;
  int vd;
  C half_inv_rho, two_rho;
  C* F;
  C* dF;
  int first_pass, mode;
  unsigned long long* trunc;
  double* slip2;
  float* feat;
  uint32_t* bmap;  // band bitmap of this step (bit per node, 32-node words per row)
  int nwx;         // words per row
  const int* cond; // run only when *cond != 0 (if set)
  int mcap;        // points of the largest particle
  uint16_t* tlist; // touched box nodes per work unit (cap entries each), ascending
  int* tcount;
  double* slip_part;  // per-unit sums of |U_b - D_I u|^2 (interpolation modes 1 and 3)
  // work units: with patched == 0 the unit is the particle (box of +-D/2); otherwise
  // unit q is the run of pt_mc[q] points from pt_m0[q] of particle pt_owner[q], with the
  // box of the offset range [pt_rlo, pt_rhi]
  int patched;
  const int *pt_owner, *pt_m0, *pt_mc;
  const double *pt_rlo, *pt_rhi;
  // PDF access for the first pass
  Geo<C> geo;
  SlotPtrs slot;
  C inv_s;
};

// The work unit of block q: its particle, first point, point count and box.
template <int DIM, class C>
__device__ __forceinline__ void unit_of(const LdsArgs<C>& a, int q, int& p, int& m0, int& mc,
                                        PBox<DIM>& b) {
  if (a.patched) {
    p = a.pt_owner[q];
    m0 = a.pt_m0[q];
    mc = a.pt_mc[q];
  } else {
    p = q;
    m0 = a.mstart[p];
    mc = a.mcount[p];
  }
  const double Xc[3] = {a.P.X[3 * p], a.P.X[3 * p + 1], DIM == 3 ? a.P.X[3 * p + 2] : 0.0};
  if (a.patched)
    b = range_box<DIM>(Xc, a.pt_rlo + 3 * (size_t)q, a.pt_rhi + 3 * (size_t)q, a.g.kind);
  else
    b = particle_box<DIM>(Xc, 0.5 * a.D[p], a.g.kind);
}


// List entries a lane loads before it uses any of them, so that their global-memory
// latencies overlap.
constexpr int LIST_BATCH = 4;
// nodes whose PDFs a lane of the first interpolation pass loads before it uses any
constexpr int FIRST_BATCH = 3;

// LDS layout of the per-particle interpolation kernel (the host sizes the dynamic LDS
// with the same function): C ub[DIM][cap] staged velocities, uint8 flag[cap] touched
// nodes, uint16 list[cap] the touched nodes in ascending order, int wcnt[17] per-wave
// counts.
struct InterpLayout {
  size_t flag, list, wcnt, total;
};
__host__ __device__ inline InterpLayout interp_layout(int dim, size_t cs, int cap) {
  InterpLayout L;
  size_t o = ((size_t)dim * cap * cs + 7) & ~(size_t)7;
  L.flag = o;
  o += ((size_t)cap + 3) & ~(size_t)3;
  L.list = o;
  o += ((size_t)cap * 2 + 3) & ~(size_t)3;
  L.wcnt = o;
  o += 17 * 4;
  L.total = o;
  return L;
}

// List the flagged nodes of a box in ascending order into out[] (ballot compaction: each
// wave scans one chunk of the box, then writes at its offset); returns the count.  The
// whole block calls it; wcnt holds 17 ints.
__device__ inline int list_flags(const uint8_t* flag, int n, uint16_t* out, int* wcnt) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int chunk = ((n + nw - 1) / nw + 63) & ~63;
  const int c0 = wid * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
  int cnt = 0;
  for (int t0 = c0; t0 < c1; t0 += 64) {
    const int t = t0 + lane;
    cnt += __popcll(__ballot(t < c1 && flag[t]));
  }
  if (lane == 0) wcnt[wid] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int v = 0; v < nw; v++) {
      int k = wcnt[v];
      wcnt[v] = s;
      s += k;
    }
    wcnt[16] = s;
  }
  __syncthreads();
  int pos = wcnt[wid];
  for (int t0 = c0; t0 < c1; t0 += 64) {
    const int t = t0 + lane;
    const bool f = t < c1 && flag[t];
    const unsigned long long m = __ballot(f);
    if (f) out[pos + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)t;
    pos += __popcll(m);
  }
  __syncthreads();
  return wcnt[16];
}

// Set the flagged nodes of a particle's box in the band bitmap, one lane per box row and
// one atomic per (row, 32-node word).  A row of the box spans any number of words: the
// lane walks the row in x order and flushes each word's mask when the next word begins.
// Flagged nodes lie inside the walls (the supports skip wall nodes), so x stays in
// [0, n0) and the word stays inside the row.
template <int DIM>
__device__ __forceinline__ void band_rows(const MarkerGeo& g, const PBox<DIM>& b,
                                          const uint8_t* flag, uint32_t* bmap, int nwx) {
  int rows = b.B[1] * b.B[2];
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    int y = b.lo[1] + r % b.B[1], z = b.lo[2] + r / b.B[1];
    if (y < 0 || y >= g.n[1] || z < 0 || z >= g.n[2]) continue;
    uint32_t* row = bmap + (size_t)nwx * (y + g.n[1] * z);
    int wcur = -1;
    uint32_t m = 0u;
    for (int xl = 0; xl < b.B[0]; xl++) {
      if (!flag[xl + b.B[0] * r]) continue;
      const int x = b.lo[0] + xl;
      if (x < 0 || x >= g.n[0]) continue;
      const int wi = x >> 5;
      if (wi != wcur) {
        if (m) atomicOr(row + wcur, m);
        wcur = wi;
        m = 0u;
      }
      m |= 1u << (x & 31);
    }
    if (m) atomicOr(row + wcur, m);
  }
}

// Interpolation (+ point force) for one forcing pass through the particle's LDS box.
// The touched nodes of the step are listed in ascending order (so that neighbouring
// lanes stage neighbouring nodes), staged into LDS as u = u* + f/(2 rho0) (Eq. 7), and
// gathered by one lane per point.  Later passes (FIRST = 0) take the list from the step's
// first pass, u* from the lattice u* array.  The first pass (FIRST = 1, 2) makes the band:
// the nodes are flagged (one lane per point), listed by ballot compaction and kept for
// the later passes, their force is cleared, and they enter the band bitmap; u* comes from
// their PDFs (FIRST = 1) or from the lattice u* array (FIRST = 2).
template <int DIM, class T, int PAR, int FIRST>
__global__ __launch_bounds__(LDS_THREADS) void k_interp_lds(LdsArgs<typename Store<T>::C> a) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  extern __shared__ double smem_d[];
  if (a.cond && *a.cond == 0) return;
  // tested with the box below, so that its load overlaps the particle's
  const bool stop = halted(a.P.status);
  char* base = reinterpret_cast<char*>(smem_d);
  const InterpLayout Ly = interp_layout(DIM, sizeof(C), a.cap);
  C* ub = reinterpret_cast<C*>(base);
  // touched-node flags, one byte per box node: every writer stores 1, so concurrent
  // plain stores need no atomics
  uint8_t* flag = reinterpret_cast<uint8_t*>(base + Ly.flag);
  uint16_t* list = reinterpret_cast<uint16_t*>(base + Ly.list);
  int* wcnt = reinterpret_cast<int*>(base + Ly.wcnt);
  const int q = blockIdx.x;
  int p, m0, mc;
  PBox<DIM> b;
  unit_of<DIM>(a, q, p, m0, mc, b);
  // the host sizes cap and the block for the largest unit
  if (stop || b.n > a.cap || mc > (int)blockDim.x) {
    if ((a.mode == 1 || a.mode == 3) && threadIdx.x == 0) a.slip_part[q] = 0.0;
    return;
  }
  // this lane's point, loaded and weighted before the box is staged so that the
  // latencies overlap; with an accumulating pass also its force so far
  const int k = m0 + (int)threadIdx.x;
  const bool has = (int)threadIdx.x < mc;
  double X[3] = {0, 0, 0}, Ub[3] = {0, 0, 0};
  PointWeights<C> pw;
  C Fold[3] = {C(0), C(0), C(0)};
  if (has) {
    marker_pos_vel(a.P, k, X, Ub, DIM);
    if ((a.mode == 0 || a.mode == 3) && !a.first_pass) {
#pragma unroll
      for (int c = 0; c < DIM; c++) Fold[c] = a.F[4 * (size_t)k + c];
    }
    point_weights<DIM, C>(a.g.kind, X, pw);
  }
  uint16_t* tl = a.tlist + (size_t)q * a.cap;
  int ntouch;
  const uint16_t* nodes;
  if (FIRST) {
    // the touched nodes of this step, kept for the later passes
    for (int t = threadIdx.x; t < (b.n + 3) / 4; t += blockDim.x) reinterpret_cast<uint32_t*>(flag)[t] = 0u;
    __syncthreads();
    if (has) visit_support<DIM, C>(a.g, b, pw, [&](int loc, C) { flag[loc] = 1; });
    __syncthreads();
    ntouch = list_flags(flag, b.n, list, wcnt);
    if (threadIdx.x == 0) a.tcount[q] = ntouch;
    for (int j = threadIdx.x; j < ntouch; j += blockDim.x) tl[j] = list[j];
    nodes = list;
  } else {
    ntouch = a.tcount[q];
    nodes = tl;
  }
  T* slot[L::Q - 1];
  if (FIRST == 1) slots_of<DIM, T>(a.slot, slot);
  if (FIRST == 2) {
    // u* of the listed nodes from the lattice u* array; their force starts at zero
    for (int j0 = threadIdx.x; j0 < ntouch; j0 += LIST_BATCH * blockDim.x) {
      int t[LIST_BATCH];
      size_t ii[LIST_BATCH];
      typename NodeVec<C, DIM>::T us[LIST_BATCH];
#pragma unroll
      for (int u = 0; u < LIST_BATCH; u++) {
        const int j = j0 + u * (int)blockDim.x;
        t[u] = j < ntouch ? (int)nodes[j] : -1;
        if (t[u] < 0) continue;
        int x, y, z;
        b.at(t[u], x, y, z);
        ii[u] = (size_t)(x + a.g.n[0] * (y + a.g.n[1] * z)) * a.vd;
        us[u] = load_node<DIM>(a.ustar, ii[u]);
      }
#pragma unroll
      for (int u = 0; u < LIST_BATCH; u++) {
        if (t[u] < 0) continue;
#pragma unroll
        for (int c = 0; c < DIM; c++) ub[c * a.cap + t[u]] = comp<C>(us[u], c);
        const C zero[3] = {C(0), C(0), C(0)};
        store_node<DIM>(a.facc, ii[u], zero);
      }
    }
  } else if (FIRST == 1) {
    // u* from the PDFs at the listed nodes (Eqs. 4-5); the force there starts at zero.
    // FIRST_BATCH nodes per lane at a time, their PDF loads issued before any is used, so
    // that the loads of several nodes share one memory latency
    for (int j0 = threadIdx.x; j0 < ntouch; j0 += FIRST_BATCH * blockDim.x) {
      int t[FIRST_BATCH], ii[FIRST_BATCH];
      C f[FIRST_BATCH][L::Q];
#pragma unroll
      for (int v = 0; v < FIRST_BATCH; v++) {
        const int j = j0 + v * (int)blockDim.x;
        t[v] = j < ntouch ? (int)nodes[j] : -1;
        if (t[v] < 0) continue;
        int x, y, z;
        b.at(t[v], x, y, z);
        ii[v] = x + a.g.n[0] * (y + a.g.n[1] * z);
        load_all<DIM, T, PAR>(slot, a.geo, x, y, z, ii[v], a.inv_s, f[v]);
      }
#pragma unroll
      for (int v = 0; v < FIRST_BATCH; v++) {
        if (t[v] < 0) continue;
        const size_t i = (size_t)ii[v] * a.vd;
        C S, u[3];
        moments<DIM, C>(f[v], a.geo.rho0, S, u);
#pragma unroll
        for (int c = 0; c < DIM; c++) ub[c * a.cap + t[v]] = u[c];
        store_node<DIM>(a.ustar, i, u);
        const C zero[3] = {C(0), C(0), C(0)};
        store_node<DIM>(a.facc, i, zero);
      }
    }
  } else {
    // u* + F / (2 rho0) at the listed nodes, LIST_BATCH entries per lane at a time
    for (int j0 = threadIdx.x; j0 < ntouch; j0 += LIST_BATCH * blockDim.x) {
      int t[LIST_BATCH];
#pragma unroll
      for (int u = 0; u < LIST_BATCH; u++) {
        const int j = j0 + u * (int)blockDim.x;
        t[u] = j < ntouch ? (int)nodes[j] : -1;
      }
      typename NodeVec<C, DIM>::T us[LIST_BATCH], fa[LIST_BATCH];
#pragma unroll
      for (int u = 0; u < LIST_BATCH; u++) {
        if (t[u] < 0) continue;
        int x, y, z;
        b.at(t[u], x, y, z);
        const size_t i = (size_t)(x + a.g.n[0] * (y + a.g.n[1] * z)) * a.vd;
        us[u] = load_node<DIM>(a.ustar, i);
        // the step's first pass finds the force cleared at every listed node: not read
        if (!a.first_pass) fa[u] = load_node<DIM>(a.facc, i);
      }
#pragma unroll
      for (int u = 0; u < LIST_BATCH; u++) {
        if (t[u] < 0) continue;
#pragma unroll
        for (int c = 0; c < DIM; c++)
          ub[c * a.cap + t[u]] = a.first_pass ? comp<C>(us[u], c)
                                              : comp<C>(us[u], c) + comp<C>(fa[u], c) * a.half_inv_rho;
      }
    }
  }
  if (FIRST) band_rows<DIM>(a.g, b, flag, a.bmap, a.nwx);
  __syncthreads();
  // gather each support from LDS (Eq. 9 with Eq. 12) and form the point force (Eq. 10)
  unsigned long long ntr = 0;
  double s2 = 0.0;  // mode 1: this lane's |U_b - D_I u|^2
  if (has) {
    C acc[3] = {0, 0, 0};
    ntr += visit_support<DIM, C>(a.g, b, pw, [&](int loc, C w) {
#pragma unroll
      for (int c = 0; c < DIM; c++) acc[c] += w * ub[c * a.cap + loc];
    });
    if (a.mode == 1 || a.mode == 3) {
      for (int c = 0; c < DIM; c++) {
        double e = Ub[c] - double(acc[c]);
        s2 += e * e;
      }
    }
    if (a.mode == 0 || a.mode == 3) {
      C* F = a.F + 4 * (size_t)k;
      C* dF = a.dF + 4 * (size_t)k;
      for (int c = 0; c < DIM; c++) {
        C d = a.two_rho * (C(Ub[c]) - acc[c]);
        dF[c] = d;
        F[c] = a.first_pass ? d : Fold[c] + d;
      }
    } else if (a.mode == 2) {
      for (int c = 0; c < 3; c++)
        a.feat[10 * (size_t)k + c] = c < DIM ? float(Ub[c] - double(acc[c])) : 0.f;
    }
  }
  if (a.mode == 1 || a.mode == 3) {
    // the unit's sum, over each wavefront (blocks are whole wavefronts) and then over the
    // wavefronts in order, stored for a fixed-order sum over the units: atomics on the
    // one global word serialise (about 9 ns each at 256^3), and the order is fixed
    __shared__ double wsum[INTERP_STATIC_LDS / sizeof(double)];
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += wsum[w];
      a.slip_part[q] = t;
    }
  }
  if (a.first_pass && a.mode == 0 && ntr) atomicAdd(a.trunc, ntr);
}

// Fixed-point accumulators of the spreading kernel: 32-bit for FP32 (and for the 16-bit
// storage forms, which compute in FP32), 64-bit for FP64.  Integer additions are exact
// and associative, so a node's sum does not depend on the order of its contributions,
// and integer LDS atomics run at full rate on gfx950, where float LDS atomics do not.
template <class C>
struct Fixed;
template <>
struct Fixed<float> {
  using U = unsigned int;
  static constexpr int BITS = 30;  // |node sum| < 2^30
  static constexpr int EMAX = 100; // largest scale exponent (keeps 2^-e a normal float)
  __device__ static U quant(float x) { return (U)__float2int_rn(x); }
  __device__ static float value(U u) { return float((int)u); }
};
template <>
struct Fixed<double> {
  using U = unsigned long long;
  static constexpr int BITS = 62;
  static constexpr int EMAX = 900;
  __device__ static U quant(double x) { return (U)__double2ll_rn(x); }
  __device__ static double value(U u) { return double((long long)u); }
};

// dynamic LDS of the spreading kernel: Fixed<C>::U acc[DIM][cap], then double red[16]
// and uint16 list[cap]
__host__ __device__ inline size_t spread_acc_bytes(int dim, size_t cs, int cap) {
  return ((size_t)dim * cap * (cs == 8 ? 8 : 4) + 7) & ~(size_t)7;
}

// Spreading of one forcing pass (Eq. 11 with Eq. 13) through the particle's LDS box,
// one lane per point.  The box holds fixed-point sums: the scale 2^e is chosen per
// particle so that the sum of max_c |F_c drs ds| over all points, times the largest
// product of 1-D weights, stays below 2^BITS; no node sum can exceed it, so none
// overflows.  Each touched node of the step's list then reaches the global force once,
// one lane per (node, component) so that neighbouring lanes hit neighbouring addresses.
template <int DIM, class C>
__global__ __launch_bounds__(LDS_THREADS) void k_spread_lds(LdsArgs<C> a) {
  using FX = Fixed<C>;
  using U = typename FX::U;
  extern __shared__ double smem_d[];
  if (a.cond && *a.cond == 0) return;
  // tested with the box below, so that its load overlaps the particle's
  const bool stop = halted(a.P.status);
  U* acc = reinterpret_cast<U*>(smem_d);
  double* red = reinterpret_cast<double*>(reinterpret_cast<char*>(smem_d) +
                                          spread_acc_bytes(DIM, sizeof(C), a.cap));
  const int q = blockIdx.x;
  int p, m0, mc;
  PBox<DIM> b;
  unit_of<DIM>(a, q, p, m0, mc, b);
  // the host sizes the box and the block for the largest unit
  if (stop || b.n > a.cap || mc > (int)blockDim.x) return;
  const int kind = a.g.kind, width = a.g.width;
  // this lane's point: 1-D weights, first support node, force times drs*ds (Eq. 13)
  const int kl = threadIdx.x;
  const bool has = kl < mc;
  C w[3][4] = {};
  int g0[3] = {0, 0, 0};
  C F[3] = {C(0), C(0), C(0)};
  double mag = 0.0;
  if (has) {
    const int k = m0 + kl;
    double X[3], Ub[3];
    marker_pos_vel(a.P, k, X, Ub, DIM);
    const C* d = a.dF + 4 * (size_t)k;
    const C dV = C(a.P.mdV[k]);
    const C sc = axis_scale<C>(kind);
#pragma unroll
    for (int ax = 0; ax < DIM; ax++) {
      C f, s;
      g0[ax] = axis_fs<C>(kind, X[ax], f, s);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const AxisForm<C> fm = axis_form<C>(kind, q);
        w[ax][q] = (fm.k0 + fm.k1 * f + fm.k2 * s) * sc;
      }
    }
#pragma unroll
    for (int c = 0; c < DIM; c++) {
      F[c] = d[c] * dV;
      mag = fmax(mag, fabs(double(F[c])));
    }
  }
  // the touched nodes of the step (listed by the step's first interpolation pass),
  // copied into LDS after the point loads above are issued, so that the latencies overlap
  uint16_t* tl = reinterpret_cast<uint16_t*>(red + 16);
  const uint16_t* gl = a.tlist + (size_t)q * a.cap;
  const int ntouch = a.tcount[q];
  for (int j0 = threadIdx.x; j0 < ntouch; j0 += LIST_BATCH * blockDim.x) {
    int t[LIST_BATCH];
#pragma unroll
    for (int u = 0; u < LIST_BATCH; u++) {
      const int j = j0 + u * (int)blockDim.x;
      t[u] = j < ntouch ? (int)gl[j] : -1;
    }
#pragma unroll
    for (int u = 0; u < LIST_BATCH; u++) {
      if (t[u] < 0) continue;
      tl[j0 + u * blockDim.x] = (uint16_t)t[u];
#pragma unroll
      for (int c = 0; c < DIM; c++) acc[c * a.cap + t[u]] = U(0);
    }
  }
  for (int o = 32; o > 0; o >>= 1) mag += __shfl_xor(mag, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mag;
  __syncthreads();
  double bound = 0.0;
  for (int v = 0; v < (int)(blockDim.x >> 6); v++) bound += red[v];
  // largest 1-D weight: 1/2 (Peskin, at r = 0) or 2/3 (Roma); 1% margin for rounding
  const double wmax = kind == 0 ? 0.5 : 2.0 / 3.0;
  bound *= 1.01 * (DIM == 3 ? wmax * wmax * wmax : wmax * wmax);
  int e = bound > 0.0 ? FX::BITS - 1 - ilogb(bound) : 0;
  e = e > FX::EMAX ? FX::EMAX : e;
  const C scale = C(ldexp(1.0, e)), inv = C(ldexp(1.0, -e));
  // a point whose whole support lies inside the lattice and the box (all but those next
  // to a wall) adds without per-node tests; scaling by 2^e is exact, so F scale ww equals
  // the F ww scale of the general loop bit for bit
  bool whole = has;
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    const int wd = ax < DIM ? width : 1;
    whole = whole && g0[ax] >= 0 && g0[ax] + wd <= a.g.n[ax] && g0[ax] >= b.lo[ax] &&
            g0[ax] + wd <= b.lo[ax] + b.B[ax];
  }
  if (whole) {
    C Fs[3];
#pragma unroll
    for (int c = 0; c < DIM; c++) Fs[c] = F[c] * scale;
    const int t0 = (g0[0] - b.lo[0]) + b.B[0] * ((g0[1] - b.lo[1]) + b.B[1] * (g0[2] - b.lo[2]));
#pragma unroll
    for (int iz = 0; iz < (DIM == 3 ? 4 : 1); iz++)
#pragma unroll
      for (int iy = 0; iy < 4; iy++) {
        if ((DIM == 3 && iz >= width) || iy >= width) continue;
        const int trow = t0 + b.B[0] * (iy + b.B[1] * iz);
        const C wyz = DIM == 3 ? w[1][iy] : C(1);
#pragma unroll
        for (int ix = 0; ix < 4; ix++) {
          if (ix >= width) continue;
          // (phi_x phi_y) phi_z, the product order of Eq. 12
          const C ww = DIM == 3 ? (w[0][ix] * wyz) * w[2][iz] : w[0][ix] * w[1][iy];
#pragma unroll
          for (int c = 0; c < DIM; c++) atomicAdd(&acc[c * a.cap + trow + ix], FX::quant(Fs[c] * ww));
        }
      }
  } else if (has) {
#pragma unroll
    for (int iz = 0; iz < (DIM == 3 ? 4 : 1); iz++)
#pragma unroll
      for (int iy = 0; iy < 4; iy++)
#pragma unroll
        for (int ix = 0; ix < 4; ix++) {
          if ((DIM == 3 && iz >= width) || iy >= width || ix >= width) continue;
          const int gx = g0[0] + ix, gy = g0[1] + iy, gz = g0[2] + iz;
          if (gx < 0 || gx >= a.g.n[0] || gy < 0 || gy >= a.g.n[1] || gz < 0 || gz >= a.g.n[2])
            continue;  // outside the walls: skipped (counted by the interpolation)
          // (phi_x phi_y) phi_z, the product order of Eq. 12
          const C ww = DIM == 3 ? (w[0][ix] * w[1][iy]) * w[2][iz] : w[0][ix] * w[1][iy];
          const int lx = gx - b.lo[0], ly = gy - b.lo[1], lz = gz - b.lo[2];
          if (lx >= 0 && lx < b.B[0] && ly >= 0 && ly < b.B[1] && lz >= 0 && lz < b.B[2]) {
            const int t = lx + b.B[0] * (ly + b.B[1] * lz);
#pragma unroll
            for (int c = 0; c < DIM; c++) atomicAdd(&acc[c * a.cap + t], FX::quant(F[c] * ww * scale));
          } else {
            // a support node outside the box (not produced by the box construction)
            C* f = a.facc + (size_t)(gx + a.g.n[0] * (gy + a.g.n[1] * gz)) * a.vd;
#pragma unroll
            for (int c = 0; c < DIM; c++) unsafeAtomicAdd(f + c, F[c] * ww);
          }
        }
  }
  __syncthreads();
  const int nu = ntouch * DIM;
  for (int u0 = threadIdx.x; u0 < nu; u0 += LIST_BATCH * blockDim.x) {
    int t[LIST_BATCH];
    U q[LIST_BATCH];
#pragma unroll
    for (int v = 0; v < LIST_BATCH; v++) {
      const int u = u0 + v * (int)blockDim.x;
      const int j = u / DIM, c = u - j * DIM;
      t[v] = u < nu ? (int)tl[j] : 0;
      q[v] = u < nu ? acc[c * a.cap + t[v]] : U(0);
    }
#pragma unroll
    for (int v = 0; v < LIST_BATCH; v++) {
      if (q[v] == U(0)) continue;
      const int u = u0 + v * (int)blockDim.x;
      const int c = u - (u / DIM) * DIM;
      int x, y, z;
      b.at(t[v], x, y, z);
      if (x < 0 || x >= a.g.n[0] || y < 0 || y >= a.g.n[1] || z < 0 || z >= a.g.n[2]) continue;
      unsafeAtomicAdd(a.facc + (size_t)(x + a.g.n[0] * (y + a.g.n[1] * z)) * a.vd + c,
                      FX::value(q[v]) * inv);
    }
  }
}

// slip2 += the per-unit sums, in unit order (one block)
__global__ __launch_bounds__(256) void k_sum_units(const double* part, int n, double* slip2) {
  __shared__ double red[256];
  double t = 0.0;
  const int per = (n + 255) / 256, lo = threadIdx.x * per;
  for (int i = lo; i < lo + per && i < n; i++) t += part[i];
  red[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < 256; k++) s += red[k];
    *slip2 += s;
  }
}

// Fallback band u*: at the nodes of every listed segment compute u* from the PDFs,
// clear the force, and mark the segment's nodes in the band bitmap.
template <int DIM, class T, int PAR>
__global__ __launch_bounds__(256) void k_band_prep(LdsArgs<typename Store<T>::C> a,
                                                    const int* seglist, const int* count, int nsegx) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  if ((a.cond && *a.cond == 0) || halted(a.P.status)) return;
  int n = *count;
  int lane = threadIdx.x & (SEG - 1);
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  int groups = gridDim.x * (blockDim.x / SEG);
  for (int s = blockIdx.x * (blockDim.x / SEG) + threadIdx.x / SEG; s < n; s += groups) {
    int seg = seglist[s];
    int sx = seg % nsegx, row = seg / nsegx;
    int x = sx * SEG + lane;
    if (lane == 0) atomicOr(a.bmap + (size_t)a.nwx * row + (x >> 5), 0xffffu << (x & 31));
    if (x >= a.g.n[0]) continue;
    int y = row % a.g.n[1], z = row / a.g.n[1];
    int i = x + a.g.n[0] * row;
    C f[L::Q];
    load_all<DIM, T, PAR>(slot, a.geo, x, y, z, i, a.inv_s, f);
    C S, us[3];
    moments<DIM, C>(f, a.geo.rho0, S, us);
    C* u = a.ustar + (size_t)i * a.vd;
    C* fa = a.facc + (size_t)i * a.vd;
    for (int c = 0; c < DIM; c++) {
      u[c] = us[c];
      fa[c] = C(0);
    }
  }
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
  P.status = c->dstatus;
  return P;
}

template <class C>
InterpArgs<C> make_interp_args(iblbm_ctx* c, int first, int mode) {
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
  a.cond = c->cond;
  return a;
}

// points of the largest particle
// points of the largest work unit
int max_points(const iblbm_ctx* c) {
  int mx = 1;
  for (int m : c->hpt_mc) mx = m > mx ? m : mx;
  return mx;
}

template <class T>
LdsArgs<typename Store<T>::C> make_lds_args(iblbm_ctx* c, int first, int mode) {
  using C = typename Store<T>::C;
  LdsArgs<C> a;
  a.g = make_mgeo(c);
  a.P = make_pview(c);
  a.D = c->D;
  a.mstart = c->mstart;
  a.mcount = c->mcount;
  a.cap = c->box_cap;
  a.ustar = (C*)c->ustar;
  a.facc = (C*)c->facc;
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
  a.bmap = c->bmap + (size_t)c->fbuf * c->nwords;
  a.nwx = (int)c->nwx;
  a.cond = c->cond;
  a.mcap = max_points(c);
  a.tlist = c->tlist;
  a.tcount = c->tcount;
  a.slip_part = c->slip_part;
  a.patched = c->patched ? 1 : 0;
  a.pt_owner = c->pt_owner;
  a.pt_m0 = c->pt_m0;
  a.pt_mc = c->pt_mc;
  a.pt_rlo = c->pt_rlo;
  a.pt_rhi = c->pt_rhi;
  a.geo = make_geo<C>(c);
  a.slot = make_slots(c);
  a.inv_s = inv_scale<T>(c);
  return a;
}

// one lane per point of the largest particle (at most 16 waves)
int lds_threads(const iblbm_ctx* c) {
  int t = ((max_points(c) + 63) / 64) * 64;
  return t < 64 ? 64 : (t > LDS_THREADS ? LDS_THREADS : t);
}

// dynamic LDS of the per-particle kernels: interpolation stages DIM velocity
// components and a flag byte per box node; spreading keeps fixed-point sums per node
// and component plus a small reduction area
size_t lds_bytes(const iblbm_ctx* c, size_t cs, bool interp) {
  if (interp) return interp_layout(c->dim, cs, c->box_cap).total;
  return spread_acc_bytes(c->dim, cs, c->box_cap) + 16 * sizeof(double) +
         (((size_t)c->box_cap * 2 + 7) & ~(size_t)7);
}

// interpolation: one lane per point; in 3-D also enough lanes to stage the touched
// nodes of a box (about an eighth of it) in a few rounds (2-D boxes are small, and
// one-wave blocks keep more particles per compute unit)
int interp_threads(const iblbm_ctx* c) {
  long long m = std::max<long long>(max_points(c), c->dim == 3 ? c->box_cap / 8 : 0);
  long long t = ((m + 63) / 64) * 64;
  return (int)std::min<long long>(std::max<long long>(t, 64), LDS_THREADS);
}

// Raise a kernel's dynamic-LDS limit to the device maximum, once per kernel: a
// host-side attribute, so that launches recorded into a graph set none.
void raise_lds_limit(const void* k, int bytes) {
  static std::mutex mu;
  static std::set<const void*> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count(k)) return;
  (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  done.insert(k);
}

template <int DIM, class T>
struct RunInterp {
  static void limits(iblbm_ctx* c) {
    // the dynamic limit leaves room for the kernel's static LDS
    const int dyn = c->lds_max - (int)INTERP_STATIC_LDS;
    raise_lds_limit((const void*)k_interp_lds<DIM, T, 0, 0>, dyn);
    raise_lds_limit((const void*)k_interp_lds<DIM, T, 0, 1>, dyn);
    raise_lds_limit((const void*)k_interp_lds<DIM, T, 1, 1>, dyn);
    raise_lds_limit((const void*)k_interp_lds<DIM, T, 0, 2>, dyn);
  }
  static void run(iblbm_ctx* c, int first, int mode, bool* done) {
    using C = typename Store<T>::C;
    *done = false;
    size_t bytes = lds_bytes(c, sizeof(C), true);
    if (!ibm_uses_lds(c)) return;
    auto a = make_lds_args<T>(c, first, mode);
    if (c->band_pending == 2) {
      go<0, 2>(c, a, bytes);
    } else if (c->band_pending == 1) {
      if (c->parity == 0) go<0, 1>(c, a, bytes); else go<1, 1>(c, a, bytes);
    } else {
      go<0, 0>(c, a, bytes);
    }
    c->band_pending = 0;
    *done = true;
  }
  template <int PAR, int FIRST>
  static void go(iblbm_ctx* c, LdsArgs<typename Store<T>::C>& a, size_t bytes) {
    using C = typename Store<T>::C;
    // later passes stage from the step's list: only the velocity box is needed
    if (!FIRST) bytes = ((size_t)DIM * c->box_cap * sizeof(C) + 7) & ~(size_t)7;
    auto k = k_interp_lds<DIM, T, PAR, FIRST>;
    raise_lds_limit((const void*)k, c->lds_max - (int)INTERP_STATIC_LDS);
    hipEvent_t t0, t1;
    if (kernel_events(c, IBLBM_T_INTERP, &t0, &t1))
      hipExtLaunchKernelGGL(k, dim3(c->npatch), dim3(interp_threads(c)), (uint32_t)bytes, c->stream,
                            t0, t1, 0, a);
    else
      hipLaunchKernelGGL(k, dim3(c->npatch), dim3(interp_threads(c)), bytes, c->stream, a);
    if (a.mode == 1 || a.mode == 3)
      hipLaunchKernelGGL(k_sum_units, dim3(1), dim3(256), 0, c->stream, c->slip_part, c->npatch,
                         c->dstats);
  }
};

template <int DIM, class T>
struct RunLdsLimits {
  static void run(iblbm_ctx* c) {
    RunInterp<DIM, T>::limits(c);
    raise_lds_limit((const void*)k_spread_lds<DIM, typename Store<T>::C>, c->lds_max);
  }
};

template <int DIM, class T>
struct RunSpread {
  static void run(iblbm_ctx* c, bool* done) {
    using C = typename Store<T>::C;
    *done = false;
    size_t bytes = lds_bytes(c, sizeof(C), false);
    if (!ibm_uses_lds(c)) return;
    auto a = make_lds_args<T>(c, 0, 0);
    auto k = k_spread_lds<DIM, C>;
    raise_lds_limit((const void*)k, c->lds_max);
    hipEvent_t t0, t1;
    if (kernel_events(c, IBLBM_T_SPREAD, &t0, &t1))
      hipExtLaunchKernelGGL(k, dim3(c->npatch), dim3(lds_threads(c)), (uint32_t)bytes, c->stream,
                            t0, t1, 0, a);
    else
      hipLaunchKernelGGL(k, dim3(c->npatch), dim3(lds_threads(c)), bytes, c->stream, a);
    *done = true;
  }
};

template <int DIM, class T>
struct RunBandPrep {
  static void run(iblbm_ctx* c) {
    auto a = make_lds_args<T>(c, 0, 0);
    int blocks = (int)std::min<long long>(4096, (c->nseg + 15) / 16);
    if (blocks < 1) blocks = 1;
    if (c->parity == 0)
      hipLaunchKernelGGL((k_band_prep<DIM, T, 0>), dim3(blocks), dim3(256), 0, c->stream, a,
                         c->seglist, c->segcount, (int)c->nsegx);
    else
      hipLaunchKernelGGL((k_band_prep<DIM, T, 1>), dim3(blocks), dim3(256), 0, c->stream, a,
                         c->seglist, c->segcount, (int)c->nsegx);
  }
};

template <int DIM, class C>
void run_point_interp(iblbm_ctx* c, int first, int mode) {
  constexpr int per = DIM == 3 ? 4 : 16;
  int blocks = (c->nmk + per - 1) / per;
  hipLaunchKernelGGL((k_interp<DIM, C>), dim3(blocks), dim3(256), 0, c->stream,
                     make_interp_args<C>(c, first, mode));
}

template <int DIM, class C>
void run_point_spread(iblbm_ctx* c) {
  SpreadArgs<C> a;
  a.g = make_mgeo(c);
  a.P = make_pview(c);
  a.nmk = c->nmk;
  a.dF = (const C*)c->mdF;
  a.facc = (C*)c->facc;
  a.vd = c->vd;
  a.cond = c->cond;
  constexpr int per = DIM == 3 ? 4 : 16;
  int blocks = (c->nmk + per - 1) / per;
  hipLaunchKernelGGL((k_spread<DIM, C>), dim3(blocks), dim3(256), 0, c->stream, a);
}

}  // namespace

bool ibm_uses_lds(const iblbm_ctx* c) {
  size_t cs = c->fp64 ? 8 : 4;
  return c->ibm_lds && c->patch_ok && c->box_cap > 0 && c->box_cap <= 65536 &&
         max_points(c) <= LDS_THREADS &&
         lds_bytes(c, cs, true) + INTERP_STATIC_LDS <= (size_t)c->lds_max &&
         lds_bytes(c, cs, false) <= (size_t)c->lds_max;
}

// Band u*: from a lattice-ordered pass over every node after the collision, or at the
// touched nodes inside the first interpolation pass.  The lattice pass is the default in
// 3-D, where the band covers a large part of the lattice and overlapping particle boxes
// would read shared nodes repeatedly, and in 2-D where the units' boxes cover at least
// half the lattice, so that the first pass would read more PDFs than one pass over every
// node (2048^2 with 5340 disks of diameter 20, coverage 0.80: measured 2.6% faster; 4096
// disks of diameter 10, coverage 0.22: 8% slower).
static bool band_pass(const iblbm_ctx* c) {
  if (c->band_pass >= 0) return c->band_pass != 0;
  return c->dim == 3 || c->box_cover >= 0.5;
}

bool ibm_ustar_lattice(const iblbm_ctx* c) { return c->np > 0 && ibm_uses_lds(c) && band_pass(c); }

// Band of this step.  On the per-particle path the first interpolation pass builds it;
// otherwise list the touched segments and compute u* there now.
void ibm_band(iblbm_ctx* c) {
  c->band_pending = 0;
  if (c->np == 0) return;
  if (ibm_uses_lds(c)) {
    // the first interpolation pass marks the band
    if (band_pass(c)) {
      if (!c->ustar_valid) lbm_ustar_all(c);
      c->band_pending = 2;
    } else {
      c->band_pending = 1;
    }
    return;
  }
  hipLaunchKernelGGL(k_clear, dim3(256), dim3(256), 0, c->stream, c->bflag, c->seglist,
                     c->segcount);
  hipLaunchKernelGGL(k_reset_count, dim3(1), dim3(1), 0, c->stream, c->segcount);
  MarkArgs a;
  a.g = make_mgeo(c);
  a.P = make_pview(c);
  a.D = c->D;
  a.mstart = c->mstart;
  a.mcount = c->mcount;
  a.bflag = c->bflag;
  a.seglist = c->seglist;
  a.count = c->segcount;
  a.nsegx = (int)c->nsegx;
  {
    // box side <= floor(D) + 7 nodes, so <= side/16 + 2 segments per row
    int side = c->full_side + 3;
    long long nbits = (long long)(side / SEG + 2) * (c->dim == 3 ? (long long)side * side : side);
    a.words = (int)std::min<long long>((nbits + 31) / 32, 8192);
  }
  if (c->dim == 2)
    hipLaunchKernelGGL(k_mark<2>, dim3(c->np), dim3(256), a.words * 4, c->stream, a);
  else
    hipLaunchKernelGGL(k_mark<3>, dim3(c->np), dim3(256), a.words * 4, c->stream, a);
  dispatch<RunBandPrep>(c);
}

// Recompute u* and clear the force at the band before a forcing redo (the per-particle
// path does it in its first interpolation pass).
void ibm_prepare_launches(iblbm_ctx* c) { dispatch<RunLdsLimits>(c); }

void ibm_band_redo(iblbm_ctx* c) {
  if (c->np == 0) return;
  if (ibm_uses_lds(c)) {
    // the next first pass marks the band again and clears its force; u* is unchanged
    c->band_pending = band_pass(c) ? 2 : 1;
  } else {
    dispatch<RunBandPrep>(c);
  }
}

void ibm_interp(iblbm_ctx* c, int first_pass, int mode) {
  if (c->nmk == 0) return;
  bool done = false;
  dispatch<RunInterp>(c, first_pass, mode, &done);
  if (done) return;
  if (c->dim == 2) {
    if (c->fp64) run_point_interp<2, double>(c, first_pass, mode); else run_point_interp<2, float>(c, first_pass, mode);
  } else {
    if (c->fp64) run_point_interp<3, double>(c, first_pass, mode); else run_point_interp<3, float>(c, first_pass, mode);
  }
}

void ibm_spread(iblbm_ctx* c, int) {
  if (c->nmk == 0) return;
  bool done = false;
  dispatch<RunSpread>(c, &done);
  if (done) return;
  if (c->dim == 2) {
    if (c->fp64) run_point_spread<2, double>(c); else run_point_spread<2, float>(c);
  } else {
    if (c->fp64) run_point_spread<3, double>(c); else run_point_spread<3, float>(c);
  }
}

// Fluid kernels for gfx950: the fused collide + Guo force + A-A in-place stream step,
// the band u* pass of the immersed boundary, and state initialisation / gathers.
//
// Layout: SoA, slot a-1 holds direction a = 1..q-1 for all N nodes (f_0 is never
// needed: it enters neither u* nor p, Sec. 3.1).  A-A pattern: after an even step the
// post-collision value of direction a at node x sits in the opposite slot at x; an odd
// step reads it from the neighbour x - e_a and pushes its own results to x + e_a, so
// each thread reads and writes the same set of locations and the update is in place
// and race free.  Links that leave through a wall bounce back half-way with the
// moving-wall term 2 w_a rho0 (e_a . u_w)/c_s^2.
#include <hip/hip_ext.h>

#include "index_math.h"
#include "pdf_access.h"

namespace {

using namespace pdf;


template <class C>
struct K1Args {
  Geo<C> g;
  SlotPtrs slot;
  const uint32_t* bmap;  // band bitmap of this step: force present at set nodes
  uint32_t* bmap_next;   // next step's bitmap, cleared here
  int nwx;               // 32-node words per row
  const C* facc;
  int vd;
  C omega, kforce, rho0, body[3];
  C inv_s;
  int nbx, bx_shift, nblk, xcd_per;
};

// Fused collision (Eq. 1 with Eqs. 4-8), half-way bounce-back and A-A streaming.
template <int DIM, class T, int PAR, int BX>
__global__ __launch_bounds__(BX) void k_collide_stream(K1Args<typename Store<T>::C> a) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  // XCD-aware order: consecutive logical blocks (adjacent rows) share an XCD and its L2
  int b = blockIdx.x;
  int lb = a.xcd_per > 0 ? (b & 7) * a.xcd_per + (b >> 3) : b;
  int bx = lb % a.nbx, row = lb / a.nbx;
  int x = bx * BX + threadIdx.x;
  int y = row % a.g.n[1], z = row / a.g.n[1];
  if (x >= a.g.n[0]) return;
  int i = x + a.g.n[0] * row;
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  C f[L::Q];
  // odd step: nodes away from every wall take the direct-offset path
  const int sy = a.g.n[0], sz = a.g.n[0] * a.g.n[1];
  const bool inner = PAR == 1 && x > 0 && x < a.g.n[0] - 1 && y > 0 && y < a.g.n[1] - 1 &&
                     (DIM == 2 || (z > 0 && z < a.g.n[2] - 1));
  if (inner)
    load_odd_interior<DIM, T>(slot, i, sy, sz, a.inv_s, f);
  else
    load_all<DIM, T, PAR>(slot, a.g, x, y, z, i, a.inv_s, f);
  C S, us[3];
  moments<DIM, C>(f, a.rho0, S, us);
  const C w0 = C(L::w[0]);
  // Eq. 6 with u*
  C p = (C(1) / C(3)) / (C(1) - w0) *
        (S - a.rho0 * w0 * (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]) * C(1.5));
  // IB force where the band flag is set, plus the uniform body force
  C ff[3] = {a.body[0], a.body[1], a.body[2]};
  int wi = (x >> 5) + a.nwx * row;
  if ((x & 31) == 0) a.bmap_next[wi] = 0u;
  if ((a.bmap[wi] >> (x & 31)) & 1u) {
    const C* fa = a.facc + (size_t)i * a.vd;
    ff[0] += fa[0];
    ff[1] += fa[1];
    if (DIM == 3) ff[2] += fa[2];
  }
  C hr = C(0.5) / a.rho0;
  C u[3] = {us[0] + ff[0] * hr, us[1] + ff[1] * hr, DIM == 3 ? us[2] + ff[2] * hr : C(0)};  // Eq. 7
  C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  C uf = u[0] * ff[0] + u[1] * ff[1] + u[2] * ff[2];
  C post[L::Q];
  // equilibrium (Eq. 4) and forcing (Eq. 8) split into parts even and odd in e_a
  // (Eqs. 37-40): opposite directions share the even part.
#pragma unroll
  for (int d = 1; d <= L::H; d++) {
    const int o = d + L::H;
    C eu = L::ex[d] * u[0] + L::ey[d] * u[1] + (DIM == 3 ? L::ez[d] * u[2] : C(0));
    C ef = L::ex[d] * ff[0] + L::ey[d] * ff[1] + (DIM == 3 ? L::ez[d] * ff[2] : C(0));
    C wd = C(L::w[d]);
    C ce = wd * (C(3) * p + a.rho0 * (C(4.5) * eu * eu - C(1.5) * uu));
    C oe = wd * a.rho0 * C(3) * eu;
    C cf = a.kforce * wd * (C(9) * eu * ef - C(3) * uf);
    C of = a.kforce * wd * C(3) * ef;
    post[d] = f[d] - a.omega * (f[d] - (ce + oe)) + (cf + of);
    post[o] = f[o] - a.omega * (f[o] - (ce - oe)) + (cf - of);
  }
  if (inner)
    store_odd_interior<DIM, T>(slot, i, sy, sz, a.inv_s, post);
  else
    store_all<DIM, T, PAR>(slot, a.g, x, y, z, i, a.inv_s, post);
}

template <class C>
struct GatherArgs {
  Geo<C> g;
  SlotPtrs slot;
  const uint32_t* bmap;
  int nwx;
  const C* facc;
  int vd;
  C inv_s;
  double *p, *u, *force, *fout;
};

// natural-order gather of p, u* (Eqs. 5-6), the band force, and/or all PDFs
template <int DIM, class T, int PAR>
__global__ void k_gather(GatherArgs<typename Store<T>::C> a) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  int x = int(i % a.g.n[0]), row = int(i / a.g.n[0]);
  int y = row % a.g.n[1], z = row / a.g.n[1];
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  C f[L::Q];
  load_all<DIM, T, PAR>(slot, a.g, x, y, z, int(i), a.inv_s, f);
  if (a.fout)
    for (int d = 1; d < L::Q; d++) a.fout[(size_t)(d - 1) * a.g.N + i] = double(f[d]);
  C S, us[3];
  moments<DIM, C>(f, a.g.rho0, S, us);
  const double w0 = L::w[0];
  double uu = double(us[0]) * us[0] + double(us[1]) * us[1] + double(us[2]) * us[2];
  if (a.p) a.p[i] = (1.0 / 3.0) / (1.0 - w0) * (double(S) - double(a.g.rho0) * w0 * uu * 1.5);
  for (int c = 0; c < DIM; c++) {
    if (a.u) a.u[(size_t)c * a.g.N + i] = double(us[c]);
    if (a.force)
      a.force[(size_t)c * a.g.N + i] =
          ((a.bmap[(x >> 5) + a.nwx * row] >> (x & 31)) & 1u) ? double(a.facc[(size_t)i * a.vd + c])
                                                              : 0.0;
  }
}

template <class C>
struct ScatterArgs {
  Geo<C> g;
  SlotPtrs slot;
  C inv_s;
  const double *fin, *p, *u;
};

// write PDFs in the natural (even) layout: given values, or f_eq(p, u) of Eq. 4
template <int DIM, class T>
__global__ void k_scatter(ScatterArgs<typename Store<T>::C> a) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  if (a.fin) {
    for (int d = 1; d < L::Q; d++)
      slot[d - 1][i] = Store<T>::save(C(a.fin[(size_t)(d - 1) * a.g.N + i]), a.inv_s);
    return;
  }
  double p = a.p ? a.p[i] : 0.0;
  double u[3] = {0, 0, 0};
  if (a.u)
    for (int c = 0; c < DIM; c++) u[c] = a.u[(size_t)c * a.g.N + i];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double rho0 = double(a.g.rho0);
  for (int d = 1; d < L::Q; d++) {
    double eu = L::ex[d] * u[0] + L::ey[d] * u[1] + L::ez[d] * u[2];
    double feq = 3.0 * L::w[d] * p + rho0 * L::w[d] * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    slot[d - 1][i] = Store<T>::save(C(feq), a.inv_s);
  }
}

// Inflow and outflow faces (Sec. 6.1) by non-equilibrium extrapolation, after the
// collide-stream kernel: on the face's node layer, the populations the next step reads
// become f_eq(p_b, u_b) + (f - f_eq(p_f, u_f)) at the next node inward x_f (Eq. 4 for
// f_eq, Eqs. 5-6 for p_f and u_f).  A velocity face sets u_b and takes p_b = p_f; a
// pressure face sets p_b and takes u_b = u_f.  One lane per face node.  The lanes write
// only the links into face nodes and read only links into inward nodes, which are never
// face nodes (the extrapolated faces share one axis of at least 3 nodes), so the update
// is race free.
template <class C>
struct FaceArgs {
  Geo<C> g;
  SlotPtrs slot;
  C inv_s, rho0;
  int face, kind;  // kind 1: velocity (ub), 2: pressure (pb)
  C ub[3], pb;
};

template <int DIM, class C>
__device__ __forceinline__ C eq_pressure(C S, const C* u, C rho0) {
  const C w0 = C(Lat<DIM>::w[0]);
  return (C(1) / C(3)) / (C(1) - w0) * (S - rho0 * w0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * C(1.5));
}

template <int DIM, class C>
__device__ __forceinline__ C feq_dir(int d, C p, const C* u, C rho0) {
  using L = Lat<DIM>;
  const C eu = L::ex[d] * u[0] + L::ey[d] * u[1] + (DIM == 3 ? L::ez[d] * u[2] : C(0));
  const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return C(L::w[d]) * (C(3) * p + rho0 * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
}

template <int DIM, class T, int PN>
__global__ __launch_bounds__(256) void k_face_bc(FaceArgs<typename Store<T>::C> a) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  const int ax = a.face / 2, hi = a.face & 1;
  const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;  // the face's own axes
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)a.g.n[o0] * a.g.n[o1]) return;
  int cb[3], cf[3];
  cb[o0] = (int)(k % a.g.n[o0]);
  cb[o1] = (int)(k / a.g.n[o0]);
  cb[ax] = hi ? a.g.n[ax] - 1 : 0;
  for (int d = 0; d < 3; d++) cf[d] = cb[d];
  cf[ax] += hi ? -1 : 1;
  const int ib = cb[0] + a.g.n[0] * (cb[1] + a.g.n[1] * cb[2]);
  const int jf = cf[0] + a.g.n[0] * (cf[1] + a.g.n[1] * cf[2]);
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  C f[L::Q];
  load_all<DIM, T, PN>(slot, a.g, cf[0], cf[1], cf[2], jf, a.inv_s, f);
  C S, uf[3];
  moments<DIM, C>(f, a.rho0, S, uf);
  const C pf = eq_pressure<DIM, C>(S, uf, a.rho0);
  C ub[3] = {uf[0], uf[1], uf[2]};
  C pb = a.pb;
  if (a.kind == 1) {
    for (int d = 0; d < 3; d++) ub[d] = a.ub[d];
    pb = pf;
  }
  C fb[L::Q];
  fb[0] = C(0);
#pragma unroll
  for (int d = 1; d < L::Q; d++)
    fb[d] = feq_dir<DIM, C>(d, pb, ub, a.rho0) + (f[d] - feq_dir<DIM, C>(d, pf, uf, a.rho0));
  set_incoming_all<DIM, T, PN>(slot, a.g, cb[0], cb[1], cb[2], ib, a.inv_s, fb);
}

template <class C>
struct InteriorArgs {
  Geo<C> g;
  SlotPtrs slot;
  C inv_s;
  const double *X, *D;
  double *P, *L;
  const C* ustar;  // u* of every node (FROMU), else computed from the PDFs
  int vd;
  const int* status;  // device status word (the interior pass stops once a runaway is flagged)
};

// u* = sum_a e_a f_a / rho0 (Eq. 5) at every node, from the PDFs after streaming, in
// row order (the A-A access of the step's parity).  The immersed-boundary passes of the
// next step and the interior momentum of the particles read it instead of the PDFs.
template <int DIM, class T, int PAR>
__global__ __launch_bounds__(256) void k_ustar_all(InteriorArgs<typename Store<T>::C> a, int nbx,
                                                   int xcd_per) {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  // XCD-aware order (xcd_per > 0), as in the collide-stream step: adjacent rows share an
  // XCD and its L2
  const int b = blockIdx.x;
  const int lb = xcd_per > 0 ? (b & 7) * xcd_per + (b >> 3) : b;
  const int bx = lb % nbx, row = lb / nbx;
  const int x = bx * 256 + threadIdx.x;
  if (x >= a.g.n[0]) return;
  const int y = row % a.g.n[1], z = row / a.g.n[1];
  const int i = x + a.g.n[0] * row;
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  C f[L::Q];
  const bool inner = PAR == 1 && x > 0 && x < a.g.n[0] - 1 && y > 0 && y < a.g.n[1] - 1 &&
                     (DIM == 2 || (z > 0 && z < a.g.n[2] - 1));
  if (inner)
    load_odd_interior<DIM, T>(slot, i, a.g.n[0], a.g.n[0] * a.g.n[1], a.inv_s, f);
  else
    load_all<DIM, T, PAR>(slot, a.g, x, y, z, i, a.inv_s, f);
  C S, u[3];
  moments<DIM, C>(f, a.g.rho0, S, u);
  store_node<DIM>(const_cast<C*>(a.ustar), (size_t)i * a.vd, u);
}

// Momentum and angular momentum of the fluid inside each particle volume,
// P = sum chi rho0 u*, L = sum chi (x - X_c) x rho0 u*, with chi = clamp(R + 1/2 - |x - X_c|,
// 0, 1): the interior-fluid terms F_f, T_f of Eqs. 14-15 are their changes per step.
// One workgroup per particle, FP64 accumulation and a fixed-order reduction.
template <int DIM, class T, int PAR, int FROMU>
__global__ __launch_bounds__(256) void k_interior(InteriorArgs<typename Store<T>::C> a) {
  // tested once the particle's loads are issued, so that the latencies overlap
  const bool stop = halted(a.status);
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  __shared__ double red[6][256];
  int p = blockIdx.x;
  double Xc[3] = {a.X[3 * p], a.X[3 * p + 1], DIM == 3 ? a.X[3 * p + 2] : 0.0};
  double R = 0.5 * a.D[p];
  int lo[3], hi[3];
  interior_box(Xc, R, a.g.n, DIM, lo, hi);
  int wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, wz = hi[2] - lo[2] + 1;
  int total = (wx > 0 && wy > 0 && wz > 0) ? wx * wy * wz : 0;
  if (stop) return;
  T* slot[L::Q - 1];
  slots_of<DIM, T>(a.slot, slot);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double rho0 = double(a.g.rho0);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int x = lo[0] + t % wx, y = lo[1] + (t / wx) % wy, z = lo[2] + t / (wx * wy);
    double r[3] = {x - Xc[0], y - Xc[1], DIM == 3 ? z - Xc[2] : 0.0};
    double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double chi = R + 0.5 - sqrt(d2);
    if (chi <= 0.0) continue;
    chi = chi > 1.0 ? 1.0 : chi;
    int i = x + a.g.n[0] * (y + a.g.n[1] * z);
    C us[3] = {C(0), C(0), C(0)};
    if (FROMU) {
#pragma unroll
      for (int c = 0; c < DIM; c++) us[c] = a.ustar[(size_t)i * a.vd + c];
    } else {
      C f[L::Q];
      load_all<DIM, T, PAR>(slot, a.g, x, y, z, i, a.inv_s, f);
      C S;
      moments<DIM, C>(f, a.g.rho0, S, us);
    }
    double m[3] = {chi * (rho0 * double(us[0])), chi * (rho0 * double(us[1])),
                   DIM == 3 ? chi * (rho0 * double(us[2])) : 0.0};
    acc[0] += m[0];
    acc[1] += m[1];
    acc[2] += m[2];
    acc[3] += r[1] * m[2] - r[2] * m[1];
    acc[4] += r[2] * m[0] - r[0] * m[2];
    acc[5] += r[0] * m[1] - r[1] * m[0];
  }
  for (int k = 0; k < 6; k++) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 6; k++) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; k++) {
      a.P[3 * p + k] = red[k][0];
      a.L[3 * p + k] = red[3 + k][0];
    }
}


template <int DIM, class T>
struct RunCollide {
  template <int BX>
  static void go(iblbm_ctx* c, K1Args<typename Store<T>::C>& a) {
    a.nbx = (c->cfg.n[0] + BX - 1) / BX;
    a.nblk = a.nbx * c->cfg.n[1] * c->cfg.n[2];
    a.xcd_per = (a.nblk % 8 == 0) ? a.nblk / 8 : 0;
    auto k = c->parity == 0 ? k_collide_stream<DIM, T, 0, BX> : k_collide_stream<DIM, T, 1, BX>;
    hipEvent_t t0, t1;
    if (kernel_events(c, IBLBM_T_COLLIDE, &t0, &t1))
      hipExtLaunchKernelGGL(k, dim3(a.nblk), dim3(BX), 0, c->stream, t0, t1, 0, a);
    else
      hipLaunchKernelGGL(k, dim3(a.nblk), dim3(BX), 0, c->stream, a);
  }
  static void run(iblbm_ctx* c) {
    using C = typename Store<T>::C;
    K1Args<C> a;
    a.g = make_geo<C>(c);
    a.slot = make_slots(c);
    a.bmap = c->bmap + (size_t)c->fbuf * c->nwords;
    a.bmap_next = c->bmap + (size_t)(1 - c->fbuf) * c->nwords;
    a.nwx = (int)c->nwx;
    a.facc = (const C*)c->facc;
    a.vd = c->vd;
    a.omega = C(1.0 / c->cfg.tau);
    a.kforce = C(1.0 - 0.5 / c->cfg.tau);
    a.rho0 = C(c->cfg.rho0);
    for (int k = 0; k < 3; k++) a.body[k] = k < DIM ? C(c->cfg.body_force[k]) : C(0);
    a.inv_s = inv_scale<T>(c);
    int nx = c->cfg.n[0];
    // 16-bit storage: 64-lane blocks (measured faster on the odd step of 384^3)
    if (sizeof(T) == 2)
      go<64>(c, a);
    else if (nx % 256 == 0 || nx > 1024)
      go<256>(c, a);
    else if (nx % 128 == 0)
      go<128>(c, a);
    else
      go<64>(c, a);
  }
};

template <int DIM, class T>
struct RunGather {
  static void run(iblbm_ctx* c, double* p, double* u, double* force, double* fout) {
    using C = typename Store<T>::C;
    GatherArgs<C> a;
    a.g = make_geo<C>(c);
    a.slot = make_slots(c);
    // the bitmap of the most recent step
    a.bmap = c->bmap + (size_t)c->fbuf * c->nwords;
    a.nwx = (int)c->nwx;
    a.facc = (const C*)c->facc;
    a.vd = c->vd;
    a.inv_s = inv_scale<T>(c);
    a.p = p;
    a.u = u;
    a.force = force;
    a.fout = fout;
    unsigned blocks = unsigned((c->N + 255) / 256);
    if (c->parity == 0)
      hipLaunchKernelGGL((k_gather<DIM, T, 0>), dim3(blocks), dim3(256), 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_gather<DIM, T, 1>), dim3(blocks), dim3(256), 0, c->stream, a);
  }
};

template <int DIM, class T>
struct RunScatter {
  static void run(iblbm_ctx* c, const double* fin, const double* p, const double* u) {
    using C = typename Store<T>::C;
    ScatterArgs<C> a;
    a.g = make_geo<C>(c);
    a.slot = make_slots(c);
    a.inv_s = inv_scale<T>(c);
    a.fin = fin;
    a.p = p;
    a.u = u;
    unsigned blocks = unsigned((c->N + 255) / 256);
    hipLaunchKernelGGL((k_scatter<DIM, T>), dim3(blocks), dim3(256), 0, c->stream, a);
  }
};

template <int DIM, class T>
struct RunInterior {
  static InteriorArgs<typename Store<T>::C> args(iblbm_ctx* c, double* P, double* Lm) {
    using C = typename Store<T>::C;
    InteriorArgs<C> a;
    a.g = make_geo<C>(c);
    a.slot = make_slots(c);
    a.inv_s = inv_scale<T>(c);
    a.X = c->X;
    a.D = c->D;
    a.P = P;
    a.L = Lm;
    a.ustar = (const C*)c->ustar;
    a.vd = c->vd;
    a.status = c->dstatus;
    return a;
  }
  static void run(iblbm_ctx* c, double* P, double* Lm, bool from_u) {
    auto a = args(c, P, Lm);
    if (from_u)
      hipLaunchKernelGGL((k_interior<DIM, T, 0, 1>), dim3(c->np), dim3(256), 0, c->stream, a);
    else if (c->parity == 0)
      hipLaunchKernelGGL((k_interior<DIM, T, 0, 0>), dim3(c->np), dim3(256), 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_interior<DIM, T, 1, 0>), dim3(c->np), dim3(256), 0, c->stream, a);
  }
};

template <int DIM, class T>
struct RunFaceBc {
  static void run(iblbm_ctx* c) {
    using C = typename Store<T>::C;
    for (int face = 0; face < 6; face++) {
      const int kind = c->cfg.face_bc[face];
      if (kind == 0) continue;
      FaceArgs<C> a;
      a.g = make_geo<C>(c);
      a.slot = make_slots(c);
      a.inv_s = inv_scale<T>(c);
      a.rho0 = C(c->cfg.rho0);
      a.face = face;
      a.kind = kind;
      for (int d = 0; d < 3; d++) a.ub[d] = d < DIM ? C(c->cfg.wall_u[face][d]) : C(0);
      a.pb = C(c->cfg.face_p[face]);
      const int ax = face / 2;
      const long long nodes = c->N / c->cfg.n[ax];
      const unsigned blocks = (unsigned)((nodes + 255) / 256);
      // the populations the next step reads, in its parity's layout
      if (c->parity == 0)
        hipLaunchKernelGGL((k_face_bc<DIM, T, 0>), dim3(blocks), dim3(256), 0, c->stream, a);
      else
        hipLaunchKernelGGL((k_face_bc<DIM, T, 1>), dim3(blocks), dim3(256), 0, c->stream, a);
    }
  }
};

template <int DIM, class T>
struct RunUstarAll {
  static void run(iblbm_ctx* c) {
    auto a = RunInterior<DIM, T>::args(c, nullptr, nullptr);
    int nbx = (c->cfg.n[0] + 255) / 256;
    unsigned nblk = (unsigned)((long long)nbx * c->cfg.n[1] * c->cfg.n[2]);
    // XCD-aware order in 2-D only (measured slower at 256^3, where a row's z neighbours
    // lie a whole plane of rows away)
    int xcd_per = DIM == 2 && nblk % 8 == 0 ? (int)(nblk / 8) : 0;
    if (c->parity == 0)
      hipLaunchKernelGGL((k_ustar_all<DIM, T, 0>), dim3(nblk), dim3(256), 0, c->stream, a, nbx,
                         xcd_per);
    else
      hipLaunchKernelGGL((k_ustar_all<DIM, T, 1>), dim3(nblk), dim3(256), 0, c->stream, a, nbx,
                         xcd_per);
  }
};

}  // namespace

void lbm_interior_momentum(iblbm_ctx* c, double* P, double* L, bool from_ustar) {
  if (c->np > 0) dispatch<RunInterior>(c, P, L, from_ustar);
}
void lbm_ustar_all(iblbm_ctx* c) {
  dispatch<RunUstarAll>(c);
  c->ustar_valid = true;
}

void lbm_collide_stream(iblbm_ctx* c) { dispatch<RunCollide>(c); }
void lbm_face_bc(iblbm_ctx* c) {
  for (int f = 0; f < 6; f++)
    if (c->cfg.face_bc[f] != 0) {
      dispatch<RunFaceBc>(c);
      return;
    }
}
void lbm_get_fields(iblbm_ctx* c, double* p, double* u, double* force) {
  dispatch<RunGather>(c, p, u, force, (double*)nullptr);
}
void lbm_get_pdfs(iblbm_ctx* c, double* f) {
  dispatch<RunGather>(c, (double*)nullptr, (double*)nullptr, (double*)nullptr, f);
}
void lbm_set_pdfs(iblbm_ctx* c, const double* f) {
  dispatch<RunScatter>(c, f, (const double*)nullptr, (const double*)nullptr);
  c->parity = 0;
  c->ustar_valid = false;
  c->graph_dirty = true;
}
void lbm_init_equilibrium(iblbm_ctx* c, const double* p, const double* u) {
  dispatch<RunScatter>(c, (const double*)nullptr, p, u);
  c->parity = 0;
  c->ustar_valid = false;
  c->graph_dirty = true;
}

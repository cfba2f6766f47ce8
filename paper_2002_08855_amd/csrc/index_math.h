// Index arithmetic from particle and point positions: delta-function supports and their
// weights (Eq. 12 with the kernels of Fig. 2b), the LDS boxes of the per-particle IB
// kernels, cell coordinates (Eqs. 49-51) and the box of a particle's interior.  The
// functions are __host__ __device__ so that a host build can replay any particle state
// through exactly the arithmetic the kernels use.
//
// Positions reach integer arithmetic only through floor_idx / ceil_idx, which limit the
// result to [-IDX_LIMIT, IDX_LIMIT] and send NaN to -IDX_LIMIT.  Converting a double
// outside the int range (or NaN) to int is undefined behaviour; with the limit, every
// later sum of a few box sides and offsets stays far inside int, and a particle that has
// run away (or turned NaN) maps to nodes outside every lattice, which the bounds tests
// below then skip.  Lattices are far smaller than the limit (at most 2^31 / 8 nodes).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

constexpr int IDX_LIMIT = 1 << 24;

__host__ __device__ __forceinline__ int floor_idx(double v) {
  if (!(v > -double(IDX_LIMIT))) return -IDX_LIMIT;  // also NaN
  if (v >= double(IDX_LIMIT)) return IDX_LIMIT;
  return (int)floor(v);
}
__host__ __device__ __forceinline__ int ceil_idx(double v) {
  if (!(v > -double(IDX_LIMIT))) return -IDX_LIMIT;  // also NaN
  if (v >= double(IDX_LIMIT)) return IDX_LIMIT;
  return (int)ceil(v);
}

// Lattice and delta-function kind of the immersed boundary kernels.
struct MarkerGeo {
  int n[3], periodic[3];
  int dim, kind, width;  // kind 0: Peskin 4-point (width 4), 1: Roma 3-point (width 3)
};

// The regularised delta functions of Fig. 2(b), dh = 1.
template <class C>
__host__ __device__ __forceinline__ C phi(int kind, C r) {
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

// The support node handled by lane l of a point at X: node index or -1 (outside a
// wall axis, or a lane beyond the support width), its weight, and whether it was cut
// by a wall.
template <int DIM, class C>
__host__ __device__ __forceinline__ int support_node(const MarkerGeo& g, const double* X, int l, C& w,
                                            bool& trunc) {
  int id[3] = {l & 3, (l >> 2) & 3, (l >> 4) & 3};
  w = C(1);
  trunc = false;
  int c[3] = {0, 0, 0};
  bool inside = true;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    if (id[a] >= g.width) inside = false;
    int lo = g.kind == 0 ? floor_idx(X[a]) - 1 : floor_idx(X[a] + 0.5) - 1;
    int cc = lo + id[a];
    w *= phi<C>(g.kind, C(double(cc) - X[a]));
    if (cc < 0 || cc >= g.n[a]) {
      if (g.periodic[a])
        cc = cc < 0 ? cc + g.n[a] : cc - g.n[a];
      if (cc < 0 || cc >= g.n[a]) trunc = true;  // a wall axis, or a point far outside
    }
    c[a] = cc;
  }
  if (!inside) {
    trunc = false;
    return -1;
  }
  if (trunc) return -1;
  return c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

// A box of lattice nodes lo .. lo + B - 1 per axis (n = B0 B1 B2 nodes, INT32_MAX when
// that product does not fit an int), with box node t = lx + B0 (ly + B1 lz).
template <int DIM>
struct PBox {
  int lo[3], B[3], n;
  float rb0, rb01;  // 1 / B0 and 1 / (B0 B1)
  // Lattice coordinates of box node t.  The quotients come from float reciprocals: for
  // t < 2^16 the rounding error of (t + 1/2) / B stays below 2^-6 / B while the fraction
  // of (t + 1/2) / B is at least 1/(2B) from an integer, so truncation gives the exact
  // quotient without an integer division.
  __host__ __device__ __forceinline__ void at(int t, int& x, int& y, int& z) const {
    const int lz = (int)(((float)t + 0.5f) * rb01);
    const int r = t - lz * (B[0] * B[1]);
    const int ly = (int)(((float)r + 0.5f) * rb0);
    x = lo[0] + r - ly * B[0];
    y = lo[1] + ly;
    z = lo[2] + lz;
  }
};

// The box of nodes that the supports of points at offsets in [rlo, rhi] from Xc can
// reach.  The range is widened by 1e-9 so that a point whose offset rounds slightly
// outside still has its support inside; the box side is at most
// floor(rhi - rlo + 2e-9) + 5 nodes.
template <int DIM>
__host__ __device__ __forceinline__ PBox<DIM> range_box(const double* Xc, const double* rlo,
                                                        const double* rhi, int kind) {
  PBox<DIM> b;
  long long n = 1;
  for (int d = 0; d < 3; d++) {
    if (d < DIM) {
      const double l = Xc[d] + (rlo[d] - 1e-9), h = Xc[d] + (rhi[d] + 1e-9);
      int lo = kind == 0 ? floor_idx(l) - 1 : floor_idx(l + 0.5) - 1;
      int hi = kind == 0 ? floor_idx(h) + 2 : floor_idx(h + 0.5) + 1;
      b.lo[d] = lo;
      b.B[d] = hi - lo + 1;
    } else {
      b.lo[d] = 0;
      b.B[d] = 1;
    }
    n *= b.B[d];
  }
  b.n = n > (long long)INT32_MAX ? INT32_MAX : (int)n;
  b.rb0 = 1.0f / (float)b.B[0];
  b.rb01 = 1.0f / ((float)b.B[0] * (float)b.B[1]);
  return b;
}

// the box of a whole particle: offsets within +-R of its centre
template <int DIM>
__host__ __device__ __forceinline__ PBox<DIM> particle_box(const double* Xc, double R, int kind) {
  const double rlo[3] = {-R, -R, -R}, rhi[3] = {R, R, R};
  return range_box<DIM>(Xc, rlo, rhi, kind);
}

// 1-D weights of a point's support (the factors of Eq. 12).  With f the offset of X
// past its first support node (Peskin 4-point) or from its nearest node (Roma
// 3-point) and s the one square root both kernels need, the weight of support node q
// is (k0 + k1 f + k2 s) * scale with constants that depend on q alone; this equals the
// kernel evaluated at the node.
template <class C>
struct AxisForm {
  C k0, k1, k2;
};
template <class C>
__host__ __device__ __forceinline__ AxisForm<C> axis_form(int kind, int q) {
  // Peskin: (3 - 2f - s, 3 - 2f + s, 1 + 2f + s, 1 + 2f - s) / 8
  // Roma:   (2 - 3e - s, 2 + 2s, 2 + 3e - s, 0) / 6
  const float P0[4] = {3, 3, 1, 1}, P1[4] = {-2, -2, 2, 2}, P2[4] = {-1, 1, 1, -1};
  const float R0[4] = {2, 2, 2, 0}, R1[4] = {-3, 0, 3, 0}, R2[4] = {-1, 2, -1, 0};
  AxisForm<C> r;
  r.k0 = C(kind == 0 ? P0[q] : R0[q]);
  r.k1 = C(kind == 0 ? P1[q] : R1[q]);
  r.k2 = C(kind == 0 ? P2[q] : R2[q]);
  return r;
}
template <class C>
__host__ __device__ __forceinline__ C axis_scale(int kind) {
  return kind == 0 ? C(0.125) : C(1) / C(6);
}
// first support node of X along one axis, with f and s as above
template <class C>
__host__ __device__ __forceinline__ int axis_fs(int kind, double X, C& f, C& s) {
  if (kind == 0) {
    const double fl = floor(X);
    f = C(X - fl);
    s = sqrt(C(1) + C(4) * f - C(4) * f * f);
    return floor_idx(X) - 1;
  }
  const double cn = floor(X + 0.5);
  f = C(X - cn);
  s = sqrt(C(1) - C(3) * f * f);
  return floor_idx(X + 0.5) - 1;
}

// the support of one point: per-axis weights and first node
template <class C>
struct PointWeights {
  C w[3][4];
  int g0[3];
};
template <int DIM, class C>
__host__ __device__ __forceinline__ void point_weights(int kind, const double* X, PointWeights<C>& pw) {
  const C sc = axis_scale<C>(kind);
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    pw.g0[ax] = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) pw.w[ax][q] = C(ax < DIM ? 0 : (q == 0 ? 1 : 0));
  }
#pragma unroll
  for (int ax = 0; ax < DIM; ax++) {
    C f, s;
    pw.g0[ax] = axis_fs<C>(kind, X[ax], f, s);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const AxisForm<C> fm = axis_form<C>(kind, q);
      pw.w[ax][q] = (fm.k0 + fm.k1 * f + fm.k2 * s) * sc;
    }
  }
}

// Visit every support node inside the walls and the box: fn(box-local index, weight
// with the (phi_x phi_y) phi_z product order of Eq. 12).  Returns the number of support
// nodes outside the walls.
template <int DIM, class C, class Fn>
__host__ __device__ __forceinline__ int visit_support(const MarkerGeo& g, const PBox<DIM>& b,
                                                      const PointWeights<C>& pw, Fn fn) {
  bool ok[3][4];
  int nin[3] = {1, 1, 1}, lo[3] = {0, 0, 0};
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    if (ax < DIM) {
      nin[ax] = 0;
      lo[ax] = pw.g0[ax] - b.lo[ax];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int c = pw.g0[ax] + q;
      const bool wall_in = ax >= DIM ? q == 0 : (q < g.width && c >= 0 && c < g.n[ax]);
      if (ax < DIM) nin[ax] += wall_in ? 1 : 0;
      ok[ax][q] = wall_in && (ax >= DIM || (lo[ax] + q >= 0 && lo[ax] + q < b.B[ax]));
    }
  }
  const int base = lo[0] + b.B[0] * (lo[1] + b.B[1] * lo[2]);
#pragma unroll
  for (int iz = 0; iz < (DIM == 3 ? 4 : 1); iz++) {
    if (!ok[2][iz]) continue;
#pragma unroll
    for (int iy = 0; iy < 4; iy++) {
      if (!ok[1][iy]) continue;
      const int row = base + b.B[0] * (iy + b.B[1] * iz);
#pragma unroll
      for (int ix = 0; ix < 4; ix++) {
        if (!ok[0][ix]) continue;
        const C ww = DIM == 3 ? (pw.w[0][ix] * pw.w[1][iy]) * pw.w[2][iz] : pw.w[0][ix] * pw.w[1][iy];
        fn(row + ix, ww);
      }
    }
  }
  const int full = DIM == 3 ? g.width * g.width * g.width : g.width * g.width;
  return full - nin[0] * nin[1] * nin[2];
}

// Cell coordinate of a position along one axis (Eqs. 49-51): floor((x + 1/2) n_c / n),
// limited to the grid.
__host__ __device__ __forceinline__ int cell_coord(double x, double invh, int nc) {
  const int c = floor_idx((x + 0.5) * invh);
  return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Nodes that can lie inside a particle of radius R at Xc (the indicator of the interior
// momentum reaches R + 1/2), limited to the lattice: lo .. hi per axis (empty when
// hi < lo).
__host__ __device__ __forceinline__ void interior_box(const double* Xc, double R, const int* n,
                                                      int dim, int* lo, int* hi) {
  for (int d = 0; d < 3; d++) {
    lo[d] = 0;
    hi[d] = 0;
  }
  for (int d = 0; d < dim; d++) {
    const int l = floor_idx(Xc[d] - R - 0.5), h = ceil_idx(Xc[d] + R + 0.5);
    lo[d] = l > 0 ? l : 0;
    hi[d] = h < n[d] - 1 ? h : n[d] - 1;
  }
}

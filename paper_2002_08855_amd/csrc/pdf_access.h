// Device access to the PDF array in its A-A layout, shared by the fluid and the
// immersed-boundary kernels, plus the host helpers that fill the geometry arguments.
//
// Layout: SoA, slot a-1 holds direction a = 1..q-1 for all N nodes.  After an even
// step the post-collision value of direction a at node x sits in the opposite slot at
// x; an odd step reads it from the neighbour x - e_a.  Links that leave through a
// wall bounce back half-way with the moving-wall term 2 w_a rho0 (e_a . u_w)/c_s^2.
#pragma once
#include "common.h"

namespace pdf {

// Streaming access to the PDF slots: every value is read once and written once per
// step.  NT selects non-temporal access (no cache retention).  It is used for the even
// step of 3-D lattices, whose accesses are row-aligned and whose slots far exceed the
// last-level cache; the odd step's accesses shifted by one node in x share cache lines
// with the neighbouring wavefront and stay cached (measured faster), and 2-D lattices of
// the sizes used here fit the last-level cache.
template <bool NT, class T>
__device__ __forceinline__ T ld_pdf(const T* p) {
  if constexpr (NT) {
    if constexpr (sizeof(T) == 2) {
      uint16_t u = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
      T r;
      __builtin_memcpy(&r, &u, 2);
      return r;
    } else {
      return __builtin_nontemporal_load(p);
    }
  } else {
    return *p;
  }
}
template <bool NT, class T>
__device__ __forceinline__ void st_pdf(T* p, T v) {
  if constexpr (NT) {
    if constexpr (sizeof(T) == 2) {
      uint16_t u;
      __builtin_memcpy(&u, &v, 2);
      __builtin_nontemporal_store(u, reinterpret_cast<uint16_t*>(p));
    } else {
      __builtin_nontemporal_store(v, p);
    }
  } else {
    *p = v;
  }
}

// Neighbour along +d (d = +-e_a) of node (x,y,z) and whether the link leaves through a
// wall (then 'face' is the first wall face crossed, in axis order).
template <int DX, int DY, int DZ, class C>
__device__ __forceinline__ int neighbour(const Geo<C>& g, int x, int y, int z, bool& wall,
                                         int& face) {
  int c[3] = {x + DX, y + DY, z + DZ};
  const int d[3] = {DX, DY, DZ};
  wall = false;
  face = 0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (d[a] == 0) continue;
    bool lo = c[a] < 0, hi = c[a] >= g.n[a];
    if (lo || hi) {
      if (g.periodic[a]) {
        c[a] = lo ? c[a] + g.n[a] : c[a] - g.n[a];
      } else if (!wall) {
        wall = true;
        face = 2 * a + (hi ? 1 : 0);
      }
    }
  }
  return c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

template <int DIM, class T, int PAR, int A>
struct LoadDir {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  __device__ __forceinline__ static C run(T* const* slot, const Geo<C>& g, int x, int y, int z,
                                          int i, C inv_s) {
    if (PAR == 0) return Store<T>::load(ld_pdf<DIM == 3>(&slot[A - 1][i]), inv_s);
    bool wall;
    int face;
    int j = neighbour<-L::ex[A], -L::ey[A], -L::ez[A], C>(g, x, y, z, wall, face);
    constexpr int O = opp_dir(A, L::H);
    if (!wall) return Store<T>::load(ld_pdf<false>(&slot[O - 1][j]), inv_s);
    return Store<T>::load(ld_pdf<false>(&slot[A - 1][i]), inv_s) + g.wt[A][face];
  }
};

template <int DIM, class T, int PAR, int A>
struct StoreDir {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  __device__ __forceinline__ static void run(T* const* slot, const Geo<C>& g, int x, int y, int z,
                                             int i, C v, C inv_s) {
    constexpr int O = opp_dir(A, L::H);
    if (PAR == 0) {
      st_pdf<DIM == 3>(&slot[O - 1][i], Store<T>::save(v, inv_s));
      return;
    }
    bool wall;
    int face;
    int j = neighbour<L::ex[A], L::ey[A], L::ez[A], C>(g, x, y, z, wall, face);
    if (!wall)
      st_pdf<false>(&slot[A - 1][j], Store<T>::save(v, inv_s));
    else
      st_pdf<false>(&slot[O - 1][i], Store<T>::save(v - g.wt[A][face], inv_s));
  }
};

// Set the value that LoadDir<DIM, T, PAR, A> reads at node (x, y, z): its own slot (even
// layout), the opposite slot of the upstream neighbour, or, for a link from outside a
// wall, its own slot less the wall term that the load adds back.
template <int DIM, class T, int PAR, int A>
struct SetIncomingDir {
  using C = typename Store<T>::C;
  using L = Lat<DIM>;
  __device__ __forceinline__ static void run(T* const* slot, const Geo<C>& g, int x, int y, int z,
                                             int i, C v, C inv_s) {
    if (PAR == 0) {
      st_pdf<false>(&slot[A - 1][i], Store<T>::save(v, inv_s));
      return;
    }
    bool wall;
    int face;
    int j = neighbour<-L::ex[A], -L::ey[A], -L::ez[A], C>(g, x, y, z, wall, face);
    constexpr int O = opp_dir(A, L::H);
    if (!wall)
      st_pdf<false>(&slot[O - 1][j], Store<T>::save(v, inv_s));
    else
      st_pdf<false>(&slot[A - 1][i], Store<T>::save(v - g.wt[A][face], inv_s));
  }
};

// The populations a step of parity PAR reads at node (x, y, z) become f[1..q-1].
template <int DIM, class T, int PAR, int A = 1>
__device__ __forceinline__ void set_incoming_all(T* const* slot, const Geo<typename Store<T>::C>& g,
                                                 int x, int y, int z, int i,
                                                 typename Store<T>::C inv_s,
                                                 const typename Store<T>::C* f) {
  if constexpr (A < Lat<DIM>::Q) {
    SetIncomingDir<DIM, T, PAR, A>::run(slot, g, x, y, z, i, f[A], inv_s);
    set_incoming_all<DIM, T, PAR, A + 1>(slot, g, x, y, z, i, inv_s, f);
  }
}

template <int DIM, class T, int PAR, int A = 1>
__device__ __forceinline__ void load_all(T* const* slot, const Geo<typename Store<T>::C>& g, int x,
                                         int y, int z, int i, typename Store<T>::C inv_s,
                                         typename Store<T>::C* f) {
  if constexpr (A < Lat<DIM>::Q) {
    f[A] = LoadDir<DIM, T, PAR, A>::run(slot, g, x, y, z, i, inv_s);
    load_all<DIM, T, PAR, A + 1>(slot, g, x, y, z, i, inv_s, f);
  }
}

template <int DIM, class T, int PAR, int A = 1>
__device__ __forceinline__ void store_all(T* const* slot, const Geo<typename Store<T>::C>& g, int x,
                                          int y, int z, int i, typename Store<T>::C inv_s,
                                          const typename Store<T>::C* f) {
  if constexpr (A < Lat<DIM>::Q) {
    StoreDir<DIM, T, PAR, A>::run(slot, g, x, y, z, i, f[A], inv_s);
    store_all<DIM, T, PAR, A + 1>(slot, g, x, y, z, i, inv_s, f);
  }
}

// Odd step at a node whose neighbours all lie inside the domain: the neighbour of
// direction a is a fixed index offset, so no wall tests are needed.
template <int DIM, class T, int A = 1>
__device__ __forceinline__ void load_odd_interior(T* const* slot, int i, int sy, int sz,
                                                  typename Store<T>::C inv_s,
                                                  typename Store<T>::C* f) {
  using L = Lat<DIM>;
  if constexpr (A < L::Q) {
    constexpr int O = opp_dir(A, L::H);
    // 3-D directions without an x component read a whole row that no other wavefront
    // touches: non-temporal; those with one share lines across wavefronts: cached
    constexpr bool NT = DIM == 3 && L::ex[A] == 0;
    f[A] = Store<T>::load(
        ld_pdf<NT>(&slot[O - 1][i - (L::ex[A] + sy * L::ey[A] + sz * L::ez[A])]), inv_s);
    load_odd_interior<DIM, T, A + 1>(slot, i, sy, sz, inv_s, f);
  }
}

template <int DIM, class T, int A = 1>
__device__ __forceinline__ void store_odd_interior(T* const* slot, int i, int sy, int sz,
                                                   typename Store<T>::C inv_s,
                                                   const typename Store<T>::C* f) {
  using L = Lat<DIM>;
  if constexpr (A < L::Q) {
    constexpr bool NT = DIM == 3 && L::ex[A] == 0;
    st_pdf<NT>(&slot[A - 1][i + (L::ex[A] + sy * L::ey[A] + sz * L::ez[A])],
               Store<T>::save(f[A], inv_s));
    store_odd_interior<DIM, T, A + 1>(slot, i, sy, sz, inv_s, f);
  }
}

// u* = sum_a e_a f_a / rho0 (Eq. 5) and S = sum_{a>=1} f_a
template <int DIM, class C>
__device__ __forceinline__ void moments(const C* f, C rho0, C& S, C* us) {
  using L = Lat<DIM>;
  C s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 1; a < L::Q; a++) {
    s += f[a];
    if (L::ex[a] != 0) jx += L::ex[a] * f[a];
    if (L::ey[a] != 0) jy += L::ey[a] * f[a];
    if (DIM == 3 && L::ez[a] != 0) jz += L::ez[a] * f[a];
  }
  C ir = C(1) / rho0;
  S = s;
  us[0] = jx * ir;
  us[1] = jy * ir;
  us[2] = DIM == 3 ? jz * ir : C(0);
}

struct SlotPtrs {
  void* p[18];
};

template <int DIM, class T>
__device__ __forceinline__ void slots_of(const SlotPtrs& sp, T** s) {
#pragma unroll
  for (int a = 0; a < Lat<DIM>::Q - 1; a++) s[a] = reinterpret_cast<T*>(sp.p[a]);
}

template <class C>
Geo<C> make_geo(const iblbm_ctx* c) {
  Geo<C> g;
  for (int a = 0; a < 3; a++) {
    g.n[a] = c->cfg.n[a];
    g.periodic[a] = c->cfg.periodic[a];
  }
  g.N = c->N;
  g.rho0 = C(c->cfg.rho0);
  const int* ex = c->dim == 2 ? Lat<2>::ex : Lat<3>::ex;
  const int* ey = c->dim == 2 ? Lat<2>::ey : Lat<3>::ey;
  const int* ez = c->dim == 2 ? Lat<2>::ez : Lat<3>::ez;
  const double* w = c->dim == 2 ? Lat<2>::w : Lat<3>::w;
  for (int d = 0; d < 19; d++)
    for (int fc = 0; fc < 6; fc++) {
      double v = 0;
      if (d < c->q) {
        double eu = ex[d] * c->cfg.wall_u[fc][0] + ey[d] * c->cfg.wall_u[fc][1] +
                    ez[d] * c->cfg.wall_u[fc][2];
        v = 2.0 * w[d] * c->cfg.rho0 * eu * 3.0;
      }
      g.wt[d][fc] = C(v);
    }
  return g;
}

inline SlotPtrs make_slots(const iblbm_ctx* c) {
  SlotPtrs s;
  for (int a = 0; a < 18; a++)
    s.p[a] = a < c->q - 1 ? (char*)c->f + (size_t)a * c->N * c->sbytes : nullptr;
  return s;
}

template <class T>
typename Store<T>::C inv_scale(const iblbm_ctx* c) {
  return c->storage == IBLBM_F16 ? typename Store<T>::C(1.0 / c->cfg.f16_scale)
                                 : typename Store<T>::C(1);
}

// dispatch over (dim, storage) to a functor templated on <DIM, T>
template <template <int, class> class F, class... Args>
void dispatch(iblbm_ctx* c, Args... args) {
  if (c->dim == 2) {
    switch (c->storage) {
      case IBLBM_F64: F<2, double>::run(c, args...); break;
      case IBLBM_F32: F<2, float>::run(c, args...); break;
      case IBLBM_BF16: F<2, bf16s>::run(c, args...); break;
      default: F<2, __half>::run(c, args...); break;
    }
  } else {
    switch (c->storage) {
      case IBLBM_F64: F<3, double>::run(c, args...); break;
      case IBLBM_F32: F<3, float>::run(c, args...); break;
      case IBLBM_BF16: F<3, bf16s>::run(c, args...); break;
      default: F<3, __half>::run(c, args...); break;
    }
  }
}

}  // namespace pdf

template <class C, int DIM>
struct NodeVec;
template <>
struct NodeVec<float, 2> {
  using T = float2;
};
// 3-D nodes of u* and the force are packed 12-byte (24-byte in FP64) triples: a 64-byte
// line holds 16 useful words rather than the 12 of a padded float4 layout, which cuts the
// line requests of the spreading flush's atomics and of the staging loads
struct Node3f {
  float v[3];
};
struct Node3d {
  double v[3];
};
template <>
struct NodeVec<float, 3> {
  using T = Node3f;
};
template <>
struct NodeVec<double, 2> {
  using T = double2;
};
template <>
struct NodeVec<double, 3> {
  using T = Node3d;
};
template <int DIM, class C>
__device__ __forceinline__ typename NodeVec<C, DIM>::T load_node(const C* v, size_t i) {
  return *reinterpret_cast<const typename NodeVec<C, DIM>::T*>(v + i);
}
template <class C, class V>
__device__ __forceinline__ C comp(const V& v, int c) {
  return reinterpret_cast<const C*>(&v)[c];
}

// whole-node store of the DIM values of x, so that a node is written by one store rather
// than one component at a time
template <int DIM, class C>
__device__ __forceinline__ void store_node(C* v, size_t i, const C* x) {
  typename NodeVec<C, DIM>::T w;
  C* e = reinterpret_cast<C*>(&w);
#pragma unroll
  for (int c = 0; c < DIM; c++) e[c] = x[c];
  *reinterpret_cast<typename NodeVec<C, DIM>::T*>(v + i) = w;
}


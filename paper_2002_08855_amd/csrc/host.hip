// Host side of the gfx950 IB-LBM library: the C ABI of include/iblbm.h, device memory,
// the per-step kernel sequence, status read-back and event timing.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "common.h"

void part_zero_cells(iblbm_ctx* c);
void mlp_step_forcing(iblbm_ctx* c);  // learned forcing stage (mlp.hip)

namespace {

const double PI = 3.14159265358979323846;

struct Fail {
  iblbm_status st;
};

iblbm_status fail(iblbm_ctx* c, iblbm_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st == IBLBM_E_DEVICE || st == IBLBM_E_UNSTABLE) c->sticky = st;
  }
  return st;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw Fail{fail(c, IBLBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))}; \
  } while (0)

void* dalloc(iblbm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (c->cfg.dev_alloc) {
    p = c->cfg.dev_alloc(bytes, c->cfg.alloc_user);
    if (!p) throw Fail{fail(c, IBLBM_E_NOMEM, "device allocation failed")};
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Fail{fail(c, IBLBM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e))};
  }
  c->allocs.push_back(p);
  return p;
}

void dfree(iblbm_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  if (c->cfg.dev_free)
    c->cfg.dev_free(p, c->cfg.alloc_user);
  else
    (void)hipFree(p);
}

template <class T>
T* dzeros(iblbm_ctx* c, size_t n) {
  T* p = (T*)dalloc(c, n * sizeof(T));
  HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), c->stream));
  return p;
}

// grow a device array from old_n to new_n elements, keeping the old contents
template <class T>
void grow(iblbm_ctx* c, T*& p, size_t old_n, size_t new_n) {
  T* q = dzeros<T>(c, new_n);
  if (p && old_n) HIPCHK(hipMemcpyAsync(q, p, old_n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
  if (p) {
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, p);
  }
  p = q;
}

void growv(iblbm_ctx* c, void*& p, size_t old_b, size_t new_b) {
  char* q = (char*)p;
  grow<char>(c, q, old_b, new_b);
  p = q;
}

__global__ void k_fill_d(double* p, int n, double v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

iblbm_status check_ready(iblbm_ctx* c) {
  if (!c) return IBLBM_E_ARG;
  if (c->sticky) {
    c->err = "context is in an error state: " + c->err;
    return IBLBM_E_STATE;
  }
  return IBLBM_OK;
}

double compute_H(const iblbm_ctx* c) {
  double dmax = 0, dmin = 1e300;
  for (double d : c->hD) {
    dmax = std::max(dmax, d);
    dmin = std::min(dmin, d);
  }
  double H = c->cfg.cell_h;
  if (!(H > 0.0)) {
    // Eq. 50 (2H > D + zeta) and Eq. 49 (cell diagonal < D)
    double lo = 0.5 * (dmax + c->cfg.zeta);
    double hi = dmin / sqrt((double)c->dim);
    H = lo < hi ? 0.5 * (lo + hi) : 1.05 * lo;
  }
  return H;
}

// Work units of the per-particle LDS kernels.  A particle whose support box fits in
// half of a compute unit's LDS (at most floor(D) + 5 nodes a side, the box of +-R) and
// whose points fit one workgroup is one unit.  Any other particle is split into runs of
// consecutive points -- bands of the spiral on a sphere, arcs on a circle -- each with
// the box of its own points' offset range: two runs if the whole box fits one workgroup
// but leaves no room for a second (a 16-wide FP32 sphere: about 5% faster steps, while
// three or more runs cost more in atomics at the seams than they gain), else runs
// halved until every box fits.  A particle for which even runs of 32 points do not fit
// has no plan (the point-wise kernels are used).
struct UnitPlan {
  int m0, mc;          // run of points, from the particle's first point
  double lo[3], hi[3]; // offset range of the run's points (the whole +-R for one unit)
  long long nodes;     // nodes of the box planned for the unit (an upper bound)
};

// box nodes per axis for an offset range of width w (see the device box)
long long unit_side(double w) { return (long long)floor(w + 1e-6) + 5; }

// largest box (nodes) one workgroup can hold: interpolation (u, flag, list) and spreading
// (sums, list) per node, 1 KB for the rest
long long unit_nmax(int dim, size_t cs, int lds_max) {
  const long long per_node = (long long)std::max<size_t>(dim * cs + 3, dim * cs + 2);
  return std::min<long long>((lds_max - 1024) / per_node, 65536);
}

// plan of one particle of diameter D with mc points at offsets offs (4 doubles a point)
bool plan_particle(int dim, long long nmax, double D, const double* offs, int mc,
                   std::vector<UnitPlan>& out) {
  const double R = 0.5 * D;
  long long full = 1;
  for (int a = 0; a < dim; a++) full *= unit_side(D);
  if (2 * full <= nmax && mc <= LDS_THREADS) {
    UnitPlan u{0, mc, {0, 0, 0}, {0, 0, 0}, full};
    for (int a = 0; a < dim; a++) {
      u.lo[a] = -R;
      u.hi[a] = R;
    }
    out.push_back(u);
    return true;
  }
  const int P0 = full <= nmax && mc >= 64 ? (mc + 1) / 2 : mc;
  for (int P = std::min(P0, LDS_THREADS); P >= 32; P /= 2) {
    std::vector<UnitPlan> v;
    bool ok = true;
    for (int s = 0; s < mc && ok; s += P) {
      const int e = std::min(mc, s + P);
      UnitPlan u{s, e - s, {0, 0, 0}, {0, 0, 0}, 1};
      for (int a = 0; a < dim; a++) {
        u.lo[a] = 1e300;
        u.hi[a] = -1e300;
        for (int k = s; k < e; k++) {
          const double r = offs[4 * (size_t)k + a];
          u.lo[a] = std::min(u.lo[a], r);
          u.hi[a] = std::max(u.hi[a], r);
        }
        u.nodes *= unit_side(u.hi[a] - u.lo[a]);
      }
      if (u.nodes > nmax) ok = false;
      v.push_back(u);
    }
    if (!ok) continue;
    out.insert(out.end(), v.begin(), v.end());
    return true;
  }
  return false;
}

// The units of every particle, the largest box (box_cap) and patch_ok (false when a
// particle has no plan) are set on the context and copied to the device.
void build_patches(iblbm_ctx* c) {
  const int dim = c->dim;
  const long long nmax = unit_nmax(dim, c->fp64 ? 8 : 4, c->lds_max);
  std::vector<int> own, m0v, mcv;
  std::vector<double> rlo, rhi;
  long long cap = 1;
  double box_total = 0.0;
  bool ok_all = true;
  c->full_side = 0;
  for (int p = 0; p < c->np; p++) {
    const int m0 = c->hstart[p], mc = c->hcount[p];
    c->full_side = std::max<int>(c->full_side, (int)unit_side(c->hD[p]));
    std::vector<UnitPlan> units;
    if (!plan_particle(dim, nmax, c->hD[p], &c->hmr[4 * (size_t)m0], mc, units)) {
      ok_all = false;
      continue;
    }
    for (const UnitPlan& u : units) {
      own.push_back(p);
      m0v.push_back(m0 + u.m0);
      mcv.push_back(u.mc);
      for (int a = 0; a < 3; a++) {
        rlo.push_back(u.lo[a]);
        rhi.push_back(u.hi[a]);
      }
      cap = std::max(cap, u.nodes);
      box_total += (double)u.nodes;
    }
  }
  c->box_cover = box_total / (double)c->N;
  int* ip[] = {c->pt_owner, c->pt_m0, c->pt_mc};
  for (int* q : ip)
    if (q) dfree(c, q);
  if (c->pt_rlo) dfree(c, c->pt_rlo);
  if (c->pt_rhi) dfree(c, c->pt_rhi);
  c->pt_owner = c->pt_m0 = c->pt_mc = nullptr;
  c->pt_rlo = c->pt_rhi = nullptr;
  c->patch_ok = ok_all;
  c->npatch = ok_all ? (int)own.size() : c->np;
  c->patched = ok_all && c->npatch > c->np;
  c->box_cap = (int)std::min<long long>(cap, 1LL << 30);
  c->hpt_mc = ok_all ? mcv : c->hcount;
  if (!ok_all || c->npatch == 0) return;
  c->pt_owner = dzeros<int>(c, own.size());
  c->pt_m0 = dzeros<int>(c, own.size());
  c->pt_mc = dzeros<int>(c, own.size());
  c->pt_rlo = dzeros<double>(c, rlo.size());
  c->pt_rhi = dzeros<double>(c, rhi.size());
  HIPCHK(hipMemcpyAsync(c->pt_owner, own.data(), own.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pt_m0, m0v.data(), m0v.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pt_mc, mcv.data(), mcv.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pt_rlo, rlo.data(), rlo.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pt_rhi, rhi.data(), rhi.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// Lagrangian points: equal angles on a circle (2-D); golden-angle spiral on a sphere
// (3-D), z_k = 1 - (2k+1)/N_L, azimuth k pi (3 - sqrt 5).
void marker_offsets(int dim, double R, int nl, std::vector<double>& r) {
  for (int k = 0; k < nl; k++) {
    double v[3];
    if (dim == 2) {
      double th = 2.0 * PI * k / nl;
      v[0] = R * cos(th);
      v[1] = R * sin(th);
      v[2] = 0.0;
    } else {
      double z = 1.0 - (2.0 * k + 1.0) / nl;
      double ph = k * (PI * (3.0 - sqrt(5.0)));
      double s = sqrt(1.0 - z * z);
      v[0] = R * (s * cos(ph));
      v[1] = R * (s * sin(ph));
      v[2] = R * z;
    }
    r.push_back(v[0]);
    r.push_back(v[1]);
    r.push_back(v[2]);
    r.push_back(0.0);
  }
}

void read_status(iblbm_ctx* c, int* flags) {
  int st[8];
  HIPCHK(hipMemcpyAsync(st, c->dstatus, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *flags = st[0];
  unsigned long long t;
  memcpy(&t, st + 2, sizeof(t));
  c->truncated = (long long)t;
  c->fallbacks = st[4];
}

void flush_timing(iblbm_ctx* c) {
  if (!c->timing || c->ev_used == 0) return;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
    c->time_ms[c->ev_group[k]] += ms;
    c->launches[c->ev_group[k]] += 1;
  }
  c->ev_used = 0;
}

void enqueue_step(iblbm_ctx* c) {
  bool parts = c->np > 0;
  c->fbuf = (int)(c->step & 1);
  if (parts) {
    tbegin(c, IBLBM_T_PARTICLE);
    part_cells_pairs(c);
    tend(c);
    tbegin(c, IBLBM_T_BAND);
    ibm_band(c);
    tend(c);
    if (c->cfg.forcing == IBLBM_FORCING_LEARNED && c->has_mlp) {
      mlp_step_forcing(c);
    } else {
      for (int m = 0; m < c->cfg.mdf_iters; m++) {
        tbegin(c, IBLBM_T_INTERP);
        ibm_interp(c, m == 0, 0);
        tend(c);
        tbegin(c, IBLBM_T_SPREAD);
        ibm_spread(c, 0);
        tend(c);
      }
      if (c->cfg.mdf_iters == 0)
        hipLaunchKernelGGL(k_fill_d, dim3((c->nmk * 4 + 255) / 256), dim3(256), 0, c->stream,
                           (double*)c->mF, c->fp64 ? c->nmk * 4 : c->nmk * 2, 0.0);
    }
    if (c->cfg.stats_every > 0 && c->step % c->cfg.stats_every == 0) {
      tbegin(c, IBLBM_T_OTHER);
      hipLaunchKernelGGL(k_fill_d, dim3(1), dim3(64), 0, c->stream, c->dstats, 1, 0.0);
      ibm_interp(c, 0, 1);
      tend(c);
    }
  }
  tbegin(c, IBLBM_T_COLLIDE);
  lbm_collide_stream(c);
  c->parity ^= 1;
  lbm_face_bc(c);
  tend(c);
  c->ustar_valid = false;
  if (parts) {
    // u* of the new PDFs at every node for the interior momentum and the next step's
    // forcing passes (per-particle path with the lattice-ordered u* pass)
    const bool lat = ibm_ustar_lattice(c);
    if (lat) {
      tbegin(c, IBLBM_T_BAND);
      lbm_ustar_all(c);
      tend(c);
    }
    tbegin(c, IBLBM_T_INTERIOR);
    lbm_interior_momentum(c, c->Pin, c->Lin, lat);
    tend(c);
    tbegin(c, IBLBM_T_PARTICLE);
    part_loads_newton(c);
    tend(c);
  }
  c->step++;
}

void drop_graphs(iblbm_ctx* c) {
  for (int k = 0; k < 4; k++)
    if (c->gexec[k]) {
      (void)hipGraphExecDestroy(c->gexec[k]);
      c->gexec[k] = nullptr;
    }
}

// One step through a HIP graph.  The first time a (PDF parity, bitmap buffer) pair
// occurs, the step's launches are captured from enqueue_step (which also advances the
// host-side state) and instantiated; later steps with the same pair replay the graph
// and restore the host-side state the captured step left behind.  The step contains
// kernel launches only (no memory set or copy nodes).
void step_graph(iblbm_ctx* c) {
  if (c->graph_dirty) {
    HIPCHK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->graph_dirty = false;
  }
  const int key = (c->parity & 1) * 2 + (int)(c->step & 1);
  if (!c->gexec[key]) {
    ibm_prepare_launches(c);  // kernel attributes are set before capture
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
      c->capturing = true;
      enqueue_step(c);
      c->capturing = false;
    } catch (...) {
      c->capturing = false;
      (void)hipStreamEndCapture(c->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(c->stream, &g));
    hipError_t e = hipGraphInstantiate(&c->gexec[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec[key] = nullptr;
      throw Fail{fail(c, IBLBM_E_DEVICE, "graph instantiation failed")};
    }
    c->gend_band_pending[key] = c->band_pending;
    c->gend_ustar_valid[key] = c->ustar_valid;
    HIPCHK(hipGraphLaunch(c->gexec[key], c->stream));
    return;
  }
  HIPCHK(hipGraphLaunch(c->gexec[key], c->stream));
  c->fbuf = (int)(c->step & 1);
  c->parity ^= 1;
  c->step++;
  c->band_pending = c->gend_band_pending[key];
  c->ustar_valid = c->gend_ustar_valid[key];
}

}  // namespace

void hip_check(iblbm_ctx* c, hipError_t e, const char* expr) {
  if (e != hipSuccess)
    throw Fail{fail(c, IBLBM_E_DEVICE, std::string(expr) + ": " + hipGetErrorString(e))};
}

void* ctx_alloc(iblbm_ctx* c, size_t bytes) {
  try {
    return dalloc(c, bytes);
  } catch (const Fail&) {
    return nullptr;
  }
}

namespace {

bool timed_now(const iblbm_ctx* c, int group) {
  return c->timing && ((c->timing_mask >> group) & 1) && c->step % c->timing_every == 0;
}

bool kernel_timed_group(int group) {
  return group == IBLBM_T_COLLIDE || group == IBLBM_T_INTERP || group == IBLBM_T_SPREAD;
}

void reserve_events(iblbm_ctx* c) {
  if (c->ev_used + 2 > c->ev.size()) {
    for (int k = 0; k < 64; k++) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      c->ev.push_back(e);
      c->ev_group.push_back(0);
    }
  }
}

}  // namespace

void tbegin(iblbm_ctx* c, int group) {
  c->t_open = false;
  if (!timed_now(c, group)) return;
  if (c->timing_kernel && kernel_timed_group(group)) return;  // the launch records them
  c->t_open = true;
  reserve_events(c);
  c->ev_group[c->ev_used] = group;
  HIPCHK(hipEventRecord(c->ev[c->ev_used], c->stream));
  c->ev_used++;
}

bool kernel_events(iblbm_ctx* c, int group, hipEvent_t* start, hipEvent_t* stop) {
  if (!c->timing_kernel || !kernel_timed_group(group) || !timed_now(c, group)) return false;
  reserve_events(c);
  c->ev_group[c->ev_used] = group;
  c->ev_group[c->ev_used + 1] = -1;
  *start = c->ev[c->ev_used];
  *stop = c->ev[c->ev_used + 1];
  c->ev_used += 2;
  return true;
}

void tend(iblbm_ctx* c) {
  if (!c->timing || !c->t_open) return;
  c->t_open = false;
  c->ev_group[c->ev_used] = -1;
  HIPCHK(hipEventRecord(c->ev[c->ev_used], c->stream));
  c->ev_used++;
}

extern "C" {

iblbm_status iblbm_create(const iblbm_config* cfg, iblbm_ctx** out) {
  if (!cfg || !out) return IBLBM_E_ARG;
  *out = nullptr;
  if (cfg->struct_size != sizeof(iblbm_config)) return IBLBM_E_ARG;
  if (cfg->dim != 2 && cfg->dim != 3) return IBLBM_E_ARG;
  if (!(cfg->tau > 0.5) || !(cfg->rho0 > 0)) return IBLBM_E_ARG;
  if (cfg->storage < 0 || cfg->storage > 3 || cfg->delta < 0 || cfg->delta > 1) return IBLBM_E_ARG;
  if (cfg->mdf_iters < 0 || cfg->forcing < 0 || cfg->forcing > 1) return IBLBM_E_ARG;
  if (cfg->storage == IBLBM_F16 && !(cfg->f16_scale > 0)) return IBLBM_E_ARG;
  long long N = 1;
  for (int a = 0; a < 3; a++) {
    int n = a < cfg->dim ? cfg->n[a] : 1;
    if (n < 1 || (a < cfg->dim && n < 2)) return IBLBM_E_ARG;
    N *= n;
  }
  int q = cfg->dim == 2 ? 9 : 19;
  if ((long long)(q - 1) * N >= (1LL << 31)) return IBLBM_E_ARG;
  // extrapolated faces: all on one non-periodic axis of at least 3 nodes, so that no
  // face node is the inward neighbour of another
  {
    int axis = -1;
    for (int f = 0; f < 6; f++) {
      const int k = cfg->face_bc[f];
      if (k < IBLBM_BC_WALL || k > IBLBM_BC_PRESSURE) return IBLBM_E_ARG;
      if (k == IBLBM_BC_WALL) continue;
      const int a = f / 2;
      if (a >= cfg->dim || cfg->periodic[a] || cfg->n[a] < 3) return IBLBM_E_ARG;
      if (axis >= 0 && axis != a) return IBLBM_E_ARG;
      axis = a;
    }
  }
  iblbm_ctx* c = new iblbm_ctx();
  c->cfg = *cfg;
  c->dim = cfg->dim;
  if (c->dim == 2) c->cfg.n[2] = 1;
  c->q = q;
  c->N = N;
  c->storage = cfg->storage;
  c->fp64 = cfg->storage == IBLBM_F64;
  c->sbytes = cfg->storage == IBLBM_F64 ? 8 : (cfg->storage == IBLBM_F32 ? 4 : 2);
  c->vd = c->dim == 2 ? 2 : 3;
  try {
    HIPCHK(hipGetDevice(&c->device));
    HIPCHK(hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    if (cfg->stream) {
      c->stream = (hipStream_t)cfg->stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    size_t cs = c->fp64 ? 8 : 4;
    c->f = dalloc(c, (size_t)(q - 1) * N * c->sbytes);
    HIPCHK(hipMemsetAsync(c->f, 0, (size_t)(q - 1) * N * c->sbytes, c->stream));
    c->ustar = dzeros<char>(c, (size_t)N * c->vd * cs);
    c->facc = dzeros<char>(c, (size_t)N * c->vd * cs);
    c->nsegx = (c->cfg.n[0] + SEG - 1) / SEG;
    c->nseg = c->nsegx * c->cfg.n[1] * c->cfg.n[2];
    c->bflag = dzeros<uint32_t>(c, (size_t)c->nseg);
    c->nwx = (c->cfg.n[0] + 31) / 32;
    c->nwords = c->nwx * c->cfg.n[1] * c->cfg.n[2];
    c->bmap = dzeros<uint32_t>(c, 2 * (size_t)c->nwords);
    c->seglist = dzeros<int>(c, (size_t)c->nseg);
    c->segcount = dzeros<int>(c, 1);
    c->dstatus = dzeros<int>(c, 8);
    c->dstats = dzeros<double>(c, 4);
    c->dcond = dzeros<int>(c, 1);
    HIPCHK(hipStreamSynchronize(c->stream));
  } catch (Fail& f) {
    iblbm_destroy(c);
    return f.st;
  }
  *out = c;
  return IBLBM_OK;
}

void iblbm_destroy(iblbm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->ev_flag) (void)hipEventDestroy(c->ev_flag);
  if (c->hflag) (void)hipHostFree(c->hflag);
  drop_graphs(c);
  std::vector<void*> all = c->allocs;
  for (void* p : all) dfree(c, p);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* iblbm_last_error(const iblbm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

iblbm_status iblbm_set_equilibrium(iblbm_ctx* c, const double* p, const double* u) {
  iblbm_status s = check_ready(c);
  if (s) return s;
  try {
    HIPCHK(hipSetDevice(c->device));
    double *dp = nullptr, *du = nullptr;
    if (p) {
      dp = (double*)dalloc(c, c->N * sizeof(double));
      HIPCHK(hipMemcpyAsync(dp, p, c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    if (u) {
      du = (double*)dalloc(c, c->N * c->dim * sizeof(double));
      HIPCHK(hipMemcpyAsync(du, u, c->N * c->dim * sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    lbm_init_equilibrium(c, dp, du);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, dp);
    dfree(c, du);
  } catch (Fail& f) {
    return f.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_set_pdfs(iblbm_ctx* c, const double* f) {
  iblbm_status s = check_ready(c);
  if (s) return s;
  if (!f) return fail(c, IBLBM_E_ARG, "null PDF array");
  try {
    HIPCHK(hipSetDevice(c->device));
    size_t b = (size_t)(c->q - 1) * c->N * sizeof(double);
    double* d = (double*)dalloc(c, b);
    HIPCHK(hipMemcpyAsync(d, f, b, hipMemcpyHostToDevice, c->stream));
    lbm_set_pdfs(c, d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, d);
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_pdfs(iblbm_ctx* c, double* f) {
  if (!c || !f) return IBLBM_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    size_t b = (size_t)(c->q - 1) * c->N * sizeof(double);
    double* d = (double*)dalloc(c, b);
    lbm_get_pdfs(c, d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(f, d, b, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, d);
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_add_particles(iblbm_ctx* c, int32_t n, const double* center,
                                 const double* diameter, const double* density,
                                 const double* velocity, const double* omega,
                                 int32_t markers_per_particle) {
  iblbm_status s = check_ready(c);
  if (s) return s;
  if (n < 0 || (n > 0 && (!center || !diameter || !density)))
    return fail(c, IBLBM_E_ARG, "bad particle arrays");
  if (n == 0) return IBLBM_OK;
  int dim = c->dim;
  for (int a = 0; a < 3; a++)
    if (c->cfg.periodic[a]) return fail(c, IBLBM_E_ARG, "particles need walls on every axis");
  // validation on the host in FP64
  std::vector<double> allX = c->hX;
  std::vector<double> allD = c->hD;
  for (int i = 0; i < n; i++) {
    double D = diameter[i], R = 0.5 * D;
    if (!(D > 0) || !(density[i] > 0)) return fail(c, IBLBM_E_ARG, "diameter and density must be > 0");
    if (dim == 3 && D > 40.0) return fail(c, IBLBM_E_ARG, "3-D diameter above 40 lattice units");
    for (int a = 0; a < dim; a++)
      if (center[3 * i + a] - R < -0.5 || center[3 * i + a] + R > c->cfg.n[a] - 0.5)
        return fail(c, IBLBM_E_ARG, "particle surface outside the walls");
    for (size_t j = 0; j < allD.size(); j++) {
      double d2 = 0;
      for (int a = 0; a < dim; a++) {
        double dx = center[3 * i + a] - allX[3 * j + a];
        d2 += dx * dx;
      }
      double sr = 0.5 * (D + allD[j]);
      if (d2 < sr * sr) return fail(c, IBLBM_E_ARG, "overlapping particles");
    }
    for (int a = 0; a < 3; a++) allX.push_back(a < dim ? center[3 * i + a] : 0.0);
    allD.push_back(D);
  }
  try {
    HIPCHK(hipSetDevice(c->device));
    int np0 = c->np, np = c->np + n;
    double gmag = sqrt(c->cfg.gravity[0] * c->cfg.gravity[0] + c->cfg.gravity[1] * c->cfg.gravity[1] +
                       c->cfg.gravity[2] * c->cfg.gravity[2]);
    std::vector<double> X(3 * n), U(3 * n, 0.0), W(3 * n, 0.0), Dv(n), rho(n), M(n), V(n), I(n), cb(n);
    std::vector<int> mstart(n), mcount(n);
    std::vector<double> mr, mdV;
    std::vector<int> mown;
    int nmk = c->nmk;
    for (int i = 0; i < n; i++) {
      double D = diameter[i], R = 0.5 * D;
      for (int a = 0; a < 3; a++) {
        X[3 * i + a] = a < dim ? center[3 * i + a] : 0.0;
        U[3 * i + a] = (velocity && a < dim) ? velocity[3 * i + a] : 0.0;
        W[3 * i + a] = omega ? omega[3 * i + a] : 0.0;
      }
      if (dim == 2) W[3 * i] = W[3 * i + 1] = 0.0;
      Dv[i] = D;
      rho[i] = density[i];
      V[i] = dim == 2 ? PI * R * R : 4.0 / 3.0 * PI * R * R * R;
      M[i] = density[i] * V[i];
      I[i] = dim == 2 ? 0.5 * M[i] * R * R : 0.4 * M[i] * R * R;
      cb[i] = (density[i] - c->cfg.rho0) * V[i] * gmag;
      int nl = markers_per_particle > 0
                   ? markers_per_particle
                   : (int)floor((dim == 2 ? PI * D : PI * D * D) + 0.5);
      mstart[i] = nmk;
      mcount[i] = nl;
      double ds = dim == 2 ? PI * D / nl : PI * D * D / nl;
      marker_offsets(dim, R, nl, mr);
      for (int k = 0; k < nl; k++) {
        mdV.push_back(c->cfg.drs * ds);
        mown.push_back(np0 + i);
      }
      nmk += nl;
    }
    if ((long long)nmk * 64 >= (1LL << 31)) throw Fail{fail(c, IBLBM_E_ARG, "too many surface points")};
    // particle arrays
    size_t o3 = 3 * (size_t)np0, n3 = 3 * (size_t)np;
    double** a3[] = {&c->X, &c->U, &c->Om, &c->Fh, &c->Th, &c->Fc, &c->Pin, &c->Lin,
                     &c->Pprev, &c->Lprev, &c->Hprev, &c->Gprev};
    for (auto pp : a3) grow<double>(c, *pp, o3, n3);
    double** a1[] = {&c->D, &c->rho, &c->M, &c->V, &c->I, &c->cb};
    for (auto pp : a1) grow<double>(c, *pp, np0, np);
    grow<int>(c, c->mstart, np0, np);
    grow<int>(c, c->mcount, np0, np);
    HIPCHK(hipMemcpyAsync(c->X + o3, X.data(), 3 * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->U + o3, U.data(), 3 * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->Om + o3, W.data(), 3 * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->D + np0, Dv.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->rho + np0, rho.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->M + np0, M.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->V + np0, V.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->I + np0, I.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->cb + np0, cb.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->mstart + np0, mstart.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->mcount + np0, mcount.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    // markers
    int nm0 = c->nmk, nadd = nmk - nm0;
    size_t cs = c->fp64 ? 8 : 4;
    grow<int>(c, c->mown, nm0, nmk);
    grow<double>(c, c->mr, 4 * (size_t)nm0, 4 * (size_t)nmk);
    grow<double>(c, c->mdV, nm0, nmk);
    growv(c, c->mF, 4 * nm0 * cs, 4 * (size_t)nmk * cs);
    growv(c, c->mdF, 4 * nm0 * cs, 4 * (size_t)nmk * cs);
    growv(c, c->mFprev, 4 * nm0 * cs, 4 * (size_t)nmk * cs);
    {
      float* nf = nullptr;
      grow<float>(c, nf, 0, 10 * (size_t)nmk);
      if (c->feat) dfree(c, c->feat);
      c->feat = nf;
    }
    HIPCHK(hipMemcpyAsync(c->mown + nm0, mown.data(), nadd * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->mr + 4 * (size_t)nm0, mr.data(), 4 * (size_t)nadd * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->mdV + nm0, mdV.data(), nadd * 8, hipMemcpyHostToDevice, c->stream));
    c->np = np;
    c->nmk = nmk;
    c->hX = allX;
    c->hD = allD;
    c->hcount.insert(c->hcount.end(), mcount.begin(), mcount.end());
    c->hstart.insert(c->hstart.end(), mstart.begin(), mstart.end());
    c->hmr.insert(c->hmr.end(), mr.begin(), mr.end());
    // cell grid (Eqs. 49-50) and pair buffers
    double H = compute_H(c);
    long long ncell = 1;
    for (int a = 0; a < 3; a++) {
      c->nc[a] = 1;
      c->invh[a] = 0.0;
      if (a < dim) {
        int m = (int)floor(c->cfg.n[a] / H);
        if (m < 1) m = 1;
        c->nc[a] = m;
        c->invh[a] = (double)m / (double)c->cfg.n[a];
      }
      ncell *= c->nc[a];
    }
    if (c->cell_count) dfree(c, c->cell_count);
    if (c->cell_items) dfree(c, c->cell_items);
    c->ncell = ncell;
    c->cell_count = dzeros<int>(c, (size_t)ncell);
    c->cell_items = dzeros<int>(c, (size_t)ncell * CELL_CAP);
    if (c->cell_of) dfree(c, c->cell_of);
    if (c->pair_up) dfree(c, c->pair_up);
    if (c->pair_nup) dfree(c, c->pair_nup);
    if (c->pair_all) dfree(c, c->pair_all);
    if (c->pair_nall) dfree(c, c->pair_nall);
    // work units of the per-particle LDS kernels and their touched-node lists
    build_patches(c);
    if (c->tlist) dfree(c, c->tlist);
    if (c->tcount) dfree(c, c->tcount);
    if (c->slip_part) dfree(c, c->slip_part);
    c->tlist = dzeros<uint16_t>(c, (size_t)c->npatch * (c->box_cap <= 65536 ? c->box_cap : 1));
    c->tcount = dzeros<int>(c, (size_t)c->npatch);
    c->slip_part = dzeros<double>(c, (size_t)c->npatch);
    c->cell_of = dzeros<int>(c, 3 * (size_t)np);
    c->pair_up = dzeros<int>(c, (size_t)np * PAIR_CAP);
    c->pair_nup = dzeros<int>(c, (size_t)np);
    c->pair_all = dzeros<int>(c, (size_t)np * PAIR_CAP);
    c->pair_nall = dzeros<int>(c, (size_t)np);
    // cells and pairs of the initial positions; then empty the cells again
    part_cells_pairs(c);
    part_zero_cells(c);
    // interior fluid momentum of the new particles in the current fluid
    lbm_interior_momentum(c, c->Pin, c->Lin, false);
    HIPCHK(hipMemcpyAsync(c->Pprev + o3, c->Pin + o3, 3 * n * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->Lprev + o3, c->Lin + o3, 3 * n * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->graph_dirty = true;
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_step(iblbm_ctx* c, int32_t nsteps) {
  iblbm_status s = check_ready(c);
  if (s) return s;
  if (nsteps < 0) return fail(c, IBLBM_E_ARG, "negative step count");
  try {
    HIPCHK(hipSetDevice(c->device));
    for (int k = 0; k < nsteps; k++) {
      // graphs replay plain steps; timed steps and steps that gather the slip
      // statistic are launched one kernel at a time
      const bool stats_step = c->cfg.stats_every > 0 && c->step % c->cfg.stats_every == 0;
      if (c->use_graph && !c->timing && !stats_step)
        step_graph(c);
      else
        enqueue_step(c);
      if (c->timing && c->ev_used > 4000) flush_timing(c);
    }
    HIPCHK(hipGetLastError());
    int flags = 0;
    read_status(c, &flags);
    flush_timing(c);
    if (c->cfg.stats_every > 0 && c->nmk > 0) {
      double s2 = 0;
      HIPCHK(hipMemcpy(&s2, c->dstats, sizeof(double), hipMemcpyDeviceToHost));
      c->slip_rms = sqrt(s2 / c->nmk);
    }
    if (flags & ST_NAN) return fail(c, IBLBM_E_UNSTABLE, "NaN/Inf or runaway particle velocity");
    if (flags & ST_CELL_OVERFLOW)
      return fail(c, IBLBM_E_CELL_OVERFLOW, "more particle centres in a search cell than it holds");
    if (flags & ST_PAIR_OVERFLOW)
      return fail(c, IBLBM_E_CAPACITY, "pair list capacity exceeded");
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_fields(iblbm_ctx* c, double* p, double* u, double* force) {
  if (!c) return IBLBM_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    size_t N = c->N;
    double* dp = p ? (double*)dalloc(c, N * 8) : nullptr;
    double* du = u ? (double*)dalloc(c, N * c->dim * 8) : nullptr;
    double* df = force ? (double*)dalloc(c, N * c->dim * 8) : nullptr;
    lbm_get_fields(c, dp, du, df);
    HIPCHK(hipGetLastError());
    if (p) HIPCHK(hipMemcpyAsync(p, dp, N * 8, hipMemcpyDeviceToHost, c->stream));
    if (u) HIPCHK(hipMemcpyAsync(u, du, N * c->dim * 8, hipMemcpyDeviceToHost, c->stream));
    if (force) HIPCHK(hipMemcpyAsync(force, df, N * c->dim * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    dfree(c, dp);
    dfree(c, du);
    dfree(c, df);
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_forces(iblbm_ctx* c, double* X, double* U, double* Om, double* Fh,
                              double* Th, double* Fc, double* marker_F) {
  if (!c) return IBLBM_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    size_t b = 3 * (size_t)c->np * 8;
    const double* src[] = {c->X, c->U, c->Om, c->Fh, c->Th, c->Fc};
    double* dst[] = {X, U, Om, Fh, Th, Fc};
    for (int k = 0; k < 6; k++)
      if (dst[k] && c->np) HIPCHK(hipMemcpyAsync(dst[k], src[k], b, hipMemcpyDeviceToHost, c->stream));
    std::vector<char> mf;
    size_t cs = c->fp64 ? 8 : 4;
    if (marker_F && c->nmk) {
      mf.resize(4 * (size_t)c->nmk * cs);
      HIPCHK(hipMemcpyAsync(mf.data(), c->mF, mf.size(), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if (marker_F)
      for (int k = 0; k < c->nmk; k++)
        for (int a = 0; a < 3; a++)
          marker_F[3 * k + a] = c->fp64 ? ((double*)mf.data())[4 * k + a] : ((float*)mf.data())[4 * k + a];
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_pairs(iblbm_ctx* c, int32_t* ij, int64_t cap, int64_t* n_pairs) {
  if (!c || !n_pairs) return IBLBM_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    std::vector<int> nup(c->np), up((size_t)c->np * PAIR_CAP);
    if (c->np) {
      HIPCHK(hipMemcpyAsync(nup.data(), c->pair_nup, c->np * 4, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(up.data(), c->pair_up, up.size() * 4, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    int64_t m = 0;
    for (int i = 0; i < c->np; i++)
      for (int k = 0; k < nup[i]; k++) {
        if (ij && m < cap) {
          ij[2 * m] = i;
          ij[2 * m + 1] = up[(size_t)i * PAIR_CAP + k];
        }
        m++;
      }
    *n_pairs = m;
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_cells(iblbm_ctx* c, int32_t* cell, int32_t* dims) {
  if (!c) return IBLBM_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    if (dims)
      for (int a = 0; a < 3; a++) dims[a] = c->nc[a];
    if (cell && c->np) {
      HIPCHK(hipMemcpyAsync(cell, c->cell_of, 3 * (size_t)c->np * 4, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
  } catch (Fail& e) {
    return e.st;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_get_stats(iblbm_ctx* c, iblbm_stats* o) {
  if (!c || !o) return IBLBM_E_ARG;
  memset(o, 0, sizeof(*o));
  try {
    HIPCHK(hipSetDevice(c->device));
    int st[4];
    std::vector<uint32_t> bm((size_t)c->nwords);
    HIPCHK(hipMemcpyAsync(st, c->dstatus, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(bm.data(), c->bmap + (size_t)c->fbuf * c->nwords, bm.size() * 4,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    long long band = 0;
    for (uint32_t w : bm) band += __builtin_popcount(w);
    o->flags = st[0];
    unsigned long long t;
    memcpy(&t, st + 2, sizeof(t));
    o->truncated = (long long)t;
    o->band_nodes = band;
    int64_t npairs = 0;
    iblbm_get_pairs(c, nullptr, 0, &npairs);
    o->n_pairs = npairs;
  } catch (Fail& e) {
    return e.st;
  }
  o->step = c->step;
  o->slip_rms = c->slip_rms;
  o->fallbacks = c->fallbacks;
  o->band_lattice = ibm_ustar_lattice(c) ? 1 : 0;
  for (int g = 0; g < IBLBM_NGROUPS; g++) {
    o->time_ms[g] = c->time_ms[g];
    o->launches[g] = c->launches[g];
  }
  return IBLBM_OK;
}

iblbm_status iblbm_num_particles(iblbm_ctx* c, int32_t* np, int32_t* nmk) {
  if (!c) return IBLBM_E_ARG;
  if (np) *np = c->np;
  if (nmk) *nmk = c->nmk;
  return IBLBM_OK;
}

iblbm_status iblbm_set_timing(iblbm_ctx* c, int32_t mask) {
  if (!c) return IBLBM_E_ARG;
  c->timing = mask != 0;
  c->timing_mask = mask == -1 ? 0xff : mask;
  return IBLBM_OK;
}

iblbm_status iblbm_reset_stats(iblbm_ctx* c) {
  if (!c) return IBLBM_E_ARG;
  for (int g = 0; g < IBLBM_NGROUPS; g++) {
    c->time_ms[g] = 0;
    c->launches[g] = 0;
  }
  c->ev_used = 0;
  return IBLBM_OK;
}

iblbm_status iblbm_set_option(iblbm_ctx* c, int32_t option, int32_t value) {
  if (!c) return IBLBM_E_ARG;
  if (option == IBLBM_OPT_IBM_LDS) {
    c->ibm_lds = value != 0;
    c->graph_dirty = true;
    return IBLBM_OK;
  }
  if (option == IBLBM_OPT_BAND_PASS) {
    c->band_pass = value != 0 ? 1 : 0;
    c->graph_dirty = true;
    return IBLBM_OK;
  }
  if (option == IBLBM_OPT_TIMING_KERNEL) {
    if (value != 0 && value != 1) return fail(c, IBLBM_E_ARG, "timing_kernel must be 0 or 1");
    c->timing_kernel = value == 1;
    return IBLBM_OK;
  }
  if (option == IBLBM_OPT_TIMING_EVERY) {
    if (value < 1) return fail(c, IBLBM_E_ARG, "timing_every must be >= 1");
    c->timing_every = value;
    return IBLBM_OK;
  }
  if (option == IBLBM_OPT_STATS_EVERY) {
    if (value < 0) return fail(c, IBLBM_E_ARG, "stats_every must be >= 0");
    c->cfg.stats_every = value;
    c->graph_dirty = true;
    return IBLBM_OK;
  }
  return fail(c, IBLBM_E_ARG, "unknown option");
}

iblbm_status iblbm_plan_units(int32_t dim, int32_t storage, int32_t lds_bytes, double diameter,
                              int32_t n_points, int32_t cap, int32_t* n_units, int32_t* first,
                              int32_t* count, int64_t* box_nodes) {
  if ((dim != 2 && dim != 3) || storage < IBLBM_F64 || storage > IBLBM_F16 || lds_bytes < 0 ||
      !(diameter > 0.0 && diameter <= 4096.0) || n_points < 0 || n_points > (1 << 24) ||
      cap < 0 || !n_units)
    return IBLBM_E_ARG;
  const int lds = lds_bytes > 0 ? lds_bytes : 160 * 1024;
  const int nl = n_points > 0 ? n_points
                              : (int)floor((dim == 2 ? PI * diameter : PI * diameter * diameter) + 0.5);
  if (lds <= 1024 || nl < 1 || nl > (1 << 24)) return IBLBM_E_ARG;
  try {
    std::vector<double> offs;
    marker_offsets(dim, 0.5 * diameter, nl, offs);
    std::vector<UnitPlan> units;
    const bool ok = plan_particle(dim, unit_nmax(dim, storage == IBLBM_F64 ? 8 : 4, lds), diameter,
                                  offs.data(), nl, units);
    *n_units = ok ? (int32_t)units.size() : 0;
    for (int u = 0; ok && u < (int)units.size() && u < cap; u++) {
      if (first) first[u] = units[u].m0;
      if (count) count[u] = units[u].mc;
      if (box_nodes) box_nodes[u] = units[u].nodes;
    }
  } catch (const std::bad_alloc&) {
    return IBLBM_E_NOMEM;
  }
  return IBLBM_OK;
}

iblbm_status iblbm_set_graph(iblbm_ctx* c, int32_t on) {
  if (!c) return IBLBM_E_ARG;
  c->use_graph = on != 0;
  c->graph_dirty = true;
  return IBLBM_OK;
}

}  // extern "C"

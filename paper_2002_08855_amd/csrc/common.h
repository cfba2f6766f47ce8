// Internal declarations of the gfx950 IB-LBM library: lattice tables, storage traits,
// device-state layout and the launchers each translation unit provides.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/iblbm.h"

// ---------------------------------------------------------------------------
// Lattices.  D2Q9 follows Eq. 2 and D3Q19 Eq. 3 (third row completed so that
// e_9 = (-1,0,1)); directions alpha > (q-1)/2 are the negatives of alpha-(q-1)/2.
template <int DIM>
struct Lat;
template <>
struct Lat<2> {
  static constexpr int Q = 9, H = 4;
  static constexpr int ex[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
  static constexpr int ey[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36,
                                  1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};
};
template <>
struct Lat<3> {
  static constexpr int Q = 19, H = 9;
  static constexpr int ex[19] = {0, 1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 0, 0, -1, 1, 0, 0, -1, 1};
  static constexpr int ey[19] = {0, 0, 1, 0, 1, 1, 1, -1, 0, 0, 0, -1, 0, -1, -1, -1, 1, 0, 0};
  static constexpr int ez[19] = {0, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
__host__ __device__ constexpr int opp_dir(int a, int h) { return a <= h ? a + h : a - h; }

// ---------------------------------------------------------------------------
// PDF storage types.  The compute type is double for FP64 storage, float otherwise.
struct bf16s {
  uint16_t v;
};
template <class T>
struct Store;
template <>
struct Store<double> {
  using C = double;
  __device__ static double load(double s, double) { return s; }
  __device__ static double save(double f, double) { return f; }
};
template <>
struct Store<float> {
  using C = float;
  __device__ static float load(float s, float) { return s; }
  __device__ static float save(float f, float) { return f; }
};
template <>
struct Store<bf16s> {
  using C = float;
  __device__ static float load(bf16s s, float) { return __uint_as_float(uint32_t(s.v) << 16); }
  // round to nearest even; NaN stays NaN
  __device__ static bf16s save(float f, float) {
    uint32_t u = __float_as_uint(f);
    bf16s r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      r.v = uint16_t((u >> 16) | 0x40u);
      return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    r.v = uint16_t(u >> 16);
    return r;
  }
};
template <>
struct Store<__half> {
  using C = float;
  // stored value = scale * f; load multiplies by 1/scale (exact for a power of two)
  __device__ static float load(__half s, float inv_scale) { return __half2float(s) * inv_scale; }
  __device__ static __half save(float f, float inv_scale) { return __float2half(f / inv_scale); }
};

// ---------------------------------------------------------------------------
// Geometry shared by the fluid kernels.
template <class C>
struct Geo {
  int n[3];
  int periodic[3];
  long long N;
  C rho0;
  C wt[19][6];  // 2 w_a rho0 (e_a . u_wall[face]) / cs^2
};

// Segment flags: one 32-bit word per 16 consecutive x-nodes of a row.
constexpr int SEG = 16;

// ---------------------------------------------------------------------------
// Host-side context.
struct iblbm_ctx {
  iblbm_config cfg;
  int dim = 2, q = 9;
  long long N = 0;
  int storage = 0;
  size_t sbytes = 8;  // bytes per stored PDF
  bool fp64 = true;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::string err;
  int sticky = 0;
  long long step = 0;
  int parity = 0;  // 0: natural layout; 1: A-A swapped layout
  // fluid
  void* f = nullptr;        // (q-1) x N, storage type
  void* ustar = nullptr;    // band u*, N x VD compute type
  void* facc = nullptr;     // IB force density, N x VD compute type
  int vd = 2;               // vector stride of ustar / facc (2 in 2-D, 3 in 3-D, packed)
  uint32_t* bmap = nullptr;   // 2 x nwords band bitmaps (bit per node), one per step parity
  long long nwords = 0, nwx = 0;  // words per bitmap, 32-node words per row
  int fbuf = 0;               // bitmap of the most recent step
  uint32_t* bflag = nullptr;  // nseg segment flags (per-point fallback band)
  int* seglist = nullptr;     // flagged segments
  int* segcount = nullptr;    // number of listed segments
  long long nseg = 0, nsegx = 0;
  // particles (FP64)
  int np = 0, capp = 0;
  double *X = nullptr, *U = nullptr, *Om = nullptr, *Fh = nullptr, *Th = nullptr,
         *Fc = nullptr, *Pin = nullptr, *Lin = nullptr, *Pprev = nullptr, *Lprev = nullptr,
         *Hprev = nullptr, *Gprev = nullptr;
  double *D = nullptr, *rho = nullptr, *M = nullptr, *V = nullptr, *I = nullptr,
         *cb = nullptr;
  int *mstart = nullptr, *mcount = nullptr;
  std::vector<double> hD, hX;  // host copies used for validation
  std::vector<int> hcount;
  double dmax = 0.0;
  int box_cap = 0;     // nodes in the largest work unit's support box
  int full_side = 0;   // nodes a side of the largest particle's whole support box
  int lds_max = 65536; // LDS bytes a workgroup may use on this device
  bool ibm_lds = true; // per-particle LDS kernels for interpolation and spreading
  int band_pass = -1;   // band u* in its own pass (1) or in the first interpolation (0);
                        // -1: by dimension and box coverage (box_cover)
  // the next interpolation pass builds the band: 0 no, 1 with u* from the PDFs at the
  // band, 2 with u* from the lattice u* pass
  int band_pending = 0;
  bool ustar_valid = false;   // ustar holds u* of every node for the current PDFs
  // markers
  int nmk = 0, capm = 0;
  int* mown = nullptr;
  double* mr = nullptr;     // nmk x 4 offsets r_k (FP64)
  double* mdV = nullptr;    // nmk
  void* mF = nullptr;       // accumulated force, nmk x 4 compute type
  void* mdF = nullptr;      // pass increment, nmk x 4
  void* mFprev = nullptr;   // previous-step force, nmk x 4
  // cells and pairs
  int nc[3] = {1, 1, 1};
  double invh[3] = {0, 0, 0};
  long long ncell = 0;
  int* cell_count = nullptr;
  int* cell_items = nullptr;  // ncell x CELL_CAP
  int* cell_of = nullptr;     // np x 3
  int* pair_up = nullptr;     // np x PAIR_CAP partners j > i, ascending
  int* pair_nup = nullptr;    // np
  int* pair_all = nullptr;    // np x PAIR_CAP all partners, ascending
  int* pair_nall = nullptr;   // np
  // work units of the per-particle LDS kernels: one per particle, or runs of consecutive
  // points of a particle too large for one workgroup, each with its own box
  int npatch = 0;
  bool patched = false;       // some particle has more than one unit
  bool patch_ok = false;      // every unit fits one workgroup
  double box_cover = 0.0;     // sum of the units' box nodes over the lattice nodes
  int *pt_owner = nullptr, *pt_m0 = nullptr, *pt_mc = nullptr;  // npatch
  double *pt_rlo = nullptr, *pt_rhi = nullptr;                  // npatch x 3 offset range
  std::vector<int> hpt_mc;    // host copy of pt_mc
  std::vector<int> hstart;    // host copy of mstart
  std::vector<double> hmr;    // host copy of the point offsets (4 per point)
  uint16_t* tlist = nullptr;  // npatch x box_cap: touched box nodes of each unit, ascending
  int* tcount = nullptr;      // npatch: entries of tlist per unit
  double* slip_part = nullptr;  // npatch: per-unit sums of the slip statistic
  // status and statistics
  int* dstatus = nullptr;     // [0] flags, [1] truncated (int64 at [2..3]), ...
  double* dstats = nullptr;   // [0] slip sum of squares
  long long truncated = 0;
  double slip_rms = 0.0;
  int fallbacks = 0;
  // learned forcing
  bool has_mlp = false;
  void* mlp_w = nullptr;      // packed weights for inference
  float* mlp_norm = nullptr;  // 26 floats
  float* feat = nullptr;      // nmk x 10 scratch
  int* dcond = nullptr;       // device flag: run the MDF fallback of this step
  const int* cond = nullptr;  // when set, IBM kernels run only if *cond != 0
  // timing
  bool timing = false;
  int timing_mask = 0;  // bit g: time kernel group g
  int timing_every = 1; // time the launches of every timing_every-th step only
  bool timing_kernel = false;  // collide, interp, spread: events with the kernel launch
  bool t_open = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_group;
  size_t ev_used = 0;
  double time_ms[IBLBM_NGROUPS] = {0};
  long long launches[IBLBM_NGROUPS] = {0};
  // graphs
  bool use_graph = false;
  // one captured step per (PDF parity, band-bitmap buffer), and the host-side flags the
  // captured step left behind
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  int gend_band_pending[4] = {0, 0, 0, 0};
  bool gend_ustar_valid[4] = {false, false, false, false};
  bool graph_dirty = true;
  bool capturing = false;  // enqueue_step is being recorded into a graph
  int* hflag = nullptr;          // pinned host word: the learned step's fallback verdict
  hipEvent_t ev_flag = nullptr;  // recorded once the verdict has been copied to hflag
  // allocations
  std::vector<void*> allocs;
};

constexpr int CELL_CAP = 8;
constexpr int LDS_THREADS = 1024;  // largest workgroup of the per-particle LDS kernels
constexpr int PAIR_CAP = 24;
constexpr int MAX_BOX_3D = 46;  // D <= 40 with a 4-point stencil

// status bits
constexpr int ST_CELL_OVERFLOW = 1, ST_PAIR_OVERFLOW = 2, ST_NAN = 4;

// Once a runaway particle (|U| > 1 lattice unit per step, or NaN) has been flagged in the
// device status word, the particle and IB kernels of later launches return at once: a
// diverging run stops moving its bodies through the lattice, and iblbm_step reports
// IBLBM_E_UNSTABLE when it returns.  The flag is set only inside the particle update,
// which does not test it, so every other launch sees one value throughout.
__device__ __forceinline__ bool halted(const int* status) {
  return status != nullptr && (*status & ST_NAN) != 0;
}

// ---------------------------------------------------------------------------
// Launchers (all enqueue on ctx->stream).
void lbm_init_equilibrium(iblbm_ctx* c, const double* dp, const double* du);
void lbm_set_pdfs(iblbm_ctx* c, const double* df);
void lbm_get_pdfs(iblbm_ctx* c, double* df);
void lbm_get_fields(iblbm_ctx* c, double* dp, double* du, double* dforce);
void lbm_collide_stream(iblbm_ctx* c);
void lbm_face_bc(iblbm_ctx* c);  // after the parity flip: extrapolated faces for the next step
void ibm_band(iblbm_ctx* c);
bool ibm_uses_lds(const iblbm_ctx* c);
void ibm_interp(iblbm_ctx* c, int first_pass, int mode);
void ibm_spread(iblbm_ctx* c, int use_set);
void lbm_interior_momentum(iblbm_ctx* c, double* P, double* L, bool from_ustar);
void lbm_ustar_all(iblbm_ctx* c);
bool ibm_ustar_lattice(const iblbm_ctx* c);
void ibm_slip(iblbm_ctx* c);
void part_cells_pairs(iblbm_ctx* c);
void part_loads_newton(iblbm_ctx* c);
void mlp_features(iblbm_ctx* c);
void ibm_band_redo(iblbm_ctx* c);
void ibm_prepare_launches(iblbm_ctx* c);
void mlp_infer(iblbm_ctx* c);

// timing helpers (host.hip)
void tbegin(iblbm_ctx* c, int group);
// with kernel-only timing of `group` due in this step: a start and a stop event for the
// group's kernel launch (hipExtLaunchKernelGGL); false otherwise
bool kernel_events(iblbm_ctx* c, int group, hipEvent_t* start, hipEvent_t* stop);
// a failed HIP call inside a step: records the error on the context and unwinds the
// step (to the entry point, which returns IBLBM_E_DEVICE)
void hip_check(iblbm_ctx* c, hipError_t e, const char* expr);
// device memory through the caller's allocator callbacks when given (else hipMalloc),
// released with the context; nullptr (and the context's error set) on failure
void* ctx_alloc(iblbm_ctx* c, size_t bytes);
void tend(iblbm_ctx* c);

// Learned boundary force for gfx950: a 10-64-64-3 MLP (tanh hidden layers) predicts the
// converged multi-direct-forcing force of every Lagrangian point from its pass-0 slip,
// its previous-step force, its unit normal and the gap to the nearest other surface.
//
// Inference runs on the BF16 matrix cores with FP32 accumulation (v_mfma_f32_16x16x16_bf16
// for the 10-input layer, v_mfma_f32_16x16x32_bf16 for the two 64-input layers).  Each
// layer is computed transposed, H^T = W X^T: the weights are the A operand and a 16-point
// tile of activations the B operand, so the D fragment of one layer is the B fragment the
// next layer needs and no data moves between layers.  One wavefront walks 16-point tiles
// with all weights held in registers.
//
// Training uses the same library: FP32 GEMMs through LDS tiles (the weight gradients with
// the batch split over blocks and the partials added in a fixed order), fused elementwise
// kernels and Adam, all on the GPU.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.h"

void ibm_band(iblbm_ctx* c);
void part_cells_pairs(iblbm_ctx* c);
void part_zero_cells(iblbm_ctx* c);

namespace {

constexpr int NI = 10, NH = 64, NO = 3;
constexpr int INFER_WAVES = 256 * 4 * 3;
constexpr int NPARAM = NI * NH + NH + NH * NH + NH + NH * NO + NO;
constexpr int OFF_W1 = 0, OFF_B1 = NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NO;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  // round to nearest even (v_cvt_pk_bf16_f32)
  return __builtin_bit_cast(short, (__bf16)f);
}

// tanh x = 1 - 2 / (e^{2x} + 1): one exponential and one reciprocal, saturating to +-1
// without a clamp (e^{2x} overflows to inf or underflows to 0).  Its error, about one
// FP32 ulp of 1, is far below the BF16 rounding that follows.
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 / ln 2
  return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

struct InferArgs {
  const float* P;     // FP32 parameters
  const float* norm;  // mean[10], std[10], tmean[3], tstd[3]
  const float* feat;  // n x 10, un-normalised
  int n;
  int dim;
  void* F;   // n x 4 compute type (set to the prediction)
  void* dF;  // n x 4 compute type
  const void* Fprev;  // n x 4 compute type: the previous step's force
  int fp64;
  float* y;  // optional n x 3 raw outputs (normalised units)
};

// Layer 1 (K = 10 inputs, padded to 16) uses v_mfma_f32_16x16x16_bf16: lane l holds
// A = W[rb*16 + l%16][4(l/16) + v] and B = X[4(l/16) + v][point l%16], v < 4.
__device__ __forceinline__ bf16x4 wfrag16(const float* W, int rows, int cols, int rb, int lane) {
  bf16x4 a;
  const int i = rb * 16 + (lane & 15), k0 = 4 * (lane >> 4);
  for (int v = 0; v < 4; v++) {
    const int k = k0 + v;
    a[v] = (i < rows && k < cols) ? to_bf16(W[i * cols + k]) : short(0);
  }
  return a;
}

// Layers 2 and 3 (K = 64) use v_mfma_f32_16x16x32_bf16, two K blocks of 32.  A layer's
// D fragment leaves lane l with units 16 rb + 4(l/16) + v (v < 4) of each 16-unit row
// block rb; the B fragment of K block kb takes, in its 8 slots, those of row blocks 2kb
// (slots 0-3) and 2kb+1 (slots 4-7).  The contraction runs over whatever order the
// slots stand for, so the weights are loaded in the same order: slot v of lane l holds
// unit 32 kb + 16 (v/4) + 4(l/16) + v%4, and no data moves between layers.
__device__ __forceinline__ int kunit(int kb, int lane, int v) {
  return 32 * kb + 16 * (v >> 2) + 4 * (lane >> 4) + (v & 3);
}

__device__ __forceinline__ bf16x8 wfrag32(const float* W, int rows, int cols, int rb, int kb,
                                          int lane) {
  bf16x8 a;
  const int i = rb * 16 + (lane & 15);
  for (int v = 0; v < 8; v++) a[v] = i < rows ? to_bf16(W[i * cols + kunit(kb, lane, v)]) : short(0);
  return a;
}

// bias in the D layout: lane l holds units rb*16 + 4(l/16) + v
__device__ __forceinline__ floatx4 bfrag(const float* b, int rows, int rb, int lane) {
  floatx4 c;
  for (int v = 0; v < 4; v++) {
    int i = rb * 16 + 4 * (lane >> 4) + v;
    c[v] = i < rows ? b[i] : 0.f;
  }
  return c;
}

// One wavefront walks 16-point tiles with every weight in registers; the features of
// the next tile are loaded before the current one is computed.
__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  const float* P = a.P;
  bf16x4 a1[4];
  bf16x8 a2[4][2], a3[2];
  floatx4 c1[4], c2[4], c3;
  for (int rb = 0; rb < 4; rb++) {
    a1[rb] = wfrag16(P + OFF_W1, NH, NI, rb, lane);
    c1[rb] = bfrag(P + OFF_B1, NH, rb, lane);
    c2[rb] = bfrag(P + OFF_B2, NH, rb, lane);
    for (int kb = 0; kb < 2; kb++) a2[rb][kb] = wfrag32(P + OFF_W2, NH, NH, rb, kb, lane);
  }
  for (int kb = 0; kb < 2; kb++) a3[kb] = wfrag32(P + OFF_W3, NO, NH, 0, kb, lane);
  c3 = bfrag(P + OFF_B3, NO, 0, lane);
  // this lane's four input features: mean and reciprocal standard deviation
  const int j = lane & 15, kq = 4 * (lane >> 4);
  float mu[4], isd[4];
  for (int v = 0; v < 4; v++) {
    const int k = kq + v;
    mu[v] = k < NI ? a.norm[k] : 0.f;
    isd[v] = k < NI ? 1.f / a.norm[NI + k] : 0.f;
  }
  const float* tmean = a.norm + 2 * NI;
  const float* tsd = a.norm + 2 * NI + NO;
  float xin[4];
  auto load_tile = [&](int t0) {
    const int m = t0 + j;
    for (int v = 0; v < 4; v++) {
      const int k = kq + v;
      xin[v] = (m < a.n && k < NI) ? a.feat[(size_t)m * NI + k] : 0.f;
    }
  };
  int t0 = wave * 16;
  if (t0 < a.n) load_tile(t0);
  for (; t0 < a.n; t0 += nwaves * 16) {
    const int m = t0 + j;
    const bool ok = m < a.n;
    bf16x4 b1;
    for (int v = 0; v < 4; v++) b1[v] = to_bf16((xin[v] - mu[v]) * isd[v]);
    if (t0 + nwaves * 16 < a.n) load_tile(t0 + nwaves * 16);
    bf16x8 b2[2], b3[2];
    for (int rb = 0; rb < 4; rb++) {
      const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[rb], b1, c1[rb], 0, 0, 0);
      for (int v = 0; v < 4; v++) b2[rb >> 1][4 * (rb & 1) + v] = to_bf16(fast_tanh(d[v]));
    }
    for (int rb = 0; rb < 4; rb++) {
      floatx4 d = c2[rb];
      for (int kb = 0; kb < 2; kb++)
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[rb][kb], b2[kb], d, 0, 0, 0);
      for (int v = 0; v < 4; v++) b3[rb >> 1][4 * (rb & 1) + v] = to_bf16(fast_tanh(d[v]));
    }
    floatx4 d = c3;
    for (int kb = 0; kb < 2; kb++)
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[kb], b3[kb], d, 0, 0, 0);
    // lanes 0..15 hold the three outputs of point m in d[0..2]
    if (lane < 16 && ok) {
      if (a.y)
        for (int o = 0; o < NO; o++) a.y[(size_t)m * NO + o] = d[o];
      if (a.F) {
        // the network predicts the change over the previous step's force
        for (int o = 0; o < 3; o++) {
          const float dv = tmean[o] + tsd[o] * d[o];
          if (a.fp64) {
            const double val = o < a.dim ? ((const double*)a.Fprev)[4 * (size_t)m + o] + double(dv) : 0.0;
            ((double*)a.F)[4 * (size_t)m + o] = val;
            ((double*)a.dF)[4 * (size_t)m + o] = val;
          } else {
            const float val = o < a.dim ? ((const float*)a.Fprev)[4 * (size_t)m + o] + dv : 0.f;
            ((float*)a.F)[4 * (size_t)m + o] = val;
            ((float*)a.dF)[4 * (size_t)m + o] = val;
          }
        }
      }
    }
  }
}

// Features 3..9 of every point (0..2, the pass-0 slip, come from the interpolation
// kernel): previous-step force, unit normal r_k/R, and the gap to the nearest other
// surface (pair partners only) or wall plane, clamped to [0, zeta].
struct FeatArgs {
  int nmk, dim;
  int n[3];
  double zeta;
  const int* mown;
  const double* mr;
  const double *X, *D;
  const void* Fprev;
  int fp64;
  const int *part_all, *part_nall;  // all partners of each particle
  float* feat;
};

__global__ void k_features(FeatArgs a) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.nmk) return;
  int p = a.mown[k];
  double R = 0.5 * a.D[p];
  const double* r = a.mr + 4 * (size_t)k;
  double Xk[3] = {a.X[3 * p] + r[0], a.X[3 * p + 1] + r[1], a.dim == 3 ? a.X[3 * p + 2] + r[2] : 0.0};
  float* F = a.feat + 10 * (size_t)k;
  for (int c = 0; c < 3; c++) {
    F[3 + c] = a.fp64 ? float(((const double*)a.Fprev)[4 * (size_t)k + c])
                      : ((const float*)a.Fprev)[4 * (size_t)k + c];
    F[6 + c] = float(r[c] / R);
  }
  double gap = a.zeta;
  int cnt = a.part_nall[p];
  for (int s = 0; s < cnt; s++) {
    int o = a.part_all[p * PAIR_CAP + s];
    double d2 = 0.0;
    for (int c = 0; c < a.dim; c++) {
      double dx = Xk[c] - a.X[3 * o + c];
      d2 = d2 + dx * dx;
    }
    double g = sqrt(d2) - 0.5 * a.D[o];
    if (g < gap) gap = g;
  }
  for (int c = 0; c < a.dim; c++) {
    double lo = Xk[c] + 0.5, hi = (a.n[c] - 0.5) - Xk[c];
    if (lo < gap) gap = lo;
    if (hi < gap) gap = hi;
  }
  F[9] = float(gap < 0.0 ? 0.0 : gap);
}

// slip check after the correction pass: request the MDF fallback when the rms slip
// exceeds the tolerance
__global__ void k_slip_check(const double* slip2, int nmk, double tol, int* cond, int* nfall) {
  double s = sqrt(*slip2 / nmk);
  int fb = !(s <= tol);
  *cond = fb;
  if (fb) atomicAdd(nfall, 1);
}

__global__ void k_set_int(int* p, int v) { *p = v; }
__global__ void k_zero_d(double* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// training kernels (FP32)

// C[M x N] = op(A) op(B) (+ C if acc), row-major; op(A) is M x K, op(B) is K x N.
// tA: A stored K x M; tB: B stored N x K.  16x16 output tile per 256-thread block.
__global__ void k_gemm(const float* A, const float* B, float* Cm, int M, int N, int K, int tA, int tB,
                       int acc) {
  __shared__ float As[16][17], Bs[16][17];
  int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  float s = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (row < M && ka < K) ? (tA ? A[(size_t)ka * M + row] : A[(size_t)row * K + ka]) : 0.f;
    Bs[ty][tx] = (kb < K && col < N) ? (tB ? B[(size_t)col * K + kb] : B[(size_t)kb * N + col]) : 0.f;
    __syncthreads();
    for (int k = 0; k < 16; k++) s += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  if (row < M && col < N) Cm[(size_t)row * N + col] = acc ? Cm[(size_t)row * N + col] + s : s;
}

// Weight gradients C[M x N] = A^T B with A stored K x M and B stored K x N, K the batch:
// the K range is split over SPLITK blocks per 16x16 output tile (one tile per block would
// leave the chip idle on a 64 x 64 output), each block writing its partial tile; the
// partials are then added in split order, so the result does not depend on scheduling.
constexpr int SPLITK = 32;
__global__ void k_gemm_tn_split(const float* A, const float* B, float* part, int M, int N, int K) {
  __shared__ float As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16, z = blockIdx.z;
  const int per = (K + SPLITK - 1) / SPLITK, klo = z * per, khi = min(K, klo + per);
  float s = 0.f;
  for (int k0 = klo; k0 < khi; k0 += 16) {
    const int k = k0 + ty;  // one K row per thread row: coalesced along tx
    As[ty][tx] = (k < khi && m0 + tx < M) ? A[(size_t)k * M + m0 + tx] : 0.f;
    Bs[ty][tx] = (k < khi && n0 + tx < N) ? B[(size_t)k * N + n0 + tx] : 0.f;
    __syncthreads();
    for (int kk = 0; kk < 16; kk++) s += As[kk][ty] * Bs[kk][tx];
    __syncthreads();
  }
  const int row = m0 + ty, col = n0 + tx;
  if (row < M && col < N) part[((size_t)z * M + row) * N + col] = s;
}

__global__ void k_sum_splits(const float* part, float* C, int M, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  float s = 0.f;
  for (int z = 0; z < SPLITK; z++) s += part[(size_t)z * M * N + i];
  C[i] = s;
}

// Z[M x N] += bias[N]; H = tanh(Z) (act) or H = Z
__global__ void k_bias_act(float* Z, const float* bias, int M, int N, int act) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)M * N) return;
  float z = Z[i] + bias[i % N];
  Z[i] = act ? tanhf(z) : z;
}

// dY = 2 (Y - T) / (M N); per-block partial loss sums
__global__ void k_mse(const float* Y, const float* T, float* dY, int M, int N, float* loss_part) {
  __shared__ float red[256];
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float e = 0.f;
  if (i < (size_t)M * N) {
    e = Y[i] - T[i];
    dY[i] = 2.f * e / float((size_t)M * N);
  }
  red[threadIdx.x] = e * e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// dZ = dH * (1 - H^2)
__global__ void k_tanh_back(float* dH, const float* H, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dH[i] *= 1.f - H[i] * H[i];
}

// db[N] = column sums of dZ[M x N]
__global__ void k_colsum(const float* dZ, float* db, int M, int N) {
  __shared__ float red[256];
  int col = blockIdx.x;
  float s = 0.f;
  for (int r = threadIdx.x; r < M; r += blockDim.x) s += dZ[(size_t)r * N + col];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int t = blockDim.x / 2; t > 0; t >>= 1) {
    if ((int)threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[col] = red[0];
}

__global__ void k_adam(float* P, const float* G, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float g = G[i];
  float mi = b1 * m[i] + (1.f - b1) * g;
  float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// gather a batch of samples by index
__global__ void k_gather_rows(const float* src, const int* idx, float* dst, int rows, int cols) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)rows * cols) return;
  size_t r = i / cols, c = i % cols;
  dst[i] = src[(size_t)idx[r] * cols + c];
}

struct Net {
  float *P, *G;            // params, grads (NPARAM)
  float *Z1, *Z2, *Y, *dY; // activations (B x 64, B x 64, B x 3)
  float *dH1, *dH2;
  float* loss_part;
  float* part;  // SPLITK x 64 x 64 partial weight gradients
  int B;
};

void gemm(hipStream_t s, const float* A, const float* B, float* C, int M, int N, int K, int tA, int tB,
          int acc = 0) {
  dim3 grid((N + 15) / 16, (M + 15) / 16);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, A, B, C, M, N, K, tA, tB, acc);
}

// weight gradient C = A^T B over the batch (A: K x M, B: K x N; M, N <= 64)
void gemm_wgrad(hipStream_t s, const float* A, const float* B, float* C, int M, int N, int K,
                float* part) {
  dim3 grid((N + 15) / 16, (M + 15) / 16, SPLITK);
  hipLaunchKernelGGL(k_gemm_tn_split, grid, dim3(256), 0, s, A, B, part, M, N, K);
  hipLaunchKernelGGL(k_sum_splits, dim3((M * N + 255) / 256), dim3(256), 0, s, part, C, M, N);
}

// forward and backward of the MSE loss on a batch X (B x 10), T (B x 3); grads into n.G
void fwd_bwd(hipStream_t s, Net& n, const float* X, const float* T, int B) {
  float* P = n.P;
  float* G = n.G;
  auto blocks = [](size_t e) { return dim3((unsigned)((e + 255) / 256)); };
  // forward: Z1 = X W1^T + b1, H1 = tanh; Z2 = H1 W2^T + b2, H2 = tanh; Y = H2 W3^T + b3
  gemm(s, X, P + OFF_W1, n.Z1, B, NH, NI, 0, 1);
  hipLaunchKernelGGL(k_bias_act, blocks((size_t)B * NH), dim3(256), 0, s, n.Z1, P + OFF_B1, B, NH, 1);
  gemm(s, n.Z1, P + OFF_W2, n.Z2, B, NH, NH, 0, 1);
  hipLaunchKernelGGL(k_bias_act, blocks((size_t)B * NH), dim3(256), 0, s, n.Z2, P + OFF_B2, B, NH, 1);
  gemm(s, n.Z2, P + OFF_W3, n.Y, B, NO, NH, 0, 1);
  hipLaunchKernelGGL(k_bias_act, blocks((size_t)B * NO), dim3(256), 0, s, n.Y, P + OFF_B3, B, NO, 0);
  hipLaunchKernelGGL(k_mse, blocks((size_t)B * NO), dim3(256), 0, s, n.Y, T, n.dY, B, NO, n.loss_part);
  // backward
  gemm_wgrad(s, n.dY, n.Z2, G + OFF_W3, NO, NH, B, n.part);  // dW3 = dY^T H2
  hipLaunchKernelGGL(k_colsum, dim3(NO), dim3(256), 0, s, n.dY, G + OFF_B3, B, NO);
  gemm(s, n.dY, P + OFF_W3, n.dH2, B, NH, NO, 0, 0);  // dH2 = dY W3
  hipLaunchKernelGGL(k_tanh_back, blocks((size_t)B * NH), dim3(256), 0, s, n.dH2, n.Z2, (size_t)B * NH);
  gemm_wgrad(s, n.dH2, n.Z1, G + OFF_W2, NH, NH, B, n.part);  // dW2 = dZ2^T H1
  hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, n.dH2, G + OFF_B2, B, NH);
  gemm(s, n.dH2, P + OFF_W2, n.dH1, B, NH, NH, 0, 0);  // dH1 = dZ2 W2
  hipLaunchKernelGGL(k_tanh_back, blocks((size_t)B * NH), dim3(256), 0, s, n.dH1, n.Z1, (size_t)B * NH);
  gemm_wgrad(s, n.dH1, X, G + OFF_W1, NH, NI, B, n.part);  // dW1 = dZ1^T X
  hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, n.dH1, G + OFF_B1, B, NH);
}

struct DevBuf {
  std::vector<void*> ptrs;
  template <class T>
  T* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T) + 16) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (T*)p;
  }
  ~DevBuf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

Net make_net(DevBuf& db, int B) {
  Net n;
  n.B = B;
  n.P = db.get<float>(NPARAM);
  n.G = db.get<float>(NPARAM);
  n.Z1 = db.get<float>((size_t)B * NH);
  n.Z2 = db.get<float>((size_t)B * NH);
  n.Y = db.get<float>((size_t)B * NO);
  n.dY = db.get<float>((size_t)B * NO);
  n.dH1 = db.get<float>((size_t)B * NH);
  n.dH2 = db.get<float>((size_t)B * NH);
  n.loss_part = db.get<float>(((size_t)B * NO + 255) / 256);
  n.part = db.get<float>((size_t)SPLITK * NH * NH);
  return n;
}

float read_loss(hipStream_t s, const Net& n, int B) {
  int parts = (B * NO + 255) / 256;
  std::vector<float> h(parts);
  (void)hipMemcpyAsync(h.data(), n.loss_part, parts * 4, hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  double t = 0;
  for (float v : h) t += v;
  return float(t / (double(B) * NO));
}

void run_infer(iblbm_ctx* c, float* y_out) {
  InferArgs a;
  a.P = (const float*)c->mlp_w;
  a.norm = c->mlp_norm;
  a.feat = c->feat;
  a.n = c->nmk;
  a.dim = c->dim;
  a.F = c->mF;
  a.dF = c->mdF;
  a.Fprev = c->mFprev;
  a.fp64 = c->fp64;
  a.y = y_out;
  // three waves per SIMD fit the kernel's registers: 256 CUs x 4 SIMDs x 3
  int waves = std::min((c->nmk + 15) / 16, INFER_WAVES);
  hipLaunchKernelGGL(k_mlp_infer, dim3((waves + 3) / 4), dim3(256), 0, c->stream, a);
}

void run_features(iblbm_ctx* c) {
  FeatArgs a;
  a.nmk = c->nmk;
  a.dim = c->dim;
  for (int d = 0; d < 3; d++) a.n[d] = c->cfg.n[d];
  a.zeta = c->cfg.zeta;
  a.mown = c->mown;
  a.mr = c->mr;
  a.X = c->X;
  a.D = c->D;
  a.Fprev = c->mFprev;
  a.fp64 = c->fp64;
  a.part_all = c->pair_all;
  a.part_nall = c->pair_nall;
  a.feat = c->feat;
  hipLaunchKernelGGL(k_features, dim3((c->nmk + 255) / 256), dim3(256), 0, c->stream, a);
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free gradient entry point: the activations
// Z1, Z2 (tanh outputs), dH1, dH2 (n x 64 each), Y, dY (n x 3) and the per-block partial
// losses of up to NOALLOC_MAX samples, and the split partial weight gradients, 9.1 MB.
// Each device holds its own copy for the
// life of the process.  In host code `scratch` is only a stand-in symbol: its device
// address comes from hipGetSymbolAddress, once per device, and only that address is
// handed to kernels.
constexpr int NOALLOC_MAX = 8192;
constexpr size_t NOALLOC_PARTS = ((size_t)NOALLOC_MAX * NO + 255) / 256;
constexpr size_t NOALLOC_FLOATS = 4 * (size_t)NOALLOC_MAX * NH + 2 * (size_t)NOALLOC_MAX * NO +
                                  ((NOALLOC_PARTS + 63) & ~(size_t)63) + (size_t)SPLITK * NH * NH;
__device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_ptr[MAX_DEVICES] = {nullptr};

// device address of this device's scratch (looked up on the first call on the device)
hipError_t scratch_of_device(int dev, float** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = (float*)p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

// mean squared error from the per-block partial sums, summed in block order in FP64 as
// the host does for iblbm_nn_grad
__global__ void k_loss_total(const float* part, int parts, double count, float* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0;
  for (int i = 0; i < parts; i++) t += part[i];
  *loss = float(t / count);
}

}  // namespace

// Learned forcing stage of one step (after the cells/pairs and the band request):
// features, MLP prediction, its spreading, one plain correction pass, the slip check and,
// when the slip exceeds the tolerance, a full MDF redo with fallback_iters passes whose
// kernels run only when the device flag is set.
#define HIP_STEP(expr) hip_check(c, (expr), #expr)

// The MDF fallback of the learned step: u* and the band force recomputed, then
// fallback_iters plain passes.
void mlp_fallback(iblbm_ctx* c) {
  ibm_band_redo(c);  // the redo recomputes u* and clears the force at the band
  for (int m = 0; m < c->cfg.fallback_iters; m++) {
    ibm_interp(c, m == 0, 0);
    ibm_spread(c, 0);
  }
}

void mlp_step_forcing(iblbm_ctx* c) {
  tbegin(c, IBLBM_T_INTERP);
  ibm_interp(c, 1, 2);  // pass-0 slip into the features (also builds u* and the band)
  tend(c);
  tbegin(c, IBLBM_T_MLP);
  run_features(c);
  run_infer(c, nullptr);
  tend(c);
  tbegin(c, IBLBM_T_SPREAD);
  ibm_spread(c, 1);
  tend(c);
  // the correction pass; its interpolation also measures the slip the prediction left,
  // which judges the prediction
  tbegin(c, IBLBM_T_OTHER);
  hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, c->stream, c->dstats, 1);
  tend(c);
  tbegin(c, IBLBM_T_INTERP);
  ibm_interp(c, 0, 3);
  tend(c);
  tbegin(c, IBLBM_T_OTHER);
  hipLaunchKernelGGL(k_slip_check, dim3(1), dim3(1), 0, c->stream, c->dstats, c->nmk,
                     c->cfg.slip_tol, c->dcond, c->dstatus + 4);
  // outside a graph the verdict goes to the host, which reads it while the correction's
  // spreading runs and launches the fallback only when it is needed (launching its
  // workgroups every step only to have them return costs a third of a millisecond at
  // 256^3); inside a graph the decision stays on the device
  const bool host_decides = !c->capturing && c->hflag;
  if (host_decides) {
    HIP_STEP(hipMemcpyAsync(c->hflag, c->dcond, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_STEP(hipEventRecord(c->ev_flag, c->stream));
  }
  tend(c);
  tbegin(c, IBLBM_T_SPREAD);
  ibm_spread(c, 0);
  tend(c);
  if (host_decides) {
    HIP_STEP(hipEventSynchronize(c->ev_flag));
    if (*c->hflag) {
      tbegin(c, IBLBM_T_OTHER);
      mlp_fallback(c);
      tend(c);
    }
  } else {
    tbegin(c, IBLBM_T_OTHER);
    c->cond = c->dcond;
    mlp_fallback(c);
    c->cond = nullptr;
    tend(c);
  }
}

void mlp_features(iblbm_ctx* c) { run_features(c); }
void mlp_infer(iblbm_ctx* c) { run_infer(c, nullptr); }

extern "C" {

iblbm_status iblbm_set_mlp(iblbm_ctx* c, const float* params, const float* norm) {
  if (!c || !params || !norm) return IBLBM_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return IBLBM_E_DEVICE;
  if (!c->mlp_w) {
    // through the context's allocator, released with the context
    c->mlp_w = ctx_alloc(c, NPARAM * sizeof(float));
    c->mlp_norm = c->mlp_w ? (float*)ctx_alloc(c, 32 * sizeof(float)) : nullptr;
    if (!c->mlp_w || !c->mlp_norm) {
      c->mlp_w = nullptr;
      return IBLBM_E_NOMEM;
    }
  }
  if (!c->hflag) {
    if (hipHostMalloc((void**)&c->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
      c->hflag = nullptr;
      return IBLBM_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&c->ev_flag, hipEventDisableTiming) != hipSuccess) {
      c->ev_flag = nullptr;
      return IBLBM_E_DEVICE;
    }
  }
  if (hipMemcpyAsync(c->mlp_w, params, NPARAM * sizeof(float), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(c->mlp_norm, norm, 26 * sizeof(float), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    c->err = "copying the MLP parameters failed";
    return IBLBM_E_DEVICE;
  }
  c->has_mlp = true;
  c->graph_dirty = true;
  return IBLBM_OK;
}

iblbm_status iblbm_capture_samples(iblbm_ctx* c, float* feat, float* target) {
  if (!c || c->nmk == 0) return IBLBM_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return IBLBM_E_DEVICE;
  // a dry run of the next step's forcing stage; the PDFs and particles are unchanged
  c->fbuf = (int)(c->step & 1);
  part_cells_pairs(c);
  ibm_band(c);
  ibm_interp(c, 1, 2);
  run_features(c);
  ibm_band_redo(c);
  for (int m = 0; m < c->cfg.mdf_iters; m++) {
    ibm_interp(c, m == 0, 0);
    ibm_spread(c, 0);
  }
  std::vector<char> mf((size_t)c->nmk * 4 * (c->fp64 ? 8 : 4));
  bool ok = hipMemcpyAsync(feat, c->feat, (size_t)c->nmk * 10 * 4, hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
            hipMemcpyAsync(mf.data(), c->mF, mf.size(), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
            hipStreamSynchronize(c->stream) == hipSuccess;
  // the cells were filled for the dry run; the next step refills them
  part_zero_cells(c);
  if (!ok) return IBLBM_E_DEVICE;
  for (int k = 0; k < c->nmk; k++)
    for (int o = 0; o < 3; o++)
      target[3 * k + o] = c->fp64 ? float(((double*)mf.data())[4 * k + o]) : ((float*)mf.data())[4 * k + o];
  return IBLBM_OK;
}

iblbm_status iblbm_nn_forward(const float* x, int64_t n, const float* params, float* y) {
  if (!x || !params || !y || n <= 0) return IBLBM_E_ARG;
  DevBuf db;
  float* dP = db.get<float>(NPARAM);
  float* dX = db.get<float>((size_t)n * NI);
  float* dY = db.get<float>((size_t)n * NO);
  float* dN = db.get<float>(32);
  if (!dP || !dX || !dY || !dN) return IBLBM_E_NOMEM;
  // inputs are already normalised: identity normalisation
  float norm[26];
  for (int i = 0; i < NI; i++) {
    norm[i] = 0.f;
    norm[NI + i] = 1.f;
  }
  for (int o = 0; o < NO; o++) {
    norm[2 * NI + o] = 0.f;
    norm[2 * NI + NO + o] = 1.f;
  }
  if (hipMemcpy(dP, params, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dX, x, (size_t)n * NI * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dN, norm, sizeof(norm), hipMemcpyHostToDevice) != hipSuccess)
    return IBLBM_E_DEVICE;
  InferArgs a;
  a.P = dP;
  a.norm = dN;
  a.feat = dX;
  a.n = (int)n;
  a.dim = 3;
  a.F = nullptr;
  a.dF = nullptr;
  a.Fprev = nullptr;
  a.fp64 = 0;
  a.y = dY;
  int waves = (int)std::min<int64_t>((n + 15) / 16, INFER_WAVES);
  hipLaunchKernelGGL(k_mlp_infer, dim3((waves + 3) / 4), dim3(256), 0, 0, a);
  if (hipMemcpy(y, dY, (size_t)n * NO * 4, hipMemcpyDeviceToHost) != hipSuccess) return IBLBM_E_DEVICE;
  return IBLBM_OK;
}

iblbm_status iblbm_nn_grad(const float* x, const float* t, int64_t n, const float* params,
                           float* loss, float* grad) {
  if (!x || !t || !params || n <= 0 || n > (1 << 24)) return IBLBM_E_ARG;
  DevBuf db;
  Net net = make_net(db, (int)n);
  float* dX = db.get<float>((size_t)n * NI);
  float* dT = db.get<float>((size_t)n * NO);
  if (!net.P || !dX || !dT) return IBLBM_E_NOMEM;
  hipStream_t s = 0;
  if (hipMemcpy(net.P, params, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dX, x, (size_t)n * NI * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dT, t, (size_t)n * NO * 4, hipMemcpyHostToDevice) != hipSuccess)
    return IBLBM_E_DEVICE;
  fwd_bwd(s, net, dX, dT, (int)n);
  if (loss) *loss = read_loss(s, net, (int)n);
  if (grad && hipMemcpy(grad, net.G, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return IBLBM_E_DEVICE;
  return IBLBM_OK;
}

iblbm_status iblbm_nn_grad_noalloc(const float* x, const float* t, int64_t n, const float* params,
                                   float* loss, float* grad, void* stream) {
  if (!x || !t || !params || !loss || !grad || n <= 0) return IBLBM_E_ARG;
  if (n > NOALLOC_MAX) return IBLBM_E_CAPACITY;
  int dev = 0;
  float* base = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || scratch_of_device(dev, &base) != hipSuccess)
    return IBLBM_E_DEVICE;
  const int B = (int)n;
  Net net;
  net.B = B;
  net.P = const_cast<float*>(params);  // read only: fwd_bwd writes gradients to net.G
  net.G = grad;
  float* q = base;
  net.Z1 = q;
  q += (size_t)B * NH;
  net.Z2 = q;
  q += (size_t)B * NH;
  net.dH1 = q;
  q += (size_t)B * NH;
  net.dH2 = q;
  q += (size_t)B * NH;
  net.Y = q;
  q += (size_t)B * NO;
  net.dY = q;
  q += (size_t)B * NO;
  net.loss_part = q;
  q += (NOALLOC_PARTS + 63) & ~(size_t)63;
  net.part = q;
  hipStream_t s = (hipStream_t)stream;
  fwd_bwd(s, net, x, t, B);
  const int parts = (B * NO + 255) / 256;
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, net.loss_part, parts, double(B) * NO, loss);
  if (hipGetLastError() != hipSuccess) return IBLBM_E_DEVICE;
  return IBLBM_OK;
}

iblbm_status iblbm_nn_train(const float* x, const float* t, int64_t n, float* params,
                            const iblbm_train_opts* o, float* curve) {
  if (!x || !t || !params || !o || n <= 0 || o->epochs < 0 || o->batch <= 0) return IBLBM_E_ARG;
  int B = (int)std::min<int64_t>(o->batch, n);
  DevBuf db;
  Net net = make_net(db, B);
  float* dXall = db.get<float>((size_t)n * NI);
  float* dTall = db.get<float>((size_t)n * NO);
  float* dX = db.get<float>((size_t)B * NI);
  float* dT = db.get<float>((size_t)B * NO);
  float* m = db.get<float>(NPARAM);
  float* v = db.get<float>(NPARAM);
  int* dIdx = db.get<int>((size_t)n);
  if (!net.P || !dXall || !dTall || !dX || !dT || !m || !v || !dIdx) return IBLBM_E_NOMEM;
  hipStream_t s = 0;
  if (hipMemcpy(net.P, params, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dXall, x, (size_t)n * NI * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dTall, t, (size_t)n * NO * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m, 0, NPARAM * 4) != hipSuccess || hipMemset(v, 0, NPARAM * 4) != hipSuccess)
    return IBLBM_E_DEVICE;
  // a seeded SplitMix64 shuffle of the sample order each epoch (host, indices only)
  std::vector<int> idx(n);
  for (int64_t i = 0; i < n; i++) idx[i] = (int)i;
  uint64_t st = o->seed;
  auto next = [&st]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  int stepn = 0;
  for (int e = 0; e < o->epochs; e++) {
    for (int64_t i = n - 1; i > 0; i--) std::swap(idx[i], idx[next() % (uint64_t)(i + 1)]);
    if (hipMemcpy(dIdx, idx.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) return IBLBM_E_DEVICE;
    double esum = 0;
    int nb = 0, nread = 0;
    for (int64_t b0 = 0; b0 + B <= n; b0 += B) {
      hipLaunchKernelGGL(k_gather_rows, dim3((B * NI + 255) / 256), dim3(256), 0, s, dXall, dIdx + b0, dX, B, NI);
      hipLaunchKernelGGL(k_gather_rows, dim3((B * NO + 255) / 256), dim3(256), 0, s, dTall, dIdx + b0, dT, B, NO);
      fwd_bwd(s, net, dX, dT, B);
      stepn++;
      float c1 = 1.f - powf(o->beta1, (float)stepn), c2 = 1.f - powf(o->beta2, (float)stepn);
      hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, net.P, net.G, m, v, NPARAM,
                         o->lr, o->beta1, o->beta2, o->eps, c1, c2);
      if (nb % 16 == 0) {
        esum += read_loss(s, net, B);
        nread++;
      }
      nb++;
    }
    if (curve) curve[e] = float(esum / std::max(1, nread));
  }
  if (hipMemcpy(params, net.P, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) return IBLBM_E_DEVICE;
  return IBLBM_OK;
}

}  // extern "C"

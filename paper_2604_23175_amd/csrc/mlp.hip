// Learned warm start (an extension of the paper's method): a per-area MLP
// maps the area's measurements, normalised by sigma, to a starting (|V|,
// theta) for its own buses.  Weights are bfloat16 copies of FP32 master
// weights; every product runs on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation; biases, pre-activations, the loss and all gradients stay FP32;
// Adam updates the FP32 masters.  A prediction is used only if its objective
// J(x_pred) is not worse than J(flat start) (Eq. 2), snapshot by snapshot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"

using namespace mase;

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

enum { EPI_STORE = 0, EPI_LIN = 1, EPI_RELU = 2, EPI_MASK = 3 };

// float -> bfloat16 bits, round to nearest even
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GemmDesc {
  const uint16_t* A;  // A(i, k) = A[i * sar + k * sac]  (bfloat16 bits)
  long long sar, sac;
  const uint16_t* B;  // B(k, j) = B[k * sbr + j * sbc]
  long long sbr, sbc;
  float* C;           // [M x ldc] float32 output
  uint16_t* Cb;       // [M x ldc] bfloat16 output (EPI_RELU, EPI_MASK)
  const float* bias;  // [N] (EPI_LIN, EPI_RELU)
  const float* mask;  // [M x ldc] pre-activation, relu' = (mask > 0) (EPI_MASK)
  int M, N, K, ldc;
};

// ---------------------------------------------------------------------------
// Grouped GEMM C = A B over many small problems (one per area) in one launch.
// A workgroup computes a 64x64 tile of one group: four waves, each 32x32 as
// 2x2 MFMA tiles of 16x16, K in steps of 32 staged through LDS (A as
// [row][k], B transposed to [col][k], so each lane's 8 operands are one
// 16-byte LDS read).  v_mfma_f32_16x16x32_bf16 lane layout on gfx950: lane l
// holds A[l%16][8(l/16) + j] and B[8(l/16) + j][l%16], j < 8, and
// accumulator element q is D[4(l/16) + q][l%16].
// ---------------------------------------------------------------------------
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc* gd, const int4* tiles) {
  const int4 tm = tiles[blockIdx.x];
  const GemmDesc g = gd[tm.x];
  constexpr int P = 40;  // LDS row pitch in bfloat16 (80 bytes: rows stay 16-byte aligned)
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * P];
  __shared__ __attribute__((aligned(16))) uint16_t Bt[64 * P];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  f4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    for (int e = 0; e < 8; ++e) {
      const int L = tid + 256 * e;
      int r, kk;
      if (g.sac == 1) { r = L >> 5; kk = L & 31; } else { r = L & 63; kk = L >> 6; }
      const int i = tm.y + r, k = k0 + kk;
      As[r * P + kk] = (i < g.M && k < g.K) ? g.A[(long long)i * g.sar + (long long)k * g.sac] : (uint16_t)0;
    }
    for (int e = 0; e < 8; ++e) {
      const int L = tid + 256 * e;
      int c, kk;
      if (g.sbc == 1) { c = L & 63; kk = L >> 6; } else { c = L >> 5; kk = L & 31; }
      const int j = tm.z + c, k = k0 + kk;
      Bt[c * P + kk] = (j < g.N && k < g.K) ? g.B[(long long)k * g.sbr + (long long)j * g.sbc] : (uint16_t)0;
    }
    __syncthreads();
    const int kb = 8 * (lane >> 4);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      const b8 av = *reinterpret_cast<const b8*>(&As[(wm * 32 + ti * 16 + (lane & 15)) * P + kb]);
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        const b8 bv = *reinterpret_cast<const b8*>(&Bt[(wn * 32 + tj * 16 + (lane & 15)) * P + kb]);
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ti][tj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = tm.y + wm * 32 + ti * 16 + 4 * (lane >> 4) + q;
        const int j = tm.z + wn * 32 + tj * 16 + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        const long long o = (long long)i * g.ldc + j;
        const float v = acc[ti][tj][q];
        if (EPI == EPI_STORE) {
          g.C[o] = v;
        } else if (EPI == EPI_LIN) {
          g.C[o] = v + g.bias[j];
        } else if (EPI == EPI_RELU) {
          const float p = v + g.bias[j];
          g.C[o] = p;
          g.Cb[o] = to_bf16(p > 0.f ? p : 0.f);
        } else {
          const float gg = g.mask[o] > 0.f ? v : 0.f;
          g.C[o] = gg;
          g.Cb[o] = to_bf16(gg);
        }
      }
}

// X_k[b][i] = bf16((z[b][meas] - mu[meas]) / sigma[meas]) for every input.
__global__ void k_mlp_gather(const double* z, int n_meas, int B, const double* mu, const double* sigma,
                             const int* in_area, const int* in_idx, const int* in_meas,
                             const long long* xoff, const int* mk, uint16_t* X) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * n_meas) return;
  const int b = (int)(t / n_meas), r = (int)(t - (long long)b * n_meas);
  const int k = in_area[r], m = in_meas[r];
  const double x = (z[(long long)b * n_meas + m] - mu[m]) / sigma[m];
  X[xoff[k] + (long long)b * mk[k] + in_idx[r]] = to_bf16((float)x);
}

// T_k[b][j] = (x_target - mean) / std as float32 (variable id: even = theta,
// odd = |V|).
__global__ void k_mlp_target(const double* vm, const double* va, int n_bus, int B, int n_out,
                             const double* ym, const double* ys, const int* out_area, const int* out_idx,
                             const int* out_var, const long long* yoff, const int* ok, float* T) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * n_out) return;
  const int b = (int)(t / n_out), o = (int)(t - (long long)b * n_out);
  const int var = out_var[o], bus = var >> 1;
  const double x = (var & 1) ? vm[(long long)b * n_bus + bus] : va[(long long)b * n_bus + bus];
  T[yoff[out_area[o]] + (long long)b * ok[out_area[o]] + out_idx[o]] = (float)((x - ym[var]) / ys[var]);
}

// dY = 2 (Y - T) / (B n_out); per-workgroup partial sums of (Y - T)^2.
__global__ void __launch_bounds__(256) k_mlp_dy(const float* Y, const float* T, int B, int n_out,
                                                const int* out_area, const int* out_idx,
                                                const long long* yoff, const int* ok, float* G,
                                                uint16_t* Gb, double* lossp) {
  __shared__ double red[4];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (t < (long long)B * n_out) {
    const int b = (int)(t / n_out), o = (int)(t - (long long)b * n_out);
    const long long p = yoff[out_area[o]] + (long long)b * ok[out_area[o]] + out_idx[o];
    const float e = Y[p] - T[p];
    const float g = 2.0f * e / (float)((double)B * n_out);
    G[p] = g;
    Gb[p] = to_bf16(g);
    e2 = (double)e * (double)e;
  }
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_down(e2, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Bias gradients: column sums (over the batch) of per-area float32 matrices.
__global__ void k_mlp_colsum(const float* G, int B, int ncol, const int* col_area, const int* col_idx,
                             const long long* goff, const int* gw, const long long* boff, float* grad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int k = col_area[c], j = col_idx[c];
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += G[goff[k] + (long long)b * gw[k] + j];
  grad[boff[k] + j] = s;
}

// Adam (Kingma and Ba, 2015) on the FP32 masters; refreshes the bf16 copies.
__global__ void k_adam(float* theta, const float* g, float* m, float* v, uint16_t* tb, long long n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  theta[i] = th;
  tb[i] = to_bf16(th);
}

// Normalisation statistics of a training set.  Per column of X [n][ncol]
// (one thread per column, rows in order, so the sums are deterministic): the
// mean, and with sd the sample standard deviation (denominator n - 1)
// replaced by 1 where it is at most 1e-6 (a variable that does not vary).
// Results go to mean[col * ostride + ooff] (and sd likewise).
__global__ void k_col_stats(const double* X, long long n, int ncol, double* mean, double* sd, int ostride,
                            int ooff) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double acc = 0.0;
  for (long long r = 0; r < n; ++r) acc += X[r * ncol + col];
  const double mu = acc / (double)n;
  mean[(long long)col * ostride + ooff] = mu;
  if (sd) {
    double q = 0.0;
    for (long long r = 0; r < n; ++r) {
      const double e = X[r * ncol + col] - mu;
      q += e * e;
    }
    const double v = n > 1 ? sqrt(q / (double)(n - 1)) : 0.0;
    sd[(long long)col * ostride + ooff] = v > 1e-6 ? v : 1.0;
  }
}

// Mean over the n rows of ((z - mu) / sigma)^2 per measurement.
__global__ void k_norm_ms(const double* z, long long n, int n_meas, const double* mu, const double* sigma,
                          double* ms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_meas) return;
  double acc = 0.0;
  for (long long r = 0; r < n; ++r) {
    const double e = (z[r * n_meas + i] - mu[i]) / sigma[i];
    acc += e * e;
  }
  ms[i] = acc / (double)n;
}

// Per area (one workgroup each): RMS of the normalised inputs, sqrt of the
// mean of ms over the area's input measurements (fixed-order reduction).
__global__ void __launch_bounds__(256) k_area_rms(const double* ms, const int* in_meas, const int* mk, double* rms) {
  __shared__ double red[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  int off = 0;
  for (int j = 0; j < k; ++j) off += mk[j];
  const int m = mk[k];
  double acc = 0.0;
  for (int i = tid; i < m; i += 256) acc += ms[in_meas[off + i]];
  red[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) rms[k] = m > 0 ? sqrt(red[0] / (double)m) : 0.0;
}

__global__ void k_to_bf16(const float* a, uint16_t* b, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = to_bf16(a[i]);
}

// Predicted state x = y * std + mean for every output (variable id: even =
// theta, odd = |V|); the slack angle is 0.
__global__ void k_mlp_compose(const float* Y, int B, int n_out, int n_bus, int slack, const double* ym,
                              const double* ys, const int* out_area, const int* out_idx,
                              const int* out_var, const long long* yoff, const int* ok, double* vm,
                              double* va, double2* x) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * n_out) return;
  const int b = (int)(t / n_out), o = (int)(t - (long long)b * n_out);
  const int var = out_var[o], bus = var >> 1;
  double val = (double)Y[yoff[out_area[o]] + (long long)b * ok[out_area[o]] + out_idx[o]] * ys[var] + ym[var];
  if (!(var & 1) && bus == slack) val = 0.0;
  const long long q = (long long)b * n_bus + bus;
  if (x) {
    if (var & 1) x[q].y = val;
    else x[q].x = val;
  } else {
    if (var & 1) vm[q] = val;
    else va[q] = val;
  }
}

// Per snapshot: keep the prediction iff J(pred) <= J(flat) (sums over areas
// in area order), then copy the chosen state.
__global__ void __launch_bounds__(256) k_choose(const double* jp, const double* jf, int n_area, int n_bus,
                                                double j_cap, const double2* xp, const double2* xf,
                                                double2* x, int* accepted) {
  const int s = blockIdx.x;
  __shared__ int acc;
  if (threadIdx.x == 0) {
    double a = 0.0, f = 0.0;
    for (int k = 0; k < n_area; ++k) {
      a += jp[(long long)s * n_area + k];
      f += jf[(long long)s * n_area + k];
    }
    acc = (a <= f && a <= j_cap) ? 1 : 0;  // false for NaN
    accepted[s] = acc;
  }
  __syncthreads();
  const double2* src = acc ? xp : xf;
  for (int i = threadIdx.x; i < n_bus; i += blockDim.x) x[(long long)s * n_bus + i] = src[(long long)s * n_bus + i];
}

int fail(int code, const std::string& msg) { return set_error(code, msg); }

#define HIPTRY(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(MASE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

enum Op { FWD1, FWD2, FWD3, BWD2, BWD1, DW3, DW2, DW1, N_OP };

}  // namespace

struct mase_mlp {
  mase_ctx* ctx = nullptr;
  int K = 0, H = 0, Bmax = 0, n_meas = 0, n_bus = 0, n_out = 0;
  long long nparam = 0;
  std::vector<int> mk, ok;
  std::vector<long long> poff, xoff, hoff, yoff;
  std::vector<std::vector<int>> in_meas, out_var;
  // device
  std::vector<void*> allocs;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* thb = nullptr;
  uint16_t *X = nullptr, *H1b = nullptr, *H2b = nullptr, *G3b = nullptr, *G2b = nullptr, *G1b = nullptr;
  float *P1 = nullptr, *P2 = nullptr, *Y = nullptr, *T = nullptr, *G3 = nullptr, *G2 = nullptr, *G1 = nullptr;
  double *zmean = nullptr, *ymean = nullptr, *ystd = nullptr, *sigma = nullptr, *lossp = nullptr;
  double *zms = nullptr, *area_rms = nullptr;  // input statistics (mase_mlp_fit_norm)
  int *d_in_area = nullptr, *d_in_idx = nullptr, *d_in_meas = nullptr;
  int *d_out_area = nullptr, *d_out_idx = nullptr, *d_out_var = nullptr, *d_mk = nullptr, *d_ok = nullptr;
  long long *d_xoff = nullptr, *d_hoff = nullptr, *d_yoff = nullptr, *d_poff_b1 = nullptr,
            *d_poff_b2 = nullptr, *d_poff_b3 = nullptr;
  int *d_hcol_area = nullptr, *d_hcol_idx = nullptr, *d_ocol_area = nullptr, *d_ocol_idx = nullptr;
  int *d_H = nullptr;
  double2 *xpred = nullptr, *xflat = nullptr;
  double *jpred = nullptr, *jflat = nullptr;
  int* d_accepted = nullptr;
  int step = 0;
  int last_ws = 0;  // snapshots of the last warm start (0: none yet)
  double j_cap = INFINITY;
  bool have_norm = false;
  std::map<std::pair<int, int>, std::pair<std::pair<GemmDesc*, int4*>, int>> gcache;
};

namespace {

template <class T>
int mdalloc(mase_mlp* m, size_t n, T** out) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(1, n) * sizeof(T));
  if (e != hipSuccess) return fail(MASE_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  m->allocs.push_back(p);
  *out = static_cast<T*>(p);
  return 0;
}

template <class T>
int mupload(mase_mlp* m, const std::vector<T>& v, T** out) {
  int rc = mdalloc(m, v.size(), out);
  if (rc) return rc;
  if (!v.empty()) HIPTRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

// Descriptors and tiles of one grouped GEMM (cached per op and batch size).
int gemm(mase_mlp* m, int op, int B) {
  const auto key = std::make_pair(op, B);
  auto it = m->gcache.find(key);
  if (it == m->gcache.end()) {
    std::vector<GemmDesc> gd(m->K);
    std::vector<int4> tiles;
    const int H = m->H;
    for (int k = 0; k < m->K; ++k) {
      const long long po = m->poff[k];
      const int mk = m->mk[k], ok = m->ok[k];
      const uint16_t* W1 = m->thb + po;
      const uint16_t* W2 = W1 + (long long)mk * H + H;
      const uint16_t* W3 = W2 + (long long)H * H + H;
      const float* b1 = m->theta + po + (long long)mk * H;
      const float* b2 = b1 + H + (long long)H * H;
      const float* b3 = b2 + H + (long long)H * ok;
      float* gW1 = m->grad + po;
      float* gW2 = gW1 + (long long)mk * H + H;
      float* gW3 = gW2 + (long long)H * H + H;
      const long long xo = m->xoff[k], ho = m->hoff[k], yo = m->yoff[k];
      GemmDesc g{};
      switch (op) {
        case FWD1:  // P1 = X W1 + b1, H1 = relu
          g = GemmDesc{m->X + xo, mk, 1, W1, H, 1, m->P1 + ho, m->H1b + ho, b1, nullptr, B, H, mk, H};
          break;
        case FWD2:
          g = GemmDesc{m->H1b + ho, H, 1, W2, H, 1, m->P2 + ho, m->H2b + ho, b2, nullptr, B, H, H, H};
          break;
        case FWD3:
          g = GemmDesc{m->H2b + ho, H, 1, W3, ok, 1, m->Y + yo, nullptr, b3, nullptr, B, ok, H, ok};
          break;
        case BWD2:  // dH2 = (dY W3^T) * relu'(P2)
          g = GemmDesc{m->G3b + yo, ok, 1, W3, 1, ok, m->G2 + ho, m->G2b + ho, nullptr, m->P2 + ho, B, H, ok, H};
          break;
        case BWD1:  // dH1 = (dH2 W2^T) * relu'(P1)
          g = GemmDesc{m->G2b + ho, H, 1, W2, 1, H, m->G1 + ho, m->G1b + ho, nullptr, m->P1 + ho, B, H, H, H};
          break;
        case DW3:  // dW3 = H2^T dY
          g = GemmDesc{m->H2b + ho, 1, H, m->G3b + yo, ok, 1, gW3, nullptr, nullptr, nullptr, H, ok, B, ok};
          break;
        case DW2:
          g = GemmDesc{m->H1b + ho, 1, H, m->G2b + ho, H, 1, gW2, nullptr, nullptr, nullptr, H, H, B, H};
          break;
        case DW1:
          g = GemmDesc{m->X + xo, 1, mk, m->G1b + ho, H, 1, gW1, nullptr, nullptr, nullptr, mk, H, B, H};
          break;
      }
      gd[k] = g;
      for (int i = 0; i < g.M; i += 64)
        for (int j = 0; j < g.N; j += 64) tiles.push_back(int4{k, i, j, 0});
    }
    GemmDesc* dg = nullptr;
    int4* dt = nullptr;
    int rc = mupload(m, gd, &dg);
    if (rc) return rc;
    if ((rc = mupload(m, tiles, &dt))) return rc;
    it = m->gcache.emplace(key, std::make_pair(std::make_pair(dg, dt), (int)tiles.size())).first;
  }
  GemmDesc* dg = it->second.first.first;
  int4* dt = it->second.first.second;
  const int nt = it->second.second;
  hipStream_t st = m->ctx->stream;
  switch (op) {
    case FWD1: case FWD2: hipLaunchKernelGGL(k_gemm<EPI_RELU>, dim3(nt), dim3(256), 0, st, dg, dt); break;
    case FWD3: hipLaunchKernelGGL(k_gemm<EPI_LIN>, dim3(nt), dim3(256), 0, st, dg, dt); break;
    case BWD2: case BWD1: hipLaunchKernelGGL(k_gemm<EPI_MASK>, dim3(nt), dim3(256), 0, st, dg, dt); break;
    default: hipLaunchKernelGGL(k_gemm<EPI_STORE>, dim3(nt), dim3(256), 0, st, dg, dt); break;
  }
  HIPTRY(hipGetLastError());
  return 0;
}

unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int forward(mase_mlp* m, const double* z, int B) {
  hipStream_t st = m->ctx->stream;
  hipLaunchKernelGGL(k_mlp_gather, dim3(nblk((long long)B * m->n_meas)), dim3(256), 0, st, z, m->n_meas, B,
                     m->zmean, m->sigma, m->d_in_area, m->d_in_idx, m->d_in_meas, m->d_xoff, m->d_mk, m->X);
  HIPTRY(hipGetLastError());
  int rc;
  if ((rc = gemm(m, FWD1, B))) return rc;
  if ((rc = gemm(m, FWD2, B))) return rc;
  return gemm(m, FWD3, B);
}

int backward(mase_mlp* m, const double* vm, const double* va, int B, double* loss) {
  hipStream_t st = m->ctx->stream;
  const long long nout = (long long)B * m->n_out;
  hipLaunchKernelGGL(k_mlp_target, dim3(nblk(nout)), dim3(256), 0, st, vm, va, m->n_bus, B, m->n_out,
                     m->ymean, m->ystd, m->d_out_area, m->d_out_idx, m->d_out_var, m->d_yoff, m->d_ok, m->T);
  HIPTRY(hipGetLastError());
  const unsigned nb = nblk(nout);
  hipLaunchKernelGGL(k_mlp_dy, dim3(nb), dim3(256), 0, st, m->Y, m->T, B, m->n_out, m->d_out_area,
                     m->d_out_idx, m->d_yoff, m->d_ok, m->G3, m->G3b, m->lossp);
  HIPTRY(hipGetLastError());
  int rc;
  if ((rc = gemm(m, DW3, B))) return rc;
  if ((rc = gemm(m, BWD2, B))) return rc;
  if ((rc = gemm(m, DW2, B))) return rc;
  if ((rc = gemm(m, BWD1, B))) return rc;
  if ((rc = gemm(m, DW1, B))) return rc;
  const int hcols = m->K * m->H;
  hipLaunchKernelGGL(k_mlp_colsum, dim3(nblk(hcols)), dim3(256), 0, st, m->G1, B, hcols, m->d_hcol_area,
                     m->d_hcol_idx, m->d_hoff, m->d_H, m->d_poff_b1, m->grad);
  hipLaunchKernelGGL(k_mlp_colsum, dim3(nblk(hcols)), dim3(256), 0, st, m->G2, B, hcols, m->d_hcol_area,
                     m->d_hcol_idx, m->d_hoff, m->d_H, m->d_poff_b2, m->grad);
  hipLaunchKernelGGL(k_mlp_colsum, dim3(nblk(m->n_out)), dim3(256), 0, st, m->G3, B, m->n_out,
                     m->d_ocol_area, m->d_ocol_idx, m->d_yoff, m->d_ok, m->d_poff_b3, m->grad);
  HIPTRY(hipGetLastError());
  if (loss) {
    std::vector<double> lp(nb);
    HIPTRY(hipMemcpyAsync(lp.data(), m->lossp, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s / (double)nout;
  }
  return 0;
}

int check_mlp(mase_mlp* m, int B) {
  if (!m) return fail(MASE_ERR_ARG, "null mlp");
  if (B < 1 || B > m->Bmax) return fail(MASE_ERR_ARG, "batch size out of range");
  if (!m->have_norm) return fail(MASE_ERR_STATE, "normalisation not set (mase_mlp_set_norm)");
  return 0;
}

}  // namespace

extern "C" {

int mase_mlp_create(mase_ctx* c, int32_t hidden, int32_t max_batch, mase_mlp** out) {
  if (!c || !out) return fail(MASE_ERR_ARG, "null argument");
  *out = nullptr;
  if (c->host_only) return fail(MASE_ERR_NO_DEVICE, "host-only context");
  if (hidden < 1 || max_batch < 1) return fail(MASE_ERR_ARG, "hidden and max_batch must be >= 1");
  const Plan& p = c->plan;
  mase_mlp* m = new mase_mlp();
  m->ctx = c;
  m->K = p.n_area;
  m->H = hidden;
  m->Bmax = std::max<int>(max_batch, p.n_snap);
  m->n_meas = p.n_meas;
  m->n_bus = p.n_bus;
  const int K = m->K, H = m->H;
  m->in_meas.assign(K, {});
  m->out_var.assign(K, {});
  for (int k = 0; k < K; ++k) {
    m->in_meas[k] = p.tpl[k].row_meas;
    std::vector<int> own;
    for (int b = 0; b < p.n_bus; ++b)
      if (p.bus_area[b] == k) own.push_back(b);
    for (int b : own) { m->out_var[k].push_back(2 * b); m->out_var[k].push_back(2 * b + 1); }
    m->mk.push_back((int)m->in_meas[k].size());
    m->ok.push_back((int)m->out_var[k].size());
  }
  std::vector<int> in_area, in_idx, in_meas, out_area, out_idx, out_var, hca, hci, oca, oci, Hv(K, H);
  std::vector<long long> pb1, pb2, pb3;
  long long po = 0, xo = 0, ho = 0, yo = 0;
  for (int k = 0; k < K; ++k) {
    const long long mk = m->mk[k], ok = m->ok[k];
    m->poff.push_back(po);
    pb1.push_back(po + mk * H);
    pb2.push_back(po + mk * H + H + (long long)H * H);
    pb3.push_back(po + mk * H + H + (long long)H * H + H + (long long)H * ok);
    po += mk * H + H + (long long)H * H + H + (long long)H * ok + ok;
    m->xoff.push_back(xo);
    xo += (long long)m->Bmax * mk;
    m->hoff.push_back(ho);
    ho += (long long)m->Bmax * H;
    m->yoff.push_back(yo);
    yo += (long long)m->Bmax * ok;
    for (int i = 0; i < (int)mk; ++i) { in_area.push_back(k); in_idx.push_back(i); in_meas.push_back(m->in_meas[k][i]); }
    for (int j = 0; j < (int)ok; ++j) {
      out_area.push_back(k); out_idx.push_back(j); out_var.push_back(m->out_var[k][j]);
      oca.push_back(k); oci.push_back(j);
    }
    for (int j = 0; j < H; ++j) { hca.push_back(k); hci.push_back(j); }
  }
  m->nparam = po;
  m->n_out = (int)out_var.size();
  int rc = 0;
  if (!rc) rc = mdalloc(m, po, &m->theta);
  if (!rc) rc = mdalloc(m, po, &m->grad);
  if (!rc) rc = mdalloc(m, po, &m->m);
  if (!rc) rc = mdalloc(m, po, &m->v);
  if (!rc) rc = mdalloc(m, po, &m->thb);
  if (!rc) rc = mdalloc(m, xo, &m->X);
  if (!rc) rc = mdalloc(m, ho, &m->P1);
  if (!rc) rc = mdalloc(m, ho, &m->H1b);
  if (!rc) rc = mdalloc(m, ho, &m->P2);
  if (!rc) rc = mdalloc(m, ho, &m->H2b);
  if (!rc) rc = mdalloc(m, ho, &m->G2);
  if (!rc) rc = mdalloc(m, ho, &m->G2b);
  if (!rc) rc = mdalloc(m, ho, &m->G1);
  if (!rc) rc = mdalloc(m, ho, &m->G1b);
  if (!rc) rc = mdalloc(m, yo, &m->Y);
  if (!rc) rc = mdalloc(m, yo, &m->T);
  if (!rc) rc = mdalloc(m, yo, &m->G3);
  if (!rc) rc = mdalloc(m, yo, &m->G3b);
  if (!rc) rc = mdalloc(m, p.n_meas, &m->zmean);
  if (!rc) rc = mdalloc(m, 2 * (size_t)p.n_bus, &m->ymean);
  if (!rc) rc = mdalloc(m, 2 * (size_t)p.n_bus, &m->ystd);
  if (!rc) rc = mupload(m, p.sigma, &m->sigma);
  if (!rc) rc = mdalloc(m, p.n_meas, &m->zms);
  if (!rc) rc = mdalloc(m, K, &m->area_rms);
  if (!rc) rc = mdalloc(m, nblk((long long)m->Bmax * m->n_out), &m->lossp);
  if (!rc) rc = mupload(m, in_area, &m->d_in_area);
  if (!rc) rc = mupload(m, in_idx, &m->d_in_idx);
  if (!rc) rc = mupload(m, in_meas, &m->d_in_meas);
  if (!rc) rc = mupload(m, out_area, &m->d_out_area);
  if (!rc) rc = mupload(m, out_idx, &m->d_out_idx);
  if (!rc) rc = mupload(m, out_var, &m->d_out_var);
  if (!rc) rc = mupload(m, m->mk, &m->d_mk);
  if (!rc) rc = mupload(m, m->ok, &m->d_ok);
  if (!rc) rc = mupload(m, m->xoff, &m->d_xoff);
  if (!rc) rc = mupload(m, m->hoff, &m->d_hoff);
  if (!rc) rc = mupload(m, m->yoff, &m->d_yoff);
  if (!rc) rc = mupload(m, pb1, &m->d_poff_b1);
  if (!rc) rc = mupload(m, pb2, &m->d_poff_b2);
  if (!rc) rc = mupload(m, pb3, &m->d_poff_b3);
  if (!rc) rc = mupload(m, hca, &m->d_hcol_area);
  if (!rc) rc = mupload(m, hci, &m->d_hcol_idx);
  if (!rc) rc = mupload(m, oca, &m->d_ocol_area);
  if (!rc) rc = mupload(m, oci, &m->d_ocol_idx);
  if (!rc) rc = mupload(m, Hv, &m->d_H);
  const size_t SN = (size_t)p.n_snap * p.n_bus;
  if (!rc) rc = mdalloc(m, SN, &m->xpred);
  if (!rc) rc = mdalloc(m, SN, &m->xflat);
  if (!rc) rc = mdalloc(m, (size_t)p.n_snap * K, &m->jpred);
  if (!rc) rc = mdalloc(m, (size_t)p.n_snap * K, &m->jflat);
  if (!rc) rc = mdalloc(m, p.n_snap, &m->d_accepted);
  if (!rc) {
    hipError_t e = hipMemset(m->theta, 0, sizeof(float) * po);
    if (e == hipSuccess) e = hipMemset(m->m, 0, sizeof(float) * po);
    if (e == hipSuccess) e = hipMemset(m->v, 0, sizeof(float) * po);
    if (e == hipSuccess) e = hipMemset(m->thb, 0, sizeof(uint16_t) * po);
    if (e != hipSuccess) rc = fail(MASE_ERR_HIP, hipGetErrorString(e));
  }
  if (rc) {
    mase_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return 0;
}

void mase_mlp_destroy(mase_mlp* m) {
  if (!m) return;
  if (m->ctx && m->ctx->stream) (void)hipStreamSynchronize(m->ctx->stream);
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
}

int mase_mlp_info(const mase_mlp* m, int32_t area, int32_t* n_in, int32_t* n_out, int64_t* n_param) {
  if (!m) return fail(MASE_ERR_ARG, "null mlp");
  if (area < -1 || area >= m->K) return fail(MASE_ERR_ARG, "area out of range");
  if (area >= 0) {
    if (n_in) *n_in = m->mk[area];
    if (n_out) *n_out = m->ok[area];
  } else {
    if (n_in) *n_in = m->n_meas;
    if (n_out) *n_out = m->n_out;
  }
  if (n_param) *n_param = m->nparam;
  return 0;
}

int mase_mlp_io_map(const mase_mlp* m, int32_t area, int32_t* in_meas, int32_t* out_var) {
  if (!m || area < 0 || area >= m->K) return fail(MASE_ERR_ARG, "bad argument");
  if (in_meas) std::copy(m->in_meas[area].begin(), m->in_meas[area].end(), in_meas);
  if (out_var) std::copy(m->out_var[area].begin(), m->out_var[area].end(), out_var);
  return 0;
}

int mase_mlp_set_params(mase_mlp* m, const float* params) {
  if (!m || !params) return fail(MASE_ERR_ARG, "null argument");
  HIPTRY(hipMemcpy(m->theta, params, sizeof(float) * m->nparam, hipMemcpyHostToDevice));
  HIPTRY(hipMemset(m->m, 0, sizeof(float) * m->nparam));
  HIPTRY(hipMemset(m->v, 0, sizeof(float) * m->nparam));
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(m->nparam)), dim3(256), 0, m->ctx->stream, m->theta, m->thb, m->nparam);
  HIPTRY(hipGetLastError());
  HIPTRY(hipStreamSynchronize(m->ctx->stream));
  m->step = 0;
  return 0;
}

int mase_mlp_get_params(mase_mlp* m, float* params) {
  if (!m || !params) return fail(MASE_ERR_ARG, "null argument");
  HIPTRY(hipStreamSynchronize(m->ctx->stream));
  HIPTRY(hipMemcpy(params, m->theta, sizeof(float) * m->nparam, hipMemcpyDeviceToHost));
  return 0;
}

int mase_mlp_set_norm(mase_mlp* m, const double* z_mean, const double* y_mean, const double* y_std) {
  if (!m || !z_mean || !y_mean || !y_std) return fail(MASE_ERR_ARG, "null argument");
  for (int i = 0; i < 2 * m->n_bus; ++i)
    if (!(y_std[i] > 0.0)) return fail(MASE_ERR_ARG, "y_std must be > 0");
  HIPTRY(hipMemcpy(m->zmean, z_mean, sizeof(double) * m->n_meas, hipMemcpyHostToDevice));
  HIPTRY(hipMemcpy(m->ymean, y_mean, sizeof(double) * 2 * m->n_bus, hipMemcpyHostToDevice));
  HIPTRY(hipMemcpy(m->ystd, y_std, sizeof(double) * 2 * m->n_bus, hipMemcpyHostToDevice));
  m->have_norm = true;
  return 0;
}

int mase_mlp_fit_norm(mase_mlp* m, const double* z_dev, const double* vm_dev, const double* va_dev, int32_t n,
                      double* in_rms) {
  if (!m || !z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null argument");
  if (n < 1) return fail(MASE_ERR_ARG, "need at least one training snapshot");
  hipStream_t st = m->ctx->stream;
  const long long nn = n;
  const int nb = m->n_bus;
  hipLaunchKernelGGL(k_col_stats, dim3((m->n_meas + 255) / 256), dim3(256), 0, st, z_dev, nn, m->n_meas,
                     m->zmean, (double*)nullptr, 1, 0);
  // outputs interleaved per bus: (theta, |V|)
  hipLaunchKernelGGL(k_col_stats, dim3((nb + 255) / 256), dim3(256), 0, st, va_dev, nn, nb, m->ymean, m->ystd,
                     2, 0);
  hipLaunchKernelGGL(k_col_stats, dim3((nb + 255) / 256), dim3(256), 0, st, vm_dev, nn, nb, m->ymean, m->ystd,
                     2, 1);
  hipLaunchKernelGGL(k_norm_ms, dim3((m->n_meas + 255) / 256), dim3(256), 0, st, z_dev, nn, m->n_meas, m->zmean,
                     m->sigma, m->zms);
  hipLaunchKernelGGL(k_area_rms, dim3(m->K), dim3(256), 0, st, m->zms, m->d_in_meas, m->d_mk, m->area_rms);
  HIPTRY(hipGetLastError());
  if (in_rms) HIPTRY(hipMemcpyAsync(in_rms, m->area_rms, sizeof(double) * m->K, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  m->have_norm = true;
  return 0;
}

int mase_mlp_get_norm(const mase_mlp* m, double* z_mean, double* y_mean, double* y_std) {
  if (!m || !z_mean || !y_mean || !y_std) return fail(MASE_ERR_ARG, "null argument");
  if (!m->have_norm) return fail(MASE_ERR_STATE, "normalisation not set");
  HIPTRY(hipMemcpy(z_mean, m->zmean, sizeof(double) * m->n_meas, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(y_mean, m->ymean, sizeof(double) * 2 * m->n_bus, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(y_std, m->ystd, sizeof(double) * 2 * m->n_bus, hipMemcpyDeviceToHost));
  return 0;
}

int mase_mlp_loss_grad(mase_mlp* m, const double* z_dev, const double* vm_dev, const double* va_dev,
                       int32_t batch, double* loss, float* grad) {
  int rc = check_mlp(m, batch);
  if (rc) return rc;
  if (!z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null device pointer");
  if ((rc = forward(m, z_dev, batch))) return rc;
  if ((rc = backward(m, vm_dev, va_dev, batch, loss))) return rc;
  if (grad) {
    HIPTRY(hipStreamSynchronize(m->ctx->stream));
    HIPTRY(hipMemcpy(grad, m->grad, sizeof(float) * m->nparam, hipMemcpyDeviceToHost));
  }
  return 0;
}

int mase_mlp_train_step(mase_mlp* m, const double* z_dev, const double* vm_dev, const double* va_dev,
                        int32_t batch, float lr, double* loss) {
  int rc = check_mlp(m, batch);
  if (rc) return rc;
  if (!z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null device pointer");
  if ((rc = forward(m, z_dev, batch))) return rc;
  if ((rc = backward(m, vm_dev, va_dev, batch, loss))) return rc;
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(m->nparam)), dim3(256), 0, m->ctx->stream, m->theta, m->grad, m->m,
                     m->v, m->thb, m->nparam, lr, b1, b2, 1e-8f, c1, c2);
  HIPTRY(hipGetLastError());
  return 0;
}

int mase_mlp_predict_dev(mase_mlp* m, const double* z_dev, int32_t batch, double* vm_dev, double* va_dev) {
  int rc = check_mlp(m, batch);
  if (rc) return rc;
  if (!z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null device pointer");
  if ((rc = forward(m, z_dev, batch))) return rc;
  const long long nout = (long long)batch * m->n_out;
  hipLaunchKernelGGL(k_mlp_compose, dim3(nblk(nout)), dim3(256), 0, m->ctx->stream, m->Y, batch, m->n_out,
                     m->n_bus, m->ctx->plan.slack, m->ymean, m->ystd, m->d_out_area, m->d_out_idx,
                     m->d_out_var, m->d_yoff, m->d_ok, vm_dev, va_dev, (double2*)nullptr);
  HIPTRY(hipGetLastError());
  return 0;
}

int mase_warm_start(mase_ctx* c, mase_mlp* m, int32_t* accepted) {
  if (!c || !m || m->ctx != c) return fail(MASE_ERR_ARG, "mlp does not belong to this context");
  const int S = c->plan.n_snap;
  int rc = check_mlp(m, S);
  if (rc) return rc;
  if (!c->have_z) return fail(MASE_ERR_STATE, "no measurements set");
  hipStream_t st = c->stream;
  if (m->j_cap < 0.0) {
    // J >= 0, so no prediction can pass a negative cap: flat start for every
    // snapshot without evaluating the network or the objectives
    HIPTRY(launch_pack_state(c->d, nullptr, nullptr, c->d.x, st));
    HIPTRY(launch_reset_flags(c->d, st));
    for (int s = 0; s < S; ++s) c->h_active[s] = 1;
    m->last_ws = -S;
    if (accepted) std::memset(accepted, 0, sizeof(int32_t) * S);
    return 0;
  }
  if ((rc = forward(m, c->d.z, S))) return rc;
  const long long nout = (long long)S * m->n_out;
  hipLaunchKernelGGL(k_mlp_compose, dim3(nblk(nout)), dim3(256), 0, st, m->Y, S, m->n_out, m->n_bus,
                     c->plan.slack, m->ymean, m->ystd, m->d_out_area, m->d_out_idx, m->d_out_var,
                     m->d_yoff, m->d_ok, (double*)nullptr, (double*)nullptr, m->xpred);
  HIPTRY(hipGetLastError());
  HIPTRY(launch_pack_state(c->d, nullptr, nullptr, m->xflat, st));
  if ((rc = objective_at(c, m->xpred, m->jpred))) return rc;
  if ((rc = objective_at(c, m->xflat, m->jflat))) return rc;
  hipLaunchKernelGGL(k_choose, dim3(S), dim3(256), 0, st, m->jpred, m->jflat, c->plan.n_area, c->plan.n_bus,
                     m->j_cap, m->xpred, m->xflat, c->d.x, m->d_accepted);
  HIPTRY(hipGetLastError());
  m->last_ws = S;
  HIPTRY(launch_reset_flags(c->d, st));
  for (int s = 0; s < S; ++s) c->h_active[s] = 1;
  if (accepted) {
    HIPTRY(hipMemcpyAsync(accepted, m->d_accepted, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
  }
  return 0;
}

int mase_mlp_set_accept_cap(mase_mlp* m, double j_cap) {
  if (!m) return fail(MASE_ERR_ARG, "null mlp");
  if (std::isnan(j_cap)) return fail(MASE_ERR_ARG, "j_cap is NaN");
  m->j_cap = j_cap;
  return 0;
}

int mase_warm_start_objectives(const mase_mlp* m, double* j_pred, double* j_flat) {
  if (!m || !j_pred || !j_flat) return fail(MASE_ERR_ARG, "null argument");
  if (m->last_ws == 0) return fail(MASE_ERR_STATE, "no warm start evaluated yet");
  if (m->last_ws < 0) {  // short-circuited by a negative cap: nothing evaluated
    for (int s = 0; s < -m->last_ws; ++s) j_pred[s] = j_flat[s] = std::nan("");
    return 0;
  }
  const int S = m->last_ws, K = m->ctx->plan.n_area;
  std::vector<double> jp((size_t)S * K), jf((size_t)S * K);
  HIPTRY(hipStreamSynchronize(m->ctx->stream));
  HIPTRY(hipMemcpy(jp.data(), m->jpred, sizeof(double) * jp.size(), hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(jf.data(), m->jflat, sizeof(double) * jf.size(), hipMemcpyDeviceToHost));
  for (int s = 0; s < S; ++s) {
    double a = 0.0, f = 0.0;
    for (int k = 0; k < K; ++k) {
      a += jp[(size_t)s * K + k];
      f += jf[(size_t)s * K + k];
    }
    j_pred[s] = a;
    j_flat[s] = f;
  }
  return 0;
}

}  // extern "C"

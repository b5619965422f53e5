// Warm-start network on the device: a multilayer perceptron
//   inputs -> [Linear -> GELU] x n_layers -> Linear -> outputs
// with bfloat16 GEMM operands on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16, float32 accumulation), fused bias / GELU /
// GELU' epilogues, a hand-written backward pass, Adam on float32 master
// weights and a bfloat16 copy of the weights (and of their transpose, for the
// input-gradient GEMM) refreshed after every step.
//
// Every GEMM is C[M][N] = sum_k A[m][k] B[n][k] with both operands K-contiguous,
// so each lane reads its 8-element MFMA fragment with one 16-byte load.  The
// producers write each activation and each back-propagated gradient in both
// [batch][feature] and [feature][batch] layouts, which is what the weight-
// gradient GEMM (reduction over the batch) needs.  A wave computes a 32x32
// tile (2x2 MFMA tiles); the layer widths are multiples of 32 (inputs padded
// to 32, outputs to the next multiple of 32 with zero weights).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "internal.h"

struct absorber_mlp;

namespace absorber {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TT = 32;  // tile edge (M, N) and K step

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_BWD = 2, EPI_WGRAD = 3 };

struct Epi {
  const float* bias = nullptr;  // [N]                                   (HIDDEN, OUT)
  float* zf = nullptr;          // pre-activation [M][ldz]: written (HIDDEN), read (BWD)
  int ldz = 0;
  __bf16* h = nullptr;          // bf16 result [M][ldh]: activation (HIDDEN) or dL/dZ (BWD)
  int ldh = 0;
  __bf16* ht = nullptr;         // the same, transposed [N][ldht] (optional)
  int ldht = 0;
  float* y = nullptr;           // float result [M][ldy] (OUT: outputs, WGRAD: weight gradient)
  int ldy = 0;
  int m_real = 0, n_real = 0;   // OUT / WGRAD store rows < m_real and cols < n_real only
  int n_par = 0;                // OUT: entries of the bias and standardisation arrays
  const float* omean = nullptr; // OUT: optional un-standardisation y * ostd + omean
  const float* ostd = nullptr;
};

// C = A B^T on 32x32 tiles, one wave per tile.  MFMA 16x16x32 operand layout:
// lane l supplies A[l % 16][8 (l / 16) + 0..7] and B^T[l % 16][8 (l / 16) + 0..7];
// it receives C[4 (l / 16) + r][l % 16], r = 0..3.
template <int EPI>
__global__ __launch_bounds__(64) void k_gemm(const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B,
                                             int ldb, int M, int N, int K, Epi e) {
  const int lane = threadIdx.x;
  const int m0 = blockIdx.x * TT, n0 = blockIdx.y * TT;
  const int li = lane & 15, lk = (lane >> 4) * 8;
  const int ma = m0 + li, mb = m0 + 16 + li;
  const bool va = ma < M, vb = mb < M;
  const __bf16* pa0 = A + (long long)(va ? ma : 0) * lda + lk;
  const __bf16* pa1 = A + (long long)(vb ? mb : 0) * lda + lk;
  const __bf16* pb0 = B + (long long)(n0 + li) * ldb + lk;
  const __bf16* pb1 = B + (long long)(n0 + 16 + li) * ldb + lk;
  f32x4 c00 = {0.f, 0.f, 0.f, 0.f}, c01 = c00, c10 = c00, c11 = c00;
  const bf16x8 zero = {};
  for (int k = 0; k < K; k += TT) {
    const bf16x8 a0 = va ? *(const bf16x8*)(pa0 + k) : zero;
    const bf16x8 a1 = vb ? *(const bf16x8*)(pa1 + k) : zero;
    const bf16x8 b0 = *(const bf16x8*)(pb0 + k);
    const bf16x8 b1 = *(const bf16x8*)(pb1 + k);
    c00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, c00, 0, 0, 0);
    c01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, c01, 0, 0, 0);
    c10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, c10, 0, 0, 0);
    c11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, c11, 0, 0, 0);
  }
  const f32x4 cc[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + 16 * b + li;
      const int mr = m0 + 16 * a + 4 * (lane >> 4);
      float o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mr + r;
        const float acc = cc[a][b][r];
        if (EPI == EPI_HIDDEN) {
          const float z = acc + e.bias[n];
          const float hv = gelu_f(z);
          o[r] = hv;
          if (m < M) {
            if (e.zf) e.zf[(long long)m * e.ldz + n] = z;
            e.h[(long long)m * e.ldh + n] = (__bf16)hv;
          }
        } else if (EPI == EPI_OUT) {
          // the output bias and the standardisation arrays hold n_par entries: a
          // padded column (n >= n_par, zero weights) takes bias 0 and is never
          // un-standardised, so no read leaves those arrays
          if (m < M && m < e.m_real && n < e.n_real) {
            float yv = acc + (n < e.n_par ? e.bias[n] : 0.0f);
            if (e.ostd && n < e.n_par) yv = yv * e.ostd[n] + e.omean[n];
            e.y[(long long)m * e.ldy + n] = yv;
          }
        } else if (EPI == EPI_BWD) {
          const float g = m < M ? acc * gelu_d(e.zf[(long long)m * e.ldz + n]) : 0.0f;
          o[r] = g;
          if (m < M) e.h[(long long)m * e.ldh + n] = (__bf16)g;
        } else {  // EPI_WGRAD
          if (m < M && m < e.m_real && n < e.n_real) e.y[(long long)m * e.ldy + n] = acc;
        }
      }
      if ((EPI == EPI_HIDDEN || EPI == EPI_BWD) && e.ht) {
        // four consecutive rows of column n: one 8-byte store into the transpose
        // (rows beyond M are stored as computed: zero inputs give finite values,
        // and the transposed buffers are padded to a multiple of 32 rows)
        bf16x4 q;
#pragma unroll
        for (int r = 0; r < 4; ++r) q[r] = mr + r < M ? (__bf16)o[r] : (__bf16)0.0f;
        *(bf16x4*)(e.ht + (long long)n * e.ldht + mr) = q;
      }
    }
}

// minibatch assembly: standardised inputs (bf16, padded to kin columns, both
// layouts) and standardised float targets; src = perm[b0 + b] or b0 + b
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ T, const int* __restrict__ perm,
                         long long b0, int B, int n_in, int kin, int n_out, int ldht,
                         const float* __restrict__ imean, const float* __restrict__ istd,
                         const float* __restrict__ omean, const float* __restrict__ ostd, __bf16* __restrict__ H0,
                         __bf16* __restrict__ H0t, float* __restrict__ Tstd) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int wi = kin > n_out ? kin : n_out;
  if (i >= (long long)B * wi) return;
  const int b = (int)(i / wi), j = (int)(i % wi);
  const long long src = perm ? (long long)perm[b0 + b] : b0 + b;
  if (j < kin) {
    const float v = j < n_in ? (X[src * n_in + j] - imean[j]) / istd[j] : 0.0f;
    H0[(long long)b * kin + j] = (__bf16)v;
    if (H0t) H0t[(long long)j * ldht + b] = (__bf16)v;
  }
  if (T && j < n_out) Tstd[(long long)b * n_out + j] = (T[src * n_out + j] - omean[j]) / ostd[j];
}

// dL/dY of the mean squared error over B x n_out entries, as bf16 in both
// layouts (padded columns get 0), and per-block partial sums of the squared error
__global__ void k_loss(const float* __restrict__ Y, int ldy, const float* __restrict__ Tstd, int B, int n_out,
                       int nout_p, int ldgt, __bf16* __restrict__ G, __bf16* __restrict__ Gt,
                       float* __restrict__ part) {
  __shared__ float sm[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  float se = 0.0f;
  if (i < (long long)B * nout_p) {
    const int b = (int)(i / nout_p), j = (int)(i % nout_p);
    float g = 0.0f;
    if (j < n_out) {
      const float r = Y[(long long)b * ldy + j] - Tstd[(long long)b * n_out + j];
      se = r * r;
      g = 2.0f * r / ((float)B * (float)n_out);
    }
    G[(long long)b * nout_p + j] = (__bf16)g;
    Gt[(long long)j * ldgt + b] = (__bf16)g;
  }
  sm[threadIdx.x] = se;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// bias gradient: db[j] = sum over the batch of Gt[j][0..B), one wave per j (fixed order)
__global__ __launch_bounds__(64) void k_bias_grad(const __bf16* __restrict__ Gt, int ldgt, int B,
                                                  float* __restrict__ db) {
  const int j = blockIdx.x;
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 64) s += (float)Gt[(long long)j * ldgt + b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) db[j] = s;
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies of W [out][in]: Wq [out][ldq] and its transpose Wqt [in][ldqt]
__global__ void k_refresh(const float* __restrict__ W, int out, int in, __bf16* __restrict__ Wq, int ldq,
                          __bf16* __restrict__ Wqt, int ldqt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)out * in) return;
  const int r = (int)(i / in), c = (int)(i % in);
  const __bf16 q = (__bf16)W[i];
  Wq[(long long)r * ldq + c] = q;
  if (Wqt) Wqt[(long long)c * ldqt + r] = q;
}

// column mean and standard deviation of a float matrix [n][w] (float64 sums,
// one thread per column, fixed order); std floored at 1e-6 times (1 + |mean|)
__global__ void k_colstats(const float* __restrict__ X, long long n, int w, float* __restrict__ mean,
                           float* __restrict__ sd) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= w) return;
  double s = 0.0;
  for (long long i = 0; i < n; ++i) s += X[i * w + j];
  const double mu = s / (double)n;
  double q = 0.0;
  for (long long i = 0; i < n; ++i) {
    const double d = X[i * w + j] - mu;
    q += d * d;
  }
  const double sdv = sqrt(q / (double)n);
  mean[j] = (float)mu;
  sd[j] = (float)fmax(sdv, 1e-6 * (1.0 + fabs(mu)));
}

__global__ void k_fill_f(float* p, float v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline int pad32(int v) { return (v + 31) / 32 * 32; }

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit_normal(uint64_t& s) {  // Box-Muller on two uniforms in (0, 1]
  const double u1 = ((splitmix64(s) >> 11) + 1) * (1.0 / 9007199254740992.0);
  const double u2 = ((splitmix64(s) >> 11) + 1) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace

struct MlpImpl {
  absorber_mlp_config cfg{};
  int L = 0;                                   // linear layers
  std::vector<int> din, dout, kin, nout;       // real and padded widths per layer
  std::vector<long long> offW, offb;           // offsets in the flat parameter vector
  long long nparam = 0;
  float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  std::vector<__bf16*> Wq, Wqt, H, Ht, G, Gt;  // H[l]: input of layer l; G[l]: dL/dZ_l
  std::vector<float*> Z;                       // pre-activations of the hidden layers
  float *Y = nullptr, *Tstd = nullptr, *lpart = nullptr;
  float *imean = nullptr, *istd = nullptr, *omean = nullptr, *ostd = nullptr;
  int* perm = nullptr;
  int* perm_h = nullptr;                       // pinned
  float* lpart_h = nullptr;                    // pinned
  long long perm_cap = 0;
  int t = 0;                                   // Adam step counter
  std::vector<void*> allocs;

  template <class T>
  hipError_t dal(T** p, long long n) {
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)(n > 0 ? n : 1));
    if (e == hipSuccess) {
      allocs.push_back((void*)*p);
      e = hipMemset(*p, 0, sizeof(T) * (size_t)(n > 0 ? n : 1));
    }
    return e;
  }
  ~MlpImpl() {
    for (void* p : allocs) (void)hipFree(p);
    if (perm_h) (void)hipHostFree(perm_h);
    if (lpart_h) (void)hipHostFree(lpart_h);
  }

  int refresh(hipStream_t st) {
    for (int l = 0; l < L; ++l) {
      const long long n = (long long)dout[l] * din[l];
      hipLaunchKernelGGL(k_refresh, dim3(nblk(n, 256)), dim3(256), 0, st, P + offW[l], dout[l], din[l], Wq[l], kin[l],
                         Wqt[l], nout[l]);
    }
    HIP_TRY(hipGetLastError());
    return ABS_OK;
  }

  // forward over rows [0, B) of H[0]; train: keep Z and the transposed activations
  int forward(int B, bool train, float* yout, int ldy, int m_real, const float* om, const float* os, hipStream_t st) {
    const int Bp = cfg.max_batch;
    for (int l = 0; l < L; ++l) {
      dim3 grid(nblk(B, TT), nout[l] / TT);
      Epi e;
      e.bias = P + offb[l];
      if (l < L - 1) {
        e.zf = train ? Z[l] : nullptr;
        e.ldz = nout[l];
        e.h = H[l + 1];
        e.ldh = kin[l + 1];
        e.ht = train ? Ht[l + 1] : nullptr;
        e.ldht = Bp;
        hipLaunchKernelGGL(k_gemm<EPI_HIDDEN>, grid, dim3(64), 0, st, H[l], kin[l], Wq[l], kin[l], B, nout[l], kin[l], e);
      } else {
        e.y = yout;
        e.ldy = ldy;
        e.m_real = m_real;
        e.n_real = train ? nout[l] : dout[l];
        e.n_par = dout[l];
        e.omean = om;
        e.ostd = os;
        hipLaunchKernelGGL(k_gemm<EPI_OUT>, grid, dim3(64), 0, st, H[l], kin[l], Wq[l], kin[l], B, nout[l], kin[l], e);
      }
    }
    HIP_TRY(hipGetLastError());
    return ABS_OK;
  }

  // loss and gradient of one assembled minibatch of B rows (B % 32 == 0) into g
  int backward(int B, hipStream_t st, int* nparts) {
    const int Bp = cfg.max_batch;
    const int no = dout[L - 1], nop = nout[L - 1];
    const int np = (int)nblk((long long)B * nop, 256);
    hipLaunchKernelGGL(k_loss, dim3(np), dim3(256), 0, st, Y, nop, Tstd, B, no, nop, Bp, G[L - 1], Gt[L - 1], lpart);
    *nparts = np;
    for (int l = L - 1; l >= 0; --l) {
      {  // dW_l = G_l^T H_l  (M = out, N = in, K = batch)
        Epi e;
        e.y = g + offW[l];
        e.ldy = din[l];
        e.m_real = dout[l];
        e.n_real = din[l];
        dim3 grid(nblk(nout[l], TT), kin[l] / TT);
        hipLaunchKernelGGL(k_gemm<EPI_WGRAD>, grid, dim3(64), 0, st, Gt[l], Bp, Ht[l], Bp, nout[l], kin[l], B, e);
      }
      hipLaunchKernelGGL(k_bias_grad, dim3(dout[l]), dim3(64), 0, st, Gt[l], Bp, B, g + offb[l]);
      if (l > 0) {  // G_{l-1} = (G_l W_l) * GELU'(Z_{l-1})  (M = batch, N = in, K = out)
        Epi e;
        e.zf = Z[l - 1];
        e.ldz = nout[l - 1];
        e.h = G[l - 1];
        e.ldh = nout[l - 1];
        e.ht = Gt[l - 1];
        e.ldht = Bp;
        dim3 grid(nblk(B, TT), kin[l] / TT);
        hipLaunchKernelGGL(k_gemm<EPI_BWD>, grid, dim3(64), 0, st, G[l], nout[l], Wqt[l], nout[l], B, kin[l], nout[l],
                           e);
      }
    }
    HIP_TRY(hipGetLastError());
    return ABS_OK;
  }

  int adam(const float* grad, double lr, const absorber_mlp_train_options& o, hipStream_t st) {
    ++t;
    const float c1 = (float)(1.0 - pow(o.beta1, t)), c2 = (float)(1.0 - pow(o.beta2, t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(nparam, 256)), dim3(256), 0, st, P, m, v, grad, nparam, (float)lr,
                       (float)o.beta1, (float)o.beta2, (float)o.eps, c1, c2);
    HIP_TRY(hipGetLastError());
    return refresh(st);
  }

  int gather(const float* X, const float* T, const int* pm, long long b0, int B, hipStream_t st) {
    const int wi = std::max(kin[0], dout[L - 1]);
    hipLaunchKernelGGL(k_gather, dim3(nblk((long long)B * wi, 256)), dim3(256), 0, st, X, T, pm, b0, B, cfg.n_in,
                       kin[0], dout[L - 1], cfg.max_batch, imean, istd, omean, ostd, H[0], Ht[0], Tstd);
    HIP_TRY(hipGetLastError());
    return ABS_OK;
  }

  double loss_from_parts(int np, hipStream_t st) {
    if (hipMemcpyAsync(lpart_h, lpart, sizeof(float) * np, hipMemcpyDeviceToHost, st) != hipSuccess) return NAN;
    if (hipStreamSynchronize(st) != hipSuccess) return NAN;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += lpart_h[i];
    return s;
  }
};

}  // namespace absorber

struct absorber_mlp {
  absorber::MlpImpl impl;
};

using absorber::MlpImpl;
using absorber::set_error;

namespace {
hipStream_t as_stream(void* s) { return (hipStream_t)s; }

bool check_batch(const MlpImpl& M, long long n, bool train) {
  if (n <= 0 || n > M.cfg.max_batch || (train && n % 32 != 0)) {
    set_error("warm-start network: batch size out of range (1..max_batch, a multiple of 32 for training)");
    return false;
  }
  return true;
}
}  // namespace

extern "C" {

void absorber_mlp_default_config(absorber_mlp_config* c) {
  if (!c) return;
  c->n_in = 3;
  c->n_hidden = 256;
  c->n_layers = 3;
  c->n_out = 210;
  c->max_batch = 512;
}

void absorber_mlp_default_train_options(absorber_mlp_train_options* o) {
  if (!o) return;
  o->epochs = 300;
  o->batch = 512;
  o->lr = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  o->seed = 4;
  o->cosine = 1;
}

int absorber_mlp_create(const absorber_mlp_config* cfg, uint64_t seed, absorber_mlp** out) {
  if (!cfg || !out || cfg->n_in < 1 || cfg->n_in > 32 || cfg->n_hidden < 32 || cfg->n_hidden % 32 != 0 ||
      cfg->n_layers < 1 || cfg->n_out < 1 || cfg->max_batch < 32 || cfg->max_batch % 32 != 0) {
    set_error("absorber_mlp_create: bad configuration (n_in 1..32, n_hidden and max_batch multiples of 32)");
    return ABS_ERR_ARG;
  }
  absorber_mlp* w = new (std::nothrow) absorber_mlp;
  if (!w) return ABS_ERR_OOM;
  MlpImpl& M = w->impl;
  M.cfg = *cfg;
  M.L = cfg->n_layers + 1;
  for (int l = 0; l < M.L; ++l) {
    const int i = l == 0 ? cfg->n_in : cfg->n_hidden;
    const int o = l == M.L - 1 ? cfg->n_out : cfg->n_hidden;
    M.din.push_back(i);
    M.dout.push_back(o);
    M.kin.push_back(absorber::pad32(i));
    M.nout.push_back(absorber::pad32(o));
    M.offW.push_back(M.nparam);
    M.nparam += (long long)o * i;
    M.offb.push_back(M.nparam);
    M.nparam += o;
  }
  const int Bp = cfg->max_batch;
  int rc = ABS_OK;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && rc == ABS_OK) {
      set_error(std::string("absorber_mlp_create: ") + hipGetErrorString(e));
      rc = e == hipErrorOutOfMemory ? ABS_ERR_OOM : ABS_ERR_HIP;
    }
  };
  chk(M.dal(&M.P, M.nparam));
  chk(M.dal(&M.m, M.nparam));
  chk(M.dal(&M.v, M.nparam));
  chk(M.dal(&M.g, M.nparam));
  M.Wq.resize(M.L);
  M.Wqt.resize(M.L);
  M.H.resize(M.L);
  M.Ht.resize(M.L);
  M.G.resize(M.L);
  M.Gt.resize(M.L);
  M.Z.resize(M.L);
  for (int l = 0; l < M.L; ++l) {
    chk(M.dal(&M.Wq[l], (long long)M.nout[l] * M.kin[l]));
    chk(M.dal(&M.Wqt[l], (long long)M.kin[l] * M.nout[l]));
    chk(M.dal(&M.H[l], (long long)Bp * M.kin[l]));
    chk(M.dal(&M.Ht[l], (long long)M.kin[l] * Bp));
    chk(M.dal(&M.G[l], (long long)Bp * M.nout[l]));
    chk(M.dal(&M.Gt[l], (long long)M.nout[l] * Bp));
    if (l < M.L - 1) chk(M.dal(&M.Z[l], (long long)Bp * M.nout[l]));
  }
  chk(M.dal(&M.Y, (long long)Bp * M.nout[M.L - 1]));
  chk(M.dal(&M.Tstd, (long long)Bp * cfg->n_out));
  chk(M.dal(&M.lpart, (long long)Bp * M.nout[M.L - 1] / 256 + 8));
  chk(M.dal(&M.imean, cfg->n_in));
  chk(M.dal(&M.istd, cfg->n_in));
  chk(M.dal(&M.omean, cfg->n_out));
  chk(M.dal(&M.ostd, cfg->n_out));
  if (rc == ABS_OK &&
      hipHostMalloc((void**)&M.lpart_h, sizeof(float) * ((size_t)Bp * M.nout[M.L - 1] / 256 + 8)) != hipSuccess) {
    set_error("absorber_mlp_create: pinned host allocation failed");
    rc = ABS_ERR_OOM;
  }
  if (rc == ABS_OK) {
    // He-normal weights, zero biases; identity standardisation
    std::vector<float> p((size_t)M.nparam, 0.0f);
    uint64_t s = seed;
    for (int l = 0; l < M.L; ++l) {
      const double sc = sqrt(2.0 / M.din[l]);
      for (long long i = 0; i < (long long)M.dout[l] * M.din[l]; ++i)
        p[(size_t)(M.offW[l] + i)] = (float)(absorber::unit_normal(s) * sc);
    }
    chk(hipMemcpy(M.P, p.data(), sizeof(float) * p.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(absorber::k_fill_f, dim3(1), dim3(64), 0, 0, M.istd, 1.0f, (long long)cfg->n_in);
    hipLaunchKernelGGL(absorber::k_fill_f, dim3(absorber::nblk(cfg->n_out, 256)), dim3(256), 0, 0, M.ostd, 1.0f,
                       (long long)cfg->n_out);
    if (rc == ABS_OK) rc = M.refresh(0);
    chk(hipDeviceSynchronize());
  }
  if (rc != ABS_OK) {
    delete w;
    return rc;
  }
  *out = w;
  return ABS_OK;
}

void absorber_mlp_destroy(absorber_mlp* w) { delete w; }

int64_t absorber_mlp_num_params(const absorber_mlp* w) { return w ? w->impl.nparam : -1; }

int absorber_mlp_get_config(const absorber_mlp* w, absorber_mlp_config* out) {
  if (!w || !out) {
    set_error("absorber_mlp_get_config: bad argument");
    return ABS_ERR_ARG;
  }
  *out = w->impl.cfg;
  return ABS_OK;
}

int absorber_mlp_set_params(absorber_mlp* w, const float* params_host) {
  if (!w || !params_host) {
    set_error("absorber_mlp_set_params: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  HIP_TRY(hipMemcpy(M.P, params_host, sizeof(float) * M.nparam, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(M.m, 0, sizeof(float) * M.nparam));
  HIP_TRY(hipMemset(M.v, 0, sizeof(float) * M.nparam));
  M.t = 0;
  int rc = M.refresh(0);
  if (rc) return rc;
  HIP_TRY(hipDeviceSynchronize());
  return ABS_OK;
}

int absorber_mlp_get_params(const absorber_mlp* w, float* params_host) {
  if (!w || !params_host) {
    set_error("absorber_mlp_get_params: bad argument");
    return ABS_ERR_ARG;
  }
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(params_host, w->impl.P, sizeof(float) * w->impl.nparam, hipMemcpyDeviceToHost));
  return ABS_OK;
}

int absorber_mlp_set_normalization(absorber_mlp* w, const float* in_mean, const float* in_std,
                                   const float* out_mean, const float* out_std) {
  if (!w || !in_mean || !in_std || !out_mean || !out_std) {
    set_error("absorber_mlp_set_normalization: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  HIP_TRY(hipMemcpy(M.imean, in_mean, sizeof(float) * M.cfg.n_in, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(M.istd, in_std, sizeof(float) * M.cfg.n_in, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(M.omean, out_mean, sizeof(float) * M.cfg.n_out, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(M.ostd, out_std, sizeof(float) * M.cfg.n_out, hipMemcpyHostToDevice));
  return ABS_OK;
}

int absorber_mlp_get_normalization(const absorber_mlp* w, float* in_mean, float* in_std, float* out_mean,
                                   float* out_std) {
  if (!w || !in_mean || !in_std || !out_mean || !out_std) {
    set_error("absorber_mlp_get_normalization: bad argument");
    return ABS_ERR_ARG;
  }
  const MlpImpl& M = w->impl;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(in_mean, M.imean, sizeof(float) * M.cfg.n_in, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(in_std, M.istd, sizeof(float) * M.cfg.n_in, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(out_mean, M.omean, sizeof(float) * M.cfg.n_out, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(out_std, M.ostd, sizeof(float) * M.cfg.n_out, hipMemcpyDeviceToHost));
  return ABS_OK;
}

int absorber_mlp_fit_normalization(absorber_mlp* w, const float* X_dev, const float* T_dev, int64_t n,
                                   void* stream) {
  if (!w || !X_dev || !T_dev || n < 1) {
    set_error("absorber_mlp_fit_normalization: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(absorber::k_colstats, dim3(1), dim3(64), 0, st, X_dev, (long long)n, M.cfg.n_in, M.imean,
                     M.istd);
  hipLaunchKernelGGL(absorber::k_colstats, dim3(absorber::nblk(M.cfg.n_out, 64)), dim3(64), 0, st, T_dev,
                     (long long)n, M.cfg.n_out, M.omean, M.ostd);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

int absorber_mlp_forward(absorber_mlp* w, const float* X_dev, int64_t n, float* Y_dev, void* stream) {
  if (!w || !X_dev || !Y_dev || n < 0) {
    set_error("absorber_mlp_forward: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  hipStream_t st = as_stream(stream);
  const int no = M.cfg.n_out;
  for (long long b0 = 0; b0 < n; b0 += M.cfg.max_batch) {
    const int B = (int)std::min<long long>(M.cfg.max_batch, n - b0);
    int rc = M.gather(X_dev, nullptr, nullptr, b0, B, st);
    if (!rc) rc = M.forward(B, false, Y_dev + b0 * no, no, B, M.omean, M.ostd, st);
    if (rc) return rc;
  }
  return ABS_OK;
}

int absorber_mlp_loss_grad(absorber_mlp* w, const float* X_dev, const float* T_dev, int64_t n, float* grad_dev,
                           double* loss_host, void* stream) {
  if (!w || !X_dev || !T_dev || !grad_dev) {
    set_error("absorber_mlp_loss_grad: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  if (!check_batch(M, n, true)) return ABS_ERR_ARG;
  hipStream_t st = as_stream(stream);
  const int B = (int)n;
  int rc = M.gather(X_dev, T_dev, nullptr, 0, B, st);
  if (!rc) rc = M.forward(B, true, M.Y, M.nout[M.L - 1], B, nullptr, nullptr, st);
  int np = 0;
  if (!rc) rc = M.backward(B, st, &np);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(grad_dev, M.g, sizeof(float) * M.nparam, hipMemcpyDeviceToDevice, st));
  const double se = M.loss_from_parts(np, st);
  if (loss_host) *loss_host = se / ((double)B * M.cfg.n_out);
  return ABS_OK;
}

int absorber_mlp_adam_step(absorber_mlp* w, const float* grad_dev, const absorber_mlp_train_options* opts,
                           double lr, void* stream) {
  if (!w || !grad_dev || !opts) {
    set_error("absorber_mlp_adam_step: bad argument");
    return ABS_ERR_ARG;
  }
  return w->impl.adam(grad_dev, lr, *opts, as_stream(stream));
}

int absorber_mlp_train(absorber_mlp* w, const float* X_dev, const float* T_dev, int64_t n,
                       const absorber_mlp_train_options* opts, absorber_mlp_train_result* res) {
  if (!w || !X_dev || !T_dev || !opts || opts->epochs < 0) {
    set_error("absorber_mlp_train: bad argument");
    return ABS_ERR_ARG;
  }
  MlpImpl& M = w->impl;
  if (!check_batch(M, opts->batch, true)) return ABS_ERR_ARG;
  if (n < opts->batch) {
    set_error("absorber_mlp_train: fewer samples than one batch");
    return ABS_ERR_ARG;
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = nullptr;
  if (M.perm_cap < n) {
    if (M.perm_h) (void)hipHostFree(M.perm_h);
    M.perm_h = nullptr;
    HIP_TRY(hipHostMalloc((void**)&M.perm_h, sizeof(int) * n));
    HIP_TRY(M.dal(&M.perm, n));
    M.perm_cap = n;
  }
  int rc = absorber_mlp_fit_normalization(w, X_dev, T_dev, n, st);
  if (rc) return rc;
  const int B = opts->batch;
  const long long per_epoch = n / B;  // the remainder of each shuffled epoch is dropped
  const long long total = per_epoch * opts->epochs;
  uint64_t s = opts->seed;
  std::vector<int> idx((size_t)n);
  for (long long i = 0; i < n; ++i) idx[(size_t)i] = (int)i;
  long long step = 0;
  double last = NAN;
  for (int ep = 0; ep < opts->epochs; ++ep) {
    for (long long i = n - 1; i > 0; --i) {  // Fisher-Yates
      const long long j = (long long)(absorber::splitmix64(s) % (uint64_t)(i + 1));
      std::swap(idx[(size_t)i], idx[(size_t)j]);
    }
    HIP_TRY(hipStreamSynchronize(st));  // the previous epoch's gathers have read perm
    memcpy(M.perm_h, idx.data(), sizeof(int) * n);
    HIP_TRY(hipMemcpyAsync(M.perm, M.perm_h, sizeof(int) * n, hipMemcpyHostToDevice, st));
    double ep_loss = 0.0;
    for (long long k = 0; k < per_epoch; ++k, ++step) {
      const double lr = opts->cosine ? 0.5 * opts->lr * (1.0 + cos(3.14159265358979323846 * (double)step / (double)total)) : opts->lr;
      rc = M.gather(X_dev, T_dev, M.perm, k * B, B, st);
      if (!rc) rc = M.forward(B, true, M.Y, M.nout[M.L - 1], B, nullptr, nullptr, st);
      int np = 0;
      if (!rc) rc = M.backward(B, st, &np);
      if (!rc) rc = M.adam(M.g, lr, *opts, st);
      if (rc) return rc;
      if (k == per_epoch - 1) ep_loss = M.loss_from_parts(np, st) / ((double)B * M.cfg.n_out);
    }
    last = ep_loss;
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (res) {
    res->final_loss = last;
    res->steps = step;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return ABS_OK;
}

}  // extern "C"

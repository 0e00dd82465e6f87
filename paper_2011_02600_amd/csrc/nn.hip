// Kernels of the learned surrogate (a spectral neural operator trained on the
// solver's own seismograms): a batched, strided BF16 matrix-core GEMM with
// FP32 accumulation, which carries every contraction of the forward and
// backward passes (spectral transforms, per-mode channel mixing, pointwise
// channel mixing, the trace head), and the small elementwise and reduction
// kernels around it.  C ABI in include/sbp_nn.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/sbp_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for M x N x K with arbitrary
// element strides.  A 256-thread block computes a 64 x 64 tile of C as a 2 x 2
// arrangement of waves, each wave 32 x 32 = 2 x 2 matrix-core tiles of
// 16 x 16 x 32 (bf16 inputs, fp32 accumulators).  Operands are read as fp32,
// rounded to bf16 (round to nearest even) and staged in LDS per K-step of 32:
// As[m][k] and Bs[n][k], so that a lane's eight consecutive k values are one
// 16-byte LDS read.  Lane l of a 16 x 16 x 32 tile supplies A row l % 16 and
// B column l % 16 at k = 8 (l / 16) .. 8 (l / 16) + 7, and receives C rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
constexpr int BM = 64, BN = 64, BK = 32, KP = BK + 8;  // KP: padded row (bf16), 80 bytes

struct GemmArgs {
  int M, N, K;
  float alpha, beta;
  const float* A;
  long long sAb, sAm, sAk;
  const float* B;
  long long sBb, sBk, sBn;
  float* C;
  long long sCb, sCm, sCn;
};

__global__ __launch_bounds__(256) void gemm_kernel(const GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM * KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN * KP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long long b = blockIdx.z;
  const float* A = g.A + b * g.sAb;
  const float* B = g.B + b * g.sBb;
  float* C = g.C + b * g.sCb;
  // staging order: the unit-stride index runs fastest across threads
  const bool a_kfast = g.sAk == 1 || g.sAm != 1;
  const bool b_nfast = g.sBn == 1 || g.sBk != 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / 256; ++r) {
      const int e = tid + r * 256;
      const int mm = a_kfast ? e / BK : e % BM;
      const int kk = a_kfast ? e % BK : e / BM;
      const int m = m0 + mm, k = k0 + kk;
      const float v = (m < g.M && k < g.K) ? A[m * g.sAm + k * g.sAk] : 0.f;
      As[mm * KP + kk] = (__bf16)v;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / 256; ++r) {
      const int e = tid + r * 256;
      const int nn = b_nfast ? e % BN : e / BK;
      const int kk = b_nfast ? e / BN : e % BK;
      const int n = n0 + nn, k = k0 + kk;
      const float v = (n < g.N && k < g.K) ? B[k * g.sBk + n * g.sBn] : 0.f;
      Bs[nn * KP + kk] = (__bf16)v;
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 32 + i * 16 + (lane & 15);
      af[i] = *reinterpret_cast<const bf16x8*>(&As[row * KP + kq]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + j * 16 + (lane & 15);
      bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[col * KP + kq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + t;
        if (m < g.M && n < g.N) {
          float* c = C + m * g.sCm + n * g.sCn;
          const float v = g.alpha * acc[i][j][t];
          *c = g.beta != 0.f ? v + g.beta * *c : v;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// GELU, tanh form: gelu(z) = z/2 (1 + tanh(s (z + 0.044715 z^3))), s = sqrt(2/pi)
__device__ __forceinline__ float gelu(float z) {
  const float s = 0.7978845608028654f;
  return 0.5f * z * (1.f + tanhf(s * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float s = 0.7978845608028654f;
  const float u = s * (z + 0.044715f * z * z * z);
  const float t = tanhf(u);
  return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * s * (1.f + 3.f * 0.044715f * z * z);
}

__global__ void bias_act_kernel(int S, int C, long long P, const float* k, const float* u, const float* bias,
                                float* z, float* h, int act) {
  const long long n = (long long)S * C * P;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)((e / P) % C);
    const float v = (k ? k[e] : 0.f) + (u ? u[e] : 0.f) + (bias ? bias[c] : 0.f);
    if (z) z[e] = v;
    h[e] = act ? gelu(v) : v;
  }
}

__global__ void act_bwd_kernel(long long n, const float* z, const float* dh, float* dz, int act) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    dz[e] = act ? dh[e] * gelu_grad(z[e]) : dh[e];
}

// out[c] (+)= sum over s, p of x[s][c][p] (times w[s][p] if w): one block per
// channel, fixed-order tree reduction (deterministic)
__global__ __launch_bounds__(1024) void channel_sum_kernel(int S, int C, long long P, const float* x, const float* w,
                                                           float* out, int accumulate) {
  __shared__ double red[1024];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) {
    const float* xs = x + ((long long)s * C + c) * P;
    const float* ws = w ? w + (long long)s * P : nullptr;
    for (long long p = threadIdx.x; p < P; p += blockDim.x) acc += ws ? (double)xs[p] * ws[p] : (double)xs[p];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = (float)(accumulate ? out[c] + red[0] : red[0]);
}

// h[s][c][p] = w[c] x[s][p] + b[c]
__global__ void lift_kernel(int S, int C, long long P, const float* x, const float* w, const float* b, float* h) {
  const long long n = (long long)S * C * P;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long p = e % P;
    const int c = (int)((e / P) % C);
    const int s = (int)(e / ((long long)C * P));
    h[e] = w[c] * x[(long long)s * P + p] + b[c];
  }
}

// f[s][r][c] = h[s][c][pos[r]];  backward: dh[s][c][pos[r]] += df[s][r][c]
// (one thread per (s, c); the receivers are visited in order, so repeated
// positions accumulate deterministically)
__global__ void gather_kernel(int S, int C, long long P, int R, const int* pos, const float* h, float* f) {
  const long long n = (long long)S * R * C;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int r = (int)((e / C) % R);
    const int s = (int)(e / ((long long)C * R));
    f[e] = h[((long long)s * C + c) * P + pos[r]];
  }
}

__global__ void scatter_kernel(int S, int C, long long P, int R, const int* pos, const float* df, float* dh) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * C) return;
  const int c = e % C, s = e / C;
  for (int r = 0; r < R; ++r) dh[((long long)s * C + c) * P + pos[r]] += df[((long long)s * R + r) * C + c];
}

// y[s][i] += b[i] for the rows of a (S, n) array
__global__ void add_rows_kernel(int S, long long n, const float* b, float* y) {
  const long long tot = (long long)S * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x)
    y[e] += b[e % n];
}

// out[i] (+)= sum over rows s of x[s][i]
__global__ void sum_rows_kernel(int S, long long n, const float* x, float* out, int accumulate) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int s = 0; s < S; ++s) a += x[(long long)s * n + i];
    out[i] = accumulate ? out[i] + a : a;
  }
}

// dy = scale (y - t); per-block partial sums of (y - t)^2 in double
__global__ __launch_bounds__(256) void mse_kernel(long long n, const float* y, const float* t, float* dy, float scale,
                                                  double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const float d = y[e] - t[e];
    if (dy) dy[e] = scale * d;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(long long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void axpy_kernel(long long n, float a, const float* x, float* y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

int blocks_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 1 << 16); }

// ---- allocation-free misfit (sbp_nn_mse_noalloc) ------------------------------
// Its scratch lives in a file-scope device array (one copy per GPU, held
// until the process ends): kMseMaxParts partial sums, one per chunk of
// kMseChunk elements, then the total.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): it
// uses the device address hipGetSymbolAddress returns for the current GPU.
constexpr int kMseChunk = 1024;
constexpr int kMseMaxParts = 65536;
static __device__ __align__(256) double scratch[kMseMaxParts + 1];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current GPU (looked up once per GPU);
// null (error text set) on failure
double* scratch_on_current_device(char* err, std::size_t nerr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    snprintf(err, nerr, "no usable current device (%s)", hipGetErrorString(e));
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      snprintf(err, nerr, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}

// part[b] = sum over elements [b chunk, (b + 1) chunk) of (y - t)^2, dy =
// scale (y - t); 256 threads per chunk, fixed-order tree reduction
__global__ __launch_bounds__(256) void mse_chunk_kernel(long long n, const float* y, const float* t, float* dy,
                                                        float scale, long long chunk, double* part) {
  __shared__ double red[256];
  const long long e0 = (long long)blockIdx.x * chunk;
  const long long e1 = min(n, e0 + chunk);
  double acc = 0.0;
  for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const float d = y[e] - t[e];
    if (dy) dy[e] = scale * d;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of part[0 .. nparts-1] (one block, fixed order)
__global__ __launch_bounds__(1024) void sum_parts_kernel(int nparts, const double* part, double* out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

thread_local char g_nn_err[256] = "";

int nn_fail(const char* msg) {
  snprintf(g_nn_err, sizeof(g_nn_err), "%s", msg);
  return SBP_NN_EINVAL;
}

int nn_status() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(g_nn_err, sizeof(g_nn_err), "HIP error: %s", hipGetErrorString(e));
    return SBP_NN_EHIP;
  }
  return SBP_NN_OK;
}

}  // namespace

extern "C" {

const char* sbp_nn_last_error(void) { return g_nn_err; }

int sbp_nn_gemm(int batch, int M, int N, int K, float alpha, const float* A, long long sAb, long long sAm,
                long long sAk, const float* B, long long sBb, long long sBk, long long sBn, float beta, float* C,
                long long sCb, long long sCm, long long sCn, void* stream) {
  if (batch < 0 || M < 0 || N < 0 || K < 0) return nn_fail("negative size");
  if (batch == 0 || M == 0 || N == 0) return SBP_NN_OK;
  if (!A || !B || !C) return nn_fail("NULL operand");
  if (batch > 65535) return nn_fail("batch must be <= 65535");
  if ((M + BM - 1) / BM > 65535) return nn_fail("M too large");
  GemmArgs g{M, N, K, alpha, beta, A, sAb, sAm, sAk, B, sBb, sBk, sBn, C, sCb, sCm, sCn};
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, (hipStream_t)stream, g);
  return nn_status();
}

int sbp_nn_bias_act(int S, int C, long long P, const float* k, const float* u, const float* bias, float* z, float* h,
                    int act, void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || !h) return nn_fail("invalid bias_act arguments");
  const long long n = (long long)S * C * P;
  if (n == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, S, C, P, k, u, bias, z,
                     h, act);
  return nn_status();
}

int sbp_nn_act_bwd(long long n, const float* z, const float* dh, float* dz, int act, void* stream) {
  if (n < 0 || !dh || !dz || (act && !z)) return nn_fail("invalid act_bwd arguments");
  if (n == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(act_bwd_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, n, z, dh, dz, act);
  return nn_status();
}

int sbp_nn_channel_sum(int S, int C, long long P, const float* x, const float* w, float* out, int accumulate,
                       void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || !x || !out) return nn_fail("invalid channel_sum arguments");
  hipLaunchKernelGGL(channel_sum_kernel, dim3(C), dim3(1024), 0, (hipStream_t)stream, S, C, P, x, w, out, accumulate);
  return nn_status();
}

int sbp_nn_lift(int S, int C, long long P, const float* x, const float* w, const float* b, float* h, void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || !x || !w || !b || !h) return nn_fail("invalid lift arguments");
  const long long n = (long long)S * C * P;
  if (n == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(lift_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, S, C, P, x, w, b, h);
  return nn_status();
}

int sbp_nn_gather(int S, int C, long long P, int R, const int* pos, const float* h, float* f, void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || R <= 0 || !pos || !h || !f) return nn_fail("invalid gather arguments");
  const long long n = (long long)S * R * C;
  if (n == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, S, C, P, R, pos, h, f);
  return nn_status();
}

int sbp_nn_scatter(int S, int C, long long P, int R, const int* pos, const float* df, float* dh, void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || R <= 0 || !pos || !df || !dh) return nn_fail("invalid scatter arguments");
  if (S == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(scatter_kernel, dim3((S * C + 255) / 256), dim3(256), 0, (hipStream_t)stream, S, C, P, R, pos,
                     df, dh);
  return nn_status();
}

int sbp_nn_add_rows(int S, long long n, const float* b, float* y, void* stream) {
  if (S < 0 || n <= 0 || !b || !y) return nn_fail("invalid add_rows arguments");
  if (S == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(add_rows_kernel, dim3(blocks_for((long long)S * n)), dim3(256), 0, (hipStream_t)stream, S, n, b,
                     y);
  return nn_status();
}

int sbp_nn_sum_rows(int S, long long n, const float* x, float* out, int accumulate, void* stream) {
  if (S < 0 || n <= 0 || !x || !out) return nn_fail("invalid sum_rows arguments");
  hipLaunchKernelGGL(sum_rows_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, S, n, x, out,
                     accumulate);
  return nn_status();
}

int sbp_nn_mse(long long n, const float* y, const float* t, float* dy, float scale, double* part, double* loss,
               void* stream) {
  if (n <= 0 || !y || !t || !part || !loss) return nn_fail("invalid mse arguments");
  hipLaunchKernelGGL(mse_kernel, dim3(SBP_NN_MSE_PARTS), dim3(256), 0, (hipStream_t)stream, n, y, t, dy, scale, part);
  double h[SBP_NN_MSE_PARTS];
  hipError_t e = hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return nn_status();
  double s = 0.0;
  for (int i = 0; i < SBP_NN_MSE_PARTS; ++i) s += h[i];
  *loss = 0.5 * s;
  return nn_status();
}

int sbp_nn_mse_noalloc(long long n, const float* y, const float* t, float* dy, float scale, double* loss,
                       void* stream) {
  if (n <= 0 || !y || !t || !loss) return nn_fail("invalid mse arguments");
  const long long nparts = (n + kMseChunk - 1) / kMseChunk;
  if (nparts > kMseMaxParts) {
    snprintf(g_nn_err, sizeof(g_nn_err),
             "n = %lld exceeds the static scratch of sbp_nn_mse_noalloc: at most %lld elements (%d partial sums of "
             "%d); use sbp_nn_mse with a workspace",
             n, (long long)kMseMaxParts * kMseChunk, kMseMaxParts, kMseChunk);
    return SBP_NN_EINVAL;
  }
  double* sc = scratch_on_current_device(g_nn_err, sizeof(g_nn_err));
  if (!sc) return SBP_NN_EHIP;
  hipStream_t st = (hipStream_t)stream;
  // every partial is written before it is read: nothing to clear
  hipLaunchKernelGGL(mse_chunk_kernel, dim3((unsigned)nparts), dim3(256), 0, st, n, y, t, dy, scale,
                     (long long)kMseChunk, sc);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(1024), 0, st, (int)nparts, sc, sc + kMseMaxParts);
  double h = 0.0;
  hipError_t e = hipMemcpyAsync(&h, sc + kMseMaxParts, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return nn_status();
  *loss = 0.5 * h;
  return nn_status();
}

int sbp_nn_adam(long long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                int step, void* stream) {
  if (n <= 0 || !p || !g || !m || !v || step < 1) return nn_fail("invalid adam arguments");
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, n, p, g, m, v, lr, b1, b2,
                     eps, c1, c2);
  return nn_status();
}

int sbp_nn_axpy(long long n, float a, const float* x, float* y, void* stream) {
  if (n < 0 || !x || !y) return nn_fail("invalid axpy arguments");
  if (n == 0) return SBP_NN_OK;
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, n, a, x, y);
  return nn_status();
}

}  // extern "C"

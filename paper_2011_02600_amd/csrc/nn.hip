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
//
// Each K-step's operand tiles (64 rows x 32 k, 8 values per thread) are
// loaded into registers while the previous step's matrix-core work runs and
// then stored to the other of two LDS buffers (one barrier per step).  A tile
// is loaded 16 bytes at a time along its unit-stride index when that index is
// k (MODE 1) or the row index (MODE 2) and the addresses are 16-byte aligned
// (checked on the host), else one element at a time along the unit-stride
// index (MODE 0).
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

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// tile rows r0 .. r0+63 (m of A, n of B) x k0 .. k0+31 of an operand with
// element strides s_row, s_k, R rows and K columns in all
template <int MODE>
__device__ __forceinline__ void gemm_load(const float* X, long long s_row, long long s_k, int R, int K, int r0,
                                          int k0, int tid, bool kfast, float v[8]) {
  if constexpr (MODE == 1) {  // float4 along k (s_k == 1)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + 256 * h, r = r0 + (g >> 3), k = k0 + (g & 7) * 4;
      if (r < R && k + 3 < K) {
        const f32x4v x = *reinterpret_cast<const f32x4v*>(X + r * s_row + k);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * h + i] = x[i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * h + i] = (r < R && k + i < K) ? X[r * s_row + (k + i)] : 0.f;
      }
    }
  } else if constexpr (MODE == 2) {  // float4 along the row index (s_row == 1)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + 256 * h, k = k0 + (g >> 4), r = r0 + (g & 15) * 4;
      if (k < K && r + 3 < R) {
        const f32x4v x = *reinterpret_cast<const f32x4v*>(X + k * s_k + r);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * h + i] = x[i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * h + i] = (k < K && r + i < R) ? X[k * s_k + (r + i)] : 0.f;
      }
    }
  } else {  // one element at a time, the unit-stride index fastest across threads
#pragma unroll
    for (int e8 = 0; e8 < 8; ++e8) {
      const int e = tid + 256 * e8;
      const int rr = kfast ? e / BK : e % 64;
      const int kk = kfast ? e % BK : e / 64;
      const int r = r0 + rr, k = k0 + kk;
      v[e8] = (r < R && k < K) ? X[r * s_row + k * s_k] : 0.f;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void gemm_store(__bf16* S, const float v[8], int tid, bool kfast) {
  if constexpr (MODE == 1) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + 256 * h, rr = g >> 3, kq = (g & 7) * 4;
      const bf16x4 w = {(__bf16)v[4 * h], (__bf16)v[4 * h + 1], (__bf16)v[4 * h + 2], (__bf16)v[4 * h + 3]};
      *reinterpret_cast<bf16x4*>(&S[rr * KP + kq]) = w;
    }
  } else if constexpr (MODE == 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + 256 * h, kk = g >> 4, rq = (g & 15) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) S[(rq + i) * KP + kk] = (__bf16)v[4 * h + i];
    }
  } else {
#pragma unroll
    for (int e8 = 0; e8 < 8; ++e8) {
      const int e = tid + 256 * e8;
      const int rr = kfast ? e / BK : e % 64;
      const int kk = kfast ? e % BK : e / 64;
      S[rr * KP + kk] = (__bf16)v[e8];
    }
  }
}

template <int AM, int BMODE>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * KP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long long b = blockIdx.z;
  const float* A = g.A + b * g.sAb;
  const float* B = g.B + b * g.sBb;
  float* C = g.C + b * g.sCb;
  // scalar staging order: the unit-stride index runs fastest across threads
  const bool a_kfast = g.sAk == 1 || g.sAm != 1;
  const bool b_kfast = !(g.sBn == 1 || g.sBk != 1);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  float ra[8], rb[8];
  gemm_load<AM>(A, g.sAm, g.sAk, g.M, g.K, m0, 0, tid, a_kfast, ra);
  gemm_load<BMODE>(B, g.sBn, g.sBk, g.N, g.K, n0, 0, tid, b_kfast, rb);
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // the buffer written here was last read two steps ago, before the
    // barrier of the previous step
    gemm_store<AM>(As[buf], ra, tid, a_kfast);
    gemm_store<BMODE>(Bs[buf], rb, tid, b_kfast);
    __syncthreads();
    if (k0 + BK < g.K) {  // the next step's tiles, in flight during this step's matrix-core work
      gemm_load<AM>(A, g.sAm, g.sAk, g.M, g.K, m0, k0 + BK, tid, a_kfast, ra);
      gemm_load<BMODE>(B, g.sBn, g.sBk, g.N, g.K, n0, k0 + BK, tid, b_kfast, rb);
    }
    const int kq = 8 * (lane >> 4);
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 32 + i * 16 + (lane & 15);
      af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][row * KP + kq]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + j * 16 + (lane & 15);
      bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][col * KP + kq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    buf ^= 1;
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

// staging mode of an operand (see gemm_kernel): 1 if k has unit stride, 2 if
// the row index has, each only when every 4-element group is 16-byte aligned
int gemm_mode(const float* X, long long sb, long long s_row, long long s_k) {
  const bool al = ((std::uintptr_t)X % 16) == 0 && sb % 4 == 0;
  if (al && s_k == 1 && s_row % 4 == 0) return 1;
  if (al && s_row == 1 && s_k % 4 == 0) return 2;
  return 0;
}

template <int AM>
void gemm_launch_b(int bm, dim3 grid, hipStream_t st, const GemmArgs& g) {
  if (bm == 1)
    hipLaunchKernelGGL((gemm_kernel<AM, 1>), grid, dim3(256), 0, st, g);
  else if (bm == 2)
    hipLaunchKernelGGL((gemm_kernel<AM, 2>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_kernel<AM, 0>), grid, dim3(256), 0, st, g);
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

// out[c] (+)= sum over s, p of x[s][c][p] (times w[s][p] if w), in two
// passes with fixed orders (deterministic): block (c, j) of the first sums
// slice j of channel c's S * P values (four interleaved double accumulators
// per thread, then a tree) into part[c * kChanSplit + j]; the second adds a
// channel's kChanSplit partial sums in order.
constexpr int kChanSplit = 64;

__global__ __launch_bounds__(256) void channel_part_kernel(int S, int C, long long P, const float* x, const float* w,
                                                           double* part) {
  __shared__ double red[256];
  const int c = blockIdx.x, j = blockIdx.y;
  const long long n = (long long)S * P;
  const long long per = (n + kChanSplit - 1) / kChanSplit;
  const long long e0 = (long long)j * per, e1 = e0 + per < n ? e0 + per : n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long e = e0 + threadIdx.x; e < e1; e += 4 * 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long f = e + (long long)u * 256;
      if (f < e1) {
        const long long s = f / P, p = f - s * P;
        const double v = x[(s * C + c) * P + p];
        acc[u] += w ? v * (double)w[s * P + p] : v;
      }
    }
  }
  red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)c * kChanSplit + j] = red[0];
}

__global__ void channel_sum_kernel(int C, const double* part, float* out, int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double v = 0.0;
  for (int j = 0; j < kChanSplit; ++j) v += part[(long long)c * kChanSplit + j];
  out[c] = (float)(accumulate ? out[c] + v : v);
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

// out[i] (+)= sum over rows s of x[s][i].  A block covers 32 columns with 8
// row lanes: lane g sums rows g, g + 8, g + 16, ... into four interleaved
// accumulators (loads in flight together), and the 8 lane sums of a column
// are added in lane order (a fixed order: the same result on every call).
__global__ __launch_bounds__(256) void sum_rows_kernel(int S, long long n, const float* x, float* out, int accumulate) {
  __shared__ float red[8][32];
  const int ci = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long i = blockIdx.x * 32LL + ci;
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  if (i < n) {
    int s = g;
    for (; s + 24 < S; s += 32) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += x[(long long)(s + 8 * u) * n + i];
    }
    for (; s < S; s += 8) a[0] += x[(long long)s * n + i];
  }
  red[g][ci] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  if (g == 0 && i < n) {
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) v += red[k][ci];
    out[i] = accumulate ? out[i] + v : v;
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
  const int am = gemm_mode(A, sAb, sAm, sAk), bm = gemm_mode(B, sBb, sBn, sBk);
  const hipStream_t st = (hipStream_t)stream;
  if (am == 1)
    gemm_launch_b<1>(bm, grid, st, g);
  else if (am == 2)
    gemm_launch_b<2>(bm, grid, st, g);
  else
    gemm_launch_b<0>(bm, grid, st, g);
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
                       double* part, void* stream) {
  if (S < 0 || C <= 0 || P <= 0 || !x || !out || !part) return nn_fail("invalid channel_sum arguments");
  if (C > 65535) return nn_fail("channel_sum: C must be <= 65535");
  const hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(channel_part_kernel, dim3(C, kChanSplit), dim3(256), 0, st, S, C, P, x, w, part);
  hipLaunchKernelGGL(channel_sum_kernel, dim3((C + 255) / 256), dim3(256), 0, st, C, part, out, accumulate);
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
  if ((n + 31) / 32 > 0x7fffffffLL) return nn_fail("sum_rows: n too large");
  hipLaunchKernelGGL(sum_rows_kernel, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, (hipStream_t)stream, S, n, x, out,
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

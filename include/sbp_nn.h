/*
 * sbp_nn.h -- C ABI of the surrogate kernels: the building blocks of a
 * spectral neural operator (a Fourier-neural-operator-style network with a
 * truncated cosine basis) that maps a material field to receiver traces and
 * is trained on traces the solver itself computes.  Not part of the paper's
 * method: a learned stand-in for the solver, which stays the fallback and
 * the reference the surrogate's error is measured against.
 *
 * Conventions: device pointers to fp32 arrays owned by the caller; sizes and
 * element strides in elements; every call is asynchronous on `stream` (a
 * hipStream_t cast to void*, NULL = null stream) unless stated otherwise;
 * every call returns SBP_NN_OK or a negative SBP_NN_E* code, with the text
 * of the last failure of the calling thread in sbp_nn_last_error().  The
 * library allocates no memory.
 */
#ifndef SBP_NN_H
#define SBP_NN_H

#ifdef __cplusplus
extern "C" {
#endif

enum { SBP_NN_OK = 0, SBP_NN_EINVAL = -1, SBP_NN_EHIP = -3 };
enum { SBP_NN_MSE_PARTS = 256 };

/*
 * C[b] = alpha A[b] B[b] + beta C[b] for b < batch, A M x K, B K x N, C M x N,
 * element (i, j) of A[b] at A + b sAb + i sAm + j sAk (likewise B, C), so any
 * transpose or batched/strided view is one call.  Operands are rounded to
 * bf16 (nearest even) and multiplied on the matrix cores (16 x 16 x 32 bf16
 * MFMA) with fp32 accumulation; C is fp32.  beta = 0 does not read C.
 * batch <= 65535, ceil(M / 64) <= 65535.
 */
int sbp_nn_gemm(int batch, int M, int N, int K, float alpha, const float* A, long long sAb, long long sAm,
                long long sAk, const float* B, long long sBb, long long sBk, long long sBn, float beta, float* C,
                long long sCb, long long sCm, long long sCn, void* stream);

/*
 * z = k + u + bias[c] (each of k, u, bias may be NULL) over an (S, C, P)
 * array, h = gelu(z) if act else z (tanh form of GELU); z may be NULL.
 */
int sbp_nn_bias_act(int S, int C, long long P, const float* k, const float* u, const float* bias, float* z, float* h,
                    int act, void* stream);

/* dz = dh gelu'(z) if act else dh, n values. */
int sbp_nn_act_bwd(long long n, const float* z, const float* dh, float* dz, int act, void* stream);

/*
 * out[c] = sum over s < S and p < P of x[s][c][p] (times w[s][p] if w is not
 * NULL), accumulated in double in a fixed order (the same result on every
 * call); added to out if accumulate.  part: caller-owned device workspace of
 * 64 * C doubles (partial sums), overwritten.  C <= 65535.
 */
int sbp_nn_channel_sum(int S, int C, long long P, const float* x, const float* w, float* out, int accumulate,
                       double* part, void* stream);

/* h[s][c][p] = w[c] x[s][p] + b[c] (the lifting layer). */
int sbp_nn_lift(int S, int C, long long P, const float* x, const float* w, const float* b, float* h, void* stream);

/* f[s][r][c] = h[s][c][pos[r]] for R receiver positions pos (device ints). */
int sbp_nn_gather(int S, int C, long long P, int R, const int* pos, const float* h, float* f, void* stream);

/* dh[s][c][pos[r]] += df[s][r][c] (the gather's transpose; dh not cleared). */
int sbp_nn_scatter(int S, int C, long long P, int R, const int* pos, const float* df, float* dh, void* stream);

/* y[s][i] += b[i] for an (S, n) array y. */
int sbp_nn_add_rows(int S, long long n, const float* b, float* y, void* stream);

/* out[i] = sum over s of x[s][i] (added to out if accumulate). */
int sbp_nn_sum_rows(int S, long long n, const float* x, float* out, int accumulate, void* stream);

/*
 * Mean-square misfit: dy = scale (y - t) (dy may be NULL) and *loss (host) =
 * 1/2 sum (y - t)^2, summed in double; part is device scratch of
 * SBP_NN_MSE_PARTS doubles.  Synchronises the stream.
 */
int sbp_nn_mse(long long n, const float* y, const float* t, float* dy, float scale, double* part, double* loss,
               void* stream);

/*
 * sbp_nn_mse without the workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): dy = scale (y - t) (dy may be NULL) and
 * *loss = 1/2 sum (y - t)^2, summed in double (per chunk of 1024 elements,
 * then over the chunks, both in a fixed order; equal to sbp_nn_mse up to
 * the order of the double sums).  Allocates nothing: its scratch is a
 * static device array of 65536 + 1 doubles (512 KiB per GPU, held until the
 * process ends), so n is at most 65536 * 1024 = 67108864 elements; larger n
 * is SBP_NN_EINVAL with a message naming the limit.  Calls on one GPU share
 * that array: calls that overlap in time on one GPU (other streams, other
 * threads) race and must not be issued.  Synchronises the stream.
 */
int sbp_nn_mse_noalloc(long long n, const float* y, const float* t, float* dy, float scale, double* loss,
                       void* stream);

/* One Adam step (Kingma & Ba) on n parameters, step >= 1 (bias correction). */
int sbp_nn_adam(long long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                int step, void* stream);

/* y += a x. */
int sbp_nn_axpy(long long n, float a, const float* x, float* y, void* stream);

/* Text of the last failure on the calling thread. */
const char* sbp_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif

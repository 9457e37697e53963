// Kernels of the layer-batched FP64 network forward (model_f64.hip), shared
// with the FP64 backward (grad_f64.hip).
#pragma once

#include "model.hpp"

namespace nnqs {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Previous-token input embeddings h[b*K + s][c] and the token of every row.
__global__ void k64_embed(ModelView M, const uint64_t *__restrict__ keys, int64_t B, int8_t *__restrict__ tok,
                          double *__restrict__ h);
// LayerNorm (eps 1e-5) of rows of width 64, one wave per row.
__global__ void k64_layernorm(const double *__restrict__ in, const double *__restrict__ g,
                              const double *__restrict__ b, int64_t rows, double *__restrict__ out);
// C[r][j] = epi(bias[j] + sum_k A[r][k] B[k][j]); B[k][j] = W[k*ldw + j], or
// W[j*ldw + k] with TB (the transposed weight, y W^T); EPI 0 stores, 1 adds
// to C, 2 stores GELU.
template <int EPI, bool TB = false>
__global__ void k64_gemm(const double *__restrict__ A, int lda, const double *__restrict__ W, int ldw,
                         const double *__restrict__ bias, int64_t M, int N, int Kd, double *__restrict__ C, int ldc);
// Causal attention of [B*K][64] rows, one wave per (configuration, head).
__global__ void k64_attention(const double *__restrict__ q, const double *__restrict__ k,
                              const double *__restrict__ v, int64_t B, int K, double scale, double *__restrict__ o);
// Output head: log-probability of each row's token (and the conditionals of position cpos).
__global__ void k64_head(ModelView M, const double *__restrict__ a, const int8_t *__restrict__ tok, int64_t B,
                         double *__restrict__ lp, int cpos, double *__restrict__ cond);
// log|psi| = 1/2 sum of the rows' log-probabilities; phase = b3 + z2 . w3.
__global__ void k64_finish(ModelView M, const double *__restrict__ lp, const double *__restrict__ z2, int64_t B,
                           double *__restrict__ logabs, double *__restrict__ phase);

__device__ __forceinline__ double gelu_f64(double v) { return 0.5 * v * (1.0 + erf(v * 0.70710678118654752440)); }

}  // namespace nnqs

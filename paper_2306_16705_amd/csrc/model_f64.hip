// FP64 network forward, layer by layer over batches of configurations (the
// ansatz of Section 3.1, Eq. 11 and Fig. 2, with the Eq. 12 mask and the
// phase MLP of Section 4.1).  Every step is a plain kernel over the rows of
// a whole batch: LayerNorm one wave per row, the dense layers an LDS-tiled
// FP64 MFMA product (64 x 64 output tile per block) with bias, GELU or
// residual-add epilogues, causal attention on FP64 MFMA one wave per
// (configuration, head).  Activations live in model-owned scratch between steps.
// The arithmetic is the FP64 definition of the network; only the summation
// order differs from a one-configuration-at-a-time evaluation.
#include <cmath>
#include <climits>
#include <vector>

#include "f64_kernels.hpp"

namespace nnqs {

constexpr int64_t kF64Batch = 4096;  // configurations per pass

// Tokens (previous-token input) and embeddings: h[b*K + s][c].
__global__ void k64_embed(ModelView M, const uint64_t *__restrict__ keys, int64_t B, int8_t *__restrict__ tok,
                          double *__restrict__ h) {
    const int K = M.K, d = M.d;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * K * d) return;
    const int64_t row = e / d;
    const int c = (int)(e - row * d);
    const int64_t b = row / K;
    const int s = (int)(row - b * K);
    Key x;
    x.lo = keys[2 * b];
    x.hi = keys[2 * b + 1];
    auto token = [&](int pos) {
        const int i = K - 1 - pos;  // position s holds spatial orbital K-1-s
        return key_bit(x, 2 * i) + 2 * key_bit(x, 2 * i + 1);
    };
    if (c == 0) tok[row] = (int8_t)token(s);
    const int prev = s == 0 ? 4 : token(s - 1);
    h[e] = M.w64[M.off.tok_emb + prev * d + c] + M.w64[M.off.pos_emb + (int64_t)s * d + c];
}

// LayerNorm (eps 1e-5) of rows of width 64: one wave per row, lane = column.
__global__ void __launch_bounds__(256) k64_layernorm(const double *__restrict__ in, const double *__restrict__ g,
                                                     const double *__restrict__ b, int64_t rows,
                                                     double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const double v = in[row * 64 + lane];
    double s = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const double mean = s / 64.0;
    double q = (v - mean) * (v - mean);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off, 64);
    const double r = 1.0 / sqrt(q / 64.0 + 1e-5);
    out[row * 64 + lane] = (v - mean) * r * g[lane] + b[lane];
}

// The same row statistics alone, st[row] = (mean, 1/sqrt(var + eps)), for
// products that normalise their A rows while staging them (gemm64_tile with
// NORM), which saves writing and re-reading the normalised rows.
__global__ void __launch_bounds__(256) k64_ln_stats(const double *__restrict__ in, int64_t rows,
                                                    double *__restrict__ st) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const double v = in[row * 64 + lane];
    double s = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const double mean = s / 64.0;
    double q = (v - mean) * (v - mean);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off, 64);
    if (lane == 0) {
        st[2 * row] = mean;
        st[2 * row + 1] = 1.0 / sqrt(q / 64.0 + 1e-5);
    }
}

// C[r][j] = epi(bias[j] + sum_k A[r][k] B[k][j]) for r < M, j < N, with
// B[k][j] = W[k][j], or W[j][k] with TB (products with a transposed weight in
// the backward); EPI 0 stores, 1 adds to C (residual), 2 stores GELU.  Block: 64 x 64 tile of C,
// four waves of 16 rows each, on v_mfma_f64_16x16x4_f64 (lane l holds
// A[l & 15][l >> 4] and B[l >> 4][l & 15]; accumulator register i of lane l
// holds row (l >> 4) + 4 i, column l & 15, unlike the BF16 16x16 variants);
// k in slices of 32 through LDS, the next slice's global loads in flight
// during the current slice's products.  FP64 throughout: only the summation
// order differs from a plain dot product.
// With NORM (Kd = 64) the A rows are LayerNorm inputs: each staged element
// becomes (a - mean) rstd g[k] + b[k] with the row's statistics from lnst
// (k64_ln_stats) and the scale and shift lng, lnb.  With STATS (EPI 1, N = 64,
// one column block) the wave holds all 64 columns of its 16 updated rows and
// also writes their LayerNorm statistics (mean, rstd) to stout, as
// k64_ln_stats would.
template <int EPI, bool TB, bool NORM = false, bool STATS = false>
__device__ __forceinline__ void gemm64_tile(const double *__restrict__ A, int lda, const double *__restrict__ W,
                                            int ldw, const double *__restrict__ bias, int64_t M, int N, int Kd,
                                            double *__restrict__ C, int ldc, int c0,
                                            const double *__restrict__ lnst = nullptr,
                                            const double *__restrict__ lng = nullptr,
                                            const double *__restrict__ lnb = nullptr,
                                            double *__restrict__ stout = nullptr) {
    constexpr int KS = 32;  // k per slice
    __shared__ double As[64][KS + 1];
    __shared__ double Ws[KS][64 + 1];
    __shared__ double Ln[NORM ? 4 * 64 : 1];  // mean and rstd of the tile's rows, then g and b
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = l & 15, lk = l >> 4;
    const int64_t r0 = (int64_t)blockIdx.y * 64;
    if constexpr (NORM) {  // read after the first barrier of the slice loop
        const int t = threadIdx.x & 63, part = threadIdx.x >> 6;
        const int64_t r = r0 + t;
        if (part == 0) Ln[t] = r < M ? lnst[2 * r] : 0.0;
        else if (part == 1) Ln[64 + t] = r < M ? lnst[2 * r + 1] : 0.0;
        else if (part == 2) Ln[128 + t] = lng[t];
        else Ln[192 + t] = lnb[t];
    }
    // slice loads: thread t takes A[r0 + (t >> 5) + 8 e][k0 + (t & 31)] and
    // W[k0 + (t >> 6) + 4 e][c0 + (t & 63)], e = 0..7 (coalesced rows); with
    // TB, W[c0 + (t >> 5) + 8 e][k0 + (t & 31)] into the slice's column
    const int at = threadIdx.x & 31, ar = threadIdx.x >> 5, wc = threadIdx.x & 63, wr = threadIdx.x >> 6;
    double pa[8], pw[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int64_t r = r0 + ar + 8 * e;
            pa[e] = (r < M && k0 + at < Kd) ? A[r * lda + k0 + at] : 0.0;
            if (TB) {
                const int cw = c0 + ar + 8 * e;
                pw[e] = (cw < N && k0 + at < Kd) ? W[(int64_t)cw * ldw + k0 + at] : 0.0;
            } else {
                const int kw = k0 + wr + 4 * e;
                pw[e] = (kw < Kd && c0 + wc < N) ? W[(int64_t)kw * ldw + c0 + wc] : 0.0;
            }
        }
    };
    f64x4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    load(0);
    for (int k0 = 0; k0 < Kd; k0 += KS) {
        __syncthreads();  // the previous slice is consumed
#pragma unroll
        for (int e = 0; e < 8; e++) {
            if constexpr (NORM) {
                const int rr = ar + 8 * e, kk = k0 + at;
                As[rr][at] = (pa[e] - Ln[rr]) * Ln[64 + rr] * Ln[128 + kk] + Ln[192 + kk];
            } else {
                As[ar + 8 * e][at] = pa[e];
            }
            if (TB) Ws[at][ar + 8 * e] = pw[e];
            else Ws[wr + 4 * e][wc] = pw[e];
        }
        __syncthreads();
        if (k0 + KS < Kd) load(k0 + KS);  // the next slice's loads overlap this slice's products
#pragma unroll
        for (int k4 = 0; k4 < KS; k4 += 4) {
            const double a = As[16 * w + lr][k4 + lk];
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ws[k4 + lk][cb * 16 + lr], acc[cb], 0, 0, 0);
        }
    }
    if constexpr (STATS) {
        static_assert(EPI == 1, "statistics of the updated residual rows");
        double nv[4][4];
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            const int c = cb * 16 + lr;
            const double bc = bias ? bias[c] : 0.0;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t r = r0 + 16 * w + lk + 4 * i;
                nv[cb][i] = 0.0;
                if (r < M) {
                    double *dst = C + r * ldc + c;
                    nv[cb][i] = *dst + (bc + acc[cb][i]);
                    *dst = nv[cb][i];
                }
            }
        }
        // row lk + 4 i of the wave: its 64 columns are cb * 16 + lr over the
        // 16 lanes lr of lane group lk
#pragma unroll
        for (int i = 0; i < 4; i++) {
            double sm = (nv[0][i] + nv[1][i]) + (nv[2][i] + nv[3][i]);
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) sm += __shfl_xor(sm, off, 16);
            const double mean = sm / 64.0;
            double q = 0.0;
#pragma unroll
            for (int cb = 0; cb < 4; cb++) q += (nv[cb][i] - mean) * (nv[cb][i] - mean);
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) q += __shfl_xor(q, off, 16);
            const int64_t r = r0 + 16 * w + lk + 4 * i;
            if (lr == 0 && r < M) {
                stout[2 * r] = mean;
                stout[2 * r + 1] = 1.0 / sqrt(q / 64.0 + 1e-5);
            }
        }
        return;
    }
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
        const int c = c0 + cb * 16 + lr;
        if (c >= N) continue;
        const double bc = bias ? bias[c] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t r = r0 + 16 * w + lk + 4 * i;
            if (r >= M) continue;
            const double v = bc + acc[cb][i];
            double *dst = C + r * ldc + c;
            if (EPI == 1) *dst += v;
            else if (EPI == 2) *dst = gelu_f64(v);
            else *dst = v;
        }
    }
}

// The products run four waves per SIMD (four 33.5 KB blocks per CU): the
// register budget that sets holds the tile without spills.
template <int EPI, bool TB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k64_gemm(const double *__restrict__ A, int lda, const double *__restrict__ W, int ldw, const double *__restrict__ bias,
         int64_t M, int N, int Kd, double *__restrict__ C, int ldc) {
    gemm64_tile<EPI, TB>(A, lda, W, ldw, bias, M, N, Kd, C, ldc, blockIdx.x * 64);
}

// Residual products h += A W + b of 64-wide rows whose inner dimension is
// fixed at compile time: the model width 64 (output projection) and the FFN
// width 256 (FFN output) of the networks measured here; no run-time bounds
// on k; the next LayerNorm's statistics of the updated rows go to stout.
template <int KD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k64_gemm_res(const double *__restrict__ A, int lda, const double *__restrict__ W, const double *__restrict__ bias,
             int64_t M, double *__restrict__ h, double *__restrict__ stout) {
    gemm64_tile<1, false, false, true>(A, lda, W, 64, bias, M, 64, KD, h, 64, 0, nullptr, nullptr, nullptr, stout);
}

// FFN output product h += f W2 + b2 over R rows (inner dimension F), and the
// LayerNorm statistics of the updated rows into lst.
static void ffn_out(const double *f, int ldf, const double *W2, const double *b2, int64_t R, int F, double *h,
                    double *lst, hipStream_t st) {
    const dim3 grid(1, (unsigned)((R + 63) / 64));
    if (F == 256) {
        hipLaunchKernelGGL(k64_gemm_res<256>, grid, dim3(256), 0, st, f, ldf, W2, b2, R, h, lst);
    } else {
        hipLaunchKernelGGL(k64_gemm<1>, grid, dim3(256), 0, st, f, ldf, W2, 64, b2, R, 64, F, h, 64);
        hipLaunchKernelGGL(k64_ln_stats, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, st, h, R, lst);
    }
}

// FFN input product of LayerNorm(h) (statistics lnst, scale and shift lng,
// lnb) without the normalised rows in memory.
template <int EPI>
__global__ void __launch_bounds__(256) k64_gemm_ln(const double *__restrict__ h, const double *__restrict__ W, int ldw,
                                                   const double *__restrict__ bias, int64_t M, int N,
                                                   double *__restrict__ C, int ldc, const double *__restrict__ lnst,
                                                   const double *__restrict__ lng, const double *__restrict__ lnb) {
    gemm64_tile<EPI, false, true>(h, 64, W, ldw, bias, M, N, 64, C, ldc, blockIdx.x * 64, lnst, lng, lnb);
}

// Q, K and V of LayerNorm(h) in one launch: column block x = 0, 1, 2 of the
// grid takes the weight and bias at W + x ws, bias + x ws (the layer block
// keeps W_q, b_q, W_k, b_k, W_v, b_v at equal strides) and writes C + x cs.
__global__ void __launch_bounds__(256) k64_gemm_qkv(const double *__restrict__ h, const double *__restrict__ W,
                                                    const double *__restrict__ bias, int64_t ws, int64_t M,
                                                    double *__restrict__ C, int64_t cs,
                                                    const double *__restrict__ lnst, const double *__restrict__ lng,
                                                    const double *__restrict__ lnb) {
    const int x = blockIdx.x;
    gemm64_tile<0, false, true>(h, 64, W + x * ws, 64, bias + x * ws, M, 64, 64, C + x * cs, 64, 0, lnst, lng,
                                lnb);
}

// Causal attention on FP64 MFMA: one wave per (configuration, head), the four
// heads of one configuration per block; q, k, v and the output are [B*K][64]
// with head hh in columns 16 hh .. 16 hh + 15.  Per block of 16 queries:
// S = Q K^T in 16 x 16 x 4 tiles (accumulator register i of lane l holds
// query (l >> 4) + 4 i, key l & 15 of the tile), the softmax of each query
// row over the 16 lanes that hold it (the largest score, then one
// exponential per key), P through LDS into the A-operand layout, O = P V.
// Rows at or beyond K read as zero and are never written.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k64_attention(const double *__restrict__ q, const double *__restrict__ k, const double *__restrict__ v, int64_t B, int K,
              double scale, double *__restrict__ o) {
    __shared__ double Ps[4][16][64 + 1];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = l & 15, lk = l >> 4;
    const int64_t g = (int64_t)blockIdx.x * 4 + w;
    if (g >= B * 4) return;  // wave-uniform; the kernel has no block barrier
    const int64_t b = g >> 2;
    const int hh = (int)(g & 3);
    const double *qh = q + b * K * 64 + hh * 16, *kh = k + b * K * 64 + hh * 16, *vh = v + b * K * 64 + hh * 16;
    auto ld = [&](const double *base, int s, int c) { return s < K ? base[(int64_t)s * 64 + c] : 0.0; };
    // Four adjacent head columns of row s (lane lk's share of the score
    // product's contraction, column 4 lk + k4): one 32-byte load.
    auto ld4 = [&](const double *base, int s) {
        return s < K ? *reinterpret_cast<const f64x4 *>(base + (int64_t)s * 64 + 4 * lk) : f64x4{0.0, 0.0, 0.0, 0.0};
    };
    // B operands: K^T tiles kf[kb][k4] = K[16 kb + lr][4 lk + k4]; the V tiles
    // V[4 kk + lk][lr] are read where the P V product takes them
    f64x4 kf[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) kf[kb] = ld4(kh, kb * 16 + lr);
    double(*P)[64 + 1] = Ps[w];
#pragma unroll
    for (int qb = 0; qb < 4; qb++) {
        const f64x4 qf = ld4(qh, qb * 16 + lr);
        f64x4 st[4];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            st[kb] = f64x4{0.0, 0.0, 0.0, 0.0};
            if (kb <= qb)
#pragma unroll
                for (int k4 = 0; k4 < 4; k4++)
                    st[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(qf[k4], kf[kb][k4], st[kb], 0, 0, 0);
        }
        // key 16 kb + lr is visible to query 16 qb + lk + 4 i when kb < qb, or kb == qb and lr <= lk + 4 i
        double mx[4], den[4], rden[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            mx[i] = -INFINITY;
#pragma unroll
            for (int kb = 0; kb <= qb; kb++)
                if (kb < qb || lr <= lk + 4 * i) mx[i] = fmax(mx[i], st[kb][i]);
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) mx[i] = fmax(mx[i], __shfl_xor(mx[i], off, 16));
            den[i] = 0.0;
#pragma unroll
            for (int kb = 0; kb < 4; kb++) {
                const double p =
                    (kb < qb || (kb == qb && lr <= lk + 4 * i)) ? exp((st[kb][i] - mx[i]) * scale) : 0.0;
                st[kb][i] = p;
                den[i] += p;
            }
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) den[i] += __shfl_xor(den[i], off, 16);
            rden[i] = 1.0 / den[i];
        }
#pragma unroll
        for (int kb = 0; kb < 4; kb++)
#pragma unroll
            for (int i = 0; i < 4; i++) P[lk + 4 * i][kb * 16 + lr] = st[kb][i] * rden[i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f64x4 ot = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4 * (qb + 1); kk++)
            ot = __builtin_amdgcn_mfma_f64_16x16x4f64(P[lr][4 * kk + lk], ld(vh, 4 * kk + lk, lr), ot, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int s = qb * 16 + lk + 4 * i;
            if (s < K) o[(b * K + s) * 64 + hh * 16 + lr] = ot[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Output head with the logit bias, the mask (Eq. 12, read with the lower
// bound too) and the log-probability of the actual token: one wave per
// (config, position).
// With `cond`, the masked conditional log-probabilities of all four tokens at
// position cpos are also written to cond[b][4] (batch sampling).
__global__ void __launch_bounds__(256) k64_head(ModelView M, const double *__restrict__ a,
                                                const int8_t *__restrict__ tok, int64_t B, double *__restrict__ lp,
                                                int cpos, double *__restrict__ cond) {
    // lane = model column (d = 64)
    const int K = M.K;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= B * K) return;  // wave-uniform
    const int64_t b = row / K;
    const int s = (int)(row - b * K);
    // electrons placed before position s (lanes r < s hold token r)
    const int tr = lane < s ? tok[b * K + lane] : 0;
    const int up = __popcll(__ballot(tr & 1)), dn = __popcll(__ballot(tr >> 1));
    const double *W = M.w64;
    const double av = a[row * 64 + lane];
    double z[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        double v = av * W[M.off.head_w + lane * 4 + t];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        z[t] = v;
    }
    if (lane != 0) return;
    const int rem = K - 1 - s, orb = K - 1 - s;
    bool ok[4];
    double mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        z[t] += W[M.off.head_b + t] + W[M.off.bias + orb * 4 + t];
        const int bu = t & 1, bd = t >> 1;
        ok[t] = (up + bu <= M.n_up) && (dn + bd <= M.n_dn) && (M.n_up - up - bu <= rem) && (M.n_dn - dn - bd <= rem);
        if (ok[t] && z[t] > mx) mx = z[t];
    }
    double den = 0.0;
#pragma unroll
    for (int t = 0; t < 4; t++)
        if (ok[t]) den += exp(z[t] - mx);
    const int ts = tok[row];
    const double lden = log(den);
    lp[row] = ok[ts] ? (z[ts] - mx) - lden : -INFINITY;
    if (cond && s == cpos)
#pragma unroll
        for (int t = 0; t < 4; t++) cond[b * 4 + t] = ok[t] ? (z[t] - mx) - lden : -INFINITY;
}

// First phase layer from the occupation bits: z1[b][j] = GELU(b1[j] + sum
// over set bits p of W1[p][j]).
__global__ void k64_phase1(ModelView M, const uint64_t *__restrict__ keys, int64_t B, double *__restrict__ z1) {
    const int P = M.P;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * P) return;
    const int64_t b = e / P;
    const int j = (int)(e - b * P);
    Key x;
    x.lo = keys[2 * b];
    x.hi = keys[2 * b + 1];
    double acc = M.w64[M.off.ph_b1 + j];
    for (int p = 0; p < 2 * M.K; p++)
        if (key_bit(x, p)) acc += M.w64[M.off.ph_w1 + (int64_t)p * P + j];
    z1[e] = gelu_f64(acc);
}

// Per configuration: log|psi| = 1/2 sum_s lp, phase = b3 + z2 . w3 (one wave
// each, fixed-order lane sums).
__global__ void __launch_bounds__(256) k64_finish(ModelView M, const double *__restrict__ lp,
                                                  const double *__restrict__ z2, int64_t B,
                                                  double *__restrict__ logabs, double *__restrict__ phase) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= B) return;
    double s = 0.0;
    for (int t = lane; t < M.K; t += 64) s += lp[b * M.K + t];
    double ph = 0.0;
    for (int i = lane; i < M.P; i += 64) ph += z2[b * M.P + i] * M.w64[M.off.ph_w3 + i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        ph += __shfl_xor(ph, off, 64);
    }
    if (lane == 0) {
        logabs[b] = 0.5 * s;
        phase[b] = M.w64[M.off.ph_b3] + ph;
    }
}

// ------------------------------------------------ prefix reuse in FP64
// Cache of a configuration's forward for the prefix-reusing evaluation of its
// connections: per configuration [L][2][K][64] doubles, every layer's keys
// then values (all heads, as the attention used them), and pre[K + 1] with
// pre[s] = sum_{t < s} log pi_t.  By causality of the attention and of the
// autoregressive product of Eq. 8, a connected x' whose first changed
// position is s0 has the same rows s <= s0 as its sample, so its forward can
// start at row s0 from the cache.
__global__ void k64_cache_kv(const double *__restrict__ kk, const double *__restrict__ v, int64_t B, int K, int l,
                             int L, double *__restrict__ kvc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)K * 64;
    if (e >= B * per) return;
    const int64_t b = e / per, r = e - b * per;
    double *dst = kvc + ((b * L + l) * 2) * per + r;
    dst[0] = kk[e];
    dst[per] = v[e];
}

__global__ void k64_prefix(const double *__restrict__ lp, int64_t B, int K, double *__restrict__ pre) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int t = 0; t < K; t++) {
        pre[b * (K + 1) + t] = s;
        s += lp[b * K + t];
    }
    pre[b * (K + 1) + K] = s;
}

// First changed sequence position of x' against its sample x (position s
// holds orbital K-1-s); the sample itself restarts at the last position.
__device__ __forceinline__ int first_change(int K, const uint64_t *x, const uint64_t *xp) {
    const uint64_t d0 = x[0] ^ xp[0], d1 = x[1] ^ xp[1];
    if (!d0 && !d1) return K - 1;
    const int p = d1 ? 127 - __clzll(d1) : 63 - __clzll(d0);
    return K - 1 - (p >> 1);
}

// Per listed connection i (x' = xkeys[list[i]], sample list[i] / C of the
// chunk): its start s0 and row count K - s0.
__global__ void k64x_count(const uint64_t *__restrict__ xkeys, const int32_t *__restrict__ list, int64_t n,
                           const uint64_t *__restrict__ keys, int64_t C, int K, int32_t *__restrict__ s0v,
                           int32_t *__restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t e = list[i];
    const int s0 = first_change(K, keys + 2 * (e / C), xkeys + 2 * e);
    s0v[i] = s0;
    rows[i] = K - s0;
}

// Row maps of one batch of B listed connections: rows off[i] - off0 ..
// + K - s0[i] belong to connection i, position s0[i] + j; and the batch's
// keys gathered into ckeys.
__global__ void k64x_rowmap(const uint64_t *__restrict__ xkeys, const int32_t *__restrict__ list,
                            const int32_t *__restrict__ s0v, const int32_t *__restrict__ off, int32_t off0, int64_t B,
                            int K, int32_t *__restrict__ row_cfg, int32_t *__restrict__ row_pos,
                            uint64_t *__restrict__ ckeys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const int s0 = s0v[i];
    const int r0 = off[i] - off0;
    for (int j = 0; j < K - s0; j++) {
        row_cfg[r0 + j] = (int32_t)i;
        row_pos[r0 + j] = s0 + j;
    }
    const int64_t e = list[i];
    ckeys[2 * i] = xkeys[2 * e];
    ckeys[2 * i + 1] = xkeys[2 * e + 1];
}

// Embeddings of the mapped rows: h[r][c] = tok_emb[token at s-1][c] + pos_emb[s][c].
__global__ void k64x_embed(ModelView M, const uint64_t *__restrict__ ckeys, const int32_t *__restrict__ row_cfg,
                           const int32_t *__restrict__ row_pos, int64_t R, double *__restrict__ h) {
    const int K = M.K, d = M.d;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R * d) return;
    const int64_t row = e / d;
    const int c = (int)(e - row * d);
    const int64_t i = row_cfg[row];
    const int s = row_pos[row];
    Key x;
    x.lo = ckeys[2 * i];
    x.hi = ckeys[2 * i + 1];
    int prev = 4;
    if (s > 0) {
        const int o = K - s;  // orbital of position s - 1
        prev = key_bit(x, 2 * o) + 2 * key_bit(x, 2 * o + 1);
    }
    h[e] = M.w64[M.off.tok_emb + prev * d + c] + M.w64[M.off.pos_emb + (int64_t)s * d + c];
}

// Causal attention of the mapped rows on FP64 MFMA (the tiling of
// k64_attention): one wave per (connection, head); query blocks from the one
// holding s0 on, queries below s0 read as zero and are not written; keys and
// values below s0 come from the cache of the connection's sample (list[i] / C
// in the chunk), the rest from this pass (row off[i] - off0 + s - s0).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k64x_attention(const double *__restrict__ q, const double *__restrict__ k, const double *__restrict__ v,
               const double *__restrict__ kvc, const int32_t *__restrict__ list, const int32_t *__restrict__ s0v,
               const int32_t *__restrict__ off, int32_t off0, int64_t C, int64_t B, int K, int L, int l, double scale,
               double *__restrict__ o) {
    __shared__ double Ps[4][16][64 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t g = (int64_t)blockIdx.x * 4 + w;
    if (g >= B * 4) return;  // wave-uniform; the kernel has no block barrier
    const int64_t i = g >> 2;
    const int hh = (int)(g & 3);
    const int s0 = s0v[i];
    const int64_t smp = list[i] / C;
    const int64_t per = (int64_t)K * 64;
    const double *kc = kvc + ((smp * L + l) * 2) * per + hh * 16, *vc = kc + per;
    const int64_t rb = (int64_t)(off[i] - off0) * 64 + hh * 16;  // row s0 of this connection, head hh
    const double *qh = q + rb, *kh = k + rb, *vh = v + rb;
    auto ldv = [&](int s, int c) { return s >= K ? 0.0 : s < s0 ? vc[(int64_t)s * 64 + c] : vh[(int64_t)(s - s0) * 64 + c]; };
    // The score product's contraction index is the head column 4 lk + k4, so
    // a lane's four operands of one key (or query) row are contiguous: one
    // 32-byte load, and the four lanes of a row read its 128 bytes.  The
    // values are read where the P V product takes them (16 lanes of a row,
    // 128 bytes), not held: 114 registers, four waves per SIMD.
    f64x4 kf[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        const int s = kb * 16 + lr;
        kf[kb] = s >= K ? f64x4{0.0, 0.0, 0.0, 0.0}
                        : *reinterpret_cast<const f64x4 *>((s < s0 ? kc + (int64_t)s * 64 : kh + (int64_t)(s - s0) * 64) +
                                                           4 * lk);
    }
    double(*P)[64 + 1] = Ps[w];
    const int qb0 = s0 >> 4;
#pragma unroll
    for (int qb = 0; qb < 4; qb++) {
        if (qb < qb0 || 16 * qb >= K) continue;  // wave-uniform
        const int sq = qb * 16 + lr;
        const f64x4 qf = (sq >= s0 && sq < K) ? *reinterpret_cast<const f64x4 *>(qh + (int64_t)(sq - s0) * 64 + 4 * lk)
                                              : f64x4{0.0, 0.0, 0.0, 0.0};
        f64x4 st[4];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            st[kb] = f64x4{0.0, 0.0, 0.0, 0.0};
            if (kb <= qb)
#pragma unroll
                for (int k4 = 0; k4 < 4; k4++)
                    st[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(qf[k4], kf[kb][k4], st[kb], 0, 0, 0);
        }
        double mx[4], den[4], rden[4];
#pragma unroll
        for (int ii = 0; ii < 4; ii++) {
            mx[ii] = -INFINITY;
#pragma unroll
            for (int kb = 0; kb <= qb; kb++)
                if (kb < qb || lr <= lk + 4 * ii) mx[ii] = fmax(mx[ii], st[kb][ii]);
#pragma unroll
            for (int off2 = 8; off2 >= 1; off2 >>= 1) mx[ii] = fmax(mx[ii], __shfl_xor(mx[ii], off2, 16));
            den[ii] = 0.0;
#pragma unroll
            for (int kb = 0; kb < 4; kb++) {
                const double p =
                    (kb < qb || (kb == qb && lr <= lk + 4 * ii)) ? exp((st[kb][ii] - mx[ii]) * scale) : 0.0;
                st[kb][ii] = p;
                den[ii] += p;
            }
#pragma unroll
            for (int off2 = 8; off2 >= 1; off2 >>= 1) den[ii] += __shfl_xor(den[ii], off2, 16);
            rden[ii] = 1.0 / den[ii];
        }
#pragma unroll
        for (int kb = 0; kb < 4; kb++)
#pragma unroll
            for (int ii = 0; ii < 4; ii++) P[lk + 4 * ii][kb * 16 + lr] = st[kb][ii] * rden[ii];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f64x4 ot = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4 * (qb + 1); kk++)
            ot = __builtin_amdgcn_mfma_f64_16x16x4f64(P[lr][4 * kk + lk], ldv(4 * kk + lk, lr), ot, 0, 0, 0);
#pragma unroll
        for (int ii = 0; ii < 4; ii++) {
            const int s = qb * 16 + lk + 4 * ii;
            if (s >= s0 && s < K) o[rb + (int64_t)(s - s0) * 64 + lr] = ot[ii];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Output head of the mapped rows (as k64_head): one wave per row; the
// electrons placed before position s are counted from the key.
__global__ void __launch_bounds__(256) k64x_head(ModelView M, const double *__restrict__ a,
                                                 const uint64_t *__restrict__ ckeys,
                                                 const int32_t *__restrict__ row_cfg,
                                                 const int32_t *__restrict__ row_pos, int64_t R,
                                                 double *__restrict__ lp) {
    const int K = M.K;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= R) return;  // wave-uniform
    const int64_t i = row_cfg[row];
    const int s = row_pos[row];
    Key x;
    x.lo = ckeys[2 * i];
    x.hi = ckeys[2 * i + 1];
    auto token = [&](int pos) {
        const int oo = K - 1 - pos;
        return key_bit(x, 2 * oo) + 2 * key_bit(x, 2 * oo + 1);
    };
    const int tr = lane < s ? token(lane) : 0;
    const int up = __popcll(__ballot(tr & 1)), dn = __popcll(__ballot(tr >> 1));
    const double *W = M.w64;
    const double av = a[row * 64 + lane];
    double z[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        double vv = av * W[M.off.head_w + lane * 4 + t];
#pragma unroll
        for (int off2 = 32; off2 >= 1; off2 >>= 1) vv += __shfl_xor(vv, off2, 64);
        z[t] = vv;
    }
    if (lane != 0) return;
    const int rem = K - 1 - s, orb = K - 1 - s;
    bool ok[4];
    double mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        z[t] += W[M.off.head_b + t] + W[M.off.bias + orb * 4 + t];
        const int bu = t & 1, bd = t >> 1;
        ok[t] = (up + bu <= M.n_up) && (dn + bd <= M.n_dn) && (M.n_up - up - bu <= rem) && (M.n_dn - dn - bd <= rem);
        if (ok[t] && z[t] > mx) mx = z[t];
    }
    double den = 0.0;
#pragma unroll
    for (int t = 0; t < 4; t++)
        if (ok[t]) den += exp(z[t] - mx);
    const int ts = token(s);
    lp[row] = ok[ts] ? (z[ts] - mx) - log(den) : -INFINITY;
}

// Per listed connection: log|psi| = 1/2 (pre[sample][s0] + sum of its rows'
// log pi), phase = b3 + z2 . w3, written to xla / xph at list[i] (one wave each).
__global__ void __launch_bounds__(256) k64x_finish(ModelView M, const double *__restrict__ lp,
                                                   const double *__restrict__ z2, const double *__restrict__ pre,
                                                   const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ s0v,
                                                   const int32_t *__restrict__ off, int32_t off0, int64_t C,
                                                   int64_t B, double *__restrict__ xla, double *__restrict__ xph) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= B) return;
    const int K = M.K, s0 = s0v[i];
    const int64_t r0 = off[i] - off0;
    double s = 0.0;
    for (int t = lane; t < K - s0; t += 64) s += lp[r0 + t];
    double ph = 0.0;
    for (int j = lane; j < M.P; j += 64) ph += z2[i * M.P + j] * M.w64[M.off.ph_w3 + j];
#pragma unroll
    for (int off2 = 32; off2 >= 1; off2 >>= 1) {
        s += __shfl_xor(s, off2, 64);
        ph += __shfl_xor(ph, off2, 64);
    }
    if (lane == 0) {
        const int64_t e = list[i];
        xla[e] = 0.5 * (pre[(e / C) * (K + 1) + s0] + s);
        xph[e] = M.w64[M.off.ph_b3] + ph;
    }
}

static unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int64_t f64_cache_doubles(const nnqs_model *m) { return (int64_t)m->desc.n_layers * 2 * m->desc.n_orb * 64; }

bool f64_shape_ok(const nnqs_model_desc &m) { return m.d_model == 64 && m.n_heads == 4 && m.d_ff % 64 == 0; }

nnqs_status enqueue_logpsi_f64(const nnqs_model *cm, const uint64_t *keys, int64_t n, double *logabs,
                               double *phase, hipStream_t st, int cpos, double *cond, double *kvc, double *pre) {
    nnqs_model *m = const_cast<nnqs_model *>(cm);  // owns its scratch (one call at a time per model)
    const ModelView M = model_view(m);
    const int K = M.K, d = M.d, F = M.F, P = M.P;
    const int64_t Bmax = n < kF64Batch ? n : kF64Batch;
    const int64_t rows_max = Bmax * K;
    // h, a, q, k, v [rows][64]; f [rows][F] (also z1, z2 [B][P]); lp [rows]; LayerNorm statistics [rows][2];
    // tok [rows]
    const size_t need = (size_t)rows_max * (5 * d + (F > 2 * P / K + 1 ? F : 2 * P / K + 1) + 3) * 8 + rows_max + 256;
    if (m->f64cap < need) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        hipFree(m->d_f64s);
        m->d_f64s = nullptr;
        m->f64cap = 0;
        if (hipMalloc(&m->d_f64s, need) != hipSuccess) return fail(NNQS_ENOMEM, "FP64 forward scratch (%zu bytes)", need);
        m->f64cap = need;
    }
    const size_t fcols = (size_t)(F > 2 * P / K + 1 ? F : 2 * P / K + 1);
    double *h = reinterpret_cast<double *>(m->d_f64s);
    double *a = h + rows_max * d, *q = a + rows_max * d, *kk = q + rows_max * d, *v = kk + rows_max * d;
    double *f = v + rows_max * d;
    double *lp = f + rows_max * fcols, *lst = lp + rows_max;
    int8_t *tok = reinterpret_cast<int8_t *>(lst + 2 * rows_max);
    const LayerOffsets LO = layer_offsets(d, F);
    const double *W = m->d_w64;
    const double scale = 1.0 / sqrt((double)(d / M.H));
    for (int64_t b0 = 0; b0 < n; b0 += kF64Batch) {
        const int64_t B = n - b0 < kF64Batch ? n - b0 : kF64Batch;
        const int64_t R = B * K;
        const unsigned gy = (unsigned)((R + 63) / 64);
        hipLaunchKernelGGL(k64_embed, dim3(blocks_for(R * d)), dim3(256), 0, st, M, keys + 2 * b0, B, tok, h);
        for (int l = 0; l < M.L; l++) {
            const double *Lw = W + M.off.layer0 + (int64_t)l * M.off.layer_stride;
            if (l == 0)  // later layers: the statistics come with the previous FFN output
                hipLaunchKernelGGL(k64_ln_stats, dim3(blocks_for(R, 4)), dim3(256), 0, st, h, R, lst);
            hipLaunchKernelGGL(k64_gemm_qkv, dim3(3, gy), dim3(256), 0, st, h, Lw + LO.wq, Lw + LO.bq,
                               LO.wk - LO.wq, R, q, (int64_t)(kk - q), lst, Lw + LO.ln1_g, Lw + LO.ln1_b);
            if (kvc)
                hipLaunchKernelGGL(k64_cache_kv, dim3(blocks_for(R * 64)), dim3(256), 0, st, kk, v, B, K, l, M.L,
                                   kvc + b0 * M.L * 2 * K * 64);
            hipLaunchKernelGGL(k64_attention, dim3((unsigned)B), dim3(256), 0, st, q, kk, v, B, K, scale, a);
            hipLaunchKernelGGL(k64_gemm_res<64>, dim3(1, gy), dim3(256), 0, st, a, 64, Lw + LO.wo, Lw + LO.bo, R, h,
                               lst);
            hipLaunchKernelGGL(k64_gemm_ln<2>, dim3((unsigned)((F + 63) / 64), gy), dim3(256), 0, st, h, Lw + LO.w1, F,
                               Lw + LO.b1, R, F, f, (int)fcols, lst, Lw + LO.ln2_g, Lw + LO.ln2_b);
            ffn_out(f, (int)fcols, Lw + LO.w2, Lw + LO.b2, R, F, h, lst, st);
        }
        hipLaunchKernelGGL(k64_layernorm, dim3(blocks_for(R, 4)), dim3(256), 0, st, h, W + M.off.lnf_g,
                           W + M.off.lnf_b, R, a);
        hipLaunchKernelGGL(k64_head, dim3(blocks_for(R, 4)), dim3(256), 0, st, M, a, tok, B, lp, cpos,
                           cond ? cond + 4 * b0 : (double *)nullptr);
        if (pre)
            hipLaunchKernelGGL(k64_prefix, dim3(blocks_for(B)), dim3(256), 0, st, lp, B, K,
                               pre + (int64_t)(K + 1) * b0);
        double *z1 = f, *z2 = f + (size_t)B * P;
        hipLaunchKernelGGL(k64_phase1, dim3(blocks_for(B * P)), dim3(256), 0, st, M, keys + 2 * b0, B, z1);
        hipLaunchKernelGGL(k64_gemm<2>, dim3((unsigned)((P + 63) / 64), (unsigned)((B + 63) / 64)), dim3(256), 0, st,
                           z1, P, W + M.off.ph_w2, P, W + M.off.ph_b2, B, P, P, z2, P);
        hipLaunchKernelGGL(k64_finish, dim3(blocks_for(B, 4)), dim3(256), 0, st, M, lp, z2, B, logabs + b0,
                           phase + b0);
        NNQS_HIP_CHECK(hipGetLastError());
    }
    return NNQS_OK;
}

// FP64 forward of n listed connections with prefix reuse (see k64_cache_kv):
// each x' runs only its rows from its first changed position s0 on (the
// sample itself: the last row), in batches of up to kF64Batch connections
// whose rows are packed one after another; kvc / pre: the cache of the
// chunk's samples (keys [m][2]), indexed by list entry / C.  Results go to
// xla / xph.  Synchronises `st` once (the row counts set the batches).
nnqs_status enqueue_f64_list(const nnqs_model *cm, const uint64_t *xkeys, int64_t C, const int32_t *list, int64_t n,
                             const uint64_t *keys, const double *kvc, const double *pre, double *xla, double *xph,
                             hipStream_t st) {
    if (n <= 0) return NNQS_OK;
    nnqs_model *m = const_cast<nnqs_model *>(cm);
    const ModelView M = model_view(m);
    const int K = M.K, d = M.d, F = M.F, P = M.P;
    // per-connection starts and row counts, then their offsets (host scan);
    // offsets are 32-bit (a chunk holds at most 2^24 connections of <= 64 rows)
    if (n * K > (int64_t)INT32_MAX)
        return fail(NNQS_EINVAL, "%lld refined connections exceed 32-bit row offsets", (long long)n);
    const size_t rag_need = (size_t)(3 * n + 1) * sizeof(int32_t);
    if (m->ragcap < rag_need) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        hipFree(m->d_rag);
        m->d_rag = nullptr;
        m->ragcap = 0;
        if (hipMalloc(&m->d_rag, rag_need) != hipSuccess) return fail(NNQS_ENOMEM, "row maps (%zu bytes)", rag_need);
        m->ragcap = rag_need;
    }
    int32_t *s0v = reinterpret_cast<int32_t *>(m->d_rag), *rows = s0v + n, *off = rows + n;
    hipLaunchKernelGGL(k64x_count, dim3(blocks_for(n)), dim3(256), 0, st, xkeys, list, n, keys, C, K, s0v, rows);
    NNQS_HIP_CHECK(hipGetLastError());
    std::vector<int32_t> h_rows((size_t)n), h_off((size_t)n + 1);
    NNQS_HIP_CHECK(hipMemcpyAsync(h_rows.data(), rows, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    h_off[0] = 0;
    for (int64_t i = 0; i < n; i++) h_off[(size_t)i + 1] = h_off[(size_t)i] + h_rows[(size_t)i];
    NNQS_HIP_CHECK(hipMemcpyAsync(off, h_off.data(), (size_t)(n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const int64_t Bmax = n < kF64Batch ? n : kF64Batch;
    const int64_t Rmax = Bmax * K;
    // h, a, q, k, v [rows][64]; f [rows][F]; z1, z2 [B][P]; lp [rows]; LayerNorm statistics [rows][2];
    // ckeys [B][2]; row maps [rows][2]
    const size_t need = ((size_t)Rmax * (5 * d + F + 3) + (size_t)Bmax * (2 * P + 2)) * 8 + (size_t)Rmax * 8 + 256;
    if (m->f64cap < need) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        hipFree(m->d_f64s);
        m->d_f64s = nullptr;
        m->f64cap = 0;
        if (hipMalloc(&m->d_f64s, need) != hipSuccess) return fail(NNQS_ENOMEM, "FP64 forward scratch (%zu bytes)", need);
        m->f64cap = need;
    }
    double *h = reinterpret_cast<double *>(m->d_f64s);
    double *a = h + Rmax * d, *qb = a + Rmax * d, *kk = qb + Rmax * d, *v = kk + Rmax * d;
    double *f = v + Rmax * d, *z1 = f + Rmax * F, *z2 = z1 + Bmax * P, *lp = z2 + Bmax * P;
    double *lst = lp + Rmax;  // LayerNorm statistics [rows][2]
    uint64_t *ckeys = reinterpret_cast<uint64_t *>(lst + 2 * Rmax);
    int32_t *row_cfg = reinterpret_cast<int32_t *>(ckeys + 2 * Bmax), *row_pos = row_cfg + Rmax;
    const LayerOffsets LO = layer_offsets(d, F);
    const double *W = m->d_w64;
    const double scale = 1.0 / sqrt((double)(d / M.H));
    for (int64_t b0 = 0; b0 < n; b0 += kF64Batch) {
        const int64_t B = n - b0 < kF64Batch ? n - b0 : kF64Batch;
        const int32_t off0 = h_off[(size_t)b0];
        const int64_t R = h_off[(size_t)(b0 + B)] - off0;
        const unsigned gy = (unsigned)((R + 63) / 64);
        const int32_t *lq = list + b0, *sq = s0v + b0, *oq = off + b0;
        hipLaunchKernelGGL(k64x_rowmap, dim3(blocks_for(B)), dim3(256), 0, st, xkeys, lq, sq, oq, off0, B, K, row_cfg,
                           row_pos, ckeys);
        hipLaunchKernelGGL(k64x_embed, dim3(blocks_for(R * d)), dim3(256), 0, st, M, ckeys, row_cfg, row_pos, R, h);
        for (int l = 0; l < M.L; l++) {
            const double *Lw = W + M.off.layer0 + (int64_t)l * M.off.layer_stride;
            if (l == 0)  // later layers: the statistics come with the previous FFN output
                hipLaunchKernelGGL(k64_ln_stats, dim3(blocks_for(R, 4)), dim3(256), 0, st, h, R, lst);
            hipLaunchKernelGGL(k64_gemm_qkv, dim3(3, gy), dim3(256), 0, st, h, Lw + LO.wq, Lw + LO.bq,
                               LO.wk - LO.wq, R, qb, (int64_t)(kk - qb), lst, Lw + LO.ln1_g, Lw + LO.ln1_b);
            hipLaunchKernelGGL(k64x_attention, dim3((unsigned)B), dim3(256), 0, st, qb, kk, v, kvc, lq, sq, oq, off0,
                               C, B, K, M.L, l, scale, a);
            hipLaunchKernelGGL(k64_gemm_res<64>, dim3(1, gy), dim3(256), 0, st, a, 64, Lw + LO.wo, Lw + LO.bo, R, h,
                               lst);
            hipLaunchKernelGGL(k64_gemm_ln<2>, dim3((unsigned)((F + 63) / 64), gy), dim3(256), 0, st, h, Lw + LO.w1, F,
                               Lw + LO.b1, R, F, f, F, lst, Lw + LO.ln2_g, Lw + LO.ln2_b);
            ffn_out(f, F, Lw + LO.w2, Lw + LO.b2, R, F, h, lst, st);
        }
        hipLaunchKernelGGL(k64_layernorm, dim3(blocks_for(R, 4)), dim3(256), 0, st, h, W + M.off.lnf_g,
                           W + M.off.lnf_b, R, a);
        hipLaunchKernelGGL(k64x_head, dim3(blocks_for(R, 4)), dim3(256), 0, st, M, a, ckeys, row_cfg, row_pos, R, lp);
        hipLaunchKernelGGL(k64_phase1, dim3(blocks_for(B * P)), dim3(256), 0, st, M, ckeys, B, z1);
        hipLaunchKernelGGL(k64_gemm<2>, dim3((unsigned)((P + 63) / 64), (unsigned)((B + 63) / 64)), dim3(256), 0, st,
                           z1, P, W + M.off.ph_w2, P, W + M.off.ph_b2, B, P, P, z2, P);
        hipLaunchKernelGGL(k64x_finish, dim3(blocks_for(B, 4)), dim3(256), 0, st, M, lp, z2, pre, lq, sq, oq, off0, C,
                           B, xla, xph);
        NNQS_HIP_CHECK(hipGetLastError());
    }
    return NNQS_OK;
}

// Instances launched from other files (the FP64 backward).
template __global__ void k64_gemm<0, false>(const double *, int, const double *, int, const double *, int64_t, int,
                                            int, double *, int);
template __global__ void k64_gemm<1, false>(const double *, int, const double *, int, const double *, int64_t, int,
                                            int, double *, int);
template __global__ void k64_gemm<0, true>(const double *, int, const double *, int, const double *, int64_t, int,
                                           int, double *, int);
template __global__ void k64_gemm<1, true>(const double *, int, const double *, int, const double *, int64_t, int,
                                           int, double *, int);

}  // namespace nnqs

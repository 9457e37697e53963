// FP64 parameter gradients of the ansatz (Section 3.1, Eq. 11 and Fig. 2,
// the Eq. 12 mask, the phase MLP of Section 4.1) and the VMC step around them:
// the gradient estimator of Eq. 7 (Section 2.1), AdamW and the warm-up
// learning rate of Eq. 13 (Section 4.1).
//
// The forward runs layer by layer over passes of kGradBatch configurations
// with the kernels of the FP64 forward, keeping every activation the backward
// needs (about 33 KB per sequence row at d 64, F 256, four layers).  The
// backward walks the layers in reverse with one kernel per step: row kernels
// (one wave per row) for the head and LayerNorm, one wave per (configuration,
// head) for attention, FP64 MFMA products with the transposed weight for the
// input gradients, and a split-k FP64 MFMA product X^T dY for every weight
// gradient whose per-split partials are added in a fixed order, so results
// are reproducible bit for bit.  The token and position embeddings take their
// gradients through the same product with one-hot row matrices.
#include <cmath>
#include <vector>

#include "f64_kernels.hpp"

namespace nnqs {

constexpr int64_t kGradBatch = 256;  // configurations per pass
constexpr int64_t kTnRows = 512;     // rows per split of the weight-gradient products
constexpr int kTnMaxSplits = (int)((kGradBatch * 64 + kTnRows - 1) / kTnRows);

__device__ __forceinline__ double gelu_grad_f64(double u) {
    // d/du [u Phi(u)] = Phi(u) + u phi(u)
    const double cdf = 0.5 * (1.0 + erf(u * 0.70710678118654752440));
    const double pdf = 0.39894228040143267794 * exp(-0.5 * u * u);
    return cdf + u * pdf;
}

__global__ void kg_fill(double *__restrict__ p, int64_t n, double v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void kg_copy(const double *__restrict__ src, int64_t n, double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

__global__ void kg_gelu(const double *__restrict__ u, int64_t n, double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = gelu_f64(u[e]);
}

// d[e] *= GELU'(u[e])
__global__ void kg_gelu_back(const double *__restrict__ u, int64_t n, double *__restrict__ d) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) d[e] *= gelu_grad_f64(u[e]);
}

// Occupation bits as a [B][N2] matrix of 0 / 1 (the phase MLP's input).
__global__ void kg_bits(const uint64_t *__restrict__ keys, int64_t B, int N2, double *__restrict__ bits) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * N2) return;
    const int64_t b = e / N2;
    const int p = (int)(e - b * N2);
    Key x;
    x.lo = keys[2 * b];
    x.hi = keys[2 * b + 1];
    bits[e] = (double)key_bit(x, p);
}

// One-hot rows of the input token (previous token, begin token 4 at s = 0)
// [R][5] and of the position [R][K], for the embedding gradients.
__global__ void kg_onehots(const int8_t *__restrict__ tok, int64_t B, int K, double *__restrict__ oh_tok,
                           double *__restrict__ oh_pos) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= B * K) return;
    const int s = (int)(row % K);
    const int prev = s == 0 ? 4 : tok[row - 1];
    for (int t = 0; t < 5; t++) oh_tok[row * 5 + t] = t == prev ? 1.0 : 0.0;
    for (int j = 0; j < K; j++) oh_pos[row * K + j] = j == s ? 1.0 : 0.0;
}

// Output head backward, one wave per row (lane = model column, d = 64).  The
// row's log-probability lp = z_t - log sum_{allowed u} exp z_u enters log|psi|
// with weight 1/2, so with the configuration's cotangent cl:
// dz_u = cl/2 (delta_{u t} - pi_u) over allowed tokens u, 0 for masked ones;
// d(af) = W_head dz.
__global__ void __launch_bounds__(256) kg_head_back(ModelView M, const double *__restrict__ af,
                                                    const int8_t *__restrict__ tok, int64_t B,
                                                    const double *__restrict__ cl, double *__restrict__ dz,
                                                    double *__restrict__ daf) {
    const int K = M.K;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= B * K) return;  // wave-uniform
    const int64_t b = row / K;
    const int s = (int)(row - b * K);
    const int tr = lane < s ? tok[b * K + lane] : 0;
    const int up = __popcll(__ballot(tr & 1)), dn = __popcll(__ballot(tr >> 1));
    const double *W = M.w64;
    const double av = af[row * 64 + lane];
    double z[4], wc[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        wc[t] = W[M.off.head_w + lane * 4 + t];
        double v = av * wc[t];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        z[t] = v;
    }
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
    const double coef = 0.5 * cl[b];
    double g[4], acc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        g[t] = ok[t] ? coef * ((t == ts ? 1.0 : 0.0) - exp(z[t] - mx) / den) : 0.0;
        acc += g[t] * wc[t];
    }
    daf[row * 64 + lane] = acc;
    if (lane < 4) dz[row * 4 + lane] = lane == 0 ? g[0] : lane == 1 ? g[1] : lane == 2 ? g[2] : g[3];
}

// LayerNorm backward (eps 1e-5), one wave per row of width 64: with
// xh = (x - mean) r and gy = dy * gamma,
// dx = r (gy - mean(gy) - xh mean(gy xh)); writes dx (+ add) and
// prod = dy * xh (summed over rows for the gain's gradient).  add may alias dx.
__global__ void __launch_bounds__(256) kg_layernorm_back(const double *__restrict__ x, const double *__restrict__ g,
                                                         const double *__restrict__ dy, int64_t rows,
                                                         const double *add, double *dx,
                                                         double *__restrict__ prod) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int64_t e = row * 64 + lane;
    const double v = x[e];
    double s = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const double mean = s / 64.0;
    double q = (v - mean) * (v - mean);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off, 64);
    const double r = 1.0 / sqrt(q / 64.0 + 1e-5);
    const double xh = (v - mean) * r;
    const double d = dy[e];
    const double gy = d * g[lane];
    double m1 = gy, m2 = gy * xh;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        m1 += __shfl_xor(m1, off, 64);
        m2 += __shfl_xor(m2, off, 64);
    }
    const double out = r * (gy - m1 / 64.0 - xh * (m2 / 64.0));
    dx[e] = (add ? add[e] : 0.0) + out;
    prod[e] = d * xh;
}

// Causal attention backward, one wave per (configuration, head), lane i =
// query row i (K <= 64): recompute P = softmax(scale Q K^T) row by row, then
// dV = P^T dO, dS = P o (dO V^T - D) with D_i = dO_i . O_i, dQ = scale dS K,
// dK = scale dS^T Q.  q, k, v, o, dout and the outputs are [B*K][64] with head
// hh in columns 16 hh .. 16 hh + 15.
__global__ void __launch_bounds__(64) kg_attention_back(const double *__restrict__ q, const double *__restrict__ k,
                                                        const double *__restrict__ v, const double *__restrict__ o,
                                                        const double *__restrict__ dout, int64_t B, int K,
                                                        double scale, double *__restrict__ dq,
                                                        double *__restrict__ dk, double *__restrict__ dv) {
    __shared__ double Qs[64][17], Ks[64][17], Vs[64][17], Gs[64][17];
    __shared__ double P[64][65];
    const int i = threadIdx.x;
    const int64_t b = blockIdx.x >> 2;
    const int hh = (int)(blockIdx.x & 3);
    if (b >= B) return;  // block-uniform
    const int64_t base = (b * K + i) * 64 + hh * 16;
    double Di = 0.0;
    for (int c = 0; c < 16; c++) {
        const bool in = i < K;
        Qs[i][c] = in ? q[base + c] : 0.0;
        Ks[i][c] = in ? k[base + c] : 0.0;
        Vs[i][c] = in ? v[base + c] : 0.0;
        const double gd = in ? dout[base + c] : 0.0;
        Gs[i][c] = gd;
        Di += gd * (in ? o[base + c] : 0.0);
    }
    __syncthreads();
    if (i < K) {
        double mx = -INFINITY;
        for (int j = 0; j <= i; j++) {
            double sc = 0.0;
            for (int c = 0; c < 16; c++) sc += Qs[i][c] * Ks[j][c];
            P[i][j] = sc;
            mx = fmax(mx, sc);
        }
        double den = 0.0;
        for (int j = 0; j <= i; j++) {
            const double p = exp((P[i][j] - mx) * scale);
            P[i][j] = p;
            den += p;
        }
        const double inv = 1.0 / den;
        for (int j = 0; j <= i; j++) P[i][j] *= inv;
    }
    __syncthreads();
    double acc[16];
    // dV[j] = sum_{i >= j} P[i][j] dO[i]   (lane = key j)
    for (int c = 0; c < 16; c++) acc[c] = 0.0;
    for (int r = i; r < K; r++) {
        const double p = P[r][i];
        for (int c = 0; c < 16; c++) acc[c] += p * Gs[r][c];
    }
    if (i < K)
        for (int c = 0; c < 16; c++) dv[base + c] = acc[c];
    __syncthreads();  // every column of P is read before rows become dS
    if (i < K) {
        for (int j = 0; j <= i; j++) {
            double dp = 0.0;
            for (int c = 0; c < 16; c++) dp += Gs[i][c] * Vs[j][c];
            P[i][j] = P[i][j] * (dp - Di);
        }
        for (int c = 0; c < 16; c++) acc[c] = 0.0;
        for (int j = 0; j <= i; j++) {
            const double ds = P[i][j];
            for (int c = 0; c < 16; c++) acc[c] += ds * Ks[j][c];
        }
        for (int c = 0; c < 16; c++) dq[base + c] = scale * acc[c];
    }
    __syncthreads();
    // dK[j] = scale sum_{i >= j} dS[i][j] Q[i]   (lane = key j)
    for (int c = 0; c < 16; c++) acc[c] = 0.0;
    for (int r = i; r < K; r++) {
        const double ds = P[r][i];
        for (int c = 0; c < 16; c++) acc[c] += ds * Qs[r][c];
    }
    if (i < K)
        for (int c = 0; c < 16; c++) dk[base + c] = scale * acc[c];
}

// Phase MLP output layer backward: du2[b][i] = cp[b] w3[i] GELU'(u2[b][i]).
__global__ void kg_phase_top(const double *__restrict__ u2, const double *__restrict__ w3,
                             const double *__restrict__ cp, int64_t B, int P, double *__restrict__ du2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * P) return;
    const int64_t b = e / P;
    const int j = (int)(e - b * P);
    du2[e] = cp[b] * w3[j] * gelu_grad_f64(u2[e]);
}

// Weight-gradient partials on FP64 MFMA: part[z][i][j] = sum over rows r of
// split z of X[r][i] D[r][j] for i < M, j < N (X null: a column of ones, M = 1,
// the bias gradients).  Block: 64 x 64 tile of the [M][N] result, four waves
// of 16 rows; rows in slices of 32 through LDS (the MFMA layout as in k64_gemm).
__global__ void __launch_bounds__(256) kg_gemm_tn(const double *__restrict__ X, int ldx,
                                                  const double *__restrict__ D, int ldd, int64_t R, int M, int N,
                                                  int64_t rows_per_split, double *__restrict__ part) {
    constexpr int KS = 32;
    __shared__ double Xs[KS][64 + 1];
    __shared__ double Ds[KS][64 + 1];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = l & 15, lk = l >> 4;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int64_t rs = (int64_t)blockIdx.z * rows_per_split;
    const int64_t re = rs + rows_per_split < R ? rs + rows_per_split : R;
    const int tc = threadIdx.x & 63, tr = threadIdx.x >> 6;
    f64x4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = rs; k0 < re; k0 += KS) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int kk = tr + 4 * e;
            const int64_t r = k0 + kk;
            const bool rin = r < re;
            Xs[kk][tc] = (rin && i0 + tc < M) ? (X ? X[r * ldx + i0 + tc] : 1.0) : 0.0;
            Ds[kk][tc] = (rin && j0 + tc < N) ? D[r * ldd + j0 + tc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < KS; k4 += 4) {
            const double a = Xs[k4 + lk][16 * w + lr];
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ds[k4 + lk][cb * 16 + lr], acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
        const int j = j0 + cb * 16 + lr;
        if (j >= N) continue;
#pragma unroll
        for (int ii = 0; ii < 4; ii++) {
            const int i = i0 + 16 * w + lk + 4 * ii;
            if (i < M) part[((int64_t)blockIdx.z * M + i) * N + j] = acc[cb][ii];
        }
    }
}

// grad[e] += sum_{z < S} part[z][e], in order of z.
__global__ void kg_reduce_add(const double *__restrict__ part, int S, int64_t MN, double *__restrict__ grad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MN) return;
    double s = 0.0;
    for (int z = 0; z < S; z++) s += part[(int64_t)z * MN + e];
    grad[e] += s;
}

// Eq. 7 cotangents: with p = c / sum c and E = energy[0] + i energy[1],
// cl = 2 p Re(E_loc - E) (for log|psi|), cp = 2 p Im(E_loc - E) (for the phase).
__global__ void kg_vmc_coef(const uint32_t *__restrict__ counts, const double *__restrict__ eloc, int64_t n,
                            const double *__restrict__ energy, double *__restrict__ cl, double *__restrict__ cp) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double p = (double)counts[b] / energy[2];
    cl[b] = 2.0 * p * (eloc[2 * b] - energy[0]);
    cp[b] = 2.0 * p * (eloc[2 * b + 1] - energy[1]);
}

// AdamW (decoupled weight decay): w <- w (1 - lr wd) - lr mh / (sqrt(vh) + eps)
// with bias-corrected moments; entries in [fix0, fix1) (the fixed logit-bias
// table) are left unchanged with zero moments.
__global__ void kg_adamw(double *__restrict__ w, const double *__restrict__ g, double *__restrict__ m,
                         double *__restrict__ v, int64_t n, int64_t fix0, int64_t fix1, double lr, double b1,
                         double b2, double eps, double wd, double bc1, double bc2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (e >= fix0 && e < fix1) {
        m[e] = 0.0;
        v[e] = 0.0;
        return;
    }
    const double ge = g[e];
    const double me = b1 * m[e] + (1.0 - b1) * ge;
    const double ve = b2 * v[e] + (1.0 - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const double mh = me / bc1, vh = ve / bc2;
    w[e] = w[e] * (1.0 - lr * wd) - lr * mh / (sqrt(vh) + eps);
}

static unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Device scratch of one pass (doubles unless noted), carved from one buffer.
struct GradScratch {
    double *Hin, *A1, *Q, *Kb, *V, *O, *Hmid, *A2, *U, *G;  // per layer (Hin: L + 1)
    double *AF, *LP, *bits, *U1, *Z1, *U2, *Z2, *la, *ph;
    double *dH, *dA, *dO, *dQ, *dK, *dV, *dU, *prod, *dz, *ohtok, *ohpos, *dP1, *dP2;
    double *part, *epart, *energy, *cl, *cp;
    int8_t *tok;
};

static size_t grad_scratch_doubles(const nnqs_model_desc &m, int64_t Bmax, int64_t nmax, size_t &part_elems) {
    const int64_t K = m.n_orb, d = m.d_model, F = m.d_ff, P = m.phase_hidden, L = m.n_layers;
    const int64_t R = Bmax * K;
    int64_t mn = d * F;
    if (P * P > mn) mn = P * P;
    if (2 * K * P > mn) mn = 2 * K * P;
    part_elems = (size_t)kTnMaxSplits * (size_t)mn;
    size_t n = 0;
    n += (size_t)(L + 1) * R * d + (size_t)7 * L * R * d + (size_t)2 * L * R * F;  // saved layers
    n += (size_t)R * d + R + (size_t)Bmax * 2 * K + (size_t)4 * Bmax * P + 2 * Bmax;
    n += (size_t)7 * R * d + (size_t)R * F + (size_t)R * 4 + (size_t)R * 5 + (size_t)R * K + (size_t)2 * Bmax * P;
    n += part_elems + (size_t)kPartialBlocks * 8 + 8 + (size_t)2 * nmax;
    n += (size_t)(R + 7) / 8 + 1;  // tokens (bytes)
    return n;
}

static nnqs_status grad_scratch(nnqs_model *m, int64_t n, GradScratch &S) {
    const nnqs_model_desc &md = m->desc;
    const int64_t Bmax = n < kGradBatch ? n : kGradBatch;
    size_t part_elems = 0;
    const size_t need = grad_scratch_doubles(md, kGradBatch, n, part_elems) * sizeof(double);
    if (m->gradcap < need) {
        (void)hipFree(m->d_grads);
        m->d_grads = nullptr;
        m->gradcap = 0;
        if (hipMalloc(&m->d_grads, need) != hipSuccess)
            return fail(NNQS_ENOMEM, "FP64 gradient scratch (%zu bytes)", need);
        m->gradcap = need;
    }
    (void)Bmax;
    const int64_t K = md.n_orb, d = md.d_model, F = md.d_ff, P = md.phase_hidden, L = md.n_layers;
    const int64_t R = kGradBatch * K, B = kGradBatch;
    double *at = reinterpret_cast<double *>(m->d_grads);
    auto take = [&](size_t cnt) {
        double *p = at;
        at += cnt;
        return p;
    };
    S.Hin = take((size_t)(L + 1) * R * d);
    S.A1 = take((size_t)L * R * d);
    S.Q = take((size_t)L * R * d);
    S.Kb = take((size_t)L * R * d);
    S.V = take((size_t)L * R * d);
    S.O = take((size_t)L * R * d);
    S.Hmid = take((size_t)L * R * d);
    S.A2 = take((size_t)L * R * d);
    S.U = take((size_t)L * R * F);
    S.G = take((size_t)L * R * F);
    S.AF = take((size_t)R * d);
    S.LP = take((size_t)R);
    S.bits = take((size_t)B * 2 * K);
    S.U1 = take((size_t)B * P);
    S.Z1 = take((size_t)B * P);
    S.U2 = take((size_t)B * P);
    S.Z2 = take((size_t)B * P);
    S.la = take((size_t)B);
    S.ph = take((size_t)B);
    S.dH = take((size_t)R * d);
    S.dA = take((size_t)R * d);
    S.dO = take((size_t)R * d);
    S.dQ = take((size_t)R * d);
    S.dK = take((size_t)R * d);
    S.dV = take((size_t)R * d);
    S.prod = take((size_t)R * d);
    S.dU = take((size_t)R * F);
    S.dz = take((size_t)R * 4);
    S.ohtok = take((size_t)R * 5);
    S.ohpos = take((size_t)R * K);
    S.dP1 = take((size_t)B * P);
    S.dP2 = take((size_t)B * P);
    S.part = take(part_elems);
    S.epart = take((size_t)kPartialBlocks * 8);
    S.energy = take(8);
    S.cl = take((size_t)n);
    S.cp = take((size_t)n);
    S.tok = reinterpret_cast<int8_t *>(at);
    return NNQS_OK;
}

// grad[goff ..] += X^T D over R rows (X null: column sums of D).
static void tn_add(const double *X, int ldx, const double *D, int ldd, int64_t R, int M, int N, double *part,
                   double *grad, hipStream_t st) {
    const int S = (int)((R + kTnRows - 1) / kTnRows);
    hipLaunchKernelGGL(kg_gemm_tn, dim3((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S), dim3(256),
                       0, st, X, ldx, D, ldd, R, M, N, (int64_t)kTnRows, part);
    const int64_t MN = (int64_t)M * N;
    hipLaunchKernelGGL(kg_reduce_add, dim3(nblocks(MN)), dim3(256), 0, st, part, S, MN, grad);
}

// C = A W^T (EPI 0) or C += A W^T (EPI 1) for a weight W [in][out]: A [M][out], C [M][in].
template <int EPI>
static void gemm_wt(const double *A, const double *W, int in, int out, int64_t M, double *C, hipStream_t st) {
    hipLaunchKernelGGL((k64_gemm<EPI, true>), dim3((unsigned)((in + 63) / 64), (unsigned)((M + 63) / 64)), dim3(256),
                       0, st, A, out, W, out, (const double *)nullptr, M, in, out, C, in);
}

// C = A W + b for a weight W [in][out]: A [M][in], C [M][out].
static void gemm_w(const double *A, const double *W, const double *b, int in, int out, int64_t M, double *C,
                   hipStream_t st) {
    hipLaunchKernelGGL((k64_gemm<0, false>), dim3((unsigned)((out + 63) / 64), (unsigned)((M + 63) / 64)),
                       dim3(256), 0, st, A, in, W, out, b, M, out, in, C, out);
}

static void gemm_w_add(const double *A, const double *W, const double *b, int in, int out, int64_t M, double *C,
                       hipStream_t st) {
    hipLaunchKernelGGL((k64_gemm<1, false>), dim3((unsigned)((out + 63) / 64), (unsigned)((M + 63) / 64)),
                       dim3(256), 0, st, A, in, W, out, b, M, out, in, C, out);
}

bool grad_shape_ok(const nnqs_model_desc &m) { return f64_shape_ok(m) && m.n_orb <= 64; }

// grad = sum_b cl[b] d log|psi_b| / dw + cp[b] d phi_b / dw (device arrays; the
// logit-bias entries stay zero).  With la / ph, the pass's forward values too.
nnqs_status enqueue_model_grad(nnqs_model *m, const uint64_t *keys, int64_t n, const double *cl, const double *cp,
                               double *grad, double *la_out, double *ph_out, hipStream_t st) {
    if (!grad_shape_ok(m->desc))
        return fail(NNQS_EUNSUPPORTED, "gradients need d_model 64, 4 heads, d_ff a multiple of 64 and n_orb <= 64");
    GradScratch S{};
    nnqs_status rc = grad_scratch(m, n, S);
    if (rc != NNQS_OK) return rc;
    const ModelView M = model_view(m);
    const int K = M.K, d = M.d, F = M.F, P = M.P, L = M.L;
    const LayerOffsets LO = layer_offsets(d, F);
    const ModelOffsets &OF = m->off;
    double *W = m->d_w64;
    const double scale = 1.0 / sqrt((double)(d / M.H));
    hipLaunchKernelGGL(kg_fill, dim3(nblocks(OF.total)), dim3(256), 0, st, grad, OF.total, 0.0);
    for (int64_t b0 = 0; b0 < n; b0 += kGradBatch) {
        const int64_t B = n - b0 < kGradBatch ? n - b0 : kGradBatch;
        const int64_t R = B * K, Rd = R * d, RF = R * F;
        const int64_t Rs = (int64_t)kGradBatch * K;  // layer stride in the saved buffers
        auto hin = [&](int l) { return S.Hin + (size_t)l * Rs * d; };
        auto lay = [&](double *base, int l, int w) { return base + (size_t)l * Rs * w; };
        // ---------------------------------------------------------- forward
        hipLaunchKernelGGL(k64_embed, dim3(nblocks(Rd)), dim3(256), 0, st, M, keys + 2 * b0, B, S.tok, hin(0));
        for (int l = 0; l < L; l++) {
            const double *Lw = W + OF.layer0 + (int64_t)l * OF.layer_stride;
            double *a1 = lay(S.A1, l, d), *q = lay(S.Q, l, d), *kk = lay(S.Kb, l, d), *v = lay(S.V, l, d);
            double *o = lay(S.O, l, d), *hm = lay(S.Hmid, l, d), *a2 = lay(S.A2, l, d);
            double *u = lay(S.U, l, F), *g = lay(S.G, l, F);
            hipLaunchKernelGGL(k64_layernorm, dim3(nblocks(R, 4)), dim3(256), 0, st, hin(l), Lw + LO.ln1_g,
                               Lw + LO.ln1_b, R, a1);
            gemm_w(a1, Lw + LO.wq, Lw + LO.bq, d, d, R, q, st);
            gemm_w(a1, Lw + LO.wk, Lw + LO.bk, d, d, R, kk, st);
            gemm_w(a1, Lw + LO.wv, Lw + LO.bv, d, d, R, v, st);
            hipLaunchKernelGGL(k64_attention, dim3((unsigned)B), dim3(256), 0, st, q, kk, v, B, K, scale, o);
            hipLaunchKernelGGL(kg_copy, dim3(nblocks(Rd)), dim3(256), 0, st, hin(l), Rd, hm);
            gemm_w_add(o, Lw + LO.wo, Lw + LO.bo, d, d, R, hm, st);
            hipLaunchKernelGGL(k64_layernorm, dim3(nblocks(R, 4)), dim3(256), 0, st, hm, Lw + LO.ln2_g,
                               Lw + LO.ln2_b, R, a2);
            gemm_w(a2, Lw + LO.w1, Lw + LO.b1, d, F, R, u, st);
            hipLaunchKernelGGL(kg_gelu, dim3(nblocks(RF)), dim3(256), 0, st, u, RF, g);
            hipLaunchKernelGGL(kg_copy, dim3(nblocks(Rd)), dim3(256), 0, st, hm, Rd, hin(l + 1));
            gemm_w_add(g, Lw + LO.w2, Lw + LO.b2, F, d, R, hin(l + 1), st);
        }
        hipLaunchKernelGGL(k64_layernorm, dim3(nblocks(R, 4)), dim3(256), 0, st, hin(L), W + OF.lnf_g, W + OF.lnf_b,
                           R, S.AF);
        hipLaunchKernelGGL(k64_head, dim3(nblocks(R, 4)), dim3(256), 0, st, M, S.AF, S.tok, B, S.LP, -1,
                           (double *)nullptr);
        hipLaunchKernelGGL(kg_bits, dim3(nblocks(B * 2 * K)), dim3(256), 0, st, keys + 2 * b0, B, 2 * K, S.bits);
        gemm_w(S.bits, W + OF.ph_w1, W + OF.ph_b1, 2 * K, P, B, S.U1, st);
        hipLaunchKernelGGL(kg_gelu, dim3(nblocks(B * P)), dim3(256), 0, st, S.U1, B * P, S.Z1);
        gemm_w(S.Z1, W + OF.ph_w2, W + OF.ph_b2, P, P, B, S.U2, st);
        hipLaunchKernelGGL(kg_gelu, dim3(nblocks(B * P)), dim3(256), 0, st, S.U2, B * P, S.Z2);
        if (la_out && ph_out)
            hipLaunchKernelGGL(k64_finish, dim3(nblocks(B, 4)), dim3(256), 0, st, M, S.LP, S.Z2, B, la_out + b0,
                               ph_out + b0);
        // --------------------------------------------------------- backward
        hipLaunchKernelGGL(kg_head_back, dim3(nblocks(R, 4)), dim3(256), 0, st, M, S.AF, S.tok, B, cl + b0, S.dz,
                           S.dA);
        tn_add(S.AF, d, S.dz, 4, R, d, 4, S.part, grad + OF.head_w, st);
        tn_add(nullptr, 0, S.dz, 4, R, 1, 4, S.part, grad + OF.head_b, st);
        hipLaunchKernelGGL(kg_layernorm_back, dim3(nblocks(R, 4)), dim3(256), 0, st, hin(L), W + OF.lnf_g, S.dA, R,
                           (const double *)nullptr, S.dH, S.prod);
        tn_add(nullptr, 0, S.prod, d, R, 1, d, S.part, grad + OF.lnf_g, st);
        tn_add(nullptr, 0, S.dA, d, R, 1, d, S.part, grad + OF.lnf_b, st);
        for (int l = L - 1; l >= 0; l--) {
            const double *Lw = W + OF.layer0 + (int64_t)l * OF.layer_stride;
            double *Gl = grad + OF.layer0 + (int64_t)l * OF.layer_stride;
            double *a1 = lay(S.A1, l, d), *q = lay(S.Q, l, d), *kk = lay(S.Kb, l, d), *v = lay(S.V, l, d);
            double *o = lay(S.O, l, d), *hm = lay(S.Hmid, l, d), *a2 = lay(S.A2, l, d);
            double *u = lay(S.U, l, F), *g = lay(S.G, l, F);
            // feed-forward block: out = hm + GELU(LN2(hm) W1 + b1) W2 + b2
            tn_add(g, F, S.dH, d, R, F, d, S.part, Gl + LO.w2, st);
            tn_add(nullptr, 0, S.dH, d, R, 1, d, S.part, Gl + LO.b2, st);
            gemm_wt<0>(S.dH, Lw + LO.w2, F, d, R, S.dU, st);
            hipLaunchKernelGGL(kg_gelu_back, dim3(nblocks(RF)), dim3(256), 0, st, u, RF, S.dU);
            tn_add(a2, d, S.dU, F, R, d, F, S.part, Gl + LO.w1, st);
            tn_add(nullptr, 0, S.dU, F, R, 1, F, S.part, Gl + LO.b1, st);
            gemm_wt<0>(S.dU, Lw + LO.w1, d, F, R, S.dA, st);
            hipLaunchKernelGGL(kg_layernorm_back, dim3(nblocks(R, 4)), dim3(256), 0, st, hm, Lw + LO.ln2_g, S.dA, R,
                               S.dH, S.dH, S.prod);
            tn_add(nullptr, 0, S.prod, d, R, 1, d, S.part, Gl + LO.ln2_g, st);
            tn_add(nullptr, 0, S.dA, d, R, 1, d, S.part, Gl + LO.ln2_b, st);
            // attention block: hm = h + Attn(LN1(h)) Wo + bo
            tn_add(o, d, S.dH, d, R, d, d, S.part, Gl + LO.wo, st);
            tn_add(nullptr, 0, S.dH, d, R, 1, d, S.part, Gl + LO.bo, st);
            gemm_wt<0>(S.dH, Lw + LO.wo, d, d, R, S.dO, st);
            hipLaunchKernelGGL(kg_attention_back, dim3((unsigned)(B * 4)), dim3(64), 0, st, q, kk, v, o, S.dO, B, K,
                               scale, S.dQ, S.dK, S.dV);
            tn_add(a1, d, S.dQ, d, R, d, d, S.part, Gl + LO.wq, st);
            tn_add(nullptr, 0, S.dQ, d, R, 1, d, S.part, Gl + LO.bq, st);
            tn_add(a1, d, S.dK, d, R, d, d, S.part, Gl + LO.wk, st);
            tn_add(nullptr, 0, S.dK, d, R, 1, d, S.part, Gl + LO.bk, st);
            tn_add(a1, d, S.dV, d, R, d, d, S.part, Gl + LO.wv, st);
            tn_add(nullptr, 0, S.dV, d, R, 1, d, S.part, Gl + LO.bv, st);
            gemm_wt<0>(S.dQ, Lw + LO.wq, d, d, R, S.dA, st);
            gemm_wt<1>(S.dK, Lw + LO.wk, d, d, R, S.dA, st);
            gemm_wt<1>(S.dV, Lw + LO.wv, d, d, R, S.dA, st);
            hipLaunchKernelGGL(kg_layernorm_back, dim3(nblocks(R, 4)), dim3(256), 0, st, hin(l), Lw + LO.ln1_g, S.dA,
                               R, S.dH, S.dH, S.prod);
            tn_add(nullptr, 0, S.prod, d, R, 1, d, S.part, Gl + LO.ln1_g, st);
            tn_add(nullptr, 0, S.dA, d, R, 1, d, S.part, Gl + LO.ln1_b, st);
        }
        // embeddings: h0[b, s] = tok_emb[token at s-1] + pos_emb[s]
        hipLaunchKernelGGL(kg_onehots, dim3(nblocks(R)), dim3(256), 0, st, S.tok, B, K, S.ohtok, S.ohpos);
        tn_add(S.ohtok, 5, S.dH, d, R, 5, d, S.part, grad + OF.tok_emb, st);
        tn_add(S.ohpos, K, S.dH, d, R, K, d, S.part, grad + OF.pos_emb, st);
        // phase MLP: phi = b3 + GELU(GELU(bits W1 + b1) W2 + b2) w3
        tn_add(S.Z2, P, cp + b0, 1, B, P, 1, S.part, grad + OF.ph_w3, st);
        tn_add(nullptr, 0, cp + b0, 1, B, 1, 1, S.part, grad + OF.ph_b3, st);
        hipLaunchKernelGGL(kg_phase_top, dim3(nblocks(B * P)), dim3(256), 0, st, S.U2, W + OF.ph_w3, cp + b0, B, P,
                           S.dP2);
        tn_add(S.Z1, P, S.dP2, P, B, P, P, S.part, grad + OF.ph_w2, st);
        tn_add(nullptr, 0, S.dP2, P, B, 1, P, S.part, grad + OF.ph_b2, st);
        gemm_wt<0>(S.dP2, W + OF.ph_w2, P, P, B, S.dP1, st);
        hipLaunchKernelGGL(kg_gelu_back, dim3(nblocks(B * P)), dim3(256), 0, st, S.U1, B * P, S.dP1);
        tn_add(S.bits, 2 * K, S.dP1, P, B, 2 * K, P, S.part, grad + OF.ph_w1, st);
        tn_add(nullptr, 0, S.dP1, P, B, 1, P, S.part, grad + OF.ph_b1, st);
        NNQS_HIP_CHECK(hipGetLastError());
    }
    return NNQS_OK;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

nnqs_status nnqs_model_grad(nnqs_model *m, const uint64_t *keys, int64_t n, const double *c_logabs,
                            const double *c_phase, double *grad, double *logabs, double *phase, void *stream) {
    clear_error();
    if (!m || !keys || !c_logabs || !c_phase || !grad) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if ((logabs == nullptr) != (phase == nullptr)) return fail(NNQS_EINVAL, "logabs and phase go together");
    return enqueue_model_grad(m, keys, n, c_logabs, c_phase, grad, logabs, phase, as_stream(stream));
}

nnqs_status nnqs_vmc_gradient(nnqs_model *m, const uint64_t *keys, const uint32_t *counts, const double *eloc,
                              int64_t n, double *grad, double *energy, void *stream) {
    clear_error();
    if (!m || !keys || !counts || !eloc || !grad) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if (!grad_shape_ok(m->desc))
        return fail(NNQS_EUNSUPPORTED, "gradients need d_model 64, 4 heads, d_ff a multiple of 64 and n_orb <= 64");
    hipStream_t st = as_stream(stream);
    GradScratch S{};
    nnqs_status rc = grad_scratch(m, n, S);
    if (rc != NNQS_OK) return rc;
    double *E = energy ? energy : S.energy;
    rc = enqueue_energy_partials(S.epart, counts, eloc, n, E, st);
    if (rc != NNQS_OK) return rc;
    hipLaunchKernelGGL(kg_vmc_coef, dim3(nblocks(n)), dim3(256), 0, st, counts, eloc, n, E, S.cl, S.cp);
    NNQS_HIP_CHECK(hipGetLastError());
    return enqueue_model_grad(m, keys, n, S.cl, S.cp, grad, nullptr, nullptr, st);
}

double nnqs_lr_schedule(int64_t step, int32_t d_model, int32_t warmup) {
    if (step < 1 || d_model < 1 || warmup < 1) return 0.0;
    const double i = (double)step;
    const double a = 1.0 / std::sqrt(i), b = i * std::pow((double)warmup, -1.5);
    return (a < b ? a : b) / std::sqrt((double)d_model);
}

nnqs_status nnqs_model_adamw_step(nnqs_model *m, const double *grad, int64_t step, double lr, double beta1,
                                  double beta2, double eps, double weight_decay, double *mom1, double *mom2,
                                  void *stream) {
    clear_error();
    if (!m || !grad || !mom1 || !mom2) return fail(NNQS_EINVAL, "null pointer argument");
    if (step < 1) return fail(NNQS_EINVAL, "step counts from 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0 && lr >= 0.0 &&
          weight_decay >= 0.0))
        return fail(NNQS_EINVAL, "AdamW hyper-parameters out of range");
    hipStream_t st = as_stream(stream);
    const int64_t nw = m->off.total;
    const double bc1 = 1.0 - std::pow(beta1, (double)step), bc2 = 1.0 - std::pow(beta2, (double)step);
    hipLaunchKernelGGL(kg_adamw, dim3(nblocks(nw)), dim3(256), 0, st, m->d_w64, grad, mom1, mom2, nw, m->off.bias,
                       m->off.bias + 4 * (int64_t)m->desc.n_orb, lr, beta1, beta2, eps, weight_decay, bc1, bc2);
    NNQS_HIP_CHECK(hipGetLastError());
    // the reduced-precision copies follow the FP64 master weights
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    std::vector<double> w64((size_t)nw);
    NNQS_HIP_CHECK(hipMemcpy(w64.data(), m->d_w64, nw * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<float> w32(w64.begin(), w64.end());
    bf16_model_free(m);
    return bf16_model_init(m, w32.data());
}

nnqs_status nnqs_model_get_weights(const nnqs_model *m, double *out, void *stream) {
    clear_error();
    if (!m || !out) return fail(NNQS_EINVAL, "null pointer argument");
    hipStream_t st = as_stream(stream);
    NNQS_HIP_CHECK(hipMemcpyAsync(out, m->d_w64, m->off.total * sizeof(double), hipMemcpyDeviceToDevice, st));
    return NNQS_OK;
}

}  // extern "C"

// BF16 MFMA forward of the amplitude transformer and the phase MLP (the
// networks of Section 3.1 / Fig. 2; phase MLP sizes of Section 4.1), for the
// shape d_model 64, 4 heads, FFN 256, phase hidden 512, K <= 64 orbitals.
//
// Transformer: two 64-lane waves own one configuration (64 sequence rows;
// rows >= K are padding that no real row attends to), each holding the
// residual stream of 32 rows in registers as eight 16x16 FP32 accumulator
// tiles of v_mfma_f32_16x16x32_bf16; eight waves per block serve four
// configurations, two waves per SIMD.  Every matrix product runs on that
// MFMA with BF16 operands and FP32 accumulation: LayerNorm output -> LDS
// (BF16) -> A tiles; weights are staged transposed (k contiguous) in LDS,
// shared by the block, and read as B tiles.  Attention is computed
// transposed, S^T = K Q^T, so that each lane owns one query and the causal
// softmax over keys is a register reduction plus two cross-lane steps;
// O^T = V^T P^T.  LayerNorm, softmax, GELU and the output head stay FP32.
//
// Phase MLP: a second kernel runs 16 configurations per wave through
// bits[16x128] @ W1 and GELU(z1)[16x512] @ W2 on the same MFMA, B tiles read
// from the L2-resident BF16 weights.
#include <cmath>
#include <cstring>
#include <vector>

#include "model.hpp"

namespace nnqs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kD = 64, kH = 4, kDh = 16, kF = 256, kP = 512, kRows = 64;
constexpr int kLd = 72;        // padded LDS row length (BF16) of 64-wide tiles
constexpr int kQLd = 24;       // padded row length of the per-head Q / K tiles
constexpr int kWaves = 4;      // waves per block of the phase MLP
constexpr int kPhaseBits = 128;

// Device layout of the BF16 weights (element offsets into d_bf16).
struct Bf16Layout {
    int64_t layer0, layer_stride;   // per layer: wqkvT[192][64] woT[64][64] w1T[256][64] w2T[64][256]
    int64_t ph_w1T, ph_w2T, total;  // ph_w1T[512][128] (rows: hidden unit, cols: bit), ph_w2T[512][512]
};
// FP32 vectors (element offsets into d_f32).
struct F32Layout {
    int64_t tok_emb, pos_emb, layer0, layer_stride;  // per layer: ln1_g ln1_b bqkv[192] bo ln2_g ln2_b b1[256] b2
    int64_t lnf_g, lnf_b, head_w, head_b, bias, ph_b1, ph_b2, ph_w3, ph_b3, gelu, total;
};

// The transformer's FFN GELU, v * Phi(v), takes the normal CDF Phi from a
// table of kGeluN (value, step) pairs at spacing 1/kGeluScale on [-8, 8):
// linear interpolation errs by at most h^2/8 max|Phi''| = 3e-5 (h = 1/32),
// well below the BF16 rounding of the result; Phi is clamped to its end
// values outside the range (Phi(-8) = 6e-16).  It replaces the exp and
// reciprocal of a closed-form erf by one LDS read (16384 GELUs per layer and
// configuration make this the largest VALU cost of the forward).
constexpr int kGeluN = 512;
constexpr float kGeluScale = 32.0f, kGeluOff = 256.0f, kGeluMaxU = 511.99997f;

static Bf16Layout bf16_layout(int L) {
    Bf16Layout o{};
    o.layer0 = 0;
    o.layer_stride = 192 * 64 + 64 * 64 + 256 * 64 + 64 * 256;
    o.ph_w1T = L * o.layer_stride;
    o.ph_w2T = o.ph_w1T + (int64_t)kP * kPhaseBits;
    o.total = o.ph_w2T + (int64_t)kP * kP;
    return o;
}

static F32Layout f32_layout(int K, int L) {
    F32Layout o{};
    int64_t at = 0;
    o.tok_emb = at; at += 5 * kD;
    o.pos_emb = at; at += (int64_t)K * kD;
    o.layer0 = at;
    o.layer_stride = 2 * kD + 192 + kD + 2 * kD + kF + kD;
    at += L * o.layer_stride;
    o.lnf_g = at; at += kD;
    o.lnf_b = at; at += kD;
    o.head_w = at; at += 4 * kD;
    o.head_b = at; at += 4;
    o.bias = at; at += 4 * (int64_t)K;
    o.ph_b1 = at; at += kP;
    o.ph_b2 = at; at += kP;
    o.ph_w3 = at; at += kP;
    o.ph_b3 = at; at += 1;
    o.gelu = at; at += 2 * kGeluN;
    o.total = at;
    return o;
}

// per-layer FP32 vector offsets
constexpr int kV_ln1_g = 0, kV_ln1_b = 64, kV_bqkv = 128, kV_bo = 320, kV_ln2_g = 384, kV_ln2_b = 448,
              kV_b1 = 512, kV_b2 = 768;

struct Bf16View {
    int K, L, n_up, n_dn;
    const __bf16 *wb;
    const float *wf;
    Bf16Layout bl;
    F32Layout fl;
};

// ------------------------------------------------------------ fragments
// v_mfma_f32_16x16x32_bf16 operand layout: A/B lane l holds row/column
// (l & 15) and k = 8 (l >> 4) .. 8 (l >> 4) + 7; the accumulator lane l holds
// column (l & 15) and rows 4 (l >> 4) .. 4 (l >> 4) + 3.
__device__ __forceinline__ f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 lds_frag(const __bf16 *base, int row, int ld, int k0) {
    return *reinterpret_cast<const bf16x8 *>(base + row * ld + k0);
}

__device__ __forceinline__ float dpp_row_sum(float v) {
    // sum over the 16 lanes of a DPP row (all lanes receive the total)
    v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));  // xor 1
    v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));  // xor 2
    v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x141, 0xF, 0xF, true)); // half mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x140, 0xF, 0xF, true)); // mirror
    return v;
}

__device__ __forceinline__ float gelu32(float v) { return gelu_bf16path(v); }

// GELU from the LDS table (see kGeluN): u = 32 (v + 8) clamped to [0, 512),
// entry floor(u), fraction u - floor(u).
__device__ __forceinline__ float gelu_tab(const float2 *tab, float v) {
    const float u = __builtin_amdgcn_fmed3f(fmaf(v, kGeluScale, kGeluOff), 0.0f, kGeluMaxU);
    const float2 e = tab[(int)u];
    return v * fmaf(__builtin_amdgcn_fractf(u), e.y, e.x);
}

// Cooperative copy of `rows` rows of `cols` BF16 (global, row stride gld) into
// LDS rows of stride lld.  cols is a multiple of 8.
__device__ __forceinline__ void stage_rows(__bf16 *dst, int lld, const __bf16 *src, int gld, int rows, int cols) {
    const int per_row = cols / 8;
    for (int e = threadIdx.x; e < rows * per_row; e += blockDim.x) {
        const int rr = e / per_row, cc = (e - rr * per_row) * 8;
        *reinterpret_cast<bf16x8 *>(dst + rr * lld + cc) = *reinterpret_cast<const bf16x8 *>(src + (int64_t)rr * gld + cc);
    }
}

// ------------------------------------------------------ transformer forward
// Two waves per configuration: wave half hf owns row blocks {hf, 3 - hf}
// (16 rows each), which balances the causal attention (row block b attends
// to b + 1 key blocks, and 1 + 4 = 2 + 3).  Eight waves per block serve four
// configurations.  With half the rows a wave holds half the residual stream
// and half the FFN tile, so two waves share a SIMD and hide each other's LDS,
// MFMA and barrier latency (one configuration per wave leaves one wave per
// SIMD).  The LayerNorm, attention and GELU outputs are per row and stay with
// the wave that owns the rows; only each head's K and V cross between the
// two waves, with block barriers around the attention of every head.
constexpr int kRsWaves = 8;             // waves per block
constexpr int kRsCfg = kRsWaves / 2;    // configurations per block

struct Tile32 {
    f32x4 t[8];  // tile (j, cb) = t[j * 4 + cb]: own row block j, column block cb
};

// acc += X[own rows][0..k_len) (LDS, BF16, row stride kLd) @ W, Wt[n][k] in LDS.
__device__ __forceinline__ void gemm_rows(Tile32 &acc, const __bf16 *X, int rb0, int rb1, const __bf16 *Wt, int wld,
                                          int k_len) {
    const int l = threadIdx.x & 63;
    const int r = l & 15, kq = 8 * (l >> 4);
    for (int ks = 0; ks < k_len; ks += 32) {
        bf16x8 a[2], b[4];
        a[0] = lds_frag(X, rb0 * 16 + r, kLd, ks + kq);
        a[1] = lds_frag(X, rb1 * 16 + r, kLd, ks + kq);
#pragma unroll
        for (int cb = 0; cb < 4; cb++) b[cb] = lds_frag(Wt, cb * 16 + r, wld, ks + kq);
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int cb = 0; cb < 4; cb++) acc.t[j * 4 + cb] = mfma16(a[j], b[cb], acc.t[j * 4 + cb]);
    }
}

// LayerNorm of the own rows (C layout) into X (LDS, BF16).
__device__ __forceinline__ void layer_norm_rows(const Tile32 &h, const float *g, const float *b, __bf16 *X, int rb0,
                                                int rb1) {
    const int l = threadIdx.x & 63;
    const int c = l & 15, r0 = 4 * (l >> 4);
    float gg[4], bb[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
        gg[cb] = g[cb * 16 + c];
        bb[cb] = b[cb * 16 + c];
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int rb = j ? rb1 : rb0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float s = 0.f;
#pragma unroll
            for (int cb = 0; cb < 4; cb++) s += h.t[j * 4 + cb][i];
            const float mean = dpp_row_sum(s) * (1.0f / kD);
            float v = 0.f;
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                const float dlt = h.t[j * 4 + cb][i] - mean;
                v += dlt * dlt;
            }
            const float rstd = rsqrtf(dpp_row_sum(v) * (1.0f / kD) + 1e-5f);
            const int row = rb * 16 + r0 + i;
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
                X[row * kLd + cb * 16 + c] = (__bf16)((h.t[j * 4 + cb][i] - mean) * rstd * gg[cb] + bb[cb]);
        }
    }
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Causal attention of query block QB for head hh: S^T[key][query] = K Q^T
// (lane owns query c16 + 16 QB and keys 16 kb + r0 + i), softmax over keys
// in base 2 (the scale and log2(e) are folded into Q), P[query][key] -> Pb,
// then O^T[c][query] = V^T P^T into Ob[query][16 hh + c].
template <int QB>
__device__ __forceinline__ void attend_block(const __bf16 *Qs, const __bf16 *Ks, const __bf16 *Vt, __bf16 *Pb,
                                             __bf16 *Ob, int hh) {
    const int l = threadIdx.x & 63;
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    const int qi = QB * 16 + c16;
    const bf16x8 zero8 = {};
    const bf16x8 bqf = l < 32 ? lds_frag(Qs, qi, kQLd, kq) : zero8;
    f32x4 st[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        st[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (kb <= QB) {
            const bf16x8 akf = l < 32 ? lds_frag(Ks, kb * 16 + c16, kQLd, kq) : zero8;
            st[kb] = mfma16(akf, bqf, st[kb]);
        }
    }
    // key 16 kb + r0 + i is visible to query 16 QB + c16 when kb < QB, or
    // kb == QB and r0 + i <= c16
    float mx = -INFINITY;
#pragma unroll
    for (int kb = 0; kb <= QB; kb++)
#pragma unroll
        for (int i = 0; i < 4; i++)
            if (kb < QB || r0 + i <= c16) mx = fmaxf(mx, st[kb][i]);
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float sum = 0.f;
#pragma unroll
    for (int kb = 0; kb < 4; kb++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float p = (kb < QB || (kb == QB && r0 + i <= c16)) ? __builtin_amdgcn_exp2f(st[kb][i] - mx) : 0.f;
            st[kb][i] = p;
            sum += p;
        }
    sum += __shfl_xor(sum, 16, 64);
    sum += __shfl_xor(sum, 32, 64);
    const float inv = 1.0f / sum;
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        bf16x4 pk;
#pragma unroll
        for (int i = 0; i < 4; i++) pk[i] = (__bf16)(st[kb][i] * inv);
        *reinterpret_cast<bf16x4 *>(Pb + c16 * kLd + kb * 16 + r0) = pk;
    }
    wave_lds_sync();
    f32x4 ot = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 64; ks += 32) {
        if (ks <= QB * 16 + 15) {
            const bf16x8 av = lds_frag(Vt, c16, kLd, ks + kq);
            const bf16x8 bp = lds_frag(Pb, c16, kLd, ks + kq);
            ot = mfma16(av, bp, ot);
        }
    }
    bf16x4 o4;
#pragma unroll
    for (int i = 0; i < 4; i++) o4[i] = (__bf16)ot[i];
    *reinterpret_cast<bf16x4 *>(Ob + qi * kLd + hh * kDh + r0) = o4;
    wave_lds_sync();  // Pb is rewritten by the next block
}

__global__ void __launch_bounds__(kRsWaves * 64) k_transformer_bf16(Bf16View M, const uint64_t *__restrict__ keys,
                                                                       int64_t n, double *__restrict__ logabs) {
    __shared__ __align__(16) __bf16 wbuf[192 * kLd];
    __shared__ __align__(16) float2 gtab[kGeluN];
    __shared__ __align__(16) __bf16 xs[kRsCfg][kRows * kLd];
    __shared__ __align__(16) __bf16 os[kRsCfg][kRows * kLd];
    __shared__ __align__(16) __bf16 qs[kRsCfg][kRows * kQLd];
    __shared__ __align__(16) __bf16 ks_[kRsCfg][kRows * kQLd];
    __shared__ __align__(16) __bf16 vt[kRsCfg][kDh * kLd];
    __shared__ __align__(16) __bf16 ps[kRsWaves][16 * kLd];
    __shared__ float red[kRsWaves];

    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cs = w >> 1, hf = w & 1;
    const int rb0 = hf, rb1 = 3 - hf;  // own row blocks
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    const int K = M.K;
    __bf16 *X = xs[cs], *Ob = os[cs], *Qs = qs[cs], *Ks = ks_[cs], *Vt = vt[cs], *Pb = ps[w];
    const float *wf = M.wf;
    for (int i = threadIdx.x; i < kGeluN; i += blockDim.x)
        gtab[i] = make_float2(wf[M.fl.gelu + 2 * i], wf[M.fl.gelu + 2 * i + 1]);
    __syncthreads();

    for (int64_t base = (int64_t)blockIdx.x * kRsCfg; base < n; base += (int64_t)gridDim.x * kRsCfg) {
        const int64_t cfg = base + cs;
        const bool active = cfg < n;
        Key x;
        x.lo = active ? keys[2 * cfg] : 0ull;
        x.hi = active ? keys[2 * cfg + 1] : 0ull;
        // token of position q (orbital K-1-q) = up bit + 2 down bit, as two
        // wave-uniform 64-bit masks over positions
        const bool inq = l < K;
        const uint64_t upm = __ballot(inq && key_bit(x, 2 * (K - 1 - l)));
        const uint64_t dnm = __ballot(inq && key_bit(x, 2 * (K - 1 - l) + 1));
        auto token = [&](int q) -> int { return (int)((upm >> q) & 1ull) | ((int)((dnm >> q) & 1ull) << 1); };
        // embeddings of the own rows: h[s][c] = tok_emb[prev token][c] + pos_emb[s][c], padding rows 0
        Tile32 h;
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int s = (j ? rb1 : rb0) * 16 + r0 + i;
                const int prev = s == 0 ? 4 : (s < K ? token(s - 1) : 0);
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    const int c = cb * 16 + c16;
                    h.t[j * 4 + cb][i] = s < K ? wf[M.fl.tok_emb + prev * kD + c] + wf[M.fl.pos_emb + s * kD + c] : 0.f;
                }
            }

        for (int layer = 0; layer < M.L; layer++) {
            const float *lv = wf + M.fl.layer0 + layer * M.fl.layer_stride;
            const __bf16 *lw = M.wb + M.bl.layer0 + layer * M.bl.layer_stride;
            layer_norm_rows(h, lv + kV_ln1_g, lv + kV_ln1_b, X, rb0, rb1);
            __syncthreads();  // previous users of wbuf are done
            stage_rows(wbuf, kLd, lw, 64, 192, 64);
            __syncthreads();
            for (int hh = 0; hh < kH; hh++) {
                // q, k, v columns of this head for the own rows: one column tile each
                f32x4 q[2], kk[2], v[2];
#pragma unroll
                for (int j = 0; j < 2; j++) q[j] = kk[j] = v[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 64; ks += 32) {
                    const bf16x8 bq = lds_frag(wbuf, hh * kDh + c16, kLd, ks + kq);
                    const bf16x8 bk = lds_frag(wbuf, 64 + hh * kDh + c16, kLd, ks + kq);
                    const bf16x8 bv = lds_frag(wbuf, 128 + hh * kDh + c16, kLd, ks + kq);
#pragma unroll
                    for (int j = 0; j < 2; j++) {
                        const bf16x8 a = lds_frag(X, (j ? rb1 : rb0) * 16 + c16, kLd, ks + kq);
                        q[j] = mfma16(a, bq, q[j]);
                        kk[j] = mfma16(a, bk, kk[j]);
                        v[j] = mfma16(a, bv, v[j]);
                    }
                }
                const float bqc = lv[kV_bqkv + hh * kDh + c16], bkc = lv[kV_bqkv + 64 + hh * kDh + c16],
                            bvc = lv[kV_bqkv + 128 + hh * kDh + c16];
                // Q, K row-major [position][dim]; V transposed [dim][position]
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const int s = (j ? rb1 : rb0) * 16 + r0 + i;
                        // 1/sqrt(16) and log2(e) folded into Q: the scores come out in
                        // base-2 units and the softmax takes exp2 directly
                        Qs[s * kQLd + c16] = (__bf16)((q[j][i] + bqc) * (0.25f * 1.44269504f));
                        Ks[s * kQLd + c16] = (__bf16)(kk[j][i] + bkc);
                        Vt[c16 * kLd + s] = (__bf16)(v[j][i] + bvc);
                    }
                __syncthreads();  // K and V of both halves written
                if (hf == 0) {
                    attend_block<0>(Qs, Ks, Vt, Pb, Ob, hh);
                    attend_block<3>(Qs, Ks, Vt, Pb, Ob, hh);
                } else {
                    attend_block<1>(Qs, Ks, Vt, Pb, Ob, hh);
                    attend_block<2>(Qs, Ks, Vt, Pb, Ob, hh);
                }
                __syncthreads();  // both halves done with this head's K and V (and the QKV weights)
            }
            stage_rows(wbuf, kLd, lw + 192 * 64, 64, 64, 64);
            __syncthreads();
            gemm_rows(h, Ob, rb0, rb1, wbuf, kLd, 64);
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                const float bo = lv[kV_bo + cb * 16 + c16];
#pragma unroll
                for (int j = 0; j < 2; j++) h.t[j * 4 + cb] += bo;
            }
            layer_norm_rows(h, lv + kV_ln2_g, lv + kV_ln2_b, X, rb0, rb1);
            // FFN in four hidden chunks of 64
            for (int chunk = 0; chunk < 4; chunk++) {
                __syncthreads();
                stage_rows(wbuf, kLd, lw + 192 * 64 + 64 * 64 + chunk * 64 * 64, 64, 64, 64);  // w1T rows
                stage_rows(wbuf + 64 * kLd, kLd, lw + 192 * 64 + 64 * 64 + 256 * 64 + chunk * 64, 256, 64, 64);
                __syncthreads();
                Tile32 f;
#pragma unroll
                for (int t = 0; t < 8; t++) f.t[t] = f32x4{0.f, 0.f, 0.f, 0.f};
                gemm_rows(f, X, rb0, rb1, wbuf, kLd, 64);
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    const float b1 = lv[kV_b1 + chunk * 64 + cb * 16 + c16];
#pragma unroll
                    for (int j = 0; j < 2; j++)
#pragma unroll
                        for (int i = 0; i < 4; i++)
                            Ob[((j ? rb1 : rb0) * 16 + r0 + i) * kLd + cb * 16 + c16] =
                                (__bf16)gelu_tab(gtab, f.t[j * 4 + cb][i] + b1);
                }
                wave_lds_sync();
                gemm_rows(h, Ob, rb0, rb1, wbuf + 64 * kLd, kLd, 64);
            }
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                const float b2 = lv[kV_b2 + cb * 16 + c16];
#pragma unroll
                for (int j = 0; j < 2; j++) h.t[j * 4 + cb] += b2;
            }
        }
        // final LayerNorm, head, mask, log-probability of the actual tokens (own rows)
        float lsum = 0.f;
        {
            const float *g = wf + M.fl.lnf_g, *b = wf + M.fl.lnf_b, *hw = wf + M.fl.head_w;
#pragma unroll
            for (int j = 0; j < 2; j++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    float rs = 0.f;
#pragma unroll
                    for (int cb = 0; cb < 4; cb++) rs += h.t[j * 4 + cb][i];
                    const float mean = dpp_row_sum(rs) * (1.0f / kD);
                    float v = 0.f;
#pragma unroll
                    for (int cb = 0; cb < 4; cb++) {
                        const float dlt = h.t[j * 4 + cb][i] - mean;
                        v += dlt * dlt;
                    }
                    const float rstd = rsqrtf(dpp_row_sum(v) * (1.0f / kD) + 1e-5f);
                    float z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int cb = 0; cb < 4; cb++) {
                        const int c = cb * 16 + c16;
                        const float y = (h.t[j * 4 + cb][i] - mean) * rstd * g[c] + b[c];
#pragma unroll
                        for (int t = 0; t < 4; t++) z[t] += y * hw[c * 4 + t];
                    }
#pragma unroll
                    for (int t = 0; t < 4; t++) z[t] = dpp_row_sum(z[t]);
                    const int s = (j ? rb1 : rb0) * 16 + r0 + i;
                    if (c16 == 0 && s < K) {
                        const uint64_t below = (1ull << s) - 1ull;  // s < K <= 64
                        const int up = __popcll(upm & below), dn = __popcll(dnm & below);
                        const int rem = K - 1 - s, orb = K - 1 - s;
                        float mx = -INFINITY;
                        bool ok[4];
#pragma unroll
                        for (int t = 0; t < 4; t++) {
                            z[t] += wf[M.fl.head_b + t] + wf[M.fl.bias + orb * 4 + t];
                            const int bu = t & 1, bd = t >> 1;
                            ok[t] = (up + bu <= M.n_up) && (dn + bd <= M.n_dn) && (M.n_up - up - bu <= rem) &&
                                    (M.n_dn - dn - bd <= rem);
                            if (ok[t]) mx = fmaxf(mx, z[t]);
                        }
                        float den = 0.f;
#pragma unroll
                        for (int t = 0; t < 4; t++)
                            if (ok[t]) den += __expf(z[t] - mx);
                        const int ts = token(s);
                        lsum += ok[ts] ? (z[ts] - mx) - __logf(den) : -INFINITY;
                    }
                }
        }
        // rows live in lanes 0, 16, 32, 48; then the two halves of the configuration
        lsum += __shfl_xor(lsum, 16, 64);
        lsum += __shfl_xor(lsum, 32, 64);
        if (l == 0) red[w] = lsum;
        __syncthreads();
        if (active && hf == 0 && l == 0) logabs[cfg] = 0.5 * ((double)red[w] + (double)red[w + 1]);
    }
}

// Phase MLP: 16 configurations per wave, B tiles from global (L2) memory.
__global__ void __launch_bounds__(256) k_phase_bf16(Bf16View M, const uint64_t *__restrict__ keys, int64_t n,
                                                    double *__restrict__ phase) {
    __shared__ __align__(16) __bf16 zs[kWaves][16 * (kP + 8)];
    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    __bf16 *Z = zs[w];
    const int zld = kP + 8;
    const __bf16 *w1T = M.wb + M.bl.ph_w1T, *w2T = M.wb + M.bl.ph_w2T;
    const float *b1 = M.wf + M.fl.ph_b1, *b2 = M.wf + M.fl.ph_b2, *w3 = M.wf + M.fl.ph_w3;
    const int nbits = 2 * M.K;
    for (int64_t base = ((int64_t)blockIdx.x * kWaves + w) * 16; base < n; base += (int64_t)gridDim.x * kWaves * 16) {
        // A tiles of the bit matrix: row = configuration (c16), k = bit index
        const int64_t cr = base + c16;
        Key x;
        x.lo = cr < n ? keys[2 * cr] : 0ull;
        x.hi = cr < n ? keys[2 * cr + 1] : 0ull;
        bf16x8 abits[kPhaseBits / 32];
#pragma unroll
        for (int ks = 0; ks < kPhaseBits / 32; ks++)
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int p = ks * 32 + kq + e;
                abits[ks][e] = (__bf16)((p < nbits && key_bit(x, p)) ? 1.0f : 0.0f);
            }
        // z1 = GELU(bits @ W1 + b1) -> Z (BF16)
        for (int nb = 0; nb < kP / 16; nb++) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kPhaseBits / 32; ks++) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(w1T + (int64_t)(nb * 16 + c16) * kPhaseBits + ks * 32 + kq);
                acc = mfma16(abits[ks], b, acc);
            }
            const float bb = b1[nb * 16 + c16];
#pragma unroll
            for (int i = 0; i < 4; i++) Z[(r0 + i) * zld + nb * 16 + c16] = (__bf16)gelu32(acc[i] + bb);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // phi = GELU(z1 @ W2 + b2) . w3 + b3
        float part[4] = {0.f, 0.f, 0.f, 0.f};
        for (int nb = 0; nb < kP / 16; nb++) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < kP; ks += 32) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(Z + c16 * zld + ks + kq);
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(w2T + (int64_t)(nb * 16 + c16) * kP + ks + kq);
                acc = mfma16(a, b, acc);
            }
            const float bb = b2[nb * 16 + c16], ww = w3[nb * 16 + c16];
#pragma unroll
            for (int i = 0; i < 4; i++) part[i] += gelu32(acc[i] + bb) * ww;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) part[i] = dpp_row_sum(part[i]);
        if (c16 == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t cfg = base + r0 + i;
                if (cfg < n) phase[cfg] = (double)(part[i] + M.wf[M.fl.ph_b3]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

static Bf16View bf16_view(const nnqs_model *m) {
    Bf16View v{};
    v.K = m->desc.n_orb;
    v.L = m->desc.n_layers;
    v.n_up = m->desc.n_up;
    v.n_dn = m->desc.n_dn;
    v.wb = reinterpret_cast<const __bf16 *>(m->d_bf16);
    v.wf = m->d_f32;
    v.bl = bf16_layout(v.L);
    v.fl = f32_layout(v.K, v.L);
    return v;
}

static uint16_t to_bf16_bits(float f) {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

nnqs_status bf16_model_init(nnqs_model *m, const float *weights) {
    const nnqs_model_desc &d = m->desc;
    m->bf16_ok = d.d_model == kD && d.n_heads == kH && d.d_ff == kF && d.phase_hidden == kP && d.n_orb <= 64 &&
                 2 * d.n_orb <= kPhaseBits;
    if (!m->bf16_ok) return NNQS_OK;
    const int K = d.n_orb, L = d.n_layers;
    const ModelOffsets &o = m->off;
    const Bf16Layout bl = bf16_layout(L);
    const F32Layout fl = f32_layout(K, L);
    std::vector<uint16_t> wb((size_t)bl.total, 0);
    std::vector<float> wf((size_t)fl.total, 0.f);
    auto W = [&](int64_t off) { return weights + off; };
    // transposed copy: dst[n][k] = src[k][n] for a [kdim][ndim] source matrix
    auto put_t = [&](int64_t dst, int dst_ld, const float *src, int kdim, int ndim, int row0) {
        for (int k = 0; k < kdim; k++)
            for (int nn = 0; nn < ndim; nn++) wb[dst + (int64_t)(row0 + nn) * dst_ld + k] = to_bf16_bits(src[k * ndim + nn]);
    };
    for (int l = 0; l < L; l++) {
        const int64_t lo = o.layer0 + l * o.layer_stride;
        const int64_t base = bl.layer0 + l * bl.layer_stride;
        const int64_t dd = kD * kD;
        // layer block layout of the FP32 weights: ln1_g ln1_b wq bq wk bk wv bv wo bo ln2_g ln2_b w1 b1 w2 b2
        const float *wq = W(lo + 2 * kD), *bq = wq + dd, *wk = bq + kD, *bk = wk + dd, *wv = bk + kD, *bv = wv + dd,
                    *wo = bv + kD, *bo = wo + dd, *ln2g = bo + kD, *ln2b = ln2g + kD, *w1 = ln2b + kD,
                    *b1 = w1 + kD * kF, *w2 = b1 + kF, *b2 = w2 + kF * kD;
        put_t(base, 64, wq, kD, kD, 0);
        put_t(base, 64, wk, kD, kD, 64);
        put_t(base, 64, wv, kD, kD, 128);
        put_t(base + 192 * 64, 64, wo, kD, kD, 0);
        put_t(base + 192 * 64 + 64 * 64, 64, w1, kD, kF, 0);
        put_t(base + 192 * 64 + 64 * 64 + 256 * 64, 256, w2, kF, kD, 0);
        float *lv = wf.data() + fl.layer0 + l * fl.layer_stride;
        std::memcpy(lv + kV_ln1_g, W(lo), kD * 4);
        std::memcpy(lv + kV_ln1_b, W(lo + kD), kD * 4);
        std::memcpy(lv + kV_bqkv, bq, kD * 4);
        std::memcpy(lv + kV_bqkv + 64, bk, kD * 4);
        std::memcpy(lv + kV_bqkv + 128, bv, kD * 4);
        std::memcpy(lv + kV_bo, bo, kD * 4);
        std::memcpy(lv + kV_ln2_g, ln2g, kD * 4);
        std::memcpy(lv + kV_ln2_b, ln2b, kD * 4);
        std::memcpy(lv + kV_b1, b1, kF * 4);
        std::memcpy(lv + kV_b2, b2, kD * 4);
    }
    std::memcpy(wf.data() + fl.tok_emb, W(o.tok_emb), 5 * kD * 4);
    std::memcpy(wf.data() + fl.pos_emb, W(o.pos_emb), (size_t)K * kD * 4);
    std::memcpy(wf.data() + fl.lnf_g, W(o.lnf_g), kD * 4);
    std::memcpy(wf.data() + fl.lnf_b, W(o.lnf_b), kD * 4);
    std::memcpy(wf.data() + fl.head_w, W(o.head_w), 4 * kD * 4);
    std::memcpy(wf.data() + fl.head_b, W(o.head_b), 4 * 4);
    std::memcpy(wf.data() + fl.bias, W(o.bias), (size_t)4 * K * 4);
    std::memcpy(wf.data() + fl.ph_b1, W(o.ph_b1), kP * 4);
    std::memcpy(wf.data() + fl.ph_b2, W(o.ph_b2), kP * 4);
    std::memcpy(wf.data() + fl.ph_w3, W(o.ph_w3), kP * 4);
    wf[fl.ph_b3] = *W(o.ph_b3);
    for (int i = 0; i < kGeluN; i++) {  // Phi at the knots, in FP64
        const double v0 = (i - (double)kGeluOff) / kGeluScale, v1 = v0 + 1.0 / kGeluScale;
        const double p0 = 0.5 * std::erfc(-v0 / std::sqrt(2.0)), p1 = 0.5 * std::erfc(-v1 / std::sqrt(2.0));
        wf[fl.gelu + 2 * i] = (float)p0;
        wf[fl.gelu + 2 * i + 1] = (float)(p1 - p0);
    }
    // phase W1 [2K][512] -> ph_w1T[512][128] (bits beyond 2K stay zero)
    put_t(bl.ph_w1T, kPhaseBits, W(o.ph_w1), 2 * K, kP, 0);
    put_t(bl.ph_w2T, kP, W(o.ph_w2), kP, kP, 0);
    if (hipMalloc(&m->d_bf16, wb.size() * 2) != hipSuccess || hipMalloc(&m->d_f32, wf.size() * 4) != hipSuccess)
        return fail(NNQS_ENOMEM, "device allocation of the BF16 model failed");
    if (hipMemcpy(m->d_bf16, wb.data(), wb.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_f32, wf.data(), wf.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(NNQS_EHIP, "copy of the BF16 model failed");
    return NNQS_OK;
}

void bf16_model_free(nnqs_model *m) {
    hipFree(m->d_bf16);
    hipFree(m->d_f32);
    m->d_bf16 = nullptr;
    m->d_f32 = nullptr;
}

nnqs_status enqueue_logpsi_bf16(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, double *phase,
                                hipStream_t st) {
    if (!m->bf16_ok) return fail(NNQS_EUNSUPPORTED, "BF16 forward needs d_model 64, 4 heads, FFN 256, P 512, K <= 64");
    const Bf16View v = bf16_view(m);
    int dev = 0, cus = 256;
    NNQS_HIP_CHECK(hipGetDevice(&dev));
    NNQS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t cap = (int64_t)cus * 8;
    int64_t blocks = (n + kRsCfg - 1) / kRsCfg;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_transformer_bf16, dim3((unsigned)blocks), dim3(kRsWaves * 64), 0, st, v, keys, n, logabs);
    int64_t pblocks = (n + kWaves * 16 - 1) / (kWaves * 16);
    if (pblocks > cap) pblocks = cap;
    hipLaunchKernelGGL(k_phase_bf16, dim3((unsigned)pblocks), dim3(kWaves * 64), 0, st, v, keys, n, phase);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

}  // namespace nnqs

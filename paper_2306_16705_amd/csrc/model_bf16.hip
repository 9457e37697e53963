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
// Phase MLP: a second kernel runs bits[128 x 128] @ W1 and
// GELU(z1)[128 x 512] @ W2 on the same MFMA for 128 configurations per block,
// each wave owning 64 output columns (weight fragments from L2, read once per
// block pass; z1 in LDS).
#include <algorithm>
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
    o.layer_stride = 2 * kD + 192 + kD + 2 * kD + kF + kD + 12;
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
// FP8 scales of one layer's six weight matrices (q, k, v, o, w1, w2): for
// each, the power of two s applied before quantisation and 1/s.
constexpr int kV_f8 = 832;

struct Bf16View {
    int K, L, n_up, n_dn;
    const __bf16 *wb;
    const uint8_t *w8;  // FP8 E4M3 copy of the transformer matrices, same element layout as wb
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

// Operands of the four weight products (QKV, output, FFN in and out):
// BF16 on v_mfma_f32_16x16x32_bf16, or OCP FP8 E4M3 bytes on
// v_mfma_f32_16x16x32_fp8_fp8 (same lane layout, eight 1-byte elements per
// lane; activations are not scaled, each weight matrix has a power-of-two
// scale that the accumulators undo).
template <bool kF8>
struct Op;

template <>
struct Op<false> {
    typedef __bf16 T;
    typedef bf16x8 Frag;
    static constexpr int ld = kLd;  // padded LDS row length of 64-wide tiles
    static __device__ __forceinline__ Frag frag(const T *base, int row, int k0) { return lds_frag(base, row, ld, k0); }
    static __device__ __forceinline__ f32x4 mma(const Frag &a, const Frag &b, const f32x4 &c) { return mfma16(a, b, c); }
    static __device__ __forceinline__ T cvt(float v) { return (__bf16)v; }
};

template <>
struct Op<true> {
    typedef uint8_t T;
    typedef long Frag;
    static constexpr int ld = 80;  // bytes; keeps 16-byte staging stores aligned
    static __device__ __forceinline__ Frag frag(const T *base, int row, int k0) {
        return *reinterpret_cast<const long *>(base + row * ld + k0);
    }
    static __device__ __forceinline__ f32x4 mma(const Frag &a, const Frag &b, const f32x4 &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ T cvt(float v) {  // E4M3, round to nearest even, saturated at 448
        return (T)(__builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v, -448.f, 448.f), 0.f, 0, false) & 0xff);
    }
};

__device__ __forceinline__ uint32_t fp8x4(const f32x4 &v) {
    int r = 0;
    r = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v[0], -448.f, 448.f),
                                        __builtin_amdgcn_fmed3f(v[1], -448.f, 448.f), r, false);
    r = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v[2], -448.f, 448.f),
                                        __builtin_amdgcn_fmed3f(v[3], -448.f, 448.f), r, true);
    return (uint32_t)r;
}

// Cooperative copy of `rows` rows of `cols` operands (global, row stride
// gld) into LDS rows of stride lld, in 16-byte pieces.
template <typename T>
__device__ __forceinline__ void stage_rows_t(T *dst, int lld, const T *src, int gld, int rows, int cols) {
    constexpr int per16 = 16 / (int)sizeof(T);
    const int per_row = cols / per16;
    for (int e = threadIdx.x; e < rows * per_row; e += blockDim.x) {
        const int rr = e / per_row, cc = (e - rr * per_row) * per16;
        *reinterpret_cast<uint4 *>(dst + rr * lld + cc) = *reinterpret_cast<const uint4 *>(src + (int64_t)rr * gld + cc);
    }
}

// ------------------------------------------------------ transformer forward
// Work of one launch, in one of two modes.
//  * Sample mode: configurations keys[0..n), every row evaluated; log|psi|
//    to logabs[i].  With `kv_out` and `pre_out` it also keeps, per configuration,
//    every layer's keys and values (BF16, as the attention used them) and the
//    prefix sums pre[i][b] of its per-position log-probabilities over the
//    first 16 b positions: the cache that list mode reads.
//  * List mode: connected configurations x' of cached samples, as chunk-local
//    connection indices e (key xkeys[e], sample e / C) sorted into four
//    classes (hdr = {count[4], offset[4]} on the device).  Class b holds the
//    x' whose first position that differs from their sample lies at or after
//    16 b: by causality the rows s <= 16 b of x' equal the sample's, so only
//    row blocks b..3 are evaluated; their attention reads the keys and values
//    of blocks < b from the sample's cache, and the log-probabilities of
//    positions < 16 b are the sample's prefix sum.  log|psi| goes to xla[e].
//    Results are bit-identical to sample mode on x' (same per-row arithmetic,
//    same summation order).
struct TfArgs {
    const uint64_t *keys;
    int64_t n;
    double *logabs;
    __bf16 *kv_out;        // sample mode: cache written (may be null)
    double *pre_out;
    const __bf16 *kv_in;   // list mode: cache read
    const double *pre_in;
    const int32_t *list;
    const int64_t *hdr;
    const uint64_t *xkeys;
    int64_t C;
    double *xla;
    int list_mode;
    int cond_pos;      // sample mode, batch sampling: position whose conditionals are written
    double *cond_out;  // [n][4] masked log-probabilities of the four tokens there (may be null)
};

// A block evaluates one tile of 16 row-block slots (16 rows each), two per
// wave.  Class-0 tiles hold four configurations, wave pair (2c, 2c+1) owning
// configuration c's row blocks {0, 3} and {1, 2} (row block b attends to
// b + 1 key blocks, and 1 + 4 = 2 + 3); class b > 0 tiles hold
// floor(16 / (4 - b)) configurations whose blocks b..3 fill consecutive slots.
constexpr int kSlots = 16;
constexpr int kVLd = 24;  // padded row length of a slot's V^T (16 keys)
constexpr int kKvPerHead = 64 * kDh + kDh * 64;  // cached K [64][16] then V^T [16][64]

__device__ __forceinline__ int cls_cpt(int cls) { return cls == 0 ? 4 : cls == 1 ? 5 : cls == 2 ? 8 : 16; }

__device__ __forceinline__ void slot_info(int cls, int q, int &c, int &rb) {
    if (cls == 0) {
        c = q >> 2;
        const int r = q & 3;
        rb = r == 0 ? 0 : r == 1 ? 3 : r == 2 ? 1 : 2;
    } else {
        const int nb = 4 - cls;
        c = q / nb;
        rb = cls + (q - c * nb);
    }
}

__device__ __forceinline__ int slot_of(int cls, int c, int kb) {
    if (cls == 0) return 4 * c + (kb == 0 ? 0 : kb == 1 ? 2 : kb == 2 ? 3 : 1);
    return c * (4 - cls) + (kb - cls);
}

struct Tile32 {
    f32x4 t[8];  // tile (j, cb) = t[j * 4 + cb]: own slot j, column block cb
};

// acc += X_j[16 rows][0..k_len) (LDS, row stride Op::ld) @ W for both own
// slots, Wt[n][k] in LDS.
template <bool kF8>
__device__ __forceinline__ void gemm_slots(Tile32 &acc, const typename Op<kF8>::T *X0, const typename Op<kF8>::T *X1,
                                           const typename Op<kF8>::T *Wt, int k_len) {
    typedef Op<kF8> OP;
    const int l = threadIdx.x & 63;
    const int r = l & 15, kq = 8 * (l >> 4);
    for (int ks = 0; ks < k_len; ks += 32) {
        typename OP::Frag a[2], b[4];
        a[0] = OP::frag(X0, r, ks + kq);
        a[1] = OP::frag(X1, r, ks + kq);
#pragma unroll
        for (int cb = 0; cb < 4; cb++) b[cb] = OP::frag(Wt, cb * 16 + r, ks + kq);
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int cb = 0; cb < 4; cb++) acc.t[j * 4 + cb] = OP::mma(a[j], b[cb], acc.t[j * 4 + cb]);
    }
}

// Normalised rows (h - mean) / sqrt(var + eps) of both own slots into X_j
// (LDS).  The LayerNorm's scale and shift are folded into the weights of the
// product that reads X.
template <bool kF8>
__device__ __forceinline__ void normalize_rows(const Tile32 &h, typename Op<kF8>::T *X0, typename Op<kF8>::T *X1) {
    typedef Op<kF8> OP;
    const int l = threadIdx.x & 63;
    const int c = l & 15, r0 = 4 * (l >> 4);
#pragma unroll
    for (int j = 0; j < 2; j++) {
        typename OP::T *X = j ? X1 : X0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float s = 0.f, s2 = 0.f;
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                const float v = h.t[j * 4 + cb][i];
                s += v;
                s2 = fmaf(v, v, s2);
            }
            const float mean = dpp_row_sum(s) * (1.0f / kD);
            const float var = fmaxf(dpp_row_sum(s2) * (1.0f / kD) - mean * mean, 0.0f);
            const float rstd = rsqrtf(var + 1e-5f);
            const float sh = -mean * rstd;
#pragma unroll
            for (int cb = 0; cb < 4; cb++) X[(r0 + i) * OP::ld + cb * 16 + c] = OP::cvt(fmaf(h.t[j * 4 + cb][i], rstd, sh));
        }
    }
}

// The residual stream is kept transposed: tile t[j * 4 + db] of slot j holds,
// in lane l, sequence row (l & 15) of the slot and model columns
// 16 db + 4 (l >> 4) + i, i = 0..3.  Products that feed it are computed as
// C^T = W^T A^T (weights as the A operand, activations as the B operand), so
// each lane's four outputs are consecutive columns of one row: LDS stores of
// normalised rows and GELU outputs are one 8-byte write per four values.
// acc^T += W^T X_j^T for both own slots; Wt[n][k] in LDS, X_j row-major.
template <bool kF8>
__device__ __forceinline__ void gemm_slots_t(Tile32 &acc, const typename Op<kF8>::T *X0, const typename Op<kF8>::T *X1,
                                             const typename Op<kF8>::T *Wt, int k_len) {
    typedef Op<kF8> OP;
    const int l = threadIdx.x & 63;
    const int r = l & 15, kq = 8 * (l >> 4);
    for (int ks = 0; ks < k_len; ks += 32) {
        typename OP::Frag a[4], b[2];
        b[0] = OP::frag(X0, r, ks + kq);
        b[1] = OP::frag(X1, r, ks + kq);
#pragma unroll
        for (int db = 0; db < 4; db++) a[db] = OP::frag(Wt, db * 16 + r, ks + kq);
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int db = 0; db < 4; db++) acc.t[j * 4 + db] = OP::mma(a[db], b[j], acc.t[j * 4 + db]);
    }
}

// Four consecutive values of one row into LDS (BF16, or FP8 E4M3).
template <bool kF8>
__device__ __forceinline__ void store4(typename Op<kF8>::T *dst, const f32x4 &v);
template <>
__device__ __forceinline__ void store4<false>(__bf16 *dst, const f32x4 &v) {
    bf16x4 o;
#pragma unroll
    for (int i = 0; i < 4; i++) o[i] = (__bf16)v[i];
    *reinterpret_cast<bf16x4 *>(dst) = o;
}
template <>
__device__ __forceinline__ void store4<true>(uint8_t *dst, const f32x4 &v) {
    int r = 0;
    r = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v[0], -448.f, 448.f),
                                        __builtin_amdgcn_fmed3f(v[1], -448.f, 448.f), r, false);
    r = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(v[2], -448.f, 448.f),
                                        __builtin_amdgcn_fmed3f(v[3], -448.f, 448.f), r, true);
    *reinterpret_cast<int *>(dst) = r;
}

// Mean and 1/sqrt(var + eps) of the row of slot j held by this lane's group
// of four lanes (l, l ^ 16, l ^ 32, l ^ 48), one-pass statistics.
__device__ __forceinline__ void row_stats_t(const Tile32 &h, int j, float &rstd, float &shift) {
    float s = 0.f, s2 = 0.f;
#pragma unroll
    for (int db = 0; db < 4; db++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float v = h.t[j * 4 + db][i];
            s += v;
            s2 = fmaf(v, v, s2);
        }
    s += __shfl_xor(s, 16, 64);
    s2 += __shfl_xor(s2, 16, 64);
    s += __shfl_xor(s, 32, 64);
    s2 += __shfl_xor(s2, 32, 64);
    const float mean = s * (1.0f / kD);
    const float var = fmaxf(s2 * (1.0f / kD) - mean * mean, 0.0f);
    rstd = rsqrtf(var + 1e-5f);
    shift = -mean * rstd;
}

// Normalised rows of both own slots into X_j (LDS, row-major); the
// LayerNorm's scale and shift are folded into the next product's weights.
template <bool kF8>
__device__ __forceinline__ void normalize_rows_t(const Tile32 &h, typename Op<kF8>::T *X0, typename Op<kF8>::T *X1) {
    const int l = threadIdx.x & 63;
    const int c16 = l & 15, r0 = 4 * (l >> 4);
#pragma unroll
    for (int j = 0; j < 2; j++) {
        float rstd, sh;
        row_stats_t(h, j, rstd, sh);
        typename Op<kF8>::T *X = (j ? X1 : X0) + c16 * Op<kF8>::ld + r0;
#pragma unroll
        for (int db = 0; db < 4; db++) {
            f32x4 y;
#pragma unroll
            for (int i = 0; i < 4; i++) y[i] = fmaf(h.t[j * 4 + db][i], rstd, sh);
            store4<kF8>(X + db * 16, y);
        }
    }
}

__device__ __forceinline__ f32x4 ld4(const float *p) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return f32x4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x4 cvt4(const f32x4 &v) {
    bf16x4 o;
#pragma unroll
    for (int i = 0; i < 4; i++) o[i] = (__bf16)v[i];
    return o;
}

// Where the keys and values of one configuration's key blocks live for
// one head: blocks < sb in the sample's cache (global), the others in the
// tile's slots (LDS).
struct KvSrc {
    const __bf16 *kc, *vc;  // cached K [64][16] and V^T [16][64] of this head (blocks < sb)
    const __bf16 *ks, *vt;  // LDS slot arrays of the tile
    int cls, c, sb;
};

// Causal attention of query block QB (a slot of configuration c) for one
// head: S^T[key][query] = K Q^T (the lane owns query c16 + 16 QB and keys
// 16 kb + r0 + i), softmax over keys in base 2 (scale and log2(e) are folded
// into Q): unnormalised P[query][key] -> Pb, then O^T[c][query] = V^T P^T
// divided by the row sums 1^T P^T (the same MFMA with an all-ones operand)
// into Oq[query][16 hh + c].
template <int QB, bool kF8>
__device__ __forceinline__ void attend_block(const __bf16 *Qq, const KvSrc &S, __bf16 *Pb, typename Op<kF8>::T *Oq,
                                             int hh) {
    const int l = threadIdx.x & 63;
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    const bf16x8 zero8 = {};
    const bf16x8 bqf = l < 32 ? lds_frag(Qq, c16, kQLd, kq) : zero8;
    f32x4 st[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        st[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (kb <= QB) {
            bf16x8 akf = zero8;
            if (l < 32) {
                if (kb < S.sb) akf = *reinterpret_cast<const bf16x8 *>(S.kc + (kb * 16 + c16) * kDh + kq);
                else akf = lds_frag(S.ks + slot_of(S.cls, S.c, kb) * (16 * kQLd), c16, kQLd, kq);
            }
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
    // unnormalised weights p = 2^(s - max) in BF16; the denominator of each
    // query is the sum of the same BF16 values, taken by one more MFMA with an
    // all-ones operand, and divides the output (four values per lane)
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        bf16x4 pk;
#pragma unroll
        for (int i = 0; i < 4; i++)
            pk[i] = (__bf16)((kb < QB || (kb == QB && r0 + i <= c16)) ? __builtin_amdgcn_exp2f(st[kb][i] - mx) : 0.f);
        *reinterpret_cast<bf16x4 *>(Pb + c16 * kLd + kb * 16 + r0) = pk;
    }
    wave_lds_sync();
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; e++) ones[e] = (__bf16)1.0f;
    f32x4 ot = {0.f, 0.f, 0.f, 0.f}, den = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 64; ks += 32) {
        if (ks <= QB * 16 + 15) {
            const int kb = (ks >> 4) + (kq >> 4);  // key block of this lane's eight keys
            bf16x8 av;
            if (kb < S.sb) av = *reinterpret_cast<const bf16x8 *>(S.vc + c16 * 64 + ks + kq);
            else av = *reinterpret_cast<const bf16x8 *>(S.vt + slot_of(S.cls, S.c, kb) * (kDh * kVLd) + c16 * kVLd + (kq & 15));
            const bf16x8 bp = lds_frag(Pb, c16, kLd, ks + kq);
            ot = mfma16(av, bp, ot);
            den = mfma16(ones, bp, den);
        }
    }
    ot *= __builtin_amdgcn_rcpf(den[0]);
    if constexpr (kF8)
        *reinterpret_cast<uint32_t *>(Oq + c16 * Op<true>::ld + hh * kDh + r0) = fp8x4(ot);
    else
        *reinterpret_cast<bf16x4 *>(Oq + c16 * kLd + hh * kDh + r0) = cvt4(ot);
    wave_lds_sync();  // Pb is rewritten by the next block
}

template <bool kF8>
__device__ __forceinline__ void attend(int QB, const __bf16 *Qq, const KvSrc &S, __bf16 *Pb, typename Op<kF8>::T *Oq,
                                       int hh) {
    switch (QB) {
        case 0: attend_block<0, kF8>(Qq, S, Pb, Oq, hh); break;
        case 1: attend_block<1, kF8>(Qq, S, Pb, Oq, hh); break;
        case 2: attend_block<2, kF8>(Qq, S, Pb, Oq, hh); break;
        default: attend_block<3, kF8>(Qq, S, Pb, Oq, hh); break;
    }
}

// One item of a batched list-mode launch: a system's model and work.
struct TfItem {
    Bf16View M;
    TfArgs A;
};
constexpr int kMaxTfItems = 64;

template <bool kList, bool kF8, bool kBatch>
__device__ __forceinline__ void transformer_bf16(const Bf16View &M0, const TfArgs &A0, const TfItem *items,
                                                 int n_items) {
    typedef Op<kF8> OP;
    typedef typename OP::T AT;
    constexpr int kLdA = OP::ld;
    __shared__ __align__(16) AT wbuf[192 * kLdA];
    __shared__ __align__(16) float2 gtab[kGeluN];
    __shared__ __align__(16) AT xs[kSlots][16 * kLdA];
    __shared__ __align__(16) AT os[kSlots][16 * kLdA];
    __shared__ __align__(16) __bf16 qs[kSlots][16 * kQLd];
    __shared__ __align__(16) __bf16 ks_[kSlots][16 * kQLd];
    __shared__ __align__(16) __bf16 vt[kSlots][kDh * kVLd];
    __shared__ __align__(16) __bf16 ps[8][16 * kLd];
    __shared__ double slot_lp[kSlots];
    __shared__ int64_t sh_hdr[8];
    // batched launch: first global tile of every (item, class), in item-major order
    __shared__ int64_t sh_tile0[kBatch ? 4 * kMaxTfItems + 1 : 1];

    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    __bf16 *Pb = ps[w];
    for (int i = threadIdx.x; i < kGeluN; i += blockDim.x)  // the same table in every model
        gtab[i] = make_float2(M0.wf[M0.fl.gelu + 2 * i], M0.wf[M0.fl.gelu + 2 * i + 1]);
    if (!kBatch && kList && threadIdx.x < 8) sh_hdr[threadIdx.x] = A0.hdr[threadIdx.x];
    if constexpr (kBatch) {
        if (threadIdx.x == 0) {
            int64_t acc = 0;
            for (int it = 0; it < n_items; it++)
                for (int c = 0; c < 4; c++) {
                    sh_tile0[4 * it + c] = acc;
                    acc += (items[it].A.hdr[c] + cls_cpt(c) - 1) / cls_cpt(c);
                }
            sh_tile0[4 * n_items] = acc;
        }
    }
    __syncthreads();
    int64_t tiles[4] = {0, 0, 0, 0}, T;
    if (kBatch) {
        T = sh_tile0[4 * n_items];
    } else if (kList) {
        T = 0;
        for (int c = 0; c < 4; c++) {
            tiles[c] = (sh_hdr[c] + cls_cpt(c) - 1) / cls_cpt(c);
            T += tiles[c];
        }
    } else {
        T = (A0.n + 3) / 4;
    }

    for (int64_t tile = blockIdx.x; tile < T; tile += gridDim.x) {
        int cls = 0;
        int64_t tb = tile * 4, cnt = A0.n, lbase = 0;
        Bf16View M = M0;
        TfArgs A = A0;
        if constexpr (kBatch) {
            int q = 0;  // the last (item, class) whose first tile is at or before `tile`
            for (int step = 4 * kMaxTfItems; step >= 1; step >>= 1)
                if (q + step < 4 * n_items && sh_tile0[q + step] <= tile) q += step;
            const int it = q >> 2;
            cls = q & 3;
            M = items[it].M;
            A = items[it].A;
            tb = (tile - sh_tile0[q]) * cls_cpt(cls);
            cnt = A.hdr[cls];
            lbase = A.hdr[4 + cls];
        } else if (kList) {
            int64_t tt = tile;
            cls = 3;
            for (int c = 0; c < 3; c++) {
                if (tt < tiles[c]) {
                    cls = c;
                    break;
                }
                tt -= tiles[c];
            }
            tb = tt * cls_cpt(cls);
            cnt = sh_hdr[cls];
            lbase = sh_hdr[4 + cls];
        }
        const int K = M.K;
        const float *wf = M.wf;
        const int64_t kv_cfg = (int64_t)M.L * kH * kKvPerHead;  // cache elements per configuration
        const int cpt = cls_cpt(cls);
        // the wave's two slots: configuration, row block, key, sample
        int sc[2], srb[2];
        uint64_t upm[2], dnm[2];
        int64_t ssmp[2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            slot_info(cls, 2 * w + j, sc[j], srb[j]);
            const bool valid = sc[j] < cpt && tb + sc[j] < cnt;
            Key x{0ull, 0ull};
            ssmp[j] = 0;
            if (valid) {
                if (kList) {
                    const int64_t e = A.list[lbase + tb + sc[j]];
                    x.lo = A.xkeys[2 * e];
                    x.hi = A.xkeys[2 * e + 1];
                    ssmp[j] = e / A.C;
                } else {
                    x.lo = A.keys[2 * (tb + sc[j])];
                    x.hi = A.keys[2 * (tb + sc[j]) + 1];
                }
            }
            // token of position q (orbital K-1-q) = up bit + 2 down bit, as
            // two wave-uniform 64-bit masks over positions
            const bool inq = l < K;
            upm[j] = __ballot(inq && key_bit(x, 2 * (K - 1 - l)));
            dnm[j] = __ballot(inq && key_bit(x, 2 * (K - 1 - l) + 1));
        }
        auto token = [&](int j, int q) -> int {
            return (int)((upm[j] >> q) & 1ull) | ((int)((dnm[j] >> q) & 1ull) << 1);
        };
        AT *X0 = xs[2 * w], *X1 = xs[2 * w + 1], *O0 = os[2 * w], *O1 = os[2 * w + 1];
        // embeddings of the own rows (transposed layout): h[s][c] = tok_emb[prev token][c] +
        // pos_emb[s][c], padding rows 0
        Tile32 h;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int s = srb[j] * 16 + c16;
            const int prev = s == 0 ? 4 : (s < K ? token(j, s - 1) : 0);
#pragma unroll
            for (int db = 0; db < 4; db++) {
                const int c = db * 16 + r0;
                h.t[j * 4 + db] = s < K ? ld4(wf + M.fl.tok_emb + prev * kD + c) + ld4(wf + M.fl.pos_emb + s * kD + c)
                                        : f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }

        for (int layer = 0; layer < M.L; layer++) {
            const float *lv = wf + M.fl.layer0 + layer * M.fl.layer_stride;
            const AT *lw = (kF8 ? reinterpret_cast<const AT *>(M.w8) : reinterpret_cast<const AT *>(M.wb)) +
                           M.bl.layer0 + layer * M.bl.layer_stride;
            // FP8: power-of-two scale s of each weight matrix and 1/s
            const float *f8 = lv + kV_f8;
            normalize_rows_t<kF8>(h, X0, X1);
            __syncthreads();  // previous users of wbuf are done
            stage_rows_t(wbuf, kLdA, lw, 64, 192, 64);
            __syncthreads();
            for (int hh = 0; hh < kH; hh++) {
                // Q^T and K^T (dims x positions) and V (positions x dims) of the
                // own slots, biases in the accumulators
                f32x4 qt[2], kt[2], v[2];
                const float bv = lv[kV_bqkv + 128 + hh * kDh + c16] * (kF8 ? f8[4] : 1.0f);
                f32x4 bq, bk;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    bq[i] = lv[kV_bqkv + hh * kDh + r0 + i] * (kF8 ? f8[0] : 1.0f);
                    bk[i] = lv[kV_bqkv + 64 + hh * kDh + r0 + i] * (kF8 ? f8[2] : 1.0f);
                }
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    qt[j] = bq;
                    kt[j] = bk;
                    v[j] = f32x4{bv, bv, bv, bv};
                }
#pragma unroll
                for (int ks = 0; ks < 64; ks += 32) {
                    const typename OP::Frag wq = OP::frag(wbuf, hh * kDh + c16, ks + kq);
                    const typename OP::Frag wk = OP::frag(wbuf, 64 + hh * kDh + c16, ks + kq);
                    const typename OP::Frag wv = OP::frag(wbuf, 128 + hh * kDh + c16, ks + kq);
#pragma unroll
                    for (int j = 0; j < 2; j++) {
                        const typename OP::Frag a = OP::frag(j ? X1 : X0, c16, ks + kq);
                        qt[j] = OP::mma(wq, a, qt[j]);
                        kt[j] = OP::mma(wk, a, kt[j]);
                        v[j] = OP::mma(a, wv, v[j]);
                    }
                }
                if constexpr (kF8) {
#pragma unroll
                    for (int j = 0; j < 2; j++) {
                        qt[j] *= f8[1];
                        kt[j] *= f8[3];
                        v[j] *= f8[5];
                    }
                }
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int q = 2 * w + j;
                    const bf16x4 k4 = cvt4(kt[j]), v4 = cvt4(v[j]);
                    *reinterpret_cast<bf16x4 *>(qs[q] + c16 * kQLd + r0) = cvt4(qt[j]);
                    *reinterpret_cast<bf16x4 *>(ks_[q] + c16 * kQLd + r0) = k4;
                    *reinterpret_cast<bf16x4 *>(vt[q] + c16 * kVLd + r0) = v4;
                    if (A.kv_out && sc[j] < cpt && tb + sc[j] < cnt) {  // sample mode: keep them for list mode
                        __bf16 *kc = A.kv_out + (tb + sc[j]) * kv_cfg + ((int64_t)layer * kH + hh) * kKvPerHead;
                        *reinterpret_cast<bf16x4 *>(kc + (srb[j] * 16 + c16) * kDh + r0) = k4;
                        *reinterpret_cast<bf16x4 *>(kc + 64 * kDh + c16 * 64 + srb[j] * 16 + r0) = v4;
                    }
                }
                __syncthreads();  // K and V of every slot written
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    KvSrc S;
                    const __bf16 *kc = A.kv_in ? A.kv_in + ssmp[j] * kv_cfg + ((int64_t)layer * kH + hh) * kKvPerHead : nullptr;
                    S.kc = kc;
                    S.vc = kc + 64 * kDh;
                    S.ks = &ks_[0][0];
                    S.vt = &vt[0][0];
                    S.cls = cls;
                    S.c = sc[j];
                    S.sb = kList ? cls : 0;
                    attend<kF8>(srb[j], qs[2 * w + j], S, Pb, j ? O1 : O0, hh);
                }
                __syncthreads();  // every slot done with this head's K and V (and the QKV weights)
            }
            stage_rows_t(wbuf, kLdA, lw + 192 * 64, 64, 64, 64);
            __syncthreads();
#pragma unroll
            for (int db = 0; db < 4; db++) {
                const f32x4 bo = ld4(lv + kV_bo + db * 16 + r0);
#pragma unroll
                for (int j = 0; j < 2; j++) h.t[j * 4 + db] += bo;
            }
            // FP8: the products come out scaled by the matrix's power of two s;
            // the residual is scaled by s around them (exact)
            if constexpr (kF8) {
#pragma unroll
                for (int q = 0; q < 8; q++) h.t[q] *= f8[6];
            }
            gemm_slots_t<kF8>(h, O0, O1, wbuf, 64);
            if constexpr (kF8) {
#pragma unroll
                for (int q = 0; q < 8; q++) h.t[q] *= f8[7];
            }
            normalize_rows_t<kF8>(h, X0, X1);
            if constexpr (kF8) {
#pragma unroll
                for (int q = 0; q < 8; q++) h.t[q] *= f8[10];
            }
            // FFN in four hidden chunks of 64
            for (int chunk = 0; chunk < 4; chunk++) {
                __syncthreads();
                stage_rows_t(wbuf, kLdA, lw + 192 * 64 + 64 * 64 + chunk * 64 * 64, 64, 64, 64);  // w1T rows
                stage_rows_t(wbuf + 64 * kLdA, kLdA, lw + 192 * 64 + 64 * 64 + 256 * 64 + chunk * 64, 256, 64, 64);
                __syncthreads();
                // f^T: lane (row c16, hidden units 16 hb + r0 + i) of the chunk
                Tile32 f;
#pragma unroll
                for (int hb = 0; hb < 4; hb++) {
                    f32x4 b1 = ld4(lv + kV_b1 + chunk * 64 + hb * 16 + r0);
                    if constexpr (kF8) b1 *= f8[8];
#pragma unroll
                    for (int j = 0; j < 2; j++) f.t[j * 4 + hb] = b1;
                }
                gemm_slots_t<kF8>(f, X0, X1, wbuf, 64);
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    AT *O = (j ? O1 : O0) + c16 * kLdA + r0;
#pragma unroll
                    for (int hb = 0; hb < 4; hb++) {
                        f32x4 g;
#pragma unroll
                        for (int i = 0; i < 4; i++) g[i] = gelu_tab(gtab, kF8 ? f.t[j * 4 + hb][i] * f8[9] : f.t[j * 4 + hb][i]);
                        store4<kF8>(O + hb * 16, g);
                    }
                }
                wave_lds_sync();
                gemm_slots_t<kF8>(h, O0, O1, wbuf + 64 * kLdA, 64);
            }
            if constexpr (kF8) {
#pragma unroll
                for (int q = 0; q < 8; q++) h.t[q] *= f8[11];
            }
#pragma unroll
            for (int db = 0; db < 4; db++) {
                const f32x4 b2 = ld4(lv + kV_b2 + db * 16 + r0);
#pragma unroll
                for (int j = 0; j < 2; j++) h.t[j * 4 + db] += b2;
            }
        }
        // final LayerNorm (scale folded into the head), head, mask and the
        // log-probability of the actual token, per own slot: lane l's group of
        // four lanes holds row c16; lanes 0..15 finish it
#pragma unroll
        for (int j = 0; j < 2; j++) {
            float rstd, sh;
            row_stats_t(h, j, rstd, sh);
            float z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int db = 0; db < 4; db++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const float y = fmaf(h.t[j * 4 + db][i], rstd, sh);
                    const f32x4 hw4 = ld4(wf + M.fl.head_w + (db * 16 + r0 + i) * 4);
#pragma unroll
                    for (int t = 0; t < 4; t++) z[t] = fmaf(y, hw4[t], z[t]);
                }
#pragma unroll
            for (int t = 0; t < 4; t++) {
                z[t] += __shfl_xor(z[t], 16, 64);
                z[t] += __shfl_xor(z[t], 32, 64);
            }
            float lsum = 0.f;
            const int s = srb[j] * 16 + c16;
            if (l < 16 && s < K) {
                const uint64_t below = (1ull << s) - 1ull;  // s < K <= 64
                const int up = __popcll(upm[j] & below), dn = __popcll(dnm[j] & below);
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
                const int ts = token(j, s);
                const float lden = __logf(den);
                lsum = ok[ts] ? (z[ts] - mx) - lden : -INFINITY;
                if (!kList && A.cond_out && s == A.cond_pos && sc[j] < cpt && tb + sc[j] < cnt)
#pragma unroll
                    for (int t = 0; t < 4; t++)
                        A.cond_out[(tb + sc[j]) * 4 + t] = ok[t] ? (double)((z[t] - mx) - lden) : -INFINITY;
            }
            // the slot's rows live in lanes 0..15
            lsum = dpp_row_sum(lsum);
            if (l == 0) slot_lp[2 * w + j] = (double)lsum;
        }
        __syncthreads();
        // per configuration: sum of its row blocks in block order
        if ((int)threadIdx.x < cpt && tb + (int)threadIdx.x < cnt) {
            const int c = threadIdx.x;
            if (kList) {
                const int64_t e = A.list[lbase + tb + c];
                double acc = A.pre_in[(e / A.C) * 4 + cls];
                for (int kb = cls; kb < 4; kb++) acc += slot_lp[slot_of(cls, c, kb)];
                A.xla[e] = 0.5 * acc;
            } else {
                double acc = 0.0;
                for (int kb = 0; kb < 4; kb++) {
                    if (A.pre_out) A.pre_out[(tb + c) * 4 + kb] = acc;
                    acc += slot_lp[slot_of(0, c, kb)];
                }
                A.logabs[tb + c] = 0.5 * acc;
            }
        }
        __syncthreads();  // slot_lp and the slots are reused by the next tile
    }
}

__global__ void __launch_bounds__(512) k_transformer_bf16(Bf16View M, TfArgs A) {
    transformer_bf16<false, false, false>(M, A, nullptr, 0);
}

__global__ void __launch_bounds__(512) k_transformer_bf16_list(Bf16View M, TfArgs A) {
    transformer_bf16<true, false, false>(M, A, nullptr, 0);
}

__global__ void __launch_bounds__(512) k_transformer_fp8(Bf16View M, TfArgs A) {
    transformer_bf16<false, true, false>(M, A, nullptr, 0);
}

__global__ void __launch_bounds__(512) k_transformer_fp8_list(Bf16View M, TfArgs A) {
    transformer_bf16<true, true, false>(M, A, nullptr, 0);
}

// Many systems in one persistent launch: the list-mode work of every item
// (its four class lists, hdr on the device) as one tile space; each block
// takes tiles in turn and runs them with that item's model.
__global__ void __launch_bounds__(512) k_transformer_bf16_batch(Bf16View M0, const TfItem *items, int n_items) {
    transformer_bf16<true, false, true>(M0, items[0].A, items, n_items);
}

// Phase MLP (Section 4.1): phi = b3 + w3 . GELU(GELU(bits W1 + b1) W2 + b2)
// on BF16 MFMA with FP32 accumulation.  A block of kPhWaves waves takes 128
// configurations per pass; wave w owns output columns 64 w .. 64 w + 63 of
// both layers, so each weight fragment is read once per 128 configurations
// (held in registers across the eight groups of 16), the hidden layer z1
// stays in LDS, and the four per-wave partial dot products of each
// configuration are added in wave order at the end.
// In list mode (see TfArgs) the configurations are xkeys[list[k]] for k
// below the total of the four class counts, and phase[list[k]] receives them.
constexpr int kPhWaves = 8, kPhRows = 16 * kPhWaves, kZld = kP + 8;
__global__ void __launch_bounds__(64 * kPhWaves) k_phase_bf16(Bf16View M, TfArgs A, double *__restrict__ phase) {
    __shared__ __align__(16) __bf16 zs[kPhRows * kZld];
    __shared__ float parts[kPhWaves][kPhRows];
    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c16 = l & 15, r0 = 4 * (l >> 4), kq = 8 * (l >> 4);
    const int col0 = 64 * w;  // this wave's output columns
    const __bf16 *w1T = M.wb + M.bl.ph_w1T, *w2T = M.wb + M.bl.ph_w2T;
    const float *b1 = M.wf + M.fl.ph_b1, *b2 = M.wf + M.fl.ph_b2, *w3 = M.wf + M.fl.ph_w3;
    const int nbits = 2 * M.K;
    const int64_t n = A.list_mode ? A.hdr[0] + A.hdr[1] + A.hdr[2] + A.hdr[3] : A.n;
    for (int64_t base = (int64_t)blockIdx.x * kPhRows; base < n; base += (int64_t)gridDim.x * kPhRows) {
        // z1 = GELU(bits @ W1 + b1) for the block's 128 configurations, this wave's 64 columns;
        // the layer-1 B fragments (W1^T rows col0 + 16 cb + c16) serve all eight groups
        bf16x8 bw1[kPhaseBits / 32][4];
#pragma unroll
        for (int ks = 0; ks < kPhaseBits / 32; ks++)
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
                bw1[ks][cb] =
                    *reinterpret_cast<const bf16x8 *>(w1T + (int64_t)(col0 + cb * 16 + c16) * kPhaseBits + ks * 32 + kq);
        for (int rg = 0; rg < kPhWaves; rg++) {
            const int64_t cr = base + 16 * rg + c16;
            Key x{0ull, 0ull};
            if (cr < n) {
                const uint64_t *kp = A.list_mode ? A.xkeys + 2 * (int64_t)A.list[cr] : A.keys + 2 * cr;
                x.lo = kp[0];
                x.hi = kp[1];
            }
            f32x4 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; cb++) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kPhaseBits / 32; ks++) {
                bf16x8 ab;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int p = ks * 32 + kq + e;
                    ab[e] = (__bf16)((p < nbits && key_bit(x, p)) ? 1.0f : 0.0f);
                }
#pragma unroll
                for (int cb = 0; cb < 4; cb++) acc[cb] = mfma16(ab, bw1[ks][cb], acc[cb]);
            }
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                const float bb = b1[col0 + cb * 16 + c16];
#pragma unroll
                for (int i = 0; i < 4; i++)
                    zs[(16 * rg + r0 + i) * kZld + col0 + cb * 16 + c16] = (__bf16)gelu32(acc[cb][i] + bb);
            }
        }
        __syncthreads();  // z1 of every column written
        // phi partials: w3 . GELU(z1 @ W2 + b2) over this wave's columns, in two
        // halves of 32 columns (every W2 fragment is still read once per pass)
        float part[kPhWaves][4];
#pragma unroll
        for (int rg = 0; rg < kPhWaves; rg++)
#pragma unroll
            for (int i = 0; i < 4; i++) part[rg][i] = 0.f;
#pragma unroll 1
        for (int half = 0; half < 2; half++) {
            f32x4 acc2[kPhWaves][2];
#pragma unroll
            for (int rg = 0; rg < kPhWaves; rg++)
#pragma unroll
                for (int cb = 0; cb < 2; cb++) acc2[rg][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
            for (int ks = 0; ks < kP; ks += 32) {
                bf16x8 bw[2];
#pragma unroll
                for (int cb = 0; cb < 2; cb++)
                    bw[cb] = *reinterpret_cast<const bf16x8 *>(w2T + (int64_t)(col0 + (2 * half + cb) * 16 + c16) * kP +
                                                               ks + kq);
#pragma unroll
                for (int rg = 0; rg < kPhWaves; rg++) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(zs + (16 * rg + c16) * kZld + ks + kq);
#pragma unroll
                    for (int cb = 0; cb < 2; cb++) acc2[rg][cb] = mfma16(a, bw[cb], acc2[rg][cb]);
                }
            }
#pragma unroll
            for (int cb = 0; cb < 2; cb++) {
                const int col = col0 + (2 * half + cb) * 16 + c16;
                const float bb = b2[col], ww = w3[col];
#pragma unroll
                for (int rg = 0; rg < kPhWaves; rg++)
#pragma unroll
                    for (int i = 0; i < 4; i++) part[rg][i] += gelu32(acc2[rg][cb][i] + bb) * ww;
            }
        }
#pragma unroll
        for (int rg = 0; rg < kPhWaves; rg++) {
#pragma unroll
            for (int i = 0; i < 4; i++) part[rg][i] = dpp_row_sum(part[rg][i]);
            if (c16 == 0)
#pragma unroll
                for (int i = 0; i < 4; i++) parts[w][16 * rg + r0 + i] = part[rg][i];
        }
        __syncthreads();  // every wave's partials written, z1 consumed
        if ((int)threadIdx.x < kPhRows) {
            const int64_t cfg = base + threadIdx.x;
            if (cfg < n) {
                float s = 0.f;
                for (int q = 0; q < kPhWaves; q++) s += parts[q][threadIdx.x];
                phase[A.list_mode ? (int64_t)A.list[cfg] : cfg] = (double)(s + M.wf[M.fl.ph_b3]);
            }
        }
        __syncthreads();  // parts read before the next pass rewrites them
    }
}

static Bf16View bf16_view(const nnqs_model *m) {
    Bf16View v{};
    v.K = m->desc.n_orb;
    v.L = m->desc.n_layers;
    v.n_up = m->desc.n_up;
    v.n_dn = m->desc.n_dn;
    v.wb = reinterpret_cast<const __bf16 *>(m->d_bf16);
    v.w8 = reinterpret_cast<const uint8_t *>(m->d_fp8);
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

// OCP FP8 E4M3 (bias 7, 3 mantissa bits, largest finite 448), round to
// nearest even, saturated at +-448.
static uint8_t to_e4m3(float f) {
    const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
    double a = std::fabs((double)f);
    if (!(a == a)) return 0x7F;
    if (a >= 448.0) return sign | 0x7E;
    auto rne = [](double v) {  // round half to even
        const double fl = std::floor(v), d = v - fl;
        if (d > 0.5) return fl + 1.0;
        if (d < 0.5) return fl;
        return std::fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
    };
    if (a < std::ldexp(1.0, -6)) {  // subnormal: m * 2^-9 (m = 8 carries into the smallest normal)
        return sign | (uint8_t)rne(a * 512.0);
    }
    int e = 0;
    const double fr = std::frexp(a, &e);  // a = fr * 2^e, fr in [0.5, 1)
    e -= 1;                               // a = (2 fr) * 2^e, 2 fr in [1, 2)
    double q = rne((2.0 * fr - 1.0) * 8.0);
    if (q >= 8.0) {
        q = 0.0;
        e += 1;
    }
    const int code = ((e + 7) << 3) | (int)q;
    return sign | (uint8_t)(code > 0x7E ? 0x7E : code);
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
    std::vector<uint8_t> w8((size_t)bl.total, 0);
    std::vector<float> wf((size_t)fl.total, 0.f);
    auto W = [&](int64_t off) { return weights + off; };
    // transposed copy: dst[n][k] = src[k][n] for a [kdim][ndim] source matrix
    auto put_t = [&](int64_t dst, int dst_ld, const float *src, int kdim, int ndim, int row0) {
        for (int k = 0; k < kdim; k++)
            for (int nn = 0; nn < ndim; nn++) wb[dst + (int64_t)(row0 + nn) * dst_ld + k] = to_bf16_bits(src[k * ndim + nn]);
    };
    // FP8 copy of a [kdim][ndim] matrix, transposed like put_t, with the power
    // of two s that brings its largest magnitude to at most 448; stores s, 1/s
    auto put_t8 = [&](int64_t dst, int dst_ld, const float *src, int kdim, int ndim, int row0, float *sc) {
        double mx = 0.0;
        for (int64_t e = 0; e < (int64_t)kdim * ndim; e++) mx = std::max(mx, std::fabs((double)src[e]));
        int k2 = mx > 0.0 ? (int)std::floor(std::log2(448.0 / mx)) : 0;
        k2 = std::min(60, std::max(-60, k2));
        const double s = std::ldexp(1.0, k2);
        for (int k = 0; k < kdim; k++)
            for (int nn = 0; nn < ndim; nn++)
                w8[dst + (int64_t)(row0 + nn) * dst_ld + k] = to_e4m3((float)(s * src[k * ndim + nn]));
        sc[0] = (float)s;
        sc[1] = (float)(1.0 / s);
    };
    // A LayerNorm's scale g and shift b fold into the product y W + c that
    // reads it: (n * g + b) W + c = n (diag(g) W) + (b W + c), n = the
    // normalised row; the attention scale 1/sqrt(16) and log2(e) (the softmax
    // runs in base 2) fold into W_q and b_q.  Folded in FP64, then rounded.
    auto fold = [&](const float *Wm, const float *bm, const float *g, const float *beta, int kdim, int ndim,
                    double scale, std::vector<float> &Wf, std::vector<float> &bf) {
        Wf.assign((size_t)kdim * ndim, 0.f);
        bf.assign((size_t)ndim, 0.f);
        for (int nn = 0; nn < ndim; nn++) {
            double acc = bm[nn];
            for (int k = 0; k < kdim; k++) {
                Wf[(size_t)k * ndim + nn] = (float)(scale * (double)g[k] * (double)Wm[(size_t)k * ndim + nn]);
                acc += (double)beta[k] * (double)Wm[(size_t)k * ndim + nn];
            }
            bf[nn] = (float)(scale * acc);
        }
    };
    const double qscale = 0.25 * 1.4426950408889634;
    std::vector<float> fw, fb;
    for (int l = 0; l < L; l++) {
        const int64_t lo = o.layer0 + l * o.layer_stride;
        const int64_t base = bl.layer0 + l * bl.layer_stride;
        const int64_t dd = kD * kD;
        // layer block layout of the FP32 weights: ln1_g ln1_b wq bq wk bk wv bv wo bo ln2_g ln2_b w1 b1 w2 b2
        const float *ln1g = W(lo), *ln1b = W(lo + kD);
        const float *wq = W(lo + 2 * kD), *bq = wq + dd, *wk = bq + kD, *bk = wk + dd, *wv = bk + kD, *bv = wv + dd,
                    *wo = bv + kD, *bo = wo + dd, *ln2g = bo + kD, *ln2b = ln2g + kD, *w1 = ln2b + kD,
                    *b1 = w1 + kD * kF, *w2 = b1 + kF, *b2 = w2 + kF * kD;
        float *lv = wf.data() + fl.layer0 + l * fl.layer_stride;
        fold(wq, bq, ln1g, ln1b, kD, kD, qscale, fw, fb);
        put_t(base, 64, fw.data(), kD, kD, 0);
        put_t8(base, 64, fw.data(), kD, kD, 0, lv + kV_f8 + 0);
        std::memcpy(lv + kV_bqkv, fb.data(), kD * 4);
        fold(wk, bk, ln1g, ln1b, kD, kD, 1.0, fw, fb);
        put_t(base, 64, fw.data(), kD, kD, 64);
        put_t8(base, 64, fw.data(), kD, kD, 64, lv + kV_f8 + 2);
        std::memcpy(lv + kV_bqkv + 64, fb.data(), kD * 4);
        fold(wv, bv, ln1g, ln1b, kD, kD, 1.0, fw, fb);
        put_t(base, 64, fw.data(), kD, kD, 128);
        put_t8(base, 64, fw.data(), kD, kD, 128, lv + kV_f8 + 4);
        std::memcpy(lv + kV_bqkv + 128, fb.data(), kD * 4);
        put_t(base + 192 * 64, 64, wo, kD, kD, 0);
        put_t8(base + 192 * 64, 64, wo, kD, kD, 0, lv + kV_f8 + 6);
        fold(w1, b1, ln2g, ln2b, kD, kF, 1.0, fw, fb);
        put_t(base + 192 * 64 + 64 * 64, 64, fw.data(), kD, kF, 0);
        put_t8(base + 192 * 64 + 64 * 64, 64, fw.data(), kD, kF, 0, lv + kV_f8 + 8);
        std::memcpy(lv + kV_b1, fb.data(), kF * 4);
        put_t(base + 192 * 64 + 64 * 64 + 256 * 64, 256, w2, kF, kD, 0);
        put_t8(base + 192 * 64 + 64 * 64 + 256 * 64, 256, w2, kF, kD, 0, lv + kV_f8 + 10);
        std::memcpy(lv + kV_ln1_g, ln1g, kD * 4);
        std::memcpy(lv + kV_ln1_b, ln1b, kD * 4);
        std::memcpy(lv + kV_bo, bo, kD * 4);
        std::memcpy(lv + kV_ln2_g, ln2g, kD * 4);
        std::memcpy(lv + kV_ln2_b, ln2b, kD * 4);
        std::memcpy(lv + kV_b2, b2, kD * 4);
    }
    std::memcpy(wf.data() + fl.tok_emb, W(o.tok_emb), 5 * kD * 4);
    std::memcpy(wf.data() + fl.pos_emb, W(o.pos_emb), (size_t)K * kD * 4);
    std::memcpy(wf.data() + fl.lnf_g, W(o.lnf_g), kD * 4);
    std::memcpy(wf.data() + fl.lnf_b, W(o.lnf_b), kD * 4);
    fold(W(o.head_w), W(o.head_b), W(o.lnf_g), W(o.lnf_b), kD, 4, 1.0, fw, fb);
    std::memcpy(wf.data() + fl.head_w, fw.data(), 4 * kD * 4);
    std::memcpy(wf.data() + fl.head_b, fb.data(), 4 * 4);
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
    if (hipMalloc(&m->d_bf16, wb.size() * 2) != hipSuccess || hipMalloc(&m->d_f32, wf.size() * 4) != hipSuccess ||
        hipMalloc(&m->d_fp8, w8.size()) != hipSuccess)
        return fail(NNQS_ENOMEM, "device allocation of the BF16 model failed");
    if (hipMemcpy(m->d_fp8, w8.data(), w8.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_bf16, wb.data(), wb.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_f32, wf.data(), wf.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(NNQS_EHIP, "copy of the BF16 model failed");
    return NNQS_OK;
}

void bf16_model_free(nnqs_model *m) {
    hipFree(m->d_bf16);
    hipFree(m->d_f32);
    hipFree(m->d_fp8);
    m->d_fp8 = nullptr;
    m->d_bf16 = nullptr;
    m->d_f32 = nullptr;
}

static int cu_count() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return cus;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus;
}

// One block per CU is resident (the slots take 157 KB of LDS); blocks loop
// over tiles.
static unsigned tf_grid(int64_t tiles) {
    const int64_t cap = cu_count();
    return (unsigned)(tiles < 1 ? 1 : tiles < cap ? tiles : cap);
}

static unsigned phase_grid(int64_t n) {
    const int64_t cap = (int64_t)cu_count();  // one block per CU (z1 fills most of its LDS)
    const int64_t b = (n + kPhRows - 1) / kPhRows;
    return (unsigned)(b < 1 ? 1 : b < cap ? b : cap);
}

nnqs_status enqueue_logpsi_bf16(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, double *phase,
                                hipStream_t st, bool fp8) {
    if (!m->bf16_ok) return fail(NNQS_EUNSUPPORTED, "BF16 forward needs d_model 64, 4 heads, FFN 256, P 512, K <= 64");
    const Bf16View v = bf16_view(m);
    TfArgs A{};
    A.keys = keys;
    A.n = n;
    A.logabs = logabs;
    if (fp8) {
        TimedRegion tr("k_transformer_fp8", st);
        hipLaunchKernelGGL(k_transformer_fp8, dim3(tf_grid((n + 3) / 4)), dim3(512), 0, st, v, A);
    } else {
        TimedRegion tr("k_transformer_bf16", st);
        hipLaunchKernelGGL(k_transformer_bf16, dim3(tf_grid((n + 3) / 4)), dim3(512), 0, st, v, A);
    }
    {
        TimedRegion tr("k_phase_bf16", st);
        hipLaunchKernelGGL(k_phase_bf16, dim3(phase_grid(n)), dim3(kPhWaves * 64), 0, st, v, A, phase);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

nnqs_status enqueue_bf16_cond(const nnqs_model *m, const uint64_t *keys, int64_t n, int cpos, double *cond,
                              double *logabs, hipStream_t st) {
    if (!m->bf16_ok) return fail(NNQS_EUNSUPPORTED, "BF16 forward needs d_model 64, 4 heads, FFN 256, P 512, K <= 64");
    TfArgs A{};
    A.keys = keys;
    A.n = n;
    A.logabs = logabs;
    A.cond_pos = cpos;
    A.cond_out = cond;
    TimedRegion tr("k_transformer_bf16", st);
    hipLaunchKernelGGL(k_transformer_bf16, dim3(tf_grid((n + 3) / 4)), dim3(512), 0, st, bf16_view(m), A);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

int64_t bf16_cache_elems(const nnqs_model *m) { return (int64_t)m->desc.n_layers * kH * kKvPerHead; }

nnqs_status enqueue_bf16_cached(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, __bf16 *kv,
                                double *pre, hipStream_t st, bool fp8) {
    if (!m->bf16_ok) return fail(NNQS_EUNSUPPORTED, "BF16 forward needs d_model 64, 4 heads, FFN 256, P 512, K <= 64");
    TfArgs A{};
    A.keys = keys;
    A.n = n;
    A.logabs = logabs;
    A.kv_out = kv;
    A.pre_out = pre;
    if (fp8) {
        TimedRegion tr("k_transformer_fp8", st);
        hipLaunchKernelGGL(k_transformer_fp8, dim3(tf_grid((n + 3) / 4)), dim3(512), 0, st, bf16_view(m), A);
    } else {
        TimedRegion tr("k_transformer_bf16", st);
        hipLaunchKernelGGL(k_transformer_bf16, dim3(tf_grid((n + 3) / 4)), dim3(512), 0, st, bf16_view(m), A);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

nnqs_status enqueue_bf16_list(const nnqs_model *m, const uint64_t *xkeys, int64_t C, const int32_t *list,
                              const int64_t *hdr, int64_t max_entries, const __bf16 *kv, const double *pre,
                              double *xla, double *xph, hipStream_t st, bool fp8) {
    if (!m->bf16_ok) return fail(NNQS_EUNSUPPORTED, "BF16 forward needs d_model 64, 4 heads, FFN 256, P 512, K <= 64");
    const Bf16View v = bf16_view(m);
    TfArgs A{};
    A.kv_in = kv;
    A.pre_in = pre;
    A.list = list;
    A.hdr = hdr;
    A.xkeys = xkeys;
    A.C = C;
    A.xla = xla;
    A.list_mode = 1;  // kv_out / pre_out stay null: list mode only reads the cache
    if (fp8) {
        TimedRegion tr("k_transformer_fp8_list", st);
        hipLaunchKernelGGL(k_transformer_fp8_list, dim3(tf_grid((max_entries + 3) / 4)), dim3(512), 0, st, v, A);
    } else {
        TimedRegion tr("k_transformer_bf16_list", st);
        hipLaunchKernelGGL(k_transformer_bf16_list, dim3(tf_grid((max_entries + 3) / 4)), dim3(512), 0, st, v, A);
    }
    {
        TimedRegion tr("k_phase_bf16", st);
        hipLaunchKernelGGL(k_phase_bf16, dim3(phase_grid(max_entries)), dim3(kPhWaves * 64), 0, st, v, A, xph);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

size_t bf16_item_bytes() { return sizeof(TfItem); }

int bf16_batch_max_items() { return kMaxTfItems; }

void bf16_list_item(const nnqs_model *m, const uint64_t *xkeys, int64_t C, const int32_t *list, const int64_t *hdr,
                    const __bf16 *kv, const double *pre, double *xla, void *dst) {
    TfItem it{};
    it.M = bf16_view(m);
    it.A.kv_in = kv;
    it.A.pre_in = pre;
    it.A.list = list;
    it.A.hdr = hdr;
    it.A.xkeys = xkeys;
    it.A.C = C;
    it.A.xla = xla;
    it.A.list_mode = 1;
    std::memcpy(dst, &it, sizeof(it));
}

nnqs_status enqueue_bf16_phase_list(const nnqs_model *m, const uint64_t *xkeys, const int32_t *list, const int64_t *hdr,
                                    int64_t max_entries, double *xph, hipStream_t st) {
    TfArgs A{};
    A.list = list;
    A.hdr = hdr;
    A.xkeys = xkeys;
    A.list_mode = 1;
    TimedRegion tr("k_phase_bf16", st);
    hipLaunchKernelGGL(k_phase_bf16, dim3(phase_grid(max_entries)), dim3(kPhWaves * 64), 0, st, bf16_view(m), A, xph);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

nnqs_status enqueue_bf16_batch(const nnqs_model *m0, const void *d_items, int n_items, hipStream_t st) {
    TimedRegion tr("k_transformer_bf16_batch", st);
    hipLaunchKernelGGL(k_transformer_bf16_batch, dim3((unsigned)cu_count()), dim3(512), 0, st, bf16_view(m0),
                       static_cast<const TfItem *>(d_items), n_items);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

}  // namespace nnqs

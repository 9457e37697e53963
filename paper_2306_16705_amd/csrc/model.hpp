// Internal definitions of the wave-function model (see model.hip).
#pragma once

#include "internal.hpp"

namespace nnqs {

struct ModelOffsets {  // element offsets into the flat weight array
    int64_t tok_emb, pos_emb, layer0, layer_stride, lnf_g, lnf_b, head_w, head_b, bias;
    int64_t ph_w1, ph_b1, ph_w2, ph_b2, ph_w3, ph_b3, total;
};

struct LayerOffsets {  // element offsets inside one layer block
    int64_t ln1_g, ln1_b, wq, bq, wk, bk, wv, bv, wo, bo, ln2_g, ln2_b, w1, b1, w2, b2;
};

struct ModelView {
    int K, d, L, H, F, P, n_up, n_dn;
    const double *w64;
    ModelOffsets off;
};

ModelOffsets model_offsets(const nnqs_model_desc &m);

// Offsets inside one layer block.
__host__ __device__ inline LayerOffsets layer_offsets(int d, int F) {
    LayerOffsets L{};
    int64_t at = 0;
    L.ln1_g = at; at += d;
    L.ln1_b = at; at += d;
    L.wq = at; at += (int64_t)d * d;
    L.bq = at; at += d;
    L.wk = at; at += (int64_t)d * d;
    L.bk = at; at += d;
    L.wv = at; at += (int64_t)d * d;
    L.bv = at; at += d;
    L.wo = at; at += (int64_t)d * d;
    L.bo = at; at += d;
    L.ln2_g = at; at += d;
    L.ln2_b = at; at += d;
    L.w1 = at; at += (int64_t)d * F;
    L.b1 = at; at += F;
    L.w2 = at; at += (int64_t)F * d;
    L.b2 = at; at += d;
    return L;
}


}  // namespace nnqs

struct nnqs_model {
    nnqs_model_desc desc{};
    nnqs::ModelOffsets off{};
    double *d_w64 = nullptr;
    int max_lds = 0;
    // scratch of the layer-batched FP64 forward (model_f64.hip), grown on demand
    void *d_f64s = nullptr;
    size_t f64cap = 0;
    // scratch of the FP64 backward (grad_f64.hip): saved activations of one
    // pass, their gradients and the weight-gradient partials
    void *d_grads = nullptr;
    size_t gradcap = 0;
    // BF16 path: transposed BF16 matrices and FP32 vectors (model_bf16.hip)
    void *d_bf16 = nullptr;
    float *d_f32 = nullptr;
    void *d_fp8 = nullptr;  // FP8 E4M3 transformer matrices (same layout as d_bf16)
    bool bf16_ok = false;
    // full-E_loc scratch (eloc_model.hip), grown on demand
    uint64_t *d_xkeys = nullptr;
    double *d_xla = nullptr, *d_xph = nullptr, *d_sla = nullptr, *d_sph = nullptr;
    int64_t xcap = 0, scap = 0;
    double *d_partials = nullptr;
    // screen scratch (eloc_model.hip)
    uint8_t *d_xexc = nullptr;
    float *d_pred = nullptr;
    float *d_loghx = nullptr;       // log|H_xx'| per connection (selection rules)
    int32_t *d_sel = nullptr;       // survivor indices (chunk-local)
    int32_t *d_blockcnt = nullptr;  // per-block survivor counts / offsets
    uint64_t *d_ckeys = nullptr;    // compacted survivor keys
    double *d_cla = nullptr, *d_cph = nullptr;
    int64_t *d_nsel = nullptr;
    // prefix-reusing BF16 path (eloc_model.hip): the chunk samples' key /
    // value cache and prefix sums, their BF16 log|psi|, the class header
    // {count[4], offset[4]} and the evaluated-connection counter
    __bf16 *d_kv = nullptr;
    double *d_pre = nullptr, *d_csla = nullptr;
    int64_t *d_hdr = nullptr;
    int64_t kvcap = 0;
    // FP64 refinement with prefix reuse: the chunk samples' FP64 keys and
    // values of every layer and their prefix log-probability sums
    double *d_kv64 = nullptr, *d_pre64 = nullptr;
    int64_t kv64cap = 0;
    void *d_rag = nullptr;  // starts, row counts and row offsets of the refined connections
    size_t ragcap = 0;
    // evaluation of distinct x' (dedup): sort keys / payloads, run heads,
    // best representative per run, representative of every kept connection,
    // the second list, and per-connection masks (representatives, refined runs)
    uint64_t *d_ddk = nullptr;
    uint32_t *d_ddi = nullptr;
    int32_t *d_ddhead = nullptr, *d_ddrep = nullptr, *d_sel2 = nullptr;
    unsigned long long *d_ddbest = nullptr;
    uint8_t *d_repmask = nullptr, *d_refmask = nullptr;
    int64_t ddcap = 0, maskcap = 0;
};

namespace nnqs {
ModelView model_view(const nnqs_model *m);
nnqs_status enqueue_logpsi(const nnqs_model *m, const uint64_t *keys, int64_t n, int32_t precision, double *logabs,
                           double *phase, hipStream_t st);
nnqs_status bf16_model_init(nnqs_model *m, const float *weights);
void bf16_model_free(nnqs_model *m);
nnqs_status enqueue_logpsi_bf16(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs,
                                double *phase, hipStream_t st, bool fp8 = false);
// BF16 cache of sample-mode forwards for the prefix-reusing list mode: per
// configuration bf16_cache_elems(m) BF16 values (keys and values of every
// layer and head) and 4 doubles of prefix log-probability sums.
int64_t bf16_cache_elems(const nnqs_model *m);
nnqs_status enqueue_bf16_cached(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, __bf16 *kv,
                                double *pre, hipStream_t st, bool fp8);
// BF16 forward of n configurations writing only the masked conditionals of
// position cpos into cond[n][4] (batch sampling; logabs is scratch).
nnqs_status enqueue_bf16_cond(const nnqs_model *m, const uint64_t *keys, int64_t n, int cpos, double *cond,
                              double *logabs, hipStream_t st);
// Batched list mode (one persistent launch over many systems): bytes of one
// device launch descriptor, the largest item count, the descriptor of one
// item written to host memory `dst`, the phase MLP of one item's lists, and
// the launch over a device array of descriptors (models must all be BF16-capable).
size_t bf16_item_bytes();
int bf16_batch_max_items();
void bf16_list_item(const nnqs_model *m, const uint64_t *xkeys, int64_t C, const int32_t *list, const int64_t *hdr,
                    const __bf16 *kv, const double *pre, double *xla, void *dst);
nnqs_status enqueue_bf16_phase_list(const nnqs_model *m, const uint64_t *xkeys, const int32_t *list, const int64_t *hdr,
                                    int64_t max_entries, double *xph, hipStream_t st);
nnqs_status enqueue_bf16_batch(const nnqs_model *m0, const void *d_items, int n_items, hipStream_t st);
// log|psi| and phase of the connections listed by class (hdr on the device:
// count[4], offset[4]; at most max_entries in total) into xla / xph.
nnqs_status enqueue_bf16_list(const nnqs_model *m, const uint64_t *xkeys, int64_t C, const int32_t *list,
                              const int64_t *hdr, int64_t max_entries, const __bf16 *kv, const double *pre,
                              double *xla, double *xph, hipStream_t st, bool fp8);
void eloc_model_free(nnqs_model *m);
bool f64_shape_ok(const nnqs_model_desc &m);
// FP64 forward; with cond, also the masked conditionals of position cpos
// into cond[n][4] (batch sampling).
nnqs_status enqueue_logpsi_f64(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, double *phase,
                               hipStream_t st, int cpos = -1, double *cond = nullptr, double *kvc = nullptr,
                               double *pre = nullptr);
// FP64 prefix-reusing forward of n listed connections from a sample cache
// written by enqueue_logpsi_f64's kvc / pre outputs (per sample
// [L][2][K][64] + [K + 1] doubles); each x' from its first changed position
// on; see model_f64.hip.
int64_t f64_cache_doubles(const nnqs_model *m);

// Ascending bitonic sort of P (a power of two >= 2) 128-bit keys sk[2 i],
// sk[2 i + 1] (word 1 major) with 32-bit payloads si[i] as the final
// tie-break, in place (nnqs_core.hip).
void bitonic_sort128(uint64_t *sk, uint32_t *si, int64_t P, hipStream_t st);
nnqs_status enqueue_f64_list(const nnqs_model *m, const uint64_t *xkeys, int64_t C, const int32_t *list, int64_t n,
                             const uint64_t *keys, const double *kvc, const double *pre, double *xla, double *xph,
                             hipStream_t st);
nnqs_status screen_infer(nnqs_screen *s, const uint64_t *keys, const uint8_t *exc, int64_t n, float *pred,
                         hipStream_t st, bool fp8);
}  // namespace nnqs

// Wave-function ansatz on the device (paper: Section 3.1, Eq. 11 and Fig. 2;
// Section 3.3, Eq. 12 mask; Section 4.1 phase MLP sizes): model object,
// FP64 forward kernel (parity path) and the entry point that dispatches the
// FP64 or BF16 forward.
#include <cmath>
#include <cstring>
#include <vector>

#include "model.hpp"

namespace nnqs {

// Offsets of every tensor in the flat weight layout of the header.
ModelOffsets model_offsets(const nnqs_model_desc &m) {
    ModelOffsets o{};
    const int64_t K = m.n_orb, d = m.d_model, F = m.d_ff, P = m.phase_hidden;
    int64_t at = 0;
    o.tok_emb = at;
    at += 5 * d;
    o.pos_emb = at;
    at += K * d;
    o.layer0 = at;
    o.layer_stride = 2 * d + 4 * (d * d + d) + 2 * d + d * F + F + F * d + d;
    at += m.n_layers * o.layer_stride;
    o.lnf_g = at;
    at += d;
    o.lnf_b = at;
    at += d;
    o.head_w = at;
    at += 4 * d;
    o.head_b = at;
    at += 4;
    o.bias = at;
    at += 4 * K;
    o.ph_w1 = at;
    at += 2 * K * P;
    o.ph_b1 = at;
    at += P;
    o.ph_w2 = at;
    at += P * P;
    o.ph_b2 = at;
    at += P;
    o.ph_w3 = at;
    at += P;
    o.ph_b3 = at;
    at += 1;
    o.total = at;
    return o;
}

__device__ __forceinline__ double gelu64(double v) { return 0.5 * v * (1.0 + erf(v * 0.70710678118654752440)); }

// out[s][j] = b[j] + sum_i in[s][i] W[i][j] for s < rows, j < n (block-wide)
__device__ void dense_rows64(const double *in, int in_stride, int m, const double *W, int w_stride,
                             const double *b, int rows, int n, double *out, int out_stride, bool accumulate) {
    for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
        const int s = e / n, j = e - (e / n) * n;
        double acc = b ? b[j] : 0.0;
        const double *x = in + (size_t)s * in_stride;
        for (int i = 0; i < m; i++) acc += x[i] * W[(size_t)i * w_stride + j];
        if (accumulate) out[(size_t)s * out_stride + j] += acc;
        else out[(size_t)s * out_stride + j] = acc;
    }
}

__device__ void layer_norm_rows64(const double *in, const double *g, const double *b, int rows, int d,
                                  double *out) {
    for (int s = threadIdx.x; s < rows; s += blockDim.x) {
        const double *x = in + (size_t)s * d;
        double m = 0.0;
        for (int c = 0; c < d; c++) m += x[c];
        m /= d;
        double v = 0.0;
        for (int c = 0; c < d; c++) v += (x[c] - m) * (x[c] - m);
        v /= d;
        const double r = 1.0 / sqrt(v + 1e-5);
        for (int c = 0; c < d; c++) out[(size_t)s * d + c] = (x[c] - m) * r * g[c] + b[c];
    }
}

// Token at autoregressive position s (orbital K-1-s).
__device__ __forceinline__ int token_of(const Key &x, int K, int s) {
    const int i = K - 1 - s;
    return key_bit(x, 2 * i) + 2 * key_bit(x, 2 * i + 1);
}

// One block per configuration, FP64 throughout (model shapes the
// layer-batched forward of model_f64.hip does not cover).
__global__ void __launch_bounds__(256) k_logpsi_f64(ModelView M, const uint64_t *__restrict__ keys, int64_t n,
                                                    double *__restrict__ logabs, double *__restrict__ phase) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int K = M.K, d = M.d, H = M.H, F = M.F, P = M.P, dh = d / H;
    double *h = reinterpret_cast<double *>(smem);
    double *a = h + K * d;
    double *o = a + K * d;
    double *qh = o + K * d;
    double *kh = qh + K * dh;
    double *vh = kh + K * dh;
    double *lp = vh + K * dh;
    double *z1 = lp + K;
    double *z2 = z1 + P;
    int *tok = reinterpret_cast<int *>(z2 + P);
    const double *W = M.w64;
    const LayerOffsets LO = layer_offsets(d, F);
    const double scale = 1.0 / sqrt((double)dh);

    for (int64_t cfg = blockIdx.x; cfg < n; cfg += gridDim.x) {
        Key x;
        x.lo = keys[2 * cfg];
        x.hi = keys[2 * cfg + 1];
        for (int s = threadIdx.x; s < K; s += blockDim.x) tok[s] = token_of(x, K, s);
        __syncthreads();
        for (int e = threadIdx.x; e < K * d; e += blockDim.x) {
            const int s = e / d, c = e - s * d;
            const int prev = s == 0 ? 4 : tok[s - 1];
            h[e] = W[M.off.tok_emb + prev * d + c] + W[M.off.pos_emb + (int64_t)s * d + c];
        }
        __syncthreads();
        for (int l = 0; l < M.L; l++) {
            const double *Lw = W + M.off.layer0 + (int64_t)l * M.off.layer_stride;
            layer_norm_rows64(h, Lw + LO.ln1_g, Lw + LO.ln1_b, K, d, a);
            for (int e = threadIdx.x; e < K * d; e += blockDim.x) o[e] = 0.0;
            __syncthreads();
            for (int hh = 0; hh < H; hh++) {
                dense_rows64(a, d, d, Lw + LO.wq + hh * dh, d, Lw + LO.bq + hh * dh, K, dh, qh, dh, false);
                dense_rows64(a, d, d, Lw + LO.wk + hh * dh, d, Lw + LO.bk + hh * dh, K, dh, kh, dh, false);
                dense_rows64(a, d, d, Lw + LO.wv + hh * dh, d, Lw + LO.bv + hh * dh, K, dh, vh, dh, false);
                __syncthreads();
                // causal attention, one row per thread, streaming softmax
                for (int s = threadIdx.x; s < K; s += blockDim.x) {
                    double mx = -INFINITY, den = 0.0;
                    double *out = o + (size_t)s * d + hh * dh;
                    for (int r = 0; r <= s; r++) {
                        double z = 0.0;
                        for (int c = 0; c < dh; c++) z += qh[s * dh + c] * kh[r * dh + c];
                        z *= scale;
                        const double mn = z > mx ? z : mx;
                        const double corr = exp(mx - mn), p = exp(z - mn);
                        den = den * corr + p;
                        for (int c = 0; c < dh; c++) out[c] = out[c] * corr + p * vh[r * dh + c];
                        mx = mn;
                    }
                    for (int c = 0; c < dh; c++) out[c] /= den;
                }
                __syncthreads();
            }
            dense_rows64(o, d, d, Lw + LO.wo, d, Lw + LO.bo, K, d, h, d, true);
            __syncthreads();
            layer_norm_rows64(h, Lw + LO.ln2_g, Lw + LO.ln2_b, K, d, a);
            __syncthreads();
            for (int c0 = 0; c0 < F; c0 += d) {
                const int wdt = F - c0 < d ? F - c0 : d;
                dense_rows64(a, d, d, Lw + LO.w1 + c0, F, Lw + LO.b1 + c0, K, wdt, o, d, false);
                __syncthreads();
                for (int e = threadIdx.x; e < K * d; e += blockDim.x) {
                    const int c = e - (e / d) * d;
                    if (c < wdt) o[e] = gelu64(o[e]);
                }
                __syncthreads();
                dense_rows64(o, d, wdt, Lw + LO.w2 + (int64_t)c0 * d, d, c0 == 0 ? Lw + LO.b2 : nullptr, K, d, h,
                             d, true);
                __syncthreads();
            }
        }
        // output head, mask and log-probability of the actual token per position
        layer_norm_rows64(h, W + M.off.lnf_g, W + M.off.lnf_b, K, d, a);
        __syncthreads();
        for (int s = threadIdx.x; s < K; s += blockDim.x) {
            int up = 0, dn = 0;
            for (int r = 0; r < s; r++) {
                up += tok[r] & 1;
                dn += tok[r] >> 1;
            }
            const int rem = K - 1 - s, orb = K - 1 - s;
            double z[4];
            double mx = -INFINITY;
            bool ok[4];
            for (int t = 0; t < 4; t++) {
                double acc = W[M.off.head_b + t] + W[M.off.bias + orb * 4 + t];
                for (int c = 0; c < d; c++) acc += a[s * d + c] * W[M.off.head_w + c * 4 + t];
                z[t] = acc;
                const int bu = t & 1, bd = t >> 1;
                ok[t] = (up + bu <= M.n_up) && (dn + bd <= M.n_dn) && (M.n_up - up - bu <= rem) &&
                        (M.n_dn - dn - bd <= rem);
                if (ok[t] && z[t] > mx) mx = z[t];
            }
            double den = 0.0;
            for (int t = 0; t < 4; t++)
                if (ok[t]) den += exp(z[t] - mx);
            const int ts = tok[s];
            lp[s] = ok[ts] ? (z[ts] - mx) - log(den) : -INFINITY;
        }
        // phase MLP on the occupation bits
        for (int j = threadIdx.x; j < P; j += blockDim.x) {
            double acc = W[M.off.ph_b1 + j];
            for (int p = 0; p < 2 * K; p++)
                if (key_bit(x, p)) acc += W[M.off.ph_w1 + (int64_t)p * P + j];
            z1[j] = gelu64(acc);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < P; j += blockDim.x) {
            double acc = W[M.off.ph_b2 + j];
            for (int i = 0; i < P; i++) acc += z1[i] * W[M.off.ph_w2 + (int64_t)i * P + j];
            z2[j] = gelu64(acc);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int t = 0; t < K; t++) s += lp[t];
            double ph = W[M.off.ph_b3];
            for (int i = 0; i < P; i++) ph += z2[i] * W[M.off.ph_w3 + i];
            logabs[cfg] = 0.5 * s;
            phase[cfg] = ph;
        }
        __syncthreads();
    }
}

size_t f64_lds_bytes(const nnqs_model_desc &m) {
    const size_t K = m.n_orb, d = m.d_model, dh = m.d_model / m.n_heads;
    return (3 * K * d + 3 * K * dh + K + 2 * (size_t)m.phase_hidden) * sizeof(double) + K * sizeof(int);
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

int64_t nnqs_model_weight_count(const nnqs_model_desc *m) {
    if (!m) return -1;
    if (m->n_orb < 2 || m->n_orb > 64 || m->d_model < 1 || m->d_model > 128 || m->n_heads < 1 ||
        m->d_model % m->n_heads || m->n_layers < 1 || m->d_ff < 1 || m->d_ff > 1024 || m->phase_hidden < 1 ||
        m->phase_hidden > 1024 || m->n_up < 0 || m->n_dn < 0 || m->n_up > m->n_orb || m->n_dn > m->n_orb)
        return -1;
    return model_offsets(*m).total;
}

nnqs_status nnqs_model_create(nnqs_model **out, const nnqs_model_desc *desc, const float *weights) {
    clear_error();
    if (!out || !desc || !weights) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    const int64_t nw = nnqs_model_weight_count(desc);
    if (nw < 0) return fail(NNQS_EINVAL, "invalid model description");
    int dev = 0;
    NNQS_HIP_CHECK(hipGetDevice(&dev));
    int lds = 0;
    NNQS_HIP_CHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (f64_lds_bytes(*desc) > (size_t)lds) return fail(NNQS_EUNSUPPORTED, "model too large for the FP64 path");
    nnqs_model *m = new nnqs_model();
    m->desc = *desc;
    m->off = model_offsets(*desc);
    m->max_lds = lds;
    std::vector<double> w64(weights, weights + nw);
    if (hipMalloc(&m->d_w64, nw * sizeof(double)) != hipSuccess) {
        delete m;
        return fail(NNQS_ENOMEM, "device allocation of the model failed");
    }
    if (hipMemcpy(m->d_w64, w64.data(), nw * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        nnqs_model_destroy(m);
        return fail(NNQS_EHIP, "copy of the model weights failed");
    }
    nnqs_status st = bf16_model_init(m, weights);
    if (st != NNQS_OK) {
        nnqs_model_destroy(m);
        return st;
    }
    *out = m;
    return NNQS_OK;
}

nnqs_status nnqs_model_destroy(nnqs_model *m) {
    if (!m) return NNQS_OK;
    hipFree(m->d_w64);
    hipFree(m->d_f64s);
    hipFree(m->d_grads);
    bf16_model_free(m);
    eloc_model_free(m);
    delete m;
    return NNQS_OK;
}

nnqs_status nnqs_model_logpsi(const nnqs_model *m, const uint64_t *keys, int64_t n, int32_t precision,
                              double *logabs, double *phase, void *stream) {
    clear_error();
    if (!m || !keys || !logabs || !phase) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    return enqueue_logpsi(m, keys, n, precision, logabs, phase, as_stream(stream));
}

}  // extern "C"

namespace nnqs {

ModelView model_view(const nnqs_model *m) {
    ModelView v{};
    v.K = m->desc.n_orb;
    v.d = m->desc.d_model;
    v.L = m->desc.n_layers;
    v.H = m->desc.n_heads;
    v.F = m->desc.d_ff;
    v.P = m->desc.phase_hidden;
    v.n_up = m->desc.n_up;
    v.n_dn = m->desc.n_dn;
    v.w64 = m->d_w64;
    v.off = m->off;
    return v;
}

nnqs_status enqueue_logpsi(const nnqs_model *m, const uint64_t *keys, int64_t n, int32_t precision,
                           double *logabs, double *phase, hipStream_t st) {
    if (precision == NNQS_FP64 && f64_shape_ok(m->desc)) return enqueue_logpsi_f64(m, keys, n, logabs, phase, st);
    if (precision == NNQS_FP64) {  // other shapes: one block per configuration
        const size_t lds = f64_lds_bytes(m->desc);
        NNQS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_logpsi_f64),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        const int64_t grid = n < 65536 ? n : 65536;
        hipLaunchKernelGGL(k_logpsi_f64, dim3((unsigned)grid), dim3(256), lds, st, model_view(m), keys, n, logabs,
                           phase);
        NNQS_HIP_CHECK(hipGetLastError());
        return NNQS_OK;
    }
    if (precision == NNQS_BF16) return enqueue_logpsi_bf16(m, keys, n, logabs, phase, st, false);
    if (precision == NNQS_FP8) return enqueue_logpsi_bf16(m, keys, n, logabs, phase, st, true);
    return fail(NNQS_EUNSUPPORTED, "unknown precision %d", precision);
}

}  // namespace nnqs

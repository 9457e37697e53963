// Batch autoregressive sampling (paper: Section 3.1) on the device: the
// samples of one VMC iteration are drawn together by following the unique
// prefixes of the autoregressive ansatz with their weights.  At sequence
// position s every unique prefix u (weight c_u) gets its conditional
// pi(t | prefix) from the network (the Eq. 12 mask included), each of its
// c_u sample slots draws one token from a counter-based generator, which
// splits c_u multinomially among the four children, and children with zero
// weight are dropped.  After K positions the prefixes are the unique samples
// and their weights the occurrence counts.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011),
// counter (slot mod 2^32, slot / 2^32, s, 0x42415300), key = the seed, the
// top 53 bits of the first two output words; slots are numbered in prefix
// order, children are kept in (parent, token) order, so the result depends
// only on the seed and the conditionals.
#include <algorithm>
#include <cmath>

#include "model.hpp"

namespace nnqs {

__device__ __forceinline__ double bas_uniform(uint64_t seed, int s, uint64_t i) {
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = (uint32_t)s, c3 = 0x42415300u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    const uint64_t x = ((uint64_t)c0 << 32) | c1;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

// Token of a slot: the allowed tokens in order 0..3, probabilities summed
// until the running sum exceeds u (the last allowed one if rounding leaves u
// above the total).
__device__ __forceinline__ int bas_token(const double *logp, double u) {
    double acc = 0.0;
    int last = -1;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        if (!(logp[t] > -INFINITY)) continue;
        last = t;
        acc += exp(logp[t]);
        if (u < acc) return t;
    }
    return last;
}

// One token per sample slot i < total; slot i belongs to the prefix u with
// offs[u] <= i < offs[u + 1].  The lanes of a wave that land on the same
// (prefix, token) add their count with one atomic.
__global__ void __launch_bounds__(256) k_bas_draw(uint64_t total, int s, uint64_t seed,
                                                  const uint64_t *__restrict__ offs, int64_t n,
                                                  const double *__restrict__ cond,
                                                  unsigned long long *__restrict__ child) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < total; base += stride) {
        const uint64_t i = base + lane;
        int64_t key = -1;
        if (i < total) {
            int64_t lo = 0, hi = n;  // offs[lo] <= i < offs[hi]
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (offs[mid] <= i) lo = mid;
                else hi = mid;
            }
            const int t = bas_token(cond + 4 * lo, bas_uniform(seed, s, i));
            key = t >= 0 ? 4 * lo + t : -1;  // no allowed token: the prefix leaves the sector (not for valid models)
        }
        uint64_t pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int64_t lk = __shfl(key, leader, 64);
            const uint64_t same = __ballot(key == lk);
            if (lane == leader) atomicAdd(child + lk, (unsigned long long)__popcll(same));
            pending &= ~same;
        }
    }
}

// Exclusive prefix sums of n values (one block; each thread scans a
// contiguous run) into out[0..n], out[n] = the total.
template <typename T, typename F>
__global__ void __launch_bounds__(1024) k_bas_scan(int64_t n, F value, T *__restrict__ out) {
    __shared__ T part[1025];
    const int64_t per = (n + 1023) / 1024;
    const int64_t b0 = threadIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
    T run = 0;
    for (int64_t k = b0; k < b1; k++) run += value(k);
    part[threadIdx.x + 1] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[0] = 0;
        for (int t = 1; t <= 1024; t++) part[t] += part[t - 1];
    }
    __syncthreads();
    T pos = part[threadIdx.x];
    for (int64_t k = b0; k < b1; k++) {
        out[k] = pos;
        pos += value(k);
    }
    if (threadIdx.x == 0) out[n] = part[1024];
}

struct CountOf {
    const uint64_t *c;
    __device__ uint64_t operator()(int64_t k) const { return c[k]; }
};
struct ChildrenOf {
    const unsigned long long *child;
    __device__ int64_t operator()(int64_t k) const {
        return (int64_t)(child[4 * k] > 0) + (child[4 * k + 1] > 0) + (child[4 * k + 2] > 0) + (child[4 * k + 3] > 0);
    }
};

__global__ void k_bas_zero(unsigned long long *p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0;
}

// Children of prefix u, in token order, at pos[u]...: the parent's key with
// the token of position s (spatial orbital K-1-s: up bit 2i, down bit 2i+1),
// its slot count and the path's log-probability.
__global__ void k_bas_expand(int64_t n, int K, int s, const uint64_t *__restrict__ keys, const double *__restrict__ lp,
                             const double *__restrict__ cond, const unsigned long long *__restrict__ child,
                             const int64_t *__restrict__ pos, uint64_t *__restrict__ nkeys, uint64_t *__restrict__ ncnt,
                             double *__restrict__ nlp) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int i = K - 1 - s;
    int64_t p = pos[u];
    for (int t = 0; t < 4; t++) {
        const unsigned long long c = child[4 * u + t];
        if (!c) continue;
        Key x;
        x.lo = keys[2 * u];
        x.hi = keys[2 * u + 1];
        if (t & 1) key_flip(x, 2 * i);
        if (t & 2) key_flip(x, 2 * i + 1);
        nkeys[2 * p] = x.lo;
        nkeys[2 * p + 1] = x.hi;
        ncnt[p] = c;
        nlp[p] = lp[u] + cond[4 * u + t];
        p++;
    }
}

__global__ void k_bas_finish(int64_t n, const uint64_t *__restrict__ cnt, const double *__restrict__ lp,
                             uint32_t *__restrict__ counts_out, double *__restrict__ logabs_out) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    counts_out[u] = (uint32_t)cnt[u];
    logabs_out[u] = 0.5 * lp[u];
}

__global__ void k_bas_init(uint64_t *keys, uint64_t *cnt, double *lp, uint64_t total) {
    keys[0] = 0ull;
    keys[1] = 0ull;
    cnt[0] = total;
    lp[0] = 0.0;
}

struct BasScratch {
    uint64_t *pk = nullptr, *nk = nullptr, *pc = nullptr, *nc = nullptr, *offs = nullptr;
    double *pl = nullptr, *nl = nullptr, *cond = nullptr, *la = nullptr, *ph = nullptr;
    unsigned long long *child = nullptr;
    int64_t *pos = nullptr;
    ~BasScratch() {
        hipFree(pk);
        hipFree(nk);
        hipFree(pc);
        hipFree(nc);
        hipFree(offs);
        hipFree(pl);
        hipFree(nl);
        hipFree(cond);
        hipFree(la);
        hipFree(ph);
        hipFree(child);
        hipFree(pos);
    }
};

}  // namespace nnqs

using namespace nnqs;

extern "C" nnqs_status nnqs_bas(nnqs_model *model, int32_t precision, uint64_t seed, uint64_t n_samples,
                                int64_t capacity, uint64_t *keys_out, uint32_t *counts_out, double *logabs_out,
                                double *phase_out, int64_t *n_unique, void *stream) {
    clear_error();
    if (!model || !keys_out || !counts_out || !logabs_out || !n_unique) return fail(NNQS_EINVAL, "null pointer argument");
    if (n_samples < 1 || n_samples > 0xFFFFFFFFull) return fail(NNQS_EINVAL, "n_samples must be in [1, 2^32 - 1]");
    if (capacity < 1) return fail(NNQS_EINVAL, "capacity must be positive");
    if (precision == NNQS_FP64 && !f64_shape_ok(model->desc))
        return fail(NNQS_EUNSUPPORTED, "FP64 sampling needs d_model 64 and 4 heads");
    if (precision == NNQS_BF16 && !model->bf16_ok) return fail(NNQS_EUNSUPPORTED, "model shape has no BF16 path");
    if (precision != NNQS_FP64 && precision != NNQS_BF16) return fail(NNQS_EUNSUPPORTED, "sampling runs in FP64 or BF16");
    hipStream_t st = as_stream(stream);
    const int K = model->desc.n_orb;
    const size_t cap = (size_t)capacity;
    BasScratch S;
    if (hipMalloc(&S.pk, cap * 16) != hipSuccess || hipMalloc(&S.nk, cap * 16) != hipSuccess ||
        hipMalloc(&S.pc, cap * 8) != hipSuccess || hipMalloc(&S.nc, cap * 8) != hipSuccess ||
        hipMalloc(&S.offs, (cap + 1) * 8) != hipSuccess || hipMalloc(&S.pl, cap * 8) != hipSuccess ||
        hipMalloc(&S.nl, cap * 8) != hipSuccess || hipMalloc(&S.cond, cap * 32) != hipSuccess ||
        hipMalloc(&S.la, cap * 8) != hipSuccess || hipMalloc(&S.ph, cap * 8) != hipSuccess ||
        hipMalloc(&S.child, cap * 32) != hipSuccess || hipMalloc(&S.pos, (cap + 1) * 8) != hipSuccess)
        return fail(NNQS_ENOMEM, "sampling scratch for %lld prefixes", (long long)capacity);
    hipLaunchKernelGGL(k_bas_init, dim3(1), dim3(1), 0, st, S.pk, S.pc, S.pl, (uint64_t)n_samples);
    int64_t n = 1;
    for (int s = 0; s < K; s++) {
        nnqs_status r = precision == NNQS_FP64 ? enqueue_logpsi_f64(model, S.pk, n, S.la, S.ph, st, s, S.cond)
                                               : enqueue_bf16_cond(model, S.pk, n, s, S.cond, S.la, st);
        if (r != NNQS_OK) return r;
        hipLaunchKernelGGL((k_bas_scan<uint64_t, CountOf>), dim3(1), dim3(1024), 0, st, n, CountOf{S.pc}, S.offs);
        hipLaunchKernelGGL(k_bas_zero, dim3((unsigned)std::min<int64_t>((4 * n + 255) / 256, 4096)), dim3(256), 0, st,
                           S.child, 4 * n);
        const unsigned dg = (unsigned)std::min<uint64_t>((n_samples + 255) / 256, 8192);
        hipLaunchKernelGGL(k_bas_draw, dim3(dg), dim3(256), 0, st, (uint64_t)n_samples, s, seed, (const uint64_t *)S.offs,
                           n, (const double *)S.cond, S.child);
        hipLaunchKernelGGL((k_bas_scan<int64_t, ChildrenOf>), dim3(1), dim3(1024), 0, st, n, ChildrenOf{S.child},
                           S.pos);
        int64_t m = 0;
        NNQS_HIP_CHECK(hipMemcpyAsync(&m, S.pos + n, 8, hipMemcpyDeviceToHost, st));
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        if (m > capacity) return fail(NNQS_ERANGE, "%lld prefixes at position %d exceed the capacity %lld", (long long)m, s,
                                      (long long)capacity);
        hipLaunchKernelGGL(k_bas_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, K, s,
                           (const uint64_t *)S.pk, (const double *)S.pl, (const double *)S.cond,
                           (const unsigned long long *)S.child, (const int64_t *)S.pos, S.nk, S.nc, S.nl);
        NNQS_HIP_CHECK(hipGetLastError());
        std::swap(S.pk, S.nk);
        std::swap(S.pc, S.nc);
        std::swap(S.pl, S.nl);
        n = m;
    }
    NNQS_HIP_CHECK(hipMemcpyAsync(keys_out, S.pk, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_bas_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, (const uint64_t *)S.pc,
                       (const double *)S.pl, counts_out, logabs_out);
    NNQS_HIP_CHECK(hipGetLastError());
    if (phase_out) {
        nnqs_status r = enqueue_logpsi(model, keys_out, n, precision, S.la, phase_out, st);
        if (r != NNQS_OK) return r;
    }
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    *n_unique = n;
    return NNQS_OK;
}

// Core objects of libnnqs_eloc: error reporting, the Hamiltonian system,
// the sorted sample table (device bitonic sort, membership filter and staged
// search keys) and the deterministic weighted-energy reduction of Eq. 6.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <atomic>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace nnqs {

static thread_local char g_err[512] = "";

nnqs_status fail(nnqs_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

// SplitMix64 (Steele, Lea, Flood 2014): fills the per-spin-orbital hash words.
static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

TableView table_view(const nnqs_table *t) {
    TableView v{};
    v.keys = t->keys;
    v.logabs = t->logabs;
    v.phase = t->phase;
    v.filter = t->filter;
    v.split = t->split;
    v.amp = t->amp;
    v.lmax = t->lmax;
    v.n = t->n;
    int L = 0;
    while ((int64_t(1) << L) < t->n) L++;
    v.log2n = L;
    v.filter_log2 = t->filter_log2;
    v.split_levels = t->split_levels < L ? t->split_levels : L;
    return v;
}

// The view a build of n samples with the table's current tune will produce.
TableView table_view_planned(const nnqs_table *t, int64_t n) {
    TableView v = table_view(t);
    v.n = n;
    int L = 0;
    while ((int64_t(1) << L) < n) L++;
    v.log2n = L;
    v.filter_log2 = t->tune.filter_log2_bits;
    v.split_levels = t->tune.splitter_levels < L ? t->tune.splitter_levels : L;
    return v;
}

// ------------------------------------------------------------- sorting
// Total order on (key word 1, key word 0, original index): padding entries
// carry index 0xFFFFFFFF and sort last even against an all-ones key.
__device__ __forceinline__ bool elem_greater(uint64_t ahi, uint64_t alo, uint32_t ai, uint64_t bhi, uint64_t blo,
                                             uint32_t bi) {
    if (ahi != bhi) return ahi > bhi;
    if (alo != blo) return alo > blo;
    return ai > bi;
}

__global__ void k_sort_init(const uint64_t *__restrict__ keys, int64_t n, int64_t P, uint64_t *__restrict__ sk,
                            uint32_t *__restrict__ si) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    if (i < n) {
        sk[2 * i] = keys[2 * i];
        sk[2 * i + 1] = keys[2 * i + 1];
        si[i] = (uint32_t)i;
    } else {
        sk[2 * i] = ~0ull;
        sk[2 * i + 1] = ~0ull;
        si[i] = 0xFFFFFFFFu;
    }
}

// One compare-exchange stage (k, j) of the bitonic network over P entries.
__global__ void k_bitonic_global(uint64_t *__restrict__ sk, uint32_t *__restrict__ si, int64_t P, int64_t k,
                                 int64_t j) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P / 2) return;
    int64_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    int64_t l = i + j;
    bool asc = (i & k) == 0;
    uint64_t alo = sk[2 * i], ahi = sk[2 * i + 1], blo = sk[2 * l], bhi = sk[2 * l + 1];
    uint32_t ai = si[i], bi = si[l];
    bool g = elem_greater(ahi, alo, ai, bhi, blo, bi);
    if (g == asc) {
        sk[2 * i] = blo;
        sk[2 * i + 1] = bhi;
        si[i] = bi;
        sk[2 * l] = alo;
        sk[2 * l + 1] = ahi;
        si[l] = ai;
    }
}

// Two consecutive global stages (k, j) and (k, j/2) in one pass: thread t
// owns the four elements a, a + h, a + 2h, a + 3h (h = j/2; a has bits h and
// j clear), which both stages only compare among themselves.
__device__ __forceinline__ void bitonic_cas(uint64_t &alo, uint64_t &ahi, uint32_t &ai, uint64_t &blo, uint64_t &bhi,
                                            uint32_t &bi, bool asc) {
    if (elem_greater(ahi, alo, ai, bhi, blo, bi) == asc) {
        uint64_t tl = alo, th = ahi;
        uint32_t ti = ai;
        alo = blo;
        ahi = bhi;
        ai = bi;
        blo = tl;
        bhi = th;
        bi = ti;
    }
}
__global__ void k_bitonic_global2(uint64_t *__restrict__ sk, uint32_t *__restrict__ si, int64_t P, int64_t k,
                                  int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P / 4) return;
    const int64_t h = j >> 1;
    const int64_t a = ((t & ~(h - 1)) << 2) | (t & (h - 1));
    const bool asc = (a & k) == 0;
    uint64_t lo[4], hi[4];
    uint32_t ix[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t e = a + q * h;
        lo[q] = sk[2 * e];
        hi[q] = sk[2 * e + 1];
        ix[q] = si[e];
    }
    // stage j: (0, 2), (1, 3); stage j/2: (0, 1), (2, 3)
    bitonic_cas(lo[0], hi[0], ix[0], lo[2], hi[2], ix[2], asc);
    bitonic_cas(lo[1], hi[1], ix[1], lo[3], hi[3], ix[3], asc);
    bitonic_cas(lo[0], hi[0], ix[0], lo[1], hi[1], ix[1], asc);
    bitonic_cas(lo[2], hi[2], ix[2], lo[3], hi[3], ix[3], asc);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t e = a + q * h;
        sk[2 * e] = lo[q];
        sk[2 * e + 1] = hi[q];
        si[e] = ix[q];
    }
}

// All stages with j < tile inside one LDS tile.  Runs k = k_lo..k_hi
// (powers of two); the first k starts at j = j_start, later ones at k/2.
__global__ void k_bitonic_local(uint64_t *__restrict__ sk, uint32_t *__restrict__ si, int tile, int64_t k_lo,
                                int64_t k_hi, int64_t j_start) {
    extern __shared__ uint8_t smem[];
    uint64_t *lk = reinterpret_cast<uint64_t *>(smem);
    uint32_t *li = reinterpret_cast<uint32_t *>(smem + (size_t)tile * 16);
    const int64_t base = (int64_t)blockIdx.x * tile;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) {
        lk[2 * e] = sk[2 * (base + e)];
        lk[2 * e + 1] = sk[2 * (base + e) + 1];
        li[e] = si[base + e];
    }
    __syncthreads();
    // A stage with stride j <= 64 pairs only elements of the 128-element
    // block of one wave (thread t takes pair t), so two consecutive such
    // stages need no block barrier, only the wave's own LDS ordering.
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k == k_lo ? j_start : k >> 1); j >= 1; j >>= 1) {
            const int64_t jn = j > 1 ? j >> 1 : (k < k_hi ? k : 0);  // stride of the next stage (0: none)
            for (int t = threadIdx.x; t < tile / 2; t += blockDim.x) {
                int i = (int)(((t & ~(j - 1)) << 1) | (t & (j - 1)));
                int l = i + (int)j;
                bool asc = ((base + i) & k) == 0;
                uint64_t alo = lk[2 * i], ahi = lk[2 * i + 1], blo = lk[2 * l], bhi = lk[2 * l + 1];
                uint32_t ai = li[i], bi = li[l];
                bool g = elem_greater(ahi, alo, ai, bhi, blo, bi);
                if (g == asc) {
                    lk[2 * i] = blo;
                    lk[2 * i + 1] = bhi;
                    li[i] = bi;
                    lk[2 * l] = alo;
                    lk[2 * l + 1] = ahi;
                    li[l] = ai;
                }
            }
            if (j > 64 || jn > 64 || jn == 0 || tile / 2 > (int)blockDim.x) {
                __syncthreads();
            } else {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    for (int e = threadIdx.x; e < tile; e += blockDim.x) {
        sk[2 * (base + e)] = lk[2 * e];
        sk[2 * (base + e) + 1] = lk[2 * e + 1];
        si[base + e] = li[e];
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ bool key_conserves(const SysView &S, uint64_t lo, uint64_t hi) {
    if ((lo & ~S.valid0) | (hi & ~S.valid1)) return false;
    int up = __popcll(lo & EVEN_BITS) + __popcll(hi & EVEN_BITS);
    int dn = __popcll(lo & ODD_BITS) + __popcll(hi & ODD_BITS);
    return up == S.n_up && dn == S.n_dn;
}

// GF(2)-linear hash of a key: XOR of the hash words of its set bits.
__device__ __forceinline__ uint64_t key_hash(const SysView &S, uint64_t lo, uint64_t hi) {
    uint64_t h = 0;
    while (lo) {
        int b = __ffsll((unsigned long long)lo) - 1;
        lo &= lo - 1;
        h ^= S.hashT[b];
    }
    while (hi) {
        int b = __ffsll((unsigned long long)hi) - 1;
        hi &= hi - 1;
        h ^= S.hashT[64 + b];
    }
    return h;
}

// Gather the payload in sorted order, check the table, set filter bits.
__global__ void k_table_finalize(SysView S, const uint64_t *__restrict__ sk, const uint32_t *__restrict__ si,
                                 const double *__restrict__ la_in, const double *__restrict__ ph_in, int64_t n,
                                 uint64_t *__restrict__ keys, double *__restrict__ la, double *__restrict__ ph,
                                 uint32_t *__restrict__ filter, int filter_log2, int *status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t lo = sk[2 * i], hi = sk[2 * i + 1];
    uint32_t src = si[i];
    keys[2 * i] = lo;
    keys[2 * i + 1] = hi;
    double l = la_in[src];
    la[i] = l;
    ph[i] = ph_in[src];
    if (i > 0 && sk[2 * i - 2] == lo && sk[2 * i - 1] == hi) set_status(status, NNQS_EDUP);
    if (!isfinite(l) || !isfinite(ph_in[src])) set_status(status, NNQS_ERANGE);
    if (!key_conserves(S, lo, hi)) set_status(status, NNQS_ECONSERVE);
    const uint32_t h = (uint32_t)key_hash(S, lo, hi);
    const uint32_t words_mask = (1u << (filter_log2 - 5)) - 1u;
    atomicOr(&filter[filter_word(h, words_mask)], filter_bits(h));
}

// Largest log-amplitude of the table: block maxima, then one block folds
// them (max is exact, so the result does not depend on the order).
__global__ void __launch_bounds__(256) k_table_max_partial(const double *__restrict__ la, int64_t n,
                                                           double *__restrict__ part) {
    __shared__ double sh[256];
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, la[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[1 + blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_table_max_final(double *__restrict__ part, int nblocks) {
    __shared__ double sh[256];
    double m = -INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmax(m, part[1 + b]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = sh[0];
}

// amp[i] = exp(logabs[i] - lmax) (cos phase[i], sin phase[i]): the hit path
// of the sample-aware kernel multiplies this by exp(lmax - log|psi(x)|)
// e^{-i phase(x)} instead of evaluating exp and sincos per hit.
__global__ void k_table_amp(const double *__restrict__ la, const double *__restrict__ ph, int64_t n,
                            const double *__restrict__ lmax, double *__restrict__ amp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = exp(la[i] - lmax[0]);
    double sn, cs;
    sincos(ph[i], &sn, &cs);
    amp[2 * i] = r * cs;
    amp[2 * i + 1] = r * sn;
}

__global__ void k_table_split(const uint64_t *__restrict__ keys, int64_t n, int log2n, int levels,
                              uint64_t *__restrict__ split) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t cnt = (int64_t(1) << levels) - 1;
    if (j >= cnt) return;
    int64_t pos = ((j + 1) << (log2n - levels)) - 1;
    if (pos < n) {
        split[2 * j] = keys[2 * pos];
        split[2 * j + 1] = keys[2 * pos + 1];
    } else {
        split[2 * j] = ~0ull;
        split[2 * j + 1] = ~0ull;
    }
}

// ----------------------------------------------------- energy reduction
// Eq. 6 over unique samples in two passes, each a deterministic compensated
// tree: pass 1 sums (c, c Re, c Im) and fixes E = sum c Re / sum c; pass 2
// sums c (Re - E)^2 with E read back from the device, so the variance keeps
// its digits as it approaches zero (an eigenstate gives E_loc = E for every
// sample).  Each pass: every block reduces a strided share of the samples
// into partials (value and compensation per quantity), one block folds them
// in a fixed order.
template <int Q>
__device__ __forceinline__ void block_fold(NSum (&acc)[Q], double (*sh)[8]) {
    for (int q = 0; q < Q; q++) {
        sh[threadIdx.x][2 * q] = acc[q].s;
        sh[threadIdx.x][2 * q + 1] = acc[q].c;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < Q; q++) {
                double a = sh[threadIdx.x][2 * q], ac = sh[threadIdx.x][2 * q + 1];
                nsum_merge(a, ac, sh[threadIdx.x + w][2 * q], sh[threadIdx.x + w][2 * q + 1]);
                sh[threadIdx.x][2 * q] = a;
                sh[threadIdx.x][2 * q + 1] = ac;
            }
        }
        __syncthreads();
    }
}

// Pass 1, stage 1: partials of (c, c Re, c Im), six doubles per block.
__global__ void __launch_bounds__(256) k_energy_partial(const uint32_t *__restrict__ counts,
                                                        const double *__restrict__ eloc, int64_t n,
                                                        double *__restrict__ partials) {
    __shared__ double sh[256][8];
    NSum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double c = (double)counts[k];
        acc[0].add(c);
        acc[1].add(c * eloc[2 * k]);
        acc[2].add(c * eloc[2 * k + 1]);
    }
    block_fold<3>(acc, sh);
    if (threadIdx.x < 6) partials[blockIdx.x * 8 + threadIdx.x] = sh[0][threadIdx.x];
}

// Pass 1, stage 2: E, Im and the weight sum into energy[0..2].
__global__ void __launch_bounds__(256) k_energy_mean(const double *__restrict__ partials, int nblocks,
                                                     double *__restrict__ energy) {
    __shared__ double sh[256][8];
    NSum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int q = 0; q < 3; q++) nsum_merge(acc[q].s, acc[q].c, partials[b * 8 + 2 * q], partials[b * 8 + 2 * q + 1]);
    block_fold<3>(acc, sh);
    if (threadIdx.x == 0) {
        const double W = sh[0][0] + sh[0][1];
        energy[0] = (sh[0][2] + sh[0][3]) / W;
        energy[1] = (sh[0][4] + sh[0][5]) / W;
        energy[2] = W;
    }
}

// Pass 2, stage 1: partials of c (Re - E)^2, E = energy[0].
__global__ void __launch_bounds__(256) k_energy_var_partial(const uint32_t *__restrict__ counts,
                                                            const double *__restrict__ eloc, int64_t n,
                                                            const double *__restrict__ energy,
                                                            double *__restrict__ partials) {
    __shared__ double sh[256][8];
    NSum acc[1] = {{0, 0}};
    const double E = energy[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double d = eloc[2 * k] - E;
        acc[0].add((double)counts[k] * d * d);
    }
    block_fold<1>(acc, sh);
    if (threadIdx.x < 2) partials[blockIdx.x * 8 + threadIdx.x] = sh[0][threadIdx.x];
}

// Pass 2, stage 2: the variance into energy[3].
__global__ void __launch_bounds__(256) k_energy_var(const double *__restrict__ partials, int nblocks,
                                                    double *__restrict__ energy) {
    __shared__ double sh[256][8];
    NSum acc[1] = {{0, 0}};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) nsum_merge(acc[0].s, acc[0].c, partials[b * 8], partials[b * 8 + 1]);
    block_fold<1>(acc, sh);
    if (threadIdx.x == 0) energy[3] = (sh[0][0] + sh[0][1]) / energy[2];
}

// Enqueues both passes with `partials` (>= 8 * kPartialBlocks doubles) as
// scratch; the second pass reuses it after the first has been folded.
nnqs_status enqueue_energy_partials(double *partials, const uint32_t *counts, const double *eloc, int64_t n,
                                    double *energy, hipStream_t st) {
    int64_t blocks = (n + 1023) / 1024;
    if (blocks < 1) blocks = 1;
    if (blocks > kPartialBlocks) blocks = kPartialBlocks;
    hipLaunchKernelGGL(k_energy_partial, dim3((unsigned)blocks), dim3(256), 0, st, counts, eloc, n, partials);
    hipLaunchKernelGGL(k_energy_mean, dim3(1), dim3(256), 0, st, partials, (int)blocks, energy);
    hipLaunchKernelGGL(k_energy_var_partial, dim3((unsigned)blocks), dim3(256), 0, st, counts, eloc, n,
                       (const double *)energy, partials);
    hipLaunchKernelGGL(k_energy_var, dim3(1), dim3(256), 0, st, partials, (int)blocks, energy);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

nnqs_status enqueue_energy(nnqs_table *tab, const uint32_t *counts, const double *eloc, int64_t n, double *energy,
                           hipStream_t st) {
    return enqueue_energy_partials(tab->partials, counts, eloc, n, energy, st);
}

// Scratch of nnqs_energy_noalloc: the block partials of both reduction
// passes (8 doubles for each of at most kPartialBlocks blocks, 64 KiB).
// Every GPU the library runs on holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).
static __device__ __align__(256) double scratch[kPartialBlocks * 8];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Address of `scratch` on the current device, looked up once per device.
static nnqs_status noalloc_scratch(double **out) {
    int dev = 0;
    NNQS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NNQS_EUNSUPPORTED, "device ordinal %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NNQS_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return NNQS_OK;
}

// ------------------------------------------------------------- timing
struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
static std::mutex g_timing_mu;
static std::atomic<bool> g_timing{false};
static std::vector<TimingRec> g_timing_recs;

static void timing_clear_locked() {
    for (auto &r : g_timing_recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_timing_recs.clear();
}

TimedRegion::TimedRegion(const char *name, hipStream_t st) : name_(name), st_(st) {
    if (!g_timing.load(std::memory_order_relaxed)) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess ||
        hipEventRecord(a_, st_) != hipSuccess) {
        if (a_) hipEventDestroy(a_);
        if (b_) hipEventDestroy(b_);
        a_ = b_ = nullptr;
    }
}

TimedRegion::~TimedRegion() {
    if (!a_) return;
    if (hipEventRecord(b_, st_) != hipSuccess) {
        hipEventDestroy(a_);
        hipEventDestroy(b_);
        return;
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_recs.push_back({name_, a_, b_});
}

nnqs_status read_status(nnqs_table *tab, hipStream_t st, bool clear) {
    int h = 0;
    NNQS_HIP_CHECK(hipMemcpyAsync(&h, tab->status, sizeof(int), hipMemcpyDeviceToHost, st));
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    if (clear && h != 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, reinterpret_cast<uint32_t *>(tab->status), 1, 0u);
        NNQS_HIP_CHECK(hipGetLastError());
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
    }
    return (nnqs_status)h;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

const char *nnqs_last_error(void) { return g_err; }

const char *nnqs_version(void) { return "nnqs_eloc 0.1 (gfx950)"; }

nnqs_status nnqs_system_create(nnqs_system **out, int32_t n_spin_orb, int32_t n_up, int32_t n_dn, const double *h,
                               const double *g, double e_core) {
    clear_error();
    if (!out || !h || !g) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n_spin_orb < 4 || n_spin_orb > 128 || (n_spin_orb & 1))
        return fail(NNQS_EINVAL, "n_spin_orb=%d must be even and in [4, 128]", n_spin_orb);
    const int K = n_spin_orb / 2;
    if (n_up < 0 || n_dn < 0 || n_up > K || n_dn > K)
        return fail(NNQS_EINVAL, "electron numbers (%d, %d) outside [0, K=%d]", n_up, n_dn, K);
    if (!std::isfinite(e_core)) return fail(NNQS_EINVAL, "e_core is not finite");
    int dev = 0;
    NNQS_HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    NNQS_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(NNQS_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);

    const size_t KK = (size_t)K * K, K4 = KK * KK;
    std::vector<double> J(KK), Kx(KK);
    for (int i = 0; i < K; i++)
        for (int j = 0; j < K; j++) {
            J[i * K + j] = g[(((size_t)i * K + i) * K + j) * K + j];
            Kx[i * K + j] = g[(((size_t)i * K + j) * K + j) * K + i];
        }
    std::vector<uint64_t> hashT(128);
    uint64_t seed = 0x2306167050000000ull;
    for (auto &v : hashT) v = splitmix64(seed);

    nnqs_system *s = new nnqs_system();
    auto cleanup = [&](nnqs_status st) {
        nnqs_system_destroy(s);
        return st;
    };
    if (hipMalloc(&s->d_h, KK * sizeof(double)) != hipSuccess || hipMalloc(&s->d_g, K4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->d_J, KK * sizeof(double)) != hipSuccess || hipMalloc(&s->d_K, KK * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->d_hash, 128 * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&s->d_status, sizeof(int)) != hipSuccess)
        return cleanup(fail(NNQS_ENOMEM, "device allocation of the integrals failed"));
    if (hipMemcpy(s->d_h, h, KK * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_g, g, K4 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_J, J.data(), KK * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_K, Kx.data(), KK * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_hash, hashT.data(), 128 * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(NNQS_EHIP, "copy of the integrals to the device failed"));

    SysView &v = s->view;
    v.K = K;
    v.N = n_spin_orb;
    v.n_up = n_up;
    v.n_dn = n_dn;
    const int64_t vu = K - n_up, vd = K - n_dn;
    v.C = 1 + n_up * vu + n_dn * vd + (int64_t)n_up * (n_up - 1) / 2 * (vu * (vu - 1) / 2) +
          (int64_t)n_dn * (n_dn - 1) / 2 * (vd * (vd - 1) / 2) + n_up * vu * n_dn * vd;
    v.h = s->d_h;
    v.g = s->d_g;
    v.Jm = s->d_J;
    v.Km = s->d_K;
    v.hashT = s->d_hash;
    v.ecore = e_core;
    v.valid0 = n_spin_orb >= 64 ? ~0ull : ((1ull << n_spin_orb) - 1ull);
    v.valid1 = n_spin_orb <= 64 ? 0ull : (n_spin_orb == 128 ? ~0ull : ((1ull << (n_spin_orb - 64)) - 1ull));
    s->device = dev;
    s->cu_count = prop.multiProcessorCount;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
        lds = 65536;
    s->max_lds = lds;
    *out = s;
    return NNQS_OK;
}

nnqs_status nnqs_system_destroy(nnqs_system *s) {
    if (!s) return NNQS_OK;
    hipFree(s->d_h);
    hipFree(s->d_g);
    hipFree(s->d_J);
    hipFree(s->d_K);
    hipFree(s->d_hash);
    hipFree(s->d_status);
    delete s;
    return NNQS_OK;
}

int64_t nnqs_connection_count(const nnqs_system *s) { return s ? s->view.C : -1; }

nnqs_status nnqs_table_create(nnqs_table **out, const nnqs_system *sys, int64_t capacity) {
    clear_error();
    if (!out || !sys) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    if (capacity <= 0 || capacity > (int64_t(1) << 31))
        return fail(NNQS_EINVAL, "capacity %lld outside [1, 2^31]", (long long)capacity);
    nnqs_table *t = new nnqs_table();
    t->sys = sys;
    t->capacity = capacity;
    int64_t P = 2;
    while (P < capacity) P <<= 1;
    t->padded = P;
    auto cleanup = [&](nnqs_status st) {
        nnqs_table_destroy(t);
        return st;
    };
    if (hipMalloc(&t->keys, capacity * 16) != hipSuccess || hipMalloc(&t->logabs, capacity * 8) != hipSuccess ||
        hipMalloc(&t->phase, capacity * 8) != hipSuccess || hipMalloc(&t->sort_keys, P * 16) != hipSuccess ||
        hipMalloc(&t->sort_idx, P * 4) != hipSuccess ||
        hipMalloc(&t->filter, (size_t(1) << kMaxFilterLog2) / 8) != hipSuccess ||
        hipMalloc(&t->split, ((size_t(1) << kMaxSplitLevels) - 1) * 16) != hipSuccess ||
        hipMalloc(&t->status, sizeof(int)) != hipSuccess ||
        hipMalloc(&t->partials, kPartialBlocks * 8 * sizeof(double)) != hipSuccess ||
        hipMalloc(&t->amp, capacity * 16) != hipSuccess ||
        hipMalloc(&t->lmax, (kPartialBlocks + 1) * sizeof(double)) != hipSuccess)
        return cleanup(fail(NNQS_ENOMEM, "device allocation of a table of %lld failed", (long long)capacity));
    if (hipMemset(t->status, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return cleanup(fail(NNQS_EHIP, "table initialisation failed"));
    nnqs_table_set_tune(t, nullptr);
    *out = t;
    return NNQS_OK;
}

nnqs_status nnqs_table_destroy(nnqs_table *t) {
    if (!t) return NNQS_OK;
    hipFree(t->keys);
    hipFree(t->logabs);
    hipFree(t->phase);
    hipFree(t->sort_keys);
    hipFree(t->sort_idx);
    hipFree(t->filter);
    hipFree(t->split);
    hipFree(t->status);
    hipFree(t->partials);
    hipFree(t->amp);
    hipFree(t->lmax);
    delete t;
    return NNQS_OK;
}

nnqs_status nnqs_table_set_tune(nnqs_table *t, const nnqs_tune *tune) {
    clear_error();
    if (!t) return fail(NNQS_EINVAL, "null table");
    nnqs_tune d{};
    d.waves_per_block = 12;
    d.blocks_per_cu = 1;
    d.filter_log2_bits = 20;
    d.splitter_levels = 10;
    d.search = 1;
    d.tile_samples = 256;
    if (tune) {
        if (tune->waves_per_block) d.waves_per_block = tune->waves_per_block;
        if (tune->blocks_per_cu) d.blocks_per_cu = tune->blocks_per_cu;
        if (tune->filter_log2_bits) d.filter_log2_bits = tune->filter_log2_bits;
        if (tune->splitter_levels) d.splitter_levels = tune->splitter_levels;
        if (tune->search) d.search = tune->search;
        if (tune->tile_samples) d.tile_samples = tune->tile_samples;
    }
    if (!tune_valid(d)) return fail(NNQS_EINVAL, "tuning parameters out of range");
    t->tune = d;
    return NNQS_OK;
}

nnqs_status nnqs_table_get_tune(const nnqs_table *t, nnqs_tune *tune) {
    if (!t || !tune) return fail(NNQS_EINVAL, "null pointer argument");
    *tune = t->tune;
    return NNQS_OK;
}

}  // extern "C"

namespace nnqs {

// Ascending bitonic sort of P (a power of two >= 2) entries: 128-bit keys
// sk[2 i], sk[2 i + 1] (word 1 major) with 32-bit payloads si[i] as the
// final tie-break, in place on `st`.
void bitonic_sort128(uint64_t *sk, uint32_t *si, int64_t P, hipStream_t st) {
    const int tile = P < 2048 ? (int)P : 2048;
    const int thr = 256;
    const size_t lds = (size_t)tile * 20;
    const int lthreads = tile / 2 < 1024 ? tile / 2 : 1024;
    hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(P / tile)), dim3(lthreads), lds, st, sk, si, tile,
                       (int64_t)2, (int64_t)tile, (int64_t)1);
    for (int64_t k = (int64_t)tile * 2; k <= P; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= 2 * (int64_t)tile; j >>= 2)  // stages j and j/2 together
            hipLaunchKernelGGL(k_bitonic_global2, dim3((unsigned)((P / 4 + thr - 1) / thr)), dim3(thr), 0, st, sk,
                               si, P, k, j);
        if (j >= tile)
            hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((P / 2 + thr - 1) / thr)), dim3(thr), 0, st, sk,
                               si, P, k, j);
        hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(P / tile)), dim3(lthreads), lds, st, sk, si, tile, k, k,
                           (int64_t)(tile / 2));
    }
}

}  // namespace nnqs

extern "C" {

nnqs_status nnqs_table_build(nnqs_table *t, const uint64_t *keys, const double *logabs, const double *phase,
                             int64_t n, uint32_t flags, void *stream) {
    clear_error();
    if (!t || !keys || !logabs || !phase) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n=%lld must be positive", (long long)n);
    if (n > t->capacity)
        return fail(NNQS_ERANGE, "n=%lld exceeds the table capacity %lld", (long long)n, (long long)t->capacity);
    hipStream_t st = as_stream(stream);
    int64_t P = 2;
    while (P < n) P <<= 1;
    const int thr = 256;
    hipLaunchKernelGGL(k_sort_init, dim3((unsigned)((P + thr - 1) / thr)), dim3(thr), 0, st, keys, n, P, t->sort_keys,
                       t->sort_idx);
    bitonic_sort128(t->sort_keys, t->sort_idx, P, st);
    const int fl = t->tune.filter_log2_bits;
    const int64_t fwords = int64_t(1) << (fl - 5);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((fwords + thr - 1) / thr)), dim3(thr), 0, st, t->filter, fwords,
                       0u);
    hipLaunchKernelGGL(k_table_finalize, dim3((unsigned)((n + thr - 1) / thr)), dim3(thr), 0, st, t->sys->view,
                       t->sort_keys, t->sort_idx, logabs, phase, n, t->keys, t->logabs, t->phase, t->filter, fl,
                       t->status);
    {
        int mb = (int)((n + thr - 1) / thr);
        if (mb > kPartialBlocks) mb = kPartialBlocks;
        hipLaunchKernelGGL(k_table_max_partial, dim3((unsigned)mb), dim3(thr), 0, st, t->logabs, n, t->lmax);
        hipLaunchKernelGGL(k_table_max_final, dim3(1), dim3(thr), 0, st, t->lmax, mb);
        hipLaunchKernelGGL(k_table_amp, dim3((unsigned)((n + thr - 1) / thr)), dim3(thr), 0, st, t->logabs,
                           t->phase, n, t->lmax, t->amp);
    }
    int L = 0;
    while ((int64_t(1) << L) < n) L++;
    int sl = t->tune.splitter_levels < L ? t->tune.splitter_levels : L;
    if (sl > 0) {
        int64_t cnt = (int64_t(1) << sl) - 1;
        hipLaunchKernelGGL(k_table_split, dim3((unsigned)((cnt + thr - 1) / thr)), dim3(thr), 0, st, t->keys, n, L, sl,
                           t->split);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    t->n = n;
    t->filter_log2 = fl;
    t->split_levels = sl;
    if (flags & NNQS_VALIDATE) {
        nnqs_status s = read_status(t, st, true);
        if (s != NNQS_OK) {
            t->n = 0;
            return fail(s, "table validation failed (%s)",
                        s == NNQS_EDUP ? "duplicate key" : s == NNQS_ECONSERVE ? "wrong particle number"
                                                                               : "non-finite amplitude");
        }
    }
    return NNQS_OK;
}

nnqs_status nnqs_table_export(const nnqs_table *t, uint64_t *keys_out, double *logabs_out, double *phase_out,
                              int64_t *n_out, void *stream) {
    clear_error();
    if (!t || !n_out) return fail(NNQS_EINVAL, "null pointer argument");
    hipStream_t st = as_stream(stream);
    if (keys_out)
        NNQS_HIP_CHECK(hipMemcpyAsync(keys_out, t->keys, t->n * 16, hipMemcpyDeviceToDevice, st));
    if (logabs_out)
        NNQS_HIP_CHECK(hipMemcpyAsync(logabs_out, t->logabs, t->n * 8, hipMemcpyDeviceToDevice, st));
    if (phase_out)
        NNQS_HIP_CHECK(hipMemcpyAsync(phase_out, t->phase, t->n * 8, hipMemcpyDeviceToDevice, st));
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    *n_out = t->n;
    return NNQS_OK;
}

nnqs_status nnqs_table_status(nnqs_table *t, void *stream) {
    clear_error();
    if (!t) return fail(NNQS_EINVAL, "null table");
    return read_status(t, as_stream(stream), true);
}

nnqs_status nnqs_energy(nnqs_table *t, const uint32_t *counts, const double *eloc, int64_t n, double *energy,
                        void *stream) {
    clear_error();
    if (!t || !counts || !eloc || !energy) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    return enqueue_energy(t, counts, eloc, n, energy, as_stream(stream));
}


nnqs_status nnqs_energy_noalloc(const uint32_t *counts, const double *eloc, int64_t n, double *energy, void *stream) {
    clear_error();
    if (!counts || !eloc || !energy) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if (n > NNQS_ENERGY_NOALLOC_MAX_N)
        return fail(NNQS_ERANGE, "n=%lld exceeds the no-allocation limit of %lld samples", (long long)n,
                    (long long)NNQS_ENERGY_NOALLOC_MAX_N);
    double *sc = nullptr;
    const nnqs_status s = noalloc_scratch(&sc);
    if (s != NNQS_OK) return s;
    return enqueue_energy_partials(sc, counts, eloc, n, energy, as_stream(stream));
}


nnqs_status nnqs_timing_enable(int32_t enable) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_timing_mu);
    timing_clear_locked();
    g_timing.store(enable != 0);
    return NNQS_OK;
}

nnqs_status nnqs_timing_read(const char *kernel, double *total_ms, int64_t *launches) {
    clear_error();
    if (!kernel || !total_ms) return fail(NNQS_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(g_timing_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &r : g_timing_recs) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        NNQS_HIP_CHECK(hipEventSynchronize(r.b));
        float ms = 0.f;
        NNQS_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
        cnt++;
    }
    *total_ms = tot;
    if (launches) *launches = cnt;
    return NNQS_OK;
}

}  // extern "C"

// Internal definitions shared by the translation units of libnnqs_eloc.
// Device helpers for 128-bit occupation keys, Jordan-Wigner signs and
// Slater-Condon matrix elements of the Hamiltonian of Eq. 9.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "nnqs_eloc.h"

namespace nnqs {

// ------------------------------------------------------------------ errors
nnqs_status fail(nnqs_status code, const char *fmt, ...);
void clear_error();

#define NNQS_HIP_CHECK(call)                                                              \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::nnqs::fail(NNQS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Measurement of the library's own launches (nnqs_timing_enable/_read):
// while timing is on, a TimedRegion records HIP events on `st` around the
// launches enqueued during its lifetime, under the kernel name given.
class TimedRegion {
  public:
    TimedRegion(const char *name, hipStream_t st);
    ~TimedRegion();
    TimedRegion(const TimedRegion &) = delete;
    TimedRegion &operator=(const TimedRegion &) = delete;

  private:
    const char *name_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ------------------------------------------------------ device-side views
// Everything a kernel needs about the Hamiltonian, passed by value.
struct SysView {
    int K, N, n_up, n_dn;
    int64_t C;               // connections per sample, diagonal included
    const double *h;         // [K*K]
    const double *g;         // [K^4] chemists' (ij|kl)
    const double *Jm;        // [K*K] (ii|jj)
    const double *Km;        // [K*K] (ij|ji)
    const uint64_t *hashT;   // [128] per-spin-orbital hash words (GF(2)-linear hash)
    double ecore;
    uint64_t valid0, valid1; // masks of the N valid key bits
};

// Sorted sample table as seen by kernels.
struct TableView {
    const uint64_t *keys;    // [n][2] sorted ascending (word 1 major)
    const double *logabs;    // [n]
    const double *phase;     // [n]
    const uint32_t *filter;  // membership filter, 2^filter_log2 bits
    const uint64_t *split;   // [2^split_levels - 1][2] staged search keys
    const double *amp;       // [n][2] exp(logabs - lmax) (cos phase, sin phase)
    const double *lmax;      // [1] max logabs of the table
    int64_t n;
    int log2n;               // ceil(log2(n)), 0 for n == 1
    int filter_log2;         // bits of the filter = 2^filter_log2
    int split_levels;        // levels of the search tree staged in LDS
};

constexpr uint64_t EVEN_BITS = 0x5555555555555555ull;
constexpr uint64_t ODD_BITS = 0xAAAAAAAAAAAAAAAAull;

// Sticky device status: first error wins.
__device__ inline void set_status(int *status, int code) {
    if (status) atomicCAS(status, 0, code);
}

// ---------------------------------------------------------- 128-bit keys
struct Key {
    uint64_t lo, hi;
};

__device__ __forceinline__ bool key_less(const Key &a, const Key &b) {
    return (a.hi < b.hi) || (a.hi == b.hi && a.lo < b.lo);
}
__device__ __forceinline__ bool key_eq(const Key &a, const Key &b) { return a.lo == b.lo && a.hi == b.hi; }

__device__ __forceinline__ void key_flip(Key &k, int p) {
    uint64_t m = 1ull << (p & 63);
    if (p < 64) k.lo ^= m;
    else k.hi ^= m;
}

__device__ __forceinline__ int key_bit(const Key &k, int p) {
    return (int)(((p < 64 ? k.lo : k.hi) >> (p & 63)) & 1ull);
}

// popcount of the bits of k strictly below position p (0 <= p <= 128)
__device__ __forceinline__ int popc_below(const Key &k, int p) {
    if (p <= 0) return 0;
    if (p < 64) return __popcll(k.lo & ((1ull << p) - 1ull));
    if (p == 64) return __popcll(k.lo);
    int q = p - 64;
    uint64_t mh = (q >= 64) ? ~0ull : ((1ull << q) - 1ull);
    return __popcll(k.lo) + __popcll(k.hi & mh);
}

// -------------------------------------------------- Hamiltonian elements
__device__ __forceinline__ double g_at(const SysView &S, int i, int j, int k, int l) {
    const int K = S.K;
    return S.g[(((size_t)i * K + j) * K + k) * K + l];
}

// <pq|rs> over spin orbitals = (i_p i_r | i_q i_s) if spins of (p,r), (q,s) agree
__device__ __forceinline__ double phys_el(const SysView &S, int p, int q, int r, int s) {
    if (((p ^ r) & 1) | ((q ^ s) & 1)) return 0.0;
    return g_at(S, p >> 1, r >> 1, q >> 1, s >> 1);
}

// Diagonal element <x|H|x>, evaluated by one lane (loops over occupied orbitals).
__device__ inline double diag_element(const SysView &S, const Key &x) {
    double e = S.ecore;
    const int K = S.K;
    for (int p = 0; p < S.N; p++) {
        if (!key_bit(x, p)) continue;
        const int ip = p >> 1;
        double acc = S.h[ip * K + ip];
        for (int q = 0; q < S.N; q++) {
            if (!key_bit(x, q)) continue;
            const int iq = q >> 1;
            double v = S.Jm[ip * K + iq];
            if (((p ^ q) & 1) == 0) v -= S.Km[ip * K + iq];
            acc += 0.5 * v;
        }
        e += acc;
    }
    return e;
}

// Sign parity of a+_p a_q acting on x (q occupied, p empty, p != q): the
// number of occupied orbitals strictly between them.
__device__ __forceinline__ int single_parity(const Key &x, int q, int p) {
    int lo = q < p ? q : p, hi = q < p ? p : q;
    return (popc_below(x, hi) - popc_below(x, lo + 1)) & 1;
}

// Sign parity of a+_a a+_b a_j a_i acting on x, with i<j occupied and a<b empty.
__device__ __forceinline__ int double_parity(const Key &x, int i, int j, int a, int b) {
    Key y = x;
    int par = popc_below(y, i);
    key_flip(y, i);
    par += popc_below(y, j);
    key_flip(y, j);
    par += popc_below(y, b);
    key_flip(y, b);
    par += popc_below(y, a);
    return par & 1;
}

// Single-excitation element (without the sign): h_pq + sum_{k in x}
// [(pq|kk) - delta(s_k, s_p) (pk|kq)], spatial indices of p, q.
__device__ inline double single_element(const SysView &S, const Key &x, int q, int p) {
    const int K = S.K;
    const int ip = p >> 1, iq = q >> 1, sp = p & 1;
    double v = S.h[ip * K + iq];
    for (int w = 0; w < 2; w++) {
        uint64_t m = w ? x.hi : x.lo;
        while (m) {
            int b = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            int k = w * 64 + b;
            int ik = k >> 1;
            double t = g_at(S, ip, iq, ik, ik);
            if ((k & 1) == sp) t -= g_at(S, ip, ik, ik, iq);
            v += t;
        }
    }
    return v;
}

// Full element <x'|H|x> for an excitation given by raw indices: i == 255 is
// the diagonal (value `diag`), j == 255 a single q=i -> p=a, otherwise a
// double removing {i, j} and adding {a, b} (any order).  *sign_out gets +-1.
__device__ inline double excitation_element(const SysView &S, const Key &x, double diag, int i, int j, int a,
                                            int b, int *sign_out) {
    if (i == 255) {
        *sign_out = 1;
        return diag;
    }
    if (j == 255) {
        int s = single_parity(x, i, a) ? -1 : 1;
        *sign_out = s;
        return s * single_element(S, x, i, a);
    }
    int i0 = i < j ? i : j, j0 = i < j ? j : i;
    int a0 = a < b ? a : b, b0 = a < b ? b : a;
    int s = double_parity(x, i0, j0, a0, b0) ? -1 : 1;
    *sign_out = s;
    return s * (phys_el(S, a0, b0, i0, j0) - phys_el(S, a0, b0, j0, i0));
}

// erf in FP32 for the BF16 forwards: Abramowitz & Stegun 7.1.26 (Hastings'
// rational approximation), |error| <= 1.5e-7, far below the BF16 rounding of
// the results it feeds; one reciprocal, one exponential, no branches.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float y = fmaf(1.061405429f, t, -1.453152027f);
    y = fmaf(y, t, 1.421413741f);
    y = fmaf(y, t, -0.284496736f);
    y = fmaf(y, t, 0.254829592f);
    y = 1.0f - y * t * __expf(-ax * ax);
    return copysignf(y, x);
}

// GELU with the erf above (BF16 forwards and the screen's inference).
__device__ __forceinline__ float gelu_bf16path(float v) { return 0.5f * v * (1.0f + erf_as(v * 0.70710678118654752f)); }

// -------------------------------------------------- compensated summation
struct NSum {  // Neumaier
    double s, c;
    __device__ __forceinline__ void add(double v) {
        double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
};

// Combine two compensated partial sums exactly up to the final rounding
// (Knuth's TwoSum on the leading parts).
__device__ __forceinline__ void nsum_merge(double &s, double &c, double s2, double c2) {
    double t = s + s2;
    double bp = t - s;
    double ap = t - bp;
    double err = (s - ap) + (s2 - bp);
    s = t;
    c = (c + c2) + err;
}

// Wave-wide sum of compensated pairs (butterfly, fixed order: every lane
// ends with the same bits).
__device__ __forceinline__ void wave_nsum(double &s, double &c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double s2 = __shfl_xor(s, off, 64);
        double c2 = __shfl_xor(c, off, 64);
        nsum_merge(s, c, s2, c2);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------- host-side objects
}  // namespace nnqs

struct nnqs_system {
    nnqs::SysView view;
    double *d_h = nullptr, *d_g = nullptr, *d_J = nullptr, *d_K = nullptr;
    uint64_t *d_hash = nullptr;
    int *d_status = nullptr;  // scratch status word for validation of connection exports
    int device = 0;
    int cu_count = 0;
    int max_lds = 0;  // bytes of LDS a block may use
};

struct nnqs_table {
    const nnqs_system *sys = nullptr;
    int64_t capacity = 0;
    int64_t n = 0;
    int64_t padded = 0;            // power of two >= capacity (sort buffers)
    uint64_t *keys = nullptr;      // [capacity][2] sorted
    double *logabs = nullptr, *phase = nullptr;
    uint64_t *sort_keys = nullptr; // [padded][2]
    uint32_t *sort_idx = nullptr;  // [padded]
    uint32_t *filter = nullptr;    // 2^20 bits maximum
    uint64_t *split = nullptr;     // [2^13 - 1][2] maximum
    int *status = nullptr;         // sticky device status
    double *partials = nullptr;    // energy reduction scratch
    double *amp = nullptr;         // [capacity][2] scaled complex amplitudes
    double *lmax = nullptr;        // [kPartialBlocks + 1]: block maxima, then the max at [0]
    int filter_log2 = 0;           // as built
    int split_levels = 0;          // as built
    nnqs_tune tune{};
};

namespace nnqs {
nnqs::TableView table_view(const nnqs_table *t);
// Enqueue the two-stage deterministic energy reduction.
nnqs_status enqueue_energy(nnqs_table *tab, const uint32_t *counts, const double *eloc, int64_t n,
                           double *energy, hipStream_t st);
nnqs_status enqueue_energy_partials(double *partials, const uint32_t *counts, const double *eloc, int64_t n,
                                    double *energy, hipStream_t st);
// Synchronise and read/clear the sticky status.
nnqs_status read_status(nnqs_table *tab, hipStream_t st, bool clear);
constexpr int kMaxFilterLog2 = 20;

inline bool tune_valid(const nnqs_tune &d) {
    return d.waves_per_block >= 1 && d.waves_per_block <= 16 && d.blocks_per_cu >= 1 && d.blocks_per_cu <= 64 &&
           d.filter_log2_bits >= 10 && d.filter_log2_bits <= kMaxFilterLog2 && d.splitter_levels >= 1 &&
           d.splitter_levels <= 13 && (d.search == 1 || d.search == 2) && d.tile_samples >= 1 &&
           d.tile_samples <= 65536;
}

// One system of a batched sample-aware launch (device array).
struct SaBatchItem {
    SysView S;
    TableView T;
    int lds_filter_log2;
    const uint64_t *keys;
    const double *logabs, *phase;
    double *eloc;
    int *status;
};

// A run of samples of one system (device array, in system order).
struct SaTile {
    int32_t item, count;
    int64_t begin;
};

// Sample-aware kernel plumbing shared by the single-system and batched
// entry points (eloc_sa.hip).
size_t sa_lds_bytes(int filter_log2, int split_levels, int W, int waves);
const void *sa_kernel_ptr(int W, int search, int waves);
const void *sa_batch_kernel_ptr(int W, int search, bool exact);
nnqs_status sa_check_no_spill(const void *fn);
void sa_launch_batch(int W, int search, unsigned grid, int waves, size_t lds, hipStream_t st,
                     const SaBatchItem *items, const SaTile *tiles, int ntiles, int *counter);
void sa_launch_reset(int *counter, hipStream_t st);
TableView table_view_planned(const nnqs_table *t, int64_t n);

// Membership-filter geometry, read from the low 32 bits of the linear key
// hash: bits 0-4 and 5-9 give bit positions p1 and p2 of a 32-bit filter
// word, and a third position is p1 + p2 mod 32 (double hashing: three bits
// per member for one more add, which cuts the false-positive rate of the
// blocked filter by about a third); bits 10..(filter_log2 + 4) select the
// word.  Bits 25-31 are never read, which lets the enumeration kernel pack
// an orbital index into them.
constexpr int kFilterWordShift = 10;
constexpr uint32_t kFilterHashMask = 0x01FFFFFFu;
static_assert(kMaxFilterLog2 - 5 + kFilterWordShift <= 25, "filter word index must stay below bit 25");

__device__ __forceinline__ uint32_t filter_word(uint32_t h, uint32_t wmask) { return (h >> kFilterWordShift) & wmask; }
__device__ __forceinline__ uint32_t filter_bits(uint32_t h) {
    return (1u << (h & 31u)) | (1u << ((h >> 5) & 31u)) | (1u << ((h + (h >> 5)) & 31u));
}
// Nonzero when all three bits of h are set in filter word w (the bit
// extracts read the low five bits of their offset operand).
__device__ __forceinline__ uint32_t filter_test(uint32_t w, uint32_t h) {
    const uint32_t h5 = h >> 5;
    return __builtin_amdgcn_ubfe(w, h, 1u) & __builtin_amdgcn_ubfe(w, h5, 1u) & __builtin_amdgcn_ubfe(w, h + h5, 1u);
}
constexpr int kMaxSplitLevels = 13;
constexpr int kPartialBlocks = 1024;
}  // namespace nnqs

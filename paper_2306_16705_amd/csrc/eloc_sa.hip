// Sample-aware local energy (paper: Section 3.4 items 2-5 and Algorithm 2,
// re-designed for CDNA4) and the canonical connection export.
//
// One 64-lane wavefront owns one sample x at a time (persistent grid-stride
// loop).  The wave enumerates every single and double excitation of x that
// conserves the up and down electron numbers.  Instead of building each key
// x' and binary-searching it, the hot loop carries only a GF(2)-linear hash
// of x' (hash(x ^ m) = hash(x) ^ hash(m)), probes an LDS-resident blocked
// membership filter of the table, and pushes the few survivors into a
// per-wave LDS queue.  Full batches of 64 queued candidates are resolved by
// a binary search whose top levels come from LDS and the rest from the
// L2-resident sorted table; hits get the Slater-Condon element, the FP64
// log-polar amplitude ratio and a per-lane Neumaier sum (Eq. 4 fused with
// the accumulation as in Section 3.4 item 2).  The filter has no false
// negatives, so every table member connected to x is found.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "enumerate.hpp"

namespace nnqs {

// Block sizes of the sample-aware kernels: builds for up to 12 waves (three
// per SIMD, up to 168 VGPRs: the exact pass and the batched kernels, which
// need more than 128) and builds for up to 16 waves (four per SIMD, at most
// 128 VGPRs: the single-system scaled pass, both search variants).
constexpr int kSaMaxThreads = 768;
constexpr int kSaWideThreads = 1024;

// Dynamic LDS layout of the sample-aware kernel: the filter words, the staged
// search keys, the low 32 bits of the 128 hash words, then one WaveLds per
// wave (16-byte aligned).
struct SaLayout {
    size_t split, hash, waves, total;
};

__host__ __device__ inline SaLayout sa_layout(int filter_log2, int split_levels, int W, int waves) {
    SaLayout L;
    L.split = ((size_t)1 << (filter_log2 - 5)) * 4;
    L.hash = L.split + (((size_t)1 << split_levels) - 1) * 8 * W;
    L.waves = (L.hash + 128 * 4 + 15) & ~(size_t)15;
    L.total = L.waves + sizeof(WaveLds) * waves;
    return L;
}

// Probe of the blocked filter (geometry and bit test in internal.hpp).  The
// filter is the first object of the kernel's dynamic LDS, and the kernels
// that probe it declare no static LDS, so it starts at LDS address 0 and a
// word's byte offset is its LDS address (sa_stage checks this): the probe
// needs no base add.
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
__device__ __forceinline__ uint32_t filter_load(uint32_t wmask, uint32_t h) {
    // byte offset of word filter_word(h, wmask)
    const uint32_t off = (h >> (kFilterWordShift - 2)) & (wmask << 2);
    return *reinterpret_cast<lds_u32 *>((size_t)off);
}
__device__ __forceinline__ uint32_t filter_probe(uint32_t wmask, uint32_t h) {
    return filter_test(filter_load(wmask, h), h);
}

template <int W>
__device__ __forceinline__ Key load_key(const uint64_t *k, uint32_t i) {
    Key r;
    r.lo = k[2 * (size_t)i];
    r.hi = (W == 2) ? k[2 * (size_t)i + 1] : 0ull;
    return r;
}

// Lower-bound search for t in the sorted table (positions fit 32 bits: a
// table holds at most 2^31 keys); both variants start with the first
// split_levels levels from LDS copies of the keys they probe (every key at
// position (m+1)*2^(L-s) - 1).
template <int W>
__device__ __forceinline__ uint32_t search_lds_levels(const TableView &T, const uint64_t *s_lds, const Key &t) {
    const int L = T.log2n, s = T.split_levels;
    uint32_t lo = 0;
    for (int lvl = 0; lvl < s; lvl++) {
        const uint32_t step = 1u << (L - 1 - lvl);
        const uint32_t j = ((lo + step) >> (L - s)) - 1u;
        Key k;
        k.lo = s_lds[j * W];
        k.hi = (W == 2) ? s_lds[j * W + 1] : 0ull;
        if (key_less(k, t)) lo += step;
    }
    return lo;
}

// Variant 1: the remaining levels one dependent load at a time, then the
// key the search ends on.
template <int W>
__device__ __forceinline__ int64_t table_find_binary(const TableView &T, const uint64_t *s_lds, const Key &t) {
    const int L = T.log2n;
    const uint32_t n = (uint32_t)T.n;
    uint32_t lo = search_lds_levels<W>(T, s_lds, t);
    for (int lvl = T.split_levels; lvl < L; lvl++) {
        const uint32_t step = 1u << (L - 1 - lvl);
        const uint32_t idx = lo + step - 1u;
        if (idx < n && key_less(load_key<W>(T.keys, idx), t)) lo += step;
    }
    if (lo < n && key_eq(load_key<W>(T.keys, lo), t)) return lo;
    return -1;
}

// Variant 2: the remaining levels up to three at a time by 8-way rounds
// whose probes are independent loads.  The last round loads the keys from
// the current lower bound on and counts them as they arrive: the lower
// bound moves past every key below t, and t is present exactly when one of
// the keys of the final range equals it (keys are distinct), so no key has
// to be kept for a separate equality test.
template <int W>
__device__ __forceinline__ int64_t table_find_8way(const TableView &T, const uint64_t *s_lds, const Key &t) {
    uint32_t lo = search_lds_levels<W>(T, s_lds, t);
    const uint32_t n = (uint32_t)T.n, last = n - 1u;
    int r = T.log2n - T.split_levels;
    if (r == 0) return (lo < n && key_eq(load_key<W>(T.keys, lo), t)) ? (int64_t)lo : -1;
    int q = r % 3 == 0 ? 3 : r % 3;  // levels taken by the first round
    while (r > q) {
        const uint32_t st = 1u << (r - q);
        uint32_t c = 0;
        for (int k = 1; k < (1 << q); k++) {
            const uint32_t idx = lo + k * st - 1u;
            const Key kk = load_key<W>(T.keys, idx < last ? idx : last);
            c += (idx < n && key_less(kk, t)) ? 1u : 0u;
        }
        lo += c * st;
        r -= q;
        q = 3;
    }
    const int probes = (1 << q) - 1;  // the final range is lo .. lo + probes
    uint32_t c = 0;
    bool eq = false;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t p = lo + k;
        const Key kk = load_key<W>(T.keys, p < last ? p : last);
        const bool in = k <= probes && p < n;
        c += (in && k < probes && key_less(kk, t)) ? 1u : 0u;
        eq = eq || (in && key_eq(kk, t));
    }
    return eq ? (int64_t)(lo + c) : -1;
}

__device__ __forceinline__ uint32_t wave_xor32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off, 64);
    return v;
}

// LDS-resident per-system data of the sample-aware kernels.
struct SaStage {
    const uint32_t *f_lds;  // membership filter words
    const uint64_t *s_lds;  // staged search keys
    const uint32_t *h_lds;  // low 32 bits of the hash words
    WaveLds *waves;         // one per wave
    uint32_t wmask;         // filter words - 1
    bool at_zero;           // the filter starts at LDS address 0
};

// Stage the filter (folded to the LDS size: OR of aliasing words keeps every
// member), the top search levels and the hash words.  Block-wide; ends with a
// barrier.
template <int W>
__device__ __forceinline__ SaStage sa_stage(const SysView &S, const TableView &T, int lds_filter_log2,
                                            uint8_t *smem) {
    const int nwords = 1 << (lds_filter_log2 - 5);
    const int big_words = 1 << (T.filter_log2 - 5);
    const int nsplit = (1 << T.split_levels) - 1;
    const SaLayout lay = sa_layout(lds_filter_log2, T.split_levels, W, blockDim.x >> 6);
    uint32_t *f_lds = reinterpret_cast<uint32_t *>(smem);
    uint64_t *s_lds = reinterpret_cast<uint64_t *>(smem + lay.split);
    uint32_t *h_lds = reinterpret_cast<uint32_t *>(smem + lay.hash);
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) {
        uint32_t v = 0;
        for (int k = i; k < big_words; k += nwords) v |= T.filter[k];
        f_lds[i] = v;
    }
    for (int i = threadIdx.x; i < nsplit; i += blockDim.x) {
        s_lds[(size_t)i * W] = T.split[2 * i];
        if (W == 2) s_lds[(size_t)i * W + 1] = T.split[2 * i + 1];
    }
    for (int i = threadIdx.x; i < 128; i += blockDim.x) h_lds[i] = (uint32_t)S.hashT[i];
    __syncthreads();
    SaStage G;
    G.f_lds = f_lds;
    G.s_lds = s_lds;
    G.h_lds = h_lds;
    G.waves = reinterpret_cast<WaveLds *>(smem + lay.waves);
    G.wmask = (uint32_t)nwords - 1u;
    G.at_zero = (uint32_t)(size_t)(lds_u32 *)f_lds == 0u;  // address-space cast to an LDS address
    return G;
}

// E_loc of sample smp by the calling wave (see the file comment).  S8 picks
// the search variant of the queued candidates.  Hits take the amplitude
// ratio from the table's scaled amplitudes (EX = 0), except for samples more
// than 600 nats below the table's largest amplitude (or with a non-finite
// one), which a second pass (EX = 1) evaluates with exp and sincos per hit;
// each pass leaves the other pass's samples alone.
template <int W, int S8, int EX>
__device__ __forceinline__ void sa_sample(const SysView &S, const TableView &T, const SaStage &G, WaveLds &wl,
                                          int64_t smp, const uint64_t *__restrict__ keys,
                                          const double *__restrict__ logabs, const double *__restrict__ phase,
                                          double *__restrict__ eloc, int *status) {
    const int lane = lane_id();
    const int K = S.K, nu = S.n_up, nd = S.n_dn, vu = K - nu, vd = K - nd;
    const uint32_t *f_lds = G.f_lds, *h_lds = G.h_lds;
    const uint32_t wmask = G.wmask;
    Key x;
    x.lo = keys[2 * smp];
    x.hi = keys[2 * smp + 1];
    const double la = logabs[smp], ph = phase[smp];
    const double lmax = T.lmax[0];
    if ((la - lmax >= -600.0) == (EX == 1)) return;  // the other pass's sample
    if (!sample_conserves(S, x) || !isfinite(la) || !isfinite(ph)) {
        if (lane == 0) {
            eloc[2 * smp] = NAN;
            eloc[2 * smp + 1] = NAN;
            set_status(status, sample_conserves(S, x) ? NNQS_ERANGE : NNQS_ECONSERVE);
        }
        return;
    }
    build_lists(S, x, wl);
    uint32_t part = 0;
    if (lane < K) {
        if (key_bit(x, 2 * lane)) part ^= h_lds[2 * lane];
        if (key_bit(x, 2 * lane + 1)) part ^= h_lds[2 * lane + 1];
    }
    const uint32_t hx = wave_xor32(part);
    const double diag = wave_diag(S, x, wl);
    // Hit ratios of the scaled pass: psi(x')/psi(x) = amp[x'] exp(lmax -
    // log|psi(x)|) e^{-i phase(x)} (amp cannot underflow for a term that
    // counts, as the sample is within 600 nats of lmax).  The per-sample
    // constants sit in LDS: they are read on hits only.
    if (lane == 0) {
        if (EX == 0) {
            double xsn, xcs;
            sincos(ph, &xsn, &xcs);
            wl.hit[0] = exp(lmax - la);
            wl.hit[1] = xcs;
            wl.hit[2] = xsn;
        } else {
            wl.hit[3] = la;
            wl.hit[4] = ph;
        }
    }
    wave_sync();
    // Lane l holds entry l of the occupied-up, occupied-down and empty-up
    // lists as (low hash bits | orbital << 25); the loops read them with
    // wave-uniform readlane, which yields the orbital with a scalar shift.
    auto pack = [&](int p) -> uint32_t { return (h_lds[p] & kFilterHashMask) | ((uint32_t)p << 25); };
    const uint32_t po_u = lane < nu ? pack(wl.occ[0][lane]) : 0u;
    const uint32_t po_d = lane < nd ? pack(wl.occ[1][lane]) : 0u;
    const uint32_t pv_u = lane < vu ? pack(wl.vir[0][lane]) : 0u;

    NSum are{0.0, 0.0}, aim{0.0, 0.0};
    int qh = 0, qt = 0;  // wave-uniform ring counters (ring of 256)

    // Resolve one queued candidate: lookup, then on a hit the Slater-Condon
    // element and the log-polar amplitude ratio into the lane's compensated
    // sums.
    auto process = [&](uint32_t e) {
        const int i = e & 255, j = (e >> 8) & 255, a = (e >> 16) & 255, b = e >> 24;
        Key xp = x;
        if (i != 255) {
            key_flip(xp, i);
            key_flip(xp, a);
            if (j != 255) {
                key_flip(xp, j);
                key_flip(xp, b);
            }
        }
        // The matrix element needs only x and the excitation, so its integral
        // loads are issued before the search and overlap it.
        int sg;
        const double hv = excitation_element(S, x, diag, i, j, a, b, &sg);
        const int64_t idx = S8 ? table_find_8way<W>(T, G.s_lds, xp) : table_find_binary<W>(T, G.s_lds, xp);
        if (EX == 0) {
            // branch-free: a miss reads entry 0 and adds an exact zero, which
            // leaves the lane's compensated sums unchanged (the scaled
            // amplitudes are finite)
            const bool hit = idx >= 0;
            const uint32_t k = hit ? (uint32_t)idx : 0u;
            const double ar = T.amp[2 * (size_t)k], ai = T.amp[2 * (size_t)k + 1];
            const double xs = wl.hit[0], xcs = wl.hit[1], xsn = wl.hit[2];
            const double w = hit ? hv : 0.0;
            are.add(w * (xs * (ar * xcs + ai * xsn)));
            aim.add(w * (xs * (ai * xcs - ar * xsn)));
        } else if (idx >= 0) {
            const double r = exp(T.logabs[idx] - wl.hit[3]);
            double sn, cs;
            sincos(T.phase[idx] - wl.hit[4], &sn, &cs);
            are.add(hv * (r * cs));
            aim.add(hv * (r * sn));
        }
    };
    auto drain_full = [&]() {
        while (qt - qh >= 64) {
            wave_sync();
            process(wl.queue[(qh + lane) & 255]);
            qh += 64;
            wave_sync();
        }
    };
    // Append the candidates of ballot mask m (uniform) in lane order: the
    // mask itself selects the writing lanes (inverse ballot, no per-lane
    // test) and the ring position is qt plus the count of set lanes below.
    auto push = [&](uint64_t m, uint32_t code) {
        if (__builtin_amdgcn_inverse_ballot_w64(m)) {
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)qt));
            wl.queue[pos & 255] = code;
        }
        qt += __popcll(m);
    };

    // diagonal: resolved through the table like any x'
    push(1ull, 0xFFFFFFFFu);

    // singles
    const int nsu = nu * vu, nsin = nsu + nd * vd;
    for (int base = 0; base < nsin; base += 64) {
        const int t = base + lane;
        const bool ok = t < nsin;
        int sp = 0, o = 0, v = 0;
        if (ok) {
            if (t < nsu) {
                o = t / vu;
                v = t - o * vu;
            } else {
                sp = 1;
                o = (t - nsu) / vd;
                v = (t - nsu) - o * vd;
            }
        }
        const int q = wl.occ[sp][o], p = wl.vir[sp][v];
        const uint32_t hh = hx ^ h_lds[q] ^ h_lds[p];
        const uint64_t m = __ballot(ok && filter_probe(wmask, hh) != 0u);
        if (m) {
            push(m, (uint32_t)q | 0xFF00u | ((uint32_t)p << 16) | 0xFF000000u);
            drain_full();
        }
    }

    // same-spin doubles: lane = empty pair (a<b), loops = occupied pair
    // (i<j), the inner one two connections per step
    for (int sp = 0; sp < 2; sp++) {
        const int ns = sp ? nd : nu, nv = sp ? vd : vu;
        const int npv = nv * (nv - 1) / 2;
        const uint32_t po_s = sp ? po_d : po_u;
        if (ns < 2 || npv == 0) continue;
        for (int base = 0; base < npv; base += 64) {
            const int vp = base + lane;
            const uint64_t okm = __ballot(vp < npv);
            int r1 = 0, rem = vp < npv ? vp : 0;
            while (rem >= nv - 1 - r1) {
                rem -= nv - 1 - r1;
                r1++;
            }
            const int a = wl.vir[sp][r1], b = wl.vir[sp][r1 + 1 + rem];
            const uint32_t hab = hx ^ h_lds[a] ^ h_lds[b];
            const uint32_t cab = ((uint32_t)a << 16) | ((uint32_t)b << 24);
            for (int o1 = 0; o1 < ns - 1; o1++) {
                const uint32_t s1 = (uint32_t)readlane32((int)po_s, o1);
                const uint32_t h1 = hab ^ s1, ci = s1 >> 25;
                for (int o2 = o1 + 1; o2 < ns; o2 += 2) {
                    const bool two = o2 + 1 < ns;
                    const uint32_t sa = (uint32_t)readlane32((int)po_s, o2);
                    const uint32_t sb = (uint32_t)readlane32((int)po_s, two ? o2 + 1 : o2);
                    const uint32_t ha = h1 ^ sa, hb = h1 ^ sb;
                    const uint32_t wa = filter_load(wmask, ha);
                    const uint32_t wb = filter_load(wmask, hb);
                    __builtin_amdgcn_sched_barrier(0);  // both filter reads in flight before the tests
                    const uint32_t pa = filter_test(wa, ha), pb = filter_test(wb, hb);
                    const uint64_t ma = __ballot(pa != 0u) & okm;
                    const uint64_t mb = __ballot(pb != 0u) & (two ? okm : 0ull);
                    if (ma | mb) {
                        push(ma, cab | ci | ((sa >> 25) << 8));
                        push(mb, cab | ci | ((sb >> 25) << 8));
                        drain_full();
                    }
                }
            }
        }
    }

    // opposite-spin doubles: lane = down single (j -> b), loops = up single
    // (i -> a), the inner one two connections per step
    const int nsd = nd * vd;
    if (nsu > 0 && nsd > 0) {
        for (int base = 0; base < nsd; base += 64) {
            const int d = base + lane;
            const uint64_t okm = __ballot(d < nsd);
            const int od = d < nsd ? d / vd : 0;
            const int bd = d < nsd ? d - od * vd : 0;
            const int j = wl.occ[1][od], b = wl.vir[1][bd];
            const uint32_t hd = hx ^ h_lds[j] ^ h_lds[b];
            const uint32_t cjb = ((uint32_t)j << 8) | ((uint32_t)b << 24);
            for (int o = 0; o < nu; o++) {
                const uint32_t s1 = (uint32_t)readlane32((int)po_u, o);
                const uint32_t h1 = hd ^ s1, ci = s1 >> 25;
                for (int v = 0; v < vu; v += 2) {
                    const bool two = v + 1 < vu;
                    const uint32_t sa = (uint32_t)readlane32((int)pv_u, v);
                    const uint32_t sb = (uint32_t)readlane32((int)pv_u, two ? v + 1 : v);
                    const uint32_t ha = h1 ^ sa, hb = h1 ^ sb;
                    const uint32_t wa = filter_load(wmask, ha);
                    const uint32_t wb = filter_load(wmask, hb);
                    __builtin_amdgcn_sched_barrier(0);  // both filter reads in flight before the tests
                    const uint32_t pa = filter_test(wa, ha), pb = filter_test(wb, hb);
                    const uint64_t ma = __ballot(pa != 0u) & okm;
                    const uint64_t mb = __ballot(pb != 0u) & (two ? okm : 0ull);
                    if (ma | mb) {
                        push(ma, cjb | ci | ((sa >> 25) << 16));
                        push(mb, cjb | ci | ((sb >> 25) << 16));
                        drain_full();
                    }
                }
            }
        }
    }
    while (qt > qh) {
        const int cnt = qt - qh < 64 ? qt - qh : 64;
        wave_sync();
        if (lane < cnt) process(wl.queue[(qh + lane) & 255]);
        qh += cnt;
        wave_sync();
    }

    double rs = are.s, rc = are.c, is = aim.s, ic = aim.c;
    wave_nsum(rs, rc);
    wave_nsum(is, ic);
    if (lane == 0) {
        eloc[2 * smp] = rs + rc;
        eloc[2 * smp + 1] = is + ic;
    }
    wave_sync();
}

// One system: persistent grid, wave-strided samples.  NT is the largest
// block the build is for (1024 threads only for the variant that fits in 128
// registers).
template <int W, int S8, int NT>
__global__ void __launch_bounds__(NT) k_eloc_sa(SysView S, TableView T, int lds_filter_log2,
                                                  const uint64_t *__restrict__ keys,
                                                  const double *__restrict__ logabs,
                                                  const double *__restrict__ phase, int64_t n,
                                                  double *__restrict__ eloc, int *status) {
    extern __shared__ __align__(16) uint8_t smem[];
    const SaStage G = sa_stage<W>(S, T, lds_filter_log2, smem);
    if (!G.at_zero) {
        if (threadIdx.x == 0) set_status(status, NNQS_EUNSUPPORTED);
        return;
    }
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    for (int64_t smp = (int64_t)blockIdx.x * nw + wid; smp < n; smp += (int64_t)gridDim.x * nw)
        sa_sample<W, S8, 0>(S, T, G, G.waves[wid], smp, keys, logabs, phase, eloc, status);
}

// The exact pass of one system (samples far below the table's largest
// amplitude; usually none, and then every wave only reads log|psi|).
template <int W>
__global__ void __launch_bounds__(kSaMaxThreads) k_eloc_sa_exact(SysView S, TableView T, int lds_filter_log2,
                                                        const uint64_t *__restrict__ keys,
                                                        const double *__restrict__ logabs,
                                                        const double *__restrict__ phase, int64_t n,
                                                        double *__restrict__ eloc, int *status) {
    extern __shared__ __align__(16) uint8_t smem[];
    const SaStage G = sa_stage<W>(S, T, lds_filter_log2, smem);
    if (!G.at_zero) {
        if (threadIdx.x == 0) set_status(status, NNQS_EUNSUPPORTED);
        return;
    }
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    for (int64_t smp = (int64_t)blockIdx.x * nw + wid; smp < n; smp += (int64_t)gridDim.x * nw)
        sa_sample<W, 0, 1>(S, T, G, G.waves[wid], smp, keys, logabs, phase, eloc, status);
}

// Many systems in one persistent launch: blocks pull tiles (a system and a
// run of its samples, in system order) from a device counter, restage the
// LDS data only when the system changes, and give each wave one sample at a
// time.  Every block leaves the loop when the counter passes the last tile.
template <int W, int S8, int EX>
__global__ void __launch_bounds__(kSaMaxThreads) k_eloc_sa_batch(const SaBatchItem *__restrict__ items,
                                                        const SaTile *__restrict__ tiles, int ntiles,
                                                        int *counter, uint32_t slot_off) {
    extern __shared__ __align__(16) uint8_t smem[];
    // the next-tile slot sits after the largest system's layout (dynamic LDS,
    // so that the filter keeps LDS address 0)
    int &next_tile = *reinterpret_cast<int *>(smem + slot_off);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    int staged = -1;
    SaStage G{};
    for (;;) {
        if (threadIdx.x == 0) next_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = next_tile;
        __syncthreads();
        if (t >= ntiles) break;
        const SaTile tl = tiles[t];
        const SaBatchItem &it = items[tl.item];
        if (tl.item != staged) {
            G = sa_stage<W>(it.S, it.T, it.lds_filter_log2, smem);
            staged = tl.item;
            if (!G.at_zero) {  // uniform: every block of the launch sees the same layout
                if (threadIdx.x == 0) set_status(it.status, NNQS_EUNSUPPORTED);
                break;
            }
        }
        for (int64_t smp = tl.begin + wid; smp < tl.begin + tl.count; smp += nw)
            sa_sample<W, S8, EX>(it.S, it.T, G, G.waves[wid], smp, it.keys, it.logabs, it.phase, it.eloc,
                                 it.status);
        __syncthreads();
    }
}

__global__ void k_reset_counter(int *c) { *c = 0; }

// Canonical-order export of every connection (tests): one wave per sample,
// lanes stride over the canonical index.
__global__ void __launch_bounds__(256) k_connections(SysView S, const uint64_t *__restrict__ keys, int64_t n,
                                                     uint64_t *__restrict__ xprime, int8_t *__restrict__ sign,
                                                     uint8_t *__restrict__ exc, double *__restrict__ hxx,
                                                     int *status) {
    __shared__ WaveLds wl_all[4];
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    WaveLds &wl = wl_all[wid];
    const int64_t C = S.C;
    for (int64_t smp = (int64_t)blockIdx.x * nw + wid; smp < n; smp += (int64_t)gridDim.x * nw) {
        Key x;
        x.lo = keys[2 * smp];
        x.hi = keys[2 * smp + 1];
        if (!sample_conserves(S, x)) {
            for (int64_t c = lane; c < C; c += 64) {
                const int64_t o = smp * C + c;
                if (xprime) {
                    xprime[2 * o] = 0;
                    xprime[2 * o + 1] = 0;
                }
                if (sign) sign[o] = 0;
                if (exc) exc[4 * o] = exc[4 * o + 1] = exc[4 * o + 2] = exc[4 * o + 3] = 255;
                if (hxx) hxx[o] = NAN;
            }
            if (lane == 0) set_status(status, NNQS_ECONSERVE);
            continue;
        }
        build_lists(S, x, wl);
        const double diag = wave_diag(S, x, wl);
        for (int64_t c0 = lane; c0 < C; c0 += 64) {
            int i, j, a, b;
            decode_canonical(S, wl, c0, i, j, a, b);
            int sg;
            const double hv = excitation_element(S, x, diag, i, j, a, b, &sg);
            Key xp = x;
            int e[4] = {255, 255, 255, 255};
            if (i != 255) {
                key_flip(xp, i);
                key_flip(xp, a);
                if (j == 255) {
                    e[0] = i;
                    e[2] = a;
                } else {
                    key_flip(xp, j);
                    key_flip(xp, b);
                    e[0] = i < j ? i : j;
                    e[1] = i < j ? j : i;
                    e[2] = a < b ? a : b;
                    e[3] = a < b ? b : a;
                }
            }
            const int64_t o = smp * C + c0;
            if (xprime) {
                xprime[2 * o] = xp.lo;
                xprime[2 * o + 1] = xp.hi;
            }
            if (sign) sign[o] = (int8_t)sg;
            if (exc) {
                exc[4 * o] = (uint8_t)e[0];
                exc[4 * o + 1] = (uint8_t)e[1];
                exc[4 * o + 2] = (uint8_t)e[2];
                exc[4 * o + 3] = (uint8_t)e[3];
            }
            if (hxx) hxx[o] = hv;
        }
        wave_sync();
    }
}

__global__ void k_validate_samples(SysView S, const uint64_t *__restrict__ keys, const double *__restrict__ logabs,
                                   const double *__restrict__ phase, int64_t n, int *status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Key x;
    x.lo = keys[2 * i];
    x.hi = keys[2 * i + 1];
    if (!sample_conserves(S, x)) set_status(status, NNQS_ECONSERVE);
    if (logabs && !isfinite(logabs[i])) set_status(status, NNQS_ERANGE);
    if (phase && !isfinite(phase[i])) set_status(status, NNQS_ERANGE);
}

__global__ void k_zero_int(int *p) { *p = 0; }

size_t sa_lds_bytes(int filter_log2, int split_levels, int W, int waves) {
    return sa_layout(filter_log2, split_levels, W, waves).total;
}

const void *sa_kernel_ptr(int W, int search, int waves) {
    const bool wide = waves > kSaMaxThreads / 64;
    if (W == 1) {
        if (search == 2)
            return wide ? reinterpret_cast<const void *>(k_eloc_sa<1, 1, kSaWideThreads>)
                        : reinterpret_cast<const void *>(k_eloc_sa<1, 1, kSaMaxThreads>);
        return wide ? reinterpret_cast<const void *>(k_eloc_sa<1, 0, kSaWideThreads>)
                    : reinterpret_cast<const void *>(k_eloc_sa<1, 0, kSaMaxThreads>);
    }
    if (search == 2)
        return wide ? reinterpret_cast<const void *>(k_eloc_sa<2, 1, kSaWideThreads>)
                    : reinterpret_cast<const void *>(k_eloc_sa<2, 1, kSaMaxThreads>);
    return wide ? reinterpret_cast<const void *>(k_eloc_sa<2, 0, kSaWideThreads>)
                : reinterpret_cast<const void *>(k_eloc_sa<2, 0, kSaMaxThreads>);
}

// Launch one build of the single-system kernel (the pointer from sa_kernel_ptr).
template <int W, int S8, int NT>
static void sa_launch_one(dim3 g, dim3 b, size_t lds, hipStream_t st, const SysView &S, const TableView &T, int fl,
                          const uint64_t *keys, const double *logabs, const double *phase, int64_t n, double *eloc,
                          int *status) {
    hipLaunchKernelGGL((k_eloc_sa<W, S8, NT>), g, b, lds, st, S, T, fl, keys, logabs, phase, n, eloc, status);
}

const void *sa_batch_kernel_ptr(int W, int search, bool exact) {
    if (exact) return W == 1 ? reinterpret_cast<const void *>(k_eloc_sa_batch<1, 0, 1>)
                             : reinterpret_cast<const void *>(k_eloc_sa_batch<2, 0, 1>);
    if (W == 1) return search == 2 ? reinterpret_cast<const void *>(k_eloc_sa_batch<1, 1, 0>)
                                   : reinterpret_cast<const void *>(k_eloc_sa_batch<1, 0, 0>);
    return search == 2 ? reinterpret_cast<const void *>(k_eloc_sa_batch<2, 1, 0>)
                       : reinterpret_cast<const void *>(k_eloc_sa_batch<2, 0, 0>);
}

// The sample-aware kernels are built to keep every value in registers; the
// library refuses to run a build that spills to private memory.
nnqs_status sa_check_no_spill(const void *fn) {
    hipFuncAttributes fa;
    NNQS_HIP_CHECK(hipFuncGetAttributes(&fa, fn));
    if (fa.localSizeBytes != 0)
        return fail(NNQS_EUNSUPPORTED, "sample-aware kernel uses %zu bytes of private memory per lane",
                    (size_t)fa.localSizeBytes);
    return NNQS_OK;
}

void sa_launch_batch(int W, int search, unsigned grid, int waves, size_t lds, hipStream_t st,
                     const SaBatchItem *items, const SaTile *tiles, int ntiles, int *counter) {
    const dim3 g(grid), b(waves * 64);
    // lds = the largest layout + the 16-byte next-tile slot at its end
    const uint32_t slot = (uint32_t)(lds - 16);
    // scaled pass, then the exact pass over the same tiles
    sa_launch_reset(counter, st);
    if (W == 1) {
        if (search == 2) hipLaunchKernelGGL((k_eloc_sa_batch<1, 1, 0>), g, b, lds, st, items, tiles, ntiles, counter, slot);
        else hipLaunchKernelGGL((k_eloc_sa_batch<1, 0, 0>), g, b, lds, st, items, tiles, ntiles, counter, slot);
    } else {
        if (search == 2) hipLaunchKernelGGL((k_eloc_sa_batch<2, 1, 0>), g, b, lds, st, items, tiles, ntiles, counter, slot);
        else hipLaunchKernelGGL((k_eloc_sa_batch<2, 0, 0>), g, b, lds, st, items, tiles, ntiles, counter, slot);
    }
    sa_launch_reset(counter, st);
    if (W == 1) hipLaunchKernelGGL((k_eloc_sa_batch<1, 0, 1>), g, b, lds, st, items, tiles, ntiles, counter, slot);
    else hipLaunchKernelGGL((k_eloc_sa_batch<2, 0, 1>), g, b, lds, st, items, tiles, ntiles, counter, slot);
}

void sa_launch_reset(int *counter, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter);
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

nnqs_status nnqs_connections(const nnqs_system *sys, const uint64_t *keys, int64_t n, uint64_t *xprime, int8_t *sign,
                             uint8_t *exc, double *hxx, uint32_t flags, void *stream) {
    clear_error();
    if (!sys || !keys) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    hipStream_t st = as_stream(stream);
    if (flags & NNQS_VALIDATE) {
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, sys->d_status);
        hipLaunchKernelGGL(k_validate_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sys->view, keys,
                           (const double *)nullptr, (const double *)nullptr, n, sys->d_status);
        int h = 0;
        NNQS_HIP_CHECK(hipMemcpyAsync(&h, sys->d_status, sizeof(int), hipMemcpyDeviceToHost, st));
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        if (h) return fail(h, "a sample violates the particle numbers");
    }
    int64_t blocks = (n + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_connections, dim3((unsigned)blocks), dim3(256), 0, st, sys->view, keys, n, xprime, sign, exc,
                       hxx, (int *)nullptr);
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

nnqs_status nnqs_eloc_table(const nnqs_system *sys, nnqs_table *tab, const uint64_t *keys, const uint32_t *counts,
                            const double *logabs, const double *phase, int64_t n, double *eloc, double *energy,
                            uint32_t flags, void *stream) {
    clear_error();
    if (!sys || !tab || !keys || !logabs || !phase || !eloc) return fail(NNQS_EINVAL, "null pointer argument");
    if (energy && !counts) return fail(NNQS_EINVAL, "energy requested without counts");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if (tab->sys != sys) return fail(NNQS_EINVAL, "table belongs to another system");
    if (tab->n <= 0) return fail(NNQS_EINVAL, "table is empty (build it first)");
    hipStream_t st = as_stream(stream);
    if (flags & NNQS_VALIDATE) {
        nnqs_status s = read_status(tab, st, true);
        if (s != NNQS_OK) return fail(s, "sticky table status set by an earlier call");
        hipLaunchKernelGGL(k_validate_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sys->view, keys,
                           logabs, phase, n, tab->status);
        NNQS_HIP_CHECK(hipGetLastError());
        s = read_status(tab, st, true);
        if (s != NNQS_OK)
            return fail(s, "sample validation failed (%s)",
                        s == NNQS_ECONSERVE ? "wrong particle number" : "non-finite amplitude");
    }
    const TableView tv = table_view(tab);
    const int W = sys->view.N > 64 ? 2 : 1;
    const int search = tab->tune.search;
    int waves = tab->tune.waves_per_block;
    const int max_waves = kSaWideThreads / 64;
    if (waves > max_waves) waves = max_waves;
    const void *fn = sa_kernel_ptr(W, search, waves);
    nnqs_status s0 = sa_check_no_spill(fn);
    if (s0 != NNQS_OK) return s0;
    int fl = tv.filter_log2;
    size_t lds = sa_lds_bytes(fl, tv.split_levels, W, waves);
    while (lds > (size_t)sys->max_lds && fl > 10) {  // fold the filter to fit
        fl--;
        lds = sa_lds_bytes(fl, tv.split_levels, W, waves);
    }
    if (lds > (size_t)sys->max_lds) return fail(NNQS_EINVAL, "LDS budget exceeded (%zu bytes)", lds);
    const unsigned grid = (unsigned)(sys->cu_count * tab->tune.blocks_per_cu);
    NNQS_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const dim3 g(grid), b(waves * 64);
    const bool wide = waves > kSaMaxThreads / 64;
    const SysView &SV = sys->view;
    int *stt = tab->status;
    if (W == 1) {
        if (search == 2) {
            if (wide) sa_launch_one<1, 1, kSaWideThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
            else sa_launch_one<1, 1, kSaMaxThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
        } else {
            if (wide) sa_launch_one<1, 0, kSaWideThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
            else sa_launch_one<1, 0, kSaMaxThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
        }
    } else {
        if (search == 2) {
            if (wide) sa_launch_one<2, 1, kSaWideThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
            else sa_launch_one<2, 1, kSaMaxThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
        } else {
            if (wide) sa_launch_one<2, 0, kSaWideThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
            else sa_launch_one<2, 0, kSaMaxThreads>(g, b, lds, st, SV, tv, fl, keys, logabs, phase, n, eloc, stt);
        }
    }
    {  // exact pass (12-wave blocks, filter folded to fit)
        const int ew = kSaMaxThreads / 64;
        int efl = tv.filter_log2;
        size_t elds = sa_lds_bytes(efl, tv.split_levels, W, ew);
        while (elds > (size_t)sys->max_lds && efl > 10) elds = sa_lds_bytes(--efl, tv.split_levels, W, ew);
        const void *efn = W == 1 ? reinterpret_cast<const void *>(k_eloc_sa_exact<1>)
                                 : reinterpret_cast<const void *>(k_eloc_sa_exact<2>);
        const nnqs_status se = sa_check_no_spill(efn);
        if (se != NNQS_OK) return se;
        NNQS_HIP_CHECK(hipFuncSetAttribute(efn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)elds));
        const dim3 eg((unsigned)sys->cu_count), eb(ew * 64);
        if (W == 1)
            hipLaunchKernelGGL((k_eloc_sa_exact<1>), eg, eb, elds, st, sys->view, tv, efl, keys, logabs, phase, n,
                               eloc, tab->status);
        else
            hipLaunchKernelGGL((k_eloc_sa_exact<2>), eg, eb, elds, st, sys->view, tv, efl, keys, logabs, phase, n,
                               eloc, tab->status);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    if (energy) return enqueue_energy(tab, counts, eloc, n, energy, st);
    return NNQS_OK;
}

// Autotuner of the single-system path: for every candidate schedule the
// table is rebuilt from the samples, one untimed call warms up, and the best
// of `reps` timed calls counts.  Candidates: waves per block {8, 12, 16} x
// splitter levels {8, 10, 12} x search {1, 2}.
nnqs_status nnqs_table_autotune(const nnqs_system *sys, nnqs_table *tab, const uint64_t *keys, const double *logabs,
                                const double *phase, int64_t n, double *eloc, int32_t reps, nnqs_tune *best_out,
                                double *best_ms, void *stream) {
    clear_error();
    if (!sys || !tab || !keys || !logabs || !phase || !eloc) return fail(NNQS_EINVAL, "null pointer argument");
    if (n <= 0 || n > tab->capacity) return fail(NNQS_EINVAL, "n outside 1..table capacity");
    if (reps < 1) reps = 1;
    hipStream_t st = as_stream(stream);
    hipEvent_t e0, e1;
    NNQS_HIP_CHECK(hipEventCreate(&e0));
    NNQS_HIP_CHECK(hipEventCreate(&e1));
    const nnqs_tune start = tab->tune;
    nnqs_tune best = start;
    float best_t = 1e30f;
    nnqs_status s = NNQS_OK;
    for (int waves : {8, 12, 16})
        for (int sl : {8, 10, 12})
            for (int search : {1, 2}) {
                nnqs_tune c = start;
                c.waves_per_block = waves;
                c.splitter_levels = sl;
                c.search = search;
                tab->tune = c;
                s = nnqs_table_build(tab, keys, logabs, phase, n, 0, stream);
                if (s != NNQS_OK) goto done;
                s = nnqs_eloc_table(sys, tab, keys, nullptr, logabs, phase, n, eloc, nullptr, 0, stream);
                if (s == NNQS_EINVAL) continue;  // does not fit: skip the candidate
                if (s != NNQS_OK) goto done;
                float tmin = 1e30f;
                for (int r = 0; r < reps; r++) {
                    if (hipEventRecord(e0, st) != hipSuccess) {
                        s = fail(NNQS_EHIP, "event record failed");
                        goto done;
                    }
                    s = nnqs_eloc_table(sys, tab, keys, nullptr, logabs, phase, n, eloc, nullptr, 0, stream);
                    if (s != NNQS_OK) goto done;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        s = fail(NNQS_EHIP, "event timing failed");
                        goto done;
                    }
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    tmin = ms < tmin ? ms : tmin;
                }
                if (tmin < best_t) {
                    best_t = tmin;
                    best = c;
                }
            }
    s = NNQS_OK;
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    tab->tune = best;
    {
        const nnqs_status s2 = nnqs_table_build(tab, keys, logabs, phase, n, 0, stream);
        if (s == NNQS_OK) s = s2;
    }
    if (s == NNQS_OK) {
        if (best_out) *best_out = best;
        if (best_ms) *best_ms = best_t;
    }
    return s;
}

// Autotuner cache: a text file of lines
//   <key> <waves_per_block> <blocks_per_cu> <filter_log2_bits> <splitter_levels> <search> <tile_samples> <ms>
// written whole to a temporary file and renamed over the old one.
nnqs_status nnqs_tune_key(const nnqs_system *sys, int64_t n, char *out, int64_t cap) {
    clear_error();
    if (!sys || !out) return fail(NNQS_EINVAL, "null pointer argument");
    hipDeviceProp_t prop{};
    NNQS_HIP_CHECK(hipGetDeviceProperties(&prop, sys->device));
    char arch[64];
    int a = 0;
    for (const char *c = prop.gcnArchName; *c && *c != ':' && a < 63; c++) arch[a++] = *c;  // drop feature flags
    arch[a] = 0;
    const int w = std::snprintf(out, (size_t)(cap > 0 ? cap : 0), "%s:cu%d:K%d:u%d:d%d:n%lld", arch, sys->cu_count,
                                sys->view.K, sys->view.n_up, sys->view.n_dn, (long long)n);
    if (w < 0 || w >= cap) return fail(NNQS_ERANGE, "key needs %d bytes", w + 1);
    return NNQS_OK;
}

static bool key_ok(const char *key) {
    if (!key || !*key) return false;
    for (const char *c = key; *c; c++)
        if (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r') return false;
    return true;
}

nnqs_status nnqs_tune_cache_lookup(const char *path, const char *key, nnqs_tune *tune, double *ms, int32_t *found) {
    clear_error();
    if (!path || !tune || !found) return fail(NNQS_EINVAL, "null pointer argument");
    if (!key_ok(key)) return fail(NNQS_EINVAL, "key must be non-empty without white space");
    *found = 0;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return NNQS_OK;  // no cache yet
    char line[512], k[256];
    while (std::fgets(line, sizeof line, f)) {
        nnqs_tune t{};
        double v = 0.0;
        if (std::sscanf(line, "%255s %d %d %d %d %d %d %lf", k, &t.waves_per_block, &t.blocks_per_cu,
                        &t.filter_log2_bits, &t.splitter_levels, &t.search, &t.tile_samples, &v) != 8)
            continue;  // not an entry
        if (std::strcmp(k, key) != 0 || !tune_valid(t)) continue;
        *tune = t;
        if (ms) *ms = v;
        *found = 1;  // the last valid entry of the key wins
    }
    std::fclose(f);
    return NNQS_OK;
}

nnqs_status nnqs_tune_cache_store(const char *path, const char *key, const nnqs_tune *tune, double ms) {
    clear_error();
    if (!path || !tune) return fail(NNQS_EINVAL, "null pointer argument");
    if (!key_ok(key)) return fail(NNQS_EINVAL, "key must be non-empty without white space");
    if (!tune_valid(*tune)) return fail(NNQS_EINVAL, "tuning parameters out of range");
    std::vector<std::string> keep;
    if (std::FILE *f = std::fopen(path, "r")) {
        char line[512], k[256];
        while (std::fgets(line, sizeof line, f)) {
            if (std::sscanf(line, "%255s", k) == 1 && std::strcmp(k, key) == 0) continue;  // replaced below
            keep.emplace_back(line);
        }
        std::fclose(f);
    }
    const std::string tmp = std::string(path) + ".tmp";
    std::FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(NNQS_EINVAL, "cannot write %s", tmp.c_str());
    for (const std::string &l : keep) std::fputs(l.c_str(), f);
    std::fprintf(f, "%s %d %d %d %d %d %d %.6f\n", key, tune->waves_per_block, tune->blocks_per_cu,
                 tune->filter_log2_bits, tune->splitter_levels, tune->search, tune->tile_samples, ms);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return fail(NNQS_EINVAL, "cannot replace %s", path);
    return NNQS_OK;
}

}  // extern "C"

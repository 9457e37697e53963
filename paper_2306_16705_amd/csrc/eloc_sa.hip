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

#include "enumerate.hpp"

namespace nnqs {

// Largest block of the sample-aware kernel: 12 waves, i.e. three per SIMD,
// which leaves the kernel up to 168 VGPRs (it needs about 150) so that
// nothing spills to private memory.
constexpr int kSaMaxThreads = 768;

// Blocked membership filter: the word is picked by the low hash bits, two
// bit positions inside it by the high word.
__device__ __forceinline__ bool filter_hit(const uint32_t *f, uint32_t wmask, uint64_t hh) {
    uint32_t w = f[(uint32_t)hh & wmask];
    uint32_t hb = (uint32_t)(hh >> 32);
    return (__builtin_amdgcn_ubfe(w, hb & 31u, 1u) & __builtin_amdgcn_ubfe(w, (hb >> 5) & 31u, 1u)) != 0u;
}

template <int W>
__device__ __forceinline__ Key load_key(const uint64_t *k, int64_t i) {
    Key r;
    r.lo = k[2 * i];
    r.hi = (W == 2) ? k[2 * i + 1] : 0ull;
    return r;
}

// Lower-bound search; the first `split_levels` levels read LDS copies of the
// keys they probe (every key at positions (m+1)*2^(L-s) - 1).
template <int W>
__device__ __forceinline__ int64_t table_find(const TableView &T, const uint64_t *s_lds, const Key &t) {
    const int L = T.log2n, s = T.split_levels;
    int64_t lo = 0;
    for (int lvl = 0; lvl < s; lvl++) {
        const int64_t step = int64_t(1) << (L - 1 - lvl);
        const int64_t j = ((lo + step) >> (L - s)) - 1;
        Key k;
        k.lo = s_lds[j * W];
        k.hi = (W == 2) ? s_lds[j * W + 1] : 0ull;
        if (key_less(k, t)) lo += step;
    }
    for (int lvl = s; lvl < L; lvl++) {
        const int64_t step = int64_t(1) << (L - 1 - lvl);
        const int64_t idx = lo + step - 1;
        if (idx < T.n && key_less(load_key<W>(T.keys, idx), t)) lo += step;
    }
    if (lo < T.n && key_eq(load_key<W>(T.keys, lo), t)) return lo;
    return -1;
}

template <int W>
__global__ void __launch_bounds__(kSaMaxThreads) k_eloc_sa(SysView S, TableView T, int lds_filter_log2,
                                                  const uint64_t *__restrict__ keys,
                                                  const double *__restrict__ logabs,
                                                  const double *__restrict__ phase, int64_t n,
                                                  double *__restrict__ eloc, int *status) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int nwords = 1 << (lds_filter_log2 - 5);
    const int big_words = 1 << (T.filter_log2 - 5);
    const int nsplit = (1 << T.split_levels) - 1;
    uint32_t *f_lds = reinterpret_cast<uint32_t *>(smem);
    uint64_t *s_lds = reinterpret_cast<uint64_t *>(smem + (size_t)nwords * 4);
    uint64_t *h_lds = s_lds + (size_t)nsplit * W;
    WaveLds *wl_all = reinterpret_cast<WaveLds *>(h_lds + 128);

    // Stage the filter (folded to the LDS size: OR of aliasing words keeps
    // every member), the top search levels and the hash words.
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) {
        uint32_t v = 0;
        for (int k = i; k < big_words; k += nwords) v |= T.filter[k];
        f_lds[i] = v;
    }
    for (int i = threadIdx.x; i < nsplit; i += blockDim.x) {
        s_lds[(size_t)i * W] = T.split[2 * i];
        if (W == 2) s_lds[(size_t)i * W + 1] = T.split[2 * i + 1];
    }
    for (int i = threadIdx.x; i < 128; i += blockDim.x) h_lds[i] = S.hashT[i];
    __syncthreads();

    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    WaveLds &wl = wl_all[wid];
    const uint32_t wmask = (uint32_t)nwords - 1u;
    const int K = S.K, nu = S.n_up, nd = S.n_dn, vu = K - nu, vd = K - nd;

    for (int64_t smp = (int64_t)blockIdx.x * nw + wid; smp < n; smp += (int64_t)gridDim.x * nw) {
        Key x;
        x.lo = keys[2 * smp];
        x.hi = keys[2 * smp + 1];
        const double la = logabs[smp], ph = phase[smp];
        if (!sample_conserves(S, x) || !isfinite(la) || !isfinite(ph)) {
            if (lane == 0) {
                eloc[2 * smp] = NAN;
                eloc[2 * smp + 1] = NAN;
                set_status(status, sample_conserves(S, x) ? NNQS_ERANGE : NNQS_ECONSERVE);
            }
            continue;
        }
        build_lists(S, x, wl);
        // hash of x and per-lane list values held in registers
        uint64_t part = 0;
        if (lane < K) {
            if (key_bit(x, 2 * lane)) part ^= h_lds[2 * lane];
            if (key_bit(x, 2 * lane + 1)) part ^= h_lds[2 * lane + 1];
        }
        const uint64_t hx = wave_xor64(part);
        const double diag = wave_diag(S, x, wl);
        // per-lane copies of the lists (lane l holds entry l) for wave-uniform
        // readlane access in the outer loops
        const int occ_u = lane < nu ? wl.occ[0][lane] : 0;
        const int occ_d = lane < nd ? wl.occ[1][lane] : 0;
        const int vir_u = lane < vu ? wl.vir[0][lane] : 0;
        const uint64_t hocc_u = h_lds[occ_u], hocc_d = h_lds[occ_d], hvir_u = h_lds[vir_u];

        NSum are{0.0, 0.0}, aim{0.0, 0.0};
        int qh = 0, qt = 0;  // wave-uniform ring counters

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
            const int64_t idx = table_find<W>(T, s_lds, xp);
            if (idx >= 0) {
                int sg;
                const double hv = excitation_element(S, x, diag, i, j, a, b, &sg);
                const double r = exp(T.logabs[idx] - la);
                double sn, cs;
                sincos(T.phase[idx] - ph, &sn, &cs);
                are.add(hv * r * cs);
                aim.add(hv * r * sn);
            }
        };
        auto drain = [&](int cnt) {
            wave_sync();
            if (lane < cnt) process(wl.queue[(qh + lane) & 127]);
            qh += cnt;
            wave_sync();
        };
        auto push = [&](bool cand, uint32_t code) {
            const uint64_t m = __ballot(cand);
            if (m) {
                if (cand) wl.queue[(qt + mbcnt(m)) & 127] = code;
                qt += __popcll(m);
                if (qt - qh >= 64) drain(64);
            }
        };

        // diagonal: always resolved through the table like any x'
        push(lane == 0, 0xFFFFFFFFu);

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
            const int q = ok ? wl.occ[sp][o] : 0, p = ok ? wl.vir[sp][v] : 0;
            const uint64_t hh = hx ^ h_lds[q] ^ h_lds[p];
            push(ok && filter_hit(f_lds, wmask, hh), (uint32_t)q | 0xFF00u | ((uint32_t)p << 16) | 0xFF000000u);
        }

        // same-spin doubles: lane = empty pair (a<b), loop = occupied pair (i<j)
        for (int sp = 0; sp < 2; sp++) {
            const int ns = sp ? nd : nu, nv = sp ? vd : vu;
            const int npv = nv * (nv - 1) / 2;
            const int occ_s = sp ? occ_d : occ_u;
            const uint64_t hocc_s = sp ? hocc_d : hocc_u;
            if (ns < 2 || npv == 0) continue;
            for (int base = 0; base < npv; base += 64) {
                const int vp = base + lane;
                const bool ok = vp < npv;
                int r1 = 0, rem = ok ? vp : 0;
                while (rem >= nv - 1 - r1) {
                    rem -= nv - 1 - r1;
                    r1++;
                }
                const int a = wl.vir[sp][r1], b = wl.vir[sp][r1 + 1 + rem];
                const uint64_t hab = hx ^ h_lds[a] ^ h_lds[b];
                const uint32_t cab = ((uint32_t)a << 16) | ((uint32_t)b << 24);
                for (int o1 = 0; o1 < ns - 1; o1++) {
                    const int i = readlane32(occ_s, o1);
                    const uint64_t hi_ = hab ^ readlane64(hocc_s, o1);
                    for (int o2 = o1 + 1; o2 < ns; o2++) {
                        const int j = readlane32(occ_s, o2);
                        const uint64_t hh = hi_ ^ readlane64(hocc_s, o2);
                        push(ok && filter_hit(f_lds, wmask, hh), cab | (uint32_t)i | ((uint32_t)j << 8));
                    }
                }
            }
        }

        // opposite-spin doubles: lane = down single (j -> b), loop = up single (i -> a)
        const int nsd = nd * vd;
        if (nsu > 0 && nsd > 0) {
            for (int base = 0; base < nsd; base += 64) {
                const int d = base + lane;
                const bool ok = d < nsd;
                const int od = ok ? d / vd : 0;
                const int bd = ok ? d - od * vd : 0;
                const int j = wl.occ[1][od], b = wl.vir[1][bd];
                const uint64_t hd = hx ^ h_lds[j] ^ h_lds[b];
                const uint32_t cjb = ((uint32_t)j << 8) | ((uint32_t)b << 24);
                for (int o = 0; o < nu; o++) {
                    const int i = readlane32(occ_u, o);
                    const uint64_t hdi = hd ^ readlane64(hocc_u, o);
                    for (int v = 0; v < vu; v++) {
                        const int a = readlane32(vir_u, v);
                        const uint64_t hh = hdi ^ readlane64(hvir_u, v);
                        push(ok && filter_hit(f_lds, wmask, hh), cjb | (uint32_t)i | ((uint32_t)a << 16));
                    }
                }
            }
        }
        if (qt > qh) drain(qt - qh);

        double rs = are.s, rc = are.c, is = aim.s, ic = aim.c;
        wave_nsum(rs, rc);
        wave_nsum(is, ic);
        if (lane == 0) {
            eloc[2 * smp] = rs + rc;
            eloc[2 * smp + 1] = is + ic;
        }
        wave_sync();
    }
}

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

static size_t sa_lds_bytes(int filter_log2, int split_levels, int W, int waves) {
    return ((size_t)1 << (filter_log2 - 5)) * 4 + (((size_t)1 << split_levels) - 1) * 8 * W + 128 * 8 +
           sizeof(WaveLds) * waves;
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
    int waves = tab->tune.waves_per_block;
    if (waves * 64 > kSaMaxThreads) waves = kSaMaxThreads / 64;
    // The kernel is built to keep every value in registers; refuse to run a
    // build that spills to private memory.
    {
        hipFuncAttributes fa;
        const void *fn = W == 1 ? reinterpret_cast<const void *>(k_eloc_sa<1>)
                                : reinterpret_cast<const void *>(k_eloc_sa<2>);
        NNQS_HIP_CHECK(hipFuncGetAttributes(&fa, fn));
        if (fa.localSizeBytes != 0)
            return fail(NNQS_EUNSUPPORTED, "sample-aware kernel uses %zu bytes of private memory per lane",
                        (size_t)fa.localSizeBytes);
    }
    int fl = tv.filter_log2;
    size_t lds = sa_lds_bytes(fl, tv.split_levels, W, waves);
    while (lds > (size_t)sys->max_lds && fl > 10) {  // fold the filter to fit
        fl--;
        lds = sa_lds_bytes(fl, tv.split_levels, W, waves);
    }
    if (lds > (size_t)sys->max_lds) return fail(NNQS_EINVAL, "LDS budget exceeded (%zu bytes)", lds);
    const unsigned grid = (unsigned)(sys->cu_count * tab->tune.blocks_per_cu);
    if (W == 1) {
        NNQS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_eloc_sa<1>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_eloc_sa<1>, dim3(grid), dim3(waves * 64), lds, st, sys->view, tv, fl, keys, logabs, phase,
                           n, eloc, tab->status);
    } else {
        NNQS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_eloc_sa<2>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_eloc_sa<2>, dim3(grid), dim3(waves * 64), lds, st, sys->view, tv, fl, keys, logabs, phase,
                           n, eloc, tab->status);
    }
    NNQS_HIP_CHECK(hipGetLastError());
    if (energy) return enqueue_energy(tab, counts, eloc, n, energy, st);
    return NNQS_OK;
}

}  // extern "C"

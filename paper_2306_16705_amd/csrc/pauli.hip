// Second backend: the Hamiltonian as compressed Pauli strings and the
// sample-aware local energy over them (paper: Section 3.4 items 1, 2, 4, 5;
// Algorithm 1 builds the grouped layout, Algorithm 2 evaluates it).
//
// Builder (host, once per system).  The Jordan-Wigner images of the ladder
// operators (strings over lower indices) are multiplied out in the
// X^x Z^z form, with (X^x1 Z^z1)(X^x2 Z^z2) = (-1)^{|z1 & x2|} X^{x1^x2}
// Z^{z1^z2}, for every term of
//   H = E_core + sum_pq h_pq a+_p a_q
//     + sum_{p<q, r<s} (<pq|rs> - <pq|sr>) a+_p a+_q a_s a_r,
// and equal strings are summed.  Strings are grouped by their X part (the
// paper's XY tuple): every string of a group moves a configuration x to the
// same x' = x ^ XY.  For the matrix element, X^x Z^z |x'> = (-1)^{|x' & z|}
// |x' ^ x>, so <x|X^xm Z^zm|x ^ xm> = (-1)^{|xm & zm|} (-1)^{|x & zm|}: the
// first sign is folded into the stored coefficient (the paper folds
// (-i)^{#Y} the same way), the second is the per-sample parity of the YZ
// tuple (here zm).  A real Hamiltonian has real coefficients in this basis.
//
// Kernel.  One wave per sample; lanes take groups, probe the table's
// membership filter with the linear hash of x ^ XY (hash(x) ^ hash(XY)),
// queue survivors, and resolve them 64 at a time: table search, then the
// group's coefficient sum with the parities and the log-polar ratio.
#include <algorithm>
#include <cmath>
#include <complex>
#include <unordered_map>
#include <vector>

#include "enumerate.hpp"

struct nnqs_pauli {
    const nnqs_system *sys = nullptr;
    int64_t n_groups = 0, n_strings = 0;
    uint64_t *d_xy = nullptr;     // [NK][2] X part of each group
    uint32_t *d_ghash = nullptr;  // [NK] low 32 bits of the linear hash of the X part
    int64_t *d_idx = nullptr;     // [NK + 1] string range of each group
    uint64_t *d_zm = nullptr;     // [NT][2] Z part of each string
    double *d_coef = nullptr;     // [NT] coefficient with (-1)^{|xm & zm|} folded in
};

namespace nnqs {

// ------------------------------------------------------------ host builder
struct PStr {
    uint64_t x0, x1, z0, z1;
    bool operator==(const PStr &o) const { return x0 == o.x0 && x1 == o.x1 && z0 == o.z0 && z1 == o.z1; }
};
struct PStrHash {
    size_t operator()(const PStr &p) const {
        uint64_t h = p.x0 * 0x9E3779B97F4A7C15ull ^ (p.x1 + 0x632BE59BD9B4E019ull);
        h ^= (p.z0 + 0x94D049BB133111EBull) * 0xBF58476D1CE4E5B9ull;
        h ^= p.z1 * 0xD6E8FEB86659FD93ull;
        return (size_t)(h ^ (h >> 29));
    }
};
struct PTerm {
    PStr s;
    std::complex<double> c;
};

static inline int popc2(uint64_t a, uint64_t b) { return __builtin_popcountll(a) + __builtin_popcountll(b); }

static PTerm pmul(const PTerm &a, const PTerm &b) {
    PTerm r;
    const int sg = popc2(a.s.z0 & b.s.x0, a.s.z1 & b.s.x1) & 1;
    r.s = PStr{a.s.x0 ^ b.s.x0, a.s.x1 ^ b.s.x1, a.s.z0 ^ b.s.z0, a.s.z1 ^ b.s.z1};
    r.c = a.c * b.c * (sg ? -1.0 : 1.0);
    return r;
}

// Jordan-Wigner image of a_p (dagger = false) or a+_p: Z_{<p} (X_p +- i Y_p)/2
// = 1/2 X^{e_p} Z^{<p} -+ 1/2 X^{e_p} Z^{<p or p} (with Y = i X Z).
static void ladder(int p, bool dagger, PTerm out[2]) {
    uint64_t e0 = 0, e1 = 0, s0 = 0, s1 = 0;
    if (p < 64) {
        e0 = 1ull << p;
        s0 = e0 - 1;
    } else {
        e1 = 1ull << (p - 64);
        s0 = ~0ull;
        s1 = e1 - 1;
    }
    out[0] = PTerm{PStr{e0, e1, s0, s1}, 0.5};
    out[1] = PTerm{PStr{e0, e1, s0 ^ e0, s1 ^ e1}, dagger ? 0.5 : -0.5};
}

struct PauliBuilt {
    std::vector<uint64_t> xy;  // [NK][2]
    std::vector<int64_t> idx;  // [NK + 1]
    std::vector<uint64_t> zm;  // [NT][2]
    std::vector<double> coef;  // [NT]
};

static nnqs_status build_pauli(int N, const double *h, const double *g, double e_core, PauliBuilt &out) {
    const int K = N / 2;
    std::unordered_map<PStr, std::complex<double>, PStrHash> acc;
    acc.reserve((size_t)N * N * N * N / 16 + 1024);
    auto add_product = [&](const int *ops, const bool *dag, int nops, double c) {
        PTerm l[4][2];
        for (int t = 0; t < nops; t++) ladder(ops[t], dag[t], l[t]);
        const int combos = 1 << nops;
        for (int m = 0; m < combos; m++) {
            PTerm r = PTerm{PStr{0, 0, 0, 0}, c};
            for (int t = 0; t < nops; t++) r = pmul(r, l[t][(m >> t) & 1]);
            acc[r.s] += r.c;
        }
    };
    if (e_core != 0.0) acc[PStr{0, 0, 0, 0}] += e_core;
    // one-body: h_pq a+_p a_q, same spin
    for (int p = 0; p < N; p++)
        for (int q = 0; q < N; q++) {
            if ((p ^ q) & 1) continue;
            const double v = h[(p >> 1) * K + (q >> 1)];
            if (v == 0.0) continue;
            const int ops[2] = {p, q};
            const bool dag[2] = {true, false};
            add_product(ops, dag, 2, v);
        }
    // two-body: (<pq|rs> - <pq|sr>) a+_p a+_q a_s a_r for p<q, r<s, with
    // <pq|rs> = (i_p i_r | i_q i_s) when spin(p) = spin(r) and spin(q) = spin(s)
    auto chem = [&](int a, int b, int c, int d) { return g[(((int64_t)a * K + b) * K + c) * K + d]; };
    auto phys = [&](int p, int q, int r, int s) -> double {
        if (((p ^ r) & 1) || ((q ^ s) & 1)) return 0.0;
        return chem(p >> 1, r >> 1, q >> 1, s >> 1);
    };
    for (int p = 0; p < N; p++)
        for (int q = p + 1; q < N; q++)
            for (int r = 0; r < N; r++)
                for (int s = r + 1; s < N; s++) {
                    const double v = phys(p, q, r, s) - phys(p, q, s, r);
                    if (v == 0.0) continue;
                    const int ops[4] = {p, q, s, r};
                    const bool dag[4] = {true, true, false, false};
                    add_product(ops, dag, 4, v);
                }
    // drop cancelled strings, check reality, fold (-1)^{|xm & zm|}, group by X part
    double cmax = 0.0;
    for (const auto &kv : acc) cmax = std::max(cmax, std::abs(kv.second));
    std::vector<PTerm> terms;
    terms.reserve(acc.size());
    for (const auto &kv : acc) {
        if (std::abs(kv.second) <= 1e-13 * cmax) continue;
        if (std::abs(kv.second.imag()) > 1e-10 * std::max(1.0, cmax))
            return fail(NNQS_EINVAL, "the Pauli expansion has an imaginary coefficient (integrals not real-symmetric?)");
        const int sg = popc2(kv.first.x0 & kv.first.z0, kv.first.x1 & kv.first.z1) & 1;
        terms.push_back(PTerm{kv.first, sg ? -kv.second.real() : kv.second.real()});
    }
    std::sort(terms.begin(), terms.end(), [](const PTerm &a, const PTerm &b) {
        if (a.s.x1 != b.s.x1) return a.s.x1 < b.s.x1;
        if (a.s.x0 != b.s.x0) return a.s.x0 < b.s.x0;
        if (a.s.z1 != b.s.z1) return a.s.z1 < b.s.z1;
        return a.s.z0 < b.s.z0;
    });
    out.xy.clear();
    out.idx.clear();
    out.zm.clear();
    out.coef.clear();
    for (size_t t = 0; t < terms.size(); t++) {
        if (t == 0 || terms[t].s.x0 != terms[t - 1].s.x0 || terms[t].s.x1 != terms[t - 1].s.x1) {
            out.xy.push_back(terms[t].s.x0);
            out.xy.push_back(terms[t].s.x1);
            out.idx.push_back((int64_t)t);
        }
        out.zm.push_back(terms[t].s.z0);
        out.zm.push_back(terms[t].s.z1);
        out.coef.push_back(terms[t].c.real());
    }
    out.idx.push_back((int64_t)terms.size());
    return NNQS_OK;
}

// --------------------------------------------------------------- kernel
template <int W>
__global__ void __launch_bounds__(768) k_eloc_pauli(SysView S, TableView T, int lds_filter_log2,
                                                  const uint64_t *__restrict__ gxy,
                                                  const uint32_t *__restrict__ ghash,
                                                  const int64_t *__restrict__ gidx,
                                                  const uint64_t *__restrict__ zm,
                                                  const double *__restrict__ coef, int64_t NK,
                                                  const uint64_t *__restrict__ keys,
                                                  const double *__restrict__ logabs,
                                                  const double *__restrict__ phase, int64_t n,
                                                  double *__restrict__ eloc, int *status) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int nwords = 1 << (lds_filter_log2 - 5);
    const int big_words = 1 << (T.filter_log2 - 5);
    const int nsplit = (1 << T.split_levels) - 1;
    // layout: filter words, staged keys, low hash words, one WaveLds per wave
    const size_t off_split = (size_t)nwords * 4;
    const size_t off_hash = off_split + (size_t)nsplit * 8 * W;
    const size_t off_waves = (off_hash + 128 * 4 + 15) & ~(size_t)15;
    uint32_t *f_lds = reinterpret_cast<uint32_t *>(smem);
    uint64_t *s_lds = reinterpret_cast<uint64_t *>(smem + off_split);
    uint32_t *h_lds = reinterpret_cast<uint32_t *>(smem + off_hash);
    WaveLds *wl_all = reinterpret_cast<WaveLds *>(smem + off_waves);
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
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    WaveLds &wl = wl_all[wid];
    const uint32_t wmask = (uint32_t)nwords - 1u;
    const int L = T.log2n, sl = T.split_levels;

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
        uint32_t part = 0;
        if (lane < S.K) {
            if (key_bit(x, 2 * lane)) part ^= h_lds[2 * lane];
            if (key_bit(x, 2 * lane + 1)) part ^= h_lds[2 * lane + 1];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) part ^= __shfl_xor(part, off, 64);
        const uint32_t hx = part;
        NSum are{0.0, 0.0}, aim{0.0, 0.0};
        int qh = 0, qt = 0;
        auto process = [&](uint32_t k) {
            Key xp;
            xp.lo = x.lo ^ gxy[2 * (int64_t)k];
            xp.hi = x.hi ^ gxy[2 * (int64_t)k + 1];
            // lower-bound search: LDS levels, then one load per level
            int64_t lo = 0;
            for (int lvl = 0; lvl < sl; lvl++) {
                const int64_t step = int64_t(1) << (L - 1 - lvl);
                const int64_t j = ((lo + step) >> (L - sl)) - 1;
                Key kk;
                kk.lo = s_lds[j * W];
                kk.hi = (W == 2) ? s_lds[j * W + 1] : 0ull;
                if (key_less(kk, xp)) lo += step;
            }
            for (int lvl = sl; lvl < L; lvl++) {
                const int64_t step = int64_t(1) << (L - 1 - lvl);
                const int64_t i = lo + step - 1;
                Key kk;
                kk.lo = i < T.n ? T.keys[2 * i] : 0ull;
                kk.hi = (W == 2 && i < T.n) ? T.keys[2 * i + 1] : 0ull;
                if (i < T.n && key_less(kk, xp)) lo += step;
            }
            if (lo >= T.n || T.keys[2 * lo] != xp.lo || (W == 2 && T.keys[2 * lo + 1] != xp.hi)) return;
            double hv = 0.0;
            for (int64_t i = gidx[k]; i < gidx[k + 1]; i++) {
                const int par = (__popcll(x.lo & zm[2 * i]) + __popcll(x.hi & zm[2 * i + 1])) & 1;
                hv += par ? -coef[i] : coef[i];
            }
            const double r = exp(T.logabs[lo] - la);
            double sn, cs;
            sincos(T.phase[lo] - ph, &sn, &cs);
            are.add(hv * r * cs);
            aim.add(hv * r * sn);
        };
        auto drain = [&](int cnt) {
            wave_sync();
            if (lane < cnt) process(wl.queue[(qh + lane) & 255]);
            qh += cnt;
            wave_sync();
        };
        for (int64_t base = 0; base < NK; base += 64) {
            const int64_t k = base + lane;
            const bool ok = k < NK;
            const uint32_t hh = hx ^ (ok ? ghash[k] : 0u);
            const uint32_t w = f_lds[filter_word(hh, wmask)];
            const bool cand = ok && filter_test(w, hh) != 0u;
            const uint64_t m = __ballot(cand);
            if (m) {
                if (cand) wl.queue[(qt + mbcnt(m)) & 255] = (uint32_t)k;
                qt += __popcll(m);
                if (qt - qh >= 64) drain(64);
            }
        }
        while (qt > qh) drain(qt - qh < 64 ? qt - qh : 64);
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

static size_t pauli_lds_bytes(int filter_log2, int split_levels, int W, int waves) {
    const size_t off_split = ((size_t)1 << (filter_log2 - 5)) * 4;
    const size_t off_hash = off_split + (((size_t)1 << split_levels) - 1) * 8 * W;
    const size_t off_waves = (off_hash + 128 * 4 + 15) & ~(size_t)15;
    return off_waves + sizeof(WaveLds) * waves;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" {

nnqs_status nnqs_pauli_build_host(int32_t n_spin_orb, const double *h, const double *g, double e_core,
                                  int64_t *n_groups, int64_t *n_strings, uint64_t *xy, int64_t *idx, uint64_t *zm,
                                  double *coef) {
    clear_error();
    if (!h || !g || !n_groups || !n_strings) return fail(NNQS_EINVAL, "null pointer argument");
    if (n_spin_orb < 2 || n_spin_orb > 128 || (n_spin_orb & 1))
        return fail(NNQS_EINVAL, "n_spin_orb must be even, 2..128");
    PauliBuilt b;
    nnqs_status s = build_pauli(n_spin_orb, h, g, e_core, b);
    if (s != NNQS_OK) return s;
    const int64_t NK = (int64_t)b.idx.size() - 1, NT = (int64_t)b.coef.size();
    if (xy || idx || zm || coef) {
        if (*n_groups < NK || *n_strings < NT) {
            *n_groups = NK;
            *n_strings = NT;
            return fail(NNQS_ERANGE, "output arrays too small (%lld groups, %lld strings needed)", (long long)NK,
                        (long long)NT);
        }
        if (xy) std::copy(b.xy.begin(), b.xy.end(), xy);
        if (idx) std::copy(b.idx.begin(), b.idx.end(), idx);
        if (zm) std::copy(b.zm.begin(), b.zm.end(), zm);
        if (coef) std::copy(b.coef.begin(), b.coef.end(), coef);
    }
    *n_groups = NK;
    *n_strings = NT;
    return NNQS_OK;
}

nnqs_status nnqs_pauli_create(nnqs_pauli **out, const nnqs_system *sys) {
    clear_error();
    if (!out || !sys) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    const int N = sys->view.N, K = sys->view.K;
    std::vector<double> h((size_t)K * K), g((size_t)K * K * K * K);
    std::vector<uint64_t> hashT(128);
    NNQS_HIP_CHECK(hipMemcpy(h.data(), sys->d_h, h.size() * 8, hipMemcpyDeviceToHost));
    NNQS_HIP_CHECK(hipMemcpy(g.data(), sys->d_g, g.size() * 8, hipMemcpyDeviceToHost));
    NNQS_HIP_CHECK(hipMemcpy(hashT.data(), sys->d_hash, 128 * 8, hipMemcpyDeviceToHost));
    PauliBuilt b;
    nnqs_status s = build_pauli(N, h.data(), g.data(), sys->view.ecore, b);
    if (s != NNQS_OK) return s;
    const int64_t NK = (int64_t)b.idx.size() - 1, NT = (int64_t)b.coef.size();
    std::vector<uint32_t> gh(NK);
    for (int64_t k = 0; k < NK; k++) {
        uint64_t hsh = 0;
        for (int w = 0; w < 2; w++)
            for (uint64_t m = b.xy[2 * k + w]; m; m &= m - 1) hsh ^= hashT[64 * w + __builtin_ctzll(m)];
        gh[k] = (uint32_t)hsh;
    }
    nnqs_pauli *p = new nnqs_pauli();
    p->sys = sys;
    p->n_groups = NK;
    p->n_strings = NT;
    if (hipMalloc(&p->d_xy, NK * 16) != hipSuccess || hipMalloc(&p->d_ghash, NK * 4 + 4) != hipSuccess ||
        hipMalloc(&p->d_idx, (NK + 1) * 8) != hipSuccess || hipMalloc(&p->d_zm, NT * 16 + 16) != hipSuccess ||
        hipMalloc(&p->d_coef, NT * 8 + 8) != hipSuccess) {
        nnqs_pauli_destroy(p);
        return fail(NNQS_ENOMEM, "Pauli Hamiltonian allocation failed");
    }
    if (hipMemcpy(p->d_xy, b.xy.data(), NK * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_ghash, gh.data(), NK * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_idx, b.idx.data(), (NK + 1) * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_zm, b.zm.data(), NT * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_coef, b.coef.data(), NT * 8, hipMemcpyHostToDevice) != hipSuccess) {
        nnqs_pauli_destroy(p);
        return fail(NNQS_EHIP, "Pauli Hamiltonian upload failed");
    }
    *out = p;
    return NNQS_OK;
}

nnqs_status nnqs_pauli_destroy(nnqs_pauli *p) {
    if (!p) return NNQS_OK;
    hipFree(p->d_xy);
    hipFree(p->d_ghash);
    hipFree(p->d_idx);
    hipFree(p->d_zm);
    hipFree(p->d_coef);
    delete p;
    return NNQS_OK;
}

nnqs_status nnqs_pauli_info(const nnqs_pauli *p, int64_t *n_groups, int64_t *n_strings, int64_t *bytes_grouped,
                            int64_t *bytes_flat) {
    clear_error();
    if (!p) return fail(NNQS_EINVAL, "null pointer argument");
    const int64_t wb = p->sys->view.N > 64 ? 16 : 8;  // bytes of one N-bit tuple
    if (n_groups) *n_groups = p->n_groups;
    if (n_strings) *n_strings = p->n_strings;
    // grouped (Algorithm 1): per group an XY tuple and an index; per string a YZ tuple and a coefficient
    if (bytes_grouped) *bytes_grouped = p->n_groups * (wb + 8) + p->n_strings * (wb + 8);
    // flat: per string XY and YZ tuples, a Y count and a coefficient
    if (bytes_flat) *bytes_flat = p->n_strings * (2 * wb + 4 + 8);
    return NNQS_OK;
}

nnqs_status nnqs_eloc_pauli(const nnqs_pauli *p, nnqs_table *tab, const uint64_t *keys, const uint32_t *counts,
                            const double *logabs, const double *phase, int64_t n, double *eloc, double *energy,
                            uint32_t flags, void *stream) {
    clear_error();
    if (!p || !tab || !keys || !logabs || !phase || !eloc) return fail(NNQS_EINVAL, "null pointer argument");
    if (energy && !counts) return fail(NNQS_EINVAL, "energy requested without counts");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    const nnqs_system *sys = p->sys;
    if (tab->sys != sys) return fail(NNQS_EINVAL, "table belongs to another system");
    if (tab->n <= 0) return fail(NNQS_EINVAL, "table is empty (build it first)");
    if (p->n_groups > (int64_t)UINT32_MAX) return fail(NNQS_EUNSUPPORTED, "too many Pauli groups");
    hipStream_t st = as_stream(stream);
    (void)flags;
    const TableView tv = table_view(tab);
    const int W = sys->view.N > 64 ? 2 : 1;
    const int waves = 12;
    int fl = tv.filter_log2;
    size_t lds = pauli_lds_bytes(fl, tv.split_levels, W, waves);
    while (lds > (size_t)sys->max_lds && fl > 10) lds = pauli_lds_bytes(--fl, tv.split_levels, W, waves);
    if (lds > (size_t)sys->max_lds) return fail(NNQS_EINVAL, "LDS budget exceeded (%zu bytes)", lds);
    const void *fn = W == 1 ? reinterpret_cast<const void *>(k_eloc_pauli<1>)
                            : reinterpret_cast<const void *>(k_eloc_pauli<2>);
    nnqs_status s0 = sa_check_no_spill(fn);
    if (s0 != NNQS_OK) return s0;
    NNQS_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const dim3 g((unsigned)sys->cu_count), b(waves * 64);
    if (W == 1)
        hipLaunchKernelGGL(k_eloc_pauli<1>, g, b, lds, st, sys->view, tv, fl, p->d_xy, p->d_ghash, p->d_idx,
                           p->d_zm, p->d_coef, p->n_groups, keys, logabs, phase, n, eloc, tab->status);
    else
        hipLaunchKernelGGL(k_eloc_pauli<2>, g, b, lds, st, sys->view, tv, fl, p->d_xy, p->d_ghash, p->d_idx,
                           p->d_zm, p->d_coef, p->n_groups, keys, logabs, phase, n, eloc, tab->status);
    NNQS_HIP_CHECK(hipGetLastError());
    if (energy) return enqueue_energy(tab, counts, eloc, n, energy, st);
    return NNQS_OK;
}

}  // extern "C"

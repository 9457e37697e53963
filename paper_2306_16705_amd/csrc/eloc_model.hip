// Full local energy with every connected amplitude from the network
// (paper: Eq. 4 summed over all x' with H_xx' != 0; the amplitude network of
// Section 3.1).  Pipeline per chunk of samples, all on the caller's stream:
//   1. k_enum_keys   writes the key of every connection in canonical order;
//   2. the network (FP64 or BF16 forward) gives log|psi| and phase of each x';
//   3. k_eloc_partial recomputes each (x, x') excitation, its Slater-Condon
//      element and the FP64 amplitude ratio, and sums them (Neumaier) per
//      block of connections; k_eloc_finish folds the blocks of a sample in a
//      fixed order.
// The samples' own amplitudes come from the same network in the same
// precision, so the ratio psi(x')/psi(x) is taken between like numbers.
#include <algorithm>
#include <cmath>
#include <vector>

#include "enumerate.hpp"
#include "model.hpp"

namespace nnqs {

constexpr int kConnPerBlock = 4096;            // connections handled by one block
constexpr int64_t kMaxChunkConnections = 1 << 24;
constexpr int64_t kMaxChunkConnectionsDedup = 1 << 27;  // many samples per chunk, so that x' are shared
constexpr int64_t kMaxChunkSamplesBf16 = 4096;  // samples whose key / value cache is kept at once

__global__ void __launch_bounds__(256) k_enum_keys(SysView S, const uint64_t *__restrict__ keys, int64_t m,
                                                   int64_t blocks_per_sample, uint64_t *__restrict__ out,
                                                   uint8_t *__restrict__ exc_out, float *__restrict__ loghx_out) {
    __shared__ WaveLds wl_all[4];
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveLds &wl = wl_all[wid];
    const int64_t C = S.C;
    const int64_t smp = blockIdx.x / blocks_per_sample;
    const int64_t c0 = (blockIdx.x % blocks_per_sample) * kConnPerBlock;
    if (smp >= m) return;
    Key x;
    x.lo = keys[2 * smp];
    x.hi = keys[2 * smp + 1];
    if (!sample_conserves(S, x)) return;  // left to the validator / NaN path
    build_lists(S, x, wl);
    const int64_t c1 = c0 + kConnPerBlock < C ? c0 + kConnPerBlock : C;
    for (int64_t c = c0 + wid * 64 + lane; c < c1; c += 256) {
        int i, j, a, b;
        decode_canonical(S, wl, c, i, j, a, b);
        const Key xp = apply_excitation(x, i, j, a, b);
        out[2 * (smp * C + c)] = xp.lo;
        out[2 * (smp * C + c) + 1] = xp.hi;
        if (loghx_out) {  // log|H_xx'| for the selection rules; the diagonal is always kept
            int sg;
            const double hv = c == 0 ? 0.0 : excitation_element(S, x, 0.0, i, j, a, b, &sg);
            loghx_out[smp * C + c] = c == 0 ? INFINITY : logf((float)fabs(hv));
        }
        if (exc_out) {  // sorted spin-orbital indices, 255 absent (screen input)
            uint8_t *e = exc_out + 4 * (smp * C + c);
            if (j == 255) {
                e[0] = (uint8_t)i;
                e[1] = 255;
                e[2] = (uint8_t)a;
                e[3] = 255;
            } else {
                e[0] = (uint8_t)(i < j ? i : j);
                e[1] = (uint8_t)(i < j ? j : i);
                e[2] = (uint8_t)(a < b ? a : b);
                e[3] = (uint8_t)(a < b ? b : a);
            }
        }
    }
}

// Selection of connections by a score against the sample's own log|psi|:
// keep e when score(e) >= sla[sample] - thr, where score is a float or double
// per-connection value (a screen prediction, or the first-pass log|psi(x')|)
// plus, optionally, log|H_xx'|.  The diagonal is always kept.  Two-pass
// deterministic compaction in canonical order.
constexpr int kSelBlock = 1024;

struct SelRule {
    const float *pf;   // per-connection score (float), or
    const double *pd;  // per-connection score (double)
    const float *lh;   // optional log|H_xx'| added to the score
    const double *sla; // the samples' own log|psi| (chunk-local)
    int64_t C;
    double thr;
};

__device__ __forceinline__ bool sel_keep(const SelRule &R, int64_t e) {
    const int64_t smp = e / R.C, cc = e - smp * R.C;
    if (cc == 0) return true;
    double v = R.pf ? (double)R.pf[e] : R.pd[e];
    if (R.lh) v += (double)R.lh[e];
    return v >= R.sla[smp] - R.thr;
}

__global__ void __launch_bounds__(256) k_sel_count(SelRule R, int64_t total, int32_t *__restrict__ cnt) {
    __shared__ int sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    int c = 0;
    for (int64_t e = b0 + threadIdx.x; e < b0 + kSelBlock && e < total; e += 256) c += sel_keep(R, e) ? 1 : 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

__global__ void k_sel_scan(int32_t *__restrict__ cnt, int nblocks, int64_t *__restrict__ total_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t run = 0;
    for (int b = 0; b < nblocks; b++) {
        const int v = cnt[b];
        cnt[b] = (int32_t)run;
        run += v;
    }
    *total_out = run;
}

// One wave walks its block's range in order; ballots keep canonical order.
// With `clear`, connections left out get log|psi| = -inf (they contribute
// zero) in xla / xph.
__global__ void __launch_bounds__(64) k_sel_write(SelRule R, int64_t total, const int32_t *__restrict__ off,
                                                  int32_t *__restrict__ sel, const uint64_t *__restrict__ xkeys,
                                                  uint64_t *__restrict__ ckeys, bool clear,
                                                  double *__restrict__ xla, double *__restrict__ xph) {
    const int lane = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    int64_t pos = off[blockIdx.x];
    for (int64_t e0 = b0; e0 < b0 + kSelBlock && e0 < total; e0 += 64) {
        const int64_t e = e0 + lane;
        bool keep = false;
        if (e < total && e < b0 + kSelBlock) {
            keep = sel_keep(R, e);
            if (clear) {
                xla[e] = -INFINITY;
                xph[e] = 0.0;
            }
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int64_t p = pos + __popcll(m & ((1ull << lane) - 1ull));
            sel[p] = (int32_t)e;
            ckeys[2 * p] = xkeys[2 * e];
            ckeys[2 * p + 1] = xkeys[2 * e + 1];
        }
        pos += __popcll(m);
    }
}

__global__ void k_scatter_sel(const int32_t *__restrict__ sel, const int64_t *__restrict__ nsel,
                              const double *__restrict__ cla, const double *__restrict__ cph, double *__restrict__ xla,
                              double *__restrict__ xph) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *nsel) return;
    xla[sel[k]] = cla[k];
    xph[sel[k]] = cph[k];
}

// ------------------------------------------------ prefix classes (BF16)
// Class of a connection x' of sample x for the prefix-reusing BF16 forward:
// min(3, s0 / 16) with s0 the first sequence position whose token differs
// (position s holds orbital K-1-s, so s0 = K-1-(highest differing orbital);
// the diagonal has none and gets min(3, K / 16)).
__device__ __forceinline__ int conn_class(int K, const uint64_t *x, const uint64_t *xp) {
    const uint64_t d0 = x[0] ^ xp[0], d1 = x[1] ^ xp[1];
    const int p = d1 ? 127 - __clzll(d1) : (d0 ? 63 - __clzll(d0) : -2);
    const int s0 = K - 1 - (p >> 1);
    return s0 >= 48 ? 3 : s0 >> 4;
}

struct ClsArgs {
    SelRule R;                  // keep rule, used when `rule`
    bool rule;
    const uint8_t *mask;        // optional: keep only connections with mask[e] != 0
    const uint64_t *keys;       // chunk samples [m][2]
    const uint64_t *xkeys;      // chunk connections [m*C][2]
    int64_t total;
    int K;
};

__device__ __forceinline__ bool cls_keep(const ClsArgs &a, int64_t e) {
    return (!a.rule || sel_keep(a.R, e)) && (!a.mask || a.mask[e]);
}

// ------------------------------------------------ distinct x' (dedup)
// First changed sequence position of x' against its sample x (the sample
// itself: K - 1, its last row).
__device__ __forceinline__ int conn_s0(int K, const uint64_t *x, uint64_t lo, uint64_t hi) {
    const uint64_t d0 = x[0] ^ lo, d1 = x[1] ^ hi;
    if (!d0 && !d1) return K - 1;
    const int p = d1 ? 127 - __clzll(d1) : 63 - __clzll(d0);
    return K - 1 - (p >> 1);
}

// Keys of the n kept connections (list sel) for the sort, padded to P with
// all-ones keys behind every real one.
__global__ void k_dd_gather(const uint64_t *__restrict__ xkeys, const int32_t *__restrict__ sel, int64_t n,
                            int64_t P, uint64_t *__restrict__ sk, uint32_t *__restrict__ si,
                            unsigned long long *__restrict__ best) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    if (i < n) {
        const int64_t e = sel[i];
        sk[2 * i] = xkeys[2 * e];
        sk[2 * i + 1] = xkeys[2 * e + 1];
        si[i] = (uint32_t)i;
        best[i] = 0ull;
    } else {
        sk[2 * i] = ~0ull;
        sk[2 * i + 1] = ~0ull;
        si[i] = 0xFFFFFFFFu;
    }
}

// Sorted position p < n: the head of its run of equal keys, and at the head
// the largest score (s0 << 32) | (2^32 - 1 - e) of the run's members: the
// latest first change, then the smallest connection index (max is
// independent of the order of the atomic updates).  The positions j <= p
// whose key equals p's are exactly those from the head on, so the head is
// found by doubling steps back from p and then bisecting: O(log L) loads
// for a run of length L (an x' shared by many samples makes L large).
__global__ void k_dd_score(const uint64_t *__restrict__ sk, const uint32_t *__restrict__ si, int64_t n,
                           const int32_t *__restrict__ sel, const uint64_t *__restrict__ keys, int64_t C, int K,
                           int32_t *__restrict__ head, unsigned long long *__restrict__ best) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint64_t lo = sk[2 * p], hi = sk[2 * p + 1];
    auto same = [&](int64_t j) { return sk[2 * j] == lo && sk[2 * j + 1] == hi; };
    int64_t in = p, out = -1;  // same(in) holds; out < in is outside the run, or -1
    for (int64_t step = 1; p - step >= 0; step <<= 1) {
        if (!same(p - step)) {
            out = p - step;
            break;
        }
        in = p - step;
    }
    while (in - out > 1) {
        const int64_t mid = out + (in - out) / 2;
        if (same(mid)) in = mid;
        else out = mid;
    }
    const int64_t h = in;
    head[p] = (int32_t)h;
    const int64_t e = sel[si[p]];
    const int s0 = conn_s0(K, keys + 2 * (e / C), lo, hi);
    atomicMax(best + h, ((unsigned long long)s0 << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)e));
}

// Representative of every kept connection (rep[i] for list position i), and
// the mask of the representatives over the chunk.
__global__ void k_dd_mark(const uint32_t *__restrict__ si, const int32_t *__restrict__ sel, int64_t n,
                          const int32_t *__restrict__ head, const unsigned long long *__restrict__ best,
                          int32_t *__restrict__ rep, uint8_t *__restrict__ repmask) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = si[p];
    const int32_t e = sel[i];
    const int32_t r = (int32_t)(0xFFFFFFFFu - (uint32_t)(best[head[p]] & 0xFFFFFFFFull));
    rep[i] = r;
    if (e == r) repmask[e] = 1;
}

// Copies each representative's log|psi| and phase to the other members of
// its run (representatives are only read here).
__global__ void k_dd_scatter(const int32_t *__restrict__ sel, const int32_t *__restrict__ rep, int64_t n,
                             double *__restrict__ xla, double *__restrict__ xph) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t e = sel[i], r = rep[i];
    if (e != r) {
        xla[e] = xla[r];
        xph[e] = xph[r];
    }
}

// Marks the representative of every kept connection that the refinement
// rule selects (all writers store 1).
__global__ void k_dd_refmark(const int32_t *__restrict__ sel, const int32_t *__restrict__ rep, int64_t n, SelRule R,
                             uint8_t *__restrict__ refmask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (sel_keep(R, sel[i])) refmask[rep[i]] = 1;
}

__global__ void k_dd_zero_u32(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Kept connections per class in each block of kSelBlock connections.
__global__ void __launch_bounds__(256) k_cls_count(ClsArgs a, int32_t *__restrict__ cnt) {
    __shared__ int sh[4][256];
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    int c[4] = {0, 0, 0, 0};
    for (int64_t e = b0 + threadIdx.x; e < b0 + kSelBlock && e < a.total; e += 256) {
        if (!cls_keep(a, e)) continue;
        const int64_t smp = e / a.R.C;
        const int k = conn_class(a.K, a.keys + 2 * smp, a.xkeys + 2 * e);
        c[0] += k == 0;
        c[1] += k == 1;
        c[2] += k == 2;
        c[3] += k == 3;
    }
    for (int k = 0; k < 4; k++) sh[k][threadIdx.x] = c[k];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) cnt[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Turns the per-block counts into absolute list positions (classes stored
// one after another), writes hdr = {count[4], offset[4]} and adds the kept
// total and the per-class counts to evaluated[0..4].  One block; each thread
// scans a contiguous run of blocks.
__global__ void __launch_bounds__(256) k_cls_scan(int32_t *__restrict__ cnt, int nblocks, int64_t *__restrict__ hdr,
                                                  int64_t *__restrict__ evaluated) {
    __shared__ int64_t part[4][257];
    const int per = (nblocks + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(nblocks, b0 + per);
    int64_t run[4] = {0, 0, 0, 0};
    for (int b = b0; b < b1; b++)
        for (int k = 0; k < 4; k++) run[k] += cnt[b * 4 + k];
    for (int k = 0; k < 4; k++) part[k][threadIdx.x + 1] = run[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        part[k][0] = 0;
        for (int t = 1; t <= 256; t++) part[k][t] += part[k][t - 1];
    }
    __syncthreads();
    int64_t off[4], tot[4];
    int64_t acc = 0;
    for (int k = 0; k < 4; k++) {
        tot[k] = part[k][256];
        off[k] = acc;
        acc += tot[k];
    }
    int64_t pos[4];
    for (int k = 0; k < 4; k++) pos[k] = off[k] + part[k][threadIdx.x];
    for (int b = b0; b < b1; b++)
        for (int k = 0; k < 4; k++) {
            const int v = cnt[b * 4 + k];
            cnt[b * 4 + k] = (int32_t)pos[k];
            pos[k] += v;
        }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; k++) {
            hdr[k] = tot[k];
            hdr[4 + k] = off[k];
            if (evaluated) evaluated[1 + k] += tot[k];
        }
        if (evaluated) evaluated[0] += acc;
    }
}

// One wave walks its block's connections in order and appends the kept ones
// to their class list (ballots keep canonical order within a class).  With
// `clear`, connections left out get log|psi| = -inf (they contribute zero).
__global__ void __launch_bounds__(64) k_cls_write(ClsArgs a, const int32_t *__restrict__ pos0,
                                                  int32_t *__restrict__ list, bool clear, double *__restrict__ xla,
                                                  double *__restrict__ xph) {
    const int lane = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    int64_t pos[4];
    for (int k = 0; k < 4; k++) pos[k] = pos0[blockIdx.x * 4 + k];
    for (int64_t e0 = b0; e0 < b0 + kSelBlock && e0 < a.total; e0 += 64) {
        const int64_t e = e0 + lane;
        int k = -1;
        if (e < a.total && e < b0 + kSelBlock) {
            if (cls_keep(a, e)) {
                const int64_t smp = e / a.R.C;
                k = conn_class(a.K, a.keys + 2 * smp, a.xkeys + 2 * e);
            } else if (clear) {
                xla[e] = -INFINITY;
                xph[e] = 0.0;
            }
        }
        for (int q = 0; q < 4; q++) {
            const uint64_t m = __ballot(k == q);
            if (k == q) list[pos[q] + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)e;
            pos[q] += __popcll(m);
        }
    }
}

// The rows and attended keys the kept connections need at the least (rows
// s0 .. K-1 from the first changed position; the diagonal: its last row),
// summed into req[0], req[1] (integers: the totals do not depend on order).
__global__ void __launch_bounds__(256) k_req_work(ClsArgs a, unsigned long long *__restrict__ req) {
    __shared__ unsigned long long sh[2][256];
    unsigned long long rows = 0, keys = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.total; e += (int64_t)gridDim.x * blockDim.x) {
        if (!cls_keep(a, e)) continue;
        const uint64_t *x = a.keys + 2 * (e / a.R.C), *xp = a.xkeys + 2 * e;
        const uint64_t d0 = x[0] ^ xp[0], d1 = x[1] ^ xp[1];
        const int p = d1 ? 127 - __clzll(d1) : (d0 ? 63 - __clzll(d0) : 0);
        const int s0 = (d0 | d1) ? a.K - 1 - (p >> 1) : a.K - 1;
        rows += (unsigned long long)(a.K - s0);
        keys += (unsigned long long)(a.K * (a.K + 1) / 2 - s0 * (s0 + 1) / 2);
    }
    sh[0][threadIdx.x] = rows;
    sh[1][threadIdx.x] = keys;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(req, sh[0][0]);
        atomicAdd(req + 1, sh[1][0]);
    }
}

__global__ void k_zero_i64(int64_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_eloc_partial(SysView S, const uint64_t *__restrict__ keys,
                                                      const double *__restrict__ sla,
                                                      const double *__restrict__ sph, int64_t m,
                                                      int64_t blocks_per_sample, const double *__restrict__ xla,
                                                      const double *__restrict__ xph,
                                                      double *__restrict__ partials) {
    __shared__ WaveLds wl_all[4];
    __shared__ double red[256][4];
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveLds &wl = wl_all[wid];
    const int64_t C = S.C;
    const int64_t smp = blockIdx.x / blocks_per_sample;
    const int64_t blk = blockIdx.x % blocks_per_sample;
    const int64_t c0 = blk * kConnPerBlock;
    if (smp >= m) return;
    Key x;
    x.lo = keys[2 * smp];
    x.hi = keys[2 * smp + 1];
    const bool valid = sample_conserves(S, x);
    NSum re{0.0, 0.0}, im{0.0, 0.0};
    if (valid) {
        build_lists(S, x, wl);
        const double diag = wave_diag(S, x, wl);
        const double la = sla[smp], ph = sph[smp];
        const int64_t c1 = c0 + kConnPerBlock < C ? c0 + kConnPerBlock : C;
        for (int64_t c = c0 + wid * 64 + lane; c < c1; c += 256) {
            int i, j, a, b;
            decode_canonical(S, wl, c, i, j, a, b);
            int sg;
            const double hv = excitation_element(S, x, diag, i, j, a, b, &sg);
            const double r = exp(xla[smp * C + c] - la);
            double sn, cs;
            sincos(xph[smp * C + c] - ph, &sn, &cs);
            re.add(hv * r * cs);
            im.add(hv * r * sn);
        }
    }
    red[threadIdx.x][0] = re.s;
    red[threadIdx.x][1] = re.c;
    red[threadIdx.x][2] = im.s;
    red[threadIdx.x][3] = im.c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 2; q++) {
                double s = red[threadIdx.x][2 * q], c = red[threadIdx.x][2 * q + 1];
                nsum_merge(s, c, red[threadIdx.x + w][2 * q], red[threadIdx.x + w][2 * q + 1]);
                red[threadIdx.x][2 * q] = s;
                red[threadIdx.x][2 * q + 1] = c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[(smp * blocks_per_sample + blk) * 4 + threadIdx.x] = valid ? red[0][threadIdx.x] : NAN;
}

__global__ void k_eloc_finish(const double *__restrict__ partials, int64_t m, int64_t blocks_per_sample,
                              double *__restrict__ eloc) {
    const int64_t smp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (smp >= m) return;
    double rs = 0.0, rc = 0.0, is = 0.0, ic = 0.0;
    for (int64_t b = 0; b < blocks_per_sample; b++) {
        const double *p = partials + (smp * blocks_per_sample + b) * 4;
        nsum_merge(rs, rc, p[0], p[1]);
        nsum_merge(is, ic, p[2], p[3]);
    }
    eloc[2 * smp] = rs + rc;
    eloc[2 * smp + 1] = is + ic;
}

__global__ void k_check_samples(SysView S, const uint64_t *__restrict__ keys, int64_t n, int *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Key x;
    x.lo = keys[2 * i];
    x.hi = keys[2 * i + 1];
    if (!sample_conserves(S, x)) set_status(status, NNQS_ECONSERVE);
}

__global__ void k_zero_status(int *p) { *p = 0; }

static nnqs_status grow(void **p, size_t bytes) {
    hipFree(*p);
    *p = nullptr;
    if (hipMalloc(p, bytes) != hipSuccess) return fail(NNQS_ENOMEM, "scratch allocation of %zu bytes failed", bytes);
    return NNQS_OK;
}

void eloc_model_free(nnqs_model *m) {
    hipFree(m->d_xkeys);
    hipFree(m->d_xla);
    hipFree(m->d_xph);
    hipFree(m->d_sla);
    hipFree(m->d_sph);
    hipFree(m->d_partials);
    hipFree(m->d_xexc);
    hipFree(m->d_pred);
    hipFree(m->d_loghx);
    m->d_loghx = nullptr;
    hipFree(m->d_sel);
    hipFree(m->d_blockcnt);
    hipFree(m->d_ckeys);
    hipFree(m->d_cla);
    hipFree(m->d_cph);
    hipFree(m->d_nsel);
    hipFree(m->d_kv);
    hipFree(m->d_pre);
    hipFree(m->d_csla);
    hipFree(m->d_hdr);
    hipFree(m->d_kv64);
    hipFree(m->d_pre64);
    hipFree(m->d_rag);
    hipFree(m->d_ddk);
    hipFree(m->d_ddi);
    hipFree(m->d_ddhead);
    hipFree(m->d_ddrep);
    hipFree(m->d_sel2);
    hipFree(m->d_ddbest);
    hipFree(m->d_repmask);
    hipFree(m->d_refmask);
    m->d_ddk = nullptr;
    m->d_ddi = nullptr;
    m->d_ddhead = m->d_ddrep = m->d_sel2 = nullptr;
    m->d_ddbest = nullptr;
    m->d_repmask = m->d_refmask = nullptr;
    m->ddcap = m->maskcap = 0;
    m->d_kv64 = m->d_pre64 = nullptr;
    m->d_rag = nullptr;
    m->kv64cap = 0;
    m->ragcap = 0;
    m->d_kv = nullptr;
    m->d_pre = m->d_csla = nullptr;
    m->d_hdr = nullptr;
    m->kvcap = 0;
    m->d_xexc = nullptr;
    m->d_pred = nullptr;
    m->d_sel = m->d_blockcnt = nullptr;
    m->d_ckeys = nullptr;
    m->d_cla = m->d_cph = nullptr;
    m->d_nsel = nullptr;
    m->d_xkeys = nullptr;
    m->d_xla = m->d_xph = m->d_sla = m->d_sph = m->d_partials = nullptr;
    m->xcap = m->scap = 0;
}

// Compact the connections of one chunk that pass rule R, evaluate them with
// the network in `precision` and scatter the results into xla / xph.  With
// `clear`, connections that fail the rule get log|psi| = -inf.  Returns the
// number evaluated (the call synchronises the stream to read it).
static nnqs_status select_and_evaluate(nnqs_model *model, const SelRule &R, int64_t total, bool clear,
                                       int32_t precision, hipStream_t st, int64_t *evaluated) {
    const int nb = (int)((total + kSelBlock - 1) / kSelBlock);
    hipLaunchKernelGGL(k_sel_count, dim3(nb), dim3(256), 0, st, R, total, model->d_blockcnt);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1), 0, st, model->d_blockcnt, nb, model->d_nsel);
    hipLaunchKernelGGL(k_sel_write, dim3(nb), dim3(64), 0, st, R, total, model->d_blockcnt, model->d_sel,
                       model->d_xkeys, model->d_ckeys, clear, model->d_xla, model->d_xph);
    NNQS_HIP_CHECK(hipGetLastError());
    int64_t nsel = 0;
    NNQS_HIP_CHECK(hipMemcpyAsync(&nsel, model->d_nsel, 8, hipMemcpyDeviceToHost, st));
    NNQS_HIP_CHECK(hipStreamSynchronize(st));
    if (nsel > 0) {
        nnqs_status s1 = enqueue_logpsi(model, model->d_ckeys, nsel, precision, model->d_cla, model->d_cph, st);
        if (s1 != NNQS_OK) return s1;
        hipLaunchKernelGGL(k_scatter_sel, dim3((unsigned)((nsel + 255) / 256)), dim3(256), 0, st, model->d_sel,
                           model->d_nsel, model->d_cla, model->d_cph, model->d_xla, model->d_xph);
        NNQS_HIP_CHECK(hipGetLastError());
    }
    *evaluated = nsel;
    return NNQS_OK;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" nnqs_status nnqs_eloc_model(const nnqs_system *sys, nnqs_model *model, nnqs_screen *screen,
                                       const nnqs_eloc_opts *opts, int32_t precision, const uint64_t *keys,
                                       const uint32_t *counts, int64_t n, double *eloc, double *energy,
                                       nnqs_stats *stats, uint32_t flags, void *stream) {
    clear_error();
    if (!sys || !model || !keys || !eloc) return fail(NNQS_EINVAL, "null pointer argument");
    if (energy && !counts) return fail(NNQS_EINVAL, "energy requested without counts");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if (model->desc.n_orb != sys->view.K || model->desc.n_up != sys->view.n_up || model->desc.n_dn != sys->view.n_dn)
        return fail(NNQS_EINVAL, "model and system disagree on orbitals or electron numbers");
    if (precision != NNQS_FP64 && precision != NNQS_BF16 && precision != NNQS_FP8)
        return fail(NNQS_EUNSUPPORTED, "unknown precision");
    if (precision != NNQS_FP64 && !model->bf16_ok) return fail(NNQS_EUNSUPPORTED, "model shape has no BF16 / FP8 path");
    nnqs_eloc_opts o{12.0, NNQS_SKIP_RATIO, 0.0, NNQS_BF16, 0};
    if (opts) o = *opts;
    if (o.screen_precision != NNQS_BF16 && o.screen_precision != NNQS_FP8)
        return fail(NNQS_EINVAL, "screen precision must be NNQS_BF16 or NNQS_FP8");
    if (screen && !(o.skip_nats > 0.0)) return fail(NNQS_EINVAL, "skip_nats must be positive");
    if (o.skip_rule != NNQS_SKIP_RATIO && o.skip_rule != NNQS_SKIP_CONTRIBUTION)
        return fail(NNQS_EINVAL, "unknown skip rule %d", o.skip_rule);
    if (!(o.refine_nats >= 0.0)) return fail(NNQS_EINVAL, "refine_nats must be >= 0");
    const bool refine = o.refine_nats > 0.0 && precision != NNQS_FP64;
    const bool need_lh = refine || (screen && o.skip_rule == NNQS_SKIP_CONTRIBUTION);
    hipStream_t st = as_stream(stream);
    if (flags & NNQS_VALIDATE) {
        hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(1), 0, st, sys->d_status);
        hipLaunchKernelGGL(k_check_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sys->view, keys, n,
                           sys->d_status);
        int h = 0;
        NNQS_HIP_CHECK(hipMemcpyAsync(&h, sys->d_status, sizeof(int), hipMemcpyDeviceToHost, st));
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        if (h) return fail(h, "a sample violates the particle numbers");
    }
    const int64_t C = sys->view.C;
    const bool bf16 = precision == NNQS_BF16 || precision == NNQS_FP8;  // prefix-reusing MFMA paths
    const bool fp8 = precision == NNQS_FP8;
    const bool dedup = bf16 && o.dedup != 0;  // each distinct x' of a chunk evaluated once
    int64_t chunk = (dedup ? kMaxChunkConnectionsDedup : kMaxChunkConnections) / C;
    if (chunk < 1) chunk = 1;
    if (bf16 && chunk > kMaxChunkSamplesBf16) chunk = kMaxChunkSamplesBf16;  // bounds the key / value cache
    if (chunk > n) chunk = n;
    const int64_t bps = (C + kConnPerBlock - 1) / kConnPerBlock;
    if (model->xcap < chunk * C) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));  // scratch may be in use by earlier work on this stream
        const size_t cc = (size_t)chunk * C;
        nnqs_status s1 = grow(reinterpret_cast<void **>(&model->d_xkeys), cc * 16);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_xla), cc * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_xph), cc * 8);
        if (s1 == NNQS_OK)
            s1 = grow(reinterpret_cast<void **>(&model->d_partials),
                      std::max<size_t>((size_t)chunk * bps * 4, kPartialBlocks * 8) * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_xexc), cc * 4);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_pred), cc * 4);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_loghx), cc * 4);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_sel), cc * 4);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_blockcnt), (cc / kSelBlock + 2) * 16);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_ckeys), cc * 16);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_cla), cc * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_cph), cc * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_nsel), 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_hdr), 32 * 8);
        if (s1 != NNQS_OK) {
            eloc_model_free(model);
            return s1;
        }
        model->xcap = chunk * C;
    }
    if (bf16 && model->kvcap < chunk) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        nnqs_status s1 =
            grow(reinterpret_cast<void **>(&model->d_kv), (size_t)chunk * bf16_cache_elems(model) * sizeof(__bf16));
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_pre), (size_t)chunk * 4 * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_csla), (size_t)chunk * 8);
        if (s1 != NNQS_OK) {
            eloc_model_free(model);
            return s1;
        }
        model->kvcap = chunk;
    }
    const bool refine64 = refine && bf16;  // FP64 refinement with the samples' FP64 prefix cache
    if (refine64 && model->kv64cap < chunk) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        nnqs_status s1 =
            grow(reinterpret_cast<void **>(&model->d_kv64), (size_t)chunk * f64_cache_doubles(model) * sizeof(double));
        if (s1 == NNQS_OK)
            s1 = grow(reinterpret_cast<void **>(&model->d_pre64),
                      (size_t)chunk * (sys->view.K + 1) * sizeof(double));
        if (s1 != NNQS_OK) {
            eloc_model_free(model);
            return s1;
        }
        model->kv64cap = chunk;
    }
    if (model->scap < n) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        nnqs_status s1 = grow(reinterpret_cast<void **>(&model->d_sla), (size_t)n * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_sph), (size_t)n * 8);
        if (s1 != NNQS_OK) {
            eloc_model_free(model);
            return s1;
        }
        model->scap = n;
    }
    // the samples' own amplitudes: in the top precision of the evaluation
    // (with FP64 refinement of the BF16 / FP8 path, chunk by chunk below,
    // together with their FP64 prefix cache)
    nnqs_status s1 = NNQS_OK;
    if (!refine64) {
        s1 = enqueue_logpsi(model, keys, n, refine ? NNQS_FP64 : precision, model->d_sla, model->d_sph, st);
        if (s1 != NNQS_OK) return s1;
    }
    int64_t evaluated = 0, refined = 0;
    int64_t *d_evalcnt = model->d_hdr + 8;   // [8, 15): forward's lists (total, classes), required rows / keys
    int64_t *d_keptcnt = model->d_hdr + 24;  // [24, 29): kept connections before dedup (total, classes)
    if (bf16) {
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, d_evalcnt, 7);
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, d_keptcnt, 5);
    }
    int64_t n_kept = 0;  // dedup: kept connections of the current chunk
    for (int64_t s0 = 0; s0 < n; s0 += chunk) {
        const int64_t m = n - s0 < chunk ? n - s0 : chunk;
        const int64_t total = m * C;
        const unsigned grid = (unsigned)(m * bps);
        hipLaunchKernelGGL(k_enum_keys, dim3(grid), dim3(256), 0, st, sys->view, keys + 2 * s0, m, bps,
                           model->d_xkeys, screen ? model->d_xexc : (uint8_t *)nullptr,
                           need_lh ? model->d_loghx : (float *)nullptr);
        if (refine64) {
            s1 = enqueue_logpsi_f64(model, keys + 2 * s0, m, model->d_sla + s0, model->d_sph + s0, st, -1, nullptr,
                                    model->d_kv64, model->d_pre64);
            if (s1 != NNQS_OK) return s1;
        }
        if (bf16) {
            // the chunk's samples once through the forward, keeping their keys,
            // values and log-probability prefix sums; then every kept x'
            // evaluates only the row blocks from its first changed position on
            s1 = enqueue_bf16_cached(model, keys + 2 * s0, m, model->d_csla, model->d_kv, model->d_pre, st, fp8);
            if (s1 != NNQS_OK) return s1;
            if (screen) {
                s1 = screen_infer(screen, model->d_xkeys, model->d_xexc, total, model->d_pred, st, o.screen_precision == NNQS_FP8);
                if (s1 != NNQS_OK) return s1;
            }
            ClsArgs ca{};
            ca.R = SelRule{screen ? model->d_pred : nullptr, nullptr,
                           screen && o.skip_rule == NNQS_SKIP_CONTRIBUTION ? model->d_loghx : nullptr,
                           model->d_sla + s0, C, o.skip_nats};
            ca.rule = screen != nullptr;
            ca.keys = keys + 2 * s0;
            ca.xkeys = model->d_xkeys;
            ca.total = total;
            ca.K = sys->view.K;
            const int nb = (int)((total + kSelBlock - 1) / kSelBlock);
            hipLaunchKernelGGL(k_cls_count, dim3(nb), dim3(256), 0, st, ca, model->d_blockcnt);
            hipLaunchKernelGGL(k_cls_scan, dim3(1), dim3(256), 0, st, model->d_blockcnt, nb, model->d_hdr,
                               dedup ? d_keptcnt : d_evalcnt);
            hipLaunchKernelGGL(k_cls_write, dim3(nb), dim3(64), 0, st, ca, model->d_blockcnt, model->d_sel,
                               screen != nullptr, model->d_xla, model->d_xph);
            NNQS_HIP_CHECK(hipGetLastError());
            const int32_t *flist = model->d_sel;  // the list the forward runs
            if (dedup) {
                // the kept connections sorted by key; each run of equal x' is
                // evaluated once, from its representative's sample
                int64_t kh[4];
                NNQS_HIP_CHECK(hipMemcpyAsync(kh, model->d_hdr, sizeof(kh), hipMemcpyDeviceToHost, st));
                NNQS_HIP_CHECK(hipStreamSynchronize(st));
                n_kept = kh[0] + kh[1] + kh[2] + kh[3];
                int64_t P = 2;
                while (P < n_kept) P <<= 1;
                if (model->ddcap < P || model->maskcap < total) {
                    const size_t pc = (size_t)std::max<int64_t>(P, model->ddcap);
                    const size_t mc = (size_t)std::max<int64_t>(total, model->maskcap);
                    s1 = grow(reinterpret_cast<void **>(&model->d_ddk), pc * 16);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_ddi), pc * 4);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_ddhead), pc * 4);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_ddrep), pc * 4);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_sel2), pc * 4);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_ddbest), pc * 8);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_repmask), (mc + 3) / 4 * 4);
                    if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_refmask), (mc + 3) / 4 * 4);
                    if (s1 != NNQS_OK) {
                        eloc_model_free(model);
                        return s1;
                    }
                    model->ddcap = (int64_t)pc;
                    model->maskcap = (int64_t)mc;
                }
                const int64_t mw = (total + 3) / 4;
                hipLaunchKernelGGL(k_dd_zero_u32, dim3((unsigned)((mw + 255) / 256)), dim3(256), 0, st,
                                   reinterpret_cast<uint32_t *>(model->d_repmask), mw);
                hipLaunchKernelGGL(k_dd_gather, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, model->d_xkeys,
                                   model->d_sel, n_kept, P, model->d_ddk, model->d_ddi, model->d_ddbest);
                bitonic_sort128(model->d_ddk, model->d_ddi, P, st);
                const unsigned gk = (unsigned)((n_kept + 255) / 256);
                hipLaunchKernelGGL(k_dd_score, dim3(gk), dim3(256), 0, st, model->d_ddk, model->d_ddi, n_kept,
                                   model->d_sel, keys + 2 * s0, C, sys->view.K, model->d_ddhead, model->d_ddbest);
                hipLaunchKernelGGL(k_dd_mark, dim3(gk), dim3(256), 0, st, model->d_ddi, model->d_sel, n_kept,
                                   model->d_ddhead, model->d_ddbest, model->d_ddrep, model->d_repmask);
                ClsArgs cr = ca;
                cr.mask = model->d_repmask;
                hipLaunchKernelGGL(k_cls_count, dim3(nb), dim3(256), 0, st, cr, model->d_blockcnt);
                hipLaunchKernelGGL(k_cls_scan, dim3(1), dim3(256), 0, st, model->d_blockcnt, nb, model->d_hdr,
                                   d_evalcnt);
                hipLaunchKernelGGL(k_cls_write, dim3(nb), dim3(64), 0, st, cr, model->d_blockcnt, model->d_sel2,
                                   false, (double *)nullptr, (double *)nullptr);
                if (stats)
                    hipLaunchKernelGGL(k_req_work, dim3(1024), dim3(256), 0, st, cr,
                                       reinterpret_cast<unsigned long long *>(d_evalcnt + 5));
                NNQS_HIP_CHECK(hipGetLastError());
                flist = model->d_sel2;
            } else if (stats) {
                hipLaunchKernelGGL(k_req_work, dim3(1024), dim3(256), 0, st, ca,
                                   reinterpret_cast<unsigned long long *>(d_evalcnt + 5));
                NNQS_HIP_CHECK(hipGetLastError());
            }
            s1 = enqueue_bf16_list(model, model->d_xkeys, C, flist, model->d_hdr, total, model->d_kv,
                                   model->d_pre, model->d_xla, model->d_xph, st, fp8);
            if (s1 != NNQS_OK) return s1;
            if (dedup) {
                hipLaunchKernelGGL(k_dd_scatter, dim3((unsigned)((n_kept + 255) / 256)), dim3(256), 0, st,
                                   model->d_sel, model->d_ddrep, n_kept, model->d_xla, model->d_xph);
                NNQS_HIP_CHECK(hipGetLastError());
            }
        } else if (!screen) {
            s1 = enqueue_logpsi(model, model->d_xkeys, total, precision, model->d_xla, model->d_xph, st);
            if (s1 != NNQS_OK) return s1;
            evaluated += total;
        } else {
            s1 = screen_infer(screen, model->d_xkeys, model->d_xexc, total, model->d_pred, st, o.screen_precision == NNQS_FP8);
            if (s1 != NNQS_OK) return s1;
            SelRule R{model->d_pred, nullptr, o.skip_rule == NNQS_SKIP_CONTRIBUTION ? model->d_loghx : nullptr,
                      model->d_sla + s0, C, o.skip_nats};
            int64_t k = 0;
            s1 = select_and_evaluate(model, R, total, true, precision, st, &k);
            if (s1 != NNQS_OK) return s1;
            evaluated += k;
        }
        if (refine64) {
            // FP64 for every connection whose first-pass contribution is not
            // negligible, each from its first changed position on, from the
            // samples' FP64 cache
            ClsArgs ra{};
            ra.R = SelRule{nullptr, model->d_xla, model->d_loghx, model->d_sla + s0, C, o.refine_nats};
            ra.rule = true;
            ra.keys = keys + 2 * s0;
            ra.xkeys = model->d_xkeys;
            ra.total = total;
            ra.K = sys->view.K;
            int32_t *rlist = model->d_sel;
            if (dedup) {  // refine a run's representative when any member qualifies
                const int64_t mw = (total + 3) / 4;
                hipLaunchKernelGGL(k_dd_zero_u32, dim3((unsigned)((mw + 255) / 256)), dim3(256), 0, st,
                                   reinterpret_cast<uint32_t *>(model->d_refmask), mw);
                hipLaunchKernelGGL(k_dd_refmark, dim3((unsigned)((n_kept + 255) / 256)), dim3(256), 0, st,
                                   model->d_sel, model->d_ddrep, n_kept, ra.R, model->d_refmask);
                ra.rule = false;
                ra.mask = model->d_refmask;
                rlist = model->d_sel2;  // the first list stays for the copies below
            }
            const int nb = (int)((total + kSelBlock - 1) / kSelBlock);
            int64_t *d_rhdr = model->d_hdr + 16;
            hipLaunchKernelGGL(k_cls_count, dim3(nb), dim3(256), 0, st, ra, model->d_blockcnt);
            hipLaunchKernelGGL(k_cls_scan, dim3(1), dim3(256), 0, st, model->d_blockcnt, nb, d_rhdr,
                               (int64_t *)nullptr);
            hipLaunchKernelGGL(k_cls_write, dim3(nb), dim3(64), 0, st, ra, model->d_blockcnt, rlist, false,
                               (double *)nullptr, (double *)nullptr);
            NNQS_HIP_CHECK(hipGetLastError());
            int64_t rh[8];
            NNQS_HIP_CHECK(hipMemcpyAsync(rh, d_rhdr, sizeof(rh), hipMemcpyDeviceToHost, st));
            NNQS_HIP_CHECK(hipStreamSynchronize(st));
            const int64_t nref = rh[0] + rh[1] + rh[2] + rh[3];
            refined += nref;
            s1 = enqueue_f64_list(model, model->d_xkeys, C, rlist, nref, keys + 2 * s0, model->d_kv64,
                                  model->d_pre64, model->d_xla, model->d_xph, st);
            if (s1 != NNQS_OK) return s1;
            if (dedup) {
                hipLaunchKernelGGL(k_dd_scatter, dim3((unsigned)((n_kept + 255) / 256)), dim3(256), 0, st,
                                   model->d_sel, model->d_ddrep, n_kept, model->d_xla, model->d_xph);
                NNQS_HIP_CHECK(hipGetLastError());
            }
        } else if (refine) {  // FP64 for every connection whose first-pass contribution is not negligible
            SelRule R{nullptr, model->d_xla, model->d_loghx, model->d_sla + s0, C, o.refine_nats};
            int64_t k = 0;
            s1 = select_and_evaluate(model, R, total, false, NNQS_FP64, st, &k);
            if (s1 != NNQS_OK) return s1;
            refined += k;
        }
        hipLaunchKernelGGL(k_eloc_partial, dim3(grid), dim3(256), 0, st, sys->view, keys + 2 * s0,
                           model->d_sla + s0, model->d_sph + s0, m, bps, model->d_xla, model->d_xph,
                           model->d_partials);
        hipLaunchKernelGGL(k_eloc_finish, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, model->d_partials, m,
                           bps, eloc + 2 * s0);
        NNQS_HIP_CHECK(hipGetLastError());
    }
    if (energy) {
        s1 = enqueue_energy_partials(model->d_partials, counts, eloc, n, energy, st);
        if (s1 != NNQS_OK) return s1;
    }
    if (stats) {
        int64_t ev[7] = {0, 0, 0, 0, 0, 0, 0}, kept = 0;
        if (bf16) NNQS_HIP_CHECK(hipMemcpyAsync(ev, d_evalcnt, sizeof(ev), hipMemcpyDeviceToHost, st));
        if (dedup) NNQS_HIP_CHECK(hipMemcpyAsync(&kept, d_keptcnt, sizeof(kept), hipMemcpyDeviceToHost, st));
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        if (bf16) evaluated = dedup ? kept : ev[0];
        for (int k = 0; k < 4; k++) stats->evaluated_class[k] = ev[1 + k];
        stats->evaluated_rows = ev[5];
        stats->evaluated_keys = ev[6];
        stats->evaluated_distinct = bf16 ? ev[0] : evaluated;
        stats->connections = n * C;
        stats->evaluated = evaluated;
        stats->refined = refined;
    }
    return NNQS_OK;
}

// ------------------------------------------------ batched transformer mode
// Full local energies of many systems (uneven N, electron and sample
// counts), the network in BF16: every item's connections are enumerated,
// its samples run once through the network (keys / values cached) and its
// connections sorted into prefix classes; then ONE persistent launch of the
// prefix-reusing forward covers the connections of all items, each tile
// with its item's model; then every item's sums and energy.  A step neither
// synchronises nor allocates, so it can be captured into a hipGraph.
struct BmItem {
    nnqs_batch_model_item in;
    int64_t C, total, bps;
    int nb;  // selection blocks
    double *sla = nullptr, *sph = nullptr, *xla = nullptr, *xph = nullptr, *partials = nullptr, *pre = nullptr,
           *csla = nullptr;
    uint64_t *xkeys = nullptr;
    int32_t *list = nullptr, *blockcnt = nullptr;
    int64_t *hdr = nullptr;  // {count[4], offset[4], evaluated, per-class evaluated[4]}
    __bf16 *kv = nullptr;
};

struct nnqs_batch_model {
    std::vector<BmItem> items;
    void *d_items = nullptr;  // device array of list-mode launch descriptors (model_bf16.hip)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace nnqs {

static void bm_free(nnqs_batch_model *b) {
    for (auto &it : b->items) {
        hipFree(it.sla);
        hipFree(it.sph);
        hipFree(it.xla);
        hipFree(it.xph);
        hipFree(it.partials);
        hipFree(it.pre);
        hipFree(it.csla);
        hipFree(it.xkeys);
        hipFree(it.list);
        hipFree(it.blockcnt);
        hipFree(it.hdr);
        hipFree(it.kv);
    }
    hipFree(b->d_items);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
}

static nnqs_status bm_step(nnqs_batch_model *b, hipStream_t st) {
    for (auto &it : b->items) {
        const nnqs_batch_model_item &in = it.in;
        nnqs_status s = enqueue_logpsi(in.model, in.keys, in.n, NNQS_BF16, it.sla, it.sph, st);
        if (s != NNQS_OK) return s;
        hipLaunchKernelGGL(k_enum_keys, dim3((unsigned)(in.n * it.bps)), dim3(256), 0, st, in.system->view, in.keys,
                           in.n, it.bps, it.xkeys, (uint8_t *)nullptr, (float *)nullptr);
        s = enqueue_bf16_cached(in.model, in.keys, in.n, it.csla, it.kv, it.pre, st, false);
        if (s != NNQS_OK) return s;
        ClsArgs ca{};
        ca.R = SelRule{nullptr, nullptr, nullptr, it.sla, it.C, 0.0};
        ca.rule = false;
        ca.keys = in.keys;
        ca.xkeys = it.xkeys;
        ca.total = it.total;
        ca.K = in.system->view.K;
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, it.hdr + 8, 5);
        hipLaunchKernelGGL(k_cls_count, dim3(it.nb), dim3(256), 0, st, ca, it.blockcnt);
        hipLaunchKernelGGL(k_cls_scan, dim3(1), dim3(256), 0, st, it.blockcnt, it.nb, it.hdr, it.hdr + 8);
        hipLaunchKernelGGL(k_cls_write, dim3(it.nb), dim3(64), 0, st, ca, it.blockcnt, it.list, false, it.xla, it.xph);
        s = enqueue_bf16_phase_list(in.model, it.xkeys, it.list, it.hdr, it.total, it.xph, st);
        if (s != NNQS_OK) return s;
    }
    nnqs_status s = enqueue_bf16_batch(b->items.front().in.model, b->d_items, (int)b->items.size(), st);
    if (s != NNQS_OK) return s;
    for (auto &it : b->items) {
        const nnqs_batch_model_item &in = it.in;
        const unsigned grid = (unsigned)(in.n * it.bps);
        hipLaunchKernelGGL(k_eloc_partial, dim3(grid), dim3(256), 0, st, in.system->view, in.keys, it.sla, it.sph, in.n,
                           it.bps, it.xla, it.xph, it.partials);
        hipLaunchKernelGGL(k_eloc_finish, dim3((unsigned)((in.n + 255) / 256)), dim3(256), 0, st, it.partials, in.n,
                           it.bps, in.eloc);
        if (in.energy) {
            s = enqueue_energy_partials(it.partials, in.counts, in.eloc, in.n, in.energy, st);
            if (s != NNQS_OK) return s;
        }
    }
    NNQS_HIP_CHECK(hipGetLastError());
    return NNQS_OK;
}

}  // namespace nnqs

extern "C" {

nnqs_status nnqs_batch_model_create(nnqs_batch_model **out, const nnqs_batch_model_item *items, int32_t n_items) {
    clear_error();
    if (!out || !items) return fail(NNQS_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n_items < 1 || n_items > bf16_batch_max_items())
        return fail(NNQS_EINVAL, "n_items=%d outside [1, %d]", n_items, bf16_batch_max_items());
    for (int i = 0; i < n_items; i++) {
        const nnqs_batch_model_item &in = items[i];
        if (!in.system || !in.model || !in.keys || !in.eloc) return fail(NNQS_EINVAL, "item %d: null pointer", i);
        if (in.energy && !in.counts) return fail(NNQS_EINVAL, "item %d: energy requested without counts", i);
        if (in.n <= 0 || in.n > kMaxChunkSamplesBf16)
            return fail(NNQS_EINVAL, "item %d: n=%lld outside [1, %lld]", i, (long long)in.n,
                        (long long)kMaxChunkSamplesBf16);
        if (!in.model->bf16_ok) return fail(NNQS_EUNSUPPORTED, "item %d: model shape has no BF16 path", i);
        const nnqs_model_desc &d = in.model->desc;
        if (d.n_orb != in.system->view.K || d.n_up != in.system->view.n_up || d.n_dn != in.system->view.n_dn)
            return fail(NNQS_EINVAL, "item %d: model and system disagree", i);
        if (in.n * in.system->view.C > (int64_t)INT32_MAX)
            return fail(NNQS_ERANGE, "item %d: %lld connections exceed 2^31 - 1", i,
                        (long long)(in.n * in.system->view.C));
        for (int j = 0; j < i; j++)
            if (items[j].model == in.model) return fail(NNQS_EINVAL, "items %d and %d share a model", j, i);
    }
    nnqs_batch_model *b = new nnqs_batch_model();
    b->items.resize(n_items);
    const size_t isz = bf16_item_bytes();
    std::vector<unsigned char> host(n_items * isz);
    bool ok = true;
    for (int i = 0; i < n_items && ok; i++) {
        BmItem &it = b->items[i];
        it.in = items[i];
        it.C = items[i].system->view.C;
        it.total = items[i].n * it.C;
        it.bps = (it.C + kConnPerBlock - 1) / kConnPerBlock;
        it.nb = (int)((it.total + kSelBlock - 1) / kSelBlock);
        const size_t n = (size_t)items[i].n, tot = (size_t)it.total;
        ok = hipMalloc(&it.sla, n * 8) == hipSuccess && hipMalloc(&it.sph, n * 8) == hipSuccess &&
             hipMalloc(&it.xla, tot * 8) == hipSuccess && hipMalloc(&it.xph, tot * 8) == hipSuccess &&
             hipMalloc(&it.partials, std::max<size_t>(n * it.bps * 4, kPartialBlocks * 8) * 8) == hipSuccess &&
             hipMalloc(&it.pre, n * 4 * 8) == hipSuccess && hipMalloc(&it.csla, n * 8) == hipSuccess &&
             hipMalloc(&it.xkeys, tot * 16) == hipSuccess && hipMalloc(&it.list, tot * 4) == hipSuccess &&
             hipMalloc(&it.blockcnt, ((size_t)it.nb + 2) * 16) == hipSuccess &&
             hipMalloc(&it.hdr, 16 * 8) == hipSuccess &&
             hipMalloc(&it.kv, n * bf16_cache_elems(items[i].model) * sizeof(__bf16)) == hipSuccess;
        if (ok) bf16_list_item(items[i].model, it.xkeys, it.C, it.list, it.hdr, it.kv, it.pre, it.xla, host.data() + i * isz);
    }
    if (ok) ok = hipMalloc(&b->d_items, n_items * isz) == hipSuccess;
    if (!ok) {
        bm_free(b);
        delete b;
        return fail(NNQS_ENOMEM, "batch scratch allocation failed");
    }
    if (hipMemcpy(b->d_items, host.data(), n_items * isz, hipMemcpyHostToDevice) != hipSuccess) {
        bm_free(b);
        delete b;
        return fail(NNQS_EHIP, "batch descriptor upload failed");
    }
    *out = b;
    return NNQS_OK;
}

nnqs_status nnqs_batch_model_destroy(nnqs_batch_model *b) {
    if (!b) return NNQS_OK;
    bm_free(b);
    delete b;
    return NNQS_OK;
}

nnqs_status nnqs_batch_model_run(nnqs_batch_model *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    return bm_step(b, as_stream(stream));
}

nnqs_status nnqs_batch_model_capture(nnqs_batch_model *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    if (!stream) return fail(NNQS_EINVAL, "graph capture needs a created (non-null) stream");
    hipStream_t st = as_stream(stream);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    NNQS_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const nnqs_status s = bm_step(b, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (s != NNQS_OK) {
        if (g) hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(NNQS_EHIP, "stream capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        b->graph = nullptr;
        b->exec = nullptr;
        return fail(NNQS_EHIP, "graph instantiation failed");
    }
    return NNQS_OK;
}

nnqs_status nnqs_batch_model_launch(nnqs_batch_model *b, void *stream) {
    clear_error();
    if (!b) return fail(NNQS_EINVAL, "null batch");
    if (!b->exec) return fail(NNQS_EINVAL, "no captured graph (call nnqs_batch_model_capture first)");
    NNQS_HIP_CHECK(hipGraphLaunch(b->exec, as_stream(stream)));
    return NNQS_OK;
}

}  // extern "C"

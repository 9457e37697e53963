// Per-sample orbital lists, canonical connection decoding and wave-level
// helpers shared by the enumeration kernels.
#pragma once

#include "internal.hpp"

namespace nnqs {

struct WaveLds {
    uint8_t occ[2][64];  // occupied spin orbitals per spin, ascending
    uint8_t vir[2][64];  // empty spin orbitals per spin, ascending
    uint32_t queue[256]; // candidate ring: i | j<<8 | a<<16 | b<<24 (255 = none)
    double hit[6];       // per-sample constants of the hit path (sample-aware kernel)
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int readlane32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ uint64_t wave_xor64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_plain(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ bool sample_conserves(const SysView &S, const Key &x) {
    if ((x.lo & ~S.valid0) | (x.hi & ~S.valid1)) return false;
    int up = __popcll(x.lo & EVEN_BITS) + __popcll(x.hi & EVEN_BITS);
    int dn = __popcll(x.lo & ODD_BITS) + __popcll(x.hi & ODD_BITS);
    return up == S.n_up && dn == S.n_dn;
}

// Occupied / empty lists per spin into LDS (lane i inspects spatial orbital i).
__device__ __forceinline__ void build_lists(const SysView &S, const Key &x, WaveLds &wl) {
    const int lane = lane_id();
    const bool in = lane < S.K;
    const bool ou = in && key_bit(x, 2 * lane);
    const bool od = in && key_bit(x, 2 * lane + 1);
    const uint64_t bu = __ballot(ou), bd = __ballot(od);
    const int ru = mbcnt(bu), rd = mbcnt(bd);
    if (in) {
        if (ou) wl.occ[0][ru] = (uint8_t)(2 * lane);
        else wl.vir[0][lane - ru] = (uint8_t)(2 * lane);
        if (od) wl.occ[1][rd] = (uint8_t)(2 * lane + 1);
        else wl.vir[1][lane - rd] = (uint8_t)(2 * lane + 1);
    }
    wave_sync();
}

// Diagonal element: E_core + sum_p h_pp + 1/2 sum_{p,q} [J_pq - delta_spin K_pq]
// over occupied p, q.  Lanes take the (p, q) pairs, so that all their
// integral loads are independent; fixed-order wave sum.
__device__ __forceinline__ double wave_diag(const SysView &S, const Key &x, const WaveLds &wl) {
    const int lane = lane_id();
    const int nu = S.n_up, ntot = S.n_up + S.n_dn;
    const int K = S.K;
    auto occ = [&](int t) -> int { return t < nu ? wl.occ[0][t] : wl.occ[1][t - nu]; };
    double part = 0.0;
    for (int t = lane; t < ntot; t += 64) {
        const int ip = occ(t) >> 1;
        part += S.h[ip * K + ip];
    }
    const int npairs = ntot * ntot;
    for (int t = lane; t < npairs; t += 64) {
        const int a = t / ntot, b = t - a * ntot;
        const int p = occ(a), q = occ(b);
        const int ip = p >> 1, iq = q >> 1;
        double v = S.Jm[ip * K + iq];
        if (((p ^ q) & 1) == 0) v -= S.Km[ip * K + iq];
        part += 0.5 * v;
    }
    return S.ecore + wave_sum_plain(part);
}


// Decode canonical connection index c (see nnqs_connections) into raw
// excitation indices (i, j, a, b), 255 where absent: singles give (q, 255,
// p, 255); opposite-spin doubles give (i_up, j_dn, a_up, b_dn).
__device__ inline void decode_canonical(const SysView &S, const WaveLds &wl, int64_t c, int &i, int &j, int &a,
                                        int &b) {
    const int K = S.K, nu = S.n_up, nd = S.n_dn, vu = K - nu, vd = K - nd;
    const int64_t nsu = (int64_t)nu * vu, nsd = (int64_t)nd * vd;
    const int64_t pou = (int64_t)nu * (nu - 1) / 2, pvu = (int64_t)vu * (vu - 1) / 2;
    const int64_t pod = (int64_t)nd * (nd - 1) / 2, pvd = (int64_t)vd * (vd - 1) / 2;
    i = j = a = b = 255;
    auto pair = [](int64_t t, int m, int &r1, int &r2) {
        r1 = 0;
        while (t >= m - 1 - r1) {
            t -= m - 1 - r1;
            r1++;
        }
        r2 = r1 + 1 + (int)t;
    };
    if (c == 0) return;
    c -= 1;
    if (c < nsu) {
        i = wl.occ[0][c / vu];
        a = wl.vir[0][c % vu];
        return;
    }
    c -= nsu;
    if (c < nsd) {
        i = wl.occ[1][c / vd];
        a = wl.vir[1][c % vd];
        return;
    }
    c -= nsd;
    if (c < pou * pvu) {
        int r1, r2, s1, s2;
        pair(c / pvu, nu, r1, r2);
        pair(c % pvu, vu, s1, s2);
        i = wl.occ[0][r1];
        j = wl.occ[0][r2];
        a = wl.vir[0][s1];
        b = wl.vir[0][s2];
        return;
    }
    c -= pou * pvu;
    if (c < pod * pvd) {
        int r1, r2, s1, s2;
        pair(c / pvd, nd, r1, r2);
        pair(c % pvd, vd, s1, s2);
        i = wl.occ[1][r1];
        j = wl.occ[1][r2];
        a = wl.vir[1][s1];
        b = wl.vir[1][s2];
        return;
    }
    c -= pod * pvd;
    const int64_t bd = c % vd;
    c /= vd;
    const int64_t od = c % nd;
    c /= nd;
    const int64_t au = c % vu;
    const int64_t ou = c / vu;
    i = wl.occ[0][ou];
    a = wl.vir[0][au];
    j = wl.occ[1][od];
    b = wl.vir[1][bd];
}

// x' of raw excitation indices.
__device__ __forceinline__ Key apply_excitation(Key x, int i, int j, int a, int b) {
    if (i != 255) {
        key_flip(x, i);
        key_flip(x, a);
        if (j != 255) {
            key_flip(x, j);
            key_flip(x, b);
        }
    }
    return x;
}

}  // namespace nnqs

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

#include "enumerate.hpp"
#include "model.hpp"

namespace nnqs {

constexpr int kConnPerBlock = 4096;            // connections handled by one block
constexpr int64_t kMaxChunkConnections = 1 << 24;

__global__ void __launch_bounds__(256) k_enum_keys(SysView S, const uint64_t *__restrict__ keys, int64_t m,
                                                   int64_t blocks_per_sample, uint64_t *__restrict__ out) {
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
    }
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
    m->d_xkeys = nullptr;
    m->d_xla = m->d_xph = m->d_sla = m->d_sph = m->d_partials = nullptr;
    m->xcap = m->scap = 0;
}

}  // namespace nnqs

using namespace nnqs;

extern "C" nnqs_status nnqs_eloc_model(const nnqs_system *sys, nnqs_model *model, int32_t precision,
                                       const uint64_t *keys, const uint32_t *counts, int64_t n, double *eloc,
                                       double *energy, nnqs_stats *stats, uint32_t flags, void *stream) {
    clear_error();
    if (!sys || !model || !keys || !eloc) return fail(NNQS_EINVAL, "null pointer argument");
    if (energy && !counts) return fail(NNQS_EINVAL, "energy requested without counts");
    if (n <= 0) return fail(NNQS_EINVAL, "n must be positive");
    if (model->desc.n_orb != sys->view.K || model->desc.n_up != sys->view.n_up || model->desc.n_dn != sys->view.n_dn)
        return fail(NNQS_EINVAL, "model and system disagree on orbitals or electron numbers");
    if (precision != NNQS_FP64 && precision != NNQS_BF16) return fail(NNQS_EUNSUPPORTED, "unknown precision");
    if (precision == NNQS_BF16 && !model->bf16_ok) return fail(NNQS_EUNSUPPORTED, "model shape has no BF16 path");
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
    int64_t chunk = kMaxChunkConnections / C;
    if (chunk < 1) chunk = 1;
    if (chunk > n) chunk = n;
    const int64_t bps = (C + kConnPerBlock - 1) / kConnPerBlock;
    if (model->xcap < chunk * C) {
        NNQS_HIP_CHECK(hipStreamSynchronize(st));  // scratch may be in use by earlier work on this stream
        nnqs_status s1 = grow(reinterpret_cast<void **>(&model->d_xkeys), (size_t)chunk * C * 16);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_xla), (size_t)chunk * C * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_xph), (size_t)chunk * C * 8);
        if (s1 == NNQS_OK) s1 = grow(reinterpret_cast<void **>(&model->d_partials),
                                     std::max<size_t>((size_t)chunk * bps * 4, kPartialBlocks * 8) * 8);
        if (s1 != NNQS_OK) {
            eloc_model_free(model);
            return s1;
        }
        model->xcap = chunk * C;
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
    nnqs_status s1 = enqueue_logpsi(model, keys, n, precision, model->d_sla, model->d_sph, st);
    if (s1 != NNQS_OK) return s1;
    for (int64_t s0 = 0; s0 < n; s0 += chunk) {
        const int64_t m = n - s0 < chunk ? n - s0 : chunk;
        const unsigned grid = (unsigned)(m * bps);
        hipLaunchKernelGGL(k_enum_keys, dim3(grid), dim3(256), 0, st, sys->view, keys + 2 * s0, m, bps,
                           model->d_xkeys);
        s1 = enqueue_logpsi(model, model->d_xkeys, m * C, precision, model->d_xla, model->d_xph, st);
        if (s1 != NNQS_OK) return s1;
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
        NNQS_HIP_CHECK(hipStreamSynchronize(st));
        stats->connections = n * C;
        stats->evaluated = n * C;
    }
    return NNQS_OK;
}

/*
 * nnqs_eloc.h -- C ABI of the MI355X (gfx950) local-energy library.
 *
 * The library evaluates the local energy of a neural-network quantum state
 * for a second-quantised molecular Hamiltonian (paper: Section 2.1, Eq. 4):
 *
 *     E_loc(x) = sum_{x'} H_{x x'} psi(x') / psi(x),
 *
 * over a batch of unique sampled occupation bit strings x, and the sample
 * mean of Eq. 6 weighted by each unique sample's occurrence count (Section
 * 3.1, batch autoregressive sampling keeps unique samples with weights).
 * The Hamiltonian is Eq. 9 (Section 2.3), given by its one- and two-electron
 * integrals; connected configurations x' are single and double excitations
 * that conserve the up and down electron numbers (Eq. 12 constraint).
 *
 * Conventions used by every entry point:
 *  - K spatial orbitals, N = 2K spin orbitals (4 <= N <= 128, N even);
 *    spin orbital p = 2*i + s, s = 0 up, s = 1 down (Section 3.3: spatial
 *    orbital i maps to an adjacent up/down qubit pair).
 *  - A configuration is a 128-bit key of two uint64 words, key[0] holding
 *    bits 0..63 and key[1] bits 64..127; bit p = occupation of spin orbital p
 *    (Section 3.4 item 5: samples packed into one or two integers).  Keys of
 *    N <= 64 systems have key[1] == 0.  Tables are ordered as unsigned
 *    128-bit integers, key[1] major.
 *  - Jordan-Wigner strings run over lower indices:
 *      a_p |x> = x_p (-1)^{#occupied q<p} |x - e_p>.
 *  - Integrals are spatial, chemists' notation, row-major doubles:
 *      h[i*K + j],  g[((i*K + j)*K + k)*K + l] = (ij|kl)  (8-fold symmetric),
 *    so that H = E_core + sum h_pq a+_p a_q
 *              + 1/2 sum <pq|rs> a+_p a+_q a_s a_r,
 *    <pq|rs> = (i_p i_r|i_q i_s) when spins of (p,r) and of (q,s) agree.
 *  - Amplitudes travel in log-polar form: psi(x) = exp(logabs + i*phase).
 *    Complex outputs are interleaved (re, im) doubles.
 *  - Device pointers are HIP device (or managed) memory on the current
 *    device; host pointers are marked "host".  The caller owns every pointer
 *    it passes.  Objects created by *_create own their device memory until
 *    the matching *_destroy.  No entry point allocates caller-visible output.
 *  - `stream` is a hipStream_t cast to void* (NULL = the null stream).  All
 *    device work is enqueued asynchronously on it; entry points return after
 *    enqueueing unless they say they synchronise.
 *  - Errors are reported by return code (nnqs_status) and a thread-local
 *    message (nnqs_last_error).  Host-side checks run before anything is
 *    enqueued; on such an error no output is touched.
 */
#ifndef NNQS_ELOC_H
#define NNQS_ELOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nnqs_status;

enum {
    NNQS_OK = 0,
    NNQS_EINVAL = -1,       /* bad argument: null pointer, size, N odd or > 128, n_s > K */
    NNQS_EDUP = -2,         /* a table holds the same key twice */
    NNQS_ECONSERVE = -3,    /* a key has the wrong number of up or down electrons */
    NNQS_ERANGE = -4,       /* a log-amplitude is not finite, or a size exceeds a capacity */
    NNQS_ENOMEM = -5,       /* device allocation failed */
    NNQS_EHIP = -6,         /* a HIP runtime call failed */
    NNQS_EUNSUPPORTED = -7  /* no gfx950 GPU, or a kernel build that spills to private memory */
};

/* Flags for calls that read device-resident inputs. */
enum {
    /* Validate the device inputs before computing: the call synchronises
     * `stream`, returns NNQS_ECONSERVE / NNQS_ERANGE / NNQS_EDUP if the check
     * fails and then leaves every output untouched.  Without this flag the
     * call never synchronises (it can be captured in a HIP graph); invalid
     * samples then get NaN outputs and set the sticky device status that
     * nnqs_table_status reports. */
    NNQS_VALIDATE = 1u
};

/* Message of the last failing call on this thread ("" if none).  Valid
 * until the next call on the same thread. */
const char *nnqs_last_error(void);

/* Library version string. */
const char *nnqs_version(void);

/* ------------------------------------------------------------------ system */
/* Molecular Hamiltonian of Eq. 9 resident on the current device. */
typedef struct nnqs_system nnqs_system;

/* Copies the integrals (host arrays, layouts above) to the device and
 * precomputes the diagonal Coulomb/exchange tables.
 *   n_spin_orb: N, even, 4..128;  n_up, n_dn: electrons per spin, 0..K.
 * Synchronous.  Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED. */
nnqs_status nnqs_system_create(nnqs_system **out, int32_t n_spin_orb, int32_t n_up, int32_t n_dn,
                               const double *h, const double *g, double e_core);

/* Releases the device copies.  NULL is accepted. */
nnqs_status nnqs_system_destroy(nnqs_system *sys);

/* Number C of connected configurations per sample, the diagonal included:
 * C = 1 + n_u v_u + n_d v_d + C(n_u,2) C(v_u,2) + C(n_d,2) C(v_d,2)
 *       + n_u v_u n_d v_d,  v_s = K - n_s.  Returns -1 for NULL. */
int64_t nnqs_connection_count(const nnqs_system *sys);

/* -------------------------------------------------------------------- table */
/* Sorted table of unique samples with their amplitudes (Section 3.4 item 5:
 * the id and wave-function lookup tables), plus the device-side search
 * structures of the sample-aware lookup. */
typedef struct nnqs_table nnqs_table;

/* Allocates a table for up to `capacity` samples of `sys` (which must
 * outlive it).  Synchronous.  Errors: EINVAL, ENOMEM, EHIP. */
nnqs_status nnqs_table_create(nnqs_table **out, const nnqs_system *sys, int64_t capacity);

/* Releases the table.  NULL is accepted. */
nnqs_status nnqs_table_destroy(nnqs_table *tab);

/* Builds the table from n samples (device arrays): keys [n][2], logabs [n],
 * phase [n].  Sorts the keys (payload permuted alongside), and builds the
 * search structures.  Duplicate keys set the sticky status NNQS_EDUP.
 * flags: NNQS_VALIDATE (see above).  Errors: EINVAL, ERANGE (n > capacity),
 * EDUP / ECONSERVE / ERANGE with NNQS_VALIDATE, EHIP. */
nnqs_status nnqs_table_build(nnqs_table *tab, const uint64_t *keys, const double *logabs,
                             const double *phase, int64_t n, uint32_t flags, void *stream);

/* Copies the sorted table into device arrays keys_out [n][2], logabs_out [n],
 * phase_out [n] (n = current size, written to *n_out on the host).
 * Synchronises `stream`.  For tests. */
nnqs_status nnqs_table_export(const nnqs_table *tab, uint64_t *keys_out, double *logabs_out,
                              double *phase_out, int64_t *n_out, void *stream);

/* Synchronises `stream`, then returns and clears the sticky device status
 * set by earlier builds / evaluations on this table (NNQS_OK if none). */
nnqs_status nnqs_table_status(nnqs_table *tab, void *stream);

/* ------------------------------------------------------------ enumeration */
/* Connected configurations of n samples in canonical order (for parity
 * checks): diagonal; singles up then down, (occupied rank, virtual rank);
 * same-spin doubles up then down, (occupied pair, virtual pair), pairs in
 * lexicographic rank order; opposite-spin doubles (i_up, a_up, j_dn, b_dn).
 * Outputs are device arrays of n*C entries (C = nnqs_connection_count):
 *   xprime [n][C][2] keys of x';
 *   sign   [n][C]    sign of the excitation operator a+_a a+_b a_j a_i
 *                    (i<j, a<b) or a+_p a_q acting on x, +1 on the diagonal;
 *   exc    [n][C][4] spin-orbital indices (i, j, a, b) sorted, 255 absent;
 *   hxx    [n][C]    H_{x x'} (sign included).
 * Any output pointer may be NULL to skip it.  Samples with wrong particle
 * numbers get sign 0 and NaN hxx.  Errors: EINVAL, ECONSERVE (VALIDATE). */
nnqs_status nnqs_connections(const nnqs_system *sys, const uint64_t *keys, int64_t n,
                             uint64_t *xprime, int8_t *sign, uint8_t *exc, double *hxx,
                             uint32_t flags, void *stream);

/* -------------------------------------------------- sample-aware E_loc */
/* Local energies of n samples with psi(x') taken from the table and x'
 * outside the table skipped (Section 3.4 item 4, sample-aware evaluation;
 * Algorithm 2 fuses the lookup with the accumulation).  Inputs (device):
 * keys [n][2], counts [n] occurrence weights, logabs [n], phase [n] of the
 * samples themselves.  Outputs (device): eloc [n][2] complex E_loc(x);
 * energy [4] = { sum c Re E_loc / sum c, sum c Im E_loc / sum c, sum c,
 * sum c (Re E_loc - E)^2 / sum c } (Eq. 6 over unique samples); energy may
 * be NULL.  A count of zero removes its sample from the sums; with every
 * count zero the energy's ratios are NaN.  Matrix elements, ratios and sums
 * are FP64; per-sample sums are
 * compensated (Neumaier) and the reduction order is fixed, so repeated
 * calls give bit-identical results.  Calls sharing one table must be ordered
 * on one stream (the energy reduction uses the table's scratch).
 * Errors: EINVAL, ECONSERVE / ERANGE (VALIDATE), EHIP. */
nnqs_status nnqs_eloc_table(const nnqs_system *sys, nnqs_table *tab, const uint64_t *keys,
                            const uint32_t *counts, const double *logabs, const double *phase,
                            int64_t n, double *eloc, double *energy, uint32_t flags, void *stream);

/* Weighted energy of Eq. 6 alone from precomputed local energies (device
 * arrays counts [n], eloc [n][2]) into energy [4] (layout as above), using
 * the table's scratch.  Errors: EINVAL, EHIP. */
nnqs_status nnqs_energy(nnqs_table *tab, const uint32_t *counts, const double *eloc, int64_t n,
                        double *energy, void *stream);

/* Largest n that nnqs_energy_noalloc accepts. */
#define NNQS_ENERGY_NOALLOC_MAX_N 2147483647LL

/* nnqs_energy for callers that cannot allocate device memory or that need a
 * call free of allocations (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same weighted energy (Eq. 6,
 * same kernels, same reduction order, so bit-identical results) without a
 * table.  Its scratch, the block partials of the two reduction passes, is a
 * library-owned 64 KiB device array per GPU, held until the process ends;
 * the call allocates and frees nothing.  Inputs (device): counts [n],
 * eloc [n][2]; output (device): energy [4] as in nnqs_eloc_table.  The
 * scratch is shared by every call on one GPU, so calls that overlap on one
 * GPU (different streams without ordering, or several host threads) race:
 * order them on one stream.  Errors: EINVAL (null pointer, n <= 0), ERANGE
 * (n > NNQS_ENERGY_NOALLOC_MAX_N), EHIP, EUNSUPPORTED (device ordinal >= 64). */
nnqs_status nnqs_energy_noalloc(const uint32_t *counts, const double *eloc, int64_t n, double *energy,
                                void *stream);

/* ------------------------------------------------------------------ model */
/* Wave-function ansatz of Section 3.1 (Eq. 11, Fig. 2): a decoder-only
 * transformer gives |psi|^2 autoregressively (Eq. 8) over tokens that are
 * spatial-orbital pairs taken in reverse orbital order with the electron
 * number mask of Eq. 12 (Section 3.3); an MLP of three dense layers
 * N x P x P x 1 gives the phase (Section 4.1).  Readings where the paper is
 * silent: pre-LN blocks (eps 1e-5), causal multi-head attention scaled by
 * 1/sqrt(d_model/n_heads), FFN with exact-erf GELU, input of position s = the
 * embedding of the token at s-1 (a begin token 4 at s = 0) + a learned
 * position embedding, final LN and a d_model -> 4 head plus a fixed bias
 * table[orbital][token], a mask that also forbids leaving more electrons than
 * remaining positions, log|psi| = 1/2 sum_s log pi(t_s | t_<s), and GELU
 * between the phase layers.  Token of orbital i: t = n_up(i) + 2 n_dn(i);
 * position s holds orbital K-1-s. */
typedef struct nnqs_model nnqs_model;

typedef struct {
    int32_t n_orb;        /* K spatial orbitals = sequence length, 2..64 */
    int32_t d_model;      /* multiple of n_heads, <= 128 */
    int32_t n_layers;     /* >= 1 */
    int32_t n_heads;
    int32_t d_ff;         /* <= 1024 */
    int32_t phase_hidden; /* P, <= 1024 */
    int32_t n_up, n_dn;   /* electron numbers used by the mask */
} nnqs_model_desc;

/* Precision of the network evaluation. */
enum {
    NNQS_FP64 = 0, /* every operation in FP64 (parity path) */
    NNQS_BF16 = 1, /* BF16 MFMA with FP32 accumulation and FP32 normalisation
                      and softmax; log|psi| and phase returned as FP64.
                      Needs d_model 64, n_heads 4, d_ff 256, P 512. */
    NNQS_FP32 = 2, /* FP32 arithmetic (screen training) */
    NNQS_FP8 = 3   /* OCP FP8 E4M3 MFMA operands (activations unscaled, each weight
                      matrix with a power-of-two scale) and FP32 accumulation;
                      the rest as NNQS_BF16 */
};

/* Number of FP32 weights the layout below holds for `desc`; -1 if invalid. */
int64_t nnqs_model_weight_count(const nnqs_model_desc *desc);

/* Copies host FP32 weights (row-major matrices [in][out], y = x W + b) in
 * this order:
 *   tok_emb[5][d] pos_emb[K][d]
 *   per layer: ln1_g[d] ln1_b[d] wq[d][d] bq[d] wk[d][d] bk[d] wv[d][d] bv[d]
 *              wo[d][d] bo[d] ln2_g[d] ln2_b[d] w1[d][F] b1[F] w2[F][d] b2[d]
 *   lnf_g[d] lnf_b[d] head_w[d][4] head_b[4] logit_bias[K][4]
 *   ph_w1[2K][P] ph_b1[P] ph_w2[P][P] ph_b2[P] ph_w3[P][1] ph_b3[1]
 * to the device in FP64 and BF16 forms.  Synchronous.
 * Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED. */
nnqs_status nnqs_model_create(nnqs_model **out, const nnqs_model_desc *desc, const float *weights);

/* Releases the model.  NULL is accepted. */
nnqs_status nnqs_model_destroy(nnqs_model *model);

/* log|psi| and phase of n configurations (device keys [n][2]) into device
 * arrays logabs [n], phase [n].  Keys outside the model's electron sector get
 * logabs = -inf.  Errors: EINVAL, EUNSUPPORTED (precision), EHIP. */
nnqs_status nnqs_model_logpsi(const nnqs_model *model, const uint64_t *keys, int64_t n, int32_t precision,
                              double *logabs, double *phase, void *stream);

/* Batch autoregressive sampling (Section 3.1) of n_samples samples from the
 * model, the network in `precision` (NNQS_FP64 or NNQS_BF16).  At sequence
 * position s every unique prefix u of weight c_u gets its conditional
 * pi(t | prefix) (the Eq. 12 mask included); its c_u sample slots (numbered
 * in prefix order) each draw a token with the uniform of Philox4x32-10
 * (Salmon et al., SC 2011) at counter (slot mod 2^32, slot / 2^32, s,
 * 0x42415300) and key `seed` (top 53 bits of the first two output words),
 * splitting c_u multinomially among the four children; children of zero
 * weight are dropped and the rest kept in (parent, token) order.  Outputs
 * (device, `capacity` entries): keys_out [m][2] the unique samples,
 * counts_out [m] their counts (sum n_samples), logabs_out [m] = 1/2 sum of
 * log pi along the path, phase_out [m] (may be NULL) the phase MLP; *n_unique
 * (host) = m.  Synchronises `stream` once per position.  Errors: EINVAL,
 * ERANGE (more than `capacity` prefixes), ENOMEM, EUNSUPPORTED, EHIP. */
nnqs_status nnqs_bas(nnqs_model *model, int32_t precision, uint64_t seed, uint64_t n_samples, int64_t capacity,
                     uint64_t *keys_out, uint32_t *counts_out, double *logabs_out, double *phase_out,
                     int64_t *n_unique, void *stream);

/* ------------------------------------------------------- VMC gradient step */
/* Weighted parameter gradient of the ansatz in FP64 (the derivative that
 * Eq. 7 of Section 2.1 contracts): for device keys [n][2] and cotangents
 * c_logabs [n], c_phase [n],
 *   grad[w] = sum_b c_logabs[b] d log|psi(x_b)|/dw + c_phase[b] d phi(x_b)/dw
 * over every weight of the layout of nnqs_model_create (device grad
 * [nnqs_model_weight_count], overwritten).  The logit-bias table is a fixed
 * part of the ansatz: its entries are zero.  With logabs / phase (device [n],
 * both or neither) the forward values of the same pass are written too.
 * Needs d_model 64, 4 heads, d_ff a multiple of 64 (the FP64 batched
 * forward).  Grows model-owned scratch (about 33 KB per sequence row of a
 * 256-configuration pass); calls on one model must not overlap.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EHIP. */
nnqs_status nnqs_model_grad(nnqs_model *model, const uint64_t *keys, int64_t n, const double *c_logabs,
                            const double *c_phase, double *grad, double *logabs, double *phase, void *stream);

/* The VMC energy gradient of Eq. 7 (Section 2.1) over unique samples with
 * the weights of Eq. 6: with p_b = counts[b] / sum counts and
 * E = sum_b p_b E_loc(b) (complex),
 *   grad = 2 Re sum_b p_b (E_loc(b) - E) d ln psi*(x_b)
 *        = sum_b 2 p_b [Re(E_loc(b) - E) d log|psi(x_b)| + Im(E_loc(b) - E) d phi(x_b)].
 * Inputs (device): keys [n][2], counts [n], eloc [n][2] (re, im); outputs
 * (device): grad [nnqs_model_weight_count]; energy [4] as in nnqs_eloc_table
 * (may be NULL).  Errors: as nnqs_model_grad. */
nnqs_status nnqs_vmc_gradient(nnqs_model *model, const uint64_t *keys, const uint32_t *counts, const double *eloc,
                              int64_t n, double *grad, double *energy, void *stream);

/* Learning rate of Eq. 13 (Section 4.1) at iteration step >= 1:
 * d_model^-1/2 min(step^-1/2, step warmup^-3/2); 0 for invalid arguments. */
double nnqs_lr_schedule(int64_t step, int32_t d_model, int32_t warmup);

/* One AdamW step (decoupled weight decay; Section 4.1 names the optimizer,
 * hyper-parameters are the caller's) of the model's FP64 weights with device
 * grad and moments mom1, mom2 [nnqs_model_weight_count] (zero before step 1,
 * updated in place): w <- w (1 - lr wd) - lr mh / (sqrt(vh) + eps) with
 * mh = mom1 / (1 - beta1^step), vh = mom2 / (1 - beta2^step).  The fixed
 * logit-bias table is left unchanged (its moments stay zero).  Afterwards the
 * BF16 / FP8 copies of the weights are rebuilt from the FP64 ones
 * (synchronises `stream`); batched-model objects made from the model must be
 * made again.  Errors: EINVAL (step < 1, beta outside [0, 1), eps <= 0,
 * lr < 0, weight_decay < 0), ENOMEM, EHIP. */
nnqs_status nnqs_model_adamw_step(nnqs_model *model, const double *grad, int64_t step, double lr, double beta1,
                                  double beta2, double eps, double weight_decay, double *mom1, double *mom2,
                                  void *stream);

/* Copies the model's FP64 weights (layout of nnqs_model_create) to device
 * out [nnqs_model_weight_count].  Errors: EINVAL, EHIP. */
nnqs_status nnqs_model_get_weights(const nnqs_model *model, double *out, void *stream);

/* ----------------------------------------------------------------- screen */
/* Learned screen (an addition to the paper, whose only filter is the
 * sample-aware restriction of Section 3.4 item 4): an MLP that predicts
 * log|psi(x')| of a connected configuration from
 *   u = [bits of x' (N) | one-hot(i) | one-hot(j) | one-hot(a) | one-hot(b)]
 * (5N inputs; (i, j, a, b) sorted spin-orbital indices, 255 = absent, as in
 * nnqs_connections), z1 = GELU(u W1 + b1), z2 = GELU(z1 W2 + b2),
 * y = z2 . w3 + b3.  It is trained on the network's own amplitudes (mean
 * squared error, Adam) by these kernels; nnqs_eloc_model can then skip the
 * transformer for connections whose prediction lies more than `skip_nats`
 * below the sample's own log|psi|. */
typedef struct nnqs_screen nnqs_screen;

/* Weights in order W1[5N][H] b1[H] W2[H][H] b2[H] w3[H] b3[1]; -1 if invalid
 * (N even 4..128, 1 <= H <= 1024). */
int64_t nnqs_screen_weight_count(int32_t n_spin_orb, int32_t hidden);

/* Creates a screen from host FP64 weights (layout above); Adam moments start
 * at zero.  Synchronous.  Errors: EINVAL, ENOMEM, EHIP. */
nnqs_status nnqs_screen_create(nnqs_screen **out, int32_t n_spin_orb, int32_t hidden, const double *weights);

/* Releases the screen.  NULL is accepted. */
nnqs_status nnqs_screen_destroy(nnqs_screen *screen);

/* Copies the current FP64 weights to the host.  Synchronises `stream`. */
nnqs_status nnqs_screen_get_weights(const nnqs_screen *screen, double *host_out, void *stream);

/* Adam state of the screen (checkpoint and resume of its training): the
 * first and second moments (host m_out, v_out, weight-count doubles each)
 * and the step count *t_out; nnqs_screen_set_state loads them back (host m,
 * v; t >= 0), so that the next nnqs_screen_adam_step continues exactly where
 * the saved run left off.  Both synchronise `stream`.  Callers: those that
 * save a partly trained screen.  Errors: EINVAL, EHIP. */
nnqs_status nnqs_screen_get_state(const nnqs_screen *screen, double *m_out, double *v_out, int64_t *t_out,
                                  void *stream);
nnqs_status nnqs_screen_set_state(nnqs_screen *screen, const double *m, const double *v, int64_t t, void *stream);

/* Predictions for n connections (device xkeys [n][2], exc [n][4]) into device
 * pred [n].  Key bits at or above N and excitation codes >= N (255 included)
 * contribute no input.  precision: NNQS_FP64, NNQS_FP32, NNQS_BF16 or NNQS_FP8 (the
 * inference kernels of nnqs_eloc_model; need H = 256).  Errors: EINVAL, EUNSUPPORTED,
 * ENOMEM, EHIP. */
nnqs_status nnqs_screen_forward(nnqs_screen *screen, const uint64_t *xkeys, const uint8_t *exc, int64_t n,
                                int32_t precision, double *pred, void *stream);

/* Gradient of loss = mean_k (pred_k - target_k)^2 over the weights (device
 * grad [count], layout as the weights) and the loss (device loss [1], may be
 * NULL).  precision NNQS_FP64 or NNQS_FP32; reductions in a fixed order.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EHIP. */
nnqs_status nnqs_screen_gradient(nnqs_screen *screen, const uint64_t *xkeys, const uint8_t *exc,
                                 const double *target, int64_t n, int32_t precision, double *grad, double *loss,
                                 void *stream);

/* One Adam step (Kingma & Ba, bias-corrected) of the FP64 weights with a
 * device gradient.  Errors: EINVAL, EHIP. */
nnqs_status nnqs_screen_adam_step(nnqs_screen *screen, const double *grad, double lr, double beta1, double beta2,
                                  double eps, void *stream);

/* Counters of a full evaluation (host struct). */
typedef struct {
    int64_t connections; /* connected configurations enumerated, diagonal included */
    int64_t evaluated;   /* of these, evaluated by the network in `precision` (all without a screen) */
    int64_t refined;     /* of these, evaluated again by the FP64 network (refinement) */
    /* BF16 only: `evaluated` split by prefix class b = 0..3, the connections
     * whose first changed sequence position is in [16 b, 16 b + 16) (b = 3:
     * from 48 on); the forward evaluates their rows from 16 b on (see
     * nnqs_eloc_model).  Zero for FP64. */
    int64_t evaluated_class[4];
    /* BF16 only: the rows the evaluated x' need at the least, sum over them
     * of K - s0 (the positions from the first changed one on), and sum over
     * those rows s of s + 1 (the keys row s attends to): the work a
     * prefix-reusing forward cannot avoid.  Zero for FP64. */
    int64_t evaluated_rows;
    int64_t evaluated_keys;
    /* BF16 only: the distinct x' the forward evaluated (equal to `evaluated`
     * without dedup; with it, evaluated_class / rows / keys count these). */
    int64_t evaluated_distinct;
} nnqs_stats;

/* Screen rules: a connection x' goes to the network when
 *   NNQS_SKIP_RATIO:        pred(x') >= log|psi(x)| - skip_nats
 *   NNQS_SKIP_CONTRIBUTION: log|H_xx'| + pred(x') >= log|psi(x)| - skip_nats
 * (the second bounds the skipped term |H_xx' psi(x')/psi(x)| by
 * exp(-skip_nats) Ha when the prediction is right). */
enum { NNQS_SKIP_RATIO = 0, NNQS_SKIP_CONTRIBUTION = 1 };

/* Options of nnqs_eloc_model (NULL = {12, NNQS_SKIP_RATIO, 0, NNQS_BF16, 0}).
 * screen_precision selects the screen's inference: NNQS_BF16 or NNQS_FP8
 * (hidden layer on FP8 MFMA).
 * refine_nats > 0 turns on the precision ladder for a lower-precision
 * network: the samples' own amplitudes come from the FP64 network, and every
 * connection whose first-pass contribution |H_xx' psi(x')/psi(x)| is at
 * least exp(-refine_nats) Ha (and the diagonal) is evaluated again by the
 * FP64 network, so the lower precision only touches the terms below that
 * size. */
typedef struct {
    double skip_nats;
    int32_t skip_rule;
    double refine_nats;
    int32_t screen_precision;
    /* BF16 / FP8 only: nonzero evaluates every distinct x' of a chunk once,
     * however many samples connect to it (the kept connections are sorted by
     * key; each run of equal keys is evaluated from the sample whose first
     * changed position is the latest, the fewest rows, and the result copied
     * to the others; with refinement a run is refined when any of its terms
     * qualifies).  Chunks then hold up to 2^27 connections, so that many
     * samples share one chunk.  Synchronises `stream` once per chunk. */
    int32_t dedup;
} nnqs_eloc_opts;

/* Full local energies (Eq. 4 over every connected x', psi from the model,
 * the samples' own psi from the model too) of n samples (device keys [n][2],
 * counts [n]) into device eloc [n][2] and energy [4] (layout as in
 * nnqs_eloc_table; energy may be NULL).  With a screen (may be NULL), only
 * the diagonal and the connections the screen rule of `opts` keeps are
 * evaluated by the network; the rest contribute zero.  The network runs in
 * `precision` (then, with refinement, FP64 for the large terms); matrix
 * elements, amplitude ratios and all sums are FP64 with compensated
 * summation.  In BF16 each chunk's samples run through the network once,
 * keeping every layer's keys and values; a connected x' whose first changed
 * sequence position s0 lies in row block b = min(3, s0 / 16) then evaluates
 * only rows from 16 b on, attending to the sample's cached rows before (by
 * causality of the attention and of the autoregressive product of Eq. 8 the
 * rows up to s0 equal the sample's; results are identical to the whole
 * forward of x').  The FP64 refinement runs each refined x' from row s0
 * itself, reading the sample's FP64 keys and values below it.  `stats`
 * (host, may be NULL) receives the counters; with refinement (or a screen in
 * FP64) or stats the call synchronises `stream` (the refined and selected
 * counts size the following launches), so such a call cannot be captured
 * into a graph; without them, once its scratch has grown (a first call of
 * the same size), the call makes no host synchronisation and can be.
 * Uses library-owned scratch sized at first use (one call at a time per
 * model).
 * Errors: EINVAL, ECONSERVE (VALIDATE), ENOMEM, EUNSUPPORTED, EHIP. */
nnqs_status nnqs_eloc_model(const nnqs_system *sys, nnqs_model *model, nnqs_screen *screen,
                            const nnqs_eloc_opts *opts, int32_t precision, const uint64_t *keys,
                            const uint32_t *counts, int64_t n, double *eloc, double *energy, nnqs_stats *stats,
                            uint32_t flags, void *stream);

/* Fallback judge of a screen (the plain evaluation is the fallback): the
 * root-mean-square error, in nats, of its predictions in `precision` against
 * target log|psi| on pairs it was not trained on (device xkeys [n][2],
 * exc [n][4], target [n]) into *rmse (host), and *usable (host, may be NULL)
 * = 1 when rmse <= max_rmse, else 0.  Synchronises `stream`.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EHIP. */
nnqs_status nnqs_screen_judge(nnqs_screen *screen, const uint64_t *xkeys, const uint8_t *exc, const double *target,
                              int64_t n, int32_t precision, double max_rmse, double *rmse, int32_t *usable,
                              void *stream);

/* ---------------------------------------------------------- measurement */
/* Timing of the library's own hot launches: with enable = 1 (which also
 * clears earlier records) every launch of k_transformer_bf16 (whole
 * sequences), k_transformer_bf16_list (prefix-reusing connections),
 * k_phase_bf16 and k_screen_infer is bracketed by HIP events recorded on the
 * stream it runs on; enable = 0 stops recording.  Not for use while a stream
 * is being captured into a graph. */
nnqs_status nnqs_timing_enable(int32_t enable);

/* Waits for the recorded events and returns the summed duration (ms) and
 * the number of recorded launches of `kernel` since the last enable.
 * Errors: EINVAL, EHIP. */
nnqs_status nnqs_timing_read(const char *kernel, double *total_ms, int64_t *launches);

/* ------------------------------------------------------------- tuning */
/* Launch parameters of the sample-aware kernel (0 = library default). */
typedef struct {
    int32_t waves_per_block;   /* 1..16 (the batched launch uses at most 12) */
    int32_t blocks_per_cu;     /* grid = blocks_per_cu * CU count */
    int32_t filter_log2_bits;  /* LDS membership filter size, 10..20 (2^k bits) */
    int32_t splitter_levels;   /* binary-search levels staged in LDS, 1..13 */
    int32_t search;            /* table levels below the LDS ones: 1 = one load per level,
                                  2 = three levels per round of independent loads */
    int32_t tile_samples;      /* batched launch: samples per work tile, 1..65536 */
} nnqs_tune;

/* Sets the launch parameters used by later nnqs_eloc_table calls on `tab`.
 * NULL restores the defaults.  Errors: EINVAL (out of range). */
nnqs_status nnqs_table_set_tune(nnqs_table *tab, const nnqs_tune *tune);

/* Reads back the parameters in use. */
nnqs_status nnqs_table_get_tune(const nnqs_table *tab, nnqs_tune *tune);

/* Autotuner of nnqs_eloc_table: times every candidate schedule (waves per
 * block {8, 12, 16} x splitter levels {8, 10, 12} x search {1, 2}) on the samples themselves (the table is
 * rebuilt from keys / logabs / phase for each), best of `reps` calls after
 * one warm-up call, and leaves `tab` built with the fastest, which it
 * returns (best, best_ms may be NULL).  eloc [n][2] is scratch.  Results do
 * not depend on the schedule beyond rounding order.  Synchronises `stream`.
 * Errors: EINVAL, EHIP and those of the build and evaluation. */
nnqs_status nnqs_table_autotune(const nnqs_system *sys, nnqs_table *tab, const uint64_t *keys, const double *logabs,
                                const double *phase, int64_t n, double *eloc, int32_t reps, nnqs_tune *best,
                                double *best_ms, void *stream);

/* Autotuner cache (host file, no GPU work).  nnqs_tune_key writes the key of
 * a sample-aware workload, "<arch>:cu<CUs>:K<K>:u<n_up>:d<n_dn>:n<samples>",
 * into out[cap] (ERANGE when it does not fit).  The cache is a text file of
 * lines "<key> <waves_per_block> <blocks_per_cu> <filter_log2_bits>
 * <splitter_levels> <search> <tile_samples> <ms>".  nnqs_tune_cache_lookup
 * sets *found = 1 and fills tune (and *ms, may be NULL) from the last valid
 * line of `key`, else *found = 0 (also when the file does not exist).
 * nnqs_tune_cache_store replaces the line of `key` (or appends one),
 * writing a temporary file next to `path` and renaming it over `path`.
 * Keys hold no white space.  Errors: EINVAL (null, bad key, tune out of
 * range, file not writable), ERANGE, EHIP. */
nnqs_status nnqs_tune_key(const nnqs_system *sys, int64_t n, char *out, int64_t cap);
nnqs_status nnqs_tune_cache_lookup(const char *path, const char *key, nnqs_tune *tune, double *ms, int32_t *found);
nnqs_status nnqs_tune_cache_store(const char *path, const char *key, const nnqs_tune *tune, double ms);

/* ------------------------------------------------- Pauli-string backend */
/* The paper's own formulation of the sample-aware local energy (Section 3.4
 * items 1, 2, 4, 5; Algorithms 1 and 2): the qubit Hamiltonian as Pauli
 * strings X^x Z^z, grouped by their X part (every string of a group couples
 * x to x ^ X), each group's strings listed with their Z part and a real
 * coefficient that already holds the sign (-1)^{|X & Z|}; then
 *   H_{x, x^X} = sum over the group of coef * (-1)^{|x & Z|}.
 * Jordan-Wigner strings over lower indices, spin orbital p = 2i + spin. */
typedef struct nnqs_pauli nnqs_pauli;

/* Host-only builder (no GPU): the grouped Pauli form of the Hamiltonian of
 * Eq. 9 from spatial chemists' integrals (layout as nnqs_system_create).
 * With all four arrays NULL it only returns the sizes in *n_groups and
 * *n_strings; otherwise *n_groups / *n_strings give the capacities on entry
 * and receive the sizes: xy [n_groups][2] (X part, groups sorted by it),
 * idx [n_groups + 1] (string ranges), zm [n_strings][2], coef [n_strings].
 * Errors: EINVAL (arguments, complex coefficients), ERANGE (capacity). */
nnqs_status nnqs_pauli_build_host(int32_t n_spin_orb, const double *h, const double *g, double e_core,
                                  int64_t *n_groups, int64_t *n_strings, uint64_t *xy, int64_t *idx, uint64_t *zm,
                                  double *coef);

/* Builds the grouped Pauli form of `sys` on the host and uploads it.
 * Synchronous.  Errors: EINVAL, ENOMEM, EHIP. */
nnqs_status nnqs_pauli_create(nnqs_pauli **out, const nnqs_system *sys);

/* Releases it.  NULL is accepted. */
nnqs_status nnqs_pauli_destroy(nnqs_pauli *pauli);

/* Sizes: groups, strings, bytes of the grouped layout (per group an X tuple
 * and an index, per string a Z tuple and a coefficient) and of the flat
 * layout (per string X and Z tuples, a Y count and a coefficient); tuples
 * take 8 bytes for N <= 64, else 16.  Any output may be NULL. */
nnqs_status nnqs_pauli_info(const nnqs_pauli *pauli, int64_t *n_groups, int64_t *n_strings, int64_t *bytes_grouped,
                            int64_t *bytes_flat);

/* Sample-aware E_loc over the Pauli groups (same inputs, outputs and error
 * model as nnqs_eloc_table; the same operator, so the same result up to
 * rounding).  Errors: EINVAL, EUNSUPPORTED, EHIP. */
nnqs_status nnqs_eloc_pauli(const nnqs_pauli *pauli, nnqs_table *tab, const uint64_t *keys, const uint32_t *counts,
                            const double *logabs, const double *phase, int64_t n, double *eloc, double *energy,
                            uint32_t flags, void *stream);

/* ------------------------------------------------------------ batching */
/* Many systems (uneven N, electron and sample counts) evaluated by one
 * persistent sample-aware launch.  A step of a batch: for every item with a
 * model, log|psi| and phase of its samples from the BF16 network (written to
 * the item's logabs / phase); for every item, its table built from the
 * samples; one persistent launch over all (system, sample-tile) work items,
 * pulled by blocks from a device counter; for every item with `energy`, the
 * weighted energy (Eq. 6).  A step neither synchronises the host nor
 * allocates, so it can be captured into a hipGraph and replayed. */
typedef struct nnqs_batch nnqs_batch;

typedef struct {
    const nnqs_system *system;
    nnqs_table *table;        /* of `system`, capacity >= n; rebuilt every step */
    nnqs_model *model;        /* NULL: logabs / phase are inputs; else outputs of the model (BF16) */
    const uint64_t *keys;     /* device [n][2], unique samples */
    const uint32_t *counts;   /* device [n], may be NULL when energy is NULL */
    double *logabs, *phase;   /* device [n] */
    int64_t n;
    double *eloc;             /* device [n][2] output */
    double *energy;           /* device [4] output, may be NULL */
} nnqs_batch_item;

/* Plans a batch over n_items items (device buffers stay owned by the caller
 * and must outlive the batch; the tables take the batch's tune).  The tune
 * starts from the first table's.  Synchronous.  Errors: EINVAL, ENOMEM,
 * EUNSUPPORTED, EHIP. */
nnqs_status nnqs_batch_create(nnqs_batch **out, const nnqs_batch_item *items, int32_t n_items);

/* Releases the batch (and its graph).  NULL is accepted. */
nnqs_status nnqs_batch_destroy(nnqs_batch *batch);

/* Enqueues one step on `stream`.  Errors: EHIP and those of the table build. */
nnqs_status nnqs_batch_run(nnqs_batch *batch, void *stream);

/* Records one step on `stream` (a created stream, not the null stream) into
 * a hipGraph owned by the batch, replacing any earlier one.  Nothing runs. */
nnqs_status nnqs_batch_capture(nnqs_batch *batch, void *stream);

/* Replays the captured step on `stream`.  Errors: EINVAL (nothing captured). */
nnqs_status nnqs_batch_launch(nnqs_batch *batch, void *stream);

/* Schedule of the batch (waves_per_block, blocks_per_cu, filter_log2_bits,
 * splitter_levels, search, tile_samples; 0 keeps a field).  Changing it
 * drops a captured graph.  Synchronous. */
nnqs_status nnqs_batch_set_tune(nnqs_batch *batch, const nnqs_tune *tune);
nnqs_status nnqs_batch_get_tune(const nnqs_batch *batch, nnqs_tune *tune);

/* Autotuner: times every candidate schedule (waves per block {8, 12} x
 * splitter levels {8, 10, 12} x search {1, 2} x tile samples {64, 256, 1024})
 * on the batch itself, best of `reps` steps after one warm-up step each,
 * keeps the fastest and returns it (best, best_ms may be NULL).  Runs many
 * steps on `stream` and synchronises it; drops a captured graph. */
nnqs_status nnqs_batch_autotune(nnqs_batch *batch, int32_t reps, nnqs_tune *best, double *best_ms, void *stream);

/* ------------------------------------------- batched transformer mode */
/* Full local energies (nnqs_eloc_model in BF16, no screen) of many systems
 * of uneven N, electron and sample counts in one step: per item its
 * connections are enumerated, its samples run once through its network
 * (keys and values cached) and its connections are sorted into prefix
 * classes; one persistent launch of the prefix-reusing forward then covers
 * the connections of every item (each tile evaluated with its item's
 * model); then per item the FP64 sums and the energy (Eq. 6).  A step
 * neither synchronises nor allocates, so it can be captured into a
 * hipGraph and replayed. */
typedef struct nnqs_batch_model nnqs_batch_model;

typedef struct {
    const nnqs_system *system;
    nnqs_model *model;        /* of `system`, BF16-capable; one item per model */
    const uint64_t *keys;     /* device [n][2], unique samples */
    const uint32_t *counts;   /* device [n], may be NULL when energy is NULL */
    int64_t n;                /* 1..4096 samples, n * C < 2^31 */
    double *eloc;             /* device [n][2] output */
    double *energy;           /* device [4] output (layout as nnqs_eloc_table), may be NULL */
} nnqs_batch_model_item;

/* Plans a batch of 1..64 items (device buffers stay owned by the caller and
 * must outlive the batch) and allocates its scratch (per item about
 * 40 n C bytes plus 64 KiB per sample).  Synchronous.
 * Errors: EINVAL, ERANGE, ENOMEM, EUNSUPPORTED, EHIP. */
nnqs_status nnqs_batch_model_create(nnqs_batch_model **out, const nnqs_batch_model_item *items, int32_t n_items);

/* Releases the batch, its scratch and its graph.  NULL is accepted. */
nnqs_status nnqs_batch_model_destroy(nnqs_batch_model *batch);

/* Enqueues one step on `stream`.  Errors: EHIP. */
nnqs_status nnqs_batch_model_run(nnqs_batch_model *batch, void *stream);

/* Records one step on `stream` (a created stream) into a hipGraph owned by
 * the batch, replacing any earlier one.  Nothing runs. */
nnqs_status nnqs_batch_model_capture(nnqs_batch_model *batch, void *stream);

/* Replays the captured step.  Errors: EINVAL (nothing captured), EHIP. */
nnqs_status nnqs_batch_model_launch(nnqs_batch_model *batch, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NNQS_ELOC_H */

/*
 * Plain FP64 CPU oracle for the local energy of a second-quantised molecular
 * Hamiltonian.  TEST INFRASTRUCTURE: only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library; the product
 * path never does.  It shares no source with the HIP library.
 *
 * What it computes (paper: Section 2.1 Eq. 4 local energy; Eq. 6 sample mean
 * with the unique-sample weights of Section 3.1; Eq. 9 Hamiltonian; Section
 * 3.4 items 4-5 sample-aware evaluation over a sorted table of packed keys):
 *
 *   E_loc(x) = sum_{x'} H_{x x'} psi(x') / psi(x)
 *            = sum_{x'} H_{x x'} exp((l' - l) + i (phi' - phi))
 *
 * with psi = exp(l + i phi) and, in the sample-aware form, x' restricted to
 * the table of unique samples.
 *
 * Conventions (readings of the paper, stated once):
 *  - spin orbital p = 2*i + s, s = 0 up, 1 down; key bit p = occupation of p;
 *    word 0 holds bits 0..63, word 1 bits 64..127;
 *  - Jordan-Wigner string over lower indices:
 *      a_p |x> = x_p (-1)^{#occupied q < p} |x - e_p>,
 *      a+_p|x> = (1 - x_p) (-1)^{#occupied q < p} |x + e_p>;
 *  - H = E_core + sum_pq h_pq a+_p a_q + 1/2 sum_pqrs <pq|rs> a+_p a+_q a_s a_r
 *    with <pq|rs> = (i_p i_r | i_q i_s) delta(s_p,s_r) delta(s_q,s_s) and
 *    (ij|kl) the spatial chemists'-notation integrals g[((i*K+j)*K+k)*K+l].
 *
 * Every matrix element is found by the textbook Slater-Condon rules from the
 * pair (x, x') and its sign by literally applying the operator string to x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------ bit helpers */
static int bit_of(const uint64_t *x, int p) { return (int)((x[p >> 6] >> (p & 63)) & 1u); }
static void flip_bit(uint64_t *x, int p) { x[p >> 6] ^= (uint64_t)1 << (p & 63); }

/* number of occupied spin orbitals with index below p (the JW string) */
static int occupied_below(const uint64_t *x, int p) {
    int c = 0;
    for (int q = 0; q < p; q++) c += bit_of(x, q);
    return c;
}

/* apply a_p in place; returns the sign, or 0 if the result vanishes */
static int apply_annihilate(uint64_t *x, int p) {
    if (!bit_of(x, p)) return 0;
    int s = (occupied_below(x, p) & 1) ? -1 : 1;
    flip_bit(x, p);
    return s;
}

/* apply a+_p in place; returns the sign, or 0 if the result vanishes */
static int apply_create(uint64_t *x, int p) {
    if (bit_of(x, p)) return 0;
    int s = (occupied_below(x, p) & 1) ? -1 : 1;
    flip_bit(x, p);
    return s;
}

static int popcount128(const uint64_t *x) {
    int c = 0;
    for (int p = 0; p < 128; p++) c += bit_of(x, p);
    return c;
}

/* ------------------------------------------------------------- integrals */
typedef struct {
    int K;
    const double *h;
    const double *g;
    double ecore;
} ora_ham;

static double one_body(const ora_ham *H, int p, int q) {
    if ((p & 1) != (q & 1)) return 0.0;
    return H->h[(p >> 1) * H->K + (q >> 1)];
}

/* physicists' <pq|rs> over spin orbitals */
static double phys(const ora_ham *H, int p, int q, int r, int s) {
    if ((p & 1) != (r & 1) || (q & 1) != (s & 1)) return 0.0;
    int K = H->K;
    int i = p >> 1, j = r >> 1, k = q >> 1, l = s >> 1; /* (p r | q s) */
    return H->g[(((size_t)i * K + j) * K + k) * K + l];
}

/* ----------------------------------------------------- Slater-Condon rules */
/* <x'|H|x> (= <x|H|x'>, H is real symmetric).  *sign_out receives the sign of
 * the excitation operator applied to x (1 for the diagonal, 0 if unconnected). */
static double slater_condon(const ora_ham *H, const uint64_t *x, const uint64_t *xp, int *sign_out) {
    int N = 2 * H->K;
    int removed[4], added[4], nr = 0, na = 0;
    for (int p = 0; p < N; p++) {
        int a = bit_of(x, p), b = bit_of(xp, p);
        if (a && !b) {
            if (nr == 4) { *sign_out = 0; return 0.0; }
            removed[nr++] = p;
        } else if (!a && b) {
            if (na == 4) { *sign_out = 0; return 0.0; }
            added[na++] = p;
        }
    }
    if (nr != na || nr > 2) { *sign_out = 0; return 0.0; }
    if (nr == 0) { /* diagonal */
        double e = H->ecore;
        for (int p = 0; p < N; p++) {
            if (!bit_of(x, p)) continue;
            e += one_body(H, p, p);
            for (int q = 0; q < N; q++) {
                if (!bit_of(x, q)) continue;
                e += 0.5 * (phys(H, p, q, p, q) - phys(H, p, q, q, p));
            }
        }
        *sign_out = 1;
        return e;
    }
    if (nr == 1) { /* single: x' = a+_p a_q x */
        int q = removed[0], p = added[0];
        uint64_t y[2] = {x[0], x[1]};
        int s = apply_annihilate(y, q);
        s *= apply_create(y, p);
        double v = one_body(H, p, q);
        for (int k = 0; k < N; k++) {
            if (!bit_of(x, k)) continue;
            v += phys(H, p, k, q, k) - phys(H, p, k, k, q);
        }
        *sign_out = s;
        return s * v;
    }
    /* double: x' = a+_a a+_b a_j a_i x with i<j, a<b */
    int i = removed[0], j = removed[1], a = added[0], b = added[1];
    uint64_t y[2] = {x[0], x[1]};
    int s = apply_annihilate(y, i);
    s *= apply_annihilate(y, j);
    s *= apply_create(y, b);
    s *= apply_create(y, a);
    *sign_out = s;
    return s * (phys(H, a, b, i, j) - phys(H, a, b, j, i));
}

/* ------------------------------------------------------ connection lists */
typedef struct {
    int n_occ[2], n_vir[2];
    int occ[2][64], vir[2][64];
} orbital_lists;

static void build_lists(int K, const uint64_t *x, orbital_lists *L) {
    for (int s = 0; s < 2; s++) {
        L->n_occ[s] = L->n_vir[s] = 0;
        for (int i = 0; i < K; i++) {
            int p = 2 * i + s;
            if (bit_of(x, p)) L->occ[s][L->n_occ[s]++] = p;
            else L->vir[s][L->n_vir[s]++] = p;
        }
    }
}

int64_t ora_n_connections(int K, int n_up, int n_dn) {
    int64_t vu = K - n_up, vd = K - n_dn;
    int64_t pu = (int64_t)n_up * (n_up - 1) / 2, pd = (int64_t)n_dn * (n_dn - 1) / 2;
    return 1 + n_up * vu + n_dn * vd + pu * (vu * (vu - 1) / 2) + pd * (vd * (vd - 1) / 2) +
           n_up * vu * n_dn * vd;
}

/* Enumerates the connected configurations of x in the canonical order
 *   diagonal; singles up, singles down (occupied rank, virtual rank);
 *   same-spin doubles up, down (occupied pair, virtual pair, each
 *   lexicographic in rank); opposite-spin doubles (i_up, a_up, j_dn, b_dn).
 * exc receives (i, j, a, b) as sorted spin-orbital indices, 255 where absent.
 * Returns the number written. */
static int64_t enumerate(int K, const uint64_t *x, uint64_t *xp, uint8_t *exc) {
    orbital_lists L;
    build_lists(K, x, &L);
    int64_t c = 0;
#define EMIT(I, J, A, B)                                                                     \
    do {                                                                                     \
        uint64_t y[2] = {x[0], x[1]};                                                        \
        int e_[4] = {(I), (J), (A), (B)};                                                    \
        for (int t_ = 0; t_ < 4; t_++)                                                       \
            if (e_[t_] >= 0) flip_bit(y, e_[t_]);                                            \
        xp[2 * c] = y[0];                                                                    \
        xp[2 * c + 1] = y[1];                                                                \
        if (exc) {                                                                           \
            int lo = (I), hi = (J), al = (A), ah = (B);                                      \
            if (hi >= 0 && hi < lo) { int t2 = lo; lo = hi; hi = t2; }                       \
            if (ah >= 0 && ah < al) { int t2 = al; al = ah; ah = t2; }                       \
            exc[4 * c + 0] = (uint8_t)(lo < 0 ? 255 : lo);                                   \
            exc[4 * c + 1] = (uint8_t)(hi < 0 ? 255 : hi);                                   \
            exc[4 * c + 2] = (uint8_t)(al < 0 ? 255 : al);                                   \
            exc[4 * c + 3] = (uint8_t)(ah < 0 ? 255 : ah);                                   \
        }                                                                                    \
        c++;                                                                                 \
    } while (0)
    EMIT(-1, -1, -1, -1);
    for (int s = 0; s < 2; s++)
        for (int o = 0; o < L.n_occ[s]; o++)
            for (int v = 0; v < L.n_vir[s]; v++) EMIT(L.occ[s][o], -1, L.vir[s][v], -1);
    for (int s = 0; s < 2; s++)
        for (int o1 = 0; o1 < L.n_occ[s]; o1++)
            for (int o2 = o1 + 1; o2 < L.n_occ[s]; o2++)
                for (int v1 = 0; v1 < L.n_vir[s]; v1++)
                    for (int v2 = v1 + 1; v2 < L.n_vir[s]; v2++)
                        EMIT(L.occ[s][o1], L.occ[s][o2], L.vir[s][v1], L.vir[s][v2]);
    for (int ou = 0; ou < L.n_occ[0]; ou++)
        for (int vu = 0; vu < L.n_vir[0]; vu++)
            for (int od = 0; od < L.n_occ[1]; od++)
                for (int vd = 0; vd < L.n_vir[1]; vd++)
                    EMIT(L.occ[0][ou], L.occ[1][od], L.vir[0][vu], L.vir[1][vd]);
#undef EMIT
    return c;
}

/* Public: general matrix element <x'|H|x>; sign_out may be NULL. */
double ora_hxx(int K, const double *h, const double *g, double ecore, const uint64_t *x,
               const uint64_t *xp, int *sign_out) {
    ora_ham H = {K, h, g, ecore};
    int s;
    double v = slater_condon(&H, x, xp, &s);
    if (sign_out) *sign_out = s;
    return v;
}

/* Public: all connections of one configuration, canonical order.  Returns the
 * count, or -1 if x violates the particle numbers. */
int64_t ora_connections(int K, int n_up, int n_dn, const double *h, const double *g, double ecore,
                        const uint64_t *x, uint64_t *xp, int8_t *sign, uint8_t *exc, double *hxx) {
    int nu = 0, nd = 0;
    for (int i = 0; i < K; i++) {
        nu += bit_of(x, 2 * i);
        nd += bit_of(x, 2 * i + 1);
    }
    if (nu != n_up || nd != n_dn || popcount128(x) != nu + nd) return -1;
    ora_ham H = {K, h, g, ecore};
    int64_t C = enumerate(K, x, xp, exc);
    for (int64_t c = 0; c < C; c++) {
        int s;
        double v = slater_condon(&H, x, xp + 2 * c, &s);
        if (sign) sign[c] = (int8_t)s;
        if (hxx) hxx[c] = v;
    }
    return C;
}

/* ------------------------------------------------ compensated summation */
/* Neumaier's improved Kahan-Babuska summation. */
typedef struct { double s, c; } neumaier;
static void nsum_add(neumaier *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_value(const neumaier *a) { return a->s + a->c; }

/* ------------------------------------------------ sorted sample table */
typedef struct {
    uint64_t w0, w1;
    double logabs, phase;
} table_entry;

/* unsigned 128-bit order, word 1 major */
static int cmp_entry(const void *pa, const void *pb) {
    const table_entry *a = (const table_entry *)pa, *b = (const table_entry *)pb;
    if (a->w1 != b->w1) return a->w1 < b->w1 ? -1 : 1;
    if (a->w0 != b->w0) return a->w0 < b->w0 ? -1 : 1;
    return 0;
}

static table_entry *make_table(const uint64_t *tkeys, const double *tl, const double *tp, int64_t nt) {
    table_entry *T = (table_entry *)malloc(sizeof(table_entry) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t i = 0; i < nt; i++) {
        T[i].w0 = tkeys[2 * i];
        T[i].w1 = tkeys[2 * i + 1];
        T[i].logabs = tl[i];
        T[i].phase = tp[i];
    }
    qsort(T, (size_t)nt, sizeof(table_entry), cmp_entry);
    return T;
}

/* Public: sort a table (keys + payload) with the C library's qsort; used to
 * check the device table build.  Returns 1 if the keys are unique, 0 if not. */
int ora_sort_table(const uint64_t *tkeys, const double *tl, const double *tp, int64_t nt,
                   uint64_t *keys_out, double *l_out, double *p_out) {
    table_entry *T = make_table(tkeys, tl, tp, nt);
    int unique = 1;
    for (int64_t i = 0; i < nt; i++) {
        keys_out[2 * i] = T[i].w0;
        keys_out[2 * i + 1] = T[i].w1;
        l_out[i] = T[i].logabs;
        p_out[i] = T[i].phase;
        if (i > 0 && cmp_entry(&T[i - 1], &T[i]) == 0) unique = 0;
    }
    free(T);
    return unique;
}

/* Public: sample-aware local energies (x' restricted to the table).
 * eloc[2*k] = Re, eloc[2*k+1] = Im; absum[k] (optional) receives
 * sum |H_xx'| |psi(x')/psi(x)| over the hits, the scale used for tolerances.
 * Returns 0, or -1 if a sample violates the particle numbers. */
int ora_eloc_table(int K, int n_up, int n_dn, const double *h, const double *g, double ecore,
                   const uint64_t *tkeys, const double *tlogabs, const double *tphase, int64_t nt,
                   const uint64_t *keys, const double *logabs, const double *phase, int64_t n,
                   double *eloc, double *absum, int nthreads) {
    ora_ham H = {K, h, g, ecore};
    table_entry *T = make_table(tkeys, tlogabs, tphase, nt);
    int64_t C = ora_n_connections(K, n_up, n_dn);
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        uint64_t *xp = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)C);
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < n; k++) {
            const uint64_t *x = keys + 2 * k;
            int nu = 0, nd = 0;
            for (int i = 0; i < K; i++) {
                nu += bit_of(x, 2 * i);
                nd += bit_of(x, 2 * i + 1);
            }
            if (nu != n_up || nd != n_dn || popcount128(x) != nu + nd) {
#pragma omp atomic write
                bad = 1;
                eloc[2 * k] = eloc[2 * k + 1] = NAN;
                continue;
            }
            int64_t cnt = enumerate(K, x, xp, NULL);
            neumaier re = {0, 0}, im = {0, 0}, ab = {0, 0};
            for (int64_t c = 0; c < cnt; c++) {
                table_entry probe = {xp[2 * c], xp[2 * c + 1], 0, 0};
                const table_entry *hit =
                    (const table_entry *)bsearch(&probe, T, (size_t)nt, sizeof(table_entry), cmp_entry);
                if (!hit) continue;
                int s;
                double hv = slater_condon(&H, x, xp + 2 * c, &s);
                double mag = exp(hit->logabs - logabs[k]);
                double ang = hit->phase - phase[k];
                nsum_add(&re, hv * mag * cos(ang));
                nsum_add(&im, hv * mag * sin(ang));
                nsum_add(&ab, fabs(hv) * mag);
            }
            eloc[2 * k] = nsum_value(&re);
            eloc[2 * k + 1] = nsum_value(&im);
            if (absum) absum[k] = nsum_value(&ab);
        }
        free(xp);
    }
    free(T);
    return bad ? -1 : 0;
}

/* Public: weighted energy of Eq. 6 over unique samples with occurrence
 * counts: out = {sum c Re / sum c, sum c Im / sum c, sum c,
 *                sum c (Re - E)^2 / sum c}. */
void ora_energy(const uint32_t *counts, const double *eloc, int64_t n, double *out) {
    neumaier w = {0, 0}, re = {0, 0}, im = {0, 0};
    for (int64_t k = 0; k < n; k++) {
        double c = (double)counts[k];
        nsum_add(&w, c);
        nsum_add(&re, c * eloc[2 * k]);
        nsum_add(&im, c * eloc[2 * k + 1]);
    }
    double W = nsum_value(&w);
    double E = nsum_value(&re) / W;
    neumaier var = {0, 0};
    for (int64_t k = 0; k < n; k++) {
        double d = eloc[2 * k] - E;
        nsum_add(&var, (double)counts[k] * d * d);
    }
    out[0] = E;
    out[1] = nsum_value(&im) / W;
    out[2] = W;
    out[3] = nsum_value(&var) / W;
}

/* ======================================================================
 * Amplitude and phase networks (paper: Section 3.1, Eq. 11 and Fig. 2:
 * a decoder-only transformer gives |psi|^2 autoregressively, an MLP gives the
 * phase; Section 4.1: phase MLP of three dense layers N x 512 x 512 x 1;
 * Section 3.3, Eq. 12: tokens are spatial-orbital pairs sampled in reverse
 * qubit order with the electron-number mask).  Readings where the paper is
 * silent: pre-LN blocks (eps 1e-5), causal multi-head attention scaled by
 * 1/sqrt(head dim), FFN with exact-erf GELU, input = embedding of the
 * previous token (a begin token 4 at the first position) + learned position
 * embedding, output head -> 4 logits + a fixed per-orbital bias, the mask also
 * forbids leaving more electrons than remaining positions, and
 * log|psi| = 1/2 sum_s log pi(t_s | t_<s).
 *
 * Weights arrive as one float64 array in this order (matrices [in][out]):
 *   tok_emb[5][d] pos_emb[K][d]
 *   per layer: ln1_g[d] ln1_b[d] wq[d][d] bq[d] wk[d][d] bk[d] wv[d][d] bv[d]
 *              wo[d][d] bo[d] ln2_g[d] ln2_b[d] w1[d][F] b1[F] w2[F][d] b2[d]
 *   lnf_g[d] lnf_b[d] head_w[d][4] head_b[4] logit_bias[K][4]
 *   ph_w1[2K][P] ph_b1[P] ph_w2[P][P] ph_b2[P] ph_w3[P][1] ph_b3[1]
 * ====================================================================== */
typedef struct {
    int K, d, L, H, F, P, n_up, n_dn;
} ora_net;

static double gelu(double v) { return 0.5 * v * (1.0 + erf(v / sqrt(2.0))); }

static void layer_norm(const double *x, const double *g, const double *b, int d, double *y) {
    double m = 0.0, v = 0.0;
    for (int c = 0; c < d; c++) m += x[c];
    m /= d;
    for (int c = 0; c < d; c++) v += (x[c] - m) * (x[c] - m);
    v /= d;
    double r = 1.0 / sqrt(v + 1e-5);
    for (int c = 0; c < d; c++) y[c] = (x[c] - m) * r * g[c] + b[c];
}

/* y[n] = x[m] W[m][n] + b[n] */
static void dense(const double *x, const double *W, const double *b, int m, int n, double *y) {
    for (int j = 0; j < n; j++) {
        double s = b ? b[j] : 0.0;
        for (int i = 0; i < m; i++) s += x[i] * W[(size_t)i * n + j];
        y[j] = s;
    }
}

int64_t ora_net_size(int K, int d, int L, int H, int F, int P) {
    (void)H;
    int64_t per = 2 * d + 4 * ((int64_t)d * d + d) + 2 * d + (int64_t)d * F + F + (int64_t)F * d + d;
    return 5 * (int64_t)d + (int64_t)K * d + L * per + 2 * d + 4 * (int64_t)d + 4 + 4 * (int64_t)K +
           (int64_t)2 * K * P + P + (int64_t)P * P + P + P + 1;
}

/* Token of the configuration at autoregressive position s (orbital K-1-s):
 * t = n_up + 2 n_dn of that spatial orbital. */
static int token_at(const uint64_t *x, int K, int s) {
    int i = K - 1 - s;
    return bit_of(x, 2 * i) + 2 * bit_of(x, 2 * i + 1);
}

/* Conditional log-probabilities logp[K][4] (masked entries -inf) of one
 * configuration under the amplitude transformer. */
static void transformer_conditionals(const ora_net *net, const double *w, const uint64_t *x, double *logp) {
    const int K = net->K, d = net->d, L = net->L, H = net->H, F = net->F;
    const int dh = d / H;
    const double *tok_emb = w, *pos_emb = w + 5 * d;
    const double *p = pos_emb + (size_t)K * d;
    double *h = (double *)malloc(sizeof(double) * K * d);
    double *a = (double *)malloc(sizeof(double) * K * d);
    double *q = (double *)malloc(sizeof(double) * K * d);
    double *k = (double *)malloc(sizeof(double) * K * d);
    double *v = (double *)malloc(sizeof(double) * K * d);
    double *o = (double *)malloc(sizeof(double) * K * d);
    double *f = (double *)malloc(sizeof(double) * F);
    double *t = (double *)malloc(sizeof(double) * d);
    double *sc = (double *)malloc(sizeof(double) * K);
    for (int s = 0; s < K; s++) {
        int prev = s == 0 ? 4 : token_at(x, K, s - 1);
        for (int c = 0; c < d; c++) h[s * d + c] = tok_emb[prev * d + c] + pos_emb[s * d + c];
    }
    for (int l = 0; l < L; l++) {
        const double *ln1_g = p, *ln1_b = p + d, *wq = p + 2 * d, *bq = wq + d * d, *wk = bq + d, *bk = wk + d * d,
                     *wv = bk + d, *bv = wv + d * d, *wo = bv + d, *bo = wo + d * d, *ln2_g = bo + d,
                     *ln2_b = ln2_g + d, *w1 = ln2_b + d, *b1 = w1 + (size_t)d * F, *w2 = b1 + F,
                     *b2 = w2 + (size_t)F * d;
        p = b2 + d;
        for (int s = 0; s < K; s++) {
            layer_norm(h + s * d, ln1_g, ln1_b, d, a + s * d);
            dense(a + s * d, wq, bq, d, d, q + s * d);
            dense(a + s * d, wk, bk, d, d, k + s * d);
            dense(a + s * d, wv, bv, d, d, v + s * d);
        }
        for (int s = 0; s < K; s++) {
            for (int hh = 0; hh < H; hh++) {
                double mx = -INFINITY;
                for (int r = 0; r <= s; r++) {
                    double z = 0.0;
                    for (int c = 0; c < dh; c++) z += q[s * d + hh * dh + c] * k[r * d + hh * dh + c];
                    sc[r] = z / sqrt((double)dh);
                    if (sc[r] > mx) mx = sc[r];
                }
                double den = 0.0;
                for (int r = 0; r <= s; r++) {
                    sc[r] = exp(sc[r] - mx);
                    den += sc[r];
                }
                for (int c = 0; c < dh; c++) {
                    double z = 0.0;
                    for (int r = 0; r <= s; r++) z += sc[r] * v[r * d + hh * dh + c];
                    o[s * d + hh * dh + c] = z / den;
                }
            }
        }
        for (int s = 0; s < K; s++) {
            dense(o + s * d, wo, bo, d, d, t);
            for (int c = 0; c < d; c++) h[s * d + c] += t[c];
            layer_norm(h + s * d, ln2_g, ln2_b, d, t);
            dense(t, w1, b1, d, F, f);
            for (int c = 0; c < F; c++) f[c] = gelu(f[c]);
            double *u = a + s * d; /* reuse as scratch row */
            dense(f, w2, b2, F, d, u);
            for (int c = 0; c < d; c++) h[s * d + c] += u[c];
        }
    }
    const double *lnf_g = p, *lnf_b = p + d, *head_w = p + 2 * d, *head_b = head_w + 4 * d,
                 *bias = head_b + 4;
    int up = 0, dn = 0;
    for (int s = 0; s < K; s++) {
        double z[4];
        layer_norm(h + s * d, lnf_g, lnf_b, d, t);
        dense(t, head_w, head_b, d, 4, z);
        int i = K - 1 - s, rem = K - 1 - s;
        double mx = -INFINITY;
        int allowed[4];
        for (int c = 0; c < 4; c++) {
            z[c] += bias[i * 4 + c];
            int bu = c & 1, bd = c >> 1;
            allowed[c] = (up + bu <= net->n_up) && (dn + bd <= net->n_dn) && (net->n_up - up - bu <= rem) &&
                         (net->n_dn - dn - bd <= rem);
            if (allowed[c] && z[c] > mx) mx = z[c];
        }
        double den = 0.0;
        for (int c = 0; c < 4; c++)
            if (allowed[c]) den += exp(z[c] - mx);
        for (int c = 0; c < 4; c++) logp[s * 4 + c] = allowed[c] ? (z[c] - mx) - log(den) : -INFINITY;
        int tk = token_at(x, K, s);
        up += tk & 1;
        dn += tk >> 1;
    }
    free(h); free(a); free(q); free(k); free(v); free(o); free(f); free(t); free(sc);
}

static const double *phase_weights(const ora_net *net, const double *w) {
    const int K = net->K, d = net->d, L = net->L, F = net->F;
    int64_t per = 2 * d + 4 * ((int64_t)d * d + d) + 2 * d + (int64_t)d * F + F + (int64_t)F * d + d;
    return w + 5 * (int64_t)d + (int64_t)K * d + L * per + 2 * d + 4 * (int64_t)d + 4 + 4 * (int64_t)K;
}

/* log|psi(x)| and phi(x) of one configuration. */
static void net_logpsi(const ora_net *net, const double *w, const uint64_t *x, double *logabs, double *phase) {
    const int K = net->K, N = 2 * K, P = net->P;
    double *lp = (double *)malloc(sizeof(double) * K * 4);
    transformer_conditionals(net, w, x, lp);
    double s = 0.0;
    for (int t = 0; t < K; t++) s += lp[t * 4 + token_at(x, K, t)];
    *logabs = 0.5 * s;
    free(lp);
    const double *w1 = phase_weights(net, w), *b1 = w1 + (size_t)N * P, *w2 = b1 + P, *b2 = w2 + (size_t)P * P,
                 *w3 = b2 + P, *b3 = w3 + P;
    double *in = (double *)malloc(sizeof(double) * N);
    double *z1 = (double *)malloc(sizeof(double) * P);
    double *z2 = (double *)malloc(sizeof(double) * P);
    for (int q = 0; q < N; q++) in[q] = bit_of(x, q);
    dense(in, w1, b1, N, P, z1);
    for (int c = 0; c < P; c++) z1[c] = gelu(z1[c]);
    dense(z1, w2, b2, P, P, z2);
    for (int c = 0; c < P; c++) z2[c] = gelu(z2[c]);
    double ph;
    dense(z2, w3, b3, P, 1, &ph);
    *phase = ph;
    free(in); free(z1); free(z2);
}

/* Public: conditionals of one configuration (for causality checks). */
void ora_net_conditionals(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w,
                          const uint64_t *x, double *logp) {
    ora_net net = {K, d, L, H, F, P, n_up, n_dn};
    transformer_conditionals(&net, w, x, logp);
}

/* Public: log|psi| and phase of n configurations. */
void ora_net_logpsi(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w,
                    const uint64_t *keys, int64_t n, double *logabs, double *phase, int nthreads) {
    ora_net net = {K, d, L, H, F, P, n_up, n_dn};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; k++) net_logpsi(&net, w, keys + 2 * k, logabs + k, phase + k);
}

/* Public: full local energies, every connected x' evaluated by the networks
 * (Eq. 4 over all x' with H_xx' != 0).  The sample's own amplitude is the
 * network's as well.  absum as in ora_eloc_table. */
int ora_eloc_model(int K, int n_up, int n_dn, const double *h, const double *g, double ecore, int d, int L,
                   int H, int F, int P, const double *w, const uint64_t *keys, int64_t n, double *eloc,
                   double *absum, int nthreads) {
    ora_ham Ham = {K, h, g, ecore};
    ora_net net = {K, d, L, H, F, P, n_up, n_dn};
    int64_t C = ora_n_connections(K, n_up, n_dn);
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int64_t k = 0; k < n; k++) {
        const uint64_t *x = keys + 2 * k;
        int nu = 0, nd = 0;
        for (int i = 0; i < K; i++) {
            nu += bit_of(x, 2 * i);
            nd += bit_of(x, 2 * i + 1);
        }
        if (nu != n_up || nd != n_dn || popcount128(x) != nu + nd) {
            bad = 1;
            eloc[2 * k] = eloc[2 * k + 1] = NAN;
            continue;
        }
        double l0, p0;
        net_logpsi(&net, w, x, &l0, &p0);
        uint64_t *xp = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)C);
        double *lv = (double *)malloc(sizeof(double) * (size_t)C);
        double *pv = (double *)malloc(sizeof(double) * (size_t)C);
        int64_t cnt = enumerate(K, x, xp, NULL);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t c = 0; c < cnt; c++) net_logpsi(&net, w, xp + 2 * c, lv + c, pv + c);
        neumaier re = {0, 0}, im = {0, 0}, ab = {0, 0};
        for (int64_t c = 0; c < cnt; c++) {
            int s;
            double hv = slater_condon(&Ham, x, xp + 2 * c, &s);
            double mag = exp(lv[c] - l0);
            nsum_add(&re, hv * mag * cos(pv[c] - p0));
            nsum_add(&im, hv * mag * sin(pv[c] - p0));
            nsum_add(&ab, fabs(hv) * mag);
        }
        eloc[2 * k] = nsum_value(&re);
        eloc[2 * k + 1] = nsum_value(&im);
        if (absum) absum[k] = nsum_value(&ab);
        free(xp); free(lv); free(pv);
    }
    return bad ? -1 : 0;
}

/* ======================================================================
 * Learned screen (not in the paper: its only filter is the sample-aware
 * restriction of Section 3.4 item 4).  An MLP predicts log|psi(x')| from the
 * occupation bits of x' and one-hot codes of the excitation indices
 * (i, j, a, b) (sorted, absent indices give all-zero codes):
 *   u = [bits(x') | onehot(i) | onehot(j) | onehot(a) | onehot(b)]  (5N)
 *   z1 = GELU(u W1 + b1), z2 = GELU(z1 W2 + b2), y = z2 . w3 + b3.
 * Weights (float64): W1[5N][H] b1[H] W2[H][H] b2[H] w3[H] b3[1].
 * Training: mean squared error, Adam with bias correction.
 * ====================================================================== */
int64_t ora_screen_size(int N, int H) { return (int64_t)5 * N * H + H + (int64_t)H * H + H + H + 1; }

static void screen_input(int N, const uint64_t *x, const uint8_t *e, double *u) {
    for (int p = 0; p < 5 * N; p++) u[p] = 0.0;
    for (int p = 0; p < N; p++) u[p] = bit_of(x, p);
    for (int t = 0; t < 4; t++) /* 255 marks an absent index; other codes >= N are ignored too */
        if (e[t] < N) u[(t + 1) * N + e[t]] = 1.0;
}

static double gelu_grad(double v) {
    const double pdf = exp(-0.5 * v * v) * 0.39894228040143267794; /* 1/sqrt(2 pi) */
    return 0.5 * (1.0 + erf(v / sqrt(2.0))) + v * pdf;
}

/* forward of one example; keeps pre-activations for the backward pass */
static double screen_one(int N, int H, const double *w, const double *u, double *a1, double *a2) {
    const double *W1 = w, *b1 = W1 + (size_t)5 * N * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H, *w3 = b2 + H,
                 *b3 = w3 + H;
    dense(u, W1, b1, 5 * N, H, a1);
    double *z1 = (double *)calloc((size_t)H, sizeof(double));
    for (int c = 0; c < H; c++) z1[c] = gelu(a1[c]);
    dense(z1, W2, b2, H, H, a2);
    double y = b3[0];
    for (int c = 0; c < H; c++) y += gelu(a2[c]) * w3[c];
    free(z1);
    return y;
}

void ora_screen_forward(int N, int H, const double *w, const uint64_t *keys, const uint8_t *exc, int64_t n,
                        double *pred) {
    double *u = (double *)malloc(sizeof(double) * 5 * N);
    double *a1 = (double *)malloc(sizeof(double) * H), *a2 = (double *)malloc(sizeof(double) * H);
    for (int64_t k = 0; k < n; k++) {
        screen_input(N, keys + 2 * k, exc + 4 * k, u);
        pred[k] = screen_one(N, H, w, u, a1, a2);
    }
    free(u); free(a1); free(a2);
}

/* loss = mean_k (pred_k - target_k)^2 and its gradient w.r.t. every weight */
double ora_screen_loss_grad(int N, int H, const double *w, const uint64_t *keys, const uint8_t *exc,
                            const double *target, int64_t n, double *grad) {
    const int64_t size = ora_screen_size(N, H);
    const double *W2 = w + (size_t)5 * N * H + H, *w3 = W2 + (size_t)H * H + H;
    double *gW1 = grad, *gb1 = gW1 + (size_t)5 * N * H, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H,
           *gw3 = gb2 + H, *gb3 = gw3 + H;
    for (int64_t q = 0; q < size; q++) grad[q] = 0.0;
    double *u = (double *)malloc(sizeof(double) * 5 * N);
    double *a1 = (double *)malloc(sizeof(double) * H), *a2 = (double *)malloc(sizeof(double) * H);
    double *d2 = (double *)malloc(sizeof(double) * H), *d1 = (double *)malloc(sizeof(double) * H);
    double loss = 0.0;
    for (int64_t k = 0; k < n; k++) {
        screen_input(N, keys + 2 * k, exc + 4 * k, u);
        const double y = screen_one(N, H, w, u, a1, a2);
        const double r = y - target[k];
        loss += r * r;
        const double gy = 2.0 * r / (double)n;
        gb3[0] += gy;
        for (int c = 0; c < H; c++) {
            gw3[c] += gy * gelu(a2[c]);
            d2[c] = gy * w3[c] * gelu_grad(a2[c]);
        }
        for (int c = 0; c < H; c++) {
            gb2[c] += d2[c];
            const double z = gelu(a1[c]);
            for (int j = 0; j < H; j++) gW2[(size_t)c * H + j] += z * d2[j];
        }
        for (int c = 0; c < H; c++) {
            double s = 0.0;
            for (int j = 0; j < H; j++) s += W2[(size_t)c * H + j] * d2[j];
            d1[c] = s * gelu_grad(a1[c]);
            gb1[c] += d1[c];
        }
        for (int p = 0; p < 5 * N; p++)
            if (u[p] != 0.0)
                for (int c = 0; c < H; c++) gW1[(size_t)p * H + c] += u[p] * d1[c];
    }
    free(u); free(a1); free(a2); free(d1); free(d2);
    return loss / (double)n;
}

/* Adam (Kingma & Ba 2015) with bias correction, step number t >= 1 */
void ora_adam_step(double *w, const double *grad, double *m, double *v, int64_t size, double lr, double beta1,
                   double beta2, double eps, int t) {
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t q = 0; q < size; q++) {
        m[q] = beta1 * m[q] + (1.0 - beta1) * grad[q];
        v[q] = beta2 * v[q] + (1.0 - beta2) * grad[q] * grad[q];
        w[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
    }
}

/* ------------------------------------------- batch autoregressive sampling */
/* Counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of
 * two 32x32 -> 64-bit multiplications, the key bumped by the Weyl constants
 * between rounds. */
void ora_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1, n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    for (int i = 0; i < 4; i++) out[i] = c[i];
}

/* Uniform draw in [0, 1) of sample slot i at sequence position s: counter
 * (i mod 2^32, i / 2^32, s, 0x42415300), key the seed's two halves; the top
 * 53 bits of the first two output words. */
double ora_bas_uniform(uint64_t seed, int s, uint64_t i) {
    const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)s, 0x42415300u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    ora_philox4x32_10(ctr, key, o);
    const uint64_t x = ((uint64_t)o[0] << 32) | o[1];
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* Token of one sample slot from its uniform u and the prefix's masked
 * conditional log-probabilities: walk the allowed tokens in order 0..3,
 * adding their probabilities, and take the first whose running sum exceeds
 * u (the last allowed token if rounding leaves u above the total). */
static int bas_token(const double *logp, double u) {
    double acc = 0.0;
    int last = -1;
    for (int t = 0; t < 4; t++) {
        if (!(logp[t] > -INFINITY)) continue;
        last = t;
        acc += exp(logp[t]);
        if (u < acc) return t;
    }
    return last;
}

/* Batch autoregressive sampling (Section 3.1): n_samples samples drawn at
 * once by following unique prefixes with their weights.  At position s every
 * unique prefix u (weight c_u) gets its conditional distribution
 * pi(t | prefix) from the network (the Eq. 12 mask included); the c_u sample
 * slots of u (slots numbered in prefix order) each draw one token, which
 * splits c_u multinomially among the four children; children with zero
 * weight are dropped.  After K positions the prefixes are the unique samples
 * and their weights the occurrence counts; logabs = 1/2 sum log pi along the
 * path.  Returns the number of unique samples, or -1 when more than
 * `capacity` prefixes would be needed. */
int64_t ora_bas(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w, uint64_t n_samples,
                uint64_t seed, int64_t capacity, uint64_t *keys_out, uint32_t *counts_out, double *logabs_out) {
    ora_net net = {K, d, L, H, F, P, n_up, n_dn};
    uint64_t *pk = (uint64_t *)calloc((size_t)capacity * 2, sizeof(uint64_t));
    uint64_t *nk = (uint64_t *)calloc((size_t)capacity * 2, sizeof(uint64_t));
    uint64_t *pc = (uint64_t *)calloc((size_t)capacity, sizeof(uint64_t));
    uint64_t *nc = (uint64_t *)calloc((size_t)capacity, sizeof(uint64_t));
    double *pl = (double *)calloc((size_t)capacity, sizeof(double));
    double *nl = (double *)calloc((size_t)capacity, sizeof(double));
    double *cond = (double *)calloc((size_t)capacity * 4, sizeof(double));
    uint64_t *child = (uint64_t *)calloc((size_t)capacity * 4, sizeof(uint64_t));
    int64_t n = 1, result = -1;
    pc[0] = n_samples;
    for (int s = 0; s < K; s++) {
        #pragma omp parallel for schedule(dynamic)
        for (int64_t u = 0; u < n; u++) {
            double *lp = (double *)malloc(sizeof(double) * K * 4);
            transformer_conditionals(&net, w, pk + 2 * u, lp);
            for (int t = 0; t < 4; t++) cond[u * 4 + t] = lp[s * 4 + t];
            free(lp);
        }
        memset(child, 0, sizeof(uint64_t) * 4 * (size_t)n);
        uint64_t slot = 0;
        for (int64_t u = 0; u < n; u++)
            for (uint64_t j = 0; j < pc[u]; j++, slot++) {
                const int t = bas_token(cond + 4 * u, ora_bas_uniform(seed, s, slot));
                child[u * 4 + t]++;
            }
        int64_t m = 0;
        const int i = K - 1 - s;  /* position s holds spatial orbital K-1-s */
        for (int64_t u = 0; u < n; u++)
            for (int t = 0; t < 4; t++) {
                if (!child[u * 4 + t]) continue;
                if (m >= capacity) goto done;
                nk[2 * m] = pk[2 * u];
                nk[2 * m + 1] = pk[2 * u + 1];
                if (t & 1) flip_bit(nk + 2 * m, 2 * i);
                if (t & 2) flip_bit(nk + 2 * m, 2 * i + 1);
                nc[m] = child[u * 4 + t];
                nl[m] = pl[u] + cond[u * 4 + t];
                m++;
            }
        { uint64_t *tk = pk; pk = nk; nk = tk; }
        { uint64_t *tc = pc; pc = nc; nc = tc; }
        { double *tl = pl; pl = nl; nl = tl; }
        n = m;
    }
    for (int64_t u = 0; u < n; u++) {
        keys_out[2 * u] = pk[2 * u];
        keys_out[2 * u + 1] = pk[2 * u + 1];
        counts_out[u] = (uint32_t)pc[u];
        logabs_out[u] = 0.5 * pl[u];
    }
    result = n;
done:
    free(pk); free(nk); free(pc); free(nc); free(pl); free(nl); free(cond); free(child);
    return result;
}

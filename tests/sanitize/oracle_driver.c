/* Sanitizer driver of the FP64 oracle (test infrastructure): calls every
 * public oracle routine on small seeded inputs so that an AddressSanitizer /
 * UndefinedBehaviorSanitizer build of oracle/nnqs_oracle.c checks its memory
 * accesses and arithmetic.  Prints "ok" and exits 0 when nothing fired. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t ora_n_connections(int K, int n_up, int n_dn);
double ora_hxx(int K, const double *h, const double *g, double ecore, const uint64_t *x, const uint64_t *xp,
               int *sign);
int64_t ora_connections(int K, int n_up, int n_dn, const double *h, const double *g, double ecore,
                        const uint64_t *x, uint64_t *xp, int8_t *sign, uint8_t *exc, double *hxx);
int ora_sort_table(const uint64_t *tkeys, const double *tl, const double *tp, int64_t nt, uint64_t *ko, double *lo,
                   double *po);
int ora_eloc_table(int K, int n_up, int n_dn, const double *h, const double *g, double ecore,
                   const uint64_t *tkeys, const double *tlogabs, const double *tphase, int64_t nt,
                   const uint64_t *keys, const double *logabs, const double *phase, int64_t n, double *eloc,
                   double *absum, int nthreads);
void ora_energy(const uint32_t *counts, const double *eloc, int64_t n, double *out);
int64_t ora_net_size(int K, int d, int L, int H, int F, int P);
void ora_net_conditionals(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w,
                          const uint64_t *x, double *logp);
void ora_net_logpsi(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w,
                    const uint64_t *keys, int64_t n, double *logabs, double *phase, int nthreads);
int ora_eloc_model(int K, int n_up, int n_dn, const double *h, const double *g, double ecore, int d, int L, int H,
                   int F, int P, const double *w, const uint64_t *keys, int64_t n, double *eloc, double *absum,
                   int nthreads);
int64_t ora_screen_size(int N, int H);
void ora_screen_forward(int N, int H, const double *w, const uint64_t *keys, const uint8_t *exc, int64_t n,
                        double *pred);
double ora_screen_loss_grad(int N, int H, const double *w, const uint64_t *keys, const uint8_t *exc,
                            const double *target, int64_t n, double *grad);
void ora_adam_step(double *w, const double *grad, double *m, double *v, int64_t size, double lr, double beta1,
                   double beta2, double eps, int t);
void ora_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out);
double ora_bas_uniform(uint64_t seed, int s, uint64_t i);
int64_t ora_bas(int K, int d, int L, int H, int F, int P, int n_up, int n_dn, const double *w, uint64_t n_samples,
                uint64_t seed, int64_t capacity, uint64_t *keys_out, uint32_t *counts_out, double *logabs_out);

static uint64_t lcg = 0x2306167050ULL;
static double urand(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(void) {
    const int K = 5, nu = 2, nd = 2;
    double *h = malloc(sizeof(double) * K * K), *g = malloc(sizeof(double) * K * K * K * K);
    for (int i = 0; i < K; i++)
        for (int j = 0; j <= i; j++) h[i * K + j] = h[j * K + i] = urand();
    for (int e = 0; e < K * K * K * K; e++) g[e] = 0.0;
    for (int p = 0; p < K; p++)
        for (int q = 0; q < K; q++)
            for (int r = 0; r < K; r++)
                for (int s = 0; s < K; s++) {
                    const double v = 0.1 * urand();
                    const int idx[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                                           {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
                    if (g[((p * K + q) * K + r) * K + s] != 0.0) continue;
                    for (int t = 0; t < 8; t++)
                        g[((idx[t][0] * K + idx[t][1]) * K + idx[t][2]) * K + idx[t][3]] = v;
                }
    /* the whole (2, 2) sector */
    uint64_t keys[200 * 2];
    int64_t n = 0;
    for (uint32_t b = 0; b < (1u << (2 * K)); b++) {
        int u = 0, dd = 0;
        for (int i = 0; i < K; i++) {
            u += (b >> (2 * i)) & 1;
            dd += (b >> (2 * i + 1)) & 1;
        }
        if (u == nu && dd == nd) {
            keys[2 * n] = b;
            keys[2 * n + 1] = 0;
            n++;
        }
    }
    CHECK(n == 100);
    const int64_t C = ora_n_connections(K, nu, nd);
    uint64_t *xp = malloc(sizeof(uint64_t) * 2 * C);
    int8_t *sg = malloc((size_t)C);
    uint8_t *exc = malloc((size_t)C * 4);
    double *hv = malloc(sizeof(double) * C);
    for (int64_t k = 0; k < n; k++) {
        const int64_t c = ora_connections(K, nu, nd, h, g, 0.3, keys + 2 * k, xp, sg, exc, hv);
        CHECK(c == C);
        int s;
        (void)ora_hxx(K, h, g, 0.3, keys + 2 * k, xp + 2 * (C - 1), &s);
    }
    double *la = malloc(sizeof(double) * n), *ph = malloc(sizeof(double) * n);
    for (int64_t k = 0; k < n; k++) {
        la[k] = -1.0 + 0.3 * urand();
        ph[k] = urand();
    }
    uint64_t *ko = malloc(sizeof(uint64_t) * 2 * n);
    double *lo = malloc(sizeof(double) * n), *po = malloc(sizeof(double) * n);
    CHECK(ora_sort_table(keys, la, ph, n, ko, lo, po) == 1);
    double *el = malloc(sizeof(double) * 2 * n), *ab = malloc(sizeof(double) * n), en[4];
    CHECK(ora_eloc_table(K, nu, nd, h, g, 0.3, keys, la, ph, n, keys, la, ph, n, el, ab, 1) == 0);
    uint32_t *cnt = malloc(sizeof(uint32_t) * n);
    for (int64_t k = 0; k < n; k++) cnt[k] = 1 + (uint32_t)(k % 7);
    ora_energy(cnt, el, n, en);
    CHECK(isfinite(en[0]));
    /* network */
    const int d = 8, L = 2, H = 2, F = 16, P = 12;
    const int64_t nw = ora_net_size(K, d, L, H, F, P);
    double *w = malloc(sizeof(double) * nw);
    for (int64_t e = 0; e < nw; e++) w[e] = 0.3 * urand();
    double logp[5 * 4];
    ora_net_conditionals(K, d, L, H, F, P, nu, nd, w, keys, logp);
    ora_net_logpsi(K, d, L, H, F, P, nu, nd, w, keys, n, la, ph, 1);
    CHECK(ora_eloc_model(K, nu, nd, h, g, 0.3, d, L, H, F, P, w, keys, 8, el, ab, 1) == 0);
    uint64_t bk[2 * 128];
    uint32_t bc[128];
    double bl[128];
    const int64_t m = ora_bas(K, d, L, H, F, P, nu, nd, w, 10000, 7, 128, bk, bc, bl);
    CHECK(m > 0 && m <= 100);
    CHECK(ora_bas(K, d, L, H, F, P, nu, nd, w, 10000, 7, 2, bk, bc, bl) == -1);
    /* screen */
    const int N = 2 * K, HS = 8;
    const int64_t ns = ora_screen_size(N, HS);
    double *sw = malloc(sizeof(double) * ns), *gr = malloc(sizeof(double) * ns);
    double *m1 = calloc((size_t)ns, sizeof(double)), *m2 = calloc((size_t)ns, sizeof(double));
    for (int64_t e = 0; e < ns; e++) sw[e] = 0.2 * urand();
    uint64_t sk[2 * 16];
    uint8_t se[4 * 16];
    double pred[16], tgt[16];
    (void)ora_connections(K, nu, nd, h, g, 0.3, keys, xp, sg, exc, hv);
    for (int k = 0; k < 16; k++) {
        sk[2 * k] = xp[2 * k];
        sk[2 * k + 1] = xp[2 * k + 1];
        for (int t = 0; t < 4; t++) se[4 * k + t] = exc[4 * k + t];
        tgt[k] = urand();
    }
    ora_screen_forward(N, HS, sw, sk, se, 16, pred);
    const double loss = ora_screen_loss_grad(N, HS, sw, sk, se, tgt, 16, gr);
    CHECK(isfinite(loss));
    ora_adam_step(sw, gr, m1, m2, ns, 1e-3, 0.9, 0.999, 1e-8, 1);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    ora_philox4x32_10(ctr, key, out);
    const double uu = ora_bas_uniform(7, 3, 11);
    CHECK(uu >= 0.0 && uu < 1.0);
    free(h); free(g); free(xp); free(sg); free(exc); free(hv); free(la); free(ph); free(ko); free(lo); free(po);
    free(el); free(ab); free(cnt); free(w); free(sw); free(gr); free(m1); free(m2);
    printf("ok\n");
    return 0;
}

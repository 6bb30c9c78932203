/*
 * pt_oracle.c -- plain FP64 CPU oracle for the phylogenetic tree likelihood,
 * its branch-length derivatives and coordinate-wise Newton optimisation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or table with the GPU library and on purpose uses other numerical
 * methods: e^{Qt} by scaling-and-squaring of the Taylor series (no
 * eigendecomposition), the incomplete gamma function by series / continued
 * fraction with a bisection inverse, and every partial likelihood recomputed
 * from scratch by recursion.  Nothing is blocked, fused or cached beyond what
 * the definitions below state.
 *
 * What is computed (the paper, Methods, "Methods Overview" and "Phylogenetic
 * Topographer": visiting a topology means optimising its branch lengths to
 * maximise the tree log-likelihood under JC69+Gamma or GTR; the likelihood
 * itself is delegated to a library and not written out, so the textbook
 * definitions are used):
 *
 *   L_p = sum_k (1/K) sum over ancestral states of prod_edges P(r_k t_e)
 *         times pi at the root, evaluated by Felsenstein pruning;
 *   lnL = sum_p w_p ln L_p.
 *
 * Conventions: states A,C,G,T; exchangeabilities AC,AG,AT,CG,CT,GT;
 * Q_ij = r_ij pi_j (i != j), rows sum to 0, scaled so that
 * -sum_i pi_i Q_ii = 1; K discrete Gamma categories of weight 1/K whose
 * rates are the category means of Gamma(alpha, rate alpha) (Yang 1994);
 * K = 1 means rate 1.  Per-pattern scaling multiplies a partial by 2^256
 * when its largest entry is below 2^-256 and counts the event; it is exact.
 *
 * Trees: n taxa, 2n-3 edges as node pairs, leaves 0..n-1, internal nodes
 * n..2n-3, every internal node of degree 3 (n = 2: the single edge (0,1)).
 *
 * Error codes: 0 success, -1 invalid argument, -2 out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_SCALE_EXP 256
#define OR_MAXK 16

/* ------------------------------------------------------------ 4x4 algebra */

static void mat_mul(const double *a, const double *b, double *c)
{
    double t[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int m = 0; m < 4; ++m) s += a[i * 4 + m] * b[m * 4 + j];
            t[i * 4 + j] = s;
        }
    memcpy(c, t, sizeof t);
}

/* GTR rate matrix, normalised to one expected substitution per unit time. */
void or_rate_matrix(const double *rates, const double *freqs, double *Q)
{
    static const int pi_[6] = {0, 0, 0, 1, 1, 2};
    static const int pj_[6] = {1, 2, 3, 2, 3, 3};
    memset(Q, 0, 16 * sizeof(double));
    for (int x = 0; x < 6; ++x) {
        Q[pi_[x] * 4 + pj_[x]] = rates[x] * freqs[pj_[x]];
        Q[pj_[x] * 4 + pi_[x]] = rates[x] * freqs[pi_[x]];
    }
    double mu = 0.0;
    for (int i = 0; i < 4; ++i) {
        double row = 0.0;
        for (int j = 0; j < 4; ++j) if (j != i) row += Q[i * 4 + j];
        Q[i * 4 + i] = -row;
        mu += freqs[i] * row;
    }
    for (int x = 0; x < 16; ++x) Q[x] /= mu;
}

/* e^{A} by scaling and squaring of the Taylor series (Higham 2005 style:
 * scale so the 1-norm is at most 1/2, sum terms until they no longer change
 * the result, square back). */
void or_expm(const double *A, double *E)
{
    double norm = 0.0;
    for (int j = 0; j < 4; ++j) {
        double c = 0.0;
        for (int i = 0; i < 4; ++i) c += fabs(A[i * 4 + j]);
        if (c > norm) norm = c;
    }
    int s = 0;
    while (norm > 0.5) { norm *= 0.5; ++s; }
    double B[16], term[16];
    double f = ldexp(1.0, -s);
    for (int x = 0; x < 16; ++x) B[x] = A[x] * f;
    for (int x = 0; x < 16; ++x) { E[x] = (x % 5 == 0) ? 1.0 : 0.0; term[x] = E[x]; }
    for (int k = 1; k <= 40; ++k) {
        mat_mul(term, B, term);
        double mx = 0.0;
        for (int x = 0; x < 16; ++x) { term[x] /= (double)k; E[x] += term[x]; if (fabs(term[x]) > mx) mx = fabs(term[x]); }
        if (mx < 1e-18) break;
    }
    for (int q = 0; q < s; ++q) mat_mul(E, E, E);
}

/* P(t) = e^{Qt}, dP/dt = Q P, d2P/dt2 = Q Q P (Q commutes with e^{Qt}). */
void or_pmatrix(const double *Q, double t, double *P, double *dP, double *d2P)
{
    double A[16];
    for (int x = 0; x < 16; ++x) A[x] = Q[x] * t;
    or_expm(A, P);
    if (dP) mat_mul(Q, P, dP);
    if (d2P) { double QP[16]; mat_mul(Q, P, QP); mat_mul(Q, QP, d2P); }
}

/* ---------------------------------------------------- discrete Gamma rates */

/* Regularised lower incomplete gamma P(a, x): series for x < a + 1,
 * Lentz continued fraction for the complement otherwise (Numerical Recipes,
 * section 6.2). */
double or_gammp(double a, double x)
{
    if (x <= 0.0) return 0.0;
    double lg = lgamma(a);
    if (x < a + 1.0) {
        double ap = a, sum = 1.0 / a, del = sum;
        for (int n = 0; n < 100000; ++n) {
            ap += 1.0; del *= x / ap; sum += del;
            if (fabs(del) < fabs(sum) * 1e-17) break;
        }
        return sum * exp(-x + a * log(x) - lg);
    }
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        double an = -i * (i - a);
        b += 2.0;
        d = an * d + b; if (fabs(d) < tiny) d = tiny;
        c = b + an / c; if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return 1.0 - exp(-x + a * log(x) - lg) * h;
}

/* y with P(a, y) = q, by bracketing and bisection to full precision. */
static double gammp_inv(double a, double q)
{
    double lo = 0.0, hi = 1.0;
    while (or_gammp(a, hi) < q) hi *= 2.0;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (or_gammp(a, mid) < q) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Mean rates of K equal-probability categories of Gamma(alpha, alpha). */
int or_gamma_rates(double alpha, int K, double *r)
{
    if (K < 1 || K > OR_MAXK) return -1;
    if (K == 1) { r[0] = 1.0; return 0; }
    if (!(alpha > 0.0)) return -1;
    double prev = 0.0;            /* P(alpha+1, alpha * xi_{i-1}) */
    for (int i = 0; i < K; ++i) {
        double cur;
        if (i == K - 1) cur = 1.0;
        else {
            double y = gammp_inv(alpha, (double)(i + 1) / K);  /* alpha * xi_i */
            cur = or_gammp(alpha + 1.0, y);
        }
        r[i] = K * (cur - prev);
        prev = cur;
    }
    return 0;
}

/* ------------------------------------------------------------------ trees */

typedef struct {
    int n, n_nodes, n_edges;
    int *nbr;   /* [n_nodes][3] */
    int *nedge; /* [n_nodes][3] */
    int *deg;   /* [n_nodes] */
} tree_t;

static void tree_free(tree_t *t) { free(t->nbr); free(t->nedge); free(t->deg); }

static int tree_build(int n, const int32_t *edges, tree_t *t)
{
    memset(t, 0, sizeof *t);
    if (n < 2) return -1;
    t->n = n;
    t->n_nodes = (n == 2) ? 2 : 2 * n - 2;
    t->n_edges = (n == 2) ? 1 : 2 * n - 3;
    t->nbr = malloc(sizeof(int) * 3 * t->n_nodes);
    t->nedge = malloc(sizeof(int) * 3 * t->n_nodes);
    t->deg = calloc(t->n_nodes, sizeof(int));
    if (!t->nbr || !t->nedge || !t->deg) { tree_free(t); return -2; }
    for (int e = 0; e < t->n_edges; ++e) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= t->n_nodes || b >= t->n_nodes || a == b) { tree_free(t); return -1; }
        if (t->deg[a] >= 3 || t->deg[b] >= 3) { tree_free(t); return -1; }
        t->nbr[a * 3 + t->deg[a]] = b; t->nedge[a * 3 + t->deg[a]] = e; t->deg[a]++;
        t->nbr[b * 3 + t->deg[b]] = a; t->nedge[b * 3 + t->deg[b]] = e; t->deg[b]++;
    }
    for (int v = 0; v < t->n_nodes; ++v) {
        int want = (v < n) ? 1 : 3;
        if (t->deg[v] != want) { tree_free(t); return -1; }
    }
    /* connectivity: n_nodes - 1 edges and connected means a tree */
    int *seen = calloc(t->n_nodes, sizeof(int)), *stack = malloc(sizeof(int) * t->n_nodes);
    if (!seen || !stack) { free(seen); free(stack); tree_free(t); return -2; }
    int top = 0, count = 0;
    stack[top++] = 0; seen[0] = 1;
    while (top) {
        int v = stack[--top]; ++count;
        for (int j = 0; j < t->deg[v]; ++j) {
            int c = t->nbr[v * 3 + j];
            if (!seen[c]) { seen[c] = 1; stack[top++] = c; }
        }
    }
    free(seen); free(stack);
    if (count != t->n_nodes) { tree_free(t); return -1; }
    return 0;
}

/* ------------------------------------------------------------ likelihoods */

typedef struct {
    int n, P, K;
    const uint8_t *tips;    /* [n][P] */
    const double *w;        /* [P] */
    double freqs[4];
    double Q[16];
    double r[OR_MAXK];
    int scaling;            /* 1: per-pattern scaling on */
} data_t;

static int data_init(data_t *d, int n, int P, const uint8_t *tips, const double *w,
                     const double *rates, const double *freqs, double alpha, int K, int scaling)
{
    if (P < 0 || K < 1 || K > OR_MAXK) return -1;
    d->n = n; d->P = P; d->K = K; d->tips = tips; d->w = w; d->scaling = scaling;
    double s = 0.0;
    for (int i = 0; i < 4; ++i) { if (!(freqs[i] > 0.0)) return -1; d->freqs[i] = freqs[i]; s += freqs[i]; }
    if (fabs(s - 1.0) > 1e-9) return -1;
    for (int x = 0; x < 6; ++x) if (!(rates[x] > 0.0)) return -1;
    or_rate_matrix(rates, freqs, d->Q);
    return or_gamma_rates(alpha, K, d->r);
}

/* Partial likelihood of the subtree hanging from `node` away from `from`:
 * out[p][k][i] = Pr(data below | state i at node, category k), times
 * 2^(256 cnt[p]) when scaling is on. */
static int partial(const tree_t *t, const data_t *d, const double *brlen,
                   int node, int from, double *out, int *cnt)
{
    const int P = d->P, K = d->K;
    if (node < t->n) {
        for (int p = 0; p < P; ++p) {
            uint8_t c = d->tips[(size_t)node * P + p];
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < 4; ++i)
                    out[((size_t)p * K + k) * 4 + i] = ((c >> i) & 1) ? 1.0 : 0.0;
            cnt[p] = 0;
        }
        return 0;
    }
    size_t len = (size_t)P * K * 4;
    double *child = malloc(sizeof(double) * (len ? len : 1));
    int *ccnt = malloc(sizeof(int) * (P ? P : 1));
    if (!child || !ccnt) { free(child); free(ccnt); return -2; }
    for (size_t x = 0; x < len; ++x) out[x] = 1.0;
    for (int p = 0; p < P; ++p) cnt[p] = 0;
    for (int j = 0; j < 3; ++j) {
        int c = t->nbr[node * 3 + j];
        if (c == from) continue;
        int e = t->nedge[node * 3 + j];
        int rc = partial(t, d, brlen, c, node, child, ccnt);
        if (rc) { free(child); free(ccnt); return rc; }
        for (int k = 0; k < K; ++k) {
            double Pm[16];
            or_pmatrix(d->Q, brlen[e] * d->r[k], Pm, NULL, NULL);
            for (int p = 0; p < P; ++p) {
                double *o = out + ((size_t)p * K + k) * 4;
                const double *x = child + ((size_t)p * K + k) * 4;
                for (int i = 0; i < 4; ++i) {
                    double s = 0.0;
                    for (int m = 0; m < 4; ++m) s += Pm[i * 4 + m] * x[m];
                    o[i] *= s;
                }
            }
        }
        for (int p = 0; p < P; ++p) cnt[p] += ccnt[p];
    }
    if (d->scaling) {
        const double thr = ldexp(1.0, -OR_SCALE_EXP);
        for (int p = 0; p < P; ++p) {
            double mx = 0.0;
            for (int x = 0; x < K * 4; ++x) { double v = out[(size_t)p * K * 4 + x]; if (v > mx) mx = v; }
            if (mx > 0.0 && mx < thr) {
                for (int x = 0; x < K * 4; ++x) out[(size_t)p * K * 4 + x] = ldexp(out[(size_t)p * K * 4 + x], OR_SCALE_EXP);
                cnt[p] += 1;
            }
        }
    }
    free(child); free(ccnt);
    return 0;
}

/* Neumaier (compensated) summation. */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *a, double x)
{
    double t = a->s + x;
    if (!isfinite(t)) { a->s = t; return; }   /* -inf stays -inf */
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
    a->s = t;
}
static double ks_get(const ksum *a) { return isfinite(a->s) ? a->s + a->c : a->s; }

/* lnL, d lnL/dt and d2 lnL/dt2 for edge length t between partials A (one
 * side) and B (other side):  L_p(t) = sum_k (1/K) sum_ij pi_i A_i P_ij(r_k t) B_j. */
static void edge_eval(const data_t *d, const double *A, const int *cA, const double *B,
                      const int *cB, double t, double *lnl, double *d1, double *d2)
{
    const int P = d->P, K = d->K;
    double Pm[OR_MAXK][16], D1[OR_MAXK][16], D2[OR_MAXK][16];
    for (int k = 0; k < K; ++k) {
        or_pmatrix(d->Q, t * d->r[k], Pm[k], D1[k], D2[k]);
        for (int x = 0; x < 16; ++x) { D1[k][x] *= d->r[k]; D2[k][x] *= d->r[k] * d->r[k]; }
    }
    ksum sl = {0, 0}, s1 = {0, 0}, s2 = {0, 0};
    const double ln2 = log(2.0);
    for (int p = 0; p < P; ++p) {
        double L = 0.0, L1 = 0.0, L2 = 0.0;
        for (int k = 0; k < K; ++k) {
            const double *a = A + ((size_t)p * K + k) * 4, *b = B + ((size_t)p * K + k) * 4;
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    double f = d->freqs[i] * a[i] * b[j] / K;
                    L += f * Pm[k][i * 4 + j];
                    L1 += f * D1[k][i * 4 + j];
                    L2 += f * D2[k][i * 4 + j];
                }
        }
        double w = d->w[p];
        int c = (cA ? cA[p] : 0) + (cB ? cB[p] : 0);
        ks_add(&sl, w * (log(L) - (double)c * OR_SCALE_EXP * ln2));
        ks_add(&s1, w * L1 / L);
        ks_add(&s2, w * (L2 / L - (L1 / L) * (L1 / L)));
    }
    if (lnl) *lnl = ks_get(&sl);
    if (d1) *d1 = ks_get(&s1);
    if (d2) *d2 = ks_get(&s2);
}

typedef struct { double *A, *B; int *cA, *cB; } sides_t;

static int sides_alloc(sides_t *s, int P, int K)
{
    size_t len = (size_t)P * K * 4;
    s->A = malloc(sizeof(double) * (len ? len : 1));
    s->B = malloc(sizeof(double) * (len ? len : 1));
    s->cA = malloc(sizeof(int) * (P ? P : 1));
    s->cB = malloc(sizeof(int) * (P ? P : 1));
    return (s->A && s->B && s->cA && s->cB) ? 0 : -2;
}
static void sides_free(sides_t *s) { free(s->A); free(s->B); free(s->cA); free(s->cB); }

static int edge_sides(const tree_t *t, const data_t *d, const double *brlen, int32_t const *edges,
                      int e, sides_t *s)
{
    int u = edges[2 * e], v = edges[2 * e + 1];
    int rc = partial(t, d, brlen, u, v, s->A, s->cA);
    if (!rc) rc = partial(t, d, brlen, v, u, s->B, s->cB);
    return rc;
}

static int check_lengths(int E, const double *brlen)
{
    for (int e = 0; e < E; ++e) if (!(brlen[e] >= 0.0) || !isfinite(brlen[e])) return -1;
    return 0;
}

/* Log-likelihood evaluated across edge `at_edge` (any edge gives the same
 * value: the pulley principle). */
int or_loglik_at(int n, const int32_t *edges, const double *brlen,
                 int P, const uint8_t *tips, const double *w,
                 const double *rates, const double *freqs, double alpha, int K,
                 int scaling, int at_edge, double *lnl)
{
    tree_t t; data_t d;
    int rc = tree_build(n, edges, &t);
    if (rc) return rc;
    if ((rc = data_init(&d, n, P, tips, w, rates, freqs, alpha, K, scaling)) ||
        (rc = check_lengths(t.n_edges, brlen)) || at_edge < 0 || at_edge >= t.n_edges) {
        tree_free(&t); return rc ? rc : -1;
    }
    sides_t s;
    if (sides_alloc(&s, P, K)) { sides_free(&s); tree_free(&t); return -2; }
    rc = edge_sides(&t, &d, brlen, edges, at_edge, &s);
    if (!rc) edge_eval(&d, s.A, s.cA, s.B, s.cB, brlen[at_edge], lnl, NULL, NULL);
    sides_free(&s); tree_free(&t);
    return rc;
}

/* Log-likelihood with the root placed on internal node `root` (n >= 3):
 * L_p = sum_k (1/K) sum_i pi_i prod_{3 neighbours} (P X)_i. */
int or_loglik_node(int n, const int32_t *edges, const double *brlen,
                   int P, const uint8_t *tips, const double *w,
                   const double *rates, const double *freqs, double alpha, int K,
                   int scaling, int root, double *lnl)
{
    tree_t t; data_t d;
    int rc = tree_build(n, edges, &t);
    if (rc) return rc;
    if ((rc = data_init(&d, n, P, tips, w, rates, freqs, alpha, K, scaling)) ||
        (rc = check_lengths(t.n_edges, brlen)) || root < n || root >= t.n_nodes) {
        tree_free(&t); return rc ? rc : -1;
    }
    size_t len = (size_t)P * K * 4;
    double *X = malloc(sizeof(double) * (len ? len : 1));
    int *cnt = malloc(sizeof(int) * (P ? P : 1));
    if (!X || !cnt) { free(X); free(cnt); tree_free(&t); return -2; }
    rc = partial(&t, &d, brlen, root, -1, X, cnt);
    if (!rc) {
        ksum sl = {0, 0};
        for (int p = 0; p < P; ++p) {
            double L = 0.0;
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < 4; ++i) L += d.freqs[i] * X[((size_t)p * K + k) * 4 + i] / K;
            ks_add(&sl, w[p] * (log(L) - (double)cnt[p] * OR_SCALE_EXP * log(2.0)));
        }
        *lnl = ks_get(&sl);
    }
    free(X); free(cnt); tree_free(&t);
    return rc;
}

/* Edge derivatives of lnL with respect to the length of edge `e`. */
int or_edge_derivs(int n, const int32_t *edges, const double *brlen,
                   int P, const uint8_t *tips, const double *w,
                   const double *rates, const double *freqs, double alpha, int K,
                   int e, double *lnl, double *d1, double *d2)
{
    tree_t t; data_t d;
    int rc = tree_build(n, edges, &t);
    if (rc) return rc;
    if ((rc = data_init(&d, n, P, tips, w, rates, freqs, alpha, K, 1)) ||
        (rc = check_lengths(t.n_edges, brlen)) || e < 0 || e >= t.n_edges) {
        tree_free(&t); return rc ? rc : -1;
    }
    sides_t s;
    if (sides_alloc(&s, P, K)) { sides_free(&s); tree_free(&t); return -2; }
    rc = edge_sides(&t, &d, brlen, edges, e, &s);
    if (!rc) edge_eval(&d, s.A, s.cA, s.B, s.cB, brlen[e], lnl, d1, d2);
    sides_free(&s); tree_free(&t);
    return rc;
}

/* Gradient (and diagonal of the Hessian) for every edge, each edge handled
 * by re-rooting on it: O(n^2) partial computations, plain and independent. */
int or_gradient(int n, const int32_t *edges, const double *brlen,
                int P, const uint8_t *tips, const double *w,
                const double *rates, const double *freqs, double alpha, int K,
                double *lnl, double *grad, double *hdiag)
{
    tree_t t; data_t d;
    int rc = tree_build(n, edges, &t);
    if (rc) return rc;
    if ((rc = data_init(&d, n, P, tips, w, rates, freqs, alpha, K, 1)) ||
        (rc = check_lengths(t.n_edges, brlen))) {
        tree_free(&t); return rc;
    }
    sides_t s;
    if (sides_alloc(&s, P, K)) { sides_free(&s); tree_free(&t); return -2; }
    for (int e = 0; e < t.n_edges && !rc; ++e) {
        double l, g, h;
        rc = edge_sides(&t, &d, brlen, edges, e, &s);
        if (rc) break;
        edge_eval(&d, s.A, s.cA, s.B, s.cB, brlen[e], &l, &g, &h);
        if (e == 0 && lnl) *lnl = l;
        grad[e] = g;
        if (hdiag) hdiag[e] = h;
    }
    sides_free(&s); tree_free(&t);
    return rc;
}

/* ------------------------------------------------------------ optimisation */

/* One edge: safeguarded, projected Newton on t in [t_min, t_max] for the
 * objective lnL(t) - prior_rate * t (prior_rate = 0: maximum likelihood; > 0:
 * the log density of an exponential prior on the length added, so the first
 * derivative loses prior_rate and the second is unchanged).
 *  - the bracket (lo, hi) starts as [t_min, t_max] and shrinks to t from
 *    the side the first derivative points away from;
 *  - a Newton step is taken when d2 < 0 and the step stays in the bracket
 *    (the original bounds themselves count as inside), else the bracket is
 *    bisected geometrically;
 *  - a bound with the derivative pointing outwards is an optimum;
 *  - stop when the step is at most tol * max(t, 1e-6). */
static double newton_edge(const data_t *d, const sides_t *s, double t0, double t_min, double t_max,
                          double tol, int max_iter, double prior_rate, int *iters)
{
    double lo = t_min, hi = t_max;
    double t = t0 < t_min ? t_min : (t0 > t_max ? t_max : t0);
    int it = 0;
    for (; it < max_iter; ++it) {
        double d1, d2;
        edge_eval(d, s->A, s->cA, s->B, s->cB, t, NULL, &d1, &d2);
        d1 -= prior_rate;
        if (d1 > 0.0) lo = t;
        else if (d1 < 0.0) hi = t;
        else break;
        if ((t <= t_min && d1 <= 0.0) || (t >= t_max && d1 >= 0.0)) break;
        double tn = (d2 < 0.0) ? t - d1 / d2 : NAN;
        if (tn < t_min) tn = t_min;
        if (tn > t_max) tn = t_max;
        int inside = (tn > lo || (lo == t_min && tn == t_min)) &&
                     (tn < hi || (hi == t_max && tn == t_max));
        if (!(inside) || isnan(tn)) tn = sqrt(lo * hi);
        double step = fabs(tn - t);
        t = tn;
        if (step <= tol * fmax(t, 1e-6)) { ++it; break; }
    }
    if (iters) *iters = it;
    return t;
}

/* Log density of independent exponential priors of rate `rate` on every
 * length, sum over e of log(rate) - rate * t_e (0 when rate is 0). */
static double log_prior(int n_edges, const double *brlen, double rate)
{
    if (!(rate > 0.0)) return 0.0;
    double s = 0.0;
    for (int e = 0; e < n_edges; ++e) s += log(rate) - rate * brlen[e];
    return s;
}

/* Coordinate-wise Newton over the masked edges (ascending edge index) until
 * a pass raises the objective by less than tol_lnl and moves no edge by more
 * than tol_t relative, or max_passes passes.  The objective is lnL, plus with
 * prior_rate > 0 the log density of an exponential branch-length prior of
 * that rate on every edge (MAP lengths; Methods, "Phylogenetic Topographer",
 * the optional branch-length prior).  Returns the final objective, the
 * number of passes and whether the stopping rule was met (1) or not (0). */
int or_optimize(int n, const int32_t *edges, double *brlen, const uint8_t *mask,
                int P, const uint8_t *tips, const double *w,
                const double *rates, const double *freqs, double alpha, int K,
                double t_min, double t_max, double tol_lnl, double tol_t,
                double tol_newton, int max_passes, int max_newton, double prior_rate,
                double *lnl_out, int *passes_out, int *converged_out)
{
    tree_t t; data_t d;
    int rc = tree_build(n, edges, &t);
    if (rc) return rc;
    if ((rc = data_init(&d, n, P, tips, w, rates, freqs, alpha, K, 1)) ||
        (rc = check_lengths(t.n_edges, brlen)) || !(t_min > 0.0) || !(t_max > t_min) ||
        !(prior_rate >= 0.0) || !isfinite(prior_rate)) {
        tree_free(&t); return rc ? rc : -1;
    }
    sides_t s;
    if (sides_alloc(&s, P, K)) { sides_free(&s); tree_free(&t); return -2; }
    for (int e = 0; e < t.n_edges; ++e) {
        if (brlen[e] < t_min) brlen[e] = t_min;
        if (brlen[e] > t_max) brlen[e] = t_max;
    }
    double prev = -INFINITY, cur = -INFINITY;
    int pass = 0, conv = 0;
    for (pass = 1; pass <= max_passes && !rc; ++pass) {
        double max_rel = 0.0;
        for (int e = 0; e < t.n_edges; ++e) {
            if (mask && !mask[e]) continue;
            rc = edge_sides(&t, &d, brlen, edges, e, &s);
            if (rc) break;
            double old = brlen[e];
            brlen[e] = newton_edge(&d, &s, old, t_min, t_max, tol_newton, max_newton, prior_rate, NULL);
            double rel = fabs(brlen[e] - old) / fmax(old, 1e-6);
            if (rel > max_rel) max_rel = rel;
        }
        if (rc) break;
        /* lnL of the whole tree after the pass */
        rc = edge_sides(&t, &d, brlen, edges, 0, &s);
        if (rc) break;
        edge_eval(&d, s.A, s.cA, s.B, s.cB, brlen[0], &cur, NULL, NULL);
        cur += log_prior(t.n_edges, brlen, prior_rate);
        if (cur - prev < tol_lnl && max_rel < tol_t) { conv = 1; break; }
        prev = cur;
    }
    if (pass > max_passes) pass = max_passes;
    if (!rc) {
        if (lnl_out) *lnl_out = cur;
        if (passes_out) *passes_out = pass;
        if (converged_out) *converged_out = conv;
    }
    sides_free(&s); tree_free(&t);
    return rc;
}

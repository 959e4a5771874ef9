/*
 * tcol_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 reference of one iteration of the
 * population-based gradient-descent colouring method (TensCol) of Goudet,
 * Duval and Hao, "Population-based Gradient Descent Weight Learning for Graph
 * Coloring Problems".  It exists so the GPU library can be checked against
 * something written straight from the paper; only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or table with the GPU library.
 *
 * Every sum over "j with c_d(j) = l" below is the plain definition of the
 * product X * S_d for a one-hot S_d, so no dense n x n x k product is formed.
 *
 * Conventions (readings of the paper where it is silent or inconsistent):
 *  - arrays are row-major; W is [D][n][k], A is [n][n] uint8 0/1;
 *  - argmax ties go to the lowest colour index;
 *  - c1 = floor(n/k), c2 = ceil(n/k)  (= floor(n/k)+1 unless k divides n);
 *  - kappa and varpi sum over ordered pairs (i, j), both triangles;
 *  - the bonus matrix J - A includes the diagonal when bonus_diag = 1;
 *  - 0^p = 0 for p > 0;
 *  - the loss and its gradient use the iteration counter t that starts at 0;
 *  - smoothing W /= rho follows the update of iteration t when
 *    (t+1) mod nb_iter == 0;
 *  - an iteration whose population holds a legal member stops before its
 *    update, and the lowest such member is returned.
 *
 * Problems (Sections 3 and 6): 0 k-colouring (GCP step), 1 equitable colouring
 * (ECP), 2 k-partitioning, 3 balanced k-partitioning, 4 minimum sum colouring.
 * For partitioning every association matrix M is replaced by J - M, so the
 * fitness is the number of cut edges and the group concentration enters the
 * penalty and bonus as D - mt; the balanced variant adds the equity fitness.
 * For minimum sum colouring the equity fitness is replaced by the colour cost
 * sum_i z_{c(i)} with z_l = l + 1.  With momentum gamma > 0 the update is the
 * heavy-ball step v <- gamma v + gW, W <- W - eta v (v starts at zero).  Problem 5,
 * multicolouring, selects c_i colours per vertex (orc_select and the *_multi functions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t problem;   /* 0 k-COL, 1 ECP, 2 k-partitioning, 3 balanced k-partitioning, 4 min-sum colouring */
    int32_t n, k, D;
    double eta, rho;
    int32_t nb_iter;
    double alpha, lambda, beta, mu, nu;
    int32_t bonus_diag;
    int32_t stop_on_legal;
    double momentum;   /* heavy-ball coefficient gamma in [0, 1); 0 = plain gradient step */
} orc_params;

static int is_partition(const orc_params *p) { return p->problem == 2 || p->problem == 3; }
static int has_equity(const orc_params *p) { return p->problem == 1 || p->problem == 3; }

/* Step 1 (vertex to colour assignment): c_d(i) = argmax_l W[d,i,l].
 * Returns 0, or -5 if some row holds a non-finite weight. */
int orc_colors(int D, int n, int k, const double *W, int16_t *c)
{
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < n; ++i) {
            const double *w = W + ((size_t)d * n + i) * k;
            int best = 0;
            for (int l = 0; l < k; ++l) {
                if (!isfinite(w[l]))
                    return -5;
                if (w[l] > w[best])
                    best = l;
            }
            c[(size_t)d * n + i] = (int16_t)best;
        }
    return 0;
}

/* #V_{d,l}: number of vertices of member d that receive colour l. */
void orc_class_sizes(int D, int n, int k, const int16_t *c, int32_t *V)
{
    memset(V, 0, sizeof(int32_t) * (size_t)D * k);
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < n; ++i)
            V[(size_t)d * k + c[(size_t)d * n + i]] += 1;
}

/* Step 2, individual fitness: f_color(S_d) = 1/2 sum_ij a_ij m_dij, i.e. the
 * number of edges {i, j} whose two ends share a colour in member d. */
void orc_fcolor(int D, int n, const uint8_t *A, const int16_t *c, int64_t *fcol)
{
    for (int d = 0; d < D; ++d) {
        const int16_t *cd = c + (size_t)d * n;
        int64_t f = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (A[(size_t)i * n + j] && cd[i] == cd[j])
                    f += 1;
        fcol[d] = f;
    }
}

/* Class-conflict matrix of each member, S_d^T A S_d (k x k): entry (l, l') counts the ordered
 * pairs (i, j) with a_ij = 1, c_d(i) = l and c_d(j) = l', i.e. the edges between colour classes
 * l and l' (twice the edges inside class l on the diagonal), so its trace is 2 f_color(S_d).
 * Counted by brute force over the ordered edges.  C is [D][k][k]. */
void orc_class_conflicts(int D, int n, int k, const uint8_t *A, const int16_t *c, int32_t *C)
{
    memset(C, 0, sizeof(int32_t) * (size_t)D * k * k);
    for (int d = 0; d < D; ++d) {
        const int16_t *cd = c + (size_t)d * n;
        int32_t *Cd = C + (size_t)d * k * k;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (A[(size_t)i * n + j])
                    Cd[(size_t)cd[i] * k + cd[j]] += 1;
    }
}

/* Bounds of the equity constraint: c1 = floor(n/k); c2 = floor(n/k)+1, equal
 * to c1 when k divides n. */
void orc_equity_bounds(int n, int k, int32_t *c1, int32_t *c2)
{
    *c1 = n / k;
    *c2 = (n % k == 0) ? n / k : n / k + 1;
}

/* Equity fitness: f_eq(S_d) = sum_l min(|#V_dl - c1|, |#V_dl - c2|). */
void orc_feq(int D, int n, int k, const int32_t *V, int64_t *feq)
{
    int32_t c1, c2;
    orc_equity_bounds(n, k, &c1, &c2);
    for (int d = 0; d < D; ++d) {
        int64_t f = 0;
        for (int l = 0; l < k; ++l) {
            int64_t v = V[(size_t)d * k + l];
            int64_t a = llabs(v - c1), b = llabs(v - c2);
            f += a < b ? a : b;
        }
        feq[d] = f;
    }
}

/* Cut of a partition: f_cut(S_d) = 1/2 sum_ij a_ij (1 - m_dij), the number of
 * edges {i, j} whose ends lie in different groups of member d. */
void orc_fcut(int D, int n, const uint8_t *A, const int16_t *c, int64_t *fcut)
{
    for (int d = 0; d < D; ++d) {
        const int16_t *cd = c + (size_t)d * n;
        int64_t f = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (A[(size_t)i * n + j] && cd[i] != cd[j])
                    f += 1;
        fcut[d] = f;
    }
}

/* Colour cost of minimum sum colouring: f_mscp(S_d) = sum_i z_{c_d(i)} with
 * z_l = l + 1, i.e. sum_l (l + 1) #V_dl. */
void orc_fmscp(int D, int k, const int32_t *V, int64_t *fsum)
{
    for (int d = 0; d < D; ++d) {
        int64_t f = 0;
        for (int l = 0; l < k; ++l)
            f += (int64_t)(l + 1) * V[(size_t)d * k + l];
        fsum[d] = f;
    }
}

/* Fitness of each member for the problem: fmain is f_color (colouring) or
 * f_cut (partitioning), fsec the added term (f_eq, f_mscp or 0), f their sum. */
void orc_fitness(const orc_params *p, const uint8_t *A, const int16_t *c, const int32_t *V,
                 int64_t *fmain, int64_t *fsec, int64_t *f)
{
    const int n = p->n, k = p->k, D = p->D;
    if (is_partition(p))
        orc_fcut(D, n, A, c, fmain);
    else
        orc_fcolor(D, n, A, c, fmain);
    if (has_equity(p))
        orc_feq(D, n, k, V, fsec);
    else if (p->problem == 4)
        orc_fmscp(D, k, V, fsec);
    else
        memset(fsec, 0, sizeof(int64_t) * D);
    for (int d = 0; d < D; ++d)
        f[d] = fmain[d] + fsec[d];
}

/* Group concentration matrix: mt_ij = sum_d m_dij = #{d : c_d(i) = c_d(j)}. */
void orc_mtilde(int D, int n, const int16_t *c, int32_t *Mt)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            int32_t m = 0;
            for (int d = 0; d < D; ++d)
                if (c[(size_t)d * n + i] == c[(size_t)d * n + j])
                    m += 1;
            Mt[(size_t)i * n + j] = m;
        }
}

/* x^p with the convention 0^p = 0 (p > 0). */
static double pow0(double x, double p)
{
    return x == 0.0 ? 0.0 : pow(x, p);
}

/* Derivative of the equity fitness with respect to s_{d,i,l}: +1 if the class
 * is above c2, -1 if below c1, 0 otherwise. */
static double dfeq(int32_t v, int32_t c1, int32_t c2)
{
    if (v > c2)
        return 1.0;
    if (v < c1)
        return -1.0;
    return 0.0;
}

/* Gradient of the global loss with respect to the one-hot tensor S,
 * colouring problems:
 *   gS = A.S + 2 alpha lambda t (A o Mt^(alpha-1)).S
 *        - 2 beta mu t ((J - A) o Mt^(beta-1)).S + nu t (grad f_eq or z)
 * partitioning (M -> J - M, so mt -> D - mt and the fitness is the cut):
 *   gS = -A.S - 2 alpha lambda t (A o (D - Mt)^(alpha-1)).S
 *        + 2 beta mu t ((J - A) o (D - Mt)^(beta-1)).S [+ nu t grad f_eq]
 * evaluated at the hard assignment of step 1.  The two element-wise powered
 * n x n matrices are formed once, then each product with S_d is the sum over
 * the vertices j that member d colours l.  gS is [D][n][k]. */
void orc_grad_s(const orc_params *p, int64_t t, const uint8_t *A, const int16_t *c,
                const int32_t *Mt, const int32_t *V, double *gS)
{
    const int n = p->n, k = p->k, D = p->D;
    const double tt = (double)t;
    const double cpen = 2.0 * p->alpha * p->lambda * tt;
    const double cbon = 2.0 * p->beta * p->mu * tt;
    const double ceq = p->nu * tt;
    const int part = is_partition(p);
    const double sgn = part ? -1.0 : 1.0;
    int32_t c1, c2;
    orc_equity_bounds(n, k, &c1, &c2);
    /* P = A o X^(alpha-1), Q = (J - A) o X^(beta-1), X = Mt or D - Mt */
    double *P = (double *)calloc((size_t)n * n, sizeof(double));
    double *Q = (double *)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const size_t e = (size_t)i * n + j;
            const double m = part ? (double)(D - Mt[e]) : (double)Mt[e];
            if (A[e])
                P[e] = pow0(m, p->alpha - 1.0);
            else if (j != i || p->bonus_diag)
                Q[e] = pow0(m, p->beta - 1.0);
        }
    memset(gS, 0, sizeof(double) * (size_t)D * n * k);
    for (int d = 0; d < D; ++d) {
        const int16_t *cd = c + (size_t)d * n;
        for (int i = 0; i < n; ++i) {
            double *g = gS + ((size_t)d * n + i) * k;
            const uint8_t *Ai = A + (size_t)i * n;
            const double *Pi = P + (size_t)i * n;
            const double *Qi = Q + (size_t)i * n;
            for (int j = 0; j < n; ++j) {
                const int l = cd[j];
                g[l] += sgn * (double)Ai[j];    /* gamma matrix term */
                g[l] += sgn * cpen * Pi[j];     /* shared-conflict (shared-cut) penalisation */
                g[l] -= sgn * cbon * Qi[j];     /* shared-assignment (shared-split) bonus */
            }
            if (has_equity(p))
                for (int l = 0; l < k; ++l)
                    g[l] += ceq * dfeq(V[(size_t)d * k + l], c1, c2);
            else if (p->problem == 4)
                for (int l = 0; l < k; ++l)
                    g[l] += ceq * (double)(l + 1);
        }
    }
    free(P);
    free(Q);
}

/* Straight-through softmax gradient:
 *   s_hat = softmax(w) along the colour axis (max subtracted),
 *   gW_j = s_hat_j gS_j - s_hat_j sum_l s_hat_l gS_l. */
void orc_grad_w(int D, int n, int k, const double *W, const double *gS, double *gW)
{
    double *sh = (double *)malloc(sizeof(double) * (size_t)k);
    for (size_t r = 0; r < (size_t)D * n; ++r) {
        const double *w = W + r * k;
        const double *g = gS + r * k;
        double *o = gW + r * k;
        double mx = w[0];
        for (int l = 1; l < k; ++l)
            if (w[l] > mx)
                mx = w[l];
        double z = 0.0;
        for (int l = 0; l < k; ++l) {
            sh[l] = exp(w[l] - mx);
            z += sh[l];
        }
        double rs = 0.0;
        for (int l = 0; l < k; ++l) {
            sh[l] /= z;
            rs += sh[l] * g[l];
        }
        for (int l = 0; l < k; ++l)
            o[l] = sh[l] * g[l] - sh[l] * rs;
    }
    free(sh);
}

/* Step 4 iii-iv: W <- W - eta gW (or, with momentum gamma > 0, v <- gamma v +
 * gW and W <- W - eta v), then W <- W / rho after the update of iteration t
 * when (t+1) mod nb_iter == 0.  vel [D*n*k] is the velocity (unused when
 * gamma = 0). */
void orc_update(const orc_params *p, int64_t t, double *W, const double *gW, double *vel)
{
    const size_t cnt = (size_t)p->D * p->n * p->k;
    const int smooth = p->nb_iter > 0 && ((t + 1) % p->nb_iter) == 0;
    for (size_t e = 0; e < cnt; ++e) {
        double step = gW[e];
        if (p->momentum != 0.0) {
            vel[e] = p->momentum * vel[e] + gW[e];
            step = vel[e];
        }
        double w = W[e] - p->eta * step;
        if (smooth)
            w = w / p->rho;
        W[e] = w;
    }
}

/* Global loss L(t) = sum fmain + nu t sum fsec + lambda t kappa - mu t varpi,
 * with kappa = sum_ij a_ij x_ij^alpha and varpi = sum_ij (1 - a_ij) x_ij^beta
 * (the diagonal in varpi only with bonus_diag), x = mt (colouring) or D - mt
 * (partitioning); fmain is f_color or f_cut, fsec f_eq, f_mscp or 0 (k-COL,
 * where the nu term is absent).  out = {L, sum fmain, sum fsec, kappa, varpi}. */
void orc_loss(const orc_params *p, int64_t t, const uint8_t *A, const int32_t *Mt,
              const int64_t *fmain, const int64_t *fsec, double *out)
{
    const int n = p->n, D = p->D;
    const int part = is_partition(p);
    double sf = 0.0, se = 0.0, kappa = 0.0, varpi = 0.0;
    for (int d = 0; d < D; ++d) {
        sf += (double)fmain[d];
        se += (double)fsec[d];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int32_t mt = Mt[(size_t)i * n + j];
            const double m = part ? (double)(D - mt) : (double)mt;
            if (A[(size_t)i * n + j])
                kappa += pow0(m, p->alpha);
            else if (j != i || p->bonus_diag)
                varpi += pow0(m, p->beta);
        }
    const double tt = (double)t;
    out[0] = sf + p->nu * tt * se + p->lambda * tt * kappa - p->mu * tt * varpi;
    out[1] = sf;
    out[2] = se;
    out[3] = kappa;
    out[4] = varpi;
}

/* ---- multicolouring (Section 6) ----
 * Vertex i has a demand c_i >= 1 and takes c_i different colours: step 1 selects, in each
 * member, the c_i colour groups of largest weight in w_{d,i} (ties go to the lower colour,
 * as for the argmax, which is the case c_i = 1).  S_d is then multi-hot ([D][n][k] bytes),
 * the association m_dij = (S_d S_d^T)_ij counts the colours i and j share, and the fitness,
 * group concentration, loss and gradient keep their tensor forms. */

/* Selection of step 1.  demand[n] (NULL: every c_i = 1).  Returns 0, -5 for a non-finite
 * weight, -1 for a demand outside 1..k. */
int orc_select(int D, int n, int k, const double *W, const int32_t *demand, uint8_t *S)
{
    memset(S, 0, (size_t)D * n * k);
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < n; ++i) {
            const double *w = W + ((size_t)d * n + i) * k;
            uint8_t *srow = S + ((size_t)d * n + i) * k;
            const int ci = demand ? demand[i] : 1;
            if (ci < 1 || ci > k)
                return -1;
            for (int l = 0; l < k; ++l)
                if (!isfinite(w[l]))
                    return -5;
            for (int sel = 0; sel < ci; ++sel) {
                int best = -1;
                for (int l = 0; l < k; ++l)
                    if (!srow[l] && (best < 0 || w[l] > w[best]))
                        best = l;
                srow[best] = 1;
            }
        }
    return 0;
}

/* f_color(S_d) = 1/2 sum_ij a_ij m_dij: over the edges {i, j}, the colours their ends share. */
void orc_fcolor_multi(int D, int n, int k, const uint8_t *A, const uint8_t *S, int64_t *fcol)
{
    for (int d = 0; d < D; ++d) {
        int64_t f = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (A[(size_t)i * n + j]) {
                    const uint8_t *si = S + ((size_t)d * n + i) * k, *sj = S + ((size_t)d * n + j) * k;
                    for (int l = 0; l < k; ++l)
                        f += si[l] & sj[l];
                }
        fcol[d] = f;
    }
}

/* mt_ij = sum_d m_dij, the colours i and j share summed over the members. */
void orc_mtilde_multi(int D, int n, int k, const uint8_t *S, int32_t *Mt)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            int32_t m = 0;
            for (int d = 0; d < D; ++d) {
                const uint8_t *si = S + ((size_t)d * n + i) * k, *sj = S + ((size_t)d * n + j) * k;
                for (int l = 0; l < k; ++l)
                    m += si[l] & sj[l];
            }
            Mt[(size_t)i * n + j] = m;
        }
}

/* #V_{d,l}: the vertices of member d holding colour l. */
void orc_class_sizes_multi(int D, int n, int k, const uint8_t *S, int32_t *V)
{
    memset(V, 0, sizeof(int32_t) * (size_t)D * k);
    for (int d = 0; d < D; ++d)
        for (int i = 0; i < n; ++i)
            for (int l = 0; l < k; ++l)
                V[(size_t)d * k + l] += S[((size_t)d * n + i) * k + l];
}

/* Gradient of the global loss with respect to S (colouring form, no added term):
 *   gS = A.S + 2 alpha lambda t (A o Mt^(alpha-1)).S - 2 beta mu t ((J - A) o Mt^(beta-1)).S
 * with the products taken over the selected colours of every j. */
void orc_grad_s_multi(const orc_params *p, int64_t t, const uint8_t *A, const uint8_t *S,
                      const int32_t *Mt, double *gS)
{
    const int n = p->n, k = p->k, D = p->D;
    const double tt = (double)t;
    const double cpen = 2.0 * p->alpha * p->lambda * tt;
    const double cbon = 2.0 * p->beta * p->mu * tt;
    memset(gS, 0, sizeof(double) * (size_t)D * n * k);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const size_t e = (size_t)i * n + j;
            const double m = (double)Mt[e];
            double w = 0.0;
            if (A[e])
                w = 1.0 + cpen * pow0(m, p->alpha - 1.0);
            else if (j != i || p->bonus_diag)
                w = -cbon * pow0(m, p->beta - 1.0);
            if (w == 0.0)
                continue;
            for (int d = 0; d < D; ++d) {
                const uint8_t *sj = S + ((size_t)d * n + j) * k;
                double *g = gS + ((size_t)d * n + i) * k;
                for (int l = 0; l < k; ++l)
                    if (sj[l])
                        g[l] += w;
            }
        }
}

/* One multicolouring iteration (steps 1-4) on W (updated in place); outputs may be NULL.
 * Returns 1 if a member is legal (f_color = 0: no update, *legal_d the lowest such member
 * when stop_on_legal), 0 after an update, or a negative error. */
int orc_iteration_multi(const orc_params *p, int64_t *t, const uint8_t *A, const int32_t *demand, double *W,
                        uint8_t *S_out, int64_t *f_out, double *gS_out, double *gW_out, int32_t *legal_d)
{
    const int n = p->n, k = p->k, D = p->D;
    const size_t dnk = (size_t)D * n * k;
    if (p->momentum != 0.0)
        return -1;
    uint8_t *S = (uint8_t *)malloc(dnk);
    int32_t *Mt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * n);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * D);
    double *gS = (double *)malloc(sizeof(double) * dnk);
    double *gW = (double *)malloc(sizeof(double) * dnk);
    int rc = (S && Mt && f && gS && gW) ? 0 : -6;
    if (!rc)
        rc = orc_select(D, n, k, W, demand, S);
    if (!rc) {
        orc_fcolor_multi(D, n, k, A, S, f);
        int best = -1;
        for (int d = 0; d < D; ++d)
            if (f[d] == 0 && best < 0) best = d;
        if (S_out) memcpy(S_out, S, dnk);
        if (f_out) memcpy(f_out, f, sizeof(int64_t) * D);
        if (legal_d) *legal_d = best;
        if (best >= 0 && p->stop_on_legal) {
            rc = 1;
        } else {
            orc_mtilde_multi(D, n, k, S, Mt);
            orc_grad_s_multi(p, *t, A, S, Mt, gS);
            orc_grad_w(D, n, k, W, gS, gW);
            if (gS_out) memcpy(gS_out, gS, sizeof(double) * dnk);
            if (gW_out) memcpy(gW_out, gW, sizeof(double) * dnk);
            orc_update(p, *t, W, gW, NULL);
            *t += 1;
        }
    }
    free(S); free(Mt); free(f); free(gS); free(gW);
    return rc;
}

/* Work arrays for one iteration. */
typedef struct {
    int16_t *c;
    int32_t *V, *Mt;
    int64_t *fcol, *feq;
    double *gS, *gW;
} orc_work;

static int work_alloc(const orc_params *p, orc_work *w)
{
    const size_t D = p->D, n = p->n, k = p->k;
    w->c = (int16_t *)malloc(sizeof(int16_t) * D * n);
    w->V = (int32_t *)malloc(sizeof(int32_t) * D * k);
    w->Mt = (int32_t *)malloc(sizeof(int32_t) * n * n);
    w->fcol = (int64_t *)malloc(sizeof(int64_t) * D);
    w->feq = (int64_t *)malloc(sizeof(int64_t) * D);
    w->gS = (double *)malloc(sizeof(double) * D * n * k);
    w->gW = (double *)malloc(sizeof(double) * D * n * k);
    return (w->c && w->V && w->Mt && w->fcol && w->feq && w->gS && w->gW) ? 0 : -6;
}

static void work_free(orc_work *w)
{
    free(w->c); free(w->V); free(w->Mt); free(w->fcol); free(w->feq);
    free(w->gS); free(w->gW);
}

/* One iteration of the algorithm on member weights W (updated in place).
 * Outputs (any may be NULL): colours c [D*n], fitness f = fmain + fsec [D],
 * fmain (f_color or f_cut) [D], fsec (f_eq, f_mscp or 0) [D], the gradients gS
 * and gW [D*n*k] of this iteration.  vel [D*n*k] is the momentum state (may be
 * NULL when momentum = 0).  Returns 1 if the population held a member with
 * f = 0 (no update; *legal_d set to the lowest such member when
 * stop_on_legal), 0 after an update, or a negative error (-5 non-finite
 * weight, -6 out of memory). */
int orc_iteration(const orc_params *p, int64_t *t, const uint8_t *A, double *W, double *vel,
                  int16_t *c_out, int64_t *f_out, int64_t *fmain_out, int64_t *fsec_out,
                  double *gS_out, double *gW_out, int32_t *legal_d)
{
    const int n = p->n, k = p->k, D = p->D;
    if (p->momentum != 0.0 && !vel)
        return -1;
    orc_work w;
    if (work_alloc(p, &w)) {
        work_free(&w);
        return -6;
    }
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * D);
    if (!f) {
        work_free(&w);
        return -6;
    }
    int rc = orc_colors(D, n, k, W, w.c);
    if (rc) {
        free(f);
        work_free(&w);
        return rc;
    }
    orc_class_sizes(D, n, k, w.c, w.V);
    orc_fitness(p, A, w.c, w.V, w.fcol, w.feq, f);
    int best = -1;
    for (int d = 0; d < D; ++d)
        if (f[d] == 0 && best < 0) best = d;
    if (f_out) memcpy(f_out, f, sizeof(int64_t) * D);
    free(f);
    if (c_out) memcpy(c_out, w.c, sizeof(int16_t) * (size_t)D * n);
    if (fmain_out) memcpy(fmain_out, w.fcol, sizeof(int64_t) * D);
    if (fsec_out) memcpy(fsec_out, w.feq, sizeof(int64_t) * D);
    if (legal_d) *legal_d = best;
    if (best >= 0 && p->stop_on_legal) {
        work_free(&w);
        return 1;
    }
    orc_mtilde(D, n, w.c, w.Mt);
    orc_grad_s(p, *t, A, w.c, w.Mt, w.V, w.gS);
    orc_grad_w(D, n, k, W, w.gS, w.gW);
    if (gS_out) memcpy(gS_out, w.gS, sizeof(double) * (size_t)D * n * k);
    if (gW_out) memcpy(gW_out, w.gW, sizeof(double) * (size_t)D * n * k);
    orc_update(p, *t, W, w.gW, vel);
    *t += 1;
    work_free(&w);
    return 0;
}

/* Algorithm loop: up to max_steps iterations (momentum state from zero).
 * Returns the number of updates performed; *legal_d is the returned member (or
 * -1) and colors_out [n] its colouring when one was found. */
int orc_run(const orc_params *p, int64_t *t, const uint8_t *A, double *W, int max_steps,
            int32_t *legal_d, int16_t *colors_out)
{
    const int n = p->n, D = p->D;
    int16_t *c = (int16_t *)malloc(sizeof(int16_t) * (size_t)D * n);
    double *vel = p->momentum != 0.0 ? (double *)calloc((size_t)D * n * p->k, sizeof(double)) : NULL;
    int done = 0;
    *legal_d = -1;
    for (int s = 0; s < max_steps; ++s) {
        int32_t ld = -1;
        int rc = orc_iteration(p, t, A, W, vel, c, NULL, NULL, NULL, NULL, NULL, &ld);
        if (rc < 0) {
            free(c);
            free(vel);
            return rc;
        }
        if (rc == 1) {
            *legal_d = ld;
            if (colors_out)
                memcpy(colors_out, c + (size_t)ld * n, sizeof(int16_t) * n);
            break;
        }
        done += 1;
    }
    free(c);
    free(vel);
    return done;
}

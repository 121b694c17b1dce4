/*
 * vest_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for VeST
 * (M. Park, J.-G. Jang, L. Sael, "VeST: Very Sparse Tucker Factorization of
 * Large-Scale Tensors", arXiv:1904.02603).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library; the two meet only through the seeded synthetic
 * inputs.  Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math.  An
 * optional OpenMP build of the same source (-fopenmp) splits only loops whose
 * iterations are independent sums (factor rows, residual entries, keys), so
 * it returns the same bits; the sequential core update stays sequential.
 *
 * Conventions (all 0-based):
 *   idx[e*N + n]        mode-n index of observed entry e (canonical entry id e)
 *   A_n[i*J_n + j]      factor matrix n, row-major
 *   G[beta]             core, row-major flat index (last mode fastest)
 *   fmask_n[i*J_n + j]  1 = pruned (marking table, Sec. 3.3), same for cmask
 *
 * Readings of the paper that this file takes:
 *   - Within a factor row the update is Gauss-Seidel over j ascending, in
 *     place (Alg. 4).  delta, v and the numerator sum do not depend on row
 *     i_n of A^(n), so they are formed once per row instead of once per j;
 *     the values are identical.
 *   - The L1 factor rule (Eq. 13) uses g = -2 (sum X delta(j) - sum_{t!=j}
 *     v(t) a_t), d = 2 v(j): the gradient of the squared error at a = 0,
 *     consistent with g_c of Eq. 14.  The printed g_fm drops the sign and the
 *     factor 2 on its second term.
 *   - The sequential core update visits beta in row-major flat order and
 *     skips marked elements (Sec. 3.5 leaves the order open).
 *   - ||X||_F in Eq. 4 is taken over the observed entries Omega.
 *   - Pruning ranks by the key Delta(e) = SSE(e set to 0) - SSE, which is
 *     ||X||^2 (RE(e)^2 - RE^2) and orders exactly like Resp(e) of Eq. 3 when
 *     RE > 0; ties are broken by ascending flat index.  The core step of
 *     Alg. 3 omits the square; Eq. 5 is used.
 *   - The paper fixes no summation order.  Every sum of this file (delta and
 *     B over the core elements, the row and core statistics over entries, the
 *     loss) is Neumaier-compensated, so that its result is close to the
 *     correctly rounded one whatever the order; the FP64 comparison with the
 *     GPU is then a comparison with (nearly) the exact value.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_MAX_ORDER 10
#define OR_MAX_RANK 64                 /* row_stats holds a delta of this length */

typedef struct {
    int32_t order;                    /* N */
    int32_t reg;                      /* 0 = L_F (Eq. 1), 1 = L_1 (Eq. 2) */
    double lambda;
    int64_t nnz;                      /* |Omega| */
    int64_t dims[OR_MAX_ORDER];       /* I_n */
    int32_t ranks[OR_MAX_ORDER];      /* J_n */
    const int32_t *idx;               /* nnz*N */
    const double *val;                /* nnz */
    double *factors[OR_MAX_ORDER];    /* I_n*J_n */
    double *core;                     /* prod J_n */
    uint8_t *fmask[OR_MAX_ORDER];     /* I_n*J_n */
    uint8_t *cmask;                   /* prod J_n */
    /* Omega_{i_n}^{(n)} (Table 1): entries of row i of mode n, ascending id */
    int64_t *row_ptr[OR_MAX_ORDER];   /* I_n + 1 */
    int64_t *row_ent[OR_MAX_ORDER];   /* nnz */
} or_state;

/* ---------------- Neumaier compensated summation ------------------------- */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else                       k->c += (x - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

static int64_t core_size(const or_state *st)
{
    int64_t s = 1;
    for (int n = 0; n < st->order; ++n) s *= st->ranks[n];
    return s;
}

/* Decompose a row-major flat core index into (j_1..j_N). */
static void unflatten(const or_state *st, int64_t beta, int32_t *j)
{
    for (int n = st->order - 1; n >= 0; --n) {
        j[n] = (int32_t)(beta % st->ranks[n]);
        beta /= st->ranks[n];
    }
}

/* ---------------- Omega_{i_n}^{(n)} row lists ---------------------------- */
/* Stable counting sort of the entry ids by their mode-n index. */
int or_build_rows(or_state *st)
{
    for (int n = 0; n < st->order; ++n) {
        int64_t I = st->dims[n];
        int64_t *ptr = (int64_t *)calloc((size_t)I + 1, sizeof(int64_t));
        int64_t *ent = (int64_t *)malloc((size_t)(st->nnz > 0 ? st->nnz : 1) * sizeof(int64_t));
        int64_t *cur = (int64_t *)malloc((size_t)I * sizeof(int64_t));
        if (!ptr || !ent || !cur) { free(ptr); free(ent); free(cur); return -1; }
        for (int64_t e = 0; e < st->nnz; ++e) {
            int32_t i = st->idx[e * st->order + n];
            if (i < 0 || i >= I) { free(ptr); free(ent); free(cur); return -2; }
            ptr[i + 1]++;
        }
        for (int64_t i = 0; i < I; ++i) ptr[i + 1] += ptr[i];
        for (int64_t i = 0; i < I; ++i) cur[i] = ptr[i];
        for (int64_t e = 0; e < st->nnz; ++e) {
            int32_t i = st->idx[e * st->order + n];
            ent[cur[i]++] = e;
        }
        free(cur);
        st->row_ptr[n] = ptr;
        st->row_ent[n] = ent;
    }
    return 0;
}

void or_free_rows(or_state *st)
{
    for (int n = 0; n < st->order; ++n) {
        free(st->row_ptr[n]); st->row_ptr[n] = NULL;
        free(st->row_ent[n]); st->row_ent[n] = NULL;
    }
}

/* ---------------- Eq. 11: delta_alpha^{(n)} ------------------------------ */
/* delta(j) = sum over core elements beta with beta_n = j of
 *            G_beta * prod_{k != n} a^(k)_{i_k beta_k}
 * evaluated directly over every beta in flat order (no factoring). */
void or_delta(const or_state *st, int32_t n, int64_t e, double *delta)
{
    int32_t j[OR_MAX_ORDER];
    const int32_t *a = st->idx + e * st->order;
    int64_t G = core_size(st);
    ksum acc[OR_MAX_RANK];
    for (int32_t t = 0; t < st->ranks[n]; ++t) acc[t].s = acc[t].c = 0.0;
    for (int64_t beta = 0; beta < G; ++beta) {
        unflatten(st, beta, j);
        double p = st->core[beta];
        for (int k = 0; k < st->order; ++k) {
            if (k == n) continue;
            p *= st->factors[k][(int64_t)a[k] * st->ranks[k] + j[k]];
        }
        ks_add(&acc[j[n]], p);
    }
    for (int32_t t = 0; t < st->ranks[n]; ++t) delta[t] = ks_val(&acc[t]);
}

/* ---------------- Eq. 7: entry-wise reconstruction B(alpha) -------------- */
double or_recon(const or_state *st, int64_t e)
{
    int32_t j[OR_MAX_ORDER];
    const int32_t *a = st->idx + e * st->order;
    int64_t G = core_size(st);
    ksum b = {0, 0};
    for (int64_t beta = 0; beta < G; ++beta) {
        unflatten(st, beta, j);
        double p = st->core[beta];
        for (int k = 0; k < st->order; ++k)
            p *= st->factors[k][(int64_t)a[k] * st->ranks[k] + j[k]];
        ks_add(&b, p);
    }
    return ks_val(&b);
}

/* Residuals X_alpha - B(alpha) for every observed entry (first step of Alg. 3). */
void or_residual(const or_state *st, double *res)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < st->nnz; ++e) res[e] = st->val[e] - or_recon(st, e);
}

/* ---------------- one-dimensional minimisers ----------------------------- */
/* Minimiser along one coordinate of  den*x^2 - 2*num*x + regulariser(x):
 *   L_F (Eq. 9 / Eq. 12):  num / (den + lambda)
 *   L_1 (Eq. 13 / Eq. 14): soft threshold with g = -2 num, d = 2 den. */
static double coord_min(int reg, double lambda, double num, double den)
{
    if (reg == 0) return num / (den + lambda);
    double g = -2.0 * num, d = 2.0 * den;
    if (g > lambda)  return (lambda - g) / d;
    if (g < -lambda) return -(lambda + g) / d;
    return 0.0;
}

/* ---------------- Alg. 4: one factor row --------------------------------- */
/* Accumulate, over Omega_i^{(n)}, c(j) = sum X delta(j) and the symmetric
 * v(t, j) = sum delta(t) delta(j) (Eq. 9 numerator, Eq. 10), compensated. */
static void row_stats(const or_state *st, int32_t n, int64_t i, double *c, double *V)
{
    int32_t J = st->ranks[n];
    double delta[64];
    ksum *kc = (ksum *)calloc((size_t)J, sizeof(ksum));
    ksum *kv = (ksum *)calloc((size_t)J * J, sizeof(ksum));
    for (int64_t p = st->row_ptr[n][i]; p < st->row_ptr[n][i + 1]; ++p) {
        int64_t e = st->row_ent[n][p];
        or_delta(st, n, e, delta);
        double x = st->val[e];
        for (int32_t t = 0; t < J; ++t) {
            ks_add(&kc[t], x * delta[t]);
            for (int32_t u = 0; u < J; ++u) ks_add(&kv[t * J + u], delta[t] * delta[u]);
        }
    }
    for (int32_t t = 0; t < J; ++t) {
        c[t] = ks_val(&kc[t]);
        for (int32_t u = 0; u < J; ++u) V[t * J + u] = ks_val(&kv[t * J + u]);
    }
    free(kc); free(kv);
}

/* Coordinate update of a^(n)_{i j} given the row statistics. */
static void update_coord(const or_state *st, int32_t n, int64_t i, int32_t j,
                         const double *c, const double *V)
{
    int32_t J = st->ranks[n];
    double *a = st->factors[n] + i * J;
    double r = c[j];
    for (int32_t t = 0; t < J; ++t) {
        if (t == j) continue;
        r -= V[j * J + t] * a[t];
    }
    a[j] = coord_min(st->reg, st->lambda, r, V[j * J + j]);
}

/* Update every unpruned element of row i of A^(n), j ascending (Alg. 4). */
void or_update_row(or_state *st, int32_t n, int64_t i)
{
    int32_t J = st->ranks[n];
    double c[64], V[64 * 64];
    row_stats(st, n, i, c, V);
    for (int32_t j = 0; j < J; ++j) {
        if (st->fmask[n][i * J + j]) continue;
        update_coord(st, n, i, j, c, V);
    }
}

/* Update a single element a^(n)_{i j} (Lemma for Eq. 9 / Eq. 13). */
void or_update_factor_elem(or_state *st, int32_t n, int64_t i, int32_t j)
{
    int32_t J = st->ranks[n];
    double c[64], V[64 * 64];
    if (st->fmask[n][i * J + j]) return;
    row_stats(st, n, i, c, V);
    update_coord(st, n, i, j, c, V);
}

/* One pass of Alg. 4 over all rows of mode n. */
void or_sweep_factor(or_state *st, int32_t n)
{
    /* rows are independent (each reads the other modes and writes its own
       row), so the optional OpenMP build gives the same bits */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < st->dims[n]; ++i) or_update_row(st, n, i);
}

/* ---------------- Eq. 12 / Eq. 14: core update --------------------------- */
/* w_beta(alpha) = prod_n a^(n)_{i_n beta_n} */
static double core_weight(const or_state *st, int64_t e, const int32_t *j)
{
    const int32_t *a = st->idx + e * st->order;
    double w = 1.0;
    for (int k = 0; k < st->order; ++k)
        w *= st->factors[k][(int64_t)a[k] * st->ranks[k] + j[k]];
    return w;
}

/* Update G_beta given the current residuals res (= X - B), then correct res. */
static void core_coord(or_state *st, int64_t beta, double *res)
{
    int32_t j[OR_MAX_ORDER];
    unflatten(st, beta, j);
    double g = st->core[beta];
    ksum num = {0, 0}, den = {0, 0};
    for (int64_t e = 0; e < st->nnz; ++e) {
        double w = core_weight(st, e, j);
        /* X - sum_{gamma != beta} G_gamma w_gamma = res + G_beta w_beta */
        ks_add(&num, (res[e] + g * w) * w);
        ks_add(&den, w * w);
    }
    double gn = coord_min(st->reg, st->lambda, ks_val(&num), ks_val(&den));
    double dg = gn - g;
    if (dg != 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < st->nnz; ++e) res[e] -= dg * core_weight(st, e, j);
    }
    st->core[beta] = gn;
}

/* Update a single unpruned core element (residuals recomputed from scratch). */
void or_update_core_elem(or_state *st, int64_t beta)
{
    if (st->cmask[beta]) return;
    double *res = (double *)malloc((size_t)(st->nnz > 0 ? st->nnz : 1) * sizeof(double));
    or_residual(st, res);
    core_coord(st, beta, res);
    free(res);
}

/* Sequential pass over all unpruned core elements in flat order (Sec. 3.5). */
void or_sweep_core(or_state *st)
{
    int64_t G = core_size(st);
    double *res = (double *)malloc((size_t)(st->nnz > 0 ? st->nnz : 1) * sizeof(double));
    or_residual(st, res);
    for (int64_t beta = 0; beta < G; ++beta) {
        if (st->cmask[beta]) continue;
        core_coord(st, beta, res);
    }
    free(res);
}

/* ---------------- Eq. 1 / 2 / 4: loss and RE ----------------------------- */
/* out = {SSE, ||X||^2 over Omega, regulariser, loss, RE} */
void or_loss(const or_state *st, double *out)
{
    ksum sse = {0, 0}, xx = {0, 0}, reg = {0, 0};
    for (int64_t e = 0; e < st->nnz; ++e) {
        double r = st->val[e] - or_recon(st, e);
        ks_add(&sse, r * r);
        ks_add(&xx, st->val[e] * st->val[e]);
    }
    int64_t G = core_size(st);
    for (int64_t b = 0; b < G; ++b) {
        double g = st->core[b];
        ks_add(&reg, st->reg == 0 ? g * g : fabs(g));
    }
    for (int n = 0; n < st->order; ++n) {
        int64_t cnt = st->dims[n] * st->ranks[n];
        for (int64_t q = 0; q < cnt; ++q) {
            double a = st->factors[n][q];
            ks_add(&reg, st->reg == 0 ? a * a : fabs(a));
        }
    }
    out[0] = ks_val(&sse);
    out[1] = ks_val(&xx);
    out[2] = st->lambda * ks_val(&reg);
    out[3] = out[0] + out[2];
    out[4] = out[1] > 0 ? sqrt(out[0]) / sqrt(out[1]) : 0.0;
}

/* ---------------- Eq. 5 / Eq. 6: responsibility keys --------------------- */
/* Delta(e) = SSE with e set to 0 minus SSE, from one snapshot of the state:
 *   core   (Eq. 5): sum_Omega (2 res + G_g w_g) G_g w_g
 *   factor (Eq. 6): sum_{Omega_i} (2 res + B_{j_n=j}) B_{j_n=j},
 *                   B_{j_n=j}(alpha) = a_ij delta_alpha(j)      (Eq. 8)
 * Pruned elements get +infinity so that they are never selected again. */
void or_responsibility(const or_state *st, double *core_key, double **factor_key)
{
    double *res = (double *)malloc((size_t)(st->nnz > 0 ? st->nnz : 1) * sizeof(double));
    or_residual(st, res);
    int64_t G = core_size(st);
    /* every key is its own sum from the same snapshot: the optional OpenMP
       build gives the same bits */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t beta = 0; beta < G; ++beta) {
        int32_t j[OR_MAX_ORDER];
        if (st->cmask[beta]) { core_key[beta] = INFINITY; continue; }
        unflatten(st, beta, j);
        double g = st->core[beta];
        ksum k = {0, 0};
        for (int64_t e = 0; e < st->nnz; ++e) {
            double part = g * core_weight(st, e, j);
            ks_add(&k, (2.0 * res[e] + part) * part);
        }
        core_key[beta] = ks_val(&k);
    }
    for (int n = 0; n < st->order; ++n) {
        int32_t J = st->ranks[n];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < st->dims[n]; ++i) {
            double delta[OR_MAX_RANK];
            ksum k[OR_MAX_RANK];
            const double *a = st->factors[n] + i * J;
            for (int32_t t = 0; t < J; ++t) k[t].s = k[t].c = 0.0;
            for (int64_t p = st->row_ptr[n][i]; p < st->row_ptr[n][i + 1]; ++p) {
                int64_t e = st->row_ent[n][p];
                or_delta(st, n, e, delta);
                for (int32_t t = 0; t < J; ++t) {
                    double part = a[t] * delta[t];
                    ks_add(&k[t], (2.0 * res[e] + part) * part);
                }
            }
            for (int32_t t = 0; t < J; ++t)
                factor_key[n][i * J + t] = st->fmask[n][i * J + t] ? INFINITY : ks_val(&k[t]);
        }
    }
    free(res);
}

/* ---------------- Sec. 3.3 / Alg. 3: pruning ----------------------------- */
typedef struct { double key; int64_t pos; } kp;
static int kp_cmp(const void *x, const void *y)
{
    const kp *a = (const kp *)x, *b = (const kp *)y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* Zero and mark the k unmarked elements with the smallest (key, flat index).
 * Returns the number pruned, or -1 if k exceeds the unmarked count. */
static int64_t prune_tensor(double *vals, uint8_t *mask, const double *key, int64_t cnt, int64_t k)
{
    if (k <= 0) return 0;
    kp *c = (kp *)malloc((size_t)cnt * sizeof(kp));
    int64_t m = 0;
    for (int64_t q = 0; q < cnt; ++q)
        if (!mask[q]) { c[m].key = key[q]; c[m].pos = q; ++m; }
    if (k > m) { free(c); return -1; }
    qsort(c, (size_t)m, sizeof(kp), kp_cmp);
    for (int64_t q = 0; q < k; ++q) { vals[c[q].pos] = 0.0; mask[c[q].pos] = 1; }
    free(c);
    return k;
}

int or_prune(or_state *st, const double *core_key, double *const *factor_key,
             int64_t core_k, const int64_t *factor_k)
{
    if (prune_tensor(st->core, st->cmask, core_key, core_size(st), core_k) < 0) return -1;
    for (int n = 0; n < st->order; ++n)
        if (prune_tensor(st->factors[n], st->fmask[n], factor_key[n],
                         st->dims[n] * st->ranks[n], factor_k[n]) < 0) return -1;
    return 0;
}

/* ---------------- Alg. 2, final step: column normalisation -------------- */
/* A^(n) = U^(n) B^(n), columns of U unit length, B diagonal of column norms;
 * G <- G x_n B^(n).  A zero column stays zero and scales its core slice by 0. */
void or_normalize(or_state *st)
{
    int32_t j[OR_MAX_ORDER];
    int64_t G = core_size(st);
    for (int n = 0; n < st->order; ++n) {
        int32_t J = st->ranks[n];
        double nrm[64];
        for (int32_t t = 0; t < J; ++t) {
            ksum k = {0, 0};
            for (int64_t i = 0; i < st->dims[n]; ++i) {
                double a = st->factors[n][i * J + t];
                ks_add(&k, a * a);
            }
            nrm[t] = sqrt(ks_val(&k));
            for (int64_t i = 0; i < st->dims[n]; ++i)
                if (nrm[t] > 0) st->factors[n][i * J + t] /= nrm[t];
        }
        for (int64_t beta = 0; beta < G; ++beta) {
            unflatten(st, beta, j);
            st->core[beta] *= nrm[j[n]];
        }
    }
}

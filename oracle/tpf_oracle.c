/*
 * tpf_oracle.c -- plain FP64 CPU oracle of the batched fixed-point power flow.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * Paper: J. S. Giraldo / E. Salazar Duque et al., "Tensor Power Flow Formulations
 * for Multidimensional Analyses in Distribution Systems" (arXiv 2403.04578).
 *
 * What it computes, each step written out plainly in double complex arithmetic
 * (compiled with -ffp-contract=off, no BLAS, no blocking, no fusion):
 *   oracle_build     Sec. II Eq. (1): nodal admittance Y from the branch list,
 *                    partition into slack (s) and demand (d) blocks; Eq. (2) with
 *                    constant-power loads (alpha_P = 1, alpha_Z = alpha_I = 0):
 *                    B = Y_dd, F = -B^-1 diag(s*), w = -B^-1 Y_ds v_s.  We keep
 *                    Z = -Y_dd^-1 (Algorithm 1's Z_B with the sign Eq. (2) needs).
 *   oracle_fpi       Algorithm 1 (dense tensor power flow) applied column by
 *                    column: flat start 1 + j0, update V <- Z conj(S ./ V) + w,
 *                    stop when max_i |V'_i - V_i| < tol or after max_iter sweeps.
 *   oracle_mismatch  Power balance of Eq. (1): m = S + V .* conj(Y_ds v_s + Y_dd V),
 *                    reported as max_i |m_i| per column.
 *   oracle_build_3ph Sec. II Eq. (1) written per phase node for a three-phase network:
 *                    each branch's 3x3 series impedance matrix is inverted and stamped
 *                    as a block; the slack bus's three nodes form the slack block.
 *   oracle_fpi_zip   Eq. (2) with a ZIP load model whose constant-impedance share is
 *                    zero: per column A = diag(alpha_P .* s*), B = Y_dd,
 *                    c = Y_ds v_s + alpha_I .* s*, F = -B^-1 A, w = -B^-1 c, then
 *                    Algorithm 1 with v <- F conj(v)^-1 + w.
 *   oracle_fpi_zipz  Eq. (2) with the full ZIP model: per column B = diag(alpha_Z .* s*)
 *                    + Y_dd now depends on s, so F = -B^-1 A and w = -B^-1 c are formed
 *                    per column by Gauss-Jordan elimination with partial pivoting on
 *                    [B | A | c], then Algorithm 1 with v <- F conj(v)^-1 + w.
 *   oracle_mismatch_zip  The power balance of the same loads: a load draws
 *                    v .* conj(i) with i = alpha_I .* s* + alpha_P .* s* ./ conj(v),
 *                    i.e. s .* (alpha_P + alpha_I .* v), so
 *                    m = S .* (alpha_P + alpha_I .* V) + V .* conj(Y_ds v_s + Y_dd V);
 *                    a constant-impedance share adds the current alpha_Z .* s* .* v,
 *                    drawing alpha_Z .* s .* |v|^2.
 *
 * Readings where the paper is silent or garbled (listed in the design notes):
 *   - the stopping measure is the complex modulus of the voltage step,
 *     per column, not squared, with a strict test d < tol;
 *   - a column whose iterate becomes non-finite stops with status NONFINITE;
 *   - max_iter = 0 returns the start voltages with status MAX_ITER.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID -1
#define OR_ERR_SINGULAR -2
#define OR_ERR_OOM -4

#define ST_CONVERGED 0
#define ST_MAX_ITER 1
#define ST_NONFINITE 2

/* Sec. II Eq. (1) and Eq. (2).  Outputs (caller-allocated, interleaved re/im):
 *   Ydd [n*n], Yds [n], Z [n*n] = -Y_dd^-1, w [n] = -Y_dd^-1 Y_ds v_s,
 * with n = n_bus - 1 and PQ bus order = ascending bus index, slack removed. */
int oracle_build(int n_bus, int n_branch, const int32_t *frm, const int32_t *to,
                 const double *r, const double *x, int slack, double vs_re,
                 double vs_im, double complex *Ydd, double complex *Yds,
                 double complex *Z, double complex *w)
{
    if (n_bus < 2 || n_branch < 1 || slack < 0 || slack >= n_bus)
        return OR_ERR_INVALID;
    const int n = n_bus - 1;
    double complex *Y = calloc((size_t)n_bus * n_bus, sizeof(double complex));
    double complex *M = calloc((size_t)n * 2 * n, sizeof(double complex));
    int *pq = malloc(sizeof(int) * n);
    if (!Y || !M || !pq) {
        free(Y); free(M); free(pq);
        return OR_ERR_OOM;
    }
    int rc = OR_OK;
    /* Eq. (1): series branch admittance y = 1/(r + jx) stamped into Y. */
    for (int k = 0; k < n_branch; ++k) {
        int f = frm[k], t = to[k];
        if (f < 0 || f >= n_bus || t < 0 || t >= n_bus || f == t ||
            !isfinite(r[k]) || !isfinite(x[k]) || (r[k] == 0.0 && x[k] == 0.0)) {
            rc = OR_ERR_INVALID;
            goto done;
        }
        double complex y = 1.0 / (r[k] + I * x[k]);
        Y[(size_t)f * n_bus + f] += y;
        Y[(size_t)t * n_bus + t] += y;
        Y[(size_t)f * n_bus + t] -= y;
        Y[(size_t)t * n_bus + f] -= y;
    }
    /* Partition: demand nodes are every bus but the slack, ascending. */
    for (int b = 0, i = 0; b < n_bus; ++b)
        if (b != slack) pq[i++] = b;
    for (int i = 0; i < n; ++i) {
        Yds[i] = Y[(size_t)pq[i] * n_bus + slack];
        for (int j = 0; j < n; ++j)
            Ydd[(size_t)i * n + j] = Y[(size_t)pq[i] * n_bus + pq[j]];
    }
    /* Y_dd^-1 by Gauss-Jordan elimination with partial pivoting on [Y_dd | 1]. */
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[(size_t)i * 2 * n + j] = Ydd[(size_t)i * n + j];
        M[(size_t)i * 2 * n + n + i] = 1.0;
    }
    double scale = 0.0;
    for (size_t e = 0; e < (size_t)n * n; ++e) scale = fmax(scale, cabs(Ydd[e]));
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = cabs(M[(size_t)c * 2 * n + c]);
        for (int i = c + 1; i < n; ++i) {
            double v = cabs(M[(size_t)i * 2 * n + c]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > 1e-13 * scale)) { rc = OR_ERR_SINGULAR; goto done; }
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double complex tmp = M[(size_t)c * 2 * n + j];
                M[(size_t)c * 2 * n + j] = M[(size_t)p * 2 * n + j];
                M[(size_t)p * 2 * n + j] = tmp;
            }
        double complex piv = M[(size_t)c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) M[(size_t)c * 2 * n + j] /= piv;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            double complex f = M[(size_t)i * 2 * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j)
                M[(size_t)i * 2 * n + j] -= f * M[(size_t)c * 2 * n + j];
        }
    }
    /* Z = -Y_dd^-1 ; w = -Y_dd^-1 Y_ds v_s = Z (Y_ds v_s). */
    double complex vs = vs_re + I * vs_im;
    for (int i = 0; i < n; ++i) {
        double complex acc = 0.0;
        for (int j = 0; j < n; ++j) {
            Z[(size_t)i * n + j] = -M[(size_t)i * 2 * n + n + j];
            acc += Z[(size_t)i * n + j] * (Yds[j] * vs);
        }
        w[i] = acc;
    }
done:
    free(Y); free(M); free(pq);
    return rc;
}

/* Inverse of an m x m complex matrix by Gauss-Jordan elimination with partial pivoting
 * on [A | 1]; work holds m * 2m entries.  Returns 0, or OR_ERR_SINGULAR. */
static int gj_inverse(const double complex *A, int m, double complex *Ainv, double complex *work)
{
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < 2 * m; ++j) work[(size_t)i * 2 * m + j] = 0.0;
        for (int j = 0; j < m; ++j) work[(size_t)i * 2 * m + j] = A[(size_t)i * m + j];
        work[(size_t)i * 2 * m + m + i] = 1.0;
    }
    double scale = 0.0;
    for (size_t e = 0; e < (size_t)m * m; ++e) scale = fmax(scale, cabs(A[e]));
    for (int c = 0; c < m; ++c) {
        int p = c;
        double best = cabs(work[(size_t)c * 2 * m + c]);
        for (int i = c + 1; i < m; ++i) {
            double v = cabs(work[(size_t)i * 2 * m + c]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > 1e-13 * scale)) return OR_ERR_SINGULAR;
        if (p != c)
            for (int j = 0; j < 2 * m; ++j) {
                double complex tmp = work[(size_t)c * 2 * m + j];
                work[(size_t)c * 2 * m + j] = work[(size_t)p * 2 * m + j];
                work[(size_t)p * 2 * m + j] = tmp;
            }
        double complex piv = work[(size_t)c * 2 * m + c];
        for (int j = 0; j < 2 * m; ++j) work[(size_t)c * 2 * m + j] /= piv;
        for (int i = 0; i < m; ++i) {
            if (i == c) continue;
            double complex f = work[(size_t)i * 2 * m + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * m; ++j) work[(size_t)i * 2 * m + j] -= f * work[(size_t)c * 2 * m + j];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Ainv[(size_t)i * m + j] = work[(size_t)i * 2 * m + m + j];
    return OR_OK;
}

/* Sec. II Eq. (1) per phase node (three phases).  Node 3 b + p is phase p of bus b.
 * Each branch stamps Y_b = zabc_k^-1 (zabc: [n_branch][3][3]) as a 3x3 block; the slack
 * bus's nodes are the slack block with voltages vs[3].  Outputs: Ydd [n*n], c [n] =
 * Y_ds v_s (the product of the n x 3 slack block and vs), Z [n*n] = -Y_dd^-1, w [n] =
 * Z c, with n = 3 (n_bus - 1) demand nodes in ascending node order. */
int oracle_build_3ph(int n_bus, int n_branch, const int32_t *frm, const int32_t *to,
                     const double complex *zabc, int slack, const double complex *vs,
                     double complex *Ydd, double complex *c, double complex *Z, double complex *w)
{
    if (n_bus < 2 || n_branch < 1 || slack < 0 || slack >= n_bus)
        return OR_ERR_INVALID;
    const int N = 3 * n_bus, n = 3 * (n_bus - 1);
    double complex *Y = calloc((size_t)N * N, sizeof(double complex));
    double complex *work = malloc(sizeof(double complex) * (size_t)n * 2 * n + 64);
    double complex *Yinv = malloc(sizeof(double complex) * (size_t)n * n);
    int *dn = malloc(sizeof(int) * n);
    if (!Y || !work || !Yinv || !dn) {
        free(Y); free(work); free(Yinv); free(dn);
        return OR_ERR_OOM;
    }
    int rc = OR_OK;
    for (int k = 0; k < n_branch; ++k) {
        int f = frm[k], t = to[k];
        if (f < 0 || f >= n_bus || t < 0 || t >= n_bus || f == t) { rc = OR_ERR_INVALID; goto done; }
        double complex yb[9];
        if (gj_inverse(zabc + 9 * (size_t)k, 3, yb, work) != OR_OK) { rc = OR_ERR_INVALID; goto done; }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                Y[(size_t)(3 * f + i) * N + 3 * f + j] += yb[3 * i + j];
                Y[(size_t)(3 * t + i) * N + 3 * t + j] += yb[3 * i + j];
                Y[(size_t)(3 * f + i) * N + 3 * t + j] -= yb[3 * i + j];
                Y[(size_t)(3 * t + i) * N + 3 * f + j] -= yb[3 * i + j];
            }
    }
    for (int b = 0, i = 0; b < n_bus; ++b)
        if (b != slack)
            for (int p = 0; p < 3; ++p) dn[i++] = 3 * b + p;
    for (int i = 0; i < n; ++i) {
        c[i] = 0.0;
        for (int p = 0; p < 3; ++p) c[i] += Y[(size_t)dn[i] * N + 3 * slack + p] * vs[p];
        for (int j = 0; j < n; ++j) Ydd[(size_t)i * n + j] = Y[(size_t)dn[i] * N + dn[j]];
    }
    if (gj_inverse(Ydd, n, Yinv, work) != OR_OK) { rc = OR_ERR_SINGULAR; goto done; }
    for (size_t e = 0; e < (size_t)n * n; ++e) Z[e] = -Yinv[e];
    for (int i = 0; i < n; ++i) {
        double complex acc = 0.0;
        for (int j = 0; j < n; ++j) acc += Z[(size_t)i * n + j] * c[j];
        w[i] = acc;
    }
done:
    free(Y); free(work); free(Yinv); free(dn);
    return rc;
}

/* Algorithm 1, one column at a time (the reshape to tau columns changes no
 * iterate, Sec. IV-A).  S, V0, V: [tau][n] interleaved complex; V0 may be NULL
 * (flat start 1 + j0).  Per column: iters (sweeps done), status, and the last
 * step size d (INFINITY when no sweep ran). */
void oracle_fpi(int n, const double complex *Z, const double complex *w, int64_t tau,
                const double complex *S, double tol, int max_iter,
                const double complex *V0, double complex *V, int32_t *iters,
                int8_t *status, double *dlast)
{
#pragma omp parallel
    {
        double complex *cur = malloc(sizeof(double complex) * n);
        double complex *nxt = malloc(sizeof(double complex) * n);
        double complex *cinj = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < tau; ++col) {
            const double complex *s = S + col * n;
            for (int i = 0; i < n; ++i) cur[i] = V0 ? V0[col * n + i] : 1.0;
            double d = INFINITY;
            int k = 0, bad = 0;
            while (d >= tol && k < max_iter) {
                /* current injection conj(S ./ V) */
                for (int i = 0; i < n; ++i) cinj[i] = conj(s[i] / cur[i]);
                /* V' = Z I + w */
                for (int i = 0; i < n; ++i) {
                    double complex acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += Z[(size_t)i * n + j] * cinj[j];
                    nxt[i] = acc + w[i];
                }
                d = 0.0;
                for (int i = 0; i < n; ++i) {
                    if (!isfinite(creal(nxt[i])) || !isfinite(cimag(nxt[i]))) bad = 1;
                    double e = cabs(nxt[i] - cur[i]);
                    if (e > d) d = e;
                }
                memcpy(cur, nxt, sizeof(double complex) * n);
                ++k;
                if (bad) break;
            }
            memcpy(V + col * n, cur, sizeof(double complex) * n);
            iters[col] = k;
            status[col] = bad ? ST_NONFINITE : (d < tol ? ST_CONVERGED : ST_MAX_ITER);
            if (dlast) dlast[col] = bad ? NAN : d;
        }
        free(cur); free(nxt); free(cinj);
    }
}

/* Power-balance mismatch from Eq. (1): with -i_d = Y_ds v_s + Y_dd v, the power a
 * load draws is v .* conj(i_d), so m = S + V .* conj(Y_ds v_s + Y_dd V).  Writes
 * max_i |m_i| per column. */
void oracle_mismatch(int n, const double complex *Ydd, const double complex *Yds,
                     double vs_re, double vs_im, int64_t tau, const double complex *S,
                     const double complex *V, double *mmax)
{
    double complex vs = vs_re + I * vs_im;
#pragma omp parallel for schedule(static)
    for (int64_t col = 0; col < tau; ++col) {
        const double complex *v = V + col * n;
        double worst = 0.0;
        for (int i = 0; i < n; ++i) {
            double complex acc = Yds[i] * vs;
            for (int j = 0; j < n; ++j) acc += Ydd[(size_t)i * n + j] * v[j];
            double complex m = S[col * n + i] + v[i] * conj(acc);
            double a = cabs(m);
            if (!(a <= worst)) worst = a; /* NaN propagates */
        }
        mmax[col] = worst;
    }
}

/* Eq. (2) for ZIP loads with alpha_Z = 0, one column at a time.  Z = -Y_dd^-1 is
 * -B^-1 (B = Y_dd when alpha_Z = 0); each column forms its own F = Z diag(alpha_P .* s*)
 * and w = Z (Y_ds v_s + alpha_I .* s*) and iterates v <- F conj(v)^-1 + w with the same
 * start, stopping rule and outputs as oracle_fpi.  alpha_i, alpha_p: [n] per PQ bus. */
void oracle_fpi_zip(int n, const double complex *Z, const double complex *Yds, double vs_re,
                    double vs_im, const double *alpha_i, const double *alpha_p, int64_t tau,
                    const double complex *S, double tol, int max_iter,
                    const double complex *V0, double complex *V, int32_t *iters,
                    int8_t *status, double *dlast)
{
    double complex vs = vs_re + I * vs_im;
#pragma omp parallel
    {
        double complex *F = malloc(sizeof(double complex) * (size_t)n * n);
        double complex *wc = malloc(sizeof(double complex) * n);
        double complex *cc = malloc(sizeof(double complex) * n);
        double complex *cur = malloc(sizeof(double complex) * n);
        double complex *nxt = malloc(sizeof(double complex) * n);
        double complex *rec = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < tau; ++col) {
            const double complex *s = S + col * n;
            /* F = -B^-1 A = Z diag(alpha_P .* s*) */
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    F[(size_t)i * n + j] = Z[(size_t)i * n + j] * (alpha_p[j] * conj(s[j]));
            /* c = Y_ds v_s + alpha_I .* s*,  w = -B^-1 c = Z c */
            for (int i = 0; i < n; ++i) cc[i] = Yds[i] * vs + alpha_i[i] * conj(s[i]);
            for (int i = 0; i < n; ++i) {
                double complex acc = 0.0;
                for (int j = 0; j < n; ++j) acc += Z[(size_t)i * n + j] * cc[j];
                wc[i] = acc;
            }
            for (int i = 0; i < n; ++i) cur[i] = V0 ? V0[col * n + i] : 1.0;
            double d = INFINITY;
            int k = 0, bad = 0;
            while (d >= tol && k < max_iter) {
                /* conj(v)^-1, element-wise */
                for (int i = 0; i < n; ++i) rec[i] = 1.0 / conj(cur[i]);
                /* v' = F conj(v)^-1 + w */
                for (int i = 0; i < n; ++i) {
                    double complex acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += F[(size_t)i * n + j] * rec[j];
                    nxt[i] = acc + wc[i];
                }
                d = 0.0;
                for (int i = 0; i < n; ++i) {
                    if (!isfinite(creal(nxt[i])) || !isfinite(cimag(nxt[i]))) bad = 1;
                    double e = cabs(nxt[i] - cur[i]);
                    if (e > d) d = e;
                }
                memcpy(cur, nxt, sizeof(double complex) * n);
                ++k;
                if (bad) break;
            }
            memcpy(V + col * n, cur, sizeof(double complex) * n);
            iters[col] = k;
            status[col] = bad ? ST_NONFINITE : (d < tol ? ST_CONVERGED : ST_MAX_ITER);
            if (dlast) dlast[col] = bad ? NAN : d;
        }
        free(F); free(wc); free(cc); free(cur); free(nxt); free(rec);
    }
}

/* Eq. (2) with alpha_Z != 0.  Per column: A = diag(alpha_P .* s*),
 * B = diag(alpha_Z .* s*) + Y_dd, c = Y_ds v_s + alpha_I .* s*, and
 * [F | w] = -B^-1 [A | c] from Gauss-Jordan elimination with partial pivoting on the
 * n x (n + 1 + n) array [B | c | A]; then the same iteration as oracle_fpi_zip.
 * A column whose B is numerically singular ends NONFINITE after 0 sweeps. */
void oracle_fpi_zipz(int n, const double complex *Ydd, const double complex *Yds, double vs_re,
                     double vs_im, const double *alpha_z, const double *alpha_i,
                     const double *alpha_p, int64_t tau, const double complex *S, double tol,
                     int max_iter, const double complex *V0, double complex *V, int32_t *iters,
                     int8_t *status, double *dlast)
{
    double complex vs = vs_re + I * vs_im;
    const int W = 2 * n + 1; /* columns of the augmented array */
#pragma omp parallel
    {
        double complex *M = malloc(sizeof(double complex) * (size_t)n * W);
        double complex *cur = malloc(sizeof(double complex) * n);
        double complex *nxt = malloc(sizeof(double complex) * n);
        double complex *rec = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < tau; ++col) {
            const double complex *s = S + col * n;
            /* [B | c | A] */
            double scale = 0.0;
            for (int i = 0; i < n; ++i) {
                double complex *row = M + (size_t)i * W;
                for (int j = 0; j < n; ++j) row[j] = Ydd[(size_t)i * n + j];
                row[i] += alpha_z[i] * conj(s[i]);
                row[n] = Yds[i] * vs + alpha_i[i] * conj(s[i]);
                for (int j = 0; j < n; ++j) row[n + 1 + j] = (i == j) ? alpha_p[i] * conj(s[i]) : 0.0;
                for (int j = 0; j < n; ++j) scale = fmax(scale, cabs(row[j]));
            }
            int singular = 0;
            for (int c = 0; c < n && !singular; ++c) {
                int p = c;
                double best = cabs(M[(size_t)c * W + c]);
                for (int i = c + 1; i < n; ++i) {
                    double v = cabs(M[(size_t)i * W + c]);
                    if (v > best) { best = v; p = i; }
                }
                if (!(best > 1e-13 * scale)) { singular = 1; break; }
                if (p != c)
                    for (int j = 0; j < W; ++j) {
                        double complex tmp = M[(size_t)c * W + j];
                        M[(size_t)c * W + j] = M[(size_t)p * W + j];
                        M[(size_t)p * W + j] = tmp;
                    }
                double complex piv = M[(size_t)c * W + c];
                for (int j = 0; j < W; ++j) M[(size_t)c * W + j] /= piv;
                for (int i = 0; i < n; ++i) {
                    if (i == c) continue;
                    double complex f = M[(size_t)i * W + c];
                    if (f == 0.0) continue;
                    for (int j = 0; j < W; ++j) M[(size_t)i * W + j] -= f * M[(size_t)c * W + j];
                }
            }
            if (singular) {
                for (int i = 0; i < n; ++i) V[col * n + i] = NAN;
                iters[col] = 0;
                status[col] = ST_NONFINITE;
                if (dlast) dlast[col] = NAN;
                continue;
            }
            /* now M = [1 | B^-1 c | B^-1 A]: w_i = -M[i][n], F_ij = -M[i][n + 1 + j] */
            for (int i = 0; i < n; ++i) cur[i] = V0 ? V0[col * n + i] : 1.0;
            double d = INFINITY;
            int k = 0, bad = 0;
            while (d >= tol && k < max_iter) {
                for (int i = 0; i < n; ++i) rec[i] = 1.0 / conj(cur[i]);
                for (int i = 0; i < n; ++i) {
                    double complex acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += -M[(size_t)i * W + n + 1 + j] * rec[j];
                    nxt[i] = acc - M[(size_t)i * W + n];
                }
                d = 0.0;
                for (int i = 0; i < n; ++i) {
                    if (!isfinite(creal(nxt[i])) || !isfinite(cimag(nxt[i]))) bad = 1;
                    double e = cabs(nxt[i] - cur[i]);
                    if (e > d) d = e;
                }
                memcpy(cur, nxt, sizeof(double complex) * n);
                ++k;
                if (bad) break;
            }
            memcpy(V + col * n, cur, sizeof(double complex) * n);
            iters[col] = k;
            status[col] = bad ? ST_NONFINITE : (d < tol ? ST_CONVERGED : ST_MAX_ITER);
            if (dlast) dlast[col] = bad ? NAN : d;
        }
        free(M); free(cur); free(nxt); free(rec);
    }
}

/* Power balance of ZIP loads: m = S .* (alpha_P + alpha_I .* V + alpha_Z .* |V|^2)
 * + V .* conj(Y_ds v_s + Y_dd V); max_i |m_i| per column.  alpha_z may be NULL (zero). */
void oracle_mismatch_zip(int n, const double complex *Ydd, const double complex *Yds,
                         double vs_re, double vs_im, const double *alpha_z, const double *alpha_i,
                         const double *alpha_p, int64_t tau, const double complex *S,
                         const double complex *V, double *mmax)
{
    double complex vs = vs_re + I * vs_im;
#pragma omp parallel for schedule(static)
    for (int64_t col = 0; col < tau; ++col) {
        const double complex *v = V + col * n;
        double worst = 0.0;
        for (int i = 0; i < n; ++i) {
            double complex acc = Yds[i] * vs;
            for (int j = 0; j < n; ++j) acc += Ydd[(size_t)i * n + j] * v[j];
            double az = alpha_z ? alpha_z[i] : 0.0;
            double v2 = creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
            double complex load = S[col * n + i] * (alpha_p[i] + alpha_i[i] * v[i] + az * v2);
            double complex m = load + v[i] * conj(acc);
            double a = cabs(m);
            if (!(a <= worst)) worst = a; /* NaN propagates */
        }
        mmax[col] = worst;
    }
}

int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

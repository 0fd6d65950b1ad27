/*
 * oracle.c -- plain, slow FP64 reference of the algebraic-distance setup path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * library; the two are tied together only by the published definitions they
 * both implement and by the seeded inputs the tests feed them.
 *
 * Every routine is the paper's definition written out in FP64 with plain
 * loops, in the order the definition states it.  Paper references are to
 * Brandt, Brannick, Kahl, Livshits, "An algebraic distances measure of AMG
 * strength of connection" (arXiv:1106.5990).
 *
 * Conventions shared with the caller (Python wrapper in __init__.py):
 *   CSR: rp[n+1], ci[nnz] (sorted per row, diagonal present), a[nnz] FP64.
 *   Panels: row-major n x K, entry (i, k) at X[i*K + k].
 *   Weights w[K] (NULL means all ones).
 *   A row subset `rows` (NULL = every row) selects which rows are computed;
 *   per-row outputs are then packed in the order of `rows`.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TARGET_PLAIN 0
#define TARGET_RESIDUAL 1

/* ---------------------------------------------------------------------- */
/* Test-vector start: splitmix64 (Steele, Lea and Flood, OOPSLA 2014).     */
/* The generator's state advances by the golden-ratio increment; each      */
/* output is the state pushed through its xor-shift-multiply finaliser.    */
/* Entry (r, k) of the start panel is the (r*K + k + 1)-th output of the   */
/* generator seeded with `seed`; its top 53 bits give u in [0, 1) and the  */
/* entry is 2u - 1, uniform on [-1, 1).                                    */
/* ---------------------------------------------------------------------- */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9e3779b97f4a7c15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64_nth(uint64_t seed, uint64_t n_outputs)
{
    /* the n-th output (n >= 1) of the generator seeded with `seed` */
    uint64_t s = seed, z = 0, m;
    for (m = 0; m < n_outputs; ++m) z = splitmix64_next(&s);
    return z;
}

void oracle_tv_init(int64_t row0, int64_t nrows, int K, uint64_t seed, double *X)
{
    int64_t r;
    int k;
    for (r = 0; r < nrows; ++r)
        for (k = 0; k < K; ++k) {
            /* jump the state straight to just before output number c + 1 */
            uint64_t c = (uint64_t)(row0 + r) * (uint64_t)K + (uint64_t)k;
            uint64_t s = seed + c * 0x9e3779b97f4a7c15ULL;
            uint64_t z = splitmix64_next(&s);
            double u = (double)(z >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
            X[r * K + k] = 2.0 * u - 1.0;
        }
}

/* ---------------------------------------------------------------------- */
/* helpers                                                                 */
/* ---------------------------------------------------------------------- */
static double diag_of(const int *rp, const int *ci, const double *a, int i)
{
    int e;
    for (e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] == i) return a[e];
    return 0.0;
}

static double weight(const double *w, int k) { return w ? w[k] : 1.0; }

/* (A x)_i for every column k of the panel */
static void row_apply(const int *rp, const int *ci, const double *a, int K,
                      const double *X, int i, double *y)
{
    int e, k;
    for (k = 0; k < K; ++k) y[k] = 0.0;
    for (e = rp[i]; e < rp[i + 1]; ++e)
        for (k = 0; k < K; ++k) y[k] += a[e] * X[(int64_t)ci[e] * K + k];
}

/* ---------------------------------------------------------------------- */
/* Relaxation of the homogeneous system A x = 0 (Sec. 3: test vectors are  */
/* produced by relaxing Ax = 0 from distinct starts).                      */
/* ---------------------------------------------------------------------- */

/* Damped Jacobi, whole vector at once: x <- x - omega D^{-1} A x.
 * A row with a zero diagonal is left unchanged.  Returns the number of
 * zero-diagonal rows met (0 when all is well). */
int oracle_jacobi(int n, const int *rp, const int *ci, const double *a, int K,
                  double omega, int sweeps, double *X)
{
    double *nx = (double *)malloc(sizeof(double) * (size_t)n * K);
    double *y = (double *)malloc(sizeof(double) * K);
    int s, i, k, zero = 0;
    for (s = 0; s < sweeps; ++s) {
        for (i = 0; i < n; ++i) {
            double d = diag_of(rp, ci, a, i);
            if (d == 0.0) {
                for (k = 0; k < K; ++k) nx[(int64_t)i * K + k] = X[(int64_t)i * K + k];
                if (s == 0) ++zero;
                continue;
            }
            row_apply(rp, ci, a, K, X, i, y);
            for (k = 0; k < K; ++k)
                nx[(int64_t)i * K + k] = X[(int64_t)i * K + k] - omega * y[k] / d;
        }
        memcpy(X, nx, sizeof(double) * (size_t)n * K);
    }
    free(nx);
    free(y);
    return zero;
}

/* One Jacobi sweep evaluated only on `rows`: out (packed) = x - omega D^-1 A x. */
void oracle_jacobi_rows(int n, const int *rp, const int *ci, const double *a, int K,
                        double omega, const double *X, int nrows, const int *rows,
                        double *out)
{
    double *y = (double *)malloc(sizeof(double) * K);
    int r, k;
    (void)n;
    for (r = 0; r < nrows; ++r) {
        int i = rows[r];
        double d = diag_of(rp, ci, a, i);
        if (d == 0.0) {
            for (k = 0; k < K; ++k) out[(int64_t)r * K + k] = X[(int64_t)i * K + k];
            continue;
        }
        row_apply(rp, ci, a, K, X, i, y);
        for (k = 0; k < K; ++k)
            out[(int64_t)r * K + k] = X[(int64_t)i * K + k] - omega * y[k] / d;
    }
    free(y);
}

/* Colour-phase Gauss-Seidel (omega = 1).  Within one sweep the colours are
 * visited in the order 0, 1, ..., ncolors-1; a row of colour c is replaced by
 *     x_i - (A z)_i / a_ii,   z_j = new x_j if colour(j) < c, else old x_j,
 * i.e. neighbours already updated in this sweep are read new and every other
 * value (same colour, later colours, the row itself) is read as it was when
 * the sweep began.  For a valid colouring this is Gauss-Seidel in colour
 * order.  Rows whose colour is outside [0, ncolors) and rows with a zero
 * diagonal are held fixed.  Returns the number of such rows. */
int oracle_color_gs(int n, const int *rp, const int *ci, const double *a, int K,
                    const int *color, int ncolors, int sweeps, double *X)
{
    double *nx = (double *)malloc(sizeof(double) * (size_t)n * K);
    double *y = (double *)malloc(sizeof(double) * K);
    int s, c, i, e, k, held = 0;
    for (s = 0; s < sweeps; ++s) {
        for (i = 0; i < n; ++i)
            if (color[i] < 0 || color[i] >= ncolors || diag_of(rp, ci, a, i) == 0.0) {
                for (k = 0; k < K; ++k) nx[(int64_t)i * K + k] = X[(int64_t)i * K + k];
                if (s == 0) ++held;
            }
        for (c = 0; c < ncolors; ++c) {
            for (i = 0; i < n; ++i) {
                double d;
                if (color[i] != c) continue;
                d = diag_of(rp, ci, a, i);
                if (d == 0.0) continue;
                for (k = 0; k < K; ++k) y[k] = 0.0;
                for (e = rp[i]; e < rp[i + 1]; ++e) {
                    int j = ci[e];
                    const double *z = (color[j] >= 0 && color[j] < c) ? nx : X;
                    for (k = 0; k < K; ++k) y[k] += a[e] * z[(int64_t)j * K + k];
                }
                for (k = 0; k < K; ++k)
                    nx[(int64_t)i * K + k] = X[(int64_t)i * K + k] - y[k] / d;
            }
        }
        memcpy(X, nx, sizeof(double) * (size_t)n * K);
    }
    free(nx);
    free(y);
    return held;
}

/* The colour-phase rule evaluated on `rows` only, given the panel at the
 * start of a sweep (Xold) and at its end (Xnew): out (packed) is what the
 * sweep must produce for those rows. */
void oracle_color_gs_rows(int n, const int *rp, const int *ci, const double *a, int K,
                          const int *color, int ncolors, const double *Xold,
                          const double *Xnew, int nrows, const int *rows, double *out)
{
    int r, e, k;
    double *y = (double *)malloc(sizeof(double) * K);
    (void)n;
    for (r = 0; r < nrows; ++r) {
        int i = rows[r], c = color[i];
        double d = diag_of(rp, ci, a, i);
        if (c < 0 || c >= ncolors || d == 0.0) {
            for (k = 0; k < K; ++k) out[(int64_t)r * K + k] = Xold[(int64_t)i * K + k];
            continue;
        }
        for (k = 0; k < K; ++k) y[k] = 0.0;
        for (e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            const double *z = (color[j] >= 0 && color[j] < c) ? Xnew : Xold;
            for (k = 0; k < K; ++k) y[k] += a[e] * z[(int64_t)j * K + k];
        }
        for (k = 0; k < K; ++k)
            out[(int64_t)r * K + k] = Xold[(int64_t)i * K + k] - y[k] / d;
    }
    free(y);
}

/* ---------------------------------------------------------------------- */
/* Fit target of row i: v_i (plain LS functional, Sec. 3.1 eq:LSfuncrowi)  */
/* or v_i - r_i / a_ii with r = A v (residual form, Sec. 3.1 eq:modls and  */
/* Sec. 4.1 eq:measure).  Returns 1 if a residual target met a zero        */
/* diagonal (the plain value is used then), else 0.                        */
/* ---------------------------------------------------------------------- */
static int fit_target(const int *rp, const int *ci, const double *a, int K,
                      const double *X, int i, int target, double *t, double *scratch)
{
    int k;
    for (k = 0; k < K; ++k) t[k] = X[(int64_t)i * K + k];
    if (target == TARGET_RESIDUAL) {
        double d = diag_of(rp, ci, a, i);
        if (d == 0.0) return 1;
        row_apply(rp, ci, a, K, X, i, scratch);
        for (k = 0; k < K; ++k) t[k] = t[k] - scratch[k] / d;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Algebraic distance (Sec. 4.1, eq:measure).  For every stored entry      */
/* (i, j) of the selected rows, the one-point least-squares problem        */
/*     min_p  sum_k w_k (t_i^k - p x_j^k)^2                               */
/* is solved by its normal equation p = <t, x_j>_w / <x_j, x_j>_w (p = 0   */
/* when x_j vanishes), and mu_ij is the functional at that p, evaluated    */
/* as written.  The paper's strength is r_ij = 1 / mu_ij.                  */
/* mu (and p, if not NULL) are packed over the selected rows' entries.     */
/* Returns the number of residual targets that met a zero diagonal.        */
/* ---------------------------------------------------------------------- */
int oracle_algdist(int n, const int *rp, const int *ci, const double *a, int K,
                   const double *X, const double *w, int target, int nrows,
                   const int *rows, double *mu, double *p)
{
    double *t = (double *)malloc(sizeof(double) * K);
    double *sc = (double *)malloc(sizeof(double) * K);
    int64_t out = 0;
    int r, e, k, bad = 0;
    int cnt = rows ? nrows : n;
    for (r = 0; r < cnt; ++r) {
        int i = rows ? rows[r] : r;
        bad += fit_target(rp, ci, a, K, X, i, target, t, sc);
        for (e = rp[i]; e < rp[i + 1]; ++e, ++out) {
            const double *xj = X + (int64_t)ci[e] * K;
            double sab = 0.0, sbb = 0.0, pij, m = 0.0;
            for (k = 0; k < K; ++k) {
                sab += weight(w, k) * t[k] * xj[k];
                sbb += weight(w, k) * xj[k] * xj[k];
            }
            pij = (sbb > 0.0) ? sab / sbb : 0.0;
            for (k = 0; k < K; ++k) {
                double res = t[k] - pij * xj[k];
                m += weight(w, k) * res * res;
            }
            mu[out] = m;
            if (p) p[out] = pij;
        }
    }
    free(t);
    free(sc);
    return bad;
}

/* ---------------------------------------------------------------------- */
/* Strength graph (Sec. 4.2, eq:strength_graph): for i in F, the edge      */
/* (i, j), j in F, j != i, is strong iff r_ij > theta * max_k r_ik over    */
/* the row's F-neighbours k != i.  With r = 1/mu this is                   */
/*     m_i > theta * mu_ij,   m_i = min_k mu_ik,                           */
/* and when m_i = 0 (an infinite strength) exactly the zero-distance edges */
/* are strong.  fmask[i] != 0 marks F (NULL: every row is in F).  The      */
/* comparison is made in FP64.                                             */
/* ---------------------------------------------------------------------- */
void oracle_strength(int n, const int *rp, const int *ci, const double *mu, double theta,
                     const unsigned char *fmask, unsigned char *strong, int *nstrong)
{
    int i, e;
    for (i = 0; i < n; ++i) {
        double m = INFINITY;
        int cnt = 0;
        int in_f = fmask ? (fmask[i] != 0) : 1;
        for (e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (!in_f || j == i || (fmask && !fmask[j])) continue;
            if (mu[e] < m) m = mu[e];
        }
        for (e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e], s = 0;
            if (in_f && j != i && (!fmask || fmask[j])) {
                if (m > 0.0) s = (theta * mu[e] < m);
                else s = (mu[e] == 0.0);
            }
            strong[e] = (unsigned char)s;
            cnt += s;
        }
        if (nstrong) nstrong[i] = cnt;
    }
}

/* ---------------------------------------------------------------------- */
/* Least-squares interpolation (Sec. 3.1 eq:LSfuncrowi / eq:modls) on a    */
/* set C_i chosen by the one-sided distances (Sec. 4.3, final remark: a    */
/* systematic scan guided by the one-point measure): C_i is the caliber    */
/* C-neighbours j != i with the smallest mu_ij (ties: lower column).       */
/*                                                                         */
/* The weighted problem min_p sum_k w_k (t^k - sum_j p_j x_j^k)^2 is       */
/* solved by Householder QR of the sqrt(w)-scaled K x |C_i| matrix, the    */
/* columns taken in increasing-mu order.  A column whose part orthogonal   */
/* to the columns already kept has squared norm <= 1e-12 times its own     */
/* squared norm is dropped (status 2).  The uniqueness remark of Sec. 3.1  */
/* (K >= caliber and spanning vectors) is what makes the kept columns      */
/* well posed.  ls_val is the functional at the minimiser, evaluated by    */
/* its definition.                                                         */
/*                                                                         */
/* Output per row i (row-major n x caliber): P_col (fine column index,     */
/* -1 padded, in increasing-mu order), P_val, ls_val, status:              */
/*   0 ok, 1 F row without C-neighbour, 2 column(s) dropped, 3 residual    */
/*   target with zero diagonal.  A C row interpolates itself with weight 1.*/
/* ---------------------------------------------------------------------- */
#define ORACLE_MAX_CAL 16

static int is_candidate(const int *ci, const unsigned char *cf, const double *mu, int i, int e)
{
    int j = ci[e];
    return j != i && cf[j] && !isnan(mu[e]);
}

void oracle_ls_interp(int n, const int *rp, const int *ci, const double *a, int K,
                      const double *X, const double *w, const unsigned char *cf,
                      const double *mu, int caliber, int target, int nrows, const int *rows,
                      int *P_col, double *P_val, double *ls_val, int *status)
{
    int cnt = rows ? nrows : n;
    int r, k, s, e, jj;
    double *t = (double *)malloc(sizeof(double) * K);
    double *sc = (double *)malloc(sizeof(double) * K);
    double *M = (double *)malloc(sizeof(double) * K * ORACLE_MAX_CAL); /* column-major */
    double *b = (double *)malloc(sizeof(double) * K);
    double *v = (double *)malloc(sizeof(double) * K);
    (void)n;
    for (r = 0; r < cnt; ++r) {
        int i = rows ? rows[r] : r;
        int *pc = P_col + (int64_t)r * caliber;
        double *pv = P_val + (int64_t)r * caliber;
        int sel_e[ORACLE_MAX_CAL];
        int nsel = 0, st = 0, kept = 0;
        int kept_col[ORACLE_MAX_CAL];
        double R[ORACLE_MAX_CAL][ORACLE_MAX_CAL];
        double coef[ORACLE_MAX_CAL];
        double val;

        for (s = 0; s < caliber; ++s) { pc[s] = -1; pv[s] = 0.0; }
        if (cf[i]) { /* a C point interpolates itself */
            pc[0] = i;
            pv[0] = 1.0;
            ls_val[r] = 0.0;
            status[r] = 0;
            continue;
        }
        if (fit_target(rp, ci, a, K, X, i, target, t, sc)) st = 3;

        /* C_i: repeatedly take the unselected candidate of least (mu, column) */
        for (s = 0; s < caliber; ++s) {
            int best = -1;
            for (e = rp[i]; e < rp[i + 1]; ++e) {
                int taken = 0, q;
                if (!is_candidate(ci, cf, mu, i, e)) continue;
                for (q = 0; q < nsel; ++q) taken |= (sel_e[q] == e);
                if (taken) continue;
                if (best < 0 || mu[e] < mu[best] || (mu[e] == mu[best] && ci[e] < ci[best]))
                    best = e;
            }
            if (best < 0) break;
            sel_e[nsel++] = best;
        }
        if (nsel == 0) {
            double f = 0.0;
            for (k = 0; k < K; ++k) f += weight(w, k) * t[k] * t[k];
            ls_val[r] = f;
            status[r] = st ? st : 1;
            continue;
        }

        /* scaled system: column q is sqrt(w) .* x_{c_q}, right side sqrt(w) .* t */
        for (s = 0; s < nsel; ++s)
            for (k = 0; k < K; ++k)
                M[s * K + k] = sqrt(weight(w, k)) * X[(int64_t)ci[sel_e[s]] * K + k];
        for (k = 0; k < K; ++k) b[k] = sqrt(weight(w, k)) * t[k];

        /* Householder QR with the column-drop rule */
        for (s = 0; s < nsel; ++s) {
            double *col = M + s * K;
            double full = 0.0, tail = 0.0, alpha, vnorm2, dot;
            int q;
            for (k = 0; k < K; ++k) full += col[k] * col[k];
            for (k = kept; k < K; ++k) tail += col[k] * col[k];
            if (kept >= K || tail <= 1e-12 * full) { /* (numerically) dependent column */
                st = st ? st : 2;
                continue;
            }
            /* reflector H = I - 2 v v^T / (v^T v) mapping col[kept:] to alpha e_kept */
            alpha = (col[kept] > 0.0) ? -sqrt(tail) : sqrt(tail);
            for (k = 0; k < K; ++k) v[k] = 0.0;
            for (k = kept; k < K; ++k) v[k] = col[k];
            v[kept] -= alpha;
            vnorm2 = 0.0;
            for (k = kept; k < K; ++k) vnorm2 += v[k] * v[k];
            /* apply to this and every later column, and to b */
            for (q = s; q < nsel; ++q) {
                double *cq = M + q * K;
                dot = 0.0;
                for (k = kept; k < K; ++k) dot += v[k] * cq[k];
                for (k = kept; k < K; ++k) cq[k] -= 2.0 * dot / vnorm2 * v[k];
            }
            dot = 0.0;
            for (k = kept; k < K; ++k) dot += v[k] * b[k];
            for (k = kept; k < K; ++k) b[k] -= 2.0 * dot / vnorm2 * v[k];
            /* row `kept` of R holds this column's entries for the kept columns */
            for (q = 0; q <= kept; ++q) R[q][kept] = col[q];
            kept_col[kept] = s;
            ++kept;
            /* columns already dropped are never revisited; later columns now
               carry their rotated entries in M and are read when kept */
        }
        /* back substitution R coef = Q^T b (first `kept` entries of b) */
        for (jj = kept - 1; jj >= 0; --jj) {
            double acc = b[jj];
            int q;
            for (q = jj + 1; q < kept; ++q) acc -= R[jj][q] * coef[q];
            coef[jj] = acc / R[jj][jj];
        }
        /* LS functional at the minimiser, by its definition */
        val = 0.0;
        for (k = 0; k < K; ++k) {
            double res = t[k];
            for (s = 0; s < kept; ++s)
                res -= coef[s] * X[(int64_t)ci[sel_e[kept_col[s]]] * K + k];
            val += weight(w, k) * res * res;
        }
        for (s = 0; s < kept; ++s) {
            pc[s] = ci[sel_e[kept_col[s]]];
            pv[s] = coef[s];
        }
        ls_val[r] = val;
        status[r] = st;
    }
    free(t);
    free(sc);
    free(M);
    free(b);
    free(v);
}

/* ---------------------------------------------------------------------- */
/* LS interpolation loss and its gradient.                                 */
/*                                                                         */
/* x^0 = X0, x^{s+1} = x^s - omega D^{-1} A x^s (s < sweeps), and          */
/*     L = sum_{i in F} sum_k w_k (x_i^k - sum_j p_ij x_j^k)^2             */
/* with the plain target and p the LS rows fitted to x^sweeps (C_i chosen  */
/* by the distances of x^sweeps, as oracle_ls_interp does).  Because p     */
/* minimises each row's functional, dL/dx^S is the partial derivative at   */
/* fixed p; it is then carried back through the sweeps by the chain rule:  */
/*     y = D^{-1} g,  g <- g - omega A^T y,                                */
/*     dL/domega -= <y, A x^s>,                                            */
/*     dL/da_ij  -= omega <y_i, x_j^s>, and for j = i also                 */
/*     dL/da_ii  += omega <y_i, (A x^s)_i> / a_ii.                         */
/* Returns L.                                                              */
/* ---------------------------------------------------------------------- */
static void ls_rows_for(int n, const int *rp, const int *ci, const double *a, int K,
                        const double *X, const double *w, const unsigned char *cf, int caliber,
                        int *Pc, double *Pv, double *ls, int *st)
{
    int64_t nnz = rp[n];
    double *mu = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    oracle_algdist(n, rp, ci, a, K, X, w, TARGET_PLAIN, 0, NULL, mu, NULL);
    oracle_ls_interp(n, rp, ci, a, K, X, w, cf, mu, caliber, TARGET_PLAIN, 0, NULL, Pc, Pv, ls, st);
    free(mu);
}

double oracle_ls_loss(int n, const int *rp, const int *ci, const double *a, int K,
                      const double *X0, int sweeps, double omega, const double *w,
                      const unsigned char *cf, int caliber)
{
    size_t nk = (size_t)n * K;
    double *X = (double *)malloc(sizeof(double) * nk);
    int *Pc = (int *)malloc(sizeof(int) * (size_t)n * caliber);
    double *Pv = (double *)malloc(sizeof(double) * (size_t)n * caliber);
    double *ls = (double *)malloc(sizeof(double) * n);
    int *st = (int *)malloc(sizeof(int) * n);
    double L = 0.0;
    int i;
    memcpy(X, X0, sizeof(double) * nk);
    oracle_jacobi(n, rp, ci, a, K, omega, sweeps, X);
    ls_rows_for(n, rp, ci, a, K, X, w, cf, caliber, Pc, Pv, ls, st);
    for (i = 0; i < n; ++i)
        if (!cf[i]) L += ls[i];
    free(X); free(Pc); free(Pv); free(ls); free(st);
    return L;
}

double oracle_ls_loss_grad(int n, const int *rp, const int *ci, const double *a, int K,
                           const double *X0, int sweeps, double omega, const double *w,
                           const unsigned char *cf, int caliber, double *grad_val,
                           double *grad_omega)
{
    size_t nk = (size_t)n * K;
    int64_t nnz = rp[n];
    double **it = (double **)malloc(sizeof(double *) * (sweeps + 1));
    double *g = (double *)malloc(sizeof(double) * nk);
    double *gn = (double *)malloc(sizeof(double) * nk);
    double *yv = (double *)malloc(sizeof(double) * nk);
    double *z = (double *)malloc(sizeof(double) * K);
    int *Pc = (int *)malloc(sizeof(int) * (size_t)n * caliber);
    double *Pv = (double *)malloc(sizeof(double) * (size_t)n * caliber);
    double *ls = (double *)malloc(sizeof(double) * n);
    int *st = (int *)malloc(sizeof(int) * n);
    double L = 0.0, gw = 0.0;
    int s, i, k, e, q;
    int64_t ee;

    /* forward, keeping every iterate */
    for (s = 0; s <= sweeps; ++s) it[s] = (double *)malloc(sizeof(double) * nk);
    memcpy(it[0], X0, sizeof(double) * nk);
    for (s = 0; s < sweeps; ++s) {
        memcpy(it[s + 1], it[s], sizeof(double) * nk);
        oracle_jacobi(n, rp, ci, a, K, omega, 1, it[s + 1]);
    }
    ls_rows_for(n, rp, ci, a, K, it[sweeps], w, cf, caliber, Pc, Pv, ls, st);

    /* dL/dx^S at fixed p */
    for (ee = 0; ee < (int64_t)nk; ++ee) g[ee] = 0.0;
    for (i = 0; i < n; ++i) {
        const double *x = it[sweeps];
        if (cf[i]) continue;
        L += ls[i];
        for (k = 0; k < K; ++k) {
            double res = x[(int64_t)i * K + k];
            for (q = 0; q < caliber; ++q)
                if (Pc[(int64_t)i * caliber + q] >= 0)
                    res -= Pv[(int64_t)i * caliber + q] * x[(int64_t)Pc[(int64_t)i * caliber + q] * K + k];
            g[(int64_t)i * K + k] += 2.0 * weight(w, k) * res;
            for (q = 0; q < caliber; ++q) {
                int j = Pc[(int64_t)i * caliber + q];
                if (j >= 0)
                    g[(int64_t)j * K + k] -= 2.0 * weight(w, k) * res * Pv[(int64_t)i * caliber + q];
            }
        }
    }

    for (e = 0; e < nnz; ++e) grad_val[e] = 0.0;
    /* backward through the sweeps */
    for (s = sweeps - 1; s >= 0; --s) {
        const double *x = it[s];
        for (i = 0; i < n; ++i) {
            double d = diag_of(rp, ci, a, i);
            for (k = 0; k < K; ++k) yv[(int64_t)i * K + k] = (d != 0.0) ? g[(int64_t)i * K + k] / d : 0.0;
        }
        memcpy(gn, g, sizeof(double) * nk);
        for (i = 0; i < n; ++i) {
            double d = diag_of(rp, ci, a, i);
            if (d == 0.0) continue;
            row_apply(rp, ci, a, K, x, i, z);
            for (k = 0; k < K; ++k) gw -= yv[(int64_t)i * K + k] * z[k];
            for (e = rp[i]; e < rp[i + 1]; ++e) {
                int j = ci[e];
                double acc = 0.0;
                for (k = 0; k < K; ++k) acc += yv[(int64_t)i * K + k] * x[(int64_t)j * K + k];
                grad_val[e] -= omega * acc;
                if (j == i) {
                    double acc2 = 0.0;
                    for (k = 0; k < K; ++k) acc2 += yv[(int64_t)i * K + k] * z[k];
                    grad_val[e] += omega * acc2 / d;
                }
                /* (A^T y)_j gets a_ij y_i */
                for (k = 0; k < K; ++k) gn[(int64_t)j * K + k] -= omega * a[e] * yv[(int64_t)i * K + k];
            }
        }
        memcpy(g, gn, sizeof(double) * nk);
    }
    *grad_omega = gw;

    for (s = 0; s <= sweeps; ++s) free(it[s]);
    free(it); free(g); free(gn); free(yv); free(z);
    free(Pc); free(Pv); free(ls); free(st);
    return L;
}

/* ---------------------------------------------------------------------- */
/* The same loss with the test vectors relaxed by colour-phase Gauss-      */
/* Seidel (Sec. 3 test vectors, relaxed by Gauss-Seidel as in Sec. 5.2),   */
/* and its gradient with respect to the stored values of A and to the LS   */
/* weights w_k (eq:LSfuncrowi).                                            */
/*                                                                         */
/* One colour phase of oracle_color_gs is the linear map                   */
/*     v' = v - E_c D^{-1} A v,                                            */
/* E_c selecting the rows of colour c (rows with an invalid colour or a    */
/* zero diagonal are never selected): every value a phase reads is the     */
/* state before it.  Its adjoint is g = g' - A^T y with y = D^{-1} E_c g', */
/* and the phase contributes -y_i v_j to dL/da_ij (i of colour c) and      */
/* y_i (A v)_i / a_ii to dL/da_ii through D^{-1}.  A sweep's adjoint runs  */
/* its phases in reverse colour order.                                     */
/*                                                                         */
/* w_k enters L directly and through the fitted p; p minimises each row's  */
/* functional, so dL/dw_k = sum over F rows of (x_i^k - sum_j p_ij x_j^k)^2 */
/* at the final panel.                                                     */
/* ---------------------------------------------------------------------- */
static void gs_phase(int n, const int *rp, const int *ci, const double *a, int K,
                     const int *color, int ncolors, int c, const double *v, double *out)
{
    int i, e, k;
    memcpy(out, v, sizeof(double) * (size_t)n * K);
    for (i = 0; i < n; ++i) {
        double d;
        if (color[i] != c || c < 0 || c >= ncolors) continue;
        d = diag_of(rp, ci, a, i);
        if (d == 0.0) continue;
        for (k = 0; k < K; ++k) {
            double y = 0.0;
            for (e = rp[i]; e < rp[i + 1]; ++e) y += a[e] * v[(int64_t)ci[e] * K + k];
            out[(int64_t)i * K + k] = v[(int64_t)i * K + k] - y / d;
        }
    }
}

double oracle_ls_loss_gs(int n, const int *rp, const int *ci, const double *a, int K,
                         const double *X0, int sweeps, const int *color, int ncolors,
                         const double *w, const unsigned char *cf, int caliber)
{
    size_t nk = (size_t)n * K;
    double *X = (double *)malloc(sizeof(double) * nk);
    int *Pc = (int *)malloc(sizeof(int) * (size_t)n * caliber);
    double *Pv = (double *)malloc(sizeof(double) * (size_t)n * caliber);
    double *ls = (double *)malloc(sizeof(double) * n);
    int *st = (int *)malloc(sizeof(int) * n);
    double L = 0.0;
    int i;
    memcpy(X, X0, sizeof(double) * nk);
    oracle_color_gs(n, rp, ci, a, K, color, ncolors, sweeps, X);
    ls_rows_for(n, rp, ci, a, K, X, w, cf, caliber, Pc, Pv, ls, st);
    for (i = 0; i < n; ++i)
        if (!cf[i]) L += ls[i];
    free(X); free(Pc); free(Pv); free(ls); free(st);
    return L;
}

/* dL/dw_k at the final panel X (p refitted there). */
void oracle_ls_grad_w(int n, const int *rp, const int *ci, const double *a, int K,
                      const double *X, const double *w, const unsigned char *cf, int caliber,
                      double *grad_w)
{
    int *Pc = (int *)malloc(sizeof(int) * (size_t)n * caliber);
    double *Pv = (double *)malloc(sizeof(double) * (size_t)n * caliber);
    double *ls = (double *)malloc(sizeof(double) * n);
    int *st = (int *)malloc(sizeof(int) * n);
    int i, k, q;
    ls_rows_for(n, rp, ci, a, K, X, w, cf, caliber, Pc, Pv, ls, st);
    for (k = 0; k < K; ++k) grad_w[k] = 0.0;
    for (i = 0; i < n; ++i) {
        if (cf[i]) continue;
        for (k = 0; k < K; ++k) {
            double res = X[(int64_t)i * K + k];
            for (q = 0; q < caliber; ++q) {
                int j = Pc[(int64_t)i * caliber + q];
                if (j >= 0) res -= Pv[(int64_t)i * caliber + q] * X[(int64_t)j * K + k];
            }
            grad_w[k] += res * res;
        }
    }
    free(Pc); free(Pv); free(ls); free(st);
}

double oracle_ls_loss_grad_gs(int n, const int *rp, const int *ci, const double *a, int K,
                              const double *X0, int sweeps, const int *color, int ncolors,
                              const double *w, const unsigned char *cf, int caliber,
                              double *grad_val, double *grad_w)
{
    size_t nk = (size_t)n * K;
    int64_t nnz = rp[n];
    int nst = sweeps * ncolors + 1;   /* the state before every phase, and the last */
    double **v = (double **)malloc(sizeof(double *) * (size_t)nst);
    double *g = (double *)malloc(sizeof(double) * nk);
    double *gn = (double *)malloc(sizeof(double) * nk);
    double *yv = (double *)malloc(sizeof(double) * nk);
    double *z = (double *)malloc(sizeof(double) * K);
    int *Pc = (int *)malloc(sizeof(int) * (size_t)n * caliber);
    double *Pv = (double *)malloc(sizeof(double) * (size_t)n * caliber);
    double *ls = (double *)malloc(sizeof(double) * n);
    int *st = (int *)malloc(sizeof(int) * n);
    double L = 0.0;
    int s, c, i, k, e, q, t;
    int64_t ee;

    for (t = 0; t < nst; ++t) v[t] = (double *)malloc(sizeof(double) * nk);
    memcpy(v[0], X0, sizeof(double) * nk);
    for (s = 0; s < sweeps; ++s)
        for (c = 0; c < ncolors; ++c) {
            t = s * ncolors + c;
            gs_phase(n, rp, ci, a, K, color, ncolors, c, v[t], v[t + 1]);
        }
    {
        const double *x = v[nst - 1];
        ls_rows_for(n, rp, ci, a, K, x, w, cf, caliber, Pc, Pv, ls, st);
        for (ee = 0; ee < (int64_t)nk; ++ee) g[ee] = 0.0;
        for (k = 0; k < K; ++k) grad_w[k] = 0.0;
        for (i = 0; i < n; ++i) {
            if (cf[i]) continue;
            L += ls[i];
            for (k = 0; k < K; ++k) {
                double res = x[(int64_t)i * K + k];
                for (q = 0; q < caliber; ++q)
                    if (Pc[(int64_t)i * caliber + q] >= 0)
                        res -= Pv[(int64_t)i * caliber + q] * x[(int64_t)Pc[(int64_t)i * caliber + q] * K + k];
                grad_w[k] += res * res;
                g[(int64_t)i * K + k] += 2.0 * weight(w, k) * res;
                for (q = 0; q < caliber; ++q) {
                    int j = Pc[(int64_t)i * caliber + q];
                    if (j >= 0)
                        g[(int64_t)j * K + k] -= 2.0 * weight(w, k) * res * Pv[(int64_t)i * caliber + q];
                }
            }
        }
    }
    for (e = 0; e < nnz; ++e) grad_val[e] = 0.0;
    for (t = nst - 2; t >= 0; --t) {
        const double *x = v[t];      /* state before the phase */
        c = t % ncolors;
        for (i = 0; i < n; ++i) {
            double d = diag_of(rp, ci, a, i);
            int on = color[i] == c && d != 0.0;
            for (k = 0; k < K; ++k) yv[(int64_t)i * K + k] = on ? g[(int64_t)i * K + k] / d : 0.0;
        }
        memcpy(gn, g, sizeof(double) * nk);
        for (i = 0; i < n; ++i) {
            double d = diag_of(rp, ci, a, i);
            if (color[i] != c || d == 0.0) continue;
            row_apply(rp, ci, a, K, x, i, z);
            for (e = rp[i]; e < rp[i + 1]; ++e) {
                int j = ci[e];
                double acc = 0.0;
                for (k = 0; k < K; ++k) acc += yv[(int64_t)i * K + k] * x[(int64_t)j * K + k];
                grad_val[e] -= acc;
                if (j == i) {
                    double acc2 = 0.0;
                    for (k = 0; k < K; ++k) acc2 += yv[(int64_t)i * K + k] * z[k];
                    grad_val[e] += acc2 / d;
                }
                for (k = 0; k < K; ++k) gn[(int64_t)j * K + k] -= a[e] * yv[(int64_t)i * K + k];
            }
        }
        memcpy(g, gn, sizeof(double) * nk);
    }

    for (t = 0; t < nst; ++t) free(v[t]);
    free(v); free(g); free(gn); free(yv); free(z);
    free(Pc); free(Pv); free(ls); free(st);
    return L;
}

/* ====================================================================== */
/* Long-range connectivity and the search over interpolatory sets          */
/* ====================================================================== */

/* ---------------------------------------------------------------------- */
/* Pattern of A^d (Sec. 4.1, eq. graph).  Read structurally: j is in row i */
/* of A^d iff a walk of exactly d steps joins i to j in the graph of A;    */
/* with every diagonal stored this is every j within graph distance d of   */
/* i.  A^d itself is never formed (the remark closing Sec. 4.2): the rows  */
/* come from a breadth-first search of depth d over the graph of A.        */
/* ---------------------------------------------------------------------- */

/* Vertices within distance d of i, unsorted, into list; returns the count.
 * mark[] must hold values != i on entry for every vertex. */
static int reach(const int *rp, const int *ci, int d, int i, int *mark, int *list)
{
    int head = 0, tail = 0, lev, e;
    list[tail++] = i;
    mark[i] = i;
    for (lev = 0; lev < d; ++lev) {
        int end = tail;
        for (; head < end; ++head) {
            int u = list[head];
            for (e = rp[u]; e < rp[u + 1]; ++e) {
                int j = ci[e];
                if (mark[j] != i) {
                    mark[j] = i;
                    list[tail++] = j;
                }
            }
        }
    }
    return tail;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* cnt[i] = number of entries of row i of A^d.  Returns their sum. */
int64_t oracle_power_counts(int n, const int *rp, const int *ci, int d, int *cnt)
{
    int *mark = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *list = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int64_t total = 0;
    int i;
    for (i = 0; i < n; ++i) mark[i] = -1;
    for (i = 0; i < n; ++i) {
        cnt[i] = reach(rp, ci, d, i, mark, list);
        total += cnt[i];
    }
    free(mark);
    free(list);
    return total;
}

/* Columns of A^d, sorted per row, at the row pointers rpd (from the counts). */
void oracle_power_fill(int n, const int *rp, const int *ci, int d, const int *rpd, int *cid)
{
    int *mark = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *list = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int i, m;
    for (i = 0; i < n; ++i) mark[i] = -1;
    for (i = 0; i < n; ++i) {
        m = reach(rp, ci, d, i, mark, list);
        qsort(list, (size_t)m, sizeof(int), cmp_int);
        memcpy(cid + rpd[i], list, sizeof(int) * (size_t)m);
    }
    free(mark);
    free(list);
}

/* ---------------------------------------------------------------------- */
/* Algebraic distance on a graph G other than that of A (Sec. 4.1,         */
/* eq:measure with j ranging over V_i of eq. graph, e.g. G = A^d): for     */
/* every entry (i, j) of G the one-point problem of oracle_algdist, the    */
/* target of row i formed from A (plain, or with A's residual).  mu (and   */
/* p) per entry of G, packed over the selected rows.                       */
/* ---------------------------------------------------------------------- */
int oracle_algdist_graph(int n, const int *rp, const int *ci, const double *a, const int *rpg,
                         const int *cig, int K, const double *X, const double *w, int target,
                         int nrows, const int *rows, double *mu, double *p)
{
    double *t = (double *)malloc(sizeof(double) * K);
    double *sc = (double *)malloc(sizeof(double) * K);
    int64_t out = 0;
    int r, e, k, bad = 0;
    int cnt = rows ? nrows : n;
    for (r = 0; r < cnt; ++r) {
        int i = rows ? rows[r] : r;
        bad += fit_target(rp, ci, a, K, X, i, target, t, sc);
        for (e = rpg[i]; e < rpg[i + 1]; ++e, ++out) {
            const double *xj = X + (int64_t)cig[e] * K;
            double sab = 0.0, sbb = 0.0, pij, m = 0.0;
            for (k = 0; k < K; ++k) {
                sab += weight(w, k) * t[k] * xj[k];
                sbb += weight(w, k) * xj[k] * xj[k];
            }
            pij = (sbb > 0.0) ? sab / sbb : 0.0;
            for (k = 0; k < K; ++k) {
                double res = t[k] - pij * xj[k];
                m += weight(w, k) * res * res;
            }
            mu[out] = m;
            if (p) p[out] = pij;
        }
    }
    free(t);
    free(sc);
    return bad;
}

/* ---------------------------------------------------------------------- */
/* Least-squares fit of target t by the panel rows cols[0..m) (Sec. 3.1,   */
/* eq:LSfuncrowi / eq:modls for a given set W): Householder QR of the      */
/* sqrt(w)-scaled K x m system.  Returns 1 (and nothing else) when a       */
/* column is numerically dependent on the ones before it (the part of it   */
/* the earlier reflections leave, squared, <= 1e-8 of its squared norm,   */
/* i.e. a relative part below 1e-4: the reading of the basis condition of  */
/* the uniqueness remark in Sec. 3.1 for the search; a set closer to       */
/* dependence fits through cancelling weights, and its functional is not   */
/* resolvable from FP64 normal equations), else 0 with coef[0..m) the      */
/* minimiser and *val the functional at it, evaluated by its definition.   */
/* M: K*m scratch, b, v: K scratch.                                        */
/* ---------------------------------------------------------------------- */
static int qr_fit(int K, const double *X, const double *w, const double *t, const int *cols,
                  int m, double *coef, double *val, double *M, double *b, double *v)
{
    double R[ORACLE_MAX_CAL][ORACLE_MAX_CAL];
    int s, q, k;
    for (s = 0; s < m; ++s)
        for (k = 0; k < K; ++k) M[s * K + k] = sqrt(weight(w, k)) * X[(int64_t)cols[s] * K + k];
    for (k = 0; k < K; ++k) b[k] = sqrt(weight(w, k)) * t[k];
    for (s = 0; s < m; ++s) {
        double *col = M + s * K;
        double full = 0.0, tail = 0.0, alpha, vnorm2, dot;
        for (k = 0; k < K; ++k) full += col[k] * col[k];
        for (k = s; k < K; ++k) tail += col[k] * col[k];
        if (s >= K || tail <= 1e-8 * full) return 1;
        alpha = (col[s] > 0.0) ? -sqrt(tail) : sqrt(tail);
        for (k = 0; k < K; ++k) v[k] = 0.0;
        for (k = s; k < K; ++k) v[k] = col[k];
        v[s] -= alpha;
        vnorm2 = 0.0;
        for (k = s; k < K; ++k) vnorm2 += v[k] * v[k];
        for (q = s; q < m; ++q) {
            double *cq = M + q * K;
            dot = 0.0;
            for (k = s; k < K; ++k) dot += v[k] * cq[k];
            for (k = s; k < K; ++k) cq[k] -= 2.0 * dot / vnorm2 * v[k];
        }
        dot = 0.0;
        for (k = s; k < K; ++k) dot += v[k] * b[k];
        for (k = s; k < K; ++k) b[k] -= 2.0 * dot / vnorm2 * v[k];
        for (q = 0; q <= s; ++q) R[q][s] = col[q];
    }
    for (s = m - 1; s >= 0; --s) {
        double acc = b[s];
        for (q = s + 1; q < m; ++q) acc -= R[s][q] * coef[q];
        coef[s] = acc / R[s][s];
    }
    *val = 0.0;
    for (k = 0; k < K; ++k) {
        double res = t[k];
        for (s = 0; s < m; ++s) res -= coef[s] * X[(int64_t)cols[s] * K + k];
        *val += weight(w, k) * res * res;
    }
    return 0;
}

/* LS rows for given interpolatory sets: sets (row-major nrows x caliber,
 * -1 padded, the set of rows[r] in row r) are fitted by qr_fit; P_val and
 * ls_val receive the minimiser and the functional, rankdef[r] = 1 (and
 * zeros) for a numerically dependent set.  Target as in oracle_algdist. */
void oracle_ls_fit_sets(int n, const int *rp, const int *ci, const double *a, int K,
                        const double *X, const double *w, int target, int caliber, int nrows,
                        const int *rows, const int *sets, double *P_val, double *ls_val,
                        int *rankdef)
{
    double *t = (double *)malloc(sizeof(double) * K);
    double *sc = (double *)malloc(sizeof(double) * K);
    double *M = (double *)malloc(sizeof(double) * K * ORACLE_MAX_CAL);
    double *b = (double *)malloc(sizeof(double) * K);
    double *v = (double *)malloc(sizeof(double) * K);
    int r, s, k;
    (void)n;
    for (r = 0; r < nrows; ++r) {
        int i = rows[r], m = 0;
        const int *set = sets + (int64_t)r * caliber;
        double coef[ORACLE_MAX_CAL], val = 0.0;
        fit_target(rp, ci, a, K, X, i, target, t, sc);
        while (m < caliber && set[m] >= 0) ++m;
        for (s = 0; s < caliber; ++s) P_val[(int64_t)r * caliber + s] = 0.0;
        rankdef[r] = 0;
        if (m == 0) {
            for (k = 0; k < K; ++k) val += weight(w, k) * t[k] * t[k];
            ls_val[r] = val;
            continue;
        }
        if (qr_fit(K, X, w, t, set, m, coef, &val, M, b, v)) {
            rankdef[r] = 1;
            ls_val[r] = 0.0;
            continue;
        }
        for (s = 0; s < m; ++s) P_val[(int64_t)r * caliber + s] = coef[s];
        ls_val[r] = val;
    }
    free(t); free(sc); free(M); free(b); free(v);
}

/* ---------------------------------------------------------------------- */
/* Interpolatory sets by search (Sec. 4.3).  For an F row i the candidates */
/* are N_i = C-points of row i of the graph G (eq:nbhd with G the pattern  */
/* of A^{d_LS}), i excluded, in increasing column order.  Every W within   */
/* N_i with 1 <= |W| <= caliber is fitted (qr_fit; a numerically dependent */
/* W is skipped: within the rule its span is a smaller set's), and         */
/* for each size m the least functional best_m is kept (ties: the first W  */
/* in lexicographic order of candidate positions).  Values are normalised  */
/* by the functional of the empty set, S = sum_k w_k t_k^2 (the reading of */
/* the penalty's exponent as acting on a relative value).  The size is     */
/* then chosen by the penalty rule read as a scan in increasing size: the  */
/* incumbent starts at size 1 and is replaced by the best set of size m    */
/* when best_m / S < (incumbent / S)^(gamma (m - incumbent size)).  With   */
/* S = 0 every fit is exact and size 1 is kept.                            */
/*                                                                         */
/* Outputs per selected row (row-major nrows x caliber): P_col (the chosen */
/* W, increasing columns, -1 padded; C rows: i itself), P_val, ls_val (the */
/* functional at the minimiser, not normalised), status (0 ok, 1 no        */
/* candidate or every W dependent, 3 residual target with zero diagonal),  */
/* best (nrows x (caliber + 1), may be NULL): S, then best_m / S for m =   */
/* 1..caliber (-1 where no W of that size was fitted), ncand (may be NULL):*/
/* |N_i|.                                                                  */
/* ---------------------------------------------------------------------- */
void oracle_ls_search(int n, const int *rp, const int *ci, const double *a, const int *rpg,
                      const int *cig, int K, const double *X, const double *w,
                      const unsigned char *cf, int caliber, double gamma, int target, int nrows,
                      const int *rows, int *P_col, double *P_val, double *ls_val, int *status,
                      double *best, int *ncand)
{
    int cnt = rows ? nrows : n;
    double *t = (double *)malloc(sizeof(double) * K);
    double *sc = (double *)malloc(sizeof(double) * K);
    double *M = (double *)malloc(sizeof(double) * K * ORACLE_MAX_CAL);
    double *b = (double *)malloc(sizeof(double) * K);
    double *v = (double *)malloc(sizeof(double) * K);
    int *cand = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int r, s, k, e;
    for (r = 0; r < cnt; ++r) {
        int i = rows ? rows[r] : r;
        int *pc = P_col + (int64_t)r * caliber;
        double *pv = P_val + (int64_t)r * caliber;
        double *bo = best ? best + (int64_t)r * (caliber + 1) : NULL;
        int nc = 0, st = 0, m, inc_m = 0;
        double S = 0.0, bestv[ORACLE_MAX_CAL + 1];
        int bestset[ORACLE_MAX_CAL + 1][ORACLE_MAX_CAL];
        double inc_v = 0.0;

        for (s = 0; s < caliber; ++s) { pc[s] = -1; pv[s] = 0.0; }
        if (cf[i]) {
            pc[0] = i;
            pv[0] = 1.0;
            ls_val[r] = 0.0;
            status[r] = 0;
            if (bo) for (s = 0; s <= caliber; ++s) bo[s] = -1.0;
            if (ncand) ncand[r] = 0;
            continue;
        }
        if (fit_target(rp, ci, a, K, X, i, target, t, sc)) st = 3;
        for (k = 0; k < K; ++k) S += weight(w, k) * t[k] * t[k];
        for (e = rpg[i]; e < rpg[i + 1]; ++e)
            if (cig[e] != i && cf[cig[e]]) cand[nc++] = cig[e];
        if (ncand) ncand[r] = nc;

        /* every subset of each size, positions idx[0] < ... < idx[m-1] */
        for (m = 1; m <= caliber; ++m) {
            int idx[ORACLE_MAX_CAL], cols[ORACLE_MAX_CAL], q;
            bestv[m] = -1.0;
            if (m > nc) continue;
            for (q = 0; q < m; ++q) idx[q] = q;
            for (;;) {
                double coef[ORACLE_MAX_CAL], val;
                for (q = 0; q < m; ++q) cols[q] = cand[idx[q]];
                if (!qr_fit(K, X, w, t, cols, m, coef, &val, M, b, v) &&
                    (bestv[m] < 0.0 || val < bestv[m])) {
                    bestv[m] = val;
                    for (q = 0; q < m; ++q) bestset[m][q] = cols[q];
                }
                /* next combination in lexicographic order */
                q = m - 1;
                while (q >= 0 && idx[q] == nc - m + q) --q;
                if (q < 0) break;
                ++idx[q];
                for (++q; q < m; ++q) idx[q] = idx[q - 1] + 1;
            }
        }
        if (bo) {
            bo[0] = S;
            for (m = 1; m <= caliber; ++m)
                bo[m] = (bestv[m] < 0.0) ? -1.0 : (S > 0.0 ? bestv[m] / S : 0.0);
        }
        /* penalty rule, sizes in increasing order */
        for (m = 1; m <= caliber; ++m) {
            double rel, inc_rel;
            if (bestv[m] < 0.0) continue;
            if (inc_m == 0) {
                inc_m = m;
                inc_v = bestv[m];
                continue;
            }
            rel = S > 0.0 ? bestv[m] / S : 0.0;
            inc_rel = S > 0.0 ? inc_v / S : 0.0;
            if (rel < pow(inc_rel, gamma * (double)(m - inc_m))) {
                inc_m = m;
                inc_v = bestv[m];
            }
        }
        if (inc_m == 0) {
            ls_val[r] = S;
            status[r] = st ? st : 1;
            continue;
        }
        {
            double coef[ORACLE_MAX_CAL], val;
            qr_fit(K, X, w, t, bestset[inc_m], inc_m, coef, &val, M, b, v);
            for (s = 0; s < inc_m; ++s) {
                pc[s] = bestset[inc_m][s];
                pv[s] = coef[s];
            }
            ls_val[r] = val;
            status[r] = st;
        }
    }
    free(t); free(sc); free(M); free(b); free(v); free(cand);
}

/* ---------------------------------------------------------------------- */
/* Compatible relaxation (Sec. 3.2) and the coarsening loop of Sec. 4.2    */
/* (Algorithm 1).                                                          */
/*                                                                         */
/* F-relaxation (eq:frelax): relaxation applied to the F variables of the  */
/* homogeneous system, the C variables held at zero, so that each sweep is */
/* u_f <- (I - M_ff^{-1} A_ff) u_f.  M is the colour-phase Gauss-Seidel    */
/* splitting of oracle_color_gs (C rows take no colour and stay fixed).    */
/* The start is the constant 1 on F (Algorithm 1 starts every CR run from  */
/* a constant vector), 0 on C.                                             */
/*                                                                         */
/* Rate estimate (eq:meas1): rho_f = (||u_f^nu||_2 / ||u_f^0||_2)^(1/nu).  */
/* Candidate measure (remark after Algorithm 1): sigma_i = |u_i^nu| /      */
/* ||u^nu||_inf, and the candidates are the F points with sigma_i > tol,   */
/* tol = 1 - rho_f (Sec. 5.2).                                             */
/* ---------------------------------------------------------------------- */

/* nu F-relaxation sweeps from the constant start; u (n) receives u^nu.
 * Returns rho_f (0 when F is empty). */
double oracle_cr_rate(int n, const int *rp, const int *ci, const double *a, const int *color,
                      int ncolors, const unsigned char *cf, int nu, double *u)
{
    int *fcol = (int *)malloc(sizeof(int) * (size_t)(n ? n : 1));
    double n0 = 0.0, n1 = 0.0;
    int i;
    for (i = 0; i < n; ++i) {
        fcol[i] = cf[i] ? -1 : color[i];
        u[i] = cf[i] ? 0.0 : 1.0;
        n0 += u[i] * u[i];
    }
    oracle_color_gs(n, rp, ci, a, 1, fcol, ncolors, nu, u);
    for (i = 0; i < n; ++i)
        if (!cf[i]) n1 += u[i] * u[i];
    free(fcol);
    if (n0 == 0.0 || nu <= 0) return 0.0;
    return pow(sqrt(n1) / sqrt(n0), 1.0 / (double)nu);
}

/* z[i] = 1 for the F points with sigma_i = |u_i| / max_F |u| > tol. */
void oracle_cr_candidates(int n, const unsigned char *cf, const double *u, double tol,
                          unsigned char *z)
{
    double m = 0.0;
    int i;
    for (i = 0; i < n; ++i)
        if (!cf[i] && fabs(u[i]) > m) m = fabs(u[i]);
    for (i = 0; i < n; ++i)
        z[i] = (unsigned char)(!cf[i] && m > 0.0 && fabs(u[i]) / m > tol);
}

/* ---------------------------------------------------------------------- */
/* Independent set of the candidates on the strength graph (Algorithm 1,   */
/* "independent set of Z based on M^d").  Two candidates are neighbours    */
/* when either is strongly connected to the other (strong[e] for entry e   */
/* = (i, j) of the pattern).  Following the weighting of the classical     */
/* colouring (Sec. 2), a point's weight is the number of points strongly   */
/* depending on it, lambda_i = |S_i^T|; the set is the greedy maximal one  */
/* taken in decreasing (lambda_i, h_i, i), h_i the (i+1)-th output of      */
/* splitmix64 seeded with `seed`.  sel[i] = 1 for the chosen points.       */
/* ---------------------------------------------------------------------- */
static const int *g_lam;
static const uint64_t *g_h;

static int cmp_priority_desc(const void *pa, const void *pb)
{
    int a = *(const int *)pa, b = *(const int *)pb;
    if (g_lam[a] != g_lam[b]) return g_lam[a] > g_lam[b] ? -1 : 1;
    if (g_h[a] != g_h[b]) return g_h[a] > g_h[b] ? -1 : 1;
    return a > b ? -1 : (a < b ? 1 : 0);
}

int oracle_independent_set(int n, const int *rp, const int *ci, const unsigned char *strong,
                           const unsigned char *z, uint64_t seed, unsigned char *sel)
{
    int *lam = (int *)calloc((size_t)(n ? n : 1), sizeof(int));
    uint64_t *h = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    int *order = (int *)malloc(sizeof(int) * (size_t)(n ? n : 1));
    /* transpose of the strong graph: tp[j] .. tp[j+1] lists the rows i with
     * a strong entry (i, j) */
    int *tp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *trow, *fill;
    uint64_t st = seed;
    int i, e, m = 0, count = 0;
    for (i = 0; i < n; ++i) h[i] = splitmix64_next(&st);
    for (i = 0; i < n; ++i)
        for (e = rp[i]; e < rp[i + 1]; ++e)
            if (strong[e]) {
                ++lam[ci[e]];
                ++tp[ci[e] + 1];
            }
    for (i = 0; i < n; ++i) tp[i + 1] += tp[i];
    trow = (int *)malloc(sizeof(int) * (size_t)(tp[n] ? tp[n] : 1));
    fill = (int *)calloc((size_t)(n ? n : 1), sizeof(int));
    for (i = 0; i < n; ++i)
        for (e = rp[i]; e < rp[i + 1]; ++e)
            if (strong[e]) trow[tp[ci[e]] + fill[ci[e]]++] = i;
    for (i = 0; i < n; ++i) {
        sel[i] = 0;
        if (z[i]) order[m++] = i;
    }
    g_lam = lam;
    g_h = h;
    qsort(order, (size_t)m, sizeof(int), cmp_priority_desc);
    for (i = 0; i < m; ++i) {
        int v = order[i], blocked = 0, q;
        for (e = rp[v]; e < rp[v + 1] && !blocked; ++e)
            if (strong[e] && ci[e] != v && sel[ci[e]]) blocked = 1;
        for (q = tp[v]; q < tp[v + 1] && !blocked; ++q)
            if (trow[q] != v && sel[trow[q]]) blocked = 1;
        if (!blocked) {
            sel[v] = 1;
            ++count;
        }
    }
    free(lam); free(h); free(order); free(tp); free(trow); free(fill);
    return count;
}

/* Algorithm 1 (Sec. 4.2): start from C_0 (cf[i] = 1 marks C), run nu CR
 * sweeps, and while rho_f > delta: candidates Z (sigma_i > 1 - rho_f), the
 * strength graph restricted to F (oracle_strength with the F mask, on the
 * distances mu of the pattern), C grown by the independent set of Z, and
 * CR again.  Stops also when Z is empty or after max_stages growth steps.
 * rho[s] and ncoarse[s] record rho_f and |C| after s growth steps
 * (arrays of max_stages + 1).  Returns the number of growth steps.
 * The strength graph and the independent set live on the pattern
 * (rpg, cig) with mu given per entry of it: the graph of A^d for M^d
 * (Sec. 4.2), the pattern of A itself for d = 1; CR relaxes with A. */
int oracle_cr_coarsen_graph(int n, const int *rp, const int *ci, const double *a,
                            const int *rpg, const int *cig, const int *color, int ncolors,
                            const double *mu, double theta, int nu, double delta, int max_stages,
                            uint64_t seed, unsigned char *cf, double *rho, int64_t *ncoarse)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    unsigned char *z = (unsigned char *)malloc((size_t)(n ? n : 1));
    unsigned char *fm = (unsigned char *)malloc((size_t)(n ? n : 1));
    unsigned char *sel = (unsigned char *)malloc((size_t)(n ? n : 1));
    int64_t nnz = n ? rpg[n] : 0;
    unsigned char *strong = (unsigned char *)malloc((size_t)(nnz ? nnz : 1));
    int stage = 0, i;
    int64_t nc = 0;
    double r;
    for (i = 0; i < n; ++i) nc += cf[i] != 0;
    r = oracle_cr_rate(n, rp, ci, a, color, ncolors, cf, nu, u);
    rho[0] = r;
    ncoarse[0] = nc;
    while (r > delta && stage < max_stages) {
        int any = 0;
        oracle_cr_candidates(n, cf, u, 1.0 - r, z);
        for (i = 0; i < n; ++i) any |= z[i];
        if (!any) break;
        for (i = 0; i < n; ++i) fm[i] = (unsigned char)!cf[i];
        oracle_strength(n, rpg, cig, mu, theta, fm, strong, NULL);
        oracle_independent_set(n, rpg, cig, strong, z, seed + (uint64_t)stage, sel);
        for (i = 0; i < n; ++i)
            if (sel[i]) {
                cf[i] = 1;
                ++nc;
            }
        ++stage;
        r = oracle_cr_rate(n, rp, ci, a, color, ncolors, cf, nu, u);
        rho[stage] = r;
        ncoarse[stage] = nc;
    }
    free(u); free(z); free(fm); free(sel); free(strong);
    return stage;
}

/* Algorithm 1 with M^1: the strength graph on the pattern of A */
int oracle_cr_coarsen(int n, const int *rp, const int *ci, const double *a, const int *color,
                      int ncolors, const double *mu, double theta, int nu, double delta,
                      int max_stages, uint64_t seed, unsigned char *cf, double *rho,
                      int64_t *ncoarse)
{
    return oracle_cr_coarsen_graph(n, rp, ci, a, rp, ci, color, ncolors, mu, theta, nu, delta,
                                   max_stages, seed, cf, rho, ncoarse);
}

/* ====================================================================== */
/* Galerkin coarse operator and the two-grid method of Sec. 5.2            */
/* ====================================================================== */

/* ---------------------------------------------------------------------- */
/* Interpolation as a matrix.  Row i of P (n x nc) holds P_val[i][q] in    */
/* column cidx(P_col[i][q]) for P_col[i][q] >= 0, where cidx numbers the C */
/* points (cf != 0) in increasing fine index.  A_c = P^T A P (the Galerkin */
/* operator of the two-grid method, Sec. 5.2), formed row by row: coarse   */
/* row I accumulates p_iI * a_ij * p_jJ into column J, over the fine rows  */
/* i with p_iI != 0 in increasing i, row i's entries in CSR order and row  */
/* j's weights in their stored order; each product is formed as            */
/* (p_iI * a_ij) * p_jJ and added in that order.                           */
/* ---------------------------------------------------------------------- */
static int *coarse_index(int n, const unsigned char *cf, int *nc)
{
    int *cidx = (int *)malloc(sizeof(int) * (size_t)(n ? n : 1));
    int i, c = 0;
    for (i = 0; i < n; ++i) cidx[i] = cf[i] ? c++ : -1;
    *nc = c;
    return cidx;
}

/* P^T as lists: pt[I] .. pt[I+1] index (prow, pval) pairs, by increasing i */
static void p_transpose(int n, int caliber, const int *Pc, const double *Pv, const int *cidx,
                        int nc, int **pt_out, int **prow_out, double **pval_out)
{
    int *pt = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *fill = (int *)calloc((size_t)(nc ? nc : 1), sizeof(int));
    int i, q, m;
    int *prow;
    double *pval;
    for (i = 0; i < n; ++i)
        for (q = 0; q < caliber; ++q)
            if (Pc[(int64_t)i * caliber + q] >= 0) ++pt[cidx[Pc[(int64_t)i * caliber + q]] + 1];
    for (m = 0; m < nc; ++m) pt[m + 1] += pt[m];
    prow = (int *)malloc(sizeof(int) * (size_t)(pt[nc] ? pt[nc] : 1));
    pval = (double *)malloc(sizeof(double) * (size_t)(pt[nc] ? pt[nc] : 1));
    for (i = 0; i < n; ++i)
        for (q = 0; q < caliber; ++q) {
            int c = Pc[(int64_t)i * caliber + q];
            if (c < 0) continue;
            c = cidx[c];
            prow[pt[c] + fill[c]] = i;
            pval[pt[c] + fill[c]] = Pv[(int64_t)i * caliber + q];
            ++fill[c];
        }
    free(fill);
    *pt_out = pt;
    *prow_out = prow;
    *pval_out = pval;
}

static int cmp_int_asc(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* cnt[I] = stored entries of coarse row I (every J reached by a product,
 * also if the products cancel).  Returns nc. */
int oracle_galerkin_counts(int n, const int *rp, const int *ci, int caliber, const int *Pc,
                           const double *Pv, const unsigned char *cf, int *cnt)
{
    int nc, I, t, e, q, m;
    int *cidx = coarse_index(n, cf, &nc);
    int *pt, *prow, *mark, *list;
    double *pval;
    p_transpose(n, caliber, Pc, Pv, cidx, nc, &pt, &prow, &pval);
    mark = (int *)malloc(sizeof(int) * (size_t)(nc ? nc : 1));
    list = (int *)malloc(sizeof(int) * (size_t)(nc ? nc : 1));
    for (I = 0; I < nc; ++I) mark[I] = -1;
    for (I = 0; I < nc; ++I) {
        m = 0;
        for (t = pt[I]; t < pt[I + 1]; ++t) {
            int i = prow[t];
            for (e = rp[i]; e < rp[i + 1]; ++e) {
                int j = ci[e];
                for (q = 0; q < caliber; ++q) {
                    int c = Pc[(int64_t)j * caliber + q];
                    if (c < 0) continue;
                    c = cidx[c];
                    if (mark[c] != I) {
                        mark[c] = I;
                        list[m++] = c;
                    }
                }
            }
        }
        cnt[I] = m;
    }
    free(cidx); free(pt); free(prow); free(pval); free(mark); free(list);
    return nc;
}

void oracle_galerkin_fill(int n, const int *rp, const int *ci, const double *a, int caliber,
                          const int *Pc, const double *Pv, const unsigned char *cf, const int *rpc,
                          int *colc, double *valc)
{
    int nc, I, t, e, q, m, r;
    int *cidx = coarse_index(n, cf, &nc);
    int *pt, *prow, *mark, *list;
    double *pval, *acc;
    p_transpose(n, caliber, Pc, Pv, cidx, nc, &pt, &prow, &pval);
    mark = (int *)malloc(sizeof(int) * (size_t)(nc ? nc : 1));
    list = (int *)malloc(sizeof(int) * (size_t)(nc ? nc : 1));
    acc = (double *)malloc(sizeof(double) * (size_t)(nc ? nc : 1));
    for (I = 0; I < nc; ++I) mark[I] = -1;
    for (I = 0; I < nc; ++I) {
        m = 0;
        for (t = pt[I]; t < pt[I + 1]; ++t) {
            int i = prow[t];
            double piI = pval[t];
            for (e = rp[i]; e < rp[i + 1]; ++e) {
                int j = ci[e];
                double pa = piI * a[e];
                for (q = 0; q < caliber; ++q) {
                    int c = Pc[(int64_t)j * caliber + q];
                    double prod;
                    if (c < 0) continue;
                    c = cidx[c];
                    prod = pa * Pv[(int64_t)j * caliber + q];
                    if (mark[c] != I) {
                        mark[c] = I;
                        list[m++] = c;
                        acc[c] = prod;
                    } else {
                        acc[c] = acc[c] + prod;
                    }
                }
            }
        }
        qsort(list, (size_t)m, sizeof(int), cmp_int_asc);
        for (r = 0; r < m; ++r) {
            colc[rpc[I] + r] = list[r];
            valc[rpc[I] + r] = acc[list[r]];
        }
    }
    free(cidx); free(pt); free(prow); free(pval); free(mark); free(list); free(acc);
}

/* ---------------------------------------------------------------------- */
/* Two-grid method of Sec. 5.2 on the homogeneous system A e = 0: `pre`    */
/* colour-phase Gauss-Seidel sweeps, the coarse-grid correction            */
/* e <- e - P A_c^{-1} P^T A e with the coarse system solved directly      */
/* (dense Cholesky factorisation of A_c), `post` sweeps; `iters` cycles    */
/* from the K columns of E0.  rho[k] = ||e^iters||_A / ||e^(iters-1)||_A   */
/* for column k; hist (may be NULL, (iters + 1) x K) receives ||e^t||_A.   */
/* Returns 0, or 1 if A_c has a non-positive pivot.                        */
/* ---------------------------------------------------------------------- */
static double a_norm(int n, const int *rp, const int *ci, const double *a, int K,
                     const double *E, int k)
{
    double s = 0.0;
    int i, e;
    for (i = 0; i < n; ++i) {
        double y = 0.0;
        for (e = rp[i]; e < rp[i + 1]; ++e) y += a[e] * E[(int64_t)ci[e] * K + k];
        s += E[(int64_t)i * K + k] * y;
    }
    return sqrt(s > 0.0 ? s : 0.0);
}

int oracle_two_grid(int n, const int *rp, const int *ci, const double *a, const int *color,
                    int ncolors, int caliber, const int *Pc, const double *Pv,
                    const unsigned char *cf, const int *rpc, const int *colc, const double *valc,
                    int K, const double *E0, int iters, int pre, int post, double *rho,
                    double *hist)
{
    int nc, i, j, k, e, q, it, I;
    int *cidx = coarse_index(n, cf, &nc);
    double *L = (double *)calloc((size_t)nc * (nc ? nc : 1), sizeof(double));
    double *E = (double *)malloc(sizeof(double) * (size_t)n * K);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *rc = (double *)malloc(sizeof(double) * (size_t)(nc ? nc : 1));
    double *prev = (double *)malloc(sizeof(double) * K);
    int bad = 0;
    memcpy(E, E0, sizeof(double) * (size_t)n * K);
    /* dense A_c, then its Cholesky factor in the lower triangle */
    for (I = 0; I < nc; ++I)
        for (e = rpc[I]; e < rpc[I + 1]; ++e) L[(int64_t)I * nc + colc[e]] = valc[e];
    for (j = 0; j < nc && !bad; ++j) {
        double d = L[(int64_t)j * nc + j];
        for (q = 0; q < j; ++q) d -= L[(int64_t)j * nc + q] * L[(int64_t)j * nc + q];
        if (!(d > 0.0)) {
            bad = 1;
            break;
        }
        d = sqrt(d);
        L[(int64_t)j * nc + j] = d;
        for (i = j + 1; i < nc; ++i) {
            double s = L[(int64_t)i * nc + j];
            for (q = 0; q < j; ++q) s -= L[(int64_t)i * nc + q] * L[(int64_t)j * nc + q];
            L[(int64_t)i * nc + j] = s / d;
        }
    }
    for (k = 0; k < K; ++k) {
        rho[k] = 0.0;
        prev[k] = 0.0;
        if (hist) hist[k] = a_norm(n, rp, ci, a, K, E, k);
    }
    for (it = 0; it < iters && !bad; ++it) {
        oracle_color_gs(n, rp, ci, a, K, color, ncolors, pre, E);
        for (k = 0; k < K; ++k) {
            /* r = -A e (b = 0), r_c = P^T r */
            for (i = 0; i < n; ++i) {
                double y = 0.0;
                for (e = rp[i]; e < rp[i + 1]; ++e) y += a[e] * E[(int64_t)ci[e] * K + k];
                r[i] = -y;
            }
            for (I = 0; I < nc; ++I) rc[I] = 0.0;
            for (i = 0; i < n; ++i)
                for (q = 0; q < caliber; ++q) {
                    int c = Pc[(int64_t)i * caliber + q];
                    if (c >= 0) rc[cidx[c]] += Pv[(int64_t)i * caliber + q] * r[i];
                }
            /* A_c e_c = r_c: L y = r_c, then L^T e_c = y */
            for (I = 0; I < nc; ++I) {
                double s = rc[I];
                for (q = 0; q < I; ++q) s -= L[(int64_t)I * nc + q] * rc[q];
                rc[I] = s / L[(int64_t)I * nc + I];
            }
            for (I = nc - 1; I >= 0; --I) {
                double s = rc[I];
                for (q = I + 1; q < nc; ++q) s -= L[(int64_t)q * nc + I] * rc[q];
                rc[I] = s / L[(int64_t)I * nc + I];
            }
            /* e += P e_c */
            for (i = 0; i < n; ++i) {
                double s = 0.0;
                for (q = 0; q < caliber; ++q) {
                    int c = Pc[(int64_t)i * caliber + q];
                    if (c >= 0) s += Pv[(int64_t)i * caliber + q] * rc[cidx[c]];
                }
                E[(int64_t)i * K + k] += s;
            }
        }
        oracle_color_gs(n, rp, ci, a, K, color, ncolors, post, E);
        for (k = 0; k < K; ++k) {
            double an = a_norm(n, rp, ci, a, K, E, k);
            if (it == iters - 1) rho[k] = prev[k] > 0.0 ? an / prev[k] : 0.0;
            prev[k] = an;
            if (hist) hist[(int64_t)(it + 1) * K + k] = an;
        }
    }
    free(cidx); free(L); free(E); free(r); free(rc); free(prev);
    return bad;
}

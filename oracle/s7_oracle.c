/*
 * FP64 CPU oracle for BiCGStab on the 7-point variable-coefficient stencil
 * system (and on the 2D 9-point operator of section IV, "SpMV (2D)").  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU
 * baseline of the benchmark call it; the GPU library never does, and the two
 * share no code.
 *
 * What it computes (paper: "Fast Stencil-Code Computation on a Wafer-Scale
 * Processor", SC20):
 *   - the linear system A x = b of Eq. (1), section III;
 *   - A is the 7-point stencil operator on an X x Y x Z mesh (section IV,
 *     "SpMV (3D)"): row (i,j,k) has the main diagonal and the six
 *     direction-named off-diagonals xm, xp, ym, yp, zm, zp, where xp
 *     multiplies the value at (i+1,j,k) and xm the value at (i-1,j,k), and
 *     likewise in y and z.  Neighbours outside the mesh are zero (Dirichlet);
 *     their coefficients are not entered in the matrix;
 *   - optional diagonal (Jacobi) preconditioning, which the paper applies so
 *     that the main diagonal becomes all ones (section IV, first
 *     paragraph): row i and b_i are divided by a_ii;
 *   - the "Standard BiCGStab" iteration of Algorithm 1, with the readings
 *     listed below, in FP64 with plain left-to-right loops.
 *
 * Readings of Algorithm 1 (the paper is silent or garbled on these):
 *   - r_0 = b - A x_0 (the listing writes r_0 := b, i.e. x_0 = 0);
 *   - the shadow vector r_hat = r_0 is fixed for the whole solve;
 *   - the solution update writes x_{i+1} (the listing overwrites x_i);
 *   - stopping: after the q-step, if ||q||/||b|| <= tol then x += alpha p
 *     and stop ("half-step" exit); after the full step, stop if
 *     ||r_{i+1}||/||b|| <= tol, or when max_iter full iterations are done;
 *   - breakdown: (r_hat, s) == 0, (y, y) == 0 or (r_hat, r_{i+1}) == 0
 *     exactly, or a non-finite scalar.
 * The CSR uses ascending column order; all sums run left to right.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_BREAKDOWN 2
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define OR_REASON_NONE 0
#define OR_REASON_RHO_ZERO 1
#define OR_REASON_RS_ZERO 2
#define OR_REASON_YY_ZERO 3
#define OR_REASON_NONFINITE 4

typedef struct {
    double rho;     /* (r_hat, r_i) */
    double alpha;
    double omega;
    double beta;
    double sigma;   /* (r_hat, s_i) */
    double nb;      /* ||b|| */
    double tol;
    double res_rec; /* last recurrence residual ||r||/||b|| (or ||q||/||b|| at a half-step exit) */
    int64_t iter;   /* full iterations done (a half-step exit counts as one) */
    int64_t max_iter;
    int32_t status;
    int32_t reason;
    int32_t done;
    int32_t half_exit;
} oracle_bicg;

/* Number of stored entries of the CSR of the nx x ny x nz stencil. */
int64_t oracle_csr_nnz(int32_t nx, int32_t ny, int32_t nz) {
    int64_t n = (int64_t)nx * ny * nz;
    int64_t nnz = n;                          /* diagonal */
    nnz += 2 * (int64_t)(nx - 1) * ny * nz;   /* x links */
    nnz += 2 * (int64_t)nx * (ny - 1) * nz;   /* y links */
    nnz += 2 * (int64_t)nx * ny * (nz - 1);   /* z links */
    return nnz;
}

/*
 * Assemble the CSR of A from the seven coefficient arrays
 * (diag, xm, xp, ym, yp, zm, zp; each nx*ny*nz floats, x fastest).
 * Values are the FP32 inputs widened exactly to FP64.
 */
int64_t oracle_build_csr(int32_t nx, int32_t ny, int32_t nz,
                         const float *diag, const float *xm, const float *xp,
                         const float *ym, const float *yp,
                         const float *zm, const float *zp,
                         int64_t *rowptr, int64_t *col, double *val) {
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    int64_t e = 0;
    rowptr[0] = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = i + nx * (j + ny * k);
                /* ascending column order: z-, y-, x-, centre, x+, y+, z+ */
                if (k > 0)      { col[e] = c - sz; val[e] = (double)zm[c]; ++e; }
                if (j > 0)      { col[e] = c - sy; val[e] = (double)ym[c]; ++e; }
                if (i > 0)      { col[e] = c - sx; val[e] = (double)xm[c]; ++e; }
                col[e] = c; val[e] = (double)diag[c]; ++e;
                if (i < nx - 1) { col[e] = c + sx; val[e] = (double)xp[c]; ++e; }
                if (j < ny - 1) { col[e] = c + sy; val[e] = (double)yp[c]; ++e; }
                if (k < nz - 1) { col[e] = c + sz; val[e] = (double)zp[c]; ++e; }
                rowptr[c + 1] = e;
            }
    return e;
}

/*
 * The 2D 9-point operator (section IV, "SpMV (2D)"): on an nx x ny mesh, row
 * (i,j) holds the main diagonal and eight off-diagonals w, e, s, n (the four
 * axis neighbours: w multiplies the value at (i-1,j), e at (i+1,j), s at
 * (i,j-1), n at (i,j+1)) and sw, se, nw, ne (the corners: sw multiplies the
 * value at (i-1,j-1), se at (i+1,j-1), nw at (i-1,j+1), ne at (i+1,j+1)).
 * Neighbours outside the mesh are zero and their coefficients are not
 * entered.  Arrays are nx*ny floats, x fastest.
 */
int64_t oracle_csr_nnz_2d9(int32_t nx, int32_t ny) {
    int64_t e = 0;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t dj = -1; dj <= 1; ++dj)
                for (int64_t di = -1; di <= 1; ++di)
                    if (i + di >= 0 && i + di < nx && j + dj >= 0 && j + dj < ny) ++e;
    return e;
}

int64_t oracle_build_csr_2d9(int32_t nx, int32_t ny, const float *diag, const float *w,
                             const float *e, const float *s, const float *n,
                             const float *sw, const float *se, const float *nw,
                             const float *ne, int64_t *rowptr, int64_t *col, double *val) {
    /* the coefficient of neighbour (di, dj), by (dj+1)*3 + (di+1): ascending columns */
    const float *by[9] = {sw, s, se, w, diag, e, nw, n, ne};
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t c = i + nx * j;
            for (int64_t dj = -1; dj <= 1; ++dj)
                for (int64_t di = -1; di <= 1; ++di) {
                    if (i + di < 0 || i + di >= nx || j + dj < 0 || j + dj >= ny) continue;
                    col[k] = c + di + nx * dj;
                    val[k] = (double)by[(dj + 1) * 3 + (di + 1)][c];
                    ++k;
                }
            rowptr[c + 1] = k;
        }
    return k;
}

/*
 * Threads of the row loop of oracle_spmv (1 by default).  Rows are independent
 * and each is still summed left to right, so the product is the same for any
 * count; only the CPU baseline of the benchmark sets more than one, to time
 * the oracle on all host cores.  Inner products and vector updates stay
 * single-threaded.
 */
static int g_threads = 1;
void oracle_set_threads(int32_t t) { g_threads = t > 1 ? t : 1; }

/* y = A x, each row summed left to right over its entries. */
void oracle_spmv(int64_t n, const int64_t *rowptr, const int64_t *col,
                 const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) acc += val[e] * x[col[e]];
        y[r] = acc;
    }
}

/* Rows [r0, r1) only: y[r - r0] = (A x)_r. */
void oracle_spmv_rows(int64_t r0, int64_t r1, const int64_t *rowptr, const int64_t *col,
                      const double *val, const double *x, double *y) {
    for (int64_t r = r0; r < r1; ++r) {
        double acc = 0.0;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) acc += val[e] * x[col[e]];
        y[r - r0] = acc;
    }
}

double oracle_dot(int64_t n, const double *a, const double *b) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/* Left diagonal scaling: row r of A and b_r divided by a_rr.  Returns -1 if a_rr == 0. */
int oracle_jacobi_scale(int64_t n, const int64_t *rowptr, const int64_t *col,
                        double *val, double *b) {
    for (int64_t r = 0; r < n; ++r) {
        double d = 0.0;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
            if (col[e] == r) d = val[e];
        if (d == 0.0) return -1;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) val[e] = val[e] / d;
        if (b) b[r] = b[r] / d;
    }
    return 0;
}

/*
 * Start of Algorithm 1: r = b - A x0, r_hat = r, p = r, rho = (r_hat, r),
 * nb = ||b||.  Decides the trivial exits (b = 0, already converged,
 * max_iter = 0).
 */
int oracle_bicgstab_init(int64_t n, const int64_t *rowptr, const int64_t *col,
                         const double *val, const double *b, double *x,
                         double *r, double *rhat, double *p, double tol,
                         int64_t max_iter, oracle_bicg *st) {
    memset(st, 0, sizeof(*st));
    st->tol = tol;
    st->max_iter = max_iter;
    st->nb = sqrt(oracle_dot(n, b, b));
    if (st->nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = 0.0; rhat[i] = 0.0; p[i] = 0.0; }
        st->status = OR_OK;
        st->done = 1;
        return st->status;
    }
    oracle_spmv(n, rowptr, col, val, x, r);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - r[i];
        rhat[i] = r[i];
        p[i] = r[i];
    }
    st->rho = oracle_dot(n, rhat, r);
    st->res_rec = sqrt(oracle_dot(n, r, r)) / st->nb;
    if (!isfinite(st->res_rec)) {
        st->status = OR_BREAKDOWN; st->reason = OR_REASON_NONFINITE; st->done = 1;
    } else if (st->res_rec <= tol) {
        st->status = OR_OK; st->done = 1;
    } else if (max_iter <= 0) {
        st->status = OR_NOT_CONVERGED; st->done = 1;
    }
    return st->status;
}

static void set_breakdown(oracle_bicg *st, int32_t reason) {
    st->status = OR_BREAKDOWN;
    st->reason = reason;
    st->done = 1;
}

/* One iteration of Algorithm 1 (s, alpha, q, y, omega, x, r, beta, p). */
int oracle_bicgstab_step(int64_t n, const int64_t *rowptr, const int64_t *col,
                         const double *val, double *x, double *r, const double *rhat,
                         double *p, double *s, double *q, double *y, oracle_bicg *st) {
    if (st->done) return st->status;
    /* s_i = A p_i ; alpha_i = (r0, r_i) / (r0, s_i) */
    oracle_spmv(n, rowptr, col, val, p, s);
    st->sigma = oracle_dot(n, rhat, s);
    if (st->sigma == 0.0) { set_breakdown(st, OR_REASON_RS_ZERO); return st->status; }
    st->alpha = st->rho / st->sigma;
    if (!isfinite(st->alpha)) { set_breakdown(st, OR_REASON_NONFINITE); return st->status; }
    /* q_i = r_i - alpha_i s_i */
    for (int64_t i = 0; i < n; ++i) q[i] = r[i] - st->alpha * s[i];
    double qn = sqrt(oracle_dot(n, q, q)) / st->nb;
    if (qn <= st->tol) {
        /* half-step exit: x_{i+1} = x_i + alpha_i p_i, residual is q_i */
        for (int64_t i = 0; i < n; ++i) { x[i] = x[i] + st->alpha * p[i]; r[i] = q[i]; }
        st->omega = 0.0;
        st->iter += 1;
        st->res_rec = qn;
        st->half_exit = 1;
        st->status = OR_OK;
        st->done = 1;
        return st->status;
    }
    /* y_i = A q_i ; omega_i = (q_i, y_i) / (y_i, y_i) */
    oracle_spmv(n, rowptr, col, val, q, y);
    double yy = oracle_dot(n, y, y);
    if (yy == 0.0) { set_breakdown(st, OR_REASON_YY_ZERO); return st->status; }
    st->omega = oracle_dot(n, q, y) / yy;
    if (!isfinite(st->omega)) { set_breakdown(st, OR_REASON_NONFINITE); return st->status; }
    /* x_{i+1} = x_i + alpha_i p_i + omega_i q_i ; r_{i+1} = q_i - omega_i y_i */
    for (int64_t i = 0; i < n; ++i) {
        x[i] = x[i] + st->alpha * p[i] + st->omega * q[i];
        r[i] = q[i] - st->omega * y[i];
    }
    st->iter += 1;
    double rho_new = oracle_dot(n, rhat, r);
    st->res_rec = sqrt(oracle_dot(n, r, r)) / st->nb;
    if (!isfinite(st->res_rec)) { set_breakdown(st, OR_REASON_NONFINITE); return st->status; }
    if (st->res_rec <= st->tol) { st->status = OR_OK; st->done = 1; st->rho = rho_new; return st->status; }
    if (st->iter >= st->max_iter) { st->status = OR_NOT_CONVERGED; st->done = 1; st->rho = rho_new; return st->status; }
    if (rho_new == 0.0) { set_breakdown(st, OR_REASON_RHO_ZERO); return st->status; }
    /* beta_i = (alpha_i / omega_i) (r0, r_{i+1}) / (r0, r_i) ; p_{i+1} = r_{i+1} + beta_i (p_i - omega_i s_i) */
    st->beta = (st->alpha / st->omega) * (rho_new / st->rho);
    if (!isfinite(st->beta)) { set_breakdown(st, OR_REASON_NONFINITE); return st->status; }
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + st->beta * (p[i] - st->omega * s[i]);
    st->rho = rho_new;
    return st->status;
}

/*
 * Whole solve.  x holds x0 on entry and the last iterate on exit.  If
 * ntrace > 0, alpha/omega/rho (rho = (r0, r_i) at the start of iteration i)
 * and the recurrence residual after each iteration are recorded for the
 * first ntrace iterations.
 */
int oracle_bicgstab(int64_t n, const int64_t *rowptr, const int64_t *col,
                    const double *val, const double *b, double *x, double tol,
                    int64_t max_iter, oracle_bicg *st, int64_t ntrace,
                    double *tr_rho, double *tr_alpha, double *tr_omega, double *tr_res) {
    double *buf = (double *)malloc(sizeof(double) * (size_t)n * 6);
    if (!buf) return OR_ENOMEM;
    double *r = buf, *rhat = buf + n, *p = buf + 2 * n, *s = buf + 3 * n,
           *q = buf + 4 * n, *y = buf + 5 * n;
    oracle_bicgstab_init(n, rowptr, col, val, b, x, r, rhat, p, tol, max_iter, st);
    while (!st->done) {
        int64_t it = st->iter;
        double rho = st->rho;
        oracle_bicgstab_step(n, rowptr, col, val, x, r, rhat, p, s, q, y, st);
        if (it < ntrace) {
            if (tr_rho) tr_rho[it] = rho;
            if (tr_alpha) tr_alpha[it] = st->alpha;
            if (tr_omega) tr_omega[it] = st->omega;
            if (tr_res) tr_res[it] = st->res_rec;
        }
    }
    free(buf);
    return st->status;
}

/*
 * Pipelined BiCGStab (Cools and Vanroose, "The communication-hiding pipelined
 * BiCGStab method for the parallel solution of large unsymmetric linear
 * systems", Parallel Computing 65, 2017), in a form with a single reduction
 * per iteration.  In exact arithmetic its iterates are those of Algorithm 1;
 * the matrix products are carried forward by recurrences instead:
 *   s_i = A p_i, z_i = A s_i, w_i = A r_i, t_i = A w_i, v_i = A z_i, y_i = A q_i.
 * Iteration i:
 *   p = r + beta (p - omega s),  s = w + beta (s - omega z),  z = t + beta (z - omega v)
 *   q = r - alpha s,  y = w - alpha z,  v = A z
 *   one reduction: (r,r), (q,y), (y,y), (q,q), (r0,q), (r0,y), (r0,t), (r0,v), (r0,s), (r0,z)
 *   omega = (q,y)/(y,y);  x += alpha p + omega q;  r = q - omega y;  w = y - omega (t - alpha v)
 *   rho' = (r0,q) - omega (r0,y)                       [= (r0, r_{i+1})]
 *   beta = (alpha/omega) rho'/rho
 *   sigma' = (r0,y) - omega ((r0,t) - alpha (r0,v)) + beta ((r0,s) - omega (r0,z))   [= (r0, A p_{i+1})]
 *   alpha' = rho'/sigma';  t = A w
 * with beta = 0 and p = s = z = v = 0 before iteration 0, w_0 = A r_0, t_0 = A w_0,
 * rho_0 = (r0, r_0), alpha_0 = rho_0 / (r0, w_0).
 * Readings (the method is not in the paper; these mirror Algorithm 1's):
 *   - ||r_i|| is taken in iteration i's reduction, so the stopping test on
 *     r_i, and the iteration cap, are decided there: x_i is returned and the
 *     work of that iteration before the reduction is discarded;
 *   - the half-step test on ||q|| and x += alpha p, as in Algorithm 1;
 *   - breakdown: (r0, w_0) or sigma' == 0, (y,y) == 0, or a non-finite scalar;
 *     rho' == 0 is a breakdown unless the recurrence value of ||r_{i+1}||^2,
 *     (q,q) - 2 omega (q,y) + omega^2 (y,y), already meets the tolerance.
 * x holds x0 on entry and the last iterate on exit; traces as oracle_bicgstab
 * (rho, alpha, omega of iteration i, and ||r_{i+1}||/||b|| once known).
 */
int oracle_bicgstab_pipelined(int64_t n, const int64_t *rowptr, const int64_t *col,
                              const double *val, const double *b, double *x, double tol,
                              int64_t max_iter, oracle_bicg *st, int64_t ntrace,
                              double *tr_rho, double *tr_alpha, double *tr_omega, double *tr_res) {
    memset(st, 0, sizeof(*st));
    st->tol = tol;
    st->max_iter = max_iter;
    st->nb = sqrt(oracle_dot(n, b, b));
    if (st->nb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        st->status = OR_OK;
        st->done = 1;
        return st->status;
    }
    double *buf = (double *)calloc((size_t)n * 11, sizeof(double));
    if (!buf) return OR_ENOMEM;
    double *r = buf, *rh = buf + n, *p = buf + 2 * n, *s = buf + 3 * n, *z = buf + 4 * n,
           *q = buf + 5 * n, *y = buf + 6 * n, *w = buf + 7 * n, *t = buf + 8 * n, *v = buf + 9 * n,
           *tmp = buf + 10 * n;
    oracle_spmv(n, rowptr, col, val, x, tmp);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - tmp[i];
        rh[i] = r[i];
    }
    oracle_spmv(n, rowptr, col, val, r, w);
    oracle_spmv(n, rowptr, col, val, w, t);
    st->rho = oracle_dot(n, rh, r);
    st->res_rec = sqrt(oracle_dot(n, r, r)) / st->nb;
    if (!isfinite(st->res_rec)) {
        set_breakdown(st, OR_REASON_NONFINITE);
    } else if (st->res_rec <= tol) {
        st->status = OR_OK;
        st->done = 1;
    } else if (max_iter <= 0) {
        st->status = OR_NOT_CONVERGED;
        st->done = 1;
    } else {
        st->sigma = oracle_dot(n, rh, w);
        if (st->sigma == 0.0) set_breakdown(st, OR_REASON_RS_ZERO);
        else {
            st->alpha = st->rho / st->sigma;
            if (!isfinite(st->alpha)) set_breakdown(st, OR_REASON_NONFINITE);
        }
    }
    st->beta = 0.0;
    st->omega = 0.0;
    while (!st->done) {
        const int64_t it = st->iter;
        const double a = st->alpha, bt = st->beta, om = st->omega;
        for (int64_t i = 0; i < n; ++i) {
            p[i] = r[i] + bt * (p[i] - om * s[i]);
            s[i] = w[i] + bt * (s[i] - om * z[i]);
            z[i] = t[i] + bt * (z[i] - om * v[i]);
            q[i] = r[i] - a * s[i];
            y[i] = w[i] - a * z[i];
        }
        oracle_spmv(n, rowptr, col, val, z, v);
        const double rr = oracle_dot(n, r, r), qy = oracle_dot(n, q, y), yy = oracle_dot(n, y, y),
                     qq = oracle_dot(n, q, q), rq = oracle_dot(n, rh, q), ry = oracle_dot(n, rh, y),
                     rt = oracle_dot(n, rh, t), rv = oracle_dot(n, rh, v), rs = oracle_dot(n, rh, s),
                     rz = oracle_dot(n, rh, z);
        /* stopping tests on r_i, taken in this reduction */
        const double res = sqrt(rr) / st->nb;
        st->res_rec = res;
        if (it > 0 && tr_res && it - 1 < ntrace) tr_res[it - 1] = res;
        if (!isfinite(res)) { set_breakdown(st, OR_REASON_NONFINITE); break; }
        if (res <= tol) { st->status = OR_OK; st->done = 1; break; }
        if (it >= max_iter) { st->status = OR_NOT_CONVERGED; st->done = 1; break; }
        if (it < ntrace) {
            if (tr_rho) tr_rho[it] = st->rho;
            if (tr_alpha) tr_alpha[it] = a;
        }
        const double qn = sqrt(qq) / st->nb;
        if (qn <= tol) {
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + a * p[i];
            st->omega = 0.0;
            st->iter = it + 1;
            st->res_rec = qn;
            st->half_exit = 1;
            st->status = OR_OK;
            st->done = 1;
            if (it < ntrace) {
                if (tr_omega) tr_omega[it] = 0.0;
                if (tr_res) tr_res[it] = qn;
            }
            break;
        }
        if (yy == 0.0) { set_breakdown(st, OR_REASON_YY_ZERO); break; }
        const double omn = qy / yy;
        if (!isfinite(omn)) { set_breakdown(st, OR_REASON_NONFINITE); break; }
        if (it < ntrace && tr_omega) tr_omega[it] = omn;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + a * p[i] + omn * q[i];
            r[i] = q[i] - omn * y[i];
            w[i] = y[i] - omn * (t[i] - a * v[i]);
        }
        st->iter = it + 1;
        st->omega = omn;
        const double rho_new = rq - omn * ry;
        if (rho_new == 0.0) {
            const double est = qq - 2.0 * omn * qy + omn * omn * yy;
            const double rn = sqrt(est > 0.0 ? est : 0.0) / st->nb;
            if (rn <= tol) {
                st->res_rec = rn;
                st->status = OR_OK;
                st->done = 1;
                if (it < ntrace && tr_res) tr_res[it] = rn;
            } else {
                set_breakdown(st, OR_REASON_RHO_ZERO);
            }
            break;
        }
        const double bnew = (a / omn) * (rho_new / st->rho);
        const double sig = ry - omn * (rt - a * rv) + bnew * (rs - omn * rz);
        if (!isfinite(bnew) || !isfinite(sig)) { set_breakdown(st, OR_REASON_NONFINITE); break; }
        if (sig == 0.0) { set_breakdown(st, OR_REASON_RS_ZERO); break; }
        st->beta = bnew;
        st->sigma = sig;
        st->rho = rho_new;
        st->alpha = rho_new / sig;
        if (!isfinite(st->alpha)) { set_breakdown(st, OR_REASON_NONFINITE); break; }
        oracle_spmv(n, rowptr, col, val, w, t);
    }
    free(buf);
    return st->status;
}

